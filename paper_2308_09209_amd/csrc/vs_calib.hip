// vs_calib.hip -- section 3.1 set-up: homographies from camera parameters
// (eqs. (8)-(12)) and the revision of eqs. (13)-(14), with its skew and scale
// parameters estimated from matched points on the widened overlap.  The
// corner responses, local maxima and correlation searches run on the device;
// the two-point RANSAC and the Gauss-Newton fits (FP64, a few hundred points)
// on the host.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/vstitch.h"

namespace {

void mat_mul3(const double* a, const double* b, double* c)
{
    double t[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) t[r * 3 + k] = a[r * 3] * b[k] + a[r * 3 + 1] * b[3 + k] + a[r * 3 + 2] * b[6 + k];
    std::memcpy(c, t, sizeof t);
}

bool mat_inv3(const double* a, double* out)
{
    double c[9];
    c[0] = a[4] * a[8] - a[5] * a[7];
    c[1] = a[2] * a[7] - a[1] * a[8];
    c[2] = a[1] * a[5] - a[2] * a[4];
    c[3] = a[5] * a[6] - a[3] * a[8];
    c[4] = a[0] * a[8] - a[2] * a[6];
    c[5] = a[2] * a[3] - a[0] * a[5];
    c[6] = a[3] * a[7] - a[4] * a[6];
    c[7] = a[1] * a[6] - a[0] * a[7];
    c[8] = a[0] * a[4] - a[1] * a[3];
    const double det = a[0] * c[0] + a[1] * c[3] + a[2] * c[6];
    if (det == 0.0 || !std::isfinite(det)) return false;
    for (int i = 0; i < 9; ++i) out[i] = c[i] / det;
    return true;
}

struct Hmat {
    double h[9];
};

__host__ __device__ inline void proj(const double* H, double u, double v, double& x, double& y)
{
    const double w = H[6] * u + H[7] * v + H[8];
    x = (H[0] * u + H[1] * v + H[2]) / w;
    y = (H[3] * u + H[4] * v + H[5]) / w;
}

// ---- device: luma, corner response, local maxima, correlation search ------

__global__ __launch_bounds__(256) void k_calib_luma(const uint8_t* __restrict__ F, int pitch, int w, int h,
                                                    float* __restrict__ Y)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= w * h) return;
    const uint8_t* p = F + (size_t)(i / w) * pitch + 3 * (i % w);
    Y[i] = (float)((77u * p[0] + 150u * p[1] + 29u * p[2] + 128u) >> 8);
}

// Harris response of a candidate pixel: central differences (halved), their
// products over the 5 x 5 box row by row, (Sxx Syy - Sxy^2) - 0.04 (Sxx + Syy)^2
// in FP32; candidates lie e px inside image a and project (H, FP64) into image
// b widened by `margin` and, rounded, at least eb px inside it.  0 elsewhere.
__global__ __launch_bounds__(256) void k_calib_harris(const float* __restrict__ A, int wa, int ha, const Hmat H,
                                                      int wb, int hb, int margin, int ea, int eb, float* __restrict__ R)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= wa * ha) return;
    const int x = i % wa, y = i / wa;
    float r = 0.0f;
    if (x >= ea && x < wa - ea && y >= ea && y < ha - ea) {
        double bx, by;
        proj(H.h, (double)x, (double)y, bx, by);
        const bool in = bx >= -margin && bx <= wb - 1 + margin && by >= -margin && by <= hb - 1 + margin;
        const int cx = (int)floor(bx + 0.5), cy = (int)floor(by + 0.5);
        if (in && cx >= eb && cx < wb - eb && cy >= eb && cy < hb - eb) {
            float sxx = 0.0f, sxy = 0.0f, syy = 0.0f;
            for (int dy = -2; dy <= 2; ++dy)
                for (int dx = -2; dx <= 2; ++dx) {
                    const int q = (y + dy) * wa + (x + dx);
                    const float ix = 0.5f * (A[q + 1] - A[q - 1]);
                    const float iy = 0.5f * (A[q + wa] - A[q - wa]);
                    sxx = __builtin_fmaf(ix, ix, sxx);
                    sxy = __builtin_fmaf(ix, iy, sxy);
                    syy = __builtin_fmaf(iy, iy, syy);
                }
            const float tr = sxx + syy;
            r = (sxx * syy - sxy * sxy) - 0.04f * (tr * tr);
        }
    }
    R[i] = r;
}

struct Corner {
    float r;
    int x, y;
};

// strict 3 x 3 local maxima with positive response, appended to a list
__global__ __launch_bounds__(256) void k_calib_nms(const float* __restrict__ R, int wa, int ha, int ea,
                                                   Corner* __restrict__ out, unsigned* __restrict__ count, int cap)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= wa * ha) return;
    const int x = i % wa, y = i / wa;
    if (x < ea || x >= wa - ea || y < ea || y >= ha - ea) return;
    const float v = R[i];
    if (!(v > 0.0f)) return;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx)
            if ((dx || dy) && !(v > R[(y + dy) * wa + x + dx])) return;
    const unsigned k = atomicAdd(count, 1u);
    if (k < (unsigned)cap) out[k] = Corner{v, x, y};
}

// NCC score of 11 x 11 patches: cov |cov| / (va vb), FP32, sums row by row
__device__ float ncc11(const float* __restrict__ A, int wa, int xa, int ya, const float* __restrict__ B, int wb,
                       int xb, int yb)
{
    float sa = 0.0f, sb = 0.0f;
    for (int dy = -5; dy <= 5; ++dy)
        for (int dx = -5; dx <= 5; ++dx) {
            sa += A[(ya + dy) * wa + xa + dx];
            sb += B[(yb + dy) * wb + xb + dx];
        }
    const float ma = sa / 121.0f, mb = sb / 121.0f;
    float cov = 0.0f, va = 0.0f, vb = 0.0f;
    for (int dy = -5; dy <= 5; ++dy)
        for (int dx = -5; dx <= 5; ++dx) {
            const float a = A[(ya + dy) * wa + xa + dx] - ma;
            const float b = B[(yb + dy) * wb + xb + dx] - mb;
            cov = __builtin_fmaf(a, b, cov);
            va = __builtin_fmaf(a, a, va);
            vb = __builtin_fmaf(b, b, vb);
        }
    const float d = va * vb;
    return d > 0.0f ? (cov * fabsf(cov)) / d : 0.0f;
}

struct Match {
    float best, xm, xp, ym, yp;   // score at the best position and at its 4 neighbours
    int bx, by;
};

// one block per corner: every position within +-r of round(H x) scored by a
// thread, the best (first in row-major order on ties) and its neighbours
__global__ __launch_bounds__(256) void k_calib_match(const float* __restrict__ A, int wa, const float* __restrict__ B,
                                                     int wb, const Corner* __restrict__ cs, const Hmat H, int r,
                                                     Match* __restrict__ out)
{
    __shared__ float s_s[256];
    __shared__ int s_i[256];
    const Corner c = cs[blockIdx.x];
    double bx, by;
    proj(H.h, (double)c.x, (double)c.y, bx, by);
    const int px = (int)floor(bx + 0.5), py = (int)floor(by + 0.5);
    const int n = (2 * r + 1) * (2 * r + 1);
    float best = -2.0f;
    int bi = 0x7fffffff;
    for (int k = threadIdx.x; k < n; k += 256) {
        const float s = ncc11(A, wa, c.x, c.y, B, wb, px - r + k % (2 * r + 1), py - r + k / (2 * r + 1));
        if (s > best) {   // k increases: the first of equal scores stays
            best = s;
            bi = k;
        }
    }
    s_s[threadIdx.x] = best;
    s_i[threadIdx.x] = bi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const float s2 = s_s[threadIdx.x + o];
            const int i2 = s_i[threadIdx.x + o];
            if (s2 > s_s[threadIdx.x] || (s2 == s_s[threadIdx.x] && i2 < s_i[threadIdx.x])) {
                s_s[threadIdx.x] = s2;
                s_i[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    const int k = s_i[0];
    const float sbest = s_s[0];
    const int mx = px - r + k % (2 * r + 1), my = py - r + k / (2 * r + 1);
    __shared__ float s_nb[4];
    if (threadIdx.x < 4) {
        const int dx = threadIdx.x == 0 ? -1 : (threadIdx.x == 1 ? 1 : 0);
        const int dy = threadIdx.x == 2 ? -1 : (threadIdx.x == 3 ? 1 : 0);
        s_nb[threadIdx.x] = ncc11(A, wa, c.x, c.y, B, wb, mx + dx, my + dy);
    }
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = Match{sbest, s_nb[0], s_nb[1], s_nb[2], s_nb[3], mx, my};
}

// ---- host: the model and its fits (FP64) --------------------------------

// the vertex of the parabola through (-1, sm), (0, s0), (1, sp), within 1/2
double vertex(float sm, float s0, float sp)
{
    const double a = (double)sm, b = (double)s0, c = (double)sp;
    const double den = a - 2.0 * b + c;
    if (!(den < 0.0)) return 0.0;
    const double d = 0.5 * (a - c) / den;
    return d < -0.5 ? -0.5 : (d > 0.5 ? 0.5 : d);
}

struct Pts {
    std::vector<double> ua, va, xb, yb;
};

// x_b = proj(H diag(sx, sy, 1) x_a) + (tx, ty), p = (tx, ty, sx, sy)
void model_at(const double* H, const double* p, double u, double v, double& x, double& y)
{
    proj(H, p[2] * u, p[3] * v, x, y);
    x += p[0];
    y += p[1];
}

// 10 Gauss-Newton steps over the listed correspondences (normal equations,
// Gaussian elimination with partial pivoting); false if singular or not finite
bool fit(const double* H, const Pts& m, const std::vector<int>& idx, double* p)
{
    for (int it = 0; it < 10; ++it) {
        double A[4][5] = {};
        for (int k : idx) {
            const double u = m.ua[k], v = m.va[k];
            const double su = p[2] * u, sv = p[3] * v;
            const double a = H[0] * su + H[1] * sv + H[2];
            const double b = H[3] * su + H[4] * sv + H[5];
            const double c = H[6] * su + H[7] * sv + H[8];
            const double px = a / c + p[0], py = b / c + p[1];
            const double jx[4] = {1.0, 0.0, (H[0] * u * c - a * H[6] * u) / (c * c), (H[1] * v * c - a * H[7] * v) / (c * c)};
            const double jy[4] = {0.0, 1.0, (H[3] * u * c - b * H[6] * u) / (c * c), (H[4] * v * c - b * H[7] * v) / (c * c)};
            const double rx = m.xb[k] - px, ry = m.yb[k] - py;
            for (int r = 0; r < 4; ++r) {
                for (int q = 0; q < 4; ++q) A[r][q] += jx[r] * jx[q] + jy[r] * jy[q];
                A[r][4] += jx[r] * rx + jy[r] * ry;
            }
        }
        for (int col = 0; col < 4; ++col) {
            int piv = col;
            for (int r = col + 1; r < 4; ++r)
                if (std::fabs(A[r][col]) > std::fabs(A[piv][col])) piv = r;
            if (!(std::fabs(A[piv][col]) > 1e-300)) return false;
            if (piv != col)
                for (int q = 0; q < 5; ++q) std::swap(A[col][q], A[piv][q]);
            for (int r = col + 1; r < 4; ++r) {
                const double f = A[r][col] / A[col][col];
                for (int q = col; q < 5; ++q) A[r][q] -= f * A[col][q];
            }
        }
        double d[4];
        for (int r = 3; r >= 0; --r) {
            double sacc = A[r][4];
            for (int q = r + 1; q < 4; ++q) sacc -= A[r][q] * d[q];
            d[r] = sacc / A[r][r];
        }
        for (int r = 0; r < 4; ++r) p[r] += d[r];
    }
    for (int r = 0; r < 4; ++r)
        if (!std::isfinite(p[r])) return false;
    return true;
}

int count_inliers(const double* H, const Pts& m, const double* p, std::vector<int>* out)
{
    int n = 0;
    for (size_t k = 0; k < m.ua.size(); ++k) {
        double x, y;
        model_at(H, p, m.ua[k], m.va[k], x, y);
        if ((x - m.xb[k]) * (x - m.xb[k]) + (y - m.yb[k]) * (y - m.yb[k]) < 4.0) {
            ++n;
            if (out) out->push_back((int)k);
        }
    }
    return n;
}

}  // namespace

extern "C" {

vs_status vs_calib_intrinsics(double f, double dx, double dy, double cx, double cy, double u0, double v0, double K[9])
{
    if (!K || !(dx != 0.0) || !(dy != 0.0)) return VS_E_INVAL;
    const double k[9] = {f / dx, 0.0, cx / dx + u0, 0.0, f / dy, cy / dy + v0, 0.0, 0.0, 1.0};
    std::memcpy(K, k, sizeof k);
    return VS_OK;
}

vs_status vs_calib_plane_homography(const double K[9], const double R[9], const double t[3], double H[9])
{
    if (!K || !R || !t || !H) return VS_E_INVAL;
    const double P[9] = {R[0], R[1], t[0], R[3], R[4], t[1], R[6], R[7], t[2]};
    mat_mul3(K, P, H);
    return VS_OK;
}

vs_status vs_calib_pair(const double Ha[9], const double Hb[9], double Hab[9])
{
    if (!Ha || !Hb || !Hab) return VS_E_INVAL;
    double ib[9];
    if (!mat_inv3(Hb, ib)) return VS_E_INVAL;
    mat_mul3(Ha, ib, Hab);
    return VS_OK;
}

vs_status vs_calib_refine(const double H[9], const double p[4], double Hr[9])
{
    if (!H || !p || !Hr) return VS_E_INVAL;
    const double M[9] = {1, 0, p[0], 0, 1, p[1], 0, 0, 1};
    const double N[9] = {p[2], 0, 0, 0, p[3], 0, 0, 0, 1};
    double t[9];
    mat_mul3(M, H, t);
    mat_mul3(t, N, Hr);
    return VS_OK;
}

vs_status vs_calib_estimate(const uint8_t* frame_a, int pitch_a, int wa, int ha, const uint8_t* frame_b, int pitch_b,
                            int wb, int hb, const double H[9], int margin, int radius, double p_out[4],
                            int32_t* n_matches, int32_t* n_inliers, void* stream)
{
    if (!frame_a || !frame_b || !H || !p_out || wa < 32 || ha < 32 || wb < 32 || hb < 32 || pitch_a < 3 * wa ||
        pitch_b < 3 * wb || margin < 0 || radius < 1 || radius > 7)
        return VS_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    const int ea = 8 + radius, eb = 6 + radius;
    constexpr int kMaxCorners = 256;
    const size_t na = (size_t)wa * ha, nb = (size_t)wb * hb;
    const int cap = 1 << 20;
    void* mem = nullptr;
    const size_t bytes = (na + nb + na) * 4 + (size_t)cap * sizeof(Corner) + 256 + kMaxCorners * sizeof(Corner) +
                         kMaxCorners * sizeof(Match);
    if (hipMalloc(&mem, bytes) != hipSuccess) return VS_E_NOMEM;
    float* A = (float*)mem;
    float* B = A + na;
    float* R = B + nb;
    Corner* list = (Corner*)(R + na);
    unsigned* count = (unsigned*)(list + cap);
    Corner* top = (Corner*)((uint8_t*)count + 256);
    Match* matches = (Match*)(top + kMaxCorners);
    Hmat hm;
    std::memcpy(hm.h, H, sizeof hm.h);
    vs_status st = VS_OK;
    std::vector<Corner> cs;
    std::vector<Match> ms;
    unsigned nc = 0;
    do {
        hipLaunchKernelGGL(k_calib_luma, dim3((unsigned)((na + 255) / 256)), dim3(256), 0, s, frame_a, pitch_a, wa, ha, A);
        hipLaunchKernelGGL(k_calib_luma, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, frame_b, pitch_b, wb, hb, B);
        hipLaunchKernelGGL(k_calib_harris, dim3((unsigned)((na + 255) / 256)), dim3(256), 0, s, A, wa, ha, hm, wb, hb,
                           margin, ea, eb, R);
        if (hipMemsetAsync(count, 0, 4, s) != hipSuccess) { st = VS_E_DEVICE; break; }
        hipLaunchKernelGGL(k_calib_nms, dim3((unsigned)((na + 255) / 256)), dim3(256), 0, s, R, wa, ha, ea, list, count, cap);
        if (hipGetLastError() != hipSuccess || hipMemcpyAsync(&nc, count, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) { st = VS_E_DEVICE; break; }
        nc = std::min(nc, (unsigned)cap);
        cs.resize(nc);
        if (nc && (hipMemcpy(cs.data(), list, nc * sizeof(Corner), hipMemcpyDeviceToHost) != hipSuccess)) { st = VS_E_DEVICE; break; }
        // strongest first; equal responses in scan order (row, then column)
        std::sort(cs.begin(), cs.end(), [](const Corner& a, const Corner& b) {
            if (a.r != b.r) return a.r > b.r;
            if (a.y != b.y) return a.y < b.y;
            return a.x < b.x;
        });
        if (cs.size() > (size_t)kMaxCorners) cs.resize(kMaxCorners);
        if (cs.empty()) break;
        if (hipMemcpy(top, cs.data(), cs.size() * sizeof(Corner), hipMemcpyHostToDevice) != hipSuccess) { st = VS_E_DEVICE; break; }
        hipLaunchKernelGGL(k_calib_match, dim3((unsigned)cs.size()), dim3(256), 0, s, A, wa, B, wb, top, hm, radius, matches);
        ms.resize(cs.size());
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(ms.data(), matches, ms.size() * sizeof(Match), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) { st = VS_E_DEVICE; break; }
    } while (false);
    (void)hipFree(mem);
    if (st != VS_OK) return st;
    Pts m;
    for (size_t k = 0; k < ms.size(); ++k) {
        if (!(ms[k].best >= 0.49f)) continue;
        m.ua.push_back(cs[k].x);
        m.va.push_back(cs[k].y);
        m.xb.push_back(ms[k].bx + vertex(ms[k].xm, ms[k].best, ms[k].xp));
        m.yb.push_back(ms[k].by + vertex(ms[k].ym, ms[k].best, ms[k].yp));
    }
    const int nm = (int)m.ua.size();
    if (n_matches) *n_matches = nm;
    if (n_inliers) *n_inliers = 0;
    if (nm < 2) return VS_E_INVAL;
    // RANSAC: every pair of the first 64 matches, two-point fits from (0, 0, 1, 1)
    const int ns = std::min(nm, 64);
    int best_in = -1;
    double best_p[4] = {0.0, 0.0, 1.0, 1.0};
    for (int a = 0; a < ns; ++a)
        for (int b = a + 1; b < ns; ++b) {
            double p[4] = {0.0, 0.0, 1.0, 1.0};
            if (!fit(H, m, std::vector<int>{a, b}, p)) continue;
            const int cnt = count_inliers(H, m, p, nullptr);
            if (cnt > best_in) {
                best_in = cnt;
                std::memcpy(best_p, p, sizeof p);
            }
        }
    if (best_in < 2) return VS_E_INVAL;
    std::vector<int> inl;
    count_inliers(H, m, best_p, &inl);
    double p[4];
    std::memcpy(p, best_p, sizeof p);
    if (!fit(H, m, inl, p)) return VS_E_INVAL;
    std::memcpy(p_out, p, sizeof p);
    if (n_inliers) *n_inliers = (int32_t)inl.size();
    return VS_OK;
}

}  // extern "C"
