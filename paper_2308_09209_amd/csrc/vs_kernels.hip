// vs_kernels.hip -- gfx950 kernels of the per-frame stitching path.
//
// Every floating-point result that decides a byte (coverage, resampling,
// colour application, luma, pyramid, flow, blend weights) is computed in FP32
// in one fixed operation order with explicit fused multiply-adds and
// correctly rounded division (the library is built with -ffp-contract=off),
// so the results are reproducible bit for bit on any IEEE implementation.
// The colour solve and the balancing curve are FP64; histograms and moments
// are exact integers (order-independent atomics).
#include <algorithm>

#include "vs_internal.h"

namespace vs {

// ---------------------------------------------------------------------------
// Conventions (section 3.1 pre-warp; section 2.1 eq. (4) colour application)
// ---------------------------------------------------------------------------

__device__ __forceinline__ float clampf(float v, float lo, float hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

// round half up to a byte
__device__ __forceinline__ uint32_t round8(float r)
{
    float f = floorf(r + 0.5f);
    f = f < 0.0f ? 0.0f : f;
    f = f > 255.0f ? 255.0f : f;
    return (uint32_t)(int)f;
}

// canvas -> camera homography; valid iff w > 0 and inside [0, W-1] x [0, H-1];
// position (0, 0) when w <= 0
__device__ __forceinline__ bool hom(const float* __restrict__ h, float x, float y, int W, int H,
                                    float& u, float& v)
{
    float nu = __builtin_fmaf(h[0], x, __builtin_fmaf(h[1], y, h[2]));
    float nv = __builtin_fmaf(h[3], x, __builtin_fmaf(h[4], y, h[5]));
    float w = __builtin_fmaf(h[6], x, __builtin_fmaf(h[7], y, h[8]));
    if (!(w > 0.0f)) {
        u = 0.0f;
        v = 0.0f;
        return false;
    }
    u = nu / w;
    v = nv / w;
    return (u >= 0.0f) && (u <= (float)(W - 1)) && (v >= 0.0f) && (v <= (float)(H - 1));
}

// bilinear resample of an HWC RGB byte image, position clamped into the image
__device__ __forceinline__ void bilin3(const uint8_t* __restrict__ F, int pitch, int W, int H,
                                       float u, float v, float out[3])
{
    float uc = clampf(u, 0.0f, (float)(W - 1));
    float vc = clampf(v, 0.0f, (float)(H - 1));
    float flx = floorf(uc), fly = floorf(vc);
    int x0 = (int)flx, y0 = (int)fly;
    float fx = uc - flx, fy = vc - fly;
    int x1 = x0 + 1 < W ? x0 + 1 : W - 1;
    int y1 = y0 + 1 < H ? y0 + 1 : H - 1;
    const uint8_t* r0 = F + (size_t)y0 * pitch;
    const uint8_t* r1 = F + (size_t)y1 * pitch;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float p00 = (float)r0[x0 * 3 + c];
        float p10 = (float)r0[x1 * 3 + c];
        float p01 = (float)r1[x0 * 3 + c];
        float p11 = (float)r1[x1 * 3 + c];
        float a = __builtin_fmaf(fx, p10 - p00, p00);
        float b = __builtin_fmaf(fx, p11 - p01, p01);
        out[c] = __builtin_fmaf(fy, b - a, a);
    }
}

// t_c = s . M[:, c] (row-vector convention), clamped to [0, 255]
__device__ __forceinline__ float capply(const float s[3], const float* __restrict__ M, int c)
{
    float t = __builtin_fmaf(s[0], M[c], __builtin_fmaf(s[1], M[3 + c], s[2] * M[6 + c]));
    return clampf(t, 0.0f, 255.0f);
}

__device__ __forceinline__ int batch_block(const Batch& B, int b, int& c)
{
    c = 0;
    while (c + 1 < B.n && b >= B.off[c + 1]) ++c;
    return b - B.off[c];
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Plan: coverage of every canvas pixel (section 2.1 step 1, section 3)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_plan_scan(const DevPlan* __restrict__ P, PlanScan* scan)
{
    __shared__ int s_box[MAXP][4];
    __shared__ unsigned long long s_cov;
    __shared__ uint32_t s_err;
    const int tid = threadIdx.x;
    if (tid < MAXP) {
        s_box[tid][0] = 0x3fffffff;
        s_box[tid][1] = -0x3fffffff;
        s_box[tid][2] = 0x3fffffff;
        s_box[tid][3] = -0x3fffffff;
    }
    if (tid == 0) {
        s_cov = 0;
        s_err = 0;
    }
    __syncthreads();
    const int words = P->cover_words;
    const long gid = (long)blockIdx.x * 256 + tid;
    const int y = (int)(gid / words), wx = (int)(gid % words);
    if (y < P->canvas_h) {
        const int x0 = wx * 32;
        uint32_t bits = 0, err = 0;
        unsigned long long cand = 0;
        const int mlo = P->ring ? -1 : 0, mhi = P->ring ? 1 : 0;
        for (int x = x0; x < x0 + 32 && x < P->canvas_w; ++x) {
            int nh = 0, hc[2] = {0, 0}, hm[2] = {0, 0};
            for (int k = 0; k < P->n_cams; ++k) {
                for (int m = mlo; m <= mhi; ++m) {
                    float u, v;
                    int X = x + m * P->Wp;
                    if (hom(P->hinv[k], (float)X, (float)y, P->cam_w[k], P->cam_h[k], u, v)) {
                        if (nh < 2) {
                            hc[nh] = k;
                            hm[nh] = m;
                        }
                        ++nh;
                        cand |= 1ull << (k * 3 + m + 1);
                    }
                }
            }
            {
                const int n2 = nh < 2 ? nh : 2;
                const uint32_t code = (n2 > 0 ? (uint32_t)(hc[0] * 3 + hm[0] + 1) : 0u) |
                                      (n2 > 1 ? (uint32_t)(hc[1] * 3 + hm[1] + 1) << 6 : 0u) | (uint32_t)n2 << 12;
                P->pix_code[(size_t)y * P->canvas_w + x] = (uint16_t)code;
            }
            if (nh > 0) bits |= 1u << (x - x0);
            if (nh > 2) err |= 1u;
            if (nh == 2) {
                if (hc[0] == hc[1]) {
                    err |= 2u;
                    continue;
                }
                int p = P->pair_of[hc[0]][hc[1]];
                if (p < 0) {
                    err |= 4u;
                    continue;
                }
                int jfirst = hc[0] == P->pj[p];
                int mj = jfirst ? hm[0] : hm[1];
                int mi = jfirst ? hm[1] : hm[0];
                if (mj != mi + P->psi[p]) {
                    err |= 8u;
                    continue;
                }
                int X = x + mj * P->Wp;
                atomicMin(&s_box[p][0], X);
                atomicMax(&s_box[p][1], X);
                atomicMin(&s_box[p][2], y);
                atomicMax(&s_box[p][3], y);
            }
        }
        P->cover[(size_t)y * words + wx] = bits;
        if (bits) atomicAdd(&s_cov, (unsigned long long)__popc(bits));
        if (err) atomicOr(&s_err, err);
        if (cand) atomicOr(&P->cand[(y / BL_TY) * P->blend_tx + x0 / BL_TX], cand);
    }
    __syncthreads();
    if (tid < P->n_pairs && s_box[tid][1] >= s_box[tid][0]) {
        atomicMin(&scan->bx0[tid], s_box[tid][0]);
        atomicMax(&scan->bx1[tid], s_box[tid][1]);
        atomicMin(&scan->by0[tid], s_box[tid][2]);
        atomicMax(&scan->by1[tid], s_box[tid][3]);
    }
    if (tid == 0) {
        if (s_cov) atomicAdd(&scan->n_covered, s_cov);
        if (s_err) atomicOr(&scan->err, s_err);
    }
}

hipError_t launch_plan_scan(const DevPlan* dp, const DevPlan& hp, PlanScan* scan, hipStream_t s)
{
    long items = (long)hp.canvas_h * hp.cover_words;
    int blocks = (int)((items + 255) / 256);
    hipLaunchKernelGGL(k_plan_scan, dim3(blocks), dim3(256), 0, s, dp, scan);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-frame accumulators <- 0 (a fill kernel, no memset node)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_zero(const Batch B)
{
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    uint4* p = (uint4*)B.plan[c]->acc;
    const int i = b * 256 + threadIdx.x;
    if (i < (int)(sizeof(Accum) / 16)) p[i] = make_uint4(0, 0, 0, 0);
}

// Frame and panorama pointers of every context of the group, written into its
// device plan before the frame's kernels run (they read them from there, so a
// captured frame graph replays for any input buffers).
__global__ void k_set_io(const FrameIO io)
{
    const int c = blockIdx.x;
    const int k = threadIdx.x;
    DevPlan* P = io.plan[c];
    if (k < MAXC) P->frame[k] = io.frame[c][k];
    if (k == 0) P->pano = io.pano[c];
}

// ---------------------------------------------------------------------------
// Section 2.1 steps 1-2 and eq. (1) A: overlap strips, masks, histograms and
// the exact moment A = sum p p^T of camera i's overlap pixels
// ---------------------------------------------------------------------------

__device__ __forceinline__ int find_field(const int32_t* off, int n, int b)
{
    int f = 0;
    while (f + 1 < n && b >= off[f + 1]) ++f;
    return f;
}

__device__ __forceinline__ void strips_body(const DevPlan* __restrict__ P, const int bid)
{
    __shared__ uint32_t s_hist[4][2 * 3 * 256];   // 4 copies (lane & 3) against same-value conflicts
    __shared__ uint32_t s_red[4][7];
    const int tid = threadIdx.x;
    const int p = find_field(P->strip_off, P->n_pairs, bid);
    const int t = bid - P->strip_off[p];
    const int sw = P->sw[p], sh = P->sh[p];
    const int tx0 = (t % P->strip_tx[p]) * STRIP_TX, ty0 = (t / P->strip_tx[p]) * STRIP_TY;
    for (int i = tid; i < 4 * 2 * 3 * 256; i += 256) (&s_hist[0][0])[i] = 0;
    __syncthreads();
    uint32_t* const my_hist = s_hist[tid & 3];

    const int kj = P->pj[p], ki = P->pi[p];
    const int shift_i = P->psi[p] * P->Wp;
    uint32_t* __restrict__ strip = P->strip[p];
    uint8_t* __restrict__ mask = P->mask[p];
    const int lx = tx0 + (tid & 63);
    uint32_t a00 = 0, a01 = 0, a02 = 0, a11 = 0, a12 = 0, a22 = 0, cnt = 0;
    for (int r = tid >> 6; r < STRIP_TY; r += 4) {
        const int ly = ty0 + r;
        if (lx >= sw || ly >= sh) continue;
        const int X = P->sx0[p] + lx, Y = P->sy0[p] + ly;
        float u, v, rgb[3];
        bool okj = hom(P->hinv[kj], (float)X, (float)Y, P->cam_w[kj], P->cam_h[kj], u, v);
        bilin3(P->frame[kj], P->cam_pitch[kj], P->cam_w[kj], P->cam_h[kj], u, v, rgb);
        uint32_t cj0 = round8(rgb[0]), cj1 = round8(rgb[1]), cj2 = round8(rgb[2]);
        bool oki = hom(P->hinv[ki], (float)(X - shift_i), (float)Y, P->cam_w[ki], P->cam_h[ki], u, v);
        bilin3(P->frame[ki], P->cam_pitch[ki], P->cam_w[ki], P->cam_h[ki], u, v, rgb);
        uint32_t ci0 = round8(rgb[0]), ci1 = round8(rgb[1]), ci2 = round8(rgb[2]);
        const size_t q = (size_t)ly * sw + lx;
        strip[q] = cj0 | (cj1 << 8) | (cj2 << 16);
        strip[(size_t)sh * sw + q] = ci0 | (ci1 << 8) | (ci2 << 16);
        const bool ok = okj && oki;
        mask[q] = ok ? 1 : 0;
        if (ok) {
            atomicAdd(&my_hist[0 * 256 + cj0], 1u);
            atomicAdd(&my_hist[1 * 256 + cj1], 1u);
            atomicAdd(&my_hist[2 * 256 + cj2], 1u);
            atomicAdd(&my_hist[3 * 256 + ci0], 1u);
            atomicAdd(&my_hist[4 * 256 + ci1], 1u);
            atomicAdd(&my_hist[5 * 256 + ci2], 1u);
            a00 += ci0 * ci0;
            a01 += ci0 * ci1;
            a02 += ci0 * ci2;
            a11 += ci1 * ci1;
            a12 += ci1 * ci2;
            a22 += ci2 * ci2;
            cnt += 1;
        }
    }
    uint32_t vals[7] = {a00, a01, a02, a11, a12, a22, cnt};
#pragma unroll
    for (int i = 0; i < 7; ++i) vals[i] = wave_sum(vals[i]);
    if ((tid & 63) == 0) {
#pragma unroll
        for (int i = 0; i < 7; ++i) s_red[tid >> 6][i] = vals[i];
    }
    __syncthreads();
    Accum* acc = P->acc;
    if (tid < 7) {
        unsigned long long s = (unsigned long long)s_red[0][tid] + s_red[1][tid] + s_red[2][tid] + s_red[3][tid];
        if (s) {
            if (tid < 6) atomicAdd(&acc->A[p][tid], s);
            else atomicAdd(&acc->n[p], s);
        }
    }
    uint32_t* gh = &acc->hist[p][0][0][0];
    for (int i = tid; i < 2 * 3 * 256; i += 256) {
        const uint32_t h = s_hist[0][i] + s_hist[1][i] + s_hist[2][i] + s_hist[3][i];
        if (h) atomicAdd(&gh[i], h);
    }
}

__global__ __launch_bounds__(256) void k_strips(const Batch B)
{
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    strips_body(B.plan[c], b);
}


// ---------------------------------------------------------------------------
// Section 2.1 step 3: histogram specification LUT(v) = min{w : C_j(w) >= C_i(v)}
// ---------------------------------------------------------------------------

__device__ __forceinline__ void lut_body(const DevPlan* __restrict__ P, const int bid)
{
    __shared__ uint32_t Ci[3][256], Cj[3][256];
    const int p = bid, v = threadIdx.x;
    const Accum* acc = P->acc;
    for (int c = 0; c < 3; ++c) {
        Cj[c][v] = acc->hist[p][0][c][v];
        Ci[c][v] = acc->hist[p][1][c][v];
    }
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        uint32_t ti[3], tj[3];
        for (int c = 0; c < 3; ++c) {
            ti[c] = v >= o ? Ci[c][v - o] : 0;
            tj[c] = v >= o ? Cj[c][v - o] : 0;
        }
        __syncthreads();
        for (int c = 0; c < 3; ++c) {
            Ci[c][v] += ti[c];
            Cj[c][v] += tj[c];
        }
        __syncthreads();
    }
    for (int c = 0; c < 3; ++c) {
        uint32_t target = Ci[c][v];
        int lo = 0, hi = 256;   // first w with Cj[w] >= target
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (Cj[c][mid] < target) lo = mid + 1;
            else hi = mid;
        }
        P->res->lut[p][c][v] = (uint8_t)(lo > 255 ? 255 : lo);
    }
}

__global__ __launch_bounds__(256) void k_lut(const Batch B)
{
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    lut_body(B.plan[c], b);
}


// ---------------------------------------------------------------------------
// Eq. (1) B = I_i^T I_j with I_j = LUT(I_i) (the histogram-specified image i)
// ---------------------------------------------------------------------------

__device__ __forceinline__ void moments_b_body(const DevPlan* __restrict__ P, const int bid)
{
    __shared__ uint8_t s_lut[3][256];
    __shared__ uint32_t s_red[4][9];
    const int tid = threadIdx.x;
    const int p = find_field(P->strip_off, P->n_pairs, bid);
    const int t = bid - P->strip_off[p];
    const int sw = P->sw[p], sh = P->sh[p];
    const int tx0 = (t % P->strip_tx[p]) * STRIP_TX, ty0 = (t / P->strip_tx[p]) * STRIP_TY;
    for (int i = tid; i < 3 * 256; i += 256) (&s_lut[0][0])[i] = (&P->res->lut[p][0][0])[i];
    __syncthreads();
    const uint32_t* __restrict__ strip_i = P->strip[p] + (size_t)sh * sw;
    const uint8_t* __restrict__ mask = P->mask[p];
    const int lx = tx0 + (tid & 63);
    uint32_t b[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int r = tid >> 6; r < STRIP_TY; r += 4) {
        const int ly = ty0 + r;
        if (lx >= sw || ly >= sh) continue;
        const size_t q = (size_t)ly * sw + lx;
        if (!mask[q]) continue;
        uint32_t pix = strip_i[q];
        uint32_t pv[3] = {pix & 255u, (pix >> 8) & 255u, (pix >> 16) & 255u};
        uint32_t qv[3] = {s_lut[0][pv[0]], s_lut[1][pv[1]], s_lut[2][pv[2]]};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) b[a * 3 + c] += pv[a] * qv[c];
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) b[i] = wave_sum(b[i]);
    if ((tid & 63) == 0) {
#pragma unroll
        for (int i = 0; i < 9; ++i) s_red[tid >> 6][i] = b[i];
    }
    __syncthreads();
    if (tid < 9) {
        unsigned long long s = (unsigned long long)s_red[0][tid] + s_red[1][tid] + s_red[2][tid] + s_red[3][tid];
        if (s) atomicAdd(&P->acc->B[p][tid], s);
    }
}

__global__ __launch_bounds__(256) void k_moments_b(const Batch B)
{
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    moments_b_body(B.plan[c], b);
}


// ---------------------------------------------------------------------------
// Eqs. (2)-(4): 3D-M solve (FP64) per pair, chain composition, state shift
// ---------------------------------------------------------------------------

// (A + eps I) M = B + eps I, eps = ridge * trace(A); Gaussian elimination with
// partial pivoting (first largest on ties) and back substitution.  Returns 1
// (M = I) when a pivot falls below 1e-12 of the largest |entry|.
__device__ int solve3(const double* A, const double* B, double ridge, double* M)
{
    double a[3][3], b[3][3];
    const double eps = ridge * ((A[0] + A[4]) + A[8]);
    double maxabs = 0.0;
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            a[r][k] = A[r * 3 + k] + (r == k ? eps : 0.0);
            b[r][k] = B[r * 3 + k] + (r == k ? eps : 0.0);
            if (fabs(a[r][k]) > maxabs) maxabs = fabs(a[r][k]);
        }
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        for (int r = col + 1; r < 3; ++r)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (piv != col) {
            for (int k = 0; k < 3; ++k) {
                double t = a[col][k];
                a[col][k] = a[piv][k];
                a[piv][k] = t;
                t = b[col][k];
                b[col][k] = b[piv][k];
                b[piv][k] = t;
            }
        }
        if (!(fabs(a[col][col]) >= 1e-12 * maxabs) || a[col][col] == 0.0) {
            for (int i = 0; i < 9; ++i) M[i] = (i % 4 == 0) ? 1.0 : 0.0;
            return 1;
        }
        for (int r = col + 1; r < 3; ++r) {
            double f = a[r][col] / a[col][col];
            for (int k = col; k < 3; ++k) a[r][k] = a[r][k] - f * a[col][k];
            for (int k = 0; k < 3; ++k) b[r][k] = b[r][k] - f * b[col][k];
        }
    }
    double x[3][3];
    for (int r = 2; r >= 0; --r)
        for (int k = 0; k < 3; ++k) {
            double s = b[r][k];
            for (int q = r + 1; q < 3; ++q) s = s - a[r][q] * x[q][k];
            x[r][k] = s / a[r][r];
        }
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) M[r * 3 + k] = x[r][k];
    return 0;
}

__device__ __forceinline__ void solve_body(const DevPlan* __restrict__ P, const int bid)
{
    __shared__ double s_M[MAXP][9];
    const int tid = threadIdx.x;
    Accum* acc = P->acc;
    Results* res = P->res;
    vs_color_state* st = P->state;
    if (tid < P->n_pairs) {
        const int p = tid;
        unsigned long long A[6], B[9], n;
        for (int i = 0; i < 6; ++i) A[i] = acc->A[p][i];
        for (int i = 0; i < 9; ++i) B[i] = acc->B[p][i];
        n = acc->n[p];
        for (int i = 0; i < 6; ++i) res->mom[p][i] = A[i];
        for (int i = 0; i < 9; ++i) res->mom[p][6 + i] = B[i];
        res->mom[p][15] = n;
        unsigned long long A3[6], B3[9], n3 = n;
        for (int i = 0; i < 6; ++i) A3[i] = A[i];
        for (int i = 0; i < 9; ++i) B3[i] = B[i];
        const int W = P->color_window;
        const int T = (int)st->frames_seen;
        for (int d = 1; d < W && d <= T; ++d) {
            const vs_moments* o = &st->mom[p][d - 1];
            for (int i = 0; i < 6; ++i) A3[i] += o->A[i];
            for (int i = 0; i < 9; ++i) B3[i] += o->B[i];
            n3 += o->n;
        }
        double M[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        int flag = 0;
        if (W > 0) {
            if (n3 < (unsigned long long)P->min_pixels) {
                flag = 1;
            } else {
                double Ad[9] = {(double)A3[0], (double)A3[1], (double)A3[2], (double)A3[1], (double)A3[3],
                                (double)A3[4], (double)A3[2], (double)A3[4], (double)A3[5]};
                double Bd[9];
                for (int i = 0; i < 9; ++i) Bd[i] = (double)B3[i];
                if (solve3(Ad, Bd, P->ridge, M)) flag = 2;
            }
        }
        for (int i = 0; i < 9; ++i) {
            s_M[p][i] = M[i];
            res->Mpair[p][i] = M[i];
        }
        res->flags[p] = flag;
        st->mom[p][1] = st->mom[p][0];
        for (int i = 0; i < 6; ++i) st->mom[p][0].A[i] = A[i];
        for (int i = 0; i < 9; ++i) st->mom[p][0].B[i] = B[i];
        st->mom[p][0].n = n;
    }
    __syncthreads();
    if (tid == 0) {
        double Mk[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        for (int i = 0; i < 9; ++i) res->Mk[0][i] = (float)Mk[i];
        for (int k = 1; k < P->n_cams; ++k) {
            const double* a = s_M[k - 1];
            double t[9];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c)
                    t[r * 3 + c] = (a[r * 3 + 0] * Mk[0 * 3 + c] + a[r * 3 + 1] * Mk[1 * 3 + c]) + a[r * 3 + 2] * Mk[2 * 3 + c];
            for (int i = 0; i < 9; ++i) {
                Mk[i] = t[i];
                res->Mk[k][i] = (float)t[i];
            }
        }
    }
}

__global__ __launch_bounds__(64) void k_solve(const Batch B)
{
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    solve_body(B.plan[c], b);
}


// ---------------------------------------------------------------------------
// Flow input: luma of the colour-corrected strips, then the 2x pyramid
// ---------------------------------------------------------------------------

__device__ __forceinline__ void pyr0_body(const DevPlan* __restrict__ P, const int bid)
{
    const int f = find_field(P->pyr_off[0], 2 * P->n_pairs, bid);
    const int p = f >> 1, cam = f & 1;
    const int t = bid - P->pyr_off[0][f];
    const int w = P->sw[p], h = P->sh[p];
    const int tx0 = (t % P->pyr_tx[0][f]) * PYR_TX, ty0 = (t / P->pyr_tx[0][f]) * PYR_TY;
    const float* M = P->res->Mk[cam == 0 ? P->pj[p] : P->pi[p]];
    const uint32_t* __restrict__ src = P->strip[p] + (size_t)cam * h * w;
    float* __restrict__ dst = P->pyr[p][cam][0];
    const int x = tx0 + (threadIdx.x & 63);
    for (int r = threadIdx.x >> 6; r < PYR_TY; r += 4) {
        const int y = ty0 + r;
        if (x >= w || y >= h) continue;
        uint32_t pix = src[(size_t)y * w + x];
        float s[3] = {(float)(pix & 255u), (float)((pix >> 8) & 255u), (float)((pix >> 16) & 255u)};
        uint32_t c0 = round8(capply(s, M, 0)), c1 = round8(capply(s, M, 1)), c2 = round8(capply(s, M, 2));
        dst[(size_t)y * w + x] = (float)((77u * c0 + 150u * c1 + 29u * c2 + 128u) >> 8);
    }
}

__global__ __launch_bounds__(256) void k_pyr0(const Batch B)
{
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    pyr0_body(B.plan[c], b);
}


__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// level l -> l + 1: separable [1 4 6 4 1] / 16, horizontal first, clamped,
// even positions; each pass ((((a0 + 4 a1) + 6 a2) + 4 a3) + a4) / 16
__device__ __forceinline__ void pyr_down_body(const DevPlan* __restrict__ P, const int bid, int l)
{
    const int lo = l + 1;
    const int f = find_field(P->pyr_off[lo], 2 * P->n_pairs, bid);
    const int p = f >> 1, cam = f & 1;
    const int t = bid - P->pyr_off[lo][f];
    const int ws = P->lw[p][l], hs = P->lh[p][l];
    const int wd = P->lw[p][lo], hd = P->lh[p][lo];
    const int tx0 = (t % P->pyr_tx[lo][f]) * PYR_TX, ty0 = (t / P->pyr_tx[lo][f]) * PYR_TY;
    const float* __restrict__ src = P->pyr[p][cam][l];
    float* __restrict__ dst = P->pyr[p][cam][lo];
    const int x = tx0 + (threadIdx.x & 63);
    const int xs[5] = {clampi(2 * x - 2, 0, ws - 1), clampi(2 * x - 1, 0, ws - 1), clampi(2 * x, 0, ws - 1),
                       clampi(2 * x + 1, 0, ws - 1), clampi(2 * x + 2, 0, ws - 1)};
    for (int r = threadIdx.x >> 6; r < PYR_TY; r += 4) {
        const int y = ty0 + r;
        if (x >= wd || y >= hd) continue;
        float rows[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const float* s = src + (size_t)clampi(2 * y + k - 2, 0, hs - 1) * ws;
            float acc = s[xs[0]] + 4.0f * s[xs[1]];
            acc = acc + 6.0f * s[xs[2]];
            acc = acc + 4.0f * s[xs[3]];
            acc = acc + s[xs[4]];
            rows[k] = acc * 0.0625f;
        }
        float acc = rows[0] + 4.0f * rows[1];
        acc = acc + 6.0f * rows[2];
        acc = acc + 4.0f * rows[3];
        acc = acc + rows[4];
        dst[(size_t)y * wd + x] = acc * 0.0625f;
    }
}

__global__ __launch_bounds__(256) void k_pyr_down(const Batch B, int l)
{
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    pyr_down_body(B.plan[c], b, l);
}


// ---------------------------------------------------------------------------
// Section 3.2 dense flow: pyramidal Lucas-Kanade at one level, every field
// (pair x direction), 16 x 16 pixels per block.  The template, its gradients
// and the moving image (with a halo for windows and displacements up to
// LK_D px) are staged in LDS with clamp-replicated borders; a pixel whose
// displacement leaves the staged tile reads the same clamped values from
// global memory instead.
// ---------------------------------------------------------------------------

constexpr int LK_HT = LK_R_MAX + 1;              // template halo (window + gradient)
constexpr int LK_TW = LK_T + 2 * LK_HT;          // 26
constexpr int LK_GW = LK_T + 2 * LK_R_MAX;       // 24
constexpr int LK_HM = LK_R_MAX + LK_D + 1;       // 13
constexpr int LK_MW = LK_T + 2 * LK_HM;          // 42

__device__ __forceinline__ void lk_body(const DevPlan* __restrict__ P, const int bid, int l)
{
    __shared__ float sT[LK_TW][LK_TW];
    __shared__ float sIx[LK_GW][LK_GW];
    __shared__ float sIy[LK_GW][LK_GW];
    __shared__ float sM[LK_MW][LK_MW];
    const int f = find_field(P->lk_off[l], 2 * P->n_pairs, bid);
    const int p = f >> 1, dir = f & 1;
    if (P->flow_mode != VS_FLOW_PLAIN && P->res->surr_ok[p]) return;   // the pair keeps the surrogate's flows
    const int t = bid - P->lk_off[l][f];
    const int w = P->lw[p][l], h = P->lh[p][l];
    const int x0 = (t % P->lk_tx[l][f]) * LK_T, y0 = (t / P->lk_tx[l][f]) * LK_T;
    const float* __restrict__ Tm = P->pyr[p][dir == 0 ? 0 : 1][l];
    const float* __restrict__ Mv = P->pyr[p][dir == 0 ? 1 : 0][l];
    const int tid = threadIdx.x;

    for (int i = tid; i < LK_TW * LK_TW; i += 256) {
        int yy = clampi(y0 - LK_HT + i / LK_TW, 0, h - 1), xx = clampi(x0 - LK_HT + i % LK_TW, 0, w - 1);
        sT[i / LK_TW][i % LK_TW] = Tm[(size_t)yy * w + xx];
    }
    for (int i = tid; i < LK_MW * LK_MW; i += 256) {
        int yy = clampi(y0 - LK_HM + i / LK_MW, 0, h - 1), xx = clampi(x0 - LK_HM + i % LK_MW, 0, w - 1);
        sM[i / LK_MW][i % LK_MW] = Mv[(size_t)yy * w + xx];
    }
    __syncthreads();
    for (int i = tid; i < LK_GW * LK_GW; i += 256) {
        // central differences at (x0 - R + gx, y0 - R + gy); the tile is
        // clamp-replicated, so its neighbours are the clamped neighbours
        const int gy = i / LK_GW, gx = i % LK_GW;
        const int cx = gx + 1, cy = gy + 1;  // position in sT
        sIx[gy][gx] = 0.5f * (sT[cy][cx + 1] - sT[cy][cx - 1]);
        sIy[gy][gx] = 0.5f * (sT[cy + 1][cx] - sT[cy - 1][cx]);
    }
    __syncthreads();

    const int tx = tid & (LK_T - 1), ty = tid / LK_T;
    const int x = x0 + tx, y = y0 + ty;
    if (x >= w || y >= h) return;
    if (!P->need[p][l][(size_t)y * w + x]) return;   // flow not estimated here (stays 0)

    float ux = 0.0f, uy = 0.0f;
    if (l + 1 < P->levels) {
        const int wc = P->lw[p][l + 1], hc = P->lh[p][l + 1];
        const float2* __restrict__ uc = P->flow[p][dir][l + 1];
        float cx = clampf(__builtin_fmaf((float)x, 0.5f, -0.25f), 0.0f, (float)(wc - 1));
        float cy = clampf(__builtin_fmaf((float)y, 0.5f, -0.25f), 0.0f, (float)(hc - 1));
        float flx = floorf(cx), fly = floorf(cy);
        int xa = (int)flx, ya = (int)fly;
        float fx = cx - flx, fy = cy - fly;
        int xb = xa + 1 < wc ? xa + 1 : wc - 1;
        int yb = ya + 1 < hc ? ya + 1 : hc - 1;
        float2 p00 = uc[(size_t)ya * wc + xa], p10 = uc[(size_t)ya * wc + xb];
        float2 p01 = uc[(size_t)yb * wc + xa], p11 = uc[(size_t)yb * wc + xb];
        float a = __builtin_fmaf(fx, p10.x - p00.x, p00.x);
        float b = __builtin_fmaf(fx, p11.x - p01.x, p01.x);
        float cxv = __builtin_fmaf(fy, b - a, a);
        a = __builtin_fmaf(fx, p10.y - p00.y, p00.y);
        b = __builtin_fmaf(fx, p11.y - p01.y, p01.y);
        float cyv = __builtin_fmaf(fy, b - a, a);
        ux = 2.0f * cxv;
        uy = 2.0f * cyv;
    }
    const int r = P->lk_radius;
    const int wx0 = x - r < 0 ? 0 : x - r, wx1 = x + r > w - 1 ? w - 1 : x + r;
    const int wy0 = y - r < 0 ? 0 : y - r, wy1 = y + r > h - 1 ? h - 1 : y + r;
    float g00 = 0.0f, g01 = 0.0f, g11 = 0.0f;
    for (int yy = wy0; yy <= wy1; ++yy)
        for (int xx = wx0; xx <= wx1; ++xx) {
            float ix = sIx[yy - y0 + LK_R_MAX][xx - x0 + LK_R_MAX];
            float iy = sIy[yy - y0 + LK_R_MAX][xx - x0 + LK_R_MAX];
            g00 = __builtin_fmaf(ix, ix, g00);
            g01 = __builtin_fmaf(ix, iy, g01);
            g11 = __builtin_fmaf(iy, iy, g11);
        }
    const float reg = P->lk_lambda * (float)((wy1 - wy0 + 1) * (wx1 - wx0 + 1));
    g00 = g00 + reg;
    g11 = g11 + reg;
    const float det = g00 * g11 - g01 * g01;
    const int iters = P->lk_iters;
    for (int it = 0; it < iters; ++it) {
        const float flx = floorf(ux), fly = floorf(uy);
        const int ox = (int)flx, oy = (int)fly;
        const float fx = ux - flx, fy = uy - fly;
        float bu = 0.0f, bv = 0.0f;
        const bool fast = ox >= -(LK_D + 1) && ox <= LK_D && oy >= -(LK_D + 1) && oy <= LK_D;
        if (fast) {
            for (int yy = wy0; yy <= wy1; ++yy) {
                const float* m0 = sM[yy + oy - y0 + LK_HM];
                const float* m1 = sM[yy + oy + 1 - y0 + LK_HM];
                const float* tr = sT[yy - y0 + LK_HT];
                const float* gxr = sIx[yy - y0 + LK_R_MAX];
                const float* gyr = sIy[yy - y0 + LK_R_MAX];
                for (int xx = wx0; xx <= wx1; ++xx) {
                    const int cx = xx + ox - x0 + LK_HM;
                    float p00 = m0[cx], p10 = m0[cx + 1], p01 = m1[cx], p11 = m1[cx + 1];
                    float a = __builtin_fmaf(fx, p10 - p00, p00);
                    float b = __builtin_fmaf(fx, p11 - p01, p01);
                    float m = __builtin_fmaf(fy, b - a, a);
                    float e = m - tr[xx - x0 + LK_HT];
                    bu = __builtin_fmaf(gxr[xx - x0 + LK_R_MAX], e, bu);
                    bv = __builtin_fmaf(gyr[xx - x0 + LK_R_MAX], e, bv);
                }
            }
        } else {
            for (int yy = wy0; yy <= wy1; ++yy) {
                const float* m0 = Mv + (size_t)clampi(yy + oy, 0, h - 1) * w;
                const float* m1 = Mv + (size_t)clampi(yy + oy + 1, 0, h - 1) * w;
                for (int xx = wx0; xx <= wx1; ++xx) {
                    const int xa = clampi(xx + ox, 0, w - 1), xb = clampi(xx + ox + 1, 0, w - 1);
                    float p00 = m0[xa], p10 = m0[xb], p01 = m1[xa], p11 = m1[xb];
                    float a = __builtin_fmaf(fx, p10 - p00, p00);
                    float b = __builtin_fmaf(fx, p11 - p01, p01);
                    float m = __builtin_fmaf(fy, b - a, a);
                    float e = m - sT[yy - y0 + LK_HT][xx - x0 + LK_HT];
                    bu = __builtin_fmaf(sIx[yy - y0 + LK_R_MAX][xx - x0 + LK_R_MAX], e, bu);
                    bv = __builtin_fmaf(sIy[yy - y0 + LK_R_MAX][xx - x0 + LK_R_MAX], e, bv);
                }
            }
        }
        const float du = (g01 * bv - g11 * bu) / det;
        const float dv = (g01 * bu - g00 * bv) / det;
        ux = ux + du;
        uy = uy + dv;
    }
    P->flow[p][dir][l][(size_t)y * w + x] = make_float2(ux, uy);
}

__global__ __launch_bounds__(256) void k_lk(const Batch B, int l)
{
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    lk_body(B.plan[c], b, l);
}

// 9x9-window form of the same estimator (radius 4), P vertically adjacent
// pixels per thread, a 64 x 4P block tile.  Identical arithmetic in identical
// order; what changes is data movement:
//  - (T, Ix, Iy) of every window position sit in one float4 in LDS, with
//    Ix = Iy = 0 outside the level, so a clipped window needs no predicate:
//    such a tap adds fma(0, e, acc) = acc exactly (acc is never -0);
//  - the P pixels of a thread share each (T, Ix, Iy) row they have in common;
//  - per pixel the horizontally interpolated moving-image rows slide down the
//    window in registers: the bottom row of window row r is the top row of
//    window row r + 1, so each tap costs ~1.1 moving-image LDS reads.
template <int P>
__device__ __forceinline__ void lk_w9_body(const DevPlan* __restrict__ Pl, const int bid, int l)
{
    constexpr int R = LK_R_MAX, NW = 2 * R + 1;
    constexpr int TX = LKW_TX, TY = 4 * P;
    constexpr int TIW = TX + 2 * R, TIH = TY + 2 * R;       // (T, Ix, Iy) window positions
    constexpr int TSW = TIW + 2, TSH = TIH + 2;             // template + gradient halo
    constexpr int HM = R + LK_D + 1;                        // moving-image halo
    constexpr int MW = TX + 2 * HM, MH = TY + 2 * HM;
    __shared__ float4 sTI[TIH * TIW];
    __shared__ float sT[TSH * TSW];
    __shared__ float sM[MH * MW];

    const int f = find_field(Pl->lk_off[l], 2 * Pl->n_pairs, bid);
    const int p = f >> 1, dir = f & 1;
    if (Pl->flow_mode != VS_FLOW_PLAIN && Pl->res->surr_ok[p]) return;   // the pair keeps the surrogate's flows
    const int t = bid - Pl->lk_off[l][f];
    const int w = Pl->lw[p][l], h = Pl->lh[p][l];
    const int x0 = (t % Pl->lk_tx[l][f]) * TX, y0 = (t / Pl->lk_tx[l][f]) * TY;
    const float* __restrict__ Tm = Pl->pyr[p][dir == 0 ? 0 : 1][l];
    const float* __restrict__ Mv = Pl->pyr[p][dir == 0 ? 1 : 0][l];
    const int tid = threadIdx.x;

    for (int i = tid; i < TSH * TSW; i += 256) {
        const int yy = clampi(y0 - R - 1 + i / TSW, 0, h - 1), xx = clampi(x0 - R - 1 + i % TSW, 0, w - 1);
        sT[i] = Tm[(size_t)yy * w + xx];
    }
    for (int i = tid; i < MH * MW; i += 256) {
        const int yy = clampi(y0 - HM + i / MW, 0, h - 1), xx = clampi(x0 - HM + i % MW, 0, w - 1);
        sM[i] = Mv[(size_t)yy * w + xx];
    }
    __syncthreads();
    for (int i = tid; i < TIH * TIW; i += 256) {
        const int gy = i / TIW, gx = i % TIW;
        const int X = x0 - R + gx, Y = y0 - R + gy;
        const int c = (gy + 1) * TSW + gx + 1;
        const bool in = X >= 0 && X < w && Y >= 0 && Y < h;
        const float ix = in ? 0.5f * (sT[c + 1] - sT[c - 1]) : 0.0f;
        const float iy = in ? 0.5f * (sT[c + TSW] - sT[c - TSW]) : 0.0f;
        sTI[i] = make_float4(sT[c], ix, iy, 0.0f);
    }
    __syncthreads();

    const int lane = tid & 63, wv = tid >> 6;
    const int x = x0 + lane;
    const int yb = y0 + wv * P;
    const bool has_coarse = l + 1 < Pl->levels;
    const int ncx = min(x + R, w - 1) - max(x - R, 0) + 1;
    const uint8_t* __restrict__ need = Pl->need[p][l];
    float ux[P], uy[P], g00[P], g01[P], g11[P], det[P];
    bool act[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int y = yb + q;
        act[q] = x < w && y < h && need[(size_t)y * w + x] != 0;
        ux[q] = 0.0f;
        uy[q] = 0.0f;
        if (has_coarse && act[q]) {
            const int wc = Pl->lw[p][l + 1], hc = Pl->lh[p][l + 1];
            const float2* __restrict__ uc = Pl->flow[p][dir][l + 1];
            const float cx = clampf(__builtin_fmaf((float)x, 0.5f, -0.25f), 0.0f, (float)(wc - 1));
            const float cy = clampf(__builtin_fmaf((float)y, 0.5f, -0.25f), 0.0f, (float)(hc - 1));
            const float flx = floorf(cx), fly = floorf(cy);
            const int xa = (int)flx, ya = (int)fly;
            const float fx = cx - flx, fy = cy - fly;
            const int xb = xa + 1 < wc ? xa + 1 : wc - 1;
            const int ybb = ya + 1 < hc ? ya + 1 : hc - 1;
            const float2 p00 = uc[(size_t)ya * wc + xa], p10 = uc[(size_t)ya * wc + xb];
            const float2 p01 = uc[(size_t)ybb * wc + xa], p11 = uc[(size_t)ybb * wc + xb];
            float a = __builtin_fmaf(fx, p10.x - p00.x, p00.x);
            float b = __builtin_fmaf(fx, p11.x - p01.x, p01.x);
            ux[q] = 2.0f * __builtin_fmaf(fy, b - a, a);
            a = __builtin_fmaf(fx, p10.y - p00.y, p00.y);
            b = __builtin_fmaf(fx, p11.y - p01.y, p01.y);
            uy[q] = 2.0f * __builtin_fmaf(fy, b - a, a);
        }
        g00[q] = 0.0f;
        g01[q] = 0.0f;
        g11[q] = 0.0f;
    }
    // normal matrix: rows shared by the P pixels, row-major within each window
#pragma unroll 1
    for (int j = 0; j < P + 2 * R; ++j) {
        float4 ti[NW];
#pragma unroll
        for (int c = 0; c < NW; ++c) ti[c] = sTI[(wv * P + j) * TIW + lane + c];
#pragma unroll
        for (int q = 0; q < P; ++q) {
            if (j - q < 0 || j - q > 2 * R) continue;
#pragma unroll
            for (int c = 0; c < NW; ++c) {
                g00[q] = __builtin_fmaf(ti[c].y, ti[c].y, g00[q]);
                g01[q] = __builtin_fmaf(ti[c].y, ti[c].z, g01[q]);
                g11[q] = __builtin_fmaf(ti[c].z, ti[c].z, g11[q]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int y = yb + q;
        const int ncy = min(y + R, h - 1) - max(y - R, 0) + 1;
        const float reg = act[q] ? Pl->lk_lambda * (float)(ncy * ncx) : 1.0f;
        g00[q] = g00[q] + reg;
        g11[q] = g11[q] + reg;
        det[q] = g00[q] * g11[q] - g01[q] * g01[q];
    }
    const int iters = Pl->lk_iters;
    for (int it = 0; it < iters; ++it) {
        float fx[P], fy[P], bu[P], bv[P];
        int mb[P];
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const float flx = floorf(ux[q]), fly = floorf(uy[q]);
            int ox = (int)flx, oy = (int)fly;
            fx[q] = ux[q] - flx;
            fy[q] = uy[q] - fly;
            bu[q] = 0.0f;
            bv[q] = 0.0f;
            if (act[q] && !(ox >= -(LK_D + 1) && ox <= LK_D && oy >= -(LK_D + 1) && oy <= LK_D)) {
                // the displacement leaves the staged tile: hand the pixel, with its
                // state at the start of this step, to the tail kernel
                const uint32_t slot = atomicAdd(&Pl->acc->lk_qn[l], 1u);
                if (slot < (uint32_t)Pl->lk_qcap[l])
                    Pl->lk_queue[l][slot] = make_uint4((uint32_t)f | ((uint32_t)it << 8),
                                                       (uint32_t)x | ((uint32_t)(yb + q) << 16),
                                                       __float_as_uint(ux[q]), __float_as_uint(uy[q]));
                act[q] = false;
            }
            if (!act[q]) {
                ox = 0;
                oy = 0;
            }
            mb[q] = (wv * P + q - R + HM + oy) * MW + (lane - R + HM + ox);
        }
        float hp[P][NW];
#pragma unroll 1
        for (int j = 0; j < P + 2 * R; ++j) {
            float4 ti[NW];
#pragma unroll
            for (int c = 0; c < NW; ++c) ti[c] = sTI[(wv * P + j) * TIW + lane + c];
#pragma unroll
            for (int q = 0; q < P; ++q) {
                const int jr = j - q;
                if (jr < 0 || jr > 2 * R) continue;
                if (jr == 0) {
                    const float* m0 = sM + mb[q];
                    float v0 = m0[0];
#pragma unroll
                    for (int c = 0; c < NW; ++c) {
                        const float v1 = m0[c + 1];
                        hp[q][c] = __builtin_fmaf(fx[q], v1 - v0, v0);
                        v0 = v1;
                    }
                }
                const float* m1 = sM + mb[q] + (jr + 1) * MW;
                float v0 = m1[0];
#pragma unroll
                for (int c = 0; c < NW; ++c) {
                    const float v1 = m1[c + 1];
                    const float hb = __builtin_fmaf(fx[q], v1 - v0, v0);
                    v0 = v1;
                    const float m = __builtin_fmaf(fy[q], hb - hp[q][c], hp[q][c]);
                    const float e = m - ti[c].x;
                    bu[q] = __builtin_fmaf(ti[c].y, e, bu[q]);
                    bv[q] = __builtin_fmaf(ti[c].z, e, bv[q]);
                    hp[q][c] = hb;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < P; ++q) {
            if (!act[q]) continue;
            const float du = (g01[q] * bv[q] - g11[q] * bu[q]) / det[q];
            const float dv = (g01[q] * bu[q] - g00[q] * bv[q]) / det[q];
            ux[q] = ux[q] + du;
            uy[q] = uy[q] + dv;
        }
    }
#pragma unroll
    for (int q = 0; q < P; ++q)
        if (act[q]) Pl->flow[p][dir][l][(size_t)(yb + q) * w + x] = make_float2(ux[q], uy[q]);
}

template <int P>
__global__ __launch_bounds__(256) void k_lk_w9(const Batch B, int l)
{
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    lk_w9_body<P>(B.plan[c], b, l);
}

// Pixels whose displacement left the staged tile finish here, one pixel per
// lane, every tap read from global memory with clamped indices (gradients 0
// outside the level, as in the staged kernel, so the row-major sums are the
// same).  Each window row issues all of its loads before using them: the
// kernel is latency-bound on about one round trip per window row.
__global__ __launch_bounds__(256) void k_lk_tail(const Batch B, int l)
{
    constexpr int R = LK_R_MAX, NW = 2 * R + 1;
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    const int nb = B.off[c + 1] - B.off[c];          // this context's blocks
    const DevPlan* __restrict__ Pl = B.plan[c];
    const uint32_t n = min(Pl->acc->lk_qn[l], (uint32_t)Pl->lk_qcap[l]);
    const int iters = Pl->lk_iters;
    for (uint32_t i = b * 256 + threadIdx.x; i < n; i += nb * 256) {
        const uint4 ent = Pl->lk_queue[l][i];
        const int f = (int)(ent.x & 255u), it0 = (int)(ent.x >> 8);
        const int x = (int)(ent.y & 0xffffu), y = (int)(ent.y >> 16);
        float ux = __uint_as_float(ent.z), uy = __uint_as_float(ent.w);
        const int p = f >> 1, dir = f & 1;
        const int w = Pl->lw[p][l], h = Pl->lh[p][l];
        const float* __restrict__ Tm = Pl->pyr[p][dir == 0 ? 0 : 1][l];
        const float* __restrict__ Mv = Pl->pyr[p][dir == 0 ? 1 : 0][l];
        int cxm[NW + 2];   // clamped columns x - R - 1 .. x + R + 1
        bool cin[NW];
#pragma unroll
        for (int k = 0; k < NW + 2; ++k) cxm[k] = clampi(x - R - 1 + k, 0, w - 1);
#pragma unroll
        for (int c = 0; c < NW; ++c) cin[c] = x - R + c >= 0 && x - R + c < w;
        float g00 = 0.0f, g01 = 0.0f, g11 = 0.0f;
#pragma unroll
        for (int jr = 0; jr < NW; ++jr) {
            const int yy = y - R + jr;
            const bool rin = yy >= 0 && yy < h;
            const float* t0 = Tm + (size_t)clampi(yy - 1, 0, h - 1) * w;
            const float* t1 = Tm + (size_t)clampi(yy, 0, h - 1) * w;
            const float* t2 = Tm + (size_t)clampi(yy + 1, 0, h - 1) * w;
            float a[NW + 2], up[NW], dn[NW];
#pragma unroll
            for (int k = 0; k < NW + 2; ++k) a[k] = t1[cxm[k]];
#pragma unroll
            for (int c = 0; c < NW; ++c) {
                up[c] = t0[cxm[c + 1]];
                dn[c] = t2[cxm[c + 1]];
            }
#pragma unroll
            for (int c = 0; c < NW; ++c) {
                const bool in = rin && cin[c];
                const float ix = in ? 0.5f * (a[c + 2] - a[c]) : 0.0f;
                const float iy = in ? 0.5f * (dn[c] - up[c]) : 0.0f;
                g00 = __builtin_fmaf(ix, ix, g00);
                g01 = __builtin_fmaf(ix, iy, g01);
                g11 = __builtin_fmaf(iy, iy, g11);
            }
        }
        const int ncx = min(x + R, w - 1) - max(x - R, 0) + 1;
        const int ncy = min(y + R, h - 1) - max(y - R, 0) + 1;
        const float reg = Pl->lk_lambda * (float)(ncy * ncx);
        g00 = g00 + reg;
        g11 = g11 + reg;
        const float det = g00 * g11 - g01 * g01;
        for (int it = it0; it < iters; ++it) {
            const float flx = floorf(ux), fly = floorf(uy);
            const int ox = (int)flx, oy = (int)fly;
            const float fx = ux - flx, fy = uy - fly;
            int mx[NW + 1];
#pragma unroll
            for (int k = 0; k < NW + 1; ++k) mx[k] = clampi(x - R + ox + k, 0, w - 1);
            float bu = 0.0f, bv = 0.0f;
#pragma unroll
            for (int jr = 0; jr < NW; ++jr) {
                const int yy = y - R + jr;
                const bool rin = yy >= 0 && yy < h;
                const float* t0 = Tm + (size_t)clampi(yy - 1, 0, h - 1) * w;
                const float* t1 = Tm + (size_t)clampi(yy, 0, h - 1) * w;
                const float* t2 = Tm + (size_t)clampi(yy + 1, 0, h - 1) * w;
                const float* m0 = Mv + (size_t)clampi(yy + oy, 0, h - 1) * w;
                const float* m1 = Mv + (size_t)clampi(yy + oy + 1, 0, h - 1) * w;
                float a[NW + 2], up[NW], dn[NW], ra[NW + 1], rb[NW + 1];
#pragma unroll
                for (int k = 0; k < NW + 2; ++k) a[k] = t1[cxm[k]];
#pragma unroll
                for (int c = 0; c < NW; ++c) {
                    up[c] = t0[cxm[c + 1]];
                    dn[c] = t2[cxm[c + 1]];
                }
#pragma unroll
                for (int k = 0; k < NW + 1; ++k) {
                    ra[k] = m0[mx[k]];
                    rb[k] = m1[mx[k]];
                }
#pragma unroll
                for (int c = 0; c < NW; ++c) {
                    const bool in = rin && cin[c];
                    const float ix = in ? 0.5f * (a[c + 2] - a[c]) : 0.0f;
                    const float iy = in ? 0.5f * (dn[c] - up[c]) : 0.0f;
                    const float ta = __builtin_fmaf(fx, ra[c + 1] - ra[c], ra[c]);
                    const float tb = __builtin_fmaf(fx, rb[c + 1] - rb[c], rb[c]);
                    const float e = __builtin_fmaf(fy, tb - ta, ta) - a[c + 1];
                    bu = __builtin_fmaf(ix, e, bu);
                    bv = __builtin_fmaf(iy, e, bv);
                }
            }
            const float du = (g01 * bv - g11 * bu) / det;
            const float dv = (g01 * bu - g00 * bv) / det;
            ux = ux + du;
            uy = uy + dv;
        }
        Pl->flow[p][dir][l][(size_t)y * w + x] = make_float2(ux, uy);
    }
}

// Static flow domain (plan time): level 0 = the overlap of the pair's cameras
// on the strip; level l + 1 = the bilinear footprints sampled by the needed
// pixels of level l when initialising from the coarser flow.
__global__ __launch_bounds__(256) void k_need0(const DevPlan* __restrict__ P)
{
    const int tid = threadIdx.x;
    const int p = find_field(P->strip_off, P->n_pairs, blockIdx.x);
    const int t = blockIdx.x - P->strip_off[p];
    const int sw = P->sw[p], sh = P->sh[p];
    const int tx0 = (t % P->strip_tx[p]) * STRIP_TX, ty0 = (t / P->strip_tx[p]) * STRIP_TY;
    const int kj = P->pj[p], ki = P->pi[p];
    const int lx = tx0 + (tid & 63);
    for (int r = tid >> 6; r < STRIP_TY; r += 4) {
        const int ly = ty0 + r;
        if (lx >= sw || ly >= sh) continue;
        const int X = P->sx0[p] + lx, Y = P->sy0[p] + ly;
        float u, v;
        const bool okj = hom(P->hinv[kj], (float)X, (float)Y, P->cam_w[kj], P->cam_h[kj], u, v);
        const bool oki = hom(P->hinv[ki], (float)(X - P->psi[p] * P->Wp), (float)Y, P->cam_w[ki], P->cam_h[ki], u, v);
        P->need[p][0][(size_t)ly * sw + lx] = (okj && oki) ? 1 : 0;
    }
}

__global__ __launch_bounds__(256) void k_need_down(const DevPlan* __restrict__ P, int p, int l)
{
    const int w = P->lw[p][l], h = P->lh[p][l], wc = P->lw[p][l + 1], hc = P->lh[p][l + 1];
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= w * h) return;
    const int x = i % w, y = i / w;
    if (!P->need[p][l][i]) return;
    const float cx = clampf(__builtin_fmaf((float)x, 0.5f, -0.25f), 0.0f, (float)(wc - 1));
    const float cy = clampf(__builtin_fmaf((float)y, 0.5f, -0.25f), 0.0f, (float)(hc - 1));
    const int xa = (int)floorf(cx), ya = (int)floorf(cy);
    const int xb = xa + 1 < wc ? xa + 1 : wc - 1;
    const int yc = ya + 1 < hc ? ya + 1 : hc - 1;
    uint8_t* dst = P->need[p][l + 1];
    dst[(size_t)ya * wc + xa] = 1;
    dst[(size_t)ya * wc + xb] = 1;
    dst[(size_t)yc * wc + xa] = 1;
    dst[(size_t)yc * wc + xb] = 1;
}

hipError_t launch_need(const DevPlan* dp, const DevPlan& hp, hipStream_t s)
{
    hipLaunchKernelGGL(k_need0, dim3(hp.strip_off[hp.n_pairs]), dim3(256), 0, s, dp);
    for (int l = 0; l + 1 < hp.levels; ++l)
        for (int p = 0; p < hp.n_pairs; ++p) {
            const int n = hp.lw[p][l] * hp.lh[p][l];
            hipLaunchKernelGGL(k_need_down, dim3((n + 255) / 256), dim3(256), 0, s, dp, p, l);
        }
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Eqs. (15)-(18): per canvas pixel resample, local warp and weighted fusion,
// plus the histogram of the covered output (input of section 2.2)
// ---------------------------------------------------------------------------

__device__ __forceinline__ void blend_body(const DevPlan* __restrict__ P, const int bid)
{
    // 8 copies of the histogram (lane & 7): neighbouring pixels often share a
    // value, and same-address LDS atomics from one instruction serialise
    __shared__ uint32_t s_hist[8][3 * 256];
    // per-camera constants of the frame, indexed by each lane's own camera
    __shared__ float s_hinv[MAXC][9], s_M[MAXC][9];
    __shared__ int s_cw[MAXC], s_ch[MAXC], s_cp[MAXC];
    __shared__ const uint8_t* s_fr[MAXC];
    const int tid = threadIdx.x;
    for (int i = tid; i < 8 * 3 * 256; i += BL_THREADS) (&s_hist[0][0])[i] = 0;
    for (int i = tid; i < P->n_cams * 9; i += BL_THREADS) {
        (&s_hinv[0][0])[i] = (&P->hinv[0][0])[i];
        (&s_M[0][0])[i] = (&P->res->Mk[0][0])[i];
    }
    if (tid < P->n_cams) {
        s_cw[tid] = P->cam_w[tid];
        s_ch[tid] = P->cam_h[tid];
        s_cp[tid] = P->cam_pitch[tid];
        s_fr[tid] = P->frame[tid];
    }
    __syncthreads();
    uint32_t* const my_hist = s_hist[tid & 7];
    const int bx = bid % P->blend_tx, by = bid / P->blend_tx;
    const int W = P->canvas_w, H = P->canvas_h, Wp = P->Wp;
    const int xq = bx * BL_TX + (tid & 63) * 4;
    const bool vec = (W & 3) == 0;
    for (int r = tid >> 6; r < BL_TY; r += BL_THREADS / 64) {
        const int y = by * BL_TY + r;
        if (y >= H || xq >= W) continue;
        uint32_t ob[12];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int x = xq + q;
            uint32_t o0 = 0, o1 = 0, o2 = 0;
            const uint32_t code = x < W ? P->pix_code[(size_t)y * W + x] : 0u;
            const int nh = (int)(code >> 12);
            if (nh > 0) {
                // the covering (camera, shift) candidates found at plan time, in
                // the coverage scan's order; their positions are evaluated again
                int hc[2] = {0, 0}, hm[2] = {0, 0};
                float hu[2] = {0, 0}, hv[2] = {0, 0};
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    if (e >= nh) break;
                    const int bit = (int)((code >> (6 * e)) & 63u);   // 3 camera + shift + 1
                    const int k = bit / 3, sh = bit % 3 - 1;
                    hc[e] = k;
                    hm[e] = sh;
                    hom(s_hinv[k], (float)(x + sh * Wp), (float)y, s_cw[k], s_ch[k], hu[e], hv[e]);
                }
                if (nh == 1) {
                    const int k = hc[0];
                    float s[3];
                    bilin3(s_fr[k], s_cp[k], s_cw[k], s_ch[k], hu[0], hv[0], s);
                    const float* M = s_M[k];
                    o0 = round8(capply(s, M, 0));
                    o1 = round8(capply(s, M, 1));
                    o2 = round8(capply(s, M, 2));
                } else if (nh >= 2) {
                    const int p = P->pair_of[hc[0]][hc[1]];
                    const int ji = hc[0] == P->pj[p] ? 0 : 1;
                    const int kj = hc[ji], ki = hc[1 - ji];
                    const int mj = hm[ji], mi = hm[1 - ji];
                    float dj = fminf(hu[ji], (float)(s_cw[kj] - 1) - hu[ji]);
                    float di = fminf(hu[1 - ji], (float)(s_cw[ki] - 1) - hu[1 - ji]);
                    if (dj < 0.0f) dj = 0.0f;
                    if (di < 0.0f) di = 0.0f;
                    const float sum = di + dj;
                    const float thi = sum > 0.0f ? di / sum : 0.5f;
                    const float thj = 1.0f - thi;
                    const int lx = x + mj * Wp - P->sx0[p], ly = y - P->sy0[p];
                    const size_t qf = (size_t)ly * P->sw[p] + lx;
                    const float2 fij = P->flow[p][0][0][qf];
                    const float2 fji = P->flow[p][1][0][qf];
                    const float Xi = __builtin_fmaf(thj, fij.x, (float)(x + mi * Wp));
                    const float Yi = __builtin_fmaf(thj, fij.y, (float)y);
                    const float Xj = __builtin_fmaf(thi, fji.x, (float)(x + mj * Wp));
                    const float Yj = __builtin_fmaf(thi, fji.y, (float)y);
                    float u, v, si[3], sj[3];
                    hom(s_hinv[ki], Xi, Yi, s_cw[ki], s_ch[ki], u, v);
                    bilin3(s_fr[ki], s_cp[ki], s_cw[ki], s_ch[ki], u, v, si);
                    hom(s_hinv[kj], Xj, Yj, s_cw[kj], s_ch[kj], u, v);
                    bilin3(s_fr[kj], s_cp[kj], s_cw[kj], s_ch[kj], u, v, sj);
                    const float* Mi = s_M[ki];
                    const float* Mj = s_M[kj];
                    float ti, tj;
                    ti = capply(si, Mi, 0);
                    tj = capply(sj, Mj, 0);
                    o0 = round8(__builtin_fmaf(thi, ti - tj, tj));
                    ti = capply(si, Mi, 1);
                    tj = capply(sj, Mj, 1);
                    o1 = round8(__builtin_fmaf(thi, ti - tj, tj));
                    ti = capply(si, Mi, 2);
                    tj = capply(sj, Mj, 2);
                    o2 = round8(__builtin_fmaf(thi, ti - tj, tj));
                }
                if (nh > 0) {
                    atomicAdd(&my_hist[o0], 1u);
                    atomicAdd(&my_hist[256 + o1], 1u);
                    atomicAdd(&my_hist[512 + o2], 1u);
                }
            }
            ob[q * 3 + 0] = o0;
            ob[q * 3 + 1] = o1;
            ob[q * 3 + 2] = o2;
        }
        uint8_t* row = P->pano + (size_t)y * P->pano_pitch + (size_t)xq * 3;
        if (vec && xq + 3 < W) {
            uint32_t* r32 = (uint32_t*)row;
            r32[0] = ob[0] | (ob[1] << 8) | (ob[2] << 16) | (ob[3] << 24);
            r32[1] = ob[4] | (ob[5] << 8) | (ob[6] << 16) | (ob[7] << 24);
            r32[2] = ob[8] | (ob[9] << 8) | (ob[10] << 16) | (ob[11] << 24);
        } else {
            for (int q = 0; q < 4 && xq + q < W; ++q) {
                row[q * 3 + 0] = (uint8_t)ob[q * 3 + 0];
                row[q * 3 + 1] = (uint8_t)ob[q * 3 + 1];
                row[q * 3 + 2] = (uint8_t)ob[q * 3 + 2];
            }
        }
    }
    __syncthreads();
    uint32_t* gh = &P->acc->pano_hist[0][0];
    for (int i = tid; i < 3 * 256; i += BL_THREADS) {
        uint32_t h = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) h += s_hist[k][i];
        if (h) atomicAdd(&gh[i], h);
    }
}

__global__ __launch_bounds__(BL_THREADS) void k_blend(const Batch B)
{
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    blend_body(B.plan[c], b);
}


// ---------------------------------------------------------------------------
// Section 2.2, eqs. (5)-(7): thresholds, 3-frame mean, piecewise LUT
// ---------------------------------------------------------------------------

__device__ __forceinline__ void balance_lut_body(const DevPlan* __restrict__ P, const int bid)
{
    __shared__ uint32_t C[3][256];
    __shared__ double s_m[3][2];
    __shared__ int s_q[3][2];
    const int v = threadIdx.x;
    vs_color_state* st = P->state;
    Results* res = P->res;
    for (int c = 0; c < 3; ++c) C[c][v] = P->acc->pano_hist[c][v];
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        uint32_t t[3];
        for (int c = 0; c < 3; ++c) t[c] = v >= o ? C[c][v - o] : 0;
        __syncthreads();
        for (int c = 0; c < 3; ++c) C[c][v] += t[c];
        __syncthreads();
    }
    const int pct = P->lambda_pct;
    if (v < 3) {
        const int c = v;
        const unsigned long long n = C[c][255];
        int q1 = -1, q2 = -1;
        for (int k = 0; k < 256; ++k) {
            const unsigned long long Cv = C[c][k];
            if (q1 < 0 && 100ull * Cv >= (unsigned long long)pct * n) q1 = k;
            if (q2 < 0 && 100ull * Cv >= (unsigned long long)(100 - pct) * n) q2 = k;
        }
        if (q1 < 0) q1 = 0;
        if (q2 < 0) q2 = 255;
        const int T = (int)st->frames_seen;
        int s1 = q1, s2 = q2, cnt = 1;
        for (int d = 1; d <= 2 && d <= T; ++d) {
            s1 += st->q[d - 1][c][0];
            s2 += st->q[d - 1][c][1];
            ++cnt;
        }
        s_q[c][0] = q1;
        s_q[c][1] = q2;
        s_m[c][0] = (double)s1 / (double)cnt;
        s_m[c][1] = (double)s2 / (double)cnt;
        res->quant[c][0] = q1;
        res->quant[c][1] = q2;
        res->mbar[c][0] = s_m[c][0];
        res->mbar[c][1] = s_m[c][1];
    }
    __syncthreads();
    const double lam = (double)pct / 100.0;
    const double t1 = 255.0 * lam, t2 = 255.0 * (1.0 - lam);
    for (int c = 0; c < 3; ++c) {
        const double m1 = s_m[c][0], m2 = s_m[c][1];
        uint8_t out;
        if (m2 - m1 < 1.0) {
            out = (uint8_t)v;
        } else {
            const double s = (t2 - t1) / (m2 - m1);
            double g1 = s * m1 / t1, g2 = s * (255.0 - m2) / (255.0 - t2);
            g1 = g1 < 0.125 ? 0.125 : (g1 > 8.0 ? 8.0 : g1);
            g2 = g2 < 0.125 ? 0.125 : (g2 > 8.0 ? 8.0 : g2);
            const double x = (double)v;
            double F;
            if (x < m1) F = t1 * pow(x / m1, g1);
            else if (x <= m2) F = t1 + s * (x - m1);
            else F = 255.0 - (255.0 - t2) * pow((255.0 - x) / (255.0 - m2), g2);
            double fl = floor(F + 0.5);
            fl = fl < 0.0 ? 0.0 : (fl > 255.0 ? 255.0 : fl);
            out = (uint8_t)(int)fl;
        }
        res->bal_lut[c][v] = out;
    }
    __syncthreads();
    if (v == 0) {
        for (int c = 0; c < 3; ++c) {
            st->q[1][c][0] = st->q[0][c][0];
            st->q[1][c][1] = st->q[0][c][1];
            st->q[0][c][0] = s_q[c][0];
            st->q[0][c][1] = s_q[c][1];
        }
        st->frames_seen = st->frames_seen + 1;
    }
}

__global__ __launch_bounds__(256) void k_balance_lut(const Batch B)
{
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    balance_lut_body(B.plan[c], b);
}


__device__ __forceinline__ void balance_apply_body(const DevPlan* __restrict__ P, const int bid)
{
    __shared__ uint8_t s_lut[3][256];
    const int tid = threadIdx.x;
    for (int i = tid; i < 3 * 256; i += BL_THREADS) (&s_lut[0][0])[i] = (&P->res->bal_lut[0][0])[i];
    __syncthreads();
    const int bx = bid % P->blend_tx, by = bid / P->blend_tx;
    const int W = P->canvas_w, H = P->canvas_h;
    const int xq = bx * BL_TX + (tid & 63) * 4;
    const bool vec = (W & 3) == 0;
    for (int r = tid >> 6; r < BL_TY; r += BL_THREADS / 64) {
        const int y = by * BL_TY + r;
        if (y >= H || xq >= W) continue;
        const uint32_t bits = (P->cover[(size_t)y * P->cover_words + (xq >> 5)] >> (xq & 31)) & 15u;
        if (!bits) continue;
        uint8_t* row = P->pano + (size_t)y * P->pano_pitch + (size_t)xq * 3;
        if (vec && xq + 3 < W) {
            uint32_t* r32 = (uint32_t*)row;
            uint32_t w3[3] = {r32[0], r32[1], r32[2]};
            uint32_t o3[3] = {0, 0, 0};
#pragma unroll
            for (int b = 0; b < 12; ++b) {
                uint32_t val = (w3[b >> 2] >> ((b & 3) * 8)) & 255u;
                const int q = b / 3, c = b % 3;
                if ((bits >> q) & 1u) val = s_lut[c][val];
                o3[b >> 2] |= val << ((b & 3) * 8);
            }
            r32[0] = o3[0];
            r32[1] = o3[1];
            r32[2] = o3[2];
        } else {
            for (int q = 0; q < 4 && xq + q < W; ++q) {
                if (!((bits >> q) & 1u)) continue;
                for (int c = 0; c < 3; ++c) row[q * 3 + c] = s_lut[c][row[q * 3 + c]];
            }
        }
    }
}

__global__ __launch_bounds__(BL_THREADS) void k_balance_apply(const Batch B)
{
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    balance_apply_body(B.plan[c], b);
}


// ---------------------------------------------------------------------------
// Launchers: one grid over the tiles of every context of the group
// ---------------------------------------------------------------------------

namespace {

template <typename F>
bool make_batch(const Group& g, Batch& B, F blocks_of)
{
    B.n = g.n;
    B.off[0] = 0;
    for (int c = 0; c < g.n; ++c) {
        B.plan[c] = g.dp[c];
        B.off[c + 1] = B.off[c] + blocks_of(*g.hp[c]);
    }
    for (int c = g.n + 1; c <= MAXB; ++c) B.off[c] = B.off[g.n];
    return B.off[g.n] > 0;
}

}  // namespace

hipError_t launch_set_io(const FrameIO& io, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_io, dim3(n), dim3(64), 0, s, io);
    return hipGetLastError();
}

hipError_t launch_zero(const Group& g, hipStream_t s)
{
    Batch B;
    const int per = (int)((sizeof(Accum) / 16 + 255) / 256);
    if (make_batch(g, B, [&](const DevPlan&) { return per; }))
        hipLaunchKernelGGL(k_zero, dim3(B.off[B.n]), dim3(256), 0, s, B);
    return hipGetLastError();
}

hipError_t launch_strips(const Group& g, hipStream_t s)
{
    Batch B;
    if (make_batch(g, B, [](const DevPlan& h) { return h.strip_off[h.n_pairs]; }))
        hipLaunchKernelGGL(k_strips, dim3(B.off[B.n]), dim3(256), 0, s, B);
    return hipGetLastError();
}

hipError_t launch_lut(const Group& g, hipStream_t s)
{
    Batch B;
    if (make_batch(g, B, [](const DevPlan& h) { return h.n_pairs; }))
        hipLaunchKernelGGL(k_lut, dim3(B.off[B.n]), dim3(256), 0, s, B);
    return hipGetLastError();
}

hipError_t launch_moments_b(const Group& g, hipStream_t s)
{
    Batch B;
    if (make_batch(g, B, [](const DevPlan& h) { return h.strip_off[h.n_pairs]; }))
        hipLaunchKernelGGL(k_moments_b, dim3(B.off[B.n]), dim3(256), 0, s, B);
    return hipGetLastError();
}

hipError_t launch_solve(const Group& g, hipStream_t s)
{
    Batch B;
    if (make_batch(g, B, [](const DevPlan&) { return 1; }))
        hipLaunchKernelGGL(k_solve, dim3(B.off[B.n]), dim3(64), 0, s, B);
    return hipGetLastError();
}

hipError_t launch_pyr0(const Group& g, hipStream_t s)
{
    Batch B;
    if (make_batch(g, B, [](const DevPlan& h) { return h.use_flow ? h.pyr_off[0][2 * h.n_pairs] : 0; }))
        hipLaunchKernelGGL(k_pyr0, dim3(B.off[B.n]), dim3(256), 0, s, B);
    return hipGetLastError();
}

hipError_t launch_pyr_down(const Group& g, int l, hipStream_t s)
{
    Batch B;
    // the surrogate alone reads no level beyond its own
    if (make_batch(g, B, [l](const DevPlan& h) {
            const int top = h.flow_mode == VS_FLOW_SURROGATE ? SURR_LEVEL + 1 : h.levels;
            return h.use_flow && l + 1 < top ? h.pyr_off[l + 1][2 * h.n_pairs] : 0; }))
        hipLaunchKernelGGL(k_pyr_down, dim3(B.off[B.n]), dim3(256), 0, s, B, l);
    return hipGetLastError();
}

hipError_t launch_lk(const Group& g, int l, hipStream_t s)
{
    // every context of a group runs the same flow-kernel variant at a level
    const int P = g.hp[0]->lk_P[l];
    for (int c = 1; c < g.n; ++c)
        if (g.hp[c]->lk_P[l] != P) return hipErrorInvalidValue;
    Batch B;
    // a context whose flows all come from the surrogate launches no flow blocks
    auto plain = [](const DevPlan& h) { return h.use_flow && h.flow_mode != VS_FLOW_SURROGATE; };
    if (make_batch(g, B, [&](const DevPlan& h) { return plain(h) && l < h.levels ? h.lk_off[l][2 * h.n_pairs] : 0; })) {
        const dim3 grid(B.off[B.n]);
        switch (P) {
        case 4: hipLaunchKernelGGL(k_lk_w9<4>, grid, dim3(256), 0, s, B, l); break;
        case 2: hipLaunchKernelGGL(k_lk_w9<2>, grid, dim3(256), 0, s, B, l); break;
        case 1: hipLaunchKernelGGL(k_lk_w9<1>, grid, dim3(256), 0, s, B, l); break;
        default: hipLaunchKernelGGL(k_lk, grid, dim3(256), 0, s, B, l); break;
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || P == 0) return e;
    // deferred pixels: the device-side count bounds the grid-stride loop
    if (make_batch(g, B, [&](const DevPlan& h) {
            return plain(h) && l < h.levels ? std::min(1024, std::max(1, (h.lk_qcap[l] + 255) / 256)) : 0; }))
        hipLaunchKernelGGL(k_lk_tail, dim3(B.off[B.n]), dim3(256), 0, s, B, l);
    return hipGetLastError();
}

hipError_t launch_blend(const Group& g, hipStream_t s)
{
    Batch B;
    if (make_batch(g, B, [](const DevPlan& h) { return h.blend_tx * h.blend_ty; }))
        hipLaunchKernelGGL(k_blend, dim3(B.off[B.n]), dim3(BL_THREADS), 0, s, B);
    return hipGetLastError();
}

hipError_t launch_balance_lut(const Group& g, hipStream_t s)
{
    Batch B;
    if (make_batch(g, B, [](const DevPlan&) { return 1; }))
        hipLaunchKernelGGL(k_balance_lut, dim3(B.off[B.n]), dim3(256), 0, s, B);
    return hipGetLastError();
}

hipError_t launch_balance_apply(const Group& g, hipStream_t s)
{
    Batch B;
    if (make_batch(g, B, [](const DevPlan& h) { return h.balance ? h.blend_tx * h.blend_ty : 0; }))
        hipLaunchKernelGGL(k_balance_apply, dim3(B.off[B.n]), dim3(BL_THREADS), 0, s, B);
    return hipGetLastError();
}

}  // namespace vs
