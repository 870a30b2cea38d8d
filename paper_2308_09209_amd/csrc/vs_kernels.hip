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

#include "vs_device.h"

namespace vs {

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

// n bytes at p <- v (grid-stride; a fill kernel where a caller may capture the
// stream, no memset node)
__global__ __launch_bounds__(256) void k_fill_u8(uint8_t* p, size_t n, uint8_t v)
{
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Section 3.2 flow input of a caller strip (step a5 with the identity colour
// matrix): Y = (77 R + 150 G + 29 B + 128) >> 8 per pixel of an RGB HWC byte
// image, as FP32 (grid-stride)
__global__ __launch_bounds__(256) void k_luma_rgb(const uint8_t* __restrict__ rgb, size_t n, float* __restrict__ y)
{
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        const uint32_t r = rgb[3 * i], g = rgb[3 * i + 1], b = rgb[3 * i + 2];
        y[i] = (float)((77u * r + 150u * g + 29u * b + 128u) >> 8);
    }
}

hipError_t launch_luma_rgb(const uint8_t* rgb, size_t n, float* y, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_luma_rgb, dim3((unsigned)blocks), dim3(256), 0, s, rgb, n, y);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* p, size_t n, uint8_t v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// Frame and panorama pointers of every context of the group, written into its
// device plan before the frame's kernels run (they read them from there, so a
// captured frame graph replays for any input buffers), and the frame's
// accumulators cleared (`per` blocks per context; a fill kernel, no memset):
// the per-pair arrays up to the context's pair count (the entries of the
// other pairs are never written), then the panorama histogram and counters.
__global__ __launch_bounds__(256) void k_set_io(const FrameIO io, int per)
{
    const int c = blockIdx.x / per, b = blockIdx.x % per;
    const int k = threadIdx.x;
    DevPlan* P = io.plan[c];
    if (b == 0) {
        if (k < MAXC) P->frame[k] = io.frame[c][k];
        if (k == 0) P->pano = io.pano[c];
    }
    constexpr uint32_t HW = sizeof(Accum::hist[0]) / 16, CW = sizeof(Accum::csum[0]) / 16;
    constexpr uint32_t MW = sizeof(Accum::mom[0]) / 16;
    constexpr uint32_t TW = (sizeof(Accum) - offsetof(Accum, pano_hist)) / 16;
    const uint32_t np = (uint32_t)P->n_pairs;
    uint4* const a = reinterpret_cast<uint4*>(P->acc);
    uint32_t i = (uint32_t)(b * 256 + k);
    uint4* dst = nullptr;
    if (i < np * HW) {
        dst = a + offsetof(Accum, hist) / 16 + i;
    } else if ((i -= np * HW) < np * CW) {
        dst = a + offsetof(Accum, csum) / 16 + i;
    } else if ((i -= np * CW) < np * MW) {
        dst = a + offsetof(Accum, mom) / 16 + i;
    } else if ((i -= np * MW) < TW) {
        dst = a + offsetof(Accum, pano_hist) / 16 + i;
    }
    if (dst) *dst = make_uint4(0, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Section 2.1 steps 1-2 and eq. (1) A: overlap strips, masks, histograms and
// the exact moment A = sum p p^T of camera i's overlap pixels
// ---------------------------------------------------------------------------


__device__ __forceinline__ void strips_body(const DevPlan* __restrict__ P, const int p, const int t,
                                            uint32_t (*s_hj)[3 * 256 + 1], unsigned long long (*s_hi)[3 * 256 + 1])
{
    // Copies against same-address serialisation (camera j: 4, lane & 3;
    // camera i: 2, lane & 1), each one word longer than the 3 x 256 bins so
    // that a bin's copies sit in different banks.  Camera j: counts.  Camera
    // i: per channel c and level v one 64-bit word, the count in bits 0-11 and
    // the sums of the two other channels in bits 12-31 and 32-63 (a block
    // holds at most 2048 pixels: counts < 2^12, sums < 2048 * 255 < 2^20, so
    // no field carries into the next).
    static_assert(STRIP_TX * STRIP_TY <= 4095, "strip block counts fit 12 bits");
    __shared__ uint32_t s_red[4][7];
    const int tid = threadIdx.x;
    const int sw = P->sw[p], sh = P->sh[p];
    const int tx0 = (t % P->strip_tx[p]) * STRIP_TX, ty0 = (t / P->strip_tx[p]) * STRIP_TY;
    for (int i = tid; i < 4 * (3 * 256 + 1); i += 256) (&s_hj[0][0])[i] = 0;
    for (int i = tid; i < 2 * (3 * 256 + 1); i += 256) (&s_hi[0][0])[i] = 0;
    __syncthreads();
    uint32_t* const my_hj = s_hj[tid & 3];
    unsigned long long* const my_hi = s_hi[tid & 1];

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
            atomicAdd(&my_hj[0 * 256 + cj0], 1u);
            atomicAdd(&my_hj[1 * 256 + cj1], 1u);
            atomicAdd(&my_hj[2 * 256 + cj2], 1u);
            typedef unsigned long long u64;
            atomicAdd(&my_hi[0 * 256 + ci0], 1ull | ((u64)ci1 << 12) | ((u64)ci2 << 32));
            atomicAdd(&my_hi[1 * 256 + ci1], 1ull | ((u64)ci0 << 12) | ((u64)ci2 << 32));
            atomicAdd(&my_hi[2 * 256 + ci2], 1ull | ((u64)ci0 << 12) | ((u64)ci1 << 32));
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
    if (tid < 7) {   // A (6) then n: mom slots 0-6
        unsigned long long s = (unsigned long long)s_red[0][tid] + s_red[1][tid] + s_red[2][tid] + s_red[3][tid];
        if (s) atomicAdd(&acc->mom[p][t % MOM_SPREAD][MOM_A + tid], s);
    }
    uint32_t* gh = &acc->hist[p][t % HIST_SPREAD][0][0][0];
    unsigned long long* gs = &acc->csum[p][t % CSUM_SPREAD][0][0];
    for (int i = tid; i < 3 * 256; i += 256) {
        const uint32_t hj = s_hj[0][i] + s_hj[1][i] + s_hj[2][i] + s_hj[3][i];
        if (hj) atomicAdd(&gh[i], hj);
        const unsigned long long hi = s_hi[0][i] + s_hi[1][i];
        if (hi) {
            const int c = i >> 8, v = i & 255;
            atomicAdd(&gh[3 * 256 + i], (uint32_t)(hi & 0xfffu));
            const unsigned long long s0 = (hi >> 12) & 0xfffffu, s1 = hi >> 32;
            if (s0) atomicAdd(&gs[(2 * c) * 256 + v], s0);
            if (s1) atomicAdd(&gs[(2 * c + 1) * 256 + v], s1);
        }
    }
}

// ---------------------------------------------------------------------------
// Section 2.1 step 3: histogram specification LUT(v) = min{w : C_j(w) >= C_i(v)},
// and eq. (1)'s B = I_i^T I_j with I_j = LUT(I_i) (the histogram-specified
// image i) from the histograms and conditional sums: B[a][c] = sum_v LUT_c(v)
// S_a|c(v), S_c|c(v) = v n_c(v).  256 threads, thread v every channel; Cj,
// Ci: 2 x 768 words of LDS.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void lut_body(const DevPlan* __restrict__ P, const int p)
{
    // one thread per (channel, level): tid = 256 c + v
    __shared__ uint32_t Ci[3][256], Cj[3][256];
    __shared__ unsigned long long s_red[12][3];
    const int tid = threadIdx.x, c = tid >> 8, v = tid & 255;
    const Accum* acc = P->acc;
    uint32_t sj = 0, si = 0;
#pragma unroll 8
    for (int k = 0; k < HIST_SPREAD; ++k) {
        sj += acc->hist[p][k][0][c][v];
        si += acc->hist[p][k][1][c][v];
    }
    const uint32_t ni = si;
    Cj[c][v] = sj;
    Ci[c][v] = si;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint32_t ti = v >= o ? Ci[c][v - o] : 0, tj = v >= o ? Cj[c][v - o] : 0;
        __syncthreads();
        Ci[c][v] += ti;
        Cj[c][v] += tj;
        __syncthreads();
    }
    const uint32_t target = Ci[c][v];
    int lo = 0, hi = 256;   // first w with Cj[w] >= target
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (Cj[c][mid] < target) lo = mid + 1;
        else hi = mid;
    }
    if (P->readings & VS_READ_NEAREST_CDF) {
        // the nearest cumulative count, ties to the lower level: Cj is
        // non-decreasing, so it is Cj[lo] (the first at or above the target)
        // or the first level holding the value just below it
        int w = lo > 255 ? 255 : lo;
        if (lo > 0) {
            const uint32_t below = Cj[c][lo - 1];
            if (lo > 255 || target - below <= Cj[c][lo] - target) {
                int a = 0, b = lo - 1;   // first w with Cj[w] >= below
                while (a < b) {
                    const int mid = (a + b) >> 1;
                    if (Cj[c][mid] < below) a = mid + 1;
                    else b = mid;
                }
                w = a;
            }
        }
        lo = w;
    }
    const uint32_t L = (uint32_t)(lo > 255 ? 255 : lo);
    P->res->lut[p][c][v] = (uint8_t)L;
    // column c of B (row a: channel of I_i, column c: channel of LUT(I_i)),
    // exact: B[c][c] = sum_v v LUT_c(v) n_c(v), B[a][c] = sum_v LUT_c(v) S_a|c(v)
    unsigned long long s0 = 0, s1 = 0;
#pragma unroll
    for (int k = 0; k < CSUM_SPREAD; ++k) {
        s0 += acc->csum[p][k][2 * c][v];
        s1 += acc->csum[p][k][2 * c + 1][v];
    }
    const unsigned long long bd = wave_sum64((unsigned long long)v * L * ni);
    const unsigned long long b0 = wave_sum64(s0 * L), b1 = wave_sum64(s1 * L);
    if ((tid & 63) == 0) {
        s_red[tid >> 6][0] = bd;
        s_red[tid >> 6][1] = b0;
        s_red[tid >> 6][2] = b1;
    }
    __syncthreads();
    if (v < 3) {   // thread (c, k): entry k of column c, its channel's 4 wavefronts in order
        const int w0 = 4 * c;
        const unsigned long long sum = ((s_red[w0][v] + s_red[w0 + 1][v]) + s_red[w0 + 2][v]) + s_red[w0 + 3][v];
        const int a0 = c == 0 ? 1 : 0, a1 = c == 2 ? 1 : 2;   // the two other channels, in order
        const int a = v == 0 ? c : (v == 1 ? a0 : a1);
        P->acc->mom[p][0][MOM_B + a * 3 + c] = sum;
    }
}


// ---------------------------------------------------------------------------
// Eqs. (2)-(4): 3D-M solve (FP64) per pair, chain composition, state shift
// ---------------------------------------------------------------------------

// Column k of M in (A + eps I) M = B + eps I, eps = ridge * trace(A):
// Gaussian elimination with partial pivoting (first largest on ties) and back
// substitution, the column's right-hand side carried through the same row
// operations as the whole matrix would be.  Returns 1 (M = I) when a pivot
// falls below 1e-12 of the largest |entry|.
__device__ int solve3_col(const double* A, const double* Bk, int k, double ridge, double* Mk)
{
    double a[3][3], b[3];
    const double eps = ridge * ((A[0] + A[4]) + A[8]);
    double maxabs = 0.0;
    for (int r = 0; r < 3; ++r) {
        for (int q = 0; q < 3; ++q) {
            a[r][q] = A[r * 3 + q] + (r == q ? eps : 0.0);
            if (fabs(a[r][q]) > maxabs) maxabs = fabs(a[r][q]);
        }
        b[r] = Bk[r] + (r == k ? eps : 0.0);
    }
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        for (int r = col + 1; r < 3; ++r)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (piv != col) {
            for (int q = 0; q < 3; ++q) {
                const double t = a[col][q];
                a[col][q] = a[piv][q];
                a[piv][q] = t;
            }
            const double t = b[col];
            b[col] = b[piv];
            b[piv] = t;
        }
        if (!(fabs(a[col][col]) >= 1e-12 * maxabs) || a[col][col] == 0.0) {
            for (int r = 0; r < 3; ++r) Mk[r] = r == k ? 1.0 : 0.0;
            return 1;
        }
        for (int r = col + 1; r < 3; ++r) {
            const double f = a[r][col] / a[col][col];
            for (int q = col; q < 3; ++q) a[r][q] = a[r][q] - f * a[col][q];
            b[r] = b[r] - f * b[col];
        }
    }
    for (int r = 2; r >= 0; --r) {
        double s = b[r];
        for (int q = r + 1; q < 3; ++q) s = s - a[r][q] * Mk[q];
        Mk[r] = s / a[r][r];
    }
    return 0;
}

// s_M, s_mom: LDS of the calling block (MAXP x 9 doubles, MAXP x 16 sums).
// Three threads per pair, one column of M each; three threads for the chain.
__device__ __forceinline__ void solve_body(const DevPlan* __restrict__ P, double (*s_M)[9],
                                           unsigned long long (*s_mom)[16])
{
    const int tid = threadIdx.x;
    Accum* acc = P->acc;
    Results* res = P->res;
    vs_color_state* st = P->state;
    // the copies of each sum, one (pair, sum) per thread
    static_assert(MAXP * 16 <= SOLVE_THREADS, "one thread per (pair, sum)");
    if (tid < P->n_pairs * 16) {
        const int p = tid >> 4, j = tid & 15;
        unsigned long long s = 0;
#pragma unroll 8
        for (int k = 0; k < MOM_SPREAD; ++k) s += acc->mom[p][k][j];
        s_mom[p][j] = s;
    }
    __syncthreads();
    const int W = P->color_window;
    const int T = (int)st->frames_seen;
    if (tid < 3 * P->n_pairs) {
        const int p = tid / 3, k = tid % 3;
        unsigned long long A3[6], B3[3], n3 = s_mom[p][MOM_N];
        for (int i = 0; i < 6; ++i) A3[i] = s_mom[p][MOM_A + i];
        for (int r = 0; r < 3; ++r) B3[r] = s_mom[p][MOM_B + r * 3 + k];
        for (int d = 1; d < W && d <= T; ++d) {
            const vs_moments* o = &st->mom[p][d - 1];
            for (int i = 0; i < 6; ++i) A3[i] += o->A[i];
            for (int r = 0; r < 3; ++r) B3[r] += o->B[r * 3 + k];
            n3 += o->n;
        }
        double Mk[3] = {k == 0 ? 1.0 : 0.0, k == 1 ? 1.0 : 0.0, k == 2 ? 1.0 : 0.0};
        int flag = 0;
        if (W > 0) {
            if (n3 < (unsigned long long)P->min_pixels) {
                flag = 1;
            } else {
                const double Ad[9] = {(double)A3[0], (double)A3[1], (double)A3[2], (double)A3[1], (double)A3[3],
                                      (double)A3[4], (double)A3[2], (double)A3[4], (double)A3[5]};
                const double Bd[3] = {(double)B3[0], (double)B3[1], (double)B3[2]};
                if (solve3_col(Ad, Bd, k, P->ridge, Mk)) flag = 2;
            }
        }
        for (int r = 0; r < 3; ++r) {
            s_M[p][r * 3 + k] = Mk[r];
            res->Mpair[p][r * 3 + k] = Mk[r];
        }
        if (k == 0) res->flags[p] = flag;
    }
    __syncthreads();   // the window's moments are read: shift the state
    if (tid < P->n_pairs) {
        const int p = tid;
        for (int i = 0; i < 16; ++i) res->mom[p][i < 6 ? i : (i == MOM_N ? 15 : i - 1)] = s_mom[p][i];
        st->mom[p][1] = st->mom[p][0];
        for (int i = 0; i < 6; ++i) st->mom[p][0].A[i] = s_mom[p][MOM_A + i];
        for (int i = 0; i < 9; ++i) st->mom[p][0].B[i] = s_mom[p][MOM_B + i];
        st->mom[p][0].n = s_mom[p][MOM_N];
    } else if (tid >= 64 && tid < 67) {
        // the chain to camera 0 (row vectors, M_k = M_(k-1,k) M_(k-1)), one
        // column c of every M_k per thread
        const int c = tid - 64;
        double m[3] = {c == 0 ? 1.0 : 0.0, c == 1 ? 1.0 : 0.0, c == 2 ? 1.0 : 0.0};
        for (int r = 0; r < 3; ++r) res->Mk[0][r * 3 + c] = (float)m[r];
        for (int k = 1; k < P->n_cams; ++k) {
            const double* a = s_M[k - 1];
            double t[3];
            for (int r = 0; r < 3; ++r) t[r] = (a[r * 3 + 0] * m[0] + a[r * 3 + 1] * m[1]) + a[r * 3 + 2] * m[2];
            for (int r = 0; r < 3; ++r) {
                m[r] = t[r];
                res->Mk[k][r * 3 + c] = (float)t[r];
            }
        }
        // eq. (4)'s text read literally: no whole-frame (composed) correction;
        // each pair's own matrix corrects camera i inside that overlap
        for (int p = 0; p < P->n_pairs; ++p)
            for (int r = 0; r < 3; ++r) res->Mpf[p][r * 3 + c] = (float)s_M[p][r * 3 + c];
        if (P->readings & VS_READ_OVERLAP_ONLY)
            for (int k = 0; k < P->n_cams; ++k)
                for (int r = 0; r < 3; ++r) res->Mk[k][r * 3 + c] = r == c ? 1.0f : 0.0f;
    }
}

// Section 2.1 steps 1-2 and eq. (1)'s A and B sums over every strip pixel of
// every pair.
__global__ __launch_bounds__(256) void k_strips(const Batch B)
{
    __shared__ uint32_t s_hj[4][3 * 256 + 1];
    __shared__ unsigned long long s_hi[2][3 * 256 + 1];
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    const DevPlan* __restrict__ P = B.plan[c];
    const int p = find_field(P->strip_off, P->n_pairs, b);
    strips_body(P, p, b - P->strip_off[p], s_hj, s_hi);
}

// Section 2.1 step 3 and eq. (1)'s B: one block per pair.
__global__ __launch_bounds__(768) void k_lut(const Batch B)
{
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    lut_body(B.plan[c], b);
}

// Eqs. (2)-(4): one block per context.
__global__ __launch_bounds__(SOLVE_THREADS) void k_solve(const Batch B)
{
    __shared__ double s_M[MAXP][9];
    __shared__ unsigned long long s_mom[MAXP][16];
    int c;
    batch_block(B, blockIdx.x, c);
    solve_body(B.plan[c], s_M, s_mom);
}


// ---------------------------------------------------------------------------
// Flow input: luma of the colour-corrected strips, then the 2x pyramid
// ---------------------------------------------------------------------------

// skip_kept: launched after the surrogate's decisions, for the plain
// estimator of the pairs that did not keep its flows
__device__ __forceinline__ void pyr0_body(const DevPlan* __restrict__ P, const int bid, int skip_kept)
{
    const int f = find_field(P->pyr_off[0], 2 * P->n_pairs, bid);
    const int p = f >> 1, cam = f & 1;
    if (skip_kept && kept_by_surrogate(P, p)) return;
    const int t = bid - P->pyr_off[0][f];
    const int w = P->sw[p], h = P->sh[p];
    const int tx0 = (t % P->pyr_tx[0][f]) * PYR_TX, ty0 = (t / P->pyr_tx[0][f]) * PYR_TY;
    const float* M = P->res->Mk[cam == 0 ? P->pj[p] : P->pi[p]];
    // overlap-only reading: camera i's pair matrix inside the overlap mask
    const float* Mo = (cam == 1 && (P->readings & VS_READ_OVERLAP_ONLY)) ? P->res->Mpf[p] : nullptr;
    const uint8_t* __restrict__ mk = P->mask[p];
    const uint32_t* __restrict__ src = P->strip[p] + (size_t)cam * h * w;
    float* __restrict__ dst = P->pyr[p][cam][0];
    const int x = tx0 + (threadIdx.x & 63);
    // every row's load issued before any is used
    constexpr int NR = PYR_TY / 4;
    uint32_t pix[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int y = ty0 + (threadIdx.x >> 6) + 4 * k;
        pix[k] = (x < w && y < h) ? src[(size_t)y * w + x] : 0u;
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int y = ty0 + (threadIdx.x >> 6) + 4 * k;
        if (x >= w || y >= h) continue;
        float s[3] = {(float)(pix[k] & 255u), (float)((pix[k] >> 8) & 255u), (float)((pix[k] >> 16) & 255u)};
        const float* Mx = (Mo && mk[(size_t)y * w + x]) ? Mo : M;
        uint32_t c0 = round8(capply(s, Mx, 0)), c1 = round8(capply(s, Mx, 1)), c2 = round8(capply(s, Mx, 2));
        dst[(size_t)y * w + x] = (float)((77u * c0 + 150u * c1 + 29u * c2 + 128u) >> 8);
    }
}

__global__ __launch_bounds__(256) void k_pyr0(const Batch B, int skip_kept)
{
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    pyr0_body(B.plan[c], b, skip_kept);
}



// level l -> l + 1: separable [1 4 6 4 1] / 16, horizontal first, clamped,
// even positions; each pass ((((a0 + 4 a1) + 6 a2) + 4 a3) + a4) / 16
__device__ __forceinline__ void pyr_down_body(const DevPlan* __restrict__ P, const int bid, int l, int skip_kept)
{
    const int lo = l + 1;
    const int f = find_field(P->pyr_off[lo], 2 * P->n_pairs, bid);
    const int p = f >> 1, cam = f & 1;
    if (skip_kept && kept_by_surrogate(P, p)) return;
    const int t = bid - P->pyr_off[lo][f];
    const int ws = P->lw[p][l], hs = P->lh[p][l];
    const int wd = P->lw[p][lo], hd = P->lh[p][lo];
    const int tx0 = (t % P->pyr_tx[lo][f]) * PYR_TX, ty0 = (t / P->pyr_tx[lo][f]) * PYR_TY;
    const float* __restrict__ src = P->pyr[p][cam][l];
    float* __restrict__ dst = P->pyr[p][cam][lo];
    const int x = tx0 + (threadIdx.x & 63);
    const int xs[5] = {clampi(2 * x - 2, 0, ws - 1), clampi(2 * x - 1, 0, ws - 1), clampi(2 * x, 0, ws - 1),
                       clampi(2 * x + 1, 0, ws - 1), clampi(2 * x + 2, 0, ws - 1)};
    // every source index is clamped into the level, so all rows are computed
    // (their loads scheduled together) and only the stores are predicated
#pragma unroll
    for (int r = threadIdx.x >> 6; r < PYR_TY; r += 4) {
        const int y = ty0 + r;
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
        if (x < wd && y < hd) dst[(size_t)y * wd + x] = acc * 0.0625f;
    }
}

__global__ __launch_bounds__(256) void k_pyr_down(const Batch B, int l, int skip_kept)
{
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    pyr_down_body(B.plan[c], b, l, skip_kept);
}

// Levels 0-2 in one pass (pyramids of 3 or more levels).  A block takes a
// PF_TX x PF_TY tile of level 2 of one field.  The level-0 luma of the tile's
// footprint at clamped positions (4 PF_TX + 9 columns, 4 PF_TY + 9 rows)
// goes to LDS as bytes, level 1 at the footprint's clamped positions is
// reduced from it, level 2 from that: every horizontal and vertical sum is
// the one pyr0 / pyr_down compute, with the same operands in the same order,
// done once per block instead of once per output row.  The tile interiors of
// levels 0 and 1 are written too when the plain estimator reads them this
// frame (VS_FLOW_PLAIN); otherwise only level 2, the surrogate's input.

__device__ __forceinline__ float tap5(float a0, float a1, float a2, float a3, float a4)
{
    float acc = a0 + 4.0f * a1;
    acc = acc + 6.0f * a2;
    acc = acc + 4.0f * a3;
    acc = acc + a4;
    return acc * 0.0625f;
}

template <int PF_TY>
__device__ __forceinline__ void pyr_fused_body(const DevPlan* __restrict__ P, const int bid, int after)
{
    constexpr int PF_W1 = 2 * PF_TX + 3, PF_H1 = 2 * PF_TY + 3;     // level-1 footprint
    constexpr int PF_W0 = 4 * PF_TX + 9, PF_H0 = 4 * PF_TY + 9;     // level-0 footprint
    __shared__ uint8_t s0[PF_H0][PF_W0 + 3];
    __shared__ float sh[PF_H0 * PF_W1];    // level-0 rows at level-1 columns; then level-1 rows at level-2 columns
    __shared__ float s1[PF_H1][PF_W1];
    const int tid = threadIdx.x;
    const int f = find_field(P->pyrf_off, 2 * P->n_pairs, bid);
    const int p = f >> 1, cam = f & 1;
    if (after && kept_by_surrogate(P, p)) return;
    const int t = bid - P->pyrf_off[f];
    const int w0 = P->lw[p][0], h0 = P->lh[p][0];
    const int w1 = P->lw[p][1], h1 = P->lh[p][1];
    const int w2 = P->lw[p][2], h2 = P->lh[p][2];
    const int X0 = (t % P->pyrf_tx[f]) * PF_TX, Y0 = (t / P->pyrf_tx[f]) * PF_TY;
    const int bx0 = 4 * X0 - 6, by0 = 4 * Y0 - 6;       // footprint origins, before clamping
    const int bx1 = 2 * X0 - 2, by1 = 2 * Y0 - 2;
    const bool write01 = P->flow_mode == VS_FLOW_PLAIN || after;
    const float* M = P->res->Mk[cam == 0 ? P->pj[p] : P->pi[p]];
    // overlap-only reading: camera i's pair matrix inside the overlap mask
    const float* Mo = (cam == 1 && (P->readings & VS_READ_OVERLAP_ONLY)) ? P->res->Mpf[p] : nullptr;
    const uint8_t* __restrict__ mk = P->mask[p];
    const uint32_t* __restrict__ src = P->strip[p] + (size_t)cam * h0 * w0;
    float* __restrict__ L0 = P->pyr[p][cam][0];
    float* __restrict__ L1 = P->pyr[p][cam][1];
    float* __restrict__ L2 = P->pyr[p][cam][2];

    // level 0: luma of the colour-corrected strip, 8 loads in flight per thread
    constexpr int N0 = PF_H0 * PF_W0, NB = 8;
    for (int i0 = 0; i0 < N0; i0 += 256 * NB) {
        uint32_t pix[NB];
        bool inm[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const int i = i0 + k * 256 + tid;
            pix[k] = 0u;
            inm[k] = false;
            if (i < N0) {
                const int yy = clampi(by0 + i / PF_W0, 0, h0 - 1), xx = clampi(bx0 + i % PF_W0, 0, w0 - 1);
                pix[k] = src[(size_t)yy * w0 + xx];
                if (Mo) inm[k] = mk[(size_t)yy * w0 + xx] != 0;
            }
        }
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const int i = i0 + k * 256 + tid;
            if (i >= N0) continue;
            const float s[3] = {(float)(pix[k] & 255u), (float)((pix[k] >> 8) & 255u),
                                (float)((pix[k] >> 16) & 255u)};
            const float* Mx = inm[k] ? Mo : M;
            const uint32_t c0 = round8(capply(s, Mx, 0)), c1 = round8(capply(s, Mx, 1)), c2 = round8(capply(s, Mx, 2));
            const uint32_t Y = (77u * c0 + 150u * c1 + 29u * c2 + 128u) >> 8;
            const int r = i / PF_W0, c = i % PF_W0;
            s0[r][c] = (uint8_t)Y;
            if (write01 && r >= 6 && r < 6 + 4 * PF_TY && c >= 6 && c < 6 + 4 * PF_TX) {
                const int yy = by0 + r, xx = bx0 + c;
                if (yy < h0 && xx < w0) L0[(size_t)yy * w0 + xx] = (float)Y;
            }
        }
    }
    __syncthreads();
    // level 1, horizontal: footprint rows at level-1 columns clamp(bx1 + i)
    for (int i = tid; i < PF_H0 * PF_W1; i += 256) {
        const int r = i / PF_W1, c1 = clampi(bx1 + i % PF_W1, 0, w1 - 1);
        const uint8_t* row = s0[r];
        float a[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) a[k] = (float)row[clampi(2 * c1 - 2 + k, 0, w0 - 1) - bx0];
        sh[i] = tap5(a[0], a[1], a[2], a[3], a[4]);
    }
    __syncthreads();
    // level 1, vertical: at level-1 rows clamp(by1 + j)
    for (int i = tid; i < PF_H1 * PF_W1; i += 256) {
        const int j = i / PF_W1, c = i % PF_W1;
        const int r1 = clampi(by1 + j, 0, h1 - 1);
        float a[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) a[k] = sh[(clampi(2 * r1 - 2 + k, 0, h0 - 1) - by0) * PF_W1 + c];
        const float v = tap5(a[0], a[1], a[2], a[3], a[4]);
        s1[j][c] = v;
        if (write01 && j >= 2 && j < 2 + 2 * PF_TY && c >= 2 && c < 2 + 2 * PF_TX) {
            const int yy = by1 + j, xx = bx1 + c;
            if (yy < h1 && xx < w1) L1[(size_t)yy * w1 + xx] = v;
        }
    }
    __syncthreads();
    // level 2, horizontal (into sh, free again)
    for (int i = tid; i < PF_H1 * PF_TX; i += 256) {
        const int j = i / PF_TX, x2 = X0 + i % PF_TX;
        float a[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) a[k] = s1[j][clampi(2 * x2 - 2 + k, 0, w1 - 1) - bx1];
        sh[i] = tap5(a[0], a[1], a[2], a[3], a[4]);
    }
    __syncthreads();
    // level 2, vertical
    for (int i = tid; i < PF_TY * PF_TX; i += 256) {
        const int y2 = Y0 + i / PF_TX, xi = i % PF_TX, x2 = X0 + xi;
        float a[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) a[k] = sh[(clampi(2 * y2 - 2 + k, 0, h1 - 1) - by1) * PF_TX + xi];
        if (x2 < w2 && y2 < h2) L2[(size_t)y2 * w2 + x2] = tap5(a[0], a[1], a[2], a[3], a[4]);
    }
}

// after: launched after the surrogate's decisions for the pairs that did not
// keep its flows (levels 0 and 1 written; level 2 again, the same values)
template <int PF_TY>
__global__ __launch_bounds__(256) void k_pyr_fused(const Batch B, int after)
{
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    pyr_fused_body<PF_TY>(B.plan[c], b, after);
}


// ---------------------------------------------------------------------------
// Eqs. (15)-(18): per canvas pixel resample, local warp and weighted fusion,
// plus the histogram of the covered output (input of section 2.2)
// ---------------------------------------------------------------------------

// s_hist: 8 copies of the histogram (lane & 7), LDS of the calling block:
// neighbouring pixels often share a value, and same-address LDS atomics from
// one instruction serialise (+ 1: a bin's copies in different banks)
//
// A thread's 4 pixels of a row: their 4 codes read at once, then per group of
// BG pixels three phases, so that the memory reads of a group are in flight
// together: (1) the covering candidates and their positions; the flows of the
// two-camera pixels; (2) the bilinear taps of every sample (one camera: at its
// position; two cameras: at the positions their flows move them to); (3)
// colour correction, fusion, histogram.
__device__ __forceinline__ void blend_body(const DevPlan* __restrict__ P, const int bid,
                                           uint32_t (*s_hist)[3 * 256 + 1])
{
    // per-camera constants of the frame, indexed by each lane's own camera
    __shared__ float s_hinv[MAXC][9], s_M[MAXC][9];
    __shared__ int s_cw[MAXC], s_ch[MAXC], s_cp[MAXC];
    __shared__ const uint8_t* s_fr[MAXC];
    // per-pair constants: pair of two cameras, camera j, flow-domain origin and
    // width, the two level-0 flows
    __shared__ int8_t s_pair[MAXC][MAXC];
    __shared__ int s_pj[MAXP], s_fx0[MAXP], s_fy0[MAXP], s_fw[MAXP];
    __shared__ const float2* s_fl[MAXP][2];
    const int tid = threadIdx.x;
    for (int i = tid; i < 8 * (3 * 256 + 1); i += BL_THREADS) (&s_hist[0][0])[i] = 0;
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
    if (tid < MAXC * MAXC) (&s_pair[0][0])[tid] = (int8_t)(&P->pair_of[0][0])[tid];
    if (tid < P->n_pairs) {
        s_pj[tid] = P->pj[tid];
        s_fx0[tid] = P->sx0[tid];
        s_fy0[tid] = P->sy0[tid];
        s_fw[tid] = P->sw[tid];
        s_fl[tid][0] = P->flow[tid][0][0];
        s_fl[tid][1] = P->flow[tid][1][0];
    }
    __syncthreads();
    uint32_t* const my_hist = s_hist[tid & 7];
    const int bx = bid % P->blend_tx, by = bid / P->blend_tx;
    const int W = P->canvas_w, H = P->canvas_h, Wp = P->Wp;
    const bool lit = (P->readings & VS_READ_LITERAL_EQ17) != 0;
    const bool ovl_only = (P->readings & VS_READ_OVERLAP_ONLY) != 0;
    // wavefront w takes the 64 columns [64 w, 64 w + 64) of the tile, 16 lanes
    // of 4 pixels per row, 4 rows at a time: a wavefront's pixels lie in one
    // narrow band, so few of them straddle the edge of an overlap (where both
    // the one-camera and the two-camera code would run)
    static_assert(BL_TX == 64 * (BL_THREADS / 64) && BL_TY % 4 == 0, "blend tile = 4 x 64-column bands");
    const int xq = bx * BL_TX + (tid >> 6) * 64 + (tid & 15) * 4;
    const bool vec = (W & 3) == 0;
    // pixels whose phases run together: 1 (with the 4 codes read at once and
    // the pair constants in LDS); 2 and 4 need 127 and 162 VGPRs and were
    // slower (4 x 1080p blend 71 -> 78 / 92 us)
    constexpr int BG = 1;
    for (int r = (tid & 63) >> 4; r < BL_TY; r += 4) {
        const int y = by * BL_TY + r;
        if (y >= H || xq >= W) continue;
        // (1) candidates: bits 0-5 and 6-11 (3 camera + shift + 1), bits 12+ their count
        uint32_t code[4];
        if (vec && xq + 3 < W) {
            typedef uint32_t u2v __attribute__((ext_vector_type(2)));
            const u2v c4 = *gmem((const u2v*)(P->pix_code + (size_t)y * W + xq));
            code[0] = c4.x & 0xffffu;
            code[1] = c4.x >> 16;
            code[2] = c4.y & 0xffffu;
            code[3] = c4.y >> 16;
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) code[q] = xq + q < W ? gmem(P->pix_code)[(size_t)y * W + xq + q] : 0u;
        }
        uint32_t ob[3] = {0u, 0u, 0u};
#pragma unroll
        for (int g = 0; g < 4; g += BG) {
            int nh[BG], ka[BG], kb[BG], pq[BG];
            float th[BG], ua[BG], va[BG];
            typedef float f2v __attribute__((ext_vector_type(2)));
            f2v fij[BG], fji[BG];
#pragma unroll
            for (int q = 0; q < BG; ++q) {
                const int x = xq + g + q;
                nh[q] = (int)(code[g + q] >> 12);
                ka[q] = 0;
                kb[q] = 0;
                pq[q] = 0;
                th[q] = 0.0f;
                ua[q] = 0.0f;
                va[q] = 0.0f;
                if (nh[q] <= 0) continue;
                // the covering (camera, shift) candidates found at plan time, in the
                // coverage scan's order; their positions are evaluated again
                int hc[2] = {0, 0}, hm[2] = {0, 0};
                float hu[2] = {0, 0}, hv[2] = {0, 0};
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    if (e >= nh[q]) break;
                    const int bit = (int)((code[g + q] >> (6 * e)) & 63u);
                    const int k = bit / 3, sh = bit % 3 - 1;
                    hc[e] = k;
                    hm[e] = sh;
                    hom(s_hinv[k], (float)(x + sh * Wp), (float)y, s_cw[k], s_ch[k], hu[e], hv[e]);
                }
                if (nh[q] == 1) {
                    ka[q] = hc[0];
                    ua[q] = hu[0];
                    va[q] = hv[0];
                    continue;
                }
                const int p = s_pair[hc[0]][hc[1]];
                const int ji = hc[0] == s_pj[p] ? 0 : 1;
                const int kj = hc[ji], ki = hc[1 - ji];
                const int mj = hm[ji], mi = hm[1 - ji];
                float dj = fminf(hu[ji], (float)(s_cw[kj] - 1) - hu[ji]);
                float di = fminf(hu[1 - ji], (float)(s_cw[ki] - 1) - hu[1 - ji]);
                if (dj < 0.0f) dj = 0.0f;
                if (di < 0.0f) di = 0.0f;
                const float sum = di + dj;
                th[q] = sum > 0.0f ? di / sum : 0.5f;
                const int lx = x + mj * Wp - s_fx0[p], ly = y - s_fy0[p];
                const size_t qf = (size_t)ly * s_fw[p] + lx;
                fij[q] = gmem((const f2v*)s_fl[p][0])[qf];
                fji[q] = gmem((const f2v*)s_fl[p][1])[qf];
                ka[q] = ki;
                kb[q] = kj;
                pq[q] = p;
                // the canvas columns of the two samples, shifts included
                ua[q] = (float)(x + mi * Wp);
                va[q] = (float)(x + mj * Wp);
            }
            // (2) bilinear taps: sample a (one camera, or camera i), sample b (camera j)
            BilTaps ta[BG], tb[BG];
#pragma unroll
            for (int q = 0; q < BG; ++q) {
                if (nh[q] == 1) {
                    const int k = ka[q];
                    bil_load(s_fr[k], s_cp[k], s_cw[k], s_ch[k], ua[q], va[q], ta[q]);
                } else if (nh[q] >= 2) {
                    // eq. (17): camera i moves by theta_j flow_ij, camera j by theta_i
                    // flow_ji (as printed: theta_i and theta_j, VS_READ_LITERAL_EQ17)
                    const float thi = th[q], thj = 1.0f - thi;
                    const float wi = lit ? thi : thj, wj = lit ? thj : thi;
                    const float Xi = __builtin_fmaf(wi, fij[q].x, ua[q]);
                    const float Yi = __builtin_fmaf(wi, fij[q].y, (float)y);
                    const float Xj = __builtin_fmaf(wj, fji[q].x, va[q]);
                    const float Yj = __builtin_fmaf(wj, fji[q].y, (float)y);
                    const int ki = ka[q], kj = kb[q];
                    float u, v;
                    hom(s_hinv[ki], Xi, Yi, s_cw[ki], s_ch[ki], u, v);
                    bil_load(s_fr[ki], s_cp[ki], s_cw[ki], s_ch[ki], u, v, ta[q]);
                    hom(s_hinv[kj], Xj, Yj, s_cw[kj], s_ch[kj], u, v);
                    bil_load(s_fr[kj], s_cp[kj], s_cw[kj], s_ch[kj], u, v, tb[q]);
                }
            }
            // (3) colour correction and fusion, eq. (18)
#pragma unroll
            for (int q = 0; q < BG; ++q) {
                uint32_t o0 = 0, o1 = 0, o2 = 0;
                if (nh[q] == 1) {
                    float s[3];
                    bil_rgb(ta[q], s);
                    const float* M = s_M[ka[q]];
                    o0 = round8(capply(s, M, 0));
                    o1 = round8(capply(s, M, 1));
                    o2 = round8(capply(s, M, 2));
                } else if (nh[q] >= 2) {
                    float si[3], sj[3];
                    bil_rgb(ta[q], si);
                    bil_rgb(tb[q], sj);
                    // overlap-only reading: camera i's own pair matrix (camera j's is I)
                    const float* Mi = ovl_only ? P->res->Mpf[pq[q]] : s_M[ka[q]];
                    const float* Mj = s_M[kb[q]];
                    const float thi = th[q];
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
                if (nh[q] > 0) {
                    atomicAdd(&my_hist[o0], 1u);
                    atomicAdd(&my_hist[256 + o1], 1u);
                    atomicAdd(&my_hist[512 + o2], 1u);
                }
                // byte 3 n + c of the thread's 12 output bytes (pixel n, channel c)
                const int n3 = (g + q) * 3;
                ob[n3 >> 2] |= o0 << (8 * (n3 & 3));
                ob[(n3 + 1) >> 2] |= o1 << (8 * ((n3 + 1) & 3));
                ob[(n3 + 2) >> 2] |= o2 << (8 * ((n3 + 2) & 3));
            }
        }
        uint8_t* const prow = P->pano + (size_t)y * P->pano_pitch + (size_t)xq * 3;
        auto* row = gmem(prow);
        if (vec && xq + 3 < W) {
            auto* r32 = gmem((uint32_t*)prow);
            r32[0] = ob[0];
            r32[1] = ob[1];
            r32[2] = ob[2];
        } else {
            for (int b = 0; b < 12 && xq + b / 3 < W; ++b) row[b] = (uint8_t)(ob[b >> 2] >> (8 * (b & 3)));
        }
    }
    __syncthreads();
    uint32_t* gh = &P->acc->pano_hist[bid % PANO_SPREAD][0][0];
    for (int i = tid; i < 3 * 256; i += BL_THREADS) {
        uint32_t h = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) h += s_hist[k][i];
        if (h) atomicAdd(&gh[i], h);
    }
}



// ---------------------------------------------------------------------------
// Section 2.2, eqs. (5)-(7): thresholds, 3-frame mean, piecewise LUT
// ---------------------------------------------------------------------------

// Eqs. (15)-(18) over every canvas tile.
__global__ __launch_bounds__(BL_THREADS) void k_blend(const Batch B)
{
    __shared__ uint32_t s_hist[8][3 * 256 + 1];
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    blend_body(B.plan[c], b, s_hist);
}

__device__ __forceinline__ void balance_lut_body(const DevPlan* __restrict__ P, const int bid)
{
    // one thread per (channel, level): tid = 256 c + v
    __shared__ uint32_t C[3][256];
    __shared__ double s_m[3][2];
    __shared__ int s_q[3][2];
    const int tid = threadIdx.x, c = tid >> 8, v = tid & 255;
    vs_color_state* st = P->state;
    Results* res = P->res;
    uint32_t hs = 0;
    for (int k = 0; k < PANO_SPREAD; ++k) hs += P->acc->pano_hist[k][c][v];
    C[c][v] = hs;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint32_t t = v >= o ? C[c][v - o] : 0;
        __syncthreads();
        C[c][v] += t;
        __syncthreads();
    }
    // q1, q2: the first levels whose cumulative counts reach lambda n and
    // (1 - lambda) n (the cumulative counts never decrease, so exactly one
    // level satisfies "reached here, not before")
    const int pct = P->lambda_pct;
    const unsigned long long n = C[c][255];
    const unsigned long long Cv = C[c][v], Cp = v > 0 ? C[c][v - 1] : 0ull;
    const unsigned long long lo = (unsigned long long)pct * n, hi = (unsigned long long)(100 - pct) * n;
    if (100ull * Cv >= lo && (v == 0 || 100ull * Cp < lo)) s_q[c][0] = v;
    if (100ull * Cv >= hi && (v == 0 || 100ull * Cp < hi)) s_q[c][1] = v;
    __syncthreads();
    if (v == 0) {
        const int q1 = s_q[c][0], q2 = s_q[c][1];
        const int T = (int)st->frames_seen;
        int s1 = q1, s2 = q2, cnt = 1;
        for (int d = 1; d <= 2 && d <= T; ++d) {
            s1 += st->q[d - 1][c][0];
            s2 += st->q[d - 1][c][1];
            ++cnt;
        }
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
    {
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
    if (tid == 0) {
        for (int ch = 0; ch < 3; ++ch) {
            st->q[1][ch][0] = st->q[0][ch][0];
            st->q[1][ch][1] = st->q[0][ch][1];
            st->q[0][ch][0] = s_q[ch][0];
            st->q[0][ch][1] = s_q[ch][1];
        }
        st->frames_seen = st->frames_seen + 1;
    }
}

__global__ __launch_bounds__(768) void k_balance_lut(const Batch B)
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


hipError_t launch_set_io(const FrameIO& io, int n, int max_pairs, hipStream_t s)
{
    const size_t words = (size_t)max_pairs * ((sizeof(Accum::hist[0]) + sizeof(Accum::csum[0]) + sizeof(Accum::mom[0])) / 16) +
                         (sizeof(Accum) - offsetof(Accum, pano_hist)) / 16;
    const int per = (int)((words + 255) / 256);
    hipLaunchKernelGGL(k_set_io, dim3(n * per), dim3(256), 0, s, io, per);
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
        hipLaunchKernelGGL(k_lut, dim3(B.off[B.n]), dim3(768), 0, s, B);
    return hipGetLastError();
}

hipError_t launch_solve(const Group& g, hipStream_t s)
{
    Batch B;
    if (make_batch(g, B, [](const DevPlan&) { return 1; }))
        hipLaunchKernelGGL(k_solve, dim3(B.off[B.n]), dim3(SOLVE_THREADS), 0, s, B);
    return hipGetLastError();
}

// Which contexts a level-by-level pyramid launch covers: PYR_ALL every flow
// context (the label context); PYR_UNFUSED those with fewer than 3 levels,
// before the surrogate; PYR_AFTER, after the surrogate's decisions, the levels
// above 2 of any context with plain flow, pairs that kept the surrogate's
// flows skipping them.  Levels 0-2 of pyramids with 3 or more levels come from
// k_pyr_fused: before the surrogate (all three for plain flow, level 2 in the
// surrogate modes) and, in fallback mode, after it for the pairs not kept.
static bool pyr_level_launched(const DevPlan& h, int lo, int phase)
{
    if (!h.use_flow || lo >= h.levels) return false;
    if (phase == PYR_ALL) return true;
    const bool fused = h.levels >= 3;
    if (phase == PYR_UNFUSED) return !fused;
    if (!fused) return false;
    if (lo <= 2) return false;   // levels 0-2: the fused kernel, before and (fallback) after
    return h.flow_mode != VS_FLOW_SURROGATE;
}

hipError_t launch_pyr0(const Group& g, int phase, hipStream_t s)
{
    Batch B;
    if (make_batch(g, B, [&](const DevPlan& h) {
            return pyr_level_launched(h, 0, phase) ? h.pyr_off[0][2 * h.n_pairs] : 0; }))
        hipLaunchKernelGGL(k_pyr0, dim3(B.off[B.n]), dim3(256), 0, s, B, phase == PYR_AFTER ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_pyr_fused(const Group& g, int phase, hipStream_t s)
{
    const bool after = phase == PYR_AFTER;
    // one launch per tile height present in the group
    for (const int ty : {16, 8}) {
        Batch B;
        if (make_batch(g, B, [&](const DevPlan& h) {
                const bool on = h.use_flow && h.levels >= 3 && h.pyrf_ty == ty &&
                                (!after || h.flow_mode == VS_FLOW_SURROGATE_FALLBACK);
                return on ? h.pyrf_off[2 * h.n_pairs] : 0; })) {
            if (ty == 16) hipLaunchKernelGGL(k_pyr_fused<16>, dim3(B.off[B.n]), dim3(256), 0, s, B, after ? 1 : 0);
            else hipLaunchKernelGGL(k_pyr_fused<8>, dim3(B.off[B.n]), dim3(256), 0, s, B, after ? 1 : 0);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_pyr_down(const Group& g, int l, int phase, hipStream_t s)
{
    Batch B;
    if (make_batch(g, B, [&](const DevPlan& h) {
            return pyr_level_launched(h, l + 1, phase) ? h.pyr_off[l + 1][2 * h.n_pairs] : 0; }))
        hipLaunchKernelGGL(k_pyr_down, dim3(B.off[B.n]), dim3(256), 0, s, B, l, phase == PYR_AFTER ? 1 : 0);
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
        hipLaunchKernelGGL(k_balance_lut, dim3(B.off[B.n]), dim3(768), 0, s, B);
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
