// vs_var.hip -- the variational alternative of the section 3.2 flow (flow = 2):
// coarse-to-fine warping with brightness and gradient constancy, a
// Charbonnier smoothness term and lagged Jacobi steps, on the same pyramids
// and flow domain as the plain estimator.  Every kernel is one pixel per
// thread over every field (pair x direction, or pair x camera for the
// derivatives) of every context in the group; FP32 in one prescribed order,
// correctly rounded division and square root.
#include "vs_device.h"

namespace vs {
namespace {

constexpr float VAR_EPS2 = 0.01f;   // Charbonnier epsilon^2 (epsilon = 0.1 luma)

// field f of level l for block b (fields of 256-pixel blocks, var_off)
__device__ __forceinline__ bool var_pixel(const DevPlan* __restrict__ P, int l, int b, int& f, int& x, int& y,
                                          int& w, int& h)
{
    f = find_field(P->var_off[l], 2 * P->n_pairs, b);
    const int p = f >> 1;
    w = P->lw[p][l];
    h = P->lh[p][l];
    const int i = (b - P->var_off[l][f]) * 256 + (int)threadIdx.x;
    if (i >= w * h) return false;
    x = i % w;
    y = i / w;
    return true;
}

__device__ __forceinline__ float at_clamped(const float* __restrict__ a, int w, int h, int x, int y)
{
    return a[(size_t)clampi(y, 0, h - 1) * w + clampi(x, 0, w - 1)];
}

__device__ __forceinline__ float cdx(const float* __restrict__ a, int w, int h, int x, int y)
{
    return 0.5f * (at_clamped(a, w, h, x + 1, y) - at_clamped(a, w, h, x - 1, y));
}

__device__ __forceinline__ float cdy(const float* __restrict__ a, int w, int h, int x, int y)
{
    return 0.5f * (at_clamped(a, w, h, x, y + 1) - at_clamped(a, w, h, x, y - 1));
}

// Bilinear samples of level planes at (X, Y), the position clamped into the
// level: the clamped corners and weights computed once for several planes.
struct BilAt {
    int i00, i10, i01, i11;
    float fx, fy;
};

__device__ __forceinline__ BilAt bil_at(int w, int h, float X, float Y)
{
    const float cx = clampf(X, 0.0f, (float)(w - 1)), cy = clampf(Y, 0.0f, (float)(h - 1));
    const float flx = floorf(cx), fly = floorf(cy);
    const int x0 = (int)flx, y0 = (int)fly;
    const int x1 = x0 + 1 < w ? x0 + 1 : w - 1, y1 = y0 + 1 < h ? y0 + 1 : h - 1;
    return BilAt{y0 * w + x0, y0 * w + x1, y1 * w + x0, y1 * w + x1, cx - flx, cy - fly};
}

__device__ __forceinline__ float bil_of(const float* __restrict__ a, const BilAt& B)
{
    const float p00 = a[B.i00], p10 = a[B.i10], p01 = a[B.i01], p11 = a[B.i11];
    const float t = __builtin_fmaf(B.fx, p10 - p00, p00);
    const float b = __builtin_fmaf(B.fx, p11 - p01, p01);
    return __builtin_fmaf(B.fy, b - t, t);
}

// Derivative planes of each camera's level image (field f = 2 p + camera):
// Dx, Dy central differences with clamped indices; Dxx, Dxy the central
// differences of Dx, Dyy of Dy (the first differences taken at the clamped
// neighbours, as the planes they are differences of).
__global__ __launch_bounds__(256) void k_var_deriv(const Batch B, int l)
{
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    const DevPlan* __restrict__ P = B.plan[c];
    int f, x, y, w, h;
    if (!var_pixel(P, l, b, f, x, y, w, h)) return;
    const int p = f >> 1, cam = f & 1;
    if (kept_by_surrogate(P, p)) return;
    const float* __restrict__ I = P->pyr[p][cam][l];
    float* __restrict__ D = P->var_D[p][cam][l];
    const size_t n = (size_t)w * h, q = (size_t)y * w + x;
    const int xm = clampi(x - 1, 0, w - 1), xp = clampi(x + 1, 0, w - 1);
    const int ym = clampi(y - 1, 0, h - 1), yp = clampi(y + 1, 0, h - 1);
    D[q] = cdx(I, w, h, x, y);
    D[n + q] = cdy(I, w, h, x, y);
    D[2 * n + q] = 0.5f * (cdx(I, w, h, xp, y) - cdx(I, w, h, xm, y));
    D[3 * n + q] = 0.5f * (cdx(I, w, h, x, yp) - cdx(I, w, h, x, ym));
    D[4 * n + q] = 0.5f * (cdy(I, w, h, x, yp) - cdy(I, w, h, x, ym));
}

// Level start: the flow is 0 at the coarsest level, else 2 x the bilinear
// sample of the coarser level's flow at (x / 2 - 1/4, y / 2 - 1/4).
__global__ __launch_bounds__(256) void k_var_init(const Batch B, int l)
{
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    const DevPlan* __restrict__ P = B.plan[c];
    int f, x, y, w, h;
    if (!var_pixel(P, l, b, f, x, y, w, h)) return;
    const int p = f >> 1, dir = f & 1;
    if (kept_by_surrogate(P, p)) return;
    float ux = 0.0f, uy = 0.0f;
    if (l + 1 < P->levels) {
        const int wc = P->lw[p][l + 1], hc = P->lh[p][l + 1];
        const float2* __restrict__ uc = P->flow[p][dir][l + 1];
        const float cx = clampf(__builtin_fmaf((float)x, 0.5f, -0.25f), 0.0f, (float)(wc - 1));
        const float cy = clampf(__builtin_fmaf((float)y, 0.5f, -0.25f), 0.0f, (float)(hc - 1));
        const float flx = floorf(cx), fly = floorf(cy);
        const int xa = (int)flx, ya = (int)fly;
        const float fx = cx - flx, fy = cy - fly;
        const int xb = xa + 1 < wc ? xa + 1 : wc - 1, yb = ya + 1 < hc ? ya + 1 : hc - 1;
        const float2 p00 = uc[(size_t)ya * wc + xa], p10 = uc[(size_t)ya * wc + xb];
        const float2 p01 = uc[(size_t)yb * wc + xa], p11 = uc[(size_t)yb * wc + xb];
        float a = __builtin_fmaf(fx, p10.x - p00.x, p00.x);
        float bb = __builtin_fmaf(fx, p11.x - p01.x, p01.x);
        ux = 2.0f * __builtin_fmaf(fy, bb - a, a);
        a = __builtin_fmaf(fx, p10.y - p00.y, p00.y);
        bb = __builtin_fmaf(fx, p11.y - p01.y, p01.y);
        uy = 2.0f * __builtin_fmaf(fy, bb - a, a);
    }
    P->flow[p][dir][l][(size_t)y * w + x] = make_float2(ux, uy);
}

// One warp: the moving image and its derivatives sampled at x + (u, v), the
// data and gradient terms' coefficients (Iz Ix Iy Ixz Iyz Ixx Ixy Iyy), and
// the increments reset.  With `fold` the previous warp's increments are first
// added to the flow.
__global__ __launch_bounds__(256) void k_var_warp(const Batch B, int l, int fold)
{
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    const DevPlan* __restrict__ P = B.plan[c];
    int f, x, y, w, h;
    if (!var_pixel(P, l, b, f, x, y, w, h)) return;
    const int p = f >> 1, dir = f & 1;
    if (kept_by_surrogate(P, p)) return;
    const int tc = dir == 0 ? 0 : 1, mc = 1 - tc;
    const size_t n = (size_t)w * h, q = (size_t)y * w + x;
    float2* __restrict__ U = P->flow[p][dir][l];
    float2* __restrict__ dd = P->var_dd[p][dir][l][0];
    float2 u = U[q];
    if (fold) {
        const float2 d = dd[q];
        u = make_float2(u.x + d.x, u.y + d.y);
        U[q] = u;
    }
    const float X = (float)x + u.x, Y = (float)y + u.y;
    const float* __restrict__ Mv = P->pyr[p][mc][l];
    const float* __restrict__ MD = P->var_D[p][mc][l];
    const float* __restrict__ TD = P->var_D[p][tc][l];
    const BilAt at = bil_at(w, h, X, Y);
    const float mw = bil_of(Mv, at), mx = bil_of(MD, at), my = bil_of(MD + n, at);
    const float mxx = bil_of(MD + 2 * n, at), mxy = bil_of(MD + 3 * n, at), myy = bil_of(MD + 4 * n, at);
    float* __restrict__ co = P->var_co[p][dir][l];
    co[q] = mw - P->pyr[p][tc][l][q];
    co[n + q] = mx;
    co[2 * n + q] = my;
    co[3 * n + q] = mx - TD[q];
    co[4 * n + q] = my - TD[n + q];
    co[5 * n + q] = mxx;
    co[6 * n + q] = mxy;
    co[7 * n + q] = myy;
    dd[q] = make_float2(0.0f, 0.0f);
}

// One Jacobi step of the linearised equations, increments src -> dst, on a
// VAR_TX x VAR_TY tile of one field.  The sums V = U + dU of the tile and a
// ring (one pixel left and up, two right and down) go to LDS once; from them
// the smoothness Psi' of the tile and a one-pixel ring (forward differences of
// V, 0 beyond the last column / row of the level), then each pixel's update
// from its 4 neighbours in the level.  Same operations as the per-pixel form:
// every V is the same sum, every Psi' the same expression.
__global__ __launch_bounds__(256) void k_var_jacobi(const Batch B, int l, int src)
{
    constexpr int RW = VAR_TX + 3, RH = VAR_TY + 3;   // V region: x0-1 .. x0+TX+1
    constexpr int SW = VAR_TX + 2, SH = VAR_TY + 2;   // Psi' region: x0-1 .. x0+TX
    __shared__ float2 sV[RH * RW];
    __shared__ float sS[SH * SW];
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    const DevPlan* __restrict__ P = B.plan[c];
    const int f = find_field(P->var_toff[l], 2 * P->n_pairs, b);
    const int p = f >> 1, dir = f & 1;
    if (kept_by_surrogate(P, p)) return;
    const int w = P->lw[p][l], h = P->lh[p][l];
    const int t = b - P->var_toff[l][f], ntx = (w + VAR_TX - 1) / VAR_TX;
    const int x0 = (t % ntx) * VAR_TX, y0 = (t / ntx) * VAR_TY;
    const float2* __restrict__ U = P->flow[p][dir][l];
    const float2* __restrict__ d = P->var_dd[p][dir][l][src];
    const int tid = threadIdx.x;
    const size_t n = (size_t)w * h;
    const float* __restrict__ co = P->var_co[p][dir][l];
    const int x = x0 + (tid & 63);
    // this thread's pixels' own values, loaded before the staging so that
    // their latency overlaps it
    constexpr int NP = VAR_TY / 4;
    float cf[NP][8];
    float2 uo[NP], dqo[NP];
    bool in[NP], nd[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int y = y0 + (tid >> 6) + 4 * k;
        in[k] = x < w && y < h;
        const size_t q = in[k] ? (size_t)y * w + x : 0;
        uo[k] = U[q];
        dqo[k] = d[q];
        nd[k] = in[k] && P->need[p][l][q] != 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) cf[k][j] = co[j * n + q];
    }
    for (int i = tid; i < RH * RW; i += 256) {
        const int xx = x0 - 1 + i % RW, yy = y0 - 1 + i / RW;
        float2 v = make_float2(0.0f, 0.0f);
        if (xx >= 0 && xx < w && yy >= 0 && yy < h) {
            const size_t q = (size_t)yy * w + xx;
            const float2 a = U[q], da = d[q];
            v = make_float2(a.x + da.x, a.y + da.y);
        }
        sV[i] = v;
    }
    __syncthreads();
    for (int i = tid; i < SH * SW; i += 256) {
        const int sx = i % SW, sy = i / SW;                 // region position (x0 - 1 + sx, y0 - 1 + sy)
        const int xx = x0 - 1 + sx, yy = y0 - 1 + sy;
        float s = 0.0f;
        if (xx >= 0 && xx < w && yy >= 0 && yy < h) {
            const float2 v0 = sV[sy * RW + sx];
            float ux = 0.0f, uy = 0.0f, vx = 0.0f, vy = 0.0f;
            if (xx + 1 < w) {
                const float2 r = sV[sy * RW + sx + 1];
                ux = r.x - v0.x;
                vx = r.y - v0.y;
            }
            if (yy + 1 < h) {
                const float2 r = sV[(sy + 1) * RW + sx];
                uy = r.x - v0.x;
                vy = r.y - v0.y;
            }
            s = 0.5f / sqrtf(__builtin_fmaf(ux, ux, __builtin_fmaf(uy, uy, __builtin_fmaf(vx, vx,
                                                    __builtin_fmaf(vy, vy, VAR_EPS2)))));
        }
        sS[i] = s;
    }
    __syncthreads();
    const float alpha = P->var_alpha, gamma = P->var_gamma;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int ty = (tid >> 6) + 4 * k, y = y0 + ty;
        if (!in[k]) continue;
        const size_t q = (size_t)y * w + x;
        const float2 u = uo[k], dq = dqo[k];
        float A11 = 0.0f, A12 = 0.0f, A22 = 0.0f, b1 = 0.0f, b2 = 0.0f;
        if (nd[k]) {
            const float c0 = cf[k][0], c1 = cf[k][1], c2 = cf[k][2], c3 = cf[k][3];
            const float c4 = cf[k][4], c5 = cf[k][5], c6 = cf[k][6], c7 = cf[k][7];
            const float e = __builtin_fmaf(c2, dq.y, __builtin_fmaf(c1, dq.x, c0));
            const float pd = 0.5f / sqrtf(__builtin_fmaf(e, e, VAR_EPS2));
            const float gx = __builtin_fmaf(c6, dq.y, __builtin_fmaf(c5, dq.x, c3));
            const float gy = __builtin_fmaf(c7, dq.y, __builtin_fmaf(c6, dq.x, c4));
            const float pg = gamma * (0.5f / sqrtf(__builtin_fmaf(gx, gx, __builtin_fmaf(gy, gy, VAR_EPS2))));
            A11 = __builtin_fmaf(pd, c1 * c1, pg * __builtin_fmaf(c5, c5, c6 * c6));
            A12 = __builtin_fmaf(pd, c1 * c2, pg * __builtin_fmaf(c5, c6, c6 * c7));
            A22 = __builtin_fmaf(pd, c2 * c2, pg * __builtin_fmaf(c6, c6, c7 * c7));
            b1 = -__builtin_fmaf(pd, c1 * c0, pg * __builtin_fmaf(c5, c3, c6 * c4));
            b2 = -__builtin_fmaf(pd, c2 * c0, pg * __builtin_fmaf(c6, c3, c7 * c4));
        }
        const int sx = (tid & 63) + 1, sy = ty + 1;          // (x, y) in the Psi' region
        const float s0 = sS[sy * SW + sx];
        float S = 0.0f, Su = 0.0f, Sv = 0.0f;
        const int nx[4] = {x - 1, x + 1, x, x};
        const int ny[4] = {y, y, y - 1, y + 1};
        const int ox[4] = {-1, 1, 0, 0}, oy[4] = {0, 0, -1, 1};
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) {
            if (nx[k2] < 0 || nx[k2] >= w || ny[k2] < 0 || ny[k2] >= h) continue;
            const float wn = 0.5f * (s0 + sS[(sy + oy[k2]) * SW + sx + ox[k2]]);
            const float2 vn = sV[(sy + oy[k2]) * RW + sx + ox[k2]];
            S += wn;
            Su = __builtin_fmaf(wn, vn.x - u.x, Su);
            Sv = __builtin_fmaf(wn, vn.y - u.y, Sv);
        }
        const float dx = __builtin_fmaf(alpha, Su, __builtin_fmaf(-A12, dq.y, b1)) / __builtin_fmaf(alpha, S, A11);
        const float dy = __builtin_fmaf(alpha, Sv, __builtin_fmaf(-A12, dq.x, b2)) / __builtin_fmaf(alpha, S, A22);
        P->var_dd[p][dir][l][src ^ 1][q] = make_float2(dx, dy);
    }
}

// the last warp's increments added to the flow
__global__ __launch_bounds__(256) void k_var_fold(const Batch B, int l)
{
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    const DevPlan* __restrict__ P = B.plan[c];
    int f, x, y, w, h;
    if (!var_pixel(P, l, b, f, x, y, w, h)) return;
    const int p = f >> 1, dir = f & 1;
    if (kept_by_surrogate(P, p)) return;
    const size_t q = (size_t)y * w + x;
    float2* __restrict__ U = P->flow[p][dir][l];
    const float2 u = U[q], d = P->var_dd[p][dir][l][0][q];
    U[q] = make_float2(u.x + d.x, u.y + d.y);
}

}  // namespace

// The variational flow of one level for every context of the group (their
// flow = 2): derivatives, initialisation, `var_outer` warps of `var_inner`
// Jacobi steps each (even steps end in increment buffer 0), the last
// increments folded in.
hipError_t launch_var(const Group& g, int l, hipStream_t s)
{
    Batch B;
    auto blocks = [&](const DevPlan& h) {
        return h.use_flow == 2 && h.flow_mode != VS_FLOW_SURROGATE && l < h.levels ? h.var_off[l][2 * h.n_pairs] : 0;
    };
    if (!make_batch(g, B, blocks)) return hipSuccess;
    const dim3 grid(B.off[B.n]), blk(256);
    int outer = g.hp[0]->var_outer, inner = g.hp[0]->var_inner;
    for (int c = 1; c < g.n; ++c)
        if (g.hp[c]->var_outer != outer || g.hp[c]->var_inner != inner) return hipErrorInvalidValue;
    if (inner % 2) return hipErrorInvalidValue;   // the steps end in buffer 0
    hipLaunchKernelGGL(k_var_deriv, grid, blk, 0, s, B, l);
    hipLaunchKernelGGL(k_var_init, grid, blk, 0, s, B, l);
    Batch BT;
    make_batch(g, BT, [&](const DevPlan& h) {
        return h.use_flow == 2 && h.flow_mode != VS_FLOW_SURROGATE && l < h.levels ? h.var_toff[l][2 * h.n_pairs] : 0;
    });
    const dim3 tgrid(BT.off[BT.n]);
    for (int o = 0; o < outer; ++o) {
        hipLaunchKernelGGL(k_var_warp, grid, blk, 0, s, B, l, o > 0 ? 1 : 0);
        for (int it = 0; it < inner; ++it) hipLaunchKernelGGL(k_var_jacobi, tgrid, blk, 0, s, BT, l, it & 1);
    }
    if (outer > 0) hipLaunchKernelGGL(k_var_fold, grid, blk, 0, s, B, l);
    return hipGetLastError();
}

}  // namespace vs
