// vs_surr.hip -- the learned flow surrogate inside the frame (an addition to
// the paper's method, which estimates the overlap flow with a plain
// estimator, section 3.2).
//
// Per frame, for every field f = 2 p + dir of a context (pair p, direction
// dir: template = camera j / moving = camera i, and the reverse):
//  1. the first layer: its input is the level-2 luma of the field's template
//     and moving strips as BF16 (Y - 128) / 64 in channels 0-1 and zeros in
//     channels 2-15, so k_surr_in reads the two luma images directly and
//     contracts only the 9 taps x 2 channels (one 32-long matrix-core chunk,
//     zero padded) with the layer's weights repacked at load time;
//  2. the other 3x3 convolutions on the matrix cores (vs_nn.hip), one launch
//     per layer over all fields;
//  3. up: per overlap pixel of the strip, the x4 bilinear upsampling of both
//     directions' level-2 predictions into the level-0 flow buffers, and the
//     forward-backward error e = |U_ij(x) + U_ji(x + U_ij(x))| in 1/256 px
//     fixed point, summed per block (exact integer sums);
//  4. decide: the pair's block sums are added, and the pair keeps the
//     surrogate's flows when the mode is
//     VS_FLOW_SURROGATE, or when its mean error is below the threshold; the
//     plain estimator's kernels skip the kept pairs and overwrite the others.
#include <cstddef>

#include "vs_internal.h"

namespace vs {
namespace {

__device__ __forceinline__ uint32_t bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// First layer, 16 x 16 pixels of one field per block (image f of T, whose
// tile_off counts 16 x 16 tiles).  LDS holds the tile and its one-pixel halo
// as (template, moving) BF16 pairs, zero outside the image (the convolution's
// zero padding).  Reduction index k = 2 tap + channel: lane group kg = l / 16
// holds taps 4 kg .. 4 kg + 3 of its pixel (tap 8 and zeros for kg = 2, zeros
// for kg = 3); W0 is [COUT][32] in that order.  Output: leaky ReLU, BF16,
// NHWC [pixels][COUT], as the general convolution writes it.
template <int COUT>
__global__ __launch_bounds__(256) void k_surr_in(const DevPlan* __restrict__ P, const uint16_t* __restrict__ W0,
                                                 const float* __restrict__ bias, uint16_t* __restrict__ Hout,
                                                 const nn::ImgTable T, float alpha)
{
    constexpr int NT = COUT / 16, TS = 16, TH = TS + 2;
    __shared__ uint32_t sX[TH * TH];
    const int tid = threadIdx.x;
    int f = 0;
    while (f + 1 < T.n && (int)blockIdx.x >= T.tile_off[f + 1]) ++f;
    const int p = f >> 1, dir = f & 1;
    const int W = T.w[f], H = T.h[f];
    const long base = T.pix_off[f];
    const int ntx = (W + TS - 1) / TS, t = blockIdx.x - T.tile_off[f];
    const int x0 = (t % ntx) * TS, y0 = (t / ntx) * TS;
    const float* __restrict__ yt = P->pyr[p][dir == 0 ? 0 : 1][SURR_LEVEL];
    const float* __restrict__ ym = P->pyr[p][dir == 0 ? 1 : 0][SURR_LEVEL];
    for (int i = tid; i < TH * TH; i += 256) {
        const int yy = y0 - 1 + i / TH, xx = x0 - 1 + i % TH;
        uint32_t v = 0u;
        if (yy >= 0 && yy < H && xx >= 0 && xx < W) {
            const long q = (long)yy * W + xx;
            v = bf16_rne((yt[q] - 128.0f) * (1.0f / 64.0f)) | bf16_rne((ym[q] - 128.0f) * (1.0f / 64.0f)) << 16;
        }
        sX[i] = v;
    }
    const int lane = tid & 63, wv = tid >> 6, m = lane & 15, kg = lane >> 4;
    bf16x8 wa[NT];
    float bb[NT][4];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
        wa[tt] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(W0 + (tt * 16 + m) * 32 + 8 * kg));
#pragma unroll
        for (int i = 0; i < 4; ++i) bb[tt][i] = bias[tt * 16 + 4 * kg + i];
    }
    __syncthreads();
    const int x = x0 + m;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int r = wv * 4 + g;
        uint32_t bw[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int tap = 4 * kg + i;
            bw[i] = tap < 9 ? sX[(r + tap / 3) * TH + m + tap % 3] : 0u;
        }
        const bf16x8 b = __builtin_bit_cast(bf16x8, make_uint4(bw[0], bw[1], bw[2], bw[3]));
        const int y = y0 + r;
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) {
            const f32x4 acc =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[tt], b, f32x4{0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
            if (y >= H || x >= W) continue;
            uint32_t o[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float v = acc[i] + bb[tt][i];
                v = v > 0.0f ? v : alpha * v;
                o[i] = bf16_rne(v);
            }
            reinterpret_cast<uint2*>(Hout + (base + (long)y * W + x) * COUT + tt * 16 + 4 * kg)[0] =
                make_uint2(o[0] | o[1] << 16, o[2] | o[3] << 16);
        }
    }
}

// the x4 upsampled level-2 field (pred: [pixels][2]) at level-0 position
// (X, Y); a non-finite position clamps to the border
__device__ __forceinline__ float2 up_at(const float2* __restrict__ pred, int w2, int h2, float X, float Y)
{
    const float cx = fminf(fmaxf(__builtin_fmaf(X, 0.25f, -0.375f), 0.0f), (float)(w2 - 1));
    const float cy = fminf(fmaxf(__builtin_fmaf(Y, 0.25f, -0.375f), 0.0f), (float)(h2 - 1));
    const float flx = floorf(cx), fly = floorf(cy);
    const int xa = (int)flx, ya = (int)fly;
    const float fx = cx - flx, fy = cy - fly;
    const int xb = xa + 1 < w2 ? xa + 1 : w2 - 1;
    const int yb = ya + 1 < h2 ? ya + 1 : h2 - 1;
    const float2 p00 = pred[(long)ya * w2 + xa], p10 = pred[(long)ya * w2 + xb];
    const float2 p01 = pred[(long)yb * w2 + xa], p11 = pred[(long)yb * w2 + xb];
    float a = __builtin_fmaf(fx, p10.x - p00.x, p00.x);
    float b = __builtin_fmaf(fx, p11.x - p01.x, p01.x);
    const float rx = 4.0f * __builtin_fmaf(fy, b - a, a);
    a = __builtin_fmaf(fx, p10.y - p00.y, p00.y);
    b = __builtin_fmaf(fx, p11.y - p01.y, p01.y);
    const float ry = 4.0f * __builtin_fmaf(fy, b - a, a);
    return make_float2(rx, ry);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// SURR_UP_PX overlap pixels per thread, rows 4 apart (64 x SURR_UP_ROWS px per
// block, SURR_UP_SUB blocks per strip tile): the pixels' dependent lookups
// (mask, upsampled flow, the reverse flow at the displaced position) are in
// flight together.  Each block writes its error sum and pixel count (exact
// integers, at most 2^20 * 1024 per block).
__global__ __launch_bounds__(256) void k_surr_up(const DevPlan* __restrict__ P)
{
    __shared__ uint32_t s_red[2][4];
    const int tid = threadIdx.x;
    const int tile = blockIdx.x / SURR_UP_SUB, sub = blockIdx.x % SURR_UP_SUB;
    int p = 0;
    while (p + 1 < P->n_pairs && tile >= P->strip_off[p + 1]) ++p;
    const int t = tile - P->strip_off[p];
    const int sw = P->sw[p], sh = P->sh[p];
    const int w2 = P->lw[p][SURR_LEVEL], h2 = P->lh[p][SURR_LEVEL];
    const float2* __restrict__ pij = reinterpret_cast<const float2*>(P->surr_pred) + P->surr_pix[2 * p];
    const float2* __restrict__ pji = reinterpret_cast<const float2*>(P->surr_pred) + P->surr_pix[2 * p + 1];
    const int lx = (t % P->strip_tx[p]) * STRIP_TX + (tid & 63);
    const int ly0 = (t / P->strip_tx[p]) * STRIP_TY + sub * SURR_UP_ROWS + (tid >> 6);
    bool on[SURR_UP_PX];
#pragma unroll
    for (int k = 0; k < SURR_UP_PX; ++k) {
        const int ly = ly0 + 4 * k;
        on[k] = lx < sw && ly < sh && P->need[p][0][(long)ly * sw + lx] != 0;
    }
    float2 u[SURR_UP_PX];
#pragma unroll
    for (int k = 0; k < SURR_UP_PX; ++k) {
        if (!on[k]) continue;
        const int ly = ly0 + 4 * k;
        const long q = (long)ly * sw + lx;
        u[k] = up_at(pij, w2, h2, (float)lx, (float)ly);
        P->flow[p][0][0][q] = u[k];
        P->flow[p][1][0][q] = up_at(pji, w2, h2, (float)lx, (float)ly);
    }
    uint32_t esum = 0, cnt = 0;
#pragma unroll
    for (int k = 0; k < SURR_UP_PX; ++k) {
        if (!on[k]) continue;
        const int ly = ly0 + 4 * k;
        const float2 v = up_at(pji, w2, h2, (float)lx + u[k].x, (float)ly + u[k].y);
        const float ex = u[k].x + v.x, ey = u[k].y + v.y;
        const float e = sqrtf(ex * ex + ey * ey);
        esum += (uint32_t)floorf(fminf(e * 256.0f, 1048576.0f) + 0.5f);
        cnt += 1;
    }
    esum = wave_sum(esum);
    cnt = wave_sum(cnt);
    if ((tid & 63) == 0) {
        s_red[0][tid >> 6] = esum;
        s_red[1][tid >> 6] = cnt;
    }
    __syncthreads();
    if (tid == 0) {
        P->surr_part[2 * blockIdx.x] = (unsigned long long)s_red[0][0] + s_red[0][1] + s_red[0][2] + s_red[0][3];
        P->surr_part[2 * blockIdx.x + 1] = (unsigned long long)s_red[1][0] + s_red[1][1] + s_red[1][2] + s_red[1][3];
    }
}

// one block per pair: add the pair's block partials (exact integers, so the
// order does not matter), decide
__global__ __launch_bounds__(1024) void k_surr_decide(const DevPlan* __restrict__ P, uint8_t* __restrict__ kept)
{
    __shared__ unsigned long long s_e[1024], s_n[1024];
    const int p = blockIdx.x, tid = threadIdx.x;
    const int b0 = P->strip_off[p] * SURR_UP_SUB, b1 = P->strip_off[p + 1] * SURR_UP_SUB;
    unsigned long long e = 0, n = 0;
    for (int b = b0 + tid; b < b1; b += 1024) {
        e += P->surr_part[2 * b];
        n += P->surr_part[2 * b + 1];
    }
    s_e[tid] = e;
    s_n[tid] = n;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (tid < o) {
            s_e[tid] += s_e[tid + o];
            s_n[tid] += s_n[tid + o];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const unsigned long long s = s_e[0], c = s_n[0];
        const bool ok = P->flow_mode == VS_FLOW_SURROGATE || (c > 0 && s < P->fb_tau_fix * c);
        P->res->surr_ok[p] = ok;
        kept[p] = ok;
        P->res->fb[p][0] = s;
        P->res->fb[p][1] = c;
    }
}

}  // namespace

bool surrogate_active(const Group& g, int c)
{
    const DevPlan& h = *g.hp[c];
    return h.use_flow && h.flow_mode != VS_FLOW_PLAIN;
}

hipError_t launch_surrogate_ctx(const Group& g, int c, hipStream_t s)
{
    const DevPlan& h = *g.hp[c];
    const SurrNet* net = g.net[c];
    if (!surrogate_active(g, c)) return hipSuccess;
    if (!net) return hipErrorInvalidValue;
    if (net->nl < 2 || net->ci[0] != 16) return hipErrorInvalidValue;
    nn::ImgTable T = net->tbl;   // 16 x 16 tiles
    T.tile_off[0] = 0;
    for (int i = 0; i < T.n; ++i) T.tile_off[i + 1] = T.tile_off[i] + ((T.w[i] + 15) / 16) * ((T.h[i] + 15) / 16);
    for (int i = T.n + 1; i <= nn::MAXI; ++i) T.tile_off[i] = T.tile_off[T.n];
    if (T.tile_off[T.n] > 0) {
        if (net->co[0] == 32)
            hipLaunchKernelGGL(k_surr_in<32>, dim3(T.tile_off[T.n]), dim3(256), 0, s, g.dp[c], net->w0p, net->b[0],
                               net->h[0], T, net->alpha);
        else
            hipLaunchKernelGGL(k_surr_in<16>, dim3(T.tile_off[T.n]), dim3(256), 0, s, g.dp[c], net->w0p, net->b[0],
                               net->h[0], T, net->alpha);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint16_t* in = net->h[0];
    for (int l = 1; l < net->nl; ++l) {
        const bool last = l == net->nl - 1;
        void* out = last ? (void*)net->pred : (void*)net->h[l & 1];
        e = nn::conv3x3(in, net->ci[l], net->w[l], net->b[l], out, net->co[l], net->tbl,
                        last ? nn::CONV_FLOW2 : nn::CONV_LRELU, net->alpha, s);
        if (e != hipSuccess) return e;
        in = net->h[l & 1];
    }
    hipLaunchKernelGGL(k_surr_up, dim3(h.strip_off[h.n_pairs] * SURR_UP_SUB), dim3(256), 0, s, g.dp[c]);
    uint8_t* kept = reinterpret_cast<uint8_t*>(g.dp[c]) + offsetof(DevPlan, surr_kept);
    hipLaunchKernelGGL(k_surr_decide, dim3(h.n_pairs), dim3(1024), 0, s, g.dp[c], kept);
    return hipGetLastError();
}

hipError_t launch_surrogate(const Group& g, hipStream_t s)
{
    for (int c = 0; c < g.n; ++c) {
        const hipError_t e = launch_surrogate_ctx(g, c, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace vs
