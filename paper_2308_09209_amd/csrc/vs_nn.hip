// vs_nn.hip -- the learned flow surrogate: a small 3x3 convolution network in
// BF16 with FP32 accumulation, forward and backward on the matrix cores
// (v_mfma_f32_16x16x32_bf16 forward, v_mfma_f32_16x16x16_bf16 weight
// gradient; wave64), plus the pointwise, loss and optimiser
// kernels its training needs.  Activations are NHWC with 16 or 32 channels;
// weights are [Cout][tap][Cin] (tap = 3 ky + kx).
#include <algorithm>
#include <atomic>

#include "vs_nn.h"

namespace vs {
namespace nn {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f)
{
    // round to nearest even (finite inputs)
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ int find_img(const ImgTable& T, int b)
{
    int i = 0;
    while (i + 1 < T.n && b >= T.tile_off[i + 1]) ++i;
    return i;
}

// ---------------------------------------------------------------------------
// 3x3 convolution, zero padding, as an implicit GEMM on the matrix cores with
// the weights as the A operand:
//   D[cout][pixel] = sum_k W[cout][k] X[pixel + off(tap)][cin],  k = tap CIN + cin,
// in 32-long k chunks (v_mfma_f32_16x16x32_bf16).  The grid is persistent: a
// block walks the CONV_T x CONV_T pixel tiles t = blockIdx.x, + gridDim.x, ...
// Each wavefront loads its A fragments (the weights, at most 72 VGPRs) once;
// per tile the block stages the tile and its one-pixel halo in LDS (16-byte
// vectors, pixel stride padded by one vector so that the 16 pixels a
// fragment read touches fall in distinct banks) and, while it multiplies,
// already holds the next tile's loads in flight.  A wavefront computes 4 rows
// of 16 pixels for every output channel (independent accumulator chains);
// every accumulator sums its chunks in k order.
// MFMA 16x16x32 BF16 fragments: lane l holds A[m = l % 16][k = 8 (l / 16) + i],
// B[k = 8 (l / 16) + i][n = l % 16] (i < 8) and D[m = 4 (l / 16) + i][n = l % 16]
// (i < 4): here m is the output channel and n the pixel, so a lane ends with
// 4 consecutive channels of one pixel.
// ---------------------------------------------------------------------------
constexpr int CONV_T = 16;                  // tile side (pixels)
constexpr int CONV_H = CONV_T + 2;          // tile with halo

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

struct ConvTile {
    int x0, y0, W, H;
    long base;
};

__device__ __forceinline__ ConvTile conv_tile(const ImgTable& T, int t)
{
    const int img = find_img(T, t);
    ConvTile c;
    c.W = T.w[img];
    c.H = T.h[img];
    c.base = T.pix_off[img];
    const int ntx = (c.W + CONV_T - 1) / CONV_T;
    const int r = t - T.tile_off[img];
    c.x0 = (r % ntx) * CONV_T;
    c.y0 = (r / ntx) * CONV_T;
    return c;
}

template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(256) void k_conv3x3(const uint16_t* __restrict__ X, const uint16_t* __restrict__ Wt,
                                                 const float* __restrict__ bias, void* __restrict__ Y,
                                                 const ImgTable T, float alpha)
{
    static_assert(CIN % 16 == 0 && COUT % 16 == 0, "channels in multiples of 16");
    constexpr int NT = COUT / 16;                  // 16-channel output groups
    constexpr int KT = 9 * CIN;                    // reduction length
    constexpr int NK = (KT + 31) / 32;             // 32-long chunks (the last one padded with zeros)
    constexpr int PV = CIN / 8;                    // 16-byte vectors per pixel
    constexpr int PSV = PV + 1;                    // LDS pixel stride in vectors
    constexpr int NV = CONV_H * CONV_H * PV;       // vectors per tile with halo
    constexpr int NL = (NV + 255) / 256;           // of them per thread
    __shared__ uint4 sX[CONV_H * CONV_H * PSV];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = lane & 15, kg = lane >> 4;
    const int ntiles = T.tile_off[T.n];
    const uint4* __restrict__ Xv = reinterpret_cast<const uint4*>(X);

    bf16x8 wa[NT][NK];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int kc = 0; kc < NK; ++kc) {
            const int k0 = kc * 32 + 8 * kg;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (k0 < KT) v = *reinterpret_cast<const uint4*>(Wt + (long)(tt * 16 + m) * KT + k0);
            wa[tt][kc] = __builtin_bit_cast(bf16x8, v);
        }
    float bb[NT][4];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int i = 0; i < 4; ++i) bb[tt][i] = bias ? bias[tt * 16 + 4 * kg + i] : 0.0f;

    // this thread's staging vectors, the same for every tile: halo row and
    // column and 16-byte vector of the pixel (packed r << 16 | c << 8 | v)
    int st[NL];
#pragma unroll
    for (int j = 0; j < NL; ++j) {
        const int e = tid + j * 256, px = e / PV;
        st[j] = e < NV ? (px / CONV_H) << 16 | (px % CONV_H) << 8 | (e % PV) : -1;
    }
    uint4 pf[NL];
    auto fetch = [&](const ConvTile& c) {
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (st[j] >= 0) {
                const int yy = c.y0 - 1 + (st[j] >> 16), xx = c.x0 - 1 + ((st[j] >> 8) & 255);
                if (yy >= 0 && yy < c.H && xx >= 0 && xx < c.W)
                    v = Xv[(c.base + (long)yy * c.W + xx) * PV + (st[j] & 255)];
            }
            pf[j] = v;
        }
    };

    ConvTile cur;
    if ((int)blockIdx.x < ntiles) {
        cur = conv_tile(T, blockIdx.x);
        fetch(cur);
    }
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        __syncthreads();                           // every wavefront is done with the previous tile
#pragma unroll
        for (int j = 0; j < NL; ++j)
            if (st[j] >= 0) sX[((st[j] >> 16) * CONV_H + ((st[j] >> 8) & 255)) * PSV + (st[j] & 255)] = pf[j];
        __syncthreads();
        const ConvTile c = cur;
        if (t + (int)gridDim.x < ntiles) {
            cur = conv_tile(T, t + gridDim.x);
            fetch(cur);                            // the next tile's loads overlap this tile's products
        }

        f32x4 acc[4][NT];
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int tt = 0; tt < NT; ++tt) acc[g][tt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kc = 0; kc < NK; ++kc) {
            const int k0 = kc * 32 + 8 * kg;
            const bool kin = k0 < KT;
            const int tap = kin ? k0 / CIN : 8, cv = (k0 % CIN) / 8;
            const int dy = tap / 3, dx = tap % 3;          // halo offsets 0..2
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int r = wv * 4 + g;
                uint4 v = sX[((r + dy) * CONV_H + m + dx) * PSV + cv];
                if (!kin) v = make_uint4(0u, 0u, 0u, 0u);
                const bf16x8 b = __builtin_bit_cast(bf16x8, v);
#pragma unroll
                for (int tt = 0; tt < NT; ++tt)
                    acc[g][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[tt][kc], b, acc[g][tt], 0, 0, 0);
            }
        }

        const int x = c.x0 + m;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int y = c.y0 + wv * 4 + g;
            if (y >= c.H || x >= c.W) continue;
            const long q = c.base + (long)y * c.W + x;
#pragma unroll
            for (int tt = 0; tt < NT; ++tt) {
                float v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    v[i] = acc[g][tt][i] + bb[tt][i];
                    if (MODE == CONV_LRELU) v[i] = v[i] > 0.0f ? v[i] : alpha * v[i];
                }
                const int co = tt * 16 + 4 * kg;
                if (MODE == CONV_FLOW2) {
                    if (co == 0) reinterpret_cast<float2*>(Y)[q] = make_float2(v[0], v[1]);
                } else if (MODE == CONV_F32) {
                    reinterpret_cast<float4*>(static_cast<float*>(Y) + q * COUT + co)[0] =
                        make_float4(v[0], v[1], v[2], v[3]);
                } else {
                    // round to nearest even (v_cvt_pk_bf16_f32)
                    const bf16x2 lo = {(__bf16)v[0], (__bf16)v[1]}, hi = {(__bf16)v[2], (__bf16)v[3]};
                    reinterpret_cast<uint2*>(static_cast<uint16_t*>(Y) + q * COUT + co)[0] =
                        make_uint2(__builtin_bit_cast(uint32_t, lo), __builtin_bit_cast(uint32_t, hi));
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Weight gradient: dW[cout][tap][cin] = sum_pixels dZ[p][cout] X[p + tap][cin],
// db[cout] = sum_pixels dZ[p][cout].  Each block reduces 256 pixels of one
// image on the matrix cores (M = cout, N = cin, K = pixels) and writes its
// partial sums; k_reduce_partials adds the partials in block order, so the
// result does not depend on scheduling.  Wavefront w takes taps w, w+4, w+8.
// ---------------------------------------------------------------------------
constexpr int WG_PIX = 256;

template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv3x3_wgrad(const uint16_t* __restrict__ X, const uint16_t* __restrict__ dZ,
                                                       float* __restrict__ part, const ImgTable T)
{
    constexpr int MT = COUT / 16, NC = CIN / 16, NPAR = COUT * 9 * CIN + COUT;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = lane & 15, kg = lane >> 4;
    const int img = find_img(T, blockIdx.x);
    const int W = T.w[img], H = T.h[img], npix = W * H;
    const long base = T.pix_off[img];
    const int p0 = (blockIdx.x - T.tile_off[img]) * WG_PIX;
    float* out = part + (long)blockIdx.x * NPAR;
    for (int tap = wv; tap < 9; tap += 4) {
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        f32x4 acc[MT][NC];
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[a][c] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        for (int kb = 0; kb < WG_PIX; kb += 16) {
            bf16x4 af[MT], bfr[NC];
            short av[MT][4], bv[NC][4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int p = p0 + kb + kg * 4 + i;
                const bool pv = p < npix;
                const int y = pv ? p / W : 0, x = pv ? p % W : 0;
                const int yy = y + dy, xx = x + dx;
                const bool inb = pv && yy >= 0 && yy < H && xx >= 0 && xx < W;
#pragma unroll
                for (int a = 0; a < MT; ++a) av[a][i] = pv ? (short)dZ[(base + p) * COUT + a * 16 + m] : (short)0;
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    bv[c][i] = inb ? (short)X[(base + (long)yy * W + xx) * CIN + c * 16 + m] : (short)0;
            }
#pragma unroll
            for (int a = 0; a < MT; ++a) af[a] = bf16x4{av[a][0], av[a][1], av[a][2], av[a][3]};
#pragma unroll
            for (int c = 0; c < NC; ++c) bfr[c] = bf16x4{bv[c][0], bv[c][1], bv[c][2], bv[c][3]};
#pragma unroll
            for (int a = 0; a < MT; ++a)
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    acc[a][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[a], bfr[c], acc[a][c], 0, 0, 0);
        }
#pragma unroll
        for (int a = 0; a < MT; ++a)
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int co = a * 16 + kg * 4 + i, ci = c * 16 + m;
                    out[((long)co * 9 + tap) * CIN + ci] = acc[a][c][i];
                }
    }
    // bias gradient: thread co sums its channel over the block's pixels in order
    if (tid < COUT) {
        float s = 0.0f;
        for (int k = 0; k < WG_PIX; ++k) {
            const int p = p0 + k;
            if (p < npix) s += bf2f(dZ[(base + p) * COUT + tid]);
        }
        out[COUT * 9 * CIN + tid] = s;
    }
}

__global__ __launch_bounds__(256) void k_reduce_partials(const float* __restrict__ part, int nblocks, int n,
                                                         float* __restrict__ out)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    float s = 0.0f;
    for (int b = 0; b < nblocks; ++b) s += part[(long)b * n + j];
    out[j] = s;
}

// W'[cin][tap][cout] = W[cout][8 - tap][cin]: the data-gradient convolution
// is the forward convolution with these weights.
__global__ __launch_bounds__(256) void k_flip_weights(const uint16_t* __restrict__ W, uint16_t* __restrict__ Wf,
                                                      int cin, int cout)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= cin * 9 * cout) return;
    const int co = j % cout, tap = (j / cout) % 9, ci = j / (cout * 9);
    Wf[j] = W[((long)co * 9 + (8 - tap)) * cin + ci];
}

// dZ = dH * lrelu'(Z), with the sign of Z read from H = lrelu(Z) (alpha > 0)
__global__ __launch_bounds__(256) void k_lrelu_bwd(const uint16_t* __restrict__ dH, const uint16_t* __restrict__ Hh,
                                                   uint16_t* __restrict__ dZ, long n, float alpha)
{
    const long j = (long)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const float g = bf2f(dH[j]);
    dZ[j] = f2bf(bf2f(Hh[j]) > 0.0f ? g : alpha * g);
}

// ---------------------------------------------------------------------------
// Input packing: level luma images of a template / moving pair -> 16-channel
// BF16 (channel 0 template, 1 moving, rest 0), normalised (Y - 128) / 64.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pack_pair(const float* __restrict__ Yt, const float* __restrict__ Ym,
                                                   uint16_t* __restrict__ X, long npix)
{
    const long p = (long)blockIdx.x * 256 + threadIdx.x;
    if (p >= npix) return;
    uint16_t v[16];
    v[0] = f2bf((Yt[p] - 128.0f) * (1.0f / 64.0f));
    v[1] = f2bf((Ym[p] - 128.0f) * (1.0f / 64.0f));
#pragma unroll
    for (int c = 2; c < 16; ++c) v[c] = 0;
    uint4* d = reinterpret_cast<uint4*>(X + p * 16);
    d[0] = make_uint4(v[0] | (uint32_t)v[1] << 16, 0u, 0u, 0u);
    d[1] = make_uint4(0u, 0u, 0u, 0u);
}

// ---------------------------------------------------------------------------
// Loss: mean end-point error of channels 0-1 of the FP32 prediction against
// the label flow, with its gradient (BF16, 16 channels, 2..15 zero) and one
// partial sum per block.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_epe_loss(const float* __restrict__ pred, const float* __restrict__ label,
                                                  uint16_t* __restrict__ dZ, float* __restrict__ block_loss, long npix,
                                                  float inv_n)
{
    __shared__ float s_red[4];
    const long p = (long)blockIdx.x * 256 + threadIdx.x;
    float e = 0.0f;
    uint16_t g0 = 0, g1 = 0;
    if (p < npix) {
        const float dx = pred[p * 16] - label[p * 2], dy = pred[p * 16 + 1] - label[p * 2 + 1];
        e = sqrtf(dx * dx + dy * dy + 1e-6f);
        g0 = f2bf(dx / e * inv_n);
        g1 = f2bf(dy / e * inv_n);
        uint4* d = reinterpret_cast<uint4*>(dZ + p * 16);
        d[0] = make_uint4(g0 | (uint32_t)g1 << 16, 0u, 0u, 0u);
        d[1] = make_uint4(0u, 0u, 0u, 0u);
    }
    for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) block_loss[blockIdx.x] = ((s_red[0] + s_red[1]) + s_red[2]) + s_red[3];
}

// Adam on FP32 master parameters, with a BF16 copy of the weights
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, uint16_t* __restrict__ w_bf16, long n,
                                              float lr, float b1, float b2, float eps, float c1, float c2)
{
    const long j = (long)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const float gj = g[j];
    const float mj = b1 * m[j] + (1.0f - b1) * gj;
    const float vj = b2 * v[j] + (1.0f - b2) * gj * gj;
    m[j] = mj;
    v[j] = vj;
    const float wj = w[j] - lr * (mj / c1) / (sqrtf(vj / c2) + eps);
    w[j] = wj;
    if (w_bf16) w_bf16[j] = f2bf(wj);
}

__global__ __launch_bounds__(256) void k_to_bf16(const float* __restrict__ a, uint16_t* __restrict__ b, long n)
{
    const long j = (long)blockIdx.x * 256 + threadIdx.x;
    if (j < n) b[j] = f2bf(a[j]);
}

// Sum of n per-block partial sums into one value (one block, fixed order:
// each thread adds a strided subset in index order, then a fixed tree).
__global__ __launch_bounds__(256) void k_sum_blocks(const float* __restrict__ part, int n, float* __restrict__ out)
{
    __shared__ float s_red[256];
    float acc = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
    s_red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s_red[threadIdx.x] += s_red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s_red[0];
}

// Average pooling of a flow field by f x f blocks (the last row and column of
// blocks may be partial: the mean over the pixels they hold), divided by f
// so the result is in pooled-grid pixels: training labels of a coarser level.
__global__ __launch_bounds__(256) void k_pool_flow(const float* __restrict__ flow, int w, int h, int f,
                                                   float* __restrict__ out, int wo, int ho)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= wo * ho) return;
    const int X = j % wo, Y = j / wo;
    const int x1 = min(w, (X + 1) * f), y1 = min(h, (Y + 1) * f);
    float sx = 0.0f, sy = 0.0f;
    for (int y = Y * f; y < y1; ++y)
        for (int x = X * f; x < x1; ++x) {
            sx += flow[((long)y * w + x) * 2];
            sy += flow[((long)y * w + x) * 2 + 1];
        }
    const float n = (float)((x1 - X * f) * (y1 - Y * f));
    out[(long)j * 2] = sx / n / (float)f;
    out[(long)j * 2 + 1] = sy / n / (float)f;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <int CIN, int COUT>
static hipError_t conv_mode(const uint16_t* X, const uint16_t* W, const float* b, void* Y, const ImgTable& T0,
                            int mode, float alpha, hipStream_t s)
{
    // 16-byte vector loads and stores
    const bool vec_ok = ((uintptr_t)X | (uintptr_t)W | (uintptr_t)Y) % 16 == 0;
    if (!vec_ok) return hipErrorInvalidValue;
    ImgTable T = T0;   // tiles of CONV_T x CONV_T pixels
    T.tile_off[0] = 0;
    for (int i = 0; i < T.n; ++i)
        T.tile_off[i + 1] = T.tile_off[i] + ((T.w[i] + CONV_T - 1) / CONV_T) * ((T.h[i] + CONV_T - 1) / CONV_T);
    for (int i = T.n + 1; i <= MAXI; ++i) T.tile_off[i] = T.tile_off[T.n];
    // persistent grid: as many blocks as the device holds at once
    static std::atomic<int> resident_blocks{0};
    int resident = resident_blocks.load(std::memory_order_relaxed);
    if (resident == 0) {
        int dev = 0, ncu = 0, per_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_conv3x3<CIN, COUT, CONV_LRELU>, 256, 0);
        if (e != hipSuccess) return e;
        resident = std::max(1, ncu * std::max(1, per_cu));
        resident_blocks.store(resident, std::memory_order_relaxed);
    }
    const dim3 g(std::min(T.tile_off[T.n], resident)), blk(256);
    switch (mode) {
    case CONV_LRELU: hipLaunchKernelGGL((k_conv3x3<CIN, COUT, CONV_LRELU>), g, blk, 0, s, X, W, b, Y, T, alpha); break;
    case CONV_LINEAR: hipLaunchKernelGGL((k_conv3x3<CIN, COUT, CONV_LINEAR>), g, blk, 0, s, X, W, b, Y, T, alpha); break;
    case CONV_F32: hipLaunchKernelGGL((k_conv3x3<CIN, COUT, CONV_F32>), g, blk, 0, s, X, W, b, Y, T, alpha); break;
    case CONV_FLOW2: hipLaunchKernelGGL((k_conv3x3<CIN, COUT, CONV_FLOW2>), g, blk, 0, s, X, W, b, Y, T, alpha); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t conv3x3(const uint16_t* X, int cin, const uint16_t* W, const float* b, void* Y, int cout,
                   const ImgTable& T, int mode, float alpha, hipStream_t s)
{
    if (T.tile_off[T.n] <= 0) return hipSuccess;
    if (cin == 16 && cout == 32) return conv_mode<16, 32>(X, W, b, Y, T, mode, alpha, s);
    if (cin == 32 && cout == 32) return conv_mode<32, 32>(X, W, b, Y, T, mode, alpha, s);
    if (cin == 32 && cout == 16) return conv_mode<32, 16>(X, W, b, Y, T, mode, alpha, s);
    if (cin == 16 && cout == 16) return conv_mode<16, 16>(X, W, b, Y, T, mode, alpha, s);
    return hipErrorInvalidValue;
}

int wgrad_blocks(const ImgTable& T)
{
    int n = 0;
    for (int i = 0; i < T.n; ++i) n += (T.w[i] * T.h[i] + WG_PIX - 1) / WG_PIX;
    return n;
}

hipError_t conv3x3_wgrad(const uint16_t* X, int cin, const uint16_t* dZ, int cout, const ImgTable& T, float* part,
                         float* dWb, hipStream_t s)
{
    ImgTable G = T;   // tiles of WG_PIX pixels
    G.tile_off[0] = 0;
    for (int i = 0; i < T.n; ++i) G.tile_off[i + 1] = G.tile_off[i] + (T.w[i] * T.h[i] + WG_PIX - 1) / WG_PIX;
    const int nb = G.tile_off[G.n];
    if (nb <= 0) return hipSuccess;
    if (cin == 16 && cout == 32) hipLaunchKernelGGL((k_conv3x3_wgrad<16, 32>), dim3(nb), dim3(256), 0, s, X, dZ, part, G);
    else if (cin == 32 && cout == 32) hipLaunchKernelGGL((k_conv3x3_wgrad<32, 32>), dim3(nb), dim3(256), 0, s, X, dZ, part, G);
    else if (cin == 32 && cout == 16) hipLaunchKernelGGL((k_conv3x3_wgrad<32, 16>), dim3(nb), dim3(256), 0, s, X, dZ, part, G);
    else return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int npar = cout * 9 * cin + cout;
    hipLaunchKernelGGL(k_reduce_partials, dim3((npar + 255) / 256), dim3(256), 0, s, part, nb, npar, dWb);
    return hipGetLastError();
}

hipError_t flip_weights(const uint16_t* W, uint16_t* Wf, int cin, int cout, hipStream_t s)
{
    const int n = cin * 9 * cout;
    hipLaunchKernelGGL(k_flip_weights, dim3((n + 255) / 256), dim3(256), 0, s, W, Wf, cin, cout);
    return hipGetLastError();
}

hipError_t lrelu_bwd(const uint16_t* dH, const uint16_t* H, uint16_t* dZ, long n, float alpha, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lrelu_bwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dH, H, dZ, n, alpha);
    return hipGetLastError();
}

hipError_t pack_pair(const float* Yt, const float* Ym, uint16_t* X, long npix, hipStream_t s)
{
    if (npix <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_pair, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, s, Yt, Ym, X, npix);
    return hipGetLastError();
}

hipError_t epe_loss(const float* pred, const float* label, uint16_t* dZ, float* block_loss, long npix, hipStream_t s)
{
    if (npix <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_epe_loss, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, s, pred, label, dZ, block_loss,
                       npix, 1.0f / (float)npix);
    return hipGetLastError();
}

hipError_t adam(float* w, float* m, float* v, const float* g, uint16_t* w_bf16, long n, float lr, float b1, float b2,
                float eps, int step, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, m, v, g, w_bf16, n, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

hipError_t to_bf16(const float* a, uint16_t* b, long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n);
    return hipGetLastError();
}

hipError_t sum_blocks(const float* part, int n, float* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_blocks, dim3(1), dim3(256), 0, s, part, n, out);
    return hipGetLastError();
}

hipError_t pool_flow(const float* flow, int w, int h, int f, float* out, hipStream_t s)
{
    const int wo = (w + f - 1) / f, ho = (h + f - 1) / f;
    hipLaunchKernelGGL(k_pool_flow, dim3((unsigned)((wo * ho + 255) / 256)), dim3(256), 0, s, flow, w, h, f, out, wo, ho);
    return hipGetLastError();
}

size_t wgrad_scratch_bound(long npix, int nimg, int cin, int cout)
{
    return ((size_t)(npix + WG_PIX - 1) / WG_PIX + (size_t)nimg) * (size_t)(cout * 9 * cin + cout) * sizeof(float);
}

}  // namespace nn
}  // namespace vs
