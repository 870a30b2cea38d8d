// vs_device.h -- device helpers shared by the kernel sources of libvstitch
// (vs_kernels.hip, vs_flow.hip) and the host-side group launch helper.
#pragma once
#include <algorithm>

#include "vs_internal.h"

namespace vs {

// ---------------------------------------------------------------------------
// Conventions (section 3.1 pre-warp; section 2.1 eq. (4) colour application)
// ---------------------------------------------------------------------------

// v clamped to [lo, hi] (lo <= hi, v finite): the median of the three, one
// v_med3_f32; a zero of either sign may come back for v = -0
__device__ __forceinline__ float clampf(float v, float lo, float hi)
{
    return __builtin_amdgcn_fmed3f(v, lo, hi);
}

// round half up to a byte: floor(r + 1/2) clamped to [0, 255] (the clamp
// commutes with the floor for integer bounds)
__device__ __forceinline__ uint32_t round8(float r)
{
    return (uint32_t)(int)floorf(__builtin_amdgcn_fmed3f(r + 0.5f, 0.0f, 255.0f));
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

// a pointer into device (global) memory as such: its loads and stores become
// global_* instructions, which count against the vector-memory counter only
// (flat ones also hold back the waits of LDS operations)
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p)
{
    return (__attribute__((address_space(1))) T*)p;
}

// bilinear resample of an HWC RGB byte image (W >= 2), position clamped into
// the image; a = p00 + fx (p10 - p00), b likewise on the next row, out =
// a + fy (b - a), each an FMA.  At the right border (x0 = W - 1, fx = 0) the
// pair (W - 2, W - 1) with fx = 1 gives the same values exactly (byte-valued
// samples), so every row pair is two in-row pixels.  bil_load issues the
// loads of the two rows' pixel pairs, bil_rgb combines them: callers with
// several samples issue all their loads before combining any.
struct BilTaps {
    // rows y0 and y1: the three aligned words holding the 6 bytes of the pixel
    // pair (x0, x0 + 1), the third being the second again unless the pair
    // starts at byte 3 of a word; combined they give bytes 0-3 and 4-5
    uint32_t a0, a1, a2, b0, b1, b2;
    uint32_t sa, sb;   // byte offsets of the pairs in their first words
    float fx, fy;
};

__device__ __forceinline__ void bil_load(const uint8_t* __restrict__ F, int pitch, int W, int H, float u, float v,
                                         BilTaps& t)
{
    float uc = clampf(u, 0.0f, (float)(W - 1));
    float vc = clampf(v, 0.0f, (float)(H - 1));
    float flx = floorf(uc), fly = floorf(vc);
    int x0 = (int)flx, y0 = (int)fly;
    t.fx = uc - flx;
    t.fy = vc - fly;
    if (x0 == W - 1) {
        x0 = W - 2;
        t.fx = 1.0f;
    }
    int y1 = y0 + 1 < H ? y0 + 1 : H - 1;
    const uintptr_t A = (uintptr_t)(F + (size_t)y0 * pitch + x0 * 3);
    const uintptr_t Bq = (uintptr_t)(F + (size_t)y1 * pitch + x0 * 3);
    const auto* wa = gmem((const uint32_t*)(A & ~(uintptr_t)3));
    const auto* wb = gmem((const uint32_t*)(Bq & ~(uintptr_t)3));
    t.a0 = wa[0];
    t.a1 = wa[1];
    t.a2 = *gmem((const uint32_t*)((A + 5) & ~(uintptr_t)3));
    t.b0 = wb[0];
    t.b1 = wb[1];
    t.b2 = *gmem((const uint32_t*)((Bq + 5) & ~(uintptr_t)3));
    t.sa = (uint32_t)(A & 3);
    t.sb = (uint32_t)(Bq & 3);
}

__device__ __forceinline__ void bil_rgb(const BilTaps& t, float out[3])
{
    const uint32_t l0 = __builtin_amdgcn_alignbyte(t.a1, t.a0, t.sa), h0 = __builtin_amdgcn_alignbyte(t.a2, t.a1, t.sa);
    const uint32_t l1 = __builtin_amdgcn_alignbyte(t.b1, t.b0, t.sb), h1 = __builtin_amdgcn_alignbyte(t.b2, t.b1, t.sb);
    const float p00[3] = {(float)(l0 & 255u), (float)((l0 >> 8) & 255u), (float)((l0 >> 16) & 255u)};
    const float p10[3] = {(float)(l0 >> 24), (float)(h0 & 255u), (float)((h0 >> 8) & 255u)};
    const float p01[3] = {(float)(l1 & 255u), (float)((l1 >> 8) & 255u), (float)((l1 >> 16) & 255u)};
    const float p11[3] = {(float)(l1 >> 24), (float)(h1 & 255u), (float)((h1 >> 8) & 255u)};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float a = __builtin_fmaf(t.fx, p10[c] - p00[c], p00[c]);
        float b = __builtin_fmaf(t.fx, p11[c] - p01[c], p01[c]);
        out[c] = __builtin_fmaf(t.fy, b - a, a);
    }
}

__device__ __forceinline__ void bilin3(const uint8_t* __restrict__ F, int pitch, int W, int H,
                                       float u, float v, float out[3])
{
    BilTaps t;
    bil_load(F, pitch, W, H, u, v, t);
    bil_rgb(t, out);
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


// the pair keeps the surrogate's flows this frame (the plain estimator and
// the pyramid levels only it reads skip the pair)
__device__ __forceinline__ bool kept_by_surrogate(const DevPlan* __restrict__ P, int p)
{
    return P->flow_mode == VS_FLOW_SURROGATE_FALLBACK && P->surr_kept[p];
}

__device__ __forceinline__ int find_field(const int32_t* off, int n, int b)
{
    int f = 0;
    while (f + 1 < n && b >= off[f + 1]) ++f;
    return f;
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)v, o, 64), hi = __shfl_xor((uint32_t)(v >> 32), o, 64);
        v += ((unsigned long long)hi << 32) | lo;
    }
    return v;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// host: one grid over the tiles of every context of a group

template <typename F>
inline bool make_batch(const Group& g, Batch& B, F blocks_of)
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


}  // namespace vs
