// vs_device.h -- device helpers shared by the kernel sources of libvstitch
// (vs_kernels.hip, vs_flow.hip) and the host-side group launch helper.
#pragma once
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


__device__ __forceinline__ int find_field(const int32_t* off, int n, int b)
{
    int f = 0;
    while (f + 1 < n && b >= off[f + 1]) ++f;
    return f;
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
