// vs_flow.hip -- section 3.2 dense flow: the pyramidal Lucas-Kanade kernels
// (generic 16 x 16 tile kernel, 9x9-window LDS kernel, global-memory tail),
// the static flow domain and their launchers.  Same conventions as
// vs_kernels.hip: FP32 in one fixed operation order, explicit fused
// multiply-adds, correctly rounded division.
#include "vs_device.h"

namespace vs {

// ---------------------------------------------------------------------------
// Section 3.2 dense flow: pyramidal Lucas-Kanade at one level, every field
// (pair x direction), 16 x 16 pixels per block.  The template, its gradients
// and the moving image (with a halo for windows and displacements up to
// LK_D px) are staged in LDS with clamp-replicated borders; a pixel whose
// displacement leaves the staged tile reads the same clamped values from
// global memory instead.
// ---------------------------------------------------------------------------

// Origin of flow tile `bid` (field f) of level l: from the plan's tile list
// (tiles that follow the flow domain), else the box grid.
__device__ __forceinline__ void tile_origin(const DevPlan* __restrict__ P, int l, int f, int bid, int tx, int ty,
                                            int& x0, int& y0)
{
    const uint32_t* __restrict__ list = P->lk_tiles[l];
    if (list) {
        const uint32_t e = list[bid];
        x0 = (int)(e & 0xffffu);
        y0 = (int)(e >> 16);
    } else {
        const int t = bid - P->lk_off[l][f];
        x0 = (t % P->lk_tx[l][f]) * tx;
        y0 = (t / P->lk_tx[l][f]) * ty;
    }
}

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
    if (kept_by_surrogate(P, p)) return;   // the pair keeps the surrogate's flows
    const int w = P->lw[p][l], h = P->lh[p][l];
    int x0, y0;
    tile_origin(P, l, f, bid, LK_T, LK_T, x0, y0);
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
    float g00 = 0.0f, g01 = 0.0f, g11 = 0.0f, cu = 0.0f, cv = 0.0f;
    for (int yy = wy0; yy <= wy1; ++yy)
        for (int xx = wx0; xx <= wx1; ++xx) {
            float ix = sIx[yy - y0 + LK_R_MAX][xx - x0 + LK_R_MAX];
            float iy = sIy[yy - y0 + LK_R_MAX][xx - x0 + LK_R_MAX];
            float t = sT[yy - y0 + LK_HT][xx - x0 + LK_HT];
            g00 = __builtin_fmaf(ix, ix, g00);
            g01 = __builtin_fmaf(ix, iy, g01);
            g11 = __builtin_fmaf(iy, iy, g11);
            cu = __builtin_fmaf(ix, t, cu);
            cv = __builtin_fmaf(iy, t, cv);
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
        // right-hand side regrouped: b = (SA + fy (SB - SA)) - C, SA / SB the
        // gradient-weighted sums of the moving image interpolated along x on
        // the top / bottom row of each tap
        float sau = 0.0f, sav = 0.0f, sbu = 0.0f, sbv = 0.0f;
        const bool fast = ox >= -(LK_D + 1) && ox <= LK_D && oy >= -(LK_D + 1) && oy <= LK_D;
        if (fast) {
            for (int yy = wy0; yy <= wy1; ++yy) {
                const float* m0 = sM[yy + oy - y0 + LK_HM];
                const float* m1 = sM[yy + oy + 1 - y0 + LK_HM];
                const float* gxr = sIx[yy - y0 + LK_R_MAX];
                const float* gyr = sIy[yy - y0 + LK_R_MAX];
                for (int xx = wx0; xx <= wx1; ++xx) {
                    const int cx = xx + ox - x0 + LK_HM;
                    float p00 = m0[cx], p10 = m0[cx + 1], p01 = m1[cx], p11 = m1[cx + 1];
                    float ht = __builtin_fmaf(fx, p10 - p00, p00);
                    float hb = __builtin_fmaf(fx, p11 - p01, p01);
                    const float ix = gxr[xx - x0 + LK_R_MAX], iy = gyr[xx - x0 + LK_R_MAX];
                    sau = __builtin_fmaf(ix, ht, sau);
                    sav = __builtin_fmaf(iy, ht, sav);
                    sbu = __builtin_fmaf(ix, hb, sbu);
                    sbv = __builtin_fmaf(iy, hb, sbv);
                }
            }
        } else {
            for (int yy = wy0; yy <= wy1; ++yy) {
                const float* m0 = Mv + (size_t)clampi(yy + oy, 0, h - 1) * w;
                const float* m1 = Mv + (size_t)clampi(yy + oy + 1, 0, h - 1) * w;
                for (int xx = wx0; xx <= wx1; ++xx) {
                    const int xa = clampi(xx + ox, 0, w - 1), xb = clampi(xx + ox + 1, 0, w - 1);
                    float p00 = m0[xa], p10 = m0[xb], p01 = m1[xa], p11 = m1[xb];
                    float ht = __builtin_fmaf(fx, p10 - p00, p00);
                    float hb = __builtin_fmaf(fx, p11 - p01, p01);
                    const float ix = sIx[yy - y0 + LK_R_MAX][xx - x0 + LK_R_MAX];
                    const float iy = sIy[yy - y0 + LK_R_MAX][xx - x0 + LK_R_MAX];
                    sau = __builtin_fmaf(ix, ht, sau);
                    sav = __builtin_fmaf(iy, ht, sav);
                    sbu = __builtin_fmaf(ix, hb, sbu);
                    sbv = __builtin_fmaf(iy, hb, sbv);
                }
            }
        }
        const float bu = __builtin_fmaf(fy, sbu - sau, sau) - cu;
        const float bv = __builtin_fmaf(fy, sbv - sav, sav) - cv;
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
//  - the template gradients (Ix, Iy) of every window position sit in one
//    float2 in LDS, zero outside the level, so a clipped window needs no
//    predicate: such a tap adds fma(0, h, acc) = acc exactly (acc is never -0);
//  - the P pixels of a thread share each gradient row they have in common;
//  - per pixel each row of the moving image is interpolated along x once per
//    step and used at once by the two window rows it serves: as the top row
//    of window row k (sums SA) and the bottom row of window row k - 1 (SB).
// ALT keeps the previous gradient row in a second register set (the row
// loop unrolled by two, no copies); without it that row is read again from
// LDS (fewer registers).
// INBLOCK: the block finishes its own deferred pixels at its end instead of
// queueing them for the tail kernel: after a barrier each wavefront takes its
// deferred pixels four at a time, one per 16-lane group (lk_tail_group, the
// tail kernel's routine), the staged tiles' LDS then holding the groups'
// moving windows.
// Deferred pixels (lk_tail_group): 16 lanes per pixel, lane r of a group
// taking window row r.  The moving image around the pixel's displacement is
// staged in LDS (16 x 16 values, clamped indices: the window and a margin of
// LK_TAIL_M px), so a step reads memory only when the displacement has moved
// more than the margin since the staging; the sums then run through the rows
// in order, the lane of each row adding its taps to the partial sums it
// received from the lane of the row above and handing them on, so each sum is
// the same row-major sequence of fused multiply-adds as in the staged kernel.
constexpr int LK_TAIL_G = 16;
constexpr int LK_TAIL_M = 3;
constexpr int LK_TAIL_SW = 2 * LK_R_MAX + 2 + 2 * LK_TAIL_M;   // staged window side (16)

// the value of the lane one below in its row of 16 lanes (0 for a row's first
// lane), a DPP row shift: no LDS round trip
__device__ __forceinline__ float row_shr1(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, true));
}

__device__ __forceinline__ void lk_tail_group(const DevPlan* __restrict__ Pl, int l, int f, int x, int y, int it0,
                                           float ux, float uy, int sub, float* mv);

// Tile row t of a Gauss-Newton step: pixel q interpolates its moving-image row
// k = t - q along x (g_base: this thread's gradient column 0 on the wavefront's
// first tile row); cur receives gradient row t (window row k of pixel q, sums
// SA), prev holds row t - 1 (window row k - 1, sums SB), read again from LDS
// when LOAD_PREV.
template <int P, int TIW, int MWP, bool LOAD_PREV>
__device__ __forceinline__ void lk_rhs_row(int t, const float2* __restrict__ g_base, const float* __restrict__ sM,
                                           const int (&mb)[P], const float (&fx)[P],
                                           float2 (&cur)[2 * LK_R_MAX + 1], float2 (&prev)[2 * LK_R_MAX + 1],
                                           float (&sau)[P], float (&sav)[P], float (&sbu)[P], float (&sbv)[P])
{
    constexpr int R = LK_R_MAX, NW = 2 * R + 1, NJ = P + 2 * R;
    if (t < NJ) {
#pragma unroll
        for (int c = 0; c < NW; ++c) cur[c] = g_base[t * TIW + c];
    }
    if (LOAD_PREV && t >= 1) {
#pragma unroll
        for (int c = 0; c < NW; ++c) prev[c] = g_base[(t - 1) * TIW + c];
    }
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int k = t - q;
        if (k < 0 || k > 2 * R + 1) continue;
        const float* m = sM + mb[q] + k * MWP;
        float hr[NW];
        float v0 = m[0];
#pragma unroll
        for (int c = 0; c < NW; ++c) {
            const float v1 = m[c + 1];
            hr[c] = __builtin_fmaf(fx[q], v1 - v0, v0);
            v0 = v1;
        }
        if (k <= 2 * R) {
#pragma unroll
            for (int c = 0; c < NW; ++c) {
                sau[q] = __builtin_fmaf(cur[c].x, hr[c], sau[q]);
                sav[q] = __builtin_fmaf(cur[c].y, hr[c], sav[q]);
            }
        }
        if (k >= 1) {
#pragma unroll
            for (int c = 0; c < NW; ++c) {
                sbu[q] = __builtin_fmaf(prev[c].x, hr[c], sbu[q]);
                sbv[q] = __builtin_fmaf(prev[c].y, hr[c], sbv[q]);
            }
        }
    }
}

template <int P, bool INBLOCK, bool ALT>
__device__ __forceinline__ void lk_w9_body(const DevPlan* __restrict__ Pl, const int bid, int l)
{
    constexpr int R = LK_R_MAX, NW = 2 * R + 1;
    constexpr int TX = LKW_TX, TY = 4 * P;
    constexpr int TIW = TX + 2 * R, TIH = TY + 2 * R;       // gradient window positions
    constexpr int TSW = TIW + 2, TSH = TIH + 2;             // template + gradient halo
    constexpr int HM = R + LK_D + 1;                        // moving-image halo
    constexpr int MW = TX + 2 * HM, MH = TY + 2 * HM;
    // moving-tile row pitch: a multiple of the 32 LDS banks, so lanes whose
    // displacements put them one row apart read distinct banks
    constexpr int MWP = (MW + 31) / 32 * 32;
    // the staged tiles in one buffer: with INBLOCK its first 16 KB hold the
    // deferred pixels' moving windows after the steps (4 per wavefront)
    constexpr int NGF = TIH * TIW * 2, NTF = TSH * TSW, NMF = MH * MWP;   // floats
    constexpr int NWF = 16 * LK_TAIL_SW * LK_TAIL_SW;
    constexpr int NBUF = NGF + NTF + NMF > NWF ? NGF + NTF + NMF : NWF;
    __shared__ __align__(16) float s_lds[NBUF];
    float2* const sG = reinterpret_cast<float2*>(s_lds);
    float* const sT = s_lds + NGF;
    float* const sM = s_lds + NGF + NTF;

    const int f = find_field(Pl->lk_off[l], 2 * Pl->n_pairs, bid);
    const int p = f >> 1, dir = f & 1;
    int x0, y0;
    tile_origin(Pl, l, f, bid, TX, TY, x0, y0);   // read before the check below waits
    if (kept_by_surrogate(Pl, p)) return;         // the pair keeps the surrogate's flows
    const int w = Pl->lw[p][l], h = Pl->lh[p][l];
    const float* __restrict__ Tm = Pl->pyr[p][dir == 0 ? 0 : 1][l];
    const float* __restrict__ Mv = Pl->pyr[p][dir == 0 ? 1 : 0][l];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int x = x0 + lane;
    const int yb = y0 + wv * P;
    const bool has_coarse = l + 1 < Pl->levels;

    // the pixels' flow-domain flags and the four coarse-level flows each one
    // interpolates, loaded before the staging so that their latency overlaps it
    // (the coarse positions are clamped into the coarse level, so they are read
    // for every pixel and used for the pixels in the domain)
    const uint8_t* __restrict__ need = Pl->need[p][l];
    uint32_t nd[P];
    float2 c00[P], c10[P], c01[P], c11[P];
    float cfx[P], cfy[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int y = yb + q;
        nd[q] = need[(size_t)min(y, h - 1) * w + min(x, w - 1)];   // used for x < w, y < h
        if (has_coarse) {
            const int wc = Pl->lw[p][l + 1], hc = Pl->lh[p][l + 1];
            const float2* __restrict__ uc = Pl->flow[p][dir][l + 1];
            const float cx = clampf(__builtin_fmaf((float)x, 0.5f, -0.25f), 0.0f, (float)(wc - 1));
            const float cy = clampf(__builtin_fmaf((float)y, 0.5f, -0.25f), 0.0f, (float)(hc - 1));
            const float flx = floorf(cx), fly = floorf(cy);
            const int xa = (int)flx, ya = (int)fly;
            cfx[q] = cx - flx;
            cfy[q] = cy - fly;
            const int xb = xa + 1 < wc ? xa + 1 : wc - 1;
            const int ybb = ya + 1 < hc ? ya + 1 : hc - 1;
            c00[q] = uc[(size_t)ya * wc + xa];
            c10[q] = uc[(size_t)ya * wc + xb];
            c01[q] = uc[(size_t)ybb * wc + xa];
            c11[q] = uc[(size_t)ybb * wc + xb];
        }
    }

    // staging by rows: wavefront wv takes tile rows wv, wv + 4, ...; lane c
    // columns c and c + 64 (clamped once), so a row's base address and clamp
    // are the same for the whole wavefront; every load of both tiles is issued
    // before the first LDS store (one memory round trip)
    static_assert(TSW <= 128 && MW <= 128, "two columns per lane");
    constexpr int RT = (TSH + 3) / 4, RM = (MH + 3) / 4;
    const int tc0 = clampi(x0 - R - 1 + lane, 0, w - 1), tc1 = clampi(x0 - R - 1 + 64 + lane, 0, w - 1);
    const int mc0 = clampi(x0 - HM + lane, 0, w - 1), mc1 = clampi(x0 - HM + 64 + lane, 0, w - 1);
    float vt[RT][2], vm[RM][2];
#pragma unroll
    for (int j = 0; j < RT; ++j) {
        const int r = wv + 4 * j;
        if (r < TSH) {
            const float* row = Tm + (size_t)clampi(y0 - R - 1 + r, 0, h - 1) * w;
            vt[j][0] = row[tc0];
            if (64 + lane < TSW) vt[j][1] = row[tc1];
        }
    }
#pragma unroll
    for (int j = 0; j < RM; ++j) {
        const int r = wv + 4 * j;
        if (r < MH) {
            const float* row = Mv + (size_t)clampi(y0 - HM + r, 0, h - 1) * w;
            vm[j][0] = row[mc0];
            if (64 + lane < MW) vm[j][1] = row[mc1];
        }
    }
#pragma unroll
    for (int j = 0; j < RT; ++j) {
        const int r = wv + 4 * j;
        if (r < TSH) {
            sT[r * TSW + lane] = vt[j][0];
            if (64 + lane < TSW) sT[r * TSW + 64 + lane] = vt[j][1];
        }
    }
#pragma unroll
    for (int j = 0; j < RM; ++j) {
        const int r = wv + 4 * j;
        if (r < MH) {
            sM[r * MWP + lane] = vm[j][0];
            if (64 + lane < MW) sM[r * MWP + 64 + lane] = vm[j][1];
        }
    }
    __syncthreads();
    for (int i = tid; i < TIH * TIW; i += 256) {
        const int gy = i / TIW, gx = i % TIW;
        const int X = x0 - R + gx, Y = y0 - R + gy;
        const int c = (gy + 1) * TSW + gx + 1;
        const bool in = X >= 0 && X < w && Y >= 0 && Y < h;
        const float ix = in ? 0.5f * (sT[c + 1] - sT[c - 1]) : 0.0f;
        const float iy = in ? 0.5f * (sT[c + TSW] - sT[c - TSW]) : 0.0f;
        sG[i] = make_float2(ix, iy);
    }
    __syncthreads();

    const int ncx = min(x + R, w - 1) - max(x - R, 0) + 1;
    float ux[P], uy[P], g00[P], g01[P], g11[P], cu[P], cv[P], det[P];
    bool act[P];
    int dit[P];   // step at which the pixel was deferred (-1: not deferred)
#pragma unroll
    for (int q = 0; q < P; ++q) {
        act[q] = x < w && yb + q < h && nd[q] != 0u;
        dit[q] = -1;
        ux[q] = 0.0f;
        uy[q] = 0.0f;
        if (has_coarse && act[q]) {
            const float fx = cfx[q], fy = cfy[q];
            const float2 p00 = c00[q], p10 = c10[q], p01 = c01[q], p11 = c11[q];
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
        cu[q] = 0.0f;
        cv[q] = 0.0f;
    }
    // a wavefront without a flow-domain pixel has nothing to do (it returns at
    // once unless INBLOCK, whose barrier below every wavefront reaches)
    bool any_act = false;
#pragma unroll
    for (int q = 0; q < P; ++q) any_act = any_act || act[q];
    const bool wave_live = __any(any_act);
    if (!INBLOCK && !wave_live) return;
    if (wave_live) {
        // normal matrix and template term: rows shared by the P pixels, row-major
        // within each window
        const float2* g_base = sG + wv * P * TIW + lane;
#pragma unroll 1
        for (int j = 0; j < P + 2 * R; ++j) {
            float2 g[NW];
            float tv[NW];
#pragma unroll
            for (int c = 0; c < NW; ++c) {
                g[c] = g_base[j * TIW + c];
                tv[c] = sT[(wv * P + j + 1) * TSW + lane + c + 1];
            }
#pragma unroll
            for (int q = 0; q < P; ++q) {
                if (j - q < 0 || j - q > 2 * R) continue;
#pragma unroll
                for (int c = 0; c < NW; ++c) {
                    g00[q] = __builtin_fmaf(g[c].x, g[c].x, g00[q]);
                    g01[q] = __builtin_fmaf(g[c].x, g[c].y, g01[q]);
                    g11[q] = __builtin_fmaf(g[c].y, g[c].y, g11[q]);
                    cu[q] = __builtin_fmaf(g[c].x, tv[c], cu[q]);
                    cv[q] = __builtin_fmaf(g[c].y, tv[c], cv[q]);
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
            float fx[P], fy[P], sau[P], sav[P], sbu[P], sbv[P];
            int mb[P];
#pragma unroll
            for (int q = 0; q < P; ++q) {
                const float flx = floorf(ux[q]), fly = floorf(uy[q]);
                int ox = (int)flx, oy = (int)fly;
                fx[q] = ux[q] - flx;
                fy[q] = uy[q] - fly;
                sau[q] = 0.0f;
                sav[q] = 0.0f;
                sbu[q] = 0.0f;
                sbv[q] = 0.0f;
                if (act[q] && !(ox >= -(LK_D + 1) && ox <= LK_D && oy >= -(LK_D + 1) && oy <= LK_D)) {
                    // the displacement leaves the staged tile: the pixel, with its state
                    // at the start of this step (kept from here on), goes to the tail
                    dit[q] = it;
                    act[q] = false;
                }
                if (!act[q]) {
                    ox = 0;
                    oy = 0;
                }
                mb[q] = (wv * P + q - R + HM + oy) * MWP + (lane - R + HM + ox);
            }
            // tile rows t = 0 .. P + 2R: moving-image row t - q of pixel q
            constexpr int NT = P + 2 * R + 1;
            float2 gA[NW], gB[NW];
            if (ALT && P == 1 && INBLOCK) {
                // the levels this form is for hold about one wavefront per SIMD: the
                // rows unrolled, so the next rows' LDS reads are in flight while a
                // row computes (216 VGPRs, occupancy they do not need)
#pragma unroll
                for (int t = 0; t + 1 < NT; t += 2) {
                    lk_rhs_row<P, TIW, MWP, false>(t, g_base, sM, mb, fx, gA, gB, sau, sav, sbu, sbv);
                    lk_rhs_row<P, TIW, MWP, false>(t + 1, g_base, sM, mb, fx, gB, gA, sau, sav, sbu, sbv);
                }
                if (NT % 2) lk_rhs_row<P, TIW, MWP, false>(NT - 1, g_base, sM, mb, fx, gA, gB, sau, sav, sbu, sbv);
            } else if (ALT) {
#pragma unroll 1
                for (int t = 0; t + 1 < NT; t += 2) {
                    lk_rhs_row<P, TIW, MWP, false>(t, g_base, sM, mb, fx, gA, gB, sau, sav, sbu, sbv);
                    lk_rhs_row<P, TIW, MWP, false>(t + 1, g_base, sM, mb, fx, gB, gA, sau, sav, sbu, sbv);
                }
                if (NT % 2) lk_rhs_row<P, TIW, MWP, false>(NT - 1, g_base, sM, mb, fx, gA, gB, sau, sav, sbu, sbv);
            } else {
#pragma unroll 1
                for (int t = 0; t < NT; ++t)
                    lk_rhs_row<P, TIW, MWP, true>(t, g_base, sM, mb, fx, gA, gB, sau, sav, sbu, sbv);
            }
#pragma unroll
            for (int q = 0; q < P; ++q) {
                if (!act[q]) continue;
                const float bu = __builtin_fmaf(fy[q], sbu[q] - sau[q], sau[q]) - cu[q];
                const float bv = __builtin_fmaf(fy[q], sbv[q] - sav[q], sav[q]) - cv[q];
                const float du = (g01[q] * bv - g11[q] * bu) / det[q];
                const float dv = (g01[q] * bu - g00[q] * bv) / det[q];
                ux[q] = ux[q] + du;
                uy[q] = uy[q] + dv;
            }
        }
#pragma unroll
        for (int q = 0; q < P; ++q)
            if (act[q]) Pl->flow[p][dir][l][(size_t)(yb + q) * w + x] = make_float2(ux[q], uy[q]);
    }   // wave_live
    if (INBLOCK) {
        __syncthreads();   // every wavefront is done with the staged tiles
        float* const win = s_lds + (wv * 4 + (lane >> 4)) * (LK_TAIL_SW * LK_TAIL_SW);
        const int sub = lane & 15;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            unsigned long long m = __ballot(dit[q] >= 0);
            while (m != 0ull) {   // the same for the whole wavefront
                // the next (up to) 4 deferred lanes, one per 16-lane group
                int src = -1;
                for (int g = 0; g < 4 && m != 0ull; ++g) {
                    const int s = __builtin_ctzll(m);
                    m &= m - 1ull;
                    if ((lane >> 4) == g) src = s;
                }
                const int s0 = src < 0 ? 0 : src;
                const float pux = __shfl(ux[q], s0, 64), puy = __shfl(uy[q], s0, 64);
                const int pit = __shfl(dit[q], s0, 64);
                if (src >= 0) lk_tail_group(Pl, l, f, x0 + src, yb + q, pit, pux, puy, sub, win);
            }
        }
    } else {
        // queue the deferred pixels for the tail kernel: one reservation per
        // wavefront, after the steps (a reservation returns only after a round
        // trip to the memory-side counter, which stalled the whole wavefront
        // when taken inside the steps)
        unsigned long long mq[P];
        uint32_t tot = 0;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            mq[q] = __ballot(dit[q] >= 0);
            tot += (uint32_t)__popcll(mq[q]);
        }
        if (tot != 0u) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(&Pl->acc->lk_qn[l], tot);
            base = (uint32_t)__shfl((int)base, 0, 64);
#pragma unroll
            for (int q = 0; q < P; ++q) {
                if (dit[q] >= 0) {
                    const uint32_t slot =
                        base + __builtin_amdgcn_mbcnt_hi((uint32_t)(mq[q] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mq[q], 0u));
                    if (slot < (uint32_t)Pl->lk_qcap[l])
                        Pl->lk_queue[l][slot] = make_uint4((uint32_t)f | ((uint32_t)dit[q] << 8),
                                                           (uint32_t)x | ((uint32_t)(yb + q) << 16),
                                                           __float_as_uint(ux[q]), __float_as_uint(uy[q]));
                }
                base += (uint32_t)__popcll(mq[q]);
            }
        }
    }
}

// the 4-pixel forms held to 128 VGPRs (4 blocks per compute unit) also when
// they finish their deferred pixels in-block
template <int P, bool INBLOCK, bool ALT = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P == 4 && INBLOCK ? 4 : 1)))
void k_lk_w9(const Batch B, int l)
{
    int c;
    const int b = batch_block(B, blockIdx.x, c);
    lk_w9_body<P, INBLOCK, ALT>(B.plan[c], b, l);
}


// One deferred pixel finished by the 16 lanes of a group (lane sub holding
// window row sub; mv: the group's 16 x 16 LDS window), from step it0 with the
// flow (ux, uy) it had then; lane NW writes the flow.
__device__ __forceinline__ void lk_tail_group(const DevPlan* __restrict__ Pl, int l, int f, int x, int y, int it0,
                                           float ux, float uy, int sub, float* mv)
{
    constexpr int R = LK_R_MAX, NW = 2 * R + 1, G = LK_TAIL_G, MG = LK_TAIL_M, SW = LK_TAIL_SW;
    const int jr = sub < NW ? sub : NW - 1;           // lanes past the window repeat its last row, unused
    const int iters = Pl->lk_iters;
    const int p = f >> 1, dir = f & 1;
    const int w = Pl->lw[p][l], h = Pl->lh[p][l];
    const float* __restrict__ Tm = Pl->pyr[p][dir == 0 ? 0 : 1][l];
    const float* __restrict__ Mv = Pl->pyr[p][dir == 0 ? 1 : 0][l];
    // the moving window, anchored at the displacement's integer part: lane
    // sub loads row sub (loads issued with the template rows' below)
    int oxs = (int)floorf(ux), oys = (int)floorf(uy);
    float stg[SW];
    {
        const float* mrow = Mv + (size_t)clampi(y - R + oys - MG + sub, 0, h - 1) * w;
#pragma unroll
        for (int k = 0; k < SW; ++k) stg[k] = mrow[clampi(x - R + oxs - MG + k, 0, w - 1)];
    }
    // this lane's window row: template values and gradients (0 outside the level)
    const int yy = y - R + jr;
    const bool rin = yy >= 0 && yy < h;
    float tc[NW], gx[NW], gy[NW];
    {
        const float* t0 = Tm + (size_t)clampi(yy - 1, 0, h - 1) * w;
        const float* t1 = Tm + (size_t)clampi(yy, 0, h - 1) * w;
        const float* t2 = Tm + (size_t)clampi(yy + 1, 0, h - 1) * w;
        float a[NW + 2], up[NW], dn[NW];
#pragma unroll
        for (int k = 0; k < NW + 2; ++k) a[k] = t1[clampi(x - R - 1 + k, 0, w - 1)];
#pragma unroll
        for (int c = 0; c < NW; ++c) {
            const int xc = clampi(x - R + c, 0, w - 1);
            up[c] = t0[xc];
            dn[c] = t2[xc];
        }
#pragma unroll
        for (int c = 0; c < NW; ++c) {
            const bool in = rin && x - R + c >= 0 && x - R + c < w;
            gx[c] = in ? 0.5f * (a[c + 2] - a[c]) : 0.0f;
            gy[c] = in ? 0.5f * (dn[c] - up[c]) : 0.0f;
            tc[c] = a[c + 1];
        }
    }
    __builtin_amdgcn_wave_barrier();   // the previous entry's reads of the window come first
#pragma unroll
    for (int k = 0; k < SW; ++k) mv[sub * SW + k] = stg[k];
    __builtin_amdgcn_wave_barrier();
    // normal matrix and template term: row r's lane adds its taps at hand-on r
    float g00 = 0.0f, g01 = 0.0f, g11 = 0.0f, cu = 0.0f, cv = 0.0f;
#pragma unroll
    for (int r = 0; r < NW; ++r) {
        if (sub == r) {
#pragma unroll
            for (int c = 0; c < NW; ++c) {
                g00 = __builtin_fmaf(gx[c], gx[c], g00);
                g01 = __builtin_fmaf(gx[c], gy[c], g01);
                g11 = __builtin_fmaf(gy[c], gy[c], g11);
                cu = __builtin_fmaf(gx[c], tc[c], cu);
                cv = __builtin_fmaf(gy[c], tc[c], cv);
            }
        }
        g00 = row_shr1(g00);
        g01 = row_shr1(g01);
        g11 = row_shr1(g11);
        cu = row_shr1(cu);
        cv = row_shr1(cv);
    }
    // lane NW now holds the sums; it solves each step and hands the flow on
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
        // the displacement's offset in the staged window (unsigned: any ox, oy)
        uint32_t ddx = (uint32_t)ox - (uint32_t)oxs + (uint32_t)MG;
        uint32_t ddy = (uint32_t)oy - (uint32_t)oys + (uint32_t)MG;
        if (ddx > 2u * MG || ddy > 2u * MG) {
            // the displacement left the staged window (the whole group: its
            // lanes hold the same flow): stage it again around the new one
            oxs = ox;
            oys = oy;
            ddx = MG;
            ddy = MG;
            const float* mrow = Mv + (size_t)clampi(y - R + oys - MG + sub, 0, h - 1) * w;
#pragma unroll
            for (int k = 0; k < SW; ++k) stg[k] = mrow[clampi(x - R + oxs - MG + k, 0, w - 1)];
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int k = 0; k < SW; ++k) mv[sub * SW + k] = stg[k];
            __builtin_amdgcn_wave_barrier();
        }
        // rows yy + oy and yy + oy + 1, columns x - R + ox + k, clamped as staged
        const float* m0 = mv + (jr + (int)ddy) * SW + (int)ddx;
        float ra[NW + 1], rb[NW + 1];
#pragma unroll
        for (int k = 0; k < NW + 1; ++k) {
            ra[k] = m0[k];
            rb[k] = m0[SW + k];
        }
        float ta[NW], tb[NW];
#pragma unroll
        for (int c = 0; c < NW; ++c) {
            ta[c] = __builtin_fmaf(fx, ra[c + 1] - ra[c], ra[c]);
            tb[c] = __builtin_fmaf(fx, rb[c + 1] - rb[c], rb[c]);
        }
        float sau = 0.0f, sav = 0.0f, sbu = 0.0f, sbv = 0.0f;
#pragma unroll
        for (int r = 0; r < NW; ++r) {
            if (sub == r) {
#pragma unroll
                for (int c = 0; c < NW; ++c) {
                    sau = __builtin_fmaf(gx[c], ta[c], sau);
                    sav = __builtin_fmaf(gy[c], ta[c], sav);
                    sbu = __builtin_fmaf(gx[c], tb[c], sbu);
                    sbv = __builtin_fmaf(gy[c], tb[c], sbv);
                }
            }
            sau = row_shr1(sau);
            sav = row_shr1(sav);
            sbu = row_shr1(sbu);
            sbv = row_shr1(sbv);
        }
        const float bu = __builtin_fmaf(fy, sbu - sau, sau) - cu;
        const float bv = __builtin_fmaf(fy, sbv - sav, sav) - cv;
        const float du = (g01 * bv - g11 * bu) / det;
        const float dv = (g01 * bu - g00 * bv) / det;
        ux = __shfl(ux + du, NW, G);
        uy = __shfl(uy + dv, NW, G);
    }
    if (sub == NW) Pl->flow[p][dir][l][(size_t)y * w + x] = make_float2(ux, uy);
}

__global__ __launch_bounds__(256) void k_lk_tail(const Batch B, int l)
{
    constexpr int G = LK_TAIL_G, SW = LK_TAIL_SW;
    int cx;
    const int b = batch_block(B, blockIdx.x, cx);
    const int nb = B.off[cx + 1] - B.off[cx];        // this context's blocks
    const DevPlan* __restrict__ Pl = B.plan[cx];
    const uint32_t n = min(Pl->acc->lk_qn[l], (uint32_t)Pl->lk_qcap[l]);
    __shared__ float s_mv[256 / G][SW * SW];
    float* const mv = s_mv[threadIdx.x / G];          // this group's staged window (its lanes share a wavefront)
    const int sub = (int)(threadIdx.x % G);
    // a whole group takes the same entry, so the group's lanes stay together
    for (uint32_t i = (b * 256 + threadIdx.x) / G; i < n; i += (uint32_t)nb * (256 / G)) {
        const uint4 ent = Pl->lk_queue[l][i];
        lk_tail_group(Pl, l, (int)(ent.x & 255u), (int)(ent.y & 0xffffu), (int)(ent.y >> 16), (int)(ent.x >> 8),
                      __uint_as_float(ent.z), __uint_as_float(ent.w), sub, mv);
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



hipError_t launch_lk(const Group& g, int l, hipStream_t s)
{
    // every context of a group runs the same flow-kernel variant at a level:
    // 0 generic, else pixels per thread (1, 2, 4) plus 8 for alternating row registers
    const int code = g.hp[0]->lk_P[l];
    for (int c = 1; c < g.n; ++c)
        if (g.hp[c]->lk_P[l] != code) return hipErrorInvalidValue;
    const int P = code & 15;
    Batch B;
    // a context whose flows all come from the surrogate launches no flow blocks
    auto plain = [](const DevPlan& h) { return h.use_flow == 1 && h.flow_mode != VS_FLOW_SURROGATE; };
    // fallback contexts: deferred pixels finished in-block, no tail launch
    // (and variants that ask for it: no tail launch)
    bool inblock = (code & VS_FLOW_INBLOCK) != 0;
    for (int c = 0; c < g.n; ++c) inblock = inblock || g.hp[c]->flow_mode == VS_FLOW_SURROGATE_FALLBACK;
    if (make_batch(g, B, [&](const DevPlan& h) { return plain(h) && l < h.levels ? h.lk_off[l][2 * h.n_pairs] : 0; })) {
        const dim3 grid(B.off[B.n]);
        switch (P * 2 + (inblock ? 1 : 0)) {
        case 8: hipLaunchKernelGGL((k_lk_w9<4, false>), grid, dim3(256), 0, s, B, l); break;
        case 9: hipLaunchKernelGGL((k_lk_w9<4, true>), grid, dim3(256), 0, s, B, l); break;
        case 4: hipLaunchKernelGGL((k_lk_w9<2, false>), grid, dim3(256), 0, s, B, l); break;
        case 5: hipLaunchKernelGGL((k_lk_w9<2, true>), grid, dim3(256), 0, s, B, l); break;
        case 6: hipLaunchKernelGGL((k_lk_w9<3, false>), grid, dim3(256), 0, s, B, l); break;
        case 7: hipLaunchKernelGGL((k_lk_w9<3, true>), grid, dim3(256), 0, s, B, l); break;
        case 22: hipLaunchKernelGGL((k_lk_w9<3, false, true>), grid, dim3(256), 0, s, B, l); break;
        case 23: hipLaunchKernelGGL((k_lk_w9<3, true, true>), grid, dim3(256), 0, s, B, l); break;
        case 2: hipLaunchKernelGGL((k_lk_w9<1, false>), grid, dim3(256), 0, s, B, l); break;
        case 3: hipLaunchKernelGGL((k_lk_w9<1, true>), grid, dim3(256), 0, s, B, l); break;
        case 24: hipLaunchKernelGGL((k_lk_w9<4, false, true>), grid, dim3(256), 0, s, B, l); break;
        case 25: hipLaunchKernelGGL((k_lk_w9<4, true, true>), grid, dim3(256), 0, s, B, l); break;
        case 20: hipLaunchKernelGGL((k_lk_w9<2, false, true>), grid, dim3(256), 0, s, B, l); break;
        case 21: hipLaunchKernelGGL((k_lk_w9<2, true, true>), grid, dim3(256), 0, s, B, l); break;
        case 18: hipLaunchKernelGGL((k_lk_w9<1, false, true>), grid, dim3(256), 0, s, B, l); break;
        case 19: hipLaunchKernelGGL((k_lk_w9<1, true, true>), grid, dim3(256), 0, s, B, l); break;
        default: hipLaunchKernelGGL(k_lk, grid, dim3(256), 0, s, B, l); break;
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || P == 0 || inblock) return e;
    // deferred pixels: the device-side count bounds the grid-stride loop
    if (make_batch(g, B, [&](const DevPlan& h) {
            return plain(h) && l < h.levels ? std::min(4096, std::max(1, (h.lk_qcap[l] + 256 / LK_TAIL_G - 1) / (256 / LK_TAIL_G))) : 0; }))
        hipLaunchKernelGGL(k_lk_tail, dim3(B.off[B.n]), dim3(256), 0, s, B, l);
    return hipGetLastError();
}

}  // namespace vs
