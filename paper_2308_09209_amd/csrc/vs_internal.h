// vs_internal.h -- device-side plan and workspace layout of libvstitch, shared
// by the host runtime (vs_host.cpp) and the kernels (vs_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/vstitch.h"
#include "vs_nn.h"

namespace vs {

constexpr int MAXC = VS_MAX_CAMS;
constexpr int MAXP = VS_MAX_PAIRS;
constexpr int MAXL = VS_MAX_LEVELS;
constexpr int MAXB = 8;                       // contexts in one batched launch
constexpr int SURR_LEVEL = 2;                 // pyramid level the learned surrogate works at
constexpr int SURR_MAX_LAYERS = 8;

// Tile shapes.
constexpr int STRIP_TX = 64, STRIP_TY = 32;   // strip kernels: 256 threads, 8 rows each
constexpr int PYR_TX = 64, PYR_TY = 16;       // pyramid kernels: 256 threads, 4 rows each
constexpr int PF_TX = 32;                     // fused levels 0-2: level-2 tile PF_TX x pyrf_ty (8 or 16)
constexpr int LK_T = 16;                      // generic flow kernel: 16 x 16 pixels, one per thread
constexpr int LK_R_MAX = 4;                   // window half-size limit of the staged tiles
constexpr int LK_D = 8;                       // displacement the staged moving tile covers
constexpr int LKW_TX = 64;                    // 9x9-window flow kernel: 64 px wide, 4 * P rows,
                                              // P vertically adjacent pixels per thread
constexpr int BL_TX = 256, BL_TY = 8;         // blend / balance tile: 256 x 8 px
constexpr int BL_THREADS = 256;               // 4 px per thread, 2 rows per thread
constexpr int SURR_UP_PX = 4;                 // surrogate upsampling: pixels per thread (rows 4 apart)
constexpr int SURR_UP_ROWS = 4 * SURR_UP_PX;  // 64 x 16 px per block
constexpr int SURR_UP_SUB = STRIP_TY / SURR_UP_ROWS;   // upsampling blocks per strip tile
static_assert(STRIP_TY % SURR_UP_ROWS == 0, "whole upsampling blocks per strip tile");

// Per-frame accumulators, zeroed at the start of every frame.
// Sums that many blocks add to are kept in several copies (tile t adds to copy
// t % SPREAD, the consumer adds the copies): device-scope atomics on one
// address from every block of a large grid serialise in the memory system.
constexpr int VAR_TX = 64, VAR_TY = 8;        // variational Jacobi tile: 256 threads, 2 px each
constexpr int HIST_SPREAD = 16, MOM_SPREAD = 32, PANO_SPREAD = 32, CSUM_SPREAD = 4;
constexpr int SOLVE_THREADS = 256;
enum { MOM_A = 0, MOM_N = 6, MOM_B = 7 };   // mom[][][]: A (6), n, B (9): 16 sums, one 128-byte line
struct Accum {
    uint32_t hist[MAXP][HIST_SPREAD][2][3][256];   // [pair][copy][0 = camera j, 1 = camera i][channel][level]
    // camera i's conditional channel sums over the overlap: csum[..][2 c + k][v]
    // = the sum of channel a over the pixels whose channel c is v, a the k-th
    // channel other than c (eq. (1)'s B from the LUT without a second pass)
    unsigned long long csum[MAXP][CSUM_SPREAD][6][256];
    unsigned long long mom[MAXP][MOM_SPREAD][16];
    uint32_t pano_hist[PANO_SPREAD][3][256];
    uint32_t lk_qn[8];                             // flow pixels deferred to the tail kernel, per level
};
static_assert(MAXL <= 8, "one deferral counter per level");
static_assert(sizeof(Accum) % 16 == 0, "the fill kernels clear whole 16-byte words");
static_assert(offsetof(Accum, hist) % 16 == 0 && offsetof(Accum, csum) % 16 == 0 && offsetof(Accum, mom) % 16 == 0 &&
                  offsetof(Accum, pano_hist) % 16 == 0 && offsetof(Accum, lk_qn) > offsetof(Accum, pano_hist),
              "k_set_io clears per-pair prefixes in 16-byte words, then the histogram and counters at the end");

// Per-frame results (also the taps).
struct Results {
    uint8_t lut[MAXP][3][256];
    double Mpair[MAXP][9];
    float Mk[MAXC][9];
    float Mpf[MAXP][9];               // the pair matrices in FP32 (VS_READ_OVERLAP_ONLY)
    int32_t flags[MAXP];
    unsigned long long mom[MAXP][16];
    uint8_t bal_lut[3][256];
    int32_t quant[3][2];
    double mbar[3][2];
    int32_t surr_ok[MAXP];            // 1: the pair keeps the surrogate's flows this frame
    unsigned long long fb[MAXP][2];
};

struct DevPlan {
    int32_t n_cams, n_pairs, canvas_w, canvas_h, ring, Wp, levels, pano_pitch;
    int32_t color_window, min_pixels, use_flow, balance, lambda_pct, lk_radius, lk_iters;
    int32_t readings;                 // VS_READ_* mask
    // variational flow (use_flow = 2): weights, steps, and per level the
    // 256-pixel blocks of every field (prefix sums over fields 2 p + d)
    float var_alpha, var_gamma;
    int32_t var_outer, var_inner;
    int32_t var_off[MAXL][2 * MAXP + 1];
    int32_t var_toff[MAXL][2 * MAXP + 1];   // flow = 2: Jacobi tiles (VAR_TX x VAR_TY) per field, prefix sums
    float lk_lambda;
    double ridge;
    int32_t cam_w[MAXC], cam_h[MAXC], cam_pitch[MAXC];
    float hinv[MAXC][9];
    int32_t pj[MAXP], pi[MAXP], psi[MAXP];
    int32_t sx0[MAXP], sy0[MAXP], sw[MAXP], sh[MAXP];
    int32_t pair_of[MAXC][MAXC];      // unordered camera pair -> pair index (-1: none)
    int32_t lw[MAXP][MAXL], lh[MAXP][MAXL];
    // tile tables (prefix sums over pairs / fields)
    int32_t strip_off[MAXP + 1], strip_tx[MAXP];
    int32_t pyr_off[MAXL][2 * MAXP + 1], pyr_tx[MAXL][2 * MAXP];   // field f = 2 p + cam
    int32_t pyrf_off[2 * MAXP + 1], pyrf_tx[2 * MAXP];             // fused levels 0-2: level-2 tiles
    int32_t pyrf_ty;                                               // their height: 16, or 8 for small strips
    int32_t lk_off[MAXL][2 * MAXP + 1], lk_tx[MAXL][2 * MAXP];     // field f = 2 p + dir
    int32_t lk_P[MAXL];               // 0: generic kernel (16 x 16 tiles); 1, 2, 4: 9x9 kernel, P px per thread
    // flow tiles of a level as a list: tile b (fields back to back, from
    // lk_off) has its origin at x0 = lk_tiles[l][b] & 0xffff, y0 = lk_tiles[l][b] >> 16;
    // null: the box grid, lk_tx tiles per row
    const uint32_t* lk_tiles[MAXL];
    int32_t blend_tx, blend_ty, cover_words;
    // learned surrogate (VS_FLOW_PLAIN: not used)
    int32_t flow_mode;
    alignas(16) uint8_t surr_kept[MAXP];   // this frame: 1 where the pair keeps the surrogate's flows
                                           // (written by k_surr_decide; read by the skips of later launches)
    unsigned long long fb_tau_fix;     // fallback threshold in 1/256 px
    int64_t surr_pix[2 * MAXP + 1];    // field f's level-2 pixels start at surr_pix[f] (NHWC buffers)
    const float* surr_pred;            // [pixels][2] FP32 network output (flow, level-2 px)
    unsigned long long* surr_part;     // [upsampling block][2] forward-backward error sum, pixel count
    // device buffers
    uint32_t* strip[MAXP];             // [2][sh][sw] packed R | G << 8 | B << 16
    uint8_t* mask[MAXP];               // [sh][sw]
    float* pyr[MAXP][2][MAXL];         // [h_l][w_l]
    float2* flow[MAXP][2][MAXL];       // [h_l][w_l], [0] = flow_ij, [1] = flow_ji
    uint8_t* need[MAXP][MAXL];         // [h_l][w_l] 1 where the flow is estimated (static)
    float* var_D[MAXP][2][MAXL];       // flow = 2: per camera, 5 planes [h_l][w_l]: Dx Dy Dxx Dxy Dyy
    float* var_co[MAXP][2][MAXL];      // flow = 2: per direction, 8 planes: Iz Ix Iy Ixz Iyz Ixx Ixy Iyy
    float2* var_dd[MAXP][2][MAXL][2];  // flow = 2: per direction, the increments (ping-pong)
    uint4* lk_queue[MAXL];             // deferred flow pixels: {field | iter << 8, x | y << 16, ux, uy}
    int32_t lk_qcap[MAXL];
    uint32_t* cover;                   // [canvas_h][cover_words] coverage bits
    unsigned long long* cand;          // [blend_ty][blend_tx] (camera, shift) candidates
    uint16_t* pix_code;                // [canvas_h][canvas_w] covering candidates: bits 0-5 and 6-11 the
                                       // first and second as 3 camera + shift + 1 (shift -1, 0, 1 periods),
                                       // bits 12-13 their count
    Accum* acc;
    Results* res;
    vs_color_state* state;
    // this frame's inputs and output (caller-owned), set by k_set_io
    const uint8_t* frame[MAXC];
    uint8_t* pano;
};

// One launch over several contexts: block b of the grid belongs to context c
// with off[c] <= b < off[c + 1] and is that context's block b - off[c].
struct Batch {
    int32_t n;
    int32_t off[MAXB + 1];
    const DevPlan* plan[MAXB];
};

struct FrameIO {
    DevPlan* plan[MAXB];
    const uint8_t* frame[MAXB][MAXC];
    uint8_t* pano[MAXB];
};

// host view of a context's loaded surrogate network (device buffers)
struct SurrNet {
    int nl;
    float alpha;
    int ci[SURR_MAX_LAYERS], co[SURR_MAX_LAYERS];
    const uint16_t* w[SURR_MAX_LAYERS];   // [co][9][ci] BF16
    const float* b[SURR_MAX_LAYERS];
    const uint16_t* w0p;                  // first layer [co][32] BF16: k = 2 tap + channel (0-1), zeros from k = 18
    uint16_t* h[2];                       // [pixels][32] hidden activations (ping-pong)
    float* pred;                          // [pixels][2] output (channels 0-1)
    unsigned long long* part;             // per-block forward-backward partial sums
    nn::ImgTable tbl;                     // one image per field, level-2 sizes
};

// host view of a group of contexts launched together
struct Group {
    int n;
    DevPlan* dp[MAXB];
    const DevPlan* hp[MAXB];
    const SurrNet* net[MAXB];             // null: no surrogate loaded
};

// plan-time output of the coverage kernel
struct PlanScan {
    int32_t bx0[MAXP], bx1[MAXP], by0[MAXP], by1[MAXP];
    unsigned long long n_covered;
    uint32_t err;
};

// launchers (vs_kernels.hip); all return hipGetLastError() of the launch
hipError_t launch_plan_scan(const DevPlan* dp, const DevPlan& hp, PlanScan* scan, hipStream_t s);
hipError_t launch_need(const DevPlan* dp, const DevPlan& hp, hipStream_t s);
hipError_t launch_set_io(const FrameIO& io, int n, int max_pairs, hipStream_t s);
hipError_t launch_zero(const Group& g, hipStream_t s);
hipError_t launch_strips(const Group& g, hipStream_t s);
hipError_t launch_lut(const Group& g, hipStream_t s);
hipError_t launch_solve(const Group& g, hipStream_t s);
enum { PYR_ALL = 0, PYR_UNFUSED = 1, PYR_AFTER = 2 };
hipError_t launch_pyr0(const Group& g, int phase, hipStream_t s);
hipError_t launch_pyr_fused(const Group& g, int phase, hipStream_t s);
hipError_t launch_pyr_down(const Group& g, int level, int phase, hipStream_t s);
hipError_t launch_lk(const Group& g, int level, hipStream_t s);
hipError_t launch_var(const Group& g, int level, hipStream_t s);   // vs_var.hip
hipError_t launch_surrogate(const Group& g, hipStream_t s);   // vs_surr.hip
bool surrogate_active(const Group& g, int c);
hipError_t launch_surrogate_ctx(const Group& g, int c, hipStream_t s);

// side streams of a batch: each context's surrogate chain runs on its own
// stream between a fork and a join event (captured into the graph as
// parallel branches)
struct Fork {
    hipStream_t side[MAXB];
    hipEvent_t fork;
    hipEvent_t join[MAXB];
};
hipError_t launch_blend(const Group& g, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, size_t n, uint8_t v, hipStream_t s);
hipError_t launch_luma_rgb(const uint8_t* rgb, size_t n, float* y, hipStream_t s);

// workspace of a plain-flow context (vs_flow_create, vs_flow_run_noalloc)
struct FlowLayout {
    size_t need[MAXL], pyr[2][MAXL], flow[2][MAXL], queue[MAXL], var, acc, res, state, bytes;
};
// vs_host.cpp
bool flow_plan(int w, int h, const vs_params& P, DevPlan& d, FlowLayout& L);
void flow_bind(DevPlan& d, const FlowLayout& L, uint8_t* base);
hipError_t flow_domain_fill(const DevPlan& d, hipStream_t s);
hipError_t flow_run(const DevPlan& d, DevPlan* dp, const float* yt, const float* ym, float* flow_tm,
                    float* flow_mt, hipStream_t s);
hipError_t launch_balance_lut(const Group& g, hipStream_t s);
hipError_t launch_balance_apply(const Group& g, hipStream_t s);

}  // namespace vs
