/*
 * vstitch.h -- C ABI of the MI355X (gfx950) per-frame video-stitching path of
 * "GPU Accelerated Color Correction and Frame Warping for Real-time Video
 * Stitching" (arXiv 2308.09209).
 *
 * Problem statement (section 1, section 4): N camera videos are stitched into
 * one panorama per frame.  The geometric input is the pairwise homographies of
 * neighbouring cameras (section 3.1, eqs. (12)/(14)); the colour correction
 * needs the colour information of the previous two frames (eqs. (2)-(3) and
 * (6)-(7)).  Per frame the library runs, all in hand-written HIP kernels:
 *   pre-warp of every camera's overlap strip (section 3.1) and its
 *   per-channel histograms (section 2.1 steps 1-2) -> histogram specification
 *   (step 3) -> 3D-M colour matrix (eqs. (1)-(4)) -> dense pyramidal flow on
 *   the corrected overlap strips (section 3.2) -> flow-displaced resampling and
 *   weighted fusion (eqs. (15)-(18)) -> online piecewise colour balancing of
 *   the panorama (section 2.2, eqs. (5)-(7)).
 *
 * Conventions
 *  - Images are RGB, 8 bits per channel, HWC (interleaved), row pitch in
 *    bytes.  Frames and the panorama are caller-owned DEVICE pointers; the
 *    library never frees or retains them beyond a call.
 *  - A context owns every workspace it needs (allocated in vs_create, freed in
 *    vs_destroy).  A context is not thread-safe; distinct contexts are.
 *  - Every call returns a vs_status; no exception crosses the ABI.  A device
 *    error is sticky: the context must be destroyed.
 *  - Numerical degeneracies are not errors: they are reported in
 *    vs_frame_info (identity colour matrix fallback, identity balancing).
 */
#ifndef VSTITCH_H
#define VSTITCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VS_ABI_VERSION 1
#define VS_STATE_VERSION 1
#define VS_MAX_CAMS 16
#define VS_MAX_PAIRS 16
#define VS_MAX_LEVELS 6

typedef enum {
    VS_OK = 0,
    VS_E_INVAL = -1,       /* NULL pointer, bad size, non-finite or singular homography */
    VS_E_GEOMETRY = -2,    /* neighbours do not overlap, a pixel covered 3+ times, empty canvas */
    VS_E_NOMEM = -3,       /* device allocation failed */
    VS_E_DEVICE = -4,      /* HIP error (sticky) */
    VS_E_STATE = -5,       /* colour state of another version / pair count */
    VS_E_UNSUPPORTED = -6
} vs_status;

/* Camera rig (section 3.1).  Camera k >= 1 is related to camera k-1 by
 * H_pair[k], which maps camera-k pixel coordinates to camera-(k-1) pixel
 * coordinates (the paper's H_ij with i = k, j = k-1); H_ref maps camera 0
 * pixels to canvas pixels.  All matrices row-major, column-vector
 * convention, pixel centres at integer coordinates.  In a ring (ring = 1,
 * n_cams >= 3) the canvas is periodic in x with period ring_period, which
 * must equal canvas_w, and cameras N-1 and 0 form a closing pair. */
typedef struct {
    int32_t n_cams;                     /* 2..VS_MAX_CAMS */
    int32_t cam_w[VS_MAX_CAMS];         /* >= 2 */
    int32_t cam_h[VS_MAX_CAMS];         /* >= 2 */
    int32_t cam_pitch[VS_MAX_CAMS];     /* bytes per row, >= 3 * cam_w */
    double H_pair[VS_MAX_CAMS][9];      /* entry 0 unused */
    double H_ref[9];
    int32_t ring;
    int32_t ring_period;
    int32_t canvas_w, canvas_h;         /* > 0; the panorama size */
} vs_rig;

/* Method parameters.  vs_default_params gives the paper's constants:
 * lambda = 0.05 (section 2.2), a 3-frame temporal window (eqs. (2)-(3),
 * (6)-(7)); the flow-estimator parameters are this implementation's. */
typedef struct {
    int32_t color_window;   /* 0: no colour transfer (M = I); 1: 2D-M; 2-3: 3D-M window (3) */
    double ridge;           /* relative ridge of the colour solve, x trace(A) (1e-9) */
    int32_t min_pixels;     /* fewer overlap samples over the window -> M = I (64) */
    int32_t flow;           /* 0: zero flow; 1: dense pyramidal Lucas-Kanade (1); 2: variational
                               (coarse-to-fine warping, brightness + gradient constancy, Charbonnier
                               smoothness, Jacobi steps; the var_* fields) */
    int32_t lk_levels;      /* pyramid levels, 1..VS_MAX_LEVELS (4) */
    int32_t lk_iters;       /* Gauss-Newton steps per level (5) */
    int32_t lk_radius;      /* window half-size r, window (2r+1)^2, 0..4 (4) */
    float lk_lambda;        /* Tikhonov weight per window pixel (256) */
    int32_t balance;        /* 1: apply the balancing LUT to covered pixels (1) */
    int32_t lambda_pct;     /* balancing quantile in percent, 1..49 (5) */
    int32_t debug_taps;     /* 1: keep a copy of the pre-balance panorama for vs_debug_tap (0) */
    int32_t pyr_tile_rows;  /* pyramid levels 0-2 in one pass, level-2 tile height: 8 or 16, or 0:
                               16 unless that gives under 1536 tiles (0); results do not depend on it */
    int32_t readings;       /* literal readings replacing adopted ones, a mask of VS_READ_* (0) */
    float var_alpha;        /* flow = 2: smoothness weight (128) */
    float var_gamma;        /* flow = 2: gradient-constancy weight (16) */
    int32_t var_outer;      /* flow = 2: warps per level (3) */
    int32_t var_inner;      /* flow = 2: Jacobi steps per warp, even (10) */
} vs_params;

/* Literal readings of passages the default path reads otherwise (options,
 * for measuring what the adopted readings change):
 *  VS_READ_OVERLAP_ONLY  eq. (4)'s text: each pair's matrix corrects camera i
 *      only inside that pair's overlap, uncomposed (the ring's closing pair
 *      included); pixels one camera sees keep their raw colour.  Default: the
 *      pair matrices chained to camera 0 correct every camera's whole frame.
 *  VS_READ_LITERAL_EQ17  eq. (17) as printed: camera i is displaced by
 *      theta_i flow_ij, camera j by theta_j flow_ji.  Default: theta_j flow_ij
 *      and theta_i flow_ji (the two warps meet in the middle).
 *  VS_READ_NEAREST_CDF   section 2.1 step 3 with the level whose cumulative
 *      count is nearest (ties: the lower level).  Default: the first level
 *      whose cumulative count reaches it. */
enum { VS_READ_OVERLAP_ONLY = 1, VS_READ_LITERAL_EQ17 = 2, VS_READ_NEAREST_CDF = 4 };

/* Temporal colour state: the only information carried between frames.
 * mom[p][0] / mom[p][1] hold the overlap moments of pair p at frames T-1 and
 * T-2 (A = I_i^T I_i as 00,01,02,11,12,22; B = I_i^T I_j row-major; n the
 * overlap pixel count; eqs. (1)-(3)); q[0] / q[1] hold the balancing
 * thresholds (m1, m2) per channel of frames T-1 and T-2 (eqs. (6)-(7)).
 * A plain POD: save it, restore it, move it between contexts of the same
 * rig. */
typedef struct {
    uint64_t A[6];
    uint64_t B[9];
    uint64_t n;
} vs_moments;

typedef struct {
    uint32_t version;       /* VS_STATE_VERSION */
    uint32_t size;          /* sizeof(vs_color_state) */
    uint32_t n_pairs;
    uint32_t frames_seen;   /* T of the next frame */
    vs_moments mom[VS_MAX_PAIRS][2];
    int32_t q[2][3][2];
} vs_color_state;

/* What vs_create planned. */
typedef struct {
    int32_t canvas_w, canvas_h;
    int32_t pano_pitch;                 /* bytes per panorama row (= 3 * canvas_w) */
    int32_t n_cams, n_pairs, ring, ring_period, lk_levels;
    int32_t pair_j[VS_MAX_PAIRS];       /* left / reference camera of pair p */
    int32_t pair_i[VS_MAX_PAIRS];       /* right / corrected camera of pair p */
    int32_t pair_si[VS_MAX_PAIRS];      /* periods camera i is shifted by in the pair (ring closure: 1) */
    int32_t strip_x0[VS_MAX_PAIRS], strip_y0[VS_MAX_PAIRS];  /* unwrapped canvas coordinates */
    int32_t strip_w[VS_MAX_PAIRS], strip_h[VS_MAX_PAIRS];
    int64_t n_covered;                  /* canvas pixels seen by at least one camera */
    uint64_t workspace_bytes;           /* device bytes owned by the context */
    uint32_t state_bytes;               /* sizeof(vs_color_state) */
    uint32_t pad0;
    /* The flow domain of section 3.2 as planned (VS_TAP_NEED): per pair and
     * level the pixels whose flow is estimated, and the sum over them of their
     * window clipped to the level ((2r+1)^2 inside).  The plain flow does
     * lk_iters Gauss-Newton steps over flow_taps per direction. */
    uint64_t flow_px[VS_MAX_PAIRS][VS_MAX_LEVELS];
    uint64_t flow_taps[VS_MAX_PAIRS][VS_MAX_LEVELS];
} vs_plan_info;

/* Per-frame diagnostics (valid after the call returns when requested). */
typedef struct {
    float Mk[VS_MAX_CAMS][9];           /* camera -> camera-0 colour matrix, row-vector convention (eq. (4)) */
    double Mpair[VS_MAX_PAIRS][9];      /* pair matrix, camera i -> camera j */
    int32_t flags[VS_MAX_PAIRS];        /* 0 ok, 1 too few overlap pixels (M = I), 2 singular (M = I) */
    int32_t quant[3][2];                /* m1, m2 per channel of this frame */
    double mbar[3][2];                  /* their 3-frame means (eqs. (6)-(7)) */
    uint32_t frames_seen;               /* T after this frame */
    int32_t surr_ok[VS_MAX_PAIRS];      /* learned surrogate: 1 = the pair kept its flows, 0 = plain flow */
    float fb_err[VS_MAX_PAIRS];         /* its mean forward-backward error in px (-1: surrogate off) */
} vs_frame_info;

typedef struct vs_ctx vs_ctx;

int vs_abi_version(void);
const char* vs_status_str(vs_status s);

/* Fill p with the defaults listed in vs_params. */
vs_status vs_default_params(vs_params* p);

/* Host-only helper (no device work): the camera-to-canvas homographies
 * H_k = H_ref H_pair[1] ... H_pair[k] in FP64 and their canvas-to-camera
 * inverses (a positive multiple of H_k^-1: the adjugate over |adjugate[8]|
 * with the sign of det, so its last entry is +1 or -1) rounded to FP32, exactly
 * as vs_create computes them.  Hk and Hinv hold n_cams x 9 entries. */
vs_status vs_compose_homographies(const vs_rig* rig, double* Hk, float* Hinv);

/* Plan the rig (coverage of every canvas pixel by every camera on the
 * device, overlap pairs, strip boxes, pyramid sizes), allocate every
 * workspace and reset the colour state to T = 0.  p may be NULL (defaults).
 * Synchronous; uses the null stream.  *out receives the context. */
vs_status vs_create(const vs_rig* rig, const vs_params* p, vs_ctx** out);
void vs_destroy(vs_ctx* c);
vs_status vs_query(const vs_ctx* c, vs_plan_info* out);
const char* vs_last_error(const vs_ctx* c);

/* Stitch one frame.
 *  frames[k]: device pointer to camera k's image (cam_h x cam_pitch bytes).
 *  in: optional host colour state to start from (NULL: continue from the
 *      context's own device-resident state).
 *  pano: device pointer, canvas_h x pano_pitch bytes; written completely
 *      (uncovered pixels are 0).
 *  out, info: optional host outputs; when either is non-NULL the call waits
 *      for the stream before returning.
 *  stream: hipStream_t to run on (NULL: the null stream).
 * Without out/info the call is asynchronous with respect to the host. */
vs_status vs_stitch(vs_ctx* c, const uint8_t* const frames[], const vs_color_state* in,
                    uint8_t* pano, vs_color_state* out, vs_frame_info* info, void* stream);

/* Copy the device-resident colour state out / in (synchronous). */
vs_status vs_state_get(vs_ctx* c, vs_color_state* out);
vs_status vs_state_set(vs_ctx* c, const vs_color_state* in);

/* Intermediates of the last frame, copied to host memory dst (nbytes must
 * match exactly; synchronous).  Layouts:
 *  VS_TAP_STRIP     pair, sub 0 = camera j, 1 = camera i: strip_h x strip_w x 3 u8
 *  VS_TAP_MASK      pair: strip_h x strip_w u8 (1 = covered by both cameras)
 *  VS_TAP_HIST      pair: [2][3][256] u32, [0] camera j, [1] camera i
 *  VS_TAP_LUT       pair: [3][256] u8 histogram-specification LUT
 *  VS_TAP_MOM       pair: 16 u64 = A[6], B[9], n of this frame
 *  VS_TAP_MPAIR     [n_pairs][9] f64;  VS_TAP_MK [n_cams][9] f32;  VS_TAP_FLAGS [n_pairs] i32
 *  VS_TAP_PYR       pair, sub = cam * 8 + level: level image f32 (with
 *                   VS_FLOW_SURROGATE_FALLBACK, levels above 2 of a pair that
 *                   kept the surrogate's flows are not computed that frame)
 *  VS_TAP_FLOW      pair, sub 0 = flow_ij, 1 = flow_ji: strip_h x strip_w x 2 f32
 *  VS_TAP_PANO_PRE  canvas_h x canvas_w x 3 u8 (needs debug_taps = 1)
 *  VS_TAP_PANO_HIST [3][256] u32;  VS_TAP_BAL_LUT [3][256] u8
 *  VS_TAP_QUANT     [3][2] i32;  VS_TAP_MBAR [3][2] f64
 *  VS_TAP_COVER     canvas_h x canvas_w u8 (1 = covered)
 *  VS_TAP_NEED      pair, sub = level: u8 per level pixel, 1 where the flow is
 *                   estimated (the overlap at level 0, and at coarser levels the
 *                   pixels the finer level's initialisation samples); 0 elsewhere
 *                   and the flow there is 0
 *  VS_TAP_DEFERRED  sub = level: u32, flow pixels of that level finished by the
 *                   global-memory tail kernel (displacement beyond the staged tile)
 *  VS_TAP_SURR_PRED pair, sub 0 = ij, 1 = ji: the surrogate's level-2 flow,
 *                   h_2 x w_2 x 2 f32 (needs loaded weights)
 *  VS_TAP_FB        [n_pairs][2] u64: forward-backward error sum (1/256 px), pixels
 *  VS_TAP_SURR_OK   [n_pairs] i32: 1 where the pair kept the surrogate's flows */
enum {
    VS_TAP_STRIP = 1, VS_TAP_MASK = 2, VS_TAP_HIST = 3, VS_TAP_LUT = 4, VS_TAP_MOM = 5,
    VS_TAP_MPAIR = 6, VS_TAP_MK = 7, VS_TAP_FLAGS = 8, VS_TAP_PYR = 9, VS_TAP_FLOW = 10,
    VS_TAP_PANO_PRE = 11, VS_TAP_PANO_HIST = 12, VS_TAP_BAL_LUT = 13, VS_TAP_QUANT = 14,
    VS_TAP_MBAR = 15, VS_TAP_COVER = 16, VS_TAP_NEED = 17, VS_TAP_DEFERRED = 18,
    VS_TAP_SURR_PRED = 19, VS_TAP_FB = 20, VS_TAP_SURR_OK = 21
};
vs_status vs_debug_tap(vs_ctx* c, int tap, int pair, int sub, void* dst, size_t nbytes);

/* Per-step device time (HIP events on each call's stream), summed over every
 * frame stitched since timing was last switched on, in milliseconds:
 *  [0] strips + histograms + moments + colour solve (section 2.1)
 *  [1] flow-input pyramids            [2] pyramidal flow (section 3.2)
 *  [3] warp + blend (eqs. (15)-(18))  [4] balancing (section 2.2)
 *  [5] whole frame
 * vs_set_timing(c, 1) resets the sums and records events around every later
 * frame; vs_set_timing(c, 0) stops.  vs_get_timing waits for the recorded
 * frames to finish and returns the sums and the frame count. */
vs_status vs_set_timing(vs_ctx* c, int on);
vs_status vs_get_timing(vs_ctx* c, double ms[6], uint32_t* frames);

/* Flow-kernel variant of one pyramid level: 0 = generic kernel (16 x 16
 * pixel tiles, any radius), 1, 2, 3 or 4 = the 9x9-window kernel (radius 4)
 * with that many vertically adjacent pixels per thread; + 8 (VS_FLOW_ALT):
 * the previous gradient row kept in a second register set instead of read
 * again from LDS; + 16 (VS_FLOW_INBLOCK): pixels whose displacement leaves
 * the staged tile are finished by their own block at its end instead of by a
 * tail launch.  Results are identical for every variant; only speed differs.
 * vs_create picks one per level; the autotuner below measures them. */
#define VS_FLOW_ALT 8
#define VS_FLOW_INBLOCK 16
#define VS_FLOW_VARIANTS 12  /* variants the autotuner measures: 1, 2, 3, 4, 9, 10, 11, 12, 25, 26, 27, 28 */
vs_status vs_set_flow_variant(vs_ctx* c, int level, int variant);
vs_status vs_get_flow_variant(const vs_ctx* c, int32_t variant[VS_MAX_LEVELS]);

/* Batches (several streams per frame step, uneven rigs and resolutions):
 * vs_batch_create captures one HIP graph that runs the whole per-frame path
 * of up to 8 contexts, each step as one launch over the tiles of every
 * context.  The contexts keep their own plans, workspaces and colour states
 * and must share lk_levels and lk_radius; while in a batch they must not be
 * stitched concurrently through vs_stitch.  The graph does not depend on the
 * frame or panorama addresses.
 * vs_batch_run: frames[c][k] = camera k of context c (device), panos[c] =
 * context c's panorama (device); asynchronous on stream.  A device error
 * marks every context of the batch sticky. */
typedef struct vs_batch vs_batch;
vs_status vs_batch_create(vs_ctx* const ctxs[], int n, vs_batch** out);
vs_status vs_batch_run(vs_batch* b, const uint8_t* const* const frames[], uint8_t* const panos[], void* stream);
vs_status vs_batch_destroy(vs_batch* b);
const char* vs_batch_last_error(const vs_batch* b);

/* Autotuner: for every pyramid level, run the batch on the given frames with
 * each 9x9 flow-kernel variant (1, 2, 3, 4, 9, 10, 11, 12, 25, 26, 27, 28),
 * `reps` timed runs each, and keep the fastest.  ms[l][i] receives the mean
 * frame time of the i-th of those variants at level l (may be NULL);
 * choice[l] the variant kept.  Then, with 3 or more levels, the fused
 * pyramid's tile height (8 or 16 level-2 rows) the same way.  Every context's
 * choice is recorded in the tuning records (vs_tune_put).
 * The colour states are restored afterwards.  Synchronous. */
vs_status vs_batch_autotune(vs_batch* b, const uint8_t* const* const frames[], uint8_t* const panos[], int reps,
                            float ms[VS_MAX_LEVELS][VS_FLOW_VARIANTS], int32_t choice[VS_MAX_LEVELS]);

/* Tuning records: what the autotuner chose for one device architecture and
 * one plan shape, kept process-wide by the library (thread-safe), written to
 * and read from a text file (one record per line: "vstune1 arch n_cams
 * canvas_w canvas_h lk_levels lk_radius v0 .. v5 pyr_tile_rows"), and applied
 * by vs_create to a context whose key matches (its flow variants per level
 * and its fused-pyramid tile height).  vs_batch_autotune records every
 * context it tunes.  The records only pick among variants whose results are
 * identical, so applying one never changes an output.
 * vs_tune_get: VS_E_UNSUPPORTED when no record matches.
 * vs_tune_load: VS_E_INVAL (nothing loaded) on a malformed file, an unknown
 *   variant code or tile height; records replace those of equal keys.
 * vs_tune_key_of / vs_get_tuning: the key and the current choice of a
 *   context (host only). */
typedef struct {
    char arch[32];                      /* device architecture, e.g. "gfx950" (NUL-terminated) */
    int32_t n_cams, canvas_w, canvas_h, lk_levels, lk_radius;
} vs_tune_key;
typedef struct {
    int32_t flow_variant[VS_MAX_LEVELS];   /* vs_set_flow_variant codes; 0 past lk_levels */
    int32_t pyr_tile_rows;                 /* 8 or 16 (levels 0-2 in one pass), 0 = keep the default */
} vs_tune_entry;
vs_status vs_tune_put(const vs_tune_key* k, const vs_tune_entry* e);
vs_status vs_tune_get(const vs_tune_key* k, vs_tune_entry* e);
vs_status vs_tune_clear(void);
vs_status vs_tune_save(const char* path);
vs_status vs_tune_load(const char* path);
vs_status vs_tune_key_of(const vs_ctx* c, vs_tune_key* k);
vs_status vs_get_tuning(const vs_ctx* c, vs_tune_entry* e);

/* ------------------------------------------------------------------------
 * Learned flow surrogate (an addition to the paper's method): a small 3x3
 * convolution network in BF16 with FP32 accumulation, trained on flows of the
 * plain estimator.  Building blocks with device pointers, NHWC activations
 * (16 or 32 channels, BF16 stored as uint16_t) and weights [Cout][tap][Cin]
 * (tap = 3 ky + kx, zero padding).  A launch covers up to 64 images of
 * possibly different sizes stored back to back.
 * ------------------------------------------------------------------------ */
#define VS_NN_MAX_IMAGES 64
enum { VS_CONV_LRELU = 0, VS_CONV_LINEAR = 1, VS_CONV_F32 = 2, VS_CONV_FLOW2 = 3 };
typedef struct {
    int32_t n;
    int32_t w[VS_NN_MAX_IMAGES], h[VS_NN_MAX_IMAGES];
} vs_nn_images;

/* y = act(conv3x3(x, w) + bias) on the matrix cores.  (cin, cout) in
 * {(16,32), (32,32), (32,16), (16,16)}; mode VS_CONV_LRELU (BF16 out, leaky
 * ReLU slope alpha), VS_CONV_LINEAR (BF16 out), VS_CONV_F32 (FP32 out) or
 * VS_CONV_FLOW2 (FP32 channels 0-1 only, y is [pixels][2]);
 * bias may be NULL.  x, w and y must be 16-byte aligned (VS_E_INVAL
 * otherwise); x and y must not overlap.  The kernel's grid is persistent (as
 * many blocks as the device holds), each accumulator sums in (tap, cin)
 * order, so results do not depend on the grid. */
vs_status vs_nn_conv3x3(const uint16_t* x, int cin, const uint16_t* w, const float* bias, void* y, int cout,
                        const vs_nn_images* imgs, int mode, float alpha, void* stream);
/* Weight and bias gradient of that convolution: dwb[Cout][9][Cin] followed by
 * db[Cout] (FP32), from the layer input x and the pre-activation gradient dz.
 * scratch: device FP32 workspace of vs_nn_wgrad_scratch_bytes bytes (per-block
 * partial sums, added in block order: deterministic). */
size_t vs_nn_wgrad_scratch_bytes(int cin, int cout, const vs_nn_images* imgs);
vs_status vs_nn_conv3x3_wgrad(const uint16_t* x, int cin, const uint16_t* dz, int cout, const vs_nn_images* imgs,
                              float* scratch, size_t scratch_bytes, float* dwb, void* stream);
/* wf[Cin][tap][Cout] = w[Cout][8 - tap][Cin]: the data gradient is
 * vs_nn_conv3x3(dz, cout, wf, NULL, dx, cin, ..., VS_CONV_LINEAR). */
vs_status vs_nn_flip_weights(const uint16_t* w, uint16_t* wf, int cin, int cout, void* stream);
/* dz = dh * (h > 0 ? 1 : alpha) elementwise (h = leaky ReLU output). */
vs_status vs_nn_lrelu_bwd(const uint16_t* dh, const uint16_t* h, uint16_t* dz, int64_t n, float alpha, void* stream);
/* 16-channel network input from a template / moving luma pair (FP32):
 * channel 0 = (yt - 128) / 64, channel 1 = (ym - 128) / 64, others 0. */
vs_status vs_nn_pack_pair(const float* yt, const float* ym, uint16_t* x, int64_t npix, void* stream);
/* Mean end-point error of channels 0-1 of pred (FP32, 16 channels) against
 * label (FP32, 2 channels); dz (BF16, 16 channels) receives its gradient and
 * block_loss[ceil(npix / 256)] the per-block sums of the pixel errors. */
vs_status vs_nn_epe_loss(const float* pred, const float* label, uint16_t* dz, float* block_loss, int64_t npix,
                         void* stream);
/* Adam step (bias-corrected, step >= 1) on FP32 master parameters; w_bf16 (may
 * be NULL) receives their BF16 rounding. */
vs_status vs_nn_adam(float* w, float* m, float* v, const float* g, uint16_t* w_bf16, int64_t n, float lr, float b1,
                     float b2, float eps, int step, void* stream);
vs_status vs_nn_to_bf16(const float* a, uint16_t* b, int64_t n, void* stream);
/* Training labels at a coarser level: flow (FP32 [h][w][2], device) average
 * pooled over factor x factor blocks (the last block row and column may be
 * partial: the mean over the pixels they hold) and divided by factor, into out
 * (FP32 [ceil(h / factor)][ceil(w / factor)][2], device); 1 <= factor <= 64. */
vs_status vs_nn_pool_flow(const float* flow, int w, int h, int factor, float* out, void* stream);

/* The network as an object: parameters (FP32 master weights and biases),
 * Adam state, BF16 copies and every training workspace on the device.
 * Layers are 3x3 convolutions with (cin, cout) in {(16,32), (32,32), (32,16)},
 * cin[0] = 16, cout[n_layers - 1] = 16, each cin the previous cout; leaky
 * ReLU (slope alpha) after every layer but the last; the last layer's
 * channels 0-1 are the flow.  in_live: input channels that carry data (the
 * first layer's weights on the others start at 0).  max_pixels bounds the
 * pixels of one forward (all images together): the workspaces are sized for
 * it at vs_nn_create, and no later call allocates. */
#define VS_NN_MAX_LAYERS 8
typedef struct {
    int32_t n_layers;
    int32_t cin[VS_NN_MAX_LAYERS], cout[VS_NN_MAX_LAYERS];
    int32_t in_live;
    float alpha;
    int64_t max_pixels;
} vs_nn_spec;
typedef struct vs_nn vs_nn;
/* Weights He-initialised from a splitmix64 / Box-Muller stream of `seed`
 * (standard deviation sqrt(2 / (9 fan-in)), the last layer's times 0.1),
 * biases and optimiser state 0.  Synchronous. */
vs_status vs_nn_create(const vs_nn_spec* spec, uint64_t seed, vs_nn** out);
vs_status vs_nn_destroy(vs_nn* n);
/* Forward over the images of imgs (back to back, NHWC): x [pixels][16] BF16
 * (device, 16-byte aligned; it must stay unchanged until the matching
 * vs_nn_backward); pred (device, may be NULL) receives the FP32 output
 * [pixels][16].  The activations stay in the object for the backward pass. */
vs_status vs_nn_forward(vs_nn* n, const uint16_t* x, const vs_nn_images* imgs, float* pred, void* stream);
/* Sum over the last forward's pixels of the end-point error
 * sqrt(dx^2 + dy^2 + 1e-6) of output channels 0-1 against label (FP32
 * [pixels][2], device) into *loss_sum (one FP32 on the device).  VS_E_STATE
 * without a forward. */
vs_status vs_nn_loss(vs_nn* n, const float* label, float* loss_sum, void* stream);
/* Backward of the mean of that error over the pixels: every parameter's
 * gradient into the object's gradient buffer (overwritten, not accumulated);
 * loss_sum (device, may be NULL) as vs_nn_loss. */
vs_status vs_nn_backward(vs_nn* n, const float* label, float* loss_sum, void* stream);
/* One Adam step (bias-corrected; the object counts the steps) on the
 * gradients of the last backward, then the BF16 copies are refreshed. */
vs_status vs_nn_adam_step(vs_nn* n, float lr, float b1, float b2, float eps, void* stream);
/* Copies of the FP32 parameters and of the last backward's gradients (layer
 * by layer: w [cout][9][cin] then b [cout]) into caller device buffers of
 * *count floats (either may be NULL; count may be NULL); asynchronous. */
vs_status vs_nn_params(vs_nn* n, float* params, float* grads, size_t* count, void* stream);
/* The weight file of vs_load_weights (BF16 weights, FP32 biases) into a host
 * buffer of cap bytes; *nbytes receives its size (blob NULL: size only).
 * vs_nn_load reads one whose layer list equals the object's: the master
 * weights become the stored BF16 values, the Adam state restarts.  Both
 * synchronous. */
vs_status vs_nn_save(vs_nn* n, void* blob, size_t cap, size_t* nbytes);
vs_status vs_nn_load(vs_nn* n, const void* blob, size_t nbytes);

/* The learned surrogate inside the frame.  vs_load_weights copies a weight
 * file into the context: "VSNN", u32 version 1, u32 layers (2..8), f32
 * leaky-ReLU slope, per layer u32 cin and u32 cout, then per layer int16
 * w[cout][9][cin] (BF16 bits) and f32 bias[cout], little endian, packed.  The
 * first layer takes 16 channels, the last gives 16 (channels 0-1: flow),
 * every (cin, cout) is one of vs_nn_conv3x3's.  The network runs on pyramid
 * level 2 of each overlap field (needs flow = 1 and lk_levels >= 3); the
 * input is (Y - 128) / 64 of the template and moving luma in channels 0-1,
 * the output channels 0-1 the flow in level-2 pixels, upsampled x4 to the
 * strip (level-0 x reads level-2 x / 4 - 3 / 8).  Synchronous.
 * vs_set_flow_mode: VS_FLOW_PLAIN (the paper's path), VS_FLOW_SURROGATE (the
 * network's flows for every pair; the plain estimator is not run) or
 * VS_FLOW_SURROGATE_FALLBACK (a pair keeps the network's flows when its mean
 * forward-backward error |U_ij(x) + U_ji(x + U_ij(x))| over the overlap,
 * in 1/256 px fixed point, is below fb_tau_px, 0 <= fb_tau_px <= 1e6; the
 * plain estimator recomputes the other pairs: fb_tau_px = 0 gives the plain
 * path's output bit for bit).  VS_E_UNSUPPORTED without loaded weights.
 * Both calls wait for the device; a batch holding the context recaptures its
 * graph at its next run. */
enum { VS_FLOW_PLAIN = 0, VS_FLOW_SURROGATE = 1, VS_FLOW_SURROGATE_FALLBACK = 2 };
vs_status vs_load_weights(vs_ctx* c, const void* blob, size_t nbytes);
vs_status vs_set_flow_mode(vs_ctx* c, int mode, float fb_tau_px);

/* ------------------------------------------------------------------------
 * Set-up of section 3.1 (host, FP64, once per rig): the coarse pairwise
 * homography from camera parameters and its revision by a skew and a scale
 * matrix estimated on the widened overlap.  Readings of the garbled
 * equations:
 *  - eq. (8): K = [f/dx, 0, cx/dx + u0; 0, f/dy, cy/dy + v0; 0, 0, 1] (the
 *    zero fourth column dropped, the second u0 read as v0);
 *  - eq. (11) on the world plane Z_W = 0: H = K [r1 r2 t], plane coordinates
 *    (X_W, Y_W, 1) to pixels (R row-major, r1 r2 its first two columns);
 *  - eq. (12): H_ab = H_a H_b^-1 maps camera b's pixels to camera a's (so a
 *    rig's H_pair[k] is vs_calib_pair(H_(k-1), H_k));
 *  - eq. (14): H' = M H N with N = diag(s_x, s_y, 1) on the source pixel and M
 *    the translation (t_x, t_y) of the result; p = (t_x, t_y, s_x, s_y).
 * All return VS_E_INVAL on NULL or singular input. */
vs_status vs_calib_intrinsics(double f, double dx, double dy, double cx, double cy, double u0, double v0, double K[9]);
vs_status vs_calib_plane_homography(const double K[9], const double R[9], const double t[3], double H[9]);
vs_status vs_calib_pair(const double Ha[9], const double Hb[9], double Hab[9]);
vs_status vs_calib_refine(const double H[9], const double p[4], double Hr[9]);
/* Estimate p of eq. (13) for the pre-warp H (camera a pixels -> camera b
 * pixels) from two RGB frames (device pointers, HWC bytes, row pitch):
 * Harris corners of a's BT.601 luma (5 x 5 box of central-difference
 * products, k = 0.04) at pixels 8 + radius inside a whose H-image lies in b
 * widened by `margin` px and, rounded, 6 + radius inside b; strict 3 x 3
 * maxima, the 256 strongest; each matched to the integer position within
 * +-radius of its rounded H-image with the best 11 x 11 normalised
 * cross-correlation (kept at correlation >= 0.7), refined to the parabola
 * vertex of its neighbours' scores; two-point RANSAC over every pair of the
 * first 64 matches (Gauss-Newton, inliers within 2 px) and a final
 * Gauss-Newton on the inliers.  The paper matches SURF features instead
 * (the pre-warp leaves a few pixels to find, so a local correlation search
 * does).  1 <= radius <= 7; frames at least 32 x 32.  Synchronous on stream;
 * allocates its scratch.  VS_E_INVAL with fewer than 2 matches or no model
 * (*n_matches, *n_inliers still set). */
vs_status vs_calib_estimate(const uint8_t* frame_a, int pitch_a, int wa, int ha, const uint8_t* frame_b, int pitch_b,
                            int wb, int hb, const double H[9], int margin, int radius, double p[4], int32_t* n_matches,
                            int32_t* n_inliers, void* stream);

/* Plain estimator on caller image pairs (training labels, tests): a context
 * for w x h luma images; vs_flow_run computes, on the whole image, the
 * pyramidal flow of vs_stitch for template yt and moving ym (P_m(x + f) ~
 * P_t(x)) into flow_tm and the reverse flow into flow_mt (FP32 [h][w][2],
 * either may be NULL).  Inputs and outputs are device pointers. */
typedef struct vs_flow vs_flow;
vs_status vs_flow_create(int w, int h, const vs_params* p, vs_flow** out);
vs_status vs_flow_run(vs_flow* f, const float* yt, const float* ym, float* flow_tm, float* flow_mt, void* stream);
vs_status vs_flow_destroy(vs_flow* f);
/* Pyramid level `level` of the last run's template and moving images (FP32,
 * device; either may be NULL) and its size. */
vs_status vs_flow_level(vs_flow* f, int level, float* yt, float* ym, int32_t* w, int32_t* h, void* stream);

/* Steps a5-a6 of a stitch context on a caller strip pair (section 3.2):
 * strip_i (camera i, moving) and strip_j (camera j, template) are w x h RGB
 * HWC byte images (pitch 3 w, device pointers) whose colours are used as
 * given (a5 with the identity colour matrix: Y = (77 R + 150 G + 29 B + 128)
 * >> 8), and flow_ij / flow_ji (FP32 [h][w][2], device, either may be NULL)
 * receive the pyramidal flow of the context's parameters on the whole strip,
 * as vs_flow_run gives it (flow_ij: P_i(x + f) ~ P_j(x)).  The context keeps
 * a plain-flow workspace for the last strip size (allocated, after a device
 * synchronisation, when the size changes; freed by vs_destroy).
 * VS_E_INVAL: null context or strip, w or h < 1, or a size the estimator
 * cannot plan.  Asynchronous on stream. */
vs_status vs_flow_only(vs_ctx* c, const uint8_t* strip_i, const uint8_t* strip_j, int w, int h, float* flow_ij,
                       float* flow_ji, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * estimator of vs_flow_run on one w x h luma pair without a context.  Same
 * arguments and results as vs_flow_create(w, h, p) followed by vs_flow_run
 * (p may be NULL: defaults), bit for bit.  Its plan and workspace live in one
 * static device array of VS_FLOW_NOALLOC_BYTES per GPU, held until the
 * process ends; at the default 4 levels that is about 77 bytes per pixel, so
 * w * h up to about 850 000 (1088 x 768, 384 x 2160) fits.  A pair whose
 * workspace does not fit returns VS_E_INVAL before any device work.  The
 * call allocates nothing: no hipMalloc, no hipFree, no allocating library
 * routine.  It runs on the current device; stream must belong to it.  Every
 * call on a GPU shares that GPU's array and leaves its contents there, so
 * calls that overlap on one GPU (other streams, other threads) race; calls in
 * order on one stream do not.  Asynchronous on stream. */
#define VS_FLOW_NOALLOC_BYTES (64u << 20)
vs_status vs_flow_run_noalloc(int w, int h, const vs_params* p, const float* yt, const float* ym, float* flow_tm,
                              float* flow_mt, void* stream);

#ifdef __cplusplus
}
#endif
#endif
