/*
 * vso_oracle.h -- plain, slow CPU oracle of the per-frame video-stitching path
 * of "GPU Accelerated Color Correction and Frame Warping for Real-time Video
 * Stitching" (arXiv 2308.09209).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the HIP library; the two are independent
 * implementations of the same definitions.
 *
 * Precision: per-pixel geometry, resampling, colour application, the luma
 * pyramid and the flow are FP32 with every operation order spelled out
 * (explicit fmaf, no contraction), because each of them decides a uint8 output
 * and the workload fixes FP32 coordinates; the colour-matrix solve and the
 * balancing curve are FP64; histograms, quantiles and moments are exact
 * integers.
 *
 * Parity pins: see the "not gpu" tests.  The only step whose shape the paper
 * does not pin is the balancing curve of section 2.2 (its figure is missing):
 * "parity unpinned" against the paper; invariants pin it.
 */
#ifndef VSO_ORACLE_H
#define VSO_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#define VSO_MAX_CAMS 16
#define VSO_MAX_PAIRS 16
#define VSO_MAX_LEVELS 6

enum {
    VSO_OK = 0,
    VSO_E_INVAL = -1,
    VSO_E_GEOMETRY = -2,
    VSO_E_NOMEM = -3,
};

typedef struct {
    int n_cams;
    int cam_w[VSO_MAX_CAMS];
    int cam_h[VSO_MAX_CAMS];
    double H_pair[VSO_MAX_CAMS][9]; /* [k], k >= 1: camera k pixel -> camera k-1 pixel, row-major */
    double H_ref[9];                /* camera 0 pixel -> canvas pixel */
    int ring;                       /* 1: 360-degree ring, canvas periodic in x */
    int ring_period;                /* canvas period in px (ring only) */
    int canvas_w, canvas_h;
} vso_rig;

typedef struct {
    int color_window;   /* 0: no colour transfer; 1: 2D-M (frame T only); 2..3: 3D-M window */
    double ridge;       /* relative ridge of the colour solve (x trace) */
    int min_pixels;     /* fewer overlap samples than this -> M = I */
    int flow;           /* 0: zero flow; 1: pyramidal Lucas-Kanade; 2: variational (vso_var.c) */
    int lk_levels, lk_iters, lk_radius;
    float lk_lambda;
    int balance;        /* 0: skip the balancing LUT apply; 1: apply */
    int lambda_pct;     /* balancing quantile, percent (5 -> lambda = 0.05) */
    int readings;       /* the literal readings the default ones replace, a bit mask of
                           VSO_READ_*; 0: the adopted readings */
    float var_alpha;    /* flow = 2 (variational): smoothness weight */
    float var_gamma;    /*   gradient-constancy weight */
    int var_outer;      /*   warps per level */
    int var_inner;      /*   Jacobi steps per warp */
} vso_params;

/* Literal readings of passages the default path reads otherwise:
 *  OVERLAP_ONLY  eq. (4)'s text: each pair's matrix corrects camera i only
 *                inside that pair's overlap, uncomposed; every other pixel
 *                keeps its raw colour (default: the matrices chained to
 *                camera 0 correct whole frames);
 *  LITERAL_EQ17  eq. (17) as printed: camera i is displaced by theta_i flow_ij
 *                and camera j by theta_j flow_ji (default: theta_j flow_ij and
 *                theta_i flow_ji, the warps meeting in the middle);
 *  NEAREST_CDF   section 2.1 step 3 with the level whose cumulative count is
 *                nearest, ties to the lower level (default: the first level
 *                whose cumulative count reaches it). */
enum { VSO_READ_OVERLAP_ONLY = 1, VSO_READ_LITERAL_EQ17 = 2, VSO_READ_NEAREST_CDF = 4 };

void vso_default_params(vso_params* p);

typedef struct vso_ctx vso_ctx;

/* Build the plan of section 2.1 step 1 / section 3.1 (camera-to-canvas
 * homographies, coverage, overlap pairs and strips).  Returns NULL and sets
 * *status on error. */
vso_ctx* vso_create(const vso_rig* rig, const vso_params* p, int* status);
void vso_destroy(vso_ctx* c);

typedef struct {
    int canvas_w, canvas_h, n_pairs, n_cams, ring, ring_period;
    int pair_j[VSO_MAX_PAIRS], pair_i[VSO_MAX_PAIRS], pair_si[VSO_MAX_PAIRS];
    int strip_x0[VSO_MAX_PAIRS], strip_y0[VSO_MAX_PAIRS];
    int strip_w[VSO_MAX_PAIRS], strip_h[VSO_MAX_PAIRS];
    float hinv[VSO_MAX_CAMS][9];   /* canvas -> camera k, FP32 */
    double hk[VSO_MAX_CAMS][9];    /* camera k -> canvas, FP64 */
    long long n_covered;
} vso_plan_info;
int vso_plan_info_get(const vso_ctx* c, vso_plan_info* out);

/* One frame: frames[k] is camera k's HWC RGB uint8 image with row pitch
 * pitch[k] bytes; pano receives canvas_h x canvas_w x 3 uint8 (tight).  Uses
 * and advances the context's colour state. */
int vso_stitch(vso_ctx* c, const uint8_t* const frames[], const int pitch[], uint8_t* pano);
/* Forget the colour state (next frame is T = 0). */
void vso_reset(vso_ctx* c);
int vso_frames_seen(const vso_ctx* c);
/* Wall seconds spent per step since the context was created, summed over
 * frames: strips, moments (histogram specification), colour solve,
 * pyramids, flow, blend, balance.  Timing only; no effect on results. */
int vso_step_times(const vso_ctx* c, double out[7]);

enum {
    VSO_TAP_STRIP = 1,     /* pair, sub 0=j 1=i : sw*sh*3 u8 */
    VSO_TAP_MASK = 2,      /* pair : sw*sh u8 */
    VSO_TAP_HIST = 3,      /* pair : [2][3][256] u32, [0]=camera j, [1]=camera i */
    VSO_TAP_LUT = 4,       /* pair : [3][256] u8 */
    VSO_TAP_MOM = 5,       /* pair : 16 u64 = A[6] (00,01,02,11,12,22), B[9] row-major, n */
    VSO_TAP_MPAIR = 6,     /* [n_pairs][9] f64 */
    VSO_TAP_MK = 7,        /* [n_cams][9] f32 */
    VSO_TAP_FLAGS = 8,     /* [n_pairs] i32 */
    VSO_TAP_PYR = 9,       /* pair, sub = cam*8 + level : w_l*h_l f32 */
    VSO_TAP_FLOW = 10,     /* pair, sub 0=ij 1=ji : sw*sh*2 f32 */
    VSO_TAP_PANO_PRE = 11, /* canvas_h*canvas_w*3 u8 */
    VSO_TAP_PANO_HIST = 12,/* [3][256] u32 */
    VSO_TAP_BAL_LUT = 13,  /* [3][256] u8 */
    VSO_TAP_QUANT = 14,    /* [3][2] i32 : q1, q2 of frame T */
    VSO_TAP_MBAR = 15,     /* [3][2] f64 */
    VSO_TAP_COVER = 16,    /* canvas_h*canvas_w u8 : number of covering cameras */
    VSO_TAP_NEED = 17,     /* pair, sub = level : w_l*h_l u8, 1 where the flow is estimated */
    VSO_TAP_SURR_PRED = 18,/* pair, sub 0=ij 1=ji : level-2 surrogate prediction w_2*h_2*2 f32 */
    VSO_TAP_FB = 19,       /* [n_pairs][2] u64 : forward-backward error sum (1/256 px), pixel count */
    VSO_TAP_SURR_OK = 20,  /* [n_pairs] i32 : 1 where the pair kept the surrogate's flows */
};
int vso_get(const vso_ctx* c, int tap, int pair, int sub, void* dst, size_t nbytes);

/* ---- individual steps, exposed for the pins ---- */
void vso_histspec_lut(const uint32_t Gi[256], const uint32_t Gj[256], uint8_t lut[256]);
void vso_histspec_lut_nearest(const uint32_t Gi[256], const uint32_t Gj[256], uint8_t lut[256]);
/* (A + eps I) M = B + eps I, eps = ridge * trace(A); returns 0 ok, 1 singular */
int vso_solve_color(const double A[9], const double B[9], double ridge, double M[9]);
void vso_quantiles(const uint32_t hist[256], long long n, int lambda_pct, int* q1, int* q2);
void vso_balance_lut(double m1, double m2, int lambda_pct, uint8_t lut[256]);
void vso_pyr_down(const float* src, int w, int h, float* dst);
void vso_lk_level(const float* T, const float* Mv, int w, int h,
                  const float* u_coarse, int wc, int hc,
                  int radius, int iters, float lambda, const uint8_t* need, float* u_out);
void vso_lk_level_f64(const double* T, const double* Mv, int w, int h,
                      const double* u_coarse, int wc, int hc,
                      int radius, int iters, double lambda, double* u_out);
int vso_hom_valid(const float h[9], float x, float y, int W, int H, float* u, float* v);
float vso_bilinear(const uint8_t* F, int pitch, int W, int H, int ch, float u, float v);
int vso_round8(float r);
/* integer luma of the flow input: (77 R + 150 G + 29 B + 128) >> 8 */
int vso_luma(int r, int g, int b);
/* eq. (4) chained to camera 0: Mpair [n_cams - 1][9] (pair k - 1 = cameras
 * k - 1, k), Mk [n_cams][9], FP64 */
void vso_chain_colour(const double* Mpair, int n_cams, double* Mk);
/* One camera's view of a canvas pixel for the fusion of eqs. (16)-(18). */
typedef struct {
    const uint8_t* frame; /* HWC RGB uint8 */
    int pitch, W, H;      /* row pitch in bytes, image size */
    const float* hinv;    /* canvas -> camera homography, FP32 */
    const float* M;       /* the camera's colour matrix (row vectors), FP32 */
    float X;              /* the pixel's canvas x in this camera's period */
} vso_view;
/* eqs. (16)-(18) at one canvas pixel (row y) covered by cameras j (left) and
 * i (right), with the pair's flows f_ij, f_ji at the pixel */
void vso_fuse_pixel(const vso_view* vj, const vso_view* vi, float y, const float f_ij[2], const float f_ji[2],
                    uint8_t out[3]);
/* the same with eq. (17) as printed (VSO_READ_LITERAL_EQ17) */
void vso_fuse_pixel_literal(const vso_view* vj, const vso_view* vi, float y, const float f_ij[2],
                            const float f_ji[2], uint8_t out[3]);

/* learned surrogate: FP64 3x3 convolution references (NHWC, weights
 * [cout][tap][cin], zero padding) */
void vso_conv3x3(const double* x, int n, int h, int w, int cin, const double* wt, const double* b, int cout,
                 double* y);
void vso_conv3x3_bwd_data(const double* dy, int n, int h, int w, int cout, const double* wt, int cin, double* dx);
void vso_conv3x3_bwd_weight(const double* x, const double* dy, int n, int h, int w, int cin, int cout, double* dw,
                            double* db);

/* The learned flow surrogate inside the frame (an addition to the paper's
 * method).  blob: weight file ("VSNN" v1, see vso_oracle.c), copied; may be
 * NULL to keep the loaded one.  mode 0: plain flow; 1: the surrogate's flows
 * for every pair; 2: the surrogate's flows where the pair's mean
 * forward-backward error is below tau px (fixed point 1/256 px), the plain
 * estimator elsewhere.  Needs lk_levels >= 3. */
int vso_set_surrogate(vso_ctx* c, const void* blob, size_t n, int mode, float tau);
/* its steps, exposed for the pins */
int vso_surrogate_net(const void* blob, size_t n, const float* yt, const float* ym, int w, int h, float* pred);
void vso_surr_upsample(const float* pred, int w2, int h2, const uint8_t* need0, int w0, int h0, float* flow0);
void vso_fb_check(const float* pred_ij, const float* pred_ji, int w2, int h2, const uint8_t* need0, int w0, int h0,
                  unsigned long long* sum, unsigned long long* count);

/* Section 3.1 set-up (vso_calib.c): camera parameters -> homographies
 * (eqs. (8)-(12)), the revision of eqs. (13)-(14) and its estimation from
 * matched points.  Readings in vso_calib.c. */
void vso_calib_intrinsics(double f, double dx, double dy, double cx, double cy, double u0, double v0, double K[9]);
void vso_calib_plane_homography(const double K[9], const double R[9], const double t[3], double H[9]);
int vso_calib_pair(const double Ha[9], const double Hb[9], double Hab[9]);
void vso_calib_refine(const double H[9], const double p[4], double Hr[9]);
float vso_calib_harris(const float* Y, int w, int x, int y);
float vso_calib_ncc(const float* A, int wa, int xa, int ya, const float* B, int wb, int xb, int yb);
int vso_calib_estimate(const uint8_t* Fa, int pa, int wa, int ha, const uint8_t* Fb, int pb, int wb, int hb,
                       const double H[9], int margin, int radius, double out[4], int* n_matches, int* n_inliers);

/* The variational flow alternative (vso_var.c): one level on flow (in: the
 * initial flow, out: the result, [h][w][2]), and the coarse-to-fine driver. */
void vso_var_level(const float* T, const float* Mv, const uint8_t* need, int w, int h, float alpha, float gamma,
                   int outer, int inner, float* flow);
void vso_var_pyramid(const float* const* T, const float* const* Mv, const uint8_t* const* need, const int* w,
                     const int* h, int levels, float alpha, float gamma, int outer, int inner, float* flow0);
#endif
