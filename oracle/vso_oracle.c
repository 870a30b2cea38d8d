/*
 * vso_oracle.c -- plain CPU oracle of the per-frame stitching path of
 * arXiv 2308.09209.  TEST INFRASTRUCTURE ONLY (see vso_oracle.h).
 *
 * Written straight from the paper's sections and equations plus the readings
 * listed where the paper is silent; direct per-pixel sums and loops, no
 * histogram tricks, no tiling.  OpenMP is used only over independent output
 * pixels; every accumulation that crosses pixels is a serial loop.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no contraction:
 * every fused multiply-add below is an explicit fmaf).
 */
#include "vso_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define NCH 3

/* ------------------------------------------------------------------------ */
/* Global conventions                                                        */
/* ------------------------------------------------------------------------ */

/* round-half-up to a byte: clamp(floor(r + 0.5), 0, 255) */
int vso_round8(float r)
{
    float f = floorf(r + 0.5f);
    if (f < 0.0f) f = 0.0f;
    if (f > 255.0f) f = 255.0f;
    return (int)f;
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
static float clampf(float v, float lo, float hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Apply a canvas->camera homography (section 3.1) in FP32:
 *   nu = h0 x + (h1 y + h2), nv = h3 x + (h4 y + h5), w = h6 x + (h7 y + h8),
 * each as two fused multiply-adds, then u = nu / w, v = nv / w.
 * Valid iff w > 0 and (u, v) lies in [0, W-1] x [0, H-1].  When w <= 0 the
 * position is defined as (0, 0). */
int vso_hom_valid(const float h[9], float x, float y, int W, int H, float* u, float* v)
{
    float nu = fmaf(h[0], x, fmaf(h[1], y, h[2]));
    float nv = fmaf(h[3], x, fmaf(h[4], y, h[5]));
    float w = fmaf(h[6], x, fmaf(h[7], y, h[8]));
    if (!(w > 0.0f)) {
        *u = 0.0f;
        *v = 0.0f;
        return 0;
    }
    *u = nu / w;
    *v = nv / w;
    return (*u >= 0.0f) && (*u <= (float)(W - 1)) && (*v >= 0.0f) && (*v <= (float)(H - 1));
}

/* Bilinear sample of channel ch of an HWC uint8 image at (u, v): the
 * position is clamped into the image, x0 = floor(u), fx = u - x0,
 * x1 = min(x0 + 1, W - 1) (same in y), and
 *   a = fx (p10 - p00) + p00, b = fx (p11 - p01) + p01, r = fy (b - a) + a
 * each as one fused multiply-add. */
float vso_bilinear(const uint8_t* F, int pitch, int W, int H, int ch, float u, float v)
{
    float uc = clampf(u, 0.0f, (float)(W - 1));
    float vc = clampf(v, 0.0f, (float)(H - 1));
    float flx = floorf(uc), fly = floorf(vc);
    int x0 = (int)flx, y0 = (int)fly;
    float fx = uc - flx, fy = vc - fly;
    int x1 = x0 + 1 < W ? x0 + 1 : W - 1;
    int y1 = y0 + 1 < H ? y0 + 1 : H - 1;
    float p00 = (float)F[(size_t)y0 * pitch + (size_t)x0 * NCH + ch];
    float p10 = (float)F[(size_t)y0 * pitch + (size_t)x1 * NCH + ch];
    float p01 = (float)F[(size_t)y1 * pitch + (size_t)x0 * NCH + ch];
    float p11 = (float)F[(size_t)y1 * pitch + (size_t)x1 * NCH + ch];
    float a = fmaf(fx, p10 - p00, p00);
    float b = fmaf(fx, p11 - p01, p01);
    return fmaf(fy, b - a, a);
}

/* Colour application, row-vector convention of eq. (4): t = s . M, i.e.
 * t_c = s_R M[0][c] + s_G M[1][c] + s_B M[2][c], evaluated as
 * fmaf(s_R, M0c, fmaf(s_G, M1c, s_B * M2c)) and clamped to [0, 255]. */
static float color_apply(const float s[3], const float M[9], int c)
{
    float t = fmaf(s[0], M[0 * 3 + c], fmaf(s[1], M[1 * 3 + c], s[2] * M[2 * 3 + c]));
    return clampf(t, 0.0f, 255.0f);
}

/* ------------------------------------------------------------------------ */
/* Context                                                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t A[6], B[9], n;
} moments;

struct vso_ctx {
    vso_rig rig;
    vso_params prm;
    vso_plan_info plan;
    uint8_t* cover;                          /* coverage count per canvas pixel */
    /* colour state: moments of frames T-1, T-2 per pair; quantiles of T-1, T-2 */
    int T;
    moments mom_prev[VSO_MAX_PAIRS][2];
    int q_prev[2][3][2];
    /* taps of the last frame */
    uint8_t* strip[VSO_MAX_PAIRS][2];
    uint8_t* mask[VSO_MAX_PAIRS];
    uint32_t hist[VSO_MAX_PAIRS][2][3][256];
    uint8_t lut[VSO_MAX_PAIRS][3][256];
    moments mom[VSO_MAX_PAIRS];
    double Mpair[VSO_MAX_PAIRS][9];
    float Mk[VSO_MAX_CAMS][9];
    float Mpf[VSO_MAX_PAIRS][9];   /* the pair matrices in FP32 (overlap-only reading) */
    int flags[VSO_MAX_PAIRS];
    float* pyr[VSO_MAX_PAIRS][2][VSO_MAX_LEVELS];
    uint8_t* need[VSO_MAX_PAIRS][VSO_MAX_LEVELS];
    int pw[VSO_MAX_PAIRS][VSO_MAX_LEVELS], ph[VSO_MAX_PAIRS][VSO_MAX_LEVELS];
    float* flow[VSO_MAX_PAIRS][2];
    /* learned flow surrogate (mode 0: the plain estimator only) */
    int surr_mode;
    unsigned long long surr_tau_fix;          /* fallback threshold, 1/256 px */
    void* surr_blob;
    size_t surr_blob_n;
    float* surr_pred[VSO_MAX_PAIRS][2];       /* level-2 prediction, 2 channels */
    unsigned long long fb[VSO_MAX_PAIRS][2];  /* fixed-point error sum, pixel count */
    int surr_ok[VSO_MAX_PAIRS];
    double step_s[7];                        /* wall seconds per step, summed over frames */
    uint8_t* pano_pre;
    uint32_t pano_hist[3][256];
    uint8_t bal_lut[3][256];
    int quant[3][2];
    double mbar[3][2];
};

void vso_default_params(vso_params* p)
{
    p->color_window = 3;
    p->ridge = 1e-9;
    p->min_pixels = 64;
    p->flow = 1;
    p->lk_levels = 4;
    p->lk_iters = 5;
    p->lk_radius = 4;
    p->lk_lambda = 256.0f;
    p->balance = 1;
    p->lambda_pct = 5;
    p->readings = 0;
    p->var_alpha = 128.0f;
    p->var_gamma = 16.0f;
    p->var_outer = 3;
    p->var_inner = 10;
}

/* 3x3 product c = a b, each entry ((a_r0 b_0c + a_r1 b_1c) + a_r2 b_2c). */
static void mat3_mul(const double a[9], const double b[9], double c[9])
{
    double t[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k)
            t[r * 3 + k] = (a[r * 3 + 0] * b[0 * 3 + k] + a[r * 3 + 1] * b[1 * 3 + k]) + a[r * 3 + 2] * b[2 * 3 + k];
    memcpy(c, t, sizeof t);
}

/* Inverse of a homography, normalised so that its last entry is +1: the
 * adjugate divided by the adjugate's last entry.  Fails if the determinant
 * is not finite and non-zero or the last adjugate entry is zero. */
static int hom_inverse(const double a[9], double inv[9])
{
    double adj[9];
    adj[0] = a[4] * a[8] - a[5] * a[7];
    adj[1] = a[2] * a[7] - a[1] * a[8];
    adj[2] = a[1] * a[5] - a[2] * a[4];
    adj[3] = a[5] * a[6] - a[3] * a[8];
    adj[4] = a[0] * a[8] - a[2] * a[6];
    adj[5] = a[2] * a[3] - a[0] * a[5];
    adj[6] = a[3] * a[7] - a[4] * a[6];
    adj[7] = a[1] * a[6] - a[0] * a[7];
    adj[8] = a[0] * a[4] - a[1] * a[3];
    double det = (a[0] * adj[0] + a[1] * adj[3]) + a[2] * adj[6];
    if (!isfinite(det) || det == 0.0 || adj[8] == 0.0 || !isfinite(adj[8])) return -1;
    /* a positive multiple of H^-1 (so that w > 0 keeps meaning "in front of
     * the camera") whose last entry is +-1: the adjugate over |adj[8]| with the
     * sign of det */
    const double den = ((det > 0.0) == (adj[8] > 0.0)) ? adj[8] : -adj[8];
    for (int i = 0; i < 9; ++i) inv[i] = adj[i] / den;
    return 0;
}

/* Coverage of one canvas pixel: every (camera, period shift) whose image
 * contains it.  Returns the count (up to 4 recorded). */
typedef struct {
    int cam, m;
    float u, v;
} hit;

static int cover_pixel(const vso_ctx* c, int x, int y, hit h[4])
{
    const vso_plan_info* P = &c->plan;
    int n = 0;
    for (int k = 0; k < P->n_cams; ++k) {
        for (int m = -1; m <= 1; ++m) {
            if (!P->ring && m != 0) continue;
            float u, v;
            int X = x + m * P->ring_period;
            if (vso_hom_valid(P->hinv[k], (float)X, (float)y, c->rig.cam_w[k], c->rig.cam_h[k], &u, &v)) {
                if (n < 4) {
                    h[n].cam = k;
                    h[n].m = m;
                    h[n].u = u;
                    h[n].v = v;
                }
                ++n;
            }
        }
    }
    return n;
}

/* Which overlap pair a doubly covered pixel belongs to; -1 if none.
 * Pair p joins cameras (j, i); camera i sits si periods to the right of its
 * own canvas position in the pair's coordinates, so a canvas pixel covered by
 * j at shift mj and by i at shift mi belongs to p iff mj == mi + si. */
static int pair_for(const vso_plan_info* P, const hit* a, const hit* b, int* jidx)
{
    for (int p = 0; p < P->n_pairs; ++p) {
        const hit *hj = NULL, *hi = NULL;
        if (a->cam == P->pair_j[p] && b->cam == P->pair_i[p]) {
            hj = a;
            hi = b;
        } else if (b->cam == P->pair_j[p] && a->cam == P->pair_i[p]) {
            hj = b;
            hi = a;
        } else {
            continue;
        }
        if (hj->m != hi->m + P->pair_si[p]) continue;
        *jidx = (hj == a) ? 0 : 1;
        return p;
    }
    return -1;
}

/* Plan (section 2.1 step 1, section 3.1): camera k -> canvas is
 * H_k = H_ref H_{1,0} ... H_{k,k-1}; the overlap of neighbouring cameras is
 * found by testing every canvas pixel against every camera. */
static int build_plan(vso_ctx* c)
{
    const vso_rig* R = &c->rig;
    vso_plan_info* P = &c->plan;
    memset(P, 0, sizeof *P);
    if (R->n_cams < 2 || R->n_cams > VSO_MAX_CAMS) return VSO_E_INVAL;
    if (R->canvas_w <= 0 || R->canvas_h <= 0) return VSO_E_INVAL;
    if (R->ring && (R->n_cams < 3 || R->ring_period != R->canvas_w)) return VSO_E_INVAL;
    for (int k = 0; k < R->n_cams; ++k)
        if (R->cam_w[k] < 2 || R->cam_h[k] < 2) return VSO_E_INVAL;
    P->canvas_w = R->canvas_w;
    P->canvas_h = R->canvas_h;
    P->n_cams = R->n_cams;
    P->ring = R->ring;
    P->ring_period = R->ring ? R->ring_period : 0;

    double Hk[9];
    memcpy(Hk, R->H_ref, sizeof Hk);
    for (int k = 0; k < R->n_cams; ++k) {
        if (k > 0) mat3_mul(Hk, R->H_pair[k], Hk);
        for (int i = 0; i < 9; ++i)
            if (!isfinite(Hk[i])) return VSO_E_INVAL;
        memcpy(P->hk[k], Hk, sizeof Hk);
        double inv[9];
        if (hom_inverse(Hk, inv) != 0) return VSO_E_INVAL;
        for (int i = 0; i < 9; ++i) P->hinv[k][i] = (float)inv[i];
    }
    /* pairs: (k-1, k) along the chain, plus (N-1, 0) closing a ring */
    P->n_pairs = R->n_cams - 1 + (R->ring ? 1 : 0);
    for (int p = 0; p < R->n_cams - 1; ++p) {
        P->pair_j[p] = p;
        P->pair_i[p] = p + 1;
        P->pair_si[p] = 0;
    }
    if (R->ring) {
        P->pair_j[R->n_cams - 1] = R->n_cams - 1;
        P->pair_i[R->n_cams - 1] = 0;
        P->pair_si[R->n_cams - 1] = 1;
    }
    int bx0[VSO_MAX_PAIRS], bx1[VSO_MAX_PAIRS], by0[VSO_MAX_PAIRS], by1[VSO_MAX_PAIRS];
    for (int p = 0; p < P->n_pairs; ++p) {
        bx0[p] = by0[p] = 1 << 30;
        bx1[p] = by1[p] = -(1 << 30);
    }
    c->cover = (uint8_t*)calloc((size_t)P->canvas_w * P->canvas_h, 1);
    if (!c->cover) return VSO_E_NOMEM;
    int err = 0;
    long long ncov = 0;
    for (int y = 0; y < P->canvas_h; ++y) {
        for (int x = 0; x < P->canvas_w; ++x) {
            hit h[4];
            int n = cover_pixel(c, x, y, h);
            c->cover[(size_t)y * P->canvas_w + x] = (uint8_t)(n > 255 ? 255 : n);
            if (n > 0) ++ncov;
            if (n > 2) err = 1;
            if (n == 2) {
                int jidx;
                int p = pair_for(P, &h[0], &h[1], &jidx);
                if (p < 0) {
                    err = 1;
                    continue;
                }
                int X = x + h[jidx].m * P->ring_period;
                if (X < bx0[p]) bx0[p] = X;
                if (X > bx1[p]) bx1[p] = X;
                if (y < by0[p]) by0[p] = y;
                if (y > by1[p]) by1[p] = y;
            }
        }
    }
    P->n_covered = ncov;
    if (err || ncov == 0) return VSO_E_GEOMETRY;
    for (int p = 0; p < P->n_pairs; ++p) {
        if (bx1[p] < bx0[p]) return VSO_E_GEOMETRY;
        P->strip_x0[p] = bx0[p];
        P->strip_y0[p] = by0[p];
        P->strip_w[p] = bx1[p] - bx0[p] + 1;
        P->strip_h[p] = by1[p] - by0[p] + 1;
    }
    return VSO_OK;
}

static void free_ctx(vso_ctx* c)
{
    if (!c) return;
    free(c->cover);
    for (int p = 0; p < VSO_MAX_PAIRS; ++p) {
        free(c->strip[p][0]);
        free(c->strip[p][1]);
        free(c->mask[p]);
        free(c->flow[p][0]);
        free(c->flow[p][1]);
        for (int k = 0; k < 2; ++k)
            for (int l = 0; l < VSO_MAX_LEVELS; ++l) free(c->pyr[p][k][l]);
        for (int l = 0; l < VSO_MAX_LEVELS; ++l) free(c->need[p][l]);
        free(c->surr_pred[p][0]);
        free(c->surr_pred[p][1]);
    }
    free(c->surr_blob);
    free(c->pano_pre);
    free(c);
}

vso_ctx* vso_create(const vso_rig* rig, const vso_params* prm, int* status)
{
    vso_ctx* c = (vso_ctx*)calloc(1, sizeof *c);
    if (!c) {
        *status = VSO_E_NOMEM;
        return NULL;
    }
    c->rig = *rig;
    if (prm) c->prm = *prm;
    else vso_default_params(&c->prm);
    if (c->prm.lk_levels < 1 || c->prm.lk_levels > VSO_MAX_LEVELS || c->prm.lk_iters < 0 ||
        c->prm.lk_radius < 0 || c->prm.color_window < 0 || c->prm.color_window > 3 ||
        c->prm.lambda_pct < 0 || c->prm.lambda_pct >= 50) {
        *status = VSO_E_INVAL;
        free_ctx(c);
        return NULL;
    }
    int st = build_plan(c);
    if (st != VSO_OK) {
        *status = st;
        free_ctx(c);
        return NULL;
    }
    const vso_plan_info* P = &c->plan;
    for (int p = 0; p < P->n_pairs; ++p) {
        size_t n = (size_t)P->strip_w[p] * P->strip_h[p];
        c->strip[p][0] = (uint8_t*)calloc(n * 3, 1);
        c->strip[p][1] = (uint8_t*)calloc(n * 3, 1);
        c->mask[p] = (uint8_t*)calloc(n, 1);
        c->flow[p][0] = (float*)calloc(n * 2, sizeof(float));
        c->flow[p][1] = (float*)calloc(n * 2, sizeof(float));
        int w = P->strip_w[p], h = P->strip_h[p];
        for (int l = 0; l < c->prm.lk_levels; ++l) {
            c->pw[p][l] = w;
            c->ph[p][l] = h;
            for (int k = 0; k < 2; ++k) c->pyr[p][k][l] = (float*)calloc((size_t)w * h, sizeof(float));
            c->need[p][l] = (uint8_t*)calloc((size_t)w * h, 1);
            w = (w + 1) / 2;
            h = (h + 1) / 2;
        }
    }
    c->pano_pre = (uint8_t*)calloc((size_t)P->canvas_w * P->canvas_h * 3, 1);
    *status = VSO_OK;
    return c;
}

void vso_destroy(vso_ctx* c) { free_ctx(c); }

int vso_plan_info_get(const vso_ctx* c, vso_plan_info* out)
{
    *out = c->plan;
    return VSO_OK;
}

void vso_reset(vso_ctx* c)
{
    c->T = 0;
    memset(c->mom_prev, 0, sizeof c->mom_prev);
    memset(c->q_prev, 0, sizeof c->q_prev);
}

int vso_frames_seen(const vso_ctx* c) { return c->T; }

int vso_step_times(const vso_ctx* c, double out[7])
{
    if (!c || !out) return VSO_E_INVAL;
    memcpy(out, c->step_s, sizeof c->step_s);
    return VSO_OK;
}

/* ------------------------------------------------------------------------ */
/* Section 2.1: 3D-M colour transfer                                         */
/* ------------------------------------------------------------------------ */

/* Step 3, histogram specification of G_i onto G_j (image j is the reference):
 * with cumulative counts C_i, C_j over the same overlap pixels,
 *   LUT(v) = min { w : C_j(w) >= C_i(v) }. */
void vso_histspec_lut(const uint32_t Gi[256], const uint32_t Gj[256], uint8_t lut[256])
{
    uint64_t Ci[256], Cj[256];
    uint64_t si = 0, sj = 0;
    for (int v = 0; v < 256; ++v) {
        si += Gi[v];
        sj += Gj[v];
        Ci[v] = si;
        Cj[v] = sj;
    }
    for (int v = 0; v < 256; ++v) {
        int w = 0;
        while (w < 255 && Cj[w] < Ci[v]) ++w;
        lut[v] = (uint8_t)w;
    }
}

/* Step 3 read with the nearest cumulative count (VSO_READ_NEAREST_CDF):
 *   LUT(v) = the smallest w minimising |C_j(w) - C_i(v)|, by brute force. */
void vso_histspec_lut_nearest(const uint32_t Gi[256], const uint32_t Gj[256], uint8_t lut[256])
{
    long long Ci[256], Cj[256];
    long long si = 0, sj = 0;
    for (int v = 0; v < 256; ++v) {
        si += Gi[v];
        sj += Gj[v];
        Ci[v] = si;
        Cj[v] = sj;
    }
    for (int v = 0; v < 256; ++v) {
        int best = 0;
        long long bd = -1;
        for (int w = 0; w < 256; ++w) {
            long long d = Cj[w] - Ci[v];
            if (d < 0) d = -d;
            if (bd < 0 || d < bd) {
                bd = d;
                best = w;
            }
        }
        lut[v] = (uint8_t)best;
    }
}

/* Eq. (1)/(3): M = [I_i^T I_i]^-1 I_i^T I_j with the 3D stacking of eq. (2)
 * entering as summed moments.  Solved as (A + eps I) M = B + eps I with
 * eps = ridge * trace(A) (a small pull toward the identity that keeps A = B
 * exactly at M = I), by Gaussian elimination with partial pivoting (first
 * largest |pivot| on ties) and back substitution, all FP64.  Returns 1 and
 * M = I if the smallest pivot is below 1e-12 of the largest |entry|. */
int vso_solve_color(const double A[9], const double B[9], double ridge, double M[9])
{
    double a[3][3], b[3][3];
    double eps = ridge * ((A[0] + A[4]) + A[8]);
    double maxabs = 0.0;
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            a[r][k] = A[r * 3 + k] + (r == k ? eps : 0.0);
            b[r][k] = B[r * 3 + k] + (r == k ? eps : 0.0);
            if (fabs(a[r][k]) > maxabs) maxabs = fabs(a[r][k]);
        }
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        for (int r = col + 1; r < 3; ++r)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (piv != col) {
            for (int k = 0; k < 3; ++k) {
                double t = a[col][k];
                a[col][k] = a[piv][k];
                a[piv][k] = t;
                t = b[col][k];
                b[col][k] = b[piv][k];
                b[piv][k] = t;
            }
        }
        if (!(fabs(a[col][col]) >= 1e-12 * maxabs) || a[col][col] == 0.0) {
            for (int i = 0; i < 9; ++i) M[i] = (i % 4 == 0) ? 1.0 : 0.0;
            return 1;
        }
        for (int r = col + 1; r < 3; ++r) {
            double f = a[r][col] / a[col][col];
            for (int k = col; k < 3; ++k) a[r][k] = a[r][k] - f * a[col][k];
            for (int k = 0; k < 3; ++k) b[r][k] = b[r][k] - f * b[col][k];
        }
    }
    double x[3][3];
    for (int r = 2; r >= 0; --r) {
        for (int k = 0; k < 3; ++k) {
            double s = b[r][k];
            for (int q = r + 1; q < 3; ++q) s = s - a[r][q] * x[q][k];
            x[r][k] = s / a[r][r];
        }
    }
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) M[r * 3 + k] = x[r][k];
    return 0;
}

/* Steps 1-2: pre-warp both cameras of every pair onto its overlap strip
 * (bilinear, rounded to bytes), the overlap mask (covered by both), and the
 * per-channel histograms over the mask. */
static void step_strips(vso_ctx* c, const uint8_t* const F[], const int pitch[])
{
    const vso_plan_info* P = &c->plan;
    for (int p = 0; p < P->n_pairs; ++p) {
        int sw = P->strip_w[p], sh = P->strip_h[p];
        int cams[2] = {P->pair_j[p], P->pair_i[p]};
        int shifts[2] = {0, P->pair_si[p]};
#pragma omp parallel for schedule(static)
        for (int ly = 0; ly < sh; ++ly) {
            for (int lx = 0; lx < sw; ++lx) {
                int X = P->strip_x0[p] + lx, Y = P->strip_y0[p] + ly;
                int ok = 1;
                for (int s = 0; s < 2; ++s) {
                    int k = cams[s];
                    float u, v;
                    int xs = X - shifts[s] * P->ring_period;
                    int val = vso_hom_valid(P->hinv[k], (float)xs, (float)Y, c->rig.cam_w[k], c->rig.cam_h[k], &u, &v);
                    ok = ok && val;
                    for (int ch = 0; ch < 3; ++ch) {
                        float r = vso_bilinear(F[k], pitch[k], c->rig.cam_w[k], c->rig.cam_h[k], ch, u, v);
                        c->strip[p][s][((size_t)ly * sw + lx) * 3 + ch] = (uint8_t)vso_round8(r);
                    }
                }
                c->mask[p][(size_t)ly * sw + lx] = (uint8_t)ok;
            }
        }
        memset(c->hist[p], 0, sizeof c->hist[p]);
        for (size_t q = 0; q < (size_t)sw * sh; ++q) {
            if (!c->mask[p][q]) continue;
            for (int s = 0; s < 2; ++s)
                for (int ch = 0; ch < 3; ++ch) c->hist[p][s][ch][c->strip[p][s][q * 3 + ch]]++;
        }
    }
}

/* Steps 3-4: histogram-specification LUT per channel and the exact integer
 * moments A = I_i^T I_i and B = I_i^T I_j, where I_i holds the raw overlap
 * pixels of camera i and I_j the same pixels revised by the LUT (eq. (1)). */
static void step_moments(vso_ctx* c)
{
    const vso_plan_info* P = &c->plan;
    for (int p = 0; p < P->n_pairs; ++p) {
        for (int ch = 0; ch < 3; ++ch) {
            if (c->prm.readings & VSO_READ_NEAREST_CDF)
                vso_histspec_lut_nearest(c->hist[p][1][ch], c->hist[p][0][ch], c->lut[p][ch]);
            else
                vso_histspec_lut(c->hist[p][1][ch], c->hist[p][0][ch], c->lut[p][ch]);
        }
        moments m;
        memset(&m, 0, sizeof m);
        size_t N = (size_t)P->strip_w[p] * P->strip_h[p];
        for (size_t q = 0; q < N; ++q) {
            if (!c->mask[p][q]) continue;
            uint64_t pv[3], qv[3];
            for (int ch = 0; ch < 3; ++ch) {
                pv[ch] = c->strip[p][1][q * 3 + ch];
                qv[ch] = c->lut[p][ch][pv[ch]];
            }
            m.A[0] += pv[0] * pv[0];
            m.A[1] += pv[0] * pv[1];
            m.A[2] += pv[0] * pv[2];
            m.A[3] += pv[1] * pv[1];
            m.A[4] += pv[1] * pv[2];
            m.A[5] += pv[2] * pv[2];
            for (int r = 0; r < 3; ++r)
                for (int k = 0; k < 3; ++k) m.B[r * 3 + k] += pv[r] * qv[k];
            m.n += 1;
        }
        c->mom[p] = m;
    }
}

/* Eq. (4) across a chain of cameras: pair k - 1 joins cameras (k - 1, k) and
 * its matrix takes camera k's colours (row vectors) to camera k - 1's, so
 * camera k reaches camera 0 through M_k = M_(k-1,k) M_(k-1), M_0 = I (FP64). */
void vso_chain_colour(const double* Mpair, int n_cams, double* Mk)
{
    double acc[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    memcpy(Mk, acc, sizeof acc);
    for (int k = 1; k < n_cams; ++k) {
        mat3_mul(Mpair + (size_t)(k - 1) * 9, acc, acc);
        memcpy(Mk + (size_t)k * 9, acc, sizeof acc);
    }
}

/* Eqs. (2)-(3) (3D-M): the stacked rows of frames T, T-1, T-2 enter the
 * normal equations as summed moments (frames before 0 do not exist), then
 * eq. (4)'s matrix per pair; cameras are chained to camera 0 as
 * M_0 = I, M_k = M_(k-1,k) M_(k-1) (row vectors: camera k -> k-1 -> ... -> 0). */
static void step_solve(vso_ctx* c)
{
    const vso_plan_info* P = &c->plan;
    int W = c->prm.color_window;
    for (int p = 0; p < P->n_pairs; ++p) {
        c->flags[p] = 0;
        double M[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        if (W > 0) {
            uint64_t A3[6], B3[9], n3;
            memcpy(A3, c->mom[p].A, sizeof A3);
            memcpy(B3, c->mom[p].B, sizeof B3);
            n3 = c->mom[p].n;
            for (int d = 1; d < W && d <= c->T; ++d) {
                const moments* o = &c->mom_prev[p][d - 1];
                for (int i = 0; i < 6; ++i) A3[i] += o->A[i];
                for (int i = 0; i < 9; ++i) B3[i] += o->B[i];
                n3 += o->n;
            }
            if (n3 < (uint64_t)c->prm.min_pixels) {
                c->flags[p] = 1;
            } else {
                double A[9] = {(double)A3[0], (double)A3[1], (double)A3[2],
                               (double)A3[1], (double)A3[3], (double)A3[4],
                               (double)A3[2], (double)A3[4], (double)A3[5]};
                double B[9];
                for (int i = 0; i < 9; ++i) B[i] = (double)B3[i];
                if (vso_solve_color(A, B, c->prm.ridge, M)) c->flags[p] = 2;
            }
        }
        memcpy(c->Mpair[p], M, sizeof M);
    }
    double Mk[VSO_MAX_CAMS][9];
    vso_chain_colour(&c->Mpair[0][0], P->n_cams, &Mk[0][0]);
    for (int k = 0; k < P->n_cams; ++k)
        for (int i = 0; i < 9; ++i) c->Mk[k][i] = (float)Mk[k][i];
    /* eq. (4)'s text read literally: no whole-frame (composed) correction;
     * each pair's own matrix applies to camera i inside that overlap */
    for (int p = 0; p < P->n_pairs; ++p)
        for (int i = 0; i < 9; ++i) c->Mpf[p][i] = (float)c->Mpair[p][i];
    if (c->prm.readings & VSO_READ_OVERLAP_ONLY)
        for (int k = 0; k < P->n_cams; ++k)
            for (int i = 0; i < 9; ++i) c->Mk[k][i] = (i % 4 == 0) ? 1.0f : 0.0f;
}

/* ------------------------------------------------------------------------ */
/* Section 3.2: dense flow on the overlap strips                             */
/* ------------------------------------------------------------------------ */

/* One 2x reduction of the Gaussian pyramid: separable [1 4 6 4 1]/16,
 * horizontal pass first, clamped indices, kept at even positions.  Each pass
 * sums ((((a0 + 4 a1) + 6 a2) + 4 a3) + a4) and scales by 1/16. */
void vso_pyr_down(const float* src, int w, int h, float* dst)
{
    int wd = (w + 1) / 2, hd = (h + 1) / 2;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < hd; ++y) {
        for (int x = 0; x < wd; ++x) {
            float rows[5];
            for (int t = 0; t < 5; ++t) {
                const float* s = src + (size_t)clampi(2 * y + t - 2, 0, h - 1) * w;
                float a0 = s[clampi(2 * x - 2, 0, w - 1)];
                float a1 = s[clampi(2 * x - 1, 0, w - 1)];
                float a2 = s[clampi(2 * x, 0, w - 1)];
                float a3 = s[clampi(2 * x + 1, 0, w - 1)];
                float a4 = s[clampi(2 * x + 2, 0, w - 1)];
                float acc = a0 + 4.0f * a1;
                acc = acc + 6.0f * a2;
                acc = acc + 4.0f * a3;
                acc = acc + a4;
                rows[t] = acc * 0.0625f;
            }
            float acc = rows[0] + 4.0f * rows[1];
            acc = acc + 6.0f * rows[2];
            acc = acc + 4.0f * rows[3];
            acc = acc + rows[4];
            dst[(size_t)y * wd + x] = acc * 0.0625f;
        }
    }
}

static float img_at(const float* I, int w, int h, int x, int y)
{
    return I[(size_t)clampi(y, 0, h - 1) * w + clampi(x, 0, w - 1)];
}

/* Dense pyramidal Lucas-Kanade at one level (the flow estimator reading),
 * evaluated at the pixels marked in `need` (all pixels when need is NULL;
 * the others get flow 0):
 * for every pixel x, with template T and moving image Mv, minimise
 * sum_{x' in window} (Mv(x' + u) - T(x'))^2 over the (2r+1)^2 window clipped
 * to the level, by `iters` Gauss-Newton steps with the template gradient
 * (central differences, clamped) and a Tikhonov term lambda * |window|:
 *   G = sum [Ix^2, Ix Iy; Ix Iy, Iy^2] + lambda |window| I,
 *   b = sum [Ix e, Iy e], e = bilinear(Mv, x' + u) - T(x'),
 *   du = (G01 bv - G11 bu) / det, dv = (G01 bu - G00 bv) / det.
 * The warp position x' + u is split once per step into floor(u) = (ox, oy)
 * and frac(u) = (fx, fy) so that every tap is the exact bilinear
 * interpolation at x' + u (indices clamped): with ht, hb the moving image
 * interpolated along x on rows y' + oy and y' + oy + 1, the sample is
 * ht + fy (hb - ht).  b is evaluated with the sums regrouped (the same sum,
 * another FP32 rounding order; vso_lk_level_f64 below keeps the plain form):
 *   bu = (SA + fy (SB - SA)) - C, SA = sum Ix ht, SB = sum Ix hb,
 *   C = sum Ix T (once per level), and bv alike with Iy,
 * so the interpolation along y happens once per window instead of per tap.
 * Sums run over the window in row-major order.  The initial flow is 0 at
 * the coarsest level, else twice the bilinear sample of the coarser flow at
 * ((x + 1/2)/2 - 1/2, (y + 1/2)/2 - 1/2). */
void vso_lk_level(const float* T, const float* Mv, int w, int h,
                  const float* uc, int wc, int hc,
                  int r, int iters, float lambda, const uint8_t* need, float* u_out)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int y = 0; y < h; ++y) {
        for (int x = 0; x < w; ++x) {
            if (need && !need[(size_t)y * w + x]) {
                u_out[((size_t)y * w + x) * 2 + 0] = 0.0f;
                u_out[((size_t)y * w + x) * 2 + 1] = 0.0f;
                continue;
            }
            float ux = 0.0f, uy = 0.0f;
            if (uc) {
                float cx = clampf(fmaf((float)x, 0.5f, -0.25f), 0.0f, (float)(wc - 1));
                float cy = clampf(fmaf((float)y, 0.5f, -0.25f), 0.0f, (float)(hc - 1));
                float flx = floorf(cx), fly = floorf(cy);
                int x0 = (int)flx, y0 = (int)fly;
                float fx = cx - flx, fy = cy - fly;
                int x1 = x0 + 1 < wc ? x0 + 1 : wc - 1;
                int y1 = y0 + 1 < hc ? y0 + 1 : hc - 1;
                float comp[2];
                for (int d = 0; d < 2; ++d) {
                    float p00 = uc[((size_t)y0 * wc + x0) * 2 + d];
                    float p10 = uc[((size_t)y0 * wc + x1) * 2 + d];
                    float p01 = uc[((size_t)y1 * wc + x0) * 2 + d];
                    float p11 = uc[((size_t)y1 * wc + x1) * 2 + d];
                    float a = fmaf(fx, p10 - p00, p00);
                    float b = fmaf(fx, p11 - p01, p01);
                    comp[d] = fmaf(fy, b - a, a);
                }
                ux = 2.0f * comp[0];
                uy = 2.0f * comp[1];
            }
            int wx0 = x - r < 0 ? 0 : x - r, wx1 = x + r > w - 1 ? w - 1 : x + r;
            int wy0 = y - r < 0 ? 0 : y - r, wy1 = y + r > h - 1 ? h - 1 : y + r;
            float g00 = 0.0f, g01 = 0.0f, g11 = 0.0f, cu = 0.0f, cv = 0.0f;
            for (int yy = wy0; yy <= wy1; ++yy)
                for (int xx = wx0; xx <= wx1; ++xx) {
                    float ix = 0.5f * (img_at(T, w, h, xx + 1, yy) - img_at(T, w, h, xx - 1, yy));
                    float iy = 0.5f * (img_at(T, w, h, xx, yy + 1) - img_at(T, w, h, xx, yy - 1));
                    float t = T[(size_t)yy * w + xx];
                    g00 = fmaf(ix, ix, g00);
                    g01 = fmaf(ix, iy, g01);
                    g11 = fmaf(iy, iy, g11);
                    cu = fmaf(ix, t, cu);
                    cv = fmaf(iy, t, cv);
                }
            float reg = lambda * (float)((wy1 - wy0 + 1) * (wx1 - wx0 + 1));
            g00 = g00 + reg;
            g11 = g11 + reg;
            float det = g00 * g11 - g01 * g01;
            for (int it = 0; it < iters; ++it) {
                float flx = floorf(ux), fly = floorf(uy);
                int ox = (int)flx, oy = (int)fly;
                float fx = ux - flx, fy = uy - fly;
                float sau = 0.0f, sav = 0.0f, sbu = 0.0f, sbv = 0.0f;
                for (int yy = wy0; yy <= wy1; ++yy)
                    for (int xx = wx0; xx <= wx1; ++xx) {
                        float p00 = img_at(Mv, w, h, xx + ox, yy + oy);
                        float p10 = img_at(Mv, w, h, xx + ox + 1, yy + oy);
                        float p01 = img_at(Mv, w, h, xx + ox, yy + oy + 1);
                        float p11 = img_at(Mv, w, h, xx + ox + 1, yy + oy + 1);
                        float ht = fmaf(fx, p10 - p00, p00);
                        float hb = fmaf(fx, p11 - p01, p01);
                        float ix = 0.5f * (img_at(T, w, h, xx + 1, yy) - img_at(T, w, h, xx - 1, yy));
                        float iy = 0.5f * (img_at(T, w, h, xx, yy + 1) - img_at(T, w, h, xx, yy - 1));
                        sau = fmaf(ix, ht, sau);
                        sav = fmaf(iy, ht, sav);
                        sbu = fmaf(ix, hb, sbu);
                        sbv = fmaf(iy, hb, sbv);
                    }
                float bu = fmaf(fy, sbu - sau, sau) - cu;
                float bv = fmaf(fy, sbv - sav, sav) - cv;
                float du = (g01 * bv - g11 * bu) / det;
                float dv = (g01 * bu - g00 * bv) / det;
                ux = ux + du;
                uy = uy + dv;
            }
            u_out[((size_t)y * w + x) * 2 + 0] = ux;
            u_out[((size_t)y * w + x) * 2 + 1] = uy;
        }
    }
}

/* The same estimator in FP64 (no prescribed rounding), used only to bound how
 * far FP32 rounding moves the flow. */
static double img_at_d(const double* I, int w, int h, int x, int y)
{
    return I[(size_t)clampi(y, 0, h - 1) * w + clampi(x, 0, w - 1)];
}

void vso_lk_level_f64(const double* T, const double* Mv, int w, int h,
                      const double* uc, int wc, int hc,
                      int r, int iters, double lambda, double* u_out)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int y = 0; y < h; ++y) {
        for (int x = 0; x < w; ++x) {
            double ux = 0.0, uy = 0.0;
            if (uc) {
                double cx = x * 0.5 - 0.25, cy = y * 0.5 - 0.25;
                cx = cx < 0 ? 0 : (cx > wc - 1 ? wc - 1 : cx);
                cy = cy < 0 ? 0 : (cy > hc - 1 ? hc - 1 : cy);
                int x0 = (int)floor(cx), y0 = (int)floor(cy);
                double fx = cx - x0, fy = cy - y0;
                int x1 = x0 + 1 < wc ? x0 + 1 : wc - 1;
                int y1 = y0 + 1 < hc ? y0 + 1 : hc - 1;
                double comp[2];
                for (int d = 0; d < 2; ++d) {
                    double p00 = uc[((size_t)y0 * wc + x0) * 2 + d];
                    double p10 = uc[((size_t)y0 * wc + x1) * 2 + d];
                    double p01 = uc[((size_t)y1 * wc + x0) * 2 + d];
                    double p11 = uc[((size_t)y1 * wc + x1) * 2 + d];
                    double a = p00 + fx * (p10 - p00), b = p01 + fx * (p11 - p01);
                    comp[d] = a + fy * (b - a);
                }
                ux = 2.0 * comp[0];
                uy = 2.0 * comp[1];
            }
            int wx0 = x - r < 0 ? 0 : x - r, wx1 = x + r > w - 1 ? w - 1 : x + r;
            int wy0 = y - r < 0 ? 0 : y - r, wy1 = y + r > h - 1 ? h - 1 : y + r;
            double g00 = 0, g01 = 0, g11 = 0;
            for (int yy = wy0; yy <= wy1; ++yy)
                for (int xx = wx0; xx <= wx1; ++xx) {
                    double ix = 0.5 * (img_at_d(T, w, h, xx + 1, yy) - img_at_d(T, w, h, xx - 1, yy));
                    double iy = 0.5 * (img_at_d(T, w, h, xx, yy + 1) - img_at_d(T, w, h, xx, yy - 1));
                    g00 += ix * ix;
                    g01 += ix * iy;
                    g11 += iy * iy;
                }
            double reg = lambda * (double)((wy1 - wy0 + 1) * (wx1 - wx0 + 1));
            g00 += reg;
            g11 += reg;
            double det = g00 * g11 - g01 * g01;
            for (int it = 0; it < iters; ++it) {
                double flx = floor(ux), fly = floor(uy);
                int ox = (int)flx, oy = (int)fly;
                double fx = ux - flx, fy = uy - fly;
                double bu = 0, bv = 0;
                for (int yy = wy0; yy <= wy1; ++yy)
                    for (int xx = wx0; xx <= wx1; ++xx) {
                        double p00 = img_at_d(Mv, w, h, xx + ox, yy + oy);
                        double p10 = img_at_d(Mv, w, h, xx + ox + 1, yy + oy);
                        double p01 = img_at_d(Mv, w, h, xx + ox, yy + oy + 1);
                        double p11 = img_at_d(Mv, w, h, xx + ox + 1, yy + oy + 1);
                        double a = p00 + fx * (p10 - p00), b = p01 + fx * (p11 - p01);
                        double e = a + fy * (b - a) - T[(size_t)yy * w + xx];
                        double ix = 0.5 * (img_at_d(T, w, h, xx + 1, yy) - img_at_d(T, w, h, xx - 1, yy));
                        double iy = 0.5 * (img_at_d(T, w, h, xx, yy + 1) - img_at_d(T, w, h, xx, yy - 1));
                        bu += ix * e;
                        bv += iy * e;
                    }
                ux += (g01 * bv - g11 * bu) / det;
                uy += (g01 * bu - g00 * bv) / det;
            }
            u_out[((size_t)y * w + x) * 2 + 0] = ux;
            u_out[((size_t)y * w + x) * 2 + 1] = uy;
        }
    }
}

/* Integer luma of an RGB byte triple with the BT.601 weights 0.299, 0.587,
 * 0.114 in 8-bit fixed point (77, 150, 29 over 256), rounded half up. */
int vso_luma(int r, int g, int b) { return (77 * r + 150 * g + 29 * b + 128) >> 8; }

/* Flow input: the colour-corrected strips (every strip pixel), reduced to
 * integer luma Y = (77 R + 150 G + 29 B + 128) >> 8, then the pyramid. */
static void step_pyramids(vso_ctx* c)
{
    const vso_plan_info* P = &c->plan;
    for (int p = 0; p < P->n_pairs; ++p) {
        int sw = P->strip_w[p], sh = P->strip_h[p];
        int cams[2] = {P->pair_j[p], P->pair_i[p]};
        for (int s = 0; s < 2; ++s) {
            const float* M = c->Mk[cams[s]];
            const int ovl = (c->prm.readings & VSO_READ_OVERLAP_ONLY) && s == 1;
            float* Y = c->pyr[p][s][0];
#pragma omp parallel for schedule(static)
            for (int q = 0; q < sw * sh; ++q) {
                float px[3];
                int cc[3];
                const float* Mq = (ovl && c->mask[p][q]) ? c->Mpf[p] : M;
                for (int ch = 0; ch < 3; ++ch) px[ch] = (float)c->strip[p][s][(size_t)q * 3 + ch];
                for (int ch = 0; ch < 3; ++ch) cc[ch] = vso_round8(color_apply(px, Mq, ch));
                Y[q] = (float)vso_luma(cc[0], cc[1], cc[2]);
            }
            for (int l = 1; l < c->prm.lk_levels; ++l)
                vso_pyr_down(c->pyr[p][s][l - 1], c->pw[p][l - 1], c->ph[p][l - 1], c->pyr[p][s][l]);
        }
    }
}

/* Where the flow is estimated (section 3.2 computes it between the overlap
 * regions): at level 0 the overlap pixels of the strip (the mask); at a
 * coarser level the pixels that the finer level's initialisation samples
 * (the two-by-two bilinear footprint of every needed finer pixel). */
static void build_need(vso_ctx* c, int p)
{
    size_t n0 = (size_t)c->pw[p][0] * c->ph[p][0];
    memcpy(c->need[p][0], c->mask[p], n0);
    for (int l = 0; l + 1 < c->prm.lk_levels; ++l) {
        int w = c->pw[p][l], h = c->ph[p][l], wc = c->pw[p][l + 1], hc = c->ph[p][l + 1];
        uint8_t* dst = c->need[p][l + 1];
        memset(dst, 0, (size_t)wc * hc);
        for (int y = 0; y < h; ++y)
            for (int x = 0; x < w; ++x) {
                if (!c->need[p][l][(size_t)y * w + x]) continue;
                float cx = clampf(fmaf((float)x, 0.5f, -0.25f), 0.0f, (float)(wc - 1));
                float cy = clampf(fmaf((float)y, 0.5f, -0.25f), 0.0f, (float)(hc - 1));
                int x0 = (int)floorf(cx), y0 = (int)floorf(cy);
                int x1 = x0 + 1 < wc ? x0 + 1 : wc - 1;
                int y1 = y0 + 1 < hc ? y0 + 1 : hc - 1;
                dst[(size_t)y0 * wc + x0] = 1;
                dst[(size_t)y0 * wc + x1] = 1;
                dst[(size_t)y1 * wc + x0] = 1;
                dst[(size_t)y1 * wc + x1] = 1;
            }
    }
}

/* flow_ij satisfies P_i(x + flow_ij(x)) ~ P_j(x): template j, moving i;
 * flow_ji the other way round.  Coarse to fine. */
static int surrogate_pair(vso_ctx* c, int p);

static void step_flow(vso_ctx* c)
{
    const vso_plan_info* P = &c->plan;
    int L = c->prm.lk_levels;
    for (int p = 0; p < P->n_pairs; ++p) {
        size_t n0 = (size_t)P->strip_w[p] * P->strip_h[p];
        build_need(c, p);
        c->surr_ok[p] = 0;
        if (c->prm.flow && c->surr_mode && surrogate_pair(c, p)) continue;
        for (int dir = 0; dir < 2; ++dir) {
            if (!c->prm.flow) {
                memset(c->flow[p][dir], 0, n0 * 2 * sizeof(float));
                continue;
            }
            int tmpl = dir == 0 ? 0 : 1; /* 0 = camera j, 1 = camera i */
            int mov = 1 - tmpl;
            if (c->prm.flow == 2) {
                const float* Tl[VSO_MAX_LEVELS];
                const float* Ml[VSO_MAX_LEVELS];
                const uint8_t* Nl[VSO_MAX_LEVELS];
                for (int l = 0; l < L; ++l) {
                    Tl[l] = c->pyr[p][tmpl][l];
                    Ml[l] = c->pyr[p][mov][l];
                    Nl[l] = c->need[p][l];
                }
                vso_var_pyramid(Tl, Ml, Nl, c->pw[p], c->ph[p], L, c->prm.var_alpha, c->prm.var_gamma,
                                c->prm.var_outer, c->prm.var_inner, c->flow[p][dir]);
                continue;
            }
            float* prev = NULL;
            int pwc = 0, phc = 0;
            for (int l = L - 1; l >= 0; --l) {
                int w = c->pw[p][l], h = c->ph[p][l];
                float* u = (l == 0) ? c->flow[p][dir] : (float*)malloc((size_t)w * h * 2 * sizeof(float));
                vso_lk_level(c->pyr[p][tmpl][l], c->pyr[p][mov][l], w, h, prev, pwc, phc,
                             c->prm.lk_radius, c->prm.lk_iters, c->prm.lk_lambda, c->need[p][l], u);
                free(prev);
                prev = (l == 0) ? NULL : u;
                pwc = w;
                phc = h;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* The learned flow surrogate inside the frame (not in the paper).            */
/*                                                                            */
/* A chain of 3x3 convolutions maps the level-2 luma pair of a field          */
/* (template, moving) to the field's flow in level-2 pixels.  Network input:  */
/* channel 0 = bf16((Y_t - 128) / 64), channel 1 = bf16((Y_m - 128) / 64),     */
/* other channels 0.  Each layer: its BF16 products (each exact in FP64)     */
/* accumulated with the bias in FP64, rounded once to FP32; hidden layers     */
/* apply a leaky ReLU in FP32 and store BF16 (round to nearest even); the     */
/* last layer stays FP32 and                                                  */
/* its channels 0-1 are the flow.  The level-0 flow is the bilinear          */
/* upsampling x4 (level-0 x maps to level-2 x / 4 - 3 / 8).  A pair keeps     */
/* the surrogate's flows when its forward-backward error                      */
/*   e(x) = | U_ij(x) + U_ji(x + U_ij(x)) |  (U the upsampled fields)          */
/* averaged over the overlap, in 1/256 px fixed point, is below the           */
/* threshold; otherwise the plain estimator runs for that pair.               */
/* ------------------------------------------------------------------------ */

#define SURR_LEVEL 2
#define SURR_MAX_LAYERS 8

static float bf16_round(float v)
{
    uint32_t u;
    memcpy(&u, &v, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    float r;
    memcpy(&r, &u, 4);
    return r;
}

typedef struct {
    int nl;
    float alpha;
    int ci[SURR_MAX_LAYERS], co[SURR_MAX_LAYERS];
    const int16_t* w[SURR_MAX_LAYERS];   /* [co][9][ci] BF16 bits */
    const float* b[SURR_MAX_LAYERS];
} net_view;

/* Weight file: "VSNN", u32 version (1), u32 layers, f32 leaky-ReLU slope,
 * per layer u32 cin, u32 cout, then per layer int16 w[cout][9][cin] (BF16
 * bits) and f32 bias[cout], little endian, packed. */
static int parse_net(const void* blob, size_t n, net_view* v)
{
    const uint8_t* b = (const uint8_t*)blob;
    if (!b || n < 16 || memcmp(b, "VSNN", 4) != 0) return VSO_E_INVAL;
    uint32_t version, nl;
    memcpy(&version, b + 4, 4);
    memcpy(&nl, b + 8, 4);
    memcpy(&v->alpha, b + 12, 4);
    if (version != 1 || nl < 1 || nl > SURR_MAX_LAYERS || !isfinite(v->alpha)) return VSO_E_INVAL;
    v->nl = (int)nl;
    size_t off = 16;
    if (n < off + 8 * (size_t)nl) return VSO_E_INVAL;
    for (int l = 0; l < v->nl; ++l) {
        uint32_t ci, co;
        memcpy(&ci, b + off, 4);
        memcpy(&co, b + off + 4, 4);
        off += 8;
        if (ci < 1 || co < 1 || ci > 256 || co > 256) return VSO_E_INVAL;
        v->ci[l] = (int)ci;
        v->co[l] = (int)co;
    }
    if (v->ci[0] < 2 || v->co[v->nl - 1] < 2) return VSO_E_INVAL;
    for (int l = 1; l < v->nl; ++l)
        if (v->ci[l] != v->co[l - 1]) return VSO_E_INVAL;
    for (int l = 0; l < v->nl; ++l) {
        size_t nw = (size_t)v->co[l] * 9 * v->ci[l];
        if (n < off + 2 * nw + 4 * (size_t)v->co[l]) return VSO_E_INVAL;
        v->w[l] = (const int16_t*)(b + off);
        off += 2 * nw;
        v->b[l] = (const float*)(b + off);
        off += 4 * (size_t)v->co[l];
    }
    return off == n ? VSO_OK : VSO_E_INVAL;
}

static double bf16_bits_to_double(int16_t h)
{
    uint32_t u = (uint32_t)(uint16_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* The network on one luma pair (w x h, FP32); pred receives channels 0-1 of
 * the last layer, [h][w][2]. */
static void net_forward(const net_view* v, const float* Yt, const float* Ym, int w, int h, float* pred)
{
    size_t npx = (size_t)w * h;
    int cmax = v->ci[0];
    for (int l = 0; l < v->nl; ++l) cmax = v->co[l] > cmax ? v->co[l] : cmax;
    double* x = (double*)calloc(npx * cmax, sizeof(double));
    double* y = (double*)calloc(npx * cmax, sizeof(double));
    double* wt = (double*)malloc((size_t)256 * 9 * 256 * sizeof(double));
    int cin = v->ci[0];
    for (size_t q = 0; q < npx; ++q) {
        x[q * cin + 0] = (double)bf16_round((Yt[q] - 128.0f) * (1.0f / 64.0f));
        x[q * cin + 1] = (double)bf16_round((Ym[q] - 128.0f) * (1.0f / 64.0f));
    }
    for (int l = 0; l < v->nl; ++l) {
        int ci = v->ci[l], co = v->co[l];
        for (size_t i = 0; i < (size_t)co * 9 * ci; ++i) wt[i] = bf16_bits_to_double(v->w[l][i]);
        /* the sums of products accumulated in FP64 (each product of two BF16
         * values is exact in FP64; the running sum is rounded to FP64), plus
         * the bias */
        double bias[256];
        for (int o = 0; o < co; ++o) bias[o] = (double)v->b[l][o];
        vso_conv3x3(x, 1, h, w, ci, wt, bias, co, y);
        const int last = l == v->nl - 1;
#pragma omp parallel for schedule(static)
        for (long long q = 0; q < (long long)npx; ++q)
            for (int o = 0; o < co; ++o) {
                float t = (float)y[(size_t)q * co + o];
                if (last) {
                    if (o < 2) pred[(size_t)q * 2 + o] = t;
                } else {
                    t = t > 0.0f ? t : v->alpha * t;
                    y[(size_t)q * co + o] = (double)bf16_round(t);
                }
            }
        double* tmp = x;
        x = y;
        y = tmp;
    }
    free(x);
    free(y);
    free(wt);
}

int vso_surrogate_net(const void* blob, size_t n, const float* yt, const float* ym, int w, int h, float* pred)
{
    net_view v;
    if (parse_net(blob, n, &v) != VSO_OK || w < 1 || h < 1) return VSO_E_INVAL;
    net_forward(&v, yt, ym, w, h, pred);
    return VSO_OK;
}

/* the x4 upsampled level-2 field at level-0 position (X, Y); the clamp
 * takes a non-finite position (a non-finite displacement) to the border */
static void up_sample(const float* pred, int w2, int h2, float X, float Y, float* fx_out, float* fy_out)
{
    float cx = fminf(fmaxf(fmaf(X, 0.25f, -0.375f), 0.0f), (float)(w2 - 1));
    float cy = fminf(fmaxf(fmaf(Y, 0.25f, -0.375f), 0.0f), (float)(h2 - 1));
    float flx = floorf(cx), fly = floorf(cy);
    int xa = (int)flx, ya = (int)fly;
    float fx = cx - flx, fy = cy - fly;
    int xb = xa + 1 < w2 ? xa + 1 : w2 - 1;
    int yb = ya + 1 < h2 ? ya + 1 : h2 - 1;
    const float* p00 = pred + ((size_t)ya * w2 + xa) * 2;
    const float* p10 = pred + ((size_t)ya * w2 + xb) * 2;
    const float* p01 = pred + ((size_t)yb * w2 + xa) * 2;
    const float* p11 = pred + ((size_t)yb * w2 + xb) * 2;
    float r[2];
    for (int k = 0; k < 2; ++k) {
        float a = fmaf(fx, p10[k] - p00[k], p00[k]);
        float b = fmaf(fx, p11[k] - p01[k], p01[k]);
        r[k] = 4.0f * fmaf(fy, b - a, a);
    }
    *fx_out = r[0];
    *fy_out = r[1];
}

void vso_surr_upsample(const float* pred, int w2, int h2, const uint8_t* need0, int w0, int h0, float* flow0)
{
    for (int y = 0; y < h0; ++y)
        for (int x = 0; x < w0; ++x) {
            size_t q = (size_t)y * w0 + x;
            float fx = 0.0f, fy = 0.0f;
            if (!need0 || need0[q]) up_sample(pred, w2, h2, (float)x, (float)y, &fx, &fy);
            flow0[q * 2] = fx;
            flow0[q * 2 + 1] = fy;
        }
}

/* per-pixel error in 1/256 px, saturated at 2^20 (a non-finite error too) */
static unsigned fb_fixed(float ex, float ey)
{
    float e = sqrtf(ex * ex + ey * ey);
    return (unsigned)floorf(fminf(e * 256.0f, 1048576.0f) + 0.5f);
}

void vso_fb_check(const float* pred_ij, const float* pred_ji, int w2, int h2, const uint8_t* need0, int w0, int h0,
                  unsigned long long* sum, unsigned long long* count)
{
    unsigned long long s = 0, n = 0;
    for (int y = 0; y < h0; ++y)
        for (int x = 0; x < w0; ++x) {
            if (need0 && !need0[(size_t)y * w0 + x]) continue;
            float ux, uy, vx, vy;
            up_sample(pred_ij, w2, h2, (float)x, (float)y, &ux, &uy);
            up_sample(pred_ji, w2, h2, (float)x + ux, (float)y + uy, &vx, &vy);
            s += fb_fixed(ux + vx, uy + vy);
            n += 1;
        }
    *sum = s;
    *count = n;
}

int vso_set_surrogate(vso_ctx* c, const void* blob, size_t n, int mode, float tau)
{
    if (!c || mode < 0 || mode > 2 || !(tau >= 0.0f) || tau > 1e6f) return VSO_E_INVAL;
    if (blob) {
        net_view v;
        if (parse_net(blob, n, &v) != VSO_OK) return VSO_E_INVAL;
        void* cp = malloc(n);
        if (!cp) return VSO_E_NOMEM;
        memcpy(cp, blob, n);
        free(c->surr_blob);
        c->surr_blob = cp;
        c->surr_blob_n = n;
    }
    if (mode != 0 && (!c->surr_blob || c->prm.lk_levels <= SURR_LEVEL)) return VSO_E_INVAL;
    c->surr_mode = mode;
    c->surr_tau_fix = (unsigned long long)llround((double)tau * 256.0);
    return VSO_OK;
}

/* Surrogate flows of pair p in both directions (template j / moving i and the
 * reverse, as in step_flow); returns 1 when the pair keeps them. */
static int surrogate_pair(vso_ctx* c, int p)
{
    net_view v;
    parse_net(c->surr_blob, c->surr_blob_n, &v);
    const int w2 = c->pw[p][SURR_LEVEL], h2 = c->ph[p][SURR_LEVEL];
    const int w0 = c->pw[p][0], h0 = c->ph[p][0];
    for (int dir = 0; dir < 2; ++dir) {
        free(c->surr_pred[p][dir]);
        c->surr_pred[p][dir] = (float*)malloc((size_t)w2 * h2 * 2 * sizeof(float));
        int tmpl = dir == 0 ? 0 : 1, mov = 1 - tmpl;
        net_forward(&v, c->pyr[p][tmpl][SURR_LEVEL], c->pyr[p][mov][SURR_LEVEL], w2, h2, c->surr_pred[p][dir]);
    }
    vso_fb_check(c->surr_pred[p][0], c->surr_pred[p][1], w2, h2, c->need[p][0], w0, h0, &c->fb[p][0], &c->fb[p][1]);
    int ok = c->surr_mode == 1 || (c->fb[p][1] > 0 && c->fb[p][0] < c->surr_tau_fix * c->fb[p][1]);
    c->surr_ok[p] = ok;
    if (ok) {
        vso_surr_upsample(c->surr_pred[p][0], w2, h2, c->need[p][0], w0, h0, c->flow[p][0]);
        vso_surr_upsample(c->surr_pred[p][1], w2, h2, c->need[p][0], w0, h0, c->flow[p][1]);
    }
    return ok;
}

/* ------------------------------------------------------------------------ */
/* Eqs. (15)-(18): local warp and weighted fusion                            */
/* ------------------------------------------------------------------------ */

static void sample_view(const vso_view* v, float X, float Y, float t[3])
{
    float u, w;
    vso_hom_valid(v->hinv, X, Y, v->W, v->H, &u, &w);
    float s[3];
    for (int ch = 0; ch < 3; ++ch) s[ch] = vso_bilinear(v->frame, v->pitch, v->W, v->H, ch, u, w);
    for (int ch = 0; ch < 3; ++ch) t[ch] = color_apply(s, v->M, ch);
}

/* One canvas pixel covered by one camera: its colour-corrected resample. */
static void single_pixel(const vso_view* v, float y, uint8_t out[3])
{
    float t[3];
    sample_view(v, v->X, y, t);
    for (int ch = 0; ch < 3; ++ch) out[ch] = (uint8_t)vso_round8(t[ch]);
}

/* One canvas pixel covered by two cameras, j (left) and i (right):
 *  eq. (16): the weights come from the pixel's distance to each camera's own
 *    vertical border, measured in that camera's unwarped coordinates,
 *    d_k = max(0, min(u_k, W_k - 1 - u_k)); theta_i = d_i / (d_i + d_j)
 *    (1/2 when both are 0) and theta_j = 1 - theta_i, so camera i's weight
 *    rises from 0 at its own border;
 *  eq. (17): the local warp meets in the middle -- camera i is sampled at
 *    x + theta_j flow_ij(x), camera j at x + theta_i flow_ji(x);
 *  eq. (18): out = round8(theta_i (t_i - t_j) + t_j), t the colour-corrected
 *    samples of the two camera frames at those points. */
void vso_fuse_pixel(const vso_view* vj, const vso_view* vi, float y, const float f_ij[2], const float f_ji[2],
                    uint8_t out[3])
{
    float uj, vjv, ui, viv;
    vso_hom_valid(vj->hinv, vj->X, y, vj->W, vj->H, &uj, &vjv);
    vso_hom_valid(vi->hinv, vi->X, y, vi->W, vi->H, &ui, &viv);
    float dj = fminf(uj, (float)(vj->W - 1) - uj);
    float di = fminf(ui, (float)(vi->W - 1) - ui);
    if (dj < 0.0f) dj = 0.0f;
    if (di < 0.0f) di = 0.0f;
    float sum = di + dj;
    float th_i = sum > 0.0f ? di / sum : 0.5f;
    float th_j = 1.0f - th_i;
    float Xi = fmaf(th_j, f_ij[0], vi->X);
    float Yi = fmaf(th_j, f_ij[1], y);
    float Xj = fmaf(th_i, f_ji[0], vj->X);
    float Yj = fmaf(th_i, f_ji[1], y);
    float ti[3], tj[3];
    sample_view(vi, Xi, Yi, ti);
    sample_view(vj, Xj, Yj, tj);
    for (int ch = 0; ch < 3; ++ch) out[ch] = (uint8_t)vso_round8(fmaf(th_i, ti[ch] - tj[ch], tj[ch]));
}

/* Eq. (17) as printed: camera i at x + theta_i flow_ij(x), camera j at
 * x + theta_j flow_ji(x); eqs. (16) and (18) as in vso_fuse_pixel. */
void vso_fuse_pixel_literal(const vso_view* vj, const vso_view* vi, float y, const float f_ij[2],
                            const float f_ji[2], uint8_t out[3])
{
    float uj, vjv, ui, viv;
    vso_hom_valid(vj->hinv, vj->X, y, vj->W, vj->H, &uj, &vjv);
    vso_hom_valid(vi->hinv, vi->X, y, vi->W, vi->H, &ui, &viv);
    float dj = fminf(uj, (float)(vj->W - 1) - uj);
    float di = fminf(ui, (float)(vi->W - 1) - ui);
    if (dj < 0.0f) dj = 0.0f;
    if (di < 0.0f) di = 0.0f;
    float sum = di + dj;
    float th_i = sum > 0.0f ? di / sum : 0.5f;
    float th_j = 1.0f - th_i;
    float Xi = fmaf(th_i, f_ij[0], vi->X);
    float Yi = fmaf(th_i, f_ij[1], y);
    float Xj = fmaf(th_j, f_ji[0], vj->X);
    float Yj = fmaf(th_j, f_ji[1], y);
    float ti[3], tj[3];
    sample_view(vi, Xi, Yi, ti);
    sample_view(vj, Xj, Yj, tj);
    for (int ch = 0; ch < 3; ++ch) out[ch] = (uint8_t)vso_round8(fmaf(th_i, ti[ch] - tj[ch], tj[ch]));
}

static void make_view(const vso_ctx* c, const uint8_t* const F[], const int pitch[], const hit* h, int x,
                      vso_view* v)
{
    const int k = h->cam;
    v->frame = F[k];
    v->pitch = pitch[k];
    v->W = c->rig.cam_w[k];
    v->H = c->rig.cam_h[k];
    v->hinv = c->plan.hinv[k];
    v->M = c->Mk[k];
    v->X = (float)(x + h->m * c->plan.ring_period);
}

/* Per canvas pixel: uncovered -> 0; one camera -> its colour-corrected
 * resample; two cameras -> the fusion of eqs. (16)-(18) with the pair's
 * flows at the pixel. */
static void step_blend(vso_ctx* c, const uint8_t* const F[], const int pitch[])
{
    const vso_plan_info* P = &c->plan;
    int W = P->canvas_w, H = P->canvas_h;
#pragma omp parallel for schedule(dynamic, 4)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            uint8_t* o = c->pano_pre + ((size_t)y * W + x) * 3;
            hit h[4];
            int n = cover_pixel(c, x, y, h);
            if (n == 0) {
                o[0] = o[1] = o[2] = 0;
            } else if (n == 1) {
                vso_view v;
                make_view(c, F, pitch, &h[0], x, &v);
                single_pixel(&v, (float)y, o);
            } else {
                int jidx;
                int p = pair_for(P, &h[0], &h[1], &jidx);
                vso_view vj, vi;
                make_view(c, F, pitch, &h[jidx], x, &vj);
                make_view(c, F, pitch, &h[1 - jidx], x, &vi);
                if (c->prm.readings & VSO_READ_OVERLAP_ONLY) vi.M = c->Mpf[p];
                int X = x + h[jidx].m * P->ring_period;
                int lx = X - P->strip_x0[p], ly = y - P->strip_y0[p];
                size_t q = ((size_t)ly * P->strip_w[p] + lx) * 2;
                if (c->prm.readings & VSO_READ_LITERAL_EQ17)
                    vso_fuse_pixel_literal(&vj, &vi, (float)y, c->flow[p][0] + q, c->flow[p][1] + q, o);
                else
                    vso_fuse_pixel(&vj, &vi, (float)y, c->flow[p][0] + q, c->flow[p][1] + q, o);
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Section 2.2, eqs. (5)-(7): online colour balancing                        */
/* ------------------------------------------------------------------------ */

/* m1 = smallest level whose cumulative count reaches lambda of the n pixels,
 * m2 the same for 1 - lambda (integer comparisons, lambda in percent). */
void vso_quantiles(const uint32_t hist[256], long long n, int lambda_pct, int* q1, int* q2)
{
    long long C = 0;
    *q1 = -1;
    *q2 = -1;
    for (int v = 0; v < 256; ++v) {
        C += hist[v];
        if (*q1 < 0 && 100LL * C >= (long long)lambda_pct * n) *q1 = v;
        if (*q2 < 0 && 100LL * C >= (long long)(100 - lambda_pct) * n) *q2 = v;
    }
    if (*q1 < 0) *q1 = 0;
    if (*q2 < 0) *q2 = 255;
}

/* Eq. (5) piecewise F per channel (reading of the missing figure): the
 * thresholds go to where an equalised histogram puts its lambda and
 * 1 - lambda quantiles, t1 = 255 lambda and t2 = 255 (1 - lambda); linear
 * on [m1, m2], gamma curves a + T (x / T)^b on [0, m1] and [m2, 255] whose
 * exponents make F continuously differentiable at m1 and m2 (clamped to
 * [1/8, 8]).  Identity if m2 - m1 < 1.  FP64, rounded half up. */
void vso_balance_lut(double m1, double m2, int lambda_pct, uint8_t lut[256])
{
    double lam = (double)lambda_pct / 100.0;
    double t1 = 255.0 * lam, t2 = 255.0 * (1.0 - lam);
    if (m2 - m1 < 1.0) {
        for (int v = 0; v < 256; ++v) lut[v] = (uint8_t)v;
        return;
    }
    double s = (t2 - t1) / (m2 - m1);
    double g1 = s * m1 / t1, g2 = s * (255.0 - m2) / (255.0 - t2);
    if (g1 < 0.125) g1 = 0.125;
    if (g1 > 8.0) g1 = 8.0;
    if (g2 < 0.125) g2 = 0.125;
    if (g2 > 8.0) g2 = 8.0;
    for (int v = 0; v < 256; ++v) {
        double x = (double)v, F;
        if (x < m1) F = t1 * pow(x / m1, g1);
        else if (x <= m2) F = t1 + s * (x - m1);
        else F = 255.0 - (255.0 - t2) * pow((255.0 - x) / (255.0 - m2), g2);
        double f = floor(F + 0.5);
        if (f < 0) f = 0;
        if (f > 255) f = 255;
        lut[v] = (uint8_t)f;
    }
}

static void step_balance(vso_ctx* c, uint8_t* pano)
{
    const vso_plan_info* P = &c->plan;
    size_t N = (size_t)P->canvas_w * P->canvas_h;
    memset(c->pano_hist, 0, sizeof c->pano_hist);
    long long n = 0;
    for (size_t q = 0; q < N; ++q) {
        if (!c->cover[q]) continue;
        ++n;
        for (int ch = 0; ch < 3; ++ch) c->pano_hist[ch][c->pano_pre[q * 3 + ch]]++;
    }
    for (int ch = 0; ch < 3; ++ch) {
        int q1, q2;
        vso_quantiles(c->pano_hist[ch], n, c->prm.lambda_pct, &q1, &q2);
        c->quant[ch][0] = q1;
        c->quant[ch][1] = q2;
        /* eqs. (6)-(7): mean over the current frame and up to two earlier ones */
        int s1 = q1, s2 = q2, cnt = 1;
        for (int d = 1; d <= 2 && d <= c->T; ++d) {
            s1 += c->q_prev[d - 1][ch][0];
            s2 += c->q_prev[d - 1][ch][1];
            ++cnt;
        }
        c->mbar[ch][0] = (double)s1 / (double)cnt;
        c->mbar[ch][1] = (double)s2 / (double)cnt;
        vso_balance_lut(c->mbar[ch][0], c->mbar[ch][1], c->prm.lambda_pct, c->bal_lut[ch]);
    }
    for (size_t q = 0; q < N; ++q) {
        for (int ch = 0; ch < 3; ++ch) {
            uint8_t v = c->pano_pre[q * 3 + ch];
            pano[q * 3 + ch] = (c->prm.balance && c->cover[q]) ? c->bal_lut[ch][v] : v;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* One frame                                                                 */
/* ------------------------------------------------------------------------ */

static double wall_seconds(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

int vso_stitch(vso_ctx* c, const uint8_t* const frames[], const int pitch[], uint8_t* pano)
{
    if (!c || !frames || !pitch || !pano) return VSO_E_INVAL;
    for (int k = 0; k < c->plan.n_cams; ++k)
        if (!frames[k] || pitch[k] < 3 * c->rig.cam_w[k]) return VSO_E_INVAL;
    double t[8];
    t[0] = wall_seconds();
    step_strips(c, frames, pitch);
    t[1] = wall_seconds();
    step_moments(c);
    t[2] = wall_seconds();
    step_solve(c);
    t[3] = wall_seconds();
    step_pyramids(c);
    t[4] = wall_seconds();
    step_flow(c);
    t[5] = wall_seconds();
    step_blend(c, frames, pitch);
    t[6] = wall_seconds();
    step_balance(c, pano);
    t[7] = wall_seconds();
    for (int i = 0; i < 7; ++i) c->step_s[i] += t[i + 1] - t[i];
    /* state: shift the per-pair moments and the quantiles, T += 1 */
    for (int p = 0; p < c->plan.n_pairs; ++p) {
        c->mom_prev[p][1] = c->mom_prev[p][0];
        c->mom_prev[p][0] = c->mom[p];
    }
    memcpy(c->q_prev[1], c->q_prev[0], sizeof c->q_prev[0]);
    for (int ch = 0; ch < 3; ++ch) {
        c->q_prev[0][ch][0] = c->quant[ch][0];
        c->q_prev[0][ch][1] = c->quant[ch][1];
    }
    c->T += 1;
    return VSO_OK;
}

/* ------------------------------------------------------------------------ */
/* Taps                                                                      */
/* ------------------------------------------------------------------------ */

static int copy_out(void* dst, size_t nbytes, const void* src, size_t have)
{
    if (nbytes != have) return VSO_E_INVAL;
    memcpy(dst, src, have);
    return VSO_OK;
}

int vso_get(const vso_ctx* c, int tap, int p, int sub, void* dst, size_t nbytes)
{
    const vso_plan_info* P = &c->plan;
    int pair_ok = p >= 0 && p < P->n_pairs;
    size_t n = pair_ok ? (size_t)P->strip_w[p] * P->strip_h[p] : 0;
    switch (tap) {
    case VSO_TAP_STRIP:
        if (!pair_ok || sub < 0 || sub > 1) return VSO_E_INVAL;
        return copy_out(dst, nbytes, c->strip[p][sub], n * 3);
    case VSO_TAP_MASK:
        if (!pair_ok) return VSO_E_INVAL;
        return copy_out(dst, nbytes, c->mask[p], n);
    case VSO_TAP_HIST:
        if (!pair_ok) return VSO_E_INVAL;
        return copy_out(dst, nbytes, c->hist[p], sizeof c->hist[p]);
    case VSO_TAP_LUT:
        if (!pair_ok) return VSO_E_INVAL;
        return copy_out(dst, nbytes, c->lut[p], sizeof c->lut[p]);
    case VSO_TAP_MOM: {
        if (!pair_ok) return VSO_E_INVAL;
        uint64_t m[16];
        memcpy(m, c->mom[p].A, 6 * 8);
        memcpy(m + 6, c->mom[p].B, 9 * 8);
        m[15] = c->mom[p].n;
        return copy_out(dst, nbytes, m, sizeof m);
    }
    case VSO_TAP_MPAIR:
        return copy_out(dst, nbytes, c->Mpair, (size_t)P->n_pairs * 9 * sizeof(double));
    case VSO_TAP_MK:
        return copy_out(dst, nbytes, c->Mk, (size_t)P->n_cams * 9 * sizeof(float));
    case VSO_TAP_FLAGS:
        return copy_out(dst, nbytes, c->flags, (size_t)P->n_pairs * sizeof(int));
    case VSO_TAP_PYR: {
        int cam = sub / 8, l = sub % 8;
        if (!pair_ok || cam < 0 || cam > 1 || l >= c->prm.lk_levels) return VSO_E_INVAL;
        return copy_out(dst, nbytes, c->pyr[p][cam][l], (size_t)c->pw[p][l] * c->ph[p][l] * sizeof(float));
    }
    case VSO_TAP_FLOW:
        if (!pair_ok || sub < 0 || sub > 1) return VSO_E_INVAL;
        return copy_out(dst, nbytes, c->flow[p][sub], n * 2 * sizeof(float));
    case VSO_TAP_PANO_PRE:
        return copy_out(dst, nbytes, c->pano_pre, (size_t)P->canvas_w * P->canvas_h * 3);
    case VSO_TAP_PANO_HIST:
        return copy_out(dst, nbytes, c->pano_hist, sizeof c->pano_hist);
    case VSO_TAP_BAL_LUT:
        return copy_out(dst, nbytes, c->bal_lut, sizeof c->bal_lut);
    case VSO_TAP_QUANT:
        return copy_out(dst, nbytes, c->quant, sizeof c->quant);
    case VSO_TAP_MBAR:
        return copy_out(dst, nbytes, c->mbar, sizeof c->mbar);
    case VSO_TAP_COVER:
        return copy_out(dst, nbytes, c->cover, (size_t)P->canvas_w * P->canvas_h);
    case VSO_TAP_NEED:
        if (!pair_ok || sub < 0 || sub >= c->prm.lk_levels) return VSO_E_INVAL;
        return copy_out(dst, nbytes, c->need[p][sub], (size_t)c->pw[p][sub] * c->ph[p][sub]);
    case VSO_TAP_SURR_PRED:
        if (!pair_ok || sub < 0 || sub > 1 || !c->surr_pred[p][sub]) return VSO_E_INVAL;
        return copy_out(dst, nbytes, c->surr_pred[p][sub],
                        (size_t)c->pw[p][SURR_LEVEL] * c->ph[p][SURR_LEVEL] * 2 * sizeof(float));
    case VSO_TAP_FB:
        return copy_out(dst, nbytes, c->fb, (size_t)P->n_pairs * 2 * sizeof(unsigned long long));
    case VSO_TAP_SURR_OK:
        return copy_out(dst, nbytes, c->surr_ok, (size_t)P->n_pairs * sizeof(int));
    default:
        return VSO_E_INVAL;
    }
}

/* ------------------------------------------------------------------------ */
/* The learned flow surrogate (not in the paper): FP64 references of its     */
/* 3x3 convolutions, NHWC, weights [cout][tap][cin], tap = 3 ky + kx, zero    */
/* padding.  Written as the definitions, one output value at a time.          */
/* ------------------------------------------------------------------------ */

/* y[p][co] = b[co] + sum_tap sum_ci x[p + tap - (1,1)][ci] w[co][tap][ci] */
void vso_conv3x3(const double* x, int n, int h, int w, int cin, const double* wt, const double* b, int cout,
                 double* y)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int img = 0; img < n; ++img)
        for (int yy = 0; yy < h; ++yy)
            for (int xx = 0; xx < w; ++xx)
                for (int co = 0; co < cout; ++co) {
                    double acc = b ? b[co] : 0.0;
                    for (int tap = 0; tap < 9; ++tap) {
                        int sy = yy + tap / 3 - 1, sx = xx + tap % 3 - 1;
                        if (sy < 0 || sy >= h || sx < 0 || sx >= w) continue;
                        const double* src = x + (((size_t)img * h + sy) * w + sx) * cin;
                        for (int ci = 0; ci < cin; ++ci) acc += src[ci] * wt[((size_t)co * 9 + tap) * cin + ci];
                    }
                    y[(((size_t)img * h + yy) * w + xx) * cout + co] = acc;
                }
}

/* dx[p][ci] = sum over the outputs q that read p: dy[q][co] w[co][tap][ci] */
void vso_conv3x3_bwd_data(const double* dy, int n, int h, int w, int cout, const double* wt, int cin, double* dx)
{
#pragma omp parallel for schedule(static)
    for (int img = 0; img < n; ++img)
        for (int yy = 0; yy < h; ++yy)
            for (int xx = 0; xx < w; ++xx)
                for (int ci = 0; ci < cin; ++ci) {
                    double acc = 0.0;
                    for (int tap = 0; tap < 9; ++tap) {
                        /* output (oy, ox) reads (yy, xx) through tap when oy + ky - 1 = yy */
                        int oy = yy - (tap / 3 - 1), ox = xx - (tap % 3 - 1);
                        if (oy < 0 || oy >= h || ox < 0 || ox >= w) continue;
                        const double* g = dy + (((size_t)img * h + oy) * w + ox) * cout;
                        for (int co = 0; co < cout; ++co) acc += g[co] * wt[((size_t)co * 9 + tap) * cin + ci];
                    }
                    dx[(((size_t)img * h + yy) * w + xx) * cin + ci] = acc;
                }
}

/* dw[co][tap][ci] = sum_p dy[p][co] x[p + tap - (1,1)][ci];  db[co] = sum_p dy[p][co] */
void vso_conv3x3_bwd_weight(const double* x, const double* dy, int n, int h, int w, int cin, int cout, double* dw,
                            double* db)
{
#pragma omp parallel for schedule(static)
    for (int co = 0; co < cout; ++co) {
        for (int tap = 0; tap < 9; ++tap)
            for (int ci = 0; ci < cin; ++ci) {
                double acc = 0.0;
                for (int img = 0; img < n; ++img)
                    for (int yy = 0; yy < h; ++yy)
                        for (int xx = 0; xx < w; ++xx) {
                            int sy = yy + tap / 3 - 1, sx = xx + tap % 3 - 1;
                            if (sy < 0 || sy >= h || sx < 0 || sx >= w) continue;
                            acc += dy[(((size_t)img * h + yy) * w + xx) * cout + co] *
                                   x[(((size_t)img * h + sy) * w + sx) * cin + ci];
                        }
                dw[((size_t)co * 9 + tap) * cin + ci] = acc;
            }
        if (db) {
            double acc = 0.0;
            for (size_t p = 0; p < (size_t)n * h * w; ++p) acc += dy[p * cout + co];
            db[co] = acc;
        }
    }
}
