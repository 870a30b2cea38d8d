/*
 * vso_calib.c -- plain CPU oracle of the set-up step of section 3.1 of arXiv
 * 2308.09209: the coarse pairwise homography from camera parameters
 * (eqs. (8)-(12)) and its revision by a skew (translation) and a scale
 * matrix estimated from matched points on the widened overlap
 * (eqs. (13)-(14)).  TEST INFRASTRUCTURE ONLY (see vso_oracle.h).
 *
 * Readings (the paper's equations are garbled in places):
 *  - eq. (8)'s K is the 3x3 [f/dx, 0, cx/dx + u0; 0, f/dy, cy/dy + v0; 0, 0, 1]
 *    (its zero fourth column dropped, the second u0 read as v0);
 *  - eq. (11) on the world plane Z_W = 0: H_k = K_k [r1 r2 t_k] maps plane
 *    coordinates (X_W, Y_W, 1) to camera k's pixels;
 *  - eq. (12): H_ab = H_a H_b^-1 maps camera b's pixels to camera a's;
 *  - eq. (14): H' = M H N, N = diag(s_x, s_y, 1) scaling the source pixel, M
 *    the translation (t_x, t_y) of the result;
 *  - the SURF matching the paper uses is replaced by Harris corners and
 *    normalised cross-correlation: the pre-warp already brings the images
 *    within a few pixels, so a local search over integer positions matches;
 *    RANSAC draws its two-point samples as every pair of the first 64 matches
 *    in decreasing corner response (deterministic, no random numbers).
 *
 * Build: with vso_oracle.c (gcc -O2 -ffp-contract=off).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "vso_oracle.h"

void vso_calib_intrinsics(double f, double dx, double dy, double cx, double cy, double u0, double v0, double K[9])
{
    K[0] = f / dx; K[1] = 0.0;    K[2] = cx / dx + u0;
    K[3] = 0.0;    K[4] = f / dy; K[5] = cy / dy + v0;
    K[6] = 0.0;    K[7] = 0.0;    K[8] = 1.0;
}

static void mul3(const double a[9], const double b[9], double c[9])
{
    double t[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) t[r * 3 + k] = a[r * 3] * b[k] + a[r * 3 + 1] * b[3 + k] + a[r * 3 + 2] * b[6 + k];
    memcpy(c, t, sizeof t);
}

/* inverse by the adjugate over the determinant; 0 if singular */
static int inv3(const double a[9], double out[9])
{
    double c[9];
    c[0] = a[4] * a[8] - a[5] * a[7];
    c[1] = a[2] * a[7] - a[1] * a[8];
    c[2] = a[1] * a[5] - a[2] * a[4];
    c[3] = a[5] * a[6] - a[3] * a[8];
    c[4] = a[0] * a[8] - a[2] * a[6];
    c[5] = a[2] * a[3] - a[0] * a[5];
    c[6] = a[3] * a[7] - a[4] * a[6];
    c[7] = a[1] * a[6] - a[0] * a[7];
    c[8] = a[0] * a[4] - a[1] * a[3];
    double det = a[0] * c[0] + a[1] * c[3] + a[2] * c[6];
    if (det == 0.0 || !isfinite(det)) return 0;
    for (int i = 0; i < 9; ++i) out[i] = c[i] / det;
    return 1;
}

void vso_calib_plane_homography(const double K[9], const double R[9], const double t[3], double H[9])
{
    const double P[9] = {R[0], R[1], t[0], R[3], R[4], t[1], R[6], R[7], t[2]};
    mul3(K, P, H);
}

int vso_calib_pair(const double Ha[9], const double Hb[9], double Hab[9])
{
    double ib[9];
    if (!inv3(Hb, ib)) return VSO_E_INVAL;
    mul3(Ha, ib, Hab);
    return VSO_OK;
}

void vso_calib_refine(const double H[9], const double p[4], double Hr[9])
{
    const double M[9] = {1, 0, p[0], 0, 1, p[1], 0, 0, 1};
    const double N[9] = {p[2], 0, 0, 0, p[3], 0, 0, 0, 1};
    double t[9];
    mul3(M, H, t);
    mul3(t, N, Hr);
}

/* ---- matching ----------------------------------------------------------- */

/* BT.601 integer luma of an RGB byte image, as float */
static float luma_at(const uint8_t* F, int pitch, int x, int y)
{
    const uint8_t* p = F + (size_t)y * pitch + 3 * x;
    return (float)((77 * p[0] + 150 * p[1] + 29 * p[2] + 128) >> 8);
}

/* Harris response at (x, y) of luma image Y (w x h), 2 <= x < w - 2 etc.:
 * central differences Ix, Iy (halved), their products summed over the 5x5
 * box row by row, R = (Sxx Syy - Sxy^2) - 0.04 (Sxx + Syy)^2, FP32 in this
 * order; the box needs the differences at +-2, so 3 <= x < w - 3. */
float vso_calib_harris(const float* Y, int w, int x, int y)
{
    float sxx = 0.0f, sxy = 0.0f, syy = 0.0f;
    for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx) {
            const int q = (y + dy) * w + (x + dx);
            const float ix = 0.5f * (Y[q + 1] - Y[q - 1]);
            const float iy = 0.5f * (Y[q + w] - Y[q - w]);
            sxx = fmaf(ix, ix, sxx);
            sxy = fmaf(ix, iy, sxy);
            syy = fmaf(iy, iy, syy);
        }
    const float tr = sxx + syy;
    return (sxx * syy - sxy * sxy) - 0.04f * (tr * tr);
}

/* NCC score of the 11x11 patches centred at (xa, ya) in A and (xb, yb) in B:
 * cov |cov| / (va vb) (the sign of the correlation times its square), FP32,
 * sums row by row; 0 when a patch has no variance */
float vso_calib_ncc(const float* A, int wa, int xa, int ya, const float* B, int wb, int xb, int yb)
{
    float sa = 0.0f, sb = 0.0f;
    for (int dy = -5; dy <= 5; ++dy)
        for (int dx = -5; dx <= 5; ++dx) {
            sa += A[(ya + dy) * wa + xa + dx];
            sb += B[(yb + dy) * wb + xb + dx];
        }
    const float ma = sa / 121.0f, mb = sb / 121.0f;
    float cov = 0.0f, va = 0.0f, vb = 0.0f;
    for (int dy = -5; dy <= 5; ++dy)
        for (int dx = -5; dx <= 5; ++dx) {
            const float a = A[(ya + dy) * wa + xa + dx] - ma;
            const float b = B[(yb + dy) * wb + xb + dx] - mb;
            cov = fmaf(a, b, cov);
            va = fmaf(a, a, va);
            vb = fmaf(b, b, vb);
        }
    const float d = va * vb;
    return d > 0.0f ? (cov * fabsf(cov)) / d : 0.0f;
}

static void project(const double H[9], double u, double v, double* x, double* y)
{
    const double w = H[6] * u + H[7] * v + H[8];
    *x = (H[0] * u + H[1] * v + H[2]) / w;
    *y = (H[3] * u + H[4] * v + H[5]) / w;
}

/* the vertex of the parabola through scores (-1, sm), (0, s0), (1, sp), in
 * [-1/2, 1/2] (0 when the three are not a strict maximum at 0), FP64 */
static double subpixel(float sm, float s0, float sp)
{
    const double a = (double)sm, b = (double)s0, c = (double)sp;
    const double den = a - 2.0 * b + c;
    if (!(den < 0.0)) return 0.0;
    double d = 0.5 * (a - c) / den;
    return d < -0.5 ? -0.5 : (d > 0.5 ? 0.5 : d);
}

/* the model x_b = proj(H diag(sx, sy, 1) x_a) + (tx, ty); p = (tx, ty, sx, sy) */
static void model(const double H[9], const double p[4], double u, double v, double* x, double* y)
{
    project(H, p[2] * u, p[3] * v, x, y);
    *x += p[0];
    *y += p[1];
}

/* Gauss-Newton from p on the correspondences idx[0..n): 10 steps, normal
 * equations J^T J d = J^T r solved by Gaussian elimination with partial
 * pivoting; returns 0 if singular */
static int gauss_newton(const double H[9], const double* ua, const double* va, const double* xb, const double* yb,
                        const int* idx, int n, double p[4])
{
    for (int it = 0; it < 10; ++it) {
        double A[4][5];
        memset(A, 0, sizeof A);
        for (int k = 0; k < n; ++k) {
            const int m = idx[k];
            const double u = ua[m], v = va[m];
            const double su = p[2] * u, sv = p[3] * v;
            const double a = H[0] * su + H[1] * sv + H[2];
            const double b = H[3] * su + H[4] * sv + H[5];
            const double c = H[6] * su + H[7] * sv + H[8];
            const double px = a / c + p[0], py = b / c + p[1];
            /* rows of J for the x and y residuals, d/d(tx, ty, sx, sy) */
            const double jx[4] = {1.0, 0.0, (H[0] * u * c - a * H[6] * u) / (c * c), (H[1] * v * c - a * H[7] * v) / (c * c)};
            const double jy[4] = {0.0, 1.0, (H[3] * u * c - b * H[6] * u) / (c * c), (H[4] * v * c - b * H[7] * v) / (c * c)};
            const double rx = xb[m] - px, ry = yb[m] - py;
            for (int r = 0; r < 4; ++r) {
                for (int q = 0; q < 4; ++q) A[r][q] += jx[r] * jx[q] + jy[r] * jy[q];
                A[r][4] += jx[r] * rx + jy[r] * ry;
            }
        }
        for (int col = 0; col < 4; ++col) {
            int piv = col;
            for (int r = col + 1; r < 4; ++r)
                if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
            if (!(fabs(A[piv][col]) > 1e-300)) return 0;
            if (piv != col)
                for (int q = 0; q < 5; ++q) {
                    double t = A[col][q];
                    A[col][q] = A[piv][q];
                    A[piv][q] = t;
                }
            for (int r = col + 1; r < 4; ++r) {
                const double f = A[r][col] / A[col][col];
                for (int q = col; q < 5; ++q) A[r][q] -= f * A[col][q];
            }
        }
        double d[4];
        for (int r = 3; r >= 0; --r) {
            double s = A[r][4];
            for (int q = r + 1; q < 4; ++q) s -= A[r][q] * d[q];
            d[r] = s / A[r][r];
        }
        for (int r = 0; r < 4; ++r) p[r] += d[r];
    }
    for (int r = 0; r < 4; ++r)
        if (!isfinite(p[r])) return 0;
    return 1;
}

/* Estimate (tx, ty, sx, sy) of eq. (13) for the pre-warp H (camera a pixels ->
 * camera b pixels), from RGB byte frames a (wa x ha) and b (wb x hb):
 *  1. luma of both frames;
 *  2. Harris corners of a at pixels 8 + r px inside a whose H-image lies in b
 *     widened by `margin` px and at least 6 + r px inside b (r = search
 *     radius), 3x3 strict local maxima with positive response, the 256
 *     strongest (ties: lower y, then lower x);
 *  3. each matched to the integer position within +-r of round(H x) with the
 *     best NCC score (ties: first in row-major order), kept if its score is at
 *     least 0.49 (correlation 0.7), then moved in x and y to the vertex of the
 *     parabola through its score and its two neighbours' (within 1/2 px);
 *  4. RANSAC over every pair of the first 64 matches: Gauss-Newton on the two
 *     from (0, 0, 1, 1), inliers within 2 px, the most inliers kept (ties: the
 *     first pair); Gauss-Newton on its inliers from its estimate.
 * out: (tx, ty, sx, sy); *n_matches, *n_inliers.  Returns VSO_OK, or
 * VSO_E_INVAL when fewer than 2 matches or no model. */
int vso_calib_estimate(const uint8_t* Fa, int pa, int wa, int ha, const uint8_t* Fb, int pb, int wb, int hb,
                       const double H[9], int margin, int radius, double out[4], int* n_matches, int* n_inliers)
{
    float* A = malloc(sizeof(float) * (size_t)wa * ha);
    float* B = malloc(sizeof(float) * (size_t)wb * hb);
    for (int y = 0; y < ha; ++y)
        for (int x = 0; x < wa; ++x) A[y * wa + x] = luma_at(Fa, pa, x, y);
    for (int y = 0; y < hb; ++y)
        for (int x = 0; x < wb; ++x) B[y * wb + x] = luma_at(Fb, pb, x, y);
    const int r = radius, ea = 8 + r, eb = 6 + r;
    /* response map over the candidate region (0 elsewhere) */
    float* Rm = calloc((size_t)wa * ha, sizeof(float));
    for (int y = ea; y < ha - ea; ++y)
        for (int x = ea; x < wa - ea; ++x) {
            double bx, by;
            project(H, x, y, &bx, &by);
            if (!(bx >= -margin && bx <= wb - 1 + margin && by >= -margin && by <= hb - 1 + margin)) continue;
            const int cx = (int)floor(bx + 0.5), cy = (int)floor(by + 0.5);
            if (cx < eb || cx >= wb - eb || cy < eb || cy >= hb - eb) continue;
            Rm[y * wa + x] = vso_calib_harris(A, wa, x, y);
        }
    /* local maxima, strongest 256 */
    enum { MAXC = 256 };
    int cx_[MAXC], cy_[MAXC], nc = 0;
    float cr_[MAXC];
    for (int y = ea; y < ha - ea; ++y)
        for (int x = ea; x < wa - ea; ++x) {
            const float v = Rm[y * wa + x];
            if (!(v > 0.0f)) continue;
            int ok = 1;
            for (int dy = -1; dy <= 1 && ok; ++dy)
                for (int dx = -1; dx <= 1; ++dx)
                    if ((dx || dy) && !(v > Rm[(y + dy) * wa + x + dx])) {
                        ok = 0;
                        break;
                    }
            if (!ok) continue;
            /* insert in decreasing response (stable: equal responses keep scan order) */
            int pos = nc;
            while (pos > 0 && cr_[pos - 1] < v) --pos;
            if (pos >= MAXC) continue;
            const int last = nc < MAXC ? nc : MAXC - 1;
            for (int k = last; k > pos; --k) {
                cr_[k] = cr_[k - 1];
                cx_[k] = cx_[k - 1];
                cy_[k] = cy_[k - 1];
            }
            cr_[pos] = v;
            cx_[pos] = x;
            cy_[pos] = y;
            if (nc < MAXC) ++nc;
        }
    /* matches */
    double ua[MAXC], va[MAXC], xb[MAXC], yb[MAXC];
    int nm = 0;
    for (int k = 0; k < nc; ++k) {
        double bx, by;
        project(H, cx_[k], cy_[k], &bx, &by);
        const int px = (int)floor(bx + 0.5), py = (int)floor(by + 0.5);
        float best = -2.0f;
        int bxi = 0, byi = 0;
        for (int dy = -r; dy <= r; ++dy)
            for (int dx = -r; dx <= r; ++dx) {
                const float s = vso_calib_ncc(A, wa, cx_[k], cy_[k], B, wb, px + dx, py + dy);
                if (s > best) {
                    best = s;
                    bxi = px + dx;
                    byi = py + dy;
                }
            }
        if (best >= 0.49f) {
            ua[nm] = cx_[k];
            va[nm] = cy_[k];
            xb[nm] = bxi + subpixel(vso_calib_ncc(A, wa, cx_[k], cy_[k], B, wb, bxi - 1, byi), best,
                                    vso_calib_ncc(A, wa, cx_[k], cy_[k], B, wb, bxi + 1, byi));
            yb[nm] = byi + subpixel(vso_calib_ncc(A, wa, cx_[k], cy_[k], B, wb, bxi, byi - 1), best,
                                    vso_calib_ncc(A, wa, cx_[k], cy_[k], B, wb, bxi, byi + 1));
            ++nm;
        }
    }
    free(A);
    free(B);
    free(Rm);
    *n_matches = nm;
    *n_inliers = 0;
    if (nm < 2) return VSO_E_INVAL;
    const int ns = nm < 64 ? nm : 64;
    int best_in = -1;
    double best_p[4] = {0, 0, 1, 1};
    int idx[MAXC], inl[MAXC];
    for (int a = 0; a < ns; ++a)
        for (int b = a + 1; b < ns; ++b) {
            double p[4] = {0.0, 0.0, 1.0, 1.0};
            idx[0] = a;
            idx[1] = b;
            if (!gauss_newton(H, ua, va, xb, yb, idx, 2, p)) continue;
            int cnt = 0;
            for (int m = 0; m < nm; ++m) {
                double x, y;
                model(H, p, ua[m], va[m], &x, &y);
                if ((x - xb[m]) * (x - xb[m]) + (y - yb[m]) * (y - yb[m]) < 4.0) ++cnt;
            }
            if (cnt > best_in) {
                best_in = cnt;
                memcpy(best_p, p, sizeof p);
            }
        }
    if (best_in < 2) return VSO_E_INVAL;
    int ni = 0;
    for (int m = 0; m < nm; ++m) {
        double x, y;
        model(H, best_p, ua[m], va[m], &x, &y);
        if ((x - xb[m]) * (x - xb[m]) + (y - yb[m]) * (y - yb[m]) < 4.0) inl[ni++] = m;
    }
    double p[4];
    memcpy(p, best_p, sizeof p);
    if (!gauss_newton(H, ua, va, xb, yb, inl, ni, p)) return VSO_E_INVAL;
    memcpy(out, p, sizeof p);
    *n_inliers = ni;
    return VSO_OK;
}
