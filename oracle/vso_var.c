/*
 * vso_var.c -- plain CPU oracle of the variational flow alternative of
 * section 3.2 (the paper cites a flow method it does not name, whose CPU
 * time suggests a global method; this is the coarse-to-fine warping scheme of
 * Brox et al. 2004 in a discrete form fixed here).  TEST INFRASTRUCTURE ONLY
 * (see vso_oracle.h).
 *
 * Per pyramid level, template T and moving image Mv (w x h), flow (u, v)
 * initialised from the coarser level (x2 bilinear, as the plain estimator):
 *  derivatives, once per level, central differences with clamped indices
 *    Tx, Ty of T; Mx, My of Mv; Mxx, Mxy, Myy the central differences of
 *    Mx, My (Mxx, Mxy from Mx; Myy from My);
 *  `outer` warps: each pixel samples Mv, Mx, My, Mxx, Mxy, Myy bilinearly at
 *    x + (u, v) (the position clamped into the level, as every sampler here):
 *      Iz = Mv_w - T, Ixz = Mx_w - Tx, Iyz = My_w - Ty, Ix = Mx_w, Iy = My_w,
 *    then (du, dv) = 0 and `inner` Jacobi steps of the linearised
 *    Euler-Lagrange equations of
 *      E = sum_x need(x) [Psi(Iz + Ix du + Iy dv)
 *                         + gamma Psi(|(Ixz, Iyz) + H (du, dv)|)]
 *          + alpha sum_x Psi(|grad(u + du)|^2 + |grad(v + dv)|^2),
 *    Psi(s^2) = sqrt(s^2 + eps^2), eps = 0.1 (luma units), with every
 *    Psi' = 1 / (2 sqrt(. + eps^2)) lagged at the previous step's (du, dv):
 *      du' = (b1 - A12 dv + alpha sum_n w_n (u_n + du_n - u)) / (A11 + alpha sum_n w_n)
 *      dv' = (b2 - A12 du + alpha sum_n w_n (v_n + dv_n - v)) / (A22 + alpha sum_n w_n)
 *    over the 4-neighbours n inside the level, w_n = (s(x) + s(n)) / 2 with
 *    s the smoothness Psi' from forward differences of (u + du, v + dv)
 *    (0 beyond the last column / row), A and b the data and gradient terms
 *    weighted by their Psi' (zero where need = 0);
 *  then (u, v) += (du, dv).
 * FP32 in the order written (explicit fmaf), correctly rounded division and
 * square root.  OpenMP runs over independent output rows only.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "vso_oracle.h"

static float at(const float* a, int w, int h, int x, int y)
{
    x = x < 0 ? 0 : (x > w - 1 ? w - 1 : x);
    y = y < 0 ? 0 : (y > h - 1 ? h - 1 : y);
    return a[(size_t)y * w + x];
}

static float bil(const float* a, int w, int h, float X, float Y)
{
    float cx = fminf(fmaxf(X, 0.0f), (float)(w - 1));
    float cy = fminf(fmaxf(Y, 0.0f), (float)(h - 1));
    float flx = floorf(cx), fly = floorf(cy);
    int x0 = (int)flx, y0 = (int)fly;
    float fx = cx - flx, fy = cy - fly;
    int x1 = x0 + 1 < w ? x0 + 1 : w - 1;
    int y1 = y0 + 1 < h ? y0 + 1 : h - 1;
    float p00 = a[(size_t)y0 * w + x0], p10 = a[(size_t)y0 * w + x1];
    float p01 = a[(size_t)y1 * w + x0], p11 = a[(size_t)y1 * w + x1];
    float t = fmaf(fx, p10 - p00, p00);
    float b = fmaf(fx, p11 - p01, p01);
    return fmaf(fy, b - t, t);
}

static void cdiff(const float* a, int w, int h, float* dx, float* dy)
{
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            if (dx) dx[(size_t)y * w + x] = 0.5f * (at(a, w, h, x + 1, y) - at(a, w, h, x - 1, y));
            if (dy) dy[(size_t)y * w + x] = 0.5f * (at(a, w, h, x, y + 1) - at(a, w, h, x, y - 1));
        }
}

/* smoothness Psi' at pixel (x, y) from forward differences of U = u + du, V = v + dv */
static float smooth_w(const float* U, const float* Vv, int w, int h, int x, int y, float eps2)
{
    const size_t q = (size_t)y * w + x;
    const float ux = x + 1 < w ? U[q + 1] - U[q] : 0.0f;
    const float uy = y + 1 < h ? U[q + w] - U[q] : 0.0f;
    const float vx = x + 1 < w ? Vv[q + 1] - Vv[q] : 0.0f;
    const float vy = y + 1 < h ? Vv[q + w] - Vv[q] : 0.0f;
    float s = fmaf(ux, ux, fmaf(uy, uy, fmaf(vx, vx, fmaf(vy, vy, eps2))));
    return 0.5f / sqrtf(s);
}

void vso_var_level(const float* T, const float* Mv, const uint8_t* need, int w, int h, float alpha, float gamma,
                   int outer, int inner, float* flow)
{
    const size_t n = (size_t)w * h;
    const float eps2 = 0.01f;   /* eps = 0.1 */
    float* d = malloc(sizeof(float) * n * 7);
    float *Tx = d, *Ty = d + n, *Mx = d + 2 * n, *My = d + 3 * n, *Mxx = d + 4 * n, *Mxy = d + 5 * n, *Myy = d + 6 * n;
    cdiff(T, w, h, Tx, Ty);
    cdiff(Mv, w, h, Mx, My);
    cdiff(Mx, w, h, Mxx, Mxy);
    cdiff(My, w, h, NULL, Myy);
    float* co = malloc(sizeof(float) * n * 8);   /* Iz Ix Iy Ixz Iyz Ixx Ixy Iyy */
    float* u = malloc(sizeof(float) * n * 6);
    float *v = u + n, *U = u + 2 * n, *Vv = u + 3 * n, *du = u + 4 * n, *dv = u + 5 * n;
    float* nd = malloc(sizeof(float) * n * 2);
    for (size_t q = 0; q < n; ++q) {
        u[q] = flow[q * 2];
        v[q] = flow[q * 2 + 1];
    }
    for (int o = 0; o < outer; ++o) {
#pragma omp parallel for schedule(static)
        for (int y = 0; y < h; ++y)
            for (int x = 0; x < w; ++x) {
                const size_t q = (size_t)y * w + x;
                const float X = (float)x + u[q], Y = (float)y + v[q];
                float* c = co + q * 8;
                const float mw = bil(Mv, w, h, X, Y), mx = bil(Mx, w, h, X, Y), my = bil(My, w, h, X, Y);
                c[0] = mw - T[q];
                c[1] = mx;
                c[2] = my;
                c[3] = mx - Tx[q];
                c[4] = my - Ty[q];
                c[5] = bil(Mxx, w, h, X, Y);
                c[6] = bil(Mxy, w, h, X, Y);
                c[7] = bil(Myy, w, h, X, Y);
                du[q] = 0.0f;
                dv[q] = 0.0f;
            }
        for (int it = 0; it < inner; ++it) {
            for (size_t q = 0; q < n; ++q) {
                U[q] = u[q] + du[q];
                Vv[q] = v[q] + dv[q];
            }
#pragma omp parallel for schedule(static)
            for (int y = 0; y < h; ++y)
                for (int x = 0; x < w; ++x) {
                    const size_t q = (size_t)y * w + x;
                    const float* c = co + q * 8;
                    float A11 = 0.0f, A12 = 0.0f, A22 = 0.0f, b1 = 0.0f, b2 = 0.0f;
                    if (!need || need[q]) {
                        const float e = fmaf(c[2], dv[q], fmaf(c[1], du[q], c[0]));
                        const float pd = 0.5f / sqrtf(fmaf(e, e, eps2));
                        const float gx = fmaf(c[6], dv[q], fmaf(c[5], du[q], c[3]));
                        const float gy = fmaf(c[7], dv[q], fmaf(c[6], du[q], c[4]));
                        const float pg = gamma * (0.5f / sqrtf(fmaf(gx, gx, fmaf(gy, gy, eps2))));
                        A11 = fmaf(pd, c[1] * c[1], pg * fmaf(c[5], c[5], c[6] * c[6]));
                        A12 = fmaf(pd, c[1] * c[2], pg * fmaf(c[5], c[6], c[6] * c[7]));
                        A22 = fmaf(pd, c[2] * c[2], pg * fmaf(c[6], c[6], c[7] * c[7]));
                        b1 = -fmaf(pd, c[1] * c[0], pg * fmaf(c[5], c[3], c[6] * c[4]));
                        b2 = -fmaf(pd, c[2] * c[0], pg * fmaf(c[6], c[3], c[7] * c[4]));
                    }
                    const float s0 = smooth_w(U, Vv, w, h, x, y, eps2);
                    float S = 0.0f, Su = 0.0f, Sv = 0.0f;
                    const int nx[4] = {x - 1, x + 1, x, x};
                    const int ny[4] = {y, y, y - 1, y + 1};
                    for (int k = 0; k < 4; ++k) {
                        if (nx[k] < 0 || nx[k] >= w || ny[k] < 0 || ny[k] >= h) continue;
                        const size_t qn = (size_t)ny[k] * w + nx[k];
                        const float wn = 0.5f * (s0 + smooth_w(U, Vv, w, h, nx[k], ny[k], eps2));
                        S += wn;
                        Su = fmaf(wn, U[qn] - u[q], Su);
                        Sv = fmaf(wn, Vv[qn] - v[q], Sv);
                    }
                    nd[q * 2] = fmaf(alpha, Su, fmaf(-A12, dv[q], b1)) / fmaf(alpha, S, A11);
                    nd[q * 2 + 1] = fmaf(alpha, Sv, fmaf(-A12, du[q], b2)) / fmaf(alpha, S, A22);
                }
            for (size_t q = 0; q < n; ++q) {
                du[q] = nd[q * 2];
                dv[q] = nd[q * 2 + 1];
            }
        }
        for (size_t q = 0; q < n; ++q) {
            u[q] += du[q];
            v[q] += dv[q];
        }
    }
    for (size_t q = 0; q < n; ++q) {
        flow[q * 2] = u[q];
        flow[q * 2 + 1] = v[q];
    }
    free(d);
    free(co);
    free(u);
    free(nd);
}

/* The coarse-to-fine driver on one template / moving pyramid: level L-1
 * starts at 0, each finer level from 2 x the bilinear sample of the coarser
 * result at x / 2 - 1/4 (the plain estimator's initialisation). */
void vso_var_pyramid(const float* const* T, const float* const* Mv, const uint8_t* const* need, const int* w,
                     const int* h, int levels, float alpha, float gamma, int outer, int inner, float* flow0)
{
    float* prev = NULL;
    for (int l = levels - 1; l >= 0; --l) {
        const int W = w[l], H = h[l];
        float* f = l == 0 ? flow0 : malloc(sizeof(float) * (size_t)W * H * 2);
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                float* o = f + ((size_t)y * W + x) * 2;
                o[0] = o[1] = 0.0f;
                if (!prev) continue;
                const int wc = w[l + 1], hc = h[l + 1];
                float cx = fminf(fmaxf(fmaf((float)x, 0.5f, -0.25f), 0.0f), (float)(wc - 1));
                float cy = fminf(fmaxf(fmaf((float)y, 0.5f, -0.25f), 0.0f), (float)(hc - 1));
                float flx = floorf(cx), fly = floorf(cy);
                int x0 = (int)flx, y0 = (int)fly;
                float fx = cx - flx, fy = cy - fly;
                int x1 = x0 + 1 < wc ? x0 + 1 : wc - 1;
                int y1 = y0 + 1 < hc ? y0 + 1 : hc - 1;
                for (int k = 0; k < 2; ++k) {
                    float p00 = prev[((size_t)y0 * wc + x0) * 2 + k], p10 = prev[((size_t)y0 * wc + x1) * 2 + k];
                    float p01 = prev[((size_t)y1 * wc + x0) * 2 + k], p11 = prev[((size_t)y1 * wc + x1) * 2 + k];
                    float a = fmaf(fx, p10 - p00, p00);
                    float b = fmaf(fx, p11 - p01, p01);
                    o[k] = 2.0f * fmaf(fy, b - a, a);
                }
            }
        vso_var_level(T[l], Mv[l], need ? need[l] : NULL, W, H, alpha, gamma, outer, inner, f);
        free(prev);
        prev = l == 0 ? NULL : f;
    }
}
