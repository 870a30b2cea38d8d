// vs_nn_host.cpp -- C ABI of the learned flow surrogate's building blocks.
#include <cstring>

#include "../../include/vstitch.h"
#include "vs_nn.h"

using namespace vs;

namespace {

bool make_table(const vs_nn_images* im, nn::ImgTable& T)
{
    if (!im || im->n < 1 || im->n > nn::MAXI) return false;
    std::memset(&T, 0, sizeof T);
    T.n = im->n;
    T.pix_off[0] = 0;
    T.tile_off[0] = 0;
    for (int i = 0; i < im->n; ++i) {
        if (im->w[i] < 1 || im->h[i] < 1) return false;
        T.w[i] = im->w[i];
        T.h[i] = im->h[i];
        const long np = (long)im->w[i] * im->h[i];
        T.pix_off[i + 1] = T.pix_off[i] + np;
        T.tile_off[i + 1] = T.tile_off[i] + (int)((np + 63) / 64);
    }
    for (int i = im->n + 1; i <= nn::MAXI; ++i) {
        T.pix_off[i] = T.pix_off[im->n];
        T.tile_off[i] = T.tile_off[im->n];
    }
    return true;
}

vs_status st(hipError_t e) { return e == hipSuccess ? VS_OK : (e == hipErrorInvalidValue ? VS_E_INVAL : VS_E_DEVICE); }

bool shape_ok(int cin, int cout)
{
    return (cin == 16 && cout == 32) || (cin == 32 && cout == 32) || (cin == 32 && cout == 16) ||
           (cin == 16 && cout == 16);
}

}  // namespace

extern "C" {

vs_status vs_nn_conv3x3(const uint16_t* x, int cin, const uint16_t* w, const float* bias, void* y, int cout,
                        const vs_nn_images* imgs, int mode, float alpha, void* stream)
{
    nn::ImgTable T;
    if (!x || !w || !y || !shape_ok(cin, cout) || mode < 0 || mode > 3 || !make_table(imgs, T)) return VS_E_INVAL;
    return st(nn::conv3x3(x, cin, w, bias, y, cout, T, mode, alpha, (hipStream_t)stream));
}

size_t vs_nn_wgrad_scratch_bytes(int cin, int cout, const vs_nn_images* imgs)
{
    nn::ImgTable T;
    if (!make_table(imgs, T)) return 0;
    return (size_t)nn::wgrad_blocks(T) * (size_t)(cout * 9 * cin + cout) * sizeof(float);
}

vs_status vs_nn_conv3x3_wgrad(const uint16_t* x, int cin, const uint16_t* dz, int cout, const vs_nn_images* imgs,
                              float* scratch, size_t scratch_bytes, float* dwb, void* stream)
{
    nn::ImgTable T;
    if (!x || !dz || !scratch || !dwb || !(shape_ok(cin, cout) && !(cin == 16 && cout == 16)) || !make_table(imgs, T))
        return VS_E_INVAL;
    if (scratch_bytes < vs_nn_wgrad_scratch_bytes(cin, cout, imgs)) return VS_E_INVAL;
    return st(nn::conv3x3_wgrad(x, cin, dz, cout, T, scratch, dwb, (hipStream_t)stream));
}

vs_status vs_nn_flip_weights(const uint16_t* w, uint16_t* wf, int cin, int cout, void* stream)
{
    if (!w || !wf || cin < 1 || cout < 1) return VS_E_INVAL;
    return st(nn::flip_weights(w, wf, cin, cout, (hipStream_t)stream));
}

vs_status vs_nn_lrelu_bwd(const uint16_t* dh, const uint16_t* h, uint16_t* dz, int64_t n, float alpha, void* stream)
{
    if (!dh || !h || !dz || n < 0) return VS_E_INVAL;
    return st(nn::lrelu_bwd(dh, h, dz, (long)n, alpha, (hipStream_t)stream));
}

vs_status vs_nn_pack_pair(const float* yt, const float* ym, uint16_t* x, int64_t npix, void* stream)
{
    if (!yt || !ym || !x || npix < 0) return VS_E_INVAL;
    return st(nn::pack_pair(yt, ym, x, (long)npix, (hipStream_t)stream));
}

vs_status vs_nn_epe_loss(const float* pred, const float* label, uint16_t* dz, float* block_loss, int64_t npix,
                         void* stream)
{
    if (!pred || !label || !dz || !block_loss || npix < 0) return VS_E_INVAL;
    return st(nn::epe_loss(pred, label, dz, block_loss, (long)npix, (hipStream_t)stream));
}

vs_status vs_nn_adam(float* w, float* m, float* v, const float* g, uint16_t* w_bf16, int64_t n, float lr, float b1,
                     float b2, float eps, int step, void* stream)
{
    if (!w || !m || !v || !g || n < 0 || step < 1) return VS_E_INVAL;
    return st(nn::adam(w, m, v, g, w_bf16, (long)n, lr, b1, b2, eps, step, (hipStream_t)stream));
}

vs_status vs_nn_to_bf16(const float* a, uint16_t* b, int64_t n, void* stream)
{
    if (!a || !b || n < 0) return VS_E_INVAL;
    return st(nn::to_bf16(a, b, (long)n, (hipStream_t)stream));
}

vs_status vs_nn_pool_flow(const float* flow, int w, int h, int factor, float* out, void* stream)
{
    if (!flow || !out || w < 1 || h < 1 || factor < 1 || factor > 64) return VS_E_INVAL;
    return st(nn::pool_flow(flow, w, h, factor, out, (hipStream_t)stream));
}

}  // extern "C"
