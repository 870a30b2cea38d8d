// vs_nn.h -- kernels of the learned flow surrogate (vs_nn.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vs {
namespace nn {

constexpr int MAXI = 64;   // images per launch

enum { CONV_LRELU = 0, CONV_LINEAR = 1, CONV_F32 = 2, CONV_FLOW2 = 3 };

// A launch over MAXI images of possibly different sizes stored back to back
// (NHWC): image i has w[i] x h[i] pixels starting at pixel pix_off[i], and
// owns blocks tile_off[i] .. tile_off[i + 1] - 1 (each launcher rebuilds
// tile_off for its own pixels per block).
struct ImgTable {
    int32_t n;
    int32_t w[MAXI], h[MAXI];
    int64_t pix_off[MAXI + 1];
    int32_t tile_off[MAXI + 1];
};

hipError_t conv3x3(const uint16_t* X, int cin, const uint16_t* W, const float* b, void* Y, int cout,
                   const ImgTable& T, int mode, float alpha, hipStream_t s);
int wgrad_blocks(const ImgTable& T);
hipError_t conv3x3_wgrad(const uint16_t* X, int cin, const uint16_t* dZ, int cout, const ImgTable& T, float* part,
                         float* dWb, hipStream_t s);
hipError_t flip_weights(const uint16_t* W, uint16_t* Wf, int cin, int cout, hipStream_t s);
hipError_t lrelu_bwd(const uint16_t* dH, const uint16_t* H, uint16_t* dZ, long n, float alpha, hipStream_t s);
hipError_t pack_pair(const float* Yt, const float* Ym, uint16_t* X, long npix, hipStream_t s);
hipError_t epe_loss(const float* pred, const float* label, uint16_t* dZ, float* block_loss, long npix, hipStream_t s);
hipError_t adam(float* w, float* m, float* v, const float* g, uint16_t* w_bf16, long n, float lr, float b1, float b2,
                float eps, int step, hipStream_t s);
hipError_t to_bf16(const float* a, uint16_t* b, long n, hipStream_t s);
hipError_t sum_blocks(const float* part, int n, float* out, hipStream_t s);
hipError_t pool_flow(const float* flow, int w, int h, int f, float* out, hipStream_t s);
// weight-gradient scratch for any image table of at most npix pixels in nimg images
size_t wgrad_scratch_bound(long npix, int nimg, int cin, int cout);

}  // namespace nn
}  // namespace vs
