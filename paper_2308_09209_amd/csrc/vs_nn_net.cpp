// vs_nn_net.cpp -- the learned flow surrogate as a network object: its
// parameters, optimiser state and training workspaces on the device, and the
// forward / backward / Adam / save / load calls of the C ABI, each a sequence
// of the matrix-core and pointwise kernels of vs_nn.hip.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/vstitch.h"
#include "vs_nn.h"

using namespace vs;

struct vs_nn {
    vs_nn_spec spec;
    int L = 0;
    void* mem = nullptr;
    size_t n_params = 0;
    size_t off[VS_NN_MAX_LAYERS + 1] = {};   // layer l: weights at off[l], then its cout biases
    float* params = nullptr;                 // FP32 master parameters, layer by layer: w [cout][9][cin], b [cout]
    float* m = nullptr;
    float* v = nullptr;
    float* grads = nullptr;                  // same layout as params
    uint16_t* w16[VS_NN_MAX_LAYERS] = {};    // BF16 weights
    uint16_t* wf16[VS_NN_MAX_LAYERS] = {};   // flipped transposes [cin][9][cout] (data gradients)
    uint16_t* hid[VS_NN_MAX_LAYERS] = {};    // hidden activations of layers 0 .. L-2, [pixels][cout]
    float* pred = nullptr;                   // [pixels][cout of the last layer]
    uint16_t* dz[2] = {};                    // [pixels][32] gradients (ping-pong)
    uint16_t* dh = nullptr;                  // [pixels][32]
    float* scratch = nullptr;
    size_t scratch_bytes = 0;
    float* block_loss = nullptr;             // [pixels / 256 + 1]
    int step = 0;
    // the last forward
    const uint16_t* x = nullptr;
    nn::ImgTable T;
    vs_nn_images imgs;
    long npix = 0;
    int have_forward = 0;
};

namespace {

constexpr char kMagic[4] = {'V', 'S', 'N', 'N'};
constexpr uint32_t kVersion = 1;

vs_status st(hipError_t e) { return e == hipSuccess ? VS_OK : (e == hipErrorInvalidValue ? VS_E_INVAL : VS_E_DEVICE); }

bool layer_ok(int cin, int cout)
{
    // forward and weight-gradient kernels both exist
    return (cin == 16 && cout == 32) || (cin == 32 && cout == 32) || (cin == 32 && cout == 16);
}

bool spec_ok(const vs_nn_spec* s)
{
    if (!s || s->n_layers < 2 || s->n_layers > VS_NN_MAX_LAYERS) return false;
    if (s->cin[0] != 16 || s->cout[s->n_layers - 1] != 16) return false;
    if (s->in_live < 1 || s->in_live > 16 || !(s->alpha > 0.0f) || !(s->alpha < 1.0f)) return false;
    if (s->max_pixels < 1 || s->max_pixels > (int64_t)1 << 31) return false;
    for (int l = 0; l < s->n_layers; ++l) {
        if (!layer_ok(s->cin[l], s->cout[l])) return false;
        if (l > 0 && s->cin[l] != s->cout[l - 1]) return false;
    }
    return true;
}

bool make_table(const vs_nn_images* im, nn::ImgTable& T, long& npix)
{
    if (!im || im->n < 1 || im->n > nn::MAXI) return false;
    std::memset(&T, 0, sizeof T);
    T.n = im->n;
    npix = 0;
    for (int i = 0; i < im->n; ++i) {
        if (im->w[i] < 1 || im->h[i] < 1) return false;
        T.w[i] = im->w[i];
        T.h[i] = im->h[i];
        T.pix_off[i + 1] = T.pix_off[i] + (long)im->w[i] * im->h[i];
        // 64-pixel tiles (each launcher rebuilds them for its own tile size;
        // a table with no tiles launches nothing)
        T.tile_off[i + 1] = T.tile_off[i] + (int32_t)((T.pix_off[i + 1] - T.pix_off[i] + 63) / 64);
    }
    for (int i = im->n + 1; i <= nn::MAXI; ++i) {
        T.pix_off[i] = T.pix_off[im->n];
        T.tile_off[i] = T.tile_off[im->n];
    }
    npix = (long)T.pix_off[im->n];
    return true;
}

// splitmix64: a counter-based 64-bit generator (Steele, Lea and Flood 2014)
uint64_t splitmix64(uint64_t& s)
{
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// standard normal by the Box-Muller transform of two uniforms in (0, 1]
double normal(uint64_t& s)
{
    const double u1 = ((double)(splitmix64(s) >> 11) + 1.0) * 0x1.0p-53;
    const double u2 = (double)(splitmix64(s) >> 11) * 0x1.0p-53;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

float bf16_to_f32(uint16_t h)
{
    const uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// BF16 copies of the master weights and their flipped transposes
hipError_t refresh(vs_nn* n, hipStream_t s)
{
    hipError_t e = hipSuccess;
    for (int l = 0; l < n->L && e == hipSuccess; ++l) {
        const int ci = n->spec.cin[l], co = n->spec.cout[l];
        e = nn::to_bf16(n->params + n->off[l], n->w16[l], (long)co * 9 * ci, s);
        if (e == hipSuccess) e = nn::flip_weights(n->w16[l], n->wf16[l], ci, co, s);
    }
    return e;
}

}  // namespace

extern "C" {

vs_status vs_nn_destroy(vs_nn* n)
{
    if (!n) return VS_E_INVAL;
    if (n->mem) (void)hipFree(n->mem);
    delete n;
    return VS_OK;
}

vs_status vs_nn_create(const vs_nn_spec* spec, uint64_t seed, vs_nn** out)
{
    if (!out) return VS_E_INVAL;
    *out = nullptr;
    if (!spec_ok(spec)) return VS_E_INVAL;
    vs_nn* n = new (std::nothrow) vs_nn();
    if (!n) return VS_E_NOMEM;
    n->spec = *spec;
    n->L = spec->n_layers;
    const int L = n->L;
    const long P = (long)spec->max_pixels;
    for (int l = 0; l < L; ++l)
        n->off[l + 1] = n->off[l] + (size_t)spec->cout[l] * 9 * spec->cin[l] + (size_t)spec->cout[l];
    n->n_params = n->off[L];
    for (int l = 0; l < L; ++l)
        n->scratch_bytes = std::max(n->scratch_bytes, nn::wgrad_scratch_bound(P, nn::MAXI, spec->cin[l], spec->cout[l]));
    // one allocation, 256-byte aligned pieces
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    size_t bytes = 4 * al(n->n_params * 4);
    for (int l = 0; l < L; ++l) {
        const size_t nw = (size_t)spec->cout[l] * 9 * spec->cin[l];
        bytes += 2 * al(nw * 2);
        if (l + 1 < L) bytes += al((size_t)P * spec->cout[l] * 2);
    }
    bytes += al((size_t)P * spec->cout[L - 1] * 4) + 3 * al((size_t)P * 32 * 2) + al(n->scratch_bytes) +
             al(((size_t)P / 256 + 1) * 4);
    if (hipMalloc(&n->mem, bytes) != hipSuccess) {
        vs_nn_destroy(n);
        return VS_E_NOMEM;
    }
    uint8_t* p = (uint8_t*)n->mem;
    auto take = [&](size_t b) {
        uint8_t* r = p;
        p += al(b);
        return r;
    };
    n->params = (float*)take(n->n_params * 4);
    n->m = (float*)take(n->n_params * 4);
    n->v = (float*)take(n->n_params * 4);
    n->grads = (float*)take(n->n_params * 4);
    for (int l = 0; l < L; ++l) {
        const size_t nw = (size_t)spec->cout[l] * 9 * spec->cin[l];
        n->w16[l] = (uint16_t*)take(nw * 2);
        n->wf16[l] = (uint16_t*)take(nw * 2);
        if (l + 1 < L) n->hid[l] = (uint16_t*)take((size_t)P * spec->cout[l] * 2);
    }
    n->pred = (float*)take((size_t)P * spec->cout[L - 1] * 4);
    n->dz[0] = (uint16_t*)take((size_t)P * 32 * 2);
    n->dz[1] = (uint16_t*)take((size_t)P * 32 * 2);
    n->dh = (uint16_t*)take((size_t)P * 32 * 2);
    n->scratch = (float*)take(n->scratch_bytes);
    n->block_loss = (float*)take(((size_t)P / 256 + 1) * 4);
    // He initialisation over the live inputs (the first layer reads in_live
    // of its 16 channels; the others start at 0), the last layer scaled by
    // 0.1 (a near-zero first flow), biases 0
    std::vector<float> h(n->n_params, 0.0f);
    uint64_t rs = seed;
    for (int l = 0; l < L; ++l) {
        const int ci = spec->cin[l], co = spec->cout[l];
        const int live = l == 0 ? spec->in_live : ci;
        const double sd = std::sqrt(2.0 / (9.0 * live)) * (l == L - 1 ? 0.1 : 1.0);
        for (int o = 0; o < co; ++o)
            for (int t = 0; t < 9; ++t)
                for (int i = 0; i < ci; ++i) {
                    const double g = normal(rs);
                    h[n->off[l] + ((size_t)o * 9 + t) * ci + i] = i < live ? (float)(g * sd) : 0.0f;
                }
    }
    bool ok = hipMemcpy(n->params, h.data(), n->n_params * 4, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemset(n->m, 0, n->n_params * 4) == hipSuccess && hipMemset(n->v, 0, n->n_params * 4) == hipSuccess &&
              hipMemset(n->grads, 0, n->n_params * 4) == hipSuccess && refresh(n, nullptr) == hipSuccess &&
              hipDeviceSynchronize() == hipSuccess;
    if (!ok) {
        vs_nn_destroy(n);
        return VS_E_DEVICE;
    }
    *out = n;
    return VS_OK;
}

vs_status vs_nn_forward(vs_nn* n, const uint16_t* x, const vs_nn_images* imgs, float* pred, void* stream)
{
    if (!n || !x) return VS_E_INVAL;
    nn::ImgTable T;
    long npix = 0;
    if (!make_table(imgs, T, npix) || npix > n->spec.max_pixels) return VS_E_INVAL;
    if ((uintptr_t)x % 16 != 0) return VS_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    n->have_forward = 0;
    const int L = n->L;
    const uint16_t* h = x;
    hipError_t e = hipSuccess;
    for (int l = 0; l + 1 < L && e == hipSuccess; ++l) {
        e = nn::conv3x3(h, n->spec.cin[l], n->w16[l], n->params + n->off[l] + (size_t)n->spec.cout[l] * 9 * n->spec.cin[l],
                        n->hid[l], n->spec.cout[l], T, nn::CONV_LRELU, n->spec.alpha, s);
        h = n->hid[l];
    }
    const int ci = n->spec.cin[L - 1], co = n->spec.cout[L - 1];
    if (e == hipSuccess)
        e = nn::conv3x3(h, ci, n->w16[L - 1], n->params + n->off[L - 1] + (size_t)co * 9 * ci, n->pred, co, T,
                        nn::CONV_F32, n->spec.alpha, s);
    if (e == hipSuccess && pred)
        e = hipMemcpyAsync(pred, n->pred, (size_t)npix * co * 4, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return st(e);
    n->x = x;
    n->T = T;
    n->imgs = *imgs;
    n->npix = npix;
    n->have_forward = 1;
    return VS_OK;
}

vs_status vs_nn_loss(vs_nn* n, const float* label, float* loss_sum, void* stream)
{
    if (!n || !label || !loss_sum) return VS_E_INVAL;
    if (!n->have_forward) return VS_E_STATE;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = nn::epe_loss(n->pred, label, n->dz[0], n->block_loss, n->npix, s);
    if (e == hipSuccess) e = nn::sum_blocks(n->block_loss, (int)((n->npix + 255) / 256), loss_sum, s);
    return st(e);
}

vs_status vs_nn_backward(vs_nn* n, const float* label, float* loss_sum, void* stream)
{
    if (!n || !label) return VS_E_INVAL;
    if (!n->have_forward) return VS_E_STATE;
    hipStream_t s = (hipStream_t)stream;
    const long P = n->npix;
    int cur = 0;
    hipError_t e = nn::epe_loss(n->pred, label, n->dz[cur], n->block_loss, P, s);
    if (e == hipSuccess && loss_sum) e = nn::sum_blocks(n->block_loss, (int)((P + 255) / 256), loss_sum, s);
    for (int l = n->L - 1; l >= 0 && e == hipSuccess; --l) {
        const int ci = n->spec.cin[l], co = n->spec.cout[l];
        const uint16_t* in = l == 0 ? n->x : n->hid[l - 1];
        e = nn::conv3x3_wgrad(in, ci, n->dz[cur], co, n->T, n->scratch, n->grads + n->off[l], s);
        if (e != hipSuccess || l == 0) break;
        e = nn::conv3x3(n->dz[cur], co, n->wf16[l], nullptr, n->dh, ci, n->T, nn::CONV_LINEAR, n->spec.alpha, s);
        if (e == hipSuccess) e = nn::lrelu_bwd(n->dh, n->hid[l - 1], n->dz[cur ^ 1], P * ci, n->spec.alpha, s);
        cur ^= 1;
    }
    return st(e);
}

vs_status vs_nn_adam_step(vs_nn* n, float lr, float b1, float b2, float eps, void* stream)
{
    if (!n || !(lr >= 0.0f) || !(b1 >= 0.0f && b1 < 1.0f) || !(b2 >= 0.0f && b2 < 1.0f) || !(eps > 0.0f))
        return VS_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    n->step += 1;
    hipError_t e = nn::adam(n->params, n->m, n->v, n->grads, nullptr, (long)n->n_params, lr, b1, b2, eps, n->step, s);
    if (e == hipSuccess) e = refresh(n, s);
    return st(e);
}

vs_status vs_nn_params(vs_nn* n, float* params, float* grads, size_t* count, void* stream)
{
    if (!n) return VS_E_INVAL;
    if (count) *count = n->n_params;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (params) e = hipMemcpyAsync(params, n->params, n->n_params * 4, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && grads) e = hipMemcpyAsync(grads, n->grads, n->n_params * 4, hipMemcpyDeviceToDevice, s);
    return st(e);
}

vs_status vs_nn_save(vs_nn* n, void* blob, size_t cap, size_t* nbytes)
{
    if (!n || !nbytes) return VS_E_INVAL;
    const int L = n->L;
    size_t need = 16 + 8 * (size_t)L;
    for (int l = 0; l < L; ++l)
        need += (size_t)n->spec.cout[l] * 9 * n->spec.cin[l] * 2 + (size_t)n->spec.cout[l] * 4;
    *nbytes = need;
    if (!blob) return VS_OK;
    if (cap < need) return VS_E_INVAL;
    if (hipDeviceSynchronize() != hipSuccess) return VS_E_DEVICE;
    uint8_t* p = (uint8_t*)blob;
    auto put = [&](const void* src, size_t b) {
        std::memcpy(p, src, b);
        p += b;
    };
    const uint32_t ver = kVersion, nl = (uint32_t)L;
    put(kMagic, 4);
    put(&ver, 4);
    put(&nl, 4);
    put(&n->spec.alpha, 4);
    for (int l = 0; l < L; ++l) {
        const uint32_t ci = (uint32_t)n->spec.cin[l], co = (uint32_t)n->spec.cout[l];
        put(&ci, 4);
        put(&co, 4);
    }
    for (int l = 0; l < L; ++l) {
        const size_t nw = (size_t)n->spec.cout[l] * 9 * n->spec.cin[l];
        if (hipMemcpy(p, n->w16[l], nw * 2, hipMemcpyDeviceToHost) != hipSuccess) return VS_E_DEVICE;
        p += nw * 2;
        if (hipMemcpy(p, n->params + n->off[l] + nw, (size_t)n->spec.cout[l] * 4, hipMemcpyDeviceToHost) != hipSuccess)
            return VS_E_DEVICE;
        p += (size_t)n->spec.cout[l] * 4;
    }
    return VS_OK;
}

vs_status vs_nn_load(vs_nn* n, const void* blob, size_t nbytes)
{
    if (!n || !blob) return VS_E_INVAL;
    const int L = n->L;
    size_t need = 16 + 8 * (size_t)L;
    for (int l = 0; l < L; ++l)
        need += (size_t)n->spec.cout[l] * 9 * n->spec.cin[l] * 2 + (size_t)n->spec.cout[l] * 4;
    const uint8_t* p = (const uint8_t*)blob;
    uint32_t ver = 0, nl = 0;
    float alpha = 0.0f;
    if (nbytes != need || std::memcmp(p, kMagic, 4) != 0) return VS_E_INVAL;
    std::memcpy(&ver, p + 4, 4);
    std::memcpy(&nl, p + 8, 4);
    std::memcpy(&alpha, p + 12, 4);
    if (ver != kVersion || nl != (uint32_t)L || alpha != n->spec.alpha) return VS_E_INVAL;
    for (int l = 0; l < L; ++l) {
        uint32_t ci = 0, co = 0;
        std::memcpy(&ci, p + 16 + 8 * l, 4);
        std::memcpy(&co, p + 20 + 8 * l, 4);
        if ((int)ci != n->spec.cin[l] || (int)co != n->spec.cout[l]) return VS_E_INVAL;
    }
    // master weights = the stored BF16 values exactly; optimiser state reset
    std::vector<float> h(n->n_params);
    size_t q = 16 + 8 * (size_t)L;
    for (int l = 0; l < L; ++l) {
        const size_t nw = (size_t)n->spec.cout[l] * 9 * n->spec.cin[l];
        for (size_t i = 0; i < nw; ++i) {
            uint16_t b;
            std::memcpy(&b, p + q + 2 * i, 2);
            h[n->off[l] + i] = bf16_to_f32(b);
        }
        q += nw * 2;
        std::memcpy(&h[n->off[l] + nw], p + q, (size_t)n->spec.cout[l] * 4);
        q += (size_t)n->spec.cout[l] * 4;
    }
    if (hipDeviceSynchronize() != hipSuccess) return VS_E_DEVICE;
    bool ok = hipMemcpy(n->params, h.data(), n->n_params * 4, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemset(n->m, 0, n->n_params * 4) == hipSuccess && hipMemset(n->v, 0, n->n_params * 4) == hipSuccess &&
              refresh(n, nullptr) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
    if (!ok) return VS_E_DEVICE;
    n->step = 0;
    n->have_forward = 0;
    return VS_OK;
}

}  // extern "C"
