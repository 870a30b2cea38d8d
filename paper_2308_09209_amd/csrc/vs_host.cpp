// vs_host.cpp -- host runtime of libvstitch: the C ABI, the rig planner and
// the per-frame launch sequence.  Every step of the frame runs in the
// kernels of vs_kernels.hip; the host only plans once and launches.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "vs_internal.h"

using namespace vs;

struct vs_ctx {
    vs_rig rig;
    vs_params prm;
    DevPlan hp;              // host copy of the device plan (holds device pointers)
    DevPlan* dp = nullptr;   // device copy
    void* arena = nullptr;   // per-frame workspace
    size_t arena_bytes = 0;
    void* plan_mem = nullptr;  // coverage bits + candidates + pixel codes + scan
    uint8_t* pano_pre = nullptr;
    // the flow domain on the host (plan time) and the flow-tile lists built from it
    std::vector<uint8_t> need_h[MAXP][MAXL];
    uint32_t* tiles = nullptr;           // device: per level, tiles_cap[l] entries from tiles_off[l]
    size_t tiles_off[MAXL] = {}, tiles_cap[MAXL] = {};
    vs_plan_info info;
    int sticky = 0;
    std::string err;
    // step timing: a ring of event slots, 7 events per frame
    static constexpr int kSlots = 64, kEv = 7;
    int timing = 0;
    hipEvent_t ev[kSlots][kEv] = {};
    int slot_used[kSlots] = {};
    int next_slot = 0;
    double ms_sum[6] = {};
    uint32_t timed_frames = 0;
    // learned surrogate
    void* surr_mem = nullptr;
    void* var_mem = nullptr;             // variational flow workspace (flow = 2)
    SurrNet net;
    int surr_loaded = 0;
    // bumped whenever the launch sequence changes (flow variant, surrogate):
    // a batch holding this context recaptures its graph
    uint32_t gen = 0;
    char arch[32] = {};                  // device architecture at create (tuning-record key)
    // vs_flow_only: a plain-flow context for the last strip size and its two luma images
    vs_flow* fo = nullptr;
    float* fo_luma = nullptr;
    int fo_w = 0, fo_h = 0;
};

namespace {

const char* kStatus[] = {"ok", "invalid argument", "geometry", "out of memory", "device error",
                         "state mismatch", "unsupported"};

// ---- tuning records (process-wide) ----
struct TuneRec {
    vs_tune_key k;
    vs_tune_entry e;
};
std::mutex g_tune_mu;
std::vector<TuneRec> g_tune;

bool tune_key_eq(const vs_tune_key& a, const vs_tune_key& b)
{
    return std::strncmp(a.arch, b.arch, sizeof a.arch) == 0 && a.n_cams == b.n_cams && a.canvas_w == b.canvas_w &&
           a.canvas_h == b.canvas_h && a.lk_levels == b.lk_levels && a.lk_radius == b.lk_radius;
}

bool variant_code_ok(int v) { return v == 0 || ((v & 7) >= 1 && (v & 7) <= 4 && (v & ~31) == 0); }

// a record usable for its own key: known codes on the key's levels (9x9
// codes only with radius 4), 0 past them, tile height 0, 8 or 16
bool tune_rec_ok(const vs_tune_key& k, const vs_tune_entry& e)
{
    if (k.arch[0] == 0 || std::memchr(k.arch, 0, sizeof k.arch) == nullptr) return false;
    if (k.lk_levels < 1 || k.lk_levels > VS_MAX_LEVELS || k.n_cams < 2 || k.n_cams > VS_MAX_CAMS) return false;
    for (int l = 0; l < VS_MAX_LEVELS; ++l) {
        const int v = e.flow_variant[l];
        if (!variant_code_ok(v) || (l >= k.lk_levels && v != 0) || (v > 0 && k.lk_radius != LK_R_MAX)) return false;
    }
    return e.pyr_tile_rows == 0 || e.pyr_tile_rows == 8 || e.pyr_tile_rows == 16;
}

void tune_put_locked(const vs_tune_key& k, const vs_tune_entry& e)
{
    for (TuneRec& r : g_tune)
        if (tune_key_eq(r.k, k)) {
            r.e = e;
            return;
        }
    g_tune.push_back(TuneRec{k, e});
}

// the current device's architecture name without its feature suffixes
void device_arch(char out[32])
{
    std::memset(out, 0, 32);
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        std::strncpy(out, "unknown", 31);
        return;
    }
    size_t n = 0;
    while (n < 31 && prop.gcnArchName[n] && prop.gcnArchName[n] != ':') ++n;
    std::memcpy(out, prop.gcnArchName, n);
}

// fused-pyramid tile height (level-2 rows) and its tile table
void set_pyr_rows(DevPlan& h, int rows)
{
    h.pyrf_ty = rows;
    h.pyrf_off[0] = 0;
    for (int f = 0; f < 2 * h.n_pairs; ++f) {
        const int p = f >> 1;
        const int w2 = h.levels >= 3 ? h.lw[p][2] : 0, h2 = h.levels >= 3 ? h.lh[p][2] : 0;
        h.pyrf_tx[f] = (w2 + PF_TX - 1) / PF_TX;
        h.pyrf_off[f + 1] = h.pyrf_off[f] + h.pyrf_tx[f] * ((h2 + h.pyrf_ty - 1) / h.pyrf_ty);
    }
}

// 3x3 product c = a b, entries ((a_r0 b_0c + a_r1 b_1c) + a_r2 b_2c)
void mat3_mul(const double* a, const double* b, double* c)
{
    double t[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k)
            t[r * 3 + k] = (a[r * 3 + 0] * b[0 * 3 + k] + a[r * 3 + 1] * b[1 * 3 + k]) + a[r * 3 + 2] * b[2 * 3 + k];
    std::memcpy(c, t, sizeof t);
}

// inverse = a positive multiple of H^-1 (w > 0 keeps meaning "in front of
// the camera"): the adjugate over |adjugate[8]| with the sign of det, so the
// last entry is exactly +1 or -1
bool hom_inverse(const double* a, double* inv)
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
    const double det = (a[0] * adj[0] + a[1] * adj[3]) + a[2] * adj[6];
    if (!std::isfinite(det) || det == 0.0 || adj[8] == 0.0 || !std::isfinite(adj[8])) return false;
    const double den = ((det > 0.0) == (adj[8] > 0.0)) ? adj[8] : -adj[8];
    for (int i = 0; i < 9; ++i) inv[i] = adj[i] / den;
    return true;
}

vs_status validate_rig(const vs_rig* r)
{
    if (!r || r->n_cams < 2 || r->n_cams > VS_MAX_CAMS) return VS_E_INVAL;
    if (r->canvas_w <= 0 || r->canvas_h <= 0) return VS_E_INVAL;
    if (r->ring && (r->n_cams < 3 || r->ring_period != r->canvas_w)) return VS_E_INVAL;
    for (int k = 0; k < r->n_cams; ++k)
        if (r->cam_w[k] < 2 || r->cam_h[k] < 2 || r->cam_pitch[k] < 3 * r->cam_w[k]) return VS_E_INVAL;
    return VS_OK;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

vs_status fail(vs_ctx* c, vs_status s, const std::string& why)
{
    if (c) c->err = why;
    return s;
}

vs_status dev_fail(vs_ctx* c, hipError_t e, const char* where)
{
    c->sticky = 1;
    c->err = std::string(where) + ": " + hipGetErrorString(e);
    return VS_E_DEVICE;
}

#define VS_CHECK(call, where)                          \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return dev_fail(c, e_, where); \
    } while (0)

void free_ctx(vs_ctx* c)
{
    if (!c) return;
    for (auto& slot : c->ev)
        for (auto& e : slot)
            if (e) (void)hipEventDestroy(e);
    if (c->arena) (void)hipFree(c->arena);
    if (c->plan_mem) (void)hipFree(c->plan_mem);
    if (c->dp) (void)hipFree(c->dp);
    if (c->pano_pre) (void)hipFree(c->pano_pre);
    if (c->surr_mem) (void)hipFree(c->surr_mem);
    if (c->tiles) (void)hipFree(c->tiles);
    if (c->var_mem) (void)hipFree(c->var_mem);
    if (c->fo) (void)vs_flow_destroy(c->fo);
    if (c->fo_luma) (void)hipFree(c->fo_luma);
    delete c;
}

// Default 9x9 flow-kernel variant of a level, from its count of 64 x 16 tiles
// (n16) and the blocks the device holds at once (`resident`, four staged flow
// blocks per compute unit).  A level with under two waves of resident blocks
// at 1 pixel per thread takes P = 1 in the unrolled form that finishes its
// (few) deferred pixels in-block: at about one wavefront per SIMD its rows'
// LDS reads overlap, and no tail launch follows.  Otherwise the most pixels
// per thread P (4, 3, 2, 1; n16 * 4 / P blocks) that still gives at least
// one full wave of blocks, with a tail launch for the deferred pixels: over
// a sequence, frames whose deferred pixels cluster in a few blocks make
// in-block finishing end late (4x1080p p99 0.614 -> 0.638 ms, 8x4K mean
// 3.556 -> 3.584 ms with it at the coarser levels).  Every P takes the form
// that keeps the previous gradient row in registers: with the regrouped
// right-hand side it costs no occupancy at P = 4 and saves the row's second
// LDS read.
int default_lk_P(int n16, int resident)
{
    if ((long)n16 * 4 < 2L * resident) return 1 + VS_FLOW_ALT + VS_FLOW_INBLOCK;
    for (int P = 4; P >= 1; --P) {
        const long blocks = ((long)n16 * 4 + P - 1) / P;
        if (blocks >= resident) return P + VS_FLOW_ALT;
    }
    return 1 + VS_FLOW_ALT + VS_FLOW_INBLOCK;
}

// blocks of the staged flow kernel the current device holds at once
int lk_resident_blocks()
{
    static int cached = 0;
    if (cached) return cached;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        ncu <= 0)
        ncu = 256;
    cached = 4 * ncu;
    return cached;
}

// Choose the flow-kernel variant of one level (0: generic 16x16 kernel;
// 1, 2, 4: 9x9-window kernel with that many pixels per thread) and rebuild
// that level's tile table; the caller re-uploads the plan.
void set_lk_tiles(DevPlan& h, int l, int P)
{
    int tx = LK_T, ty = LK_T;
    h.lk_P[l] = P;
    h.lk_tiles[l] = nullptr;
    if (P > 0) {
        tx = LKW_TX;
        ty = 4 * (P & 7);
    }
    h.lk_off[l][0] = 0;
    for (int f = 0; f < 2 * h.n_pairs; ++f) {
        const int p = f >> 1;
        h.lk_tx[l][f] = (h.lw[p][l] + tx - 1) / tx;
        h.lk_off[l][f + 1] = h.lk_off[l][f] + h.lk_tx[l][f] * ((h.lh[p][l] + ty - 1) / ty);
    }
}

bool var_params_ok(const vs_params& P)
{
    return std::isfinite(P.var_alpha) && P.var_alpha > 0.0f && std::isfinite(P.var_gamma) && P.var_gamma >= 0.0f &&
           P.var_outer >= 0 && P.var_outer <= 64 && P.var_inner >= 0 && P.var_inner <= 1024 && P.var_inner % 2 == 0;
}

// Variational-flow blocks and workspace of a plan (its sizes set): per level
// the 256-pixel blocks of every field; the derivative planes per camera, the
// coefficients and increments per direction.  Returns the bytes needed and,
// with base non-null, points the plan's buffers into them.
size_t var_layout(DevPlan& h, uint8_t* base)
{
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off = (off + b + 255) / 256 * 256;
        return base ? base + o : nullptr;
    };
    for (int l = 0; l < h.levels; ++l) {
        h.var_off[l][0] = 0;
        h.var_toff[l][0] = 0;
        for (int f = 0; f < 2 * h.n_pairs; ++f) {
            const int p = f >> 1;
            h.var_off[l][f + 1] = h.var_off[l][f] + (int32_t)(((size_t)h.lw[p][l] * h.lh[p][l] + 255) / 256);
            h.var_toff[l][f + 1] = h.var_toff[l][f] + ((h.lw[p][l] + VAR_TX - 1) / VAR_TX) *
                                                          ((h.lh[p][l] + VAR_TY - 1) / VAR_TY);
        }
    }
    for (int p = 0; p < h.n_pairs; ++p)
        for (int k = 0; k < 2; ++k)
            for (int l = 0; l < h.levels; ++l) {
                const size_t n = (size_t)h.lw[p][l] * h.lh[p][l];
                h.var_D[p][k][l] = (float*)take(n * 5 * 4);
                h.var_co[p][k][l] = (float*)take(n * 8 * 4);
                h.var_dd[p][k][l][0] = (float2*)take(n * 8);
                h.var_dd[p][k][l][1] = (float2*)take(n * 8);
            }
    return off;
}

// The most flow tiles any variant lists for a level: a band never holds more
// tiles than a row of the box grid.
size_t lk_tile_cap(const DevPlan& h, int l)
{
    size_t n = 0;
    for (int f = 0; f < 2 * h.n_pairs; ++f) {
        const size_t w = (size_t)h.lw[f >> 1][l], hh = (size_t)h.lh[f >> 1][l];
        n += std::max(((w + LKW_TX - 1) / LKW_TX) * ((hh + 3) / 4), ((w + LK_T - 1) / LK_T) * ((hh + LK_T - 1) / LK_T));
    }
    return n;
}

// Flow tiles of one level that follow the flow domain: per band of tile rows,
// tiles from the band's first domain column to its last.  The overlap of two
// rotated cameras slants across its bounding box, so a box-grid tile at the
// slant's edge holds few domain pixels; a band's tiles start where its domain
// starts.  Sets lk_off and lk_tiles and uploads the list (the caller uploads
// the plan).  Strips wider or taller than 16 bits keep the box grid.
hipError_t band_tiles(vs_ctx* c, int l)
{
    DevPlan& h = c->hp;
    if (!c->tiles) return hipSuccess;
    int tx = LK_T, ty = LK_T;
    if (h.lk_P[l] > 0) {
        tx = LKW_TX;
        ty = 4 * (h.lk_P[l] & 7);
    }
    for (int p = 0; p < h.n_pairs; ++p)
        if (h.lw[p][l] > 65535 || h.lh[p][l] > 65535 || c->need_h[p][l].size() != (size_t)h.lw[p][l] * h.lh[p][l]) {
            h.lk_tiles[l] = nullptr;   // set_lk_tiles' grid stays
            return hipSuccess;
        }
    std::vector<uint32_t> list;
    int32_t off[2 * MAXP + 1];
    off[0] = 0;
    for (int f = 0; f < 2 * h.n_pairs; ++f) {
        const int p = f >> 1, w = h.lw[p][l], hh = h.lh[p][l];
        const uint8_t* nd = c->need_h[p][l].data();
        for (int y0 = 0; y0 < hh; y0 += ty) {
            int xa = w, xb = -1;
            for (int y = y0; y < std::min(y0 + ty, hh); ++y) {
                const uint8_t* row = nd + (size_t)y * w;
                int x = 0;
                while (x < w && !row[x]) ++x;
                if (x == w) continue;
                xa = std::min(xa, x);
                x = w - 1;
                while (!row[x]) --x;
                xb = std::max(xb, x);
            }
            for (int x0 = xa; x0 <= xb; x0 += tx) list.push_back((uint32_t)x0 | ((uint32_t)y0 << 16));
        }
        off[f + 1] = (int32_t)list.size();
    }
    if (list.size() > c->tiles_cap[l]) return hipErrorInvalidValue;
    uint32_t* dst = c->tiles + c->tiles_off[l];
    if (!list.empty()) {
        const hipError_t e = hipMemcpy(dst, list.data(), list.size() * 4, hipMemcpyHostToDevice);
        if (e != hipSuccess) return e;
    }
    for (int f = 0; f <= 2 * h.n_pairs; ++f) h.lk_off[l][f] = off[f];
    h.lk_tiles[l] = dst;
    return hipSuccess;
}

}  // namespace

extern "C" {

int vs_abi_version(void) { return VS_ABI_VERSION; }

const char* vs_status_str(vs_status s)
{
    int i = -(int)s;
    if (i < 0 || i > 6) return "unknown status";
    return kStatus[i];
}

vs_status vs_default_params(vs_params* p)
{
    if (!p) return VS_E_INVAL;
    std::memset(p, 0, sizeof *p);
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
    p->debug_taps = 0;
    p->pyr_tile_rows = 0;
    p->readings = 0;
    p->var_alpha = 128.0f;
    p->var_gamma = 16.0f;
    p->var_outer = 3;
    p->var_inner = 10;
    return VS_OK;
}

vs_status vs_compose_homographies(const vs_rig* rig, double* Hk, float* Hinv)
{
    if (!rig || !Hk || !Hinv || rig->n_cams < 1 || rig->n_cams > VS_MAX_CAMS) return VS_E_INVAL;
    double H[9];
    std::memcpy(H, rig->H_ref, sizeof H);
    for (int k = 0; k < rig->n_cams; ++k) {
        if (k > 0) mat3_mul(H, rig->H_pair[k], H);
        for (double v : H)
            if (!std::isfinite(v)) return VS_E_INVAL;
        std::memcpy(Hk + 9 * k, H, sizeof H);
        double inv[9];
        if (!hom_inverse(H, inv)) return VS_E_INVAL;
        for (int i = 0; i < 9; ++i) Hinv[9 * k + i] = (float)inv[i];
    }
    return VS_OK;
}

vs_status vs_create(const vs_rig* rig, const vs_params* prm, vs_ctx** out)
{
    if (!out) return VS_E_INVAL;
    *out = nullptr;
    vs_status st = validate_rig(rig);
    if (st != VS_OK) return st;
    vs_params P;
    if (prm) P = *prm;
    else vs_default_params(&P);
    if (P.lk_levels < 1 || P.lk_levels > VS_MAX_LEVELS || P.lk_iters < 0 || P.lk_radius < 0 ||
        P.lk_radius > LK_R_MAX || P.color_window < 0 || P.color_window > 3 || P.lambda_pct < 1 ||
        P.lambda_pct > 49 || !(P.ridge >= 0.0) || !std::isfinite(P.lk_lambda) ||
        (P.pyr_tile_rows != 0 && P.pyr_tile_rows != 8 && P.pyr_tile_rows != 16) || (P.readings & ~7) != 0 ||
        P.flow < 0 || P.flow > 2 || !var_params_ok(P))
        return VS_E_INVAL;

    vs_ctx* c = new (std::nothrow) vs_ctx();
    if (!c) return VS_E_NOMEM;
    c->rig = *rig;
    c->prm = P;
    DevPlan& h = c->hp;
    std::memset(&h, 0, sizeof h);
    const int N = rig->n_cams;
    h.n_cams = N;
    h.canvas_w = rig->canvas_w;
    h.canvas_h = rig->canvas_h;
    h.ring = rig->ring ? 1 : 0;
    h.Wp = rig->ring ? rig->ring_period : 0;
    h.levels = P.lk_levels;
    h.pano_pitch = 3 * rig->canvas_w;
    h.color_window = P.color_window;
    h.min_pixels = P.min_pixels;
    h.use_flow = P.flow;
    h.balance = P.balance;
    h.lambda_pct = P.lambda_pct;
    h.lk_radius = P.lk_radius;
    h.lk_iters = P.lk_iters;
    h.lk_lambda = P.lk_lambda;
    h.readings = P.readings;
    h.var_alpha = P.var_alpha;
    h.var_gamma = P.var_gamma;
    h.var_outer = P.var_outer;
    h.var_inner = P.var_inner;
    h.ridge = P.ridge;
    double Hk[VS_MAX_CAMS * 9];
    float Hinv[VS_MAX_CAMS * 9];
    if (vs_compose_homographies(rig, Hk, Hinv) != VS_OK) {
        free_ctx(c);
        return VS_E_INVAL;
    }
    for (int k = 0; k < N; ++k) {
        h.cam_w[k] = rig->cam_w[k];
        h.cam_h[k] = rig->cam_h[k];
        h.cam_pitch[k] = rig->cam_pitch[k];
        for (int i = 0; i < 9; ++i) h.hinv[k][i] = Hinv[9 * k + i];
    }
    // overlap pairs: (k-1, k) along the chain, (N-1, 0) closing a ring
    h.n_pairs = N - 1 + (h.ring ? 1 : 0);
    for (int a = 0; a < MAXC; ++a)
        for (int b = 0; b < MAXC; ++b) h.pair_of[a][b] = -1;
    for (int p = 0; p < h.n_pairs; ++p) {
        h.pj[p] = p < N - 1 ? p : N - 1;
        h.pi[p] = p < N - 1 ? p + 1 : 0;
        h.psi[p] = p < N - 1 ? 0 : 1;
        h.pair_of[h.pj[p]][h.pi[p]] = p;
        h.pair_of[h.pi[p]][h.pj[p]] = p;
    }
    h.cover_words = (h.canvas_w + 31) / 32;
    h.blend_tx = (h.canvas_w + BL_TX - 1) / BL_TX;
    h.blend_ty = (h.canvas_h + BL_TY - 1) / BL_TY;

    // ---- plan scan on the device: coverage, candidates, strip boxes ----
    const size_t cover_bytes = align_up((size_t)h.canvas_h * h.cover_words * 4, 256);
    const size_t cand_bytes = align_up((size_t)h.blend_tx * h.blend_ty * 8, 256);
    const size_t code_bytes = align_up((size_t)h.canvas_w * h.canvas_h * 2, 256);
    const size_t scan_bytes = align_up(sizeof(PlanScan), 256);
    hipError_t e = hipMalloc(&c->plan_mem, cover_bytes + cand_bytes + code_bytes + scan_bytes);
    if (e != hipSuccess) {
        free_ctx(c);
        return VS_E_NOMEM;
    }
    e = hipMalloc((void**)&c->dp, sizeof(DevPlan));
    if (e != hipSuccess) {
        free_ctx(c);
        return VS_E_NOMEM;
    }
    h.cover = (uint32_t*)c->plan_mem;
    h.cand = (unsigned long long*)((uint8_t*)c->plan_mem + cover_bytes);
    h.pix_code = (uint16_t*)((uint8_t*)c->plan_mem + cover_bytes + cand_bytes);
    PlanScan* dscan = (PlanScan*)((uint8_t*)c->plan_mem + cover_bytes + cand_bytes + code_bytes);
    PlanScan scan;
    std::memset(&scan, 0, sizeof scan);
    for (int p = 0; p < MAXP; ++p) {
        scan.bx0[p] = scan.by0[p] = 0x3fffffff;
        scan.bx1[p] = scan.by1[p] = -0x3fffffff;
    }
    auto cleanup_dev = [&](hipError_t err, const char* where) {
        std::fprintf(stderr, "vs_create: %s: %s\n", where, hipGetErrorString(err));
        free_ctx(c);
        return VS_E_DEVICE;
    };
    if ((e = hipMemset(h.cand, 0, cand_bytes)) != hipSuccess) return cleanup_dev(e, "hipMemset");
    if ((e = hipMemcpy(dscan, &scan, sizeof scan, hipMemcpyHostToDevice)) != hipSuccess) return cleanup_dev(e, "hipMemcpy");
    if ((e = hipMemcpy(c->dp, &h, sizeof h, hipMemcpyHostToDevice)) != hipSuccess) return cleanup_dev(e, "hipMemcpy");
    if ((e = launch_plan_scan(c->dp, h, dscan, nullptr)) != hipSuccess) return cleanup_dev(e, "plan scan launch");
    if ((e = hipMemcpy(&scan, dscan, sizeof scan, hipMemcpyDeviceToHost)) != hipSuccess) return cleanup_dev(e, "plan scan");
    if (scan.err || scan.n_covered == 0) {
        free_ctx(c);
        return VS_E_GEOMETRY;
    }
    for (int p = 0; p < h.n_pairs; ++p) {
        if (scan.bx1[p] < scan.bx0[p]) {
            free_ctx(c);
            return VS_E_GEOMETRY;
        }
        h.sx0[p] = scan.bx0[p];
        h.sy0[p] = scan.by0[p];
        h.sw[p] = scan.bx1[p] - scan.bx0[p] + 1;
        h.sh[p] = scan.by1[p] - scan.by0[p] + 1;
        int w = h.sw[p], hh = h.sh[p];
        for (int l = 0; l < h.levels; ++l) {
            h.lw[p][l] = w;
            h.lh[p][l] = hh;
            w = (w + 1) / 2;
            hh = (hh + 1) / 2;
        }
    }
    // ---- tile tables ----
    h.strip_off[0] = 0;
    for (int p = 0; p < h.n_pairs; ++p) {
        h.strip_tx[p] = (h.sw[p] + STRIP_TX - 1) / STRIP_TX;
        h.strip_off[p + 1] = h.strip_off[p] + h.strip_tx[p] * ((h.sh[p] + STRIP_TY - 1) / STRIP_TY);
    }
    // fused pyramid tiles: 32 x 16 level-2 pixels, or 32 x 8 when that grid
    // would leave the device with under ~6 blocks per compute unit
    int n16 = 0;
    for (int f = 0; f < 2 * h.n_pairs && h.levels >= 3; ++f) {
        const int p = f >> 1;
        n16 += ((h.lw[p][2] + PF_TX - 1) / PF_TX) * ((h.lh[p][2] + 15) / 16);
    }
    set_pyr_rows(h, P.pyr_tile_rows ? P.pyr_tile_rows : (n16 >= 1536 ? 16 : 8));
    for (int l = 0; l < h.levels; ++l) {
        h.pyr_off[l][0] = 0;
        for (int f = 0; f < 2 * h.n_pairs; ++f) {
            const int p = f >> 1, w = h.lw[p][l], hh = h.lh[p][l];
            h.pyr_tx[l][f] = (w + PYR_TX - 1) / PYR_TX;
            h.pyr_off[l][f + 1] = h.pyr_off[l][f] + h.pyr_tx[l][f] * ((hh + PYR_TY - 1) / PYR_TY);
        }
        // flow kernel: the 9x9-window kernel (pixels per thread from the level's
        // tile count); other radii use the generic kernel
        int n16 = 0;
        for (int f = 0; f < 2 * h.n_pairs; ++f) {
            const int p = f >> 1;
            n16 += ((h.lw[p][l] + LKW_TX - 1) / LKW_TX) * ((h.lh[p][l] + 15) / 16);
        }
        set_lk_tiles(h, l, P.lk_radius == LK_R_MAX ? default_lk_P(n16, lk_resident_blocks()) : 0);
    }
    // ---- workspace arena ----
    size_t off = 0;
    size_t o_strip[MAXP], o_mask[MAXP], o_pyr[MAXP][2][MAXL], o_flow[MAXP][2][MAXL], o_need[MAXP][MAXL];
    size_t o_queue[MAXL];
    for (int p = 0; p < h.n_pairs; ++p) {
        const size_t n = (size_t)h.sw[p] * h.sh[p];
        o_strip[p] = off;
        off = align_up(off + 2 * n * 4, 256);
        o_mask[p] = off;
        off = align_up(off + n, 256);
        for (int l = 0; l < h.levels; ++l) {
            o_need[p][l] = off;
            off = align_up(off + (size_t)h.lw[p][l] * h.lh[p][l], 256);
        }
        for (int k = 0; k < 2; ++k)
            for (int l = 0; l < h.levels; ++l) {
                o_pyr[p][k][l] = off;
                off = align_up(off + (size_t)h.lw[p][l] * h.lh[p][l] * 4, 256);
                o_flow[p][k][l] = off;
                off = align_up(off + (size_t)h.lw[p][l] * h.lh[p][l] * 8, 256);
            }
    }
    for (int l = 0; l < h.levels; ++l) {
        // every flow pixel of the level can be deferred at most once per frame
        size_t cap = 0;
        for (int p = 0; p < h.n_pairs; ++p) cap += 2 * (size_t)h.lw[p][l] * h.lh[p][l];
        h.lk_qcap[l] = h.lk_P[l] > 0 ? (int32_t)cap : 0;
        o_queue[l] = off;
        off = align_up(off + (size_t)h.lk_qcap[l] * 16, 256);
    }
    const size_t o_acc = off;
    off = align_up(off + sizeof(Accum), 256);
    const size_t o_res = off;
    off = align_up(off + sizeof(Results), 256);
    const size_t o_state = off;
    off = align_up(off + sizeof(vs_color_state), 256);
    c->arena_bytes = off;
    if (hipMalloc(&c->arena, off) != hipSuccess) {
        free_ctx(c);
        return VS_E_NOMEM;
    }
    uint8_t* base = (uint8_t*)c->arena;
    for (int l = 0; l < h.levels; ++l) h.lk_queue[l] = (uint4*)(base + o_queue[l]);
    for (int p = 0; p < h.n_pairs; ++p) {
        h.strip[p] = (uint32_t*)(base + o_strip[p]);
        h.mask[p] = base + o_mask[p];
        for (int l = 0; l < h.levels; ++l) h.need[p][l] = base + o_need[p][l];
        for (int k = 0; k < 2; ++k)
            for (int l = 0; l < h.levels; ++l) {
                h.pyr[p][k][l] = (float*)(base + o_pyr[p][k][l]);
                h.flow[p][k][l] = (float2*)(base + o_flow[p][k][l]);
            }
    }
    h.acc = (Accum*)(base + o_acc);
    h.res = (Results*)(base + o_res);
    h.state = (vs_color_state*)(base + o_state);
    if ((e = hipMemset(c->arena, 0, off)) != hipSuccess) return cleanup_dev(e, "hipMemset");
    if (h.use_flow == 2) {
        const size_t vb = var_layout(h, nullptr);
        if (hipMalloc(&c->var_mem, vb) != hipSuccess) {
            free_ctx(c);
            return VS_E_NOMEM;
        }
        var_layout(h, (uint8_t*)c->var_mem);
        if ((e = hipMemset(c->var_mem, 0, vb)) != hipSuccess) return cleanup_dev(e, "hipMemset");
        c->arena_bytes += vb;
    }
    if (P.debug_taps) {
        if (hipMalloc((void**)&c->pano_pre, (size_t)h.canvas_h * h.pano_pitch) != hipSuccess) {
            free_ctx(c);
            return VS_E_NOMEM;
        }
    }
    if ((e = hipMemcpy(c->dp, &h, sizeof h, hipMemcpyHostToDevice)) != hipSuccess) return cleanup_dev(e, "hipMemcpy");
    if ((e = launch_need(c->dp, h, nullptr)) != hipSuccess) return cleanup_dev(e, "flow domain launch");
    if ((e = hipDeviceSynchronize()) != hipSuccess) return cleanup_dev(e, "flow domain");
    vs_color_state s0;
    std::memset(&s0, 0, sizeof s0);
    s0.version = VS_STATE_VERSION;
    s0.size = sizeof(vs_color_state);
    s0.n_pairs = (uint32_t)h.n_pairs;
    if ((e = hipMemcpy(h.state, &s0, sizeof s0, hipMemcpyHostToDevice)) != hipSuccess) return cleanup_dev(e, "hipMemcpy");

    vs_plan_info& I = c->info;
    std::memset(&I, 0, sizeof I);
    I.canvas_w = h.canvas_w;
    I.canvas_h = h.canvas_h;
    I.pano_pitch = h.pano_pitch;
    I.n_cams = N;
    I.n_pairs = h.n_pairs;
    I.ring = h.ring;
    I.ring_period = h.Wp;
    I.lk_levels = h.levels;
    for (int p = 0; p < h.n_pairs; ++p) {
        I.pair_j[p] = h.pj[p];
        I.pair_i[p] = h.pi[p];
        I.pair_si[p] = h.psi[p];
        I.strip_x0[p] = h.sx0[p];
        I.strip_y0[p] = h.sy0[p];
        I.strip_w[p] = h.sw[p];
        I.strip_h[p] = h.sh[p];
    }
    I.n_covered = (int64_t)scan.n_covered;
    // flow-domain accounting (plan time, from the domain the kernels built)
    {
        const int r = h.lk_radius;
        for (int p = 0; p < h.n_pairs; ++p)
            for (int l = 0; l < h.levels; ++l) {
                const int w = h.lw[p][l], hh = h.lh[p][l];
                std::vector<uint8_t>& nb = c->need_h[p][l];
                nb.resize((size_t)w * hh);
                if ((e = hipMemcpy(nb.data(), h.need[p][l], nb.size(), hipMemcpyDeviceToHost)) != hipSuccess)
                    return cleanup_dev(e, "flow domain copy");
                uint64_t px = 0, taps = 0;
                for (int y = 0; y < hh; ++y) {
                    const uint64_t wy = (uint64_t)(std::min(y + r, hh - 1) - std::max(y - r, 0) + 1);
                    for (int x = 0; x < w; ++x) {
                        if (!nb[(size_t)y * w + x]) continue;
                        px += 1;
                        taps += wy * (uint64_t)(std::min(x + r, w - 1) - std::max(x - r, 0) + 1);
                    }
                }
                I.flow_px[p][l] = px;
                I.flow_taps[p][l] = taps;
            }
    }
    // a tuning record for this device and plan shape: its flow variants and
    // pyramid tile height (identical results, other speeds)
    device_arch(c->arch);
    {
        vs_tune_key k;
        vs_tune_entry te;
        if (vs_tune_key_of(c, &k) == VS_OK && vs_tune_get(&k, &te) == VS_OK) {
            for (int l = 0; l < h.levels; ++l)
                if (h.lk_P[l] > 0 && te.flow_variant[l] > 0) set_lk_tiles(h, l, te.flow_variant[l]);
            if (te.pyr_tile_rows && P.pyr_tile_rows == 0) set_pyr_rows(h, te.pyr_tile_rows);
        }
    }
    // flow tiles that follow the domain, every level
    size_t tiles_n = 0;
    for (int l = 0; l < h.levels; ++l) {
        c->tiles_off[l] = tiles_n;
        c->tiles_cap[l] = lk_tile_cap(h, l);
        tiles_n += c->tiles_cap[l];
    }
    if (h.use_flow && tiles_n > 0) {
        if (hipMalloc((void**)&c->tiles, tiles_n * 4) != hipSuccess) {
            free_ctx(c);
            return VS_E_NOMEM;
        }
        for (int l = 0; l < h.levels; ++l)
            if ((e = band_tiles(c, l)) != hipSuccess) return cleanup_dev(e, "flow tiles");
        if ((e = hipMemcpy(c->dp, &h, sizeof h, hipMemcpyHostToDevice)) != hipSuccess) return cleanup_dev(e, "hipMemcpy");
    }
    I.workspace_bytes = c->arena_bytes + cover_bytes + cand_bytes + code_bytes + scan_bytes + sizeof(DevPlan) +
                        tiles_n * 4;
    I.state_bytes = sizeof(vs_color_state);
    *out = c;
    return VS_OK;
}

void vs_destroy(vs_ctx* c) { free_ctx(c); }

vs_status vs_query(const vs_ctx* c, vs_plan_info* out)
{
    if (!c || !out) return VS_E_INVAL;
    *out = c->info;
    return VS_OK;
}

const char* vs_last_error(const vs_ctx* c) { return c ? c->err.c_str() : "null context"; }

static vs_status harvest_slot(vs_ctx* c, int i)
{
    if (!c->slot_used[i]) return VS_OK;
    VS_CHECK(hipEventSynchronize(c->ev[i][6]), "hipEventSynchronize");
    for (int k = 0; k < 5; ++k) {
        float ms = 0.0f;
        VS_CHECK(hipEventElapsedTime(&ms, c->ev[i][k], c->ev[i][k + 1]), "hipEventElapsedTime");
        c->ms_sum[k] += ms;
    }
    float ms = 0.0f;
    VS_CHECK(hipEventElapsedTime(&ms, c->ev[i][0], c->ev[i][6]), "hipEventElapsedTime");
    c->ms_sum[5] += ms;
    c->timed_frames += 1;
    c->slot_used[i] = 0;
    return VS_OK;
}

vs_status vs_set_timing(vs_ctx* c, int on)
{
    if (!c) return VS_E_INVAL;
    if (c->sticky) return VS_E_DEVICE;
    if (on && !c->ev[0][0])
        for (auto& slot : c->ev)
            for (auto& e : slot) VS_CHECK(hipEventCreate(&e), "hipEventCreate");
    VS_CHECK(hipDeviceSynchronize(), "hipDeviceSynchronize");
    for (int i = 0; i < vs_ctx::kSlots; ++i) c->slot_used[i] = 0;
    for (double& v : c->ms_sum) v = 0.0;
    c->timed_frames = 0;
    c->next_slot = 0;
    c->timing = on ? 1 : 0;
    return VS_OK;
}

vs_status vs_get_timing(vs_ctx* c, double ms[6], uint32_t* frames)
{
    if (!c || !ms) return VS_E_INVAL;
    if (c->sticky) return VS_E_DEVICE;
    for (int i = 0; i < vs_ctx::kSlots; ++i) {
        vs_status st = harvest_slot(c, i);
        if (st != VS_OK) return st;
    }
    for (int k = 0; k < 6; ++k) ms[k] = c->ms_sum[k];
    if (frames) *frames = c->timed_frames;
    return VS_OK;
}

static vs_status check_state(const vs_ctx* c, const vs_color_state* s)
{
    if (s->version != VS_STATE_VERSION || s->size != sizeof(vs_color_state) ||
        s->n_pairs != (uint32_t)c->hp.n_pairs)
        return VS_E_STATE;
    return VS_OK;
}

vs_status vs_state_set(vs_ctx* c, const vs_color_state* in)
{
    if (!c || !in) return VS_E_INVAL;
    if (c->sticky) return VS_E_DEVICE;
    if (check_state(c, in) != VS_OK) return fail(c, VS_E_STATE, "colour state version / size / pair count mismatch");
    VS_CHECK(hipDeviceSynchronize(), "hipDeviceSynchronize");
    VS_CHECK(hipMemcpy(c->hp.state, in, sizeof *in, hipMemcpyHostToDevice), "hipMemcpy state");
    return VS_OK;
}

vs_status vs_state_get(vs_ctx* c, vs_color_state* out)
{
    if (!c || !out) return VS_E_INVAL;
    if (c->sticky) return VS_E_DEVICE;
    VS_CHECK(hipDeviceSynchronize(), "hipDeviceSynchronize");
    VS_CHECK(hipMemcpy(out, c->hp.state, sizeof *out, hipMemcpyDeviceToHost), "hipMemcpy state");
    return VS_OK;
}

}  // extern "C"

namespace {

// The per-frame launch sequence for a group of contexts (one context for
// vs_stitch, several for a batch).  ev (7 events) brackets the steps when
// non-null; pre (single context only) receives a copy of the pre-balance
// panorama.
hipError_t enqueue_frame(const Group& g, hipStream_t s, hipEvent_t* ev, uint8_t* pre, const uint8_t* pano,
                         size_t pano_bytes, const char** where, const Fork* fk = nullptr)
{
    hipError_t e;
#define VS_STEP(call, name)              \
    do {                                 \
        if ((e = (call)) != hipSuccess) { \
            *where = name;               \
            return e;                    \
        }                                \
    } while (0)
    int levels = 0;
    for (int c = 0; c < g.n; ++c) levels = std::max(levels, (int)g.hp[c]->levels);
    if (ev) VS_STEP(hipEventRecord(ev[0], s), "hipEventRecord");
    VS_STEP(launch_strips(g, s), "strips");
    VS_STEP(launch_lut(g, s), "lut");   // + eq. (1)'s B from the strips' conditional sums
    VS_STEP(launch_solve(g, s), "solve");
    if (ev) VS_STEP(hipEventRecord(ev[1], s), "hipEventRecord");
    // pyramids of 3+ levels: levels 0-2 in one pass (plain flow: all three
    // written; surrogate modes: level 2, its input); fewer levels: level by level
    VS_STEP(launch_pyr0(g, PYR_UNFUSED, s), "pyr0");
    for (int l = 0; l + 1 < levels; ++l) VS_STEP(launch_pyr_down(g, l, PYR_UNFUSED, s), "pyr_down");
    VS_STEP(launch_pyr_fused(g, PYR_UNFUSED, s), "pyr_fused");
    if (ev) VS_STEP(hipEventRecord(ev[2], s), "hipEventRecord");
    int n_surr = 0;
    for (int c = 0; c < g.n; ++c) n_surr += surrogate_active(g, c) ? 1 : 0;
    if (fk && n_surr > 1) {
        // the contexts' surrogate chains are independent small launches: run
        // them side by side
        VS_STEP(hipEventRecord(fk->fork, s), "fork");
        for (int c = 0; c < g.n; ++c) {
            if (!surrogate_active(g, c)) continue;
            VS_STEP(hipStreamWaitEvent(fk->side[c], fk->fork, 0), "fork wait");
            VS_STEP(launch_surrogate_ctx(g, c, fk->side[c]), "surrogate");
            VS_STEP(hipEventRecord(fk->join[c], fk->side[c]), "join");
            VS_STEP(hipStreamWaitEvent(s, fk->join[c], 0), "join wait");
        }
    } else {
        VS_STEP(launch_surrogate(g, s), "surrogate");
    }
    // what the plain estimator still needs, after the surrogate's decisions
    VS_STEP(launch_pyr_fused(g, PYR_AFTER, s), "pyr_fused");
    for (int l = 0; l + 1 < levels; ++l) VS_STEP(launch_pyr_down(g, l, PYR_AFTER, s), "pyr_down");
    for (int l = levels - 1; l >= 0; --l) {
        VS_STEP(launch_lk(g, l, s), "flow");
        VS_STEP(launch_var(g, l, s), "variational flow");
    }
    if (ev) VS_STEP(hipEventRecord(ev[3], s), "hipEventRecord");
    VS_STEP(launch_blend(g, s), "blend");
    if (pre) VS_STEP(hipMemcpyAsync(pre, pano, pano_bytes, hipMemcpyDeviceToDevice, s), "pano_pre copy");
    if (ev) VS_STEP(hipEventRecord(ev[4], s), "hipEventRecord");
    VS_STEP(launch_balance_lut(g, s), "balance lut");
    VS_STEP(launch_balance_apply(g, s), "balance apply");
    if (ev) {
        VS_STEP(hipEventRecord(ev[5], s), "hipEventRecord");
        VS_STEP(hipEventRecord(ev[6], s), "hipEventRecord");
    }
#undef VS_STEP
    return hipSuccess;
}

Group single(vs_ctx* c)
{
    Group g;
    std::memset(&g, 0, sizeof g);
    g.n = 1;
    g.dp[0] = c->dp;
    g.hp[0] = &c->hp;
    g.net[0] = c->surr_loaded ? &c->net : nullptr;
    return g;
}

}  // namespace

extern "C" {

vs_status vs_stitch(vs_ctx* c, const uint8_t* const frames[], const vs_color_state* in, uint8_t* pano,
                    vs_color_state* out, vs_frame_info* info, void* stream)
{
    if (!c || !frames || !pano) return VS_E_INVAL;
    if (c->sticky) return VS_E_DEVICE;
    const DevPlan& h = c->hp;
    FrameIO io;
    std::memset(&io, 0, sizeof io);
    io.plan[0] = c->dp;
    io.pano[0] = pano;
    for (int k = 0; k < h.n_cams; ++k) {
        if (!frames[k]) return fail(c, VS_E_INVAL, "null frame pointer");
        io.frame[0][k] = frames[k];
    }
    hipStream_t s = (hipStream_t)stream;
    if (in) {
        if (check_state(c, in) != VS_OK) return fail(c, VS_E_STATE, "colour state version / size / pair count mismatch");
        VS_CHECK(hipStreamSynchronize(s), "hipStreamSynchronize");
        VS_CHECK(hipMemcpy(h.state, in, sizeof *in, hipMemcpyHostToDevice), "hipMemcpy state");
    }
    hipEvent_t* ev = nullptr;
    if (c->timing) {
        const int i = c->next_slot;
        c->next_slot = (i + 1) % vs_ctx::kSlots;
        vs_status hs = harvest_slot(c, i);  // a frame kSlots frames old: long finished
        if (hs != VS_OK) return hs;
        ev = c->ev[i];
        c->slot_used[i] = 1;
    }
    VS_CHECK(launch_set_io(io, 1, h.n_pairs, s), "set io");
    const char* where = "";
    hipError_t e = enqueue_frame(single(c), s, ev, c->pano_pre, pano, (size_t)h.canvas_h * h.pano_pitch, &where);
    if (e != hipSuccess) return dev_fail(c, e, where);
    if (out || info) {
        VS_CHECK(hipStreamSynchronize(s), "hipStreamSynchronize");
        if (out) VS_CHECK(hipMemcpy(out, h.state, sizeof *out, hipMemcpyDeviceToHost), "hipMemcpy state");
        if (info) {
            Results r;
            vs_color_state st;
            VS_CHECK(hipMemcpy(&r, h.res, sizeof r, hipMemcpyDeviceToHost), "hipMemcpy results");
            VS_CHECK(hipMemcpy(&st, h.state, sizeof st, hipMemcpyDeviceToHost), "hipMemcpy state");
            std::memset(info, 0, sizeof *info);
            std::memcpy(info->Mk, r.Mk, sizeof info->Mk);
            std::memcpy(info->Mpair, r.Mpair, sizeof info->Mpair);
            std::memcpy(info->flags, r.flags, sizeof info->flags);
            std::memcpy(info->quant, r.quant, sizeof info->quant);
            std::memcpy(info->mbar, r.mbar, sizeof info->mbar);
            info->frames_seen = st.frames_seen;
            const bool surr = h.use_flow && h.flow_mode != VS_FLOW_PLAIN;
            for (int p = 0; p < VS_MAX_PAIRS; ++p) {
                info->surr_ok[p] = surr && p < h.n_pairs ? r.surr_ok[p] : 0;
                info->fb_err[p] = surr && p < h.n_pairs && r.fb[p][1] > 0
                                      ? (float)((double)r.fb[p][0] / 256.0 / (double)r.fb[p][1])
                                      : -1.0f;
            }
        }
    }
    return VS_OK;
}

vs_status vs_set_flow_variant(vs_ctx* c, int level, int variant)
{
    if (!c || level < 0 || level >= c->hp.levels) return VS_E_INVAL;
    if (c->sticky) return VS_E_DEVICE;
    if (!(variant == 0 || ((variant & 7) >= 1 && (variant & 7) <= 4 && (variant & ~31) == 0))) return VS_E_INVAL;
    if (variant > 0 && c->hp.lk_radius != LK_R_MAX) return fail(c, VS_E_UNSUPPORTED, "9x9 kernel needs lk_radius 4");
    if (variant == 0 && c->hp.lk_qcap[level] > 0) {
        // the generic kernel finishes every pixel itself; nothing else changes
    }
    if (variant > 0 && c->hp.lk_qcap[level] == 0) return fail(c, VS_E_UNSUPPORTED, "no deferral queue for this level");
    VS_CHECK(hipDeviceSynchronize(), "hipDeviceSynchronize");
    set_lk_tiles(c->hp, level, variant);
    VS_CHECK(band_tiles(c, level), "flow tiles");
    VS_CHECK(hipMemcpy(c->dp, &c->hp, sizeof(DevPlan), hipMemcpyHostToDevice), "hipMemcpy plan");
    c->gen += 1;
    return VS_OK;
}

// ---------------------------------------------------------------------------
// The learned surrogate: weights and flow mode
// ---------------------------------------------------------------------------

vs_status vs_load_weights(vs_ctx* c, const void* blob, size_t nbytes)
{
    if (!c || !blob) return VS_E_INVAL;
    if (c->sticky) return VS_E_DEVICE;
    DevPlan& h = c->hp;
    if (!h.use_flow || h.levels <= SURR_LEVEL)
        return fail(c, VS_E_UNSUPPORTED, "the surrogate needs flow = 1 and lk_levels >= 3");
    // header
    const uint8_t* b = (const uint8_t*)blob;
    uint32_t version = 0, nl = 0;
    float alpha = 0.0f;
    if (nbytes < 16 || std::memcmp(b, "VSNN", 4) != 0) return fail(c, VS_E_INVAL, "not a surrogate weight file");
    std::memcpy(&version, b + 4, 4);
    std::memcpy(&nl, b + 8, 4);
    std::memcpy(&alpha, b + 12, 4);
    if (version != 1 || nl < 1 || nl > SURR_MAX_LAYERS || !std::isfinite(alpha))
        return fail(c, VS_E_INVAL, "weight file: version / layer count / slope");
    SurrNet net;
    std::memset(&net, 0, sizeof net);
    net.nl = (int)nl;
    net.alpha = alpha;
    size_t off = 16;
    if (nbytes < off + 8 * (size_t)nl) return fail(c, VS_E_INVAL, "weight file truncated");
    for (int l = 0; l < net.nl; ++l) {
        uint32_t ci, co;
        std::memcpy(&ci, b + off, 4);
        std::memcpy(&co, b + off + 4, 4);
        off += 8;
        const bool shape = (ci == 16 && co == 32) || (ci == 32 && co == 32) || (ci == 32 && co == 16) ||
                           (ci == 16 && co == 16);
        if (!shape || (l == 0 && ci != 16) || (l > 0 && (int)ci != net.co[l - 1]) || (l == net.nl - 1 && co != 16) ||
            nl < 2)
            return fail(c, VS_E_INVAL, "weight file: unsupported layer shapes");
        net.ci[l] = (int)ci;
        net.co[l] = (int)co;
    }
    size_t wbytes[SURR_MAX_LAYERS], woff[SURR_MAX_LAYERS], dev_w = 0;
    for (int l = 0; l < net.nl; ++l) {
        wbytes[l] = (size_t)net.co[l] * 9 * net.ci[l] * 2 + (size_t)net.co[l] * 4;
        woff[l] = off;
        off += wbytes[l];
        dev_w += align_up(wbytes[l], 256);
    }
    if (off != nbytes) return fail(c, VS_E_INVAL, "weight file size");
    // one image per field at the surrogate's level
    nn::ImgTable& T = net.tbl;
    const int nf = 2 * h.n_pairs;
    T.n = nf;
    T.pix_off[0] = 0;
    T.tile_off[0] = 0;
    for (int f = 0; f < nf; ++f) {
        const int p = f >> 1;
        T.w[f] = h.lw[p][SURR_LEVEL];
        T.h[f] = h.lh[p][SURR_LEVEL];
        const long np = (long)T.w[f] * T.h[f];
        T.pix_off[f + 1] = T.pix_off[f] + np;
        T.tile_off[f + 1] = T.tile_off[f] + (int)((np + 63) / 64);
    }
    for (int i = nf + 1; i <= nn::MAXI; ++i) {
        T.pix_off[i] = T.pix_off[nf];
        T.tile_off[i] = T.tile_off[nf];
    }
    const size_t npx = (size_t)T.pix_off[nf];
    const size_t nblk = (size_t)h.strip_off[h.n_pairs] * SURR_UP_SUB;
    // the first layer's weights on the two non-zero input channels, k = 2 tap + channel
    std::vector<uint16_t> w0p((size_t)net.co[0] * 32, 0);
    for (int co = 0; co < net.co[0]; ++co)
        for (int tap = 0; tap < 9; ++tap)
            for (int ch = 0; ch < 2; ++ch)
                std::memcpy(&w0p[(size_t)co * 32 + 2 * tap + ch], b + woff[0] + (((size_t)co * 9 + tap) * 16 + ch) * 2, 2);
    const size_t o_w0p = dev_w, o_h0 = align_up(o_w0p + w0p.size() * 2, 256), o_h1 = align_up(o_h0 + npx * 32 * 2, 256),
                 o_pred = align_up(o_h1 + npx * 32 * 2, 256), o_part = align_up(o_pred + npx * 2 * 4, 256),
                 total = align_up(o_part + nblk * 16, 256);
    VS_CHECK(hipDeviceSynchronize(), "hipDeviceSynchronize");
    void* mem = nullptr;
    if (hipMalloc(&mem, total) != hipSuccess) return fail(c, VS_E_NOMEM, "surrogate buffers");
    uint8_t* base = (uint8_t*)mem;
    size_t wo = 0;
    hipError_t e = hipSuccess;
    for (int l = 0; l < net.nl && e == hipSuccess; ++l) {
        const size_t nw = (size_t)net.co[l] * 9 * net.ci[l];
        net.w[l] = (const uint16_t*)(base + wo);
        net.b[l] = (const float*)(base + wo + nw * 2);
        e = hipMemcpy(base + wo, b + woff[l], wbytes[l], hipMemcpyHostToDevice);
        wo += align_up(wbytes[l], 256);
    }
    if (e == hipSuccess) e = hipMemcpy(base + o_w0p, w0p.data(), w0p.size() * 2, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(base + o_h0, 0, total - o_h0);
    if (e != hipSuccess) {
        (void)hipFree(mem);
        return dev_fail(c, e, "surrogate upload");
    }
    net.w0p = (const uint16_t*)(base + o_w0p);
    net.h[0] = (uint16_t*)(base + o_h0);
    net.h[1] = (uint16_t*)(base + o_h1);
    net.pred = (float*)(base + o_pred);
    net.part = (unsigned long long*)(base + o_part);
    if (c->surr_mem) (void)hipFree(c->surr_mem);
    c->surr_mem = mem;
    c->net = net;
    c->surr_loaded = 1;
    for (int f = 0; f <= nf; ++f) h.surr_pix[f] = T.pix_off[f];
    h.surr_pred = net.pred;
    h.surr_part = net.part;
    VS_CHECK(hipMemcpy(c->dp, &h, sizeof(DevPlan), hipMemcpyHostToDevice), "hipMemcpy plan");
    c->gen += 1;
    return VS_OK;
}

vs_status vs_set_flow_mode(vs_ctx* c, int mode, float fb_tau_px)
{
    if (!c || mode < VS_FLOW_PLAIN || mode > VS_FLOW_SURROGATE_FALLBACK || !(fb_tau_px >= 0.0f) || fb_tau_px > 1e6f)
        return VS_E_INVAL;
    if (c->sticky) return VS_E_DEVICE;
    if (mode != VS_FLOW_PLAIN && !c->surr_loaded) return fail(c, VS_E_UNSUPPORTED, "no surrogate weights loaded");
    VS_CHECK(hipDeviceSynchronize(), "hipDeviceSynchronize");
    c->hp.flow_mode = mode;
    c->hp.fb_tau_fix = (unsigned long long)std::llround((double)fb_tau_px * 256.0);
    VS_CHECK(hipMemcpy(c->dp, &c->hp, sizeof(DevPlan), hipMemcpyHostToDevice), "hipMemcpy plan");
    c->gen += 1;
    return VS_OK;
}

vs_status vs_get_flow_variant(const vs_ctx* c, int32_t variant[VS_MAX_LEVELS])
{
    if (!c || !variant) return VS_E_INVAL;
    for (int l = 0; l < VS_MAX_LEVELS; ++l) variant[l] = l < c->hp.levels ? c->hp.lk_P[l] : 0;
    return VS_OK;
}

// ---------------------------------------------------------------------------
// Tuning records
// ---------------------------------------------------------------------------

vs_status vs_tune_key_of(const vs_ctx* c, vs_tune_key* k)
{
    if (!c || !k) return VS_E_INVAL;
    std::memset(k, 0, sizeof *k);
    std::memcpy(k->arch, c->arch, sizeof k->arch);
    k->n_cams = c->hp.n_cams;
    k->canvas_w = c->hp.canvas_w;
    k->canvas_h = c->hp.canvas_h;
    k->lk_levels = c->hp.levels;
    k->lk_radius = c->hp.lk_radius;
    return VS_OK;
}

vs_status vs_get_tuning(const vs_ctx* c, vs_tune_entry* e)
{
    if (!c || !e) return VS_E_INVAL;
    std::memset(e, 0, sizeof *e);
    for (int l = 0; l < c->hp.levels; ++l) e->flow_variant[l] = c->hp.lk_P[l];
    e->pyr_tile_rows = c->hp.levels >= 3 ? c->hp.pyrf_ty : 0;
    return VS_OK;
}

vs_status vs_tune_put(const vs_tune_key* k, const vs_tune_entry* e)
{
    if (!k || !e || !tune_rec_ok(*k, *e)) return VS_E_INVAL;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    tune_put_locked(*k, *e);
    return VS_OK;
}

vs_status vs_tune_get(const vs_tune_key* k, vs_tune_entry* e)
{
    if (!k || !e) return VS_E_INVAL;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (const TuneRec& r : g_tune)
        if (tune_key_eq(r.k, *k)) {
            *e = r.e;
            return VS_OK;
        }
    return VS_E_UNSUPPORTED;
}

vs_status vs_tune_clear(void)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune.clear();
    return VS_OK;
}

vs_status vs_tune_save(const char* path)
{
    if (!path) return VS_E_INVAL;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    FILE* f = std::fopen(path, "w");
    if (!f) return VS_E_INVAL;
    bool ok = true;
    for (const TuneRec& r : g_tune) {
        ok = ok && std::fprintf(f, "vstune1 %s %d %d %d %d %d", r.k.arch, r.k.n_cams, r.k.canvas_w, r.k.canvas_h,
                                r.k.lk_levels, r.k.lk_radius) > 0;
        for (int l = 0; l < VS_MAX_LEVELS; ++l) ok = ok && std::fprintf(f, " %d", r.e.flow_variant[l]) > 0;
        ok = ok && std::fprintf(f, " %d\n", r.e.pyr_tile_rows) > 0;
    }
    ok = (std::fclose(f) == 0) && ok;
    return ok ? VS_OK : VS_E_INVAL;
}

vs_status vs_tune_load(const char* path)
{
    if (!path) return VS_E_INVAL;
    FILE* f = std::fopen(path, "r");
    if (!f) return VS_E_INVAL;
    std::vector<TuneRec> recs;
    char line[512];
    bool ok = true;
    while (ok && std::fgets(line, sizeof line, f)) {
        if (line[0] == '\n' || line[0] == '#') continue;
        TuneRec r;
        std::memset(&r, 0, sizeof r);
        char tag[16] = {}, arch[32] = {};
        int v[VS_MAX_LEVELS] = {}, rows = 0, used = 0;
        static_assert(VS_MAX_LEVELS == 6, "record format");
        const int got = std::sscanf(line, "%15s %31s %d %d %d %d %d %d %d %d %d %d %d %d %n", tag, arch, &r.k.n_cams,
                                    &r.k.canvas_w, &r.k.canvas_h, &r.k.lk_levels, &r.k.lk_radius, &v[0], &v[1], &v[2],
                                    &v[3], &v[4], &v[5], &rows, &used);
        ok = got == 14 && std::strcmp(tag, "vstune1") == 0 && line[used] == 0;
        std::memcpy(r.k.arch, arch, sizeof arch);
        for (int l = 0; l < VS_MAX_LEVELS; ++l) r.e.flow_variant[l] = v[l];
        r.e.pyr_tile_rows = rows;
        ok = ok && tune_rec_ok(r.k, r.e);
        if (ok) recs.push_back(r);
    }
    std::fclose(f);
    if (!ok) return VS_E_INVAL;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (const TuneRec& r : recs) tune_put_locked(r.k, r.e);
    return VS_OK;
}


// ---------------------------------------------------------------------------
// Batches: several contexts (uneven rigs / resolutions) stitched by one graph
// ---------------------------------------------------------------------------

}  // extern "C"

struct vs_batch {
    int n = 0;
    vs_ctx* ctx[MAXB] = {};
    uint32_t gen[MAXB] = {};   // each context's generation at capture
    Group g;
    hipStream_t cap = nullptr;
    Fork fk = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string err;
};

namespace {

void drop_graph(vs_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Capture the group's frame sequence once; replays read this frame's buffers
// from the device plans (k_set_io runs before every replay, outside the graph).
vs_status capture(vs_batch* b)
{
    drop_graph(b);
    for (int c = 0; c < b->n; ++c) {
        b->g.net[c] = b->ctx[c]->surr_loaded ? &b->ctx[c]->net : nullptr;
        b->gen[c] = b->ctx[c]->gen;
    }
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        b->err = std::string("hipStreamBeginCapture: ") + hipGetErrorString(e);
        return VS_E_DEVICE;
    }
    const char* where = "";
    hipError_t e1 = enqueue_frame(b->g, b->cap, nullptr, nullptr, nullptr, 0, &where, &b->fk);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(b->cap, &graph);
    if (e1 != hipSuccess || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        b->err = std::string("capture: ") + where + ": " + hipGetErrorString(e1 != hipSuccess ? e1 : e);
        return VS_E_DEVICE;
    }
    b->graph = graph;
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        b->err = std::string("hipGraphInstantiate: ") + hipGetErrorString(e);
        return VS_E_DEVICE;
    }
    return VS_OK;
}

vs_status set_variant_all(vs_batch* b, int level, int variant)
{
    for (int c = 0; c < b->n; ++c) {
        vs_status st = vs_set_flow_variant(b->ctx[c], level, variant);
        if (st != VS_OK) return st;
    }
    return VS_OK;
}

}  // namespace

extern "C" {

vs_status vs_batch_create(vs_ctx* const ctxs[], int n, vs_batch** out)
{
    if (!out || !ctxs || n < 1 || n > MAXB) return VS_E_INVAL;
    *out = nullptr;
    for (int c = 0; c < n; ++c) {
        if (!ctxs[c]) return VS_E_INVAL;
        if (ctxs[c]->sticky) return VS_E_DEVICE;
        for (int d = 0; d < c; ++d)
            if (ctxs[d] == ctxs[c]) return VS_E_INVAL;
        if (ctxs[c]->hp.levels != ctxs[0]->hp.levels || ctxs[c]->hp.lk_radius != ctxs[0]->hp.lk_radius)
            return VS_E_UNSUPPORTED;
    }
    vs_batch* b = new (std::nothrow) vs_batch();
    if (!b) return VS_E_NOMEM;
    b->n = n;
    std::memset(&b->g, 0, sizeof b->g);
    b->g.n = n;
    for (int c = 0; c < n; ++c) {
        b->ctx[c] = ctxs[c];
        b->g.dp[c] = ctxs[c]->dp;
        b->g.hp[c] = &ctxs[c]->hp;
    }
    // one flow-kernel variant per level for the whole batch (same rule as a
    // single context, applied to the batch's total tile count)
    const DevPlan& h0 = ctxs[0]->hp;
    for (int l = 0; l < h0.levels; ++l) {
        int variant = 0;
        if (h0.lk_radius == LK_R_MAX) {
            int n16 = 0;
            for (int c = 0; c < n; ++c) {
                const DevPlan& h = ctxs[c]->hp;
                for (int f = 0; f < 2 * h.n_pairs; ++f) {
                    const int p = f >> 1;
                    n16 += ((h.lw[p][l] + LKW_TX - 1) / LKW_TX) * ((h.lh[p][l] + 15) / 16);
                }
            }
            variant = default_lk_P(n16, lk_resident_blocks());
        }
        vs_status st = set_variant_all(b, l, variant);
        if (st != VS_OK) {
            delete b;
            return st;
        }
    }
    bool ok = hipStreamCreate(&b->cap) == hipSuccess &&
              hipEventCreateWithFlags(&b->fk.fork, hipEventDisableTiming) == hipSuccess;
    for (int c = 0; c < n && ok; ++c)
        ok = hipStreamCreate(&b->fk.side[c]) == hipSuccess &&
             hipEventCreateWithFlags(&b->fk.join[c], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        vs_batch_destroy(b);
        return VS_E_DEVICE;
    }
    vs_status st = capture(b);
    if (st != VS_OK) {
        vs_batch_destroy(b);
        return st;
    }
    *out = b;
    return VS_OK;
}

vs_status vs_batch_destroy(vs_batch* b)
{
    if (!b) return VS_E_INVAL;
    drop_graph(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (int c = 0; c < MAXB; ++c) {
        if (b->fk.side[c]) (void)hipStreamDestroy(b->fk.side[c]);
        if (b->fk.join[c]) (void)hipEventDestroy(b->fk.join[c]);
    }
    if (b->fk.fork) (void)hipEventDestroy(b->fk.fork);
    delete b;
    return VS_OK;
}

const char* vs_batch_last_error(const vs_batch* b) { return b ? b->err.c_str() : "null batch"; }

vs_status vs_batch_run(vs_batch* b, const uint8_t* const* const frames[], uint8_t* const panos[], void* stream)
{
    if (!b || !frames || !panos || !b->exec) return VS_E_INVAL;
    FrameIO io;
    std::memset(&io, 0, sizeof io);
    for (int c = 0; c < b->n; ++c) {
        if (b->ctx[c]->sticky) return VS_E_DEVICE;
        if (!frames[c] || !panos[c]) return VS_E_INVAL;
        io.plan[c] = b->ctx[c]->dp;
        io.pano[c] = panos[c];
        for (int k = 0; k < b->ctx[c]->hp.n_cams; ++k) {
            if (!frames[c][k]) return VS_E_INVAL;
            io.frame[c][k] = frames[c][k];
        }
    }
    for (int c = 0; c < b->n; ++c)
        if (b->gen[c] != b->ctx[c]->gen) {   // a context changed its launch sequence
            vs_status st = capture(b);
            if (st != VS_OK) return st;
            break;
        }
    hipStream_t s = (hipStream_t)stream;
    int max_pairs = 0;
    for (int c = 0; c < b->n; ++c) max_pairs = std::max(max_pairs, (int)b->ctx[c]->hp.n_pairs);
    hipError_t e = launch_set_io(io, b->n, max_pairs, s);
    if (e == hipSuccess) e = hipGraphLaunch(b->exec, s);
    if (e != hipSuccess) {
        b->err = std::string("batch run: ") + hipGetErrorString(e);
        for (int c = 0; c < b->n; ++c) b->ctx[c]->sticky = 1;
        return VS_E_DEVICE;
    }
    return VS_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: per pyramid level, time each flow-kernel variant on real frames
// and keep the fastest.  The colour state is saved and restored around it.
// ---------------------------------------------------------------------------

vs_status vs_batch_autotune(vs_batch* b, const uint8_t* const* const frames[], uint8_t* const panos[], int reps,
                            float ms_out[VS_MAX_LEVELS][VS_FLOW_VARIANTS], int32_t choice[VS_MAX_LEVELS])
{
    if (!b || reps < 1 || !choice) return VS_E_INVAL;
    const int levels = b->ctx[0]->hp.levels;
    if (b->ctx[0]->hp.lk_radius != LK_R_MAX) {
        for (int l = 0; l < VS_MAX_LEVELS; ++l) choice[l] = 0;
        return VS_OK;
    }
    std::vector<vs_color_state> saved(b->n);
    for (int c = 0; c < b->n; ++c) {
        vs_status st = vs_state_get(b->ctx[c], &saved[c]);
        if (st != VS_OK) return st;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return VS_E_DEVICE;
    const int variants[VS_FLOW_VARIANTS] = {1, 2, 3, 4, 9, 10, 11, 12, 25, 26, 27, 28};
    vs_status st = VS_OK;
    for (int l = 0; l < levels && st == VS_OK; ++l) {
        float best = 1e30f;
        int best_v = b->ctx[0]->hp.lk_P[l];
        for (int vi = 0; vi < VS_FLOW_VARIANTS && st == VS_OK; ++vi) {
            st = set_variant_all(b, l, variants[vi]);
            if (st == VS_OK) st = capture(b);
            if (st != VS_OK) break;
            st = vs_batch_run(b, frames, panos, nullptr);   // warm
            if (st != VS_OK) break;
            (void)hipEventRecord(e0, nullptr);
            for (int r = 0; r < reps && st == VS_OK; ++r) st = vs_batch_run(b, frames, panos, nullptr);
            (void)hipEventRecord(e1, nullptr);
            if (hipEventSynchronize(e1) != hipSuccess) st = VS_E_DEVICE;
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            ms /= (float)reps;
            if (ms_out) ms_out[l][vi] = ms;
            if (ms < best) {
                best = ms;
                best_v = variants[vi];
            }
        }
        if (st == VS_OK) st = set_variant_all(b, l, best_v);
        choice[l] = best_v;
    }
    for (int l = levels; l < VS_MAX_LEVELS; ++l) choice[l] = 0;
    // the fused pyramid's tile height, every context alike
    bool pyr = levels >= 3;
    for (int c = 0; c < b->n; ++c) pyr = pyr && b->ctx[c]->hp.use_flow && b->ctx[c]->prm.pyr_tile_rows == 0;
    if (pyr && st == VS_OK) {
        float best = 1e30f;
        int best_rows = b->ctx[0]->hp.pyrf_ty;
        for (const int rows : {8, 16}) {
            for (int c = 0; c < b->n && st == VS_OK; ++c) {
                vs_ctx* x = b->ctx[c];
                set_pyr_rows(x->hp, rows);
                if (hipMemcpy(x->dp, &x->hp, sizeof(DevPlan), hipMemcpyHostToDevice) != hipSuccess) st = VS_E_DEVICE;
                x->gen += 1;
            }
            if (st == VS_OK) st = capture(b);
            if (st == VS_OK) st = vs_batch_run(b, frames, panos, nullptr);   // warm
            if (st != VS_OK) break;
            (void)hipEventRecord(e0, nullptr);
            for (int r = 0; r < reps && st == VS_OK; ++r) st = vs_batch_run(b, frames, panos, nullptr);
            (void)hipEventRecord(e1, nullptr);
            if (hipEventSynchronize(e1) != hipSuccess) st = VS_E_DEVICE;
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms / (float)reps < best) {
                best = ms / (float)reps;
                best_rows = rows;
            }
        }
        for (int c = 0; c < b->n && st == VS_OK; ++c) {
            vs_ctx* x = b->ctx[c];
            set_pyr_rows(x->hp, best_rows);
            if (hipMemcpy(x->dp, &x->hp, sizeof(DevPlan), hipMemcpyHostToDevice) != hipSuccess) st = VS_E_DEVICE;
            x->gen += 1;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == VS_OK) st = capture(b);
    for (int c = 0; c < b->n && st == VS_OK; ++c) st = vs_state_set(b->ctx[c], &saved[c]);
    // record every context's choice for contexts created later on this device
    for (int c = 0; c < b->n && st == VS_OK; ++c) {
        vs_tune_key k;
        vs_tune_entry te;
        if (vs_tune_key_of(b->ctx[c], &k) == VS_OK && vs_get_tuning(b->ctx[c], &te) == VS_OK) (void)vs_tune_put(&k, &te);
    }
    return st;
}


// ---------------------------------------------------------------------------
// The plain estimator on caller image pairs (labels for the surrogate)
// ---------------------------------------------------------------------------

}  // extern "C"

namespace vs {

// Plan of a plain-flow context on one w x h luma pair: a single "pair" whose
// strip is the whole image, template = camera j, moving = camera i, every
// pixel in the flow domain.  Fills the sizes and tile tables of d and the
// workspace offsets; false on invalid sizes or parameters.
bool flow_plan(int w, int h, const vs_params& P, DevPlan& d, FlowLayout& L)
{
    if (w < 2 || h < 2 || w > 65535 || h > 65535) return false;
    if (P.lk_levels < 1 || P.lk_levels > VS_MAX_LEVELS || P.lk_iters < 0 || P.lk_radius < 0 ||
        P.lk_radius > LK_R_MAX || !std::isfinite(P.lk_lambda) || !(P.flow == 1 || P.flow == 2) || !var_params_ok(P))
        return false;
    std::memset(&d, 0, sizeof d);
    std::memset(&L, 0, sizeof L);
    d.n_cams = 2;
    d.n_pairs = 1;
    d.levels = P.lk_levels;
    d.use_flow = P.flow;
    d.var_alpha = P.var_alpha;
    d.var_gamma = P.var_gamma;
    d.var_outer = P.var_outer;
    d.var_inner = P.var_inner;
    d.lk_radius = P.lk_radius;
    d.lk_iters = P.lk_iters;
    d.lk_lambda = P.lk_lambda;
    d.pj[0] = 0;
    d.pi[0] = 1;
    d.sw[0] = w;
    d.sh[0] = h;
    int ww = w, hh = h;
    for (int l = 0; l < d.levels; ++l) {
        d.lw[0][l] = ww;
        d.lh[0][l] = hh;
        ww = (ww + 1) / 2;
        hh = (hh + 1) / 2;
    }
    for (int l = 0; l < d.levels; ++l) {
        d.pyr_off[l][0] = 0;
        for (int fl = 0; fl < 2; ++fl) {
            d.pyr_tx[l][fl] = (d.lw[0][l] + PYR_TX - 1) / PYR_TX;
            d.pyr_off[l][fl + 1] = d.pyr_off[l][fl] + d.pyr_tx[l][fl] * ((d.lh[0][l] + PYR_TY - 1) / PYR_TY);
        }
        const int n16 = 2 * ((d.lw[0][l] + LKW_TX - 1) / LKW_TX) * ((d.lh[0][l] + 15) / 16);
        set_lk_tiles(d, l, P.lk_radius == LK_R_MAX ? default_lk_P(n16, lk_resident_blocks()) : 0);
    }
    size_t off = 0;
    for (int l = 0; l < d.levels; ++l) {
        const size_t n = (size_t)d.lw[0][l] * d.lh[0][l];
        L.need[l] = off;
        off = align_up(off + n, 256);
        for (int k = 0; k < 2; ++k) {
            L.pyr[k][l] = off;
            off = align_up(off + n * 4, 256);
            L.flow[k][l] = off;
            off = align_up(off + n * 8, 256);
        }
        d.lk_qcap[l] = d.lk_P[l] > 0 ? (int32_t)(2 * n) : 0;
        L.queue[l] = off;
        off = align_up(off + (size_t)d.lk_qcap[l] * 16, 256);
    }
    if (d.use_flow == 2) {
        L.var = off;
        off = align_up(off + var_layout(d, nullptr), 256);
    }
    L.acc = off;
    off = align_up(off + sizeof(Accum), 256);
    L.res = off;
    off = align_up(off + sizeof(Results), 256);
    L.state = off;
    off = align_up(off + sizeof(vs_color_state), 256);
    L.bytes = off;
    return true;
}

// Point the plan's buffers into a workspace of L.bytes at base.
void flow_bind(DevPlan& d, const FlowLayout& L, uint8_t* base)
{
    for (int l = 0; l < d.levels; ++l) {
        d.need[0][l] = base + L.need[l];
        d.lk_queue[l] = (uint4*)(base + L.queue[l]);
        for (int k = 0; k < 2; ++k) {
            d.pyr[0][k][l] = (float*)(base + L.pyr[k][l]);
            d.flow[0][k][l] = (float2*)(base + L.flow[k][l]);
        }
    }
    d.acc = (Accum*)(base + L.acc);
    d.res = (Results*)(base + L.res);
    d.state = (vs_color_state*)(base + L.state);
    if (d.use_flow == 2) var_layout(d, base + L.var);
}

// Mark every pixel of every level as flow domain (a fill kernel, no memset node).
hipError_t flow_domain_fill(const DevPlan& d, hipStream_t s)
{
    hipError_t e = hipSuccess;
    for (int l = 0; l < d.levels && e == hipSuccess; ++l)
        e = launch_fill_u8(d.need[0][l], (size_t)d.lw[0][l] * d.lh[0][l], 1, s);
    return e;
}

// One run of the plain estimator: the pair into level 0, the pyramids, the
// flow coarse to fine, the level-0 flows out (every step on stream s).
hipError_t flow_run(const DevPlan& d, DevPlan* dp, const float* yt, const float* ym, float* flow_tm,
                    float* flow_mt, hipStream_t s)
{
    const size_t n = (size_t)d.sw[0] * d.sh[0];
    Group g;
    std::memset(&g, 0, sizeof g);
    g.n = 1;
    g.dp[0] = dp;
    g.hp[0] = &d;
    hipError_t e = hipMemcpyAsync(d.pyr[0][0][0], yt, n * 4, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d.pyr[0][1][0], ym, n * 4, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = launch_zero(g, s);
    for (int l = 0; l + 1 < d.levels && e == hipSuccess; ++l) e = launch_pyr_down(g, l, PYR_ALL, s);
    for (int l = d.levels - 1; l >= 0 && e == hipSuccess; --l) {
        e = launch_lk(g, l, s);
        if (e == hipSuccess) e = launch_var(g, l, s);
    }
    if (e == hipSuccess && flow_tm) e = hipMemcpyAsync(flow_tm, d.flow[0][0][0], n * 8, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && flow_mt) e = hipMemcpyAsync(flow_mt, d.flow[0][1][0], n * 8, hipMemcpyDeviceToDevice, s);
    return e;
}

}  // namespace vs

struct vs_flow {
    DevPlan hp;
    DevPlan* dp = nullptr;
    void* arena = nullptr;
};

extern "C" {

vs_status vs_flow_destroy(vs_flow* f)
{
    if (!f) return VS_E_INVAL;
    if (f->arena) (void)hipFree(f->arena);
    if (f->dp) (void)hipFree(f->dp);
    delete f;
    return VS_OK;
}

vs_status vs_flow_create(int w, int h, const vs_params* prm, vs_flow** out)
{
    if (!out) return VS_E_INVAL;
    *out = nullptr;
    vs_params P;
    if (prm) P = *prm;
    else vs_default_params(&P);
    vs_flow* f = new (std::nothrow) vs_flow();
    if (!f) return VS_E_NOMEM;
    FlowLayout L;
    if (!flow_plan(w, h, P, f->hp, L)) {
        delete f;
        return VS_E_INVAL;
    }
    if (hipMalloc(&f->arena, L.bytes) != hipSuccess || hipMalloc((void**)&f->dp, sizeof(DevPlan)) != hipSuccess) {
        vs_flow_destroy(f);
        return VS_E_NOMEM;
    }
    flow_bind(f->hp, L, (uint8_t*)f->arena);
    bool ok = hipMemset(f->arena, 0, L.bytes) == hipSuccess;
    ok = ok && flow_domain_fill(f->hp, nullptr) == hipSuccess;   // the whole image is the flow domain
    ok = ok && hipMemcpy(f->dp, &f->hp, sizeof f->hp, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipDeviceSynchronize() == hipSuccess;
    if (!ok) {
        vs_flow_destroy(f);
        return VS_E_DEVICE;
    }
    *out = f;
    return VS_OK;
}

vs_status vs_flow_run(vs_flow* f, const float* yt, const float* ym, float* flow_tm, float* flow_mt, void* stream)
{
    if (!f || !yt || !ym) return VS_E_INVAL;
    return flow_run(f->hp, f->dp, yt, ym, flow_tm, flow_mt, (hipStream_t)stream) == hipSuccess ? VS_OK
                                                                                              : VS_E_DEVICE;
}

vs_status vs_flow_only(vs_ctx* c, const uint8_t* strip_i, const uint8_t* strip_j, int w, int h, float* flow_ij,
                       float* flow_ji, void* stream)
{
    if (!c || !strip_i || !strip_j || w < 1 || h < 1) return VS_E_INVAL;
    if (c->sticky) return VS_E_DEVICE;
    if (!c->fo || c->fo_w != w || c->fo_h != h) {
        // a plain-flow context of this size with the stitch context's parameters
        VS_CHECK(hipDeviceSynchronize(), "hipDeviceSynchronize");
        if (c->fo) (void)vs_flow_destroy(c->fo);
        if (c->fo_luma) (void)hipFree(c->fo_luma);
        c->fo = nullptr;
        c->fo_luma = nullptr;
        c->fo_w = c->fo_h = 0;
        const vs_status st = vs_flow_create(w, h, &c->prm, &c->fo);
        if (st != VS_OK) return fail(c, st, "vs_flow_only: strip size");
        if (hipMalloc((void**)&c->fo_luma, 2 * (size_t)w * h * sizeof(float)) != hipSuccess) {
            (void)vs_flow_destroy(c->fo);
            c->fo = nullptr;
            return fail(c, VS_E_NOMEM, "vs_flow_only: luma buffers");
        }
        c->fo_w = w;
        c->fo_h = h;
    }
    hipStream_t s = (hipStream_t)stream;
    const size_t n = (size_t)w * h;
    float* yj = c->fo_luma;
    float* yi = c->fo_luma + n;
    VS_CHECK(launch_luma_rgb(strip_j, n, yj, s), "luma launch");
    VS_CHECK(launch_luma_rgb(strip_i, n, yi, s), "luma launch");
    // flow_ij: template camera j, moving camera i (and the reverse)
    return vs_flow_run(c->fo, yj, yi, flow_ij, flow_ji, stream);
}

vs_status vs_flow_level(vs_flow* f, int level, float* yt, float* ym, int32_t* w_out, int32_t* h_out, void* stream)
{
    if (!f || level < 0 || level >= f->hp.levels) return VS_E_INVAL;
    const DevPlan& d = f->hp;
    if (w_out) *w_out = d.lw[0][level];
    if (h_out) *h_out = d.lh[0][level];
    const size_t n = (size_t)d.lw[0][level] * d.lh[0][level] * 4;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (yt) e = hipMemcpyAsync(yt, d.pyr[0][0][level], n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && ym) e = hipMemcpyAsync(ym, d.pyr[0][1][level], n, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? VS_OK : VS_E_DEVICE;
}

vs_status vs_debug_tap(vs_ctx* c, int tap, int p, int sub, void* dst, size_t nbytes)
{
    if (!c || !dst) return VS_E_INVAL;
    if (c->sticky) return VS_E_DEVICE;
    const DevPlan& h = c->hp;
    const bool pair_ok = p >= 0 && p < h.n_pairs;
    const size_t n = pair_ok ? (size_t)h.sw[p] * h.sh[p] : 0;
    auto copy = [&](const void* src, size_t have) -> vs_status {
        if (nbytes != have) return fail(c, VS_E_INVAL, "tap size mismatch");
        VS_CHECK(hipDeviceSynchronize(), "hipDeviceSynchronize");
        VS_CHECK(hipMemcpy(dst, src, have, hipMemcpyDeviceToHost), "hipMemcpy tap");
        return VS_OK;
    };
    // a sum kept in `copies` consecutive copies of `words` 32-bit counters
    auto copy_summed = [&](const uint32_t* src, size_t words, int copies) -> vs_status {
        if (nbytes != words * 4) return fail(c, VS_E_INVAL, "tap size mismatch");
        std::vector<uint32_t> all(words * copies);
        VS_CHECK(hipDeviceSynchronize(), "hipDeviceSynchronize");
        VS_CHECK(hipMemcpy(all.data(), src, all.size() * 4, hipMemcpyDeviceToHost), "hipMemcpy tap");
        uint32_t* d = (uint32_t*)dst;
        for (size_t i = 0; i < words; ++i) {
            uint32_t t = 0;
            for (int k = 0; k < copies; ++k) t += all[(size_t)k * words + i];
            d[i] = t;
        }
        return VS_OK;
    };
    switch (tap) {
    case VS_TAP_STRIP: {
        if (!pair_ok || sub < 0 || sub > 1) return VS_E_INVAL;
        if (nbytes != n * 3) return fail(c, VS_E_INVAL, "tap size mismatch");
        std::string tmp(n * 4, '\0');
        VS_CHECK(hipDeviceSynchronize(), "hipDeviceSynchronize");
        VS_CHECK(hipMemcpy(&tmp[0], h.strip[p] + (size_t)sub * n, n * 4, hipMemcpyDeviceToHost), "hipMemcpy tap");
        const uint32_t* px = (const uint32_t*)tmp.data();
        uint8_t* d = (uint8_t*)dst;
        for (size_t q = 0; q < n; ++q) {
            d[3 * q + 0] = (uint8_t)(px[q] & 255u);
            d[3 * q + 1] = (uint8_t)((px[q] >> 8) & 255u);
            d[3 * q + 2] = (uint8_t)((px[q] >> 16) & 255u);
        }
        return VS_OK;
    }
    case VS_TAP_MASK:
        if (!pair_ok) return VS_E_INVAL;
        return copy(h.mask[p], n);
    case VS_TAP_HIST:
        if (!pair_ok) return VS_E_INVAL;
        return copy_summed(&h.acc->hist[p][0][0][0][0], 2 * 3 * 256, HIST_SPREAD);
    case VS_TAP_LUT:
        if (!pair_ok) return VS_E_INVAL;
        return copy(&h.res->lut[p][0][0], 3 * 256);
    case VS_TAP_MOM:
        if (!pair_ok) return VS_E_INVAL;
        return copy(&h.res->mom[p][0], 16 * 8);
    case VS_TAP_MPAIR:
        return copy(&h.res->Mpair[0][0], (size_t)h.n_pairs * 9 * 8);
    case VS_TAP_MK:
        return copy(&h.res->Mk[0][0], (size_t)h.n_cams * 9 * 4);
    case VS_TAP_FLAGS:
        return copy(&h.res->flags[0], (size_t)h.n_pairs * 4);
    case VS_TAP_PYR: {
        const int cam = sub / 8, l = sub % 8;
        if (!pair_ok || cam < 0 || cam > 1 || l >= h.levels) return VS_E_INVAL;
        return copy(h.pyr[p][cam][l], (size_t)h.lw[p][l] * h.lh[p][l] * 4);
    }
    case VS_TAP_FLOW:
        if (!pair_ok || sub < 0 || sub > 1) return VS_E_INVAL;
        return copy(h.flow[p][sub][0], n * 8);
    case VS_TAP_PANO_PRE:
        if (!c->pano_pre) return fail(c, VS_E_UNSUPPORTED, "pre-balance panorama needs debug_taps = 1");
        return copy(c->pano_pre, (size_t)h.canvas_h * h.pano_pitch);
    case VS_TAP_PANO_HIST:
        return copy_summed(&h.acc->pano_hist[0][0][0], 3 * 256, PANO_SPREAD);
    case VS_TAP_BAL_LUT:
        return copy(&h.res->bal_lut[0][0], 3 * 256);
    case VS_TAP_QUANT:
        return copy(&h.res->quant[0][0], 6 * 4);
    case VS_TAP_MBAR:
        return copy(&h.res->mbar[0][0], 6 * 8);
    case VS_TAP_NEED:
        if (!pair_ok || sub < 0 || sub >= h.levels) return VS_E_INVAL;
        return copy(h.need[p][sub], (size_t)h.lw[p][sub] * h.lh[p][sub]);
    case VS_TAP_DEFERRED:
        if (sub < 0 || sub >= h.levels) return VS_E_INVAL;
        return copy(&h.acc->lk_qn[sub], 4);
    case VS_TAP_SURR_PRED: {
        if (!pair_ok || sub < 0 || sub > 1) return VS_E_INVAL;
        if (!c->surr_loaded) return fail(c, VS_E_UNSUPPORTED, "no surrogate weights loaded");
        const int f = 2 * p + sub;
        const size_t np = (size_t)(h.surr_pix[f + 1] - h.surr_pix[f]);
        return copy(c->net.pred + h.surr_pix[f] * 2, np * 8);
    }
    case VS_TAP_FB:
        return copy(&h.res->fb[0][0], (size_t)h.n_pairs * 16);
    case VS_TAP_SURR_OK:
        return copy(&h.res->surr_ok[0], (size_t)h.n_pairs * 4);
    case VS_TAP_COVER: {
        const size_t npx = (size_t)h.canvas_w * h.canvas_h;
        if (nbytes != npx) return fail(c, VS_E_INVAL, "tap size mismatch");
        std::string bits((size_t)h.canvas_h * h.cover_words * 4, '\0');
        VS_CHECK(hipDeviceSynchronize(), "hipDeviceSynchronize");
        VS_CHECK(hipMemcpy(&bits[0], h.cover, bits.size(), hipMemcpyDeviceToHost), "hipMemcpy tap");
        const uint32_t* w = (const uint32_t*)bits.data();
        uint8_t* d = (uint8_t*)dst;
        for (int y = 0; y < h.canvas_h; ++y)
            for (int x = 0; x < h.canvas_w; ++x)
                d[(size_t)y * h.canvas_w + x] = (uint8_t)((w[(size_t)y * h.cover_words + (x >> 5)] >> (x & 31)) & 1u);
        return VS_OK;
    }
    default:
        return VS_E_INVAL;
    }
}

}  // extern "C"
