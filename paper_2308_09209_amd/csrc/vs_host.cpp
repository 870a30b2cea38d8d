// vs_host.cpp -- host runtime of libvstitch: the C ABI, the rig planner and
// the per-frame launch sequence.  Every step of the frame runs in the
// kernels of vs_kernels.hip; the host only plans once and launches.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "vs_internal.h"

using namespace vs;

struct vs_ctx {
    vs_rig rig;
    vs_params prm;
    DevPlan hp;              // host copy of the device plan (holds device pointers)
    DevPlan* dp = nullptr;   // device copy
    void* arena = nullptr;   // per-frame workspace
    size_t arena_bytes = 0;
    void* plan_mem = nullptr;  // coverage bits + candidates + scan
    uint8_t* pano_pre = nullptr;
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
};

namespace {

const char* kStatus[] = {"ok", "invalid argument", "geometry", "out of memory", "device error",
                         "state mismatch", "unsupported"};

// 3x3 product c = a b, entries ((a_r0 b_0c + a_r1 b_1c) + a_r2 b_2c)
void mat3_mul(const double* a, const double* b, double* c)
{
    double t[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k)
            t[r * 3 + k] = (a[r * 3 + 0] * b[0 * 3 + k] + a[r * 3 + 1] * b[1 * 3 + k]) + a[r * 3 + 2] * b[2 * 3 + k];
    std::memcpy(c, t, sizeof t);
}

// inverse = adjugate / adjugate[8] (last entry exactly 1)
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
    for (int i = 0; i < 9; ++i) inv[i] = adj[i] / adj[8];
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
    delete c;
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
    p->lk_lambda = 1.0f;
    p->balance = 1;
    p->lambda_pct = 5;
    p->debug_taps = 0;
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
        P.lambda_pct > 49 || !(P.ridge >= 0.0) || !std::isfinite(P.lk_lambda))
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
    const size_t scan_bytes = align_up(sizeof(PlanScan), 256);
    hipError_t e = hipMalloc(&c->plan_mem, cover_bytes + cand_bytes + scan_bytes);
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
    PlanScan* dscan = (PlanScan*)((uint8_t*)c->plan_mem + cover_bytes + cand_bytes);
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
    for (int l = 0; l < h.levels; ++l) {
        h.pyr_off[l][0] = 0;
        for (int f = 0; f < 2 * h.n_pairs; ++f) {
            const int p = f >> 1, w = h.lw[p][l], hh = h.lh[p][l];
            h.pyr_tx[l][f] = (w + PYR_TX - 1) / PYR_TX;
            h.pyr_off[l][f + 1] = h.pyr_off[l][f] + h.pyr_tx[l][f] * ((hh + PYR_TY - 1) / PYR_TY);
        }
        // flow kernel: the 9x9-window kernel with 4 px per thread where that still
        // gives >= 1024 blocks, else 1 px per thread; other radii use the generic kernel
        auto tiles = [&](int tx, int ty) {
            int n = 0;
            for (int f = 0; f < 2 * h.n_pairs; ++f) {
                const int p = f >> 1;
                n += ((h.lw[p][l] + tx - 1) / tx) * ((h.lh[p][l] + ty - 1) / ty);
            }
            return n;
        };
        int tx = LK_T, ty = LK_T;
        h.lk_P[l] = 0;
        if (P.lk_radius == LK_R_MAX) {
            h.lk_P[l] = tiles(LKW_TX, 16) >= 1024 ? 4 : 1;
            tx = LKW_TX;
            ty = 4 * h.lk_P[l];
        }
        h.lk_off[l][0] = 0;
        for (int f = 0; f < 2 * h.n_pairs; ++f) {
            const int p = f >> 1, w = h.lw[p][l], hh = h.lh[p][l];
            h.lk_tx[l][f] = (w + tx - 1) / tx;
            h.lk_off[l][f + 1] = h.lk_off[l][f] + h.lk_tx[l][f] * ((hh + ty - 1) / ty);
        }
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
    I.workspace_bytes = c->arena_bytes + cover_bytes + cand_bytes + scan_bytes + sizeof(DevPlan);
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

vs_status vs_stitch(vs_ctx* c, const uint8_t* const frames[], const vs_color_state* in, uint8_t* pano,
                    vs_color_state* out, vs_frame_info* info, void* stream)
{
    if (!c || !frames || !pano) return VS_E_INVAL;
    if (c->sticky) return VS_E_DEVICE;
    const DevPlan& h = c->hp;
    FrameSet fs;
    std::memset(&fs, 0, sizeof fs);
    for (int k = 0; k < h.n_cams; ++k) {
        if (!frames[k]) return fail(c, VS_E_INVAL, "null frame pointer");
        fs.f[k] = frames[k];
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
    if (ev) VS_CHECK(hipEventRecord(ev[0], s), "hipEventRecord");
    VS_CHECK(launch_zero(c->dp, h.acc, s), "zero");
    VS_CHECK(launch_strips(c->dp, h, fs, s), "strips");
    VS_CHECK(launch_lut(c->dp, h, s), "lut");
    VS_CHECK(launch_moments_b(c->dp, h, s), "moments");
    VS_CHECK(launch_solve(c->dp, s), "solve");
    if (ev) VS_CHECK(hipEventRecord(ev[1], s), "hipEventRecord");
    if (h.use_flow) {
        VS_CHECK(launch_pyr0(c->dp, h, s), "pyr0");
        for (int l = 0; l + 1 < h.levels; ++l) VS_CHECK(launch_pyr_down(c->dp, h, l, s), "pyr_down");
    }
    if (ev) VS_CHECK(hipEventRecord(ev[2], s), "hipEventRecord");
    if (h.use_flow)
        for (int l = h.levels - 1; l >= 0; --l) VS_CHECK(launch_lk(c->dp, h, l, s), "flow");
    if (ev) VS_CHECK(hipEventRecord(ev[3], s), "hipEventRecord");
    VS_CHECK(launch_blend(c->dp, h, fs, pano, s), "blend");
    if (c->pano_pre)
        VS_CHECK(hipMemcpyAsync(c->pano_pre, pano, (size_t)h.canvas_h * h.pano_pitch, hipMemcpyDeviceToDevice, s),
                 "hipMemcpyAsync pano_pre");
    if (ev) VS_CHECK(hipEventRecord(ev[4], s), "hipEventRecord");
    VS_CHECK(launch_balance_lut(c->dp, s), "balance lut");
    if (h.balance) VS_CHECK(launch_balance_apply(c->dp, h, pano, s), "balance apply");
    if (ev) {
        VS_CHECK(hipEventRecord(ev[5], s), "hipEventRecord");
        VS_CHECK(hipEventRecord(ev[6], s), "hipEventRecord");
    }
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
        }
    }
    return VS_OK;
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
        return copy(&h.acc->hist[p][0][0][0], sizeof(uint32_t) * 2 * 3 * 256);
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
        return copy(&h.acc->pano_hist[0][0], 3 * 256 * 4);
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
