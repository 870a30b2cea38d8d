// vs_noalloc.hip -- the plain flow estimator of vs_flow_run for callers that
// cannot allocate device memory: its plan and workspace live in one static
// device array per GPU instead of a context's allocations.
#include <cstring>
#include <mutex>

#include "vs_internal.h"

namespace vs {
namespace {

// The workspace every call on a GPU shares: the device plan first, then the
// pyramids, level flows, flow domain, deferred-pixel queues and accumulators
// of one w x h luma pair (the layout of flow_plan).  Kernels never see this
// name: host code passes the address hipGetSymbolAddress returns for the
// current device.
__device__ __align__(256) uint8_t scratch[VS_FLOW_NOALLOC_BYTES];

constexpr int kMaxDevices = 64;
constexpr size_t kPlanBytes = (sizeof(DevPlan) + 255) / 256 * 256;

std::mutex g_mu;
uint8_t* g_base[kMaxDevices];        // scratch's address on each device (null: not looked up yet)
DevPlan g_plan[kMaxDevices];         // the plan last uploaded to each device
bool g_plan_ok[kMaxDevices];

// The plan reaches the device as kernel arguments, 2 KB per launch: no host
// buffer has to outlive the call and no copy node depends on pageable memory.
struct Words {
    uint32_t v[512];
};
static_assert(sizeof(DevPlan) % 4 == 0, "the plan is copied in 32-bit words");

__global__ __launch_bounds__(256) void k_put_words(uint32_t* __restrict__ dst, const Words w, int n)
{
    for (int i = threadIdx.x; i < n; i += 256) dst[i] = w.v[i];
}

hipError_t upload_plan(const DevPlan& h, uint8_t* base, hipStream_t s)
{
    const uint32_t* src = (const uint32_t*)&h;
    const int total = (int)(sizeof(DevPlan) / 4);
    for (int o = 0; o < total; o += 512) {
        Words w;
        const int n = total - o < 512 ? total - o : 512;
        std::memcpy(w.v, src + o, (size_t)n * 4);
        hipLaunchKernelGGL(k_put_words, dim3(1), dim3(256), 0, s, (uint32_t*)base + o, w, n);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace
}  // namespace vs

using namespace vs;

extern "C" vs_status vs_flow_run_noalloc(int w, int h, const vs_params* prm, const float* yt, const float* ym,
                                         float* flow_tm, float* flow_mt, void* stream)
{
    if (!yt || !ym) return VS_E_INVAL;
    vs_params P;
    if (prm) P = *prm;
    else vs_default_params(&P);
    DevPlan d;
    FlowLayout L;
    if (!flow_plan(w, h, P, d, L)) return VS_E_INVAL;
    if (kPlanBytes + L.bytes > (size_t)VS_FLOW_NOALLOC_BYTES) return VS_E_INVAL;   // beyond the static workspace
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return VS_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_base[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return VS_E_DEVICE;
        g_base[dev] = (uint8_t*)ptr;
    }
    uint8_t* base = g_base[dev];
    flow_bind(d, L, base + kPlanBytes);
    hipStream_t s = (hipStream_t)stream;
    DevPlan* dp = (DevPlan*)base;
    hipError_t e = hipSuccess;
    if (!g_plan_ok[dev] || std::memcmp(&g_plan[dev], &d, sizeof d) != 0) {
        g_plan_ok[dev] = false;
        e = upload_plan(d, base, s);
        if (e != hipSuccess) return VS_E_DEVICE;
        std::memcpy(&g_plan[dev], &d, sizeof d);
        g_plan_ok[dev] = true;
    }
    // the previous call may have left another shape's data: the flow domain is
    // marked again (the whole image); flow_run clears the accumulators itself
    e = flow_domain_fill(d, s);
    if (e == hipSuccess) e = flow_run(d, dp, yt, ym, flow_tm, flow_mt, s);
    if (e != hipSuccess) {
        g_plan_ok[dev] = false;
        return VS_E_DEVICE;
    }
    return VS_OK;
}
