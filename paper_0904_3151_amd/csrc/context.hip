// Context lifetime, error reporting and scratch memory of libmsm.
#include "msm_internal.h"

#include <cstring>
#include <mutex>

// Work memory of msm_enumerate_pairs_noalloc, for callers that cannot
// allocate device memory. Every device the library runs on holds its own
// copy until the process ends. In host code this name is only a handle for
// hipGetSymbolAddress: kernels are given the device address it returns
// (kept per device in g_noalloc_ptr), never the name itself.
static __device__ __align__(256) unsigned char scratch[msm::NOALLOC_SCRATCH_BYTES];

namespace {
thread_local std::string g_create_err;

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// The device address of `scratch` on `device`, which must be current:
// resolved on the first call for that device, then reused.
hipError_t noalloc_address(int device, void** out)
{
    *out = nullptr;
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipSuccess;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_noalloc_ptr[device] = ptr;
    }
    *out = g_noalloc_ptr[device];
    return hipSuccess;
}
}  // namespace

namespace msm {

msm_status fail(msm_ctx* ctx, msm_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx)
        ctx->err = buf;
    else
        g_create_err = buf;
    return st;
}

msm_status hip_fail(msm_ctx* ctx, hipError_t e, const char* what)
{
    return fail(ctx, MSM_E_HIP, "%s failed: %s", what, hipGetErrorString(e));
}

msm_status use_device(msm_ctx* ctx)
{
    int cur = -1;
    MSM_HIP(ctx, hipGetDevice(&cur));
    if (cur != ctx->device) MSM_HIP(ctx, hipSetDevice(ctx->device));
    return MSM_OK;
}

msm_status ctx_scratch(msm_ctx* ctx, size_t bytes, hipStream_t stream, void** out)
{
    bytes = align_up(bytes < 256 ? 256 : bytes, 256);
    if (bytes > ctx->scratch_bytes) {
        // Work already enqueued on the stream may still read the old buffer.
        MSM_HIP(ctx, hipStreamSynchronize(stream));
        if (ctx->scratch) {
            MSM_HIP(ctx, hipFree(ctx->scratch));
            ctx->scratch = nullptr;
            ctx->scratch_bytes = 0;
        }
        const size_t want = align_up(bytes + bytes / 4, 1 << 20);
        void* p = nullptr;
        if (hipMalloc(&p, want) != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, MSM_E_NOMEM, "device scratch of %zu bytes could not be allocated", want);
        }
        ctx->scratch = p;
        ctx->scratch_bytes = want;
    }
    *out = ctx->scratch;
    return MSM_OK;
}

static hipEvent_t take_event(msm_ctx* ctx)
{
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

KernelTimer::KernelTimer(msm_ctx* ctx, hipStream_t s, const char* name) : ctx_(ctx), s_(s), name_(name)
{
    if (!ctx_->prof) return;
    if (!ctx_->prof_only.empty() && ctx_->prof_only != name_) return;
    a_ = take_event(ctx_);
    if (a_ && hipEventRecord(a_, s_) != hipSuccess) {
        (void)hipGetLastError();
        ctx_->event_pool.push_back(a_);
        a_ = nullptr;
    }
}

KernelTimer::~KernelTimer()
{
    if (!a_) return;
    hipEvent_t b = take_event(ctx_);
    if (!b || hipEventRecord(b, s_) != hipSuccess) {
        (void)hipGetLastError();
        ctx_->event_pool.push_back(a_);
        if (b) ctx_->event_pool.push_back(b);
        return;
    }
    ctx_->pending.push_back({name_, a_, b});
}

msm_status profile_collect(msm_ctx* ctx)
{
    for (auto& p : ctx->pending) {
        MSM_HIP(ctx, hipEventSynchronize(p.b));
        float ms = 0.f;
        MSM_HIP(ctx, hipEventElapsedTime(&ms, p.a, p.b));
        auto& acc = ctx->prof_acc[p.name];
        acc.first += 1;
        acc.second += ms;
        ctx->event_pool.push_back(p.a);
        ctx->event_pool.push_back(p.b);
    }
    ctx->pending.clear();
    return MSM_OK;
}

}  // namespace msm

extern "C" {

int32_t msm_version(void) { return 100; }

msm_status msm_create(int32_t device, msm_ctx** out)
{
    if (!out) return msm::fail(nullptr, MSM_E_INVALID, "msm_create: out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return msm::hip_fail(nullptr, e, "hipGetDeviceCount");
    if (device < 0 || device >= count)
        return msm::fail(nullptr, MSM_E_INVALID, "msm_create: device %d not in [0, %d)", device, count);
    msm_ctx* ctx = new msm_ctx();
    ctx->device = device;
    msm_status st = msm::use_device(ctx);
    if (st != MSM_OK) {
        g_create_err = ctx->err;
        delete ctx;
        return st;
    }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) {
        delete ctx;
        return msm::hip_fail(nullptr, e, "hipGetDeviceProperties");
    }
    ctx->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    e = hipHostMalloc((void**)&ctx->host_words, 64 * sizeof(uint64_t), hipHostMallocDefault);
    if (e != hipSuccess) {
        delete ctx;
        return msm::hip_fail(nullptr, e, "hipHostMalloc");
    }
    e = hipHostMalloc((void**)&ctx->host_stage, msm::NOALLOC_STAGE_BYTES, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipHostFree(ctx->host_words);
        delete ctx;
        return msm::hip_fail(nullptr, e, "hipHostMalloc");
    }
    // the no-allocation scratch of this device, with the device current
    e = noalloc_address(device, &ctx->noalloc_scratch);
    if (e != hipSuccess) {
        (void)hipHostFree(ctx->host_stage);
        (void)hipHostFree(ctx->host_words);
        delete ctx;
        return msm::hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
    }
    *out = ctx;
    return MSM_OK;
}

void msm_destroy(msm_ctx* ctx)
{
    if (!ctx) return;
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != ctx->device) (void)hipSetDevice(ctx->device);
    for (auto& p : ctx->pending) {
        (void)hipEventSynchronize(p.b);
        ctx->event_pool.push_back(p.a);
        ctx->event_pool.push_back(p.b);
    }
    for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->host_words) (void)hipHostFree(ctx->host_words);
    if (ctx->host_stage) (void)hipHostFree(ctx->host_stage);
    if (cur >= 0 && cur != ctx->device) (void)hipSetDevice(cur);
    delete ctx;
}

const char* msm_last_error(const msm_ctx* ctx)
{
    return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

}  // extern "C"

extern "C" msm_status msm_profile_enable(msm_ctx* ctx, int32_t enable)
{
    if (!ctx) return msm::fail(nullptr, MSM_E_INVALID, "msm_profile_enable: ctx is NULL");
    ctx->err.clear();
    ctx->prof = enable != 0;
    return MSM_OK;
}

extern "C" msm_status msm_profile_only(msm_ctx* ctx, const char* name)
{
    if (!ctx) return msm::fail(nullptr, MSM_E_INVALID, "msm_profile_only: ctx is NULL");
    ctx->err.clear();
    if (name && std::strlen(name) >= sizeof(((msm_kernel_time*)nullptr)->name))
        return msm::fail(ctx, MSM_E_INVALID, "msm_profile_only: name too long");
    ctx->prof_only = name ? name : "";
    return MSM_OK;
}

extern "C" msm_status msm_profile_reset(msm_ctx* ctx)
{
    if (!ctx) return msm::fail(nullptr, MSM_E_INVALID, "msm_profile_reset: ctx is NULL");
    ctx->err.clear();
    msm_status st = msm::profile_collect(ctx);
    ctx->prof_acc.clear();
    return st;
}

extern "C" int32_t msm_profile_read(msm_ctx* ctx, msm_kernel_time* out, int32_t cap)
{
    if (!ctx || cap < 0 || (cap > 0 && !out)) return -1;
    ctx->err.clear();
    if (msm::profile_collect(ctx) != MSM_OK) return -1;
    int32_t i = 0;
    for (const auto& kv : ctx->prof_acc) {
        if (i < cap) {
            msm_kernel_time& t = out[i];
            memset(&t, 0, sizeof(t));
            strncpy(t.name, kv.first.c_str(), sizeof(t.name) - 1);
            t.launches = kv.second.first;
            t.total_ms = kv.second.second;
        }
        ++i;
    }
    return i;
}
