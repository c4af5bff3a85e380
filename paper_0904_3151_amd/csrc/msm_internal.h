// Internal declarations of libmsm: the context, error helpers and the
// device helpers shared by the kernels. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "msm.h"

struct msm_ctx {
    int device = 0;
    int num_cu = 256;
    std::string err;
    // Grow-only device scratch shared by the calls made through the context.
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    // Pinned host words used to read counters back from the device.
    uint64_t* host_words = nullptr;
    // Pinned host staging for table uploads of the calls that allocate
    // nothing (NOALLOC_STAGE_BYTES).
    char* host_stage = nullptr;
    // Device address, on this context's device, of the library's static
    // no-allocation scratch (NOALLOC_SCRATCH_BYTES), or NULL when it could
    // not be resolved.
    void* noalloc_scratch = nullptr;
    // Groupings (and j of a hierarchical grouping, else 0) of the last
    // enumeration.
    int32_t last_groupings = 0;
    int32_t last_jblocks = 0;
    // Per-kernel timing: a pair of HIP events around every launch while on.
    bool prof = false;
    std::string prof_only;  // when not empty, the one kernel name that is timed
    struct Pending {
        const char* name;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> event_pool;
    std::vector<Pending> pending;
    std::map<std::string, std::pair<int64_t, double>> prof_acc;  // launches, ms
};

namespace msm {

// Size of the static device array that msm_enumerate_pairs_noalloc works in
// (one per device, held until the process ends), and of the pinned host
// buffer through which that call uploads its tables.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
constexpr size_t NOALLOC_STAGE_BYTES = (size_t)2 << 20;

msm_status fail(msm_ctx* ctx, msm_status st, const char* fmt, ...);
msm_status hip_fail(msm_ctx* ctx, hipError_t e, const char* what);
// Make the device of ctx current.
msm_status use_device(msm_ctx* ctx);
// Device scratch of at least `bytes` (256-byte aligned). Synchronises
// `stream` before replacing a smaller buffer.
msm_status ctx_scratch(msm_ctx* ctx, size_t bytes, hipStream_t stream, void** out);

// Records a HIP event before and after the launches in its scope, on the
// launch stream, when profiling is on.
class KernelTimer {
public:
    KernelTimer(msm_ctx* ctx, hipStream_t s, const char* name);
    ~KernelTimer();

private:
    msm_ctx* ctx_;
    hipStream_t s_;
    const char* name_;
    hipEvent_t a_ = nullptr;
};

// Resolves recorded events into per-kernel totals (waits for them).
msm_status profile_collect(msm_ctx* ctx);

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Batched projection (eq. (3) for many instances in one launch).
struct ProjInst {
    const float* X;   // DEVICE, n rows, ldx stride
    int64_t n;
    int64_t ldx;
    const float* R;   // DEVICE, d x ell
    uint64_t* S;      // DEVICE, the instance's strings
    uint64_t* S2;     // DEVICE, second copy (the concatenation), or NULL
    int32_t d;
    int32_t vec4;     // X 16-byte aligned with ldx % 4 == 0
};
struct ProjEntry {    // a run of rows of one instance
    int64_t row0;
    int32_t rows;
    uint32_t inst;
};
// Rows per tile of the batched projection kernel for ell bits (entries
// should hold a multiple of it).
int batch_project_rows(int ell);
// Enqueues the batched projection over `nentries` entries with a grid of
// `grid` persistent workgroups that claim entries from *work (which must be
// zero when the kernel starts); max_d bounds every instance's d.
hipError_t batch_project(const ProjInst* inst, const ProjEntry* entries, int nentries, int ell, int max_d, int grid,
                         unsigned int* work, hipStream_t stream);

// Carves consecutive 256-byte-aligned pieces out of one scratch buffer.
struct Carver {
    size_t off = 0;
    char* base = nullptr;
    template <class T>
    T* take(size_t count) {
        off = align_up(off, 256);
        T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
        off += count * sizeof(T);
        return p;
    }
};

#define MSM_HIP(ctx, call)                                              \
    do {                                                                \
        hipError_t e_ = (call);                                         \
        if (e_ != hipSuccess) return ::msm::hip_fail((ctx), e_, #call); \
    } while (0)

// ----------------------------------------------------------------------
// Device helpers

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const int l = __lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Inclusive prefix sum across the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int l = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o, 64);
        if (l >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Appends the calling lanes' `ok` results to a global list: one atomic per
// wave, slots in lane order. Must be reached by every lane of the wave.
// Returns this lane's slot (meaningful only where ok).
__device__ __forceinline__ unsigned long long wave_append(bool ok, unsigned long long* counter)
{
    const uint64_t mask = __ballot(ok);
    unsigned long long base = 0;
    if (mask) {
        const int leader = __builtin_ctzll(mask);
        if (__lane_id() == leader) base = atomicAdd(counter, (unsigned long long)__popcll(mask));
        base = __shfl(base, leader, 64);
    }
    return base + (unsigned long long)__popcll(mask & lanemask_lt());
}

// Collects a workgroup's output pairs in LDS so that the global output
// counter is touched once per flush instead of once per wave step.
// `buf` (CAPB entries) and `cnt` live in LDS; `cnt` must start at 0.
// push() is called by every lane of a wave (converged); pairs that do not
// fit in LDS are appended to the global list directly. flush() and
// maybe_flush() are called by every thread of the workgroup.
template <int CAPB>
struct PairStager {
    uint2* buf;
    uint32_t* cnt;
    unsigned long long* gbase;  // LDS scratch word for the flush
    uint32_t* out;
    unsigned long long cap;
    unsigned long long* counter;

    __device__ __forceinline__ void push(bool ok, uint32_t i, uint32_t j)
    {
        const uint64_t mask = __ballot(ok);
        if (!mask) return;
        const int leader = __builtin_ctzll(mask);
        uint32_t base = 0;
        if (__lane_id() == leader) base = atomicAdd(cnt, (uint32_t)__popcll(mask));
        base = __shfl(base, leader, 64);
        const uint32_t pos = base + (uint32_t)__popcll(mask & lanemask_lt());
        const bool spill = ok && pos >= (uint32_t)CAPB;
        if (ok && !spill) buf[pos] = make_uint2(i, j);
        const unsigned long long slot = wave_append(spill, counter);
        if (spill && slot < cap) *reinterpret_cast<uint2*>(out + 2 * slot) = make_uint2(i, j);
    }

    __device__ __forceinline__ void flush()
    {
        __syncthreads();
        const uint32_t n = min(*cnt, (uint32_t)CAPB);
        if (n > 0) {
            if (threadIdx.x == 0) *gbase = atomicAdd(counter, (unsigned long long)n);
            __syncthreads();
            const unsigned long long g = *gbase;
            for (uint32_t e = threadIdx.x; e < n; e += blockDim.x)
                if (g + e < cap) *reinterpret_cast<uint2*>(out + 2 * (g + e)) = buf[e];
            __syncthreads();
        }
        if (threadIdx.x == 0) *cnt = 0;
        __syncthreads();
    }

    // Flushes when at least `threshold` pairs are staged.
    __device__ __forceinline__ void maybe_flush(uint32_t threshold)
    {
        __syncthreads();
        if (*cnt >= threshold) flush();
    }
};

}  // namespace msm
