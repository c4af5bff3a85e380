// Distance verification of candidate pairs (Section 4.1, Definition 1.1).
//
// A team of VF_TEAM lanes handles one pair: each lane reads consecutive
// 16-byte pieces of x_i and x_j (a team covers VF_TEAM * 16 contiguous bytes
// per row per step), two consecutive pairs and two steps at a time so that
// eight loads per lane are in flight, accumulates in FP32, and the team
// reduces with DPP adds. The next pairs' indices are fetched while the
// current pairs are computed. The team leaders then append the kept pairs
// with one LDS atomic per wave.
//
// The kernel is bound by the per-pair work every lane of a team repeats
// (indices, addresses, reduction, decision, append: about 60 % VALU-busy
// with eight lanes per pair at d = 128) and by the vector-memory path that
// carries both rows of every pair. Four lanes per pair halve the repeated
// work at the same bytes per pair; two lanes make each team's row pieces
// too short for the memory path.
#include "msm_internal.h"

#include <type_traits>

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int VF_THREADS = 256;
constexpr int VF_TEAM = 4;
constexpr int VF_PP = 2;     // consecutive pairs a team takes per iteration
constexpr int VF_OUT = 1024;  // staged kept pairs per workgroup
constexpr int NUM_XCD = 8;
static_assert(VF_TEAM == 4, "team_sum adds over the four lanes of a quad");

// Sum over the four lanes of a team (a DPP quad) with DPP adds: lanes xor 1,
// then lanes xor 2. Every lane ends with the same sum (each step adds the
// same two values in either order).
__device__ __forceinline__ float team_sum(float v)
{
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));  // quad [1,0,3,2]
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));  // quad [2,3,0,1]
    return v;
}

template <int METRIC, bool VEC4>
__global__ __launch_bounds__(VF_THREADS) void k_verify(const float* __restrict__ X, int64_t n, int d,
                                                       int64_t ldx, const uint32_t* __restrict__ pairs,
                                                       int64_t m, float eps, uint32_t* __restrict__ out,
                                                       unsigned long long cap, unsigned long long* counter,
                                                       uint32_t* bad)
{
    __shared__ uint2 obuf[VF_OUT];
    __shared__ uint32_t ocnt;
    __shared__ unsigned long long ogb;
    if (threadIdx.x == 0) ocnt = 0;
    __syncthreads();
    msm::PairStager<VF_OUT> stage{obuf, &ocnt, &ogb, out, cap, counter};
    const int tl = threadIdx.x & (VF_TEAM - 1);
    // Workgroups are dispatched round-robin over the NUM_XCD dies, each with
    // its own L2; the workgroups of die x take the contiguous x-th part of
    // the list, where adjacent pairs often share a row. gridDim.x is a
    // multiple of NUM_XCD.
    const int xcd = (int)(blockIdx.x % NUM_XCD);
    const int64_t per_die = gridDim.x / NUM_XCD;
    const int64_t lo = m * xcd / NUM_XCD, hi = m * (xcd + 1) / NUM_XCD;
    const int64_t team = ((int64_t)(blockIdx.x / NUM_XCD) * VF_THREADS + threadIdx.x) / VF_TEAM;
    const int64_t nteams = (per_die * VF_THREADS) / VF_TEAM;
    // every lane of a workgroup runs the same number of iterations, so
    // wave_append and the flushes are reached uniformly; a team takes VF_PP
    // consecutive pairs per iteration
    const int64_t span = nteams * VF_PP;
    const int64_t rounds = (hi - lo + span - 1) / span;
    uint2 nxt[VF_PP];
#pragma unroll
    for (int pp = 0; pp < VF_PP; ++pp) {
        const int64_t q = lo + team * VF_PP + pp;
        nxt[pp] = q < hi ? *reinterpret_cast<const uint2*>(pairs + 2 * q) : make_uint2(0u, 0u);
    }
    bool check_far = true;  // wave-uniform
    for (int64_t it = 0; it < rounds; ++it) {
        const int64_t q0 = lo + (team + it * nteams) * VF_PP;
        bool live[VF_PP];
        uint32_t pi[VF_PP], pj[VF_PP];
        const float* xi[VF_PP];
        const float* xj[VF_PP];
#pragma unroll
        for (int pp = 0; pp < VF_PP; ++pp) {
            live[pp] = q0 + pp < hi;
            pi[pp] = nxt[pp].x;
            pj[pp] = nxt[pp].y;
            if (q0 + span + pp < hi) nxt[pp] = *reinterpret_cast<const uint2*>(pairs + 2 * (q0 + span + pp));
            if (live[pp] && ((int64_t)pi[pp] >= n || (int64_t)pj[pp] >= n)) {
                if (tl == 0) atomicAdd(bad, 1u);
                live[pp] = false;
            }
            // a dead slot reads row 0 (n >= 1) and its result is dropped
            xi[pp] = X + (live[pp] ? (int64_t)pi[pp] * ldx : 0);
            xj[pp] = X + (live[pp] ? (int64_t)pj[pp] * ldx : 0);
        }
        float a0[VF_PP], a1[VF_PP], a2[VF_PP];
#pragma unroll
        for (int pp = 0; pp < VF_PP; ++pp) a0[pp] = a1[pp] = a2[pp] = 0.f;
        auto acc = [&](int pp, float u, float v) {
            if (METRIC == MSM_EUCLIDEAN) {
                const float e = u - v;
                a0[pp] = fmaf(e, e, a0[pp]);
            } else {
                a0[pp] = fmaf(u, v, a0[pp]);
                a1[pp] = fmaf(u, u, a1[pp]);
                a2[pp] = fmaf(v, v, a2[pp]);
            }
        };
        // Euclidean: a pair whose partial sum over the team already exceeds
        // eps^2 is decided (each lane's FP32 sum only grows as terms are
        // added, and so does the team's sum of them), and its remaining
        // row pieces are not read. The check is made while at least half of
        // the wave's pairs were rejected in its last round (far pairs);
        // otherwise the rows are read straight through.
        bool far[VF_PP];
#pragma unroll
        for (int pp = 0; pp < VF_PP; ++pp) far[pp] = false;
        const float eps2 = eps * eps;
        if (VEC4) {
            constexpr int STEP = VF_TEAM * 4;
            constexpr int UN = 4 / VF_PP;  // row steps per pair in flight
            // team-uniform steps, so that the team sum sees all lanes; lane
            // tl takes elements tl * 4 + k * STEP in order of k
            auto rows = [&](auto check_tag) {
                constexpr bool CHECK = decltype(check_tag)::value;
                int base = 0;
                for (; base + UN * STEP <= d; base += UN * STEP) {
                    floatx4 u[VF_PP][UN], v[VF_PP][UN];
#pragma unroll
                    for (int pp = 0; pp < VF_PP; ++pp) {
                        if (CHECK && far[pp]) continue;
#pragma unroll
                        for (int r = 0; r < UN; ++r) {
                            u[pp][r] = *reinterpret_cast<const floatx4*>(xi[pp] + base + tl * 4 + r * STEP);
                            v[pp][r] = *reinterpret_cast<const floatx4*>(xj[pp] + base + tl * 4 + r * STEP);
                        }
                    }
#pragma unroll
                    for (int pp = 0; pp < VF_PP; ++pp) {
                        if (CHECK && far[pp]) continue;
#pragma unroll
                        for (int r = 0; r < UN; ++r)
#pragma unroll
                            for (int c = 0; c < 4; ++c) acc(pp, u[pp][r][c], v[pp][r][c]);
                    }
                    if (CHECK && base + UN * STEP < d) {
                        bool all_far = true;
#pragma unroll
                        for (int pp = 0; pp < VF_PP; ++pp) {
                            if (!far[pp]) far[pp] = team_sum(a0[pp]) > eps2;
                            all_far = all_far && far[pp];
                        }
                        if (all_far) break;
                    }
                }
                for (int t = base + tl * 4; t < d; t += STEP) {
#pragma unroll
                    for (int pp = 0; pp < VF_PP; ++pp) {
                        if (CHECK && far[pp]) continue;
                        const floatx4 u = *reinterpret_cast<const floatx4*>(xi[pp] + t);
                        const floatx4 v = *reinterpret_cast<const floatx4*>(xj[pp] + t);
#pragma unroll
                        for (int c = 0; c < 4; ++c) acc(pp, u[c], v[c]);
                    }
                }
            };
            if (METRIC == MSM_EUCLIDEAN && check_far)
                rows(std::true_type{});
            else
                rows(std::false_type{});
        } else {
#pragma unroll
            for (int pp = 0; pp < VF_PP; ++pp) {
                int t = tl;
                for (; t + 3 * VF_TEAM < d; t += 4 * VF_TEAM) {
                    float u[4], v[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        u[r] = xi[pp][t + r * VF_TEAM];
                        v[r] = xj[pp][t + r * VF_TEAM];
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc(pp, u[r], v[r]);
                }
                for (; t < d; t += VF_TEAM) acc(pp, xi[pp][t], xj[pp][t]);
            }
        }
        uint32_t nlive = 0, nrej = 0;  // this round's pairs of the wave, and rejected ones
#pragma unroll
        for (int pp = 0; pp < VF_PP; ++pp) {
            a0[pp] = team_sum(a0[pp]);
            if (METRIC == MSM_COSINE) {
                a1[pp] = team_sum(a1[pp]);
                a2[pp] = team_sum(a2[pp]);
            }
            bool keep = false;
            if (live[pp] && tl == 0 && !far[pp]) {
                if (METRIC == MSM_EUCLIDEAN) {
                    keep = a0[pp] <= eps2;
                } else {
                    const float dist = (a1[pp] == 0.f || a2[pp] == 0.f)
                                           ? 1.0f
                                           : 1.0f - a0[pp] / (sqrtf(a1[pp]) * sqrtf(a2[pp]));
                    keep = dist <= eps;
                }
            }
            stage.push(keep, pi[pp], pj[pp]);
            nlive += (uint32_t)__popcll(__ballot(live[pp] && tl == 0));
            nrej += (uint32_t)__popcll(__ballot(live[pp] && tl == 0 && !keep));
        }
        check_far = 2 * nrej >= nlive;
        if ((it & (16 / VF_PP - 1)) == 16 / VF_PP - 1) stage.maybe_flush(VF_OUT / 2);
    }
    stage.flush();
}

__global__ void k_zero_words(unsigned long long* a, int n)
{
    const int i = threadIdx.x;
    if (i < n) a[i] = 0ull;
}

template <int METRIC>
void launch(bool vec4, dim3 grid, hipStream_t s, const float* X, int64_t n, int d, int64_t ldx,
            const uint32_t* pairs, int64_t m, float eps, uint32_t* out, int64_t cap,
            unsigned long long* counter, uint32_t* bad)
{
    if (vec4)
        hipLaunchKernelGGL((k_verify<METRIC, true>), grid, dim3(VF_THREADS), 0, s, X, n, d, ldx, pairs, m, eps,
                           out, (unsigned long long)cap, counter, bad);
    else
        hipLaunchKernelGGL((k_verify<METRIC, false>), grid, dim3(VF_THREADS), 0, s, X, n, d, ldx, pairs, m, eps,
                           out, (unsigned long long)cap, counter, bad);
}

}  // namespace

extern "C" msm_status msm_verify(msm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                                 const uint32_t* pairs, int64_t m, int32_t metric, float eps,
                                 uint32_t* out, int64_t cap, int64_t* m_out, void* stream)
{
    if (!ctx) return msm::fail(nullptr, MSM_E_INVALID, "msm_verify: ctx is NULL");
    ctx->err.clear();
    if (!m_out) return msm::fail(ctx, MSM_E_INVALID, "msm_verify: m_out is NULL");
    *m_out = 0;
    if (n < 0 || n > 0xFFFFFFFFll || d < 1 || ldx < d || m < 0 || cap < 0)
        return msm::fail(ctx, MSM_E_INVALID, "msm_verify: sizes out of range");
    if (metric != MSM_EUCLIDEAN && metric != MSM_COSINE)
        return msm::fail(ctx, MSM_E_INVALID, "msm_verify: unknown metric %d", metric);
    if (!(eps >= 0.0f) || eps == __builtin_inff())
        return msm::fail(ctx, MSM_E_INVALID, "msm_verify: eps must be finite and >= 0");
    if (m == 0) return MSM_OK;
    if (!X || !pairs) return msm::fail(ctx, MSM_E_INVALID, "msm_verify: NULL X or pairs");
    if (n == 0) return msm::fail(ctx, MSM_E_INVALID, "msm_verify: %lld pairs index an empty X", (long long)m);
    if (cap > 0 && !out) return msm::fail(ctx, MSM_E_INVALID, "msm_verify: out is NULL with cap > 0");
    if ((reinterpret_cast<uintptr_t>(pairs) & 7) || (out && (reinterpret_cast<uintptr_t>(out) & 7)))
        return msm::fail(ctx, MSM_E_INVALID, "msm_verify: pair buffers must be 8-byte aligned");
    msm_status st = msm::use_device(ctx);
    if (st != MSM_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    void* scr = nullptr;
    st = msm::ctx_scratch(ctx, 256, s, &scr);
    if (st != MSM_OK) return st;
    unsigned long long* counter = static_cast<unsigned long long*>(scr);
    uint32_t* bad = reinterpret_cast<uint32_t*>(counter + 1);
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, counter, 2);
    const bool vec4 = ((reinterpret_cast<uintptr_t>(X) & 15) == 0) && (ldx % 4 == 0) && (d % 4 == 0);
    const int64_t pairs_per_block = VF_THREADS / VF_TEAM * VF_PP;
    int64_t blocks = (m + pairs_per_block - 1) / pairs_per_block;
    const int64_t max_blocks = (int64_t)ctx->num_cu * 16;
    if (blocks > max_blocks) blocks = max_blocks;
    blocks = (blocks + NUM_XCD - 1) / NUM_XCD * NUM_XCD;
    {
        msm::KernelTimer kt(ctx, s, "k_verify");
        if (metric == MSM_EUCLIDEAN)
            launch<MSM_EUCLIDEAN>(vec4, dim3((unsigned)blocks), s, X, n, d, ldx, pairs, m, eps, out, cap, counter,
                                  bad);
        else
            launch<MSM_COSINE>(vec4, dim3((unsigned)blocks), s, X, n, d, ldx, pairs, m, eps, out, cap, counter, bad);
    }
    MSM_HIP(ctx, hipGetLastError());
    MSM_HIP(ctx, hipMemcpyAsync(ctx->host_words, counter, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    MSM_HIP(ctx, hipStreamSynchronize(s));
    const int64_t kept = (int64_t)ctx->host_words[0];
    const uint32_t nbad = (uint32_t)(ctx->host_words[1] & 0xFFFFFFFFull);
    if (nbad)
        return msm::fail(ctx, MSM_E_INVALID, "msm_verify: %u pairs have an index >= n", nbad);
    *m_out = kept;
    if (kept > cap && !(out == nullptr && cap == 0))
        return msm::fail(ctx, MSM_E_CAPACITY, "msm_verify: %lld pairs do not fit in cap=%lld", (long long)kept,
                         (long long)cap);
    return MSM_OK;
}
