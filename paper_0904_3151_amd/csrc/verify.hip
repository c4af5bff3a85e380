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

#include <algorithm>
#include <cmath>
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
                                                       uint32_t* bad, const uint32_t* run_if)
{
    if (run_if && *run_if == 0u) return;  // the other form was chosen
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

// ---------------------------------------------------------------------------
// Certified FP16 screen (Euclidean metric, lists of at least as many pairs as
// rows). The rows are rounded once to FP16 (round to nearest even) with, per
// row, an upper bound b_i on ||fl16(x_i) - x_i||_2. A coordinate v rounds with
// |fl16(v) - v| <= 2^-11 |v| + 2^-14 (half an ulp of an 11-bit significand,
// or a subnormal flushed to zero), so b_i = 2^-11 ||x_i|| + 2^-14 sqrt(d),
// raised by a relative 2^-10 + d 2^-23 that covers its own FP32 evaluation.
// A row with a coordinate above 32752 in magnitude, or not finite, gets
// b_i = inf; otherwise no difference of two rows overflows FP16.
//
// A team of four lanes (k_verify's layout on 16-byte pieces of eight halves)
// forms t_k = fl16(h_ik - h_jk) with packed FP16 subtractions and
// accumulates S = sum t_k^2 with FP32 fused multiply-adds on the halves.
// Every t_k, as the FMA reads it, is within 2^-11 |h_ik - h_jk| + 2 * 2^-14
// of the exact difference of the FP16 rows (a subnormal result of the
// subtraction, a flush inside the FMA), so with A = b_i + b_j,
// c = 2^-13 sqrt(d) and gamma a bound on the relative error of the FP32
// sum, the distance D of the FP32 rows satisfies
//     (sqrt(S / (1 + gamma)) - c) / (1 + 2^-11) - A  <=  D
//     D  <=  (sqrt(S / (1 - gamma)) + c) / (1 - 2^-11) + A.
// The pair is kept for certain when S <= ((eps - A)(1 - 2^-11) - c)^2 (1 - gamma)
// and rejected for certain when S > ((eps + A)(1 + 2^-11) + c)^2 (1 + gamma). Pairs in between are summed again from the FP32
// rows by the same lanes in k_verify's order, so their decision is
// k_verify's; certified decisions are the exact ones. The screen reads half
// the bytes of k_verify per pair and makes one packed subtraction and one
// mixed FMA per two coordinates.
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr float VH_MAXABS = 32752.0f;  // largest FP16 value at most half the FP16 maximum
constexpr int VH_ROW_LANES = 16;       // lanes per row in the rounding kernel
constexpr int VH_ROWS = 256 / VH_ROW_LANES;
// the FP32 kernel verifies the first max(VH_SAMPLE_MIN, m / VH_SAMPLE_DIV)
// pairs, from which the form of the rest is chosen
constexpr int64_t VH_SAMPLE_MIN = 1 << 16;
constexpr int64_t VH_SAMPLE_DIV = 256;

__device__ __forceinline__ half2v as_h2(uint32_t u) { return __builtin_bit_cast(half2v, u); }

// Constants of the certified thresholds, rounded on the host in the safe
// direction. With A = b_i + b_j (the row bounds' relative slack of 2^-10
// also covers the rounding of this sum):
//   rejection: t = fma(A, r1, r0) >= ((eps + A)(1 + 2^-11) + c), as r1 and
//     r0 carry a factor 1 + 2^-19 over the exact coefficients, more than the
//     fma's rounding; threshold t^2 g_up with g_up >= 1 + gamma + 2^-18.
//   keep: t = fma(-A, 1 - 2^-11, k0) <= (eps - A)(1 - 2^-11) - c whenever it
//     is positive, as k0 sits 2^-19 (eps + c) below its exact value, more
//     than the fma's rounding of a result below eps; threshold t^2 g_dn with
//     g_dn <= 1 - gamma - 2^-18. The 2^-18 absorbs the two final products.
struct ScreenConsts {
    float r0, r1, k0, g_up, g_dn;
};

// After the FP32 kernel has verified the list's first m0 pairs: the FP16
// screen takes the rest (run[0] = 1, run[1] = 0) when at least an eighth of
// them were kept, the FP32 kernel otherwise (pairs that are mostly far are
// rejected after a few coordinates by the FP32 kernel, and the rows' FP16
// copy would not pay for itself).
__global__ void k_choose_form(const unsigned long long* counter, int64_t m0, uint32_t* run)
{
    if (threadIdx.x == 0) {
        const bool screen = (int64_t)(*counter) * 8 >= m0;
        run[0] = screen ? 1u : 0u;
        run[1] = screen ? 0u : 1u;
    }
}

// Rounds rows to FP16, ldw 32-bit words (2 ldw >= d, a multiple of 8 halves,
// zero beyond d) per row, and writes each row's bound b_i. Sixteen lanes
// take a row; the grid strides over the rows.
__global__ __launch_bounds__(256) void k_half_rows(const float* __restrict__ X, int64_t n, int d, int64_t ldx,
                                                   int vec4, uint32_t* __restrict__ Xh, int64_t ldw,
                                                   float* __restrict__ bnd, const uint32_t* run_if)
{
    if (*run_if == 0u) return;
    const int lane = threadIdx.x & (VH_ROW_LANES - 1);
    for (int64_t row = (int64_t)blockIdx.x * VH_ROWS + threadIdx.x / VH_ROW_LANES; row < n;
         row += (int64_t)gridDim.x * VH_ROWS) {
        // the sixteen lanes of a row iterate together
        const float* x = X + row * ldx;
        uint32_t* h = Xh + row * ldw;
        float ss = 0.f;
        int ok = 1;
        for (int64_t w = (int64_t)lane * 4; w < ldw; w += VH_ROW_LANES * 4) {
            const int64_t e = 2 * w;  // first of this lane's eight halves
            float v[8];
            if (vec4 && e + 8 <= d) {
                const floatx4 p = *reinterpret_cast<const floatx4*>(x + e);
                const floatx4 q = *reinterpret_cast<const floatx4*>(x + e + 4);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    v[c] = p[c];
                    v[4 + c] = q[c];
                }
            } else {
#pragma unroll
                for (int c = 0; c < 8; ++c) v[c] = e + c < d ? x[e + c] : 0.f;
            }
            u32x4 o;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                ss = fmaf(v[2 * c], v[2 * c], ss);
                ss = fmaf(v[2 * c + 1], v[2 * c + 1], ss);
                ok &= (fabsf(v[2 * c]) <= VH_MAXABS) & (fabsf(v[2 * c + 1]) <= VH_MAXABS);
                const half2v hv = {(_Float16)v[2 * c], (_Float16)v[2 * c + 1]};
                o[c] = __builtin_bit_cast(uint32_t, hv);
            }
            *reinterpret_cast<u32x4*>(h + w) = o;
        }
#pragma unroll
        for (int off = VH_ROW_LANES / 2; off >= 1; off >>= 1) {
            ss += __shfl_xor(ss, off, VH_ROW_LANES);
            ok &= __shfl_xor(ok, off, VH_ROW_LANES);
        }
        if (lane == 0)
            bnd[row] = ok ? sqrtf(ss) * 0x1p-11f * (1.0f + 0x1p-10f + (float)d * 0x1p-23f) +
                                sqrtf((float)d) * 0x1p-14f * (1.0f + 0x1p-10f)
                          : __builtin_inff();
    }
}

template <bool VEC4>
__global__ __launch_bounds__(VF_THREADS) void k_verify_h(const uint32_t* __restrict__ Xh, int64_t ldw,
                                                         const float* __restrict__ bnd,
                                                         const float* __restrict__ X, int64_t n, int d,
                                                         int64_t ldx, const uint32_t* __restrict__ pairs,
                                                         int64_t m, float eps, ScreenConsts k,
                                                         uint32_t* __restrict__ out, unsigned long long cap,
                                                         unsigned long long* counter, uint32_t* bad,
                                                         const uint32_t* run_if)
{
    if (*run_if == 0u) return;  // the FP32 kernel was chosen
    __shared__ uint2 obuf[VF_OUT];
    __shared__ uint32_t ocnt;
    __shared__ unsigned long long ogb;
    if (threadIdx.x == 0) ocnt = 0;
    __syncthreads();
    msm::PairStager<VF_OUT> stage{obuf, &ocnt, &ogb, out, cap, counter};
    const int tl = threadIdx.x & (VF_TEAM - 1);
    const int xcd = (int)(blockIdx.x % NUM_XCD);
    const int64_t per_die = gridDim.x / NUM_XCD;
    const int64_t lo = m * xcd / NUM_XCD, hi = m * (xcd + 1) / NUM_XCD;
    const int64_t team = ((int64_t)(blockIdx.x / NUM_XCD) * VF_THREADS + threadIdx.x) / VF_TEAM;
    const int64_t nteams = (per_die * VF_THREADS) / VF_TEAM;
    const int64_t span = nteams * VF_PP;
    const int64_t rounds = (hi - lo + span - 1) / span;
    const float eps2 = eps * eps;
    // Thresholds of a pair from its two row bounds (ScreenConsts): certified
    // keep at or below the first, certified rejection above the second.
    auto keep_thr = [&](float bi, float bj) {
        const float tk = fmaf(-(bi + bj), 1.0f - 0x1p-11f, k.k0);
        return tk > 0.f ? tk * tk * k.g_dn : -1.f;
    };
    auto rej_thr = [&](float bi, float bj) {
        const float tr = fmaf(bi + bj, k.r1, k.r0);
        return tr * tr * k.g_up;
    };
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
        const uint32_t* hi_[VF_PP];
        const uint32_t* hj_[VF_PP];
        float bi[VF_PP], bj[VF_PP];
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
            const int64_t ri = live[pp] ? (int64_t)pi[pp] : 0, rj = live[pp] ? (int64_t)pj[pp] : 0;
            hi_[pp] = Xh + ri * ldw;
            hj_[pp] = Xh + rj * ldw;
            bi[pp] = bnd[ri];
            bj[pp] = bnd[rj];
        }
        float a[VF_PP];
        bool far[VF_PP];
#pragma unroll
        for (int pp = 0; pp < VF_PP; ++pp) {
            a[pp] = 0.f;
            far[pp] = false;
        }
        auto acc = [&](int pp, uint32_t u, uint32_t v) {
            const half2v t = as_h2(u) - as_h2(v);
            a[pp] = fmaf((float)t[0], (float)t[0], a[pp]);
            a[pp] = fmaf((float)t[1], (float)t[1], a[pp]);
        };
        constexpr int STEPW = VF_TEAM * 4;  // words of a team step
        auto rows = [&](auto check_tag) {
            constexpr bool CHECK = decltype(check_tag)::value;
            // while checking, one team step (32 coordinates) between checks
            constexpr int UN = CHECK ? 1 : 4 / VF_PP;
            int64_t base = 0;
            for (; base + UN * STEPW <= ldw; base += UN * STEPW) {
                u32x4 u[VF_PP][UN], v[VF_PP][UN];
#pragma unroll
                for (int pp = 0; pp < VF_PP; ++pp) {
                    if (CHECK && far[pp]) continue;
#pragma unroll
                    for (int r = 0; r < UN; ++r) {
                        u[pp][r] = *reinterpret_cast<const u32x4*>(hi_[pp] + base + tl * 4 + r * STEPW);
                        v[pp][r] = *reinterpret_cast<const u32x4*>(hj_[pp] + base + tl * 4 + r * STEPW);
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
                if (CHECK && base + UN * STEPW < ldw) {
                    // partial sums only grow, so a partial sum above the
                    // rejection threshold rejects the pair for certain
                    bool all_far = true;
#pragma unroll
                    for (int pp = 0; pp < VF_PP; ++pp) {
                        if (!far[pp]) far[pp] = team_sum(a[pp]) > rej_thr(bi[pp], bj[pp]);
                        all_far = all_far && far[pp];
                    }
                    if (all_far) break;
                }
            }
            for (int64_t t = base + tl * 4; t < ldw; t += STEPW) {
#pragma unroll
                for (int pp = 0; pp < VF_PP; ++pp) {
                    if (CHECK && far[pp]) continue;
                    const u32x4 u = *reinterpret_cast<const u32x4*>(hi_[pp] + t);
                    const u32x4 v = *reinterpret_cast<const u32x4*>(hj_[pp] + t);
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc(pp, u[c], v[c]);
                }
            }
        };
        if (check_far)
            rows(std::true_type{});
        else
            rows(std::false_type{});
        uint32_t nlive = 0, nrej = 0;
#pragma unroll
        for (int pp = 0; pp < VF_PP; ++pp) {
            const float sum = team_sum(a[pp]);
            // every lane of a team holds the same sum and bounds, so the
            // branch below is taken by whole teams
            bool keep = false, undecided = false;
            if (live[pp] && !far[pp]) {
                keep = sum <= keep_thr(bi[pp], bj[pp]);
                undecided = !keep && !(sum > rej_thr(bi[pp], bj[pp]));
            }
            if (undecided) {
                const float* xi = X + (int64_t)pi[pp] * ldx;
                const float* xj = X + (int64_t)pj[pp] * ldx;
                // the team sums as k_verify's four lanes do
                float s32 = 0.f;
                if (VEC4) {
                    for (int t = tl * 4; t < d; t += VF_TEAM * 4) {
                        const floatx4 u = *reinterpret_cast<const floatx4*>(xi + t);
                        const floatx4 v = *reinterpret_cast<const floatx4*>(xj + t);
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            const float e = u[c] - v[c];
                            s32 = fmaf(e, e, s32);
                        }
                    }
                } else {
                    for (int t = tl; t < d; t += VF_TEAM) {
                        const float e = xi[t] - xj[t];
                        s32 = fmaf(e, e, s32);
                    }
                }
                keep = team_sum(s32) <= eps2;
            }
            keep = keep && tl == 0;
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
            unsigned long long* counter, uint32_t* bad, const uint32_t* run_if = nullptr)
{
    if (vec4)
        hipLaunchKernelGGL((k_verify<METRIC, true>), grid, dim3(VF_THREADS), 0, s, X, n, d, ldx, pairs, m, eps,
                           out, (unsigned long long)cap, counter, bad, run_if);
    else
        hipLaunchKernelGGL((k_verify<METRIC, false>), grid, dim3(VF_THREADS), 0, s, X, n, d, ldx, pairs, m, eps,
                           out, (unsigned long long)cap, counter, bad, run_if);
}

// Workgroups for a list of m pairs: one team slot per pair up to 16 per CU,
// a multiple of the die count.
int64_t verify_blocks(int64_t m, int num_cu)
{
    const int64_t pairs_per_block = VF_THREADS / VF_TEAM * VF_PP;
    int64_t blocks = (m + pairs_per_block - 1) / pairs_per_block;
    const int64_t max_blocks = (int64_t)num_cu * 16;
    if (blocks > max_blocks) blocks = max_blocks;
    return std::max<int64_t>(NUM_XCD, (blocks + NUM_XCD - 1) / NUM_XCD * NUM_XCD);
}

float round_up_f(double v) { return std::nextafter((float)v, __builtin_inff()); }
float round_down_f(double v) { return std::nextafter((float)v, -__builtin_inff()); }

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
    // The FP16 screen pays for rounding the rows once when the list has at
    // least as many pairs as X has rows (and most of them are near: see
    // k_choose_form).
    bool screen = metric == MSM_EUCLIDEAN && m >= n;
    const int64_t ldw = ((int64_t)d + 7) / 8 * 4;  // 32-bit words of an FP16 row
    const size_t bnd_bytes = msm::align_up((size_t)n * sizeof(float), 256);
    void* scr = nullptr;
    st = msm::ctx_scratch(ctx, screen ? 256 + bnd_bytes + (size_t)n * (size_t)ldw * 4 : 256, s, &scr);
    if (st == MSM_E_NOMEM && screen) {
        // no room for the FP16 copy: the FP32 kernel verifies the whole list
        ctx->err.clear();
        screen = false;
        st = msm::ctx_scratch(ctx, 256, s, &scr);
    }
    if (st != MSM_OK) return st;
    unsigned long long* counter = static_cast<unsigned long long*>(scr);
    uint32_t* bad = reinterpret_cast<uint32_t*>(counter + 1);
    uint32_t* run = reinterpret_cast<uint32_t*>(counter + 2);
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, counter, 2);
    const bool vec4 = ((reinterpret_cast<uintptr_t>(X) & 15) == 0) && (ldx % 4 == 0) && (d % 4 == 0);
    const int64_t m0 = screen ? std::min(m, std::max<int64_t>(VH_SAMPLE_MIN, m / VH_SAMPLE_DIV)) : m;
    {
        msm::KernelTimer kt(ctx, s, "k_verify");
        if (metric == MSM_EUCLIDEAN)
            launch<MSM_EUCLIDEAN>(vec4, dim3((unsigned)verify_blocks(m0, ctx->num_cu)), s, X, n, d, ldx, pairs, m0,
                                  eps, out, cap, counter, bad);
        else
            launch<MSM_COSINE>(vec4, dim3((unsigned)verify_blocks(m0, ctx->num_cu)), s, X, n, d, ldx, pairs, m0,
                               eps, out, cap, counter, bad);
    }
    if (m0 < m) {
        const uint32_t* rest = pairs + 2 * m0;
        const int64_t mr = m - m0;
        const dim3 grid((unsigned)verify_blocks(mr, ctx->num_cu));
        hipLaunchKernelGGL(k_choose_form, dim3(1), dim3(64), 0, s, counter, m0, run);
        float* bnd = reinterpret_cast<float*>(static_cast<char*>(scr) + 256);
        uint32_t* Xh = reinterpret_cast<uint32_t*>(static_cast<char*>(scr) + 256 + bnd_bytes);
        {
            msm::KernelTimer kt(ctx, s, "k_half_rows");
            const int64_t hb = std::min<int64_t>((n + VH_ROWS - 1) / VH_ROWS, (int64_t)ctx->num_cu * 32);
            hipLaunchKernelGGL(k_half_rows, dim3((unsigned)hb), dim3(256), 0, s, X, n, d, ldx, vec4 ? 1 : 0, Xh,
                               ldw, bnd, run);
        }
        // gamma: relative error of the FP32 sum, a chain of ldw / 2 fused adds
        // per lane and two team adds, each within one ulp; plus the margin
        // 2^-18 of the threshold products
        const double gam = (double)(ldw + 8) * 0x1p-23 + 0x1p-18;
        const double c = 0x1p-13 * std::sqrt((double)d) * (1.0 + 0x1p-10);
        const double e = (double)eps;
        ScreenConsts kc;
        kc.r1 = round_up_f((1.0 + 0x1p-11) * (1.0 + 0x1p-19));
        kc.r0 = round_up_f((e * (1.0 + 0x1p-11) + c) * (1.0 + 0x1p-19));
        kc.k0 = round_down_f(e * (1.0 - 0x1p-11) - c - 0x1p-19 * (e + c));
        kc.g_up = round_up_f(1.0 + gam);
        kc.g_dn = round_down_f(1.0 - gam);
        {
            msm::KernelTimer kt(ctx, s, "k_verify_h");
            if (vec4)
                hipLaunchKernelGGL((k_verify_h<true>), grid, dim3(VF_THREADS), 0, s, Xh, ldw, bnd, X, n, d,
                                   ldx, rest, mr, eps, kc, out, (unsigned long long)cap, counter, bad, run);
            else
                hipLaunchKernelGGL((k_verify_h<false>), grid, dim3(VF_THREADS), 0, s, Xh, ldw, bnd, X, n,
                                   d, ldx, rest, mr, eps, kc, out, (unsigned long long)cap, counter, bad, run);
        }
        msm::KernelTimer kt(ctx, s, "k_verify");
        launch<MSM_EUCLIDEAN>(vec4, grid, s, X, n, d, ldx, rest, mr, eps, out, cap, counter, bad, run + 1);
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
