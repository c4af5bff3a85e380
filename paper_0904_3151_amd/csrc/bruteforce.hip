// Exhaustive epsilon-neighbour enumeration (Definition 1.1), used as the
// exhaustive reference of the missing-edge ratio (Section 4.2) on a subsample.
//
// The O(n^2) distances come from a Gram matrix on the FP32 matrix cores:
// ||x_i - x_j||^2 = |x_i|^2 + |x_j|^2 - 2 x_i.x_j (cosine: 1 - x_i.x_j /
// (|x_i||x_j|)). That form loses accuracy to cancellation, so it only
// screens: a pair is a candidate when the FP32 value is within eps plus a
// rounding band (below), and every candidate is decided by a direct FP64
// evaluation of the distance from the FP32 inputs. The result therefore
// equals the FP64 definition.
//
// Band: with u = 2^-24, the dot product and the norms each carry at most
// d u (|x_i|^2 + |x_j|^2) error, and forming the sum adds three roundings,
// so |error| <= (2 d + 16) u (|x_i|^2 + |x_j|^2) for Euclidean and
// (2 d + 16) u for the cosine form (relative to |x_i||x_j|).
//
// Tiles: a workgroup of 4 waves computes a 64 x 64 block (i-tile <= j-tile)
// with v_mfma_f32_16x16x4_f32; both operands are rows of X, loaded as float4
// with the same K-order trick as the projection kernel.
#include "msm_internal.h"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int BF_THREADS = 256;
constexpr int BF_TILE = 64;

__global__ __launch_bounds__(256) void k_row_norms(const float* __restrict__ X, int64_t n, int d, int64_t ldx,
                                                   float* __restrict__ nrm)
{
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    float s = 0.f;
    for (int t = lane; t < d; t += 64) {
        const float v = X[i * ldx + t];
        s = fmaf(v, v, s);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) nrm[i] = s;
}

__device__ __forceinline__ double exact_distance(const float* xi, const float* xj, int d, int metric)
{
    if (metric == MSM_EUCLIDEAN) {
        double q = 0.0;
        for (int t = 0; t < d; ++t) {
            const double e = (double)xi[t] - (double)xj[t];
            q = fma(e, e, q);
        }
        return q;  // squared distance
    }
    double xy = 0.0, xx = 0.0, yy = 0.0;
    for (int t = 0; t < d; ++t) {
        const double a = xi[t], b = xj[t];
        xy = fma(a, b, xy);
        xx = fma(a, a, xx);
        yy = fma(b, b, yy);
    }
    if (xx == 0.0 || yy == 0.0) return 1.0;
    return 1.0 - xy / (sqrt(xx) * sqrt(yy));
}

template <int METRIC>
__global__ __launch_bounds__(BF_THREADS) void k_bruteforce(const float* __restrict__ X, int64_t n, int d,
                                                           int64_t ldx, const float* __restrict__ nrm, float eps,
                                                           double eps_cmp, uint32_t* __restrict__ out,
                                                           unsigned long long cap, unsigned long long* counter,
                                                           unsigned long long* screened, int vec4)
{
    const int64_t T = (n + BF_TILE - 1) / BF_TILE;
    const int64_t u = blockIdx.x;
    // (ti, tj), ti <= tj, row-major over the upper triangle with diagonal
    const double q = (double)(2 * T + 1);
    int64_t ti = (int64_t)((q - sqrt(q * q - 8.0 * (double)u)) * 0.5);
    ti = max<int64_t>(0, min<int64_t>(ti, T - 1));
    while (ti < T - 1 && (ti + 1) * (2 * T - ti) / 2 <= u) ++ti;
    while (ti > 0 && ti * (2 * T - ti + 1) / 2 > u) --ti;
    const int64_t tj = ti + (u - ti * (2 * T - ti + 1) / 2);

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int r16 = lane & 15;
    // wave (wr, wc) owns rows i0 + 32 wr .. +31 and columns j0 + 32 wc .. +31
    const int wr = wave >> 1, wc = wave & 1;
    const int64_t i0 = ti * BF_TILE + 32 * wr;
    const int64_t j0 = tj * BF_TILE + 32 * wc;
    if (ti == tj && wc < wr) return;  // block entirely below the diagonal

    floatx4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < d; k0 += 16) {
        const int kb = k0 + 4 * g;
        floatx4 av[2], bv[2];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const int64_t ri = i0 + 16 * rb + r16;
            const int64_t rj = j0 + 16 * rb + r16;
            floatx4 va = floatx4{0.f, 0.f, 0.f, 0.f}, vb = floatx4{0.f, 0.f, 0.f, 0.f};
            if (ri < n) {
                const float* p = X + ri * ldx;
                if (vec4 && kb + 3 < d) {
                    va = *reinterpret_cast<const floatx4*>(p + kb);
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        if (kb + c < d) va[c] = p[kb + c];
                }
            }
            if (rj < n) {
                const float* p = X + rj * ldx;
                if (vec4 && kb + 3 < d) {
                    vb = *reinterpret_cast<const floatx4*>(p + kb);
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        if (kb + c < d) vb[c] = p[kb + c];
                }
            }
            av[rb] = va;
            bv[rb] = vb;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a][c], bv[b][c], acc[a][b], 0, 0, 0);
    }

    const float band_c = (float)(2 * d + 16) * 5.9604645e-08f;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + 16 * a + 4 * g + r;
                const int64_t j = j0 + 16 * b + r16;
                bool cand = i < n && j < n && j > i;
                if (cand) {
                    const float ni = nrm[i], nj = nrm[j], dot = acc[a][b][r];
                    if (METRIC == MSM_EUCLIDEAN) {
                        const float d2 = ni + nj - 2.0f * dot;
                        cand = d2 <= eps * eps + band_c * (ni + nj);
                    } else {
                        const float den = sqrtf(ni) * sqrtf(nj);
                        const float dist = (ni == 0.f || nj == 0.f) ? 1.0f : 1.0f - dot / den;
                        cand = dist <= eps + band_c;
                    }
                }
                bool ok = false;
                if (cand) {
                    atomicAdd(screened, 1ull);
                    const double D = exact_distance(X + i * ldx, X + j * ldx, d, METRIC);
                    ok = D <= eps_cmp;
                }
                const unsigned long long slot = msm::wave_append(ok, counter);
                if (ok && slot < cap)
                    *reinterpret_cast<uint2*>(out + 2 * slot) = make_uint2((uint32_t)i, (uint32_t)j);
            }
}

__global__ void k_zero2(unsigned long long* a)
{
    if (threadIdx.x < 2) a[threadIdx.x] = 0ull;
}

}  // namespace

extern "C" msm_status msm_bruteforce_eps(msm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                                         int32_t metric, float eps, uint32_t* out, int64_t cap, int64_t* m_out,
                                         void* stream)
{
    if (!ctx) return msm::fail(nullptr, MSM_E_INVALID, "msm_bruteforce_eps: ctx is NULL");
    ctx->err.clear();
    if (!m_out) return msm::fail(ctx, MSM_E_INVALID, "msm_bruteforce_eps: m_out is NULL");
    *m_out = 0;
    if (n < 0 || n > 0xFFFFFFFFll || d < 1 || ldx < d || cap < 0)
        return msm::fail(ctx, MSM_E_INVALID, "msm_bruteforce_eps: sizes out of range");
    if (metric != MSM_EUCLIDEAN && metric != MSM_COSINE)
        return msm::fail(ctx, MSM_E_INVALID, "msm_bruteforce_eps: unknown metric %d", metric);
    if (!(eps >= 0.0f) || eps == __builtin_inff())
        return msm::fail(ctx, MSM_E_INVALID, "msm_bruteforce_eps: eps must be finite and >= 0");
    if (cap > 0 && !out) return msm::fail(ctx, MSM_E_INVALID, "msm_bruteforce_eps: out is NULL with cap > 0");
    if (out && (reinterpret_cast<uintptr_t>(out) & 7))
        return msm::fail(ctx, MSM_E_INVALID, "msm_bruteforce_eps: out must be 8-byte aligned");
    if (n < 2) return MSM_OK;
    if (!X) return msm::fail(ctx, MSM_E_INVALID, "msm_bruteforce_eps: X is NULL");
    const int64_t T = (n + BF_TILE - 1) / BF_TILE;
    const int64_t tiles = T * (T + 1) / 2;
    if (tiles > 0x7FFFFFFFll)
        return msm::fail(ctx, MSM_E_UNSUPPORTED, "msm_bruteforce_eps: n=%lld is too large", (long long)n);
    msm_status st = msm::use_device(ctx);
    if (st != MSM_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    msm::Carver cv;
    cv.take<unsigned long long>(2);
    cv.take<float>((size_t)n);
    void* scr = nullptr;
    st = msm::ctx_scratch(ctx, cv.off, s, &scr);
    if (st != MSM_OK) return st;
    msm::Carver c2;
    c2.base = static_cast<char*>(scr);
    unsigned long long* counters = c2.take<unsigned long long>(2);
    float* nrm = c2.take<float>((size_t)n);
    hipLaunchKernelGGL(k_zero2, dim3(1), dim3(64), 0, s, counters);
    {
        msm::KernelTimer kt(ctx, s, "k_row_norms");
        hipLaunchKernelGGL(k_row_norms, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, X, n, d, ldx, nrm);
    }
    const int vec4 = ((reinterpret_cast<uintptr_t>(X) & 15) == 0) && (ldx % 4 == 0);
    const double e64 = (double)eps;
    {
        msm::KernelTimer kt(ctx, s, "k_bruteforce");
        if (metric == MSM_EUCLIDEAN)
            hipLaunchKernelGGL(k_bruteforce<MSM_EUCLIDEAN>, dim3((unsigned)tiles), dim3(BF_THREADS), 0, s, X, n, d,
                               ldx, nrm, eps, e64 * e64, out, (unsigned long long)cap, counters, counters + 1, vec4);
        else
            hipLaunchKernelGGL(k_bruteforce<MSM_COSINE>, dim3((unsigned)tiles), dim3(BF_THREADS), 0, s, X, n, d,
                               ldx, nrm, eps, e64, out, (unsigned long long)cap, counters, counters + 1, vec4);
    }
    MSM_HIP(ctx, hipGetLastError());
    MSM_HIP(ctx, hipMemcpyAsync(ctx->host_words, counters, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    MSM_HIP(ctx, hipStreamSynchronize(s));
    const int64_t m = (int64_t)ctx->host_words[0];
    *m_out = m;
    if (m > cap && !(out == nullptr && cap == 0))
        return msm::fail(ctx, MSM_E_CAPACITY, "msm_bruteforce_eps: %lld pairs do not fit in cap=%lld", (long long)m,
                         (long long)cap);
    return MSM_OK;
}
