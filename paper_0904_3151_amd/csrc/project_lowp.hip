// Random-projection LSH (Section 3.2, eq. (3)) with low-precision products.
//
// z = X R is computed on the gfx950 matrix cores from BF16 or FP8 (e4m3)
// copies of X and R with FP32 accumulation: v_mfma_f32_16x16x32_bf16 or
// v_mfma_f32_16x16x32_fp8_fp8, 32 products deep per instruction. FP8 copies
// are scaled so that each row of X and each column of R spans the format
// (x_t * ia_i, R_tc * ib_c with ia_i = 240 / max_t |x_it|, ib_c = 240 /
// max_t |R_tc|; 240 is finite in both e4m3 encodings); the estimate of z is
// the accumulator divided by ia_i ib_c. A positive scale never changes a
// sign, so only the margin test below uses the scales.
//
// Margin recompute: an entry whose estimate satisfies |z| < tau ||x_i|| is
// recomputed as a plain FP32 dot product and takes its sign from it; every
// other entry takes the sign of the low-precision estimate.
//
// The X operand is read as FP32 and converted in registers, so the kernel
// reads X once from HBM (a first pass over each 16-row block computes the
// row norms and FP8 scales; the second pass finds the rows in cache).
// The K-order trick of the FP32 kernel applies: lane l supplies the values
// for k = k0 + 8 (l / 16) + i, i = 0..7, in both operands.
#include "msm_internal.h"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int LP_THREADS = 256;
constexpr int LP_WAVES = LP_THREADS / 64;
constexpr int LP_LDS_BYTES = 65536;
constexpr float FP8_MAX = 240.0f;
constexpr int LP_RQ = 512;          // recompute queue entries per wave
constexpr int LP_KREG_CHUNKS = 8;   // rows with d <= 256 are held in registers

// One lane's K-slice of the B operand (8 values of column c).
template <int DT>
struct BOp;
template <>
struct BOp<MSM_BF16> {
    typedef bf16x8 T;
};
template <>
struct BOp<MSM_FP8_E4M3> {
    typedef long T;
};

template <int DT>
__device__ __forceinline__ typename BOp<DT>::T pack8(const float (&v)[8], float scale)
{
    if constexpr (DT == MSM_BF16) {
        bf16x8 r;
#pragma unroll
        for (int i = 0; i < 8; ++i) r[i] = (__bf16)v[i];  // round to nearest even
        return r;
    } else {
        int lo = __builtin_amdgcn_cvt_pk_fp8_f32(v[0] * scale, v[1] * scale, 0, false);
        lo = __builtin_amdgcn_cvt_pk_fp8_f32(v[2] * scale, v[3] * scale, lo, true);
        int hi = __builtin_amdgcn_cvt_pk_fp8_f32(v[4] * scale, v[5] * scale, 0, false);
        hi = __builtin_amdgcn_cvt_pk_fp8_f32(v[6] * scale, v[7] * scale, hi, true);
        return (long)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
    }
}

template <int DT>
__device__ __forceinline__ floatx4 mfma(typename BOp<DT>::T a, typename BOp<DT>::T b, floatx4 c)
{
    if constexpr (DT == MSM_BF16)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
}

__global__ void k_lp_zero(unsigned long long* c)
{
    if (threadIdx.x == 0) *c = 0ull;
}

// Column scales of R: ib[c] = 240 / max_t |R_tc| (1 for a zero column).
// One wave per column: lanes stride over t, then a shuffle maximum.
__global__ void k_lp_col_scale(const float* __restrict__ R, int d, int ell, float* __restrict__ ib)
{
    const int c = blockIdx.x;
    const int lane = threadIdx.x;
    float m = 0.f;
    for (int t = lane; t < d; t += 64) m = fmaxf(m, fabsf(R[(int64_t)t * ell + c]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if (lane == 0) ib[c] = m > 0.f ? FP8_MAX / m : 1.0f;
}

// R transposed to ell x d (FP32) for the margin recompute.
__global__ void k_lp_transpose(const float* __restrict__ R, int d, int ell, float* __restrict__ Rt)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= d * ell) return;
    const int c = e / d, t = e % d;
    Rt[e] = R[(int64_t)t * ell + c];
}

// R converted into the B-operand layout: entry (kc * ncb + cb) * 64 + l
// holds R[32 kc + 8 (l / 16) + i][16 cb + l % 16], i = 0..7.
template <int DT>
__global__ void k_lp_prep_r(const float* __restrict__ R, int d, int ell, int ncb, int nkc,
                            const float* __restrict__ ib, typename BOp<DT>::T* __restrict__ Rp)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nkc * ncb * 64) return;
    const int l = e & 63;
    const int cb = (e >> 6) % ncb;
    const int kc = (e >> 6) / ncb;
    const int c = cb * 16 + (l & 15);
    const int kb = kc * 32 + 8 * (l >> 4);
    float v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = (kb + i < d && c < ell) ? R[(int64_t)(kb + i) * ell + c] : 0.0f;
    const float s = (DT == MSM_FP8_E4M3 && c < ell) ? ib[c] : 1.0f;
    Rp[e] = pack8<DT>(v, s);
}

// Recomputes the queued margin entries of one wave as FP32 dot products of
// a row of X and a row of R^T: four teams of 16 lanes, each lane reading
// 16-byte pieces, then a shuffle reduction inside the team. A positive
// result sets the entry's bit in the wave's LDS copy of its output words
// (16 rows x 4 words). Called by the whole wave.
__device__ __forceinline__ void recompute_queue(const float* __restrict__ X, int64_t ldx, int d,
                                                const float* __restrict__ Rt, int64_t row0, int vec4,
                                                const uint32_t* q, uint32_t& qn, unsigned long long* words)
{
    const int lane = __lane_id();
    const int team = lane >> 4, tl = lane & 15;
    const uint32_t cnt = qn;
    for (uint32_t q0 = 0; q0 < cnt; q0 += 4) {
        const uint32_t qi = q0 + team;
        float z = 0.f;
        uint32_t e = 0;
        if (qi < cnt) {
            e = q[qi];
            const int rr = (int)(e >> 8);
            const int c = (int)(e & 0xFF);
            const float* xg = X + (row0 + rr) * ldx;
            const float* rg = Rt + (int64_t)c * d;
            if (vec4) {
                for (int t = 4 * tl; t < d; t += 64) {
                    const floatx4 a = *reinterpret_cast<const floatx4*>(xg + t);
                    const floatx4 b = *reinterpret_cast<const floatx4*>(rg + t);
                    z = fmaf(a[0], b[0], z);
                    z = fmaf(a[1], b[1], z);
                    z = fmaf(a[2], b[2], z);
                    z = fmaf(a[3], b[3], z);
                }
            } else {
                for (int t = tl; t < d; t += 16) z = fmaf(xg[t], rg[t], z);
            }
        }
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) z += __shfl_xor(z, o, 64);
        if (qi < cnt && tl == 0 && z > 0.f) {
            const int rr = (int)(e >> 8), c = (int)(e & 0xFF);
            atomicOr(&words[rr * 4 + (c >> 6)], 1ull << (c & 63));
        }
    }
    qn = 0;
}

template <int DT, int NCB>
__global__ __launch_bounds__(LP_THREADS) void k_project_lp(
    const float* __restrict__ X, int64_t n, int d, int64_t ldx, const float* __restrict__ Rt, int ell,
    const typename BOp<DT>::T* __restrict__ Rp, const float* __restrict__ ib, uint64_t* __restrict__ S, int W,
    int kt_chunks, int nkc, int vec4, float tau, unsigned long long* recomputed)
{
    typedef typename BOp<DT>::T BT;
    extern __shared__ __attribute__((aligned(16))) char lds_raw[];
    BT* Bl = reinterpret_cast<BT*>(lds_raw);  // [kt_chunks][NCB][64]
    // Margin entries of a wave wait in a queue and are recomputed by teams
    // of 16 lanes; the resulting sign bits reach their owners through LDS.
    __shared__ uint32_t rq[LP_WAVES][LP_RQ];
    __shared__ unsigned long long wordsL[LP_WAVES][16 * 4];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int r16 = lane & 15;
    constexpr int ROWS_PER_TILE = LP_WAVES * 16;
    const int64_t ntiles = (n + ROWS_PER_TILE - 1) / ROWS_PER_TILE;
    const int nkt = (nkc + kt_chunks - 1) / kt_chunks;

    auto stage = [&](int kc0) {
        const int cnt = min(kt_chunks, nkc - kc0) * NCB * 64;
        const BT* src = Rp + (size_t)kc0 * NCB * 64;
        for (int e = threadIdx.x; e < cnt; e += LP_THREADS) Bl[e] = src[e];
    };
    if (nkt == 1) {
        stage(0);
        __syncthreads();
    }
    float ibc[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        const int c = cb * 16 + r16;
        ibc[cb] = (DT == MSM_FP8_E4M3 && c < ell) ? ib[c] : 1.0f;
    }

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t row0 = tile * ROWS_PER_TILE + (int64_t)wave * 16;
        const int64_t row = row0 + r16;  // the row whose A values this lane loads
        const float* xr = X + row * ldx;
        const bool rv = row < n;

        floatx4 acc[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[cb] = floatx4{0.f, 0.f, 0.f, 0.f};
        float nrm2 = 0.f, mx = 0.f, ia = 1.0f;
        if (nkc <= LP_KREG_CHUNKS) {
            // The lane's whole slice of the row sits in registers: all its
            // loads are in flight together, and X is read once.
            float xv[LP_KREG_CHUNKS][8];
#pragma unroll
            for (int kc = 0; kc < LP_KREG_CHUNKS; ++kc) {
                const int kb = kc * 32 + 8 * g;
#pragma unroll
                for (int i = 0; i < 8; ++i) xv[kc][i] = 0.f;
                if (kc < nkc && rv) {
                    if (vec4 && kb + 7 < d) {
                        const floatx4 u0 = *reinterpret_cast<const floatx4*>(xr + kb);
                        const floatx4 u1 = *reinterpret_cast<const floatx4*>(xr + kb + 4);
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            xv[kc][i] = u0[i];
                            xv[kc][4 + i] = u1[i];
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < 8; ++i)
                            if (kb + i < d) xv[kc][i] = xr[kb + i];
                    }
                }
            }
#pragma unroll
            for (int kc = 0; kc < LP_KREG_CHUNKS; ++kc)
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    nrm2 = fmaf(xv[kc][i], xv[kc][i], nrm2);
                    mx = fmaxf(mx, fabsf(xv[kc][i]));
                }
            nrm2 += __shfl_xor(nrm2, 16, 64);
            nrm2 += __shfl_xor(nrm2, 32, 64);
            mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
            mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
            ia = (DT == MSM_FP8_E4M3 && mx > 0.f) ? FP8_MAX / mx : 1.0f;
            for (int kt = 0; kt < nkt; ++kt) {
                const int kc0 = kt * kt_chunks;
                if (nkt > 1) {
                    __syncthreads();
                    stage(kc0);
                    __syncthreads();
                }
#pragma unroll
                for (int kc = 0; kc < LP_KREG_CHUNKS; ++kc) {
                    if (kc >= kc0 && kc < min(nkc, kc0 + kt_chunks)) {
                        const BT a = pack8<DT>(xv[kc], ia);
#pragma unroll
                        for (int cb = 0; cb < NCB; ++cb)
                            acc[cb] = mfma<DT>(a, Bl[((kc - kc0) * NCB + cb) * 64 + lane], acc[cb]);
                    }
                }
            }
        } else {
            // pass 1: squared norm and largest magnitude of the row (4 lanes per row)
            if (rv) {
                for (int kb = 8 * g; kb < d; kb += 32) {
                    float v[8];
                    if (vec4 && kb + 7 < d) {
                        const floatx4 u0 = *reinterpret_cast<const floatx4*>(xr + kb);
                        const floatx4 u1 = *reinterpret_cast<const floatx4*>(xr + kb + 4);
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            v[i] = u0[i];
                            v[4 + i] = u1[i];
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < 8; ++i) v[i] = kb + i < d ? xr[kb + i] : 0.f;
                    }
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        nrm2 = fmaf(v[i], v[i], nrm2);
                        mx = fmaxf(mx, fabsf(v[i]));
                    }
                }
            }
            nrm2 += __shfl_xor(nrm2, 16, 64);
            nrm2 += __shfl_xor(nrm2, 32, 64);
            mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
            mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
            ia = (DT == MSM_FP8_E4M3 && mx > 0.f) ? FP8_MAX / mx : 1.0f;
            // pass 2: products, the rows now in cache
            for (int kt = 0; kt < nkt; ++kt) {
                const int kc0 = kt * kt_chunks;
                if (nkt > 1) {
                    __syncthreads();
                    stage(kc0);
                    __syncthreads();
                }
                const int kcn = min(kt_chunks, nkc - kc0);
                for (int kc = 0; kc < kcn; ++kc) {
                    const int kb = (kc0 + kc) * 32 + 8 * g;
                    float v[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) v[i] = 0.f;
                    if (rv) {
                        if (vec4 && kb + 7 < d) {
                            const floatx4 u0 = *reinterpret_cast<const floatx4*>(xr + kb);
                            const floatx4 u1 = *reinterpret_cast<const floatx4*>(xr + kb + 4);
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                v[i] = u0[i];
                                v[4 + i] = u1[i];
                            }
                        } else {
#pragma unroll
                            for (int i = 0; i < 8; ++i)
                                if (kb + i < d) v[i] = xr[kb + i];
                        }
                    }
                    const BT a = pack8<DT>(v, ia);
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb)
                        acc[cb] = mfma<DT>(a, Bl[(kc * NCB + cb) * 64 + lane], acc[cb]);
                }
            }
        }

        // Epilogue: lane l holds z for rows 4 (l / 16) + i, column l % 16 of
        // each 16 x 16 block. For accumulator register i, one ballot gives
        // the signs and one the margin entries (|z| < tau ||x|| ia ib in
        // scaled units); ballot bits 16 q .. 16 q + 15 belong to row
        // 4 q + i. Signs of margin entries are cleared and queued for the
        // FP32 recompute, which sets them in the LDS copy of the words.
        float thr[4];
        bool rowok[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rr = 4 * g + i;
            const float nr2 = __shfl(nrm2, rr, 64);
            const float iar = __shfl(ia, rr, 64);
            thr[i] = tau * sqrtf(nr2) * iar;
            rowok[i] = row0 + rr < n;
        }
        const int orow = lane & 15, oword = lane >> 4;
        uint64_t word = 0;
        uint32_t qn = 0;  // wave-uniform queue length
        unsigned long long nre = 0;
        bool queued = false;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const int c = cb * 16 + r16;
            const bool colok = c < ell;
            uint64_t m[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float zt = acc[cb][i];
                const uint64_t pos = __ballot(zt > 0.f);
                const uint64_t mar = __ballot(rowok[i] && colok && fabsf(zt) < thr[i] * ibc[cb]);
                m[i] = pos & ~mar;
                if (mar) {  // rare: queue this register's margin entries
                    queued = true;
                    if ((mar >> lane) & 1ull) {
                        const uint32_t q = qn + (uint32_t)__popcll(mar & msm::lanemask_lt());
                        rq[wave][q] = ((uint32_t)(4 * g + i) << 8) | (uint32_t)c;
                    }
                    qn += (uint32_t)__popcll(mar);
                }
            }
            const uint64_t mi = m[orow & 3];
            const uint64_t bits = (mi >> (16 * (orow >> 2))) & 0xFFFFull;
            if ((cb >> 2) == oword) word |= bits << (16 * (cb & 3));
            if (qn > LP_RQ - 4 * 64) {  // flush before the queue can overflow
                wordsL[wave][orow * 4 + oword] = word;
                nre += qn;
                recompute_queue(X, ldx, d, Rt, row0, vec4, rq[wave], qn, wordsL[wave]);
                word = wordsL[wave][orow * 4 + oword];
            }
        }
        if (queued) {
            wordsL[wave][orow * 4 + oword] = word;
            nre += qn;
            recompute_queue(X, ldx, d, Rt, row0, vec4, rq[wave], qn, wordsL[wave]);
            word = wordsL[wave][orow * 4 + oword];
        }
        const int64_t grow = row0 + orow;
        if (grow < n && oword < W) S[grow * W + oword] = word;
        if (recomputed && lane == 0 && nre) atomicAdd(recomputed, nre);
    }
}

// Recomputes the queued margin entries of one wave (rows of at most 256
// aligned floats) as FP32 dot products of a row of X and a row of R^T:
// eight teams of eight lanes, each lane with four 16-byte pieces of both
// rows in flight at a time, then a shuffle sum inside the team. A positive
// result sets the entry's bit in the wave's LDS copy of its output words.
// Called by the whole wave.
__device__ __forceinline__ void recompute_queue8(const float* __restrict__ X, int64_t ldx, int d,
                                                 const float* __restrict__ Rt, int64_t row0, const uint32_t* q,
                                                 uint32_t& qn, unsigned long long* words)
{
    const int lane = __lane_id();
    const int team = lane >> 3, tl = lane & 7;
    const uint32_t cnt = qn;
    for (uint32_t q0 = 0; q0 < cnt; q0 += 8) {
        const uint32_t qi = q0 + team;
        const bool ok = qi < cnt;
        const uint32_t e = ok ? q[qi] : 0u;
        const int rr = (int)(e >> 8), c = (int)(e & 0xFF);
        const float* xg = X + (row0 + rr) * ldx;
        const float* rg = Rt + (int64_t)c * d;
        float z = 0.f;
#pragma unroll
        for (int h = 0; h < 2; ++h) {  // two halves of four pieces, all loads of a half in flight
            floatx4 a[4], b[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int t = 4 * tl + 32 * (4 * h + s);
                const bool in = ok && t < d;
                a[s] = in ? *reinterpret_cast<const floatx4*>(xg + t) : floatx4{0.f, 0.f, 0.f, 0.f};
                b[s] = in ? *reinterpret_cast<const floatx4*>(rg + t) : floatx4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                z = fmaf(a[s][0], b[s][0], z);
                z = fmaf(a[s][1], b[s][1], z);
                z = fmaf(a[s][2], b[s][2], z);
                z = fmaf(a[s][3], b[s][3], z);
            }
        }
#pragma unroll
        for (int o = 4; o > 0; o >>= 1) z += __shfl_xor(z, o, 64);
        if (ok && tl == 0 && z > 0.f) atomicOr(&words[rr * 4 + (c >> 6)], 1ull << (c & 63));
    }
    qn = 0;
}

// Rows of at most 256 floats with 16-byte alignment: all of R's operand
// copy stays in LDS for the whole launch (at most 128 KB for BF16), one
// persistent workgroup of LPR_THREADS per CU (two for FP8), and each wave
// requests its next 16 rows as soon as the current rows' products are
// issued, so their loads overlap the epilogue and the margin recompute.
constexpr int LPR_THREADS = 512;
constexpr int LPR_WAVES = LPR_THREADS / 64;
constexpr int LPR_RQ = 512;  // recompute queue entries per wave

template <int DT, int NCB>
__global__ __launch_bounds__(LPR_THREADS) void k_project_lp_res(
    const float* __restrict__ X, int64_t n, int d, int64_t ldx, const float* __restrict__ Rt, int ell,
    const typename BOp<DT>::T* __restrict__ Rp, const float* __restrict__ ib, uint64_t* __restrict__ S, int W,
    int nkc, float tau, unsigned long long* recomputed)
{
    typedef typename BOp<DT>::T BT;
    extern __shared__ __attribute__((aligned(16))) char lds_raw[];
    BT* Bl = reinterpret_cast<BT*>(lds_raw);  // [nkc][NCB][64]
    __shared__ uint32_t rq[LPR_WAVES][LPR_RQ];
    __shared__ unsigned long long wordsL[LPR_WAVES][16 * 4];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int r16 = lane & 15;
    constexpr int ROWS_PER_TILE = LPR_WAVES * 16;
    const int64_t ntiles = (n + ROWS_PER_TILE - 1) / ROWS_PER_TILE;
    {
        const int cnt = nkc * NCB * 64;
        for (int e = threadIdx.x; e < cnt; e += LPR_THREADS) Bl[e] = Rp[e];
    }
    __syncthreads();
    float ibc[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        const int c = cb * 16 + r16;
        ibc[cb] = (DT == MSM_FP8_E4M3 && c < ell) ? ib[c] : 1.0f;
    }
    // the lane's slice of its row: k = 32 kc + 8 g + i
    float xv[LP_KREG_CHUNKS][8];
    auto load_rows = [&](int64_t tile) {
        const int64_t row = tile * ROWS_PER_TILE + (int64_t)wave * 16 + r16;
        const bool rv = tile < ntiles && row < n;
        const float* xr = X + (rv ? row : 0) * ldx;
#pragma unroll
        for (int kc = 0; kc < LP_KREG_CHUNKS; ++kc) {
            const int kb = kc * 32 + 8 * g;
            const bool in = rv && kc < nkc && kb < d;  // d % 4 == 0: kb < d covers kb .. kb + 3
            const floatx4 u0 = in ? *reinterpret_cast<const floatx4*>(xr + kb) : floatx4{0.f, 0.f, 0.f, 0.f};
            const floatx4 u1 =
                (in && kb + 4 < d) ? *reinterpret_cast<const floatx4*>(xr + kb + 4) : floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                xv[kc][i] = u0[i];
                xv[kc][4 + i] = u1[i];
            }
        }
    };
    int64_t tile = blockIdx.x;
    load_rows(tile);
    for (; tile < ntiles; tile += gridDim.x) {
        const int64_t row0 = tile * ROWS_PER_TILE + (int64_t)wave * 16;
        float nrm2 = 0.f, mx = 0.f;
#pragma unroll
        for (int kc = 0; kc < LP_KREG_CHUNKS; ++kc)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                nrm2 = fmaf(xv[kc][i], xv[kc][i], nrm2);
                mx = fmaxf(mx, fabsf(xv[kc][i]));
            }
        nrm2 += __shfl_xor(nrm2, 16, 64);
        nrm2 += __shfl_xor(nrm2, 32, 64);
        mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
        mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
        const float ia = (DT == MSM_FP8_E4M3 && mx > 0.f) ? FP8_MAX / mx : 1.0f;
        floatx4 acc[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[cb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < LP_KREG_CHUNKS; ++kc) {
            if (kc < nkc) {
                const BT a = pack8<DT>(xv[kc], ia);
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) acc[cb] = mfma<DT>(a, Bl[(kc * NCB + cb) * 64 + lane], acc[cb]);
            }
        }
        // the next rows' loads go out before this tile's epilogue
        load_rows(tile + gridDim.x);

        // Epilogue as in k_project_lp: signs by ballot, margin entries
        // (|z| < tau ||x|| in scaled units) queued for the FP32 recompute.
        float thr[4];
        bool rowok[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rr = 4 * g + i;
            const float nr2 = __shfl(nrm2, rr, 64);
            const float iar = __shfl(ia, rr, 64);
            thr[i] = tau * sqrtf(nr2) * iar;
            rowok[i] = row0 + rr < n;
        }
        const int orow = lane & 15, oword = lane >> 4;
        uint64_t word = 0;
        uint32_t qn = 0;  // wave-uniform queue length
        unsigned long long nre = 0;
        bool queued = false;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const int c = cb * 16 + r16;
            const bool colok = c < ell;
            uint64_t m[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float zt = acc[cb][i];
                const uint64_t pos = __ballot(zt > 0.f);
                const uint64_t mar = __ballot(rowok[i] && colok && fabsf(zt) < thr[i] * ibc[cb]);
                m[i] = pos & ~mar;
                if (mar) {
                    queued = true;
                    if ((mar >> lane) & 1ull) {
                        const uint32_t q = qn + (uint32_t)__popcll(mar & msm::lanemask_lt());
                        rq[wave][q] = ((uint32_t)(4 * g + i) << 8) | (uint32_t)c;
                    }
                    qn += (uint32_t)__popcll(mar);
                }
            }
            const uint64_t mi = m[orow & 3];
            const uint64_t bits = (mi >> (16 * (orow >> 2))) & 0xFFFFull;
            if ((cb >> 2) == oword) word |= bits << (16 * (cb & 3));
            if (qn > LPR_RQ - 4 * 64) {  // flush before the queue can overflow
                wordsL[wave][orow * 4 + oword] = word;
                nre += qn;
                recompute_queue8(X, ldx, d, Rt, row0, rq[wave], qn, wordsL[wave]);
                word = wordsL[wave][orow * 4 + oword];
            }
        }
        if (queued) {
            wordsL[wave][orow * 4 + oword] = word;
            nre += qn;
            recompute_queue8(X, ldx, d, Rt, row0, rq[wave], qn, wordsL[wave]);
            word = wordsL[wave][orow * 4 + oword];
        }
        const int64_t grow = row0 + orow;
        if (grow < n && oword < W) S[grow * W + oword] = word;
        if (recomputed && lane == 0 && nre) atomicAdd(recomputed, nre);
    }
}

template <int DT, int NCB>
msm_status launch_lp(msm_ctx* ctx, const float* X, int64_t n, int d, int64_t ldx, const float* R, int ell,
                     float tau, uint64_t* S, int64_t* n_recomputed, hipStream_t stream)
{
    typedef typename BOp<DT>::T BT;
    const int W = (ell + 63) / 64;
    const int nkc = (d + 31) / 32;
    const int max_chunks = max(1, (int)(LP_LDS_BYTES / (NCB * 64 * sizeof(BT))));
    const int kt_chunks = min(nkc, max_chunks);
    const size_t lds = (size_t)kt_chunks * NCB * 64 * sizeof(BT);
    msm::Carver cv;
    cv.take<unsigned long long>(1);
    cv.take<float>((size_t)NCB * 16);
    cv.take<BT>((size_t)nkc * NCB * 64);
    cv.take<float>((size_t)ell * d);
    void* scr = nullptr;
    msm_status st = msm::ctx_scratch(ctx, cv.off, stream, &scr);
    if (st != MSM_OK) return st;
    msm::Carver c2;
    c2.base = static_cast<char*>(scr);
    unsigned long long* counter = c2.take<unsigned long long>(1);
    float* ib = c2.take<float>((size_t)NCB * 16);
    BT* Rp = c2.take<BT>((size_t)nkc * NCB * 64);
    float* Rt = c2.take<float>((size_t)ell * d);
    hipLaunchKernelGGL(k_lp_zero, dim3(1), dim3(64), 0, stream, counter);
    {
        msm::KernelTimer kt(ctx, stream, "k_lp_prep_r");
        if (DT == MSM_FP8_E4M3)
            hipLaunchKernelGGL(k_lp_col_scale, dim3(ell), dim3(64), 0, stream, R, d, ell, ib);
        const int ne = nkc * NCB * 64;
        hipLaunchKernelGGL((k_lp_prep_r<DT>), dim3((ne + 255) / 256), dim3(256), 0, stream, R, d, ell, NCB, nkc,
                           (const float*)ib, Rp);
        hipLaunchKernelGGL(k_lp_transpose, dim3((d * ell + 255) / 256), dim3(256), 0, stream, R, d, ell, Rt);
    }
    const int vec4 = ((reinterpret_cast<uintptr_t>(X) & 15) == 0) && (ldx % 4 == 0) && (d % 4 == 0);
    const size_t lds_res = (size_t)nkc * NCB * 64 * sizeof(BT);
    if (vec4 && nkc <= LP_KREG_CHUNKS) {
        // R resident in LDS; one workgroup per CU, two when R is small
        const void* f = reinterpret_cast<const void*>(&k_project_lp_res<DT, NCB>);
        MSM_HIP(ctx, hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_res));
        const int per_cu = lds_res <= 64 * 1024 ? 2 : 1;
        const int64_t ntiles = (n + LPR_WAVES * 16 - 1) / (LPR_WAVES * 16);
        const int64_t cap = (int64_t)ctx->num_cu * per_cu;
        const int64_t grid = ntiles < cap ? ntiles : cap;
        msm::KernelTimer kt(ctx, stream, DT == MSM_BF16 ? "k_project_bf16" : "k_project_fp8");
        hipLaunchKernelGGL((k_project_lp_res<DT, NCB>), dim3((unsigned)grid), dim3(LPR_THREADS), lds_res, stream, X,
                           n, d, ldx, (const float*)Rt, ell, (const BT*)Rp, (const float*)ib, S, W, nkc, tau,
                           n_recomputed ? counter : nullptr);
    } else {
        const int64_t ntiles = (n + LP_WAVES * 16 - 1) / (LP_WAVES * 16);
        const int64_t grid = ntiles < (int64_t)ctx->num_cu * 4 ? ntiles : (int64_t)ctx->num_cu * 4;
        msm::KernelTimer kt(ctx, stream, DT == MSM_BF16 ? "k_project_bf16" : "k_project_fp8");
        hipLaunchKernelGGL((k_project_lp<DT, NCB>), dim3((unsigned)grid), dim3(LP_THREADS), lds, stream, X, n, d,
                           ldx, (const float*)Rt, ell, (const BT*)Rp, (const float*)ib, S, W, kt_chunks, nkc, vec4, tau,
                           n_recomputed ? counter : nullptr);
    }
    MSM_HIP(ctx, hipGetLastError());
    if (n_recomputed) {
        MSM_HIP(ctx, hipMemcpyAsync(ctx->host_words, counter, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                    stream));
        MSM_HIP(ctx, hipStreamSynchronize(stream));
        *n_recomputed = (int64_t)ctx->host_words[0];
    }
    return MSM_OK;
}

template <int DT>
msm_status dispatch_lp(msm_ctx* ctx, const float* X, int64_t n, int d, int64_t ldx, const float* R, int ell,
                       float tau, uint64_t* S, int64_t* n_recomputed, hipStream_t s)
{
    switch ((ell + 15) / 16) {
        case 1: return launch_lp<DT, 1>(ctx, X, n, d, ldx, R, ell, tau, S, n_recomputed, s);
        case 2: return launch_lp<DT, 2>(ctx, X, n, d, ldx, R, ell, tau, S, n_recomputed, s);
        case 3: return launch_lp<DT, 3>(ctx, X, n, d, ldx, R, ell, tau, S, n_recomputed, s);
        case 4: return launch_lp<DT, 4>(ctx, X, n, d, ldx, R, ell, tau, S, n_recomputed, s);
        case 5: return launch_lp<DT, 5>(ctx, X, n, d, ldx, R, ell, tau, S, n_recomputed, s);
        case 6: return launch_lp<DT, 6>(ctx, X, n, d, ldx, R, ell, tau, S, n_recomputed, s);
        case 7: return launch_lp<DT, 7>(ctx, X, n, d, ldx, R, ell, tau, S, n_recomputed, s);
        case 8: return launch_lp<DT, 8>(ctx, X, n, d, ldx, R, ell, tau, S, n_recomputed, s);
        case 9: return launch_lp<DT, 9>(ctx, X, n, d, ldx, R, ell, tau, S, n_recomputed, s);
        case 10: return launch_lp<DT, 10>(ctx, X, n, d, ldx, R, ell, tau, S, n_recomputed, s);
        case 11: return launch_lp<DT, 11>(ctx, X, n, d, ldx, R, ell, tau, S, n_recomputed, s);
        case 12: return launch_lp<DT, 12>(ctx, X, n, d, ldx, R, ell, tau, S, n_recomputed, s);
        case 13: return launch_lp<DT, 13>(ctx, X, n, d, ldx, R, ell, tau, S, n_recomputed, s);
        case 14: return launch_lp<DT, 14>(ctx, X, n, d, ldx, R, ell, tau, S, n_recomputed, s);
        case 15: return launch_lp<DT, 15>(ctx, X, n, d, ldx, R, ell, tau, S, n_recomputed, s);
        default: return launch_lp<DT, 16>(ctx, X, n, d, ldx, R, ell, tau, S, n_recomputed, s);
    }
}

}  // namespace

extern "C" msm_status msm_project_lowp(msm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                                       const float* R, int32_t ell, int32_t dtype, float tau, uint64_t* S,
                                       int64_t* n_recomputed, void* stream)
{
    if (!ctx) return msm::fail(nullptr, MSM_E_INVALID, "msm_project_lowp: ctx is NULL");
    ctx->err.clear();
    if (n_recomputed) *n_recomputed = 0;
    if (n < 0 || n > 0xFFFFFFFFll)
        return msm::fail(ctx, MSM_E_INVALID, "msm_project_lowp: n=%lld out of range", (long long)n);
    if (d < 1 || ldx < d)
        return msm::fail(ctx, MSM_E_INVALID, "msm_project_lowp: need d >= 1 and ldx >= d");
    if (ell < 1 || ell > 256)
        return msm::fail(ctx, MSM_E_INVALID, "msm_project_lowp: ell=%d not in [1, 256]", ell);
    if (dtype != MSM_BF16 && dtype != MSM_FP8_E4M3)
        return msm::fail(ctx, MSM_E_INVALID, "msm_project_lowp: dtype %d is not BF16 or FP8_E4M3", dtype);
    if (!(tau >= 0.0f) || tau == __builtin_inff())
        return msm::fail(ctx, MSM_E_INVALID, "msm_project_lowp: tau must be finite and >= 0");
    if (n == 0) return MSM_OK;
    if (!X || !R || !S) return msm::fail(ctx, MSM_E_INVALID, "msm_project_lowp: NULL X, R or S");
    msm_status st = msm::use_device(ctx);
    if (st != MSM_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (dtype == MSM_BF16) return dispatch_lp<MSM_BF16>(ctx, X, n, d, ldx, R, ell, tau, S, n_recomputed, s);
    return dispatch_lp<MSM_FP8_E4M3>(ctx, X, n, d, ldx, R, ell, tau, S, n_recomputed, s);
}
