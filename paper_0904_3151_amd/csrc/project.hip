// Random-projection LSH (Section 3.2, eq. (3)) on the gfx950 matrix cores.
//
// z = X R is computed with v_mfma_f32_16x16x4_f32 (FP32 products, FP32
// accumulation); bit c of string i is 1 iff z_ic > 0. The sign test and the
// packing into 64-bit words happen in registers: one wave ballot per
// accumulator register turns 64 comparisons into a scalar mask, so z never
// reaches memory.
//
// Work split: a workgroup of 4 waves owns tiles of 4 * RB * 16 rows and all
// ell columns (ell <= 256, in NCB blocks of 16). R is staged in LDS in the
// exact register layout of the MFMA B operand (one 16-byte read per lane per
// 16-deep K chunk); workgroups are persistent, so R is staged once per
// workgroup when it fits in 64 KB and once per row tile otherwise.
//
// Split-BF16 form (d <= 256 when R's three parts fit in LDS): each FP32
// value v is written as hi + mid + lo with hi = bf16(v), mid = bf16(v - hi),
// lo = bf16(v - hi - mid) (both differences are exact in FP32), so the three
// parts carry v to about 24 bits. z = sum of the six products whose parts
// are not both small (hi hi, hi mid, mid hi, mid mid, hi lo, lo hi) on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation; the dropped terms are
// below 2^-24 of |x_t R_tc| each, the order of FP32 rounding itself, and the
// BF16 matrix cores do the six products in about a third of the time of
// one FP32 product.
//
// K-order trick: in a 16-deep chunk lane l loads the four consecutive
// values X[row][k0 + 4g .. k0 + 4g + 3] (g = l / 16) with one 16-byte load,
// and MFMA j (j = 0..3) consumes component j. The MFMA's internal k index g
// therefore stands for the true index k0 + 4g + j, and the B operand in LDS
// is laid out with the same mapping, so the chunk's sum covers all 16 k.
#include "msm_internal.h"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int PJ_THREADS = 256;
constexpr int PJ_WAVES = PJ_THREADS / 64;
constexpr int PJ_LDS_BYTES = 65536;

// Rl[(kc * NCB + cb) * 64 + l][j] = R[k0 + 16 kc + 4 (l / 16) + j][16 cb + l % 16]
template <int NCB>
__device__ __forceinline__ void stage_r(floatx4* Rl, const float* __restrict__ R, int d, int ell, int k0,
                                        int kt_chunks)
{
    const int total = kt_chunks * NCB * 64;
    for (int e = threadIdx.x; e < total; e += PJ_THREADS) {
        const int l = e & 63;
        const int cb = (e >> 6) % NCB;
        const int kc = (e >> 6) / NCB;
        const int c = cb * 16 + (l & 15);
        const int kb = k0 + kc * 16 + 4 * (l >> 4);
        floatx4 v;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = kb + j;
            v[j] = (k < d && c < ell) ? R[(int64_t)k * ell + c] : 0.0f;
        }
        Rl[e] = v;
    }
}

// One tile of 4 * RB * 16 rows starting at row_tile (rows at or above
// row_end are skipped): z = X R on the MFMA, signs packed into S (and into
// S2 when it is not NULL). With nkt == 1 the caller has staged all of R in
// Rl; otherwise R is staged here kt_rows at a time. Called by every thread.
template <int NCB, int RB>
__device__ __forceinline__ void project_tile(const float* __restrict__ X, int64_t row_tile, int64_t row_end, int d,
                                             int64_t ldx, const float* __restrict__ R, int ell,
                                             uint64_t* __restrict__ S, uint64_t* __restrict__ S2, int W,
                                             int kt_rows, int nkt, int vec4, floatx4* Rl)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int r16 = lane & 15;
    const int kt_chunks = kt_rows / 16;
    const int64_t row_w = row_tile + (int64_t)wave * RB * 16;
    floatx4 acc[RB][NCB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = floatx4{0.f, 0.f, 0.f, 0.f};

    for (int kt = 0; kt < nkt; ++kt) {
        const int k0 = kt * kt_rows;
        if (nkt > 1) {
            __syncthreads();
            stage_r<NCB>(Rl, R, d, ell, k0, kt_chunks);
            __syncthreads();
        }
        const int kcn = min(kt_chunks, (d - k0 + 15) / 16);
        // X values of chunk kc; the next chunk's are requested before this
        // chunk's products
        auto load_a = [&](int kc, floatx4 (&a)[RB]) {
            const int kbase = k0 + kc * 16 + 4 * g;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const int64_t row = row_w + rb * 16 + r16;
                floatx4 v = floatx4{0.f, 0.f, 0.f, 0.f};
                if (row < row_end) {
                    const float* xr = X + row * ldx;
                    if (vec4 && kbase + 3 < d) {
                        v = *reinterpret_cast<const floatx4*>(xr + kbase);
                    } else {
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            if (kbase + j < d) v[j] = xr[kbase + j];
                    }
                }
                a[rb] = v;
            }
        };
        floatx4 an[RB];
        if (kcn > 0) load_a(0, an);
        for (int kc = 0; kc < kcn; ++kc) {
            floatx4 a[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) a[rb] = an[rb];
            if (kc + 1 < kcn) load_a(kc + 1, an);
            floatx4 b[NCB];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) b[cb] = Rl[(kc * NCB + cb) * 64 + lane];
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][j], b[cb][j], acc[rb][cb], 0, 0, 0);
        }
    }

    // Epilogue. Accumulator register i of lane l holds z for row
    // 4 (l / 16) + i and column l % 16 of the 16 x 16 block, so
    // ballot(acc[i] > 0) gives, in bits 16 q .. 16 q + 15, the 16 signs
    // of row 4 q + i. Lane l then assembles word l / 16 of row l % 16.
    const int orow = lane & 15;
    const int oword = lane >> 4;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        uint64_t word = 0;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const uint64_t m0 = __ballot(acc[rb][cb][0] > 0.0f);
            const uint64_t m1 = __ballot(acc[rb][cb][1] > 0.0f);
            const uint64_t m2 = __ballot(acc[rb][cb][2] > 0.0f);
            const uint64_t m3 = __ballot(acc[rb][cb][3] > 0.0f);
            const int i = orow & 3;
            const uint64_t mi = i == 0 ? m0 : (i == 1 ? m1 : (i == 2 ? m2 : m3));
            const uint64_t bits = (mi >> (16 * (orow >> 2))) & 0xFFFFull;
            if ((cb >> 2) == oword) word |= bits << (16 * (cb & 3));
        }
        const int64_t row = row_w + rb * 16 + orow;
        if (row < row_end && oword < W) {
            S[row * W + oword] = word;
            if (S2) S2[row * W + oword] = word;
        }
    }
}

template <int NCB, int RB>
__global__ __launch_bounds__(PJ_THREADS) void k_project_f32(
    const float* __restrict__ X, int64_t n, int d, int64_t ldx, const float* __restrict__ R,
    int ell, uint64_t* __restrict__ S, int W, int kt_rows, int vec4)
{
    extern __shared__ floatx4 Rl[];  // [kt_rows / 16][NCB][64]
    constexpr int ROWS_PER_TILE = PJ_WAVES * RB * 16;
    const int64_t ntiles = (n + ROWS_PER_TILE - 1) / ROWS_PER_TILE;
    const int nkt = (d + kt_rows - 1) / kt_rows;
    if (nkt == 1) {
        stage_r<NCB>(Rl, R, d, ell, 0, kt_rows / 16);
        __syncthreads();
    }
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
        project_tile<NCB, RB>(X, tile * ROWS_PER_TILE, n, d, ldx, R, ell, S, nullptr, W, kt_rows, nkt, vec4, Rl);
}

// Batched projection: workgroups claim entries (a run of rows of one
// instance) from a counter (*work, zero at launch), so that entries of
// different d even out; R of the entry's instance is staged once per entry,
// only as deep as its d.
template <int NCB, int RB>
__global__ __launch_bounds__(PJ_THREADS) void k_project_batch(const msm::ProjInst* __restrict__ inst,
                                                              const msm::ProjEntry* __restrict__ entries,
                                                              int nentries, int ell, int W, int kt_rows,
                                                              unsigned int* __restrict__ work)
{
    extern __shared__ floatx4 Rl[];
    __shared__ int s_entry;
    constexpr int ROWS_PER_TILE = PJ_WAVES * RB * 16;
    for (;;) {
        __syncthreads();  // the previous entry is done with Rl and s_entry
        if (threadIdx.x == 0) s_entry = (int)atomicAdd(work, 1u);
        __syncthreads();
        const int e = s_entry;
        if (e >= nentries) break;
        const msm::ProjEntry en = entries[e];
        const msm::ProjInst& in = inst[en.inst];
        const int d = in.d;
        const int nkt = (d + kt_rows - 1) / kt_rows;
        if (nkt == 1) {
            stage_r<NCB>(Rl, in.R, d, ell, 0, (d + 15) / 16);
            __syncthreads();
        }
        const int64_t end = en.row0 + en.rows;
        for (int64_t r0 = en.row0; r0 < end; r0 += ROWS_PER_TILE)
            project_tile<NCB, RB>(in.X, r0, end, d, in.ldx, in.R, ell, in.S, in.S2, W, kt_rows, nkt, in.vec4, Rl);
    }
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int X3_THREADS = 512;
constexpr int X3_WAVES = X3_THREADS / 64;
constexpr int X3_CHUNKS = 8;                 // 32-deep chunks: d <= 256
constexpr int X3_LDS_BYTES = 144 * 1024;     // the three parts of R
constexpr int X3_MAX_NCB = 8;                // ell <= 128
constexpr int X3_RB4 = 2;                    // row blocks per wave when d <= 128

__device__ __forceinline__ void split3(const float (&v)[8], bf16x8& h, bf16x8& m, bf16x8& l)
{
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const __bf16 a = (__bf16)v[i];
        const float r1 = v[i] - (float)a;
        const __bf16 b = (__bf16)r1;
        const float r2 = r1 - (float)b;
        h[i] = a;
        m[i] = b;
        l[i] = (__bf16)r2;
    }
}

// Persistent workgroups of X3_WAVES waves, 16 * RB rows per wave and all
// ell columns (NCB blocks of 16). The parts of R sit in LDS in the B-operand
// layout: entry (kc * NCB + cb) * 64 + l holds R[32 kc + 8 (l / 16) + i]
// [16 cb + l % 16], i = 0..7; lane l supplies X[row l % 16][32 kc +
// 8 (l / 16) + i], so each MFMA sums one 32-deep chunk, and each B read
// serves the wave's RB row blocks. A wave keeps its lane's slices of the
// rows (KC chunks of 8 values) in registers and requests the next tile's
// slices before the current tile's products.
template <int NCB, int KC, int RB>
__global__ __launch_bounds__(X3_THREADS) void k_project_x3(const float* __restrict__ X, int64_t n, int d,
                                                           int64_t ldx, const float* __restrict__ R, int ell,
                                                           uint64_t* __restrict__ S, int W, int nkc, int vec4)
{
    extern __shared__ __attribute__((aligned(16))) char x3_lds[];
    const int per = nkc * NCB * 64;
    bf16x8* Bh = reinterpret_cast<bf16x8*>(x3_lds);
    bf16x8* Bm = Bh + per;
    bf16x8* Bl = Bm + per;
    for (int e = threadIdx.x; e < per; e += X3_THREADS) {
        const int l = e & 63;
        const int cb = (e >> 6) % NCB;
        const int kc = (e >> 6) / NCB;
        const int c = cb * 16 + (l & 15);
        const int kb = kc * 32 + 8 * (l >> 4);
        float v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = (kb + i < d && c < ell) ? R[(int64_t)(kb + i) * ell + c] : 0.0f;
        bf16x8 h, m, lo;
        split3(v, h, m, lo);
        Bh[e] = h;
        Bm[e] = m;
        Bl[e] = lo;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int r16 = lane & 15;
    constexpr int ROWS_PER_TILE = X3_WAVES * 16 * RB;
    const int64_t ntiles = (n + ROWS_PER_TILE - 1) / ROWS_PER_TILE;
    auto load_rows = [&](int64_t tile, float (&xv)[RB][KC][8]) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const int64_t row = tile * ROWS_PER_TILE + ((int64_t)wave * RB + rb) * 16 + r16;
            const bool rv = tile < ntiles && row < n;
            const float* xr = X + (rv ? row : 0) * ldx;
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                const int kb = kc * 32 + 8 * g;
#pragma unroll
                for (int i = 0; i < 8; ++i) xv[rb][kc][i] = 0.f;
                if (kc < nkc && rv) {
                    if (vec4 && kb + 7 < d) {
                        const floatx4 u0 = *reinterpret_cast<const floatx4*>(xr + kb);
                        const floatx4 u1 = *reinterpret_cast<const floatx4*>(xr + kb + 4);
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            xv[rb][kc][i] = u0[i];
                            xv[rb][kc][4 + i] = u1[i];
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < 8; ++i)
                            if (kb + i < d) xv[rb][kc][i] = xr[kb + i];
                    }
                }
            }
        }
    };
    float xn[RB][KC][8];
    if ((int64_t)blockIdx.x < ntiles) load_rows(blockIdx.x, xn);
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        float xv[RB][KC][8];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int kc = 0; kc < KC; ++kc)
#pragma unroll
                for (int i = 0; i < 8; ++i) xv[rb][kc][i] = xn[rb][kc][i];
        if (tile + gridDim.x < ntiles) load_rows(tile + gridDim.x, xn);
        floatx4 acc[RB][NCB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            if (kc < nkc) {
                bf16x8 ah[RB], am[RB], al[RB];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) split3(xv[rb][kc], ah[rb], am[rb], al[rb]);
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) {
                    const int e = (kc * NCB + cb) * 64 + lane;
                    const bf16x8 bh = Bh[e], bm = Bm[e], bl = Bl[e];
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) {
                        // the small terms first
                        floatx4 a = acc[rb][cb];
                        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[rb], bh, a, 0, 0, 0);
                        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rb], bl, a, 0, 0, 0);
                        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[rb], bm, a, 0, 0, 0);
                        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[rb], bh, a, 0, 0, 0);
                        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rb], bm, a, 0, 0, 0);
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rb], bh, a, 0, 0, 0);
                    }
                }
            }
        }
        // signs: the accumulator layout is that of the FP32 kernel
        const int orow = lane & 15;
        const int oword = lane >> 4;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            uint64_t word = 0;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const uint64_t m0 = __ballot(acc[rb][cb][0] > 0.0f);
                const uint64_t m1 = __ballot(acc[rb][cb][1] > 0.0f);
                const uint64_t m2 = __ballot(acc[rb][cb][2] > 0.0f);
                const uint64_t m3 = __ballot(acc[rb][cb][3] > 0.0f);
                const int i = orow & 3;
                const uint64_t mi = i == 0 ? m0 : (i == 1 ? m1 : (i == 2 ? m2 : m3));
                const uint64_t bits = (mi >> (16 * (orow >> 2))) & 0xFFFFull;
                if ((cb >> 2) == oword) word |= bits << (16 * (cb & 3));
            }
            const int64_t grow = tile * ROWS_PER_TILE + ((int64_t)wave * RB + rb) * 16 + orow;
            if (grow < n && oword < W) S[grow * W + oword] = word;
        }
    }
}

// Launches k_project_x3 with the chunk count that covers d and the row
// blocks per wave that fit the registers.
template <int NCB, int KC, int RB>
msm_status launch_x3(msm_ctx* ctx, const float* X, int64_t n, int d, int64_t ldx, const float* R, int ell,
                     uint64_t* S, int nkc, size_t lds3, hipStream_t stream)
{
    constexpr int ROWS3 = X3_WAVES * 16 * RB;
    const int W = (ell + 63) / 64;
    const int vec4 = ((reinterpret_cast<uintptr_t>(X) & 15) == 0) && (ldx % 4 == 0);
    const int64_t ntiles = (n + ROWS3 - 1) / ROWS3;
    const int64_t grid = ntiles < (int64_t)ctx->num_cu ? ntiles : (int64_t)ctx->num_cu;
    if (lds3 > 65536)
        MSM_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(&k_project_x3<NCB, KC, RB>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, X3_LDS_BYTES));
    {
        msm::KernelTimer kt(ctx, stream, "k_project_x3");
        hipLaunchKernelGGL((k_project_x3<NCB, KC, RB>), dim3((unsigned)grid), dim3(X3_THREADS), lds3, stream, X, n,
                           d, ldx, R, ell, S, W, nkc, vec4);
    }
    MSM_HIP(ctx, hipGetLastError());
    return MSM_OK;
}

// Batched projection in the split form (three BF16 parts, six products per
// FP32 product, as k_project_x3) for ell <= 128 when the parts of R fit in
// LDS: workgroups claim entries (runs of rows of one instance) from a
// device counter as k_project_batch does, split the entry's instance's R
// into LDS as deep as its d, and each wave takes 16 rows at a time.
constexpr int BX3_THREADS = 256;
constexpr int BX3_WAVES = BX3_THREADS / 64;

template <int NCB, int KC>
__global__ __launch_bounds__(BX3_THREADS) void k_project_batch_x3(const msm::ProjInst* __restrict__ inst,
                                                                  const msm::ProjEntry* __restrict__ entries,
                                                                  int nentries, int ell, int W,
                                                                  unsigned int* __restrict__ work)
{
    extern __shared__ __attribute__((aligned(16))) char bx3_lds[];
    __shared__ int s_entry;
    constexpr int PER = KC * NCB * 64;
    bf16x8* Bh = reinterpret_cast<bf16x8*>(bx3_lds);
    bf16x8* Bm = Bh + PER;
    bf16x8* Bl = Bm + PER;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    const int r16 = lane & 15;
    constexpr int ROWS_PER_TILE = BX3_WAVES * 16;
    for (;;) {
        __syncthreads();  // the previous entry is done with the parts and s_entry
        if (threadIdx.x == 0) s_entry = (int)atomicAdd(work, 1u);
        __syncthreads();
        const int e = s_entry;
        if (e >= nentries) break;
        const msm::ProjEntry en = entries[e];
        const msm::ProjInst& in = inst[en.inst];
        const int d = in.d;
        const int nkc = (d + 31) / 32;
        // the instance's R in the B-operand layout of k_project_x3
        for (int q = threadIdx.x; q < nkc * NCB * 64; q += BX3_THREADS) {
            const int l = q & 63;
            const int cb = (q >> 6) % NCB;
            const int kc = (q >> 6) / NCB;
            const int c = cb * 16 + (l & 15);
            const int kb = kc * 32 + 8 * (l >> 4);
            float v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = (kb + i < d && c < ell) ? in.R[(int64_t)(kb + i) * ell + c] : 0.0f;
            bf16x8 h, m, lo;
            split3(v, h, m, lo);
            Bh[q] = h;
            Bm[q] = m;
            Bl[q] = lo;
        }
        __syncthreads();
        const int64_t end = en.row0 + en.rows;
        // the lane's slice of its row of the tile at r0 (zero past the
        // entry's rows and past d)
        auto load_rows = [&](int64_t r0, float (&xv)[KC][8]) {
            const int64_t row = r0 + (int64_t)wave * 16 + r16;
            const bool rv = row < end;
            const float* xr = in.X + (rv ? row : 0) * in.ldx;
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                const int kb = kc * 32 + 8 * g;
#pragma unroll
                for (int i = 0; i < 8; ++i) xv[kc][i] = 0.f;
                if (kc < nkc && rv) {
                    if (in.vec4 && kb + 7 < d) {
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
        };
        float xn[KC][8];
        load_rows(en.row0, xn);
        for (int64_t r0 = en.row0; r0 < end; r0 += ROWS_PER_TILE) {
            float xv[KC][8];
#pragma unroll
            for (int kc = 0; kc < KC; ++kc)
#pragma unroll
                for (int i = 0; i < 8; ++i) xv[kc][i] = xn[kc][i];
            // the next tile's rows are requested before this tile's products
            if (r0 + ROWS_PER_TILE < end) load_rows(r0 + ROWS_PER_TILE, xn);
            floatx4 acc[NCB];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[cb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                if (kc < nkc) {
                    bf16x8 ah, am, al;
                    split3(xv[kc], ah, am, al);
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb) {
                        const int q = (kc * NCB + cb) * 64 + lane;
                        const bf16x8 bh = Bh[q], bm = Bm[q], bl = Bl[q];
                        // the small terms first, as k_project_x3
                        floatx4 a = acc[cb];
                        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, a, 0, 0, 0);
                        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, a, 0, 0, 0);
                        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm, a, 0, 0, 0);
                        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh, a, 0, 0, 0);
                        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm, a, 0, 0, 0);
                        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, a, 0, 0, 0);
                    }
                }
            }
            const int orow = lane & 15;
            const int oword = lane >> 4;
            uint64_t word = 0;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const uint64_t m0 = __ballot(acc[cb][0] > 0.0f);
                const uint64_t m1 = __ballot(acc[cb][1] > 0.0f);
                const uint64_t m2 = __ballot(acc[cb][2] > 0.0f);
                const uint64_t m3 = __ballot(acc[cb][3] > 0.0f);
                const int i = orow & 3;
                const uint64_t mi = i == 0 ? m0 : (i == 1 ? m1 : (i == 2 ? m2 : m3));
                const uint64_t bits = (mi >> (16 * (orow >> 2))) & 0xFFFFull;
                if ((cb >> 2) == oword) word |= bits << (16 * (cb & 3));
            }
            const int64_t grow = r0 + (int64_t)wave * 16 + orow;
            if (grow < end && oword < W) {
                in.S[grow * W + oword] = word;
                if (in.S2) in.S2[grow * W + oword] = word;
            }
        }
    }
}

template <int NCB>
msm_status launch_project(msm_ctx* ctx, const float* X, int64_t n, int d, int64_t ldx,
                          const float* R, int ell, uint64_t* S, hipStream_t stream)
{
    // the split form for ell <= 128 (wider rows would not keep the X slice,
    // the next tile's slice and the accumulators in registers)
    const int nkc = (d + 31) / 32;
    const size_t lds3 = (size_t)3 * nkc * NCB * 64 * sizeof(bf16x8);
    if constexpr (NCB <= X3_MAX_NCB) {
        if (nkc <= 4 && lds3 <= (size_t)X3_LDS_BYTES)
            return launch_x3<NCB, 4, X3_RB4>(ctx, X, n, d, ldx, R, ell, S, nkc, lds3, stream);
        if (nkc <= X3_CHUNKS && lds3 <= (size_t)X3_LDS_BYTES)
            return launch_x3<NCB, X3_CHUNKS, 1>(ctx, X, n, d, ldx, R, ell, S, nkc, lds3, stream);
    }
    constexpr int RB = NCB <= 4 ? 4 : (NCB <= 8 ? 2 : 1);
    constexpr int ROWS_PER_TILE = PJ_WAVES * RB * 16;
    const int W = (ell + 63) / 64;
    const int dpad = (d + 15) / 16 * 16;
    const int max_chunks = PJ_LDS_BYTES / (NCB * 64 * 16);
    const int kt_rows = min(dpad, max_chunks * 16);
    const size_t lds = (size_t)(kt_rows / 16) * NCB * 64 * sizeof(floatx4);
    const int vec4 = ((reinterpret_cast<uintptr_t>(X) & 15) == 0) && (ldx % 4 == 0);
    const int64_t ntiles = (n + ROWS_PER_TILE - 1) / ROWS_PER_TILE;
    const int64_t grid = ntiles < (int64_t)ctx->num_cu * 2 ? ntiles : (int64_t)ctx->num_cu * 2;
    {
        msm::KernelTimer kt(ctx, stream, "k_project_f32");
        hipLaunchKernelGGL((k_project_f32<NCB, RB>), dim3((unsigned)grid), dim3(PJ_THREADS), lds, stream,
                           X, n, d, ldx, R, ell, S, W, kt_rows, vec4);
    }
    MSM_HIP(ctx, hipGetLastError());
    return MSM_OK;
}

}  // namespace

extern "C" msm_status msm_project(msm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                                  const float* R, int32_t ell, uint64_t* S, void* stream)
{
    if (!ctx) return msm::fail(nullptr, MSM_E_INVALID, "msm_project: ctx is NULL");
    ctx->err.clear();
    if (n < 0 || n > 0xFFFFFFFFll)
        return msm::fail(ctx, MSM_E_INVALID, "msm_project: n=%lld out of range", (long long)n);
    if (d < 1 || ldx < d)
        return msm::fail(ctx, MSM_E_INVALID, "msm_project: need d >= 1 and ldx >= d (d=%d, ldx=%lld)",
                         d, (long long)ldx);
    if (ell < 1 || ell > 256)
        return msm::fail(ctx, MSM_E_INVALID, "msm_project: ell=%d not in [1, 256]", ell);
    if (n == 0) return MSM_OK;
    if (!X || !R || !S) return msm::fail(ctx, MSM_E_INVALID, "msm_project: NULL X, R or S");
    msm_status st = msm::use_device(ctx);
    if (st != MSM_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    switch ((ell + 15) / 16) {
        case 1: return launch_project<1>(ctx, X, n, d, ldx, R, ell, S, s);
        case 2: return launch_project<2>(ctx, X, n, d, ldx, R, ell, S, s);
        case 3: return launch_project<3>(ctx, X, n, d, ldx, R, ell, S, s);
        case 4: return launch_project<4>(ctx, X, n, d, ldx, R, ell, S, s);
        case 5: return launch_project<5>(ctx, X, n, d, ldx, R, ell, S, s);
        case 6: return launch_project<6>(ctx, X, n, d, ldx, R, ell, S, s);
        case 7: return launch_project<7>(ctx, X, n, d, ldx, R, ell, S, s);
        case 8: return launch_project<8>(ctx, X, n, d, ldx, R, ell, S, s);
        case 9: return launch_project<9>(ctx, X, n, d, ldx, R, ell, S, s);
        case 10: return launch_project<10>(ctx, X, n, d, ldx, R, ell, S, s);
        case 11: return launch_project<11>(ctx, X, n, d, ldx, R, ell, S, s);
        case 12: return launch_project<12>(ctx, X, n, d, ldx, R, ell, S, s);
        case 13: return launch_project<13>(ctx, X, n, d, ldx, R, ell, S, s);
        case 14: return launch_project<14>(ctx, X, n, d, ldx, R, ell, S, s);
        case 15: return launch_project<15>(ctx, X, n, d, ldx, R, ell, S, s);
        default: return launch_project<16>(ctx, X, n, d, ldx, R, ell, S, s);
    }
}

namespace {

// Row blocks per wave of the batched projection (measured on the batched
// mix of d = 32, 64 and 128: at ell <= 64 one block per wave and more
// workgroups per CU beat the single projection's four blocks).
constexpr int batch_rb(int ncb) { return ncb <= 4 ? 1 : (ncb <= 8 ? 2 : 1); }

template <int NCB>
hipError_t launch_batch(const msm::ProjInst* inst, const msm::ProjEntry* entries, int nentries, int ell,
                        int max_d, int grid, unsigned int* work, hipStream_t stream)
{
    // the split form when the parts of R fit in LDS for the deepest instance
    if constexpr (NCB <= X3_MAX_NCB) {
        const int kc = max_d <= 128 ? 4 : (max_d <= 256 ? 8 : 0);
        const size_t lds3 = (size_t)3 * kc * NCB * 64 * sizeof(bf16x8);
        if (kc && lds3 <= (size_t)X3_LDS_BYTES) {
            const int W = (ell + 63) / 64;
            if (kc == 4) {
                if (lds3 > 65536)
                    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_project_batch_x3<NCB, 4>),
                                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds3);
                hipLaunchKernelGGL((k_project_batch_x3<NCB, 4>), dim3((unsigned)grid), dim3(BX3_THREADS), lds3,
                                   stream, inst, entries, nentries, ell, W, work);
            } else {
                if (lds3 > 65536)
                    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_project_batch_x3<NCB, 8>),
                                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds3);
                hipLaunchKernelGGL((k_project_batch_x3<NCB, 8>), dim3((unsigned)grid), dim3(BX3_THREADS), lds3,
                                   stream, inst, entries, nentries, ell, W, work);
            }
            return hipGetLastError();
        }
    }
    constexpr int RB = batch_rb(NCB);
    const int W = (ell + 63) / 64;
    const int dpad = (max_d + 15) / 16 * 16;
    const int max_chunks = PJ_LDS_BYTES / (NCB * 64 * 16);
    const int kt_rows = min(dpad, max_chunks * 16);
    const size_t lds = (size_t)(kt_rows / 16) * NCB * 64 * sizeof(floatx4);
    hipLaunchKernelGGL((k_project_batch<NCB, RB>), dim3((unsigned)grid), dim3(PJ_THREADS), lds, stream, inst,
                       entries, nentries, ell, W, kt_rows, work);
    return hipGetLastError();
}

}  // namespace

namespace msm {

int batch_project_rows(int ell)
{
    const int ncb = (ell + 15) / 16;
    return PJ_WAVES * 16 * batch_rb(ncb);
}

hipError_t batch_project(const ProjInst* inst, const ProjEntry* entries, int nentries, int ell, int max_d, int grid,
                         unsigned int* work, hipStream_t stream)
{
    switch ((ell + 15) / 16) {
        case 1: return launch_batch<1>(inst, entries, nentries, ell, max_d, grid, work, stream);
        case 2: return launch_batch<2>(inst, entries, nentries, ell, max_d, grid, work, stream);
        case 3: return launch_batch<3>(inst, entries, nentries, ell, max_d, grid, work, stream);
        case 4: return launch_batch<4>(inst, entries, nentries, ell, max_d, grid, work, stream);
        case 5: return launch_batch<5>(inst, entries, nentries, ell, max_d, grid, work, stream);
        case 6: return launch_batch<6>(inst, entries, nentries, ell, max_d, grid, work, stream);
        case 7: return launch_batch<7>(inst, entries, nentries, ell, max_d, grid, work, stream);
        case 8: return launch_batch<8>(inst, entries, nentries, ell, max_d, grid, work, stream);
        case 9: return launch_batch<9>(inst, entries, nentries, ell, max_d, grid, work, stream);
        case 10: return launch_batch<10>(inst, entries, nentries, ell, max_d, grid, work, stream);
        case 11: return launch_batch<11>(inst, entries, nentries, ell, max_d, grid, work, stream);
        case 12: return launch_batch<12>(inst, entries, nentries, ell, max_d, grid, work, stream);
        case 13: return launch_batch<13>(inst, entries, nentries, ell, max_d, grid, work, stream);
        case 14: return launch_batch<14>(inst, entries, nentries, ell, max_d, grid, work, stream);
        case 15: return launch_batch<15>(inst, entries, nentries, ell, max_d, grid, work, stream);
        default: return launch_batch<16>(inst, entries, nentries, ell, max_d, grid, work, stream);
    }
}

}  // namespace msm
