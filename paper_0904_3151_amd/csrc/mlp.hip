// Learned projection: a two-layer network in place of the random projection
// (Section 6 of the paper names non-random hashing as a replacement for it).
//
//   a1 = x W1 + b1,  g = GELU(a1),  a2 = g W2 + b2,  u = tanh(a2),
//   bit c of x's string is 1 iff a2_c > 0 (the sign, as in eq. (3)).
//
// Parameters are one packed FP32 vector [W1 (d x hid) | b1 | W2 (hid x ell) |
// b2], row-major. Every product runs on the matrix cores in BF16
// (v_mfma_f32_16x16x32_bf16) with FP32 accumulation: weights and
// activations are rounded to BF16 when they are staged, the FP32 master
// parameters are what Adam updates.
//
// Training loss over labelled pairs (y = 1 for an epsilon-pair), with the
// relaxed Hamming distance D = (ell - u_i . u_j) / 2 (the Hamming distance of
// the sign strings when u is +-1):
//   mean over pairs of  y relu(D - h/2)^2 + (1 - y) relu(3h - D)^2
//                       + lam (sum_c (1 - |u_ic|)^2 + sum_c (1 - |u_jc|)^2)
#include "msm_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float gelu(float a) { return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float a)
{
    return 0.5f * (1.0f + erff(a * 0.70710678118654752f)) + a * expf(-0.5f * a * a) * 0.3989422804014327f;
}

__device__ __forceinline__ floatx4 mfma_bf16(bf16x8 a, bf16x8 b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ----------------------------------------------------------------------
// Generic strided GEMM, used by training and by inference shapes the fused
// kernel does not take.

constexpr int GT = 64;  // block tile (rows and columns)
constexpr int GK = 32;  // K per stage (one bf16 MFMA)
constexpr int G_THREADS = 256;

enum Epi {
    EPI_BIAS_GELU = 1,     // C = acc + bias (a1), C2 = GELU(a1)
    EPI_BIAS_TANH = 2,     // C = tanh(acc + bias)
    EPI_MUL_GELUGRAD = 3,  // C = acc * GELU'(aux)
    EPI_ATOMIC = 4,        // C += acc (split K)
    EPI_SIGNPACK = 5       // bit (m, n) of S set iff acc + bias > 0
};

struct GemmArgs {
    int M, N, K;
    const float* A;  // A(m, k) = A[m * sam + k * sak]
    int64_t sam, sak;
    const float* B;  // B(k, n) = B[k * sbk + n * sbn]
    int64_t sbk, sbn;
    float* C;        // C(m, n) = C[m * ldc + n]
    int64_t ldc;
    float* C2;       // second output of EPI_BIAS_GELU (ldc layout)
    const float* bias;
    const float* aux;  // a1 for EPI_MUL_GELUGRAD (ldc layout)
    uint64_t* S;       // EPI_SIGNPACK strings, W words per row
    int W;
    int ksplit;        // K range per blockIdx.z
};

// C = A B. A workgroup owns a 64 x 64 tile, wave (wr, wc) a 32 x 32 quarter
// of 2 x 2 MFMA blocks. A and B are staged through LDS in operand layout (A
// as [row][k], B as [col][k]) so that each lane reads its 8 K-values with one
// 16-byte load.
template <int EPI>
__global__ __launch_bounds__(G_THREADS) void k_gemm_bf16(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) __bf16 As[GT][GK + 8];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[GT][GK + 8];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int kbeg = blockIdx.z * g.ksplit;
    const int kend = min(g.K, kbeg + g.ksplit);
    floatx4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = kbeg; k0 < kend; k0 += GK) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < GT * GK / G_THREADS; ++r) {
            const int e = threadIdx.x + r * G_THREADS;
            // consecutive threads walk the unit-stride dimension of each operand
            int am, ak;
            if (g.sak == 1) {
                am = e / GK;
                ak = e % GK;
            } else {
                am = e % GT;
                ak = e / GT;
            }
            const int gm = m0 + am, gk = k0 + ak;
            const float av = (gm < g.M && gk < kend) ? g.A[(int64_t)gm * g.sam + (int64_t)gk * g.sak] : 0.f;
            As[am][ak] = (__bf16)av;
            int bk, bn;
            if (g.sbn == 1) {
                bn = e % GT;
                bk = e / GT;
            } else {
                bk = e % GK;
                bn = e / GK;
            }
            const int gn = n0 + bn, gk2 = k0 + bk;
            const float bv = (gn < g.N && gk2 < kend) ? g.B[(int64_t)gk2 * g.sbk + (int64_t)gn * g.sbn] : 0.f;
            Bs[bn][bk] = (__bf16)bv;
        }
        __syncthreads();
        const int kk = 8 * (lane >> 4);
        bf16x8 av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = *reinterpret_cast<const bf16x8*>(&As[32 * wr + 16 * a + (lane & 15)][kk]);
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = *reinterpret_cast<const bf16x8*>(&Bs[32 * wc + 16 * b + (lane & 15)][kk]);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = mfma_bf16(av[a], bv[b], acc[a][b]);
    }

    // lane holds rows 4 (lane / 16) + i, column lane % 16 of each 16 x 16 block
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = m0 + 32 * wr + 16 * a + 4 * (lane >> 4) + i;
                const int n = n0 + 32 * wc + 16 * b + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                const float v = acc[a][b][i];
                const int64_t o = (int64_t)m * g.ldc + n;
                if (EPI == EPI_BIAS_GELU) {
                    const float a1 = v + g.bias[n];
                    g.C[o] = a1;
                    g.C2[o] = gelu(a1);
                } else if (EPI == EPI_BIAS_TANH) {
                    g.C[o] = tanhf(v + g.bias[n]);
                } else if (EPI == EPI_MUL_GELUGRAD) {
                    g.C[o] = v * gelu_grad(g.aux[o]);
                } else if (EPI == EPI_ATOMIC) {
                    atomicAdd(g.C + o, v);
                } else if (EPI == EPI_SIGNPACK) {
                    if (v + g.bias[n] > 0.f)
                        atomicOr(reinterpret_cast<unsigned long long*>(g.S + (int64_t)m * g.W + (n >> 6)),
                                 1ull << (n & 63));
                }
            }
}

template <int EPI>
void gemm(hipStream_t s, GemmArgs a, int splits = 1)
{
    a.ksplit = splits > 1 ? ((a.K + splits - 1) / splits + GK - 1) / GK * GK : a.K;
    const int z = splits > 1 ? (a.K + a.ksplit - 1) / a.ksplit : 1;
    dim3 grid((a.N + GT - 1) / GT, (a.M + GT - 1) / GT, z);
    hipLaunchKernelGGL((k_gemm_bf16<EPI>), grid, dim3(G_THREADS), 0, s, a);
}

// ----------------------------------------------------------------------
// Fused inference: x -> bits for a 256-row tile per workgroup, with the
// hidden layer produced and consumed 64 units at a time in LDS. Each wave
// owns 32 rows: its slice of X stays in registers as BF16 MFMA operands,
// the 32 x ell output accumulates in registers across the hidden chunks.
// Weights are pre-packed in BF16 operand layout and staged per chunk.

constexpr int FU_THREADS = 512;
constexpr int FU_ROWS = 256;  // 8 waves x 32 rows
constexpr int FU_HC = 64;     // hidden units per chunk
constexpr int FU_MAXKD = 8;   // d <= 256
constexpr int FU_MAXNB = 8;   // ell <= 128
constexpr int FU_PAD = 8;     // bf16 elements of row padding in LDS

struct Packed {
    const __bf16* W1p;  // [chunk][64 hidden][Kp]   (Kp = 32 KD)
    const __bf16* W2p;  // [chunk][Np][64 hidden]   (Np = 16 NB)
    const float* b1p;   // [chunk * 64]
    const float* b2p;   // [Np]
};

// Rounds W1, W2 to BF16 into the fused kernel's operand layout, zero-padded
// to whole chunks, K steps and column blocks.
__global__ void k_mlp_pack(const float* __restrict__ params, int d, int hid, int ell, int KD, int nch, int NB,
                           __bf16* __restrict__ W1p, __bf16* __restrict__ W2p, float* __restrict__ b1p,
                           float* __restrict__ b2p)
{
    const float* W1 = params;
    const float* b1 = W1 + (int64_t)d * hid;
    const float* W2 = b1 + hid;
    const float* b2 = W2 + (int64_t)hid * ell;
    const int Kp = 32 * KD, Np = 16 * NB;
    const int64_t n1 = (int64_t)nch * FU_HC * Kp, n2 = (int64_t)nch * Np * FU_HC;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n1) {
        const int k = (int)(e % Kp);
        const int64_t jc = e / Kp;  // chunk * 64 + j = hidden unit
        W1p[e] = (__bf16)((k < d && jc < hid) ? W1[(int64_t)k * hid + jc] : 0.f);
    } else if (e < n1 + n2) {
        const int64_t f = e - n1;
        const int k = (int)(f % FU_HC);
        const int64_t cn = f / FU_HC;
        const int nn = (int)(cn % Np);
        const int64_t c = cn / Np;
        const int64_t hu = c * FU_HC + k;
        W2p[f] = (__bf16)((hu < hid && nn < ell) ? W2[hu * ell + nn] : 0.f);
    } else if (e < n1 + n2 + (int64_t)nch * FU_HC) {
        const int64_t j = e - n1 - n2;
        b1p[j] = j < hid ? b1[j] : 0.f;
    } else if (e < n1 + n2 + (int64_t)nch * FU_HC + Np) {
        const int nn = (int)(e - n1 - n2 - (int64_t)nch * FU_HC);
        b2p[nn] = nn < ell ? b2[nn] : 0.f;
    }
}

template <int KD, int NB, bool VEC>
__global__ __launch_bounds__(FU_THREADS) void k_mlp_fused(const float* __restrict__ X, int64_t n, int d, int64_t ldx,
                                                          Packed P, int nch, int W, uint64_t* __restrict__ S)
{
    constexpr int Kp = 32 * KD, Np = 16 * NB;
    constexpr int L1 = Kp + FU_PAD, L2 = FU_HC + FU_PAD;
    extern __shared__ __attribute__((aligned(16))) char fu_lds[];
    __bf16* W1s = reinterpret_cast<__bf16*>(fu_lds);   // [64][L1]
    __bf16* W2s = W1s + FU_HC * L1;                    // [Np][L2]
    __bf16* Gs = W2s + Np * L2;                        // [8 waves][32][L2]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * FU_ROWS + 32 * wave;
    __bf16* Gw = Gs + wave * 32 * L2;

    // the wave's 32 rows as A operands: row 16a + lane % 16, k = 32 ks + 8 (lane / 16) + 0..7
    bf16x8 xa[2][KD];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int64_t r = row0 + 16 * a + (lane & 15);
        const bool rok = r < n;
        const float* xr = X + (rok ? r : 0) * ldx;
#pragma unroll
        for (int ks = 0; ks < KD; ++ks) {
            const int k = 32 * ks + 8 * (lane >> 4);
            float v[8];
            if (VEC) {
                float4 p = rok ? *reinterpret_cast<const float4*>(xr + k) : float4{0.f, 0.f, 0.f, 0.f};
                float4 q = rok ? *reinterpret_cast<const float4*>(xr + k + 4) : float4{0.f, 0.f, 0.f, 0.f};
                v[0] = p.x; v[1] = p.y; v[2] = p.z; v[3] = p.w;
                v[4] = q.x; v[5] = q.y; v[6] = q.z; v[7] = q.w;
            } else {
#pragma unroll
                for (int t = 0; t < 8; ++t) v[t] = (rok && k + t < d) ? xr[k + t] : 0.f;
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) xa[a][ks][t] = (__bf16)v[t];
        }
    }

    floatx4 u[2][NB];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) u[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};

    // The next chunk's weights are fetched into registers while the current
    // one is multiplied, then written to LDS at the top of the next step.
    constexpr int N1 = FU_HC * Kp / 8, N2 = Np * FU_HC / 8;  // 16-byte pieces
    constexpr int R1 = (N1 + FU_THREADS - 1) / FU_THREADS, R2 = (N2 + FU_THREADS - 1) / FU_THREADS;
    uint4 p1[R1], p2[R2];
    auto fetch = [&](int c) {
        const uint4* s1 = reinterpret_cast<const uint4*>(P.W1p + (int64_t)c * FU_HC * Kp);
        const uint4* s2 = reinterpret_cast<const uint4*>(P.W2p + (int64_t)c * Np * FU_HC);
#pragma unroll
        for (int r = 0; r < R1; ++r) {
            const int e = threadIdx.x + r * FU_THREADS;
            p1[r] = e < N1 ? s1[e] : uint4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int r = 0; r < R2; ++r) {
            const int e = threadIdx.x + r * FU_THREADS;
            p2[r] = e < N2 ? s2[e] : uint4{0u, 0u, 0u, 0u};
        }
    };
    fetch(0);
    for (int c = 0; c < nch; ++c) {
        __syncthreads();  // the previous chunk is no longer read from LDS
#pragma unroll
        for (int r = 0; r < R1; ++r) {
            const int e = threadIdx.x + r * FU_THREADS;
            if (e < N1) *reinterpret_cast<uint4*>(W1s + (e / (Kp / 8)) * L1 + (e % (Kp / 8)) * 8) = p1[r];
        }
#pragma unroll
        for (int r = 0; r < R2; ++r) {
            const int e = threadIdx.x + r * FU_THREADS;
            if (e < N2) *reinterpret_cast<uint4*>(W2s + (e / (FU_HC / 8)) * L2 + (e % (FU_HC / 8)) * 8) = p2[r];
        }
        if (c + 1 < nch) fetch(c + 1);
        __syncthreads();
        // hidden pre-activations of the wave's rows for the chunk's 64 units
        floatx4 hacc[2][4];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) hacc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KD; ++ks)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const bf16x8 wb =
                    *reinterpret_cast<const bf16x8*>(W1s + (16 * b + (lane & 15)) * L1 + 32 * ks + 8 * (lane >> 4));
#pragma unroll
                for (int a = 0; a < 2; ++a) hacc[a][b] = mfma_bf16(xa[a][ks], wb, hacc[a][b]);
            }
        // bias and GELU, rounded to BF16 into the wave's LDS slice [row][unit]
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const float bias = P.b1p[c * FU_HC + 16 * b + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    Gw[(16 * a + 4 * (lane >> 4) + i) * L2 + 16 * b + (lane & 15)] = (__bf16)gelu(hacc[a][b][i] + bias);
        }
        __syncthreads();
        // output accumulation over the chunk's 64 hidden units
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            bf16x8 ga[2];
#pragma unroll
            for (int a = 0; a < 2; ++a)
                ga[a] = *reinterpret_cast<const bf16x8*>(Gw + (16 * a + (lane & 15)) * L2 + 32 * ks + 8 * (lane >> 4));
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const bf16x8 wb =
                    *reinterpret_cast<const bf16x8*>(W2s + (16 * b + (lane & 15)) * L2 + 32 * ks + 8 * (lane >> 4));
#pragma unroll
                for (int a = 0; a < 2; ++a) u[a][b] = mfma_bf16(ga[a], wb, u[a][b]);
            }
        }
    }

    // signs: a ballot over a 16 x 16 block gives, in bits 16q..16q+15, row
    // 4q + i of the block's 16 columns; lane l stores word l / 32 of row l % 32
    const int my_row = lane & 31, my_w = lane >> 5;
    uint64_t out = 0;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            uint64_t wq[4][2] = {{0ull, 0ull}, {0ull, 0ull}, {0ull, 0ull}, {0ull, 0ull}};
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const float bias = P.b2p[16 * b + (lane & 15)];
                const uint64_t m = __ballot(u[a][b][i] + bias > 0.f);
#pragma unroll
                for (int q = 0; q < 4; ++q) wq[q][b >> 2] |= ((m >> (16 * q)) & 0xFFFFull) << (16 * (b & 3));
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int w = 0; w < 2; ++w)
                    if (my_row == 16 * a + 4 * q + i && my_w == w) out = wq[q][w];
        }
    const int64_t r = row0 + my_row;
    if (r < n && my_w < W) S[r * W + my_w] = out;
}

size_t fused_lds_bytes(int KD, int NB)
{
    return sizeof(__bf16) * ((size_t)FU_HC * (32 * KD + FU_PAD) + (size_t)16 * NB * (FU_HC + FU_PAD) +
                             (size_t)(FU_THREADS / 64) * 32 * (FU_HC + FU_PAD));
}

template <int KD, int NB, bool VEC>
hipError_t launch_fused_kd_nb(hipStream_t s, const float* X, int64_t n, int d, int64_t ldx, Packed P, int nch, int W,
                              uint64_t* S)
{
    const size_t lds = fused_lds_bytes(KD, NB);
    if (lds > 65536) {  // above the default dynamic LDS limit of a launch
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mlp_fused<KD, NB, VEC>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const unsigned grid = (unsigned)((n + FU_ROWS - 1) / FU_ROWS);
    hipLaunchKernelGGL((k_mlp_fused<KD, NB, VEC>), dim3(grid), dim3(FU_THREADS), lds, s, X, n, d, ldx, P, nch, W,
                       S);
    return hipGetLastError();
}

template <int KD, bool VEC>
hipError_t launch_fused_kd(hipStream_t s, int NB, const float* X, int64_t n, int d, int64_t ldx, Packed P, int nch,
                           int W, uint64_t* S)
{
    // NB is rounded up to an even count, so at most four instances per KD
    if (NB <= 2) return launch_fused_kd_nb<KD, 2, VEC>(s, X, n, d, ldx, P, nch, W, S);
    if (NB <= 4) return launch_fused_kd_nb<KD, 4, VEC>(s, X, n, d, ldx, P, nch, W, S);
    if (NB <= 6) return launch_fused_kd_nb<KD, 6, VEC>(s, X, n, d, ldx, P, nch, W, S);
    return launch_fused_kd_nb<KD, 8, VEC>(s, X, n, d, ldx, P, nch, W, S);
}

template <bool VEC>
hipError_t launch_fused(hipStream_t s, int KD, int NB, const float* X, int64_t n, int d, int64_t ldx, Packed P,
                        int nch, int W, uint64_t* S)
{
    if (KD <= 2) return launch_fused_kd<2, VEC>(s, NB, X, n, d, ldx, P, nch, W, S);
    if (KD <= 4) return launch_fused_kd<4, VEC>(s, NB, X, n, d, ldx, P, nch, W, S);
    return launch_fused_kd<8, VEC>(s, NB, X, n, d, ldx, P, nch, W, S);
}

int fused_kd(int d) { return d <= 64 ? 2 : (d <= 128 ? 4 : 8); }
int fused_nb(int ell)
{
    const int nb = (ell + 15) / 16;
    return nb <= 2 ? 2 : (nb <= 4 ? 4 : (nb <= 6 ? 6 : 8));
}

// ----------------------------------------------------------------------
// Training pieces

// Rows of X listed in idx, copied into a dense (P x d) block.
__global__ void k_gather_rows(const float* __restrict__ X, int64_t ldx, int d, const uint32_t* __restrict__ idx,
                              int64_t P, float* __restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * d) return;
    const int64_t r = e / d;
    const int c = (int)(e % d);
    out[e] = X[(int64_t)idx[r] * ldx + c];
}

// Counts the listed indices that are not below n.
__global__ void k_check_index(const uint32_t* __restrict__ idx, int64_t count, int64_t n,
                              unsigned long long* __restrict__ bad)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool b = e < count && (int64_t)idx[e] >= n;
    const uint64_t m = __ballot(b);
    if (m && (int)(threadIdx.x & 63) == __builtin_ctzll(m)) atomicAdd(bad, (unsigned long long)__popcll(m));
}

// Loss of each pair and its gradient with respect to a2 (one wave per pair;
// rows 2p and 2p + 1 of U are the pair's points). The batch mean's terms are
// accumulated into *loss_acc.
__global__ __launch_bounds__(256) void k_pair_loss(const float* __restrict__ U, int ell, int B,
                                                   const float* __restrict__ labels, float h, float lam,
                                                   float* __restrict__ dA2, double* loss_acc)
{
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= B) return;
    const float* ui = U + (int64_t)(2 * p) * ell;
    const float* uj = U + (int64_t)(2 * p + 1) * ell;
    float dot = 0.f, qi = 0.f, qj = 0.f;
    for (int c = lane; c < ell; c += 64) {
        const float a = ui[c], b = uj[c];
        dot = fmaf(a, b, dot);
        qi += (1.f - fabsf(a)) * (1.f - fabsf(a));
        qj += (1.f - fabsf(b)) * (1.f - fabsf(b));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        dot += __shfl_xor(dot, o, 64);
        qi += __shfl_xor(qi, o, 64);
        qj += __shfl_xor(qj, o, 64);
    }
    const float y = labels[p];
    const float D = 0.5f * ((float)ell - dot);
    const float rp = fmaxf(D - 0.5f * h, 0.f);
    const float rn = fmaxf(3.f * h - D, 0.f);
    const float invB = 1.0f / (float)B;
    const float dD = (2.f * y * rp - 2.f * (1.f - y) * rn) * invB;
    const float lr = lam * invB;
    float* gi = dA2 + (int64_t)(2 * p) * ell;
    float* gj = dA2 + (int64_t)(2 * p + 1) * ell;
    for (int c = lane; c < ell; c += 64) {
        const float a = ui[c], b = uj[c];
        const float sa = (float)((a > 0.f) - (a < 0.f)), sb = (float)((b > 0.f) - (b < 0.f));
        const float dua = -0.5f * dD * b - 2.f * lr * (1.f - fabsf(a)) * sa;
        const float dub = -0.5f * dD * a - 2.f * lr * (1.f - fabsf(b)) * sb;
        gi[c] = dua * (1.f - a * a);
        gj[c] = dub * (1.f - b * b);
    }
    if (lane == 0)
        atomicAdd(loss_acc, (double)((y * rp * rp + (1.f - y) * rn * rn + lam * (qi + qj)) * invB));
}

// Column sums of a (P x N) row-major block, added into out.
__global__ void k_colsum(const float* __restrict__ A, int64_t P, int N, int64_t rows_per_block,
                         float* __restrict__ out)
{
    const int nn = blockIdx.x * blockDim.x + threadIdx.x;
    if (nn >= N) return;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per_block;
    const int64_t r1 = min(P, r0 + rows_per_block);
    float s = 0.f;
    for (int64_t r = r0; r < r1; ++r) s += A[r * N + nn];
    atomicAdd(out + nn, s);
}

__global__ void k_fill(float* a, int64_t n, float v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ void k_fill_u64(uint64_t* a, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0ull;
}

__global__ void k_fill_d(double* a, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0.0;
}

// Adam (Kingma and Ba) on the packed FP32 parameters; c1 and c2 are the
// bias corrections 1 - beta1^t and 1 - beta2^t.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

unsigned blocks(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

int64_t n_params(int d, int hid, int ell) { return (int64_t)d * hid + hid + (int64_t)hid * ell + ell; }

msm_status check_shape(msm_ctx* ctx, const char* fn, int64_t n, int d, int64_t ldx, int hid, int ell)
{
    if (n < 0 || n > 0xFFFFFFFFll || d < 1 || d > 65536 || ldx < d || hid < 1 || hid > 65536 || ell < 1 ||
        ell > 256)
        return msm::fail(ctx, MSM_E_INVALID, "%s: sizes out of range (n=%lld d=%d ldx=%lld hid=%d ell=%d)", fn,
                         (long long)n, d, (long long)ldx, hid, ell);
    return MSM_OK;
}

// Device buffers of one training batch of B pairs (P = 2B rows).
struct TrainBufs {
    float *Xb, *A1, *G, *U, *dA2, *dA1;
};

size_t train_carve(msm::Carver& cv, int64_t P, int d, int hid, int ell, TrainBufs* tb)
{
    tb->Xb = cv.take<float>((size_t)P * d);
    tb->A1 = cv.take<float>((size_t)P * hid);
    tb->G = cv.take<float>((size_t)P * hid);
    tb->U = cv.take<float>((size_t)P * ell);
    tb->dA2 = cv.take<float>((size_t)P * ell);
    tb->dA1 = cv.take<float>((size_t)P * hid);
    return cv.off;
}

// Enqueues loss and gradient of one batch. Indices must have been checked.
void launch_loss_grad(hipStream_t s, const float* X, int d, int64_t ldx, const float* params, int hid, int ell,
                      const uint32_t* pairs, const float* labels, int B, float h, float lam, float* grad,
                      double* loss, const TrainBufs& t)
{
    const int64_t P = 2ll * B;
    const float* W1 = params;
    const float* b1 = W1 + (int64_t)d * hid;
    const float* W2 = b1 + hid;
    const float* b2 = W2 + (int64_t)hid * ell;
    float* gW1 = grad;
    float* gb1 = gW1 + (int64_t)d * hid;
    float* gW2 = gb1 + hid;
    float* gb2 = gW2 + (int64_t)hid * ell;
    const int64_t np = n_params(d, hid, ell);
    hipLaunchKernelGGL(k_fill, dim3(blocks(np)), dim3(256), 0, s, grad, np, 0.f);
    hipLaunchKernelGGL(k_gather_rows, dim3(blocks(P * d)), dim3(256), 0, s, X, ldx, d, pairs, P, t.Xb);
    {   // a1 = x W1 + b1, g = GELU(a1)
        GemmArgs a{};
        a.M = (int)P; a.N = hid; a.K = d;
        a.A = t.Xb; a.sam = d; a.sak = 1;
        a.B = W1; a.sbk = hid; a.sbn = 1;
        a.C = t.A1; a.ldc = hid; a.C2 = t.G; a.bias = b1;
        gemm<EPI_BIAS_GELU>(s, a);
    }
    {   // u = tanh(g W2 + b2)
        GemmArgs a{};
        a.M = (int)P; a.N = ell; a.K = hid;
        a.A = t.G; a.sam = hid; a.sak = 1;
        a.B = W2; a.sbk = ell; a.sbn = 1;
        a.C = t.U; a.ldc = ell; a.bias = b2;
        gemm<EPI_BIAS_TANH>(s, a);
    }
    hipLaunchKernelGGL(k_pair_loss, dim3(blocks(B, 4)), dim3(256), 0, s, t.U, ell, B, labels, h, lam, t.dA2, loss);
    const int splits = (int)std::min<int64_t>(256, std::max<int64_t>(1, P / 128));
    {   // gW2 = g^T dA2
        GemmArgs a{};
        a.M = hid; a.N = ell; a.K = (int)P;
        a.A = t.G; a.sam = 1; a.sak = hid;
        a.B = t.dA2; a.sbk = ell; a.sbn = 1;
        a.C = gW2; a.ldc = ell;
        gemm<EPI_ATOMIC>(s, a, splits);
    }
    {   // dA1 = (dA2 W2^T) * GELU'(a1)
        GemmArgs a{};
        a.M = (int)P; a.N = hid; a.K = ell;
        a.A = t.dA2; a.sam = ell; a.sak = 1;
        a.B = W2; a.sbk = 1; a.sbn = ell;
        a.C = t.dA1; a.ldc = hid; a.aux = t.A1;
        gemm<EPI_MUL_GELUGRAD>(s, a);
    }
    {   // gW1 = x^T dA1
        GemmArgs a{};
        a.M = d; a.N = hid; a.K = (int)P;
        a.A = t.Xb; a.sam = 1; a.sak = d;
        a.B = t.dA1; a.sbk = hid; a.sbn = 1;
        a.C = gW1; a.ldc = hid;
        gemm<EPI_ATOMIC>(s, a, splits);
    }
    const int64_t rpb = std::max<int64_t>(32, (P + 16383) / 16384);
    const unsigned gy = (unsigned)((P + rpb - 1) / rpb);
    hipLaunchKernelGGL(k_colsum, dim3(blocks(ell), gy), dim3(256), 0, s, t.dA2, P, ell, rpb, gb2);
    hipLaunchKernelGGL(k_colsum, dim3(blocks(hid), gy), dim3(256), 0, s, t.dA1, P, hid, rpb, gb1);
}

void launch_adam(hipStream_t s, float* params, const float* grad, float* m, float* v, int64_t count, int64_t step,
                 float lr, float beta1, float beta2, float eps)
{
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)step));
    hipLaunchKernelGGL(k_adam, dim3(blocks(count)), dim3(256), 0, s, params, grad, m, v, count, lr, beta1, beta2, eps,
                       c1, c2);
}

bool adam_args_ok(float lr, float beta1, float beta2, float eps)
{
    return lr >= 0.f && std::isfinite(lr) && beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f &&
           eps > 0.f && std::isfinite(eps);
}

// Host check that every pair index is below n (one synchronisation).
msm_status check_pairs(msm_ctx* ctx, const char* fn, hipStream_t s, const uint32_t* pairs, int64_t count, int64_t n,
                       unsigned long long* bad_dev)
{
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, reinterpret_cast<uint64_t*>(bad_dev), (int64_t)1);
    hipLaunchKernelGGL(k_check_index, dim3(blocks(count)), dim3(256), 0, s, pairs, count, n, bad_dev);
    MSM_HIP(ctx, hipGetLastError());
    MSM_HIP(ctx, hipMemcpyAsync(ctx->host_words, bad_dev, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    MSM_HIP(ctx, hipStreamSynchronize(s));
    if (ctx->host_words[0] != 0)
        return msm::fail(ctx, MSM_E_INVALID, "%s: %llu pair indices are not below n=%lld", fn,
                         (unsigned long long)ctx->host_words[0], (long long)n);
    return MSM_OK;
}

}  // namespace

extern "C" msm_status msm_project_mlp(msm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                                      const float* params, int32_t hid, int32_t ell, uint64_t* S, void* stream)
{
    if (!ctx) return msm::fail(nullptr, MSM_E_INVALID, "msm_project_mlp: ctx is NULL");
    ctx->err.clear();
    msm_status st = check_shape(ctx, "msm_project_mlp", n, d, ldx, hid, ell);
    if (st != MSM_OK) return st;
    if (n == 0) return MSM_OK;
    if (!X || !params || !S) return msm::fail(ctx, MSM_E_INVALID, "msm_project_mlp: NULL X, params or S");
    st = msm::use_device(ctx);
    if (st != MSM_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int W = (ell + 63) / 64;

    if (d <= 32 * FU_MAXKD && ell <= 16 * FU_MAXNB) {
        const int KD = fused_kd(d), NB = fused_nb(ell);
        const int Kp = 32 * KD, Np = 16 * NB;
        const int nch = (hid + FU_HC - 1) / FU_HC;
        msm::Carver cv;
        cv.take<__bf16>((size_t)nch * FU_HC * Kp);
        cv.take<__bf16>((size_t)nch * Np * FU_HC);
        cv.take<float>((size_t)nch * FU_HC);
        cv.take<float>((size_t)Np);
        void* scr = nullptr;
        st = msm::ctx_scratch(ctx, cv.off, s, &scr);
        if (st != MSM_OK) return st;
        msm::Carver c2;
        c2.base = static_cast<char*>(scr);
        __bf16* W1p = c2.take<__bf16>((size_t)nch * FU_HC * Kp);
        __bf16* W2p = c2.take<__bf16>((size_t)nch * Np * FU_HC);
        float* b1p = c2.take<float>((size_t)nch * FU_HC);
        float* b2p = c2.take<float>((size_t)Np);
        const int64_t total = (int64_t)nch * FU_HC * Kp + (int64_t)nch * Np * FU_HC + (int64_t)nch * FU_HC + Np;
        {
            msm::KernelTimer kt(ctx, s, "k_mlp_pack");
            hipLaunchKernelGGL(k_mlp_pack, dim3(blocks(total)), dim3(256), 0, s, params, d, hid, ell, KD, nch, NB,
                               W1p, W2p, b1p, b2p);
        }
        Packed P{W1p, W2p, b1p, b2p};
        const bool vec = (d == Kp) && (ldx % 4 == 0) && (reinterpret_cast<uintptr_t>(X) % 16 == 0);
        MSM_HIP(ctx, hipGetLastError());
        msm::KernelTimer kt(ctx, s, "k_mlp_fused");
        MSM_HIP(ctx, vec ? launch_fused<true>(s, KD, NB, X, n, d, ldx, P, nch, W, S)
                         : launch_fused<false>(s, KD, NB, X, n, d, ldx, P, nch, W, S));
        return MSM_OK;
    }

    // other shapes: the two layers as separate GEMMs over row chunks that
    // keep the hidden activations near 256 MB each
    const int64_t chunk = std::max<int64_t>(GT, ((int64_t)(64 << 20) / hid) / GT * GT);
    const int64_t rows_max = std::min(n, chunk);
    msm::Carver cv;
    cv.take<float>((size_t)rows_max * hid);
    cv.take<float>((size_t)rows_max * hid);
    void* scr = nullptr;
    st = msm::ctx_scratch(ctx, cv.off, s, &scr);
    if (st != MSM_OK) return st;
    msm::Carver c2;
    c2.base = static_cast<char*>(scr);
    float* A1 = c2.take<float>((size_t)rows_max * hid);
    float* G = c2.take<float>((size_t)rows_max * hid);
    const float* W1 = params;
    const float* b1 = W1 + (int64_t)d * hid;
    const float* W2 = b1 + hid;
    const float* b2 = W2 + (int64_t)hid * ell;
    msm::KernelTimer kt(ctx, s, "k_mlp_gemm");
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks(n * W)), dim3(256), 0, s, S, n * W);
    for (int64_t r0 = 0; r0 < n; r0 += chunk) {
        const int rows = (int)std::min(chunk, n - r0);
        GemmArgs a{};
        a.M = rows; a.N = hid; a.K = d;
        a.A = X + r0 * ldx; a.sam = ldx; a.sak = 1;
        a.B = W1; a.sbk = hid; a.sbn = 1;
        a.C = A1; a.ldc = hid; a.C2 = G; a.bias = b1;
        gemm<EPI_BIAS_GELU>(s, a);
        GemmArgs b{};
        b.M = rows; b.N = ell; b.K = hid;
        b.A = G; b.sam = hid; b.sak = 1;
        b.B = W2; b.sbk = ell; b.sbn = 1;
        b.bias = b2; b.S = S + r0 * W; b.W = W;
        gemm<EPI_SIGNPACK>(s, b);
    }
    MSM_HIP(ctx, hipGetLastError());
    return MSM_OK;
}

extern "C" msm_status msm_mlp_loss_grad(msm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                                        const float* params, int32_t hid, int32_t ell, const uint32_t* pairs,
                                        const float* labels, int32_t B, float h, float lam, float* grad,
                                        float* loss_out, void* stream)
{
    if (!ctx) return msm::fail(nullptr, MSM_E_INVALID, "msm_mlp_loss_grad: ctx is NULL");
    ctx->err.clear();
    msm_status st = check_shape(ctx, "msm_mlp_loss_grad", n, d, ldx, hid, ell);
    if (st != MSM_OK) return st;
    if (B < 1 || B > (1 << 24) || !(h >= 0.f) || !std::isfinite(h) || !(lam >= 0.f) || !std::isfinite(lam))
        return msm::fail(ctx, MSM_E_INVALID, "msm_mlp_loss_grad: need 1 <= B <= 2^24, finite h >= 0 and lam >= 0");
    if (!X || !params || !pairs || !labels || !grad)
        return msm::fail(ctx, MSM_E_INVALID, "msm_mlp_loss_grad: NULL pointer");
    st = msm::use_device(ctx);
    if (st != MSM_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    msm::Carver cv;
    cv.take<double>(1);
    cv.take<unsigned long long>(1);
    TrainBufs tb;
    const size_t bytes = train_carve(cv, 2ll * B, d, hid, ell, &tb);
    void* scr = nullptr;
    st = msm::ctx_scratch(ctx, bytes, s, &scr);
    if (st != MSM_OK) return st;
    msm::Carver c2;
    c2.base = static_cast<char*>(scr);
    double* loss = c2.take<double>(1);
    unsigned long long* bad = c2.take<unsigned long long>(1);
    train_carve(c2, 2ll * B, d, hid, ell, &tb);
    st = check_pairs(ctx, "msm_mlp_loss_grad", s, pairs, 2ll * B, n, bad);
    if (st != MSM_OK) return st;
    {
        msm::KernelTimer kt(ctx, s, "k_mlp_loss_grad");
        hipLaunchKernelGGL(k_fill_d, dim3(1), dim3(64), 0, s, loss, (int64_t)1);
        launch_loss_grad(s, X, d, ldx, params, hid, ell, pairs, labels, B, h, lam, grad, loss, tb);
    }
    MSM_HIP(ctx, hipGetLastError());
    MSM_HIP(ctx, hipMemcpyAsync(ctx->host_words, loss, sizeof(double), hipMemcpyDeviceToHost, s));
    MSM_HIP(ctx, hipStreamSynchronize(s));
    if (loss_out) {
        double lv;
        std::memcpy(&lv, ctx->host_words, sizeof(double));
        *loss_out = (float)lv;
    }
    return MSM_OK;
}

extern "C" msm_status msm_mlp_adam(msm_ctx* ctx, float* params, const float* grad, float* m, float* v, int64_t count,
                                   int64_t step, float lr, float beta1, float beta2, float eps, void* stream)
{
    if (!ctx) return msm::fail(nullptr, MSM_E_INVALID, "msm_mlp_adam: ctx is NULL");
    ctx->err.clear();
    if (count < 0 || step < 1 || !adam_args_ok(lr, beta1, beta2, eps))
        return msm::fail(ctx, MSM_E_INVALID, "msm_mlp_adam: arguments out of range");
    if (count == 0) return MSM_OK;
    if (!params || !grad || !m || !v) return msm::fail(ctx, MSM_E_INVALID, "msm_mlp_adam: NULL pointer");
    msm_status st = msm::use_device(ctx);
    if (st != MSM_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    msm::KernelTimer kt(ctx, s, "k_adam");
    launch_adam(s, params, grad, m, v, count, step, lr, beta1, beta2, eps);
    MSM_HIP(ctx, hipGetLastError());
    return MSM_OK;
}

extern "C" msm_status msm_mlp_train(msm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx, float* params,
                                    float* m, float* v, int32_t hid, int32_t ell, const uint32_t* pairs,
                                    const float* labels, int64_t npairs, int32_t batch, int64_t steps,
                                    int64_t first_step, float lr, float h, float lam, float* losses, void* stream)
{
    if (!ctx) return msm::fail(nullptr, MSM_E_INVALID, "msm_mlp_train: ctx is NULL");
    ctx->err.clear();
    msm_status st = check_shape(ctx, "msm_mlp_train", n, d, ldx, hid, ell);
    if (st != MSM_OK) return st;
    if (npairs < 1 || npairs > 0x7FFFFFFFll || batch < 1 || batch > (1 << 24) || steps < 0 || steps > (1 << 24) ||
        first_step < 1 || !adam_args_ok(lr, 0.9f, 0.999f, 1e-8f) || !(h >= 0.f) || !std::isfinite(h) ||
        !(lam >= 0.f) || !std::isfinite(lam))
        return msm::fail(ctx, MSM_E_INVALID, "msm_mlp_train: arguments out of range");
    if (!X || !params || !m || !v || !pairs || !labels)
        return msm::fail(ctx, MSM_E_INVALID, "msm_mlp_train: NULL pointer");
    if (steps == 0) return MSM_OK;
    st = msm::use_device(ctx);
    if (st != MSM_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int B = (int)std::min<int64_t>(batch, npairs);
    const int64_t np = n_params(d, hid, ell);
    msm::Carver cv;
    cv.take<double>((size_t)steps);
    cv.take<unsigned long long>(1);
    cv.take<float>((size_t)np);
    TrainBufs tb;
    const size_t bytes = train_carve(cv, 2ll * B, d, hid, ell, &tb);
    void* scr = nullptr;
    st = msm::ctx_scratch(ctx, bytes, s, &scr);
    if (st != MSM_OK) return st;
    msm::Carver c2;
    c2.base = static_cast<char*>(scr);
    double* loss = c2.take<double>((size_t)steps);
    unsigned long long* bad = c2.take<unsigned long long>(1);
    float* grad = c2.take<float>((size_t)np);
    train_carve(c2, 2ll * B, d, hid, ell, &tb);
    st = check_pairs(ctx, "msm_mlp_train", s, pairs, 2 * npairs, n, bad);
    if (st != MSM_OK) return st;
    {
        msm::KernelTimer kt(ctx, s, "k_mlp_train");
        hipLaunchKernelGGL(k_fill_d, dim3(blocks(steps)), dim3(256), 0, s, loss, steps);
        // batch t takes the next B pairs in list order; a batch that would
        // run past the end starts again at pair 0
        int64_t off = 0;
        for (int64_t t = 0; t < steps; ++t) {
            if (off + B > npairs) off = 0;
            launch_loss_grad(s, X, d, ldx, params, hid, ell, pairs + 2 * off, labels + off, B, h, lam, grad,
                             loss + t, tb);
            launch_adam(s, params, grad, m, v, np, first_step + t, lr, 0.9f, 0.999f, 1e-8f);
            off += B;
        }
    }
    MSM_HIP(ctx, hipGetLastError());
    if (losses) {
        std::vector<double> hl((size_t)steps);
        MSM_HIP(ctx, hipMemcpyAsync(hl.data(), loss, sizeof(double) * steps, hipMemcpyDeviceToHost, s));
        MSM_HIP(ctx, hipStreamSynchronize(s));
        for (int64_t t = 0; t < steps; ++t) losses[t] = (float)hl[(size_t)t];
    }
    return MSM_OK;
}
