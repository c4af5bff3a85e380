// Device code of the multiple sorting method with blockwise masking
// (Sections 2.1-2.2): combination tables, the partition, bucket and
// overflow kernels. Included by the single-problem driver (enumerate.hip)
// and the batched driver (batch.hip); not part of the public ABI.
//
// For every set B of h masked blocks the points must be grouped by their
// B-masked string s^B, and pairs inside a group tested. Only grouping is
// needed, not a full order (the paper's own radix-sort trick makes the same
// observation), so the sort key is a 32-bit mix of the masked string rather
// than the string itself:
//
//   1. partition  one MSD radix pass over HBM on the top r1 bits of the mix:
//                 LDS histograms per tile (k_part_count), a column scan of
//                 the (tile, bucket) counts (k_part_colscan, k_part_scan), and a scatter of
//                 (mix << 32 | index) into bucket order (k_part_scatter).
//   2. bucket     a workgroup takes a few buckets (about 512 points each):
//                 the next 11 bits of the mix are counted in an LDS
//                 histogram (the second radix digit), whose bins with two or
//                 more members are the runs; a wavefront prefix scan places
//                 the run members in LDS and a flat, balanced loop tests all
//                 pairs inside runs (k_bucket).
//   3. overflow   buckets larger than the LDS capacity are tested tile by
//                 tile straight from HBM (k_big).
//
// Equal masked strings always share a mix, so no pair is lost. Different
// strings can share a mix; that only adds candidates, because the pair test
// below is exact:
//
//   x = s_i xor s_j;  keep iff popcount(x) <= h            (Hamming filter)
//                     and x has no bit outside the blocks of B  (s_i^B == s_j^B)
//                     and B is the canonical set for the blocks where x != 0.
//
// Canonical set: a pair whose differing blocks form D (|D| <= h) falls into
// one group under every h-set B containing D. It is written only under
// D plus the smallest blocks not in D, i.e. iff D is a subset of B and every
// block of B above the smallest unmasked block is in D. So each pair comes
// out exactly once without any exchange between combinations.
#pragma once

#include "msm_internal.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <vector>

namespace {

constexpr int MAXW = 4;
constexpr int MAXK = 64;
constexpr int PART_THREADS = 256;
constexpr int SCAT_THREADS = 1024;  // scatter: threads, and points per thread in a chunk
constexpr int SCAT_PPT = 16;
constexpr int BPART_PPT = 16;       // points per thread of a batched partition tile
constexpr int BSCAT_THREADS = 256;  // threads of the batched scatter
constexpr int SCAN_THREADS = 1024;
constexpr int BK_THREADS = 256;
constexpr int BK_WAVES = BK_THREADS / 64;
constexpr int BK_MAXB = 4;                        // 64-element batches per wave
constexpr int BK_CAP = BK_WAVES * 64 * BK_MAXB;   // largest bucket sorted in LDS
// The first pass with twice the threads at the same capacity, for strings of
// three or four words and for later string pools (which test each passing
// pair's strings in the earlier pools): more waves to hide the gathers.
// Measured at paper scale: radius, second pool 1.63 -> 1.32 ms; ell = 240
// radius 3.33 -> 2.44 ms, coord 3.26 -> 2.63 ms; ell = 192 radius 2.80 ->
// 2.28 ms; but one-pool radius 1.09 -> 1.17 ms and coord 0.67 -> 0.83 ms at
// ell = 128, which keep 256 threads.
constexpr int BK_THREADS_WIDE = 512;
constexpr int BK_MAXB_WIDE = 2;
static_assert(BK_THREADS_WIDE * BK_MAXB_WIDE == BK_CAP, "both first-pass shapes hold the same buckets");
constexpr int BK_PAIR_MAX = 128;                  // consecutive pairs per lane and round, at most
static_assert(BK_PAIR_MAX <= 128, "a lane keeps its results in four 32-bit words");
// Buckets per workgroup of the first pass, and whether sibling buckets that
// fit in LDS together are taken as one unit. With four-word strings the
// kernel keeps few workgroups per CU and each bucket's gathers and barriers
// are exposed: eight buckets per workgroup, siblings merged, measured 5-11 %
// faster at ell = 240 on lone and on clustered points; with narrower strings
// two buckets per workgroup, unmerged, measured best.
template <int W>
constexpr int bk_group() { return W >= 4 ? 8 : 2; }
template <int W>
constexpr bool bk_merge() { return W >= 4; }
static_assert(bk_group<1>() % 2 == 0 && bk_group<4>() % 2 == 0, "sibling buckets share a workgroup");
constexpr int BK_OUT = 512;                       // staged output pairs per workgroup
constexpr int BK_DIGIT = 10;                      // mix bits counted inside a bucket
constexpr int BK_DIGIT_L = 12;                    // the same in the second pass over large buckets
constexpr int BK_BINS = 1 << BK_DIGIT;
constexpr int BIG_TILE = 256;
constexpr int MAX_BUCKETS = 8192;
constexpr int TARGET_BUCKET = 512;

constexpr int MAXHI = 4;   // blocks of `hi` tested from unrolled masks
constexpr int DT_LDS_K = 12;  // family bitmaps over up to 2^12 difference sets are read from LDS
constexpr int DT_LDS_WORDS = 1 << (DT_LDS_K - 5);

// Threads and points per thread of the second bucket pass, sized so that
// its LDS stays below 160 KB (capacity 4096 points for W <= 2, else 2048).
// One workgroup fits a CU; with strings of one or two words it takes 1024
// threads of four points each (512 threads of eight measured 0.71 against
// 0.49 ms on the two-pool paper-scale step), with wider strings 512.
template <int W>
constexpr int large_threads()
{
    return W <= 2 ? 1024 : 512;
}
template <int W>
constexpr int large_maxb()
{
    return 4;
}

struct Combo {                    // one set B of masked blocks (or, grouped
                                  // hierarchically, one set A of kept blocks)
    uint64_t keep[MAXW];          // characters below ell outside the blocks of B
    uint64_t hi;                  // blocks of B above the smallest block not in B
    int32_t nhi;                  // number of blocks in hi
    int32_t nfam;                 // hierarchical: difference sets of the family
    uint64_t amask;               // the masked blocks B (per combination) or the partition's blocks A
    uint32_t famoff;              // hierarchical: first family entry in Params::fam
    uint32_t dtoff;               // hierarchical: first word of its bitmap in Params::dtab
    uint64_t himask[MAXHI][MAXW]; // character masks of the first MAXHI blocks of hi
};
static_assert(sizeof(Combo) == 192, "Combo layout");

struct Ovf {
    uint32_t c, beg, m, pad;
};

struct Params {
    const uint64_t* S;       // strings of the replicate being enumerated
    const uint64_t* Sall;    // all replicates, replicate-major
    uint64_t rep_stride;     // words between replicates (n * W)
    int rep;                 // index of the replicate being enumerated
    int64_t n;
    const Combo* combos;     // combinations of this launch group
    const uint64_t* bm;      // [k][MAXW] block masks
    int k, h;
    uint64_t valid[MAXW];    // bits below ell
    int r1;                  // bucket bits (top bits of the mix)
    int nb;                  // 1 << r1
    int T, nt;               // partition tile size and count
    int sch;                 // points per sorted scatter chunk (at most SCAT_THREADS * SCAT_PPT)
    int units;               // combinations of the group x tiles
    uint32_t* counts;        // [c][t][b] tile counts, then tile offsets
    uint32_t* base;          // [c][nb + 1] bucket starts
    uint64_t* part;          // [c][n] (mix << 32 | index) in bucket order
    uint32_t* keys;          // [c][n] masked mixes from the count pass, or NULL (the scatter recomputes them)
    uint32_t* pairs;
    unsigned long long cap;
    unsigned long long* counter;
    Ovf* ovf;
    uint32_t* ovf_count;
    // hierarchical grouping on j blocks (see diff_blocks)
    int hier;                // 0: one group per combination of masked blocks
    int blk_r, blk_L;        // the first blk_r blocks hold blk_L + 1 characters, the rest blk_L
    uint64_t blk_m1, blk_m0; // 2^32 / (blk_L + 1) and 2^32 / blk_L, rounded up
    int dL;                  // 8, 16 or 32 when every block has that many characters, else 0
    const uint64_t* fam;     // minimal difference sets of each partition's family
    const uint32_t* dtab;    // per partition, a bitmap over difference sets D: D is in its family
    // second pass over the overflow list (k_bucket with LIST)
    const Ovf* list;
    const uint32_t* list_count;
    uint32_t list_cap;
    Ovf* ovf2;
    uint32_t* ovf2_count;
};

// Batched enumeration over many independent instances at once: their
// points are concatenated, and every instance owns its own range of
// partition buckets, so a bucket never mixes instances.
struct BInst {
    uint64_t off;       // first point of the instance in the concatenation
    uint32_t n;         // its points
    int32_t r;          // bucket bits: the instance owns 2^r buckets
    uint32_t bstart;    // its first global bucket
    uint32_t tstart;    // its first partition tile
    uint32_t ntiles;    // its partition tiles
    uint32_t pad;
    uint64_t cnt_off;   // its tile counts inside one combination's counts
    uint32_t* pairs;    // its output pairs (local indices)
    int64_t cap;        // their capacity
};

struct BatchArgs {
    const BInst* inst;
    const uint32_t* tile_inst;    // [tiles] instance of each partition tile
    const uint32_t* bucket_inst;  // [buckets] instance of each bucket
    uint64_t cnt_stride;          // words of tile counts per combination
    int group;                    // buckets per workgroup
    unsigned long long* m_dev;    // per-instance pair counters
    int bk_lo, bk_hi;             // buckets [bk_lo, bk_hi) of this launch of the bucket kernel
};

// The output finalizer of SplitMix64 (Steele, Lea and Flood, "Fast
// splittable pseudorandom number generators", OOPSLA 2014), with its
// published shift and multiplier constants: a bijection of 64-bit words
// whose output bits each depend on every input bit. Used only to spread
// masked strings over buckets; equal strings always get equal mixes.
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

template <int W>
__device__ __forceinline__ uint32_t masked_mix(const uint64_t (&s)[W], const uint64_t (&keep)[W])
{
    uint64_t z = 0x9e3779b97f4a7c15ull;
#pragma unroll
    for (int w = 0; w < W; ++w) z = mix64(z ^ (s[w] & keep[w]));
    return (uint32_t)(z >> 32);
}

template <int W>
__device__ __forceinline__ void load_string(const uint64_t* __restrict__ S, uint64_t i, uint64_t (&s)[W])
{
    const uint64_t* p = S + i * W;
#pragma unroll
    for (int w = 0; w < W; ++w) s[w] = p[w];
}

template <int W>
__device__ __forceinline__ void load_keep(const Combo* cb, uint64_t (&keep)[W])
{
#pragma unroll
    for (int w = 0; w < W; ++w) keep[w] = cb->keep[w];
}

// -------------------------------------------------------------------------
// 1. partition
//
// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2. The (combination, tile) units are cut into 8 contiguous ranges in
// combination-major order and XCD x runs range x, so all tiles of a
// combination scatter through one L2, where the partial lines that
// neighbouring tiles write into the same bucket can merge.
constexpr int NUM_XCD = 8;

__device__ __forceinline__ bool xcd_unit(int units, int& cl, int& t, int nt)
{
    const int per = (units + NUM_XCD - 1) / NUM_XCD;
    const int u = (int)(blockIdx.x % NUM_XCD) * per + (int)(blockIdx.x / NUM_XCD);
    if (u >= units) return false;
    cl = u / nt;
    t = u % nt;
    return true;
}

template <int W>
__global__ __launch_bounds__(PART_THREADS) void k_part_count(Params p)
{
    extern __shared__ uint32_t hist[];
    int cl, t;
    if (!xcd_unit(p.units, cl, t, p.nt)) return;
    uint64_t keep[W];
    load_keep<W>(p.combos + cl, keep);
    for (int b = threadIdx.x; b < p.nb; b += PART_THREADS) hist[b] = 0;
    __syncthreads();
    const int64_t beg = (int64_t)t * p.T;
    const int64_t end = min(p.n, beg + p.T);
    for (int64_t i = beg + threadIdx.x; i < end; i += PART_THREADS) {
        uint64_t s[W];
        load_string<W>(p.S, (uint64_t)i, s);
        const uint32_t mx = masked_mix<W>(s, keep);
        const uint32_t b = p.r1 ? (mx >> (32 - p.r1)) : 0u;
        atomicAdd(&hist[b], 1u);
        if (p.keys) p.keys[(size_t)cl * (size_t)p.n + (size_t)i] = mx;
    }
    __syncthreads();
    uint32_t* out = p.counts + ((size_t)cl * p.nt + t) * p.nb;
    for (int b = threadIdx.x; b < p.nb; b += PART_THREADS) out[b] = hist[b];
}

// Per combination: counts[t][b] -> offset of tile t inside bucket b, and
// base[b] = start of bucket b, in two launches: a column scan over the
// tiles with one thread per bucket (grid: buckets / PART_THREADS x
// combinations), which leaves bucket totals in base, then one workgroup
// per combination turns the totals into starts.
__global__ __launch_bounds__(PART_THREADS) void k_part_colscan(Params p)
{
    const int cl = blockIdx.y;
    const int b = blockIdx.x * PART_THREADS + threadIdx.x;
    if (b >= p.nb) return;
    uint32_t* cnt = p.counts + (size_t)cl * p.nt * p.nb;
    uint32_t run = 0;
    int t = 0;
    for (; t + 8 <= p.nt; t += 8) {
        uint32_t v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = cnt[(size_t)(t + q) * p.nb + b];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            cnt[(size_t)(t + q) * p.nb + b] = run;
            run += v[q];
        }
    }
    for (; t < p.nt; ++t) {
        const uint32_t v = cnt[(size_t)t * p.nb + b];
        cnt[(size_t)t * p.nb + b] = run;
        run += v;
    }
    p.base[(size_t)cl * (p.nb + 1) + b] = run;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_part_scan(Params p)
{
    extern __shared__ uint32_t tot[];  // nb totals, then one word per wave
    const int cl = blockIdx.x;
    uint32_t* base = p.base + (size_t)cl * (p.nb + 1);
    for (int b = threadIdx.x; b < p.nb; b += SCAN_THREADS) tot[b] = base[b];
    __syncthreads();
    uint32_t* wsum = tot + p.nb;
    const int per = (p.nb + SCAN_THREADS - 1) / SCAN_THREADS;
    const int b0 = threadIdx.x * per;
    const int b1 = min(p.nb, b0 + per);
    uint32_t s = 0;
    for (int b = b0; b < b1; ++b) s += tot[b];
    const uint32_t incl = msm::wave_incl_scan(s);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t pre = 0;
    for (int w = 0; w < wave; ++w) pre += wsum[w];
    uint32_t run = pre + incl - s;
    for (int b = b0; b < b1; ++b) {
        const uint32_t v = tot[b];
        base[b] = run;
        run += v;
    }
    if (threadIdx.x == 0) base[p.nb] = (uint32_t)p.n;
}

// Scatter of one tile in chunks of p.sch points: the chunk is counting-
// sorted by bucket in LDS (its points' buckets counted, the counts scanned,
// the entries placed), then written out in that order, so consecutive
// threads write consecutive entries of one bucket. With 4096-point tiles a
// tile holds about two points per bucket and nearly every 8-byte write is a
// partial line; sorted chunks of 16384 points write runs of about eight.
// SCAT_THREADS threads; dynamic LDS: sch entries, then 2 * nb words.
template <int W>
__global__ __launch_bounds__(SCAT_THREADS) void k_part_scatter(Params p)
{
    extern __shared__ unsigned long long scat_lds[];
    __shared__ uint32_t wsum[SCAT_THREADS / 64];
    int cl, t;
    if (!xcd_unit(p.units, cl, t, p.nt)) return;
    uint64_t* staged = reinterpret_cast<uint64_t*>(scat_lds);  // p.sch entries
    uint32_t* lcnt = reinterpret_cast<uint32_t*>(staged + p.sch);  // chunk counts, then starts
    uint32_t* gb = lcnt + p.nb;                                    // next global slot per bucket
    uint64_t keep[W];
    load_keep<W>(p.combos + cl, keep);
    const uint32_t* off = p.counts + ((size_t)cl * p.nt + t) * p.nb;
    const uint32_t* base = p.base + (size_t)cl * (p.nb + 1);
    for (int b = threadIdx.x; b < p.nb; b += SCAT_THREADS) gb[b] = base[b] + off[b];
    uint64_t* part = p.part + (size_t)cl * p.n;
    const int shift = 32 - p.r1;
    const int64_t tbeg = (int64_t)t * p.T;
    const int64_t tend = min(p.n, tbeg + p.T);
    for (int64_t beg = tbeg; beg < tend; beg += p.sch) {
        const int cnt = (int)min<int64_t>(p.sch, tend - beg);
        for (int b = threadIdx.x; b < p.nb; b += SCAT_THREADS) lcnt[b] = 0;
        __syncthreads();  // lcnt is zero, gb is set, staged is free
        uint32_t mx[SCAT_PPT], rk[SCAT_PPT];
#pragma unroll
        for (int k = 0; k < SCAT_PPT; ++k) {
            const int e = (int)threadIdx.x + k * SCAT_THREADS;
            mx[k] = 0u;
            rk[k] = 0u;
            if (e < cnt) {
                if (p.keys) {
                    // the count pass wrote the mix: 4 bytes instead of the string
                    mx[k] = p.keys[(size_t)cl * (size_t)p.n + (size_t)(beg + e)];
                } else {
                    uint64_t s[W];
                    load_string<W>(p.S, (uint64_t)(beg + e), s);
                    mx[k] = masked_mix<W>(s, keep);
                }
                rk[k] = atomicAdd(&lcnt[p.r1 ? (mx[k] >> shift) : 0u], 1u);
            }
        }
        __syncthreads();
        // exclusive scan of the chunk's bucket counts: each thread a run of
        // consecutive buckets, a wave scan of the run sums, then the waves
        const int per = (p.nb + SCAT_THREADS - 1) / SCAT_THREADS;
        const int b0 = (int)threadIdx.x * per, b1 = min(p.nb, b0 + per);
        uint32_t sum = 0;
        for (int b = b0; b < b1; ++b) sum += lcnt[b];
        const uint32_t incl = msm::wave_incl_scan(sum);
        if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = incl;
        __syncthreads();
        uint32_t run = incl - sum;
        for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) run += wsum[w];
        for (int b = b0; b < b1; ++b) {
            const uint32_t c = lcnt[b];
            lcnt[b] = run;
            run += c;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < SCAT_PPT; ++k) {
            const int e = (int)threadIdx.x + k * SCAT_THREADS;
            if (e < cnt) {
                const uint32_t b = p.r1 ? (mx[k] >> shift) : 0u;
                staged[lcnt[b] + rk[k]] = ((uint64_t)mx[k] << 32) | (uint64_t)(uint32_t)(beg + e);
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < cnt; e += SCAT_THREADS) {
            const uint64_t v = staged[e];
            const uint32_t b = p.r1 ? ((uint32_t)(v >> 32) >> shift) : 0u;
            part[gb[b] + (uint32_t)e - lcnt[b]] = v;
        }
        __syncthreads();  // every read of gb and lcnt is done
        // the next chunk's entries of a bucket follow this chunk's
        for (int b = threadIdx.x; b < p.nb; b += SCAT_THREADS) {
            const uint32_t next = (b + 1 < p.nb ? lcnt[b + 1] : (uint32_t)cnt);
            gb[b] += next - lcnt[b];
        }
        __syncthreads();  // lcnt is read before the next chunk clears it
    }
}

// -------------------------------------------------------------------------
// Batched partition: the same three steps over the concatenated points of
// many instances. Partition tiles never straddle instances; instance i owns
// 2^r_i buckets and the point range [off_i, off_i + n_i) of each
// combination's partition array.

template <int W>
__global__ __launch_bounds__(PART_THREADS) void k_bpart_count(Params p, BatchArgs ba)
{
    extern __shared__ uint32_t hist[];
    int cl, t;
    if (!xcd_unit(p.units, cl, t, p.nt)) return;
    const BInst& in = ba.inst[ba.tile_inst[t]];
    const int r = in.r;
    const int nbi = 1 << r;
    uint64_t keep[W];
    load_keep<W>(p.combos + cl, keep);
    for (int b = threadIdx.x; b < nbi; b += PART_THREADS) hist[b] = 0;
    __syncthreads();
    const int64_t beg = (int64_t)in.off + (int64_t)(t - in.tstart) * p.T;
    const int64_t end = min((int64_t)(in.off + in.n), beg + p.T);
    for (int64_t i = beg + threadIdx.x; i < end; i += PART_THREADS) {
        uint64_t s[W];
        load_string<W>(p.S, (uint64_t)i, s);
        const uint32_t mx = masked_mix<W>(s, keep);
        atomicAdd(&hist[r ? (mx >> (32 - r)) : 0u], 1u);
    }
    __syncthreads();
    uint32_t* out = p.counts + (size_t)cl * ba.cnt_stride + in.cnt_off + (size_t)(t - in.tstart) * nbi;
    for (int b = threadIdx.x; b < nbi; b += PART_THREADS) out[b] = hist[b];
}

// One workgroup per (instance, combination): tile offsets inside each
// bucket, then bucket starts (global point positions) of the instance.
__global__ __launch_bounds__(SCAN_THREADS) void k_bpart_scan(Params p, BatchArgs ba)
{
    extern __shared__ uint32_t tot[];  // bucket totals, then one word per wave
    const BInst& in = ba.inst[blockIdx.x];
    const int cl = blockIdx.y;
    const int nbi = 1 << in.r;
    const int ntl = (int)in.ntiles;
    uint32_t* cnt = p.counts + (size_t)cl * ba.cnt_stride + in.cnt_off;
    for (int b = threadIdx.x; b < nbi; b += SCAN_THREADS) {
        uint32_t run = 0;
        for (int t = 0; t < ntl; ++t) {
            const uint32_t v = cnt[(size_t)t * nbi + b];
            cnt[(size_t)t * nbi + b] = run;
            run += v;
        }
        tot[b] = run;
    }
    __syncthreads();
    uint32_t* wsum = tot + nbi;
    const int per = (nbi + SCAN_THREADS - 1) / SCAN_THREADS;
    const int b0 = threadIdx.x * per;
    const int b1 = min(nbi, b0 + per);
    uint32_t s = 0;
    for (int b = b0; b < b1; ++b) s += tot[b];
    const uint32_t incl = msm::wave_incl_scan(s);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t pre = 0;
    for (int w = 0; w < wave; ++w) pre += wsum[w];
    uint32_t run = (uint32_t)in.off + pre + incl - s;
    uint32_t* base = p.base + (size_t)cl * (p.nb + 1) + in.bstart;
    for (int b = b0; b < b1; ++b) {
        const uint32_t v = tot[b];
        base[b] = run;
        run += v;
    }
    // the end of the instance's last bucket; the next instance writes the
    // same value as its first start
    if (threadIdx.x == 0) base[nbi] = (uint32_t)(in.off + in.n);
}

// As k_part_scatter, one tile (p.T <= BSCAT_THREADS * BPART_PPT points) at a
// time: sorted by bucket in LDS, then written in bucket runs. Dynamic LDS:
// p.T entries, then 2 * (the largest instance bucket count) words.
template <int W>
__global__ __launch_bounds__(BSCAT_THREADS) void k_bpart_scatter(Params p, BatchArgs ba, int max_nbi)
{
    extern __shared__ unsigned long long bscat_lds[];
    __shared__ uint32_t wsum[BSCAT_THREADS / 64];
    int cl, t;
    if (!xcd_unit(p.units, cl, t, p.nt)) return;
    const BInst& in = ba.inst[ba.tile_inst[t]];
    const int r = in.r;
    const int nbi = 1 << r;
    uint64_t* staged = reinterpret_cast<uint64_t*>(bscat_lds);
    uint32_t* lcnt = reinterpret_cast<uint32_t*>(staged + p.T);
    uint32_t* gb = lcnt + max_nbi;
    uint64_t keep[W];
    load_keep<W>(p.combos + cl, keep);
    const uint32_t* off = p.counts + (size_t)cl * ba.cnt_stride + in.cnt_off + (size_t)(t - in.tstart) * nbi;
    const uint32_t* base = p.base + (size_t)cl * (p.nb + 1) + in.bstart;
    for (int b = threadIdx.x; b < nbi; b += BSCAT_THREADS) {
        gb[b] = base[b] + off[b];
        lcnt[b] = 0;
    }
    __syncthreads();
    uint64_t* part = p.part + (size_t)cl * p.n;
    const int64_t beg = (int64_t)in.off + (int64_t)(t - in.tstart) * p.T;
    const int cnt = (int)min<int64_t>(p.T, (int64_t)(in.off + in.n) - beg);
    uint32_t mx[BPART_PPT], rk[BPART_PPT];
#pragma unroll
    for (int k = 0; k < BPART_PPT; ++k) {
        const int e = (int)threadIdx.x + k * BSCAT_THREADS;
        mx[k] = 0u;
        rk[k] = 0u;
        if (e < cnt) {
            uint64_t s[W];
            load_string<W>(p.S, (uint64_t)(beg + e), s);
            mx[k] = masked_mix<W>(s, keep);
            rk[k] = atomicAdd(&lcnt[r ? (mx[k] >> (32 - r)) : 0u], 1u);
        }
    }
    __syncthreads();
    const int per = (nbi + BSCAT_THREADS - 1) / BSCAT_THREADS;
    const int b0 = (int)threadIdx.x * per, b1 = min(nbi, b0 + per);
    uint32_t sum = 0;
    for (int b = b0; b < b1; ++b) sum += lcnt[b];
    const uint32_t incl = msm::wave_incl_scan(sum);
    if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) run += wsum[w];
    for (int b = b0; b < b1; ++b) {
        const uint32_t c = lcnt[b];
        lcnt[b] = run;
        run += c;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < BPART_PPT; ++k) {
        const int e = (int)threadIdx.x + k * BSCAT_THREADS;
        if (e < cnt) {
            const uint32_t b = r ? (mx[k] >> (32 - r)) : 0u;
            staged[lcnt[b] + rk[k]] = ((uint64_t)mx[k] << 32) | (uint64_t)(uint32_t)(beg + e);
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < cnt; e += BSCAT_THREADS) {
        const uint64_t v = staged[e];
        const uint32_t b = r ? ((uint32_t)(v >> 32) >> (32 - r)) : 0u;
        part[gb[b] + (uint32_t)e - lcnt[b]] = v;
    }
}

// -------------------------------------------------------------------------
// Exact pair test of one candidate (see the file comment).

template <int W>
__device__ __forceinline__ uint32_t diff_blocks(const uint64_t (&x)[W], const Params& p);
__device__ __forceinline__ bool in_family(const uint32_t* tab, uint32_t D);

template <int W>
__device__ __forceinline__ bool pair_ok(const uint64_t* a, const uint64_t* b, const Params& p,
                                        const uint64_t (&keep)[W], uint64_t hi, const uint32_t* dtab,
                                        const uint64_t* __restrict__ bmL)
{
    uint64_t x[W];
    int ham = 0;
    uint64_t outside = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        x[w] = (a[w] ^ b[w]) & p.valid[w];
        ham += __popcll(x[w]);
        outside |= x[w] & keep[w];
    }
    bool ok = (ham <= p.h) && (outside == 0);
    if (p.hier) return ok && in_family(dtab, diff_blocks<W>(x, p));
    uint64_t need = hi;
    while (ok && need) {
        const int blk = __builtin_ctzll(need);
        need &= need - 1;
        uint64_t any = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) any |= x[w] & bmL[blk * W + w];
        ok = any != 0;
    }
    return ok;
}

// The same test, branch-free, with the masks of the first MAXHI blocks of
// `hi` held in registers (hm). Combinations with more blocks in `hi` finish
// with a loop over the block masks in LDS. HM is 0 for one grouping per
// combination; -8, -16 or -32 for the same with blocks of that many
// characters, where the test is on the difference set D itself (hi <= D <=
// B, with B the combination's masked blocks bmask); positive for the
// hierarchical partitions with that block layout (see diff_blocks_of). GT
// reads the family bitmap from global memory (k > DT_LDS_K), else from LDS.
// A hierarchical partition keeps every block outside its family's union, so
// the bitmap alone also rejects pairs that differ in a kept block.
template <int W, int HM, bool GT>
__device__ __forceinline__ bool pair_ok_fast(const uint64_t* a, const uint64_t* b, const Params& p,
                                             const uint64_t (&keep)[W], const uint64_t (&hm)[MAXHI][W], int nhi,
                                             uint64_t hi_rest, uint64_t bmask, uint64_t hi,
                                             const uint32_t* dtabL, const uint32_t* dtabG,
                                             const uint64_t* __restrict__ bmL)
{
    // the strings in LDS are already cut to ell characters
    uint64_t x[W];
    int ham = 0;
    uint64_t outside = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        x[w] = a[w] ^ b[w];
        ham += __popcll(x[w]);
        if constexpr (HM == 0) outside |= x[w] & keep[w];
    }
    bool ok = (ham <= p.h) & (outside == 0);
    if constexpr (HM < 0) {
        const uint32_t D = diff_blocks_of<W, -HM>(x, p);
        const uint32_t Bm = (uint32_t)bmask, H = (uint32_t)hi;
        return ok & ((D & ~Bm) == 0u) & ((D & H) == H);
    }
    if constexpr (HM > 0) {
        // the pair's difference set must be in the partition's family
        uint32_t D = 0;
        if constexpr (HM != 1) D = diff_blocks_of<W, HM>(x, p);
        else if (ok) D = diff_blocks_of<W, 1>(x, p);
        uint32_t word;
        if constexpr (GT) word = dtabG[D >> 5];
        else word = dtabL[D >> 5];
        return ok & (((word >> (D & 31)) & 1u) != 0u);
    }
#pragma unroll
    for (int s = 0; s < MAXHI; ++s) {
        uint64_t any = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) any |= x[w] & hm[s][w];
        ok &= (s >= nhi) | (any != 0);
    }
    if (hi_rest) {
        uint64_t need = hi_rest;
        while (need) {
            const int blk = __builtin_ctzll(need);
            need &= need - 1;
            uint64_t any = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) any |= x[w] & bmL[blk * W + w];
            ok &= any != 0;
        }
    }
    return ok;
}

// Cross-replicate dedup: a pair found in replicate q is written only if its
// Hamming distance exceeds h in every earlier replicate g < q.
template <int W>
__device__ __forceinline__ bool far_in_earlier(const Params& p, uint32_t i, uint32_t j)
{
    for (int g = 0; g < p.rep; ++g) {
        const uint64_t* a = p.Sall + (uint64_t)g * p.rep_stride + (uint64_t)i * W;
        const uint64_t* b = p.Sall + (uint64_t)g * p.rep_stride + (uint64_t)j * W;
        int ham = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) ham += __popcll((a[w] ^ b[w]) & p.valid[w]);
        if (ham <= p.h) return false;
    }
    return true;
}

// -------------------------------------------------------------------------
// Hierarchical grouping (the concluding remarks' shared sorting, here one
// level): instead of one grouping per set B of h masked blocks, points are
// grouped by j < k - h blocks A, which serves every B whose unmasked blocks
// contain A. A pair with differing blocks D (|D| <= h) has the canonical
// set B*(D) = D plus the smallest blocks not in D (h in all); it is written
// only in the partition whose A is the j smallest blocks not in B*(D), so
// every pair is still written once. A partition's family is the set of D
// that map to it: a pair within distance h is written iff its D is in the
// family (one bit of a per-partition bitmap), and a run whose varying blocks
// contain no member of the family cannot hold a pair to write.

__device__ __forceinline__ int block_of(const Params& p, int c)
{
    const int split = p.blk_r * (p.blk_L + 1);
    return c < split ? (int)(((uint64_t)c * p.blk_m1) >> 32)
                     : p.blk_r + (int)(((uint64_t)(c - split) * p.blk_m0) >> 32);
}

// The blocks in which a pair differs, as a bit mask, from its differing
// characters x. With blocks of 8, 16 or 32 characters each block is one
// field of a 32-bit half-word: a field is nonzero iff its top bit is set or
// adding all-ones to its lower bits carries into the top bit (the sum stays
// inside the field), and the top bits are then gathered into consecutive
// bits. Other layouts visit the set characters one by one; the caller does
// that only for pairs within distance h, so at most h of them.
// HM is the block layout: 8, 16 or 32 for blocks of that many characters,
// 1 for any other layout.
template <int W, int HM>
__device__ __forceinline__ uint32_t diff_blocks_of(const uint64_t (&x)[W], const Params& p)
{
    uint32_t D = 0;
    if constexpr (HM == 16) {
        // min(field, 1) on both 16-bit halves at once (one packed VALU op;
        // left to itself the compiler tests each field with a compare and a
        // select); then bit 0 and bit 16 of each half-word (the second one
        // shifted up by two) are the word's four block bits
#pragma unroll
        for (int w = 0; w < W; ++w) {
            uint32_t f0, f1;
            asm("v_pk_min_u16 %0, %1, %2" : "=v"(f0) : "v"((uint32_t)x[w]), "s"(0x10001u));
            asm("v_pk_min_u16 %0, %1, %2" : "=v"(f1) : "v"((uint32_t)(x[w] >> 32)), "s"(0x10001u));
            const uint32_t c = f0 | (f1 << 2);  // bits 0, 2, 16, 18
            D |= ((c | (c >> 15)) & 0xFu) << (4 * w);
        }
    } else if constexpr (HM == 8) {
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
            for (int hf = 0; hf < 2; ++hf) {
                const uint32_t v = (uint32_t)(x[w] >> (32 * hf));
                const uint32_t t = (((v & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | v) & 0x80808080u;
                // top bits at 7, 15, 23, 31 -> 0, 8, 16, 24; the product puts
                // them at 21..24 with no two partial products overlapping
                D |= ((((t >> 7) * 0x00204081u) >> 21) & 0xFu) << (8 * w + 4 * hf);
            }
    } else if constexpr (HM == 32) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
            D |= (uint32_t)((uint32_t)x[w] != 0u) << (2 * w);
            D |= (uint32_t)((uint32_t)(x[w] >> 32) != 0u) << (2 * w + 1);
        }
    } else {
#pragma unroll
        for (int w = 0; w < W; ++w) {
            uint64_t v = x[w];
            while (v) {
                D |= 1u << block_of(p, 64 * w + __builtin_ctzll(v));
                v &= v - 1;
            }
        }
    }
    return D;
}

template <int W>
__device__ __forceinline__ uint32_t diff_blocks(const uint64_t (&x)[W], const Params& p)
{
    if (p.dL == 16) return diff_blocks_of<W, 16>(x, p);
    if (p.dL == 8) return diff_blocks_of<W, 8>(x, p);
    if (p.dL == 32) return diff_blocks_of<W, 32>(x, p);
    return diff_blocks_of<W, 1>(x, p);
}

__device__ __forceinline__ bool in_family(const uint32_t* tab, uint32_t D)
{
    return ((tab[D >> 5] >> (D & 31)) & 1u) != 0u;
}

// -------------------------------------------------------------------------
// 2. buckets, bk_group<W>() consecutive ones per workgroup
//
// Inside a bucket one more radix digit (BK_DIGIT bits of the mix, below the
// bucket bits) is counted in an LDS histogram; the count returned by each
// element's atomic is its rank in its bin. The histogram is the run
// segmentation: a bin with c >= 2 members is a run (equal masked strings
// always share a bin) with c (c - 1) / 2 candidate pairs; singleton bins are
// dropped. The first member of each run claims the run's index and its place
// in a compact LDS array of run members with one packed 64-bit LDS atomic,
// so no scan over the bins is needed. Members are scattered there with their
// strings; each run then either claims a range of the flat pair index space
// the same way or is dropped when it cannot hold a pair to write (below),
// and a flat loop over the claimed pairs tests them. Bins that mix several
// masked strings only add candidates, which the exact test rejects.

// TH threads take buckets of up to TH * MAXB points. Without LIST a
// workgroup takes `group` consecutive buckets of combination blockIdx.y;
// with LIST it takes entries of an overflow list (buckets another pass
// found too large), and lists the ones too large for it in p.ovf2.
// The first pass for W <= 2 fits four workgroups per CU in LDS; its
// register budget is held to the matching four waves per SIMD.
template <int W, int DIGIT, bool BATCH, int TH, bool LIST, int MAXB, int HM, bool GT>
__global__ __launch_bounds__(TH, (!LIST && W <= 2 && DIGIT <= 10) ? 4 : 1) void k_bucket(Params p,
                                                                                                   BatchArgs ba)
{
    constexpr bool HIER = HM > 0;
    constexpr int BINS = 1 << DIGIT;
    constexpr int CAP = TH * MAXB;
    // hist holds the digit counts, then (for bins that form runs) the run's
    // first slot in the member arrays | run index << 16
    __shared__ uint32_t hist[BINS];
    __shared__ uint32_t idxB[CAP];
    __shared__ uint64_t sl[CAP * W];
    __shared__ uint16_t runS[CAP / 2];
    __shared__ uint16_t runL[CAP / 2];
    __shared__ unsigned long long runBlk[CAP / 2];  // blocks of hi that vary inside the run
    __shared__ uint16_t liveS[CAP / 2];
    __shared__ uint16_t liveL[CAP / 2];
    __shared__ uint32_t liveP[CAP / 2];
    __shared__ uint64_t bmL[MAXK * W];
    __shared__ uint32_t dtabL[DT_LDS_WORDS];
    __shared__ unsigned long long claimRun;   // runs << 32 | members
    __shared__ unsigned long long claimPair;  // live runs << 32 | pairs
    __shared__ uint2 obuf[BK_OUT];
    __shared__ uint32_t ocnt;
    __shared__ unsigned long long ogb;

    // the combination's masks in registers; hb holds the block indices of
    // the first MAXHI blocks of hi, blocks beyond them (hi_rest) are tested
    // from bmL
    int cl = -1;
    uint64_t keep[W];
    uint64_t hi = 0;
    uint64_t bmask = 0;
    int nhi = 0;
    uint64_t hm[MAXHI][W];
    int hb[MAXHI];
    uint64_t hi_rest = 0;
    int nfam = 0;
    const uint64_t* fam = nullptr;
    const uint32_t* dtabG = nullptr;  // the partition's family bitmap
    int tab_c = -1;                   // the partition whose bitmap is in dtabL
    auto load_combo = [&](int c) {
        const Combo* cb = p.combos + c;
        load_keep<W>(cb, keep);
        hi = cb->hi;
        bmask = cb->amask;
        nhi = cb->nhi;
        nfam = cb->nfam;
        fam = p.fam ? p.fam + cb->famoff : nullptr;
        dtabG = p.dtab ? p.dtab + cb->dtoff : nullptr;
#pragma unroll
        for (int s2 = 0; s2 < MAXHI; ++s2)
#pragma unroll
            for (int w = 0; w < W; ++w) hm[s2][w] = cb->himask[s2][w];
        hi_rest = hi;
#pragma unroll
        for (int s2 = 0; s2 < MAXHI; ++s2) {
            hb[s2] = hi_rest ? __builtin_ctzll(hi_rest) : 0;
            if (hi_rest) hi_rest &= hi_rest - 1;
        }
    };
    if (!LIST) {
        cl = (int)blockIdx.y;
        load_combo(cl);
    }
    for (int e = threadIdx.x; e < p.k * W; e += TH) bmL[e] = p.bm[(e / W) * MAXW + (e % W)];
    for (int e = threadIdx.x; e < BINS; e += TH) hist[e] = 0;
    if (threadIdx.x == 0) ocnt = 0;
    // output destination; in a batch it follows the instance of the bucket
    uint32_t* o_pairs = p.pairs;
    unsigned long long o_cap = p.cap;
    unsigned long long* o_counter = p.counter;
    uint32_t o_off = 0;
    uint32_t cur_inst = 0xFFFFFFFFu;
    msm::PairStager<BK_OUT> out{obuf, &ocnt, &ogb, o_pairs, o_cap, o_counter};
    const uint32_t* base = LIST ? nullptr : p.base + (size_t)cl * (p.nb + 1);
    const uint64_t* part = LIST ? p.part : p.part + (size_t)cl * p.n;
    const int group = BATCH ? ba.group : bk_group<W>();
    const int bk0 = LIST ? 0 : (BATCH ? ba.bk_lo : 0) + (int)blockIdx.x * group;
    const int bk1 = LIST ? 0 : min(BATCH ? ba.bk_hi : p.nb, bk0 + group);
    const uint32_t nlist = LIST ? min(*p.list_count, p.list_cap) : 0u;
    const int dsh0 = 64 - p.r1 - DIGIT;
    int dsh = dsh0;
    // The first pass takes its buckets in units: two sibling buckets (keys
    // that differ only in the last partition bit) that fit in LDS together
    // form one unit, whose in-bucket digit starts one bit higher, at the
    // sibling bit, so that the two never share a run; the unit's fixed
    // latency (gathers, barriers) is paid once (bk_merge). Other buckets are
    // units of their own. group is even, so siblings share a workgroup.
    auto merged_at = [&](int b) {
        return bk_merge<W>() && !LIST && !BATCH && ((b - bk0) & 1) == 0 && b + 1 < bk1 &&
               base[b + 2] - base[b] <= (uint32_t)CAP;
    };
    int ub = bk0;               // first bucket of the next unit
    bool um = merged_at(bk0);   // whether that unit is a merged pair

    // keys of the current unit, loaded one unit ahead
    uint64_t key[MAXB];
    uint32_t nbeg = 0, ncnt = 0;
    if (!LIST) {
        nbeg = base[bk0];
        ncnt = base[bk0 + (um ? 2 : 1)] - nbeg;
#pragma unroll
        for (int b = 0; b < MAXB; ++b) {
            const int pos = threadIdx.x + b * TH;
            key[b] = (ncnt <= (uint32_t)CAP && pos < (int)ncnt) ? part[nbeg + pos] : ~0ull;
        }
    }

    // one-word strings of the next bucket of the first pass, gathered while
    // the current one is processed; pre: they are there (the same on every
    // lane). Wider strings would take registers the pair loop needs.
    constexpr bool PREF = !LIST && W == 1;
    uint64_t nsreg[MAXB][W];
    bool pre = false;
    for (int it = 0;; ++it) {
        uint32_t beg, cnt;
        uint32_t inst_id = 0;
        uint64_t cur[MAXB];
        const bool use_pre = pre;
        pre = false;
        bool has_next = false;
        if (LIST) {
            const uint32_t li = blockIdx.x + (uint32_t)it * gridDim.x;
            if (li >= nlist) break;
            const Ovf e = p.list[li];
            if ((int)e.c != cl) {
                cl = (int)e.c;
                load_combo(cl);
                part = p.part + (size_t)cl * p.n;
            }
            beg = e.beg;
            cnt = e.m;
            inst_id = e.pad;
#pragma unroll
            for (int b = 0; b < MAXB; ++b) {
                const int pos = threadIdx.x + b * TH;
                cur[b] = (cnt <= (uint32_t)CAP && pos < (int)cnt) ? part[beg + pos] : ~0ull;
            }
        } else {
            if (ub >= bk1) break;
            beg = nbeg;
            cnt = ncnt;
            dsh = dsh0 + (um ? 1 : 0);
#pragma unroll
            for (int b = 0; b < MAXB; ++b) cur[b] = key[b];
            const int bk = ub;
            ub += um ? 2 : 1;
            has_next = ub < bk1;
            if (has_next) {
                um = merged_at(ub);
                nbeg = base[ub];
                ncnt = base[ub + (um ? 2 : 1)] - nbeg;
#pragma unroll
                for (int b = 0; b < MAXB; ++b) {
                    const int pos = threadIdx.x + b * TH;
                    key[b] = (ncnt <= (uint32_t)CAP && pos < (int)ncnt) ? part[nbeg + pos] : ~0ull;
                }
            }
            if (BATCH) inst_id = ba.bucket_inst[bk];
        }
        if (BATCH) {
            const int r = ba.inst[inst_id].r;
            dsh = 64 - r - DIGIT;
            if (inst_id != cur_inst) {
                out.flush();
                cur_inst = inst_id;
                o_pairs = ba.inst[inst_id].pairs;
                o_cap = (unsigned long long)ba.inst[inst_id].cap;
                o_counter = ba.m_dev + inst_id;
                o_off = (uint32_t)ba.inst[inst_id].off;
                out.out = o_pairs;
                out.cap = o_cap;
                out.counter = o_counter;
            }
        }
        __syncthreads();  // LDS of the previous bucket is free, hist is zero
        if (HIER && !GT && tab_c != cl) {
            // the partition's bitmap, read only after the histogram's barrier
            const int words = max(1, (1 << p.k) >> 5);
            for (int e = threadIdx.x; e < words; e += TH) dtabL[e] = dtabG[e];
            tab_c = cl;
        }
        if (cnt < 2) continue;
        if (cnt > (uint32_t)CAP) {
            if (threadIdx.x == 0) {
                if (LIST) {
                    const uint32_t o = atomicAdd(p.ovf2_count, 1u);
                    p.ovf2[o] = Ovf{(uint32_t)cl, beg, cnt, inst_id};
                } else {
                    const uint32_t o = atomicAdd(p.ovf_count, 1u);
                    p.ovf[o] = Ovf{(uint32_t)cl, beg, cnt, inst_id};
                }
            }
            continue;
        }
        const int m = (int)cnt;
        if (threadIdx.x == 0) {
            claimRun = 0;
            claimPair = 0;
        }
        // Strings of the bucket's points, requested now and used after the
        // histogram and the run claims, which hide the load latency.
        // Batches of slots at or above m are empty for every thread; the
        // uniform tests on b * TH < m skip them with scalar branches.
        uint64_t sreg[MAXB][W];
        if (PREF && use_pre) {
#pragma unroll
            for (int b = 0; b < MAXB; ++b)
#pragma unroll
                for (int w = 0; w < W; ++w) sreg[b][w] = nsreg[b][w];
        } else {
#pragma unroll
            for (int b = 0; b < MAXB; ++b) {
                const int pos = threadIdx.x + b * TH;
#pragma unroll
                for (int w = 0; w < W; ++w) sreg[b][w] = 0ull;
                if (b * TH < m && pos < m) {
                    const uint64_t idx = (uint32_t)cur[b];
#pragma unroll
                    for (int w = 0; w < W; ++w) sreg[b][w] = p.S[idx * W + w];
                }
            }
        }

        // histogram of the in-bucket digit; the returned count is the rank
        uint32_t dig[MAXB], rank[MAXB];
#pragma unroll
        for (int b = 0; b < MAXB; ++b) {
            const int pos = threadIdx.x + b * TH;
            dig[b] = (uint32_t)(cur[b] >> dsh) & (BINS - 1);
            rank[b] = 0xFFFFFFFFu;
            if (b * TH < m && pos < m) rank[b] = atomicAdd(&hist[dig[b]], 1u);
        }
        __syncthreads();

        // the first member of each run claims the run and its member range
        uint32_t c[MAXB];
#pragma unroll
        for (int b = 0; b < MAXB; ++b) {
            c[b] = 0u;
            if (b * TH >= m) continue;
            c[b] = rank[b] != 0xFFFFFFFFu ? hist[dig[b]] : 0u;
        }
        __syncthreads();  // every count is read before the claims reuse hist
#pragma unroll
        for (int b = 0; b < MAXB; ++b) {
            if (b * TH < m && rank[b] == 0 && c[b] >= 2) {
                const unsigned long long old = atomicAdd(&claimRun, (1ull << 32) | (unsigned long long)c[b]);
                const uint32_t r = (uint32_t)(old >> 32);
                const uint32_t ms = (uint32_t)old;
                hist[dig[b]] = ms | (r << 16);
                runS[r] = (uint16_t)ms;
                runL[r] = (uint16_t)c[b];
                runBlk[r] = 0ull;
            }
        }
        __syncthreads();

        // the next bucket's strings are requested now (its keys arrived
        // long ago) and arrive behind this bucket's pairs
        if (PREF && has_next && ncnt >= 2u && ncnt <= (uint32_t)CAP) {
#pragma unroll
            for (int b = 0; b < MAXB; ++b) {
                const int pos = threadIdx.x + b * TH;
#pragma unroll
                for (int w = 0; w < W; ++w) nsreg[b][w] = 0ull;
                if (b * TH < (int)ncnt && pos < (int)ncnt) {
                    const uint64_t idx = (uint32_t)key[b];
#pragma unroll
                    for (int w = 0; w < W; ++w) nsreg[b][w] = p.S[idx * W + w];
                }
            }
            pre = true;
        }
        // scatter run members and gather their strings
        uint32_t rfirst[MAXB], rrun[MAXB];
#pragma unroll
        for (int b = 0; b < MAXB; ++b) {
            rfirst[b] = 0u;
            rrun[b] = 0u;
            if (b * TH < m && c[b] >= 2) {
                const uint32_t packed = hist[dig[b]];
                rfirst[b] = packed & 0xFFFFu;
                rrun[b] = packed >> 16;
                const uint32_t q = rfirst[b] + rank[b];
                idxB[q] = (uint32_t)cur[b];
#pragma unroll
                for (int w = 0; w < W; ++w) sl[q * W + w] = sreg[b][w] & p.valid[w];
            }
        }
        const uint32_t nruns = (uint32_t)(claimRun >> 32);
        __syncthreads();
        // Each member marks the blocks of hi (hierarchically: all blocks) in
        // which it differs from the run's first member; the histogram is
        // cleared for the next bucket.
#pragma unroll
        for (int b = 0; b < MAXB; ++b) {
            if (b * TH < m && rank[b] != 0xFFFFFFFFu) {
                if ((hi || HIER) && c[b] >= 2 && rank[b] > 0) {
                    const uint32_t first = rfirst[b];
                    const uint32_t q = first + rank[b];
                    uint64_t x[W];
#pragma unroll
                    for (int w = 0; w < W; ++w) x[w] = sl[q * W + w] ^ sl[first * W + w];
                    uint64_t bits = 0;
                    if constexpr (HIER) {
                        // every block in which the member differs from the first
                        if constexpr (HM != 1) {
                            bits = diff_blocks_of<W, HM>(x, p);
                        } else {
                            for (int blk = 0; blk < p.k; ++blk) {
                                uint64_t any = 0;
#pragma unroll
                                for (int w = 0; w < W; ++w) any |= x[w] & bmL[blk * W + w];
                                bits |= any ? (1ull << blk) : 0ull;
                            }
                        }
                        if (bits) atomicOr(&runBlk[rrun[b]], (unsigned long long)bits);
                    } else if constexpr (HM < 0) {
                        bits = diff_blocks_of<W, -HM>(x, p) & hi;
                        if (bits) atomicOr(&runBlk[rrun[b]], (unsigned long long)bits);
                    } else {
#pragma unroll
                        for (int s2 = 0; s2 < MAXHI; ++s2) {
                            uint64_t any = 0;
#pragma unroll
                            for (int w = 0; w < W; ++w) any |= x[w] & hm[s2][w];
                            bits |= (s2 < nhi && any) ? (1ull << hb[s2]) : 0ull;
                        }
                        uint64_t need = hi_rest;
                        while (need) {
                            const int blk = __builtin_ctzll(need);
                            need &= need - 1;
                            uint64_t any = 0;
#pragma unroll
                            for (int w = 0; w < W; ++w) any |= x[w] & bmL[blk * W + w];
                            bits |= any ? (1ull << blk) : 0ull;
                        }
                        if (bits) atomicOr(&runBlk[rrun[b]], (unsigned long long)bits);
                    }
                }
                hist[dig[b]] = 0;
            }
        }
        if (nruns == 0) continue;
        if (hi || HIER) __syncthreads();

        // Each run claims its pairs, unless it cannot hold a pair to write:
        // a pair is written only if it differs in every block of `hi`, so a
        // block of `hi` that is constant over the whole run rules it out.
        for (uint32_t r = threadIdx.x; r < nruns; r += TH) {
            const int s0 = runS[r], L = runL[r];
            bool live;
            if constexpr (HIER) {
                // some difference set of the family fits in the run's varying blocks
                const uint64_t v = runBlk[r];
                live = nfam < 0;  // no family stored: keep every run
                for (int f = 0; f < nfam; ++f) live |= (fam[f] & ~v) == 0ull;
            } else {
                live = (runBlk[r] & hi) == hi;
            }
            if (live) {
                const unsigned long long old =
                    atomicAdd(&claimPair, (1ull << 32) | (unsigned long long)(L * (L - 1) / 2));
                const uint32_t q = (uint32_t)(old >> 32);
                liveS[q] = (uint16_t)s0;
                liveL[q] = (uint16_t)L;
                liveP[q] = (uint32_t)old;
            }
        }
        __syncthreads();
        const uint32_t nlive = (uint32_t)(claimPair >> 32);
        const uint32_t P = (uint32_t)claimPair;
        if (P == 0) continue;

        // Flat loop over all claimed pairs (a < b), row-major per run. Each
        // lane walks cpl consecutive pairs: as few as spread P over the
        // workgroup, at most PMAX, so that most buckets take a single
        // round with every lane busy. It keeps the results in a bit mask and
        // appends the passing pairs once per round, walking its pairs a
        // second time for their point indices.
        constexpr uint32_t PMAX = LIST ? BK_PAIR_MAX / 2 : BK_PAIR_MAX;  // the second pass has more lanes
        const int cpl = (int)min(PMAX, (P + TH - 1) / TH);
        // next pair in row-major order over the live runs; the walk keeps
        // the member slots ia < ib of the pair and the end e of its run
        // (slot s0 + L), so every slot it yields lies inside a run and
        // below CAP; past the last run it stays on the last run
        auto advance = [&](int& r, int& ia, int& ib, int& e) {
            ++ib;
            if (ib == e) {
                ++ia;
                ib = ia + 1;
                if (ib >= e) {
                    ++r;
                    const int rr = min(r, (int)nlive - 1);
                    ia = liveS[rr];
                    ib = ia + 1;
                    e = ia + liveL[rr];
                }
            }
        };
        for (uint32_t t0 = 0; t0 < P; t0 += TH * (uint32_t)cpl) {
            const uint32_t t = t0 + threadIdx.x * (uint32_t)cpl;
            int r = 0, ia = 0, ib = 1, e = 2;
            int nq = 0;  // pairs of this lane
            if (t < P) {
                int lo = 0, hi2 = (int)nlive;
                while (hi2 - lo > 1) {
                    const int mid = (lo + hi2) >> 1;
                    if (liveP[mid] <= t) lo = mid;
                    else hi2 = mid;
                }
                r = lo;
                const int L = liveL[r];
                const int s0 = liveS[r];
                const uint32_t u = t - liveP[r];
                // row a of the upper triangle starts at f(a) = a (2L - a - 1) / 2;
                // the float root is within one of the integer answer
                const float q = (float)(2 * L - 1);
                int aa = (int)((q - sqrtf(q * q - 8.0f * (float)u)) * 0.5f);
                aa = max(0, min(aa, L - 2));
                if (aa < L - 2 && (uint32_t)((aa + 1) * (2 * L - aa - 2) / 2) <= u) ++aa;
                if (aa > 0 && (uint32_t)(aa * (2 * L - aa - 1) / 2) > u) --aa;
                ia = s0 + aa;
                ib = ia + 1 + (int)(u - (uint32_t)(aa * (2 * L - aa - 1) / 2));
                e = s0 + L;
                nq = (int)min((uint32_t)cpl, P - t);
            }
            const int r_0 = r, ia_0 = ia, ib_0 = ib, e_0 = e;
            uint64_t ok0 = 0, ok1 = 0;  // results of pairs 0-63 and 64-127
            {
                // the next candidate's strings are requested before the
                // current one is tested; two candidates per trip so that
                // the two string sets swap roles without copies. Results go
                // to four 32-pair words, each its own unrolled loop.
                uint64_t sa[W], sb[W], na[W], nb[W];
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    sa[w] = sl[ia * W + w];
                    sb[w] = sl[ib * W + w];
                }
                uint32_t wd[4];
#pragma unroll
                for (int qw = 0; qw < 4; ++qw) {
                    uint32_t cur = 0;
                    if (qw * 32 < cpl) {  // the same on every lane
                        for (int qi = 0; qi < 32; qi += 2) {
                            if (qw * 32 + qi >= nq) break;
                            advance(r, ia, ib, e);
#pragma unroll
                            for (int w = 0; w < W; ++w) {
                                na[w] = sl[ia * W + w];
                                nb[w] = sl[ib * W + w];
                            }
                            cur |= (uint32_t)pair_ok_fast<W, HM, GT>(sa, sb, p, keep, hm, nhi, hi_rest, bmask, hi,
                                                                     dtabL, dtabG, bmL)
                                   << qi;
                            if (qw * 32 + qi + 1 >= nq) break;
                            advance(r, ia, ib, e);
#pragma unroll
                            for (int w = 0; w < W; ++w) {
                                sa[w] = sl[ia * W + w];
                                sb[w] = sl[ib * W + w];
                            }
                            cur |= (uint32_t)pair_ok_fast<W, HM, GT>(na, nb, p, keep, hm, nhi, hi_rest, bmask, hi,
                                                                     dtabL, dtabG, bmL)
                                   << (qi + 1);
                        }
                    }
                    wd[qw] = cur;
                }
                ok0 = (uint64_t)wd[0] | ((uint64_t)wd[1] << 32);
                ok1 = (uint64_t)wd[2] | ((uint64_t)wd[3] << 32);
            }
            // point indices are read from LDS only for the pairs that pass
            auto bit_of = [&](int q) -> bool { return q < 64 ? ((ok0 >> q) & 1ull) : ((ok1 >> (q - 64)) & 1ull); };
            if (p.rep > 0 && (ok0 | ok1)) {
                int r2 = r_0, ia2 = ia_0, ib2 = ib_0, e2 = e_0;
                for (int q = 0; q < nq; ++q) {
                    if (bit_of(q) && !far_in_earlier<W>(p, idxB[ia2], idxB[ib2])) {
                        if (q < 64) ok0 &= ~(1ull << q);
                        else ok1 &= ~(1ull << (q - 64));
                    }
                    advance(r2, ia2, ib2, e2);
                }
            }
            // one append per lane per round: wave prefix of the counts, one
            // LDS atomic per wave
            const uint32_t nmine = (uint32_t)(__popcll(ok0) + __popcll(ok1));
            const uint32_t incl = msm::wave_incl_scan(nmine);
            const uint32_t wtot = __shfl(incl, 63, 64);
            uint32_t wbase = 0;
            if (wtot) {
                if (__lane_id() == 0) wbase = atomicAdd(&ocnt, wtot);
                wbase = __shfl(wbase, 0, 64);
            }
            uint32_t slot = wbase + incl - nmine;
            // slots at or above BK_OUT do not fit in LDS: they go to the
            // global list directly, reserved with one atomic per wave
            const uint32_t first_out = max(wbase, (uint32_t)BK_OUT);
            const uint32_t nover = (wtot && wbase + wtot > (uint32_t)BK_OUT) ? wbase + wtot - first_out : 0u;
            unsigned long long gbase = 0;
            if (nover) {
                if (__lane_id() == 0) gbase = atomicAdd(o_counter, (unsigned long long)nover);
                gbase = __shfl(gbase, 0, 64);
            }
            if (nmine) {
                int r2 = r_0, ia2 = ia_0, ib2 = ib_0, e2 = e_0;
                // up to the last passing pair
                const int qend = ok1 ? 128 - __builtin_clzll(ok1) : 64 - __builtin_clzll(ok0);
                for (int q = 0; q < qend; ++q) {
                    if (bit_of(q)) {
                        const uint32_t iq = idxB[ia2], jq = idxB[ib2];
                        const uint32_t lo2 = (iq < jq ? iq : jq) - o_off;
                        const uint32_t hi3 = (iq < jq ? jq : iq) - o_off;
                        if (slot < (uint32_t)BK_OUT) {
                            obuf[slot] = make_uint2(lo2, hi3);
                        } else {
                            const unsigned long long g = gbase + (slot - first_out);
                            if (g < o_cap) *reinterpret_cast<uint2*>(o_pairs + 2 * g) = make_uint2(lo2, hi3);
                        }
                        ++slot;
                    }
                    advance(r2, ia2, ib2, e2);
                }
            }
            if (t0 + TH * (uint32_t)cpl < P) out.maybe_flush(BK_OUT / 2);
        }
        out.maybe_flush(BK_OUT / 2);
    }
    out.flush();
}

// -------------------------------------------------------------------------
// 3. buckets above BK_CAP: all pairs, tile against tile, from HBM. A pair
// is tested only when the full 32-bit mixes agree.

struct BigShared {
    uint64_t* kR;
    uint64_t* kC;
    uint64_t* sR;
    uint64_t* sC;
    const uint64_t* bmL;
};

// Tile pair u (row-major over the upper triangle, diagonal included) of
// overflow bucket e. Called by every thread of the workgroup.
template <int W>
__device__ __forceinline__ void big_tile(const Params& p, const Ovf& e, int64_t u, BigShared sh,
                                         msm::PairStager<BK_OUT>& out, uint32_t o_off)
{
    const int64_t nT = (e.m + BIG_TILE - 1) / BIG_TILE;
    const double q = (double)(2 * nT + 1);
    int64_t ta = (int64_t)((q - sqrt(q * q - 8.0 * (double)u)) * 0.5);
    ta = max<int64_t>(0, min<int64_t>(ta, nT - 1));
    while (ta < nT - 1 && (ta + 1) * (2 * nT - ta) / 2 <= u) ++ta;
    while (ta > 0 && ta * (2 * nT - ta + 1) / 2 > u) --ta;
    const int64_t tb = ta + (u - ta * (2 * nT - ta + 1) / 2);

    const Combo* cb = p.combos + e.c;
    uint64_t keep[W];
    load_keep<W>(cb, keep);
    const uint64_t hi = cb->hi;
    const uint64_t* part = p.part + (size_t)e.c * p.n + e.beg;
    const int64_t ra = ta * BIG_TILE + threadIdx.x;
    const int64_t ca = tb * BIG_TILE + threadIdx.x;
    const bool rv = ra < (int64_t)e.m;
    const bool cv = ca < (int64_t)e.m;
    __syncthreads();  // the previous tile's LDS is free
    sh.kR[threadIdx.x] = rv ? part[ra] : 0ull;
    sh.kC[threadIdx.x] = cv ? part[ca] : 0ull;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        sh.sR[threadIdx.x * W + w] = rv ? p.S[(uint64_t)(uint32_t)sh.kR[threadIdx.x] * W + w] : 0ull;
        sh.sC[threadIdx.x * W + w] = cv ? p.S[(uint64_t)(uint32_t)sh.kC[threadIdx.x] * W + w] : 0ull;
    }
    __syncthreads();
    const int ncol = (int)min<int64_t>(BIG_TILE, (int64_t)e.m - tb * BIG_TILE);
    const uint32_t mine = (uint32_t)(sh.kR[threadIdx.x] >> 32);
    const bool diag = ta == tb;
    const uint32_t ii = (uint32_t)sh.kR[threadIdx.x];
    for (int jj = 0; jj < ncol; ++jj) {
        const uint64_t kc = sh.kC[jj];
        bool ok = rv && (!diag || jj > (int)threadIdx.x) && (uint32_t)(kc >> 32) == mine;
        if (ok) ok = pair_ok<W>(&sh.sR[threadIdx.x * W], &sh.sC[jj * W], p, keep, hi,
                                        p.dtab ? p.dtab + cb->dtoff : nullptr, sh.bmL);
        const uint32_t jv = (uint32_t)kc;
        if (ok && p.rep > 0) ok = far_in_earlier<W>(p, ii, jv);
        out.push(ok, (ii < jv ? ii : jv) - o_off, (ii < jv ? jv : ii) - o_off);
        if ((jj & 7) == 7) out.maybe_flush(BK_OUT / 2);
    }
    out.flush();
}

// Tile-pair counts of the overflow list, prefix-summed on the device:
// tile0[o] = first tile pair of entry o, tile0[novf] = total. One workgroup.
__global__ __launch_bounds__(1024) void k_ovf_prefix(const Ovf* __restrict__ ovf,
                                                     const uint32_t* __restrict__ ovf_count, uint32_t ovf_cap,
                                                     uint64_t* __restrict__ tile0)
{
    __shared__ unsigned long long wsum[16];
    __shared__ unsigned long long carry;
    const uint32_t novf = min(*ovf_count, ovf_cap);
    if (threadIdx.x == 0) {
        carry = 0;
        tile0[0] = 0;
    }
    __syncthreads();
    for (uint32_t c0 = 0; c0 < novf; c0 += 1024) {
        const uint32_t o = c0 + threadIdx.x;
        unsigned long long v = 0;
        if (o < novf) {
            const unsigned long long t = (ovf[o].m + BIG_TILE - 1) / BIG_TILE;
            v = t * (t + 1) / 2;
        }
        unsigned long long incl = v;
        const int l = threadIdx.x & 63;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const unsigned long long t = __shfl_up(incl, off, 64);
            if (l >= off) incl += t;
        }
        if (l == 63) wsum[threadIdx.x >> 6] = incl;
        __syncthreads();
        unsigned long long pre = carry;
        for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) pre += wsum[w];
        if (o < novf) tile0[o + 1] = pre + incl;
        __syncthreads();
        if (threadIdx.x == 1023) carry = pre + incl;
        __syncthreads();
    }
}

// Buckets above every LDS pass's capacity: a fixed grid takes tile pairs
// from a device work counter until the total of the overflow list
// (k_ovf_prefix) is reached, so the launch needs nothing from the host. In a
// batch (BATCH) output goes to the instance of the overflowing bucket
// (Ovf::pad) with indices local to it, else to p.pairs. With `too_big` set,
// a list of more than BIG_TILE_LIMIT tile pairs (a group of some 16M equal
// strings) is not started and the flag is raised instead.
constexpr uint64_t BIG_TILE_LIMIT = 0x7FFFFFFFull;

template <int W, bool BATCH>
__global__ __launch_bounds__(BIG_TILE) void k_big(Params p, BatchArgs ba, const Ovf* __restrict__ ovf,
                                                 const uint32_t* __restrict__ ovf_count, uint32_t ovf_cap,
                                                 const uint64_t* __restrict__ tile0,
                                                 unsigned long long* __restrict__ work, uint32_t* too_big)
{
    __shared__ uint64_t kR[BIG_TILE], kC[BIG_TILE];
    __shared__ uint64_t sR[BIG_TILE * W], sC[BIG_TILE * W];
    __shared__ uint64_t bmL[MAXK * W];
    __shared__ uint2 obuf[BK_OUT];
    __shared__ uint32_t ocnt;
    __shared__ unsigned long long ogb;
    __shared__ unsigned long long task;
    if (threadIdx.x == 0) ocnt = 0;
    msm::PairStager<BK_OUT> out{obuf, &ocnt, &ogb, p.pairs, p.cap, p.counter};
    for (int x = threadIdx.x; x < p.k * W; x += BIG_TILE) bmL[x] = p.bm[(x / W) * MAXW + (x % W)];
    const int novf = (int)min(*ovf_count, ovf_cap);
    const uint64_t total = tile0[novf];
    if (too_big && total > BIG_TILE_LIMIT) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *too_big = 1u;
        return;
    }
    while (true) {
        __syncthreads();  // everyone has read the previous task
        if (threadIdx.x == 0) task = atomicAdd(work, 1ull);
        __syncthreads();
        const uint64_t tix = task;
        if (tix >= total) break;
        int lo = 0, hi2 = novf;
        while (hi2 - lo > 1) {
            const int mid = (lo + hi2) >> 1;
            if (tile0[mid] <= tix) lo = mid;
            else hi2 = mid;
        }
        const Ovf e = ovf[lo];
        uint32_t o_off = 0;
        if (BATCH) {
            // output to the bucket's instance
            const BInst& in = ba.inst[e.pad];
            out.out = in.pairs;
            out.cap = (unsigned long long)in.cap;
            out.counter = ba.m_dev + e.pad;
            o_off = (uint32_t)in.off;
        }
        big_tile<W>(p, e, (int64_t)(tix - tile0[lo]), BigShared{kR, kC, sR, sC, bmL}, out, o_off);
    }
}

// Grouping probe: the first `sample` strings hashed on one grouping's kept
// characters into PROBE_BINS bins.
constexpr int PROBE_LOG = 14;
constexpr int PROBE_BINS = 1 << PROBE_LOG;
constexpr int PROBE_HIER = 64;  // hierarchical groupings probed, at most
constexpr int PROBE_STD = 4;    // per-combination groupings probed

// Rows blockIdx.y < nh of the grid probe hierarchical groupings hc + y * hs,
// the next ns rows per-combination groupings sc + (y - nh) * ss, the last
// row the whole string (full). The sum of squared bin sizes of each kind is
// accumulated on the way into sumsq[kind]: a bin going from c to c + 1
// members adds 2c + 1 to it. 256 threads per workgroup.
template <int W>
__global__ __launch_bounds__(256) void k_probe_groups(const uint64_t* __restrict__ S, int64_t sample,
                                                      const Combo* __restrict__ hc, int nh, int hs,
                                                      const Combo* __restrict__ sc, int ns, int ss,
                                                      const Combo* __restrict__ full, uint32_t* __restrict__ hist,
                                                      unsigned long long* sumsq)
{
    __shared__ unsigned long long wsum[4];
    const int y = (int)blockIdx.y;
    const int kind = y < nh ? 0 : (y < nh + ns ? 1 : 2);
    const Combo* cb = kind == 0 ? hc + (size_t)y * hs : (kind == 1 ? sc + (size_t)(y - nh) * ss : full);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long v = 0;
    if (i < sample) {
        uint64_t keep[W], s[W];
        load_keep<W>(cb, keep);
        load_string<W>(S, (uint64_t)i, s);
        const uint32_t old =
            atomicAdd(&hist[(size_t)y * PROBE_BINS + (masked_mix<W>(s, keep) >> (32 - PROBE_LOG))], 1u);
        v = 2ull * old + 1ull;
    }
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = wsum[0] + wsum[1] + wsum[2] + wsum[3];
        if (t) atomicAdd(sumsq + kind, t);
    }
}

__global__ void k_zero_u64(unsigned long long* a, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0ull;
}

__global__ void k_zero_u32(uint32_t* a, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0u;
}

int64_t binom(int a, int b)
{
    if (b < 0 || b > a) return 0;
    int64_t r = 1;
    for (int t = 1; t <= b; ++t) {
        r = r * (a - b + t) / t;
        if (r > (1ll << 40)) return r;
    }
    return r;
}

// Block masks (the first ell mod k blocks get one extra bit), the mask of
// the ell valid characters, and one Combo per h-subset of the k blocks.
inline void build_tables(int ell, int k, int h, std::vector<uint64_t>& bm, uint64_t (&valid)[MAXW],
                         std::vector<Combo>& combos)
{
    // Blocks of nearly equal length: the first ell mod k get one extra bit.
    bm.assign((size_t)k * MAXW, 0ull);
    {
        int pos = 0;
        for (int b = 0; b < k; ++b) {
            const int len = ell / k + (b < ell % k ? 1 : 0);
            for (int c = pos; c < pos + len; ++c) bm[(size_t)b * MAXW + (c >> 6)] |= 1ull << (c & 63);
            pos += len;
        }
    }
    for (int w = 0; w < MAXW; ++w) valid[w] = 0;
    for (int c = 0; c < ell; ++c) valid[c >> 6] |= 1ull << (c & 63);

    // All h-subsets of the k blocks.
    combos.clear();
    {
        std::vector<int> sel(h);
        for (int t = 0; t < h; ++t) sel[t] = t;
        while (true) {
            Combo cb{};
            uint64_t Bm = 0;
            for (int t = 0; t < h; ++t) Bm |= 1ull << sel[t];
            for (int w = 0; w < MAXW; ++w) {
                uint64_t kw = valid[w];
                for (int t = 0; t < h; ++t) kw &= ~bm[(size_t)sel[t] * MAXW + w];
                cb.keep[w] = kw;
            }
            int lowest_kept = 0;
            while (lowest_kept < k && ((Bm >> lowest_kept) & 1ull)) ++lowest_kept;
            uint64_t hi = 0;
            for (int b = lowest_kept + 1; b < k; ++b)
                if ((Bm >> b) & 1ull) hi |= 1ull << b;
            cb.hi = hi;
            cb.amask = Bm;
            cb.nhi = __builtin_popcountll(hi);
            {
                int slot = 0;
                for (int b = 0; b < k && slot < MAXHI; ++b)
                    if ((hi >> b) & 1ull) {
                        for (int w = 0; w < MAXW; ++w) cb.himask[slot][w] = bm[(size_t)b * MAXW + w];
                        ++slot;
                    }
            }
            combos.push_back(cb);
            int t = h - 1;
            while (t >= 0 && sel[t] == k - h + t) --t;
            if (t < 0) break;
            sel[t]++;
            for (int u = t + 1; u < h; ++u) sel[u] = sel[u - 1] + 1;
        }
    }
}

// Partitions of the hierarchical grouping on j blocks (see diff_blocks)
// with each one's family of difference sets: its minimal members (fam, for
// the run pruning) and all of them as a bitmap over the 2^k sets (dtab).
// Every member of a family leaves the blocks outside the family's union
// unchanged, so a partition groups on all of those, A among them: pairs
// that differ there can never be written in it. The smallest j is taken
// whose j * floor(ell / k) characters of A reach log2(n) + 8, so that
// unrelated points rarely share a group; returns false when no such j needs
// fewer groupings than the C(k, h) combinations, or when k is too large to
// list the difference sets.
inline bool build_hier_tables(int ell, int k, int h, int64_t n, const std::vector<uint64_t>& bm,
                              const uint64_t (&valid)[MAXW], std::vector<Combo>& parts, std::vector<uint64_t>& fam,
                              std::vector<uint32_t>& dtab, int& jsel)
{
    if (k > 16 || h < 1 || k - h < 1) return false;
    const uint64_t kmask = (1ull << k) - 1;
    const double need = std::log2((double)std::max<int64_t>(n, 2)) + 8.0;
    const int64_t ncomb = binom(k, h);
    for (int j = 1; j <= k - h; ++j) {
        if ((double)(j * (ell / k)) < need) continue;
        std::map<uint64_t, std::vector<uint64_t>> fams;
        for (uint64_t D = 0; D <= kmask; ++D) {
            if (__builtin_popcountll(D) > h) continue;
            uint64_t B = D, fill = kmask & ~D;
            for (int t = __builtin_popcountll(D); t < h; ++t) {
                B |= fill & (~fill + 1);
                fill &= fill - 1;
            }
            uint64_t U = kmask & ~B, A = 0;
            for (int t = 0; t < j; ++t) {
                A |= U & (~U + 1);
                U &= U - 1;
            }
            fams[A].push_back(D);
        }
        if ((int64_t)fams.size() >= ncomb) return false;  // a larger j only adds partitions
        parts.clear();
        fam.clear();
        dtab.clear();
        const size_t words = std::max<size_t>(1, ((size_t)1 << k) / 32);
        for (const auto& kv : fams) {
            Combo cb{};
            uint64_t uni = 0;
            for (uint64_t D : kv.second) uni |= D;
            const uint64_t keepb = kmask & ~uni;  // contains A
            for (int w = 0; w < MAXW; ++w) {
                uint64_t kw = 0;
                for (int b = 0; b < k; ++b)
                    if ((keepb >> b) & 1ull) kw |= bm[(size_t)b * MAXW + w];
                cb.keep[w] = kw & valid[w];
            }
            cb.hi = 0;
            cb.nhi = 0;
            cb.amask = kv.first;
            cb.dtoff = (uint32_t)dtab.size();
            dtab.resize(dtab.size() + words, 0u);
            for (uint64_t D : kv.second) dtab[cb.dtoff + (D >> 5)] |= 1u << (D & 31);
            cb.famoff = (uint32_t)fam.size();
            for (uint64_t D : kv.second) {
                bool minimal = true;
                for (uint64_t E : kv.second)
                    if (E != D && (E & ~D) == 0) {
                        minimal = false;
                        break;
                    }
                if (minimal) fam.push_back(D);
            }
            cb.nfam = (int32_t)(fam.size() - cb.famoff);
            parts.push_back(cb);
        }
        jsel = j;
        return true;
    }
    return false;
}

}  // namespace
