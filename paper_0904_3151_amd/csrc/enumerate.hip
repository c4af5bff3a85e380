// Multiple sorting method with blockwise masking (Sections 2.1-2.2) on gfx950:
// host driver of msm_enumerate_pairs and msm_enumerate_replicates. The
// method and its kernels are described in msm_enum.h.
#include "msm_enum.h"

#include <cstring>

namespace {

// The bucket kernel instantiated for the grouping mode hm (one grouping per
// combination: 0, or -8, -16, -32 for blocks of that many characters;
// hierarchical: 8, 16 or 32 for blocks of that many characters, 1 for other
// layouts; GT when the family bitmaps over 2^k
// difference sets are too large for LDS): the first pass, or (large) the
// second pass over buckets above the first pass's capacity.
template <int W, int HM, bool GT>
void launch_bucket_mode(bool large, dim3 grid, hipStream_t stream, const Params& p)
{
    if (large)
        hipLaunchKernelGGL((k_bucket<W, BK_DIGIT_L, false, large_threads<W>(), true, large_maxb<W>(), HM, GT>),
                           grid, dim3(large_threads<W>()), 0, stream, p, BatchArgs{});
    else if (W >= 3 || p.rep > 0)
        hipLaunchKernelGGL((k_bucket<W, BK_DIGIT, false, BK_THREADS_WIDE, false, BK_MAXB_WIDE, HM, GT>), grid,
                           dim3(BK_THREADS_WIDE), 0, stream, p, BatchArgs{});
    else if constexpr (W <= 2)
        hipLaunchKernelGGL((k_bucket<W, BK_DIGIT, false, BK_THREADS, false, BK_MAXB, HM, GT>), grid,
                           dim3(BK_THREADS), 0, stream, p, BatchArgs{});
}

template <int W, bool GT>
void launch_bucket_hier(int hm, bool large, dim3 grid, hipStream_t stream, const Params& p)
{
    switch (hm) {
    case 8: launch_bucket_mode<W, 8, GT>(large, grid, stream, p); break;
    case 16: launch_bucket_mode<W, 16, GT>(large, grid, stream, p); break;
    case 32: launch_bucket_mode<W, 32, GT>(large, grid, stream, p); break;
    default: launch_bucket_mode<W, 1, GT>(large, grid, stream, p); break;
    }
}

template <int W>
void launch_bucket(int hm, bool large, dim3 grid, hipStream_t stream, const Params& p)
{
    if (hm == 0) launch_bucket_mode<W, 0, false>(large, grid, stream, p);
    else if (hm == -8) launch_bucket_mode<W, -8, false>(large, grid, stream, p);
    else if (hm == -16) launch_bucket_mode<W, -16, false>(large, grid, stream, p);
    else if (hm == -32) launch_bucket_mode<W, -32, false>(large, grid, stream, p);
    else if (p.k <= DT_LDS_K) launch_bucket_hier<W, false>(hm, large, grid, stream, p);
    else launch_bucket_hier<W, true>(hm, large, grid, stream, p);
}

// Device memory of one enumeration, carved from one buffer: the host tables
// first (in one piece, so that one copy uploads them), then the counters,
// the probe's histograms and the partition arrays of Cg groupings.
struct EnumMem {
    Combo* combos_std;
    Combo* combos_h;
    Combo* full;
    uint64_t* fam;
    uint32_t* dtab;
    uint64_t* bm;
    size_t table_bytes;
    unsigned long long* counter;
    uint32_t* ovfc;
    uint64_t* part;
    uint32_t* keys;
    uint32_t* counts;
    uint32_t* probe;
    unsigned long long* work;
    uint32_t* base;
    Ovf* ovf;
    Ovf* ovf2;
    uint64_t* tile0;
};

// Lays EnumMem out from c.base (NULL: only sizes, in c.off).
inline EnumMem carve_enum(msm::Carver& c, int Cstd, int Ch, size_t nfam, size_t ndtab, int k, bool probe,
                          int Cg, int64_t n, int nt, int nb, bool keys)
{
    EnumMem m{};
    m.combos_std = c.take<Combo>((size_t)Cstd);
    m.combos_h = c.take<Combo>((size_t)std::max(1, Ch));
    m.full = c.take<Combo>(1);
    m.fam = c.take<uint64_t>(std::max<size_t>(1, nfam));
    m.dtab = c.take<uint32_t>(std::max<size_t>(1, ndtab));
    m.bm = c.take<uint64_t>((size_t)k * MAXW);
    m.table_bytes = c.off;
    m.counter = c.take<unsigned long long>(4);
    m.ovfc = c.take<uint32_t>(4);
    m.part = c.take<uint64_t>((size_t)Cg * n);
    m.keys = c.take<uint32_t>(keys ? (size_t)Cg * n : 1);
    m.counts = c.take<uint32_t>((size_t)Cg * nt * nb);
    m.probe = c.take<uint32_t>(probe ? (size_t)(PROBE_HIER + PROBE_STD + 1) * PROBE_BINS : 1);
    m.work = c.take<unsigned long long>(1);
    m.base = c.take<uint32_t>((size_t)Cg * (nb + 1));
    m.ovf = c.take<Ovf>((size_t)Cg * nb);
    m.ovf2 = c.take<Ovf>((size_t)Cg * nb);
    m.tile0 = c.take<uint64_t>((size_t)Cg * nb + 1);
    return m;
}

// ext == NULL: the work memory is the context's scratch, grown as needed and
// at most about 3 GB of partition arrays per launch group. Otherwise it is
// the ext_bytes at ext (device memory the call does not own) and the host
// tables go up through the context's pinned staging buffer, so the call
// allocates nothing; it fails with MSM_E_UNSUPPORTED when one grouping's
// arrays do not fit.
template <int W>
msm_status run_enumerate(msm_ctx* ctx, const uint64_t* S, int64_t n, int ell, int Q, int k, int h,
                         uint32_t* pairs, int64_t cap, int64_t* m_out, hipStream_t stream, void* ext,
                         size_t ext_bytes)
{
    std::vector<uint64_t> bm;
    uint64_t valid[MAXW];
    std::vector<Combo> combos;
    build_tables(ell, k, h, bm, valid, combos);
    // grouping on fewer blocks when it needs fewer passes (a candidate;
    // a probe of the data below decides)
    std::vector<Combo> parts;
    std::vector<uint64_t> fam;
    std::vector<uint32_t> dtab;
    int jsel = 0;
    const bool hier_cand = build_hier_tables(ell, k, h, n, bm, valid, parts, fam, dtab, jsel);
    const int Cstd = (int)combos.size();
    const int Ch = hier_cand ? (int)parts.size() : 0;
    const int Cmax = std::max(Cstd, Ch);

    // Partition shape.
    int r1 = 0;
    while (r1 < 13 && ((int64_t)1 << r1) * TARGET_BUCKET < n) ++r1;
    const int nb = 1 << r1;
    // points per partition tile (at most 256 tiles per combination); the
    // scatter sorts a tile in LDS chunks of sch points, as many as fit
    // beside its two words per bucket
    int T = SCAT_THREADS * SCAT_PPT;
    while ((n + T - 1) / T > 256) T *= 2;
    const int nt = (int)((n + T - 1) / T);
    int sch = SCAT_THREADS * SCAT_PPT;
    while (sch > SCAT_THREADS && (size_t)sch * 8 + (size_t)nb * 8 > (size_t)150 * 1024) sch /= 2;
    const size_t scat_lds = (size_t)sch * 8 + (size_t)nb * 8;

    // Combinations per launch group, bounded by the memory for them. The
    // count pass keeps the masked mixes for the scatter (4 bytes per point
    // and combination instead of its string), except in the no-allocation
    // call, whose buffer then holds more points.
    const bool keys = ext == nullptr;
    const size_t per_combo = msm::align_up((size_t)n * 8, 256) + (keys ? msm::align_up((size_t)n * 4, 256) : 0) +
                             msm::align_up((size_t)nt * nb * 4, 256) +
                             msm::align_up((size_t)(nb + 1) * 4, 256) + 3 * msm::align_up((size_t)nb * sizeof(Ovf), 256);
    auto bytes_for = [&](int cg) {
        msm::Carver c;
        carve_enum(c, Cstd, Ch, fam.size(), dtab.size(), k, hier_cand, cg, n, nt, nb, keys);
        return c.off;
    };
    const size_t budget = (size_t)3 << 30;
    int Cg = (int)std::max<size_t>(1, std::min<size_t>((size_t)Cmax, budget / per_combo));
    Cg = std::min(Cg, 65535);
    if (ext) {
        const size_t fixed = bytes_for(0);
        if (fixed >= ext_bytes || bytes_for(1) > ext_bytes)
            return msm::fail(ctx, MSM_E_UNSUPPORTED,
                             "msm_enumerate_pairs_noalloc: n=%lld strings need %zu bytes of work memory, above "
                             "the %zu of the no-allocation buffer",
                             (long long)n, bytes_for(1), ext_bytes);
        Cg = (int)std::min<size_t>((size_t)Cg, (ext_bytes - fixed) / per_combo);
        Cg = std::max(Cg, 1);
        while (Cg > 1 && bytes_for(Cg) > ext_bytes) --Cg;
    }

    void* scr = ext;
    if (!ext) {
        msm_status st = msm::ctx_scratch(ctx, bytes_for(Cg), stream, &scr);
        if (st != MSM_OK) return st;
    }
    msm::Carver c2;
    c2.base = static_cast<char*>(scr);
    const EnumMem mem = carve_enum(c2, Cstd, Ch, fam.size(), dtab.size(), k, hier_cand, Cg, n, nt, nb, keys);
    const size_t table_bytes = mem.table_bytes;
    if (ext && table_bytes > msm::NOALLOC_STAGE_BYTES)
        return msm::fail(ctx, MSM_E_UNSUPPORTED,
                         "msm_enumerate_pairs_noalloc: %zu bytes of tables for k=%d, h=%d exceed the %zu-byte "
                         "staging buffer",
                         table_bytes, k, h, msm::NOALLOC_STAGE_BYTES);
    Combo* d_combos_std = mem.combos_std;
    Combo* d_combos_h = mem.combos_h;
    Combo* d_full = mem.full;
    uint64_t* d_fam = mem.fam;
    uint32_t* d_dtab = mem.dtab;
    uint64_t* d_bm = mem.bm;
    unsigned long long* d_counter = mem.counter;
    uint32_t* d_ovfc = mem.ovfc;
    uint64_t* d_part = mem.part;
    uint32_t* d_counts = mem.counts;
    uint32_t* d_probe = mem.probe;
    unsigned long long* d_work = mem.work;
    uint32_t* d_base = mem.base;
    Ovf* d_ovf = mem.ovf;
    Ovf* d_ovf2 = mem.ovf2;
    uint64_t* d_tile0 = mem.tile0;

    {
        Combo full{};  // the whole string kept: groups of identical strings
        for (int w = 0; w < MAXW; ++w) full.keep[w] = valid[w];
        // pageable host memory, or the pinned staging buffer when nothing may
        // be allocated (the call synchronises the stream before it returns,
        // so the copy has read the buffer before its next use)
        std::vector<char> own(ext ? 0 : table_bytes, 0);
        char* blob = ext ? ctx->host_stage : own.data();
        if (ext) std::memset(blob, 0, table_bytes);
        auto put = [&](const void* dev, const void* src, size_t bytes) {
            if (bytes) std::memcpy(blob + (static_cast<const char*>(dev) - c2.base), src, bytes);
        };
        put(d_combos_std, combos.data(), sizeof(Combo) * Cstd);
        put(d_combos_h, parts.data(), sizeof(Combo) * Ch);
        put(d_full, &full, sizeof(Combo));
        put(d_fam, fam.data(), sizeof(uint64_t) * fam.size());
        put(d_dtab, dtab.data(), sizeof(uint32_t) * dtab.size());
        put(d_bm, bm.data(), sizeof(uint64_t) * bm.size());
        MSM_HIP(ctx, hipMemcpyAsync(c2.base, blob, table_bytes, hipMemcpyHostToDevice, stream));
    }
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, stream, d_counter, 4);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, stream, d_ovfc, 4);

    Params p{};
    p.S = S;
    p.Sall = S;
    p.rep_stride = (uint64_t)n * W;
    p.rep = 0;
    p.n = n;
    p.bm = d_bm;
    p.k = k;
    p.h = h;
    for (int w = 0; w < MAXW; ++w) p.valid[w] = valid[w];
    p.r1 = r1;
    p.nb = nb;
    p.T = T;
    p.nt = nt;
    p.sch = sch;
    p.counts = d_counts;
    p.base = d_base;
    p.part = d_part;
    p.keys = keys ? mem.keys : nullptr;
    p.pairs = pairs;
    p.cap = (unsigned long long)cap;
    p.counter = d_counter;
    p.ovf = d_ovf;
    p.ovf_count = d_ovfc;
    p.blk_r = ell % k;
    p.blk_L = ell / k;
    p.dL = (p.blk_r == 0 && (p.blk_L == 8 || p.blk_L == 16 || p.blk_L == 32)) ? p.blk_L : 0;
    p.blk_m1 = ((1ull << 32) + (uint64_t)(p.blk_L + 1) - 1) / (uint64_t)(p.blk_L + 1);
    p.blk_m0 = ((1ull << 32) + (uint64_t)p.blk_L - 1) / (uint64_t)p.blk_L;
    p.list = d_ovf;
    p.list_count = d_ovfc;
    p.ovf2 = d_ovf2;
    p.ovf2_count = d_ovfc + 1;

    // Probe: the first PROBE_BINS strings are grouped (a 14-bit hash of the
    // kept characters) on every hierarchical grouping (up to PROBE_HIER,
    // evenly spaced), on PROBE_STD per-combination groupings and on the
    // whole string. Pairs of identical strings are dropped by the run
    // pruning in all but one grouping of either kind, every other pair in a
    // group is tested; so each kind costs about its groupings times (pairs
    // in groups - identical pairs + one unit per point), scaled to n.
    // Strings with little entropy in some blocks (learned codes, for one)
    // merge many groups when only those j blocks are kept.
    bool hier = hier_cand;
    if (hier_cand) {
        const int nsh = std::min(PROBE_HIER, Ch), nss = std::min(PROBE_STD, Cstd);
        const int hst = Ch / nsh, sst = Cstd / nss;
        const int64_t sample = std::min<int64_t>(n, PROBE_BINS);
        uint32_t* hist = d_probe;
        const int nh = nsh + nss + 1;
        hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)(((int64_t)nh * PROBE_BINS + 255) / 256)), dim3(256), 0,
                           stream, hist, nh * PROBE_BINS);
        const unsigned pg = (unsigned)((sample + 255) / 256);
        hipLaunchKernelGGL((k_probe_groups<W>), dim3(pg, nh), dim3(256), 0, stream, S, sample, d_combos_h, nsh, hst,
                           d_combos_std, nss, sst, d_full, hist, d_counter + 1);
        MSM_HIP(ctx, hipGetLastError());
        MSM_HIP(ctx, hipMemcpyAsync(ctx->host_words, d_counter + 1, 3 * sizeof(uint64_t), hipMemcpyDeviceToHost,
                                    stream));
        MSM_HIP(ctx, hipStreamSynchronize(stream));
        // sum of squared group sizes = points + 2 * pairs in groups; pairs
        // grow as (n / sample)^2 and points as n / sample to the full data
        const double sq_h = (double)ctx->host_words[0] / nsh, sq_s = (double)ctx->host_words[1] / nss;
        const double sq_f = (double)ctx->host_words[2];
        const double pts = (double)sample, up = (double)n / (double)sample;
        const double cost_h = (double)Ch * (std::max(0.0, sq_h - sq_f) / 2.0 * up + pts);
        const double cost_s = (double)Cstd * (std::max(0.0, sq_s - sq_f) / 2.0 * up + pts);
        hier = cost_h < cost_s;
    }
    Combo* d_combos = hier ? d_combos_h : d_combos_std;
    const int C = hier ? Ch : Cstd;
    Cg = std::min(Cg, C);
    p.hier = hier ? 1 : 0;
    p.fam = hier ? d_fam : nullptr;
    p.dtab = hier ? d_dtab : nullptr;
    const int hm = hier ? (p.dL ? p.dL : 1) : -p.dL;
    ctx->last_groupings = C;
    ctx->last_jblocks = hier ? jsel : 0;

    if (scat_lds > 65536)  // above the default dynamic LDS limit of a launch
        MSM_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(&k_part_scatter<W>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)scat_lds));
    for (int rep = 0; rep < Q; ++rep) {
    p.rep = rep;
    p.S = S + (uint64_t)rep * p.rep_stride;
    for (int c0 = 0; c0 < C; c0 += Cg) {
        const int cc = std::min(Cg, C - c0);
        p.combos = d_combos + c0;
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, stream, d_ovfc, 3);  // [3] is the too-big flag
        p.units = cc * nt;
        const unsigned part_grid = (unsigned)((p.units + NUM_XCD - 1) / NUM_XCD * NUM_XCD);
        {
            msm::KernelTimer kt(ctx, stream, "k_part_count");
            hipLaunchKernelGGL((k_part_count<W>), dim3(part_grid), dim3(PART_THREADS), nb * sizeof(uint32_t), stream,
                               p);
        }
        {
            msm::KernelTimer kt(ctx, stream, "k_part_scan");
            hipLaunchKernelGGL(k_part_colscan, dim3((nb + PART_THREADS - 1) / PART_THREADS, cc), dim3(PART_THREADS), 0,
                               stream, p);
            hipLaunchKernelGGL(k_part_scan, dim3(cc), dim3(SCAN_THREADS), (nb + 32) * sizeof(uint32_t), stream, p);
        }
        {
            msm::KernelTimer kt(ctx, stream, "k_part_scatter");
            hipLaunchKernelGGL((k_part_scatter<W>), dim3(part_grid), dim3(SCAT_THREADS), scat_lds, stream, p);
        }
        {
            msm::KernelTimer kt(ctx, stream, "k_bucket");
            launch_bucket<W>(hm, false, dim3((nb + bk_group<W>() - 1) / bk_group<W>(), cc), stream, p);
        }
        // Buckets above the first pass's capacity: a second pass with more
        // threads and LDS takes those up to its own capacity, then tile pairs
        // take the rest. Both read their work lists on the device with fixed
        // grids, so the host does not wait for the first pass.
        const uint32_t list_cap = (uint32_t)cc * (uint32_t)nb;
        p.list_cap = list_cap;
        const unsigned pgrid = (unsigned)std::min<int64_t>(list_cap, 2 * (int64_t)ctx->num_cu);
        {
            msm::KernelTimer kt(ctx, stream, "k_bucket_large");
            launch_bucket<W>(hm, true, dim3(pgrid), stream, p);
        }
        {
            msm::KernelTimer kt(ctx, stream, "k_big");
            hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, stream, d_work, 1);
            hipLaunchKernelGGL(k_ovf_prefix, dim3(1), dim3(1024), 0, stream, d_ovf2, d_ovfc + 1, list_cap, d_tile0);
            hipLaunchKernelGGL((k_big<W, false>), dim3((unsigned)(2 * ctx->num_cu)), dim3(BIG_TILE), 0, stream, p,
                               BatchArgs{}, d_ovf2, d_ovfc + 1, list_cap, d_tile0, d_work, d_ovfc + 3);
        }
        MSM_HIP(ctx, hipGetLastError());
    }
    }
    MSM_HIP(ctx, hipMemcpyAsync(ctx->host_words, d_counter, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                stream));
    MSM_HIP(ctx, hipMemcpyAsync(ctx->host_words + 1, d_ovfc + 3, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    MSM_HIP(ctx, hipStreamSynchronize(stream));
    if (static_cast<uint32_t>(ctx->host_words[1]) != 0u)
        return msm::fail(ctx, MSM_E_UNSUPPORTED, "msm_enumerate_pairs: a group of equal strings is too large");
    const int64_t m = (int64_t)ctx->host_words[0];
    *m_out = m;
    if (m > cap && !(pairs == nullptr && cap == 0))
        return msm::fail(ctx, MSM_E_CAPACITY, "msm_enumerate_pairs: %lld pairs do not fit in cap=%lld",
                         (long long)m, (long long)cap);
    return MSM_OK;
}

}  // namespace

static msm_status enumerate_entry(const char* fn, msm_ctx* ctx, const uint64_t* S, int64_t n, int32_t ell,
                                  int32_t Q, int32_t k, int32_t h, uint32_t* pairs, int64_t cap, int64_t* m_out,
                                  void* stream, bool noalloc = false)
{
    if (!ctx) return msm::fail(nullptr, MSM_E_INVALID, "%s: ctx is NULL", fn);
    ctx->err.clear();
    if (!m_out) return msm::fail(ctx, MSM_E_INVALID, "%s: m_out is NULL", fn);
    *m_out = 0;
    if (n < 0 || n > 0xFFFFFFFFll) return msm::fail(ctx, MSM_E_INVALID, "%s: n=%lld out of range", fn, (long long)n);
    if (ell < 1 || ell > 256) return msm::fail(ctx, MSM_E_INVALID, "%s: ell=%d not in [1, 256]", fn, ell);
    if (Q < 1 || Q > 4096) return msm::fail(ctx, MSM_E_INVALID, "%s: Q=%d not in [1, 4096]", fn, Q);
    if (h < 0 || k <= h || k > ell)
        return msm::fail(ctx, MSM_E_INVALID, "%s: need 0 <= h < k <= ell (k=%d, h=%d)", fn, k, h);
    if (k > MAXK) return msm::fail(ctx, MSM_E_UNSUPPORTED, "%s: k=%d above %d", fn, k, MAXK);
    if (binom(k, h) > 65536)
        return msm::fail(ctx, MSM_E_UNSUPPORTED, "%s: C(%d, %d) combinations above 65536", fn, k, h);
    if (cap < 0) return msm::fail(ctx, MSM_E_INVALID, "%s: cap < 0", fn);
    if (cap > 0 && !pairs) return msm::fail(ctx, MSM_E_INVALID, "%s: pairs is NULL with cap > 0", fn);
    if (pairs && (reinterpret_cast<uintptr_t>(pairs) & 7))
        return msm::fail(ctx, MSM_E_INVALID, "%s: pairs must be 8-byte aligned", fn);
    if (n < 2) return MSM_OK;
    if (!S) return msm::fail(ctx, MSM_E_INVALID, "%s: S is NULL", fn);
    msm_status st = msm::use_device(ctx);
    if (st != MSM_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    void* ext = nullptr;
    size_t ext_bytes = 0;
    if (noalloc) {
        if (!ctx->noalloc_scratch || !ctx->host_stage)
            return msm::fail(ctx, MSM_E_UNSUPPORTED, "%s: no static scratch on device %d", fn, ctx->device);
        ext = ctx->noalloc_scratch;
        ext_bytes = msm::NOALLOC_SCRATCH_BYTES;
    }
    switch ((ell + 63) / 64) {
        case 1: return run_enumerate<1>(ctx, S, n, ell, Q, k, h, pairs, cap, m_out, s, ext, ext_bytes);
        case 2: return run_enumerate<2>(ctx, S, n, ell, Q, k, h, pairs, cap, m_out, s, ext, ext_bytes);
        case 3: return run_enumerate<3>(ctx, S, n, ell, Q, k, h, pairs, cap, m_out, s, ext, ext_bytes);
        default: return run_enumerate<4>(ctx, S, n, ell, Q, k, h, pairs, cap, m_out, s, ext, ext_bytes);
    }
}

extern "C" msm_status msm_enumerate_pairs(msm_ctx* ctx, const uint64_t* S, int64_t n, int32_t ell,
                                          int32_t k, int32_t h, uint32_t* pairs, int64_t cap,
                                          int64_t* m_out, void* stream)
{
    return enumerate_entry("msm_enumerate_pairs", ctx, S, n, ell, 1, k, h, pairs, cap, m_out, stream);
}

extern "C" msm_status msm_enumerate_pairs_noalloc(msm_ctx* ctx, const uint64_t* S, int64_t n, int32_t ell,
                                                  int32_t k, int32_t h, uint32_t* pairs, int64_t cap,
                                                  int64_t* m_out, void* stream)
{
    return enumerate_entry("msm_enumerate_pairs_noalloc", ctx, S, n, ell, 1, k, h, pairs, cap, m_out, stream, true);
}

extern "C" msm_status msm_enumerate_replicates(msm_ctx* ctx, const uint64_t* S, int64_t n, int32_t ell,
                                               int32_t Q, int32_t k, int32_t h, uint32_t* pairs, int64_t cap,
                                               int64_t* m_out, void* stream)
{
    return enumerate_entry("msm_enumerate_replicates", ctx, S, n, ell, Q, k, h, pairs, cap, m_out, stream);
}

extern "C" msm_status msm_enumerate_groupings(int64_t n, int32_t ell, int32_t k, int32_t h, int32_t* groupings,
                                              int32_t* jblocks)
{
    if (!groupings || !jblocks || n < 0 || ell < 1 || ell > 256 || h < 0 || k <= h || k > ell || k > MAXK ||
        binom(k, h) > 65536)
        return MSM_E_INVALID;
    std::vector<uint64_t> bm;
    uint64_t valid[MAXW];
    std::vector<Combo> combos, parts;
    std::vector<uint64_t> fam;
    std::vector<uint32_t> dtab;
    build_tables(ell, k, h, bm, valid, combos);
    int jsel = 0;
    if (build_hier_tables(ell, k, h, n, bm, valid, parts, fam, dtab, jsel)) {
        *groupings = (int32_t)parts.size();
        *jblocks = jsel;
    } else {
        *groupings = (int32_t)combos.size();
        *jblocks = 0;
    }
    return MSM_OK;
}

extern "C" msm_status msm_enumerate_last_plan(const msm_ctx* ctx, int32_t* groupings, int32_t* jblocks)
{
    if (!ctx || !groupings || !jblocks) return MSM_E_INVALID;
    *groupings = ctx->last_groupings;
    *jblocks = ctx->last_jblocks;
    return MSM_OK;
}
