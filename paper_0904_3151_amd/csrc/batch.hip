// Many independent instances of the whole path (eq. (3) projection, then
// MSM with blockwise masking, Sections 2.1-2.2) in one enqueue that can be
// captured into a HIP graph.
//
// The instances' points are concatenated. Partition tiles never straddle an
// instance and every instance owns its own range of buckets, so the kernels
// of the single-problem path run once over the whole batch without ever
// pairing points of different instances. Tables (instance offsets, tile and
// bucket owners, combinations) are built and uploaded when the plan is
// created; a run only launches kernels: no copies, fills by kernel, no
// host synchronisation. Buckets too large for LDS are listed on the device
// and finished by a persistent kernel that takes tile pairs from a device
// work counter.
//
// The bucket size aimed at, the width of the in-bucket radix digit and the
// number of buckets per workgroup are chosen per class of instance size
// (all instances share ell, k and h, so the key width is the same for all):
// the instances are laid out class by class (points, tiles and buckets),
// the bucket kernel runs once per class with that class's digit and group,
// and at plan creation each class's candidates are timed on the batch itself
// while the other classes keep their best configuration so far.
#include "msm_enum.h"

#include <algorithm>
#include <cstring>
#include <memory>

namespace {

struct Config {
    int target;  // points per bucket aimed at
    int digit;   // in-bucket digit bits
    int group;   // buckets per workgroup
};

constexpr int BATCH_T = BSCAT_THREADS * BPART_PPT;  // points per partition tile
constexpr int MAX_R = 13;            // at most 8192 buckets per instance
constexpr int PROJ_ENTRY_ROWS = 1024;  // rows per projection entry (a multiple of the tile)

int bits_for(int64_t n, int target)
{
    int r = 0;
    while (r < MAX_R && ((int64_t)1 << r) * target < n) ++r;
    return r;
}

// Size classes of instances: [0, 8192), [8192, 65536), [65536, 2^32).
constexpr int NCLS = 3;
constexpr int64_t CLS_LO[NCLS] = {0, 8192, 65536};
constexpr int64_t CLS_HI[NCLS] = {8192, 65536, (int64_t)1 << 32};

int class_of(int64_t n)
{
    int c = 0;
    while (c + 1 < NCLS && n >= CLS_LO[c + 1]) ++c;
    return c;
}

}  // namespace

struct msm_batch {
    msm_ctx* ctx = nullptr;
    int count = 0, ell = 0, k = 0, h = 0, W = 1, C = 0, Cg = 1;
    int64_t N = 0;
    int max_d = 1;
    std::vector<msm_instance> inst;  // the caller's descriptors
    std::vector<int64_t> off;        // first point of each instance
    std::vector<int> ord;            // instances in layout order (by size class)
    std::vector<int> cls;            // size class of each instance
    int cls_b0[NCLS] = {0, 0, 0};    // buckets of each class: [cls_b0, cls_b1)
    int cls_b1[NCLS] = {0, 0, 0};
    std::vector<Combo> combos;
    std::vector<uint64_t> bm;
    uint64_t valid[MAXW] = {0, 0, 0, 0};

    // device memory owned by the plan
    void* mem = nullptr;
    msm::ProjInst* d_pinst = nullptr;
    msm::ProjEntry* d_pent = nullptr;
    int npent = 0;
    BInst* d_inst = nullptr;
    uint32_t* d_tile_inst = nullptr;
    uint32_t* d_bucket_inst = nullptr;
    Combo* d_combos = nullptr;
    uint64_t* d_bm = nullptr;
    uint64_t* d_S = nullptr;
    uint64_t* d_part = nullptr;
    uint32_t* d_counts = nullptr;
    uint32_t* d_base = nullptr;
    Ovf* d_ovf = nullptr;
    Ovf* d_ovf2 = nullptr;
    uint32_t* d_ovfc = nullptr;
    uint64_t* d_tile0 = nullptr;
    unsigned long long* d_work = nullptr;
    uint32_t* d_pwork = nullptr;  // entry counter of the projection

    // current configuration, per size class
    Config cfg[NCLS] = {{512, 10, 8}, {512, 10, 8}, {512, 10, 8}};
    int nt = 0;        // partition tiles
    int NB = 0;        // buckets
    int max_nbi = 1;   // largest bucket count of one instance
    uint64_t cnt_stride = 0;
    std::vector<msm_batch_config> tried;
    msm_batch_config chosen[NCLS] = {};

    // graph of one run, captured on a private stream
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t* graph_m = nullptr;
    // recorded on the caller's stream after each graph launch: the exec is
    // only destroyed once its last launch has finished
    hipEvent_t graph_done = nullptr;

    ~msm_batch()
    {
        if (graph_done) {
            (void)hipEventSynchronize(graph_done);
            (void)hipEventDestroy(graph_done);
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        if (mem) (void)hipFree(mem);
    }
};

namespace {

struct Sizes {
    int nt;
    int NB;
    int max_nbi;
    uint64_t cnt_stride;
};

Sizes sizes_for(const msm_batch& b, int target)
{
    Sizes z{0, 0, 1, 0};
    for (int i = 0; i < b.count; ++i) {
        const int64_t n = b.inst[i].n;
        const int r = bits_for(n, target);
        const int ntl = (int)((n + BATCH_T - 1) / BATCH_T);
        z.nt += ntl;
        z.NB += 1 << r;
        z.max_nbi = std::max(z.max_nbi, 1 << r);
        z.cnt_stride += (uint64_t)ntl << r;
    }
    return z;
}

// Builds and uploads the instance, tile and bucket tables of a
// configuration (one per size class). Instances are laid out in b.ord.
msm_status set_config(msm_batch& b, const Config (&c)[NCLS])
{
    msm_ctx* ctx = b.ctx;
    std::vector<BInst> bi(b.count);
    std::vector<uint32_t> tile_inst, bucket_inst;
    uint32_t tstart = 0, bstart = 0;
    uint64_t cnt_off = 0;
    int max_nbi = 1;
    for (int q = 0; q < NCLS; ++q) b.cls_b0[q] = b.cls_b1[q] = 0;
    int prev_cls = -1;
    for (int i : b.ord) {
        const int64_t n = b.inst[i].n;
        const int q = b.cls[i];
        if (q != prev_cls) {
            b.cls_b0[q] = (int)bstart;
            prev_cls = q;
        }
        const int r = bits_for(n, c[q].target);
        const uint32_t ntl = (uint32_t)((n + BATCH_T - 1) / BATCH_T);
        BInst& e = bi[i];
        e.off = (uint64_t)b.off[i];
        e.n = (uint32_t)n;
        e.r = r;
        e.bstart = bstart;
        e.tstart = tstart;
        e.ntiles = ntl;
        e.pad = 0;
        e.cnt_off = cnt_off;
        e.pairs = b.inst[i].pairs;
        e.cap = b.inst[i].cap;
        for (uint32_t t = 0; t < ntl; ++t) tile_inst.push_back((uint32_t)i);
        for (int x = 0; x < (1 << r); ++x) bucket_inst.push_back((uint32_t)i);
        tstart += ntl;
        bstart += 1u << r;
        b.cls_b1[q] = (int)bstart;
        cnt_off += (uint64_t)ntl << r;
        max_nbi = std::max(max_nbi, 1 << r);
    }
    MSM_HIP(ctx, hipMemcpy(b.d_inst, bi.data(), sizeof(BInst) * bi.size(), hipMemcpyHostToDevice));
    if (!tile_inst.empty())
        MSM_HIP(ctx, hipMemcpy(b.d_tile_inst, tile_inst.data(), 4 * tile_inst.size(), hipMemcpyHostToDevice));
    MSM_HIP(ctx, hipMemcpy(b.d_bucket_inst, bucket_inst.data(), 4 * bucket_inst.size(), hipMemcpyHostToDevice));
    for (int q = 0; q < NCLS; ++q) b.cfg[q] = c[q];
    b.nt = (int)tstart;
    b.NB = (int)bstart;
    b.max_nbi = max_nbi;
    b.cnt_stride = cnt_off;
    return MSM_OK;
}

// The bucket kernel over buckets [ba.bk_lo, ba.bk_hi).
template <int W, int DIGIT>
void launch_bucket(const Params& p, const BatchArgs& ba, int cc, hipStream_t s)
{
    const int nb = ba.bk_hi - ba.bk_lo;
    hipLaunchKernelGGL((k_bucket<W, DIGIT, true, BK_THREADS, false, BK_MAXB, 0, false>),
                       dim3((nb + ba.group - 1) / ba.group, cc), dim3(BK_THREADS), 0, s, p, ba);
}

template <int W>
void launch_bucket_digit(const Params& p, const BatchArgs& ba, int digit, int cc, hipStream_t s)
{
    if (digit <= 8) launch_bucket<W, 8>(p, ba, cc, s);
    else if (digit <= 10) launch_bucket<W, 10>(p, ba, cc, s);
    else launch_bucket<W, 12>(p, ba, cc, s);
}

// Enqueues the enumeration of every instance; the strings are in d_S.
template <int W>
msm_status enqueue_enumerate(msm_batch& b, int64_t* m_dev, hipStream_t s, bool timed)
{
    msm_ctx* ctx = b.ctx;
    const bool prof = timed && ctx->prof;
    Params p{};
    p.S = b.d_S;
    p.Sall = b.d_S;
    p.rep_stride = (uint64_t)b.N * W;
    p.rep = 0;
    p.n = b.N;
    p.bm = b.d_bm;
    p.k = b.k;
    p.h = b.h;
    for (int w = 0; w < MAXW; ++w) p.valid[w] = b.valid[w];
    p.r1 = 0;
    p.nb = b.NB;
    p.T = BATCH_T;
    p.nt = b.nt;
    p.counts = b.d_counts;
    p.base = b.d_base;
    p.part = b.d_part;
    p.pairs = nullptr;
    p.cap = 0;
    p.counter = nullptr;
    p.ovf = b.d_ovf;
    p.ovf_count = b.d_ovfc;
    p.list = b.d_ovf;
    p.list_count = b.d_ovfc;
    p.ovf2 = b.d_ovf2;
    p.ovf2_count = b.d_ovfc + 1;
    BatchArgs ba{b.d_inst, b.d_tile_inst, b.d_bucket_inst, b.cnt_stride, b.cfg[0].group,
                 reinterpret_cast<unsigned long long*>(m_dev), 0, b.NB};
    const int big_grid = 2 * ctx->num_cu;
    for (int c0 = 0; c0 < b.C; c0 += b.Cg) {
        const int cc = std::min(b.Cg, b.C - c0);
        p.combos = b.d_combos + c0;
        p.units = cc * b.nt;
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, b.d_ovfc, 4);
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, b.d_work, 1);
        if (p.units > 0) {
            const unsigned part_grid = (unsigned)((p.units + NUM_XCD - 1) / NUM_XCD * NUM_XCD);
            std::unique_ptr<msm::KernelTimer> kt;
            if (prof) kt.reset(new msm::KernelTimer(ctx, s, "k_bpart_count"));
            hipLaunchKernelGGL((k_bpart_count<W>), dim3(part_grid), dim3(PART_THREADS),
                               b.max_nbi * sizeof(uint32_t), s, p, ba);
            kt.reset();
            if (prof) kt.reset(new msm::KernelTimer(ctx, s, "k_bpart_scan"));
            hipLaunchKernelGGL(k_bpart_scan, dim3(b.count, cc), dim3(SCAN_THREADS), (b.max_nbi + 32) * sizeof(uint32_t),
                               s, p, ba);
            kt.reset();
            if (prof) kt.reset(new msm::KernelTimer(ctx, s, "k_bpart_scatter"));
            hipLaunchKernelGGL((k_bpart_scatter<W>), dim3(part_grid), dim3(BSCAT_THREADS),
                               (size_t)BATCH_T * 8 + (size_t)b.max_nbi * 8, s, p, ba, b.max_nbi);
            kt.reset();
            if (prof) kt.reset(new msm::KernelTimer(ctx, s, "k_bucket_batch"));
            for (int q = 0; q < NCLS; ++q) {
                if (b.cls_b1[q] <= b.cls_b0[q]) continue;
                BatchArgs bq = ba;
                bq.bk_lo = b.cls_b0[q];
                bq.bk_hi = b.cls_b1[q];
                bq.group = b.cfg[q].group;
                launch_bucket_digit<W>(p, bq, b.cfg[q].digit, cc, s);
            }
            kt.reset();
            // buckets above the first pass's capacity: a persistent second
            // pass with more threads and LDS, then tile pairs for the rest
            const uint32_t ovf_cap = (uint32_t)cc * (uint32_t)b.NB;
            p.list_cap = ovf_cap;
            if (prof) kt.reset(new msm::KernelTimer(ctx, s, "k_bucket_large_batch"));
            hipLaunchKernelGGL((k_bucket<W, BK_DIGIT_L, true, large_threads<W>(), true, large_maxb<W>(), 0, false>),
                               dim3((unsigned)std::min<uint32_t>(ovf_cap, (uint32_t)big_grid)),
                               dim3(large_threads<W>()), 0, s, p, ba);
            kt.reset();
            if (prof) kt.reset(new msm::KernelTimer(ctx, s, "k_big_batch"));
            hipLaunchKernelGGL(k_ovf_prefix, dim3(1), dim3(1024), 0, s, b.d_ovf2, b.d_ovfc + 1, ovf_cap, b.d_tile0);
            hipLaunchKernelGGL((k_big<W, true>), dim3(big_grid), dim3(BIG_TILE), 0, s, p, ba, b.d_ovf2, b.d_ovfc + 1,
                               ovf_cap, b.d_tile0, b.d_work, nullptr);
        }
        MSM_HIP(ctx, hipGetLastError());
    }
    return MSM_OK;
}

msm_status enqueue(msm_batch& b, int64_t* m_dev, hipStream_t s, bool timed)
{
    msm_ctx* ctx = b.ctx;
    hipLaunchKernelGGL(k_zero_u64, dim3((b.count + 255) / 256), dim3(256), 0, s,
                       reinterpret_cast<unsigned long long*>(m_dev), b.count);
    if (b.npent > 0) {
        std::unique_ptr<msm::KernelTimer> kt;
        if (timed && ctx->prof) kt.reset(new msm::KernelTimer(ctx, s, "k_project_batch"));
        const int grid = std::min(b.npent, 4 * ctx->num_cu);
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, b.d_pwork, 1);
        MSM_HIP(ctx, msm::batch_project(b.d_pinst, b.d_pent, b.npent, b.ell, b.max_d, grid, b.d_pwork, s));
    }
    switch (b.W) {
        case 1: return enqueue_enumerate<1>(b, m_dev, s, timed);
        case 2: return enqueue_enumerate<2>(b, m_dev, s, timed);
        case 3: return enqueue_enumerate<3>(b, m_dev, s, timed);
        default: return enqueue_enumerate<4>(b, m_dev, s, timed);
    }
}

msm_status enqueue_enum_any(msm_batch& b, int64_t* m_dev, hipStream_t s)
{
    return b.W == 1 ? enqueue_enumerate<1>(b, m_dev, s, false)
                    : (b.W == 2 ? enqueue_enumerate<2>(b, m_dev, s, false)
                                : (b.W == 3 ? enqueue_enumerate<3>(b, m_dev, s, false)
                                            : enqueue_enumerate<4>(b, m_dev, s, false)));
}

// Times the enumeration under the candidate configurations of each size
// class in turn (the strings must be in d_S), the other classes at their
// best so far, and keeps each class's fastest.
msm_status autotune(msm_batch& b, int64_t* m_dev, hipStream_t s)
{
    static const int targets[] = {256, 512, 1024};
    static const int digits[] = {8, 10, 12};
    static const int groups[] = {2, 8};
    msm_ctx* ctx = b.ctx;
    hipEvent_t e0, e1;
    MSM_HIP(ctx, hipEventCreate(&e0));
    MSM_HIP(ctx, hipEventCreate(&e1));
    Config best[NCLS];
    for (int q = 0; q < NCLS; ++q) best[q] = b.cfg[q];
    float best_ms[NCLS] = {-1.f, -1.f, -1.f};
    bool present[NCLS] = {false, false, false};
    for (int i = 0; i < b.count; ++i)
        if (b.inst[i].n > 0) present[b.cls[i]] = true;
    msm_status st = MSM_OK;
    for (int q = 0; q < NCLS && st == MSM_OK; ++q) {
        if (!present[q]) continue;
        for (int t : targets)
            for (int dg : digits)
                for (int g : groups) {
                    if (st != MSM_OK) break;
                    Config c[NCLS];
                    for (int x = 0; x < NCLS; ++x) c[x] = best[x];
                    c[q] = Config{t, dg, g};
                    MSM_HIP(ctx, hipStreamSynchronize(s));  // tables are replaced below
                    st = set_config(b, c);
                    if (st != MSM_OK) break;
                    hipLaunchKernelGGL(k_zero_u64, dim3((b.count + 255) / 256), dim3(256), 0, s,
                                       reinterpret_cast<unsigned long long*>(m_dev), b.count);
                    st = enqueue_enum_any(b, m_dev, s);  // warm-up
                    if (st != MSM_OK) break;
                    (void)hipEventRecord(e0, s);
                    st = enqueue_enum_any(b, m_dev, s);
                    if (st != MSM_OK) break;
                    (void)hipEventRecord(e1, s);
                    if (hipEventSynchronize(e1) != hipSuccess) {
                        st = msm::fail(ctx, MSM_E_HIP, "msm_batch_create: timing a configuration failed");
                        break;
                    }
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    b.tried.push_back(msm_batch_config{t, dg, g, ms, CLS_LO[q], CLS_HI[q]});
                    if (best_ms[q] < 0.f || ms < best_ms[q]) {
                        best_ms[q] = ms;
                        best[q] = c[q];
                    }
                }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != MSM_OK) return st;
    for (int q = 0; q < NCLS; ++q)
        b.chosen[q] = msm_batch_config{best[q].target, best[q].digit, best[q].group, best_ms[q], CLS_LO[q], CLS_HI[q]};
    return set_config(b, best);
}

}  // namespace

extern "C" msm_status msm_batch_create(msm_ctx* ctx, const msm_instance* inst, int32_t count, int32_t ell,
                                       int32_t k, int32_t h, int32_t autotune_flag, msm_batch** out, void* stream)
{
    if (!ctx) return msm::fail(nullptr, MSM_E_INVALID, "msm_batch_create: ctx is NULL");
    ctx->err.clear();
    if (!out) return msm::fail(ctx, MSM_E_INVALID, "msm_batch_create: out is NULL");
    *out = nullptr;
    if (!inst || count < 1 || count > 65535)
        return msm::fail(ctx, MSM_E_INVALID, "msm_batch_create: need 1 <= count <= 65535 and instances");
    if (ell < 1 || ell > 256) return msm::fail(ctx, MSM_E_INVALID, "msm_batch_create: ell=%d not in [1, 256]", ell);
    if (h < 0 || k <= h || k > ell)
        return msm::fail(ctx, MSM_E_INVALID, "msm_batch_create: need 0 <= h < k <= ell (k=%d, h=%d)", k, h);
    if (k > MAXK) return msm::fail(ctx, MSM_E_UNSUPPORTED, "msm_batch_create: k=%d above %d", k, MAXK);
    if (binom(k, h) > 65536)
        return msm::fail(ctx, MSM_E_UNSUPPORTED, "msm_batch_create: C(%d, %d) combinations above 65536", k, h);
    int64_t N = 0;
    int max_d = 1;
    for (int i = 0; i < count; ++i) {
        const msm_instance& e = inst[i];
        if (e.n < 0 || e.cap < 0)
            return msm::fail(ctx, MSM_E_INVALID, "msm_batch_create: instance %d has n < 0 or cap < 0", i);
        if (e.n > 0 && (!e.X || !e.R || !e.S || e.d < 1 || e.d > 65536 || e.ldx < e.d))
            return msm::fail(ctx, MSM_E_INVALID, "msm_batch_create: instance %d needs X, R, S and 1 <= d <= ldx", i);
        if (e.cap > 0 && (!e.pairs || (reinterpret_cast<uintptr_t>(e.pairs) & 7)))
            return msm::fail(ctx, MSM_E_INVALID,
                             "msm_batch_create: instance %d needs an 8-byte aligned pairs buffer for cap > 0", i);
        N += e.n;
        if (e.n > 0) max_d = std::max(max_d, (int)e.d);
    }
    if (N >= 0xFFFFFFFFll)
        return msm::fail(ctx, MSM_E_INVALID, "msm_batch_create: %lld points in total, need < 2^32", (long long)N);
    msm_status st = msm::use_device(ctx);
    if (st != MSM_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    std::unique_ptr<msm_batch> b(new msm_batch());
    b->ctx = ctx;
    b->count = count;
    b->ell = ell;
    b->k = k;
    b->h = h;
    b->W = (ell + 63) / 64;
    b->N = N;
    b->max_d = max_d;
    b->inst.assign(inst, inst + count);
    b->off.resize(count);
    b->cls.resize(count);
    b->ord.resize(count);
    for (int i = 0; i < count; ++i) {
        b->cls[i] = class_of(inst[i].n);
        b->ord[i] = i;
    }
    // instances laid out class by class, in their order within a class
    std::stable_sort(b->ord.begin(), b->ord.end(), [&](int x, int y) { return b->cls[x] < b->cls[y]; });
    {
        int64_t o = 0;
        for (int i : b->ord) {
            b->off[i] = o;
            o += inst[i].n;
        }
    }
    build_tables(ell, k, h, b->bm, b->valid, b->combos);
    b->C = (int)b->combos.size();

    // projection entries: runs of whole tiles of one instance
    std::vector<msm::ProjInst> pinst(count);
    std::vector<msm::ProjEntry> pent;
    const int rows_per_entry = std::max(PROJ_ENTRY_ROWS, msm::batch_project_rows(ell));
    for (int i = 0; i < count; ++i) {
        const msm_instance& e = inst[i];
        msm::ProjInst& q = pinst[i];
        q.X = e.X;
        q.n = e.n;
        q.ldx = e.ldx;
        q.R = e.R;
        q.S = e.S;
        q.d = e.d;
        q.vec4 = ((reinterpret_cast<uintptr_t>(e.X) & 15) == 0) && (e.ldx % 4 == 0);
        for (int64_t r0 = 0; r0 < e.n; r0 += rows_per_entry)
            pent.push_back(msm::ProjEntry{r0, (int32_t)std::min<int64_t>(rows_per_entry, e.n - r0), (uint32_t)i});
    }
    // costliest entries first: claimed in this order, they even out at the end
    std::stable_sort(pent.begin(), pent.end(), [&](const msm::ProjEntry& x, const msm::ProjEntry& y) {
        return (int64_t)x.rows * inst[x.inst].d > (int64_t)y.rows * inst[y.inst].d;
    });
    b->npent = (int)pent.size();

    // sizes: the smallest bucket target has the most buckets
    const Sizes zs = sizes_for(*b, autotune_flag ? 256 : 512);
    const size_t per_combo = msm::align_up((size_t)N * 8, 256) + msm::align_up(zs.cnt_stride * 4, 256) +
                             msm::align_up((size_t)(zs.NB + 1) * 4, 256) +
                             2 * msm::align_up((size_t)zs.NB * sizeof(Ovf), 256) +
                             msm::align_up((size_t)(zs.NB + 1) * 8, 256);
    const size_t budget = (size_t)3 << 30;
    b->Cg = (int)std::max<size_t>(1, std::min<size_t>((size_t)b->C, budget / std::max<size_t>(per_combo, 1)));
    b->Cg = std::min(b->Cg, 65535);
    const int Cg = b->Cg;
    msm::Carver cv;
    cv.take<msm::ProjInst>((size_t)count);
    cv.take<msm::ProjEntry>(std::max<size_t>(1, pent.size()));
    cv.take<BInst>((size_t)count);
    cv.take<uint32_t>((size_t)std::max(1, zs.nt));
    cv.take<uint32_t>((size_t)zs.NB);
    cv.take<Combo>((size_t)b->C);
    cv.take<uint64_t>((size_t)k * MAXW);
    cv.take<uint64_t>(std::max<size_t>(1, (size_t)N * b->W));
    cv.take<uint64_t>(std::max<size_t>(1, (size_t)Cg * N));
    cv.take<uint32_t>(std::max<size_t>(1, (size_t)Cg * zs.cnt_stride));
    cv.take<uint32_t>((size_t)Cg * (zs.NB + 1));
    cv.take<Ovf>((size_t)Cg * zs.NB);
    cv.take<Ovf>((size_t)Cg * zs.NB);
    cv.take<uint32_t>(4);
    cv.take<uint64_t>((size_t)Cg * zs.NB + 1);
    cv.take<unsigned long long>(1);
    cv.take<uint32_t>(1);
    {
        const hipError_t e = hipMalloc(&b->mem, cv.off);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            b->mem = nullptr;
            return msm::fail(ctx, MSM_E_NOMEM, "msm_batch_create: cannot allocate %zu bytes", cv.off);
        }
    }
    msm::Carver c2;
    c2.base = static_cast<char*>(b->mem);
    b->d_pinst = c2.take<msm::ProjInst>((size_t)count);
    b->d_pent = c2.take<msm::ProjEntry>(std::max<size_t>(1, pent.size()));
    b->d_inst = c2.take<BInst>((size_t)count);
    b->d_tile_inst = c2.take<uint32_t>((size_t)std::max(1, zs.nt));
    b->d_bucket_inst = c2.take<uint32_t>((size_t)zs.NB);
    b->d_combos = c2.take<Combo>((size_t)b->C);
    b->d_bm = c2.take<uint64_t>((size_t)k * MAXW);
    b->d_S = c2.take<uint64_t>(std::max<size_t>(1, (size_t)N * b->W));
    b->d_part = c2.take<uint64_t>(std::max<size_t>(1, (size_t)Cg * N));
    b->d_counts = c2.take<uint32_t>(std::max<size_t>(1, (size_t)Cg * zs.cnt_stride));
    b->d_base = c2.take<uint32_t>((size_t)Cg * (zs.NB + 1));
    b->d_ovf = c2.take<Ovf>((size_t)Cg * zs.NB);
    b->d_ovf2 = c2.take<Ovf>((size_t)Cg * zs.NB);
    b->d_ovfc = c2.take<uint32_t>(4);
    b->d_tile0 = c2.take<uint64_t>((size_t)Cg * zs.NB + 1);
    b->d_work = c2.take<unsigned long long>(1);
    b->d_pwork = c2.take<uint32_t>(1);
    for (int i = 0; i < count; ++i) pinst[i].S2 = b->d_S + (size_t)b->off[i] * b->W;
    MSM_HIP(ctx, hipMemcpy(b->d_pinst, pinst.data(), sizeof(msm::ProjInst) * count, hipMemcpyHostToDevice));
    if (!pent.empty())
        MSM_HIP(ctx, hipMemcpy(b->d_pent, pent.data(), sizeof(msm::ProjEntry) * pent.size(), hipMemcpyHostToDevice));
    MSM_HIP(ctx, hipMemcpy(b->d_combos, b->combos.data(), sizeof(Combo) * b->C, hipMemcpyHostToDevice));
    MSM_HIP(ctx, hipMemcpy(b->d_bm, b->bm.data(), sizeof(uint64_t) * b->bm.size(), hipMemcpyHostToDevice));
    MSM_HIP(ctx, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    MSM_HIP(ctx, hipEventCreateWithFlags(&b->graph_done, hipEventDisableTiming));
    {
        // the partition scatter stages a whole tile and two words per bucket in LDS
        const int lds = BATCH_T * 8 + (1 << MAX_R) * 8;
        const void* f = b->W == 1   ? reinterpret_cast<const void*>(&k_bpart_scatter<1>)
                        : b->W == 2 ? reinterpret_cast<const void*>(&k_bpart_scatter<2>)
                        : b->W == 3 ? reinterpret_cast<const void*>(&k_bpart_scatter<3>)
                                    : reinterpret_cast<const void*>(&k_bpart_scatter<4>);
        MSM_HIP(ctx, hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    }

    {
        const Config c0[NCLS] = {{512, 10, 8}, {512, 10, 8}, {512, 10, 8}};
        st = set_config(*b, c0);
        if (st != MSM_OK) return st;
        for (int q = 0; q < NCLS; ++q) b->chosen[q] = msm_batch_config{512, 10, 8, -1.f, CLS_LO[q], CLS_HI[q]};
    }
    if (autotune_flag && N >= 2) {
        // project once, then time the enumeration under each candidate
        int64_t* m_tmp = nullptr;
        MSM_HIP(ctx, hipMalloc(&m_tmp, sizeof(int64_t) * count));
        st = enqueue(*b, m_tmp, s, false);
        if (st == MSM_OK) st = autotune(*b, m_tmp, s);
        const hipError_t e = hipStreamSynchronize(s);
        (void)hipFree(m_tmp);
        if (st != MSM_OK) return st;
        MSM_HIP(ctx, e);
    }
    *out = b.release();
    return MSM_OK;
}

extern "C" msm_status msm_batch_run(msm_batch* b, int64_t* m_dev, void* stream)
{
    if (!b) return msm::fail(nullptr, MSM_E_INVALID, "msm_batch_run: batch is NULL");
    msm_ctx* ctx = b->ctx;
    ctx->err.clear();
    if (!m_dev || (reinterpret_cast<uintptr_t>(m_dev) & 7))
        return msm::fail(ctx, MSM_E_INVALID, "msm_batch_run: m_dev must be an 8-byte aligned device array");
    msm_status st = msm::use_device(ctx);
    if (st != MSM_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    MSM_HIP(ctx, hipStreamIsCapturing(s, &cs));
    return enqueue(*b, m_dev, s, cs == hipStreamCaptureStatusNone);
}

extern "C" msm_status msm_batch_launch_graph(msm_batch* b, int64_t* m_dev, void* stream)
{
    if (!b) return msm::fail(nullptr, MSM_E_INVALID, "msm_batch_launch_graph: batch is NULL");
    msm_ctx* ctx = b->ctx;
    ctx->err.clear();
    if (!m_dev || (reinterpret_cast<uintptr_t>(m_dev) & 7))
        return msm::fail(ctx, MSM_E_INVALID, "msm_batch_launch_graph: m_dev must be an 8-byte aligned device array");
    msm_status st = msm::use_device(ctx);
    if (st != MSM_OK) return st;
    if (!b->exec || b->graph_m != m_dev) {
        if (b->exec) {
            // the old exec was launched on a caller's stream: wait for it
            MSM_HIP(ctx, hipEventSynchronize(b->graph_done));
            MSM_HIP(ctx, hipGraphExecDestroy(b->exec));
            b->exec = nullptr;
        }
        if (b->graph) {
            MSM_HIP(ctx, hipGraphDestroy(b->graph));
            b->graph = nullptr;
        }
        MSM_HIP(ctx, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
        st = enqueue(*b, m_dev, b->cap_stream, false);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
        if (st != MSM_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        MSM_HIP(ctx, e);
        b->graph = g;
        MSM_HIP(ctx, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->graph_m = m_dev;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    std::unique_ptr<msm::KernelTimer> kt;
    if (ctx->prof) kt.reset(new msm::KernelTimer(ctx, s, "batch_graph"));
    MSM_HIP(ctx, hipGraphLaunch(b->exec, s));
    MSM_HIP(ctx, hipEventRecord(b->graph_done, s));
    return MSM_OK;
}

extern "C" msm_status msm_batch_tuning(const msm_batch* b, msm_batch_config* chosen, int32_t chosen_cap,
                                       int32_t* n_chosen, msm_batch_config* tried, int32_t cap, int32_t* n_tried)
{
    if (!b) return msm::fail(nullptr, MSM_E_INVALID, "msm_batch_tuning: batch is NULL");
    if (cap < 0 || (cap > 0 && !tried) || chosen_cap < 0 || (chosen_cap > 0 && !chosen))
        return msm::fail(b->ctx, MSM_E_INVALID, "msm_batch_tuning: bad cap");
    // the classes that hold instances, in order of size
    int nc = 0;
    for (int q = 0; q < NCLS; ++q) {
        bool present = false;
        for (int i = 0; i < b->count; ++i) present = present || (b->inst[i].n > 0 && b->cls[i] == q);
        if (!present) continue;
        if (nc < chosen_cap) chosen[nc] = b->chosen[q];
        ++nc;
    }
    if (n_chosen) *n_chosen = nc;
    if (n_tried) *n_tried = (int32_t)b->tried.size();
    for (int i = 0; i < cap && i < (int)b->tried.size(); ++i) tried[i] = b->tried[i];
    return MSM_OK;
}

extern "C" void msm_batch_destroy(msm_batch* b)
{
    if (!b) return;
    if (b->ctx) (void)msm::use_device(b->ctx);
    delete b;
}
