/*
 * CPU oracle for neighbourhood-graph construction by the multiple sorting
 * method (MSM) with a cosine-LSH front end.
 *
 * TEST INFRASTRUCTURE ONLY. This is the plain, slow, obviously correct
 * reference that the HIP library is checked against. Only the test suite,
 * the package smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header, table or helper with the GPU library, and the
 * product path never calls it.
 *
 * Data conventions (an interface both sides implement on their own):
 *   X      float32, n rows of d values; row i starts at X + i*ldx.
 *   R      float32, d x ell row-major; R[t*ell + c] is entry (t, c), so
 *          column c is the random direction r_c of bit c.
 *   S      uint64, n rows of W = ceil(ell/64) words; bit c of row i is
 *          (S[i*W + c/64] >> (c%64)) & 1. Bits at and above ell are 0.
 *   pairs  uint32, interleaved (i, j) with i < j.
 * All floating point is FP64. Entry points return a count; when the count
 * exceeds `cap`, only the first `cap` results are written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXW 4

static int popcount64(uint64_t v) { return __builtin_popcountll(v); }

static int words_for(int32_t ell) { return (ell + 63) / 64; }

/* Hamming distance between two packed strings (the number of disagreeing
 * characters, Section 2.1). */
static int hamming(const uint64_t* a, const uint64_t* b, int W)
{
    int t = 0;
    for (int w = 0; w < W; ++w) t += popcount64(a[w] ^ b[w]);
    return t;
}

/* ------------------------------------------------------------------------ */
/* Projection, Section 3.2, eq. (3): s_ic = '1' iff r_c^T x_i > 0, else '0'.
 * z_ic is accumulated in FP64 from the FP32 inputs. When `rows` is non-NULL
 * only rows[0..nrows) are projected and output row r belongs to rows[r];
 * otherwise all n rows are. Z (nrows x ell) and xnorm (nrows) are optional
 * outputs: the FP64 value of z_ic and of the Euclidean norm of x_i. */
void oracle_project(const float* X, int64_t n, int32_t d, int64_t ldx,
                    const float* R, int32_t ell,
                    const int64_t* rows, int64_t nrows,
                    uint64_t* S, double* Z, double* xnorm)
{
    const int W = words_for(ell);
    const int64_t count = rows ? nrows : n;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < count; ++r) {
        const int64_t i = rows ? rows[r] : r;
        const float* x = X + i * ldx;
        uint64_t* s = S + r * W;
        for (int w = 0; w < W; ++w) s[w] = 0;
        for (int32_t c = 0; c < ell; ++c) {
            double z = 0.0;
            for (int32_t t = 0; t < d; ++t)
                z += (double)x[t] * (double)R[(int64_t)t * ell + c];
            if (Z) Z[r * ell + c] = z;
            if (z > 0.0) s[c >> 6] |= (uint64_t)1 << (c & 63);
        }
        if (xnorm) {
            double q = 0.0;
            for (int32_t t = 0; t < d; ++t) q += (double)x[t] * (double)x[t];
            xnorm[r] = sqrt(q);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* The Hamming neighbour problem of Section 2.1 by its definition (eq. (1)):
 * every pair (i, j), i < j, with HamDist(s_i, s_j) <= h, by exhaustive
 * comparison. Pairs come out in lexicographic order. */
int64_t oracle_hamming_pairs(const uint64_t* S, int64_t n, int32_t W, int32_t h,
                             uint32_t* out, int64_t cap)
{
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j)
            if (hamming(S + i * W, S + j * W, W) <= h) {
                if (m < cap) { out[2 * m] = (uint32_t)i; out[2 * m + 1] = (uint32_t)j; }
                ++m;
            }
    return m;
}

/* The same definition restricted to listed rows: for each rows[r], every
 * j != rows[r] with HamDist <= h, written as (min, max) in the order of
 * rows then j. Used to check full-size results on a sample of rows. */
int64_t oracle_hamming_partners(const uint64_t* S, int64_t n, int32_t W, int32_t h,
                                const int64_t* rows, int64_t nrows,
                                uint32_t* out, int64_t cap)
{
    int64_t* cnt = (int64_t*)calloc((size_t)nrows + 1, sizeof(int64_t));
    if (!cnt) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t i = rows[r];
        int64_t c = 0;
        for (int64_t j = 0; j < n; ++j)
            if (j != i && hamming(S + i * W, S + j * W, W) <= h) ++c;
        cnt[r + 1] = c;
    }
    for (int64_t r = 0; r < nrows; ++r) cnt[r + 1] += cnt[r];
    const int64_t total = cnt[nrows];
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t i = rows[r];
        int64_t m = cnt[r];
        for (int64_t j = 0; j < n; ++j)
            if (j != i && hamming(S + i * W, S + j * W, W) <= h) {
                if (m < cap) {
                    out[2 * m] = (uint32_t)(i < j ? i : j);
                    out[2 * m + 1] = (uint32_t)(i < j ? j : i);
                }
                ++m;
            }
    }
    free(cnt);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Multiple sorting method with blockwise masking (Sections 2.1-2.2).
 *
 * The ell characters are divided into k blocks of approximately equal
 * length: the first (ell mod k) blocks hold ceil(ell/k) characters and the
 * rest floor(ell/k), in order. For every set B of h distinct block indices
 * (taken in lexicographic order) the B-masked strings s_i^B are sorted, the
 * sorted list is cut into equivalence classes of equal masked strings, and
 * every pair inside a class is kept if its true Hamming distance is at most
 * h. The same pair can fall into one class under several B; it is written
 * once, under the first B (in the enumeration order) whose masked strings
 * agree, found by an explicit check of all earlier B.
 *
 * A string with its B-blocks removed equals another one with the same blocks
 * removed exactly when the two agree on every character outside those
 * blocks, so the masked string is held here as the full string with the
 * B-block characters cleared.
 *
 * stats (optional, 4 entries): [0] number of sorts performed, [1] candidate
 * pairs examined (pairs inside classes), [2] candidates rejected by the
 * Hamming filter, [3] candidates dropped as already found under an earlier B.
 */
typedef struct {
    uint64_t w[OR_MAXW];
    uint32_t idx;
} or_key;

static int or_key_cmp(const void* pa, const void* pb)
{
    const or_key* a = (const or_key*)pa;
    const or_key* b = (const or_key*)pb;
    for (int w = 0; w < OR_MAXW; ++w) {
        if (a->w[w] < b->w[w]) return -1;
        if (a->w[w] > b->w[w]) return 1;
    }
    return (a->idx > b->idx) - (a->idx < b->idx);
}

typedef struct {
    uint32_t* v;
    int64_t len, cap;
} or_vec;

static int or_push(or_vec* vec, uint32_t i, uint32_t j)
{
    if (vec->len == vec->cap) {
        int64_t nc = vec->cap ? 2 * vec->cap : 1024;
        uint32_t* nv = (uint32_t*)realloc(vec->v, (size_t)nc * 2 * sizeof(uint32_t));
        if (!nv) return -1;
        vec->v = nv;
        vec->cap = nc;
    }
    vec->v[2 * vec->len] = i;
    vec->v[2 * vec->len + 1] = j;
    vec->len++;
    return 0;
}

static int64_t binom(int a, int b)
{
    if (b < 0 || b > a) return 0;
    int64_t r = 1;
    for (int t = 1; t <= b; ++t) r = r * (a - b + t) / t;
    return r;
}

int64_t oracle_msm(const uint64_t* S, int64_t n, int32_t ell, int32_t k, int32_t h,
                   uint32_t* out, int64_t cap, int64_t* stats)
{
    const int W = words_for(ell);
    if (W > OR_MAXW || k < 1 || k > ell || h < 0 || h >= k) return -1;

    /* Block b covers characters [start[b], start[b] + len[b]). */
    int start[256], len[256];
    {
        int pos = 0;
        for (int b = 0; b < k; ++b) {
            len[b] = ell / k + (b < ell % k ? 1 : 0);
            start[b] = pos;
            pos += len[b];
        }
    }

    /* All h-subsets of {0..k-1} in lexicographic order, each turned into
     * the mask of characters that survive the masking. */
    const int64_t ncomb = binom(k, h);
    uint64_t* keep = (uint64_t*)calloc((size_t)(ncomb > 0 ? ncomb : 1) * OR_MAXW, sizeof(uint64_t));
    if (!keep) return -1;
    {
        int sel[256];
        for (int t = 0; t < h; ++t) sel[t] = t;
        for (int64_t q = 0; q < ncomb; ++q) {
            uint64_t* kq = keep + q * OR_MAXW;
            for (int c = 0; c < ell; ++c) kq[c >> 6] |= (uint64_t)1 << (c & 63);
            for (int t = 0; t < h; ++t)
                for (int c = start[sel[t]]; c < start[sel[t]] + len[sel[t]]; ++c)
                    kq[c >> 6] &= ~((uint64_t)1 << (c & 63));
            /* next subset in lexicographic order */
            int t = h - 1;
            while (t >= 0 && sel[t] == k - h + t) --t;
            if (t < 0) break;
            sel[t]++;
            for (int u = t + 1; u < h; ++u) sel[u] = sel[u - 1] + 1;
        }
    }

    or_vec* found = (or_vec*)calloc((size_t)(ncomb > 0 ? ncomb : 1), sizeof(or_vec));
    int64_t st_cand = 0, st_rej = 0, st_dup = 0;
    int failed = 0;

#pragma omp parallel reduction(+ : st_cand, st_rej, st_dup)
    {
        or_key* keys = (or_key*)malloc((size_t)(n > 0 ? n : 1) * sizeof(or_key));
        if (!keys) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < ncomb; ++q) {
            if (!keys) continue;
            const uint64_t* kq = keep + q * OR_MAXW;
            /* masked strings s_i^B, then sort */
            for (int64_t i = 0; i < n; ++i) {
                for (int w = 0; w < OR_MAXW; ++w)
                    keys[i].w[w] = w < W ? (S[i * W + w] & kq[w]) : 0;
                keys[i].idx = (uint32_t)i;
            }
            qsort(keys, (size_t)n, sizeof(or_key), or_key_cmp);
            /* equivalence classes of the sorted list */
            int64_t a = 0;
            while (a < n) {
                int64_t b = a + 1;
                while (b < n && memcmp(keys[b].w, keys[a].w, sizeof(keys[a].w)) == 0) ++b;
                for (int64_t u = a; u < b; ++u)
                    for (int64_t v = u + 1; v < b; ++v) {
                        const uint32_t i = keys[u].idx, j = keys[v].idx; /* i < j */
                        const uint64_t* si = S + (int64_t)i * W;
                        const uint64_t* sj = S + (int64_t)j * W;
                        ++st_cand;
                        if (hamming(si, sj, W) > h) { ++st_rej; continue; }
                        int earlier = 0;
                        for (int64_t p = 0; p < q && !earlier; ++p) {
                            const uint64_t* kp = keep + p * OR_MAXW;
                            int same = 1;
                            for (int w = 0; w < W; ++w)
                                if ((si[w] ^ sj[w]) & kp[w]) { same = 0; break; }
                            earlier = same;
                        }
                        if (earlier) { ++st_dup; continue; }
                        if (or_push(&found[q], i, j)) {
#pragma omp atomic write
                            failed = 1;
                        }
                    }
                a = b;
            }
        }
        free(keys);
    }

    int64_t m = 0;
    for (int64_t q = 0; q < ncomb; ++q) {
        for (int64_t t = 0; t < found[q].len; ++t) {
            if (m < cap) {
                out[2 * m] = found[q].v[2 * t];
                out[2 * m + 1] = found[q].v[2 * t + 1];
            }
            ++m;
        }
        free(found[q].v);
    }
    free(found);
    free(keep);
    if (stats) {
        stats[0] = ncomb;
        stats[1] = st_cand;
        stats[2] = st_rej;
        stats[3] = st_dup;
    }
    return failed ? -1 : m;
}

/* ------------------------------------------------------------------------ */
/* Distances of Definition 1.1. metric 0: Euclidean distance. metric 1: the
 * cosine distance of eq. (2), 1 - x.y / (|x||y|); a pair involving a zero
 * vector is given distance 1 (eq. (2) is undefined there). */
static double distance(const float* x, const float* y, int32_t d, int32_t metric)
{
    if (metric == 0) {
        double q = 0.0;
        for (int32_t t = 0; t < d; ++t) {
            const double e = (double)x[t] - (double)y[t];
            q += e * e;
        }
        return sqrt(q);
    }
    double xy = 0.0, xx = 0.0, yy = 0.0;
    for (int32_t t = 0; t < d; ++t) {
        xy += (double)x[t] * (double)y[t];
        xx += (double)x[t] * (double)x[t];
        yy += (double)y[t] * (double)y[t];
    }
    if (xx == 0.0 || yy == 0.0) return 1.0;
    return 1.0 - xy / (sqrt(xx) * sqrt(yy));
}

/* Verification step of Section 4.1: keep the listed pairs whose distance is
 * at most eps. `dist` (optional, m entries) receives every pair's distance.
 * Output order follows the input order. */
int64_t oracle_verify(const float* X, int64_t n, int32_t d, int64_t ldx,
                      const uint32_t* pairs, int64_t m, int32_t metric, double eps,
                      uint32_t* out, int64_t cap, double* dist)
{
    (void)n;
    int64_t kept = 0;
    for (int64_t p = 0; p < m; ++p) {
        const uint32_t i = pairs[2 * p], j = pairs[2 * p + 1];
        const double D = distance(X + (int64_t)i * ldx, X + (int64_t)j * ldx, d, metric);
        if (dist) dist[p] = D;
        if (D <= eps) {
            if (kept < cap) { out[2 * kept] = i; out[2 * kept + 1] = j; }
            ++kept;
        }
    }
    return kept;
}

/* Definition 1.1 by exhaustive comparison: every (i, j), i < j, with
 * distance <= eps, in lexicographic order. */
int64_t oracle_eps_pairs(const float* X, int64_t n, int32_t d, int64_t ldx,
                         int32_t metric, double eps, uint32_t* out, int64_t cap)
{
    int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cnt) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int64_t j = i + 1; j < n; ++j)
            if (distance(X + i * ldx, X + j * ldx, d, metric) <= eps) ++c;
        cnt[i + 1] = c;
    }
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    const int64_t total = cnt[n];
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        int64_t m = cnt[i];
        for (int64_t j = i + 1; j < n; ++j)
            if (distance(X + i * ldx, X + j * ldx, d, metric) <= eps) {
                if (m < cap) { out[2 * m] = (uint32_t)i; out[2 * m + 1] = (uint32_t)j; }
                ++m;
            }
    }
    free(cnt);
    return total;
}
