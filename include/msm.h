/*
 * msm.h - C ABI of libmsm, neighbourhood-graph construction by the multiple
 * sorting method (MSM) on AMD Instinct MI355X (gfx950).
 *
 * Method: Uno, Sugiyama and Tsuda, "Efficient Construction of Neighborhood
 * Graphs by the Multiple Sorting Method" (arXiv:0904.3151).
 *
 * The library computes the three steps of the method's data-parallel path:
 *
 *   msm_project          vectors -> ell-bit sign strings       (Section 3.2, eq. (3))
 *   msm_enumerate_pairs  strings -> pairs within Hamming h     (Sections 2.1-2.2, eq. (1))
 *   msm_verify           pairs   -> pairs within distance eps  (Section 4.1, Definition 1.1)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every data pointer is a DEVICE pointer on the context's device, owned by
 *   the caller. The library never frees or keeps caller memory.
 * - Host pointers are marked HOST. They are written before the call returns.
 * - `stream` is a hipStream_t (NULL means the default stream). Work is
 *   enqueued on it. Calls that return a count (`m_out`) synchronise the
 *   stream before returning; msm_project does not synchronise.
 * - Indices are 0-based uint32; n must be below 2^32.
 * - X is FP32, n rows of d values, row i at X + i*ldx (ldx >= d, in floats).
 * - R is FP32, d x ell, row-major: R[t*ell + c]; column c is the random
 *   direction r_c of bit c.
 * - S is uint64, n rows of W = ceil(ell/64) words. Bit c of row i is
 *   (S[i*W + c/64] >> (c%64)) & 1. msm_project writes padding bits (at and
 *   above ell) as 0; msm_enumerate_pairs ignores them.
 * - A pair list is uint32 interleaved (i, j) with i < j: pair p is
 *   pairs[2p], pairs[2p+1]. Its order is unspecified; it is a set.
 * - Every call returns an msm_status; nothing throws across the ABI. On
 *   failure msm_last_error(ctx) describes the cause.
 * - A context may be used by one host thread at a time. Calls on one context
 *   share its scratch memory, so they must be ordered on one stream.
 */
#ifndef MSM_H
#define MSM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MSM_OK = 0,
    MSM_E_INVALID = -1,     /* an argument is out of range or a needed pointer is NULL */
    MSM_E_CAPACITY = -2,    /* the output did not fit; *m_out holds the required count */
    MSM_E_UNSUPPORTED = -3, /* valid but outside what this build implements */
    MSM_E_NOMEM = -4,       /* device scratch allocation failed */
    MSM_E_HIP = -5          /* a HIP runtime call failed */
} msm_status;

typedef enum {
    MSM_EUCLIDEAN = 0, /* Delta(x, y) = ||x - y||_2 */
    MSM_COSINE = 1     /* Delta(x, y) = 1 - x.y / (||x|| ||y||), eq. (2); 1 if either is zero */
} msm_metric;

typedef enum {
    MSM_F32 = 0,      /* FP32 products, FP32 accumulation (msm_project) */
    MSM_BF16 = 1,     /* BF16 products, FP32 accumulation */
    MSM_FP8_E4M3 = 2  /* FP8 e4m3 products of row/column-scaled copies, FP32 accumulation */
} msm_dtype;

typedef struct msm_ctx msm_ctx;

/* Library version as 10000*major + 100*minor + patch. */
int32_t msm_version(void);

/* Create a context on HIP device `device`. The context owns the scratch
 * memory of the calls made through it; it grows on demand and is released
 * by msm_destroy. Calls through one context share that memory: make them
 * from one host thread, on one stream, or wait for the previous call's work
 * before a call on another stream (a call that grows the scratch waits only
 * for its own stream before releasing the old buffer). Returns
 * MSM_E_INVALID if out is NULL, MSM_E_HIP if the device cannot be
 * selected. */
msm_status msm_create(int32_t device, msm_ctx** out);

/* Release a context and its scratch memory. NULL is ignored. The caller
 * must make sure no work using the context is still running. */
void msm_destroy(msm_ctx* ctx);

/* Message for the last failed call on ctx ("" if none). The string is owned
 * by the context and valid until its next call. ctx may be NULL, in which
 * case the message of the last failed msm_create is returned. */
const char* msm_last_error(const msm_ctx* ctx);

/* Random-projection LSH, Section 3.2, eq. (3):
 *   z_ic = sum_t X[i,t] * R[t,c],   bit c of S_i = 1 iff z_ic > 0, else 0.
 * FP32 accumulation on the matrix cores. For ell <= 128 and d <= 256 each
 * FP32 input is split into three BF16 parts (hi, mid, lo) and z sums the six
 * products whose parts are not both small, which carries the products to
 * about FP32 precision; other shapes use FP32 products.
 *   X    DEVICE float[n rows, ldx stride]   input vectors
 *   R    DEVICE float[d * ell]              projection matrix, row-major
 *   S    DEVICE uint64[n * W]               output strings (fully written)
 * Limits: n >= 0, 1 <= d, ldx >= d, 1 <= ell <= 256.
 * Errors: MSM_E_INVALID for a NULL ctx, out-of-range sizes, or NULL X, R, S
 * with n > 0. Asynchronous: returns once the work is enqueued. */
msm_status msm_project(msm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                       const float* R, int32_t ell, uint64_t* S, void* stream);

/* Random-projection LSH with low-precision products (eq. (3)). z = X R is
 * estimated from BF16 copies of X and R, or from FP8 e4m3 copies scaled per
 * row of X and per column of R (each to a largest magnitude of 240), with
 * FP32 accumulation on the matrix cores; X is read as FP32 and converted on
 * the fly. An entry whose estimate satisfies |z| < tau * ||x_i|| is
 * recomputed as an FP32 dot product and takes its sign from that; every
 * other entry takes the sign of the estimate. Outside the margin a sign can
 * still differ from the exact one when the product error exceeds |z|.
 *   X, R, S          as for msm_project
 *   dtype            MSM_BF16 or MSM_FP8_E4M3
 *   tau              margin relative to ||x_i|| (for example 2^-8), >= 0
 *   n_recomputed     HOST, optional: number of entries recomputed in FP32;
 *                    when non-NULL the call synchronises `stream`
 * Errors: as msm_project, plus MSM_E_INVALID for another dtype or a negative
 * or non-finite tau. */
msm_status msm_project_lowp(msm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                            const float* R, int32_t ell, int32_t dtype, float tau, uint64_t* S,
                            int64_t* n_recomputed, void* stream);

/* All pairs within Hamming distance h, Sections 2.1-2.2 and eq. (1):
 *   { (i, j) : i < j, popcount(S_i xor S_j) <= h }
 * found by blockwise masking: the ell bits are split into k blocks of
 * nearly equal length (the first ell mod k blocks get one extra bit), and
 * for each of the C(k, h) sets B of masked blocks the strings are grouped by
 * their unmasked part; pairs inside a group are tested and each pair is
 * written under exactly one B, so the output has no duplicates. When it
 * takes fewer passes the strings are instead grouped on sets of j blocks
 * shared by several B (see msm_enumerate_groupings); the output is the
 * same set.
 *   S      DEVICE uint64[n * W]       input strings
 *   pairs  DEVICE uint32[2 * cap]     output pairs; may be NULL when cap == 0
 *   m_out  HOST   int64               number of pairs (always written on OK
 *                                     and on MSM_E_CAPACITY)
 * The result set does not depend on k; k only changes the work.
 * Limits: n < 2^32, 1 <= ell <= 256, 0 <= h < k <= min(ell, 64),
 * C(k, h) <= 65536.
 * Errors: MSM_E_INVALID (sizes, NULL pointers), MSM_E_UNSUPPORTED (k > 64,
 * too many combinations, or a group of more than about 16.7M strings that
 * agree under some grouping: its pairs are not tested), MSM_E_CAPACITY when
 * the count exceeds cap:
 * *m_out then holds the required count and the contents of pairs are
 * undefined. pairs == NULL with cap == 0 is a count-only call. Synchronises
 * `stream` before returning. */
msm_status msm_enumerate_pairs(msm_ctx* ctx, const uint64_t* S, int64_t n, int32_t ell,
                               int32_t k, int32_t h, uint32_t* pairs, int64_t cap,
                               int64_t* m_out, void* stream);

/* msm_enumerate_pairs for callers that cannot allocate memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, same pair set, same errors, but the work memory is a fixed
 * 64 MiB device buffer that the library holds per device (a static array,
 * kept until the process ends) instead of the context's growing scratch,
 * and the host tables go up through a pinned buffer the context allocated
 * when it was created. The call makes no device or host allocation.
 * Additional errors: MSM_E_UNSUPPORTED when the work memory for n strings
 * does not fit in the buffer (n above about 6 million; the message gives
 * the bytes needed) or the tables of the C(k, h) combinations exceed 2 MiB
 * (C(k, h) above about 10000); nothing is computed then and *m_out is 0.
 * All calls on one device share that device's buffer, and a call leaves its
 * contents behind (the next call clears what it needs): calls that overlap
 * on one device, from several host threads, streams or contexts, race and
 * give undefined results. Synchronises `stream` before returning. */
msm_status msm_enumerate_pairs_noalloc(msm_ctx* ctx, const uint64_t* S, int64_t n, int32_t ell,
                                       int32_t k, int32_t h, uint32_t* pairs, int64_t cap,
                                       int64_t* m_out, void* stream);

/* How msm_enumerate_pairs may group n strings of ell bits for (k, h): the
 * number of groupings (partition passes) it makes and, when it groups on
 * j < k - h blocks (hierarchically: one grouping on a set A of j blocks
 * serves every combination of masked blocks whose unmasked blocks contain
 * A; taken when j * floor(ell / k) >= log2(n) + 8 and it needs fewer
 * groupings than C(k, h)), that j; else *jblocks = 0 and *groupings =
 * C(k, h). Host-only, needs no context or device.
 *   groupings, jblocks  HOST int32
 * Errors: MSM_E_INVALID for NULL outputs or arguments outside the limits of
 * msm_enumerate_pairs. */
msm_status msm_enumerate_groupings(int64_t n, int32_t ell, int32_t k, int32_t h, int32_t* groupings,
                                   int32_t* jblocks);

/* The groupings the last msm_enumerate_pairs or msm_enumerate_replicates
 * call on ctx made, and its j (0 when it grouped per combination). When a
 * hierarchical grouping is possible the call first counts a few groupings
 * of each kind and keeps the hierarchical one only if its groupings times
 * their sum of squared bucket sizes is the smaller, so this can differ from
 * msm_enumerate_groupings. Zero before the first call.
 *   groupings, jblocks  HOST int32
 * Errors: MSM_E_INVALID for NULL arguments. */
msm_status msm_enumerate_last_plan(const msm_ctx* ctx, int32_t* groupings, int32_t* jblocks);

/* Union of the Hamming pairs of Q independent string pools, Section 4.1,
 * eq. (5): E = E_1 u ... u E_Q with E_q = {(i, j) : i < j,
 * popcount(S^q_i xor S^q_j) <= h}. Pool q is enumerated as in
 * msm_enumerate_pairs, and, following the first acceleration trick of the
 * paper's appendix, a pair found in pool q is written only if its Hamming
 * distance exceeds h in every earlier pool g < q, so every pair of E is
 * written exactly once.
 *   S      DEVICE uint64[Q * n * W]   pools, replicate-major: string i of
 *                                     pool q at S + (q * n + i) * W
 *   Q      number of pools, 1 <= Q <= 4096
 * Other arguments, limits and errors as for msm_enumerate_pairs (Q = 1 is
 * the same call). Synchronises `stream`. */
msm_status msm_enumerate_replicates(msm_ctx* ctx, const uint64_t* S, int64_t n, int32_t ell,
                                    int32_t Q, int32_t k, int32_t h, uint32_t* pairs, int64_t cap,
                                    int64_t* m_out, void* stream);

/* Verification step of Section 4.1: keep the pairs of a list whose true
 * distance is at most eps (Definition 1.1). FP32 arithmetic: Euclidean
 * compares sum (x_t - y_t)^2 with eps^2; cosine compares eq. (2) with eps.
 * Euclidean lists of at least n pairs are first decided on FP16 copies of
 * the rows with a proven error bound: a pair outside the bound's band is
 * kept or dropped exactly as the real-valued distance decides, and only the
 * pairs inside it are evaluated in FP32 as above. The copies take
 * n * (2 * ceil8(d) + 4) bytes of the context's device scratch; when that
 * memory cannot be had, the FP32 kernel verifies the whole list.
 *   X      DEVICE float[n rows, ldx stride]
 *   pairs  DEVICE uint32[2 * m]         candidate pairs (i, j), both < n
 *   out    DEVICE uint32[2 * cap]       kept pairs (may alias nothing else)
 *   m_out  HOST   int64                 number kept
 * Errors: MSM_E_INVALID (sizes, NULL pointers, unknown metric, eps < 0 or
 * not finite, a pair index >= n: such pairs are skipped and reported),
 * MSM_E_CAPACITY as for msm_enumerate_pairs. Pair buffers must be 8-byte
 * aligned. Synchronises `stream`. */
msm_status msm_verify(msm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                      const uint32_t* pairs, int64_t m, int32_t metric, float eps,
                      uint32_t* out, int64_t cap, int64_t* m_out, void* stream);

/* Exhaustive epsilon-neighbour enumeration, Definition 1.1: every (i, j),
 * i < j, with Delta(x_i, x_j) <= eps. This is the exhaustive reference for the
 * missing-edge ratio of Section 4.2 (|F2| / |E*| on a subsample), not part
 * of the MSM path. FP32 Gram-matrix screening on the matrix cores with a
 * rounding band, then an FP64 evaluation of each screened pair from the
 * FP32 inputs: the result is the FP64 definition. Euclidean compares the
 * squared distance with eps^2; cosine uses eq. (2), 1 for a zero vector.
 *   X      DEVICE float[n rows, ldx stride]
 *   out    DEVICE uint32[2 * cap]     pairs (i, j), i < j, 8-byte aligned
 *   m_out  HOST   int64               number of pairs
 * Limits: n <= about 3e6 (the upper triangle of 64 x 64 tiles must stay
 * below 2^31 workgroups). Errors as for msm_verify; MSM_E_CAPACITY when the
 * count exceeds cap. Synchronises `stream`. */
msm_status msm_bruteforce_eps(msm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                              int32_t metric, float eps, uint32_t* out, int64_t cap,
                              int64_t* m_out, void* stream);

/* Learned projection: a two-layer network in place of the random
 * projection, the non-random hashing named in Section 6. For a row x:
 *   a1 = x W1 + b1,  g = GELU(a1) = a1 (1 + erf(a1 / sqrt 2)) / 2,
 *   a2 = g W2 + b2,  u = tanh(a2),  bit c of S_i = 1 iff a2_c > 0.
 * Products use BF16 copies of the operands with FP32 accumulation on the
 * matrix cores; biases, activations and the loss are FP32.
 *   params DEVICE float[d*hid + hid + hid*ell + ell], packed row-major as
 *          [W1 (d x hid) | b1 (hid) | W2 (hid x ell) | b2 (ell)]
 * The strings can be used wherever msm_project's are.
 *   X, S   as for msm_project (S fully written, padding bits 0)
 * Limits: n >= 0, 1 <= d, ldx >= d, 1 <= hid <= 65536, 1 <= ell <= 256.
 * Errors: MSM_E_INVALID for sizes or NULL pointers with n > 0; MSM_E_NOMEM
 * when scratch for the BF16 weights cannot be allocated. Asynchronous. */
msm_status msm_project_mlp(msm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                           const float* params, int32_t hid, int32_t ell, uint64_t* S, void* stream);

/* Loss and gradient of the learned projection over B labelled pairs. With
 * D = (ell - u_i . u_j) / 2 (the Hamming distance of the sign strings when
 * u is +-1), the loss is the mean over the pairs of
 *   y relu(D - h/2)^2 + (1 - y) relu(3h - D)^2
 *     + lam (sum_c (1 - |u_ic|)^2 + sum_c (1 - |u_jc|)^2),
 * pulling epsilon-pairs (y = 1) inside the MSM threshold h and pushing other
 * pairs beyond 3h, with a term that drives u towards +-1.
 *   pairs  DEVICE uint32[2 * B]     (i, j) row indices into X, each < n
 *   labels DEVICE float[B]          y in [0, 1]
 *   grad   DEVICE float[#params]    d loss / d params, packed like params
 *   loss_out HOST float, optional   the loss
 * Errors: MSM_E_INVALID for sizes, NULL pointers, B outside [1, 2^24],
 * negative or non-finite h or lam, or a pair index >= n (nothing is
 * computed then). Synchronises `stream`. */
msm_status msm_mlp_loss_grad(msm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                             const float* params, int32_t hid, int32_t ell, const uint32_t* pairs,
                             const float* labels, int32_t B, float h, float lam, float* grad,
                             float* loss_out, void* stream);

/* One Adam step (Kingma and Ba, 2015) on `count` FP32 parameters:
 *   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
 *   p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * params, m, v are updated in place (DEVICE, count floats each); step >= 1
 * counts from 1. Errors: MSM_E_INVALID for NULL pointers with count > 0,
 * step < 1, lr < 0, b1 or b2 outside [0, 1), eps <= 0. Asynchronous. */
msm_status msm_mlp_adam(msm_ctx* ctx, float* params, const float* grad, float* m, float* v,
                        int64_t count, int64_t step, float lr, float beta1, float beta2, float eps,
                        void* stream);

/* `steps` training steps of the learned projection, each msm_mlp_loss_grad
 * on the next `batch` pairs of the list followed by msm_mlp_adam (beta1 0.9,
 * beta2 0.999, eps 1e-8) with Adam step numbers first_step, first_step + 1,
 * ... A batch that would run past the end of the list starts again at pair
 * 0, so the caller shuffles the list. Batches hold min(batch, npairs) pairs.
 *   params, m, v DEVICE float[#params], updated in place
 *   pairs, labels as for msm_mlp_loss_grad, npairs entries
 *   losses HOST float[steps], optional: the loss of every step
 * Errors as for msm_mlp_loss_grad (all pair indices are checked once before
 * the first step). Synchronises `stream` when losses is non-NULL or a pair
 * index is checked (always). */
msm_status msm_mlp_train(msm_ctx* ctx, const float* X, int64_t n, int32_t d, int64_t ldx,
                         float* params, float* m, float* v, int32_t hid, int32_t ell,
                         const uint32_t* pairs, const float* labels, int64_t npairs, int32_t batch,
                         int64_t steps, int64_t first_step, float lr, float h, float lam,
                         float* losses, void* stream);

/* Batched form: many independent instances of the whole path, each its own
 * problem of Definition 1.1's Hamming stage: strings by eq. (3) from its
 * own X and R, then all its pairs within Hamming distance h (Sections
 * 2.1-2.2), written with indices local to the instance. All instances share
 * ell, k and h. */
typedef struct {
    const float* X;  /* DEVICE float[n rows, ldx stride] */
    const float* R;  /* DEVICE float[d * ell], row-major */
    uint64_t* S;     /* DEVICE uint64[n * W], written by every run */
    uint32_t* pairs; /* DEVICE uint32[2 * cap], 8-byte aligned; NULL with cap == 0 */
    int64_t n;       /* points, >= 0 */
    int64_t ldx;     /* >= d */
    int64_t cap;     /* pairs that fit */
    int32_t d;       /* >= 1 when n > 0 */
    int32_t reserved;
} msm_instance;

/* A tuning parameter set of the batched enumeration for the instances with
 * n_min <= n < n_max, and the measured time of the whole batch's
 * enumeration with it. */
typedef struct {
    int32_t bucket_target;     /* points per partition bucket aimed at */
    int32_t digit_bits;        /* width of the radix digit counted inside a bucket */
    int32_t buckets_per_group; /* buckets taken by one workgroup */
    float ms;                  /* enumeration time of the whole batch, -1 if untimed */
    int64_t n_min, n_max;      /* the size class it applies to */
} msm_batch_config;

typedef struct msm_batch msm_batch;

/* Plan a batch: checks the instances, allocates the plan's device memory
 * (about 8 * N * min(C(k,h), groups) bytes of partition plus the
 * concatenated strings, N = total points) and uploads its tables. With
 * autotune != 0 the candidate configurations (bucket target 256, 512 or
 * 1024 points, digit 8, 10 or 12 bits, 2 or 8 buckets per workgroup) are
 * timed on this batch for each class of instance size (n below 8192, below
 * 65536, above) in turn, the other classes at their best so far, and each
 * class keeps its fastest; this runs the batch, so S and pairs of the
 * instances are written. The descriptors are copied: the
 * buffers they point to must stay valid for the plan's life.
 *   inst   HOST msm_instance[count], 1 <= count <= 65535
 *   out    HOST, receives the plan
 * Limits as msm_enumerate_pairs; total points below 2^32.
 * Errors: MSM_E_INVALID (arguments), MSM_E_UNSUPPORTED (k, C(k,h)),
 * MSM_E_NOMEM, MSM_E_HIP. Synchronises `stream`. */
msm_status msm_batch_create(msm_ctx* ctx, const msm_instance* inst, int32_t count, int32_t ell,
                            int32_t k, int32_t h, int32_t autotune, msm_batch** out, void* stream);

/* Enqueue one run of the batch on `stream`: projection of every instance
 * (the arithmetic of msm_project: for ell <= 128 and d <= 256 the three-part
 * BF16 split with six products, else FP32 products), then its Hamming
 * pairs. Only kernel launches are enqueued (counters are
 * cleared by kernels, nothing is copied, nothing waits on the host), so the
 * call may be captured into a HIP graph.
 *   m_dev  DEVICE int64[count]: pairs of each instance. When m_dev[i] >
 *          cap_i the instance's list holds an unspecified cap_i of them.
 * Runs of one plan must not overlap: they share its device memory.
 * Errors: MSM_E_INVALID (NULL plan, NULL or unaligned m_dev). */
msm_status msm_batch_run(msm_batch* b, int64_t* m_dev, void* stream);

/* msm_batch_run captured once into a HIP graph (on the plan's own stream;
 * again whenever m_dev changes) and launched on `stream` as one graph. A
 * re-capture for a new m_dev first waits for the previous graph launch to
 * finish (an event recorded after each launch), whichever stream it ran on. */
msm_status msm_batch_launch_graph(msm_batch* b, int64_t* m_dev, void* stream);

/* The configuration in use for each size class that holds instances (up
 * to chosen_cap HOST records, smallest class first; *n_chosen gets their
 * number) and, when the plan was tuned, every candidate tried with its time
 * (up to cap HOST records; *n_tried gets their number). Any of the
 * outputs may be NULL with its cap 0. Errors: MSM_E_INVALID. */
msm_status msm_batch_tuning(const msm_batch* b, msm_batch_config* chosen, int32_t chosen_cap, int32_t* n_chosen,
                            msm_batch_config* tried, int32_t cap, int32_t* n_tried);

/* Release a plan and its device memory; no run of it may be in flight.
 * NULL is ignored. */
void msm_batch_destroy(msm_batch* b);

/* Per-kernel timing. While enabled, every kernel launch of the context is
 * bracketed by two HIP events on its stream (a few microseconds of overhead
 * per launch). Timings accumulate per kernel name until msm_profile_reset. */
typedef struct {
    char name[48];     /* kernel name, NUL-terminated */
    int64_t launches;  /* launches timed */
    double total_ms;   /* summed event-to-event time */
} msm_kernel_time;

/* Turn timing on (enable != 0) or off. Errors: MSM_E_INVALID for NULL ctx. */
msm_status msm_profile_enable(msm_ctx* ctx, int32_t enable);

/* Time only the kernel named `name` (as in msm_kernel_time::name) while
 * timing is on, so that the other launches carry no events; NULL or "" times
 * every kernel again. The name is copied. Errors: MSM_E_INVALID for NULL ctx
 * or a name of 48 characters or more. */
msm_status msm_profile_only(msm_ctx* ctx, const char* name);

/* Wait for the recorded events and clear the totals. */
msm_status msm_profile_reset(msm_ctx* ctx);

/* Wait for the recorded events, then write up to cap HOST records to out.
 * Returns the number of kernels with records (may exceed cap), or -1 on
 * error (NULL ctx, cap < 0, out NULL with cap > 0, a HIP failure). */
int32_t msm_profile_read(msm_ctx* ctx, msm_kernel_time* out, int32_t cap);

#ifdef __cplusplus
}
#endif

#endif /* MSM_H */
