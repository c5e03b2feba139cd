/*
 * lrbg.h -- batched low-rank GEMM on AMD Instinct MI355X (gfx950), C ABI.
 *
 * The products are those of a low-rank matrix multiplication (Deshmukh,
 * Yokota, Bosilca, arXiv 2311.07602): a low-rank block is a tuple
 * (U, S, V) with A ~ U S V^T (Sec. 2, dense-to-low-rank equation), and the
 * low-rank product of Alg. 1 starts with the rank-sized inner product of two
 * skinny bases; the batched form takes per-instance arrays of operands
 * (Alg. 2, Alg. 3).  Three product kinds are exposed:
 *
 *   LRBG_OP_DENSE_TS  C = A * U          A m x k, U k x n, C m x n
 *                     (dense block times a tall-skinny basis: m = k = b,
 *                      n = r; the skinny products of Sec. 3 and the BLR
 *                      matrix times multiple right-hand sides of Sec. 7)
 *   LRBG_OP_INNER     T = V1^T * U2      V1 k x m, U2 k x n, T m x n
 *                     (Alg. 1 step 1, C_temp = A_{V^T} B_U; the loop-4
 *                      accumulation C_MN of Alg. 2; k = b, m, n = ranks)
 *   LRBG_OP_RECOMP    W = U1 * (S * V2^T) U1 m x k, S k x k, V2 n x k, W m x n
 *                     (rebuild a block from the rank x rank core of a
 *                      low-rank product, the small-core-times-skinny role of
 *                      Alg. 1 steps 2-3; k = r, m = n = b)
 *   LRBG_OP_LRMULT    G = X_A * (V_A^T * U_B) * X_B
 *                     V_A k x m (a), U_B k x n (b), X_A m x m (s),
 *                     X_B n x n (e), G m x n (c): the paper's low-rank
 *                     product of two blocks (Alg. 1: C_temp = A_{V^T} B_U,
 *                     E_temp = A_X C_temp, G_XY = E_temp B_X), evaluated in
 *                     that order with the rank-sized intermediates kept on
 *                     chip (the fusion of Alg. 2); k = b, m = rank_A,
 *                     n = rank_B; FP64; m, n <= 128.
 *
 * Conventions for every entry point:
 *   - All matrices are column-major: element (i, j) of X is at
 *     X[i + j * ldX], with ldX >= max(1, rows).  V matrices are stored
 *     b x r, so V^T is implied by the operation, never materialised.
 *   - The output is overwritten (beta = 0): Alg. 2 accumulates G with "+="
 *     but G is defined as the result of the product (Alg. 1).  k = 0 yields
 *     a zero-filled output; m = 0 or n = 0 makes an instance a no-op.
 *   - Precisions: LRBG_FP64 takes and returns IEEE binary64.  LRBG_BF16X3
 *     (DENSE_TS and INNER only) takes FP32 operands (A/U or V1/U2 are
 *     float *), splits each value into three bfloat16 terms, multiplies the
 *     six term pairs of order <= 2 on the bf16 matrix cores with FP32
 *     accumulation and returns the output in FP64 (double *).  RECOMP is
 *     FP64 only (LRBG_EUNSUPPORTED otherwise).
 *   - Limits: rank-type dimensions (DENSE_TS n; INNER m, n; RECOMP k;
 *     LRMULT m, n) at most 128, except the ranks and kmax of
 *     lr_batched_lrmult_round (at most 64, the largest core its batched SVD
 *     takes); block-type dimensions at most 65536; violating either is
 *     LRBG_EUNSUPPORTED.
 *   - Pointers named "device" are device (HBM) addresses on the current HIP
 *     device, naturally aligned (8 bytes for FP64, 4 for FP32).  Host arrays
 *     (sizes, leading dimensions, pointer arrays, descriptor arrays) are read
 *     during the call only.  The caller owns every buffer; the library never
 *     frees caller memory.  A buffer may be NULL only if it has no elements.
 *   - Outputs must not overlap each other or any input of the same call,
 *     except through a dependency that a plan or grouped call orders (an
 *     input that is exactly another product's output, see lrbg_grouped).
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL is the null
 *     stream).  Every argument is validated before anything is launched; an
 *     invalid call launches nothing and returns a status code.  Launch
 *     failures return LRBG_EDEVICE; faults inside kernels surface at the
 *     caller's next synchronisation.  lrbg_last_error() gives a thread-local
 *     text for the last failure.
 *   - Results are deterministic: the same inputs and tile configuration give
 *     the same bits, whatever else runs in the same launch.
 */
#ifndef LRBG_H
#define LRBG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lrbg_status {
    LRBG_OK = 0,
    LRBG_EINVAL = 1,        /* malformed argument (null, negative, ld, alias) */
    LRBG_EUNSUPPORTED = 2,  /* outside the supported op / precision / size set */
    LRBG_ENOMEM = 3,        /* a host or device allocation failed */
    LRBG_EDEVICE = 4,       /* a HIP call or kernel launch failed */
    LRBG_EBUDGET = 5        /* a request does not fit the memory budget */
} lrbg_status;

typedef enum lrbg_op {
    LRBG_OP_DENSE_TS = 0,
    LRBG_OP_INNER = 1,
    LRBG_OP_RECOMP = 2,
    LRBG_OP_LRMULT = 3
} lrbg_op;

typedef enum lrbg_prec {
    LRBG_FP64 = 0,
    LRBG_BF16X3 = 1
} lrbg_prec;

/* One product of a grouped call.  a/b/c are device pointers whose element
 * type follows `prec` (see above); s is the RECOMP core (k x k) or the
 * LRMULT X_A (m x m), e the LRMULT X_B (n x n), both FP64 with lds/lde >=
 * their rows; NULL (and ld ignored) for the ops that do not use them.
 * `flags` and `reserved` must be 0. */
typedef struct lrbg_desc {
    int32_t op, prec;
    int32_t m, n, k;
    int32_t lda, ldb, lds, ldc;
    int32_t flags;
    int32_t lde;
    int32_t reserved;
    const void *a;
    const void *b;
    const double *s;
    void *c;
    const double *e;
} lrbg_desc;

/*
 * lr_batched_gemm -- `count` independent products of one kind and precision.
 *   op, prec      : lrbg_op, lrbg_prec.
 *   m, n, k       : host arrays [count] of sizes, meaning per op above.
 *   A, lda        : host arrays [count]: device pointer of the first operand
 *                   (A | V1 | U1) and its leading dimension.
 *   B, ldb        : second operand (U | U2 | V2).
 *   S, lds        : RECOMP core pointers and leading dimensions; NULL for the
 *                   other ops.
 *   C, ldc        : output (C | T | W).
 *   stream        : hipStream_t.
 * The batched problem statement is Alg. 2's per-instance operand arrays.
 */
lrbg_status lr_batched_gemm(int32_t op, int32_t prec, int64_t count,
                            const int32_t *m, const int32_t *n, const int32_t *k,
                            const void *const *A, const int32_t *lda,
                            const void *const *B, const int32_t *ldb,
                            const double *const *S, const int32_t *lds,
                            void *const *C, const int32_t *ldc,
                            void *stream);

/*
 * lr_batched_lrmult -- `count` low-rank products G_i = X_A,i (V_A,i^T U_B,i)
 * X_B,i, the paper's batched Alg. 1 (Alg. 2's operand arrays), FP64.
 *   b             : host array [count]: the shared inner (block) dimension.
 *   ra, rb        : host arrays [count]: ranks of the two operands (<= 128).
 *   AV, ldav      : device V_A, b x ra (the stored A_{V^T} transposed).
 *   BU, ldbu      : device U_B, b x rb.
 *   AX, ldax      : device X_A, ra x ra.
 *   BX, ldbx      : device X_B, rb x rb.
 *   G, ldg        : device G, ra x rb (overwritten).
 *   stream        : hipStream_t.
 * Same as lrbg_grouped over LRBG_OP_LRMULT descriptors (m = ra, n = rb,
 * k = b; a = AV, b = BU, s = AX, e = BX, c = G).
 */
lrbg_status lr_batched_lrmult(int64_t count, const int32_t *b,
                              const int32_t *ra, const int32_t *rb,
                              const double *const *AV, const int32_t *ldav,
                              const double *const *BU, const int32_t *ldbu,
                              const double *const *AX, const int32_t *ldax,
                              const double *const *BX, const int32_t *ldbx,
                              double *const *G, const int32_t *ldg,
                              void *stream);

/*
 * lr_batched_lrmult_round -- `count` products of two low-rank blocks,
 * recompressed: A = A_U A_X A_V^T and B = B_U B_X B_V^T (b x b blocks, ranks
 * ra and rb, orthonormal outer bases A_U, B_V) give A B = A_U G B_V^T with
 * the core G = A_X (A_V^T B_U) B_X of Alg. 1; G = X S Y^T (singular value
 * decomposition) is truncated to the k largest singular values with
 * sigma_i > tol * sigma_1, k <= kmax, and the result is returned as
 * U diag(sigma) V^T with U = A_U X_k, V = B_V Y_k.  FP64.
 *   b, ra, rb     : host arrays [count]; ra, rb <= 64.
 *   AU, AV        : device b x ra (A_U, and A_V: the stored A_{V^T} transposed).
 *   AX            : device ra x ra.
 *   BU, BV        : device b x rb.   BX: device rb x rb.
 *   kmax, tol     : 1 <= kmax <= 64; relative truncation threshold tol >= 0.
 *   U, V          : device b x kmax outputs (columns beyond the kept rank
 *                   are zero).
 *   sigma         : device array [count * kmax], instance t at t * kmax,
 *                   descending, zero beyond the kept rank.
 *   kout          : device array [count]: the rank kept.
 * The singular vectors (columns of U, V) are unique up to sign; U diag(sigma)
 * V^T is unique when sigma_k > sigma_{k+1}.  Scratch for G, X, Y is
 * allocated by the library (pooled, reused once the call's work has run).
 */
lrbg_status lr_batched_lrmult_round(int64_t count, const int32_t *b, const int32_t *ra, const int32_t *rb,
                                    const double *const *AU, const int32_t *ldau,
                                    const double *const *AV, const int32_t *ldav,
                                    const double *const *AX, const int32_t *ldax,
                                    const double *const *BU, const int32_t *ldbu,
                                    const double *const *BX, const int32_t *ldbx,
                                    const double *const *BV, const int32_t *ldbv,
                                    int32_t kmax, double tol,
                                    double *const *U, const int32_t *ldu,
                                    double *const *V, const int32_t *ldv,
                                    double *sigma, int32_t *kout, void *stream);

/*
 * lr_batched_lradd_round -- `count` rounded additions of two low-rank
 * blocks: A = A_U A_X A_V^T and B = B_U B_X B_V^T (b x b blocks of ranks ra
 * and rb; the bases need not be orthonormal and may share columns) give
 *   A + B = [A_U | B_U] diag(A_X, B_X) [A_V | B_V]^T,
 * recompressed by a Householder QR of both stacked bases ([A_U | B_U] =
 * Q_U R_U, [A_V | B_V] = Q_V R_V), the singular value decomposition of the
 * small core M = R_U diag(A_X, B_X) R_V^T = X S Y^T, truncation to the k
 * largest singular values with sigma_i > tol * sigma_1, k <= kmax, and the
 * new bases U = Q_U X_k, V = Q_V Y_k.  The result is A + B ~ U diag(sigma)
 * V^T: the rounded addition whose first step is the low-rank product of
 * Alg. 1 (Sec. 2).  FP64.
 *   b, ra, rb     : host arrays [count]; ra + rb <= 64.
 *   AU, AV        : device b x ra.   AX: device ra x ra.
 *   BU, BV        : device b x rb.   BX: device rb x rb.
 *   kmax, tol     : 1 <= kmax <= 64; relative truncation threshold tol >= 0.
 *   U, V, sigma, kout : as lr_batched_lrmult_round (U, V b x kmax, zero
 *                   beyond the kept rank; sigma [count * kmax] descending;
 *                   kout [count]).
 * Errors as lr_batched_lrmult_round; in addition every output (U, V,
 * sigma, kout) must be disjoint from the others and from every input.
 * Uniqueness as lr_batched_lrmult_round.  Scratch for the reflectors, the
 * factors and the cores is allocated by the library (pooled, reused once
 * the call's work has run).
 */
lrbg_status lr_batched_lradd_round(int64_t count, const int32_t *b, const int32_t *ra, const int32_t *rb,
                                   const double *const *AU, const int32_t *ldau,
                                   const double *const *AV, const int32_t *ldav,
                                   const double *const *AX, const int32_t *ldax,
                                   const double *const *BU, const int32_t *ldbu,
                                   const double *const *BX, const int32_t *ldbx,
                                   const double *const *BV, const int32_t *ldbv,
                                   int32_t kmax, double tol,
                                   double *const *U, const int32_t *ldu,
                                   double *const *V, const int32_t *ldv,
                                   double *sigma, int32_t *kout, void *stream);

/*
 * lr_batched_lrmult_round_noalloc -- lr_batched_lrmult_round for callers
 * that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, same
 * kernels and schedules, and so the same results bit for bit; the cores G,
 * the singular vectors X, Y and the launch tables live in a fixed device
 * array of LRBG_NOALLOC_SCRATCH_BYTES that each GPU holds from the first
 * call on it until the process ends, instead of library allocations.  The
 * call allocates no device or pinned host memory; it uploads its tables
 * with one hipMemcpyAsync from host memory on `stream`.
 *   Limit: a call whose cores, singular vectors (8 bytes per element of
 *   each ra x rb core and of the ra x kmax and rb x kmax vector blocks,
 *   each rounded up to 256 bytes) and tables (about 90 bytes per product
 *   plus 16 per tile) exceed the array returns LRBG_EUNSUPPORTED before
 *   anything is launched; split the batch.
 *   Concurrency: every call on a GPU uses that GPU's one array and leaves
 *   its contents behind; calls on one stream are ordered, but calls that
 *   overlap on one GPU (different streams or threads) race and must not be
 *   issued.  Nothing in the array needs to start at zero (every element a
 *   call reads, it has written first).
 */
#define LRBG_NOALLOC_SCRATCH_BYTES (128ull << 20)
lrbg_status lr_batched_lrmult_round_noalloc(int64_t count, const int32_t *b, const int32_t *ra,
                                            const int32_t *rb,
                                            const double *const *AU, const int32_t *ldau,
                                            const double *const *AV, const int32_t *ldav,
                                            const double *const *AX, const int32_t *ldax,
                                            const double *const *BU, const int32_t *ldbu,
                                            const double *const *BX, const int32_t *ldbx,
                                            const double *const *BV, const int32_t *ldbv,
                                            int32_t kmax, double tol,
                                            double *const *U, const int32_t *ldu,
                                            double *const *V, const int32_t *ldv,
                                            double *sigma, int32_t *kout, void *stream);

/*
 * lrbg_round_plan -- lr_batched_lrmult_round built once and replayed: the
 * same arguments (without the stream), validated and scheduled at creation;
 * the plan owns the scratch for G, X, Y, the schedules of the fused core
 * and of the new bases, the SVD descriptors, and one captured hipGraph over
 * the whole sequence.  The caller's buffers must stay valid (and at the
 * same addresses) until the plan is destroyed; each execute recomputes U,
 * V, sigma and kout from the current contents of the inputs.  Create
 * allocates device memory and may block; execute only enqueues the graph on
 * `stream`; destroy waits for the last execute to finish.  A plan is not
 * thread-safe, and two executes of one plan must not overlap (they share
 * the scratch).  Errors as lr_batched_lrmult_round; *out is NULL on error.
 */
typedef struct lrbg_round_plan lrbg_round_plan;
lrbg_status lrbg_round_plan_create(lrbg_round_plan **out, int64_t count, const int32_t *b, const int32_t *ra,
                                   const int32_t *rb,
                                   const double *const *AU, const int32_t *ldau,
                                   const double *const *AV, const int32_t *ldav,
                                   const double *const *AX, const int32_t *ldax,
                                   const double *const *BU, const int32_t *ldbu,
                                   const double *const *BX, const int32_t *ldbx,
                                   const double *const *BV, const int32_t *ldbv,
                                   int32_t kmax, double tol,
                                   double *const *U, const int32_t *ldu,
                                   double *const *V, const int32_t *ldv,
                                   double *sigma, int32_t *kout);
lrbg_status lrbg_round_plan_execute(lrbg_round_plan *plan, void *stream);
lrbg_status lrbg_round_plan_destroy(lrbg_round_plan *plan);

/*
 * lrbg_grouped -- one launch sequence over `count` heterogeneous products
 * (any mix of ops, precisions, sizes).  Products whose input is exactly the
 * output buffer of another product of the same call (e.g. a RECOMP whose
 * core S is an INNER's T: the low-rank x low-rank chain) run after it; all
 * others run together in one grouped launch.  Same semantics as
 * lr_batched_gemm otherwise.
 */
lrbg_status lrbg_grouped(const lrbg_desc *descs, int64_t count, void *stream);

/* ------------------------------------------------------------ plans ---- */

typedef struct lrbg_plan lrbg_plan;

/* Plan flags. */
#define LRBG_PLAN_PERSISTENT 0x1u  /* persistent workgroups pulling tiles from
                                      per-XCD queues (default: one workgroup
                                      per tile, hardware-dispatched) */
#define LRBG_PLAN_NO_GRAPH   0x2u  /* replay by direct launches instead of a
                                      captured hipGraph */
#define LRBG_PLAN_DUAL       0x8u  /* role-steered dispatch: a starting
                                      workgroup takes a matrix-core-bound tile
                                      if none runs on its CU, else a
                                      memory-bound one, so both kinds share
                                      every CU (takes precedence over
                                      PERSISTENT) */
#define LRBG_PLAN_SCHED_MIX  0x4u  /* interleave compute-bound and memory-bound
                                      tiles instead of longest-first order */
#define LRBG_PLAN_UNTIMED    0x10u /* execute records no events (less host work
                                      per replay; lrbg_plan_last_ms returns a
                                      negative value, and destroy waits for the
                                      whole device instead of the last replay) */

typedef struct lrbg_plan_stats {
    int64_t products;     /* descriptors in the plan */
    int64_t tiles;        /* workgroup tiles over all levels */
    int32_t levels;       /* dependent launch levels (1 unless chained) */
    int32_t grid;         /* workgroups of the largest level's launch */
    double useful_flops;  /* 2 flops per multiply-add, no padding */
    double hbm_bytes;     /* compulsory: each operand read once, output written once */
} lrbg_plan_stats;

/*
 * lrbg_plan_create -- validate `count` descriptors, pick a tile variant per
 * (op, prec, b, r) bucket (from `tune_cache`, a file written by
 * lrbg_autotune, or built-in defaults when NULL or absent), build the
 * XCD-aware tile schedule, upload it to the device and capture the launch
 * sequence in a hipGraph (a plan whose work is one or two small launches,
 * at most 4096 tiles, replays by direct launches instead: a graph launch
 * costs more than the kernels there).  The plan keeps the device pointers; the caller's
 * buffers must stay valid while the plan is executed.  On success *out owns
 * device memory until lrbg_plan_destroy.
 */
lrbg_status lrbg_plan_create(lrbg_plan **out, const lrbg_desc *descs, int64_t count,
                             const char *tune_cache, uint32_t flags);

/* Replay the plan on `stream` (hipGraphLaunch, or the direct launches of a
 * small or LRBG_PLAN_NO_GRAPH plan; no host work per tile). */
lrbg_status lrbg_plan_execute(lrbg_plan *plan, void *stream);

/* Free the plan's device memory and graph.  Waits for the plan's work to
 * finish first.  NULL is a no-op. */
lrbg_status lrbg_plan_destroy(lrbg_plan *plan);

lrbg_status lrbg_plan_get_stats(const lrbg_plan *plan, lrbg_plan_stats *out);

/*
 * lrbg_plan_last_kernel_ms -- device time of the plan's most recent
 * execution, measured with HIP events recorded on the execution stream
 * around the grouped kernel(s) (only when the plan was created with
 * LRBG_PLAN_NO_GRAPH; otherwise around the graph launch).  Returns a
 * negative value if no execution has completed.
 */
double lrbg_plan_last_ms(lrbg_plan *plan);

/*
 * lrbg_schedule_stats -- validate `count` descriptors and build the tile
 * schedule exactly as lrbg_plan_create would, on the host only (no device
 * memory, no launch), and report its statistics.  Lets callers (and tests)
 * check sizes, levels and the work accounting without a GPU.
 */
lrbg_status lrbg_schedule_stats(const lrbg_desc *descs, int64_t count, const char *tune_cache,
                                uint32_t flags, lrbg_plan_stats *out);

/*
 * lrbg_schedule_variants -- the tile variant that lrbg_plan_create with the
 * same arguments would run for each product (host only, nothing launched).
 * variant_out: host array [count], receives variant ids (0 for a no-op
 * product); lrbg_variant_name gives their names.
 */
lrbg_status lrbg_schedule_variants(const lrbg_desc *descs, int64_t count, const char *tune_cache,
                                   uint32_t flags, int32_t *variant_out);

/* ---------------------------------------------------------- tuning ---- */

/*
 * lrbg_autotune -- for every (op, prec, b, r) bucket present in `sample`,
 * time each candidate tile variant on the sample's own buffers (outputs are
 * overwritten) and write the fastest to `cache_out` (text, one bucket per
 * line, plus a "#cand" line per candidate with its time).  Candidates are
 * the variants that fit every product of the bucket and belong to the kernel
 * family of the bucket's built-in default (a variant of another family would
 * add a launch to every plan level holding the bucket).  `reps` timed
 * repetitions per candidate (>= 1), minimum kept.  Synchronous.
 */
lrbg_status lrbg_autotune(const lrbg_desc *sample, int64_t count,
                          const char *cache_out, int32_t reps);

/*
 * lrbg_autotune_mix -- refine a tuning cache inside a mixed batch.  Starting
 * from the picks of `cache_in` (a file written by lrbg_autotune; built-in
 * defaults for buckets it lacks), each (op, prec, b, r) bucket of `sample`,
 * largest estimated share of the batch first, tries each compatible variant
 * of the same kernel family whose isolated time in `cache_in` is within
 * 1.5x of the bucket's best:
 * the whole sample is planned (with `flags`, as the caller's plans will be)
 * with that one change and replayed alternately with the current plan
 * (`reps` timed replays each, medians compared); a change that is faster by
 * more than 0.4% twice in a row is kept.  At most `passes` passes over the
 * buckets, stopping after a pass that keeps nothing.  `cache_out` gets the
 * input's candidate lines, one "#mix" line per trial and every bucket's pick
 * with its own isolated time.  Synchronous; outputs of the sample are
 * overwritten.  The paper tunes its kernels per processor empirically
 * (Table 1, the B_skinny sweep of Sec. 6); this is the batch-level analogue.
 */
lrbg_status lrbg_autotune_mix(const lrbg_desc *sample, int64_t count, const char *cache_in,
                              const char *cache_out, int32_t reps, int32_t passes, uint32_t flags);

/* Number of tile variants compiled in, and the name of one (for tooling). *//* Number of tile variants compiled in, and the name of one (for tooling). */
int32_t lrbg_variant_count(void);
const char *lrbg_variant_name(int32_t v);

/* ----------------------------------------------------------- misc ---- */

const char *lrbg_status_string(lrbg_status s);
const char *lrbg_last_error(void);   /* thread-local detail of the last failure */
int32_t lrbg_version(void);           /* major*10000 + minor*100 + patch */

#ifdef __cplusplus
}
#endif

#endif /* LRBG_H */
