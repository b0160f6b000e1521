/*
 * leg2cheb.h -- C ABI of the MI355X (gfx950) Legendre <-> Chebyshev transform.
 *
 * The operation (Mortensen, arXiv 2411.00033, Sec. 1, Eqs. (AfCf), (directmv)):
 *
 *   leg2cheb:  out = C^{-1} A in        (Legendre coefficients -> Chebyshev coefficients)
 *   cheb2leg:  out = A^{-1} C in        (Chebyshev coefficients -> Legendre coefficients)
 *
 * with a_ij = Lambda((j-i)/2) Lambda((j+i)/2) for j >= i, j - i even, zero otherwise
 * (Eqs. (aij), (Lambda)), Lambda(x) = Gamma(x+1/2)/Gamma(x+1), and C = diag(c_i pi/2),
 * c_0 = 2, c_i = 1 otherwise.  Both are applied in O(n) work by the modal fast
 * multipole method of Alg. 4: near-diagonal leaf blocks done directly, an upward
 * pass (Eq. (wtk), App. A2), low-rank far-field products with Chebyshev
 * coefficient matrices Ahat (Eq. (aklmore)), and the downward spreading of
 * step (4).  cheb2leg uses the reverse kernel of Eq. (Lxymod) with c applied to
 * the input first (Sec. 4.1).
 *
 * Conventions
 *   - All data pointers passed to leg2cheb_execute are DEVICE pointers on the
 *     device that was current when the plan was made.  Layout: contiguous FP64
 *     [batch][n], row-major (item b starts at ptr + b*n).  in and out must not
 *     overlap.
 *   - stream is a hipStream_t (NULL = the null stream).  Execution is
 *     asynchronous with respect to the host; errors in arguments are reported
 *     synchronously before anything is enqueued.
 *   - Every call returns an l2c_status code; no exception crosses the ABI.
 *   - Plans own their device tables; they are freed by leg2cheb_destroy.  A plan
 *     may be used from one host thread at a time.
 */
#ifndef LEG2CHEB_H
#define LEG2CHEB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct l2c_plan_s *l2c_plan_t;

enum l2c_direction { L2C_LEG2CHEB = 0, L2C_CHEB2LEG = 1 };

/* Arithmetic of the execute.  Inputs and outputs are FP64 in every form, and the
 * plan builds its tables in FP64.
 *   L2C_FP64    every product and sum in FP64.
 *   L2C_FP32    the batched form (not in the paper: it serves batches of transforms):
 *               the far part (steps (1)-(5)) from FP32 tables, every product on the
 *               matrix cores in FP32 with FP32 accumulation, 16 transforms per 16 x 16
 *               tile; the near field of step (6) (the dense near-diagonal leaf blocks),
 *               the sum of near and far parts and step (7) in FP64 (FP64 matrix cores).
 *               Needs rank <= 16, leaf_size <= 64 and n <= 2^28; E_inf about 1e-6 of the
 *               far part's magnitude (rank 16): ~1e-9 on decaying inputs f_j ~ 1/j, up to
 *               ~1e-7 on undecayed ones.
 *   L2C_BF16X2  the same batched form with every FP32 operand x split as hi = bf16(x),
 *               lo = bf16(x - hi) and each product formed as hi*hi + hi*lo + lo*hi on the
 *               BF16 matrix cores with FP32 accumulation (products accurate to about
 *               2^-17); same limits as L2C_FP32.
 *   L2C_FP16X2  the same with FP16 hi + lo operands (about 2^-22 per product) on the FP16
 *               matrix cores with FP32 accumulation.  FP16 spans only 2^-24 .. 2^16, so
 *               each Ahat submatrix is stored scaled by a power of two (undone after its
 *               product) and each column of every runtime operand (one transform) is
 *               scaled by a power of two from its largest magnitude before it is split;
 *               same limits as L2C_FP32. */
enum l2c_precision { L2C_FP64 = 0, L2C_FP32 = 1, L2C_BF16X2 = 2, L2C_FP16X2 = 3 };

/* Execution path of a plan (l2c_plan_info.path). */
enum l2c_path {
    L2C_PATH_DIRECT = 0, /* the whole product directly, row by row (Alg. 1): plans with
                            L = 0, and short FP64 plans (L2C_OPT_DIRECT) */
    L2C_PATH_THREE = 1,  /* three launches: upward pass, top levels, far field + rest */
    L2C_PATH_SINGLE = 2, /* one launch, workgroups exchange tree nodes through ready flags */
    L2C_PATH_BATCHED = 3, /* L2C_FP32 / L2C_BF16X2 / L2C_FP16X2 plans: 16 transforms per matrix-core tile */
    L2C_PATH_DENSE = 4,   /* FP64 plans with n <= 4096 and max_batch >= 64: Alg. 1 as dense
                             per-parity products on the FP64 matrix cores */
    L2C_PATH_REGEN = 5    /* three launches plus one, for plans made with L2C_TABLES_REGEN: the
                             far-field blocks below the subtree roots are recomputed from the
                             kernel samples in every execute instead of read from a table */
};

/* Plan options (leg2cheb_plan_set_option). */
enum l2c_option {
    L2C_OPT_SINGLE_LAUNCH = 1, /* 1: single-launch path when the plan allows it (default); 0: three launches */
    L2C_OPT_DIRECT = 2,        /* 1: Alg. 1 directly for short FP64 plans (default); 0: Alg. 4 */
    L2C_OPT_EXCHANGE_TIMEOUT_US = 3 /* bound of the single-launch path's waits for other workgroups */
};

/* Status bits of the single-launch path (leg2cheb_plan_status).  Every wait inside that
 * kernel is bounded on the device's wall clock; one that gives up sets its bit, and the
 * output of that execute is wrong. */
enum l2c_status_bit {
    L2C_STATUS_EXCHANGE = 1, /* a wait for another workgroup's exchanged tree nodes */
    L2C_STATUS_WORKERS = 2,  /* a barrier among the waves of one workgroup */
    L2C_STATUS_STREAM = 4    /* the far-field streaming wave waiting for its operands */
};

enum l2c_status {
    L2C_OK = 0,
    L2C_EINVAL = -1,      /* invalid argument (null pointer, bad size, overlap, ...) */
    L2C_ENOMEM = -2,      /* device or host allocation failed */
    L2C_EHIP = -3,        /* a HIP runtime call or kernel launch failed */
    L2C_EUNSUPPORTED = -4 /* valid request that the library does not implement */
};

struct l2c_plan_info {
    int64_t n;             /* input length */
    int64_t n_pad;         /* N = s 2^(L+2) >= n, Eq. (numlevels); n_pad = n when direct-only */
    int32_t levels;        /* L; 0 means the plan applies the whole product directly (Alg. 1) */
    int32_t s;             /* half the side of the smallest submatrices, Sec. 3.1 */
    int32_t rank;          /* M, Chebyshev expansion rank, Eq. (Aij) */
    int32_t direction;     /* l2c_direction */
    int32_t precision;     /* l2c_precision */
    int32_t path;          /* l2c_path used by leg2cheb_execute */
    int64_t n_blocks;      /* N_b, Eq. (total_blocks_and_mats) */
    int64_t n_submatrices; /* N_c = 3 N_b */
    int64_t table_bytes;   /* device bytes of the plan tables (Ahat, T, B, ...) */
    int64_t workspace_bytes; /* device bytes of the execution workspace for the current batch capacity */
    int64_t ahat_bytes;    /* bytes of the Ahat table alone (read once per execute) */
    int32_t basis;         /* l2c_basis */
    int32_t reserved;      /* zero */
};

/*
 * Build a plan for transforms of length n (Sec. 3.1 sizes; Secs. 3.2, 4.3 tables).
 *   plan       [out] receives the new plan handle (set to NULL on error).
 *   n          input length, n >= 1.
 *   direction  L2C_LEG2CHEB or L2C_CHEB2LEG.
 *   leaf_size  side 2*s_hat of the smallest far-field submatrices (Eq. (numlevels)
 *              uses s_hat); even, 4 <= leaf_size <= 128.  The paper uses s = 32,
 *              i.e. leaf_size 64 (Sec. 5).  The effective s lies in [s_hat/2, s_hat].
 *   rank       M, number of Chebyshev modes per axis; one of the ranks the library
 *              has kernels for (leg2cheb_rank_supported).  The paper uses 18.
 * The device tables are built with kernels on the current device and stream 0;
 * the call returns after they are complete.
 * Errors: L2C_EINVAL, L2C_EUNSUPPORTED (rank), L2C_ENOMEM, L2C_EHIP.
 */
int leg2cheb_plan(l2c_plan_t *plan, int64_t n, int direction, int leaf_size, int rank);

/*
 * As leg2cheb_plan, plus:
 *   precision  l2c_precision: L2C_FP64, or L2C_FP32 / L2C_BF16X2 / L2C_FP16X2 (rank <= 16,
 *              leaf_size <= 64, n <= 2^28, else L2C_EUNSUPPORTED);
 *   max_batch  workspace is sized for this many items (>= 1); execute grows it on
 *              demand (a synchronizing allocation) when a larger batch arrives;
 *   stream     hipStream_t on which the table-building kernels run (NULL = null stream).
 */
int leg2cheb_plan_ex(l2c_plan_t *plan, int64_t n, int direction, int leaf_size, int rank,
                     int precision, int64_t max_batch, void *stream);

/* Basis of the far-field expansions (leg2cheb_plan_basis).
 *   L2C_MODAL  Chebyshev coefficients (the paper's method, Secs. 3.2 and 4.1): Ahat from a
 *              2-D DCT of the kernel samples, T(sigma) Chebyshev polynomials, the exact
 *              dyadic B(0), B(1) (App. A3).
 *   L2C_NODAL  values at the Chebyshev-Gauss nodes with the Lagrange basis (Alpert and
 *              Rokhlin's nodal method, Sec. 3.2, Eq. (AijLag)): the far-field blocks are
 *              the kernel samples themselves, the leaf matrices hold l_k(X_m^sigma), and
 *              the transfers are the dense interpolation matrices l_k((X_j + 2l - 1)/2).
 *              Mathematically the same approximation (the interpolant of degree M-1 at the
 *              nodes); the upward and downward transfers cost dense M x M products
 *              instead of the modal triangular ones (Sec. 4.2). */
enum l2c_basis { L2C_MODAL = 0, L2C_NODAL = 1 };

/*
 * As leg2cheb_plan_ex, with the expansion basis.  L2C_NODAL is served by the batched
 * kernels only: precision L2C_FP32, L2C_BF16X2 or L2C_FP16X2, or L2C_FP64 with rank <= 16,
 * leaf_size <= 64 and a batch large enough for the FP64 tile form (max_batch >= 16, and
 * n above the short-transform paths' bounds); otherwise L2C_EUNSUPPORTED.
 */
int leg2cheb_plan_basis(l2c_plan_t *plan, int64_t n, int direction, int leaf_size, int rank, int precision,
                        int64_t max_batch, int basis, void *stream);

/* What a plan keeps of the far-field submatrices (leg2cheb_plan_tables).
 *   L2C_TABLES_STORED  every Ahat submatrix (Eq. (aklmore)), built once at plan time and read
 *                      by every execute: 8 M^2 bytes per submatrix, the dominant traffic of an
 *                      execute (127 MB at n = 10^6, rank 18).
 *   L2C_TABLES_REGEN   only the submatrices of the tree's top levels; every execute recomputes
 *                      the others (all but a few hundred) from the kernel samples and applies
 *                      each in the factored form D (S (D^T w)) of its 2-D DCT, so it is never
 *                      formed.  The samples use Sec. 4.3's split of the kernel: the factor
 *                      Lambda((y-x)/2) depends only on the level and the offset from the
 *                      diagonal and is tabulated at plan time (2 M^2 doubles per level); the
 *                      factor in (x+y)/2 is evaluated per sample (Eq. (tau)).  The stored
 *                      submatrices are those of levels 0..L-1-kd, where kd (<= 7) is the
 *                      depth of the subtrees the execute kernels take, so the plan holds about
 *                      2^kd times fewer (at n = 10^6: 127 MB -> 2 MB) and builds faster; each
 *                      execute trades the table's bytes for the samples' arithmetic.  The same
 *                      approximation as L2C_TABLES_STORED, up to rounding. */
enum l2c_tables { L2C_TABLES_STORED = 0, L2C_TABLES_REGEN = 1 };

/*
 * An FP64 plan in the modal basis, with the far-field submatrices kept as `tables` says
 * (l2c_tables); the other arguments as in leg2cheb_plan_ex.  L2C_TABLES_STORED is
 * leg2cheb_plan_ex with precision L2C_FP64.  A plan with L2C_TABLES_REGEN and L >= 1 always
 * executes on L2C_PATH_REGEN (the direct, dense, tile and single-launch paths need the
 * stored blocks); leg2cheb_execute_noalloc refuses it (L2C_EUNSUPPORTED), and
 * leg2cheb_plan_export has no table 0 for it (L2C_EUNSUPPORTED).
 * Errors: L2C_EINVAL (tables not one of l2c_tables, and those of leg2cheb_plan_ex),
 * L2C_EUNSUPPORTED (rank), L2C_ENOMEM, L2C_EHIP.
 */
int leg2cheb_plan_tables(l2c_plan_t *plan, int64_t n, int direction, int leaf_size, int rank, int64_t max_batch,
                         int tables, void *stream);

/*
 * The plan cache (planning costs about 3 times an execute, Sec. 5.2): returns the shared
 * plan made with exactly these arguments on the current device, building it on the first
 * call, and takes one reference to it; leg2cheb_destroy releases one reference and frees
 * the plan with the last.  A shared plan is one plan: executes through it on different
 * streams must be ordered by the caller, as for any plan.  Thread-safe.
 * Errors: those of leg2cheb_plan_basis.
 */
int leg2cheb_plan_cached(l2c_plan_t *plan, int64_t n, int direction, int leaf_size, int rank, int precision,
                         int64_t max_batch, int basis, void *stream);

/* Plans in the cache and the references they hold (either pointer may be NULL). */
int leg2cheb_plan_cache_size(int64_t *plans, int64_t *references);

/*
 * out[b, 0:n] = T(in[b, 0:n]) for b < batch, T = C^{-1}A (leg2cheb) or A^{-1}C
 * (cheb2leg) as fixed at plan time (Alg. 4, steps (1)-(7)).
 *   in, out  device pointers, FP64 [batch][n], non-overlapping.
 *   batch    >= 0; 0 is a no-op.
 *   stream   hipStream_t.
 * Enqueues the kernels and returns.  Allocates only when batch exceeds the
 * workspace capacity.  On L2C_EHIP, out is undefined.  Returns L2C_EHIP without
 * enqueuing anything while a status bit of an earlier, finished single-launch execute
 * of the plan is set (its output was wrong; see leg2cheb_plan_status, which clears the
 * bits).  The check reads host memory and does not wait for executes still running.
 */
int leg2cheb_execute(l2c_plan_t plan, const double *in, double *out, int64_t batch, void *stream);

/*
 * leg2cheb_execute for callers that cannot allocate memory (code under HIP graph capture,
 * serving loops, harnesses that forbid it): the same transform, with no hipMalloc, hipFree
 * or other allocation in the call.  FP64 plans only.  Plans on the dense or direct path
 * run as in leg2cheb_execute (those kernels use no workspace); every other plan runs the
 * three-launch path of Alg. 4 with its upward vectors in a workspace of 64 MiB that the
 * library holds in a fixed device array per device for the life of the process, instead
 * of the plan's own workspace.  That array is shared by every call on the device: calls
 * that overlap on one device (other streams, other threads) race and must not be made.
 * The output agrees bit for bit with leg2cheb_execute on the three-launch path.
 *   in, out, batch, stream  as in leg2cheb_execute.
 * Errors: L2C_EINVAL as leg2cheb_execute, and when batch x (2^(L+2) - 4) x 2 x rank x 8
 * bytes exceeds 64 MiB (at n = 10^6, rank 18: batch > 7); L2C_EUNSUPPORTED (a plan of a
 * batched precision form, or one made with L2C_TABLES_REGEN); L2C_EHIP as leg2cheb_execute.
 */
int leg2cheb_execute_noalloc(l2c_plan_t plan, const double *in, double *out, int64_t batch, void *stream);

/* Release the plan and its device memory (synchronizes the device first); for a plan of
 * the plan cache, release one reference (the memory goes with the last).  NULL is a no-op. */
int leg2cheb_destroy(l2c_plan_t plan);

/* Sizes and memory of a plan. */
int leg2cheb_plan_info(l2c_plan_t plan, struct l2c_plan_info *info);

/*
 * Copy one plan table to host memory, in the paper's canonical layout
 * (used by tests to check the plan stage).
 *   table 0 = Ahat: [level][block][r][k][l], levels 0..L-1, b_gamma = 2^(gamma+1)-1
 *                   blocks each, r = p + q(q+1)/2 (Eq. (cfrompq)), M x M row-major;
 *         1 = T:    [sigma][m][k] = T_k(-1 + (2m+sigma)/s), 2 x s x M (Eq. (Xs));
 *         2 = B:    B(0) then B(1), 2 x M x M row-major (Eq. (Tky));
 *         3 = w:    the upward vectors of steps (1)-(2) (Eqs. (wMM), (wtk)) of the first
 *                   item of the last execute on the three-launch path, as its workspace
 *                   holds them: [node][sigma][k], every node of every level, level g
 *                   (2^(g+2) nodes) starting at node 2^(g+2) - 4, 2^(L+2) - 4 nodes in
 *                   all.  Column node 2b + q + 2 of level g is the w(g, b, q) of the
 *                   paper.  After executes on other paths the contents are unspecified.
 *   dst   host buffer of at least `bytes` bytes; bytes must equal the table size
 *         (query with dst = NULL: *needed receives the size and nothing is copied).
 *         Copies are synchronous on the null stream.
 * Errors: L2C_EINVAL (bad table id, size mismatch, direct-only plan), L2C_EUNSUPPORTED
 * (table 0 of an L2C_FP32 or L2C_BF16X2 plan, which keeps Ahat only in its own layout;
 * table 3 of a plan without an FP64 workspace), L2C_EHIP.
 */
int leg2cheb_plan_export(l2c_plan_t plan, int table, void *dst, int64_t bytes, int64_t *needed);

/*
 * Set a plan option (enum l2c_option).
 *   L2C_OPT_SINGLE_LAUNCH  value 1 (default) runs Alg. 4 as one kernel launch when the
 *       geometry allows it: every subtree of 2^kd finest nodes gets one workgroup, and
 *       all workgroups of an item must be resident at once (at most one per compute
 *       unit).  The workgroups exchange only subtree roots, the two boundary nodes of
 *       each depth, and the upward vectors above the subtrees.  Value 0 selects the
 *       three-launch path.  Both paths use the same plan tables and agree to rounding.
 *   L2C_OPT_DIRECT  value 1 (default) runs short FP64 transforms (L >= 1, n <= 8192
 *       and max_batch n^2 <= W, W = 2^27 for n <= 4096 and 2^26 above) as Alg. 1, every
 *       output row one sum over its band, on many small workgroups: at these lengths a
 *       multipole launch is dominated by its dependency chain.  An execute with
 *       batch n^2 > W takes Alg. 4 instead.
 *       Value 0 selects Alg. 4 (the path L2C_OPT_SINGLE_LAUNCH chooses).  The plan
 *       builds the multipole tables either way.  Plans on the dense path (n <= 4096,
 *       max_batch >= 64) use it regardless.
 *   L2C_OPT_EXCHANGE_TIMEOUT_US  0 <= value <= 6e7 (default 1e6): how long a workgroup of
 *       the single-launch kernel waits for tree nodes from another workgroup before it
 *       gives up and sets L2C_STATUS_EXCHANGE.  A wait that gives up ends normally, so the
 *       kernel still ends.  Value 0 makes every such wait give up after its first poll and
 *       set the bit whether or not it found its values: tests use it to take this error
 *       path on purpose.
 * Single-launch kernels of one device are ordered by the library (a launch on another
 * stream waits for all work enqueued so far on the stream of the previous one, which must
 * therefore still exist), so they never compete for compute units; other work may delay
 * but not block them.  A plan must not be executed on two streams at the same time.
 * Errors: L2C_EINVAL (plan, option or value), L2C_EUNSUPPORTED (value 1 on a plan whose
 * geometry has no single-launch form, or that is not a short FP64 plan).
 */
int leg2cheb_plan_set_option(l2c_plan_t plan, int option, int64_t value);

/*
 * Status of the plan's single-launch executes since it was made or since the last call:
 * the l2c_status_bit bits of every wait that gave up (the output of that execute is
 * wrong).  A wait for another workgroup gives up after L2C_OPT_EXCHANGE_TIMEOUT_US
 * (default one second), every other wait after one second.  Synchronizes the device,
 * then clears the bits.  *status = 0 for plans without a single-launch path.
 */
int leg2cheb_plan_status(l2c_plan_t plan, int *status);

/*
 * Optional timing hook for benchmarks: when both events (hipEvent_t) are
 * non-NULL, execute records `before` immediately before and `after`
 * immediately after the kernel that streams Ahat (the single-launch kernel, or
 * the far-field kernel of the three-launch path), on the execute stream, for the
 * first launch of the call.  Pass NULLs to turn it off.
 */
int leg2cheb_set_timing_events(l2c_plan_t plan, void *before, void *after);

/*
 * Ragged batches: count independent transforms of different lengths and directions
 * (Alg. 4 for each), planned together and executed as one call.
 */
typedef struct l2c_batch_s *l2c_batch_t;

/*
 * Leaf size and rank of the transforms of a ragged batch, chosen per size bucket:
 * bucket k covers the lengths n with buckets[k-1].n_max < n <= buckets[k].n_max, and
 * the last bucket covers every larger n.  leaf_size and rank as in leg2cheb_plan_ex.
 */
struct l2c_tuning_bucket {
    int64_t n_max;
    int32_t leaf_size;
    int32_t rank;
};
struct l2c_tuning {
    int32_t count;                            /* 1 .. 32, n_max strictly increasing */
    const struct l2c_tuning_bucket *buckets;  /* host array [count] */
};

/*
 * Plan a ragged batch.  Transforms with the same size bucket, levels L (Eq. (numlevels))
 * and direction form one group with one set of tables (the tables depend on L, s, M and
 * the kernel only): every group is planned with its bucket's full half-leaf
 * s = leaf_size / 2, so its shorter transforms only see more zero padding, and each item
 * keeps its own length.  Results therefore agree with a separately planned transform
 * (whose s may be smaller) to the method's accuracy, not bit for bit.  L = 0 transforms
 * (Alg. 1 directly) group by bucket and direction.  FP64 groups execute concurrently on
 * side streams of the batch (the three-launch path, or the dense path for n <= 4096 with
 * 64 or more items); the batched forms execute all groups in one launch per kernel shape.
 *   batch      [out] receives the new handle (NULL on error).
 *   count      number of transforms, >= 1.
 *   n          host array [count], each >= 1 (lengths are not limited otherwise).
 *   direction  host array [count] of L2C_LEG2CHEB / L2C_CHEB2LEG.
 *   precision  as in leg2cheb_plan_ex, shared by all transforms.
 *   tuning     the size buckets, or NULL for the library's own table for the precision
 *              (made by its autotuner from timings of ragged batches; leg2cheb_batch_tuning
 *              returns it).
 *   stream     hipStream_t for the table-building kernels (NULL = null stream).
 * The call returns after every group's tables are built.  Device memory: one plan per
 * group plus count entries of lengths and pointers.
 * Errors: L2C_EINVAL (arguments, bucket order, leaf size), L2C_EUNSUPPORTED (a rank
 * without kernels; rank > 16, leaf_size > 64 or n > 2^28 in a batched form), L2C_ENOMEM,
 * L2C_EHIP.
 */
int leg2cheb_batch_plan(l2c_batch_t *batch, int64_t count, const int64_t *n, const int *direction, int precision,
                        const struct l2c_tuning *tuning, void *stream);

/*
 * The library's size buckets for a precision (the tuning used when leg2cheb_batch_plan
 * gets NULL).  Writes min(cap, *count) buckets to buckets (host memory; may be NULL when
 * cap is 0) and the table's length to *count.  No device call.
 * Errors: L2C_EINVAL (precision, count NULL, cap < 0, buckets NULL with cap > 0).
 */
int leg2cheb_batch_tuning(int precision, struct l2c_tuning_bucket *buckets, int32_t cap, int32_t *count);

/*
 * out[i][0:n[i]] = T_i(in[i][0:n[i]]) for i < count, T_i the transform of item i.
 *   in, out  host arrays [count] of device pointers (FP64, n[i] values each); no output
 *            may overlap any input or another output.
 *   stream   hipStream_t.
 * Copies the pointer lists to the device (through pinned memory owned by the batch)
 * and enqueues every group; work on the batch's side streams is ordered after the
 * copies on stream, and stream waits for it before anything enqueued later.  Allocates
 * nothing.  A later call first waits on the host for the previous call's pointer copy,
 * and orders its own work on its stream after the whole previous call (which may have
 * used another stream).  On L2C_EHIP, the outputs are undefined.
 */
int leg2cheb_batch_execute(l2c_batch_t batch, const double *const *in, double *const *out, void *stream);

/* Groups of the batch and the total device bytes of their tables. */
int leg2cheb_batch_info(l2c_batch_t batch, int64_t *groups, int64_t *table_bytes);

/* Release the batch (synchronizes the device first).  NULL is a no-op. */
int leg2cheb_batch_destroy(l2c_batch_t batch);

/*
 * Discrete cosine transforms (Sec. 1: the fast cosine transforms on the Chebyshev side of
 * the transform; Sec. 5.2 compares the FMM's time with a DCT of type 2), in FP64:
 *   kind 2:  y_k = sum_{j<n} x_j cos(pi k (j + 1/2) / n),   k < n;
 *   kind 3:  y_j = sum_{k<n} x_k cos(pi k (j + 1/2) / n),   j < n
 * (no normalization; kind 3 evaluates the Chebyshev series sum_k x_k T_k at the
 * Chebyshev-Gauss points cos((j + 1/2) pi / n)).  Computed through an n-point complex FFT
 * (hand-written, radices 2, 3, 4, 5, 7, 8): n must have no prime factor above 7 and
 * n <= 2^27, else L2C_EUNSUPPORTED.
 *   dct        [out] receives the plan (NULL on error).
 *   kind       2 or 3.
 *   max_batch  workspace (n > 4096: 16 n bytes per transform) is sized for this many
 *              transforms; execute grows it on demand (a synchronizing allocation).
 *   stream     hipStream_t on which the root tables are built (the call waits for them).
 * Errors: L2C_EINVAL, L2C_EUNSUPPORTED, L2C_ENOMEM, L2C_EHIP.
 */
typedef struct l2c_dct_s *l2c_dct_t;
int leg2cheb_dct_plan(l2c_dct_t *dct, int64_t n, int kind, int64_t max_batch, void *stream);

/*
 * out[b, :] = DCT(in[b, :]) for b < batch: caller-owned device arrays of batch x n FP64
 * values, row-major, not overlapping (L2C_EINVAL).  Asynchronous on stream; batch = 0 is a
 * no-op.  On L2C_EHIP the output is undefined.  Calls on one plan must not overlap in time
 * on different streams (they share the plan's workspace).
 */
int leg2cheb_dct_execute(l2c_dct_t dct, const double *in, double *out, int64_t batch, void *stream);

/* Release the plan (synchronizes the device first).  NULL is a no-op. */
int leg2cheb_dct_destroy(l2c_dct_t dct);

/*
 * Legendre series on the Chebyshev-Gauss grid and back (the use of the transform that
 * Sec. 1 describes): with x_j = cos((j + 1/2) pi / n),
 *   L2C_LEG2GRID:  out_j = sum_{k<n} in_k P_k(x_j)  (leg2cheb, then the DCT of kind 3);
 *   L2C_GRID2LEG:  out = the Legendre coefficients of the degree < n polynomial that
 *                  takes the values in_j at x_j (the DCT of kind 2 scaled by
 *                  (2 - delta_k0) / n, i.e. Chebyshev-Gauss quadrature, then cheb2leg).
 * The two are inverse to each other up to the FMM's error.  leaf_size and rank as in
 * leg2cheb_plan (FP64); n as for the DCT (prime factors 2, 3, 5, 7; n <= 2^27).
 * Owns an FMM plan, a DCT plan and an intermediate array of max_batch x n FP64 values
 * (grown on demand by execute, synchronizing).
 * Errors: L2C_EINVAL, L2C_EUNSUPPORTED, L2C_ENOMEM, L2C_EHIP.
 */
enum l2c_grid_direction { L2C_LEG2GRID = 0, L2C_GRID2LEG = 1 };
typedef struct l2c_grid_s *l2c_grid_t;
int leg2cheb_grid_plan(l2c_grid_t *grid, int64_t n, int direction, int leaf_size, int rank, int64_t max_batch,
                       void *stream);

/* out[b, :] = the grid transform of in[b, :]; arguments and errors as leg2cheb_dct_execute,
 * plus those of leg2cheb_execute on the owned FMM plan. */
int leg2cheb_grid_execute(l2c_grid_t grid, const double *in, double *out, int64_t batch, void *stream);

/* The FMM plan and the DCT plan a grid plan owns (for leg2cheb_plan_info and for timing
 * the two stages apart); owned by the grid plan, never destroyed by the caller. */
l2c_plan_t leg2cheb_grid_fmm(l2c_grid_t grid);
l2c_dct_t leg2cheb_grid_dct(l2c_grid_t grid);

/* Release the grid plan and what it owns (synchronizes the device first).  NULL is a no-op. */
int leg2cheb_grid_destroy(l2c_grid_t grid);

/* Non-zero if the library has kernels for rank M. */
int leg2cheb_rank_supported(int rank);

/*
 * Test hook for the error paths (no paper passage: the method allocates nothing itself).
 * Every device and pinned host allocation the library makes (plans, workspaces, batches,
 * plan_export's staging) counts down a process-wide counter: with fail_at = k >= 1 the
 * k-th allocation after this call fails as if memory were exhausted, and the call that
 * made it returns L2C_ENOMEM having released everything it had allocated; fail_at = 0
 * disarms the hook; fail_at = -1 only queries.
 *   pending  [out, may be NULL] the countdown before this call (0: disarmed or fired).
 *   live     [out, may be NULL] allocations the library holds now (for leak checks).
 * Errors: L2C_EINVAL (fail_at < -1).
 */
int leg2cheb_debug_alloc_hook(int64_t fail_at, int64_t *pending, int64_t *live);

/*
 * Test hook for the index arithmetic (no paper passage): for the plan geometry that
 * leg2cheb_plan would make from (n, leaf_size, rank) -- L, s of Eq. (numlevels) and the
 * kernels' subtree depths -- evaluates on the host every index map of the execute kernels
 * (local block <-> depth and index, table groups, workspace nodes of every block's column
 * nodes, the LDS layouts, each single-launch unit's tree-top table, the regenerated
 * blocks' output and factor rows) and compares each index with the size of the buffer it
 * addresses.  Makes no device call and allocates no device memory.
 * Returns L2C_OK when every index is in bounds (and for direct-only geometries, L = 0), a
 * positive number naming the first check that fails (1 block map, 2 table groups,
 * 3 workspace, 4 three-launch LDS, 5 single-launch LDS, 6 tree-top items, 7 tree-top
 * schedule, 8 regenerated blocks, 9 subtree count), or L2C_EINVAL for arguments
 * leg2cheb_plan refuses.
 */
int leg2cheb_debug_check_geometry(int64_t n, int leaf_size, int rank);

/* Static description of a status code. */
const char *leg2cheb_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* LEG2CHEB_H */
