/*
 * ooc.h -- C ABI of the MI355X out-of-core FP64 matrix product.
 *
 * The operation (the MMOOC kernel of Hanlon, Khalighzadeh, Manumachu and
 * Lastovetsky, "libhclooc", Section V, text after Fig. 2):
 *     C = alpha * A * B + beta * C
 * with A (M x K), B (K x N) and C (M x N) row-major in host memory, leading
 * dimensions lda >= K, ldb >= N, ldc >= N (elements), and a device-memory
 * budget smaller than the operands.  The library partitions the operands into
 * tiles that fit the budget, moves tiles host-to-device, runs a tile product
 * on each, and moves C tiles back, overlapping the three on HIP streams
 * (Section V, Figs. 3 and 4: stages S(b), S(a), S(c), DGEMM, R(c)).
 *
 * Conventions for every entry point
 *   - Sizes are element counts unless the name ends in _bytes.
 *   - Host pointers are borrowed: the caller owns A, B, C and any arena it
 *     passes; the library never frees them.  A, B and C must be page-locked
 *     host memory (ooc_host_alloc, or hipHostMalloc).
 *   - Calls are synchronous: they return after C is complete in host memory
 *     (the paper's final stream synchronisation, Fig. 2).
 *   - Errors are reported by the return code only (no exception crosses the
 *     ABI); ooc_last_error() gives a message for the calling thread.  On an
 *     error C is unspecified except for the blocks counted in
 *     ooc_stats.blocks_done, which were written back completely.
 *   - Quick returns follow the reference BLAS: M == 0 or N == 0 does nothing;
 *     alpha == 0 or K == 0 gives C = beta*C without reading A or B; beta == 0
 *     does not read C (NaN in C does not propagate).
 *   - One call at a time per device; calls on one device from several host
 *     threads are serialised by the library.
 */
#ifndef OOC_H
#define OOC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  OOC_OK = 0,
  OOC_ERR_ARG = 1,        /* invalid size, leading dimension, pointer, plan or option */
  OOC_ERR_BUDGET = 2,     /* no plan fits in budget_bytes (or the plan's footprint exceeds it) */
  OOC_ERR_DEVICE_MEM = 3, /* budget above the device's free memory, or device allocation failed */
  OOC_ERR_NOT_PINNED = 4, /* A, B or C is not page-locked host memory */
  OOC_ERR_HIP = 5,        /* a HIP runtime call failed (message in ooc_last_error) */
  OOC_ERR_NO_DEVICE = 6,  /* no usable gfx950 device with that ordinal */
  OOC_ERR_INJECTED = 7,   /* failure injected by OOC_FAIL_AT (tests of error paths) */
  OOC_ERR_CAPACITY = 8,   /* an output array is too small (ooc_schedule, ooc_plan_candidates) */
  OOC_ERR_NOT_SPD = 9     /* ooc_potrf: the matrix is not positive definite (see its info) */
} ooc_status;

/* FP64: tile products in FP64 on matrix cores.  SPLIT_BF16: each tile product
 * is formed from s BF16 slices per operand (error-free splitting, Ozaki et al.
 * 2012): slice products are exact with FP32 accumulation over windows of
 * 64-256 k, window sums are added exactly in int32, and the weighted slice
 * sums are combined in FP64; only the slices beyond s are dropped (truncation error
 * about (s+1) 2^(-8s) relative to (|A||B|)_ij times the row/column spread).
 * SPLIT_INT8: the same scheme with s INT8 slices of 7 bits each (digits
 * truncated toward zero, |digit| <= 127) multiplied on INT8 matrix cores with
 * exact INT32 sums; twice the BF16 rate per slice product, one bit less per
 * slice (truncation error about (s+2) 2^(-7s) relative, as above). */
typedef enum { OOC_FP64 = 0, OOC_SPLIT_BF16 = 1, OOC_SPLIT_INT8 = 2 } ooc_precision;

/* How a plan is chosen.  PAPER: the paper's partitioner (Section V: fewest
 * vertical B slices, then fewest horizontal A slices, such that two C blocks of
 * a column, their A slices and the column's B slice fit), two streams used
 * round robin, A and C double-buffered, B single-buffered.  MODEL: the
 * candidate with the smallest simulated pipeline time under the analytic
 * cost model.  SWEEP: the measured sweep -- the cost model's n best
 * candidates (n = 8, or OOC_SWEEP_TOP in the environment) are each timed by
 * one product on the caller's A and B into a page-locked scratch C of C's
 * shape (after one warm-up product; C itself is written once, by the chosen
 * plan), and the fastest is used and remembered for the process, keyed by
 * the problem (sizes, beta != 0, budget, precision, slices, stream count,
 * transposed B, lower triangle).  It applies to ooc_gemm, ooc_gemm_ex and
 * ooc_syrk; the planning-only calls, the accumulation sessions and the
 * products inside ooc_potrf and ooc_trsm take the cost model's choice.  If
 * the scratch C cannot be allocated the cost model's choice is used and not
 * remembered.  MLP: among the cost model's 8 best candidates, the one with
 * the smallest time predicted by the loaded network (the network shipped
 * beside the library is loaded on first use).  The network declines when
 * none is loaded, for split-BF16 plans when it was trained on FP64 timings
 * only (which it records as a constant slice-count feature), for split-INT8
 * plans (the shipped network has not seen their timings), and for problems
 * whose M, N, K or budget lies more than four standard deviations (log
 * scale) from the training problems' mean; then the product calls that
 * SWEEP applies to plan by the measured sweep, and every other call takes
 * the cost model's choice.  AUTO = MODEL. */
typedef enum {
  OOC_PLAN_AUTO = 0,
  OOC_PLAN_PAPER = 1,
  OOC_PLAN_MODEL = 2,
  OOC_PLAN_MLP = 3,
  OOC_PLAN_SWEEP = 4
} ooc_planner;

/* Task orders over the grid of C blocks (i: block row, j: block column) and
 * K panels p.  COLS is the paper's order (column by column, Fig. 2).
 * COLS_P keeps a whole block column of C resident and walks K panels outside
 * the block rows, so each B panel is loaded once; ROWS_P is its transpose.
 * With group g > 0 the _P orders walk groups of g blocks of the column (row)
 * K panel by K panel.  The _PS orders are the _P orders with every other
 * column (row) walked backwards: groups, K panels and blocks in reverse, so
 * it starts with the panels the previous column (row) ended with, which are
 * still resident (a C block then accumulates its K panels in descending
 * order). */
typedef enum {
  OOC_ORDER_COLS = 0,    /* for j, for i, for p */
  OOC_ORDER_ROWS = 1,    /* for i, for j, for p */
  OOC_ORDER_COLS_P = 2,  /* for j, for p, for i */
  OOC_ORDER_ROWS_P = 3,  /* for i, for p, for j */
  OOC_ORDER_COLS_PS = 4, /* COLS_P, odd block columns backwards */
  OOC_ORDER_ROWS_PS = 5  /* ROWS_P, odd block rows backwards */
} ooc_order;

/* A tiling and pipeline plan. */
typedef struct {
  int64_t mb, nb, kb;   /* C block rows and columns; K panel length (kb == K: no K split) */
  int32_t order;        /* ooc_order */
  int32_t nbuf_a;       /* device buffers for A panels (mb x kb) */
  int32_t nbuf_b;       /* device buffers for B panels (kb x nb) */
  int32_t nbuf_c;       /* device buffers for C blocks (mb x nb) */
  int32_t nstreams;     /* 1: one stream; 2: the paper's two streams used round robin by
                           block parity; 3: one stream each for H2D, kernels and D2H */
  int32_t precision;    /* ooc_precision */
  int32_t slices;       /* split slice count s (1..8); ignored for FP64 */
  int32_t nbuf_d;       /* 0: each C block is loaded into its own buffer before its first K panel.
                           >0 (beta != 0 only): C blocks start from zero and the initial C of a block
                           is staged in one of nbuf_d extra buffers (mb x nb) and added, scaled by
                           beta, at one K-panel step chosen to spread these copies over time */
  int32_t group;        /* orders COLS_P and ROWS_P: C blocks per group; the blocks of a group are
                           walked K panel by K panel, groups one after another (0: the whole block
                           column or row is one group); ignored by the other orders */
} ooc_plan_t;

/* Options; a NULL pointer means all defaults (zero-initialised struct). */
typedef struct {
  int32_t device;       /* HIP device ordinal (default 0) */
  int32_t planner;      /* ooc_planner (default AUTO) */
  int32_t precision;    /* ooc_precision (default FP64) */
  int32_t slices;       /* split slices (0: 6) */
  int32_t nstreams;     /* restrict candidate plans to this stream count (0: any) */
  int32_t profile;      /* 1: time every operation with HIP events (fills the busy times) */
  void* arena;          /* optional caller-owned device memory used instead of allocating */
  size_t arena_bytes;   /* its size; must be >= the plan's footprint */
  double* timeline;     /* optional (profile == 1): receives start and end of op x, in seconds
                           from the first op's start, at timeline[2x] and timeline[2x+1] */
  int64_t timeline_cap; /* number of ops timeline can hold */
  void* streams[3];     /* optional caller-owned hipStream_t (borrowed, never destroyed): pipeline
                           stream x runs on streams[x] when it is not NULL, else on a stream the
                           library owns.  The call still returns only after every stream it used
                           has drained; work the caller queued on a borrowed stream before the call
                           runs before the pipeline's first operation on that stream */
  int32_t release_arena;/* 1: free the device arena before returning (every call allocates anew);
                           0 (default): keep it cached for the next call on the device until
                           ooc_release() -- saves the allocation on repeated calls */
} ooc_opts;

/* Outcome of a call. */
typedef struct {
  ooc_plan_t plan;
  double t_total_s;      /* host wall time from entry to return */
  double t_pipeline_s;   /* first operation issued to last one complete */
  double t_h2d_busy_s;   /* sum of H2D copy durations (profile == 1) */
  double t_d2h_busy_s;   /* sum of D2H copy durations (profile == 1) */
  double t_kernel_busy_s;/* sum of kernel durations (profile == 1) */
  double t_predicted_s;  /* the cost model's prediction for the plan */
  double flops;          /* 2*M*N*K */
  uint64_t bytes_h2d, bytes_d2h;
  uint64_t arena_bytes;  /* device bytes used by the call (<= budget) */
  int64_t ops, tasks, kernels;
  int64_t blocks_done;   /* C blocks completely written back to the host */
  double t_plan_s;       /* host time from entry until the operation list was ready: choosing the plan
                            (unless given), its layout, the schedule and the cost model's prediction */
  double overlap;        /* (profile == 1) fraction of the time some host-device copy was in flight
                            during which a tile kernel ran too: the share of the transfers hidden
                            behind computation (0 without profiling) */
  double t_mma_busy_s;   /* (profile == 1) sum of the durations of the matrix-core kernels alone: the
                            FP64 tile kernels, or the slice-product kernels of split plans without
                            their slicing kernels */
  int64_t mma_launches;  /* (profile == 1) number of those kernel launches */
} ooc_stats;

/* ---- the out-of-core product ---------------------------------------------------- */

/* C = alpha*A*B + beta*C through a device budget of budget_bytes.
 * All device memory the call uses (tile buffers and split workspace) is at most
 * budget_bytes; it is allocated for the call (or taken from opts->arena) and
 * cached for the next call on the device until ooc_release(), or freed before
 * returning with opts->release_arena = 1.
 * Errors: OOC_ERR_ARG (negative sizes, ld too small, NULL operand with a
 * nonzero extent), OOC_ERR_BUDGET (nothing fits), OOC_ERR_DEVICE_MEM,
 * OOC_ERR_NOT_PINNED, OOC_ERR_NO_DEVICE, OOC_ERR_HIP.
 * OOC_LOG=1 in the environment prints one line per call on stderr (problem,
 * plan, times, status).
 * Test hooks read from the environment at each call: OOC_FAIL_AT=n stops
 * issuing at operation n (OOC_ERR_INJECTED after draining the streams);
 * OOC_STRESS_SEED=s fills the device buffers with NaN first and, chosen by
 * the seed, enqueues a wait of up to OOC_STRESS_US microseconds (default 300,
 * at most 5000) before a third of the operations on their streams. */
ooc_status ooc_gemm(int64_t M, int64_t N, int64_t K, double alpha,
                    const double* A, int64_t lda, const double* B, int64_t ldb,
                    double beta, double* C, int64_t ldc, size_t budget_bytes,
                    const ooc_opts* opts, ooc_stats* stats);

/* The product with a transposed B and an optional triangular result:
 *     C = alpha * A * op(B) + beta * C
 * op(B) = B (transb == 0; B is K x N, ldb >= N) or B^T (transb == 1; B is
 * N x K, ldb >= K: the symmetric rank-k update and the Cholesky updates use
 * op(B) = A^T).  lower == 1 computes only the elements C_ij with i >= j (FP64
 * precision only, OOC_ERR_ARG otherwise): C blocks wholly above the diagonal
 * are skipped, and the elements with i < j of blocks that straddle it are
 * copied to the device and back unchanged (never read by the arithmetic, so
 * NaN there stays NaN).  Everything else as for ooc_gemm. */
ooc_status ooc_gemm_ex(int32_t transb, int32_t lower, int64_t M, int64_t N, int64_t K, double alpha,
                       const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                       int64_t ldc, size_t budget_bytes, const ooc_opts* opts, ooc_stats* stats);

/* Choose a plan for the problem and budget (host only, no device access). */
ooc_status ooc_plan(int64_t M, int64_t N, int64_t K, double beta, size_t budget_bytes,
                    const ooc_opts* opts, ooc_plan_t* out);

/* The product with a caller-given plan; fails with OOC_ERR_BUDGET if its
 * footprint exceeds budget_bytes and OOC_ERR_ARG if the plan is malformed. */
ooc_status ooc_gemm_planned(int64_t M, int64_t N, int64_t K, double alpha,
                            const double* A, int64_t lda, const double* B, int64_t ldb,
                            double beta, double* C, int64_t ldc, size_t budget_bytes,
                            const ooc_plan_t* plan, const ooc_opts* opts, ooc_stats* stats);

/* Device bytes a plan needs (tile buffers, alignment, split workspace). */
ooc_status ooc_plan_footprint(int64_t M, int64_t N, int64_t K, double beta,
                              const ooc_plan_t* plan, uint64_t* bytes);

/* The paper's partitioner alone: h horizontal A slices and w vertical B slices
 * (Section V; fewest w, then fewest h, with footprint 2*mb*K + K*nb + 2*mb*nb
 * elements, or M*K + K*N + M*N for a single block). OOC_ERR_BUDGET if none fits. */
ooc_status ooc_partition(int64_t M, int64_t N, int64_t K, size_t budget_bytes,
                         int64_t* h, int64_t* w);

/* All candidate plans the MODEL/MLP planners consider (host only).  Writes up
 * to cap plans and their modelled times; *n receives the total count
 * (OOC_ERR_CAPACITY if it exceeds cap). */
ooc_status ooc_plan_candidates(int64_t M, int64_t N, int64_t K, double beta, size_t budget_bytes,
                               const ooc_opts* opts, ooc_plan_t* plans, double* model_s,
                               int64_t cap, int64_t* n);

/* The analytic cost model's simulated time of a plan (host only). */
ooc_status ooc_plan_predict(int64_t M, int64_t N, int64_t K, double beta, const ooc_plan_t* plan,
                            double* seconds);

/* The cost model's timeline of the plan's operation list (host only): start and
 * end of op x at times[2x], times[2x+1] (seconds).  *nops receives the op
 * count; OOC_ERR_CAPACITY if it exceeds cap. */
ooc_status ooc_plan_simulate(int64_t M, int64_t N, int64_t K, double beta, const ooc_plan_t* plan,
                             double* times, int64_t cap, int64_t* nops);

/* ---- the operation list (what the HIP backend issues), for inspection ---------- */

typedef enum {
  OOC_OP_H2D = 0,        /* host submatrix -> device buffer (2-D pitched copy) */
  OOC_OP_D2H = 1,        /* device buffer -> host submatrix */
  OOC_OP_GEMM = 2,       /* FP64 tile product c = alpha*a*b + beta*c + gamma*d on device buffers */
  OOC_OP_SPLIT_GEMM = 3, /* the same product from BF16 or INT8 slices (the plan's precision): slices
                            and exponents of the A and B panels are written to the workspace
                            (off_w, len_w), then multiplied */
  OOC_OP_POTRF = 4,      /* Cholesky factorisation in place of the rows x rows block at off_c (ld_c):
                            its lower triangle becomes L with block = L L^T, the strict upper triangle
                            is untouched; a pivot that is not positive stores k0 + its column + 1 in
                            the double at off_w if that is still 0 (later columns unspecified) */
  OOC_OP_TRSM = 5        /* X <- X L^{-T}, or X <- X L^{-1} with flag OOC_OPF_BACK: X is rows x cols
                            at off_c (ld_c), L the cols x cols lower triangle at off_a (ld_a) */
} ooc_op_kind;

#define OOC_MAX_WAITS 6

/* Flags of product ops.  TRANSB: the B panel holds B^T (n x k, leading
 * dimension ld_b >= k).  LOWER: only elements of c on or below the diagonal
 * of the whole result are written, element (r, c) of the block at
 * (row0, col0) when row0 + r >= col0 + c; the others are neither read nor
 * written (FP64 products only). */
#define OOC_OPF_TRANSB 1
#define OOC_OPF_LOWER 2
/* Flag of TRSM ops: back substitution X <- X L^{-1} instead of X <- X L^{-T}. */
#define OOC_OPF_BACK 4
/* Flags of SPLIT_GEMM ops: the slices of the A (B) panel are still in the
 * workspace, left there by the previous SPLIT_GEMM op of the list, so this op
 * skips slicing that operand.  Allowed when that op had the same extents
 * (rows, cols, k <= 8192), workspace, TRANSB flag and A (B) panel offset and
 * leading dimension, and read the same data there: the caller vouches for the
 * data, and orders the two ops (ooc_check_ops finds unordered uses of the
 * workspace). */
#define OOC_OPF_REUSE_A 8
#define OOC_OPF_REUSE_B 16

typedef struct {
  int32_t kind;               /* ooc_op_kind */
  int32_t stream;             /* stream index, 0 .. nstreams-1 */
  int32_t task;               /* index of the tile task this op serves */
  int32_t nwait;              /* entries used in wait[] */
  int32_t wait[OOC_MAX_WAITS];/* earlier ops (other streams) that must complete first */
  int32_t mat;                /* copies: host matrix index (ooc_gemm: 0 = A, 1 = B, 2 = C) */
  int32_t slot;               /* device buffer index within its operand's pool */
  int32_t flags;              /* GEMM: OOC_OPF_TRANSB, OOC_OPF_LOWER; SPLIT_GEMM: OOC_OPF_TRANSB,
                                 OOC_OPF_REUSE_A, OOC_OPF_REUSE_B; TRSM: OOC_OPF_BACK */
  int32_t reserved;           /* 0 */
  int64_t row0, col0;         /* copies: host submatrix origin; GEMM: C block origin (i0, j0) */
  int64_t rows, cols;         /* copies: submatrix extent; GEMM: m, n */
  int64_t k0, k;              /* GEMM: K panel origin and length */
  int64_t off_a, ld_a;        /* GEMM: arena element offset / leading dim of the A panel */
  int64_t off_b, ld_b;        /* GEMM: same for the B panel */
  int64_t off_c, ld_c;        /* GEMM: C block; copies: the device side of the copy */
  int64_t off_d, ld_d;        /* GEMM: staged initial C block added with weight gamma */
  int64_t off_w, len_w;       /* split ops: workspace element offset and length */
  double alpha, beta, gamma;  /* GEMM: effective scalars of this panel step (beta == 0: c not
                                 read; gamma == 0: d not read) */
} ooc_op;

/* The operation list a plan produces (host only).  Writes up to cap ops;
 * *nops receives the count and *arena_bytes the arena size the offsets assume. */
ooc_status ooc_schedule(int64_t M, int64_t N, int64_t K, double alpha, double beta,
                        const ooc_plan_t* plan, ooc_op* ops, int64_t cap, int64_t* nops,
                        uint64_t* arena_bytes);

/* ooc_schedule for the ooc_gemm_ex forms (host only). */
ooc_status ooc_schedule_ex(int32_t transb, int32_t lower, int64_t M, int64_t N, int64_t K, double alpha,
                           double beta, const ooc_plan_t* plan, ooc_op* ops, int64_t cap, int64_t* nops,
                           uint64_t* arena_bytes);

/* ---- the general pipeline: operation lists on the HIP backend --------------------
 * The product is planned (ooc_plan), turned into an operation list
 * (ooc_schedule) and run by an executor.  The executor is open to other
 * out-of-core algorithms built from the same operations -- copies between
 * host submatrices and a device arena, and the kernels of ooc_op_kind -- the
 * paper's host-controls-device model (Sections III-IV: the host issues
 * asynchronous copies and kernels on streams, ordered by events) as an
 * interface.  ooc_potrf is built this way. */
typedef struct {
  double* ptr;            /* page-locked host memory, row-major */
  int64_t rows, cols, ld; /* ld >= cols (elements) */
} ooc_host_matrix;

/* Run ops[0 .. nops) on device opts->device.  Op x first waits for the ops
 * in its wait set (earlier ops only, any stream), then runs on stream
 * op.stream (0, 1 or 2; a stream runs its ops in list order).  Copies move
 * the rows x cols submatrix at (row0, col0) of mats[op.mat] to or from the
 * arena at element off_c with leading dimension ld_c; kernels read and
 * write the arena as ooc_op_kind states.  The arena is arena_bytes of device
 * memory: opts->arena when given, else the device's cached arena; SPLIT_GEMM
 * ops use opts->precision and opts->slices.  Before anything is issued every
 * op is validated (kind, stream, waits, copies inside their host matrix,
 * every kernel operand inside the arena): OOC_ERR_ARG names the first
 * offender.  The ordering is the caller's: two ops that touch a common arena
 * element, one of them writing it, must be ordered by a stream or a chain of
 * waits (ooc_check_ops finds violations).  Returns after every stream has
 * drained; stats as for ooc_gemm (plan left zero). */
ooc_status ooc_run_ops(const ooc_op* ops, int64_t nops, const ooc_host_matrix* mats, int32_t nmats,
                       uint64_t arena_bytes, const ooc_opts* opts, ooc_stats* stats);

/* Ordering check of an operation list (host only): OOC_OK if every two ops
 * that touch a common arena element, one of them writing it, are ordered;
 * else OOC_ERR_ARG with *x > *y the first such pair.  OOC_ERR_CAPACITY above
 * 32768 ops (the check keeps an nops x nops bit matrix). */
ooc_status ooc_check_ops(const ooc_op* ops, int64_t nops, int64_t* x, int64_t* y);

/* ---- out-of-core level-3 routines built on the pipeline ---------------------------
 * The paper names level-3 routines and dense factorisations whose bulk of
 * work is the out-of-core product as the next step (Section VII). */

/* Symmetric rank-k update C = alpha * A * A^T + beta * C on the lower
 * triangle (i >= j) of the N x N matrix C (ldc >= N); A is N x K (lda >= K).
 * The strict upper triangle of C is left unchanged.  This is
 * ooc_gemm_ex(1, 1, N, N, K, alpha, A, lda, A, lda, beta, C, ldc, ...): the
 * blocks wholly above the diagonal are not computed. */
ooc_status ooc_syrk(int64_t N, int64_t K, double alpha, const double* A, int64_t lda, double beta, double* C,
                    int64_t ldc, size_t budget_bytes, const ooc_opts* opts, ooc_stats* stats);

/* Cholesky factorisation A = L L^T of the N x N symmetric positive definite
 * matrix A in place (row-major, lda >= N, page-locked): the lower triangle is
 * read and overwritten by L; the strict upper triangle is left unchanged.
 * Left-looking by block columns of b columns (the largest multiple of 64 up
 * to 8192 whose b x b block takes at most a quarter of the budget, the rest
 * holding two chunks of at least 256 rows): the
 * update of a block column by the columns to its left is one out-of-core
 * product (C = C - A B^T on the lower triangle, ooc_gemm_ex); its diagonal
 * block is factored on the device and the rows below are solved against it
 * chunk by chunk (an operation list of POTRF and TRSM ops on the executor).
 * Every quotient is a true division: an integer SPD matrix with an integer
 * factor gets it exactly.  *info = 0 on success; OOC_ERR_NOT_SPD with
 * *info = j + 1 for the first column j whose pivot is not positive (the
 * block columns before j's hold L, the rest of the lower triangle is
 * unspecified).  The products run in FP64 whatever opts->precision says.
 * stats: totals over the calls (flops = N^3/3 + N^2/2 + N/6, bytes, times;
 * blocks_done = block columns finished). */
ooc_status ooc_potrf(int64_t N, double* A, int64_t lda, size_t budget_bytes, const ooc_opts* opts, int64_t* info,
                     ooc_stats* stats);

/* Triangular solve Y L^T = X out of core: X (M x N, row-major, ldx >= N,
 * page-locked) is overwritten by Y = X L^{-T} for the lower-triangular N x N
 * matrix L (row-major, ldl >= N, page-locked; only its lower triangle is
 * read, its diagonal must be nonzero: a zero divides into Inf or NaN).  In
 * column-major terms this is the forward substitution L Y' = X' for the
 * columns of X' = X^T, the solve with the factor of ooc_potrf.  Left-looking
 * by block columns of b columns (the panel rule of ooc_potrf): the update of
 * a block column of X by the solved columns to its left is one out-of-core
 * product (ooc_gemm_ex with a transposed B), then the block column is solved
 * against L's diagonal block on the device, chunk by chunk (TRSM ops on the
 * executor).  Every quotient is a true division: integer data with an
 * integer solution gets it exactly.  FP64 whatever opts->precision says.
 * stats: totals (flops = M N^2, bytes, times; blocks_done = block columns). */
ooc_status ooc_trsm(int64_t M, int64_t N, const double* L, int64_t ldl, double* X, int64_t ldx, size_t budget_bytes,
                    const ooc_opts* opts, ooc_stats* stats);

/* ooc_trsm with the transposition chosen: trans = 1 solves Y L^T = X (as
 * ooc_trsm, forward substitution), trans = 0 solves Y L = X (X <- X L^{-1},
 * back substitution: in column-major terms L^T Y' = X', the second solve with
 * the factor of ooc_potrf), walking the block columns from the last one, each
 * updated by the solved columns to its right (an out-of-core product without
 * transposition).  Other arguments, errors and stats as for ooc_trsm. */
ooc_status ooc_trsm_ex(int32_t trans, int64_t M, int64_t N, const double* L, int64_t ldl, double* X, int64_t ldx,
                       size_t budget_bytes, const ooc_opts* opts, ooc_stats* stats);

/* Solve with the Cholesky factor out of core: B (M x N, row-major, ldb >= N,
 * page-locked) is overwritten by X with X A = B for A = L L^T (L from
 * ooc_potrf, N x N lower-triangular, ldl >= N): each row of B is a
 * right-hand side b of A x = b (A symmetric).  Two triangular solves: Y L^T =
 * B, then X L = Y (ooc_trsm_ex with trans 1, then 0).  stats: totals (flops =
 * 2 M N^2). */
ooc_status ooc_potrs(int64_t M, int64_t N, const double* L, int64_t ldl, double* B, int64_t ldb, size_t budget_bytes,
                     const ooc_opts* opts, ooc_stats* stats);

/* ---- accumulation sessions: repeated invocation ----------------------------------
 * The paper's MMOOC can serve as the local step of an outer algorithm (SUMMA or
 * HSUMMA, Section V: the step/nsteps logic of Fig. 2): over steps s = 0..S-1
 * it adds alpha_s * A_s * B_s to C, reading C at the first step only and
 * writing back the blocks still on the device after the last step.  A session
 * computes
 *     C = beta * C_in + sum over steps of alpha_s * A_s * B_s
 * (A_s M x K_s, B_s K_s x N, row-major, page-locked; K_s may differ per
 * step), each step rounded as C = alpha_s * A_s B_s + C.  The first R rows of
 * C (ooc_accum_resident_rows: all of C when it takes at most half the budget,
 * else as many rows as fit in half, a multiple of 128 from 128 on) stay on the
 * device for the whole session: loaded once at ooc_accum_begin (if beta != 0),
 * updated in place by every step and written back once by ooc_accum_end.
 * The remaining rows are streamed through the rest of the budget by the
 * ordinary pipeline at every step (read and written back).  The session
 * allocates budget_bytes of device memory at begin and frees it at end.
 * Host C must stay valid and untouched by the caller until ooc_accum_end;
 * A_s and B_s only during their step.  Rows >= R of C hold the running sum
 * after each step; rows < R only after ooc_accum_end.  Steps and end are
 * synchronous.  On an error inside a step C is unspecified; the session must
 * still be ended (which frees it). */
typedef struct ooc_accum_s* ooc_accum;

/* Open a session for C (M x N, page-locked, leading dimension ldc >= N).
 * Errors as ooc_gemm (OOC_ERR_DEVICE_MEM if budget_bytes exceeds the free
 * device memory).  opts as for ooc_gemm (the timeline and arena are ignored). */
ooc_status ooc_accum_begin(int64_t M, int64_t N, double beta, double* C, int64_t ldc, size_t budget_bytes,
                           const ooc_opts* opts, ooc_accum* out);

/* One step: C += alpha * A * B with A (M x K, lda >= K) and B (K x N, ldb >= N).
 * alpha == 0 or K == 0 leave C unchanged (beta is applied at the first step). */
ooc_status ooc_accum_step(ooc_accum acc, int64_t K, double alpha, const double* A, int64_t lda,
                          const double* B, int64_t ldb, ooc_stats* stats);

/* Write the resident rows back and free the session (also after an error).
 * A session without steps returns C = beta * C_in. */
ooc_status ooc_accum_end(ooc_accum acc, ooc_stats* stats);

/* Rows of C a session of this size keeps on the device (host only). */
ooc_status ooc_accum_resident_rows(int64_t M, int64_t N, size_t budget_bytes, int64_t* rows);

/* The operation lists of one session step (host only): part 0 updates the
 * resident rows [0, R) in place (C at arena element 0, leading dimension N;
 * no C copies), part 1 streams rows [R, M) through buffers placed after
 * them (its host rows count from row R).  beta_eff is beta at the first
 * step and 1 afterwards.  A part with no rows returns *nops = 0. */
ooc_status ooc_accum_schedule(int64_t M, int64_t N, int64_t K, double alpha, double beta_eff, size_t budget_bytes,
                              const ooc_opts* opts, int32_t part, ooc_op* ops, int64_t cap, int64_t* nops,
                              uint64_t* arena_bytes);

/* ---- memory helpers ----------------------------------------------------------- */

ooc_status ooc_host_alloc(void** ptr, size_t bytes);  /* page-locked host memory */
ooc_status ooc_host_free(void* ptr);
ooc_status ooc_device_alloc(int32_t device, void** ptr, size_t bytes);
ooc_status ooc_device_free(int32_t device, void* ptr);
/* Synchronous copies between host and device memory (for tests and tools). */
ooc_status ooc_copy_to_device(int32_t device, void* dst, const void* src, size_t bytes);
ooc_status ooc_copy_to_host(int32_t device, void* dst, const void* src, size_t bytes);

/* Device-to-device copy with a plain streaming kernel (16-byte aligned pointers,
 * bytes a multiple of 16); a reference workload for hardware traffic counters. */
ooc_status ooc_device_copy(int32_t device, void* dst, const void* src, size_t bytes);

/* Free the device buffers, streams and events cached for a device (-1: all). */
ooc_status ooc_release(int32_t device);

/* ---- in-core tile kernels on device memory (building blocks, for tests) ------- */

/* C = alpha*A*B + beta*C on device pointers with the FP64 MFMA tile kernel (the
 * paper's DGEMM stage, Section V).  Row-major, lda >= k, ldb >= n, ldc >= n.
 * If ms_out is not NULL the kernel is timed with HIP events (milliseconds). */
ooc_status ooc_dgemm_device(int32_t device, int64_t m, int64_t n, int64_t k, double alpha,
                            const double* A, int64_t lda, const double* B, int64_t ldb,
                            double beta, double* C, int64_t ldc, int32_t reps, double* ms_out);

/* The split-BF16 tile product on device pointers (s = slices, 1..8): the
 * error-free slicing of Ozaki et al. (2012) on BF16 matrix cores with exact
 * FP32 chunk sums (see ooc_precision).  Row-major; C = alpha*A*B + beta*C
 * rounded as alpha*S + beta*C with separate roundings.  The call allocates
 * and frees its own workspace.  ms_out as for ooc_dgemm_device. */
ooc_status ooc_split_gemm_device(int32_t device, int64_t m, int64_t n, int64_t k, int32_t s, double alpha,
                                 const double* A, int64_t lda, const double* B, int64_t ldb,
                                 double beta, double* C, int64_t ldc, int32_t reps, double* ms_out);

/* For callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid allocation): ooc_split_gemm_device
 * without any allocation.  The slice workspace is a static device array of
 * OOC_NOALLOC_SCRATCH_BYTES per device, held by every device the library runs
 * on until the process ends; the call is OOC_ERR_CAPACITY when the workspace
 * of (m, n, min(k, 8192), s) exceeds it (m = n = k = 1024 at s = 8 needs
 * 40 MiB).  A, B and C are device pointers as for ooc_split_gemm_device, the
 * result is the same bit for bit.  The kernels are enqueued on `stream` (a
 * hipStream_t; NULL: the null stream) and the call returns without waiting:
 * C is complete when that stream's work is.  Every call on a device shares
 * its one scratch array, so calls whose work overlaps in time on one device
 * (on different streams, or from several host threads) race and give
 * unspecified results; calls queued on one stream are safe.  Errors:
 * OOC_ERR_ARG as ooc_split_gemm_device, OOC_ERR_CAPACITY, OOC_ERR_NO_DEVICE,
 * OOC_ERR_HIP (launch failure). */
#define OOC_NOALLOC_SCRATCH_BYTES (64u << 20)
ooc_status ooc_split_gemm_device_noalloc(int32_t device, int64_t m, int64_t n, int64_t k, int32_t s, double alpha,
                                         const double* A, int64_t lda, const double* B, int64_t ldb,
                                         double beta, double* C, int64_t ldc, void* stream);

/* The same with s INT8 slices of 7 bits (OOC_SPLIT_INT8) on INT8 matrix cores
 * with exact INT32 sums; arguments, rounding and errors as above. */
ooc_status ooc_split_int8_gemm_device(int32_t device, int64_t m, int64_t n, int64_t k, int32_t s, double alpha,
                                      const double* A, int64_t lda, const double* B, int64_t ldb,
                                      double beta, double* C, int64_t ldc, int32_t reps, double* ms_out);

/* Tile width of the INT8 slice products of an m x n block on a device with
 * `cus` compute units: 1 if they run on 256 x 256 tiles (half the plane bytes
 * per product of 256 x 128 ones, about 1.9 times the time per tile), when
 * those tiles' waves over the CUs end sooner, else 0; -1 for m, n or cus
 * below 1.  Host only (the library's own choice; for reports). */
int32_t ooc_split_int8_wide_tiles(int64_t m, int64_t n, int32_t cus);

/* ---- the learned planner ------------------------------------------------------ */
/* A small regression network predicts the log run time of a candidate plan
 * from its features; OOC_PLAN_MLP takes the candidate with the smallest
 * prediction.  (The paper fixes its plan by rule, Section V, and observes that
 * the best stream count depends on the device, Section VI.)  Network: x (d) ->
 * tanh(x W1 + b1) (H) -> tanh(. W2 + b2) (H) -> . W3 + b3, FP32 on the GPU;
 * parameters are one flat float array W1 (d x H, row-major), b1 (H), W2 (H x H),
 * b2 (H), W3 (H), b3 (1).  Host arrays throughout; device work uses `device`. */

#define OOC_MLP_FEATURES 19

/* Features of candidate plans: X_out receives n x OOC_MLP_FEATURES floats
 * (log2 of M, N, K+1, budget, mb, nb, kb+1; order one-hot (4; COLS_PS and
 * ROWS_PS set the COLS_P and ROWS_P entries); nbuf_a, nbuf_b,
 * log2 nbuf_c, nbuf_d, nstreams; log2 of the cost model's time and of the H2D
 * bytes; split slices or 0).  Host only. */
ooc_status ooc_mlp_features(int64_t M, int64_t N, int64_t K, double beta, size_t budget_bytes,
                            const ooc_plan_t* plans, int64_t n, float* X_out);

/* Network forward pass for n inputs (X: n x d), y_out: n predictions. */
ooc_status ooc_mlp_forward(int32_t device, int32_t d, int32_t hidden, const float* params, const float* X,
                           int64_t n, float* y_out);

/* Objective = mean squared error of the predictions against t plus
 * (weight_decay/2) times the sum of squares of the weight matrices W1, W2, W3
 * (biases unpenalised; weight_decay >= 0), and its gradient with respect to
 * every parameter (grad_out: same layout as params). */
ooc_status ooc_mlp_grad(int32_t device, int32_t d, int32_t hidden, const float* params, const float* X,
                        const float* t, int64_t n, float weight_decay, float* grad_out, float* loss_out);

/* One Adam step (bias-corrected; step counts from 1) on count parameters;
 * params, m and v are updated in place. */
ooc_status ooc_mlp_adam(int32_t device, int64_t count, float* params, const float* grad, float* m, float* v,
                        int32_t step, float lr, float beta1, float beta2, float eps);

/* epochs of full-batch Adam (lr, betas 0.9/0.999, eps 1e-8) on the GPU on the
 * objective of ooc_mlp_grad, params updated in place; loss_hist (optional)
 * receives the objective before each step. */
ooc_status ooc_mlp_train(int32_t device, int32_t d, int32_t hidden, float* params, const float* X,
                         const float* t, int64_t n, int32_t epochs, float lr, float weight_decay,
                         float* loss_hist);

/* Train the planner network from measured timings (seconds) of candidate
 * plans whose features are X (n x OOC_MLP_FEATURES): features and log-times
 * are standardised, weights drawn from seed, then ooc_mlp_train; the result
 * becomes the network OOC_PLAN_MLP uses. */
ooc_status ooc_mlp_fit(int32_t device, const float* X, const float* y_seconds, int64_t n, int32_t hidden,
                       int32_t epochs, float lr, float weight_decay, uint64_t seed, float* loss_hist);

/* Save / load the planner network (text file: sizes, standardisation, weights). */
ooc_status ooc_mlp_save(const char* path);
ooc_status ooc_mlp_load(const char* path);
int32_t ooc_mlp_loaded(void);  /* 1 if a planner network is loaded */

/* The planner network's predicted run time (seconds) of each candidate plan. */
ooc_status ooc_mlp_predict(int64_t M, int64_t N, int64_t K, double beta, size_t budget_bytes,
                           const ooc_plan_t* plans, int64_t n, double* seconds_out);

/* ---- messages and version ----------------------------------------------------- */

const char* ooc_last_error(void);   /* message of the calling thread's last error */
const char* ooc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* OOC_H */
