/*
 * wsmul.h -- exact Strassen-Winograd matrix products over Z/pZ on MI355X,
 * run under the memory schedules of Boyer, Dumas, Pernet and Zhou,
 * "Memory efficient scheduling of Strassen-Winograd's matrix multiplication
 * algorithm" (ISSAC 2009).
 *
 * One operation sits behind this header (Section 3.2):
 *
 *     C <- (alpha * A * B + beta * C) mod p
 *
 * with A m x k, B k x n, C m x n, every entry a canonical residue in [0, p).
 * Winograd's 2x2 recursion (Section 2: 8 pre-additions, 7 products,
 * 7 post-additions) is applied `levels` times; below that the base case is a
 * classical product on the GPU's matrix cores.  The schedule selects where
 * every intermediate block lives (the "loc." column of the paper's tables).
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Matrices are HIP device pointers, row-major, with leading dimensions
 *   lda >= k, ldb >= n, ldc >= n (in elements).  Storage is binary64 holding
 *   integers (WS_F64) or int64 (WS_I64).  The caller owns A, B, C and any
 *   workspace it attaches; the library frees none of them.
 * - Execution is asynchronous on the stream given in ws_args (or the one set
 *   with wsmul_set_stream; NULL means the null stream).  A return of WS_OK
 *   means the work was enqueued.
 * - Errors are status codes; nothing is thrown across this boundary.  All
 *   argument checks run before any launch, so WS_EINVAL, WS_ESHAPE,
 *   WS_EMODULUS and WS_ESCHEDULE leave A, B and C untouched.  After WS_EHIP
 *   the contents of C (and of A, B for overwriting schedules) are
 *   unspecified, and memory the call allocated is released (stream-ordered)
 *   all the same.  wsmul_last_error() returns a thread-local message.  For
 *   tests of that path, the environment variable WSMUL_FAULT_AT=i makes a
 *   single-product call stop before launching its operation i and return
 *   WS_EHIP (nothing is launched when i = 0).
 * - Read-only schedules leave A and B bitwise unchanged.  WS_OVERWRITE (and
 *   the sub-schedules that overwrite) leave A and/or B in a state that is a
 *   fixed function of the inputs and the schedule's tables.
 * - Calls on one stream are ordered; two concurrent calls on different
 *   streams must not share a workspace.
 */
#ifndef WSMUL_H
#define WSMUL_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define WSMUL_API __attribute__((visibility("default")))
#else
#define WSMUL_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WS_OK = 0,
    WS_EINVAL = 1,     /* bad pointer, negative size, bad leading dimension */
    WS_ESHAPE = 2,     /* shape not supported by the chosen schedule       */
    WS_EMODULUS = 3,   /* p outside [2, 2^24) or beyond the base's bound   */
    WS_ERANGE = 4,     /* WS_FLAG_CHECK: an entry outside [0, p)           */
    WS_ESCHEDULE = 5,  /* unknown schedule, or beta != 0 where not allowed */
    WS_ENOMEM = 6,     /* attached workspace too small / allocation failed */
    WS_EHIP = 7        /* a HIP runtime call failed                        */
} ws_status;

typedef enum {
    WS_CLASSICAL = 0,        /* no Winograd level: one base product (comparator)    */
    WS_TWO_TEMP = 1,         /* beta == 0: Table 1; beta != 0: Table 9 (square)    */
    WS_OVERWRITE = 2,        /* square: Table 3 (beta == 0) or Table 6; otherwise
                                Algorithm 1 (beta == 0) or Table 8; destroys A and/or B */
    WS_READONLY_INPLACE = 3, /* Algorithm 2; beta must be 0; no temporary at all   */
    WS_HL_THREE_TEMP = 4,    /* Table 2 (three temporaries, any beta)              */
    WS_AUTO = 5,             /* schedule, depth and base chosen by the autotuner   */
    WS_OVR = 6,              /* Table 5: C = A*B, one temporary, destroys B        */
    WS_ACCR = 7,             /* Table 7: two temporaries, destroys B (square)      */
    WS_BLOCKED = 8,          /* Section 7.2 over Table 2: C in t x t blocks, see below */
    WS_BLOCKED_ACC = 9,      /* Section 7.2 over Table 9 (m == k == n, t | n)      */
    WS_OVL = 10,             /* Table 4: C = A*B, one temporary, destroys A (square) */
    WS_ACR = 11,             /* Table 8: any even shape, two temporaries, destroys B */
    WS_IPMM_ACC = 12,        /* Algorithm 2 with Table 9 for the accumulating chunks
                                (end of Section 7.1; beta == 0, k >= n/2)          */
    WS_ROWS = 13             /* a schedule given as rows (wsmul_register_rows); its
                                id goes in ws_args.blocks; square shapes, any beta   */
} ws_schedule;

/*
 * The rectangular overwriting schedules (Section 5.3).  Table 8 takes any
 * m, k, n divisible by 2^levels; its temporaries are max(m/2, k/2) x n/2
 * and m/2 x k/2 per level (below 2n^2/3 when square).  Algorithm 1 (WS_OVERWRITE
 * with beta == 0 and a non-square shape) needs n = min(m, k, n) dividing m
 * and k, and n divisible by 2^levels; it cuts A, B, C into n x n squares and
 * uses no workspace at all: with m > n the first square of C by Table 1 with
 * its temporaries in the second, then the Table 4 products and Table 2
 * accumulations with their temporaries in the freed square A_11 (A is
 * destroyed, B kept); with m == n, Table 3 and then Table 6 calls with their
 * temporaries in the freed A_1 (A and B destroyed).
 */

/*
 * Blocked accumulation (Section 7.2).  A, B and C are cut along every
 * dimension into t = ws_args.blocks consecutive parts (n/t each when t
 * divides the dimension; otherwise ceil(n/t) rounded up to a multiple of
 * 2^levels, with a shorter last part).  Block C_ij accumulates the t products
 * A_il * B_lj in order of l, the first with beta and the others with 1, each
 * by one call of the base schedule with `levels` levels: Table 2 for
 * WS_BLOCKED (any shape), Table 9 for WS_BLOCKED_ACC (square blocks).  The
 * calls run one after the other and share one set of temporaries, so the
 * extra memory is that of a single call on an (n/t)-block: below (n/t)^2 for
 * Table 2 (n^2/4 at t = 2, n^2/9 at t = 3) and below 2(n/t)^2/3 for Table 9,
 * against n^2 and 2n^2/3 unblocked.  The arithmetic grows to
 * R_t(n) = t^3 W_acc(n/t) (Section 7.2).  A and B are read only; any beta.
 * blocks = 0 means t = 2; t lies in [1, 64].  The other schedules ignore
 * ws_args.blocks; wsmul_mod_p, wsmul_mod_p_i64 and wsmul_workspace_bytes use
 * t = 2 (wsmul_plan_info reports any t).
 */

typedef enum { WS_F64 = 0, WS_I64 = 1 } ws_dtype;

typedef enum {
    WS_BASE_AUTO = 0,        /* library choice                                      */
    WS_BASE_F64_MFMA = 1,    /* binary64 matrix cores, delayed modular reduction    */
    WS_BASE_I8_LIMBS = 2     /* centred residues as signed 8-bit digits, int32 sums:
                                three digits (nine digit products), two (four) when
                                p <= 65536; p <= 16711423 and k <= 32768 */
} ws_base;

enum {
    WS_FLAG_CHECK = 1u << 0,   /* verify every entry lies in [0, p) first (WS_ERANGE) */
    WS_FLAG_NOFUSE = 1u << 1,  /* one launch per schedule row (no row fusion)         */
    WS_FLAG_TRACE = 1u << 2,   /* time every launch with events (wsmul_get_trace)     */
    WS_FLAG_SYNC = 1u << 3     /* wsmul_batched: wait for completion, report errors   */
};

/* Full argument block.  Zero lda/ldb/ldc mean dense (k, n, n). */
typedef struct ws_args {
    int64_t m, k, n, p;
    int64_t lda, ldb, ldc;
    int64_t alpha, beta;       /* any int64; reduced mod p                          */
    void *A, *B, *C;
    int32_t dtype;             /* ws_dtype                                           */
    int32_t schedule;          /* ws_schedule                                        */
    int32_t levels;            /* Winograd depth >= 0; -1 lets the autotuner choose  */
    int32_t base;              /* ws_base                                            */
    void *workspace;           /* NULL: use the attached one or allocate (stream-ordered) */
    uint64_t workspace_bytes;
    void *stream;              /* hipStream_t; NULL: the stream from wsmul_set_stream */
    uint32_t flags;
    uint32_t blocks;           /* WS_BLOCKED / WS_BLOCKED_ACC: t (0 means 2)        */
} ws_args;

/* Counters of the most recent call on this thread. */
typedef struct ws_stats {
    uint64_t workspace_bytes;      /* temporaries of the schedule (its extra memory)   */
    uint64_t peak_temp_bytes;      /* high-water mark of temporaries since reset       */
    uint64_t internal_alloc_bytes; /* bytes the library allocated itself for the call  */
    uint64_t add_launches;         /* fused addition launches                         */
    uint64_t gemm_launches;        /* base-product launches                           */
    uint64_t element_additions;    /* schedule addition rows x block elements          */
    uint64_t base_flops;           /* sum of 2*M*N*K over base products               */
    uint64_t rows;                 /* schedule rows before fusion                     */
    uint64_t levels;               /* Winograd depth actually used                    */
    int64_t schedule;              /* table actually run (see wsmul_schedule_name)    */
    int64_t base;                  /* base kind actually used                         */
    uint64_t scratch_bytes;        /* INT8 base: digit planes of the largest base product
                                      and of inputs read as planes (kernel scratch,
                                      not a schedule temporary)                        */
    uint64_t batch_phases;         /* batches: persistent launches (phases) issued     */
    uint64_t live_alloc_bytes;     /* device bytes still held by single-product calls of
                                      this process after the call returned (owned
                                      workspace and digit scratch not yet released);
                                      0 once every call has cleaned up, errors included */
} ws_stats;

/*
 * The spec call: binary64 storage, dense leading dimensions, default
 * stream and workspace.  C <- (alpha*A*B + beta*C) mod p with `levels`
 * Winograd levels under `schedule` (Section 3.2; schedules of Tables 1-9,
 * Algorithm 2 and the blocked accumulation of Section 7.2).
 */
WSMUL_API int wsmul_mod_p(int64_t m, int64_t k, int64_t n, int64_t p,
                void *A, void *B, void *C, int64_t alpha, int64_t beta,
                int schedule, int levels);

/* The same with int64 storage. */
WSMUL_API int wsmul_mod_p_i64(int64_t m, int64_t k, int64_t n, int64_t p,
                    void *A, void *B, void *C, int64_t alpha, int64_t beta,
                    int schedule, int levels);

/* Everything explicit (leading dimensions, dtype, base, stream, workspace). */
WSMUL_API int wsmul_mod_p_ex(const ws_args *args);

/*
 * Schedules given as data: the rows of one level of a memory schedule, as
 * the exhaustive search of Section 4 produces them, run by the library at
 * every level.  A row names blocks of the current call: 0-3 the quadrants
 * C11, C12, C21, C22 of its C; 4-7 A11, A12, A21, A22 and 8-11 B11..B22
 * (read only: never a destination); 12 .. 12+ntemps-1 its temporaries, each
 * the size of a quadrant of C (at most WS_ROW_MAX_TEMPS per call, one set per
 * call depth in the workspace).
 *   WS_ROW_ADD: dst <- cx*x + cy*y (an addition row; dst may be x or y);
 *   WS_ROW_MUL: dst <- sign*alpha*x*y, a recursive plain product (Table 1
 *               below this level, the classical base at the last);
 *   WS_ROW_ACC: dst <- sign*alpha*x*y + cs*dst, a recursive call of this same
 *               schedule with beta' = cs (the classical base at the last).
 * Coefficients cx, cy, cs are WS_COEF_* codes (1, -1, beta, -beta of the
 * call); sign is +1 or -1; a product's destination is neither operand.
 * The library checks the rows' form, not their algebra: a list that does not
 * compute alpha*A*B + beta*C gives a wrong C (the caller's search or replay
 * proves it does).  Square shapes only, n divisible by 2^levels.
 */
enum { WS_ROW_ADD = 0, WS_ROW_MUL = 1, WS_ROW_ACC = 2 };
enum { WS_COEF_ONE = 1, WS_COEF_MINUS_ONE = 2, WS_COEF_BETA = 3, WS_COEF_MINUS_BETA = 4 };
#define WS_ROW_MAX_TEMPS 4
#define WS_ROW_MAX_ROWS 64
typedef struct ws_row {
    int32_t op;
    int32_t dst, x, y;
    int32_t cx, cy;
    int32_t cs, sign;
} ws_row;

/* Check and register a row schedule (nrows rows, ntemps temporaries per
 * call); *id receives its id (equal rows give equal ids), to be passed as
 * ws_args.blocks with schedule WS_ROWS to any entry point (wsmul_mod_p_ex,
 * wsmul_plan_info, wsmul_batched, ...).  WS_EINVAL for malformed rows.
 * Registered schedules live until the process ends. */
WSMUL_API int wsmul_register_rows(const ws_row *rows, int nrows, int ntemps, int *id);

/* Register and run in one call: C <- (alpha*A*B + beta*C) mod p under the
 * row schedule with args->levels levels; the other fields of args as for
 * wsmul_mod_p_ex (args->schedule and args->blocks are ignored).  WS_EINVAL
 * for malformed rows, WS_ESHAPE for non-square shapes or n not divisible by
 * 2^levels; A and B are read only. */
WSMUL_API int wsmul_mod_p_rows(const ws_args *args, const ws_row *rows, int nrows, int ntemps);

/* Size of the static device scratch of wsmul_mod_p_noalloc, per GPU. */
#define WSMUL_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/*
 * wsmul_mod_p_ex for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The same product, plan and kernels, with the schedule's temporaries and the
 * 8-bit digit planes taken from one static device array of
 * WSMUL_NOALLOC_SCRATCH_BYTES bytes per GPU instead of an allocation: no
 * hipMalloc, hipFree or other allocating call, no synchronisation.  The first
 * call on a GPU looks the array's device address up, which makes the runtime
 * map it there (it then stays until the process ends): make that first call
 * outside any graph capture.  The caller passes A, B and C as for
 * wsmul_mod_p_ex; args->workspace must be NULL (the attached workspace of
 * wsmul_set_workspace is not used either), and WS_FLAG_CHECK / WS_FLAG_TRACE
 * are rejected (WS_EINVAL).  A product whose temporaries (rounded up to 256
 * bytes) plus digit planes exceed the scratch returns WS_ENOMEM before any
 * launch.  Every call on one GPU uses the same array, which keeps the last
 * call's contents (no kernel needs it cleared): calls that overlap in time on
 * one GPU, on any streams, race, so order them.
 */
WSMUL_API int wsmul_mod_p_noalloc(const ws_args *args);

/*
 * Bytes of temporaries the schedule needs (its "extra memory": Eq. (1) for
 * Table 1, Eq. (2) for Table 2, the bounds of Sections 5-6 for Tables 4-9,
 * zero for Table 3 and Algorithms 1 and 2, one (n/t)-block call for
 * Section 7.2 with t = 2), for dense binary64 or int64 storage.
 * Returns 0 for unsupported combinations (check wsmul_last_error()).
 */
WSMUL_API size_t wsmul_workspace_bytes(int64_t m, int64_t k, int64_t n, int dtype, int schedule,
                             int levels, int beta_nonzero);

/* Attach a caller-owned device workspace used when ws_args.workspace is NULL
 * (NULL/0 detaches).  The library never frees it.  Every such call uses the
 * same memory: calls on different streams that use it must not overlap in
 * time (order them, or pass each its own ws_args.workspace). */
WSMUL_API int wsmul_set_workspace(void *ptr, size_t bytes);

/* Default stream for calls whose ws_args.stream is NULL. */
WSMUL_API int wsmul_set_stream(void *stream);

/* Kernel time per class, summed over calls made with WS_FLAG_TRACE since the
 * last wsmul_reset_stats (events recorded on the call's stream around every
 * launch; a traced call waits for its own completion). */
typedef struct ws_trace {
    uint64_t add_launches, gemm_launches;
    double add_ms, gemm_ms;    /* gemm_ms: the product kernels only (digit splits apart) */
    double add_bytes;          /* algorithmic bytes of the addition launches: 8*(nin+nout)*elements */
    double gemm_flops;         /* 2*M*N*K of the base products */
    uint64_t split_launches;   /* digit base: operand-split kernels                      */
    double split_ms;
    double split_bytes;        /* 8 bytes read and 3 written per (padded) operand entry */
    uint64_t digit_adds;       /* digit base: addition groups reading or writing digit planes */
    uint64_t unsplit_operands; /* digit base: product operands read as planes, not split     */
} ws_trace;

WSMUL_API int wsmul_get_stats(ws_stats *out);
WSMUL_API int wsmul_get_trace(ws_trace *out);
WSMUL_API int wsmul_reset_stats(void);
WSMUL_API const char *wsmul_last_error(void);
WSMUL_API const char *wsmul_schedule_name(int table_id);
WSMUL_API const char *wsmul_version(void);

/* ------------------------------------------------------------------------
 * Batches.  Many independent products (binary64 storage and base), each with
 * its own shape, modulus and schedule (WS_AUTO and levels = -1 allowed).  A
 * product left at WS_BASE_AUTO runs on the binary64 base (the autotuner then
 * prices only that base); WS_BASE_I8_LIMBS or int64 storage is WS_EINVAL.
 * Operation j of every product forms phase j; the operations of a phase are
 * independent, so each phase is ONE persistent launch whose workgroups walk
 * its tasks -- one 64 x 64 output tile of a base product or one chunk of an
 * addition group -- round-robin, with no atomics and no waiting.  A batch of
 * single-operation products (classical products, which the autotuner picks
 * for sizes up to 2048) is therefore one launch.  All products' temporaries
 * are live at once: the call needs the sum of their workspaces (attached
 * with wsmul_set_workspace, else allocated stream-ordered), reported in
 * ws_stats.workspace_bytes.  The stream is probs[0].stream.  With
 * WS_FLAG_SYNC the call waits for completion and reports HIP errors.
 */
WSMUL_API int wsmul_batched(const ws_args *probs, int count, unsigned flags);

/* The same batch captured once into a hipGraph (one persistent launch per
 * phase) with its device state; *graph_exec receives an opaque handle.
 * Pointers in probs are baked in: replays recompute the same products from
 * whatever A, B, C then hold. */
WSMUL_API int wsmul_graph_capture(const ws_args *probs, int count, void **graph_exec);
WSMUL_API int wsmul_graph_launch(void *graph_exec, void *stream);
/* Wait for the stream; WS_EHIP if a HIP error was raised. */
WSMUL_API int wsmul_graph_check(void *graph_exec, void *stream);
WSMUL_API int wsmul_graph_destroy(void *graph_exec);

/* Choose schedule, Winograd depth and base for one product: every candidate
 * whose temporaries fit mem_budget is expanded into its fused plan and costed
 * with per-kernel rates measured on MI355X (base products by tile class and
 * base kind, addition groups by bytes moved, a floor per launch).  Fills
 * choice->schedule, ->levels, ->base and ->blocks (t of the blocked
 * accumulation, a candidate for accumulating products when the budget is
 * below the unblocked schedules' temporaries); other fields are left as
 * passed.  choice->beta says whether the product accumulates; a fixed
 * choice->schedule, ->levels, ->base or ->blocks is kept.
 * Decisions are cached in memory and, when WSMUL_TUNE_CACHE names a file, in
 * that file (one JSON object per line). */
WSMUL_API int wsmul_autotune(int64_t m, int64_t k, int64_t n, int64_t p, int dtype,
                             size_t mem_budget, ws_args *choice);

/* ------------------------------------------------------------------------
 * Tile choice of the binary64 base products.  By default a product's kernel
 * follows a fixed rule by shape (the larger tiles for the larger products).
 * wsmul_tune_tiles times every kernel kind that can take an m x k by k x n
 * product mod p on the current device (dense operands it allocates itself,
 * `reps` timed launches each after one warm-up) and remembers the fastest
 * for that (m, k, n, p, dtype) in this process; later base products of that
 * shape use it wherever their views allow.  times_us (NULL or WS_TILE_KINDS
 * entries) receives the average time per launch, -1 for kinds that cannot
 * take the shape; *best (may be NULL) the kind kept.  The call synchronises.
 * wsmul_set_tile pins a kind for a shape instead (-1 restores the rule);
 * wsmul_tune_plan tunes every distinct base-product shape of the plan of
 * `args` (binary64 base; no-op for the 8-bit digit base).  The choice never
 * changes a result: every kind computes the same exact product.
 */
enum {
    WS_TILE_BIG128 = 0,  /* 128 x 128, operands loaded straight into LDS, pipelined  */
    WS_TILE_LDS128 = 1,  /* 128 x 128, staged through registers (any shape)          */
    WS_TILE_DMA64 = 2,   /* 64 x 64, straight into LDS, inner dimension split by wave */
    WS_TILE_LDS64 = 3,   /* 64 x 64, staged through registers (any shape)            */
    WS_TILE_DMA32 = 4,   /* 32 x 32, straight into LDS, inner dimension split by wave */
    WS_TILE_SK32 = 5,    /* 32 x 32, from global memory, inner dimension split (any)  */
    WS_TILE_DMA16 = 6,   /* 16 x 16, straight into LDS, inner dimension split by wave */
    WS_TILE_KINDS = 7
};
WSMUL_API int wsmul_tune_tiles(int64_t m, int64_t k, int64_t n, int64_t p, int dtype, int reps,
                               int *best, double *times_us);
WSMUL_API int wsmul_set_tile(int64_t m, int64_t k, int64_t n, int64_t p, int dtype, int kind);
WSMUL_API int wsmul_tune_plan(const ws_args *args, int reps);

/* ------------------------------------------------------------------------
 * Plan introspection (host only, no GPU needed).
 *
 * A plan is the schedule expanded to `levels`: a list of operations on views
 * of A, B, C and the workspace.  Consecutive addition rows of a table are
 * fused into one operation when every view has the same shape and distinct
 * views do not overlap; addition rows right after a base product become its
 * epilogue under the same rule (plus: no epilogue output may overlap the
 * product's operands).
 */
#define WS_MAX_IN 8
#define WS_MAX_OUT 6

enum { WS_BUF_A = 0, WS_BUF_B = 1, WS_BUF_C = 2, WS_BUF_W = 3 };
enum { WS_OP_ADD = 0, WS_OP_GEMM = 1 };

typedef struct ws_view {
    int32_t buf;               /* WS_BUF_*                                 */
    int32_t form;              /* WS_FORM_*: how the view's block holds its values */
    int64_t off, rows, cols, ld;  /* element offset, shape, leading dim   */
} ws_view;

/* A view holds residues (one storage-type entry per element) unless the
 * plan runs on the 8-bit digit base: there a workspace temporary that is
 * written by an addition group and read only by base products (in one
 * operand role) and by addition groups may hold the three signed digit
 * planes of its centred residues instead, in the layout the product reads
 * (rows of 128 x 64 tiles, the inner index contiguous, 16-byte chunks
 * XOR-swizzled by row; B operands transposed), 3 bytes per element at the
 * start of its block.  Such a view is dense (ld == cols), even-offset, has
 * whole tiles (A role: rows % 128 == 0, cols % 64 == 0; B role:
 * cols % 128 == 0, rows % 64 == 0) and is never read as residues before
 * something rewrites it.  The forms appear in wsmul_plan_export's output
 * for the digit base (the execution list it runs).  Views of A and B may
 * carry a form too when the plan never writes that input: the call then
 * splits the whole input into digit planes once, in its digit scratch, and
 * such views (whole tiles of those planes) are read from there.  In that
 * list, epilogue
 * rows that do not read the product may move into an addition group of their
 * own just before it, and a product with four or more epilogue streams
 * besides its own store keeps only an output that is the product itself,
 * its other rows moving into an addition group right after it. */
enum { WS_FORM_RESIDUES = 0, WS_FORM_DIGITS_A = 1, WS_FORM_DIGITS_B = 2 };

/* out[o] <- sum_i coef[o][i] * in[i]  (mod p), elementwise.  For a base
 * product, in[0] stands for alpha*a*b (already reduced) and is not read. */
typedef struct ws_op_desc {
    int32_t kind;              /* WS_OP_ADD or WS_OP_GEMM   */
    int32_t nin, nout, depth;
    int64_t alpha;
    ws_view a, b;
    ws_view in[WS_MAX_IN];
    ws_view out[WS_MAX_OUT];
    int64_t coef[WS_MAX_OUT][WS_MAX_IN];
} ws_op_desc;

/* Fill `stats` (workspace bytes, launches, counts) for args without running.
 * Pointers in args are not dereferenced and may be NULL. */
WSMUL_API int wsmul_plan_info(const ws_args *args, ws_stats *stats);

/* Copy up to `cap` operations of the plan into `ops`; *count receives the
 * total number (call with cap = 0 to size the buffer).  On the digit base
 * (args->base, or the base the autotuner picks) this is the execution list,
 * with view forms as described at ws_view. */
WSMUL_API int wsmul_plan_export(const ws_args *args, ws_op_desc *ops, int64_t cap, int64_t *count);

#ifdef __cplusplus
}
#endif
#endif /* WSMUL_H */
