/*
 * msp.h — masked sparse matrix-matrix products on AMD Instinct MI355X (gfx950).
 *
 * Computes C = M .* (A B) over a semiring (Section "Background and Notation":
 * M is m x n, A is m x k, B is k x n, C is m x n), or C = !M .* (A B) with a
 * complemented mask (Introduction; Section "Masked Sparse Accumulator" for
 * the complemented accumulator). Only the pattern of M is used; M's values
 * are never read.
 *
 * An entry C(i,j) exists iff the mask admits (i,j) and at least one k has
 * both A(i,k) and B(k,j) stored, whatever the values (the accumulator's
 * remove() returns "none" only when nothing was inserted, Section
 * "Accumulator"). Its value folds the products a (x) b with (+). Rows of C
 * are emitted in ascending column order for both mask modes.
 *
 * Conventions for every entry point:
 *  - All matrix pointers are DEVICE pointers, borrowed: the caller owns them
 *    and keeps them alive until the work enqueued on `stream` has finished.
 *    Inputs are never modified.
 *  - CSR: int64 row pointers (nrows+1 entries, rowptr[0] = 0,
 *    rowptr[nrows] = nnz), int32 column indices, sorted ascending and
 *    duplicate-free within each row, 0-based. `values` may be NULL: every
 *    stored entry then holds the semiring's multiplicative one.
 *    Violations are reported as MSP_ERR_INVALID_CSR when options->validate
 *    is set and are undefined behaviour otherwise.
 *  - `stream` is a hipStream_t (NULL = the default stream). Kernels are
 *    enqueued asynchronously; calls that return a host value say that they
 *    synchronize the stream.
 *  - No exception crosses the ABI. Every call returns an msp_status; the
 *    thread-local msp_last_error() gives a message. An asynchronous device
 *    fault surfaces as MSP_ERR_DEVICE at the next synchronizing call.
 *  - Dimension rule: A.ncols == B.nrows, M.nrows == A.nrows,
 *    M.ncols == B.ncols; a violation returns MSP_ERR_DIMENSION_MISMATCH.
 *    Empty shapes (m, n or k = 0, nnz = 0) are valid and give an empty C.
 *  - Device memory: the library allocates none. Every device buffer it works
 *    in is the caller's: the operands, the outputs, and workspaces whose
 *    sizes the *_workspace_size queries give (see "Workspaces" below). A
 *    workspace smaller than its query's size returns
 *    MSP_ERR_INSUFFICIENT_CAPACITY before any work is enqueued. Workspaces
 *    need no initialisation: the library clears what it uses.
 */
#ifndef MSP_H
#define MSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum msp_status {
    MSP_OK = 0,
    MSP_ERR_INVALID_ARGUMENT = 1,
    MSP_ERR_DIMENSION_MISMATCH = 2,
    MSP_ERR_INVALID_CSR = 3,
    MSP_ERR_UNSUPPORTED = 4,
    MSP_ERR_INSUFFICIENT_CAPACITY = 5,
    MSP_ERR_OUT_OF_MEMORY = 6,
    MSP_ERR_DEVICE = 7
} msp_status;

/*
 * Semirings (input value type -> output value type). The paper describes its
 * accumulators on the arithmetic semiring and evaluates graph algorithms that
 * use others (Section "Background and Notation"); these are the ones here:
 *  PLUS_TIMES_F64  double -> double   IEEE binary64; sums may be reordered
 *  PLUS_PAIR_I64   (values ignored) -> int64: counts contributing products
 *  LOR_LAND_BOOL   uint8 -> uint8     (x) = a&&b, (+) = ||, result 0 or 1
 *  PLUS_TIMES_I32  int32 -> int32     wrap-around mod 2^32
 *  PLUS_TIMES_I64  int64 -> int64     wrap-around mod 2^64
 */
typedef enum msp_semiring {
    MSP_PLUS_TIMES_F64 = 0,
    MSP_PLUS_PAIR_I64 = 1,
    MSP_LOR_LAND_BOOL = 2,
    MSP_PLUS_TIMES_I32 = 3,
    MSP_PLUS_TIMES_I64 = 4
} msp_semiring;

/*
 * Accumulator kinds. The library picks one per row (or per column tile /
 * mask chunk of a heavy row) unless options->force_kind is set.
 *  DENSE    dense state over a column tile held in LDS: admitted bitmap,
 *           inserted bitmap and values, emitted by a scan of the tile
 *           (the masked sparse accumulator of Section "Masked Sparse
 *           Accumulator", re-laid out per tile). Normal and complemented.
 *  HASH     open-addressing table in LDS keyed by the mask's columns
 *           (Section "Hash Accumulator"). Normal mask only.
 *  MASKIDX  slot = rank of the column in the row of M, found by binary
 *           search over the mask row staged in LDS (Section "Mask
 *           Compressed Accumulator"). Normal mask only.
 *           HASH and MASKIDX first test each product's column against a
 *           bitmap filter of the mask row in LDS; only products that pass
 *           are looked up (the accumulator still holds one slot per mask
 *           entry, as in the paper).
 *  INNER    pull formulation: one sparse dot product of A(i,:) with B(:,j)
 *           per admitted (i,j) (Section "Pull-based Algorithms"). Needs the
 *           transpose of B, built by the plan unless options->b_transpose is
 *           given. Normal mask only.
 *  HEAP     one lane per row: a k-way merge of the rows of B selected by
 *           A(i,:), ordered by a min-heap of row iterators in LDS keyed by
 *           (column, position in A's row), so that products of one column
 *           come out consecutively and the row is emitted sorted without a
 *           sort (Section "Masked Heap SpGEVM Algorithm"). Before an
 *           iterator enters the heap it is advanced past columns the mask
 *           does not admit (a binary search of the mask row per product),
 *           so only admitted products are merged. Normal and complemented.
 *           Rows whose row of A has more than 8 entries, or with 2^24
 *           products or more, take the automatic choice instead.
 * Forcing MASKIDX, HASH or INNER together with a complemented mask returns
 * MSP_ERR_UNSUPPORTED.
 */
typedef enum msp_kind {
    MSP_KIND_AUTO = -1,
    MSP_KIND_DENSE = 0,
    MSP_KIND_HASH = 1,
    MSP_KIND_MASKIDX = 2,
    MSP_KIND_INNER = 3,
    MSP_KIND_HEAP = 4
} msp_kind;

/* Read-only CSR view of device memory (see the conventions above). */
typedef struct msp_csr {
    int64_t nrows;
    int64_t ncols;
    int64_t nnz;
    const int64_t* rowptr;  /* device, nrows + 1 */
    const int32_t* colidx;  /* device, nnz */
    const void* values;     /* device, nnz of the semiring's input type, or NULL */
} msp_csr;

/*
 * Output CSR, allocated by the caller. rowptr has nrows + 1 entries;
 * colidx/values have `capacity` entries (values of the semiring's output
 * type). On success the library writes rowptr (rowptr[nrows] = nnz(C)),
 * and the first nnz(C) entries of colidx and values.
 */
typedef struct msp_csr_out {
    int64_t nrows;
    int64_t ncols;
    int64_t capacity;
    int64_t* rowptr;
    int32_t* colidx;
    void* values;
} msp_csr_out;

typedef struct msp_options {
    int32_t phase;        /* 1: one-phase (numeric into staging, then compaction,
                             Section "Symbolic and Numeric Phases");
                             2: two-phase (symbolic count, then numeric). 0 = 1. */
    int32_t force_kind;   /* msp_kind; MSP_KIND_AUTO (-1) lets the binner choose */
    int32_t validate;     /* nonzero: check the CSR invariants of A, B and M on
                             the device at plan creation */
    int32_t inner_ratio;  /* auto mode: use INNER for a row when its pull cost
                             (sum over mask columns of nnz(B(:,j))) times this
                             ratio is below its push cost (products). 0 = never
                             choose INNER automatically. */
    const msp_csr* b_transpose; /* optional CSR of B^T (n x k); NULL = built by the
                                   plan when INNER is used */
    int32_t maskidx_max;  /* auto mode: rows whose mask has at most this many
                             entries use MASKIDX whatever their product count;
                             light rows (at most block_flops products) with at
                             most 256 mask entries use MASKIDX too, other rows
                             with at most 512 use HASH (-1 = default 8) */
    int32_t heap_flops;   /* auto mode, matrices of more than 512 columns:
                             rows whose row of A has at most 8 entries use HEAP
                             when they have at most this many products, or at
                             most twice as many and a mask row with at least 8
                             entries per product; under a complemented mask,
                             when they have at most this many products, or,
                             with more than 4096 columns, more than 4096
                             (rows between go to the sorting bin) (-1 =
                             default 32; 0 = never). An automatic heap bin
                             runs in the MASKIDX wave kernel instead when it
                             has at most 32768 rows, all with normal mask rows
                             of at most 256 entries, or in the MASKIDX block
                             kernel when it has at most 4096 rows, all with
                             normal mask rows of 257 to 2048 entries; another
                             bin of at most 32768 rows, all under 256
                             products, runs in the one-wave sorting kernel: a
                             small heap launch costs more than it saves. */
    int64_t block_flops;  /* rows with more products than this run on a whole
                             workgroup (256 threads; 512 for mask-indexed
                             rows of at least 65536 products) instead of
                             one wavefront, except dense-kind rows of
                             matrices of at most 512 columns, which do so
                             only above 32 times this (-1 = default 8192) */
    int64_t split_flops;  /* dense-kind rows (at most 4096 columns) with more
                             products than this are split over several
                             workgroups by chunks of A's row (-1 = default
                             262144; 0 = never split) */
    const int8_t* kind_table; /* auto mode: optional accumulator kind per row
                             class (host, MSP_KIND_CLASSES bytes, read at plan
                             creation): entry [fb * MSP_ROW_BUCKETS + mb] is the
                             msp_kind of the rows whose product count falls in
                             bucket fb and whose mask row length falls in bucket
                             mb (bucket b: 4^b <= x < 4^(b+1), bucket 0 also
                             holds 0, the last one everything above), or -1 to
                             keep the rules above. An entry that does not fit
                             the row (a complemented mask with other than
                             DENSE or HEAP, HEAP for a row of A with more than
                             8 entries or more than 2^24 - 1 products) is
                             ignored for that row. NULL = no table. */
} msp_options;

#define MSP_ROW_BUCKETS 12
#define MSP_KIND_CLASSES (MSP_ROW_BUCKETS * MSP_ROW_BUCKETS)

/* Fills `opt` with the defaults: phase 1, auto kind, no validation,
   inner_ratio 0, no B^T, maskidx_max 8, heap_flops 32, block_flops 8192,
   split_flops 262144, no kind table. */
void msp_options_default(msp_options* opt);

/* Plan statistics, filled by msp_plan_info. */
typedef struct msp_plan_info_t {
    int64_t upper_bound;     /* sum over rows of min(admitted columns, products):
                                the exact per-row output bound; a one-phase
                                output needs capacity >= this */
    int64_t products;        /* sum over rows of products (flops_i) */
    int64_t units;           /* work units (rows or row tiles) */
    int64_t staging;         /* staging entries used by one-phase execution */
    int64_t mask_nnz;        /* nnz(M) */
    int64_t kind_units[8];   /* units per msp_kind (0..4), and [5]: units of the sorting bin */
    int64_t bin_units[16];   /* units per kernel bin (MSP_BIN_*; MSP_NBINS used) */
} msp_plan_info_t;

/*
 * Kernel bins: every work unit runs in the numeric kernel of its bin. The
 * "wave" bins give one wavefront per unit, the "block" bins one 256-thread
 * workgroup per unit (512 threads for the units of MSP_BIN_MASKIDX_BLOCK
 * whose row has at least 65536 products).
 */
enum {
    MSP_BIN_DENSE_WAVE = 0,
    MSP_BIN_DENSE_BLOCK = 1,
    MSP_BIN_HASH_WAVE = 2,
    MSP_BIN_HASH_BLOCK = 3,
    MSP_BIN_MASKIDX_WAVE = 4,
    MSP_BIN_MASKIDX_BLOCK = 5,
    MSP_BIN_INNER_WAVE = 6,
    MSP_BIN_DENSE_BLOCK_NARROW = 7,  /* dense state over <= 512 columns, one workgroup per row */
    MSP_BIN_DENSE_SPLIT = 8,         /* rows with many products: one workgroup per chunk of the
                                        row of A, merged into a per-row accumulator */
    MSP_BIN_HEAP_LANE = 9,           /* one lane per row, k-way merge (HEAP kind) */
    MSP_BIN_HEAP_LANE_LONG_MASK = 10,  /* the same, normal mask rows of more than 256 entries */
    MSP_BIN_MASKIDX_PACKED = 11,     /* eight lanes per row: normal mask rows of <= 16 entries,
                                        <= 256 products, <= 32 entries in the row of A
                                        (automatic choice only) */
    MSP_BIN_SORT_BLOCK = 12,         /* one workgroup per row: complemented mask rows of matrices
                                        wider than 4096 columns with more than heap_flops and
                                        < 1024 products (<= 4096 from 40961 columns on):
                                        products expanded, sorted by column, folded and
                                        filtered (automatic choice only) */
    MSP_NBINS = 13
};

/* Stage slots of msp_execute_profiled: 0..15 = numeric kernel of bin b,
   then these. */
enum {
    MSP_STAGE_SYMBOLIC = 16,  /* all symbolic count kernels (two-phase) */
    MSP_STAGE_SCAN = 17,      /* prefix sums of the unit counts */
    MSP_STAGE_ROWPTR = 18,    /* row pointers of C */
    MSP_STAGE_COMPACT = 19,   /* one-phase staging -> C */
    MSP_STAGE_SPLIT_EMIT = 20,  /* emission of the split rows */
    MSP_STAGE_PLACE = 21,       /* placement of the work units in the execution workspace */
    MSP_NSTAGES = 22
};

typedef struct msp_plan msp_plan;

/*
 * ---- Workspaces ----
 * A plan works in two caller-owned device buffers (any device allocation
 * aligned to 256 bytes, e.g. a torch tensor of bytes):
 *  - the PLAN workspace, given to msp_plan_create and held by the plan until
 *    msp_plan_destroy (the caller keeps it alive and does not touch it):
 *    per-row product counts, tile counts and bins, the plan statistics, the
 *    unit-list segment offsets, and B^T when the inner kind may run. Its
 *    size depends only on the operands' shapes and nnz, so
 *    msp_plan_workspace_size computes it on the host without GPU work.
 *  - the EXECUTION workspace, given to every call that runs the product
 *    (msp_execute*, msp_symbolic, msp_numeric, msp_batch_bind): the work-unit
 *    lists (placed at the start of each such call), per-unit counts and
 *    prefix sums, the one-phase staging (Section "Symbolic and Numeric
 *    Phases": the output of the one-phase method is written to storage sized
 *    by an upper bound and then copied), the accumulators of rows split
 *    over several workgroups, and, for a single product over at most 512
 *    columns whose dense rows re-read B at least 4 times over, a 16-bit copy
 *    of B's column indices that each call makes before its numeric kernels.
 *    Its size depends on the binning, known after
 *    msp_plan_create: msp_workspace_size. Its contents matter only within a
 *    call, except from msp_symbolic to msp_numeric, and from msp_batch_bind
 *    to the batch's executions.
 * Executions of one plan with DIFFERENT execution workspaces may run
 * concurrently on different streams; two executions that share one
 * workspace must be ordered by the caller. A plan is used by one host thread
 * at a time.
 */

/* Plan workspace bytes for these operands and options (host only; the same
   argument checks as msp_plan_create). */
msp_status msp_plan_workspace_size(const msp_csr* A, const msp_csr* B, const msp_csr* M, int complement,
                                   msp_semiring semiring, const msp_options* opt, size_t* bytes);

/*
 * Analyse the operands and bind a plan to them (row analysis and row
 * binning). Computes per row the product count
 * flops_i = sum over stored A(i,k) of nnz(B(k,:)), the mask count, the
 * output bound, and the accumulator kind and tiling, and counts the work
 * units of every bin. Works in `workspace` (device, workspace_bytes >=
 * msp_plan_workspace_size), which the plan holds until msp_plan_destroy,
 * and SYNCHRONIZES `stream` once to read the sizes. The operands must stay
 * alive and unchanged while the plan is used. `opt` may be NULL (defaults).
 */
msp_status msp_plan_create(msp_plan** plan, const msp_csr* A, const msp_csr* B, const msp_csr* M,
                           int complement, msp_semiring semiring, const msp_options* opt,
                           void* workspace, size_t workspace_bytes, void* stream);

/* Execution workspace bytes of a plan or batch (host; for a single-product
   plan, those of its phase: the one-phase bytes include the staging). */
msp_status msp_workspace_size(const msp_plan* plan, size_t* bytes);

/* Copies the plan's statistics into `info` (host). */
msp_status msp_plan_info(const msp_plan* plan, msp_plan_info_t* info);

/*
 * Two-phase, symbolic step: counts nnz(C(i,:)) from indices only and writes
 * the row pointers of C into C_rowptr (device, nrows + 1). If nnz_host is not
 * NULL, SYNCHRONIZES and stores nnz(C) there. The execution workspace keeps
 * the unit lists and counts for msp_numeric.
 */
msp_status msp_symbolic(msp_plan* plan, int64_t* C_rowptr, int64_t* nnz_host, void* workspace,
                        size_t workspace_bytes, void* stream);

/*
 * Two-phase, numeric step (after msp_symbolic on the same plan, with the same
 * C->rowptr and the same, untouched execution workspace): writes colidx and
 * values of C. C->capacity must be >= nnz(C): when msp_symbolic did not
 * return nnz(C) and the capacity is below the plan's upper bound, this call
 * SYNCHRONIZES once to read nnz(C). A short capacity returns
 * MSP_ERR_INSUFFICIENT_CAPACITY before any kernel runs.
 */
msp_status msp_numeric(msp_plan* plan, msp_csr_out* C, void* workspace, size_t workspace_bytes,
                       void* stream);

/*
 * Runs the whole product on a plan: phase 1 (numeric into staging sized by
 * the per-unit bounds, then prefix sum of the counts and compaction into C)
 * or phase 2 (symbolic, prefix sum, numeric), as options->phase says.
 * Phase 1 needs C->capacity >= info.upper_bound; phase 2 needs
 * C->capacity >= nnz(C) and SYNCHRONIZES once to check it.
 * If nnz_host is not NULL, SYNCHRONIZES and stores nnz(C) there.
 * Works in the execution workspace (device, workspace_bytes >=
 * msp_workspace_size). May be called repeatedly on one plan (e.g. after the
 * values of A or B changed in place).
 */
msp_status msp_execute(msp_plan* plan, msp_csr_out* C, int64_t* nnz_host, void* workspace,
                       size_t workspace_bytes, void* stream);

/*
 * msp_execute with timing: records HIP events on `stream` around every
 * stage, SYNCHRONIZES, and ADDS each stage's elapsed milliseconds to
 * stage_ms[MSP_NSTAGES] (host; stages that did not run add 0). For
 * measurement; the results are those of msp_execute.
 */
msp_status msp_execute_profiled(msp_plan* plan, msp_csr_out* C, int64_t* nnz_host, void* workspace,
                                size_t workspace_bytes, double* stage_ms, void* stream);

/*
 * Timing sessions: stage timing without a synchronization per execution.
 * msp_execute_timed runs msp_execute and records the stages' HIP events into
 * the session (it synchronizes only when nnz_host is not NULL);
 * msp_timing_collect waits for the recorded events and ADDS each stage's
 * milliseconds, summed over the executions since the last collect, to
 * stage_ms[MSP_NSTAGES] (host). A session belongs to the device current at
 * its creation and to one host thread at a time; it owns its events.
 */
typedef struct msp_timing msp_timing;
/* `executions`: events for this many executions are created up front (more
   are created on demand); 0 creates none. `stages`: bit s set times stage s
   (MSP_STAGE_* or a bin number); 0 times every stage. Each timed stage costs
   the events attached to its launches. */
msp_status msp_timing_create(msp_timing** timing, int32_t executions, uint32_t stages);
msp_status msp_execute_timed(msp_plan* plan, msp_csr_out* C, int64_t* nnz_host, void* workspace,
                             size_t workspace_bytes, msp_timing* timing, void* stream);
msp_status msp_timing_collect(msp_timing* timing, double* stage_ms);
void msp_timing_destroy(msp_timing* timing);

/* Copies the kernel bin of every row (MSP_BIN_*, or -1 for rows with no
   possible output) into bins (host, nrows entries). SYNCHRONIZES. */
msp_status msp_plan_row_bins(const msp_plan* plan, int8_t* bins, void* stream);

/* Releases the plan's host state and graph. The plan frees no device memory
   (its workspaces are the caller's); the caller may reuse them once the work
   it enqueued with the plan has finished. */
void msp_plan_destroy(msp_plan* plan);

/*
 * One-shot product: plan, execute, destroy, in ONE caller-owned device
 * workspace that holds the plan workspace followed by the execution
 * workspace. C->capacity must be at least the upper bound (phase 1) or
 * nnz(C) (phase 2); otherwise returns MSP_ERR_INSUFFICIENT_CAPACITY and
 * writes the bound into *nnz_host when it is not NULL. A workspace that is
 * too small returns MSP_ERR_INSUFFICIENT_CAPACITY and, when ws_needed is not
 * NULL, the bytes needed: the plan workspace alone if even that does not
 * fit (a second call then learns the whole size), else the whole size.
 * SYNCHRONIZES.
 */
msp_status msp_masked_spgemm(const msp_csr* A, const msp_csr* B, const msp_csr* M, int complement,
                             msp_semiring semiring, const msp_options* opt, msp_csr_out* C,
                             int64_t* nnz_host, void* workspace, size_t workspace_bytes, size_t* ws_needed,
                             void* stream);

/*
 * For callers that cannot allocate device memory (code that must not call
 * hipMalloc, such as tight serving loops or harnesses that forbid it): the
 * one-shot product of msp_masked_spgemm with the same arguments and results,
 * but working in a fixed scratch array of MSP_NOALLOC_SCRATCH_BYTES bytes
 * that the library holds in device memory instead of a caller workspace.
 * Allocates no device memory and no page-locked host memory. Each GPU the
 * library runs on holds its own copy of the array until the process ends;
 * its device address is looked up once per device on the first call there,
 * with that device current, and `stream` must belong to the current device.
 * The caller still passes the operands and the output C (capacity rules as
 * msp_masked_spgemm). A product whose workspace would exceed the array
 * returns MSP_ERR_INSUFFICIENT_CAPACITY with *ws_needed (when not NULL) set
 * to the bytes msp_masked_spgemm reports. Every call on one GPU shares that
 * GPU's array and leaves its contents behind (the next call clears what it
 * needs): calls that overlap on one GPU, from several host threads or
 * streams, race and must be serialized by the caller. SYNCHRONIZES.
 */
#define MSP_NOALLOC_SCRATCH_BYTES (64u << 20)

msp_status msp_masked_spgemm_noalloc(const msp_csr* A, const msp_csr* B, const msp_csr* M, int complement,
                                     msp_semiring semiring, const msp_options* opt, msp_csr_out* C,
                                     int64_t* nnz_host, size_t* ws_needed, void* stream);

/* Exact per-row output bound summed over rows (see msp_plan_info_t), by the
   row analysis in `workspace` (device, at least msp_plan_workspace_size of
   the same operands under MSP_PLUS_PAIR_I64 and default options).
   SYNCHRONIZES. */
msp_status msp_upper_bound(const msp_csr* A, const msp_csr* B, const msp_csr* M, int complement,
                           int64_t* upper_bound, void* workspace, size_t workspace_bytes, void* stream);

/*
 * (+)-reduction of n output values of the semiring's output type into one
 * value written to `result` (device, one element of the output type); the
 * post-reduction of triangle counting (sum of L .* (L L), Section "Triangle
 * Counting"). Deterministic for a given n. n = 0 writes the identity.
 * Works in `workspace` (device, at least msp_reduce_workspace_size bytes).
 */
msp_status msp_reduce(const void* values, int64_t n, msp_semiring semiring, void* result,
                      void* workspace, size_t workspace_bytes, void* stream);

/* Workspace bytes of msp_reduce and msp_reduce_csr (the per-block partial
   sums; the same for every n). */
msp_status msp_reduce_workspace_size(size_t* bytes);

/*
 * msp_reduce over the entries of an output CSR without reading its size on
 * the host: reduces values[0 .. rowptr[nrows]) (rowptr and values device;
 * the count is read on the device, clamped to [0, capacity], the length of
 * `values`). Does not synchronize.
 */
msp_status msp_reduce_csr(const int64_t* rowptr, int64_t nrows, const void* values, int64_t capacity,
                          msp_semiring semiring, void* result, void* workspace, size_t workspace_bytes,
                          void* stream);

/*
 * ---- Batches: many products in one set of launches ----
 * A batch is a plan over `count` products on one semiring (one-phase only).
 * All products are analysed together; their work units are binned jointly,
 * so each kernel bin runs ONE launch over the units of every product, then
 * one prefix sum, one row-pointer and one compaction kernel serve all
 * outputs. msp_plan_info, msp_plan_row_bins and msp_plan_destroy accept a
 * batch; msp_execute/msp_symbolic/msp_numeric take single products only.
 */
typedef struct msp_problem {
    msp_csr A, B, M;      /* device views, as for msp_plan_create */
    int32_t complement;   /* 0 or 1 */
    int32_t reserved;     /* 0 */
} msp_problem;

/* Plan workspace bytes of a batch (host only). */
msp_status msp_batch_workspace_size(const msp_problem* problems, int64_t count, msp_semiring semiring,
                                    const msp_options* opt, size_t* bytes);

/* Analyses and bins all products (one synchronization) in the plan
   workspace (device, at least msp_batch_workspace_size bytes), which the
   batch holds until msp_plan_destroy. Without pull costs (inner_ratio 0)
   the row sums, the analysis and the unit placement run as one launch each
   for all products; with them, one product at a time. */
msp_status msp_batch_create(msp_plan** batch, const msp_problem* problems, int64_t count,
                            msp_semiring semiring, const msp_options* opt, void* workspace,
                            size_t workspace_bytes, void* stream);

/* Number of products of a batch (1 for a single-product plan). */
int64_t msp_batch_count(const msp_plan* batch);

/* Statistics of product p (0 <= p < count), or of all products (p = -1). */
msp_status msp_batch_info(const msp_plan* batch, int64_t p, msp_plan_info_t* info);

/* Binds the outputs C[0..count) (capacity of C[p] >= its upper bound) and
   the execution workspace (device, at least msp_workspace_size bytes), and
   places the work units there; the batch's executions use both until the
   next bind or msp_plan_destroy, so the caller keeps them alive and leaves
   the workspace untouched. SYNCHRONIZES. Invalidates a previously captured
   graph. */
msp_status msp_batch_bind(msp_plan* batch, const msp_csr_out* C, void* workspace, size_t workspace_bytes,
                          void* stream);

/* Enqueues the whole batch on `stream`: kernels only, no allocation, no
   memset and no synchronization, so the sequence may be captured. */
msp_status msp_batch_execute(msp_plan* batch, void* stream);

/* msp_batch_execute with the stage events recorded into a timing session
   (see msp_timing_create): per kernel bin and stage, the time of all
   products' units together. Not for graph capture. */
msp_status msp_batch_execute_timed(msp_plan* batch, msp_timing* timing, void* stream);

/* First call on a stream: captures msp_batch_execute into a HIP graph on
   `stream` (which must not be the default stream) and instantiates it; every
   call then launches the graph once. */
msp_status msp_batch_graph_launch(msp_plan* batch, void* stream);

/* nnz of every product's output into nnz[0..count) (host). SYNCHRONIZES. */
msp_status msp_batch_nnz(const msp_plan* batch, int64_t* nnz, void* stream);

/*
 * Device memory of the iterated products below, whose sizes depend on the
 * data (every level or iteration sizes the next): the library asks the
 * caller's allocator for each buffer and returns it when done.
 *  alloc(ctx, bytes, stream)   device memory of at least `bytes` bytes,
 *                              256-byte aligned, usable by work enqueued on
 *                              `stream`; NULL when none is left (the call
 *                              then returns MSP_ERR_OUT_OF_MEMORY).
 *  release(ctx, ptr, stream)   `ptr` (from alloc) may be reused by work
 *                              enqueued on `stream` after this point.
 * Every buffer is released before the call returns, on success or error.
 */
typedef struct msp_allocator {
    void* (*alloc)(void* ctx, size_t bytes, void* stream);
    void (*release)(void* ctx, void* ptr, void* stream);
    void* ctx;
} msp_allocator;

/*
 * Betweenness-centrality dependencies of a batch of sources (Section
 * "Betweenness Centrality": the multi-source two-stage algorithm of Brandes
 * on masked products). Forward stage, level d = 1, 2, ... until the frontier
 * is empty: F_d = !V_{d-1} .* (A F_{d-1}) with a complemented mask, F_0 holding
 * column j = source j with value 1, V = the union of the frontiers so far;
 * F_d's values are the shortest-path counts. Backward stage, d = D..2:
 * delta_{d-1} = sigma_{d-1} .* (F_{d-1} .* (A ((1 + delta_d) ./ sigma_d)))
 * with a normal mask. All products use PLUS_TIMES_F64.
 *
 *  A        n x n device CSR holding the SYMMETRIC pattern of an unweighted
 *           undirected graph; its values are ignored.
 *  sources  HOST array of nsrc vertex ids in [0, n) (repeats allowed: each
 *           entry is its own column).
 *  bc       DEVICE array of n doubles; the library ADDS, for every vertex v,
 *           the sum over the batch's sources s != v of delta_s(v) (not
 *           halved). The caller zeroes it for a fresh result.
 *  info     optional host struct filled with level and product counts and
 *           the wall time of each stage.
 *  mem      the caller's allocator (required) for every working buffer.
 * SYNCHRONIZES (every level sizes the next). Errors:
 * MSP_ERR_DIMENSION_MISMATCH (A not square), MSP_ERR_INVALID_ARGUMENT (NULL
 * pointers, a source out of range), MSP_ERR_OUT_OF_MEMORY (alloc returned
 * NULL).
 */
typedef struct msp_bc_info {
    int64_t levels;            /* D: frontiers F_1..F_D were non-empty */
    int64_t frontier_nnz;      /* sum of nnz(F_d), d >= 1 */
    int64_t forward_products;  /* products of the forward masked products */
    int64_t backward_products; /* products of the backward masked products */
    double forward_ms;         /* host wall time of each stage */
    double backward_ms;
} msp_bc_info_t;

msp_status msp_bc_batch(const msp_csr* A, const int32_t* sources, int64_t nsrc, double* bc,
                        msp_bc_info_t* info, const msp_allocator* mem, void* stream);

/*
 * k-truss (Section "Experimental Setup": the edges supported by at least
 * k - 2 triangles, found by masked products repeated while pruning changes
 * the graph): C = A; repeat S = C .* (C C) over PLUS_PAIR_I64 (the support
 * of every edge: its triangles inside C), C = the entries of S with support
 * >= k - 2; until no edge is removed.
 *
 *  A          n x n device CSR of an undirected graph (symmetric pattern,
 *             no self loops); values ignored.
 *  k          >= 3 runs the iteration; k <= 2 returns A (every edge
 *             qualifies) with supports 0.
 *  C_rowptr   device, n + 1 entries; C_colidx (int32) and C_support (int64)
 *             device arrays of at least nnz(A) entries, caller-allocated.
 *             The truss is written there, rows sorted, each edge with its
 *             support inside the truss.
 *  nnz_host   host: nnz of the truss.
 *  info       optional: iterations, products summed over all iterations,
 *             wall time.
 *  mem        the caller's allocator (required) for every working buffer.
 * SYNCHRONIZES every iteration.
 */
typedef struct msp_ktruss_info {
    int64_t iterations;
    int64_t products;  /* products of all masked products */
    double ms;
} msp_ktruss_info_t;

msp_status msp_ktruss(const msp_csr* A, int32_t k, int64_t* C_rowptr, int32_t* C_colidx, int64_t* C_support,
                      int64_t* nnz_host, msp_ktruss_info_t* info, const msp_allocator* mem, void* stream);

/* Static message for a status code. */
const char* msp_status_string(msp_status status);

/* Detail of the last error on the calling thread ("" if none). */
const char* msp_last_error(void);

/* Library version: major * 10000 + minor * 100 + patch. */
int msp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MSP_H */
