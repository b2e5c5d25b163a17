/*
 * mpk.h -- C-ABI of the level-blocked sparse matrix power kernel (MPK) for
 * AMD Instinct MI355X (gfx950).
 *
 * The method follows "Level-based Blocking for Sparse Matrices: Sparse
 * Matrix-Power-Vector Multiplication" (Alappat, Hager, Schenk, Wellein,
 * arXiv 2205.01598):
 *   - the MPK computes y_p = A^p x for p = 1..p_m and keeps every y_p
 *     (Sec. 3);
 *   - preprocessing takes A, p_m and a cache budget C, levels the graph of A
 *     by breadth-first search (Eq. 3), renumbers it level by level (Sec. 4.1),
 *     merges consecutive levels into level groups under Eq. (5) (Sec. 4.3),
 *     optionally refines bulky groups recursively (Sec. 4.4), and orders the
 *     (group, power) nodes by the diagonals of the Lp diagram (Sec. 4.2,
 *     Fig. 6) or by skewed diagonals (mpk_options.skew);
 *   - execution runs the powers over that order with point-to-point
 *     dependencies instead of barriers (Sec. 4.3, "p2p").
 * The baseline is p_m back-to-back SpMVs (Sec. 3.1, Fig. 2).
 *
 * Conventions for every entry point
 *   - All calls return mpk_status (0 = MPK_OK, < 0 = error).  No call aborts
 *     the process; on error nothing is written to caller outputs unless the
 *     entry point says otherwise, and mpk_last_error() returns a message
 *     (thread-local, valid until the next call on the same thread).
 *   - "host" pointers point to CPU memory, "device" pointers to memory on the
 *     GPU that is current when the call is made (hipMalloc / torch tensors).
 *   - Streams are passed as `void *` holding a hipStream_t (NULL = the null
 *     stream).  Device work is asynchronous on that stream.
 *   - Vectors are FP64, row-major N x k (k right-hand sides; element (i, c)
 *     at index i*k + c).  Power blocks are p x N x k: y_q occupies
 *     [(q-1)*N*k, q*N*k).
 *   - Plans and SpMV handles are not thread-safe; one run per plan may be in
 *     flight at a time (its dependency flags live in the plan).
 */
#ifndef MPK_H_
#define MPK_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPK_MAX_POWER 32
#define MPK_MAX_NRHS 32
#define MPK_MAX_SKEW 32
#define MPK_NUM_FEATURES 24

typedef int32_t mpk_status;
enum {
    MPK_OK = 0,
    MPK_ERR_ARG = -1,          /* bad argument (null pointer, p out of range, ...) */
    MPK_ERR_CSR = -2,          /* malformed CSR: rowptr not monotone, column out of range, ... */
    MPK_ERR_OOM = -3,          /* host or device allocation failed */
    MPK_ERR_HIP = -4,          /* a HIP runtime call failed */
    MPK_ERR_TIMEOUT = -5,      /* a device dependency wait exceeded the watchdog */
    MPK_ERR_UNSUPPORTED = -6,  /* valid request the library does not handle (e.g. nnz >= 2^31) */
    MPK_ERR_STATE = -7         /* call out of order (e.g. run before upload) */
};

typedef enum { MPK_F64 = 0, MPK_F32 = 1, MPK_BF16 = 2 } mpk_dtype;

/* Host CSR matrix, 0-based, square (n x n).  rowptr[n+1] (int64, monotone,
 * rowptr[0] = 0, rowptr[n] = nnz), col[nnz] (int32 in [0, n)), val[nnz].
 * Duplicate (row, col) entries are allowed and are summed like any other
 * stored entry; empty rows are allowed.  Column order inside a row is free. */
typedef struct mpk_csr {
    int64_t n;
    int64_t nnz;
    const int64_t *rowptr;
    const int32_t *col;
    const double *val;
} mpk_csr;

/* Options.  Call mpk_options_default() first, then change fields. */
typedef struct mpk_options {
    uint32_t size;            /* sizeof(mpk_options), for ABI growth */
    double safety_factor;     /* f of Eq. (5); default 0.5 as in Sec. 4.3 */
    int32_t root_mode;        /* BFS root: 0 = vertex 0 (Sec. 4.1 example), 1 = pseudo-peripheral */
    int32_t val_dtype;        /* mpk_dtype of stored matrix values (default MPK_F64) */
    int32_t nrhs;             /* k, right-hand sides per run, 1..MPK_MAX_NRHS (default 1) */
    int32_t workgroups;       /* persistent-kernel grid size; 0 = automatic */
    int32_t tile_nnz;         /* target nonzeros per device tile; 0 = 8192.  At or
                                 above one kernel chunk (4096 nonzeros at nrhs = 1,
                                 1024 at nrhs = 2, 4096/nrhs for nrhs >= 4) a tile
                                 is a run of round(tile_nnz / chunk) whole chunks */
    int32_t reserved0;        /* must be 0 */
    int64_t watchdog_spins;   /* dependency-wait polls before MPK_ERR_TIMEOUT; 0 = default */
    int32_t budget_vectors;   /* 1: Eq. (5) also counts the k vector entries per row
                                 ((p+1)(b_nz nnz + 8 k rows) < fC); 0 = the paper's form */
    int32_t skew;             /* device ticket order over the (group, power) nodes: sorted by
                                 g + skew*q, then q; 1..MPK_MAX_SKEW.  1 (default) = the Lp
                                 diagonals of Fig. 6; s >= 2 puts every dependency s - 1
                                 diagonals earlier (more work in flight without waiting, a
                                 reuse window of s*p + 1 groups instead of p + 1) */
    int32_t xcd_streams;      /* 1 (default): one ticket sequence for the whole grid.  8: the tiles
                                 of every level group (every unit of a refined plan) are cut into
                                 8 slices and slice s is run by
                                 the workgroups with blockIdx % 8 == s, which share one XCD on
                                 MI355X (the dispatcher deals workgroups round-robin over the 8
                                 XCDs), so a tile meets the same L2 at every power */
    int32_t plan_on_device;   /* 1: mpk_plan_create uses the current GPU: graph, levels (root search,
                                 breadth-first levels) and the renumbered matrix for a pattern with
                                 sorted symmetric rows; for other patterns the host builds the graph
                                 and renumbers, the GPU only levels.  Same results as the host, bit
                                 for bit.  0 (default): host only */
    int32_t force_acquire;    /* 1: every dependency wait ends with an agent-scope acquire fence even
                                 when mpk_run could do without it (see mpk_plan_info.line_closed_deps) */
    int32_t recursion_stages; /* s_m of Sec. 4.4: maximal runs of consecutive level groups that
                                 violate Eq. (5) are replaced by the breadth-first levels of the
                                 subgraph they induce, grouped again, up to this many stages.
                                 0 (default): no refinement.  A refined plan orders its tickets by
                                 a longest-path wavefront number over per-tile dependency lists and
                                 cannot be retuned (the numbering depends on p and C). */
    int32_t accum_f64;        /* FP32 / BF16 values only.  0 (default): the input vector is rounded
                                 to FP32 and products and row sums are formed in FP32, each power
                                 stored in FP64.  1: values widened to FP64, products and row sums
                                 in FP64 (the input vector as given); only the matrix storage is
                                 reduced.  FP64 values always use FP64 (the flag is ignored). */
    int32_t reserved;         /* must be 0 */
} mpk_options;

/* Plan summary (mpk_plan_query). */
typedef struct mpk_plan_info {
    int64_t n, nnz;
    int32_t p;                /* p_m */
    int32_t nrhs;
    int64_t n_levels;         /* L */
    int64_t n_groups;         /* G */
    int64_t n_tiles;          /* device tiles (row ranges inside groups) */
    int64_t n_tickets;        /* n_tiles * p: work items of one run */
    int64_t root;             /* BFS root (original index) */
    int64_t max_level_rows, max_group_nnz;
    int64_t violating_groups; /* groups that break Eq. (5) (single bulky levels) */
    uint64_t device_bytes;    /* device memory held after mpk_plan_upload */
    int32_t workgroups;       /* grid size mpk_run will launch */
    int32_t n_chunks;         /* MPK kernel work units inside the tiles (<= 4096
                                 nonzeros at nrhs = 1, 1024 at nrhs = 2,
                                 4096/nrhs for nrhs >= 4) */
    int32_t tile_nnz;
    int32_t val_dtype;
    double plan_seconds;      /* host time spent in mpk_plan_create */
    double phase_seconds[4];  /* of which: graph of A + A^T, root search + BFS, renumbering,
                                 groups/schedule/tiles */
    int32_t line_closed_deps; /* 1: mpk_run can skip the acquire fence after each dependency wait.
                                 The planner widened every dependency range to whole 128-byte lines
                                 of a vector slice and every widened dependency is an earlier
                                 ticket; mpk_run then skips the fence when Y is 128-byte aligned,
                                 N*k*8 is a multiple of 128 and force_acquire is 0.  No line of a
                                 power is read before all its rows are final, so no cache holds a
                                 stale copy; the accumulator is read with agent-scope loads. */
    int32_t last_run_fenced;  /* the last mpk_run used the acquire fence: 1, did not: 0, no run: -1 */
    int32_t recursive;        /* 1: refined levels (recursion_stages > 0, Sec. 4.4) */
    int32_t max_stage;        /* deepest refinement stage of a final group (0: none refined) */
    int64_t n_units;          /* final level groups: G, or the groups of the refined numbering */
    int64_t n_dep_ranges;     /* refined plans: tile ranges in all dependency lists together */
} mpk_plan_info;

/* Three-term recurrence epilogue for mpk_run / mpk_run_baseline (Sec. 7,
 * Eq. (7)-(8)).  For q = 1..p the kernel computes
 *     y_q = alpha[q-1] * (A y_{q-1}) + beta[q-1] * y_{q-1} + gamma[q-1] * y_{q-2}
 * with y_0 = X and y_{-1} = y_prev (device, N x k; may be NULL when every
 * gamma is 0), and, when acc != NULL,
 *     acc += coef_q * y_q
 * where coef is real (coef[q-1]) or, with complex_pairs = 1, complex
 * (coef[2(q-1)] + i coef[2(q-1)+1]) acting on k = 2 columns holding
 * (re, im) of one complex vector.  Coefficient arrays are host memory with p
 * (or 2p) entries, copied into the launch; y_prev and acc are device memory.
 * With coef0 != NULL (host, 1 value, or 2 = re, im with complex_pairs) the
 * first power starts the sum instead of adding to it:
 *     acc = coef0 * y_0 + coef_1 * y_1
 * so acc need not be initialised (a Chebyshev step's first block).
 * Chebyshev: alpha = (1, 2, 2, ...), beta = 0, gamma = (0, -1, -1, ...) in
 * the first block; later blocks pass the last two vectors of the previous
 * block as y_prev and X and use alpha = 2, gamma = -1 throughout. */
typedef struct mpk_recurrence {
    const double *alpha;
    const double *beta;
    const double *gamma;
    const double *coef;
    int32_t complex_pairs;
    const double *y_prev;
    double *acc;
    const double *coef0;
} mpk_recurrence;

typedef struct mpk_plan mpk_plan;
typedef struct mpk_spmv mpk_spmv;

/* Fill *opt with defaults (f = 0.5, root_mode 0, F64, k = 1, automatic launch). */
void mpk_options_default(mpk_options *opt);

/* Preprocessing (Sec. 4, "RACE" paragraph): validate A, build the graph of
 * A + A^T (diagonal dropped; Sec. 4 notes non-symmetric A is allowed), BFS
 * levels from the root (Eq. 3), level-by-level renumbering (Sec. 4.1), level
 * groups under Eq. (5) with budget floor(f*C) bytes and b_nz = sizeof(value)+4
 * bytes per nonzero (12 for FP64, Sec. 3.1), the Lp diagonal order of the
 * groups (Fig. 6), and device tiles with their point-to-point dependency
 * ranges (Sec. 4.3).  Host work only (no GPU call), except with
 * opt->plan_on_device = 1, where graph, levels and renumbering use the
 * current GPU, whose memory is freed before returning.  The CSR is
 * copied; the caller may free it on return.  p in [1, MPK_MAX_POWER],
 * cache_bytes > 0.  *out receives a new plan (free with mpk_plan_destroy).
 * Errors: MPK_ERR_ARG, MPK_ERR_CSR, MPK_ERR_OOM, MPK_ERR_UNSUPPORTED
 * (nnz >= 2^31 or n >= 2^31). */
mpk_status mpk_plan_create(const mpk_csr *A, int32_t p, uint64_t cache_bytes,
                           const mpk_options *opt, mpk_plan **out);

/* Preprocessing of a matrix that is already in GPU memory, which stays there
 * (the preprocessing of Sec. 6, kept next to the matrix: no copy of the CSR
 * to the host and back).  A->rowptr (int64, n+1), A->col and A->val are
 * device pointers on the current GPU; n and nnz are host values.  The CSR is
 * validated on the device with the checks of mpk_plan_create; then graph,
 * root search and BFS levels (Eq. 3), the renumbering (Sec. 4.1) and P A P^T
 * run on the GPU as with opt->plan_on_device = 1, with the same results bit
 * for bit, and the level groups, schedule and tiles are built as by
 * mpk_plan_create.  The plan keeps P A P^T in device memory (FP64, about
 * 12 bytes per nonzero plus the row pointers; FP32/BF16 values are
 * converted on the device at upload) and only the row pointers, permutation
 * and levels on the host; mpk_plan_matrix copies the matrix back on demand.
 * The caller's CSR is only read and may be freed on return.
 * Restrictions: rows sorted by column with a symmetric pattern and at most
 * 4096 stored entries per row, and recursion_stages = 0 (refinement runs on
 * the host); other matrices are planned with mpk_plan_create.
 * Errors: MPK_ERR_ARG, MPK_ERR_CSR, MPK_ERR_OOM, MPK_ERR_HIP,
 * MPK_ERR_UNSUPPORTED (the restrictions above, nnz >= 2^31 or n >= 2^31). */
mpk_status mpk_plan_create_device(const mpk_csr *A, int32_t p, uint64_t cache_bytes, const mpk_options *opt,
                                  mpk_plan **out);

/* Re-derives the level groups, schedule, tiles and tickets for a new p, cache
 * budget C and options, keeping the BFS levels and the renumbered matrix (the
 * expensive part of preprocessing; Sec. 5 notes that p_m and C do not change
 * the levels).  opt->root_mode must equal the plan's.  If the plan was
 * uploaded its device buffers are rebuilt (synchronous).  On error the plan is
 * left as it was. */
mpk_status mpk_plan_retune(mpk_plan *plan, int32_t p, uint64_t cache_bytes, const mpk_options *opt);

/* Summary of a plan: the sizes of the preprocessing results of Sec. 4 -
 * levels L (Eq. 3), level groups (Eq. 5; violating_groups counts the bulky
 * single levels of Sec. 4.4), the Lp nodes G*p of Fig. 6 as device tiles and
 * tickets - and the timing of each preprocessing phase (Sec. 6 reports the
 * preprocessing cost).  info: host, written on success; MPK_ERR_ARG for a
 * null argument. */
mpk_status mpk_plan_query(const mpk_plan *plan, mpk_plan_info *info);

/* Host copies of the plan arrays.  Any pointer may be NULL to skip it.
 *   perm[n]        perm[new] = old (the permutation vector of Sec. 4.1)
 *   level_ptr[L+1] first new row of each level (Fig. 4e)
 *   group_ptr[G+1] first level of each level group (Sec. 4.3)
 *   schedule[3*G*p] execution order of the Lp diagram: rows (d, p, i) with
 *                  d = i + p, step = row index (Fig. 6) */
mpk_status mpk_plan_arrays(const mpk_plan *plan, int32_t *perm, int32_t *level_ptr,
                           int32_t *group_ptr, int32_t *schedule);

/* Host copy of the renumbered matrix P A P^T (columns ascending per row),
 * FP64 values as given (before any dtype conversion).  rowptr[n+1],
 * col[nnz], val[nnz]; any pointer may be NULL. */
mpk_status mpk_plan_matrix(const mpk_plan *plan, int64_t *rowptr, int32_t *col, double *val);

/* Device tile table (host copies): tile_row[n_tiles+1] first row of each
 * tile, dep_lo/dep_hi[n_tiles] the first/last tile whose power q-1 a tile
 * waits for before computing power q, work[n_tickets] ticket order (tile *
 * 64 + (q-1)).  Any pointer may be NULL. */
mpk_status mpk_plan_tiles(const mpk_plan *plan, int32_t *tile_row, int32_t *dep_lo,
                          int32_t *dep_hi, int32_t *work);

/* Point-to-point dependencies of every tile (host copy), 6 int32 per tile:
 * (lo, hi) tile ranges, inclusive, in level groups g-1, g and g+1 of the
 * tile's group g (lo > hi: no dependency there).  Before computing power q a
 * tile waits for power q-1 of exactly these tiles (Sec. 4.3, with Eq. (4)
 * limiting the reads of a group to its two neighbour groups).
 * line_closed = 1 returns the same ranges widened to whole 128-byte lines of
 * a vector slice (they may reach one tile into groups g-2 and g+2), which
 * mpk_run uses when it skips the acquire fence.  A refined plan
 * (recursion_stages > 0) keeps its dependencies in per-tile lists
 * (mpk_plan_units); its ranges here are all empty (lo = 1 > hi = 0). */
mpk_status mpk_plan_tile_deps(const mpk_plan *plan, int32_t *ranges, int32_t line_closed);

/* Refined plans only (recursion_stages > 0, Sec. 4.4), host copies; any
 * pointer may be NULL.  The refined numbering (perm of mpk_plan_arrays) lists
 * the final level groups ("units") one after the other:
 *   unit_ptr[n_units+1]  first new row of every unit
 *   unit_stage[n_units]  stage at which the unit was formed: 0 = a group of
 *                        the original levels that satisfies Eq. (5), s >= 1 =
 *                        a group of the levels of a subgraph refined s times
 *   dep_ptr[n_tiles+1]   first range of every tile's dependency list
 *   dep_rng[2*n_dep_ranges] inclusive tile ranges (lo, hi), ascending: before
 *                        power q a tile waits for power q-1 of these tiles,
 *                        which hold every row it reads and every row that
 *                        shares a 128-byte line of a vector slice with them;
 *                        ranges at most 31 tiles apart are merged, so a list
 *                        may also name tiles between needed ones.
 * Level groups and the schedule of mpk_plan_arrays describe the unrefined
 * (stage-0) levels.  Errors: MPK_ERR_STATE for an unrefined plan. */
mpk_status mpk_plan_units(const mpk_plan *plan, int32_t *unit_ptr, int32_t *unit_stage, int32_t *dep_ptr,
                          int32_t *dep_rng);

/* Matrix and level features for the learned tuner, host, MPK_NUM_FEATURES
 * doubles: log10 N, log10 nnz, mean / standard deviation / log2(max+1) of the
 * row lengths, log10 of the number of levels, widest level / N, log2 p, then a
 * 16-bin histogram of the level widths (fraction of levels with width/N in
 * [2^-(b+1), 2^-b), b = 0..15, the last bin open below). */
mpk_status mpk_plan_features(const mpk_plan *plan, double *features);

/* Allocate the plan's device buffers on the current HIP device and copy the
 * renumbered matrix (converted to val_dtype, round to nearest even) and the
 * tile tables there.  Synchronous.  Errors: MPK_ERR_OOM, MPK_ERR_HIP. */
mpk_status mpk_plan_upload(mpk_plan *plan);

/* Gather/scatter between the original and the plan numbering (N x k FP64,
 * device), with the permutation vector of Sec. 4.1 (the renumbering that
 * lists the levels one after the other; the paper's MPK then runs on the
 * permuted matrix and vectors, Sec. 4.1 and the RACE paragraph of Sec. 4).
 * to_plan = 1: out[i] = in[perm[i]]; to_plan = 0: out[perm[i]] = in[i].
 * in and out must not alias (MPK_ERR_ARG); MPK_ERR_STATE before upload. */
mpk_status mpk_permute(const mpk_plan *plan, const double *in, double *out, int32_t k,
                       int32_t to_plan, void *stream);

/* One level-blocked MPK run (Sec. 4.2-4.3) in plan numbering: X (device,
 * N x k, read only) holds y_0; Y (device, p x N x k) receives y_1..y_p.  Y
 * must not overlap X, y_prev or acc, and acc must not overlap X or y_prev
 * (MPK_ERR_ARG otherwise).  rec = NULL gives plain powers.
 * k is the plan's nrhs.  Asynchronous; a dependency wait that outlives the
 * watchdog makes the kernel stop early and is reported by mpk_plan_status.
 * Runs of one plan must not overlap (its flags and counters are shared).
 * The kernel takes its run number from the plan's device memory, so the
 * launch is the same for every run and may be recorded by stream capture
 * and replayed; mpk_run itself allocates nothing and issues no memset. */
mpk_status mpk_run(mpk_plan *plan, const double *X, double *Y, const mpk_recurrence *rec,
                   void *stream);

/* mpk_run limited to the first `powers` powers (1 <= powers <= the plan's
 * p): y_1..y_powers into Y (device, powers x N x k), the recurrence arrays
 * read for powers entries (2*powers for complex coef).  Sec. 5 runs a power
 * count that is not a multiple of p_m as blocks of p_m followed by one
 * shorter block; this is that block, on the same plan: the tickets of the
 * higher powers are skipped (nothing waits for them).  Same buffer rules and
 * errors as mpk_run, plus MPK_ERR_ARG for powers out of range. */
mpk_status mpk_run_first(mpk_plan *plan, int32_t powers, const double *X, double *Y,
                         const mpk_recurrence *rec, void *stream);

/* Baseline on the renumbered matrix: p back-to-back SpMV launches (Fig. 2)
 * over the plan's device matrix, same arguments and results as mpk_run. */
mpk_status mpk_run_baseline(mpk_plan *plan, const double *X, double *Y,
                            const mpk_recurrence *rec, void *stream);
/* The baseline limited to the first `powers` powers (powers SpMV launches). */
mpk_status mpk_run_baseline_first(mpk_plan *plan, int32_t powers, const double *X, double *Y,
                                  const mpk_recurrence *rec, void *stream);

/* Level-blocked MPK with bulk synchronisation instead of point-to-point
 * flags (the variants Sec. 4.2 starts from before Sec. 4.3 replaces the
 * barriers).  MPK_SYNC_NODE: one kernel launch per Lp node (level group i,
 * power q) in the order of the plan's schedule (Fig. 6), G*p launches.
 * MPK_SYNC_WAVEFRONT: one launch per wavefront w = i + 2q with all its
 * nodes, G+2p-2 launches; node (i, q) reads groups i-1..i+1 at power q-1,
 * which lie on wavefronts w-3..w-1, so the nodes of a launch are
 * independent (a diagonal i + q of Fig. 6 is not: (i+1, q-1) feeds (i, q)).
 * The kernel boundary on `stream` is the barrier.  Plain powers only (no
 * recurrence); same arguments, layout and results as mpk_run, bit for bit,
 * since every node uses the same chunks and the same arithmetic.  Errors:
 * MPK_ERR_ARG for a bad granularity or buffer, MPK_ERR_STATE without upload,
 * MPK_ERR_UNSUPPORTED for an nrhs/dtype combination without a kernel. */
#define MPK_SYNC_NODE 0
#define MPK_SYNC_WAVEFRONT 1
mpk_status mpk_run_sync(mpk_plan *plan, const double *X, double *Y, int32_t granularity, void *stream);

/* Waits for `stream` and reports whether the last mpk_run on this plan hit
 * the watchdog (MPK_ERR_TIMEOUT) or succeeded (MPK_OK). */
mpk_status mpk_plan_status(mpk_plan *plan, void *stream);

/* Release host and device memory of a plan (NULL is ignored). */
void mpk_plan_destroy(mpk_plan *plan);

/* Baseline SpMV on a matrix in its given order (Sec. 3.1, Fig. 2).  The CSR
 * is validated, copied to the current device (values converted to
 * opt->val_dtype) and kept by the handle.  opt may be NULL. */
mpk_status spmv_create(const mpk_csr *A, const mpk_options *opt, mpk_spmv **out);
/* y = A x (device, N x k). */
mpk_status spmv_run(mpk_spmv *h, const double *x, double *y, void *stream);
/* p back-to-back SpMVs: Y[q-1] = A Y[q-2], Y[-1] = X (device). */
mpk_status spmv_powers_run(mpk_spmv *h, int32_t p, const double *X, double *Y, void *stream);
void spmv_destroy(mpk_spmv *h);

/* Load-only bandwidth probe (the analog of the paper's Fig. 1): reads
 * `bytes` (device, 16-byte aligned, multiple of 16) `reps` times with a grid
 * of `workgroups` x 256 threads and returns the sum of what it read in
 * *sink (device, one double).  Time it with events on `stream`. */
mpk_status mpk_bw_probe(const void *buf, uint64_t bytes, int32_t reps, int32_t workgroups,
                        double *sink, void *stream);

/* The same probe with `loads_per_thread` (1, 2, 4 or 8) independent 16-byte
 * loads per thread in flight and the buffer cut into `parts` (1 or 8) equal
 * contiguous parts: workgroup b reads part b % parts only.  On MI355X the
 * workgroups b, b + 8, ... of a launch share one XCD, so with parts = 8 each
 * XCD re-reads its own part: a part larger than the XCD's 4 MB L2 inside a
 * buffer smaller than the 256 MB Infinity Cache measures the Infinity Cache
 * (the memory hierarchy levels of Sec. 2, Fig. 1).  bytes must be a multiple
 * of 16*parts, buf 16-byte aligned (device), workgroups >= parts. */
mpk_status mpk_bw_probe_ex(const void *buf, uint64_t bytes, int32_t reps, int32_t workgroups,
                           int32_t loads_per_thread, int32_t parts, double *sink, void *stream);

/* XCD placement: ids[b] (device, `workgroups` int32) receives the hardware
 * XCD index (XCC_ID register) of workgroup b of a launch of `workgroups`
 * 256-thread workgroups, each of which then sleeps `spin` rounds so that the
 * later ones are placed while the earlier ones still run.  Measured on
 * MI355X: ids[b] = (b + r) % 8, the dispatcher continuing its round-robin
 * over the XCDs from the previous launch (r = 0 in a fresh process).  The
 * XCD-sliced ticket streams (mpk_options.xcd_streams = 8) need only that the
 * workgroups b, b + 8, ... share an XCD. */
mpk_status mpk_xcd_ids(int32_t *ids, int32_t workgroups, int64_t spin, void *stream);

/* Latency of a point-to-point dependency hop (Sec. 4.3 replaces barriers by
 * such hops): workgroups 0 and `peer` (1..255) of one launch pass a counter
 * back and forth through two flags in `flags` (device, 64 uint32, cleared by
 * the call), `iters` round trips.  scope 0: agent-scope flag stores and
 * loads (the device-coherent level, as mpk_run uses them); scope 1:
 * workgroup-scope stores and loads, which bypass the L1 and meet in the L2
 * of one XCD (peer = 8 shares workgroup 0's XCD; with another XCD they never
 * meet).  Every poll gives up after max_polls reads.  out (device, 2
 * uint64): elapsed wall-clock ticks of workgroup 0 and the round trips
 * completed (iters unless a poll gave up); wall_clock_khz (host, may be NULL)
 * receives the tick rate.  The flags are cleared with a memset on `stream`,
 * so the call is not meant for stream capture. */
mpk_status mpk_hop_probe(uint32_t *flags, int32_t peer, int32_t scope, int32_t iters, int64_t max_polls,
                         uint64_t *out, int32_t *wall_clock_khz, void *stream);

/* ---- learned tuner: a 3-layer perceptron, FP32, on the device -------------
 * out = w3 . relu(W2 relu(W1 x + b1) + b2) + b3 with D inputs and H hidden
 * units (H <= 256).  Parameters are one float array laid out W1[H][D], b1[H],
 * W2[H][H], b2[H], w3[H], b3 (mpk_mlp_param_count(D, H) floats).  All arrays
 * are device memory; calls are asynchronous on `stream`. */
int64_t mpk_mlp_param_count(int32_t D, int32_t H);
/* Forward pass for B samples X[B][D]: out[B]; cache[B][2H] keeps the
 * pre-activations for the backward pass. */
mpk_status mpk_mlp_forward(const float *params, int32_t D, int32_t H, const float *X, int32_t B, float *out,
                           float *cache, void *stream);
/* Gradient of the mean squared error (1/B) sum (out - y)^2 with respect to
 * every parameter, into grads[param_count]; work needs B*(2H+1) floats;
 * loss (one float, may be NULL) receives the loss.  Sums over the batch run
 * in sample order, so results are deterministic. */
mpk_status mpk_mlp_backward(const float *params, int32_t D, int32_t H, const float *X, const float *y, int32_t B,
                            const float *out, const float *cache, float *work, float *grads, float *loss,
                            void *stream);
/* mpk_mlp_backward without the workspace argument, for callers that cannot
 * allocate device memory (code under HIP stream capture, serving loops,
 * harnesses that forbid hipMalloc): the B*(2H+1) floats of work live in a
 * fixed per-GPU array of the library (16 MiB, held until the process ends),
 * so the call allocates nothing.  B*(2H+1) must be <= 4194304 (MPK_ERR_ARG
 * otherwise).  Same arguments and results as mpk_mlp_backward, bit for bit.
 * All calls on one GPU share that array: calls that overlap on one GPU (on
 * different streams or threads) race. */
mpk_status mpk_mlp_backward_noalloc(const float *params, int32_t D, int32_t H, const float *X, const float *y,
                                    int32_t B, const float *out, const float *cache, float *grads, float *loss,
                                    void *stream);
/* One Adam step (step = 1, 2, ...): m, v are the moment buffers (zero before
 * step 1), bias-corrected update params -= lr mhat / (sqrt(vhat) + eps). */
mpk_status mpk_mlp_adam(float *params, const float *grads, float *m, float *v, int64_t n, float lr, float beta1,
                        float beta2, float eps, int32_t step, void *stream);

const char *mpk_status_string(mpk_status s);
const char *mpk_last_error(void);
/* Library version string. */
const char *mpk_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MPK_H_ */
