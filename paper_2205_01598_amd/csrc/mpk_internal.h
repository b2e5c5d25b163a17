// Internal definitions shared by the host planner (plan.cpp) and the HIP
// side of the library (mpk_device.hip).  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mpk.h"

namespace mpk {

// Thread-local error message behind mpk_last_error().
void set_error(const std::string &msg);
mpk_status fail(mpk_status s, const std::string &msg);

// Host-side state of a plan, filled by the planner.
struct HostPlan {
    int64_t n = 0, nnz = 0;
    int32_t p = 1;
    uint64_t cache_bytes = 0;
    mpk_options opt{};
    int64_t root = 0;

    std::vector<int32_t> perm;       // new -> old
    std::vector<int32_t> iperm;      // old -> new
    std::vector<int32_t> level_ptr;  // L+1
    std::vector<int64_t> level_nnz;  // L
    std::vector<int32_t> group_ptr;  // G+1, indices into levels
    std::vector<int32_t> schedule;   // 3*G*p: (d, p, i)

    // renumbered matrix P A P^T, columns ascending per row
    std::vector<int32_t> rowptr;     // n+1 (nnz < 2^31)
    std::vector<int32_t> col;
    std::vector<double> val;

    // device tiles: row ranges inside level groups
    std::vector<int32_t> tile_row;   // n_tiles+1
    std::vector<int32_t> tile_group; // n_tiles
    std::vector<int32_t> dep_lo, dep_hi;  // n_tiles: all tiles a tile waits for
    std::vector<int32_t> dep3;       // 6*n_tiles: (lo, hi) in groups g-1, g, g+1 (lo > hi: none)
    std::vector<int32_t> dep3x;      // the same ranges widened to whole cache lines
    // recursive plans (Sec. 4.4): final groups ("units") of the refined
    // numbering, and per-tile dependency lists of tile ranges
    bool recursive = false;
    std::vector<int32_t> unit_ptr;   // n_units+1 row boundaries
    std::vector<int32_t> unit_stage; // n_units
    std::vector<int64_t> unit_key;   // n_units: wavefront key of the unit's position
    std::vector<int32_t> dep_ptr;    // n_tiles+1 into dep_rng pairs
    std::vector<int32_t> dep_rng;    // (lo, hi) inclusive tile ranges, line-closed
    bool line_closed_ok = false;     // every widened dependency is an earlier ticket
    std::vector<int32_t> group_tile; // G+1
    std::vector<int32_t> work;       // tickets: tile*64 + (q-1)
    std::vector<int32_t> stream_ptr; // xcd_streams+1: ticket streams, each in `work` order
    std::vector<int32_t> work_streams;  // the tickets regrouped by stream
    std::vector<int32_t> chunk_row;  // n_chunks+1: kernel work units inside tiles
    std::vector<int32_t> tile_chunk; // n_tiles+1

    // Plans created from a CSR in device memory keep P A P^T on the GPU only:
    // col and val above stay empty, rowptr is the host copy of the device row
    // pointers, and the tile dependencies are found on the device.
    const int32_t *dev_rowptr = nullptr;  // device, n+1
    const int32_t *dev_col = nullptr;     // device, nnz

    int64_t max_level_rows = 0, max_group_nnz = 0, violating_groups = 0;
    int32_t tile_nnz = 0;
    double plan_seconds = 0.0;
    double phase_seconds[4] = {0, 0, 0, 0};
};

// The fields build_schedule rewrites (saved so a failed retune can restore them).
struct ScheduleState {
    int32_t p;
    uint64_t cache_bytes;
    mpk_options opt;
    bool line_closed_ok;
    std::vector<int32_t> dep_ptr, dep_rng;
    std::vector<int32_t> group_ptr, schedule, tile_row, tile_group, dep_lo, dep_hi, dep3, dep3x, group_tile, work,
        stream_ptr, work_streams, chunk_row, tile_chunk;
    int64_t max_group_nnz, violating_groups;
    int32_t tile_nnz;
};
void save_schedule(HostPlan &hp, ScheduleState &s);     // moves the fields out
void restore_schedule(HostPlan &hp, ScheduleState &s);  // moves them back

// Runs every host step of the plan.  Returns MPK_OK or an error (message set).
mpk_status build_host_plan(const mpk_csr *A, int32_t p, uint64_t cache_bytes,
                           const mpk_options &opt, HostPlan &hp);

// The renumbered matrix P A P^T of a plan made from device memory, in device
// memory allocated with hipMalloc (freed with hipFree by its owner).
struct ResidentMatrix {
    int32_t *rowptr = nullptr;  // n+1
    int32_t *col = nullptr;     // nnz
    double *val = nullptr;      // nnz, FP64
};

// The plan of a CSR whose rowptr/col/val are device pointers on the current
// GPU (rows sorted, pattern symmetric): graph, levels and P A P^T on the GPU
// (device_plan_resident), then the schedule; M receives the device matrix
// and hp.dev_rowptr/dev_col point into it.
mpk_status build_resident_plan(const mpk_csr *A_dev, int32_t p, uint64_t cache_bytes, const mpk_options &opt,
                               HostPlan &hp, ResidentMatrix *M);

// The part of the plan that depends on p, the cache budget and the launch
// options (level groups, schedule, tiles, dependencies, tickets); reuses the
// levels and renumbered matrix already in hp.
mpk_status build_schedule(HostPlan &hp, int32_t p, uint64_t cache_bytes, const mpk_options &opt);

// Matrix/plan features for the learned tuner (MPK_NUM_FEATURES values).
void plan_features(const HostPlan &hp, double *f);

// Validation shared by plan and SpMV creation.
mpk_status validate_csr(const mpk_csr *A);

// Cuts rows [r0, r1) into chunks of at most max_nnz stored nonzeros and
// max_rows rows (a longer single row forms its own chunk); appends the start
// row of every chunk to `out`.
void append_chunks(const std::vector<int32_t> &rowptr, int64_t r0, int64_t r1, int64_t max_nnz,
                   int64_t max_rows, std::vector<int32_t> &out);
void append_chunks64(const int64_t *rowptr, int64_t r0, int64_t r1, int64_t max_nnz, int64_t max_rows,
                     std::vector<int32_t> &out);

// Products each of a chunk's 256 threads forms, for k right-hand sides.  The
// persistent MPK kernel (and the bulk-synchronous kernels, which run on the
// same tile chunks) takes 16 at k = 1 (more loads in flight per wavefront
// at 3 workgroups per CU); the baseline SpMV, one workgroup per chunk, is
// fastest at 12 there.  At k = 2 both take 8: the recurrence epilogue needs
// the registers (the SpMV with FP32 products, i.e. FP32 or BF16 values with
// FP32 arithmetic, takes 16).  For k >= 4 both take 16.  Host (chunk
// cutting) and device (chunk kernel) use the same values.
constexpr int32_t mpk_products_per_thread(int32_t k) { return k == 2 ? 8 : 16; }
constexpr int32_t spmv_products_per_thread(int32_t k, bool f32_products) {
    return k == 1 ? 12 : (k == 2 && !f32_products) ? 8 : 16;
}
// Nonzeros per kernel chunk for k right-hand sides.
constexpr int32_t mpk_chunk_nnz(int32_t k) { return 256 * mpk_products_per_thread(k) / k; }
constexpr int32_t spmv_chunk_nnz(int32_t k, bool f32_products) {
    return 256 * spmv_products_per_thread(k, f32_products) / k;
}
// FP32 products: FP32 or BF16 values without accum_f64
constexpr bool fp32_products(int32_t val_dtype, int32_t accum_f64) { return val_dtype != MPK_F64 && !accum_f64; }
// rows per chunk cap: bounds the chunk's row-pointer slice kept in LDS
constexpr int32_t kChunkRows = 1024;
// A ticket is the int32 tile * 64 + (power - 1) (powers <= 32 < 64), so a
// plan holds fewer than 2^25 tiles.
constexpr int64_t kMaxTiles = int64_t(1) << 25;

// Breadth-first levels and root on the current GPU (plan_device.hip): the
// same root, permutation and level pointers as the host planner, from the
// undirected graph (ptr[n+1], adj[ptr[n]], lists ascending, no diagonal).
mpk_status device_bfs_levels(int64_t n, const int64_t *ptr, const int32_t *adj, int32_t root_mode, int64_t *root_out,
                             std::vector<int32_t> &perm, std::vector<int32_t> &level_ptr);

// Graph, levels and renumbered matrix P A P^T on the current GPU
// (plan_device.hip) for a pattern whose rows are sorted and symmetric; the
// same results as the host planner.  *handled = false (and nothing filled)
// for other patterns.  phase_seconds[0..2]: graph, levels, renumbering.
mpk_status device_plan(const mpk_csr *A, int32_t root_mode, int64_t *root_out, std::vector<int32_t> &perm,
                       std::vector<int32_t> &level_ptr, std::vector<int32_t> &rowptr, std::vector<int32_t> &col,
                       std::vector<double> &val, bool *handled, double *phase_seconds);

// Graph, levels and P A P^T on the current GPU for a CSR already in device
// memory (plan_device.hip).  The CSR is validated on the device
// (MPK_ERR_CSR); rows must be sorted with a symmetric pattern, and no row of
// A may hold more than kResidentRowMax entries (MPK_ERR_UNSUPPORTED).  Host
// copies of perm, level_ptr and the new row pointers; M receives the device
// matrix (on error nothing is left allocated).  phase_seconds[0..2]: graph,
// levels, renumbering.
constexpr int64_t kResidentRowMax = 4096;
mpk_status device_plan_resident(const mpk_csr *A_dev, int32_t root_mode, int64_t *root_out,
                                std::vector<int32_t> &perm, std::vector<int32_t> &level_ptr,
                                std::vector<int32_t> &rowptr, ResidentMatrix *M, double *phase_seconds);

// For every tile t (rows [tile_row[t], tile_row[t+1]) of group g =
// tile_group[t]) and m = 0, 1, 2: the smallest and largest column the tile
// reads among the rows [group_row[g-1+m], group_row[g+m]) of group g-1+m,
// from the device matrix (rowptr, col): out[6t+2m] = smallest (INT32_MAX if
// none), out[6t+2m+1] = largest (-1 if none).  *bad = true if a column lies
// outside the three groups.
mpk_status device_tile_columns(const int32_t *d_rowptr, const int32_t *d_col, const std::vector<int32_t> &tile_row,
                               const std::vector<int32_t> &tile_group, const std::vector<int32_t> &group_row,
                               std::vector<int32_t> &out, bool *bad);

// Bytes per stored nonzero for Eq. (5): value bytes + 4 (int32 column).
int32_t bytes_per_nnz(int32_t dtype);

}  // namespace mpk
