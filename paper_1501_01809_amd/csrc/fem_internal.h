// Internal declarations of the HIP cell-loop assembler (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <thread>
#include <vector>

#include "fem.h"

// Where a context's device memory comes from (fem_ctx_set_allocator): the
// caller's allocator, or the HIP runtime (hipMalloc for what a plan holds,
// stream-ordered hipMallocAsync on the context stream for temporaries).
struct fem_mem {
    void *(*alloc)(size_t, void *) = nullptr;
    void (*release)(void *, void *) = nullptr;
    void *user = nullptr;
};

struct fem_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cus = 256;
    fem_mem mem;
    void *scratch = nullptr;     // this device's static scratch (fem_build_sparsity_noalloc)
    size_t scratch_bytes = 0;
    std::string err;
};

// Plan of the row-owned deterministic INC (see fem_plan_create in fem.h).
//
// Rows are split into contiguous blocks; a workgroup owns one block and
// visits the ascending list of cells incident to its rows (bcell, with their
// vertex ids in bverts).
//  * Dat/action plans: every row's incident entries (inc_ptr / ent, ascending
//    cell) name a cell of the block list (local index) and the row's local
//    index in that cell.
//  * Mat plans: the block's cells (at most Limits::cell_cap) are processed in
//    chunks of at most Limits::chunk_cells cells whose packed element tensors
//    sit in LDS together with the block's Mat values.  Every lane of the workgroup owns a set of the block's Mat
//    values and walks its own stream of 16-bit LDS indices: an index below
//    the value area's size opens that value (the running sum restarts from
//    the value held there), any other index adds one element-tensor entry
//    (or -0.0, the identity, for padding).  A value's entries come in
//    ascending cell id, the same order in every block, so the sums are
//    reproducible and an assembled symmetric form is bitwise symmetric.
//    The stream of (chunk q, wave w) of a block starts at batch index
//    wq[blk_w[b] + W q + w] (W waves per workgroup) and ends where the next
//    one starts; inside it,
//    batch i of lane l is the batch at start + 64 i + l (femk::MAT_BATCH
//    indices, two per 32-bit word, the first in the low half).
struct fem_plan {
    int is_mat = 0;
    int dim = 0, degree = 0, nloc = 0;
    int64_t ncells = 0, nrows = 0, nverts = 0;
    int64_t nnz = 0;
    int32_t nblk = 0;
    int lbits = 0;               // bits of the local index
    int64_t nchunks = 0;         // Mat plans: chunks over all blocks
    int64_t stream_entries = 0;  // Mat plans: 16-bit stream entries (padding included)
    int64_t cell_visits = 0;     // sum over blocks of cells gathered
    int32_t max_blk_cells = 0;   // most cells any block gathers
    double *red_partial = nullptr;  // Dat plans: one partial per 1024 cells (Global reductions)
    // Exterior facet plans (is_mat == 3; ncells = facets): node-to-facet
    // incidence (entries f*nloc + l, ascending) and the facet vectors.
    int64_t *f_ptr = nullptr;
    int32_t *f_ent = nullptr;
    double *f_work = nullptr;
    // Elasticity plans (is_mat == 2): per node pair of the node sparsity (a
    // 3x3 block of the vector CSR), its contributions in ascending cell id,
    // and the element-block workspace [ncells][55][9] (float64 for FEM_FP64,
    // float32 for FEM_FP32; [ncells][55][10] 16-bit values for FEM_BF16 and
    // FEM_FP16).
    int32_t *e_slot_ptr = nullptr;  // [nslots+1]
    uint32_t *e_ent = nullptr;      // (cell << 8) | (pair << 2) | (diagonal << 1) | transposed
    int32_t *e_grow = nullptr;      // [nslots/64 + 1] node row of slot 64 g
    void *e_work = nullptr;
    int64_t e_nslots = 0;
    int e_prec = 0;
    size_t bytes = 0;            // device bytes held
    fem_mem mem;                 // allocator the arrays below came from
    // device arrays (owned)
    int32_t *blk_row0 = nullptr;  // [nblk+1] first row of each block
    int32_t *blk_cptr = nullptr;  // [nblk+1] offsets into bcell
    int32_t *bcell = nullptr;     // ascending global cell ids of each block
    int32_t *bverts = nullptr;    // [visits][dim+1] vertex ids of each bcell entry
    int32_t *inc_ptr = nullptr;   // Dat plans: [nrows+1] entry range of each row
    uint16_t *ent = nullptr;      // Dat plans: (local cell << lbits) | local index
    int32_t *blk_hdr = nullptr;   // Mat plans: [nblk][8] block header (layout in fem_assemble.hip)
    int32_t *blk_w = nullptr;     // Mat plans: [nblk+1] first (chunk, wave) stream of each block
    int32_t *wq = nullptr;        // Mat plans: [streams+1] first batch of each (chunk, wave) stream
    uint16_t *pstream = nullptr;  // Mat plans: the streams
    // identity of what the plan was built for: the Maps' arrays and versions
    const int32_t *cell_node = nullptr;
    const int32_t *cell_vertex = nullptr;
    uint64_t cn_version = 0, cv_version = 0;
    const int64_t *row_ptr = nullptr;
    const int32_t *col_idx = nullptr;
};

namespace femk {

// 16-bit indices per Mat stream batch (one 16- or 8-byte load per lane).
// Batches of 4 cut the rounding padding (P2 tetrahedra: plan 702 -> 661 MB)
// but measured slower everywhere (P2 tetrahedra 503 -> 535 us): twice the
// load instructions and half the LDS reads in flight per batch.
#ifndef FEM_MAT_BATCH
#define FEM_MAT_BATCH 8
#endif
constexpr int MAT_BATCH = FEM_MAT_BATCH;
static_assert(MAT_BATCH == 4 || MAT_BATCH == 8, "Mat stream batch width");

// ---- device memory (fem_api.cpp) ----
// Persistent (plan) or temporary (freed before the call returns, stream-
// ordered on s) device memory from m; release with the same m, s and temp.
hipError_t mem_alloc(const fem_mem &m, hipStream_t s, bool temp, size_t bytes, void **p);
void mem_free(const fem_mem &m, hipStream_t s, bool temp, void *p);

// ---- incidence and sparsity (fem_sparsity.hip) ----
// Device address and size of the static scratch array on `device`, looked up
// once per device (that device must be current at the first call).
hipError_t static_scratch(int device, void **ptr, size_t *bytes);
hipError_t check_range(const int32_t *v, int64_t n, int64_t limit, int *flag, hipStream_t s);
// Fills n int32 with value (a kernel, not a memset node).
hipError_t fill_i32(int32_t *p, int64_t n, int32_t value, hipStream_t s);
// int64 elements of scratch an exclusive scan of n values needs.
int64_t scan_scratch(int64_t n);
// Row -> incidence: ptr (int64 [nrows+1]) and ent (int32 entry ids c*nloc+l,
// ascending within each row).  tmp must hold nrows+1 int32, scan
// scan_scratch(nrows) int64.
hipError_t build_incidence(const int32_t *map, int64_t ncells, int nloc, int64_t nrows,
                           int64_t *ptr, int32_t *ent, int32_t *tmp, int64_t *scan, hipStream_t s);
// Unique column counts per row (count pass) or columns (fill pass).
hipError_t row_columns(const int64_t *inc_ptr, const int32_t *inc_ent, int nloc_r,
                       const int32_t *cmap, int nloc_c, int64_t nrows, int32_t *counts,
                       const int64_t *row_ptr, int32_t *col_idx, int *overflow, hipStream_t s);
// out[0..n] = exclusive prefix sums of in[0..n) (out[n] the total); scan
// holds scan_scratch(n) int64.
hipError_t exclusive_scan(const int32_t *in, int64_t *out, int64_t n, int64_t *scan, hipStream_t s);
hipError_t i64_to_i32(const int64_t *in, int32_t *out, int64_t n, hipStream_t s);

// ---- assembly kernels (fem_assemble.hip) ----
struct AsmArgs {
    const fem_plan *plan;
    const int32_t *cell_vertex;
    const double *coords;
    const int32_t *cell_node;
    const double *coeff;     // kappa (bilinear) or f (source)
    double cstiff, cmass;
    const int64_t *row_ptr;
    const double *x;         // action input; u of the nonlinear residual
    const double *aux;       // nonlinear residual: f (residual) or lambda (adjoint)
    double *out;             // Mat values / Dat
    double *out2;            // nonlinear residual, mode 3: lambda^T dF/dkappa
    int inc;                 // 1: INC, 0: WRITE
    int num_cus;             // compute units of the device (persistent grids)
};
hipError_t launch_mat(const AsmArgs &a, hipStream_t s);
// Batched launch (request server): the Mat (op 0), source vector (op 1) or
// action (op 2) work of nreq requests whose plans share (dim, degree), in one
// launch of at most grid workgroups (twice that for the Dat kernels), each
// taking work items from a device counter.  desc: device memory of
// batch_desc_bytes(nreq) bytes, filled from the pinned host buffer hdesc (same
// size) by an asynchronous copy on s; neither may be reused before the
// launch has completed.
size_t batch_desc_bytes(int nreq);
hipError_t launch_batch(int op, const AsmArgs *reqs, int nreq, int grid, void *hdesc, void *desc, hipStream_t s);
hipError_t launch_vec(const AsmArgs &a, hipStream_t s);
hipError_t launch_action(const AsmArgs &a, hipStream_t s);
// Nonlinear residual (mode 0: F from u = x, kappa = coeff, f = aux) and its
// vector-Jacobian products (1: lambda^T dF/du, 2: lambda^T dF/dkappa, with
// lambda = aux; 3: both, into out and out2); P1 Dat plans; fp32 selects
// binary32 arithmetic.
hipError_t launch_nl(const AsmArgs &a, int mode, bool fp32, hipStream_t s);

// Global reductions over the cells (fem_global.hip): SUM / MIN / MAX (mode
// 0 / 1 / 2) of the cell energies x_K^T A_K x_K (energy) or of the integrals
// of f = coeff (not energy) into g[0]; partial holds reduce_partials(ncells).
int64_t reduce_partials(int64_t ncells);
hipError_t launch_reduce(const AsmArgs &a, double *partial, int mode, bool energy, double *g, hipStream_t s);

// Dirichlet rows and columns (fem_bc.hip).
hipError_t launch_dirichlet(const fem_sparsity *sp, double *values, const uint8_t *mask, double diag, double *b,
                            const double *g, hipStream_t s);

// Vector P2 linear elasticity (fem_elast.hip): argument checks, plan and
// assembly (element blocks by MFMA, then the pull into the CSR).
fem_status elast_check(fem_ctx *ctx, const fem_form *form, const fem_args *args);
fem_status elast_plan_create(fem_ctx *ctx, const fem_form *form, const fem_args *args, const fem_sparsity *sp,
                             fem_plan **out);
fem_status elast_assemble(fem_ctx *ctx, const fem_plan *plan, const fem_form *form, const fem_args *args,
                          fem_mat *A, fem_access acc);

// Per-(dim, degree) launch limits used by the plan builder.
struct Limits {
    int rows_per_block;     // rows a workgroup can own
    int slot_cap;           // Mat values a workgroup holds in LDS (Mat only)
    int cell_cap;           // distinct cells per block
    int chunk_cells;        // Mat: cells whose element tensors share LDS at once (one chunk)
    int ne;                 // doubles per packed element tensor (Mat only)
    int lanes;              // Mat: lanes of the workgroup (the streams are dealt to them)
};
bool limits(int dim, int degree, bool is_mat, Limits *out);

// Host threads for the setup passes (plans, renumbering): the machine's, at
// most 16.
inline int host_threads()
{
    const unsigned h = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(16u, h));
}

// Runs job(t) for t in [0, nt): t = 0 on the calling thread, the others on
// threads of their own (a job whose thread cannot be started runs on the
// calling thread instead).  Every thread is joined before returning; a job
// must not throw (jobs catch their own failures and report them).
template <typename J>
void run_jobs(int nt, J job)
{
    std::vector<std::thread> pool;
    std::vector<int> inline_jobs;
    for (int t = 1; t < nt; ++t) {
        try {
            pool.emplace_back(job, t);
        } catch (...) {
            inline_jobs.push_back(t);
        }
    }
    job(0);
    for (int t : inline_jobs) job(t);
    for (std::thread &th : pool) th.join();
}

// Runs fn(lo, hi) over [0, n) split into contiguous ranges, one per host
// thread (one range when n is small); fn must not throw.
template <typename F>
void par_ranges(int64_t n, F fn)
{
    const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), n / 65536));
    run_jobs(nt, [&](int t) { fn(n * t / nt, n * (t + 1) / nt); });
}

// The status of a C++ exception caught at the C boundary: host allocation
// failures are FEM_E_NOMEM, anything else FEM_E_DEVICE.
fem_status caught_status(fem_ctx *ctx, const char *where);


}  // namespace femk
