// C ABI of the cell-loop assembler: validation, context, sparsity, plans,
// renumbering and kernel dispatch.  See include/fem.h for the contract.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <exception>
#include <new>
#include <atomic>
#include <numeric>
#include <thread>
#include <vector>

#include "fem_internal.h"

namespace {

fem_status fail(fem_ctx *ctx, fem_status st, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}

fem_status hip_fail(fem_ctx *ctx, hipError_t e, const char *what)
{
    return fail(ctx, e == hipErrorOutOfMemory ? FEM_E_NOMEM : FEM_E_DEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

#define HIPC(call, what)                                      \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
    } while (0)

int nloc_of(int dim, int degree)
{
    if (degree < 1 || degree > 3) return -1;
    if (dim == 2) return (degree + 1) * (degree + 2) / 2;
    if (dim == 3) return (degree + 1) * (degree + 2) * (degree + 3) / 6;
    return -1;
}

bool map_ok(const fem_map *m)
{
    return m && m->from && m->to && m->arity > 0 && m->from->size >= 0 && m->to->size >= 0 &&
           (m->values || m->from->size == 0);
}

bool dat_ok(const fem_dat *d, const fem_set *set, int dim)
{
    return d && d->set && d->dim == dim && d->set->size == set->size && (d->data || set->size == 0);
}

// Temporary device buffer of a setup call, from the context's allocator,
// released at scope exit (stream-ordered on the context stream).
struct DevBuf {
    void *p = nullptr;
    const fem_ctx *ctx;
    explicit DevBuf(const fem_ctx *c) : ctx(c) {}
    hipError_t alloc(size_t bytes) { return femk::mem_alloc(ctx->mem, ctx->stream, true, bytes ? bytes : 8, &p); }
    ~DevBuf() { if (p) femk::mem_free(ctx->mem, ctx->stream, true, p); }
    template <typename T> T *as() const { return (T *)p; }
};

// Carves a caller's scratch buffer into 256-byte aligned pieces (or sizes it
// when base is NULL).
struct Carve {
    char *base;
    size_t off = 0;
    explicit Carve(void *b) : base((char *)b) {}
    template <typename T> T *take(int64_t n)
    {
        T *q = base ? (T *)(base + off) : nullptr;
        off += ((size_t)(n > 0 ? n : 1) * sizeof(T) + 255) / 256 * 256;
        return q;
    }
};

fem_status check_form(fem_ctx *ctx, const fem_form *f)
{
    if (!f) return fail(ctx, FEM_E_ARG, "form is NULL");
    // exact integration: the integrand's polynomial degree (P1 coefficients)
    const int qexact = f->kind == FEM_ELASTICITY ? 3 : f->kind == FEM_NL_RESIDUAL ? 4
                       : f->kind == FEM_SOURCE ? f->degree + 1 : 2 * f->degree;
    if (f->qdegree < 0 || (f->qdegree > 0 && f->qdegree < qexact))
        return fail(ctx, FEM_E_UNSUPPORTED,
                    "quadrature degree %d: the kernels integrate exactly (degree %d for this form); "
                    "an under-integrated rule is not provided", f->qdegree, qexact);
    if (f->kind == FEM_ELASTICITY) {
        if (f->prec < FEM_FP64 || f->prec > FEM_FP16)
            return fail(ctx, FEM_E_UNSUPPORTED, "precision %d not supported", (int)f->prec);
        return FEM_OK;   // shape, degree and value dimension: femk::elast_check
    }
    if (f->cell != FEM_TRIANGLE && f->cell != FEM_TETRAHEDRON)
        return fail(ctx, FEM_E_UNSUPPORTED, "cell %d not supported", (int)f->cell);
    if (f->degree < 1 || f->degree > 3)
        return fail(ctx, FEM_E_UNSUPPORTED, "degree %d not supported (1..3)", f->degree);
    if (f->dim != 1) return fail(ctx, FEM_E_UNSUPPORTED, "value dimension %d not supported", f->dim);
    if (f->kind < FEM_MASS || f->kind > FEM_NL_RESIDUAL)
        return fail(ctx, FEM_E_UNSUPPORTED, "form kind %d not supported", (int)f->kind);
    if (f->kind == FEM_NL_RESIDUAL && f->degree != 1)
        return fail(ctx, FEM_E_UNSUPPORTED, "the nonlinear residual is provided for P1 only");
    if (!(f->prec == FEM_FP64 || (f->prec == FEM_FP32 && f->kind == FEM_NL_RESIDUAL)))
        return fail(ctx, FEM_E_UNSUPPORTED, "precision %d not supported for form kind %d", (int)f->prec,
                    (int)f->kind);
    return FEM_OK;
}

fem_status check_args(fem_ctx *ctx, const fem_form *f, const fem_args *a, bool need_coeff)
{
    if (!a || !a->cells || !a->cell_vertex || !a->coords || !a->cell_node)
        return fail(ctx, FEM_E_ARG, "args: cells, cell_vertex, coords and cell_node are required");
    if (a->cell_coord)
        return fail(ctx, FEM_E_UNSUPPORTED, "args: a separate coordinate Map is provided for FEM_ELASTICITY only");
    const int d = (int)f->cell;
    const int nl = nloc_of(d, f->degree);
    if (!map_ok(a->cell_vertex) || !map_ok(a->cell_node))
        return fail(ctx, FEM_E_ARG, "args: malformed Map");
    if (a->cells->size < 0) return fail(ctx, FEM_E_ARG, "args: negative cell count");
    if (a->cell_vertex->from->size != a->cells->size || a->cell_node->from->size != a->cells->size)
        return fail(ctx, FEM_E_ARG, "args: Maps must start from the cell Set");
    if (a->cell_vertex->arity != d + 1)
        return fail(ctx, FEM_E_ARG, "args: cell_vertex arity %d, expected %d", a->cell_vertex->arity, d + 1);
    if (a->cell_node->arity != nl)
        return fail(ctx, FEM_E_ARG, "args: cell_node arity %d, expected %d for degree %d",
                    a->cell_node->arity, nl, f->degree);
    if (!dat_ok(a->coords, a->cell_vertex->to, d))
        return fail(ctx, FEM_E_ARG, "args: coords must be a dim-%d Dat on the vertex Set", d);
    if (a->ncoeff < 0 || a->ncoeff > 4) return fail(ctx, FEM_E_ARG, "args: ncoeff out of range");
    if (need_coeff) {
        if (a->ncoeff < 1 || !dat_ok(a->coeff[0], a->cell_vertex->to, 1))
            return fail(ctx, FEM_E_ARG, "args: coeff[0] must be a scalar P1 Dat on the vertex Set");
    }
    if (a->cells->size * (int64_t)nl > INT32_MAX || a->cell_node->to->size > INT32_MAX ||
        a->cell_vertex->to->size > INT32_MAX)
        return fail(ctx, FEM_E_OVERFLOW, "args: more than 2^31-1 cell-node entries or nodes");
    return FEM_OK;
}

void form_coeffs(fem_kind k, double *cstiff, double *cmass)
{
    *cstiff = (k == FEM_LAPLACE || k == FEM_HELMHOLTZ) ? 1.0 : 0.0;
    *cmass = (k == FEM_MASS || k == FEM_HELMHOLTZ) ? 1.0 : 0.0;
}

fem_status range_check(fem_ctx *ctx, const fem_map *m, int *dflag, const char *name)
{
    int hflag = 0;
    HIPC(femk::fill_i32(dflag, 1, 0, ctx->stream), "clear flag");
    HIPC(femk::check_range(m->values, m->from->size * (int64_t)m->arity, m->to->size, dflag, ctx->stream),
         "range check");
    HIPC(hipMemcpyAsync(&hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream), "copy");
    HIPC(hipStreamSynchronize(ctx->stream), "sync");
    if (hflag) return fail(ctx, FEM_E_RANGE, "%s: a Map entry lies outside its target Set", name);
    return FEM_OK;
}

void free_plan_arrays(fem_plan *p)
{
    void *arrs[] = {p->blk_row0, p->blk_cptr, p->bcell, p->bverts, p->inc_ptr, p->ent,
                    p->blk_hdr, p->blk_w, p->wq, p->pstream,
                    p->e_slot_ptr, p->e_ent, p->e_grow, p->e_work, p->red_partial,
                    p->f_ptr, p->f_ent, p->f_work};
    for (void *q : arrs)
        if (q) femk::mem_free(p->mem, nullptr, false, q);
}

template <typename T>
hipError_t upload(const fem_mem &m, T **dst, const std::vector<T> &src, size_t *bytes, hipStream_t s)
{
    size_t n = src.size() * sizeof(T);
    hipError_t e = femk::mem_alloc(m, s, false, n ? n : 8, (void **)dst);
    if (e != hipSuccess) return e;
    *bytes += n;
    if (n) e = hipMemcpyAsync(*dst, src.data(), n, hipMemcpyHostToDevice, s);
    return e;
}

// ---- Hilbert index (J. Skilling, "Programming the Hilbert curve", 2004):
// coordinates -> transposed Hilbert form -> bit-interleaved index.
uint64_t hilbert_index(uint32_t X[3], int n, int b)
{
    const uint32_t M = 1u << (b - 1);
    for (uint32_t Q = M; Q > 1; Q >>= 1) {
        const uint32_t P = Q - 1;
        for (int i = 0; i < n; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                const uint32_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    for (int i = 1; i < n; ++i) X[i] ^= X[i - 1];
    uint32_t t = 0;
    for (uint32_t Q = M; Q > 1; Q >>= 1)
        if (X[n - 1] & Q) t ^= Q - 1;
    for (int i = 0; i < n; ++i) X[i] ^= t;
    uint64_t h = 0;
    for (int j = b - 1; j >= 0; --j)
        for (int i = 0; i < n; ++i) h = (h << 1) | ((X[i] >> j) & 1u);
    return h;
}

// Integer barycentric weights of local node l (sum = degree), following the
// local node order of fem.h.
void local_weights(int dim, int degree, std::vector<std::vector<int>> &W)
{
    const int nv = dim + 1;
    W.clear();
    for (int v = 0; v < nv; ++v) {
        std::vector<int> w(nv, 0);
        w[v] = degree;
        W.push_back(w);
    }
    if (degree >= 2)
        for (int a = 0; a < nv; ++a)
            for (int b = a + 1; b < nv; ++b) {
                std::vector<int> w(nv, 0);
                if (degree == 2) {
                    w[a] = 1; w[b] = 1; W.push_back(w);
                } else {
                    w[a] = 2; w[b] = 1; W.push_back(w);
                    std::vector<int> w2(nv, 0);
                    w2[a] = 1; w2[b] = 2; W.push_back(w2);
                }
            }
    if (degree == 3)
        for (int a = 0; a < nv; ++a)
            for (int b = a + 1; b < nv; ++b)
                for (int c = b + 1; c < nv; ++c) {
                    std::vector<int> w(nv, 0);
                    w[a] = w[b] = w[c] = 1;
                    W.push_back(w);
                }
}

void sfc_order(const std::vector<double> &pos, int dim, int64_t n, int32_t *perm)
{
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < n; ++i)
        for (int r = 0; r < dim; ++r) {
            lo[r] = std::min(lo[r], pos[i * dim + r]);
            hi[r] = std::max(hi[r], pos[i * dim + r]);
        }
    const int bits = dim == 3 ? 21 : 31;
    const double top = (double)((1u << bits) - 1);
    std::vector<std::pair<uint64_t, int32_t>> key(n);
    femk::par_ranges(n, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
            uint32_t X[3] = {0, 0, 0};
            for (int r = 0; r < dim; ++r) {
                const double span = hi[r] > lo[r] ? hi[r] - lo[r] : 1.0;
                double u = (pos[i * dim + r] - lo[r]) / span * top;
                X[r] = (uint32_t)std::min(std::max(u, 0.0), top);
            }
            key[i] = {hilbert_index(X, dim, bits), (int32_t)i};
        }
    });
    // keys are unique (the index breaks ties), so sorting ranges on their own
    // threads and merging them gives the one sorted order
    std::vector<int64_t> cut;
    femk::par_ranges(n, [&](int64_t i0, int64_t i1) { std::sort(key.begin() + i0, key.begin() + i1); });
    {
        const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(femk::host_threads(), n / 65536));
        for (int t = 0; t <= nt; ++t) cut.push_back(n * t / nt);
    }
    while (cut.size() > 2) {
        const int nm = (int)((cut.size() - 1) / 2);   // pairs of neighbouring ranges merged this round
        femk::run_jobs(nm, [&](int j) {
            std::inplace_merge(key.begin() + cut[2 * j], key.begin() + cut[2 * j + 1], key.begin() + cut[2 * j + 2]);
        });
        std::vector<int64_t> next{cut[0]};
        for (int j = 0; j < nm; ++j) next.push_back(cut[2 * j + 2]);
        if (cut.size() % 2 == 0) next.push_back(cut.back());   // an odd range left over
        cut.swap(next);
    }
    for (int64_t i = 0; i < n; ++i) perm[i] = key[i].second;
}

}  // namespace

namespace femk {

fem_status caught_status(fem_ctx *ctx, const char *where)
{
    try {
        throw;
    } catch (const std::bad_alloc &) {
        if (ctx) ctx->err = std::string(where) + ": host allocation failed";
        return FEM_E_NOMEM;
    } catch (const std::exception &e) {
        if (ctx) ctx->err = std::string(where) + ": " + e.what();
        return FEM_E_DEVICE;
    } catch (...) {
        if (ctx) ctx->err = std::string(where) + ": unexpected host error";
        return FEM_E_DEVICE;
    }
}

hipError_t mem_alloc(const fem_mem &m, hipStream_t s, bool temp, size_t bytes, void **p)
{
    *p = nullptr;
    if (m.alloc) {
        *p = m.alloc(bytes, m.user);
        return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    return temp ? hipMallocAsync(p, bytes, s) : hipMalloc(p, bytes);
}

void mem_free(const fem_mem &m, hipStream_t s, bool temp, void *p)
{
    if (!p) return;
    if (m.release) m.release(p, m.user);
    else if (temp) (void)hipFreeAsync(p, s);
    else (void)hipFree(p);
}

}  // namespace femk

extern "C" {

fem_status fem_ctx_create(int device, void *hip_stream, fem_ctx **out)
{
    if (!out) return FEM_E_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FEM_E_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return FEM_E_DEVICE;
    fem_ctx *ctx = new (std::nothrow) fem_ctx;
    if (!ctx) return FEM_E_NOMEM;
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        ctx->num_cus = cus;
    // the device's static scratch: its address is looked up here, with the
    // device current; without it only fem_build_sparsity_noalloc fails
    if (femk::static_scratch(device, &ctx->scratch, &ctx->scratch_bytes) != hipSuccess) {
        ctx->scratch = nullptr;
        ctx->scratch_bytes = 0;
    }
    *out = ctx;
    return FEM_OK;
}

void fem_ctx_destroy(fem_ctx *ctx) { delete ctx; }

fem_status fem_ctx_set_stream(fem_ctx *ctx, void *hip_stream)
{
    if (!ctx) return FEM_E_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return FEM_OK;
}

fem_status fem_ctx_set_allocator(fem_ctx *ctx, void *(*alloc)(size_t, void *), void (*release)(void *, void *),
                                 void *user)
{
    if (!ctx) return FEM_E_ARG;
    if (!alloc != !release) return fail(ctx, FEM_E_ARG, "set_allocator: give both alloc and release, or neither");
    ctx->mem.alloc = alloc;
    ctx->mem.release = release;
    ctx->mem.user = alloc ? user : nullptr;
    return FEM_OK;
}

const char *fem_last_error(const fem_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

fem_status fem_sync(fem_ctx *ctx)
{
    if (!ctx) return FEM_E_ARG;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "stream synchronize");
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "pending device error");
    return FEM_OK;
}

namespace {

// Scratch of the sparsity build, carved from one buffer: the range/overflow
// flag, the row incidence (ptr, ent), the per-row counts and the scan's tile
// sums.
struct SparsityScratch {
    int *flag;
    int64_t *ptr, *scan;
    int32_t *ent, *tmp;
    size_t bytes;
    SparsityScratch(void *base, int64_t ncells, int arity, int64_t nrows)
    {
        Carve c(base);
        flag = c.take<int>(64);
        ptr = c.take<int64_t>(nrows + 1);
        scan = c.take<int64_t>(femk::scan_scratch(nrows));
        ent = c.take<int32_t>(ncells * arity);
        tmp = c.take<int32_t>(nrows + 1);
        bytes = c.off;
    }
};

// The two passes of fem_build_sparsity on scratch w (arguments checked).
fem_status sparsity_passes(fem_ctx *ctx, const fem_map *rmap, const fem_map *cmap, fem_sparsity *sp,
                           const SparsityScratch &w)
{
    const int64_t ncells = rmap->from->size, nrows = rmap->to->size, ncols = cmap->to->size;
    hipStream_t s = ctx->stream;
    const bool counting = sp->col_idx == nullptr;
    if (counting) {
        fem_status st = range_check(ctx, rmap, w.flag, "row Map");
        if (st != FEM_OK) return st;
        st = range_check(ctx, cmap, w.flag, "column Map");
        if (st != FEM_OK) return st;
    } else if (sp->nrows != nrows || sp->ncols != ncols) {
        return fail(ctx, FEM_E_ARG, "build_sparsity: sparsity was counted for other Maps");
    }
    HIPC(femk::build_incidence(rmap->values, ncells, rmap->arity, nrows, w.ptr, w.ent, w.tmp, w.scan, s),
         "incidence");
    HIPC(femk::fill_i32(w.flag, 1, 0, s), "clear flag");
    if (counting) {
        HIPC(femk::row_columns(w.ptr, w.ent, rmap->arity, cmap->values, cmap->arity, nrows, w.tmp, nullptr,
                               nullptr, w.flag, s),
             "row columns");
        HIPC(femk::exclusive_scan(w.tmp, sp->row_ptr, nrows, w.scan, s), "scan");
        int hflag = 0;
        int64_t nnz = 0;
        HIPC(hipMemcpyAsync(&hflag, w.flag, sizeof(int), hipMemcpyDeviceToHost, s), "copy");
        HIPC(hipMemcpyAsync(&nnz, sp->row_ptr + nrows, sizeof(int64_t), hipMemcpyDeviceToHost, s), "copy");
        HIPC(hipStreamSynchronize(s), "sync");
        if (hflag)
            return fail(ctx, FEM_E_UNSUPPORTED, "build_sparsity: a row has more than 8192 distinct columns");
        sp->nrows = nrows;
        sp->ncols = ncols;
        sp->nnz = nnz;
    } else {
        HIPC(femk::row_columns(w.ptr, w.ent, rmap->arity, cmap->values, cmap->arity, nrows, nullptr, sp->row_ptr,
                               sp->col_idx, w.flag, s),
             "row columns");
    }
    return FEM_OK;
}

fem_status check_sparsity_args(fem_ctx *ctx, const fem_map *rmap, const fem_map *cmap, const fem_sparsity *sp)
{
    if (!map_ok(rmap) || !map_ok(cmap) || !sp || !sp->row_ptr)
        return fail(ctx, FEM_E_ARG, "build_sparsity: malformed Map or NULL row_ptr");
    if (rmap->from->size != cmap->from->size)
        return fail(ctx, FEM_E_ARG, "build_sparsity: row and column Maps start from different Sets");
    const int64_t ncells = rmap->from->size, nrows = rmap->to->size, ncols = cmap->to->size;
    if (ncells * (int64_t)rmap->arity > INT32_MAX || ncells * (int64_t)cmap->arity > INT32_MAX ||
        nrows > INT32_MAX || ncols > INT32_MAX)
        return fail(ctx, FEM_E_OVERFLOW, "build_sparsity: more than 2^31-1 entries");
    return FEM_OK;
}

}  // namespace

fem_status fem_build_sparsity(fem_ctx *ctx, const fem_map *rmap, const fem_map *cmap, fem_sparsity *sp,
                              void *work, size_t *work_bytes)
{
    if (!ctx) return FEM_E_ARG;
    fem_status st = check_sparsity_args(ctx, rmap, cmap, sp);
    if (st != FEM_OK) return st;
    const int64_t ncells = rmap->from->size, nrows = rmap->to->size;
    const size_t need = SparsityScratch(nullptr, ncells, rmap->arity, nrows).bytes;
    if (work_bytes && !work) {
        *work_bytes = need;
        return FEM_OK;
    }
    if (work) {
        if (!work_bytes || *work_bytes < need)
            return fail(ctx, FEM_E_ARG, "build_sparsity: work buffer of %zu bytes, %zu needed",
                        work_bytes ? *work_bytes : (size_t)0, need);
        if ((uintptr_t)work % 256 != 0) return fail(ctx, FEM_E_ARG, "build_sparsity: work is not 256-byte aligned");
        return sparsity_passes(ctx, rmap, cmap, sp, SparsityScratch(work, ncells, rmap->arity, nrows));
    }
    DevBuf buf(ctx);
    HIPC(buf.alloc(need), "alloc");
    return sparsity_passes(ctx, rmap, cmap, sp, SparsityScratch(buf.p, ncells, rmap->arity, nrows));
}

fem_status fem_build_sparsity_noalloc(fem_ctx *ctx, const fem_map *rmap, const fem_map *cmap, fem_sparsity *sp)
{
    if (!ctx) return FEM_E_ARG;
    fem_status st = check_sparsity_args(ctx, rmap, cmap, sp);
    if (st != FEM_OK) return st;
    if (!ctx->scratch) return fail(ctx, FEM_E_DEVICE, "build_sparsity_noalloc: no static scratch on this device");
    const int64_t ncells = rmap->from->size, nrows = rmap->to->size;
    const size_t need = SparsityScratch(nullptr, ncells, rmap->arity, nrows).bytes;
    if (need > ctx->scratch_bytes)
        return fail(ctx, FEM_E_ARG, "build_sparsity_noalloc: the Maps need %zu bytes of scratch, the static scratch "
                                    "holds %zu", need, ctx->scratch_bytes);
    return sparsity_passes(ctx, rmap, cmap, sp, SparsityScratch(ctx->scratch, ncells, rmap->arity, nrows));
}

namespace {

// Host inputs of a Mat plan's stream construction, shared read-only by the
// builder threads.
struct StreamIn {
    const int64_t *hrp;     // [nrows+1] CSR row pointers
    const int32_t *hci;     // CSR column indices
    const int64_t *hptr;    // [nrows+1] row -> incidence entries
    const int32_t *hent;    // incidence entries cell*nl + local index, ascending cell
    const int32_t *hcn;     // cell-to-node Map
    int nl, MW, NW, SCAP, CCH, NE, ZIDX;
    int64_t nrows;
};

// One block's streams: per (chunk, wave) the first batch (relative to the
// block's own stream), then the batches.
struct StreamOut {
    std::vector<int32_t> wq;
    std::vector<uint16_t> stream;
    int nq = 0;
    bool missing = false;
};

// Scratch of one builder thread (reused over its blocks).
struct StreamScratch {
    std::vector<int32_t> colmark;   // [nrows], -1 outside the current row
    std::vector<int32_t> slot_ptr, lane_ptr, lane_slots, cursor;
    std::vector<uint16_t> con_idx, con_q;   // per contribution: LDS index of the entry, chunk
    std::vector<int32_t> weight, home, order, tmp_order, bucket, qstart, lane_of, load;
    std::vector<std::vector<int32_t>> by_load;
    std::vector<std::vector<uint16_t>> lane_ent;
};

// Builds the Mat streams of the block of Mat values [v0, v1) in rows
// [r0, r1) (all of their values, or a slice of one long row) whose cells are
// cells[0, nc) (ascending): every Mat value of the block collects its
// contributions (cell, li, lj) in ascending cell id, values are dealt to
// lanes by weight (one open per chunk touched plus the entries), and each
// lane's stream lists, per chunk, "open value" then the value's entries of
// that chunk.  Depends only on the block, so blocks are built in parallel.
void mat_streams(const StreamIn &in, int64_t r0, int64_t r1, int64_t v0, int64_t v1, const int32_t *cells, int64_t nc,
                 StreamScratch &w, StreamOut &o)
{
    const int nl = in.nl, MW = in.MW, NW = in.NW, SCAP = in.SCAP, CCH = in.CCH, NE = in.NE;
    auto upper = [nl](int i, int j) { if (i > j) std::swap(i, j); return i * (2 * nl - i + 1) / 2 + (j - i); };
    auto lpos = [cells, nc](int32_t c) { return (int32_t)(std::lower_bound(cells, cells + nc, c) - cells); };
    if ((int64_t)w.colmark.size() != in.nrows) w.colmark.assign(in.nrows, -1);
    if ((int)w.lane_ent.size() != MW) w.lane_ent.resize(MW);
    std::vector<int32_t> &colmark = w.colmark, &slot_ptr = w.slot_ptr, &cursor = w.cursor;
    std::vector<uint16_t> &con_idx = w.con_idx, &con_q = w.con_q;
    const int64_t sbase = v0;
    const int ns = (int)(v1 - v0);
    // a column of the row: its value's slot in the block, -2 outside the
    // block's slice; -1: not in the row (the sparsity lacks it)
    auto mark_row = [&](int64_t r) {
        for (int64_t k = in.hrp[r]; k < in.hrp[r + 1]; ++k)
            colmark[in.hci[k]] = k >= v0 && k < v1 ? (int32_t)(k - sbase) : -2;
    };
    const int nq = (int)((nc + CCH - 1) / CCH);
    o.nq = nq;
    slot_ptr.assign(ns + 1, 0);
    // contributions, grouped by value, ascending cell within a value
    for (int64_t r = r0; r < r1; ++r) {
        mark_row(r);
        for (int64_t k = in.hptr[r]; k < in.hptr[r + 1]; ++k) {
            const int32_t c = in.hent[k] / nl;
            for (int lj = 0; lj < nl; ++lj) {
                const int32_t sl = colmark[in.hcn[(int64_t)c * nl + lj]];
                if (sl == -1) o.missing = true;
                if (sl < 0) continue;
                ++slot_ptr[sl + 1];
            }
        }
        for (int64_t k = in.hrp[r]; k < in.hrp[r + 1]; ++k) colmark[in.hci[k]] = -1;
    }
    for (int t = 0; t < ns; ++t) slot_ptr[t + 1] += slot_ptr[t];
    con_idx.resize(slot_ptr[ns]);
    con_q.resize(slot_ptr[ns]);
    cursor.assign(slot_ptr.begin(), slot_ptr.end() - 1);
    for (int64_t r = r0; r < r1; ++r) {
        mark_row(r);
        for (int64_t k = in.hptr[r]; k < in.hptr[r + 1]; ++k) {
            const int32_t e = in.hent[k], c = e / nl, li = e % nl, lc = lpos(c);
            for (int lj = 0; lj < nl; ++lj) {
                const int32_t sl = colmark[in.hcn[(int64_t)c * nl + lj]];
                if (sl < 0) continue;
                const int32_t at = cursor[sl]++;
                con_idx[at] = (uint16_t)(SCAP + (lc % CCH) * NE + upper(li, lj));
                con_q[at] = (uint16_t)(lc / CCH);
            }
        }
        for (int64_t k = in.hrp[r]; k < in.hrp[r + 1]; ++k) colmark[in.hci[k]] = -1;
    }
    // Each value's stream entries per chunk it touches are one open plus
    // its entries there; its home is the chunk where it has the most.
    // A (chunk, wave) stream is as long as its longest lane, so the loads
    // are balanced chunk by chunk: the values homed in chunk q, heaviest
    // first, go to the lane with the least load in chunk q so far
    // (longest-processing-time; the load already includes what values
    // homed in earlier chunks put there).  Loads only grow, so a bucket
    // queue keyed by load finds that lane; lanes enter in wave-interleaved
    // order so ties spread over the waves.  With one chunk this is plain
    // LPT on the value weights.
    std::vector<int32_t> &home = w.home, &weight = w.weight, &bucket = w.bucket, &tmp_order = w.tmp_order;
    std::vector<int32_t> &qstart = w.qstart, &order = w.order, &lane_of = w.lane_of, &load = w.load;
    std::vector<std::vector<int32_t>> &by_load = w.by_load;
    home.resize(ns);
    weight.resize(ns);
    int wmax = 0;
    for (int t = 0; t < ns; ++t) {
        int best = 0, hq = 0;
        for (int32_t k = slot_ptr[t]; k < slot_ptr[t + 1];) {
            int32_t k1 = k;
            while (k1 < slot_ptr[t + 1] && con_q[k1] == con_q[k]) ++k1;
            if (k1 - k + 1 > best) { best = k1 - k + 1; hq = con_q[k]; }
            k = k1;
        }
        home[t] = hq;
        weight[t] = best;
        wmax = std::max(wmax, best);
    }
    // order: by home chunk, then heaviest first (two stable counting sorts)
    bucket.assign(wmax + 2, 0);
    for (int t = 0; t < ns; ++t) ++bucket[wmax - weight[t] + 1];
    for (int v = 0; v <= wmax; ++v) bucket[v + 1] += bucket[v];
    tmp_order.resize(ns);
    for (int t = 0; t < ns; ++t) tmp_order[bucket[wmax - weight[t]]++] = t;
    qstart.assign(nq + 1, 0);
    for (int t = 0; t < ns; ++t) ++qstart[home[t] + 1];
    for (int q = 0; q < nq; ++q) qstart[q + 1] += qstart[q];
    order.resize(ns);
    {
        std::vector<int32_t> fill(qstart.begin(), qstart.end() - 1);
        for (int p = 0; p < ns; ++p) order[fill[home[tmp_order[p]]]++] = tmp_order[p];
    }
    lane_of.resize(ns);
    load.assign((size_t)nq * MW, 0);
    for (int q = 0; q < nq; ++q) {
        if (qstart[q] == qstart[q + 1]) continue;
        int32_t *lq = load.data() + (size_t)q * MW;
        int kmax = 0;
        for (int l = 0; l < MW; ++l) kmax = std::max(kmax, lq[l]);
        for (auto &v : by_load) v.clear();
        if ((int)by_load.size() <= kmax) by_load.resize(kmax + 1);
        for (int i = MW - 1; i >= 0; --i) {
            const int l = (i % NW) * 64 + i / NW;
            by_load[lq[l]].push_back(l);
        }
        for (int p = qstart[q], m = 0; p < qstart[q + 1]; ++p) {
            while (by_load[m].empty()) ++m;
            const int l = by_load[m].back();
            by_load[m].pop_back();
            const int t = order[p];
            lane_of[t] = l;
            for (int32_t k = slot_ptr[t]; k < slot_ptr[t + 1];) {
                int32_t k1 = k;
                while (k1 < slot_ptr[t + 1] && con_q[k1] == con_q[k]) ++k1;
                load[(size_t)con_q[k] * MW + l] += k1 - k + 1;
                k = k1;
            }
            if ((int)by_load.size() <= lq[l]) by_load.resize(lq[l] + 1);
            by_load[lq[l]].push_back(l);
        }
    }
    std::vector<int32_t> &lane_ptr = w.lane_ptr, &lane_slots = w.lane_slots;
    lane_ptr.assign(MW + 1, 0);
    for (int t = 0; t < ns; ++t) ++lane_ptr[lane_of[t] + 1];
    for (int l = 0; l < MW; ++l) lane_ptr[l + 1] += lane_ptr[l];
    lane_slots.resize(ns);
    {
        std::vector<int32_t> fill(lane_ptr.begin(), lane_ptr.end() - 1);
        for (int p = 0; p < ns; ++p) lane_slots[fill[lane_of[order[p]]]++] = order[p];
    }
    cursor.assign(slot_ptr.begin(), slot_ptr.end() - 1);
    for (int q = 0; q < nq; ++q) {
        for (int l = 0; l < MW; ++l) {
            std::vector<uint16_t> &le = w.lane_ent[l];
            le.clear();
            for (int32_t k = lane_ptr[l]; k < lane_ptr[l + 1]; ++k) {
                const int32_t t = lane_slots[k];
                int32_t &at = cursor[t];
                if (at == slot_ptr[t + 1] || con_q[at] != q) continue;
                le.push_back((uint16_t)t);
                while (at < slot_ptr[t + 1] && con_q[at] == q) le.push_back(con_idx[at++]);
            }
        }
        for (int v = 0; v < NW; ++v) {
            o.wq.push_back((int32_t)(o.stream.size() / femk::MAT_BATCH));
            size_t len = 0;
            for (int l = 64 * v; l < 64 * v + 64; ++l) len = std::max(len, w.lane_ent[l].size());
            const size_t nb = std::max<size_t>(1, (len + femk::MAT_BATCH - 1) / femk::MAT_BATCH);   // one batch at least
            for (size_t i = 0; i < nb; ++i)
                for (int l = 64 * v; l < 64 * v + 64; ++l)
                    for (size_t j = femk::MAT_BATCH * i; j < femk::MAT_BATCH * (i + 1); ++j)
                        o.stream.push_back(j < w.lane_ent[l].size() ? w.lane_ent[l][j] : (uint16_t)in.ZIDX);
        }
    }
}

}  // namespace

static fem_status plan_create(fem_ctx *ctx, const fem_form *form, const fem_args *args, const fem_sparsity *sp,
                              fem_plan **out);

fem_status fem_plan_create(fem_ctx *ctx, const fem_form *form, const fem_args *args,
                           const fem_sparsity *sp, fem_plan **out)
{
    try {
        return plan_create(ctx, form, args, sp, out);
    } catch (...) {
        return femk::caught_status(ctx, "plan_create");
    }
}

static fem_status plan_create(fem_ctx *ctx, const fem_form *form, const fem_args *args, const fem_sparsity *sp,
                              fem_plan **out)
{
    if (!ctx) return FEM_E_ARG;
    if (!out) return fail(ctx, FEM_E_ARG, "plan_create: NULL output");
    *out = nullptr;
    fem_status st = check_form(ctx, form);
    if (st != FEM_OK) return st;
    if (form->kind == FEM_ELASTICITY) return femk::elast_plan_create(ctx, form, args, sp, out);
    st = check_args(ctx, form, args, false);
    if (st != FEM_OK) return st;
    const bool is_mat = sp != nullptr;
    const int dim = (int)form->cell, deg = form->degree, nl = nloc_of(dim, deg);
    const int64_t ncells = args->cells->size, nrows = args->cell_node->to->size;
    if (is_mat) {
        if (!sp->row_ptr || sp->nrows != nrows || sp->ncols != nrows || (!sp->col_idx && sp->nnz > 0))
            return fail(ctx, FEM_E_ARG, "plan_create: sparsity does not match the cell_node Map");
        if (form->kind == FEM_SOURCE || form->kind == FEM_NL_RESIDUAL)
            return fail(ctx, FEM_E_ARG, "plan_create: a Mat plan needs a bilinear form");
    }
    femk::Limits lim;
    if (!femk::limits(dim, deg, is_mat, &lim))
        return fail(ctx, FEM_E_UNSUPPORTED, "plan_create: no kernel for this cell/degree");
    hipStream_t s = ctx->stream;
    DevBuf flag(ctx), ptr(ctx), ent(ctx), tmp(ctx), scan(ctx);
    HIPC(flag.alloc(sizeof(int)), "alloc");
    st = range_check(ctx, args->cell_node, flag.as<int>(), "cell_node");
    if (st != FEM_OK) return st;
    st = range_check(ctx, args->cell_vertex, flag.as<int>(), "cell_vertex");
    if (st != FEM_OK) return st;
    HIPC(ptr.alloc(sizeof(int64_t) * (nrows + 1)), "alloc");
    HIPC(ent.alloc(sizeof(int32_t) * (ncells * nl)), "alloc");
    HIPC(tmp.alloc(sizeof(int32_t) * (nrows + 1)), "alloc");
    HIPC(scan.alloc(sizeof(int64_t) * femk::scan_scratch(nrows)), "alloc");
    HIPC(femk::build_incidence(args->cell_node->values, ncells, nl, nrows, ptr.as<int64_t>(),
                               ent.as<int32_t>(), tmp.as<int32_t>(), scan.as<int64_t>(), s),
         "incidence");
    std::vector<int64_t> hptr(nrows + 1);
    std::vector<int32_t> hent(ncells * nl);
    std::vector<int64_t> hrp;
    std::vector<int32_t> hcv(ncells * (dim + 1));
    if (!hcv.empty())
        HIPC(hipMemcpyAsync(hcv.data(), args->cell_vertex->values, sizeof(int32_t) * hcv.size(),
                            hipMemcpyDeviceToHost, s), "copy");
    HIPC(hipMemcpyAsync(hptr.data(), ptr.p, sizeof(int64_t) * (nrows + 1), hipMemcpyDeviceToHost, s), "copy");
    if (!hent.empty())
        HIPC(hipMemcpyAsync(hent.data(), ent.p, sizeof(int32_t) * hent.size(), hipMemcpyDeviceToHost, s), "copy");
    std::vector<int32_t> hci, hcn;
    if (is_mat) {
        hrp.resize(nrows + 1);
        HIPC(hipMemcpyAsync(hrp.data(), sp->row_ptr, sizeof(int64_t) * (nrows + 1), hipMemcpyDeviceToHost, s),
             "copy");
        HIPC(hipStreamSynchronize(s), "sync");
        if (hrp[nrows] != sp->nnz || hrp[0] != 0)
            return fail(ctx, FEM_E_ARG, "plan_create: row_ptr does not span [0, nnz]");
        hci.resize(sp->nnz);
        hcn.resize(ncells * nl);
        if (!hci.empty())
            HIPC(hipMemcpyAsync(hci.data(), sp->col_idx, sizeof(int32_t) * hci.size(), hipMemcpyDeviceToHost, s),
                 "copy");
        if (!hcn.empty())
            HIPC(hipMemcpyAsync(hcn.data(), args->cell_node->values, sizeof(int32_t) * hcn.size(),
                                hipMemcpyDeviceToHost, s), "copy");
    }
    HIPC(hipStreamSynchronize(s), "sync");
    for (int32_t c : hci)
        if (c < 0 || c >= nrows) return fail(ctx, FEM_E_RANGE, "plan_create: a column index lies outside [0, ncols)");

    // Greedy partition of the rows into contiguous blocks bounded by the
    // rows a workgroup owns, the Mat values it can hold in LDS and the
    // distinct cells it can address.  Keep at least ~2 blocks per CU when the
    // problem is small.
    int64_t rows_cap = lim.rows_per_block;
    const int64_t want = 2 * (int64_t)ctx->num_cus;
    if (nrows < std::min<int64_t>(rows_cap, 1 << 20) * want)
        rows_cap = std::min<int64_t>(rows_cap, std::max<int64_t>(1, (nrows + want - 1) / want));
    const int lbits = nl <= 4 ? 2 : nl <= 8 ? 3 : nl <= 16 ? 4 : 5;
    std::vector<int32_t> blk_row0{0}, blk_cptr{0}, bcell;
    std::vector<int32_t> stamp(ncells, -1), lpos(is_mat ? 0 : ncells, 0);
    // Dat plans: packed entries
    std::vector<uint16_t> hent16(is_mat ? 0 : hent.size());
    // Mat plans: per-lane LDS index streams (see fem_plan)
    const int MW = is_mat ? lim.lanes : 64, NW = MW / 64;
    const int SCAP = lim.slot_cap, CCH = lim.chunk_cells, NE = lim.ne;
    const int ZIDX = SCAP + CCH * NE;
    std::vector<int32_t> blk_w{0}, wq;
    std::vector<uint16_t> stream;
    std::vector<int64_t> mb_r0, mb_r1, mb_v0, mb_v1;   // Mat blocks: rows and Mat values
    int64_t nchunks = 0;
    bool missing = false;
    int32_t b = 0;
    int64_t rows = 0, slots = 0, cells = 0;
    size_t first_cell = 0;
    int64_t block_first_row = 0;
    auto close_block = [&](int64_t next_row) {
        std::sort(bcell.begin() + first_cell, bcell.end());
        if (!is_mat) {
            for (size_t i = first_cell; i < bcell.size(); ++i) lpos[bcell[i]] = (int32_t)(i - first_cell);
            for (int64_t r = block_first_row; r < next_row; ++r)
                for (int64_t k = hptr[r]; k < hptr[r + 1]; ++k) {
                    const int32_t e = hent[k];
                    hent16[k] = (uint16_t)((lpos[e / nl] << lbits) | (e % nl));
                }
        }
        // (Mat plans: the block's streams are built once the partition is done)
        if (is_mat) {
            mb_r0.push_back(block_first_row);
            mb_r1.push_back(next_row);
            mb_v0.push_back(hrp[block_first_row]);
            mb_v1.push_back(hrp[next_row]);
        }
        blk_row0.push_back((int32_t)next_row);
        blk_cptr.push_back((int32_t)bcell.size());
        first_cell = bcell.size();
        block_first_row = next_row;
        ++b;
        rows = slots = cells = 0;
    };
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t rs = is_mat ? hrp[r + 1] - hrp[r] : 0;
        int64_t fresh = 0;
        for (int64_t k = hptr[r]; k < hptr[r + 1]; ++k) fresh += stamp[hent[k] / nl] != b;
        if (rows > 0 && (rows + 1 > rows_cap || slots + rs > lim.slot_cap * (int64_t)is_mat ||
                         cells + fresh > lim.cell_cap)) {
            close_block(r);
            fresh = hptr[r + 1] - hptr[r];
        }
        // (a Mat row whose cells exceed one chunk gets a block of several chunks)
        if (!is_mat && fresh > lim.cell_cap)
            return fail(ctx, FEM_E_UNSUPPORTED, "plan_create: row %lld is too long for one workgroup",
                        (long long)r);
        if (is_mat && rs > lim.slot_cap) {
            // A Mat row with more values than a block holds: blocks of
            // consecutive slices of its values, each gathering the row's
            // cells (the block before it was closed above).
            for (int64_t k = hptr[r]; k < hptr[r + 1]; ++k) {
                const int32_t c = hent[k] / nl;
                if (stamp[c] != b) {
                    stamp[c] = b;
                    bcell.push_back(c);
                }
            }
            std::sort(bcell.begin() + first_cell, bcell.end());
            const size_t rc0 = first_cell, nrc = bcell.size() - first_cell;
            for (int64_t v0 = hrp[r]; v0 < hrp[r + 1]; v0 += lim.slot_cap) {
                if (v0 > hrp[r])
                    for (size_t i = 0; i < nrc; ++i) {
                        const int32_t c = bcell[rc0 + i];
                        bcell.push_back(c);
                    }
                mb_r0.push_back(r);
                mb_r1.push_back(r + 1);
                mb_v0.push_back(v0);
                mb_v1.push_back(std::min<int64_t>(v0 + lim.slot_cap, hrp[r + 1]));
                blk_row0.push_back((int32_t)(r + 1));
                blk_cptr.push_back((int32_t)bcell.size());
                first_cell = bcell.size();
                ++b;
            }
            block_first_row = r + 1;
            rows = slots = cells = 0;
            continue;
        }
        for (int64_t k = hptr[r]; k < hptr[r + 1]; ++k) {
            const int32_t c = hent[k] / nl;
            if (stamp[c] != b) {
                stamp[c] = b;
                bcell.push_back(c);
            }
        }
        ++rows;
        slots += rs;
        cells += fresh;
    }
    if (rows > 0) close_block(nrows);
    if (is_mat && b > 0) {
        // the blocks' streams, built on several threads (each block depends
        // only on its rows and cells), then joined in block order
        StreamIn in;
        in.hrp = hrp.data(); in.hci = hci.data(); in.hptr = hptr.data(); in.hent = hent.data();
        in.hcn = hcn.data();
        in.nl = nl; in.MW = MW; in.NW = NW; in.SCAP = SCAP; in.CCH = CCH; in.NE = NE; in.ZIDX = ZIDX;
        in.nrows = nrows;
        std::vector<StreamOut> outs((size_t)b);
        std::atomic<int32_t> next{0};
        std::atomic<bool> failed{false};
        femk::run_jobs(std::min<int>(femk::host_threads(), b), [&](int) {
            try {
                StreamScratch w;
                for (int32_t i; !failed && (i = next.fetch_add(1)) < b;)
                    mat_streams(in, mb_r0[i], mb_r1[i], mb_v0[i], mb_v1[i], bcell.data() + blk_cptr[i],
                                blk_cptr[i + 1] - blk_cptr[i], w, outs[i]);
            } catch (...) {
                failed = true;
            }
        });
        if (failed) return fail(ctx, FEM_E_NOMEM, "plan_create: host allocation failed while building the streams");
        size_t total = 0;
        for (const StreamOut &o : outs) total += o.stream.size();
        stream.reserve(total);
        for (StreamOut &o : outs) {
            missing = missing || o.missing;
            const int32_t base = (int32_t)(stream.size() / femk::MAT_BATCH);
            if (stream.size() / femk::MAT_BATCH + o.stream.size() / femk::MAT_BATCH > (size_t)INT32_MAX)
                return fail(ctx, FEM_E_OVERFLOW, "plan_create: Mat streams exceed 2^31 batches");
            for (int32_t v : o.wq) wq.push_back(base + v);
            stream.insert(stream.end(), o.stream.begin(), o.stream.end());
            nchunks += o.nq;
            blk_w.push_back((int32_t)wq.size());
            std::vector<uint16_t>().swap(o.stream);
        }
    }
    if (missing) return fail(ctx, FEM_E_ARG, "plan_create: the sparsity lacks entries the Maps reach");
    if (is_mat) {
        wq.push_back((int32_t)(stream.size() / femk::MAT_BATCH));
        if (stream.size() / femk::MAT_BATCH > (size_t)INT32_MAX)
            return fail(ctx, FEM_E_OVERFLOW, "plan_create: Mat streams exceed 2^31 batches");
    }

    fem_plan *p = new (std::nothrow) fem_plan;
    if (!p) return fail(ctx, FEM_E_NOMEM, "plan_create: host allocation");
    // frees the plan and the arrays uploaded so far on every way out but
    // success (an error status or a host allocation failure below)
    struct Release {
        fem_plan *p;
        ~Release() { if (p) { free_plan_arrays(p); delete p; } }
    } release{p};
    p->is_mat = is_mat;
    p->dim = dim; p->degree = deg; p->nloc = nl;
    p->ncells = ncells; p->nrows = nrows; p->nverts = args->cell_vertex->to->size;
    p->nnz = is_mat ? sp->nnz : 0;
    p->nblk = b;
    p->lbits = lbits;
    p->cell_visits = (int64_t)bcell.size();
    for (int32_t i = 0; i < b; ++i) p->max_blk_cells = std::max(p->max_blk_cells, blk_cptr[i + 1] - blk_cptr[i]);
    p->cell_node = args->cell_node->values;
    p->cell_vertex = args->cell_vertex->values;
    p->cn_version = args->cell_node->version;
    p->cv_version = args->cell_vertex->version;
    p->row_ptr = is_mat ? sp->row_ptr : nullptr;
    p->col_idx = is_mat ? sp->col_idx : nullptr;
    p->mem = ctx->mem;
    std::vector<int32_t> bverts(bcell.size() * (dim + 1));
    for (size_t i = 0; i < bcell.size(); ++i)
        for (int m = 0; m <= dim; ++m) bverts[i * (dim + 1) + m] = hcv[(int64_t)bcell[i] * (dim + 1) + m];
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = upload(p->mem, &p->blk_row0, blk_row0, &p->bytes, s);
    if (e == hipSuccess) e = upload(p->mem, &p->blk_cptr, blk_cptr, &p->bytes, s);
    if (e == hipSuccess) e = upload(p->mem, &p->bcell, bcell, &p->bytes, s);
    if (e == hipSuccess) e = upload(p->mem, &p->bverts, bverts, &p->bytes, s);
    if (!is_mat) {
        const size_t rb = sizeof(double) * (size_t)femk::reduce_partials(ncells);
        if (e == hipSuccess) e = femk::mem_alloc(p->mem, s, false, rb ? rb : 8, (void **)&p->red_partial);
        if (e == hipSuccess) p->bytes += rb;
        std::vector<int32_t> inc32(nrows + 1);
        for (int64_t r = 0; r <= nrows; ++r) inc32[r] = (int32_t)hptr[r];
        if (e == hipSuccess) e = upload(p->mem, &p->inc_ptr, inc32, &p->bytes, s);
        if (e == hipSuccess) e = upload(p->mem, &p->ent, hent16, &p->bytes, s);
    } else {
        p->nchunks = nchunks;
        p->stream_entries = (int64_t)stream.size();
        // one 32-byte header per block, read with a single scalar load:
        // first Mat value (lo, hi), Mat values, first cell, cells, chunks,
        // first (chunk, wave) stream, 0
        std::vector<int32_t> hdr((size_t)b * 8, 0);
        for (int32_t i = 0; i < b; ++i) {
            int32_t *hd = &hdr[(size_t)i * 8];
            const int64_t s0 = mb_v0[i];
            hd[0] = (int32_t)(uint32_t)(s0 & 0xffffffff);
            hd[1] = (int32_t)(s0 >> 32);
            hd[2] = (int32_t)(mb_v1[i] - s0);
            hd[3] = blk_cptr[i];
            hd[4] = blk_cptr[i + 1] - blk_cptr[i];
            hd[5] = (blk_w[i + 1] - blk_w[i]) / NW;
            hd[6] = blk_w[i];
        }
        if (e == hipSuccess) e = upload(p->mem, &p->blk_hdr, hdr, &p->bytes, s);
        if (e == hipSuccess) e = upload(p->mem, &p->blk_w, blk_w, &p->bytes, s);
        if (e == hipSuccess) e = upload(p->mem, &p->wq, wq, &p->bytes, s);
        if (e == hipSuccess) e = upload(p->mem, &p->pstream, stream, &p->bytes, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(ctx, e, "plan_create");
    release.p = nullptr;
    *out = p;
    return FEM_OK;
}

void fem_plan_destroy(fem_plan *p)
{
    if (!p) return;
    free_plan_arrays(p);
    delete p;
}

fem_status fem_plan_info(const fem_plan *p, int64_t *nblocks, int64_t *cell_visits, int64_t *device_bytes)
{
    if (!p) return FEM_E_ARG;
    if (nblocks) *nblocks = p->nblk;
    if (cell_visits) *cell_visits = p->cell_visits;
    if (device_bytes) *device_bytes = (int64_t)p->bytes;
    return FEM_OK;
}

static fem_status check_plan(fem_ctx *ctx, const fem_plan *plan, const fem_form *form, const fem_args *args,
                             bool want_mat)
{
    if (!plan) return fail(ctx, FEM_E_ARG, "plan is NULL");
    if (plan->is_mat != (int)want_mat)
        return fail(ctx, FEM_E_ARG, want_mat ? "a Mat plan (built with a sparsity) is required"
                                             : "a Dat plan (built without a sparsity) is required");
    if (plan->dim != (int)form->cell || plan->degree != form->degree)
        return fail(ctx, FEM_E_ARG, "plan was built for another cell/degree");
    if (plan->cell_node != args->cell_node->values || plan->cell_vertex != args->cell_vertex->values ||
        plan->ncells != args->cells->size || plan->nrows != args->cell_node->to->size ||
        plan->nverts != args->cell_vertex->to->size)
        return fail(ctx, FEM_E_ARG, "plan was built for other Maps");
    if (plan->cn_version != args->cell_node->version || plan->cv_version != args->cell_vertex->version)
        return fail(ctx, FEM_E_ARG, "plan was built for another version of its Maps (rebuild the plan)");
    return FEM_OK;
}

// The nonlinear residual's fields u, kappa (, f): scalar Dats on the node Set.
static fem_status check_nodal(fem_ctx *ctx, const fem_args *args, int need)
{
    if (args->ncoeff < need)
        return fail(ctx, FEM_E_ARG, "args: the nonlinear residual needs %d coefficient Dats", need);
    for (int i = 0; i < need; ++i)
        if (!dat_ok(args->coeff[i], args->cell_node->to, 1))
            return fail(ctx, FEM_E_ARG, "args: coeff[%d] must be a scalar Dat on the node Set", i);
    return FEM_OK;
}

static femk::AsmArgs base_args(const fem_ctx *ctx, const fem_plan *plan, const fem_args *args)
{
    femk::AsmArgs a{};
    a.plan = plan;
    a.num_cus = ctx->num_cus;
    a.cell_vertex = args->cell_vertex->values;
    a.coords = args->coords->data;
    a.cell_node = args->cell_node->values;
    return a;
}

fem_status fem_par_loop_assemble_mat(fem_ctx *ctx, const fem_plan *plan, const fem_form *form,
                                     const fem_args *args, fem_mat *A, fem_access acc)
{
    if (!ctx) return FEM_E_ARG;
    fem_status st = check_form(ctx, form);
    if (st != FEM_OK) return st;
    if (form->kind == FEM_ELASTICITY) return femk::elast_assemble(ctx, plan, form, args, A, acc);
    if (form->kind == FEM_SOURCE || form->kind == FEM_NL_RESIDUAL)
        return fail(ctx, FEM_E_ARG, "assemble_mat needs a bilinear form");
    const bool need_k = form->kind != FEM_MASS;
    if ((st = check_args(ctx, form, args, need_k)) != FEM_OK) return st;
    if ((st = check_plan(ctx, plan, form, args, true)) != FEM_OK) return st;
    if (!A || !A->sp || (!A->values && plan->nnz > 0))
        return fail(ctx, FEM_E_ARG, "assemble_mat: Mat without values");
    if (A->sp->row_ptr != plan->row_ptr || A->sp->col_idx != plan->col_idx || A->sp->nnz != plan->nnz)
        return fail(ctx, FEM_E_ARG, "assemble_mat: Mat sparsity differs from the plan's");
    if (acc != FEM_WRITE && acc != FEM_INC) return fail(ctx, FEM_E_ARG, "a Mat accepts only WRITE or INC");
    femk::AsmArgs a = base_args(ctx, plan, args);
    form_coeffs(form->kind, &a.cstiff, &a.cmass);
    a.coeff = need_k ? args->coeff[0]->data : args->coords->data;   // unread when cstiff == 0
    a.row_ptr = A->sp->row_ptr;
    a.out = A->values;
    a.inc = acc == FEM_INC;
    a.num_cus = ctx->num_cus;
    hipError_t e = femk::launch_mat(a, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "assemble_mat launch");
    return FEM_OK;
}

fem_status fem_par_loop_assemble_vec(fem_ctx *ctx, const fem_plan *plan, const fem_form *form,
                                     const fem_args *args, fem_dat *b, fem_access acc)
{
    if (!ctx) return FEM_E_ARG;
    fem_status st = check_form(ctx, form);
    if (st != FEM_OK) return st;
    if (form->kind != FEM_SOURCE && form->kind != FEM_NL_RESIDUAL)
        return fail(ctx, FEM_E_ARG, "assemble_vec needs FEM_SOURCE or FEM_NL_RESIDUAL");
    if (form->kind == FEM_NL_RESIDUAL) {
        if ((st = check_args(ctx, form, args, false)) != FEM_OK) return st;
        if ((st = check_plan(ctx, plan, form, args, false)) != FEM_OK) return st;
        if ((st = check_nodal(ctx, args, 3)) != FEM_OK) return st;
        if (!dat_ok(b, args->cell_node->to, 1))
            return fail(ctx, FEM_E_ARG, "assemble_vec: b must be a Dat on the nodes");
        if (acc != FEM_WRITE && acc != FEM_INC) return fail(ctx, FEM_E_ARG, "output access must be WRITE or INC");
        femk::AsmArgs a = base_args(ctx, plan, args);
        a.x = args->coeff[0]->data;
        a.coeff = args->coeff[1]->data;
        a.aux = args->coeff[2]->data;
        a.out = b->data;
        a.inc = acc == FEM_INC;
        hipError_t e = femk::launch_nl(a, 0, form->prec == FEM_FP32, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "assemble_vec launch");
        return FEM_OK;
    }
    if ((st = check_args(ctx, form, args, true)) != FEM_OK) return st;
    if ((st = check_plan(ctx, plan, form, args, false)) != FEM_OK) return st;
    if (!dat_ok(b, args->cell_node->to, 1)) return fail(ctx, FEM_E_ARG, "assemble_vec: b must be a Dat on the nodes");
    if (acc != FEM_WRITE && acc != FEM_INC) return fail(ctx, FEM_E_ARG, "output access must be WRITE or INC");
    femk::AsmArgs a = base_args(ctx, plan, args);
    a.coeff = args->coeff[0]->data;
    a.out = b->data;
    a.inc = acc == FEM_INC;
    hipError_t e = femk::launch_vec(a, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "assemble_vec launch");
    return FEM_OK;
}

fem_status fem_apply_action(fem_ctx *ctx, const fem_plan *plan, const fem_form *form, const fem_args *args,
                            const fem_dat *x, fem_dat *y, fem_access acc)
{
    if (!ctx) return FEM_E_ARG;
    fem_status st = check_form(ctx, form);
    if (st != FEM_OK) return st;
    if (form->kind == FEM_SOURCE || form->kind == FEM_NL_RESIDUAL)
        return fail(ctx, FEM_E_ARG, "apply_action needs a bilinear form");
    if (form->kind == FEM_ELASTICITY)
        return fail(ctx, FEM_E_UNSUPPORTED, "apply_action: no matrix-free elasticity kernel");
    const bool need_k = form->kind != FEM_MASS;
    if ((st = check_args(ctx, form, args, need_k)) != FEM_OK) return st;
    if ((st = check_plan(ctx, plan, form, args, false)) != FEM_OK) return st;
    if (!dat_ok(x, args->cell_node->to, 1) || !dat_ok(y, args->cell_node->to, 1))
        return fail(ctx, FEM_E_ARG, "apply_action: x and y must be Dats on the nodes");
    if (x->data == y->data && x->set->size > 0) return fail(ctx, FEM_E_ARG, "apply_action: x and y alias");
    if (acc != FEM_WRITE && acc != FEM_INC) return fail(ctx, FEM_E_ARG, "output access must be WRITE or INC");
    femk::AsmArgs a = base_args(ctx, plan, args);
    form_coeffs(form->kind, &a.cstiff, &a.cmass);
    a.coeff = need_k ? args->coeff[0]->data : args->coords->data;
    a.x = x->data;
    a.out = y->data;
    a.inc = acc == FEM_INC;
    hipError_t e = femk::launch_action(a, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "apply_action launch");
    return FEM_OK;
}

fem_status fem_par_loop_assemble_adjoint(fem_ctx *ctx, const fem_plan *plan, const fem_form *form,
                                         const fem_args *args, const fem_dat *lambda, fem_dat *g_u,
                                         fem_dat *g_kappa, fem_access acc)
{
    if (!ctx) return FEM_E_ARG;
    fem_status st = check_form(ctx, form);
    if (st != FEM_OK) return st;
    if (form->kind != FEM_NL_RESIDUAL) return fail(ctx, FEM_E_ARG, "assemble_adjoint needs FEM_NL_RESIDUAL");
    if ((st = check_args(ctx, form, args, false)) != FEM_OK) return st;
    if ((st = check_plan(ctx, plan, form, args, false)) != FEM_OK) return st;
    if ((st = check_nodal(ctx, args, 2)) != FEM_OK) return st;
    const fem_set *nodes = args->cell_node->to;
    if (!dat_ok(lambda, nodes, 1)) return fail(ctx, FEM_E_ARG, "assemble_adjoint: lambda must be a Dat on the nodes");
    if ((g_u && !dat_ok(g_u, nodes, 1)) || (g_kappa && !dat_ok(g_kappa, nodes, 1)))
        return fail(ctx, FEM_E_ARG, "assemble_adjoint: outputs must be Dats on the nodes");
    if (acc != FEM_WRITE && acc != FEM_INC) return fail(ctx, FEM_E_ARG, "output access must be WRITE or INC");
    for (const fem_dat *o : {(const fem_dat *)g_u, (const fem_dat *)g_kappa})
        if (o && nodes->size > 0 && (o->data == lambda->data || o->data == args->coeff[0]->data ||
                                     o->data == args->coeff[1]->data))
            return fail(ctx, FEM_E_ARG, "assemble_adjoint: an output aliases an input");
    if (g_u && g_kappa && g_u->data == g_kappa->data && nodes->size > 0)
        return fail(ctx, FEM_E_ARG, "assemble_adjoint: g_u and g_kappa alias");
    femk::AsmArgs a = base_args(ctx, plan, args);
    a.x = args->coeff[0]->data;
    a.coeff = args->coeff[1]->data;
    a.aux = lambda->data;
    a.inc = acc == FEM_INC;
    const bool fp32 = form->prec == FEM_FP32;
    // both products from one gather when both are asked for
    const int mode = g_u && g_kappa ? 3 : g_u ? 1 : 2;
    if (!g_u && !g_kappa) return FEM_OK;
    a.out = g_u ? g_u->data : g_kappa->data;
    a.out2 = g_u && g_kappa ? g_kappa->data : nullptr;
    hipError_t e = femk::launch_nl(a, mode, fp32, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "assemble_adjoint launch");
    return FEM_OK;
}

fem_status fem_par_loop_reduce(fem_ctx *ctx, const fem_plan *plan, const fem_form *form, const fem_args *args,
                               const fem_dat *x, fem_global *g, fem_access acc)
{
    if (!ctx) return FEM_E_ARG;
    fem_status st = check_form(ctx, form);
    if (st != FEM_OK) return st;
    if (form->kind == FEM_NL_RESIDUAL || form->kind == FEM_ELASTICITY)
        return fail(ctx, FEM_E_UNSUPPORTED, "reduce: the form kind has no cell reduction");
    const bool energy = form->kind != FEM_SOURCE;
    const bool need_k = form->kind != FEM_MASS;
    if ((st = check_args(ctx, form, args, need_k)) != FEM_OK) return st;
    if ((st = check_plan(ctx, plan, form, args, false)) != FEM_OK) return st;
    if (!g || !g->data) return fail(ctx, FEM_E_ARG, "reduce: Global without data");
    if (acc != FEM_SUM && acc != FEM_MIN && acc != FEM_MAX)
        return fail(ctx, FEM_E_ARG, "reduce: a Global accepts SUM, MIN or MAX");
    if (energy && !dat_ok(x, args->cell_node->to, 1))
        return fail(ctx, FEM_E_ARG, "reduce: the energy needs x, a Dat on the nodes");
    femk::AsmArgs a = base_args(ctx, plan, args);
    form_coeffs(energy ? form->kind : FEM_MASS, &a.cstiff, &a.cmass);
    a.coeff = need_k ? args->coeff[0]->data : args->coords->data;   // unread when cstiff == 0
    a.x = energy ? x->data : nullptr;
    const int mode = acc == FEM_SUM ? 0 : acc == FEM_MIN ? 1 : 2;
    hipError_t e = femk::launch_reduce(a, plan->red_partial, mode, energy, g->data, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "reduce launch");
    return FEM_OK;
}

fem_status fem_par_loop_assemble_mixed(fem_ctx *ctx, const fem_plan *plan, const fem_form *form, const fem_args *args,
                                       int32_t nfields, const fem_block *blocks, fem_mat *mats, fem_access acc)
{
    if (!ctx) return FEM_E_ARG;
    fem_status st = check_form(ctx, form);
    if (st != FEM_OK) return st;
    if (nfields < 1 || nfields > 8 || !blocks || !mats)
        return fail(ctx, FEM_E_ARG, "assemble_mixed: 1..8 fields with blocks and Mats");
    if ((st = check_args(ctx, form, args, false)) != FEM_OK) return st;
    if ((st = check_plan(ctx, plan, form, args, true)) != FEM_OK) return st;
    if (acc != FEM_WRITE && acc != FEM_INC) return fail(ctx, FEM_E_ARG, "a Mat accepts only WRITE or INC");
    for (int32_t q = 0; q < nfields * nfields; ++q) {         // validate every block before queuing any
        const fem_block &bk = blocks[q];
        if (!mats[q].values) continue;
        if (bk.kind != FEM_MASS && bk.kind != FEM_LAPLACE && bk.kind != FEM_HELMHOLTZ)
            return fail(ctx, FEM_E_ARG, "assemble_mixed: block %d must be a mass, Laplace or Helmholtz form", q);
        if (bk.kind != FEM_MASS && !dat_ok(bk.coeff, args->cell_vertex->to, 1))
            return fail(ctx, FEM_E_ARG, "assemble_mixed: block %d needs a P1 coefficient Dat", q);
        if (!mats[q].sp || mats[q].sp->row_ptr != plan->row_ptr || mats[q].sp->col_idx != plan->col_idx ||
            mats[q].sp->nnz != plan->nnz)
            return fail(ctx, FEM_E_ARG, "assemble_mixed: block %d's sparsity differs from the plan's", q);
    }
    for (int32_t q = 0; q < nfields * nfields; ++q) {
        const fem_block &bk = blocks[q];
        if (!mats[q].values) continue;
        femk::AsmArgs a = base_args(ctx, plan, args);
        form_coeffs(bk.kind, &a.cstiff, &a.cmass);
        a.cstiff *= bk.scale;
        a.cmass *= bk.scale;
        a.coeff = bk.kind != FEM_MASS ? bk.coeff->data : args->coords->data;   // unread when cstiff == 0
        a.row_ptr = mats[q].sp->row_ptr;
        a.out = mats[q].values;
        a.inc = acc == FEM_INC;
        a.num_cus = ctx->num_cus;
        hipError_t e = femk::launch_mat(a, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "assemble_mixed launch");
    }
    return FEM_OK;
}

fem_status fem_apply_dirichlet(fem_ctx *ctx, const fem_sparsity *sp, double *values, const uint8_t *mask,
                               double diag, double *b, const double *g)
{
    if (!ctx) return FEM_E_ARG;
    if (!sp || !sp->row_ptr || (!sp->col_idx && sp->nnz > 0) || sp->nrows < 0)
        return fail(ctx, FEM_E_ARG, "apply_dirichlet: malformed sparsity");
    if (sp->nrows != sp->ncols) return fail(ctx, FEM_E_ARG, "apply_dirichlet: the Mat must be square");
    if ((!values && sp->nnz > 0) || (!mask && sp->nrows > 0))
        return fail(ctx, FEM_E_ARG, "apply_dirichlet: values and mask are required");
    if (g && !b) return fail(ctx, FEM_E_ARG, "apply_dirichlet: boundary values need a right-hand side");
    hipError_t e = femk::launch_dirichlet(sp, values, mask, diag, b, g, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "apply_dirichlet launch");
    return FEM_OK;
}

static fem_status renumber(fem_ctx *ctx, const fem_form *form, const fem_args *args, int32_t *cell_perm,
                           int32_t *vertex_perm, int32_t *node_perm);

fem_status fem_renumber(fem_ctx *ctx, const fem_form *form, const fem_args *args, int32_t *cell_perm,
                        int32_t *vertex_perm, int32_t *node_perm)
{
    try {
        return renumber(ctx, form, args, cell_perm, vertex_perm, node_perm);
    } catch (...) {
        return femk::caught_status(ctx, "renumber");
    }
}

static fem_status renumber(fem_ctx *ctx, const fem_form *form, const fem_args *args, int32_t *cell_perm,
                           int32_t *vertex_perm, int32_t *node_perm)
{
    if (!ctx) return FEM_E_ARG;
    fem_status st = check_form(ctx, form);
    if (st != FEM_OK) return st;
    if (form->kind == FEM_ELASTICITY)
        return fail(ctx, FEM_E_UNSUPPORTED, "renumber: use the scalar form of the same space");
    if ((st = check_args(ctx, form, args, false)) != FEM_OK) return st;
    const int dim = (int)form->cell, deg = form->degree, nl = nloc_of(dim, deg), nv = dim + 1;
    const int64_t ncells = args->cells->size, nverts = args->cell_vertex->to->size,
                  nnodes = args->cell_node->to->size;
    DevBuf flag(ctx);
    HIPC(flag.alloc(sizeof(int)), "alloc");
    if ((st = range_check(ctx, args->cell_vertex, flag.as<int>(), "cell_vertex")) != FEM_OK) return st;
    if ((st = range_check(ctx, args->cell_node, flag.as<int>(), "cell_node")) != FEM_OK) return st;
    std::vector<int32_t> cv(ncells * nv), cn(ncells * nl);
    std::vector<double> X(nverts * dim);
    hipStream_t s = ctx->stream;
    if (!cv.empty()) HIPC(hipMemcpyAsync(cv.data(), args->cell_vertex->values, cv.size() * 4, hipMemcpyDeviceToHost, s), "copy");
    if (!cn.empty()) HIPC(hipMemcpyAsync(cn.data(), args->cell_node->values, cn.size() * 4, hipMemcpyDeviceToHost, s), "copy");
    if (!X.empty()) HIPC(hipMemcpyAsync(X.data(), args->coords->data, X.size() * 8, hipMemcpyDeviceToHost, s), "copy");
    HIPC(hipStreamSynchronize(s), "sync");
    if (cell_perm) {
        std::vector<double> cen(ncells * dim, 0.0);
        for (int64_t c = 0; c < ncells; ++c)
            for (int m = 0; m < nv; ++m)
                for (int r = 0; r < dim; ++r) cen[c * dim + r] += X[(int64_t)cv[c * nv + m] * dim + r] / nv;
        sfc_order(cen, dim, ncells, cell_perm);
    }
    if (vertex_perm) sfc_order(X, dim, nverts, vertex_perm);
    if (node_perm) {
        std::vector<std::vector<int>> W;
        local_weights(dim, deg, W);
        std::vector<double> npos(nnodes * dim, 0.0);
        std::vector<char> seen(nnodes, 0);
        for (int64_t c = 0; c < ncells; ++c)
            for (int l = 0; l < nl; ++l) {
                const int32_t n = cn[c * nl + l];
                if (seen[n]) continue;
                seen[n] = 1;
                for (int r = 0; r < dim; ++r) {
                    double v = 0.0;
                    for (int m = 0; m < nv; ++m) v += W[l][m] * X[(int64_t)cv[c * nv + m] * dim + r];
                    npos[n * dim + r] = v / deg;
                }
            }
        sfc_order(npos, dim, nnodes, node_perm);
    }
    return FEM_OK;
}

}  // extern "C"
