// Exterior facet integrals (the mesh's Set of exterior facets is an iteration
// space of the parallel loop, "The mesh abstraction"): b_i (+)= sum over the
// facets F touching node i of the integral over F of g v_i ds, g a P1 field.
//
// Two kernels, deterministic and without atomics: one lane per facet
// evaluates its local vector (facet measure times the exact reference
// integrals of fem_facet_tables.h) into the plan's workspace; one lane per
// node row then sums the facet entries of its row, in ascending facet id
// (the node-to-facet incidence of the plan), and writes the row once.
#include "fem_internal.h"
#include "fem_facet_tables.h"

#include <cstdarg>
#include <cstdio>

namespace femk {
namespace {

template <int E, int K> struct FvSel;
template <> struct FvSel<1, 1> { using T = femfacet::FV11; };
template <> struct FvSel<1, 2> { using T = femfacet::FV12; };
template <> struct FvSel<1, 3> { using T = femfacet::FV13; };
template <> struct FvSel<2, 1> { using T = femfacet::FV21; };
template <> struct FvSel<2, 2> { using T = femfacet::FV22; };
template <> struct FvSel<2, 3> { using T = femfacet::FV23; };

// E: facet dimension (1: segments of a triangle mesh, 2: triangles of a
// tetrahedral mesh); coordinates have E + 1 components.
template <int E, int K>
__global__ __launch_bounds__(256) void k_facet_vec(const int32_t *__restrict__ fvert, const int32_t *__restrict__ fnode,
                                                   const double *__restrict__ X, const double *__restrict__ g,
                                                   double *__restrict__ work, int64_t nf)
{
    using T = typename FvSel<E, K>::T;
    constexpr int D = E + 1, NV = E + 1, NL = T::NLOC;
    const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (f >= nf) return;
    double x[NV][D], gv[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        const int64_t v = fvert[f * NV + m];
#pragma unroll
        for (int r = 0; r < D; ++r) x[m][r] = X[v * D + r];
        gv[m] = g[v];
    }
    double meas;   // |F| / |reference facet|: the length, or twice the area
    if constexpr (E == 1) {
        const double dx = x[1][0] - x[0][0], dy = x[1][1] - x[0][1];
        meas = sqrt(dx * dx + dy * dy);
    } else {
        const double u0 = x[1][0] - x[0][0], u1 = x[1][1] - x[0][1], u2 = x[1][2] - x[0][2];
        const double w0 = x[2][0] - x[0][0], w1 = x[2][1] - x[0][1], w2 = x[2][2] - x[0][2];
        const double cx = u1 * w2 - u2 * w1, cy = u2 * w0 - u0 * w2, cz = u0 * w1 - u1 * w0;
        meas = sqrt(cx * cx + cy * cy + cz * cz);
    }
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < NV; ++m) s = __builtin_fma(T::W[i][m], gv[m], s);
        work[f * NL + i] = meas * s;
    }
    (void)fnode;
}

__global__ __launch_bounds__(256) void k_facet_pull(const int64_t *__restrict__ ptr, const int32_t *__restrict__ ent,
                                                    const double *__restrict__ work, double *__restrict__ out,
                                                    int64_t nrows, int inc)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= nrows) return;
    double s = 0.0;
    for (int64_t k = ptr[r]; k < ptr[r + 1]; ++k) s += work[ent[k]];
    out[r] = inc ? out[r] + s : s;
}

fem_status ffail(fem_ctx *ctx, fem_status st, const char *fmt, ...)
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
fem_status fhip(fem_ctx *ctx, hipError_t e, const char *what)
{
    return ffail(ctx, e == hipErrorOutOfMemory ? FEM_E_NOMEM : FEM_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int facet_nloc(int e, int k) { return e == 1 ? k + 1 : (k + 1) * (k + 2) / 2; }

fem_status facet_check(fem_ctx *ctx, const fem_form *form, const fem_facets *fa)
{
    if (!form || form->kind != FEM_SOURCE || form->dim != 1 || form->prec != FEM_FP64 || form->degree < 1 ||
        form->degree > 3 || (form->cell != FEM_TRIANGLE && form->cell != FEM_TETRAHEDRON))
        return ffail(ctx, FEM_E_UNSUPPORTED, "facets: FEM_SOURCE, P1..P3, FP64, triangle or tetrahedron meshes");
    const int d = (int)form->cell, e = d - 1;
    if (!fa || !fa->facets || !fa->facet_vertex || !fa->facet_node || !fa->coords || !fa->g)
        return ffail(ctx, FEM_E_ARG, "facets: facets, facet_vertex, facet_node, coords and g are required");
    const fem_map *mv = fa->facet_vertex, *mn = fa->facet_node;
    if (!mv->from || !mv->to || !mn->from || !mn->to || mv->from->size != fa->facets->size ||
        mn->from->size != fa->facets->size || mv->arity != d || mn->arity != facet_nloc(e, form->degree) ||
        (fa->facets->size > 0 && (!mv->values || !mn->values)))
        return ffail(ctx, FEM_E_ARG, "facets: Maps from the facet Set with arities %d and %d", d,
                     facet_nloc(e, form->degree));
    if (!fa->coords->set || fa->coords->dim != d || fa->coords->set->size != mv->to->size ||
        (!fa->coords->data && mv->to->size > 0))
        return ffail(ctx, FEM_E_ARG, "facets: coords must be a dim-%d Dat on facet_vertex's target Set", d);
    if (!fa->g->set || fa->g->dim != 1 || fa->g->set->size != mv->to->size || (!fa->g->data && mv->to->size > 0))
        return ffail(ctx, FEM_E_ARG, "facets: g must be a scalar Dat on facet_vertex's target Set");
    if (fa->facets->size * (int64_t)mn->arity > INT32_MAX) return ffail(ctx, FEM_E_OVERFLOW, "facets: too many entries");
    return FEM_OK;
}

}  // namespace
}  // namespace femk

extern "C" {

static fem_status fem_facet_plan_create_impl(fem_ctx *ctx, const fem_form *form, const fem_facets *fa, fem_plan **out);

fem_status fem_facet_plan_create(fem_ctx *ctx, const fem_form *form, const fem_facets *fa, fem_plan **out)
{
    try {
        return fem_facet_plan_create_impl(ctx, form, fa, out);
    } catch (...) {
        return femk::caught_status(ctx, "facet_plan_create");
    }
}

static fem_status fem_facet_plan_create_impl(fem_ctx *ctx, const fem_form *form, const fem_facets *fa, fem_plan **out)
{
    using namespace femk;
    if (!ctx) return FEM_E_ARG;
    if (!out) return ffail(ctx, FEM_E_ARG, "facet_plan_create: NULL output");
    *out = nullptr;
    fem_status st = facet_check(ctx, form, fa);
    if (st != FEM_OK) return st;
    const int d = (int)form->cell, nl = facet_nloc(d - 1, form->degree);
    const int64_t nf = fa->facets->size, nrows = fa->facet_node->to->size;
    hipStream_t s = ctx->stream;
    int *flag = nullptr, hflag = 0;
    if (mem_alloc(ctx->mem, s, true, sizeof(int), (void **)&flag) != hipSuccess)
        return ffail(ctx, FEM_E_NOMEM, "facet_plan_create: alloc");
    for (const fem_map *m : {fa->facet_vertex, fa->facet_node}) {
        hipError_t e = fill_i32(flag, 1, 0, s);
        if (e == hipSuccess) e = check_range(m->values, m->from->size * (int64_t)m->arity, m->to->size, flag, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess || hflag) {
            mem_free(ctx->mem, s, true, flag);
            return e != hipSuccess ? fhip(ctx, e, "range check")
                                   : ffail(ctx, FEM_E_RANGE, "facet_plan_create: a Map entry lies outside its target Set");
        }
    }
    mem_free(ctx->mem, s, true, flag);
    fem_plan *p = new (std::nothrow) fem_plan;
    if (!p) return ffail(ctx, FEM_E_NOMEM, "facet_plan_create: host allocation");
    p->is_mat = 3;
    p->dim = d; p->degree = form->degree; p->nloc = nl;
    p->ncells = nf; p->nrows = nrows; p->nverts = fa->facet_vertex->to->size;
    p->cell_node = fa->facet_node->values;
    p->cell_vertex = fa->facet_vertex->values;
    p->cn_version = fa->facet_node->version;
    p->cv_version = fa->facet_vertex->version;
    p->mem = ctx->mem;
    int32_t *tmp = nullptr;
    int64_t *scan = nullptr;
    hipError_t e = mem_alloc(p->mem, s, false, sizeof(int64_t) * (nrows + 1), (void **)&p->f_ptr);
    if (e == hipSuccess) e = mem_alloc(p->mem, s, false, sizeof(int32_t) * (nf * nl ? nf * nl : 1), (void **)&p->f_ent);
    if (e == hipSuccess) e = mem_alloc(p->mem, s, false, sizeof(double) * (nf * nl ? nf * nl : 1), (void **)&p->f_work);
    if (e == hipSuccess) e = mem_alloc(ctx->mem, s, true, sizeof(int32_t) * (nrows + 1), (void **)&tmp);
    if (e == hipSuccess) e = mem_alloc(ctx->mem, s, true, sizeof(int64_t) * scan_scratch(nrows), (void **)&scan);
    if (e == hipSuccess) e = build_incidence(fa->facet_node->values, nf, nl, nrows, p->f_ptr, p->f_ent, tmp, scan, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    mem_free(ctx->mem, s, true, tmp);
    mem_free(ctx->mem, s, true, scan);
    if (e != hipSuccess) {
        fem_plan_destroy(p);
        return fhip(ctx, e, "facet_plan_create");
    }
    p->bytes = sizeof(int64_t) * (nrows + 1) + (sizeof(int32_t) + sizeof(double)) * nf * nl;
    p->cell_visits = nf;
    *out = p;
    return FEM_OK;
}

fem_status fem_par_loop_assemble_facets(fem_ctx *ctx, const fem_plan *plan, const fem_form *form, const fem_facets *fa,
                                        fem_dat *b, fem_access acc)
{
    using namespace femk;
    if (!ctx) return FEM_E_ARG;
    fem_status st = facet_check(ctx, form, fa);
    if (st != FEM_OK) return st;
    if (!plan || plan->is_mat != 3 || plan->dim != (int)form->cell || plan->degree != form->degree ||
        plan->cell_node != fa->facet_node->values || plan->ncells != fa->facets->size ||
        plan->nrows != fa->facet_node->to->size)
        return ffail(ctx, FEM_E_ARG, "assemble_facets: the plan was built for other facets");
    if (plan->cn_version != fa->facet_node->version)
        return ffail(ctx, FEM_E_ARG, "assemble_facets: the plan was built for another version of its Maps");
    if (!b || !b->set || b->dim != 1 || b->set->size != plan->nrows || (!b->data && plan->nrows > 0))
        return ffail(ctx, FEM_E_ARG, "assemble_facets: b must be a Dat on facet_node's target Set");
    if (acc != FEM_WRITE && acc != FEM_INC) return ffail(ctx, FEM_E_ARG, "output access must be WRITE or INC");
    hipStream_t s = ctx->stream;
    const int64_t nf = plan->ncells;
    if (nf > 0) {
        const dim3 grid((unsigned)((nf + 255) / 256));
        const int32_t *fv = fa->facet_vertex->values, *fn = fa->facet_node->values;
        const double *X = fa->coords->data, *g = fa->g->data;
        switch ((plan->dim - 1) * 10 + plan->degree) {
        case 11: hipLaunchKernelGGL((k_facet_vec<1, 1>), grid, dim3(256), 0, s, fv, fn, X, g, plan->f_work, nf); break;
        case 12: hipLaunchKernelGGL((k_facet_vec<1, 2>), grid, dim3(256), 0, s, fv, fn, X, g, plan->f_work, nf); break;
        case 13: hipLaunchKernelGGL((k_facet_vec<1, 3>), grid, dim3(256), 0, s, fv, fn, X, g, plan->f_work, nf); break;
        case 21: hipLaunchKernelGGL((k_facet_vec<2, 1>), grid, dim3(256), 0, s, fv, fn, X, g, plan->f_work, nf); break;
        case 22: hipLaunchKernelGGL((k_facet_vec<2, 2>), grid, dim3(256), 0, s, fv, fn, X, g, plan->f_work, nf); break;
        case 23: hipLaunchKernelGGL((k_facet_vec<2, 3>), grid, dim3(256), 0, s, fv, fn, X, g, plan->f_work, nf); break;
        default: return ffail(ctx, FEM_E_UNSUPPORTED, "assemble_facets: degree");
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fhip(ctx, e, "assemble_facets launch");
    }
    if (plan->nrows > 0) {
        hipLaunchKernelGGL(k_facet_pull, dim3((unsigned)((plan->nrows + 255) / 256)), dim3(256), 0, s, plan->f_ptr,
                           plan->f_ent, plan->f_work, b->data, plan->nrows, (int)(acc == FEM_INC));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fhip(ctx, e, "assemble_facets launch");
    }
    return FEM_OK;
}

}  // extern "C"
