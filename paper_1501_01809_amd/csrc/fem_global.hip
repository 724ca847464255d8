// Global reductions over the cells (PyOP2 Globals with SUM, MIN or MAX
// access, "Global arguments"): each cell contributes one value -- its
// energy x_K^T A_K x_K under the bilinear form, or the integral of the P1
// field f over K -- and the Global receives their sum, minimum or maximum.
//
// Deterministic: cells are assigned to workgroups and lanes by index only
// (workgroup b takes cells [1024 b, 1024 (b+1)), lane t the cells
// 1024 b + t + 256 j, j = 0..3, combined in that order), each workgroup
// combines its lanes by a fixed LDS tree into one partial, and one workgroup
// combines the partials the same way.  The value is bitwise reproducible.
#include "fem_internal.h"
#include "fem_geom.h"
#include "fem_tables.h"

namespace femk {
namespace {

constexpr int RWG = 256, RPT = 4, RCH = RWG * RPT;   // cells per workgroup

template <int D, int K> struct TabSel;
template <> struct TabSel<2, 1> { using T = femtab::Tab21; };
template <> struct TabSel<2, 2> { using T = femtab::Tab22; };
template <> struct TabSel<2, 3> { using T = femtab::Tab23; };
template <> struct TabSel<3, 1> { using T = femtab::Tab31; };
template <> struct TabSel<3, 2> { using T = femtab::Tab32; };
template <> struct TabSel<3, 3> { using T = femtab::Tab33; };

struct RedArgs {
    const int32_t *__restrict__ cell_vertex;
    const double *__restrict__ coords;
    const int32_t *__restrict__ cell_node;
    const double *__restrict__ field;     // kappa (energy) or f (integral)
    const double *__restrict__ x;         // energy: the field of the P_k space
    double *__restrict__ partial;
    double cstiff, cmass;
    int64_t ncells;
    int mode;                             // 0 SUM, 1 MIN, 2 MAX
};

__device__ __forceinline__ double identity(int mode)
{
    return mode == 0 ? 0.0 : (mode == 1 ? __builtin_huge_val() : -__builtin_huge_val());
}
__device__ __forceinline__ double combine(int mode, double a, double b)
{
    return mode == 0 ? a + b : (mode == 1 ? fmin(a, b) : fmax(a, b));
}

// Fixed-shape tree over the RWG lane values in LDS; returns the result in lane 0.
__device__ __forceinline__ double tree(double *s, int mode, double v)
{
    const int t = threadIdx.x;
    s[t] = v;
    __syncthreads();
#pragma unroll
    for (int w = RWG / 2; w > 0; w >>= 1) {
        if (t < w) s[t] = combine(mode, s[t], s[t + w]);
        __syncthreads();
    }
    return s[0];
}

template <int D, int K, bool ENERGY>
__global__ __launch_bounds__(RWG) void k_reduce_cells(RedArgs a)
{
    using Tab = typename TabSel<D, K>::T;
    constexpr int NV = D + 1, NL = Tab::NLOC, NM = Geo<D>::NM;
    __shared__ double s[RWG];
    double acc = identity(a.mode);
#pragma unroll 1
    for (int j = 0; j < RPT; ++j) {
        const int64_t c = (int64_t)blockIdx.x * RCH + j * RWG + threadIdx.x;
        if (c >= a.ncells) continue;
        double x[NV][D], k[NV];
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            const int64_t v = a.cell_vertex[c * NV + m];
#pragma unroll
            for (int r = 0; r < D; ++r) x[m][r] = a.coords[v * D + r];
            k[m] = a.field[v];
        }
        double q = 0.0;
        if constexpr (ENERGY) {
            double G[NM];
            const double adet = Geo<D>::metric(x, G);
            double xl[NL], y[NL];
#pragma unroll
            for (int i = 0; i < NL; ++i) { xl[i] = a.x[a.cell_node[c * NL + i]]; y[i] = 0.0; }
            double kc[NV];
#pragma unroll
            for (int m = 0; m < NV; ++m) kc[m] = a.cstiff * k[m];
            if constexpr (K == 1) Tab::act_t(kc, G, a.cmass * adet, xl, y);   // terms grouped by metric pair
            else Tab::act_q(kc, G, a.cmass * adet, xl, y);   // stiffness at the points of an exact rule
#pragma unroll
            for (int i = 0; i < NL; ++i) q = __builtin_fma(xl[i], y[i], q);
        } else {
            double b[NL];
            Tab::vec(k, Geo<D>::absdet(x), b);
#pragma unroll
            for (int i = 0; i < NL; ++i) q += b[i];
        }
        acc = combine(a.mode, acc, q);
    }
    const double r = tree(s, a.mode, acc);
    if (threadIdx.x == 0) a.partial[blockIdx.x] = r;
}

__global__ __launch_bounds__(RWG) void k_reduce_final(const double *__restrict__ partial, int64_t n, int mode,
                                                      double *__restrict__ g)
{
    __shared__ double s[RWG];
    double acc = identity(mode);
    for (int64_t i = threadIdx.x; i < n; i += RWG) acc = combine(mode, acc, partial[i]);
    const double r = tree(s, mode, acc);
    if (threadIdx.x == 0) g[0] = combine(mode, g[0], r);
}

template <int D, int K>
hipError_t reduce_dispatch(const RedArgs &a, bool energy, hipStream_t s)
{
    const unsigned nb = (unsigned)((a.ncells + RCH - 1) / RCH);
    if (energy) hipLaunchKernelGGL((k_reduce_cells<D, K, true>), dim3(nb), dim3(RWG), 0, s, a);
    else hipLaunchKernelGGL((k_reduce_cells<D, K, false>), dim3(nb), dim3(RWG), 0, s, a);
    return hipGetLastError();
}

}  // namespace

int64_t reduce_partials(int64_t ncells) { return (ncells + RCH - 1) / RCH; }

hipError_t launch_reduce(const AsmArgs &a, double *partial, int mode, bool energy, double *g, hipStream_t s)
{
    RedArgs r;
    r.cell_vertex = a.cell_vertex; r.coords = a.coords; r.cell_node = a.cell_node;
    r.field = a.coeff; r.x = a.x; r.partial = partial;
    r.cstiff = a.cstiff; r.cmass = a.cmass;
    r.ncells = a.plan->ncells; r.mode = mode;
    hipError_t e = hipSuccess;
    if (r.ncells > 0) {
        switch (a.plan->dim * 10 + a.plan->degree) {
        case 21: e = reduce_dispatch<2, 1>(r, energy, s); break;
        case 22: e = reduce_dispatch<2, 2>(r, energy, s); break;
        case 23: e = reduce_dispatch<2, 3>(r, energy, s); break;
        case 31: e = reduce_dispatch<3, 1>(r, energy, s); break;
        case 32: e = reduce_dispatch<3, 2>(r, energy, s); break;
        case 33: e = reduce_dispatch<3, 3>(r, energy, s); break;
        default: return hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RWG), 0, s, partial, reduce_partials(r.ncells), mode, g);
    return hipGetLastError();
}

}  // namespace femk
