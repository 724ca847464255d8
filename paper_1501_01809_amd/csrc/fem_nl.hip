// Nonlinear residual and adjoint (vector-Jacobian) assembly for gfx950.
//
// The residual of a nonlinear form, F(u, kappa)_i = integral of
// kappa grad(u).grad(v_i) + u^3 v_i - f v_i on a P1 space, and the products
// lambda^T dF/du and lambda^T dF/dkappa that the adjoint of F needs (the
// paper's outlook: adjoint models derived through the same parallel loop
// abstraction).  The parallel loop is the one of the Dat plans: a workgroup
// owns a contiguous block of rows, evaluates every cell incident to them
// (gathering coordinates and the node fields through the Maps), keeps the
// local values in LDS and sums each row's entries in ascending cell id, so
// the result is bitwise reproducible and needs no atomics.
#include "fem_internal.h"

#include <algorithm>

namespace femk {
namespace {

constexpr int VWG = 512;                      // lanes per workgroup (the Dat plans' block shape)
constexpr int LDS_BYTES = 163840;             // gfx950: 160 KiB of LDS per CU
constexpr int LB = 2;                         // bits of the local index in a plan entry (P1: 3 or 4 locals)

struct NlArgs {
    const int32_t *__restrict__ blk_row0;
    const int32_t *__restrict__ blk_cptr;
    const int32_t *__restrict__ bcell;
    const int32_t *__restrict__ bverts;
    const int32_t *__restrict__ inc_ptr;
    const uint16_t *__restrict__ ent;
    const double *__restrict__ coords;
    const int32_t *__restrict__ cell_node;
    const double *__restrict__ u;
    const double *__restrict__ kappa;
    const double *__restrict__ w;             // f (residual) or lambda (products)
    double *__restrict__ out;
    double *__restrict__ out2;                // lambda^T dF/dkappa when both products are assembled
    int inc;
    int ncap;                                 // most cells of one block
};

NlArgs nl_args(const AsmArgs &a)
{
    const fem_plan &p = *a.plan;
    NlArgs k;
    k.blk_row0 = p.blk_row0; k.blk_cptr = p.blk_cptr; k.bcell = p.bcell; k.bverts = p.bverts;
    k.inc_ptr = p.inc_ptr; k.ent = p.ent;
    k.coords = a.coords; k.cell_node = a.cell_node;
    k.u = a.x; k.kappa = a.coeff; k.w = a.aux;
    k.out = a.out; k.out2 = a.out2;
    k.inc = a.inc;
    k.ncap = p.max_blk_cells;
    return k;
}

// Barrier for LDS traffic only (the kernel communicates through LDS; inputs
// are read-only and each output element is written by one lane).
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Exact integral over a simplex of dimension D of the product of the
// barycentrics l_m l_n l_p l_i (W4) or l_m l_i (W2), divided by the volume:
// D! prod(a!) / (|a| + D)! for the exponent multi-index a.
constexpr double nl_fact(int n) { return n <= 1 ? 1.0 : n * nl_fact(n - 1); }
template <int D>
constexpr double nl_moment(int m, int n, int p, int i, int deg)
{
    double num = 1.0;
    for (int v = 0; v <= D; ++v) {
        const int c = (m == v) + (n == v) + (deg == 4 ? (p == v) + (i == v) : 0);
        num *= nl_fact(c);
    }
    return nl_fact(D) * num / nl_fact(deg + D);
}
// The moments as a compile-time table (indexed by unrolled loop counters, so
// every entry is an immediate in the kernel).
template <int D>
struct NlMoments {
    double w4[D + 1][D + 1][D + 1][D + 1];
    double w2[D + 1][D + 1];
    constexpr NlMoments() : w4{}, w2{}
    {
        for (int m = 0; m <= D; ++m)
            for (int i = 0; i <= D; ++i) {
                w2[m][i] = nl_moment<D>(m, i, 0, 0, 2);
                for (int n = 0; n <= D; ++n)
                    for (int p = 0; p <= D; ++p) w4[m][n][p][i] = nl_moment<D>(m, n, p, i, 4);
            }
    }
};

// Local values of one P1 cell of the residual kappa grad(u).grad(v) +
// u^3 v - f v (MODE 0) or of its vector-Jacobian products with lambda (MODE
// 1: d/du, MODE 2: d/dkappa, MODE 3: both, d/dkappa into lk); w holds f
// (MODE 0) or lambda.  Every integral is exact: integral of kappa = |K|
// mean(kappa), |K| grad(l_m).grad(l_n) = (a_m . a_n) / (|det J| D!) with a_m
// the rows of adj(J), and the barycentric moments above.  c holds the edge
// vectors x_{q+1} - x_0, formed in FP64 by the caller so that a narrower R
// does not lose the short edges of a fine mesh to cancellation; all other
// arithmetic in R.
template <int D, int MODE, typename R>
__device__ __forceinline__ void nl_local(const R (&c)[D][D], const R (&u)[D + 1], const R (&k)[D + 1],
                                         const R (&w)[D + 1], R (&loc)[D + 1], R (&lk)[D + 1])
{
    constexpr int NV = D + 1;
    constexpr NlMoments<D> MOM{};
    R a[NV][D], det;
    if constexpr (D == 2) {
        const R c1x = c[0][0], c1y = c[0][1], c2x = c[1][0], c2y = c[1][1];
        det = c1x * c2y - c1y * c2x;
        a[1][0] = c2y; a[1][1] = -c2x; a[2][0] = -c1y; a[2][1] = c1x;
    } else {
        a[1][0] = c[1][1] * c[2][2] - c[1][2] * c[2][1];
        a[1][1] = c[1][2] * c[2][0] - c[1][0] * c[2][2];
        a[1][2] = c[1][0] * c[2][1] - c[1][1] * c[2][0];
        a[2][0] = c[2][1] * c[0][2] - c[2][2] * c[0][1];
        a[2][1] = c[2][2] * c[0][0] - c[2][0] * c[0][2];
        a[2][2] = c[2][0] * c[0][1] - c[2][1] * c[0][0];
        a[3][0] = c[0][1] * c[1][2] - c[0][2] * c[1][1];
        a[3][1] = c[0][2] * c[1][0] - c[0][0] * c[1][2];
        a[3][2] = c[0][0] * c[1][1] - c[0][1] * c[1][0];
        det = c[0][0] * a[1][0] + c[0][1] * a[1][1] + c[0][2] * a[1][2];
    }
#pragma unroll
    for (int r = 0; r < D; ++r) {
        R s = 0;
#pragma unroll
        for (int m = 1; m < NV; ++m) s += a[m][r];
        a[0][r] = -s;
    }
    const R adet = det < R(0) ? -det : det;
    constexpr double DFACT = nl_fact(D);
    const R vol = adet / R(DFACT);
    const R sc = R(1) / (adet * R(DFACT));   // |K| grad l_m . grad l_n = (a_m . a_n) * sc
    R kbar = 0;
#pragma unroll
    for (int m = 0; m < NV; ++m) kbar += k[m];
    kbar = kbar / R(NV);
    // grad(u) and grad(w) scaled: (sum_m u_m a_m)
    R gu[D], gw[D];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        gu[r] = 0; gw[r] = 0;
#pragma unroll
        for (int m = 0; m < NV; ++m) { gu[r] += u[m] * a[m][r]; gw[r] += w[m] * a[m][r]; }
    }
    if constexpr (MODE >= 2) {
        R t = 0;
#pragma unroll
        for (int r = 0; r < D; ++r) t += gu[r] * gw[r];
        t = t * sc / R(NV);
#pragma unroll
        for (int i = 0; i < NV; ++i) (MODE == 2 ? loc : lk)[i] = t;
    }
    if constexpr (MODE != 2) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            R g = 0;
#pragma unroll
            for (int r = 0; r < D; ++r) g += (MODE == 0 ? gu[r] : gw[r]) * a[i][r];
            R cub = 0;
#pragma unroll
            for (int m = 0; m < NV; ++m)
#pragma unroll
                for (int n = 0; n < NV; ++n) {
                    const R umn = u[m] * u[n];
#pragma unroll
                    for (int p = 0; p < NV; ++p)
                        cub += umn * (MODE == 0 ? u[p] : w[p]) * R(MOM.w4[m][n][p][i]);
                }
            if constexpr (MODE == 0) {
                R src = 0;
#pragma unroll
                for (int m = 0; m < NV; ++m) src += w[m] * R(MOM.w2[m][i]);
                loc[i] = kbar * g * sc + vol * (cub - src);
            } else {
                loc[i] = kbar * g * sc + R(3) * vol * cub;
            }
        }
    }
}

// Row-owned Dat assembly of the nonlinear residual or of its vector-Jacobian
// products, on a P1 Dat plan: the source vector's schedule (each lane
// computes the local values of its cells into LDS, each row sums its cells'
// values in ascending cell order), arithmetic in R.  LDS is dynamic, NOUT
// arrays of ncap x NL values.  Each lane takes two cells per pass and issues
// both cells' loads before either's arithmetic, so a block of up to 2 VWG
// cells pays one chain of dependent loads.
template <int D, int MODE, typename R>
__global__ __launch_bounds__(VWG) void k_assemble_nl(NlArgs a)
{
    constexpr int NL = D + 1;
    static_assert(NL <= (1 << LB), "P1 locals fit the entry's local bits");
    extern __shared__ double nl_lds[];
    R *vk = reinterpret_cast<R *>(nl_lds);
    const int stride = a.ncap * NL;           // offset of the second output (MODE 3)
    const int b = blockIdx.x, tid = threadIdx.x;
    const int r0 = a.blk_row0[b], r1 = a.blk_row0[b + 1];
    const int c0 = a.blk_cptr[b], nc = a.blk_cptr[b + 1] - c0;
    for (int c = tid; c < nc; c += 2 * VWG) {
        const bool two = c + VWG < nc;
        const int cc[2] = {c, two ? c + VWG : c};
        double x[2][NL][D];
        R u[2][NL], k[2][NL], w[2][NL];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t cell = a.bcell[c0 + cc[h]];
#pragma unroll
            for (int m = 0; m < NL; ++m) {
                const int64_t v = a.bverts[(int64_t)(c0 + cc[h]) * NL + m];
#pragma unroll
                for (int r = 0; r < D; ++r) x[h][m][r] = a.coords[v * D + r];
                const int64_t nd = a.cell_node[cell * NL + m];
                u[h][m] = R(a.u[nd]);
                k[h][m] = R(a.kappa[nd]);
                w[h][m] = R(a.w[nd]);
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            R e[D][D], loc[NL], lk[NL];
#pragma unroll
            for (int q = 0; q < D; ++q)
#pragma unroll
                for (int r = 0; r < D; ++r) e[q][r] = R(x[h][q + 1][r] - x[h][0][r]);
            nl_local<D, MODE, R>(e, u[h], k[h], w[h], loc, lk);
            if (h == 0 || two) {
#pragma unroll
                for (int j = 0; j < NL; ++j) {
                    vk[cc[h] * NL + j] = loc[j];
                    if constexpr (MODE == 3) vk[stride + cc[h] * NL + j] = lk[j];
                }
            }
        }
    }
    lds_barrier();
    for (int r = r0 + tid; r < r1; r += VWG) {
        R acc = 0, acc2 = 0;
        for (int e = a.inc_ptr[r]; e < a.inc_ptr[r + 1]; ++e) {
            const uint32_t pe = a.ent[e];
            const int at = (int)(pe >> LB) * NL + (int)(pe & ((1u << LB) - 1));
            acc += vk[at];
            if constexpr (MODE == 3) acc2 += vk[stride + at];
        }
        a.out[r] = a.inc ? a.out[r] + (double)acc : (double)acc;
        if constexpr (MODE == 3) a.out2[r] = a.inc ? a.out2[r] + (double)acc2 : (double)acc2;
    }
}

template <int D, int MODE, typename R>
hipError_t nl_launch_r(const AsmArgs &a, hipStream_t s)
{
    constexpr int NOUT = MODE == 3 ? 2 : 1;
    const size_t lds = (size_t)NOUT * (size_t)std::max(a.plan->max_blk_cells, 1) * (D + 1) * sizeof(R);
    if (lds > (size_t)LDS_BYTES) return hipErrorInvalidValue;
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_assemble_nl<D, MODE, R>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_assemble_nl<D, MODE, R>), dim3(a.plan->nblk), dim3(VWG), lds, s, nl_args(a));
    return hipGetLastError();
}

template <int D, int MODE>
hipError_t nl_launch(const AsmArgs &a, bool fp32, hipStream_t s)
{
    return fp32 ? nl_launch_r<D, MODE, float>(a, s) : nl_launch_r<D, MODE, double>(a, s);
}

}  // namespace

hipError_t launch_nl(const AsmArgs &a, int mode, bool fp32, hipStream_t s)
{
    if (a.plan->nblk == 0) return hipSuccess;
    if (a.plan->degree != 1 || a.plan->is_mat || a.plan->lbits != LB) return hipErrorInvalidValue;
    if (mode == 3 && !a.out2) return hipErrorInvalidValue;
    const int key = a.plan->dim * 10 + mode;
    switch (key) {
    case 20: return nl_launch<2, 0>(a, fp32, s);
    case 21: return nl_launch<2, 1>(a, fp32, s);
    case 22: return nl_launch<2, 2>(a, fp32, s);
    case 23: return nl_launch<2, 3>(a, fp32, s);
    case 30: return nl_launch<3, 0>(a, fp32, s);
    case 31: return nl_launch<3, 1>(a, fp32, s);
    case 32: return nl_launch<3, 2>(a, fp32, s);
    case 33: return nl_launch<3, 3>(a, fp32, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace femk
