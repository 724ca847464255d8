// Dirichlet rows and columns of an assembled system, applied in place (the
// boundary condition the paper's Firedrake example passes to assemble and
// applies to the right-hand side).  One lane per CSR row, rows independent:
// a boundary row becomes diag on the diagonal and zero elsewhere, with
// b[r] = diag g[r]; a free row lifts the boundary values of its boundary
// columns into b (b[r] -= A[r][c] g[c], in column order) and zeroes those
// entries.  Symmetric; no atomics; deterministic.
#include "fem_internal.h"

namespace femk {
namespace {

__global__ __launch_bounds__(256) void k_dirichlet(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                   double *__restrict__ v, int64_t nrows,
                                                   const uint8_t *__restrict__ mask, double diag,
                                                   double *__restrict__ b, const double *__restrict__ g)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= nrows) return;
    const int64_t k0 = rp[r], k1 = rp[r + 1];
    if (mask[r]) {
        for (int64_t k = k0; k < k1; ++k) v[k] = ci[k] == r ? diag : 0.0;
        if (b) b[r] = g ? diag * g[r] : 0.0;
        return;
    }
    double acc = b ? b[r] : 0.0;
    for (int64_t k = k0; k < k1; ++k) {
        const int32_t c = ci[k];
        if (mask[c]) {
            if (g) acc -= v[k] * g[c];
            v[k] = 0.0;
        }
    }
    if (b) b[r] = acc;
}

}  // namespace

hipError_t launch_dirichlet(const fem_sparsity *sp, double *values, const uint8_t *mask, double diag, double *b,
                            const double *g, hipStream_t s)
{
    if (sp->nrows == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dirichlet, dim3((unsigned)((sp->nrows + 255) / 256)), dim3(256), 0, s, sp->row_ptr,
                       sp->col_idx, values, sp->nrows, mask, diag, b, g);
    return hipGetLastError();
}

}  // namespace femk
