// Dirichlet rows and columns of an assembled system, applied in place (the
// boundary condition the paper's Firedrake example passes to assemble and
// applies to the right-hand side).  LPR lanes per CSR row (the row's column
// indices and values are read coalesced), rows independent: a boundary row
// becomes diag on the diagonal and zero elsewhere, with b[r] = diag g[r]; a
// free row lifts the boundary values of its boundary columns into b
// (b[r] -= sum over them of A[r][c] g[c], the sum taken by a fixed butterfly
// over the row's lanes) and zeroes those entries.  Symmetric; no atomics;
// bitwise reproducible.
#include "fem_internal.h"

#include <algorithm>

namespace femk {
namespace {

constexpr int LPR = 8;    // lanes per row (8 rows per wave: more independent loads in flight)

__global__ __launch_bounds__(256) void k_dirichlet(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                   double *__restrict__ v, int64_t row0, int64_t nrows,
                                                   const uint8_t *__restrict__ mask, double diag,
                                                   double *__restrict__ b, const double *__restrict__ g)
{
    // the lanes of a row share r: they leave together, and the butterfly
    // below pairs lanes of one row only
    const int64_t r = row0 + ((int64_t)blockIdx.x * 256 + threadIdx.x) / LPR;
    const int sub = threadIdx.x % LPR;
    if (r >= nrows) return;
    const int64_t k0 = rp[r], k1 = rp[r + 1];
    if (mask[r]) {
        for (int64_t k = k0 + sub; k < k1; k += LPR) v[k] = ci[k] == r ? diag : 0.0;
        if (sub == 0 && b) b[r] = g ? diag * g[r] : 0.0;
        return;
    }
    double part = 0.0;
#pragma unroll 4
    for (int64_t k = k0 + sub; k < k1; k += LPR) {
        const int32_t c = ci[k];
        if (mask[c]) {
            if (g) part += v[k] * g[c];
            v[k] = 0.0;
        }
    }
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) part += __shfl_xor(part, o, LPR);
    if (sub == 0 && b) b[r] -= part;
}

}  // namespace

hipError_t launch_dirichlet(const fem_sparsity *sp, double *values, const uint8_t *mask, double diag, double *b,
                            const double *g, hipStream_t s)
{
    if (sp->nrows == 0) return hipSuccess;
    // at most 2^25 rows (2^28 work-items) per launch
    constexpr int64_t CHUNK = (int64_t)1 << 25;
    for (int64_t row0 = 0; row0 < sp->nrows; row0 += CHUNK) {
        const int64_t lanes = std::min(CHUNK, sp->nrows - row0) * LPR;
        hipLaunchKernelGGL(k_dirichlet, dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, s, sp->row_ptr,
                           sp->col_idx, values, row0, sp->nrows, mask, diag, b, g);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace femk
