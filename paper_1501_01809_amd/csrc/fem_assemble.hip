// Cell-loop assembly kernels for gfx950 (MI355X).
//
// The parallel loop of the paper ("Parloops and kernels") runs the local
// kernel on every cell with data gathered through Maps (READ) and adds the
// element tensor into the output (INC).  Here the INC is made conflict-free
// and deterministic by owning OUTPUT ROWS instead of colouring cells: the plan
// splits the rows into contiguous blocks; one workgroup owns a block and
// visits, in ascending order, every cell incident to its rows.  Per chunk of
// cells it
//   1. gathers the cells' vertex coordinates and P1 coefficients,
//   2. computes the FP64 geometry (adjugate, |det J|, metric
//      |det J| grad(l_m).grad(l_n)) and the element tensor from the exact
//      reference integrals (generated straight-line FMA code), into LDS,
//   3. lets every lane pull, for the rows it owns, the contributions of the
//      chunk's cells in ascending cell order into an LDS accumulator,
// and finally writes its rows once, contiguously (the block's rows occupy one
// contiguous range of the CSR values).  No atomics and no inter-workgroup
// communication are used, so the result is bitwise reproducible; the price is
// that a cell straddling two row blocks is evaluated by both.
#include "fem_internal.h"
#include "fem_tables.h"

namespace femk {
namespace {

constexpr int WG = 256;

// Everything a kernel reads, by value: device pointers and scalars only.
struct KArgs {
    const int32_t *__restrict__ blk_row0;
    const int32_t *__restrict__ blk_cptr;
    const int32_t *__restrict__ bcell;
    const int32_t *__restrict__ inc_ptr;
    const uint16_t *__restrict__ ent;
    const void *__restrict__ gpos;
    int gstride;
    const int64_t *__restrict__ row_ptr;
    const int32_t *__restrict__ cell_vertex;
    const double *__restrict__ coords;
    const int32_t *__restrict__ cell_node;
    const double *__restrict__ coeff;
    const double *__restrict__ x;
    double *__restrict__ out;
    double cstiff, cmass;
    int inc;
};

KArgs kargs(const AsmArgs &a)
{
    const fem_plan &p = *a.plan;
    KArgs k;
    k.blk_row0 = p.blk_row0; k.blk_cptr = p.blk_cptr; k.bcell = p.bcell;
    k.inc_ptr = p.inc_ptr; k.ent = p.ent; k.gpos = p.gpos; k.gstride = p.gstride;
    k.row_ptr = a.row_ptr; k.cell_vertex = a.cell_vertex; k.coords = a.coords;
    k.cell_node = a.cell_node; k.coeff = a.coeff; k.x = a.x; k.out = a.out;
    k.cstiff = a.cstiff; k.cmass = a.cmass; k.inc = a.inc;
    return k;
}
constexpr int LDS_DOUBLES = 163840 / 8;    // gfx950: 160 KiB of LDS per CU

// ---------------------------------------------------------------- geometry

template <int D> struct Geo;

template <> struct Geo<2> {
    static constexpr int NM = 6;
    // Metric G[mn] = |det J| grad(l_m).grad(l_n) for m <= n (lexicographic);
    // returns |det J|.
    __device__ __forceinline__ static double metric(const double (&x)[3][2], double (&G)[NM])
    {
        const double c1x = x[1][0] - x[0][0], c1y = x[1][1] - x[0][1];
        const double c2x = x[2][0] - x[0][0], c2y = x[2][1] - x[0][1];
        const double det = c1x * c2y - c1y * c2x;
        // rows of adj(J): J^{-1} = adj(J) / det
        const double a[3][2] = {{-(c2y - c1y), -(c1x - c2x)}, {c2y, -c2x}, {-c1y, c1x}};
        const double adet = fabs(det), inv = 1.0 / adet;
        int t = 0;
        for (int m = 0; m < 3; ++m)
            for (int n = m; n < 3; ++n) G[t++] = (a[m][0] * a[n][0] + a[m][1] * a[n][1]) * inv;
        return adet;
    }
    __device__ __forceinline__ static double absdet(const double (&x)[3][2])
    {
        const double c1x = x[1][0] - x[0][0], c1y = x[1][1] - x[0][1];
        const double c2x = x[2][0] - x[0][0], c2y = x[2][1] - x[0][1];
        return fabs(c1x * c2y - c1y * c2x);
    }
};

template <> struct Geo<3> {
    static constexpr int NM = 10;
    __device__ __forceinline__ static double metric(const double (&x)[4][3], double (&G)[NM])
    {
        double c[3][3];
        for (int k = 0; k < 3; ++k)
            for (int r = 0; r < 3; ++r) c[k][r] = x[k + 1][r] - x[0][r];
        double a[4][3];
        // rows of adj(J) for J = [c1 c2 c3]: c2 x c3, c3 x c1, c1 x c2
        a[1][0] = c[1][1] * c[2][2] - c[1][2] * c[2][1];
        a[1][1] = c[1][2] * c[2][0] - c[1][0] * c[2][2];
        a[1][2] = c[1][0] * c[2][1] - c[1][1] * c[2][0];
        a[2][0] = c[2][1] * c[0][2] - c[2][2] * c[0][1];
        a[2][1] = c[2][2] * c[0][0] - c[2][0] * c[0][2];
        a[2][2] = c[2][0] * c[0][1] - c[2][1] * c[0][0];
        a[3][0] = c[0][1] * c[1][2] - c[0][2] * c[1][1];
        a[3][1] = c[0][2] * c[1][0] - c[0][0] * c[1][2];
        a[3][2] = c[0][0] * c[1][1] - c[0][1] * c[1][0];
        const double det = c[0][0] * a[1][0] + c[0][1] * a[1][1] + c[0][2] * a[1][2];
        for (int r = 0; r < 3; ++r) a[0][r] = -(a[1][r] + a[2][r] + a[3][r]);
        const double adet = fabs(det), inv = 1.0 / adet;
        int t = 0;
        for (int m = 0; m < 4; ++m)
            for (int n = m; n < 4; ++n)
                G[t++] = (a[m][0] * a[n][0] + a[m][1] * a[n][1] + a[m][2] * a[n][2]) * inv;
        return adet;
    }
    __device__ __forceinline__ static double absdet(const double (&x)[4][3])
    {
        const double c1x = x[1][0] - x[0][0], c1y = x[1][1] - x[0][1], c1z = x[1][2] - x[0][2];
        const double c2x = x[2][0] - x[0][0], c2y = x[2][1] - x[0][1], c2z = x[2][2] - x[0][2];
        const double c3x = x[3][0] - x[0][0], c3y = x[3][1] - x[0][1], c3z = x[3][2] - x[0][2];
        return fabs(c1x * (c2y * c3z - c2z * c3y) - c1y * (c2x * c3z - c2z * c3x) +
                    c1z * (c2x * c3y - c2y * c3x));
    }
};

// Gather the cell's vertex coordinates and the P1 coefficient at its vertices.
template <int D>
__device__ __forceinline__ void gather_cell(int64_t c, const int32_t *__restrict__ cv,
                                            const double *__restrict__ X,
                                            const double *__restrict__ coef, double (&x)[D + 1][D],
                                            double (&k)[D + 1])
{
#pragma unroll
    for (int m = 0; m <= D; ++m) {
        const int64_t v = cv[c * (D + 1) + m];
#pragma unroll
        for (int r = 0; r < D; ++r) x[m][r] = X[v * D + r];
        k[m] = coef[v];
    }
}

// P[k*NM + mn] = cstiff * kappa_k * G[mn]
template <int D>
__device__ __forceinline__ double cell_tensor_inputs(int64_t c, const KArgs &a,
                                                     double (&P)[(D + 1) * Geo<D>::NM],
                                                     double *madet)
{
    double x[D + 1][D], k[D + 1], G[Geo<D>::NM];
    gather_cell<D>(c, a.cell_vertex, a.coords, a.coeff, x, k);
    const double adet = Geo<D>::metric(x, G);
#pragma unroll
    for (int m = 0; m <= D; ++m) {
        const double s = a.cstiff * k[m];
#pragma unroll
        for (int t = 0; t < Geo<D>::NM; ++t) P[m * Geo<D>::NM + t] = s * G[t];
    }
    *madet = a.cmass * adet;
    return adet;
}

template <class T>
__device__ __forceinline__ void mat_group(int g, const double *P, double madet, double *E)
{
    if constexpr (T::NG == 1) {
        T::mat_group0(P, madet, E);
    } else {
        switch (g) {
        case 0: T::mat_group0(P, madet, E); break;
        case 1: T::mat_group1(P, madet, E); break;
        case 2: T::mat_group2(P, madet, E); break;
        default: T::mat_group3(P, madet, E); break;
        }
    }
}

// ---------------------------------------------------------------- configs

// CHUNK: cells evaluated per step; KR: rows owned per lane (rows per block =
// KR*WG); SLOTS: Mat values accumulated in LDS per block.
template <int D, int K> struct MatCfg;
template <> struct MatCfg<2, 1> { static constexpr int CHUNK = 256, KR = 4, SLOTS = 10240 - 256 * 9; };
template <> struct MatCfg<3, 1> { static constexpr int CHUNK = 256, KR = 2, SLOTS = 10240 - 256 * 16; };
template <> struct MatCfg<2, 2> { static constexpr int CHUNK = 64, KR = 3, SLOTS = 10240 - 64 * 36; };
template <> struct MatCfg<3, 2> { static constexpr int CHUNK = 64, KR = 2, SLOTS = LDS_DOUBLES - 64 * 100; };
template <> struct MatCfg<2, 3> { static constexpr int CHUNK = 64, KR = 4, SLOTS = LDS_DOUBLES - 64 * 100; };
template <> struct MatCfg<3, 3> { static constexpr int CHUNK = 16, KR = 2, SLOTS = LDS_DOUBLES - 16 * 400; };

template <int D, int K> struct VecCfg { static constexpr int CHUNK = 256, KR = 8; };

template <int D, int K> struct TabOf;
template <> struct TabOf<2, 1> { using T = femtab::Tab21; };
template <> struct TabOf<2, 2> { using T = femtab::Tab22; };
template <> struct TabOf<2, 3> { using T = femtab::Tab23; };
template <> struct TabOf<3, 1> { using T = femtab::Tab31; };
template <> struct TabOf<3, 2> { using T = femtab::Tab32; };
template <> struct TabOf<3, 3> { using T = femtab::Tab33; };

constexpr int lbits_for(int nloc) { return nloc <= 4 ? 2 : nloc <= 8 ? 3 : nloc <= 16 ? 4 : 5; }

// ---------------------------------------------------------------- Mat

template <int D, int K, typename PosT>
__global__ __launch_bounds__(WG) void k_assemble_mat(KArgs a)
{
    using T = typename TabOf<D, K>::T;
    using C = MatCfg<D, K>;
    constexpr int NL = T::NLOC, NN = NL * NL, LB = lbits_for(NL);
    constexpr int NP = (D + 1) * Geo<D>::NM;
    __shared__ double E[C::CHUNK * NN];
    __shared__ double acc[C::SLOTS];

    const KArgs &p = a;
    const int b = blockIdx.x, tid = threadIdx.x;
    const int r0 = p.blk_row0[b], r1 = p.blk_row0[b + 1];
    const int64_t s0 = a.row_ptr[r0];
    const int nslots = (int)(a.row_ptr[r1] - s0);
    for (int s = tid; s < nslots; s += WG) acc[s] = 0.0;

    int cur[C::KR], end[C::KR], base[C::KR];
#pragma unroll
    for (int k = 0; k < C::KR; ++k) {
        const int r = r0 + tid + WG * k;
        if (r < r1) {
            cur[k] = p.inc_ptr[r]; end[k] = p.inc_ptr[r + 1];
            base[k] = (int)(a.row_ptr[r] - s0);
        } else {
            cur[k] = end[k] = base[k] = 0;
        }
    }
    const int c0 = p.blk_cptr[b], nc = p.blk_cptr[b + 1] - c0;
    const int wave = tid >> 6, lane = tid & 63;
    const int grp = wave % T::NG;
    const int slot = (wave / T::NG) * 64 + lane;
    const PosT *__restrict__ gpos = (const PosT *)p.gpos;
    const int gs = p.gstride;
    __syncthreads();

    for (int cs = 0; cs < nc; cs += C::CHUNK) {
        if (slot < C::CHUNK && cs + slot < nc) {
            const int64_t c = p.bcell[c0 + cs + slot];
            double P[NP], madet;
            cell_tensor_inputs<D>(c, a, P, &madet);
            mat_group<T>(grp, P, madet, E + slot * NN);
        }
        __syncthreads();
        const int cend = cs + C::CHUNK;
#pragma unroll
        for (int k = 0; k < C::KR; ++k) {
            while (cur[k] < end[k]) {
                const unsigned pk = p.ent[cur[k]];
                const int lc = (int)(pk >> LB);
                if (lc >= cend) break;
                const int li = (int)(pk & ((1u << LB) - 1));
                const PosT *__restrict__ gp = gpos + (int64_t)cur[k] * gs;
                const double *__restrict__ er = E + (lc - cs) * NN + li * NL;
                double *__restrict__ ac = acc + base[k];
#pragma unroll
                for (int j = 0; j < NL; ++j) ac[gp[j]] += er[j];
                ++cur[k];
            }
        }
        __syncthreads();
    }
    double *__restrict__ out = a.out + s0;
    if (a.inc) {
        for (int s = tid; s < nslots; s += WG) out[s] += acc[s];
    } else {
        for (int s = tid; s < nslots; s += WG) out[s] = acc[s];
    }
}

// ---------------------------------------------------------------- Dat (source)

template <int D, int K>
__global__ __launch_bounds__(WG) void k_assemble_vec(KArgs a)
{
    using T = typename TabOf<D, K>::T;
    using C = VecCfg<D, K>;
    constexpr int NL = T::NLOC, LB = lbits_for(NL);
    __shared__ double bk[C::CHUNK * NL];
    const KArgs &p = a;
    const int b = blockIdx.x, tid = threadIdx.x;
    const int r0 = p.blk_row0[b], r1 = p.blk_row0[b + 1];
    int cur[C::KR], end[C::KR];
    double acc[C::KR];
#pragma unroll
    for (int k = 0; k < C::KR; ++k) {
        const int r = r0 + tid + WG * k;
        cur[k] = r < r1 ? p.inc_ptr[r] : 0;
        end[k] = r < r1 ? p.inc_ptr[r + 1] : 0;
        acc[k] = 0.0;
    }
    const int c0 = p.blk_cptr[b], nc = p.blk_cptr[b + 1] - c0;
    for (int cs = 0; cs < nc; cs += C::CHUNK) {
        if (cs + tid < nc) {
            const int64_t c = p.bcell[c0 + cs + tid];
            double x[D + 1][D], f[D + 1];
            gather_cell<D>(c, a.cell_vertex, a.coords, a.coeff, x, f);
            T::vec(f, Geo<D>::absdet(x), bk + tid * NL);
        }
        __syncthreads();
        const int cend = cs + C::CHUNK;
#pragma unroll
        for (int k = 0; k < C::KR; ++k) {
            while (cur[k] < end[k]) {
                const unsigned pk = p.ent[cur[k]];
                const int lc = (int)(pk >> LB);
                if (lc >= cend) break;
                acc[k] += bk[(lc - cs) * NL + (int)(pk & ((1u << LB) - 1))];
                ++cur[k];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < C::KR; ++k) {
        const int r = r0 + tid + WG * k;
        if (r < r1) a.out[r] = a.inc ? a.out[r] + acc[k] : acc[k];
    }
}

// ---------------------------------------------------------------- action

template <int D, int K>
__global__ __launch_bounds__(WG) void k_apply_action(KArgs a)
{
    using T = typename TabOf<D, K>::T;
    using C = VecCfg<D, K>;
    constexpr int NL = T::NLOC, LB = lbits_for(NL);
    constexpr int NP = (D + 1) * Geo<D>::NM;
    __shared__ double yk[C::CHUNK * NL];
    const KArgs &p = a;
    const int b = blockIdx.x, tid = threadIdx.x;
    const int r0 = p.blk_row0[b], r1 = p.blk_row0[b + 1];
    int cur[C::KR], end[C::KR];
    double acc[C::KR];
#pragma unroll
    for (int k = 0; k < C::KR; ++k) {
        const int r = r0 + tid + WG * k;
        cur[k] = r < r1 ? p.inc_ptr[r] : 0;
        end[k] = r < r1 ? p.inc_ptr[r + 1] : 0;
        acc[k] = 0.0;
    }
    const int c0 = p.blk_cptr[b], nc = p.blk_cptr[b + 1] - c0;
    for (int cs = 0; cs < nc; cs += C::CHUNK) {
        if (cs + tid < nc) {
            const int64_t c = p.bcell[c0 + cs + tid];
            double P[NP], madet, xl[NL], yl[NL];
            cell_tensor_inputs<D>(c, a, P, &madet);
#pragma unroll
            for (int j = 0; j < NL; ++j) {
                xl[j] = a.x[a.cell_node[c * NL + j]];
                yl[j] = 0.0;
            }
            T::act(P, madet, xl, yl);
#pragma unroll
            for (int j = 0; j < NL; ++j) yk[tid * NL + j] = yl[j];
        }
        __syncthreads();
        const int cend = cs + C::CHUNK;
#pragma unroll
        for (int k = 0; k < C::KR; ++k) {
            while (cur[k] < end[k]) {
                const unsigned pk = p.ent[cur[k]];
                const int lc = (int)(pk >> LB);
                if (lc >= cend) break;
                acc[k] += yk[(lc - cs) * NL + (int)(pk & ((1u << LB) - 1))];
                ++cur[k];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < C::KR; ++k) {
        const int r = r0 + tid + WG * k;
        if (r < r1) a.out[r] = a.inc ? a.out[r] + acc[k] : acc[k];
    }
}

template <int D, int K>
hipError_t mat_dispatch(const AsmArgs &a, hipStream_t s)
{
    if (a.plan->pos_bytes == 1)
        hipLaunchKernelGGL((k_assemble_mat<D, K, uint8_t>), dim3(a.plan->nblk), dim3(WG), 0, s, kargs(a));
    else
        hipLaunchKernelGGL((k_assemble_mat<D, K, uint16_t>), dim3(a.plan->nblk), dim3(WG), 0, s, kargs(a));
    return hipGetLastError();
}

}  // namespace

bool limits(int dim, int degree, bool is_mat, Limits *out)
{
    const int nloc = dim == 2 ? (degree + 1) * (degree + 2) / 2
                              : (degree + 1) * (degree + 2) * (degree + 3) / 6;
    const int lb = lbits_for(nloc);
    out->cell_cap = 1 << (16 - lb);
    out->slot_cap = 0;
#define FEM_LIM(D, K)                                                        \
    if (dim == D && degree == K) {                                           \
        if (is_mat) {                                                        \
            out->rows_per_block = MatCfg<D, K>::KR * WG;                     \
            out->slot_cap = MatCfg<D, K>::SLOTS;                             \
        } else {                                                             \
            out->rows_per_block = VecCfg<D, K>::KR * WG;                     \
        }                                                                    \
        return true;                                                         \
    }
    FEM_LIM(2, 1) FEM_LIM(2, 2) FEM_LIM(2, 3) FEM_LIM(3, 1) FEM_LIM(3, 2) FEM_LIM(3, 3)
#undef FEM_LIM
    return false;
}

#define FEM_DISPATCH(FN, ...)                                                  \
    switch (a.plan->dim * 10 + a.plan->degree) {                               \
    case 21: return FN<2, 1>(__VA_ARGS__);                                     \
    case 22: return FN<2, 2>(__VA_ARGS__);                                     \
    case 23: return FN<2, 3>(__VA_ARGS__);                                     \
    case 31: return FN<3, 1>(__VA_ARGS__);                                     \
    case 32: return FN<3, 2>(__VA_ARGS__);                                     \
    case 33: return FN<3, 3>(__VA_ARGS__);                                     \
    default: return hipErrorInvalidValue;                                      \
    }

namespace {
template <int D, int K>
hipError_t vec_dispatch(const AsmArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL((k_assemble_vec<D, K>), dim3(a.plan->nblk), dim3(WG), 0, s, kargs(a));
    return hipGetLastError();
}
template <int D, int K>
hipError_t action_dispatch(const AsmArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL((k_apply_action<D, K>), dim3(a.plan->nblk), dim3(WG), 0, s, kargs(a));
    return hipGetLastError();
}
}  // namespace

hipError_t launch_mat(const AsmArgs &a, hipStream_t s)
{
    if (a.plan->nblk == 0) return hipSuccess;
    FEM_DISPATCH(mat_dispatch, a, s)
}

hipError_t launch_vec(const AsmArgs &a, hipStream_t s)
{
    if (a.plan->nblk == 0) return hipSuccess;
    FEM_DISPATCH(vec_dispatch, a, s)
}

hipError_t launch_action(const AsmArgs &a, hipStream_t s)
{
    if (a.plan->nblk == 0) return hipSuccess;
    FEM_DISPATCH(action_dispatch, a, s)
}

}  // namespace femk
