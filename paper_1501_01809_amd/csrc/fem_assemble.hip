// Cell-loop assembly kernels for gfx950 (MI355X).
//
// The parallel loop of the paper ("Parloops and kernels") runs the local
// kernel on every cell with data gathered through Maps (READ) and adds the
// element tensor into the output (INC).  Here the INC is made conflict-free
// and deterministic by owning OUTPUT ROWS instead of colouring cells: the plan
// splits the rows into contiguous blocks; one workgroup owns a block and
// visits every cell incident to its rows, in an order fixed by the plan.  Per
// chunk of cells it
//   1. gathers the cells' vertex coordinates and P1 coefficients,
//   2. computes the FP64 geometry (adjugate, |det J|, metric
//      |det J| grad(l_m).grad(l_n)) and the element tensor from the exact
//      reference integrals (generated straight-line FMA code), into LDS,
//   3. adds the chunk's contributions to the block's rows, held in LDS, in a
//      static schedule whose steps touch distinct rows (Mat), or lets each
//      lane sum the contributions to the rows it owns (Dat, action),
// and finally writes its rows once, contiguously (the block's rows occupy one
// contiguous range of the CSR values).  No atomics and no inter-workgroup
// communication are used, so the result is bitwise reproducible; the price is
// that a cell straddling two row blocks is evaluated by both.
#include "fem_internal.h"
#include "fem_tables.h"

#include <algorithm>

namespace femk {
namespace {


// Everything a kernel reads, by value: device pointers and scalars only.
struct KArgs {
    const int32_t *__restrict__ blk_row0;
    const int32_t *__restrict__ blk_cptr;
    const int32_t *__restrict__ bcell;
    const int32_t *__restrict__ bverts;
    const int32_t *__restrict__ inc_ptr;
    const uint16_t *__restrict__ ent;
    const int32_t *__restrict__ blk_q;
    const int32_t *__restrict__ q_ent;
    const int32_t *__restrict__ q_nrank;
    const uint32_t *__restrict__ sched;
    const int64_t *__restrict__ row_ptr;
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
    k.blk_row0 = p.blk_row0; k.blk_cptr = p.blk_cptr; k.bcell = p.bcell; k.bverts = p.bverts;
    k.inc_ptr = p.inc_ptr; k.ent = p.ent;
    k.blk_q = p.blk_q; k.q_ent = p.q_ent; k.q_nrank = p.q_nrank; k.sched = p.sched;
    k.row_ptr = a.row_ptr; k.coords = a.coords;
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

// ---------------------------------------------------------------- configs

// Mat kernels: workgroups of MWG lanes, one row per lane; CHUNK cells are
// evaluated per step (NG waves share a cell, one entry group each) and their
// packed upper-triangle element tensors (E doubles each) live in LDS next to
// the block's Mat values.
constexpr int MWG = 512;
template <int D, int K> struct MatCfg;
template <> struct MatCfg<2, 1> { static constexpr int CHUNK = 512, CB = 9, E = 6; };
template <> struct MatCfg<3, 1> { static constexpr int CHUNK = 512, CB = 9, E = 10; };
template <> struct MatCfg<2, 2> { static constexpr int CHUNK = 128, CB = 7, E = 21; };
template <> struct MatCfg<3, 2> { static constexpr int CHUNK = 128, CB = 7, E = 55; };
template <> struct MatCfg<2, 3> { static constexpr int CHUNK = 128, CB = 7, E = 55; };
template <> struct MatCfg<3, 3> { static constexpr int CHUNK = 32, CB = 5, E = 210; };
template <int D, int K> constexpr int mat_slots()
{
    return LDS_DOUBLES - MatCfg<D, K>::CHUNK * MatCfg<D, K>::E;
}

// Dat and action kernels: workgroups of VWG lanes, KR rows per lane; the
// per-cell local vectors of the whole block live in LDS (VLDS doubles, two
// workgroups per CU).
constexpr int VWG = 512;
constexpr int VKR = 2;
constexpr int VLDS = LDS_DOUBLES / 2;
constexpr int VPRE = 8;     // entries of a row fetched per batch

template <int D, int K> struct TabOf;
template <> struct TabOf<2, 1> { using T = femtab::Tab21; };
template <> struct TabOf<2, 2> { using T = femtab::Tab22; };
template <> struct TabOf<2, 3> { using T = femtab::Tab23; };
template <> struct TabOf<3, 1> { using T = femtab::Tab31; };
template <> struct TabOf<3, 2> { using T = femtab::Tab32; };
template <> struct TabOf<3, 3> { using T = femtab::Tab33; };

constexpr int lbits_for(int nloc) { return nloc <= 4 ? 2 : nloc <= 8 ? 3 : nloc <= 16 ? 4 : 5; }

template <class T>
__device__ __forceinline__ void mat_group_n(int g, const double *P, double madet, double *E)
{
    if constexpr (T::NG == 1) {
        T::mat_group0(P, madet, E);
    } else if constexpr (T::NG == 4) {
        switch (g) {
        case 0: T::mat_group0(P, madet, E); break;
        case 1: T::mat_group1(P, madet, E); break;
        case 2: T::mat_group2(P, madet, E); break;
        default: T::mat_group3(P, madet, E); break;
        }
    } else {
        switch (g) {
        case 0: T::mat_group0(P, madet, E); break;
        case 1: T::mat_group1(P, madet, E); break;
        case 2: T::mat_group2(P, madet, E); break;
        case 3: T::mat_group3(P, madet, E); break;
        case 4: T::mat_group4(P, madet, E); break;
        case 5: T::mat_group5(P, madet, E); break;
        case 6: T::mat_group6(P, madet, E); break;
        default: T::mat_group7(P, madet, E); break;
        }
    }
}

// Vertex coordinates and P1 coefficient of one cell, gathered through the
// plan's per-visit vertex ids.
template <int D> struct CellIn {
    double x[D + 1][D];
    double k[D + 1];
};

template <int D>
__device__ __forceinline__ void load_cell(const int32_t *__restrict__ bverts, int64_t visit,
                                          const double *__restrict__ X, const double *__restrict__ coef,
                                          CellIn<D> &c)
{
    int32_t v[D + 1];
#pragma unroll
    for (int m = 0; m <= D; ++m) v[m] = bverts[visit * (D + 1) + m];
#pragma unroll
    for (int m = 0; m <= D; ++m) {
#pragma unroll
        for (int r = 0; r < D; ++r) c.x[m][r] = X[(int64_t)v[m] * D + r];
        c.k[m] = coef[v[m]];
    }
}

template <int D>
__device__ __forceinline__ void tensor_inputs(const CellIn<D> &c, double cstiff, double cmass,
                                              double (&P)[(D + 1) * Geo<D>::NM], double *madet)
{
    double G[Geo<D>::NM];
    const double adet = Geo<D>::metric(c.x, G);
#pragma unroll
    for (int m = 0; m <= D; ++m) {
        const double s = cstiff * c.k[m];
#pragma unroll
        for (int t = 0; t < Geo<D>::NM; ++t) P[m * Geo<D>::NM + t] = s * G[t];
    }
    *madet = cmass * adet;
}

// ---------------------------------------------------------------- Mat

template <int D, int K, typename PosT>
__global__ __launch_bounds__(MWG) void k_assemble_mat(KArgs a)
{
    using T = typename TabOf<D, K>::T;
    using Cf = MatCfg<D, K>;
    constexpr int NL = T::NLOC, NE = T::NE, LB = lbits_for(NL), CB = Cf::CB;
    constexpr int NP = (D + 1) * Geo<D>::NM;
    constexpr int SLOTS = mat_slots<D, K>();
    constexpr int PER = 4 / (int)sizeof(PosT);              // positions per word
    constexpr int W = 1 + (NL + PER - 1) / PER;              // words per record
    constexpr int MM = (Cf::CHUNK * NL + MWG - 1) / MWG;     // records per lane and chunk
    static_assert(NE == Cf::E && (1 << CB) == Cf::CHUNK, "config");
    static_assert(SLOTS < 32768, "slot offsets are 15-bit");
    __shared__ double E[Cf::CHUNK * NE];
    __shared__ double acc[SLOTS];

    const int b = blockIdx.x, tid = threadIdx.x;
    const int r0 = a.blk_row0[b], r1 = a.blk_row0[b + 1];
    const int64_t s0 = a.row_ptr[r0];
    const int nslots = (int)(a.row_ptr[r1] - s0);
    for (int s = tid; s < nslots; s += MWG) acc[s] = 0.0;

    const int q0 = a.blk_q[b], nq = a.blk_q[b + 1] - q0;
    const int c0 = a.blk_cptr[b], nc = a.blk_cptr[b + 1] - c0;
    const int wave = tid >> 6, lane = tid & 63;
    const int grp = wave % T::NG;
    const int slot = (wave / T::NG) * 64 + lane;
    const bool computes = slot < Cf::CHUNK;

    // records of the next chunk, fetched one chunk ahead
    uint32_t rw[MM][W];
    bool rv[MM];
    auto fetch_records = [&](int q) {
        const int e0 = a.q_ent[q], e1 = a.q_ent[q + 1];
#pragma unroll
        for (int m = 0; m < MM; ++m) {
            const int e = e0 + tid + m * MWG;
            rv[m] = e < e1;
            if (rv[m]) {
#pragma unroll
                for (int w = 0; w < W; ++w) rw[m][w] = a.sched[(int64_t)e * W + w];
            }
        }
    };
    CellIn<D> cin;
    if (computes && slot < nc) load_cell<D>(a.bverts, c0 + slot, a.coords, a.coeff, cin);
    if (nq > 0) fetch_records(q0);
    __syncthreads();

    for (int qi = 0; qi < nq; ++qi) {
        const int cs = qi * Cf::CHUNK;
        if (computes && cs + slot < nc) {
            double P[NP], madet;
            tensor_inputs<D>(cin, a.cstiff, a.cmass, P, &madet);
            mat_group_n<T>(grp, P, madet, E + slot * NE);
        }
        uint32_t cw[MM][W];
        bool cv[MM];
#pragma unroll
        for (int m = 0; m < MM; ++m) {
            cv[m] = rv[m];
#pragma unroll
            for (int w = 0; w < W; ++w) cw[m][w] = rw[m][w];
        }
        const int nrank = a.q_nrank[q0 + qi];
        if (qi + 1 < nq) {
            fetch_records(q0 + qi + 1);
            if (computes && cs + Cf::CHUNK + slot < nc)
                load_cell<D>(a.bverts, c0 + cs + Cf::CHUNK + slot, a.coords, a.coeff, cin);
        }
        __syncthreads();
        for (int rk = 0; rk < nrank; ++rk) {
#pragma unroll
            for (int m = 0; m < MM; ++m) {
                const uint32_t h = cw[m][0];
                if (!cv[m] || (int)(h >> (15 + CB + LB)) != rk) continue;
                const int base = (int)(h & 0x7fffu);
                const int lcc = (int)((h >> 15) & ((1u << CB) - 1));
                const int li = (int)((h >> (15 + CB)) & ((1u << LB) - 1));
                const double *__restrict__ Ec = E + lcc * NE;
                const int ul = li * (2 * NL - li - 1) / 2;
                int pos[NL];
#pragma unroll
                for (int j = 0; j < NL; ++j)
                    pos[j] = base + (int)((cw[m][1 + j / PER] >> (8 * sizeof(PosT) * (j % PER))) &
                                          ((1u << (8 * sizeof(PosT))) - 1));
                double t[NL];
#pragma unroll
                for (int j = 0; j < NL; ++j) t[j] = acc[pos[j]];
#pragma unroll
                for (int j = 0; j < NL; ++j) {
                    const int uj = j * (2 * NL - j - 1) / 2;
                    t[j] += Ec[j >= li ? ul + j : uj + li];
                }
#pragma unroll
                for (int j = 0; j < NL; ++j) acc[pos[j]] = t[j];
            }
            __syncthreads();
        }
    }
    double *__restrict__ out = a.out + s0;
    if (a.inc) {
        for (int s = tid; s < nslots; s += MWG) out[s] += acc[s];
    } else {
        for (int s = tid; s < nslots; s += MWG) out[s] = acc[s];
    }
}

// ---------------------------------------------------------------- Dat / action

template <int D, int K, bool ACTION>
__global__ __launch_bounds__(VWG) void k_assemble_vec(KArgs a)
{
    using T = typename TabOf<D, K>::T;
    constexpr int NL = T::NLOC, LB = lbits_for(NL);
    constexpr int NP = (D + 1) * Geo<D>::NM;
    constexpr int CAP = VLDS / NL;
    __shared__ double vk[CAP * NL];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int r0 = a.blk_row0[b], r1 = a.blk_row0[b + 1];
    int cur[VKR], end[VKR];
    uint32_t pe[VKR][VPRE];
    double acc[VKR];
#pragma unroll
    for (int k = 0; k < VKR; ++k) {
        const int r = r0 + tid + VWG * k;
        cur[k] = r < r1 ? a.inc_ptr[r] : 0;
        end[k] = r < r1 ? a.inc_ptr[r + 1] : 0;
        acc[k] = 0.0;
#pragma unroll
        for (int m = 0; m < VPRE; ++m) pe[k][m] = cur[k] + m < end[k] ? a.ent[cur[k] + m] : 0u;
    }
    const int c0 = a.blk_cptr[b], nc = a.blk_cptr[b + 1] - c0;
    CellIn<D> cin;
    double xl[ACTION ? NL : 1];
    auto fetch = [&](int c) {
        load_cell<D>(a.bverts, c0 + c, a.coords, a.coeff, cin);
        if constexpr (ACTION) {
            const int64_t cell = a.bcell[c0 + c];
#pragma unroll
            for (int j = 0; j < NL; ++j) xl[j] = a.x[a.cell_node[cell * NL + j]];
        }
    };
    if (tid < nc) fetch(tid);
    for (int cs = 0; cs < nc; cs += VWG) {
        if (cs + tid < nc) {
            double loc[NL];
            if constexpr (ACTION) {
                double P[NP], madet;
                tensor_inputs<D>(cin, a.cstiff, a.cmass, P, &madet);
#pragma unroll
                for (int j = 0; j < NL; ++j) loc[j] = 0.0;
                T::act(P, madet, xl, loc);
            } else {
                T::vec(cin.k, Geo<D>::absdet(cin.x), loc);
            }
#pragma unroll
            for (int j = 0; j < NL; ++j) vk[(cs + tid) * NL + j] = loc[j];
        }
        if (cs + VWG + tid < nc) fetch(cs + VWG + tid);
    }
    __syncthreads();
    // every row sums its cells' local values in ascending cell order
#pragma unroll
    for (int k = 0; k < VKR; ++k) {
        while (cur[k] < end[k]) {
#pragma unroll
            for (int m = 0; m < VPRE; ++m)
                if (cur[k] + m < end[k])
                    acc[k] += vk[(int)(pe[k][m] >> LB) * NL + (int)(pe[k][m] & ((1u << LB) - 1))];
            cur[k] += VPRE;
#pragma unroll
            for (int m = 0; m < VPRE; ++m) pe[k][m] = cur[k] + m < end[k] ? a.ent[cur[k] + m] : 0u;
        }
    }
#pragma unroll
    for (int k = 0; k < VKR; ++k) {
        const int r = r0 + tid + VWG * k;
        if (r < r1) a.out[r] = a.inc ? a.out[r] + acc[k] : acc[k];
    }
}

template <int D, int K>
hipError_t mat_dispatch(const AsmArgs &a, hipStream_t s)
{
    if (a.plan->pos_bytes == 1)
        hipLaunchKernelGGL((k_assemble_mat<D, K, uint8_t>), dim3(a.plan->nblk), dim3(MWG), 0, s, kargs(a));
    else
        hipLaunchKernelGGL((k_assemble_mat<D, K, uint16_t>), dim3(a.plan->nblk), dim3(MWG), 0, s, kargs(a));
    return hipGetLastError();
}

}  // namespace

bool limits(int dim, int degree, bool is_mat, Limits *out)
{
    const int nloc = dim == 2 ? (degree + 1) * (degree + 2) / 2
                              : (degree + 1) * (degree + 2) * (degree + 3) / 6;
    const int lb = lbits_for(nloc);
    out->slot_cap = 0;
    out->chunk = out->chunk_bits = out->rank_bits = 0;
#define FEM_LIM(D, K)                                                             \
    if (dim == D && degree == K) {                                                \
        if (is_mat) {                                                             \
            out->rows_per_block = MWG;                                            \
            out->slot_cap = mat_slots<D, K>();                                    \
            out->chunk = MatCfg<D, K>::CHUNK;                                     \
            out->chunk_bits = MatCfg<D, K>::CB;                                   \
            out->rank_bits = 32 - 15 - MatCfg<D, K>::CB - lb;                     \
            out->cell_cap = 1 << 20;                                              \
        } else {                                                                  \
            out->rows_per_block = VKR * VWG;                                      \
            out->cell_cap = std::min(1 << (16 - lb), VLDS / nloc);                \
        }                                                                         \
        return true;                                                              \
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
    hipLaunchKernelGGL((k_assemble_vec<D, K, false>), dim3(a.plan->nblk), dim3(VWG), 0, s, kargs(a));
    return hipGetLastError();
}
template <int D, int K>
hipError_t action_dispatch(const AsmArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL((k_assemble_vec<D, K, true>), dim3(a.plan->nblk), dim3(VWG), 0, s, kargs(a));
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
