// Vector Lagrange linear elasticity on tetrahedra for gfx950: element blocks
// by batched MFMA contractions, then a deterministic pull into the CSR.
//
// The form is 2 mu eps(u):eps(v) + lam div(u) div(v) on the P2 vector space
// (DOF 3*node + component), mu and lam P1 fields, with the coordinate field
// read through its own Map (a per-cell, discontinuous coordinate field lets
// single cells be badly shaped; the paper treats coordinates as an ordinary
// field, "The mesh abstraction").
//
// Stage 1, k_elast_element: every element matrix is the contraction
//   A[(i,a),(j,b)] = sum_q G[ab][q] T[q][ij],  q = (k, r, s), 36 terms,
// of a per-cell geometry/coefficient factor G (9 x 36, formed in FP64 from
// the FP64 inverse Jacobian) with the reference tensor T (36 x 55 upper node
// pairs, fem_elast_tables.h).  Stacked over cells this is one tall GEMM
//   D[pair][(cell, ab)] = sum_q T^T[pair][q] G^T[q][(cell, ab)],
// run on 16x16 MFMA tiles: 4 tiles of pairs (55 padded to 64) by 9 tiles of
// (cell, ab) columns for every 16 cells, K = 36 (FP64/FP32: 9 steps of 4;
// BF16/FP16: 3 steps of 16, K padded to 48).  For the narrow types G is
// scaled per cell by a power of two (exact) that brings its entries to
// magnitude <= 1, and the FP32 accumulator is scaled back (FP16 stores it as
// it is, with the scale's exponent); accumulation is in FP32 (FP64 for the
// FP64 path).  The blocks (i <= j, 3 x 3 each) go to a
// plan-owned workspace E[cell][pair][a*3+b] (FP64; FP32 for the FP32
// contraction; 16-bit values, ten per block, for BF16 and FP16).
//
// Stage 2, k_elast_pull: one lane per node pair (i, j) of the node sparsity,
// a 3 x 3 block of the vector CSR.  The lane walks the plan's list of
// contributions to its block, in ascending cell id, reads each cell's block
// (transposed when the lane's row node is the cell's later local node;
// symmetrised on the diagonal), sums in FP64 and writes its nine values once.
// No atomics; the order is fixed by the plan, so results are bitwise
// reproducible and the assembled matrix is bitwise symmetric.
#include "fem_internal.h"
#include "fem_elast_tables.h"

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

namespace femk {
namespace {

constexpr int NL = femelast::NLOC;        // 10 local nodes
constexpr int NP = femelast::NPAIR;       // 55 upper node pairs
constexpr int NQ = femelast::NQ;          // 36 contraction terms
constexpr int EWG = 256;                  // element kernel: 4 waves
constexpr int CPW = 16;                   // cells per wave and group

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));
typedef _Float16 v4h __attribute__((ext_vector_type(4)));

// bfloat16 bits of a float, rounded to nearest even on the hardware
// converter; x is kept opaque so that a double -> float rounding before the
// call is not folded into one double -> bfloat16 conversion (which has no
// instruction and is expanded into a correction sequence)
__device__ __forceinline__ short f2bf(float x)
{
    asm volatile("" : "+v"(x));
    return (short)__builtin_bit_cast(uint16_t, (__bf16)x);
}

// Per precision: MFMA operand type, K steps and K per lane, accumulator and
// workspace types, and the row of accumulator element v held by lane l.
template <int P> struct Mf;
template <> struct Mf<FEM_FP64> {
    typedef double In; typedef v4d Acc; typedef double Out;
    static constexpr int KS = 9, KP = 1;
    static __device__ __forceinline__ int row(int l, int v) { return (l >> 4) + 4 * v; }
    static __device__ __forceinline__ Acc mma(In a, In b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};
template <> struct Mf<FEM_FP32> {
    typedef float In; typedef v4f Acc; typedef float Out;
    static constexpr int KS = 9, KP = 1;
    static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
    static __device__ __forceinline__ Acc mma(In a, In b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
template <> struct Mf<FEM_BF16> {
    typedef v4s In; typedef v4f Acc; typedef float Out;
    static constexpr int KS = 3, KP = 4;
    static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
    static __device__ __forceinline__ Acc mma(In a, In b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }
};
template <> struct Mf<FEM_FP16> {
    typedef v4h In; typedef v4f Acc; typedef float Out;
    static constexpr int KS = 3, KP = 4;
    static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
    static __device__ __forceinline__ Acc mma(In a, In b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0); }
};

// Workspace element: FP64 and FP32 blocks of nine values (FP64 for the FP64
// contraction, FP32 for FP32).  The narrow contractions store 16-bit values,
// nine and one more per block (20-byte, 4-byte aligned blocks: the pull
// reads one with a 16-byte and a 4-byte load instead of three), which halves
// the workspace: BF16 the scaled-back values as bfloat16 bits (the tenth
// unused); FP16 the accumulator before it is scaled back, which the operand
// scaling keeps within FP16 range, as binary16 bits, the tenth holding the
// cell's scale exponent (the scale is a power of two, so the pull restores
// the value exactly).
typedef uint32_t u32x4a __attribute__((ext_vector_type(4), aligned(4)));
struct half_ws { uint16_t bits; };   // FP16 workspace element
template <typename W> struct Ws;
template <> struct Ws<double> { static constexpr int BS = 9; };
template <> struct Ws<float> { static constexpr int BS = 9; };
template <> struct Ws<uint16_t> { static constexpr int BS = 10; };
template <> struct Ws<half_ws> { static constexpr int BS = 10; };
template <int P> struct WsOf { typedef float T; };
template <> struct WsOf<FEM_FP64> { typedef double T; };
template <> struct WsOf<FEM_BF16> { typedef uint16_t T; };
template <> struct WsOf<FEM_FP16> { typedef half_ws T; };
// Stores entry ab of a block (E the block's first element); acc is the
// contraction's accumulator and scale the cell's power-of-two operand scale.
__device__ __forceinline__ void ws_put(double *E, int ab, double acc, double scale) { E[ab] = acc * scale; }
__device__ __forceinline__ void ws_put(float *E, int ab, float acc, double scale) { E[ab] = acc * (float)scale; }
__device__ __forceinline__ void ws_put(uint16_t *E, int ab, float acc, double scale)
{
    E[ab] = (uint16_t)f2bf(acc * (float)scale);
}
__device__ __forceinline__ void ws_put(half_ws *E, int ab, float acc, double)
{
    E[ab].bits = __builtin_bit_cast(uint16_t, (_Float16)acc);   // (the exponent: after the tiles)
}
__device__ __forceinline__ double bf2d(uint32_t bits16) { return (double)__uint_as_float(bits16 << 16); }
__device__ __forceinline__ double h2d(uint32_t bits16) { return (double)(float)__builtin_bit_cast(_Float16, (uint16_t)bits16); }
// One block as loaded (raw, so that a block loaded ahead is not waited for
// until it is used), and its nine values as doubles.
template <typename W> struct Blk {
    W v[9];
    __device__ __forceinline__ void load(const W *b)
    {
#pragma unroll
        for (int q = 0; q < 9; ++q) v[q] = b[q];
    }
    __device__ __forceinline__ void get(double (&d)[9]) const
    {
#pragma unroll
        for (int q = 0; q < 9; ++q) d[q] = (double)v[q];
    }
};
template <> struct Blk<uint16_t> {
    u32x4a w;
    uint32_t w4;
    __device__ __forceinline__ void load(const uint16_t *b)
    {
        w = *reinterpret_cast<const u32x4a *>(b);
        w4 = *reinterpret_cast<const uint32_t *>(b + 8);
    }
    __device__ __forceinline__ void get(double (&d)[9]) const
    {
        d[0] = bf2d(w.x & 0xffffu); d[1] = bf2d(w.x >> 16);
        d[2] = bf2d(w.y & 0xffffu); d[3] = bf2d(w.y >> 16);
        d[4] = bf2d(w.z & 0xffffu); d[5] = bf2d(w.z >> 16);
        d[6] = bf2d(w.w & 0xffffu); d[7] = bf2d(w.w >> 16);
        d[8] = bf2d(w4 & 0xffffu);
    }
};

template <> struct Blk<half_ws> {
    u32x4a w;
    uint32_t w4;
    __device__ __forceinline__ void load(const half_ws *b)
    {
        w = *reinterpret_cast<const u32x4a *>(b);
        w4 = *reinterpret_cast<const uint32_t *>(b + 8);
    }
    __device__ __forceinline__ void get(double (&d)[9]) const
    {
        // 2^e, e the cell's scale exponent (the block's tenth element)
        const double sc = ldexp(1.0, (int)(int16_t)(w4 >> 16));
        d[0] = h2d(w.x & 0xffffu) * sc; d[1] = h2d(w.x >> 16) * sc;
        d[2] = h2d(w.y & 0xffffu) * sc; d[3] = h2d(w.y >> 16) * sc;
        d[4] = h2d(w.z & 0xffffu) * sc; d[5] = h2d(w.z >> 16) * sc;
        d[6] = h2d(w.w & 0xffffu) * sc; d[7] = h2d(w.w >> 16) * sc;
        d[8] = h2d(w4 & 0xffffu) * sc;
    }
};

// Pack KP values of one lane's K slice into the MFMA operand type.
template <int P> __device__ __forceinline__ typename Mf<P>::In pack(const double *g);
template <> __device__ __forceinline__ double pack<FEM_FP64>(const double *g) { return g[0]; }
template <> __device__ __forceinline__ float pack<FEM_FP32>(const double *g) { return (float)g[0]; }
template <> __device__ __forceinline__ v4s pack<FEM_BF16>(const double *g)
{
    v4s r;
    r[0] = f2bf((float)g[0]); r[1] = f2bf((float)g[1]); r[2] = f2bf((float)g[2]); r[3] = f2bf((float)g[3]);
    return r;
}
// double -> float -> binary16, both roundings to nearest even on the
// hardware converters (left to itself the compiler folds the two into one
// double -> half conversion, which it expands into a long integer sequence)
__device__ __forceinline__ _Float16 d2h(double g)
{
    float f = (float)g;
    asm volatile("" : "+v"(f));
    return (_Float16)f;
}
template <> __device__ __forceinline__ v4h pack<FEM_FP16>(const double *g)
{
    v4h r;
    r[0] = d2h(g[0]); r[1] = d2h(g[1]); r[2] = d2h(g[2]); r[3] = d2h(g[3]);
    return r;
}

struct ElArgs {
    const int32_t *__restrict__ cell_vertex;   // [C][4] -> mu, lam
    const int32_t *__restrict__ cell_coord;    // [C][4] -> coordinate nodes
    const double *__restrict__ coords;         // [coordinate nodes][3]
    const double *__restrict__ mu;
    const double *__restrict__ lam;
    void *__restrict__ work;                   // [C][NP][9] of Mf<P>::Out
    int64_t ncells;
};

// Per-cell data staged in LDS by the wave that contracts the cell: Ji[9]
// (J^-1, Ji[r][p] = d xi_r / d x_p), |det J|, mu[4], lam[4], the scale, then
// M[r][s] = sum_p Ji[r][p] Ji[s][p] (9) and P[r][s][x][y] = Ji[r][x] Ji[s][y]
// (81), so that every entry of G is a few LDS reads and three FMAs:
//   G[xy][(k,r,s)] = |det J| (mu_k (delta_xy M[r][s] + P[r][s][y][x]) + lam_k P[r][s][x][y]).
constexpr int G_JI = 0, G_ADET = 9, G_MU = 10, G_LAM = 14, G_SCALE = 18, G_M = 19, G_P = 28, GEO = 109;

template <int P>
__global__ __launch_bounds__(EWG) void k_elast_element(ElArgs a)
{
    using M = Mf<P>;
    __shared__ double geo[EWG / 64][CPW][GEO];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // A operand: T^T[pair][q] for the 4 pair tiles and KS steps, resident.
    typename M::In afr[4][M::KS];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int ks = 0; ks < M::KS; ++ks) {
            double t[M::KP];
            const int pr = 16 * mt + (lane & 15);
#pragma unroll
            for (int u = 0; u < M::KP; ++u) {
                const int q = ks * 4 * M::KP + (lane >> 4) * M::KP + u;
                t[u] = (pr < NP && q < NQ) ? femelast::T[pr][q] : 0.0;
            }
            afr[mt][ks] = pack<P>(t);
        }
    typedef typename WsOf<P>::T W;
    constexpr int BS = Ws<W>::BS;
    W *E = reinterpret_cast<W *>(a.work);
    const int64_t ngroups = (a.ncells + CPW - 1) / CPW;
    // every wave of a workgroup runs the same number of iterations (barriers)
    for (int64_t g0 = (int64_t)blockIdx.x * (EWG / 64); g0 < ngroups; g0 += (int64_t)gridDim.x * (EWG / 64)) {
        const int64_t g = g0 + wv;
        // 1. geometry of the group's 16 cells, one lane each, FP64
        if (lane < CPW) {
            const int64_t c = g * CPW + lane;
            double *G = geo[wv][lane];
            if (g < ngroups && c < a.ncells) {
                double x[4][3];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int64_t v = a.cell_coord[c * 4 + m];
#pragma unroll
                    for (int r = 0; r < 3; ++r) x[m][r] = a.coords[v * 3 + r];
                }
                double J[3][3];   // J[p][r] = x_{r+1}[p] - x_0[p]
#pragma unroll
                for (int p = 0; p < 3; ++p)
#pragma unroll
                    for (int r = 0; r < 3; ++r) J[p][r] = x[r + 1][p] - x[0][p];
                // J^-1 = adj(J) / det: Ji[r][p] = cofactor(p, r) / det
                const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
                const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
                const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
                const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
                const double id = 1.0 / det;
                double ji[9];
                ji[0] = c00 * id; ji[3] = c01 * id; ji[6] = c02 * id;
                ji[1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
                ji[4] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
                ji[7] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
                ji[2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
                ji[5] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
                ji[8] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
                double jm = 0.0;
#pragma unroll
                for (int u = 0; u < 9; ++u) { G[G_JI + u] = ji[u]; jm = fmax(jm, fabs(ji[u])); }
                const double adet = fabs(det);
                G[G_ADET] = adet;
                double cm = 0.0;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int64_t v = a.cell_vertex[c * 4 + m];
                    const double mu = a.mu[v], la = a.lam[v];
                    G[G_MU + m] = mu;
                    G[G_LAM + m] = la;
                    cm = fmax(cm, 4.0 * fabs(mu) + fabs(la));
                }
                // |G| <= |det J| max|Ji|^2 (4 max mu + max lam): the power of
                // two just above that bound keeps the narrow operands in range
                const double bound = adet * jm * jm * cm;
                G[G_SCALE] = (P == FEM_FP64 || !(bound > 0.0)) ? 1.0 : ldexp(1.0, ilogb(bound) + 1);
            } else {
                for (int u = 0; u < G_M; ++u) G[u] = 0.0;
                G[G_SCALE] = 1.0;
            }
        }
        __syncthreads();
        // 1b. products of the inverse Jacobian, all lanes
        for (int idx = lane; idx < CPW * 90; idx += 64) {
            const int cq = idx / 90, w = idx - 90 * cq;
            double *G = geo[wv][cq];
            if (w < 9) {
                const int r = w / 3, s2 = w % 3;
                G[G_M + w] = G[r * 3] * G[s2 * 3] + G[r * 3 + 1] * G[s2 * 3 + 1] + G[r * 3 + 2] * G[s2 * 3 + 2];
            } else {
                const int v = w - 9, r = v / 27, s2 = (v / 9) % 3, xx = (v / 3) % 3, yy = v % 3;
                G[G_P + v] = G[r * 3 + xx] * G[s2 * 3 + yy];
            }
        }
        __syncthreads();
        // 2. nine column tiles of 16 (cell, xy) columns
#pragma unroll 1
        for (int t = 0; t < 9; ++t) {
            const int col = 16 * t + (lane & 15);
            const int cq = col / 9, ab = col - 9 * cq, ea = ab / 3, eb = ab - 3 * ea;
            const double *G = geo[wv][cq];
            const double adet = G[G_ADET], scale = G[G_SCALE], inv = 1.0 / scale;
            typename M::In bfr[M::KS];
#pragma unroll
            for (int ks = 0; ks < M::KS; ++ks) {
                double gv[M::KP];
#pragma unroll
                for (int u = 0; u < M::KP; ++u) {
                    const int q = ks * 4 * M::KP + (lane >> 4) * M::KP + u;
                    double val = 0.0;
                    if (q < NQ) {
                        const int kk = q / 9, rs = q % 9;
                        const double pd = G[G_P + rs * 9 + ea * 3 + eb];
                        const double pc = G[G_P + rs * 9 + eb * 3 + ea];
                        const double mrs = ea == eb ? G[G_M + rs] : 0.0;
                        val = adet * (G[G_MU + kk] * (mrs + pc) + G[G_LAM + kk] * pd) * inv;
                    }
                    gv[u] = val;
                }
                bfr[ks] = pack<P>(gv);
            }
            const int64_t cell = g * CPW + cq;
            const bool live = g < ngroups && cell < a.ncells;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                typename M::Acc acc = {0, 0, 0, 0};
#pragma unroll
                for (int ks = 0; ks < M::KS; ++ks) acc = M::mma(afr[mt][ks], bfr[ks], acc);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int pr = 16 * mt + M::row(lane, v);
                    if (live && pr < NP)
                        ws_put(E + cell * (NP * BS) + pr * BS, ab, acc[v], scale);
                }
            }
        }
        if constexpr (P == FEM_FP16) {
            // the tenth element of every block: the cell's scale exponent
            for (int i = lane; i < CPW * NP; i += 64) {
                const int cq = i / NP, pr = i - cq * NP;
                const int64_t cell = g * CPW + cq;
                if (g < ngroups && cell < a.ncells)
                    reinterpret_cast<half_ws *>(E)[cell * (NP * BS) + pr * BS + 9].bits =
                        (uint16_t)(int16_t)ilogb(geo[wv][cq][G_SCALE]);
            }
        }
        __syncthreads();
    }
}

// Stage 2: entry bits (cell << 8) | (pair << 2) | (diagonal << 1) | transposed.
template <typename T>
__global__ __launch_bounds__(256) void k_elast_pull(const int64_t *__restrict__ rp3, const int32_t *__restrict__ slot_ptr,
                                                    const uint32_t *__restrict__ ent, const int32_t *__restrict__ grow,
                                                    const T *__restrict__ E, double *__restrict__ out, int64_t nslots,
                                                    int inc)
{
    // XCD-grouped ranks: the 8 XCDs (blocks dealt round-robin) each take a
    // contiguous range of slots, so the cells shared by neighbouring rows are
    // read through one L2
    const int64_t per = gridDim.x / 8;
    const int64_t rank = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    const int64_t e = rank * 256 + threadIdx.x;
    if (e >= nslots) return;
    int64_t n = grow[e >> 6];
    while (rp3[3 * (n + 1)] / 9 <= e) ++n;
    const int64_t base = rp3[3 * n];
    const int64_t k = e - base / 9;
    double acc[9];
#pragma unroll
    for (int u = 0; u < 9; ++u) acc[u] = 0.0;
    const int t0 = slot_ptr[e], t1 = slot_ptr[e + 1];
    // software pipeline over the contributions: the entry word two ahead and
    // the 3x3 block one ahead are in flight while a block is added.  The
    // look-ahead indices are clamped to the slot's last contribution, so the
    // loads need no branch (a branch around them makes the compiler wait for
    // every load in flight before the adds).
    if (t0 < t1) {
        constexpr int BS = Ws<T>::BS;
        auto block_of = [&](uint32_t w) { return E + (size_t)(w >> 8) * (NP * BS) + ((w >> 2) & 63) * BS; };
        const int tl = t1 - 1;
        uint32_t w0 = ent[t0];
        uint32_t w1 = ent[min(t0 + 1, tl)];
        Blk<T> v;
        v.load(block_of(w0));
        for (int t = t0; t < t1; ++t) {
            const uint32_t w2 = ent[min(t + 2, tl)];
            Blk<T> vn;
            vn.load(block_of(w1));
            double d[9];
            v.get(d);
#pragma unroll
            for (int q = 0; q < 9; ++q) asm volatile("" : "+v"(d[q]));   // nine values, not an array indexed at run time
            // entry (x, y) is d[x][y], or d[y][x] when transposed; on the
            // diagonal the upper triangle serves both halves (bitwise
            // symmetric sums): below the diagonal the mirror is taken when
            // diagonal or transposed, above it when transposed only
            const bool dg = (w0 >> 1) & 1, tr = w0 & 1;
            const bool lo = dg || tr, up = tr && !dg;
            acc[0] += d[0];
            acc[4] += d[4];
            acc[8] += d[8];
            acc[3] += lo ? d[1] : d[3];
            acc[1] += up ? d[3] : d[1];
            acc[6] += lo ? d[2] : d[6];
            acc[2] += up ? d[6] : d[2];
            acc[7] += lo ? d[5] : d[7];
            acc[5] += up ? d[7] : d[5];
            w0 = w1;
            w1 = w2;
            v = vn;
        }
    }
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        const int64_t o = rp3[3 * n + x] + 3 * k;
#pragma unroll
        for (int y = 0; y < 3; ++y) out[o + y] = inc ? out[o + y] + acc[x * 3 + y] : acc[x * 3 + y];
    }
}

// Expansion of a node CSR to the vector CSR of block size bs (node-major).
__global__ void k_expand_rows(const int64_t *__restrict__ rp, int64_t nrows, int bs, int64_t *__restrict__ rp_out)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n > nrows) return;
    if (n == nrows) { rp_out[bs * nrows] = (int64_t)bs * bs * rp[nrows]; return; }
    const int64_t len = rp[n + 1] - rp[n];
    for (int x = 0; x < bs; ++x) rp_out[bs * n + x] = (int64_t)bs * bs * rp[n] + (int64_t)x * bs * len;
}
__global__ void k_expand_cols(const int64_t *__restrict__ rp, const int32_t *__restrict__ ci, int64_t nrows, int bs,
                              int32_t *__restrict__ ci_out)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nrows) return;
    const int64_t r0 = rp[n], len = rp[n + 1] - r0;
    for (int x = 0; x < bs; ++x) {
        const int64_t o = (int64_t)bs * bs * r0 + (int64_t)x * bs * len;
        for (int64_t k = 0; k < len; ++k) {
            const int32_t m = ci[r0 + k];
            for (int y = 0; y < bs; ++y) ci_out[o + bs * k + y] = bs * m + y;
        }
    }
}

fem_status efail(fem_ctx *ctx, fem_status st, const char *fmt, ...)
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
fem_status ehip(fem_ctx *ctx, hipError_t e, const char *what)
{
    return efail(ctx, e == hipErrorOutOfMemory ? FEM_E_NOMEM : FEM_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}
#define EHIP(call, what)                                   \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return ehip(ctx, e_, what);  \
    } while (0)

bool emap_ok(const fem_map *m, const fem_set *from, int arity)
{
    return m && m->from && m->to && m->from->size == from->size && m->arity == arity && m->to->size >= 0 &&
           (m->values || from->size == 0);
}
bool edat_ok(const fem_dat *d, const fem_set *set, int dim)
{
    return d && d->set && d->dim == dim && d->set->size == set->size && (d->data || set->size == 0);
}

int upper_pair(int i, int j) { return i * NL - i * (i - 1) / 2 + (j - i); }

template <typename T>
hipError_t put(const fem_mem &m, T **dst, const std::vector<T> &src, size_t *bytes, hipStream_t s)
{
    const size_t n = src.size() * sizeof(T);
    hipError_t e = mem_alloc(m, s, false, n ? n : 8, (void **)dst);
    if (e != hipSuccess) return e;
    *bytes += n;
    return n ? hipMemcpyAsync(*dst, src.data(), n, hipMemcpyHostToDevice, s) : hipSuccess;
}

}  // namespace

fem_status elast_check(fem_ctx *ctx, const fem_form *form, const fem_args *a)
{
    if (form->cell != FEM_TETRAHEDRON || form->degree != 2 || form->dim != 3)
        return efail(ctx, FEM_E_UNSUPPORTED, "elasticity is provided for the P2 vector space on tetrahedra");
    if (!a || !a->cells || !a->cell_vertex || !a->cell_node || !a->coords || !a->cell_coord)
        return efail(ctx, FEM_E_ARG, "elasticity args: cells, cell_vertex, cell_node, cell_coord and coords are required");
    if (!emap_ok(a->cell_vertex, a->cells, 4) || !emap_ok(a->cell_node, a->cells, NL) ||
        !emap_ok(a->cell_coord, a->cells, 4))
        return efail(ctx, FEM_E_ARG, "elasticity args: Maps must start from the cell Set with arities 4, 10, 4");
    if (!edat_ok(a->coords, a->cell_coord->to, 3))
        return efail(ctx, FEM_E_ARG, "elasticity args: coords must be a dim-3 Dat on cell_coord's target Set");
    if (a->ncoeff < 2 || !edat_ok(a->coeff[0], a->cell_vertex->to, 1) || !edat_ok(a->coeff[1], a->cell_vertex->to, 1))
        return efail(ctx, FEM_E_ARG, "elasticity args: coeff[0] = mu and coeff[1] = lam must be scalar Dats on "
                                     "cell_vertex's target Set");
    if (a->cells->size >= (int64_t)1 << 24)
        return efail(ctx, FEM_E_OVERFLOW, "elasticity: at most 2^24 - 1 cells");
    if (3 * a->cell_node->to->size > INT32_MAX) return efail(ctx, FEM_E_OVERFLOW, "elasticity: too many DOFs");
    return FEM_OK;
}

fem_status elast_plan_create(fem_ctx *ctx, const fem_form *form, const fem_args *args, const fem_sparsity *sp,
                             fem_plan **out)
{
    fem_status st = elast_check(ctx, form, args);
    if (st != FEM_OK) return st;
    const int64_t C = args->cells->size, N = args->cell_node->to->size, R = 3 * N;
    if (!sp || !sp->row_ptr || sp->nrows != R || sp->ncols != R || (!sp->col_idx && sp->nnz > 0))
        return efail(ctx, FEM_E_ARG, "elasticity plan: a vector CSR with 3 x nodes rows and columns is required");
    hipStream_t s = ctx->stream;
    // Map range checks on the device (every entry is read once)
    int *dflag = nullptr, hflag = 0;
    EHIP(mem_alloc(ctx->mem, s, true, sizeof(int), (void **)&dflag), "alloc");
    const fem_map *maps[3] = {args->cell_node, args->cell_vertex, args->cell_coord};
    for (const fem_map *m : maps) {
        hipError_t e = fill_i32(dflag, 1, 0, s);
        if (e == hipSuccess) e = check_range(m->values, m->from->size * (int64_t)m->arity, m->to->size, dflag, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { mem_free(ctx->mem, s, true, dflag); return ehip(ctx, e, "range check"); }
        if (hflag) {
            mem_free(ctx->mem, s, true, dflag);
            return efail(ctx, FEM_E_RANGE, "elasticity plan: a Map entry lies outside its target Set");
        }
    }
    mem_free(ctx->mem, s, true, dflag);
    std::vector<int32_t> cn((size_t)C * NL);
    std::vector<int64_t> rp3(R + 1);
    std::vector<int32_t> ci3((size_t)sp->nnz);
    if (!cn.empty())
        EHIP(hipMemcpyAsync(cn.data(), args->cell_node->values, cn.size() * 4, hipMemcpyDeviceToHost, s), "copy");
    EHIP(hipMemcpyAsync(rp3.data(), sp->row_ptr, (R + 1) * 8, hipMemcpyDeviceToHost, s), "copy");
    if (!ci3.empty()) EHIP(hipMemcpyAsync(ci3.data(), sp->col_idx, ci3.size() * 4, hipMemcpyDeviceToHost, s), "copy");
    EHIP(hipStreamSynchronize(s), "sync");
    // the vector CSR must be the 3 x 3 expansion of a node pattern
    std::vector<int64_t> rpn(N + 1, 0);
    if (rp3[0] != 0 || rp3[R] != sp->nnz) return efail(ctx, FEM_E_ARG, "elasticity plan: row_ptr does not span [0, nnz]");
    for (int64_t n = 0; n < N; ++n) {
        const int64_t l3 = rp3[3 * n + 1] - rp3[3 * n];
        if (l3 % 3 || rp3[3 * n + 2] - rp3[3 * n + 1] != l3 || rp3[3 * n + 3] - rp3[3 * n + 2] != l3 ||
            rp3[3 * n] != 9 * rpn[n])
            return efail(ctx, FEM_E_ARG, "elasticity plan: the CSR is not a 3x3-block expansion of a node pattern");
        rpn[n + 1] = rpn[n] + l3 / 3;
    }
    const int64_t ns = rpn[N];
    if (ns > INT32_MAX - 1) return efail(ctx, FEM_E_OVERFLOW, "elasticity plan: too many node pairs");
    std::vector<int32_t> cin((size_t)ns);
    std::atomic<bool> bad{false};
    par_ranges(N, [&](int64_t n0, int64_t n1) {
        for (int64_t n = n0; n < n1 && !bad.load(std::memory_order_relaxed); ++n) {
            const int64_t len = rpn[n + 1] - rpn[n];
            for (int64_t k = 0; k < len; ++k) {
                const int32_t c0 = ci3[rp3[3 * n] + 3 * k];
                bool ok = c0 % 3 == 0 && c0 >= 0 && c0 < R && (k == 0 || c0 / 3 > cin[rpn[n] + k - 1]);
                for (int x = 0; x < 3 && ok; ++x)
                    for (int y = 0; y < 3; ++y) ok = ok && ci3[rp3[3 * n + x] + 3 * k + y] == c0 + y;
                if (!ok) { bad = true; return; }
                cin[rpn[n] + k] = c0 / 3;
            }
        }
    });
    if (bad) return efail(ctx, FEM_E_ARG, "elasticity plan: the CSR is not a 3x3-block expansion of a node pattern");
    std::vector<int32_t>().swap(ci3);
    // contributions: slot of every (cell, li, lj), counted then filled in cell order
    std::vector<int32_t> slot_of((size_t)C * NL * NL);
    par_ranges(C, [&](int64_t ca, int64_t cb) {
        for (int64_t c = ca; c < cb && !bad.load(std::memory_order_relaxed); ++c)
            for (int li = 0; li < NL; ++li) {
                const int32_t n = cn[c * NL + li];
                const int32_t *b0 = cin.data() + rpn[n], *b1 = cin.data() + rpn[n + 1];
                for (int lj = 0; lj < NL; ++lj) {
                    const int32_t m = cn[c * NL + lj];
                    const int32_t *f = std::lower_bound(b0, b1, m);
                    if (f == b1 || *f != m) { bad = true; return; }
                    slot_of[(c * NL + li) * NL + lj] = (int32_t)(f - cin.data());
                }
            }
    });
    if (bad) return efail(ctx, FEM_E_ARG, "elasticity plan: the sparsity lacks entries the Maps reach");
    std::vector<int32_t> sptr(ns + 1, 0);
    for (int32_t e : slot_of) sptr[e + 1]++;
    for (int64_t e = 0; e < ns; ++e) sptr[e + 1] += sptr[e];
    std::vector<uint32_t> ent((size_t)C * NL * NL);
    {
        std::vector<int32_t> cur(sptr.begin(), sptr.end() - 1);
        for (int64_t c = 0; c < C; ++c)
            for (int li = 0; li < NL; ++li)
                for (int lj = 0; lj < NL; ++lj) {
                    const int32_t e = slot_of[(c * NL + li) * NL + lj];
                    const int p = li <= lj ? upper_pair(li, lj) : upper_pair(lj, li);
                    ent[cur[e]++] = ((uint32_t)c << 8) | ((uint32_t)p << 2) | ((uint32_t)(li == lj) << 1) |
                                    (uint32_t)(li > lj);
                }
    }
    std::vector<int32_t>().swap(slot_of);
    std::vector<int32_t> grow((size_t)(ns + 63) / 64 + 1, 0);
    {
        int64_t n = 0;
        for (size_t g = 0; g + 1 < grow.size(); ++g) {
            const int64_t e = (int64_t)g * 64;
            while (rpn[n + 1] <= e) ++n;
            grow[g] = (int32_t)n;
        }
    }
    fem_plan *p = new (std::nothrow) fem_plan;
    if (!p) return efail(ctx, FEM_E_NOMEM, "plan_create: host allocation");
    p->is_mat = 2;
    p->dim = 3; p->degree = 2; p->nloc = NL;
    p->ncells = C; p->nrows = N; p->nverts = args->cell_vertex->to->size;
    p->nnz = sp->nnz;
    p->nblk = 0;
    p->cell_visits = C;
    p->cell_node = args->cell_node->values;
    p->cn_version = args->cell_node->version;
    p->row_ptr = sp->row_ptr;
    p->e_nslots = ns;
    p->e_prec = (int)form->prec;
    p->mem = ctx->mem;
    hipError_t e = put(p->mem, &p->e_slot_ptr, sptr, &p->bytes, s);
    if (e == hipSuccess) e = put(p->mem, &p->e_ent, ent, &p->bytes, s);
    if (e == hipSuccess) e = put(p->mem, &p->e_grow, grow, &p->bytes, s);
    const size_t wbytes = form->prec == FEM_FP64   ? (size_t)C * NP * Ws<double>::BS * 8
                          : form->prec == FEM_BF16 ? (size_t)C * NP * Ws<uint16_t>::BS * 2
                          : form->prec == FEM_FP16 ? (size_t)C * NP * Ws<half_ws>::BS * 2
                                                   : (size_t)C * NP * Ws<float>::BS * 4;
    if (e == hipSuccess) e = mem_alloc(p->mem, s, false, wbytes ? wbytes : 8, &p->e_work);
    if (e == hipSuccess) p->bytes += wbytes;
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        fem_plan_destroy(p);
        return ehip(ctx, e, "plan_create upload");
    }
    *out = p;
    return FEM_OK;
}

fem_status elast_assemble(fem_ctx *ctx, const fem_plan *plan, const fem_form *form, const fem_args *args, fem_mat *A,
                          fem_access acc)
{
    fem_status st = elast_check(ctx, form, args);
    if (st != FEM_OK) return st;
    if (!plan || plan->is_mat != 2) return efail(ctx, FEM_E_ARG, "assemble_mat: an elasticity plan is required");
    if ((int)form->prec != plan->e_prec) return efail(ctx, FEM_E_ARG, "assemble_mat: plan built for another precision");
    if (plan->cell_node != args->cell_node->values || plan->ncells != args->cells->size ||
        plan->nrows != args->cell_node->to->size || plan->nverts != args->cell_vertex->to->size)
        return efail(ctx, FEM_E_ARG, "plan was built for other Maps");
    if (plan->cn_version != args->cell_node->version)
        return efail(ctx, FEM_E_ARG, "plan was built for another version of its Maps (rebuild the plan)");
    if (!A || !A->sp || (!A->values && plan->nnz > 0)) return efail(ctx, FEM_E_ARG, "assemble_mat: Mat without values");
    if (A->sp->row_ptr != plan->row_ptr || A->sp->nnz != plan->nnz)
        return efail(ctx, FEM_E_ARG, "assemble_mat: Mat sparsity differs from the plan's");
    if (acc != FEM_WRITE && acc != FEM_INC) return efail(ctx, FEM_E_ARG, "a Mat accepts only WRITE or INC");
    const int64_t C = plan->ncells;
    if (C == 0) return FEM_OK;
    ElArgs ea;
    ea.cell_vertex = args->cell_vertex->values;
    ea.cell_coord = args->cell_coord->values;
    ea.coords = args->coords->data;
    ea.mu = args->coeff[0]->data;
    ea.lam = args->coeff[1]->data;
    ea.work = plan->e_work;
    ea.ncells = C;
    const int64_t groups = (C + CPW - 1) / CPW;
    const int64_t want = (groups + (EWG / 64) - 1) / (EWG / 64);
    const int grid = (int)std::min<int64_t>(want, (int64_t)ctx->num_cus * 8);
    hipStream_t s = ctx->stream;
    switch (form->prec) {
    case FEM_FP64: hipLaunchKernelGGL(k_elast_element<FEM_FP64>, dim3(grid), dim3(EWG), 0, s, ea); break;
    case FEM_FP32: hipLaunchKernelGGL(k_elast_element<FEM_FP32>, dim3(grid), dim3(EWG), 0, s, ea); break;
    case FEM_BF16: hipLaunchKernelGGL(k_elast_element<FEM_BF16>, dim3(grid), dim3(EWG), 0, s, ea); break;
    case FEM_FP16: hipLaunchKernelGGL(k_elast_element<FEM_FP16>, dim3(grid), dim3(EWG), 0, s, ea); break;
    default: return efail(ctx, FEM_E_UNSUPPORTED, "precision");
    }
    EHIP(hipGetLastError(), "elasticity element launch");
    const int64_t ns = plan->e_nslots;
    if (ns == 0) return FEM_OK;
    const int pg = (int)((ns + 255) / 256 + 7) / 8 * 8;   // a multiple of 8 (XCD-grouped ranks)
    if (form->prec == FEM_FP64)
        hipLaunchKernelGGL(k_elast_pull<double>, dim3(pg), dim3(256), 0, s, plan->row_ptr, plan->e_slot_ptr, plan->e_ent,
                           plan->e_grow, (const double *)plan->e_work, A->values, ns, (int)(acc == FEM_INC));
    else if (form->prec == FEM_BF16)
        hipLaunchKernelGGL(k_elast_pull<uint16_t>, dim3(pg), dim3(256), 0, s, plan->row_ptr, plan->e_slot_ptr,
                           plan->e_ent, plan->e_grow, (const uint16_t *)plan->e_work, A->values, ns,
                           (int)(acc == FEM_INC));
    else if (form->prec == FEM_FP16)
        hipLaunchKernelGGL(k_elast_pull<half_ws>, dim3(pg), dim3(256), 0, s, plan->row_ptr, plan->e_slot_ptr,
                           plan->e_ent, plan->e_grow, (const half_ws *)plan->e_work, A->values, ns,
                           (int)(acc == FEM_INC));
    else
        hipLaunchKernelGGL(k_elast_pull<float>, dim3(pg), dim3(256), 0, s, plan->row_ptr, plan->e_slot_ptr, plan->e_ent,
                           plan->e_grow, (const float *)plan->e_work, A->values, ns, (int)(acc == FEM_INC));
    EHIP(hipGetLastError(), "elasticity pull launch");
    return FEM_OK;
}

}  // namespace femk

extern "C" fem_status fem_expand_sparsity(fem_ctx *ctx, const fem_sparsity *node, int32_t bs, fem_sparsity *out)
{
    using namespace femk;
    if (!ctx) return FEM_E_ARG;
    if (!node || !out || !node->row_ptr || !out->row_ptr || (!node->col_idx && node->nnz > 0) || node->nrows < 0)
        return efail(ctx, FEM_E_ARG, "expand_sparsity: NULL argument");
    if (bs < 1 || bs > 8) return efail(ctx, FEM_E_ARG, "expand_sparsity: block size must be 1..8");
    if ((int64_t)bs * node->ncols > INT32_MAX || (int64_t)bs * bs * node->nnz > ((int64_t)1 << 40))
        return efail(ctx, FEM_E_OVERFLOW, "expand_sparsity: expanded sizes overflow the index types");
    hipStream_t s = ctx->stream;
    const int64_t n = node->nrows;
    if (!out->col_idx) {
        out->nrows = bs * n;
        out->ncols = bs * node->ncols;
        out->nnz = (int64_t)bs * bs * node->nnz;
        hipLaunchKernelGGL(k_expand_rows, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, s, node->row_ptr, n, (int)bs,
                           out->row_ptr);
        EHIP(hipGetLastError(), "expand rows");
        return FEM_OK;
    }
    if (out->nrows != bs * n || out->nnz != (int64_t)bs * bs * node->nnz)
        return efail(ctx, FEM_E_ARG, "expand_sparsity: output sizes do not match the counting call");
    if (n > 0) {
        hipLaunchKernelGGL(k_expand_cols, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, node->row_ptr, node->col_idx,
                           n, (int)bs, out->col_idx);
        EHIP(hipGetLastError(), "expand cols");
    }
    return FEM_OK;
}
