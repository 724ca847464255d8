// Cell-loop assembly kernels for gfx950 (MI355X).
//
// The parallel loop of the paper ("Parloops and kernels") runs the local
// kernel on every cell with data gathered through Maps (READ) and adds the
// element tensor into the output (INC).  Here the INC is made conflict-free
// and deterministic by owning OUTPUT ROWS instead of colouring cells: the plan
// splits the rows into contiguous blocks; one workgroup owns a block and
// visits every cell incident to its rows, in an order fixed by the plan.  It
//   1. gathers the cells' vertex coordinates and P1 coefficients,
//   2. computes the FP64 geometry (adjugate, |det J|, metric
//      |det J| grad(l_m).grad(l_n)) and the element tensor from the exact
//      reference integrals (generated straight-line FMA code), into LDS,
//   3. sums, per output value, the entries that land on it, in ascending cell
//      id: Mat values are held in LDS and walked by a per-lane index stream;
//      Dat values are summed in registers by the lane owning the row,
// and finally writes its rows once, contiguously (the block's rows occupy one
// contiguous range of the CSR values).  No atomics and no inter-workgroup
// communication are used, so the result is bitwise reproducible; the price is
// that a cell straddling two row blocks is evaluated by both.
#include "fem_internal.h"
#include "fem_geom.h"
#include "fem_tables.h"

#include <algorithm>

namespace femk {
namespace {


typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
template <int W> struct BatchOf;
template <> struct BatchOf<8> { typedef u32x4 T; };
template <> struct BatchOf<4> { typedef u32x2 T; };
typedef BatchOf<MAT_BATCH>::T Batch;   // one lane's batch of Mat stream indices

// Everything a kernel reads, by value: device pointers and scalars only.
struct KArgs {
    const int32_t *__restrict__ blk_row0;
    const int32_t *__restrict__ blk_cptr;
    const int32_t *__restrict__ bcell;
    const int32_t *__restrict__ bverts;
    const int32_t *__restrict__ inc_ptr;
    const uint16_t *__restrict__ ent;
    const int32_t *__restrict__ blk_hdr;
    const int32_t *__restrict__ blk_w;
    const int32_t *__restrict__ wq;
    const uint32_t *__restrict__ pstream;   // batches of MAT_BATCH 16-bit indices
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
    k.blk_hdr = p.blk_hdr; k.blk_w = p.blk_w; k.wq = p.wq; k.pstream = reinterpret_cast<const uint32_t *>(p.pstream);
    k.row_ptr = a.row_ptr; k.coords = a.coords;
    k.cell_node = a.cell_node; k.coeff = a.coeff; k.x = a.x; k.out = a.out;
    k.cstiff = a.cstiff; k.cmass = a.cmass; k.inc = a.inc;
    return k;
}

constexpr int LDS_DOUBLES = 163840 / 8;    // gfx950: 160 KiB of LDS per CU

// Workgroup barrier for LDS traffic only: waits for this wave's LDS operations
// and meets the other waves, but leaves global loads in flight (the waves of
// these kernels communicate through LDS only; inputs are read-only and each
// output element is written by one lane).  __syncthreads() would also drain
// every outstanding global load, which defeats prefetching across stages.
// The memory clobber keeps the compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Wait for every global load this wave has issued (the data of a software
// pipeline stage, issued one stage earlier).
__device__ __forceinline__ void wait_loads()
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// Plan arrays are never written by a kernel.  Reading them through the
// constant address space lets the compiler use scalar loads for uniform
// addresses; their waits count on lgkmcnt instead of vmcnt, which on gfx9
// also counts stores and outstanding prefetches (a vector load of a block
// header would otherwise drain every load and store in flight).
template <typename T>
__device__ __forceinline__ T ldc(const T *p)
{
    return *(const __attribute__((address_space(4))) T *)p;
}

// ---------------------------------------------------------------- geometry: Geo<D> (fem_geom.h)

// ---------------------------------------------------------------- configs

// Mat kernels: workgroups of MWG lanes (one per CU: they take all of its
// LDS).  A chunk of CCH cells is computed LPC lanes per cell (each lane
// evaluates NG/LPC entry groups of the element tensor); LDS holds, in
// doubles, [0, SCAP) the block's Mat values, [SCAP, SCAP + CCH*NE) the
// chunk's packed element tensors and one -0.0 at ZIDX.  A block holds at
// most MCH chunks of cells (its values stay in LDS while the chunks pass
// through); MCH was measured per case: more chunks lower the redundancy
// until the value area, not the cells, bounds the block.
// WG lanes per workgroup (512 or 1024: 8 or 16 waves on the CU); NB stream
// batches of a lane held in registers (longer streams load the rest as they
// go); MT: the element tensors are formed from kc = cstiff kappa and the
// metric (terms grouped by metric pair) instead of the (d+1) x NM products
// P, which keeps fewer values live.  All measured per case: MT paid
// everywhere but on P3 triangles (P2 tetrahedra 510 -> 463 us); 1024 lanes
// paid on triangles of degree 2 and 3 (16 waves hide more latency) and lost
// on P2 tetrahedra, where the chunk cannot grow with them and the shorter
// per-lane streams pad more.  The element
// tensors take every wave only if CCH LPC reaches WG with a part that is the
// same across each wave (CCH a multiple of 64): P3 tetrahedra went from 32
// cells x 4 lanes (two of eight waves evaluating, 5.2 ms) to 64 cells x 8
// lanes (2.96 ms), although the larger chunk halves the value area and
// raises the redundancy from 3.37 to 4.09.  P1 takes 1,024-cell chunks on
// 1,024 lanes (116 VGPRs on tetrahedra): each lane's stream per chunk is as
// long as with 512 and 512 but half the blocks' chunk boundaries, and 16
// waves hide more latency (P1 triangles 2048^2 241 -> 182 us, tetrahedra
// 64^3 83 -> 73 us, 128^3 619 -> 594 us with a smaller value area).  P2
// triangles fill the 1,024 lanes with 512-cell chunks (189 -> 184 us at
// 1024^2, against 384-cell chunks on 768 lanes).
template <int D, int K> struct MatCfg;
template <> struct MatCfg<2, 1> { static constexpr int CCH = 1024, LPC = 1, MCH = 2, WG = 1024, NB = 4; static constexpr bool MT = true; };
template <> struct MatCfg<3, 1> { static constexpr int CCH = 1024, LPC = 1, MCH = 8, WG = 1024, NB = 4; static constexpr bool MT = true; };
template <> struct MatCfg<2, 2> { static constexpr int CCH = 512, LPC = 2, MCH = 1, WG = 1024, NB = 4; static constexpr bool MT = true; };
template <> struct MatCfg<3, 2> { static constexpr int CCH = 256, LPC = 2, MCH = 2, WG = 512, NB = 64 / MAT_BATCH; static constexpr bool MT = true; };
template <> struct MatCfg<2, 3> { static constexpr int CCH = 128, LPC = 4, MCH = 4, WG = 1024, NB = 4; static constexpr bool MT = false; };
template <> struct MatCfg<3, 3> { static constexpr int CCH = 64, LPC = 8, MCH = 8, WG = 512, NB = 64 / MAT_BATCH; static constexpr bool MT = true; };

// Dat and action kernels: workgroups of WG lanes, KR rows per lane; the
// per-cell local vectors of the whole block live in LDS (VLDS doubles, two
// workgroups per CU).
constexpr int VWG = 512;
constexpr int VKR = 2;
constexpr int VROWS = VKR * VWG;   // rows of a Dat plan block
// The source vector's kernel needs few registers: it runs VROWS lanes of one
// row each (twice the waves per CU: P2 tetrahedra 85 -> 68 us), except on P3
// tetrahedra, whose 78 VGPRs would then leave room for one workgroup per CU;
// the action keeps VWG lanes of VKR rows.
template <int D, int K, bool ACTION> struct VecWG {
    static constexpr int WG = ACTION || (D == 3 && K == 3) ? VWG : VROWS, KR = VROWS / WG;
};
constexpr int VLDS = LDS_DOUBLES / 2;
constexpr int VPRE = 8;     // entries of a row fetched per batch
// Action: y_K = A_K x_K from the cstiff-scaled nodal kappa and the metric.
// P1: terms grouped by metric pair (act_t), rather than formed from the
// (d+1) x NM products P, which keeps fewer registers live.  PREFETCH gathers
// the next cell's inputs while the current one is evaluated; the P2
// tetrahedron drops it to stay within 128 VGPRs (four waves per SIMD),
// which measured 125 against 153 us at 64^3 x 6 cells.
// QUAD (P2, P3): the stiffness part at the points of a rule exact for its
// degree (act_q: degree 3 for P2, about 380 instead of 835 FMAs per P2
// tetrahedron; degree 5 for P3, 15 points on the tetrahedron), the mass
// part from the exact reference mass matrix; P1 keeps act_t.
template <int D, int K> struct ActCfg {
    static constexpr bool QUAD = K >= 2;
    static constexpr bool PREFETCH = !(D == 3 && K == 2);
};

template <int D, int K> struct TabOf;
template <> struct TabOf<2, 1> { using T = femtab::Tab21; };
template <> struct TabOf<2, 2> { using T = femtab::Tab22; };
template <> struct TabOf<2, 3> { using T = femtab::Tab23; };
template <> struct TabOf<3, 1> { using T = femtab::Tab31; };
template <> struct TabOf<3, 2> { using T = femtab::Tab32; };
template <> struct TabOf<3, 3> { using T = femtab::Tab33; };

template <int D, int K> struct MatLds {
    static constexpr int NE = TabOf<D, K>::T::NE;
    static constexpr int CCH = MatCfg<D, K>::CCH;
    static constexpr int ECH = CCH * NE;                              // element tensors of a chunk
    static constexpr int SCAP = (LDS_DOUBLES - ECH - 1) / 8 * 8;       // Mat values of a block
    static constexpr int ZIDX = SCAP + ECH;                           // holds -0.0
    static constexpr int TOTAL = ZIDX + 1;
    static_assert(TOTAL <= LDS_DOUBLES && TOTAL <= 65536, "16-bit LDS indices");
    static_assert(SCAP > 0, "room for Mat values");
};

constexpr int lbits_for(int nloc) { return nloc <= 4 ? 2 : nloc <= 8 ? 3 : nloc <= 16 ? 4 : 5; }

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

template <int D>
__device__ __forceinline__ void issue_verts(const int32_t *__restrict__ bverts, int visit, int32_t (&v)[D + 1])
{
    if constexpr (D == 3) {
        const int4 q = *reinterpret_cast<const int4 *>(bverts + (int64_t)visit * 4);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
#pragma unroll
        for (int m = 0; m <= D; ++m) v[m] = bverts[(int64_t)visit * (D + 1) + m];
    }
}

// Vertex ids of one cell kept as one register tuple (a tetrahedron's four
// ids are one 16-byte load), so that a prefetched copy is not split over
// registers that the compiler would have to fill as soon as it arrives.
template <int D> struct VIds;
template <> struct VIds<3> {
    i32x4 q;
    __device__ __forceinline__ void load(const int32_t *__restrict__ bverts, int visit)
    {
        q = *reinterpret_cast<const i32x4 *>(bverts + (int64_t)visit * 4);
    }
    __device__ __forceinline__ void hold() { asm volatile("" : "+v"(q)); }
    __device__ __forceinline__ void get(int32_t (&v)[4]) const { v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w; }
};
template <> struct VIds<2> {
    int32_t q[3];
    __device__ __forceinline__ void load(const int32_t *__restrict__ bverts, int visit)
    {
#pragma unroll
        for (int m = 0; m < 3; ++m) q[m] = bverts[(int64_t)visit * 3 + m];
    }
    __device__ __forceinline__ void hold()
    {
#pragma unroll
        for (int m = 0; m < 3; ++m) asm volatile("" : "+v"(q[m]));
    }
    __device__ __forceinline__ void get(int32_t (&v)[3]) const { v[0] = q[0]; v[1] = q[1]; v[2] = q[2]; }
};

template <int D>
__device__ __forceinline__ void issue_coords(const int32_t (&v)[D + 1], const double *__restrict__ X,
                                             const double *__restrict__ coef, CellIn<D> &c)
{
#pragma unroll
    for (int m = 0; m <= D; ++m) {
#pragma unroll
        for (int r = 0; r < D; ++r) c.x[m][r] = X[(int64_t)v[m] * D + r];
        c.k[m] = coef[v[m]];
    }
}

// Entry groups [part NG/LPC, (part + 1) NG/LPC) of a cell's packed element
// tensor.  The common splits call the groups by name; others go through the
// numbered dispatch (a uniform branch when the part is the same on a wave).
template <class T, int LPC>
__device__ __forceinline__ void mat_part(int part, const double *P, double madet, double *E)
{
    static_assert(T::NG % LPC == 0, "entry groups per lane");
    if constexpr (T::NG == 1) {
        T::mat_group0(P, madet, E);
    } else if constexpr (T::NG == 4 && LPC == 1) {
        T::mat_group0(P, madet, E); T::mat_group1(P, madet, E);
        T::mat_group2(P, madet, E); T::mat_group3(P, madet, E);
    } else if constexpr (T::NG == 4 && LPC == 2) {
        if (part == 0) { T::mat_group0(P, madet, E); T::mat_group1(P, madet, E); }
        else { T::mat_group2(P, madet, E); T::mat_group3(P, madet, E); }
    } else {
        constexpr int GPL = T::NG / LPC;
#pragma unroll
        for (int i = 0; i < GPL; ++i) T::mat_group_n(part * GPL + i, P, madet, E);
    }
}

// The same entry groups from kc and the metric.
template <class T, int LPC>
__device__ __forceinline__ void mat_part_t(int part, const double *kc, const double *G, double madet, double *E)
{
    static_assert(T::NG % LPC == 0, "entry groups per lane");
    if constexpr (T::NG == 1) {
        T::mat_group_t0(kc, G, madet, E);
    } else if constexpr (T::NG == 4 && LPC == 1) {
        T::mat_group_t0(kc, G, madet, E); T::mat_group_t1(kc, G, madet, E);
        T::mat_group_t2(kc, G, madet, E); T::mat_group_t3(kc, G, madet, E);
    } else if constexpr (T::NG == 4 && LPC == 2) {
        if (part == 0) { T::mat_group_t0(kc, G, madet, E); T::mat_group_t1(kc, G, madet, E); }
        else { T::mat_group_t2(kc, G, madet, E); T::mat_group_t3(kc, G, madet, E); }
    } else {
        constexpr int GPL = T::NG / LPC;
#pragma unroll
        for (int i = 0; i < GPL; ++i) T::mat_group_tn(part * GPL + i, kc, G, madet, E);
    }
}

// Element tensor entries of this lane's part of a cell, into E.
template <int D, int K>
__device__ __forceinline__ void cell_tensor(int part, const CellIn<D> &c, double cstiff, double cmass, double *E)
{
    using T = typename TabOf<D, K>::T;
    constexpr int LPC = MatCfg<D, K>::LPC;
    if constexpr (MatCfg<D, K>::MT) {
        double G[Geo<D>::NM], kc[D + 1];
        const double adet = Geo<D>::metric(c.x, G);
#pragma unroll
        for (int m = 0; m <= D; ++m) kc[m] = cstiff * c.k[m];
        mat_part_t<T, LPC>(part, kc, G, cmass * adet, E);
    } else {
        double P[(D + 1) * Geo<D>::NM], madet;
        tensor_inputs<D>(c, cstiff, cmass, P, &madet);
        mat_part<T, LPC>(part, P, madet, E);
    }
}

// One batch of MAT_BATCH stream indices of a lane.  The lane keeps the
// running sum of the Mat value it has open in registers (acc, its LDS byte
// address in cur).  Index i < SCAP opens Mat value i: the open value is
// written back and the running sum restarts from what LDS holds at i (-0.0
// the first time, a partial sum from an earlier chunk otherwise); any other
// index adds the LDS double it names.  All loads of the batch are issued
// first: an opened value is never written earlier in the same batch (a lane
// opens each value once per chunk, and writes only values it has open).
// The sum is formed for every index and the write-back is the only masked
// step: left to itself the compiler moves the add into an if/else around
// each index, two branches and four exec-mask updates per index, which cost
// 3-5% of the Mat kernels' time.  Writing back at every index instead (no
// mask at all) was slower still: it doubles the LDS traffic of the walk.
template <int SCAP>
__device__ __forceinline__ void pull_batch(const Batch w, char *lds, uint32_t &cur, double &acc)
{
    constexpr int NI = MAT_BATCH;
    uint32_t ad[NI];
    double v[NI];
#pragma unroll
    for (int j = 0; j < NI; ++j) {
        const uint32_t wd = w[j >> 1];
        ad[j] = ((j & 1) ? (wd >> 16) : (wd & 0xffffu)) << 3;   // byte address
        v[j] = *reinterpret_cast<const double *>(lds + ad[j]);
    }
#pragma unroll
    for (int j = 0; j < NI; ++j) {
        const bool open = ad[j] < (uint32_t)SCAP * 8u;
        double sum = acc + v[j];
        asm volatile("" : "+v"(sum));   // formed here, not inside a branch
        const uint32_t pc = cur;
        const double pa = acc;
        cur = open ? ad[j] : cur;
        acc = open ? v[j] : sum;
        if (open) *reinterpret_cast<double *>(lds + pc) = pa;
    }
}

// Uniform description of one row block: the plan's 32-byte header, one
// scalar load.  [0..1] first Mat value, [2] Mat values, [3] first cell,
// [4] cells, [5] chunks, [6] first (chunk, wave) stream.
typedef int32_t i32x8 __attribute__((ext_vector_type(8)));
struct MatBlk {
    i32x8 v;
    __device__ __forceinline__ int64_t s0() const { return (int64_t)(((uint64_t)(uint32_t)v[1] << 32) | (uint32_t)v[0]); }
    __device__ __forceinline__ int ns() const { return v[2]; }
    __device__ __forceinline__ int c0() const { return v[3]; }
    __device__ __forceinline__ int nc() const { return v[4]; }
    __device__ __forceinline__ int nq() const { return v[5]; }
    __device__ __forceinline__ int w0() const { return v[6]; }
};

__device__ __forceinline__ MatBlk mat_blk(const KArgs &a, int b)
{
    MatBlk h;
    h.v = ldc(reinterpret_cast<const i32x8 *>(a.blk_hdr) + b);
    return h;
}

// Keeps the compiler from consuming a prefetched register before this point
// (it would otherwise hoist address arithmetic next to the load and wait for
// the load right there).
template <typename T>
__device__ __forceinline__ void hold(T &x)
{
    asm volatile("" : "+v"(x));
}

// Walks the lane's stream of one (chunk, wave): the first NBMAX batches were
// loaded into sv ahead of time (every stream has at least one batch), rare
// longer streams load the rest one batch at a time.  Ends by writing back
// the value left open.
template <int SCAP, int ZIDX, int NBMAX>
__device__ __forceinline__ void pull_stream(Batch (&sv)[NBMAX], const Batch *__restrict__ ps, int nb,
                                            double *lds)
{
    char *lb = reinterpret_cast<char *>(lds);
    uint32_t cur = (uint32_t)ZIDX * 8u;   // until the first open: ZIDX, which keeps -0.0
    double acc = -0.0;
#pragma unroll
    for (int i = 0; i < NBMAX; ++i)
        if (i < nb) pull_batch<SCAP>(sv[i], lb, cur, acc);
    for (int i = NBMAX; i < nb; ++i) pull_batch<SCAP>(ps[(int64_t)i * 64], lb, cur, acc);
    *reinterpret_cast<double *>(lb + cur) = acc;
}

// Waits for every prefetched stream batch at once (they were issued before
// the chunk's element tensors were computed, so they have long arrived).
// Done before any younger prefetch is issued, the stream walk then waits for
// nothing (waits count loads in issue order).
template <int NBMAX>
__device__ __forceinline__ void hold_stream(Batch (&sv)[NBMAX])
{
#pragma unroll
    for (int i = 0; i < NBMAX; ++i) asm volatile("" : "+v"(sv[i]));
}

template <int NBMAX>
__device__ __forceinline__ void load_stream(Batch (&sv)[NBMAX], const Batch *__restrict__ ps, int nb)
{
#pragma unroll
    for (int i = 0; i < NBMAX; ++i) sv[i] = ps[(int64_t)(i < nb ? i : nb - 1) * 64];
}

// Stream of chunk q of a block, for this wave.
template <int NW>
__device__ __forceinline__ void chunk_stream(const KArgs &a, const MatBlk &h, int q, int wave, int lane, int &nb,
                                             const Batch *__restrict__ &ps)
{
    const int st = ldc(a.wq + h.w0() + NW * q + wave);
    nb = (ldc(a.wq + h.w0() + NW * q + wave + 1) - st) >> 6;
    ps = reinterpret_cast<const Batch *>(a.pstream) + st + lane;
}

// Persistent: one workgroup per CU walks a contiguous range of row blocks
// (the workgroups of one XCD, launch index mod 8, take one contiguous eighth
// of the blocks, so neighbouring blocks share that XCD's L2).  Software
// pipeline over the units (block, chunk): while one unit computes and walks
// its stream, the next unit's vertex ids, coordinates and first stream
// batches are in flight (the next chunk of the block, or the first chunk of
// the next block), and the header of block b+2 is loaded.  Per unit:
//   issue the next unit's vertex ids; compute the element tensors into LDS
//   (cell data gathered during the previous unit); barrier; issue the next
//   unit's coordinates; walk the stream; issue the next unit's first stream
//   batches; barrier.
// After a block's last unit: write its Mat values out (one contiguous,
// coalesced range) and reset the value area to -0.0, the identity of the
// sums, for the next block (each lane touches the same LDS values in both
// loops).
// The common path has no branch around a global load, and every prefetched
// register is consumed before a younger load is waited for, so the
// compiler's waits stay exact and never drain the prefetches.
template <int D, int K>
__device__ __forceinline__ void mat_blocks(const KArgs &a, int bb, int be)
{
    using T = typename TabOf<D, K>::T;
    using L = MatLds<D, K>;
    constexpr int NE = T::NE, CCH = L::CCH, LPC = MatCfg<D, K>::LPC;
    constexpr int MWG = MatCfg<D, K>::WG, NW = MWG / 64;
    constexpr int CO = 4;         // Mat values per lane and round of the write-out
    static_assert(MWG == 512 || MWG == 1024, "workgroup size");
    static_assert(CCH * LPC <= MWG, "one cell item per lane");
    static_assert(T::NG % LPC == 0, "groups per lane");
    __shared__ double lds[L::TOTAL];

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int lcc = tid % CCH, part = tid / CCH;
    const bool has_item = tid < CCH * LPC;
    double *__restrict__ E = lds + L::SCAP + lcc * NE;

    MatBlk h = mat_blk(a, bb);
    MatBlk hn = bb + 1 < be ? mat_blk(a, bb + 1) : h;
    int nb = 0;
    const Batch *__restrict__ ps = nullptr;
    Batch sv[MatCfg<D, K>::NB];  // first stream batches of the current unit
    CellIn<D> cin;               // first-chunk cell data of the current block
    VIds<D> vn;                  // vertex ids of the next block's first-chunk cell
    if (h.nq() > 0) {
        chunk_stream<NW>(a, h, 0, wave, lane, nb, ps);
        load_stream(sv, ps, nb);
    }
    if (has_item && lcc < h.nc()) {
        int32_t v[D + 1];
        issue_verts<D>(a.bverts, h.c0() + lcc, v);
        issue_coords<D>(v, a.coords, a.coeff, cin);
    }
    for (int s = tid; s < h.ns(); s += MWG) lds[s] = -0.0;
    if (tid == 0) lds[L::ZIDX] = -0.0;

    for (int b = bb; b < be; ++b) {
        const bool more = b + 1 < be;
        const MatBlk hnn = b + 2 < be ? mat_blk(a, b + 2) : hn;
        // One unit per chunk.  While chunk q of block b computes and walks
        // its stream, the next unit's data are in flight: chunk q+1 of this
        // block, or after the last chunk the first chunk of the next block.
        for (int q = 0; q < h.nq(); ++q) {
            const bool last = q + 1 == h.nq();
            const MatBlk hx = last ? hn : h;
            const int qx = last ? 0 : q + 1;
            const bool sx = last ? more && hn.nq() > 0 : true;   // next unit has a stream
            const bool cx = last ? more && hn.nc() > 0 : true;   // next unit has cells
            int nbx = 0;
            const Batch *__restrict__ psx = ps;
            if (sx) chunk_stream<NW>(a, hx, qx, wave, lane, nbx, psx);
            // uniform prefetch; lanes past the next chunk's cells load a
            // duplicate of the block's last cell, unused
            const int lcx = qx * CCH + lcc;
            if (cx) vn.load(a.bverts, hx.c0() + (lcx < hx.nc() ? lcx : hx.nc() - 1));
            if (has_item && q * CCH + lcc < h.nc()) cell_tensor<D, K>(part, cin, a.cstiff, a.cmass, E);
            lds_barrier();
            hold_stream(sv);
            if (cx) {
                int32_t v[D + 1];
                vn.hold();
                vn.get(v);
                issue_coords<D>(v, a.coords, a.coeff, cin);
            }
            pull_stream<L::SCAP, L::ZIDX>(sv, ps, nb, lds);
            if (sx) {
                load_stream(sv, psx, nbx);
                nb = nbx;
                ps = psx;
            }
            lds_barrier();
        }
        if (h.nq() == 0 && more) {
            // a block without cells: start the next block's first chunk here
            if (hn.nc() > 0) {
                int32_t v[D + 1];
                issue_verts<D>(a.bverts, hn.c0() + (lcc < hn.nc() ? lcc : hn.nc() - 1), v);
                issue_coords<D>(v, a.coords, a.coeff, cin);
            }
            if (hn.nq() > 0) {
                chunk_stream<NW>(a, hn, 0, wave, lane, nb, ps);
                load_stream(sv, ps, nb);
            }
        }
        // write-out: CO values per lane in flight at once
        double *__restrict__ out = a.out + h.s0();
        for (int s0 = tid; s0 < h.ns(); s0 += CO * MWG) {
            double t[CO];
#pragma unroll
            for (int k = 0; k < CO; ++k) t[k] = s0 + k * MWG < h.ns() ? lds[s0 + k * MWG] : 0.0;
            if (a.inc) {
#pragma unroll
                for (int k = 0; k < CO; ++k)
                    if (s0 + k * MWG < h.ns()) out[s0 + k * MWG] += t[k];
            } else {
#pragma unroll
                for (int k = 0; k < CO; ++k)
                    if (s0 + k * MWG < h.ns()) out[s0 + k * MWG] = t[k];
            }
        }
        for (int s = tid; s < hn.ns(); s += MWG) lds[s] = -0.0;
        h = hn;
        hn = hnn;
    }
}

// Persistent: one workgroup per CU walks a contiguous range of the blocks
// (XCD-grouped, above).
template <int D, int K>
__global__ __launch_bounds__((MatCfg<D, K>::WG)) void k_assemble_mat(KArgs a, int nblk)
{
    const int G = gridDim.x, bid = blockIdx.x;
    const int rank = G % 8 == 0 ? (bid % 8) * (G / 8) + bid / 8 : bid;
    const int bb = (int)((int64_t)nblk * rank / G), be = (int)((int64_t)nblk * (rank + 1) / G);
    if (bb >= be) return;
    mat_blocks<D, K>(a, bb, be);
}

// ---------------------------------------------------------------- Dat / action

template <int D, int K, bool ACTION>
__device__ __forceinline__ void vec_block(const KArgs &a, int b)
{
    constexpr int WG = VecWG<D, K, ACTION>::WG, KR = VecWG<D, K, ACTION>::KR;
    using T = typename TabOf<D, K>::T;
    constexpr int NL = T::NLOC, LB = lbits_for(NL);
    constexpr int CAP = VLDS / NL;
    __shared__ double vk[CAP * NL];
    const int tid = threadIdx.x;
    const int r0 = a.blk_row0[b], r1 = a.blk_row0[b + 1];
    constexpr bool PRE = !ACTION || ActCfg<D, K>::PREFETCH;
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
    // each row's entry range, loaded at once (two registers, in flight
    // during the cell phase)
    int cur[KR], end[KR];
    auto row_range = [&]() {
#pragma unroll
        for (int k = 0; k < KR; ++k) {
            const int r = r0 + tid + WG * k;
            cur[k] = r < r1 ? a.inc_ptr[r] : 0;
            end[k] = r < r1 ? a.inc_ptr[r + 1] : 0;
        }
    };
    row_range();
    if (PRE && tid < nc) fetch(tid);
    for (int cs = 0; cs < nc; cs += WG) {
        if (cs + tid < nc) {
            if (!PRE) fetch(cs + tid);
            double loc[NL];
            if constexpr (ACTION) {
#pragma unroll
                for (int j = 0; j < NL; ++j) loc[j] = 0.0;
                double G[Geo<D>::NM], kc[D + 1];
                const double adet = Geo<D>::metric(cin.x, G);
#pragma unroll
                for (int m = 0; m <= D; ++m) kc[m] = a.cstiff * cin.k[m];
                if constexpr (ActCfg<D, K>::QUAD) T::act_q(kc, G, a.cmass * adet, xl, loc);
                else T::act_t(kc, G, a.cmass * adet, xl, loc);
            } else {
                T::vec(cin.k, Geo<D>::absdet(cin.x), loc);
            }
#pragma unroll
            for (int j = 0; j < NL; ++j) vk[(cs + tid) * NL + j] = loc[j];
        }
        if (PRE && cs + WG + tid < nc) fetch(cs + WG + tid);
    }
    // the rows' first entries are fetched only now, so that they hold no
    // registers while the cells are evaluated (one round trip: the ranges
    // have arrived)
    uint32_t pe[KR][VPRE];
    double acc[KR];
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        acc[k] = 0.0;
#pragma unroll
        for (int m = 0; m < VPRE; ++m) pe[k][m] = cur[k] + m < end[k] ? a.ent[cur[k] + m] : 0u;
    }
    lds_barrier();
    // every row sums its cells' local values in ascending cell order
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        while (cur[k] < end[k]) {
            if constexpr (K >= 2) {
                // straight-line batch: all its LDS reads first (entries past
                // the row's end read slot 0 or repeat the row's last entry),
                // the next batch's entries only if the row goes on, then the
                // adds in order, each kept or dropped by a select.  Left to
                // itself the compiler put each add behind a branch and waited
                // for each LDS read in turn (P2 tetrahedra: vector 71 -> 56 us,
                // action 131 -> 115 us; P1 rows are short and lost 2-3%).
                double v[VPRE];
#pragma unroll
                for (int m = 0; m < VPRE; ++m)
                    v[m] = vk[(int)(pe[k][m] >> LB) * NL + (int)(pe[k][m] & ((1u << LB) - 1))];
                if (cur[k] + VPRE < end[k]) {
                    const int last = end[k] - 1;
#pragma unroll
                    for (int m = 0; m < VPRE; ++m) pe[k][m] = a.ent[min(cur[k] + VPRE + m, last)];
                }
#pragma unroll
                for (int m = 0; m < VPRE; ++m) {
                    double sm = acc[k] + v[m];
                    asm volatile("" : "+v"(sm));   // formed here, not inside a branch
                    acc[k] = cur[k] + m < end[k] ? sm : acc[k];
                }
                cur[k] += VPRE;
            } else {
#pragma unroll
                for (int m = 0; m < VPRE; ++m)
                    if (cur[k] + m < end[k])
                        acc[k] += vk[(int)(pe[k][m] >> LB) * NL + (int)(pe[k][m] & ((1u << LB) - 1))];
                cur[k] += VPRE;
#pragma unroll
                for (int m = 0; m < VPRE; ++m) pe[k][m] = cur[k] + m < end[k] ? a.ent[cur[k] + m] : 0u;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        const int r = r0 + tid + WG * k;
        if (r < r1) a.out[r] = a.inc ? a.out[r] + acc[k] : acc[k];
    }
}

// One workgroup per row block.
template <int D, int K, bool ACTION>
__global__ __launch_bounds__((VecWG<D, K, ACTION>::WG)) void k_assemble_vec(KArgs a)
{
    vec_block<D, K, ACTION>(a, blockIdx.x);
}

template <int D, int K>
hipError_t mat_dispatch(const AsmArgs &a, hipStream_t s)
{
    const int nblk = a.plan->nblk;
    const int grid = std::min(nblk, std::max(a.num_cus, 1));
    hipLaunchKernelGGL((k_assemble_mat<D, K>), dim3(grid), dim3(MatCfg<D, K>::WG), 0, s, kargs(a), nblk);
    return hipGetLastError();
}

}  // namespace

bool limits(int dim, int degree, bool is_mat, Limits *out)
{
    const int nloc = dim == 2 ? (degree + 1) * (degree + 2) / 2
                              : (degree + 1) * (degree + 2) * (degree + 3) / 6;
    const int lb = lbits_for(nloc);
    out->slot_cap = 0;
    out->lanes = 0;
    out->ne = nloc * (nloc + 1) / 2;
#define FEM_LIM(D, K)                                                             \
    if (dim == D && degree == K) {                                                \
        if (is_mat) {                                                             \
            out->rows_per_block = MatLds<D, K>::SCAP;                             \
            out->slot_cap = MatLds<D, K>::SCAP;                                   \
            out->cell_cap = MatLds<D, K>::CCH * MatCfg<D, K>::MCH;                \
            out->chunk_cells = MatLds<D, K>::CCH;                                 \
            out->lanes = MatCfg<D, K>::WG;                                        \
        } else {                                                                  \
            out->rows_per_block = VROWS;                                          \
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
    hipLaunchKernelGGL((k_assemble_vec<D, K, false>), dim3(a.plan->nblk), dim3(VecWG<D, K, false>::WG), 0, s, kargs(a));
    return hipGetLastError();
}
template <int D, int K>
hipError_t action_dispatch(const AsmArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL((k_assemble_vec<D, K, true>), dim3(a.plan->nblk), dim3(VecWG<D, K, true>::WG), 0, s, kargs(a));
    return hipGetLastError();
}
// ---------------------------------------------------------------- batched launches

// One launch over the work of several requests whose plans share (dim,
// degree): the descriptor holds a work-item counter, the requests' first
// work items (prefix sums) and block counts, then their arguments.  Every
// workgroup takes the next work item from the counter until none is left (so
// every wave leaves the loop), finds its request and runs that request's
// blocks with the same code as the single-request kernels: a block's
// values do not depend on what else is in the launch.
struct BatchHdr {
    int32_t counter, nreq, bpi, total;
};

__device__ __forceinline__ int batch_item(BatchHdr *hdr, int &it)
{
    __shared__ int s_it;
    __syncthreads();                       // the previous item's LDS reads are done
    if (threadIdx.x == 0) s_it = atomicAdd(&hdr->counter, 1);
    __syncthreads();
    it = __builtin_amdgcn_readfirstlane(s_it);
    return it < ldc(&hdr->total);
}

// A request's arguments through scalar loads (the index is uniform).
__device__ __forceinline__ KArgs load_kargs(const KArgs *p)
{
    static_assert(sizeof(KArgs) % 8 == 0, "KArgs in 8-byte words");
    KArgs k;
    uint64_t *d = reinterpret_cast<uint64_t *>(&k);
    const uint64_t *src = reinterpret_cast<const uint64_t *>(p);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(KArgs) / 8); ++i) d[i] = ldc(src + i);
    return k;
}

__device__ __forceinline__ int batch_request(const int32_t *prefix, int it)
{
    int r = 0;
    while (ldc(prefix + r + 1) <= it) ++r;
    return r;
}

template <int D, int K>
__global__ __launch_bounds__((MatCfg<D, K>::WG)) void k_mat_batch(BatchHdr *hdr, const int32_t *prefix,
                                                                   const int32_t *nblk, const KArgs *reqs)
{
    const int bpi = ldc(&hdr->bpi);
    int it;
    while (batch_item(hdr, it)) {
        const int r = batch_request(prefix, it);
        const KArgs a = load_kargs(reqs + r);
        const int bb = (it - ldc(prefix + r)) * bpi;
        const int be = min(bb + bpi, ldc(nblk + r));
        mat_blocks<D, K>(a, bb, be);
    }
}

template <int D, int K, bool ACTION>
__global__ __launch_bounds__((VecWG<D, K, ACTION>::WG)) void k_vec_batch(BatchHdr *hdr, const int32_t *prefix,
                                                                          const KArgs *reqs)
{
    int it;
    while (batch_item(hdr, it)) {
        const int r = batch_request(prefix, it);
        const KArgs a = load_kargs(reqs + r);
        vec_block<D, K, ACTION>(a, it - ldc(prefix + r));
    }
}

constexpr int BATCH_BPI = 8;   // Mat blocks per work item (pipelined within the item)

struct BatchLayout {
    size_t prefix, nblk, reqs, bytes;
    explicit BatchLayout(int nreq)
    {
        prefix = 256;
        nblk = prefix + ((size_t)(nreq + 1) * 4 + 15) / 16 * 16;
        reqs = nblk + ((size_t)nreq * 4 + 15) / 16 * 16;
        bytes = (reqs + (size_t)nreq * sizeof(KArgs) + 255) / 256 * 256;
    }
};

template <int D, int K>
hipError_t batch_dispatch(int op, int grid, char *desc, const BatchLayout &L, int total, hipStream_t s)
{
    BatchHdr *hdr = reinterpret_cast<BatchHdr *>(desc);
    const int32_t *prefix = reinterpret_cast<const int32_t *>(desc + L.prefix);
    const int32_t *nblk = reinterpret_cast<const int32_t *>(desc + L.nblk);
    const KArgs *reqs = reinterpret_cast<const KArgs *>(desc + L.reqs);
    if (op == 0) {
        hipLaunchKernelGGL((k_mat_batch<D, K>), dim3(std::min(grid, total)), dim3(MatCfg<D, K>::WG), 0, s, hdr,
                           prefix, nblk, reqs);
    } else if (op == 1) {
        hipLaunchKernelGGL((k_vec_batch<D, K, false>), dim3(std::min(2 * grid, total)),
                           dim3(VecWG<D, K, false>::WG), 0, s, hdr, prefix, reqs);
    } else {
        hipLaunchKernelGGL((k_vec_batch<D, K, true>), dim3(std::min(2 * grid, total)),
                           dim3(VecWG<D, K, true>::WG), 0, s, hdr, prefix, reqs);
    }
    return hipGetLastError();
}

}  // namespace

size_t batch_desc_bytes(int nreq) { return BatchLayout(nreq).bytes; }

hipError_t launch_batch(int op, const AsmArgs *reqs, int nreq, int grid, void *hdesc, void *desc, hipStream_t s)
{
    if (nreq <= 0) return hipSuccess;
    const fem_plan &p0 = *reqs[0].plan;
    for (int r = 0; r < nreq; ++r)
        if (reqs[r].plan->dim != p0.dim || reqs[r].plan->degree != p0.degree || reqs[r].plan->is_mat != (op == 0))
            return hipErrorInvalidValue;
    const BatchLayout L(nreq);
    char *h = static_cast<char *>(hdesc);
    std::fill(h, h + L.bytes, 0);
    BatchHdr *hdr = reinterpret_cast<BatchHdr *>(h);
    int32_t *prefix = reinterpret_cast<int32_t *>(h + L.prefix);
    int32_t *nblk = reinterpret_cast<int32_t *>(h + L.nblk);
    KArgs *ka = reinterpret_cast<KArgs *>(h + L.reqs);
    const int bpi = op == 0 ? BATCH_BPI : 1;
    prefix[0] = 0;
    for (int r = 0; r < nreq; ++r) {
        nblk[r] = reqs[r].plan->nblk;
        prefix[r + 1] = prefix[r] + (nblk[r] + bpi - 1) / bpi;
        ka[r] = kargs(reqs[r]);
    }
    hdr->counter = 0;
    hdr->nreq = nreq;
    hdr->bpi = bpi;
    hdr->total = prefix[nreq];
    if (hdr->total == 0) return hipSuccess;
    hipError_t e = hipMemcpyAsync(desc, hdesc, L.bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    const int total = hdr->total;
    char *d = static_cast<char *>(desc);
    switch (p0.dim * 10 + p0.degree) {
    case 21: return batch_dispatch<2, 1>(op, grid, d, L, total, s);
    case 22: return batch_dispatch<2, 2>(op, grid, d, L, total, s);
    case 23: return batch_dispatch<2, 3>(op, grid, d, L, total, s);
    case 31: return batch_dispatch<3, 1>(op, grid, d, L, total, s);
    case 32: return batch_dispatch<3, 2>(op, grid, d, L, total, s);
    case 33: return batch_dispatch<3, 3>(op, grid, d, L, total, s);
    default: return hipErrorInvalidValue;
    }
}

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
