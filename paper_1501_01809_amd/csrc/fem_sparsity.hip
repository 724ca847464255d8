// Incidence, sparsity and position kernels of the cell-loop assembler (gfx950).
//
// The sparsity of a Mat assembled through a row Map and a column Map is the
// union, over the cells incident to each row, of the cells' columns
// (PyOP2 builds this from the pair of Maps; "Matrix arguments").  Rows are
// processed independently: one wavefront gathers the candidate columns of a
// row into LDS and ranks the first occurrence of each value, which yields
// both the row's length (count pass) and its sorted unique columns (fill
// pass) without a global sort.  Everything is deterministic: atomics are used
// only for counting and for bucketing, and every bucket is sorted afterwards.
#include "fem_internal.h"

#include <mutex>

// Scratch of fem_build_sparsity_noalloc: a fixed array in every device's
// global memory, held for the life of the process.  Host code never uses
// the array's name as an address: static_scratch() looks its device address
// up once per device.
constexpr size_t FEM_STATIC_SCRATCH_BYTES = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[FEM_STATIC_SCRATCH_BYTES];

namespace femk {
namespace {

constexpr int SCAN_T = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_T * SCAN_ITEMS;

__global__ void k_check_range(const int32_t *__restrict__ v, int64_t n, int64_t limit,
                              int *__restrict__ flag)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t x = v[i];
        if (x < 0 || x >= limit) atomicOr(flag, 1);
    }
}

__global__ void k_fill_value(int32_t *__restrict__ p, int64_t n, int32_t value)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void k_count(const int32_t *__restrict__ map, int64_t n, int32_t *__restrict__ cnt)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[map[i]], 1);
}

__global__ void k_fill(const int32_t *__restrict__ map, int64_t n, int32_t *__restrict__ cursor,
                       int32_t *__restrict__ ent)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t p = atomicAdd(&cursor[map[i]], 1);
        ent[p] = (int32_t)i;
    }
}

// Insertion sort of each row's entry ids: makes the bucket order canonical
// (ascending cell, then local index).
__global__ void k_sort_rows(const int64_t *__restrict__ ptr, int32_t *__restrict__ ent, int64_t nrows)
{
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nrows;
         r += (int64_t)gridDim.x * blockDim.x) {
        int64_t a = ptr[r], b = ptr[r + 1];
        for (int64_t i = a + 1; i < b; ++i) {
            int32_t key = ent[i];
            int64_t j = i - 1;
            while (j >= a && ent[j] > key) { ent[j + 1] = ent[j]; --j; }
            ent[j + 1] = key;
        }
    }
}

__global__ void k_i64_to_i32(const int64_t *__restrict__ in, int32_t *__restrict__ out, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (int32_t)in[i];
}

// Block-wide exclusive scan of one int64 per thread (Hillis-Steele in LDS).
__device__ int64_t block_exclusive_scan(int64_t v, int64_t *total)
{
    __shared__ int64_t s[SCAN_T];
    const int t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
        int64_t add = t >= off ? s[t - off] : 0;
        __syncthreads();
        s[t] += add;
        __syncthreads();
    }
    int64_t incl = s[t];
    *total = s[SCAN_T - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_tiles(const int32_t *__restrict__ in, int64_t n,
                                                       int64_t *__restrict__ tile_sum)
{
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int64_t s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + (int64_t)k * SCAN_T + threadIdx.x;
        if (i < n) s += in[i];
    }
    int64_t tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_sums(int64_t *__restrict__ tile_sum, int64_t ntiles,
                                                      int64_t *__restrict__ out_total)
{
    int64_t carry = 0;
    for (int64_t base = 0; base < ntiles; base += SCAN_T) {
        int64_t i = base + threadIdx.x;
        int64_t v = i < ntiles ? tile_sum[i] : 0;
        int64_t tot;
        int64_t ex = block_exclusive_scan(v, &tot);
        if (i < ntiles) tile_sum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *out_total = carry;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_apply(const int32_t *__restrict__ in, int64_t n,
                                                       const int64_t *__restrict__ tile_sum,
                                                       int64_t *__restrict__ out)
{
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int64_t v[SCAN_ITEMS];
    int64_t s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + k;
        v[k] = i < n ? in[i] : 0;
        s += v[k];
    }
    int64_t tot;
    int64_t ex = block_exclusive_scan(s, &tot) + tile_sum[blockIdx.x];
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = ex;
        ex += v[k];
    }
}

constexpr int RC_CAP = 2048;   // candidate columns of one row held in LDS
constexpr int HBITS = 13, HCAP = 1 << HBITS;   // distinct columns of one long row (LDS hash set)

// One 64-lane workgroup per row (grid-stride).  Candidates = columns of every
// incident cell; a candidate is "first" if no equal value precedes it; the
// rank of a first candidate among first candidates with smaller value is its
// position in the sorted unique row.
__global__ __launch_bounds__(64) void k_row_columns(
    const int64_t *__restrict__ inc_ptr, const int32_t *__restrict__ inc_ent, int nloc_r,
    const int32_t *__restrict__ cmap, int nloc_c, int64_t nrows, int32_t *__restrict__ counts,
    const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col_idx, int *__restrict__ overflow)
{
    __shared__ int32_t cand[RC_CAP];
    __shared__ uint8_t first[RC_CAP];
    const int t0 = threadIdx.x;
    for (int64_t r = blockIdx.x; r < nrows; r += gridDim.x) {
        const int64_t e0 = inc_ptr[r], e1 = inc_ptr[r + 1];
        const int64_t n64 = (e1 - e0) * nloc_c;
        if (n64 > RC_CAP) continue;   // a long row: k_row_columns_long
        const int n = (int)n64;
        for (int t = t0; t < n; t += 64) {
            int64_t e = inc_ent[e0 + t / nloc_c];
            int64_t c = e / nloc_r;
            cand[t] = cmap[c * nloc_c + t % nloc_c];
        }
        __syncthreads();
        int mine = 0;
        for (int t = t0; t < n; t += 64) {
            const int32_t v = cand[t];
            uint8_t f = 1;
            for (int u = 0; u < t; ++u)
                if (cand[u] == v) { f = 0; break; }
            first[t] = f;
            mine += f;
        }
        __syncthreads();
        if (!col_idx) {
            for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off);
            if (t0 == 0) counts[r] = mine;
        } else {
            const int64_t base = row_ptr[r];
            for (int t = t0; t < n; t += 64) {
                if (!first[t]) continue;
                const int32_t v = cand[t];
                int rank = 0;
                for (int u = 0; u < n; ++u) rank += (first[u] && cand[u] < v);
                col_idx[base + rank] = v;
            }
        }
        __syncthreads();
    }
}

// Rows with more than RC_CAP candidates (high-valence vertices).  64-lane
// workgroups walk groups of 64 rows: the lanes find the long rows among them,
// then take each long row together: its candidates go into an LDS hash set
// (open addressing, at most HCAP distinct columns, else *overflow), and each
// distinct column's rank among the set is its position in the sorted row.
// The result does not depend on the insertion order.
__global__ __launch_bounds__(64) void k_row_columns_long(
    const int64_t *__restrict__ inc_ptr, const int32_t *__restrict__ inc_ent, int nloc_r,
    const int32_t *__restrict__ cmap, int nloc_c, int64_t nrows, int32_t *__restrict__ counts,
    const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col_idx, int *__restrict__ overflow)
{
    __shared__ int32_t tab[HCAP];
    __shared__ int32_t nu;
    const int lane = threadIdx.x;
    for (int64_t r0 = (int64_t)blockIdx.x * 64; r0 < nrows; r0 += (int64_t)gridDim.x * 64) {
        const int64_t my = r0 + lane;
        const bool is_long = my < nrows && (inc_ptr[my + 1] - inc_ptr[my]) * nloc_c > RC_CAP;
        uint64_t pending = __ballot(is_long);
        while (pending) {
            const int j = __ffsll((unsigned long long)pending) - 1;
            pending &= pending - 1;
            const int64_t r = r0 + j;
            for (int i = lane; i < HCAP; i += 64) tab[i] = -1;
            if (lane == 0) nu = 0;
            __syncthreads();
            const int64_t e0 = inc_ptr[r], n = (inc_ptr[r + 1] - e0) * nloc_c;
            int full = 0;
            for (int64_t t = lane; t < n && !full; t += 64) {
                const int64_t e = inc_ent[e0 + t / nloc_c];
                const int32_t v = cmap[(e / nloc_r) * nloc_c + t % nloc_c];
                uint32_t h = ((uint32_t)v * 2654435761u) >> (32 - HBITS);   // Knuth's multiplicative hash
                for (int probe = 0;; ++probe) {
                    if (probe == HCAP) { full = 1; break; }
                    const int32_t old = atomicCAS(&tab[h], -1, v);
                    if (old == -1) { atomicAdd(&nu, 1); break; }
                    if (old == v) break;
                    h = (h + 1) & (HCAP - 1);
                }
            }
            __syncthreads();
            if (__ballot(full) != 0) {   // (one wave: uniform)
                if (lane == 0) atomicOr(overflow, 1);
                continue;                // the next long row clears the table first
            }
            if (!col_idx) {
                if (lane == 0) counts[r] = nu;
            } else {
                const int64_t base = row_ptr[r];
                for (int i = lane; i < HCAP; i += 64) {
                    const int32_t v = tab[i];
                    if (v < 0) continue;
                    int rank = 0;
                    for (int k = 0; k < HCAP; ++k) rank += (uint32_t)tab[k] < (uint32_t)v;
                    col_idx[base + rank] = v;
                }
            }
            __syncthreads();
        }
    }
}

inline int grid_for(int64_t n, int threads)
{
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

}  // namespace

hipError_t check_range(const int32_t *v, int64_t n, int64_t limit, int *flag, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_range, dim3(grid_for(n, 256)), dim3(256), 0, s, v, n, limit, flag);
    return hipGetLastError();
}

hipError_t static_scratch(int device, void **ptr, size_t *bytes)
{
    static std::mutex mu;
    static void *addr[64] = {};
    *ptr = nullptr;
    *bytes = 0;
    if (device < 0 || device >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = p;
    }
    *ptr = addr[device];
    *bytes = FEM_STATIC_SCRATCH_BYTES;
    return hipSuccess;
}

int64_t scan_scratch(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

hipError_t fill_i32(int32_t *p, int64_t n, int32_t value, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_value, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, value);
    return hipGetLastError();
}

hipError_t exclusive_scan(const int32_t *in, int64_t *out, int64_t n, int64_t *tile_sum, hipStream_t s)
{
    const int64_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (ntiles > 0)
        hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(SCAN_T), 0, s, in, n, tile_sum);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_T), 0, s, tile_sum, ntiles, out + n);
    if (ntiles > 0)
        hipLaunchKernelGGL(k_scan_apply, dim3(ntiles), dim3(SCAN_T), 0, s, in, n, tile_sum, out);
    return hipGetLastError();
}

hipError_t build_incidence(const int32_t *map, int64_t ncells, int nloc, int64_t nrows,
                           int64_t *ptr, int32_t *ent, int32_t *tmp, int64_t *scan, hipStream_t s)
{
    const int64_t n = ncells * nloc;
    hipError_t e = fill_i32(tmp, nrows + 1, 0, s);
    if (e != hipSuccess) return e;
    if (n > 0) hipLaunchKernelGGL(k_count, dim3(grid_for(n, 256)), dim3(256), 0, s, map, n, tmp);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = exclusive_scan(tmp, ptr, nrows, scan, s)) != hipSuccess) return e;
    if (nrows > 0)
        hipLaunchKernelGGL(k_i64_to_i32, dim3(grid_for(nrows, 256)), dim3(256), 0, s, ptr, tmp, nrows);
    if (n > 0) hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256)), dim3(256), 0, s, map, n, tmp, ent);
    if (nrows > 0)
        hipLaunchKernelGGL(k_sort_rows, dim3(grid_for(nrows, 128)), dim3(128), 0, s, ptr, ent, nrows);
    return hipGetLastError();
}

hipError_t row_columns(const int64_t *inc_ptr, const int32_t *inc_ent, int nloc_r,
                       const int32_t *cmap, int nloc_c, int64_t nrows, int32_t *counts,
                       const int64_t *row_ptr, int32_t *col_idx, int *overflow, hipStream_t s)
{
    if (nrows <= 0) return hipSuccess;
    int64_t g = nrows < 32768 ? nrows : 32768;
    hipLaunchKernelGGL(k_row_columns, dim3((unsigned)g), dim3(64), 0, s, inc_ptr, inc_ent, nloc_r,
                       cmap, nloc_c, nrows, counts, row_ptr, col_idx, overflow);
    const int64_t gl = std::min<int64_t>((nrows + 63) / 64, 4096);
    hipLaunchKernelGGL(k_row_columns_long, dim3((unsigned)gl), dim3(64), 0, s, inc_ptr, inc_ent,
                       nloc_r, cmap, nloc_c, nrows, counts, row_ptr, col_idx, overflow);
    return hipGetLastError();
}

hipError_t i64_to_i32(const int64_t *in, int32_t *out, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_i64_to_i32, dim3(grid_for(n, 256)), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}

}  // namespace femk
