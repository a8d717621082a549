// Cell binning (Sec. 2.1: "for each cell, the set of particles inside is
// known ... achieved in an O(N) procedure"): a counting sort by cell.
//   k_bin_count   cell of each particle, per-cell counts (int atomics) and the
//                 particle's slot inside its cell
//   k_bin_scan    exclusive scan of the counts -> cell_start, resets the counts
//                 for the next call, lists cells above the dense threshold
//                 (meshes up to 16^3 skip it: each scatter block scans the
//                 counts itself and the P2M kernel resets them)
//   k_bin_scatter sorted structure-of-arrays record (offset from the cell
//                 centre in cell units, charge), permutation and cell of each
//                 sorted slot
// Cell index: I = floor(r n / b) per axis, clamped to [0, n-1]; periodic
// positions are first wrapped into the box (in cell units).
//
// Batches: blockIdx.y selects one of several independent systems on meshes of
// the same size; prange[2s], prange[2s+1] bound system s's particles in the
// caller's arrays (null: one system, particles [0, n)), and its cell arrays
// sit at fixed strides (count K, start K + 1, dense list K, small 8).
#include "pmmm_internal.h"

namespace pmmm {

template <typename T>
__device__ __forceinline__ void cell_coord(T v, T inv_h, int n, int periodic, int &ic, T &u,
                                           int &outside) {
    T s = v * inv_h;
    if (periodic) {
        s = s - T(n) * floor(s / T(n));
    } else if (!(s >= T(0) && s < T(n))) {
        outside = 1;
    }
    int i = (int)floor(s);
    i = i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
    ic = i;
    u = s - T(i) - T(0.5);
}

template <typename T>
__global__ void __launch_bounds__(256) k_bin_count(const int64_t *__restrict__ prange, int64_t n,
                                                   const T *__restrict__ x,
                                                   const T *__restrict__ y,
                                                   const T *__restrict__ z, T inv_h, int nc,
                                                   int periodic, int *__restrict__ cell_of,
                                                   int *__restrict__ slot,
                                                   int *__restrict__ count,
                                                   int *__restrict__ flag) {
    int64_t p0, np;
    sys_range(prange, n, p0, np);
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= np) return;
    const int64_t i = p0 + j;
    count += (int64_t)blockIdx.y * nc * nc * nc;
    int ix, iy, iz, out = 0;
    T ux, uy, uz;
    cell_coord(x[i], inv_h, nc, periodic, ix, ux, out);
    cell_coord(y[i], inv_h, nc, periodic, iy, uy, out);
    cell_coord(z[i], inv_h, nc, periodic, iz, uz, out);
    if (out) *flag = 1;
    const int c = (iz * nc + iy) * nc + ix;
    cell_of[i] = c;
    slot[i] = atomicAdd(&count[c], 1);
}

// One workgroup of 1024 threads per system scans its K counts in tiles of 4096.
__global__ void __launch_bounds__(1024) k_bin_scan(int K, int *__restrict__ count,
                                                   int *__restrict__ start, int dense_thr,
                                                   int *__restrict__ dense_cells,
                                                   int *__restrict__ dense_count) {
    {
        const int64_t sy = blockIdx.y;
        count += sy * K;
        start += sy * (K + 1);
        dense_cells += sy * K;
        dense_count += sy * 8;
    }
    __shared__ int wtot[16];
    __shared__ int carry_s;
    __shared__ int ndense;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) {
        carry_s = 0;
        ndense = 0;
    }
    __syncthreads();
    for (int base = 0; base < K; base += 4096) {
        int v[4];
        int tot = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int idx = base + tid * 4 + j;
            v[j] = idx < K ? count[idx] : 0;
            tot += v[j];
        }
        // inclusive wave scan of thread totals
        int inc = tot;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            int t = __shfl_up(inc, off, 64);
            if (lane >= off) inc += t;
        }
        if (lane == 63) wtot[wid] = inc;
        __syncthreads();
        int wpre = 0;
        for (int w = 0; w < wid; ++w) wpre += wtot[w];
        int run = carry_s + wpre + inc - tot;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int idx = base + tid * 4 + j;
            if (idx < K) {
                start[idx] = run;
                count[idx] = 0;
                if (v[j] > dense_thr) dense_cells[atomicAdd(&ndense, 1)] = idx;
            }
            run += v[j];
        }
        __syncthreads();
        if (tid == 1023) carry_s = run;
        __syncthreads();
    }
    if (tid == 0) {
        start[K] = carry_s;
        *dense_count = ndense;
    }
}

// Exclusive scan of K <= kInBlockScanMax counts by one 256-thread block into
// LDS (s_start[0..K]); block 0 also publishes start[] and the dense list.
constexpr int kInBlockScanMax = 4096;

__device__ void block_scan_small(int K, const int *__restrict__ count, int *s_start,
                                 int publish, int *__restrict__ start, int dense_thr,
                                 int *__restrict__ dense_cells, int *__restrict__ dense_count) {
    __shared__ int wtot[4];
    __shared__ int ndense;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    constexpr int PER = kInBlockScanMax / 256;  // 16 counts per thread
    int v[PER], tot = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int idx = tid * PER + j;
        v[j] = idx < K ? count[idx] : 0;
        tot += v[j];
    }
    int inc = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(inc, off, 64);
        if (lane >= off) inc += t;
    }
    if (lane == 63) wtot[wid] = inc;
    if (tid == 0) ndense = 0;
    __syncthreads();
    int run = inc - tot;
    for (int w = 0; w < wid; ++w) run += wtot[w];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int idx = tid * PER + j;
        if (idx < K) {
            s_start[idx] = run;
            if (publish) {
                start[idx] = run;
                if (v[j] > dense_thr) dense_cells[atomicAdd(&ndense, 1)] = idx;
            }
        }
        run += v[j];
    }
    if (tid == 255) {
        s_start[K] = run;
        if (publish) start[K] = run;
    }
    __syncthreads();
    if (publish && tid == 0) *dense_count = ndense;
}

// Scatter into the sorted structure-of-arrays record.  With inblock, every
// block scans the counts itself (small meshes), else start[] comes from the
// scan kernel.
// Sorted slot g of system s is p0 + start[c] + slot: perm[g] holds the
// particle's index in the caller's arrays, scell[g] its cell.
template <typename T>
__global__ void __launch_bounds__(256) k_bin_scatter(
    const int64_t *__restrict__ prange, int64_t n, const T *__restrict__ x,
    const T *__restrict__ y, const T *__restrict__ z, const T *__restrict__ q, T inv_h, int nc,
    int periodic, const int *__restrict__ cell_of, const int *__restrict__ slot,
    int *__restrict__ start, int *__restrict__ perm, int *__restrict__ scell,
    particle4<T> *__restrict__ sorted, int inblock, const int *__restrict__ count,
    int dense_thr, int *__restrict__ dense_cells, int *__restrict__ dense_count) {
    __shared__ int s_start[kInBlockScanMax + 1];
    const int K = nc * nc * nc;
    {
        const int64_t sy = blockIdx.y;
        count += sy * K;
        start += sy * (K + 1);
        dense_cells += sy * K;
        dense_count += sy * 8;
    }
    int64_t p0, np;
    sys_range(prange, n, p0, np);
    if (inblock)
        block_scan_small(K, count, s_start, blockIdx.x == 0, start, dense_thr, dense_cells,
                         dense_count);
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= np) return;
    const int64_t i = p0 + j;
    int ix, iy, iz, out = 0;
    particle4<T> r;
    cell_coord(x[i], inv_h, nc, periodic, ix, r.ux, out);
    cell_coord(y[i], inv_h, nc, periodic, iy, r.uy, out);
    cell_coord(z[i], inv_h, nc, periodic, iz, r.uz, out);
    r.q = q != nullptr ? q[i] : T(0);
    const int c = cell_of[i];
    const int s = (inblock ? s_start[c] : start[c]) + slot[i];
    if (s < 0 || (int64_t)s >= np) return;  // only reachable with inconsistent counts
    const int64_t g = p0 + s;
    perm[g] = (int)i;
    scell[g] = c;
    sorted[g] = r;
}

template <typename T>
hipError_t launch_bin(const BinArgs &a, hipStream_t s) {
    const int K = a.ncell * a.ncell * a.ncell;
    const T inv_h = T(a.inv_h);
    const int nsys = a.nsys > 0 ? a.nsys : 1;
    const int64_t maxn = a.prange ? a.max_np : a.n;
    const int blocks = (int)((maxn + 255) / 256);
    const int inblock = K <= kInBlockScanMax ? 1 : 0;
    if (maxn > 0) {
        hipLaunchKernelGGL(k_bin_count<T>, dim3(blocks, nsys), dim3(256), 0, s, a.prange, a.n,
                           (const T *)a.x, (const T *)a.y, (const T *)a.z, inv_h, a.ncell,
                           a.periodic, a.cell_of, a.slot, a.count, a.flag);
    }
    if (!inblock || maxn == 0) {
        hipLaunchKernelGGL(k_bin_scan, dim3(1, nsys), dim3(1024), 0, s, K, a.count, a.start,
                           a.dense_threshold, a.dense_cells, a.dense_count);
    }
    if (maxn > 0) {
        hipLaunchKernelGGL(k_bin_scatter<T>, dim3(blocks, nsys), dim3(256), 0, s, a.prange, a.n,
                           (const T *)a.x, (const T *)a.y, (const T *)a.z, (const T *)a.q,
                           inv_h, a.ncell, a.periodic, a.cell_of, a.slot, a.start, a.perm,
                           a.scell, (particle4<T> *)a.sorted, inblock, a.count,
                           a.dense_threshold, a.dense_cells, a.dense_count);
    }
    return hipGetLastError();
}

template hipError_t launch_bin<float>(const BinArgs &, hipStream_t);
template hipError_t launch_bin<double>(const BinArgs &, hipStream_t);

}  // namespace pmmm
