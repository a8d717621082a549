// Cell binning (Sec. 2.1 requires that the particles of every cell be known,
// which takes linear time): a counting sort by cell.
//   k_bin_count   cell of each particle, per-cell counts (int atomics) and the
//                 particle's slot inside its cell; meshes above 16^3 count
//                 in S sub-counters per cell (particle i in sub-counter
//                 i mod S), stored sub-counter-major ([S][K], each in its own
//                 cache line), so that a cell holding a large share of the
//                 particles does not serialise all of them on one line
//   k_bin_tile_sums, k_bin_scan_tiles
//                 exclusive scan of the counts -> cell_start in tiles of 4096
//                 cells, resets the counts for the next call, lists cells above
//                 the dense threshold (meshes up to 16^3 skip it: each scatter
//                 block scans the counts itself and the P2M kernel resets them)
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
                                                   int *__restrict__ count, int logS,
                                                   int *__restrict__ flag) {
    int64_t p0, np;
    sys_range(prange, n, p0, np);
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= np) return;
    const int64_t i = p0 + j;
    count += ((int64_t)blockIdx.y * nc * nc * nc) << logS;
    // the three loads are issued together, ahead of the branches below
    const T xv = x[i], yv = y[i], zv = z[i];
    asm volatile("" ::"v"(xv), "v"(yv), "v"(zv));
    int ix, iy, iz, out = 0;
    T ux, uy, uz;
    cell_coord(xv, inv_h, nc, periodic, ix, ux, out);
    cell_coord(yv, inv_h, nc, periodic, iy, uy, out);
    cell_coord(zv, inv_h, nc, periodic, iz, uz, out);
    if (out) *flag = 1;
    const int c = (iz * nc + iy) * nc + ix;
    cell_of[i] = c;
    slot[i] = atomicAdd(&count[(int)(j & ((1 << logS) - 1)) * (nc * nc * nc) + c], 1);
}

// Four consecutive counters e .. e + 3 of the scan order (cell-major: cell
// e >> logS, sub-counter e mod S) from their sub-counter-major storage; with
// S = 1 an aligned int4.  e is a multiple of 4 and the four share one cell
// when S > 1.
__device__ __forceinline__ int4 load_counts4(const int *count, int e, int logS, int K) {
    if (logS == 0) return *(const int4 *)(count + e);
    const int c = e >> logS, sh = e & ((1 << logS) - 1);
    const int *p = count + (int64_t)sh * K + c;
    return make_int4(p[0], p[K], p[2 * K], p[3 * K]);
}
__device__ __forceinline__ void zero_counts4(int *count, int e, int logS, int K) {
    if (logS == 0) {
        *(int4 *)(count + e) = make_int4(0, 0, 0, 0);
        return;
    }
    int *p = count + (int64_t)(e & ((1 << logS) - 1)) * K + (e >> logS);
    p[0] = 0;
    p[K] = 0;
    p[2 * K] = 0;
    p[3 * K] = 0;
}

// Exclusive scan of the counts in tiles of kScanTile, one 1024-thread block
// per tile: k_bin_tile_sums adds up every tile, then k_bin_scan_tiles scans
// its tile starting from the sum of the tiles before it, resets the counts
// for the next call and lists the cells above the dense threshold (in no
// particular order: each dense cell is reduced by one block in a fixed order).
constexpr int kScanTile = 4096;

__global__ void __launch_bounds__(1024) k_bin_tile_sums(int K, int logS,
                                                        const int *__restrict__ count,
                                                        int *__restrict__ tile_sums,
                                                        int *__restrict__ dense_count) {
    const int ntiles = gridDim.x, L = K << logS;
    {
        const int64_t sy = blockIdx.y;
        count += sy * L;
        tile_sums += sy * ntiles;
        dense_count += sy * 8;
    }
    __shared__ int wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    // L = S n^3 with n >= 4 is a multiple of 64: four counters per thread
    const int idx = blockIdx.x * kScanTile + tid * 4;
    int v = 0;
    if (idx < L) {
        const int4 c4 = load_counts4(count, idx, logS, K);
        v = (c4.x + c4.y) + (c4.z + c4.w);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) wsum[wid] = v;
    __syncthreads();
    if (tid == 0) {
        int t = 0;
        for (int w = 0; w < 16; ++w) t += wsum[w];
        tile_sums[blockIdx.x] = t;
        if (blockIdx.x == 0) *dense_count = 0;
    }
}

// L = S K counters (S = 1 or kCountShards) scanned in cell-major order; with
// S > 1 sstart receives the start of every sub-counter (in that order) and
// start that of every cell (its first sub-counter), and a cell's two halves
// sit in the two lanes of an even-odd pair.
__global__ void __launch_bounds__(1024) k_bin_scan_tiles(int K, int logS, int *__restrict__ count,
                                                         const int *__restrict__ tile_sums,
                                                         int *__restrict__ start,
                                                         int *__restrict__ sstart, int dense_thr,
                                                         int *__restrict__ dense_cells,
                                                         int *__restrict__ dense_count) {
    const int ntiles = gridDim.x, t = blockIdx.x;
    const int L = K << logS;
    {
        const int64_t sy = blockIdx.y;
        count += sy * L;
        tile_sums += sy * ntiles;
        start += sy * (K + 1);
        sstart += sy * (L + 1);
        dense_cells += sy * K;
        dense_count += sy * 8;
    }
    __shared__ int wtot[16];
    __shared__ int pre_s;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int idx = t * kScanTile + tid * 4;
    int v[4] = {0, 0, 0, 0};
    if (idx < L) {
        const int4 c4 = load_counts4(count, idx, logS, K);
        v[0] = c4.x;
        v[1] = c4.y;
        v[2] = c4.z;
        v[3] = c4.w;
    }
    // sum of the tiles before this one
    int pre = 0;
    for (int k = tid; k < t; k += 1024) pre += tile_sums[k];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) pre += __shfl_xor(pre, off, 64);
    if (lane == 0) wtot[wid] = pre;
    __syncthreads();
    if (tid == 0) {
        int a = 0;
        for (int w = 0; w < 16; ++w) a += wtot[w];
        pre_s = a;
    }
    __syncthreads();
    // in-tile exclusive scan: wave scan of the thread totals, then the waves
    const int tot = (v[0] + v[1]) + (v[2] + v[3]);
    int inc = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(inc, off, 64);
        if (lane >= off) inc += u;
    }
    if (lane == 63) wtot[wid] = inc;
    __syncthreads();
    int run = pre_s + inc - tot;
    for (int w = 0; w < wid; ++w) run += wtot[w];
    if (logS == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (idx + j < L) {
                start[idx + j] = run;
                if (v[j] > dense_thr) dense_cells[atomicAdd(dense_count, 1)] = idx + j;
            }
            run += v[j];
        }
    } else {
        // kCountShards = 8 sub-counters per cell: lanes 2m and 2m + 1 hold one cell
        static_assert(kCountShards == 8, "a cell's sub-counters span one lane pair");
        const int cell_tot = tot + __shfl_xor(tot, 1, 64);
        if (idx < L && (tid & 1) == 0) {
            const int cell = idx >> logS;
            start[cell] = run;
            if (cell_tot > dense_thr) dense_cells[atomicAdd(dense_count, 1)] = cell;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (idx + j < L) sstart[idx + j] = run;
            run += v[j];
        }
    }
    if (idx < L) zero_counts4(count, idx, logS, K);
    if (t == ntiles - 1 && tid == 1023) {
        start[K] = run;
        sstart[L] = run;
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
    int *__restrict__ start, const int *__restrict__ sstart, int logS, int *__restrict__ perm,
    int *__restrict__ scell, particle4<T> *__restrict__ sorted, int inblock,
    const int *__restrict__ count, int dense_thr, int *__restrict__ dense_cells,
    int *__restrict__ dense_count, int *__restrict__ pos) {
    __shared__ int s_start[kInBlockScanMax + 1];
    const int K = nc * nc * nc;
    {
        const int64_t sy = blockIdx.y;
        count += sy * K;
        start += sy * (K + 1);
        sstart += sy * (((int64_t)K << logS) + 1);
        dense_cells += sy * K;
        dense_count += sy * 8;
    }
    int64_t p0, np;
    sys_range(prange, n, p0, np);
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // The particle's inputs are read first (clamped index, so unconditional):
    // their loads overlap those of the in-block scan.
    const int64_t i = p0 + (j < np ? j : np - 1);
    T xv = T(0), yv = T(0), zv = T(0), qv = T(0);
    int c = 0, sl = 0;
    if (np > 0) {
        const T *qp = q != nullptr ? q : x;
        xv = x[i];
        yv = y[i];
        zv = z[i];
        qv = qp[i];
        c = cell_of[i];
        sl = slot[i];
    }
    if (inblock)
        block_scan_small(K, count, s_start, blockIdx.x == 0, start, dense_thr, dense_cells,
                         dense_count);
    if (j >= np) return;
    asm volatile("" ::"v"(xv), "v"(yv), "v"(zv), "v"(qv), "v"(c), "v"(sl));
    int ix, iy, iz, out = 0;
    particle4<T> r;
    cell_coord(xv, inv_h, nc, periodic, ix, r.ux, out);
    cell_coord(yv, inv_h, nc, periodic, iy, r.uy, out);
    cell_coord(zv, inv_h, nc, periodic, iz, r.uz, out);
    r.q = q != nullptr ? qv : T(0);
    // sub-counter of the particle as in k_bin_count (sstart is start when S = 1)
    const int s =
        (inblock ? s_start[c] : sstart[(c << logS) + (int)(j & ((1 << logS) - 1))]) + sl;
    if (s < 0 || (int64_t)s >= np) return;  // only reachable with inconsistent counts
    const int64_t g = p0 + s;
    perm[g] = (int)i;
    scell[g] = c;
    sorted[g] = r;
    if (pos != nullptr) pos[i] = (int)g;
}

template <typename T>
hipError_t launch_bin(const BinArgs &a, hipStream_t s) {
    const int K = a.ncell * a.ncell * a.ncell;
    const T inv_h = T(a.inv_h);
    const int nsys = a.nsys > 0 ? a.nsys : 1;
    const int64_t maxn = a.prange ? a.max_np : a.n;
    const int blocks = (int)((maxn + 255) / 256);
    const int inblock = K <= kInBlockScanMax ? 1 : 0;
    const int logS = ilog2_shards(count_shards(K));
    int *sstart = logS ? a.sstart : a.start;
    if (logS && sstart == nullptr) return hipErrorInvalidValue;
    if (maxn > 0) {
        hipLaunchKernelGGL(k_bin_count<T>, dim3(blocks, nsys), dim3(256), 0, s, a.prange, a.n,
                           (const T *)a.x, (const T *)a.y, (const T *)a.z, inv_h, a.ncell,
                           a.periodic, a.cell_of, a.slot, a.count, logS, a.flag);
    }
    if (!inblock || maxn == 0) {
        const int ntiles = scan_tiles((int64_t)K << logS);
        hipLaunchKernelGGL(k_bin_tile_sums, dim3(ntiles, nsys), dim3(1024), 0, s, K, logS,
                           a.count, a.tile_sums, a.dense_count);
        hipLaunchKernelGGL(k_bin_scan_tiles, dim3(ntiles, nsys), dim3(1024), 0, s, K, logS,
                           a.count, a.tile_sums, a.start, sstart, a.dense_threshold,
                           a.dense_cells, a.dense_count);
    }
    if (maxn > 0) {
        hipLaunchKernelGGL(k_bin_scatter<T>, dim3(blocks, nsys), dim3(256), 0, s, a.prange, a.n,
                           (const T *)a.x, (const T *)a.y, (const T *)a.z, (const T *)a.q,
                           inv_h, a.ncell, a.periodic, a.cell_of, a.slot, a.start, sstart, logS,
                           a.perm, a.scell, (particle4<T> *)a.sorted, inblock, a.count,
                           a.dense_threshold, a.dense_cells, a.dense_count, a.pos);
    }
    return hipGetLastError();
}

template hipError_t launch_bin<float>(const BinArgs &, hipStream_t);
template hipError_t launch_bin<double>(const BinArgs &, hipStream_t);

}  // namespace pmmm
