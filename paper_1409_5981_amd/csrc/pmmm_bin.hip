// Cell binning (Sec. 2.1 requires that the particles of every cell be known,
// which takes linear time): a stable sort of the particles by cell index, as
// a least-significant-digit radix sort with digits of at most 9 bits, so the
// particles of a cell keep the caller's order and every result is bitwise
// reproducible (no atomics decide an order).
//   k_rb_keys     cell of each particle (keys) and its index (values) in
//                 tiles of 4096, and the tile histogram of the first digit
//   k_rb_hist     tile histogram of a later digit
//   k_rb_scan_sums, k_rb_scan
//                 exclusive scan of the histograms in bucket-major order (so
//                 tile t's bucket-d elements start after every smaller digit
//                 and after bucket d of the tiles before t)
//   k_rb_scatter  stable scatter of one digit: in rounds of 1024 elements,
//                 ranks among equal digits from wave ballots plus the counts
//                 of the earlier waves and rounds of the tile; the last
//                 digit's pass writes the sorted cell, the permutation, the
//                 sorted record (offset from the cell centre in cell units,
//                 charge) and, on request, each particle's sorted slot
//   k_rb_bounds   start of every cell by binary search in the sorted cells,
//                 and the list of cells above the dense threshold
// Cell index: I = floor(r n / b) per axis, clamped to [0, n-1]; periodic
// positions are first wrapped into the box (in cell units).
//
// Batches: blockIdx.y selects one of several independent systems on meshes of
// the same size; prange[2s], prange[2s+1] bound system s's particles in the
// caller's arrays (null: one system, particles [0, n)), and its per-system
// arrays sit at fixed strides (start K + 1, dense list K, small 8,
// histograms bin_hist_ints(max_np), scan sums bin_scan_tiles(max_np)).
#include "pmmm_internal.h"

namespace pmmm {

constexpr int kRadixTile = 4096;   // elements per tile (1024 threads x 4 rounds)
constexpr int kRadixMaxBits = 9;   // bucket count per pass at most 512
constexpr int kRadixBuckets = 1 << kRadixMaxBits;

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

__device__ __forceinline__ void sys_offsets(int64_t hist_ints, int64_t &hoff) {
    hoff = (int64_t)blockIdx.y * hist_ints;
}

__global__ void k_rb_reset_dense(int nsys, int *__restrict__ dense_count) {
    for (int sy = threadIdx.x; sy < nsys; sy += blockDim.x) dense_count[(int64_t)sy * 8] = 0;
}

// Tile histogram of digit (key >> shift) & (2^bits - 1) into LDS, written to
// hist[d * tiles + t] (every block writes all 2^bits of its entries).
__device__ __forceinline__ void write_tile_hist(int *s_hist, int nb, int *__restrict__ hist,
                                                int tiles, int t) {
    __syncthreads();
    for (int d = threadIdx.x; d < nb; d += blockDim.x) hist[(int64_t)d * tiles + t] = s_hist[d];
}

template <typename T>
__global__ void __launch_bounds__(1024) k_rb_keys(const int64_t *__restrict__ prange, int64_t n,
                                                  const T *__restrict__ x, const T *__restrict__ y,
                                                  const T *__restrict__ z, T inv_h, int nc,
                                                  int periodic, int *__restrict__ keys,
                                                  int *__restrict__ vals, int *__restrict__ hist,
                                                  int64_t hist_ints, int tiles, int bits,
                                                  int *__restrict__ flag,
                                                  int *__restrict__ dense_count) {
    __shared__ int s_hist[kRadixBuckets];
    int64_t p0, np;
    sys_range(prange, n, p0, np);
    const int nb = 1 << bits, t = blockIdx.x;
    for (int d = threadIdx.x; d < nb; d += blockDim.x) s_hist[d] = 0;
    if (t == 0 && threadIdx.x == 0) dense_count[(int64_t)blockIdx.y * 8] = 0;
    __syncthreads();
    // the loads of the four rounds are issued together
    T xv[4], yv[4], zv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t j = (int64_t)t * kRadixTile + r * 1024 + threadIdx.x;
        const int64_t i = p0 + (j < np ? j : (np > 0 ? np - 1 : 0));
        xv[r] = np > 0 ? x[i] : T(0);
        yv[r] = np > 0 ? y[i] : T(0);
        zv[r] = np > 0 ? z[i] : T(0);
    }
    int out = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t j = (int64_t)t * kRadixTile + r * 1024 + threadIdx.x;
        if (j >= np) continue;
        int ix, iy, iz;
        T ux, uy, uz;
        cell_coord(xv[r], inv_h, nc, periodic, ix, ux, out);
        cell_coord(yv[r], inv_h, nc, periodic, iy, uy, out);
        cell_coord(zv[r], inv_h, nc, periodic, iz, uz, out);
        const int c = (iz * nc + iy) * nc + ix;
        keys[p0 + j] = c;
        vals[p0 + j] = (int)(p0 + j);
        atomicAdd(&s_hist[c & (nb - 1)], 1);
    }
    if (out) *flag = 1;
    int64_t hoff;
    sys_offsets(hist_ints, hoff);
    write_tile_hist(s_hist, nb, hist + hoff, tiles, t);
}

__global__ void __launch_bounds__(1024) k_rb_hist(const int64_t *__restrict__ prange, int64_t n,
                                                  const int *__restrict__ keys,
                                                  int *__restrict__ hist, int64_t hist_ints,
                                                  int tiles, int shift, int bits) {
    __shared__ int s_hist[kRadixBuckets];
    int64_t p0, np;
    sys_range(prange, n, p0, np);
    const int nb = 1 << bits, t = blockIdx.x;
    for (int d = threadIdx.x; d < nb; d += blockDim.x) s_hist[d] = 0;
    __syncthreads();
    int kv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t j = (int64_t)t * kRadixTile + r * 1024 + threadIdx.x;
        kv[r] = j < np ? keys[p0 + j] : -1;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (kv[r] >= 0) atomicAdd(&s_hist[(kv[r] >> shift) & (nb - 1)], 1);
    int64_t hoff;
    sys_offsets(hist_ints, hoff);
    write_tile_hist(s_hist, nb, hist + hoff, tiles, t);
}

// Exclusive scan of the L = buckets x tiles histogram entries of every
// system, in place, in scan tiles of 4096: per-tile sums, then each tile
// scanned from the sum of the tiles before it.
__global__ void __launch_bounds__(1024) k_rb_scan_sums(int64_t L, int64_t hist_ints,
                                                       const int *__restrict__ hist,
                                                       int *__restrict__ sums) {
    __shared__ int wsum[16];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    hist += (int64_t)blockIdx.y * hist_ints;
    sums += (int64_t)blockIdx.y * gridDim.x;
    const int64_t base = (int64_t)blockIdx.x * 4096 + tid * 4;
    int v = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (base + k < L) v += hist[base + k];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) wsum[wid] = v;
    __syncthreads();
    if (tid == 0) {
        int a = 0;
        for (int w = 0; w < 16; ++w) a += wsum[w];
        sums[blockIdx.x] = a;
    }
}

__global__ void __launch_bounds__(1024) k_rb_scan(int64_t L, int64_t hist_ints,
                                                  int *__restrict__ hist,
                                                  const int *__restrict__ sums) {
    __shared__ int wtot[16];
    __shared__ int pre_s;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    hist += (int64_t)blockIdx.y * hist_ints;
    sums += (int64_t)blockIdx.y * gridDim.x;
    const int64_t base = (int64_t)blockIdx.x * 4096 + tid * 4;
    int v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = base + k < L ? hist[base + k] : 0;
    int pre = 0;
    for (int k = tid; k < (int)blockIdx.x; k += 1024) pre += sums[k];
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
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (base + k < L) hist[base + k] = run;
        run += v[k];
    }
}

// Stable scatter of one digit.  LDS: per-wave digit counts and their
// exclusive prefixes over the waves of a round, and the tile's running count
// per digit.  With `last`, the outputs are the sorted cell (keys_out), the
// permutation (vals_out), the sorted records and, if pos is not null, each
// particle's sorted slot.
template <typename T>
__global__ void __launch_bounds__(1024) k_rb_scatter(
    const int64_t *__restrict__ prange, int64_t n, const int *__restrict__ keys_in,
    const int *__restrict__ vals_in, int *__restrict__ keys_out, int *__restrict__ vals_out,
    const int *__restrict__ offs, int64_t hist_ints, int tiles, int shift, int bits, int last,
    const T *__restrict__ x, const T *__restrict__ y, const T *__restrict__ z,
    const T *__restrict__ q, T inv_h, int nc, int periodic, particle4<T> *__restrict__ sorted,
    int *__restrict__ pos) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int nb = 1 << bits;
    int *cnt = (int *)lds_raw;        // [16][nb] counts of the round
    int *pre = cnt + 16 * nb;         // [16][nb] exclusive prefixes over waves
    int *run = pre + 16 * nb;         // [nb] tile running count
    int64_t p0, np;
    sys_range(prange, n, p0, np);
    const int t = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    offs += (int64_t)blockIdx.y * hist_ints;
    for (int e = tid; e < 16 * nb; e += 1024) cnt[e] = 0;
    for (int d = tid; d < nb; d += 1024) run[d] = 0;
    int kv[4], vv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t j = (int64_t)t * kRadixTile + r * 1024 + tid;
        const bool act = j < np;
        kv[r] = act ? keys_in[p0 + j] : 0;
        vv[r] = act ? vals_in[p0 + j] : 0;
    }
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll 1
    for (int r = 0; r < 4; ++r) {
        const int64_t j = (int64_t)t * kRadixTile + r * 1024 + tid;
        const bool act = j < np;
        const int d = (kv[r] >> shift) & (nb - 1);
        // lanes of this wave holding the same digit (active lanes only)
        uint64_t peers = __ballot(act);
        for (int b = 0; b < bits; ++b) {
            const uint64_t m = __ballot(act && ((d >> b) & 1));
            peers &= ((d >> b) & 1) ? m : ~m;
        }
        const int rw = __popcll(peers & lt);
        if (act && rw == 0) cnt[wid * nb + d] = __popcll(peers);
        __syncthreads();
        for (int dd = tid; dd < nb; dd += 1024) {
            int s = run[dd];
#pragma unroll
            for (int w = 0; w < 16; ++w) {
                const int c = cnt[w * nb + dd];
                pre[w * nb + dd] = s;
                cnt[w * nb + dd] = 0;
                s += c;
            }
            run[dd] = s;
        }
        __syncthreads();
        if (act) {
            const int dest = offs[(int64_t)d * tiles + t] + pre[wid * nb + d] + rw;
            const int64_t g = p0 + dest;
            if (!last) {
                keys_out[g] = kv[r];
                vals_out[g] = vv[r];
            } else {
                const int i = vv[r];
                int ix, iy, iz, out = 0;
                particle4<T> rec;
                cell_coord(x[i], inv_h, nc, periodic, ix, rec.ux, out);
                cell_coord(y[i], inv_h, nc, periodic, iy, rec.uy, out);
                cell_coord(z[i], inv_h, nc, periodic, iz, rec.uz, out);
                rec.q = q != nullptr ? q[i] : T(0);
                keys_out[g] = kv[r];
                vals_out[g] = i;
                sorted[g] = rec;
                if (pos != nullptr) pos[i] = (int)g;
            }
        }
        __syncthreads();
    }
}

// start[c] = first sorted slot of the system with cell >= c (relative to the
// system's first particle), c = 0..K; cells above the dense threshold are
// listed (in no particular order: each dense cell is reduced by one block in
// a fixed order).
__global__ void __launch_bounds__(256) k_rb_bounds(const int64_t *__restrict__ prange, int64_t n,
                                                   int K, const int *__restrict__ skeys,
                                                   int *__restrict__ start, int dense_thr,
                                                   int *__restrict__ dense_cells,
                                                   int *__restrict__ dense_count) {
    int64_t p0, np;
    sys_range(prange, n, p0, np);
    start += (int64_t)blockIdx.y * (K + 1);
    dense_cells += (int64_t)blockIdx.y * K;
    dense_count += (int64_t)blockIdx.y * 8;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > K) return;
    const int *k = skeys + p0;
    auto lower = [&](int v) {
        int lo = 0, hi = (int)np;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (k[mid] < v) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    const int s0 = lower(c);
    start[c] = s0;
    if (c < K) {
        const int s1 = lower(c + 1);
        if (s1 - s0 > dense_thr) dense_cells[atomicAdd(dense_count, 1)] = c;
    }
}

int64_t bin_hist_ints(int64_t max_np) {
    const int64_t tiles = max_np > 0 ? (max_np + kRadixTile - 1) / kRadixTile : 1;
    return (int64_t)kRadixBuckets * tiles;
}
int64_t bin_scan_tiles(int64_t max_np) { return (bin_hist_ints(max_np) + 4095) / 4096; }

// Digit widths of the passes for keys below K (at most kRadixMaxBits each,
// as even as possible).
static int radix_passes(int K, int widths[8]) {
    int bits = 0;
    while ((1 << bits) < K) ++bits;
    if (bits == 0) bits = 1;
    const int np = (bits + kRadixMaxBits - 1) / kRadixMaxBits;
    for (int i = 0; i < np; ++i) widths[i] = bits / np + (i < bits % np ? 1 : 0);
    return np;
}

template <typename T>
hipError_t launch_bin(const BinArgs &a, hipStream_t s) {
    const int K = a.ncell * a.ncell * a.ncell;
    const T inv_h = T(a.inv_h);
    const int nsys = a.nsys > 0 ? a.nsys : 1;
    const int64_t maxn = a.prange ? a.max_np : a.n;
    const int tiles = (int)(maxn > 0 ? (maxn + kRadixTile - 1) / kRadixTile : 1);
    const int64_t hist_ints = bin_hist_ints(maxn);
    int widths[8];
    const int passes = radix_passes(K, widths);
    // ping-pong so that the last pass lands in (scell, perm)
    int *kA = a.cell_of, *vA = a.slot, *kB = a.scell, *vB = a.perm;
    int *kin = (passes & 1) ? kA : kB, *vin = (passes & 1) ? vA : vB;
    if (maxn > 0) {
        hipLaunchKernelGGL(k_rb_keys<T>, dim3(tiles, nsys), dim3(1024), 0, s, a.prange, a.n,
                           (const T *)a.x, (const T *)a.y, (const T *)a.z, inv_h, a.ncell,
                           a.periodic, kin, vin, a.count, hist_ints, tiles, widths[0], a.flag,
                           a.dense_count);
        int shift = 0;
        for (int ps = 0; ps < passes; ++ps) {
            const int bits = widths[ps];
            if (ps > 0)
                hipLaunchKernelGGL(k_rb_hist, dim3(tiles, nsys), dim3(1024), 0, s, a.prange, a.n,
                                   kin, a.count, hist_ints, tiles, shift, bits);
            const int64_t L = (int64_t)(1 << bits) * tiles;
            const int st = (int)((L + 4095) / 4096);
            hipLaunchKernelGGL(k_rb_scan_sums, dim3(st, nsys), dim3(1024), 0, s, L, hist_ints,
                               a.count, a.tile_sums);
            hipLaunchKernelGGL(k_rb_scan, dim3(st, nsys), dim3(1024), 0, s, L, hist_ints, a.count,
                               a.tile_sums);
            const int last = ps == passes - 1;
            int *kout = kin == kA ? kB : kA, *vout = vin == vA ? vB : vA;
            const size_t lds = (size_t)(33 << bits) * sizeof(int);
            if (lds > 65536) {
                const hipError_t e = set_max_lds((const void *)k_rb_scatter<T>, lds);
                if (e != hipSuccess) return e;
            }
            hipLaunchKernelGGL(k_rb_scatter<T>, dim3(tiles, nsys), dim3(1024), lds, s, a.prange,
                               a.n, kin, vin, kout, vout, a.count, hist_ints, tiles, shift, bits,
                               last, (const T *)a.x, (const T *)a.y, (const T *)a.z,
                               (const T *)a.q, inv_h, a.ncell, a.periodic,
                               (particle4<T> *)a.sorted, a.pos);
            kin = kout;
            vin = vout;
            shift += bits;
        }
    }
    // a system with no particles still gets its zero starts; the dense count
    // of an empty call is reset here
    if (maxn == 0)
        hipLaunchKernelGGL(k_rb_reset_dense, dim3(1), dim3(64), 0, s, nsys, a.dense_count);
    hipLaunchKernelGGL(k_rb_bounds, dim3((K + 1 + 255) / 256, nsys), dim3(256), 0, s, a.prange,
                       a.n, K, a.scell, a.start, a.dense_threshold, a.dense_cells, a.dense_count);
    return hipGetLastError();
}

template hipError_t launch_bin<float>(const BinArgs &, hipStream_t);
template hipError_t launch_bin<double>(const BinArgs &, hipStream_t);

}  // namespace pmmm
