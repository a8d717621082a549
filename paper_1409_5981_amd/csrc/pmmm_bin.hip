// Cell binning (Sec. 2.1 requires that the particles of every cell be known,
// which takes linear time): a stable sort of the particles by cell index, as
// a least-significant-digit radix sort with digits of at most 9 bits, so the
// particles of a cell keep the caller's order and every result is bitwise
// reproducible (no atomics decide an order).  Each pass carries the key (cell),
// the value (caller index) and the particle record, so no pass gathers.
//   k_rb_hist     tile histogram of one digit; the first pass computes the
//                 cells from the positions (and flags open-boundary particles
//                 outside the box)
//   k_rb_scan1 or k_rb_scan_sums + k_rb_scan
//                 exclusive scan of the histograms in bucket-major order (so
//                 tile t's bucket-d elements start after every smaller digit
//                 and after bucket d of the tiles before t)
//   k_rb_scatter  stable scatter of one digit: each wave ranks a contiguous
//                 chunk of the tile (wave ballots for equal digits plus the
//                 wave's running count per digit), one prefix over the waves
//                 per tile, then the tile is put in digit order in LDS and
//                 written out in runs; the first pass builds the keys and
//                 records from the positions, the last writes the sorted cell,
//                 the permutation, the sorted records and, on request, each
//                 particle's sorted slot
//   k_rb_bounds   start of every cell by binary search among the sorted slots
//                 of its last digit, and the P2M work items of the cells
//                 above the dense threshold (kDenseItem particles each)
// Cell index: I = floor(r n / b) per axis, clamped to [0, n-1]; periodic
// positions are first wrapped into the box (in cell units).
//
// Batches: blockIdx.y selects one of several independent systems on meshes of
// the same size; prange[2s], prange[2s+1] bound system s's particles in the
// caller's arrays (null: one system, particles [0, n)), and its per-system
// arrays sit at fixed strides (start K + 1, items items_cap, small 8,
// histograms bin_hist_ints(max_np), scan sums bin_scan_tiles(max_np)).
#include "pmmm_internal.h"

namespace pmmm {

constexpr int kRadixBuckets = 1 << kRadixMaxBits;
constexpr int kScanOneBlock = 16384;   // histograms up to this size: one-block scan

template <typename T>
__device__ __forceinline__ void cell_coord(T v, T inv_h, int n, int lim, int periodic, int &ic,
                                           T &u, int &outside) {
    T s = v * inv_h;
    if (periodic) {
        s = s - T(n) * floor(s / T(n));
    } else if (!(s >= T(0) && s < T(lim))) {
        outside = 1;
    }
    int i = (int)floor(s);
    i = i < 0 ? 0 : (i > n - 1 ? n - 1 : i);
    ic = i;
    u = s - T(i) - T(0.5);
}

// Tile handled by block b of G: blocks are dealt to the 8 XCDs in turn, and
// this mapping gives each XCD a contiguous range of tiles, so the runs that
// neighbouring tiles write side by side meet in one L2.
__device__ __forceinline__ int xcd_tile(int b, int G) {
    const int q = G >> 3, r = G & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// LDS of the scatter: the per-wave counts [16][nb], later reused as the
// staging area of one tile, then ls[nb], goff[nb], wtot[16].
template <typename T, int R>
__host__ __device__ constexpr size_t scatter_region(int bits) {
    return (size_t)16 * ((size_t)1 << bits) * sizeof(int) >
                   (size_t)1024 * R * sizeof(particle4<T>)
               ? (size_t)16 * ((size_t)1 << bits) * sizeof(int)
               : (size_t)1024 * R * sizeof(particle4<T>);
}
template <typename T, int R>
constexpr size_t scatter_lds(int bits) {
    return scatter_region<T, R>(bits) + (size_t)(2 * (1 << bits) + 16) * sizeof(int);
}

__global__ void k_rb_reset_items(int nsys, int *__restrict__ small) {
    for (int sy = threadIdx.x; sy < nsys; sy += blockDim.x) {
        small[(int64_t)sy * 8] = 0;
        small[(int64_t)sy * 8 + 3] = 0;
        small[(int64_t)sy * 8 + 4] = 0;
    }
}

// Tile histogram of digit (key >> shift) & (2^bits - 1), written to
// hist[d * tiles + t] (every block writes all 2^bits of its entries).
template <typename T, int R>
__global__ void __launch_bounds__(1024) k_rb_hist(
    const int64_t *__restrict__ prange, int64_t n, int first, const T *__restrict__ x,
    const T *__restrict__ y, const T *__restrict__ z, T inv_h, int nc, int3 lim, int periodic,
    const int *__restrict__ keys, int *__restrict__ hist, int64_t hist_ints, int tiles,
    int shift, int bits, int *__restrict__ flag, int *__restrict__ small) {
    __shared__ int s_hist[kRadixBuckets];
    int64_t p0, np;
    sys_range(prange, n, p0, np);
    const int nb = 1 << bits, t = blockIdx.x;
    for (int d = threadIdx.x; d < nb; d += blockDim.x) s_hist[d] = 0;
    if (first && t == 0 && threadIdx.x == 0) {
        // item, partial-slot and split-cell counts of this binning (filled by
        // k_rb_bounds)
        small[(int64_t)blockIdx.y * 8] = 0;
        small[(int64_t)blockIdx.y * 8 + 3] = 0;
        small[(int64_t)blockIdx.y * 8 + 4] = 0;
    }
    __syncthreads();
    int kv[R];
    int out = 0;
    if (first) {
        T xv[R], yv[R], zv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t j = (int64_t)t * (1024 * R) + r * 1024 + threadIdx.x;
            const int64_t i = p0 + (j < np ? j : 0);
            const bool act = j < np;
            xv[r] = act ? x[i] : T(0);
            yv[r] = act ? y[i] : T(0);
            zv[r] = act ? z[i] : T(0);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t j = (int64_t)t * (1024 * R) + r * 1024 + threadIdx.x;
            int ix, iy, iz;
            T u;
            cell_coord(xv[r], inv_h, nc, lim.x, periodic, ix, u, out);
            cell_coord(yv[r], inv_h, nc, lim.y, periodic, iy, u, out);
            cell_coord(zv[r], inv_h, nc, lim.z, periodic, iz, u, out);
            kv[r] = j < np ? (iz * nc + iy) * nc + ix : -1;
        }
        if (out && np > 0) {
            // only lanes with particles can be outside (inactive lanes read 0)
            *flag = 1;
        }
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t j = (int64_t)t * (1024 * R) + r * 1024 + threadIdx.x;
            kv[r] = j < np ? keys[p0 + j] : -1;
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (kv[r] >= 0) atomicAdd(&s_hist[(kv[r] >> shift) & (nb - 1)], 1);
    __syncthreads();
    int *h = hist + (int64_t)blockIdx.y * hist_ints;
    for (int d = threadIdx.x; d < nb; d += blockDim.x) h[(int64_t)d * tiles + t] = s_hist[d];
}

// Exclusive scan of the L (<= kScanOneBlock) histogram entries of every
// system in one block: 16 consecutive entries per thread.
__global__ void __launch_bounds__(1024) k_rb_scan1(int64_t L, int64_t hist_ints,
                                                   int *__restrict__ hist) {
    __shared__ int wtot[16];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    hist += (int64_t)blockIdx.y * hist_ints;
    const int64_t base = (int64_t)tid * 16;
    int v[16];
    int tot = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        v[k] = base + k < L ? hist[base + k] : 0;
        tot += v[k];
    }
    int inc = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(inc, off, 64);
        if (lane >= off) inc += u;
    }
    if (lane == 63) wtot[wid] = inc;
    __syncthreads();
    int run = inc - tot;
    for (int w = 0; w < wid; ++w) run += wtot[w];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (base + k < L) hist[base + k] = run;
        run += v[k];
    }
}

// The same for larger histograms, in scan tiles of 4096: per-tile sums, then
// each tile scanned from the sum of the tiles before it.
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

// Stable scatter of one digit over tiles of 1024 R elements; wave w ranks
// elements [64 R w, 64 R (w + 1)) of its tile, 64 at a time.
template <typename T, int R>
__global__ void __launch_bounds__(1024) k_rb_scatter(
    const int64_t *__restrict__ prange, int64_t n, int first, int last, const T *__restrict__ x,
    const T *__restrict__ y, const T *__restrict__ z, const T *__restrict__ q, T inv_h, int nc,
    int periodic, const int *__restrict__ keys_in, const int *__restrict__ vals_in,
    const particle4<T> *__restrict__ recs_in, int *__restrict__ keys_out,
    int *__restrict__ vals_out, particle4<T> *__restrict__ recs_out, int *__restrict__ pos,
    const int *__restrict__ offs, int64_t hist_ints, int tiles, int shift, int bits) {
    constexpr int TILE = 1024 * R;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int nb = 1 << bits;
    int *wcnt = (int *)lds_raw;                      // [16][nb] while ranking
    int *sint = (int *)lds_raw;                      // staging: TILE ints
    particle4<T> *srec = (particle4<T> *)lds_raw;    // staging: TILE records
    int *ls = (int *)(lds_raw + scatter_region<T, R>(bits));  // [nb] tile-local digit start
    int *goff = ls + nb;                             // [nb] global slot - local slot
    int *wtot = goff + nb;                           // [16]
    int64_t p0, np;
    sys_range(prange, n, p0, np);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    offs += (int64_t)blockIdx.y * hist_ints;
    const int64_t t0 = (int64_t)t * TILE;
    const int na = (int)(np - t0 <= 0 ? 0 : (np - t0 > TILE ? TILE : np - t0));
    for (int e = tid; e < 16 * nb; e += 1024) wcnt[e] = 0;

    int key[R], val[R], dig[R];
    particle4<T> rec[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = wid * 64 * R + r * 64 + lane;
        const int64_t i = p0 + t0 + (e < na ? e : 0);
        if (e < na) {
            if (first) {
                int ix, iy, iz, out = 0;
                cell_coord(x[i], inv_h, nc, nc, periodic, ix, rec[r].ux, out);
                cell_coord(y[i], inv_h, nc, nc, periodic, iy, rec[r].uy, out);
                cell_coord(z[i], inv_h, nc, nc, periodic, iz, rec[r].uz, out);
                rec[r].q = q != nullptr ? q[i] : T(0);
                key[r] = (iz * nc + iy) * nc + ix;
                val[r] = (int)i;
            } else {
                key[r] = keys_in[i];
                val[r] = vals_in[i];
                rec[r] = recs_in[i];
            }
        } else {
            key[r] = 0;
            val[r] = 0;
            rec[r] = particle4<T>{T(0), T(0), T(0), T(0)};
        }
        dig[r] = (key[r] >> shift) & (nb - 1);
    }
    __syncthreads();

    // rank among the wave's earlier elements of the same digit: the running
    // count of the digit before this group of 64, plus the lower lanes that
    // hold it; one lane per digit group then advances the count (the wave's
    // LDS reads precede its writes, and only this wave touches its counts)
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    int rank[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = wid * 64 * R + r * 64 + lane;
        const bool act = e < na;
        const int d = dig[r];
        uint64_t peers = __ballot(act);
        for (int b = 0; b < bits; ++b) {
            const uint64_t m = __ballot(act && ((d >> b) & 1));
            peers &= ((d >> b) & 1) ? m : ~m;
        }
        const int before = __popcll(peers & lt);
        const int base = act ? wcnt[wid * nb + d] : 0;
        __builtin_amdgcn_wave_barrier();
        rank[r] = base + before;
        if (act && before == 0) wcnt[wid * nb + d] = base + __popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();

    // per digit: exclusive prefix over the waves (in place) and the tile count
    int tot = 0;
    if (tid < nb) {
#pragma unroll
        for (int w = 0; w < 16; ++w) {
            const int c = wcnt[w * nb + tid];
            wcnt[w * nb + tid] = tot;
            tot += c;
        }
    }
    // exclusive scan of the tile counts over the digits
    int inc = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(inc, off, 64);
        if (lane >= off) inc += u;
    }
    if (lane == 63) wtot[wid] = inc;
    __syncthreads();
    if (tid < nb) {
        int pre = 0;
        for (int w = 0; w < wid; ++w) pre += wtot[w];
        const int l = pre + inc - tot;
        ls[tid] = l;
        goff[tid] = offs[(int64_t)tid * tiles + t] - l;
    }
    __syncthreads();
    int lidx[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = wid * 64 * R + r * 64 + lane;
        lidx[r] = e < na ? ls[dig[r]] + wcnt[wid * nb + dig[r]] + rank[r] : 0;
    }
    __syncthreads();  // the counts' region becomes the staging area

    // the tile in digit order: slot jj of the tile goes to goff[digit] + jj
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (wid * 64 * R + r * 64 + lane < na) sint[lidx[r]] = key[r];
    __syncthreads();
    int dst[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int jj = r * 1024 + tid;
        dst[r] = 0;
        if (jj < na) {
            const int k = sint[jj];
            dst[r] = goff[(k >> shift) & (nb - 1)] + jj;
            keys_out[p0 + dst[r]] = k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (wid * 64 * R + r * 64 + lane < na) sint[lidx[r]] = val[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int jj = r * 1024 + tid;
        if (jj < na) {
            const int v = sint[jj];
            vals_out[p0 + dst[r]] = v;
            if (last && pos != nullptr) pos[v] = (int)(p0 + dst[r]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (wid * 64 * R + r * 64 + lane < na) srec[lidx[r]] = rec[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int jj = r * 1024 + tid;
        if (jj < na) recs_out[p0 + dst[r]] = srec[jj];
    }
}

// start[c] = first sorted slot of the system with cell >= c (relative to the
// system's first particle), c = 0..K, searched among the slots whose last
// digit equals c's (their range comes from the last pass's scanned
// histogram).  A cell of more than dense_thr particles becomes J =
// ceil(count / kDenseItem) P2M items {cell, j, J, first partial slot (J > 1)
// or -1}, and a cell of J > 1 items is also listed as split {cell, J, first
// slot}; items, slots and list entries are reserved with atomics, so their
// positions vary from call to call, but every item covers a fixed particle
// range and the partials of a cell are added in a fixed order, so the
// moments do not.
__global__ void __launch_bounds__(256) k_rb_bounds(
    const int64_t *__restrict__ prange, int64_t n, int K, const int *__restrict__ skeys,
    int *__restrict__ start, int dense_thr, int4 *__restrict__ items, int64_t items_cap,
    int64_t splits_cap, int *__restrict__ small, const int *__restrict__ offs, int64_t hist_ints,
    int tiles, int shift, int bits) {
    int64_t p0, np;
    sys_range(prange, n, p0, np);
    start += (int64_t)blockIdx.y * (K + 1);
    if (items != nullptr) items += (int64_t)blockIdx.y * items_cap;
    small += (int64_t)blockIdx.y * 8;
    offs += (int64_t)blockIdx.y * hist_ints;
    const int c = blockIdx.x * blockDim.x + threadIdx.x, lane = threadIdx.x & 63;
    const int nb = 1 << bits;
    const int *k = skeys + p0;
    auto lower = [&](int v) {
        if (np == 0) return 0;
        const int dh = v >> shift;
        if (dh >= nb) return (int)np;
        int lo = offs[(int64_t)dh * tiles];
        int hi = dh + 1 < nb ? offs[(int64_t)(dh + 1) * tiles] : (int)np;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (k[mid] < v) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    const int s0 = lower(c < K ? c : K);
    int s1 = __shfl_down(s0, 1, 64);
    if (lane == 63 && c < K) s1 = lower(c + 1);
    if (c <= K) start[c] = s0;
    if (items != nullptr && c < K && s1 - s0 > dense_thr) {
        const int J = (s1 - s0 + kDenseItem - 1) / kDenseItem;
        const int base = atomicAdd(small, J);
        const int ps = J > 1 ? atomicAdd(small + 3, J) : -1;
        for (int j = 0; j < J; ++j)
            if (base + j < items_cap - splits_cap) items[base + j] = int4{c, j, J, ps};
        if (J > 1) {
            const int si = atomicAdd(small + 4, 1);
            if (si < splits_cap) items[items_cap - splits_cap + si] = int4{c, J, ps, 0};
        }
    }
}

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

template <typename T, int R>
static hipError_t radix_bin(const BinArgs &a, int K, int64_t maxn, hipStream_t s) {
    const T inv_h = T(a.inv_h);
    const int nsys = a.nsys > 0 ? a.nsys : 1;
    const int tiles = (int)bin_tiles(maxn);
    const int64_t hist_ints = bin_hist_ints(maxn);
    int widths[8];
    const int passes = radix_passes(K, widths);
    int *kA = a.cell_of, *vA = a.slot, *kF = a.scell, *vF = a.perm;
    particle4<T> *rA = (particle4<T> *)a.recs, *rF = (particle4<T> *)a.sorted;
    const int *kin = nullptr, *vin = nullptr;
    const particle4<T> *rin = nullptr;
    int shift = 0;
    const int3 lim = make_int3(a.lim[0] > 0 ? a.lim[0] : a.ncell, a.lim[1] > 0 ? a.lim[1] : a.ncell,
                               a.lim[2] > 0 ? a.lim[2] : a.ncell);
    for (int ps = 0; ps < passes; ++ps) {
        const int bits = widths[ps], first = ps == 0, last = ps == passes - 1;
        // alternate so that the last pass lands in (scell, perm, sorted)
        const bool to_final = ((passes - 1 - ps) & 1) == 0;
        int *ko = to_final ? kF : kA, *vo = to_final ? vF : vA;
        particle4<T> *ro = to_final ? rF : rA;
        hipLaunchKernelGGL((k_rb_hist<T, R>), dim3(tiles, nsys), dim3(1024), 0, s, a.prange, a.n,
                           first, (const T *)a.x, (const T *)a.y, (const T *)a.z, inv_h, a.ncell,
                           lim, a.periodic, kin, a.count, hist_ints, tiles, shift, bits, a.flag,
                           a.small);
        const int64_t L = (int64_t)(1 << bits) * tiles;
        if (L <= kScanOneBlock) {
            hipLaunchKernelGGL(k_rb_scan1, dim3(1, nsys), dim3(1024), 0, s, L, hist_ints, a.count);
        } else {
            const int st = (int)((L + 4095) / 4096);
            hipLaunchKernelGGL(k_rb_scan_sums, dim3(st, nsys), dim3(1024), 0, s, L, hist_ints,
                               a.count, a.tile_sums);
            hipLaunchKernelGGL(k_rb_scan, dim3(st, nsys), dim3(1024), 0, s, L, hist_ints,
                               a.count, a.tile_sums);
        }
        const size_t lds = scatter_lds<T, R>(bits);
        if (lds > 65536) {
            const hipError_t e = set_max_lds((const void *)k_rb_scatter<T, R>, lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL((k_rb_scatter<T, R>), dim3(tiles, nsys), dim3(1024), lds, s, a.prange,
                           a.n, first, last, (const T *)a.x, (const T *)a.y, (const T *)a.z,
                           (const T *)a.q, inv_h, a.ncell, a.periodic, kin, vin, rin, ko, vo, ro,
                           a.pos, a.count, hist_ints, tiles, shift, bits);
        kin = ko;
        vin = vo;
        rin = ro;
        if (!last) shift += bits;
    }
    hipLaunchKernelGGL(k_rb_bounds, dim3((K + 1 + 255) / 256, nsys), dim3(256), 0, s, a.prange,
                       a.n, K, a.scell, a.start, a.dense_threshold, a.items, a.items_cap,
                       dense_splits_cap_of(a.slots_cap), a.small, a.count, hist_ints, tiles, shift,
                       widths[passes - 1]);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_bin(const BinArgs &a, hipStream_t s) {
    const int K = a.ncell * a.ncell * a.ncell;
    const int64_t maxn = a.prange ? a.max_np : a.n;
    if (maxn == 0) {
        // every system is empty: zero starts, and the item counts reset here
        const int nsys = a.nsys > 0 ? a.nsys : 1;
        hipLaunchKernelGGL(k_rb_reset_items, dim3(1), dim3(64), 0, s, nsys, a.small);
        hipLaunchKernelGGL(k_rb_bounds, dim3((K + 1 + 255) / 256, nsys), dim3(256), 0, s,
                           a.prange, a.n, K, a.scell, a.start, a.dense_threshold, a.items,
                           a.items_cap, dense_splits_cap_of(a.slots_cap), a.small, a.count,
                           (int64_t)0, 1, 0, 1);
        return hipGetLastError();
    }
    switch (bin_tile_items(maxn)) {
    case 4: return radix_bin<T, 4>(a, K, maxn, s);
    case 2: return radix_bin<T, 2>(a, K, maxn, s);
    default: return radix_bin<T, 1>(a, K, maxn, s);
    }
}

template hipError_t launch_bin<float>(const BinArgs &, hipStream_t);
template hipError_t launch_bin<double>(const BinArgs &, hipStream_t);

}  // namespace pmmm
