// Near field (Sec. 2.1, last paragraph, and Sec. 2.3): the particles of the
// (2c+1)^3 cells masked out of the transfer kernel interact by direct
// Newtonian sums with no cutoff function.  Periodic meshes take, for each
// neighbour cell, the one image within c cells of the target cell.
//
// Tiles of targets.  A row of cells (fixed y and z) is a contiguous range of
// sorted slots, cut into tiles of kNearTile consecutive targets (one wave
// each).  For every neighbour row (dy, dz) the source cells a tile needs,
// x in [xa - c, xb + c] for targets in cells xa..xb, are contiguous sorted
// slots too (split where a periodic row wraps, each piece with its image
// shift), so a wave streams them in chunks of 64 through LDS and every lane
// reads each source as a broadcast.  A per-pair mask keeps exactly the
// neighbour cells of the lane's own target (|x offset| <= c) and drops the
// target itself.  Displacements are formed as the integer cell offset plus
// the difference of the in-cell offsets u (|u| <= 1/2), so FP32 keeps its
// relative precision on near pairs.
//
// k_near_tiles  one block: tiles per row, their exclusive prefix and the row
//               of every tile
// k_near        one wave per tile; results (caller units) are stored or added
//               to the sorted-order records that k_unpermute sends back to the
//               caller's order
#include "pmmm_internal.h"

namespace pmmm {

constexpr int kNearTile = 64;          // targets per tile (one wave)
constexpr int kNearRowsPerThread = 16; // k_near_tiles: 1024 threads x 16 rows >= 128^2 rows

__global__ void __launch_bounds__(1024) k_near_tiles(int n, const int *__restrict__ start,
                                                     int *__restrict__ tile_first,
                                                     int *__restrict__ tile_row,
                                                     int *__restrict__ ntiles) {
    __shared__ int wtot[16];
    const int rows = n * n;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int per = (rows + 1023) >> 10;  // <= kNearRowsPerThread (rows <= 16384)
    int cnt[kNearRowsPerThread];
    int tot = 0;
#pragma unroll
    for (int k = 0; k < kNearRowsPerThread; ++k) {
        const int r = tid * per + k;
        int c = 0;
        if (k < per && r < rows) {
            const int np = start[(r + 1) * n] - start[r * n];
            c = (np + kNearTile - 1) / kNearTile;
        }
        cnt[k] = c;
        tot += c;
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
    for (int k = 0; k < kNearRowsPerThread; ++k) {
        const int r = tid * per + k;
        if (k < per && r < rows) {
            tile_first[r] = run;
            for (int t = 0; t < cnt[k]; ++t) tile_row[run + t] = r;
            run += cnt[k];
        }
    }
    if (tid == 1023) ntiles[0] = run;
}

// Sources staged in LDS for one chunk: offsets u and charge, the y and z
// offsets already moved into the target row's frame (u + row offset), the
// source cell's x in the tile's unwrapped frame, and its sorted slot.
template <typename T>
struct NearSrc {
    T ux, yz[2], q;
};

// Cell-index arithmetic on rows of n cells: shifts for power-of-two n (POW2),
// divisions otherwise.
template <bool POW2>
struct RowIdx {
    int n, logn;
    __device__ __forceinline__ int mul(int v) const { return POW2 ? v << logn : v * n; }
    __device__ __forceinline__ int div(int v) const { return POW2 ? v >> logn : v / n; }  // v >= 0
    __device__ __forceinline__ int mod(int v) const { return POW2 ? v & (n - 1) : v % n; }  // v >= 0
};

template <typename T, bool POW2>
__global__ void __launch_bounds__(kNearTile) k_near(int n, int logn, int cutoff, int periodic,
                                                    const int *__restrict__ start,
                                                    const int *__restrict__ scell,
                                                    const particle4<T> *__restrict__ sorted,
                                                    const int *__restrict__ tile_first,
                                                    const int *__restrict__ tile_row,
                                                    const int *__restrict__ ntiles, T inv_h,
                                                    out4<T> *__restrict__ staged, int accumulate) {
    __shared__ NearSrc<T> src[kNearTile];
    __shared__ int2 sx_slot[kNearTile];
    const int lane = threadIdx.x;
    const int t = blockIdx.x;
    if (t >= ntiles[0]) return;  // the whole (one-wave) block leaves
    const RowIdx<POW2> ri{n, logn};
    const int r = tile_row[t];
    const int row0 = start[ri.mul(r)], row1 = start[ri.mul(r + 1)];
    const int s0 = row0 + (t - tile_first[r]) * kNearTile;
    const int s1 = min(s0 + kNearTile, row1);
    const int s = s0 + lane;
    const bool live = s < s1;
    const int sc = live ? s : s1 - 1;
    const particle4<T> me = sorted[sc];
    const int tx = ri.mod(scell[sc]);
    const int xa = ri.mod(scell[s0]), xb = ri.mod(scell[s1 - 1]);  // sorted: xa <= xb
    const int iz = ri.div(r), iy = ri.mod(r);
    const int c = cutoff;
    // each chunk of at most 64 sources is summed in T, the chunk sums in FP64:
    // a target meets ~10^3 sources, and one long FP32 running sum would lose
    // about sqrt(10^3 / 2) roundings' worth of accuracy
    double tph = 0.0, tax = 0.0, tay = 0.0, taz = 0.0;
    for (int dz = -c; dz <= c; ++dz) {
        int jz = iz + dz;
        if (jz < 0 || jz >= n) {
            if (!periodic) continue;
            jz += jz < 0 ? n : -n;      // |dz| <= c < n
        }
        for (int dy = -c; dy <= c; ++dy) {
            int jy = iy + dy;
            if (jy < 0 || jy >= n) {
                if (!periodic) continue;
                jy += jy < 0 ? n : -n;
            }
            const int jrow = ri.mul(jz) + jy;
            // unwrapped x range of the sources, in pieces that do not wrap
            int lo = xa - c, hi = xb + c;
            if (!periodic) {
                lo = lo < 0 ? 0 : lo;
                hi = hi > n - 1 ? n - 1 : hi;
            }
            for (int u0 = lo; u0 <= hi;) {
                // image shift of the piece holding u0: floor(u0 / n) n
                const int shift = ri.mul(u0 >= 0 ? ri.div(u0) : -ri.div(n - 1 - u0));
                const int x0 = u0 - shift;
                const int x1 = hi - shift < n - 1 ? hi - shift : n - 1;
                const int b0 = start[ri.mul(jrow) + x0], b1 = start[ri.mul(jrow) + x1 + 1];
                for (int c0 = b0; c0 < b1; c0 += kNearTile) {
                    const int cnt = b1 - c0 < kNearTile ? b1 - c0 : kNearTile;
                    {
                        const int js = c0 + lane < b1 ? c0 + lane : b1 - 1;
                        const particle4<T> so = sorted[js];
                        const int sxu = ri.mod(scell[js]) + shift;
                        __syncthreads();  // the previous chunk has been read
                        // target - source displacement in y and z is
                        // (u_t - u_s) - (row offset): keep u_s + offset
                        src[lane] = NearSrc<T>{so.ux, {so.uy + T(dy), so.uz + T(dz)},
                                               c0 + lane < b1 ? so.q : T(0)};
                        sx_slot[lane] = make_int2(sxu, js);
                        __syncthreads();
                    }
                    const int cnt4 = (cnt + 3) & ~3;
                    T ph = T(0), ax = T(0), ay = T(0), az = T(0);
                    for (int k0 = 0; k0 < cnt4; k0 += 4) {
#pragma unroll
                        for (int kk = 0; kk < 4; ++kk) {
                            const int k = k0 + kk;
                            const NearSrc<T> sv = src[k < cnt ? k : cnt - 1];
                            const int2 xs = sx_slot[k < cnt ? k : cnt - 1];
                            const int o = tx - xs.x;  // target - source cell offset in x
                            const bool m = k < cnt && (unsigned)(o + c) <= (unsigned)(2 * c) &&
                                           xs.y != s;
                            const T dx = T(o) + (me.ux - sv.ux);
                            const T dyv = me.uy - sv.yz[0];
                            const T dzv = me.uz - sv.yz[1];
                            const T r2 = m ? dx * dx + dyv * dyv + dzv * dzv : T(1);
                            T ri;
                            if constexpr (sizeof(T) == 4)
                                ri = __builtin_amdgcn_rsqf(r2);
                            else
                                ri = T(1) / sqrt(r2);
                            const T qr = (m ? sv.q : T(0)) * ri;
                            ph += qr;
                            const T qr3 = qr * (ri * ri);
                            ax = fma(-qr3, dx, ax);
                            ay = fma(-qr3, dyv, ay);
                            az = fma(-qr3, dzv, az);
                        }
                    }
                    tph += (double)ph;
                    tax += (double)ax;
                    tay += (double)ay;
                    taz += (double)az;
                }
                u0 = x1 + shift + 1;
            }
        }
    }
    if (!live) return;
    const double ih = (double)inv_h, ih2 = ih * ih;
    out4<T> v{T(tph * ih), T(tax * ih2), T(tay * ih2), T(taz * ih2)};
    if (accumulate) {
        const out4<T> o = staged[s];
        v.phi += o.phi;
        v.gx += o.gx;
        v.gy += o.gy;
        v.gz += o.gz;
    }
    staged[s] = v;
}

template <typename T>
hipError_t launch_near(const NearArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    if (a.ncell * a.ncell > 1024 * kNearRowsPerThread) return hipErrorInvalidValue;
    const bool pow2 = (a.ncell & (a.ncell - 1)) == 0;
    const int logn = __builtin_ctz((unsigned)a.ncell);
    hipLaunchKernelGGL(k_near_tiles, dim3(1), dim3(1024), 0, s, a.ncell, a.start, a.tile_first,
                       a.tile_row, a.ntiles);
    const int64_t max_tiles = (a.n + kNearTile - 1) / kNearTile + (int64_t)a.ncell * a.ncell;
    if (pow2)
        hipLaunchKernelGGL((k_near<T, true>), dim3((unsigned)max_tiles), dim3(kNearTile), 0, s,
                           a.ncell, logn, a.cutoff, a.periodic, a.start, a.scell,
                           (const particle4<T> *)a.sorted, a.tile_first, a.tile_row, a.ntiles,
                           T(a.inv_h), (out4<T> *)a.staged, a.accumulate);
    else
        hipLaunchKernelGGL((k_near<T, false>), dim3((unsigned)max_tiles), dim3(kNearTile), 0, s,
                           a.ncell, logn, a.cutoff, a.periodic, a.start, a.scell,
                           (const particle4<T> *)a.sorted, a.tile_first, a.tile_row, a.ntiles,
                           T(a.inv_h), (out4<T> *)a.staged, a.accumulate);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_zero_ints(int *__restrict__ p, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

hipError_t launch_zero_ints(int *p, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_ints, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p,
                       count);
    return hipGetLastError();
}

int64_t near_tile_capacity(int64_t n, int ncell) {
    return (n + kNearTile - 1) / kNearTile + (int64_t)ncell * ncell;
}

template hipError_t launch_near<float>(const NearArgs &, hipStream_t);
template hipError_t launch_near<double>(const NearArgs &, hipStream_t);

}  // namespace pmmm
