// Particle <-> cell transforms, in cell units (lengths divided by h).
//   k_p2m      eq. P2M per cell, M_l^m = sum_i q_i R_l^m(r_M - r_i), plus the
//              per-cell sum q |r_rel|^2 used by the periodic correction.
//              Light cells: a group of G lanes strides over the cell's sorted
//              particles and reduces with cross-lane shuffles.  Dense cells
//              (more than the dense threshold): extra workgroups of the same
//              launch, one per cell, with FP64 accumulation and a fixed-order
//              block reduction.
//   k_l2p      eq. L2P for Phi; eq. L2L to destination order one and
//              eq. phigrad for grad Phi; the per-particle terms of a charged
//              periodic system (App. B, correction procedure; the uniform
//              corrections are already in L); results rescaled to the
//              caller's units and scattered to input order -- for large N
//              as one 16-byte record per particle instead, at the caller's
//              index (or in sorted order when the near field adds to it),
//              which k_unpermute splits into the four outputs (after a
//              16-byte gather in the sorted case), in place of four
//              scattered 4-byte stores.
#include "pmmm_internal.h"

namespace pmmm {

// Sum of v[0..64) over the 64 lanes of a wave, scattered: on return lane L
// holds in v[0] the total of component L.  Six exchange steps, each halving
// the components a lane keeps (the lower half if its bit is clear, else the
// upper half, the other half going to the partner lane), so 63 shuffles in
// place of 6 per component; the pattern is fixed, so the sums are
// reproducible.
template <int H, typename A>
__device__ __forceinline__ void wave_rs_step(A *v, int lane) {
    if constexpr (H >= 1) {
        const bool up = (lane & H) != 0;
        static_for<0, H>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            const A send = up ? v[i] : v[i + H];
            const A keep = up ? v[i + H] : v[i];
            v[i] = keep + __shfl_xor(send, H, 64);
        });
        wave_rs_step<H / 2, A>(v, lane);
    }
}

// Light cells (at most dense_thr particles): a group of G lanes per cell
// strides over its sorted particles and reduces with cross-lane shuffles.
template <int PO, typename T, int G>
__global__ void __launch_bounds__(256) k_p2m(int K, const int *__restrict__ start,
                                             const particle4<T> *__restrict__ sorted,
                                             int dense_thr, T *__restrict__ M,
                                             const int64_t *__restrict__ prange) {
    constexpr int P = nreal(PO);
    constexpr int NV = P + 1;
    {
        // system blockIdx.y of a batch: its cell arrays and sorted particles
        const int64_t sy = blockIdx.y;
        start += sy * (K + 1);
        M += sy * NV * K;
        if (prange != nullptr) sorted += prange[2 * sy];
    }
    const int gid = blockIdx.x * 256 + threadIdx.x;
    const int cell = gid / G;
    const int lane = gid & (G - 1);
    int s0 = 0, s1 = 0;
    bool write = false;
    if (cell < K) {
        s0 = start[cell];
        s1 = start[cell + 1];
        write = (s1 - s0) <= dense_thr;
        if (!write) s1 = s0;
    }
    T acc[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) acc[c] = T(0);
    // two particles per lane and round, both loads in flight together; a
    // clamped second particle past the cell's end enters with charge 0
    // (same summation order as one particle per round)
    for (int s = s0 + lane; s < s1; s += 2 * G) {
        const bool two = s + G < s1;
        const particle4<T> r0 = sorted[s];
        const particle4<T> r1 = sorted[two ? s + G : s];
        const T q1 = two ? r1.q : T(0);
        accumulate_regular<PO, T>(-r0.ux, -r0.uy, -r0.uz, r0.q, acc);  // q R(r_M - r_i)
        acc[P] += r0.q * (r0.ux * r0.ux + r0.uy * r0.uy + r0.uz * r0.uz);
        accumulate_regular<PO, T>(-r1.ux, -r1.uy, -r1.uz, q1, acc);
        acc[P] += q1 * (r1.ux * r1.ux + r1.uy * r1.uy + r1.uz * r1.uz);
    }
#pragma unroll
    for (int off = G / 2; off >= 1; off >>= 1) {
#pragma unroll
        for (int c = 0; c < NV; ++c) acc[c] += __shfl_xor(acc[c], off, 64);
    }
    if (write) {
#pragma unroll
        for (int c = 0; c < NV; ++c)
            if ((c & (G - 1)) == lane) M[(int64_t)c * K + cell] = acc[c];
    }
}

// Dense items of the binning, one wave each: the item's kDenseItem sorted
// particles (eight per lane), a scattered wave sum per group of 64
// components, then the moments written directly (a cell of one item) or as
// the cell's partial sum of this item (added by k_p2m_combine in FP64).
template <int PO, typename T>
__global__ void __launch_bounds__(256) k_p2m_dense(int K, const int *__restrict__ start,
                                                   const particle4<T> *__restrict__ sorted,
                                                   const int4 *__restrict__ items,
                                                   int64_t items_cap,
                                                   const int *__restrict__ small,
                                                   float *__restrict__ partial,
                                                   int64_t slots_cap, T *__restrict__ M,
                                                   const int64_t *__restrict__ prange) {
    constexpr int P = nreal(PO);
    constexpr int NV = P + 1;
    constexpr int NG = (NV + 63) / 64;
    {
        const int64_t sy = blockIdx.y;
        start += sy * (K + 1);
        items += sy * items_cap;
        small += sy * 8;
        partial += sy * slots_cap * NV;
        M += sy * NV * K;
        if (prange != nullptr) sorted += prange[2 * sy];
    }
    const int lane = threadIdx.x & 63;
    const int nitems = small[0] < items_cap ? small[0] : (int)items_cap;
    const int nwaves = gridDim.x * 4;
    for (int it = blockIdx.x * 4 + (threadIdx.x >> 6); it < nitems; it += nwaves) {
        const int4 e = items[it];
        const int cell = e.x, j = e.y, J = e.z, ps = e.w;
        const int s0 = start[cell] + j * kDenseItem;
        const int s1e = start[cell + 1];
        const int s1 = s0 + kDenseItem < s1e ? s0 + kDenseItem : s1e;
        constexpr int U = kDenseItem / 64;
        particle4<T> r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int s = s0 + u * 64 + lane;
            r[u] = sorted[s < s1 ? s : s1 - 1];
        }
        T acc[NG * 64];
#pragma unroll
        for (int c = 0; c < NG * 64; ++c) acc[c] = T(0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const T q = s0 + u * 64 + lane < s1 ? r[u].q : T(0);
            accumulate_regular<PO, T>(-r[u].ux, -r[u].uy, -r[u].uz, q, acc);
            acc[P] += q * (r[u].ux * r[u].ux + r[u].uy * r[u].uy + r[u].uz * r[u].uz);
        }
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            wave_rs_step<32, T>(acc + 64 * g, lane);
            const int c = 64 * g + lane;
            if (c < NV) {
                if (J == 1) M[(int64_t)c * K + cell] = acc[64 * g];
                else if (ps + j < slots_cap) partial[(int64_t)(ps + j) * NV + c] = (float)acc[64 * g];
            }
        }
    }
}

// Moments of the cells split into several dense items: one block per split
// cell; wave w adds the partial sums of items w, w + 4, ... in FP64 (eight
// running sums, item k in sum (k / 4) mod 8, so eight loads are in flight),
// then the waves' totals are added in order -- a fixed order, so the
// moments are reproducible.  Lanes run over the components.
template <typename T>
__global__ void __launch_bounds__(256) k_p2m_combine(int K, int NV, const int4 *__restrict__ items,
                                                     int64_t items_cap,
                                                     const int *__restrict__ small,
                                                     const float *__restrict__ partial,
                                                     int64_t slots_cap, T *__restrict__ M) {
    __shared__ double red[4][nreal(PMMM_PMAX) + 1];
    const int64_t splits_cap = dense_splits_cap_of(slots_cap);
    {
        const int64_t sy = blockIdx.y;
        items += sy * items_cap;
        small += sy * 8;
        partial += sy * slots_cap * NV;
        M += sy * NV * K;
    }
    const int4 *splits = items + items_cap - splits_cap;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nsplit = small[4] < splits_cap ? small[4] : (int)splits_cap;
    for (int si = blockIdx.x; si < nsplit; si += gridDim.x) {
        const int4 e = splits[si];
        const int cell = e.x, J = e.y, ps = e.z;
        const bool ok = ps >= 0 && ps + J <= slots_cap;
        for (int c = lane; c < NV; c += 64) {
            const float *pc = partial + (int64_t)ps * NV + c;
            double acc[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u] = 0.0;
            for (int k0 = wid; ok && k0 < J; k0 += 32) {
                float v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    v[u] = k0 + 4 * u < J ? pc[(int64_t)(k0 + 4 * u) * NV] : 0.0f;
#pragma unroll
                for (int u = 0; u < 8; ++u) acc[u] += (double)v[u];
            }
            red[wid][c] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) +
                          ((acc[4] + acc[5]) + (acc[6] + acc[7]));
        }
        __syncthreads();
        for (int c = threadIdx.x; c < NV; c += 256)
            if (ok) M[(int64_t)c * K + cell] = T((red[0][c] + red[1][c]) + (red[2][c] + red[3][c]));
        __syncthreads();
    }
}

template <int PO, typename T>
__global__ void __launch_bounds__(256) k_l2p(int64_t n, int K, int periodic,
                                             const particle4<T> *__restrict__ sorted,
                                             const int *__restrict__ scell,
                                             const int *__restrict__ perm,
                                             const T *__restrict__ L,
                                             const double *__restrict__ sums, T alpha_c,
                                             T inv_h, T *__restrict__ phi_out,
                                             T *__restrict__ gx_out, T *__restrict__ gy_out,
                                             T *__restrict__ gz_out,
                                             out4<T> *__restrict__ staged,
                                             int staged_caller,
                                             const int64_t *__restrict__ prange) {
    constexpr int P = nreal(PO);
    int64_t p0, np;
    sys_range(prange, n, p0, np);
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= np) return;
    const int64_t s = p0 + j;                 // sorted slot (caller-array numbering)
    L += (int64_t)blockIdx.y * P * K;
    sums += (int64_t)blockIdx.y * 8;
    const particle4<T> r = sorted[s];
    const int c = scell[s];
    T Lc[P];
#pragma unroll
    for (int a = 0; a < P; ++a) Lc[a] = L[(int64_t)a * K + c];
    // charged periodic system: Phi += 2 pi/(3V) Q (|u|^2 - 3/(2 alpha^2)),
    // grad += 4 pi/(3V) Q u, with V = K in cell units
    const T qtot_term = periodic ? T(sums[0] * 3.14159265358979323846 / (3.0 * (double)K)) : T(0);
    T R[P];
    regular_harmonics<PO, T>(r.ux, r.uy, r.uz, R);
    // Phi = sum_l [L_l^0 R_l^0 + 2 sum_{m>0} Re(L_l^m R_l^m)]; every
    // multiply-add below is one FMA into a running sum (a product difference
    // inside += would cost a product, an FMA and an add), and the m > 0 terms
    // are summed apart so that the factor 2 is applied once
    T ph = T(0), ph2 = T(0);
#pragma unroll
    for (int l = 0; l <= PO; ++l) {
        ph = fma(Lc[ridx(l, 0)], R[ridx(l, 0)], ph);
#pragma unroll
        for (int m = 1; m <= l; ++m) {
            ph2 = fma(Lc[ridx(l, m)], R[ridx(l, m)], ph2);
            ph2 = fma(-Lc[ridx(l, -m)], R[ridx(l, -m)], ph2);
        }
    }
    ph = fma(T(2), ph2, ph);
    // L'_1^0 and L'_1^1 (eq. L2L with destination order one)
    T d0 = T(0), d02 = T(0), d1re = T(0), d1im = T(0);
#pragma unroll
    for (int lam = 1; lam <= PO; ++lam) {
        const int k = lam - 1;
        d0 = fma(Lc[ridx(lam, 0)], R[ridx(k, 0)], d0);
#pragma unroll
        for (int mu = 1; mu <= k; ++mu) {
            d02 = fma(Lc[ridx(lam, mu)], R[ridx(k, mu)], d02);
            d02 = fma(-Lc[ridx(lam, -mu)], R[ridx(k, -mu)], d02);
        }
        // + sum_{mu=1..lam} L_lam^mu R_k^{mu-1}
#pragma unroll
        for (int mu = 1; mu <= lam; ++mu) {
            const T lre = Lc[ridx(lam, mu)], lim = Lc[ridx(lam, -mu)];
            const T rre = R[ridx(k, mu - 1)];
            d1re = fma(lre, rre, d1re);
            d1im = fma(lim, rre, d1im);
            if (mu - 1 > 0) {
                const T rim = R[ridx(k, -(mu - 1))];
                d1re = fma(-lim, rim, d1re);
                d1im = fma(lre, rim, d1im);
            }
        }
        // - sum_{nu=0..lam-2} conj(L_lam^nu R_k^{nu+1})
#pragma unroll
        for (int nu = 0; nu <= lam - 2; ++nu) {
            const T lre = Lc[ridx(lam, nu)];
            const T rre = R[ridx(k, nu + 1)], rim = R[ridx(k, -(nu + 1))];
            d1re = fma(-lre, rre, d1re);
            d1im = fma(lre, rim, d1im);  // minus the conjugate's imaginary part
            if (nu > 0) {
                const T lim = Lc[ridx(lam, -nu)];
                d1re = fma(lim, rim, d1re);
                d1im = fma(lim, rre, d1im);
            }
        }
    }
    d0 = fma(T(2), d02, d0);
    T gx = -d1re, gy = d1im, gz = d0;
    if (periodic) {
        const T u2 = r.ux * r.ux + r.uy * r.uy + r.uz * r.uz;
        ph += T(2) * qtot_term * (u2 - T(1.5) / (alpha_c * alpha_c));
        gx += T(4) * qtot_term * r.ux;
        gy += T(4) * qtot_term * r.uy;
        gz += T(4) * qtot_term * r.uz;
    }
    const T ih2 = inv_h * inv_h;
    if (staged != nullptr) {
        // one 16-byte store, in sorted order (the near field adds to it
        // there) or at the caller's index; k_unpermute writes the outputs
        staged[staged_caller ? (int64_t)perm[s] : s] =
            out4<T>{ph * inv_h, gx * ih2, gy * ih2, gz * ih2};
        return;
    }
    const int i = perm[s];
    phi_out[i] = ph * inv_h;
    gx_out[i] = gx * ih2;
    gy_out[i] = gy * ih2;
    gz_out[i] = gz * ih2;
}

// Results back to the caller's order: particle i reads its sorted slot's
// record (one 16-byte gather; pos null: the records are in the caller's
// order already) and writes the four outputs coalesced.
template <typename T>
__global__ void __launch_bounds__(256) k_unpermute(int64_t n, const int *__restrict__ pos,
                                                   const out4<T> *__restrict__ staged,
                                                   T *__restrict__ phi_out, T *__restrict__ gx_out,
                                                   T *__restrict__ gy_out, T *__restrict__ gz_out,
                                                   int accumulate) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t g = pos != nullptr ? (int64_t)pos[i] : i;
    if (g < 0 || g >= n) return;  // only reachable with inconsistent counts
    const out4<T> v = staged[g];
    if (accumulate) {
        phi_out[i] += v.phi;
        gx_out[i] += v.gx;
        gy_out[i] += v.gy;
        gz_out[i] += v.gz;
    } else {
        phi_out[i] = v.phi;
        gx_out[i] = v.gx;
        gy_out[i] = v.gy;
        gz_out[i] = v.gz;
    }
}

// ------------------------------------------------------------- launchers
template <int PO, typename T>
static hipError_t p2m_dispatch_g(const P2MArgs &a, hipStream_t s) {
    const int K = a.ncell * a.ncell * a.ncell;
    const int G = a.group;
    const int nlight = (int)(((int64_t)K * G + 255) / 256);
    const int nsys = a.nsys > 0 ? a.nsys : 1;
    const int *st = a.start;
    const particle4<T> *so = (const particle4<T> *)a.sorted;
    T *M = (T *)a.M;
#define PMMM_P2M_G(GG)                                                                     \
    case GG:                                                                               \
        hipLaunchKernelGGL((k_p2m<PO, T, GG>), dim3(nlight, nsys), dim3(256), 0, s, K, st, \
                           so, a.dense_threshold, M, a.prange);                            \
        break;
    switch (G) {
        PMMM_P2M_G(4)
        PMMM_P2M_G(8)
        PMMM_P2M_G(16)
        PMMM_P2M_G(32)
        PMMM_P2M_G(64)
        default:
            return hipErrorInvalidValue;
    }
#undef PMMM_P2M_G
    if (a.items != nullptr) {
        // waves for the dense items: up to the capacity, at most 8192 (they loop)
        const int64_t dwaves = a.items_cap < 8192 ? a.items_cap : 8192;
        const int dblocks = (int)((dwaves + 3) / 4);
        hipLaunchKernelGGL((k_p2m_dense<PO, T>), dim3(dblocks, nsys), dim3(256), 0, s, K, st, so,
                           a.items, a.items_cap, a.small, a.partial, a.slots_cap, M, a.prange);
        // one block per split cell, up to 2048 (they loop)
        const int64_t nsplit = dense_splits_cap_of(a.slots_cap);
        const int cblocks = (int)(nsplit < 2048 ? nsplit : 2048);
        hipLaunchKernelGGL(k_p2m_combine<T>, dim3(cblocks, nsys), dim3(256),
                           0, s, K, nreal(PO) + 1, a.items, a.items_cap, a.small, a.partial,
                           a.slots_cap, M);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_p2m(const P2MArgs &a, hipStream_t s) {
    switch (a.p) {
        case 0: return p2m_dispatch_g<0, T>(a, s);
        case 1: return p2m_dispatch_g<1, T>(a, s);
        case 2: return p2m_dispatch_g<2, T>(a, s);
        case 3: return p2m_dispatch_g<3, T>(a, s);
        case 4: return p2m_dispatch_g<4, T>(a, s);
        case 5: return p2m_dispatch_g<5, T>(a, s);
        case 6: return p2m_dispatch_g<6, T>(a, s);
        case 7: return p2m_dispatch_g<7, T>(a, s);
        case 8: return p2m_dispatch_g<8, T>(a, s);
        case 9: return p2m_dispatch_g<9, T>(a, s);
        case 10: return p2m_dispatch_g<10, T>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int PO, typename T>
static hipError_t l2p_launch(const L2PArgs &a, hipStream_t s) {
    const int K = a.ncell * a.ncell * a.ncell;
    const int64_t maxn = a.prange ? a.max_np : a.n;
    const int blocks = (int)((maxn + 255) / 256);
    const int nsys = a.nsys > 0 ? a.nsys : 1;
    hipLaunchKernelGGL((k_l2p<PO, T>), dim3(blocks, nsys), dim3(256), 0, s, a.n, K, a.periodic,
                       (const particle4<T> *)a.sorted, a.scell, a.perm, (const T *)a.L,
                       a.sums, T(a.alpha_cell), T(a.inv_h), (T *)a.phi,
                       (T *)a.gx, (T *)a.gy, (T *)a.gz, (out4<T> *)a.staged,
                       a.pos == nullptr ? 1 : 0, a.prange);
    if (a.staged != nullptr && a.prange != nullptr) return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename T>
hipError_t launch_unpermute(int64_t n, const int *pos, const void *staged, void *phi, void *gx,
                            void *gy, void *gz, int accumulate, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (staged == nullptr) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_unpermute<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, pos,
                       (const out4<T> *)staged, (T *)phi, (T *)gx, (T *)gy, (T *)gz, accumulate);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_l2p(const L2PArgs &a, hipStream_t s) {
    if ((a.prange ? a.max_np : a.n) == 0) return hipSuccess;
    switch (a.p) {
        case 0: return l2p_launch<0, T>(a, s);
        case 1: return l2p_launch<1, T>(a, s);
        case 2: return l2p_launch<2, T>(a, s);
        case 3: return l2p_launch<3, T>(a, s);
        case 4: return l2p_launch<4, T>(a, s);
        case 5: return l2p_launch<5, T>(a, s);
        case 6: return l2p_launch<6, T>(a, s);
        case 7: return l2p_launch<7, T>(a, s);
        case 8: return l2p_launch<8, T>(a, s);
        case 9: return l2p_launch<9, T>(a, s);
        case 10: return l2p_launch<10, T>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_p2m<float>(const P2MArgs &, hipStream_t);
template hipError_t launch_p2m<double>(const P2MArgs &, hipStream_t);
template hipError_t launch_l2p<float>(const L2PArgs &, hipStream_t);
template hipError_t launch_l2p<double>(const L2PArgs &, hipStream_t);
template hipError_t launch_unpermute<float>(int64_t, const int *, const void *, void *, void *,
                                            void *, void *, int, hipStream_t);
template hipError_t launch_unpermute<double>(int64_t, const int *, const void *, void *, void *,
                                             void *, void *, int, hipStream_t);

}  // namespace pmmm
