// Column kernel of the wave-space convolution: for w (ky, kx) columns of ALL
// components, the complex FFT along z, the M2L of eq. realmatrix at every
// frequency of the columns and the inverse FFT along z.  Only z < n is read
// and written back (the rest of the padded mesh is zero on input and
// aliasing on output for open boundaries).  One template, instantiated per
// order in the pmmm_column_*.hip units so that they compile in parallel.
//
// Wave-space M2L: every transfer-kernel component of order k is even or odd
// under d -> -d, so its spectrum is real (k even) or imaginary (k odd); the
// plan stores one real number g per component and frequency (Re or Im).
// Each real-matrix coefficient (A, B, C, D combinations of eq. realmatrix)
// built from order-k components is therefore (1 or i) x (a signed sum of at
// most two g values).  Writing i^(k mod 2) = i^(l mod 2) i^(lam mod 2) s with
// s = -1 when l and lam are both odd, the moments are pre-multiplied by
// i^(lam mod 2), accumulated with real coefficients, and the outputs of odd
// order l are post-multiplied by i.
#pragma once

#include "pmmm_internal.h"

namespace pmmm {

// Global loads each thread keeps in flight before writing them to LDS.
constexpr int kColumnLoadBatch = 8;

// ---------------------------------------------------------------- columns
// floor(t / d) for 0 <= t < 2^22 - 1 and 1 <= d < 2^24 from inv_d = fl(1/d):
// x = (t + 1/2) / d lies at least 1/(2d) from an integer, and the two FP32
// roundings move it by at most x 2^-23 (1 + 2^-24) < 1/(2d).
__device__ __forceinline__ int small_div(int t, float inv_d) {
    return (int)(((float)t + 0.5f) * inv_d);
}

template <typename T>
__device__ __forceinline__ T term2(const T *g, Term a, int sa, Term b, int sb) {
    // sa * a + sb * b with compile-time signs after unrolling
    const int s1 = a.sgn * sa, s2 = b.sgn * sb;
    if (s1 != 0 && s2 != 0) {
        return (s1 > 0 ? g[a.off] : -g[a.off]) + (s2 > 0 ? g[b.off] : -g[b.off]);
    }
    if (s1 != 0) return s1 > 0 ? g[a.off] : -g[a.off];
    if (s2 != 0) return s2 > 0 ? g[b.off] : -g[b.off];
    return T(0);
}

template <typename T>
__device__ __forceinline__ void mac(cplx<T> &acc, T c, cplx<T> m) {
    acc.re = fma(c, m.re, acc.re);
    acc.im = fma(c, m.im, acc.im);
}

// Output orders are dealt to kRowSplit subsets at compile time, largest
// first, each to the subset with the fewest rows so far (2l+1 rows per order).
constexpr int kRowSplit = kColumnRowSplit;

__host__ __device__ constexpr int order_subset(int PO, int RS, int l) {
    int load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int owner = 0;
    for (int o = PO; o >= 0; --o) {
        int best = 0;
        for (int s = 1; s < RS; ++s)
            if (load[s] < load[best]) best = s;
        load[best] += 2 * o + 1;
        if (o == l) owner = best;
    }
    return owner;
}

// Does subset S need the kernel values of order NN?
__host__ __device__ constexpr bool subset_needs(int PO, int RS, int S, int NN) {
    for (int l = 0; l <= PO; ++l)
        if (order_subset(PO, RS, l) == S && NN - l >= 0 && NN - l <= PO) return true;
    return false;
}

// acc[a] += sum_b t_ab(g of order NN) * M~_b over the output orders l of
// subset S with lam = NN - l; M~ of order lam is read from LDS (column
// `mcol`, row stride `mstride`, plus `odd` for odd rows b when the rows are
// swizzled) and pre-multiplied by i^(lam mod 2).  Every index is a
// compile-time constant (static_for), so acc, Mh and g stay in registers.
template <int PO, int NN, int RS, int S, typename T>
__device__ __forceinline__ void m2l_order(const T *g, const cplx<T> *mcol, int mstride,
                                          cplx<T> *acc, int odd = 0) {
    constexpr int lo = NN - PO > 0 ? NN - PO : 0;
    constexpr int hi = NN < PO ? NN : PO;
    static_for<lo, hi + 1>([&](auto il) {
        constexpr int l = decltype(il)::value;
        if constexpr (order_subset(PO, RS, l) == S) {
            constexpr int lam = NN - l;
            constexpr int s = ((l & 1) && (lam & 1)) ? -1 : 1;
            cplx<T> Mh[2 * lam + 1];
            static_for<0, 2 * lam + 1>([&](auto ik) {
                constexpr int k = decltype(ik)::value;
                constexpr int mu = k - lam;
                const cplx<T> v = mcol[ridx(lam, mu) * mstride + ((ridx(lam, mu) & 1) ? odd : 0)];
                Mh[k] = (lam & 1) ? cplx<T>{-v.im, v.re} : v;
            });
            static_for<0, l + 1>([&](auto im) {
                constexpr int m = decltype(im)::value;
                cplx<T> are = acc[ridx(l, m)];
                cplx<T> aim = (m > 0) ? acc[ridx(l, -m)] : cplx<T>{T(0), T(0)};
                // mu = 0 column: G^{m,0} = S_NN^{-m}
                {
                    const cplx<T> x = Mh[lam];
                    mac(are, term2(g, re_S(NN, -m), s, Term{0, 0}, 0), x);
                    if constexpr (m > 0) mac(aim, term2(g, im_S(NN, -m), s, Term{0, 0}, 0), x);
                }
                static_for<1, lam + 1>([&](auto iu) {
                    constexpr int mu = decltype(iu)::value;
                    const cplx<T> xr = Mh[lam + mu];   // Re M_lam^mu
                    const cplx<T> xi = Mh[lam - mu];   // Im M_lam^mu
                    constexpr int sg = (mu & 1) ? -1 : 1;  // (-1)^mu of C and D
                    // Re row: (A + C) ReM - (B - D) ImM
                    mac(are, term2(g, re_S(NN, -(m + mu)), s, re_S(NN, -(m - mu)), s * sg), xr);
                    mac(are, term2(g, im_S(NN, -(m + mu)), -s, im_S(NN, -(m - mu)), s * sg), xi);
                    if constexpr (m > 0) {
                        // Im row: (B + D) ReM + (A - C) ImM
                        mac(aim, term2(g, im_S(NN, -(m + mu)), s, im_S(NN, -(m - mu)), s * sg), xr);
                        mac(aim, term2(g, re_S(NN, -(m + mu)), s, re_S(NN, -(m - mu)), -s * sg), xi);
                    }
                });
                acc[ridx(l, m)] = are;
                if constexpr (m > 0) acc[ridx(l, -m)] = aim;
            });
        }
    });
}

// Kernel values g of order NN come from the block's LDS tile (component j
// at gcol[j * gstride]) of the stored quadrant ky, kz in [0, nf/2].  A
// frequency with ky > nf/2 reads ky' = nf - ky and negates the Im-part
// components (S(x, -y, z) = conj S); kz > nf/2 reads kz' = nf - kz and
// multiplies component (n, k) by (-1)^(n+|k|) (S_n^k(x, y, -z) =
// (-1)^(n+k) S_n^k).  flip = 1 for a mirrored ky, 2 for a mirrored kz.
template <int PO, int NN, int RS, int S, typename T>
struct M2LOrders {
    __device__ static __forceinline__ void run(const T *gcol, int gstride, int flip,
                                               const cplx<T> *mcol, int mstride, cplx<T> *acc) {
        if constexpr (subset_needs(PO, RS, S, NN)) {
            T g[2 * NN + 1];
            static_for<0, 2 * NN + 1>([&](auto ik) {
                constexpr int k = decltype(ik)::value;
                constexpr int kk = k - NN;
                constexpr int odd_z = (NN + (kk < 0 ? -kk : kk)) & 1;
                const int neg = ((flip & 1) && kk < 0) ^ ((flip & 2) && odd_z);
                const T v = gcol[(NN * NN + k) * gstride];
                g[k] = neg ? -v : v;
            });
            m2l_order<PO, NN, RS, S, T>(g, mcol, mstride, acc);
            // keep the next order's loads after this one's arithmetic so that
            // the (2p+1)^2 kernel values are never all live at once
            __builtin_amdgcn_sched_barrier(0);
        }
        M2LOrders<PO, NN + 1, RS, S, T>::run(gcol, gstride, flip, mcol, mstride, acc);
    }
};
template <int PO, int RS, int S, typename T>
struct M2LOrders<PO, 2 * PO + 1, RS, S, T> {
    __device__ static __forceinline__ void run(const T *, int, int, const cplx<T> *, int,
                                               cplx<T> *) {}
};

// Uniform corrections of a periodic system at the zero frequency (added to
// the final L~, i.e. after the i^(l mod 2) factor).  Adding c to every cell
// of L equals adding c * nf^3 to L~(k = 0).
struct DCCorr {
    bool on;
    double l00, l10, l11re, l11im;
};

// Rows of subset S in increasing row index, and their count.
__host__ __device__ constexpr int subset_rank(int PO, int RS, int S, int a) {
    int r = 0;
    for (int l = 0; l <= PO; ++l)
        for (int m = -l; m <= l; ++m)
            if (order_subset(PO, RS, l) == S && ridx(l, m) < a) ++r;
    return r;
}
__host__ __device__ constexpr int subset_rows_max(int PO, int RS) {
    int mx = 0;
    for (int S = 0; S < RS; ++S) {
        const int r = subset_rank(PO, RS, S, ridx(PO, PO) + 1);
        mx = r > mx ? r : mx;
    }
    return mx;
}

// Rows of subset S: M~ read from `mcol`; res[rank] = L~ = i^(l mod 2) acc
// plus the zero-frequency corrections.
template <int PO, int RS, int S, typename T>
__device__ __forceinline__ void m2l_rows(const T *gcol, int gstride, int flip,
                                         const cplx<T> *mcol, int stride, DCCorr dc,
                                         cplx<T> *res) {
    constexpr int P = nreal(PO);
    cplx<T> acc[P];
    static_for<0, P>([&](auto ia) { acc[decltype(ia)::value] = {T(0), T(0)}; });
    M2LOrders<PO, 0, RS, S, T>::run(gcol, gstride, flip, mcol, stride, acc);
    static_for<0, PO + 1>([&](auto il) {
        constexpr int l = decltype(il)::value;
        if constexpr (order_subset(PO, RS, l) == S) {
            static_for<-l, l + 1>([&](auto im) {
                constexpr int m = decltype(im)::value;
                constexpr int a = ridx(l, m);
                const cplx<T> v = acc[a];
                cplx<T> o = (l & 1) ? cplx<T>{-v.im, v.re} : v;
                if (dc.on) {
                    if constexpr (a == 0) o.re += T(dc.l00);
                    if constexpr (PO >= 1 && a == ridx(1, 0)) o.re += T(dc.l10);
                    if constexpr (PO >= 1 && a == ridx(1, 1)) o.re += T(dc.l11re);
                    if constexpr (PO >= 1 && a == ridx(1, -1)) o.re += T(dc.l11im);
                }
                res[subset_rank(PO, RS, S, a)] = o;
            });
        }
    });
}

// res of subset S to its rows of `ocol`.
template <int PO, int RS, int S, typename T>
__device__ __forceinline__ void m2l_put(const cplx<T> *res, cplx<T> *ocol, int stride,
                                        int odd = 0) {
    static_for<0, PO + 1>([&](auto il) {
        constexpr int l = decltype(il)::value;
        if constexpr (order_subset(PO, RS, l) == S) {
            static_for<-l, l + 1>([&](auto im) {
                constexpr int a = ridx(l, decltype(im)::value);
                ocol[a * stride + ((a & 1) ? odd : 0)] = res[subset_rank(PO, RS, S, a)];
            });
        }
    });
}

// Block = rs row subsets x (w columns x nf frequencies) threads (at most
// column_max_threads); with rs < kRowSplit each thread runs kRowSplit / rs
// of the subsets.  LDS: moment spectra buf[P][w][nf], local spectra
// obuf[P][w][nf] (buf itself when rs = kRowSplit: the results wait in
// registers for a barrier after the last read of buf) and the block's
// transfer-kernel tile gt[w][Q][nhp] (kz' in [0, nf/2], padded).
template <int PO, typename T>
__global__ void __launch_bounds__(PO <= 6 ? 512 : 256, (PO == 7 && sizeof(T) == 4) ? 2 : 1) k_column(int nz, int logn, int w, int rs, int ncol,
                                                int ngroups,
                                                const T *__restrict__ green,
                                                cplx<T> *__restrict__ spec,
                                                const cplx<T> *__restrict__ tw_g, int periodic,
                                                const double *__restrict__ qr2_partial,
                                                double *__restrict__ sums) {
    constexpr int P = nreal(PO);
    constexpr int Q = nreal(2 * PO);
    constexpr int RS = kRowSplit;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int nf = 1 << logn, nh = nf / 2 + 1, nhp = (nh + 3) & ~3, ls = lds_line(nf);
    const int nfreq = w * nf;
    const int cstride = w * ls;                 // component stride in buf / obuf
    const bool inplace = rs == RS;              // one row subset per thread
    cplx<T> *tw = (cplx<T> *)lds_raw;
    cplx<T> *buf = tw + nf / 2;
    cplx<T> *obuf = inplace ? buf : buf + P * cstride;
    T *gt = (T *)(obuf + P * cstride);
    // XCD-aware order: consecutive column groups stay on one XCD (blocks are
    // dealt round-robin over the 8 XCDs).
    const int per_xcd = (ngroups + 7) / 8;
    const int grp = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (grp >= ngroups) return;
    {
        // system blockIdx.y of a batch: spectra and sums at fixed strides
        const int64_t sy = blockIdx.y;
        spec += sy * P * nz * ncol;
        qr2_partial += sy * nz;
        sums += sy * 8;
    }
    const int col0 = grp * w;
    const int tid = threadIdx.x, nthr = blockDim.x;
    // Global reads: the twiddles, the transfer-kernel tile (reduced column
    // (ky', kx) of each block column is a contiguous, 16-byte aligned
    // [Q][nhp] slab) and the moment spectra of z < nz (the rest of the padded
    // column is zero).  Indices are clamped so that every load is
    // unconditional; the first batch of each kind is issued before any LDS
    // store, so small meshes take one round trip to HBM.
    const int logw = __builtin_ctz(w);          // w and nf are powers of two
    const int vec = 16 / (int)sizeof(T);
    const int slab = Q * nhp;                   // one column's tile
    const int per_col = slab / vec;
    const float inv_per_col = 1.0f / (float)per_col, inv_nh = 1.0f / (float)nh;
    const int gtotal = w * per_col;
    const float4 *green4 = (const float4 *)green;
    // tile element t: float4 r4 of block column ci; returns its index in the
    // stored transfer kernel and sets its LDS offset (clamped duplicates
    // rewrite the same value; columns past ncol fill slots never read)
    auto g_at = [&](int t, int &loff) {
        const int tc = t < gtotal ? t : gtotal - 1;
        const int ci = small_div(tc, inv_per_col), r4 = tc - ci * per_col;
        const int col = col0 + ci < ncol ? col0 + ci : ncol - 1;
        const int ky = small_div(col, inv_nh), kx = col - ky * nh;
        const int kyr = ky <= nf / 2 ? ky : nf - ky;
        loff = ci * slab + r4 * vec;
        return (kyr * nh + kx) * per_col + r4;
    };
    auto g_put = [&](int loff, float4 v) {
        T *dst = gt + loff;
        if (sizeof(T) == 4) {
            const float *vf = (const float *)&v;
            dst[0] = vf[0];
            dst[1] = vf[1];
            dst[2] = vf[2];
            dst[3] = vf[3];
        } else {
            const double *vd = (const double *)&v;
            dst[0] = vd[0];
            dst[1] = vd[1];
        }
    };
    // spectra: blockDim.x = rs * w * nf, so the elements of a thread share
    // block column s_i and z; the component advances by s_db per element
    const int s_i = tid & (w - 1);
    const int s_z = (tid >> logw) & (nf - 1);
    const int s_b0 = tid >> (logw + logn);
    const int s_db = nthr >> (logw + logn);
    const bool s_live = s_z < nz && col0 + s_i < ncol;
    const int s_g = (s_z < nz ? s_z : nz - 1) * ncol + (col0 + s_i < ncol ? col0 + s_i : ncol - 1);
    auto s_comp = [&](int u) { return s_b0 + u * s_db < P ? s_b0 + u * s_db : P - 1; };
    auto s_load = [&](int u) { return spec[s_comp(u) * nz * ncol + s_g]; };
    auto s_store = [&](int u, cplx<T> v) {
        buf[(s_comp(u) * w + s_i) * ls + s_z] = cplx<T>{s_live ? v.re : T(0), s_live ? v.im : T(0)};
    };
    constexpr int GB = kColumnLoadBatch, SB = 2 * kColumnLoadBatch;
    {
        const cplx<T> twv = tw_g[tid < nf / 2 ? tid : 0];   // nf/2 <= blockDim.x
        float4 gv[GB];
        int gl[GB];
        cplx<T> sv[SB];
#pragma unroll
        for (int u = 0; u < GB; ++u) gv[u] = green4[g_at(tid + u * nthr, gl[u])];
#pragma unroll
        for (int u = 0; u < SB; ++u) sv[u] = s_load(u);
        asm volatile("" ::"v"(twv.re), "v"(twv.im));
#pragma unroll
        for (int u = 0; u < GB; ++u) asm volatile("" ::"v"(gv[u].x), "v"(gv[u].y), "v"(gv[u].z), "v"(gv[u].w));
#pragma unroll
        for (int u = 0; u < SB; ++u) asm volatile("" ::"v"(sv[u].re), "v"(sv[u].im));
        if (tid < nf / 2) tw[tid] = twv;
#pragma unroll
        for (int u = 0; u < GB; ++u) g_put(gl[u], gv[u]);
#pragma unroll
        for (int u = 0; u < SB; ++u) s_store(u, sv[u]);
    }
    // remaining batches (large meshes)
    for (int base = tid + GB * nthr; base < gtotal; base += GB * nthr) {
        float4 gv[GB];
        int gl[GB];
#pragma unroll
        for (int u = 0; u < GB; ++u) gv[u] = green4[g_at(base + u * nthr, gl[u])];
#pragma unroll
        for (int u = 0; u < GB; ++u) asm volatile("" ::"v"(gv[u].x), "v"(gv[u].y), "v"(gv[u].z), "v"(gv[u].w));
#pragma unroll
        for (int u = 0; u < GB; ++u) g_put(gl[u], gv[u]);
    }
    for (int u0 = SB; s_b0 + u0 * s_db < P; u0 += SB) {
        cplx<T> sv[SB];
#pragma unroll
        for (int u = 0; u < SB; ++u) sv[u] = s_load(u0 + u);
#pragma unroll
        for (int u = 0; u < SB; ++u) asm volatile("" ::"v"(sv[u].re), "v"(sv[u].im));
#pragma unroll
        for (int u = 0; u < SB; ++u) s_store(u0 + u, sv[u]);
    }
    __syncthreads();
    fft_lines<T, false>(buf, logn, P * w, ls, 1, tw, tid, nthr);
    // M2L: thread = (row subset, frequency)
    const int sub = tid / nfreq, f = tid - sub * nfreq;
    const int i = f >> logn, pos = f & (nf - 1);
    const int col = col0 + i;
    const int kz = pos;
    DCCorr dcc = {false, 0.0, 0.0, 0.0, 0.0};
    if (periodic && col == 0 && kz == 0) {
        // zero frequency: M~_c(0) = sum over cells of M_c (real)
        const cplx<T> *m0 = buf + i * ls + pos;
        const double V = (double)nf * nf * nf;  // box volume in cell units (nf = n)
        const double pi = 3.14159265358979323846;
        double qr2 = 0.0;
        for (int z = 0; z < nz; ++z) qr2 += qr2_partial[z];
        const double m10 = PO >= 1 ? (double)m0[ridx(1, 0) * cstride].re : 0.0;
        const double m11 = PO >= 1 ? (double)m0[ridx(1, 1) * cstride].re : 0.0;
        const double m1m1 = PO >= 1 ? (double)m0[ridx(1, -1) * cstride].re : 0.0;
        // per-cell constants of the correction procedure, times nf^3 (= V)
        dcc.l00 = 2.0 * pi / (3.0 * V) * qr2 * V;
        dcc.l10 = 4.0 * pi / (3.0 * V) * m10 * V;
        dcc.l11re = 8.0 * pi / (3.0 * V) * m11 * V;
        dcc.l11im = -8.0 * pi / (3.0 * V) * m1m1 * V;
        dcc.on = true;
        if (sub == 0) sums[0] = (double)m0[0].re;  // total charge
    }
    {
        const bool live = col < ncol;
        const int ky = col / nh;
        const int kzr = kz <= nf / 2 ? kz : nf - kz;
        const int flip = (ky > nf / 2 ? 1 : 0) | (kz > nf / 2 ? 2 : 0);
        const T *gp = gt + i * slab + kzr;
        const int gstride = nhp;
        const cplx<T> *mp = buf + i * ls + pos;
        cplx<T> *op = obuf + i * ls + pos;
        // rs divides RS: every thread runs RS / rs passes (one when in place)
        for (int ss = sub; ss < RS; ss += rs) {
            cplx<T> res[subset_rows_max(PO, RS)];
            if (live) {
                switch (ss) {
                    case 0: m2l_rows<PO, RS, 0, T>(gp, gstride, flip, mp, cstride, dcc, res); break;
                    case 1: m2l_rows<PO, RS, 1, T>(gp, gstride, flip, mp, cstride, dcc, res); break;
                    case 2: m2l_rows<PO, RS, 2, T>(gp, gstride, flip, mp, cstride, dcc, res); break;
                    default: m2l_rows<PO, RS, 3, T>(gp, gstride, flip, mp, cstride, dcc, res); break;
                }
            }
            if (inplace) __syncthreads();       // every read of buf is done
            if (live) {
                switch (ss) {
                    case 0: m2l_put<PO, RS, 0, T>(res, op, cstride); break;
                    case 1: m2l_put<PO, RS, 1, T>(res, op, cstride); break;
                    case 2: m2l_put<PO, RS, 2, T>(res, op, cstride); break;
                    default: m2l_put<PO, RS, 3, T>(res, op, cstride); break;
                }
            }
        }
    }
    __syncthreads();
    fft_lines<T, true>(obuf, logn, P * w, ls, 1, tw, tid, nthr);
    // local spectra of z < nz back to HBM, LDS reads in batches; a thread's
    // elements share block column o_i and z, the component advances by o_da
    const int lognz = __builtin_ctz(nz);
    const int o_i = tid & (w - 1);
    const int o_z = (tid >> logw) & (nz - 1);
    const int o_a0 = tid >> (logw + lognz);
    const int o_da = nthr >> (logw + lognz);
    const bool o_live = col0 + o_i < ncol;
    for (int u0 = 0; o_a0 + u0 * o_da < P; u0 += kColumnLoadBatch) {
        cplx<T> v[kColumnLoadBatch];
#pragma unroll
        for (int u = 0; u < kColumnLoadBatch; ++u) {
            const int a = o_a0 + (u0 + u) * o_da < P ? o_a0 + (u0 + u) * o_da : P - 1;
            v[u] = obuf[(a * w + o_i) * ls + o_z];
        }
#pragma unroll
        for (int u = 0; u < kColumnLoadBatch; ++u) {
            const int a = o_a0 + (u0 + u) * o_da;
            if (a < P && o_live) spec[(a * nz + o_z) * ncol + col0 + o_i] = v[u];
        }
    }
}

// ------------------------------------------- streamed-kernel column variant
// For large FFT meshes the block's transfer-kernel tile (Q x (nf/2+1) values
// per column) would fill most of the LDS, leaving room for one block per CU.
// This variant reads the kernel values straight from the stored quadrant at
// the thread's frequency (lanes at consecutive kz read consecutive addresses
// of a column's [Q][nhp] slab), one order ahead of their use, so LDS holds
// only the twiddles and one column's spectra and several blocks share a CU.
// Each thread runs RSP of the kRowSplit row subsets one after another and
// keeps their results in registers until every read of the moment spectra
// is done; they then overwrite the spectra in place.
//
// Next order >= from whose kernel values subset S needs (2 PO + 1: none).
__host__ __device__ constexpr int next_order(int PO, int RS, int S, int from) {
    for (int NN = from; NN <= 2 * PO; ++NN)
        if (subset_needs(PO, RS, S, NN)) return NN;
    return 2 * PO + 1;
}

// The stored kernel values of one column: a buffer resource over the
// column's [Q][nhp] slab (block-uniform, so it lives in scalar registers),
// the byte offset of the thread's frequency, and the bytes between
// components -- every load then takes its address from one vector register
// plus a scalar offset, with no per-load address arithmetic.
struct GSlab {
    __amdgpu_buffer_rsrc_t rsrc;
    int voff, sstride;
};
template <typename T>
__device__ __forceinline__ GSlab make_gslab(const T *slab, int nvals, int kzr, int gstride) {
    // word 3: 32-bit data format, as raw (untyped) buffer loads require
    return GSlab{__builtin_amdgcn_make_buffer_rsrc((void *)slab, 0, nvals * (int)sizeof(T),
                                                   0x00020000),
                 kzr * (int)sizeof(T), gstride * (int)sizeof(T)};
}
template <typename T>
__device__ __forceinline__ T gslab_load(const GSlab &g, int j) {
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(g.rsrc, g.voff,
                                                                          j * g.sstride, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(g.rsrc, g.voff,
                                                                          j * g.sstride, 0));
}

// Stored kernel values of order NN (component j = NN^2 + k).
template <int NN, typename T>
__device__ __forceinline__ void load_order(const GSlab &gs, T *raw) {
    static_for<0, 2 * NN + 1>([&](auto ik) {
        constexpr int k = decltype(ik)::value;
        raw[k] = gslab_load<T>(gs, NN * NN + k);
    });
}

// Orders NN, next_order(NN + 1), ... of subset S: the values of the next
// needed order are loaded before this order's products are issued.
template <int PO, int NN, int RS, int S, typename T>
struct M2LOrdersG {
    __device__ static __forceinline__ void run(const GSlab &gs, int flip,
                                               const cplx<T> *mcol, int mstride, cplx<T> *acc,
                                               const T *raw, int odd) {
        constexpr int NX = next_order(PO, RS, S, NN + 1);
        constexpr int NXL = NX <= 2 * PO ? 2 * NX + 1 : 1;
        T nxt[NXL];
        if constexpr (NX <= 2 * PO) load_order<NX, T>(gs, nxt);
        T g[2 * NN + 1];
        static_for<0, 2 * NN + 1>([&](auto ik) {
            constexpr int k = decltype(ik)::value;
            constexpr int kk = k - NN;
            constexpr int odd_z = (NN + (kk < 0 ? -kk : kk)) & 1;
            const int neg = ((flip & 1) && kk < 0) ^ ((flip & 2) && odd_z);
            g[k] = neg ? -raw[k] : raw[k];
        });
        m2l_order<PO, NN, RS, S, T>(g, mcol, mstride, acc, odd);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (NX <= 2 * PO)
            M2LOrdersG<PO, NX, RS, S, T>::run(gs, flip, mcol, mstride, acc, nxt, odd);
    }
};

// As m2l_rows, with the kernel values streamed from global memory.
template <int PO, int RS, int S, typename T>
__device__ __forceinline__ void m2l_rows_g(const GSlab &gs, int flip,
                                           const cplx<T> *mcol, int stride, DCCorr dc,
                                           cplx<T> *res, int odd) {
    constexpr int P = nreal(PO);
    constexpr int N0 = next_order(PO, RS, S, 0);
    cplx<T> acc[P];
    static_for<0, P>([&](auto ia) { acc[decltype(ia)::value] = {T(0), T(0)}; });
    if constexpr (N0 <= 2 * PO) {
        T raw[2 * N0 + 1];
        load_order<N0, T>(gs, raw);
        M2LOrdersG<PO, N0, RS, S, T>::run(gs, flip, mcol, stride, acc, raw, odd);
    }
    static_for<0, PO + 1>([&](auto il) {
        constexpr int l = decltype(il)::value;
        if constexpr (order_subset(PO, RS, l) == S) {
            static_for<-l, l + 1>([&](auto im) {
                constexpr int m = decltype(im)::value;
                constexpr int a = ridx(l, m);
                const cplx<T> v = acc[a];
                cplx<T> o = (l & 1) ? cplx<T>{-v.im, v.re} : v;
                if (dc.on) {
                    if constexpr (a == 0) o.re += T(dc.l00);
                    if constexpr (PO >= 1 && a == ridx(1, 0)) o.re += T(dc.l10);
                    if constexpr (PO >= 1 && a == ridx(1, 1)) o.re += T(dc.l11re);
                    if constexpr (PO >= 1 && a == ridx(1, -1)) o.re += T(dc.l11im);
                }
                res[subset_rank(PO, RS, S, a)] = o;
            });
        }
    });
}

// One block per column; NSUB = kRowSplit / RSP threads per frequency, so
// NSUB * nf threads (nf = 2^LOGN = 64 or 128, a compile-time size: the
// index arithmetic folds and the kernel needs fewer registers).  LDS:
// twiddles and the column's spectra buf[P][nf] in the swizzled layout.  Open
// boundaries (nz = nf / 2) skip the zero half of the forward transforms and
// the discarded half of the inverse ones.
template <int PO, typename T, int RSP, int LOGN>
__global__ void __launch_bounds__((kRowSplit / RSP) * 128, RSP == 2 ? (sizeof(T) == 4 ? 3 : 2) : (RSP == 4 ? 2 : 1))
    k_column_g(int nz, int ncol, int ngroups, const T *__restrict__ green,
               cplx<T> *__restrict__ spec, const cplx<T> *__restrict__ tw_g, int periodic,
               const double *__restrict__ qr2_partial, double *__restrict__ sums) {
    constexpr int P = nreal(PO);
    constexpr int Q = nreal(2 * PO);
    constexpr int RS = kRowSplit;
    constexpr int NSUB = RS / RSP;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    constexpr int logn = LOGN, nf = 1 << LOGN, nh = nf / 2 + 1, nhp = (nh + 3) & ~3, ls = nf;
    const bool half = 2 * nz == nf;
    cplx<T> *tw = (cplx<T> *)lds_raw;
    cplx<T> *buf = tw + nf;
    // XCD-aware order: consecutive columns stay on one XCD (blocks are dealt
    // round-robin over the 8 XCDs)
    const int per_xcd = (ngroups + 7) / 8;
    const int col = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (col >= ngroups) return;
    {
        const int64_t sy = blockIdx.y;
        spec += sy * P * nz * ncol;
        qr2_partial += sy * nz;
        sums += sy * 8;
    }
    const int tid = threadIdx.x;
    constexpr int nthr = NSUB * nf;
    // spectra of z < nz: thread element u is component s_b0 + u * s_db at z = s_z
    const int s_z = tid & (nf - 1);
    const int s_b0 = tid >> logn;
    constexpr int s_db = nthr >> logn;
    const bool s_live = s_z < nz;
    const int s_g = (s_z < nz ? s_z : nz - 1) * ncol + col;
    auto s_comp = [&](int u) { return s_b0 + u * s_db < P ? s_b0 + u * s_db : P - 1; };
    constexpr int SB = 2 * kColumnLoadBatch;
    {
        // the zero half of an open column is never read (pruned transform)
        if (s_live) {
            for (int u0 = 0; s_b0 + u0 * s_db < P; u0 += SB) {
                cplx<T> sv[SB];
#pragma unroll
                for (int u = 0; u < SB; ++u) sv[u] = spec[s_comp(u0 + u) * nz * ncol + s_g];
#pragma unroll
                for (int u = 0; u < SB; ++u) asm volatile("" ::"v"(sv[u].re), "v"(sv[u].im));
#pragma unroll
                for (int u = 0; u < SB; ++u) {
                    const int c = s_comp(u0 + u);
                    buf[c * ls + cpos(c, s_z)] = sv[u];
                }
            }
        }
        fill_twiddles<T>(tw, tw_g, nf, tid, nthr);
    }
    __syncthreads();
    fft_col_rt<T, false, nf>(buf, half, P, tw, tid, nthr);
    // M2L: thread = (row-subset group sub, frequency kz)
    const int sub = tid >> logn, kz = tid & (nf - 1);
    DCCorr dcc = {false, 0.0, 0.0, 0.0, 0.0};
    if (periodic && col == 0 && kz == 0) {
        // zero frequency: M~_c(0) = sum over cells of M_c (real)
        auto m0 = [&](int c) { return (double)buf[c * ls + cpos(c, 0)].re; };
        const double V = (double)nf * nf * nf;  // box volume in cell units (nf = n)
        const double pi = 3.14159265358979323846;
        double qr2 = 0.0;
        for (int z = 0; z < nz; ++z) qr2 += qr2_partial[z];
        const double m10 = PO >= 1 ? m0(ridx(1, 0)) : 0.0;
        const double m11 = PO >= 1 ? m0(ridx(1, 1)) : 0.0;
        const double m1m1 = PO >= 1 ? m0(ridx(1, -1)) : 0.0;
        dcc.l00 = 2.0 * pi / (3.0 * V) * qr2 * V;
        dcc.l10 = 4.0 * pi / (3.0 * V) * m10 * V;
        dcc.l11re = 8.0 * pi / (3.0 * V) * m11 * V;
        dcc.l11im = -8.0 * pi / (3.0 * V) * m1m1 * V;
        dcc.on = true;
        if (sub == 0) sums[0] = m0(0);  // total charge
    }
    {
        const int ky = small_div(col, 1.0f / (float)nh), kx = col - ky * nh;
        const int kyr = ky <= nf / 2 ? ky : nf - ky;
        const int kzr = kz <= nf / 2 ? kz : nf - kz;
        const int flip = (ky > nf / 2 ? 1 : 0) | (kz > nf / 2 ? 2 : 0);
        const GSlab gs = make_gslab<T>(green + (int64_t)(kyr * nh + kx) * Q * nhp, Q * nhp, kzr, nhp);
        // row b of the thread's frequency sits at buf + b * ls + kpos (+ odd
        // for odd b)
        const int kpos = cpos(0, kz), odd = cpos(1, kz) - kpos;
        const cplx<T> *mp = buf + kpos;
        cplx<T> res[RSP][subset_rows_max(PO, RS)];
        static_for<0, RSP>([&](auto ik) {
            constexpr int k = decltype(ik)::value;
            static_for<0, NSUB>([&](auto is) {
                constexpr int s = decltype(is)::value;
                if (sub == s)
                    m2l_rows_g<PO, RS, k * NSUB + s, T>(gs, flip, mp, ls, dcc, res[k], odd);
            });
        });
        __syncthreads();  // every read of the moment spectra is done
        static_for<0, RSP>([&](auto ik) {
            constexpr int k = decltype(ik)::value;
            static_for<0, NSUB>([&](auto is) {
                constexpr int s = decltype(is)::value;
                if (sub == s) m2l_put<PO, RS, k * NSUB + s, T>(res[k], buf + kpos, ls, odd);
            });
        });
    }
    __syncthreads();
    fft_col_rt<T, true, nf>(buf, half, P, tw, tid, nthr);
    // local spectra of z < nz back to HBM, LDS reads in batches
    const int lognz = __builtin_ctz(nz);
    const int o_z = tid & (nz - 1);
    const int o_a0 = tid >> lognz;
    const int o_da = nthr >> lognz;
    for (int u0 = 0; o_a0 + u0 * o_da < P; u0 += kColumnLoadBatch) {
        cplx<T> v[kColumnLoadBatch];
#pragma unroll
        for (int u = 0; u < kColumnLoadBatch; ++u) {
            const int a = o_a0 + (u0 + u) * o_da < P ? o_a0 + (u0 + u) * o_da : P - 1;
            v[u] = buf[a * ls + cpos(a, o_z)];
        }
#pragma unroll
        for (int u = 0; u < kColumnLoadBatch; ++u) {
            const int a = o_a0 + (u0 + u) * o_da;
            if (a < P) spec[(a * nz + o_z) * ncol + col] = v[u];
        }
    }
}

// --------------------------------------------------------------- launcher
inline int column_ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

template <int PO, typename T, int RSP, int LOGN>
hipError_t column_launch_g(const FFTArgs &a, hipStream_t s) {
    constexpr int nf = 1 << LOGN, nh = nf / 2 + 1, ncol = nf * nh;
    const size_t lds = column_g_lds(PO, nf, sizeof(T));
    if (lds == 0 || a.nf != nf || (a.n != nf && 2 * a.n != nf)) return hipErrorInvalidValue;
    const int threads = (kRowSplit / RSP) * nf;
    if (threads < 64) return hipErrorInvalidValue;
    const int grid = ((ncol + 7) / 8) * 8;
    hipError_t e =
        lds <= 65536 ? hipSuccess : set_max_lds((const void *)k_column_g<PO, T, RSP, LOGN>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_column_g<PO, T, RSP, LOGN>), dim3(grid, a.nsys > 0 ? a.nsys : 1),
                       dim3(threads), lds, s, a.n, ncol, ncol, (const T *)a.green,
                       (cplx<T> *)a.spec, (const cplx<T> *)a.tw, a.open ? 0 : 1, a.qr2_partial,
                       a.sums);
    return hipGetLastError();
}

// The streamed form at the plan's FFT size (64 or 128 points; FP64 plans
// stop at 64).
template <int PO, typename T, int RSP>
hipError_t column_launch_g(const FFTArgs &a, hipStream_t s) {
    if constexpr (sizeof(T) == 4)
        if (a.nf == 128) return column_launch_g<PO, T, RSP, 7>(a, s);
    if (a.nf == 64) return column_launch_g<PO, T, RSP, 6>(a, s);
    return hipErrorInvalidValue;
}

template <int PO, typename T>
hipError_t column_launch(const FFTArgs &a, hipStream_t s) {
    const int kind = a.col_kernel > 0 ? a.col_kernel : column_default_kernel(PO, a.nf, sizeof(T));
    switch (kind) {
        case PMMM_COLUMN_STREAM_1: return column_launch_g<PO, T, 1>(a, s);
        case PMMM_COLUMN_STREAM_2:
            if constexpr (PO < 9) return column_launch_g<PO, T, 2>(a, s);
            return hipErrorInvalidValue;
        case PMMM_COLUMN_STREAM_4:
            if constexpr (PO < 7) return column_launch_g<PO, T, 4>(a, s);
            return hipErrorInvalidValue;
        case PMMM_COLUMN_TILE: break;
        default: return hipErrorInvalidValue;
    }
    const int nf = a.nf, logn = column_ilog2(nf), nh = nf / 2 + 1, ncol = nf * nh;
    int w = 1, rs = 1;
    size_t lds = column_shape(PO, nf, sizeof(T), &w, &rs);
    if (lds == 0) return hipErrorInvalidValue;
    if (a.col_w > 0 && a.col_w < w) {
        // a narrower tuned shape (always fits when the widest one does)
        w = a.col_w;
        lds = column_lds_w(PO, nf, sizeof(T), w, &rs);
        if (lds == 0) return hipErrorInvalidValue;
    }
    if ((w & (w - 1)) != 0) return hipErrorInvalidValue;   // the kernel splits indices by shifts
    const int threads = rs * w * nf;
    const int ngroups = (ncol + w - 1) / w;
    const int grid = ((ngroups + 7) / 8) * 8;
    hipError_t e = lds <= 65536 ? hipSuccess : set_max_lds((const void *)k_column<PO, T>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_column<PO, T>), dim3(grid, a.nsys > 0 ? a.nsys : 1), dim3(threads), lds, s, a.n, logn, w, rs,
                       ncol, ngroups, (const T *)a.green, (cplx<T> *)a.spec,
                       (const cplx<T> *)a.tw, a.open ? 0 : 1, a.qr2_partial, a.sums);
    return hipGetLastError();
}

}  // namespace pmmm
