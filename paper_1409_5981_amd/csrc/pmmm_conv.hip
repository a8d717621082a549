// FFT convolution of the moment meshes with the transfer kernel (Sec. 2.1,
// the four-line FFT procedure: forward transforms of the (p+1)^2 moment
// meshes, element-wise M2L in wave space, inverse transforms).
//
// Three launches, all LDS-resident:
//   k_plane_fwd  one z-plane of one component: real-to-complex FFT along x
//                (two real rows packed as one complex row) then a complex
//                FFT along y.  Open boundaries read the n x n data rows and
//                treat the rest of the 2n x 2n plane as zeros (App. C).
//   k_column     w (ky, kx) columns of ALL components: complex FFT along z,
//                the M2L of eq. realmatrix at every frequency of the columns,
//                inverse FFT along z.  Only z < n is read and written back
//                (the rest of the padded mesh is zero on input and aliasing
//                on output for open boundaries).
//   k_plane_inv  inverse of k_plane_fwd restricted to the y < n, x < n
//                block, scaled by 1/nf^3.
// The 3-D spectrum therefore never reaches HBM in full: the buffer between
// the kernels holds [P][n][nf][nf/2+1] complex values.
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
#include "pmmm_internal.h"

namespace pmmm {

// ------------------------------------------------------------------ planes
template <typename T>
__global__ void __launch_bounds__(256) k_plane_fwd(int nin, int logn,
                                                   const T *__restrict__ M,
                                                   cplx<T> *__restrict__ spec,
                                                   const cplx<T> *__restrict__ tw_g) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int nf = 1 << logn, nh = nf / 2 + 1, npair = nin / 2;
    cplx<T> *tw = (cplx<T> *)lds_raw;
    cplx<T> *buf1 = tw + nf / 2;           // [npair][nf]
    cplx<T> *buf2 = buf1 + npair * nf;     // [nf][nh]
    const int z = blockIdx.x, c = blockIdx.y;
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int k = tid; k < nf / 2; k += nthr) tw[k] = tw_g[k];
    const T *plane = M + ((int64_t)c * nin + z) * nin * nin;
    for (int idx = tid; idx < npair * nf; idx += nthr) {
        const int j = idx >> logn, x = idx & (nf - 1);
        cplx<T> v = {T(0), T(0)};
        if (x < nin) {
            v.re = plane[(2 * j) * nin + x];
            v.im = plane[(2 * j + 1) * nin + x];
        }
        buf1[idx] = v;
    }
    __syncthreads();
    lds_fft_dif<T, false>(buf1, logn, npair, nf, 1, tw, tid, nthr);
    for (int idx = tid; idx < nf * nh; idx += nthr) {
        const int y = idx / nh, k = idx - y * nh;
        cplx<T> v = {T(0), T(0)};
        if (y < nin) {
            const cplx<T> *row = buf1 + (y >> 1) * nf;
            const cplx<T> zk = row[bitrev(k & (nf - 1), logn)];
            const cplx<T> zm = row[bitrev((nf - k) & (nf - 1), logn)];
            if ((y & 1) == 0) {
                v.re = T(0.5) * (zk.re + zm.re);
                v.im = T(0.5) * (zk.im - zm.im);
            } else {
                v.re = T(0.5) * (zk.im + zm.im);
                v.im = T(-0.5) * (zk.re - zm.re);
            }
        }
        buf2[idx] = v;
    }
    __syncthreads();
    lds_fft_dif<T, false>(buf2, logn, nh, 1, nh, tw, tid, nthr);
    cplx<T> *out = spec + ((int64_t)c * nin + z) * nf * nh;
    for (int idx = tid; idx < nf * nh; idx += nthr) {
        const int pos = idx / nh, k = idx - pos * nh;
        out[bitrev(pos, logn) * nh + k] = buf2[idx];
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_plane_inv(int nout, int logn,
                                                   const cplx<T> *__restrict__ spec,
                                                   T *__restrict__ L,
                                                   const cplx<T> *__restrict__ tw_g, T scale) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int nf = 1 << logn, nh = nf / 2 + 1, npair = nout / 2;
    cplx<T> *tw = (cplx<T> *)lds_raw;
    cplx<T> *buf2 = tw + nf / 2;           // [nf][nh]
    cplx<T> *buf1 = buf2 + nf * nh;        // [npair][nf]
    const int z = blockIdx.x, c = blockIdx.y;
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int k = tid; k < nf / 2; k += nthr) tw[k] = tw_g[k];
    const cplx<T> *in = spec + ((int64_t)c * nout + z) * nf * nh;
    for (int idx = tid; idx < nf * nh; idx += nthr) buf2[idx] = in[idx];
    __syncthreads();
    lds_fft_dif<T, true>(buf2, logn, nh, 1, nh, tw, tid, nthr);
    for (int idx = tid; idx < npair * nf; idx += nthr) {
        const int j = idx >> logn, k = idx & (nf - 1);
        const cplx<T> *ra = buf2 + bitrev(2 * j, logn) * nh;
        const cplx<T> *rb = buf2 + bitrev(2 * j + 1, logn) * nh;
        cplx<T> A, B;
        if (k <= nf / 2) {
            A = ra[k];
            B = rb[k];
        } else {
            A = ra[nf - k];
            B = rb[nf - k];
            A.im = -A.im;
            B.im = -B.im;
        }
        buf1[idx] = {A.re - B.im, A.im + B.re};
    }
    __syncthreads();
    lds_fft_dif<T, true>(buf1, logn, npair, nf, 1, tw, tid, nthr);
    T *plane = L + ((int64_t)c * nout + z) * nout * nout;
    for (int idx = tid; idx < nout * nout; idx += nthr) {
        const int y = idx / nout, x = idx - y * nout;
        const cplx<T> v = buf1[(y >> 1) * nf + bitrev(x, logn)];
        plane[idx] = ((y & 1) ? v.im : v.re) * scale;
    }
}

// ---------------------------------------------------------------- columns
// Value of Re S_n^k and Im S_n^k (any k) as sign * g[n + idx] where g holds
// the stored components of order n at offsets k + n (k = -n..n): offset n+k
// (k >= 0) is Re S_n^k, offset n-k (k > 0) is Im S_n^k.  sign 0 = zero.
struct Term {
    int off;
    int sgn;
};
__host__ __device__ constexpr Term re_S(int n, int k) {
    return (k > n || k < -n) ? Term{0, 0}
           : (k >= 0)        ? Term{n + k, 1}
                             : Term{n - k, ((-k) & 1) ? -1 : 1};
}
__host__ __device__ constexpr Term im_S(int n, int k) {
    return (k > n || k < -n || k == 0) ? Term{0, 0}
           : (k > 0)                   ? Term{n - k, 1}
                                       : Term{n + k, ((-k) & 1) ? 1 : -1};
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

// acc[a] += sum_b t_ab(g of order nn) * Mh[b] for all (l, lam) with l + lam = nn.
template <int PO, int NN, typename T>
__device__ __forceinline__ void m2l_order(const T *g, const cplx<T> *Mh, cplx<T> *acc) {
    constexpr int lo = NN - PO > 0 ? NN - PO : 0;
    constexpr int hi = NN < PO ? NN : PO;
#pragma unroll
    for (int l = lo; l <= hi; ++l) {
        const int lam = NN - l;
        const int s = ((l & 1) && (lam & 1)) ? -1 : 1;
#pragma unroll
        for (int m = 0; m <= l; ++m) {
            cplx<T> are = acc[ridx(l, m)];
            cplx<T> aim = (m > 0) ? acc[ridx(l, -m)] : cplx<T>{T(0), T(0)};
            // mu = 0 column: G^{m,0} = S_nn^{-m}
            {
                const cplx<T> x = Mh[ridx(lam, 0)];
                const T A = term2(g, re_S(NN, -m), s, Term{0, 0}, 0);
                mac(are, A, x);
                if (m > 0) {
                    const T B = term2(g, im_S(NN, -m), s, Term{0, 0}, 0);
                    mac(aim, B, x);
                }
            }
#pragma unroll
            for (int mu = 1; mu <= lam; ++mu) {
                const cplx<T> xr = Mh[ridx(lam, mu)];
                const cplx<T> xi = Mh[ridx(lam, -mu)];
                const int sg = (mu & 1) ? -1 : 1;  // (-1)^mu of C and D
                // Re row: (A + C) ReM - (B - D) ImM
                const T apc = term2(g, re_S(NN, -(m + mu)), s, re_S(NN, -(m - mu)), s * sg);
                const T bmd = term2(g, im_S(NN, -(m + mu)), -s, im_S(NN, -(m - mu)), s * sg);
                mac(are, apc, xr);
                mac(are, bmd, xi);
                if (m > 0) {
                    // Im row: (B + D) ReM + (A - C) ImM
                    const T bpd = term2(g, im_S(NN, -(m + mu)), s, im_S(NN, -(m - mu)), s * sg);
                    const T amc = term2(g, re_S(NN, -(m + mu)), s, re_S(NN, -(m - mu)), -s * sg);
                    mac(aim, bpd, xr);
                    mac(aim, amc, xi);
                }
            }
            acc[ridx(l, m)] = are;
            if (m > 0) acc[ridx(l, -m)] = aim;
        }
    }
}

template <int PO, int NN, typename T>
struct M2LOrders {
    __device__ static __forceinline__ void run(const T *__restrict__ gcol, int nf, int kz,
                                               const cplx<T> *Mh, cplx<T> *acc) {
        T g[2 * NN + 1];
#pragma unroll
        for (int k = 0; k <= 2 * NN; ++k) g[k] = gcol[(int64_t)(NN * NN + k) * nf + kz];
        m2l_order<PO, NN, T>(g, Mh, acc);
        M2LOrders<PO, NN + 1, T>::run(gcol, nf, kz, Mh, acc);
    }
};
template <int PO, typename T>
struct M2LOrders<PO, 2 * PO + 1, T> {
    __device__ static __forceinline__ void run(const T *__restrict__, int, int, const cplx<T> *,
                                               cplx<T> *) {}
};

template <int PO, typename T>
__global__ void __launch_bounds__(256) k_column(int nz, int logn, int w, int ncol, int ngroups,
                                                const T *__restrict__ green,
                                                cplx<T> *__restrict__ spec,
                                                const cplx<T> *__restrict__ tw_g) {
    constexpr int P = nreal(PO);
    constexpr int Q = nreal(2 * PO);
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int nf = 1 << logn;
    cplx<T> *tw = (cplx<T> *)lds_raw;
    cplx<T> *buf = tw + nf / 2;  // [P][w][nf]
    // XCD-aware order: consecutive column groups stay on one XCD (blocks are
    // dealt round-robin over the 8 XCDs).
    const int per_xcd = (ngroups + 7) / 8;
    const int grp = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (grp >= ngroups) return;
    const int col0 = grp * w;
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int k = tid; k < nf / 2; k += nthr) tw[k] = tw_g[k];
    const int64_t zstride = (int64_t)ncol;
    // load z < nz, zero the padding
    for (int idx = tid; idx < P * nf * w; idx += nthr) {
        const int i = idx % w;
        const int rest = idx / w;
        const int zz = rest & (nf - 1);
        const int b = rest >> logn;
        const int col = col0 + i;
        cplx<T> v = {T(0), T(0)};
        if (zz < nz && col < ncol) v = spec[((int64_t)b * nz + zz) * zstride + col];
        buf[(b * w + i) * nf + zz] = v;
    }
    __syncthreads();
    lds_fft_dif<T, false>(buf, logn, P * w, nf, 1, tw, tid, nthr);
    // M2L, one thread per frequency of the block's columns
    for (int t = tid; t < w * nf; t += nthr) {
        const int i = t >> logn, pos = t & (nf - 1);
        const int col = col0 + i;
        if (col >= ncol) continue;
        const int kz = bitrev(pos, logn);
        cplx<T> Mh[P], acc[P];
#pragma unroll
        for (int lam = 0; lam <= PO; ++lam) {
#pragma unroll
            for (int mu = -lam; mu <= lam; ++mu) {
                const int b = ridx(lam, mu);
                const cplx<T> v = buf[(b * w + i) * nf + pos];
                Mh[b] = (lam & 1) ? cplx<T>{-v.im, v.re} : v;  // i^(lam mod 2) M~
                acc[b] = {T(0), T(0)};
            }
        }
        M2LOrders<PO, 0, T>::run(green + (int64_t)col * Q * nf, nf, kz, Mh, acc);
#pragma unroll
        for (int l = 0; l <= PO; ++l) {
#pragma unroll
            for (int m = -l; m <= l; ++m) {
                const int a = ridx(l, m);
                const cplx<T> v = acc[a];
                buf[(a * w + i) * nf + pos] = (l & 1) ? cplx<T>{-v.im, v.re} : v;
            }
        }
    }
    __syncthreads();
    lds_fft_dit<T, true>(buf, logn, P * w, nf, 1, tw, tid, nthr);
    for (int idx = tid; idx < P * nz * w; idx += nthr) {
        const int i = idx % w;
        const int rest = idx / w;
        const int zz = rest % nz;
        const int a = rest / nz;
        const int col = col0 + i;
        if (col < ncol) spec[((int64_t)a * nz + zz) * zstride + col] = buf[(a * w + i) * nf + zz];
    }
}

// --------------------------------------------------------------- launcher
static int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

template <typename Kern>
static hipError_t ensure_lds(Kern k, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

template <int PO, typename T>
static hipError_t column_launch(const FFTArgs &a, hipStream_t s) {
    constexpr int P = nreal(PO);
    const int nf = a.nf, logn = ilog2(nf), nh = nf / 2 + 1, ncol = nf * nh;
    const size_t csz = sizeof(cplx<T>);
    const size_t budget = 80 * 1024;
    int w = 256 / nf;
    if (w < 1) w = 1;
    while (w > 1 && (size_t)P * w * nf * csz + nf / 2 * csz > budget) w >>= 1;
    // prefer more, narrower blocks while the mesh has few columns
    while (w > 1 && (ncol + w - 1) / w < 512) w >>= 1;
    const int threads = (w * nf < 64) ? 64 : (w * nf > 256 ? 256 : w * nf);
    const int ngroups = (ncol + w - 1) / w;
    const int grid = ((ngroups + 7) / 8) * 8;
    const size_t lds = (size_t)P * w * nf * csz + nf / 2 * csz;
    hipError_t e = ensure_lds(k_column<PO, T>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_column<PO, T>), dim3(grid), dim3(threads), lds, s, a.n, logn, w, ncol,
                       ngroups, (const T *)a.green, (cplx<T> *)a.spec,
                       (const cplx<T> *)a.tw);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_convolution(const FFTArgs &a, hipStream_t s) {
    const int P = nreal(a.p);
    const int nf = a.nf, logn = ilog2(nf), nh = nf / 2 + 1, n = a.n;
    const size_t csz = sizeof(cplx<T>);
    const size_t lds_plane = (size_t)(nf / 2 + (n / 2) * nf + nf * nh) * csz;
    hipError_t e = ensure_lds(k_plane_fwd<T>, lds_plane);
    if (e != hipSuccess) return e;
    e = ensure_lds(k_plane_inv<T>, lds_plane);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_plane_fwd<T>, dim3(n, P), dim3(256), lds_plane, s, n, logn,
                       (const T *)a.M, (cplx<T> *)a.spec, (const cplx<T> *)a.tw);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (a.p) {
        case 0: e = column_launch<0, T>(a, s); break;
        case 1: e = column_launch<1, T>(a, s); break;
        case 2: e = column_launch<2, T>(a, s); break;
        case 3: e = column_launch<3, T>(a, s); break;
        case 4: e = column_launch<4, T>(a, s); break;
        case 5: e = column_launch<5, T>(a, s); break;
        case 6: e = column_launch<6, T>(a, s); break;
        case 7: e = column_launch<7, T>(a, s); break;
        case 8: e = column_launch<8, T>(a, s); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    const T scale = T(1.0 / ((double)nf * nf * nf));
    hipLaunchKernelGGL(k_plane_inv<T>, dim3(n, P), dim3(256), lds_plane, s, n, logn,
                       (const cplx<T> *)a.spec, (T *)a.L, (const cplx<T> *)a.tw, scale);
    return hipGetLastError();
}

template hipError_t launch_convolution<float>(const FFTArgs &, hipStream_t);
template hipError_t launch_convolution<double>(const FFTArgs &, hipStream_t);

}  // namespace pmmm
