// Periodic meshes whose edge n is not a power of two (Sec. 1: the mesh may
// be any product of three integers).  The power-of-two transforms do not
// apply, so the convolution of eq. pmmm runs here as
//   forward : real DFT along x (n -> n/2 + 1 frequencies), complex DFTs
//             along y and z, in place on spec [P][z][y][kx];
//   M2L     : the real-matrix form of eq. realmatrix per frequency, from the
//             folded transfer kernel, into spec2, plus the zero-frequency
//             corrections of App. B (correction procedure);
//   inverse : complex DFTs along z and y on spec2, then the real inverse
//             along x into L, scaled by 1/n^3.
// Every DFT is a direct sum over the line (n <= kGenericMaxN), with the
// twiddle e^(-+2 pi i j k / n) read from a table of the n roots of unity at
// index (j k) mod n.  A block stages a tile of lines in LDS, so that the
// loads and stores stay coalesced along the contiguous axis.  The plan-time
// FP64 line DFT of the transfer kernel is here too.
#include "pmmm_internal.h"

namespace pmmm {
namespace {

constexpr int kGenThreads = 256;
constexpr int kGenTile = 32;    // contiguous lines per block (complex passes)
constexpr int kGenRows = 8;     // rows per block (real x passes)

// Complex DFT of lines with elements j at base + j * se; line (o, i) starts
// at o * so + i, i in [0, inner).  Block: one o, kGenTile consecutive i.
template <typename T, bool INV>
__global__ __launch_bounds__(kGenThreads) void k_gen_dft_c(cplx<T> *__restrict__ data, int n,
                                                           int64_t inner, int64_t so, int64_t se,
                                                           const cplx<T> *__restrict__ w_g) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    cplx<T> *w = (cplx<T> *)lds_raw;
    cplx<T> *buf = w + n;                       // [n][kGenTile]
    const int tid = threadIdx.x;
    const int64_t o = blockIdx.y, i0 = (int64_t)blockIdx.x * kGenTile;
    const int ni = (int)(inner - i0 < kGenTile ? inner - i0 : kGenTile);
    cplx<T> *base = data + o * so + i0;
    for (int k = tid; k < n; k += kGenThreads) {
        cplx<T> v = w_g[k];
        if (INV) v.im = -v.im;
        w[k] = v;
    }
    for (int e = tid; e < n * kGenTile; e += kGenThreads) {
        const int j = e / kGenTile, ii = e - j * kGenTile;
        if (ii < ni) buf[e] = base[(int64_t)j * se + ii];
    }
    __syncthreads();
    const int ii = tid % kGenTile;
    if (ii < ni) {
        for (int k = tid / kGenTile; k < n; k += kGenThreads / kGenTile) {
            T re = T(0), im = T(0);
            int m = 0;                          // (j k) mod n
            for (int j = 0; j < n; ++j) {
                const cplx<T> x = buf[j * kGenTile + ii], t = w[m];
                // one FMA per multiply-add into the running sums
                re = fma(x.re, t.re, re);
                re = fma(-x.im, t.im, re);
                im = fma(x.re, t.im, im);
                im = fma(x.im, t.re, im);
                m += k;
                if (m >= n) m -= n;
            }
            base[(int64_t)k * se + ii] = {re, im};
        }
    }
}

// Real DFT along x: rows r of n reals (M[r n + x]) to n/2 + 1 frequencies
// (spec[r nh + k]).  Block: kGenRows rows.
template <typename T>
__global__ __launch_bounds__(kGenThreads) void k_gen_dft_x_fwd(const T *__restrict__ M, int64_t rows,
                                                               int n, const cplx<T> *__restrict__ w_g,
                                                               cplx<T> *__restrict__ spec) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    cplx<T> *w = (cplx<T> *)lds_raw;
    T *buf = (T *)(w + n);                      // [kGenRows][n]
    const int tid = threadIdx.x, nh = n / 2 + 1;
    const int64_t r0 = (int64_t)blockIdx.x * kGenRows;
    const int nr = (int)(rows - r0 < kGenRows ? rows - r0 : kGenRows);
    for (int k = tid; k < n; k += kGenThreads) w[k] = w_g[k];
    for (int e = tid; e < nr * n; e += kGenThreads) buf[e] = M[r0 * n + e];
    __syncthreads();
    for (int e = tid; e < nr * nh; e += kGenThreads) {
        const int r = e / nh, k = e - r * nh;
        const T *x = buf + r * n;
        T re = T(0), im = T(0);
        int m = 0;
        for (int j = 0; j < n; ++j) {
            re += x[j] * w[m].re;
            im += x[j] * w[m].im;
            m += k;
            if (m >= n) m -= n;
        }
        spec[(r0 + r) * nh + k] = {re, im};
    }
}

// Real inverse along x: x_j = X_0 + sum_{0<k<n/2} 2 Re(X_k e^(+2 pi i j k/n))
// (+ X_{n/2} (-1)^j for even n), the imaginary parts of X_0 and X_{n/2}
// discarded, times `scale`.
template <typename T>
__global__ __launch_bounds__(kGenThreads) void k_gen_dft_x_inv(const cplx<T> *__restrict__ spec,
                                                               int64_t rows, int n,
                                                               const cplx<T> *__restrict__ w_g,
                                                               T scale, T *__restrict__ L) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    cplx<T> *w = (cplx<T> *)lds_raw;
    const int nh = n / 2 + 1;
    cplx<T> *buf = w + n;                       // [kGenRows][nh]
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * kGenRows;
    const int nr = (int)(rows - r0 < kGenRows ? rows - r0 : kGenRows);
    for (int k = tid; k < n; k += kGenThreads) w[k] = w_g[k];
    for (int e = tid; e < nr * nh; e += kGenThreads) buf[e] = spec[r0 * nh + e];
    __syncthreads();
    const bool even = (n & 1) == 0;
    const int kmax = even ? n / 2 : nh;         // k < kmax take the factor 2
    for (int e = tid; e < nr * n; e += kGenThreads) {
        const int r = e / n, j = e - r * n;
        const cplx<T> *X = buf + r * nh;
        T acc = X[0].re;
        int m = j;                              // (j k) mod n for k = 1
        for (int k = 1; k < kmax; ++k) {
            // e^(+2 pi i m / n) = conj(w[m])
            acc += T(2) * (X[k].re * w[m].re + X[k].im * w[m].im);
            m += j;
            if (m >= n) m -= n;
        }
        if (even) acc += (j & 1) ? -X[n / 2].re : X[n / 2].re;
        L[(r0 + r) * n + j] = acc * scale;
    }
}

// q|u|^2 per z-plane of the extra moment row (component P), fixed order.
template <typename T>
__global__ __launch_bounds__(kGenThreads) void k_gen_qr2(const T *__restrict__ Mq, int n,
                                                         double *__restrict__ out) {
    __shared__ double red[kGenThreads / 64];
    const int z = blockIdx.x, tid = threadIdx.x;
    const T *pl = Mq + (int64_t)z * n * n;
    double acc = 0.0;
    for (int e = tid; e < n * n; e += kGenThreads) acc += (double)pl[e];
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < kGenThreads / 64; ++w) t += red[w];
        out[z] = t;
    }
}

// Folded transfer kernel g_j(k) (Re G~ for even orders, Im G~ for odd ones,
// on ky, kz <= n/2) at frequency (kx, ky, kz): the y reflection negates the
// components of Im S (m < 0), the z reflection multiplies component (nn, m)
// by (-1)^(nn + |m|).
template <typename T>
struct GenKernel {
    const T *g;                                 // [(ky' nh + kx) Q + j] nhp + kz'
    int64_t colbase;                            // (ky' nh + kx) Q
    int nhp, kz, fy, fz;
    __device__ __forceinline__ T at(int nn, int m) const {
        const int j = nn * (nn + 1) + m;
        T v = g[(colbase + j) * nhp + kz];
        if (fy && m < 0) v = -v;
        if (fz && ((nn + (m < 0 ? -m : m)) & 1)) v = -v;
        return v;
    }
    // spectrum of the mesh Re S_nn^m / Im S_nn^m, any -nn <= m <= nn, as the
    // real factor of i^(nn mod 2)
    __device__ __forceinline__ T re_s(int nn, int m) const {
        if (m > nn || -m > nn) return T(0);
        if (m >= 0) return at(nn, m);
        return ((-m) & 1) ? -at(nn, -m) : at(nn, -m);
    }
    __device__ __forceinline__ T im_s(int nn, int m) const {
        if (m == 0 || m > nn || -m > nn) return T(0);
        if (m > 0) return at(nn, -m);
        return ((-m) & 1) ? at(nn, m) : -at(nn, m);
    }
};

// One thread per (output row (l, m >= 0), frequency): L~ = T(G~) M~ by
// eq. realmatrix, from spec into spec2.  Thread t = ((row n + ky) nh + kx) n
// + kz: consecutive threads take consecutive kz, whose folded transfer-kernel
// values are contiguous; the spectrum index is f = (kz n + ky) nh + kx.
template <typename T>
__global__ __launch_bounds__(kGenThreads) void k_gen_m2l(const cplx<T> *__restrict__ spec,
                                                         cplx<T> *__restrict__ out,
                                                         const T *__restrict__ green, int n, int p,
                                                         const double *__restrict__ qr2_partial,
                                                         double *__restrict__ sums) {
    const int nh = n / 2 + 1, nhp = (nh + 3) & ~3, Q = (2 * p + 1) * (2 * p + 1);
    const int64_t nspec = (int64_t)n * n * nh;
    const int nrows = (p + 1) * (p + 2) / 2;
    const int64_t t = (int64_t)blockIdx.x * kGenThreads + threadIdx.x;
    if (t >= nspec * nrows) return;
    const int kz = (int)(t % n);
    const int64_t rest = t / n;
    const int kx = (int)(rest % nh), ky = (int)((rest / nh) % n);
    int row = (int)(rest / ((int64_t)nh * n));
    int l = 0;
    while (row > l) {
        row -= l + 1;
        ++l;
    }
    const int m = row;
    const int64_t f = ((int64_t)kz * n + ky) * nh + kx;
    GenKernel<T> G;
    G.g = green;
    G.nhp = nhp;
    G.fy = ky > n / 2;
    G.fz = kz > n / 2;
    G.kz = G.fz ? n - kz : kz;
    G.colbase = ((int64_t)(G.fy ? n - ky : ky) * nh + kx) * Q;
    const cplx<T> *F = spec + f;
    T are = T(0), aim = T(0), bre = T(0), bim = T(0);   // acc_re, acc_im (complex)
    for (int lam = 0; lam <= p; ++lam) {
        const int nn = l + lam;
        T xr = T(0), xi = T(0), yr = T(0), yi = T(0);    // before the i^(nn mod 2) factor
        {
            const cplx<T> M0 = F[(int64_t)(lam * (lam + 1)) * nspec];
            const T A = G.re_s(nn, -m), B = G.im_s(nn, -m);
            xr = fma(A, M0.re, xr);
            xi = fma(A, M0.im, xi);
            yr = fma(B, M0.re, yr);
            yi = fma(B, M0.im, yi);
        }
        for (int mu = 1; mu <= lam; ++mu) {
            const T sg = (mu & 1) ? T(-1) : T(1);
            const T A = G.re_s(nn, -(m + mu)), B = G.im_s(nn, -(m + mu));
            const T C = sg * G.re_s(nn, -(m - mu)), D = sg * G.im_s(nn, -(m - mu));
            const cplx<T> Mr = F[(int64_t)(lam * (lam + 1) + mu) * nspec];
            const cplx<T> Mi = F[(int64_t)(lam * (lam + 1) - mu) * nspec];
            // one FMA per multiply-add into the running sums
            const T ac = A + C, bd = B - D, bpd = B + D, amc = A - C;
            xr = fma(ac, Mr.re, xr);
            xr = fma(-bd, Mi.re, xr);
            xi = fma(ac, Mr.im, xi);
            xi = fma(-bd, Mi.im, xi);
            yr = fma(bpd, Mr.re, yr);
            yr = fma(amc, Mi.re, yr);
            yi = fma(bpd, Mr.im, yi);
            yi = fma(amc, Mi.im, yi);
        }
        if (nn & 1) {       // times i
            are -= xi;
            aim += xr;
            bre -= yi;
            bim += yr;
        } else {
            are += xr;
            aim += xi;
            bre += yr;
            bim += yi;
        }
    }
    if (f == 0) {
        // zero frequency: the uniform corrections of App. B times n^3
        // (the box volume in cell units): L_0^0 += 2 pi/(3V) sum q|u|^2,
        // L_1^0 += 4 pi/(3V) sum M_1^0, L_1^1 += 8 pi/(3V) conj(sum M_1^1)
        const double pi = 3.14159265358979323846;
        if (l == 0) {
            double qr2 = 0.0;
            for (int z = 0; z < n; ++z) qr2 += qr2_partial[z];
            are += T(2.0 * pi / 3.0 * qr2);
        } else if (l == 1 && m == 0) {
            are += T(4.0 * pi / 3.0 * (double)F[(int64_t)2 * nspec].re);
        } else if (l == 1 && m == 1) {
            are += T(8.0 * pi / 3.0 * (double)F[(int64_t)3 * nspec].re);
            bre += T(-8.0 * pi / 3.0 * (double)F[(int64_t)1 * nspec].re);
        }
    }
    out[(int64_t)(l * (l + 1) + m) * nspec + f] = {are, aim};
    if (m > 0) out[(int64_t)(l * (l + 1) - m) * nspec + f] = {bre, bim};
    if (f == 0 && l == 0) sums[0] = (double)F[0].re;      // total charge, for L2P
}

template <typename T>
size_t dft_c_lds(int n) { return sizeof(cplx<T>) * ((size_t)n + (size_t)n * kGenTile); }

template <typename T, bool INV>
hipError_t dft_c(cplx<T> *data, int n, int64_t outer, int64_t inner, int64_t so, int64_t se,
                 const cplx<T> *w, hipStream_t s) {
    const size_t lds = dft_c_lds<T>(n);
    const dim3 grid((unsigned)((inner + kGenTile - 1) / kGenTile), (unsigned)outer);
    hipLaunchKernelGGL((k_gen_dft_c<T, INV>), grid, dim3(kGenThreads), lds, s, data, n, inner, so,
                       se, w);
    return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_generic_stage(const FFTArgs &a, int stage, hipStream_t s) {
    const int n = a.n, nh = n / 2 + 1, P = nreal(a.p);
    if (n > kGenericMaxN || a.open) return hipErrorInvalidValue;
    const int64_t K = (int64_t)n * n * n, rows = (int64_t)P * n * n, plane = (int64_t)n * nh;
    const cplx<T> *w = (const cplx<T> *)a.tw;
    cplx<T> *spec = (cplx<T> *)a.spec, *spec2 = (cplx<T> *)a.spec2;
    const unsigned rblocks = (unsigned)((rows + kGenRows - 1) / kGenRows);
    hipError_t e = hipSuccess;
    if (stage == 0) {
        hipLaunchKernelGGL(k_gen_qr2<T>, dim3(n), dim3(kGenThreads), 0, s,
                           (const T *)a.M + (int64_t)P * K, n, a.qr2_partial);
        hipLaunchKernelGGL(k_gen_dft_x_fwd<T>, dim3(rblocks), dim3(kGenThreads),
                           sizeof(cplx<T>) * n + sizeof(T) * kGenRows * n, s, (const T *)a.M, rows,
                           n, w, spec);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // y: lines (c z, kx), elements at stride nh; z: lines (c, y kx), stride n nh
        if ((e = dft_c<T, false>(spec, n, (int64_t)P * n, nh, plane, nh, w, s)) != hipSuccess)
            return e;
        return dft_c<T, false>(spec, n, P, plane, (int64_t)n * plane, plane, w, s);
    }
    if (stage == 1) {
        const int64_t nthr = (int64_t)n * plane * ((a.p + 1) * (a.p + 2) / 2);
        hipLaunchKernelGGL(k_gen_m2l<T>, dim3((unsigned)((nthr + kGenThreads - 1) / kGenThreads)),
                           dim3(kGenThreads), 0, s, (const cplx<T> *)spec, spec2,
                           (const T *)a.green, n, a.p, (const double *)a.qr2_partial, a.sums);
        return hipGetLastError();
    }
    if ((e = dft_c<T, true>(spec2, n, P, plane, (int64_t)n * plane, plane, w, s)) != hipSuccess)
        return e;
    if ((e = dft_c<T, true>(spec2, n, (int64_t)P * n, nh, plane, nh, w, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_gen_dft_x_inv<T>, dim3(rblocks), dim3(kGenThreads),
                       sizeof(cplx<T>) * ((size_t)n + (size_t)kGenRows * nh), s,
                       (const cplx<T> *)spec2, rows, n, w, T(1.0 / ((double)K)), (T *)a.L);
    return hipGetLastError();
}

template hipError_t launch_generic_stage<float>(const FFTArgs &, int, hipStream_t);
template hipError_t launch_generic_stage<double>(const FFTArgs &, int, hipStream_t);

hipError_t launch_line_dft_f64(cplx<double> *data, int n, int64_t nlines, int64_t stride,
                               const cplx<double> *w, hipStream_t s) {
    // lines L = (o, i): o = L / stride, i = L % stride, start o stride n + i
    return dft_c<double, false>(data, n, nlines / stride, stride, stride * n, stride, w, s);
}

}  // namespace pmmm
