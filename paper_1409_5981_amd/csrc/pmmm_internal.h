// Internal declarations shared by the HIP translation units of the PMMM
// far-field library (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <type_traits>

#include "../../include/pmmm.h"

namespace pmmm {

// ----------------------------------------------------------------- helpers
template <typename T>
struct cplx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {  // a * conj(b)
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}

// Sorted particle record: offsets from the cell centre in cell units and the charge.
template <typename T>
struct alignas(4 * sizeof(T)) particle4 {
    T ux, uy, uz, q;
};

// Potential and gradient of one particle, in sorted order before they are
// sent back to the caller's order.
template <typename T>
struct alignas(4 * sizeof(T)) out4 {
    T phi, gx, gy, gz;
};

__host__ __device__ constexpr int nreal(int p) { return (p + 1) * (p + 1); }
__host__ __device__ constexpr int ridx(int l, int m) { return l * (l + 1) + m; }

__device__ __forceinline__ int bitrev(int v, int logn) {
    return (int)(__builtin_bitreverse32((unsigned)v) >> (32 - logn));
}

// Regular solid harmonics R_l^m(x, y, z), 0 <= l <= P_ORD, in real storage
// (index l(l+1)+m holds Re R_l^|m| for m >= 0 and Im R_l^|m| for m < 0).
// Recursion of App. A.5 rewritten for R = Q/(l+m)! directly:
//   R_m^m     = -(x + i y) / (2m) * R_{m-1}^{m-1}
//   R_{m+1}^m = z R_m^m
//   R_l^m     = ((2l-1) z R_{l-1}^m - r^2 R_{l-2}^m) / ((l-m)(l+m))
// All loops have compile-time bounds so R stays in registers.
template <int P_ORD, typename T>
__device__ __forceinline__ void regular_harmonics(T x, T y, T z, T *R) {
    const T r2 = x * x + y * y + z * z;
    T cre = T(1), cim = T(0);
#pragma unroll
    for (int m = 0; m <= P_ORD; ++m) {
        if (m > 0) {
            const T f = T(-1.0 / (2.0 * m));
            const T nre = f * (x * cre - y * cim);
            const T nim = f * (x * cim + y * cre);
            cre = nre;
            cim = nim;
        }
        R[ridx(m, m)] = cre;
        if (m > 0) R[ridx(m, -m)] = cim;
        T pre = cre, pim = cim;  // R_{l-2}^m
        T ure = T(0), uim = T(0);  // R_{l-1}^m
        if (m + 1 <= P_ORD) {
            ure = z * cre;
            uim = z * cim;
            R[ridx(m + 1, m)] = ure;
            if (m > 0) R[ridx(m + 1, -m)] = uim;
        }
#pragma unroll
        for (int l = m + 2; l <= P_ORD; ++l) {
            const T a = T((2.0 * l - 1.0) / ((double)(l - m) * (double)(l + m)));
            const T b = T(1.0 / ((double)(l - m) * (double)(l + m)));
            const T nre = a * z * ure - b * r2 * pre;
            const T nim = a * z * uim - b * r2 * pim;
            R[ridx(l, m)] = nre;
            if (m > 0) R[ridx(l, -m)] = nim;
            pre = ure;
            pim = uim;
            ure = nre;
            uim = nim;
        }
    }
}

// acc[c] += q * R_c(x, y, z) for the real-storage components c of orders
// <= P_ORD, with the same recursion as regular_harmonics; each value is
// consumed as soon as it is produced, so no R array stays live.
template <int P_ORD, typename T>
__device__ __forceinline__ void accumulate_regular(T x, T y, T z, T q, T *acc) {
    const T r2 = x * x + y * y + z * z;
    T cre = q, cim = T(0);  // q R_m^m
#pragma unroll
    for (int m = 0; m <= P_ORD; ++m) {
        if (m > 0) {
            const T f = T(-1.0 / (2.0 * m));
            const T nre = f * (x * cre - y * cim);
            const T nim = f * (x * cim + y * cre);
            cre = nre;
            cim = nim;
        }
        acc[ridx(m, m)] += cre;
        if (m > 0) acc[ridx(m, -m)] += cim;
        T pre = cre, pim = cim;
        T ure = T(0), uim = T(0);
        if (m + 1 <= P_ORD) {
            ure = z * cre;
            uim = z * cim;
            acc[ridx(m + 1, m)] += ure;
            if (m > 0) acc[ridx(m + 1, -m)] += uim;
        }
#pragma unroll
        for (int l = m + 2; l <= P_ORD; ++l) {
            const T a = T((2.0 * l - 1.0) / ((double)(l - m) * (double)(l + m)));
            const T b = T(1.0 / ((double)(l - m) * (double)(l + m)));
            const T nre = a * z * ure - b * r2 * pre;
            const T nim = a * z * uim - b * r2 * pim;
            acc[ridx(l, m)] += nre;
            if (m > 0) acc[ridx(l, -m)] += nim;
            pre = ure;
            pim = uim;
            ure = nre;
            uim = nim;
        }
    }
}

// --------------------------------------------------------- LDS radix-2 FFT
// `nlines` transforms of length N = 2^logn stored in LDS; element e of line
// t lives at buf[t * lstride + e * estride].  tw[k] = exp(-2 pi i k / N)
// (k < N/2) in LDS.  INV selects exp(+...).  Barrier after every stage.
//
// DIF: natural-order input, bit-reversed output.
template <typename T, bool INV>
__device__ void lds_fft_dif(cplx<T> *buf, int logn, int nlines, int lstride, int estride,
                            const cplx<T> *tw, int tid, int nthr) {
    const int N = 1 << logn;
    const int hN = N >> 1;
    const int total = nlines * hN;
    for (int lh = logn - 1; lh >= 0; --lh) {  // half = 2^lh
        const int half = 1 << lh;
        const int twshift = logn - 1 - lh;    // twiddle step N / (2 half)
        for (int t = tid; t < total; t += nthr) {
            const int line = t >> (logn - 1);
            const int k = t & (hN - 1);
            const int j = k & (half - 1);
            const int g = k >> lh;
            const int i0 = (g << (lh + 1)) + j;
            cplx<T> *base = buf + line * lstride;
            cplx<T> a = base[i0 * estride];
            cplx<T> b = base[(i0 + half) * estride];
            cplx<T> w = tw[j << twshift];
            if (INV) w.im = -w.im;
            cplx<T> s = {a.re + b.re, a.im + b.im};
            cplx<T> d = {a.re - b.re, a.im - b.im};
            base[i0 * estride] = s;
            base[(i0 + half) * estride] = cmul(d, w);
        }
        __syncthreads();
    }
}

// DIT: bit-reversed input, natural-order output.
template <typename T, bool INV>
__device__ void lds_fft_dit(cplx<T> *buf, int logn, int nlines, int lstride, int estride,
                            const cplx<T> *tw, int tid, int nthr) {
    const int N = 1 << logn;
    const int hN = N >> 1;
    const int total = nlines * hN;
    for (int lh = 0; lh < logn; ++lh) {
        const int half = 1 << lh;
        const int twshift = logn - 1 - lh;
        for (int t = tid; t < total; t += nthr) {
            const int line = t >> (logn - 1);
            const int k = t & (hN - 1);
            const int j = k & (half - 1);
            const int g = k >> lh;
            const int i0 = (g << (lh + 1)) + j;
            cplx<T> *base = buf + line * lstride;
            cplx<T> a = base[i0 * estride];
            cplx<T> w = tw[j << twshift];
            if (INV) w.im = -w.im;
            cplx<T> b = cmul(base[(i0 + half) * estride], w);
            base[i0 * estride] = {a.re + b.re, a.im + b.im};
            base[(i0 + half) * estride] = {a.re - b.re, a.im - b.im};
        }
        __syncthreads();
    }
}

// ------------------------------------------------- register / LDS FFTs
// Compile-time loop: f(std::integral_constant<int, i>) for i in [B, E).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

__host__ __device__ constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v >> 1); }
__host__ __device__ constexpr int brevc(int v, int bits) {
    return bits == 0 ? 0 : ((v & 1) << (bits - 1)) | brevc(v >> 1, bits - 1);
}

// exp(-+ 2 pi i k / 32) for 0 <= k < 16 (forward: minus sign).
template <typename T, bool INV, int K>
__device__ __forceinline__ cplx<T> w32() {
    constexpr double C1 = 0.98078528040323044913, S1 = 0.19509032201612826785;  // pi/16
    constexpr double C2 = 0.92387953251128674, S2 = 0.38268343236508978;          // pi/8
    constexpr double C3 = 0.83146961230254523708, S3 = 0.55557023301960222474;  // 3 pi/16
    constexpr double R2 = 0.70710678118654752;
    constexpr double c[16] = {1.0, C1, C2, C3, R2, S3, S2, S1, 0.0, -S1, -S2, -S3, -R2, -C3, -C2, -C1};
    constexpr double sn[16] = {0.0, S1, S2, S3, R2, C3, C2, C1, 1.0, C1, C2, C3, R2, S3, S2, S1};
    return {T(c[K]), INV ? T(sn[K]) : T(-sn[K])};
}

// In-register FFT of R = 1..32 points, natural order in and out (radix-2
// decimation in time on the bit-reversed copy), unnormalised.
template <int R, bool INV, typename T>
__device__ __forceinline__ void fft_reg(cplx<T> *v) {
    if constexpr (R > 1) {
        constexpr int LG = ilog2c(R);
        cplx<T> a[R];
        static_for<0, R>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            a[brevc(i, LG)] = v[i];
        });
        static_for<0, LG>([&](auto is) {
            constexpr int half = 1 << decltype(is)::value;
            constexpr int span = 2 * half;
            static_for<0, half>([&](auto ij) {
                constexpr int j = decltype(ij)::value;
                constexpr int k32 = j * (32 / span);
                static_for<0, R / span>([&](auto ig) {
                    constexpr int i0 = decltype(ig)::value * span + j, i1 = i0 + half;
                    cplx<T> b = a[i1];
                    // W = -+i is a swap and a sign: no multiplications (a
                    // product by the constant 0 does not fold in IEEE code)
                    if constexpr (k32 == 8) b = INV ? cplx<T>{-b.im, b.re} : cplx<T>{b.im, -b.re};
                    else if constexpr (k32 != 0) b = cmul(b, w32<T, INV, k32>());
                    a[i1] = {a[i0].re - b.re, a[i0].im - b.im};
                    a[i0] = {a[i0].re + b.re, a[i0].im + b.im};
                });
            });
        });
        static_for<0, R>([&](auto ii) { v[decltype(ii)::value] = a[decltype(ii)::value]; });
    }
}

// In-place FFTs of `nlines` lines of N points in LDS, natural order in and
// out; element e of line t at buf[t * lstride + e * estride].  tw[k] =
// exp(-2 pi i k / N), k < N/2, in LDS.  N <= 16: one thread per line in
// registers.  N = 16 N2 (N2 = 2, 4, 8): four-step scheme, 16-point register
// FFTs over n1 for each t2 (x[n1 N2 + t2]), twiddle W_N^(t2 k1), then N2-point
// FFTs over t2; X[k1 + 16 k2] ends at position k1 + 16 k2.  nthr must be a
// multiple of 64.  Ends with a barrier.
template <typename T, bool INV, int N>
__device__ void fft_lines_n(cplx<T> *buf, int nlines, int lstride, int estride,
                            const cplx<T> *tw, int tid, int nthr) {
    if constexpr (N <= 16) {
        for (int line = tid; line < nlines; line += nthr) {
            cplx<T> *b = buf + line * lstride;
            cplx<T> v[N];
            static_for<0, N>([&](auto ie) { v[decltype(ie)::value] = b[decltype(ie)::value * estride]; });
            fft_reg<N, INV, T>(v);
            static_for<0, N>([&](auto ie) { b[decltype(ie)::value * estride] = v[decltype(ie)::value]; });
        }
        __syncthreads();
    } else {
        constexpr int N2 = N / 16;
        const int items = nlines * N2;
        const int rounds = (items + nthr - 1) / nthr;
        for (int r = 0; r < rounds; ++r) {
            const int it = r * nthr + tid;
            const bool act = it < items;
            const int line = it / N2, t2 = it - line * N2;
            cplx<T> *b = buf + line * lstride;
            cplx<T> v[16];
            if (act) {
                static_for<0, 16>([&](auto in) {
                    constexpr int n1 = decltype(in)::value;
                    v[n1] = b[(n1 * N2 + t2) * estride];
                });
                fft_reg<16, INV, T>(v);
                static_for<1, 16>([&](auto ik) {
                    constexpr int k1 = decltype(ik)::value;
                    const int e = t2 * k1;  // < N
                    cplx<T> w = e < N / 2 ? tw[e] : tw[e - N / 2];
                    if (e >= N / 2) {
                        w.re = -w.re;
                        w.im = -w.im;
                    }
                    if (INV) w.im = -w.im;
                    v[k1] = cmul(v[k1], w);
                });
            }
            __syncthreads();  // every load of this round's lines is done
            if (act) {
                static_for<0, 16>([&](auto ik) {
                    constexpr int k1 = decltype(ik)::value;
                    b[(t2 * 16 + k1) * estride] = v[k1];
                });
            }
        }
        __syncthreads();
        for (int it = tid; it < nlines * 16; it += nthr) {
            const int line = it >> 4, k1 = it & 15;
            cplx<T> *b = buf + line * lstride;
            cplx<T> u[N2];
            static_for<0, N2>([&](auto it2) {
                constexpr int t2 = decltype(it2)::value;
                u[t2] = b[(t2 * 16 + k1) * estride];
            });
            fft_reg<N2, INV, T>(u);
            static_for<0, N2>([&](auto ik2) {
                constexpr int k2 = decltype(ik2)::value;
                b[(k2 * 16 + k1) * estride] = u[k2];
            });
        }
        __syncthreads();
    }
}

template <typename T, bool INV>
__device__ void fft_lines(cplx<T> *buf, int logn, int nlines, int lstride, int estride,
                          const cplx<T> *tw, int tid, int nthr) {
    switch (logn) {
        case 2: fft_lines_n<T, INV, 4>(buf, nlines, lstride, estride, tw, tid, nthr); break;
        case 3: fft_lines_n<T, INV, 8>(buf, nlines, lstride, estride, tw, tid, nthr); break;
        case 4: fft_lines_n<T, INV, 16>(buf, nlines, lstride, estride, tw, tid, nthr); break;
        case 5: fft_lines_n<T, INV, 32>(buf, nlines, lstride, estride, tw, tid, nthr); break;
        case 6: fft_lines_n<T, INV, 64>(buf, nlines, lstride, estride, tw, tid, nthr); break;
        default: fft_lines_n<T, INV, 128>(buf, nlines, lstride, estride, tw, tid, nthr); break;
    }
}

// Swizzled LDS rows of N complex values (no padding): element e of row b at
// b * N + cpos(b, e), the low three bits of e flipped by bits 4..6 of e and
// bit 3 by the row's parity.  For 128-point rows every access of fft_col --
// and any 16 consecutive elements of a row -- then falls on 16 distinct
// 8-byte bank pairs (64- and 32-point rows keep some two- and four-way
// conflicts in the first FFT pass).
__device__ __forceinline__ constexpr int cpos(int row, int e) {
    return e ^ (((e >> 4) & 7) | ((row & 1) << 3));
}

// In-place FFTs of nlines rows of N = 16 N2 points (N = 32, 64, 128) in the
// layout above: 16-point register FFTs over n1 of x[n1 N2 + t2], twiddles
// W_N^(t2 k1) from a full-circle table tw[e] = exp(-2 pi i e / N), e < N
// (see fill_twiddles), then N2-point FFTs over t2.  The lanes of one row's items sit
// in one wave, so each in-place pass needs no barrier between its reads and
// writes (a wave's LDS operations complete in order; the asm statement keeps
// the compiler from moving the writes up).  HALF: only the first N/2 inputs
// are non-zero (forward) or only the first N/2 outputs are kept (inverse).
// Full-circle twiddle table tw[e] = exp(-2 pi i e / N), e < N, in LDS from
// the half table tw_g[e], e < N/2 (tw[e + N/2] = -tw[e]); call with at least
// N/2 threads, before the barrier that precedes the first use.
template <typename T>
__device__ __forceinline__ void fill_twiddles(cplx<T> *tw, const cplx<T> *__restrict__ tw_g,
                                              int N, int tid, int nthr) {
    for (int e = tid; e < N / 2; e += nthr) {
        const cplx<T> w = tw_g[e];
        tw[e] = w;
        tw[e + N / 2] = {-w.re, -w.im};
    }
}

template <typename T, bool INV, int N, bool HALF>
__device__ __forceinline__ void fft_col(cplx<T> *buf, int nlines, const cplx<T> *tw, int tid,
                                        int nthr) {
    constexpr int N2 = N / 16, L2 = ilog2c(N2);
    const int items = nlines * N2;
    for (int it = tid; it < items; it += nthr) {
        const int line = it >> L2, t2 = it & (N2 - 1);
        cplx<T> *b = buf + line * N;
        cplx<T> v[16];
        static_for<0, 16>([&](auto in) {
            constexpr int n1 = decltype(in)::value;
            if constexpr (!INV && HALF && n1 >= 8) v[n1] = {T(0), T(0)};
            else v[n1] = b[cpos(line, n1 * N2 + t2)];
        });
        fft_reg<16, INV, T>(v);
        static_for<1, 16>([&](auto ik) {
            constexpr int k1 = decltype(ik)::value;
            cplx<T> w = tw[t2 * k1];  // full-circle table: t2 k1 < N
            if (INV) w.im = -w.im;
            v[k1] = cmul(v[k1], w);
        });
        asm volatile("" ::: "memory");
        static_for<0, 16>([&](auto ik) {
            constexpr int k1 = decltype(ik)::value;
            b[cpos(line, t2 * 16 + k1)] = v[k1];
        });
    }
    __syncthreads();
    for (int it = tid; it < nlines * 16; it += nthr) {
        const int line = it >> 4, k1 = it & 15;
        cplx<T> *b = buf + line * N;
        cplx<T> u[N2];
        static_for<0, N2>([&](auto it2) {
            constexpr int t2 = decltype(it2)::value;
            u[t2] = b[cpos(line, t2 * 16 + k1)];
        });
        fft_reg<N2, INV, T>(u);
        asm volatile("" ::: "memory");
        static_for<0, N2>([&](auto ik2) {
            constexpr int k2 = decltype(ik2)::value;
            if constexpr (!(INV && HALF && k2 >= N2 / 2)) b[cpos(line, k2 * 16 + k1)] = u[k2];
        });
    }
    __syncthreads();
}

template <typename T, bool INV, int N>
__device__ __forceinline__ void fft_col_rt(cplx<T> *buf, bool half, int nlines,
                                           const cplx<T> *tw, int tid, int nthr) {
    if (half) fft_col<T, INV, N, true>(buf, nlines, tw, tid, nthr);
    else fft_col<T, INV, N, false>(buf, nlines, tw, tid, nthr);
}

// Line stride in LDS for lines of n complex values, padded by one element:
// the lanes of a wave work on different lines at the same offsets (one line
// per lane for n <= 16, n / 16 lanes per line above), and an odd stride puts
// those lines in different LDS banks.
__host__ __device__ constexpr int lds_line(int n) { return n + 1; }

// ------------------------------------------------- transfer-kernel terms
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

// Particle range of a block's system in a batch (blockIdx.y selects the
// system; prange[2s], prange[2s+1] bound its particles in the caller's
// arrays).  Without a batch (prange null) the one system holds [0, n).
__device__ __forceinline__ void sys_range(const int64_t *prange, int64_t n, int64_t &p0,
                                          int64_t &np) {
    if (prange == nullptr) {
        p0 = 0;
        np = n;
    } else {
        p0 = prange[2 * blockIdx.y];
        np = prange[2 * blockIdx.y + 1] - p0;
    }
}

// ------------------------------------------------------------ host side
struct Plan;  // defined in pmmm_api.hip

// Row subsets of the column kernel's M2L (threads per frequency at most).
constexpr int kColumnRowSplit = 4;

// Threads per block of the column kernel: 512 up to order 6 (the 128-point
// columns then still run one row subset per thread), else 256.
inline int column_max_threads(int p) { return p <= 6 ? 512 : 256; }

// LDS bytes of the column kernel for w columns of nf frequencies per block
// (0 if over 160 KB), and its row subsets rs (rs * w * nf threads).
// LDS holds the moment spectra [P][w][nf] (the local spectra overwrite them
// when every thread runs one row subset, else they get a buffer of their
// own), the kernel tile [w][Q][nhp] and the twiddles.
inline size_t column_lds_w(int p, int nf, size_t tsize, int w, int *rs_out) {
    if (w < 1 || (size_t)w * nf > 256) return 0;
    const size_t P = (size_t)(p + 1) * (p + 1), Q = (size_t)(2 * p + 1) * (2 * p + 1);
    const size_t nhp = ((size_t)nf / 2 + 1 + 3) & ~(size_t)3;
    const int fit = column_max_threads(p) / (w * nf);
    const int rs = fit < kColumnRowSplit ? fit : kColumnRowSplit;
    const size_t nbuf = rs == kColumnRowSplit ? 1 : 2;
    const size_t lds = nbuf * P * w * (size_t)lds_line(nf) * 2 * tsize + Q * w * nhp * tsize +
                       (size_t)nf / 2 * 2 * tsize;
    if (lds > 160 * 1024) return 0;
    if (rs_out) *rs_out = rs;
    return lds;
}

// LDS bytes of the streamed-kernel column variant (the full-circle twiddle
// table and one column's spectra, rows of nf without padding; 0 if over
// 160 KB).
inline size_t column_g_lds(int p, int nf, size_t tsize) {
    const size_t P = (size_t)(p + 1) * (p + 1);
    const size_t lds = P * (size_t)nf * 2 * tsize + (size_t)nf * 2 * tsize;
    return lds > 160 * 1024 ? 0 : lds;
}

// Column kernel forms (PMMM_COLUMN_* in pmmm.h): the kernel tile staged in
// LDS for w columns per block, or streamed from memory with each thread
// running 1, 2 or 4 row subsets (FFT meshes of 64 and 128 points).
inline bool column_kernel_fits(int kind, int p, int nf, size_t tsize);
// Default form: the streamed kernel with two subsets per thread (one from
// order 9 on) for FFT meshes of 64 points and more, else the staged tile.
inline int column_default_kernel(int p, int nf, size_t tsize);

// Widest shape that fits (w from 64 / nf down to 1).
inline size_t column_shape(int p, int nf, size_t tsize, int *w_out, int *rs_out) {
    for (int w = nf >= 64 ? 1 : 64 / nf; w >= 1; w >>= 1) {
        int rs = 1;
        const size_t lds = column_lds_w(p, nf, tsize, w, &rs);
        if (lds > 0) {
            if (w_out) *w_out = w;
            if (rs_out) *rs_out = rs;
            return lds;
        }
    }
    return 0;
}

inline bool column_kernel_fits(int kind, int p, int nf, size_t tsize) {
    switch (kind) {
        case PMMM_COLUMN_TILE: return column_shape(p, nf, tsize, nullptr, nullptr) > 0;
        case PMMM_COLUMN_STREAM_1:
        case PMMM_COLUMN_STREAM_2:
        case PMMM_COLUMN_STREAM_4:
            // more row subsets per thread hold more results in registers:
            // four from order 7 and two from order 9 on would spill
            if ((kind == PMMM_COLUMN_STREAM_4 && p >= 7) || (kind == PMMM_COLUMN_STREAM_2 && p >= 9))
                return false;
            return (nf == 64 || nf == 128) && column_g_lds(p, nf, tsize) > 0;
        default: return false;
    }
}

inline int column_default_kernel(int p, int nf, size_t tsize) {
    if (nf >= 64 && column_kernel_fits(PMMM_COLUMN_STREAM_2, p, nf, tsize))
        return PMMM_COLUMN_STREAM_2;
    if (nf >= 64 && column_kernel_fits(PMMM_COLUMN_STREAM_1, p, nf, tsize))
        return PMMM_COLUMN_STREAM_1;
    if (column_kernel_fits(PMMM_COLUMN_TILE, p, nf, tsize)) return PMMM_COLUMN_TILE;
    if (column_kernel_fits(PMMM_COLUMN_STREAM_2, p, nf, tsize)) return PMMM_COLUMN_STREAM_2;
    return 0;
}

// Raise a kernel's dynamic-LDS limit once (later calls with no larger size
// make no runtime call, so they are safe while a stream is being captured).
hipError_t set_max_lds(const void *kernel, size_t bytes);

// Error bookkeeping (thread-local message).
void set_error(const std::string &msg);
int hip_fail(hipError_t e, const char *what);

#define PMMM_HIP(call)                                      \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return ::pmmm::hip_fail(e_, #call); \
    } while (0)

// Launchers (each returns a HIP error code; they only enqueue).
struct BinArgs {
    int64_t n;
    const void *x, *y, *z, *q;
    int ncell;         // cells per axis
    double inv_h;      // n / b
    int periodic;
    // open boundary: cells per axis (x, y, z) of the caller's box, which may
    // be a corner of the ncell^3 mesh; a particle beyond it sets flag
    // (0: ncell)
    int lim[3] = {0, 0, 0};
    // [n] key/value/record ping-pong arrays of the radix sort; the sorted
    // cell, the permutation (caller index of every sorted slot) and the
    // sorted records end in scell, perm, sorted
    int *cell_of, *slot, *scell, *perm;
    void *recs;        // particle4<T>[n] records between passes
    int *start;        // [nsys][K + 1] first sorted slot of every cell (system-relative)
    int *flag;         // set when an open-boundary particle lies outside the box
    // [nsys][items_cap] dense-cell items {cell, chunk, chunks, first partial
    // slot or -1} followed by the split cells (or null: none built);
    // small[8 s + 0] counts the items, small[8 s + 3] the partial slots and
    // small[8 s + 4] the split cells of system s
    int4 *items;
    int64_t items_cap, slots_cap;
    int *small;
    int *count;        // [nsys][bin_hist_ints(max_np)] radix histograms / offsets
    int *tile_sums;    // [nsys][bin_scan_tiles(max_np)] scan scratch
    int *pos;          // [n] sorted slot of each particle in the caller's order (or null)
    int dense_threshold;
    void *sorted;      // particle4<T>[n]
    // batch of nsys systems on this mesh (prange null: one system of n)
    const int64_t *prange;
    int nsys;
    int64_t max_np;
};
template <typename T>
hipError_t launch_bin(const BinArgs &a, hipStream_t s);
// Radix-sort tiles: 1024 R elements, R = 1, 2 or 4 growing with the
// particle count, and at most 2^9 buckets per digit.
constexpr int kRadixMaxBits = 9;
constexpr int bin_tile_items(int64_t max_np) {
    return max_np >= (int64_t(1) << 21) ? 4 : (max_np >= (int64_t(1) << 20) ? 2 : 1);
}
constexpr int64_t bin_tiles(int64_t max_np) {
    return max_np > 0 ? (max_np + 1024 * bin_tile_items(max_np) - 1) /
                            (1024 * bin_tile_items(max_np))
                      : 1;
}
constexpr int64_t bin_max64(int64_t a, int64_t b) { return a > b ? a : b; }
constexpr int64_t bin_min64(int64_t a, int64_t b) { return a < b ? a : b; }
// Histogram ints per system for every particle count up to max_np (the tile
// count is not monotonic where R steps up, hence the maximum).
constexpr int64_t bin_hist_ints(int64_t max_np) {
    return (int64_t(1) << kRadixMaxBits) *
           bin_max64(bin_tiles(max_np),
                     bin_max64(bin_tiles(bin_min64(max_np, (int64_t(1) << 21) - 1)),
                               bin_tiles(bin_min64(max_np, (int64_t(1) << 20) - 1))));
}
constexpr int64_t bin_scan_tiles(int64_t max_np) { return (bin_hist_ints(max_np) + 4095) / 4096; }

// Dense cells (above the P2M threshold, never below kDenseMinThreshold) are
// cut into items of kDenseItem sorted particles, one wave each; a cell of J
// items (J > 1) leaves J partial sums that a second pass adds in item order.
constexpr int kDenseItem = 512;
constexpr int kDenseMinThreshold = 64;
// Partial slots: a split cell has count > kDenseItem and J < 2 count / kDenseItem.
constexpr int64_t dense_slots_cap(int64_t max_np) { return 2 * max_np / kDenseItem + 1; }
// Split cells (two items or more): at most half the partial slots.
constexpr int64_t dense_splits_cap(int64_t max_np) { return dense_slots_cap(max_np) / 2 + 1; }
// The same from a partial-slot capacity (slots_cap = dense_slots_cap(n)).
constexpr int64_t dense_splits_cap_of(int64_t slots_cap) { return slots_cap / 2 + 1; }
// Table of a system of up to max_np particles on K cells: the items (each
// dense cell gives at most count / kDenseItem + 1, and there are at most
// max_np / (threshold + 1) dense cells), then the list of split cells
// {cell, J, first partial slot} at offset items_cap - dense_splits_cap.
constexpr int64_t dense_items_cap(int64_t max_np, int64_t K) {
    return max_np / kDenseItem + bin_min64(K, max_np / (kDenseMinThreshold + 1)) + 1 +
           dense_splits_cap(max_np);
}

struct P2MArgs {
    int p, ncell, group;            // lanes per cell in the light path
    const int *start;
    int dense_threshold;            // cells above it are reduced as dense items
    const int4 *items;              // dense items of the binning (see BinArgs)
    int64_t items_cap;
    const int *small;
    float *partial;                 // [nsys][slots_cap][P + 1] sums of the items of split cells
    int64_t slots_cap;
    const void *sorted;
    void *M;                        // [P + 1][K]: moments, then sum q |u|^2
    const int64_t *prange;          // batch (see BinArgs)
    int nsys;
};
template <typename T>
hipError_t launch_p2m(const P2MArgs &a, hipStream_t s);

struct FFTArgs {
    int p, n, nf, open;
    double *qr2_partial;            // [n] per-plane sums of q|u|^2 (periodic)
    double *sums;                   // [0] = total charge (periodic, for L2P)
    const void *M;                  // [P(+1)][n^3] real mesh
    void *spec;                     // [P][n][nf][nf/2+1] complex
    const void *green;              // [nf*(nf/2+1)][Q][nf]
    const void *tw;                 // cplx<T>[nf/2]
    void *L;                        // [P][n^3]
    int nsys;                       // batch of systems at fixed strides (1: one)
    int col_w;                      // columns per column-kernel block (0: largest that fits)
    int col_kernel;                 // PMMM_COLUMN_* form (0: column_default_kernel)
    // periodic n not a power of two: direct DFTs, tw = cplx<T>[n] roots of
    // unity e^(-2 pi i m / n), and the M2L output in spec2 (same size as spec)
    int generic;
    void *spec2;
};
// stage 0: forward plane FFTs, 1: column FFT + M2L + inverse, 2: inverse planes
template <typename T>
hipError_t launch_conv_stage(const FFTArgs &a, int stage, hipStream_t s);
// The same three stages for a generic periodic mesh (n <= kGenericMaxN).
constexpr int kGenericMaxN = 64;
template <typename T>
hipError_t launch_generic_stage(const FFTArgs &a, int stage, hipStream_t s);
// In-place forward FP64 DFT of nlines lines of n points; line L starts at
// (L / stride) * stride * n + (L % stride) and steps by stride (any n).
hipError_t launch_line_dft_f64(cplx<double> *data, int n, int64_t nlines, int64_t stride,
                               const cplx<double> *w, hipStream_t s);

struct L2PArgs {
    int64_t n;
    int p, ncell, periodic;
    const void *sorted;
    const int *scell, *perm;
    const void *L;                  // [P][K]
    const double *sums;             // [0] = total charge
    double alpha_cell;              // alpha h
    double inv_h;                   // 1 / h in the caller's length unit
    void *phi, *gx, *gy, *gz;
    void *staged;                   // out4<T>[n] results, or null: scatter directly
    const int *pos;                 // with staged: [n] sorted slot per caller index, and the
                                    // records in sorted order; null: records at caller indices
    const int64_t *prange;          // batch (see BinArgs)
    int nsys;
    int64_t max_np;
};
template <typename T>
hipError_t launch_l2p(const L2PArgs &a, hipStream_t s);

// Staged results into the caller's outputs (out[i] = or += staged[pos[i]],
// or staged[i] when pos is null).
template <typename T>
hipError_t launch_unpermute(int64_t n, const int *pos, const void *staged, void *phi, void *gx,
                            void *gy, void *gz, int accumulate, hipStream_t s);

struct NearArgs {
    int64_t n;
    int ncell, cutoff, periodic;
    int accumulate;                 // add into staged (a far field already there) or store
    const int *start, *scell;
    const void *sorted;
    double inv_h;
    int *tile_first, *tile_row, *ntiles;  // [ncell^2], [near_tile_capacity], [1] scratch
    void *staged;                   // out4<T>[n] sorted-order results
};
template <typename T>
hipError_t launch_near(const NearArgs &a, hipStream_t s);
// Upper bound of the near-field tiles of n particles on ncell^3 cells.
int64_t near_tile_capacity(int64_t n, int ncell);
// p[0 .. count) = 0 with a fill kernel.
hipError_t launch_zero_ints(int *p, int64_t count, hipStream_t s);

// Plan-time transfer kernel (FP64 on the GPU), stored in precision T.
struct GreenArgs {
    int p, n, nf, open, cutoff, images;
    double alpha_cell;              // alpha h
    void *green_out;                // [nf*(nf/2+1)][Q][nf] in T
};
template <typename T>
hipError_t build_green(const GreenArgs &a, hipStream_t s);

// Multi-charge periodic pipeline (FP32 storage; M2L on the BF16 matrix
// cores).  Meshes are point-major with the set index fastest: component b of
// set s at point x lives at [x][b S + s], so the particle kernels (one lane
// per set) and the FFT kernels (tiles of consecutive components) both make
// contiguous accesses.
constexpr int kMultiMaxSets = 64;
constexpr int kMultiPMax = 8;         // highest order of the multi-charge kernels
constexpr int kMultiSetTile = 8;       // sets per column-GEMM block
constexpr int kMultiCompTile = 16;     // components per plane-FFT block

// t-matrix map of one (P x P) real M2L matrix in MFMA A-fragment order:
// [RT][KS][64 lanes][8] codes, RT = ceil(P/16), KS = ceil(P/32).  Code bits
// 0-8: index of the first kernel value, 9-10: its sign (0 none, 1 +, 2 -),
// 11-19 and 20-21: the second.
size_t multi_map_entries(int p);
void build_multi_map(int p, unsigned *out);

struct MultiArgs {
    int p, n, nsets;                // n = nf (periodic)
    int split;                      // bf16 terms per operand: 2 or 3
    int64_t np;                     // particles
    int64_t ld;                     // row stride of q and the outputs (sets)
    const int *start, *perm;
    int *zero_count;                // counts to reset for the next binning (or null)
    const void *sorted;             // particle4<float>[np]
    const float *q;                 // [np][ld], this chunk's first set at column 0
    float *M;                       // [K][P+1][S] moments and q|u|^2; then L [K][P][S]
    void *Y;                        // cplx<float>[nf][nf][nf/2+1][P S (+1: even)] spectra
    const float *green;             // [nh][nh][Q][nhp]
    const void *tw;                 // cplx<float>[nf/2]
    const unsigned *tmap;           // build_multi_map(p)
    double *qr2_partial;            // [nf][S] per-plane sums of q|u|^2
    double *qtot;                   // [S]
    double alpha_cell, inv_h;
    float *phi, *gx, *gy, *gz;      // [np][ld]
};
// stage 0: P2M, 1: forward x-y FFTs, 2: column (z FFT, M2L GEMM, inverse z
// FFT), 3: inverse y-x FFTs, 4: L2P
hipError_t launch_multi_stage(const MultiArgs &a, int stage, hipStream_t s);
// Orders and meshes the multi-charge kernels are built for.
bool multi_supported(int p, int nf);

}  // namespace pmmm
