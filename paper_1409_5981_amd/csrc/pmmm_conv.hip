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
//                inverse FFT along z (pmmm_column.h).
//   k_plane_inv  inverse of k_plane_fwd restricted to the y < n, x < n
//                block, scaled by 1/nf^3.
// The 3-D spectrum therefore never reaches HBM in full: the buffer between
// the kernels holds [P][n][nf][nf/2+1] complex values.
#include <type_traits>

#include "pmmm_internal.h"

namespace pmmm {

// Global loads each thread keeps in flight before writing them to LDS.
constexpr int kLoadBatch = 8;

// ------------------------------------------------------------------ planes
// Row y, column k of the x spectra from the packed FFT of the row pair
// (y & ~1, y | 1) held as one complex row (zero rows y >= nin).
template <typename T>
__device__ __forceinline__ cplx<T> unpack_row_pair(const cplx<T> *buf1, int ls, int nf, int nin,
                                                   int y, int k) {
    cplx<T> v = {T(0), T(0)};
    if (y < nin) {
        const cplx<T> *row = buf1 + (y >> 1) * ls;
        const cplx<T> zk = row[k & (nf - 1)];
        const cplx<T> zm = row[(nf - k) & (nf - 1)];
        if ((y & 1) == 0) {
            v.re = T(0.5) * (zk.re + zm.re);
            v.im = T(0.5) * (zk.im - zm.im);
        } else {
            v.re = T(0.5) * (zk.im + zm.im);
            v.im = T(-0.5) * (zk.re - zm.re);
        }
    }
    return v;
}

template <typename T>
__global__ void __launch_bounds__(512) k_plane_fwd(int nin, int logn,
                                                   const T *__restrict__ M,
                                                   cplx<T> *__restrict__ spec,
                                                   const cplx<T> *__restrict__ tw_g,
                                                   int P, double *__restrict__ qr2_partial,
                                                   int cw, int cws, int cpb) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int nf = 1 << logn, nh = nf / 2 + 1, npair = nin / 2, ls = lds_line(nf);
    const int z = blockIdx.x;
    const int btid = threadIdx.x, bnthr = blockDim.x;
    {
        // system blockIdx.z of a batch: meshes at fixed strides
        const int64_t sy = blockIdx.z, K = (int64_t)nin * nin * nin;
        M += sy * (P + 1) * K;
        spec += sy * P * nin * nf * nh;
        if (qr2_partial != nullptr) qr2_partial += sy * nin;
    }
    if ((int)blockIdx.y == (P + cpb - 1) / cpb) {
        // blocks of the extra row: sum over plane z of the per-cell q|u|^2
        // (component P of M), fixed-order reduction
        __shared__ double red[8];
        const T *pl = M + ((int64_t)P * nin + z) * nin * nin;
        double acc = 0.0;
        for (int idx = btid; idx < nin * nin; idx += bnthr) acc += (double)pl[idx];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if ((btid & 63) == 0) red[btid >> 6] = acc;
        __syncthreads();
        if (btid == 0) {
            double t = 0.0;
            for (int w = 0; w < (bnthr >> 6); ++w) t += red[w];
            qr2_partial[z] = t;
        }
        return;
    }
    // cpb components per block, one group of blockDim.x / cpb threads each
    // with its own LDS lines (a group past the last component repeats it and
    // stores nothing); tid, nthr below are the group's
    const int nthr = bnthr / cpb, grp = btid / nthr, tid = btid - grp * nthr;
    const bool live = (int)blockIdx.y * cpb + grp < P;
    const int c = live ? (int)blockIdx.y * cpb + grp : P - 1;
    cplx<T> *tw = (cplx<T> *)lds_raw;      // shared by the groups (each writes all of it)
    cplx<T> *buf1 = tw + nf / 2 + grp * (npair * ls + nf * cws);   // [npair][ls] row pairs
    cplx<T> *buf2 = buf1 + npair * ls;     // [nf][cws]: kx columns k0 .. k0 + cw - 1
    // twiddle load in flight together with the plane's loads (nf/2 <= blockDim.x)
    const cplx<T> twv = tw_g[tid < nf / 2 ? tid : 0];
    const T *plane = M + ((int64_t)c * nin + z) * nin * nin;
    // rows are paired (2j, 2j+1) into one complex row; loads are issued in
    // batches of kLoadBatch before their LDS stores
    for (int base = tid; base < npair * nf; base += nthr * kLoadBatch) {
        cplx<T> v[kLoadBatch];
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int idx = base + u * nthr;
            const int j = idx >> logn, x = idx & (nf - 1);
            v[u] = {T(0), T(0)};
            if (idx < npair * nf && x < nin) {
                v[u].re = plane[(2 * j) * nin + x];
                v[u].im = plane[(2 * j + 1) * nin + x];
            }
        }
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int idx = base + u * nthr;
            if (idx < npair * nf) buf1[(idx >> logn) * ls + (idx & (nf - 1))] = v[u];
        }
    }
    asm volatile("" ::"v"(twv.re), "v"(twv.im));   // keeps the load above this point
    if (tid < nf / 2) tw[tid] = twv;
    __syncthreads();
    fft_lines<T, false>(buf1, logn, npair, ls, 1, tw, tid, nthr);
    cplx<T> *out = spec + ((int64_t)c * nin + z) * nf * nh;
    // y FFTs: all nh kx columns at once, or in chunks of cw when LDS is short
    if (cw >= nh) {
        for (int idx = tid; idx < nf * nh; idx += nthr) {
            const int y = idx / nh, k = idx - y * nh;
            buf2[idx] = unpack_row_pair(buf1, ls, nf, nin, y, k);
        }
        __syncthreads();
        fft_lines<T, false>(buf2, logn, nh, 1, nh, tw, tid, nthr);
        if (live)
            for (int idx = tid; idx < nf * nh; idx += nthr) out[idx] = buf2[idx];
        return;
    }
    for (int k0 = 0; k0 < nh; k0 += cw) {
        const int cn = nh - k0 < cw ? nh - k0 : cw;
        for (int idx = tid; idx < nf * cn; idx += nthr) {
            const int y = idx / cn, kk = idx - y * cn;
            buf2[y * cws + kk] = unpack_row_pair(buf1, ls, nf, nin, y, k0 + kk);
        }
        __syncthreads();
        fft_lines<T, false>(buf2, logn, cn, 1, cws, tw, tid, nthr);
        for (int idx = tid; live && idx < nf * cn; idx += nthr) {
            const int y = idx / cn, kk = idx - y * cn;
            out[y * nh + k0 + kk] = buf2[y * cws + kk];
        }
        __syncthreads();   // buf2 is refilled by the next chunk
    }
}

template <typename T>
__global__ void __launch_bounds__(512) k_plane_inv(int nout, int logn,
                                                   const cplx<T> *__restrict__ spec,
                                                   T *__restrict__ L,
                                                   const cplx<T> *__restrict__ tw_g, T scale,
                                                   int P, int cw, int cws, int cpb) {
    {
        // system blockIdx.z of a batch: meshes at fixed strides
        const int64_t sy = blockIdx.z;
        const int nf_ = 1 << logn;
        spec += sy * P * nout * nf_ * (nf_ / 2 + 1);
        L += sy * P * nout * nout * nout;
    }
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int nf = 1 << logn, nh = nf / 2 + 1, npair = nout / 2, ls = lds_line(nf);
    const int z = blockIdx.x;
    // cpb components per block as in k_plane_fwd; tid, nthr are the group's
    const int nthr = blockDim.x / cpb, grp = threadIdx.x / nthr, tid = threadIdx.x - grp * nthr;
    const bool live = (int)blockIdx.y * cpb + grp < P;
    const int c = live ? (int)blockIdx.y * cpb + grp : P - 1;
    cplx<T> *tw = (cplx<T> *)lds_raw;      // shared by the groups (each writes all of it)
    cplx<T> *buf2 = tw + nf / 2 + grp * (nf * cws + npair * ls);   // [nf][cws]: kx columns k0 .. k0 + cw - 1
    cplx<T> *buf1 = buf2 + nf * cws;       // [npair][ls]
    // twiddle load in flight together with the spectrum's (nf/2 <= blockDim.x)
    const cplx<T> twv = tw_g[tid < nf / 2 ? tid : 0];
    const cplx<T> *in = spec + ((int64_t)c * nout + z) * nf * nh;
    // y inverse FFTs: all nh kx columns at once, or in chunks of cw when LDS
    // is short; the results are packed into the C2R rows of buf1 (columns kx
    // and nf - kx of a row pair come from column kx)
    const int nchunk = cw >= nh ? 1 : (nh + cw - 1) / cw;
    const int cwl = cw >= nh ? nh : cw;
    for (int ch = 0; ch < nchunk; ++ch) {
        const int k0 = ch * cwl;
        const int cn = nh - k0 < cwl ? nh - k0 : cwl;
        const int ld = nchunk == 1 ? nh : cws;       // row stride of buf2
        for (int base = tid; base < nf * cn; base += nthr * kLoadBatch) {
            cplx<T> v[kLoadBatch];
#pragma unroll
            for (int u = 0; u < kLoadBatch; ++u) {
                // clamped, unconditional loads: the whole batch is issued at once
                const int idx = base + u * nthr < nf * cn ? base + u * nthr : nf * cn - 1;
                v[u] = in[nchunk == 1 ? idx : (idx / cn) * nh + k0 + idx % cn];
            }
#pragma unroll
            for (int u = 0; u < kLoadBatch; ++u) asm volatile("" ::"v"(v[u].re), "v"(v[u].im));
#pragma unroll
            for (int u = 0; u < kLoadBatch; ++u) {
                const int idx = base + u * nthr;
                if (idx < nf * cn) buf2[nchunk == 1 ? idx : (idx / cn) * ld + idx % cn] = v[u];
            }
        }
        if (ch == 0) {
            asm volatile("" ::"v"(twv.re), "v"(twv.im));
            if (tid < nf / 2) tw[tid] = twv;
        }
        __syncthreads();
        fft_lines<T, true>(buf2, logn, cn, 1, ld, tw, tid, nthr);
        if (nchunk == 1) {
            for (int idx = tid; idx < npair * nf; idx += nthr) {
                const int j = idx >> logn, k = idx & (nf - 1);
                const int kk = k <= nf / 2 ? k : nf - k;
                cplx<T> A = buf2[(2 * j) * nh + kk];
                cplx<T> B = buf2[(2 * j + 1) * nh + kk];
                if (k > nf / 2) {
                    A.im = -A.im;
                    B.im = -B.im;
                }
                buf1[j * ls + k] = {A.re - B.im, A.im + B.re};
            }
        } else {
            for (int idx = tid; idx < npair * cn; idx += nthr) {
                const int j = idx / cn, kk = idx - j * cn, k = k0 + kk;
                const cplx<T> A = buf2[(2 * j) * ld + kk];
                const cplx<T> B = buf2[(2 * j + 1) * ld + kk];
                buf1[j * ls + k] = {A.re - B.im, A.im + B.re};
                if (k >= 1 && k < nf / 2) buf1[j * ls + nf - k] = {A.re + B.im, B.re - A.im};
            }
        }
        __syncthreads();   // buf1 complete / buf2 refilled by the next chunk
    }
    fft_lines<T, true>(buf1, logn, npair, ls, 1, tw, tid, nthr);
    T *plane = L + ((int64_t)c * nout + z) * nout * nout;
    for (int idx = tid; live && idx < nout * nout; idx += nthr) {
        const int y = idx / nout, x = idx - y * nout;
        const cplx<T> v = buf1[(y >> 1) * ls + x];
        plane[idx] = ((y & 1) ? v.im : v.re) * scale;
    }
}

// ------------------------------------------------- planes of 64 and 128
// Same transforms for FFT sizes N = 64 and 128, one (plane z, component c)
// per block of 256 threads, with register FFTs in four steps (fft_col) and
// the open boundary's zero half pruned.  The row pairs live in swizzled LDS
// rows xb[npair][N]; the y pass runs over chunks of up to 17 kx columns
// through yb[N][CWS] (y-major, kx fastest, so the lanes of a wave take
// consecutive kx: conflict-free in LDS and coalesced in memory): its first
// step reads the row pairs straight from xb (unpacking the R2C of two real
// rows), its second writes the spectrum to memory (forward) or into the
// C2R row pairs (inverse).  Open: nin = N / 2 rows and columns in, and the
// y and x transforms skip the zero half; periodic: nin = N.
// Chunks of 17 columns keep a 128-point block at 51 KB of LDS, three blocks
// per CU (33 columns: 68 KB, two blocks, and the inverse planes 28% slower;
// 5 columns: 39 KB, four blocks, but 13 chunks' barriers make both passes
// about 60% slower).
constexpr int kPlaneThreads = 256;
constexpr int kPlaneChunk = 17;

// W_N^e (conjugate for the inverse) from the full-circle table.
template <typename T>
__device__ __forceinline__ cplx<T> tw_n(const cplx<T> *tw, int e, bool inv) {
    cplx<T> w = tw[e];
    if (inv) w.im = -w.im;
    return w;
}

template <typename T, int N, bool HALF>
__global__ void __launch_bounds__(kPlaneThreads) k_plane_fwd_n(const T *__restrict__ M,
                                                               cplx<T> *__restrict__ spec,
                                                               const cplx<T> *__restrict__ tw_g,
                                                               int P,
                                                               double *__restrict__ qr2_partial) {
    constexpr int nin = HALF ? N / 2 : N, npair = nin / 2, nh = N / 2 + 1, N2 = N / 16;
    constexpr int CWS = kPlaneChunk;  // odd row stride of yb
    extern __shared__ __align__(16) unsigned char lds_raw[];
    cplx<T> *tw = (cplx<T> *)lds_raw;
    cplx<T> *xb = tw + N;
    cplx<T> *yb = xb + npair * N;
    const int z = blockIdx.x, tid = threadIdx.x;
    {
        const int64_t sy = blockIdx.z, K = (int64_t)nin * nin * nin;
        M += sy * (P + 1) * K;
        spec += sy * P * nin * N * nh;
        if (qr2_partial != nullptr) qr2_partial += sy * nin;
    }
    if ((int)blockIdx.y == P) {
        // blocks of the extra row: sum over plane z of the per-cell q|u|^2
        // (component P of M), fixed-order reduction
        __shared__ double red[kPlaneThreads / 64];
        const T *pl = M + ((int64_t)P * nin + z) * nin * nin;
        double acc = 0.0;
        for (int idx = tid; idx < nin * nin; idx += kPlaneThreads) acc += (double)pl[idx];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if ((tid & 63) == 0) red[tid >> 6] = acc;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int w = 0; w < kPlaneThreads / 64; ++w) t += red[w];
            qr2_partial[z] = t;
        }
        return;
    }
    const int c = blockIdx.y;
    const T *plane = M + ((int64_t)c * nin + z) * nin * nin;
    // rows (2j, 2j+1) as one complex row; the loads of a batch are issued
    // before their LDS stores
    constexpr int NL = npair * nin;
    constexpr int LB = (NL + kPlaneThreads - 1) / kPlaneThreads < 8
                           ? (NL + kPlaneThreads - 1) / kPlaneThreads : 8;
    for (int base = tid; base < NL; base += kPlaneThreads * LB) {
        cplx<T> v[LB];
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            const int idx = base + u * kPlaneThreads < NL ? base + u * kPlaneThreads : NL - 1;
            const int j = idx / nin, x = idx - j * nin;
            v[u] = {plane[(2 * j) * nin + x], plane[(2 * j + 1) * nin + x]};
        }
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            const int idx = base + u * kPlaneThreads;
            if (idx < NL) {
                const int j = idx / nin, x = idx - j * nin;
                xb[j * N + cpos(j, x)] = v[u];
            }
        }
    }
    fill_twiddles<T>(tw, tw_g, N, tid, kPlaneThreads);
    __syncthreads();
    fft_col<T, false, N, HALF>(xb, npair, tw, tid, kPlaneThreads);   // ends with a barrier
    cplx<T> *out = spec + ((int64_t)c * nin + z) * N * nh;
    for (int k0 = 0; k0 < nh; k0 += kPlaneChunk) {
        const int cn = nh - k0 < kPlaneChunk ? nh - k0 : kPlaneChunk;
        // y transforms, first step: 16-point FFTs over n1 of x[n1 N2 + t2]
        for (int it = tid; it < cn * N2; it += kPlaneThreads) {
            const int t2 = it / cn, kl = it - t2 * cn, k = k0 + kl;
            cplx<T> v[16];
            static_for<0, 16>([&](auto in) {
                constexpr int n1 = decltype(in)::value;
                if constexpr (HALF && n1 >= 8) {
                    v[n1] = {T(0), T(0)};
                } else {
                    const int y = n1 * N2 + t2, j = y >> 1;
                    const cplx<T> zk = xb[j * N + cpos(j, k & (N - 1))];
                    const cplx<T> zm = xb[j * N + cpos(j, (N - k) & (N - 1))];
                    if ((y & 1) == 0) v[n1] = {T(0.5) * (zk.re + zm.re), T(0.5) * (zk.im - zm.im)};
                    else v[n1] = {T(0.5) * (zk.im + zm.im), T(-0.5) * (zk.re - zm.re)};
                }
            });
            fft_reg<16, false, T>(v);
            static_for<0, 16>([&](auto ik) {
                constexpr int k1 = decltype(ik)::value;
                const cplx<T> w = k1 == 0 ? cplx<T>{T(1), T(0)} : tw_n(tw, t2 * k1, false);
                yb[(t2 * 16 + k1) * CWS + kl] = k1 == 0 ? v[k1] : cmul(v[k1], w);
            });
        }
        __syncthreads();
        // second step: N2-point FFTs over t2, spectrum rows y = k2 * 16 + k1
        for (int it = tid; it < cn * 16; it += kPlaneThreads) {
            const int k1 = it / cn, kl = it - k1 * cn;
            cplx<T> u[N2];
            static_for<0, N2>([&](auto it2) {
                constexpr int t2 = decltype(it2)::value;
                u[t2] = yb[(t2 * 16 + k1) * CWS + kl];
            });
            fft_reg<N2, false, T>(u);
            static_for<0, N2>([&](auto ik2) {
                constexpr int k2 = decltype(ik2)::value;
                out[(k2 * 16 + k1) * nh + k0 + kl] = u[k2];
            });
        }
        __syncthreads();   // yb is refilled by the next chunk
    }
}

template <typename T, int N, bool HALF>
__global__ void __launch_bounds__(kPlaneThreads) k_plane_inv_n(const cplx<T> *__restrict__ spec,
                                                               T *__restrict__ L,
                                                               const cplx<T> *__restrict__ tw_g,
                                                               T scale, int P) {
    constexpr int nout = HALF ? N / 2 : N, npair = nout / 2, nh = N / 2 + 1, N2 = N / 16;
    constexpr int CWS = kPlaneChunk;
    constexpr int K2 = HALF ? N2 / 2 : N2;   // y rows kept: k2 * 16 + k1 < nout
    extern __shared__ __align__(16) unsigned char lds_raw[];
    cplx<T> *tw = (cplx<T> *)lds_raw;
    cplx<T> *xb = tw + N;
    cplx<T> *yb = xb + npair * N;
    const int z = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
    {
        const int64_t sy = blockIdx.z;
        spec += sy * P * nout * N * nh;
        L += sy * P * nout * nout * nout;
    }
    fill_twiddles<T>(tw, tw_g, N, tid, kPlaneThreads);
    __syncthreads();
    const cplx<T> *in = spec + ((int64_t)c * nout + z) * N * nh;
    for (int k0 = 0; k0 < nh; k0 += kPlaneChunk) {
        const int cn = nh - k0 < kPlaneChunk ? nh - k0 : kPlaneChunk;
        // y inverse transforms, first step, straight from memory (lanes take
        // consecutive kx)
        for (int it = tid; it < cn * N2; it += kPlaneThreads) {
            const int t2 = it / cn, kl = it - t2 * cn;
            cplx<T> v[16];
            static_for<0, 16>([&](auto in1) {
                constexpr int n1 = decltype(in1)::value;
                v[n1] = in[(n1 * N2 + t2) * nh + k0 + kl];
            });
            fft_reg<16, true, T>(v);
            static_for<0, 16>([&](auto ik) {
                constexpr int k1 = decltype(ik)::value;
                const cplx<T> w = k1 == 0 ? cplx<T>{T(1), T(0)} : tw_n(tw, t2 * k1, true);
                yb[(t2 * 16 + k1) * CWS + kl] = k1 == 0 ? v[k1] : cmul(v[k1], w);
            });
        }
        __syncthreads();
        // second step, rows y = k2 * 16 + k1 < nout, into the C2R row pairs:
        // even rows y = 2j give A, odd rows B, and Z_j[k] = A[k] + i B[k],
        // Z_j[N - k] = conj(A[k]) + i conj(B[k]) (0 < k < N/2); the even rows
        // are written first, the odd ones added after a barrier
        for (int parity = 0; parity < 2; ++parity) {
            for (int it = tid; it < cn * 8; it += kPlaneThreads) {
                const int kh = it / cn, kl = it - kh * cn, k1 = 2 * kh + parity, k = k0 + kl;
                cplx<T> u[N2];
                static_for<0, N2>([&](auto it2) {
                    constexpr int t2 = decltype(it2)::value;
                    u[t2] = yb[(t2 * 16 + k1) * CWS + kl];
                });
                fft_reg<N2, true, T>(u);
                static_for<0, K2>([&](auto ik2) {
                    constexpr int k2 = decltype(ik2)::value;
                    const int j = (k2 * 16 + k1) >> 1;
                    cplx<T> *row = xb + j * N;
                    const cplx<T> a = u[k2];
                    if (parity == 0) {
                        row[cpos(j, k)] = a;
                        if (k >= 1 && k < N / 2) row[cpos(j, N - k)] = {a.re, -a.im};
                    } else {
                        cplx<T> &zk = row[cpos(j, k)];
                        zk = {zk.re - a.im, zk.im + a.re};
                        if (k >= 1 && k < N / 2) {
                            cplx<T> &zm = row[cpos(j, N - k)];
                            zm = {zm.re + a.im, zm.im + a.re};
                        }
                    }
                });
            }
            __syncthreads();
        }
    }
    // x inverse transforms of the row pairs, the first nout outputs kept
    fft_col<T, true, N, HALF>(xb, npair, tw, tid, kPlaneThreads);
    T *plane = L + ((int64_t)c * nout + z) * nout * nout;
    for (int idx = tid; idx < nout * nout; idx += kPlaneThreads) {
        const int y = idx / nout, x = idx - y * nout, j = y >> 1;
        const cplx<T> v = xb[j * N + cpos(j, x)];
        plane[idx] = ((y & 1) ? v.im : v.re) * scale;
    }
}

template <typename T, int N>
static size_t plane_n_lds(bool half) {
    const int npair = (half ? N / 2 : N) / 2;
    return (size_t)(N + npair * N + N * kPlaneChunk) * sizeof(cplx<T>);
}

template <typename T, int N>
static hipError_t plane_n_launch(const FFTArgs &a, int stage, hipStream_t s) {
    const int P = nreal(a.p), n = a.n, nsys = a.nsys > 0 ? a.nsys : 1;
    const bool half = a.open != 0;
    const size_t lds = plane_n_lds<T, N>(half);
    hipError_t e = hipSuccess;
    if (stage == 0) {
        const void *k = half ? (const void *)k_plane_fwd_n<T, N, true>
                             : (const void *)k_plane_fwd_n<T, N, false>;
        if (lds > 65536 && (e = set_max_lds(k, lds)) != hipSuccess) return e;
        const int rows = half ? P : P + 1;   // periodic: one extra row of q|u|^2 sums
        if (half)
            hipLaunchKernelGGL((k_plane_fwd_n<T, N, true>), dim3(n, rows, nsys),
                               dim3(kPlaneThreads), lds, s, (const T *)a.M, (cplx<T> *)a.spec,
                               (const cplx<T> *)a.tw, P, nullptr);
        else
            hipLaunchKernelGGL((k_plane_fwd_n<T, N, false>), dim3(n, rows, nsys),
                               dim3(kPlaneThreads), lds, s, (const T *)a.M, (cplx<T> *)a.spec,
                               (const cplx<T> *)a.tw, P, a.qr2_partial);
    } else {
        const void *k = half ? (const void *)k_plane_inv_n<T, N, true>
                             : (const void *)k_plane_inv_n<T, N, false>;
        if (lds > 65536 && (e = set_max_lds(k, lds)) != hipSuccess) return e;
        const T scale = T(1.0 / ((double)N * N * N));
        if (half)
            hipLaunchKernelGGL((k_plane_inv_n<T, N, true>), dim3(n, P, nsys), dim3(kPlaneThreads),
                               lds, s, (const cplx<T> *)a.spec, (T *)a.L, (const cplx<T> *)a.tw,
                               scale, P);
        else
            hipLaunchKernelGGL((k_plane_inv_n<T, N, false>), dim3(n, P, nsys), dim3(kPlaneThreads),
                               lds, s, (const cplx<T> *)a.spec, (T *)a.L, (const cplx<T> *)a.tw,
                               scale, P);
    }
    return hipGetLastError();
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
    return set_max_lds((const void *)k, bytes);
}

// Column stage, one instantiation per order in the pmmm_column_*.hip units.
template <int PO, typename T>
hipError_t column_launch(const FFTArgs &a, hipStream_t s);

// Shape of a plane block: 256 threads in cpb groups, one component each.
// Small planes keep only a few lanes busy per FFT stage, so when there are
// planes enough to fill the GPU (at least 1024 of them) a block takes 8
// components up to 16 points, 4 at 32, 2 at 64; a launch with fewer planes is
// latency-bound and keeps one component per block (shorter chains).  The y
// pass of a 128-point plane runs in chunks of 16 kx columns (row stride 17
// against bank conflicts), so that a block needs 50 KB of LDS instead of
// 100 KB and three share a CU.
struct PlaneShape {
    int threads, cw, cws, cpb;
    size_t lds;
};
static PlaneShape plane_shape(int n, int nf, int P, int nsys, size_t csz) {
    const int nh = nf / 2 + 1;
    PlaneShape ps;
    ps.threads = 256;
    ps.cpb = nf <= 16 ? 8 : (nf == 32 ? 4 : (nf == 64 ? 2 : 1));
    if ((int64_t)n * P * nsys < 1024) ps.cpb = 1;
    ps.cw = nf >= 128 ? 16 : nh;
    ps.cws = ps.cw == nh ? nh : ps.cw + 1;
    ps.lds = (size_t)(nf / 2 + ps.cpb * ((n / 2) * lds_line(nf) + nf * ps.cws)) * csz;
    return ps;
}

template <typename T>
hipError_t launch_conv_stage(const FFTArgs &a, int stage, hipStream_t s) {
    if (a.generic) return launch_generic_stage<T>(a, stage, s);
    const int P = nreal(a.p);
    const int nf = a.nf, logn = ilog2(nf), nh = nf / 2 + 1, n = a.n;
    const int nsys = a.nsys > 0 ? a.nsys : 1;
    const size_t csz = sizeof(cplx<T>);
    const PlaneShape ps = plane_shape(n, nf, P, nsys, csz);
    const size_t lds_plane = ps.lds;
    hipError_t e = hipSuccess;
    if (stage != 1 && (nf == 64 || nf == 128)) {
        if (sizeof(T) == 8 && nf == 128) return hipErrorInvalidValue;
        return nf == 64 ? plane_n_launch<T, 64>(a, stage, s) : plane_n_launch<T, 128>(a, stage, s);
    }
    if (stage == 0) {
        e = ensure_lds(k_plane_fwd<T>, lds_plane);
        if (e != hipSuccess) return e;
        // periodic: one extra row of blocks sums q|u|^2 per plane
        const int crows = (P + ps.cpb - 1) / ps.cpb;
        const int rows = a.open ? crows : crows + 1;
        hipLaunchKernelGGL(k_plane_fwd<T>, dim3(n, rows, nsys), dim3(ps.threads), lds_plane, s, n,
                           logn, (const T *)a.M, (cplx<T> *)a.spec, (const cplx<T> *)a.tw, P,
                           a.open ? nullptr : a.qr2_partial, ps.cw, ps.cws, ps.cpb);
        return hipGetLastError();
    }
    if (stage == 1) {
        switch (a.p) {
            case 0: return column_launch<0, T>(a, s);
            case 1: return column_launch<1, T>(a, s);
            case 2: return column_launch<2, T>(a, s);
            case 3: return column_launch<3, T>(a, s);
            case 4: return column_launch<4, T>(a, s);
            case 5: return column_launch<5, T>(a, s);
            case 6: return column_launch<6, T>(a, s);
            case 7: return column_launch<7, T>(a, s);
            case 8: return column_launch<8, T>(a, s);
            case 9: return column_launch<9, T>(a, s);
            case 10: return column_launch<10, T>(a, s);
            default: return hipErrorInvalidValue;
        }
    }
    e = ensure_lds(k_plane_inv<T>, lds_plane);
    if (e != hipSuccess) return e;
    const T scale = T(1.0 / ((double)nf * nf * nf));
    hipLaunchKernelGGL(k_plane_inv<T>, dim3(n, (P + ps.cpb - 1) / ps.cpb, nsys), dim3(ps.threads),
                       lds_plane, s, n, logn, (const cplx<T> *)a.spec, (T *)a.L,
                       (const cplx<T> *)a.tw, scale, P, ps.cw, ps.cws, ps.cpb);
    return hipGetLastError();
}

template hipError_t launch_conv_stage<float>(const FFTArgs &, int, hipStream_t);
template hipError_t launch_conv_stage<double>(const FFTArgs &, int, hipStream_t);

}  // namespace pmmm
