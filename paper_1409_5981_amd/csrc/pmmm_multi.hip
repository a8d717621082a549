// Multi-charge far field: S charge sets on one set of positions and one
// periodic mesh.  Every step of Sec. 2.1 is linear in the charges, so the
// binning, the harmonics of each particle and the transfer kernel are shared
// and each set runs the same P2M / FFT / M2L / FFT / L2P sequence.  Stacking
// the sets turns the wave-space M2L of eq. realmatrix at one frequency into a
// real (P x P) matrix times (P x 2S) matrix product, which runs on the BF16
// matrix cores with split operands: an FP32 value v is written as
// h0 + h1 (+ h2), h_i = bf16(v - h0 - ... - h_{i-1}), and the products
// h_i g_j with i + j < terms are accumulated in FP32.  Two terms (three
// products) keep about 16 bits of each operand; three terms (six products)
// keep all 24.
//
//   k_p2m_multi     one wave per cell, one lane per set: eq. P2M with the
//                   harmonics R(r_M - r_i) of the cell's particles staged in
//                   LDS and read by every lane.
//   k_slab_fwd      one component of one set and the B planes z1 + 4 j:
//                   x and y FFTs, then the first z stage.
//   k_column_multi  one (ky, kx) column, one z residue r and a tile of sets:
//                   last z stage, the M2L product at the four frequencies
//                   kz = B q + r, inverse z stage.
//   k_slab_inv      inverse of k_slab_fwd, scaled by 1/nf^3.
//   k_l2p_multi     one wave per cell, one lane per set: eq. L2P and the
//                   order-one eq. L2L of eq. phigrad, with the cell's local
//                   expansion folded into per-set coefficient vectors.
//
// Split z transform, nf = 4 B, z = z1 + 4 j, kz = B q + r:
//   M~(B q + r) = sum_z1 W_4^(z1 q) W_nf^(z1 r) sum_j W_B^(j r) M(z1 + 4 j)
//   L(z1 + 4 j) = sum_r W_B^(-j r) W_nf^(-z1 r) sum_q W_4^(-z1 q) L~(B q + r)
// Between the slab and column kernels the spectra live as
// X[r][col][z1][s P + b] (col = ky (nf/2+1) + kx), so one column block reads
// and writes one contiguous range per z1.
#include "pmmm_internal.h"

namespace pmmm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kZA = kMultiZA;

// LDS written by some lanes of a wave and read by others of the same wave:
// the wave's LDS operations complete in order, so a wave-scope fence and a
// compiler barrier suffice.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__host__ __device__ constexpr int order_of(int a) {
    int l = 0;
    while ((l + 1) * (l + 1) <= a) ++l;
    return l;
}

// exp(-2 pi i e / nf) from the half table tw[k] = exp(-2 pi i k / nf).
__device__ __forceinline__ cplx<float> tw_at(const cplx<float> *tw, int e, int nf) {
    e &= nf - 1;
    if (e < nf / 2) return tw[e];
    const cplx<float> w = tw[e - nf / 2];
    return {-w.re, -w.im};
}

// ------------------------------------------------------------------- P2M
// Row stride of the staged harmonics (16-byte rows for vector LDS reads).
__host__ __device__ constexpr int stage_row(int cols) { return (cols + 3) & ~3; }

template <int PO>
__global__ void __launch_bounds__(256) k_p2m_multi(int K, int cells_per_block,
                                                   const int *__restrict__ start,
                                                   const particle4<float> *__restrict__ sorted,
                                                   const int *__restrict__ perm,
                                                   const float *__restrict__ q, int64_t ld, int S,
                                                   float *__restrict__ M,
                                                   int *__restrict__ zero_count) {
    constexpr int P = nreal(PO);
    constexpr int RS = stage_row(P + 1);     // harmonics, then |u|^2
    __shared__ __align__(16) float rb[4][64 * RS];
    __shared__ int oi[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (zero_count != nullptr) {
        const int gid = blockIdx.x * 256 + threadIdx.x;
        if (gid < K) zero_count[gid] = 0;
    }
    float *R = rb[w];
    int *O = oi[w];
    const int c0 = blockIdx.x * cells_per_block;
    const int c1 = min(c0 + cells_per_block, K);
    for (int c = c0 + w; c < c1; c += 4) {
        const int s0 = start[c], s1 = start[c + 1];
        float acc[P + 1];
#pragma unroll
        for (int a = 0; a <= P; ++a) acc[a] = 0.f;
        for (int base = s0; base < s1; base += 64) {
            const int cnt = min(64, s1 - base);
            if (lane < cnt) {
                const particle4<float> r = sorted[base + lane];
                float h[P];
                regular_harmonics<PO, float>(-r.ux, -r.uy, -r.uz, h);   // R(r_M - r_i)
#pragma unroll
                for (int a = 0; a < P; ++a) R[lane * RS + a] = h[a];
                R[lane * RS + P] = r.ux * r.ux + r.uy * r.uy + r.uz * r.uz;
                O[lane] = perm[base + lane];
            }
            wave_lds_sync();
            if (lane < S) {
                for (int j0 = 0; j0 < cnt; j0 += 8) {
                    float qv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        qv[u] = (j0 + u < cnt) ? q[(int64_t)O[j0 + u] * ld + lane] : 0.f;
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        if (j0 + u < cnt) {
                            const float *rj = R + (j0 + u) * RS;
#pragma unroll
                            for (int a = 0; a <= P; ++a) acc[a] = fmaf(qv[u], rj[a], acc[a]);
                        }
                    }
                }
            }
            wave_lds_sync();   // every lane is done with this chunk
        }
        if (lane < S) {
#pragma unroll
            for (int a = 0; a <= P; ++a) M[((int64_t)lane * (P + 1) + a) * K + c] = acc[a];
        }
    }
}

// ------------------------------------------------------------------- L2P
// Per-set coefficient vectors of one cell: Phi = sum_a lh[a] R_a(u) and
// grad Phi = sum_a' (vx, vy, vz)[a'] R_a'(u) over the components of order
// <= p - 1 (eq. L2P; eq. L2L to destination order one, eq. phigrad).
template <int PO>
__device__ __forceinline__ void l2p_vectors(const float *Lc, float *lh, float *vx, float *vy,
                                            float *vz) {
    static_for<0, PO + 1>([&](auto il) {
        constexpr int l = decltype(il)::value;
        lh[ridx(l, 0)] = Lc[ridx(l, 0)];
        static_for<1, l + 1>([&](auto im) {
            constexpr int m = decltype(im)::value;
            lh[ridx(l, m)] = 2.f * Lc[ridx(l, m)];
            lh[ridx(l, -m)] = -2.f * Lc[ridx(l, -m)];
        });
    });
    static_for<0, PO>([&](auto ik) {
        constexpr int k = decltype(ik)::value;
        constexpr int lam = k + 1;
        auto lre = [&](int mu) { return Lc[ridx(lam, mu)]; };
        static_for<0, k + 1>([&](auto iu) {
            constexpr int mu = decltype(iu)::value;
            const float re_up = Lc[ridx(lam, mu + 1)];
            const float im_up = Lc[ridx(lam, -(mu + 1))];
            if constexpr (mu == 0) {
                vx[ridx(k, 0)] = -re_up;
                vy[ridx(k, 0)] = im_up;
                vz[ridx(k, 0)] = lre(0);
            } else {
                const float re_dn = Lc[ridx(lam, mu - 1)];
                const float im_dn = (mu - 1 > 0) ? Lc[ridx(lam, -(mu - 1))] : 0.f;
                // d1re coefficients of Re R_k^mu and Im R_k^mu; gx = -d1re
                vx[ridx(k, mu)] = -(re_up - re_dn);
                vx[ridx(k, -mu)] = -(-im_up + im_dn);
                // gy = d1im
                vy[ridx(k, mu)] = im_up + im_dn;
                vy[ridx(k, -mu)] = re_up + re_dn;
                // gz = d0
                vz[ridx(k, mu)] = 2.f * Lc[ridx(lam, mu)];
                vz[ridx(k, -mu)] = -2.f * Lc[ridx(lam, -mu)];
            }
        });
    });
}

template <int PO>
__global__ void __launch_bounds__(256) k_l2p_multi(int K, int cells_per_block,
                                                   const int *__restrict__ start,
                                                   const particle4<float> *__restrict__ sorted,
                                                   const int *__restrict__ perm,
                                                   const float *__restrict__ L, int S,
                                                   const double *__restrict__ qtot,
                                                   float alpha_c, float inv_h, int64_t ld,
                                                   float *__restrict__ phi_out,
                                                   float *__restrict__ gx_out,
                                                   float *__restrict__ gy_out,
                                                   float *__restrict__ gz_out) {
    constexpr int P = nreal(PO);
    constexpr int PD = nreal(PO - 1);        // components of order <= p - 1
    constexpr int RS = stage_row(P + 3);     // harmonics, then u
    __shared__ __align__(16) float rb[4][64 * RS];
    __shared__ int oi[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    float *R = rb[w];
    int *O = oi[w];
    const float ih2 = inv_h * inv_h;
    const int c0 = blockIdx.x * cells_per_block;
    const int c1 = min(c0 + cells_per_block, K);
    for (int c = c0 + w; c < c1; c += 4) {
        const int s0 = start[c], s1 = start[c + 1];
        if (s1 == s0) continue;
        float lh[P], vx[PD > 0 ? PD : 1], vy[PD > 0 ? PD : 1], vz[PD > 0 ? PD : 1];
        float qt = 0.f;
        if (lane < S) {
            float Lc[P];
#pragma unroll
            for (int a = 0; a < P; ++a) Lc[a] = L[((int64_t)lane * P + a) * K + c];
            l2p_vectors<PO>(Lc, lh, vx, vy, vz);
            // charged periodic system: Phi += 2 pi/(3V) Q (|u|^2 - 3/(2 alpha^2)),
            // grad += 4 pi/(3V) Q u, V = K in cell units
            qt = (float)(qtot[lane] * 3.14159265358979323846 / (3.0 * (double)K));
        }
        const float shift = 1.5f / (alpha_c * alpha_c);
        for (int base = s0; base < s1; base += 64) {
            const int cnt = min(64, s1 - base);
            if (lane < cnt) {
                const particle4<float> r = sorted[base + lane];
                float h[P];
                regular_harmonics<PO, float>(r.ux, r.uy, r.uz, h);
#pragma unroll
                for (int a = 0; a < P; ++a) R[lane * RS + a] = h[a];
                R[lane * RS + P] = r.ux;
                R[lane * RS + P + 1] = r.uy;
                R[lane * RS + P + 2] = r.uz;
                O[lane] = perm[base + lane];
            }
            wave_lds_sync();
            if (lane < S) {
                for (int j = 0; j < cnt; ++j) {
                    const float *rj = R + j * RS;
                    float ph = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
                    for (int a = 0; a < PD; ++a) {
                        const float v = rj[a];
                        ph = fmaf(lh[a], v, ph);
                        gx = fmaf(vx[a], v, gx);
                        gy = fmaf(vy[a], v, gy);
                        gz = fmaf(vz[a], v, gz);
                    }
#pragma unroll
                    for (int a = PD; a < P; ++a) ph = fmaf(lh[a], rj[a], ph);
                    const float ux = rj[P], uy = rj[P + 1], uz = rj[P + 2];
                    ph += 2.f * qt * (ux * ux + uy * uy + uz * uz - shift);
                    gx += 4.f * qt * ux;
                    gy += 4.f * qt * uy;
                    gz += 4.f * qt * uz;
                    const int64_t o = (int64_t)O[j] * ld + lane;
                    phi_out[o] = ph * inv_h;
                    gx_out[o] = gx * ih2;
                    gy_out[o] = gy * ih2;
                    gz_out[o] = gz * ih2;
                }
            }
            wave_lds_sync();
        }
    }
}

// ----------------------------------------------------------------- slabs
// Block -> (z1, component): each XCD (blocks are dealt round-robin over the
// 8 XCDs) takes a contiguous range, so the blocks that run together on one
// XCD share z1 and hold neighbouring components; their 8-byte stores to
// X[r][col][z1][.] then meet in the same L2 lines.
__device__ __forceinline__ int slab_block(int nblk) {
    const int per_xcd = (nblk + 7) / 8;
    return (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
}

template <int B>
__global__ void __launch_bounds__(256) k_slab_fwd(int logn, int S, int P,
                                                  const float *__restrict__ M,
                                                  cplx<float> *__restrict__ X,
                                                  const cplx<float> *__restrict__ tw_g,
                                                  double *__restrict__ qr2_partial) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int nf = 1 << logn, nh = nf / 2 + 1, npair = nf / 2, ls = lds_line(nf);
    const int ncol = nf * nh, SP = S * P;
    const int64_t K = (int64_t)nf * nf * nf;
    cplx<float> *tw = (cplx<float> *)lds_raw;
    cplx<float> *rows = tw + nf / 2;                 // [B][npair][ls]
    cplx<float> *slab = rows + B * npair * ls;       // [nf y][B j][nh kx]
    const int v = slab_block(kZA * SP);
    if (v >= kZA * SP) return;
    const int z1 = v / SP, c = v - z1 * SP;
    const int s = c / P, b = c - s * P;
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int k = tid; k < nf / 2; k += nthr) tw[k] = tw_g[k];
    const float *comp = M + ((int64_t)s * (P + 1) + b) * K;
    // planes z = z1 + 4 j as pairs of real rows packed into complex rows
    const int nrow = B * npair * nf;
    for (int base = tid; base < nrow; base += nthr * 8) {
        cplx<float> vv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = base + u * nthr;
            if (idx < nrow) {
                const int j = idx / (npair * nf), rem = idx - j * npair * nf;
                const int jj = rem >> logn, x = rem & (nf - 1);
                const float *pl = comp + (int64_t)(z1 + kZA * j) * nf * nf;
                vv[u].re = pl[(2 * jj) * nf + x];
                vv[u].im = pl[(2 * jj + 1) * nf + x];
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = base + u * nthr;
            if (idx < nrow) {
                const int j = idx / (npair * nf), rem = idx - j * npair * nf;
                const int jj = rem >> logn, x = rem & (nf - 1);
                rows[(j * npair + jj) * ls + x] = vv[u];
            }
        }
    }
    __syncthreads();
    fft_lines<float, false>(rows, logn, B * npair, ls, 1, tw, tid, nthr);
    for (int idx = tid; idx < B * nf * nh; idx += nthr) {
        const int j = idx / (nf * nh), rem = idx - j * nf * nh;
        const int y = rem / nh, k = rem - y * nh;
        const cplx<float> *row = rows + (j * npair + (y >> 1)) * ls;
        const cplx<float> zk = row[k & (nf - 1)];
        const cplx<float> zm = row[(nf - k) & (nf - 1)];
        cplx<float> o;
        if ((y & 1) == 0) {
            o.re = 0.5f * (zk.re + zm.re);
            o.im = 0.5f * (zk.im - zm.im);
        } else {
            o.re = 0.5f * (zk.im + zm.im);
            o.im = -0.5f * (zk.re - zm.re);
        }
        slab[(y * B + j) * nh + k] = o;
    }
    __syncthreads();
    // y transforms: line (j, kx) starts at j nh + kx, elements B nh apart
    fft_lines<float, false>(slab, logn, B * nh, 1, B * nh, tw, tid, nthr);
    // first z stage: B-point DFT over j, twiddle W_nf^(z1 r)
    for (int pt = tid; pt < ncol; pt += nthr) {
        const int y = pt / nh, kx = pt - y * nh;
        cplx<float> w8[B];
#pragma unroll
        for (int j = 0; j < B; ++j) w8[j] = slab[(y * B + j) * nh + kx];
        fft_reg<B, false, float>(w8);
#pragma unroll
        for (int r = 0; r < B; ++r) {
            const cplx<float> o = r == 0 ? w8[0] : cmul(w8[r], tw_at(tw, z1 * r, nf));
            X[(((int64_t)r * ncol + pt) * kZA + z1) * SP + c] = o;
        }
    }
    if (b == 0) {
        // this set's sum of q|u|^2 over the block's planes (component P of M),
        // fixed-order reduction
        __shared__ double red[256];
        const float *pq = M + ((int64_t)s * (P + 1) + P) * K;
        double acc = 0.0;
        for (int idx = tid; idx < B * nf * nf; idx += nthr) {
            const int j = idx / (nf * nf), rem = idx - j * nf * nf;
            acc += (double)pq[(int64_t)(z1 + kZA * j) * nf * nf + rem];
        }
        red[tid] = acc;
        __syncthreads();
        for (int off = 128; off >= 1; off >>= 1) {
            if (tid < off) red[tid] += red[tid + off];
            __syncthreads();
        }
        if (tid == 0) qr2_partial[s * kZA + z1] = red[0];
    }
}

template <int B>
__global__ void __launch_bounds__(256) k_slab_inv(int logn, int S, int P,
                                                  const cplx<float> *__restrict__ X,
                                                  float *__restrict__ L,
                                                  const cplx<float> *__restrict__ tw_g,
                                                  float scale) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int nf = 1 << logn, nh = nf / 2 + 1, npair = nf / 2, ls = lds_line(nf);
    const int ncol = nf * nh, SP = S * P;
    const int64_t K = (int64_t)nf * nf * nf;
    cplx<float> *tw = (cplx<float> *)lds_raw;
    cplx<float> *rows = tw + nf / 2;
    cplx<float> *slab = rows + B * npair * ls;
    const int v = slab_block(kZA * SP);
    if (v >= kZA * SP) return;
    const int z1 = v / SP, c = v - z1 * SP;
    const int s = c / P, b = c - s * P;
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int k = tid; k < nf / 2; k += nthr) tw[k] = tw_g[k];
    // last z stage: B-point inverse DFT over r into the planes z1 + 4 j
    for (int pt = tid; pt < ncol; pt += nthr) {
        cplx<float> w8[B];
#pragma unroll
        for (int r = 0; r < B; ++r) w8[r] = X[(((int64_t)r * ncol + pt) * kZA + z1) * SP + c];
        fft_reg<B, true, float>(w8);
        const int y = pt / nh, kx = pt - y * nh;
#pragma unroll
        for (int j = 0; j < B; ++j) slab[(y * B + j) * nh + kx] = w8[j];
    }
    __syncthreads();
    fft_lines<float, true>(slab, logn, B * nh, 1, B * nh, tw, tid, nthr);
    // C2R along x: rows 2jj and 2jj+1 of a plane packed into one complex row
    for (int idx = tid; idx < B * npair * nf; idx += nthr) {
        const int j = idx / (npair * nf), rem = idx - j * npair * nf;
        const int jj = rem >> logn, k = rem & (nf - 1);
        const cplx<float> *ra = slab + ((2 * jj) * B + j) * nh;
        const cplx<float> *rb = slab + ((2 * jj + 1) * B + j) * nh;
        cplx<float> A, Bv;
        if (k <= nf / 2) {
            A = ra[k];
            Bv = rb[k];
        } else {
            A = ra[nf - k];
            Bv = rb[nf - k];
            A.im = -A.im;
            Bv.im = -Bv.im;
        }
        rows[(j * npair + jj) * ls + k] = {A.re - Bv.im, A.im + Bv.re};
    }
    __syncthreads();
    fft_lines<float, true>(rows, logn, B * npair, ls, 1, tw, tid, nthr);
    float *comp = L + ((int64_t)s * P + b) * K;
    for (int idx = tid; idx < B * nf * nf; idx += nthr) {
        const int j = idx / (nf * nf), rem = idx - j * nf * nf;
        const int y = rem / nf, x = rem - y * nf;
        const cplx<float> o = rows[(j * npair + (y >> 1)) * ls + x];
        comp[(int64_t)(z1 + kZA * j) * nf * nf + rem] = ((y & 1) ? o.im : o.re) * scale;
    }
}

// ----------------------------------------------------------- column GEMM
template <int NS>
__device__ __forceinline__ void split_bf16(float v, __bf16 (&h)[NS]) {
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        h[i] = (__bf16)v;
        v -= (float)h[i];
    }
}

__device__ __forceinline__ float decode_term(const float *g, unsigned code) {
    const unsigned s1 = (code >> 9) & 3u, s2 = (code >> 20) & 3u;
    const float f1 = (float)((int)(s1 & 1u) - (int)(s1 >> 1));
    const float f2 = (float)((int)(s2 & 1u) - (int)(s2 >> 1));
    return f1 * g[code & 511u] + f2 * g[(code >> 11) & 511u];
}

template <int PO, int NS>
struct ColumnMultiShape {
    static constexpr int P = nreal(PO), Q = nreal(2 * PO);
    static constexpr int RT = (P + 15) / 16, KS = (P + 31) / 32;
    static constexpr int ITEMS = RT * KS * 64;          // A fragments of one split
    static constexpr int NIT = (ITEMS + 255) / 256;     // per thread
    static constexpr size_t abuf_bytes = (size_t)NS * ITEMS * 16;
    static constexpr size_t gq_bytes = ((size_t)kZA * Q * 4 + 15) & ~(size_t)15;
    static size_t lds(int st) {
        return abuf_bytes + gq_bytes + (size_t)st * 4 * 4 + (size_t)kZA * st * P * 8;
    }
};

// Block: 256 threads, one (ky, kx) column, one residue r and sets
// [st0, st0 + ST).  LDS: A fragments of the current frequency (every split),
// the kernel values of the four frequencies, the zero-frequency moments for
// the corrections, and xb[q][s P + b] (moment spectra, then local spectra).
template <int PO, int NS>
__global__ void __launch_bounds__(256) k_column_multi(int logn, int S, int ST,
                                                      const float *__restrict__ green,
                                                      cplx<float> *__restrict__ X,
                                                      const cplx<float> *__restrict__ tw_g,
                                                      const unsigned *__restrict__ tmap,
                                                      const double *__restrict__ qr2_partial,
                                                      double *__restrict__ qtot) {
    using Sh = ColumnMultiShape<PO, NS>;
    constexpr int P = Sh::P, Q = Sh::Q, RT = Sh::RT, KS = Sh::KS;
    constexpr int ITEMS = Sh::ITEMS, NIT = Sh::NIT;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    bf16x8 *abuf = (bf16x8 *)lds_raw;                                   // [NS][RT][KS][64]
    float *gq = (float *)(lds_raw + Sh::abuf_bytes);                    // [4][Q]
    float *dcm = (float *)(lds_raw + Sh::abuf_bytes + Sh::gq_bytes);    // [ST][4]
    cplx<float> *xb = (cplx<float> *)(dcm + ST * 4);                   // [4][ST P]
    const int nf = 1 << logn, nh = nf / 2 + 1, nhp = (nh + 3) & ~3, ncol = nf * nh;
    const int B = nf / kZA;
    const int SP = S * P, STP = ST * P;
    const int nst = (S + ST - 1) / ST;
    const int nblk = B * ncol * nst;
    const int per_xcd = (nblk + 7) / 8;
    const int v = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (v >= nblk) return;
    const int tile = v % nst, rest = v / nst;
    const int r = rest % B, col = rest / B;
    const int st0 = tile * ST, stc = min(ST, S - st0);
    const int ky = col / nh, kx = col - ky * nh;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const bool dc_block = (r == 0 && col == 0);

    // kernel values of kz = B q + r from the stored quadrant, mirrored
    // (ky > nf/2: Im-part components negate; kz > nf/2: (n, k) times
    // (-1)^(n+|k|))
    {
        const int kyr = ky <= nf / 2 ? ky : nf - ky;
        const float *gcol = green + (int64_t)(kyr * nh + kx) * Q * nhp;
        for (int idx = tid; idx < kZA * Q; idx += 256) {
            const int qq = idx / Q, j = idx - qq * Q;
            const int kz = B * qq + r;
            const int kzr = kz <= nf / 2 ? kz : nf - kz;
            const int nn = order_of(j), kk = j - nn * nn - nn;
            const int ak = kk < 0 ? -kk : kk;
            const bool neg = ((ky > nf / 2) && kk < 0) != ((kz > nf / 2) && ((nn + ak) & 1));
            const float gv = gcol[j * nhp + kzr];
            gq[idx] = neg ? -gv : gv;
        }
    }
    // moment spectra of this tile, four z1 rows
    {
        const cplx<float> *src = X + ((int64_t)r * ncol + col) * kZA * SP + (int64_t)st0 * P;
        const int tot = kZA * stc * P, rowlen = stc * P;
        for (int base = tid; base < tot; base += 256 * 8) {
            cplx<float> vv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int idx = base + u * 256;
                if (idx < tot) {
                    const int z1 = idx / rowlen, i = idx - z1 * rowlen;
                    vv[u] = src[(int64_t)z1 * SP + i];
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int idx = base + u * 256;
                if (idx < tot) {
                    const int z1 = idx / rowlen, i = idx - z1 * rowlen;
                    xb[z1 * STP + i] = vv[u];
                }
            }
        }
    }
    // this thread's t-map codes (the same at every frequency)
    unsigned tm[NIT][8];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int item = tid + it * 256;
#pragma unroll
        for (int e = 0; e < 8; ++e) tm[it][e] = item < ITEMS ? tmap[item * 8 + e] : 0u;
    }
    __syncthreads();
    // last forward z stage (4-point DFT over z1), pre-multiply by i^(lam mod 2)
    for (int i = tid; i < stc * P; i += 256) {
        cplx<float> w4[kZA];
#pragma unroll
        for (int z1 = 0; z1 < kZA; ++z1) w4[z1] = xb[z1 * STP + i];
        fft_reg<kZA, false, float>(w4);
        const int sl = i / P, bb = i - sl * P;
        if (dc_block) {
            // zero frequency: M~_b(0) = sum over cells of M_b
            const int slot = bb == 0 ? 0 : bb == ridx(1, 0) ? 1 : bb == ridx(1, 1) ? 2
                             : bb == ridx(1, -1) ? 3 : -1;
            if (slot >= 0) dcm[sl * 4 + slot] = w4[0].re;
        }
        const bool odd = order_of(bb) & 1;
#pragma unroll
        for (int qq = 0; qq < kZA; ++qq) {
            const cplx<float> o = odd ? cplx<float>{-w4[qq].im, w4[qq].re} : w4[qq];
            xb[qq * STP + i] = o;
        }
    }
    __syncthreads();
    const double pi = 3.14159265358979323846;
    const int ntile = (2 * stc + 15) / 16;                // 16-column tiles of this block
    for (int qq = 0; qq < kZA; ++qq) {
        // A fragments of t(kz = B qq + r), every split
        const float *g = gq + qq * Q;
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int item = tid + it * 256;
            if (item < ITEMS) {
                bf16x8 fr[NS];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    __bf16 h[NS];
                    split_bf16<NS>(decode_term(g, tm[it][e]), h);
#pragma unroll
                    for (int sp = 0; sp < NS; ++sp) fr[sp][e] = h[sp];
                }
#pragma unroll
                for (int sp = 0; sp < NS; ++sp) abuf[sp * ITEMS + item] = fr[sp];
            }
        }
        __syncthreads();
        cplx<float> *xq = xb + qq * STP;
        for (int nt = wv; nt < ntile; nt += 4) {
            const int n = nt * 16 + (lane & 15);
            const int sl = n >> 1, part = n & 1;
            const bool colok = sl < stc;
            // B fragments: rows k = ks 32 + (lane/16) 8 + e, column n
            bf16x8 bfr[KS][NS];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int k = ks * 32 + (lane >> 4) * 8 + e;
                    float val = 0.f;
                    if (colok && k < P) {
                        const cplx<float> m = xq[sl * P + k];
                        val = part ? m.im : m.re;
                    }
                    __bf16 h[NS];
                    split_bf16<NS>(val, h);
#pragma unroll
                    for (int sp = 0; sp < NS; ++sp) bfr[ks][sp][e] = h[sp];
                }
            }
            f32x4 acc[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                acc[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    bf16x8 afr[NS];
#pragma unroll
                    for (int sp = 0; sp < NS; ++sp) afr[sp] = abuf[sp * ITEMS + (rt * KS + ks) * 64 + lane];
                    // smallest products first
#pragma unroll
                    for (int d = NS - 1; d >= 0; --d) {
#pragma unroll
                        for (int i = d; i >= 0; --i) {
                            acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[i], bfr[ks][d - i],
                                                                           acc[rt], 0, 0, 0);
                        }
                    }
                }
            }
            // D rows a = rt 16 + (lane/16) 4 + i, column n; L~_a = i^(l mod 2) acc
            if (colok) {
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int a = rt * 16 + (lane >> 4) * 4 + i;
                        if (a < P) {
                            const bool odd = order_of(a) & 1;
                            float val = acc[rt][i];
                            int dst;                      // 0: Re, 1: Im
                            if (!odd) {
                                dst = part;
                            } else {
                                dst = part ^ 1;
                                if (part) val = -val;
                            }
                            if (dc_block && qq == 0 && dst == 0) {
                                // uniform corrections of App. B at k = 0 (times nf^3)
                                const float *dm = dcm + sl * 4;
                                double add = 0.0;
                                if (a == 0) {
                                    double qr2 = 0.0;
                                    for (int z1 = 0; z1 < kZA; ++z1)
                                        qr2 += qr2_partial[(st0 + sl) * kZA + z1];
                                    add = 2.0 * pi / 3.0 * qr2;
                                } else if (PO >= 1 && a == ridx(1, 0)) {
                                    add = 4.0 * pi / 3.0 * (double)dm[1];
                                } else if (PO >= 1 && a == ridx(1, 1)) {
                                    add = 8.0 * pi / 3.0 * (double)dm[2];
                                } else if (PO >= 1 && a == ridx(1, -1)) {
                                    add = -8.0 * pi / 3.0 * (double)dm[3];
                                }
                                val += (float)add;
                            }
                            float *pv = (float *)(xq + sl * P + a);
                            pv[dst] = val;
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (dc_block) {
        for (int sl = tid; sl < stc; sl += 256) qtot[st0 + sl] = (double)dcm[sl * 4];
    }
    // inverse z stage over q, twiddle W_nf^(-z1 r), back to X
    cplx<float> *dst = X + ((int64_t)r * ncol + col) * kZA * SP + (int64_t)st0 * P;
    for (int i = tid; i < stc * P; i += 256) {
        cplx<float> w4[kZA];
#pragma unroll
        for (int qq = 0; qq < kZA; ++qq) w4[qq] = xb[qq * STP + i];
        fft_reg<kZA, true, float>(w4);
#pragma unroll
        for (int z1 = 0; z1 < kZA; ++z1) {
            cplx<float> o = w4[z1];
            if (z1 * r != 0) {
                cplx<float> wt = tw_at(tw_g, z1 * r, nf);
                wt.im = -wt.im;
                o = cmul(o, wt);
            }
            dst[(int64_t)z1 * SP + i] = o;
        }
    }
}

// --------------------------------------------------------------- host side
size_t multi_map_entries(int p) {
    const int P = nreal(p), RT = (P + 15) / 16, KS = (P + 31) / 32;
    return (size_t)RT * KS * 64 * 8;
}

// Code of t_ab (rows a = (l, +-m), columns b = (lam, +-mu)) in the real
// form of eq. realmatrix used by the single-system column kernel: inputs
// pre-multiplied by i^(lam mod 2), outputs post-multiplied by i^(l mod 2),
// s = -1 when l and lam are both odd.
static unsigned t_code(int a, int b, int P) {
    if (a >= P || b >= P) return 0u;
    const int l = order_of(a), ms = a - l * (l + 1);
    const int lam = order_of(b), mus = b - lam * (lam + 1);
    const int nn = l + lam;
    const int s = ((l & 1) && (lam & 1)) ? -1 : 1;
    const bool re_row = ms >= 0;
    const int m = re_row ? ms : -ms;
    Term t1{0, 0}, t2{0, 0};
    int g1 = 0, g2 = 0;
    if (mus == 0) {
        t1 = re_row ? re_S(nn, -m) : im_S(nn, -m);
        g1 = s;
    } else {
        const int mu = mus > 0 ? mus : -mus;
        const int sg = (mu & 1) ? -1 : 1;
        if (mus > 0) {           // Re M_lam^mu column
            t1 = re_row ? re_S(nn, -(m + mu)) : im_S(nn, -(m + mu));
            t2 = re_row ? re_S(nn, -(m - mu)) : im_S(nn, -(m - mu));
            g1 = s;
            g2 = s * sg;
        } else {                 // Im M_lam^mu column
            t1 = re_row ? im_S(nn, -(m + mu)) : re_S(nn, -(m + mu));
            t2 = re_row ? im_S(nn, -(m - mu)) : re_S(nn, -(m - mu));
            g1 = re_row ? -s : s;
            g2 = re_row ? s * sg : -s * sg;
        }
    }
    auto field = [&](Term t, int g) -> unsigned {
        const int sgn = t.sgn * g;
        if (sgn == 0) return 0u;
        return (unsigned)(nn * nn + t.off) | ((sgn > 0 ? 1u : 2u) << 9);
    };
    return field(t1, g1) | (field(t2, g2) << 11);
}

void build_multi_map(int p, unsigned *out) {
    const int P = nreal(p), RT = (P + 15) / 16, KS = (P + 31) / 32;
    for (int rt = 0; rt < RT; ++rt)
        for (int ks = 0; ks < KS; ++ks)
            for (int lane = 0; lane < 64; ++lane)
                for (int e = 0; e < 8; ++e) {
                    const int a = rt * 16 + (lane & 15);
                    const int b = ks * 32 + (lane >> 4) * 8 + e;
                    out[(((size_t)rt * KS + ks) * 64 + lane) * 8 + e] = t_code(a, b, P);
                }
}

template <int PO>
static size_t column_lds_po(int split, int st) {
    return split == 2 ? ColumnMultiShape<PO, 2>::lds(st) : ColumnMultiShape<PO, 3>::lds(st);
}

size_t multi_column_lds(int p, int split, int st) {
    size_t b = 0;
    switch (p) {
        case 0: b = column_lds_po<0>(split, st); break;
        case 1: b = column_lds_po<1>(split, st); break;
        case 2: b = column_lds_po<2>(split, st); break;
        case 3: b = column_lds_po<3>(split, st); break;
        case 4: b = column_lds_po<4>(split, st); break;
        case 5: b = column_lds_po<5>(split, st); break;
        case 6: b = column_lds_po<6>(split, st); break;
        case 7: b = column_lds_po<7>(split, st); break;
        case 8: b = column_lds_po<8>(split, st); break;
        default: return 0;
    }
    return b <= 160 * 1024 ? b : 0;
}

template <typename Kern>
static hipError_t lds_attr(Kern k, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

static int ilog2i(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

constexpr int kMultiCellsPerBlock = 16;

template <int PO>
static hipError_t multi_particles(const MultiArgs &a, int stage, hipStream_t s) {
    const int K = a.n * a.n * a.n;
    const int grid = (K + kMultiCellsPerBlock - 1) / kMultiCellsPerBlock;
    if (stage == 0) {
        hipLaunchKernelGGL((k_p2m_multi<PO>), dim3(grid), dim3(256), 0, s, K,
                           kMultiCellsPerBlock, a.start, (const particle4<float> *)a.sorted,
                           a.perm, a.q, a.ld, a.nsets, a.M, a.zero_count);
    } else {
        if (a.np == 0) return hipSuccess;
        hipLaunchKernelGGL((k_l2p_multi<PO>), dim3(grid), dim3(256), 0, s, K,
                           kMultiCellsPerBlock, a.start, (const particle4<float> *)a.sorted,
                           a.perm, (const float *)a.M, a.nsets, a.qtot, (float)a.alpha_cell,
                           (float)a.inv_h, a.ld, a.phi, a.gx, a.gy, a.gz);
    }
    return hipGetLastError();
}

template <int PO, int NS>
static hipError_t multi_column(const MultiArgs &a, hipStream_t s) {
    const int nf = a.n, logn = ilog2i(nf), nh = nf / 2 + 1, ncol = nf * nh, B = nf / kZA;
    const int ST = a.set_tile;
    const size_t lds = ColumnMultiShape<PO, NS>::lds(ST);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipError_t e = lds_attr(k_column_multi<PO, NS>, lds);
    if (e != hipSuccess) return e;
    const int nst = (a.nsets + ST - 1) / ST;
    const int nblk = B * ncol * nst;
    const int grid = ((nblk + 7) / 8) * 8;
    hipLaunchKernelGGL((k_column_multi<PO, NS>), dim3(grid), dim3(256), lds, s, logn, a.nsets, ST,
                       a.green, (cplx<float> *)a.X, (const cplx<float> *)a.tw, a.tmap,
                       a.qr2_partial, a.qtot);
    return hipGetLastError();
}

template <int PO>
static hipError_t multi_column_po(const MultiArgs &a, hipStream_t s) {
    return a.split == 2 ? multi_column<PO, 2>(a, s) : multi_column<PO, 3>(a, s);
}

template <int B>
static hipError_t multi_slab(const MultiArgs &a, int inverse, hipStream_t s) {
    const int nf = a.n, logn = ilog2i(nf), nh = nf / 2 + 1, P = nreal(a.p);
    const size_t lds = (size_t)(nf / 2 + B * (nf / 2) * lds_line(nf) + nf * B * nh) *
                       sizeof(cplx<float>);
    const int nblk = kZA * a.nsets * P;
    const int grid = ((nblk + 7) / 8) * 8;
    hipError_t e;
    if (!inverse) {
        e = lds_attr(k_slab_fwd<B>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_slab_fwd<B>, dim3(grid), dim3(256), lds, s, logn, a.nsets, P,
                           (const float *)a.M, (cplx<float> *)a.X, (const cplx<float> *)a.tw,
                           a.qr2_partial);
    } else {
        e = lds_attr(k_slab_inv<B>, lds);
        if (e != hipSuccess) return e;
        const float scale = (float)(1.0 / ((double)nf * nf * nf));
        hipLaunchKernelGGL(k_slab_inv<B>, dim3(grid), dim3(256), lds, s, logn, a.nsets, P,
                           (const cplx<float> *)a.X, a.M, (const cplx<float> *)a.tw, scale);
    }
    return hipGetLastError();
}

hipError_t launch_multi_stage(const MultiArgs &a, int stage, hipStream_t s) {
    if (stage == 0 || stage == 4) {
        switch (a.p) {
            case 0: return multi_particles<0>(a, stage, s);
            case 1: return multi_particles<1>(a, stage, s);
            case 2: return multi_particles<2>(a, stage, s);
            case 3: return multi_particles<3>(a, stage, s);
            case 4: return multi_particles<4>(a, stage, s);
            case 5: return multi_particles<5>(a, stage, s);
            case 6: return multi_particles<6>(a, stage, s);
            case 7: return multi_particles<7>(a, stage, s);
            case 8: return multi_particles<8>(a, stage, s);
            default: return hipErrorInvalidValue;
        }
    }
    if (stage == 1 || stage == 3) {
        switch (a.n / kZA) {
            case 1: return multi_slab<1>(a, stage == 3, s);
            case 2: return multi_slab<2>(a, stage == 3, s);
            case 4: return multi_slab<4>(a, stage == 3, s);
            case 8: return multi_slab<8>(a, stage == 3, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (a.p) {
        case 0: return multi_column_po<0>(a, s);
        case 1: return multi_column_po<1>(a, s);
        case 2: return multi_column_po<2>(a, s);
        case 3: return multi_column_po<3>(a, s);
        case 4: return multi_column_po<4>(a, s);
        case 5: return multi_column_po<5>(a, s);
        case 6: return multi_column_po<6>(a, s);
        case 7: return multi_column_po<7>(a, s);
        case 8: return multi_column_po<8>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pmmm
