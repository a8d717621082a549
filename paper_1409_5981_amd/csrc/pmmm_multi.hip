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
// Meshes are point-major with the set index fastest (component b of set s at
// point x is element [x][b S + s]): the particle kernels give each set one
// lane, the FFT kernels take tiles of consecutive components, and all their
// global accesses are contiguous runs.
//   k_p2m_multi     one wave per cell, one lane per set: eq. P2M with the
//                   harmonics R(r_M - r_i) of the cell's particles staged in
//                   LDS and read by every lane.
//   k_xy_fwd        one z-plane and 16 components: real FFT along x (two
//                   rows per complex transform) and FFT along y, in
//                   registers, through one LDS transpose.
//   k_z_fft         FFT along z (forward or inverse), one thread per
//                   (column, component) line, in registers.
//   k_m2l_gemm      one frequency: t (eq. realmatrix) built once in MFMA
//                   fragments and applied to all sets at once.
//   k_xy_inv        inverse of k_xy_fwd, scaled by 1/nf^3.
//   k_l2p_multi     one wave per cell, one lane per set: eq. L2P and the
//                   order-one eq. L2L of eq. phigrad, with the cell's local
//                   expansion folded into per-set coefficient vectors.
#include "pmmm_internal.h"

namespace pmmm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4v __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

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

// Order of real component a (a < 2^20) without a loop: sqrt(a + 1/2) lies
// strictly between l and l + 1.
__device__ __forceinline__ int order_fast(int a) { return (int)__builtin_sqrtf((float)a + 0.5f); }

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
            for (int a = 0; a <= P; ++a) M[((int64_t)c * (P + 1) + a) * S + lane] = acc[a];
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
            for (int a = 0; a < P; ++a) Lc[a] = L[((int64_t)c * P + a) * S + lane];
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

// ------------------------------------------------------- x-y plane FFTs
// Block -> (z-plane, component tile) with the tile fastest; each XCD (blocks
// are dealt round-robin over the 8 XCDs) takes a contiguous range, so
// neighbouring tiles, which share cache lines, run on one XCD.
__device__ __forceinline__ int xcd_block(int nblk) {
    const int per_xcd = (nblk + 7) / 8;
    return (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
}

template <int NF>
__global__ void __launch_bounds__(256) k_xy_fwd(int S, int P, const float *__restrict__ M,
                                                cplx<float> *__restrict__ Y,
                                                double *__restrict__ qr2_partial) {
    constexpr int NH = NF / 2 + 1, CT = kMultiCompTile, NPAIR = NF / 2;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    cplx<float> *Z = (cplx<float> *)lds_raw;          // [NF y][NH kx][CT]
    const int SP = S * P, SP1 = S * (P + 1), sps = (SP + 1) & ~1;
    const int ntile = (SP + CT - 1) / CT;
    const int v = xcd_block(NF * ntile);
    if (v >= NF * ntile) return;
    const int z = v / ntile, tile = v - z * ntile;
    const int c0 = tile * CT;
    const int tid = threadIdx.x;
    const float *plane = M + (int64_t)z * NF * NF * SP1;
    // x transforms: rows 2jj and 2jj+1 as the real and imaginary parts
    for (int item = tid; item < NPAIR * CT; item += 256) {
        const int jj = item / CT, ct = item - jj * CT, c = c0 + ct;
        const bool ok = c < SP;
        cplx<float> w[NF];
#pragma unroll
        for (int x = 0; x < NF; ++x) {
            w[x].re = ok ? plane[((int64_t)(2 * jj) * NF + x) * SP1 + c] : 0.f;
            w[x].im = ok ? plane[((int64_t)(2 * jj + 1) * NF + x) * SP1 + c] : 0.f;
        }
        fft_reg<NF, false, float>(w);
#pragma unroll
        for (int k = 0; k < NH; ++k) {
            const cplx<float> zk = w[k], zm = w[(NF - k) & (NF - 1)];
            Z[((2 * jj) * NH + k) * CT + ct] = {0.5f * (zk.re + zm.re), 0.5f * (zk.im - zm.im)};
            Z[((2 * jj + 1) * NH + k) * CT + ct] = {0.5f * (zk.im + zm.im), -0.5f * (zk.re - zm.re)};
        }
    }
    __syncthreads();
    // y transforms, written straight to the spectra
    for (int item = tid; item < NH * CT; item += 256) {
        const int kx = item / CT, ct = item - kx * CT, c = c0 + ct;
        cplx<float> w[NF];
#pragma unroll
        for (int y = 0; y < NF; ++y) w[y] = Z[(y * NH + kx) * CT + ct];
        fft_reg<NF, false, float>(w);
        if (c < SP) {
#pragma unroll
            for (int ky = 0; ky < NF; ++ky) Y[((int64_t)(z * NF + ky) * NH + kx) * sps + c] = w[ky];
        }
    }
    if (c0 < S) {
        // sum over this plane of q|u|^2 (component P) for the sets [c0, c0 + CT),
        // fixed-order reduction
        constexpr int PARTS = 256 / CT;
        __syncthreads();
        double *red = (double *)lds_raw;
        const int ct = tid % CT, part = tid / CT, s = c0 + ct;
        double acc = 0.0;
        if (s < S)
            for (int cell = part; cell < NF * NF; cell += PARTS)
                acc += (double)plane[(int64_t)cell * SP1 + SP + s];
        red[part * CT + ct] = acc;
        __syncthreads();
        if (tid < CT && c0 + tid < S) {
            double t = 0.0;
            for (int pp = 0; pp < PARTS; ++pp) t += red[pp * CT + tid];
            qr2_partial[(int64_t)z * S + c0 + tid] = t;
        }
    }
}

template <int NF>
__global__ void __launch_bounds__(256) k_xy_inv(int S, int P, const cplx<float> *__restrict__ Y,
                                                float *__restrict__ L, float scale) {
    constexpr int NH = NF / 2 + 1, CT = kMultiCompTile, NPAIR = NF / 2;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    cplx<float> *Z = (cplx<float> *)lds_raw;          // [NF y][NH kx][CT]
    const int SP = S * P, sps = (SP + 1) & ~1;
    const int ntile = (SP + CT - 1) / CT;
    const int v = xcd_block(NF * ntile);
    if (v >= NF * ntile) return;
    const int z = v / ntile, tile = v - z * ntile;
    const int c0 = tile * CT;
    const int tid = threadIdx.x;
    for (int item = tid; item < NH * CT; item += 256) {
        const int kx = item / CT, ct = item - kx * CT, c = c0 + ct;
        const bool ok = c < SP;
        cplx<float> w[NF];
#pragma unroll
        for (int ky = 0; ky < NF; ++ky)
            w[ky] = ok ? Y[((int64_t)(z * NF + ky) * NH + kx) * sps + c] : cplx<float>{0.f, 0.f};
        fft_reg<NF, true, float>(w);
#pragma unroll
        for (int y = 0; y < NF; ++y) Z[(y * NH + kx) * CT + ct] = w[y];
    }
    __syncthreads();
    // C2R along x: rows 2jj and 2jj+1 packed into one complex transform
    for (int item = tid; item < NPAIR * CT; item += 256) {
        const int jj = item / CT, ct = item - jj * CT, c = c0 + ct;
        cplx<float> w[NF];
#pragma unroll
        for (int k = 0; k < NF; ++k) {
            const int kk = k <= NF / 2 ? k : NF - k;
            cplx<float> A = Z[((2 * jj) * NH + kk) * CT + ct];
            cplx<float> B = Z[((2 * jj + 1) * NH + kk) * CT + ct];
            if (k > NF / 2) {
                A.im = -A.im;
                B.im = -B.im;
            }
            w[k] = {A.re - B.im, A.im + B.re};
        }
        fft_reg<NF, true, float>(w);
        if (c < SP) {
            float *r0 = L + ((int64_t)(z * NF + 2 * jj) * NF) * SP + c;
#pragma unroll
            for (int x = 0; x < NF; ++x) {
                r0[(int64_t)x * SP] = w[x].re * scale;
                r0[(int64_t)(NF + x) * SP] = w[x].im * scale;
            }
        }
    }
}

// ----------------------------------------------------------- column GEMM
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Two values at once: h[i] holds term i of both (one packed conversion per
// term).
template <int NS>
__device__ __forceinline__ void split_pair(float a, float b, bf16x2 (&h)[NS]) {
    f32x2 v = {a, b};
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        h[i] = __builtin_convertvector(v, bf16x2);
        if (i + 1 < NS) v = v - __builtin_convertvector(h[i], f32x2);
    }
}

// Eight values (in pairs) into the NS bf16x8 fragments of their terms.
template <int NS>
__device__ __forceinline__ void split8(const float (&v)[8], bf16x8 (&fr)[NS]) {
    bf16x2 h[4][NS];
#pragma unroll
    for (int q = 0; q < 4; ++q) split_pair<NS>(v[2 * q], v[2 * q + 1], h[q]);
#pragma unroll
    for (int sp = 0; sp < NS; ++sp) {
        const bf16x4v lo = __builtin_shufflevector(h[0][sp], h[1][sp], 0, 1, 2, 3);
        const bf16x4v hi = __builtin_shufflevector(h[2][sp], h[3][sp], 0, 1, 2, 3);
        fr[sp] = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
    }
}

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

// z transforms of the spectra, in place: one thread per (column, component)
// line, in registers; consecutive threads hold consecutive components.  The
// forward transform leaves component b multiplied by i^(lam mod 2) (lam the
// order of b), the form the M2L product takes.
template <int NF, bool INV>
__global__ void __launch_bounds__(256) k_z_fft(int SP, int S, cplx<float> *__restrict__ Y) {
    constexpr int NH = NF / 2 + 1, NCOL = NF * NH;
    const int nchunk = (SP + 255) / 256;
    const int v = xcd_block(NCOL * nchunk);
    if (v >= NCOL * nchunk) return;
    const int col = v / nchunk, chunk = v - col * nchunk;
    const int c = chunk * 256 + threadIdx.x;
    if (c >= SP) return;
    const int sps = (SP + 1) & ~1;
    cplx<float> *base = Y + (int64_t)col * sps + c;
    const int64_t zs = (int64_t)NCOL * sps;
    cplx<float> w[NF];
#pragma unroll
    for (int z = 0; z < NF; ++z) w[z] = base[z * zs];
    fft_reg<NF, INV, float>(w);
    if (!INV && (order_fast(c / S) & 1)) {
        // forward: pre-multiply component b = c / S by i^(lam mod 2) for the
        // real form of the M2L product
#pragma unroll
        for (int z = 0; z < NF; ++z) w[z] = {-w[z].im, w[z].re};
    }
#pragma unroll
    for (int z = 0; z < NF; ++z) base[z * zs] = w[z];
}

template <int PO, int NS>
struct GemmShape {
    static constexpr int P = nreal(PO), Q = nreal(2 * PO);
    static constexpr int RT = (P + 15) / 16, KS = (P + 31) / 32;
    static constexpr int NT = (2 * kMultiMaxSets) / 16;           // column tiles at most
    // spectra / results in LDS: component rows of 2S + 1 floats (the odd
    // stride puts rows 8 apart in different banks)
    static constexpr size_t raw_bytes = (size_t)P * (2 * kMultiMaxSets + 1) * 4;
    static constexpr size_t abuf_bytes = (size_t)NS * RT * KS * 64 * 16;
    static constexpr size_t raw_al = (raw_bytes + 15) / 16 * 16;
    static constexpr size_t lds = raw_al + abuf_bytes + ((size_t)Q * 4 + 15) / 16 * 16 +
                                  (size_t)kMultiMaxSets * 16;
};

constexpr int kGemmThreads = 512;

// One frequency per block (512 threads): L~_a = i^(l mod 2) sum_b t_ab
// i^(lam mod 2) M~_b for every set at once, as the real product of t (rows
// a, columns b) and the (P x 2S) matrix of the sets' real and imaginary
// parts.  The frequency's P S spectra (contiguous) come in with one batch of
// 16-byte loads into LDS; the waves build the A fragments of t together;
// wave w then owns column tile w (8 sets): it splits its own B fragments
// from LDS, multiplies every row tile, and writes the results over its own
// columns, which no other wave reads.  The results leave with 16-byte
// stores.  (The spectra of the frequency are read into LDS before any
// result is written back to the same place.)
template <int PO, int NS>
__global__ void __launch_bounds__(kGemmThreads, PO >= 8 ? 2 : 6) k_m2l_gemm(int logn, int S,
                                                           const float *__restrict__ green,
                                                           cplx<float> *__restrict__ Y,
                                                           const unsigned *__restrict__ tmap,
                                                           const double *__restrict__ qr2_partial,
                                                           double *__restrict__ qtot) {
    using Sh = GemmShape<PO, NS>;
    constexpr int P = Sh::P, Q = Sh::Q, RT = Sh::RT, KS = Sh::KS, NTM = Sh::NT;
    constexpr int NTH = kGemmThreads, NW = NTH / 64;
    constexpr int AITEMS = RT * KS * 64, AIT = (AITEMS + NTH - 1) / NTH;
    constexpr int MAXV4 = (P * kMultiMaxSets / 2 + NTH - 1) / NTH;   // float4 loads per thread
    extern __shared__ __align__(16) unsigned char lds_raw[];
    float *rawf = (float *)lds_raw;                                    // [P][2S+1]
    bf16x8 *abuf = (bf16x8 *)(lds_raw + Sh::raw_al);                   // [NS][RT][KS][64]
    float *gq = (float *)(lds_raw + Sh::raw_al + Sh::abuf_bytes);      // [Q]
    float *dcm = gq + (Q + 3) / 4 * 4;                                 // [64][4]
    const int nf = 1 << logn, nh = nf / 2 + 1, nhp = (nh + 3) & ~3, ncol = nf * nh;
    const int SP = S * P, rsf = 2 * S + 1;
    const int NT = (2 * S + 15) / 16;
    const int nfreq = nf * ncol;
    const int f = xcd_block(nfreq);
    if (f >= nfreq) return;
    const int kz = f / ncol, col = f - kz * ncol;
    const int ky = col / nh, kx = col - ky * nh;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const bool dc = f == 0;
    // frequency slices are padded to an even number of complex values, so
    // each starts 16-byte aligned
    const int sps = (SP + 1) & ~1;
    cplx<float> *Yf = Y + (int64_t)f * sps;
    // every global load of the block goes out first: the spectra, this
    // thread's t-map codes and the kernel values
    const int nv4 = sps / 2;                      // float4 = two complex values
    f32x4 rv[MAXV4];
#pragma unroll
    for (int u = 0; u < MAXV4; ++u) rv[u] = ((const f32x4 *)Yf)[min(tid + u * NTH, nv4 - 1)];
    uint4 cd[AIT][2];
#pragma unroll
    for (int it = 0; it < AIT; ++it) {
        const int item = min(tid + it * NTH, AITEMS - 1);
        cd[it][0] = ((const uint4 *)tmap)[item * 2];
        cd[it][1] = ((const uint4 *)tmap)[item * 2 + 1];
    }
    constexpr int GIT = (Q + NTH - 1) / NTH;
    float gv[GIT];
    {
        const int kyr = ky <= nf / 2 ? ky : nf - ky;
        const int kzr = kz <= nf / 2 ? kz : nf - kz;
        const float *gcol = green + (int64_t)(kyr * nh + kx) * Q * nhp;
#pragma unroll
        for (int it = 0; it < GIT; ++it) gv[it] = gcol[min(tid + it * NTH, Q - 1) * nhp + kzr];
    }
    // keep the loads in flight together: the empty statements below need
    // every value here, so no load is sunk next to its LDS store
#pragma unroll
    for (int u = 0; u < MAXV4; ++u) asm volatile("" : "+v"(rv[u]));
#pragma unroll
    for (int it = 0; it < GIT; ++it) asm volatile("" : "+v"(gv[it]));
#pragma unroll
    for (int it = 0; it < GIT; ++it) {
        const int j = tid + it * NTH;
        if (j < Q) {
            const int nn = order_fast(j), kk = j - nn * nn - nn;
            const int ak = kk < 0 ? -kk : kk;
            // mirrors: ky > nf/2 negates the Im-part components, kz > nf/2
            // multiplies (n, k) by (-1)^(n+|k|)
            const bool neg = ((ky > nf / 2) && kk < 0) != ((kz > nf / 2) && ((nn + ak) & 1));
            gq[j] = neg ? -gv[it] : gv[it];
        }
    }
    // spectra into padded rows: complex 2i and 2i+1 of the slice
#pragma unroll
    for (int u = 0; u < MAXV4; ++u) {
        const int i = tid + u * NTH;
        if (i < nv4) {
            const int c0 = 2 * i, k0 = c0 / S, s0 = c0 - k0 * S;
            const int c1 = c0 + 1, k1 = s0 + 1 < S ? k0 : k0 + 1, s1 = s0 + 1 < S ? s0 + 1 : 0;
            rawf[k0 * rsf + 2 * s0] = rv[u][0];
            rawf[k0 * rsf + 2 * s0 + 1] = rv[u][1];
            if (c1 < SP) {
                rawf[k1 * rsf + 2 * s1] = rv[u][2];
                rawf[k1 * rsf + 2 * s1 + 1] = rv[u][3];
            }
        }
    }
    __syncthreads();
    if (dc) {
        // zero frequency: M~_b(0) = sum over cells of M_b (real); the order-one
        // components arrive multiplied by i, so their value is the Im part
        for (int s = tid; s < S; s += NTH) {
            dcm[s * 4 + 0] = rawf[2 * s];
            dcm[s * 4 + 1] = PO >= 1 ? rawf[ridx(1, 0) * rsf + 2 * s + 1] : 0.f;
            dcm[s * 4 + 2] = PO >= 1 ? rawf[ridx(1, 1) * rsf + 2 * s + 1] : 0.f;
            dcm[s * 4 + 3] = PO >= 1 ? rawf[ridx(1, -1) * rsf + 2 * s + 1] : 0.f;
        }
    }
    // A fragments of t at this frequency
#pragma unroll
    for (int it = 0; it < AIT; ++it) {
        const int item = tid + it * NTH;
        if (item < AITEMS) {
            const unsigned codes[8] = {cd[it][0].x, cd[it][0].y, cd[it][0].z, cd[it][0].w,
                                       cd[it][1].x, cd[it][1].y, cd[it][1].z, cd[it][1].w};
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = decode_term(gq, codes[e]);
            bf16x8 fr[NS];
            split8<NS>(v, fr);
#pragma unroll
            for (int sp = 0; sp < NS; ++sp) abuf[sp * AITEMS + item] = fr[sp];
        }
    }
    __syncthreads();
    if (dc) {
        for (int s = tid; s < S; s += NTH) qtot[s] = (double)dcm[s * 4];
    }
    // wave w: column tile nt = w (columns n = 16 nt + lane % 16 = 2 s + part);
    // B fragments (the spectra arrive pre-multiplied by i^(lam mod 2)): rows
    // k = ks 32 + (lane/16) 8 + e
    const int n0 = lane & 15, part = n0 & 1;
    for (int nt = wv; nt < NT; nt += NW) {
        const int s = nt * 8 + (n0 >> 1);
        const bool sok = s < S;
        const float *rp = rawf + 2 * min(s, S - 1) + part;
        bf16x8 bfr[KS][NS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = ks * 32 + (lane >> 4) * 8 + e;
                const float x = rp[min(k, P - 1) * rsf];
                v[e] = (sok && k < P) ? x : 0.f;
            }
            split8<NS>(v, bfr[ks]);
        }
        f32x4 acc[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            acc[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                bf16x8 afr[NS];
#pragma unroll
                for (int sp = 0; sp < NS; ++sp) afr[sp] = abuf[(sp * RT + rt) * KS * 64 + ks * 64 + lane];
                // smallest products first
#pragma unroll
                for (int d = NS - 1; d >= 0; --d) {
#pragma unroll
                    for (int i = d; i >= 0; --i)
                        acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[i], bfr[ks][d - i],
                                                                       acc[rt], 0, 0, 0);
                }
            }
        }
        // D rows a = rt 16 + (lane/16) 4 + i over this wave's own columns
        if (sok) {
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int a = rt * 16 + (lane >> 4) * 4 + i;
                    if (a >= P) continue;
                    float val = acc[rt][i];
                    int dst = part;                      // 0: Re, 1: Im
                    if (order_fast(a) & 1) {
                        dst = part ^ 1;
                        if (part) val = -val;
                    }
                    rawf[a * rsf + 2 * s + dst] = val;
                }
            }
        }
    }
    __syncthreads();
    if (dc) {
        // uniform corrections of App. B at k = 0 (times nf^3)
        const double pi = 3.14159265358979323846;
        for (int s = tid; s < S; s += NTH) {
            double qr2 = 0.0;
            for (int z = 0; z < nf; ++z) qr2 += qr2_partial[(int64_t)z * S + s];
            rawf[2 * s] += (float)(2.0 * pi / 3.0 * qr2);
            if (PO >= 1) {
                rawf[ridx(1, 0) * rsf + 2 * s] += (float)(4.0 * pi / 3.0 * (double)dcm[s * 4 + 1]);
                rawf[ridx(1, 1) * rsf + 2 * s] += (float)(8.0 * pi / 3.0 * (double)dcm[s * 4 + 2]);
                rawf[ridx(1, -1) * rsf + 2 * s] += (float)(-8.0 * pi / 3.0 * (double)dcm[s * 4 + 3]);
            }
        }
        __syncthreads();
    }
    // results out, complex 2i and 2i+1 per 16-byte store
#pragma unroll
    for (int u = 0; u < MAXV4; ++u) {
        const int i = tid + u * NTH;
        if (i < nv4) {
            const int c0 = 2 * i, k0 = c0 / S, s0 = c0 - k0 * S;
            const int c1 = c0 + 1, k1 = s0 + 1 < S ? k0 : k0 + 1, s1 = s0 + 1 < S ? s0 + 1 : 0;
            f32x4 o;
            o[0] = rawf[k0 * rsf + 2 * s0];
            o[1] = rawf[k0 * rsf + 2 * s0 + 1];
            o[2] = c1 < SP ? rawf[k1 * rsf + 2 * s1] : 0.f;
            o[3] = c1 < SP ? rawf[k1 * rsf + 2 * s1 + 1] : 0.f;
            ((f32x4 *)Yf)[i] = o;
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

bool multi_supported(int p, int nf) {
    if (nf != 4 && nf != 8 && nf != 16 && nf != 32) return false;
    return p >= 0 && p <= kMultiPMax;
}

template <typename Kern>
static hipError_t lds_attr(Kern k, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return set_max_lds((const void *)k, bytes);
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
    const int nf = a.n, logn = ilog2i(nf), ncol = nf * (nf / 2 + 1);
    const size_t lds = GemmShape<PO, NS>::lds;
    hipError_t e = lds_attr(k_m2l_gemm<PO, NS>, lds);
    if (e != hipSuccess) return e;
    const int nblk = nf * ncol;
    const int grid = ((nblk + 7) / 8) * 8;
    hipLaunchKernelGGL((k_m2l_gemm<PO, NS>), dim3(grid), dim3(kGemmThreads), lds, s, logn, a.nsets,
                       a.green, (cplx<float> *)a.Y, a.tmap, a.qr2_partial, a.qtot);
    return hipGetLastError();
}

template <int PO>
static hipError_t multi_column_po(const MultiArgs &a, hipStream_t s) {
    return a.split == 2 ? multi_column<PO, 2>(a, s) : multi_column<PO, 3>(a, s);
}

template <int NF>
static hipError_t multi_planes(const MultiArgs &a, int inverse, hipStream_t s) {
    const int P = nreal(a.p), SP = a.nsets * P;
    // spectra tile, also the 256-double reduction buffer of the forward kernel
    size_t lds = (size_t)NF * (NF / 2 + 1) * kMultiCompTile * sizeof(cplx<float>);
    if (lds < 256 * sizeof(double)) lds = 256 * sizeof(double);
    const int ntile = (SP + kMultiCompTile - 1) / kMultiCompTile;
    const int nblk = NF * ntile;
    const int grid = ((nblk + 7) / 8) * 8;
    const int zblk = NF * (NF / 2 + 1) * ((SP + 255) / 256);
    const int zgrid = ((zblk + 7) / 8) * 8;
    hipError_t e;
    if (!inverse) {
        e = lds_attr(k_xy_fwd<NF>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_xy_fwd<NF>, dim3(grid), dim3(256), lds, s, a.nsets, P,
                           (const float *)a.M, (cplx<float> *)a.Y, a.qr2_partial);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_z_fft<NF, false>), dim3(zgrid), dim3(256), 0, s, SP, a.nsets,
                           (cplx<float> *)a.Y);
    } else {
        hipLaunchKernelGGL((k_z_fft<NF, true>), dim3(zgrid), dim3(256), 0, s, SP, a.nsets,
                           (cplx<float> *)a.Y);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = lds_attr(k_xy_inv<NF>, lds);
        if (e != hipSuccess) return e;
        const float scale = (float)(1.0 / ((double)NF * NF * NF));
        hipLaunchKernelGGL(k_xy_inv<NF>, dim3(grid), dim3(256), lds, s, a.nsets, P,
                           (const cplx<float> *)a.Y, a.M, scale);
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
        switch (a.n) {
            case 4: return multi_planes<4>(a, stage == 3, s);
            case 8: return multi_planes<8>(a, stage == 3, s);
            case 16: return multi_planes<16>(a, stage == 3, s);
            case 32: return multi_planes<32>(a, stage == 3, s);
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
