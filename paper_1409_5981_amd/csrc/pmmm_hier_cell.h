// Fine-level kernel of the two-level hierarchical far field (Sec. 5.2),
// instantiated once per order by pmmm_hier_inst.hip.  The local expansion of
// fine cell I gathers eq. M2L of the moments of every fine cell J whose
// coarse cell is within c of I's and which is itself more than c from I, in
// the real-matrix form of eq. realmatrix with the real values of S at the
// displacement I - J (cell units), read from a table over the margin
// |d_a| <= D = (c + 1) r - 1.  The sum is taken directly, cell pair by cell
// pair (the paper's local FFT convolution computes the same sum).
#pragma once

#include "pmmm_hier.h"

namespace pmmm {
namespace hier_detail {

// Table value of Re S_nn^k / Im S_nn^k (any -nn <= k <= nn, conjugate
// relation) with nn and k known at compile time: a fixed address and sign.
template <int NN, int KK>
__device__ __forceinline__ float re_s_c(const float *g) {
    if constexpr (KK > NN || -KK > NN) return 0.0f;
    else if constexpr (KK >= 0) return g[NN * (NN + 1) + KK];
    else if constexpr (((-KK) & 1) != 0) return -g[NN * (NN + 1) - KK];
    else return g[NN * (NN + 1) - KK];
}
template <int NN, int KK>
__device__ __forceinline__ float im_s_c(const float *g) {
    if constexpr (KK == 0 || KK > NN || -KK > NN) return 0.0f;
    else if constexpr (KK > 0) return g[NN * (NN + 1) - KK];
    else if constexpr (((-KK) & 1) != 0) return g[NN * (NN + 1) + KK];
    else return -g[NN * (NN + 1) + KK];
}

// Output orders of the row groups of the kernel: group g takes the orders
// [hier_cut(PO, g), hier_cut(PO, g + 1)).  Up to order 4 one group holds
// every row; above it [0, 4), [4, 6) and one order per group from 6 on, so
// that a lane's FP64 sums, the moments it holds and the coefficient sums in
// flight stay within the register file (no spills up to order 10).
__host__ __device__ constexpr int hier_ngroups(int po) { return po <= 4 ? 1 : po - 3; }
__host__ __device__ constexpr int hier_cut(int po, int g) {
    return g == 0 ? 0 : g == hier_ngroups(po) ? po + 1 : (g == 1 ? 4 : g == 2 ? 6 : g + 4);
}

// Index of output row (l, m >= 0) in l-major order.
__host__ __device__ constexpr int hier_row(int l, int m) { return l * (l + 1) / 2 + m; }

// A group of `split` lanes per target fine cell and row group: the lanes of
// a group take the cell's source cells in turn, and per source cell the
// moments and the table row are read once and the rows of orders
// [LA, LE) of the (P x P) product of eq. realmatrix are unrolled at compile
// time (order PO).  Per-source sums in FP32, the sums over sources and over
// the group's lanes in FP64.  split is a power of two <= 64 (several lanes
// per cell fill the chip's SIMDs when a fine mesh has few cells for a kernel
// of this register size).
constexpr int kHierCellThreads = 64;
template <int PO, int LA, int LE>
__device__ __forceinline__ void hier_cell_rows(const float *__restrict__ M, float *__restrict__ L,
                                               const float *__restrict__ table, int nf, int r,
                                               int cutoff, int D, int split) {
    constexpr int P = nreal(PO), Q = nreal(2 * PO);
    constexpr int A0 = LA * LA, NA = LE * LE - A0;
    constexpr int NR = hier_row(LE, 0) - hier_row(LA, 0);   // rows (l, m >= 0), LA <= l < LE
    const int64_t K = (int64_t)nf * nf * nf;
    const int part = (int)threadIdx.x & (split - 1);
    const int64_t I = ((int64_t)blockIdx.x * kHierCellThreads + threadIdx.x) / split;
    const bool active = I < K;
    const int W = 2 * D + 1;
    const int64_t Ic = active ? I : 0;
    const int ix = (int)(Ic % nf), iy = (int)((Ic / nf) % nf), iz = (int)(Ic / ((int64_t)nf * nf));
    const int nc = nf / r;
    int lo[3], w[3];
    const int ii[3] = {ix, iy, iz};
    for (int a = 0; a < 3; ++a) {
        const int C = ii[a] / r;
        lo[a] = (C - cutoff > 0 ? C - cutoff : 0) * r;
        w[a] = (C + cutoff < nc - 1 ? C + cutoff : nc - 1) * r + r - lo[a];
    }
    const int count = active ? w[0] * w[1] * w[2] : 0;
    double acc[NA];
    static_for<0, NA>([&](auto ia) { acc[decltype(ia)::value] = 0.0; });
    for (int sidx = part; sidx < count; sidx += split) {
        const int jx = lo[0] + sidx % w[0];
        const int t = sidx / w[0];
        const int jy = lo[1] + t % w[1];
        const int jz = lo[2] + t / w[1];
        const int dx = ix - jx, dy = iy - jy, dz = iz - jz;
        int cheb = abs(dx) > abs(dy) ? abs(dx) : abs(dy);
        cheb = cheb > abs(dz) ? cheb : abs(dz);
        if (cheb <= cutoff) continue;
        const float *g = table + (((int64_t)(dz + D) * W + (dy + D)) * W + (dx + D)) * Q;
        const float *MJ = M + ((int64_t)jz * nf + jy) * nf + jx;
        float mj[P];
        static_for<0, P>([&](auto ia) {
            constexpr int a = decltype(ia)::value;
            mj[a] = MJ[(int64_t)a * K];
        });
        // FP32 sums of this source, one per output row (l, m >= 0); the
        // coefficient sums of a (nn, m, mu) are formed once and serve every
        // split nn = l + lambda
        float sre[NR], sim[NR];
        static_for<0, NR>([&](auto ir) {
            sre[decltype(ir)::value] = 0.0f;
            sim[decltype(ir)::value] = 0.0f;
        });
        static_for<LA, LE + PO>([&](auto inn) {
            constexpr int nn = decltype(inn)::value;
            static_for<0, (nn < LE - 1 ? nn : LE - 1) + 1>([&](auto im) {
                constexpr int m = decltype(im)::value;
                static_for<0, (nn < PO ? nn : PO) + 1>([&](auto imu) {
                    constexpr int mu = decltype(imu)::value;
                    // splits l + lambda = nn with LA <= l < LE, m <= l,
                    // mu <= lambda <= PO
                    constexpr int l_lo0 = nn - PO > LA ? nn - PO : LA;
                    constexpr int l_lo = l_lo0 > m ? l_lo0 : m;
                    constexpr int l_hi0 = nn - mu < LE - 1 ? nn - mu : LE - 1;
                    if constexpr (l_lo <= l_hi0) {
                        if constexpr (mu == 0) {
                            const float a0 = re_s_c<nn, -m>(g);
                            const float b0 = im_s_c<nn, -m>(g);
                            static_for<l_lo, l_hi0 + 1>([&](auto il) {
                                constexpr int l = decltype(il)::value;
                                constexpr int lam = nn - l;
                                constexpr int row = hier_row(l, m) - hier_row(LA, 0);
                                const float M0 = mj[lam * (lam + 1)];
                                sre[row] = __builtin_fmaf(a0, M0, sre[row]);
                                if constexpr (m > 0) sim[row] = __builtin_fmaf(b0, M0, sim[row]);
                            });
                        } else {
                            constexpr float sg = (mu & 1) ? -1.0f : 1.0f;
                            const float A = re_s_c<nn, -(m + mu)>(g);
                            const float B = im_s_c<nn, -(m + mu)>(g);
                            const float C = sg * re_s_c<nn, -(m - mu)>(g);
                            const float Dv = sg * im_s_c<nn, -(m - mu)>(g);
                            const float s1 = A + C, s2 = B - Dv, s3 = B + Dv, s4 = A - C;
                            static_for<l_lo, l_hi0 + 1>([&](auto il) {
                                constexpr int l = decltype(il)::value;
                                constexpr int lam = nn - l;
                                constexpr int row = hier_row(l, m) - hier_row(LA, 0);
                                const float Mr = mj[lam * (lam + 1) + mu];
                                const float Mi = mj[lam * (lam + 1) - mu];
                                // one FMA per multiply-add into the running
                                // sums (a - b inside += would cost a product,
                                // an FMA and an add)
                                sre[row] = __builtin_fmaf(s1, Mr, sre[row]);
                                sre[row] = __builtin_fmaf(-s2, Mi, sre[row]);
                                if constexpr (m > 0) {
                                    sim[row] = __builtin_fmaf(s3, Mr, sim[row]);
                                    sim[row] = __builtin_fmaf(s4, Mi, sim[row]);
                                }
                            });
                        }
                    }
                });
            });
        });
        static_for<LA, LE>([&](auto il) {
            constexpr int l = decltype(il)::value;
            static_for<0, l + 1>([&](auto im) {
                constexpr int m = decltype(im)::value;
                constexpr int row = hier_row(l, m) - hier_row(LA, 0);
                acc[l * (l + 1) + m - A0] += (double)sre[row];
                if constexpr (m > 0) acc[l * (l + 1) - m - A0] += (double)sim[row];
            });
        });
    }
    for (int off = 1; off < split; off <<= 1)
        static_for<0, NA>([&](auto ia) {
            constexpr int a = decltype(ia)::value;
            acc[a] += __shfl_xor(acc[a], off, kHierCellThreads);
        });
    if (!active || part != 0) return;
    static_for<0, NA>([&](auto ia) {
        constexpr int a = decltype(ia)::value;
        L[(int64_t)(A0 + a) * K + I] = (float)acc[a];
    });
}

// blockIdx.y selects the row group.
template <int PO>
__global__ __launch_bounds__(kHierCellThreads) void k_hier_m2l_cell(
    const float *__restrict__ M, float *__restrict__ L, const float *__restrict__ table, int nf,
    int r, int cutoff, int D, int split) {
    static_for<0, hier_ngroups(PO)>([&](auto ig) {
        constexpr int gi = decltype(ig)::value;
        if (blockIdx.y == gi)
            hier_cell_rows<PO, hier_cut(PO, gi), hier_cut(PO, gi + 1)>(M, L, table, nf, r, cutoff,
                                                                        D, split);
    });
}

}  // namespace hier_detail

// Launch of the kernel for order PO (one compile unit per order).
template <int PO>
hipError_t hier_cell_launch(const HierArgs &a, hipStream_t s) {
    const int64_t K = (int64_t)a.nf * a.nf * a.nf;
    constexpr int NG = hier_detail::hier_ngroups(PO);
    // Lanes per cell and row group: enough waves for four per SIMD
    // (256 CUs x 4 SIMDs), at most 8.
    int split = 1;
    while (split < 8 && K * NG * split < (int64_t)4 * 1024 * hier_detail::kHierCellThreads) split <<= 1;
    const int64_t nthr = K * split;
    hipLaunchKernelGGL(hier_detail::k_hier_m2l_cell<PO>,
                       dim3((unsigned)((nthr + hier_detail::kHierCellThreads - 1) / hier_detail::kHierCellThreads), NG),
                       dim3(hier_detail::kHierCellThreads), 0, s, a.M, a.L, a.table, a.nf, a.r, a.cutoff, a.D,
                       split);
    return hipGetLastError();
}

}  // namespace pmmm
