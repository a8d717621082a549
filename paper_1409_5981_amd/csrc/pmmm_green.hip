// Plan-time transfer kernel G~ in FP64 on the GPU (Sec. 2.1: (2p+1)^2
// transforms performed once and saved), in cell units (h = 1).
//   k_green_open      App. C layout on the (2n)^3 mesh: index d -> offset d
//                     (d < n) or d - 2n (d > n); zero on the index-n planes
//                     and on the near cube max|offset| <= c; S_k^j(offset)
//                     elsewhere, for orders k <= 2p.
//   k_green_recip     reciprocal-space terms of eq. greenPBC for every lattice
//                     vector 0 < |n| <= images (shared by all mesh points)
//   k_green_periodic  eq. greenPBC at each minimum-image offset: incomplete-
//                     gamma weighted real-space image sum plus the reciprocal
//                     sum; at offset 0 the singular n = 0 real-space term is
//                     left out; for 0 < max|offset| <= c the image covered by
//                     the near field, S(offset), is subtracted (App. B), as
//                     -P(l + 1/2, alpha^2 r^2) S in place of Q S - S.
//   k_line_fft        FP64 complex FFT of mesh lines (LDS, radix 2)
//   k_fold            keeps Re G~ (even order) or Im G~ (odd order) on the
//                     quadrant ky, kz <= nf/2, rounded to the plan precision
// Singular harmonics use the order recursion (derived from App. A.5 with
// S_l^m = (-1)^(l+m) (l-m)! Q_l^m / r^(2l+1)):
//   S_m^m = -(2m-1) (x+iy)/r^2 S_{m-1}^{m-1},  S_{m+1}^m = -(2m+1) z/r^2 S_m^m,
//   S_l^m = -((2l-1) z S_{l-1}^m + (l+m-1)(l-m-1) S_{l-2}^m) / r^2.
#include <vector>
#include <cmath>

#include "pmmm_hier.h"

namespace pmmm {

constexpr int kMaxL = 2 * PMMM_PMAX;
constexpr int kMaxTri = (kMaxL + 1) * (kMaxL + 2) / 2;

__device__ __forceinline__ int tri_idx(int l, int m) { return l * (l + 1) / 2 + m; }

// S_l^m (m >= 0) as complex numbers at tri_idx(l, m).
__device__ void singular_tri(int lmax, double x, double y, double z, double *sre, double *sim) {
    const double r2 = x * x + y * y + z * z;
    const double ir2 = 1.0 / r2;
    double cre = 1.0 / sqrt(r2), cim = 0.0;  // S_m^m
    for (int m = 0; m <= lmax; ++m) {
        if (m > 0) {
            const double f = -(2.0 * m - 1.0) * ir2;
            const double nre = f * (x * cre - y * cim);
            const double nim = f * (x * cim + y * cre);
            cre = nre;
            cim = nim;
        }
        sre[tri_idx(m, m)] = cre;
        sim[tri_idx(m, m)] = cim;
        double pre = cre, pim = cim, ure = 0.0, uim = 0.0;
        if (m + 1 <= lmax) {
            const double f = -(2.0 * m + 1.0) * z * ir2;
            ure = f * cre;
            uim = f * cim;
            sre[tri_idx(m + 1, m)] = ure;
            sim[tri_idx(m + 1, m)] = uim;
        }
        for (int l = m + 2; l <= lmax; ++l) {
            const double a = (2.0 * l - 1.0) * z, b = (double)(l + m - 1) * (double)(l - m - 1);
            const double nre = -(a * ure + b * pre) * ir2;
            const double nim = -(a * uim + b * pim) * ir2;
            sre[tri_idx(l, m)] = nre;
            sim[tri_idx(l, m)] = nim;
            pre = ure;
            pim = uim;
            ure = nre;
            uim = nim;
        }
    }
}

__global__ void k_green_open(int n, int nf, int lmax, int cutoff, double *__restrict__ G) {
    const int64_t npts = (int64_t)nf * nf * nf;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= npts) return;
    const int ix = (int)(idx % nf), iy = (int)((idx / nf) % nf), iz = (int)(idx / ((int64_t)nf * nf));
    const int Q = (lmax + 1) * (lmax + 1);
    const int dx = ix < n ? ix : ix - nf, dy = iy < n ? iy : iy - nf, dz = iz < n ? iz : iz - nf;
    int cheb = abs(dx) > abs(dy) ? abs(dx) : abs(dy);
    cheb = cheb > abs(dz) ? cheb : abs(dz);
    const bool zero = ix == n || iy == n || iz == n || cheb <= cutoff;
    if (zero) {
        for (int j = 0; j < Q; ++j) G[(int64_t)j * npts + idx] = 0.0;
        return;
    }
    double sre[kMaxTri], sim[kMaxTri];
    singular_tri(lmax, (double)dx, (double)dy, (double)dz, sre, sim);
    for (int l = 0; l <= lmax; ++l) {
        G[(int64_t)(l * (l + 1)) * npts + idx] = sre[tri_idx(l, 0)];
        for (int m = 1; m <= l; ++m) {
            G[(int64_t)(l * (l + 1) + m) * npts + idx] = sre[tri_idx(l, m)];
            G[(int64_t)(l * (l + 1) - m) * npts + idx] = sim[tri_idx(l, m)];
        }
    }
}

// Reciprocal terms: coef_l(k) S_l^m(k) with
// coef_l = (-i pi)^l / sqrt(pi) exp(-(pi |k| / alpha)^2) / Gamma(l + 1/2) |k|^(2l-1) / V,
// k = nvec / b, for every listed lattice vector.  table[t][tri] = (re, im).
__global__ void k_green_recip(int nk, const int *__restrict__ kvec, double box, double alpha,
                              int lmax, double *__restrict__ table) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nk) return;
    const int ntri = (lmax + 1) * (lmax + 2) / 2;
    const double kx = kvec[3 * t] / box, ky = kvec[3 * t + 1] / box, kz = kvec[3 * t + 2] / box;
    const double kk = sqrt(kx * kx + ky * ky + kz * kz);
    const double pi = 3.14159265358979323846;
    double sre[kMaxTri], sim[kMaxTri];
    singular_tri(lmax, kx, ky, kz, sre, sim);
    const double V = box * box * box;
    const double e = exp(-(pi * kk / alpha) * (pi * kk / alpha));
    double gam = sqrt(pi);      // Gamma(l + 1/2)
    double kp = 1.0 / kk;       // |k|^(2l-1)
    double pil = 1.0;           // pi^l
    for (int l = 0; l <= lmax; ++l) {
        const double c = pil / sqrt(pi) * e / gam * kp / V;
        // (-i)^l
        const int ph = l & 3;
        const double cr = ph == 0 ? c : (ph == 2 ? -c : 0.0);
        const double ci = ph == 1 ? -c : (ph == 3 ? c : 0.0);
        for (int m = 0; m <= l; ++m) {
            const int u = tri_idx(l, m);
            table[((int64_t)t * ntri + u) * 2] = cr * sre[u] - ci * sim[u];
            table[((int64_t)t * ntri + u) * 2 + 1] = cr * sim[u] + ci * sre[u];
        }
        pil *= pi;
        gam *= (l + 0.5);
        kp *= kk * kk;
    }
}

// Regularised incomplete gammas of half-integer order for l = 0..lmax at x:
// upper Q(l + 1/2, x) by Q(1/2, x) = erfc(sqrt x), Q(a + 1) = Q(a) +
// x^a e^-x / Gamma(a + 1); with `lower`, minus the lower one, -P(l + 1/2, x),
// by its power series x^a e^-x sum_k x^k / Gamma(a + k + 1) where x < a + 1
// (no cancellation where P is small) and as Q - 1 above.
__device__ void inc_gamma_half_dev(int lmax, double x, bool lower, double *out) {
    const double pi = 3.14159265358979323846;
    const double sx = sqrt(x), ex = exp(-x);
    out[0] = erfc(sx);
    {
        double xa = sx, g1 = 0.5 * sqrt(pi);  // x^(1/2), Gamma(3/2)
        for (int l = 0; l < lmax; ++l) {
            out[l + 1] = out[l] + xa * ex / g1;
            xa *= x;
            g1 *= (l + 1.5);
        }
    }
    if (!lower) return;
    double xa = sx, g1 = 0.5 * sqrt(pi);      // x^a, Gamma(a + 1) for a = 1/2
    for (int l = 0; l <= lmax; ++l) {
        const double a = l + 0.5;
        if (x < a + 1.0) {
            double term = xa * ex / g1, sum = 0.0;
            for (int k = 0; k < 400 && term > 1e-18 * sum; ++k) {
                sum += term;
                term *= x / (a + k + 1.0);
            }
            out[l] = -sum;
        } else {
            out[l] = out[l] - 1.0;
        }
        xa *= x;
        g1 *= a + 1.0;
    }
}

__global__ void k_green_periodic(int n, int lmax, int cutoff, double alpha, int images, int nk,
                                 const int *__restrict__ kvec,
                                 const double *__restrict__ table, double *__restrict__ G) {
    const int64_t npts = (int64_t)n * n * n;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= npts) return;
    const int ix = (int)(idx % n), iy = (int)((idx / n) % n), iz = (int)(idx / ((int64_t)n * n));
    const int dx = ix <= n / 2 ? ix : ix - n;
    const int dy = iy <= n / 2 ? iy : iy - n;
    const int dz = iz <= n / 2 ? iz : iz - n;
    const int ntri = (lmax + 1) * (lmax + 2) / 2;
    const double box = (double)n;
    const double pi = 3.14159265358979323846;
    double are[kMaxTri], aim[kMaxTri], sre[kMaxTri], sim[kMaxTri], Qg[kMaxL + 2];
    for (int u = 0; u < ntri; ++u) are[u] = aim[u] = 0.0;
    const bool origin = dx == 0 && dy == 0 && dz == 0;
    // the near field covers the primary image of the near cells: that
    // image's real-space term Q S - S is taken as -P S (same value, no
    // cancellation of two nearly equal large terms)
    int cheb = abs(dx) > abs(dy) ? abs(dx) : abs(dy);
    cheb = cheb > abs(dz) ? cheb : abs(dz);
    const bool near = cheb > 0 && cheb <= cutoff;
    // real-space images: every offset + n b within `images` box lengths of
    // the origin (a ball in distance: the image sets of d and -d mirror each
    // other, whichever image of a half-box offset d is)
    const double rmax2 = (double)images * images * box * box;
    for (int a = -images - 1; a <= images + 1; ++a)
        for (int b = -images - 1; b <= images + 1; ++b)
            for (int c = -images - 1; c <= images + 1; ++c) {
                if (origin && a == 0 && b == 0 && c == 0) continue;
                const double vx = dx + a * box, vy = dy + b * box, vz = dz + c * box;
                const double r2 = vx * vx + vy * vy + vz * vz;
                if (r2 > rmax2) continue;
                const double x = alpha * alpha * r2;
                inc_gamma_half_dev(lmax, x, near && a == 0 && b == 0 && c == 0, Qg);
                singular_tri(lmax, vx, vy, vz, sre, sim);
                for (int l = 0; l <= lmax; ++l)
                    for (int m = 0; m <= l; ++m) {
                        const int u = tri_idx(l, m);
                        are[u] += Qg[l] * sre[u];
                        aim[u] += Qg[l] * sim[u];
                    }
            }
    for (int t = 0; t < nk; ++t) {
        const double ph = 2.0 * pi * (kvec[3 * t] * dx + kvec[3 * t + 1] * dy + kvec[3 * t + 2] * dz) / box;
        double s, c;
        sincos(ph, &s, &c);
        const double *row = table + (int64_t)t * ntri * 2;
        for (int u = 0; u < ntri; ++u) {
            are[u] += row[2 * u] * c - row[2 * u + 1] * s;
            aim[u] += row[2 * u] * s + row[2 * u + 1] * c;
        }
    }
    for (int l = 0; l <= lmax; ++l) {
        G[(int64_t)(l * (l + 1)) * npts + idx] = are[tri_idx(l, 0)];
        for (int m = 1; m <= l; ++m) {
            G[(int64_t)(l * (l + 1) + m) * npts + idx] = are[tri_idx(l, m)];
            G[(int64_t)(l * (l + 1) - m) * npts + idx] = aim[tri_idx(l, m)];
        }
    }
}

__global__ void k_to_complex(int64_t count, const double *__restrict__ src,
                             cplx<double> *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = {src[i], 0.0};
}

// In-place forward FFT of `nlines` lines; line L starts at
// (L / stride) * stride * nf + (L % stride) and steps by `stride`.
__global__ void __launch_bounds__(64) k_line_fft(cplx<double> *__restrict__ data, int logn,
                                                 int64_t nlines, int64_t stride, int lpb,
                                                 const cplx<double> *__restrict__ tw_g) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int nf = 1 << logn;
    cplx<double> *tw = (cplx<double> *)lds_raw;
    cplx<double> *buf = tw + nf / 2;
    const int tid = threadIdx.x;
    for (int k = tid; k < nf / 2; k += 64) tw[k] = tw_g[k];
    const int64_t l0 = (int64_t)blockIdx.x * lpb;
    int nl = (int)((nlines - l0) < lpb ? (nlines - l0) : lpb);
    for (int idx = tid; idx < nl * nf; idx += 64) {
        const int li = idx % nl, e = idx / nl;
        const int64_t L = l0 + li;
        const int64_t base = (L / stride) * stride * nf + (L % stride);
        buf[li * nf + e] = data[base + (int64_t)e * stride];
    }
    __syncthreads();
    lds_fft_dif<double, false>(buf, logn, nl, nf, 1, tw, tid, 64);
    for (int idx = tid; idx < nl * nf; idx += 64) {
        const int li = idx % nl, pos = idx / nl;
        const int64_t L = l0 + li;
        const int64_t base = (L / stride) * stride * nf + (L % stride);
        data[base + (int64_t)bitrev(pos, logn) * stride] = buf[li * nf + pos];
    }
}

// Keeps Re G~ (even order) or Im G~ (odd order) for ky, kz in [0, nf/2]
// (the other quadrants follow from the y and z reflection symmetries of
// S_n^k), layout [ky' * nh + kx][Q][nhp] with nh = nf/2 + 1 and nhp = nh
// rounded up to 4 (padding zero).  self_shift is added to component 0 at
// every frequency: a kernel weight at offset zero, i.e. the self term
// -(2 alpha/sqrt(pi)) M_0^0(cell) of the periodic correction procedure
// (App. B) applied inside the convolution.
template <typename T>
__global__ void k_fold(int nf, int Q, int j0, int jcount, const cplx<double> *__restrict__ Gc,
                       double self_shift, T *__restrict__ out) {
    const int nh = nf / 2 + 1, nhp = (nh + 3) & ~3;
    const int64_t total = (int64_t)nh * nh * jcount * nhp;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int kz = (int)(i % nhp);
    const int jl = (int)((i / nhp) % jcount);
    const int64_t colr = i / ((int64_t)nhp * jcount);
    const int ky = (int)(colr / nh), kx = (int)(colr % nh);
    const int j = j0 + jl;
    int order = 0;
    while ((order + 1) * (order + 1) <= j) ++order;
    double g = 0.0;
    if (kz < nh) {
        const cplx<double> v = Gc[(((int64_t)jl * nf + kz) * nf + ky) * nf + kx];
        g = (order & 1) ? v.im : v.re + (j == 0 ? self_shift : 0.0);
    }
    out[(colr * Q + j) * nhp + kz] = T(g);
}

static int ilog2i(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

template <typename T>
hipError_t build_green(const GreenArgs &a, hipStream_t s) {
    const int lmax = 2 * a.p, Q = (lmax + 1) * (lmax + 1);
    const int nf = a.nf, logn = ilog2i(nf);
    const int64_t npts = (int64_t)nf * nf * nf;
    double *G = nullptr;
    cplx<double> *Gc = nullptr, *tw = nullptr;
    int *kvec = nullptr;
    double *table = nullptr;
    hipError_t e = hipMalloc(&G, sizeof(double) * Q * npts);
    if (e != hipSuccess) return e;
    const int QB = 8;
    e = hipMalloc(&Gc, sizeof(cplx<double>) * QB * npts);
    if (e != hipSuccess) {
        hipFree(G);
        return e;
    }
    // power-of-two nf: the nf/2 twiddles of the radix-2 transform; any
    // other nf: the nf roots of unity of the direct DFT
    const bool pow2 = (nf & (nf - 1)) == 0;
    const int ntw = pow2 ? (nf / 2 > 0 ? nf / 2 : 1) : nf;
    std::vector<cplx<double>> twh(ntw);
    for (int k = 0; k < ntw; ++k)
        twh[k] = {std::cos(2.0 * M_PI * k / nf), -std::sin(2.0 * M_PI * k / nf)};
    e = hipMalloc(&tw, sizeof(cplx<double>) * twh.size());
    if (e == hipSuccess)
        e = hipMemcpyAsync(tw, twh.data(), sizeof(cplx<double>) * twh.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        const int blocks = (int)((npts + 127) / 128);
        if (a.open) {
            hipLaunchKernelGGL(k_green_open, dim3(blocks), dim3(128), 0, s, a.n, nf, lmax,
                               a.cutoff, G);
        } else {
            std::vector<int> kv;
            for (int x = -a.images; x <= a.images; ++x)
                for (int y = -a.images; y <= a.images; ++y)
                    for (int z = -a.images; z <= a.images; ++z)
                        if ((x || y || z) && x * x + y * y + z * z <= a.images * a.images) {
                            kv.push_back(x);
                            kv.push_back(y);
                            kv.push_back(z);
                        }
            const int nk = (int)kv.size() / 3;
            const int ntri = (lmax + 1) * (lmax + 2) / 2;
            e = hipMalloc(&kvec, sizeof(int) * kv.size());
            if (e == hipSuccess) e = hipMalloc(&table, sizeof(double) * 2 * ntri * nk);
            if (e == hipSuccess)
                e = hipMemcpyAsync(kvec, kv.data(), sizeof(int) * kv.size(),
                                   hipMemcpyHostToDevice, s);
            if (e == hipSuccess) {
                hipLaunchKernelGGL(k_green_recip, dim3((nk + 63) / 64), dim3(64), 0, s, nk, kvec,
                                   (double)a.n, a.alpha_cell, lmax, table);
                hipLaunchKernelGGL(k_green_periodic, dim3(blocks), dim3(128), 0, s, a.n, lmax,
                                   a.cutoff, a.alpha_cell, a.images, nk, kvec, table, G);
            }
        }
        if (e == hipSuccess) e = hipGetLastError();
    }
    const int lpb = nf >= 128 ? 4 : 8;
    const size_t lds = sizeof(cplx<double>) * (nf / 2 + lpb * nf);
    for (int j0 = 0; e == hipSuccess && j0 < Q; j0 += QB) {
        const int jc = (Q - j0) < QB ? (Q - j0) : QB;
        const int64_t cnt = (int64_t)jc * npts;
        hipLaunchKernelGGL(k_to_complex, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                           cnt, G + (int64_t)j0 * npts, Gc);
        for (int axis = 0; axis < 3 && e == hipSuccess; ++axis) {
            const int64_t stride = axis == 0 ? 1 : (axis == 1 ? nf : (int64_t)nf * nf);
            const int64_t nlines = (int64_t)jc * nf * nf;
            if (pow2)
                hipLaunchKernelGGL(k_line_fft, dim3((unsigned)((nlines + lpb - 1) / lpb)),
                                   dim3(64), lds, s, Gc, logn, nlines, stride, lpb, tw);
            else
                e = launch_line_dft_f64(Gc, nf, nlines, stride, tw, s);
        }
        const int nhp = ((nf / 2 + 1) + 3) & ~3;
        const int64_t tot = (int64_t)(nf / 2 + 1) * (nf / 2 + 1) * jc * nhp;
        const double shift = a.open ? 0.0 : -2.0 * a.alpha_cell / std::sqrt(M_PI);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_fold<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, nf, Q,
                           j0, jc, Gc, shift, (T *)a.green_out);
        e = hipGetLastError();
    }
    hipError_t e2 = hipStreamSynchronize(s);
    if (e == hipSuccess) e = e2;
    hipFree(G);
    hipFree(Gc);
    if (tw) hipFree(tw);
    if (kvec) hipFree(kvec);
    if (table) hipFree(table);
    return e;
}

// Fine-level table of the hierarchical far field (one thread per offset).
__global__ void k_hier_table(int lmax, int cutoff, int D, float *__restrict__ out) {
    const int W = 2 * D + 1, Q = (lmax + 1) * (lmax + 1);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)W * W * W) return;
    const int dx = (int)(t % W) - D, dy = (int)((t / W) % W) - D, dz = (int)(t / ((int64_t)W * W)) - D;
    float *o = out + t * Q;
    int cheb = abs(dx) > abs(dy) ? abs(dx) : abs(dy);
    cheb = cheb > abs(dz) ? cheb : abs(dz);
    if (cheb <= cutoff) {
        for (int j = 0; j < Q; ++j) o[j] = 0.0f;
        return;
    }
    double sre[kMaxTri], sim[kMaxTri];
    singular_tri(lmax, (double)dx, (double)dy, (double)dz, sre, sim);
    for (int l = 0; l <= lmax; ++l) {
        o[l * (l + 1)] = (float)sre[tri_idx(l, 0)];
        for (int m = 1; m <= l; ++m) {
            o[l * (l + 1) + m] = (float)sre[tri_idx(l, m)];
            o[l * (l + 1) - m] = (float)sim[tri_idx(l, m)];
        }
    }
}

hipError_t build_hier_table_f32(int p, int cutoff, int D, float *out, hipStream_t s) {
    const int64_t W = 2 * D + 1, cnt = W * W * W;
    hipLaunchKernelGGL(k_hier_table, dim3((unsigned)((cnt + 127) / 128)), dim3(128), 0, s, 2 * p,
                       cutoff, D, out);
    return hipGetLastError();
}

template hipError_t build_green<float>(const GreenArgs &, hipStream_t);
template hipError_t build_green<double>(const GreenArgs &, hipStream_t);

}  // namespace pmmm
