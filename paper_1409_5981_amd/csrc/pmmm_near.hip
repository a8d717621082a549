// Near field, for checking totals only (Sec. 2.1, last paragraph: the cells
// masked out of the transfer kernel interact by direct Newtonian sums, with
// no cutoff function).  One thread per sorted particle walks the (2c+1)^3
// neighbour cells of its own cell; periodic meshes wrap the cell offset and
// shift the partner by the box.  Works in cell units from the sorted
// records of the last far-field call.
#include "pmmm_internal.h"

namespace pmmm {

template <typename T>
__global__ void __launch_bounds__(256) k_near(int64_t n, int nc, int cutoff, int periodic,
                                              int accumulate, const int *__restrict__ start,
                                              const int *__restrict__ scell,
                                              const int *__restrict__ perm,
                                              const particle4<T> *__restrict__ sorted, T inv_h,
                                              T *__restrict__ phi, T *__restrict__ gx,
                                              T *__restrict__ gy, T *__restrict__ gz) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const particle4<T> ri = sorted[s];
    const int c = scell[s];
    const int ix = c % nc, iy = (c / nc) % nc, iz = c / (nc * nc);
    T p = T(0), ax = T(0), ay = T(0), az = T(0);
    for (int oz = -cutoff; oz <= cutoff; ++oz) {
        int jz = iz + oz, sz = 0;
        if (jz < 0 || jz >= nc) {
            if (!periodic) continue;
            sz = jz < 0 ? -nc : nc;
            jz -= sz;
        }
        for (int oy = -cutoff; oy <= cutoff; ++oy) {
            int jy = iy + oy, sy = 0;
            if (jy < 0 || jy >= nc) {
                if (!periodic) continue;
                sy = jy < 0 ? -nc : nc;
                jy -= sy;
            }
            for (int ox = -cutoff; ox <= cutoff; ++ox) {
                int jx = ix + ox, sx = 0;
                if (jx < 0 || jx >= nc) {
                    if (!periodic) continue;
                    sx = jx < 0 ? -nc : nc;
                    jx -= sx;
                }
                const int cj = (jz * nc + jy) * nc + jx;
                // displacement r_i - r_j in cell units: -(offset) + (u_i - u_j)
                const T bx = T(-ox), by = T(-oy), bz = T(-oz);
                for (int t = start[cj]; t < start[cj + 1]; ++t) {
                    if (t == s) continue;
                    const particle4<T> rj = sorted[t];
                    const T dx = bx + (ri.ux - rj.ux);
                    const T dy = by + (ri.uy - rj.uy);
                    const T dz = bz + (ri.uz - rj.uz);
                    const T r2 = dx * dx + dy * dy + dz * dz;
                    const T rinv = T(1) / sqrt(r2);
                    const T qr = rj.q * rinv;
                    p += qr;
                    const T qr3 = qr * rinv * rinv;
                    ax -= qr3 * dx;
                    ay -= qr3 * dy;
                    az -= qr3 * dz;
                }
                (void)sx;
                (void)sy;
                (void)sz;
            }
        }
    }
    const int i = perm[s];
    const T ih2 = inv_h * inv_h;
    if (accumulate) {
        phi[i] += p * inv_h;
        gx[i] += ax * ih2;
        gy[i] += ay * ih2;
        gz[i] += az * ih2;
    } else {
        phi[i] = p * inv_h;
        gx[i] = ax * ih2;
        gy[i] = ay * ih2;
        gz[i] = az * ih2;
    }
}

template <typename T>
hipError_t launch_near(const NearArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_near<T>, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a.n,
                       a.ncell, a.cutoff, a.periodic, a.accumulate, a.start, a.scell, a.perm,
                       (const particle4<T> *)a.sorted, T(a.inv_h), (T *)a.phi, (T *)a.gx,
                       (T *)a.gy, (T *)a.gz);
    return hipGetLastError();
}

template hipError_t launch_near<float>(const NearArgs &, hipStream_t);
template hipError_t launch_near<double>(const NearArgs &, hipStream_t);

}  // namespace pmmm
