// Coefficient storage variants for moment and local-expansion meshes:
//   * per-order fixed-point cell records (Sec. 5.3): a word of order l takes
//     b_l = 3 (p + 1 - l) bits, so a cell takes 3 (p+1)(p+2)(2p+3)/6 bits
//     (612 at p = 7) instead of 32 (p+1)^2;
//   * the complex composition of two real coefficient sets and its split
//     (App. D).
// Meshes are component-major, [(p+1)^2][ncell], in the real storage of the
// pipeline (index l(l+1)+m: Re X_l^|m| for m >= 0, Im X_l^|m| for m < 0).
// Records are cell-major, [ncell][words], each a little-endian bit stream of
// b_l-bit two's-complement codes in real-storage order, zero-padded.
// All kernels are HBM-bound streams; a block stages 256 records in LDS so
// that both the component rows and the record array move coalesced.
#include "pmmm_internal.h"

namespace pmmm {
namespace {

constexpr int kStoreThreads = 256;

__host__ __device__ constexpr int record_bits(int p) {
    return 3 * (p + 1) * (p + 2) * (2 * p + 3) / 6;
}
__host__ __device__ constexpr int record_words(int p) { return (record_bits(p) + 31) / 32; }
// LDS row stride of a staged record: odd, so that lanes reading word w of
// consecutive records fall in different banks.
__host__ __device__ constexpr int record_stride(int p) { return record_words(p) | 1; }

// Binary exponent E of a positive finite float with a = f 2^E, 1/2 <= f < 1
// (subnormals included), from its bit pattern.
__device__ __forceinline__ int frexp_exponent(unsigned abits) {
    const int ef = (int)(abits >> 23);
    if (ef != 0) return ef - 126;
    return -117 - __clz(abits & 0x7fffffu);
}

// Unit exponent of an order from the largest |word| (as a bit pattern): the
// smallest power of two under which that word rounds inside b bits.
__device__ __forceinline__ int unit_exponent(unsigned amax, int b) {
    if (amax >= 0x7f800000u) return PMMM_COEF_EXP_INVALID;
    if (amax == 0u) return 0;
    int e = frexp_exponent(amax) - (b - 1);
    if (rintf(ldexpf(__uint_as_float(amax), -e)) >= ldexpf(1.0f, b - 1)) ++e;
    return e;
}

__global__ void k_coef_fill(int *__restrict__ a, int n, int v) {
    const int i = threadIdx.x;
    if (i < n) a[i] = v;
}

// Largest |word| of each order, as float bit patterns (for non-negative
// floats the unsigned order of the patterns is the order of the values; a
// non-finite word gives a pattern >= 0x7f800000).  Grid (chunks, components):
// each block reduces a strided share of one component row and writes its
// maximum to part[component * chunks + chunk], or, with part == nullptr (a
// mesh too small to lend its record array), merges it into amax[order].
__global__ __launch_bounds__(kStoreThreads) void k_coef_max(const float *__restrict__ coef,
                                                            int64_t ncell,
                                                            unsigned *__restrict__ part,
                                                            unsigned *__restrict__ amax) {
    __shared__ unsigned red[kStoreThreads / 64];
    const int k = blockIdx.y;
    const float *row = coef + (int64_t)k * ncell;
    const int64_t stride = (int64_t)gridDim.x * kStoreThreads;
    int64_t c = (int64_t)blockIdx.x * kStoreThreads + threadIdx.x;
    unsigned m = 0;
    for (; c + 3 * stride < ncell; c += 4 * stride) {
        const unsigned a0 = __float_as_uint(row[c]), a1 = __float_as_uint(row[c + stride]);
        const unsigned a2 = __float_as_uint(row[c + 2 * stride]);
        const unsigned a3 = __float_as_uint(row[c + 3 * stride]);
        m = max(m, max(max(a0 & 0x7fffffffu, a1 & 0x7fffffffu),
                       max(a2 & 0x7fffffffu, a3 & 0x7fffffffu)));
    }
    for (; c < ncell; c += stride) m = max(m, __float_as_uint(row[c]) & 0x7fffffffu);
    for (int o = 32; o > 0; o >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int w = 1; w < kStoreThreads / 64; ++w) m = max(m, red[w]);
    if (part) {
        part[(int64_t)k * gridDim.x + blockIdx.x] = m;
    } else if (m != 0) {
        int l = 0;
        while ((l + 1) * (l + 1) <= k) ++l;
        atomicMax(amax + l, m);
    }
}

// Unit exponents from the partial maxima (one block of kFinalThreads):
// wave w reduces components w, w + waves, ... across their chunks with
// shuffles, and the per-order maxima meet in LDS.
constexpr int kFinalThreads = 1024;
__global__ __launch_bounds__(kFinalThreads) void k_coef_max_final(const unsigned *__restrict__ part,
                                                                  int chunks, int p,
                                                                  int *__restrict__ exps) {
    __shared__ unsigned red[PMMM_PMAX + 1];
    if (threadIdx.x <= p) red[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = wave; k < nreal(p); k += kFinalThreads / 64) {
        unsigned m = 0;
        for (int i = lane; i < chunks; i += 64) m = max(m, part[(int64_t)k * chunks + i]);
        for (int o = 32; o > 0; o >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, o));
        if (lane == 0 && m != 0) {
            int l = 0;
            while ((l + 1) * (l + 1) <= k) ++l;
            atomicMax(&red[l], m);
        }
    }
    __syncthreads();
    if (threadIdx.x <= p) exps[threadIdx.x] = unit_exponent(red[threadIdx.x], 3 * (p + 1 - threadIdx.x));
}

__global__ void k_coef_exps(int *__restrict__ exps, int p) {
    const int l = threadIdx.x;
    if (l <= p) exps[l] = unit_exponent((unsigned)exps[l], 3 * (p + 1 - l));
}

// One thread per cell: codes of the (p+1)^2 words appended to a 64-bit bit
// buffer that is flushed to the staged record 32 bits at a time.  With the
// loops unrolled every shift and flush position is a compile-time constant.
template <int PO>
__global__ __launch_bounds__(kStoreThreads) void k_coef_pack(const float *__restrict__ coef,
                                                             int64_t ncell,
                                                             const int *__restrict__ exps,
                                                             uint32_t *__restrict__ records) {
    constexpr int W = record_words(PO), WS = record_stride(PO);
    __shared__ uint32_t rec[kStoreThreads * WS];
    __shared__ int se[PO + 1];
    const int tid = threadIdx.x;
    if (tid <= PO) se[tid] = exps[tid];
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kStoreThreads;
    const int64_t c = base + tid;
    if (c < ncell) {
        // every word of the cell in flight at once, then the bit stream
        float xs[nreal(PO)];
#pragma unroll
        for (int k = 0; k < nreal(PO); ++k) xs[k] = coef[(int64_t)k * ncell + c];
        uint32_t *r = rec + tid * WS;
        uint64_t acc = 0;
        int nb = 0, w = 0;
#pragma unroll
        for (int l = 0; l <= PO; ++l) {
            const int b = 3 * (PO + 1 - l);
            const int e = se[l];
            const float flim = ldexpf(1.0f, b - 1);
            const int64_t ilim = ((int64_t)1 << (b - 1)) - 1;
            const uint64_t mask = ((uint64_t)1 << b) - 1;
#pragma unroll
            for (int j = 0; j < 2 * l + 1; ++j) {
                const float x = xs[l * l + j];
                int64_t code = 0;
                if (e != PMMM_COEF_EXP_INVALID) {
                    float v = rintf(ldexpf(x, -e));
                    if (v != v) v = 0.0f;
                    v = fminf(fmaxf(v, -flim), flim);
                    code = (int64_t)v;
                    code = code > ilim ? ilim : (code < -ilim ? -ilim : code);
                }
                acc |= ((uint64_t)code & mask) << nb;
                nb += b;
                while (nb >= 32) {
                    r[w++] = (uint32_t)acc;
                    acc >>= 32;
                    nb -= 32;
                }
            }
        }
        if (nb > 0) r[w] = (uint32_t)acc;
    }
    __syncthreads();
    const int nvalid = (int)min<int64_t>(kStoreThreads, ncell - base);
    uint32_t *dst = records + base * W;
    for (int i = tid; i < nvalid * W; i += kStoreThreads) {
        const int cc = i / W;
        dst[i] = rec[cc * WS + (i - cc * W)];
    }
}

template <int PO>
__global__ __launch_bounds__(kStoreThreads) void k_coef_unpack(const uint32_t *__restrict__ records,
                                                               int64_t ncell,
                                                               const int *__restrict__ exps,
                                                               float *__restrict__ coef) {
    constexpr int W = record_words(PO), WS = record_stride(PO);
    __shared__ uint32_t rec[kStoreThreads * WS];
    __shared__ int se[PO + 1];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kStoreThreads;
    const int nvalid = (int)min<int64_t>(kStoreThreads, ncell - base);
    const uint32_t *src = records + base * W;
    for (int i = tid; i < nvalid * W; i += kStoreThreads) {
        const int cc = i / W;
        rec[cc * WS + (i - cc * W)] = src[i];
    }
    if (tid <= PO) se[tid] = exps[tid];
    __syncthreads();
    const int64_t c = base + tid;
    if (c >= ncell) return;
    const uint32_t *r = rec + tid * WS;
    uint64_t acc = 0;
    int nb = 0, w = 0;
#pragma unroll
    for (int l = 0; l <= PO; ++l) {
        const int b = 3 * (PO + 1 - l);
        const int e = se[l];
        const uint64_t mask = ((uint64_t)1 << b) - 1;
#pragma unroll
        for (int j = 0; j < 2 * l + 1; ++j) {
            while (nb < b) {
                acc |= (uint64_t)r[w++] << nb;
                nb += 32;
            }
            const uint64_t u = acc & mask;
            acc >>= b;
            nb -= b;
            const int64_t v = (int64_t)(u << (64 - b)) >> (64 - b);
            const float f = b <= 24 ? (float)(int)v : (float)v;
            coef[(int64_t)(l * l + j) * ncell + c] =
                e == PMMM_COEF_EXP_INVALID ? __int_as_float(0x7fc00000) : ldexpf(f, e);
        }
    }
}

// App. D composition: C_l^m = A_l^m + i B_l^m over every -l <= m <= l, with
// A_l^{-m} = (-1)^m conj(A_l^m) (likewise B), written as (re, im) pairs.
__global__ __launch_bounds__(kStoreThreads) void k_coef_compose(const float *__restrict__ a,
                                                                const float *__restrict__ b,
                                                                int64_t ncell, int p,
                                                                float2 *__restrict__ cmp) {
    const int64_t stride = (int64_t)gridDim.x * kStoreThreads;
    for (int64_t c = (int64_t)blockIdx.x * kStoreThreads + threadIdx.x; c < ncell; c += stride) {
        for (int l = 0; l <= p; ++l) {
            const int64_t k0 = (int64_t)ridx(l, 0) * ncell + c;
            cmp[k0] = make_float2(a[k0], b[k0]);
            for (int m = 1; m <= l; ++m) {
                const int64_t kp = (int64_t)ridx(l, m) * ncell + c;
                const int64_t km = (int64_t)ridx(l, -m) * ncell + c;
                const float ar = a[kp], ai = a[km], br = b[kp], bi = b[km];
                const float s = (m & 1) ? -1.0f : 1.0f;
                cmp[kp] = make_float2(ar - bi, br + ai);
                cmp[km] = make_float2(s * (ar + bi), s * (br - ai));
            }
        }
    }
}

// App. D split: A_l^m = Re[C^m + s C^-m]/2 + i Im[C^m - s C^-m]/2 and
// B_l^m = Im[C^m + s C^-m]/2 - i Re[C^m - s C^-m]/2 with s = (-1)^m.
__global__ __launch_bounds__(kStoreThreads) void k_coef_split(const float2 *__restrict__ cmp,
                                                              int64_t ncell, int p,
                                                              float *__restrict__ a,
                                                              float *__restrict__ b) {
    const int64_t stride = (int64_t)gridDim.x * kStoreThreads;
    for (int64_t c = (int64_t)blockIdx.x * kStoreThreads + threadIdx.x; c < ncell; c += stride) {
        for (int l = 0; l <= p; ++l) {
            const int64_t k0 = (int64_t)ridx(l, 0) * ncell + c;
            const float2 c0 = cmp[k0];
            a[k0] = c0.x;
            b[k0] = c0.y;
            for (int m = 1; m <= l; ++m) {
                const int64_t kp = (int64_t)ridx(l, m) * ncell + c;
                const int64_t km = (int64_t)ridx(l, -m) * ncell + c;
                const float2 cp = cmp[kp], cq = cmp[km];
                const float s = (m & 1) ? -1.0f : 1.0f;
                const float sr = cp.x + s * cq.x, si = cp.y + s * cq.y;
                const float dr = cp.x - s * cq.x, di = cp.y - s * cq.y;
                a[kp] = 0.5f * sr;
                a[km] = 0.5f * di;
                b[kp] = 0.5f * si;
                b[km] = -0.5f * dr;
            }
        }
    }
}

template <int PO>
hipError_t pack_launch(int64_t ncell, const float *coef, uint32_t *records, int *exps,
                       int auto_exp, hipStream_t s) {
    if (auto_exp) {
        // the partial maxima borrow the record array, which the pack below
        // overwrites; a mesh too small to hold them merges with atomics
        const int64_t room = ncell * record_words(PO) / nreal(PO);
        const int64_t chunks = std::min<int64_t>(
            std::min<int64_t>(128, (ncell + 8 * kStoreThreads - 1) / (8 * kStoreThreads)), room);
        if (chunks >= 1) {
            const dim3 grid((unsigned)chunks, nreal(PO));
            k_coef_max<<<grid, kStoreThreads, 0, s>>>(coef, ncell, records, nullptr);
            k_coef_max_final<<<1, kFinalThreads, 0, s>>>(records, (int)chunks, PO, exps);
        } else {
            k_coef_fill<<<1, 64, 0, s>>>(exps, PO + 1, 0);
            if (ncell > 0)
                k_coef_max<<<dim3(1, nreal(PO)), kStoreThreads, 0, s>>>(coef, ncell, nullptr,
                                                                         (unsigned *)exps);
            k_coef_exps<<<1, 64, 0, s>>>(exps, PO);
        }
    }
    if (ncell > 0) {
        const int64_t blocks = (ncell + kStoreThreads - 1) / kStoreThreads;
        k_coef_pack<PO><<<(unsigned)blocks, kStoreThreads, 0, s>>>(coef, ncell, exps, records);
    }
    return hipGetLastError();
}

template <int PO>
hipError_t unpack_launch(int64_t ncell, const uint32_t *records, const int *exps, float *coef,
                         hipStream_t s) {
    if (ncell == 0) return hipSuccess;
    const int64_t blocks = (ncell + kStoreThreads - 1) / kStoreThreads;
    k_coef_unpack<PO><<<(unsigned)blocks, kStoreThreads, 0, s>>>(records, ncell, exps, coef);
    return hipGetLastError();
}

template <int PO>
hipError_t dispatch_pack(int p, int64_t ncell, const float *coef, uint32_t *records, int *exps,
                         int auto_exp, hipStream_t s) {
    if constexpr (PO > PMMM_PMAX) {
        return hipErrorInvalidValue;
    } else {
        if (p == PO) return pack_launch<PO>(ncell, coef, records, exps, auto_exp, s);
        return dispatch_pack<PO + 1>(p, ncell, coef, records, exps, auto_exp, s);
    }
}

template <int PO>
hipError_t dispatch_unpack(int p, int64_t ncell, const uint32_t *records, const int *exps,
                           float *coef, hipStream_t s) {
    if constexpr (PO > PMMM_PMAX) {
        return hipErrorInvalidValue;
    } else {
        if (p == PO) return unpack_launch<PO>(ncell, records, exps, coef, s);
        return dispatch_unpack<PO + 1>(p, ncell, records, exps, coef, s);
    }
}

unsigned elementwise_blocks(int64_t ncell) {
    return (unsigned)std::min<int64_t>((ncell + kStoreThreads - 1) / kStoreThreads, 8192);
}

int check_common(int p, int64_t ncell, const char *fn) {
    if (p < 0 || p > PMMM_PMAX) {
        set_error(std::string(fn) + ": order p outside 0..PMMM_PMAX");
        return PMMM_EINVAL;
    }
    if (ncell < 0 || ncell > ((int64_t)1 << 31)) {
        set_error(std::string(fn) + ": cell count outside 0..2^31");
        return PMMM_EINVAL;
    }
    return PMMM_OK;
}

}  // namespace
}  // namespace pmmm

using namespace pmmm;

extern "C" {

int pmmm_coef_record_words(int p) {
    if (p < 0 || p > PMMM_PMAX) return -1;
    return record_words(p);
}

int pmmm_coef_pack_f32(int p, int64_t ncell, const float *coef, uint32_t *records, int32_t *exps,
                       unsigned flags, void *stream) {
    if (int rc = check_common(p, ncell, "pmmm_coef_pack_f32")) return rc;
    if (flags & ~(unsigned)PMMM_COEF_AUTO_EXP) {
        set_error("pmmm_coef_pack_f32: unknown flag bits");
        return PMMM_EINVAL;
    }
    if (!exps || (ncell > 0 && (!coef || !records))) {
        set_error("pmmm_coef_pack_f32: null pointer");
        return PMMM_EINVAL;
    }
    PMMM_HIP(dispatch_pack<0>(p, ncell, coef, records, (int *)exps,
                              (flags & PMMM_COEF_AUTO_EXP) ? 1 : 0, (hipStream_t)stream));
    return PMMM_OK;
}

int pmmm_coef_unpack_f32(int p, int64_t ncell, const uint32_t *records, const int32_t *exps,
                         float *coef, void *stream) {
    if (int rc = check_common(p, ncell, "pmmm_coef_unpack_f32")) return rc;
    if (ncell > 0 && (!records || !exps || !coef)) {
        set_error("pmmm_coef_unpack_f32: null pointer");
        return PMMM_EINVAL;
    }
    PMMM_HIP(dispatch_unpack<0>(p, ncell, records, (const int *)exps, coef, (hipStream_t)stream));
    return PMMM_OK;
}

int pmmm_coef_compose_f32(int p, int64_t ncell, const float *a, const float *b, float *c,
                          void *stream) {
    if (int rc = check_common(p, ncell, "pmmm_coef_compose_f32")) return rc;
    if (ncell == 0) return PMMM_OK;
    if (!a || !b || !c) {
        set_error("pmmm_coef_compose_f32: null pointer");
        return PMMM_EINVAL;
    }
    k_coef_compose<<<elementwise_blocks(ncell), kStoreThreads, 0, (hipStream_t)stream>>>(
        a, b, ncell, p, (float2 *)c);
    PMMM_HIP(hipGetLastError());
    return PMMM_OK;
}

int pmmm_coef_split_f32(int p, int64_t ncell, const float *c, float *a, float *b, void *stream) {
    if (int rc = check_common(p, ncell, "pmmm_coef_split_f32")) return rc;
    if (ncell == 0) return PMMM_OK;
    if (!a || !b || !c) {
        set_error("pmmm_coef_split_f32: null pointer");
        return PMMM_EINVAL;
    }
    k_coef_split<<<elementwise_blocks(ncell), kStoreThreads, 0, (hipStream_t)stream>>>(
        (const float2 *)c, ncell, p, a, b);
    PMMM_HIP(hipGetLastError());
    return PMMM_OK;
}

}  // extern "C"
