// Device-side helpers shared by the kernels of this library.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace wsmul {

// Canonical residue of an integer-valued double |x| < 2^53.  With
// q = floor(x * fl(1/p)) the remainder x - q*p lies in [-p, 2p) (the rounding
// error of x * fl(1/p) is below one unit), and being a small integer it is
// computed exactly by one fused multiply-add; one correction each way
// finishes the job.
__device__ __forceinline__ double mod_reduce(double x, double p, double pinv) {
    const double q = floor(x * pinv);
    double r = fma(-q, p, x);
    r = r < 0.0 ? r + p : r;
    r = r >= p ? r - p : r;
    return r;
}

// Residues below 2^31 travel through the low 32 bits of int64 storage.
__device__ __forceinline__ double to_f64(double x) { return x; }
__device__ __forceinline__ double to_f64(int64_t x) { return (double)(int32_t)x; }
template <typename T> __device__ __forceinline__ T from_f64(double x);
template <> __device__ __forceinline__ double from_f64<double>(double x) { return x; }
template <> __device__ __forceinline__ int64_t from_f64<int64_t>(double x) {
    return (int64_t)(int32_t)x;
}

// Two consecutive elements through one 16-byte access.
__device__ __forceinline__ void load2(const double *p, double &a, double &b) {
    const double2 v = *reinterpret_cast<const double2 *>(p);
    a = v.x;
    b = v.y;
}
__device__ __forceinline__ void load2(const int64_t *p, double &a, double &b) {
    const longlong2 v = *reinterpret_cast<const longlong2 *>(p);
    a = (double)(int32_t)v.x;
    b = (double)(int32_t)v.y;
}
__device__ __forceinline__ void store2(double *p, double a, double b) {
    *reinterpret_cast<double2 *>(p) = make_double2(a, b);
}
__device__ __forceinline__ void store2(int64_t *p, double a, double b) {
    *reinterpret_cast<longlong2 *>(p) = make_longlong2((int64_t)(int32_t)a, (int64_t)(int32_t)b);
}

// Unsigned 32-bit division by a runtime constant d >= 1 with a precomputed
// multiplier (round-up method): with l = ceil(log2 d) and
// m = floor(2^32 * (2^l - d) / d) + 1, floor(x / d) = (mulhi(x, m) + x) >> l
// for every 32-bit x (the sum is formed in 64 bits).
struct FastDiv {
    uint32_t d, m, l;
    __host__ void init(uint32_t divisor) {
        d = divisor;
        l = 0;
        while ((uint64_t(1) << l) < d)
            ++l;
        m = (uint32_t)(((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1);
    }
    __device__ __forceinline__ uint32_t div(uint32_t x) const {
        const uint64_t hi = __umulhi(x, m);
        return (uint32_t)((hi + x) >> l);
    }
};

}  // namespace wsmul
