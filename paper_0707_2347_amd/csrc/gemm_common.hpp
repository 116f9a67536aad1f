// Shared pieces of the base-product kernels: parameters, tile order and the
// fused epilogue.
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"
#include "wsmul.h"

namespace wsmul {

// Base product D-group <- alpha*A*B (mod p) on the binary64 matrix cores
// (v_mfma_f64_16x16x4_f64), then the epilogue group of addition rows fused
// behind it.  Entries are integers, so every partial sum is exact while it
// stays below 2^53; the accumulators are folded back to residues every
// `kc_tiles` K-tiles, and operands are centred into (-p/2, p/2] when p is
// large enough for that to lengthen the fold period.
typedef double f64x4 __attribute__((ext_vector_type(4)));

struct GemmParams {
    const void *A;
    const void *B;
    int64_t lda, ldb;
    int64_t M, N, K;
    double p, pinv, half, alpha;
    int32_t kc_tiles;   // fold period in K-tiles of the kernel (0 = only at the end)
    int32_t tiles_m, tiles_n;
    int32_t nin, nout;
    const void *ein[WS_MAX_IN];
    int64_t eldi[WS_MAX_IN];
    void *eout[WS_MAX_OUT];
    int64_t eldo[WS_MAX_OUT];
    double coef[WS_MAX_OUT][WS_MAX_IN];
};

// Workgroup ids are dealt round-robin to the 8 XCDs; renumber them so that
// consecutive tile numbers run on one XCD (sharing its L2), then walk tiles
// in bands of 8 tile-rows so neighbouring workgroups share A and B panels.
__device__ __forceinline__ void tile_of(int32_t tiles_m, int32_t tiles_n, int32_t &tm,
                                        int32_t &tn) {
    const uint32_t G = gridDim.x, b = blockIdx.x;
    const uint32_t q = G / 8, r = G % 8, x = b % 8;
    const uint32_t pid = x * q + min(x, r) + b / 8;
    const int32_t band = 8;
    const int32_t per_band = band * tiles_n;
    const int32_t g = pid / per_band;
    const int32_t first = g * band;
    const int32_t rows_here = min(band, tiles_m - first);
    const int32_t in_band = pid % per_band;
    tm = first + in_band % rows_here;
    tn = in_band / rows_here;
}

template <typename T>
__device__ __forceinline__ double centred(T raw, double p, double half, bool centre) {
    double x = to_f64(raw);
    return (centre && x > half) ? x - p : x;
}

// Product of one element, reduced: alpha * (acc mod p) mod p, where acc is
// the exact dot product (|acc| < 2^53).
__device__ __forceinline__ double product_residue(const GemmParams &P, double acc) {
    return mod_reduce(P.alpha * mod_reduce(acc, P.p, P.pinv), P.p, P.pinv);
}

// Epilogue inputs 1.. of the fused group at (row, col).
template <typename T>
__device__ __forceinline__ void epilogue_load(const GemmParams &P, double (&x)[WS_MAX_IN],
                                              int64_t row, int64_t col) {
#pragma unroll
    for (int i = 1; i < WS_MAX_IN; ++i)
        if (i < P.nin)
            x[i] = to_f64(static_cast<const T *>(P.ein[i])[row * P.eldi[i] + col]);
}

// Every output of the fused group at (row, col); x[0] is the reduced product.
template <typename T>
__device__ __forceinline__ void epilogue_store(const GemmParams &P, const double (&x)[WS_MAX_IN],
                                               int64_t row, int64_t col) {
#pragma unroll
    for (int o = 0; o < WS_MAX_OUT; ++o) {
        if (o >= P.nout)
            break;
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < WS_MAX_IN; ++i)
            if (i < P.nin)
                s = fma(P.coef[o][i], x[i], s);
        static_cast<T *>(P.eout[o])[row * P.eldo[o] + col] = from_f64<T>(mod_reduce(s, P.p, P.pinv));
    }
}

// Epilogue for one element: prod is the reduced product, input 0 of the
// fused group; the other inputs are read at (row, col) and every output of
// the group is stored there.
template <typename T>
__device__ __forceinline__ void epilogue_apply(const GemmParams &P, double prod, int64_t row,
                                               int64_t col) {
    double x[WS_MAX_IN];
    x[0] = prod;
    epilogue_load<T>(P, x, row, col);
    epilogue_store<T>(P, x, row, col);
}


}  // namespace wsmul
