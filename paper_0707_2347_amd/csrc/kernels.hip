// HIP kernels for gfx950: fused addition rows and the binary64 matrix-core
// base product with its fused epilogue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "device.hpp"
#include "gemm_common.hpp"
#include "kernels.hpp"

namespace wsmul {

LaunchTiming &launch_timing() {
    static thread_local LaunchTiming t;
    return t;
}

// ===================================================================== adds
// One launch executes a group of consecutive addition rows of a schedule:
// for every element position, out[o] <- sum_i coef[o][i] * in[i] (mod p).
// Inputs are all loaded before any output is stored, which is what makes the
// group equal to running its rows one after the other (the planner only
// groups views that are identical or disjoint).  HBM-bound: each thread moves
// VEC consecutive elements per input and output with 16-byte accesses.
struct LinParams {
    const void *in[WS_MAX_IN];
    int64_t ldi[WS_MAX_IN];
    void *out[WS_MAX_OUT];
    int64_t ldo[WS_MAX_OUT];
    double coef[WS_MAX_OUT][WS_MAX_IN];
    int32_t nout;
    uint32_t items;  // rows * cols / VEC
    FastDiv per_row; // cols / VEC
    double p, pinv;
};

template <typename T, int VEC, int NI, int ITEMS>
__global__ __launch_bounds__(256) void lincomb_kernel(LinParams P) {
    // ITEMS vector items per thread, a grid-size apart (every load instruction
    // of a wave stays contiguous); all loads are issued before any store.
    const uint32_t stride = gridDim.x * 256u;
    const uint32_t first = blockIdx.x * 256u + threadIdx.x;
    double x[ITEMS][NI][VEC];
    int64_t rr[ITEMS], cc[ITEMS];
    bool ok[ITEMS];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const uint32_t idx = first + it * stride;
        ok[it] = idx < P.items;
        const uint32_t r = P.per_row.div(ok[it] ? idx : 0u);
        rr[it] = r;
        cc[it] = (int64_t)((ok[it] ? idx : 0u) - r * P.per_row.d) * VEC;
        if (!ok[it])
            continue;
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const T *src = static_cast<const T *>(P.in[i]) + rr[it] * P.ldi[i] + cc[it];
            if constexpr (VEC == 2)
                load2(src, x[it][i][0], x[it][i][1]);
            else
                x[it][i][0] = to_f64(src[0]);
        }
    }
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        if (!ok[it])
            continue;
#pragma unroll
        for (int o = 0; o < WS_MAX_OUT; ++o) {
            if (o >= P.nout)
                break;
            T *dst = static_cast<T *>(P.out[o]) + rr[it] * P.ldo[o] + cc[it];
            double y[VEC];
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                double acc = 0.0;
#pragma unroll
                for (int i = 0; i < NI; ++i)
                    acc = fma(P.coef[o][i], x[it][i][v], acc);
                y[v] = mod_reduce(acc, P.p, P.pinv);
            }
            if constexpr (VEC == 2)
                store2(dst, y[0], y[1]);
            else
                dst[0] = from_f64<T>(y[0]);
        }
    }
}

template <typename T, int VEC, int ITEMS>
static hipError_t launch_lin_items(const LinParams &P, int nin, hipStream_t s) {
    const uint32_t threads = (P.items + ITEMS - 1) / ITEMS;
    const dim3 grid((threads + 255) / 256), block(256);
    switch (nin) {
#define WS_LIN_CASE(N) \
    case N: ws_launch((lincomb_kernel<T, VEC, N, ITEMS>), grid, block, 0, s, P); break;
        WS_LIN_CASE(1) WS_LIN_CASE(2) WS_LIN_CASE(3) WS_LIN_CASE(4)
        WS_LIN_CASE(5) WS_LIN_CASE(6) WS_LIN_CASE(7) WS_LIN_CASE(8)
#undef WS_LIN_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Large blocks: several items per thread keep more bytes in flight per wave;
// small blocks: one item per thread keeps every CU busy.
template <typename T, int VEC>
static hipError_t launch_lin_t(const LinParams &P, int nin, hipStream_t s) {
    if (P.items >= (1u << 21))
        return launch_lin_items<T, VEC, 4>(P, nin, s);
    return launch_lin_items<T, VEC, 1>(P, nin, s);
}

static bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

hipError_t launch_add(const ws_op_desc &op, const DevBufs &bufs, int dtype, int64_t p,
                      hipStream_t stream) {
    const int64_t rows = op.out[0].rows, cols = op.out[0].cols;
    if (rows == 0 || cols == 0)
        return hipSuccess;
    const size_t esz = 8;
    LinParams P{};
    bool vec2 = (cols % 2) == 0;
    for (int i = 0; i < op.nin; ++i) {
        const ws_view &v = op.in[i];
        P.in[i] = static_cast<const char *>(bufs.ptr[v.buf]) + v.off * esz;
        P.ldi[i] = v.ld;
        vec2 = vec2 && (v.ld % 2 == 0) && aligned16(P.in[i]);
    }
    for (int o = 0; o < op.nout; ++o) {
        const ws_view &v = op.out[o];
        P.out[o] = static_cast<char *>(bufs.ptr[v.buf]) + v.off * esz;
        P.ldo[o] = v.ld;
        vec2 = vec2 && (v.ld % 2 == 0) && aligned16(P.out[o]);
        for (int i = 0; i < op.nin; ++i)
            P.coef[o][i] = (double)op.coef[o][i];
    }
    P.nout = op.nout;
    P.p = (double)p;
    P.pinv = 1.0 / (double)p;
    const int vec = vec2 ? 2 : 1;
    const uint64_t items = (uint64_t)rows * (uint64_t)(cols / vec);
    if (items >= (uint64_t(1) << 31))
        return hipErrorInvalidValue;
    P.items = (uint32_t)items;
    P.per_row.init((uint32_t)(cols / vec));
    if (dtype == WS_I64)
        return vec2 ? launch_lin_t<int64_t, 2>(P, op.nin, stream)
                    : launch_lin_t<int64_t, 1>(P, op.nin, stream);
    return vec2 ? launch_lin_t<double, 2>(P, op.nin, stream)
                : launch_lin_t<double, 1>(P, op.nin, stream);
}

// ==================================================================== gemm
// Base product D-group <- alpha*A*B (mod p) on the binary64 matrix cores
// (v_mfma_f64_16x16x4_f64), then the epilogue group of addition rows fused
// behind it (parameters and epilogue in gemm_common.hpp).

// ---- LDS-tiled kernel: BM x BN tile per workgroup, four waves in a 2 x 2
// grid, each wave (BM/2) x (BN/2) of 16 x 16 matrix-core tiles, K-tiles of 16
// double-buffered through LDS.  In the matrix-core step s of a K-tile, lane l
// supplies k = 4*(l/16) + s, so each lane's four A values are contiguous in
// LDS; B uses the same k assignment.  PF register stages: with PF = 2 the
// loads of K-tile t+2 are issued while t is multiplied and t+1 waits in the
// other stage, so every load has a whole K-tile of cover (worth it only where
// the extra registers do not cost occupancy).
template <typename T, int BM, int BN, bool CENTRE, bool VEC2, int PF = 1>
__device__ __forceinline__ void gemm_lds_tile(const GemmParams &P, int32_t tm, int32_t tn,
                                              double (*As)[BM * (16 + 2)], double (*Bs)[16 * BN]) {
    constexpr int BK = 16, APAD = 2;
    constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 16, FN = WN / 16;
    constexpr int AST = BK + APAD;                       // A row stride in LDS
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int li = lane & 15, kq = lane >> 4;

    const T *A = static_cast<const T *>(P.A);
    const T *B = static_cast<const T *>(P.B);

    // Global -> register staging: A tile BM x 16, B tile 16 x BN, two
    // elements per access.
    constexpr int A_PAIRS = BM * BK / 2 / 256;   // per thread
    constexpr int B_PAIRS = BK * BN / 2 / 256;
    static_assert(PF == 1 || PF == 2, "one or two register stages");
    double ra[A_PAIRS][2], rb[B_PAIRS][2], ra2[A_PAIRS][2], rb2[B_PAIRS][2];

    auto gload = [&](int64_t k0, double (&ra)[A_PAIRS][2], double (&rb)[B_PAIRS][2]) {
#pragma unroll
        for (int j = 0; j < A_PAIRS; ++j) {
            const int v = tid + 256 * j, row = v / (BK / 2), cp = v % (BK / 2);
            const int64_t gr = m0 + row, gk = k0 + 2 * cp;
            double x0 = 0.0, x1 = 0.0;
            if (gr < P.M) {
                const T *src = A + gr * P.lda + gk;
                if (VEC2) {
                    if (gk < P.K)
                        load2(src, x0, x1);
                } else {
                    if (gk < P.K)
                        x0 = to_f64(src[0]);
                    if (gk + 1 < P.K)
                        x1 = to_f64(src[1]);
                }
            }
            ra[j][0] = (CENTRE && x0 > P.half) ? x0 - P.p : x0;
            ra[j][1] = (CENTRE && x1 > P.half) ? x1 - P.p : x1;
        }
#pragma unroll
        for (int j = 0; j < B_PAIRS; ++j) {
            const int v = tid + 256 * j, kr = v / (BN / 2), np = v % (BN / 2);
            const int64_t gk = k0 + kr, gn = n0 + 2 * np;
            double x0 = 0.0, x1 = 0.0;
            if (gk < P.K) {
                const T *src = B + gk * P.ldb + gn;
                if (VEC2) {
                    if (gn < P.N)
                        load2(src, x0, x1);
                } else {
                    if (gn < P.N)
                        x0 = to_f64(src[0]);
                    if (gn + 1 < P.N)
                        x1 = to_f64(src[1]);
                }
            }
            rb[j][0] = (CENTRE && x0 > P.half) ? x0 - P.p : x0;
            rb[j][1] = (CENTRE && x1 > P.half) ? x1 - P.p : x1;
        }
    };
    auto sstore = [&](int buf, const double (&ra)[A_PAIRS][2], const double (&rb)[B_PAIRS][2]) {
#pragma unroll
        for (int j = 0; j < A_PAIRS; ++j) {
            const int v = tid + 256 * j, row = v / (BK / 2), cp = v % (BK / 2);
            *reinterpret_cast<double2 *>(&As[buf][row * AST + 2 * cp]) = make_double2(ra[j][0], ra[j][1]);
        }
#pragma unroll
        for (int j = 0; j < B_PAIRS; ++j) {
            const int v = tid + 256 * j, kr = v / (BN / 2), np = v % (BN / 2);
            *reinterpret_cast<double2 *>(&Bs[buf][kr * BN + 2 * np]) = make_double2(rb[j][0], rb[j][1]);
        }
    };

    f64x4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
            acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

    auto fold = [&]() {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    acc[i][j][v] = mod_reduce(acc[i][j][v], P.p, P.pinv);
    };

    const int64_t ktiles = (P.K + BK - 1) / BK;
    if (ktiles > 0) {
        gload(0, ra, rb);
        sstore(0, ra, rb);
    }
    if (PF == 2 && ktiles > 1)
        gload(BK, ra2, rb2);
    __syncthreads();
    int since_fold = 0;
    // K-tile t from LDS buffer cur: first request K-tile t+PF into (la, lb),
    // multiply, then move K-tile t+1 from (sa, sb) into the other buffer.
    auto step = [&](int64_t t, int cur, double (&la)[A_PAIRS][2], double (&lb)[B_PAIRS][2],
                    const double (&sa)[A_PAIRS][2], const double (&sb)[B_PAIRS][2]) {
        if (t + PF < ktiles)
            gload((t + PF) * BK, la, lb);
        double af[FM][4];
#pragma unroll
        for (int i = 0; i < FM; ++i) {
            const double *src = &As[cur][(wm * WM + i * 16 + li) * AST + 4 * kq];
            const double2 lo = *reinterpret_cast<const double2 *>(src);
            const double2 hi = *reinterpret_cast<const double2 *>(src + 2);
            af[i][0] = lo.x;
            af[i][1] = lo.y;
            af[i][2] = hi.x;
            af[i][3] = hi.y;
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            double bf[FN];
#pragma unroll
            for (int j = 0; j < FN; ++j)
                bf[j] = Bs[cur][(4 * kq + s) * BN + wn * WN + j * 16 + li];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i][s], bf[j], acc[i][j], 0, 0, 0);
        }
        if (t + 1 < ktiles)
            sstore(cur ^ 1, sa, sb);
        __syncthreads();
        if (P.kc_tiles > 0 && ++since_fold == P.kc_tiles) {
            fold();
            since_fold = 0;
        }
    };
    if (PF == 1) {
        for (int64_t t = 0; t < ktiles; ++t)
            step(t, (int)(t & 1), ra, rb, ra, rb);
    } else {
        for (int64_t t = 0; t < ktiles; t += 2) {
            step(t, 0, ra, rb, ra2, rb2);
            if (t + 1 < ktiles)
                step(t + 1, 1, ra2, rb2, ra, rb);
        }
    }

    // Output layout of the 16 x 16 x 4 binary64 matrix-core op (measured on
    // gfx950): lane l, accumulator element v holds row l/16 + 4*v of column
    // l % 16.  The reduced products go
    // through LDS (reusing the operand buffers) so that the fused epilogue
    // reads and writes whole rows; a 128 x 128 tile takes two rounds, one per
    // half of the wave grid.
    constexpr int LDS_DOUBLES = 2 * BM * AST + 2 * BK * BN;
    constexpr int ROUNDS = (BM * BN <= LDS_DOUBLES) ? 1 : 2;
    static_assert(BM * BN / ROUNDS <= LDS_DOUBLES, "epilogue staging does not fit");
    double *stage = &As[0][0];   // As and Bs are one contiguous block (see callers)
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                acc[i][j][v] = product_residue(P, acc[i][j][v]);
    constexpr int RROWS = BM / ROUNDS;
#pragma unroll
    for (int h = 0; h < ROUNDS; ++h) {
        if (ROUNDS == 1 || wm == h) {
            const int rbase = (ROUNDS == 1 ? wm * WM : 0);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        stage[(rbase + i * 16 + kq + 4 * v) * BN + wn * WN + j * 16 + li] = acc[i][j][v];
        }
        __syncthreads();
        for (int e = tid; e < RROWS * BN; e += 256) {
            const int r = e / BN, c = e % BN;
            const int64_t row = m0 + h * RROWS + r, col = n0 + c;
            if (row < P.M && col < P.N)
                epilogue_apply<T>(P, stage[e], row, col);
        }
        __syncthreads();
    }
}

// ---- Small products: a 32 x 32 output tile per workgroup whose WAVES waves
// split the K-tiles round-robin (so every SIMD holds two waves even when the
// product has only a few hundred output tiles).  Operands are read straight
// from global memory, CH K-tiles of a wave at a time so that all of their
// loads are in flight together; the epilogue's extra inputs are fetched at
// kernel start; partial tiles are summed through LDS.
// LDS operand buffers of one BM x BN tile, contiguous so that the epilogue
// can reuse them as one staging area.
template <int BM, int BN>
struct LdsTile {
    double As[2][BM * (16 + 2)];
    double Bs[2][16 * BN];
};

template <typename T, int BM, int BN, bool CENTRE, bool VEC2>
__global__ __launch_bounds__(256, 2) void gemm_lds_kernel(GemmParams P) {
    __shared__ LdsTile<BM, BN> sh;
    int32_t tm, tn;
    tile_of(P.tiles_m, P.tiles_n, tm, tn);
    gemm_lds_tile<T, BM, BN, CENTRE, VEC2>(P, tm, tn, sh.As, sh.Bs);
}

#ifndef WS_SK_WAVES
#define WS_SK_WAVES 8   // waves splitting K in the small-product kernel
#endif
#ifndef WS_SK_CHUNK
#define WS_SK_CHUNK 1   // K-tiles per wave whose loads are in flight together
#endif

template <typename T, bool CENTRE, bool VEC2, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void gemm_sk_kernel(GemmParams P) {
    constexpr int BM = 32, BN = 32, BK = 16, CH = WS_SK_CHUNK;
    constexpr int EPT = BM * BN / (64 * WAVES);        // epilogue elements per thread
    __shared__ double part[WAVES][BM * BN];
    int32_t tm, tn;
    tile_of(P.tiles_m, P.tiles_n, tm, tn);
    const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, kq = lane >> 4;
    const T *A = static_cast<const T *>(P.A);
    const T *B = static_cast<const T *>(P.B);

    // Epilogue inputs do not depend on the product: start fetching them now.
    double ex[EPT][WS_MAX_IN];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const int e = tid + 64 * WAVES * u;
        const int64_t row = m0 + e / BN, col = n0 + e % BN;
        if (row < P.M && col < P.N)
            epilogue_load<T>(P, ex[u], row, col);
    }

    auto cvt = [&](double x) { return (CENTRE && x > P.half) ? x - P.p : x; };
    // Operands of K-tile t for this lane: A rows m0 + 16i + li at
    // k = 16t + 4kq .. +3, B columns n0 + 16j + li at the same k.
    auto load = [&](int64_t t, double (&af)[2][4], double (&bf)[2][4]) {
        const int64_t k0 = t * BK + 4 * kq;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int64_t gr = m0 + i * 16 + li;
            if (VEC2) {
                double x0 = 0, x1 = 0, x2 = 0, x3 = 0;
                if (gr < P.M && k0 < P.K) {
                    const T *src = A + gr * P.lda + k0;
                    load2(src, x0, x1);
                    load2(src + 2, x2, x3);
                }
                af[i][0] = cvt(x0);
                af[i][1] = cvt(x1);
                af[i][2] = cvt(x2);
                af[i][3] = cvt(x3);
            } else {
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    af[i][s] = (gr < P.M && k0 + s < P.K) ? cvt(to_f64(A[gr * P.lda + k0 + s])) : 0.0;
            }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t gn = n0 + j * 16 + li;
#pragma unroll
            for (int s = 0; s < 4; ++s)
                bf[j][s] = (gn < P.N && k0 + s < P.K) ? cvt(to_f64(B[(k0 + s) * P.ldb + gn])) : 0.0;
        }
    };

    f64x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
    int since_fold = 0;

    const int64_t ktiles = (P.K + BK - 1) / BK;
    double af[CH][2][4], bf[CH][2][4];
    for (int64_t t0 = wave; t0 < ktiles; t0 += CH * WAVES) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int64_t t = t0 + (int64_t)c * WAVES;
            if (t < ktiles) {
                load(t, af[c], bf[c]);
            } else {
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        af[c][i][s] = bf[c][i][s] = 0.0;
            }
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[c][i][s], bf[c][j][s], acc[i][j], 0, 0, 0);
            if (P.kc_tiles > 0 && ++since_fold == P.kc_tiles) {
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            acc[i][j][v] = mod_reduce(acc[i][j][v], P.p, P.pinv);
                since_fold = 0;
            }
        }
    }

#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                part[wave][(i * 16 + kq + 4 * v) * BN + j * 16 + li] =
                    mod_reduce(acc[i][j][v], P.p, P.pinv);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const int e = tid + 64 * WAVES * u;
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w)
            s += part[w][e];
        const int64_t row = m0 + e / BN, col = n0 + e % BN;
        if (row < P.M && col < P.N) {
            ex[u][0] = product_residue(P, s);
            epilogue_store<T>(P, ex[u], row, col);
        }
    }
}

// Base products whose shape is whole TM x TM output tiles (TM = 32 or 64)
// and whole SK-deep inner sub-chunks with 16-byte aligned rows (every
// Winograd leaf of a power-of-two product): one TM x TM output tile per
// workgroup over the full inner dimension, split among the waves.  Wave w owns the SK-deep sub-chunks
// w, w + WAVES, w + 2*WAVES, ... of the inner dimension; it streams their A
// (TM x SK) and B (SK x TM) blocks into STAGES private LDS buffers by direct
// global-to-LDS loads, waits on its own load counter and needs no workgroup
// barrier until the partial tiles are summed in LDS before the fused
// epilogue.
//
// A load instruction writes lane l's 16 bytes at base + 16*l, so the LDS
// layout is fixed by the instruction and the permutation lives in the global
// addresses: 16-byte pieces are XOR-swizzled within each A-row and B-row so
// that the matrix-core operand reads spread over the LDS banks.
#ifndef WS_DMA_WAVES
#define WS_DMA_WAVES 8
#endif
#ifndef WS_DMA_STAGES
#define WS_DMA_STAGES 2
#endif
#ifndef WS_DMA_SK
#define WS_DMA_SK 16
#endif
#ifndef WS_DMA16_WAVES
#define WS_DMA16_WAVES 4
#endif
#ifndef WS_DMA16_STAGES
#define WS_DMA16_STAGES 2
#endif
#ifndef WS_DMA64_WAVES
#define WS_DMA64_WAVES 8
#endif
#ifndef WS_DMA64_STAGES
#define WS_DMA64_STAGES 2
#endif
#ifndef WS_DMA64_SK
#define WS_DMA64_SK 8
#endif
namespace dmak {
// Piece swizzles: A-rows of SK*8 bytes, B-rows of TM*8 bytes.
template <int SK>
__device__ __forceinline__ int aswz(int r) {
    return SK == 16 ? ((r & 7) ^ ((r >> 3) & 1)) : (((r >> 2) & 3) ^ (((r >> 1) & 1) << 1));
}
template <int SK>
__device__ __forceinline__ int bswz(int k) {
    return SK == 16 ? 8 * ((k >> 2) & 1) : 8 * ((k >> 1) & 1);
}
// Wait until at most n of this wave's loads are in flight (n a multiple of 4).
__device__ __forceinline__ void wait_loads(int n) {
    if (n >= 24) asm volatile("s_waitcnt vmcnt(24)" ::: "memory");
    else if (n >= 16) asm volatile("s_waitcnt vmcnt(16)" ::: "memory");
    else if (n >= 12) asm volatile("s_waitcnt vmcnt(12)" ::: "memory");
    else if (n >= 8) asm volatile("s_waitcnt vmcnt(8)" ::: "memory");
    else if (n >= 4) asm volatile("s_waitcnt vmcnt(4)" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}
}  // namespace dmak

template <typename T>
struct alignas(16) Pair {
    T x, y;
};

template <typename T, bool CENTRE, int TM, int WAVES, int STAGES, int SK>
__global__ __launch_bounds__(64 * WAVES) void gemm_dma_kernel(GemmParams P) {
    using namespace dmak;
    constexpr int NB = TM / 16;                        // 16 x 16 blocks per tile side
    constexpr int NT = 64 * WAVES, EPT = TM * TM / NT;
    constexpr int S = SK / 4;                          // matrix-core steps per sub-chunk
    constexpr int A_BYTES = TM * SK * 8, SUB_BYTES = 2 * A_BYTES;
    constexpr int AROWS = 1024 / (SK * 8), AI = TM / AROWS;   // A: rows per instruction, instructions
    constexpr int BPR = TM / 2, BROWS = 64 / BPR, BI = SK / BROWS;   // B: pieces per row, rows, instructions
    constexpr int LPS = AI + BI;                       // load instructions per sub-chunk
    constexpr int LDS_BYTES = WAVES * STAGES * SUB_BYTES;
    constexpr bool PREFETCH = EPT <= 2;                // epilogue inputs fetched up front
    // Partial tiles for the split-K sum, rows padded by two when there is
    // room; PW of them fit the buffers at once (all, or half the waves').
    constexpr int PROW = WAVES * TM * (TM + 2) * 8 <= LDS_BYTES ? TM + 2 : TM;
    constexpr int PSTRIDE = TM * PROW;
    constexpr int PW = WAVES * PSTRIDE * 8 <= LDS_BYTES ? WAVES : WAVES / 2;
    static_assert(TM == 16 || TM == 32 || TM == 64, "16, 32 or 64");
    static_assert(SK == 8 || SK == 16, "sub-chunks of 8 or 16");
    static_assert(TM != 16 || (SK == 16 && EPT >= 1), "16-wide tiles: 16-deep sub-chunks, <= 4 waves");
    static_assert(STAGES >= 2 && (STAGES - 2) * LPS <= 24, "load counter range");
    static_assert(PW * PSTRIDE * 8 <= LDS_BYTES, "partials fit the buffers");
    __shared__ __attribute__((aligned(16))) char lds[LDS_BYTES];
    int32_t tm, tn;
    tile_of(P.tiles_m, P.tiles_n, tm, tn);
    const int64_t m0 = (int64_t)tm * TM, n0 = (int64_t)tn * TM;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, kq = lane >> 4;
    const char *A = static_cast<const char *>(P.A);
    const char *B = static_cast<const char *>(P.B);
    char *mine = lds + wave * (STAGES * SUB_BYTES);

    // Small tiles: epilogue inputs do not depend on the product, fetch them
    // first.
    double ex[PREFETCH ? EPT : 1][WS_MAX_IN];
    if (PREFETCH) {
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int e = tid + NT * u;
            epilogue_load<T>(P, ex[u], m0 + e / TM, n0 + e % TM);
        }
    }

    const int64_t nsub = (P.K / SK - wave + WAVES - 1) / WAVES;   // this wave's sub-chunks
    // Sub-chunk u of this wave into buffer st.
    auto issue = [&](int st, int64_t u) {
        const int64_t k0 = (wave + (int64_t)WAVES * u) * SK;
        char *base = mine + st * SUB_BYTES;
#pragma unroll
        for (int j = 0; j < AI; ++j) {
            const int r = AROWS * j + lane / (SK / 2);
            const int piece = (lane % (SK / 2)) ^ aswz<SK>(r);
            __builtin_amdgcn_global_load_lds(A + ((m0 + r) * P.lda + k0) * 8 + piece * 16,
                                             base + j * 1024, 16, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < BI; ++j) {
            // 16-wide tiles: B-rows of 128 bytes, so instead of a piece swizzle
            // rows k and k ^ 1 trade places when bit 2 of k is set (an
            // involution on the rows one instruction fills).
            const int lr = BROWS * j + lane / BPR;
            const int k = TM == 16 ? lr ^ ((lr >> 2) & 1) : lr;
            const int piece = TM == 16 ? lane % BPR : (lane % BPR) ^ bswz<SK>(k);
            __builtin_amdgcn_global_load_lds(B + ((k0 + k) * P.ldb + n0) * 8 + piece * 16,
                                             base + A_BYTES + j * 1024, 16, 0, 0);
        }
    };
    auto cvt = [&](T raw) {
        const double x = to_f64(raw);
        return (CENTRE && x > P.half) ? x - P.p : x;
    };

    f64x4 acc[NB][NB];
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
            acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
    int since_fold = 0;

#pragma unroll
    for (int st = 0; st < STAGES - 1; ++st)
        if (st < nsub)
            issue(st, st);
    // Step u: sub-chunk u resident (only sub-chunks issued after it may be in
    // flight), refill the buffer of sub-chunk u-1, read the fragments of u
    // (lane (li, kq) holds inner indices S*kq + s, s < S) and multiply.
    for (int64_t u = 0; u < nsub; ++u) {
        wait_loads(LPS * (int)std::max<int64_t>(0, std::min<int64_t>(u + STAGES - 2, nsub - 1) - u));
        if (u + STAGES - 1 < nsub)
            issue((int)((u + STAGES - 1) % STAGES), u + STAGES - 1);
        const char *sa = mine + (int)(u % STAGES) * SUB_BYTES;
        const char *sb = sa + A_BYTES;
        double a[NB][S], b[NB][S];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int r = 16 * i + li;
#pragma unroll
            for (int h = 0; h < S / 2; ++h) {
                const Pair<T> v = *reinterpret_cast<const Pair<T> *>(
                    sa + r * (SK * 8) + (((S / 2) * kq + h) ^ aswz<SK>(r)) * 16);
                a[i][2 * h] = cvt(v.x);
                a[i][2 * h + 1] = cvt(v.y);
            }
        }
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int k = S * kq + s, col = 16 * j + li;
                const int off = TM == 16 ? (k ^ ((k >> 2) & 1)) * (TM * 8) + (col >> 1) * 16
                                         : k * (TM * 8) + ((col >> 1) ^ bswz<SK>(k)) * 16;
                b[j][s] = cvt(*reinterpret_cast<const T *>(sb + off + (col & 1) * 8));
            }
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][s], b[j][s], acc[i][j], 0, 0, 0);
        if (P.kc_tiles > 0 && ++since_fold == P.kc_tiles) {
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        acc[i][j][v] = mod_reduce(acc[i][j][v], P.p, P.pinv);
            since_fold = 0;
        }
    }

    // Split-K sum through LDS, then every thread sums the parked partials of
    // its epilogue elements.  When the whole inner dimension fits below 2^53
    // the raw partials are summed and reduced once.  Output of the 16 x 16 x 4
    // op: lane l, element v is row l/16 + 4v, column l%16.
    const double mx = CENTRE ? P.half + 1.0 : P.p - 1.0;
    const bool raw = P.kc_tiles == 0 && (double)P.K * mx * mx < 9.0e15;
    double *part = reinterpret_cast<double *>(lds);
    auto park = [&](int slot) {
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    part[slot * PSTRIDE + (16 * i + kq + 4 * v) * PROW + 16 * j + li] =
                        raw ? acc[i][j][v] : mod_reduce(acc[i][j][v], P.p, P.pinv);
    };
    __syncthreads();
    if (PW == WAVES) {
        park(wave);
    } else {
        // Two halves: the upper waves park their partials, the lower waves
        // add them to their own and park the sums.
        if (wave >= PW)
            park(wave - PW);
        __syncthreads();
        if (wave < PW) {
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const double mine_v = raw ? acc[i][j][v] : mod_reduce(acc[i][j][v], P.p, P.pinv);
                        acc[i][j][v] = mine_v + part[wave * PSTRIDE + (16 * i + kq + 4 * v) * PROW + 16 * j + li];
                    }
        }
        __syncthreads();
        if (wave < PW)
            park(wave);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const int e = tid + NT * u;
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < PW; ++w)
            sum += part[w * PSTRIDE + (e / TM) * PROW + e % TM];
        const double prod = product_residue(P, sum);
        if (PREFETCH) {
            ex[u][0] = prod;
            epilogue_store<T>(P, ex[u], m0 + e / TM, n0 + e % TM);
        } else {
            epilogue_apply<T>(P, prod, m0 + e / TM, n0 + e % TM);
        }
    }
}

// Large base products of whole 128 x 128 tiles and 16-deep K-steps with
// 16-byte aligned rows: one 128 x 128 output tile per workgroup, eight waves
// in a 2 x 4 grid of 64 x 32 wave tiles (two waves per SIMD), K-steps of 16 in
// four LDS buffers filled by direct global-to-LDS loads three steps ahead, one
// workgroup barrier per K-step (the buffers are shared by the waves).  The
// finished tile is staged through the buffers so that the fused epilogue runs
// on whole rows.  A-rows of 128 bytes and B-rows of 1 KB are piece-swizzled as
// in gemm_dma_kernel.
#ifndef WS_BIG_ENABLE
#define WS_BIG_ENABLE 1
#endif
namespace dmak {
// This wave's loads of a K-step have landed (at most n of its loads, the
// later K-steps', in flight), then every wave's; no fence, so the later loads
// stay in flight across the barrier.
__device__ __forceinline__ void wait_loads_barrier(int n) {
    if (n >= 8) asm volatile("s_waitcnt vmcnt(8)\n\ts_barrier" ::: "memory");
    else if (n >= 4) asm volatile("s_waitcnt vmcnt(4)\n\ts_barrier" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
}
constexpr int BIG_TM = 128, BIG_SK = 16, BIG_STAGES = 4;
constexpr int BIG_A_BYTES = BIG_TM * BIG_SK * 8, BIG_SUB_BYTES = 2 * BIG_A_BYTES;
}  // namespace dmak

template <typename T, bool CENTRE>
__global__ __launch_bounds__(512) void gemm_big_kernel(GemmParams P) {
    using namespace dmak;
    constexpr int TM = BIG_TM, SK = BIG_SK, STAGES = BIG_STAGES, A_BYTES = BIG_A_BYTES,
                  SUB_BYTES = BIG_SUB_BYTES;
    static_assert(STAGES * SUB_BYTES >= TM * TM * 8, "the output tile fits the buffers");
    __shared__ __attribute__((aligned(16))) char lds[BIG_STAGES * BIG_SUB_BYTES];
    int32_t tm, tn;
    tile_of(P.tiles_m, P.tiles_n, tm, tn);
    const int64_t m0 = (int64_t)tm * TM, n0 = (int64_t)tn * TM;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 2, wn = wave & 3;        // 2 x 4 waves of 64 x 32
    const int li = lane & 15, kq = lane >> 4;
    const char *A = static_cast<const char *>(P.A);
    const char *B = static_cast<const char *>(P.B);
    const int64_t nst = P.K / SK;

    // Loads of K-step t: sixteen instructions of 8 A-rows (128 bytes each),
    // sixteen of one B-row (1 KB each); four per wave.
    auto issue = [&](int st, int64_t t) {
        const int64_t k0 = t * SK;
        char *base = lds + st * SUB_BYTES;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int q = wave + 8 * j;
            if (j < 2) {
                const int r = 8 * q + (lane >> 3), piece = (lane & 7) ^ aswz<16>(r);
                __builtin_amdgcn_global_load_lds(A + ((m0 + r) * P.lda + k0) * 8 + piece * 16,
                                                 base + q * 1024, 16, 0, 0);
            } else {
                const int k = q - 16, piece = lane ^ bswz<16>(k);
                __builtin_amdgcn_global_load_lds(B + ((k0 + k) * P.ldb + n0) * 8 + piece * 16,
                                                 base + A_BYTES + k * 1024, 16, 0, 0);
            }
        }
    };
    auto cvt = [&](T raw) {
        const double x = to_f64(raw);
        return (CENTRE && x > P.half) ? x - P.p : x;
    };

    f64x4 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
    int since_fold = 0;

#pragma unroll
    for (int st = 0; st < STAGES - 1; ++st)
        if (st < nst)
            issue(st, st);
    for (int64_t t = 0; t < nst; ++t) {
        wait_loads_barrier(4 * (int)std::max<int64_t>(0, std::min<int64_t>(t + STAGES - 2, nst - 1) - t));
        if (t + STAGES - 1 < nst)
            issue((int)((t + STAGES - 1) % STAGES), t + STAGES - 1);
        const char *sa = lds + (int)(t % STAGES) * SUB_BYTES;
        const char *sb = sa + A_BYTES;
        // lane (li, kq) holds inner indices 4*kq + s, s < 4
        double a[4][4], b[2][4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = wm * 64 + 16 * i + li;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const Pair<T> v = *reinterpret_cast<const Pair<T> *>(
                    sa + r * (SK * 8) + ((2 * kq + h) ^ aswz<16>(r)) * 16);
                a[i][2 * h] = cvt(v.x);
                a[i][2 * h + 1] = cvt(v.y);
            }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int k = 4 * kq + s, col = wn * 32 + 16 * j + li;
                b[j][s] = cvt(*reinterpret_cast<const T *>(
                    sb + k * (TM * 8) + ((col >> 1) ^ bswz<16>(k)) * 16 + (col & 1) * 8));
            }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][s], b[j][s], acc[i][j], 0, 0, 0);
        if (P.kc_tiles > 0 && ++since_fold == P.kc_tiles) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        acc[i][j][v] = mod_reduce(acc[i][j][v], P.p, P.pinv);
            since_fold = 0;
        }
    }

    // Stage the reduced products (alpha applied) and run the epilogue on
    // whole rows.  Output of the 16 x 16 x 4 op: lane l, element v is row
    // l/16 + 4v, column l%16.
    __syncthreads();
    double *stage = reinterpret_cast<double *>(lds);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                stage[(wm * 64 + 16 * i + kq + 4 * v) * TM + wn * 32 + 16 * j + li] =
                    product_residue(P, acc[i][j][v]);
    __syncthreads();
    for (int e = tid; e < TM * TM; e += 512)
        epilogue_apply<T>(P, stage[e], m0 + e / TM, n0 + e % TM);
}

// Fold period of gemm_dma_kernel in sub-chunks: each adds sk products of
// magnitude at most m^2 to a wave's accumulators; 0 if a wave's whole share
// of the inner dimension fits below 2^53.
static int32_t fold_chunks(int64_t p, bool centre, int64_t K, int waves, int sk) {
    const double mx = centre ? (double)((p - 1) / 2 + 1) : (double)(p - 1);
    const double lim = 9007199254740992.0 - 4.0 * (double)p;
    const double t = std::floor(lim / std::max((double)sk * mx * mx, 1.0));
    const double per_wave = std::ceil((double)K / (double)sk / (double)waves);
    if (t >= per_wave)
        return 0;
    return (int32_t)std::max(1.0, std::min(t, 1.0e9));
}

// Whether gemm_dma_kernel centres its operands.  Centring costs a few vector
// ops per operand element on every sub-chunk; a fold costs a reduction of
// every accumulator (TM^2/64 per lane).  Centre only when, uncentred, the
// folds would come often enough to cost more.
static bool dma_centre(int64_t p, int64_t K, int tm, int waves, int sk) {
    const int32_t t = fold_chunks(p, false, K, waves, sk);
    if (t == 0)
        return false;
    const double fold_ops = 12.0 * (double)(tm * tm / 64);
    const double centre_ops = 4.0 * (double)(2 * (tm / 16) * (sk / 4));
    return fold_ops / (double)t > centre_ops;
}


// Fold period: the largest number of K-tiles t with
// t*16*m^2 + 2p < 2^53 where m bounds |operand| (p-1, or (p-1)/2 centred).
static int32_t fold_tiles(int64_t p, bool centre, int64_t K) {
    const double mx = centre ? (double)((p - 1) / 2 + 1) : (double)(p - 1);
    const double lim = 9007199254740992.0 - 4.0 * (double)p;
    const double per_tile = 16.0 * mx * mx;
    const double t = std::floor(lim / std::max(per_tile, 1.0));
    if (t * 16.0 >= (double)K + 16.0)
        return 0;  // the whole inner dimension fits: fold only at the end
    return (int32_t)std::max(1.0, std::min(t, 1.0e9));
}

// Kinds of binary64 base-product kernels (TILE_* in kernels.hpp).  A kind
// is admissible for a product when the kernel's shape and alignment
// assumptions hold; the default choice is a fixed rule by tile counts, and a
// kind measured faster for the shape (wsmul_tune_tiles) or pinned by the
// caller (wsmul_set_tile) replaces it when admissible.
static bool dma_aligned(const GemmParams &P) {
    return P.lda % 2 == 0 && P.ldb % 2 == 0 && aligned16(P.A) && aligned16(P.B);
}

static bool tile_admissible(int kind, const GemmParams &P) {
    switch (kind) {
    case TILE_BIG128:
        return WS_BIG_ENABLE && P.M % 128 == 0 && P.N % 128 == 0 && P.K % 16 == 0 && P.K > 0 &&
               dma_aligned(P);
    // The split kernels deal whole sub-chunks of the inner dimension to their
    // waves (some waves get one fewer): K only has to be a multiple of the
    // sub-chunk depth.
    case TILE_DMA64:
        return P.M % 64 == 0 && P.N % 64 == 0 && P.K % WS_DMA64_SK == 0 && P.K > 0 &&
               dma_aligned(P);
    case TILE_DMA32:
        return P.M % 32 == 0 && P.N % 32 == 0 && P.K % WS_DMA_SK == 0 && P.K > 0 &&
               dma_aligned(P);
    case TILE_DMA16:
        return P.M % 16 == 0 && P.N % 16 == 0 && P.K % 16 == 0 && P.K > 0 && dma_aligned(P);
    case TILE_LDS128:
    case TILE_LDS64:
    case TILE_SK32:
        return true;
    default:
        return false;
    }
}

static int default_tile(const GemmParams &P) {
    if (P.K == 0)
        return TILE_SK32;   // C <- beta*C only
    const int64_t big = ((P.M + 127) / 128) * ((P.N + 127) / 128);
    const int64_t mid = ((P.M + 63) / 64) * ((P.N + 63) / 64);
    // Whole 128 x 128 tiles: the pipelined kernel, unless its last round of
    // workgroups (one per CU) would be so partial that the 64 x 64 direct
    // kernel (also one per CU, four times the workgroups) finishes first; a
    // 64 x 64 round measured 0.26 of a 128 x 128 one.
    // (Every shape the pipelined kernel takes, the direct one takes too.)
    if (tile_admissible(TILE_BIG128, P) && mid >= 256 &&
        std::ceil((double)big / 256.0) <= 0.26 * std::ceil((double)mid / 256.0))
        return TILE_BIG128;
    if (big >= 512 && !tile_admissible(TILE_DMA64, P)) {
        // Register-staged tiles for large products of other shapes: 128 x 128
        // tiles (two workgroups per CU) cover an area about 4% faster than
        // 64 x 64 tiles (four per CU), but a partial last round of workgroups
        // costs a whole round, so compare rounds (a 64 x 64 round measured
        // 0.52 of a 128 x 128 one).
        const double r128 = std::ceil((double)big / 512.0);
        const double r64 = 0.52 * std::ceil((double)mid / 1024.0);
        if (r128 <= r64)
            return TILE_LDS128;
    }
    const int64_t small = ((P.M + 31) / 32) * ((P.N + 31) / 32);
    const int64_t tiny = ((P.M + 15) / 16) * ((P.N + 15) / 16);
    // Direct 32 x 32 tiles, or 16 x 16 ones: for at most three quarters of
    // the CUs' worth of 32 x 32 tiles the 16 x 16 kernel spreads the product
    // over four times as many workgroups (measured faster up to 128 such
    // tiles, slower at 225); beyond that compare rounds (five 16 x 16
    // workgroups per CU, a round measured 1.1 to 1.36 of a 32 x 32 one).
    auto direct32 = [&]() {
        if (tile_admissible(TILE_DMA16, P) &&
            (small <= 192 ||
             1.25 * std::ceil((double)tiny / 1280.0) <= std::ceil((double)small / 256.0)))
            return (int)TILE_DMA16;
        return (int)TILE_DMA32;
    };
    // Direct 64 x 64 or 32 x 32 tiles (one workgroup per CU either way): the
    // same round count, a 32 x 32 round measured 0.29 of a 64 x 64 one.
    if (mid >= 256 && tile_admissible(TILE_DMA64, P)) {
        if (tile_admissible(TILE_DMA32, P) &&
            std::ceil((double)mid / 256.0) > 0.29 * std::ceil((double)small / 256.0))
            return direct32();
        return TILE_DMA64;
    }
    if (mid >= 256)
        return TILE_LDS64;
    if (tile_admissible(TILE_DMA32, P))
        return direct32();
    if (small <= 192 && tile_admissible(TILE_DMA16, P))
        return TILE_DMA16;
    return TILE_SK32;
}

template <typename T>
static hipError_t launch_tile(int kind, GemmParams &P, bool vec2, hipStream_t s) {
    const bool centre = fold_tiles((int64_t)P.p, false, P.K) != 0;
    P.kc_tiles = fold_tiles((int64_t)P.p, centre, P.K);
    P.half = std::floor(P.p / 2.0);
    switch (kind) {
    case TILE_BIG128: {
        // Centre only when uncentred folds (a reduction of 32 accumulators
        // per lane) would cost more than centring 24 operands per K-step.
        const int32_t t_nc = fold_chunks((int64_t)P.p, false, P.K, 1, 16);
        const bool c2 = t_nc != 0 && 12.0 * 32.0 / (double)t_nc > 4.0 * 24.0;
        P.kc_tiles = fold_chunks((int64_t)P.p, c2, P.K, 1, 16);
        P.tiles_m = (int32_t)(P.M / 128);
        P.tiles_n = (int32_t)(P.N / 128);
        const dim3 grid((uint32_t)(P.tiles_m * P.tiles_n)), block(512);
        if (c2) ws_launch((gemm_big_kernel<T, true>), grid, block, 0, s, P);
        else ws_launch((gemm_big_kernel<T, false>), grid, block, 0, s, P);
        break;
    }
    case TILE_LDS128: {
        P.tiles_m = (int32_t)((P.M + 127) / 128);
        P.tiles_n = (int32_t)((P.N + 127) / 128);
        const dim3 grid((uint32_t)(P.tiles_m * P.tiles_n)), block(256);
        if (centre) {
            if (vec2) ws_launch((gemm_lds_kernel<T, 128, 128, true, true>), grid, block, 0, s, P);
            else ws_launch((gemm_lds_kernel<T, 128, 128, true, false>), grid, block, 0, s, P);
        } else {
            if (vec2) ws_launch((gemm_lds_kernel<T, 128, 128, false, true>), grid, block, 0, s, P);
            else ws_launch((gemm_lds_kernel<T, 128, 128, false, false>), grid, block, 0, s, P);
        }
        break;
    }
    case TILE_DMA64: {
        constexpr int W = WS_DMA64_WAVES, ST = WS_DMA64_STAGES, SK = WS_DMA64_SK;
        const bool c2 = dma_centre((int64_t)P.p, P.K, 64, W, SK);
        P.kc_tiles = fold_chunks((int64_t)P.p, c2, P.K, W, SK);
        P.tiles_m = (int32_t)(P.M / 64);
        P.tiles_n = (int32_t)(P.N / 64);
        const dim3 grid((uint32_t)(P.tiles_m * P.tiles_n)), block(64 * W);
        if (c2) ws_launch((gemm_dma_kernel<T, true, 64, W, ST, SK>), grid, block, 0, s, P);
        else ws_launch((gemm_dma_kernel<T, false, 64, W, ST, SK>), grid, block, 0, s, P);
        break;
    }
    case TILE_LDS64: {
        P.tiles_m = (int32_t)((P.M + 63) / 64);
        P.tiles_n = (int32_t)((P.N + 63) / 64);
        const dim3 grid((uint32_t)(P.tiles_m * P.tiles_n)), block(256);
        if (centre) {
            if (vec2) ws_launch((gemm_lds_kernel<T, 64, 64, true, true>), grid, block, 0, s, P);
            else ws_launch((gemm_lds_kernel<T, 64, 64, true, false>), grid, block, 0, s, P);
        } else {
            if (vec2) ws_launch((gemm_lds_kernel<T, 64, 64, false, true>), grid, block, 0, s, P);
            else ws_launch((gemm_lds_kernel<T, 64, 64, false, false>), grid, block, 0, s, P);
        }
        break;
    }
    case TILE_DMA32: {
        constexpr int W = WS_DMA_WAVES, ST = WS_DMA_STAGES, SK = WS_DMA_SK;
        const bool c2 = dma_centre((int64_t)P.p, P.K, 32, W, SK);
        P.kc_tiles = fold_chunks((int64_t)P.p, c2, P.K, W, SK);
        P.tiles_m = (int32_t)(P.M / 32);
        P.tiles_n = (int32_t)(P.N / 32);
        const dim3 grid((uint32_t)(P.tiles_m * P.tiles_n)), block(64 * W);
        if (c2) ws_launch((gemm_dma_kernel<T, true, 32, W, ST, SK>), grid, block, 0, s, P);
        else ws_launch((gemm_dma_kernel<T, false, 32, W, ST, SK>), grid, block, 0, s, P);
        break;
    }
    case TILE_DMA16: {
        constexpr int W = WS_DMA16_WAVES, ST = WS_DMA16_STAGES, SK = 16;
        const bool c2 = dma_centre((int64_t)P.p, P.K, 16, W, SK);
        P.kc_tiles = fold_chunks((int64_t)P.p, c2, P.K, W, SK);
        P.tiles_m = (int32_t)(P.M / 16);
        P.tiles_n = (int32_t)(P.N / 16);
        const dim3 grid((uint32_t)(P.tiles_m * P.tiles_n)), block(64 * W);
        if (c2) ws_launch((gemm_dma_kernel<T, true, 16, W, ST, SK>), grid, block, 0, s, P);
        else ws_launch((gemm_dma_kernel<T, false, 16, W, ST, SK>), grid, block, 0, s, P);
        break;
    }
    default: {
        P.tiles_m = (int32_t)((P.M + 31) / 32);
        P.tiles_n = (int32_t)((P.N + 31) / 32);
        const dim3 grid((uint32_t)(P.tiles_m * P.tiles_n)), block(64 * WS_SK_WAVES);
        const bool v4 = vec2 && (P.K % 4 == 0);
        if (centre) {
            if (v4) ws_launch((gemm_sk_kernel<T, true, true, WS_SK_WAVES>), grid, block, 0, s, P);
            else ws_launch((gemm_sk_kernel<T, true, false, WS_SK_WAVES>), grid, block, 0, s, P);
        } else {
            if (v4) ws_launch((gemm_sk_kernel<T, false, true, WS_SK_WAVES>), grid, block, 0, s, P);
            else ws_launch((gemm_sk_kernel<T, false, false, WS_SK_WAVES>), grid, block, 0, s, P);
        }
    }
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_gemm_t(GemmParams &P, bool vec2, hipStream_t s, int dtype) {
    int kind = default_tile(P);
    const int chosen = chosen_tile(P.M, P.N, P.K, (int64_t)P.p, dtype);
    if (chosen >= 0 && P.K > 0 && tile_admissible(chosen, P))
        kind = chosen;
    return launch_tile<T>(kind, P, vec2, s);
}

// ------------------------------------------------------- tile choices
namespace {
using TileKey = std::tuple<int64_t, int64_t, int64_t, int64_t, int>;
std::mutex g_tile_mu;
std::map<TileKey, int> g_tiles;
std::atomic<bool> g_tiles_any{false};
}  // namespace

int chosen_tile(int64_t M, int64_t N, int64_t K, int64_t p, int dtype) {
    if (!g_tiles_any.load(std::memory_order_acquire))
        return -1;
    std::lock_guard<std::mutex> lock(g_tile_mu);
    auto it = g_tiles.find(TileKey{M, N, K, p, dtype});
    return it == g_tiles.end() ? -1 : it->second;
}

void choose_tile(int64_t M, int64_t N, int64_t K, int64_t p, int dtype, int kind) {
    std::lock_guard<std::mutex> lock(g_tile_mu);
    if (kind < 0)
        g_tiles.erase(TileKey{M, N, K, p, dtype});
    else
        g_tiles[TileKey{M, N, K, p, dtype}] = kind;
    g_tiles_any.store(!g_tiles.empty(), std::memory_order_release);
}

template <typename T>
static hipError_t time_tiles_t(const GemmParams &base, bool vec2, int reps, hipStream_t s,
                               double *us) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess)
        e = hipEventCreate(&e1);
    for (int kind = 0; kind < TILE_KINDS && e == hipSuccess; ++kind) {
        if (!tile_admissible(kind, base))
            continue;
        GemmParams P = base;
        e = launch_tile<T>(kind, P, vec2, s);            // warm-up
        if (e == hipSuccess)
            e = hipEventRecord(e0, s);
        for (int r = 0; r < reps && e == hipSuccess; ++r) {
            P = base;
            e = launch_tile<T>(kind, P, vec2, s);
        }
        if (e == hipSuccess)
            e = hipEventRecord(e1, s);
        if (e == hipSuccess)
            e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess)
            us[kind] = 1000.0 * (double)ms / (double)reps;
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    return e;
}

hipError_t time_tiles(int64_t M, int64_t N, int64_t K, int64_t p, int dtype, int reps,
                      double *us) {
    for (int k = 0; k < TILE_KINDS; ++k)
        us[k] = -1.0;
    const size_t esz = 8;
    void *A = nullptr, *B = nullptr, *C = nullptr;
    hipStream_t s = nullptr;
    hipError_t e = hipMalloc(&A, std::max<size_t>(1, (size_t)(M * K) * esz));
    if (e == hipSuccess)
        e = hipMalloc(&B, std::max<size_t>(1, (size_t)(K * N) * esz));
    if (e == hipSuccess)
        e = hipMalloc(&C, std::max<size_t>(1, (size_t)(M * N) * esz));
    if (e == hipSuccess)   // zeros are residues in both storage types
        e = hipMemset(A, 0, (size_t)(M * K) * esz);
    if (e == hipSuccess)
        e = hipMemset(B, 0, (size_t)(K * N) * esz);
    if (e == hipSuccess)
        e = hipStreamCreate(&s);
    if (e == hipSuccess) {
        GemmParams P{};
        P.A = A;
        P.B = B;
        P.lda = K;
        P.ldb = N;
        P.M = M;
        P.N = N;
        P.K = K;
        P.p = (double)p;
        P.pinv = 1.0 / (double)p;
        P.alpha = 1.0;
        P.nin = 1;
        P.nout = 1;
        P.eout[0] = C;
        P.eldo[0] = N;
        P.coef[0][0] = 1.0;
        const bool vec2 = K % 2 == 0 && N % 2 == 0;
        e = dtype == WS_I64 ? time_tiles_t<int64_t>(P, vec2, std::max(reps, 1), s, us)
                            : time_tiles_t<double>(P, vec2, std::max(reps, 1), s, us);
    }
    if (s)
        (void)hipStreamSynchronize(s), (void)hipStreamDestroy(s);
    (void)hipFree(A);
    (void)hipFree(B);
    (void)hipFree(C);
    return e;
}

hipError_t launch_gemm(const ws_op_desc &op, const DevBufs &bufs, int dtype, int64_t p,
                       hipStream_t stream) {
    const int64_t M = op.a.rows, K = op.a.cols, N = op.b.cols;
    if (M == 0 || N == 0)
        return hipSuccess;
    const size_t esz = 8;
    GemmParams P{};
    P.A = static_cast<const char *>(bufs.ptr[op.a.buf]) + op.a.off * esz;
    P.B = static_cast<const char *>(bufs.ptr[op.b.buf]) + op.b.off * esz;
    P.lda = op.a.ld;
    P.ldb = op.b.ld;
    P.M = M;
    P.N = N;
    P.K = K;
    P.p = (double)p;
    P.pinv = 1.0 / (double)p;
    P.alpha = (double)op.alpha;
    P.nin = op.nin;
    P.nout = op.nout;
    for (int i = 1; i < op.nin; ++i) {
        P.ein[i] = static_cast<const char *>(bufs.ptr[op.in[i].buf]) + op.in[i].off * esz;
        P.eldi[i] = op.in[i].ld;
    }
    for (int o = 0; o < op.nout; ++o) {
        P.eout[o] = static_cast<char *>(bufs.ptr[op.out[o].buf]) + op.out[o].off * esz;
        P.eldo[o] = op.out[o].ld;
        for (int i = 0; i < op.nin; ++i)
            P.coef[o][i] = (double)op.coef[o][i];
    }
    const bool vec2 = (K % 2 == 0) && (N % 2 == 0) && (P.lda % 2 == 0) && (P.ldb % 2 == 0) &&
                      aligned16(P.A) && aligned16(P.B);
    if ((M + 31) / 32 * ((N + 31) / 32) >= (int64_t(1) << 31))
        return hipErrorInvalidValue;
    return dtype == WS_I64 ? launch_gemm_t<int64_t>(P, vec2, stream, dtype)
                           : launch_gemm_t<double>(P, vec2, stream, dtype);
}

}  // namespace wsmul

namespace wsmul {

// ============================================================ range check
template <typename T>
__global__ __launch_bounds__(256) void range_check_kernel(const T *ptr, int64_t rows,
                                                          int64_t cols, int64_t ld, double p,
                                                          int *flag) {
    const int64_t total = rows * cols;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * 256) {
        const int64_t r = idx / cols, c = idx % cols;
        const T raw = ptr[r * ld + c];
        bool bad;
        if constexpr (sizeof(T) == 8 && T(0.5) != T(0)) {
            const double x = (double)raw;
            bad = !(x >= 0.0 && x < p && x == floor(x));
        } else {
            bad = raw < 0 || (double)raw >= p;
        }
        if (bad)
            *flag = 1;
    }
}

hipError_t launch_range_check(const void *ptr, int64_t rows, int64_t cols, int64_t ld,
                              int dtype, int64_t p, int *flag, hipStream_t stream) {
    if (rows == 0 || cols == 0)
        return hipSuccess;
    const int64_t total = rows * cols;
    const uint32_t blocks = (uint32_t)std::min<int64_t>((total + 255) / 256, 4096);
    if (dtype == WS_I64)
        ws_launch(range_check_kernel<int64_t>, dim3(blocks), dim3(256), 0, stream,
                  static_cast<const int64_t *>(ptr), rows, cols, ld, (double)p, flag);
    else
        ws_launch(range_check_kernel<double>, dim3(blocks), dim3(256), 0, stream,
                  static_cast<const double *>(ptr), rows, cols, ld, (double)p, flag);
    return hipGetLastError();
}

}  // namespace wsmul

namespace wsmul {

// ================================================================= batched
// Persistent launch over many independent products.  The host groups the
// operations of all products into phases -- phase j holds the j-th operation
// of every product that has one -- so that the operations of a phase never
// depend on each other; phases are ordered by the stream (one launch each,
// all captured in one graph).  Each operation is cut into tasks: one 64 x 64
// output tile of a base product or one chunk of an addition group.  The
// workgroups of a launch walk the phase's task list round-robin (task w,
// w + G, w + 2G, ... for workgroup w of G): no atomics and no waiting, every
// workgroup ends after its last task.

// Addition group of a batch op: elements [chunk*BATCH_CHUNK, ...) of the
// M x N views, inputs ein[0..nin), outputs eout[0..nout).
__device__ void batch_add_chunk(const GemmParams &P, int64_t chunk) {
    const int64_t total = P.M * P.N;
    const int64_t base = chunk * BATCH_CHUNK;
#pragma unroll
    for (int u = 0; u < BATCH_CHUNK / 256; ++u) {
        const int64_t e = base + threadIdx.x + 256 * u;
        if (e >= total)
            break;
        const int64_t r = e / P.N, c = e % P.N;
        double x[WS_MAX_IN];
#pragma unroll
        for (int i = 0; i < WS_MAX_IN; ++i)
            if (i < P.nin)
                x[i] = static_cast<const double *>(P.ein[i])[r * P.eldi[i] + c];
#pragma unroll
        for (int o = 0; o < WS_MAX_OUT; ++o) {
            if (o >= P.nout)
                break;
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < WS_MAX_IN; ++i)
                if (i < P.nin)
                    s = fma(P.coef[o][i], x[i], s);
            static_cast<double *>(P.eout[o])[r * P.eldo[o] + c] = mod_reduce(s, P.p, P.pinv);
        }
    }
}

// Base products run as 64 x 64 tiles here: with many products in flight the
// launch is throughput-bound, and the smaller tile keeps register use low
// enough for several workgroups per CU.  Two register stages of operand
// loads, held to three waves per SIMD (three workgroups per CU).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void batch_kernel(const BatchOp *ops, const int2 *tasks,
                                                    int64_t ntasks) {
    __shared__ LdsTile<64, 64> sh;
    // Records and tasks do not change during the launch: read them through
    // the constant address space, so that the parameters are fetched by
    // scalar loads into scalar registers instead of every lane's registers.
    typedef const __attribute__((address_space(4))) BatchOp ConstOp;
    typedef const __attribute__((address_space(4))) int ConstInt;
    ConstOp *cops = (ConstOp *)ops;
    ConstInt *ctasks = (ConstInt *)tasks;
    for (int64_t q = blockIdx.x; q < ntasks; q += gridDim.x) {
        const int2 t = make_int2(ctasks[2 * q], ctasks[2 * q + 1]);
        const BatchOp &op = *(const BatchOp *)&cops[t.x];
        if (op.kind == WS_OP_GEMM) {
            const int32_t tm = t.y / op.g.tiles_n, tn = t.y % op.g.tiles_n;
            if (op.centre) {
                if (op.vec2) gemm_lds_tile<double, 64, 64, true, true, 2>(op.g, tm, tn, sh.As, sh.Bs);
                else gemm_lds_tile<double, 64, 64, true, false, 2>(op.g, tm, tn, sh.As, sh.Bs);
            } else {
                if (op.vec2) gemm_lds_tile<double, 64, 64, false, true, 2>(op.g, tm, tn, sh.As, sh.Bs);
                else gemm_lds_tile<double, 64, 64, false, false, 2>(op.g, tm, tn, sh.As, sh.Bs);
            }
        } else {
            batch_add_chunk(op.g, t.y);
        }
        __syncthreads();   // LDS is reused by the next task
    }
}

int batch_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel, 256, 0) != hipSuccess || n < 1)
        n = 2;
    return n;
}

hipError_t launch_batch(const BatchOp *ops, const int2 *tasks, int64_t ntasks, int grid,
                        hipStream_t stream) {
    if (ntasks == 0)
        return hipSuccess;
    const int g = (int)std::min<int64_t>(grid, ntasks);
    ws_launch(batch_kernel, dim3(g), dim3(256), 0, stream, ops, tasks, ntasks);
    return hipGetLastError();
}

// Host helper: fill the GemmParams of one batch op from a plan operation.
void fill_batch_op(BatchOp &b, const ws_op_desc &op, const DevBufs &bufs, int64_t p) {
    std::memset(&b, 0, sizeof(b));
    GemmParams &P = b.g;
    const size_t esz = 8;
    P.p = (double)p;
    P.pinv = 1.0 / (double)p;
    P.half = std::floor((double)p / 2.0);
    P.nin = op.nin;
    P.nout = op.nout;
    b.kind = op.kind;
    const int first = op.kind == WS_OP_GEMM ? 1 : 0;
    for (int i = first; i < op.nin; ++i) {
        P.ein[i] = static_cast<const char *>(bufs.ptr[op.in[i].buf]) + op.in[i].off * esz;
        P.eldi[i] = op.in[i].ld;
    }
    for (int o = 0; o < op.nout; ++o) {
        P.eout[o] = static_cast<char *>(bufs.ptr[op.out[o].buf]) + op.out[o].off * esz;
        P.eldo[o] = op.out[o].ld;
        for (int i = 0; i < op.nin; ++i)
            P.coef[o][i] = (double)op.coef[o][i];
    }
    if (op.kind == WS_OP_GEMM) {
        P.A = static_cast<const char *>(bufs.ptr[op.a.buf]) + op.a.off * esz;
        P.B = static_cast<const char *>(bufs.ptr[op.b.buf]) + op.b.off * esz;
        P.lda = op.a.ld;
        P.ldb = op.b.ld;
        P.M = op.a.rows;
        P.K = op.a.cols;
        P.N = op.b.cols;
        P.alpha = (double)op.alpha;
        const bool centre = fold_tiles(p, false, P.K) != 0;
        P.kc_tiles = fold_tiles(p, centre, P.K);
        b.centre = centre;
        b.vec2 = (P.K % 2 == 0) && (P.N % 2 == 0) && (P.lda % 2 == 0) && (P.ldb % 2 == 0) &&
                 aligned16(P.A) && aligned16(P.B);
        b.tile = 64;
        P.tiles_m = (int32_t)((P.M + b.tile - 1) / b.tile);
        P.tiles_n = (int32_t)((P.N + b.tile - 1) / b.tile);
        b.ntiles = P.tiles_m * P.tiles_n;
    } else {
        P.M = op.out[0].rows;
        P.N = op.out[0].cols;
        b.ntiles = (int32_t)((P.M * P.N + BATCH_CHUNK - 1) / BATCH_CHUNK);
    }
}

}  // namespace wsmul
