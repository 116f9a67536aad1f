// Base products from signed 8-bit digits of centred residues on the INT8
// matrix cores (v_mfma_i32_16x16x64_i8).
//
// A residue x in [0, p) is centred (c = x - p when x > h) and written in
// balanced base 256: c = d0 + 2^8 d1 + 2^16 d2 with every digit in
// [-128, 127] (enough for p <= 16,711,423; h = (p-1)/2).  For p <= 65536 the
// threshold is h = 32639, so that c lies in [-32896, 32639], where d2 = 0:
// two digits, and the product needs four digit products instead of nine.
// The product becomes
//     A*B = sum_{w=0..4} 2^(8w) * sum_{i+j=w} A_i * B_j,
// where every digit product is exact in int32: a weight class holds at most
// three digit products of magnitude <= K * 2^14, below 2^31 for K <= 32768.
// The epilogue folds the five classes into two exact binary64 sums, reduces
// them mod p, recombines, applies alpha and runs the fused addition rows.
//
// Digits are first written to a scratch area as three int8 planes per
// operand, each R x Kp with the inner dimension contiguous (B transposed),
// rows padded to the 128-row tile and Kp to the 64-wide K-step with zeros.
// A plane is stored tile by tile in the order the product consumes it: the
// 128 x 64 block of row-tile i and K-step t is 8 KB at ((i * Kp/64) + t) * 8K,
// rows of 64 bytes, with the 16-byte chunks of each row XOR-swizzled exactly
// as the product's LDS tiles are, so that every load copies contiguous bytes.
#include "gemm_common.hpp"
#include "wsmul_internal.hpp"

namespace wsmul {

bool limbs_supported(int64_t p) { return p <= 16711423; }

int digit_count(int64_t p) { return p <= 65536 ? 2 : 3; }

double digit_threshold(int64_t p) { return p <= 65536 ? 32639.0 : std::floor((double)p / 2.0); }

namespace {

constexpr int TILE = 128;     // output tile per workgroup (both dimensions)
constexpr int KSTEP = 64;     // inner dimension per matrix-core op

int64_t round_up(int64_t x, int64_t q) { return (x + q - 1) / q * q; }

// Byte offset of digit (r, k) in a tiled plane of Kp columns.
__device__ __forceinline__ int64_t tiled_pos(int64_t r, int64_t k, int64_t Kp) {
    const int64_t rt = r / TILE, kt = k / KSTEP;
    const int rr = (int)(r % TILE), kk = (int)(k % KSTEP);
    const int chunk = (kk >> 4) ^ ((rr >> 2) & 3);
    return (rt * (Kp / KSTEP) + kt) * (TILE * KSTEP) + rr * KSTEP + chunk * 16 + (kk & 15);
}

__device__ __forceinline__ void digits3(double x, double p, double half, int8_t &d0, int8_t &d1,
                                        int8_t &d2) {
    const int32_t c = (int32_t)(x > half ? x - p : x);
    const int32_t e0 = ((c + 128) & 255) - 128;
    const int32_t c1 = (c - e0) >> 8;
    const int32_t e1 = ((c1 + 128) & 255) - 128;
    const int32_t c2 = (c1 - e1) >> 8;
    d0 = (int8_t)e0;
    d1 = (int8_t)e1;
    d2 = (int8_t)c2;
}

// A (R x K, row-major) -> tiled planes of digits (r, k).  One workgroup per
// 128 x 64 block (row-tile, K-step): rows are read whole (32 lanes x 16
// bytes per row), the digits assembled in LDS in the tile's swizzled order,
// and each plane's 8 KB block written out contiguously.
template <typename T>
__global__ __launch_bounds__(256) void split_rows_kernel(const T *X, int64_t ld, int64_t R,
                                                         int64_t K, int64_t Rp, int64_t Kp,
                                                         int8_t *planes, double p, double half,
                                                         int vec2) {
    __shared__ __attribute__((aligned(16))) int8_t tile[3][TILE * KSTEP];
    const int64_t ksteps = Kp / KSTEP;
    const int64_t rt = (int64_t)blockIdx.x / ksteps, kt = (int64_t)blockIdx.x % ksteps;
    const int tid = threadIdx.x;
    const int kk = 2 * (tid & 31);
    const int64_t k = kt * KSTEP + kk;
#pragma unroll 4
    for (int j = 0; j < TILE / 8; ++j) {
        const int rr = (tid >> 5) + 8 * j;
        const int64_t r = rt * TILE + rr;
        double x0 = 0.0, x1 = 0.0;
        if (r < R) {
            const T *row = X + r * ld;
            if (vec2 && k + 1 < K) {
                load2(row + k, x0, x1);
            } else {
                x0 = k < K ? to_f64(row[k]) : 0.0;
                x1 = k + 1 < K ? to_f64(row[k + 1]) : 0.0;
            }
        }
        int8_t a0, a1, a2, b0, b1, b2;
        digits3(x0, p, half, a0, a1, a2);
        digits3(x1, p, half, b0, b1, b2);
        const int at = rr * KSTEP + 16 * ((kk >> 4) ^ ((rr >> 2) & 3)) + (kk & 15);
        tile[0][at] = a0;
        tile[0][at + 1] = b0;
        tile[1][at] = a1;
        tile[1][at + 1] = b1;
        tile[2][at] = a2;
        tile[2][at + 1] = b2;
    }
    __syncthreads();
    const int64_t plane = Rp * Kp;
    int8_t *dst = planes + (rt * ksteps + kt) * (TILE * KSTEP);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const int e = tid + 256 * q;                 // 16-byte piece e of 3 x 512
        const int d = e / 512, off = (e % 512) * 16;
        *reinterpret_cast<uint4 *>(dst + d * plane + off) =
            *reinterpret_cast<const uint4 *>(&tile[d][off]);
    }
}

// B (K x N, row-major) -> tiled planes of digits (n, k), transposed through
// LDS in 64 x 64 tiles so that both the reads and the writes are contiguous.
template <typename T>
__global__ __launch_bounds__(256) void split_cols_kernel(const T *X, int64_t ld, int64_t K,
                                                         int64_t N, int64_t Np, int64_t Kp,
                                                         int8_t *planes, double p, double half) {
    __shared__ __attribute__((aligned(16))) int8_t tile[3][64][64 + 16];
    const int64_t k0 = (int64_t)blockIdx.x * 64, n0 = (int64_t)blockIdx.y * 64;
    const int tid = threadIdx.x;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int e = tid + 256 * t;
        const int kk = e / 64, nn = e % 64;
        const int64_t k = k0 + kk, n = n0 + nn;
        const double x = (k < K && n < N) ? to_f64(X[k * ld + n]) : 0.0;
        int8_t d0, d1, d2;
        digits3(x, p, half, d0, d1, d2);
        tile[0][nn][kk] = d0;
        tile[1][nn][kk] = d1;
        tile[2][nn][kk] = d2;
    }
    __syncthreads();
    const int64_t plane = Np * Kp;
    // 3 digits x 64 rows x 64 bytes = 768 chunks of 16 bytes.
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const int q = tid + 256 * t;
        const int d = q / 256, nn = (q % 256) / 4, part = q % 4;
        const int64_t n = n0 + nn;
        if (n < Np && k0 + 16 * part < Kp) {
            const uint4 v = *reinterpret_cast<const uint4 *>(&tile[d][nn][16 * part]);
            *reinterpret_cast<uint4 *>(planes + d * plane + tiled_pos(n, k0 + 16 * part, Kp)) = v;
        }
    }
}

// ---- Addition rows on digit planes.  A temporary that only feeds base
// products (and the next addition rows) may be kept as the three digit
// planes the product consumes instead of as residues: the A-role layout of
// the tiled planes above (R x K, K inner), or the B-role one (a K x N block
// stored as N x K).  This kernel runs one addition group of at most four
// inputs and four outputs, each a residue view or digit planes, on 64 x 64
// tiles: every input tile is read (and decoded) into LDS as residues first,
// so outputs may overwrite inputs; then every output tile is formed and
// written (encoded).  Digit tiles of 64 inner indices are one K-step of the
// tiled layout, so every access is a contiguous 16-byte chunk.
__device__ __forceinline__ int32_t undigit(int8_t d0, int8_t d1, int8_t d2, int32_t p) {
    const int32_t c = (int32_t)d0 + 256 * (int32_t)d1 + 65536 * (int32_t)d2;
    return c < 0 ? c + p : c;
}

template <typename T>
__global__ __launch_bounds__(256) void lin_digits_kernel(LinDigitsParams L) {
    // nin tiles of 64 x 65 int32 (dynamic: fewer inputs, more workgroups per CU)
    extern __shared__ int32_t lin_lds[];
    auto val = reinterpret_cast<int32_t(*)[64][65]>(lin_lds);
    const int64_t r0 = (int64_t)(blockIdx.x / L.tiles_c) * 64;
    const int64_t c0 = (int64_t)(blockIdx.x % L.tiles_c) * 64;
    const int tid = threadIdx.x;
    const int32_t pi = (int32_t)L.p;
    // Chunk q (16 bytes) of row `row` of the 64-wide K-step block `kt` of a
    // plane tiled by 128-row tiles.
    auto chunk_at = [&](const DigitIO &io, int64_t row, int64_t kt, int q) {
        const int64_t rt = row / TILE;
        const int rr = (int)(row % TILE);
        return ((rt * (io.ld / KSTEP) + kt) * (TILE * KSTEP)) + rr * KSTEP + 16 * q;
    };
    for (int i = 0; i < L.nin; ++i) {
        const DigitIO &io = L.in[i];
        if (io.kind == 0) {
            const T *X = static_cast<const T *>(io.ptr);
            const int cc = tid & 63;
#pragma unroll 4
            for (int j = 0; j < 16; ++j) {
                const int rr = (tid >> 6) + 4 * j;
                val[i][rr][cc] = (int32_t)to_f64(X[(r0 + rr) * io.ld + c0 + cc]);
            }
        } else {
            // A-role: row r0+a of the plane, inner block c0/64.  B-role: row
            // c0+a of the (transposed) plane, inner block r0/64.
            const int a = tid >> 2, q = tid & 3;
            const bool arole = io.kind == 1;
            const int64_t row = arole ? r0 + a : c0 + a;
            const int64_t off = chunk_at(io, row, (arole ? c0 : r0) / KSTEP, q);
            const int8_t *b = static_cast<const int8_t *>(io.ptr) + off;
            union {
                uint4 u;
                int8_t d[16];
            } x0, x1, x2;
            x0.u = *reinterpret_cast<const uint4 *>(b);
            x1.u = *reinterpret_cast<const uint4 *>(b + io.plane);
            x2.u = *reinterpret_cast<const uint4 *>(b + 2 * io.plane);
            const int lc = q ^ (((int)(row % TILE) >> 2) & 3);     // logical chunk
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int32_t v = undigit(x0.d[e], x1.d[e], x2.d[e], pi);
                if (arole)
                    val[i][a][16 * lc + e] = v;
                else
                    val[i][16 * lc + e][a] = v;
            }
        }
    }
    __syncthreads();
    for (int o = 0; o < L.nout; ++o) {
        const DigitIO &io = L.out[o];
        if (io.kind == 0) {
            T *Y = static_cast<T *>(const_cast<void *>(io.ptr));
            const int cc = tid & 63;
#pragma unroll 4
            for (int j = 0; j < 16; ++j) {
                const int rr = (tid >> 6) + 4 * j;
                double sum = 0.0;
                for (int i = 0; i < L.nin; ++i)
                    sum = fma(L.coef[o][i], (double)val[i][rr][cc], sum);
                Y[(r0 + rr) * io.ld + c0 + cc] = from_f64<T>(mod_reduce(sum, L.p, L.pinv));
            }
        } else {
            const int a = tid >> 2, q = tid & 3;
            const bool arole = io.kind == 1;
            const int64_t row = arole ? r0 + a : c0 + a;
            const int64_t off = chunk_at(io, row, (arole ? c0 : r0) / KSTEP, q);
            const int lc = q ^ (((int)(row % TILE) >> 2) & 3);
            union {
                uint4 u;
                int8_t d[16];
            } y0, y1, y2;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                double sum = 0.0;
                for (int i = 0; i < L.nin; ++i)
                    sum = fma(L.coef[o][i],
                              (double)(arole ? val[i][a][16 * lc + e] : val[i][16 * lc + e][a]), sum);
                digits3(mod_reduce(sum, L.p, L.pinv), L.p, L.half, y0.d[e], y1.d[e], y2.d[e]);
            }
            int8_t *b = static_cast<int8_t *>(const_cast<void *>(io.ptr)) + off;
            *reinterpret_cast<uint4 *>(b) = y0.u;
            *reinterpret_cast<uint4 *>(b + io.plane) = y1.u;
            *reinterpret_cast<uint4 *>(b + 2 * io.plane) = y2.u;
        }
    }
}

// Addition groups whose digit-plane operands all have one role, and whose
// residue operands (if any) are in the A role: each thread takes one 16-byte
// chunk position of the tiled layout (16 consecutive inner indices of one
// plane row) in every operand, so nothing is transposed and no LDS is used.
// 512 consecutive threads cover one 128 x 64 block, 8 KB of every plane.
template <typename T, int NIN>
__global__ __launch_bounds__(256) void lin_chunks_kernel(LinDigitsParams L, int role) {
    const int64_t inner = role == 1 ? L.Cc : L.R;      // K-direction length of the planes
    const int64_t ksteps = inner / KSTEP;
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t blk = g / 512, within = g % 512;
    const int64_t pt = blk / ksteps, kt = blk % ksteps;
    const int rr = (int)(within / 4), slot = (int)(within % 4);
    const int64_t prow = pt * TILE + rr;                    // plane row (A: row, B: column)
    const int lc = slot ^ ((rr >> 2) & 3);                  // logical 16-wide chunk
    const int64_t col0 = kt * KSTEP + 16 * lc;              // first inner index of the chunk
    const int32_t pi = (int32_t)L.p;
    int32_t val[NIN][16];
#pragma unroll
    for (int i = 0; i < NIN; ++i) {
        const DigitIO &io = L.in[i];
        if (io.kind == 0) {                                 // A role: row prow, columns col0..
            const T *X = static_cast<const T *>(io.ptr) + prow * io.ld + col0;
#pragma unroll
            for (int e = 0; e < 16; ++e)
                val[i][e] = (int32_t)to_f64(X[e]);
        } else {
            const int8_t *b = static_cast<const int8_t *>(io.ptr) +
                              (pt * (io.ld / KSTEP) + kt) * (TILE * KSTEP) + within * 16;
            union {
                uint4 u;
                int8_t d[16];
            } x0, x1, x2;
            x0.u = *reinterpret_cast<const uint4 *>(b);
            x1.u = *reinterpret_cast<const uint4 *>(b + io.plane);
            x2.u = *reinterpret_cast<const uint4 *>(b + 2 * io.plane);
#pragma unroll
            for (int e = 0; e < 16; ++e)
                val[i][e] = undigit(x0.d[e], x1.d[e], x2.d[e], pi);
        }
    }
    for (int o = 0; o < L.nout; ++o) {
        const DigitIO &io = L.out[o];
        auto at = [&](int e) {
            double sum = 0.0;
#pragma unroll
            for (int i = 0; i < NIN; ++i)
                sum = fma(L.coef[o][i], (double)val[i][e], sum);
            return mod_reduce(sum, L.p, L.pinv);
        };
        if (io.kind == 0) {
            T *Y = static_cast<T *>(const_cast<void *>(io.ptr)) + prow * io.ld + col0;
#pragma unroll
            for (int e = 0; e < 16; ++e)
                Y[e] = from_f64<T>(at(e));
        } else {
            union {
                uint4 u;
                int8_t d[16];
            } y0, y1, y2;
#pragma unroll
            for (int e = 0; e < 16; ++e)
                digits3(at(e), L.p, L.half, y0.d[e], y1.d[e], y2.d[e]);
            int8_t *b = static_cast<int8_t *>(const_cast<void *>(io.ptr)) +
                        (pt * (io.ld / KSTEP) + kt) * (TILE * KSTEP) + within * 16;
            *reinterpret_cast<uint4 *>(b) = y0.u;
            *reinterpret_cast<uint4 *>(b + io.plane) = y1.u;
            *reinterpret_cast<uint4 *>(b + 2 * io.plane) = y2.u;
        }
    }
}

template <typename T>
void launch_chunks(const LinDigitsParams &P, int role, uint32_t blocks, hipStream_t stream) {
    switch (P.nin) {
    case 1: ws_launch(lin_chunks_kernel<T, 1>, dim3(blocks), dim3(256), 0, stream, P, role); break;
    case 2: ws_launch(lin_chunks_kernel<T, 2>, dim3(blocks), dim3(256), 0, stream, P, role); break;
    case 3: ws_launch(lin_chunks_kernel<T, 3>, dim3(blocks), dim3(256), 0, stream, P, role); break;
    default: ws_launch(lin_chunks_kernel<T, 4>, dim3(blocks), dim3(256), 0, stream, P, role); break;
    }
}

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

struct DigitParams {
    GemmParams g;              // shapes, modulus, alpha and the fused epilogue
    const int8_t *Ad;          // 3 planes; tile (row-tile i, K-step t) at (i * a_kstride + t) * 8 KB
    const int8_t *Bd;          // 3 planes, the same for B's column tiles
    int64_t Mp, Np, Kp;
    int64_t a_plane, b_plane;  // bytes from one digit's plane to the next
    int64_t a_kstride, b_kstride;  // K-steps per row of tiles in the planes read
    double c24;                // 2^24 mod p
};

// 128 x 128 output tile per workgroup, 2 x WN waves (wave tiles of 64 x
// 128/WN: with WN = 4 the five int32 accumulator sets, one per weight class,
// take 160 registers and two waves share each SIMD), digit tiles of 64 inner
// elements in STAGES LDS buffers filled by direct global-to-LDS loads issued
// STAGES-1 K-steps ahead (no staging registers).  A load instruction places
// lane l's 16 bytes at base + 16*l; the planes are tiled and swizzled so that
// each instruction copies 1 KB of contiguous bytes, and within a 64-byte row
// the 16-byte chunk c of row r sits at slot c ^ ((r >> 2) & 3), so the 16
// lanes reading one chunk of 16 consecutive rows hit 16 distinct slots of the
// 256 LDS bytes they span.
#ifndef WS_I8_WN
#define WS_I8_WN 4
#endif
#ifndef WS_I8_STAGES
#define WS_I8_STAGES 2
#endif
template <typename T, int WN, int STAGES, int ND>
__global__ __launch_bounds__(128 * WN) void gemm_digits_kernel(DigitParams D) {
    constexpr int PLANE = TILE * KSTEP;                     // bytes of one digit tile
    constexpr int WAVES = 2 * WN, NT = 64 * WAVES;
    constexpr int WCOLS = TILE / WN, JB = WCOLS / 16;       // wave tile columns, 16-column blocks
    constexpr int LPW = 16 * ND / WAVES;                    // load instructions per wave and K-step
    static_assert(STAGES == 2 || STAGES == 3, "two or three buffers");
    static_assert(ND == 2 || ND == 3, "two or three digits");
    static_assert(16 * ND % WAVES == 0 && (LPW == 4 || LPW == 6 || LPW == 12),
                  "whole load instructions per wave");
    // [stage][A|B][digit], sized for three buffers whatever STAGES is: with a
    // template-dependent extent the host compiler drops the kernel's launch
    // stub without a diagnostic.
    __shared__ __attribute__((aligned(16))) int8_t lds[3][2][3][PLANE];
    const GemmParams &P = D.g;
    int32_t tm, tn;
    tile_of(P.tiles_m, P.tiles_n, tm, tn);
    const int64_t m0 = (int64_t)tm * TILE, n0 = (int64_t)tn * TILE;
    const int tid = threadIdx.x, lane = tid & 63;
    // The wave index is uniform: read it into a scalar register so that the
    // load addresses are scalar bases plus the lane's offset (22 fewer
    // vector registers, 1% faster at 16384^3).
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WN, wn = wave % WN;
    const int li = lane & 15, g = lane >> 4;
    const int64_t plA = D.a_plane, plB = D.b_plane;

    // 48 load instructions per K-step (2 operands x 3 digits x 8 blocks of
    // 16 rows), LPW per wave.  The planes are tiled (one contiguous, already
    // swizzled 8 KB block per row-tile and K-step), so instruction blk of a
    // block copies its bytes blk*1024 .. blk*1024 + 1023 to the same LDS
    // offsets.
    const int64_t ksteps = D.Kp / KSTEP;
    auto issue = [&](int st, int64_t t) {
#pragma unroll
        for (int j = 0; j < LPW; ++j) {
            const int i = wave + WAVES * j;
            const int op = i / (8 * ND), d = (i % (8 * ND)) / 8, blk = i % 8;
            const int8_t *src = op == 0 ? D.Ad + d * plA + ((int64_t)tm * D.a_kstride + t) * PLANE
                                        : D.Bd + d * plB + ((int64_t)tn * D.b_kstride + t) * PLANE;
            __builtin_amdgcn_global_load_lds(src + blk * 1024 + 16 * lane, &lds[st][op][d][blk * 1024], 16, 0, 0);
        }
    };
    auto frag = [&](int st, int op, int d, int row) {
        return *reinterpret_cast<const i32x4 *>(
            &lds[st][op][d][row * KSTEP + 16 * (g ^ ((row >> 2) & 3))]);
    };

    i32x4 acc[5][4][JB];
#pragma unroll
    for (int w = 0; w < 5; ++w)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < JB; ++j)
                acc[w][i][j] = i32x4{0, 0, 0, 0};

    // A digit outer, B inner: the compiler reads each fragment once either
    // way, but this order of the 72 products measured 1.5-2% faster.
    auto compute = [&](int cur) {
#pragma unroll
        for (int a = 0; a < ND; ++a) {
            i32x4 af[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                af[i] = frag(cur, 0, a, wm * 64 + i * 16 + li);
#pragma unroll
            for (int b = 0; b < ND; ++b) {
                i32x4 bf[JB];
#pragma unroll
                for (int j = 0; j < JB; ++j)
                    bf[j] = frag(cur, 1, b, wn * WCOLS + j * 16 + li);
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < JB; ++j)
                        acc[a + b][i][j] =
                            __builtin_amdgcn_mfma_i32_16x16x64_i8(af[i], bf[j], acc[a + b][i][j], 0, 0, 0);
            }
        }
    };

    if (STAGES == 2) {
        if (ksteps > 0)
            issue(0, 0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        for (int64_t t = 0; t < ksteps; ++t) {
            const int cur = (int)(t & 1);
            if (t + 1 < ksteps)
                issue(cur ^ 1, t + 1);
            compute(cur);
            __builtin_amdgcn_s_waitcnt(0);   // this wave's loads of the next K-step have landed
            __syncthreads();
        }
    } else {
        if (ksteps > 0)
            issue(0, 0);
        if (ksteps > 1)
            issue(1, 1);
        for (int64_t t = 0; t < ksteps; ++t) {
            // This wave's loads of step t have landed (only step t+1's may
            // still be in flight), then every wave's, and every wave is done
            // with step t-1: a plain barrier with no fence, so that the loads
            // of step t+1 stay in flight across it.
            if (t + 1 < ksteps) {
                if (LPW == 4) asm volatile("s_waitcnt vmcnt(4)\n\ts_barrier" ::: "memory");
                else if (LPW == 6) asm volatile("s_waitcnt vmcnt(6)\n\ts_barrier" ::: "memory");
                else asm volatile("s_waitcnt vmcnt(12)\n\ts_barrier" ::: "memory");
            } else {
                asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
            }
            if (t + 2 < ksteps)
                issue((int)((t + 2) % 3), t + 2);
            compute((int)(t % 3));
        }
        __syncthreads();
    }

    // Recombine the weight classes into residues, apply alpha, stage the
    // whole 128 x 128 tile of residues in LDS (128 KB: the operand buffers
    // are free by now) and run the fused epilogue on whole rows.  Output
    // layout of the 16 x 16 x 64 int8 op: lane l, element v holds row
    // 4*(l/16) + v of column l % 16.
    // With |class| < 2^31, t = c0 + 2^8 c1 + 2^16 c2 (< 2^48) and
    // u = c3 + 2^8 c4 (< 2^40) are exact in binary64, and the product is
    // t + 2^24 u: two reductions, a multiply-add by 2^24 mod p, and a third.
    static_assert(sizeof(lds) >= TILE * TILE * sizeof(double), "tile stage fits the buffers");
    double *stage = reinterpret_cast<double *>(&lds[0][0][0][0]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < JB; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double t = fma(65536.0, (double)acc[2][i][j][v],
                                     fma(256.0, (double)acc[1][i][j][v], (double)acc[0][i][j][v]));
                const double u = fma(256.0, (double)acc[4][i][j][v], (double)acc[3][i][j][v]);
                const double s = fma(D.c24, mod_reduce(u, P.p, P.pinv), mod_reduce(t, P.p, P.pinv));
                const int r = wm * 64 + i * 16 + 4 * g + v;
                stage[r * TILE + wn * WCOLS + j * 16 + li] = product_residue(P, s);
            }
    __syncthreads();
    for (int e = tid; e < TILE * TILE; e += NT) {
        const int r = e / TILE, c = e % TILE;
        const int64_t row = m0 + r, col = n0 + c;
        if (row < P.M && col < P.N)
            epilogue_apply<T>(P, stage[e], row, col);
    }
}

}  // namespace

size_t digit_scratch_bytes(int64_t M, int64_t N, int64_t K) {
    const int64_t Kp = round_up(std::max<int64_t>(K, 1), KSTEP);
    return (size_t)(3 * (round_up(M, TILE) + round_up(N, TILE)) * Kp);
}

hipError_t launch_lin_digits(const LinDigitsParams &L, int dtype, hipStream_t stream) {
    if (L.R <= 0 || L.Cc <= 0)
        return hipSuccess;
    if (L.R % 64 || L.Cc % 64 || L.nin < 1 || L.nin > LD_MAX || L.nout < 1 || L.nout > LD_MAX)
        return hipErrorInvalidValue;
    LinDigitsParams P = L;
    // One role among the digit operands, and residues only beside the A
    // role: the chunk kernel (no transposition) takes the group.
    int role = 0;
    bool residues = false, mixed = false;
    for (int i = 0; i < L.nin + L.nout; ++i) {
        const int kind = i < L.nin ? L.in[i].kind : L.out[i - L.nin].kind;
        if (kind == 0)
            residues = true;
        else if (role && role != kind)
            mixed = true;
        else
            role = kind;
    }
    const int64_t prows = role == 1 ? L.R : L.Cc, inner = role == 1 ? L.Cc : L.R;
    if (role && !mixed && !(residues && role != 1) && prows % TILE == 0 && inner % KSTEP == 0) {
        const uint32_t blocks = (uint32_t)(L.R * L.Cc / 16 / 256);
        if (dtype == WS_I64)
            launch_chunks<int64_t>(P, role, blocks, stream);
        else
            launch_chunks<double>(P, role, blocks, stream);
        return hipGetLastError();
    }
    P.tiles_c = (int32_t)(L.Cc / 64);
    const dim3 grid((uint32_t)((L.R / 64) * (L.Cc / 64)));
    const uint32_t lds = (uint32_t)(L.nin * 64 * 65 * sizeof(int32_t));
    if (dtype == WS_I64)
        ws_launch(lin_digits_kernel<int64_t>, grid, dim3(256), lds, stream, P);
    else
        ws_launch(lin_digits_kernel<double>, grid, dim3(256), lds, stream, P);
    return hipGetLastError();
}

hipError_t launch_split_rows(const void *X, int64_t ld, int64_t R, int64_t K, int8_t *planes,
                             int dtype, int64_t p, hipStream_t stream) {
    if (R <= 0)
        return hipSuccess;
    // K = 0 still writes one K-step of zero digits: the product reads it
    const int64_t Rp = round_up(R, TILE), Kp = round_up(std::max<int64_t>(K, 1), KSTEP);
    const double pd = (double)p, half = digit_threshold(p);
    const uint32_t blocks = (uint32_t)((Rp / TILE) * (Kp / KSTEP));
    const int vec2 = (ld % 2 == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0) ? 1 : 0;
    if (dtype == WS_I64)
        ws_launch(split_rows_kernel<int64_t>, dim3(blocks), dim3(256), 0, stream,
                  static_cast<const int64_t *>(X), ld, R, K, Rp, Kp, planes, pd, half, vec2);
    else
        ws_launch(split_rows_kernel<double>, dim3(blocks), dim3(256), 0, stream,
                  static_cast<const double *>(X), ld, R, K, Rp, Kp, planes, pd, half, vec2);
    return hipGetLastError();
}

hipError_t launch_split_cols(const void *X, int64_t ld, int64_t K, int64_t N, int8_t *planes,
                             int dtype, int64_t p, hipStream_t stream) {
    if (N <= 0)
        return hipSuccess;
    const int64_t Np = round_up(N, TILE), Kp = round_up(std::max<int64_t>(K, 1), KSTEP);
    const double pd = (double)p, half = digit_threshold(p);
    const dim3 grid((uint32_t)(Kp / 64), (uint32_t)(Np / 64));
    if (dtype == WS_I64)
        ws_launch(split_cols_kernel<int64_t>, grid, dim3(256), 0, stream,
                  static_cast<const int64_t *>(X), ld, K, N, Np, Kp, planes, pd, half);
    else
        ws_launch(split_cols_kernel<double>, grid, dim3(256), 0, stream,
                  static_cast<const double *>(X), ld, K, N, Np, Kp, planes, pd, half);
    return hipGetLastError();
}

hipError_t launch_gemm_limbs(const ws_op_desc &op, const DevBufs &bufs, int dtype, int64_t p,
                             hipStream_t stream, const PlaneRef *pa, const PlaneRef *pb) {
    const int64_t M = op.a.rows, K = op.a.cols, N = op.b.cols;
    if (M == 0 || N == 0)
        return hipSuccess;
    if (K > 32768 || !limbs_supported(p))
        return hipErrorInvalidValue;
    const size_t own = (pa ? 0 : 3 * (size_t)round_up(M, TILE) * round_up(std::max<int64_t>(K, 1), KSTEP)) +
                       (pb ? 0 : 3 * (size_t)round_up(N, TILE) * round_up(std::max<int64_t>(K, 1), KSTEP));
    if (own && (!bufs.scratch || bufs.scratch_bytes < bufs.split_offset + own))
        return hipErrorInvalidValue;
    const size_t esz = 8;
    DigitParams D{};
    GemmParams &P = D.g;
    P.M = M;
    P.N = N;
    P.K = K;
    P.p = (double)p;
    P.pinv = 1.0 / (double)p;
    P.half = std::floor((double)p / 2.0);
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
    D.Mp = round_up(M, TILE);
    D.Np = round_up(N, TILE);
    D.Kp = round_up(std::max<int64_t>(K, 1), KSTEP);
    // Operands already held as digit planes (whole tiles, so the padded
    // sizes are the sizes) are read where they are; the others are split
    // into the scratch area past bufs.split_offset.
    if ((pa && (M % TILE || K % KSTEP)) || (pb && (N % TILE || K % KSTEP)))
        return hipErrorInvalidValue;
    int8_t *own_a = static_cast<int8_t *>(bufs.scratch) + bufs.split_offset;
    int8_t *own_b = own_a + (pa ? 0 : 3 * D.Mp * D.Kp);
    D.Ad = pa ? pa->ptr : own_a;
    D.Bd = pb ? pb->ptr : own_b;
    D.a_plane = pa ? pa->plane : D.Mp * D.Kp;
    D.b_plane = pb ? pb->plane : D.Np * D.Kp;
    D.a_kstride = pa ? pa->kstride : D.Kp / KSTEP;
    D.b_kstride = pb ? pb->kstride : D.Kp / KSTEP;
    D.c24 = (double)((int64_t(1) << 24) % p);
    const void *Aop = static_cast<const char *>(bufs.ptr[op.a.buf]) + op.a.off * esz;
    const void *Bop = static_cast<const char *>(bufs.ptr[op.b.buf]) + op.b.off * esz;
    // Traced runs time the splits on their own event pair.
    const LaunchTiming timing = launch_timing();
    if (timing.split_start)
        launch_timing() = LaunchTiming{timing.split_start, timing.split_stop, false, nullptr, nullptr};
    hipError_t e = hipSuccess;
    if (!pa)
        e = launch_split_rows(Aop, op.a.ld, M, K, own_a, dtype, p, stream);
    if (e == hipSuccess && !pb)
        e = launch_split_cols(Bop, op.b.ld, K, N, own_b, dtype, p, stream);
    launch_timing() = timing;
    if (e != hipSuccess)
        return e;
    P.tiles_m = (int32_t)(D.Mp / TILE);
    P.tiles_n = (int32_t)(D.Np / TILE);
    constexpr int WN = WS_I8_WN, ST = WS_I8_STAGES;
    const dim3 grid((uint32_t)(P.tiles_m * P.tiles_n)), block(128 * WN);
    // Two digits load two thirds as much per K-step; there three buffers
    // (loads two steps ahead) measured 2% faster at 16384^3, with three
    // digits 8% slower.
    const bool two = digit_count(p) == 2;
    if (dtype == WS_I64) {
        if (two)
            ws_launch(gemm_digits_kernel<int64_t, WN, 3, 2>, grid, block, 0, stream, D);
        else
            ws_launch(gemm_digits_kernel<int64_t, WN, ST, 3>, grid, block, 0, stream, D);
    } else {
        if (two)
            ws_launch(gemm_digits_kernel<double, WN, 3, 2>, grid, block, 0, stream, D);
        else
            ws_launch(gemm_digits_kernel<double, WN, ST, 3>, grid, block, 0, stream, D);
    }
    return hipGetLastError();
}

}  // namespace wsmul
