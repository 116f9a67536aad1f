// Host-side launchers of the device kernels.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "gemm_common.hpp"
#include "wsmul.h"

namespace wsmul {

// Kernel timing of traced runs.  While `start`/`stop` are set, the launches
// of this thread stamp `start` when the first kernel begins and `stop` when
// the last one ends: the dispatch records them, so the interval is the
// kernels' own execution time, as a kernel-trace profiler reports it.
// The digit base times its operand splits apart from its product: while
// `split_start`/`split_stop` are set, the split launches stamp those instead.
struct LaunchTiming {
    hipEvent_t start = nullptr, stop = nullptr;
    bool started = false;
    hipEvent_t split_start = nullptr, split_stop = nullptr;
};
LaunchTiming &launch_timing();

template <typename F, typename... Args>
inline void ws_launch(F kernel, const dim3 &grid, const dim3 &block, uint32_t shmem, hipStream_t s,
                      Args... args) {
    LaunchTiming &t = launch_timing();
    hipEvent_t first = nullptr;
    if (t.start && !t.started) {
        first = t.start;
        t.started = true;
    }
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, first, t.stop, 0u, args...);
}

// Base pointers of the four buffers a plan refers to (WS_BUF_A .. WS_BUF_W).
struct DevBufs {
    void *ptr[4];
    void *scratch;          // digit planes of the INT8 base (WS_BASE_I8_LIMBS)
    size_t scratch_bytes;
    size_t split_offset = 0;  // where a base product's own splits go in scratch
};

// One fused group of addition rows (elementwise, HBM-bound).
hipError_t launch_add(const ws_op_desc &op, const DevBufs &bufs, int dtype, int64_t p,
                      hipStream_t stream);

// Kinds of binary64 base-product kernels (the values of WS_TILE_* in the
// header): 128 x 128 tiles pipelined through LDS by direct loads, or staged
// through registers; 64 x 64 tiles by direct loads with split inner
// dimension, or register-staged; 32 x 32 tiles by direct loads with split
// inner dimension, or straight from global memory; 16 x 16 tiles by direct
// loads with split inner dimension.
enum : int {
    TILE_BIG128 = 0, TILE_LDS128 = 1, TILE_DMA64 = 2, TILE_LDS64 = 3, TILE_DMA32 = 4,
    TILE_SK32 = 5, TILE_DMA16 = 6, TILE_KINDS = 7
};
// Kind chosen for products of this shape and modulus (measured or pinned),
// or -1 for the default rule.  choose_tile with kind -1 forgets the choice.
int chosen_tile(int64_t M, int64_t N, int64_t K, int64_t p, int dtype);
void choose_tile(int64_t M, int64_t N, int64_t K, int64_t p, int dtype, int kind);
// Time every admissible kind on a dense M x K by K x N product mod p on the
// current device (us[kind] in microseconds, -1 when not admissible).
hipError_t time_tiles(int64_t M, int64_t N, int64_t K, int64_t p, int dtype, int reps, double *us);

// One base product with its epilogue group (binary64 matrix cores).
hipError_t launch_gemm(const ws_op_desc &op, const DevBufs &bufs, int dtype, int64_t p,
                       hipStream_t stream);

// Sets *flag to 1 if some entry of the rows x cols view is not an integer in
// [0, p).  The flag must be cleared by the caller beforehand.
hipError_t launch_range_check(const void *ptr, int64_t rows, int64_t cols, int64_t ld,
                              int dtype, int64_t p, int *flag, hipStream_t stream);

// One operation of a product in a batched launch (see launch_batch).
constexpr int BATCH_CHUNK = 256 * 8;   // elements per addition task
struct BatchOp {
    GemmParams g;    // base product, or addition group (inputs ein[0..nin), M x N views)
    int32_t kind;    // WS_OP_ADD or WS_OP_GEMM
    int32_t tile;    // base product: 64
    int32_t centre, vec2;
    int32_t ntiles;  // tasks of this operation
    int32_t phase;   // position of the operation in its product's plan
};

void fill_batch_op(BatchOp &b, const ws_op_desc &op, const DevBufs &bufs, int64_t p);

// Resident workgroups of the batch kernel per CU (its persistent grid is
// this many per CU).
int batch_blocks_per_cu();

// One persistent launch over the independent tasks of one phase: workgroup w
// of `grid` runs tasks w, w + grid, ...
hipError_t launch_batch(const BatchOp *ops, const int2 *tasks, int64_t ntasks, int grid,
                        hipStream_t stream);

}  // namespace wsmul
