// Declarations shared by the host-side translation units of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"
#include "wsmul.h"

namespace wsmul {

void set_error(const std::string &msg);
void set_stats(const ws_stats &s);
void set_batch_phases(uint64_t n);
hipStream_t default_stream();
void attached_workspace(void **ptr, size_t *bytes);
// Estimated time (microseconds) of a plan under a base kind.
double plan_cost_us(const Plan &plan, int base);
std::shared_ptr<Plan> get_plan(const PlanKey &key);
int prepare(const ws_args *in, ws_args &a, PlanKey &key, Resolved &res);
int execute(const ws_args &a, const PlanKey &key);
struct DigitExec;
int run_plan(const Plan &plan, const ws_args &a, void *ws, hipStream_t stream, bool trace,
             void *scratch, size_t scratch_bytes, const DigitExec *dexec);
int check_ranges(const ws_args &a, hipStream_t stream);

// Fill a.schedule / a.levels / a.base for WS_AUTO or levels < 0.
int autotune_choice(ws_args &a, bool beta_nonzero);

// Base products from signed 8-bit digits of centred residues.
bool limbs_supported(int64_t p);
// Digits per residue (2 for p <= 65536, else 3) and the centring threshold
// (residues above it are taken minus p) that keeps the top digit in range.
int digit_count(int64_t p);
double digit_threshold(int64_t p);
size_t digit_scratch_bytes(int64_t M, int64_t N, int64_t K);
// Digit planes an operand is read from instead of being split: tile
// (row-tile i, K-step t) of digit d at ptr + d * plane + (i * kstride + t) * 8 KB.
struct PlaneRef {
    const int8_t *ptr;
    int64_t plane, kstride;
};
// pa / pb: that operand is already held as digit planes (whole tiles), so it
// is not split; the others are split into bufs.scratch past split_offset.
hipError_t launch_gemm_limbs(const ws_op_desc &op, const DevBufs &bufs, int dtype, int64_t p,
                             hipStream_t stream, const PlaneRef *pa = nullptr,
                             const PlaneRef *pb = nullptr);
// Digit planes of a whole R x K matrix in the A-operand layout, or of a whole
// K x N matrix in the B-operand layout (rows padded to 128, K to 64).
hipError_t launch_split_rows(const void *X, int64_t ld, int64_t R, int64_t K, int8_t *planes,
                             int dtype, int64_t p, hipStream_t stream);
hipError_t launch_split_cols(const void *X, int64_t ld, int64_t K, int64_t N, int8_t *planes,
                             int dtype, int64_t p, hipStream_t stream);

// One addition group on residue views and digit planes (see limbs.hip).
constexpr int LD_MAX = 4;
struct DigitIO {
    int32_t kind;          // 0 residues (storage type), 1 A-role planes, 2 B-role planes
    int32_t pad;
    const void *ptr;       // element (0, 0) of the view, or plane 0 of the digits
    int64_t ld;            // residues: leading dimension; digits: inner length of the planes
    int64_t plane;         // digits: bytes per plane
};
struct LinDigitsParams {
    DigitIO in[LD_MAX], out[LD_MAX];
    int32_t nin, nout, tiles_c, pad;
    int64_t R, Cc;         // rows and columns of the group's views (multiples of 64)
    double p, pinv, half;
    double coef[LD_MAX][LD_MAX];
};
hipError_t launch_lin_digits(const LinDigitsParams &L, int dtype, hipStream_t stream);

// An operation of a plan as the digit base runs it: which inputs and
// outputs of an addition group are digit planes (0 residues, 1 A-role,
// 2 B-role) and which operands of a base product already are.  A view of A
// or B with a form is read from the planes of the whole input, split once
// at the start of the call.
struct ExecOp {
    OpDesc op;
    int8_t in_enc[WS_MAX_IN];
    int8_t out_enc[WS_MAX_OUT];
    bool pre_a, pre_b;
};
struct DigitExec {
    std::vector<ExecOp> ops;
    bool split_a = false, split_b = false;  // whole A (B) split into planes first
    int64_t a_rows = 0, a_kp = 0;           // padded sizes of those planes
    int64_t b_cols = 0, b_kp = 0;
    size_t input_bytes = 0;                 // scratch bytes of the input planes
    size_t split_bytes = 0;                 // largest own split of a base product
};
// The digit base's execution list of a plan (digit_temps.cpp), built once.
std::shared_ptr<const DigitExec> digit_exec(const Plan &plan);
bool exec_uses_digits(const ExecOp &e);
hipError_t launch_exec_add(const DigitExec &x, const ExecOp &e, const DevBufs &bufs, int dtype,
                           int64_t p, hipStream_t stream);
hipError_t launch_exec_gemm(const DigitExec &x, const ExecOp &e, const DevBufs &bufs, int dtype,
                            int64_t p, hipStream_t stream);
// Split the whole inputs the list reads as planes (start of a call).
hipError_t launch_input_splits(const DigitExec &x, const DevBufs &bufs, int64_t lda, int64_t ldb,
                               int64_t m, int64_t k, int64_t n, int dtype, int64_t p,
                               hipStream_t stream);

}  // namespace wsmul
