// Declarations shared by the host-side translation units of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <string>

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
int run_plan(const Plan &plan, const ws_args &a, void *ws, hipStream_t stream, bool trace,
             void *scratch, size_t scratch_bytes);
int check_ranges(const ws_args &a, hipStream_t stream);

// Fill a.schedule / a.levels / a.base for WS_AUTO or levels < 0.
int autotune_choice(ws_args &a, bool beta_nonzero);

// Base products from signed 8-bit digits of centred residues.
bool limbs_supported(int64_t p);
size_t digit_scratch_bytes(int64_t M, int64_t N, int64_t K);
hipError_t launch_gemm_limbs(const ws_op_desc &op, const DevBufs &bufs, int dtype, int64_t p,
                             hipStream_t stream);

}  // namespace wsmul
