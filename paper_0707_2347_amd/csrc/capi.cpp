// The C-ABI: argument checks, plan cache, workspace, launch loop, counters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"
#include "wsmul.h"
#include "wsmul_internal.hpp"

using namespace wsmul;

namespace {

thread_local std::string g_err;
thread_local ws_stats g_stats{};
thread_local ws_trace g_trace{};

std::mutex g_mu;
void *g_ws = nullptr;
size_t g_ws_bytes = 0;
std::atomic<hipStream_t> g_stream{nullptr};   // set and read from any thread
// Device bytes the single-product calls hold at the moment (workspace and
// digit scratch they allocated and have not yet released, stream-ordered).
std::atomic<uint64_t> g_live_bytes{0};

struct KeyHash {
    size_t operator()(const PlanKey &k) const {
        const int64_t v[] = {k.m, k.k, k.n, k.p, k.lda, k.ldb, k.ldc, k.alpha, k.beta,
                             k.dtype, k.table, k.levels, k.fuse, k.blocks};
        uint64_t h = 1469598103934665603ull;
        for (int64_t x : v) {
            h ^= (uint64_t)x;
            h *= 1099511628211ull;
        }
        return (size_t)h;
    }
};
std::unordered_map<PlanKey, std::shared_ptr<Plan>, KeyHash> g_plans;
size_t g_plan_ops = 0;   // operations held by the cached plans (about 1 KB each)
constexpr size_t PLAN_CACHE_PLANS = 512, PLAN_CACHE_OPS = size_t(1) << 20;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int64_t canon(int64_t x, int64_t p) {
    const int64_t r = x % p;
    return r < 0 ? r + p : r;
}

}  // namespace

namespace wsmul {

void set_error(const std::string &msg) { g_err = msg; }

void set_stats(const ws_stats &s) {
    const uint64_t peak = std::max<uint64_t>(g_stats.peak_temp_bytes, s.workspace_bytes);
    g_stats = s;
    g_stats.peak_temp_bytes = peak;
}

hipStream_t default_stream() { return g_stream.load(); }

void set_batch_phases(uint64_t n) { g_stats.batch_phases = n; }

void attached_workspace(void **ptr, size_t *bytes) {
    std::lock_guard<std::mutex> lock(g_mu);
    *ptr = g_ws;
    *bytes = g_ws_bytes;
}

std::shared_ptr<Plan> get_plan(const PlanKey &key) {
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end())
        return it->second;
    auto plan = std::make_shared<Plan>();
    build_plan(key, *plan);
    // Bounded cache: start over when it would hold too many plans or
    // operations (plans in use stay alive through their shared pointers).
    if (g_plans.size() >= PLAN_CACHE_PLANS || g_plan_ops + plan->ops.size() > PLAN_CACHE_OPS) {
        g_plans.clear();
        g_plan_ops = 0;
    }
    g_plans.emplace(key, plan);
    g_plan_ops += plan->ops.size();
    return plan;
}

// Normalise and check a request.  On success fills the plan key.
int prepare(const ws_args *in, ws_args &a, PlanKey &key, Resolved &res) {
    if (!in)
        return fail(WS_EINVAL, "null argument block");
    a = *in;
    if (a.m < 0 || a.k < 0 || a.n < 0)
        return fail(WS_EINVAL, "negative dimension");
    if (a.p < 2 || a.p >= (int64_t(1) << 24))
        return fail(WS_EMODULUS, "p must lie in [2, 2^24)");
    if (a.dtype != WS_F64 && a.dtype != WS_I64)
        return fail(WS_EINVAL, "dtype must be WS_F64 or WS_I64");
    if (a.lda == 0)
        a.lda = a.k;
    if (a.ldb == 0)
        a.ldb = a.n;
    if (a.ldc == 0)
        a.ldc = a.n;
    if (a.lda < a.k || a.ldb < a.n || a.ldc < a.n || a.lda < 0 || a.ldb < 0 || a.ldc < 0)
        return fail(WS_EINVAL, "leading dimension smaller than the row length");
    if ((a.m > 0 && a.k > 0 && !a.A) || (a.k > 0 && a.n > 0 && !a.B) ||
        (a.m > 0 && a.n > 0 && !a.C))
        return fail(WS_EINVAL, "null matrix pointer");
    if (a.base != WS_BASE_AUTO && a.base != WS_BASE_F64_MFMA && a.base != WS_BASE_I8_LIMBS)
        return fail(WS_EINVAL, "unknown base kind");
    const bool beta_nz = canon(a.beta, a.p) != 0;
    if (a.blocks == 0 && a.schedule != WS_ROWS)
        a.blocks = 2;
    if (a.schedule == WS_ROWS && a.levels < 0)
        return fail(WS_EINVAL, "a row schedule needs levels >= 0");
    if (a.schedule != WS_ROWS && (a.schedule == WS_AUTO || a.levels < 0 || a.base == WS_BASE_AUTO)) {
        const int rc = autotune_choice(a, beta_nz);
        if (rc != WS_OK)
            return rc;
    }
    if (a.base == WS_BASE_AUTO)
        a.base = WS_BASE_F64_MFMA;
    if (a.base == WS_BASE_I8_LIMBS && !limbs_supported(a.p))
        return fail(WS_EMODULUS, "p too large for three signed 8-bit digits (p <= 16711423)");
    if (a.base == WS_BASE_I8_LIMBS && a.k > 32768)
        return fail(WS_ESHAPE, "the 8-bit digit base needs k <= 32768 (exact int32 sums)");
    res = resolve_schedule(a.schedule, a.m, a.k, a.n, beta_nz, a.levels,
                           (int)std::min<uint32_t>(a.blocks, 1u << 20));
    if (res.status != WS_OK)
        return fail(res.status, res.error);
    std::memset(&key, 0, sizeof(key));
    key.m = a.m;
    key.k = a.k;
    key.n = a.n;
    key.p = a.p;
    key.lda = a.lda;
    key.ldb = a.ldb;
    key.ldc = a.ldc;
    key.alpha = canon(a.alpha, a.p);
    key.beta = canon(a.beta, a.p);
    key.dtype = a.dtype;
    key.table = res.table;
    key.levels = res.levels;
    key.fuse = (a.flags & WS_FLAG_NOFUSE) ? 0 : 1;
    key.blocks = (res.table == TAB_BLOCKED_HL || res.table == TAB_BLOCKED_ACC ||
                  res.table == TAB_ROWS) ? (int32_t)a.blocks : 0;
    if (res.table == TAB_ROWS && !rows_registered(key.blocks))
        return fail(WS_ESCHEDULE, "WS_ROWS runs a schedule registered by wsmul_mod_p_rows");
    return WS_OK;
}

static void fill_stats(const Plan &plan, const ws_args &a, ws_stats &s) {
    s.workspace_bytes = (uint64_t)plan.ws_elems * 8u;
    s.add_launches = (uint64_t)plan.add_ops;
    s.gemm_launches = (uint64_t)plan.gemm_ops;
    s.element_additions = (uint64_t)plan.element_additions;
    s.base_flops = (uint64_t)plan.base_flops;
    s.rows = (uint64_t)plan.rows;
    s.levels = (uint64_t)plan.key.levels;
    s.schedule = plan.key.table;
    s.base = a.base;
}

// One addition group.  The elementwise kernel indexes fewer than 2^31 items
// per launch, so groups over blocks of 2^31 elements or more (quadrants of a
// C of 2^33 entries, which fits the device when k is small) run as slices of
// whole rows: the same group on fewer rows, one launch each.
static hipError_t launch_add_rows(const OpDesc &op, const DevBufs &bufs, int dtype, int64_t p,
                                  hipStream_t stream) {
    const int64_t rows = op.out[0].rows, cols = op.out[0].cols;
    const int64_t limit = (int64_t(1) << 31) - 1;
    const int64_t per = std::max<int64_t>(1, limit / std::max<int64_t>(cols, 1));
    if (rows <= per)
        return launch_add(op, bufs, dtype, p, stream);
    hipError_t err = hipSuccess;
    for (int64_t r0 = 0; r0 < rows && err == hipSuccess; r0 += per) {
        OpDesc s = op;
        const int64_t nr = std::min(per, rows - r0);
        for (int i = 0; i < s.nin; ++i) {
            s.in[i].off += r0 * s.in[i].ld;
            s.in[i].rows = nr;
        }
        for (int o = 0; o < s.nout; ++o) {
            s.out[o].off += r0 * s.out[o].ld;
            s.out[o].rows = nr;
        }
        err = launch_add(s, bufs, dtype, p, stream);
    }
    return err;
}

// The digit base runs a plan's execution list (temporaries that only feed
// base products and addition groups stay digit planes, inputs may be read
// from planes of the whole input) when the workspace is 16-byte aligned.
std::shared_ptr<const DigitExec> exec_list(const Plan &plan, const ws_args &a, const void *ws) {
    if (a.base != WS_BASE_I8_LIMBS || !ws || reinterpret_cast<uintptr_t>(ws) % 16 != 0)
        return nullptr;
    return digit_exec(plan);
}

// Digit scratch of one call: the input planes and the largest split of a
// base product (execution list), or the largest base product's splits.
size_t digit_scratch_need(const Plan &plan, const ws_args &a, const DigitExec *x) {
    if (a.base != WS_BASE_I8_LIMBS)
        return 0;
    if (x)
        return x->input_bytes + x->split_bytes;
    size_t bytes = 0;
    for (const OpDesc &op : plan.ops)
        if (op.kind == WS_OP_GEMM)
            bytes = std::max(bytes, digit_scratch_bytes(op.a.rows, op.b.cols, op.a.cols));
    return bytes;
}

// Launch every operation of a plan on `stream`.
int run_plan(const Plan &plan, const ws_args &a, void *ws, hipStream_t stream, bool trace,
             void *scratch, size_t scratch_bytes, const DigitExec *dexec) {
    DevBufs bufs{{a.A, a.B, a.C, ws}, scratch, scratch_bytes};
    if (dexec && scratch_bytes < dexec->input_bytes + dexec->split_bytes)
        return fail(WS_EINVAL, "digit scratch smaller than the execution list needs");
    // Traced runs: a start/stop event pair per operation, stamped by the
    // kernel dispatches themselves.
    // The digit base gets a second pair per operation for its splits, and
    // one more pair for the splits of whole inputs.
    const size_t per_op = a.base == WS_BASE_I8_LIMBS ? 4 : 2;
    const size_t nops = dexec ? dexec->ops.size() : plan.ops.size();
    auto op_at = [&](size_t i) -> const OpDesc & { return dexec ? dexec->ops[i].op : plan.ops[i]; };
    std::vector<hipEvent_t> ev;
    if (trace) {
        ev.assign(per_op * nops + 2, nullptr);
        for (auto &e : ev)
            if (hipEventCreate(&e) != hipSuccess) {
                for (auto &d : ev)
                    if (d)
                        (void)hipEventDestroy(d);
                return fail(WS_EHIP, "hipEventCreate failed");
            }
    }
    // Host-side failure injection for tests of the error path: with
    // WSMUL_FAULT_AT=i the call stops before launching operation i and
    // reports WS_EHIP, as if that launch had failed.
    long fault_at = -1;
    if (const char *f = std::getenv("WSMUL_FAULT_AT"))
        fault_at = std::strtol(f, nullptr, 10);
    int rc = WS_OK;
    const bool input_splits = dexec && (dexec->split_a || dexec->split_b);
    if (input_splits) {
        if (trace)
            launch_timing() = LaunchTiming{ev[per_op * nops], ev[per_op * nops + 1], false};
        const hipError_t err = launch_input_splits(*dexec, bufs, a.lda, a.ldb, a.m, a.k, a.n,
                                                   a.dtype, a.p, stream);
        if (err != hipSuccess)
            rc = fail(WS_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(err));
    }
    for (size_t i = 0; i < nops && rc == WS_OK; ++i) {
        const OpDesc &op = op_at(i);
        if (fault_at >= 0 && (size_t)fault_at == i) {
            rc = fail(WS_EHIP, "injected failure before operation " + std::to_string(i) +
                                   " (WSMUL_FAULT_AT)");
            break;
        }
        if (trace)
            launch_timing() = per_op == 4 ? LaunchTiming{ev[4 * i], ev[4 * i + 1], false,
                                                         ev[4 * i + 2], ev[4 * i + 3]}
                                          : LaunchTiming{ev[2 * i], ev[2 * i + 1], false};
        hipError_t err;
        if (dexec)
            err = op.kind == WS_OP_ADD
                      ? (exec_uses_digits(dexec->ops[i])
                             ? launch_exec_add(*dexec, dexec->ops[i], bufs, a.dtype, a.p, stream)
                             : launch_add_rows(op, bufs, a.dtype, a.p, stream))
                      : launch_exec_gemm(*dexec, dexec->ops[i], bufs, a.dtype, a.p, stream);
        else if (op.kind == WS_OP_ADD)
            err = launch_add_rows(op, bufs, a.dtype, a.p, stream);
        else if (a.base == WS_BASE_I8_LIMBS)
            err = launch_gemm_limbs(op, bufs, a.dtype, a.p, stream);
        else
            err = launch_gemm(op, bufs, a.dtype, a.p, stream);
        if (err != hipSuccess)
            rc = fail(WS_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(err));
    }
    launch_timing() = LaunchTiming{};
    if (trace) {
        if (rc == WS_OK && hipStreamSynchronize(stream) != hipSuccess)
            rc = fail(WS_EHIP, "hipStreamSynchronize failed");
        if (rc == WS_OK && input_splits) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[per_op * nops], ev[per_op * nops + 1]) == hipSuccess) {
                const double Ka = (double)dexec->a_kp, Kb = (double)dexec->b_kp;
                g_trace.split_launches += (dexec->split_a ? 1 : 0) + (dexec->split_b ? 1 : 0);
                g_trace.split_ms += ms;
                g_trace.split_bytes += (dexec->split_a ? 8.0 * a.m * a.k + 3.0 * dexec->a_rows * Ka : 0.0) +
                                       (dexec->split_b ? 8.0 * a.k * a.n + 3.0 * dexec->b_cols * Kb : 0.0);
            }
        }
        for (size_t i = 0; i < nops && rc == WS_OK; ++i) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[per_op * i], ev[per_op * i + 1]) != hipSuccess)
                ms = 0.f;   // an operation with no kernel (empty view)
            const OpDesc &op = op_at(i);
            const bool pre_a = dexec && dexec->ops[i].pre_a, pre_b = dexec && dexec->ops[i].pre_b;
            g_trace.unsplit_operands += (pre_a ? 1 : 0) + (pre_b ? 1 : 0);
            if (dexec && op.kind == WS_OP_ADD && exec_uses_digits(dexec->ops[i]))
                g_trace.digit_adds += 1;
            if (per_op == 4 && op.kind == WS_OP_GEMM && !(pre_a && pre_b)) {
                float sms = 0.f;
                if (hipEventElapsedTime(&sms, ev[4 * i + 2], ev[4 * i + 3]) == hipSuccess) {
                    const double M = (double)op.a.rows, K = (double)op.a.cols, N = (double)op.b.cols;
                    const double Mp = std::ceil(M / 128) * 128, Np = std::ceil(N / 128) * 128,
                                 Kp = std::ceil(std::max(K, 1.0) / 64) * 64;
                    g_trace.split_launches += (pre_a ? 0 : 1) + (pre_b ? 0 : 1);
                    g_trace.split_ms += sms;
                    g_trace.split_bytes += (pre_a ? 0.0 : 8.0 * M * K + 3.0 * Mp * Kp) +
                                           (pre_b ? 0.0 : 8.0 * K * N + 3.0 * Np * Kp);
                }
            }
            if (op.kind == WS_OP_ADD) {
                // 8 bytes per residue entry, 3 per entry held as digit planes
                double per_entry = 0.0;
                for (int k = 0; k < op.nin; ++k)
                    per_entry += dexec && dexec->ops[i].in_enc[k] ? 3.0 : 8.0;
                for (int o = 0; o < op.nout; ++o)
                    per_entry += dexec && dexec->ops[i].out_enc[o] ? 3.0 : 8.0;
                g_trace.add_launches += 1;
                g_trace.add_ms += ms;
                g_trace.add_bytes += per_entry * (double)op.out[0].rows * (double)op.out[0].cols;
            } else {
                g_trace.gemm_launches += 1;
                g_trace.gemm_ms += ms;
                g_trace.gemm_flops += 2.0 * (double)op.a.rows * (double)op.a.cols * (double)op.b.cols;
            }
        }
        for (auto &e : ev)
            (void)hipEventDestroy(e);
    }
    return rc;
}

int execute(const ws_args &a, const PlanKey &key) {
    std::shared_ptr<Plan> plan;
    try {
        plan = get_plan(key);
    } catch (const std::exception &e) {
        return fail(WS_EINVAL, std::string("planner: ") + e.what());
    }
    hipStream_t stream = a.stream ? static_cast<hipStream_t>(a.stream) : g_stream.load();
    const size_t ws_bytes = (size_t)plan->ws_elems * 8u;
    void *ws = nullptr;
    bool owned = false;
    if (ws_bytes) {
        if (a.workspace) {
            if (a.workspace_bytes < ws_bytes)
                return fail(WS_ENOMEM, "attached workspace smaller than the schedule needs");
            ws = a.workspace;
        } else {
            std::lock_guard<std::mutex> lock(g_mu);
            if (g_ws && g_ws_bytes >= ws_bytes)
                ws = g_ws;
        }
        if (!ws) {
            if (hipMallocAsync(&ws, ws_bytes, stream) != hipSuccess)
                return fail(WS_ENOMEM, "workspace allocation failed");
            owned = true;
            g_live_bytes += ws_bytes;
        }
    }
    auto release_ws = [&]() {
        if (owned) {
            (void)hipFreeAsync(ws, stream);
            g_live_bytes -= ws_bytes;
        }
    };
    if (a.flags & WS_FLAG_CHECK) {
        const int rc = check_ranges(a, stream);
        if (rc != WS_OK) {
            release_ws();
            g_stats.live_alloc_bytes = g_live_bytes.load();
            return rc;
        }
    }
    // Digit planes for the INT8 base.
    std::shared_ptr<const DigitExec> dexec;
    try {
        dexec = exec_list(*plan, a, ws);
    } catch (const std::exception &e) {
        release_ws();
        g_stats.live_alloc_bytes = g_live_bytes.load();
        return fail(WS_ENOMEM, std::string("digit execution list: ") + e.what());
    }
    const size_t scratch_bytes = digit_scratch_need(*plan, a, dexec.get());
    void *scratch = nullptr;
    if (scratch_bytes) {
        if (hipMallocAsync(&scratch, scratch_bytes, stream) != hipSuccess) {
            release_ws();
            g_stats.live_alloc_bytes = g_live_bytes.load();
            return fail(WS_ENOMEM, "digit scratch allocation failed");
        }
        if (scratch)
            g_live_bytes += scratch_bytes;
    }
    const int rc = run_plan(*plan, a, ws, stream, (a.flags & WS_FLAG_TRACE) != 0, scratch,
                            scratch_bytes, dexec.get());
    if (scratch) {
        (void)hipFreeAsync(scratch, stream);
        g_live_bytes -= scratch_bytes;
    }
    release_ws();
    fill_stats(*plan, a, g_stats);
    g_stats.live_alloc_bytes = g_live_bytes.load();
    g_stats.internal_alloc_bytes = (owned ? ws_bytes : 0) + scratch_bytes;
    g_stats.scratch_bytes = scratch_bytes;
    if (g_stats.workspace_bytes > g_stats.peak_temp_bytes)
        g_stats.peak_temp_bytes = g_stats.workspace_bytes;
    return rc;
}

// Scratch of the no-allocation entry point: one file-scope device array per
// GPU, held from module load until the process ends.  Host code never uses
// the array's name as an address; it asks the runtime for the device address
// once per device and passes that pointer to the kernels.
static __device__ __align__(256) unsigned char scratch[WSMUL_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[64] = {nullptr};
}

// Device address of this GPU's scratch array (looked up on the first call
// made with the device current).
int noalloc_scratch(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return fail(WS_EHIP, "hipGetDevice failed");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(WS_EHIP, std::string("hipGetSymbolAddress of the static scratch failed: ") +
                                     hipGetErrorString(e));
        g_noalloc_ptr[dev] = ptr;
    }
    *out = g_noalloc_ptr[dev];
    return WS_OK;
}

// The plan of one product with its workspace and digit scratch carved from
// the static scratch: no device allocation, no synchronisation.
int execute_noalloc(const ws_args &a, const PlanKey &key) {
    std::shared_ptr<Plan> plan;
    try {
        plan = get_plan(key);
    } catch (const std::exception &e) {
        return fail(WS_EINVAL, std::string("planner: ") + e.what());
    }
    hipStream_t stream = a.stream ? static_cast<hipStream_t>(a.stream) : g_stream.load();
    const size_t ws_bytes = ((size_t)plan->ws_elems * 8u + 255) & ~size_t(255);
    void *base = nullptr;
    const int st = noalloc_scratch(&base);
    if (st != WS_OK)
        return st;
    unsigned char *b = static_cast<unsigned char *>(base);
    std::shared_ptr<const DigitExec> dexec;
    try {
        dexec = exec_list(*plan, a, ws_bytes ? b : nullptr);
    } catch (const std::exception &e) {
        return fail(WS_ENOMEM, std::string("digit execution list: ") + e.what());
    }
    const size_t scratch_bytes = digit_scratch_need(*plan, a, dexec.get());
    const size_t need = ws_bytes + scratch_bytes;
    if (need > (size_t)WSMUL_NOALLOC_SCRATCH_BYTES)
        return fail(WS_ENOMEM, "the product needs " + std::to_string(need) +
                                   " bytes of workspace and digit scratch; the static scratch of "
                                   "wsmul_mod_p_noalloc holds " +
                                   std::to_string((size_t)WSMUL_NOALLOC_SCRATCH_BYTES));
    const int rc = run_plan(*plan, a, ws_bytes ? b : nullptr, stream, false,
                            scratch_bytes ? b + ws_bytes : nullptr, scratch_bytes, dexec.get());
    fill_stats(*plan, a, g_stats);
    g_stats.internal_alloc_bytes = 0;
    g_stats.scratch_bytes = scratch_bytes;
    g_stats.live_alloc_bytes = g_live_bytes.load();
    if (g_stats.workspace_bytes > g_stats.peak_temp_bytes)
        g_stats.peak_temp_bytes = g_stats.workspace_bytes;
    return rc;
}

// WS_FLAG_CHECK: every entry of A, B (and C when beta != 0) in [0, p).
int check_ranges(const ws_args &a, hipStream_t stream) {
    static std::mutex mu;
    static int *flag_dev[64] = {nullptr};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return fail(WS_EHIP, "hipGetDevice failed");
    int *flag;
    {
        std::lock_guard<std::mutex> lock(mu);
        if (!flag_dev[dev] && hipMalloc(&flag_dev[dev], sizeof(int)) != hipSuccess)
            return fail(WS_EHIP, "hipMalloc of the check flag failed");
        flag = flag_dev[dev];
    }
    if (hipMemsetAsync(flag, 0, sizeof(int), stream) != hipSuccess)
        return fail(WS_EHIP, "hipMemsetAsync failed");
    hipError_t e = launch_range_check(a.A, a.m, a.k, a.lda, a.dtype, a.p, flag, stream);
    if (e == hipSuccess)
        e = launch_range_check(a.B, a.k, a.n, a.ldb, a.dtype, a.p, flag, stream);
    if (e == hipSuccess && canon(a.beta, a.p) != 0)
        e = launch_range_check(a.C, a.m, a.n, a.ldc, a.dtype, a.p, flag, stream);
    int host = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&host, flag, sizeof(int), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(stream);
    if (e != hipSuccess)
        return fail(WS_EHIP, std::string("range check failed: ") + hipGetErrorString(e));
    if (host)
        return fail(WS_ERANGE, "an entry of A, B or C is not a residue in [0, p)");
    return WS_OK;
}

}  // namespace wsmul

extern "C" {

int wsmul_mod_p_ex(const ws_args *args) {
    ws_args a;
    PlanKey key;
    Resolved res;
    int rc = prepare(args, a, key, res);
    if (rc != WS_OK)
        return rc;
    if (a.m == 0 || a.n == 0) {
        g_stats.workspace_bytes = 0;
        return WS_OK;
    }
    return execute(a, key);
}

int wsmul_register_rows(const ws_row *rows, int nrows, int ntemps, int *id) {
    if (!id)
        return fail(WS_EINVAL, "null id");
    std::string err;
    *id = register_rows(rows, nrows, ntemps, &err);
    if (*id == 0)
        return fail(WS_EINVAL, "row schedule: " + err);
    return WS_OK;
}

int wsmul_mod_p_rows(const ws_args *args, const ws_row *rows, int nrows, int ntemps) {
    if (!args)
        return fail(WS_EINVAL, "null argument block");
    std::string err;
    const int id = register_rows(rows, nrows, ntemps, &err);
    if (id == 0)
        return fail(WS_EINVAL, "row schedule: " + err);
    ws_args r = *args;
    r.schedule = WS_ROWS;
    r.blocks = (uint32_t)id;
    ws_args a;
    PlanKey key;
    Resolved res;
    int rc = prepare(&r, a, key, res);
    if (rc != WS_OK)
        return rc;
    if (a.m == 0 || a.n == 0) {
        g_stats.workspace_bytes = 0;
        return WS_OK;
    }
    return execute(a, key);
}

int wsmul_mod_p_noalloc(const ws_args *args) {
    if (args && (args->workspace || args->workspace_bytes))
        return fail(WS_EINVAL, "wsmul_mod_p_noalloc takes its workspace from its static scratch; "
                               "pass no workspace");
    if (args && (args->flags & (WS_FLAG_CHECK | WS_FLAG_TRACE)))
        return fail(WS_EINVAL, "wsmul_mod_p_noalloc takes no WS_FLAG_CHECK or WS_FLAG_TRACE");
    ws_args a;
    PlanKey key;
    Resolved res;
    int rc = prepare(args, a, key, res);
    if (rc != WS_OK)
        return rc;
    if (a.m == 0 || a.n == 0) {
        g_stats.workspace_bytes = 0;
        return WS_OK;
    }
    return execute_noalloc(a, key);
}

static int simple_call(int dtype, int64_t m, int64_t k, int64_t n, int64_t p, void *A, void *B,
                       void *C, int64_t alpha, int64_t beta, int schedule, int levels) {
    ws_args a;
    std::memset(&a, 0, sizeof(a));
    a.m = m;
    a.k = k;
    a.n = n;
    a.p = p;
    a.A = A;
    a.B = B;
    a.C = C;
    a.alpha = alpha;
    a.beta = beta;
    a.dtype = dtype;
    a.schedule = schedule;
    a.levels = levels;
    a.base = WS_BASE_F64_MFMA;
    return wsmul_mod_p_ex(&a);
}

int wsmul_mod_p(int64_t m, int64_t k, int64_t n, int64_t p, void *A, void *B, void *C,
                int64_t alpha, int64_t beta, int schedule, int levels) {
    return simple_call(WS_F64, m, k, n, p, A, B, C, alpha, beta, schedule, levels);
}

int wsmul_mod_p_i64(int64_t m, int64_t k, int64_t n, int64_t p, void *A, void *B, void *C,
                    int64_t alpha, int64_t beta, int schedule, int levels) {
    return simple_call(WS_I64, m, k, n, p, A, B, C, alpha, beta, schedule, levels);
}

size_t wsmul_workspace_bytes(int64_t m, int64_t k, int64_t n, int dtype, int schedule, int levels,
                             int beta_nonzero) {
    if (m < 0 || k < 0 || n < 0 || (dtype != WS_F64 && dtype != WS_I64)) {
        set_error("bad dimensions or dtype");
        return 0;
    }
    Resolved r = resolve_schedule(schedule, m, k, n, beta_nonzero != 0, levels);
    if (r.status != WS_OK) {
        set_error(r.error);
        return 0;
    }
    if (m == 0 || n == 0)
        return 0;
    try {
        return (size_t)workspace_elems(r.table, m, k, n, r.levels) * 8u;
    } catch (const std::exception &e) {
        set_error(e.what());
        return 0;
    }
}

int wsmul_tune_tiles(int64_t m, int64_t k, int64_t n, int64_t p, int dtype, int reps, int *best,
                     double *times_us) {
    if (m <= 0 || k <= 0 || n <= 0 || (dtype != WS_F64 && dtype != WS_I64) || reps < 1 ||
        reps > 10000)
        return fail(WS_EINVAL, "wsmul_tune_tiles: bad shape, dtype or repetition count");
    if (p < 2 || p >= (int64_t(1) << 24))
        return fail(WS_EMODULUS, "p must lie in [2, 2^24)");
    double us[TILE_KINDS];
    const hipError_t e = time_tiles(m, n, k, p, dtype, reps, us);
    if (e != hipSuccess)
        return fail(WS_EHIP, std::string("wsmul_tune_tiles: ") + hipGetErrorString(e));
    int kind = -1;
    for (int t = 0; t < TILE_KINDS; ++t)
        if (us[t] >= 0.0 && (kind < 0 || us[t] < us[kind]))
            kind = t;
    choose_tile(m, n, k, p, dtype, kind);
    if (best)
        *best = kind;
    if (times_us)
        for (int t = 0; t < TILE_KINDS; ++t)
            times_us[t] = us[t];
    return WS_OK;
}

int wsmul_set_tile(int64_t m, int64_t k, int64_t n, int64_t p, int dtype, int kind) {
    if (m < 0 || k < 0 || n < 0 || (dtype != WS_F64 && dtype != WS_I64) || kind < -1 ||
        kind >= TILE_KINDS)
        return fail(WS_EINVAL, "wsmul_set_tile: bad shape, dtype or kind");
    choose_tile(m, n, k, p, dtype, kind);
    return WS_OK;
}

int wsmul_tune_plan(const ws_args *args, int reps) {
    ws_args a;
    PlanKey key;
    Resolved res;
    int rc = prepare(args, a, key, res);
    if (rc != WS_OK)
        return rc;
    if (a.m == 0 || a.n == 0 || a.base == WS_BASE_I8_LIMBS)
        return WS_OK;
    std::shared_ptr<Plan> plan;
    try {
        plan = get_plan(key);
    } catch (const std::exception &e) {
        return fail(WS_EINVAL, std::string("planner: ") + e.what());
    }
    std::set<std::tuple<int64_t, int64_t, int64_t>> shapes;
    for (const OpDesc &op : plan->ops)
        if (op.kind == WS_OP_GEMM && op.a.rows > 0 && op.a.cols > 0 && op.b.cols > 0)
            shapes.insert(std::make_tuple(op.a.rows, op.a.cols, op.b.cols));
    for (const auto &sh : shapes) {
        rc = wsmul_tune_tiles(std::get<0>(sh), std::get<1>(sh), std::get<2>(sh), a.p, a.dtype,
                              reps, nullptr, nullptr);
        if (rc != WS_OK)
            return rc;
    }
    return WS_OK;
}

int wsmul_plan_info(const ws_args *args, ws_stats *stats) {
    ws_args a;
    PlanKey key;
    Resolved res;
    if (!stats)
        return fail(WS_EINVAL, "null stats");
    ws_args probe = args ? *args : ws_args{};
    // Pointers are not dereferenced: stand-ins keep the null checks quiet.
    static char dummy[16];
    if (!probe.A) probe.A = dummy;
    if (!probe.B) probe.B = dummy;
    if (!probe.C) probe.C = dummy;
    int rc = prepare(&probe, a, key, res);
    if (rc != WS_OK)
        return rc;
    std::memset(stats, 0, sizeof(*stats));
    if (a.m == 0 || a.n == 0)
        return WS_OK;
    try {
        auto plan = get_plan(key);
        fill_stats(*plan, a, *stats);
    } catch (const std::exception &e) {
        return fail(WS_EINVAL, std::string("planner: ") + e.what());
    }
    return WS_OK;
}

int wsmul_plan_export(const ws_args *args, ws_op_desc *ops, int64_t cap, int64_t *count) {
    ws_args a;
    PlanKey key;
    Resolved res;
    if (!count || (cap > 0 && !ops))
        return fail(WS_EINVAL, "null output");
    ws_args probe = args ? *args : ws_args{};
    static char dummy[16];
    if (!probe.A) probe.A = dummy;
    if (!probe.B) probe.B = dummy;
    if (!probe.C) probe.C = dummy;
    int rc = prepare(&probe, a, key, res);
    if (rc != WS_OK)
        return rc;
    *count = 0;
    if (a.m == 0 || a.n == 0)
        return WS_OK;
    try {
        auto plan = get_plan(key);
        if (a.base == WS_BASE_I8_LIMBS && plan->ws_elems > 0) {
            auto ex = digit_exec(*plan);
            *count = (int64_t)ex->ops.size();
            for (int64_t i = 0; i < cap && i < *count; ++i) {
                const ExecOp &e = ex->ops[i];
                ops[i] = e.op;
                for (int k = 0; k < e.op.nin; ++k)
                    ops[i].in[k].form = e.in_enc[k];
                for (int o = 0; o < e.op.nout; ++o)
                    ops[i].out[o].form = e.out_enc[o];
                ops[i].a.form = e.pre_a ? WS_FORM_DIGITS_A : WS_FORM_RESIDUES;
                ops[i].b.form = e.pre_b ? WS_FORM_DIGITS_B : WS_FORM_RESIDUES;
            }
        } else {
            *count = (int64_t)plan->ops.size();
            for (int64_t i = 0; i < cap && i < *count; ++i)
                ops[i] = plan->ops[i];
        }
    } catch (const std::exception &e) {
        return fail(WS_EINVAL, std::string("planner: ") + e.what());
    }
    return WS_OK;
}

int wsmul_set_workspace(void *ptr, size_t bytes) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_ws = bytes ? ptr : nullptr;
    g_ws_bytes = ptr ? bytes : 0;
    return WS_OK;
}

int wsmul_set_stream(void *stream) {
    g_stream.store(static_cast<hipStream_t>(stream));
    return WS_OK;
}

int wsmul_get_stats(ws_stats *out) {
    if (!out)
        return fail(WS_EINVAL, "null stats");
    *out = g_stats;
    return WS_OK;
}

int wsmul_reset_stats(void) {
    std::memset(&g_stats, 0, sizeof(g_stats));
    std::memset(&g_trace, 0, sizeof(g_trace));
    return WS_OK;
}

int wsmul_get_trace(ws_trace *out) {
    if (!out)
        return fail(WS_EINVAL, "null trace");
    *out = g_trace;
    return WS_OK;
}

const char *wsmul_last_error(void) { return g_err.c_str(); }

const char *wsmul_schedule_name(int table) {
    switch (table) {
    case TAB_CLASSICAL: return "classical";
    case TAB_T1: return "table1-two-temporaries";
    case TAB_HL: return "table2-three-temporaries";
    case TAB_IP: return "table3-in-place-overwrite";
    case TAB_OVR: return "table5-overwrite-B";
    case TAB_ACLR: return "table6-accumulate-overwrite";
    case TAB_ACCR: return "table7-accumulate-overwrite-B";
    case TAB_ACC: return "table9-accumulate-two-temporaries";
    case TAB_IPMM: return "algorithm2-read-only-in-place";
    case TAB_IPMM_ACC: return "algorithm2-read-only-in-place-table9";
    case TAB_OVL: return "table4-overwrite-A";
    case TAB_ACR: return "table8-accumulate-overwrite-B-rectangular";
    case TAB_IP0VMM: return "algorithm1-in-place-overwrite-rectangular";
    case TAB_BLOCKED_HL: return "section7.2-blocked-accumulation-table2";
    case TAB_BLOCKED_ACC: return "section7.2-blocked-accumulation-table9";
    default: return "unknown";
    }
}

const char *wsmul_version(void) { return "wsmul 0.1 (gfx950)"; }

}  // extern "C"
