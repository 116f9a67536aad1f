// Many independent products in one persistent launch, optionally captured
// once into a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"
#include "wsmul.h"
#include "wsmul_internal.hpp"

namespace wsmul {

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int fail(int code, const std::string &msg) {
    set_error(msg);
    return code;
}

// Host and device state of one batch.  The device block holds the operation
// records, the task list and the products' temporaries.  Records and tasks
// are grouped by phase (the position of an operation within its product's
// plan); phase_task[j] .. phase_task[j+1] are the tasks of phase j.
struct Batch {
    std::vector<std::shared_ptr<Plan>> plans;
    std::vector<ws_args> norm;
    std::vector<size_t> ws_off;
    std::vector<BatchOp> ops;
    std::vector<int2> tasks;
    std::vector<size_t> phase_task;
    size_t ws_bytes = 0;
    size_t off_tasks = 0, off_ws = 0, dev_bytes = 0;
    char *dev = nullptr;
    int grid = 0;
};

int plan_batch(const ws_args *probs, int count, Batch &b) {
    if (!probs || count < 0)
        return fail(WS_EINVAL, "null batch");
    b.plans.assign(count, nullptr);
    b.norm.resize(count);
    b.ws_off.assign(count, 0);
    size_t ws_total = 0;
    for (int i = 0; i < count; ++i) {
        PlanKey key;
        Resolved res;
        // The batch kernel runs the binary64 base only: a product that leaves
        // the base to the library gets that base before the autotuner prices
        // its schedule and depth.
        ws_args req = probs[i];
        if (req.base == WS_BASE_AUTO)
            req.base = WS_BASE_F64_MFMA;
        const int rc = prepare(&req, b.norm[i], key, res);
        if (rc != WS_OK)
            return rc;
        if (b.norm[i].dtype != WS_F64 || b.norm[i].base == WS_BASE_I8_LIMBS)
            return fail(WS_EINVAL, "batched launches take binary64 storage and the binary64 base");
        if (b.norm[i].m == 0 || b.norm[i].n == 0)
            continue;
        try {
            b.plans[i] = get_plan(key);
        } catch (const std::exception &e) {
            return fail(WS_EINVAL, std::string("planner: ") + e.what());
        }
        b.ws_off[i] = ws_total;
        ws_total += align256((size_t)b.plans[i]->ws_elems * 8u);
    }
    b.ws_bytes = ws_total;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    b.grid = std::max(1, cus * batch_blocks_per_cu());
    return WS_OK;
}

// Records grouped by phase: operation j of every product forms phase j.
void fill_records(Batch &b, void *ws_base) {
    size_t max_ops = 0;
    for (auto &pl : b.plans)
        if (pl)
            max_ops = std::max(max_ops, pl->ops.size());
    b.ops.clear();
    b.tasks.clear();
    b.phase_task.assign(1, 0);
    for (size_t j = 0; j < max_ops; ++j) {
        for (size_t i = 0; i < b.plans.size(); ++i) {
            const auto &pl = b.plans[i];
            if (!pl || j >= pl->ops.size())
                continue;
            const ws_args &a = b.norm[i];
            DevBufs bufs{{a.A, a.B, a.C, static_cast<char *>(ws_base) + b.ws_off[i]}, nullptr, 0};
            BatchOp op;
            fill_batch_op(op, pl->ops[j], bufs, a.p);
            op.phase = (int32_t)j;
            const int o = (int)b.ops.size();
            b.ops.push_back(op);
            for (int t = 0; t < op.ntiles; ++t)
                b.tasks.push_back(make_int2(o, t));
        }
        // Longest tasks first: the persistent grid deals tasks round-robin,
        // so every workgroup then gets one task from each cost band and the
        // phase ends evenly.  A product tile costs its inner dimension (plus
        // a fixed part); an addition chunk a fixed amount.
        auto cost = [&](const int2 &t) {
            const BatchOp &op = b.ops[t.x];
            return op.kind == WS_OP_GEMM ? op.g.K + 64 : (int64_t)32;
        };
        std::stable_sort(b.tasks.begin() + (std::ptrdiff_t)b.phase_task.back(), b.tasks.end(),
                         [&](const int2 &x, const int2 &y) { return cost(x) > cost(y); });
        b.phase_task.push_back(b.tasks.size());
    }
}

// Allocate the device block (stream-ordered) and upload records and tasks.
int materialise(Batch &b, hipStream_t stream, void *ws_attached, size_t ws_attached_bytes,
                bool ordered_alloc) {
    fill_records(b, nullptr);   // sizes only
    const bool own_ws = !(ws_attached && ws_attached_bytes >= b.ws_bytes);
    b.off_tasks = align256(std::max<size_t>(b.ops.size(), 1) * sizeof(BatchOp));
    b.off_ws = b.off_tasks + align256(std::max<size_t>(b.tasks.size(), 1) * sizeof(int2));
    b.dev_bytes = b.off_ws + (own_ws ? b.ws_bytes : 0);
    void *p = nullptr;
    const hipError_t e = ordered_alloc ? hipMallocAsync(&p, b.dev_bytes, stream)
                                       : hipMalloc(&p, b.dev_bytes);
    if (e != hipSuccess)
        return fail(WS_ENOMEM, "batch allocation failed");
    b.dev = static_cast<char *>(p);
    fill_records(b, own_ws ? static_cast<void *>(b.dev + b.off_ws) : ws_attached);
    if (hipMemcpyAsync(b.dev, b.ops.data(), b.ops.size() * sizeof(BatchOp), hipMemcpyHostToDevice,
                       stream) != hipSuccess ||
        hipMemcpyAsync(b.dev + b.off_tasks, b.tasks.data(), b.tasks.size() * sizeof(int2),
                       hipMemcpyHostToDevice, stream) != hipSuccess)
        return fail(WS_EHIP, "batch upload failed");
    // The host-side records must outlive the copies.
    if (hipStreamSynchronize(stream) != hipSuccess)
        return fail(WS_EHIP, "batch upload failed");
    return WS_OK;
}

// One launch per phase, in phase order on the stream.
int enqueue(const Batch &b, hipStream_t stream) {
    const BatchOp *ops = reinterpret_cast<const BatchOp *>(b.dev);
    const int2 *tasks = reinterpret_cast<const int2 *>(b.dev + b.off_tasks);
    for (size_t j = 0; j + 1 < b.phase_task.size(); ++j) {
        const size_t t0 = b.phase_task[j], t1 = b.phase_task[j + 1];
        const hipError_t e = launch_batch(ops, tasks + t0, (int64_t)(t1 - t0), b.grid, stream);
        if (e != hipSuccess)
            return fail(WS_EHIP, std::string("batch launch failed: ") + hipGetErrorString(e));
    }
    return WS_OK;
}

int wait_done(hipStream_t stream) {
    const hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess)
        return fail(WS_EHIP, std::string("batch failed: ") + hipGetErrorString(e));
    return WS_OK;
}

void record_stats(const Batch &b, size_t internal) {
    ws_stats s{};
    for (auto &pl : b.plans)
        if (pl) {
            s.add_launches += (uint64_t)pl->add_ops;
            s.gemm_launches += (uint64_t)pl->gemm_ops;
            s.element_additions += (uint64_t)pl->element_additions;
            s.base_flops += (uint64_t)pl->base_flops;
            s.rows += (uint64_t)pl->rows;
        }
    s.workspace_bytes = b.ws_bytes;
    s.internal_alloc_bytes = internal;
    s.schedule = -1;
    s.base = WS_BASE_F64_MFMA;
    set_stats(s);
}

// A captured batch: device block and instantiated graph, both kept alive
// until wsmul_graph_destroy.
struct GraphBatch {
    Batch b;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
};

}  // namespace
}  // namespace wsmul

using namespace wsmul;

extern "C" {

int wsmul_batched(const ws_args *probs, int count, unsigned flags) {
    Batch b;
    int rc = plan_batch(probs, count, b);
    if (rc != WS_OK)
        return rc;
    hipStream_t stream = (count > 0 && probs[0].stream) ? static_cast<hipStream_t>(probs[0].stream)
                                                        : default_stream();
    void *ws = nullptr;
    size_t ws_bytes = 0;
    attached_workspace(&ws, &ws_bytes);
    rc = materialise(b, stream, ws, ws_bytes, true);
    if (rc == WS_OK && !b.tasks.empty())
        rc = enqueue(b, stream);
    if (rc == WS_OK && (flags & WS_FLAG_SYNC))
        rc = wait_done(stream);
    if (b.dev)
        (void)hipFreeAsync(b.dev, stream);
    record_stats(b, b.dev_bytes);
    set_batch_phases(b.phase_task.empty() ? 0 : b.phase_task.size() - 1);
    return rc;
}

int wsmul_graph_capture(const ws_args *probs, int count, void **graph_exec) {
    if (!graph_exec)
        return fail(WS_EINVAL, "null graph handle");
    *graph_exec = nullptr;
    auto g = std::make_unique<GraphBatch>();
    int rc = plan_batch(probs, count, g->b);
    if (rc != WS_OK)
        return rc;
    (void)hipGetDevice(&g->device);
    hipStream_t cap = nullptr;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
        return fail(WS_EHIP, "stream creation failed");
    rc = materialise(g->b, cap, nullptr, 0, false);
    if (rc == WS_OK && hipStreamSynchronize(cap) != hipSuccess)
        rc = fail(WS_EHIP, "batch upload failed");
    if (rc == WS_OK) {
        // The graph holds one persistent launch per phase (no memset nodes).
        if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
            rc = fail(WS_EHIP, "hipStreamBeginCapture failed");
        else {
            const int erc = g->b.tasks.empty() ? WS_OK : enqueue(g->b, cap);
            const hipError_t e = hipStreamEndCapture(cap, &g->graph);
            if (erc != WS_OK)
                rc = erc;
            else if (e != hipSuccess)
                rc = fail(WS_EHIP, "hipStreamEndCapture failed");
            else if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
                rc = fail(WS_EHIP, "hipGraphInstantiate failed");
        }
    }
    (void)hipStreamDestroy(cap);
    if (rc != WS_OK) {
        if (g->exec)
            (void)hipGraphExecDestroy(g->exec);
        if (g->graph)
            (void)hipGraphDestroy(g->graph);
        if (g->b.dev)
            (void)hipFree(g->b.dev);
        return rc;
    }
    record_stats(g->b, g->b.dev_bytes);
    set_batch_phases(g->b.phase_task.size() - 1);
    *graph_exec = g.release();
    return WS_OK;
}

int wsmul_graph_launch(void *graph_exec, void *stream) {
    auto *g = static_cast<GraphBatch *>(graph_exec);
    if (!g || !g->exec)
        return fail(WS_EINVAL, "null graph handle");
    hipStream_t s = stream ? static_cast<hipStream_t>(stream) : default_stream();
    if (hipGraphLaunch(g->exec, s) != hipSuccess)
        return fail(WS_EHIP, "hipGraphLaunch failed");
    return WS_OK;
}

int wsmul_graph_check(void *graph_exec, void *stream) {
    auto *g = static_cast<GraphBatch *>(graph_exec);
    if (!g)
        return fail(WS_EINVAL, "null graph handle");
    hipStream_t s = stream ? static_cast<hipStream_t>(stream) : default_stream();
    return wait_done(s);
}

int wsmul_graph_destroy(void *graph_exec) {
    auto *g = static_cast<GraphBatch *>(graph_exec);
    if (!g)
        return WS_OK;
    (void)hipDeviceSynchronize();
    if (g->exec)
        (void)hipGraphExecDestroy(g->exec);
    if (g->graph)
        (void)hipGraphDestroy(g->graph);
    if (g->b.dev)
        (void)hipFree(g->b.dev);
    delete g;
    return WS_OK;
}

}  // extern "C"
