// Choice of schedule, Winograd depth and base kind per product.
//
// Every admissible candidate is expanded into its real fused plan (the plan
// cache keeps this cheap) and costed operation by operation with rates
// measured on MI355X for the kernels of this library:
//   base products, binary64 matrix cores: 60 TFLOP/s (57 when folding) for
//     whole 128 x 128 tiles, 58 (50) for ragged large products, 45 / 30
//     TFLOP/s for the 64 x 64 class with whole / ragged tiles, 25 / 19 for
//     the small class, 7 us floor per launch;
//   base products, 8-bit digits: 318 / 310 / 255 / 210 / 45 TFLOP/s
//     (equivalent) by 128 x 128 tile count (16384^3, 8192^3 and 12288^3,
//     4096^3, 2048^3, 1024^3 measured, the product's store included; every
//     other epilogue stream
//     at 3.2 TB/s, measured per product inside Tables 1 and 2), plus the
//     digit split passes of operands that are not already digit planes
//     (bytes at 5.5 TB/s);
//   addition groups: bytes moved at 4.5 TB/s (5.0 TB/s for the digit base's
//     groups on digit-plane temporaries, 3 bytes per such entry), 4 us floor
//     per launch.
// The cheapest candidate whose temporaries fit the memory budget wins; a
// candidate with temporaries is charged 1% extra (the model's error), so that
// within it the schedule without extra memory is kept.
// Overwriting schedules are never chosen automatically (they destroy A, B).
// For accumulating products the blocked accumulation of Section 7.2 (t = 2,
// 3, 4 over Table 2, or over Table 9 when square) is a candidate too: it is
// never the fastest, but it keeps Winograd's saving when the budget is below
// the unblocked schedules' temporaries.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "wsmul_internal.hpp"

namespace wsmul {

namespace {

double gemm_f64_us(int64_t M, int64_t N, int64_t K, int64_t p) {
    const double flops = 2.0 * (double)M * (double)N * (double)K;
    const int64_t big = ((M + 127) / 128) * ((N + 127) / 128);
    const int64_t mid = ((M + 63) / 64) * ((N + 63) / 64);
    const double per_tile = 16.0 * (double)(p - 1) * (double)(p - 1);
    const bool folds = per_tile * ((double)K / 16.0 + 1.0) >= 9.0e15;
    double rate;
    if (big >= 256 && M % 128 == 0 && N % 128 == 0 && K % 16 == 0)
        rate = folds ? 57e12 : 60e12;             // pipelined 128 x 128 tiles
    else if (big >= 512)
        rate = folds ? 50e12 : 58e12;             // large products of other shapes, register-staged
    else if (mid >= 256)
        rate = (M % 64 == 0 && N % 64 == 0 && K % 64 == 0) ? 45e12 : 30e12;
    else
        rate = (M % 32 == 0 && N % 32 == 0 && K % 64 == 0) ? 25e12 : 19e12;
    return std::max(7.0, flops / rate * 1e6);
}

double gemm_digits_us(int64_t M, int64_t N, int64_t K, int64_t p, bool pre_a = false,
                      bool pre_b = false) {
    // the rates are for three digits (nine digit products); two take four
    const double nd = (double)digit_count(p);
    const double flops = 2.0 * (double)M * (double)N * (double)K * nd * nd / 9.0;
    const int64_t tiles = ((M + 127) / 128) * ((N + 127) / 128);
    const double rate = tiles >= 16384  ? 318e12
                        : tiles >= 2048 ? 310e12
                        : tiles >= 512  ? 255e12
                        : tiles >= 128  ? 210e12
                                        : 45e12;
    const double split_bytes = 11.0 * ((pre_a ? 0.0 : (double)M * (double)K) +
                                       (pre_b ? 0.0 : (double)K * (double)N));
    const int splits = (pre_a ? 0 : 1) + (pre_b ? 0 : 1);
    return std::max(8.0, flops / rate * 1e6) + 5.0 * splits + split_bytes / 5.5e12 * 1e6;
}

struct Key {
    int64_t m, k, n, p;
    int dtype, beta_nz, schedule, levels, base, blocks;
    size_t budget;
    bool operator<(const Key &o) const {
        return std::tie(m, k, n, p, dtype, beta_nz, schedule, levels, base, blocks, budget) <
               std::tie(o.m, o.k, o.n, o.p, o.dtype, o.beta_nz, o.schedule, o.levels, o.base,
                        o.blocks, o.budget);
    }
};
struct Choice {
    int schedule, levels, base, blocks;
    double cost_us;
};

std::mutex g_tune_mu;
std::map<Key, Choice> g_tune;
bool g_loaded = false;

const char *cache_path() { return std::getenv("WSMUL_TUNE_CACHE"); }

void load_cache() {
    if (g_loaded)
        return;
    g_loaded = true;
    const char *path = cache_path();
    if (!path)
        return;
    FILE *f = std::fopen(path, "r");
    if (!f)
        return;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        Key k{};
        Choice c{};
        long long m, kk, n, p;
        unsigned long long budget;
        if (std::sscanf(line,
                        "{\"m\": %lld, \"k\": %lld, \"n\": %lld, \"p\": %lld, \"dtype\": %d, "
                        "\"beta_nz\": %d, \"schedule_in\": %d, \"levels_in\": %d, \"base_in\": %d, "
                        "\"blocks_in\": %d, \"budget\": %llu, \"schedule\": %d, \"levels\": %d, "
                        "\"base\": %d, \"blocks\": %d, \"cost_us\": %lf}",
                        &m, &kk, &n, &p, &k.dtype, &k.beta_nz, &k.schedule, &k.levels, &k.base,
                        &k.blocks, &budget, &c.schedule, &c.levels, &c.base, &c.blocks,
                        &c.cost_us) == 16) {
            k.m = m;
            k.k = kk;
            k.n = n;
            k.p = p;
            k.budget = (size_t)budget;
            g_tune[k] = c;
        }
    }
    std::fclose(f);
}

void save_entry(const Key &k, const Choice &c) {
    const char *path = cache_path();
    if (!path)
        return;
    FILE *f = std::fopen(path, "a");
    if (!f)
        return;
    std::fprintf(f,
                 "{\"m\": %lld, \"k\": %lld, \"n\": %lld, \"p\": %lld, \"dtype\": %d, "
                 "\"beta_nz\": %d, \"schedule_in\": %d, \"levels_in\": %d, \"base_in\": %d, "
                 "\"blocks_in\": %d, \"budget\": %llu, \"schedule\": %d, \"levels\": %d, "
                 "\"base\": %d, \"blocks\": %d, \"cost_us\": %.3f}\n",
                 (long long)k.m, (long long)k.k, (long long)k.n, (long long)k.p, k.dtype, k.beta_nz,
                 k.schedule, k.levels, k.base, k.blocks, (unsigned long long)k.budget, c.schedule,
                 c.levels, c.base, c.blocks, c.cost_us);
    std::fclose(f);
}

// Search every admissible candidate; returns false if none fits.  When no
// candidate passes the schedule's own checks, *reject holds the status and
// message of the last check (WS_OK when some candidate only missed the
// memory budget).
bool search(const Key &key, Choice &best, Resolved *reject) {
    bool found = false, admissible = false;
    best.cost_us = 1e300;
    reject->status = WS_OK;
    // (schedule, t) pairs; t only matters for the blocked schedules.
    std::vector<std::pair<int, int>> cands;
    if (key.schedule != WS_AUTO) {
        cands.push_back({key.schedule, key.blocks});
    } else {
        // Read-only candidates: classical, the two-temporary schedules
        // (Table 1 / Table 9), Algorithm 2 for C = A*B; for accumulating
        // products also Table 2 (non-square shapes) and the blocked
        // accumulation of Section 7.2 (small memory budgets).
        cands.push_back({WS_CLASSICAL, 0});
        cands.push_back({WS_TWO_TEMP, 0});
        if (!key.beta_nz) {
            cands.push_back({WS_READONLY_INPLACE, 0});
        } else {
            cands.push_back({WS_HL_THREE_TEMP, 0});
            for (int t : {2, 3, 4}) {
                cands.push_back({WS_BLOCKED, t});
                cands.push_back({WS_BLOCKED_ACC, t});
            }
        }
    }
    std::vector<int> bases;
    if (key.base != WS_BASE_AUTO)
        bases.push_back(key.base);
    else {
        bases.push_back(WS_BASE_F64_MFMA);
        if (limbs_supported(key.p) && key.k <= 32768 && key.k > 0)
            bases.push_back(WS_BASE_I8_LIMBS);
    }
    const int64_t mn = std::min(key.m, std::min(key.k, key.n));
    for (const auto &cand : cands) {
        const int sched = cand.first, t = cand.second;
        const bool blocked = sched == WS_BLOCKED || sched == WS_BLOCKED_ACC;
        // deepest level that keeps base products of at least 64 (per block)
        const int64_t mb = blocked ? mn / std::max(t, 1) : mn;
        int top = 0;
        while (top < 5 && (mb >> (top + 1)) >= 64)
            ++top;
        const int lo = key.levels >= 0 ? key.levels : (sched == WS_CLASSICAL ? 0 : 1);
        int hi = key.levels >= 0 ? key.levels : (sched == WS_CLASSICAL ? 0 : top);
        if (key.schedule != WS_AUTO)
            hi = std::max(hi, lo);   // a schedule the caller fixed gets at least one depth

        for (int l = lo; l <= hi; ++l) {
            const Resolved r = resolve_schedule(sched, key.m, key.k, key.n, key.beta_nz != 0, l, t);
            if (r.status != WS_OK) {
                if (!admissible)
                    *reject = r;
                continue;
            }
            admissible = true;
            reject->status = WS_OK;
            // A plan of depth l runs at least 7^l base products (t^3 times
            // that when blocked), each costed at no less than the 7 us
            // launch floor: once that bound passes the best cost found, the
            // candidate cannot win and its (large) plan is not built.
            const double floor_us =
                7.0 * std::pow(7.0, (double)r.levels) * (blocked ? (double)t * t * t : 1.0);
            if (found && floor_us >= best.cost_us)
                continue;
            PlanKey pk{};
            pk.m = key.m;
            pk.k = key.k;
            pk.n = key.n;
            pk.p = key.p;
            pk.lda = key.k;
            pk.ldb = key.n;
            pk.ldc = key.n;
            pk.alpha = 1;
            pk.beta = key.beta_nz ? 1 : 0;
            pk.dtype = key.dtype;
            pk.table = r.table;
            pk.levels = r.levels;
            pk.fuse = 1;
            pk.blocks = blocked ? t : 0;
            std::shared_ptr<Plan> plan;
            try {
                plan = get_plan(pk);
            } catch (...) {
                continue;
            }
            if ((size_t)plan->ws_elems * 8u > key.budget)
                continue;
            for (int base : bases) {
                // A plan with temporaries must win by more than the cost
                // model's error (about 1%) over one without: within that,
                // less memory decides.
                const double c = plan_cost_us(*plan, base) * (plan->ws_elems > 0 ? 1.01 : 1.0);
                if (c < best.cost_us) {
                    best = Choice{sched, l, base, blocked ? t : key.blocks, c};
                    found = true;
                }
            }
        }
    }
    return found;
}

}  // namespace

double plan_cost_us(const Plan &plan, int base) {
    double t = 0.0;
    if (base == WS_BASE_I8_LIMBS) {
        // the digit base's execution list: temporaries held as digit planes
        // move 3 bytes per entry and spare their products' splits
        const auto x = digit_exec(plan);
        // whole inputs split once into planes
        t += (x->split_a ? 5.0 + 11.0 * (double)plan.key.m * (double)plan.key.k / 5.5e12 * 1e6 : 0.0) +
             (x->split_b ? 5.0 + 11.0 * (double)plan.key.k * (double)plan.key.n / 5.5e12 * 1e6 : 0.0);
        for (const ExecOp &e : x->ops) {
            const OpDesc &op = e.op;
            const double elems = (double)op.out[0].rows * (double)op.out[0].cols;
            if (op.kind == WS_OP_GEMM) {
                // the rates include the product's own store; every further
                // epilogue stream adds its bytes at ~3.2 TB/s (all tiles of a
                // round run their epilogues together, after their products)
                t += gemm_digits_us(op.a.rows, op.b.cols, op.a.cols, plan.key.p, e.pre_a, e.pre_b);
                t += 8.0 * (double)(op.nin - 1 + op.nout - 1) * elems / 3.2e12 * 1e6;
            } else {
                double per = 0.0;
                for (int i = 0; i < op.nin; ++i)
                    per += e.in_enc[i] ? 3.0 : 8.0;
                for (int o = 0; o < op.nout; ++o)
                    per += e.out_enc[o] ? 3.0 : 8.0;
                const bool digits = exec_uses_digits(e);
                t += std::max(4.0, per * elems / (digits ? 5.0e12 : 4.5e12) * 1e6);
            }
        }
        return t;
    }
    for (const OpDesc &op : plan.ops) {
        if (op.kind == WS_OP_GEMM) {
            t += base == WS_BASE_I8_LIMBS ? gemm_digits_us(op.a.rows, op.b.cols, op.a.cols, plan.key.p)
                                          : gemm_f64_us(op.a.rows, op.b.cols, op.a.cols, plan.key.p);
            t += 8.0 * (double)(op.nin - 1 + op.nout) * (double)op.out[0].rows *
                 (double)op.out[0].cols / 4.5e12 * 1e6;   // epilogue traffic
        } else {
            const double bytes = 8.0 * (double)(op.nin + op.nout) * (double)op.out[0].rows *
                                 (double)op.out[0].cols;
            t += std::max(4.0, bytes / 4.5e12 * 1e6);
        }
    }
    return t;
}

// Called by the entry points for WS_AUTO / levels < 0 / WS_BASE_AUTO.
int autotune_choice(ws_args &a, bool beta_nonzero) {
    ws_args c = a;
    const size_t budget = a.workspace ? (size_t)a.workspace_bytes : (size_t)-1;
    const int rc = wsmul_autotune(a.m, a.k, a.n, a.p, a.dtype, budget, &c);
    (void)beta_nonzero;
    if (rc != WS_OK)
        return rc;
    a.schedule = c.schedule;
    a.levels = c.levels;
    a.base = c.base;
    a.blocks = c.blocks;
    return WS_OK;
}

}  // namespace wsmul

using namespace wsmul;

extern "C" int wsmul_autotune(int64_t m, int64_t k, int64_t n, int64_t p, int dtype,
                              size_t mem_budget, ws_args *choice) {
    if (!choice || m < 0 || k < 0 || n < 0 || p < 2 || p >= (int64_t(1) << 24) ||
        (dtype != WS_F64 && dtype != WS_I64)) {
        set_error("wsmul_autotune: bad arguments");
        return WS_EINVAL;
    }
    const bool beta_nz = ((choice->beta % p) + p) % p != 0;
    const int blocks = choice->blocks == 0 ? 2 : (int)std::min<uint32_t>(choice->blocks, 1u << 20);
    Key key{m, k, n, p, dtype, beta_nz ? 1 : 0, choice->schedule, choice->levels, choice->base,
            blocks, mem_budget};
    if (key.schedule != WS_AUTO && key.schedule != WS_CLASSICAL && key.schedule != WS_TWO_TEMP &&
        key.schedule != WS_OVERWRITE && key.schedule != WS_READONLY_INPLACE &&
        key.schedule != WS_HL_THREE_TEMP && key.schedule != WS_OVR && key.schedule != WS_ACCR &&
        key.schedule != WS_BLOCKED && key.schedule != WS_BLOCKED_ACC && key.schedule != WS_OVL &&
        key.schedule != WS_ACR && key.schedule != WS_IPMM_ACC) {
        set_error("wsmul_autotune: unknown schedule");
        return WS_ESCHEDULE;
    }
    if (m == 0 || n == 0 || k == 0) {
        choice->schedule = key.schedule == WS_AUTO ? WS_CLASSICAL : key.schedule;
        choice->levels = 0;
        choice->base = key.base == WS_BASE_AUTO ? WS_BASE_F64_MFMA : key.base;
        choice->blocks = (uint32_t)blocks;
        return WS_OK;
    }
    Choice best{};
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        load_cache();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            best = it->second;
            choice->schedule = best.schedule;
            choice->levels = best.levels;
            choice->base = best.base;
            choice->blocks = (uint32_t)best.blocks;
            return WS_OK;
        }
    }
    Resolved reject;
    if (!search(key, best, &reject)) {
        if (reject.status != WS_OK) {
            set_error(reject.error);
            return reject.status;
        }
        set_error("wsmul_autotune: no schedule fits the memory budget at this shape");
        return WS_ENOMEM;
    }
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune[key] = best;
        save_entry(key, best);
    }
    choice->schedule = best.schedule;
    choice->levels = best.levels;
    choice->base = best.base;
    choice->blocks = (uint32_t)best.blocks;
    return WS_OK;
}
