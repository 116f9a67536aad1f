"""Benchmark: exact Winograd products over Z/pZ on one MI355X.

Default workload (t1_16384_p1048573): C = A*B mod 1048573 with m = k = n =
16384, the largest single-GPU configuration, with schedule, Winograd depth and
base (binary64 matrix cores or 8-bit digits on the int8 matrix cores) chosen
by the autotuner.  One step is one such product on inputs already resident in
HBM.  The same product is also timed as the classical product on both bases,
as Table 1 at one level on the digit base and as Table 1 at two levels on the
binary64 base, so the line carries Winograd against classical on each base.

--workload selects one of the other configurations instead:
  acc_4096_p65521_l3            C <- A*B + C mod 65521, 4096^3, three Winograd levels under
                                the read-only two-temporary accumulating schedule (Table 9),
                                binary64 base; against the input-overwriting accumulating
                                schedule (Table 6; A and B restored from pristine copies
                                outside the timed window) and classical
  t1_512_p65521_l1_i64          C = A*B mod 65521, 512^3, int64 storage, Table 1, one level
  ipmm_8192x4096x8192_p8388593  C = A*B mod 8388593, Algorithm 2 (read-only, in place),
                                one level, against Table 1 and classical
  overwrite_8192x16384x8192_p8388593
                                C = A*B mod 8388593 on the largest shape the paper times,
                                Algorithm 1 (here Table 3, then Table 6 in the freed block:
                                no workspace, A and B overwritten and restored from copies
                                outside the timed window), one level, against classical,
                                Table 1 and Algorithm 2
  acc_4096_p65521_blocked       the 4096^3 accumulation under Section 7.2's blocked
                                accumulation: C in t x t blocks (--blocks, default 2), each
                                block by t Table 9 calls of two levels, extra memory below
                                2(n/t)^2/3; against unblocked Table 9, the Table 2 base and
                                classical
  batch_2000                    2000 products, sizes log-uniform in [64, 2048], moduli
                                from {65521, 1048573, 8388593}, autotuned, one hipGraph
                                replay of the persistent batched launches

Prints one JSON line on stdout.  Extra fields: the peak temporary bytes of
each schedule, the comparator rates, a roofline entry for the dominant kernel
class (time from start/stop events that the kernel dispatches stamp on the
launch stream) and the oracle's rate on a bounded sample of the same work on
the host cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_F64_MFMA_TFLOPS = 78.6
PEAK_I8_MFMA_TOPS = 5000.0
PEAK_HBM_GBS = 8000.0
METRIC = "mod-p matmul effective Gop/s (2mnk/s) + peak temp bytes vs classical mod-p GEMM"
SCHEDULE_NAMES = {0: "classical", 1: "two temporaries (Table 1 / Table 9)",
                  2: "input-overwriting (Table 3 / Table 6)",
                  3: "read-only in place (Algorithm 2)", 4: "three temporaries (Table 2)",
                  6: "overwrite, accumulate right (Table 5)", 7: "accumulate right (Table 7)",
                  8: "blocked accumulation over Table 2 (Section 7.2)",
                  9: "blocked accumulation over Table 9 (Section 7.2)",
                  10: "overwrite left (Table 4)", 11: "accumulate, overwrite B, rectangular (Table 8)",
                  12: "read-only in place with Table 9 accumulations (Algorithm 2)"}
WORKLOADS = ("t1_16384_p1048573", "acc_4096_p65521_l3", "t1_512_p65521_l1_i64",
             "ipmm_8192x4096x8192_p8388593", "overwrite_8192x16384x8192_p8388593",
             "acc_4096_p65521_blocked", "batch_2000")
INPUTS_OF = {"acc_4096_p65521_blocked": "acc_4096_p65521_l3"}   # same product, other schedule


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernels_digest():
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels.hip", "limbs.hip", "gemm_common.hpp", "device.hpp", "digit_temps.cpp"):
        with open(os.path.join(ROOT, "paper_0707_2347_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, gemm_dominant):
    """HBM bytes per launch of the dominant kernel, from the FETCH_SIZE and
    WRITE_SIZE counter runs recorded in profiles/ (scaled by the plain-copy
    calibration there); None when there is no record for the workload or the
    kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernels_digest") != kernels_digest():
        return None
    key = "base_product" if gemm_dominant else "addition_group"
    return rec.get(key, {}).get("bytes_per_launch")


def measured_split_traffic(workload):
    """HBM bytes per digit-split launch from the same record, or None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernels_digest") != kernels_digest():
        return None
    return rec.get("digit_split", {}).get("bytes_per_launch")


class Ctx:
    """Device, stream and timing helpers shared by the workloads."""

    def __init__(self, args):
        import torch
        from paper_0707_2347_amd import capi, inputs
        self.torch, self.capi, self.inputs, self.args = torch, capi, inputs, args
        self.dev = torch.device("cuda:0")
        self.stream = torch.cuda.current_stream()
        self.split_roof = None

    def to_dev(self, x, dtype=None):
        t = self.torch.from_numpy(x)
        return t.to(self.dev) if dtype is None else t.to(self.dev).to(dtype)

    def timed(self, fn, steps, warmup):
        """Wall time per call of fn over `steps` calls after `warmup` calls,
        bracketed by device synchronisation."""
        for _ in range(warmup):
            fn()
        self.torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        self.torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    def event_ms(self, fn, reps, before=None):
        """Average event-timed duration of fn on the current stream."""
        torch = self.torch
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tot = 0.0
        for i in range(reps + 1):
            if before:
                before()
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            if i > 0:
                tot += e0.elapsed_time(e1)
        return tot / reps

    def traced(self, args, ntraced, int8_ops=False):
        """Kernel-class times of `ntraced` traced calls -> roofline entry."""
        capi = self.capi
        capi.wsmul_reset_stats()
        targs = capi.ws_args.from_buffer_copy(args)
        targs.flags |= capi.WS_FLAG_TRACE
        for _ in range(ntraced):
            capi.check(capi.wsmul_mod_p_ex(targs))
        tr = capi.wsmul_get_trace()
        gemm_avg_ms = tr.gemm_ms / max(tr.gemm_launches, 1)
        add_avg_ms = tr.add_ms / max(tr.add_launches, 1)
        gemm_flops_per = tr.gemm_flops / max(tr.gemm_launches, 1)
        add_bytes_per = tr.add_bytes / max(tr.add_launches, 1)
        log("trace: base products %d x %.4f ms, additions %d x %.4f ms"
            % (tr.gemm_launches, gemm_avg_ms, tr.add_launches, add_avg_ms))
        per_step = {"base_products": round(tr.gemm_ms / ntraced, 4),
                    "additions": round(tr.add_ms / ntraced, 4)}
        if tr.split_launches:
            per_step["digit_splits"] = round(tr.split_ms / ntraced, 4)
        gemm_dominant = tr.gemm_ms >= tr.add_ms
        traffic = measured_traffic(self.args.workload, gemm_dominant)
        if gemm_dominant and tr.gemm_launches:
            if int8_ops:
                # nd^2 digit products of 2*M*N*K int8 ops each per base product
                # (nd = 3 digits, 2 for p <= 65536); the time is the product
                # kernel's own (the splits are apart)
                nd = 2 if args.p <= 65536 else 3
                ops = nd * nd * gemm_flops_per
                ach = ops / (gemm_avg_ms * 1e-3) / 1e12
                roof = {"bound": "mfma", "kernel": "gemm_digits_kernel (int8 16x16x64 matrix "
                        "cores, %d x %d digit products of 2mnk int8 ops each)" % (nd, nd),
                        "achieved": round(ach, 2), "peak": PEAK_I8_MFMA_TOPS, "unit": "TOP/s",
                        "frac": round(ach / PEAK_I8_MFMA_TOPS, 4), "traffic": traffic,
                        "avg_launch_ms": round(gemm_avg_ms, 5), "int8_ops_per_launch": ops}
            else:
                ach = gemm_flops_per / (gemm_avg_ms * 1e-3) / 1e12
                roof = {"bound": "mfma", "kernel": "base product (f64 16x16x4 matrix cores)",
                        "achieved": round(ach, 3), "peak": PEAK_F64_MFMA_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(ach / PEAK_F64_MFMA_TFLOPS, 4),
                        "traffic": traffic, "avg_launch_ms": round(gemm_avg_ms, 5),
                        "flops_per_launch": gemm_flops_per}
        else:
            gbs = add_bytes_per / (add_avg_ms * 1e-3) / 1e9
            roof = {"bound": "hbm", "kernel": "fused addition rows", "achieved": round(gbs, 1),
                    "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
                    "traffic": traffic, "avg_launch_ms": round(add_avg_ms, 5),
                    "bytes_per_launch": add_bytes_per}
        counts = {"base_products": int(tr.gemm_launches // ntraced),
                  "addition_groups": int(tr.add_launches // ntraced)}
        add_roof = None
        if tr.split_launches:
            gbs = tr.split_bytes / (tr.split_ms * 1e-3) / 1e9
            self.split_roof = {"bound": "hbm", "kernel": "split_rows/split_cols (digit planes)",
                               "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                               "frac": round(gbs / PEAK_HBM_GBS, 4),
                               "traffic": measured_split_traffic(self.args.workload),
                               "avg_launch_ms": round(tr.split_ms / tr.split_launches, 5),
                               "bytes_per_launch": tr.split_bytes / tr.split_launches}
        if tr.add_launches:
            gbs = add_bytes_per / (add_avg_ms * 1e-3) / 1e9
            add_roof = {"bound": "hbm", "kernel": "fused addition rows", "achieved": round(gbs, 1),
                        "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
                        "traffic": measured_traffic(self.args.workload, False),
                        "avg_launch_ms": round(add_avg_ms, 5), "bytes_per_launch": add_bytes_per}
        return roof, per_step, counts, add_roof


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline_rows(A, B, C, alpha, beta, p, budget_s=12.0):
    """The oracle on the first rows of the same product (the whole product if
    it fits the budget), timed on the host cores."""
    from oracle import ref
    threads = ref.threads_available()
    m, k = A.shape
    n = B.shape[1]
    Ai, Bi = A.astype(np.int64, copy=False), B.astype(np.int64, copy=False)
    Ci = None if C is None else C.astype(np.int64, copy=False)

    def timed(r):
        t_s = time.perf_counter()
        ref.matmul_mod_p(Ai[:r], Bi, None if Ci is None else Ci[:r], alpha, beta, p,
                         threads=threads)
        return max(time.perf_counter() - t_s, 1e-4)

    # Calibrate on a sample large enough to keep every thread busy (a few
    # rows per thread undercount the rate), then fill the budget.
    rows = min(m, 16)
    dt = timed(rows)
    while rows < m and dt < 0.5:
        rows = min(m, rows * 4)
        dt = timed(rows)
    rows = m if dt / rows * m <= budget_s else int(max(16, budget_s * rows / dt))
    log("cpu baseline: oracle on %d rows x %d x %d, %d threads" % (rows, k, n, threads))
    # Repeat the sample while another run still fits the budget.
    elapsed, reps = 0.0, 0
    while reps == 0 or elapsed + elapsed / reps <= budget_s:
        elapsed += timed(rows)
        reps += 1
    dt = elapsed / reps
    return {"value": round(2.0 * rows * k * n / dt / 1e9, 3), "unit": "Gop/s",
            "cores": threads, "cpu": cpu_model(), "kind": "oracle",
            "sample": "rows 0..%d of the same product (%d x %d x %d), %d run(s) of %.3f s"
                      % (rows - 1, rows, k, n, reps, dt)}


def line(ctx, value, ms_step, dtype, config, roofline, cpu, extra):
    a = ctx.args
    out = {"metric": METRIC, "value": round(value, 3), "unit": "Gop/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic", "config": config, "roofline": roofline, "cpu_baseline": cpu}
    out.update(extra)
    return out


# ---------------------------------------------------------------- workloads
def single_product(ctx, name):
    """The four single-product workloads."""
    capi, inputs, torch = ctx.capi, ctx.inputs, ctx.torch
    a = ctx.args
    w = inputs.WORKLOADS[INPUTS_OF.get(name, name)]
    m, k, n, p = w["m"], w["k"], w["n"], w["p"]
    alpha, beta = w["alpha"], w["beta"]
    i64 = w["dtype"] == "i64"
    dt = capi.WS_I64 if i64 else capi.WS_F64
    log("generating inputs %dx%dx%d p=%d" % (m, k, n, p))
    if i64:
        A, B, C = inputs.uniform(w["seed"], m, k, n, p, with_c=beta != 0)
    else:
        A, B, C = inputs.uniform_f64(w["seed"], m, k, n, p, with_c=beta != 0)
    dA, dB = ctx.to_dev(A), ctx.to_dev(B)
    dC = ctx.to_dev(C) if C is not None else torch.zeros((m, n), dtype=dA.dtype, device=ctx.dev)
    flops = 2.0 * m * n * k

    def mkargs(schedule, levels, base=capi.WS_BASE_F64_MFMA, ws=None, nbytes=0, blocks=0):
        return capi.make_args(m, k, n, p, dA, dB, dC, alpha, beta, schedule, levels, dtype=dt,
                              base=base, stream=ctx.stream, workspace=ws, workspace_bytes=nbytes,
                              blocks=blocks)

    def ws_for(schedule, levels, blocks=0):
        nbytes = capi.wsmul_plan_info(mkargs(schedule, levels, blocks=blocks)).workspace_bytes
        return torch.empty(max(nbytes // 8, 1), dtype=torch.float64, device=ctx.dev), nbytes

    def run(args):
        capi.check(capi.wsmul_mod_p_ex(args))

    extra = {}
    int8 = False
    blocks = 0
    lev_or = lambda d: d if a.levels is None else a.levels
    if name == "acc_4096_p65521_l3":
        sched, lev, base, label = capi.WS_TWO_TEMP, lev_or(3), capi.WS_BASE_F64_MFMA, \
            "table9-accumulate-two-temporaries"
        config = {"workload": name, "m": m, "k": k, "n": n, "p": p, "op": "C <- A*B + C",
                  "schedule": label, "levels": lev, "base": "f64 matrix cores",
                  "parallelism": "single GPU"}
    elif name == "overwrite_8192x16384x8192_p8388593":
        sched, lev, base = capi.WS_OVERWRITE, lev_or(1), capi.WS_BASE_F64_MFMA
        config = {"workload": name, "m": m, "k": k, "n": n, "p": p, "op": "C = A*B",
                  "schedule": "algorithm1-in-place-overwrite-rectangular", "levels": lev,
                  "base": "f64 matrix cores", "inputs": "A and B restored from copies "
                  "before each step, outside the timed window", "parallelism": "single GPU"}
    elif name == "acc_4096_p65521_blocked":
        sched, lev, base, blocks = capi.WS_BLOCKED_ACC, lev_or(2), capi.WS_BASE_F64_MFMA, \
            a.blocks
        config = {"workload": name, "m": m, "k": k, "n": n, "p": p, "op": "C <- A*B + C",
                  "schedule": "section7.2-blocked-accumulation-table9", "blocks": blocks,
                  "levels": lev, "base": "f64 matrix cores", "parallelism": "single GPU"}
    elif name == "t1_512_p65521_l1_i64":
        sched, lev, base = capi.WS_TWO_TEMP, 1, capi.WS_BASE_F64_MFMA
        config = {"workload": name, "m": m, "k": k, "n": n, "p": p, "op": "C = A*B",
                  "schedule": "table1-two-temporaries", "levels": lev,
                  "base": "f64 matrix cores", "storage": "int64", "parallelism": "single GPU"}
    elif name == "ipmm_8192x4096x8192_p8388593":
        sched, lev, base = capi.WS_READONLY_INPLACE, 1, capi.WS_BASE_F64_MFMA
        config = {"workload": name, "m": m, "k": k, "n": n, "p": p, "op": "C = A*B",
                  "schedule": "algorithm2-readonly-inplace", "levels": lev,
                  "base": "f64 matrix cores", "parallelism": "single GPU"}
    else:   # t1_16384_p1048573: the autotuner decides
        st, sched, lev, base, _ = capi.wsmul_autotune(m, k, n, p, dt, 2 ** 62, capi.WS_AUTO, -1,
                                                      capi.WS_BASE_AUTO, beta)
        capi.check(st)
        int8 = base == capi.WS_BASE_I8_LIMBS
        config = {"workload": name, "m": m, "k": k, "n": n, "p": p, "op": "C = A*B",
                  "schedule": "autotuned: " + SCHEDULE_NAMES.get(sched, str(sched)),
                  "levels": lev,
                  "base": "int8 digits (3 balanced base-256 digits)" if int8
                  else "f64 matrix cores", "parallelism": "single GPU"}

    ws, nbytes = ws_for(sched, lev, blocks)
    head = mkargs(sched, lev, base, ws, nbytes, blocks)
    steps, warmup = a.steps, a.warmup
    log("timing %d steps (%s, %d levels)" % (steps, config["schedule"], lev))
    overwrites = sched in (capi.WS_OVERWRITE, capi.WS_OVR, capi.WS_ACCR, capi.WS_OVL,
                           capi.WS_ACR)
    if overwrites:
        # each step starts from the pristine inputs; the copies are not timed
        A0, B0 = dA.clone(), dB.clone()

        def restore():
            dA.copy_(A0)
            dB.copy_(B0)
        for _ in range(warmup):
            restore()
            run(head)
        ms_step = ctx.event_ms(lambda: run(head), steps, restore)
    else:
        ms_step = ctx.timed(lambda: run(head), steps, warmup)
    stats = capi.wsmul_get_stats()
    value = flops / (ms_step * 1e-3) / 1e9
    log("%s: %.3f ms/step, %.1f Gop/s, temporaries %d B" % (name, ms_step, value,
                                                           stats.workspace_bytes))
    roof, per_step, counts, add_roof = ctx.traced(head, max(1, min(steps, 5)), int8_ops=int8)
    if add_roof is not None and roof["bound"] != "hbm":
        extra["roofline_additions"] = add_roof
    if ctx.split_roof is not None:
        extra["roofline_digit_splits"] = ctx.split_roof
    extra["peak_temp_bytes"] = int(stats.workspace_bytes)
    if stats.scratch_bytes:
        extra["digit_scratch_bytes"] = int(stats.scratch_bytes)
    if nbytes > 0:
        # Device-measured temporaries: one more call on a workspace filled,
        # with a guard band behind it, by a value that is not a residue.
        guard = 4096
        wsg = torch.full((nbytes // 8 + guard,), -7, dtype=dA.dtype, device=ctx.dev)
        if overwrites:
            restore()
        run(mkargs(sched, lev, base, wsg, nbytes, blocks))
        torch.cuda.synchronize()
        w = wsg.cpu().numpy()
        extra["temp_bytes_touched"] = int(np.count_nonzero(w[:nbytes // 8] != -7) * 8)
        extra["temp_guard_intact"] = bool(np.all(w[nbytes // 8:] == -7))
        del wsg
    extra["launches_per_step"] = counts
    extra["kernel_time_per_step_ms"] = per_step
    del ws

    if not a.no_compare:
        reps = max(3, steps // 2)

        def compare(key, schedule, levels, base=capi.WS_BASE_F64_MFMA, restore=False, blocks=0):
            w2, nb2 = (ws_for(schedule, levels, blocks) if schedule != capi.WS_CLASSICAL
                       else (None, 0))
            args2 = mkargs(schedule, levels, base, w2, nb2, blocks)
            run(args2)
            torch.cuda.synchronize()
            before = None
            if restore:
                A0, B0 = dA.clone(), dB.clone()

                def before():
                    dA.copy_(A0)
                    dB.copy_(B0)
            if before is None:
                # the same back-to-back timing as the headline
                ms = ctx.timed(lambda: run(args2), reps, 1)
            else:
                ms = ctx.event_ms(lambda: run(args2), reps, before)
            extra[key] = {"ms_per_step": round(ms, 4),
                          "gops": round(flops / (ms * 1e-3) / 1e9, 2),
                          "peak_temp_bytes": int(nb2)}
            st2 = capi.wsmul_get_stats()
            if st2.scratch_bytes:
                extra[key]["digit_scratch_bytes"] = int(st2.scratch_bytes)
            log("%s: %.3f ms, %.1f Gop/s" % (key, ms, flops / (ms * 1e-3) / 1e9))
            return ms

        if name == "t1_16384_p1048573":
            # Classical on both bases; Winograd (Table 1) on each base at its
            # best depth; the speed-up is against the faster classical product.
            cl_f64 = compare("classical_f64", capi.WS_CLASSICAL, 0)
            cl_i8 = compare("classical_int8_digits", capi.WS_CLASSICAL, 0, capi.WS_BASE_I8_LIMBS)
            t1_i8 = compare("table1_1_level_int8_digits", capi.WS_TWO_TEMP, 1,
                            capi.WS_BASE_I8_LIMBS)
            t1_f64 = compare("table1_2_levels_f64", capi.WS_TWO_TEMP, 2)
            cl_ms = min(cl_f64, cl_i8)
            extra["fastest_classical"] = ("classical_int8_digits" if cl_i8 <= cl_f64
                                          else "classical_f64")
            extra["winograd_vs_classical_same_base"] = {
                "f64 (Table 1, 2 levels)": round(cl_f64 / t1_f64, 4),
                "int8 digits (Table 1, 1 level)": round(cl_i8 / t1_i8, 4)}
        else:
            cl_ms = compare("classical", capi.WS_CLASSICAL, 0)
        if name == "acc_4096_p65521_l3":
            compare("overwrite_table6", capi.WS_OVERWRITE, lev, restore=True)
        elif name == "ipmm_8192x4096x8192_p8388593":
            compare("two_temporaries_table1", capi.WS_TWO_TEMP, 1)
        elif name == "overwrite_8192x16384x8192_p8388593":
            compare("algorithm1_2_levels", capi.WS_OVERWRITE, 2, restore=True)
            compare("table1_1_level", capi.WS_TWO_TEMP, 1)
            compare("algorithm2_1_level", capi.WS_READONLY_INPLACE, 1)
        elif name == "acc_4096_p65521_blocked":
            compare("table9_unblocked_3_levels", capi.WS_TWO_TEMP, 3)
            compare("blocked_t2_table2_2_levels", capi.WS_BLOCKED, 2, blocks=2)
            compare("blocked_t2_table2_1_level", capi.WS_BLOCKED, 1, blocks=2)
            compare("blocked_t2_table9_1_level", capi.WS_BLOCKED_ACC, 1, blocks=2)
            compare("blocked_t3_table2_1_level", capi.WS_BLOCKED, 1, blocks=3)
            compare("blocked_t4_table9_1_level", capi.WS_BLOCKED_ACC, 1, blocks=4)
        extra["speedup_vs_classical"] = round(cl_ms / ms_step, 4)

    cpu = None
    if not a.no_cpu:
        cpu = cpu_baseline_rows(A, B, C, alpha, beta, p)
    # the arithmetic type: 8-bit digit products (int32 sums) on the digit base
    dtype = "i8" if config.get("base", "").startswith("int8") else ("int64" if i64 else "f64")
    if dtype == "i8":
        config["storage"] = "int64" if i64 else "f64"
    return line(ctx, value, ms_step, dtype, config, roof, cpu, extra)


def batch_2000(ctx):
    """2000 autotuned products in one captured graph; one step is one replay."""
    capi, inputs, torch = ctx.capi, ctx.inputs, ctx.torch
    a = ctx.args
    probs = inputs.batch_problems()
    log("generating %d batch products" % len(probs))
    args, keep = [], []
    flops = 0.0
    for pr in probs:
        m, k, n, p = pr["m"], pr["k"], pr["n"], pr["p"]
        A, B = inputs.batch_inputs(pr)
        dA, dB = ctx.to_dev(A), ctx.to_dev(B)
        dC = torch.empty((m, n), dtype=torch.float64, device=ctx.dev)
        keep.append((dA, dB, dC))
        flops += 2.0 * m * n * k
        args.append(capi.make_args(m, k, n, p, dA, dB, dC, 1, 0, capi.WS_AUTO, -1,
                                   base=capi.WS_BASE_F64_MFMA, stream=ctx.stream))
    st, handle = capi.wsmul_graph_capture(args)
    capi.check(st)
    stats = capi.wsmul_get_stats()
    phases = capi.wsmul_get_stats().batch_phases
    try:
        def replay():
            capi.check(capi.wsmul_graph_launch(handle, ctx.stream))
        log("timing %d graph replays" % a.steps)
        ms_step = ctx.timed(replay, a.steps, a.warmup)
        value = flops / (ms_step * 1e-3) / 1e9
        log("batch: %.3f ms/replay, %.1f Gop/s" % (ms_step, value))
        ach = flops / (ms_step * 1e-3) / 1e12
        roof = {"bound": "mfma", "kernel": "batch_kernel (persistent; one launch per phase, "
                "%d phases, phase 0 holds every classical product)" % phases,
                "achieved": round(ach, 3), "peak": PEAK_F64_MFMA_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / PEAK_F64_MFMA_TFLOPS, 4), "traffic": None,
                "avg_launch_ms": None, "flops_per_replay": flops}
        extra = {"peak_temp_bytes": int(stats.workspace_bytes),
                 "device_block_bytes": int(stats.internal_alloc_bytes), "phases": int(phases)}
        if not a.no_compare:
            def separate():
                for x in args:
                    capi.check(capi.wsmul_mod_p_ex(x))
            ms2 = ctx.event_ms(separate, 2)
            extra["separate_calls"] = {"ms_per_step": round(ms2, 3),
                                       "gops": round(flops / (ms2 * 1e-3) / 1e9, 2)}
            log("separate calls: %.3f ms" % ms2)
    finally:
        capi.wsmul_graph_destroy(handle)
    cpu = None
    if not a.no_cpu:
        # The products in order, their inputs regenerated from the seed,
        # until 12 s of oracle time (the generation is not timed).
        from oracle import ref
        threads = ref.threads_available()
        done, fl, dt = 0, 0.0, 0.0
        for pr in probs:
            A, B = inputs.batch_inputs(pr)
            Ai, Bi = A.astype(np.int64), B.astype(np.int64)
            t_s = time.perf_counter()
            ref.matmul_mod_p(Ai, Bi, None, 1, 0, pr["p"], threads=threads)
            dt += time.perf_counter() - t_s
            done += 1
            fl += 2.0 * pr["m"] * pr["k"] * pr["n"]
            if dt > 12.0:
                break
        cpu = {"value": round(fl / dt / 1e9, 3), "unit": "Gop/s", "cores": threads,
               "cpu": cpu_model(), "kind": "oracle", "sample": "the first %d of the 2000 products, %.1f s"
                                           % (done, dt)}
    config = {"workload": "batch_2000", "products": len(probs), "sizes": "m, k, n log-uniform "
              "in [64, 2048]", "moduli": list(inputs.PRIMES), "op": "C = A*B",
              "schedule": "autotuned per product", "base": "f64 matrix cores",
              "launch": "hipGraph of persistent batched launches", "parallelism": "single GPU"}
    return line(ctx, value, ms_step, "f64", config, roof, cpu, extra)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--levels", type=int, default=None,
                    help="Winograd levels of the 4096^3 accumulation (default 3; 2 when "
                         "blocked) and of the Algorithm 1 workload (default 1)")
    ap.add_argument("--blocks", type=int, default=2,
                    help="t of the blocked accumulation workload")
    ap.add_argument("--workload", default=WORKLOADS[0], choices=WORKLOADS)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-compare", action="store_true", help="skip the comparator schedules")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run plain device copies of MIB MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 8, "copies": 5}))
        return

    ctx = Ctx(args)
    if args.workload == "batch_2000":
        out = batch_2000(ctx)
    else:
        out = single_product(ctx, args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
