"""Benchmark: exact Winograd products over Z/pZ on one MI355X.

Default workload: C <- A*B + C mod 65521 with m = k = n = 4096, three
Winograd levels under the read-only two-temporary accumulating schedule
(Table 9), binary64 matrix-core base case.  One step is one such product on
inputs already resident in HBM.  The same workload is also timed under the
input-overwriting accumulating schedule (Table 6; A and B are restored from
pristine copies outside the timed window) and as one classical product.

Prints one JSON line on stdout.  Extra fields: the peak temporary bytes of
each schedule, the comparator rates, a roofline entry for the dominant kernel
class (time from events on the launch stream), and the oracle's rate on a
bounded sample of the same product on the host cores.
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
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernels_digest():
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels.hip", "gemm_common.hpp", "device.hpp"):
        with open(os.path.join(ROOT, "paper_0707_2347_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(gemm_dominant):
    """HBM bytes per launch of the dominant kernel, from the FETCH_SIZE and
    WRITE_SIZE counter runs recorded in profiles/ (scaled by the plain-copy
    calibration there); None when the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", "traffic_acc_4096_p65521_l3.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernels_digest") != kernels_digest():
        return None
    key = "base_product" if gemm_dominant else "addition_group"
    return rec.get(key, {}).get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--levels", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-compare", action="store_true", help="skip the comparator schedules")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run plain device copies of MIB MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_0707_2347_amd import capi, inputs

    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 8, "copies": 5}))
        return

    w = inputs.WORKLOADS["acc_4096_p65521_l3"]
    m, k, n, p = w["m"], w["k"], w["n"], w["p"]
    L = args.levels
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    log("generating inputs %dx%dx%d p=%d" % (m, k, n, p))
    A, B, C = inputs.uniform_f64(w["seed"], m, k, n, p, with_c=True)
    dA = torch.from_numpy(A).to(dev)
    dB = torch.from_numpy(B).to(dev)
    dC = torch.from_numpy(C).to(dev)
    A0, B0 = dA.clone(), dB.clone()

    def ws_for(schedule):
        nbytes = capi.wsmul_workspace_bytes(m, k, n, capi.WS_F64, schedule, L, 1)
        buf = torch.empty(max(nbytes // 8, 1), dtype=torch.float64, device=dev)
        return buf, nbytes

    def mkargs(schedule, ws, nbytes, flags=0):
        return capi.make_args(m, k, n, p, dA, dB, dC, 1, 1, schedule, L, stream=stream,
                              workspace=ws, workspace_bytes=nbytes, flags=flags)

    flops = 2.0 * m * n * k

    # ---------------------------------------------------- headline: Table 9
    ws, nbytes = ws_for(capi.WS_TWO_TEMP)
    a_acc = mkargs(capi.WS_TWO_TEMP, ws, nbytes)
    for _ in range(args.warmup):
        capi.check(capi.wsmul_mod_p_ex(a_acc))
    torch.cuda.synchronize()
    log("timing %d steps (table 9, %d levels)" % (args.steps, L))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        capi.check(capi.wsmul_mod_p_ex(a_acc))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    stats = capi.wsmul_get_stats()
    value = flops / (ms_step * 1e-3) / 1e9
    log("table 9: %.3f ms/step, %.1f Gop/s, temporaries %d B" % (ms_step, value,
                                                                  stats.workspace_bytes))

    # kernel-class times from events on the launch stream (separate traced steps)
    capi.wsmul_reset_stats()
    traced = mkargs(capi.WS_TWO_TEMP, ws, nbytes, flags=capi.WS_FLAG_TRACE)
    ntraced = max(1, min(args.steps, 5))
    for _ in range(ntraced):
        capi.check(capi.wsmul_mod_p_ex(traced))
    tr = capi.wsmul_get_trace()
    gemm_avg_ms = tr.gemm_ms / max(tr.gemm_launches, 1)
    add_avg_ms = tr.add_ms / max(tr.add_launches, 1)
    gemm_flops_per = tr.gemm_flops / max(tr.gemm_launches, 1)
    add_bytes_per = tr.add_bytes / max(tr.add_launches, 1)
    gemm_tfs = gemm_flops_per / (gemm_avg_ms * 1e-3) / 1e12
    add_gbs = add_bytes_per / (add_avg_ms * 1e-3) / 1e9
    log("trace: base products %d x %.4f ms (%.2f TFLOP/s), additions %d x %.4f ms (%.0f GB/s)"
        % (tr.gemm_launches, gemm_avg_ms, gemm_tfs, tr.add_launches, add_avg_ms, add_gbs))
    traffic = measured_traffic(tr.gemm_ms >= tr.add_ms)
    if tr.gemm_ms >= tr.add_ms:
        roofline = {"bound": "mfma", "kernel": "base product (f64 16x16x4 matrix cores)",
                    "achieved": round(gemm_tfs, 3), "peak": PEAK_F64_MFMA_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(gemm_tfs / PEAK_F64_MFMA_TFLOPS, 4),
                    "traffic": traffic, "avg_launch_ms": round(gemm_avg_ms, 5),
                    "flops_per_launch": gemm_flops_per}
    else:
        roofline = {"bound": "hbm", "kernel": "fused addition rows",
                    "achieved": round(add_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": round(add_gbs / PEAK_HBM_GBS, 4), "traffic": traffic,
                    "avg_launch_ms": round(add_avg_ms, 5), "bytes_per_launch": add_bytes_per}
    del ws

    extra = {"peak_temp_bytes": int(stats.workspace_bytes),
             "launches_per_step": {"base_products": int(stats.gemm_launches),
                                   "addition_groups": int(stats.add_launches)},
             "kernel_time_per_step_ms": {"base_products": round(tr.gemm_ms / ntraced, 4),
                                         "additions": round(tr.add_ms / ntraced, 4)}}

    # ---------------------------------------------------- comparators
    if not args.no_compare:
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        # classical: one base product over the whole shape
        a_cl = mkargs(capi.WS_CLASSICAL, None, 0)
        capi.check(capi.wsmul_mod_p_ex(a_cl))
        torch.cuda.synchronize()
        reps = max(3, args.steps // 2)
        ev0.record()
        for _ in range(reps):
            capi.check(capi.wsmul_mod_p_ex(a_cl))
        ev1.record()
        torch.cuda.synchronize()
        cl_ms = ev0.elapsed_time(ev1) / reps
        extra["classical"] = {"ms_per_step": round(cl_ms, 4),
                              "gops": round(flops / (cl_ms * 1e-3) / 1e9, 2),
                              "peak_temp_bytes": 0}
        log("classical: %.3f ms, %.1f Gop/s" % (cl_ms, flops / (cl_ms * 1e-3) / 1e9))
        # Table 6 (overwrites A and B): restore the inputs outside the window
        ws6, nb6 = ws_for(capi.WS_OVERWRITE)
        a_ov = mkargs(capi.WS_OVERWRITE, ws6, nb6)
        tot = 0.0
        for i in range(reps + 1):
            dA.copy_(A0)
            dB.copy_(B0)
            ev0.record()
            capi.check(capi.wsmul_mod_p_ex(a_ov))
            ev1.record()
            torch.cuda.synchronize()
            if i > 0:
                tot += ev0.elapsed_time(ev1)
        ov_ms = tot / reps
        extra["overwrite_table6"] = {"ms_per_step": round(ov_ms, 4),
                                     "gops": round(flops / (ov_ms * 1e-3) / 1e9, 2),
                                     "peak_temp_bytes": int(nb6)}
        extra["speedup_vs_classical"] = round(cl_ms / ms_step, 4)
        log("table 6: %.3f ms, %.1f Gop/s" % (ov_ms, flops / (ov_ms * 1e-3) / 1e9))
        del ws6

    # ---------------------------------------------------- CPU baseline
    cpu = None
    if not args.no_cpu:
        from oracle import ref
        threads = ref.threads_available()
        Ai = A.astype(np.int64)
        Bi = B.astype(np.int64)
        Ci = C.astype(np.int64)
        rows = 16
        t_s = time.perf_counter()
        ref.matmul_mod_p(Ai[:rows], Bi, Ci[:rows], 1, 1, p, threads=threads)
        dt = time.perf_counter() - t_s
        rows = int(min(m, max(16, rows * 12.0 / max(dt, 1e-3))))
        reps = 1 if rows < m else max(1, int(10.0 / max(dt * m / 16.0, 1e-3)))
        log("cpu baseline: oracle on %d rows x %d x %d, %d threads, %d run(s)"
            % (rows, k, n, threads, reps))
        t_s = time.perf_counter()
        for _ in range(reps):
            ref.matmul_mod_p(Ai[:rows], Bi, Ci[:rows], 1, 1, p, threads=threads)
        dt = (time.perf_counter() - t_s) / reps
        cpu = {"value": round(2.0 * rows * k * n / dt / 1e9, 3), "unit": "Gop/s",
               "cores": threads, "kind": "oracle",
               "sample": "rows 0..%d of the same product (%d x %d x %d), %d run(s) of %.1f s"
                         % (rows - 1, rows, k, n, reps, dt)}

    out = {"metric": "mod-p matmul effective Gop/s (2mnk/s) + peak temp bytes vs classical "
                     "mod-p GEMM",
           "value": round(value, 3), "unit": "Gop/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "acc_4096_p65521_l3", "m": m, "k": k, "n": n, "p": p,
                      "op": "C <- A*B + C", "schedule": "table9-accumulate-two-temporaries",
                      "levels": L, "base": "f64 matrix cores", "parallelism": "single GPU"},
           "roofline": roofline, "cpu_baseline": cpu}
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
