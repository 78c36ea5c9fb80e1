"""Benchmark of the NGS-FAS Richards solver on one MI355X.

A step is one BDF time step of the 3-D Haverkamp drainage block (257^3 nodes,
BDF2, dt = 120 s, FP64): step set-up (lagged K*, history, right-hand side on
every level), FAS V(2,2) cycles with red-black NGS (3 Newton steps per cell,
32 sweeps on the coarsest level) until the residual reaches the tolerance or
stops decreasing, and the history update.  Warm-up steps advance the same time
loop.  The state is resident in HBM throughout; only one residual norm per
cycle crosses to the host.

Printed: one JSON line with the NGS cell-update rate (all levels) over the
timed steps, the roofline of the finest-level sweep kernel (HIP events on the
library's stream around every finest-level sweep launch inside the timed
steps), and the CPU oracle timed on the host on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = 32.0   # FP64 sweep: read psi, K*, g and write psi, 8 B each


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_run(args):
    import torch
    import paper_2606_04292_amd as rsl
    from paper_2606_04292_amd import workloads as W

    torch.cuda.set_device(0)
    if args.copy_calibration:
        # a plain device copy of known size, for scaling HBM byte counters
        src = torch.empty(64 << 20, dtype=torch.float64, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: %d bytes read, %d bytes written" % (src.numel() * 8, src.numel() * 8))
        del src, dst
    w = W.config3(args.n)
    G = rsl.Grid(w, device="cuda:0")
    opts = rsl.solve_opts(w.nu1, w.nu2, w.nu_coarse, max_cycles=args.max_cycles,
                          tol_abs=args.tol, stagnation=1)
    for s in range(args.warmup):
        code, st = G.bdf_step(opts=opts)
        log("warmup step %d: code %d cycles %d res %.2e" % (s, code, st.cycles, st.res))
        if code != rsl.RS_OK:
            raise SystemExit("warm-up step failed: " + rsl.lib().rs_last_error().decode())
    G.profile_enable(True)
    G.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    updates = 0.0
    cycles = []
    for s in range(args.steps):
        code, st = G.bdf_step(opts=opts)
        if code != rsl.RS_OK:
            raise SystemExit("timed step failed: " + rsl.lib().rs_last_error().decode())
        updates += st.cell_updates
        cycles.append(st.cycles)
        log("timed step %d: cycles %d res %.2e updates %.3e" % (s, st.cycles, st.res,
                                                                 st.cell_updates))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sweep_ms, launches, sweep_cells = G.profile_read(reset=True)
    G.profile_enable(False)
    psi_fp64 = G.get_state()[0]
    avg_launch_s = sweep_ms * 1e-3 / max(launches, 1)
    bytes_per_launch = BYTES_PER_UPDATE * sweep_cells / max(launches, 1)
    achieved = bytes_per_launch / avg_launch_s / 1e9
    mixed = None
    if not args.no_mixed:
        # the same steps with FP32 correction cycles inside FP64 defect correction
        H = rsl.Grid(w, precision=rsl.RS_MIXED, device="cuda:0")
        for s in range(args.warmup):
            H.bdf_step(opts=opts)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        mup, outer = 0.0, []
        for s in range(args.steps):
            code, st = H.bdf_step(opts=opts)
            if code != rsl.RS_OK:
                raise SystemExit("mixed step failed: " + rsl.lib().rs_last_error().decode())
            mup += st.cell_updates
            outer.append(st.cycles)
        torch.cuda.synchronize()
        el2 = time.perf_counter() - t1
        psi_mp = H.get_state()[0]
        err = float((psi_mp - psi_fp64).abs().max() / psi_fp64.abs().max())
        mixed = {"ms_per_step": round(el2 * 1e3 / args.steps, 3),
                 "speedup_vs_fp64": round(elapsed / el2, 3),
                 "fp32_cell_updates_per_s": mup / el2,
                 "outer_corrections_per_step": outer,
                 "rel_err_vs_fp64": err,
                 "note": "same steps and tolerance; FP64 path is parity-tested against the oracle"}
        log("mixed: %.2f ms/step, rel diff vs FP64 %.2e" % (el2 * 1e3 / args.steps, err))
        H.close()
    res = dict(
        w=w, elapsed=elapsed, updates=updates, cycles=cycles, mixed=mixed,
        roofline={"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                  "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                  "kernel": "k_sweep_colour (finest level, one colour per launch)",
                  "avg_launch_us": round(avg_launch_s * 1e6, 2),
                  "bytes_per_launch": bytes_per_launch, "launches": launches,
                  "sweep_updates_per_s": sweep_cells / (sweep_ms * 1e-3)},
    )
    G.close()
    return res


def cpu_baseline(args, n):
    import numpy as np
    import oracle
    from paper_2606_04292_amd import workloads as W

    w = W.config3(n)
    S = oracle.Solver(w, oracle.ORDER_RB)
    unk = [int((S.kinds(l) == 0).sum()) for l in range(S.nlev)]
    per_cycle = sum((w.nu1 + w.nu2) * u for u in unk[:-1]) + w.nu_coarse * unk[-1]
    t0 = time.perf_counter()
    S.begin_step()
    cycles = 0
    while True:
        S.vcycle()
        S.residual()
        cycles += 1
        if time.perf_counter() - t0 >= args.cpu_seconds:
            break
    el = time.perf_counter() - t0
    return {"value": per_cycle * cycles / el, "unit": "cell-updates/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": "first BDF step of the same %d^3 block: set-up + %d FAS V(2,2) cycles "
                      "(red-black, OpenMP) with a residual norm after each, %.1f s" % (n, cycles, el)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=257, help="nodes per axis (2^k+1)")
    ap.add_argument("--tol", type=float, default=1e-13, help="residual max-norm tolerance (1/s)")
    ap.add_argument("--max-cycles", type=int, default=40)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 512 MiB device copy first (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    r = gpu_run(args)
    w = r["w"]
    ms = r["elapsed"] * 1e3 / args.steps
    out = {
        "metric": "NGS cell-updates/s + HBM-roofline % at 257^3",
        "value": r["updates"] / r["elapsed"],
        "unit": "cell-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "%s: %d^3 nodes, Haverkamp, BDF2 dt=%g s, FAS V(%d,%d), "
                               "red-black NGS, %d Newton steps/cell, tol %.0e" % (
                                   w.name, args.n, w.dt, w.nu1, w.nu2, w.law.newton_iters,
                                   args.tol),
                   "nodes": args.n ** 3, "cycles_per_step": r["cycles"],
                   "parallelism": "single GPU"},
        "roofline": r["roofline"],
    }
    if r["mixed"] is not None:
        out["mixed_precision"] = r["mixed"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, args.n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
