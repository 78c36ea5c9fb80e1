"""Benchmark of the NGS-FAS Richards solver on one MI355X.

A step is one BDF time step of the 3-D Haverkamp drainage block (257^3 nodes,
BDF2, dt = 120 s, FP64): step set-up (lagged K*, history, right-hand side on
every level), FAS V(2,2) cycles with red-black NGS (at most 3 Newton steps per
cell, 32 sweeps on the coarsest level) until the residual reaches the
tolerance or the rounding floor, and the history update.  The timed region is
steps 1..K of the configuration's 20-step time loop from t = 0 (K = --steps,
20 by default: the whole configuration); the warm-up steps run first and the
state is then reset to t = 0.  The state is resident in HBM throughout; only
one residual norm per cycle crosses to the host.

Printed: one JSON line with the NGS cell-update rate (all levels) over the
timed steps, the cycles and final residual of every step, the roofline of the
finest-level sweep kernel (HIP events on the library's stream around every
finest-level sweep launch inside the timed steps), the same steps in mixed
precision, the serving stream, and the CPU oracle timed on the host on a
bounded sample.
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
BYTES_PER_UPDATE_32 = 20.0   # FP32 correction sweep: read delta, K*, rhs, psi_b and write delta, 4 B each


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "sweep_fp64_block3d_haverkamp_257_traffic.md")
COUNTERS_PROFILE = os.path.join(ROOT, "profiles", "sweep_fp64_block3d_haverkamp_257_counters.md")


# The translation units of the FP64 and FP32 sweep kernels: their counters
# stay valid while these sources are unchanged.
SWEEP_SOURCES = ["kernels_fp64.hip", "rs_internal.h", "soil_device.h", "grid_device.h",
                 "transfer.h", "cell64.h"]
SWEEP32_SOURCES = ["kernels_mp.hip", "rs_internal.h", "soil_device.h", "grid_device.h",
                   "transfer.h", "soil_mp.h", "cell32.h"]


def kernel_sources_sha256(sources=SWEEP_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for name in sources:
        p = os.path.join(ROOT, "paper_2606_04292_amd", "csrc", name)
        h.update(name.encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profiled_value(path, key, sources=SWEEP_SOURCES):
    """The number recorded as `key=value kernel_sources_sha256=...` in a
    committed counter summary, or None when the summary is missing or the
    kernel sources changed since the counters were taken."""
    import re
    try:
        with open(path) as f:
            m = re.search(key + r"=([0-9.]+) kernel_sources_sha256=([0-9a-f]+)", f.read())
    except OSError:
        return None
    if not m or m.group(2) != kernel_sources_sha256(sources):
        return None
    return float(m.group(1))


def profiled_traffic(key="sweep_traffic_bytes", sources=SWEEP_SOURCES):
    """Calibrated HBM bytes (read + write) per finest-level sweep launch."""
    v = profiled_value(TRAFFIC_PROFILE, key, sources)
    return None if v is None else int(v)


def profiled_valu_busy(key="sweep_valu_busy_pct", sources=SWEEP_SOURCES):
    """VALUBusy (%) of the finest-level sweep launches."""
    return profiled_value(COUNTERS_PROFILE, key, sources)


def time_loop(G, w, psi0, steps, opts, label):
    """Steps 1..steps of the configuration's time loop from t = 0 (after every
    w.steps steps the loop starts again from psi0, so any step count runs the
    configuration as stated).  A step that ends without convergence is recorded
    and its last iterate accepted so that the loop goes on; a non-finite
    residual ends the loop.  Returns per-step (status, cycles, res, updates)."""
    import paper_2606_04292_amd as rsl
    out = []
    for s in range(steps):
        if s % w.steps == 0 and s > 0:
            G.set_state(psi0)
        code, st = G.bdf_step(opts=opts)
        out.append((code, st.cycles, st.res, st.cell_updates))
        log("%s step %d: code %d cycles %d res0 %.2e res %.2e updates %.3e" % (
            label, s + 1, code, st.cycles, st.res0, st.res, st.cell_updates))
        if code == rsl.RS_ENOTCONV:
            G.end_step()
        elif code != rsl.RS_OK:
            break
    return out


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
    psi0 = torch.as_tensor(w.psi0, device="cuda:0")
    G = rsl.Grid(w, device="cuda:0")
    opts = rsl.solve_opts(w.nu1, w.nu2, w.nu_coarse, max_cycles=args.max_cycles,
                          tol_abs=args.tol, stagnation=1, mp_inner_cycles=args.mp_inner)
    # warm-up: the first steps of the same time loop, then back to t = 0
    warm = time_loop(G, w, psi0, args.warmup, opts, "warmup")
    G.set_state(psi0)
    G.profile_enable(True)
    G.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = time_loop(G, w, psi0, args.steps, opts, "fp64")
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
        mwarm = time_loop(H, w, psi0, args.warmup, opts, "mixed warmup")
        H.set_state(psi0)
        H.profile_enable(True)
        H.profile_read(reset=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        msteps = time_loop(H, w, psi0, args.steps, opts, "mixed")
        torch.cuda.synchronize()
        el2 = time.perf_counter() - t1
        ms32, l32, c32 = H.profile_read(reset=True)
        H.profile_enable(False)
        psi_mp = H.get_state()[0]
        err = float((psi_mp - psi_fp64).abs().max() / psi_fp64.abs().max())
        t32 = ms32 * 1e-3 / max(l32, 1)
        b32 = BYTES_PER_UPDATE_32 * c32 / max(l32, 1)
        mbad = [k + 1 for k, x in enumerate(msteps) if x[0] != rsl.RS_OK]
        tr32 = profiled_traffic("sweep32_traffic_bytes", SWEEP32_SOURCES)
        mixed = {"ms_per_step": round(el2 * 1e3 / args.steps, 3),
                 "speedup_vs_fp64": round(elapsed / el2, 3),
                 "fp32_cell_updates_per_s": sum(x[3] for x in msteps) / el2,
                 "outer_corrections_per_step": [x[1] for x in msteps],
                 "fp32_cycles_per_correction": args.mp_inner,
                 "steps_not_converged": mbad,
                 "warmup_ok": all(x[0] == rsl.RS_OK for x in mwarm),
                 "rel_err_vs_fp64": err,
                 "fp32_sweep_roofline": {"bound": "hbm", "achieved": round(b32 / t32 / 1e9, 1),
                                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                         "frac": round(b32 / t32 / 1e9 / HBM_PEAK_GBS, 4),
                                         "kernel": "k_sweep32_pair (finest level, one colour per launch, two nodes per lane)",
                                         "bytes_per_update": BYTES_PER_UPDATE_32,
                                         "traffic": tr32,
                                         "traffic_per_algorithmic": (round(tr32 / b32, 3)
                                                                     if tr32 else None),
                                         "valu_busy_pct": profiled_valu_busy(
                                             "sweep32_valu_busy_pct", SWEEP32_SOURCES),
                                         "avg_launch_us": round(t32 * 1e6, 2), "launches": l32},
                 "note": "the same %d steps from t = 0 to the same tolerance; rel_err_vs_fp64 = "
                         "max|psi_MP - psi_FP64| / max|psi_FP64| after the last step" % args.steps}
        log("mixed: %.2f ms/step, rel diff vs FP64 %.2e" % (el2 * 1e3 / args.steps, err))
        H.close()
    traffic = profiled_traffic()
    res = dict(
        w=w, elapsed=elapsed, updates=sum(x[3] for x in steps), steps=steps, mixed=mixed,
        warmup_ok=all(x[0] == rsl.RS_OK for x in warm),
        roofline={"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                  "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                  "traffic_per_algorithmic": (round(traffic / bytes_per_launch, 3)
                                              if traffic else None),
                  "traffic_source": os.path.relpath(TRAFFIC_PROFILE, ROOT),
                  "valu_busy_pct": profiled_valu_busy(),
                  "counters_source": os.path.relpath(COUNTERS_PROFILE, ROOT),
                  "kernel": "k_sweep_pair (finest level, one colour per launch, two nodes per lane)",
                  "avg_launch_us": round(avg_launch_s * 1e6, 2),
                  "bytes_per_launch": bytes_per_launch, "launches": launches,
                  "sweep_updates_per_s": sweep_cells / (sweep_ms * 1e-3)},
    )
    G.close()
    return res


def serving_leg(args):
    """Continuous batching of the serving stream against one-at-a-time FP64.

    1. engine, closed loop: all requests present at t = 0; capacity
       C = requests / makespan;
    2. engine, open loop: Poisson arrivals at 0.7 C over the whole stream;
       per-request latency = completion - arrival, step-solves/s = steps of the
       finished requests / (last completion - first arrival); failed requests
       are counted apart and left out of both;
    3. one-at-a-time FP64 baseline on the first --serve-baseline requests:
       (a) back to back, which gives its capacity C_b (each request: grid set-up,
       rs_bdf_step to the rounding floor per step, result read back);
       (b) served first come first served against the wall clock on a Poisson
       trace at 0.7 C_b, a rate it sustains: measured latencies;
       (c) the engine on the same requests and the same arrival times;
       the engine's final states are compared with the FP64 results.
    """
    import numpy as np
    import torch
    import paper_2606_04292_amd as rsl
    from paper_2606_04292_amd import serve
    from paper_2606_04292_amd import workloads as W

    pct = lambda x, p: round(1e3 * float(np.percentile(x, p)), 2) if len(x) else None
    reqs = W.serving_requests(args.serve_requests)
    opts = serve.engine_opts()
    arena = int(args.serve_arena_gib * (1 << 30))
    E = serve.Engine(arena, opts, device="cuda:0")
    # warm-up: a few requests through the engine (graph, kernels, allocator)
    serve.run_stream(E, reqs[:16])
    _, comp, st, _ = serve.run_stream(E, reqs)
    makespan = float(np.nanmax(comp))
    cap = len(reqs) / makespan
    bad = [q for q, s in enumerate(st) if s[0] != rsl.RS_OK]
    log("serving closed loop: %d requests in %.3f s (%.1f req/s), %d failed" % (
        len(reqs), makespan, cap, len(bad)))
    rate = 0.7 * cap
    arr = W.poisson_arrivals(len(reqs), rate)
    arr2, comp2, st2, _ = serve.run_stream(E, reqs, arrivals=arr)
    ok2 = np.array([s[0] == rsl.RS_OK for s in st2])
    lat = (comp2 - arr2)[ok2]
    span = float(np.nanmax(comp2[ok2]) - arr2[0])
    steps_ok = sum(reqs[q].steps for q in range(len(reqs)) if ok2[q])
    log("serving open loop at %.1f req/s: p50 %.1f ms p99 %.1f ms, %d failed" % (
        rate, 1e3 * np.percentile(lat, 50), 1e3 * np.percentile(lat, 99), int((~ok2).sum())))

    # one-at-a-time FP64 on the first M requests
    M = min(args.serve_baseline, len(reqs))
    fp_opts = rsl.solve_opts(max_cycles=200, tol_abs=0.0, stagnation=1)

    def serve_one(w):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        G = rsl.Grid(w, device="cuda:0")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        code = rsl.RS_OK
        for _ in range(w.steps):
            code, _s = G.bdf_step(opts=fp_opts)
            if code != rsl.RS_OK:
                break
        psi = G.get_state()[0]
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        G.close()
        return code, psi, t1 - t0, t2 - t1

    setup, solve, bcodes = [], [], []
    tb = time.perf_counter()
    for q in range(M):
        code, _, a, b = serve_one(reqs[q])
        setup.append(a)
        solve.append(b)
        bcodes.append(code)
    cap_b = M / (time.perf_counter() - tb)
    rate_b = 0.7 * cap_b
    arr_b = W.poisson_arrivals(M, rate_b, seed_path=(3,))
    log("baseline closed loop: %d requests, %.1f req/s; open loop at %.1f req/s" % (M, cap_b, rate_b))
    # the engine on the same requests and arrival times
    arr_e, comp_e, st_e, kept = serve.run_stream(E, reqs[:M], arrivals=arr_b, keep=range(M))
    E.close()
    del E
    torch.cuda.empty_cache()
    # the baseline against the wall clock, first come first served
    lat_b, errs, codes_b = [], [], []
    t0 = time.perf_counter()
    for q in range(M):
        wait = arr_b[q] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        code, psi, _, _ = serve_one(reqs[q])
        lat_b.append(time.perf_counter() - t0 - arr_b[q])
        codes_b.append(code)
        if code == rsl.RS_OK and st_e[q][0] == rsl.RS_OK:
            errs.append(float((kept[q] - psi).abs().max() / psi.abs().max()))
    okb = np.array([c == rsl.RS_OK for c in codes_b])
    oke = np.array([s[0] == rsl.RS_OK for s in st_e])
    lat_b = np.array(lat_b)[okb]
    lat_e = (comp_e - arr_e)[oke]
    log("baseline open loop: p50 %.1f ms p99 %.1f ms; engine on the same trace: p50 %.1f ms "
        "p99 %.1f ms" % (1e3 * np.percentile(lat_b, 50), 1e3 * np.percentile(lat_b, 99),
                         1e3 * np.percentile(lat_e, 50), 1e3 * np.percentile(lat_e, 99)))
    return {
        "requests": len(reqs), "steps_per_request": reqs[0].steps,
        "step_solves_per_s": steps_ok / span,
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)},
        "arrival_rate_req_per_s": round(rate, 2),
        "closed_loop_capacity_req_per_s": round(cap, 2),
        "failed": {"closed_loop": len(bad), "open_loop": int((~ok2).sum())},
        "corrections_per_step": round(sum(s[2] for s in st2 if s[0] == rsl.RS_OK) / steps_ok, 2),
        "engine": {"precision": "FP32 correction cycles, FP64 defect/history",
                   "max_slots": opts.max_slots, "tail_nodes": opts.tail_nodes,
                   "rounds_per_tick": opts.rounds_per_tick, "graph": bool(opts.use_graph),
                   "arena_gib": args.serve_arena_gib},
        "baseline_one_at_a_time_fp64": {
            "requests": M,
            "closed_loop_capacity_req_per_s": round(cap_b, 2),
            "step_solves_per_s": round(cap_b * reqs[0].steps, 1),
            "arrival_rate_req_per_s": round(rate_b, 2),
            "latency_ms": {"p50": pct(lat_b, 50), "p99": pct(lat_b, 99)},
            "engine_latency_ms_same_trace": {"p50": pct(lat_e, 50), "p99": pct(lat_e, 99)},
            "service_ms": {"setup_mean": round(1e3 * float(np.mean(setup)), 2),
                           "solve_p50": pct(solve, 50), "solve_p99": pct(solve, 99)},
            "failed": {"baseline": int((~okb).sum()), "engine": int((~oke).sum())},
            "kind": "measured: requests served one at a time against the wall clock, first come "
                    "first served (grid set-up, steps to the rounding floor, result), on a Poisson "
                    "trace at 0.7 x its own closed-loop capacity; the engine on the same trace"},
        "rel_err_vs_fp64_max": max(errs) if errs else None,
    }


def paper_1d_table(args):
    """The solver comparison of the paper's 1-D infiltration benchmark
    (N = 2048, tau = 0.1 s, t = 360 s) on the GPU: V-cycle(5,5) and FMG(5,5)
    per step until ||r||_inf <= 1e-12, and GS(100) (100 red-black sweeps per
    step).  The paper's CPU times, on unstated hardware, are context only."""
    import torch
    import paper_2606_04292_amd as rsl
    from paper_2606_04292_amd import workloads as W

    w = W.celia_column(2049)
    steps = args.paper_steps
    out = {"workload": "%s: 2049 nodes over 40 cm, Haverkamp, BDF1, tau 0.1 s, %d steps" % (
        w.name, steps), "paper_cpu_seconds_context": {"V-cycle(5,5)": 20, "FMG(5,5)": 42,
                                                      "GS(100)": 69}}
    finals = {}
    for name, fmg in (("V-cycle(5,5)", 0), ("FMG(5,5)", 1)):
        G = rsl.Grid(w, device="cuda:0")
        opts = rsl.solve_opts(5, 5, 32, max_cycles=60, tol_abs=1e-12, stagnation=0, fmg=fmg)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cyc = 0
        for _ in range(steps):
            code, st = G.bdf_step(opts=opts)
            if code != rsl.RS_OK:
                raise SystemExit("%s step failed: %s" % (name, rsl.lib().rs_last_error().decode()))
            cyc += st.cycles
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        finals[name] = G.get_state()[0].cpu().numpy()
        out[name] = {"seconds": round(el, 3), "cycles_per_step": round(cyc / steps, 2)}
        log("%s: %.2f s, %.2f cycles/step" % (name, el, cyc / steps))
        G.close()
    G = rsl.Grid(w, device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = 0.0
    for _ in range(steps):
        G.begin_step()
        G.sweep(100)
        G.end_step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    gs = G.get_state()[0].cpu().numpy()
    out["GS(100)"] = {"seconds": round(el, 3)}
    # the layered column of the same section (Gardner / Haverkamp / vGM zones)
    wc = W.celia_composite(2049)
    G2 = rsl.Grid(wc, device="cuda:0")
    opts = rsl.solve_opts(5, 5, 32, max_cycles=60, tol_abs=1e-12, stagnation=0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    cyc = 0
    for _ in range(steps):
        code, st = G2.bdf_step(opts=opts)
        if code != rsl.RS_OK:
            raise SystemExit("composite step failed: " + rsl.lib().rs_last_error().decode())
        cyc += st.cycles
    torch.cuda.synchronize()
    out["V-cycle(5,5), layered column"] = {"seconds": round(time.perf_counter() - t1, 3),
                                            "cycles_per_step": round(cyc / steps, 2)}
    G2.close()
    ref = finals["V-cycle(5,5)"]
    scale = float(abs(ref).max())
    out["max_diff_vs_vcycle"] = {"FMG(5,5)": float(abs(finals["FMG(5,5)"] - ref).max()) / scale,
                                 "GS(100)": float(abs(gs - ref).max()) / scale}
    log("GS(100): %.2f s" % el)
    G.close()
    return out


def paper_2d_table(args):
    """The paper's 2-D cases on the GPU, each step iterated until
    ||r||_inf <= 1e-10 or the rounding floor: the Gardner infiltration
    (129^2, tau 0.1 day, 3 days, V(5,5)) whose CPU time the paper prints
    (context only: unstated hardware), and the two-layer vGM medium (257^2,
    tau 0.01 day, to 1.75 days, an FMG(10,10) cycle then V(10,10) cycles; the
    paper prints a total CPU time without stating the run length); each
    also with GS(100), 100 red-black sweeps per step, against the multigrid result."""
    import torch
    import paper_2606_04292_amd as rsl
    from paper_2606_04292_amd import workloads as W

    out = {}
    for key, w, fmg, ctx in (
            ("gardner_2d", W.gardner_2d(129), 0, 2.216),
            ("two_layer_vg", W.two_layer_vg(257, steps=args.paper_2d_steps), 1, 2320.0)):
        G = rsl.Grid(w, device="cuda:0")
        opts = rsl.solve_opts(w.nu1, w.nu2, w.nu_coarse, max_cycles=200, tol_abs=1e-10,
                              stagnation=1, fmg=fmg)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cyc, upd = 0, 0.0
        for _ in range(w.steps):
            code, st = G.bdf_step(opts=opts)
            if code != rsl.RS_OK:
                raise SystemExit("%s step failed: %s" % (key, rsl.lib().rs_last_error().decode()))
            cyc += st.cycles
            upd += st.cell_updates
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[key] = {"workload": "%s: %s nodes, %d steps of %g, %s" % (
                        w.name, "x".join(str(v) for v in w.grid.n), w.steps, w.dt,
                        "FMG(%d,%d) start" % (w.nu1, w.nu2) if fmg else "V(%d,%d)" % (w.nu1, w.nu2)),
                    "seconds": round(el, 3), "ms_per_step": round(el * 1e3 / w.steps, 3),
                    "cycles_per_step": round(cyc / w.steps, 2),
                    "cell_updates_per_s": upd / el}
        if ctx is not None:
            out[key]["paper_cpu_seconds_context"] = ctx
        log("%s: %.2f s, %.2f cycles/step" % (key, el, cyc / w.steps))
        ref = G.get_state()[0].cpu().numpy()
        G.close()
        # the paper's GS(k) comparison: k = 100 red-black sweeps per step
        G = rsl.Grid(w, device="cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(w.steps):
            G.begin_step()
            G.sweep(100)
            G.end_step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        gs = G.get_state()[0].cpu().numpy()
        out[key]["GS(100)"] = {"seconds": round(el, 3),
                               "max_diff_vs_multigrid": float(abs(gs - ref).max() / abs(ref).max())}
        log("%s GS(100): %.2f s" % (key, el))
        G.close()
    return out


def paper_order(args):
    """The paper's temporal-order study of the 1-D infiltration (section 4.1):
    N = 1024 with tau = 0.1 / 2^k, k = 0..5, against a reference on N = 2048
    with tau = 1e-4, at t = args.order_t seconds; L-infinity errors on the
    common nodes and the observed orders log2(e_k / e_{k+1}).  Each step
    V(5,5) cycles to ||r||_inf <= 1e-10 or the rounding floor."""
    import dataclasses
    import math
    import numpy as np
    import torch
    import paper_2606_04292_amd as rsl
    from paper_2606_04292_amd import workloads as W

    def run(n, dt):
        steps = int(round(args.order_t / dt))
        w = dataclasses.replace(W.celia_column(n), dt=dt, steps=steps)
        G = rsl.Grid(w, device="cuda:0")
        opts = rsl.solve_opts(5, 5, 32, max_cycles=100, tol_abs=1e-10, stagnation=1)
        for _ in range(steps):
            code, _ = G.bdf_step(opts=opts)
            if code != rsl.RS_OK:
                raise SystemExit("order study step failed: " + rsl.lib().rs_last_error().decode())
        psi = G.get_state()[0].cpu().numpy()
        G.close()
        return psi, steps

    t0 = time.perf_counter()
    ref, nref = run(2049, 1e-4)
    log("order study reference: %d steps, %.1f s" % (nref, time.perf_counter() - t0))
    out = {"workload": "celia_column: N = 1024 vs N = 2048 reference (tau 1e-4), t = %g s" % args.order_t,
           "tau": [], "linf_error": [], "observed_order": []}
    for k in range(6):
        dt = 0.1 / 2 ** k
        psi, _ = run(1025, dt)
        out["tau"].append(dt)
        out["linf_error"].append(float(np.abs(psi - ref[::2]).max()))
        log("order study tau %.5f: error %.3e" % (dt, out["linf_error"][-1]))
    e = out["linf_error"]
    out["observed_order"] = [math.log2(e[k] / e[k + 1]) for k in range(len(e) - 1)]
    out["seconds"] = round(time.perf_counter() - t0, 1)
    return out


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


def config_leg(args, cfg):
    """One configuration end to end on the GPU: its whole time loop from t = 0
    in FP64 and in mixed precision (the same steps and tolerance), ms per step
    and V-cycles (outer corrections) per step, the mixed result against the
    FP64 one after the last step, and the CPU oracle.  The 257-node column
    (config 1) is small enough for the oracle to run all 50 steps with
    lexicographic NGS (the configuration's ordering): the GPU's red-black steps
    are compared with them and its time is the whole run on one core.  For the
    513^2 slice and the 257 x 257 x 129 root box the oracle is timed on a
    bounded sample (V-cycles of the first step on all cores, about
    --cpu-seconds) and reported in cell-updates/s; their results are
    parity-tested against it at reduced size."""
    import numpy as np
    import torch
    import oracle
    import paper_2606_04292_amd as rsl
    from paper_2606_04292_amd import workloads as W

    torch.cuda.set_device(0)
    w = {1: W.config1, 2: W.config2, 4: W.config4}[cfg]()
    psi0 = torch.as_tensor(np.ascontiguousarray(w.psi0), device="cuda:0")
    tol = args.config_tol
    # one FP32 cycle per correction: on these grids (iterated to the rounding
    # floor) three were slower (column 2.6 -> 3.8, slice 5.7 -> 7.1, root box
    # 10.4 -> 14.4 ms per mixed step)
    opts = rsl.solve_opts(w.nu1, w.nu2, w.nu_coarse, max_cycles=args.max_cycles, tol_abs=tol,
                          stagnation=1, mp_inner_cycles=1)
    out = {"config": cfg, "workload": "%s: %s nodes, %s, dt %g s, %d steps, V(%d,%d), every step "
                                      "to %s" % (
               w.name, "x".join(str(v) for v in w.grid.n),
               "BDF1" if w.order == 1 else "BDF2 history, conductivity lagged at psi^n",
               w.dt, w.steps, w.nu1, w.nu2,
               "the rounding floor" if tol == 0 else "tol %.0e or the rounding floor" % tol)}
    finals = {}
    for prec, name in ((rsl.RS_FP64, "fp64"), (rsl.RS_MIXED, "mixed")):
        G = rsl.Grid(w, precision=prec, device="cuda:0")
        time_loop(G, w, psi0, 1, opts, "%s warmup" % name)
        G.set_state(psi0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = time_loop(G, w, psi0, w.steps, opts, name)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        finals[name] = G.get_state()[0].cpu().numpy()
        G.close()
        out[name] = {"ms_per_step": round(el * 1e3 / w.steps, 3), "seconds": round(el, 4),
                     "cycles_per_step": [x[1] for x in steps],
                     "mean_cycles_per_step": round(float(np.mean([x[1] for x in steps])), 2),
                     "cell_updates_per_s": sum(x[3] for x in steps) / el,
                     "steps_not_converged": [k + 1 for k, x in enumerate(steps) if x[0] != 0]}
    ref = finals["fp64"]
    out["mixed"]["rel_err_vs_fp64"] = float(np.abs(finals["mixed"] - ref).max() / np.abs(ref).max())
    out["mixed"]["speedup_vs_fp64"] = round(out["fp64"]["seconds"] / out["mixed"]["seconds"], 3)
    if cfg == 1:
        S = oracle.Solver(w, oracle.ORDER_LEX)
        t0 = time.perf_counter()
        cyc = 0
        for _ in range(w.steps):
            S.begin_step()
            hist = oracle.solve_to_floor(S, args.max_cycles, tol)
            cyc += len(hist) - 1
            S.end_step()
        el = time.perf_counter() - t0
        o = S.get(oracle.FIELD_PSI_N)
        out["fp64"]["rel_err_vs_lexicographic_oracle"] = float(np.abs(ref - o).max() / np.abs(o).max())
        out["cpu_baseline"] = {"value": round(el * 1e3 / w.steps, 3), "unit": "ms per step",
                               "cores": 1, "kind": "oracle",
                               "sample": "all %d steps, lexicographic NGS (serial), %.1f cycles per "
                                         "step, %.2f s" % (w.steps, cyc / w.steps, el)}
    else:
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
        out["cpu_baseline"] = {"value": per_cycle * cycles / el, "unit": "cell-updates/s",
                               "cores": oracle.threads(), "kind": "oracle",
                               "sample": "first step: set-up + %d V(%d,%d) cycles (red-black, "
                                         "OpenMP) with a residual norm after each, %.1f s" % (
                                             cycles, w.nu1, w.nu2, el)}
    return out


def shard_share(args):
    """One GPU's share of the 257^3 block split into eight z-slabs (the
    decomposition a several-GPU run would use): 257 x 257 x 33 nodes, i.e. the
    31 owned planes of slab s plus its halo planes 32 s and 32 s + 32, held
    as Dirichlet faces with the current state (what a halo plane is during
    one colour pass).  On the state of the timed 257^3 steps, times the
    finest sweep (HIP events per colour launch) and the defect on every
    share and on the whole grid; the slowest share sets the time of a
    several-GPU step."""
    import dataclasses
    import torch
    import paper_2606_04292_amd as rsl
    from paper_2606_04292_amd import workloads as W

    def timed(G, d, reps=10):
        G.profile_enable(True)
        G.profile_read(reset=True)
        G.sweep(reps)
        torch.cuda.synchronize()
        ms, n, _ = G.profile_read(reset=True)
        G.profile_enable(False)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(G.stream)
        for _ in range(reps):
            rsl.check(rsl.lib().rs_residual(G.h, G._dev(d)))
        e1.record(G.stream)
        torch.cuda.synchronize()
        return ms * 1e3 / n, e0.elapsed_time(e1) * 1e3 / reps

    w = W.config3(257)
    G = rsl.Grid(w, device="cuda:0")
    opts = rsl.solve_opts(w.nu1, w.nu2, w.nu_coarse, max_cycles=args.max_cycles, tol_abs=args.tol,
                          stagnation=1)
    for _ in range(args.warmup + 1):
        code, _ = G.bdf_step(opts=opts)
        if code != rsl.RS_OK:
            raise SystemExit("step failed: " + rsl.lib().rs_last_error().decode())
    pn, pm, nstep, t = G.get_state()
    G.begin_step()
    full_sweep, full_res = timed(G, G.empty())
    G.close()
    out = {"workload": "257^3 Haverkamp block after %d BDF2 steps; share = 257 x 257 x 33 nodes "
                       "(31 owned planes and two halo planes as state-valued Dirichlet faces)"
                       % (args.warmup + 1),
           "whole_grid": {"sweep_us_per_colour": round(full_sweep, 2), "defect_us": round(full_res, 2),
                          "nodes": 257 ** 3},
           "shares": []}
    g = dataclasses.replace(w.grid, n=[257, 257, 33], L=[1.0, 1.0, 32.0 / 256.0],
                            face_bc=[W.BC_NOFLUX] * 4 + [W.BC_DIRICHLET_STATE] * 2,
                            face_value=[0.0] * 6)
    for sl in range(8):
        k0 = 32 * sl
        a = pn[k0:k0 + 33].contiguous()
        b = pm[k0:k0 + 33].contiguous()
        ws = dataclasses.replace(w, name="block3d_share%d" % sl, grid=g, psi0=a.cpu().numpy())
        H = rsl.Grid(ws, device="cuda:0")
        H.set_state(a, b, nstep, t)
        H.begin_step()
        sw, rs = timed(H, H.empty())
        H.close()
        out["shares"].append({"planes": [k0, k0 + 32], "sweep_us_per_colour": round(sw, 2),
                              "defect_us": round(rs, 2)})
        log("share %d: sweep %.2f us/colour, defect %.2f us" % (sl, sw, rs))
    worst = max(x["sweep_us_per_colour"] for x in out["shares"])
    out["slowest_share_sweep_us"] = worst
    out["halo_plane_bytes"] = 257 * 257 * 8
    out["halo_us_at_153GBps"] = round(257 * 257 * 8 / 153e9 * 1e6, 2)
    out["sweep_speedup_8_shares_vs_whole"] = round(full_sweep / worst, 2)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="timed steps of the 20-step time loop from t = 0")
    ap.add_argument("--warmup", type=int, default=2,
                    help="untimed steps first (the state is then reset to t = 0)")
    ap.add_argument("--n", type=int, default=257, help="nodes per axis (2^k+1)")
    ap.add_argument("--tol", type=float, default=1e-13, help="residual max-norm tolerance (1/s)")
    ap.add_argument("--max-cycles", type=int, default=150)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg")
    ap.add_argument("--mp-inner", type=int, default=3,
                    help="FP32 V-cycles per FP64 defect correction in the 257^3 mixed-precision leg "
                         "(measured at 257^3: 1 / 2 / 3 / 4 / 6 give 30.7 / 27.9 / 27.0 / 27.6 / "
                         "27.7 ms per step)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-requests", type=int, default=4096)
    ap.add_argument("--serve-baseline", type=int, default=256,
                    help="requests of the trace solved one at a time in FP64")
    ap.add_argument("--serve-arena-gib", type=float, default=16.0)
    ap.add_argument("--serve-only", action="store_true", help="run only the serving leg")
    ap.add_argument("--paper-1d", action="store_true",
                    help="run only the paper's 1-D solver comparison (V-cycle, FMG, GS)")
    ap.add_argument("--paper-steps", type=int, default=3600)
    ap.add_argument("--paper-2d", action="store_true",
                    help="run only the paper's 2-D cases (Gardner infiltration, two-layer medium)")
    ap.add_argument("--paper-2d-steps", type=int, default=175)
    ap.add_argument("--paper-order", action="store_true",
                    help="run only the paper's temporal-order study of the 1-D infiltration")
    ap.add_argument("--order-t", type=float, default=10.0, help="final time of the order study (s)")
    ap.add_argument("--config", type=str, default=None,
                    help="run only the end-to-end legs of these configurations (comma list "
                         "of 1, 2, 4: the vG column, the 513^2 slice, the root box); one JSON "
                         "line each")
    ap.add_argument("--config-tol", type=float, default=0.0,
                    help="residual tolerance of the --config legs (0: every step to the "
                         "rounding floor)")
    ap.add_argument("--shard-share", action="store_true",
                    help="time the sweep and defect on one GPU's share of an eight-slab split")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 512 MiB device copy first (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.serve_only:
        print(json.dumps({"serving": serving_leg(args)}), flush=True)
        return
    if args.paper_1d:
        print(json.dumps({"paper_1d_table": paper_1d_table(args)}), flush=True)
        return
    if args.paper_2d:
        print(json.dumps({"paper_2d_table": paper_2d_table(args)}), flush=True)
        return
    if args.paper_order:
        print(json.dumps({"paper_order_study": paper_order(args)}), flush=True)
        return
    if args.config:
        if any(c not in ("1", "2", "4") for c in args.config.split(",")):
            print("--config takes 1, 2 and 4 (the 257^3 block is the default run)", file=sys.stderr)
            sys.exit(2)
        for c in args.config.split(","):
            print(json.dumps({"config_leg": config_leg(args, int(c))}), flush=True)
        return
    if args.shard_share:
        print(json.dumps({"shard_share": shard_share(args)}), flush=True)
        return
    r = gpu_run(args)
    w = r["w"]
    ms = r["elapsed"] * 1e3 / args.steps
    bad = [k + 1 for k, x in enumerate(r["steps"]) if x[0] != 0]
    out = {
        "metric": "NGS cell-updates/s + HBM-roofline % at 257^3",
        "value": r["updates"] / r["elapsed"],
        "unit": "cell-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "%s: %d^3 nodes, Haverkamp, BDF2 history with the conductivity "
                               "lagged at psi^n (first order in time), dt=%g s, steps 1-%d of the "
                               "%d-step drainage from t = 0, FAS V(%d,%d), red-black NGS, at most "
                               "%d Newton steps/cell, tol %.0e or the rounding floor" % (
                                   w.name, args.n, w.dt, min(args.steps, w.steps), w.steps,
                                   w.nu1, w.nu2, w.law.newton_iters, args.tol),
                   "nodes": args.n ** 3, "cycles_per_step": [x[1] for x in r["steps"]],
                   "final_residual_per_step": [x[2] for x in r["steps"]],
                   "steps_not_converged": bad, "warmup_ok": r["warmup_ok"],
                   "parallelism": "single GPU"},
        "roofline": r["roofline"],
    }
    if r["mixed"] is not None:
        out["mixed_precision"] = r["mixed"]
    if not args.no_serving:
        out["serving"] = serving_leg(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, args.n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
