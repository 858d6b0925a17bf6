#!/usr/bin/env python3
"""GSW-MTP throughput on one MI355X, float32 and split-precision products.

Workload: a 1152 x 1920 unit-amplitude pupil with 1000 foci at seeded random
non-grid positions in a 200 x 200 focal-unit ROI (minimum spacing 2), targets
uniform in [0.5, 1].  One step is one pass of Algorithm 1 (forward matrix
triple product, focus gather, statistics and weight update, scatter, adjoint
product with the phase-only projection).  Inputs are resident in HBM when the
timed region starts; the plan (index work, kernel matrices) is built before.

Every precision mode is timed on the same workload.  Its error against the
FP64 oracle is measured twice: the forward field of the seeded start phase
(operator error) and the foci intensities after the same k passes the CPU
baseline ran (trajectory error).  The headline is the fastest mode whose
trajectory error is at most twice float32's ("equal error").

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published dense peaks (TFLOP/s)
PEAK_TFLOPS = {"f32": 157.3, "bf16": 2516.6, "f16": 2516.6}
MODE_DTYPE = {"fp32": ("f32", 1), "bf16x3": ("bf16", 3), "fp16x3": ("f16", 3),
              "bf16x6": ("bf16", 6)}
METRIC = "GSW-MTP iter/s, 1152x1920 pupil, 1000 foci; BF16-split vs FP32 at equal error"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--modes", default="fp32,bf16x3,fp16x3,bf16x6")
    ap.add_argument("--cpu-passes", type=int, default=100,
                    help="oracle passes of the CPU sample and of the trajectory-error "
                         "check (the workload's 100 iterations, about 28 s on 16 host "
                         "cores; 0 disables)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stage-iters", type=int, default=20)
    ap.add_argument("--no-library-reference", action="store_true",
                    help="skip timing the vendor BLAS on the product shapes")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 128 MiB device copy 3 times (the known-size "
                         "reference that scales FETCH_SIZE / WRITE_SIZE counters) and exit")
    ap.add_argument("--sweep", action="store_true",
                    help="also run the foci-count sweep (k x k arrays up to 227 x 227 on a "
                         "1000 x 1000 pupil) and the continuous double-heart pattern")
    ap.add_argument("--adam-steps", type=int, default=200,
                    help="Adam steps of the differentiable 50x50-grid design (0 disables)")
    ap.add_argument("--small-steps", type=int, default=1000,
                    help="graph-replayed passes per small configuration (0 skips)")
    ap.add_argument("--batch-steps", type=int, default=20,
                    help="timed passes of the 64-hologram batch (0 disables)")
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed repeats of --steps passes (the median is reported)")
    ap.add_argument("--sweep-cases", default="9,51,227",
                    help="k of the k x k foci arrays of the sweep leg ('' skips it)")
    ap.add_argument("--legs", default="headline,small,batch,adam,sweep",
                    help="legs to run; without 'headline' the line carries only the "
                         "named legs' results (for profiling one leg alone)")
    return ap.parse_args()


# HBM traffic of the product kernels from rocprofv3 FETCH_SIZE / WRITE_SIZE
# runs (committed summary, scaled by the copy calibration); valid only while
# the kernel sources hash to what they were when the counters were taken.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic__gsw-1152x1920-1000foci.md")
KERNEL_SOURCES = {
    "f32": ["paper_2206_12661_amd/csrc/gemm.hip", "paper_2206_12661_amd/csrc/gswmtp_internal.h"],
    "split": ["paper_2206_12661_amd/csrc/gemm_split.hip",
              "paper_2206_12661_amd/csrc/gswmtp_internal.h"],
}


def sources_sha(kind: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(mode: str, stage: str):
    """HBM bytes per launch of the mode's product kernel for `stage`, or None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kind = "f32" if mode == "fp32" else "split"
    sha = sources_sha(kind)
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if not line.startswith("traffic-record: "):
                continue
            r = json.loads(line[len("traffic-record: "):])
            if r["mode"] == mode and r["stage"] == stage:
                if r["sources_sha256"] != sha:
                    return None
                return {"bytes": r["fetch_kib"] * 1024 * r["fetch_scale"] +
                        r["write_kib"] * 1024 * r["write_scale"],
                        "fetch_bytes": r["fetch_kib"] * 1024 * r["fetch_scale"],
                        "write_bytes": r["write_kib"] * 1024 * r["write_scale"]}
    return None


def library_reference(torch, idx, reps: int = 20) -> dict:
    """The vendor BLAS (torch.bmm -> hipBLASLt) on plain real GEMMs of the
    forward product's shape (U_r x R' by R' x C'): 4 float32 products (the
    4M complex product) and 12 float16 products (the same, split into three
    16-bit term products each).  A ceiling reference for the hand-written
    kernels, not part of the path."""
    if idx["axis"] == 0:
        M, K, N = idx["uy"], idx["ny_kept"], idx["nx_kept"]
    else:
        M, K, N = idx["ux"], idx["nx_kept"], idx["ny_kept"]
    out = {"shape": [M, K, N]}
    for name, dt, B in (("f32_x4", torch.float32, 4), ("f16_x12", torch.float16, 12)):
        a = torch.randn(B, M, K, device="cuda", dtype=dt)
        b = torch.randn(B, K, N, device="cuda", dtype=dt)
        c = torch.empty(B, M, N, device="cuda", dtype=dt)
        for _ in range(3):
            torch.bmm(a, b, out=c)
        torch.cuda.synchronize()
        # back-to-back launches between one event pair: per-launch kernel time
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            torch.bmm(a, b, out=c)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"ms": round(ms, 5), "tflops": round(2.0 * B * M * N * K / ms / 1e9, 1)}
        del a, b, c
    return out


def algorithmic_flops(idx, n_foci) -> dict:
    """Real flops of one pass, 8 per complex multiply-accumulate, unpadded
    sizes: forward U_r x R' x C' plus the fused gather N x C', scatter N x C',
    adjoint R' x U_r x C'."""
    if idx["axis"] == 0:
        ur, rk, ck = idx["uy"], idx["ny_kept"], idx["nx_kept"]
    else:
        ur, rk, ck = idx["ux"], idx["nx_kept"], idx["ny_kept"]
    prod = 8.0 * ur * rk * ck
    gath = 8.0 * n_foci * ck          # focus gather, fused into the forward product
    return {"forward_product": prod + gath, "adjoint_product_project": prod,
            "scatter": gath, "pass": 2 * prod + 2 * gath}


def cpu_baseline(h, passes: int):
    """Time the oracle (as it stands) on the first ``passes`` passes of the same
    workload from the same start phase.  A fixed pass count (not a time
    budget) keeps the trajectory-error point, and so the equal-error
    decision, the same on every host."""
    import oracle
    t0 = time.perf_counter()
    r = oracle.gsw(h, n_iter=passes)
    t = time.perf_counter() - t0
    return {"value": passes / t, "unit": "iter/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{passes} passes of the same 1152x1920 / 1000-foci workload from the same "
                      f"start phase in one FP64 oracle call ({t:.1f} s, including its phasor "
                      f"tables and one final forward)"}, r, passes


def run_mode(g, torch, h, mode, args):
    plan_ms = plan_time_ms(g, torch, h, mode)
    plan = g.Plan(h, precision=mode)
    plan.sync()
    idx = plan.index()
    fl = algorithmic_flops(idx, plan.n_foci)
    theta0 = plan.foci_field()                      # field of phi0 (operator error)
    plan.iterate(args.warmup)                       # includes graph capture
    plan.sync()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    # `repeats` timed regions of exactly `steps` passes each, synchronised on
    # both sides; HIP events on the stream the plan orders its passes with
    # (the wall clock, if longer, is taken instead); the median is reported
    reps = []
    for _ in range(max(1, args.repeats)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record()
        plan.iterate(args.steps)
        ev1.record()
        plan.sync()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        reps.append(max(wall, ev0.elapsed_time(ev1) / 1e3))
    elapsed = float(np.median(reps))
    ips = args.steps / elapsed
    # per-stage kernel durations: eager launches bracketed by HIP events on the
    # plan's stream
    stages = plan.time_stages(args.stage_iters)
    dom = max(("forward_product", "adjoint_product_project"), key=lambda k: stages[k])
    dt, terms = MODE_DTYPE[mode]
    achieved = fl[dom] / (stages[dom] * 1e-3) / 1e12
    peak = PEAK_TFLOPS[dt]
    roof = {"bound": "mfma", "kernel": plan.stage_kernel(0 if dom == "forward_product" else 3),
            "stage": dom, "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": None,
            "flops_per_launch": fl[dom], "mean_launch_ms": round(stages[dom], 5)}
    tr = traffic_for(mode, dom)
    if tr is not None:
        roof["traffic"] = round(tr["bytes"])
        roof["traffic_fetch"] = round(tr["fetch_bytes"])
        roof["traffic_write"] = round(tr["write_bytes"])
    if terms > 1:
        # each algorithmic real product issues `terms` 16-bit MFMA products
        roof["term_products"] = terms
        roof["issued_tflops"] = round(achieved * terms, 3)
        roof["issued_frac"] = round(achieved * terms / peak, 4)
    plan.close()
    return {"mode": mode, "value": ips, "ms_per_step": 1e3 / ips, "roofline": roof, "index": idx,
            "stage_ms": {k: round(v, 5) for k, v in stages.items()}, "plan_ms": plan_ms,
            "pass_tflops": fl["pass"] * ips / 1e12, "theta0": theta0, "dtype": dt,
            "repeats_ms_per_step": [round(1e3 * r / args.steps, 5) for r in reps]}


def run_small(g, torch, args, modes):
    """The latency-bound configurations (64 x 64 / 16 foci and 512 x 512 /
    100 foci): microseconds per pass under graph replay."""
    import synth_ofa
    out = {}
    for name, h in (("config1-64x64-16foci", synth_ofa.config1()),
                    ("config2-512x512-100foci", synth_ofa.config2())):
        out[name] = {}
        for m in dict.fromkeys(modes):
            with g.Plan(h, precision=m) as p:
                p.iterate(20)
                p.sync()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                p.iterate(args.small_steps)
                p.sync()
                dt = time.perf_counter() - t0
            out[name][m] = {"us_per_pass": round(1e6 * dt / args.small_steps, 2)}
        if not args.no_cpu_baseline:
            # the oracle on one host thread and on all of them
            import oracle
            passes = 20 if h.ny <= 64 else 2
            full = oracle.num_threads()
            for label, th in (("cpu_oracle_1thread", 1), ("cpu_oracle_all_threads", full)):
                oracle.set_threads(th)
                t0 = time.perf_counter()
                oracle.gsw(h, n_iter=passes)
                dt = time.perf_counter() - t0
                out[name][label] = {"us_per_pass": round(1e6 * dt / passes, 1), "cores": th,
                                    "passes": passes}
            oracle.set_threads(full)
    return out


def _batch_time(g, torch, hs, mode, args, persist: bool):
    os.environ["GSWMTP_BATCH_PERSIST"] = "1" if persist else "0"
    t0 = time.perf_counter()
    plans = [g.Plan(h, precision=mode) for h in hs]
    flops = sum(algorithmic_flops(p.index(), p.n_foci)["pass"] for p in plans)
    b = g.Batch(plans)
    b.sync()
    setup_ms = (time.perf_counter() - t0) * 1e3
    b.iterate(max(1, args.warmup // 4))
    b.sync()
    reps = []
    for _ in range(max(1, args.repeats)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.iterate(args.batch_steps)
        b.sync()
        torch.cuda.synchronize()
        reps.append(time.perf_counter() - t0)
    classes, tiles, tune_ms = b.classes(), b.tiles(), b.tune_ms()
    b.close()
    for p in plans:
        p.close()
    os.environ.pop("GSWMTP_BATCH_PERSIST", None)
    return args.batch_steps / float(np.median(reps)), flops, setup_ms, classes, tiles, tune_ms


def run_batch(g, torch, args):
    """The 64-hologram batch (uneven sides 256-1024, 16-2000 foci) in float32
    and in BF16x3: batched passes per second, each pass advancing every
    hologram by one; per-class kernel configurations and the tuning table
    (full table on stderr); the persistent work-list launches against one
    workgroup per tile; the oracle on a stated subset."""
    import collections
    import synth_ofa
    hs = synth_ofa.config4()
    out = {"workload": "gsw-batch-64-holograms-256to1024px-16to2000foci",
           "holograms": len(hs), "steps": args.batch_steps, "repeats": args.repeats}
    for mode in ("fp32", "bf16x3"):
        ips, flops, setup_ms, classes, tiles, tune_ms = _batch_time(g, torch, hs, mode, args, True)
        ips_u, *_ = _batch_time(g, torch, hs, mode, args, False)
        hist = {"forward": collections.Counter(), "adjoint": collections.Counter()}
        for c in classes:
            hist[c["product"]][c["config"]] += c["plans"]
        top = sorted(classes, key=lambda c: -c["mnk"][0] * c["mnk"][1] * c["mnk"][2] *
                     c["plans"])[:2]
        r = {"batch_iter_s": round(ips, 3), "hologram_iter_s": round(ips * len(hs), 2),
             "ms_per_batch_iter": round(1e3 / ips, 4), "flops_per_batch_iter": flops,
             "tflops": round(flops * ips / 1e12, 3),
             "per_tile_launch_ms_per_batch_iter": round(1e3 / ips_u, 4),
             "classes": len(classes),
             "sources": dict(collections.Counter(c["source"] for c in classes)),
             "plans_per_config": {k: dict(v) for k, v in hist.items()},
             "tuning_top_classes": [{"product": c["product"], "mnk": c["mnk"],
                                     "config": c["config"],
                                     "tried_ms": {k: round(v, 4) for k, v in c["tried"].items()}}
                                    for c in top],
             "tiles_largest_class": {"forward": tiles["forward"], "adjoint": tiles["adjoint"]},
             "tune_ms": round(tune_ms, 1), "setup_ms": round(setup_ms, 1)}
        if mode == "fp32":
            r["frac_f32_peak"] = round(flops * ips / 1e12 / PEAK_TFLOPS["f32"], 4)
        out[mode] = r
        for c in classes:
            print(f"[batch {mode}] {c['product']} {c['mnk']} x{c['plans']}: {c['config']} "
                  f"({c['source']}) {c['tried']}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        import oracle
        order = sorted(range(len(hs)), key=lambda k: hs[k].ny * hs[k].nx * hs[k].fx.shape[0])
        sub = [hs[k] for k in order[:8] + order[-1:]]
        t0 = time.perf_counter()
        for h in sub:
            oracle.gsw(h, n_iter=1)
        dt = time.perf_counter() - t0
        out["cpu_oracle_subset"] = {
            "sample": "one pass of each of the 8 smallest holograms and the largest",
            "hologram_passes_s": round(len(sub) / dt, 3), "seconds": round(dt, 2),
            "cores": oracle.num_threads()}
    return out


def plan_time_ms(g, torch, h, mode, reps: int = 3) -> float:
    """Median wall time of creating a plan (host validation, copies, index
    and kernel-matrix kernels, one synchronisation), after one creation that
    warms the code paths."""
    ts = []
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p = g.Plan(h, precision=mode)
        p.sync()
        ts.append((time.perf_counter() - t0) * 1e3)
        p.close()
    return round(float(np.median(ts[1:])), 3)


def run_sweep(g, torch, args):
    """Foci-count sweep (Sec. 2, Fig. 2(e)): time of 100 passes for uniform
    k x k arrays on the 1000 x 1000 pupil, FP32 and FP16x3, and the
    continuous double-heart pattern; accuracy / efficiency after the run.
    Plan-creation time per case, and at the largest focus count a plan takes
    (262144 foci, a 512 x 512 grid on a 1024 x 1024 pupil)."""
    import synth_ofa
    ks = (9, 25, 51, 101, 151, 227) if args.sweep else \
        tuple(int(k) for k in args.sweep_cases.split(",") if k.strip())
    cases = [synth_ofa.sweep_case(k) for k in ks]
    cases.append(synth_ofa.double_heart())
    out = []
    for h in cases:
        row = {"case": h.name, "n_foci": int(h.n_foci)}
        for mode in ("fp32", "fp16x3"):
            with g.Plan(h, precision=mode) as p:
                idx = p.index()
                p.iterate(10)
                p.sync()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                p.iterate(100)
                p.sync()
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                st = p.stats()
            row["reduced_grid"] = [idx["uy"], idx["ux"]]
            row[mode] = {"ms_per_100_passes": round(dt * 1e3, 3), "xi": round(st["xi"], 5),
                         "eta": round(st["eta"], 4),
                         "plan_ms": plan_time_ms(g, torch, h, mode)}
        out.append(row)
        print(f"[sweep] {row}", file=sys.stderr, flush=True)
    big = synth_ofa.random_case(50, 1024, 1024, 0, grid=(512, 512))
    big.fx, big.fy = synth_ofa.grid_foci(512, 512, 0.45)
    big.target = np.random.default_rng(51).uniform(0.5, 1.0, big.fx.shape[0])
    out.append({"case": "plan-only-1024x1024-512x512grid", "n_foci": int(big.n_foci),
                "fp32": {"plan_ms": plan_time_ms(g, torch, big, "fp32")},
                "fp16x3": {"plan_ms": plan_time_ms(g, torch, big, "fp16x3")}})
    print(f"[sweep] {out[-1]}", file=sys.stderr, flush=True)
    return out


def run_adam(g, torch, args):
    """The differentiable form: phase design of a 50 x 50 grid on the
    1152 x 1920 pupil by Adam (lr 0.05) through the forward product and the
    adjoint-gradient epilogue; steps per second over the whole run, with each
    step replayed from one captured graph (the eager loop, which launches every
    step from the host, is timed beside it over a quarter of the steps)."""
    import synth_ofa
    h = synth_ofa.config5()
    n = args.adam_steps
    with g.Plan(h) as p:
        g.adam_design(p, 5, phi0=h.phi0, target=h.target)      # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phi, hist = g.adam_design(p, n, phi0=h.phi0, target=h.target)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        n_e = max(1, n // 4)
        g.adam_design(p, 2, phi0=h.phi0, target=h.target, graph=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.adam_design(p, n_e, phi0=h.phi0, target=h.target, graph=False)
        torch.cuda.synchronize()
        dt_e = time.perf_counter() - t0
        p.set_phase(phi)
        st = p.stats()
        idx = p.index()
    hist = hist.cpu().numpy()
    fl = algorithmic_flops(idx, len(h.fx))
    step_flops = fl["forward_product"] + fl["adjoint_product_project"] + fl["scatter"]
    return {"workload": "gsw-adam-1152x1920-50x50grid", "steps": n,
            "steps_s": round(n / dt, 2),
            "ms_per_step": round(1e3 * dt / n, 4),
            "form": "one captured graph per step, replayed",
            "eager_steps": n_e, "eager_steps_s": round(n_e / dt_e, 2),
            "eager_ms_per_step": round(1e3 * dt_e / n_e, 4),
            "loss_first": float(hist[0]), "loss_last": float(hist[-1]),
            "uniformity": round(st["uniformity"], 5), "efficiency": round(st["eta"], 5),
            "flops_per_step": step_flops}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the "
              "multi-GPU sharding is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibration:
        n = 128 * 1024 * 1024 // 4
        x = torch.rand(n, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 4, "copies": 3}), flush=True)
        return
    import paper_2206_12661_amd as g
    import synth_ofa

    h = synth_ofa.config3()
    torch.cuda.init()
    legs = {x.strip() for x in args.legs.split(",") if x.strip()}
    if "headline" not in legs:
        part = {}
        if "small" in legs and args.small_steps > 0:
            part["small_configs"] = run_small(g, torch, args, ("fp32", "bf16x3"))
        if "batch" in legs and args.batch_steps > 0:
            part["batch"] = run_batch(g, torch, args)
        if "adam" in legs and args.adam_steps > 0:
            part["differentiable"] = run_adam(g, torch, args)
        if "sweep" in legs and args.sweep_cases.strip():
            part["sweep"] = run_sweep(g, torch, args)
        print(json.dumps({"legs": sorted(legs), **part}), flush=True)
        return
    modes = [m.strip() for m in args.modes.split(",") if m.strip()]
    res = {m: run_mode(g, torch, h, m, args) for m in modes}

    base, r_or, k = None, None, 0
    if not args.no_cpu_baseline and args.cpu_passes > 0:
        base, r_or, k = cpu_baseline(h, args.cpu_passes)
    xi_ckpt = [c for c in (1, 2, 5, 10, 20, 50, 100, 200) if c <= k]
    xi_oracle = None
    if r_or is not None:
        import oracle
        theta_ref0 = oracle.forward(oracle.pupil_field(h), h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
        theta_ref1 = oracle.gsw(h, n_iter=1)["theta"]          # one pass from phi0
        I_ref = np.abs(r_or["theta"]) ** 2
        xi_oracle = [round(float(r_or["history"][c - 1, 0]), 6) for c in xi_ckpt]
        rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))  # noqa: E731
        for m in modes:
            with g.Plan(h, precision=m) as p2:
                p2.iterate(1)
                th1 = p2.foci_field().astype(np.complex128)
                p2.iterate(k - 1)
                th = p2.foci_field()
                hist = p2.history()
            I = np.abs(th.astype(np.complex128)) ** 2
            res[m]["traj_err"] = rel(I, I_ref)
            res[m]["one_step_err"] = rel(th1, theta_ref1)
            res[m]["op_err"] = rel(res[m]["theta0"].astype(np.complex128), theta_ref0)
            res[m]["xi"] = [round(float(hist[c - 1, 0]), 6) for c in xi_ckpt]

    # headline: BF16x3 (the metric's BF16 split) when it meets equal error
    # (trajectory error <= 2x float32's), else the fastest mode that does
    head = "bf16x3" if "bf16x3" in res else ("fp32" if "fp32" in res else modes[0])
    if r_or is not None and "fp32" in res:
        ref_err = res["fp32"]["traj_err"]
        ok = [m for m in modes if res[m]["traj_err"] <= 2 * ref_err]
        if head not in ok:
            head = max(ok, key=lambda m: res[m]["value"])
    hr = res[head]
    libref = library_reference(torch, hr["index"]) if not args.no_library_reference else None
    small = (run_small(g, torch, args, ("fp32", head))
             if args.small_steps > 0 and "small" in legs else None)
    batch = run_batch(g, torch, args) if args.batch_steps > 0 and "batch" in legs else None
    adam = run_adam(g, torch, args) if args.adam_steps > 0 and "adam" in legs else None
    sweep = (run_sweep(g, torch, args)
             if (args.sweep or args.sweep_cases.strip()) and "sweep" in legs else None)
    out = {
        "metric": METRIC,
        "value": round(hr["value"], 3), "unit": "iter/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(hr["ms_per_step"], 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": head if head != "fp32" else "f32",
        "data": "synthetic (seeded dart-throw foci, unit-amplitude rectangle)",
        "config": {"workload": "gsw-1152x1920-1000foci", "pupil": [1152, 1920], "n_foci": 1000,
                   "precision": head, "passes_timed": args.steps},
        "repeats": args.repeats,
        "median_ms_per_step": round(hr["ms_per_step"], 5),
        "repeats_ms_per_step": hr["repeats_ms_per_step"],
        "roofline": hr["roofline"],
        "stage_ms": hr["stage_ms"],
        "pass_tflops": round(hr["pass_tflops"], 3),
        "plan_ms": round(hr["plan_ms"], 2),
        "cpu_baseline": base,
        "modes": {m: {"iter_s": round(v["value"], 2), "ms_per_step": round(v["ms_per_step"], 5),
                      "speedup_vs_fp32": (round(v["value"] / res["fp32"]["value"], 3)
                                          if "fp32" in res else None),
                      "op_err": v.get("op_err"), "one_step_err": v.get("one_step_err"),
                      "traj_err": v.get("traj_err"), "xi": v.get("xi"),
                      "equal_error": (v.get("traj_err") is not None and "fp32" in res and
                                      v["traj_err"] <= 2 * res["fp32"]["traj_err"]),
                      "roofline": v["roofline"], "stage_ms": v["stage_ms"]}
                  for m, v in res.items()},
        "error_passes": k,
        "xi_passes": xi_ckpt, "xi_oracle": xi_oracle,
        "small_configs": small,
        "library_gemm_reference": libref,
        "batch": batch,
        "differentiable": adam,
        "sweep": sweep,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
