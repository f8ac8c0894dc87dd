#!/usr/bin/env python
"""Benchmark of one dual-time pseudo-iteration (Steps 3-7) of the implicit
unsteady UGKS on MI355X, on the Ma 5 cylinder workload: O-mesh 128 x 64
cells, 64 x 64 velocity grid on [-15, 15]^2, Kn 0.01, hard-sphere gas,
isothermal wall, far field, dt = 20 dt_s.

Prints one JSON line: (cell x velocity) updates per second per pseudo-step
for the FP64 path (`value`), the FP32-storage path beside it, the roofline
of the dominant kernel (timed live with HIP events on the library's stream)
and the FP64 CPU oracle timed on a bounded sample of the same workload.
Inputs are resident in HBM before the timed region starts.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic values moved per (cell, velocity) pair by each measured kernel
# (storage-precision values of h, b, the sources and the D/residual buffer):
#   face_eq      face-moment march: read h, b
#   flux         flux march: read h, b; write D_h, D_b
#   micro_rhs    micro residual: read S, f, D; write r over D
#   micro_sweep  forward: read r, write dF*; backward: read dF*, f, write f
#                (residual fused into the forward sweep: read D, S, f instead
#                of r, and no micro_rhs pass)
#   step7        Step-7 moments: read h, b
KERNEL_VALUES = {"face_eq": 2, "flux": 4, "micro_rhs": 8, "micro_sweep": 10, "step7": 2}
FUSED_SWEEP_VALUES = 14
KERNEL_NAMES = {"face_eq": "k_march (face-moment pass, MODE 0)", "flux": "k_march (flux pass, MODE 1)",
                "micro_rhs": "k_micro_rhs", "micro_sweep": "k_micro", "step7": "k_step7"}
KERNEL_KEYS = {"face_eq": "k_march<{re}, {t}, {t}, 0>", "flux": "k_march<{rf}, {t}, {t}, 1>",
               "micro_rhs": "k_micro_rhs<{t}>", "micro_sweep": "k_micro<2, {t}, {kc}, {mp}, {mr}>",
               "step7": "k_step7<{t}>"}


def kernel_values(micro):
    """Algorithmic values per pair of the kernels that run for this micro
    sweep shape (kc, rows, depth, fused)."""
    kv = dict(KERNEL_VALUES)
    if micro[3]:
        del kv["micro_rhs"]
        kv["micro_sweep"] = FUSED_SWEEP_VALUES
    return kv


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50, help="timed pseudo-iterations")
    ap.add_argument("--warmup", type=int, default=10, help="untimed pseudo-iterations")
    ap.add_argument("--cpu-steps", type=int, default=2, help="oracle pseudo-iterations (0: skip)")
    ap.add_argument("--no-f32", action="store_true")
    ap.add_argument("--workload-steps", type=int, default=5,
                    help="pseudo-iterations timed on each of the other workloads (0: skip)")
    ap.add_argument("--nvx", type=int, default=64)
    ap.add_argument("--workload", default=None,
                    help="run only this workload (sod, plate, two_body, batch) and print its line")
    ap.add_argument("--adjoint-calls", type=int, default=3,
                    help="timed reverse passes of one pseudo-iteration (FP64; 0: skip)")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                    help="only run a plain device copy of GIB GiB (HBM counter calibration) and exit")
    return ap.parse_args()


def traffic_from_profiles(kernel, prec, workload):
    """HBM bytes per launch from the committed counter summary, if it was
    measured on this workload and still matches the kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
        ent = data.get(f"{kernel}:{prec}")
        if not ent or ent.get("workload") != workload:
            return None
        import hashlib
        src = open(os.path.join(ROOT, "paper_2604_09984_amd", "csrc", "ugks_kernels.hip"), "rb").read()
        if ent.get("source_sha1") != hashlib.sha1(src).hexdigest():
            return None
        return ent["bytes_per_launch"]
    except Exception:
        return None


def run_gpu(case, prec_name, steps, warmup, adjoint_calls=0):
    import torch
    from paper_2604_09984_amd import ugks
    prec = ugks.F64 if prec_name == "f64" else ugks.F32
    s = ugks.Solver(case, prec)
    dts, _ = s.timesteps()
    dt = case.dt_over_dts * dts
    h, b, W, q = s.init_state()
    Wn = W.clone()
    Sh, Sb, Fn = s.begin_step(dt, h, b, W, q)
    chunk = 10  # one physical step's inner loop per graph replay
    # warm-up: eager, the launch-shape autotuner (on copies of the state),
    # then the first replay captures the graph
    if warmup > 0:
        s.step(dt, warmup, h, b, W, Wn, q, Sh, Sb, Fn)
    tuning, _ = s.autotune(dt, 3, h, b, W, Wn, q, Sh, Sb, Fn)
    s.step_graph(dt, chunk, h, b, W, Wn, q, Sh, Sb, Fn)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    left = steps
    while left > 0:
        n = min(chunk, left)
        (s.step_graph if n == chunk else s.step)(dt, n, h, b, W, Wn, q, Sh, Sb, Fn)
        left -= n
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    # the same pseudo-iterations launched one kernel at a time, for comparison
    t1 = time.perf_counter()
    s.step(dt, chunk, h, b, W, Wn, q, Sh, Sb, Fn)
    torch.cuda.synchronize()
    eager_ms = 1e3 * (time.perf_counter() - t1) / chunk
    # per-kernel timing: HIP events on the library's stream, separate run
    prof = s.step_profile(dt, chunk, h, b, W, Wn, q, Sh, Sb, Fn)
    torch.cuda.synchronize()
    adj_ms = adj_finite = None
    if adjoint_calls > 0 and prec == ugks.F64:
        # reverse pass of one pseudo-iteration at the current state with random
        # cotangents (one call = the iteration's forward recomputation plus the
        # reverse kernels); the first call allocates the workspace
        gen = torch.Generator(device=h.device).manual_seed(1)
        ys = [torch.randn(t.shape, dtype=torch.float64, device=h.device, generator=gen) for t in (h, b, W, q)]
        s.step_adjoint(dt, h, b, W, Wn, q, Sh, Sb, Fn, *ys)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(adjoint_calls):
            s.step_adjoint(dt, h, b, W, Wn, q, Sh, Sb, Fn, *ys)
        torch.cuda.synchronize()
        adj_ms = 1e3 * (time.perf_counter() - t2) / adjoint_calls
        bars = s.step_adjoint(dt, h, b, W, Wn, q, Sh, Sb, Fn, *ys)
        adj_finite = all(bool(torch.isfinite(t).all().item()) for t in bars)
        del bars
    pairs = int((s.types() == 1).sum()) * s.nv
    out = dict(prec=prec_name, pairs=pairs, wall_s=wall_s, eager_ms=eager_ms, steps=steps, stages=prof,
               tuning=dict(zip(("kc_max", "rg_eq", "rg_flux"), tuning)), micro=s.micro_shape(),
               finite=bool(torch.isfinite(h).all().item() and torch.isfinite(W).all().item()), adjoint_ms=adj_ms,
               adjoint_finite=adj_finite)
    out["h"] = h.to(torch.float64).cpu()
    s.close()
    return out


def time_workload(case, prec_name, iters, t_pose=0.0):
    """One workload at its full size: the state at its initial Maxwellian
    after Steps 1-2 (moving overset: the pose at t_pose assembled first),
    launch shapes autotuned, then `iters` pseudo-iterations replayed from
    one captured graph and timed (wall clock around the replay)."""
    import torch
    from paper_2604_09984_amd import ugks
    prec = ugks.F64 if prec_name == "f64" else ugks.F32
    s = ugks.Solver(case, prec)
    out = {"prec": prec_name}
    if case.overset is not None:
        s.set_poses(case.poses(t_pose))
        t0 = time.perf_counter()
        s.assemble(case.overset["wrule"], case.overset["overlap"])
        out["assembly_ms"] = round(1e3 * (time.perf_counter() - t0), 2)
    dts, _ = s.timesteps()
    dt = case.dt if case.dt is not None else case.dt_over_dts * dts
    h, b, W, q = s.init_state()
    Wn = W.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Sh, Sb, Fn = s.begin_step(dt, h, b, W, q)
    torch.cuda.synchronize()
    out["begin_step_ms"] = round(1e3 * (time.perf_counter() - t0), 3)
    tuning, _ = s.autotune(dt, 1, h, b, W, Wn, q, Sh, Sb, Fn)
    s.step_graph(dt, iters, h, b, W, Wn, q, Sh, Sb, Fn)  # capture, warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step_graph(dt, iters, h, b, W, Wn, q, Sh, Sb, Fn)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / iters
    finite = bool(torch.isfinite(h).all().item() and torch.isfinite(W).all().item())
    live = s.types() == 1
    rho_min = float(W[torch.as_tensor(live, device=W.device), 0].min().item()) if case.dim == 2 else None
    pairs = int(live.sum()) * s.nv
    tuning_d = dict(zip(("kc_max", "rg_eq", "rg_flux"), tuning))
    micro = s.micro_shape()
    # per-kernel times (HIP events on the library's stream), the dominant
    # kernel's roofline and the whole iteration's algorithmic HBM rate
    prof = s.step_profile(dt, 2, h, b, W, Wn, q, Sh, Sb, Fn)
    torch.cuda.synchronize()
    kv = kernel_values(micro)
    nbytes = 8 if prec_name == "f64" else 4
    step_bytes = sum(kv.values()) * nbytes * pairs
    out.update(pairs=pairs, pseudo_steps=iters, ms_per_pseudo_step=round(ms, 4), value=pairs / (ms * 1e-3),
               launch_shapes=tuning_d, finite=finite, rho_min=rho_min,
               stages_ms={k: round(v, 4) for k, v in prof.items()},
               hbm_algorithmic_frac=round(step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               roofline=roofline(prof, pairs, prec_name, tuning_d, micro, case.name) if case.dim == 2 else None)
    if case.overset is not None:
        # the same assembly on the GPU (identical tables)
        t0 = time.perf_counter()
        s.assemble(case.overset["wrule"], case.overset["overlap"], device=True)
        out["assembly_device_ms"] = round(1e3 * (time.perf_counter() - t0), 2)
    s.close()
    del h, b, W, Wn, q, Sh, Sb, Fn
    torch.cuda.empty_cache()
    return out


def time_batch(count, prec_name, iters):
    """The seeded batch of ragged cavity / plate cases advanced together from
    one captured graph (per-case launch shapes autotuned first), against the
    same cases advanced one after another, each from its own graph."""
    import torch
    from paper_2604_09984_amd import ugks, workloads as wl
    prec = ugks.F64 if prec_name == "f64" else ugks.F32
    cases = wl.batch_cases(count)
    solvers = [ugks.Solver(c, prec) for c in cases]
    dts, states = [], []
    for c, s in zip(cases, solvers):
        d, _ = s.timesteps()
        dt = c.dt_over_dts * d
        h, b, W, q = s.init_state()
        Wn = W.clone()
        Sh, Sb, Fn = s.begin_step(dt, h, b, W, q)
        s.autotune(dt, 1, h, b, W, Wn, q, Sh, Sb, Fn)
        dts.append(dt)
        states.append([h, b, W, Wn, q, Sh, Sb, Fn])
    def timed(mode):
        batch = ugks.Batch(solvers, mode=mode)
        batch.step(dts, iters, states)  # capture, warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.step(dts, iters, states)
        torch.cuda.synchronize()
        out = 1e3 * (time.perf_counter() - t0) / iters
        batch.close()
        return out
    # one launch per stage (persistent march and micro grids), then the
    # cases' own chains on concurrent branches
    ms = timed(1)
    ms_branches = timed(0)
    for s, st, dt in zip(solvers, states, dts):
        s.step_graph(dt, iters, *st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, st, dt in zip(solvers, states, dts):
        s.step_graph(dt, iters, *st)
    torch.cuda.synchronize()
    ms_seq = 1e3 * (time.perf_counter() - t0) / iters
    pairs = sum(int((s.types() == 1).sum()) * s.nv for s in solvers)
    for s in solvers:
        s.close()
    del states
    torch.cuda.empty_cache()
    return {"prec": prec_name, "cases": count, "pairs": pairs, "pseudo_steps": iters,
            "ms_per_pseudo_step": round(ms, 4), "value": pairs / (ms * 1e-3),
            "launch": "one launch per stage (persistent march and micro-sweep grids over work items)",
            "branches_ms_per_pseudo_step": round(ms_branches, 4),
            "sequential_ms_per_pseudo_step": round(ms_seq, 4)}


def time_batch_adjoint(count, group=8):
    """The reverse pass of one pseudo-iteration (ugks_step_adjoint, FP64
    contexts) of every case of the seeded batch at its state after Steps
    1-2, with random cotangents: the cases one after another, and `group`
    cases at a time on their own streams (default priority).  Contexts are
    made `group` at a time so that the reverse workspaces fit."""
    import torch
    from paper_2604_09984_amd import ugks, workloads as wl
    cases = wl.batch_cases(count)
    seq_ms = par_ms = 0.0
    for g0 in range(0, count, group):
        solvers, runs = [], []
        for c in cases[g0:g0 + group]:
            s = ugks.Solver(c, ugks.F64)
            d, _ = s.timesteps()
            dt = c.dt_over_dts * d
            h, b, W, q = s.init_state()
            Wn = W.clone()
            Sh, Sb, Fn = s.begin_step(dt, h, b, W, q)
            gen = torch.Generator(device=h.device).manual_seed(len(runs))
            ys = [torch.randn(t.shape, dtype=torch.float64, device=h.device, generator=gen) for t in (h, b, W, q)]
            solvers.append(s)
            runs.append((dt, (h, b, W, Wn, q, Sh, Sb, Fn), ys))
        streams = [torch.cuda.Stream() for _ in solvers]
        for s, (dt, x, ys), st in zip(solvers, runs, streams):  # first calls: workspaces and colourings
            with torch.cuda.stream(st):
                s.step_adjoint(dt, *x, *ys)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s, (dt, x, ys) in zip(solvers, runs):
            s.step_adjoint(dt, *x, *ys)
        torch.cuda.synchronize()
        seq_ms += 1e3 * (time.perf_counter() - t0)
        t0 = time.perf_counter()
        for s, (dt, x, ys), st in zip(solvers, runs, streams):
            with torch.cuda.stream(st):
                s.step_adjoint(dt, *x, *ys)
        torch.cuda.synchronize()
        par_ms += 1e3 * (time.perf_counter() - t0)
        for s in solvers:
            s.close()
        del solvers, runs, streams
        torch.cuda.empty_cache()
    return {"what": "ugks_step_adjoint of one pseudo-iteration for every case (FP64 contexts)",
            "sequential_ms": round(seq_ms, 3), "streams_ms": round(par_ms, 3), "streams": group}


def copy_calibration(gib):
    """A plain device-to-device copy of known size (read n bytes, write n
    bytes), the reference of the HBM counters."""
    import torch
    n = int(gib * (1 << 30)) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": 8 * n, "launches": 3}), flush=True)


def cpu_baseline(case, nsteps, one_thread=True):
    """The FP64 oracle, as it stands, on the host cores: Steps 1-2 untimed,
    then `nsteps` pseudo-iterations timed on the full workload."""
    import numpy as np
    from oracle.oracle import Oracle
    o = Oracle(case)
    h, b, W, q = o.init_state()
    dts, dtp = o.timesteps()
    dt = case.dt_over_dts * dts
    Wn = W.copy()
    Sh, Sb, Fn = o.begin_step(dt, dts, h, b, W, q)
    t0 = time.perf_counter()
    for _ in range(nsteps):
        o.pseudo_step(dt, dts, dtp, h, b, W, Wn, q, Sh, Sb, Fn)
    sec = time.perf_counter() - t0
    pairs = o.ncell * o.nv
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {"value": pairs * nsteps / sec, "unit": "pair-updates/s", "cores": cores, "kind": "oracle",
           "sample": f"{nsteps} pseudo-iterations (after Steps 1-2) of the full workload, "
                     f"{pairs} pairs, {sec:.1f} s", "cpu_model": cpu_model()}
    if one_thread:
        # the same oracle on one thread (its OpenMP loops run over independent
        # velocities or cells, so the results are the same), one iteration
        import ctypes
        omp = ctypes.CDLL("libgomp.so.1")
        omp.omp_set_num_threads(1)
        try:
            t0 = time.perf_counter()
            o.pseudo_step(dt, dts, dtp, h, b, W, Wn, q, Sh, Sb, Fn)
            sec1 = time.perf_counter() - t0
        finally:
            omp.omp_set_num_threads(cores)
        out["one_thread"] = {"value": pairs / sec1, "sample": f"1 pseudo-iteration, {sec1:.1f} s"}
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def roofline(stages, pairs, prec, tuning, micro, workload):
    """Dominant measured kernel: algorithmic bytes per launch over its mean
    launch time (HIP events), against the HBM peak."""
    kv = kernel_values(micro)
    dom = max(kv, key=lambda k: stages[k])
    nbytes = 8 if prec == "f64" else 4
    algo = kv[dom] * nbytes * pairs
    t = stages[dom] * 1e-3
    achieved = algo / t / 1e9
    key = KERNEL_KEYS[dom].format(t="double" if prec == "f64" else "float", re=tuning["rg_eq"],
                                  rf=tuning["rg_flux"], kc=micro[0], mp=micro[2], mr=micro[1])
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_from_profiles(key, prec, workload),
            "kernel": KERNEL_NAMES[dom], "kernel_instance": key, "kernel_ms": round(stages[dom], 4), "algorithmic_bytes_per_launch": algo}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for {max(args.gpus, world)}): the pseudo-iteration "
              "is measured on a single MI355X; sharding the velocities over GPUs is designed, not built.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2604_09984_amd import workloads as wl
    from paper_2604_09984_amd import ugks
    ugks.lib()  # fail loudly when the HIP library is missing
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(3)
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
        return
    if args.workload is not None:
        k = max(args.workload_steps, 1)
        if args.workload == "sod":
            r = time_workload(wl.sod_1d(), "f64", 10 * k)
        elif args.workload == "plate":
            plate = wl.mems_plate(kn=0.1)
            r = {p: time_workload(plate, p, k, t_pose=plate.dt) for p in ("f32", "f64")}
        elif args.workload == "two_body":
            r = {p: time_workload(wl.two_body(), p, k, t_pose=0.25) for p in ("f32", "f64")}
        elif args.workload == "batch":
            r = time_batch(64, "f32", k)
            r["adjoint_f64"] = time_batch_adjoint(64)
        else:
            print(f"unknown workload {args.workload}", file=sys.stderr)
            sys.exit(2)
        print(json.dumps({"workload": args.workload, "result": r}), flush=True)
        return
    case = wl.cylinder(nvx=args.nvx)
    cyl_key = f"cylinder_128x64_v{args.nvx}x{args.nvx}"  # workload key of profiles/traffic.json
    r64 = run_gpu(case, "f64", args.steps, args.warmup, adjoint_calls=args.adjoint_calls)
    r32 = None if args.no_f32 else run_gpu(case, "f32", args.steps, args.warmup)
    ms64 = 1e3 * r64["wall_s"] / args.steps
    value = r64["pairs"] * args.steps / r64["wall_s"]
    st = r64["stages"]
    per_kernel = {}
    kv64 = kernel_values(r64["micro"])
    for k, nv in kv64.items():
        gbs = nv * 8 * r64["pairs"] / (st[k] * 1e-3) / 1e9
        per_kernel[k] = {"ms": round(st[k], 4), "algorithmic_GBs": round(gbs, 1)}
    total_values = sum(kv64.values())
    line = {
        "metric": "(cell x velocity) updates/s per pseudo-step",
        "value": value,
        "unit": "pair-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms64,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"Ma5 cylinder, O-mesh 128x64 cells, {args.nvx}x{args.nvx} velocities on "
                               f"[-15,15]^2, Kn 0.01 hard sphere, isothermal wall, dt = 20 dt_s",
                   "pairs": r64["pairs"], "pseudo_steps": args.steps, "launch": "hipGraph replay, 10 per replay"},
        "roofline": roofline(st, r64["pairs"], "f64", r64["tuning"], r64["micro"], cyl_key),
        "kernels_f64": per_kernel,
        "stages_ms_f64": {k: round(v, 4) for k, v in st.items()},
        "eager_ms_per_step_f64": round(r64["eager_ms"], 4),
        "launch_shapes_f64": dict(r64["tuning"], micro_kc=r64["micro"][0], micro_rows=r64["micro"][1],
                                  micro_fused_residual=bool(r64["micro"][3])),
        "hbm_algorithmic_GBs_f64": round(total_values * 8 * r64["pairs"] / (ms64 * 1e-3) / 1e9, 1),
    }
    if r32 is not None:
        ms32 = 1e3 * r32["wall_s"] / args.steps
        import numpy as np
        h64 = r64["h"].numpy().ravel()
        h32 = r32["h"].numpy().ravel()
        rel = float(np.linalg.norm(h32 - h64) / np.linalg.norm(h64))
        line["f32"] = {"value": r32["pairs"] * args.steps / r32["wall_s"], "ms_per_step": ms32,
                       "speedup_vs_f64": ms64 / ms32,
                       "rel_l2_h_vs_f64_after_run": rel,
                       "roofline": roofline(r32["stages"], r32["pairs"], "f32", r32["tuning"], r32["micro"], cyl_key),
                       "launch_shapes": r32["tuning"],
                       "stages_ms": {k: round(v, 4) for k, v in r32["stages"].items()}}
    if r64["adjoint_ms"] is not None:
        line["adjoint_f64"] = {"ms_per_pseudo_step": round(r64["adjoint_ms"], 3),
                               "ratio_to_forward_eager": round(r64["adjoint_ms"] / r64["eager_ms"], 2),
                               "finite": r64["adjoint_finite"],
                               "what": "ugks_step_adjoint: recomputation of one pseudo-iteration and its "
                                       "reverse pass (vector-Jacobian product w.r.t. f, W, q, S, Fn, block "
                                       "velocity and wall temperature)"}
    line["finite"] = r64["finite"] and (r32 is None or r32["finite"])
    if args.workload_steps > 0:
        # the other workloads at their full sizes (same metric, pair-updates/s)
        k = args.workload_steps
        wk = {}
        wk["sod_1d_f64"] = time_workload(wl.sod_1d(), "f64", 10 * k)
        for kn in (0.1, 1.0):
            plate = wl.mems_plate(kn=kn)
            for p in ("f32", "f64"):
                wk[f"mems_plate_kn{kn:g}_{p}"] = time_workload(plate, p, k, t_pose=plate.dt)
        tb = wl.two_body()
        for p in ("f32", "f64"):
            wk[f"two_body_{p}"] = time_workload(tb, p, k, t_pose=0.25)
        wk["batch64_f32"] = time_batch(64, "f32", k)
        wk["batch64_f32"]["adjoint_f64"] = time_batch_adjoint(64)
        line["workloads"] = wk
    if args.cpu_steps > 0:
        line["cpu_baseline"] = cpu_baseline(case, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
