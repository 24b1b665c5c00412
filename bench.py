"""Benchmark of the free-energy MRT lattice Boltzmann step on one MI355X.

Default workload: the batched sweep of 256 binary-fluid capillaries of uneven
size (H ~ U{10..80}, tube length ~ U[500, 4000], reservoir 256 x (H+40),
viscosity ratio log-uniform in [1, 100], contact angle ~ U[30, 90] degrees,
master seed 4), all advanced by one kernel launch per time step, replayed from
HIP graphs, with the filled length of every capillary recorded every 625 steps.
A step is one time step of all capillaries.  The metric is fluid-node updates
per second (MLUPS) with the populations resident in HBM before timing starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sweep|single4096|single1024|vdw4096|vdw16k|single16k]

Prints one JSON line.  Adds the roofline of the step kernel (algorithmic bytes
per fluid-node update x updates per launch / HIP-event launch time), the FP64
CPU oracle timed on a bounded sample of the same workload, and (sweep
workload) the wall time of the whole 100000-step sweep three ways: plain
sequential runs, one batched run, and the batched run with learned early
stopping, with the true error of every accepted tail.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per fluid-node update of the method: every FP32 population
# (and, binary, phi) read and written once.  The roofline's `achieved` uses these.
BYTES_PER_LUP = {"vdw": 72, "binary": 80}
BYTES_PER_LUP_MOMENT_STORAGE = 64            # schedule 6 (binary): 7 state planes + phi, read and written


def stored_bytes_per_lup(model: str, schedule: int) -> float:
    """Bytes per fluid-node update that the launch shape's own storage must
    move: the method's figure; 64 B for the binary moment storage, which
    stores the seven numbers that fix the post-collision populations; half the
    method's figure with two time steps per sweep, which reads and writes the
    populations once per two updates."""
    if model == "binary" and schedule == 6:
        return BYTES_PER_LUP_MOMENT_STORAGE
    return BYTES_PER_LUP[model] / 2 if schedule == 5 else BYTES_PER_LUP[model]


# the step kernels and the strip table that shapes their traffic
KERNEL_SOURCES = ("lb_internal.h", "lb_kernels.h", "lb_strip.h", "lb_strip_table.h", "lb_wide.h", "lb_wide2.h", "lb_wmom.h")


def code_of(text: str) -> str:
    """C++ source without its comments and blank space, so that editing a
    comment does not count as a change of the kernel."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash() -> str:
    """Hash of the code of the step kernels (the counter summary in profiles/
    is only used while it matches)."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(code_of(open(os.path.join(ROOT, "paper_0911_0459_amd", "csrc", name)).read()).encode())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel: str, workload: str, launch: dict):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if absent, taken on another version of the kernel source or taken
    with another strip chunking or arithmetic."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    keys = ("schedule", "chunk_rows", "fp64_arith", "tile_rows")
    for entry in [d] + d.get("other_launches", []):
        taken = entry.get("launch", {})
        if all(taken.get(k) == launch.get(k) for k in keys):
            return entry.get("hbm_bytes_per_launch")
    return None


def build_workload(name: str):
    from paper_0911_0459_amd import inputs as I
    if name == "sweep":
        return I.sweep_batch(4, 256, 100_000), {"workload": "sweep_256_binary_capillaries", "n_capillaries": 256,
                                              "master_seed": 4, "steps_per_run": 100_000, "sample_every": 625}
    if name == "single4096":
        w = I.binary_capillary_4096x256()
        return [w], {"workload": "binary_4096x256_ratio10_60deg", "lattice": "4096x256", "tube_h": 100,
                     "tube_len": 3072}
    if name == "vdw4096":
        w = I.vdw_capillary_4096x256()
        return [w], {"workload": "vdw_4096x256_60deg", "lattice": "4096x256", "tube_h": 100, "tube_len": 3072}
    if name == "vdw16k":
        w = I.vdw_capillary_16384x1024()
        return [w], {"workload": "vdw_16384x1024_60deg", "lattice": "16384x1024", "tube_h": 400,
                     "tube_len": 12288}
    if name == "single16k":
        w = I.binary_capillary_16384x1024()
        return [w], {"workload": "binary_16384x1024_ratio10_60deg", "lattice": "16384x1024", "tube_h": 400,
                     "tube_len": 12288}
    if name == "single1024":
        w = I.binary_capillary_1024x128()
        return [w], {"workload": "binary_1024x128_ratio10_60deg", "lattice": "1024x128", "tube_h": 40,
                     "tube_len": 768}
    raise SystemExit(f"unknown workload {name}")


def copy_bandwidth(L, reps: int = 20, nbytes: int = 1 << 31):
    """Read+write GB/s of the library's plain copy kernel on 2 GiB buffers."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    L.lb_stream_copy(b, a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        L.lb_stream_copy(b, a)
    e1.record()
    torch.cuda.synchronize()
    us = 1000.0 * e0.elapsed_time(e1) / reps
    return {"bytes_per_copy": 2 * nbytes, "us_per_copy": round(us, 1), "gbps": round(2 * nbytes / us / 1e3, 1)}


def make_oracle(w):
    """The FP64 oracle set up on workload w (the timing legs only)."""
    from oracle import Oracle, OracleGeom, OracleParams
    from oracle import physics as P
    G = w.wall_grad if w.wall_grad is not None else (
        P.binary_wall_gradient(w.theta_deg, w.kappa, w.A, w.B) if w.model == "binary"
        else P.vdw_wall_gradient(w.theta_deg, w.kappa, w.a, w.b, w.T))
    p = OracleParams(model=w.model, kappa=w.kappa, a=w.a, b=w.b, T=w.T, A=w.A, B=w.B, Gamma=w.Gamma,
                     nu_l=w.nu_l, nu_g=w.nu_g, wall_grad=G)
    return Oracle(p, OracleGeom(**w.geom.asdict()), w.initial_field())


def cpu_model() -> str:
    """Model name of the host CPU (first 'model name' line of /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(w, target_s: float = 15.0):
    """The FP64 oracle on one capillary of the workload, for a bounded number
    of steps (calibrated to about target_s seconds)."""
    import oracle
    o = make_oracle(w)
    fluid = w.geom.fluid_count()
    t0 = time.perf_counter()
    o.step(5)
    dt = time.perf_counter() - t0
    n = max(5, int(target_s / max(dt / 5, 1e-6)))
    t0 = time.perf_counter()
    o.step(n)
    dt = time.perf_counter() - t0
    return {"value": fluid * n / dt / 1e6, "unit": "MLUPS", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"capillary {w.name} ({w.geom.nx}x{w.geom.ny}, {fluid} fluid nodes), "
                      f"{n} steps, {dt:.1f} s",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def oracle_next_to_gpu(L, log):
    """The FP64 oracle and the GPU on the three single-lattice configurations:
    vdW 256x64 for 2000 steps, binary 1024x128 for 10^4 steps and binary
    4096x256 for 2000 steps (its 2*10^5-step run extrapolated linearly)."""
    import oracle
    import torch
    from paper_0911_0459_amd import inputs as I
    cases = [("vdw_256x64", I.vdw_capillary_256x64(), 2000, 2000),
             ("binary_1024x128", I.binary_capillary_1024x128(), 10_000, 10_000),
             ("binary_4096x256", I.binary_capillary_4096x256(), 2000, 200_000)]
    out = []
    for name, w, n, full in cases:
        fluid = w.geom.fluid_count()
        o = make_oracle(w)
        t0 = time.perf_counter()
        for k in range(0, n, 500):
            o.step(min(500, n - k))
            log(f"oracle {name}: {k + min(500, n - k)} of {n} steps, {time.perf_counter() - t0:.0f} s")
        t_cpu = time.perf_counter() - t0
        lat = L.Lattice(L.params_from_workload(w), L.geometry_from_workload(w), w.initial_field())
        lat.autotune(trial_steps=10)
        lat.step(50)
        lat.check()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(n)
        torch.cuda.synchronize()
        t_gpu = time.perf_counter() - t0
        lat.check()
        launch = lat.launch_config().asdict()
        lat.close()
        out.append({"config": name, "fluid_nodes": fluid, "steps": n,
                    "oracle_mlups": round(fluid * n / t_cpu / 1e6, 2), "oracle_s": round(t_cpu, 1),
                    "oracle_full_run_s": round(t_cpu * full / n, 1),
                    "gpu_mlups": round(fluid * n / t_gpu / 1e6, 1), "gpu_s": round(t_gpu, 4),
                    "gpu_launch": launch, "full_run_steps": full})
        log(f"{name}: oracle {out[-1]['oracle_mlups']} MLUPS, GPU {out[-1]['gpu_mlups']} MLUPS")
    return {"oracle_threads": oracle.threads(), "configs": out}


def plain_subset(works, n: int = 16):
    """n capillaries spanning the size range: every (len/n)-th by fluid-node count."""
    order = sorted(range(len(works)), key=lambda k: works[k].geom.fluid_count())
    return [order[(2 * j + 1) * len(order) // (2 * n)] for j in range(n)]


def sweep_compare(works, log, plain_full: bool = False):
    """Wall time of the 256-capillary sweep: plain sequential runs, one batched
    run, and the batched run with learned early stopping; the true error of
    every accepted tail is taken from the full batched run.  The plain time is
    measured, every capillary alone for all its steps, with plain_full;
    otherwise it is estimated from 1000 timed steps of each run, and 16 runs
    spanning the size range are also run in full to check the estimate."""
    import numpy as np
    from paper_0911_0459_amd import surrogate as S
    net_path = os.path.join(S.DATA_DIR, "surrogate_net.npz")
    if not os.path.exists(net_path):
        return None
    T = works[0].steps
    full = S.run_sweep(works, T, None, log=log)
    sur = S.Surrogate.load(net_path)
    early = S.run_sweep(works, T, sur, log=log)
    if plain_full:
        meas = S.plain_sequential(works, T, log=log)
        plain_s, note = meas["measured_s"], "measured: every capillary alone for all its steps"
        check = None
    else:
        est = S.plain_sequential_estimate(works, T, log=log)
        plain_s = est["estimated_s"]
        note = f"estimated from {est['sample_steps']} timed steps of each run"
        idx = plain_subset(works)
        meas = S.plain_sequential([works[k] for k in idx], T, log=log)
        est_sub = float(sum(est["per_run_s"][k] for k in idx))
        check = {"runs": len(idx), "measured_s": round(meas["measured_s"], 2), "estimated_s": round(est_sub, 2),
                 "measured_over_estimated": round(meas["measured_s"] / est_sub, 4)}
    hist = np.stack(full["hist"])
    p = S.RunParams.of(works)
    truth = S.interp_history(hist, T, S.out_times(T))
    acc = early["accept"]
    err = (np.abs(early["pred"] - truth) / truth).max(axis=1)
    wb = S.washburn_predict(p, hist[:, :S.N_EARLY], T)
    ev_wb = S.evaluate(p, wb, hist, T)
    acc_wb = ev_wb["accept"]
    return {
        "capillaries": len(works), "steps_per_run": T,
        "plain_sequential_s": round(plain_s, 1),
        "plain_sequential_note": note,
        "plain_subset_full_runs": check,
        "batched_s": round(full["wall_s"], 1),
        "batched_surrogate_s": round(early["wall_s"], 1),
        "speedup_batched_surrogate_vs_plain": round(plain_s / early["wall_s"], 2),
        "speedup_batched_surrogate_vs_batched": round(full["wall_s"] / early["wall_s"], 2),
        "accepted": int(acc.sum()),
        "accepted_true_err_max": round(float(err[acc].max()), 5) if acc.any() else None,
        "accepted_over_1pct": int(np.sum(acc & (err > 0.01))),
        "washburn_gate": {"accepted": int(acc_wb.sum()),
                          "accepted_over_1pct": int(np.sum(acc_wb & (ev_wb["true_err"] > 0.01)))},
        "unstable": int(np.sum(full["health"] != 0)),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="sweep",
                    choices=["sweep", "single4096", "single1024", "vdw4096", "vdw16k", "single16k"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tile-rows", type=int, default=0, help="pin the launch shape (with --schedule)")
    ap.add_argument("--schedule", type=int, default=-1)
    ap.add_argument("--fp64-arith", type=int, default=-1)
    ap.add_argument("--chunk-rows", type=int, default=-1)
    ap.add_argument("--graph-steps", type=int, default=-1, help="steps per HIP graph (0: direct launches)")
    ap.add_argument("--copy-probe", action="store_true", help="time the plain copy kernel only")
    ap.add_argument("--no-sweep", action="store_true", help="skip the sweep wall-time comparison")
    ap.add_argument("--plain-full", action="store_true",
                    help="measure the plain sequential sweep in full (every capillary alone for all its steps, "
                         "about 5 minutes) instead of estimating it")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="time the FP64 oracle next to the GPU on the three single-lattice configurations only")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the capillaries of a sweep are independent and would be dealt to ranks by fluid-node count)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_0911_0459_amd import lbcap as L

    torch.cuda.set_device(0)
    if args.copy_probe:
        print(json.dumps({"copy_probe": copy_bandwidth(L, args.steps)}))
        return
    if args.oracle_timing:
        log = lambda m: print(m, file=sys.stderr, flush=True)
        print(json.dumps({"oracle_next_to_gpu": oracle_next_to_gpu(L, log)}))
        return
    works, config = build_workload(args.workload)
    model = works[0].model
    params = [L.params_from_workload(w) for w in works]
    geoms = [L.geometry_from_workload(w) for w in works]
    fields = [w.initial_field() for w in works]
    lat = L.Lattice(params[0], geoms[0], fields[0]) if len(works) == 1 else L.Lattice(params, geoms, fields)
    del fields
    if not args.no_autotune:
        cfg, _ = lat.autotune(trial_steps=128)   # long trials: chunkings 1 % apart are told apart
    cfg = lat.launch_config()
    if args.tile_rows or args.schedule >= 0 or args.fp64_arith >= 0 or args.chunk_rows >= 0 or args.graph_steps >= 0:
        lat.set_launch_config(args.tile_rows or cfg.tile_rows, cfg.schedule if args.schedule < 0 else args.schedule,
                              cfg.persist_blocks_per_cu, cfg.graph_steps if args.graph_steps < 0 else args.graph_steps,
                              cfg.fp64_arith if args.fp64_arith < 0 else args.fp64_arith,
                              cfg.chunk_rows if args.chunk_rows < 0 else args.chunk_rows)
        cfg = lat.launch_config()
    sample_every = config.get("sample_every", 0)

    lat.step(args.warmup)
    lat.check()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(args.steps, sample_every=sample_every)
    us_kernel = lat.last_step_kernel_us()      # HIP events on the library's stream; synchronises
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    lat.check()

    fluid = lat.fluid_nodes
    mlups = fluid * args.steps / elapsed / 1e6
    bpl = BYTES_PER_LUP[model]
    sbpl = stored_bytes_per_lup(model, cfg.schedule)
    achieved = bpl * fluid / (us_kernel * 1e-6) / 1e9 if us_kernel > 0 else None
    kname = ({3: "lb_strip_", 4: "lb_wide_", 5: "lb_wide2_", 6: "lb_wmom_"}[cfg.schedule] + ("bin" if model == "binary" else "vdw")
             if cfg.schedule in (3, 4, 5, 6) else f"lb_step_kernel_{model}_{cfg.tile_rows}")
    traffic = traffic_from_profiles(kname, args.workload, cfg.asdict())
    config.update({"model": model, "fluid_nodes": fluid, "launch": cfg.asdict(), "bytes_per_lup": bpl,
                   "stored_bytes_per_lup": sbpl})
    out = {
        "metric": "MLUPS & %HBM peak; sweep wall-time batched+surrogate vs plain at <=1% l(t) err",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000 * elapsed / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": config,
        "roofline": {
            "bound": "hbm",
            "kernel": kname,
            "achieved": round(achieved, 1) if achieved else None,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
            "traffic": traffic,
            "frac_of_stored_bytes": round(sbpl / bpl * achieved / HBM_PEAK_GBS, 4) if achieved else None,
            "kernel_us": round(us_kernel, 3),
            "copy_kernel_gbps": copy_bandwidth(L, 10)["gbps"],
        },
        "cpu_baseline": None,
    }
    lat.close()
    del lat
    log = lambda m: print(m, file=sys.stderr, flush=True)
    if args.workload == "sweep" and not args.no_sweep:
        out["sweep"] = sweep_compare(works, log, plain_full=args.plain_full)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(works[0])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
