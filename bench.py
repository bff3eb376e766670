#!/usr/bin/env python
"""Throughput of the well-balanced phase-field LBM step on one MI355X.

Workload: 16384 x 16384 periodic grid, 2000 seeded non-overlapping drops with
radius ~ U(20, 80), density ratio 100, nu 0.1/0.1, sigma 5e-4, M 0.05, W 4
(synthetic input; there is no dataset).  One step = phi, mu, both
collisions and the pull streaming, through the C ABI; the library's
automatic path runs FP32 steps on this grid two per launch (k_step2, the
intermediate state kept on chip) and FP64 steps one per launch.

Prints one JSON line: FP32 (deviation storage) MLUPS as the value, the FP64
step beside it, the roofline of the step kernel measured with HIP events on
the library's stream, the one-step, two-kernel and MRT forms of the FP32
step, the
4096^2 two-drop coalescence in both precisions, the adjoint/forward cost
ratio of the 1024^2 (and 2048^2) inverse problem, and the CPU oracle timed
on a bounded sample of the workload (the same recipe on a periodic 1024^2
grid), with the FP64 and FP32 GPU errors against it on that sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & % HBM roofline, FP32 vs FP64 step; adjoint/forward step cost ratio"
HBM_PEAK_GBPS = 8000.0
# Algorithmic HBM bytes per lattice update (per cell) of one step: the
# method's state, 18 populations and the previous-step source, each read once
# and written once (152 B in FP32, 304 B in FP64).  The roofline fraction is
# taken on these.
STEP_BYTES = {32: 2 * 19 * 4, 64: 2 * 19 * 8}
# What the fused step kernel itself moves: in FP32 also the 16-bit low word
# of the rest population of f (read and written) that keeps f_0 to about
# 2^-40; phi and mu stay on chip.
STEP_IMPL_BYTES = {32: 2 * (18 * 4 + 2 + 4), 64: STEP_BYTES[64]}
# Two steps per launch: the state read and written once per two steps (with
# the 32-bit low word of f_0, which the library keeps on that path).
TWO_STEP_IMPL_BYTES = {32: (18 * 4 + 4 + 4) * 2 / 2}
# The two-kernel design: the phi/mu pass also reads the 9 f planes and writes
# phi and mu, and the collide pass reads them back: +(9 + 2 + 2) planes.
TWO_KERNEL_BYTES = {32: STEP_BYTES[32] + (9 + 2 + 2) * 4, 64: STEP_BYTES[64] + (9 + 2 + 2) * 8}
# ... and with the low word of f_0 (read twice, written once) in FP32
TWO_KERNEL_IMPL_BYTES = {32: STEP_IMPL_BYTES[32] + (9 + 2 + 2) * 4 + 2, 64: TWO_KERNEL_BYTES[64]}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step_fused_many_drops_16384.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the HIP sources (the counters are only valid for this code)."""
    d = os.path.join(ROOT, "paper_2311_10827_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name), "rb") as fh:
            h.update(name.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(key: str):
    """HBM bytes per launch of a step kernel ("two_step_32": two steps,
    "two_step_32_mrt" with the MRT collision; "32", "64": one step), or per
    step of the two-kernel path ("two_kernel_32"),
    from the committed rocprofv3 counter summary, if it was taken on the
    current kernel source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    rec = t.get(key)
    if not rec or t.get("source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch", rec.get("bytes_per_step"))


# MRT rates of the MRT leg: f (e, eps, q, p), g ((rho, e, eps), q)
MRT_LEG = dict(collision=1, mrt_f=(1.3, 1.1, 1.6, 1.4), mrt_g=(1.5, 1.7))


def run_gpu(phi0_dev, prec: int, steps: int, warmup: int, kernel_steps: int, wl, kernel_path: int = 0,
            mrt: bool = False, bufs=None):
    """kernel_path 0: the library's choice (two steps per launch for FP32
    here), 2: one fused step per launch, 1: the two-kernel step."""
    import torch
    from paper_2311_10827_amd.sim import Sim, derive, make_params

    p = make_params(wl, precision=prec, kernel_path=kernel_path, **(MRT_LEG if mrt else {}))
    per_launch = 2 if derive(p)["two_step"] else 1
    state, ws = bufs if bufs is not None else (None, None)
    sim = Sim(p, phi0_dev, device=phi0_dev.device, state=state, workspace=ws)
    stream = sim.stream
    ncell = wl.nx * wl.ny
    form = {1: "two-kernel", 2: "one-step"}.get(kernel_path, "two-step" if per_launch == 2 else "one-step")
    tag = f"fp{prec} {form}{' MRT' if mrt else ''}"
    log(f"[bench] {tag}: warmup {warmup}")
    sim.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    log(f"[bench] {tag}: timing {steps} steps")
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    # kernel durations with HIP events the library records on its own stream
    log(f"[bench] {tag}: per-kernel timing over {kernel_steps} steps")
    sim.timing(True)
    sim.step(kernel_steps)
    kms, n = sim.kernel_times()
    sim.timing(False)
    m = sim.moments()
    d = m["diag"]
    del m
    sim.close()
    del sim
    torch.cuda.empty_cache()
    avg = kms / n  # ms per step
    if kernel_path == 1:
        alg, impl, key = TWO_KERNEL_BYTES[prec], TWO_KERNEL_IMPL_BYTES[prec], f"two_kernel_{prec}"
    elif per_launch == 2:
        alg, impl, key = STEP_BYTES[prec], TWO_STEP_IMPL_BYTES[prec], f"two_step_{prec}"
    else:
        alg, impl, key = STEP_BYTES[prec], STEP_IMPL_BYTES[prec], str(prec)
    # algorithmic bytes per launch (steps per launch x cells x bytes per
    # cell update) over the launch's duration
    ach = alg * ncell / (avg * 1e-3) / 1e9
    # counters were taken for the MRT collision on the two-step path only
    traffic = measured_traffic(key + "_mrt" if per_launch == 2 else "") if mrt else measured_traffic(key)
    launch_ms = avg * (per_launch if kernel_path != 1 else 1)
    return {
        "mlups": ncell * steps / (ms * 1e-3) / 1e6,
        "ms_per_step": ms / steps,
        "wall_s": wall,
        "kernel_ms": avg,
        "steps_per_launch": per_launch if kernel_path != 1 else 1,
        "algorithmic_bytes_per_cell": alg,
        "implementation_bytes_per_cell": impl,
        "implementation_GBps": round(impl * ncell / (avg * 1e-3) / 1e9, 1),
        "roofline": {
            "bound": "hbm",
            "achieved": round(ach, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBPS, 4),
            "traffic": traffic,
        },
        # the counted HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE,
        # calibrated) over the same live launch time
        "measured_bytes_frac": None if traffic is None
        else round(traffic / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        # the same counted bytes per cell update (two steps per launch: the
        # state is read and written once for two updates)
        "counted_bytes_per_cell_update": None if traffic is None
        else round(traffic / ((per_launch if kernel_path != 1 else 1) * ncell), 1),
        "diag_after": {k: d[k] for k in ("sum_phi", "max_u", "min_rho", "n_nonfinite", "step")},
    }


def placement_median(times, alg_bytes, ncell):
    """The median of the placement probe's per-step times (every allocation it
    tried) and the roofline fraction on algorithmic bytes at that median, to
    stand beside the kept (fastest) allocation's."""
    import statistics
    med = statistics.median(times)
    return {"ms_per_step": round(med, 4),
            "frac": round(alg_bytes * ncell / (med * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}


def stream_copy_probe(device, nbytes=4 << 30, reps=10):
    import torch
    from paper_2311_10827_amd.sim import stream_copy
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=device).fill_(1.0)
    b = torch.empty_like(a)
    stream_copy(b, a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        stream_copy(b, a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, seconds: float, dev):
    """FP64 oracle (plain loops, OpenMP over rows) timed on a 1024^2 sample
    of the workload: the same many-drop recipe on a periodic 1024^2 grid
    (drops scaled with the area, 8 of them).  A window cut out of the
    16384^2 field would not do: drops cut at its edges meet across the
    periodic seam as phi jumps of up to 2 between neighbours, and the run
    diverges within 50 steps.  The GPU then runs the same field for the
    same steps in FP64 and FP32, and their phi and velocity errors against
    the oracle are returned beside the timing."""
    import numpy as np
    import torch
    import oracle
    from paper_2311_10827_amd import inputs
    from paper_2311_10827_amd.sim import Sim, make_params
    oracle.build(force=False)
    n = 1024
    nd = round(wl.extra["ndrops"] * n * n / (wl.nx * wl.ny))
    phi = inputs.many_drops(n, nd, wl.extra["rmin"], wl.extra["rmax"], wl.W)
    o = oracle.Sim(oracle.params_for(wl, nx=n, ny=n)).init(phi)
    t = time.perf_counter()
    o.step(2)
    per = (time.perf_counter() - t) / 2
    k = max(2, int(seconds / max(per, 1e-6)))
    t = time.perf_counter()
    o.step(k)
    dt = time.perf_counter() - t
    sample = (f"1024x1024 periodic grid, the many-drop recipe with {nd} drops (the 16384^2 density), "
              f"{k} FP64 steps, {dt:.1f} s")
    base = {
        "value": round(n * n * k / dt / 1e6, 3),
        "unit": "MLUPS",
        "cores": oracle.get_threads(),
        "kind": "oracle",
        "sample": sample,
    }
    om = o.moments()
    del o
    # the same oracle on one thread, a few steps of the same field
    threads = oracle.get_threads()
    oracle.set_threads(1)
    o1 = oracle.Sim(oracle.params_for(wl, nx=n, ny=n)).init(phi)
    t = time.perf_counter()
    o1.step(2)
    k1 = max(2, int(min(seconds / 3, 5.0) / max(time.perf_counter() - t, 1e-6) * 2))
    t = time.perf_counter()
    o1.step(k1)
    dt1 = time.perf_counter() - t
    del o1
    oracle.set_threads(threads)
    base["single_thread"] = {"value": round(n * n * k1 / dt1 / 1e6, 3), "unit": "MLUPS", "steps": k1,
                             "seconds": round(dt1, 2)}
    base["cpu_model"] = cpu_model()
    err = {"sample": f"the same 1024^2 field, {k + 2} steps on the GPU (the step form it takes at that size)",
           "oracle_max_u": float(np.hypot(om["ux"], om["uy"]).max())}
    phi_dev = torch.from_numpy(phi).to(dev)
    for prec in (64, 32):
        sim = Sim(make_params(wl, precision=prec, nx=n, ny=n), phi_dev, device=dev)
        sim.step(k + 2)
        m = sim.moments(diag=False)
        err[f"fp{prec}"] = {
            "max_abs_phi": float(np.abs(m["phi"].cpu().numpy() - om["phi"]).max()),
            "max_abs_u": max(float(np.abs(m["ux"].cpu().numpy() - om["ux"]).max()),
                             float(np.abs(m["uy"].cpu().numpy() - om["uy"]).max())),
        }
        sim.close()
        del sim, m
    log(f"[bench] errors against the oracle: {err}")
    return base, err


def coalescence_leg(dev, steps: int, warmup: int):
    """Two-drop coalescence at 4096^2 (R 400, W 5, seeded noise 1e-3,
    density ratio 1000, dynamic viscosity ratio 100): ms per step and MLUPS
    in FP32 and FP64, with HIP events on the library's stream."""
    import torch
    from paper_2311_10827_amd import inputs
    from paper_2311_10827_amd.sim import Sim, make_params
    wl = inputs.COALESCENCE
    phi = inputs.two_drops(wl.nx, wl.ny, wl.extra["R"], wl.W, noise=wl.extra["noise"], workload_id=3)
    phi_dev = torch.from_numpy(phi).to(dev)
    out = {"workload": f"{wl.name}: {wl.nx}x{wl.ny} periodic, two drops R {wl.extra['R']:g} touching at "
                       f"the centre, noise 1e-3, density ratio 1000, viscosity ratio 100, sigma 1e-3, "
                       f"M 0.05, W 5; {steps} timed steps"}
    for prec in (32, 64):
        sim = Sim(make_params(wl, precision=prec), phi_dev, device=dev)
        sim.step(warmup)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        sim.step(steps)
        e1.record(sim.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out[f"fp{prec}"] = {"ms_per_step": round(ms, 5), "mlups": round(wl.nx * wl.ny / (ms * 1e-3) / 1e6, 1)}
        sim.close()
        del sim
    del phi_dev
    torch.cuda.empty_cache()
    log(f"[bench] coalescence 4096^2: {out}")
    return out


def adjoint_leg(nsteps: int, K: int, n: int = 0):
    """Inverse-problem gradient on the 1024^2 two-drop workload (FP32): the
    adjoint step's cost, including its share of the checkpoint recompute,
    relative to a forward step on the fastest of the library's step forms at
    this size (fused, two-kernel, two steps per launch; at 1024^2 the
    forward state fits in the GPU's caches and the fused step is the
    fastest).  n > 0: the same workload on an n x n grid, drop radius scaled
    with it."""
    import dataclasses

    import torch
    from paper_2311_10827_amd import inputs
    from paper_2311_10827_amd.adjoint import misfit, params_from_theta, rollout
    from paper_2311_10827_amd.sim import Sim, derive, make_params

    wl = inputs.ADJOINT
    if n:
        wl = dataclasses.replace(wl, name=f"adjoint_{n}", nx=n, ny=n,
                                 extra={**wl.extra, "R": wl.extra["R"] * n / wl.nx})
    base = make_params(wl, precision=32)
    d = derive(base)
    theta = [d["kappa"], d["beta"], base.M, d["tau_f"], d["tau_gA"], d["tau_gB"]]
    phi0 = inputs.two_drops(wl.nx, wl.ny, wl.extra["R"], wl.W, workload_id=5)
    s1, s2 = inputs.rng_for(5).uniform(0.5, 2.0, size=2)
    hidden = list(theta)
    hidden[0] *= s1
    hidden[1] *= s1          # sigma scaled by s1 at fixed W
    hidden[2] *= s2          # M scaled by s2
    log(f"[bench] adjoint: target with hidden (sigma, M) x ({s1:.3f}, {s2:.3f})")
    tgt = Sim(params_from_theta(base, hidden), phi0).step(nsteps).moments(diag=False)["phi"]
    # forward step time of the same workload on every step form; the fastest
    # is the reference.  The rollout (and so its checkpoint recompute, which
    # writes every state to a snapshot of its own) runs the fused kernel,
    # which writes fewer bytes per recomputed state.
    # Both parts of the ratio are the median of three timed runs (each run
    # varies by 1-2 % from the next).
    import statistics
    t_fwd, runs_fwd = {}, {}
    for kp in (2, 1, 3):
        base.kernel_path = kp
        sim = Sim(params_from_theta(base, theta), phi0)
        sim.step(20)
        runs = []
        for _ in range(3):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(sim.stream)
            sim.step(nsteps)
            e1.record(sim.stream)
            torch.cuda.synchronize()
            runs.append(e0.elapsed_time(e1) / nsteps)
        t_fwd[kp], runs_fwd[kp] = statistics.median(runs), runs
        sim.close()
        del sim
    kp_best = min(t_fwd, key=t_fwd.get)
    base.kernel_path = 2
    log(f"[bench] adjoint: forward ms/step fused {t_fwd[2]:.4f}, two-kernel {t_fwd[1]:.4f}, "
        f"two steps per launch {t_fwd[3]:.4f}")
    log(f"[bench] adjoint: rollout {nsteps} steps, checkpoint every {K} (one warm-up gradient, "
        "then three timed ones: buffers come from torch's caching allocator)")
    runs_bwd = []
    for i in range(4):
        ph = torch.from_numpy(phi0).cuda().requires_grad_(True)
        th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
        stats = {}
        L = misfit(rollout(ph, th, base, nsteps, K, stats), tgt)
        L.backward()
        if i:
            runs_bwd.append(stats["backward_s"] * 1e3 / nsteps)
    t_bwd = statistics.median(runs_bwd)
    return {
        "workload": f"{wl.name}: {wl.nx}x{wl.ny} two drops R {wl.extra['R']:g}, density ratio 100, FP32, "
                    f"{nsteps} steps, checkpoint every {K}",
        "forward_ms_per_step": round(t_fwd[kp_best], 5),
        "forward_ms_per_step_fused": round(t_fwd[2], 5),
        "forward_ms_per_step_two_kernel": round(t_fwd[1], 5),
        "forward_ms_per_step_two_step": round(t_fwd[3], 5),
        "forward_reference": {2: "fused", 1: "two-kernel", 3: "two steps per launch"}[kp_best],
        "rollout_step_form": "fused",
        "adjoint_ms_per_step_incl_recompute": round(t_bwd, 5),
        "ratio": round(t_bwd / t_fwd[kp_best], 3),
        "runs_ms_per_step": {"forward": [round(t, 5) for t in runs_fwd[kp_best]],
                             "adjoint": [round(t, 5) for t in runs_bwd]},
        "loss": float(L.detach()),
        "dL_dtheta": dict(zip(("kappa", "beta", "M", "tau_f", "tau_gA", "tau_gB"),
                              [float(v) for v in th.grad])),
        "dL_dphi0_norm": float(ph.grad.norm()),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--fp64-steps", type=int, default=None, help="default: --steps")
    ap.add_argument("--kernel-steps", type=int, default=100)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-two-kernel", action="store_true")
    ap.add_argument("--no-one-step", action="store_true")
    ap.add_argument("--no-mrt", action="store_true")
    ap.add_argument("--no-coalescence", action="store_true")
    ap.add_argument("--coalescence-steps", type=int, default=1000)
    ap.add_argument("--place-tries", type=int, default=5,
                    help="allocations the state placement probe tries (1: take the first)")
    ap.add_argument("--adjoint-steps", type=int, default=2000)
    ap.add_argument("--adjoint-K", type=int, default=100)
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the adjoint leg and print its result (for profiling it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested); the multi-GPU "
              "slab decomposition is a design, not a build, here", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2311_10827_amd import inputs

    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_leg(args.adjoint_steps, args.adjoint_K),
                          "adjoint_2048": adjoint_leg(args.adjoint_steps, args.adjoint_K, 2048)}), flush=True)
        return

    wl = inputs.THROUGHPUT
    dev = torch.device("cuda:0")
    # the adjoint legs first, while the heap is fresh
    adj = None if args.no_adjoint else adjoint_leg(args.adjoint_steps, args.adjoint_K)
    # the same at 2048^2, where the forward state no longer fits in the caches
    adj2 = None if args.no_adjoint else adjoint_leg(args.adjoint_steps, args.adjoint_K, 2048)
    import gc
    gc.collect()
    torch.cuda.empty_cache()
    log(f"[bench] after the adjoint legs: {torch.cuda.memory_allocated() / 2**30:.2f} GiB still allocated")
    log("[bench] generating the 16384^2 many-drop field")
    phi0 = inputs.many_drops(wl.nx, wl.extra["ndrops"], wl.extra["rmin"], wl.extra["rmax"], wl.W)
    phi0_dev = torch.from_numpy(phi0).to(dev)
    del phi0
    # The step time depends (by up to about 10 %) on where in HBM the state
    # lands; the state is placed with the library's allocation probe (the
    # fastest of a few allocations over a few steps, all reported), and the
    # FP32 legs share that one allocation, which keeps them comparable.
    from paper_2311_10827_amd.sim import make_params, pick_state_buffers
    probe = {}
    log(f"[bench] fp32: placing the state (best of {args.place_tries} allocations)")
    st32, ws32, probe["fp32"] = pick_state_buffers(make_params(wl, precision=32), phi0_dev,
                                                   tries=args.place_tries)
    bufs32 = (st32, ws32)
    r32 = run_gpu(phi0_dev, 32, args.steps, args.warmup, args.kernel_steps, wl, bufs=bufs32)
    r1s = None
    if not args.no_one_step:
        r1s = run_gpu(phi0_dev, 32, max(args.steps // 4, 10), args.warmup, args.kernel_steps, wl, kernel_path=2,
                      bufs=bufs32)
    r2k = None
    if not args.no_two_kernel:
        r2k = run_gpu(phi0_dev, 32, max(args.steps // 4, 10), args.warmup, args.kernel_steps, wl, kernel_path=1,
                      bufs=bufs32)
    rmrt = None
    if not args.no_mrt:
        rmrt = run_gpu(phi0_dev, 32, max(args.steps // 4, 10), args.warmup, args.kernel_steps, wl, mrt=True,
                       bufs=bufs32)
    del bufs32, st32, ws32
    torch.cuda.empty_cache()
    r64 = None
    if not args.no_fp64:
        log(f"[bench] fp64: placing the state (best of {args.place_tries} allocations)")
        st64, ws64, probe["fp64"] = pick_state_buffers(make_params(wl, precision=64), phi0_dev,
                                                       tries=args.place_tries)
        r64 = run_gpu(phi0_dev, 64, args.fp64_steps or args.steps, args.warmup, args.kernel_steps, wl,
                      bufs=(st64, ws64))
        del st64, ws64
        torch.cuda.empty_cache()
    del phi0_dev
    torch.cuda.empty_cache()
    copy_gbps = None if args.no_copy else stream_copy_probe(dev)
    coal = None if args.no_coalescence else coalescence_leg(dev, args.coalescence_steps, args.warmup)
    cpu, err = (None, None) if args.no_cpu else cpu_baseline(wl, args.cpu_seconds, dev)

    out = {
        "metric": METRIC,
        "value": round(r32["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "many_drops_16384: 16384x16384 periodic, 2000 drops R~U(20,80), "
                        "density ratio 100, nu 0.1/0.1, sigma 5e-4, M 0.05, W 4",
            "nx": wl.nx, "ny": wl.ny, "precision": "fp32 deviation storage",
            "parallelism": "single GPU",
        },
        "roofline": r32["roofline"],
        "measured_bytes_frac": r32["measured_bytes_frac"],
        "counted_bytes_per_cell_update": r32["counted_bytes_per_cell_update"],
        "steps_per_launch": r32["steps_per_launch"],
        "cpu_baseline": cpu,
        "error_vs_oracle": err,
        "kernel_ms": round(r32["kernel_ms"], 4),
        "algorithmic_bytes_per_cell": r32["algorithmic_bytes_per_cell"],
        "implementation_bytes_per_cell": r32["implementation_bytes_per_cell"],
        "implementation_GBps": r32["implementation_GBps"],
        "stream_copy_GBps": None if copy_gbps is None else round(copy_gbps, 1),
        "placement_probe_ms_per_step": {k: [round(t, 4) for t in v] for k, v in probe.items()},
        "placement_probe_median": {k: placement_median(v, STEP_BYTES[int(k[2:])], wl.nx * wl.ny)
                                   for k, v in probe.items()},
        "fp64": None if r64 is None else {
            "value": round(r64["mlups"], 1), "unit": "MLUPS", "ms_per_step": round(r64["ms_per_step"], 4),
            "kernel_ms": round(r64["kernel_ms"], 4),
            "algorithmic_bytes_per_cell": r64["algorithmic_bytes_per_cell"],
            "roofline": r64["roofline"], "measured_bytes_frac": r64["measured_bytes_frac"],
        },
        "one_step_fp32": None if r1s is None else {
            "value": round(r1s["mlups"], 1), "unit": "MLUPS", "ms_per_step": round(r1s["ms_per_step"], 4),
            "kernel_ms": round(r1s["kernel_ms"], 4),
            "algorithmic_bytes_per_cell": r1s["algorithmic_bytes_per_cell"],
            "implementation_bytes_per_cell": r1s["implementation_bytes_per_cell"], "roofline": r1s["roofline"],
            "measured_bytes_frac": r1s["measured_bytes_frac"],
        },
        "two_kernel_fp32": None if r2k is None else {
            "value": round(r2k["mlups"], 1), "unit": "MLUPS", "ms_per_step": round(r2k["ms_per_step"], 4),
            "algorithmic_bytes_per_cell": r2k["algorithmic_bytes_per_cell"],
            "implementation_bytes_per_cell": r2k["implementation_bytes_per_cell"], "roofline": r2k["roofline"],
            "measured_bytes_frac": r2k["measured_bytes_frac"],
        },
        "mrt_fp32": None if rmrt is None else {
            "value": round(rmrt["mlups"], 1), "unit": "MLUPS", "ms_per_step": round(rmrt["ms_per_step"], 4),
            "kernel_ms": round(rmrt["kernel_ms"], 4),
            "algorithmic_bytes_per_cell": rmrt["algorithmic_bytes_per_cell"],
            "steps_per_launch": rmrt["steps_per_launch"],
            "roofline": rmrt["roofline"], "rates": {"f": MRT_LEG["mrt_f"], "g": MRT_LEG["mrt_g"]},
        },
        "fp32_fp64_ratio": None if r64 is None else round(r32["mlups"] / r64["mlups"], 3),
        "adjoint_forward_ratio": None if adj is None else adj["ratio"],
        "adjoint": adj,
        "adjoint_2048": None if adj2 is None else {
            k: adj2[k] for k in ("workload", "forward_ms_per_step", "forward_reference",
                                 "adjoint_ms_per_step_incl_recompute", "ratio")},
        "coalescence_4096": coal,
        "diag_after": r32["diag_after"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
