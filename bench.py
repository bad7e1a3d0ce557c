#!/usr/bin/env python3
"""Benchmark of the PonD f+g step (DDF-BGK, total-energy split, D2Q16) on one MI355X.

Workload: 512 x 512 periodic grid, uniform background (rho = 1, T = 1) advected
at Mach 2 (30 degrees), plus 8 seeded random-phase shear / acoustic / entropy
Fourier modes of amplitude 1e-3; tau = 0.55, Pr = 0.71, gamma = 1.4; FP32
populations with FP64 conserved moments and frame iteration (``--precision
fp64`` for the all-double path).  A step is one pass of the whole hot path over
the grid: moment pre-pass + step kernel (gather, predictor-corrector,
re-projection, collision, store).  Inputs are resident in HBM before the timed
region; W untimed warm-up steps, then exactly K timed steps bracketed by
synchronisations, timed with HIP events on the context's stream.

Prints ONE JSON line on stdout (everything else goes to stderr).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published MI355X peaks (dense, no sparsity).
PEAK_FP32_TFLOPS = 157.3        # vector FP32 with packed (dual) FMA
PEAK_FP32_NONPACKED_TFLOPS = 78.6
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# Algorithmic flops of the step kernel per node-update, from the method's
# arithmetic in interpolate-then-transform form (derivation in the design notes):
#   per predictor-corrector iteration: departure points and cubic weights 112,
#   interpolation 16 velocities x 16 taps x (1 weight product + 20 moments x FMA)
#   = 10496, frame transformation 16 velocities x 2 distributions x 65 = 2080;
#   once per node: moments of the gathered populations 784, re-projection 110,
#   collision 60, reconstruction 640.
FLOPS_PER_ITER = 112 + 10496 + 2080
FLOPS_PER_NODE = 784 + 110 + 60 + 640
# double-precision part: conserved sums and frame per iteration, equilibrium once
FLOPS64_PER_ITER = 140
FLOPS64_PER_NODE = 60
# Algorithmic HBM bytes of the step kernel per node (FP32 mode): frame read 24,
# moment planes read 80, populations + frame written 128 + 24.
BYTES_STEP_FP32 = 24 + 80 + 152
BYTES_STEP_FP64 = 24 + 160 + 280
TILE_DIMS = {0: "16,16", 1: "32,8", 2: "16,8", 3: "8,8", 4: "256,1", 5: "64,1"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """sha256 over the kernel sources (csrc/*.h, *.hip, by file name): ties an
    HBM-traffic record in profiles/ to the code it was measured on."""
    import hashlib
    d = os.path.join(ROOT, "paper_2405_11489_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".h", ".hip")):
            with open(os.path.join(d, name), "rb") as fh:
                h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def traffic_record(kernel, precision):
    """HBM bytes per launch of ``kernel`` from a 'traffic-record:' line of a
    profiles/*.md summary (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled
    by the same counter's reading for a plain copy of known size), or None when
    no record matches the current kernel sources."""
    d = os.path.join(ROOT, "profiles")
    if not os.path.isdir(d):
        return None
    want = kernel_source_hash()
    for name in sorted(os.listdir(d)):
        if not name.endswith(".md"):
            continue
        with open(os.path.join(d, name)) as fh:
            for line in fh:
                if not line.startswith("traffic-record:"):
                    continue
                kv = dict(t.split("=", 1) for t in line.split()[1:] if "=" in t)
                if (kv.get("kernel") == kernel and kv.get("precision") == precision
                        and kv.get("sources_sha256") == want):
                    return float(kv["bytes_per_launch"])
    return None


def cpu_baseline(w, seconds):
    """The FP64 oracle, unmodified, timed on this host's cores: whole-grid steps
    of the same workload from its initial state, as many as fit in
    ~``seconds`` (at least one); if one whole-grid step would take much
    longer, one step at a random sample of nodes instead."""
    import oracle
    P = oracle.params(w.nx, w.ny, tau=w.tau, gamma=w.gamma, prandtl=w.prandtl, bc_x=w.bc_x,
                      bc_y=w.bc_y)
    s = oracle.init(P, w.rho.ravel(), w.ux.ravel(), w.uy.ravel(), w.T.ravel())
    rng = np.random.default_rng(0)
    pilot = rng.integers(0, w.nodes, 512)
    t0 = time.perf_counter()
    oracle.step_nodes(P, s, pilot)
    step_s = (time.perf_counter() - t0) / len(pilot) * w.nodes
    if step_s <= seconds:
        nsteps, iters, dt = 0, 0, 0.0
        while dt < seconds:
            t0 = time.perf_counter()
            s, st = oracle.step(P, s, 1)
            dt += time.perf_counter() - t0
            nsteps += 1
            iters += st.total_iters
        updates = nsteps * w.nodes
        sample = (f"{nsteps} whole-grid step(s) of the {w.nx}x{w.ny} workload from its initial "
                  f"state (mean {iters / updates:.2f} PC gathers), {dt:.1f} s")
    else:
        count = int(max(1024, seconds / step_s * w.nodes))
        nodes = rng.permutation(w.nodes)[:count]
        t0 = time.perf_counter()
        _, _, _, iters, _ = oracle.step_nodes(P, s, nodes)
        dt = time.perf_counter() - t0
        updates = count
        sample = (f"one step at {count} random nodes of the {w.nx}x{w.ny} workload "
                  f"(initial state, mean {iters.mean():.2f} PC gathers), {dt:.1f} s")
    return {"value": updates / dt / 1e6, "unit": "MLUPS", "cores": oracle.num_threads(),
            "kind": "oracle", "sample": sample}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--interp-points", type=int, default=4, choices=[3, 4])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel", choices=["tiled", "global"], default="tiled")
    ap.add_argument("--tile", type=int, default=None, help="POND_TILE_* id (default: library's)")
    ap.add_argument("--lds-nodes", type=int, default=None)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the timed region, run 3 plain device copies of MIB MiB each "
                         "(the reference kernel for scaling HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "sharding of the step is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2405_11489_amd import pond, workloads

    torch.cuda.set_device(0)
    prec = pond.PREC_FP32 if args.precision == "fp32" else pond.PREC_FP64
    w = workloads.fourier_modes(n=512, mach=2.0, angle_deg=30.0, amplitude=1e-3, seed=0,
                                tau=0.55, prandtl=0.71, gamma=1.4, steps=2000)
    stream = torch.cuda.Stream()
    tuning = {"kernel": pond.KERNEL_TILED if args.kernel == "tiled" else pond.KERNEL_GLOBAL}
    if args.tile is not None:
        tuning["tile"] = args.tile
    if args.lds_nodes is not None:
        tuning["lds_nodes"] = args.lds_nodes
    sol = pond.Solver.from_workload(w, precision=prec, stream=stream.cuda_stream,
                                    interp_points=args.interp_points, tuning=tuning)
    tun = pond.pond_get_tuning(sol.ctx)
    log(f"workload {w.name} {w.nx}x{w.ny}, {args.precision}, warmup {args.warmup}, "
        f"steps {args.steps}")
    sol.step(args.warmup)
    sol.synchronize()
    st0 = sol.stats()

    pond.pond_profile_enable(sol.ctx, True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    sol.step(args.steps)
    ev1.record(stream)
    ev1.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    prof = pond.pond_profile_read(sol.ctx)
    pond.pond_profile_enable(sol.ctx, False)
    st1 = sol.stats()
    sol.close()
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 x {n * 4} bytes read + written")
        del a, b

    N = w.nodes
    updates = N * args.steps
    mlups = updates / (ms * 1e-3) / 1e6
    kbar = (st1.pc_iterations - st0.pc_iterations) / updates
    step_ms = prof.step_ms / max(prof.launches, 1)
    pre_ms = prof.prepass_ms / max(prof.launches, 1)
    log(f"time {ms:.1f} ms (host {wall * 1e3:.1f} ms), {mlups:.1f} MLUPS, K {kbar:.3f}, "
        f"kernels: step {step_ms:.4f} ms, prepass {pre_ms:.4f} ms per launch")

    flops = N * (FLOPS_PER_ITER * kbar + FLOPS_PER_NODE)
    kname = f"step_tiled_kernel<{'float' if prec == pond.PREC_FP32 else 'double'},{args.interp_points}," \
            f"{TILE_DIMS[tun.tile]}>" if args.kernel == "tiled" else \
            f"step_kernel<{'float' if prec == pond.PREC_FP32 else 'double'},{args.interp_points}>"
    traffic = traffic_record(kname, args.precision)
    if prec == pond.PREC_FP32:
        achieved = flops / (step_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                "traffic_unit": "HBM bytes per launch",
                "peak_nonpacked": PEAK_FP32_NONPACKED_TFLOPS,
                "frac_nonpacked": achieved / PEAK_FP32_NONPACKED_TFLOPS,
                "kernel": kname, "flops_per_launch": flops,
                "hbm_GBs_algorithmic": N * BYTES_STEP_FP32 / (step_ms * 1e-3) / 1e9}
    else:
        achieved = flops / (step_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                "traffic_unit": "HBM bytes per launch",
                "kernel": kname, "flops_per_launch": flops,
                "hbm_GBs_algorithmic": N * BYTES_STEP_FP64 / (step_ms * 1e-3) / 1e9}

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle ...")
        cpu = cpu_baseline(w, args.cpu_seconds)
        log(f"oracle: {cpu['value']:.4f} MLUPS on {cpu['cores']} threads ({cpu['sample']})")

    out = {
        "metric": "PonD f+g MLUPS", "value": mlups, "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if prec == pond.PREC_FP32 else "f64", "data": "synthetic",
        "config": {"workload": "mach2_fourier_modes_512x512", "nx": w.nx, "ny": w.ny,
                   "mach": 2.0, "tau": w.tau, "prandtl": w.prandtl, "gamma": w.gamma,
                   "precision": args.precision, "interp_points": args.interp_points,
                   "parallelism": "single_gpu"},
        "tuning": {"kernel": args.kernel, "tile": tun.tile, "lds_nodes": tun.lds_nodes},
        "pc_iterations_mean": kbar,
        "nonconverged_node_steps": st1.nonconverged - st0.nonconverged,
        "kernel_ms": {"step": step_ms, "prepass": pre_ms},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
