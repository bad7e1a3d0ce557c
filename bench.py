#!/usr/bin/env python3
"""Benchmark of the PonD f+g step (DDF-BGK, total-energy split, D2Q16) on one MI355X.

Headline workload (the default): the 2048 x 2048 periodic four-quadrant 2-D
Riemann problem (seeded quadrant states: rho in [0.5, 2], p in [0.3, 1.5],
Mach up to 1.5, lattice T = 0.04 p / rho), gamma = 1.4, Pr = 0.71, nu = 2e-3;
FP32 populations and interpolation with FP64 conserved moments, temperature
recovery and frame iteration.  A step is one pass of the whole hot path over
the grid (one step-kernel launch: staging, gather, predictor-corrector,
re-projection, collision, store of the new state and of its moments).  Inputs
are resident in HBM before the timed region; W untimed warm-up steps, then
exactly K timed steps bracketed by device synchronisations, timed with HIP
events on the context's stream.  Nothing else runs inside the timed region.

After the timed region (all untimed):
  * kernel durations: the state saved (on the device) before the timed region
    is restored and the same K steps run again with per-launch HIP events
    (pond_profile_*); the replay produces the same iterations, bit for bit;
  * the roofline of the step kernel: canonical flops per node-update
    FP32 2750 + 13730 K, FP64 150 K + 30 (K = mean predictor-corrector gathers
    per node), against the published MI355X peaks; HBM traffic from the
    committed rocprofv3 counter record of the same kernel sources, if any;
  * the FP32 result's error: the same W + K steps in FP64 (the path that
    matches the CPU oracle to 1e-12), relative L1 and L-infinity of rho, u, T;
  * the 512^2 Mach-2 Fourier-mode workload (same K, W) as a second line of
    figures, a batched subset (instances through pond_batch against each
    alone) and a served subset (a Poisson request stream through pond_server
    against serial FIFO through the plain path, with p50 / p99 latency);
  * the CPU oracle on a bounded sample of the headline workload.

Other workloads (``--workload``): ``modes512`` (512^2 Mach-2 modes),
``sod400`` (the 400 x 1 shock tube), ``batch`` (256 mixed instances) and
``serve`` (the full request stream); these print their own line.

Prints ONE JSON line on stdout (everything else goes to stderr).
"""
import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PonD f+g MLUPS & roofline %, batched/served vs plain; p50/p99 solve latency"

# Published MI355X peaks (dense, no sparsity).
PEAK_FP32_TFLOPS = 157.3        # vector FP32 with packed (dual) FMA
PEAK_FP32_NONPACKED_TFLOPS = 78.6
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# Canonical algorithmic cost of a node-update of the D2Q16 step (the cost model
# the roofline is quoted on): per predictor-corrector gather 13730 FP32 flops
# (interpolation of 20 moments over 16 taps for 16 velocities 10240, the
# moment-to-Grad transformation 2720, the reconstruction 640, departure points
# and weights 130), once per node 2750 (source moments, re-projection,
# collision, store); FP64: 150 per gather (conserved sums, frame) + 30.
CANON_F32_PER_ITER = 13730
CANON_F32_PER_NODE = 2750
CANON_F64_PER_ITER = 150
CANON_F64_PER_NODE = 30
# Canonical HBM bytes of a node-update: the state (32 FP32 populations + the
# FP64 frame) read once and written once.
CANON_BYTES_FP32 = 2 * (128 + 24)
CANON_BYTES_FP64 = 2 * (256 + 24)


# This build's own count of the flops its step kernel performs per
# node-update, in interpolate-then-transform form:
#   per predictor-corrector iteration: departure points and weights 112,
#   interpolation 16 velocities x NP^2 taps x (1 weight product + 20 moments x
#   FMA) = 10496 for the cubic stencil (NP = 4), 5904 for the quadratic one,
#   frame transformation 16 velocities x 2 distributions x 65 = 2080;
#   once per node: moments of the gathered populations 784, re-projection 110,
#   collision 60, reconstruction 640, and the moments of the stored populations
#   for the next step 784 (the step kernel writes them; no separate pre-pass).
# D2Q25 (Grad order 4, 15 moments per distribution), same accounting: per
# iteration departure points 175, interpolation 25 x NP^2 x (1 + 15 x 4),
# transformation 25 x 2 x 85 (30 FMAs and the shared order-4 shift/scale);
# once per node 1850 + 250 + 80 + 1500 + 1850.
def flops_per_iter(np_, q=16, shared_rows=None):
    """Per predictor-corrector gather.  shared_rows: the FP32 D2Q16 kernel's
    mean rows per x-pass (the union of the four row stencils of an
    x-component, see shared_rows_mean); per x-component it interpolates that
    many rows along x (NP taps x 20 moments, FMA), and each velocity takes its
    NP rows through its coefficients (20 FMA + 1 per row); per velocity the
    coefficients (45); once, the reference moments' share of the sums (30).
    D2Q25 (q = 25): the per-velocity count (30 moments at NP^2 taps for each
    of the 25 velocities), the D2Q25 form of the canonical count; its FP32
    kernel shares the x-pass, which this count takes as speed."""
    if q == 25:
        return 175 + 25 * np_ * np_ * 61 + 4250
    if shared_rows is not None:
        return 112 + 4 * (shared_rows * np_ * 20 * 2) + 16 * np_ * 21 * 2 + 16 * 45 + 30
    return 112 + 16 * np_ * np_ * 41 + 2080


def shared_rows_mean(w, np_=4):
    """Mean rows per x-pass of the shared gather over the workload's initial
    frames: the union of the row stencils of the four y-departures
    y - u_y - sqrt(T) c_b (cubic: floor - 1 .. floor + 2), or the four separate
    stencils (4 NP rows) where the union is longer."""
    c_out = 2.3344142183389773
    yy = np.arange(w.ny, dtype=np.float64)[:, None] - w.uy
    s = np.sqrt(w.T)
    if np_ == 4:
        span = np.floor(yy + s * c_out) - np.floor(yy - s * c_out) + 4
    else:
        span = np.floor(yy + s * c_out + 0.5) - np.floor(yy - s * c_out + 0.5) + 3
    return float(np.mean(np.minimum(span, 4 * np_)))


def flops_per_node(q=16):
    return 1850 + 250 + 80 + 1500 + 1850 if q == 25 else 784 + 110 + 60 + 640 + 784


# internal-energy split, once per node: velocity gradient and d_t u 10, and per
# velocity the pre-collision population (10 FMA) and the source term 17
FLOPS_SOURCE_PER_NODE = 10 + 16 * (20 + 17)
# The step kernel's own HBM bytes per node (FP32 mode): frame read 24, moment
# planes read 80, populations + frame written 128 + 24, the new moment planes
# written 80.
BYTES_STEP_FP32 = 24 + 80 + 152 + 80
BYTES_STEP_FP64 = 24 + 160 + 280 + 160
TILE_DIMS = {0: "16,16", 1: "32,8", 2: "16,8", 3: "8,8", 4: "256,1", 5: "64,1", 6: "32,16"}


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


def traffic_record(kernel, precision, workload):
    """HBM bytes per launch of ``kernel`` on ``workload`` from a
    'traffic-record:' line of a profiles/*.md summary (FETCH_SIZE and
    WRITE_SIZE per dispatch, each scaled by the same counter's reading for a
    plain copy of known size), or None when no record matches the workload and
    the current kernel sources."""
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
                        and kv.get("workload") == workload and kv.get("sources_sha256") == want):
                    return float(kv["bytes_per_launch"])
    return None


def host_description():
    """CPU model (as lscpu reports it, from /proc/cpuinfo), logical CPUs of the
    host and CPUs this process may run on."""
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc_host": os.cpu_count(), "nproc_usable": usable}


def cpu_baseline(w, seconds, split=0, lattice=16, threads=0):
    """The FP64 oracle, unmodified, timed on this host's cores: whole-grid steps
    of the same workload from its initial state, as many as fit in
    ~``seconds`` (at least one); if one whole-grid step would take much
    longer, one step at a random sample of nodes instead."""
    import oracle
    if threads > 0:
        oracle.set_num_threads(threads)
    P = oracle.params(w.nx, w.ny, tau=w.tau, gamma=w.gamma, prandtl=w.prandtl, bc_x=w.bc_x,
                      bc_y=w.bc_y, split=split, lattice=lattice)
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
            "kind": "oracle", "sample": sample, **host_description()}


def cpu_subset(ws, seconds, threads=0):
    """The oracle on a representative subset of a set of instances: 8 of them
    spanning the size range (every size-sorted eighth), each timed for about
    seconds / 8 (cpu_baseline); every instance of the set is then projected at
    the rate of the sampled instance nearest to it in node count, giving the
    projected serial oracle time of the whole set."""
    order = sorted(range(len(ws)), key=lambda i: ws[i].nodes)
    pick = sorted({order[min(len(order) - 1, (2 * k + 1) * len(order) // 16)] for k in range(8)})
    rates = []
    for i in pick:
        r = cpu_baseline(ws[i], seconds / len(pick), threads=threads)
        rates.append((ws[i].nodes, r["value"], r["sample"]))
        log(f"oracle subset: {ws[i].nx}x{ws[i].ny}: {r['value']:.4f} MLUPS")
    total_s = 0.0
    for w in ws:
        rate = min(rates, key=lambda t: abs(math.log(t[0]) - math.log(w.nodes)))[1]
        total_s += w.nodes * w.steps / (rate * 1e6)
    updates = sum(w.nodes * w.steps for w in ws)
    return {"kind": "oracle", "unit": "MLUPS", "subset": [
                {"nodes": n, "MLUPS": v, "sample": smp} for n, v, smp in rates],
            "projected_serial_s": total_s, "projected_MLUPS": updates / total_s / 1e6,
            "how": "each instance at the rate of the sampled instance nearest in node count",
            **host_description()}


def _ctx_for(pond, w, prec, stream=None):
    p = pond.pond_params_default(nx=w.nx, ny=w.ny, tau=w.tau, gamma=w.gamma, prandtl=w.prandtl,
                                 bc_x=w.bc_x, bc_y=w.bc_y, precision=prec)
    c = pond.pond_create(p, stream)
    pond.pond_init_fields(c, *[np.ascontiguousarray(a.ravel()) for a in (w.rho, w.ux, w.uy, w.T)])
    return c


def bench_batch(args, pond, workloads):
    """Mixed batch: half quasi-1-D shock tubes (256..8192 nodes), half 2-D
    perturbed flows (64^2..1024^2), Mach 0.5..3, 200..2000 steps each.  Timed:
    every instance to its own step count through batches (one batch per
    phase; a phase runs until the next instance finishes, then the finished
    ones leave).  Plain: each instance alone with pond_step, timed over its
    first min(steps, 200) steps and scaled to its step count."""
    import torch
    prec = pond.PREC_FP32 if args.precision == "fp32" else pond.PREC_FP64
    max_size = args.max_size or 1024
    max_steps = args.max_steps or 2000
    ws = workloads.batch_instances(seed=0, count=args.instances, flow_range=(64, max_size),
                                   steps_range=(min(200, max_steps), max_steps))
    updates = sum(w.nodes * w.steps for w in ws)
    log(f"batch: {len(ws)} instances, {sum(w.nodes for w in ws)} nodes, {updates:.3e} node-updates")
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    # autotune one instance of every size class (untimed)
    t0 = time.perf_counter()
    pond.pond_tuning_cache_clear()
    seen = {}
    for w in ([] if args.no_autotune else ws):
        key = (w.ny == 1, round(math.log2(w.nx)), round(math.log2(max(w.ny, 1))))
        if key in seen:
            continue
        c = _ctx_for(pond, w, prec, sp)
        t = pond.pond_autotune(c, 3)
        seen[key] = (t.tile, t.batch_tile_width)
        pond.pond_destroy(c)
    log(f"autotuned {len(seen)} size classes in {time.perf_counter() - t0:.1f} s: "
        + ", ".join(f"{k}: tile {v[0]} width {v[1]}" for k, v in sorted(seen.items())))

    # plain path
    plain_s = 0.0
    for i, w in enumerate(ws):
        c = _ctx_for(pond, w, prec, sp)
        k = min(w.steps, 200)
        pond.pond_step(c, 2)
        pond.pond_synchronize(c)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        pond.pond_step(c, k)
        e1.record(stream)
        e1.synchronize()
        plain_s += e0.elapsed_time(e1) * 1e-3 * w.steps / k
        pond.pond_destroy(c)
        if i % 32 == 31:
            log(f"plain: {i + 1} instances timed")
    plain = updates / plain_s / 1e6

    # batched
    ctxs = [_ctx_for(pond, w, prec, sp) for w in ws]
    remaining = [w.steps for w in ws]
    active = list(range(len(ws)))
    torch.cuda.synchronize()
    phases = 0
    tiles = []
    t0 = time.perf_counter()
    while active:
        b = pond.pond_batch_create([ctxs[i] for i in active], sp)
        tiles.append(pond.pond_batch_get_info(b).tiles)
        k = min(remaining[i] for i in active)
        pond.pond_batch_step(b, k)
        pond.pond_batch_synchronize(b)
        pond.pond_batch_destroy(b)
        for i in active:
            remaining[i] -= k
        active = [i for i in active if remaining[i] > 0]
        phases += 1
        if phases % 32 == 0:
            log(f"batched: {phases} phases, {len(active)} instances left")
    wall = time.perf_counter() - t0
    nonconv = sum(pond.pond_stats(c).nonconverged for c in ctxs)
    iters = sum(pond.pond_stats(c).pc_iterations for c in ctxs)
    for c in ctxs:
        pond.pond_destroy(c)
    batched = updates / wall / 1e6
    log(f"batched {batched:.1f} MLUPS in {wall:.2f} s over {phases} phases; plain {plain:.1f} MLUPS")
    return {
        "metric": "PonD f+g MLUPS (batched)", "value": batched, "unit": "MLUPS", "n_gpus": 1,
        "steps": None, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if prec == pond.PREC_FP32 else "f64", "data": "synthetic",
        "config": {"workload": f"mixed_batch_{len(ws)}", "instances": len(ws),
                   "tubes": "nx 256..8192 x 1, clamp x", "flows": f"64^2..{max_size}^2 periodic",
                   "mach": "0.5..3", "steps": f"{min(200, max_steps)}..{max_steps}",
                   "precision": args.precision, "parallelism": "single_gpu"},
        "node_updates": updates, "wall_s": wall, "phases": phases,
        "tiles_first_phase": tiles[0], "pc_iterations_mean": iters / updates,
        "autotuned": {f"{'tube' if k[0] else 'flow'} 2^{k[1]} x 2^{k[2]}": {"tile": v[0], "batch_width": v[1]}
                      for k, v in sorted(seen.items())},
        "nonconverged_node_steps": nonconv,
        "plain": {"value": plain, "unit": "MLUPS",
                  "how": "each instance alone (pond_step), min(steps, 200) steps timed with "
                         "HIP events, scaled to its step count"},
        "speedup_vs_plain": batched / plain,
        **({"cpu_subset": cpu_subset(ws, args.cpu_seconds, args.cpu_threads)}
           if args.cpu_subset else {}),
    }


def bench_serve(args, pond, workloads):
    """Serving: requests of three kinds (shock tube on an N x N grid, shear
    flow, 2-D Riemann), N log-uniform in [64, max_size], steps log-uniform in
    [100, max_steps].  First every request runs alone (plain path, FIFO) to
    measure its service time; the plain capacity is requests / total service
    time.  Then the same requests arrive as a Poisson stream at ``load`` times
    that capacity and go through the continuous-batching server (HBM budget
    ``budget_gib``); the serial FIFO latencies for the same arrival times
    follow from the measured service times."""
    import torch
    max_size = args.max_size or 1024
    max_steps = args.max_steps or 2000
    reqs = workloads.serving_requests(seed=0, count=args.instances, size_range=(64, max_size),
                                      steps_range=(100, max_steps))
    ws = [w for _, w in reqs]
    updates = sum(w.nodes * w.steps for w in ws)
    log(f"serve: {len(ws)} requests, {updates:.3e} node-updates")
    stream = torch.cuda.Stream()
    sp = stream.cuda_stream
    service, plain_failed = [], 0
    for i, w in enumerate(ws):
        t0 = time.perf_counter()
        c = _ctx_for(pond, w, pond.PREC_FP32, sp)
        pond.pond_step(c, w.steps)
        try:
            pond.pond_moments(c, np.zeros(w.nodes))
        except pond.PondError as e:
            if e.status != pond.ERR_NONPHYSICAL:
                raise
            plain_failed += 1
            log(f"request {i} ({w.name} {w.nx}x{w.ny}) went non-physical")
        pond.pond_destroy(c)
        service.append(time.perf_counter() - t0)
        if i % 32 == 31:
            log(f"plain: {i + 1} requests served")
    total = sum(service)
    capacity = len(ws) / total
    rng = np.random.default_rng(1)
    if args.load > 0:
        arrivals = np.cumsum(rng.exponential(1.0 / (args.load * capacity), size=len(ws)))
    else:
        # saturated: every request is queued at t = 0
        arrivals = np.zeros(len(ws))
    end, serial_lat = 0.0, []
    for a, s_ in zip(arrivals, service):
        end = max(end, a) + s_
        serial_lat.append(end - a)

    cfg = pond.pond_server_config_default(hbm_budget_bytes=int(args.budget_gib * (1 << 30)))
    if args.fill_nodes is not None:
        cfg.fill_nodes = args.fill_nodes
    srv = pond.pond_server_create(cfg)
    ids = []
    t0 = time.perf_counter()
    for i, (a, w) in enumerate(zip(arrivals, ws)):
        delay = a - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        p = pond.pond_params_default(nx=w.nx, ny=w.ny, tau=w.tau, gamma=w.gamma,
                                     prandtl=w.prandtl, bc_x=w.bc_x, bc_y=w.bc_y)
        ids.append(pond.pond_server_submit(srv, p, w.rho, w.ux, w.uy, w.T, w.steps))
        if i % 32 == 31:
            log(f"served: {i + 1} requests submitted")
    pond.pond_server_wait(srv, 0)
    wall = time.perf_counter() - t0
    infos = [pond.pond_server_poll(srv, i) for i in ids]
    st = pond.pond_server_get_stats(srv)
    pond.pond_server_destroy(srv)
    failed = sum(inf.state != pond.REQ_DONE for inf in infos)
    if args.dump:
        with open(args.dump, "w") as fh:
            json.dump([{"i": i, "kind": w.name, "nx": w.nx, "ny": w.ny, "steps": w.steps,
                        "arrival": float(a), "service_plain": s_, "serial_latency": sl_,
                        "t_submit": inf.t_submit, "t_admit": inf.t_admit, "t_done": inf.t_done,
                        "state": inf.state}
                       for i, (w, a, s_, sl_, inf) in enumerate(zip(ws, arrivals, service,
                                                                   serial_lat, infos))], fh)
    lat = np.array([inf.t_done - inf.t_submit for inf in infos])
    first = min(inf.t_submit for inf in infos)
    last = max(inf.t_done for inf in infos)
    served = updates / (last - first) / 1e6
    plain = updates / total / 1e6
    sl = np.array(serial_lat)
    log(f"served {served:.1f} MLUPS, p50 {np.percentile(lat, 50):.3f} s, p99 "
        f"{np.percentile(lat, 99):.3f} s; serial FIFO p50 {np.percentile(sl, 50):.3f} s, p99 "
        f"{np.percentile(sl, 99):.3f} s; plain {plain:.1f} MLUPS")
    return {
        "metric": "PonD f+g MLUPS (served)", "value": served, "unit": "MLUPS", "n_gpus": 1,
        "steps": None, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"poisson_requests_{len(ws)}", "requests": len(ws),
                   "sizes": f"N x N, N log-uniform 64..{max_size}",
                   "steps": f"log-uniform 100..{max_steps}", "load": args.load,
                   "hbm_budget_gib": args.budget_gib, "chunk_steps": cfg.chunk_steps,
                   "fill_nodes": cfg.fill_nodes,
                   "parallelism": "single_gpu"},
        "node_updates": updates, "failed": failed, "failed_plain": plain_failed, "wall_s": wall,
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "mean": float(lat.mean())},
        "serial_fifo": {"plain_MLUPS": plain, "capacity_req_per_s": capacity,
                        "latency_s": {"p50": float(np.percentile(sl, 50)),
                                      "p99": float(np.percentile(sl, 99)),
                                      "mean": float(sl.mean())}},
        "server_stats": {k: getattr(st, k) for k, _ in st._fields_},
        **({"cpu_subset": cpu_subset(ws, args.cpu_seconds, args.cpu_threads)}
           if args.cpu_subset else {}),
    }


def load_workload(name, args, workloads):
    """(workload, config name, extra config keys) of a single-instance workload."""
    if name == "sod400":
        w = workloads.sod_tube(nx=400, nu=2e-3)
        return w, "sod_tube_400x1", {"nu": 2e-3, "T_scale": 0.04}
    if name == "quadrants2048":
        w = workloads.riemann_quadrants(n=2048, seed=0)
        return w, "riemann_quadrants_2048x2048", {"nu": w.meta["nu"], "seed": 0,
                                                  "states_rho_ux_uy_T": w.meta["states"]}
    n = args.size
    w = workloads.fourier_modes(n=n, mach=args.mach, angle_deg=30.0, amplitude=1e-3, seed=0,
                                tau=args.tau, prandtl=0.71, gamma=1.4, steps=2000)
    wname = f"mach{args.mach:g}_fourier_modes_{n}x{n}" + ("" if args.tau == 0.55 else f"_tau{args.tau:g}")
    return w, wname, {"mach": args.mach}


def measure(pond, torch, w, args, prec, split=0, lattice=16, interp_points=4, tuning=None,
            replay=True, autotune=False):
    """Time K steps (after W warm-up steps) of workload w with HIP events on the
    context stream; then, untimed, restore the state saved before the timed
    region and replay the same K steps with per-launch events for the kernel
    durations.  Returns a dict of figures."""
    stream = torch.cuda.Stream()
    sol = pond.Solver.from_workload(w, precision=prec, stream=stream.cuda_stream,
                                    interp_points=interp_points, split=split,
                                    lattice=lattice, pc_tol=args.pc_tol, tuning=tuning)
    autotuned = False
    if autotune:
        # the library's autotuner times its candidate launch configurations on a
        # copy of the initial state (untimed; every configuration gives the same
        # bits) and keeps the fastest
        pond.pond_autotune(sol.ctx, 3)
        autotuned = True
    tun = pond.pond_get_tuning(sol.ctx)
    sol.step(args.warmup)
    sol.synchronize()
    st0 = sol.stats()
    saved = None
    if replay:
        N, Q = w.nodes, lattice
        dev = torch.device("cuda")
        # f, g, frame on the device; u_ref is written through a host pointer
        saved = [torch.empty((Q, N), dtype=torch.float64, device=dev),
                 torch.empty((Q, N), dtype=torch.float64, device=dev),
                 torch.empty((3, N), dtype=torch.float64, device=dev),
                 np.zeros(2)]
        pond.pond_export_state(sol.ctx, *saved)
    # ---- timed region: K steps, nothing else
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
    # ---- end of the timed region
    ms = ev0.elapsed_time(ev1)
    st1 = sol.stats()
    updates = w.nodes * args.steps
    kbar = (st1.pc_iterations - st0.pc_iterations) / updates
    out = {"ms": ms, "wall_s": wall, "mlups": updates / (ms * 1e-3) / 1e6, "kbar": kbar,
           "nonconverged": st1.nonconverged - st0.nonconverged,
           "nonphysical": int(st1.nonphysical), "tuning": tun, "updates": updates,
           "autotuned": autotuned}
    if replay:
        pond.pond_import_state(sol.ctx, *saved)
        del saved
        pond.pond_profile_enable(sol.ctx, True)
        sol.step(args.steps)
        prof = pond.pond_profile_read(sol.ctx)
        pond.pond_profile_enable(sol.ctx, False)
        st2 = sol.stats()
        out["step_kernel_ms"] = prof.step_ms / max(prof.launches, 1)
        out["prepass_ms_once"] = prof.prepass_ms
        out["replay_identical"] = st2.pc_iterations == st1.pc_iterations - st0.pc_iterations
        if not out["replay_identical"]:
            log(f"warning: replay took {st2.pc_iterations} gathers, the timed run "
                f"{st1.pc_iterations - st0.pc_iterations}")
    sol.close()
    torch.cuda.synchronize()
    return out


def roofline(m, N, prec, interp_points, lattice, split, kname, traffic, shared_rows=None):
    """Roofline of the step kernel from the replayed per-launch duration."""
    t = m["step_kernel_ms"] * 1e-3
    k = m["kbar"]
    own = N * (flops_per_iter(interp_points, lattice, shared_rows) * k +
               flops_per_node(lattice) + (FLOPS_SOURCE_PER_NODE if split == 1 else 0))
    if prec == "fp32":
        f32 = N * (CANON_F32_PER_NODE + CANON_F32_PER_ITER * k)
        f64 = N * (CANON_F64_PER_NODE + CANON_F64_PER_ITER * k)
        # FP32-equivalent rate: FP64 flops weighted by the ratio of the peaks
        achieved = (f32 + f64 * PEAK_FP32_TFLOPS / PEAK_FP64_TFLOPS) / t / 1e12
        peak, own_peak, canon_bytes, own_bytes = (PEAK_FP32_TFLOPS, PEAK_FP32_TFLOPS,
                                                  CANON_BYTES_FP32, BYTES_STEP_FP32)
        extra = {"peak_nonpacked": PEAK_FP32_NONPACKED_TFLOPS,
                 "frac_nonpacked": achieved / PEAK_FP32_NONPACKED_TFLOPS}
    else:
        f32, f64 = 0.0, N * (CANON_F32_PER_NODE + CANON_F32_PER_ITER * k +
                             CANON_F64_PER_NODE + CANON_F64_PER_ITER * k)
        achieved = f64 / t / 1e12
        peak, own_peak, canon_bytes, own_bytes = (PEAK_FP64_TFLOPS, PEAK_FP64_TFLOPS,
                                                  CANON_BYTES_FP64, BYTES_STEP_FP64)
        extra = {}
    return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                            "copy-calibrated)",
            "kernel": kname, "kernel_ms": m["step_kernel_ms"],
            "flops": "canonical per node-update: FP32 2750 + 13730 K, FP64 150 K + 30 "
                     "(FP64 weighted by the FP32/FP64 peak ratio)",
            "flops_fp32_per_launch": f32, "flops_fp64_per_launch": f64,
            "hbm_bytes_algorithmic_per_launch": N * canon_bytes,
            "hbm_GBs_algorithmic": N * canon_bytes / t / 1e9,
            "hbm_frac": N * canon_bytes / t / 1e9 / PEAK_HBM_GBS,
            "own_count": {"flops_per_launch": own, "achieved": own / t / 1e12,
                          "shared_rows_mean": shared_rows,
                          "frac": own / t / 1e12 / own_peak,
                          "hbm_bytes_per_launch": N * own_bytes},
            **extra}


def kernel_name(m, prec, interp_points, split, lattice, kernel):
    ptype = "float" if prec == "fp32" else "double"
    lat = f"D2Q{lattice}"
    if kernel == "tiled":
        return f"step_tiled_kernel<{ptype},{interp_points},{split},{lat},{TILE_DIMS[m['tuning'].tile]}>"
    return f"step_kernel<{ptype},{interp_points},{split},{lat}>"


def fp32_error(pond, torch, w, args, split, lattice, interp_points):
    """The W + K steps of w in FP32 and in FP64 (the path that agrees with the CPU
    oracle to 1e-12): relative L1 and L-infinity of rho, u, T (u scaled by
    max(|u|, sqrt(T)) of the FP64 field)."""
    res = {}
    for prec in (pond.PREC_FP32, pond.PREC_FP64):
        with pond.Solver.from_workload(w, precision=prec, interp_points=interp_points,
                                       split=split, lattice=lattice) as s:
            s.step(args.warmup + args.steps)
            res[prec] = s.moments()
    a, b = res[pond.PREC_FP32], res[pond.PREC_FP64]
    uscale = max(float(np.max(np.hypot(b["ux"], b["uy"]))), float(np.sqrt(np.max(b["T"]))))
    out = {}
    for k in ("rho", "ux", "uy", "T"):
        d = np.abs(a[k] - b[k])
        sc = uscale if k in ("ux", "uy") else float(np.max(np.abs(b[k])))
        out[k] = {"L1_rel": float(np.mean(d) / (np.mean(np.abs(b[k])) if k not in ("ux", "uy")
                                                else uscale)),
                  "Linf_rel": float(np.max(d) / sc)}
    return {"steps": args.warmup + args.steps, "vs": "GPU FP64 path (FP64 parity with the "
            "CPU oracle <= 1e-12 is tested)", "fields": out,
            "L1_rel_max": max(v["L1_rel"] for v in out.values()),
            "Linf_rel_max": max(v["Linf_rel"] for v in out.values())}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--interp-points", type=int, default=4, choices=[3, 4])
    ap.add_argument("--pc-tol", type=float, default=0.0,
                    help="predictor-corrector tolerance (0: the library default)")
    ap.add_argument("--size", type=int, default=512,
                    help="modes512 workload: grid edge (other sizes are diagnostics)")
    ap.add_argument("--mach", type=float, default=2.0,
                    help="modes512 workload: Mach number of the background flow")
    ap.add_argument("--tau", type=float, default=0.55,
                    help="modes512 workload: relaxation time")
    ap.add_argument("--split", choices=["total", "internal", "nontrans"], default="total",
                    help="energy split carried by g (single-instance workloads); nontrans "
                         "runs at Pr = 1")
    ap.add_argument("--lattice", type=int, choices=[16, 25], default=16,
                    help="D2Q16 or D2Q25 (single-instance workloads)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the CPU oracle baseline (0: all of the host's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-subset", action="store_true",
                    help="batch / serve: time the oracle on 8 instances spanning the sizes "
                         "and project its serial time for the whole set")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline only: no FP32 error run, no 512^2 line, no batched or "
                         "served subsets")
    ap.add_argument("--kernel", choices=["tiled", "global"], default="tiled")
    ap.add_argument("--tile", type=int, default=None, help="POND_TILE_* id (default: library's)")
    ap.add_argument("--lds-nodes", type=int, default=None)
    ap.add_argument("--workload",
                    choices=["quadrants2048", "modes512", "sod400", "batch", "serve"],
                    default="quadrants2048",
                    help="quadrants2048: the 2048^2 four-quadrant Riemann problem (headline); "
                         "modes512: one 512^2 Mach-2 instance; sod400: the 400x1 shock tube; "
                         "batch: the mixed 256-instance batch; serve: a Poisson request "
                         "stream through the server")
    ap.add_argument("--instances", type=int, default=256, help="batch / serve: instance count")
    ap.add_argument("--max-size", type=int, default=None,
                    help="batch: largest 2-D side (default 1024); serve: largest side (default 1024)")
    ap.add_argument("--max-steps", type=int, default=None,
                    help="batch: most steps (default 2000); serve: most steps (default 2000)")
    ap.add_argument("--budget-gib", type=float, default=2.0, help="serve: HBM admission budget")
    ap.add_argument("--load", type=float, default=0.7,
                    help="serve: arrival rate / plain capacity (<= 0: every request queued at "
                         "t = 0)")
    ap.add_argument("--dump", default=None, help="serve: write per-request records (JSON) here")
    ap.add_argument("--no-autotune", action="store_true",
                    help="default tiles, no autotuning (single instances: the library's "
                         "default launch configuration; batch: default tile widths)")
    ap.add_argument("--fill-nodes", type=int, default=None,
                    help="serve: server fill_nodes (0 = step every admitted request each round)")
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
    if args.workload == "batch":
        print(json.dumps(bench_batch(args, pond, workloads)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(args, pond, workloads)), flush=True)
        return
    prec = pond.PREC_FP32 if args.precision == "fp32" else pond.PREC_FP64
    tuning = {"kernel": pond.KERNEL_TILED if args.kernel == "tiled" else pond.KERNEL_GLOBAL}
    if args.tile is not None:
        tuning["tile"] = args.tile
        tuning["lds_nodes"] = 0  # the tile's default unless given
    if args.lds_nodes is not None:
        tuning["lds_nodes"] = args.lds_nodes
    # the launch configuration is autotuned unless one is given
    autotune = (not args.no_autotune and args.tile is None and args.lds_nodes is None
                and args.kernel == "tiled")
    split = {"total": pond.SPLIT_TOTAL, "internal": pond.SPLIT_INTERNAL,
             "nontrans": pond.SPLIT_NONTRANS}[args.split]

    w, wname, wconf = load_workload(args.workload, args, workloads)
    if split == pond.SPLIT_NONTRANS:
        w.prandtl = 1.0
    log(f"workload {w.name} {w.nx}x{w.ny}, {args.precision}, {args.split} split, "
        f"warmup {args.warmup}, steps {args.steps}")
    m = measure(pond, torch, w, args, prec, split, args.lattice, args.interp_points, tuning,
                autotune=autotune)
    kname = kernel_name(m, args.precision, args.interp_points, split, args.lattice, args.kernel)
    shared = (shared_rows_mean(w, args.interp_points)
              if args.precision == "fp32" and args.lattice == 16 else None)
    roof = roofline(m, w.nodes, args.precision, args.interp_points, args.lattice, split, kname,
                    traffic_record(kname, args.precision, wname), shared)
    log(f"time {m['ms']:.1f} ms (host {m['wall_s'] * 1e3:.1f} ms), {m['mlups']:.1f} MLUPS, "
        f"K {m['kbar']:.3f}, step kernel {m['step_kernel_ms']:.4f} ms per launch (replay), "
        f"roofline {roof['frac']:.3f} of {roof['peak']} TFLOP/s")

    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 x {n * 4} bytes read + written")
        del a, b

    extras = {}
    if not args.no_extras and args.precision == "fp32":
        log("FP32 against FP64 over the same steps ...")
        extras["accuracy_fp32"] = fp32_error(pond, torch, w, args, split, args.lattice,
                                             args.interp_points)
        log(f"  L1 {extras['accuracy_fp32']['L1_rel_max']:.2e}, "
            f"Linf {extras['accuracy_fp32']['Linf_rel_max']:.2e}")
    if not args.no_extras and args.workload == "quadrants2048":
        # the 512^2 Mach-2 modes workload, same K and W
        a2 = argparse.Namespace(**vars(args))
        w2, wname2, _ = load_workload("modes512", a2, workloads)
        m2 = measure(pond, torch, w2, args, prec, split, args.lattice, args.interp_points, tuning,
                     autotune=autotune)
        kname2 = kernel_name(m2, args.precision, args.interp_points, split, args.lattice,
                             args.kernel)
        shared2 = (shared_rows_mean(w2, args.interp_points)
                   if args.precision == "fp32" and args.lattice == 16 else None)
        r2 = roofline(m2, w2.nodes, args.precision, args.interp_points, args.lattice, split,
                      kname2, traffic_record(kname2, args.precision, wname2), shared2)
        extras["mach2_fourier_modes_512x512"] = {
            "value": m2["mlups"], "unit": "MLUPS", "ms_per_step": m2["ms"] / args.steps,
            "pc_iterations_mean": m2["kbar"], "kernel": kname2,
            "kernel_ms": m2["step_kernel_ms"], "roofline_frac": r2["frac"],
            "roofline_achieved_TFLOPs": r2["achieved"], "traffic": r2["traffic"]}
        log(f"512^2 modes: {m2['mlups']:.1f} MLUPS, K {m2['kbar']:.3f}, kernel "
            f"{m2['step_kernel_ms']:.4f} ms, roofline {r2['frac']:.3f}")
        # batched subset
        ab = argparse.Namespace(**vars(args))
        ab.instances, ab.max_size, ab.max_steps, ab.no_autotune = 32, 512, 600, False
        bres = bench_batch(ab, pond, workloads)
        extras["batched"] = {
            "workload": f"mixed batch subset: {bres['config']['instances']} instances "
                        f"(tubes {bres['config']['tubes']}, flows {bres['config']['flows']}, "
                        f"Mach {bres['config']['mach']}, steps {bres['config']['steps']})",
            "value": bres["value"], "unit": "MLUPS", "plain_MLUPS": bres["plain"]["value"],
            "speedup_vs_plain": bres["speedup_vs_plain"], "node_updates": bres["node_updates"],
            "pc_iterations_mean": bres["pc_iterations_mean"]}
        # served subset
        asv = argparse.Namespace(**vars(args))
        asv.instances, asv.max_size, asv.max_steps, asv.dump = 64, 1024, 2000, None
        sres = bench_serve(asv, pond, workloads)
        extras["served"] = {
            "workload": f"Poisson stream subset: {sres['config']['requests']} requests, "
                        f"{sres['config']['sizes']}, steps {sres['config']['steps']}, load "
                        f"{sres['config']['load']} of the plain capacity, HBM budget "
                        f"{sres['config']['hbm_budget_gib']} GiB",
            "value": sres["value"], "unit": "MLUPS",
            "latency_s": sres["latency_s"], "failed": sres["failed"],
            "plain_serial_fifo": {"MLUPS": sres["serial_fifo"]["plain_MLUPS"],
                                  "latency_s": sres["serial_fifo"]["latency_s"]},
            "note": "throughput is capped by the arrival rate (load x the plain capacity); "
                    "served_saturated measures it with the queue full"}
        # the same requests all queued at t = 0: throughput with a full queue
        asv.load = 0.0
        ssat = bench_serve(asv, pond, workloads)
        extras["served_saturated"] = {
            "workload": "the served subset's requests, every one queued at t = 0",
            "value": ssat["value"], "unit": "MLUPS", "latency_s": ssat["latency_s"],
            "failed": ssat["failed"],
            "plain_serial_fifo": {"MLUPS": ssat["serial_fifo"]["plain_MLUPS"],
                                  "latency_s": ssat["serial_fifo"]["latency_s"]},
            "speedup_vs_plain": ssat["value"] / ssat["serial_fifo"]["plain_MLUPS"]}

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle ...")
        cpu = cpu_baseline(w, args.cpu_seconds, split, args.lattice, args.cpu_threads)
        log(f"oracle: {cpu['value']:.4f} MLUPS on {cpu['cores']} threads ({cpu['sample']})")

    out = {
        "metric": METRIC, "value": m["mlups"], "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": m["ms"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if prec == pond.PREC_FP32 else "f64", "data": "synthetic",
        "config": {"workload": wname, "nx": w.nx, "ny": w.ny, **wconf,
                   "tau": w.tau, "prandtl": w.prandtl, "gamma": w.gamma,
                   "precision": args.precision, "interp_points": args.interp_points,
                   "split": args.split, "lattice": args.lattice,
                   "parallelism": "single_gpu"},
        "tuning": {"kernel": args.kernel, "tile": m["tuning"].tile,
                   "tile_dims": TILE_DIMS[m["tuning"].tile],
                   "lds_nodes": m["tuning"].lds_nodes, "autotuned": m["autotuned"],
                   "how": "pond_autotune over the library's candidate tiles and LDS shares "
                          "before the warm-up, untimed" if m["autotuned"] else "library default"},
        "pc_iterations_mean": m["kbar"],
        "nonconverged_node_steps": m["nonconverged"],
        "nonphysical": m["nonphysical"],
        "kernel_ms": {"step": m["step_kernel_ms"], "prepass_once": m["prepass_ms_once"],
                      "how": "same K steps replayed untimed from the saved state, HIP events "
                             "around each launch", "replay_identical": m["replay_identical"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        **extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
