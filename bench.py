"""Benchmark: grid-point updates per second of the acoustic propagator.

Workload (the configuration the headline metric is quoted on): 3D smooth
random velocity model, 512^3 physical nodes + 40-cell absorbing layer on every
side (592^3 = 207,474,688 nodes updated per step), h = 10 m, space order 8,
FP32, dt = 0.5 dt_crit, one trilinear Ricker source (12 Hz), 256 x 256
trilinear receivers.  A step is one pass of the hot path: stencil update with
the fused absorbing layer, source injection and receiver recording.

  value            forward Gpts/s, constant density (nodes x steps / time)
  fwd_adjoint      forward with checkpoints + checkpointed recompute + adjoint
                   with imaging, Gpts/s counted per original step
  vd_staggered     forward Gpts/s, variable density (Gardner density), staggered
  roofline         dominant kernel (constant-density stencil): algorithmic
                   bytes per launch / average launch time from HIP events
  batch            64 shots on uneven grids (160..256 x 160..320 x 160..320 + layer,
                   own layered models, 10-20 Hz), all advanced by one stencil
                   launch per step (autotuned tiles, HIP graph), against a
                   loop of single-shot launches of the same shots on the same GPU
  cpu_baseline     FP64 oracle on the host cores, first few steps of the same
                   workload

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       python bench.py --profile-pass {const,vd,vd_adjoint}   (a short run + a 1 GiB copy, for counters)
       python bench.py --paper-shapes     (whole runs at the paper's Table 2 / 3 shapes)
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_NODE = {"const": 16, "vd_staggered": 20, "vd_centred": 20}
METRIC = "Gpts/s (grid updates/s) fwd and fwd+adjoint, 3D 512^3 SO8 FP32; % HBM peak"


# HBM bytes per launch of the dominant kernel from the counter runs recorded in
# profiles/stencil_const_smooth3d_592_traffic.md (FETCH_SIZE x 2.000 and
# WRITE_SIZE x 1.000, both calibrated on a 1 GiB copy), valid only for the
# kernel configuration that was profiled.
PROFILED = {"tiling": {"tx": 24, "nw": 8, "zc": 74, "nt": 1, "pf": 1, "wt": 0, "ts": 1, "occ": 0, "order": 1},
            "n": 512, "bytes": (1439654.0 * 2.000 + 810448.0 * 1.000) * 1024}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_prop(wl, scheme, nsteps, dt):
    import torch
    from paper_2201_05278_amd import Propagator
    prop = Propagator(wl.n, wl.h, wl.space_order, dt, nsteps, scheme=scheme, nbl=wl.nbl)
    prop.set_sources(wl.src, wl.src_interp)
    prop.set_receivers(wl.rec, wl.rec_interp)
    vel = torch.from_numpy(wl.vel).cuda()
    rho = torch.from_numpy(wl.rho).cuda() if scheme != "const" else None
    prop.prepare(vel, rho, cmax=wl.cmax)
    return prop


def time_forward(prop, wavelet, warmup, steps, with_events=True):
    import torch
    fields = (prop.new_field(), prop.new_field())
    res = prop.forward(wavelet, fields=fields, step0=0, nsteps_run=warmup)
    torch.cuda.synchronize()
    cur = (fields[res.current], fields[1 - res.current])
    ms = np.zeros(steps, dtype=np.float32) if with_events else None
    t0 = time.perf_counter()
    prop.forward(wavelet, fields=cur, step0=warmup, nsteps_run=steps, traces=res.traces,
                 stencil_ms=ms)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, ms


def time_fwd_adjoint(prop, wavelet, every):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fw = prop.forward(wavelet, checkpoint_every=every)
    grads = prop.adjoint(wavelet, fw.traces, fw.ckpt, every)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    del fw, grads
    return el


def batch_leg(nsteps, cache):
    """Batched shots against a loop of single-shot launches (same shots, same GPU)."""
    import torch
    import workloads
    from paper_2201_05278_amd import Propagator, Batch, critical_dt, ricker
    shots = workloads.batch_3d(nshots=64, nsteps=nsteps)
    props, wavs, nodes = [], [], 0.0
    for wl in shots:
        dt = workloads.CFL_FRACTION * critical_dt(wl.h, wl.space_order, wl.cmax)
        p = Propagator(wl.n, wl.h, wl.space_order, dt, nsteps, nbl=wl.nbl)
        p.set_sources(wl.src)
        p.set_receivers(wl.rec)
        p.prepare(torch.from_numpy(wl.vel).cuda(), cmax=wl.cmax)
        props.append(p)
        wavs.append(ricker(wl.f_peak, dt, nsteps).reshape(-1, 1).cuda())
        nodes += float(np.prod([k + 2 * wl.nbl for k in wl.n]))
    batch = Batch(props)
    batch.autotune(wavs, cache)
    tiling = batch.tiling
    # untimed first run: captures and instantiates the graph of the whole loop,
    # so that the timed call only replays it
    batch.forward(wavs, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.forward(wavs, use_graph=True)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    del batch
    torch.cuda.empty_cache()
    for p, w in zip(props[:2], wavs[:2]):
        p.forward(w, nsteps_run=min(10, nsteps))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, w in zip(props, wavs):
        p.forward(w)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    return {"shots": len(props), "steps": nsteps, "nodes_per_step": int(nodes),
            "batched_gpts": round(nodes * nsteps / t_batch / 1e9, 3),
            "single_loop_gpts": round(nodes * nsteps / t_loop / 1e9, 3),
            "speedup": round(t_loop / t_batch, 3), "tiling": tiling}


def profile_pass(args):
    """A short run for hardware counters with the default tiling: 5 forward
    steps of the workload (constant density, or the staggered scheme), or a
    10-step staggered forward + adjoint with checkpoints every 5 steps; then a
    plain 1 GiB device copy of known size."""
    import torch
    import workloads
    from paper_2201_05278_amd import critical_dt, ricker
    kind = args.profile_pass
    wl = workloads.smooth_3d(n=args.n, nsteps=10, scheme="vd_staggered")
    dt = workloads.CFL_FRACTION * critical_dt(wl.h, wl.space_order, wl.cmax)
    wav = ricker(wl.f_peak, dt, 10).reshape(-1, 1).cuda()
    if kind == "vd_adjoint":
        prop = make_prop(wl, "vd_staggered", 10, dt)
        time_fwd_adjoint(prop, wav, 5)
    else:
        prop = make_prop(wl, "const" if kind == "const" else "vd_staggered", 10, dt)
        prop.forward(wav, nsteps_run=5)
    del prop
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"profile pass done: {kind} at {args.n + 80}^3, 1 GiB copy", flush=True)


# The paper's benchmark shapes ("Performance evaluation", Tables 2 and 3) with
# the boundary set-up of its examples, and its times in seconds for the whole
# run (FP64, host-device transfers included) on its fastest GPU back-end per
# order, for context only.
PAPER_TIMES = {
    "paper_shape_2d": [(2, 1331, 0.36), (4, 1537, 0.43), (8, 1696, 0.47)],
    "paper_shape_3d": [(2, 2080, 28.30), (4, 2401, 40.36), (8, 2651, 63.12)],
}


def paper_shapes(dtypes=("float32", "float64")):
    """Whole runs at the paper's grid shapes, boundary conditions and step
    counts (dt at the stability limit, as its counts imply), synthetic layered
    models reaching its c_max, one source and 101 receivers, in single and
    double precision; one JSON line per run."""
    import torch
    import workloads
    from paper_2201_05278_amd import Propagator, critical_dt, steps_for, ricker
    for name, make in (("paper_shape_2d", workloads.paper_shape_2d), ("paper_shape_3d", workloads.paper_shape_3d)):
        for so, nt_paper, paper_s in PAPER_TIMES[name]:
            wl = make(space_order=so)
            cmax = wl.extra["cmax"]
            dt = critical_dt(wl.h, so, cmax)
            nt = steps_for(wl.extra["tf"], dt)
            assert nt == nt_paper, (name, so, nt, nt_paper)
            for dtype in dtypes:
                tdt = torch.float64 if dtype == "float64" else torch.float32
                prop = Propagator(wl.n, wl.h, so, dt, nt, nbl=[list(p) for p in wl.nbl],
                                  bc=[list(b) for b in wl.bc], dtype=dtype)
                prop.set_sources(wl.src, wl.src_interp)
                prop.set_receivers(wl.rec, wl.rec_interp)
                prop.prepare(torch.from_numpy(wl.vel).to(tdt).cuda(), cmax=cmax)
                wav = ricker(wl.f_peak, dt, nt).reshape(-1, 1).to(tdt).cuda()
                if wl.ndim == 3 and dtype == "float32":
                    # the library's own tiling search for this grid (2D runs are bound by
                    # launch latency, which its per-launch timing does not see)
                    prop.autotune()
                fields = (prop.new_field(), prop.new_field())
                traces = torch.zeros((nt, len(wl.rec)), dtype=tdt, device="cuda")
                graph = dtype == "float32"       # the single-precision loop as one HIP graph
                prop.forward(wav, fields=fields, traces=traces, use_graph=graph)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                prop.forward(wav, fields=fields, traces=traces, use_graph=graph)
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                nodes = float(np.prod([k + a + b for k, (a, b) in zip(wl.n, wl.nbl)]))
                print(json.dumps({"shape": name, "dtype": dtype, "nodes": int(nodes), "space_order": so,
                                  "steps": nt, "boundary": wl.bc, "seconds": round(el, 4),
                                  "gpts": round(nodes * nt / el / 1e9, 2), "paper_best_seconds": paper_s,
                                  "paper_best_gpts": round(nodes * nt / paper_s / 1e9, 3),
                                  "tiling": prop.tiling}), flush=True)
                del prop, fields, traces
                torch.cuda.empty_cache()


def cpu_baseline(wl, dt, steps):
    """FP64 oracle, constant density, first `steps` steps of the workload."""
    import oracle
    prob = oracle.Problem(n=wl.n, h=wl.h, space_order=wl.space_order, dt=dt, nsteps=steps,
                          nbl=((wl.nbl, wl.nbl),) * 3)
    st = oracle.prepare(prob, wl.vel.astype(np.float64))
    src = oracle.geometry_table(prob, wl.src, wl.src_interp)
    rec = oracle.geometry_table(prob, wl.rec, wl.rec_interp)
    wav = oracle.ricker(wl.f_peak, dt, steps)[:, None]
    t0 = time.perf_counter()
    oracle.forward(st, wav, src, rec, len(wl.rec), nsteps=steps)
    el = time.perf_counter() - t0
    nodes = float(np.prod(prob.N))
    from oracle import _native
    cores = int(_native.lib().ow_threads())
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": round(nodes * steps / el / 1e9, 4), "unit": "Gpts/s", "cores": cores,
            "kind": "oracle", "cpu_model": model,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS"),
            "omp_proc_bind": os.environ.get("OMP_PROC_BIND"),
            "sample": f"first {steps} steps of the same workload ({int(nodes)} nodes/step), "
                      f"FP64 C/OpenMP oracle ({cores} threads), {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--adj-steps", type=int, default=2000)
    ap.add_argument("--ckpt-every", type=int, default=50)
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-vd", action="store_true")
    ap.add_argument("--skip-batch", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--tune-cache", default=os.path.join("/tmp", "simwave_tune.json"))
    ap.add_argument("--profile-pass", choices=["const", "vd", "vd_adjoint"], default=None,
                    help="a short run for hardware counters (no JSON line)")
    ap.add_argument("--paper-shapes", action="store_true",
                    help="whole runs at the paper's benchmark shapes instead of the headline")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); "
              "multi-GPU sharding is not part of this library", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    from paper_2201_05278_amd import critical_dt, ricker

    torch.cuda.set_device(0)
    if args.profile_pass:
        profile_pass(args)
        return
    if args.paper_shapes:
        paper_shapes()
        return
    K, W = args.steps, args.warmup
    log(f"bench: building the smooth_3d model, n = {args.n}")
    wl = workloads.smooth_3d(n=args.n, nsteps=K + W, scheme="vd_staggered")
    dt = workloads.CFL_FRACTION * critical_dt(wl.h, wl.space_order, wl.cmax)
    nodes = float(np.prod([k + 2 * wl.nbl for k in wl.n]))
    out = {}

    # forward, constant density (headline)
    log("bench: constant-density forward")
    prop = make_prop(wl, "const", K + W, dt)
    wav = ricker(wl.f_peak, dt, K + W).reshape(-1, 1).cuda()
    el, ms = time_forward(prop, wav, W, K)
    gpts = nodes * K / el / 1e9
    avg_ms = float(ms.mean())
    achieved = nodes * BYTES_PER_NODE["const"] / (avg_ms * 1e-3) / 1e9
    out["forward"] = gpts
    out["stencil_ms"] = avg_ms
    tiling = prop.tiling
    traffic = PROFILED["bytes"] if (tiling == PROFILED["tiling"] and args.n == PROFILED["n"]) else None
    log(f"bench: forward {gpts:.1f} Gpts/s, stencil {avg_ms:.3f} ms -> {achieved:.0f} GB/s")
    del prop
    torch.cuda.empty_cache()

    # forward + adjoint with checkpointing, constant density
    log("bench: forward + adjoint")
    KA = args.adj_steps
    propa = make_prop(wl, "const", KA, dt)
    wava = ricker(wl.f_peak, dt, KA).reshape(-1, 1).cuda()
    time_fwd_adjoint(propa, wava, args.ckpt_every)          # warm-up pass
    el_a = time_fwd_adjoint(propa, wava, args.ckpt_every)
    fa = nodes * KA / el_a / 1e9
    log(f"bench: fwd+adjoint {fa:.1f} Gpts/s")
    del propa
    torch.cuda.empty_cache()

    batch = None
    if not args.skip_batch:
        log(f"bench: 64 batched shots, {args.batch_steps} steps")
        batch = batch_leg(args.batch_steps, args.tune_cache)
        log(f"bench: batch {batch}")
        torch.cuda.empty_cache()

    vd = None
    if not args.skip_vd:
        log("bench: variable-density (staggered) forward")
        propv = make_prop(wl, "vd_staggered", K + W, dt)
        el_v, ms_v = time_forward(propv, wav, W, K)
        vd = nodes * K / el_v / 1e9
        out["vd_stencil_ms"] = float(ms_v.mean())
        log(f"bench: vd staggered {vd:.1f} Gpts/s")
        del propv
        torch.cuda.empty_cache()
        # forward + adjoint with velocity and density gradients
        log("bench: variable-density forward + adjoint")
        propva = make_prop(wl, "vd_staggered", KA, dt)
        time_fwd_adjoint(propva, wava, args.ckpt_every)      # warm-up pass
        el_va = time_fwd_adjoint(propva, wava, args.ckpt_every)
        out["vd_fwd_adjoint_gpts"] = round(nodes * KA / el_va / 1e9, 3)
        log(f"bench: vd fwd+adjoint {out['vd_fwd_adjoint_gpts']:.1f} Gpts/s")
        del propva
        torch.cuda.empty_cache()

    cpu = None
    if not args.skip_cpu:
        log(f"bench: CPU oracle, {args.cpu_steps} steps")
        cpu = cpu_baseline(wl, dt, args.cpu_steps)

    line = {
        "metric": METRIC,
        "value": round(gpts, 3),
        "unit": "Gpts/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(el / K * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"smooth_3d constant density, {args.n}^3 physical + 40-cell layer "
                               f"= {args.n + 80}^3 nodes, h=10 m, SO8, dt=0.5 dt_crit, trilinear "
                               f"source + {len(wl.rec)} receivers",
                   "nodes_per_step": int(nodes), "space_order": 8},
        "fwd_adjoint_gpts": round(fa, 3),
        "fwd_adjoint_config": f"{KA} steps, checkpoints every {args.ckpt_every}, Gpts/s per "
                              f"original step (forward + recompute + adjoint with imaging)",
        "vd_staggered_gpts": None if vd is None else round(vd, 3),
        "vd_fwd_adjoint_gpts": out.get("vd_fwd_adjoint_gpts"),
        "pct_hbm_peak_forward": round(100.0 * gpts * BYTES_PER_NODE["const"] / HBM_PEAK_GBS, 2),
        # per original step: forward 16 B, recompute storing M L u 20 B, adjoint with
        # imaging in pairs of steps (16 + 8 + 8 B, then 16 B) 24 B
        "pct_hbm_peak_fwd_adjoint": round(100.0 * fa * 60 / HBM_PEAK_GBS, 2),
        "pct_hbm_peak_vd": None if vd is None else round(100.0 * vd * 20 / HBM_PEAK_GBS, 2),
        "batch": batch,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic / 1e9, 4),
                     "traffic_unit": "GB per launch", "tiling": tiling,
                     "kernel": "constant-density stencil, 16 B/node x nodes per launch",
                     "avg_launch_ms": round(avg_ms, 4)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
