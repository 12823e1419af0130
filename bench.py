"""Benchmark of the Klinkenberg lattice Boltzmann hot path on one MI355X.

One "step" is one fused D2Q9 stream + Klinkenberg + velocity + BGK/Guo
collide sweep over the whole lattice (one kernel launch).  The workload is
the two-component heterogeneous medium of Sec. IV.B scaled up: 4096 x 4096
nodes, 64 seeded overlapping discs (radius 40-200 nodes, eps 0.2,
k 1e-4) in a matrix (eps 0.5, k 1e-2), local Kn with base 0.05 in the
matrix, pressure-driven along x (rho_in/rho_out = 1.01), periodic in y.
Inputs are generated and uploaded before the timed region; the timed region
is K sweeps on the lattice's stream, bracketed by HIP events.

Prints ONE JSON line.  Headline value: FP32-storage MLUPS.  Also reported:
FP16- and BF16-storage MLUPS on the same workload, the HBM roofline of the
sweep kernel, the FP64 CPU oracle timed on a bounded sample on the host
(``cpu_baseline``), the cost of the adjoint gradient relative to the
forward sweeps on the fractured-shale medium, and a batched ensemble of
uneven samples stepped together.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS + HBM GB/s (% of peak), FP32 vs FP16-storage; adjoint-grad time/forward"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per node and step (populations read once and written
# once, three FP32 medium fields read): FP32 9*4*2 + 12 = 84, FP16/BF16
# 9*2*2 + 12 = 48.  The density plane of the storage layout (FP32 read +
# write, 8 B) is overhead on top of these and is not counted.
ALG_BYTES = {"f32": 84, "f16": 48, "bf16": 48}
LAYOUT_BYTES = {"f32": 92, "f16": 56, "bf16": 56}


PROFILE = os.path.join(ROOT, "profiles", "sweep_discs4096.md")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(storage, launch_ms, nodes):
    """HBM traffic of one launch of the storage type's pass (the automatic
    pass mode's multi-step pass) from the committed rocprofv3 counter summary (FETCH_SIZE
    and WRITE_SIZE per dispatch, each scaled by what it reads for a plain
    copy of known size), as GB/s over this run's measured launch time.  None
    if the summary is missing, covers another lattice, or was taken on
    kernel sources that have changed since."""
    try:
        text = open(PROFILE).read()
        blob = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
        cur = hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read()
                                      for f in blob["sources"])).hexdigest()[:16]
        if cur != blob["source_hash"] or blob["nodes"] != nodes:
            return None, None
        pd = blob["per_dispatch"][storage]
        byts = (pd["fetch_kib"] * blob["fetch_scale"] + pd["write_kib"] * blob["write_scale"]) * 1024
        return byts / (launch_ms * 1e-3) / 1e9, byts
    except (OSError, KeyError, AttributeError, ValueError):
        return None, None


def measured_valu_issue(storage, launch_ms, nodes):
    """Fraction of the device's vector-ALU issue rate that one launch of
    the storage type's pass uses: its VALU instruction count from the
    committed counter summary (SQ_INSTS_VALU per dispatch) over 256 compute
    units x 2.4 GHz x this run's launch time (a compute unit issues at most
    one wave64 VALU instruction per cycle).  None under the same
    conditions as measured_traffic."""
    try:
        text = open(PROFILE).read()
        blob = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
        cur = hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read()
                                      for f in blob["sources"])).hexdigest()[:16]
        if cur != blob["source_hash"] or blob["nodes"] != nodes:
            return None
        return blob["per_dispatch"][storage]["valu_instr"] / (CUS * CLOCK_HZ * launch_ms * 1e-3)
    except (OSError, KeyError, AttributeError, ValueError):
        return None


CUS, CLOCK_HZ = 256, 2.4e9  # MI355X compute units and peak engine clock

REPS = 5  # timed repetitions of every GPU leg; median, min and max reported
SPINUP_S = 0.25  # untimed steps before the timed repetitions of a sweep leg


def spread(ms_list):
    """Median, min and max of repeated timings (ms)."""
    v = sorted(ms_list)
    return {"median": v[len(v) // 2], "min": v[0], "max": v[-1], "reps": len(v)}


def time_storage(case, storage, steps, warmup, device, single=0):
    """`REPS` timed runs of `steps` steps (the automatic pass mode's
    multi-step passes) on the lattice's stream, HIP events around each, then
    `REPS` runs of whole passes alone for the pass's launch time; with
    `single` > 0 also that many single sweeps (one lbk_step(1) call each)
    for comparison."""
    import torch
    from paper_1411_7051_amd.lattice import Lattice

    lat = Lattice(case.eps, case.k, case.kn0, device=device, storage=storage,
                  **case.params)
    per_launch = lat.steps_per_launch
    lat.step(warmup)
    torch.cuda.synchronize(device)
    # clock spin-up: untimed steps for SPINUP_S seconds, so that the timed
    # repetitions (a few ms each) see the device at the clocks it holds over
    # a long run rather than while it ramps up from idle
    spin, t = 0, time.perf_counter()
    while time.perf_counter() - t < SPINUP_S:
        lat.step(steps)
        torch.cuda.synchronize(device)
        spin += steps
    stream = lat.stream
    times = []
    for _ in range(REPS):
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        lat.step(steps)
        t1.record(stream)
        torch.cuda.synchronize(device)
        times.append(t0.elapsed_time(t1))
    # the pass's own launch time: whole passes only, from a time at a
    # multiple of the lattice's check interval (100 steps), so that no
    # check or remainder pass falls inside
    launch = []
    for _ in range(REPS if per_launch > 1 else 0):
        lat.step((-lat.time) % 100)
        n = per_launch * (99 // per_launch)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        lat.step(n)
        t1.record(stream)
        torch.cuda.synchronize(device)
        launch.append(t0.elapsed_time(t1) / (n // per_launch))
    single_ms = None
    if single > 0:
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(single):
            lat.step(1)
        t1.record(stream)
        torch.cuda.synchronize(device)
        single_ms = t0.elapsed_time(t1) / single
    lat.close()
    del lat
    torch.cuda.empty_cache()
    nodes = case.nodes
    sp = spread(times)
    ms = sp["median"]
    mlups = nodes * steps / (ms * 1e-3) / 1e6
    ms_step = ms / steps
    out = {
        "storage": storage,
        "mlups": mlups,
        "ms_per_step": ms_step,
        "ms_per_step_min": sp["min"] / steps,
        "ms_per_step_max": sp["max"] / steps,
        "reps": REPS,
        "spinup_steps": spin,
        "steps_per_launch": per_launch,
        # a launch (a multi-step pass or a sweep) moves ALG_BYTES per node
        "pass_alg_GBps": nodes * ALG_BYTES[storage] / (per_launch * ms_step * 1e-3) / 1e9,
        "per_step_alg_GBps": mlups * ALG_BYTES[storage] / 1e3,
    }
    if launch:
        ls = spread(launch)
        out["launch_ms"] = ls["median"]
        out["launch_ms_min"] = ls["min"]
        out["launch_ms_max"] = ls["max"]
    if single_ms is not None:
        out["single_sweep_ms"] = single_ms
        out["single_sweep_mlups"] = nodes / (single_ms * 1e-3) / 1e6
        out["single_sweep_alg_GBps"] = nodes * ALG_BYTES[storage] / (single_ms * 1e-3) / 1e9
    return out


def storage_accuracy(case, storages, steps, device):
    """Global permeability after a fixed `steps` (untimed) from the start
    for each storage type on the same lattice, and its error relative to
    FP32."""
    import torch
    from paper_1411_7051_amd.lattice import Lattice

    k = {}
    for st in storages:
        lat = Lattice(case.eps, case.k, case.kn0, device=device, storage=st, **case.params)
        lat.step(steps)
        k[st] = lat.apparent_permeability()
        lat.close()
        del lat
        torch.cuda.empty_cache()
    out = {"steps": steps, "k_app": k}
    if "f32" in k:
        out["rel_vs_f32"] = {st: v / k["f32"] - 1 for st, v in k.items()}
    return out


def copy_bandwidth(device, mib=1024, reps=20):
    """Rate (bytes read + written per second) of a plain streaming kernel on
    the same GPU -- torch's vectorized elementwise ``b = a * 1`` over 1 GiB
    of float32, which moves more than the runtime's device-to-device copy
    on this part -- as context for the roofline fraction."""
    import torch

    n = (mib << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device=device)
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1.0, out=b)
    stream = torch.cuda.current_stream(device)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(reps):
        torch.mul(a, 1.0, out=b)
    t1.record(stream)
    torch.cuda.synchronize(device)
    ms = t0.elapsed_time(t1)
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * 4 * n * reps / (ms * 1e-3) / 1e9


def _host_cpu():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")),
                         "")
    except OSError:
        pass
    return {"host_cpu": model, "host_nproc": os.cpu_count(),
            "host_cpus_visible": len(os.sched_getaffinity(0))}


def _oracle_rate(case, steps=None, target_s=None):
    """Time the serial FP64 oracle on `case` (steady_clock around the step
    loop only): `steps` steps, or as many as fit in about `target_s`."""
    import oracle

    lat = oracle.Lattice(case.eps, case.k, case.kn0, **case.params)
    if steps is None:
        t = time.perf_counter()
        lat.step(2)
        probe = time.perf_counter() - t
        steps = max(2, int(target_s / max(probe / 2, 1e-6)))
    t = time.perf_counter()
    lat.step(steps)
    dt = time.perf_counter() - t
    return lat, steps, dt, case.nodes * steps / dt / 1e6


def _window(case, n, name):
    import numpy as np
    from paper_1411_7051_amd import inputs

    return inputs.Case(np.ascontiguousarray(case.eps[:n, :n]),
                       np.ascontiguousarray(case.k[:n, :n]),
                       np.ascontiguousarray(case.kn0[:n, :n]), case.params, name)


def oracle_legs(n_discs, quick=False):
    """Everything the CPU oracle does for the benchmark, in one process of
    its own (it runs on one host core while the GPU legs run):
    - cpu_baseline: the headline workload's medium, a 384 x 384 window of
      the 4096 x 4096 discs, as many FP64 steps as fit in about 15 s;
    - the other configurations timed as the measurement plan states: the
      64 x 32 channel for 10,000 steps, the 1024 x 512 Klinkenberg channel
      (Kn 0.1) for 2,000 steps, a 1024 x 1024 window of the 8192 x 8192
      shale for 5 steps;
    - the reference global permeability of a 256 x 256 copy of the disc
      medium (radii scaled by 1/16) after 2,000 steps, for the FP32 / FP16 /
      BF16 accuracy legs."""
    from paper_1411_7051_amd import inputs

    oracle_build()
    out = {}
    case = inputs.discs(n=n_discs, seed=2)
    win = _window(case, 384, "discs-window384")
    _, steps, dt, rate = _oracle_rate(win, target_s=15.0)
    out["cpu_baseline"] = {
        "value": rate, "unit": "MLUPS", "cores": 1, "kind": "oracle",
        "sample": f"384x384 window of the same medium, {steps} FP64 steps in {dt:.1f} s",
        **_host_cpu()}
    configs = {}
    plan = [("channel64x32", lambda: inputs.channel(64, 32, eps=0.5, k=1.024, gx=1e-6),
             10000 if not quick else 200),
            ("channel1024x512_kn0.1", lambda: inputs.channel(1024, 512, eps=0.5, k=1.024,
                                                             kn0=0.1, drive="pressure"),
             2000 if not quick else 4),
            ("shale8192_window1024", lambda: _window(inputs.shale(n=8192, seed=3), 1024,
                                                     "shale-window1024"), 5)]
    for name, make, steps in plan:
        c = make()
        _, steps, dt, rate = _oracle_rate(c, steps=steps)
        configs[name] = {"nodes": c.nodes, "steps": steps, "seconds": dt, "mlups": rate}
    out["oracle_configs"] = configs
    small = inputs.discs(n=256, seed=2)
    acc_steps = 2000 if not quick else 20
    lat, _, dt, _ = _oracle_rate(small, steps=acc_steps)
    out["oracle_discs256"] = {"steps": acc_steps, "k_app": lat.apparent_permeability(),
                              "seconds": dt}
    return out


def oracle_build():
    import oracle
    oracle.build(force=False)


def _oracle_child(q, n_discs, quick):
    try:
        q.put(("ok", oracle_legs(n_discs, quick)))
    except Exception as e:  # report, never hang the parent
        q.put(("error", repr(e)))


def time_adjoint(n, steps, ckpt, hist, device):
    """Gradient of the global permeability w.r.t. ln k on the fractured-shale
    medium (n x n, seed 3): time of ``steps`` plain sweeps (t_fwd), of the
    checkpointed forward, and of the backward (recompute + reverse)."""
    import torch
    from paper_1411_7051_amd import inputs
    from paper_1411_7051_amd.lattice import Lattice

    t = time.perf_counter()
    case = inputs.shale(n=n, seed=3)
    log(f"shale inputs: {case.nodes} nodes in {time.perf_counter() - t:.1f} s")
    torch.cuda.reset_peak_memory_stats(device)
    # the forward in two-step passes (the passes the gradient's reverse steps
    # take), timed on 2000 steps and scaled
    lat2 = Lattice(case.eps, case.k, case.kn0, device=device, pass_mode="two_step",
                   **case.params)
    lat2.step(20)
    e2 = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    n2 = min(steps, 2000)
    e2[0].record(lat2.stream)
    lat2.step(n2)
    e2[1].record(lat2.stream)
    torch.cuda.synchronize(device)
    t_fwd2 = e2[0].elapsed_time(e2[1]) * steps / n2
    lat2.close()
    del lat2
    torch.cuda.empty_cache()
    lat = Lattice(case.eps, case.k, case.kn0, device=device, **case.params)
    st = lat.stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    planned = 0
    if hist == "auto":
        hist, planned = lat.adjoint_plan(steps, ckpt, with_bytes=True)
    hist = int(hist)
    ws = torch.empty(max(planned, lat.adjoint_workspace_bytes(steps, ckpt, hist)),
                     dtype=torch.uint8, device=device)
    lat.step(20)
    torch.cuda.synchronize(device)
    ev[0].record(st)
    lat.step(steps)
    ev[1].record(st)
    ev[2].record(st)
    J, ws = lat.adjoint_forward(steps, "k_app", ckpt, hist, ws)
    ev[3].record(st)
    ev[4].record(st)
    g = lat.adjoint_backward(ws)
    ev[5].record(st)
    torch.cuda.synchronize(device)
    t_fwd = ev[0].elapsed_time(ev[1])
    t_af = ev[2].elapsed_time(ev[3])
    t_bwd = ev[4].elapsed_time(ev[5])
    gmax = float(g.abs().max())
    out = {
        "workload": f"shale{n}: {n}x{n} log-normal k (ln-sigma 1.5, corr 32, mean 1e-5), "
                    "eps U[0.05,0.15], 24 fractures (eps 0.9, k 0.1), base Kn 0.5, "
                    "pressure-driven x, periodic y",
        "objective": "global permeability",
        "steps": steps,
        "ckpt_every": ckpt,
        "hist_len": hist,
        "workspace_GB": ws.numel() / 1e9,
        "peak_device_mem_GB": torch.cuda.max_memory_allocated(device) / 1e9,
        "t_fwd_ms": t_fwd,
        "fwd_steps_per_launch": lat.steps_per_launch,
        "t_fwd_ckpt_ms": t_af,
        "t_grad_ms": t_bwd,
        "grad_over_fwd": t_bwd / t_fwd,
        "total_over_fwd": (t_af + t_bwd) / t_fwd,
        # against a forward in two-step passes (the passes the gradient's
        # reverse steps take), from 2000 steps scaled
        "t_fwd_two_step_ms": t_fwd2,
        "grad_over_fwd_two_step": t_bwd / t_fwd2,
        "total_over_fwd_two_step": (t_af + t_bwd) / t_fwd2,
        "J": J,
        "max_abs_grad": gmax,
    }
    lat.close()
    del lat, ws, g
    torch.cuda.empty_cache()
    return out


def time_ensemble(n_samples, steps, storages, graph_steps, device, launch=None, grad_steps=0,
                  grad_ckpt=500, check_every=100):
    """Batched ensemble of uneven samples (seed 4): per-sample lattices
    stepped together by one launch per step, launch shape from the tuner,
    steps replayed from HIP graphs, for each storage type in ``storages``
    (the first is the headline); for the first also the same samples stepped
    one launch per sample per step, and the batched gradient."""
    import numpy as np
    import torch
    from paper_1411_7051_amd import inputs
    from paper_1411_7051_amd.batch import Batch, ensemble_lattices

    t = time.perf_counter()
    cases = inputs.ensemble(n_samples=n_samples, seed=4)
    nodes = sum(c.nodes for c in cases)
    log(f"ensemble inputs: {len(cases)} samples, {nodes} nodes in "
        f"{time.perf_counter() - t:.1f} s")
    runs, kapps, out = {}, {}, None
    for si, storage in enumerate(storages):
        lats = ensemble_lattices(cases, device=device, storage=storage)
        b = Batch(lats)
        st = lats[0].stream
        if launch is None:
            tune_us = b.autotune(reps=5)
            tile_x, rows, grid, _ = b.launch
        else:
            tune_us = None
            tile_x, rows, grid = launch
        b.set_launch(tile_x, rows, grid, graph_steps)
        b.step(2 * graph_steps)  # records the graphs
        torch.cuda.synchronize(device)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        times = []
        for _ in range(REPS):
            # the production setting: a state check (NaN/Inf, FP16 scale)
            # of every sample once per check interval
            ev[0].record(st)
            done = 0
            while done < steps:
                n = min(check_every - (done % check_every), steps - done)
                b.step(n)
                done += n
                if done % check_every == 0:
                    b.check()
            ev[1].record(st)
            torch.cuda.synchronize(device)
            times.append(ev[0].elapsed_time(ev[1]))
        sp = spread(times)
        ms = sp["median"]
        kapps[storage] = b.apparent_permeability()
        mlups = nodes * steps / (ms * 1e-3) / 1e6
        runs[storage] = {
            "launch": {"tile_x": tile_x, "rows": rows, "grid": grid, "graph_steps": graph_steps,
                       "steps_per_launch": b.steps_per_launch},
            "autotune_best_us": tune_us, "ms_per_step": ms / steps,
            "ms_per_step_min": sp["min"] / steps, "ms_per_step_max": sp["max"] / steps,
            "reps": REPS, "check_every": check_every, "mlups": mlups,
            # one-read-one-write bytes per node-step at this rate (what a
            # one-step-per-launch sweep would move), and per launch of the
            # pass in use (a two-step pass moves ALG_BYTES for two steps)
            "alg_GBps": mlups * ALG_BYTES[storage] / 1e3,
            "alg_frac": mlups * ALG_BYTES[storage] / 1e3 / HBM_PEAK_GBS,
            "pass_alg_GBps": mlups * ALG_BYTES[storage] / 1e3 / b.steps_per_launch,
            "pass_alg_frac": mlups * ALG_BYTES[storage] / 1e3 / b.steps_per_launch / HBM_PEAK_GBS}
        if si == 0:
            loop_steps = max(2, steps // 10)
            ev[2].record(st)
            for _ in range(loop_steps):
                for l in lats:
                    l.step(1)
            ev[3].record(st)
            torch.cuda.synchronize(device)
            ms_loop = ev[2].elapsed_time(ev[3]) / loop_steps
            grad = None
            if grad_steps > 0:
                # batched gradient of every sample's global permeability
                ck = min(grad_ckpt, grad_steps)
                hist, ws_bytes = b.adjoint_plan(grad_steps, ck, with_bytes=True)
                ev2 = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
                torch.cuda.synchronize(device)
                ev2[0].record(st)
                b.step(grad_steps)
                ev2[1].record(st)
                ev2[2].record(st)
                J, g = b.gradient(grad_steps, "k_app", ckpt_every=ck, hist_len=hist,
                                  workspace_bytes=ws_bytes)
                ev2[3].record(st)
                torch.cuda.synchronize(device)
                t_fwd = ev2[0].elapsed_time(ev2[1])
                t_all = ev2[2].elapsed_time(ev2[3])
                grad = {"steps": grad_steps, "ckpt_every": ck, "hist_len": hist,
                        "workspace_GB": ws_bytes / 1e9, "t_fwd_ms": t_fwd,
                        "t_fwd_ckpt_plus_grad_ms": t_all, "total_over_fwd": t_all / t_fwd,
                        "max_abs_grad": max(float(x.abs().max()) for x in g)}
                del g
            out = {
                "workload": f"ensemble{n_samples}: square sides U[256,1536], log-normal k "
                            "(ln-sigma 1, corr 8-64, median 1e-3), eps U[0.1,0.6], base Kn "
                            "U[0.01,2], pressure-driven x, periodic y",
                "samples": len(cases), "nodes": nodes, "storage": storage, "steps": steps,
                **runs[storage],
                "per_sample_launch_ms_per_step": ms_loop,
                "batched_speedup": ms_loop / (ms / steps),
                "k_app_range": [float(kapps[storage].min()), float(kapps[storage].max())],
                "gradient": grad,
            }
        b.close()
        for l in lats:
            l.close()
        del b, lats
        torch.cuda.empty_cache()
    out["storage_runs"] = runs
    if "f32" in kapps:
        out["k_app_max_rel_vs_f32"] = {
            s: float(np.max(np.abs(k / kapps["f32"] - 1))) for s, k in kapps.items()}
    return out


ALG_BYTES3 = {"f32": 164, "f16": 88, "bf16": 88}   # 19 populations in + out, 3 fields
LAYOUT_BYTES3 = {"f32": 172, "f16": 96, "bf16": 96}


def time_d3q19(n, steps, warmup, storages, device):
    """D3Q19 sweep on the n^3 sphere medium (the disc medium of Sec. IV.B in
    three dimensions), per storage type."""
    import torch
    from paper_1411_7051_amd import inputs
    from paper_1411_7051_amd.lattice3 import Lattice3

    t = time.perf_counter()
    case = inputs.spheres(n=n, seed=7)
    log(f"spheres{n} inputs: {case.nodes} nodes in {time.perf_counter() - t:.1f} s")
    runs = {}
    for st in storages:
        lat = Lattice3(case.eps, case.k, case.kn0, device=device, storage=st, **case.params)
        lat.step(warmup)
        torch.cuda.synchronize(device)
        times = []
        for _ in range(REPS):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(lat.stream)
            lat.step(steps)
            e1.record(lat.stream)
            torch.cuda.synchronize(device)
            times.append(e0.elapsed_time(e1))
        sp = spread(times)
        ms = sp["median"]
        mlups = case.nodes * steps / (ms * 1e-3) / 1e6
        runs[st] = {"ms_per_step": ms / steps, "ms_per_step_min": sp["min"] / steps,
                    "ms_per_step_max": sp["max"] / steps, "reps": REPS, "mlups": mlups,
                    "alg_GBps": mlups * ALG_BYTES3[st] / 1e3,
                    "alg_frac": mlups * ALG_BYTES3[st] / 1e3 / HBM_PEAK_GBS,
                    "layout_GBps": mlups * LAYOUT_BYTES3[st] / 1e3,
                    "k_app_after": lat.apparent_permeability()}
        lat.close()
        del lat
        torch.cuda.empty_cache()
    return {"workload": f"spheres{n}: {n}^3 two-component medium, 96 seeded spheres "
                        "(r 8-40 scaled, eps 0.2, k 1e-4) in a matrix (eps 0.5, k 1e-2), local "
                        "Kn base 0.05, pressure-driven x (1.01/1.0), periodic y and z, tau 0.8",
            "nodes": case.nodes, "steps": steps, "bytes_per_node": ALG_BYTES3,
            "storage_runs": runs}


def kn_sweep(device, kns=(0.001, 0.01, 0.1, 1.0, 5.0)):
    """Porous-filled plates at 1024 x 512 (eps 0.5, k 1.024, tau 0.8),
    pressure-driven 1.01 / 1.0, local Kn, each base Kn run to steady state:
    k_app / k next to the Brinkman-channel closed form with the Klinkenberg
    factor f_c(Kn) (Sec. IV.A, Eqs. 6-7)."""
    import math

    from paper_1411_7051_amd import inputs
    from paper_1411_7051_amd.lattice import Lattice

    def fc(kn):  # Eqs. 6-7 with b = -1, for the closed-form column only
        if kn <= 0:
            return 1.0
        alpha = 1.358 / (1.0 + 0.170 * kn ** -0.4348)
        return (1.0 + alpha * kn) * (1.0 + 4.0 * kn / (1.0 + kn))

    nx, ny, eps, k = 1024, 512, 0.5, 1.024
    rows = []
    t = time.perf_counter()
    for kn in kns:
        case = inputs.channel(nx, ny, eps=eps, k=k, kn0=kn, drive="pressure")
        lat = Lattice(case.eps, case.k, case.kn0, device=device, **case.params)
        t_run = time.perf_counter()
        steps, res, why = lat.run_to_steady(every=200, tol=1e-9, max_steps=600000)
        t_run = time.perf_counter() - t_run  # host clock: sweeps plus a read-out every 200
        a = math.sqrt(eps / (k * fc(kn)))
        expect = fc(kn) * (1 - math.tanh(a * ny / 2) / (a * ny / 2))
        got = lat.apparent_permeability() / k
        mlups = nx * ny * steps / t_run / 1e6
        rows.append({"kn": kn, "k_app_over_k": got, "closed_form": expect,
                     "rel_diff": got / expect - 1, "steps": steps, "residual": res,
                     "stop": why, "mlups": mlups, "effective_GBps": mlups * ALG_BYTES["f32"] / 1e3})
        lat.close()
    return {"workload": "channel1024x512: eps 0.5, k 1.024, tau 0.8, walls in y, "
                        "pressure 1.01/1.0 in x, local Kn, run to residual < 1e-9 or plateau",
            "seconds": time.perf_counter() - t, "rows": rows,
            "note": "the two 21 MB levels stay in the 256 MB on-package cache, so the "
                    "effective GB/s (84 B per node-step) is not an HBM fraction"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=4096, help="lattice side")
    ap.add_argument("--storages", default="f32,f16,bf16")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--quick-cpu", action="store_true",
                    help="oracle legs on a few steps only (checks the plumbing)")
    ap.add_argument("--single-steps", type=int, default=100,
                    help="single sweeps (one step per launch) timed for comparison (0: skip)")
    ap.add_argument("--accuracy-steps", type=int, default=1000,
                    help="untimed steps before the FP16/BF16 vs FP32 permeability comparison")
    ap.add_argument("--adjoint-n", type=int, default=8192, help="shale lattice side")
    ap.add_argument("--adjoint-steps", type=int, default=20000,
                    help="steps of the gradient (the configuration's 20,000)")
    ap.add_argument("--adjoint-ckpt", type=int, default=500)
    ap.add_argument("--adjoint-hist", default="auto",
                    help="history steps recorded at a time, or 'auto' (longest that fits)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the gradient leg")
    ap.add_argument("--ensemble-samples", type=int, default=192)
    ap.add_argument("--ensemble-steps", type=int, default=400)
    ap.add_argument("--ensemble-storage", default="f16,f32",
                    help="storage types of the ensemble leg (the first is the headline)")
    ap.add_argument("--ensemble-graph", type=int, default=20, help="steps per graph replay")
    ap.add_argument("--ensemble-launch", default=None, metavar="TX,ROWS,GRID",
                    help="fixed batch launch shape instead of the tuner's choice")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the ensemble leg")
    ap.add_argument("--ensemble-grad-steps", type=int, default=1000,
                    help="steps of the batched gradient (0: skip)")
    ap.add_argument("--ensemble-grad-ckpt", type=int, default=500)
    ap.add_argument("--no-kn-sweep", action="store_true",
                    help="skip the Klinkenberg channel sweep")
    ap.add_argument("--d3q19-n", type=int, default=256, help="side of the D3Q19 sphere medium")
    ap.add_argument("--d3q19-steps", type=int, default=300)
    ap.add_argument("--d3q19-storages", default="f32,f16,bf16")
    ap.add_argument("--no-d3q19", action="store_true", help="skip the D3Q19 leg")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="only run 10 device-to-device copies of MIB MiB (a plain copy "
                         "kernel of known traffic, to scale HBM byte counters) and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sweep would shard as x-slabs with halo exchange; not built).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1411_7051_amd import inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.calib_copy:
        n = args.calib_copy << 20
        a = torch.ones(n, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize(dev)
        print(json.dumps({"calib_copy_bytes": n, "copies": 10}), flush=True)
        return

    # the CPU oracle legs run in a process of their own, on one host core,
    # while the GPU legs run
    child, q = None, None
    if not args.no_cpu:
        import multiprocessing as mp
        ctx = mp.get_context("spawn")
        q = ctx.Queue()
        child = ctx.Process(target=_oracle_child, args=(q, args.n, args.quick_cpu), daemon=True)
        child.start()

    t = time.perf_counter()
    case = inputs.discs(n=args.n, seed=2)
    log(f"inputs: {case.nodes} nodes in {time.perf_counter() - t:.1f} s")

    runs = {}
    for st in args.storages.split(","):
        r = time_storage(case, st, args.steps, args.warmup, dev, single=args.single_steps)
        log(f"{st}: {r['mlups']:.0f} MLUPS (median of {REPS}), {r['ms_per_step']:.4f} ms/step "
            f"[{r['ms_per_step_min']:.4f}, {r['ms_per_step_max']:.4f}]; single sweeps "
            f"{r.get('single_sweep_ms', float('nan')):.4f} ms")
        runs[st] = r
    acc = storage_accuracy(case, args.storages.split(","), args.accuracy_steps, dev)
    small = inputs.discs(n=256, seed=2)
    acc_small = storage_accuracy(small, args.storages.split(","), 2000, dev)
    head = runs.get("f32") or next(iter(runs.values()))
    st = head["storage"]
    # dominant kernel: the multi-step pass (one launch per three or two
    # steps) where the library's automatic pass mode takes it, else one
    # sweep a step; its launch time from whole passes alone
    per_launch = head["steps_per_launch"]
    launch_ms = head.get("launch_ms", per_launch * head["ms_per_step"])
    achieved = case.nodes * ALG_BYTES[st] / (launch_ms * 1e-3) / 1e9
    traffic, traffic_bytes = measured_traffic(st, launch_ms, case.nodes)
    roof = {
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic,
        "traffic_bytes_per_launch": traffic_bytes,
        "kernel": {3: f"sweep3x_kernel<{st}> (three steps per launch",
                   2: f"sweep2_kernel<{st}> (two steps per launch"}.get(
                       per_launch, f"sweep_kernel<{st}> (one step per launch") +
                  "; pressure x, periodic y)",
        "bytes_per_node_per_launch": ALG_BYTES[st],
        "steps_per_launch": per_launch,
        "launch_ms": launch_ms,
        "layout_bytes_per_node_per_launch": LAYOUT_BYTES[st],
        # the HBM rate a one-step-per-launch sweep would need for this
        # pass's rate
        "single_step_equivalent_GBps": per_launch * achieved,
        "single_step_equivalent_frac": per_launch * achieved / HBM_PEAK_GBS,
        # the roof that binds the multi-step pass: vector-ALU issue (counter
        # summary's instruction count over this run's launch time)
        "valu_issue_frac": measured_valu_issue(st, launch_ms, case.nodes),
        "copy_GBps": copy_bandwidth(dev),
    }
    log(f"plain streaming kernel (b = a * 1, 1 GiB f32): {roof['copy_GBps']:.0f} GB/s "
        "(read + write)")
    adj = None
    if not args.no_adjoint:
        adj = time_adjoint(args.adjoint_n, args.adjoint_steps, args.adjoint_ckpt,
                           args.adjoint_hist, dev)
        log(f"adjoint: t_grad/t_fwd = {adj['grad_over_fwd']:.2f}, "
            f"(t_fwd + t_grad)/t_fwd = {adj['total_over_fwd']:.2f} "
            f"({adj['fwd_steps_per_launch']} steps per forward launch); against two-step "
            f"forward passes {adj['grad_over_fwd_two_step']:.2f} and "
            f"{adj['total_over_fwd_two_step']:.2f}")
    ens = None
    if not args.no_ensemble:
        fixed = (tuple(int(v) for v in args.ensemble_launch.split(","))
                 if args.ensemble_launch else None)
        ens = time_ensemble(args.ensemble_samples, args.ensemble_steps,
                            args.ensemble_storage.split(","),
                            args.ensemble_graph, dev, fixed, args.ensemble_grad_steps,
                            args.ensemble_grad_ckpt)
        log(f"ensemble: {ens['mlups']:.0f} MLUPS ({ens['storage']}, launch {ens['launch']}), "
            f"{ens['batched_speedup']:.2f}x over one launch per sample")
        for sname, r in ens["storage_runs"].items():
            log(f"  ensemble {sname}: {r['mlups']:.0f} MLUPS, {r['ms_per_step']:.3f} ms/step, "
                f"k_app vs f32 {ens.get('k_app_max_rel_vs_f32', {}).get(sname, float('nan')):.2e}")
        if ens["gradient"]:
            log(f"ensemble gradient: (t_fwd + t_grad)/t_fwd = "
                f"{ens['gradient']['total_over_fwd']:.2f} (history {ens['gradient']['hist_len']})")
    d3 = None
    if not args.no_d3q19:
        d3 = time_d3q19(args.d3q19_n, args.d3q19_steps, 20, args.d3q19_storages.split(","), dev)
        for sname, r in d3["storage_runs"].items():
            log(f"d3q19 {sname}: {r['mlups']:.0f} MLUPS, {r['ms_per_step']:.4f} ms/step, "
                f"{r['alg_GBps']:.0f} GB/s algorithmic")
    kn = None
    if not args.no_kn_sweep:
        kn = kn_sweep(dev)
        log("Klinkenberg channel: " + ", ".join(
            f"Kn {r['kn']}: {r['k_app_over_k']:.4f} ({r['rel_diff']:+.2%})" for r in kn["rows"]))
        log("Klinkenberg channel runs: " + ", ".join(
            f"{r['steps']} steps at {r['mlups']:.0f} MLUPS" for r in kn["rows"]))
    cpu, oracle_out = None, None
    if child is not None:
        import queue as _queue
        try:
            status, res = q.get(timeout=900)
        except _queue.Empty:
            status, res = "error", "oracle legs did not finish in 900 s"
        child.join(timeout=30)
        if status == "ok":
            oracle_out = res
            cpu = res["cpu_baseline"]
            log(f"cpu oracle: {cpu['value']:.2f} MLUPS ({cpu['sample']}); " + ", ".join(
                f"{k}: {v['mlups']:.2f} MLUPS ({v['steps']} steps)"
                for k, v in res["oracle_configs"].items()))
        else:
            log(f"cpu oracle legs failed: {res}")
    accuracy = {"discs4096_vs_f32": acc, "discs256_vs_oracle": None}
    if oracle_out is not None:
        ko = oracle_out["oracle_discs256"]["k_app"]
        accuracy["discs256_vs_oracle"] = {
            "steps": 2000, "oracle_k_app": ko, "k_app": acc_small["k_app"],
            "rel_vs_oracle": {s_: v / ko - 1 for s_, v in acc_small["k_app"].items()}}
        log("k_app on the 256^2 discs after 2000 steps vs the FP64 oracle: " + ", ".join(
            f"{s_} {v:+.2e}" for s_, v in accuracy["discs256_vs_oracle"]["rel_vs_oracle"].items()))
    log(f"k_app on the 4096^2 discs after {acc['steps']} steps vs FP32: " + ", ".join(
        f"{s_} {v:+.2e}" for s_, v in acc.get("rel_vs_f32", {}).items()))
    out = {
        "metric": METRIC,
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f16": "f16-storage/f32-math",
                  "bf16": "bf16-storage/f32-math"}[st],
        "data": "synthetic",
        "config": {
            "workload": f"discs{args.n}: {args.n}x{args.n} two-component medium, 64 seeded "
                        "discs (r 40-200, eps 0.2, k 1e-4) in a matrix (eps 0.5, k 1e-2), "
                        "local Kn base 0.05, pressure-driven x (1.01/1.0), periodic y, tau 0.8",
            "nodes": case.nodes,
            "storage": st,
            "parallelism": "single GPU",
        },
        "roofline": roof,
        "cpu_baseline": cpu,
        "storage_runs": runs,
        "storage_accuracy": accuracy,
        "oracle_configs": oracle_out["oracle_configs"] if oracle_out else None,
        "adjoint": adj,
        "ensemble": ens,
        "klinkenberg_channel": kn,
        "d3q19": d3,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
