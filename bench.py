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


def measured_traffic(storage, ms_per_step, nodes):
    """HBM traffic of one sweep launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by what it
    reads for a plain copy of known size), as GB/s over this run's measured
    launch time.  None if the summary is missing, covers another lattice, or
    was taken on kernel sources that have changed since."""
    try:
        text = open(PROFILE).read()
        blob = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
        cur = hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read()
                                      for f in blob["sources"])).hexdigest()[:16]
        if cur != blob["source_hash"] or blob["nodes"] != nodes:
            return None, None
        pd = blob["per_dispatch"][storage]
        byts = (pd["fetch_kib"] * blob["fetch_scale"] + pd["write_kib"] * blob["write_scale"]) * 1024
        return byts / (ms_per_step * 1e-3) / 1e9, byts
    except (OSError, KeyError, AttributeError, ValueError):
        return None, None


def time_storage(case, storage, steps, warmup, device):
    import torch
    from paper_1411_7051_amd.lattice import Lattice

    lat = Lattice(case.eps, case.k, case.kn0, device=device, storage=storage,
                  **case.params)
    lat.step(warmup)
    torch.cuda.synchronize(device)
    stream = lat.stream
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    lat.step(steps)
    t1.record(stream)
    torch.cuda.synchronize(device)
    ms = t0.elapsed_time(t1)
    kapp = lat.apparent_permeability()
    lat.close()
    del lat
    torch.cuda.empty_cache()
    nodes = case.nodes
    mlups = nodes * steps / (ms * 1e-3) / 1e6
    ms_step = ms / steps
    return {
        "storage": storage,
        "mlups": mlups,
        "ms_per_step": ms_step,
        "alg_GBps": mlups * ALG_BYTES[storage] / 1e3,
        "layout_GBps": mlups * LAYOUT_BYTES[storage] / 1e3,
        "k_app_after": kapp,
    }


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


def cpu_baseline(case, target_s=15.0):
    """The FP64 oracle, single-threaded, on a 384 x 384 window of the same
    medium (same fields and boundary conditions), as many steps as fit in
    about ``target_s`` seconds."""
    import numpy as np

    import oracle
    from paper_1411_7051_amd import inputs

    oracle.build(force=False)
    n = 384
    sub = inputs.Case(np.ascontiguousarray(case.eps[:n, :n]),
                      np.ascontiguousarray(case.k[:n, :n]),
                      np.ascontiguousarray(case.kn0[:n, :n]), case.params)
    lat = oracle.Lattice(sub.eps, sub.k, sub.kn0, **sub.params)
    t = time.perf_counter()
    lat.step(2)
    probe = time.perf_counter() - t
    steps = max(2, int(target_s / max(probe / 2, 1e-6)))
    t = time.perf_counter()
    lat.step(steps)
    dt = time.perf_counter() - t
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")),
                         "")
    except OSError:
        pass
    return {
        "value": n * n * steps / dt / 1e6,
        "unit": "MLUPS",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{n}x{n} window of the same medium, {steps} FP64 steps in {dt:.1f} s",
        "host_cpu": model,
        "host_cpus_visible": len(os.sched_getaffinity(0)),
    }


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
        "t_fwd_ckpt_ms": t_af,
        "t_grad_ms": t_bwd,
        "grad_over_fwd": t_bwd / t_fwd,
        "total_over_fwd": (t_af + t_bwd) / t_fwd,
        "J": J,
        "max_abs_grad": gmax,
    }
    lat.close()
    del lat, ws, g
    torch.cuda.empty_cache()
    return out


def time_ensemble(n_samples, steps, storages, graph_steps, device, launch=None, grad_steps=0,
                  grad_ckpt=500):
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
        ev[0].record(st)
        b.step(steps)
        ev[1].record(st)
        torch.cuda.synchronize(device)
        ms = ev[0].elapsed_time(ev[1])
        kapps[storage] = b.apparent_permeability()
        mlups = nodes * steps / (ms * 1e-3) / 1e6
        runs[storage] = {
            "launch": {"tile_x": tile_x, "rows": rows, "grid": grid, "graph_steps": graph_steps},
            "autotune_best_us": tune_us, "ms_per_step": ms / steps, "mlups": mlups,
            "alg_GBps": mlups * ALG_BYTES[storage] / 1e3,
            "alg_frac": mlups * ALG_BYTES[storage] / 1e3 / HBM_PEAK_GBS}
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
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(lat.stream)
        lat.step(steps)
        e1.record(lat.stream)
        torch.cuda.synchronize(device)
        ms = e0.elapsed_time(e1)
        mlups = case.nodes * steps / (ms * 1e-3) / 1e6
        runs[st] = {"ms_per_step": ms / steps, "mlups": mlups,
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

    t = time.perf_counter()
    case = inputs.discs(n=args.n, seed=2)
    log(f"inputs: {case.nodes} nodes in {time.perf_counter() - t:.1f} s")

    runs = {}
    for st in args.storages.split(","):
        r = time_storage(case, st, args.steps, args.warmup, dev)
        log(f"{st}: {r['mlups']:.0f} MLUPS, {r['ms_per_step']:.4f} ms/step, "
            f"{r['alg_GBps']:.0f} GB/s algorithmic")
        runs[st] = r
    if "f32" in runs:
        for r in runs.values():
            r["k_app_rel_vs_f32"] = r["k_app_after"] / runs["f32"]["k_app_after"] - 1
    head = runs.get("f32") or next(iter(runs.values()))
    st = head["storage"]
    achieved = head["alg_GBps"]
    traffic, traffic_bytes = measured_traffic(st, head["ms_per_step"], case.nodes)
    roof = {
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic,
        "traffic_bytes_per_launch": traffic_bytes,
        "kernel": f"sweep_kernel<{st}> (pressure x, periodic y)",
        "bytes_per_node": ALG_BYTES[st],
        "layout_bytes_per_node": LAYOUT_BYTES[st],
        "copy_GBps": copy_bandwidth(dev),
    }
    log(f"plain streaming kernel (b = a * 1, 1 GiB f32): {roof['copy_GBps']:.0f} GB/s "
        "(read + write)")
    adj = None
    if not args.no_adjoint:
        adj = time_adjoint(args.adjoint_n, args.adjoint_steps, args.adjoint_ckpt,
                           args.adjoint_hist, dev)
        log(f"adjoint: t_grad/t_fwd = {adj['grad_over_fwd']:.2f}, "
            f"(t_fwd + t_grad)/t_fwd = {adj['total_over_fwd']:.2f}")
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
    cpu = None if args.no_cpu else cpu_baseline(case)
    if cpu:
        log(f"cpu oracle: {cpu['value']:.2f} MLUPS ({cpu['sample']})")
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
        "adjoint": adj,
        "ensemble": ens,
        "klinkenberg_channel": kn,
        "d3q19": d3,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
