#!/usr/bin/env python3
"""Benchmark of the real-space Kohn-Sham hot path on one MI355X.

A step applies the Hamiltonian (kinetic stencil + local potential +
Kleinman-Bylander projectors) to all states of the workload, as blocks of B
states, with inputs resident in HBM.  Prints one JSON line:
  value    = grid points x states per second of H psi (whole job),
  roofline = achieved HBM bandwidth of the stencil kernel (algorithmic bytes
             per launch / average launch time, HIP events on its stream),
  cpu_baseline = the FP64 C/OpenMP oracle on the host cores (bounded sample).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 2|3|5]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synthetic  # noqa: E402

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def setup(w, dtype, B):
    import torch
    import paper_1306_2953_amd as rsd
    g = rsd.Grid.for_workload(w)
    atoms = synthetic.draw_atoms(w) if w.nat else None
    xyz = g.xyz()
    v = synthetic.potential_for(w, xyz, atoms)
    nl = None
    if atoms is not None:
        nl = rsd.NonLocal(g, atoms.pos, atoms.D, w.rc, w.sigma, max_states=w.nstates)
    rng = synthetic.rng_after_atoms(w)
    npdt = np.float64 if dtype == "f64" else np.float32
    psi = synthetic.draw_states(rng, w.nstates, g.np).astype(npdt)
    dev = torch.device("cuda:0")
    tpsi = torch.from_numpy(rsd.to_blocks(psi, B)).to(dev)
    del psi
    thpsi = torch.empty_like(tpsi)
    tv = torch.from_numpy(v.astype(npdt)).to(dev)
    nblk = w.nstates // B
    proj = None
    if nl is not None:
        proj = torch.empty((nblk, nl.nat, 4, B), dtype=tpsi.dtype, device=dev)
    return dict(g=g, nl=nl, v=tv, psi=tpsi, hpsi=thpsi, proj=proj, nblk=nblk, B=B)


def time_calls(fn, n, stream):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(n):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / n * 1e-3     # seconds per call


def run_gpu(w, dtype, B, steps, warmup):
    import torch
    import paper_1306_2953_amd as rsd
    S = setup(w, dtype, B)
    stream = torch.cuda.current_stream()
    g, nl = S["g"], S["nl"]

    def step():
        rsd.hpsi_block(g, nl, S["v"], S["psi"], S["hpsi"], stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_step = time_calls(step, steps, stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the projections alone (two small kernels), to isolate the stencil kernel
    t_proj = 0.0
    if nl is not None:
        t_proj = time_calls(lambda: rsd.project_nl(g, nl, S["psi"], S["proj"], stream),
                            max(steps, 5), stream)
    s = 8 if dtype == "f64" else 4
    npts, N = g.np, w.nstates
    # algorithmic bytes of the stencil kernel per launch: read psi once,
    # write H psi once, the potential once per block
    bytes_kernel = npts * N * (2 * s) + npts * S["nblk"] * s
    t_kernel = max(t_step - t_proj, 1e-12)
    achieved = bytes_kernel / t_kernel / 1e9
    out = dict(np=npts, N=N, B=B, nblk=S["nblk"], t_step=t_step, t_proj=t_proj,
               t_kernel=t_kernel, wall=wall, bytes_kernel=bytes_kernel,
               achieved_gbs=achieved, frac=achieved / HBM_PEAK_GBS,
               ptstates_per_s=npts * N / t_step,
               gflops=npts * N * 51 / t_step / 1e9)
    del S
    torch.cuda.empty_cache()
    return out


def cpu_baseline(w, budget_s=15.0):
    """The FP64 C/OpenMP oracle on one block of B states of the workload,
    repeated for about budget_s seconds."""
    from oracle import cpu_hpsi, hamiltonian
    og, atoms, H = hamiltonian.build_system(w)
    ch = cpu_hpsi.CpuHamiltonian(H)
    B = w.block
    rng = np.random.default_rng(0)
    blk = rng.uniform(-1, 1, size=(1, og.np, B))
    ch.hpsi_blocks(blk)                      # warm-up
    reps, t0 = 0, time.perf_counter()
    while True:
        ch.hpsi_blocks(blk)
        reps += 1
        el = time.perf_counter() - t0
        if el > budget_s or reps >= 200:
            break
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=og.np * B * reps / el, unit="grid-pt*states/s", cores=threads,
                kind="oracle",
                sample=f"{reps} applications of FP64 H (stencil+V+KB) to one block of {B} "
                       f"states on the {og.np}-point grid, {el:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    w = synthetic.CONFIGS[a.config]
    B = a.block or w.block
    dtype = "f32" if a.config in (3, 4, 5) else "f64"
    log(f"workload {w.name} dtype {dtype} B {B}")
    r = run_gpu(w, dtype, B, a.steps, a.warmup)
    log(f"primary: {r}")
    extra = {}
    if a.config == 2 and not a.no_fp32:
        w3 = synthetic.CONFIGS[3]
        r3 = run_gpu(w3, "f32", B, a.steps, a.warmup)
        log(f"fp32: {r3}")
        extra["cfg3_fp32"] = {k: r3[k] for k in ("ptstates_per_s", "gflops", "t_step",
                                                 "t_kernel", "achieved_gbs", "frac")}
    cpu = None
    if not a.no_cpu:
        log("cpu baseline")
        cpu = cpu_baseline(w)
        log(f"cpu: {cpu}")
    line = {
        "metric": "Hψ grid-pt·states/s",
        "value": r["ptstates_per_s"],
        "unit": "grid-pt*states/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": r["t_step"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": w.name, "grid_points": r["np"], "states": r["N"],
                   "block": B, "atoms": w.nat, "projectors_per_atom": 4,
                   "stencil_points": 25},
        "gflops": r["gflops"],
        "roofline": {"bound": "hbm", "achieved": r["achieved_gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": r["frac"], "traffic": None,
                     "kernel": "hpsi_brick_kernel",
                     "bytes_per_launch": r["bytes_kernel"],
                     "avg_launch_s": r["t_kernel"]},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
