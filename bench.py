#!/usr/bin/env python3
"""Benchmark of the real-space Kohn-Sham hot path on one MI355X.

A step applies the Hamiltonian (kinetic stencil + local potential +
Kleinman-Bylander projectors) to all states of the workload, as blocks of B
states, with inputs resident in HBM.  Prints one JSON line:
  value    = grid points x states per second of H psi (whole job),
  roofline = achieved HBM bandwidth of the stencil kernel (algorithmic bytes
             per launch / average launch time, HIP events on its stream);
             traffic = HBM bytes per launch from the committed counter
             summary when it was taken on the current stencil source,
  eigensolve = time per RMM-DIIS step and time to 1e-6 Ha (lowest N-16
             eigenvalues against a converged FP64 reference) for the plain
             FP64 filter solve and the FP32 split-precision solve,
  cpu_baseline = the FP64 C/OpenMP oracle on the host cores (bounded sample).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                       [--no-eig] [--no-cpu] [--no-fp32] [--no-learned] [--no-cage]
       python bench.py --ordering-study
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

import synthetic  # noqa: E402

HBM_PEAK_GBS = 8000.0
# the workload the headline metric is quoted on, and the FP32 ones
PRIMARY = "sphere_r12_h0.2"
FP32_WORKLOADS = ("sphere_r12_h0.2_fp32", "periodic96_h0.25", "sphere_r18_h0.18_cage60")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def setup(w, dtype, B, lmax=1):
    import torch
    import paper_1306_2953_amd as rsd
    g = rsd.Grid.for_workload(w)
    atoms = synthetic.draw_atoms(w) if w.nat else None
    xyz = g.xyz()
    v = synthetic.potential_for(w, xyz, atoms)
    nl = None
    if atoms is not None:
        nl = rsd.NonLocal(g, atoms.pos, synthetic.couplings_lmax(w, atoms, lmax), w.rc, w.sigma,
                          max_states=-(-w.nstates // B) * B, lmax=lmax)
    rng = synthetic.rng_after_atoms(w)
    npdt = np.float64 if dtype == "f64" else np.float32
    psi = synthetic.draw_states(rng, w.nstates, g.np).astype(npdt)
    dev = torch.device("cuda:0")
    tpsi = torch.from_numpy(rsd.to_blocks(psi, B)).to(dev)
    del psi
    thpsi = torch.empty_like(tpsi)
    tv = torch.from_numpy(v.astype(npdt)).to(dev)
    nblk = int(tpsi.shape[0])        # the last block padded with zero states when B does not divide N
    proj = None
    if nl is not None:
        proj = torch.empty((nblk, nl.nat, nl.nproj, B), dtype=tpsi.dtype, device=dev)
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


def run_gpu(w, dtype, B, steps, warmup, lmax=1):
    import torch
    import paper_1306_2953_amd as rsd
    S = setup(w, dtype, B, lmax)
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
    """The FP64 C/OpenMP oracle applying H to all the workload's seeded
    states (every block), repeated for about budget_s seconds."""
    from oracle import cpu_hpsi, hamiltonian
    cpu_hpsi.build()
    og, atoms, H = hamiltonian.build_system(w)
    ch = cpu_hpsi.CpuHamiltonian(H)
    B = w.block
    nblk = -(-w.nstates // B)
    psi = synthetic.draw_states(synthetic.rng_after_atoms(w), w.nstates, og.np)
    blk = np.zeros((nblk, og.np, B))
    for k in range(w.nstates):
        blk[k // B, :, k % B] = psi[k]
    del psi
    ch.hpsi_blocks(blk)                      # warm-up
    reps, t0 = 0, time.perf_counter()
    while True:
        ch.hpsi_blocks(blk)
        reps += 1
        el = time.perf_counter() - t0
        if el > budget_s:
            break
    return dict(value=og.np * w.nstates * reps / el, unit="grid-pt*states/s", cores=cpu_hpsi.threads(),
                kind="oracle", cpu=cpu_hpsi.cpu_model(),
                sample=f"{reps} applications of FP64 H (stencil+V+KB) to all {w.nstates} seeded states "
                       f"({nblk} blocks of {B}) on the {og.np}-point grid, {el:.1f} s")


def traffic_probe(w, dtype, B):
    """Kernels for the FETCH_SIZE / WRITE_SIZE passes: an elementwise kernel
    that reads 1 GiB and writes 1 GiB (its counters calibrate bytes per
    counted KiB), then the stencil."""
    import torch
    import paper_1306_2953_amd as rsd
    n = 1 << 30
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 2.0, out=dst)
    torch.cuda.synchronize()
    del src, dst
    S = setup(w, dtype, B)
    for _ in range(3):
        rsd.hpsi_block(S["g"], S["nl"], S["v"], S["psi"], S["hpsi"])
    torch.cuda.synchronize()
    log(f"traffic probe done: 1 GiB read + 1 GiB write x3, H psi x3 ({w.name}, {dtype}, B {B})")


def _counter_means(path, counter):
    import csv
    import collections
    per = collections.defaultdict(list)
    with open(path) as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] == counter:
                per[row["Kernel_Name"]].append(float(row["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in per.items()}


# the kernels of one H psi call besides the projections: the z-marching
# stencil (FP64) or the per-brick stencil (FP32), and the projector add
STENCIL_KERNELS = ("hpsi_march_kernel", "hpsi_brick_kernel", "nl_add_kernel")


def traffic_record(w, dtype, fetch_csv, write_csv):
    """Calibrated HBM bytes per H psi call of the stencil kernel (interior
    and surface launches): counted KiB x (1 GiB / the KiB the counter shows
    for the 1 GiB calibration kernel)."""
    out = {}
    for key, path, counter in (("read", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        m = _counter_means(path, counter)
        cal = [v for k, v in m.items() if "elementwise_kernel" in k and "Fill" not in k]
        if not cal:
            raise SystemExit(f"no calibration kernel in {path}")
        factor = float(1 << 30) / (cal[0] * 1024.0)
        kib = sum(v for k, v in m.items() if any(n in k for n in STENCIL_KERNELS))
        out[key] = dict(counted_kib=kib, calibration_kib_per_gib=cal[0], bytes=kib * 1024.0 * factor)
    path = os.path.join(ROOT, "profiles", "hpsi_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        rec = {}
    rec[f"{w.name}/{dtype}"] = {
        "bytes_per_launch": out["read"]["bytes"] + out["write"]["bytes"],
        "read_bytes": out["read"]["bytes"], "write_bytes": out["write"]["bytes"],
        "fetch_counted_kib": out["read"]["counted_kib"], "write_counted_kib": out["write"]["counted_kib"],
        "fetch_kib_per_gib_read": out["read"]["calibration_kib_per_gib"],
        "write_kib_per_gib_written": out["write"]["calibration_kib_per_gib"],
        "source_sha256_16": stencil_source_hash(),
    }
    with open(path, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    log(f"traffic: {rec[f'{w.name}/{dtype}']}")


def stencil_source_hash() -> str:
    with open(os.path.join(ROOT, "paper_1306_2953_amd", "csrc", "hpsi.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(workload: str, dtype: str):
    """HBM bytes per launch of the stencil kernel from the committed counter
    summary, if it was taken on the current stencil source (else None)."""
    path = os.path.join(ROOT, "profiles", "hpsi_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    e = rec.get(f"{workload}/{dtype}")
    if not e or e.get("source_sha256_16") != stencil_source_hash():
        return None
    return e.get("bytes_per_launch")


def golden_eigs(name: str):
    """Lowest eigenvalues of the workload's FP64 H from tests/golden (an
    independent LOBPCG solve on the oracle's operator), or None."""
    path = os.path.join(ROOT, "tests", "golden", f"{name}_eigs.txt")
    if not os.path.exists(path):
        return None, path
    vals = [float(line.split()[1]) for line in open(path) if line.strip() and not line.startswith("#")]
    return np.array(vals), path


def eigensolve_run(w, dtype, B, max_steps, tol_res, ref=None, nbuf=16, log_every=20, stop_at_hit=False):
    """Steps from the seeded start until the lowest N - nbuf states all have
    residual < tol_res (or max_steps).  Returns per-step wall times, the
    eigenvalue history and the time to |eps - ref| < 1e-6 on those states."""
    import torch
    import paper_1306_2953_amd as rsd
    g = rsd.Grid.for_workload(w)
    atoms = synthetic.draw_atoms(w) if w.nat else None
    v = synthetic.potential_for(w, g.xyz(), atoms)
    nl = (rsd.NonLocal(g, atoms.pos, atoms.D, w.rc, w.sigma, max_states=-(-w.nstates // B) * B)
          if atoms is not None else None)
    npdt = np.float64 if dtype == "f64" else np.float32
    psi = synthetic.draw_states(synthetic.rng_after_atoms(w), w.nstates, g.np).astype(npdt)
    tp = torch.from_numpy(rsd.to_blocks(psi, B)).cuda()
    del psi
    tv = torch.from_numpy(v.astype(npdt)).cuda()
    solver = rsd.Eigensolver(g, nl, tv, w.nstates, B, tol=tol_res, block_stop=True)
    solver.orthonormalize(tp)          # padding states (B not dividing N) stay zero
    keep = w.nstates - nbuf
    times, eigs, t_hit, k_hit = [], [], None, None
    elapsed = 0.0
    for k in range(max_steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eig, res, _ = solver.step(tp)
        elapsed += time.perf_counter() - t0
        times.append(elapsed)
        eigs.append(eig.copy())
        if ref is not None and t_hit is None and np.max(np.abs(eig[:keep] - ref[:keep])) < 1e-6:
            t_hit, k_hit = elapsed, k + 1
        if log_every and k % log_every == 0:
            log(f"  {w.name} {dtype} step {k}: max res {res[:keep].max():.2e} eig0 {eig[0]:.10f} "
                f"t {elapsed:.2f} s")
        if np.all(res[:keep] < tol_res) or (stop_at_hit and t_hit is not None):
            break
    step_ms = 1e3 * (times[-1] - times[min(4, len(times) - 1)]) / max(1, len(times) - 1 - min(4, len(times) - 1))
    del solver, tp
    torch.cuda.empty_cache()
    return dict(steps=len(times), eig=eigs[-1], eigs=eigs, times=times, t_hit=t_hit, k_hit=k_hit,
                ms_per_step=step_ms, keep=keep, final_max_res=float(res[:keep].max()))


def learned_compare(w, max_steps=200, train_iters=30000, nbuf=16):
    """FP32 solve of the periodic workload with the trained network (a
    second direction next to the filter's in every trial step) against the
    same solve with the filter alone, from the same seeded start.  The
    network is trained first on the GPU (one crop per state from each of 60
    recorded filter steps, CG targets, energy-norm loss).  Reference eigenvalues: the golden LOBPCG
    values when present, else an FP64 filter solve run to residual 1e-6 on
    the lowest N - nbuf states."""
    import torch
    import paper_1306_2953_amd as rsd
    from paper_1306_2953_amd import learned
    keep = w.nstates - nbuf
    ref, path = golden_eigs(w.name)
    if ref is not None and len(ref) >= keep:
        refname = f"tests/golden/{os.path.basename(path)} (scipy LOBPCG on the oracle's FP64 operator)"
    else:
        log("learned compare: FP64 filter reference run")
        r64 = eigensolve_run(w, "f64", w.block, 400, 1e-6, nbuf=nbuf)
        ref = r64["eig"]
        refname = (f"FP64 filter solve to residual {r64['final_max_res']:.1e} on those states "
                   f"({r64['steps']} steps, {r64['ms_per_step']:.1f} ms per step)")
    g = rsd.Grid.for_workload(w)
    atoms = synthetic.draw_atoms(w)
    v = synthetic.potential_for(w, g.xyz(), atoms)
    nl = rsd.NonLocal(g, atoms.pos, atoms.D, w.rc, w.sigma, max_states=w.nstates)
    tv = torch.from_numpy(v.astype(np.float32)).cuda()
    psi0 = torch.from_numpy(rsd.to_blocks(
        synthetic.draw_states(synthetic.rng_after_atoms(w), w.nstates, g.np).astype(np.float32), w.block)).cuda()
    rsd.Context(g, w.nstates).orthonormalize(psi0)
    box = int(np.prod([g.nb[a] * 4 for a in range(3)]))
    net = rsd.Cnn(max(32, w.block), max(box, 16 ** 3))
    net.set_params(learned.init_params(0))
    rng = np.random.default_rng(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rec = rsd.Eigensolver(g, nl, tv, w.nstates, w.block, tol=1e-5, record=True)
    pairs = learned.collect_pairs(g, rec, psi0.clone(), net, steps=60, crops_per_state=1, crop=16, rng=rng,
                                  cg_tol=1e-5)
    del rec
    t_collect = time.perf_counter() - t0
    val = pairs.subset(pairs.state % 10 == 9)
    tr = pairs.subset(pairs.state % 10 != 9)
    t0 = time.perf_counter()
    learned.train(net, tr, g.h, iters=train_iters, batch=32, lr=learned.cosine_lr(3e-3, 1e-5, train_iters),
                  margin=3, rng=rng)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    vloss = learned.evaluate(net, val, g.h, 3, 32)
    npairs = pairs.n
    del pairs, tr, val
    torch.cuda.empty_cache()
    out = {"workload": w.name, "states": w.nstates, "measured_states": keep, "reference": refname,
           "metric": "steps and time to |eps - eps_ref| < 1e-6 Ha on the measured states",
           "training": {"pairs": npairs, "iterations": train_iters, "collect_s": t_collect,
                        "train_s": t_train, "validation_energy_norm_loss": vloss}}
    for name, pre in (("filter", None), ("learned", net)):
        s = rsd.Eigensolver(g, nl, tv, w.nstates, w.block, tol=1e-6)
        if pre is not None:
            s.set_precond(pre)
        x = psi0.clone()
        el, hit, nets = 0.0, None, []
        for k in range(max_steps):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            eig, res, _ = s.step(x)
            el += time.perf_counter() - t1
            nets.append(s.stats()["net_states"])
            err = float(np.max(np.abs(eig[:keep] - ref[:keep])))
            if k % 20 == 0:
                log(f"  learned compare {name} step {k}: max res {res[:keep].max():.2e} eig err {err:.1e} "
                    f"t {el:.2f} s")
            if err < 1e-6:
                hit = (k + 1, el)
                break
        out[name] = {"steps_run": k + 1, "final_max_residual": float(res[:keep].max()),
                     "final_median_residual": float(np.median(res[:keep])),
                     "final_max_eig_error_ha": err, "ms_per_step": 1e3 * el / (k + 1),
                     "steps_to_1e-6": None if hit is None else hit[0],
                     "time_to_1e-6_s": None if hit is None else hit[1]}
        if pre is not None:
            out[name]["mean_states_using_network"] = float(np.mean(nets))
        del s, x
        torch.cuda.empty_cache()
    return out


def eigensolve_compare(max_steps=400):
    """Plain FP64 filter solve of the 128-state sphere and the FP32
    split-precision solve of the same system, each timed until its lowest
    N - 16 eigenvalues are within 1e-6 Ha of the reference: the golden
    LOBPCG eigenvalues when present, else the FP64 run's converged end."""
    w2, w3 = synthetic.WORKLOADS["sphere_r12_h0.2"], synthetic.WORKLOADS["sphere_r12_h0.2_fp32"]
    ref, path = golden_eigs(w2.name)
    keep = w2.nstates - 16
    if ref is not None and len(ref) >= keep:
        log("eigensolve: FP64 plain run against the golden eigenvalues")
        r64 = eigensolve_run(w2, "f64", w2.block, max_steps, 1e-6, ref=ref, stop_at_hit=True)
        refname = f"tests/golden/{os.path.basename(path)} (scipy LOBPCG on the oracle's FP64 operator)"
    else:
        log("eigensolve: FP64 reference / plain run")
        r64 = eigensolve_run(w2, "f64", w2.block, 600, 1e-6)
        ref = r64["eig"]
        for k, (t, e) in enumerate(zip(r64["times"], r64["eigs"])):
            if np.max(np.abs(e[:keep] - ref[:keep])) < 1e-6:
                r64["t_hit"], r64["k_hit"] = t, k + 1
                break
        refname = f"FP64 run converged to residual < 1e-6 on those states ({r64['steps']} steps)"
    err64 = float(np.max(np.abs(r64["eig"][:keep] - ref[:keep])))
    log("eigensolve: FP32 split-precision run")
    r32 = eigensolve_run(w3, "f32", w3.block, max_steps, 1e-5, ref=ref, stop_at_hit=True)
    err32 = float(np.max(np.abs(r32["eig"][:keep] - ref[:keep])))
    return {
        "metric": "time to |eps - eps_ref| < 1e-6 Ha on the lowest N-16 states",
        "workload": w2.name, "states": w2.nstates, "measured_states": keep, "reference": refname,
        "plain_fp64_filter": {"time_s": r64["t_hit"], "steps": r64["k_hit"], "ms_per_step": r64["ms_per_step"],
                              "final_max_eig_error_ha": err64, "final_max_residual": r64["final_max_res"]},
        "fp32_split_filter": {"time_s": r32["t_hit"], "steps": r32["k_hit"],
                              "ms_per_step": r32["ms_per_step"], "steps_run": r32["steps"],
                              "final_max_eig_error_ha": err32, "final_max_residual": r32["final_max_res"]},
    }


def cage_compare(max_steps=300):
    """The large sphere (4.19M points, 60-atom cage, 240 states in blocks of
    64, the last padded): plain FP64 filter solve run to residual 1e-6 on the
    lowest N - 16 states (its end is the reference: no independent solve of
    this size exists), and the FP32 split-precision solve timed to 1e-6 Ha
    against it."""
    w = synthetic.WORKLOADS["sphere_r18_h0.18_cage60"]
    log("cage: FP64 plain run")
    r64 = eigensolve_run(w, "f64", w.block, max_steps, 1e-6)
    ref = r64["eig"]
    keep = r64["keep"]
    for k, (t, e) in enumerate(zip(r64["times"], r64["eigs"])):
        if np.max(np.abs(e[:keep] - ref[:keep])) < 1e-6:
            r64["t_hit"], r64["k_hit"] = t, k + 1
            break
    log("cage: FP32 split-precision run")
    r32 = eigensolve_run(w, "f32", w.block, max_steps, 1e-5, ref=ref, stop_at_hit=True)
    return {
        "workload": w.name, "states": w.nstates, "block": w.block, "measured_states": keep,
        "reference": (f"FP64 run's end (max residual {r64['final_max_res']:.1e} after {r64['steps']} steps); "
                      "parity unpinned: no independent solve at this size"),
        "plain_fp64_filter": {"time_s": r64["t_hit"], "steps": r64["k_hit"], "ms_per_step": r64["ms_per_step"]},
        "fp32_split_filter": {"time_s": r32["t_hit"], "steps": r32["k_hit"], "ms_per_step": r32["ms_per_step"],
                              "final_max_eig_error_ha": float(np.max(np.abs(r32["eig"][:keep] - ref[:keep])))},
    }


def hartree_rate(w, steps=10):
    """Hartree potential (Sec. 7) of a Gaussian density on the workload's grid:
    time per solve, the FFT box, and the bytes the six 1-D FFT passes move
    (each reads and writes the complex FP64 box once)."""
    import torch
    import paper_1306_2953_amd as rsd
    g = rsd.Grid.for_workload(w)
    xyz = g.xyz()
    r2 = np.sum(xyz * xyz, axis=1)
    rho = torch.from_numpy((2 * np.pi) ** -1.5 * np.exp(-r2 / 2.0)).cuda()
    ps = rsd.Poisson(g)
    out = torch.empty_like(rho)
    f = lambda: ps.solve(rho, out)
    for _ in range(2):
        f()
    t = time_calls(f, steps, torch.cuda.current_stream())
    fft_bytes = 6 * 2 * 16 * ps.nbox ** 3
    return {"workload": w.name, "grid_points": g.np, "fft_box": ps.nbox, "cutoff_radius_bohr": ps.rc,
            "ms_per_solve": t * 1e3, "fft_pass_bytes": fft_bytes,
            "fft_pass_bytes_over_solve_time_gbs": fft_bytes / t / 1e9}


def scf_run(w, nocc=8, nstates=32, max_iter=60, tol=1e-6):
    """The SCF loop on the workload's grid: nocc doubly occupied states out
    of nstates, FP64 and FP32 states; iterations and time until the density
    residual ||n_out - n_in|| is below tol (Anderson mixing, 3 eigensolver
    steps per iteration)."""
    import torch
    import paper_1306_2953_amd as rsd
    g = rsd.Grid.for_workload(w)
    atoms = synthetic.draw_atoms(w)
    v = torch.from_numpy(synthetic.potential_for(w, g.xyz(), atoms)).cuda()
    nl = rsd.NonLocal(g, atoms.pos, atoms.D, w.rc, w.sigma, max_states=nstates)
    out = {"workload": w.name, "occupied": nocc, "states": nstates,
           "criterion": f"density residual (h^3-weighted L2) < {tol:g} (FP64 states), {10 * tol:g} (FP32)"}
    # FP32 states: the density's own rounding floor is a few 1e-6, so their
    # criterion is 10 tol
    for name, dt, npdt, t_ok in (("fp64", torch.float64, np.float64, tol), ("fp32", torch.float32, np.float32, 10 * tol)):
        psi = synthetic.draw_states(synthetic.rng_after_atoms(w), nstates, g.np).astype(npdt)
        t = torch.from_numpy(rsd.to_blocks(psi, 32)).cuda()
        del psi
        s = rsd.Scf(g, nl, v, nstates, 32, nocc=nocc, dtype=dt, tol=1e-9)
        s.start(t)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist = []
        for it in range(max_iter):
            eig, res, dr = s.iterate(t)
            hist.append(dr)
            if dr < t_ok:
                break
        el = time.perf_counter() - t0
        out[name] = {"iterations": it + 1, "time_s": el, "converged": bool(hist[-1] < t_ok),
                     "final_density_residual": hist[-1], "homo_ha": float(eig[nocc - 1]),
                     "lumo_ha": float(eig[nocc]), "ms_per_iteration": 1e3 * el / (it + 1)}
        log(f"scf {name}: {out[name]}")
        del s, t
        torch.cuda.empty_cache()
    return out


def ordering_study(steps=10):
    """Sec. 5.1 (Figs. "locality", "cache", "laplacian") on the molecular
    grid: (1) the FP64 C/OpenMP oracle's H psi throughput on the host cores
    for the standard (lexicographic) order and sub-grid orders of several
    brick sizes, all 128 states in blocks of 32, plus block sizes 1..64 in
    4x4x4 order; (2) the GPU's H psi throughput (FP64 and FP32) for block
    sizes 1..64 (the kernels use 4x4x4 bricks)."""
    import torch
    import paper_1306_2953_amd as rsd
    from oracle import cpu_hpsi, grid as ogrid, hamiltonian
    w = synthetic.WORKLOADS["union_cage60_r5.5_h0.41"]
    cpu_hpsi.build()
    atoms = synthetic.draw_atoms(w)
    out = {"workload": w.name, "states": w.nstates, "cpu_threads": cpu_hpsi.threads(),
           "cpu": cpu_hpsi.cpu_model(), "unit": "grid-pt*states/s"}

    def cpu_rate(og, B, budget=3.0):
        v = synthetic.potential_for(w, og.xyz, atoms)
        from oracle import kb
        H = hamiltonian.Hamiltonian(og, v, kb.build_projectors(og, atoms.pos, atoms.D, w.rc, w.sigma))
        ch = cpu_hpsi.CpuHamiltonian(H)
        psi = synthetic.draw_states(synthetic.rng_after_atoms(w), w.nstates, og.np)
        blk = np.ascontiguousarray(psi.reshape(w.nstates // B, B, og.np).transpose(0, 2, 1))
        ch.hpsi_blocks(blk)
        reps, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < budget:
            ch.hpsi_blocks(blk)
            reps += 1
        return og.np * w.nstates * reps / (time.perf_counter() - t0)

    orders = {}
    L = None
    for name, brick in (("standard", None), ("bricks 2x2x2", (2, 2, 2)), ("bricks 4x4x4", (4, 4, 4)),
                        ("bricks 8x8x8", (8, 8, 8)), ("bricks 16x16x16", (16, 16, 16))):
        if brick is None:
            L = int(ogrid.grid_for(w).L.max())
            brick = (L, L, L)
        og = ogrid.grid_for(w, brick=brick)
        orders[name] = cpu_rate(og, 32)
        log(f"ordering study: cpu {name}: {orders[name]:.3e}")
    out["cpu_order_B32"] = orders
    og = ogrid.grid_for(w)
    out["cpu_block_size_4x4x4"] = {B: cpu_rate(og, B) for B in (1, 4, 16, 32, 64)}
    log(f"ordering study: cpu block sizes {out['cpu_block_size_4x4x4']}")
    g = rsd.Grid.for_workload(w)
    v = synthetic.potential_for(w, g.xyz(), atoms)
    nl = rsd.NonLocal(g, atoms.pos, atoms.D, w.rc, w.sigma, max_states=w.nstates)
    gpu = {}
    for dt, npdt in (("f64", np.float64), ("f32", np.float32)):
        tv = torch.from_numpy(v.astype(npdt)).cuda()
        psi = synthetic.draw_states(synthetic.rng_after_atoms(w), w.nstates, g.np).astype(npdt)
        rates = {}
        for B in (1, 2, 4, 8, 16, 32, 64):
            tp = torch.from_numpy(rsd.to_blocks(psi, B)).cuda()
            th = torch.empty_like(tp)
            f = lambda: rsd.hpsi_block(g, nl, tv, tp, th)
            f()
            t = time_calls(f, steps, torch.cuda.current_stream())
            rates[B] = g.np * w.nstates / t
        gpu[dt] = rates
        log(f"ordering study: gpu {dt} block sizes {rates}")
    out["gpu_block_size"] = gpu
    return out


def cnn_profile(k):
    """For kernel-trace runs: k applications of the learned preconditioner to
    the 256 FP32 states of the periodic 96^3 workload (the three 3x3x3
    convolution layers over the whole box, 2160 multiply-adds per box point
    and state), then k Adam training steps on batches of 32 random 16^3
    crops (loss, gradients, update).  Returns per-call times and the
    forward rate."""
    import torch
    import paper_1306_2953_amd as rsd
    from paper_1306_2953_amd import learned
    w = synthetic.WORKLOADS["periodic96_h0.25"]
    g = rsd.Grid.for_workload(w)
    r = torch.from_numpy(rsd.to_blocks(synthetic.draw_states(synthetic.rng_after_atoms(w), w.nstates, g.np)
                                       .astype(np.float32), w.block)).cuda()
    nst = int(r.shape[0]) * w.block
    sigma = torch.full((nst,), -1.0, dtype=torch.float64, device="cuda")
    net = rsd.Cnn(max(32, w.block), int(np.prod([g.nb[a] * 4 for a in range(3)])))
    net.set_params(learned.init_params(0))
    net_box = net.box(g)
    stream = torch.cuda.current_stream()
    net.precondition(g, r, sigma)
    t_pre = time_calls(lambda: net.precondition(g, r, sigma), k, stream)
    gen = torch.Generator(device="cuda").manual_seed(0)
    u = torch.randn((32, 16, 16, 16), generator=gen, device="cuda", dtype=torch.float32)
    t = torch.randn((32, 16, 16, 16), generator=gen, device="cuda", dtype=torch.float32)
    sig = torch.full((32,), -1.0, dtype=torch.float64, device="cuda")
    net.train_step(u, t, sig, g.h, 3, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(k):
        net.train_step(u, t, sig, g.h, 3, 1e-4)
    torch.cuda.synchronize()
    t_train = (time.perf_counter() - t0) / k
    npts = int(np.prod(net_box))
    flop = 2.0 * 2160 * npts * nst
    out = {"box": list(net_box), "states": nst, "precondition_s": t_pre, "forward_flop": flop,
           "forward_tflops": flop / t_pre / 1e12, "train_step_s": t_train}
    log(f"cnn profile: {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=PRIMARY, choices=sorted(synthetic.WORKLOADS))
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-eig", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--ordering-study", action="store_true",
                    help="point-ordering and block-size study on the molecular grid (host oracle and GPU); "
                         "prints one JSON line")
    ap.add_argument("--no-cage", action="store_true",
                    help="skip the large-sphere FP32 H psi throughput line")
    ap.add_argument("--cage-eig", type=int, default=0, metavar="STEPS",
                    help="also run the large-sphere eigensolve comparison (FP64 reference run of up to STEPS "
                         "steps, about 0.25 s each, then the FP32 solve timed against it)")
    ap.add_argument("--profile-eig", type=int, default=0, metavar="K",
                    help="for kernel-trace runs: K eigensolver steps of the FP64 sphere and of "
                         "its FP32 split-precision form from the seeded start; prints step times")
    ap.add_argument("--profile-cnn", type=int, default=0, metavar="K",
                    help="for kernel-trace runs: K applications of the learned preconditioner to the "
                         "periodic workload's 256 states and K training steps; prints the forward rate")
    ap.add_argument("--traffic-record", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn the counter_collection.csv files of the FETCH_SIZE and WRITE_SIZE "
                         "passes over --traffic-probe into profiles/hpsi_traffic.json")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="for counter runs: three 1 GiB device copies (calibration), then "
                         "three H psi applications of the workload; prints nothing")
    a = ap.parse_args()
    if a.gpus != 1:
        print(json.dumps({"error": "the H psi path and eigensolver run on one GPU (no multi-GPU sharding is implemented); --gpus must be 1"}))
        sys.exit(2)
    w = synthetic.WORKLOADS[a.workload]
    B = a.block or w.block
    dtype = "f32" if w.name in FP32_WORKLOADS else "f64"
    primary = w.name == PRIMARY
    if a.profile_eig:
        for name, dt in ((PRIMARY, "f64"), (PRIMARY + "_fp32", "f32")):
            wk = synthetic.WORKLOADS[name]
            r = eigensolve_run(wk, dt, wk.block, a.profile_eig, 0.0, log_every=1)
            log(f"{wk.name} {dt}: step times {np.diff([0.0] + r['times'])}")
        return
    if a.profile_cnn:
        print(json.dumps(cnn_profile(a.profile_cnn)), flush=True)
        return
    if a.ordering_study:
        print(json.dumps(ordering_study(a.steps)), flush=True)
        return
    if a.traffic_record:
        traffic_record(w, dtype, *a.traffic_record)
        return
    if a.traffic_probe:
        traffic_probe(w, dtype, B)
        return
    log(f"workload {w.name} dtype {dtype} B {B}")
    r = run_gpu(w, dtype, B, a.steps, a.warmup)
    log(f"primary: {r}")
    extra = {}
    if primary and not a.no_fp32:
        w3 = synthetic.WORKLOADS["sphere_r12_h0.2_fp32"]
        r3 = run_gpu(w3, "f32", B, a.steps, a.warmup)
        log(f"fp32: {r3}")
        extra[w3.name] = {k: r3[k] for k in ("ptstates_per_s", "gflops", "t_step",
                                                 "t_kernel", "achieved_gbs", "frac")}
    if primary and not a.no_cage:
        w5 = synthetic.WORKLOADS["sphere_r18_h0.18_cage60"]
        r5 = run_gpu(w5, "f32", w5.block, a.steps, a.warmup)
        log(f"cage fp32: {r5}")
        extra[w5.name] = {k: r5[k] for k in ("ptstates_per_s", "gflops", "t_step", "t_kernel", "achieved_gbs",
                                             "frac", "np", "N", "B", "nblk")}
        extra[w5.name]["note"] = "240 states in 4 blocks of 64 (16 zero padding states, not counted)"
    if primary:
        # projectors to l = 3 (16 per atom instead of 4): the same H psi call
        for wk, dt in ((w, dtype), (synthetic.WORKLOADS["sphere_r12_h0.2_fp32"], "f32")):
            rl = run_gpu(wk, dt, B, a.steps, a.warmup, lmax=3)
            extra[f"{wk.name}_lmax3"] = {k: rl[k] for k in ("ptstates_per_s", "t_step", "t_proj")}
            log(f"{wk.name} lmax 3: {extra[f'{wk.name}_lmax3']}")
        extra["hartree"] = hartree_rate(w)
        log(f"hartree: {extra['hartree']}")
    scf = None
    if primary and not a.no_eig:
        scf = scf_run(w)
    eig = None
    if primary and not a.no_eig:
        eig = eigensolve_compare()
        log(f"eigensolve: {eig}")
    cage = None
    if primary and a.cage_eig > 0:
        cage = cage_compare(a.cage_eig)
        log(f"cage eigensolve: {cage}")
    lrn = None
    if primary and not a.no_learned:
        log("learned preconditioner: periodic workload")
        lrn = learned_compare(synthetic.WORKLOADS["periodic96_h0.25"])
        log(f"learned: {lrn}")
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
                     "unit": "GB/s", "frac": r["frac"],
                     "traffic": measured_traffic(w.name, dtype),
                     "kernel": ("hpsi_march_kernel (full + partial chunk launches) + nl_add_kernel, "
                                "one H psi call" if dtype == "f64" else
                                "hpsi_brick_kernel (interior + surface launches), one H psi call"),
                     "bytes_per_launch": r["bytes_kernel"],
                     "avg_launch_s": r["t_kernel"]},
        "eigensolve": eig,
        "eigensolve_cage": cage,
        "scf": scf,
        "learned_preconditioner": lrn,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
