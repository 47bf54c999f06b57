#!/usr/bin/env python3
"""Throughput benchmark of the MM / HV lattice-Boltzmann Maxwell steppers on one MI355X.

Workload: the 256^3 Hertz-dipole lattice (vacuum, 16-cell quadratic sigma
sponge on every face, soft point current J_z = sin(2 pi n / 40) at the centre,
three field probes recorded every step).  One benchmark step is one time step
of the whole lattice: gather with in-place streaming, collision, sources,
scatter and the fused FP64 probe recording.  The headline value is the MM
model with FP32 population storage; the HV model, BF16 storage, the
equilibrium-shifted BF16 storage and the MM scheme in difference form (24
populations per cell, same E and B) are timed the same way and reported under
"variants".  Further sections: the batched ragged 1-D multilayer workload, the
adjoint on the 128 x 128 x 256 inverse-design lattice, the radiation pattern of
the Gaussian dipole at 256^3 (flux monitor), the refinement study of Section
IV (error against GPU time and distribution-function memory), the 384^3 precision
sweep, and the FP64 oracle on the host cores.

Prints one JSON line.  `value` is lattice updates per second (MLUPS) with the
state already resident in HBM; `roofline` prices the step kernel against the
MI355X HBM peak using the algorithmic bytes per lattice update (every
population read once and written once, plus 12 B of media).
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
VALU_LANE_PEAK = 256 * 4 * 16 * 2.4e9  # FP32 lane-instructions/s without packed FP32
VALU_PER_LU_BATCH = 335.5  # profiled VALU lane-instructions per update of the blocked multilayer batch
# every population read and written once, 12 B of media; the equilibrium-shifted
# formats also write and read one 16-byte record per cell
BYTES_PER_LU = {("mm", "f32"): 2 * 50 * 4 + 12, ("mm", "bf16"): 2 * 50 * 2 + 12,
                ("hv", "f32"): 2 * 36 * 4 + 12, ("hv", "bf16"): 2 * 36 * 2 + 12,
                ("mm", "f16"): 2 * 50 * 2 + 12, ("hv", "f16"): 2 * 36 * 2 + 12,
                ("mm", "bf16_shifted"): 2 * 50 * 2 + 12 + 32, ("hv", "bf16_shifted"): 2 * 36 * 2 + 12 + 32,
                ("mm", "f16_shifted"): 2 * 50 * 2 + 12 + 32, ("hv", "f16_shifted"): 2 * 36 * 2 + 12 + 32,
                # MM in difference form: 24 populations per cell
                ("mmd", "f32"): 2 * 24 * 4 + 12, ("mmd", "bf16"): 2 * 24 * 2 + 12,
                ("mmd", "bf16_shifted"): 2 * 24 * 2 + 12 + 32}


def workload_model(model: str) -> str:
    """The scheme whose workload (media units, sponge, source) a model runs."""
    return "mm" if model == "mmd" else model


# sources the single-lattice step kernels are compiled from
STEP_KERNEL_SOURCES = ("include/lbem.h", "paper_2309_08068_amd/csrc/lbem_common.hpp",
                       "paper_2309_08068_amd/csrc/lbem_internal.hpp", "paper_2309_08068_amd/csrc/lbem_lattice.hip",
                       "paper_2309_08068_amd/csrc/lbem_model.hpp", "paper_2309_08068_amd/csrc/lbem_util_kernels.hpp")


def kernel_source_hash() -> str:
    """Hash of the step-kernel sources with comments and blank space removed
    (a documentation edit leaves the measured kernels, and so the hash, alone)."""
    import re

    h = hashlib.sha256()
    for fn in STEP_KERNEL_SOURCES:
        with open(os.path.join(ROOT, fn), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(fn.encode())
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(model: str, storage: str, n: int):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    v = rec.get("variants", {}).get(f"{model}_{storage}")
    if not v or v.get("cells") != n:
        return None
    return v.get("bytes_per_launch")


def time_variant(model: str, storage: str, n: int, steps: int, warmup: int):
    import torch
    from paper_2309_08068_amd import inputs, lbem

    w = inputs.dipole(workload_model(model), n=n, steps=steps)
    lat = lbem.lattice_from_workload(w, storage=storage, storage_scale=0.0, model=model)
    lat.set_probes(w.probes, warmup + 2 * steps + 1)
    tuning = lat.autotune(10)
    stream = torch.cuda.current_stream()
    lat.step(warmup)
    torch.cuda.synchronize()
    # whole-job timing of `steps` steps
    t0 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # per-launch duration of the step kernel from HIP events on the library's stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lat.step(steps)
    e1.record(stream)
    e1.synchronize()
    kernel_ms = e0.elapsed_time(e1) / steps
    cells = w.n
    mlups = cells * steps / wall / 1e6
    bpl = BYTES_PER_LU[(model, storage)]
    achieved = bpl * cells / (kernel_ms * 1e-3) / 1e9
    del lat
    torch.cuda.empty_cache()
    return dict(model=model, storage=storage, cells=cells, mlups=mlups, ms_per_step=wall * 1e3 / steps,
                kernel_ms=kernel_ms, bytes_per_lu=bpl, achieved_gbs=achieved, frac=achieved / HBM_PEAK_GBS,
                traffic=measured_traffic(model, storage, cells), tuning=tuning)


def time_batch(steps: int):
    """Multilayer workload: 512 ragged 1-D MM instances (500..8000 cells), FP32.
    One persistent launch captured in a HIP graph (autotuned launch shape and
    temporal blocking) versus the same launch with one step per pass and one
    launch per instance per step (timed on a sample of steps)."""
    import torch
    from paper_2309_08068_amd import inputs, lbem

    bt = inputs.multilayer("mm", steps=steps)
    b = lbem.batch_from_inputs(bt)
    threads, gpc = b.autotune(10)
    k = b.blocking()
    total = int(bt.offsets[-1])

    def graph_wall():
        b.step_graph(steps)  # capture + warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step_graph(steps)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    wall = graph_wall()
    # one step per pass, in the fastest such shape measured on this part
    b.set_blocking(0)
    b.set_launch(1024, 1)
    wall_1 = graph_wall()
    sample = 20
    b.step_per_instance(2)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    b.step_per_instance(sample)
    torch.cuda.synchronize()
    wall_pi = (time.perf_counter() - t1) / sample * steps
    mlups = total * steps / wall / 1e6
    bpl = BYTES_PER_LU[("mm", "f32")]
    return {"workload": f"multilayer_512x[500,8000]_{steps}steps", "cells": total, "launch": [threads, gpc],
            "steps_per_pass": k, "persistent_graph_s": round(wall, 4), "mlups": round(mlups, 1),
            # bytes of one read and one write of every population per step, over the wall time: above the
            # HBM peak when passes of several steps keep the cells on chip
            "one_step_equivalent_gbs": round(bpl * total * steps / wall / 1e9, 1),
            "frac_of_one_step_roofline": round(bpl * total * steps / wall / 1e9 / HBM_PEAK_GBS, 4),
            "one_step_per_pass_s": round(wall_1, 4), "one_step_per_pass_mlups": round(total * steps / wall_1 / 1e6, 1),
            "one_step_per_pass_frac": round(bpl * total * steps / wall_1 / 1e9 / HBM_PEAK_GBS, 4),
            "per_instance_loop_s": round(wall_pi, 3), "per_instance_sample_steps": sample,
            "speedup_vs_per_instance": round(wall_pi / wall, 1),
            "speedup_vs_one_step_per_pass": round(wall_1 / wall, 2),
            # blocked passes are bound by vector-ALU issue: rocprofv3 SQ_INSTS_VALU gives about 335
            # lane-instructions per update of this workload (1024 threads, 48 steps per pass, halo
            # recomputation included); the part issues 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz without
            # packed FP32
            "roofline_blocked": {"bound": "alu", "unit": "T lane-instr/s", "peak": VALU_LANE_PEAK / 1e12,
                                 "valu_per_lu_profiled": VALU_PER_LU_BATCH,
                                 "achieved": round(mlups * 1e6 * VALU_PER_LU_BATCH / 1e12, 1),
                                 "frac": round(mlups * 1e6 * VALU_PER_LU_BATCH / VALU_LANE_PEAK, 4)}}


def time_adjoint(model: str, steps: int, K: int, keep: int, forward_model: str = None):
    """Inverse-design lattice 128 x 128 x 256 (FP32): adjoint pass (forward with
    a checkpoint every K steps, the last `keep` segments also keeping their E
    frames, + reverse pass) over the plain forward of `forward_model` (default:
    the same model) with the same detector.  Also reports the loss, the energy
    of the forward run relative to the initial pulse (largest and last, from
    an energy series every 50 steps: growth shows here) and lbem_check's
    verdict on the final state."""
    import torch
    from paper_2309_08068_amd import inputs, lbem

    fmodel = forward_model or model
    w = inputs.slab(workload_model(model), steps=steps)

    def plain_forward():
        lat = lbem.lattice_from_workload(w, model=fmodel)
        lat.autotune(5)
        lat.set_fields(*w.fields0())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(steps)
        torch.cuda.synchronize()
        fwd = time.perf_counter() - t0
        # untimed: the energy history of the same run
        lat.set_fields(*w.fields0())
        u0 = lat.energy().item()
        series = lat.set_energy_series(50, (steps + 49) // 50)
        lat.step(steps)
        try:
            # no sources: the pulse's energy can only fall (the sponges absorb)
            lat.check(2.0 * u0)
            health = "ok"
        except lbem.LbemError as e:
            health = lbem.STATUS.get(e.status, str(e.status))
        u = series.cpu().numpy()
        del lat
        return fwd, u0, u, health

    fwd, u0, u, health = plain_forward()
    lat = lbem.lattice_from_workload(w, model=model)
    lat.autotune(5)  # the recomputed segments use the step kernel's tuning
    # a short adjoint pass lets the library pick its adjoint launch tuning
    # (once per lattice) before anything is timed
    lat.set_fields(*w.fields0())
    ws = lat.adjoint_workspace(2 * K, K, 1)
    lat.adjoint_forward(2 * K, K, w.det_z, ws, 1)
    lat.adjoint_backward(ws, *w.fields0())
    del ws
    lat.set_fields(*w.fields0())
    ws = lat.adjoint_workspace(steps, K, keep)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss = lat.adjoint_forward(steps, K, w.det_z, ws, keep)
    ge, gs = lat.adjoint_backward(ws, *w.fields0())
    torch.cuda.synchronize()
    adj = time.perf_counter() - t1
    ok = bool(torch.isfinite(ge).all() and torch.isfinite(gs).all())
    out = {"model": model, "forward_model": fmodel, "keep": keep, "forward_s": round(fwd, 4),
           "adjoint_total_s": round(adj, 4), "ratio": round(adj / fwd, 3), "loss": float(f"{loss.item():.6e}"),
           "grad_eps_max": float(f"{ge.abs().max().item():.4e}"), "finite_gradients": ok,
           "energy_max_over_initial": round(float(u.max() / u0), 4),
           # first time level (every 50) whose energy exceeds the initial one
           "growth_from_step": next((50 * i for i, x in enumerate(u) if x > u0 * (1 + 1e-6)), None),
           "energy_last_over_initial": round(float(u[-1] / u0), 4), "check": health,
           "workspace_gb": round(ws.numel() / 1e9, 2)}
    del ws, lat
    torch.cuda.empty_cache()
    return out


def radiation_pattern(model: str, n: int):
    """Section IV-C radiation pattern at n^3: Gaussian dipole, flux monitor on a
    sphere of radius R; deviation of the normalised r^2 max|E x H| from
    sin^2(theta), and the largest flux per sample cell over that of the
    continuum fields of the same source (tests/dipole_theory.py: switched-on
    dipoles with their static moment, near-field terms and extent)."""
    import math

    import numpy as np
    import torch
    from paper_2309_08068_amd import inputs, lbem

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import dipole_theory

    rad = inputs.radiation(workload_model(model), n=n)
    w = rad.workload
    lat = lbem.lattice_from_workload(w, model=model)
    lat.autotune(2)
    flux = lat.set_flux_monitor(rad.cells, *rad.window)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(w.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    smax = flux.cpu().numpy()
    pattern = smax * rad.radius ** 2 / (smax * rad.radius ** 2).max()
    wm = workload_model(model)
    eps0, mu0 = inputs.VACUUM_CONSTANTS[wm]
    om = 2 * math.pi / rad.period
    theory = dipole_theory.max_flux(dipole_theory.workload_sources(w.shape, w.currents),
                                    dipole_theory.sample_points(w.shape, rad.cells),
                                    np.arange(*rad.window, dtype=np.float64), eps0, mu0, om)
    keep = np.sin(rad.theta) > 0.5
    ratio = smax[keep] / theory[keep]
    del lat
    torch.cuda.empty_cache()
    return {"model": model, "steps": w.steps, "run_s": round(wall, 4),
            "pattern_max_dev_from_sin2": round(float(np.abs(pattern - np.sin(rad.theta) ** 2).max()), 4),
            "flux_over_continuum": {"mean": round(float(ratio.mean()), 4), "min": round(float(ratio.min()), 4),
                                    "max": round(float(ratio.max()), 4)}}


def time_precision(model: str, n: int, steps: int):
    """Precision sweep on the n^3 point dipole: every storage format runs the
    same `steps` steps (after the autotuner); reports its throughput and the
    relative L2 distance of E and B from the FP32-storage run (FP32 storage
    itself is held to the FP64 oracle by the parity tests)."""
    import torch
    from paper_2309_08068_amd import inputs, lbem

    w = inputs.dipole(model, n=n, steps=steps)
    out, ref = {}, None
    for storage in ("f32", "bf16", "f16", "bf16_shifted", "f16_shifted"):
        lat = lbem.lattice_from_workload(w, storage=storage, storage_scale=1024.0 if "f16" in storage else 0.0)
        lat.autotune(5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        E, B, _, _ = lat.fields()
        del lat
        r = {"mlups": round(w.n * steps / wall / 1e6, 1),
             "frac": round(BYTES_PER_LU[(model, storage)] * w.n * steps / wall / 1e9 / HBM_PEAK_GBS, 4)}
        if ref is None:
            ref = (E, B)
            c = n // 2
            ax = torch.arange(n, device=E.device, dtype=torch.float32) - c
            r2 = ax[:, None, None] ** 2 + ax[None, :, None] ** 2 + ax[None, None, :] ** 2
            far = (r2 >= 32 ** 2).reshape(-1)  # cells at least 32 from the source
            del ax, r2
        else:
            r["rel_l2_vs_f32"] = [round(float((X.double() - R.double()).norm() / R.double().norm()), 5)
                                  for X, R in ((E, ref[0]), (B, ref[1]))]
            r["rel_l2_E_r_ge_32"] = round(float((E[:, far].double() - ref[0][:, far].double()).norm()
                                                / ref[0][:, far].double().norm()), 5)
            del E, B
        out[storage] = r
        torch.cuda.empty_cache()
        print(f"# precision {model} {n}^3 {storage}: {r}", file=sys.stderr, flush=True)
    del ref
    torch.cuda.empty_cache()
    return {"workload": f"hertz_dipole_{n}^3_{model}_{steps}steps", "formats": out}


def cpu_baseline(n: int, sample_steps: int):
    """The FP64 oracle on the host cores: a few steps of the same 256^3 MM dipole
    lattice with every OpenMP thread, and (in a child process with one thread)
    a smaller sample of the same lattice single-threaded."""
    import subprocess

    import oracle
    from paper_2309_08068_amd import inputs

    oracle.build(force=False)
    w = inputs.dipole("mm", n=n, steps=sample_steps)
    P = oracle.Problem("mm", w.shape, sigma=w.sigma, currents=w.currents)
    f = oracle.init(P, *w.fields0())
    t0 = time.perf_counter()
    oracle.run(P, f, 0, sample_steps, probes=w.probes)
    dt = time.perf_counter() - t0
    del f
    one_steps = 2
    env = dict(os.environ, OMP_NUM_THREADS="1")
    res = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-sample", str(n), str(one_steps)],
                         capture_output=True, text=True, env=env, timeout=600)
    one = json.loads(res.stdout.strip().splitlines()[-1]) if res.returncode == 0 else None
    return {"value": round(w.n * sample_steps / dt / 1e6, 2), "unit": "MLUPS", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{sample_steps} steps of the {n}^3 MM dipole lattice, FP64, {dt:.1f} s",
            "single_thread": None if one is None else {"value": round(one["mlups"], 3), "unit": "MLUPS", "cores": 1,
                                                       "sample": f"{one_steps} steps of the same lattice, "
                                                                 f"{one['seconds']:.1f} s"}}


def oracle_sample(n: int, steps: int):
    """Child process of cpu_baseline: time `steps` oracle steps, print JSON."""
    import oracle
    from paper_2309_08068_amd import inputs

    w = inputs.dipole("mm", n=n, steps=steps)
    P = oracle.Problem("mm", w.shape, sigma=w.sigma, currents=w.currents)
    f = oracle.init(P, *w.fields0())
    t0 = time.perf_counter()
    oracle.run(P, f, 0, steps, probes=w.probes)
    dt = time.perf_counter() - t0
    print(json.dumps({"mlups": w.n * steps / dt / 1e6, "seconds": dt, "threads": oracle.threads()}), flush=True)


def stream_copy_gbs():
    """A plain device copy of 1 GiB (torch copy_): read + write bytes over its
    event-timed duration, the best of 5 launches."""
    import torch

    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    best = 1e30
    for _ in range(6):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return 2 * (1 << 30) / (best * 1e-3) / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256, help="lattice edge (the workload is n^3)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--only", default="", help="comma list of model_storage variants to time")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=5000)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=1500)
    ap.add_argument("--no-sweep", action="store_true", help="skip the 384^3 precision sweep")
    ap.add_argument("--no-radiation", action="store_true", help="skip the 256^3 radiation-pattern runs")
    ap.add_argument("--no-study", action="store_true", help="skip the refinement study of Section IV")
    ap.add_argument("--sweep-n", type=int, default=384)
    ap.add_argument("--sweep-steps", type=int, default=2000)
    ap.add_argument("--profile", action="store_true",
                    help="for rocprofv3 counter runs: only `steps` steps of the --only variants, then a plain "
                         "copy of 1 GiB (torch copy_) three times as the calibration kernel of known size")
    ap.add_argument("--oracle-sample", nargs=2, type=int, metavar=("N", "STEPS"),
                    help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_sample:
        oracle_sample(*args.oracle_sample)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding is a design note, "
              "not built", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    variants = [("mm", "f32"), ("mm", "bf16"), ("hv", "f32"), ("hv", "bf16"), ("mm", "bf16_shifted"),
                ("hv", "bf16_shifted"), ("mmd", "f32"), ("mmd", "bf16"), ("mmd", "bf16_shifted")]
    if args.only:
        keep = set(args.only.split(","))
        variants = [v for v in variants if f"{v[0]}_{v[1]}" in keep]
    if args.profile:
        from paper_2309_08068_amd import inputs, lbem
        if "batch" in args.only.split(","):
            bt = inputs.multilayer("mm", steps=args.steps)
            b = lbem.batch_from_inputs(bt)
            threads, gpc = b.autotune(10)
            b.step(64)
            torch.cuda.synchronize()
            print(f"# batch: launch {threads} x {gpc}, {b.blocking()} steps per pass; timed region = the last "
                  f"launch ({args.steps} steps)", file=sys.stderr, flush=True)
            b.step(args.steps)
            torch.cuda.synchronize()
            print(f"# profiled {args.steps} steps of the multilayer batch", file=sys.stderr, flush=True)
        for model, storage in variants:
            w = inputs.dipole(workload_model(model), n=args.n, steps=args.steps)
            lat = lbem.lattice_from_workload(w, storage=storage, model=model)
            lat.set_probes(w.probes, args.steps + 1)
            tuning = lat.autotune(10)
            torch.cuda.synchronize()
            print(f"# {model} {storage}: tuning {tuning}; timed region = the last {args.steps} step launches",
                  file=sys.stderr, flush=True)
            lat.step(args.steps)
            torch.cuda.synchronize()
            print(f"# profiled {args.steps} steps of {model} {storage}", file=sys.stderr, flush=True)
            del lat
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("# calibration copy: 1 GiB read + 1 GiB written per launch, 3 launches", file=sys.stderr, flush=True)
        return
    results = {}
    for model, storage in variants:
        r = time_variant(model, storage, args.n, args.steps, args.warmup)
        results[f"{model}_{storage}"] = r
        print(f"# {model} {storage}: {r['mlups']:.0f} MLUPS, step kernel {r['kernel_ms']:.3f} ms, "
              f"{r['achieved_gbs']:.0f} GB/s ({100 * r['frac']:.1f}% of peak), tuning {r['tuning']}",
              file=sys.stderr, flush=True)
    stream = stream_copy_gbs()
    print(f"# torch copy of 1 GiB: {stream:.0f} GB/s", file=sys.stderr, flush=True)
    head = results.get("mm_f32") or next(iter(results.values()))
    traffic = head["traffic"]
    line = {
        "metric": "MLUPS & %HBM peak, MM/HV 256^3 FP32 vs BF16 storage; adjoint/forward time",
        "value": round(head["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"hertz_dipole_{args.n}^3", "model": head["model"], "storage": head["storage"],
                   "cells": head["cells"], "sponge": 16, "source": "point J_z = sin(2 pi n / 40)",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(head["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(head["frac"], 4),
                     "traffic": None if traffic is None else round(traffic / 1e9 / (head["kernel_ms"] * 1e-3), 1),
                     "traffic_bytes_per_launch": traffic, "algorithmic_bytes_per_launch": head["bytes_per_lu"] * head["cells"],
                     "kernel": f"row_step_kernel<{head['model'].upper()}, {head['storage']}>",
                     "bytes_per_lu": head["bytes_per_lu"], "kernel_ms": round(head["kernel_ms"], 4),
                     "stream_copy_gbs": round(stream, 1), "frac_of_stream_copy": round(head["achieved_gbs"] / stream, 4)},
        # per variant: MLUPS, fraction of the HBM peak, step-kernel ms, measured traffic over algorithmic bytes
        "variants": {k: {"mlups": round(v["mlups"], 1), "frac": round(v["frac"], 4), "kernel_ms": round(v["kernel_ms"], 4),
                         "traffic_over_algorithmic": None if v["traffic"] is None else
                         round(v["traffic"] / (v["bytes_per_lu"] * v["cells"]), 4)}
                     for k, v in results.items()},
        "adjoint_over_forward": None,
    }
    if not args.no_batch:
        b = time_batch(args.batch_steps)
        print(f"# batched 1-D: {b}", file=sys.stderr, flush=True)
        line["batched_1d"] = {k: b[k] for k in ("workload", "launch", "steps_per_pass", "mlups",
                                               "frac_of_one_step_roofline", "one_step_per_pass_mlups",
                                               "one_step_per_pass_frac", "speedup_vs_per_instance")}
        line["batched_1d"]["alu_frac"] = b["roofline_blocked"]["frac"]
    if not args.no_adjoint:
        # keep = segments whose E frames the first forward holds: 1 is the
        # minimal-memory schedule (every other segment recomputed); 10 holds
        # 25 GB of frames for the 128 x 128 x 256 lattice, which 288 GB parts
        # afford.  The MM gradients come from the 50-population adjoint and,
        # at 24 / 50 of its traffic, from the difference form's adjoint; both
        # are reported against the 50-population MM forward.
        # On this lattice MM grows from about step 1050 (its oblique modes,
        # see the oracle's growth spectra), so MM is also timed over 1000
        # steps, where its energy stays at or below the pulse's.  Holding the
        # frames of every segment (75 GB for HV over 1500 steps, 50 GB for MM
        # over 1000) recomputes nothing.
        bounded = min(args.adjoint_steps, 1000)
        all_hv, all_mm = -(-args.adjoint_steps // 50), -(-bounded // 50)
        runs = []
        for model, steps, keep, fwd in (("hv", args.adjoint_steps, 1, None), ("hv", args.adjoint_steps, 10, None),
                                        ("hv", args.adjoint_steps, all_hv, None),
                                        ("mm", args.adjoint_steps, 10, None), ("mm", bounded, 10, None),
                                        ("mm", bounded, all_mm, None),
                                        ("mmd", bounded, 10, "mm"), ("mmd", bounded, 10, None),
                                        ("mmd", bounded, all_mm, "mm")):
            r = time_adjoint(model, steps, 50, keep, fwd)
            r["steps"] = steps
            print(f"# adjoint: {r}", file=sys.stderr, flush=True)
            runs.append(r)
        line["adjoint"] = [{k: r[k] for k in ("model", "forward_model", "steps", "keep", "forward_s", "adjoint_total_s",
                                                "ratio", "loss", "energy_max_over_initial", "growth_from_step", "check")}
                           for r in runs]
        pick = {(r["model"], r["forward_model"], r["steps"], r["keep"]): r["ratio"] for r in runs}
        line["adjoint_over_forward"] = {"hv": pick[("hv", "hv", args.adjoint_steps, 10)],
                                        "mm": pick[("mmd", "mm", bounded, 10)],
                                        "mm_50_populations": pick[("mm", "mm", bounded, 10)],
                                        "mmd": pick[("mmd", "mmd", bounded, 10)],
                                        "all_frames": {"hv": pick[("hv", "hv", args.adjoint_steps, all_hv)],
                                                       "mm": pick[("mmd", "mm", bounded, all_mm)],
                                                       "mm_50_populations": pick[("mm", "mm", bounded, all_mm)]},
                                        "workload": f"slab_128x128x256_K50_keep10, HV {args.adjoint_steps} steps, "
                                                    f"MM {bounded} (bounded; the MM gradient through the difference "
                                                    f"form over the 50-population MM forward); all_frames: every "
                                                    f"segment's frames held, nothing recomputed"}
    if not args.no_radiation:
        line["radiation_pattern"] = [radiation_pattern(m, args.n) for m in ("mm", "hv")]
        for r in line["radiation_pattern"]:
            print(f"# radiation: {r}", file=sys.stderr, flush=True)
    if not args.no_study:
        from paper_2309_08068_amd import study
        recs = study.study()
        main_err = {"interface": "reflected", "skin": "rms", "dipole": "cost_B", "layers": "peak"}
        summary = {}
        for r in recs:
            print(f"# study: {r}", file=sys.stderr, flush=True)
            e = summary.setdefault(r["experiment"], {"measure": main_err[r["experiment"]]})
            m = e.setdefault(r["model"], {"size": [], "error": [], "gpu_ms": []})
            m["size"].append(r["size"])
            m["error"].append(float(f"{float(r[main_err[r['experiment']]]):.4g}"))
            m["gpu_ms"].append(r["gpu_ms"])
        line["refinement_study"] = summary
    if not args.no_sweep:
        sweep = {}
        for m in ("mm", "hv"):
            res = time_precision(m, args.sweep_n, args.sweep_steps)
            sweep[m] = {st: [v["frac"], v.get("rel_l2_vs_f32", [0.0, 0.0])[0], v.get("rel_l2_E_r_ge_32", 0.0)]
                        for st, v in res["formats"].items()}
        line["precision_sweep"] = {"workload": f"hertz_dipole_{args.sweep_n}^3_{args.sweep_steps}steps",
                                   "fields": "storage: [fraction of HBM peak, rel L2 of E vs FP32 storage, "
                                             "the same over cells at least 32 from the source]", **sweep}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.n, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
