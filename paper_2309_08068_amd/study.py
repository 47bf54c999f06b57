"""Refinement study of Section IV on the GPU: error against cost for the four
experiments of the paper, for each model, as the lattice is refined.

For every experiment and lattice size this runs the setup of
``inputs.study_*`` through the HIP library and reports the lattice size, the
steps, the GPU time of the stepping alone (HIP events on the library's
stream; initialisation and read-back excluded, as in the paper's timings),
the bytes of the distribution functions (the paper's memory measure) and the
errors against the closed forms the paper compares with:

* interface (Section IV-A): relative error of the reflected and transmitted
  amplitudes against the Fresnel coefficients (sqrt(r) - 1) / (sqrt(r) + 1)
  and 2 / (sqrt(r) + 1);
* skin (Section IV-B): the cost function eq. (cost), summed over the
  conductor cells, of the amplitude against A0 exp(-z / delta) with the skin
  thickness delta of the paper;
* dipole (Section IV-C): the same cost for the E and B amplitudes along a line
  perpendicular to the dipole moment, against the dipole fields of moment
  p = (J0 / omega) (pi / alpha)^1.5 (near and far terms);
* layers (Section IV-D): relative error of the transmitted pulse (peak and
  L2 over the last medium) against the exact transmitted field of the
  layered medium (transfer matrices per frequency, summed over the pulse's
  spectrum).

The closed forms and error measures are plain functions of numpy arrays, so
they apply to any stepper's output.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence

import numpy as np

from . import inputs

SIZES = {"interface": (250, 500, 1000, 2000), "skin": (500, 1000, 2000, 4000), "dipole": (48, 64, 96, 128),
         "layers": (500, 1000, 2000, 4000)}
BUILD = {"interface": inputs.study_interface, "skin": inputs.study_skin, "dipole": inputs.study_dipole,
         "layers": inputs.study_layers}
POPULATIONS = {"mm": 50, "hv": 36, "mmd": 24}


# ---------------------------------------------------------------- closed forms

def fresnel(r: float):
    """Reflected and transmitted amplitude ratios at normal incidence from
    vacuum into eps_r = r (mu_r = 1), as magnitudes (Section IV-A)."""
    s = math.sqrt(r)
    return (s - 1.0) / (s + 1.0), 2.0 / (s + 1.0)


def skin_depth(sigma: float, eps: float, mu: float, omega: float) -> float:
    """Skin thickness of a conductor with losses (Section IV-B)."""
    x = omega * eps / sigma
    return math.sqrt(2.0 / (sigma * mu * omega)) * math.sqrt(math.sqrt(1.0 + x * x) + x)


def dipole_amplitudes(r: np.ndarray, p: float, omega: float, eps0: float, mu0: float, c: float):
    """|E| and |B| of an oscillating point dipole p in its equatorial plane at
    distance r (near and far terms)."""
    k = omega / c
    E = p / (4.0 * math.pi * eps0) * np.abs(k * k / r - 1.0 / r ** 3 + 1j * k / r ** 2)
    B = mu0 * omega * k * p / (4.0 * math.pi * r) * np.sqrt(1.0 + 1.0 / (k * r) ** 2)
    return E, B


def stack_transmission(k: np.ndarray, eps: Sequence[float], bounds: Sequence[float]) -> np.ndarray:
    """Transmission amplitude t(k) of E from the first medium into the last
    through layers eps[1..-2] between the interfaces ``bounds`` (mu_r = 1,
    lossless), for vacuum wavenumbers k; the incident wave has amplitude 1 at
    the first interface and the transmitted one amplitude t at the last.
    Continuity of E and H at every interface, all multiple reflections."""
    n = np.sqrt(np.asarray(eps, dtype=np.float64))
    # in medium j: E = A e^{i k_j (z - b_j)} + B e^{-i k_j (z - b_j)}, H ~ n_j (A e^.. - B e^..)
    A = np.ones_like(k, dtype=np.complex128)   # last medium: transmitted wave only, at its interface
    B = np.zeros_like(k, dtype=np.complex128)
    for j in range(len(eps) - 1, 0, -1):
        # interface between medium j - 1 and j at bounds[j - 1]; (A, B) of medium j are referred to it
        e = A + B
        h = n[j] * (A - B)
        Am = 0.5 * (e + h / n[j - 1])
        Bm = 0.5 * (e - h / n[j - 1])
        if j - 1 > 0:
            # refer medium j - 1's amplitudes to its own left interface
            ph = np.exp(1j * n[j - 1] * k * (bounds[j - 1] - bounds[j - 2]))
            Am, Bm = Am / ph, Bm * ph
        A, B = Am, Bm
    return 1.0 / A


def layered_transmitted_field(z: np.ndarray, t: float, c: float, eps: Sequence[float], bounds: Sequence[float],
                              z_pulse: float, alpha: float, nk: int = 4096) -> np.ndarray:
    """E_x(z, t) for z beyond the last interface of the pulse
    exp(-(z - z_pulse)^2 / (2 alpha^2)) launched at t = 0 toward +z in the first
    medium (vacuum speed c): the sum over its spectrum of the transmitted
    plane waves."""
    kmax = 12.0 / alpha
    k = np.linspace(-kmax, kmax, nk)
    dk = k[1] - k[0]
    # spectrum of the pulse referred to the first interface
    G = alpha / math.sqrt(2.0 * math.pi) * np.exp(-0.5 * (alpha * k) ** 2) * np.exp(1j * k * (bounds[0] - z_pulse))
    tk = stack_transmission(k, eps, bounds)
    nN = math.sqrt(eps[-1])
    w = G * tk * dk * np.exp(-1j * c * k * t)
    out = np.empty(len(z))
    for i in range(0, len(z), 256):  # rows of the (z, k) phase matrix, in bounded blocks
        zz = np.asarray(z[i:i + 256], dtype=np.float64)
        out[i:i + 256] = np.real(np.exp(1j * nN * np.outer(zz - bounds[-1], k)) @ w)
    return out


# ---------------------------------------------------------------- error measures

def interface_errors(w, Ex: np.ndarray) -> Dict[str, float]:
    zi = w.meta["z_if"]
    r, tr = fresnel(w.meta["eps2"])
    A_ref = -Ex[:zi].min()  # the reflected pulse is inverted
    A_tr = Ex[zi:].max()
    return {"reflected": abs(A_ref - r) / r, "transmitted": abs(A_tr - tr) / tr}


def skin_cost(w, amplitude: np.ndarray, z: np.ndarray) -> Dict[str, float]:
    """eq. (cost) over the conductor cells z (amplitude per cell, last period)
    where the theoretical amplitude is at least 1e-3 of A0 (the amplitude at
    the conductor's face), and the root mean square of the per-cell relative
    errors it sums."""
    model = w.model
    eps0, mu0 = inputs.VACUUM_CONSTANTS[model]
    omega = 2.0 * math.pi / w.meta["period"]
    delta = skin_depth(w.meta["sigma"], eps0, mu0, omega)
    d = z - w.meta["z_c"]
    A0 = amplitude[d == 0][0]
    theo = A0 * np.exp(-d / delta)
    keep = (d >= 0) & (theo >= 1e-3 * A0)
    rel2 = ((amplitude[keep] - theo[keep]) / theo[keep]) ** 2
    # the cost is a sum over the cells, so it grows with their number; "rms"
    # is the per-cell relative error, which shows the convergence directly
    return {"cost": float(np.sum(rel2)), "rms": float(np.sqrt(np.mean(rel2))), "skin_depth": delta}


def dipole_cost(w, E_amp: np.ndarray, B_amp: np.ndarray) -> Dict[str, float]:
    model = w.model
    eps0, mu0 = inputs.VACUUM_CONSTANTS[model]
    c = inputs.VACUUM_SPEED[model]
    omega = 2.0 * math.pi / w.meta["period"]
    jsum = sum(cur[1][2] for cur in w.currents)
    Et, Bt = dipole_amplitudes(np.asarray(w.meta["radii"], dtype=np.float64), jsum / omega, omega, eps0, mu0, c)
    return {"cost_E": float(np.sum(((E_amp - Et) / Et) ** 2)), "cost_B": float(np.sum(((B_amp - Bt) / Bt) ** 2))}


def layers_errors(w, Ex: np.ndarray) -> Dict[str, float]:
    m = w.meta
    zN = m["bounds"][-1]
    z = np.arange(zN, w.shape[2], dtype=np.float64)
    theo = layered_transmitted_field(z, w.steps, inputs.VACUUM_SPEED[w.model], m["eps"], m["bounds"],
                                     m["z_pulse"], m["alpha"])
    sim = Ex[zN:]
    return {"peak": abs(sim.max() - theo.max()) / theo.max(),
            "l2": float(np.linalg.norm(sim - theo) / np.linalg.norm(theo))}


# ---------------------------------------------------------------- GPU runs

def run(experiment: str, model: str, size: int, storage: str = "f32") -> dict:
    """One experiment at one lattice size on the GPU (HIP library)."""
    import torch

    from . import lbem

    base = "mm" if model == "mmd" else model
    w = BUILD[experiment](base, size)
    lat = lbem.lattice_from_workload(w, storage=storage, model=model)
    series = None
    if experiment == "skin":
        L = w.meta["z_end"]
        zs = np.arange(w.meta["z_c"], L, max(1, (L - w.meta["z_c"]) // 4000 + 1))
        series = lat.set_probes(zs, w.steps)
    elif experiment == "dipole":
        series = lat.set_probes(w.probes, w.steps)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    lat.step(w.steps)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    out = {"experiment": experiment, "model": model, "size": size, "cells": w.n, "steps": w.steps,
           "gpu_ms": round(ms, 3), "dist_bytes": POPULATIONS[model] * w.n * (4 if storage == "f32" else 2)}
    if experiment in ("interface", "layers"):
        Ex = lat.fields()[0][0].double().cpu().numpy()
        out.update(interface_errors(w, Ex) if experiment == "interface" else layers_errors(w, Ex))
    elif experiment == "skin":
        T = int(round(w.meta["period"]))
        amp = series[-T:, :, 0].abs().max(dim=0).values.cpu().numpy()
        out.update(skin_cost(w, amp, zs))
    else:
        T = int(round(w.meta["period"]))
        s = series[-T:].abs().max(dim=0).values.cpu().numpy()
        out.update(dipole_cost(w, s[:, 2], s[:, 4]))
    del lat
    return out


def study(models=("mm", "hv"), experiments=("interface", "skin", "dipole", "layers"), sizes=None) -> List[dict]:
    """The whole refinement study; sizes: {experiment: sizes} overriding SIZES."""
    res = []
    for e in experiments:
        for m in models:
            for n in (sizes or {}).get(e, SIZES[e]):
                res.append(run(e, m, n))
    return res
