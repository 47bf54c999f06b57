"""Write slab_fd_32x32x128.json: central finite differences of the FP64
oracle's detector loss with respect to eps_r and sigma of single cells, on the
inverse-design lattice scaled to 32 x 32 x 128, for MM (300 steps) and HV
(600 steps).  MM's run is shorter because on this lattice the scheme's own
float32 rounding grows (its float32 build departs from the float64 one by
1.4e-5 of the largest field after 200 steps, 1.8e-3 after 400 and 1.2e-1
after 600), which would swamp any FP32 adjoint; the transmitted pulse has
crossed the detector plane by step 120.

The inverse-design problem: smooth random eps_r in [1, 4] and sigma in
[0, 0.02] over a slab tapered to the background, a plane-wave pulse, and the
loss L = sum over the collided states of sum over the detector plane of
|E|^2.  The cells are 32 draws of numpy's default_rng(2) among the slab's
cells (each a separate cell).  Each derivative is (L(theta + h) -
L(theta - h)) / (2 h) with h = 1e-3 for eps_r and 1e-5 for sigma; on the
first two cells it is also taken with h / 2, and both values are stored, so
that the truncation error can be read off (it falls by 4 when h halves).

Calls only the oracle and the seeded input generator.  Run from the
repository root:  python tests/golden/make_slab_fd.py [mm] [hv]
(about 40 minutes on 8 cores for both)."""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2309_08068_amd import inputs  # noqa: E402

SHAPE = (32, 32, 128)
SLAB_Z = (48, 80)
STEPS = {"mm": 300, "hv": 600}
H = {"eps": 1e-3, "sigma": 1e-5}
N_CELLS = 32
OUT = os.path.join(HERE, "slab_fd_32x32x128.json")


def workload(model):
    return inputs.slab(model, shape=SHAPE, slab_z=SLAB_Z, pulse_z=28.0, pulse_width=6.0, det_z=112, sponge=8,
                       steps=STEPS[model], seed=0)


def cells():
    nx, ny, _ = SHAPE
    first, last = SLAB_Z[0] * nx * ny, SLAB_Z[1] * nx * ny
    return [int(c) for c in np.random.default_rng(2).choice(np.arange(first, last), N_CELLS, replace=False)]


def loss(w, eps, sig):
    P = oracle.Problem(w.model, w.shape, eps_r=eps, sigma=sig)
    f = oracle.init(P, *w.fields0())
    return float(oracle.run(P, f, 0, w.steps, det_z=w.det_z)["detector"].sum())


def central(w, cell, which, h):
    vals = []
    for sgn in (1.0, -1.0):
        eps, sig = w.eps_r.copy(), w.sigma.copy()
        (eps if which == "eps" else sig)[cell] += sgn * h
        vals.append(loss(w, eps, sig))
    return (vals[0] - vals[1]) / (2 * h)


def main(models=("mm", "hv")):
    """Compute the models given on the command line (default both); models
    not computed keep their entries from an existing file."""
    out = {"_about": __doc__.split("\n\n")[0].replace("\n", " "), "shape": SHAPE, "slab_z": SLAB_Z,
           "steps": STEPS, "h": H, "cells": cells(), "models": {}}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            old = json.load(fh)
        for m, rec in old["models"].items():
            if m not in models and rec.get("steps") == STEPS[m]:
                out["models"][m] = rec
    for model in models:
        w = workload(model)
        t0 = time.time()
        rec = {"steps": w.steps, "loss": loss(w, w.eps_r, w.sigma), "eps": [], "sigma": [], "eps_half_h": [],
               "sigma_half_h": []}
        for k, cell in enumerate(out["cells"]):
            for which in ("eps", "sigma"):
                rec[which].append(central(w, cell, which, H[which]))
                if k < 2:
                    rec[which + "_half_h"].append(central(w, cell, which, H[which] / 2))
            print(f"{model} cell {k} ({cell}): d/deps {rec['eps'][-1]:.10e} d/dsigma {rec['sigma'][-1]:.10e} "
                  f"[{time.time() - t0:.0f} s]", flush=True)
        out["models"][model] = rec
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main(tuple(sys.argv[1:]) or ("mm", "hv"))
