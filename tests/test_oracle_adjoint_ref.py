"""Pins of the FP64 automatic-differentiation reference used to check the
adjoint: its forward equals the C oracle, and its gradient equals central
finite differences of its own loss (FP64, second order)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import torch_ref as tr


def random_case(shape, seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    N = nx * ny * nz
    d = dict(eps=rng.uniform(1, 3, N), mu=rng.uniform(1, 2, N), sig=rng.uniform(0, 0.2, N),
             E0=rng.normal(size=(3, N)), B0=rng.normal(size=(3, N)))
    T = lambda a: torch.tensor(a.reshape(-1, nz, ny, nx) if a.ndim == 2 else a.reshape(nz, ny, nx))
    return d, {k: T(v) for k, v in d.items()}


LOSS = {"mm": tr.detector_loss, "hv": tr.hv_detector_loss}
FIELDS = {"mm": tr.fields, "hv": tr.hv_fields}


@pytest.mark.parametrize("model", ["mm", "hv"])
def test_torch_reference_equals_c_oracle(model):
    shape = (4, 3, 6)
    d, t = random_case(shape, 0)
    P = oracle.Problem(model, shape, eps_r=d["eps"], mu_r=d["mu"], sigma=d["sig"])
    f = oracle.init(P, d["E0"], d["B0"])
    out = oracle.run(P, f, 0, 7, det_z=2)
    E, B, _, _ = oracle.fields(P, f, 7)
    L, ft = LOSS[model](t["eps"], t["sig"], t["mu"], t["E0"], t["B0"], 7, 2)
    Et, Bt = FIELDS[model](ft, t["eps"], t["mu"], t["sig"])
    np.testing.assert_allclose(Et.numpy().reshape(3, -1), E, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(Bt.numpy().reshape(3, -1), B, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(L.item(), out["detector"].sum(), rtol=1e-12)


@pytest.mark.parametrize("model", ["mm", "hv"])
def test_torch_reference_gradient_equals_finite_differences(model):
    shape = (3, 2, 5)
    d, t = random_case(shape, 1)
    eps = t["eps"].clone().requires_grad_(True)
    sig = t["sig"].clone().requires_grad_(True)
    L, _ = LOSS[model](eps, sig, t["mu"], t["E0"], t["B0"], 6, 3)
    ge, gs = torch.autograd.grad(L, (eps, sig))
    h = 1e-5
    rng = np.random.default_rng(2)
    for _ in range(6):
        k = tuple(int(rng.integers(0, s)) for s in eps.shape)
        for g, which in ((ge, "eps"), (gs, "sig")):
            ap, am = t["eps"].clone(), t["eps"].clone()
            sp, sm = t["sig"].clone(), t["sig"].clone()
            if which == "eps":
                ap[k] += h
                am[k] -= h
            else:
                sp[k] += h
                sm[k] -= h
            Lp, _ = LOSS[model](ap, sp, t["mu"], t["E0"], t["B0"], 6, 3)
            Lm, _ = LOSS[model](am, sm, t["mu"], t["E0"], t["B0"], 6, 3)
            fd = (Lp - Lm).item() / (2 * h)
            assert abs(fd - g[k].item()) <= 1e-6 * max(1.0, abs(fd)), (which, k, fd, g[k].item())


def test_stored_slab_finite_differences_are_converged():
    """The stored central finite differences of the oracle's inverse-design
    loss (tests/golden/slab_fd_32x32x128.json): taken again with half the
    step on two cells they change by under 1e-5 relative, so their
    truncation error (O(h^2)) is far below the 1e-3 the GPU adjoint is held
    to; the 32 cells are distinct slab cells."""
    import json
    import os

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "slab_fd_32x32x128.json")
    with open(path) as fh:
        rec = json.load(fh)
    nx, ny, nz = rec["shape"]
    cells = rec["cells"]
    assert len(set(cells)) == 32
    assert all(rec["slab_z"][0] * nx * ny <= c < rec["slab_z"][1] * nx * ny for c in cells)
    for model in ("mm", "hv"):
        m = rec["models"][model]
        assert len(m["eps"]) == len(m["sigma"]) == 32
        for which in ("eps", "sigma"):
            for full, half in zip(m[which], m[which + "_half_h"]):
                assert abs(full - half) <= 1e-5 * abs(half), (model, which, full, half)
