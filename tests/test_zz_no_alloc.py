"""lbem_adjoint_static, the adjoint entry point that allocates nothing, against
lbem_adjoint with a caller workspace: the same loss and gradients (the same
bits: both run the same kernels, and every launch form gives the same bits),
on two calls in a row, the second with a smaller lattice, and a problem too
large for the fixed workspace rejected before anything runs."""
import numpy as np
import pytest
import torch

from paper_2309_08068_amd import inputs, lbem

pytestmark = pytest.mark.gpu


def smooth_case(shape, seed):
    nx, ny, nz = shape
    u1 = inputs.smooth_field((nz, ny, nx), 2.0, seed).reshape(-1)
    u2 = inputs.smooth_field((nz, ny, nx), 2.0, seed + 1).reshape(-1)
    E0, B0 = inputs.gaussian_pulse(shape, nz * 0.25, 3.0, inputs.VACUUM_SPEED["mm"])
    return dict(eps=1.0 + 2.0 * u1, sig=0.05 * u2, E0=E0, B0=B0)


def run_both(model, shape, nsteps, K, keep, seed):
    d = smooth_case(shape, seed)
    det_z = shape[2] - 4
    out = []
    for static in (False, True):
        lat = lbem.Lattice(model, shape, d["eps"], None, d["sig"])
        lat.set_fields(d["E0"], d["B0"])
        if static:
            loss, ge, gs = lat.adjoint_static(nsteps, K, det_z, keep, d["E0"], d["B0"])
        else:
            ws = lat.adjoint_workspace(nsteps, K, keep)
            loss, ge, gs = lat.adjoint(nsteps, K, det_z, ws, keep, d["E0"], d["B0"])
        torch.cuda.synchronize()
        out.append((loss.clone(), ge.clone(), gs.clone(), lat.fields()[0].clone(), lat.time))
    return out


def test_static_adjoint_matches_workspace_adjoint():
    lib = lbem.load_library()
    assert lib.lbem_adjoint_static_bytes() == 64 << 20
    # first call: 32 x 32 x 48 HV, 80 steps (about 55 MB of the 64 MiB);
    # second: a smaller MM lattice, so the array holds the first call's data
    for model, shape, nsteps, K, keep, seed in (("hv", (32, 32, 48), 80, 20, 1, 3),
                                                 ("mm", (16, 16, 32), 40, 10, 2, 5)):
        print(f"case {model} {shape} {nsteps} steps", flush=True)
        (l0, ge0, gs0, E0, t0), (l1, ge1, gs1, E1, t1) = run_both(model, shape, nsteps, K, keep, seed)
        assert torch.isfinite(ge0).all() and ge0.abs().max() > 0
        assert torch.equal(l0, l1), (l0, l1)
        assert torch.equal(ge0, ge1) and torch.equal(gs0, gs1)
        # both leave the lattice where the forward left it
        assert t0 == t1 == nsteps and torch.equal(E0, E1)


def test_static_adjoint_rejects_large_problems():
    shape = (64, 64, 64)
    lat = lbem.Lattice("mm", shape)
    lat.set_fields(np.zeros((3, 64 ** 3)), np.zeros((3, 64 ** 3)))
    with pytest.raises(lbem.LbemError) as e:
        lat.adjoint_static(200, 50, 60)
    assert e.value.status == -2 and "fixed" in str(e.value)
    assert lat.time == 0
