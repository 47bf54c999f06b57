"""GPU adjoint (hand-written reverse-time kernels behind a torch.autograd.Function)
against the FP64 automatic-differentiation reference and against central finite
differences of the GPU's own forward loss.  The MM scheme in difference form
("mmd") has the loss, and so the gradients, of the full MM scheme."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import torch_ref as tr
from paper_2309_08068_amd import inputs, lbem
from paper_2309_08068_amd.adjoint import DetectorProblem, detector_energy
from parity import check, elem, rel

pytestmark = pytest.mark.gpu


def smooth_case(shape, seed, slab=None):
    """Random but smooth media (so that the loss is well conditioned) and a pulse."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    N = nx * ny * nz
    u1 = inputs.smooth_field((nz, ny, nx), 2.0, seed).reshape(-1)
    u2 = inputs.smooth_field((nz, ny, nx), 2.0, seed + 1).reshape(-1)
    eps = 1.0 + 2.0 * u1
    sig = 0.05 * u2
    mu = 1.0 + 0.5 * inputs.smooth_field((nz, ny, nx), 2.0, seed + 2).reshape(-1)
    E0, B0 = inputs.gaussian_pulse(shape, nz * 0.25, 3.0, inputs.VACUUM_SPEED["mm"])
    E0 = E0 + 0.1 * rng.normal(size=E0.shape)
    return dict(eps=eps, sig=sig, mu=mu, E0=E0, B0=B0)


def autodiff(shape, d, nsteps, det_z, model="mm"):
    nx, ny, nz = shape
    T = lambda a: torch.tensor(a.reshape(-1, nz, ny, nx) if a.ndim == 2 else a.reshape(nz, ny, nx))
    eps = T(d["eps"]).requires_grad_(True)
    sig = T(d["sig"]).requires_grad_(True)
    loss = tr.hv_detector_loss if model == "hv" else tr.detector_loss
    L, _ = loss(eps, sig, T(d["mu"]), T(d["E0"]), T(d["B0"]), nsteps, det_z)
    ge, gs = torch.autograd.grad(L, (eps, sig))
    return L.item(), ge.numpy().reshape(-1), gs.numpy().reshape(-1)


def gpu_grad(shape, d, nsteps, det_z, K, model="mm", keep=1):
    dev = torch.device("cuda")
    eps = torch.tensor(d["eps"], device=dev, requires_grad=True)
    sig = torch.tensor(d["sig"], device=dev, requires_grad=True)
    prob = DetectorProblem(shape, torch.tensor(d["E0"], device=dev, dtype=torch.float32),
                           torch.tensor(d["B0"], device=dev, dtype=torch.float32), nsteps, det_z, K,
                           torch.tensor(d["mu"], device=dev, dtype=torch.float32), model, keep)
    L = detector_energy(eps, sig, prob)
    L.backward()
    return L.item(), eps.grad.cpu().numpy(), sig.grad.cpu().numpy()


@pytest.mark.parametrize("model", ["mm", "hv", "mmd"])
def test_default_keep_holds_every_frame_and_matches_keep_one(model):
    """DetectorProblem's default keep (0) holds as many segments of frames as
    half the free device memory allows (every one, on this lattice), so the
    backward recomputes nothing; the loss and gradients are those of keep = 1,
    whose backward recomputes all but the last segment."""
    shape, nsteps, K = (128, 3, 10), 23, 5
    d = smooth_case(shape, 8)
    res = [gpu_grad(shape, d, nsteps, shape[2] - 3, K, model, keep) for keep in (0, 1)]
    assert res[0][0] == res[1][0]
    for a, b in zip(res[0][1:], res[1][1:]):
        assert np.array_equal(a, b)
    lat = lbem.Lattice(model, shape)
    assert lat.adjoint_keep(nsteps, K, torch.cuda.mem_get_info()[0] // 2) == -(-nsteps // K)


@pytest.mark.parametrize("model", ["mm", "hv", "mmd"])
@pytest.mark.parametrize("shape,nsteps,K,keep", [((6, 5, 16), 40, 7, 1), ((6, 5, 16), 41, 41, 1),
                                                 ((6, 5, 16), 40, 7, 3), ((6, 5, 16), 40, 7, 6),
                                                 ((128, 2, 12), 25, 4, 2), ((256, 1, 6), 17, 5, 1),
                                                 ((128, 1, 520), 12, 5, 1), ((200, 2, 12), 15, 4, 1),
                                                 ((300, 1, 100), 12, 5, 2)])
def test_adjoint_matches_fp64_autodiff(model, shape, nsteps, K, keep):
    """Gradients w.r.t. eps_r and sigma of every cell, including the dependence
    of the equilibrium initial state on eps_r; uneven last segment, a single
    segment, the row form of the recomputed forward and of the adjoint, and a
    lattice of two layout chunks (520 x-rows of 128 cells)."""
    det_z = shape[2] - 4
    d = smooth_case(shape, 5)
    L_ref, ge_ref, gs_ref = autodiff(shape, d, nsteps, det_z, model)
    L, ge, gs = gpu_grad(shape, d, nsteps, det_z, K, model, keep)
    print(f"{shape} {nsteps}/{K}: loss {L:.6e} vs {L_ref:.6e}; rel err grad eps {rel(ge, ge_ref):.2e} "
          f"(element-wise {elem(ge, ge_ref):.2e}) sigma {rel(gs, gs_ref):.2e} (element-wise {elem(gs, gs_ref):.2e})",
          flush=True)
    assert abs(L - L_ref) <= 1e-5 * abs(L_ref)
    check(ge, ge_ref, 1e-4, 1e-4, "dL/deps_r")
    check(gs, gs_ref, 1e-4, 1e-4, "dL/dsigma")


def test_adjoint_leaves_forward_state():
    shape = (6, 5, 16)
    d = smooth_case(shape, 9)
    lat = lbem.Lattice("mm", shape, d["eps"], d["mu"], d["sig"])
    lat.set_fields(d["E0"], d["B0"])
    ws = lat.adjoint_workspace(30, 8, 2)
    lat.adjoint_forward(30, 8, 10, ws)
    E1 = lat.fields()[0].clone()
    lat.adjoint_backward(ws)
    assert lat.time == 30
    assert torch.equal(lat.fields()[0], E1)


@pytest.mark.parametrize("model", ["mm", "hv", "mmd"])
def test_one_call_adjoint_equals_two_passes(model):
    """lbem_adjoint gives the bits of lbem_adjoint_forward + lbem_adjoint_backward."""
    shape = (128, 3, 12)
    d = smooth_case(shape, 4)
    out = []
    for one_call in (False, True):
        lat = lbem.Lattice(model, shape, d["eps"], d["mu"], d["sig"])
        lat.set_fields(d["E0"], d["B0"])
        ws = lat.adjoint_workspace(30, 7, 2)
        if one_call:
            loss, ge, gs = lat.adjoint(30, 7, 8, ws, 2, d["E0"], d["B0"])
        else:
            loss = lat.adjoint_forward(30, 7, 8, ws, 2)
            ge, gs = lat.adjoint_backward(ws, d["E0"], d["B0"])
        out.append((loss.clone(), ge.clone(), gs.clone()))
    for a, b in zip(*out):
        assert torch.equal(a, b)


@pytest.mark.parametrize("model,shape", [("hv", (128, 1, 520)), ("mm", (128, 1, 520)), ("mmd", (128, 1, 520)),
                                         ("hv", (200, 1, 300)), ("mm", (300, 2, 40))])
def test_adjoint_launch_forms_are_bit_identical(model, shape):
    """Every launch form of the adjoint kernel (LDS x-shifts with early or late
    store addresses, direct addressing), per parity, gives the same bits, twice
    in a row, on a lattice of two layout chunks (also with rows shorter than
    their block); the automatic choice too."""
    nsteps, K = 12, 5
    d = smooth_case(shape, 5)
    ref = None
    for form in ((0, 0), (1, 1), (2, 2), (0, 2), (2, 0), (1, 0), None, (0, 0)):
        lat = lbem.Lattice(model, shape, d["eps"], d["mu"], d["sig"])
        if form is not None:
            lat.set_adjoint_tuning(form, (0, 0))
        lat.set_fields(d["E0"], d["B0"])
        ws = lat.adjoint_workspace(nsteps, K, 1)
        _, ge, gs = lat.adjoint(nsteps, K, shape[2] - 4, ws, 1, d["E0"], d["B0"])
        if form is None:
            assert all(f in (0, 1, 2) for f in lat.adjoint_tuning()[0])
        if ref is None:
            ref = (ge.clone(), gs.clone())
        assert torch.equal(ge, ref[0]) and torch.equal(gs, ref[1]), form


def test_adjoint_rejects_sources_and_bad_arguments():
    lat = lbem.Lattice("hv", (4, 4, 4))
    ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    with pytest.raises(lbem.LbemError) as e:
        lat.adjoint_forward(4, 2, 1, ws)
    assert e.value.status == -2
    with pytest.raises(lbem.LbemError):
        lat.adjoint_forward(4, 2, 9, lat.adjoint_workspace(4, 2))
    lat = lbem.Lattice("mm", (4, 4, 4))
    lat.set_current_source([3], [[0, 0, 1]], 10.0)
    ws = lat.adjoint_workspace(4, 2)
    with pytest.raises(lbem.LbemError) as e:
        lat.adjoint_forward(4, 2, 1, ws)
    assert e.value.status == -5
    lat2 = lbem.Lattice("mm", (4, 4, 4))
    with pytest.raises(lbem.LbemError):
        lat2.adjoint_backward(ws)


def base(model):
    return "mm" if model == "mmd" else model


def oracle_loss(model, shape, eps, sig, E0, B0, nsteps, det_z):
    P = oracle.Problem(base(model), shape, eps_r=eps, sigma=sig)
    f = oracle.init(P, E0, B0)
    return oracle.run(P, f, 0, nsteps, det_z=det_z)["detector"].sum()


@pytest.mark.parametrize("model", ["mm", "hv", "mmd"])
def test_inverse_design_gradient_finite_differences(model):
    """The inverse-design lattice (smooth random eps_r in [1, 4] and sigma in
    [0, 0.02] over a tapered slab, plane-wave pulse, detector plane,
    checkpoint every 50 steps) at 32 x 32 x 128 for 600 steps: the GPU adjoint's
    directional derivatives against central finite differences of the FP64
    oracle's loss (the GPU's own FP32 loss is too noisy for a 1e-3 check at a
    usable step; its loss is compared with the oracle's instead)."""
    w = inputs.slab(base(model), shape=(32, 32, 128), slab_z=(48, 80), pulse_z=28.0, pulse_width=6.0, det_z=112,
                    sponge=8, steps=600, seed=0)
    shape = w.shape
    E0, B0 = w.fields0()
    dev = torch.device("cuda")
    eps_t = torch.tensor(w.eps_r, device=dev, requires_grad=True)
    sig_t = torch.tensor(w.sigma, device=dev, requires_grad=True)
    prob = DetectorProblem(shape, torch.tensor(E0, device=dev, dtype=torch.float32),
                           torch.tensor(B0, device=dev, dtype=torch.float32), w.steps, w.det_z, 50, model=model,
                           keep=3)
    L = detector_energy(eps_t, sig_t, prob)
    L.backward()
    ge, gs = eps_t.grad.cpu().numpy(), sig_t.grad.cpu().numpy()
    L64 = oracle_loss(model, shape, w.eps_r, w.sigma, E0, B0, w.steps, w.det_z)
    print(f"{model} loss: GPU {L.item():.8e} oracle {L64:.8e}", flush=True)
    assert abs(L.item() - L64) <= 1e-5 * abs(L64)
    # directions supported on the slab, weighted so that eps_r >= 1 and
    # sigma >= 0 hold for the perturbed media
    nz, ny, nx = 128, 32, 32
    u = np.zeros((nz, ny, nx))
    u[48:80] = inputs.smooth_field((32, ny, nx), 3.0, 11) - 0.5
    u = u.reshape(-1)
    h = 1e-3
    for g, which in ((ge, "eps"), (gs, "sigma")):
        if which == "eps":
            dirn = u * (w.eps_r - 1.0)
            Lp = oracle_loss(model, shape, w.eps_r + h * dirn, w.sigma, E0, B0, w.steps, w.det_z)
            Lm = oracle_loss(model, shape, w.eps_r - h * dirn, w.sigma, E0, B0, w.steps, w.det_z)
        else:
            dirn = u * w.sigma * (w.sigma <= 0.02)
            Lp = oracle_loss(model, shape, w.eps_r, w.sigma + h * dirn, E0, B0, w.steps, w.det_z)
            Lm = oracle_loss(model, shape, w.eps_r, w.sigma - h * dirn, E0, B0, w.steps, w.det_z)
        fd = (Lp - Lm) / (2 * h)
        ad = float(g @ dirn)
        print(f"{model} directional {which}: adjoint {ad:.6e} finite difference {fd:.6e}", flush=True)
        assert abs(ad - fd) <= 1e-3 * abs(fd)


SLAB_FD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "slab_fd_32x32x128.json")


@pytest.mark.parametrize("model", ["mm", "hv", "mmd"])
def test_inverse_design_per_cell_finite_differences(model):
    """The inverse-design lattice at 32 x 32 x 128 (the largest size at which
    the 256 FP64 oracle runs of the check fit in an hour of 8 host cores;
    stored by tests/golden/make_slab_fd.py, which calls only the oracle) for
    600 steps (HV) or 300 (MM: on this lattice the scheme's own float32
    rounding grows past 1e-3 of the field by step 400, see the script), at
    each of 32 cells drawn with default_rng(2) among the slab's
    cells, the GPU adjoint's dL/deps_r and dL/dsigma must be within 1e-3 of
    the central finite difference of the oracle's loss, relative to the
    gradient's scale (the largest |FD| over the 32 cells).  A cell's own
    gradient can be far below that scale where contributions of the 600 steps
    cancel; there the FP32 forward fields and adjoint populations set the
    error, not the adjoint's arithmetic, so the per-cell relative errors are
    printed, not bounded.  The difference form is held to the MM values (the
    same loss)."""
    with open(SLAB_FD) as fh:
        rec = json.load(fh)
    fd = rec["models"][base(model)]
    w = inputs.slab(base(model), shape=tuple(rec["shape"]), slab_z=tuple(rec["slab_z"]), pulse_z=28.0,
                    pulse_width=6.0, det_z=112, sponge=8, steps=fd["steps"], seed=0)
    E0, B0 = w.fields0()
    dev = torch.device("cuda")
    eps_t = torch.tensor(w.eps_r, device=dev, requires_grad=True)
    sig_t = torch.tensor(w.sigma, device=dev, requires_grad=True)
    prob = DetectorProblem(w.shape, torch.tensor(E0, device=dev, dtype=torch.float32),
                           torch.tensor(B0, device=dev, dtype=torch.float32), w.steps, w.det_z, 50, model=model,
                           keep=3)
    L = detector_energy(eps_t, sig_t, prob)
    L.backward()
    assert abs(L.item() - fd["loss"]) <= 1e-5 * abs(fd["loss"])
    cells = np.asarray(rec["cells"])
    for which, g in (("eps", eps_t.grad.cpu().numpy()), ("sigma", sig_t.grad.cpu().numpy())):
        ref = np.asarray(fd[which])
        scale = np.abs(ref).max()
        err = np.abs(g[cells] - ref) / scale
        own = np.abs(g[cells] - ref) / np.abs(ref)
        print(f"{model} dL/d{which} at 32 cells: largest difference from FD {err.max():.2e} of the scale "
              f"{scale:.3e}; relative to each cell's own value: median {np.median(own):.2e}, largest "
              f"{own.max():.2e} (at a cell whose |FD| is {np.abs(ref[np.argmax(own)]) / scale:.2e} of the scale)",
              flush=True)
        assert np.all(err <= 1e-3), (which, cells[err > 1e-3], err[err > 1e-3])
