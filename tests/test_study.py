"""Pins of the refinement-study analysis (closed forms the errors are measured
against) and the study's workloads run on the FP64 oracle: every error falls
as the lattice is refined (Sections IV-A to IV-D)."""
import math

import numpy as np
import pytest

import oracle
from paper_2309_08068_amd import inputs, study


def test_stack_transmission_reduces_to_known_cases():
    k = np.linspace(-2.0, 2.0, 41)
    # one interface: the Fresnel coefficient at every wavenumber
    np.testing.assert_allclose(study.stack_transmission(k, [1.0, 2.5], [7.0]), study.fresnel(2.5)[1], rtol=1e-14)
    # layers of the same medium are no interfaces at all: only the phase n k d
    # accumulated between the first and the last interface remains
    np.testing.assert_allclose(study.stack_transmission(k, [2.0, 2.0, 2.0], [0.0, 3.7]),
                               np.exp(1j * math.sqrt(2.0) * k * 3.7), rtol=1e-13)
    # a quarter-wave layer of index sqrt(n0 n2) transmits all the power: n2 |t|^2 = 1
    n2 = math.sqrt(3.0)
    n1 = math.sqrt(n2)
    lam = 40.0
    t = study.stack_transmission(np.array([2 * math.pi / lam]), [1.0, n1 ** 2, 3.0], [0.0, lam / (4 * n1)])
    assert abs(n2 * abs(t[0]) ** 2 - 1.0) < 1e-12
    # a half-wave layer is invisible: t equals the direct interface's up to phase
    t = study.stack_transmission(np.array([2 * math.pi / lam]), [1.0, 2.0, 3.0], [0.0, lam / (2 * math.sqrt(2.0))])
    assert abs(abs(t[0]) - 2.0 / (1.0 + n2)) < 1e-12


def test_transmitted_field_of_one_interface_is_the_compressed_pulse():
    """Across one interface the transmitted pulse is the incident one scaled by
    the Fresnel coefficient and compressed by the index."""
    c, n2 = 1.0 / math.sqrt(2.0), math.sqrt(2.5)
    z = np.arange(150.0, 300.0)
    E = study.layered_transmitted_field(z, 120.0, c, [1.0, 2.5], [150.0], 100.0, 5.0)
    exact = study.fresnel(2.5)[1] * np.exp(-((150.0 - 100.0) + (z - 150.0) * n2 - c * 120.0) ** 2 / 50.0)
    np.testing.assert_allclose(E, exact, atol=1e-10)


def test_skin_depth_and_dipole_limits():
    # good conductor: delta -> sqrt(2 / (sigma mu omega)); poor one: delta -> (2 / sigma) sqrt(eps / mu)
    assert abs(study.skin_depth(1e6, 1.0, 2.0, 1.0) / math.sqrt(2.0 / 2e6) - 1.0) < 1e-6
    assert abs(study.skin_depth(1e-6, 3.0, 3.0, 1.0) / (2.0 / 1e-6) - 1.0) < 1e-6
    # far field of the dipole: E = p k^2 / (4 pi eps0 r), B = E / c
    r = np.array([1e4])
    E, B = study.dipole_amplitudes(r, 2.0, 0.3, 1.0, 2.0, 1.0 / math.sqrt(2.0))
    k = 0.3 * math.sqrt(2.0)
    assert abs(E[0] / (2.0 * k * k / (4 * math.pi * 1e4)) - 1.0) < 1e-6
    assert abs(B[0] / (E[0] * math.sqrt(2.0)) - 1.0) < 1e-6


def oracle_errors(name, model, L):
    w = study.BUILD[name](model, L)
    P = oracle.Problem(model, w.shape, eps_r=w.eps_r, sigma=w.sigma, currents=w.currents, plane=w.plane)
    f = oracle.init(P, *w.fields0())
    if name == "skin":
        zs = np.arange(w.meta["z_c"], w.meta["z_end"])
        out = oracle.run(P, f, 0, w.steps, probes=list(zs))
        T = int(round(w.meta["period"]))
        return study.skin_cost(w, np.abs(out["probes"][-T:, :, 0]).max(axis=0), zs)
    if name == "dipole":
        out = oracle.run(P, f, 0, w.steps, probes=w.probes)
        T = int(round(w.meta["period"]))
        s = np.abs(out["probes"][-T:]).max(axis=0)
        return study.dipole_cost(w, s[:, 2], s[:, 4])
    oracle.run(P, f, 0, w.steps)
    Ex = oracle.fields(P, f, w.steps)[0][0]
    return study.interface_errors(w, Ex) if name == "interface" else study.layers_errors(w, Ex)


@pytest.mark.parametrize("model", ["mm", "hv"])
@pytest.mark.parametrize("name,sizes", [("interface", (250, 500)), ("layers", (250, 500)), ("skin", (500, 1000)),
                                        ("dipole", (32, 48))])
def test_study_errors_fall_under_refinement_on_the_oracle(name, model, sizes):
    coarse, fine = (oracle_errors(name, model, L) for L in sizes)
    print(name, model, coarse, fine, flush=True)
    for key, v in coarse.items():
        if key == "skin_depth":
            continue
        assert np.isfinite(v) and fine[key] < v, (key, v, fine[key])
