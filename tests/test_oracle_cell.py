"""Pins of the oracle's single-cell pieces: vector tables, equilibria, source term,
collision.  Each check is a consequence the paper or plain geometry fixes, so a
mistyped table entry, coefficient or sign in the oracle fails one of them."""
import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
RNG = np.random.default_rng(1234)


def levi_civita():
    e = np.zeros((3, 3, 3))
    for (a, b, c), s in {(0, 1, 2): 1, (1, 2, 0): 1, (2, 0, 1): 1, (0, 2, 1): -1, (2, 1, 0): -1, (1, 0, 2): -1}.items():
        e[a, b, c] = s
    return e


def test_population_counts_match_paper():
    assert oracle.NQ["mm"] == GOLDEN["mm_populations_per_cell"]["value"]
    assert oracle.NQ["hv"] == GOLDEN["hv_populations_per_cell"]["value"]
    assert oracle._lib().oracle_nq(0) == 50 and oracle._lib().oracle_nq(1) == 36
    g = GOLDEN["mm_distribution_functions_4000_cells"]
    assert oracle.NQ["mm"] * g["cells"] == g["value"]
    g = GOLDEN["hv_distribution_functions_3000_cells"]
    assert oracle.NQ["hv"] * g["cells"] == g["value"]


def test_mm_velocity_set_geometry():
    """eq. (VelocitySetMiller): 12 distinct face diagonals of the cube, |v|^2 = 2,
    plane p = 0, 1, 2 holds the vectors with zero z, y, x component."""
    v, e, b = oracle.mm_tables()
    flat = v.reshape(12, 3)
    assert len({tuple(r) for r in flat}) == 12
    np.testing.assert_array_equal((flat ** 2).sum(1), 2.0)
    for p, zero_axis in ((0, 2), (1, 1), (2, 0)):
        assert np.all(v[p, :, zero_axis] == 0)
    # directions i and i+2 are opposite (used for the opposite-slot pairing)
    np.testing.assert_array_equal(v[:, 0], -v[:, 2])
    np.testing.assert_array_equal(v[:, 1], -v[:, 3])


def test_mm_vector_sums():
    """Sum relations of the MM vectors (the 'appropriate sum relations' of
    Section II): zero first moments, isotropic second moments, and the
    Levi-Civita triple moment that carries the curl."""
    v, e, b = oracle.mm_tables()
    V = np.repeat(v[:, :, None, :], 2, axis=2).reshape(24, 3)  # v for every (p, i, j)
    Ev, Bv = e.reshape(24, 3), b.reshape(24, 3)
    for X in (V, Ev, Bv):
        np.testing.assert_allclose(X.sum(0), 0, atol=1e-15)
    np.testing.assert_allclose(Ev.T @ Ev, 4 * np.eye(3), atol=1e-15)
    np.testing.assert_allclose(Bv.T @ Bv, 8 * np.eye(3), atol=1e-15)
    np.testing.assert_allclose(V.T @ V, 16 * np.eye(3), atol=1e-15)
    for X, Y in ((Bv, Ev), (V, Ev), (V, Bv)):
        np.testing.assert_allclose(X.T @ Y, 0, atol=1e-15)
    T = np.einsum("qa,qb,qc->abc", V, Ev, Bv)
    np.testing.assert_allclose(T, 4 * levi_civita(), atol=1e-15)
    # e_{i1} = -e_{i0}, b = v x e, e perpendicular to v, |e|^2 = 1/2
    np.testing.assert_array_equal(e[:, :, 1], -e[:, :, 0])
    np.testing.assert_allclose(b, np.cross(v[:, :, None, :], e), atol=1e-15)
    np.testing.assert_allclose(np.einsum("pia,pija->pij", v, e), 0, atol=1e-15)
    np.testing.assert_allclose((e ** 2).sum(-1), 0.5)


def test_hv_velocity_second_moment():
    """eq. (Correct): sum_i v_i v_i^T = 2 I; the six axis directions."""
    V = np.array([oracle.velocity("hv", 3 * i) for i in range(6)], dtype=float)
    np.testing.assert_allclose(V.T @ V, GOLDEN["hv_velocity_second_moment"]["value"] * np.eye(3))
    np.testing.assert_allclose(V.sum(0), 0)
    assert len({tuple(r) for r in V}) == 6
    # v5 = -z and v6 = +z as printed
    np.testing.assert_array_equal(V[4], [0, 0, -1])
    np.testing.assert_array_equal(V[5], [0, 0, 1])


@pytest.mark.parametrize("trial", range(5))
def test_mm_equilibrium_moments(trial):
    """The moments of eq. (equilibriumsMiller) return the fields they were built
    from: sum f(0)eq e = eps_r E, sum f(1)eq b = B, sum f(r)eq v = J, the moving
    r = 0 populations carry no charge and the rest ones carry rho_c."""
    v, e, b = oracle.mm_tables()
    V = np.repeat(v[:, :, None, :], 2, axis=2).reshape(24, 3)
    E, B, J = RNG.normal(size=(3, 3))
    rho, er, mr = RNG.normal(), RNG.uniform(1, 4), RNG.uniform(1, 4)
    feq = oracle.equilibrium("mm", E, B, J, rho, er, mr)
    r0, r1 = feq[:24], feq[24:48]
    np.testing.assert_allclose(r0 @ e.reshape(24, 3), er * E, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(r1 @ b.reshape(24, 3), B, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(r0 @ V, J, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(r1 @ V, J, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(r0 @ b.reshape(24, 3), B / mr, rtol=1e-13, atol=1e-13)
    assert abs(r0.sum()) < 1e-13
    assert feq[48] == rho and feq[49] == rho


@pytest.mark.parametrize("trial", range(5))
def test_hv_equilibrium_moments_and_source(trial):
    """eq. (equilibriumHV): sum e_eq = D, sum h_eq = B, the first moments are the
    curl fluxes; Appendix A: sum_i T_i = -J."""
    E, B, J = RNG.normal(size=(3, 3))
    er, mr = RNG.uniform(1, 4), RNG.uniform(1, 4)
    feq = oracle.equilibrium("hv", E, B, J, 0.0, er, mr).reshape(2, 6, 3)
    eps, mu = 3 * er, 3 * mr
    np.testing.assert_allclose(feq[0].sum(0), eps * E, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(feq[1].sum(0), B, rtol=1e-13, atol=1e-13)
    V = np.array([oracle.velocity("hv", 3 * i) for i in range(6)], dtype=float)
    # flux tensors Pi_ab = sum_i v_ia f_ib: +eps_abd H_d for e and -eps_abd E_d for h,
    # whose divergences are the curls of Faraday's and Ampere's laws
    lc = levi_civita()
    np.testing.assert_allclose(V.T @ feq[0], np.einsum("abd,d->ab", lc, B / mu), atol=1e-13)
    np.testing.assert_allclose(V.T @ feq[1], -np.einsum("abd,d->ab", lc, E), atol=1e-13)
    T = oracle.hv_source(J)
    np.testing.assert_allclose(T.sum(0), -J, rtol=1e-14, atol=1e-14)
    # T_i is along v_i
    np.testing.assert_allclose(np.cross(T, V), 0, atol=1e-15)


@pytest.mark.parametrize("model", ["mm", "hv"])
def test_collision_is_involution_without_current(model):
    """With tau = 1/2 and no current, C(f) = 2 f_eq(m(f)) - f and the moments of
    C(f) equal those of f_eq, so C applied twice returns f exactly."""
    Q = oracle.NQ[model]
    for _ in range(5):
        f = RNG.normal(size=Q)
        er, mr = RNG.uniform(1, 3), RNG.uniform(1, 3)
        f1, E1, B1, J1 = oracle.collide(model, f, er, mr, 0.0)
        f2, E2, B2, J2 = oracle.collide(model, f1, er, mr, 0.0)
        np.testing.assert_allclose(f2, f, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(E2, E1, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(B2, B1, rtol=1e-12, atol=1e-12)


def test_mm_uniform_current_drains_displacement():
    """A spatially uniform state is not changed by streaming, so one collision
    must change D' by exactly -J (Ampere-Maxwell with curl H = 0), and the
    physical eps_r E must be D' - mu0 J / 4 (eq. MacroscopicEMiller), the mean of
    D' before and after.  Pins the mu0 / 4 correction, the ohmic denominator of
    eq. (MacorscopicCurrentMiller) and the v.J / 16 term together."""
    _, e, _ = oracle.mm_tables()
    f = RNG.normal(size=50)
    for er, sg in ((1.0, 0.0), (2.5, 0.0), (1.7, 0.3)):
        Jsrc = RNG.normal(size=3)
        f1, E, B, J = oracle.collide("mm", f, er, 1.3, sg, Jsrc)
        D0 = f[:24] @ e.reshape(24, 3)
        D1 = f1[:24] @ e.reshape(24, 3)
        np.testing.assert_allclose(J, sg * E + Jsrc, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(D0 - er * E, J / 2, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(D1 - D0, -J, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(er * E, 0.5 * (D0 + D1), rtol=1e-12, atol=1e-12)


def test_hv_uniform_current_drains_displacement():
    """Same for HV: one collision with T changes D by exactly -J."""
    f = RNG.normal(size=36)
    for er, sg in ((1.0, 0.0), (2.0, 0.2)):
        Jsrc = RNG.normal(size=3)
        f1, E, B, J = oracle.collide("hv", f, er, 1.0, sg, Jsrc)
        D0 = f.reshape(2, 6, 3)[0].sum(0)
        D1 = f1.reshape(2, 6, 3)[0].sum(0)
        np.testing.assert_allclose(D1 - D0, -J, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(J, sg * D0 / (3 * er) + Jsrc, rtol=1e-12, atol=1e-12)
