"""Pins of the oracle's lattice stepper: exact Fourier propagation on homogeneous
periodic lattices, the stability limits the paper states, and the behaviour of
the global operator at interfaces."""
import math

import numpy as np
import pytest

import oracle
from paper_2309_08068_amd import inputs

RNG = np.random.default_rng(99)


def collision_matrix(model, er, mr, sg):
    Q = oracle.NQ[model]
    C = np.zeros((Q, Q))
    for k in range(Q):
        u = np.zeros(Q)
        u[k] = 1.0
        C[:, k] = oracle.collide(model, u, er, mr, sg)[0]
    return C


def amplification(model, C, k):
    """A(k) = diag(exp(-i k . v_q)) C: one step of f(x + v_q) <- C f(x) in Fourier space."""
    V = oracle.velocities(model).astype(float)
    return np.exp(-1j * (V @ k))[:, None] * C


@pytest.mark.parametrize("model", ["mm", "hv"])
def test_exact_fourier_propagation(model):
    """On a homogeneous periodic lattice the scheme is a convolution: after n
    steps every Fourier mode equals A(k)^n applied to the initial mode.  Checks
    the advection direction, the periodic wrap on odd sizes and the cell order."""
    shape = (4, 3, 5)
    nx, ny, nz = shape
    N = nx * ny * nz
    Q = oracle.NQ[model]
    er, mr, sg = 1.7, 1.3, 0.05
    P = oracle.Problem(model, shape, eps_r=np.full(N, er), mu_r=np.full(N, mr), sigma=np.full(N, sg))
    f0 = RNG.normal(size=(Q, N))
    f = f0.copy()
    nsteps = 7
    oracle.run(P, f, 0, nsteps)
    C = collision_matrix(model, er, mr, sg)
    F = np.fft.fftn(f0.reshape(Q, nz, ny, nx), axes=(1, 2, 3))
    out = np.zeros_like(F)
    for iz in range(nz):
        for iy in range(ny):
            for ix in range(nx):
                k = 2 * math.pi * np.array([ix / nx, iy / ny, iz / nz])
                A = amplification(model, C, k)
                out[:, iz, iy, ix] = np.linalg.matrix_power(A, nsteps) @ F[:, iz, iy, ix]
    ref = np.real(np.fft.ifftn(out, axes=(1, 2, 3))).reshape(Q, N)
    np.testing.assert_allclose(f, ref, atol=1e-11)


def max_growth(model, er, mr, nk=24):
    """Largest |eigenvalue| of A(k) over a grid of the Brillouin zone."""
    C = collision_matrix(model, er, mr, 0.0)
    g = 0.0
    ks = np.linspace(-math.pi, math.pi, nk, endpoint=False)
    for kx in ks:
        for ky in ks[::3]:
            for kz in ks[::2]:
                g = max(g, np.abs(np.linalg.eigvals(amplification(model, C, np.array([kx, ky, kz])))).max())
    return g


@pytest.mark.parametrize("model", ["mm", "hv"])
def test_stability_limit_at_vacuum_speed(model):
    """Sections II-A and III-B: speeds above the vacuum speed (eps_r mu_r < 1) are
    unstable; the vacuum itself and slower media are not amplified."""
    # vacuum sits exactly on the limit with defective eigenvalues, so the computed
    # eigenvalues carry an error of order sqrt(machine epsilon)
    assert max_growth(model, 1.0, 1.0) < 1 + 1e-6
    assert max_growth(model, 2.5, 1.0) < 1 + 1e-9
    assert max_growth(model, 0.7, 1.0) > 1.05


def global_operator(model, eps):
    N = len(eps)
    Q = oracle.NQ[model]
    P = oracle.Problem(model, (1, 1, N), eps_r=np.asarray(eps, float))
    A = np.zeros((Q * N, Q * N))
    for k in range(Q * N):
        f = np.zeros((Q, N))
        f.reshape(-1)[k] = 1.0
        oracle.run(P, f, 0, 1)
        A[:, k] = f.reshape(-1)
    return A


def test_interface_spectral_radius():
    """Global 1-D operator with a dielectric step 1 -> 2.5 (two interfaces on the
    periodic lattice).  MM stays on the unit circle; the modified HV model has
    a growing mode (radius > 1), so long HV runs through interfaces amplify
    round-off.  This is why the multilayer and inverse-design parity uses MM."""
    eps = np.where(np.arange(32) < 16, 1.0, 2.5)
    r_mm = np.abs(np.linalg.eigvals(global_operator("mm", eps))).max()
    r_hv = np.abs(np.linalg.eigvals(global_operator("hv", eps))).max()
    assert r_mm < 1 + 1e-7
    assert r_hv > 1 + 1e-3


def test_mm_fields_depend_only_on_pair_differences():
    """The MM scheme in difference form rests on this: the E, B, D and H the MM
    scheme produces depend on its populations only through the differences
    f_{i0} - f_{i1} of each pair.  Adding the same arbitrary value to both
    populations of every pair, and arbitrary values to the rest populations,
    of a random state (random media, soft currents, a hard plane source) must
    leave every field of the next steps unchanged.  Also: both populations of
    a pair move along the same velocity, and the collision maps the pair
    differences to themselves alone."""
    shape = (5, 4, 6)
    n = int(np.prod(shape))
    rng = np.random.default_rng(17)
    eps, mu, sig = rng.uniform(1, 3, n), rng.uniform(1, 2, n), rng.uniform(0, 0.2, n)
    currents = [(int(c), tuple(rng.normal(size=3)), 13.0, 0.4) for c in rng.choice(n, 3, replace=False)]
    P = oracle.Problem("mm", shape, eps_r=eps, mu_r=mu, sigma=sig, currents=currents,
                       plane=(2, (0.3, -0.2, 0.1), (0.05, 0.4, -0.1), 17.0))
    f = rng.normal(size=(50, n))
    g = f.copy()
    pairs = [(r * 24 + p * 8 + i * 2, r * 24 + p * 8 + i * 2 + 1) for r in range(2) for p in range(3)
             for i in range(4)]
    for a, b in pairs:
        s = rng.normal(size=n)
        g[a] += s
        g[b] += s
    g[48:50] += rng.normal(size=(2, n))
    V = oracle.velocities("mm")
    assert all((V[a] == V[b]).all() for a, b in pairs)
    for steps in (1, 7):
        fa, ga = f.copy(), g.copy()
        oracle.run(P, fa, 0, steps)
        oracle.run(P, ga, 0, steps)
        for x, y in zip(oracle.fields(P, fa, steps), oracle.fields(P, ga, steps)):
            np.testing.assert_allclose(y, x, rtol=0, atol=1e-11 * np.abs(x).max())
        # the streamed pair differences agree too
        for a, b in pairs:
            np.testing.assert_allclose(ga[a] - ga[b], fa[a] - fa[b], rtol=0, atol=1e-10)
        # while changing one difference does change the fields
        h = f.copy()
        h[pairs[0][0], :] += 1.0
        oracle.run(P, h, 0, steps)
        assert np.abs(oracle.fields(P, h, steps)[0] - oracle.fields(P, fa, steps)[0]).max() > 1e-3
    # collision: the image of a pure pair sum (f_{i0} = f_{i1}) has zero differences
    C = collision_matrix("mm", 1.7, 1.3, 0.1)
    for a, b in pairs:
        u = np.zeros(50)
        u[a] = u[b] = 1.0
        out = C @ u
        assert max(abs(out[x] - out[y]) for x, y in pairs) < 1e-14
