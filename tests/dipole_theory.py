"""Continuum fields of the dipole sources of Section IV-C, for the radiation
checks.

A cell carrying the soft current J_z(t) = J0 sin(omega t), switched on at
t = 0, is a point dipole p(t) z with p = J0 (1 - cos omega t) / omega for
t > 0 (cell volume 1): the current moves charge, so besides the oscillating
moment a static one of size J0 / omega builds up.  Its fields are the
time-domain dipole fields (Jackson, Classical Electrodynamics, ch. 9, which
the paper cites for the dipole), with retarded time t* = t - r / c:

    E = 1/(4 pi eps0) { [3 n (n.p) - p] / r^3 + [3 n (n.p') - p'] / (c r^2)
                        - [(n x p'') x n] / (c^2 r) }
    H = 1/(4 pi) { (p' x n) / r^2 + (p'' x n) / (c r) }

and zero before the front (t* < 0).  A source of several cells is the sum of
their dipoles, which also gives the source's finite extent.  The energy flux
is S = E x H.  In the far field |S| peaks at mu0 omega^4 p0^2 sin^2(theta) /
(16 pi^2 c r^2) over a period; closer in, the static moment adds about
(k r)^-2 to that peak."""
import math

import numpy as np


def dipole_fields(sources, points, t, eps0, mu0, omega):
    """E and H at points [P][3] (coordinates relative to any origin) and times
    t [T]; sources: list of (position [3], J0 along z).  Returns E, H as
    [T][P][3]."""
    c = 1.0 / math.sqrt(eps0 * mu0)
    points = np.asarray(points, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    E = np.zeros((len(t), len(points), 3))
    H = np.zeros_like(E)
    z = np.array([0.0, 0.0, 1.0])
    for pos, j0 in sources:
        d = points - np.asarray(pos, dtype=np.float64)[None, :]
        r = np.linalg.norm(d, axis=1)
        n = d / r[:, None]
        ts = t[:, None] - r[None, :] / c                     # retarded time [T][P]
        on = ts > 0
        p0 = j0 / omega
        p = np.where(on, p0 * (1 - np.cos(omega * ts)), 0.0)
        p1 = np.where(on, p0 * omega * np.sin(omega * ts), 0.0)
        p2 = np.where(on, p0 * omega ** 2 * np.cos(omega * ts), 0.0)
        nz = n[:, 2]                                          # n . z
        radial = 3 * n * nz[:, None] - z[None, :]             # 3 n (n.z) - z  [P][3]
        transverse = z[None, :] - n * nz[:, None]             # (n x z) x n    [P][3]
        nxz = np.cross(z[None, :], n)                         # z x n          [P][3]
        E += (radial[None] * (p / r ** 3 + p1 / (c * r ** 2))[..., None]
              - transverse[None] * (p2 / (c ** 2 * r))[..., None]) / (4 * math.pi * eps0)
        H += nxz[None] * (p1 / r ** 2 + p2 / (c * r))[..., None] / (4 * math.pi)
    return E, H


def max_flux(sources, points, t, eps0, mu0, omega):
    """Largest |E x H| over the times t, per point."""
    E, H = dipole_fields(sources, points, t, eps0, mu0, omega)
    return np.linalg.norm(np.cross(E, H), axis=-1).max(axis=0)


def workload_sources(shape, currents):
    """(position, J0_z) of every soft current of a workload, positions as
    (x, y, z) cell coordinates."""
    nx, ny, _ = shape
    out = []
    for cell, j0, _, _ in currents:
        cell = int(cell)
        out.append((np.array([cell % nx, (cell // nx) % ny, cell // (nx * ny)], dtype=np.float64), float(j0[2])))
    return out


def sample_points(shape, cells):
    """(x, y, z) cell coordinates of flat cell indices."""
    nx, ny, _ = shape
    cells = np.asarray(cells, dtype=np.int64)
    return np.stack([cells % nx, (cells // nx) % ny, cells // (nx * ny)], axis=1).astype(np.float64)
