"""Seeded synthetic workloads for the MM and HV Maxwell lattice-Boltzmann solvers.

This module only builds inputs -- media arrays, initial fields, source and
probe descriptions -- as plain numpy arrays.  It holds none of the method's
arithmetic, so both the HIP library (through its Python binding) and the CPU
oracle can be fed from it.  Every array uses the cell order x fastest:
``cell = x + nx * (y + ny * z)``; vector fields are ``[3][N]``.

Workloads (all synthetic; the paper uses no dataset):

* ``interface``   1-D Gaussian pulse crossing one dielectric interface
                  (Section IV-A; 1 x 1 x 1000, eps_r 1 -> 2.5 at z = 500).
* ``skin``        1-D plane wave from a hard source entering a conductor
                  (Section IV-B; 1 x 1 x 4096, sigma = 0.05 for z > 2048).
* ``dipole``      3-D vacuum box with a soft point current J_z = sin(2 pi n / 40)
                  at the centre and a 16-cell quadratic sigma sponge on all
                  faces (Section IV-C, point-source form).
* ``radiation``   the dipole with the Gaussian current of Section IV-C and the
                  cells of a sphere where the radiation pattern is measured.
* ``multilayer``  ragged batch of 1-D instances with random dielectric layers
                  (Section IV-D generalised to random stacks).
* ``slab``        inverse-design lattice: smooth random eps_r and sigma in a
                  slab, plane-wave pulse, detector plane.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

# Vacuum wave speed of each model in lattice units: 1/sqrt(2) for MM
# (Section II-A, eps0 = 1, mu0 = 2) and 1/3 for HV (Section III-B).
VACUUM_SPEED = {"mm": 1.0 / math.sqrt(2.0), "hv": 1.0 / 3.0}
# Lattice vacuum constants (eps0, mu0) of each model; HV's split is a reading
# (only eps0 * mu0 = 9 follows from the speed 1/3).
VACUUM_CONSTANTS = {"mm": (1.0, 2.0), "hv": (3.0, 3.0)}


@dataclass
class Workload:
    """Everything needed to set up one lattice run."""
    name: str
    model: str
    shape: Tuple[int, int, int]              # (nx, ny, nz)
    eps_r: Optional[np.ndarray] = None       # [N] float64, None = 1
    mu_r: Optional[np.ndarray] = None        # [N] float64, None = 1
    sigma: Optional[np.ndarray] = None       # [N] float64, None = 0
    E0: Optional[np.ndarray] = None          # [3][N] float64, None = 0
    B0: Optional[np.ndarray] = None          # [3][N] float64, None = 0
    currents: List[tuple] = field(default_factory=list)  # (cell, J0[3], period, phase)
    plane: Optional[tuple] = None            # (z, E0[3], B0[3], period)
    probes: List[int] = field(default_factory=list)
    det_z: Optional[int] = None
    steps: int = 0
    meta: dict = field(default_factory=dict)  # experiment geometry used by the analysis

    @property
    def n(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz

    def fields0(self):
        E0 = np.zeros((3, self.n)) if self.E0 is None else self.E0
        B0 = np.zeros((3, self.n)) if self.B0 is None else self.B0
        return E0, B0


def cell_index(shape, x, y, z) -> int:
    nx, ny, _ = shape
    return int(x + nx * (y + ny * z))


def gaussian_pulse(shape, z0: float, width: float, speed: float, amplitude: float = 1.0):
    """E_x = A exp(-((z - z0) / width)^2), B_y = E_x / speed, uniform in x and y.

    ``speed`` is the wave speed of the medium the pulse starts in, so that the
    pulse travels toward +z (Poynting vector along x cross y)."""
    nx, ny, nz = shape
    z = np.arange(nz, dtype=np.float64)
    ex = amplitude * np.exp(-((z - z0) / width) ** 2)
    E0 = np.zeros((3, nx * ny * nz))
    B0 = np.zeros((3, nx * ny * nz))
    E0[0] = np.repeat(ex, nx * ny)
    B0[1] = E0[0] / speed
    return E0, B0


def z_profile(shape, values_along_z: np.ndarray) -> np.ndarray:
    """Broadcast a length-nz profile to an [N] array (x fastest)."""
    nx, ny, nz = shape
    return np.repeat(np.asarray(values_along_z, dtype=np.float64), nx * ny)


def interface(model: str = "mm", nz: int = 1000, eps2: float = 2.5, mu2: float = 1.0,
              steps: int = 2000) -> Workload:
    """Gaussian pulse crossing one interface (Section IV-A).

    eps_r = 1 for z < nz/2 and eps2 beyond; pulse centre 200, width 20 (the
    1 x 1 x 1000 configuration); probes at z = 300 (reflection) and 700
    (transmission)."""
    shape = (1, 1, nz)
    z = np.arange(nz)
    eps = z_profile(shape, np.where(z < nz // 2, 1.0, eps2))
    mu = z_profile(shape, np.where(z < nz // 2, 1.0, mu2))
    E0, B0 = gaussian_pulse(shape, z0=0.2 * nz, width=0.02 * nz, speed=VACUUM_SPEED[model])
    return Workload("interface", model, shape, eps_r=eps, mu_r=mu, E0=E0, B0=B0,
                    probes=[int(0.3 * nz), int(0.7 * nz)], steps=steps)


def skin(model: str = "mm", nz: int = 4096, sigma: float = 0.05, wavelength: float = 64.0,
         steps: int = 20000) -> Workload:
    """Plane wave from a hard source at z = 0 entering a conductor (Section IV-B).

    sigma on cells z > nz/2; E_imp = sin(omega n) x, B_imp = E_imp / c y with
    the vacuum wavelength ``wavelength`` cells, i.e. period wavelength / c."""
    shape = (1, 1, nz)
    z = np.arange(nz)
    sg = z_profile(shape, np.where(z > nz // 2, sigma, 0.0))
    c = VACUUM_SPEED[model]
    period = wavelength / c
    plane = (0, (1.0, 0.0, 0.0), (0.0, 1.0 / c, 0.0), period)
    return Workload("skin", model, shape, sigma=sg, plane=plane, steps=steps)


# sigma_max of the quadratic sponge per model, chosen with the 1-D oracle for
# a reflection below 1 % at the dipole frequency (see the design notes).
SPONGE_SIGMA_MAX = {"mm": 0.5, "hv": 1.0}


def sponge_profile(n: int, thickness: int, sigma_max: float) -> np.ndarray:
    """sigma(d) = sigma_max (d / thickness)^2, d = depth into the layer (1..thickness)."""
    i = np.arange(n, dtype=np.float64)
    d_lo = thickness - i            # depth from the low face
    d_hi = i - (n - 1 - thickness)  # depth from the high face
    d = np.maximum(np.maximum(d_lo, d_hi), 0.0)
    return sigma_max * (d / thickness) ** 2


def gaussian_currents(shape, centre, alpha: float, amplitude: float, period: float, radius: int = 4):
    """Soft current J_z(x) = A exp(-alpha |x - x_d|^2) sin(2 pi n / period) on the
    cells within ``radius`` of the centre (Section IV-C); list of point currents."""
    nx, ny, nz = shape
    cx, cy, cz = centre
    out = []
    for dz in range(-radius, radius + 1):
        for dy in range(-radius, radius + 1):
            for dx in range(-radius, radius + 1):
                r2 = dx * dx + dy * dy + dz * dz
                if r2 > radius * radius:
                    continue
                a = amplitude * math.exp(-alpha * r2)
                out.append((cell_index(shape, (cx + dx) % nx, (cy + dy) % ny, (cz + dz) % nz),
                            (0.0, 0.0, a), period, 0.0))
    return out


def dipole(model: str = "mm", n: int = 256, period: float = 40.0, sponge: int = 16,
           sigma_max: Optional[float] = None, steps: int = 1000, amplitude: float = 1.0,
           shape: Optional[Tuple[int, int, int]] = None, source: str = "point",
           alpha: float = 0.5) -> Workload:
    """Vacuum box with a soft current J_z = A sin(2 pi n / period) at the centre
    and a quadratic sigma sponge of ``sponge`` cells on each face.

    source = "point": one cell; "gaussian": A exp(-alpha r^2) profile of
    Section IV-C (dipole moment A (pi / alpha)^1.5 / omega)."""
    shape = shape or (n, n, n)
    nx, ny, nz = shape
    smax = SPONGE_SIGMA_MAX[model] if sigma_max is None else sigma_max
    sx = sponge_profile(nx, sponge, smax)
    sy = sponge_profile(ny, sponge, smax)
    sz = sponge_profile(nz, sponge, smax)
    sg = np.maximum(np.maximum(sx[None, None, :], sy[None, :, None]), sz[:, None, None]).reshape(-1)
    cx, cy, cz = nx // 2, ny // 2, nz // 2
    if source == "point":
        currents = [(cell_index(shape, cx, cy, cz), (0.0, 0.0, amplitude), period, 0.0)]
    else:
        currents = gaussian_currents(shape, (cx, cy, cz), alpha, amplitude, period)
    probes = [cell_index(shape, cx + d, cy, cz) for d in (4, 8, 16) if cx + d < nx]
    return Workload("dipole", model, shape, sigma=sg, currents=currents, probes=probes, steps=steps)


# ------------------------------------------------------------ refinement study
# The four experiments of Section IV with the paper's geometry, scaled to a
# lattice of L cells along z (the "refinement" is L).

def paper_pulse(shape, z0: float, alpha: float, speed: float):
    """E_x = exp(-(z - z0)^2 / (2 alpha^2)), B_y = E_x / speed (eq. Initialpulse)."""
    return gaussian_pulse(shape, z0, math.sqrt(2.0) * alpha, speed)


def study_interface(model: str, L: int) -> Workload:
    """Section IV-A: alpha = 0.05 L / sqrt(2), z0 = L/2 - L/6, eps_r 1 -> 2.5 at
    L/2; run until the pulse has travelled L/3 in vacuum time (reflected pulse
    back at L/3, transmitted one L / (6 sqrt(2.5)) past the interface)."""
    shape = (1, 1, L)
    z = np.arange(L)
    c = VACUUM_SPEED[model]
    eps = z_profile(shape, np.where(z < L // 2, 1.0, 2.5))
    E0, B0 = paper_pulse(shape, L / 2 - L / 6, 0.05 * L / math.sqrt(2.0), c)
    return Workload("study_interface", model, shape, eps_r=eps, E0=E0, B0=B0,
                    steps=int(round((L / 3) / c)), meta={"z_if": L // 2, "eps2": 2.5})


def study_skin(model: str, L: int) -> Workload:
    """Section IV-B: hard source E = sin(omega t) x, B = E / C y at z = 0,
    T = 17.68e-3 L / C, conductor sigma = 0.1 eps / T (eps = eps0, vacuum
    permittivity of the model) for L / 4 <= z < L.  The paper's far end is
    open; here L / 4 more cells carry a sin^2 sponge (up to sigma = 0.5) that
    absorbs the wave leaving the conductor and the source's backward wave
    before the periodic wrap brings either back.  Runs until the front has
    crossed the lattice and three more periods; the amplitude is taken over
    the last period."""
    S = L // 4
    shape = (1, 1, L + S)
    z = np.arange(L + S)
    c = VACUUM_SPEED[model]
    eps0 = VACUUM_CONSTANTS[model][0]
    T = 17.68e-3 * L / c
    sigma = 0.1 * eps0 / T
    zc = L // 4
    ramp = np.sin(np.pi * np.clip(z - L, 0, S) / S) ** 2
    sg = z_profile(shape, np.where(z >= zc, sigma + (0.5 - sigma) * ramp, 0.0))
    plane = (0, (1.0, 0.0, 0.0), (0.0, 1.0 / c, 0.0), T)
    steps = int(round(L / c + 3 * T))
    return Workload("study_skin", model, shape, sigma=sg, plane=plane, steps=steps,
                    meta={"z_c": zc, "z_end": L, "period": T, "sigma": sigma})


def study_dipole(model: str, n: int, sponge: int = 8) -> Workload:
    """Section IV-C: Gaussian current J0 exp(-alpha r^2) sin(omega t) z,
    alpha = 0.5, J0 = 1e-4, T = 0.1768 n / C, t_max = 70 T / 25; field
    amplitudes over the last period on the +x axis from the centre, out to
    where the wave has been established for a period."""
    c = VACUUM_SPEED[model]
    T = 0.1768 * n / c
    w = dipole(model, n=n, period=T, sponge=sponge, steps=int(round(70 * T / 25)), amplitude=1e-4,
               source="gaussian", alpha=0.5)
    cx = n // 2
    r_max = min(int(c * (w.steps - T)), cx - sponge - 1)
    rs = list(range(3, r_max + 1))
    w.name = "study_dipole"
    w.probes = [cell_index(w.shape, cx + r, cx, cx) for r in rs]
    w.meta = {"period": T, "radii": rs, "J0": 1e-4, "alpha": 0.5}
    return w


def study_layers(model: str, L: int) -> Workload:
    """Section IV-D: eps_r = 1, 1.3, 2, 3 with interfaces at z0, z0 + d, z0 + 3d
    (z0 = L / 2, d = L / 20); pulse at z0 - L / 30 with alpha = L / (100 sqrt 2).
    Runs until the transmitted pulse is L / 10 past the last interface."""
    shape = (1, 1, L)
    z = np.arange(L)
    c = VACUUM_SPEED[model]
    z0, d = L // 2, L // 20
    bounds = [z0, z0 + d, z0 + 3 * d]
    epsz = np.where(z < bounds[0], 1.0, np.where(z < bounds[1], 1.3, np.where(z < bounds[2], 2.0, 3.0)))
    alpha = L / (100.0 * math.sqrt(2.0))
    zp = z0 - L / 30
    E0, B0 = paper_pulse(shape, zp, alpha, c)
    travel = (bounds[0] - zp) + d * math.sqrt(1.3) + 2 * d * math.sqrt(2.0) + (L / 10) * math.sqrt(3.0)
    return Workload("study_layers", model, shape, eps_r=z_profile(shape, epsz), E0=E0, B0=B0,
                    steps=int(round(travel / c)),
                    meta={"bounds": bounds, "eps": [1.0, 1.3, 2.0, 3.0], "z_pulse": zp, "alpha": alpha})


@dataclass
class Radiation:
    """A radiation-pattern run (Section IV-C): a Gaussian dipole workload and
    the cells of a sphere of radius R about the dipole, sampled on four
    half-planes of constant azimuth, where the largest energy flux over one
    period is measured."""
    workload: Workload
    cells: np.ndarray         # [K] int64
    theta: np.ndarray         # [K] polar angle from the dipole axis z, radians
    phi: np.ndarray           # [K] azimuth, radians
    radius: np.ndarray        # [K] distance of each cell from the dipole centre
    window: Tuple[int, int]   # time levels [n_begin, n_end) of one period
    period: float             # steps
    wavelength: float         # cells


def radiation(model: str = "mm", n: int = 256, alpha: float = 0.5, amplitude: float = 1e-4, n_theta: int = 37,
              sponge: int = 16) -> Radiation:
    """Section IV-C radiation-pattern set-up on an n^3 vacuum box: Gaussian
    current J_z = J0 exp(-alpha r^2) sin(2 pi t / T) with T = 0.1768 n / c,
    wavelength lambda = c T, sample radius R = lambda (n / (2 lambda) - 2),
    flux maximum taken over the period R + lambda <= c t < R + 2 lambda; the
    run ends there.  Sample cells: polar angles 0..pi in n_theta steps on the
    half-planes phi = 0, pi/2, pi, 3 pi/2, rounded to the nearest cell."""
    c = VACUUM_SPEED[model]
    period = 0.1768 * n / c
    lam = c * period
    R = lam * (n / (2.0 * lam) - 2.0)
    n_begin = int(round((R + lam) / c))
    n_end = n_begin + int(round(period))
    w = dipole(model, n=n, period=period, sponge=sponge, steps=n_end, amplitude=amplitude, source="gaussian",
               alpha=alpha)
    ctr = np.array([n // 2, n // 2, n // 2], dtype=np.float64)
    cells, th, ph, rad = [], [], [], []
    for phi in (0.0, 0.5 * math.pi, math.pi, 1.5 * math.pi):
        for theta in np.linspace(0.0, math.pi, n_theta):
            d = R * np.array([math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi), math.cos(theta)])
            p = np.rint(ctr + d)
            cells.append(cell_index(w.shape, int(p[0]), int(p[1]), int(p[2])))
            th.append(theta)
            ph.append(phi)
            rad.append(float(np.linalg.norm(p - ctr)))
    return Radiation(w, np.array(cells, dtype=np.int64), np.array(th), np.array(ph), np.array(rad),
                     (n_begin, n_end), period, lam)


@dataclass
class Batch:
    """A ragged batch of independent 1-D (1 x 1 x L_b) instances, concatenated."""
    model: str
    lengths: np.ndarray       # [n] int64
    offsets: np.ndarray       # [n + 1] int64, CSR
    eps_r: np.ndarray         # [sum L] float64
    mu_r: np.ndarray
    sigma: np.ndarray
    E0: np.ndarray            # [3][sum L]
    B0: np.ndarray
    steps: int

    def instance(self, b: int) -> Workload:
        s, e = int(self.offsets[b]), int(self.offsets[b + 1])
        return Workload(f"multilayer[{b}]", self.model, (1, 1, e - s), eps_r=self.eps_r[s:e].copy(),
                        mu_r=self.mu_r[s:e].copy(), sigma=self.sigma[s:e].copy(),
                        E0=self.E0[:, s:e].copy(), B0=self.B0[:, s:e].copy(), steps=self.steps)


def multilayer(model: str = "mm", n_inst: int = 512, lmin: int = 500, lmax: int = 8000,
               lead_in: int = 200, tmin: int = 4, tmax: int = 64, log_sd: float = 0.5,
               width: float = 20.0, z0: float = 100.0, steps: int = 5000, seed: int = 0) -> Batch:
    """Random multilayer stacks (Section IV-D generalised).

    Lengths ~ U{lmin..lmax} (rng(seed)); after a vacuum lead-in, layers of
    thickness U{tmin..tmax} with eps_r = exp(|N(0, log_sd^2)|) >= 1 (rng(seed+1));
    a Gaussian pulse of the given width starts at z0 in the lead-in."""
    rl = np.random.default_rng(seed)
    lengths = rl.integers(lmin, lmax + 1, size=n_inst).astype(np.int64)
    offsets = np.zeros(n_inst + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(lengths)
    total = int(offsets[-1])
    rm = np.random.default_rng(seed + 1)
    eps = np.ones(total)
    E0 = np.zeros((3, total))
    B0 = np.zeros((3, total))
    c = VACUUM_SPEED[model]
    for b in range(n_inst):
        s, L = int(offsets[b]), int(lengths[b])
        z = lead_in
        while z < L:
            t = int(rm.integers(tmin, tmax + 1))
            eps[s + z: s + min(L, z + t)] = math.exp(abs(rm.normal(0.0, log_sd)))
            z += t
        zz = np.arange(L, dtype=np.float64)
        ex = np.exp(-((zz - z0) / width) ** 2)
        E0[0, s:s + L] = ex
        B0[1, s:s + L] = ex / c
    return Batch(model, lengths, offsets, eps, np.ones(total), np.zeros(total), E0, B0, steps)


def smooth_field(shape2: Tuple[int, int, int], sigma_f: float, seed: int) -> np.ndarray:
    """Seeded white noise, Gaussian-filtered (periodic, via FFT) and mapped to
    (0, 1) through the standard normal CDF. shape2 = (nz, ny, nx)."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape2)
    ks = [np.fft.fftfreq(n) for n in shape2]
    K = np.meshgrid(*ks, indexing="ij")
    g = np.exp(-2.0 * (math.pi * sigma_f) ** 2 * sum(k * k for k in K))
    s = np.real(np.fft.ifftn(np.fft.fftn(w) * g))
    s /= s.std()
    from scipy.special import ndtr
    return ndtr(s)


def slab(model: str = "mm", shape=(128, 128, 256), slab_z=(96, 160), eps_range=(1.0, 4.0),
         sigma_range=(0.0, 0.02), pulse_z: float = 56.0, pulse_width: float = 10.0, det_z: int = 230,
         sponge: int = 16, sigma_max: Optional[float] = None, steps: int = 1500, seed: int = 0,
         smooth: float = 4.0) -> Workload:
    """Inverse-design lattice: smooth random eps_r and sigma inside a slab
    (tapered to the background by a sin^2 window along z), fixed sigma sponges
    at both z ends, plane-wave pulse, detector plane."""
    nx, ny, nz = shape
    z0, z1 = slab_z
    eps = np.ones((nz, ny, nx))
    sg = np.zeros((nz, ny, nx))
    u1 = smooth_field((z1 - z0, ny, nx), smooth, seed)
    u2 = smooth_field((z1 - z0, ny, nx), smooth, seed + 1)
    # taper the random fields to the background at the slab faces: a sharp
    # face with eps varying along it grows an unstable mode in both models
    zz = np.arange(z1 - z0, dtype=np.float64)
    win = (np.sin(np.pi * (zz + 0.5) / (z1 - z0)) ** 2)[:, None, None]
    eps[z0:z1] = eps_range[0] + (eps_range[1] - eps_range[0]) * u1 * win
    sg[z0:z1] = sigma_range[0] + (sigma_range[1] - sigma_range[0]) * u2 * win
    smax = SPONGE_SIGMA_MAX[model] if sigma_max is None else sigma_max
    sz = sponge_profile(nz, sponge, smax)
    sg = np.maximum(sg, sz[:, None, None])
    E0, B0 = gaussian_pulse(shape, pulse_z, pulse_width, VACUUM_SPEED[model])
    return Workload("slab", model, shape, eps_r=eps.reshape(-1), sigma=sg.reshape(-1), E0=E0, B0=B0,
                    det_z=det_z, steps=steps)
