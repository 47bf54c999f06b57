"""MM stepper written with plain PyTorch float64 CPU ops, differentiable with
respect to the media -- the automatic-differentiation reference for the adjoint.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Same scheme and readings
as lbem_oracle.c (Section II; Appendix B order), written independently: the
vector tables are rebuilt here from eqs. (VelocitySetMiller) and
(ElectromagneticVectorsMiller); advection is a periodic roll by v_q.
"""
from __future__ import annotations

import math

import torch

MU0 = 2.0  # MM lattice permeability (Section II-A); eps0 = 1


def mm_tables():
    """v[p][i], e[p][i][j], b[p][i][j] (i = 0..3 is the paper's i = 1..4)."""
    v = torch.zeros(3, 4, 3, dtype=torch.float64)
    for p in range(3):
        for i in range(1, 5):
            ang = (2 * i - 1) * math.pi / 4
            c, s = round(math.sqrt(2) * math.cos(ang)), round(math.sqrt(2) * math.sin(ang))
            v[p, i - 1] = torch.tensor([(c, s, 0), (c, 0, s), (0, c, s)][p], dtype=torch.float64)
    e = torch.zeros(3, 4, 2, 3, dtype=torch.float64)
    for p in range(3):
        for i in range(1, 5):
            e[p, i - 1, 0] = 0.5 * v[p, ((i + 2) % 4)]      # v_{[(i+2) mod 4]+1}, 0-based index (i+2) mod 4
            e[p, i - 1, 1] = 0.5 * v[p, (i % 4)]            # v_{[i mod 4]+1}
    b = torch.cross(v[:, :, None, :].expand(3, 4, 2, 3), e, dim=-1)
    # population order r * 24 + p * 8 + i * 2 + j, then f_0^(0), f_0^(1)
    V = v[:, :, None, :].expand(3, 4, 2, 3).reshape(24, 3)
    return V, e.reshape(24, 3), b.reshape(24, 3)


V, EV, BV = mm_tables()


def fields(f, eps, mu, sig):
    """E, B (each [3][...]) of state f [50][nz][ny][nx] (no prescribed current)."""
    D = torch.einsum("q...,qa->a...", f[:24], EV)
    B = torch.einsum("q...,qa->a...", f[24:48], BV)
    E = (D / eps) / (1 + MU0 * sig / (4 * eps))
    return E, B


def equilibrium(E, B, J, rho, eps, mu):
    vJ = torch.einsum("qa,a...->q...", V, J) / 16
    Ee = torch.einsum("qa,a...->q...", EV, E)
    Bb = torch.einsum("qa,a...->q...", BV, B)
    f0 = vJ + eps / 4 * Ee + Bb / (8 * mu)
    f1 = vJ + Ee / 4 + Bb / 8
    return torch.cat([f0, f1, rho[None], rho[None]], dim=0)


def step(f, eps, mu, sig):
    """One collision (tau = 1/2) and advection f(x + v_q) <- f'(x), periodic."""
    E, B = fields(f, eps, mu, sig)
    J = sig * E
    rho = f[48] + f[:24].sum(0)
    fp = 2 * equilibrium(E, B, J, rho, eps, mu) - f
    out = []
    for q in range(50):
        if q >= 48:
            out.append(fp[q])
            continue
        vx, vy, vz = (int(t) for t in V[q % 24])
        out.append(torch.roll(fp[q], shifts=(vz, vy, vx), dims=(0, 1, 2)))
    return torch.stack(out)


def init(E0, B0, eps, mu):
    zero = torch.zeros_like(E0)
    return equilibrium(E0, B0, zero, torch.zeros_like(eps), eps, mu)


def detector_loss(eps, sig, mu, E0, B0, nsteps: int, det_z: int):
    """L = sum over the states collided by nsteps steps of sum_{x, y} |E(x, y, det_z)|^2.

    eps, sig, mu: [nz][ny][nx] float64 (eps, sig may require grad); E0, B0: [3][nz][ny][nx]."""
    f = init(E0, B0, eps, mu)
    L = torch.zeros((), dtype=torch.float64)
    for _ in range(nsteps):
        E, _ = fields(f, eps, mu, sig)
        L = L + (E[:, det_z] ** 2).sum()
        f = step(f, eps, mu, sig)
    return L, f


# ---------------------------------------------------------------- HV (Section III)
EPS0_HV, MU0_HV = 3.0, 3.0  # lattice constants (vacuum speed 1/3)
HVV = torch.tensor([[1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0], [0, 0, -1], [0, 0, 1]], dtype=torch.float64)


def hv_fields(f, eps, mu, sig):
    """E, B of HV state f [36][nz][ny][nx] (populations e_i then h_i, 3 components each)."""
    e = f[:18].reshape(6, 3, *f.shape[1:])
    h = f[18:].reshape(6, 3, *f.shape[1:])
    D = e.sum(0)
    B = h.sum(0)
    return D / (EPS0_HV * eps), B


def hv_equilibrium(D, B, eps, mu):
    E = D / (EPS0_HV * eps)
    H = B / (MU0_HV * mu)
    v = HVV.reshape(6, 3, *([1] * (D.dim() - 1)))
    vxH = torch.cross(v.expand(6, 3, *D.shape[1:]), H.expand(6, *H.shape), dim=1)
    vxE = torch.cross(v.expand(6, 3, *D.shape[1:]), E.expand(6, *E.shape), dim=1)
    feq_e = (D - 3 * vxH) / 6
    feq_h = (B + 3 * vxE) / 6
    return feq_e, feq_h


def hv_step(f, eps, mu, sig):
    """Modified HV collision (eq. CollisionmodifiedHV, tau = 1/2) and advection."""
    e = f[:18].reshape(6, 3, *f.shape[1:])
    h = f[18:].reshape(6, 3, *f.shape[1:])
    D = e.sum(0)
    B = h.sum(0)
    E = D / (EPS0_HV * eps)
    J = sig * E
    feq_e, feq_h = hv_equilibrium(D, B, eps, mu)
    v = HVV.reshape(6, 3, *([1] * (D.dim() - 1)))
    Jv = (J.unsqueeze(0) * v).sum(1, keepdim=True)
    T = -0.5 * Jv * v
    ep = 2 * feq_e - e + T
    hp = 2 * feq_h - h
    out = []
    for part in (ep, hp):
        for i in range(6):
            vx, vy, vz = (int(t) for t in HVV[i])
            out.append(torch.roll(part[i], shifts=(vz, vy, vx), dims=(1, 2, 3)))
    return torch.cat(out, dim=0)


def hv_init(E0, B0, eps, mu):
    D = EPS0_HV * eps * E0
    feq_e, feq_h = hv_equilibrium(D, B0, eps, mu)
    return torch.cat([feq_e.reshape(18, *E0.shape[1:]), feq_h.reshape(18, *E0.shape[1:])], dim=0)


def hv_detector_loss(eps, sig, mu, E0, B0, nsteps: int, det_z: int):
    """HV version of detector_loss."""
    f = hv_init(E0, B0, eps, mu)
    L = torch.zeros((), dtype=torch.float64)
    for _ in range(nsteps):
        E, _ = hv_fields(f, eps, mu, sig)
        L = L + (E[:, det_z] ** 2).sum()
        f = hv_step(f, eps, mu, sig)
    return L, f
