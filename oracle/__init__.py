"""Plain CPU oracle for the MM and modified-HV lattice-Boltzmann Maxwell solvers.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``.  The product library never
imports, links or calls anything here, and this package imports nothing from
the product.

Two pieces:

* ``liboracle64.so`` / ``liboracle32.so``, built from ``lbem_oracle.c`` (plain
  C, FP64; the FP32 build only measures how far single precision drifts on the
  same scheme).  Wrapped by :class:`Problem`, :func:`init`, :func:`run`,
  :func:`fields` and the single-cell helpers below.
* ``torch_ref.py``: the same scheme written with plain PyTorch float64 CPU ops,
  used for the automatic-differentiation reference of the adjoint.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
MODELS = {"mm": 0, "hv": 1}
NQ = {"mm": 50, "hv": 36}


def build(force: bool = True) -> None:
    """Compile the oracle (FP64 and FP32 builds) with gcc."""
    src = os.path.join(HERE, "lbem_oracle.c")
    for tag, real in (("64", "double"), ("32", "float")):
        out = os.path.join(HERE, f"liboracle{tag}.so")
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src):
            continue
        cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", f"-DORACLE_REAL={real}",
               "-o", out + ".tmp", src, "-lm"]
        subprocess.check_call(cmd)
        os.replace(out + ".tmp", out)


_LIBS: dict = {}


def _lib(real: str = "f64"):
    tag = {"f64": "64", "f32": "32"}[real]
    if tag not in _LIBS:
        path = os.path.join(HERE, f"liboracle{tag}.so")
        if not os.path.exists(path):
            build(force=False)
        lib = C.CDLL(path)
        P = C.c_void_p
        lib.oracle_real_bytes.restype = C.c_int
        lib.oracle_threads.restype = C.c_int
        lib.oracle_nq.argtypes = [C.c_int]
        lib.oracle_velocity.argtypes = [C.c_int, C.c_int, P]
        lib.oracle_mm_tables.argtypes = [P, P, P]
        lib.oracle_equilibrium.argtypes = [C.c_int, P, P, P, C.c_double, C.c_double, C.c_double, P]
        lib.oracle_hv_source.argtypes = [P, P]
        lib.oracle_collide.argtypes = [C.c_int, P, C.c_double, C.c_double, C.c_double, P, P, P, P, P]
        lib.oracle_init.argtypes = [P, P, P, P]
        lib.oracle_fields.argtypes = [P, P, C.c_int64, P, P, P, P]
        lib.oracle_run.argtypes = [P, P, P, C.c_int64, C.c_int64, P]
        _LIBS[tag] = lib
    return _LIBS[tag]


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class _CProblem(C.Structure):
    _fields_ = [
        ("model", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("eps_r", C.c_void_p), ("mu_r", C.c_void_p), ("sigma", C.c_void_p),
        ("n_src", C.c_int32), ("src_cell", C.c_void_p), ("src_J0", C.c_void_p),
        ("src_period", C.c_void_p), ("src_phase", C.c_void_p),
        ("plane_z", C.c_int32), ("plane_E0", C.c_double * 3), ("plane_B0", C.c_double * 3),
        ("plane_period", C.c_double),
    ]


class _CObserve(C.Structure):
    _fields_ = [
        ("n_probe", C.c_int32), ("probe_cell", C.c_void_p), ("probe_series", C.c_void_p),
        ("det_z", C.c_int32), ("det_series", C.c_void_p),
        ("energy_every", C.c_int32), ("energy_series", C.c_void_p),
    ]


@dataclass
class Problem:
    """A periodic nx*ny*nz lattice (x fastest) with per-cell media and sources."""
    model: str
    shape: tuple  # (nx, ny, nz)
    eps_r: Optional[np.ndarray] = None
    mu_r: Optional[np.ndarray] = None
    sigma: Optional[np.ndarray] = None
    # soft point currents: list of (cell, J0[3], period, phase)
    currents: Sequence = field(default_factory=list)
    # hard plane source: (z, E0[3], B0[3], period) or None
    plane: Optional[tuple] = None

    @property
    def n(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz

    def _c(self):
        keep = []
        cp = _CProblem()
        cp.model = MODELS[self.model]
        cp.nx, cp.ny, cp.nz = self.shape
        for name in ("eps_r", "mu_r", "sigma"):
            a = getattr(self, name)
            if a is not None:
                a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))
                assert a.size == self.n
                keep.append(a)
                setattr(cp, name, _ptr(a))
        if self.currents:
            cells = np.array([c[0] for c in self.currents], dtype=np.int64)
            J0 = np.array([c[1] for c in self.currents], dtype=np.float64).reshape(-1, 3)
            per = np.array([c[2] for c in self.currents], dtype=np.float64)
            ph = np.array([c[3] for c in self.currents], dtype=np.float64)
            keep += [cells, J0, per, ph]
            cp.n_src = len(cells)
            cp.src_cell, cp.src_J0, cp.src_period, cp.src_phase = map(_ptr, (cells, J0, per, ph))
        if self.plane is not None:
            z, E0, B0, per = self.plane
            cp.plane_z = int(z)
            for a in range(3):
                cp.plane_E0[a] = float(E0[a])
                cp.plane_B0[a] = float(B0[a])
            cp.plane_period = float(per)
        else:
            cp.plane_z = -1
        return cp, keep


def _dtype(real: str):
    return np.float64 if real == "f64" else np.float32


def init(prob: Problem, E0: np.ndarray, B0: np.ndarray, real: str = "f64") -> np.ndarray:
    """Equilibrium initial populations [Q][N] for fields E0, B0 given as [3][N]."""
    lib = _lib(real)
    E0 = np.ascontiguousarray(E0, dtype=np.float64).reshape(3, prob.n)
    B0 = np.ascontiguousarray(B0, dtype=np.float64).reshape(3, prob.n)
    f = np.zeros((NQ[prob.model], prob.n), dtype=_dtype(real))
    cp, keep = prob._c()
    rc = lib.oracle_init(C.byref(cp), _ptr(E0), _ptr(B0), _ptr(f))
    if rc != 0:
        raise ValueError("oracle_init rejected the problem")
    return f


def run(prob: Problem, f: np.ndarray, n0: int, nsteps: int, probes: Optional[Sequence[int]] = None,
        det_z: Optional[int] = None, energy_every: int = 0) -> dict:
    """Advance f in place by nsteps steps from time level n0; return observations."""
    real = "f64" if f.dtype == np.float64 else "f32"
    lib = _lib(real)
    assert f.flags.c_contiguous and f.shape == (NQ[prob.model], prob.n)
    scratch = np.empty_like(f)
    cp, keep = prob._c()
    ob = _CObserve()
    out = {}
    if probes is not None and len(probes):
        pc = np.ascontiguousarray(np.asarray(probes, dtype=np.int64))
        ps = np.zeros((nsteps, len(pc), 6), dtype=np.float64)
        keep += [pc, ps]
        ob.n_probe, ob.probe_cell, ob.probe_series = len(pc), _ptr(pc), _ptr(ps)
        out["probes"] = ps
    ob.det_z = -1 if det_z is None else int(det_z)
    if det_z is not None:
        ds = np.zeros(nsteps, dtype=np.float64)
        keep.append(ds)
        ob.det_series = _ptr(ds)
        out["detector"] = ds
    ob.energy_every = int(energy_every)
    if energy_every > 0:
        es = np.zeros((nsteps + energy_every - 1) // energy_every, dtype=np.float64)
        keep.append(es)
        ob.energy_series = _ptr(es)
        out["energy"] = es
    rc = lib.oracle_run(C.byref(cp), _ptr(f), _ptr(scratch), int(n0), int(nsteps), C.byref(ob))
    if rc != 0:
        raise ValueError("oracle_run rejected the problem")
    return out


def fields(prob: Problem, f: np.ndarray, n: int):
    """Reported fields (E, B, D, H), each [3][N] float64, of state f at time level n."""
    real = "f64" if f.dtype == np.float64 else "f32"
    lib = _lib(real)
    outs = [np.zeros((3, prob.n), dtype=np.float64) for _ in range(4)]
    cp, keep = prob._c()
    rc = lib.oracle_fields(C.byref(cp), _ptr(f), int(n), *map(_ptr, outs))
    if rc != 0:
        raise ValueError("oracle_fields rejected the problem")
    return tuple(outs)


def threads() -> int:
    """OpenMP threads the oracle runs with."""
    return int(_lib().oracle_threads())


# ---------------------------------------------------------------- single cell

def velocity(model: str, q: int) -> np.ndarray:
    v = np.zeros(3, dtype=np.int32)
    if _lib().oracle_velocity(MODELS[model], q, _ptr(v)) != 0:
        raise IndexError(q)
    return v


def velocities(model: str) -> np.ndarray:
    return np.stack([velocity(model, q) for q in range(NQ[model])])


def mm_tables():
    """MM vector sets: v[p][i][3], e[p][i][j][3], b[p][i][j][3] (i = 0..3 is i = 1..4)."""
    v = np.zeros((3, 4, 3)); e = np.zeros((3, 4, 2, 3)); b = np.zeros((3, 4, 2, 3))
    _lib().oracle_mm_tables(_ptr(v), _ptr(e), _ptr(b))
    return v, e, b


def equilibrium(model: str, E, B, J=(0, 0, 0), rho=0.0, eps_r=1.0, mu_r=1.0) -> np.ndarray:
    feq = np.zeros(NQ[model])
    E, B, J = (np.ascontiguousarray(x, dtype=np.float64) for x in (E, B, J))
    _lib().oracle_equilibrium(MODELS[model], _ptr(E), _ptr(B), _ptr(J), rho, eps_r, mu_r, _ptr(feq))
    return feq


def hv_source(J) -> np.ndarray:
    J = np.ascontiguousarray(J, dtype=np.float64)
    T = np.zeros((6, 3))
    _lib().oracle_hv_source(_ptr(J), _ptr(T))
    return T


def collide(model: str, f, eps_r=1.0, mu_r=1.0, sigma=0.0, Jsrc=(0, 0, 0)):
    """One-cell collision: returns (f', E, B, J)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    Jsrc = np.ascontiguousarray(Jsrc, dtype=np.float64)
    fo = np.zeros(NQ[model]); E = np.zeros(3); B = np.zeros(3); J = np.zeros(3)
    _lib().oracle_collide(MODELS[model], _ptr(f), eps_r, mu_r, sigma, _ptr(Jsrc), _ptr(fo), _ptr(E), _ptr(B), _ptr(J))
    return fo, E, B, J
