"""Thin ctypes binding of ``liblbem.so`` (include/lbem.h).

Only argument marshalling happens here: torch provides device memory and the
stream, every step of the computation runs in the library's HIP kernels.  If
the library is not built, or no GPU is present, constructing a lattice raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbem.so")

MODEL = {"mm": 0, "hv": 1, "mmd": 2}  # "mmd": MM in difference form (24 populations)
STORAGE = {"f32": 0, "bf16": 1, "f16": 2, "bf16_shifted": 3, "f16_shifted": 4}
NQ = {"mm": 50, "hv": 36, "mmd": 24}
STATUS = {0: "LBEM_OK", -1: "LBEM_EINVAL", -2: "LBEM_ENOMEM", -3: "LBEM_EHIP", -4: "LBEM_EUNSTABLE",
          -5: "LBEM_ESTATE", -6: "LBEM_ENOTFINITE"}

# every function include/lbem.h declares, with its ctypes signature
_P, _I32, _I64, _D, _SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
SIGNATURES = {
    "lbem_version": (_I32, []),
    "lbem_last_error": (C.c_char_p, []),
    "lbem_workspace_size": (_I32, [_P, C.POINTER(_SZ)]),
    "lbem_workspace_bytes": (_SZ, [_P]),
    "lbem_state_size": (_I32, [_P, C.POINTER(_SZ)]),
    "lbem_create": (_I32, [_P, _P, _P, _P, _P, _SZ, _P, C.POINTER(_P)]),
    "lbem_destroy": (_I32, [_P]),
    "lbem_set_stream": (_I32, [_P, _P]),
    "lbem_set_fields": (_I32, [_P, _P, _P]),
    "lbem_set_current_source": (_I32, [_P, _I32, _P, _P, _D, _D]),
    "lbem_set_plane_source": (_I32, [_P, _I32, _P, _P, _D]),
    "lbem_add_point_current": (_I32, [_P, _I32, _I32, _I32, _P, _D, _D]),
    "lbem_set_probes": (_I32, [_P, _I32, _P, _I64, _P]),
    "lbem_set_flux_monitor": (_I32, [_P, _I32, _P, _I64, _I64, _P]),
    "lbem_set_detector": (_I32, [_P, _I32]),
    "lbem_detector_read": (_I32, [_P, _P]),
    "lbem_set_detector_plane": (_I32, [_P, _I32, _P]),
    "lbem_check": (_I32, [_P, _D, C.POINTER(_D)]),
    "lbem_set_energy_series": (_I32, [_P, _I32, _I64, _P]),
    "lbem_step": (_I32, [_P, _I64]),
    "lbem_get_time": (_I32, [_P, C.POINTER(_I64)]),
    "lbem_get_fields": (_I32, [_P, _P, _P, _P, _P]),
    "lbem_energy": (_I32, [_P, _P]),
    "lbem_save_state": (_I32, [_P, _P]),
    "lbem_set_tuning": (_I32, [_P, _P, _P]),
    "lbem_get_tuning": (_I32, [_P, _P, _P]),
    "lbem_autotune": (_I32, [_P, _I32, _P]),
    "lbem_load_state": (_I32, [_P, _P, _I64]),
    "lbem_adjoint_workspace_size": (_I32, [_P, _I64, _I32, _I32, C.POINTER(_SZ)]),
    "lbem_adjoint_keep": (_I32, [_P, _I64, _I32, _SZ, C.POINTER(_I32)]),
    "lbem_adjoint_forward": (_I32, [_P, _I64, _I32, _I32, _I32, _P, _SZ, _P]),
    "lbem_adjoint_backward": (_I32, [_P, _P, _SZ, _P, _P, _D, _P, _P]),
    "lbem_adjoint": (_I32, [_P, _I64, _I32, _I32, _I32, _P, _P, _D, _P, _P, _P, _P, _SZ]),
    "lbem_adjoint_static_bytes": (_SZ, []),
    "lbem_adjoint_static": (_I32, [_P, _I64, _I32, _I32, _I32, _P, _P, _D, _P, _P, _P]),
    "lbem_set_adjoint_tuning": (_I32, [_P, _P, _P]),
    "lbem_get_adjoint_tuning": (_I32, [_P, _P, _P]),
    "lbem_batch_workspace_size": (_I32, [_I32, _I32, _I32, _P, C.POINTER(_SZ)]),
    "lbem_batch_create": (_I32, [_I32, _I32, _I32, _P, _P, _P, _P, _P, _SZ, _P, C.POINTER(_P)]),
    "lbem_batch_destroy": (_I32, [_P]),
    "lbem_batch_set_fields": (_I32, [_P, _P, _P]),
    "lbem_batch_set_launch": (_I32, [_P, _I32, _I32]),
    "lbem_batch_set_blocking": (_I32, [_P, _I32]),
    "lbem_batch_get_blocking": (_I32, [_P, C.POINTER(_I32)]),
    "lbem_batch_autotune": (_I32, [_P, _I32, C.POINTER(_I32), C.POINTER(_I32)]),
    "lbem_batch_step": (_I32, [_P, _I64]),
    "lbem_batch_step_graph": (_I32, [_P, _I64]),
    "lbem_batch_step_per_instance": (_I32, [_P, _I64]),
    "lbem_batch_get_fields": (_I32, [_P, _P, _P]),
    "lbem_batch_get_time": (_I32, [_P, C.POINTER(_I64)]),
}


class LbemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Desc(C.Structure):
    _fields_ = [("model", C.c_int32), ("storage", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("nz", C.c_int32), ("reserved", C.c_int32), ("storage_scale", C.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblbem.so and declare its signatures (no GPU needed to load).
    The environment variable LBEM_LIBRARY names another build to load instead."""
    global _lib
    path = os.environ.get("LBEM_LIBRARY", path)
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build()")
        lib = C.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status: int):
    if status != 0:
        raise LbemError(status, load_library().lbem_last_error().decode())


def _stream_ptr(stream: Optional[torch.cuda.Stream]) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dev_f32(a, n: int, device) -> Optional[torch.Tensor]:
    if a is None:
        return None
    t = torch.as_tensor(np.asarray(a) if not isinstance(a, torch.Tensor) else a)
    t = t.to(device=device, dtype=torch.float32).contiguous().reshape(-1)
    if t.numel() != n:
        raise ValueError(f"expected {n} values, got {t.numel()}")
    return t


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def desc(model: str, shape, storage: str = "f32", storage_scale: float = 0.0) -> Desc:
    nx, ny, nz = shape
    return Desc(MODEL[model], STORAGE[storage], nx, ny, nz, 0, float(storage_scale))


def workspace_size(model: str, shape, storage: str = "f32") -> int:
    lib = load_library()
    out = C.c_size_t()
    d = desc(model, shape, storage)
    check(lib.lbem_workspace_size(C.byref(d), C.byref(out)))
    return out.value


class Lattice:
    """One periodic nx*ny*nz lattice of the MM or HV model on the current GPU."""

    def __init__(self, model: str, shape, eps_r=None, mu_r=None, sigma=None, storage: str = "f32",
                 storage_scale: float = 0.0, device="cuda", stream: Optional[torch.cuda.Stream] = None):
        if not torch.cuda.is_available():
            raise RuntimeError("the lbem library needs a GPU; none is visible")
        self.lib = load_library()
        self.model, self.shape, self.storage = model, tuple(int(s) for s in shape), storage
        nx, ny, nz = self.shape
        self.n = nx * ny * nz
        self.device = torch.device(device)
        self._desc = desc(model, self.shape, storage, storage_scale)
        size = C.c_size_t()
        check(self.lib.lbem_workspace_size(C.byref(self._desc), C.byref(size)))
        self.workspace = torch.empty(size.value, dtype=torch.uint8, device=self.device)
        media = [_dev_f32(x, self.n, self.device) for x in (eps_r, mu_r, sigma)]
        h = C.c_void_p()
        self._stream = stream
        check(self.lib.lbem_create(C.byref(self._desc), *[_ptr(m) for m in media], _ptr(self.workspace),
                                   size.value, C.c_void_p(_stream_ptr(stream)), C.byref(h)))
        self.h = h
        self._keep = {}

    def close(self):
        if getattr(self, "h", None):
            self.lib.lbem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ set-up
    def set_fields(self, E, B):
        E = _dev_f32(E, 3 * self.n, self.device)
        B = _dev_f32(B, 3 * self.n, self.device)
        check(self.lib.lbem_set_fields(self.h, _ptr(E), _ptr(B)))
        self._keep["fields0"] = (E, B)  # kept alive until the stream has consumed them

    def set_current_source(self, cells: Sequence[int], J0, period: float, phase: float = 0.0):
        cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int64))
        J0 = np.ascontiguousarray(np.asarray(J0, dtype=np.float32).reshape(-1, 3))
        check(self.lib.lbem_set_current_source(self.h, len(cells), cells.ctypes.data_as(C.c_void_p),
                                               J0.ctypes.data_as(C.c_void_p), float(period), float(phase)))

    def set_currents(self, currents):
        """Point currents as (cell, J0[3], period, phase); replaces all sources."""
        if not currents:
            check(self.lib.lbem_set_current_source(self.h, 0, None, None, 1.0, 0.0))
            return
        periods = {c[2] for c in currents}
        phases = {c[3] for c in currents}
        if len(periods) == 1 and len(phases) == 1:
            self.set_current_source([c[0] for c in currents], [c[1] for c in currents], periods.pop(), phases.pop())
            return
        check(self.lib.lbem_set_current_source(self.h, 0, None, None, 1.0, 0.0))
        nx, ny, _ = self.shape
        for cell, J0, period, phase in currents:
            cell = int(cell)
            self.add_point_current((cell % nx, (cell // nx) % ny, cell // (nx * ny)), J0, period, phase)

    def add_point_current(self, xyz, J0, period: float, phase: float = 0.0):
        """One more soft point current at cell (x, y, z) with its own period and phase."""
        J0 = np.ascontiguousarray(np.asarray(J0, dtype=np.float32).reshape(3))
        x, y, z = (int(v) for v in xyz)
        check(self.lib.lbem_add_point_current(self.h, x, y, z, J0.ctypes.data_as(C.c_void_p), float(period),
                                              float(phase)))

    def set_plane_source(self, z: int, E0, B0, period: float):
        E0 = np.ascontiguousarray(np.asarray(E0, dtype=np.float32))
        B0 = np.ascontiguousarray(np.asarray(B0, dtype=np.float32))
        check(self.lib.lbem_set_plane_source(self.h, int(z), E0.ctypes.data_as(C.c_void_p),
                                             B0.ctypes.data_as(C.c_void_p), float(period)))

    def set_probes(self, cells: Sequence[int], cap_rows: int) -> torch.Tensor:
        cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int64))
        series = torch.zeros((cap_rows, len(cells), 6), dtype=torch.float64, device=self.device)
        check(self.lib.lbem_set_probes(self.h, len(cells), cells.ctypes.data_as(C.c_void_p), int(cap_rows),
                                       _ptr(series)))
        self._keep["probes"] = series
        return series

    def set_flux_monitor(self, cells: Sequence[int], n_begin: int, n_end: int) -> torch.Tensor:
        """Largest |E x H| in each cell over the steps that collide time levels
        n_begin .. n_end - 1 (FP64, on the device, filled as steps run)."""
        cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int64))
        out = torch.zeros(len(cells), dtype=torch.float64, device=self.device)
        check(self.lib.lbem_set_flux_monitor(self.h, len(cells), cells.ctypes.data_as(C.c_void_p), int(n_begin),
                                             int(n_end), _ptr(out)))
        self._keep["flux"] = out
        return out

    def set_detector(self, z: int):
        check(self.lib.lbem_set_detector(self.h, int(z)))

    def set_detector_plane(self, z: int) -> torch.Tensor:
        """Detector plane whose accumulated sum the library writes to the
        returned device tensor after every step call."""
        acc = torch.empty(1, dtype=torch.float64, device=self.device)
        check(self.lib.lbem_set_detector_plane(self.h, int(z), _ptr(acc)))
        self._keep["detector_acc"] = acc
        return acc

    def detector(self) -> torch.Tensor:
        out = torch.zeros(1, dtype=torch.float64, device=self.device)
        check(self.lib.lbem_detector_read(self.h, _ptr(out)))
        return out

    def set_energy_series(self, every: int, cap: int) -> torch.Tensor:
        series = torch.zeros(cap, dtype=torch.float64, device=self.device)
        check(self.lib.lbem_set_energy_series(self.h, int(every), int(cap), _ptr(series)))
        self._keep["energy"] = series
        return series

    def set_stream(self, stream: Optional[torch.cuda.Stream]):
        self._stream = stream
        check(self.lib.lbem_set_stream(self.h, C.c_void_p(_stream_ptr(stream))))

    # ------------------------------------------------------------ run
    def step(self, nsteps: int = 1):
        check(self.lib.lbem_step(self.h, int(nsteps)))

    @property
    def time(self) -> int:
        t = C.c_int64()
        check(self.lib.lbem_get_time(self.h, C.byref(t)))
        return t.value

    def fields(self):
        """(E, B, D, H), each a [3][N] float32 device tensor."""
        outs = [torch.empty((3, self.n), dtype=torch.float32, device=self.device) for _ in range(4)]
        check(self.lib.lbem_get_fields(self.h, *[_ptr(o) for o in outs]))
        return tuple(outs)

    def energy(self) -> torch.Tensor:
        out = torch.zeros(1, dtype=torch.float64, device=self.device)
        check(self.lib.lbem_energy(self.h, _ptr(out)))
        return out

    def check(self, max_energy: float = 0.0) -> float:
        """lbem_check: the energy of the current state; raises LbemError with
        LBEM_ENOTFINITE or LBEM_EUNSTABLE (see include/lbem.h)."""
        u = C.c_double()
        check(self.lib.lbem_check(self.h, float(max_energy), C.byref(u)))
        return u.value

    def state_size(self) -> int:
        out = C.c_size_t()
        check(self.lib.lbem_state_size(C.byref(self._desc), C.byref(out)))
        return out.value

    def save_state(self, dst: Optional[torch.Tensor] = None):
        if dst is None:
            dst = torch.empty(self.state_size(), dtype=torch.uint8, device=self.device)
        check(self.lib.lbem_save_state(self.h, _ptr(dst)))
        return dst, self.time

    def load_state(self, src: torch.Tensor, t: int):
        if src.numel() * src.element_size() < self.state_size():
            raise ValueError("state buffer too small")
        check(self.lib.lbem_load_state(self.h, _ptr(src), int(t)))

    # ------------------------------------------------------------ launch tuning
    def set_tuning(self, form, blocks_per_cu):
        f = (C.c_int32 * 2)(*form)
        b = (C.c_int32 * 2)(*blocks_per_cu)
        check(self.lib.lbem_set_tuning(self.h, f, b))

    def tuning(self):
        f = (C.c_int32 * 2)()
        b = (C.c_int32 * 2)()
        check(self.lib.lbem_get_tuning(self.h, f, b))
        return list(f), list(b)

    def autotune(self, trial_steps: int = 10):
        """Pick the fastest launch tuning on this lattice (state left unchanged)."""
        backup = torch.empty(self.state_size(), dtype=torch.uint8, device=self.device)
        check(self.lib.lbem_autotune(self.h, int(trial_steps), _ptr(backup)))
        return self.tuning()

    # ------------------------------------------------------------ adjoint
    def set_adjoint_tuning(self, form, blocks_per_cu):
        f = (C.c_int32 * 2)(*form)
        c = (C.c_int32 * 2)(*blocks_per_cu)
        check(self.lib.lbem_set_adjoint_tuning(self.h, f, c))

    def adjoint_tuning(self):
        f = (C.c_int32 * 2)()
        c = (C.c_int32 * 2)()
        check(self.lib.lbem_get_adjoint_tuning(self.h, f, c))
        return list(f), list(c)

    def adjoint_keep(self, nsteps: int, K: int, budget_bytes: int) -> int:
        """The largest keep whose adjoint workspace fits in budget_bytes."""
        keep = C.c_int32()
        check(self.lib.lbem_adjoint_keep(C.byref(self._desc), int(nsteps), int(K), int(budget_bytes),
                                         C.byref(keep)))
        return keep.value

    def adjoint_workspace(self, nsteps: int, K: int, keep: int = 1) -> torch.Tensor:
        size = C.c_size_t()
        check(self.lib.lbem_adjoint_workspace_size(C.byref(self._desc), int(nsteps), int(K), int(keep),
                                                   C.byref(size)))
        ws = torch.empty(size.value, dtype=torch.uint8, device=self.device)
        self._adj_keep = int(keep)
        return ws

    def adjoint_forward(self, nsteps: int, K: int, det_z: int, ws: torch.Tensor,
                        keep: Optional[int] = None) -> torch.Tensor:
        """Run nsteps with a checkpoint every K steps (the last `keep` segments also
        keep their E frames); return the detector loss (dev double [1])."""
        keep = getattr(self, "_adj_keep", 1) if keep is None else keep
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        check(self.lib.lbem_adjoint_forward(self.h, int(nsteps), int(K), int(keep), int(det_z), _ptr(ws),
                                            ws.numel(), _ptr(loss)))
        return loss

    def adjoint_backward(self, ws: torch.Tensor, E0=None, B0=None, scale: float = 1.0):
        """dL/deps_r and dL/dsigma (dev double [N]) for the last adjoint_forward."""
        ge = torch.empty(self.n, dtype=torch.float64, device=self.device)
        gs = torch.empty(self.n, dtype=torch.float64, device=self.device)
        E0 = _dev_f32(E0, 3 * self.n, self.device)
        B0 = _dev_f32(B0, 3 * self.n, self.device)
        check(self.lib.lbem_adjoint_backward(self.h, _ptr(ws), ws.numel(), _ptr(E0), _ptr(B0), float(scale),
                                             _ptr(ge), _ptr(gs)))
        self._keep["adjoint_fields0"] = (E0, B0)
        return ge, gs

    def adjoint(self, nsteps: int, K: int, det_z: int, ws: torch.Tensor, keep: int = 1, E0=None, B0=None,
                scale: float = 1.0):
        """Both passes in one library call: (loss, dL/deps_r, dL/dsigma)."""
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        ge = torch.empty(self.n, dtype=torch.float64, device=self.device)
        gs = torch.empty(self.n, dtype=torch.float64, device=self.device)
        E0 = _dev_f32(E0, 3 * self.n, self.device)
        B0 = _dev_f32(B0, 3 * self.n, self.device)
        check(self.lib.lbem_adjoint(self.h, int(nsteps), int(K), int(keep), int(det_z), _ptr(E0), _ptr(B0),
                                    float(scale), _ptr(ge), _ptr(gs), _ptr(loss), _ptr(ws), ws.numel()))
        self._keep["adjoint_fields0"] = (E0, B0)
        return loss, ge, gs

    def adjoint_static(self, nsteps: int, K: int, det_z: int, keep: int = 1, E0=None, B0=None, scale: float = 1.0,
                       out=None):
        """lbem_adjoint_static: lbem_adjoint with the library's fixed device
        workspace.  out: optional (loss [1], dL/deps_r [N], dL/dsigma [N])
        float64 device tensors to write into; E0, B0 as for adjoint (device
        float32 tensors are passed through without a copy)."""
        if out is None:
            out = (torch.zeros(1, dtype=torch.float64, device=self.device),
                   torch.empty(self.n, dtype=torch.float64, device=self.device),
                   torch.empty(self.n, dtype=torch.float64, device=self.device))
        loss, ge, gs = out
        E0 = _dev_f32(E0, 3 * self.n, self.device)
        B0 = _dev_f32(B0, 3 * self.n, self.device)
        check(self.lib.lbem_adjoint_static(self.h, int(nsteps), int(K), int(keep), int(det_z), _ptr(E0), _ptr(B0),
                                           float(scale), _ptr(ge), _ptr(gs), _ptr(loss)))
        self._keep["adjoint_fields0"] = (E0, B0)
        return loss, ge, gs


class Batch:
    """Many independent ragged 1-D lattices (1 x 1 x L_b) advanced together."""

    def __init__(self, model: str, offsets, eps_r=None, mu_r=None, sigma=None, storage: str = "f32",
                 device="cuda", stream: Optional[torch.cuda.Stream] = None):
        if not torch.cuda.is_available():
            raise RuntimeError("the lbem library needs a GPU; none is visible")
        self.lib = load_library()
        self.model, self.storage = model, storage
        self.offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        self.n = len(self.offsets) - 1
        self.total = int(self.offsets[-1])
        self.device = torch.device(device)
        size = C.c_size_t()
        op = self.offsets.ctypes.data_as(C.c_void_p)
        check(self.lib.lbem_batch_workspace_size(MODEL[model], STORAGE[storage], self.n, op, C.byref(size)))
        self.workspace = torch.empty(size.value, dtype=torch.uint8, device=self.device)
        media = [_dev_f32(x, self.total, self.device) for x in (eps_r, mu_r, sigma)]
        h = C.c_void_p()
        check(self.lib.lbem_batch_create(MODEL[model], STORAGE[storage], self.n, op, *[_ptr(m) for m in media],
                                         _ptr(self.workspace), size.value, C.c_void_p(_stream_ptr(stream)),
                                         C.byref(h)))
        self.h = h
        self._keep = None

    def close(self):
        if getattr(self, "h", None):
            self.lib.lbem_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_fields(self, E, B):
        E = _dev_f32(E, 3 * self.total, self.device)
        B = _dev_f32(B, 3 * self.total, self.device)
        check(self.lib.lbem_batch_set_fields(self.h, _ptr(E), _ptr(B)))
        self._keep = (E, B)

    def set_launch(self, threads: int, groups_per_cu: int):
        check(self.lib.lbem_batch_set_launch(self.h, int(threads), int(groups_per_cu)))

    def set_blocking(self, steps_per_pass: int):
        """Temporal blocking: steps per pass over each instance (0 = off)."""
        check(self.lib.lbem_batch_set_blocking(self.h, int(steps_per_pass)))

    def blocking(self) -> int:
        k = C.c_int32()
        check(self.lib.lbem_batch_get_blocking(self.h, C.byref(k)))
        return k.value

    def autotune(self, trial_steps: int = 20):
        """Pick the fastest launch shape and blocking (state left unchanged);
        returns (threads, groups per CU); the blocking is read with blocking()."""
        t, g = C.c_int32(), C.c_int32()
        check(self.lib.lbem_batch_autotune(self.h, int(trial_steps), C.byref(t), C.byref(g)))
        return t.value, g.value

    def step(self, nsteps: int):
        check(self.lib.lbem_batch_step(self.h, int(nsteps)))

    def step_graph(self, nsteps: int):
        check(self.lib.lbem_batch_step_graph(self.h, int(nsteps)))

    def step_per_instance(self, nsteps: int):
        check(self.lib.lbem_batch_step_per_instance(self.h, int(nsteps)))

    @property
    def time(self) -> int:
        t = C.c_int64()
        check(self.lib.lbem_batch_get_time(self.h, C.byref(t)))
        return t.value

    def fields(self):
        """(E, B), each a [3][total] float32 device tensor."""
        E = torch.empty((3, self.total), dtype=torch.float32, device=self.device)
        B = torch.empty((3, self.total), dtype=torch.float32, device=self.device)
        check(self.lib.lbem_batch_get_fields(self.h, _ptr(E), _ptr(B)))
        return E, B


def _model_for(workload_model: str, model: Optional[str]) -> str:
    # an MM workload (media in MM units) may run on either form of the MM scheme
    if model is None or model == workload_model:
        return workload_model
    if workload_model == "mm" and model == "mmd":
        return model
    raise ValueError(f"a {workload_model} workload cannot run on the {model} model")


def batch_from_inputs(bt, storage: str = "f32", model: Optional[str] = None) -> Batch:
    """Set up a Batch from an inputs.Batch (media and initial fields); model
    "mmd" runs an MM batch in difference form."""
    b = Batch(_model_for(bt.model, model), bt.offsets, bt.eps_r, bt.mu_r, bt.sigma, storage=storage)
    b.set_fields(bt.E0, bt.B0)
    return b


def lattice_from_workload(w, storage: str = "f32", storage_scale: float = 0.0,
                          model: Optional[str] = None) -> Lattice:
    """Set up a Lattice from an inputs.Workload (media, fields, sources, probes,
    detector); model "mmd" runs an MM workload in difference form."""
    lat = Lattice(_model_for(w.model, model), w.shape, w.eps_r, w.mu_r, w.sigma, storage=storage, storage_scale=storage_scale)
    lat.set_fields(*w.fields0())
    if w.currents:
        lat.set_currents(w.currents)
    if w.plane is not None:
        z, E0, B0, period = w.plane
        lat.set_plane_source(z, E0, B0, period)
    if w.det_z is not None:
        lat.set_detector(w.det_z)
    return lat
