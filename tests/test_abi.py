"""Host-side checks of the C ABI: the library loads without a GPU, exports every
function include/lbem.h declares, and rejects bad arguments before touching
the device."""
import ctypes as C

import numpy as np
import os
import re

import pytest

from paper_2309_08068_amd import lbem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(lbem_\w+)\s*\(", text))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lbem.LIB_PATH):
        from paper_2309_08068_amd import build
        build.build()
    return lbem.load_library()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    # and the binding declares a signature for each of them
    assert names <= set(lbem.SIGNATURES)


def test_version(lib):
    assert lib.lbem_version() >= 10000


def ws(model="mm", shape=(4, 4, 4), storage="f32", scale=0.0, reserved=0):
    d = lbem.desc(model, shape, storage, scale)
    d.reserved = reserved
    out = C.c_size_t()
    st = lbem.load_library().lbem_workspace_size(C.byref(d), C.byref(out))
    return st, out.value


def test_workspace_size_grows_with_model_and_storage(lib):
    st1, b_mm = ws("mm", (16, 16, 16))
    st2, b_hv = ws("hv", (16, 16, 16))
    st3, b_bf = ws("mm", (16, 16, 16), "bf16")
    assert st1 == st2 == st3 == 0
    n = 16 ** 3
    assert b_mm >= n * 50 * 4 + 12 * n
    assert b_hv >= n * 36 * 4 + 12 * n
    assert b_bf >= n * 50 * 2 + 12 * n and b_bf < b_mm
    out = C.c_size_t()
    d = lbem.desc("mm", (16, 16, 16), "bf16")
    assert lib.lbem_state_size(C.byref(d), C.byref(out)) == 0 and out.value == n * 50 * 2


def test_difference_form_sizes_and_limits(lib):
    """The MM scheme in difference form keeps 24 populations per cell (in the
    same chunked layout), runs as a batch, and its adjoint workspace holds 24
    adjoint populations per cell."""
    out = C.c_size_t()
    for shape, storage, size in (((16, 16, 16), "f32", 24 * 4 * 16 ** 3), ((16, 16, 16), "bf16", 24 * 2 * 16 ** 3),
                                 ((256, 20, 13), "f32", 9 * 24 * 8192 * 4),
                                 ((16, 16, 16), "bf16_shifted", 24 * 2 * 16 ** 3 + 16 * 16 ** 3)):
        d = lbem.desc("mmd", shape, storage)
        assert lib.lbem_state_size(C.byref(d), C.byref(out)) == 0 and out.value == size
    assert ws("mmd", (16, 16, 16))[1] < ws("mm", (16, 16, 16))[1]
    off = (C.c_int64 * 3)(0, 10, 30)
    assert lib.lbem_batch_workspace_size(lbem.MODEL["mmd"], 0, 2, off, C.byref(out)) == 0
    sizes = {}
    for model in ("mm", "mmd"):
        d = lbem.desc(model, (16, 16, 16))
        assert lib.lbem_adjoint_workspace_size(C.byref(d), 10, 2, 1, C.byref(out)) == 0
        sizes[model] = out.value
    assert sizes["mmd"] < sizes["mm"]


@pytest.mark.parametrize("storage,q", [("bf16_shifted", 50), ("f16_shifted", 50)])
def test_shifted_storage_sizes(lib, storage, q):
    """Equilibrium-shifted formats: 16-bit populations plus two planes of
    16-byte records in the workspace; a saved state holds one record plane."""
    n = 16 ** 3
    st, b_sh = ws("mm", (16, 16, 16), storage)
    _, b_bf = ws("mm", (16, 16, 16), "bf16")
    assert st == 0 and b_sh >= b_bf + 2 * 16 * n
    out = C.c_size_t()
    d = lbem.desc("mm", (16, 16, 16), storage)
    assert lib.lbem_state_size(C.byref(d), C.byref(out)) == 0 and out.value == n * q * 2 + 16 * n


@pytest.mark.parametrize("shape,storage,chunks,chunk_cells", [
    ((256, 20, 13), "f32", 9, 8192), ((384, 10, 13), "f32", 9, 8192), ((512, 3, 45), "f32", 9, 8192),
    ((128, 9, 60), "f32", 9, 8192), ((256, 16, 16), "f32", 8, 8192), ((256, 20, 13), "bf16", 5, 16384),
    ((128, 8, 8), "f32", 1, 0), ((90, 30, 40), "f32", 1, 0), ((100, 30, 40), "f32", 19, 8192),
    ((120, 9, 70), "bf16", 5, 16384), ((200, 9, 41), "f32", 12, 8192),
    ((200, 9, 41), "bf16", 6, 16384), ((60, 30, 40), "f32", 1, 0), ((600, 10, 10), "f32", 1, 0)])
def test_population_layout_chunks(lib, shape, storage, chunks, chunk_cells):
    """Row-form lattices (nx = 128, 256, 384, 512, or a row filling 3/4 of
    the next of 128, 256, 384, 512 threads) store populations in chunks of a
    power of two of x-rows with at most 32 KB per population plane, the rows
    a power of two of cells apart; the last chunk is padded.  A lattice
    that fits in one chunk (rows still padded), and any generic-form lattice,
    is one chunk."""
    out = C.c_size_t()
    d = lbem.desc("mm", shape, storage)
    assert lib.lbem_state_size(C.byref(d), C.byref(out)) == 0
    s = 4 if storage == "f32" else 2
    n = int(np.prod(shape))
    assert out.value == (chunks * 50 * chunk_cells * s if chunk_cells else 50 * n * s)


def test_batch_rejects_shifted_storage(lib):
    off = (C.c_int64 * 3)(0, 10, 30)
    out = C.c_size_t()
    for storage in ("bf16_shifted", "f16_shifted"):
        assert lib.lbem_batch_workspace_size(0, lbem.STORAGE[storage], 2, off, C.byref(out)) == -1
        assert b"batches" in lib.lbem_last_error()


@pytest.mark.parametrize("kw", [dict(shape=(0, 4, 4)), dict(shape=(4, -1, 4)), dict(reserved=1),
                                dict(storage="f16", scale=3.0), dict(storage="f16", scale=-2.0),
                                dict(storage="f16_shifted", scale=3.0), dict(shape=(2048, 1024, 1024))])
def test_bad_descriptors_rejected(lib, kw):
    st, _ = ws(**kw)
    assert st == -1
    assert lib.lbem_last_error()


def test_bad_model_and_storage_rejected(lib):
    d = lbem.desc("mm", (4, 4, 4))
    d.model = 7
    out = C.c_size_t()
    assert lib.lbem_workspace_size(C.byref(d), C.byref(out)) == -1
    d = lbem.desc("mm", (4, 4, 4))
    d.storage = 9
    assert lib.lbem_workspace_size(C.byref(d), C.byref(out)) == -1
    assert lib.lbem_workspace_size(None, C.byref(out)) == -1


def test_create_validates_host_arguments_first(lib):
    d = lbem.desc("mm", (4, 4, 4))
    h = C.c_void_p()
    # null workspace, misaligned workspace, too-small workspace, null out: no device work happens
    assert lib.lbem_create(C.byref(d), None, None, None, None, 0, None, C.byref(h)) == -1
    assert lib.lbem_create(C.byref(d), None, None, None, C.c_void_p(0x1001), 1 << 30, None, C.byref(h)) == -1
    assert lib.lbem_create(C.byref(d), None, None, None, C.c_void_p(0x100000), 16, None, C.byref(h)) == -2
    assert lib.lbem_create(C.byref(d), None, None, None, C.c_void_p(0x100000), 1 << 30, None, None) == -1


def test_null_handles_rejected(lib):
    assert lib.lbem_step(None, 1) == -1
    assert lib.lbem_destroy(None) == -1
    assert lib.lbem_get_fields(None, None, None, None, None) == -1
    assert lib.lbem_energy(None, None) == -1
    assert lib.lbem_check(None, 0.0, None) == -1
    assert lib.lbem_set_detector_plane(None, 3, None) == -1


def test_workspace_bytes_equals_workspace_size(lib):
    for model, shape, storage in (("mm", (16, 16, 16), "f32"), ("hv", (256, 20, 13), "bf16"),
                                  ("mmd", (200, 9, 41), "bf16_shifted")):
        st, size = ws(model, shape, storage)
        d = lbem.desc(model, shape, storage)
        assert st == 0 and lib.lbem_workspace_bytes(C.byref(d)) == size
    d = lbem.desc("mm", (0, 4, 4))
    assert lib.lbem_workspace_bytes(C.byref(d)) == 0 and lib.lbem_last_error()
    assert lib.lbem_workspace_bytes(None) == 0


def test_adjoint_needs_fp32_storage(lib):
    out = C.c_size_t()
    for storage in ("bf16", "f16", "bf16_shifted", "f16_shifted"):
        d = lbem.desc("hv", (16, 16, 16), storage)
        assert lib.lbem_adjoint_workspace_size(C.byref(d), 10, 2, 1, C.byref(out)) == -1
        assert b"FP32" in lib.lbem_last_error()
    d = lbem.desc("hv", (16, 16, 16))
    assert lib.lbem_adjoint_workspace_size(C.byref(d), 10, 2, 1, C.byref(out)) == 0


@pytest.mark.parametrize("model,shape,nsteps,K", [("mm", (128, 128, 256), 1500, 50), ("hv", (16, 16, 16), 41, 7),
                                                  ("mmd", (256, 2, 3), 10, 10)])
def test_adjoint_keep_is_largest_that_fits(lib, model, shape, nsteps, K):
    """lbem_adjoint_keep returns the largest keep whose workspace fits the
    budget: exact fits, one byte short, everything, and too little."""
    d = lbem.desc(model, shape)
    S = -(-nsteps // K)

    def size(keep):
        out = C.c_size_t()
        assert lib.lbem_adjoint_workspace_size(C.byref(d), nsteps, K, keep, C.byref(out)) == 0
        return out.value

    def keep_for(budget):
        k = C.c_int32()
        st = lib.lbem_adjoint_keep(C.byref(d), nsteps, K, budget, C.byref(k))
        return st, k.value

    sizes = [size(k) for k in range(1, S + 1)]
    assert sizes == sorted(sizes) and (S == 1 or sizes[-1] > sizes[0])
    for k in sorted({1, (S + 1) // 2, S}):
        assert keep_for(sizes[k - 1]) == (0, k)
        if k > 1 and sizes[k - 2] < sizes[k - 1]:
            assert keep_for(sizes[k - 1] - 1) == (0, k - 1)
    assert keep_for(1 << 62) == (0, S)
    st, _ = keep_for(sizes[0] - 1)
    assert lbem.STATUS[st] == "LBEM_ENOMEM"
    k = C.c_int32()
    assert lbem.STATUS[lib.lbem_adjoint_keep(C.byref(d), nsteps, K, 1 << 40, None)] == "LBEM_EINVAL"
    assert lbem.STATUS[lib.lbem_adjoint_keep(C.byref(d), 0, K, 1 << 40, C.byref(k))] == "LBEM_EINVAL"
