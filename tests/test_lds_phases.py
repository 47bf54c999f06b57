"""Static check of the compiled step and adjoint kernels (gfx950 assembly of
this library's own sources): in the odd-parity kernels that shift populations
along x through LDS, the LDS array is reused by the gather and the scatter, so
between the gather's first and second workgroup barrier there may only be LDS
reads and between the second and third only LDS writes.  An LDS read moved
below the second barrier reads what other threads' scatter already wrote; the
compiler has produced exactly that under register pressure, which is why the
kernels bracket those barriers with compiler memory clobbers."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2309_08068_amd", "csrc")

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc")


def odd_lds_kernels(src, tmp_path):
    asm = tmp_path / (src + ".s")
    subprocess.run(["hipcc", "-O3", "-std=c++17", "--offload-arch=gfx950", "--offload-device-only", "-Xclang",
                    "-target-feature", "-Xclang", "-packed-fp32-ops", "-S", os.path.join(CSRC, src), "-o", str(asm)],
                   check=True, capture_output=True)
    text = asm.read_text()
    for name in re.findall(r"^(_Z\S+):", text, re.M):
        # row_step_kernel<M, ODD = 1, ST, RB, LATE, DIRECT = 0, ...>, adjoint_row_kernel<M, 1, RB, LATE, 0>
        if not (("row_step_kernel" in name and re.search(r"ELi1ENS0_\w+ELi\d+ELi[01]ELi0E", name)) or
                ("adjoint_row_kernel" in name and re.search(r"ELi1ELi\d+ELi[01]ELi0E", name))):
            continue
        body = text.split(name + ":", 1)[1].split(".Lfunc_end", 1)[0]
        ops = [l.strip().split()[0] for l in body.split("\n") if l.strip() and not l.strip().startswith((";", "."))]
        yield name, ops


@pytest.mark.parametrize("src,expect", [("lbem_lattice.hip", 120), ("lbem_adjoint.hip", 24)])
def test_lds_reads_and_writes_stay_in_their_phase(src, expect, tmp_path):
    n = 0
    for name, ops in odd_lds_kernels(src, tmp_path):
        n += 1
        seg, segs = 0, [[], [], []]
        for o in ops:
            if o == "s_barrier":
                seg += 1
                if seg > 2:
                    break
            elif o.startswith("ds_"):
                segs[seg].append(o)
        assert all(o.startswith("ds_write") for o in segs[0]), name
        assert segs[1] and all(o.startswith("ds_read") for o in segs[1]), name
        assert all(o.startswith("ds_write") for o in segs[2]), (name, sorted(set(segs[2])))
    assert n == expect
