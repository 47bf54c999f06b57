"""Comparison measures shared by the GPU parity tests.

Two measures are taken on every comparison of a GPU result with the FP64
oracle (or with another GPU run):

- the relative L2 error over the whole array, the measure the FP32 parity
  target is stated in;
- the largest element-wise error relative to the largest reference value.
  A whole-array norm dilutes a mistake confined to a few cells (a row wrap, a
  layout-chunk edge, an idle-thread slot, a source cell) by about sqrt(N);
  the element-wise bound does not.

Bounds.  FP32 storage: 1e-5 relative L2 and 1e-4 of the largest reference
value element-wise.  Where the oracle's own float32 build drifts further on
the same case (vacuum sits on the schemes' stability limit, so rounding
grows), both bounds become twice that measured float32 floor, taken the same
way.  16-bit storage: the format bound on the relative L2 error, and twice it
element-wise.  With rounding errors spread over the lattice, the largest
error relative to the largest value is about the relative L2 error, so the
factor two leaves room for the spread while an error confined to a few cells
and as large as the whole-array bound still fails it."""
import numpy as np

TOL = 1e-5
ELEM = 1e-4


def rel(a, b):
    """Relative L2 error of a against b."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def elem(a, b):
    """Largest element-wise error of a against b, relative to max |b|."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    mb = np.abs(b).max() if b.size else 0.0
    return float(np.abs(a - b).max() / (mb if mb > 0 else 1.0)) if b.size else 0.0


def check(got, ref, rel_tol=TOL, elem_tol=ELEM, what=""):
    """Assert both measures; return (relative L2, element-wise) errors."""
    er, ee = rel(got, ref), elem(got, ref)
    assert er < rel_tol and ee <= elem_tol, \
        f"{what}: relative L2 {er:.3e} (bound {rel_tol:.1e}), element-wise {ee:.3e} (bound {elem_tol:.1e})"
    return er, ee


def check16(got, ref, bound, what=""):
    """16-bit storage: the format bound in relative L2, twice it element-wise."""
    return check(got, ref, bound, 2 * bound, what)


def floor_bounds(f32, f64):
    """(relative L2, element-wise) bounds from the oracle's float32 drift on a
    case: the FP32 bars, or twice the measured floor where that is larger.
    f32, f64: sequences of arrays from the float32 and float64 oracle builds."""
    fr = max(rel(a, b) for a, b in zip(f32, f64))
    fe = max(elem(a, b) for a, b in zip(f32, f64))
    return max(TOL, 2 * fr), max(ELEM, 2 * fe), fr, fe
