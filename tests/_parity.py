"""Trace comparison used by the GPU parity tests.

Besides the relative L2 error over all samples (the spec bar), every
receiver is checked on its own, so that one wrong receiver cannot hide in the
norm of hundreds of correct ones:
* its error norm is at most `tol` times the largest receiver norm (an absolute
  floor: receivers far from the source carry almost no signal);
* receivers with at least 1% of the largest receiver norm are within `10 tol`
  of their own norm.
"""
import numpy as np


def _host(a):
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.asarray(a, dtype=np.float64)


def trace_errors(got, ref):
    """(relative L2 over all samples, worst receiver error / largest receiver
    norm, worst relative error of the receivers above 1% of that norm)."""
    got, ref = _host(got), _host(ref)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    total = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    e = np.linalg.norm((got - ref).reshape(got.shape[0], -1), axis=0)
    r = np.linalg.norm(ref.reshape(ref.shape[0], -1), axis=0)
    big = r.max()
    strong = r >= 1e-2 * big
    worst_strong = float(np.max(e[strong] / r[strong])) if strong.any() else 0.0
    return float(total), float(e.max() / big), worst_strong


def assert_traces(got, ref, tol=1e-4):
    total, worst_abs, worst_strong = trace_errors(got, ref)
    assert total < tol, f"relative L2 {total:.3e} >= {tol:.1e}"
    assert worst_abs < tol, f"worst receiver error {worst_abs:.3e} of the largest receiver norm"
    assert worst_strong < 10 * tol, f"worst strong-receiver relative error {worst_strong:.3e}"
    return total
