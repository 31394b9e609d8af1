"""Tolerances of the GPU path against the FP64 oracle, and the checks that apply them.

logL: |dlogL| / |logL| <= 1e-12 (FP64), <= 1e-5 (FP32).
Gradients: ||dg||_2 / ||g||_2 <= 1e-6 (FP64), <= 1e-3 (FP32), and componentwise
|dg_i| <= tol * max(|g_i|, 1e-3 ||g||_inf), so that a small component (the
gradient of a short tip branch, a rate-matrix entry far from the diagonal) is
held to the same relative bound unless it is below a thousandth of the largest.
"""
import numpy as np

TOL_LOGL = {"fp64": 1e-12, "fp32": 1e-5}
TOL_GRAD = {"fp64": 1e-6, "fp32": 1e-3}
TOL_P = {"fp64": 1e-12, "fp32": 2e-6}


def rel(a, b):
    return abs(a - b) / abs(b)


def grad_rel(g, ref):
    return float(np.linalg.norm(g - ref) / np.linalg.norm(ref))


def assert_grad(g, ref, tol, what="gradient"):
    """Norm-wise and componentwise bound (see module docstring)."""
    g = np.asarray(g, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    r = grad_rel(g, ref)
    assert r <= tol, f"{what}: ||dg||/||g|| = {r:.3e} > {tol:.1e}"
    floor = 1e-3 * np.abs(ref).max()
    bound = tol * np.maximum(np.abs(ref), floor)
    err = np.abs(g - ref)
    worst = int(np.argmax(err / bound))
    assert err[worst] <= bound[worst], (
        f"{what}: component {worst} off by {err[worst]:.3e} (value {ref[worst]:.6e}, bound {bound[worst]:.3e})")
