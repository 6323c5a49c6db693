"""Error norms of the parity tests (GPU result against the oracle).

Every parity check reports and bounds two relative errors: the L2 error over
all targets and right-hand sides, ||got - ref||_2 / ||ref||_2, and the sup
error, max |got - ref| / max |ref| (the paper quotes its accuracy in the
relative supremum norm, Sec. 3.2).  The L2 error alone would let one bad
output vector among 2^20 pass; the sup error catches it."""
import numpy as np


def rel_l2(got, ref) -> float:
    nb = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / (nb if nb > 0 else 1.0))


def rel_sup(got, ref) -> float:
    mb = np.abs(ref).max() if np.size(ref) else 0.0
    return float(np.abs(got - ref).max() / (mb if mb > 0 else 1.0)) if np.size(ref) else 0.0


def assert_parity(got, ref, tol: float, sup_tol: float = None, what: str = "") -> tuple:
    """Both relative errors below their bars (sup_tol defaults to tol); NaN
    anywhere fails."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    assert np.isfinite(got).all(), f"{what}: non-finite output"
    e2, es = rel_l2(got, ref), rel_sup(got, ref)
    print(f"  {what} rel L2 {e2:.3e}  rel sup {es:.3e}", flush=True)
    assert e2 < tol, f"{what}: rel L2 {e2:.3e} >= {tol:.1e}"
    assert es < (tol if sup_tol is None else sup_tol), f"{what}: rel sup {es:.3e}"
    return e2, es
