"""Shared helpers of the GPU parity tests (tolerances and tensor plumbing)."""
import numpy as np
import torch

# Parity bars.
MI_TOL = 1e-4          # bits per symbol, FP32-family kernels vs the FP64 oracle
LLR_REL = 1e-3         # |dL| <= LLR_REL * max(|L_ref|, 1 nat)
FP64_TOL = 1e-11       # FP64 kernel vs the FP64 oracle


def dev():
    return torch.device("cuda", 0)


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


def tx_dev(tx):
    return to_dev(np.asarray(tx, dtype=np.int32))


def llr_err(got, ref):
    """Worst ratio |got - ref| / max(|ref|, 1) over all elements."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    assert np.isfinite(got).all(), "non-finite LLR from the kernel"
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1.0))) if got.size else 0.0


def assert_llr(got, ref, rel=LLR_REL):
    e = llr_err(got, ref)
    assert e <= rel, f"LLR error {e:.3e} > {rel:.1e}"


def assert_stats(got, ref, tol=MI_TOL, se_rel=1e-2, se_abs=1e-6):
    got = np.asarray(got, dtype=np.float64).reshape(-1, 4)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1, 4)
    d = np.abs(got[:, :2] - ref[:, :2])
    assert d.max() <= tol, f"MI/GMI error {d.max():.3e} > {tol:.1e}\n{got[:, :2]}\n{ref[:, :2]}"
    # standard errors: relative, with an absolute floor for saturated points,
    # where FP32 rounding of the per-sample terms (~1e-6 bit) dominates the spread
    gs, rs = got[:, 2:], ref[:, 2:]
    assert (np.isnan(gs) == np.isnan(rs)).all(), (gs, rs)
    ok = np.isnan(rs) | (np.abs(gs - rs) <= se_rel * np.abs(rs) + se_abs)
    assert ok.all(), (gs, rs)
