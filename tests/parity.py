"""Parity checks of a GPU result against a reference (the FP64 oracle, or
another GPU path), by the two measures of section 5.4.2:

* the noise distance over the whole result, here as the relative L2 error
  ||got - ref|| / ||ref|| = 10^(dE / 20) (1e-5 is -100 dB), asserted <= tol;
* the error of every single sample: max |got - ref| <= tol * max |ref|, so a
  few bad samples cannot hide inside a small norm, and the paper's count of
  sample components whose relative error passes a fixed threshold, skipping
  components whose reference lies within 1e3 machine epsilons (of the
  stepping precision) of zero -- printed for the record.
"""
import numpy as np

import oracle

FP32_EPS = float(np.finfo(np.float32).eps)
FP64_EPS = float(np.finfo(np.float64).eps)
COUNT_THRESHOLD = {32: 1e-3, 64: 1e-9}     # relative error per component counted by the report


def within(got, ref, tol, label="", precision=None):
    """Assert both bars; returns the relative L2 error.  precision (32 or 64)
    sets the epsilon of the component count; by default it follows tol."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (label, got.shape, ref.shape)
    assert np.all(np.isfinite(got)), label
    if precision is None:
        precision = 64 if tol < 1e-9 else 32
    err = oracle.rel_l2(got, ref)
    peak = float(np.max(np.abs(ref))) if ref.size else 0.0
    dmax = float(np.max(np.abs(got - ref))) if ref.size else 0.0
    per_sample = dmax / peak if peak > 0 else dmax
    thr = COUNT_THRESHOLD[precision]
    n_over = oracle.count_over_threshold(got, ref, thr, eps=FP64_EPS if precision == 64 else FP32_EPS) \
        if ref.size else 0
    print(f"[parity] {label} n={ref.size} rel_l2={err:.3e} max_abs/peak={per_sample:.3e} "
          f"components over {thr:g}: {n_over}/{2 * ref.size}", flush=True)
    assert err <= tol, (label, "rel_l2", err)
    assert per_sample <= tol, (label, "max_abs/peak", per_sample)
    return err
