"""Parity bars shared by the GPU tests.

A cell passes when both of these hold, for a bar tol:
  relative l2     ||got - ref||_2 / ||s||_2       <= tol
  element-wise    max_v |got(v) - ref(v)| / max_v |s(v)| <= tol
where s = ref, or, for an output that is a cancellation of two O(1) terms
(L of a collision invariant), the loss term L-[h] (reading R13 of the
design notes).  The element-wise bound catches a localised error (one
Nyquist plane, the edge of the cutoff region, a box corner) that the l2 norm
over n^3 points would dilute by up to sqrt(n^3).

Every check records its two ratios; tests/conftest.py prints the worst of
each per test at the end of the session, so that the margins to the bars are
visible in the log.
"""
import numpy as np

RECORD = []   # (test id, tol, l2 ratio, element-wise ratio)
_current = {"id": "?"}


def set_test(nodeid):
    _current["id"] = nodeid


def errors(got, ref, scale=None):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    s = ref if scale is None else np.asarray(scale, dtype=np.float64)
    d = got - ref
    ns, ms = float(np.linalg.norm(s)), float(np.max(np.abs(s)))
    l2 = float(np.linalg.norm(d)) / ns if ns > 0 else float(np.linalg.norm(d))
    mx = float(np.max(np.abs(d))) / ms if ms > 0 else float(np.max(np.abs(d)))
    return l2, mx


def check(got, ref, tol, scale=None, tag=None):
    """Asserts both bars for one cell; returns (l2, element-wise) ratios."""
    l2, mx = errors(got, ref, scale)
    RECORD.append((_current["id"], tol, l2, mx))
    assert l2 <= tol and mx <= tol, (tag, "l2", l2, "max", mx, "bar", tol)
    return l2, mx


def check_cells(got, ref, tol, cells=None, scale=None, tag=None):
    """check() on every cell of a batch (axis 0); returns the worst ratios."""
    idx = range(len(ref)) if cells is None else cells
    worst = (0.0, 0.0)
    for i, b in enumerate(idx):
        r = ref[i] if cells is not None else ref[b]
        s = None if scale is None else scale[i if cells is not None else b]
        l2, mx = check(got[b], r, tol, s, tag=(tag, b))
        worst = (max(worst[0], l2), max(worst[1], mx))
    return worst


def batch_errors(got, ref):
    """Per-cell (l2, element-wise) ratios of two batches, vectorised."""
    got = np.asarray(got, dtype=np.float64).reshape(len(got), -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(len(ref), -1)
    d = got - ref
    l2 = np.linalg.norm(d, axis=1) / np.linalg.norm(ref, axis=1)
    mx = np.max(np.abs(d), axis=1) / np.max(np.abs(ref), axis=1)
    return l2, mx


def check_batch(got, ref, tol, tag=None):
    """Both bars on every cell of a full batch (vectorised); returns the
    worst (l2, element-wise) ratios."""
    l2, mx = batch_errors(got, ref)
    RECORD.append((_current["id"], tol, float(l2.max()), float(mx.max())))
    bad = np.nonzero((l2 > tol) | (mx > tol))[0]
    assert bad.size == 0, (tag, "cells", bad[:10].tolist(), "l2", float(l2.max()), "max", float(mx.max()), "bar", tol)
    return float(l2.max()), float(mx.max())
