"""Comparison helpers of the GPU parity tests.

Every parity check compares the HIP result with the oracle element by element in two
norms: the relative l2 distance over the whole field, and the relative element-wise
maximum max|a - b| / max|b|.  The l2 bar is the test's stated tolerance; the max bar
defaults to 10 x that tolerance, so that a defect confined to a few elements -- which
the l2 norm over a large grid dilutes -- still fails, while rounding noise spread over
the field (whose max exceeds its l2 average by a small factor) passes.
"""
import numpy as np


def rel(a, b):
    """Relative l2 distance of a from b."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def relmax(a, b):
    """Relative element-wise maximum distance max|a - b| / max|b|."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def assert_close(a, b, bar, max_bar=None, what=""):
    """rel(a, b) <= bar and relmax(a, b) <= max_bar (default 10 x bar)."""
    max_bar = 10.0 * bar if max_bar is None else max_bar
    e2, em = rel(a, b), relmax(a, b)
    assert e2 <= bar, "%s relative l2 %.3e > %.1e" % (what, e2, bar)
    assert em <= max_bar, "%s relative max %.3e > %.1e" % (what, em, max_bar)
    return e2, em
