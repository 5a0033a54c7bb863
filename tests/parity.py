"""Comparison of a GPU result with the oracle's (test helper).

FP64 bar at equal cycle counts: the leaf solutions agree to a relative L2
difference of 1e-12, and every cell agrees to 1e-12 of the largest value, so
that an error confined to a few cells (a box next to a refinement boundary)
cannot hide inside a global norm.
"""

from __future__ import annotations

import numpy as np

REL = 1e-12


def leaf_errors(ug, uo):
    """(relative L2 difference, max per-cell difference / max |uo|)."""
    ug = np.asarray(ug, dtype=np.float64).ravel()
    uo = np.asarray(uo, dtype=np.float64).ravel()
    scale = max(np.abs(uo).max(), 1e-300)
    rel = np.linalg.norm(ug - uo) / max(np.linalg.norm(uo), 1e-300)
    return rel, np.abs(ug - uo).max() / scale


def assert_leaf_parity(ug, uo, rel=REL, what=""):
    r2, rmax = leaf_errors(ug, uo)
    assert r2 <= rel, (what, "rel-L2", r2)
    assert rmax <= rel, (what, "max per cell", rmax)
    return r2, rmax


def assert_norms_close(g, o, atol, rtol=1e-9, what=""):
    """A pair of residual norms (max, L2) or their per-cycle histories."""
    g = np.atleast_1d(np.asarray(g, dtype=np.float64))
    o = np.atleast_1d(np.asarray(o, dtype=np.float64))
    assert g.shape == o.shape, (what, g.shape, o.shape)
    np.testing.assert_allclose(g, o, rtol=rtol, atol=atol, err_msg=str(what))
