"""Shared test helpers (no arithmetic of the method lives here)."""
import numpy as np


def assert_bitexact(got: np.ndarray, ref: np.ndarray, what: str = ""):
    """Equal bit patterns everywhere except where both are NaN."""
    got = np.ascontiguousarray(got, dtype=np.float64)
    ref = np.ascontiguousarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    gn, rn = np.isnan(got), np.isnan(ref)
    assert np.array_equal(gn, rn), "%s: NaN pattern differs (%d vs %d)" % (what, gn.sum(), rn.sum())
    gv, rv = got[~gn].view(np.int64), ref[~rn].view(np.int64)
    bad = np.nonzero(gv != rv)[0]
    if bad.size:
        i = bad[0]
        raise AssertionError("%s: %d of %d elements differ; first: got %r want %r"
                             % (what, bad.size, gv.size, got[~gn][i], ref[~rn][i]))
