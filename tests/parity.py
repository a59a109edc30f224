"""Element-by-element comparison helpers of the GPU parity tests."""
import numpy as np


def assert_u8_close(got, ref, what=""):
    """u8 outputs within 1 LSB of the oracle's rounded value, every element."""
    d = np.abs(np.asarray(got).astype(np.int32) - np.asarray(ref).astype(np.int32))
    assert d.max() <= 1, (what, int(d.max()), np.argwhere(d > 1)[:5].tolist())


def assert_f32_close(got, ref, tol, what=""):
    """Float outputs within tol (max abs error) of the oracle, every element."""
    e = np.abs(np.asarray(got, dtype=np.float64) - np.asarray(ref, dtype=np.float64))
    assert e.max() <= tol, (what, float(e.max()), np.argwhere(e > tol)[:5].tolist())
