"""The eigenvalue comparison rule of the parity tests.

Two lists of eigenvalues agree when they have the same length and, both
sorted ascending, every pair satisfies
    |lambda_got - lambda_ref| <= rel * max(|lambda_ref|, 1e-6 ||A||),
with ||A|| = max(|lambda_min|, |lambda_max|) from the spectrum bounds. The
floor 1e-6 ||A|| only matters for eigenvalues next to zero.
"""
import numpy as np


def eig_err(got, ref, norm_a):
    """Elementwise |got - ref| / max(|ref|, 1e-6 norm_a) of two sorted lists."""
    got = np.sort(np.asarray(got, dtype=np.float64))
    ref = np.sort(np.asarray(ref, dtype=np.float64))
    assert len(got) == len(ref), (len(got), len(ref))
    if len(ref) == 0:
        return np.zeros(0)
    return np.abs(got - ref) / np.maximum(np.abs(ref), 1e-6 * abs(norm_a))


def assert_eigs_match(got, ref, norm_a, rel=1e-10):
    err = eig_err(got, ref, norm_a)
    assert len(err) == 0 or err.max() <= rel, (float(err.max()), int(np.argmax(err)))
