"""Closed-form spectra of the Dirichlet finite-difference Laplacians (h = 1).

The 5-point operator on an N x N grid has eigenvalues
4 - 2 cos(i pi/(N+1)) - 2 cos(j pi/(N+1)), i, j = 1..N, with eigenvectors
sin(i pi x/(N+1)) sin(j pi y/(N+1)); the 7-point operator on N^3 adds the third
factor (diagonal 6). These are the exact answers the oracle is pinned to.
"""
import numpy as np


def lap_eigs(N, dim):
    c = 2.0 - 2.0 * np.cos(np.arange(1, N + 1) * np.pi / (N + 1))
    if dim == 2:
        e = c[:, None] + c[None, :]
    else:
        e = c[:, None, None] + c[None, :, None] + c[None, None, :]
    return np.sort(e.ravel())


def lap_count(N, dim, lo, hi):
    """Number of eigenvalues in [lo, hi], counted by sorting only the 1-D factors."""
    c = np.sort(2.0 - 2.0 * np.cos(np.arange(1, N + 1) * np.pi / (N + 1)))
    if dim == 2:
        s = c[:, None] + c[None, :]
        return int(np.count_nonzero((s >= lo) & (s <= hi)))
    tot = 0
    for ci in c:
        s = ci + c[:, None] + c[None, :]
        tot += int(np.count_nonzero((s >= lo) & (s <= hi)))
    return tot


def lap_eigvec(N, dim, modes):
    """Unnormalised eigenvector for the mode tuple (1-based), x fastest."""
    x = np.arange(1, N + 1)
    f = [np.sin(k * np.pi * x / (N + 1)) for k in modes]
    if dim == 2:
        v = f[1][:, None] * f[0][None, :]
    else:
        v = f[2][:, None, None] * f[1][None, :, None] * f[0][None, None, :]
    return v.ravel()


def lap_eig_of(N, modes):
    return float(sum(2.0 - 2.0 * np.cos(k * np.pi / (N + 1)) for k in modes))
