"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module builds inputs only: it holds none of the eigen-solver's arithmetic.

* Finite-difference Laplacians of the kind used in the paper's experiments
  (Section 4.1, Table ``tab:lap``): the 5-point stencil on an N x N grid and the
  7-point stencil on an N x N x N grid, Dirichlet boundary, mesh width h = 1
  (diagonal 4 or 6, off-diagonal -1), lexicographic ordering with x fastest.
* An optional diagonal potential V with entries uniform in [0, 1) drawn from a
  counter-based generator, so that the matrix is ``L + diag(scale * V)``.
* Counter-based random numbers: SplitMix64 (Steele, Lea and Flood, "Fast
  splittable pseudorandom number generators", OOPSLA 2014), used as a stateless
  stream: element ``i`` of stream ``seed`` is the (i+1)-th output of SplitMix64
  whose state starts at ``seed``.

The CSR layout is the one the library expects: ``row_ptr`` int32 of length
n+1, ``col`` int32 ascending within each row (diagonal present), ``val``
float64.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, index) -> np.ndarray:
    """SplitMix64 output number ``index + 1`` of the generator seeded with ``seed``.

    ``index`` may be an int or an integer array; returns uint64 of the same shape.
    """
    idx = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (idx + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, index) -> np.ndarray:
    """Doubles in [0, 1): the top 53 bits of the SplitMix64 output times 2^-53."""
    return (splitmix64(seed, index) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def rademacher(seed: int, n: int, nvec: int) -> np.ndarray:
    """n x nvec row-major block of +-1: element (i, l) takes the sign from the top
    bit of output ``l * n + i`` (top bit set -> -1)."""
    i = np.arange(n, dtype=np.uint64)[:, None]
    l = np.arange(nvec, dtype=np.uint64)[None, :]
    bits = splitmix64(seed, l * np.uint64(n) + i) >> np.uint64(63)
    return np.where(bits == 1, -1.0, 1.0)


def potential(seed: int, n: int) -> np.ndarray:
    """Diagonal potential V_i = uniform01(seed, i), i = 0..n-1."""
    return uniform01(seed, np.arange(n, dtype=np.uint64))


class CSR:
    """Host CSR matrix (int32 row_ptr/col, float64 val)."""

    def __init__(self, n, row_ptr, col, val, grid=None, dim=None):
        self.n = int(n)
        self.row_ptr = row_ptr
        self.col = col
        self.val = val
        self.grid = grid
        self.dim = dim

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def diag(self) -> np.ndarray:
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        d = np.zeros(self.n)
        m = rows == self.col
        d[rows[m]] = self.val[m]
        return d

    def to_dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        a[rows, self.col] = self.val
        return a


def laplacian(N: int, dim: int, pot_seed: int | None = None, pot_scale: float = 1.0) -> CSR:
    """Dirichlet FD Laplacian on an N^dim grid (dim = 2: 5-point, dim = 3: 7-point),
    h = 1, plus ``pot_scale * potential(pot_seed)`` on the diagonal when a seed is
    given."""
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    n = N ** dim
    if n >= 2 ** 31 // 8:
        raise ValueError("grid too large for int32 CSR")
    p = np.arange(n, dtype=np.int64)
    coords = []
    rem = p
    for _ in range(dim):
        coords.append(rem % N)
        rem = rem // N
    # neighbour offsets in ascending column order: -N^{d-1} ... -1, 0, +1 ... +N^{d-1}
    offs, masks = [], []
    for ax in reversed(range(dim)):
        offs.append(-(N ** ax))
        masks.append(coords[ax] > 0)
    offs.append(0)
    masks.append(np.ones(n, dtype=bool))
    for ax in range(dim):
        offs.append(N ** ax)
        masks.append(coords[ax] < N - 1)
    offs = np.array(offs, dtype=np.int64)
    mask = np.stack(masks, axis=1)                     # n x (2 dim + 1)
    cols = p[:, None] + offs[None, :]
    center = 2.0 * dim
    vals = np.where(offs[None, :] == 0, center, -1.0) * np.ones((n, 1))
    if pot_seed is not None:
        vals[:, dim] += pot_scale * potential(pot_seed, n)
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = cols[mask].astype(np.int32)
    val = vals[mask].astype(np.float64)
    return CSR(n, row_ptr.astype(np.int32), col, val, grid=N, dim=dim)


def lanczos_start(seed: int, n: int, restart: int = 0) -> np.ndarray:
    """Start vector of a Lanczos run: entries 2u - 1 with u = uniform01(seed, restart * n + i).
    Not normalised."""
    idx = np.uint64(restart) * np.uint64(n) + np.arange(n, dtype=np.uint64)
    return 2.0 * uniform01(seed, idx) - 1.0


def fe_pencil(N: int) -> tuple:
    """Bilinear finite-element pencil on an N x N interior grid of the unit
    square (Dirichlet), without the mesh factors: stiffness
    A = K1 (x) M1 + M1 (x) K1 and mass B = M1 (x) M1 with K1 = tridiag(-1, 2, -1)
    and M1 = tridiag(1, 4, 1) / 6 (both N x N). 9-point CSR, x fastest, columns
    ascending; B is SPD with eigenvalues in (1/9, 1)."""
    K1 = {-1: -1.0, 0: 2.0, 1: -1.0}
    M1 = {-1: 1.0 / 6.0, 0: 4.0 / 6.0, 1: 1.0 / 6.0}
    n = N * N
    p = np.arange(n, dtype=np.int64)
    ix, iy = p % N, p // N
    cols, va, vb, mask = [], [], [], []
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            ok = (ix + dx >= 0) & (ix + dx < N) & (iy + dy >= 0) & (iy + dy < N)
            cols.append(p + dy * N + dx)
            # A = K1(x) M1(y) + M1(x) K1(y); B = M1(x) M1(y)
            va.append(np.full(n, K1[dx] * M1[dy] + M1[dx] * K1[dy]))
            vb.append(np.full(n, M1[dx] * M1[dy]))
            mask.append(ok)
    cols = np.stack(cols, axis=1)
    va, vb, mask = np.stack(va, axis=1), np.stack(vb, axis=1), np.stack(mask, axis=1)
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = cols[mask].astype(np.int32)
    A = CSR(n, row_ptr.astype(np.int32), col, va[mask].astype(np.float64), grid=N, dim=2)
    B = CSR(n, row_ptr.astype(np.int32), col.copy(), vb[mask].astype(np.float64), grid=N, dim=2)
    return A, B
