"""Seeded synthetic workloads for the simultaneous short-recurrence Krylov solvers.

This module builds test problems only: sparse matrices in CSR form and blocks of
right-hand sides.  It holds none of the solvers' arithmetic and is the one piece
of code that both the CPU oracle (``oracle/``) and the GPU path's tests and
benchmark use, so that both see byte-identical inputs.

Every generator is deterministic for a given seed (numpy PCG64 via
``numpy.random.default_rng``).  Matrices are returned as :class:`CSR` with
int64 row pointers, int32 sorted column indices and float64 / complex128
values.

Problem families (the paper's experiments, Section 5, and the stand-ins used
where the paper's matrices are not available):

* ``convdiff2d`` / ``convdiff3d``: central-difference convection-diffusion
  stencils (5- and 7-point), scaled by h^2, Dirichlet boundaries.  These cover
  the paper's Examples 1-3 and the 2D/3D workloads.
* ``wilson4d``: a Wilson-type nearest-neighbour operator on a periodic 4D
  lattice with 12 unknowns per site and Haar-random U(3) links.  It stands in
  for the lattice-QCD matrix of Example 4 (49 nonzeros per row, spectrum
  symmetric about the real axis, right half-plane).
* ``powerlaw``: a random complex sparse matrix with power-law row lengths,
  uniformly random columns and a strictly dominant diagonal.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "CSR", "convdiff2d", "convdiff3d", "wilson4d", "powerlaw", "powerlaw_exponent",
    "gaussian_block", "unit_block", "config", "CONFIGS",
]


@dataclass
class CSR:
    """Compressed sparse row matrix (square, n x n)."""

    n: int
    indptr: np.ndarray   # int64, length n+1
    indices: np.ndarray  # int32, length nnz, sorted within each row
    data: np.ndarray     # float64 or complex128, length nnz

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    @property
    def is_complex(self) -> bool:
        return np.iscomplexobj(self.data)

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_array((self.data, self.indices, self.indptr), shape=(self.n, self.n))


def _assemble(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> CSR:
    """Sort (row, col) triplets into CSR.  Triplets must be unique."""
    order = np.lexsort((cols, rows))
    rows = rows[order]
    cols = cols[order].astype(np.int32)
    vals = vals[order]
    counts = np.bincount(rows, minlength=n)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    return CSR(n, indptr, np.ascontiguousarray(cols), np.ascontiguousarray(vals))


def _stencil(shape: tuple[int, ...], centre: float, minus: list[float], plus: list[float]) -> CSR:
    """Constant-coefficient stencil on a lexicographically ordered grid (first axis
    fastest).  ``minus[d]`` couples to the neighbour at index-1 along axis d,
    ``plus[d]`` to index+1; off-grid neighbours are dropped (Dirichlet)."""
    dims = len(shape)
    n = int(np.prod(shape))
    idx = np.arange(n, dtype=np.int64)
    coord = []
    stride = 1
    strides = []
    for d in range(dims):
        coord.append((idx // stride) % shape[d])
        strides.append(stride)
        stride *= shape[d]
    rows = [idx]
    cols = [idx]
    vals = [np.full(n, centre, dtype=np.float64)]
    for d in range(dims):
        m = coord[d] > 0
        rows.append(idx[m]); cols.append(idx[m] - strides[d]); vals.append(np.full(m.sum(), minus[d]))
        m = coord[d] < shape[d] - 1
        rows.append(idx[m]); cols.append(idx[m] + strides[d]); vals.append(np.full(m.sum(), plus[d]))
    return _assemble(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def convdiff2d(m: int, beta=(20.0, 20.0), reaction: float = 0.0) -> CSR:
    """-u_xx - u_yy + beta . grad u + reaction * u on an m x m interior grid of the
    unit square, h = 1/(m+1), central differences, all entries multiplied by h^2:
    centre 4 + reaction*h^2, west/east -1 -/+ beta_x h/2, south/north -1 -/+ beta_y h/2.
    Rows are ordered with x fastest."""
    h = 1.0 / (m + 1)
    minus = [-1.0 - beta[0] * h / 2, -1.0 - beta[1] * h / 2]
    plus = [-1.0 + beta[0] * h / 2, -1.0 + beta[1] * h / 2]
    return _stencil((m, m), 4.0 + reaction * h * h, minus, plus)


def convdiff3d(m: int, beta=(30.0, 20.0, 10.0), reaction: float = 0.0) -> CSR:
    """3D analogue of :func:`convdiff2d` (7-point stencil, centre 6, x fastest)."""
    h = 1.0 / (m + 1)
    minus = [-1.0 - b * h / 2 for b in beta]
    plus = [-1.0 + b * h / 2 for b in beta]
    return _stencil((m, m, m), 6.0 + reaction * h * h, minus, plus)


# Euclidean gamma matrices used by wilson4d: Gamma_k = sigma_2 (x) sigma_k for
# k = 1, 2, 3 and Gamma_4 = sigma_1 (x) I_2.  They are Hermitian, unitary and
# mutually anticommuting, and each has exactly one nonzero per row.
_S1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_S2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_S3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
_I2 = np.eye(2, dtype=np.complex128)
GAMMAS = [np.kron(_S2, _S1), np.kron(_S2, _S2), np.kron(_S2, _S3), np.kron(_S1, _I2)]


def haar_u3(rng: np.random.Generator, count: int) -> np.ndarray:
    """``count`` Haar-distributed 3x3 unitaries: QR of a complex Ginibre matrix
    with the phases of R's diagonal moved into Q (Mezzadri, 2007)."""
    z = rng.standard_normal((count, 3, 3)) + 1j * rng.standard_normal((count, 3, 3))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    ph = d / np.abs(d)
    return q * ph[:, None, :]


def wilson4d(L: int = 16, mass: float = 0.1, seed: int = 2) -> CSR:
    """Wilson-type operator on an L^4 periodic lattice, 12 unknowns per site
    (row = 12*site + 3*spin + colour, site index with x0 fastest):

        A = (4 + m) I - 1/2 sum_mu [ (I - Gamma_mu) (x) U_mu(x) T_{+mu}
                                   + (I + Gamma_mu) (x) U_mu(x - mu)^H T_{-mu} ].

    Links U_mu(x) are Haar U(3), drawn for mu = 0..3 and, within mu, sites in
    order.  This is D_W = I - kappa D of the paper's Example 4 up to the factor
    1/(2 kappa) with kappa = 1/(8 + 2m); it has 49 nonzeros per row."""
    rng = np.random.default_rng(seed)
    V = L ** 4
    U = haar_u3(rng, 4 * V).reshape(4, V, 3, 3)
    n = 12 * V
    site = np.arange(V, dtype=np.int64)
    x = [(site // L ** d) % L for d in range(4)]

    def shift(mu, step):
        xs = [c.copy() for c in x]
        xs[mu] = (xs[mu] + step) % L
        return xs[0] + L * (xs[1] + L * (xs[2] + L * xs[3]))

    rows, cols, vals = [], [], []
    # diagonal
    rows.append(np.arange(n, dtype=np.int64)); cols.append(np.arange(n, dtype=np.int64))
    vals.append(np.full(n, 4.0 + mass, dtype=np.complex128))
    a_s, b_s = np.meshgrid(np.arange(4), np.arange(4), indexing="ij")   # spin row, spin col
    a_c, b_c = np.meshgrid(np.arange(3), np.arange(3), indexing="ij")   # colour row, colour col
    I4 = np.eye(4, dtype=np.complex128)
    for mu in range(4):
        fwd = shift(mu, +1)
        bwd = shift(mu, -1)
        for sign, nbr, link in ((-1.0, fwd, U[mu]),                                   # (I - Gamma) U(x) T+
                                (+1.0, bwd, np.conj(np.transpose(U[mu][bwd], (0, 2, 1))))):  # (I + Gamma) U(x-mu)^H T-
            spin = -0.5 * (I4 + sign * GAMMAS[mu])
            for sa in range(4):
                for sb in range(4):
                    g = spin[sa, sb]
                    if g == 0:
                        continue
                    for ca in range(3):
                        for cb in range(3):
                            rows.append(12 * site + 3 * sa + ca)
                            cols.append(12 * nbr + 3 * sb + cb)
                            vals.append(g * link[:, ca, cb])
    rows = np.concatenate(rows); cols = np.concatenate(cols); vals = np.concatenate(vals)
    return _assemble(n, rows, cols, vals)


def powerlaw_exponent(lo: int = 4, hi: int = 400, mean: float = 20.0) -> float:
    """Exponent a with sum_L L * L^-a / sum_L L^-a = mean over L in [lo, hi]
    (bisection; the mean decreases monotonically in a)."""
    Ls = np.arange(lo, hi + 1, dtype=np.float64)

    def m(a):
        w = Ls ** (-a)
        return float((Ls * w).sum() / w.sum())

    a0, a1 = 0.0, 5.0
    for _ in range(200):
        am = 0.5 * (a0 + a1)
        if m(am) > mean:
            a0 = am
        else:
            a1 = am
    return 0.5 * (a0 + a1)


def powerlaw(n: int = 1 << 20, seed: int = 2, lo: int = 4, hi: int = 400, mean: float = 20.0) -> CSR:
    """Random complex sparse matrix.

    Row i has L_i off-diagonal entries with P(L) proportional to L^-a on
    {lo..hi} (a from :func:`powerlaw_exponent`, so E[L] = ``mean``; capped at
    n-1).  Columns are distinct, uniform over j != i: drawn with replacement,
    then duplicates inside a row are redrawn until none remain.  Values are
    (N(0,1) + i N(0,1)) / sqrt(L_i); the diagonal is 2 + sum_j |a_ij|, which makes
    the matrix strictly diagonally dominant (nonsingular)."""
    rng = np.random.default_rng(seed)
    a = powerlaw_exponent(lo, hi, mean)
    Ls = np.arange(lo, hi + 1)
    p = Ls.astype(np.float64) ** (-a)
    p /= p.sum()
    L = rng.choice(Ls, size=n, p=p)
    L = np.minimum(L, n - 1).astype(np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), L)
    cols = rng.integers(0, n - 1, size=rows.size, dtype=np.int64)
    while True:
        order = np.lexsort((cols, rows))
        rows = rows[order]; cols = cols[order]
        dup = np.zeros(rows.size, dtype=bool)
        dup[1:] = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        k = int(dup.sum())
        if k == 0:
            break
        cols[dup] = rng.integers(0, n - 1, size=k, dtype=np.int64)
    cols = cols + (cols >= rows)          # skip the diagonal
    # after the shift the per-row order is preserved (monotone map per row)
    Lr = L[rows]
    vals = (rng.standard_normal(rows.size) + 1j * rng.standard_normal(rows.size)) / np.sqrt(Lr)
    diag = 2.0 + np.bincount(rows, weights=np.abs(vals), minlength=n)
    allr = np.concatenate([rows, np.arange(n, dtype=np.int64)])
    allc = np.concatenate([cols, np.arange(n, dtype=np.int64)])
    allv = np.concatenate([vals, diag.astype(np.complex128)])
    return _assemble(n, allr, allc, allv)


def gaussian_block(n: int, s: int, seed: int = 0, complex_: bool = False) -> np.ndarray:
    """n x s block with i.i.d. N(0,1) entries (real part first, then imaginary
    part, for complex blocks); row-major (C order)."""
    rng = np.random.default_rng(seed)
    if complex_:
        re = rng.standard_normal((n, s))
        im = rng.standard_normal((n, s))
        return np.ascontiguousarray(re + 1j * im)
    return np.ascontiguousarray(rng.standard_normal((n, s)))


def unit_block(n: int, s: int, complex_: bool = True) -> np.ndarray:
    """[e_0 | ... | e_{s-1}]: the first s unit vectors."""
    B = np.zeros((n, s), dtype=np.complex128 if complex_ else np.float64)
    B[np.arange(s), np.arange(s)] = 1.0
    return B


# ---------------------------------------------------------------------------
# The paper's Examples 1-3 (Section 5.1), central differences on an equispaced
# interior grid, all rows multiplied by h^2, x fastest.  Only the structure the
# section fixes is reproduced: the discretisation details it leaves open (and
# the preconditioners of its second table) are not.
# ---------------------------------------------------------------------------
def _grid_coords(shape):
    n = int(np.prod(shape))
    idx = np.arange(n, dtype=np.int64)
    out, stride = [], 1
    for m in shape:
        out.append((idx // stride) % m)
        stride *= m
    return out


def paper_example1(m: int = 200, alpha=(5.0, 5.0, 5.0)):
    """Example 1: -u_xx - u_yy + 2 a1 u_x + 2 a2 u_y - 2 a3 u = 0 on the unit square
    (a1 = a2 = a3 = 5), m x m interior points, h = 1/(m+1).  Four right-hand
    sides, one per corner: Dirichlet data continuous and piecewise linear along
    the boundary, 1 at that corner and 0 at the other three.  A boundary value
    g enters the row of its interior neighbour as -(coupling) * g."""
    a1, a2, a3 = alpha
    h = 1.0 / (m + 1)
    west, east = -1.0 - a1 * h, -1.0 + a1 * h
    south, north = -1.0 - a2 * h, -1.0 + a2 * h
    A = _stencil((m, m), 4.0 - 2.0 * a3 * h * h, [west, south], [east, north])
    ix, iy = _grid_coords((m, m))
    x = (ix + 1) * h
    y = (iy + 1) * h
    corners = [(0.0, 0.0), (1.0, 0.0), (0.0, 1.0), (1.0, 1.0)]

    def g(cx, cy, px, py):
        # hat function of the corner along the boundary: linear on each edge
        return np.maximum(0.0, 1.0 - np.abs(px - cx) - np.abs(py - cy)) * \
            ((np.isclose(px, cx)) | (np.isclose(py, cy)))

    B = np.zeros((m * m, 4))
    for k, (cx, cy) in enumerate(corners):
        b = np.zeros(m * m)
        b -= np.where(ix == 0, west * g(cx, cy, 0.0 * x, y), 0.0)
        b -= np.where(ix == m - 1, east * g(cx, cy, 0.0 * x + 1.0, y), 0.0)
        b -= np.where(iy == 0, south * g(cx, cy, x, 0.0 * y), 0.0)
        b -= np.where(iy == m - 1, north * g(cx, cy, x, 0.0 * y + 1.0), 0.0)
        B[:, k] = b
    return A, B


def paper_example2(m: int = 50, nu: float = 1000.0):
    """Example 2 (Example 3 with nu = 10): u_xx + u_yy + u_zz + nu u_x = f on the
    unit cube, m^3 interior points, h = 1/(m+1); the rows are multiplied by
    -h^2 (centre 6, x-neighbours -1 -/+ nu h / 2, others -1).  19 right-hand
    sides: f from the exact solution u = exp(xyz) sin(pi x) sin(pi y) sin(pi z)
    with zero boundary data, and 18 with f = 0 and, on one face at a time, the
    boundary data equal to each of its two tangential coordinates and to 1."""
    h = 1.0 / (m + 1)
    c = nu * h / 2.0
    minus = [-1.0 + c, -1.0, -1.0]       # -(1 - nu h / 2) for the west neighbour
    plus = [-1.0 - c, -1.0, -1.0]        # -(1 + nu h / 2) for the east neighbour
    A = _stencil((m, m, m), 6.0, minus, plus)
    ix, iy, iz = _grid_coords((m, m, m))
    x, y, z = (ix + 1) * h, (iy + 1) * h, (iz + 1) * h
    n = m ** 3
    cols = []
    # f = Laplace(u) + nu u_x for u = exp(xyz) sin(pi x) sin(pi y) sin(pi z)
    e = np.exp(x * y * z)
    sx, sy, sz = np.sin(np.pi * x), np.sin(np.pi * y), np.sin(np.pi * z)
    cx_, cy_, cz_ = np.cos(np.pi * x), np.cos(np.pi * y), np.cos(np.pi * z)
    pi = np.pi

    def d2(a, b, c_, s_, co):   # second derivative along the axis with product coordinate a*b
        return e * ((a * b) ** 2 * s_ + 2 * pi * a * b * co - pi * pi * s_)

    uxx = d2(y, z, None, sx, cx_) * sy * sz
    uyy = d2(x, z, None, sy, cy_) * sx * sz
    uzz = d2(x, y, None, sz, cz_) * sx * sy
    ux = e * (y * z * sx + pi * cx_) * sy * sz
    f = uxx + uyy + uzz + nu * ux
    cols.append(-h * h * f)
    coord = {"x": x, "y": y, "z": z}
    faces = [("x", 0, ix == 0, minus[0]), ("x", 1, ix == m - 1, plus[0]),
             ("y", 0, iy == 0, minus[1]), ("y", 1, iy == m - 1, plus[1]),
             ("z", 0, iz == 0, minus[2]), ("z", 1, iz == m - 1, plus[2])]
    for axis, side, mask, coup in faces:
        tang = [a for a in ("x", "y", "z") if a != axis]
        for gfun in (coord[tang[0]], coord[tang[1]], np.ones(n)):
            cols.append(np.where(mask, -coup * gfun, 0.0))
    return A, np.stack(cols, axis=1)


def paper_example(k: int, scale: str = "full") -> Problem:
    """Examples 1-3 of Section 5.1 (full size: 200^2 with s = 4; 50^3 with
    s = 19).  ``scale='small'`` keeps the equations and right-hand sides on a
    coarser grid (40^2, 12^3)."""
    small = scale == "small"
    if k == 1:
        A, B = paper_example1(40 if small else 200)
        name = "paper-ex1"
    elif k in (2, 3):
        A, B = paper_example2(12 if small else 50, 1000.0 if k == 2 else 10.0)
        name = f"paper-ex{k}"
    else:
        raise ValueError(k)
    return Problem(name + ("-small" if small else ""), A, B,
                   ("bl_bicg", "bl_bicg_rq", "bl_bicgstab", "bl_bicgstab_rq"), {})


@dataclass
class Problem:
    name: str
    A: CSR
    B: np.ndarray
    methods: tuple
    extra: dict


def config(k: int, scale: str = "full") -> Problem:
    """The five workloads.  ``scale='small'`` gives a scaled-down problem of the
    same family and structure for parity tests (same seeds, smaller grid)."""
    small = scale == "small"
    if k == 1:
        A = convdiff2d(32, (20.0, 20.0))
        B = gaussian_block(A.n, 4, seed=0)
        return Problem("convdiff2d-32x32-s4", A, B, ("gl_bicg", "egl_bicg"), {})
    if k == 2:
        m = 16 if small else 128
        A = convdiff3d(m, (30.0, 20.0, 10.0))
        B = gaussian_block(A.n, 16, seed=0)
        return Problem(f"convdiff3d-{m}^3-s16", A, B, ("bl_bicg_rq", "egl_qmr", "bl_bicgstab_rq"), {})
    if k == 3:
        L = 4 if small else 16
        A = wilson4d(L, 0.1, seed=2)
        B = unit_block(A.n, 12, complex_=True)
        return Problem(f"wilson4d-{L}^4x12-s12", A, B,
                       ("gl_bicg", "egl_bicg", "gl_qmr", "egl_qmr", "gl_bicgstab", "bl_bicg_rq", "bl_bicgstab_rq"), {})
    if k == 4:
        n = (1 << 14) if small else (1 << 20)
        A = powerlaw(n, seed=2)
        B = gaussian_block(n, 32, seed=0, complex_=True)
        return Problem(f"powerlaw-n{n}-s32", A, B, ("egl_bicg", "bl_bicgstab_rq"), {})
    if k == 5:
        m = 64 if small else 1024
        A = convdiff2d(m, (20.0, 20.0))
        B = gaussian_block(A.n, 8, seed=0)
        Xt = gaussian_block(A.n, 8, seed=1)
        return Problem(f"convdiff2d-{m}x{m}-s8-grad", A, B, ("egl_bicg",), {"X_target": Xt})
    raise ValueError(k)


CONFIGS = (1, 2, 3, 4, 5)
