"""Stencil / FEM-like sparse matrices and dense vectors, seeded.

Grid points are numbered lexicographically with x fastest:
``i = x + nx*y + nx*ny*z``.  A stencil is a list of integer offsets; row ``i``
holds one stored entry for every offset whose target lies inside the grid
(Dirichlet boundary: out-of-grid neighbours are simply absent).  Offsets are
emitted in increasing linear offset, so column indices are sorted within each
row and the pattern of a full stencil is symmetric.

The five named workloads follow the benchmark configurations of this project
(2D/3D Laplacians and stencils in the size range of the regular class of the
paper's test suite, Section 5 and Table 1: N of 1-6 M, row density 2-35,
row-length variance at most 10).  The paper's own SuiteSparse matrices are not
used; these seeded stand-ins replace them.
"""

from __future__ import annotations

from dataclasses import dataclass, field
import itertools

import numpy as np


@dataclass
class CsrInput:
    """A square sparse matrix in CSR form plus its provenance.

    ``row_ptr`` is int32[n+1], ``col_idx`` int32[nnz] (sorted within rows, no
    duplicates), ``vals`` float64[nnz].
    """

    name: str
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    vals: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


def _streams(seed: int, count: int):
    """``count`` independent PCG64 generators derived from ``seed``."""
    children = np.random.SeedSequence(seed).spawn(count)
    return [np.random.Generator(np.random.PCG64(c)) for c in children]


# ---------------------------------------------------------------- patterns

STENCILS = {
    "2d5": [(dx, dy) for dx, dy in itertools.product((-1, 0, 1), repeat=2) if abs(dx) + abs(dy) <= 1],
    "2d9": [(dx, dy) for dx, dy in itertools.product((-1, 0, 1), repeat=2)],
    "3d7": [o for o in itertools.product((-1, 0, 1), repeat=3) if sum(map(abs, o)) <= 1],
    "3d19": [o for o in itertools.product((-1, 0, 1), repeat=3) if sum(map(abs, o)) <= 2],
    "3d27": [o for o in itertools.product((-1, 0, 1), repeat=3)],
}


def stencil_pattern(dims, kind: str):
    """CSR pattern of a stencil on a grid.

    Returns ``(row_ptr int32[n+1], col_idx int32[nnz], is_diag bool[nnz])``.
    """
    dims = tuple(int(d) for d in dims)
    offsets = STENCILS[kind]
    if len(offsets[0]) != len(dims):
        raise ValueError(f"stencil {kind} needs a {len(offsets[0])}-D grid")
    n = int(np.prod(dims))
    strides = [1]
    for d in dims[:-1]:
        strides.append(strides[-1] * d)
    lin = [sum(o[a] * strides[a] for a in range(len(dims))) for o in offsets]
    order = np.argsort(lin, kind="stable")
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx
    for d in dims:
        coords.append(rem % d)
        rem = rem // d
    valid = np.empty((n, len(offsets)), dtype=bool)
    cols = np.empty((n, len(offsets)), dtype=np.int64)
    diag = np.zeros((n, len(offsets)), dtype=bool)
    for j, oi in enumerate(order):
        o = offsets[oi]
        ok = np.ones(n, dtype=bool)
        for a, d in enumerate(dims):
            c = coords[a] + o[a]
            ok &= (c >= 0) & (c < d)
        valid[:, j] = ok
        cols[:, j] = idx + lin[oi]
        diag[:, j] = all(v == 0 for v in o)
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = cols[valid]
    is_diag = diag[valid]
    return row_ptr.astype(np.int32), col_idx.astype(np.int32), is_diag


def laplacian(dims, kind: str, diag_value: float, off_value: float = -1.0, name: str | None = None) -> CsrInput:
    """Stencil matrix with constant diagonal and off-diagonal values."""
    row_ptr, col_idx, is_diag = stencil_pattern(dims, kind)
    vals = np.where(is_diag, float(diag_value), float(off_value)).astype(np.float64)
    return CsrInput(name or f"{kind}_{'x'.join(map(str, dims))}", int(np.prod(dims)), row_ptr, col_idx, vals,
                    {"dims": tuple(dims), "stencil": kind, "is_diag": is_diag})


def diag_dominant_values(row_ptr, is_diag, rng, lo=0.5, hi=1.5, factor=1.1):
    """Off-diagonals ``-U[lo, hi]`` drawn in CSR order; diagonal = factor * row sum of |off-diagonals|."""
    nnz = int(row_ptr[-1])
    n = len(row_ptr) - 1
    off = ~is_diag
    vals = np.zeros(nnz, dtype=np.float64)
    vals[off] = -rng.uniform(lo, hi, size=int(off.sum()))
    rows = np.repeat(np.arange(n), np.diff(row_ptr.astype(np.int64)))
    absum = np.zeros(n, dtype=np.float64)
    np.add.at(absum, rows[off], np.abs(vals[off]))
    vals[is_diag] = factor * absum[rows[is_diag]]
    return vals


def drop_offdiagonals(row_ptr, col_idx, is_diag, rng, p: float):
    """Drop each stored off-diagonal independently with probability ``p`` (one uniform per off-diagonal, CSR order)."""
    off = ~is_diag
    u = rng.uniform(0.0, 1.0, size=int(off.sum()))
    keep = np.ones(len(col_idx), dtype=bool)
    keep[np.nonzero(off)[0][u < p]] = False
    n = len(row_ptr) - 1
    rows = np.repeat(np.arange(n), np.diff(row_ptr.astype(np.int64)))
    counts = np.bincount(rows[keep], minlength=n)
    new_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=new_ptr[1:])
    return new_ptr.astype(np.int32), col_idx[keep], is_diag[keep]


def scramble_symmetric(row_ptr, col_idx, vals, rng):
    """Relabel the grid points at random: B[i', j'] = A[p[i'], p[j']] for a uniform random permutation p.

    Returns the relabelled CSR (columns sorted within rows) and ``p``.  This
    produces an input whose natural order carries no band structure.
    """
    n = len(row_ptr) - 1
    p = rng.permutation(n).astype(np.int64)  # p[new] = old
    inv = np.empty(n, dtype=np.int64)
    inv[p] = np.arange(n)
    lengths = np.diff(row_ptr.astype(np.int64))
    new_len = lengths[p]
    new_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(new_len, out=new_ptr[1:])
    # gather the old rows in new order
    src = np.repeat(row_ptr[:-1].astype(np.int64)[p] - new_ptr[:-1], new_len) + np.arange(new_ptr[-1])
    new_cols = inv[col_idx.astype(np.int64)[src]]
    new_vals = vals[src]
    rows = np.repeat(np.arange(n), new_len)
    o = np.lexsort((new_cols, rows))
    return new_ptr.astype(np.int32), new_cols[o].astype(np.int32), new_vals[o], p


def uniform_vector(n: int, rng, nrhs: int = 1, round_to_f32: bool = False) -> np.ndarray:
    """U[-1, 1] in float64, shape (n,) or (n, nrhs) row-major; optionally rounded to float32-representable values."""
    shape = (n,) if nrhs == 1 else (n, nrhs)
    v = rng.uniform(-1.0, 1.0, size=shape)
    if round_to_f32:
        v = v.astype(np.float32).astype(np.float64)
    return v


def random_sparse(n: int, avg_per_row: float, seed: int, empty_row_frac: float = 0.0,
                  with_diag: bool = True, symmetric_pattern: bool = False, name: str = "random") -> CsrInput:
    """Small random square matrix (test helper): uniform random pattern, values U[-1, 1]."""
    rng_pat, rng_val, rng_empty = _streams(seed, 3)
    m = int(round(n * avg_per_row))
    r = rng_pat.integers(0, n, size=m) if n else np.zeros(0, np.int64)
    c = rng_pat.integers(0, n, size=m) if n else np.zeros(0, np.int64)
    if symmetric_pattern:
        r, c = np.concatenate([r, c]), np.concatenate([c, r])
    if with_diag and n:
        r = np.concatenate([r, np.arange(n)])
        c = np.concatenate([c, np.arange(n)])
    if empty_row_frac > 0 and n:
        empty = rng_empty.uniform(size=n) < empty_row_frac
        keep = ~empty[r]
        if symmetric_pattern:
            keep &= ~empty[c]
        r, c = r[keep], c[keep]
    key = np.unique(r.astype(np.int64) * max(n, 1) + c)
    r = key // max(n, 1)
    c = key % max(n, 1)
    counts = np.bincount(r, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    vals = rng_val.uniform(-1.0, 1.0, size=len(c))
    return CsrInput(name, n, row_ptr.astype(np.int32), c.astype(np.int32), vals, {"seed": seed})


# ---------------------------------------------------------------- workloads

def workload_c1(seed: int = 1):
    """2D 5-point Laplacian on 64x64 (n=4096): diagonal 4, off-diagonal -1, plus U[-0.1, 0.1]
    noise on every stored entry (CSR order); x ~ U[-1, 1]; float64."""
    rv, rx, rg = _streams(seed, 3)
    A = laplacian((64, 64), "2d5", 4.0)
    A.vals = A.vals + rv.uniform(-0.1, 0.1, size=A.nnz)
    A.name = "c1_2d5pt_64"
    return {"name": "c1", "A": A, "x": uniform_vector(A.n, rx), "g": uniform_vector(A.n, rg),
            "dtype": "f64", "nrhs": 1}


def workload_c2(seed: int = 2, side: int = 128):
    """3D 7-point Laplacian on side^3 (n=2.10M at side 128), values 6/-1, grid points relabelled by a
    seeded random permutation; x ~ U[-1, 1]; float64."""
    rp, rx, rg = _streams(seed, 3)
    L = laplacian((side, side, side), "3d7", 6.0)
    rp_, ci, v, p = scramble_symmetric(L.row_ptr, L.col_idx, L.vals, rp)
    A = CsrInput(f"c2_3d7pt_{side}_scrambled", L.n, rp_, ci, v, {"dims": (side,) * 3, "stencil": "3d7", "perm0": p})
    return {"name": "c2", "A": A, "x": uniform_vector(A.n, rx), "g": uniform_vector(A.n, rg),
            "dtype": "f64", "nrhs": 1}


def workload_c3(seed: int = 3, side: int = 100):
    """3D 27-point stencil on side^3 (n=1.0M at side 100), diagonally dominant: off-diagonal -U[0.5, 1.5],
    diagonal 1.1 * row sum of |off-diagonals|; x ~ U[-1, 1]; float64 master values."""
    rv, rx, rg = _streams(seed, 3)
    row_ptr, col_idx, is_diag = stencil_pattern((side, side, side), "3d27")
    vals = diag_dominant_values(row_ptr, is_diag, rv)
    A = CsrInput(f"c3_3d27pt_{side}", side ** 3, row_ptr, col_idx, vals, {"dims": (side,) * 3, "stencil": "3d27"})
    return {"name": "c3", "A": A, "x": uniform_vector(A.n, rx), "g": uniform_vector(A.n, rg),
            "dtype": "f64", "nrhs": 1}


def workload_c4(seed: int = 4, side: int = 2048):
    """2D 9-point stencil on side^2 (n=4.19M at side 2048) with 10% of off-diagonals dropped (nonsymmetric
    pattern); values as in c3, rounded to float32; x, g ~ U[-1, 1] rounded to float32."""
    rd, rv, rx, rg = _streams(seed, 4)
    row_ptr, col_idx, is_diag = stencil_pattern((side, side), "2d9")
    row_ptr, col_idx, is_diag = drop_offdiagonals(row_ptr, col_idx, is_diag, rd, 0.1)
    vals = diag_dominant_values(row_ptr, is_diag, rv).astype(np.float32).astype(np.float64)
    A = CsrInput(f"c4_2d9pt_{side}_drop10", side * side, row_ptr, col_idx, vals,
                 {"dims": (side, side), "stencil": "2d9", "drop": 0.1})
    return {"name": "c4", "A": A, "x": uniform_vector(A.n, rx, round_to_f32=True),
            "g": uniform_vector(A.n, rg, round_to_f32=True), "dtype": "f32", "nrhs": 1}


def workload_c5(seed: int = 5, count: int = 64, lo: int = 16, hi: int = 96, nrhs: int = 8):
    """``count`` 3D 7-point Laplacians (6/-1) with sides drawn uniformly from lo..hi inclusive, each with an
    n x nrhs block of right-hand sides (and adjoint seeds) ~ U[-1, 1] rounded to float32."""
    rs, rvec = _streams(seed, 2)
    sides = rs.integers(lo, hi + 1, size=count)
    mats, xs, gs = [], [], []
    vec_streams = [np.random.Generator(np.random.PCG64(c)) for c in np.random.SeedSequence(seed + 7919).spawn(2 * count)]
    for b, s in enumerate(sides):
        A = laplacian((int(s),) * 3, "3d7", 6.0, name=f"c5_{b}_3d7pt_{int(s)}")
        mats.append(A)
        xs.append(uniform_vector(A.n, vec_streams[2 * b], nrhs=nrhs, round_to_f32=True))
        gs.append(uniform_vector(A.n, vec_streams[2 * b + 1], nrhs=nrhs, round_to_f32=True))
    return {"name": "c5", "As": mats, "xs": xs, "gs": gs, "sides": sides, "dtype": "f32", "nrhs": nrhs}


def tuning_suite(seed: int = 11, scale: float = 1.0):
    """Matrices spanning the row-density axis used to fit a size model (regular class, sigma^2 <= 10).

    Each entry is a CsrInput; ``scale`` shrinks the grids for quick runs.
    """
    def s(v):
        return max(4, int(round(v * scale)))
    out = []
    streams = _streams(seed, 16)
    out.append(laplacian((s(1448), s(1448)), "2d5", 4.0, name="t_2d5pt"))
    out.append(laplacian((s(128), s(128), s(128)), "3d7", 6.0, name="t_3d7pt"))
    rp, ci, dg = stencil_pattern((s(1448), s(1448)), "2d9")
    out.append(CsrInput("t_2d9pt", len(rp) - 1, rp, ci, diag_dominant_values(rp, dg, streams[0]), {}))
    rp, ci, dg = stencil_pattern((s(110), s(110), s(110)), "3d19")
    out.append(CsrInput("t_3d19pt", len(rp) - 1, rp, ci, diag_dominant_values(rp, dg, streams[1]), {}))
    rp, ci, dg = stencil_pattern((s(100), s(100), s(100)), "3d27")
    out.append(CsrInput("t_3d27pt", len(rp) - 1, rp, ci, diag_dominant_values(rp, dg, streams[2]), {}))
    for k, (kind, dims, p) in enumerate([("3d7", (s(128),) * 3, 0.3), ("2d9", (s(1448),) * 2, 0.3),
                                        ("3d27", (s(100),) * 3, 0.5)]):
        rp, ci, dg = stencil_pattern(dims, kind)
        rp, ci, dg = drop_offdiagonals(rp, ci, dg, streams[3 + k], p)
        out.append(CsrInput(f"t_{kind}_drop{int(p * 100)}", len(rp) - 1, rp, ci,
                            diag_dominant_values(rp, dg, streams[6 + k]), {}))
    return out


WORKLOADS = {"c1": workload_c1, "c2": workload_c2, "c3": workload_c3, "c4": workload_c4, "c5": workload_c5}
