"""Seeded synthetic stand-ins for compressed wavelet Galerkin matrices.

The paper's matrices (benzene PCM surface, unit disc, L-shaped domain with
holes; Sections 6.1-6.3) are not available, so this module builds matrices
with the same *structure*: a 2D isotropic Haar basis on a uniform 2^G x 2^G
grid of [0,1]^2, compressed by the first term of the a-priori cut-off of
Theorem 3.1 (keep an entry iff the distance of the two supports is at most
a * 2^-min(j,j')), with values that decay across levels and with distance as
the decay estimate of Section 3 suggests, and a diagonal that makes the matrix
strictly diagonally dominant, hence SPD.

Nothing here belongs to the factorization: this module only produces inputs.
Both the CPU oracle and the HIP library consume its output; it imports
neither of them.

Index model (the "canonical levelwise ordering" of Section 4):
  * index 0 is the scaling function, support [0,1]^2, level 0;
  * wavelet (j, k1, k2, t), t in {0,1,2}, has index 4^j + 3*(k2*2^j + k1) + t
    and support [k1, k1+1] x [k2, k2+1] * 2^-j, for levels j = 0..G-1,
  so N = 4^G and level j occupies indices [4^j, 4^(j+1)).

Distances are computed exactly in integer units of the grid spacing 2^-G.
The random factor xi in (-1,1) of an entry {i,j} is a counter-based draw,
SplitMix64 (Steele, Lea, Flood 2014) of seed XOR ((min << 32) | max), so the
value of an entry does not depend on the order in which pairs are visited.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

_U64 = np.uint64


def splitmix64(x: np.ndarray) -> np.ndarray:
    """One SplitMix64 output for each uint64 state in ``x`` (wrapping arithmetic)."""
    z = x.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z += _U64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> _U64(30))) * _U64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> _U64(27))) * _U64(0x94D049BB133111EB)
    return z ^ (z >> _U64(31))


def pair_uniform(seed: int, i: np.ndarray, j: np.ndarray) -> np.ndarray:
    """xi = 2u - 1 with u in [0,1) from the 53 top bits of SplitMix64(seed ^ mix(i,j))."""
    lo = np.minimum(i, j).astype(np.uint64)
    hi = np.maximum(i, j).astype(np.uint64)
    key = (lo << _U64(32)) | hi
    key ^= _U64(seed & 0xFFFFFFFFFFFFFFFF)
    u = (splitmix64(key) >> _U64(11)).astype(np.float64) * (2.0 ** -53)
    return 2.0 * u - 1.0


@dataclasses.dataclass(frozen=True)
class WaveletSpec:
    """Parameters of one synthetic instance.

    grid_exp: G, the grid is 2^G x 2^G and the wavelet levels are 0..G-1.
    a: cut-off constant of the a-priori compression (Theorem 3.1, first term).
    s: order parameter; the diagonal carries 2^(2 j s).
    kind: "exp"  -> off-diagonal 2^(-decay*|dj|) * exp(-|dc|/ell) * xi
          "alg"  -> off-diagonal 2^(-(1+s)*|dj|) * (1 + |dc|/h)^(-(2+2s)) * xi,
                    h = 2^-G (the grid spacing).
    seed: seed of the entry draws xi.
    """

    grid_exp: int
    a: float
    s: float
    kind: str = "exp"
    ell: float = 0.3
    decay: float = 1.5
    seed: int = 1000

    @property
    def n(self) -> int:
        return 4 ** self.grid_exp


def basis(G: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Level, cell x and cell y of every index in canonical levelwise order."""
    n = 4 ** G
    level = np.zeros(n, np.int32)
    kx = np.zeros(n, np.int64)
    ky = np.zeros(n, np.int64)
    for j in range(G):
        nj = 1 << j
        base = 4 ** j
        cells = np.arange(nj * nj, dtype=np.int64)
        ids = base + 3 * cells
        for t in range(3):
            level[ids + t] = j
            kx[ids + t] = cells % nj
            ky[ids + t] = cells // nj
    return level, kx, ky


def centers(G: int) -> Tuple[np.ndarray, np.ndarray]:
    """(N,2) support centres in [0,1]^2 and the level of every index."""
    level, kx, ky = basis(G)
    size = 2.0 ** (-level.astype(np.float64))
    c = np.stack([(kx + 0.5) * size, (ky + 0.5) * size], axis=1)
    return c, level


def _cell_functions(j: int, cells: np.ndarray, nj: int) -> List[np.ndarray]:
    """Indices of the functions living on the given cells of level j (one array per type)."""
    if j == 0:
        return [np.zeros_like(cells), cells * 0 + 1, cells * 0 + 2, cells * 0 + 3]
    base = 4 ** j
    return [base + 3 * cells + t for t in range(3)]


def _offsets_1d(r: int, S: int, sp: int, W: int) -> Tuple[np.ndarray, np.ndarray]:
    o = np.arange(-1 - W, r + W + 1, dtype=np.int64)
    gap = np.where(o >= r, o * sp - S, np.where(o < 0, -(o + 1) * sp, 0))
    return o, gap


def _pairs_1d(nj: int, njp: int, r: int, S: int, sp: int, W: int):
    """All (coarse k, fine m, integer gap) per dimension with the fine cell inside the grid."""
    o, gap = _offsets_1d(r, S, sp, W)
    k = np.repeat(np.arange(nj, dtype=np.int64), o.size)
    oo = np.tile(o, nj)
    gg = np.tile(gap, nj)
    m = k * r + oo
    ok = (m >= 0) & (m < njp)
    return k[ok], m[ok], gg[ok]


def _level_pair_entries(spec: WaveletSpec, j: int, jp: int):
    """Lower-triangle off-diagonal pairs (row, col) between levels j <= jp, plus the
    squared centre distance (grid units) of each pair."""
    G = spec.grid_exp
    nj, njp = 1 << j, 1 << jp
    r = 1 << (jp - j)
    S, sp = 1 << (G - j), 1 << (G - jp)
    thr = spec.a * float(1 << (G - j))        # a * 2^-min(j,j') in grid units
    thr2 = thr * thr
    W = int(math.floor(thr / sp))
    kx, mx, gx = _pairs_1d(nj, njp, r, S, sp, W)
    rows, cols, d2s = [], [], []
    # cross product of the x and y one-dimensional pair lists, in chunks
    ny = kx.size
    chunk = max(1, (1 << 22) // max(1, ny))
    for start in range(0, kx.size, chunk):
        sl = slice(start, min(kx.size, start + chunk))
        ax_k, ax_m, ax_g = kx[sl], mx[sl], gx[sl]
        # outer: x-pair index p, y-pair index q
        gxx = ax_g[:, None]
        g2 = (gxx * gxx + (gx * gx)[None, :]).astype(np.float64)
        keep = g2 <= thr2
        p, q = np.nonzero(keep)
        if p.size == 0:
            continue
        ckx, cmx = ax_k[p], ax_m[p]
        cky, cmy = kx[q], mx[q]
        ccell = cky * nj + ckx
        fcell = cmy * njp + cmx
        # centre distance squared in grid units (times 4 to stay integral)
        dx2 = (2 * cmx + 1) * sp - (2 * ckx + 1) * S
        dy2 = (2 * cmy + 1) * sp - (2 * cky + 1) * S
        cd4 = dx2 * dx2 + dy2 * dy2
        cf = _cell_functions(j, ccell, nj)
        ff = _cell_functions(jp, fcell, njp)
        for a_ids in cf:
            for b_ids in ff:
                if j == jp:
                    lower = b_ids > a_ids
                    rows.append(b_ids[lower]); cols.append(a_ids[lower]); d2s.append(cd4[lower])
                else:
                    rows.append(b_ids); cols.append(a_ids); d2s.append(cd4)
    if not rows:
        e = np.zeros(0, np.int64)
        return e, e, e
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(d2s)


def _offdiag_values(spec: WaveletSpec, row, col, cd4, lev) -> np.ndarray:
    G = spec.grid_exp
    dj = np.abs(lev[row] - lev[col]).astype(np.float64)
    dist_grid = np.sqrt(cd4.astype(np.float64)) * 0.5   # grid units
    xi = pair_uniform(spec.seed, row, col)
    if spec.kind == "exp":
        dist = dist_grid * (2.0 ** -G)
        v = np.exp2(-spec.decay * dj) * np.exp(-dist / spec.ell)
    elif spec.kind == "alg":
        v = np.exp2(-(1.0 + spec.s) * dj) * np.power(1.0 + dist_grid, -(2.0 + 2.0 * spec.s))
    else:
        raise ValueError(f"unknown value kind {spec.kind!r}")
    return v * xi


def make_matrix(spec: WaveletSpec) -> Dict[str, np.ndarray]:
    """The instance as a lower-triangular CSC (diagonal first in each column, rows sorted).

    Returns a dict with n, colptr (int64[n+1]), rowind (int32[nnz]), values
    (float64[nnz]), coords (float64[n,2] support centres), level (int32[n]).
    """
    G = spec.grid_exp
    n = spec.n
    lev, _, _ = basis(G)
    R, C, D = [], [], []
    for j in range(G):
        for jp in range(j, G):
            r, c, d = _level_pair_entries(spec, j, jp)
            R.append(r); C.append(c); D.append(d)
    # the level-0 cell also carries the scaling function: pairs inside it
    # were produced by _cell_functions(0, ...) above (4 functions per cell).
    row = np.concatenate(R)
    col = np.concatenate(C)
    cd4 = np.concatenate(D)
    del R, C, D
    off = _offdiag_values(spec, row, col, cd4, lev)
    del cd4
    absoff = np.abs(off)
    rowsum = np.bincount(row, weights=absoff, minlength=n) + np.bincount(col, weights=absoff, minlength=n)
    del absoff
    diag = 1.1 * rowsum + np.exp2(2.0 * lev.astype(np.float64) * spec.s)
    # column-major order: key = col * n + row; the diagonal sorts first in its column
    key = col * n + row
    del row
    order = np.argsort(key, kind="stable")
    key = key[order]
    off = off[order]
    del order
    col_sorted = key // n
    row_sorted = (key - col_sorted * n)
    del key
    counts = np.bincount(col_sorted, minlength=n) + 1     # + diagonal
    colptr = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=colptr[1:])
    nnz = int(colptr[-1])
    rowind = np.empty(nnz, np.int32)
    values = np.empty(nnz, np.float64)
    diag_pos = colptr[:-1]
    is_diag = np.zeros(nnz, bool)
    is_diag[diag_pos] = True
    rowind[diag_pos] = np.arange(n, dtype=np.int32)
    values[diag_pos] = diag
    rowind[~is_diag] = row_sorted.astype(np.int32)
    values[~is_diag] = off
    coords, _ = centers(G)
    return {
        "n": n,
        "colptr": colptr,
        "rowind": rowind,
        "values": values,
        "coords": coords,
        "level": lev,
    }


def full_nnz(m: Dict[str, np.ndarray]) -> int:
    """nnz of the full symmetric matrix: both triangles, diagonal once."""
    return 2 * int(m["colptr"][-1]) - m["n"]


def normal_rhs(n: int, k: int, seed: int) -> np.ndarray:
    """k right-hand sides ~ N(0,1), returned column-major (n x k, Fortran order).

    Drawn as NumPy PCG64(seed).standard_normal((n, k)) in C order, i.e. row i
    holds the k values of unknown i."""
    g = np.random.Generator(np.random.PCG64(seed))
    return np.asfortranarray(g.standard_normal((n, k)))


def make_nonsymmetric(spec: WaveletSpec, eta: float = 0.5, seed2: int = 1) -> Dict[str, np.ndarray]:
    """A nonsymmetric matrix on the symmetric pattern of make_matrix(spec):
    stand-in for the PCM system matrix ((1+eps)/2) G + (1-eps) K of Section
    5.1, whose double-layer part K is not symmetric.  Every off-diagonal value
    v of the symmetric instance becomes v (1 + eta xi) below the diagonal and
    v (1 + eta xi') above it, with xi, xi' independent counter-based draws
    (seeds spec.seed ^ seed2 and its successor); the diagonal is then
    1.1 max(row abs sum, column abs sum) + 2^(2 j s), so A is strictly
    diagonally dominant by rows and by columns (nonsingular; elimination
    without pivoting is stable and partial pivoting would exchange no rows).

    Returns the dict of make_matrix with "values" = the entries on and below
    the diagonal and "upper" = the entry above the diagonal for each stored
    lower entry (A[c][r] for the stored (r, c); the diagonal repeated)."""
    m = make_matrix(spec)
    n = m["n"]
    cols = np.repeat(np.arange(n, dtype=np.int64), np.diff(m["colptr"]))
    rows = m["rowind"].astype(np.int64)
    off = rows != cols
    v = m["values"]
    lo = v.copy()
    up = v.copy()
    lo[off] = v[off] * (1.0 + eta * pair_uniform(spec.seed ^ seed2, rows[off], cols[off]))
    up[off] = v[off] * (1.0 + eta * pair_uniform((spec.seed ^ seed2) + 1, rows[off], cols[off]))
    # row i of A holds lo on (i, c < i) and up on (i, c > i); column j the opposite
    rsum = np.bincount(rows[off], np.abs(lo[off]), n) + np.bincount(cols[off], np.abs(up[off]), n)
    csum = np.bincount(cols[off], np.abs(lo[off]), n) + np.bincount(rows[off], np.abs(up[off]), n)
    diag = 1.1 * np.maximum(rsum, csum) + np.exp2(2.0 * m["level"].astype(np.float64) * spec.s)
    dpos = m["colptr"][:-1]
    lo[dpos] = diag
    up[dpos] = diag
    m["values"] = lo
    m["upper"] = up
    return m


def mass_spec(grid_exp: int, seed: int) -> WaveletSpec:
    """Stand-in for the mass matrix G_J = [(psi_l', psi_l)] of a non-orthogonal
    wavelet basis (Section 5.3): only functions whose supports overlap or touch
    couple (cut-off a = 0, a sub-pattern of every compressed system matrix on
    the same basis), with values decaying across levels and a unit-order
    diagonal (s = 0: 1.1 row abs sum + 1)."""
    return WaveletSpec(grid_exp, 0.0, 0.0, "exp", 0.3, 1.5, seed)
