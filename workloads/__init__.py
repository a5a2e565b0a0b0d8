"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module only *builds inputs*: sparse matrices in canonical CSR form
(int32 ``row_ptr``/``col``, float64 ``val``), right-hand sides, targets and
probe vectors.  It holds none of the solver arithmetic (no SpMV, no Krylov
recurrence, no gradient), so it can serve both sides of a parity test
without coupling them.

Every random draw comes from ``numpy.random.default_rng(SeedSequence(
260113994, spawn_key=(cfg, stream, sample)))`` with

    stream 0 = coefficients / points, 1 = right-hand side b,
    2 = targets x* / probes, 3 = finite-difference picks, 4 = held-out split.

Workloads (all synthetic; the paper measures only synthetic PDE matrices):

* ``poisson2d``  -- 2D 5-point Dirichlet Laplacian, the operator of the
  paper's scalability table and of its small adjoint-correctness problem
  (N = 64^2 = 4096 interior unknowns).
* ``diffusion3d`` -- 3D 7-point cell-centred variable-coefficient diffusion
  with log-normal kappa, harmonic-mean faces and homogeneous Dirichlet ghosts,
  optionally plus first-order upwind convection (nonsymmetric).
* ``knn_laplacian`` -- shifted graph Laplacian of a symmetric k-NN graph over
  uniform points in the unit cube (distinct patterns, ragged sizes).
* ``aniso2d`` -- 2D anisotropic diffusion, 9-point stencil with the mixed
  derivative term (SPD, not an M-matrix).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ROOT_SEED = 260113994


def rng(cfg: int, stream: int, sample: int = 0) -> np.random.Generator:
    """Generator for (workload, stream, sample) as documented above."""
    return np.random.default_rng(np.random.SeedSequence(ROOT_SEED, spawn_key=(cfg, stream, sample)))


@dataclasses.dataclass
class Csr:
    """Canonical CSR: 0-based, columns strictly increasing per row, int32 indices."""

    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col: np.ndarray  # int32[nnz]
    val: np.ndarray  # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def rows(self) -> np.ndarray:
        """Row index of every stored entry (int64[nnz])."""
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        d[self.rows(), self.col] = self.val
        return d

    def with_values(self, val: np.ndarray) -> "Csr":
        return Csr(self.n, self.row_ptr, self.col, np.ascontiguousarray(val, dtype=np.float64))


def _compress(n: int, cols: np.ndarray, vals: np.ndarray, mask: np.ndarray) -> Csr:
    """Rows are the leading axis of ``cols``/``vals``/``mask`` (shape (n, s)),
    stencil slots are already in ascending column order."""
    counts = mask.sum(axis=1, dtype=np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    assert row_ptr[-1] < 2**31
    col = np.ascontiguousarray(cols[mask], dtype=np.int32)
    val = np.ascontiguousarray(vals[mask], dtype=np.float64)
    return Csr(n, row_ptr.astype(np.int32), col, val)


# ----------------------------------------------------------------------------
# Structured grids
# ----------------------------------------------------------------------------

def poisson1d(m: int) -> Csr:
    """1D Dirichlet Laplacian tridiag(-1, 2, -1) of order m."""
    i = np.arange(m)
    cols = np.stack([i - 1, i, i + 1], axis=1)
    vals = np.broadcast_to(np.array([-1.0, 2.0, -1.0]), (m, 3)).copy()
    mask = (cols >= 0) & (cols < m)
    return _compress(m, np.where(mask, cols, 0), vals, mask)


def poisson2d(m: int) -> Csr:
    """2D 5-point Dirichlet Laplacian on an m x m interior grid, unit spacing.

    Unknown (x, y) has index y*m + x; diagonal 4, neighbours -1."""
    n = m * m
    idx = np.arange(n, dtype=np.int64)
    x = idx % m
    y = idx // m
    # slots in ascending column order: S, W, C, E, N
    cols = np.stack([idx - m, idx - 1, idx, idx + 1, idx + m], axis=1)
    mask = np.stack([y > 0, x > 0, np.ones(n, bool), x < m - 1, y < m - 1], axis=1)
    vals = np.broadcast_to(np.array([-1.0, -1.0, 4.0, -1.0, -1.0]), (n, 5)).copy()
    return _compress(n, np.where(mask, cols, 0), vals, mask)


def poisson2d_rect(mx: int, my: int) -> Csr:
    """2D 5-point Dirichlet Laplacian on an mx x my interior grid (unknown
    (x, y) at y*mx + x; diagonal 4, neighbours -1): with mx != my its small
    eigenvalues are simple."""
    n = mx * my
    idx = np.arange(n, dtype=np.int64)
    x = idx % mx
    y = idx // mx
    cols = np.stack([idx - mx, idx - 1, idx, idx + 1, idx + mx], axis=1)
    mask = np.stack([y > 0, x > 0, np.ones(n, bool), x < mx - 1, y < my - 1], axis=1)
    vals = np.broadcast_to(np.array([-1.0, -1.0, 4.0, -1.0, -1.0]), (n, 5)).copy()
    return _compress(n, np.where(mask, cols, 0), vals, mask)


_D3_CACHE: dict = {}


def _d3_pattern(m: int):
    """Cached 7-point pattern pieces of an m^3 grid: (Csr with zero values,
    boolean mask (m, m, m, 7) of the stored slots)."""
    if m not in _D3_CACHE:
        n = m ** 3
        idx = np.arange(n, dtype=np.int64).reshape(m, m, m)
        z, y, x = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
        cols = np.stack([idx - m * m, idx - m, idx - 1, idx, idx + 1, idx + m, idx + m * m], axis=-1)
        mask = np.stack([z > 0, y > 0, x > 0, np.ones_like(x, bool), x < m - 1, y < m - 1, z < m - 1], axis=-1)
        a = _compress(n, np.where(mask, cols, 0).reshape(n, 7), np.zeros((n, 7)), mask.reshape(n, 7))
        _D3_CACHE.clear()
        _D3_CACHE[m] = (a, mask)
    return _D3_CACHE[m]


def diffusion3d_values(m: int, kappa: np.ndarray | None = None, velocity: float = 0.0,
                       diffusion: bool = True) -> np.ndarray:
    """Values (CSR order of the cached 7-point pattern) of diffusion3d."""
    _, mask = _d3_pattern(m)
    if kappa is None:
        kappa = np.ones(m ** 3)
    k = np.asarray(kappa, dtype=np.float64).reshape(m, m, m)  # [z, y, x]

    def face(axis: int, side: int) -> np.ndarray:
        """Face coefficient on the side (-1/+1) of each cell along axis."""
        nb = np.roll(k, -side, axis=axis)
        hm = 2.0 * k * nb / (k + nb)
        edge = [slice(None)] * 3
        edge[axis] = 0 if side < 0 else m - 1
        hm[tuple(edge)] = k[tuple(edge)]
        return hm

    if diffusion:
        # axis 0 = z, 1 = y, 2 = x
        a_zm, a_ym, a_xm = face(0, -1), face(1, -1), face(2, -1)
        a_xp, a_yp, a_zp = face(2, +1), face(1, +1), face(0, +1)
        diag = a_zm + a_ym + a_xm + a_xp + a_yp + a_zp
        vals = np.stack([-a_zm, -a_ym, -a_xm, diag, -a_xp, -a_yp, -a_zp], axis=-1)
        del a_zm, a_ym, a_xm, a_xp, a_yp, a_zp
    else:
        vals = np.zeros((m, m, m, 7))
    if velocity:
        vd = velocity / math.sqrt(3.0)
        vals[..., 3] += vd + vd + vd
        vals[..., 0] -= vd
        vals[..., 1] -= vd
        vals[..., 2] -= vd
    return np.ascontiguousarray(vals[mask], dtype=np.float64)


def diffusion3d(m: int, kappa: np.ndarray | None = None, velocity: float = 0.0,
                diffusion: bool = True) -> Csr:
    """3D 7-point cell-centred operator on an m^3 grid, unit spacing, no 1/h^2.

    * cell (x, y, z) has index (z*m + y)*m + x; columns ascending per row;
    * interior face P|Q: a = 2 kP kQ / (kP + kQ) (harmonic mean);
    * boundary face: homogeneous Dirichlet ghost, a = kP, so kappa == 1 gives
      diagonal 6 and off-diagonals -1;
    * A_PP = sum of the six face coefficients (order z-, y-, x-, x+, y+, z+),
      A_PQ = -a_PQ;
    * ``velocity`` > 0 adds first-order upwind convection with velocity
      v*(1,1,1)/sqrt(3), |v| = velocity: row P gets +(vx+vy+vz) on the
      diagonal and -v_d at the upstream neighbour P - e_d (dropped at the
      inflow boundary, ghost value 0);
    * ``diffusion=False`` keeps the 7-point pattern but stores only the
      convection part (upper entries become explicit zeros).
    """
    a, _ = _d3_pattern(m)
    return Csr(a.n, a.row_ptr, a.col, diffusion3d_values(m, kappa, velocity, diffusion))


def aniso_tensor(ratio: float, angle: float) -> tuple[float, float, float]:
    """K = R(angle) diag(1, 1/ratio) R(angle)^T -> (k11, k22, k12)."""
    c, s = math.cos(angle), math.sin(angle)
    inv = 1.0 / ratio
    return c * c + s * s * inv, s * s + c * c * inv, (1.0 - inv) * s * c


ANISO_OFFSETS = [(-1, -1), (0, -1), (1, -1), (-1, 0), (0, 0), (1, 0), (-1, 1), (0, 1), (1, 1)]  # (dx, dy)


def aniso_stencil(ratio: float, angle: float) -> np.ndarray:
    """The 9 stencil coefficients in slot order (ascending column offset):
    centre 2(k11+k22), E/W -k11, N/S -k22, NE/SW -k12/2, NW/SE +k12/2."""
    k11, k22, k12 = aniso_tensor(ratio, angle)
    coef = {(-1, -1): -k12 / 2, (0, -1): -k22, (1, -1): k12 / 2, (-1, 0): -k11, (0, 0): 2 * (k11 + k22),
            (1, 0): -k11, (-1, 1): k12 / 2, (0, 1): -k22, (1, 1): -k12 / 2}
    return np.array([coef[o] for o in ANISO_OFFSETS])


def aniso_pattern(m: int) -> tuple[Csr, np.ndarray]:
    """Full 9-point Dirichlet pattern on an m x m grid (values zero) and the
    stencil slot (0..8) of every stored entry."""
    n = m * m
    idx = np.arange(n, dtype=np.int64)
    x = idx % m
    y = idx // m
    cols = np.stack([idx + dy * m + dx for dx, dy in ANISO_OFFSETS], axis=1)
    mask = np.stack([(x + dx >= 0) & (x + dx < m) & (y + dy >= 0) & (y + dy < m) for dx, dy in ANISO_OFFSETS],
                    axis=1)
    slots = np.broadcast_to(np.arange(9), (n, 9))
    a = _compress(n, np.where(mask, cols, 0), np.zeros((n, 9)), mask)
    return a, np.ascontiguousarray(slots[mask], dtype=np.int64)


def aniso2d(m: int, ratio: float, angle: float) -> Csr:
    """2D anisotropic diffusion -div(K grad u), 9-point stencil, unit spacing,
    homogeneous Dirichlet; the full 9-point pattern is always stored (explicit
    zeros kept).  Unknown (x, y) has index y*m + x.  The values are
    aniso_stencil(ratio, angle)[slot] of each entry."""
    a, slots = aniso_pattern(m)
    a.val = aniso_stencil(ratio, angle)[slots]
    return a


# ----------------------------------------------------------------------------
# k-NN graph Laplacians (distinct ragged patterns)
# ----------------------------------------------------------------------------

def morton_order(pts: np.ndarray, bits: int = 10) -> np.ndarray:
    q = np.minimum((pts * (1 << bits)).astype(np.int64), (1 << bits) - 1)
    code = np.zeros(len(pts), dtype=np.int64)
    for b in range(bits):
        for d in range(3):
            code |= ((q[:, d] >> b) & 1) << (3 * b + d)
    return np.argsort(code, kind="stable")


def knn_laplacian(pts: np.ndarray, k: int = 8, shift: float = 0.01) -> Csr:
    """A = L + shift*I for the union-symmetrised k-NN graph of ``pts``.

    k neighbours exclude the point itself; sigma is the mean of all n*k
    directed k-NN distances; w_ij = exp(-d_ij^2 / sigma^2) with d^2 summed
    over x, y, z in that order (so w is bit-symmetric); A_ii = sum_j w_ij
    (ascending j) + shift, A_ij = -w_ij."""
    from scipy.spatial import cKDTree

    n = len(pts)
    dist, nb = cKDTree(pts).query(pts, k=k + 1)
    # drop the point itself (first hit; exact duplicates are measure-zero)
    selfpos = np.argmax(nb == np.arange(n)[:, None], axis=1)
    keep = np.ones_like(nb, bool)
    keep[np.arange(n), selfpos] = False
    nb = nb[keep].reshape(n, k)
    sigma = float(dist[keep].reshape(n, k).mean())
    i = np.repeat(np.arange(n), k)
    j = nb.ravel()
    pairs = np.unique(np.concatenate([i * n + j, j * n + i]))
    ri, cj = pairs // n, pairs % n
    d2 = (pts[ri, 0] - pts[cj, 0]) ** 2
    d2 = d2 + (pts[ri, 1] - pts[cj, 1]) ** 2
    d2 = d2 + (pts[ri, 2] - pts[cj, 2]) ** 2
    w = np.exp(-d2 / (sigma * sigma))
    # insert the diagonal; entries sorted by (row, col)
    allr = np.concatenate([ri, np.arange(n)])
    allc = np.concatenate([cj, np.arange(n)])
    order = np.lexsort((allc, allr))
    allr, allc = allr[order], allc[order]
    offv = np.concatenate([-w, np.zeros(n)])[order]
    isdiag = allr == allc
    # row sums of w in ascending column order, one column slot at a time
    counts = np.bincount(allr, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    wsorted = np.concatenate([w, np.zeros(n)])[order]
    slot = np.arange(len(allr)) - row_ptr[allr]
    pad = np.zeros((n, int(counts.max())))
    pad[allr, slot] = wsorted
    dsum = np.zeros(n)
    for c in range(pad.shape[1]):
        dsum = dsum + pad[:, c]
    diag = dsum + shift
    vals = np.where(isdiag, diag[allr], offv)
    return Csr(n, row_ptr.astype(np.int32), allc.astype(np.int32), vals.astype(np.float64))


# ----------------------------------------------------------------------------
# Small test matrices
# ----------------------------------------------------------------------------

def random_pattern(n: int, density: float, r: np.random.Generator, diag: bool = True,
                   symmetric: bool = False) -> tuple[np.ndarray, np.ndarray]:
    """Random sparsity pattern as CSR index arrays (row_ptr, col)."""
    m = r.random((n, n)) < density
    if symmetric:
        m = m | m.T
    if diag:
        np.fill_diagonal(m, True)
    counts = m.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(counts, out=row_ptr[1:])
    col = np.nonzero(m)[1].astype(np.int32)
    return row_ptr, col


def random_spd(n: int, density: float, r: np.random.Generator, shift: float = 0.1) -> Csr:
    """SPD matrix with a random symmetric pattern: symmetric off-diagonal
    values from N(0,1) and a diagonal that makes it strictly diagonally
    dominant by ``shift`` (Gershgorin), values bit-symmetric."""
    row_ptr, col = random_pattern(n, density, r, symmetric=True)
    a = Csr(n, row_ptr, col, np.zeros(len(col)))
    rows = a.rows()
    d = np.zeros((n, n))
    upper = rows < col
    d[rows[upper], col[upper]] = r.standard_normal(int(upper.sum()))
    d = d + d.T
    np.fill_diagonal(d, np.abs(d).sum(axis=1) + shift)
    a.val = d[rows, col].copy()
    return a


def random_nonsym(n: int, density: float, r: np.random.Generator, dominance: float = 1.5) -> Csr:
    """Nonsymmetric, diagonally dominant matrix on a random (nonsymmetric) pattern."""
    row_ptr, col = random_pattern(n, density, r)
    a = Csr(n, row_ptr, col, r.standard_normal(len(col)))
    rows = a.rows()
    isd = rows == col
    offsum = np.zeros(n)
    np.add.at(offsum, rows[~isd], np.abs(a.val[~isd]))
    a.val[isd] = dominance * offsum + 1.0
    return a


def from_dense(d: np.ndarray, keep: np.ndarray | None = None) -> Csr:
    """CSR of a dense matrix; ``keep`` (bool) selects stored entries (explicit
    zeros allowed), default: the nonzeros plus the diagonal."""
    n = d.shape[0]
    if keep is None:
        keep = (d != 0) | np.eye(n, dtype=bool)
    counts = keep.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(counts, out=row_ptr[1:])
    r_, c_ = np.nonzero(keep)
    return Csr(n, row_ptr, c_.astype(np.int32), d[r_, c_].astype(np.float64))


# ----------------------------------------------------------------------------
# The five benchmark workloads, by their shapes and recipes
# ----------------------------------------------------------------------------

def poisson2d_workload(m: int = 64):
    """2D 5-point Poisson, m x m interior grid, b ~ N(0,1) (workload 1)."""
    a = poisson2d(m)
    b = rng(1, 1).standard_normal(a.n)
    return a, b


def diffusion3d_kappa(m: int, cfg: int = 2, sample: int = 0) -> np.ndarray:
    """kappa = exp(g), g ~ N(0,1) i.i.d. per cell."""
    return np.exp(rng(cfg, 0, sample).standard_normal(m ** 3))


def diffusion3d_workload(m: int = 256, convection: bool = False):
    """3D 7-point log-normal diffusion on m^3 cells, b ~ N(0,1) (workload 2);
    ``convection`` adds upwind transport at cell Peclet 10 along (1,1,1)/sqrt(3)."""
    a = diffusion3d(m, diffusion3d_kappa(m), velocity=10.0 if convection else 0.0)
    b = rng(2, 1).standard_normal(a.n)
    return a, b


def knn_system(sample: int, n_lo: int = 1000, n_hi: int = 50000, morton: bool = True):
    """One ragged k-NN Laplacian system (workload 3): n ~ U{n_lo..n_hi}."""
    r = rng(3, 0, sample)
    n = int(r.integers(n_lo, n_hi + 1))
    pts = r.random((n, 3))
    if morton:
        pts = pts[morton_order(pts)]
    a = knn_laplacian(pts)
    b = rng(3, 1, sample).standard_normal(n)
    return a, b


def shared_pattern_batch(m: int = 96, batch: int = 128, workers: int = 1):
    """Workload 4: ``batch`` samples of 3D log-normal diffusion on one m^3
    pattern.  Returns (pattern Csr of sample 0, values[B, nnz], b[B, n],
    xstar[B, n]).  ``workers`` > 1 builds the samples in forked processes
    (call it before the process touches a GPU)."""
    a0, _ = _d3_pattern(m)
    n = a0.n
    vals = np.empty((batch, a0.nnz))
    bs = np.empty((batch, n))
    xs = np.empty((batch, n))
    if workers > 1 and batch > 1:
        import concurrent.futures as cf
        import functools
        import multiprocessing as mp

        with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
            for s, v in enumerate(ex.map(functools.partial(_d4_values, m), range(batch))):
                vals[s] = v
    else:
        for s in range(batch):
            vals[s] = _d4_values(m, s)
    for s in range(batch):
        bs[s] = rng(4, 1, s).standard_normal(n)
        xs[s] = rng(4, 2, s).standard_normal(n)
    return Csr(n, a0.row_ptr, a0.col, vals[0]), vals, bs, xs


def _d4_values(m: int, s: int) -> np.ndarray:
    return diffusion3d_values(m, diffusion3d_kappa(m, cfg=4, sample=s))


def aniso_params(sample: int, heldout: bool = False) -> tuple[float, float]:
    """Anisotropy ratio ~ logU[1, 1000] and angle ~ U[0, pi) (workload 5)."""
    r = rng(5, 4 if heldout else 0, sample)
    ratio = 10.0 ** r.uniform(0.0, 3.0)
    angle = r.uniform(0.0, math.pi)
    return ratio, angle


def aniso_system(sample: int, m: int = 256, heldout: bool = False):
    ratio, angle = aniso_params(sample, heldout)
    a = aniso2d(m, ratio, angle)
    b = rng(5, 5 if heldout else 1, sample).standard_normal(a.n)
    return a, b


def knn_systems(count: int, workers: int = 8, **kw):
    """The first ``count`` ragged k-NN systems (workload 3), built in forked
    processes (call it before the process touches a GPU)."""
    if workers <= 1 or count <= 1:
        return [knn_system(s, **kw) for s in range(count)]
    import concurrent.futures as cf
    import functools
    import multiprocessing as mp

    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        return list(ex.map(functools.partial(_knn_one, kw=kw), range(count), chunksize=4))


def _knn_one(s, kw):
    return knn_system(s, **kw)


def rademacher(r: np.random.Generator, shape) -> np.ndarray:
    return np.where(r.random(shape) < 0.5, -1.0, 1.0)


def inverse_truth(m: int = 64):
    """Inputs of the inverse coefficient problem (Sec. "End-to-End: Inverse
    Coefficient Learning"): the ground-truth conductivity
    kappa*(x, y) = 1 + 0.5 sin(2 pi x) sin(2 pi y) at the centres of an m x m
    grid of cells on (0, 1)^2 (cell (ix, iy) at index iy * m + ix) and the
    source f = 1 per cell."""
    c = (np.arange(m) + 0.5) / m
    x, y = np.meshgrid(c, c)  # x varies along a row of the grid
    kappa = 1.0 + 0.5 * np.sin(2.0 * np.pi * x) * np.sin(2.0 * np.pi * y)
    return kappa.reshape(-1), np.ones(m * m)
