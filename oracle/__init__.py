"""CPU oracle for the differentiable sparse Krylov solve.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package.  The product
library never does, and the two share no code: the arithmetic lives in
``oracle.c`` (plain sequential FP64 C) and in ``mpnn.py`` (plain numpy FP64),
and this module only marshals numpy arrays into it.

What each function follows (arXiv 2601.13994):

* ``spmv``                -- y = A x (local product of Eq. forward_spmv).
* ``cg``                  -- Algorithm "Distributed CG" with one process,
                            optionally Jacobi-preconditioned (the paper's
                            PyTorch-native backend, Table tab:benchmark).
* ``bicgstab``            -- van der Vorst's BiCGStab (cited in the
                            introduction for nonsymmetric systems; the paper
                            gives no steps), right Jacobi preconditioning.
* ``adjoint``             -- Eq. adjoint_master specialised to Eq.
                            adjoint_linear: solve A^T lambda = dL/dx, then
                            dL/db = lambda, dL/dA_ij = -lambda_i x_j on the
                            pattern (Sec. "Adjoint Differentiation").
* ``dense_solve``         -- dense Cholesky / LU (tiny n), used for the
                            brute-force adjoint.
* ``fsai`` / ``fsai_pcg`` -- classical FSAI on A's lower pattern (textbook,
                            Kolotilina & Yeremin); the paper lists learned
                            preconditioners only as future work.
* ``probe_loss``          -- ||G A G^T z - z||^2 summed over probes, with its
                            gradient on G's pattern.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")

OK, NOT_CONVERGED, BREAKDOWN, NONFINITE, BAD_INPUT = 0, 1, 2, 3, 4
PRECOND = {"none": 0, "jacobi": 1}

_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def build() -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, no FP contraction,
    OpenMP for the optional threaded mode)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-o", LIB_PATH, SRC_PATH, "-lm"]
    subprocess.run(cmd, check=True)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        i32, i64, f64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        i64p = ctypes.POINTER(ctypes.c_int64)
        f64p_ = ctypes.POINTER(ctypes.c_double)
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = None
        L.orc_spmv.argtypes = [i32, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.orc_dot.argtypes = [i64, _f64p, _f64p]
        L.orc_dot.restype = f64
        L.orc_residual_norm.argtypes = [i32, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.orc_residual_norm.restype = f64
        L.orc_jacobi_inverse.argtypes = [i32, _i32p, _i32p, _f64p, _f64p]
        L.orc_cg.argtypes = [i32, _i32p, _i32p, _f64p, _f64p, _f64p, ctypes.c_int, ctypes.c_int,
                             f64, f64, i64, i64p, f64p_, vp, vp]
        L.orc_bicgstab.argtypes = [i32, _i32p, _i32p, _f64p, _f64p, _f64p, ctypes.c_int, ctypes.c_int,
                                   f64, f64, i64, i64p, f64p_]
        L.orc_transpose.argtypes = [i32, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, _i32p]
        L.orc_adjoint_grad.argtypes = [i32, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.orc_dense_cholesky_solve.argtypes = [i32, _f64p, _f64p, _f64p]
        L.orc_dense_lu_solve.argtypes = [i32, _f64p, _f64p, _f64p, ctypes.c_int]
        L.orc_lower_pattern.argtypes = [i32, _i32p, _i32p, _i32p, _i32p, _i32p]
        L.orc_lower_pattern.restype = i32
        L.orc_fsai.argtypes = [i32, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p]
        L.orc_fsai_apply.argtypes = [i32, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.orc_fsai_pcg.argtypes = [i32, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, _f64p, _f64p,
                                   f64, f64, i64, i64p, f64p_]
        L.orc_probe_loss.argtypes = [i32, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, i32, _f64p, vp]
        L.orc_probe_loss.restype = f64
        _lib = L
    return _lib


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _csr(a):
    return int(a.n), _c(a.row_ptr, np.int32), _c(a.col, np.int32), _c(a.val, np.float64)


def default_max_iter(n: int) -> int:
    """min(10 n, 100000): the iteration cap used when none is given."""
    return int(min(10 * n, 100000))


# ---------------------------------------------------------------------------

_threads = 1


def set_threads(threads: int) -> None:
    """Threads of the oracle's parallel mode (1 = the plain sequential code).
    With more, SpMV rows and element-wise loops are split over the threads
    and inner products are summed as per-thread partials in thread order
    (deterministic for a given count)."""
    global _threads
    _threads = max(1, int(threads))
    lib().orc_set_threads(_threads)


class threads:
    """Context manager: run the oracle with `n` threads inside the block."""

    def __init__(self, n: int):
        self.n = n

    def __enter__(self):
        self.prev = _threads
        set_threads(self.n)
        return self

    def __exit__(self, *exc):
        set_threads(self.prev)
        return False


def spmv(a, x):
    n, rp, col, val = _csr(a)
    y = np.empty(n)
    lib().orc_spmv(n, rp, col, val, _c(x, np.float64), y)
    return y


def dot(u, v):
    u = _c(u, np.float64)
    return lib().orc_dot(len(u), u, _c(v, np.float64))


def residual_norm(a, b, x):
    n, rp, col, val = _csr(a)
    return lib().orc_residual_norm(n, rp, col, val, _c(b, np.float64), _c(x, np.float64))


class SolveResult:
    def __init__(self, x, status, iters, relres, alphas=None, betas=None):
        self.x, self.status, self.iters, self.relres = x, status, iters, relres
        self.alphas, self.betas = alphas, betas

    def __repr__(self):
        return f"SolveResult(status={self.status}, iters={self.iters}, relres={self.relres:.3e})"


def cg(a, b, precond="none", rtol=1e-10, atol=0.0, max_iter=None, x0=None, history=False):
    n, rp, col, val = _csr(a)
    max_iter = default_max_iter(n) if max_iter is None else int(max_iter)
    x = np.zeros(n) if x0 is None else _c(x0, np.float64).copy()
    it = ctypes.c_int64(0)
    rr = ctypes.c_double(0)
    al = np.zeros(max(max_iter, 1)) if history else None
    be = np.zeros(max(max_iter, 1)) if history else None
    st = lib().orc_cg(n, rp, col, val, _c(b, np.float64), x, PRECOND[precond], int(x0 is not None),
                      float(rtol), float(atol), max_iter, ctypes.byref(it), ctypes.byref(rr),
                      al.ctypes.data if history else None, be.ctypes.data if history else None)
    k = it.value
    if history:
        return SolveResult(x, st, k, rr.value, al[:k], be[:max(k - 1, 0)])
    return SolveResult(x, st, k, rr.value)


def bicgstab(a, b, precond="none", rtol=1e-10, atol=0.0, max_iter=None, x0=None):
    n, rp, col, val = _csr(a)
    max_iter = default_max_iter(n) if max_iter is None else int(max_iter)
    x = np.zeros(n) if x0 is None else _c(x0, np.float64).copy()
    it = ctypes.c_int64(0)
    rr = ctypes.c_double(0)
    st = lib().orc_bicgstab(n, rp, col, val, _c(b, np.float64), x, PRECOND[precond], int(x0 is not None),
                            float(rtol), float(atol), max_iter, ctypes.byref(it), ctypes.byref(rr))
    return SolveResult(x, st, it.value, rr.value)


def transpose(a):
    """(Csr of A^T, src) with src[k'] = position in A of A^T's entry k'."""
    from workloads import Csr

    n, rp, col, val = _csr(a)
    nnz = int(rp[-1])
    rpT = np.empty(n + 1, np.int32)
    colT = np.empty(nnz, np.int32)
    valT = np.empty(nnz)
    src = np.empty(nnz, np.int32)
    lib().orc_transpose(n, rp, col, val, rpT, colT, valT, src)
    return Csr(n, rpT, colT, valT), src


def is_symmetric(a) -> bool:
    """Pattern and values of A equal those of A^T, bit for bit."""
    t, _ = transpose(a)
    return (np.array_equal(t.row_ptr, a.row_ptr) and np.array_equal(t.col, a.col)
            and np.array_equal(t.val, np.asarray(a.val)))


def solve(a, b, method="auto", precond="none", rtol=1e-10, atol=0.0, max_iter=None):
    if method == "auto":
        method = "cg" if is_symmetric(a) else "bicgstab"
    f = cg if method == "cg" else bicgstab
    return f(a, b, precond=precond, rtol=rtol, atol=atol, max_iter=max_iter)


def adjoint_grad(a, lam, x):
    n, rp, col, _ = _csr(a)
    g = np.empty(len(col))
    lib().orc_adjoint_grad(n, rp, col, _c(lam, np.float64), _c(x, np.float64), g)
    return g


def adjoint(a, x, gx, method="auto", precond="none", rtol=1e-10, atol=0.0, max_iter=None):
    """Eq. adjoint_linear: lambda solves A^T lambda = gx; returns (gA, gb, result)."""
    sym = is_symmetric(a)
    if method == "auto":
        method = "cg" if sym else "bicgstab"
    at = a if sym else transpose(a)[0]
    f = cg if method == "cg" else bicgstab
    res = f(at, gx, precond=precond, rtol=rtol, atol=atol, max_iter=max_iter)
    lam = res.x
    return adjoint_grad(a, lam, x), lam.copy(), res


def dense_solve(A, b, spd=False, trans=False):
    A = _c(A, np.float64)
    n = A.shape[0]
    x = np.empty(n)
    if spd:
        rc = lib().orc_dense_cholesky_solve(n, A, _c(b, np.float64), x)
    else:
        rc = lib().orc_dense_lu_solve(n, A, _c(b, np.float64), x, int(trans))
    if rc != 0:
        raise np.linalg.LinAlgError("dense factorization failed")
    return x


def dense_adjoint(a, x, gx, spd=False):
    """Brute-force adjoint: lambda = A^{-T} gx by a dense factorization."""
    lam = dense_solve(a.to_dense(), gx, spd=spd, trans=not spd)
    return adjoint_grad(a, lam, x), lam


def lower_pattern(a):
    """(row_ptr_L, col_L, posA) of A's lower triangle including the diagonal."""
    n, rp, col, _ = _csr(a)
    rpL = np.empty(n + 1, np.int32)
    colL = np.empty(len(col), np.int32)
    pos = np.empty(len(col), np.int32)
    c = lib().orc_lower_pattern(n, rp, col, rpL, colL, pos)
    return rpL, colL[:c].copy(), pos[:c].copy()


def fsai(a):
    """Classical FSAI values on A's lower pattern: returns (rpL, colL, gL)."""
    n, rp, col, val = _csr(a)
    rpL, colL, _ = lower_pattern(a)
    g = np.empty(len(colL))
    if lib().orc_fsai(n, rp, col, val, rpL, colL, g) != 0:
        raise np.linalg.LinAlgError("FSAI local block not SPD")
    return rpL, colL, g


def fsai_apply(rpL, colL, gL, r):
    n = len(rpL) - 1
    z = np.empty(n)
    lib().orc_fsai_apply(n, _c(rpL, np.int32), _c(colL, np.int32), _c(gL, np.float64), _c(r, np.float64), z)
    return z


def fsai_pcg(a, rpL, colL, gL, b, rtol=1e-8, atol=0.0, max_iter=None):
    n, rp, col, val = _csr(a)
    max_iter = default_max_iter(n) if max_iter is None else int(max_iter)
    x = np.zeros(n)
    it = ctypes.c_int64(0)
    rr = ctypes.c_double(0)
    st = lib().orc_fsai_pcg(n, rp, col, val, _c(rpL, np.int32), _c(colL, np.int32), _c(gL, np.float64),
                            _c(b, np.float64), x, float(rtol), float(atol), max_iter,
                            ctypes.byref(it), ctypes.byref(rr))
    return SolveResult(x, st, it.value, rr.value)


def probe_loss(a, rpL, colL, gL, Z, grad=True):
    """sum_p ||G A G^T z_p - z_p||^2 and (optionally) its gradient on G's pattern."""
    n, rp, col, val = _csr(a)
    Z = _c(np.atleast_2d(Z), np.float64)
    g = np.empty(len(colL)) if grad else None
    loss = lib().orc_probe_loss(n, rp, col, val, _c(rpL, np.int32), _c(colL, np.int32),
                                _c(gL, np.float64), Z.shape[0], Z, g.ctypes.data if grad else None)
    return (loss, g) if grad else loss
