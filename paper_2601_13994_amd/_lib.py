"""ctypes binding of libhsla.so (the C ABI declared in include/hsla.h).

Argument marshalling only: torch tensors are checked for device, dtype and
contiguity and passed as raw device pointers together with the current
stream.  There is no fallback path: if the library is missing or no GPU is
present, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhsla.so")

OK, NOT_CONVERGED, BREAKDOWN, FELL_BACK, STAGNATED = 0, 1, 2, 3, 4
ERR_INVALID_ARG, ERR_INVALID_CSR, ERR_NONFINITE, ERR_HIP = -1, -2, -3, -4
ERR_NO_MEMORY, ERR_ZERO_DIAGONAL, ERR_INTERNAL = -5, -6, -7

METHODS = {"auto": 0, "cg": 1, "bicgstab": 2, "cg_sr": 3, "cg_sstep": 4}
METHOD_NAMES = {v: k for k, v in METHODS.items()}
PRECONDS = {"none": 0, "jacobi": 1, "fsai": 2}
FORMATS = {"auto": 0, "csr": 1, "diagonal": 2}
PATTERN_CSR = 1  # hsla_pattern_create flag

# every symbol include/hsla.h declares
EXPORTS = [
    "hsla_opts_default", "hsla_status_string", "hsla_create", "hsla_destroy", "hsla_last_error",
    "hsla_set_allocator", "hsla_workspace_size", "hsla_reserve",
    "hsla_pattern_create", "hsla_pattern_destroy", "hsla_pattern_info", "hsla_pattern_set_format",
    "hsla_pattern_format", "hsla_autotune", "hsla_pattern_transpose", "hsla_pattern_lower",
    "hsla_pattern_signature", "hsla_pattern_get_tuning", "hsla_pattern_set_tuning",
    "hsla_spmv", "hsla_solve", "hsla_solve_batched", "hsla_adjoint", "hsla_adjoint_batched",
    "hsla_outer_on_pattern", "hsla_residual_norms",
    "hsla_mpnn_num_params", "hsla_mpnn_forward", "hsla_mpnn_backward", "hsla_probe_loss", "hsla_adam_step",
    "hsla_fsai_factors", "hsla_solve_ragged", "hsla_solve_noalloc", "hsla_csr_check", "hsla_pattern_colors",
]


class HslaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"hsla status {status}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [
        ("method", ctypes.c_int32), ("precond", ctypes.c_int32),
        ("rtol", ctypes.c_double), ("atol", ctypes.c_double),
        ("max_iter", ctypes.c_int64), ("check_every", ctypes.c_int32),
        ("use_x0", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("profile", ctypes.c_int32),
        ("d_G", ctypes.c_void_p), ("d_GT", ctypes.c_void_p), ("persistent", ctypes.c_int32),
        ("stall_window", ctypes.c_int32), ("s_step", ctypes.c_int32),
    ]


SPMV_FORMS = {0: "tiles", 1: "diagonal", 2: "diagonal-half", 3: "persistent", 4: "diagonal-half-unit",
              5: "diagonal-unit"}


class TuneState(ctypes.Structure):
    _fields_ = [("signature", ctypes.c_uint64), ("tuned", ctypes.c_int32), ("dia", ctypes.c_int32),
                ("dia_cu", ctypes.c_int32), ("tile_cu", ctypes.c_int32), ("sym", ctypes.c_int32),
                ("sym_cu", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class Info(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int64), ("status", ctypes.c_int32), ("method", ctypes.c_int32),
        ("rel_residual", ctypes.c_double), ("true_residual", ctypes.c_double),
        ("spmv_ms", ctypes.c_double), ("spmv_launches", ctypes.c_int64),
        ("spmv_form", ctypes.c_int32), ("spmv_paired", ctypes.c_int32),
        ("t_start_ms", ctypes.c_double), ("t_end_ms", ctypes.c_double),
        ("workgroups", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return {"iters": self.iters, "status": self.status, "method": METHOD_NAMES.get(self.method, "?"),
                "rel_residual": self.rel_residual, "true_residual": self.true_residual,
                "spmv_ms": self.spmv_ms, "spmv_launches": self.spmv_launches,
                "spmv_form": SPMV_FORMS.get(self.spmv_form, "?"), "spmv_paired": bool(self.spmv_paired),
                "t_start_ms": self.t_start_ms, "t_end_ms": self.t_end_ms, "workgroups": self.workgroups}


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_allocators = {}  # device index -> (alloc, free) callbacks kept alive


class Tuning(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("best_us", ctypes.c_double), ("default_us", ctypes.c_double)]


_lib = None
_lock = threading.Lock()
_handles: dict[int, ctypes.c_void_p] = {}


def load() -> ctypes.CDLL:
    """Loads libhsla.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2601_13994_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        P = ctypes.POINTER
        L.hsla_opts_default.argtypes = [P(Opts)]
        L.hsla_opts_default.restype = None
        L.hsla_status_string.argtypes = [ctypes.c_int]
        L.hsla_status_string.restype = ctypes.c_char_p
        L.hsla_create.argtypes = [P(vp), ctypes.c_int]
        L.hsla_destroy.argtypes = [vp]
        L.hsla_destroy.restype = None
        L.hsla_last_error.argtypes = [vp]
        L.hsla_last_error.restype = ctypes.c_char_p
        L.hsla_set_allocator.argtypes = [vp, ALLOC_FN, FREE_FN, vp]
        L.hsla_workspace_size.argtypes = [vp, vp, i32, P(Opts), P(ctypes.c_size_t)]
        L.hsla_reserve.argtypes = [vp, ctypes.c_size_t]
        L.hsla_pattern_create.argtypes = [vp, i32, i64, vp, vp, ctypes.c_uint32, vp, P(vp)]
        L.hsla_pattern_destroy.argtypes = [vp]
        L.hsla_pattern_destroy.restype = None
        L.hsla_pattern_info.argtypes = [vp, P(i32), P(i64), P(i64), P(i32)]
        L.hsla_pattern_set_format.argtypes = [vp, i32]
        L.hsla_pattern_format.argtypes = [vp, P(i32), P(i32)]
        L.hsla_autotune.argtypes = [vp, vp, i32, i32, P(Tuning), vp]
        L.hsla_pattern_transpose.argtypes = [vp, vp, vp, vp, vp, vp]
        L.hsla_pattern_lower.argtypes = [vp, vp, vp, vp, vp, vp]
        L.hsla_pattern_signature.argtypes = [vp, P(ctypes.c_uint64)]
        L.hsla_pattern_get_tuning.argtypes = [vp, P(TuneState)]
        L.hsla_pattern_set_tuning.argtypes = [vp, P(TuneState)]
        L.hsla_spmv.argtypes = [vp, vp, i32, vp, vp, vp, vp]
        L.hsla_solve.argtypes = [vp, vp, vp, vp, vp, P(Opts), P(Info), vp]
        L.hsla_solve_batched.argtypes = [vp, vp, i32, vp, vp, vp, P(Opts), P(Info), vp]
        L.hsla_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp, P(Opts), P(Info), vp]
        L.hsla_adjoint_batched.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, P(Opts), P(Info), vp]
        L.hsla_outer_on_pattern.argtypes = [vp, vp, i32, vp, vp, vp, vp]
        L.hsla_residual_norms.argtypes = [vp, vp, i32, vp, vp, vp, P(f64), P(f64), vp]
        L.hsla_mpnn_num_params.argtypes = []
        L.hsla_mpnn_num_params.restype = i32
        L.hsla_mpnn_forward.argtypes = [vp, vp, i32, vp, vp, vp, i32, vp]
        L.hsla_mpnn_backward.argtypes = [vp, vp, i32, vp, vp, vp]
        L.hsla_probe_loss.argtypes = [vp, vp, i32, vp, vp, i32, vp, f64, P(f64), vp, vp]
        L.hsla_adam_step.argtypes = [vp, i64, vp, vp, vp, vp, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, i64, vp]
        L.hsla_fsai_factors.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp]
        L.hsla_solve_ragged.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, P(Opts), P(Info), vp]
        L.hsla_solve_noalloc.argtypes = [vp, vp, i32, vp, vp, vp, P(Opts), P(Info), vp]
        L.hsla_csr_check.argtypes = [i32, i64, vp, vp, P(i32)]
        L.hsla_pattern_colors.argtypes = [vp, vp, vp, P(i32), vp]
        _lib = L
    return _lib


def status_string(st: int) -> str:
    return load().hsla_status_string(st).decode()


def handle(device: int | None = None) -> ctypes.c_void_p:
    if not torch.cuda.is_available():
        raise RuntimeError("hsla needs a ROCm GPU; none is visible")
    dev = torch.cuda.current_device() if device is None else int(device)
    h = _handles.get(dev)
    if h is None:
        L = load()
        h = ctypes.c_void_p()
        st = L.hsla_create(ctypes.byref(h), dev)
        if st != 0:
            raise HslaError(st, f"hsla_create(device={dev}) failed: {status_string(st)}")
        _handles[dev] = h
    return h


def check(st: int, h, what: str, warn_ok: bool = True) -> int:
    if st < 0 or (st > 0 and not warn_ok):
        msg = load().hsla_last_error(h).decode() if h else ""
        raise HslaError(st, f"{what}: {status_string(st)} {msg}")
    return st


def stream_ptr(device=None) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def use_torch_allocator(device=None, enable: bool = True, counter: dict | None = None) -> None:
    """Route the handle's workspaces on `device` through torch's caching
    allocator (enable=False restores hipMalloc).  `counter`, if given, counts
    the allocator calls (keys 'alloc', 'free')."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    if not enable:
        st = load().hsla_set_allocator(handle(idx), ALLOC_FN(), FREE_FN(), None)
        check(st, handle(idx), "hsla_set_allocator")
        _allocators.pop(idx, None)
        return

    def _alloc(nbytes, ctx):
        if counter is not None:
            counter["alloc"] = counter.get("alloc", 0) + 1
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device=idx)
        except RuntimeError:
            return None

    def _free(p, ctx):
        if counter is not None:
            counter["free"] = counter.get("free", 0) + 1
        torch.cuda.caching_allocator_delete(p)

    cbs = (ALLOC_FN(_alloc), FREE_FN(_free))
    st = load().hsla_set_allocator(handle(idx), cbs[0], cbs[1], None)
    check(st, handle(idx), "hsla_set_allocator")
    _allocators[idx] = cbs


def workspace_size(pat: "Pattern", B: int = 1, opts: "Opts | None" = None) -> int:
    n = ctypes.c_size_t()
    st = load().hsla_workspace_size(pat.h, pat.p, int(B), ctypes.byref(opts) if opts is not None else None,
                                    ctypes.byref(n))
    check(st, pat.h, "hsla_workspace_size")
    return n.value


def reserve(nbytes: int, device=None) -> None:
    idx = torch.device(device).index if device is not None else torch.cuda.current_device()
    with torch.cuda.device(idx):
        st = load().hsla_reserve(handle(idx), int(nbytes))
        check(st, handle(idx), "hsla_reserve")


def ptr(t: torch.Tensor | None) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def need(t: torch.Tensor, dtype: torch.dtype, name: str, device: torch.device) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    return t.contiguous()


def make_opts(method="auto", precond="jacobi", rtol=1e-8, atol=0.0, max_iter=0, check_every=0,
              x0=False, graph=True, profile=False, G=None, GT=None, persistent=True, stall_window=0,
              s_step=4) -> Opts:
    o = Opts()
    load().hsla_opts_default(ctypes.byref(o))
    o.method = METHODS[method]
    o.precond = PRECONDS[precond]
    o.rtol = float(rtol)
    o.atol = float(atol)
    o.max_iter = int(max_iter or 0)
    o.check_every = int(check_every or 0)
    o.use_x0 = int(bool(x0))
    o.use_graph = int(bool(graph))
    o.profile = int(bool(profile))
    o.d_G = G.data_ptr() if G is not None else None
    o.d_GT = GT.data_ptr() if GT is not None else None
    o.persistent = 2 if persistent == "force" else int(bool(persistent))
    o.stall_window = int(stall_window or 0)
    o.s_step = int(s_step)
    return o


class Pattern:
    """A validated CSR pattern resident on one device (hsla_pattern)."""

    def __init__(self, row_ptr: torch.Tensor, col: torch.Tensor, csr_only: bool = False):
        """csr_only=True creates it with HSLA_PATTERN_CSR (no offset-mask forms)."""
        if not row_ptr.is_cuda:
            raise ValueError("row_ptr must be on a GPU")
        self.device = row_ptr.device
        self.row_ptr = need(row_ptr, torch.int32, "row_ptr", self.device)
        self.col = need(col, torch.int32, "col", self.device)
        self.n = self.row_ptr.numel() - 1
        self.nnz = self.col.numel()
        with torch.cuda.device(self.device):
            self.h = handle(self.device.index)
            p = ctypes.c_void_p()
            st = load().hsla_pattern_create(self.h, self.n, self.nnz, ptr(self.row_ptr), ptr(self.col),
                                            PATTERN_CSR if csr_only else 0, stream_ptr(self.device),
                                            ctypes.byref(p))
            check(st, self.h, "hsla_pattern_create")
        self.p = p
        n_ = ctypes.c_int32()
        nnz_ = ctypes.c_int64()
        nl = ctypes.c_int64()
        sym = ctypes.c_int32()
        load().hsla_pattern_info(self.p, ctypes.byref(n_), ctypes.byref(nnz_), ctypes.byref(nl), ctypes.byref(sym))
        self.nnz_lower = nl.value
        self.pattern_symmetric = bool(sym.value)

    @property
    def stencil(self) -> tuple[bool, int]:
        """(offset-mask form in use for A's SpMV, number of its diagonals or 0)."""
        use = ctypes.c_int32()
        nofs = ctypes.c_int32()
        load().hsla_pattern_format(self.p, ctypes.byref(use), ctypes.byref(nofs))
        return bool(use.value), nofs.value

    def set_format(self, fmt: str) -> None:
        """'auto' (offset-mask form where available), 'csr', or 'diagonal'
        (as 'auto', and SpMV calls also use the diagonal-major copy)."""
        st = load().hsla_pattern_set_format(self.p, FORMATS[fmt])
        if st != OK:
            raise HslaError(st, f"unknown format {fmt!r}")

    @property
    def signature(self) -> int:
        """64-bit hash of (n, nnz, row_ptr, col); equal patterns agree across processes."""
        v = ctypes.c_uint64()
        check(load().hsla_pattern_signature(self.p, ctypes.byref(v)), self.h, "hsla_pattern_signature")
        return v.value

    def get_tuning(self) -> dict:
        t = TuneState()
        check(load().hsla_pattern_get_tuning(self.p, ctypes.byref(t)), self.h, "hsla_pattern_get_tuning")
        return t.as_dict()

    def set_tuning(self, state: dict) -> None:
        t = TuneState(**{k: int(state[k]) for k, _ in TuneState._fields_})
        st = load().hsla_pattern_set_tuning(self.p, ctypes.byref(t))
        if st != OK:
            raise HslaError(st, "tuning record does not fit this pattern")

    def autotune(self, B: int = 1, effort: int = 5, cache: str | None = None) -> dict:
        """Times the solvers' SpMV forms and grid densities for a batch of B
        systems and keeps the fastest for later solves on this pattern.

        cache: a JSON file of tunings keyed by pattern signature, batch size and
        device architecture.  A stored record is applied without timing
        ({'cached': True, ...}); otherwise the timed choice is added to the
        file (written to a temporary file and renamed into place)."""
        key = None
        if cache is not None:
            arch = torch.cuda.get_device_properties(self.device).gcnArchName
            key = f"{self.signature:016x}/B{int(B)}/{arch}"
            stored = _read_tune_cache(cache).get(key)
            if stored is not None:
                self.set_tuning(stored)
                return {"cached": True, **stored}
        t = Tuning()
        with torch.cuda.device(self.device):
            st = load().hsla_autotune(self.h, self.p, int(B), int(effort), ctypes.byref(t), stream_ptr(self.device))
            check(st, self.h, "hsla_autotune")
        out = {"form": {0: "diagonal", 1: "tiles", 2: "diagonal-half"}[t.form], "blocks_per_cu": t.blocks_per_cu,
               "best_us": t.best_us, "default_us": t.default_us, "cached": False}
        if key is not None:
            _write_tune_cache(cache, key, self.get_tuning())
        return out

    def __del__(self):
        p = getattr(self, "p", None)
        if p is not None and _lib is not None:
            try:
                _lib.hsla_pattern_destroy(p)
            except Exception:
                pass
            self.p = None

    def transpose(self):
        """(row_ptr_T, col_T, src) of the transpose (device int32 tensors)."""
        rpT = torch.empty(self.n + 1, dtype=torch.int32, device=self.device)
        colT = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=self.device)
        src = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=self.device)
        with torch.cuda.device(self.device):
            st = load().hsla_pattern_transpose(self.h, self.p, ptr(rpT), ptr(colT), ptr(src), stream_ptr(self.device))
            check(st, self.h, "hsla_pattern_transpose")
        return rpT, colT[:self.nnz], src[:self.nnz]

    def colors(self):
        """(color int32 [n] on the device, number of colors): a column
        coloring in which columns sharing a row differ (hsla_pattern_colors)."""
        color = torch.empty(max(self.n, 1), dtype=torch.int32, device=self.device)
        nc = ctypes.c_int32()
        with torch.cuda.device(self.device):
            st = load().hsla_pattern_colors(self.h, self.p, ptr(color), ctypes.byref(nc), stream_ptr(self.device))
            check(st, self.h, "hsla_pattern_colors")
        return color[:self.n], nc.value

    def lower(self):
        """(row_ptr_L, col_L, pos) of the lower triangle incl. the diagonal
        (device int32 tensors; pos = position in A of each lower entry)."""
        rpL = torch.empty(self.n + 1, dtype=torch.int32, device=self.device)
        colL = torch.empty(max(self.nnz_lower, 1), dtype=torch.int32, device=self.device)
        pos = torch.empty(max(self.nnz_lower, 1), dtype=torch.int32, device=self.device)
        with torch.cuda.device(self.device):
            st = load().hsla_pattern_lower(self.h, self.p, ptr(rpL), ptr(colL), ptr(pos), stream_ptr(self.device))
            check(st, self.h, "hsla_pattern_lower")
        return rpL, colL[:self.nnz_lower], pos[:self.nnz_lower]


def _read_tune_cache(path: str) -> dict:
    import json
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _write_tune_cache(path: str, key: str, state: dict) -> None:
    import json
    d = _read_tune_cache(path)
    d[key] = state
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _batch(values: torch.Tensor, nnz: int) -> int:
    if values.dim() == 1:
        return 1
    if values.dim() == 2 and values.shape[1] == nnz:
        return values.shape[0]
    raise ValueError(f"values must have shape (nnz,) or (B, nnz), got {tuple(values.shape)}")


def spmv(pat: Pattern, values: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    values = need(values, torch.float64, "values", pat.device)
    x = need(x, torch.float64, "x", pat.device)
    B = _batch(values, pat.nnz)
    y = torch.empty_like(x)
    with torch.cuda.device(pat.device):
        st = load().hsla_spmv(pat.h, pat.p, B, ptr(values), ptr(x), ptr(y), stream_ptr(pat.device))
        check(st, pat.h, "hsla_spmv")
    return y


def solve(pat: Pattern, values: torch.Tensor, b: torch.Tensor, opts: Opts, x0: torch.Tensor | None = None):
    """Returns (x, [info dicts], status)."""
    values = need(values, torch.float64, "values", pat.device)
    b = need(b, torch.float64, "b", pat.device)
    B = _batch(values, pat.nnz)
    if b.numel() != B * pat.n:
        raise ValueError("b does not match the batch and pattern")
    x = torch.empty_like(b) if x0 is None else need(x0, torch.float64, "x0", pat.device).clone()
    infos = (Info * max(B, 1))()
    with torch.cuda.device(pat.device):
        st = load().hsla_solve_batched(pat.h, pat.p, B, ptr(values), ptr(b), ptr(x), ctypes.byref(opts),
                                       infos, stream_ptr(pat.device))
        check(st, pat.h, "hsla_solve")
    return x, [infos[i].as_dict() for i in range(B)], st


def csr_check(row_ptr, col, n: int | None = None):
    """hsla_csr_check on host arrays: (status, first bad row)."""
    import numpy as np

    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    n = len(rp) - 1 if n is None else int(n)
    bad = ctypes.c_int32()
    st = load().hsla_csr_check(n, int(cl.size), rp.ctypes.data_as(ctypes.c_void_p),
                               cl.ctypes.data_as(ctypes.c_void_p) if cl.size else None, ctypes.byref(bad))
    return st, bad.value


def solve_noalloc(pat: Pattern, values: torch.Tensor, b: torch.Tensor, x: torch.Tensor, opts: Opts):
    """hsla_solve_noalloc into the caller's x (same shape as b); returns
    ([info dicts], status).  The library allocates no device memory."""
    values = need(values, torch.float64, "values", pat.device)
    b = need(b, torch.float64, "b", pat.device)
    if not x.is_contiguous():
        raise ValueError("x must be contiguous (the solve writes into it)")
    x = need(x, torch.float64, "x", pat.device)
    B = _batch(values, pat.nnz)
    if b.numel() != B * pat.n or x.numel() != B * pat.n:
        raise ValueError("b or x does not match the batch and pattern")
    infos = (Info * max(B, 1))()
    with torch.cuda.device(pat.device):
        st = load().hsla_solve_noalloc(pat.h, pat.p, B, ptr(values), ptr(b), ptr(x), ctypes.byref(opts), infos,
                                       stream_ptr(pat.device))
        check(st, pat.h, "hsla_solve_noalloc")
    return [infos[i].as_dict() for i in range(B)], st


def adjoint(pat: Pattern, values: torch.Tensor, x: torch.Tensor, gx: torch.Tensor, opts: Opts,
            want_gA: bool = True, want_gb: bool = True):
    """Returns (gA or None, gb (lambda), [info dicts], status)."""
    values = need(values, torch.float64, "values", pat.device)
    x = need(x, torch.float64, "x", pat.device)
    gx = need(gx, torch.float64, "gx", pat.device)
    B = _batch(values, pat.nnz)
    gA = torch.empty_like(values) if want_gA else None
    gb = torch.empty_like(gx)
    infos = (Info * max(B, 1))()
    with torch.cuda.device(pat.device):
        st = load().hsla_adjoint_batched(pat.h, pat.p, B, ptr(values), ptr(x), ptr(gx), ptr(gA), ptr(gb),
                                         ctypes.byref(opts), infos, stream_ptr(pat.device))
        check(st, pat.h, "hsla_adjoint")
    return gA, gb, [infos[i].as_dict() for i in range(B)], st


def outer_on_pattern(pat: Pattern, lam: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    lam = need(lam, torch.float64, "lambda", pat.device)
    x = need(x, torch.float64, "x", pat.device)
    B = lam.numel() // max(pat.n, 1) if pat.n else 1
    gA = torch.empty((B, pat.nnz) if lam.dim() == 2 else (pat.nnz,), dtype=torch.float64, device=pat.device)
    with torch.cuda.device(pat.device):
        st = load().hsla_outer_on_pattern(pat.h, pat.p, B, ptr(lam), ptr(x), ptr(gA), stream_ptr(pat.device))
        check(st, pat.h, "hsla_outer_on_pattern")
    return gA


def residual_norms(pat: Pattern, values: torch.Tensor, b: torch.Tensor, x: torch.Tensor):
    values = need(values, torch.float64, "values", pat.device)
    b = need(b, torch.float64, "b", pat.device)
    x = need(x, torch.float64, "x", pat.device)
    B = _batch(values, pat.nnz)
    rn = (ctypes.c_double * B)()
    bn = (ctypes.c_double * B)()
    with torch.cuda.device(pat.device):
        st = load().hsla_residual_norms(pat.h, pat.p, B, ptr(values), ptr(b), ptr(x), rn, bn, stream_ptr(pat.device))
        check(st, pat.h, "hsla_residual_norms")
    return list(rn), list(bn)


# ---------------------------------------------------------------- learned FSAI

def mpnn_forward(pat: Pattern, values: torch.Tensor, params: torch.Tensor, keep: bool = False) -> torch.Tensor:
    values = need(values, torch.float64, "values", pat.device)
    params = need(params, torch.float32, "params", pat.device)
    B = _batch(values, pat.nnz)
    g = torch.empty((B, pat.nnz_lower) if values.dim() == 2 else (pat.nnz_lower,), dtype=torch.float32,
                    device=pat.device)
    with torch.cuda.device(pat.device):
        st = load().hsla_mpnn_forward(pat.h, pat.p, B, ptr(values), ptr(params), ptr(g), int(keep),
                                      stream_ptr(pat.device))
        check(st, pat.h, "hsla_mpnn_forward")
    return g


def mpnn_backward(pat: Pattern, B: int, dG: torch.Tensor) -> torch.Tensor:
    dG = need(dG, torch.float32, "dG", pat.device)
    grads = torch.empty(load().hsla_mpnn_num_params(), dtype=torch.float32, device=pat.device)
    with torch.cuda.device(pat.device):
        st = load().hsla_mpnn_backward(pat.h, pat.p, B, ptr(dG), ptr(grads), stream_ptr(pat.device))
        check(st, pat.h, "hsla_mpnn_backward")
    return grads


def probe_loss(pat: Pattern, values: torch.Tensor, G: torch.Tensor, Z: torch.Tensor, scale: float = 1.0,
               grad: bool = True):
    """(loss per system [B] (host list), dG or None)."""
    values = need(values, torch.float64, "values", pat.device)
    G = need(G, torch.float32, "G", pat.device)
    Z = need(Z, torch.float64, "Z", pat.device)
    B = _batch(values, pat.nnz)
    P = Z.numel() // (B * pat.n)
    loss = (ctypes.c_double * B)()
    dG = torch.empty_like(G) if grad else None
    with torch.cuda.device(pat.device):
        st = load().hsla_probe_loss(pat.h, pat.p, B, ptr(values), ptr(G), P, ptr(Z), float(scale), loss, ptr(dG),
                                    stream_ptr(pat.device))
        check(st, pat.h, "hsla_probe_loss")
    return list(loss), dG


def adam_step(params, grads, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    h = handle(params.device.index)
    with torch.cuda.device(params.device):
        st = load().hsla_adam_step(h, params.numel(), ptr(params), ptr(grads), ptr(m), ptr(v), float(lr),
                                   float(beta1), float(beta2), float(eps), int(step), stream_ptr(params.device))
        check(st, h, "hsla_adam_step")


def fsai_factors(pat: Pattern, values: torch.Tensor, Ghat: torch.Tensor):
    values = need(values, torch.float64, "values", pat.device)
    Ghat = need(Ghat, torch.float32, "Ghat", pat.device)
    B = _batch(values, pat.nnz)
    G = torch.empty_like(Ghat)
    GT = torch.empty_like(Ghat)
    with torch.cuda.device(pat.device):
        st = load().hsla_fsai_factors(pat.h, pat.p, B, ptr(values), ptr(Ghat), ptr(G), ptr(GT),
                                      stream_ptr(pat.device))
        check(st, pat.h, "hsla_fsai_factors")
    return G, GT


def solve_ragged(row_off: torch.Tensor, nnz_off: torch.Tensor, row_ptr: torch.Tensor, col: torch.Tensor,
                 values: torch.Tensor, b: torch.Tensor, opts: Opts):
    """Concatenated ragged batch (see hsla_solve_ragged).  Returns (x, infos, status)."""
    device = b.device
    row_off = need(row_off, torch.int64, "row_off", device)
    nnz_off = need(nnz_off, torch.int64, "nnz_off", device)
    row_ptr = need(row_ptr, torch.int32, "row_ptr", device)
    col = need(col, torch.int32, "col", device)
    values = need(values, torch.float64, "values", device)
    b = need(b, torch.float64, "b", device)
    B = row_off.numel() - 1
    x = torch.empty_like(b)
    infos = (Info * max(B, 1))()
    with torch.cuda.device(device):
        h = handle(device.index)
        st = load().hsla_solve_ragged(h, B, ptr(row_off), ptr(nnz_off), ptr(row_ptr), ptr(col), ptr(values),
                                      ptr(b), ptr(x), ctypes.byref(opts), infos, stream_ptr(device))
        check(st, h, "hsla_solve_ragged")
    return x, [infos[i].as_dict() for i in range(B)], st
