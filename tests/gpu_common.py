"""Helpers shared by the GPU parity tests: move seeded inputs to the device
and call the product path through its C-ABI binding."""
import numpy as np
import torch


def dev():
    return torch.device("cuda:0")


def t64(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(dev())


def t32(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.int32)).to(dev())


def pattern(a):
    from paper_2601_13994_amd import _lib

    return _lib.Pattern(t32(a.row_ptr), t32(a.col))


def solve(a, b, pat=None, values=None, **kw):
    from paper_2601_13994_amd import _lib

    pat = pat or pattern(a)
    vals = t64(a.val) if values is None else values
    opts = _lib.make_opts(**kw)
    x, infos, st = _lib.solve(pat, vals, t64(b), opts)
    return x.cpu().numpy(), infos, st


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def iters_close(a, b):
    """Iteration counts of two FP64 runs that differ only in rounding order."""
    return abs(a - b) <= max(2, int(0.02 * max(a, b)))
