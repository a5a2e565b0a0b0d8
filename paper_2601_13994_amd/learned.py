"""Learned FSAI preconditioner: M^{-1} = G^T G with G lower triangular on A's
lower pattern, positive diagonal, values from a message-passing network over
A's graph (kernels in csrc/mpnn.hip; the paper names learned preconditioners
as future work, so the network is this project's design).

Training minimises the probe loss E_z ||G^ A^ G^^T z - z||^2 with Rademacher
probes z, i.e. drives G^ A^ G^^T towards the identity, on systems the project
generates itself; everything runs on the GPU through the C ABI (forward,
backward, probe loss and Adam are library kernels).
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import _lib
from ._lib import Pattern

HID, HEAD, NF, LAYERS = 64, 32, 4, 3
KH = 2 * HID + NF

LAYOUT = [("W0", (NF, HID)), ("b0", (HID,))]
for _l in range(1, LAYERS + 1):
    LAYOUT += [(f"C{_l}", (NF, HID)), (f"W{_l}", (2 * HID, HID)), (f"b{_l}", (HID,))]
LAYOUT += [("H1", (KH, HEAD)), ("c1", (HEAD,)), ("H2", (HEAD,)), ("c2", (1,))]
NUM_PARAMS = sum(int(np.prod(s)) for _, s in LAYOUT)


def pack(d: dict) -> np.ndarray:
    """Packed float32 parameter vector in the library's layout."""
    return np.concatenate([np.asarray(d[k], dtype=np.float32).reshape(-1) for k, _ in LAYOUT])


def unpack(v) -> dict:
    v = np.asarray(v, dtype=np.float64)
    out, o = {}, 0
    for k, s in LAYOUT:
        c = int(np.prod(s))
        out[k] = v[o:o + c].reshape(s)
        o += c
    return out


def initial_params(seed: int = 0) -> np.ndarray:
    """He-scaled random matrices, zero biases, a small output layer, and c2
    chosen so the diagonal starts at softplus(c2) = 1 (G^ close to I, i.e.
    close to Jacobi on the scaled system)."""
    r = np.random.default_rng(seed)
    d = {}
    for k, s in LAYOUT:
        if k.startswith(("b", "c")):
            d[k] = np.zeros(s)
        elif k.startswith("C"):
            d[k] = r.standard_normal(s) * 0.5
        elif k == "H2":
            d[k] = r.standard_normal(s) * 0.01 / math.sqrt(HEAD)
        else:
            d[k] = r.standard_normal(s) * math.sqrt(2.0 / s[0])
    d["c2"] = np.array([math.log(math.e - 1.0)])
    return pack(d)


def aniso_batch_values(slots: torch.Tensor, stencils: torch.Tensor) -> torch.Tensor:
    """Values [B][nnz] of B anisotropic systems on one 9-point pattern:
    value of entry k of system s = stencils[s][slots[k]] (an exact gather)."""
    return stencils[:, slots].contiguous()


class LearnedFSAI:
    """Holds the network parameters (float32, on the GPU) and builds factors."""

    def __init__(self, params=None, device="cuda:0", seed: int = 0):
        self.device = torch.device(device)
        if params is None:
            params = initial_params(seed)
        self.params = torch.as_tensor(np.asarray(params, dtype=np.float32)).to(self.device).contiguous()
        assert self.params.numel() == _lib.load().hsla_mpnn_num_params() == NUM_PARAMS

    def ghat(self, pat: Pattern, values: torch.Tensor) -> torch.Tensor:
        return _lib.mpnn_forward(pat, values, self.params, keep=False)

    def factors(self, pat: Pattern, values: torch.Tensor, chunk: int = 64):
        """(G, G^T values) for every system (values [B][nnz] or [nnz])."""
        if values.dim() == 1:
            return _lib.fsai_factors(pat, values, self.ghat(pat, values))
        Gs, GTs = [], []
        for s in range(0, values.shape[0], chunk):
            v = values[s:s + chunk]
            G, GT = _lib.fsai_factors(pat, v, self.ghat(pat, v))
            Gs.append(G)
            GTs.append(GT)
        return torch.cat(Gs), torch.cat(GTs)

    def calibrate(self, pat: Pattern, values: torch.Tensor, b: torch.Tensor, rtol=1e-8) -> int:
        """Runs Jacobi-PCG on a sample of systems (values [B][nnz], b [B][n])
        and records its largest iteration count; solve() then caps every
        FSAI attempt at twice that count."""
        _, infos, _ = _lib.solve(pat, values, b, _lib.make_opts(method="cg", precond="jacobi", rtol=rtol))
        self.jacobi_iters = max(f["iters"] for f in infos)
        return self.jacobi_iters

    @staticmethod
    def default_stall_window(n: int) -> int:
        """Iterations within which FSAI-PCG must cut ||r|| tenfold: 2 sqrt(n),
        at least 50 (Jacobi-PCG on the 2D anisotropic operators needs about
        sqrt(n) iterations per decade at the largest anisotropy)."""
        return max(50, 2 * math.isqrt(max(n - 1, 0)) + 2)

    def solve(self, pat: Pattern, values: torch.Tensor, b: torch.Tensor, rtol=1e-8, max_iter=0, factors=None,
              stall_window: int | None = None):
        """FSAI-PCG with the learned factor, Jacobi-PCG as the fallback.

        A system's FSAI attempt is abandoned, and the system solved again with
        Jacobi-PCG and reported with status FELL_BACK, when its factor is
        invalid (a non-finite value or a non-positive diagonal: the library
        stops it before the first iteration), when ||r|| falls less than
        tenfold within `stall_window` iterations (default
        default_stall_window(n); 0 turns the test off), when it reaches the
        attempt's cap (twice the Jacobi count recorded by calibrate(), else
        max_iter or the library default), or on a breakdown.  The info of a
        fallen-back system is its Jacobi solve's, plus the FSAI attempt's
        status and iterations ('fsai_status', 'fsai_iters').
        Returns (x, infos, status)."""
        G, GT = factors if factors is not None else self.factors(pat, values)
        if stall_window is None:
            stall_window = self.default_stall_window(pat.n)
        cap = max_iter
        if not cap and getattr(self, "jacobi_iters", 0):
            cap = 2 * self.jacobi_iters
        opts = _lib.make_opts(method="cg", precond="fsai", rtol=rtol, max_iter=cap, G=G, GT=GT,
                              stall_window=stall_window)
        x, infos, st = _lib.solve(pat, values, b, opts)
        if st == _lib.OK:
            return x, infos, st
        bad = [i for i, f in enumerate(infos) if f["status"] != _lib.OK]
        jopts = _lib.make_opts(method="cg", precond="jacobi", rtol=rtol, max_iter=max_iter)
        if values.dim() == 1:
            x, fb, _ = _lib.solve(pat, values, b, jopts)
        else:
            idx = torch.as_tensor(bad, device=values.device)
            xb, fb, _ = _lib.solve(pat, values[idx].contiguous(), b.view(values.shape[0], -1)[idx].contiguous(), jopts)
            x.view(values.shape[0], -1)[idx] = xb.view(len(bad), -1)
        worst = _lib.OK
        for i, f in zip(bad, fb):
            f["fsai_status"], f["fsai_iters"] = infos[i]["status"], infos[i]["iters"]
            f["status"] = _lib.FELL_BACK if f["status"] == _lib.OK else f["status"]
            infos[i] = f
        for f in infos:
            if f["status"] not in (_lib.OK, _lib.FELL_BACK):
                worst = f["status"]
        return x, infos, (worst if worst != _lib.OK else _lib.FELL_BACK)

    def train(self, pat: Pattern, sample_values, steps: int, probes: int = 4, lr: float = 3e-3,
              log_every: int = 0, seed: int = 0, lr_final: float | None = None):
        """Adam on the mean probe loss (1/(B P n)) sum ||G^ A^ G^^T z - z||^2.
        sample_values(step) returns the values [B][nnz] of one minibatch."""
        m = torch.zeros_like(self.params)
        v = torch.zeros_like(self.params)
        gen = torch.Generator(device=self.device)
        gen.manual_seed(seed)
        hist = []
        t0 = time.time()
        for step in range(1, steps + 1):
            vals = sample_values(step)
            B = vals.shape[0]
            Z = (torch.randint(0, 2, (B, probes, pat.n), generator=gen, device=self.device, dtype=torch.int8)
                 .to(torch.float64) * 2.0 - 1.0)
            g = _lib.mpnn_forward(pat, vals, self.params, keep=True)
            scale = 1.0 / (B * probes * pat.n)
            loss, dG = _lib.probe_loss(pat, vals, g, Z, scale=scale, grad=True)
            grads = _lib.mpnn_backward(pat, B, dG)
            lr_t = lr if lr_final is None else lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * step / steps))
            _lib.adam_step(self.params, grads, m, v, lr_t, step)
            hist.append(sum(loss))
            if log_every and step % log_every == 0:
                print(f"[train] step {step} loss {np.mean(hist[-log_every:]):.4f} ({time.time() - t0:.1f}s)",
                      flush=True)
        return hist
