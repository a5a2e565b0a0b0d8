"""The allocation-free solve (hsla_solve_noalloc) against hsla_solve_batched
through the C ABI: bit-identical results on calls in a row of shrinking
size (per-iteration kernels, the persistent small-system kernel,
BiCGStab), parity with the oracle, no workspace allocation, and sizes
beyond its scratch array or batch limit rejected without writing x."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from gpu_common import dev, iters_close, pattern, rel, t64  # noqa: E402
from paper_2601_13994_amd import _lib  # noqa: E402


def _diffusion_batch(m, B, velocity=0.0):
    a = W.diffusion3d(m)
    V = np.stack([W.diffusion3d_values(m, W.diffusion3d_kappa(m, cfg=4, sample=s), velocity) for s in range(B)])
    bs = np.stack([W.rng(4, 1, s).standard_normal(a.n) for s in range(B)])
    return a, V, bs


def _poisson_batch(m, B):
    a = W.poisson2d(m)
    bs = np.stack([W.rng(1, 1, s).standard_normal(a.n) for s in range(B)])
    return a, np.stack([a.val] * B), bs


def _both(a, V, bs, **kw):
    """(x from hsla_solve_noalloc, its infos, x from hsla_solve_batched, its infos)."""
    pat = pattern(a)
    vals, b = t64(V), t64(bs)
    opts = _lib.make_opts(graph=False, **kw)
    x = torch.full_like(b, np.nan)
    infos, st = _lib.solve_noalloc(pat, vals, b, x, opts)
    assert st == _lib.OK, (st, infos)
    xr, infos_r, st_r = _lib.solve(pat, vals, b, opts)
    assert st_r == _lib.OK
    return x.cpu().numpy(), infos, xr.cpu().numpy(), infos_r


def _vs_oracle(orc, a, V, bs, x, infos, method, precond):
    for s in range(len(V)):
        ai = a.with_values(V[s])
        if method == "cg":
            ref = orc.cg(ai, bs[s], precond=precond, rtol=1e-12)
        else:
            ref = orc.bicgstab(ai, bs[s], precond=precond, rtol=1e-12)
        assert ref.status == 0
        assert rel(x[s], ref.x) <= 1e-8, (s, rel(x[s], ref.x))
        assert iters_close(infos[s]["iters"], ref.iters), (s, infos[s]["iters"], ref.iters)


def test_noalloc_matches_batched_on_shrinking_calls(orc):
    # 1) three 24^3 diffusion systems: per-iteration kernels, half copy of S A S
    a, V, bs = _diffusion_batch(24, 3)
    x, infos, xr, infos_r = _both(a, V, bs, method="cg", precond="jacobi", rtol=1e-12)
    assert np.array_equal(x, xr)
    assert [f["iters"] for f in infos] == [f["iters"] for f in infos_r]
    assert infos[0]["spmv_form"] != "persistent"
    _vs_oracle(orc, a, V, bs.reshape(3, -1), x.reshape(3, -1), infos, "cg", "jacobi")
    # 2) a smaller call right after: two 20 x 20 Poisson systems, persistent kernel
    a, V, bs = _poisson_batch(20, 2)
    x, infos, xr, infos_r = _both(a, V, bs, method="cg", precond="none", rtol=1e-12)
    assert np.array_equal(x, xr)
    assert infos[0]["spmv_form"] == "persistent"
    _vs_oracle(orc, a, V, bs, x.reshape(2, -1), infos, "cg", "none")
    # 3) smaller again: one 12^3 upwind system under Jacobi-BiCGStab
    a, V, bs = _diffusion_batch(12, 1, velocity=10.0)
    x, infos, xr, infos_r = _both(a, V, bs, method="bicgstab", precond="jacobi", rtol=1e-12)
    assert np.array_equal(x, xr)
    _vs_oracle(orc, a, V, bs, x.reshape(1, -1), infos, "bicgstab", "jacobi")


def test_noalloc_allocates_nothing_and_rejects_oversize():
    a, V, bs = _diffusion_batch(16, 2)
    pat = pattern(a)
    vals, b = t64(V), t64(bs)
    opts = _lib.make_opts(method="cg", precond="jacobi", rtol=1e-10, graph=False)
    count = {}
    # a counting allocator also releases the handle's workspace: whatever the
    # library needs next would have to come through it
    _lib.use_torch_allocator(dev(), counter=count)
    try:
        x = torch.empty_like(b)
        infos, st = _lib.solve_noalloc(pat, vals, b, x, opts)
        assert st == _lib.OK and count.get("alloc", 0) == 0, count
        xr, _, _ = _lib.solve(pat, vals, b, opts)
        assert count.get("alloc", 0) >= 1  # the ordinary entry point allocates its workspace
        assert np.array_equal(x.cpu().numpy(), xr.cpu().numpy())
    finally:
        _lib.use_torch_allocator(dev(), enable=False)
    # more systems than the entry point takes
    big = _poisson_batch(4, 1025)
    pb = pattern(big[0])
    xb = torch.zeros(1025 * big[0].n, dtype=torch.float64, device=dev())
    with pytest.raises(_lib.HslaError) as e:
        _lib.solve_noalloc(pb, t64(big[1]), t64(big[2]), xb, opts)
    assert e.value.status == _lib.ERR_INVALID_ARG
    # a workspace beyond the 64 MiB array: rejected, x untouched
    m = 100
    a2 = W.diffusion3d(m)
    assert _lib.workspace_size(pattern(a2), 1, opts) > 64 << 20
    x2 = torch.full((a2.n,), 7.0, dtype=torch.float64, device=dev())
    with pytest.raises(_lib.HslaError) as e:
        _lib.solve_noalloc(pattern(a2), t64(a2.val), t64(np.ones(a2.n)), x2, opts)
    assert e.value.status == _lib.ERR_INVALID_ARG and "scratch" in str(e.value)
    assert bool((x2 == 7.0).all())
    # the handle still serves both entry points afterwards
    x = torch.empty_like(b)
    _, st = _lib.solve_noalloc(pat, vals, b, x, opts)
    xr, _, _ = _lib.solve(pat, vals, b, opts)
    assert st == _lib.OK and np.array_equal(x.cpu().numpy(), xr.cpu().numpy())
