"""Parity at the benchmark's full sizes, in the launch configurations the
benchmark times, on outputs the oracle can compute one by one: a few
iterations of the 256^3 system, sampled systems of the ragged and
shared-pattern batches, finite differences of the loss through the GPU
solver, and the learned preconditioner at 256^2."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from gpu_common import dev, iters_close, pattern, rel, t32, t64  # noqa: E402
import paper_2601_13994_amd as hs  # noqa: E402
from paper_2601_13994_amd import _lib, learned  # noqa: E402
from oracle import mpnn  # noqa: E402


def _log(*a):
    print("[fullsize]", *a, flush=True)


def test_diffusion3d_256_first_iterations(orc):
    """n = 16.8M, nnz = 117M: the first iterations of Jacobi-PCG and of
    Jacobi-BiCGStab (upwind, cell Peclet 10) agree with the oracle's to
    rounding; both runs stop at the iteration cap."""
    a, b = W.diffusion3d_workload(256)
    pat = pattern(a)
    bt = t64(b)
    k = 4
    x, infos, st = _lib.solve(pat, t64(a.val), bt, _lib.make_opts(method="cg", precond="jacobi", rtol=1e-8,
                                                                  max_iter=k))
    assert st == _lib.NOT_CONVERGED and infos[0]["iters"] == k
    ref = orc.cg(a, b, precond="jacobi", rtol=1e-8, max_iter=k)
    assert ref.iters == k
    assert rel(x.cpu().numpy(), ref.x) <= 1e-12
    _log("cg", rel(x.cpu().numpy(), ref.x))
    conv = a.with_values(W.diffusion3d_values(256, W.diffusion3d_kappa(256), velocity=10.0))
    x, infos, st = _lib.solve(pat, t64(conv.val), bt, _lib.make_opts(method="bicgstab", precond="jacobi",
                                                                     rtol=1e-8, max_iter=k))
    assert st == _lib.NOT_CONVERGED and infos[0]["iters"] == k
    ref = orc.bicgstab(conv, b, precond="jacobi", rtol=1e-8, max_iter=k)
    assert rel(x.cpu().numpy(), ref.x) <= 1e-12
    _log("bicgstab", rel(x.cpu().numpy(), ref.x))


@pytest.mark.parametrize("persistent", [True, "force"])
def test_ragged_knn_full_sizes(orc, persistent):
    """512 systems (64 distinct full-size k-NN Laplacians, each 8 times):
    with the default routing the batch (13M rows) runs on the segmented
    per-iteration path; "force" runs it in one persistent launch.  Copies
    agree bitwise, sampled systems match the oracle at rtol 1e-12, every
    system's FP64 residual meets the tolerance; the persistent launch
    reports when each workgroup took and finished its system."""
    distinct = [W.knn_system(s) for s in range(64)]
    systems = [distinct[i % 64] for i in range(512)]
    mats = [(t64(a.val), t32(a.row_ptr), t32(a.col)) for a, _ in distinct]
    L = hs.SparseCSRList([mats[i % 64] for i in range(512)])
    xs, infos, st = L.solve([t64(b) for _, b in systems], rtol=1e-12, persistent=persistent)
    assert st == _lib.OK
    if persistent == "force":
        assert all(f["spmv_form"] == "persistent" for f in infos)
        wg = infos[0]["workgroups"]
        assert 0 < wg <= 512 and all(0.0 <= f["t_start_ms"] <= f["t_end_ms"] for f in infos)
        busy = sum(f["t_end_ms"] - f["t_start_ms"] for f in infos)
        wall = max(f["t_end_ms"] for f in infos)
        _log("persistent knn: wall", wall, "ms, load balance", busy / (wg * wall))
        assert 0.0 < busy / (wg * wall) <= 1.0 + 1e-9
    else:
        assert all(f["spmv_form"] != "persistent" for f in infos)
    for i in range(64, 512):
        assert torch.equal(xs[i], xs[i % 64])
        assert infos[i]["iters"] == infos[i % 64]["iters"]
    assert max(f["true_residual"] for f in infos) <= 5e-12
    for s in (0, 17, 63):
        a, b = distinct[s]
        ref = orc.cg(a, b, precond="jacobi", rtol=1e-12)
        assert rel(xs[s].cpu().numpy(), ref.x) <= 1e-8
        assert iters_close(infos[s]["iters"], ref.iters)
        _log("knn", s, a.n, rel(xs[s].cpu().numpy(), ref.x))


def _kappa_hat(ref):
    """Condition number estimate of the preconditioned operator from CG's
    coefficients: extreme eigenvalues of the Lanczos tridiagonal."""
    al, be = ref.alphas, ref.betas
    k = len(al)
    d = 1.0 / al
    d[1:] += be[:k - 1] / al[:k - 1]
    e = np.sqrt(be[:k - 1]) / al[:k - 1]
    ev = np.linalg.eigvalsh(np.diag(d) + np.diag(e, 1) + np.diag(e, -1))
    return ev[-1] / ev[0]


@pytest.mark.slow
@pytest.mark.parametrize("method", ["cg", "bicgstab"])
def test_diffusion3d_256_full_solve(orc, method):
    """The headline system (and its upwind variant under BiCGStab) solved to
    rtol 1e-12 on the GPU in the configuration the benchmark times and by the
    oracle on all host cores: ||x_gpu - x_oracle|| / ||x_oracle|| <= 1e-8,
    iteration counts within max(2, 2%), and the reported true residual equal
    to the oracle's ||b - A x_gpu|| / ||b||.  For CG the Lanczos estimate of
    the preconditioned condition number is logged: the worst-case bound
    kappa * 2e-12 on the difference of two rtol-1e-12 solutions."""
    import os

    a, b = W.diffusion3d_workload(256)
    if method == "bicgstab":
        a = a.with_values(W.diffusion3d_values(256, W.diffusion3d_kappa(256), velocity=10.0))
    pat = pattern(a)
    x, infos, st = _lib.solve(pat, t64(a.val), t64(b), _lib.make_opts(method=method, precond="jacobi", rtol=1e-12))
    assert st == _lib.OK
    x = x.cpu().numpy()
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    with orc.threads(threads):
        if method == "cg":
            ref = orc.cg(a, b, precond="jacobi", rtol=1e-12, history=True)
        else:
            ref = orc.bicgstab(a, b, precond="jacobi", rtol=1e-12)
        tr = orc.residual_norm(a, b, x) / np.linalg.norm(b)
    assert ref.status == 0
    err = rel(x, ref.x)
    kh = _kappa_hat(ref) if method == "cg" else float("nan")
    _log(method, "gpu iters", infos[0]["iters"], "oracle iters", ref.iters, "rel diff", err, "kappa_hat", kh,
         "true residual gpu", infos[0]["true_residual"], "oracle's", tr)
    assert err <= 1e-8
    assert iters_close(infos[0]["iters"], ref.iters)
    assert abs(infos[0]["true_residual"] - tr) <= 1e-10 * tr


def test_shared_pattern_96_adjoint_and_fd(orc):
    """128 systems on one 96^3 pattern (4 distinct coefficient fields, one b
    and x* per system), forward + adjoint batched.  System 0 against the
    oracle (x, dL/db, dL/dA at rtol 1e-12); every system's forward and
    adjoint FP64 residuals; and central finite differences (h = 1e-6 on the
    raw value) of L = 1/2 ||x - x*||^2 on 64 (system, entry) pairs drawn
    without replacement from 128 x nnz.  Each difference is taken by
    correction solves: with the converged x~, (A +- h E_ij) d = b - A x~
    -+ h x~_j e_i is solved for d (BiCGStab, the perturbed matrix being
    nonsymmetric), so x~ + d is the perturbed solution and no O(1) quantity
    is differenced; the 128 perturbed systems run as one batch."""
    m, B = 96, 128
    a0, V4, _, _ = W.shared_pattern_batch(m, 4)
    n, nnz = a0.n, a0.nnz
    pat = pattern(a0)
    V = t64(V4).repeat(B // 4, 1).contiguous()
    bs = np.stack([W.rng(4, 1, s).standard_normal(n) for s in range(B)])
    xst = np.stack([W.rng(4, 2, s).standard_normal(n) for s in range(B)])
    bt, xt = t64(bs), t64(xst)
    opts = _lib.make_opts(method="cg", precond="jacobi", rtol=1e-12)
    x, fi, st = _lib.solve(pat, V, bt, opts)
    assert st == _lib.OK
    gx = (x - xt).contiguous()
    gA, gb, bi, st2 = _lib.adjoint(pat, V, x, gx, opts)
    assert st2 == _lib.OK
    # rtol bounds the recursive residual; the recomputed FP64 residual may
    # exceed it by the recurrence's rounding drift (seen up to about 2x here)
    rn, bn = _lib.residual_norms(pat, V, bt, x)
    assert max(r / c for r, c in zip(rn, bn)) <= 5e-12
    rn, bn = _lib.residual_norms(pat, V, gx, gb)
    assert max(r / c for r, c in zip(rn, bn)) <= 5e-12
    _log("batch residuals ok")

    a = a0.with_values(V4[0])
    ref = orc.cg(a, bs[0], precond="jacobi", rtol=1e-12)
    x0 = x[0].cpu().numpy()
    assert rel(x0, ref.x) <= 1e-8
    gA_o, gb_o, _ = orc.adjoint(a, ref.x, ref.x - xst[0], method="cg", precond="jacobi", rtol=1e-12)
    assert rel(gb[0].cpu().numpy(), gb_o) <= 1e-8
    assert rel(gA[0].cpu().numpy(), gA_o) <= 1e-6
    _log("oracle", rel(x0, ref.x), rel(gA[0].cpu().numpy(), gA_o))

    h = 1e-6
    flat = W.rng(4, 3, 0).choice(B * nnz, 64, replace=False)
    sy, ks = flat // nnz, flat % nnz
    rows, cols = a0.rows()[ks], a0.col[ks]
    sel = torch.as_tensor(sy, device=dev())
    two = torch.arange(64, device=dev()) * 2
    kt = torch.as_tensor(ks, device=dev())
    rt = torch.as_tensor(rows.astype(np.int64), device=dev())
    xj = x[sel, torch.as_tensor(cols.astype(np.int64), device=dev())]
    Vs = V[sel].contiguous()
    resid = bt[sel] - _lib.spmv(pat, Vs, x[sel].contiguous())
    P = Vs.repeat_interleave(2, dim=0).contiguous()
    rhs = resid.repeat_interleave(2, dim=0).contiguous()
    P[two, kt] += h
    P[two + 1, kt] -= h
    rhs[two, rt] -= h * xj
    rhs[two + 1, rt] += h * xj
    copts = _lib.make_opts(method="bicgstab", precond="jacobi", rtol=1e-12, max_iter=4000)
    d, di, st3 = _lib.solve(pat, P, rhs, copts)
    assert st3 == _lib.OK
    dp, dm = d[0::2], d[1::2]
    e = x[sel] - xt[sel]
    dl = ((dp - dm) * e).sum(dim=1) + 0.5 * ((dp * dp).sum(dim=1) - (dm * dm).sum(dim=1))
    fd = (dl / (2 * h)).cpu().numpy()
    g = gA[sel, kt].cpu().numpy()
    err = np.linalg.norm(fd - g) / np.linalg.norm(g)
    _log("fd", err, max(f["iters"] for f in di))
    assert err <= 1e-6


@pytest.mark.parametrize("method", ["cg_sr", "cg_sstep"])
def test_single_reduction_96_batch(orc, method):
    """The single-reduction and s-step (s = 4) recurrences on the
    per-iteration kernels over a 16-system batch on one 96^3 pattern (4
    coefficient fields): a sampled system against the oracle's CG (x to 1e-8
    at rtol 1e-12, iterations within max(2, 2%)), every system's FP64
    residual, and each system's iteration count within max(2, 2%) of the
    two-reduction CG's."""
    m, B = 96, 16
    a0, V4, _, _ = W.shared_pattern_batch(m, 4)
    n = a0.n
    pat = pattern(a0)
    V = t64(V4).repeat(B // 4, 1).contiguous()
    bs = np.stack([W.rng(4, 5, s).standard_normal(n) for s in range(B)])
    bt = t64(bs)
    kw = dict(precond="jacobi", rtol=1e-12, persistent=False)
    x, fi, st = _lib.solve(pat, V, bt, _lib.make_opts(method=method, **kw))
    assert st == _lib.OK and all(f["method"] == method for f in fi)
    xc, ci, stc = _lib.solve(pat, V, bt, _lib.make_opts(method="cg", **kw))
    assert stc == _lib.OK
    assert all(iters_close(f["iters"], g["iters"]) for f, g in zip(fi, ci)), \
        [(f["iters"], g["iters"]) for f, g in zip(fi, ci)]
    rn, bn = _lib.residual_norms(pat, V, bt, x)
    assert max(r / c for r, c in zip(rn, bn)) <= 5e-12
    s = 5
    ref = orc.cg(a0.with_values(V4[s % 4]), bs[s], precond="jacobi", rtol=1e-12)
    assert rel(x[s].cpu().numpy(), ref.x) <= 1e-8
    assert iters_close(fi[s]["iters"], ref.iters), (fi[s]["iters"], ref.iters)
    _log(method, "96^3", fi[s]["iters"], ref.iters, rel(x[s].cpu().numpy(), ref.x))


def test_learned_fsai_256(orc):
    """The network at 256^2 (n = 65,536, nnz = 586,756): its output for a
    held-out system against the FP64 reference with bf16 rounding at the
    same points, and FSAI-PCG over 1024 held-out systems batched with the
    GPU's factors at rtol 1e-12: sampled systems match the oracle's FSAI-PCG
    with the same float32 factor, and every system's FP64 residual meets
    the tolerance."""
    m = 256
    pa, slots = W.aniso_pattern(m)
    pat = pattern(pa)
    E = 1024
    st_eval = t64(np.stack([W.aniso_stencil(*W.aniso_params(s, heldout=True)) for s in range(E)]))
    V = learned.aniso_batch_values(torch.as_tensor(slots).to(dev()), st_eval)
    bs = np.stack([W.rng(5, 5, s).standard_normal(pa.n) for s in range(E)])
    bt = t64(bs)
    model = learned.LearnedFSAI(seed=0)
    p64 = {k: np.asarray(v, np.float32).astype(np.float64) for k, v in learned.unpack(model.params.cpu()).items()}
    g0 = model.ghat(pat, V[:1].contiguous()).cpu().numpy().reshape(-1)
    a0 = pa.with_values(V[0].cpu().numpy())
    ref, _ = mpnn.forward(p64, a0, bf=True)
    _log("network forward vs oracle", rel(g0, ref))
    assert rel(g0, ref) <= 1e-3  # relative Frobenius bound for the bf16 network
    G, GT = model.factors(pat, V)
    assert torch.isfinite(G).all()
    x, infos, st = _lib.solve(pat, V, bt, _lib.make_opts(method="cg", precond="fsai", rtol=1e-12, G=G, GT=GT))
    assert st == _lib.OK
    rn, bn = _lib.residual_norms(pat, V, bt, x)
    assert max(r / c for r, c in zip(rn, bn)) <= 5e-12
    rpL, colL, _ = orc.lower_pattern(a0)
    for s in (0, 511, 1023):
        a = pa.with_values(V[s].cpu().numpy())
        Gs = G[s].cpu().numpy().astype(np.float64)
        ref = orc.fsai_pcg(a, rpL, colL, Gs, bs[s], rtol=1e-12)
        assert ref.status == 0
        assert rel(x[s].cpu().numpy(), ref.x) <= 1e-8
        assert iters_close(infos[s]["iters"], ref.iters)
        _log("fsai", s, infos[s]["iters"], ref.iters, rel(x[s].cpu().numpy(), ref.x))
