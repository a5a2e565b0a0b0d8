"""GPU parity of the learned-FSAI path (network forward/backward with bf16
matrix cores, probe loss, factor conversion, FSAI-PCG, Adam) against the CPU
oracle, through the C ABI."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from gpu_common import dev, iters_close, pattern, rel, t32, t64  # noqa: E402
from paper_2601_13994_amd import _lib, learned  # noqa: E402
from oracle import mpnn  # noqa: E402


def _systems(m, count, seed=0):
    pat_a, slots = W.aniso_pattern(m)
    vals = []
    for s in range(count):
        ratio, ang = W.aniso_params(seed + s)
        vals.append(W.aniso_stencil(ratio, ang)[slots])
    return pat_a, np.stack(vals)


def _oracle_params(seed):
    p = mpnn.init_params(seed)
    for k in p:
        if k.startswith(("b", "c")):
            p[k] = np.random.default_rng(seed + 11).standard_normal(p[k].shape) * 0.1
    return p


def test_packed_layout_matches_library():
    assert learned.NUM_PARAMS == _lib.load().hsla_mpnn_num_params()
    d = _oracle_params(0)
    assert all(np.array_equal(np.asarray(d[k], np.float32), learned.unpack(learned.pack(d))[k].astype(np.float32))
               for k in d)


@pytest.mark.parametrize("m,B", [(9, 1), (17, 3)])
def test_mpnn_forward_parity(m, B):
    """G^ from the bf16/MFMA kernels vs the FP64 reference with bf16 rounding
    at the same points; several tiles of 16 rows and a ragged tail."""
    a, V = _systems(m, B)
    p = _oracle_params(1)
    pv = learned.pack(p)
    pat = pattern(a)
    g = _lib.mpnn_forward(pat, t64(V), torch.as_tensor(pv).to(dev())).cpu().numpy().reshape(B, -1)
    p32 = {k: np.asarray(v, np.float32).astype(np.float64) for k, v in p.items()}
    for s in range(B):
        ref, _ = mpnn.forward(p32, a.with_values(V[s]), bf=True)
        assert g[s].shape == ref.shape
        # the same bf16 cast points: only float32 vs float64 accumulation
        # differs, so a cast rarely rounds the other way (measured ~1e-8)
        assert rel(g[s], ref) <= 1e-5, (s, rel(g[s], ref))
        assert np.max(np.abs(g[s] - ref)) <= 1e-4 * np.max(np.abs(ref))


def test_mpnn_backward_parity():
    m, B = 11, 2
    a, V = _systems(m, B, seed=5)
    p = _oracle_params(2)
    p32 = {k: np.asarray(v, np.float32).astype(np.float64) for k, v in p.items()}
    pat = pattern(a)
    params = torch.as_tensor(learned.pack(p)).to(dev())
    g = _lib.mpnn_forward(pat, t64(V), params, keep=True)
    dg = np.random.default_rng(3).standard_normal(g.shape).astype(np.float32)
    grads = _lib.mpnn_backward(pat, B, torch.as_tensor(dg).to(dev())).cpu().numpy()
    gd = learned.unpack(grads)
    tot = {k: np.zeros_like(v) for k, v in p.items()}
    for s in range(B):
        _, cache = mpnn.forward(p32, a.with_values(V[s]), bf=True)
        gr = mpnn.backward(cache, dg[s].astype(np.float64))
        for k in tot:
            tot[k] += gr[k]
    for k in tot:
        assert rel(gd[k], tot[k]) <= 1e-4, (k, rel(gd[k], tot[k]))  # measured <= 2e-6
    # a second kept forward with another batch is required before another backward
    with pytest.raises(_lib.HslaError):
        _lib.mpnn_backward(pat, B + 1, torch.as_tensor(dg).to(dev()))


def test_probe_loss_parity(orc):
    m, B, P = 10, 2, 3
    a, V = _systems(m, B, seed=9)
    pat = pattern(a)
    r = np.random.default_rng(4)
    Gs, Zs = [], []
    for s in range(B):
        ah = mpnn.scaled(a.with_values(V[s]))
        rpL, colL, g = orc.fsai(ah)
        Gs.append((g * (1 + 0.05 * r.standard_normal(g.shape))).astype(np.float32))
        Zs.append(W.rademacher(r, (P, a.n)))
    G = np.stack(Gs)
    Z = np.stack(Zs)
    loss, dG = _lib.probe_loss(pat, t64(V), torch.as_tensor(G).to(dev()), t64(Z), scale=0.5)
    dG = dG.cpu().numpy()
    for s in range(B):
        ah = mpnn.scaled(a.with_values(V[s]))
        rpL, colL, _ = orc.lower_pattern(ah)
        lo, go = orc.probe_loss(ah, rpL, colL, G[s].astype(np.float64), Z[s])
        assert abs(loss[s] - 0.5 * lo) <= 1e-12 * abs(lo)
        assert rel(dG[s], 0.5 * go) <= 1e-6


def test_fsai_pcg_parity(orc):
    """FSAI-PCG with G = G^ D^{-1/2} built on the GPU from a classical FSAI
    factor of the scaled matrix, vs the oracle's FSAI-PCG with the same
    float32 factor values."""
    m = 24
    a, V = _systems(m, 1, seed=3)
    a = a.with_values(V[0])
    b = np.random.default_rng(8).standard_normal(a.n)
    ah = mpnn.scaled(a)
    rpL, colL, gh = orc.fsai(ah)
    gh32 = gh.astype(np.float32)
    pat = pattern(a)
    G, GT = _lib.fsai_factors(pat, t64(a.val), torch.as_tensor(gh32).to(dev()))
    d = a.val[a.rows() == a.col]
    Gref = (gh32.astype(np.float64) / np.sqrt(d[colL])).astype(np.float32)
    assert np.array_equal(G.cpu().numpy(), Gref)
    opts = _lib.make_opts(method="cg", precond="fsai", rtol=1e-12, G=G, GT=GT)
    x, infos, st = _lib.solve(pat, t64(a.val), t64(b), opts)
    ref = orc.fsai_pcg(a, rpL, colL, Gref.astype(np.float64), b, rtol=1e-12)
    assert st == 0 and ref.status == 0
    assert rel(x.cpu().numpy(), ref.x) <= 1e-8
    assert abs(infos[0]["iters"] - ref.iters) <= max(2, int(0.02 * ref.iters))
    jac = orc.cg(a, b, precond="jacobi", rtol=1e-12)
    assert ref.iters < jac.iters


def test_adam_step():
    n = 1000
    r = np.random.default_rng(0)
    p, g = r.standard_normal(n).astype(np.float32), r.standard_normal(n).astype(np.float32)
    m, v = (0.1 * r.standard_normal(n)).astype(np.float32), np.abs(r.standard_normal(n)).astype(np.float32)
    tp, tg, tm, tv = (torch.as_tensor(x.copy()).to(dev()) for x in (p, g, m, v))
    _lib.adam_step(tp, tg, tm, tv, 1e-3, 5)
    m2 = 0.9 * m + 0.1 * g
    v2 = 0.999 * v + 0.001 * g * g
    p2 = p - 1e-3 * (m2 / (1 - 0.9 ** 5)) / (np.sqrt(v2 / (1 - 0.999 ** 5)) + 1e-8)
    assert np.allclose(tp.cpu().numpy(), p2, rtol=1e-5, atol=1e-7)
    assert np.allclose(tm.cpu().numpy(), m2, rtol=1e-5, atol=1e-7)


def test_training_reduces_probe_loss_and_iterations(orc):
    m = 16
    pat_a, slots = W.aniso_pattern(m)
    pat = pattern(pat_a)
    st_all = torch.as_tensor(np.stack([W.aniso_stencil(*W.aniso_params(s)) for s in range(256)])).to(dev())
    sl = torch.as_tensor(slots).to(dev())
    gen = np.random.default_rng(0)
    model = learned.LearnedFSAI(seed=0)

    def sample(step):
        idx = torch.as_tensor(gen.integers(0, 256, 4)).to(dev())
        return learned.aniso_batch_values(sl, st_all[idx])

    hist = model.train(pat, sample, steps=400, probes=4, lr=3e-3, lr_final=3e-4)
    assert np.mean(hist[-20:]) < 0.8 * np.mean(hist[:5])
    its_l, its_j = [], []
    for s in range(4):
        ratio, ang = W.aniso_params(s, heldout=True)
        a = pat_a.with_values(W.aniso_stencil(ratio, ang)[slots])
        b = np.random.default_rng(s).standard_normal(a.n)
        x, infos, st = model.solve(pat, t64(a.val), t64(b), rtol=1e-8)
        assert st == 0 and infos[0]["true_residual"] <= 1.5e-8
        its_l.append(infos[0]["iters"])
        its_j.append(orc.cg(a, b, precond="jacobi", rtol=1e-8).iters)
    assert sum(its_l) < sum(its_j)


def _forged_batch(orc, m=24, B=4):
    """B systems on one 9-point pattern with classical-FSAI factors G^ of
    their scaled matrices (float32), as the learned path would hold them."""
    a, V = _systems(m, B, seed=3)
    bs = np.stack([np.random.default_rng(40 + s).standard_normal(a.n) for s in range(B)])
    gh = []
    for s in range(B):
        rpL, colL, g = orc.fsai(mpnn.scaled(a.with_values(V[s])))
        gh.append(g.astype(np.float32))
    return a, V, bs, rpL, colL, np.stack(gh)


def test_learned_fallback_on_forged_factors(orc):
    """System 1 gets a NaN in G^, system 2 a zero diagonal entry, system 3 a
    valid but useless diagonal factor (half its rows scaled by 1e-8: ||r||
    stalls); each must come back FELL_BACK with x equal to the oracle's
    Jacobi-PCG, after an FSAI attempt that stopped early (BREAKDOWN before the
    first iteration for the invalid factors, STAGNATED at the stall window for
    the useless one); system 0 keeps its factor and matches the oracle's
    FSAI-PCG with the same float32 factor."""
    a, V, bs, rpL, colL, gh = _forged_batch(orc)
    lrow = np.repeat(np.arange(a.n), np.diff(rpL))
    diagL = colL == lrow
    gh[1][17] = np.nan
    gh[2][np.nonzero(diagL)[0][5]] = 0.0
    r = np.random.default_rng(1)
    gh[3] = np.where(diagL, np.where(r.random(len(colL)) < 0.5, 1e-8, 1.0), 0.0).astype(np.float32)
    pat = pattern(a)
    Vt, bt = t64(V), t64(bs)
    G, GT = _lib.fsai_factors(pat, Vt, torch.as_tensor(gh).to(dev()))
    model = learned.LearnedFSAI(seed=0)
    window = model.default_stall_window(a.n)
    x, infos, st = model.solve(pat, Vt, bt, rtol=1e-12, factors=(G, GT))
    assert st == _lib.FELL_BACK
    x = x.cpu().numpy().reshape(4, -1)
    assert infos[0]["status"] == _lib.OK
    ref = orc.fsai_pcg(a.with_values(V[0]), rpL, colL, G[0].cpu().numpy().astype(np.float64), bs[0], rtol=1e-12)
    assert rel(x[0], ref.x) <= 1e-8
    for s, why, its in ((1, _lib.BREAKDOWN, 0), (2, _lib.BREAKDOWN, 0), (3, _lib.STAGNATED, window)):
        f = infos[s]
        assert f["status"] == _lib.FELL_BACK and f["fsai_status"] == why and f["fsai_iters"] == its, (s, f)
        jac = orc.cg(a.with_values(V[s]), bs[s], precond="jacobi", rtol=1e-12)
        assert rel(x[s], jac.x) <= 1e-8
        assert iters_close(f["iters"], jac.iters)


def test_learned_fallback_single_system_and_budget(orc):
    """A single system (values of one dimension) takes the same path; with
    the stall test off, the Jacobi-calibrated cap (twice Jacobi's iterations)
    ends the useless factor's attempt instead."""
    a, V, bs, rpL, colL, gh = _forged_batch(orc, B=1)
    lrow = np.repeat(np.arange(a.n), np.diff(rpL))
    r = np.random.default_rng(1)
    gh[0] = np.where(colL == lrow, np.where(r.random(len(colL)) < 0.5, 1e-8, 1.0), 0.0).astype(np.float32)
    pat = pattern(a)
    v1, b1 = t64(V[0]), t64(bs[0])
    G, GT = _lib.fsai_factors(pat, v1, torch.as_tensor(gh[0]).to(dev()))
    model = learned.LearnedFSAI(seed=0)
    jac_its = model.calibrate(pat, t64(V), t64(bs), rtol=1e-12)
    jac = orc.cg(a.with_values(V[0]), bs[0], precond="jacobi", rtol=1e-12)
    assert iters_close(jac_its, jac.iters)
    x, infos, st = model.solve(pat, v1, b1, rtol=1e-12, factors=(G, GT), stall_window=0)
    f = infos[0]
    assert st == _lib.FELL_BACK and f["fsai_status"] == _lib.NOT_CONVERGED and f["fsai_iters"] == 2 * jac_its
    assert rel(x.cpu().numpy(), jac.x) <= 1e-8
