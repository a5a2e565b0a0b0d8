"""Pins of the FP64 preconditioner-network reference (no GPU)."""
import numpy as np
import pytest

import workloads as W
from oracle import mpnn


def _sys(m=5, ratio=30.0, angle=0.7):
    return W.aniso2d(m, ratio, angle)


def test_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(0).standard_normal(20000) * np.logspace(-30, 30, 20000)
    x[:3] = [0.0, -0.0, 1.0]
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mpnn.bf16(x), ref)


def test_closed_form_head_only():
    """All matrices zero: every off-diagonal value is c2, every diagonal softplus(c2)."""
    a = _sys()
    p = {k: np.zeros_like(v) for k, v in mpnn.init_params(0).items()}
    p["c2"] = np.array([0.3])
    g, _ = mpnn.forward(p, a)
    rows, col, _, _, lower = mpnn.graph(a)
    diag = col[lower] == rows[lower]
    assert np.allclose(g[diag], np.log1p(np.exp(0.3)), rtol=1e-15)
    assert np.all(g[~diag] == 0.3)


def test_graph_scaling_unit_diagonal():
    a = _sys()
    rows, col, ah, f, lower = mpnn.graph(a)
    assert np.allclose(ah[rows == col], 1.0)
    d = a.to_dense()
    dd = np.sqrt(np.diag(d))
    assert np.allclose(mpnn.scaled(a).to_dense(), d / np.outer(dd, dd), rtol=1e-14)
    assert len(lower) == int(np.sum(a.col <= rows))


@pytest.mark.parametrize("name", mpnn.MATS + ["b0", "b1", "b3", "c1", "c2"])
def test_backward_vs_finite_differences(name):
    a = _sys(m=4)
    p = mpnn.init_params(3)
    for k in p:
        if k.startswith(("b", "c")):
            p[k] = np.random.default_rng(7).standard_normal(p[k].shape) * 0.1
    g, cache = mpnn.forward(p, a)
    dg = np.random.default_rng(1).standard_normal(g.shape)
    grads = mpnn.backward(cache, dg)
    r = np.random.default_rng(2)
    flat = p[name].reshape(-1)
    for idx in r.choice(flat.size, min(6, flat.size), replace=False):
        h = 1e-6
        old = flat[idx]
        flat[idx] = old + h
        gp, _ = mpnn.forward(p, a)
        flat[idx] = old - h
        gm, _ = mpnn.forward(p, a)
        flat[idx] = old
        fd = (dg @ gp - dg @ gm) / (2 * h)
        an = grads[name].reshape(-1)[idx]
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, idx, fd, an)


def test_bf16_forward_close_to_fp64():
    a = _sys(m=6)
    p = mpnn.init_params(1)
    g64, _ = mpnn.forward(p, a, bf=False)
    g16, _ = mpnn.forward(p, a, bf=True)
    assert np.linalg.norm(g16 - g64) <= 0.05 * np.linalg.norm(g64)


# ---------------------------------------------------------------------------
# Hand-worked forward on a 3-node graph.  The expected values below were
# worked out by hand from the network's definition (features, node sums,
# gated aggregation over the row's columns, head over [h_i, h_j, f_k]); every
# intermediate is a short binary fraction, so FP64 and the bf16 mode are both
# exact.  A = [[4, -1, 0], [-1, 1, -1], [0, -1, 16]]: sqrt(diag) = 2, 1, 4, so
# a^(0,1) = a^(1,0) = -1/2, a^(1,2) = a^(2,1) = -1/4 and the diagonal is 1.
# Edge features [a^, j<i, j>i, j=i]:
#   row 0: (0,0) [1,0,0,1]   (0,1) [-1/2,0,1,0]
#   row 1: (1,0) [-1/2,1,0,0] (1,1) [1,0,0,1] (1,2) [-1/4,0,1,0]
#   row 2: (2,1) [-1/4,1,0,0] (2,2) [1,0,0,1]
# Node sums s_i: s0 = [1/2,0,1,1], s1 = [1/4,1,1,1], s2 = [3/4,1,0,1].
# W0 copies features 0, 1, 2 into channels 0, 1, 2, so
#   h0[:,0] = [1/2, 1/4, 3/4], h0[:,1] = [0, 1, 1], h0[:,2] = [1, 1, 0].
# Lower entries in pattern order: (0,0), (1,0), (1,1), (2,1), (2,2).
# ---------------------------------------------------------------------------
def _three_node():
    d = np.array([[4.0, -1.0, 0.0], [-1.0, 1.0, -1.0], [0.0, -1.0, 16.0]])
    return W.from_dense(d, keep=d != 0)


def _zero_params():
    p = {k: np.zeros_like(v) for k, v in mpnn.init_params(0).items()}
    p["W0"][0, 0] = p["W0"][1, 1] = p["W0"][2, 2] = 1.0
    for l in range(1, mpnn.LAYERS + 1):
        p[f"W{l}"][np.arange(mpnn.HID), np.arange(mpnn.HID)] = 1.0  # h passes through
    return p


def _softplus(t):
    return float(np.log1p(np.exp(t)))


@pytest.mark.parametrize("bf", [False, True])
def test_hand_worked_node_features_and_head(bf):
    """No aggregation (C_l = 0, layers pass h through).  Head channels:
    z0 = h_i[0], z1 = h_j[1] (x position 64 + 1), z2 = relu(-a^_k) (x position
    128); t = z0 + 2 z1 + 4 z2.
      (0,0): 1/2 + 0 + 0       = 1/2   -> softplus(1/2)
      (1,0): 1/4 + 0 + 4(1/2)  = 9/4
      (1,1): 1/4 + 2(1) + 0    = 9/4   -> softplus(9/4)
      (2,1): 3/4 + 2(1) + 4(1/4) = 15/4
      (2,2): 3/4 + 2(1) + 0    = 11/4  -> softplus(11/4)
    A swapped head order [h_j, h_i] gives 9/2 at (1,0); node sums taken over
    columns instead of rows give h0[:,1] = [1, 1, 0] and 17/4 at (1,0)."""
    a = _three_node()
    p = _zero_params()
    p["H1"][0, 0] = 1.0
    p["H1"][mpnn.HID + 1, 1] = 1.0
    p["H1"][2 * mpnn.HID + 0, 2] = -1.0
    p["H2"][:3] = [1.0, 2.0, 4.0]
    g, _ = mpnn.forward(p, a, bf=bf)
    want = [_softplus(0.5), 2.25, _softplus(2.25), 3.75, _softplus(2.75)]
    np.testing.assert_allclose(g, want, rtol=1e-15, atol=0)


@pytest.mark.parametrize("bf", [False, True])
@pytest.mark.parametrize("layer", [1, 2, 3])
def test_hand_worked_aggregation(layer, bf):
    """Only layer `layer` aggregates: gate channel 0 = [j<i] (C row 1),
    gate channel 1 = a^ (C row 0), so with h = h0 at its input
      m[:,0] = sum over lower neighbours j of h_j[0] = [0, 1/2, 1/4]
      m[:,1] = sum_k a^_k h_col(k)[1]:
        m0 = 1(0) - 1/2(1) = -1/2, m1 = -1/2(0) + 1(1) - 1/4(1) = 3/4,
        m2 = -1/4(1) + 1(1) = 3/4.
    W_l routes m into new channels: h[:,3] = relu(m[:,0]) = [0, 1/2, 1/4],
    h[:,4] = relu(m[:,1]) = [0, 3/4, 3/4], h[:,5] = relu(-m[:,1]) = [1/2, 0, 0].
    Head: z0 = h_i[3], z1 = h_j[4], z2 = h_i[5], t = z0 + 2 z1 + 4 z2:
      (0,0): 0 + 0 + 4(1/2) = 2 -> softplus(2)
      (1,0): 1/2 + 0 + 0    = 1/2
      (1,1): 1/2 + 3/2      = 2 -> softplus(2)
      (2,1): 1/4 + 3/2      = 7/4
      (2,2): 1/4 + 3/2      = 7/4 -> softplus(7/4)
    Gathering h at the row instead of the column gives m[:,0] = [0, 1/4, 3/4]
    and 1/4 at (1,0); the gate of the mirrored entry gives m1[0] = 0."""
    a = _three_node()
    p = _zero_params()
    C = p[f"C{layer}"]
    C[1, 0] = 1.0
    C[0, 1] = 1.0
    Wl = p[f"W{layer}"]
    Wl[mpnn.HID + 0, 3] = 1.0
    Wl[mpnn.HID + 1, 4] = 1.0
    Wl[mpnn.HID + 1, 5] = -1.0
    p["H1"][3, 0] = 1.0
    p["H1"][mpnn.HID + 4, 1] = 1.0
    p["H1"][5, 2] = 1.0
    p["H2"][:3] = [1.0, 2.0, 4.0]
    g, cache = mpnn.forward(p, a, bf=bf)
    np.testing.assert_array_equal(cache["ms"][layer - 1][:, :2], [[0.0, -0.5], [0.5, 0.75], [0.25, 0.75]])
    want = [_softplus(2.0), 0.5, _softplus(2.0), 1.75, _softplus(1.75)]
    np.testing.assert_allclose(g, want, rtol=1e-15, atol=0)


@pytest.mark.parametrize("bf", [False, True])
def test_hand_worked_biases(bf):
    """Biases: b0[6] = 1/8 makes h0[:,6] = 1/8 on every node; b_2[7] = -1/4
    with W_2[6, 7] = 4 makes h2[:,7] = relu(4/8 - 1/4) = 1/4; c1[0] = 1/2
    with H1[7, 0] = 2 gives z0 = 1/2 + 1/2 = 1, and c2 = -3/2 gives t = -1/2
    on every lower entry (softplus(-1/2) on the diagonal)."""
    a = _three_node()
    p = _zero_params()
    p["b0"][6] = 0.125
    p["W2"][6, 7] = 4.0
    p["b2"][7] = -0.25
    p["c1"][0] = 0.5
    p["H1"][7, 0] = 2.0
    p["H2"][0] = 1.0
    p["c2"][0] = -1.5
    g, _ = mpnn.forward(p, a, bf=bf)
    want = [_softplus(-0.5), -0.5, _softplus(-0.5), -0.5, _softplus(-0.5)]
    np.testing.assert_allclose(g, want, rtol=1e-15, atol=0)
