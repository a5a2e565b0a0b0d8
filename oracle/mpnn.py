"""FP64 reference of the preconditioner network -- TEST INFRASTRUCTURE.

The paper names learned preconditioners only as future work (Sec.
"Conclusion" and the backend-registration remark in Sec. "Five backends");
the network below is this project's design, written here in plain numpy so
that the GPU kernels can be checked against it.  Only tests/, the smoke
check and the benchmark's CPU baseline use it.

Graph: the sparsity pattern of A.  Scaled values a^_k = a_k / sqrt(a_ii a_jj)
for stored entry k = (i, j).  Edge features f_k = [a^_k, [j<i], [j>i], [j=i]].

    s_i   = sum_{k in row i} f_k                                 (4)
    h0_i  = relu(s_i W0 + b0)                                    (64)
    for l = 1..3:
        m_i  = sum_{k in row i} (f_k C_l) * h^{l-1}_{col k}      (64, channel-wise gate)
        h^l_i = relu([h^{l-1}_i, m_i] W_l + b_l)                 (128 -> 64)
    for each lower entry k = (i, j), j <= i:
        x_k = [h3_i, h3_j, f_k]                                  (132)
        z_k = relu(x_k H1 + c1)                                  (32)
        t_k = z_k . H2 + c2
        g^_k = softplus(t_k) if j == i else t_k

G^ (values on A's lower pattern) then preconditions the scaled system:
M^{-1} = G^T G with G = G^ D^{-1/2}, so G A G^T = G^ A^ G^^T.

With bf16=True the forward rounds to bfloat16 (round to nearest even) at the
points where the GPU stores bfloat16: the weights (all matrices and the gate
C_l), h0..h3, m, x_k and z_k; and the backward rounds the upstream gradient
of every matrix product (dz, and dpre of each layer) before the product, as
the GPU feeds them to the matrix cores.  Accumulations are FP64 here.
"""
from __future__ import annotations

import numpy as np

HID = 64
HEAD = 32
NFEAT = 4
LAYERS = 3


def bf16(a: np.ndarray) -> np.ndarray:
    """Round float values to bfloat16 (nearest even) and return them as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out[nan] = np.nan
    return out.reshape(np.shape(a))


def init_params(seed: int = 0) -> dict:
    """He-style initialisation (float64 master values)."""
    r = np.random.default_rng(seed)

    def w(k, n):
        return r.standard_normal((k, n)) * np.sqrt(2.0 / k)

    p = {"W0": w(NFEAT, HID), "b0": np.zeros(HID)}
    for l in range(1, LAYERS + 1):
        p[f"C{l}"] = r.standard_normal((NFEAT, HID)) * 0.5
        p[f"W{l}"] = w(2 * HID, HID)
        p[f"b{l}"] = np.zeros(HID)
    p["H1"] = w(2 * HID + NFEAT, HEAD)
    p["c1"] = np.zeros(HEAD)
    p["H2"] = r.standard_normal(HEAD) * np.sqrt(1.0 / HEAD)
    p["c2"] = np.zeros(1)
    return p


MATS = ["W0"] + [f"{k}{l}" for l in range(1, LAYERS + 1) for k in ("C", "W")] + ["H1", "H2"]


def _q(p: dict, bf: bool) -> dict:
    return {k: (bf16(v) if (bf and k in MATS) else v) for k, v in p.items()}


def graph(a):
    """Rows, columns, scaled values and edge features of A's entries, and the
    lower-entry index list (positions in A of entries with col <= row)."""
    rows = a.rows()
    col = a.col.astype(np.int64)
    d = np.asarray(a.val)[rows == col]
    assert len(d) == a.n and np.all(d > 0), "needs a positive stored diagonal"
    dsq = np.sqrt(d)
    ah = np.asarray(a.val) / (dsq[rows] * dsq[col])
    f = np.stack([ah, (col < rows).astype(float), (col > rows).astype(float), (col == rows).astype(float)], axis=1)
    lower = np.nonzero(col <= rows)[0]
    return rows, col, ah, f, lower


def _rowsum(rows, vals, n):
    out = np.zeros((n,) + vals.shape[1:])
    np.add.at(out, rows, vals)
    return out


def forward(p: dict, a, bf: bool = False):
    """Returns (g^ on the lower entries in pattern order, cache)."""
    q = _qp = _q(p, bf)
    rnd = bf16 if bf else (lambda v: v)
    rows, col, ah, f, lower = graph(a)
    if bf:
        f = f.astype(np.float32).astype(np.float64)  # features are float32 on the GPU
    n = a.n
    s = _rowsum(rows, f, n)
    h = rnd(np.maximum(s @ q["W0"] + q["b0"], 0.0))
    hs, ms, gates = [h], [], []
    for l in range(1, LAYERS + 1):
        gate = f @ q[f"C{l}"]
        m = rnd(_rowsum(rows, gate * h[col], n))
        h = rnd(np.maximum(np.concatenate([h, m], axis=1) @ q[f"W{l}"] + q[f"b{l}"], 0.0))
        gates.append(gate)
        ms.append(m)
        hs.append(h)
    li, lj = rows[lower], col[lower]
    x = rnd(np.concatenate([h[li], h[lj], f[lower]], axis=1))
    z = rnd(np.maximum(x @ q["H1"] + q["c1"], 0.0))
    t = z @ q["H2"] + q["c2"][0]
    diag = lj == li
    g = np.where(diag, np.logaddexp(0.0, t), t)
    cache = dict(q=q, rows=rows, col=col, f=f, lower=lower, s=s, hs=hs, ms=ms, gates=gates, x=x, z=z, t=t,
                 diag=diag, n=n, bf=bf)
    return g, cache


def backward(c: dict, dg: np.ndarray) -> dict:
    """Gradients of sum(dg * g^) with respect to every parameter."""
    q, bf, n = c["q"], c["bf"], c["n"]
    rnd = bf16 if bf else (lambda v: v)
    rows, col, f, lower = c["rows"], c["col"], c["f"], c["lower"]
    grads = {}
    dt = np.where(c["diag"], dg / (1.0 + np.exp(-c["t"])), dg)
    grads["H2"] = c["z"].T @ dt
    grads["c2"] = np.array([dt.sum()])
    dz = rnd(np.outer(dt, q["H2"]) * (c["z"] > 0))
    grads["H1"] = c["x"].T @ dz
    grads["c1"] = dz.sum(axis=0)
    dx = dz @ q["H1"].T
    li, lj = rows[lower], col[lower]
    dh = _rowsum(li, dx[:, :HID], n) + _rowsum(lj, dx[:, HID:2 * HID], n)
    for l in range(LAYERS, 0, -1):
        h_prev, m, h = c["hs"][l - 1], c["ms"][l - 1], c["hs"][l]
        dpre = rnd(dh * (h > 0))
        grads[f"W{l}"] = np.concatenate([h_prev, m], axis=1).T @ dpre
        grads[f"b{l}"] = dpre.sum(axis=0)
        dhm = dpre @ q[f"W{l}"].T
        dh_prev, dm = dhm[:, :HID], dhm[:, HID:]
        gate = c["gates"][l - 1]
        dm_e = dm[rows]
        dh_prev = dh_prev + _rowsum(col, gate * dm_e, n)
        grads[f"C{l}"] = f.T @ (dm_e * h_prev[col])
        dh = dh_prev
    dpre0 = rnd(dh * (c["hs"][0] > 0))
    grads["W0"] = c["s"].T @ dpre0
    grads["b0"] = dpre0.sum(axis=0)
    return grads


def lower_values_to_csr(a, g):
    """(rpL, colL, values) of G^ on A's lower pattern."""
    rows = a.rows()
    keep = a.col <= rows
    counts = np.bincount(rows[keep], minlength=a.n)
    rpL = np.zeros(a.n + 1, np.int32)
    np.cumsum(counts, out=rpL[1:])
    return rpL, a.col[keep].astype(np.int32), np.asarray(g, dtype=np.float64)


def scaled(a):
    """A^ = D^{-1/2} A D^{-1/2} as a Csr with the same pattern."""
    _, _, ah, _, _ = graph(a)
    return a.with_values(ah)
