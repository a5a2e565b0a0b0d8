"""The inverse coefficient problem on the GPU (Sec. "End-to-End: Inverse
Coefficient Learning"): assembly, loss and dL/dtheta through the
library's adjoint against the oracle at the paper's size (64 x 64), and the
paper's full Adam run against its reported outcome."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from gpu_common import dev, rel  # noqa: E402
from paper_2601_13994_amd import inverse  # noqa: E402
from oracle import inverse as OI  # noqa: E402


def test_assembly_matches_oracle():
    m = 64
    kt, _ = W.inverse_truth(m)
    op = inverse.VarCoefPoisson2D(m, dev())
    a = OI.assemble(kt, m)
    assert np.array_equal(op.row_ptr.cpu().numpy(), a.row_ptr) and np.array_equal(op.col.cpu().numpy(), a.col)
    v = op.values(torch.as_tensor(kt, device=dev())).cpu().numpy()
    assert rel(v, a.val) <= 1e-15


@pytest.mark.parametrize("case", ["start", "random", "near"])
def test_loss_and_gradient_match_oracle(orc, case):
    """L and dL/dtheta at three parameter fields: the start (kappa = 1), a
    random field, and kappa* perturbed; both sides solve to rtol 1e-12."""
    m = 64
    kt, f = W.inverse_truth(m)
    prob = inverse.InverseProblem(kt, f, m=m, device=dev(), rtol=1e-12)
    r = np.random.default_rng({"start": 0, "random": 1, "near": 2}[case])
    if case == "start":
        theta = np.full(m * m, np.log(np.e - 1.0))
    elif case == "random":
        theta = np.log(np.e - 1.0) + 0.3 * r.standard_normal(m * m)
    else:
        theta = np.log(np.expm1(kt)) + 0.01 * r.standard_normal(m * m)
    th = torch.tensor(theta, device=dev(), requires_grad=True)
    loss, _ = prob.loss(th)
    loss.backward()
    u_obs = OI.observe(m, kt, f, rtol=1e-12)
    lo, go, _ = OI.loss_and_grad(theta, m, u_obs, f, rtol=1e-12)
    assert abs(float(loss.detach()) - lo) <= 1e-8 * lo
    assert rel(th.grad.cpu().numpy(), go) <= 1e-6, rel(th.grad.cpu().numpy(), go)


def test_full_run_recovers_kappa():
    """The paper's run: 1500 Adam steps (lr 5e-2, here CG to rtol 1e-10)
    recover kappa to the paper's reported accuracy (relative error 2.3e-3,
    solution misfit 3.0e-5, range [0.503, 1.495]), with margin."""
    m = 64
    kt, f = W.inverse_truth(m)
    prob = inverse.InverseProblem(kt, f, m=m, device=dev(), rtol=1e-10)
    hist = [prob.step() for _ in range(1500)]
    ek, eu, kmin, kmax = prob.errors()
    print("[inverse]", hist[0], hist[-1], ek, eu, kmin, kmax, flush=True)
    assert hist[-1] < 1e-4 * hist[0]
    assert ek <= 3e-3 and eu <= 5e-5
    assert 0.49 <= kmin <= 0.52 and 1.48 <= kmax <= 1.51
