"""torch.autograd binding: differentiable rate-matrix builders (CPU) and the
chain to model parameters through the library's adjoint (GPU)."""
import numpy as np
import pytest
import torch

from oracle import epoch_oracle as O
from paper_1309_3075_amd import workloads as W
from paper_1309_3075_amd import autograd as A


def test_torch_builders_match_generator():
    rng = np.random.default_rng(0)
    pi = rng.dirichlet(np.ones(4))
    t = lambda x: torch.tensor(x, dtype=torch.float64)
    np.testing.assert_allclose(A.hky_q(t(2.5), t(pi)).numpy(), W.hky(2.5, pi), atol=1e-15)
    ex = rng.dirichlet(np.ones(6))
    np.testing.assert_allclose(A.gtr_q(t(ex), t(pi)).numpy(), W.gtr(ex, pi), atol=1e-15)
    pc = W.f3x4_frequencies(np.stack([rng.dirichlet(np.ones(4) * 10) for _ in range(3)]))
    np.testing.assert_allclose(A.gy94_q(t(3.0), t(0.4), t(pc)).numpy(), W.gy94(3.0, 0.4, pc), atol=1e-15)


def test_torch_builder_gradient_flows():
    pi = torch.full((4,), 0.25, dtype=torch.float64)
    kappa = torch.tensor(2.0, dtype=torch.float64, requires_grad=True)
    Q = A.hky_q(kappa, pi)
    Q.sum().backward()  # rows sum to zero for every kappa: d/dkappa of the total is 0
    assert abs(float(kappa.grad)) < 1e-12


@pytest.mark.gpu
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("fp32", 1e-3)])
def test_autograd_omega_and_branch_lengths(precision, tol):
    prob = W.make_config(3, n_tips=14, n_patterns=80)
    pos = np.stack([np.random.default_rng(1).dirichlet(np.ones(4) * 10) for _ in range(3)])
    pic = W.f3x4_frequencies(pos)
    omegas0 = np.array([0.2, 1.0, 2.5, 0.5])
    kappa0 = 3.0
    prob.Q = [W.gy94(kappa0, w, pic) for w in omegas0]
    prob.pi_process = [pic] * 4
    prob.pi_root = pic
    model = A.EpochModel(prob, precision=precision, reversible_pi=[pic] * 4)
    omega = torch.tensor(omegas0, dtype=torch.float64, requires_grad=True)
    kappa = torch.tensor(kappa0, dtype=torch.float64, requires_grad=True)
    ell = model.branch_lengths().requires_grad_(True)
    pit = torch.tensor(pic, dtype=torch.float64)
    Qs = [A.gy94_q(kappa, omega[s], pit) for s in range(4)]
    logL = A.EpochLogLikelihood.apply(model, ell, *Qs)
    logL.backward()
    assert abs(float(logL) - O.log_likelihood(prob)) / abs(O.log_likelihood(prob)) < (1e-12 if precision == "fp64" else 1e-5)

    def oracle_logL(om, ka):
        p = W.Problem(**{**prob.__dict__})
        p.Q = [W.gy94(ka, w, pic) for w in om]
        return O.log_likelihood(p)

    h = 1e-5
    fd = []
    for s in range(4):
        up, dn = omegas0.copy(), omegas0.copy()
        up[s] += h * omegas0[s]
        dn[s] -= h * omegas0[s]
        fd.append((oracle_logL(up, kappa0) - oracle_logL(dn, kappa0)) / (2 * h * omegas0[s]))
    fd = np.array(fd)
    g = omega.grad.numpy()
    assert np.linalg.norm(g - fd) / np.linalg.norm(fd) < tol, (g, fd)
    fdk = (oracle_logL(omegas0, kappa0 * (1 + h)) - oracle_logL(omegas0, kappa0 * (1 - h))) / (2 * h * kappa0)
    assert abs(float(kappa.grad) - fdk) / abs(fdk) < tol
    ref_b, _ = O.gradient(prob, wrt=("branch",))
    gb = ell.grad.numpy()
    assert np.linalg.norm(gb - ref_b) / np.linalg.norm(ref_b) < tol
    model.close()


@pytest.mark.gpu
def test_autograd_two_forwards_then_backwards():
    """Two forwards on one model before either backward (current and proposed state): each
    backward returns the gradient of its own forward."""
    prob = W.make_config(1, n_tips=10, n_patterns=120)
    model = A.EpochModel(prob, precision="fp64")
    Qs = [torch.tensor(Q, dtype=torch.float64) for Q in prob.Q]
    ell1 = model.branch_lengths().requires_grad_(True)
    ell2 = (model.branch_lengths() * 1.5).requires_grad_(True)
    l1 = A.EpochLogLikelihood.apply(model, ell1, *Qs)
    l2 = A.EpochLogLikelihood.apply(model, ell2, *Qs)
    l1.backward()
    l2.backward()
    p2 = W.Problem(**{**prob.__dict__})
    p2.branch_rate = prob.branch_rate * 1.5
    for lv, ell, p in ((l1, ell1, prob), (l2, ell2, p2)):
        assert abs(float(lv) - O.log_likelihood(p)) <= 1e-12 * abs(O.log_likelihood(p))
        ref_b, _ = O.gradient(p, wrt=("branch",))
        np.testing.assert_allclose(ell.grad.numpy(), ref_b, rtol=1e-6, atol=1e-9 * np.abs(ref_b).max())
    model.close()
