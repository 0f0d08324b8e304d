"""Pin the FP64 hand adjoint (oracle.grad_ref) to things other than itself:
central finite differences of the oracle's forward, torch.autograd through an
independently written differentiable forward, and the n = 0 closed form."""
import numpy as np
import pytest

from oracle import grad_ref, torch_bp
from oracle import grid_bp as gb
from synth_mrf import make_stereo


def case(seed=0, H=5, W=6, M=6):
    g32, D, _, _ = make_stereo(H, W, M, 0.05, 4.0, "rectangles", seed)
    return g32.astype(np.float64), D


def test_zero_iterations_closed_form():
    """n = 0: b = softmax(theta), so dL/dtheta = (b - onehot) / N and dL/dalpha = 0."""
    g, y = case()
    L, th, al = grad_ref.grad(g, y, 6, 2, 0.7, 0)
    b = g / g.sum(-1, keepdims=True)
    onehot = np.eye(6)[y]
    np.testing.assert_allclose(th, (b - onehot) / y.size, atol=1e-15)
    assert al == 0.0


@pytest.mark.parametrize("tied", [True, False])
def test_against_autograd(tied):
    g, y = case(1, 8, 8, 8)
    fbar = None if tied else 0.2
    L, th, al = grad_ref.grad(g, y, 8, 2, 0.9, 5, fbar=fbar)
    L2, th2, al2 = torch_bp.autograd_grad(g, y, 2, 0.9, 5, fbar=fbar)
    assert L == pytest.approx(L2, rel=1e-12)
    np.testing.assert_allclose(th, th2, rtol=0, atol=1e-10 * np.abs(th2).max())
    assert al == pytest.approx(al2, rel=1e-10)


def test_against_finite_differences():
    g, y = case(2, 5, 6, 6)
    M, T, alpha, n = 6, 2, 0.8, 6
    L, th, al = grad_ref.grad(g, y, M, T, alpha, n)
    theta = np.log(g)
    eps = 1e-3
    rng = np.random.default_rng(0)
    idx = [tuple(int(rng.integers(0, s)) for s in g.shape) for _ in range(16)]
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (grad_ref.loss_of(np.exp(tp), y, M, T, alpha, n)
              - grad_ref.loss_of(np.exp(tm), y, M, T, alpha, n)) / (2 * eps)
        assert th[i] == pytest.approx(fd, rel=1e-5, abs=1e-12)
    fd_a = (grad_ref.loss_of(g, y, M, T, alpha + eps, n)
            - grad_ref.loss_of(g, y, M, T, alpha - eps, n)) / (2 * eps)
    assert al == pytest.approx(fd_a, rel=1e-5)


def test_general_belief_loss_seed():
    """With dL/db of the cross-entropy passed explicitly, the result equals the
    built-in cross-entropy seed."""
    g, y = case(3)
    pot = gb.truncated_linear(6, 2, 0.7)
    b = gb.beliefs(g, gb.run(g, pot, gb.SUM, 4, gb.SYNC, gb.DENSE))
    dL_db = np.zeros_like(b)
    r, c = np.mgrid[0:b.shape[0], 0:b.shape[1]]
    dL_db[r, c, y] = -1.0 / (y.size * b[r, c, y])
    _, th1, al1 = grad_ref.grad(g, y, 6, 2, 0.7, 4)
    _, th2, al2 = grad_ref.grad(g, None, 6, 2, 0.7, 4, dL_db=dL_db)
    np.testing.assert_allclose(th2, th1, atol=1e-15)
    assert al2 == pytest.approx(al1, rel=1e-12)


def test_torch_forward_matches_grid_oracle():
    """The independent torch forward reproduces the grid oracle's beliefs."""
    import torch
    g, _ = case(4, 6, 7, 7)
    pot = gb.truncated_linear(7, 2, 0.6)
    b = gb.beliefs(g, gb.run(g, pot, gb.SUM, 7))
    bt = torch_bp.forward(torch.log(torch.as_tensor(g)), torch.tensor(0.6, dtype=torch.float64),
                          2, 7).numpy()
    np.testing.assert_allclose(bt, b, rtol=1e-12)
