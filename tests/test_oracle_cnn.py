"""Pins of the CPU reference of the learned warm start (oracle/cnn.py).

The network is not in the paper; its reference is pinned by a library correlation, the adjoint
identity, central finite differences of the FP64 loss, a library bfloat16 conversion and closed forms."""
import numpy as np
import pytest
import torch
from scipy.signal import correlate2d

from oracle import cnn
from paper_2107_05337_amd import workloads as W


def test_conv_matches_library_correlation():
    rng = np.random.default_rng(1)
    a = rng.standard_normal((2, 3, 9, 9))
    Wt = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    z = cnn.conv3x3(a, Wt, b)
    for n in range(2):
        for co in range(4):
            ref = b[co] + sum(correlate2d(a[n, ci], Wt[co, ci], mode="same", boundary="fill") for ci in range(3))
            assert np.allclose(z[n, co], ref, rtol=0, atol=1e-12)


def test_transpose_and_wgrad_are_adjoints():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((2, 5, 8, 8))
    g = rng.standard_normal((2, 6, 8, 8))
    Wt = rng.standard_normal((6, 5, 3, 3))
    lhs = np.sum(cnn.conv3x3(a, Wt) * g)
    assert np.isclose(lhs, np.sum(a * cnn.conv3x3_transpose(g, Wt)), rtol=1e-12)
    assert np.isclose(lhs, np.sum(Wt * cnn.conv3x3_wgrad(a, g)), rtol=1e-12)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    theta = W.net_init(7) + 0.05 * rng.standard_normal(cnn.nparams())  # non-zero biases too
    x = rng.standard_normal((2, 3, 7, 7))
    t = rng.standard_normal((2, 7, 7))
    _, g = cnn.loss_and_grad(theta, x, t)
    idx = np.concatenate([rng.choice(cnn.nparams(), 40, replace=False),
                          np.cumsum([0] + [cnn.CH[l + 1] * cnn.CH[l] * 9 + cnn.CH[l + 1] for l in range(4)])[1:] - 1])
    h = 1e-5
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (cnn.loss_and_grad(tp, x, t)[0] - cnn.loss_and_grad(tm, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), 1e-3), (i, fd, g[i])


def test_bf16_rounding_matches_library_conversion():
    rng = np.random.default_rng(4)
    v = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000),
                        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -1.0 - 2.0 ** -8, 0.0, -0.0]])
    ref = torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16(v), ref)
    assert cnn.bf16([1.0 + 2.0 ** -8])[0] == 1.0  # tie to even


def test_zero_last_layer_returns_previous_step():
    rng = np.random.default_rng(5)
    theta = W.net_init(3, zero_last=True)
    n, p = 6, 3
    nin = n + p - 2
    u = rng.standard_normal(nin * nin)
    F = rng.standard_normal(nin * nin)
    mlp = 0.5 + rng.random(nin * nin)
    K = np.eye(nin * nin)
    x, s, _ = cnn.pack(u, F, mlp, K, 1e-3, 1e-3, n, p)
    y, _ = cnn.forward(theta, x[None])
    assert np.array_equal(cnn.unpack(y[0], u, s), u)


def test_pack_closed_form():
    n, p, dt, kappa, c = 4, 2, 0.01, 2.0, -3.0
    nin = n + p - 2
    u = np.full(nin * nin, c)
    mlp = np.linspace(1.0, 2.0, nin * nin)
    # K = diag(2 mlp): the explicit increment (dt F - kappa dt K u) / m = dt (5 - 2 kappa c) everywhere
    K = np.diag(2.0 * mlp)
    F = 5.0 * mlp
    e = dt * (5.0 - 2.0 * kappa * c)
    x, s, t = cnn.pack(u, F, mlp, K, dt, kappa * dt, n, p, u_next=u + 1.0)
    assert np.isclose(s, abs(e))
    assert np.allclose(x[0, 1:-1, 1:-1], -1.0) and np.all(x[0, 0] == 0) and np.all(x[0, :, -1] == 0)
    assert np.allclose(x[1, 1:-1, 1:-1], np.sign(e))
    assert np.allclose(x[2], np.log(kappa * dt * n * n) / 4)
    assert np.allclose(t[1:-1, 1:-1], 1.0 / s) and np.all(t[0] == 0)
    x0, s0, _ = cnn.pack(np.zeros(nin * nin), np.zeros(nin * nin), mlp, K, dt, kappa * dt, n, p)
    assert s0 == 1.0 and np.all(x0[:2] == 0)


def test_pack_increment_is_a_residual_of_the_step():
    """The explicit-increment plane times the lumped mass and its scale is the residual b - A u_k of the step
    (M + kappa dt K) u_{k+1} = M u_k + w F at the previous point, with the oracle's own matrices."""
    import oracle as O
    P = O.Problem(3, 6, 1)
    rng = np.random.default_rng(8)
    u = rng.standard_normal(P.ndof)
    F = P.load_vector([(1, 2, 0.5)])
    mlp = P.lumped()[0]
    M, K = P.dense("M"), P.dense("K")
    kdt, w = 0.03, 0.01
    x, s, _ = cnn.pack(u, F, mlp, K, w, kdt, 6, 3)
    r = (M @ u + w * F) - (M + kdt * K) @ u
    nin = P.Nin
    assert np.allclose(x[1, 1:-1, 1:-1].ravel() * s * mlp, r, rtol=1e-12, atol=1e-14)


def test_adam_first_step_is_signed_lr():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    th, m, v = cnn.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(th[:3], -0.01 * np.sign(g[:3]), rtol=1e-4) and th[3] == 0.0


def test_rounded_mode_stays_close_to_fp64():
    rng = np.random.default_rng(6)
    theta = W.net_init(11)
    x = rng.standard_normal((2, 3, 10, 10))
    y64, _ = cnn.forward(theta, x)
    y16, _ = cnn.forward(theta, x, round_bf16=True)
    assert np.linalg.norm(y16 - y64) <= 3e-2 * np.linalg.norm(y64)
