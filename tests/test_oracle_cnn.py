"""Pins for the FP64 U-Net oracle of the learned direction.

Checks against facts fixed independently of the oracle: a delta kernel is
the identity; conv3_dgrad / conv3_wgrad are the adjoints of conv3 in x and w
(inner-product identities); pooling and upsampling are adjoint up to the
factor 8; the whole-network gradient matches central finite differences;
a brute-force scalar-loop convolution agrees; bfloat16 rounding matches
numpy's float32 -> truncation rules on known values.
"""
import numpy as np
import pytest

from oracle import cnn


def test_round_bf16_known_values():
    vals = np.array([1.0, 1.00390625, 1.0078125, 1.005859375, -3.0, 0.0])
    out = cnn.round_bf16(vals)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7 -> even (1.0); 1.005859375 rounds up
    assert list(out) == [1.0, 1.0, 1.0078125, 1.0078125, -3.0, 0.0]


def test_delta_kernel_is_identity():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((6, 6, 6, 3))
    w = np.zeros((27, 3, 3))
    w[13] = np.eye(3)          # centre tap (0, 0, 0)
    np.testing.assert_array_equal(cnn.conv3(x, w), x)
    w2 = np.zeros((27, 3, 3))
    t = cnn.TAPS.index((0, 0, 1))
    w2[t] = np.eye(3)          # y[v] = x[v + e_x]
    y = cnn.conv3(x, w2)
    np.testing.assert_array_equal(y[:, :, :-1], x[:, :, 1:])
    assert np.all(y[:, :, -1] == 0)


def test_conv_brute_force():
    rng = np.random.default_rng(1)
    S, ci, co = 4, 2, 3
    x = rng.standard_normal((S, S, S, ci))
    w = rng.standard_normal((27, co, ci))
    y = cnn.conv3(x, w)
    for (z, yy, xx) in [(0, 0, 0), (1, 2, 3), (3, 3, 3), (2, 0, 1)]:
        for o in range(co):
            s = 0.0
            for t, (dz, dy, dx) in enumerate(cnn.TAPS):
                a, b, c = z + dz, yy + dy, xx + dx
                if 0 <= a < S and 0 <= b < S and 0 <= c < S:
                    s += sum(w[t, o, i] * x[a, b, c, i] for i in range(ci))
            assert abs(y[z, yy, xx, o] - s) < 1e-12


def test_conv_adjoints():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((5, 5, 5, 4))
    w = rng.standard_normal((27, 3, 4))
    dy = rng.standard_normal((5, 5, 5, 3))
    lhs = np.sum(cnn.conv3(x, w) * dy)
    assert lhs == pytest.approx(np.sum(x * cnn.conv3_dgrad(dy, w)), rel=1e-12)
    assert lhs == pytest.approx(np.sum(w * cnn.conv3_wgrad(dy, x)), rel=1e-12)


def test_pool_upsample_adjoint():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((8, 8, 8, 2))
    y = rng.standard_normal((4, 4, 4, 2))
    assert np.sum(cnn.avgpool2(x) * y) == pytest.approx(np.sum(x * cnn.avgpool2_bwd(y)), rel=1e-12)
    assert np.sum(cnn.upsample2(y) * x) == pytest.approx(np.sum(y * cnn.upsample2_bwd(x)), rel=1e-12)
    assert np.allclose(cnn.avgpool2(np.ones((4, 4, 4, 1))), 1.0)


def test_network_gradient_finite_differences():
    rng = np.random.default_rng(4)
    S = 8
    W = cnn.init_weights(5)
    x0 = np.zeros((S, S, S, 16))
    x0[..., :2] = rng.standard_normal((S, S, S, 2))
    target = rng.standard_normal((S, S, S))
    mask = np.ones((S, S, S))
    out, c = cnn.forward(W, x0, store=False)
    L0, dout = cnn.mse_loss(out, target, mask)
    g = cnn.backward(W, c, dout, store=False)
    for name, idx in [("w1", (13, 3, 0)), ("w4", (2, 5, 7)), ("w6", (26, 63, 1)), ("w7", (0, 1, 95)),
                      ("w9", (14, 0, 40)), ("w11", (0, 3))]:
        eps = 1e-5
        Wp = {k: v.copy() for k, v in W.items()}
        Wm = {k: v.copy() for k, v in W.items()}
        Wp[name][idx] += eps
        Wm[name][idx] -= eps
        Lp = cnn.mse_loss(cnn.forward(Wp, x0, store=False)[0], target, mask)[0]
        Lm = cnn.mse_loss(cnn.forward(Wm, x0, store=False)[0], target, mask)[0]
        fd = (Lp - Lm) / (2 * eps)
        assert g[name][idx] == pytest.approx(fd, rel=1e-6, abs=1e-9), name


def test_pack_input_normalises():
    n, S = 7, 8
    r = np.arange(n ** 3, dtype=float) - 100
    x = cnn.pack_input(r, None, n, S)
    assert np.sqrt(np.mean(x[:n, :n, :n, 0] ** 2)) == pytest.approx(1.0)
    assert np.all(x[n:, :, :, 0] == 0) and np.all(x[..., 1:] == 0)


def _spd(n, seed):
    """A small SPD matrix (1D Laplacian plus a random diagonal)."""
    rng = np.random.default_rng(seed)
    A = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    return A + np.diag(rng.uniform(0.1, 1.0, n))


def test_energy_loss_closed_forms():
    n = 30
    A = _spd(n, 1)
    rng = np.random.default_rng(2)
    e = rng.standard_normal(n)
    r = A @ e
    # the exact error as direction leaves nothing; any multiple too
    L, g = cnn.energy_loss(e, r, e, A @ e)
    assert L == pytest.approx(0.0, abs=1e-14)
    assert np.linalg.norm(g) <= 1e-12 * np.linalg.norm(r)
    L2, _ = cnn.energy_loss(-3.5 * e, r, e, A @ (-3.5 * e))
    assert L2 == pytest.approx(0.0, abs=1e-14)
    # an A-orthogonal direction removes nothing
    d = rng.standard_normal(n)
    d -= (d @ A @ e) / (e @ A @ e) * e
    L3, _ = cnn.energy_loss(d, r, e, A @ d)
    assert L3 == pytest.approx(1.0, abs=1e-12)
    # the definition: min over c of ||e - c d||_A^2 / ||e||_A^2
    d = rng.standard_normal(n)
    cs = np.linspace(-5, 5, 200001)
    best = min(((e - c * d) @ A @ (e - c * d)) for c in cs) / (e @ A @ e)
    L4, g4 = cnn.energy_loss(d, r, e, A @ d)
    assert L4 == pytest.approx(best, rel=1e-6)
    # scale invariance: the gradient is orthogonal to d
    assert abs(g4 @ d) <= 1e-12 * np.linalg.norm(g4) * np.linalg.norm(d)


def test_energy_loss_gradient_finite_differences():
    n = 25
    A = _spd(n, 3)
    rng = np.random.default_rng(4)
    e = rng.standard_normal(n)
    r = A @ e
    d = rng.standard_normal(n)
    _, g = cnn.energy_loss(d, r, e, A @ d)
    for i in (0, 7, 24):
        h = 1e-6
        dp, dm = d.copy(), d.copy()
        dp[i] += h
        dm[i] -= h
        fd = (cnn.energy_loss(dp, r, e, A @ dp)[0] - cnn.energy_loss(dm, r, e, A @ dm)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_marginal_energy_loss_brute_force():
    # L = min over (c_Z, c_d) ||e - Z c_Z - c_d d||_A^2 / min over c_Z ||e - Z c_Z||_A^2,
    # both minimisations by dense A-norm least squares (Cholesky of A)
    n, m = 40, 4
    A = _spd(n, 5)
    rng = np.random.default_rng(6)
    e = rng.standard_normal(n)
    r = A @ e
    Z = rng.standard_normal((n, m))
    d = rng.standard_normal(n)
    L, g = cnn.marginal_energy_loss(d, r, e, A, Z, tau=1e-12)
    C = np.linalg.cholesky(A).T          # A = C^T C, ||v||_A = ||C v||
    def left(B):
        c, *_ = np.linalg.lstsq(C @ B, C @ e, rcond=None)
        v = e - B @ c
        return v @ A @ v
    expect = left(np.column_stack([Z, d])) / left(Z)
    assert L == pytest.approx(expect, rel=1e-9)
    # a direction inside span(Z) adds nothing: the loss is one, the gradient zero
    Lz, gz = cnn.marginal_energy_loss(Z @ rng.standard_normal(m) + 1e-300, r, e, A, Z, tau=1e-12)
    assert Lz == pytest.approx(1.0, abs=1e-6)
    # the gradient by central differences
    for i in (0, 13, 39):
        h = 1e-6
        dp, dm = d.copy(), d.copy()
        dp[i] += h
        dm[i] -= h
        fd = (cnn.marginal_energy_loss(dp, r, e, A, Z, 1e-12)[0] -
              cnn.marginal_energy_loss(dm, r, e, A, Z, 1e-12)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-10)
    # a singular block (a repeated column) gives the same loss as the unique columns
    Ls, _ = cnn.marginal_energy_loss(d, r, e, A, np.column_stack([Z, Z[:, :1]]), tau=1e-10)
    assert Ls == pytest.approx(L, rel=1e-8)
