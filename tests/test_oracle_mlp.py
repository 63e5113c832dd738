"""Pins of the oracle MLP: backward pass against central finite differences
of the FP64 network, BF16 rounding against its definition, Adam against a
hand-computed first step."""
import numpy as np

from oracle import mlp


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9, -3.140625, 1e-30, 0.0])
    r = mlp.bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                            # 1+2^-8 is a tie -> even (1.0)
    assert r[2] == 1.0                            # below half an ulp
    assert r[3] == 1.0 + 2 ** -7                  # above half an ulp -> up
    assert r[4] == -3.140625                      # exactly representable
    assert r[6] == 0.0


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    theta = mlp.init_params(5).astype(np.float64)
    theta[:mlp.NPARAM] += 0.05 * rng.normal(size=mlp.NPARAM)
    p = mlp.unpack(np.concatenate([theta, np.zeros(14)]))
    x = rng.normal(size=(40, 6))
    t = rng.normal(size=40)
    _, g = mlp.loss_and_grad_exact(p, x, t)
    for name in ("W1", "b1", "W2", "b3", "W4", "b4"):
        flat = p[name].reshape(-1)
        idx = rng.choice(flat.size, size=min(6, flat.size), replace=False)
        for i in idx:
            h = 1e-6
            old = flat[i]
            flat[i] = old + h
            lp, _ = mlp.loss_and_grad_exact(p, x, t)
            flat[i] = old - h
            lm, _ = mlp.loss_and_grad_exact(p, x, t)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, i, fd, an)


def test_rounded_backward_close_to_exact():
    rng = np.random.default_rng(4)
    p = mlp.unpack(np.concatenate([mlp.init_params(6), np.zeros(14)]))
    x = rng.normal(size=(256, 6))
    t = rng.normal(size=256)
    _, ge = mlp.loss_and_grad_exact(p, x, t)
    _, gr = mlp.loss_and_grad(p, x, t)
    for name in ge:
        rel = np.linalg.norm(gr[name] - ge[name]) / np.linalg.norm(ge[name])
        assert rel < 0.05, (name, rel)


def test_adam_first_step():
    theta = np.array([1.0, -2.0])
    g = np.array([0.5, -0.25])
    th, m, v = mlp.adam_step(theta, g, np.zeros(2), np.zeros(2), 1, 0.01)
    # bias-corrected first step moves each weight by lr * sign(g) (up to eps)
    assert np.allclose(th, theta - 0.01 * np.sign(g), rtol=1e-7)
