"""GPU surrogate (BF16 MFMA MLP) against the oracle: forward pass, gradients,
training progress, and the surrogate-guided Newton solve (converged T
unchanged, fewer iterations)."""
import numpy as np
import pytest

from paper_2511_17551_amd import workloads as W
from oracle import mlp
from oracle.thermo import Mixture
from tests.helpers import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dgx():
    import torch
    assert torch.cuda.is_available()
    from paper_2511_17551_amd import dgx as mod
    return mod


def state_set(n, seed):
    """Seeded packed 2D mixture states [8][n] spanning 300-12000 K and
    frozen-to-dissociated compositions, with their exact temperatures."""
    rng = np.random.default_rng(seed)
    mix = Mixture(W.Species())
    T = np.exp(rng.uniform(np.log(300.0), np.log(12000.0), n))
    f = rng.uniform(0, 1, n) ** 3
    Y = np.stack([0.767 * (1 - f), 0.233 * (1 - f), 0.02 * f, 0.767 * f, 0.213 * f], 0)
    Y = Y * rng.uniform(0.9, 1.1, (5, n))
    Y /= Y.sum(0)
    rho = 10.0 ** rng.uniform(-3, 0, n)
    rs = Y * rho
    v = rng.uniform(-3000, 3000, (2, n))
    E = mix.rho_e(rs, T) + 0.5 * rho * (v * v).sum(0)
    u = np.concatenate([rs, rho * v, E[None]], 0)
    return u, T


@pytest.fixture(scope="module")
def solver(dgx):
    mixs = W.Species()
    c = W.case_c4(lambda rs, T: Mixture(mixs).rho_e(rs, T), lambda rs, T: Mixture(mixs).rho_cv(rs, T),
                  nr=4, nth=8)
    s = dgx.Solver(c)
    yield s
    s.close()


def test_forward_matches_oracle(dgx, solver):
    import torch
    u, T = state_set(4096, 1)
    theta = mlp.init_params(11)
    raw = mlp.raw_features(u[:5], u[7] - 0.5 * (u[5] ** 2 + u[6] ** 2) / u[:5].sum(0))
    norm = np.concatenate([raw.mean(0), raw.std(0), [T.mean(), T.std()]]).astype(np.float32)
    prm = np.concatenate([theta, norm]).astype(np.float32)
    dgx.dgx_surrogate_set(solver.ctx, prm)
    Tg = torch.empty(T.size, dtype=torch.float64, device="cuda")
    dgx.dgx_surrogate_predict(solver.ctx, to_dev(u), Tg)
    got = (to_host(Tg) - norm[12]) / norm[13]
    p = mlp.unpack(prm.astype(np.float64))
    y, _ = mlp.forward(p, mlp.standardise(raw, p))
    d = np.abs(got - y)
    print("forward |dy| median %.2e p99 %.2e max %.2e" % (np.median(d), np.quantile(d, 0.99), d.max()))
    assert np.median(d) < 1e-5
    assert np.quantile(d, 0.99) < 1e-3
    assert d.max() < 5e-2


def test_gradients_match_oracle(dgx, solver):
    u, T = state_set(2048, 2)
    ud, Td = to_dev(u), to_dev(T)
    dgx.dgx_surrogate_init(solver.ctx, ud, Td, seed=7)
    prm = dgx.dgx_surrogate_get(solver.ctx)
    g, loss = dgx.dgx_surrogate_grad(solver.ctx, ud, Td)
    p = mlp.unpack(prm.astype(np.float64))
    raw = mlp.raw_features(u[:5], u[7] - 0.5 * (u[5] ** 2 + u[6] ** 2) / u[:5].sum(0))
    x = mlp.standardise(raw, p)
    t = (T - p["Tm"]) / p["Ts"]
    lo, go = mlp.loss_and_grad(p, x, t)
    gp = mlp.unpack(np.concatenate([g.astype(np.float64), np.zeros(14)]))
    print("loss gpu %.6e oracle %.6e" % (loss, lo))
    assert abs(loss - lo) < 1e-3 * lo
    for name, _ in mlp.SIZES:
        rel = np.linalg.norm(gp[name] - go[name]) / np.linalg.norm(go[name])
        print("grad %s rel L2 %.3e" % (name, rel))
        assert rel < 5e-3, name


def test_training_and_guided_newton(dgx, solver):
    import torch
    u, T = state_set(65536, 3)
    ud, Td = to_dev(u), to_dev(T)
    dgx.dgx_surrogate_init(solver.ctx, ud, Td, seed=41)
    loss = dgx.dgx_surrogate_train(solver.ctx, ud, Td, epochs=8, batch=1024, lr=2e-3, seed=42)
    print("losses", loss)
    assert loss[-1] < 0.1 * loss[0]
    uv, Tv = state_set(16384, 4)
    uvd = to_dev(uv)
    Tp = torch.empty(Tv.size, dtype=torch.float64, device="cuda")
    Ts = torch.empty_like(Tp)
    sp = dgx.dgx_thermo(solver.ctx, uvd, Tp, nstates=Tv.size, guess=dgx.GUESS_FREESTREAM)
    ss = dgx.dgx_thermo(solver.ctx, uvd, Ts, nstates=Tv.size, guess=dgx.GUESS_SURROGATE)
    a, b = to_host(Tp), to_host(Ts)
    print("plain", sp, "surrogate", ss)
    assert np.max(np.abs(a - Tv) / Tv) < 1e-10
    assert np.max(np.abs(b - Tv) / Tv) < 1e-10
    assert ss["iters_total"] < 0.85 * sp["iters_total"]
    assert ss["iters_wave_max_mean"] < sp["iters_wave_max_mean"]
