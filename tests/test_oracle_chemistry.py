"""Pins of the oracle's per-node backward-Euler chemistry step.

Exact invariants: total mass, N and O atoms, and the internal energy the step
holds fixed.  The defining equation: its residual at the returned state.
Consistency with the source term: (rho^{n+1} - rho^n)/dt -> omega(rho^n) at
first order as dt -> 0.  The long-step limit: chemical equilibrium, where
each reaction's concentration quotient equals its K_c (so the kinetics' K_c
and the implicit solve are checked against each other), and a fixed point of
further steps.  The substep path (a growing mode): the single step's Newton
fails, the substeps keep the invariants, and the result approaches the
exact chemistry flow (a library stiff integrator at tight tolerance) at
first order.  Far-from-equilibrium states (cold gas carrying atoms, hot gas
with trace atoms) converge at every step size.
"""
import numpy as np
import pytest

from paper_2511_17551_amd import workloads as W
from oracle.thermo import Mixture
from oracle.kinetics import Kinetics
from oracle.chemistry import backward_euler, newton, residual

NN = np.array([2, 0, 1, 1, 0])  # N atoms per molecule of N2, O2, NO, N, O
NO_ = np.array([0, 2, 1, 0, 1])


@pytest.fixture(scope="module")
def setup():
    sp = W.Species()
    mix = Mixture(sp)
    kin = Kinetics(sp, W.park17_reactions(4))
    rng = np.random.default_rng(7)
    n = 16
    Y = np.array([0.767, 0.233, 0.0, 0.0, 0.0])[:, None] + rng.uniform(1e-4, 0.02, (5, n))
    Y /= Y.sum(0)
    rho = 10.0 ** rng.uniform(-3.0, -1.0, n)
    T = rng.uniform(5000.0, 9000.0, n)
    rs = Y * rho
    rhoe = mix.rho_e(rs, T)
    # chemical time scale per node: rho / max_s |omega_s|
    tau = rho / np.abs(kin.omega_dot(rs, T)).max(0)
    return sp, mix, kin, rs, rhoe, T, tau


def atoms(sp, rs):
    c = rs / sp.W[:, None]
    return (NN[:, None] * c).sum(0), (NO_[:, None] * c).sum(0)


def test_invariants_and_residual(setup):
    sp, mix, kin, rs, rhoe, T, tau = setup
    dt = 10.0 * tau.min()
    r1, T1, it, nsub = backward_euler(mix, kin, rs, rhoe, dt, T)
    one = nsub == 1          # nodes whose single step converged
    assert one.sum() >= 12
    rho = rs.sum(0)
    assert np.all(r1 >= 0.0)
    assert np.max(np.abs(r1.sum(0) - rho) / rho) < 1e-13
    n0, o0 = atoms(sp, rs)
    n1, o1 = atoms(sp, r1)
    assert np.max(np.abs(n1 - n0) / n0) < 1e-12
    assert np.max(np.abs(o1 - o0) / o0) < 1e-12
    assert np.max(np.abs(mix.rho_e(r1, T1) - rhoe) / np.abs(rhoe)) < 1e-12
    G, _ = residual(mix, kin, r1[:, one], rs[:, one], rhoe[one], dt, T1[one])
    assert np.max(np.abs(G) / rho[one]) < 1e-11
    # the step did something: the composition moved by much more than the tolerance
    assert np.max(np.abs(r1 - rs) / rho) > 1e-3
    assert it[one].max() < 50


def test_first_order_in_dt(setup):
    sp, mix, kin, rs, rhoe, T, tau = setup
    w0 = kin.omega_dot(rs, T)
    errs = []
    for dt in (1e-6 * tau.min(), 0.5e-6 * tau.min()):
        r1, _, _, _ = backward_euler(mix, kin, rs, rhoe, dt, T)
        errs.append(np.max(np.abs((r1 - rs) / dt - w0)) / np.abs(w0).max())
    assert errs[0] < 1e-4
    assert 1.8 < errs[0] / errs[1] < 2.2


def test_long_step_reaches_equilibrium(setup):
    """With every reaction fast (same stoichiometry, so the same K_c), long
    steps approach equilibrium: ln Q_r - ln K_c(T) -> 0 like 1/dt."""
    sp, mix, _, rs, rhoe, T, _ = setup
    rx = W.park17_reactions(4)
    nr = rx.nreactions
    fast = W.Reactions(A=np.full(nr, 1e3), b=np.zeros(nr), theta_a=np.zeros(nr), nu=rx.nu, nup=rx.nup)
    kin = Kinetics(sp, fast)
    tau = (rs.sum(0) / np.abs(kin.omega_dot(rs, T)).max(0)).max()
    dev = []
    for dt in (1e4 * tau, 1e6 * tau):
        req, Teq, _, _ = backward_euler(mix, kin, rs, rhoe, dt, T)
        conc = req / sp.W[:, None]
        lnQ = (rx.nup - rx.nu) @ np.log(conc)
        dev.append(np.max(np.abs(lnQ - kin.ln_Kc(Teq))))
    assert dev[1] < 1e-4
    assert 50.0 < dev[0] / dev[1] < 200.0
    # equilibrium is (nearly) a fixed point of a further step
    r2, T2, _, _ = backward_euler(mix, kin, req, rhoe, tau, Teq)
    assert np.max(np.abs(r2 - req) / req.sum(0)) < 1e-6


def hot_trace_state(mix, T0=8000.0, rho=1e-2):
    """Shock-heated air with trace NO and atoms: atom-impact dissociation
    grows the atoms at a rate k [X2] from almost nothing."""
    Y = np.array([0.767, 0.233, 1e-10, 1e-12, 1e-12])
    Y = Y / Y.sum()
    rs = (Y * rho)[:, None]
    return rs, mix.rho_e(rs, np.array([T0])), np.array([T0])


def exact_flow(mix, kin, rs, rhoe, T0, dt):
    """The chemistry flow over dt at fixed rho e from a library stiff
    integrator (Radau IIA, rtol 1e-10)."""
    from scipy.integrate import solve_ivp
    Tg = [T0[0]]

    def f(t, y):
        T, _ = mix.solve_T(y[:, None], rhoe, np.array(Tg), tol=1e-14, maxit=100)
        Tg[0] = T[0]
        return kin.omega_dot(y[:, None], T)[:, 0]

    sol = solve_ivp(f, (0.0, dt), rs[:, 0], method="Radau", rtol=1e-10, atol=1e-14 * rs.sum())
    return sol.y[:, -1]


def test_substeps_when_the_single_step_fails(setup):
    sp, mix, kin = setup[:3]
    rs, rhoe, T0 = hot_trace_state(mix)
    dt = 1e-6
    _, _, _, ok = newton(mix, kin, rs, rhoe, np.array([dt]), T0)
    assert not ok[0]
    r1, T1, it, nsub = backward_euler(mix, kin, rs, rhoe, dt, T0)
    assert nsub[0] > 1
    rho = rs.sum(0)
    assert np.all(r1 >= 0.0)
    assert abs(r1.sum(0)[0] - rho[0]) / rho[0] < 1e-13
    n0, o0 = atoms(sp, rs)
    n1, o1 = atoms(sp, r1)
    assert abs(n1[0] - n0[0]) / n0[0] < 1e-12 and abs(o1[0] - o0[0]) / o0[0] < 1e-12
    assert abs(mix.rho_e(r1, T1)[0] - rhoe[0]) / abs(rhoe[0]) < 1e-12
    ex = exact_flow(mix, kin, rs, rhoe, T0, dt)
    change = np.abs(ex - rs[:, 0]).max()
    assert change > 0.1 * rho[0]          # a large change, far from the linear regime
    assert np.abs(r1[:, 0] - ex).max() < 0.05 * change


def test_first_order_convergence_to_the_exact_flow(setup):
    """m calls over dt/m: the error against the exact flow halves as m doubles."""
    sp, mix, kin = setup[:3]
    rs, rhoe, T0 = hot_trace_state(mix)
    dt = 1e-7
    ex = exact_flow(mix, kin, rs, rhoe, T0, dt)
    change = np.abs(ex - rs[:, 0]).max()
    err = []
    for m in (4, 8):
        r, T = rs.copy(), T0.copy()
        for _ in range(m):
            r, T, _, _ = backward_euler(mix, kin, r, rhoe, dt / m, T)
        err.append(np.abs(r[:, 0] - ex).max() / change)
    assert err[1] < 0.15
    assert 1.8 < err[0] / err[1] < 2.2


def far_states(mix, n, seed=11):
    rs, T = W.far_chem_states(n, seed)
    return rs, mix.rho_e(rs, T), T


@pytest.mark.parametrize("dt", [1e-9, 1e-7, 1e-5])
def test_far_from_equilibrium_states_converge(setup, dt):
    sp, mix, kin = setup[:3]
    rs, rhoe, T = far_states(mix, 300)
    r1, T1, it, nsub = backward_euler(mix, kin, rs, rhoe, dt, T)
    rho = rs.sum(0)
    assert np.all(r1 >= 0.0)
    assert np.max(np.abs(r1.sum(0) - rho) / rho) < 1e-13
    n0, o0 = atoms(sp, rs)
    n1, o1 = atoms(sp, r1)
    assert np.max(np.abs(n1 - n0) / n0) < 1e-12 and np.max(np.abs(o1 - o0) / o0) < 1e-12
    assert np.max(np.abs(mix.rho_e(r1, T1) - rhoe) / np.abs(rhoe)) < 1e-12
    one = nsub == 1
    assert one.sum() > len(one) // 2
    # Newton stops on its step (1e-13 rho); the residual is that step times the
    # Jacobian I - dt d omega/d rho, whose row-sum norm reaches 6e5 here at the
    # longest dt (median 6e2)
    G, _ = residual(mix, kin, r1[:, one], rs[:, one], rhoe[one], dt, T1[one])
    assert np.max(np.abs(G) / rho[one]) < 1e-9
