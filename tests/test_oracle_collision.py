"""Pins of the oracle's one-cell central-moment collision (eq. cmr_collision,
appendix relaxation rates, adaptive relaxation section)."""
import numpy as np
import pytest

import oracle
from lbm_textbook import feq_second_order, monomial_matrix, monomial_exponents

RNG = np.random.default_rng(2284)
C = oracle.velocities().astype(float)
W = oracle.weights()


def random_state(rng, amp=0.05, umax=0.1):
    rho = rng.uniform(0.9, 1.1)
    u = rng.uniform(-umax, umax, 3)
    f = feq_second_order(rho, u, C, W) * (1.0 + amp * rng.uniform(-1, 1, 27))
    return f


def params(**kw):
    base = dict(nu=0.02, g_max=0.1, adaptive=True)
    base.update(kw)
    return oracle.Params(**base)


@pytest.mark.parametrize("adaptive", [False, True])
@pytest.mark.parametrize("trial", range(5))
def test_collision_conserves_mass_and_momentum(adaptive, trial):
    f = random_state(RNG)
    out, _ = oracle.collide(f, params(adaptive=adaptive))
    assert out.sum() == pytest.approx(f.sum(), rel=1e-14)
    np.testing.assert_allclose(C.T @ out, C.T @ f, rtol=0, atol=1e-15)


@pytest.mark.parametrize("trial", range(5))
def test_equilibrium_is_a_fixed_point(trial):
    rho, u = RNG.uniform(0.9, 1.1), RNG.uniform(-0.1, 0.1, 3)
    feq = feq_second_order(rho, u, C, W)
    out, d = oracle.collide(feq, params())
    np.testing.assert_allclose(out, feq, rtol=0, atol=1e-15)
    assert d["G"] == pytest.approx(0.0, abs=1e-12)
    assert d["phi"] == pytest.approx(5.0, abs=1e-9)


@pytest.mark.parametrize("omega", [0.6, 1.0, 1.7, 1.99])
def test_uniform_rates_reduce_to_bgk(omega):
    """S_i = omega for all i gives f~ = f - omega (f - f^eq) with the textbook
    second-order equilibrium (T m^eq = f^eq)."""
    f = random_state(RNG, amp=0.1)
    rho = f.sum()
    u = C.T @ f / rho
    out, _ = oracle.collide(f, params(), S_override=np.full(27, omega))
    bgk = f - omega * (f - feq_second_order(rho, u, C, W))
    np.testing.assert_allclose(out, bgk, rtol=0, atol=1e-14)


def test_unit_rates_give_equilibrium():
    f = random_state(RNG, amp=0.2)
    rho = f.sum()
    u = C.T @ f / rho
    out, _ = oracle.collide(f, params(), S_override=np.ones(27))
    np.testing.assert_allclose(out, feq_second_order(rho, u, C, W), rtol=0, atol=1e-14)


def group_relaxation_reference(f, nu, phi, nu_hi):
    """Relax raw central moments by order: second-order off-diagonal and the
    deviatoric diagonal with S, the diagonal trace with the m9 rate, order
    3/4/5/6 with the m10..16 / m17..22 / m23..25 / m26 rates."""
    rho = f.sum()
    u = C.T @ f / rho
    V = monomial_matrix(C, u)
    k = V.T @ f
    keq = V.T @ feq_second_order(rho, u, C, W)
    S = 1.0 / (3.0 * nu + 0.5)
    Sg = [1.0 / (3.0 * phi * v + 0.5) for v in nu_hi]
    exps = monomial_exponents()
    idx = {e: q for q, e in enumerate(exps)}
    kstar = k.copy()
    for q, e in enumerate(exps):
        order = sum(e)
        if order in (0, 1):
            continue
        if order == 2 and 2 in e:
            continue                                  # diagonal handled below
        rate = S if order == 2 else Sg[order - 3]
        kstar[q] = k[q] - rate * (k[q] - keq[q])
    diag = [idx[(2, 0, 0)], idx[(0, 2, 0)], idx[(0, 0, 2)]]
    n = k[diag] - keq[diag]
    tr = n.sum() / 3.0
    kstar[diag] = keq[diag] + (1.0 - S) * (n - tr) + (1.0 - Sg[0]) * tr
    return np.linalg.solve(V.T, kstar)


@pytest.mark.parametrize("adaptive", [False, True])
@pytest.mark.parametrize("trial", range(4))
def test_basis_relaxation_equals_per_order_central_moment_relaxation(adaptive, trial):
    f = random_state(RNG, amp=0.02)
    p = params(adaptive=adaptive, nu=0.01, g_max=0.05)
    out, d = oracle.collide(f, p)
    ref = group_relaxation_reference(f, p.nu, d["phi"], p.nu_hi)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-14)


def chapman_enskog_state(rho, u, Pi):
    """f = f^eq + w_i/(2 cs^4) Q_i : Pi (eq. epsilon_f1), cs^2 = 1/3."""
    cs2 = 1.0 / 3.0
    f = feq_second_order(rho, u, C, W)
    Q = np.einsum("ia,ib->iab", C, C) - cs2 * np.eye(3)[None]
    return f + W / (2.0 * cs2 * cs2) * np.einsum("iab,ab->i", Q, Pi)


def test_adaptive_gradient_follows_chapman_enskog_relation():
    """With f = f^eq + eps f(1) built from a traceless stress Pi, the oracle's
    |grad u| estimate equals sqrt(2 S^:S^) with S^ = -S Pi / (2 cs^2 rho)
    (eq. pi_1)."""
    rho, u = 1.03, np.array([0.04, -0.02, 0.01])
    A = RNG.normal(size=(3, 3))
    Pi = 1e-3 * (A + A.T)
    Pi -= np.trace(Pi) / 3.0 * np.eye(3)
    p = params(nu=0.01, g_max=1.0)
    f = chapman_enskog_state(rho, u, Pi)
    _, d = oracle.collide(f, p)
    S = 1.0 / (3.0 * p.nu + 0.5)
    Shat = -S * Pi / (2.0 / 3.0 * rho)
    G = np.sqrt(2.0 * np.sum(Shat * Shat))
    assert d["G"] == pytest.approx(G, rel=1e-6)


def test_adaptive_factor_is_linear_then_clamped():
    rho, u = 1.0, np.zeros(3)
    Pi = np.array([[0, 1, 0], [1, 0, 0], [0, 0, 0]], dtype=float)
    p = params(nu=0.01, g_max=0.1)
    gs, phis = [], []
    for eps in (1e-4, 5e-4, 1e-3, 2e-3, 5e-2):
        _, d = oracle.collide(chapman_enskog_state(rho, u, eps * Pi), p)
        gs.append(d["G"])
        phis.append(d["phi"])
    for G, phi in zip(gs, phis):
        x = min(G / p.g_max, 1.0)
        assert phi == pytest.approx(-4.0 * x + 5.0, abs=1e-12)
    assert gs[-1] > p.g_max and phis[-1] == pytest.approx(1.0)
    assert gs[0] < p.g_max and 1.0 < phis[0] < 5.0


def load_golden_rates():
    rows = []
    with open(__file__.replace("test_oracle_collision.py", "golden/relaxation_rates.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                _, nu, s5, s1 = line.split()
                rows.append((float(nu), float(s5), float(s1)))
    return rows


def test_relaxation_rates_match_appendix_table():
    """At equilibrium (|grad u| = 0, phi = 5) and beyond g_max (phi = 1) the
    high-order relaxation works out to the tabulated rates.  The rates are
    recovered from the collision itself: for a perturbation of one high-order
    raw central moment, the post-collision perturbation is (1 - S) times it."""
    golden = load_golden_rates()
    rho, u = 1.0, np.zeros(3)
    exps = monomial_exponents()
    probes = {0: (1, 2, 0), 1: (2, 2, 0), 2: (1, 2, 2), 3: (2, 2, 2)}
    for phi_col, strain in ((1, 0.0), (2, 1.0)):
        for grp, e in probes.items():
            V = monomial_matrix(C, u)
            e_k = np.zeros(27)
            e_k[exps.index(e)] = 1e-6
            Pi = strain * np.array([[0, 1, 0], [1, 0, 0], [0, 0, 0]], dtype=float)
            base = chapman_enskog_state(rho, u, Pi)
            f = base + np.linalg.solve(V.T, e_k)
            p = params(nu=0.01, g_max=0.1)
            out, d = oracle.collide(f, p)
            outb, _ = oracle.collide(base, p)
            dk = V.T @ (out - outb)
            ratio = dk[exps.index(e)] / 1e-6
            assert 1.0 - ratio == pytest.approx(golden[grp][phi_col], rel=1e-6), (grp, phi_col)


def test_force_adds_exactly_F_to_momentum():
    f = random_state(RNG)
    F = np.array([1e-4, -2e-4, 3e-5])
    out, d = oracle.collide(f, params(), F=F)
    assert out.sum() == pytest.approx(f.sum(), rel=1e-14)
    np.testing.assert_allclose(C.T @ out, C.T @ f + F, rtol=0, atol=1e-15)
    np.testing.assert_allclose([d["ux"], d["uy"], d["uz"]], (C.T @ f + F / 2) / f.sum(),
                               rtol=0, atol=1e-15)
