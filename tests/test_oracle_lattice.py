"""Pins of the oracle's lattice tables: velocities, weights, the central-moment
basis M(u) and the equilibrium moments m^eq (appendix)."""
import itertools

import numpy as np
import pytest

import oracle
from lbm_textbook import feq_second_order, monomial_matrix, monomial_exponents

RNG = np.random.default_rng(1807)


def test_velocity_set_is_the_full_d3q27_cube():
    c = oracle.velocities()
    assert c.shape == (27, 3)
    assert set(map(tuple, c)) == set(itertools.product((-1, 0, 1), repeat=3))
    # rest first, then the six axis directions in +x, -x, +y, -y, +z, -z order
    assert [tuple(v) for v in c[:7]] == [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0),
                                         (0, -1, 0), (0, 0, 1), (0, 0, -1)]


def test_velocity_entries_11_to_14_after_erratum():
    # the printed c_z entry 13 repeats velocity 11; read as -1 it gives (1,0,-1)
    c = oracle.velocities()
    assert [tuple(v) for v in c[11:15]] == [(1, 0, 1), (-1, 0, 1), (1, 0, -1), (-1, 0, -1)]


def test_weight_isotropy():
    c = oracle.velocities().astype(float)
    w = oracle.weights()
    assert np.all(w > 0)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    for a in range(3):
        assert (w * c[:, a]).sum() == pytest.approx(0.0, abs=1e-15)
        for b in range(3):
            expect = 1.0 / 3.0 if a == b else 0.0
            assert (w * c[:, a] * c[:, b]).sum() == pytest.approx(expect, abs=1e-15)
            for d in range(3):
                assert (w * c[:, a] * c[:, b] * c[:, d]).sum() == pytest.approx(0.0, abs=1e-15)
    # fourth order: sum w c_a^4 = 3 cs^4 = 1/3, sum w c_a^2 c_b^2 = cs^4 = 1/9
    assert (w * c[:, 0] ** 4).sum() == pytest.approx(1.0 / 3.0, abs=1e-15)
    assert (w * c[:, 0] ** 2 * c[:, 1] ** 2).sum() == pytest.approx(1.0 / 9.0, abs=1e-15)
    assert (w * c[:, 0] ** 2 * c[:, 1] * c[:, 2]).sum() == pytest.approx(0.0, abs=1e-15)


# order of each basis column, from the appendix grouping of the relaxation
# rates: m0 | m1..3 | m4..9 | m10..16 | m17..22 | m23..25 | m26
COLUMN_ORDER = [0] + [1] * 3 + [2] * 6 + [3] * 7 + [4] * 6 + [5] * 3 + [6]


@pytest.mark.parametrize("u", [(0.0, 0.0, 0.0), (0.1, -0.07, 0.03), (-0.2, 0.15, 0.11)])
def test_basis_is_a_full_rank_recombination_of_central_monomials(u):
    """Every column of M(u) is a +-1 combination of central monomials
    c~x^m c~y^n c~z^p of one total order, and M(u) has rank 27.  A dropped
    factor, a wrong exponent or a duplicated column fails here."""
    c = oracle.velocities().astype(float)
    M = oracle.basis(u)
    V = monomial_matrix(c, u)
    coef = np.linalg.solve(V, M)               # M = V @ coef
    exps = monomial_exponents()
    assert np.linalg.matrix_rank(M) == 27
    for j in range(27):
        nz = np.flatnonzero(np.abs(coef[:, j]) > 1e-9)
        assert nz.size >= 1
        assert np.allclose(np.abs(coef[nz, j]), 1.0, atol=1e-9), (j, coef[nz, j])
        orders = {sum(exps[q]) for q in nz}
        assert orders == {COLUMN_ORDER[j]}, (j, orders)


def test_basis_determinant_is_independent_of_u():
    dets = [np.linalg.det(oracle.basis(RNG.uniform(-0.3, 0.3, 3))) for _ in range(6)]
    assert np.allclose(dets, dets[0], rtol=1e-9)
    assert abs(dets[0]) > 1.0


@pytest.mark.parametrize("trial", range(8))
def test_meq_equals_central_moments_of_textbook_equilibrium(trial):
    c = oracle.velocities().astype(float)
    w = oracle.weights()
    rho = RNG.uniform(0.8, 1.2)
    u = RNG.uniform(-0.2, 0.2, 3)
    feq = feq_second_order(rho, u, c, w)
    m_def = oracle.basis(u).T @ feq
    np.testing.assert_allclose(oracle.meq(rho, u), m_def, rtol=0, atol=1e-14)


@pytest.mark.parametrize("trial", range(8))
def test_equilibrium_initialisation_is_textbook_equilibrium(trial):
    c = oracle.velocities().astype(float)
    w = oracle.weights()
    rho = RNG.uniform(0.8, 1.2)
    u = RNG.uniform(-0.15, 0.15, 3)
    np.testing.assert_allclose(oracle.equilibrium(rho, u), feq_second_order(rho, u, c, w),
                               rtol=0, atol=1e-14)
