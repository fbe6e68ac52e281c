"""Textbook lattice Boltzmann definitions used to pin the oracle.

These are written from the general lattice Boltzmann literature, not from the
oracle: the second-order polynomial equilibrium and the raw central moments
k_mnp = sum_i f_i (c_ix - u_x)^m (c_iy - u_y)^n (c_iz - u_z)^p.  A test that
finds the oracle equal to one of these has checked the oracle against an
independent definition.
"""
import numpy as np


def feq_second_order(rho, u, c, w):
    """f^eq_i = w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u)."""
    u = np.asarray(u, dtype=np.float64)
    cu = c @ u
    return w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * (u @ u))


def monomial_exponents():
    """All (m, n, p) with m, n, p in {0, 1, 2}."""
    return [(m, n, p) for m in range(3) for n in range(3) for p in range(3)]


def monomial_matrix(c, u):
    """V[i, q] = (c_i - u)^(m_q, n_q, p_q) for the 27 exponent triples."""
    cb = c - np.asarray(u, dtype=np.float64)[None, :]
    cols = [cb[:, 0] ** m * cb[:, 1] ** n * cb[:, 2] ** p for (m, n, p) in monomial_exponents()]
    return np.stack(cols, axis=1)


def raw_central_moments(f, c, u):
    return monomial_matrix(c, u).T @ f
