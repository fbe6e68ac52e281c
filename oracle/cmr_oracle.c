/*
 * cmr_oracle.c -- plain FP64 CPU reference of the central-moment lattice
 * Boltzmann method of Li, Bai & Liu (arXiv 1807.02284).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline leg of the benchmark.  Nothing here is shared with the GPU
 * library.  Every step follows the paper's definition literally: the
 * 27x27 central-moment matrix M(u) is built explicitly, m = M^T f, and the
 * back-transform T = (M^T)^{-1} is applied by an LU solve.  No blocking,
 * fusion or reordering.
 *
 * Readings of passages the paper leaves open (each is pinned by a test
 * unless marked "parity unpinned"):
 *   - velocity list: entry 13 of c_z is read as -1 (the printed +1 repeats
 *     velocity 11 and leaves (1,0,-1) out);
 *   - basis: M_{i,20} is read as cx^2 cy cz (the printed cx^2 cy cz^2 repeats
 *     M_{i,24} and makes M singular);
 *   - weights: the product weights (2/3, 1/6, 1/6) per axis;
 *   - |grad u| of the adaptive relaxation: the local strain-rate magnitude
 *     G = sqrt(2 S^:S^) obtained from the non-equilibrium stress through the
 *     Chapman-Enskog relation Pi = -2 cs^2 rho S^ / S (section "Mapping
 *     distribution functions"); the factor is clamped, phi = a*min(G/g_max,1)+b;
 *   - body force: velocity shifted by F/2 and source (I - S/2) R with
 *     R = (0, F, 0, ...) in moment space;
 *   - boundaries: halfway bounce-back, Dirichlet equilibrium inlet,
 *     zero-gradient outflow copied from the x-1 neighbour, and the
 *     regularized no-slip wall node on flat axis-aligned walls;
 *   - passive scalar: D3Q7 BGK with g^eq_i = w_i s (1 + 4 c_i.u).
 */
#include "cmr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------
 * Lattice: appendix, D3Q27 velocity list (c_x, c_y, c_z), in the paper's
 * order.  Entry 13 of c_z reads -1 (see header comment).
 * ------------------------------------------------------------------- */
static const int CX[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1,
                           0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
static const int CY[27] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1,
                           -1, 1, -1, 1, 1, -1, -1, 1, 1, -1, -1};
static const int CZ[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1,
                           1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1};

/* D3Q7 scalar lattice: rest, then +x, -x, +y, -y, +z, -z. */
static const int SX[7] = {0, 1, -1, 0, 0, 0, 0};
static const int SY[7] = {0, 0, 0, 1, -1, 0, 0};
static const int SZ[7] = {0, 0, 0, 0, 0, 1, -1};
static const double SW[7] = {0.25, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125};

/* Lattice weight w_i (used in the Chapman-Enskog expansion of the section
 * "Mapping distribution functions"; not listed there): product of the
 * one-dimensional weights 2/3 for c = 0 and 1/6 for c = +-1. */
static double weight(int i)
{
    double w = 1.0;
    const int c[3] = {CX[i], CY[i], CZ[i]};
    for (int a = 0; a < 3; ++a) w *= (c[a] == 0) ? 2.0 / 3.0 : 1.0 / 6.0;
    return w;
}

static int opposite(int i)
{
    for (int k = 0; k < 27; ++k)
        if (CX[k] == -CX[i] && CY[k] == -CY[i] && CZ[k] == -CZ[i]) return k;
    return -1;
}

void oracle_velocities(int32_t c[81])
{
    for (int i = 0; i < 27; ++i) {
        c[3 * i + 0] = CX[i];
        c[3 * i + 1] = CY[i];
        c[3 * i + 2] = CZ[i];
    }
}

void oracle_weights(double w[27])
{
    for (int i = 0; i < 27; ++i) w[i] = weight(i);
}

/* ---------------------------------------------------------------------
 * Appendix: M_{i,j} = the j-th basis polynomial evaluated at the shifted
 * velocity (X, Y, Z) = c_i - u, in the order of the appendix list (with
 * M_{i,20} = X^2 Y Z, see header comment).
 * ------------------------------------------------------------------- */
static void basis_row(double X, double Y, double Z, double r[27])
{
    const double X2 = X * X, Y2 = Y * Y, Z2 = Z * Z;
    r[0] = 1.0;
    r[1] = X;
    r[2] = Y;
    r[3] = Z;
    r[4] = X * Y;
    r[5] = X * Z;
    r[6] = Y * Z;
    r[7] = X2 - Y2;
    r[8] = X2 - Z2;
    r[9] = X2 + Y2 + Z2;
    r[10] = X * Y2 + X * Z2;
    r[11] = X2 * Y + Y * Z2;
    r[12] = X2 * Z + Y2 * Z;
    r[13] = X * Y2 - X * Z2;
    r[14] = X2 * Y - Y * Z2;
    r[15] = X2 * Z - Y2 * Z;
    r[16] = X * Y * Z;
    r[17] = X2 * Y2 + X2 * Z2 + Y2 * Z2;
    r[18] = X2 * Y2 + X2 * Z2 - Y2 * Z2;
    r[19] = X2 * Y2 - X2 * Z2;
    r[20] = X2 * Y * Z;
    r[21] = X * Y2 * Z;
    r[22] = X * Y * Z2;
    r[23] = X * Y2 * Z2;
    r[24] = X2 * Y * Z2;
    r[25] = X2 * Y2 * Z;
    r[26] = X2 * Y2 * Z2;
}

void oracle_basis(const double u[3], double M[729])
{
    for (int i = 0; i < 27; ++i)
        basis_row(CX[i] - u[0], CY[i] - u[1], CZ[i] - u[2], &M[i * 27]);
}

/* Appendix: the 27 equilibrium central moments m^eq(rho, u). */
void oracle_meq(double rho, const double u[3], double m[27])
{
    const double x = u[0], y = u[1], z = u[2];
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    for (int j = 0; j < 27; ++j) m[j] = 0.0;
    m[0] = rho;
    m[9] = rho;
    m[10] = -rho * x * (y2 + z2);
    m[11] = -rho * y * (x2 + z2);
    m[12] = -rho * z * (x2 + y2);
    m[13] = -rho * x * (y2 - z2);
    m[14] = -rho * y * (x2 - z2);
    m[15] = -rho * z * (x2 - y2);
    m[16] = -rho * x * y * z;
    m[17] = rho / 3.0 * (9.0 * x2 * y2 + 9.0 * x2 * z2 + 9.0 * y2 * z2 + 1.0);
    m[18] = rho / 9.0 * (27.0 * x2 * y2 + 27.0 * x2 * z2 - 27.0 * y2 * z2 + 1.0);
    m[19] = 3.0 * rho * x2 * (y2 - z2);
    m[20] = 3.0 * rho * x2 * y * z;
    m[21] = 3.0 * rho * x * y2 * z;
    m[22] = 3.0 * rho * x * y * z2;
    m[23] = -rho / 3.0 * x * (18.0 * y2 * z2 + y2 + z2);
    m[24] = -rho / 3.0 * y * (18.0 * x2 * z2 + x2 + z2);
    m[25] = -rho / 3.0 * z * (18.0 * x2 * y2 + x2 + y2);
    m[26] = rho * (10.0 * x2 * y2 * z2 + x2 * y2 + x2 * z2 + y2 * z2 + 1.0 / 27.0);
}

/* Solve A x = b for a dense 27x27 matrix by Gaussian elimination with
 * partial pivoting.  A and b are overwritten.  Returns 0 or -1. */
static int solve27(double A[729], double b[27], double x[27])
{
    for (int k = 0; k < 27; ++k) {
        int piv = k;
        double best = fabs(A[k * 27 + k]);
        for (int r = k + 1; r < 27; ++r) {
            const double v = fabs(A[r * 27 + k]);
            if (v > best) {
                best = v;
                piv = r;
            }
        }
        if (best == 0.0) return -1;
        if (piv != k) {
            for (int c = 0; c < 27; ++c) {
                const double t = A[k * 27 + c];
                A[k * 27 + c] = A[piv * 27 + c];
                A[piv * 27 + c] = t;
            }
            const double t = b[k];
            b[k] = b[piv];
            b[piv] = t;
        }
        for (int r = k + 1; r < 27; ++r) {
            const double l = A[r * 27 + k] / A[k * 27 + k];
            if (l == 0.0) continue;
            for (int c = k; c < 27; ++c) A[r * 27 + c] -= l * A[k * 27 + c];
            b[r] -= l * b[k];
        }
    }
    for (int k = 26; k >= 0; --k) {
        double s = b[k];
        for (int c = k + 1; c < 27; ++c) s -= A[k * 27 + c] * x[c];
        x[k] = s / A[k * 27 + k];
    }
    return 0;
}

/* Solve M(u)^T x = r, i.e. x = T r with T = (M^T)^{-1}. */
static int apply_T(const double u[3], const double r[27], double x[27])
{
    double M[729], A[729], b[27];
    oracle_basis(u, M);
    for (int i = 0; i < 27; ++i)
        for (int j = 0; j < 27; ++j) A[j * 27 + i] = M[i * 27 + j];
    memcpy(b, r, sizeof b);
    return solve27(A, b, x);
}

/* Initialisation section: f_0 = T m^eq(rho, u). */
int oracle_equilibrium(double rho, const double u[3], double f[27])
{
    double meq[27];
    oracle_meq(rho, u, meq);
    return apply_T(u, meq, f);
}

/* D3Q7 scalar equilibrium (passive smoke scalar; not in the paper). */
static void scalar_eq(double s, const double u[3], double geq[7])
{
    for (int i = 0; i < 7; ++i)
        geq[i] = SW[i] * s * (1.0 + 4.0 * (SX[i] * u[0] + SY[i] * u[1] + SZ[i] * u[2]));
}

/* ---------------------------------------------------------------------
 * Collision: Omega = -T S (m - m^eq) (section "Non-orthogonal
 * central-moment relaxation model", eq. cmr_collision, and appendix), with
 *   S_0..3 = 0, S_4..8 = (3 nu + 1/2)^{-1}, S_i = (3 nu^_i' + 1/2)^{-1}
 *   for i > 8 (appendix), nu^_i' = phi nu_i' (section "Adaptive
 *   relaxation"), plus the body-force source (I - S/2) R.
 * ------------------------------------------------------------------- */
static int collide_impl(const double f[27], const double F[3], const oracle_params* p,
                        const double* S_override, double G_given, double out[27], double diag[6]);

int oracle_collide(const double f[27], const double F[3], const oracle_params* p,
                   const double* S_override, double out[27], double diag[6])
{
    return collide_impl(f, F, p, S_override, -1.0, out, diag);
}

int oracle_collide_g(const double f[27], const double F[3], const oracle_params* p, double G,
                     double out[27], double diag[6])
{
    return collide_impl(f, F, p, NULL, G, out, diag);
}

static int collide_impl(const double f[27], const double F[3], const oracle_params* p,
                        const double* S_override, double G_given, double out[27], double diag[6])
{
    const double Fz[3] = {0.0, 0.0, 0.0};
    if (!F) F = Fz;

    /* Macroscopic fields (eq. lbe context): rho = sum f, u = (sum c f + F/2)/rho. */
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 27; ++i) {
        rho += f[i];
        j[0] += CX[i] * f[i];
        j[1] += CY[i] * f[i];
        j[2] += CZ[i] * f[i];
    }
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * F[a]) / rho;

    /* m = M^T f and m^eq (appendix). */
    double M[729], m[27], meq[27];
    oracle_basis(u, M);
    for (int k = 0; k < 27; ++k) {
        double s = 0.0;
        for (int i = 0; i < 27; ++i) s += M[i * 27 + k] * f[i];
        m[k] = s;
    }
    oracle_meq(rho, u, meq);

    /* Adaptive factor.  Deviatoric non-equilibrium stress from m4..m8:
     * off-diagonal Pi_xy = m4, Pi_xz = m5, Pi_yz = m6; diagonal from
     * m7 = Pi_xx - Pi_yy and m8 = Pi_xx - Pi_zz.  Strain rate
     * S^ = -(3 S / (2 rho)) Pi (Chapman-Enskog relation), G = sqrt(2 S^:S^). */
    const double S_shear = 1.0 / (3.0 * p->nu + 0.5);
    const double n7 = m[7] - meq[7], n8 = m[8] - meq[8];
    const double Pxy = m[4] - meq[4], Pxz = m[5] - meq[5], Pyz = m[6] - meq[6];
    const double Pxx = (n7 + n8) / 3.0, Pyy = (n8 - 2.0 * n7) / 3.0,
                 Pzz = (n7 - 2.0 * n8) / 3.0;
    const double PP = Pxx * Pxx + Pyy * Pyy + Pzz * Pzz +
                      2.0 * (Pxy * Pxy + Pxz * Pxz + Pyz * Pyz);
    const double scale = 3.0 * S_shear / (2.0 * rho);
    const double G = (G_given >= 0.0) ? G_given : sqrt(2.0 * scale * scale * PP);
    double phi = 1.0;
    if (p->adaptive) {
        const double x = G / p->g_max;
        phi = p->a * (x < 1.0 ? x : 1.0) + p->b;
    }

    /* Relaxation rates. */
    double S[27];
    for (int k = 0; k < 27; ++k) {
        double nu_k;
        if (k <= 3) {
            S[k] = 0.0;
            continue;
        } else if (k <= 8) {
            S[k] = S_shear;
            continue;
        } else if (k <= 16) {
            nu_k = p->nu_hi[0];
        } else if (k <= 22) {
            nu_k = p->nu_hi[1];
        } else if (k <= 25) {
            nu_k = p->nu_hi[2];
        } else {
            nu_k = p->nu_hi[3];
        }
        S[k] = 1.0 / (3.0 * phi * nu_k + 0.5);
    }
    if (S_override) memcpy(S, S_override, sizeof S);

    /* r = -S (m - m^eq) + (I - S/2) R,  R = (0, F, 0, ...). */
    double r[27];
    for (int k = 0; k < 27; ++k) r[k] = -S[k] * (m[k] - meq[k]);
    for (int a = 0; a < 3; ++a) r[1 + a] += (1.0 - 0.5 * S[1 + a]) * F[a];

    /* Omega = T r; f~ = f + Omega. */
    double omega[27];
    if (apply_T(u, r, omega) != 0) return -1;
    for (int i = 0; i < 27; ++i) out[i] = f[i] + omega[i];

    if (diag) {
        diag[0] = rho;
        diag[1] = u[0];
        diag[2] = u[1];
        diag[3] = u[2];
        diag[4] = G;
        diag[5] = phi;
    }
    return 0;
}

/* ---------------------------------------------------------------------
 * Grid helpers.
 * ------------------------------------------------------------------- */
static int64_t n_cells(const oracle_domain* d)
{
    return (int64_t)d->nx * d->ny * d->nz;
}

static uint8_t kind_at(const oracle_domain* d, int64_t cell)
{
    return d->flags ? d->flags[cell] : ORACLE_FLUID;
}

/* Neighbour coordinate along one axis; returns 0 if it leaves a
 * non-periodic box (the face then acts as a wall). */
static int wrap(int x, int n, int periodic, int* out)
{
    if (x >= 0 && x < n) {
        *out = x;
        return 1;
    }
    if (!periodic) return 0;
    *out = ((x % n) + n) % n;
    return 1;
}

/* Source cell of the pull along velocity (cx, cy, cz) for cell (x, y, z);
 * -1 if the source is outside a non-periodic box. */
static int64_t source_cell(const oracle_domain* d, int x, int y, int z,
                           int cx, int cy, int cz)
{
    int xs, ys, zs;
    if (!wrap(x - cx, d->nx, d->periodic & 1, &xs)) return -1;
    if (!wrap(y - cy, d->ny, d->periodic & 2, &ys)) return -1;
    if (!wrap(z - cz, d->nz, d->periodic & 4, &zs)) return -1;
    return xs + (int64_t)d->nx * (ys + (int64_t)d->ny * zs);
}

/* Pull streaming (eq. lbe): f_i(x) = f~_i(x - c_i).  A solid or out-of-box
 * source reflects the opposite population of this cell (halfway
 * bounce-back).  gi is filled only when g is given. */
static void gather(const oracle_domain* d, const double* f, const double* g,
                   int x, int y, int z, int64_t cell, double fi[27], double gi[7])
{
    const int64_t N = n_cells(d);
    for (int i = 0; i < 27; ++i) {
        const int64_t src = source_cell(d, x, y, z, CX[i], CY[i], CZ[i]);
        if (src < 0 || kind_at(d, src) == ORACLE_SOLID)
            fi[i] = f[opposite(i) * N + cell];
        else
            fi[i] = f[i * N + src];
    }
    if (!g) return;
    for (int i = 0; i < 7; ++i) {
        const int64_t src = source_cell(d, x, y, z, SX[i], SY[i], SZ[i]);
        const int opp = (i == 0) ? 0 : ((i % 2) ? i + 1 : i - 1);
        if (src < 0 || kind_at(d, src) == ORACLE_SOLID)
            gi[i] = g[opp * N + cell];
        else
            gi[i] = g[i * N + src];
    }
}

/* A pull source the node cannot use: outside a non-periodic box or SOLID. */
static int blocked(const oracle_domain* d, int x, int y, int z, int cx, int cy, int cz)
{
    const int64_t src = source_cell(d, x, y, z, cx, cy, cz);
    return src < 0 || kind_at(d, src) == ORACLE_SOLID;
}

/* Wall normal of a WALL node (pointing from the node into the wall): the
 * one axis direction whose neighbour is blocked.  Returns 0 when the node
 * does not sit on one flat axis-aligned wall: no or several blocked axis
 * neighbours, or a blocked pull source other than those with c_i.n < 0. */
static int wall_normal(const oracle_domain* d, int x, int y, int z, int n[3])
{
    int found = 0;
    for (int a = 0; a < 3; ++a)
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            const int e[3] = {a == 0 ? sgn : 0, a == 1 ? sgn : 0, a == 2 ? sgn : 0};
            /* the neighbour x + e is the pull source of the velocity -e */
            if (blocked(d, x, y, z, -e[0], -e[1], -e[2])) {
                n[0] = e[0];
                n[1] = e[1];
                n[2] = e[2];
                ++found;
            }
        }
    if (found != 1) return 0;
    for (int i = 0; i < 27; ++i) {
        const int cn = CX[i] * n[0] + CY[i] * n[1] + CZ[i] * n[2];
        if (blocked(d, x, y, z, CX[i], CY[i], CZ[i]) != (cn < 0)) return 0;
    }
    return 1;
}

/* Regularized no-slip wall node (Latt & Chopard 2006; Latt et al. 2008,
 * "Straight velocity boundaries in the lattice Boltzmann method"), the
 * second-order wall treatment the section "Initialization and boundary
 * treatment" asks for.  The wall passes through the node and has velocity
 * zero; with the half-force velocity shift the node's velocity
 * (j + F/2)/rho vanishes when its momentum is j = -F/2.  On entry fi holds
 * the pulled populations (those with c_i.n < 0 come from the wall and are
 * unknown); on exit the regularized pre-collision state:
 *   rho   from mass and the normal momentum, rho = sum_{c.n=0} f + 2 sum_{c.n>0} f + F.n/2;
 *   f^eq  the second-order equilibrium at (rho, u_w = -F/(2 rho));
 *   f^neq known: f - f^eq; unknown: f^neq of the opposite population;
 *   Pi    = sum_i c_i c_i f^neq_i;
 *   f_i   = f^eq_i + w_i / (2 cs^4) (c_i c_i - cs^2 I) : Pi    (cs^2 = 1/3). */
static void regularize_wall(const int n[3], const double F[3], double fi[27])
{
    double rho = 0.5 * (F[0] * n[0] + F[1] * n[1] + F[2] * n[2]);
    for (int i = 0; i < 27; ++i) {
        const int cn = CX[i] * n[0] + CY[i] * n[1] + CZ[i] * n[2];
        if (cn == 0) rho += fi[i];
        else if (cn > 0) rho += 2.0 * fi[i];
    }
    const double uw[3] = {-F[0] / (2.0 * rho), -F[1] / (2.0 * rho), -F[2] / (2.0 * rho)};
    const double uu = uw[0] * uw[0] + uw[1] * uw[1] + uw[2] * uw[2];
    double feq[27], neq[27];
    for (int i = 0; i < 27; ++i) {
        const double cu = CX[i] * uw[0] + CY[i] * uw[1] + CZ[i] * uw[2];
        feq[i] = weight(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
    for (int i = 0; i < 27; ++i) {
        const int cn = CX[i] * n[0] + CY[i] * n[1] + CZ[i] * n[2];
        const int k = (cn < 0) ? opposite(i) : i;
        neq[i] = fi[k] - feq[k];
    }
    double Pi[3][3] = {{0.0}};
    for (int i = 0; i < 27; ++i) {
        const int c[3] = {CX[i], CY[i], CZ[i]};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Pi[a][b] += c[a] * c[b] * neq[i];
    }
    for (int i = 0; i < 27; ++i) {
        const int c[3] = {CX[i], CY[i], CZ[i]};
        double q = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) q += (c[a] * c[b] - (a == b ? 1.0 / 3.0 : 0.0)) * Pi[a][b];
        fi[i] = feq[i] + 4.5 * weight(i) * q;
    }
}

int oracle_wall_regularize(const double f[27], const int32_t n[3], const double F[3],
                           double out[27])
{
    int axes = 0;
    for (int a = 0; a < 3; ++a) {
        if (n[a] < -1 || n[a] > 1) return -1;
        axes += n[a] != 0;
    }
    if (axes != 1) return -1;
    const int nn[3] = {n[0], n[1], n[2]};
    const double Fz[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 27; ++i) out[i] = f[i];
    regularize_wall(nn, F ? F : Fz, out);
    return 0;
}

/* One cell of one step: pull-stream (eq. lbe) with boundary rules, then
 * collide.  fo[27 * stride] / go[7 * stride] receive the output with
 * element stride `stride`. */
static int step_one(const oracle_domain* d, const oracle_params* p,
                    const double* f, const double* g, const double* gfield, int64_t cell,
                    double* fo, double* go, int64_t stride)
{
    const int64_t N = n_cells(d);
    const int x = (int)(cell % d->nx);
    const int y = (int)((cell / d->nx) % d->ny);
    const int z = (int)(cell / ((int64_t)d->nx * d->ny));
    const uint8_t kind = kind_at(d, cell);

    if (kind == ORACLE_SOLID) {
        for (int i = 0; i < 27; ++i) fo[i * stride] = weight(i);
        if (g && go)
            for (int i = 0; i < 7; ++i) go[i * stride] = 0.0;
        return 0;
    }
    if (kind == ORACLE_GHOST) {
        for (int i = 0; i < 27; ++i) fo[i * stride] = f[i * N + cell];
        if (g && go)
            for (int i = 0; i < 7; ++i) go[i * stride] = g[i * N + cell];
        return 0;
    }
    if (kind == ORACLE_INLET) {
        double fe[27];
        if (oracle_equilibrium(1.0, d->u_in, fe) != 0) return -1;
        for (int i = 0; i < 27; ++i) fo[i * stride] = fe[i];
        if (g && go) {
            double ge[7];
            scalar_eq(d->s_in, d->u_in, ge);
            for (int i = 0; i < 7; ++i) go[i * stride] = ge[i];
        }
        return 0;
    }
    if (kind == ORACLE_NEUMANN) {
        /* Neumann (zero normal gradient) far-field boundary (section
         * "Initialization and boundary treatment"): copy the incoming state
         * of the cell one step inward along each face normal */
        int xs = x, ys = y, zs = z;
        if (!(d->periodic & 1) && d->nx > 1) xs = (x == 0) ? 1 : (x == d->nx - 1 ? d->nx - 2 : x);
        if (!(d->periodic & 2) && d->ny > 1) ys = (y == 0) ? 1 : (y == d->ny - 1 ? d->ny - 2 : y);
        if (!(d->periodic & 4) && d->nz > 1) zs = (z == 0) ? 1 : (z == d->nz - 1 ? d->nz - 2 : z);
        const int64_t from = xs + (int64_t)d->nx * (ys + (int64_t)d->ny * zs);
        for (int i = 0; i < 27; ++i) fo[i * stride] = f[i * N + from];
        if (g && go)
            for (int i = 0; i < 7; ++i) go[i * stride] = g[i * N + from];
        return 0;
    }
    if (kind == ORACLE_OUTFLOW) {
        /* zero-gradient: copy the incoming state of the x-1 neighbour */
        const int64_t src = source_cell(d, x, y, z, 1, 0, 0);
        const int64_t from = (src >= 0) ? src : cell;
        for (int i = 0; i < 27; ++i) fo[i * stride] = f[i * N + from];
        if (g && go)
            for (int i = 0; i < 7; ++i) go[i * stride] = g[i * N + from];
        return 0;
    }

    double fi[27], gi[7] = {0};
    gather(d, f, g, x, y, z, cell, fi, gi);
    double s = 0.0;
    if (g)
        for (int i = 0; i < 7; ++i) s += gi[i];

    /* Body force: per-cell field plus buoyancy along z. */
    double F[3] = {0.0, 0.0, 0.0};
    if (d->theta)
        for (int a = 0; a < 3; ++a) F[a] = d->theta[a * N + cell];
    if (g) F[2] += p->beta * (s - p->s_ref);

    if (kind == ORACLE_WALL) {
        int n[3];
        if (!wall_normal(d, x, y, z, n)) return -1;
        regularize_wall(n, F, fi);
    }

    double post[27], diag[6];
    const double Gc = gfield ? gfield[cell] : -1.0;
    if (collide_impl(fi, F, p, NULL, Gc, post, diag) != 0) return -1;
    for (int i = 0; i < 27; ++i) fo[i * stride] = post[i];

    if (g && go) {
        /* Scalar BGK: g~ = g - (g - g^eq(s, u)) / tau_s, u the fluid velocity. */
        double ge[7];
        const double u[3] = {diag[1], diag[2], diag[3]};
        scalar_eq(s, u, ge);
        for (int i = 0; i < 7; ++i) go[i * stride] = gi[i] - (gi[i] - ge[i]) / p->tau_s;
    }
    return 0;
}

int oracle_init(const oracle_domain* d, const double* rho, const double* u,
                const double* s, double* f, double* g)
{
    const int64_t N = n_cells(d);
    int err = 0;
#pragma omp parallel for schedule(static) reduction(| : err)
    for (int64_t c = 0; c < N; ++c) {
        const double uc[3] = {u[c], u[N + c], u[2 * N + c]};
        double fe[27];
        if (oracle_equilibrium(rho[c], uc, fe) != 0) err |= 1;
        for (int i = 0; i < 27; ++i) f[i * N + c] = fe[i];
        if (g) {
            double ge[7];
            scalar_eq(s ? s[c] : 0.0, uc, ge);
            for (int i = 0; i < 7; ++i) g[i * N + c] = ge[i];
        }
    }
    return err ? -1 : 0;
}

/* |grad u|_F of the read-back velocity field (central differences). */
int oracle_grad_field(const oracle_domain* d, const oracle_params* p,
                      const double* f, const double* g, double* G)
{
    const int64_t N = n_cells(d);
    double* rho = (double*)malloc(sizeof(double) * N);
    double* u = (double*)malloc(sizeof(double) * 3 * N);
    if (!rho || !u) {
        free(rho);
        free(u);
        return -1;
    }
    oracle_macro(d, p, f, g, rho, u, NULL);
    const int n[3] = {d->nx, d->ny, d->nz};
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        const int x[3] = {(int)(c % d->nx), (int)((c / d->nx) % d->ny),
                          (int)(c / ((int64_t)d->nx * d->ny))};
        double sum = 0.0;
        for (int a = 0; a < 3; ++a) {          /* derivative direction */
            int lo[3] = {x[0], x[1], x[2]}, hi[3] = {x[0], x[1], x[2]};
            double h = 2.0;
            if (d->periodic & (1 << a)) {
                lo[a] = (x[a] - 1 + n[a]) % n[a];
                hi[a] = (x[a] + 1) % n[a];
            } else {
                lo[a] = x[a] > 0 ? x[a] - 1 : x[a];
                hi[a] = x[a] < n[a] - 1 ? x[a] + 1 : x[a];
                h = (double)(hi[a] - lo[a]);
            }
            const int64_t cl = lo[0] + (int64_t)d->nx * (lo[1] + (int64_t)d->ny * lo[2]);
            const int64_t ch = hi[0] + (int64_t)d->nx * (hi[1] + (int64_t)d->ny * hi[2]);
            for (int b = 0; b < 3; ++b) {      /* velocity component */
                const double dv = (h > 0.0) ? (u[b * N + ch] - u[b * N + cl]) / h : 0.0;
                sum += dv * dv;
            }
        }
        G[c] = sqrt(sum);
    }
    free(rho);
    free(u);
    return 0;
}

int oracle_step(const oracle_domain* d, const oracle_params* p,
                const double* f, const double* g, double* f_out, double* g_out)
{
    const int64_t N = n_cells(d);
    double* gfield = NULL;
    if (p->grad_mode == 1) {
        gfield = (double*)malloc(sizeof(double) * N);
        if (!gfield || oracle_grad_field(d, p, f, g, gfield) != 0) {
            free(gfield);
            return -1;
        }
    }
    int err = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : err) if (N >= 4096)
    for (int64_t c = 0; c < N; ++c) {
        if (step_one(d, p, f, g, gfield, c, f_out + c, g_out ? g_out + c : NULL, N) != 0) err |= 1;
    }
    free(gfield);
    return err ? -1 : 0;
}

int oracle_step_cells(const oracle_domain* d, const oracle_params* p,
                      const double* f, const double* g,
                      const int64_t* cells, int64_t n, double* f_out, double* g_out)
{
    const int64_t N = n_cells(d);
    double* gfield = NULL;
    if (p->grad_mode == 1) {
        gfield = (double*)malloc(sizeof(double) * N);
        if (!gfield || oracle_grad_field(d, p, f, g, gfield) != 0) {
            free(gfield);
            return -1;
        }
    }
    int err = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : err)
    for (int64_t k = 0; k < n; ++k) {
        if (cells[k] < 0 || cells[k] >= N) {
            err |= 1;
            continue;
        }
        if (step_one(d, p, f, g, gfield, cells[k], f_out + k, g_out ? g_out + k : NULL, n) != 0)
            err |= 1;
    }
    free(gfield);
    return err ? -1 : 0;
}

int oracle_macro(const oracle_domain* d, const oracle_params* p,
                 const double* f, const double* g, double* rho, double* u, double* s)
{
    const int64_t N = n_cells(d);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        double r = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < 27; ++i) {
            const double v = f[i * N + c];
            r += v;
            j[0] += CX[i] * v;
            j[1] += CY[i] * v;
            j[2] += CZ[i] * v;
        }
        double sc = 0.0;
        if (g)
            for (int i = 0; i < 7; ++i) sc += g[i * N + c];
        double F[3] = {0.0, 0.0, 0.0};
        if (d->theta)
            for (int a = 0; a < 3; ++a) F[a] = d->theta[a * N + c];
        if (g) F[2] += p->beta * (sc - p->s_ref);
        rho[c] = r;
        for (int a = 0; a < 3; ++a) u[a * N + c] = (j[a] - 0.5 * F[a]) / r;
        if (s) s[c] = sc;
    }
    return 0;
}

int oracle_stream(const oracle_domain* d, const double* f, const double* g,
                  double* f_out, double* g_out)
{
    const int64_t N = n_cells(d);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < N; ++c) {
        const int x = (int)(c % d->nx);
        const int y = (int)((c / d->nx) % d->ny);
        const int z = (int)(c / ((int64_t)d->nx * d->ny));
        double fi[27], gi[7];
        if (kind_at(d, c) == ORACLE_FLUID) {
            gather(d, f, g, x, y, z, c, fi, gi);
        } else {
            for (int i = 0; i < 27; ++i) fi[i] = f[i * N + c];
            if (g)
                for (int i = 0; i < 7; ++i) gi[i] = g[i * N + c];
        }
        for (int i = 0; i < 27; ++i) f_out[i * N + c] = fi[i];
        if (g && g_out)
            for (int i = 0; i < 7; ++i) g_out[i * N + c] = gi[i];
    }
    return 0;
}

/* ---------------------------------------------------------------------
 * Cross-scale exchange.
 * ------------------------------------------------------------------- */

/* Source cell index along one axis with periodic wrap; -1 outside a
 * non-periodic box. */
static int64_t axis_index(int64_t i, int n, int periodic)
{
    if (i >= 0 && i < n) return i;
    if (!periodic) return -1;
    return ((i % n) + n) % n;
}

int oracle_exchange(const oracle_scale* src, const double* fA, const double* fB,
                    const double* gA, const double* gB, double w,
                    const oracle_scale* dst, const int64_t* cells, int64_t n_cells,
                    double* f_out, double* g_out)
{
    const int64_t Ns = (int64_t)src->nx * src->ny * src->nz;
    const int64_t Nd = (int64_t)dst->nx * dst->ny * dst->nz;
    const double alpha = src->dx / dst->dx;
    const double S_src = 1.0 / (3.0 * src->nu + 0.5);
    const double S_dst = 1.0 / (3.0 * dst->nu + 0.5);
    /* K^ for the stress moments m4..m8 */
    const double kappa = (1.0 - S_dst) / (1.0 - S_src) * S_src / (alpha * S_dst);
    const int with_scalar = gA && g_out;
    const double kappa_s = with_scalar ? (dst->tau_s - 1.0) / (alpha * (src->tau_s - 1.0)) : 0.0;
    int err = 0;
#pragma omp parallel for schedule(static) reduction(| : err)
    for (int64_t k = 0; k < n_cells; ++k) {
        const int64_t c = cells[k];
        if (c < 0 || c >= Nd) {
            err |= 1;
            continue;
        }
        const int x = (int)(c % dst->nx), y = (int)((c / dst->nx) % dst->ny),
                  z = (int)(c / ((int64_t)dst->nx * dst->ny));
        const double p[3] = {dst->origin[0] + x * dst->dx, dst->origin[1] + y * dst->dx,
                             dst->origin[2] + z * dst->dx};
        /* section "Spatial scale mapping": trilinear from the 8 corners of
         * the source cell containing p */
        int64_t base[3];
        double t[3];
        const int nsrc[3] = {src->nx, src->ny, src->nz};
        for (int a = 0; a < 3; ++a) {
            const double q = (p[a] - src->origin[a]) / src->dx;
            base[a] = (int64_t)floor(q);
            t[a] = q - (double)base[a];
        }
        double fi[27] = {0}, gi[7] = {0};
        for (int corner = 0; corner < 8; ++corner) {
            const int o[3] = {corner & 1, (corner >> 1) & 1, (corner >> 2) & 1};
            double wt = 1.0;
            int64_t idx[3];
            for (int a = 0; a < 3; ++a) {
                wt *= o[a] ? t[a] : 1.0 - t[a];
                idx[a] = axis_index(base[a] + o[a], nsrc[a], src->periodic & (1 << a));
            }
            if (wt == 0.0) continue;
            if (idx[0] < 0 || idx[1] < 0 || idx[2] < 0) {
                err |= 1;
                break;
            }
            const int64_t sc = idx[0] + (int64_t)src->nx * (idx[1] + (int64_t)src->ny * idx[2]);
            for (int i = 0; i < 27; ++i)
                fi[i] += wt * ((1.0 - w) * fA[i * Ns + sc] + w * fB[i * Ns + sc]);
            if (with_scalar)
                for (int i = 0; i < 7; ++i)
                    gi[i] += wt * ((1.0 - w) * gA[i * Ns + sc] + w * gB[i * Ns + sc]);
        }
        /* eq. s1_to_s2_mapping: f = T (m^eq + K^ m~^neq) */
        double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < 27; ++i) {
            rho += fi[i];
            j[0] += CX[i] * fi[i];
            j[1] += CY[i] * fi[i];
            j[2] += CZ[i] * fi[i];
        }
        const double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
        double M[729], m[27], meq[27], r[27], fo[27];
        oracle_basis(u, M);
        for (int q = 0; q < 27; ++q) {
            double acc = 0.0;
            for (int i = 0; i < 27; ++i) acc += M[i * 27 + q] * fi[i];
            m[q] = acc;
        }
        oracle_meq(rho, u, meq);
        for (int q = 0; q < 27; ++q) {
            const double Kq = (q >= 4 && q <= 8) ? kappa : 1.0;
            r[q] = meq[q] + Kq * (m[q] - meq[q]);
        }
        if (apply_T(u, r, fo) != 0) {
            err |= 1;
            continue;
        }
        for (int i = 0; i < 27; ++i) f_out[i * Nd + c] = fo[i];
        if (with_scalar) {
            double sc = 0.0, ge[7];
            for (int i = 0; i < 7; ++i) sc += gi[i];
            scalar_eq(sc, u, ge);
            for (int i = 0; i < 7; ++i) g_out[i * Nd + c] = ge[i] + kappa_s * (gi[i] - ge[i]);
        }
    }
    return err ? -1 : 0;
}

void oracle_time_interp(const double* s0, const double* s1, const double* s2,
                        double t0, double t1, double t2, double t, int64_t n, double* out)
{
    const double l0 = (t - t1) * (t - t2) / ((t0 - t1) * (t0 - t2));
    const double l1 = (t - t0) * (t - t2) / ((t1 - t0) * (t1 - t2));
    const double l2 = (t - t0) * (t - t1) / ((t2 - t0) * (t2 - t1));
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) out[k] = l0 * s0[k] + l1 * s1[k] + l2 * s2[k];
}
