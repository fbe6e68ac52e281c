/*
 * cmr_oracle.h -- plain FP64 CPU reference of the continuous-scale
 * central-moment lattice Boltzmann method (Li, Bai & Liu, "Continuous-Scale
 * Kinetic Fluid Simulation", arXiv 1807.02284).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the CPU baseline of the benchmark can compare the GPU library
 * against an obviously-correct definition.  It shares no code, header, table
 * or generator with the GPU library, and no product code may call it.
 *
 * Conventions
 *   - Populations are stored as f[i*N + cell], i = 0..26 in the order of the
 *     appendix velocity list, cell = x + nx*(y + ny*z)  (x fastest, dense,
 *     no padding).  Values are the physical populations f_i (not shifted).
 *   - The stored state of a level at step n is the post-collision field
 *     f~(n).  One step = pull-stream then collide:
 *        f_i(x) = f~_i(x - c_i, n-1),   f~(n)(x) = C(f(x)).
 *   - D3Q7 scalar populations g[i*N + cell], i = 0..6 with velocities
 *     0, +x, -x, +y, -y, +z, -z.
 *
 * Parity status: every function here is pinned by the CPU test suite
 * (closed forms, invariants, brute force, special cases that reduce to
 * textbook schemes).  The readings of passages the paper leaves open are
 * listed in cmr_oracle.c; the multi-scale schedule built on these functions
 * (multilevel.py) states which of its readings are only loosely pinned.
 */
#ifndef CMR_ORACLE_H
#define CMR_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Cell kinds (one byte per cell). */
enum {
    ORACLE_FLUID = 0,
    ORACLE_SOLID = 1,   /* halfway bounce-back obstacle; output = rest state w_i */
    ORACLE_INLET = 2,   /* Dirichlet: output = f^eq(1, u_in), g^eq(s_in, u_in) */
    ORACLE_OUTFLOW = 3, /* zero-gradient: output = input of the x-1 neighbour */
    ORACLE_GHOST = 4,   /* written only by the scale exchange; output = input */
    ORACLE_NEUMANN = 5, /* far-field zero-gradient on the box faces: output =
                           input of the neighbour one cell inward along every
                           non-periodic face the cell lies on */
    ORACLE_WALL = 6     /* no-slip wall through this node (the second-order
                           wall of section "Initialization and boundary
                           treatment"): the regularized boundary condition of
                           Latt & Chopard (Math. Comput. Simul. 72, 2006;
                           Latt et al., Phys. Rev. E 77, 056703, 2008) on a
                           flat wall aligned with a lattice axis: exactly one
                           of the 6 axis neighbours is SOLID or outside the
                           box (the wall side, normal n), and the populations
                           pulled from SOLID or outside sources are exactly
                           those with c_i.n < 0; anything else is an error */
};

typedef struct {
    double nu;        /* shear viscosity, sets S4..S8 (viscosity relation) */
    double nu_hi[4];  /* artificial viscosities of m9..m16, m17..m22, m23..m25, m26 */
    double a, b;      /* adaptive relaxation model parameters */
    double g_max;     /* gradient normalisation of the adaptive relaxation */
    int32_t adaptive; /* 0: phi = 1; 1: phi = a*min(G/g_max,1) + b */
    int32_t grad_mode; /* G of the adaptive factor: 0 = local strain-rate
                          magnitude sqrt(2 S^:S^) from the non-equilibrium
                          stress; 1 = |grad u|_F of the stored velocity field
                          by central differences (one step lagged) */
    double tau_s;     /* D3Q7 scalar BGK relaxation time */
    double beta;      /* buoyancy coefficient, F_z += beta*(s - s_ref) */
    double s_ref;
} oracle_params;

typedef struct {
    int32_t nx, ny, nz;
    int32_t periodic;          /* bit 0: x, bit 1: y, bit 2: z; a non-periodic
                                  face acts as a halfway bounce-back wall */
    const uint8_t* flags;      /* [N] or NULL (all fluid) */
    const double* theta;       /* body-force field [3][N] or NULL */
    double u_in[3];            /* inlet velocity */
    double s_in;               /* inlet scalar value */
} oracle_domain;

/* Lattice tables, exposed so that tests can pin them. */
void oracle_velocities(int32_t c[81]);        /* c[3*i + a] */
void oracle_weights(double w[27]);
void oracle_basis(const double u[3], double M[729]);   /* M[i*27 + j] = M_ij(u) */
void oracle_meq(double rho, const double u[3], double meq[27]);

/* One-cell collision by the definition.  F = body force (may be NULL).
 * S_override (may be NULL) replaces the 27 relaxation rates.
 * diag (may be NULL) receives {rho, ux, uy, uz, G, phi}.
 * Returns 0, or -1 if the linear solve fails. */
int oracle_collide(const double f[27], const double F[3], const oracle_params* p,
                   const double* S_override, double out[27], double diag[6]);

/* f = T m^eq(rho, u): the equilibrium initialisation. */
int oracle_equilibrium(double rho, const double u[3], double f[27]);

/* Initialise a whole field from rho[N], u[3][N] (s[N] may be NULL). */
int oracle_init(const oracle_domain* d, const double* rho, const double* u,
                const double* s, double* f, double* g);

/* One step for every cell.  g / g_out may be NULL (no scalar). */
/* oracle_collide with the gradient magnitude G of the adaptive factor
 * given (G >= 0) instead of estimated from the cell's own stress (G < 0). */
int oracle_collide_g(const double f[27], const double F[3], const oracle_params* p, double G,
                     double out[27], double diag[6]);

/* |grad u|_F at every cell of the velocity read back from the stored state
 * (f, g): central differences, periodic wrap on periodic axes, one-sided
 * differences at non-periodic faces.  G[N]. */
int oracle_grad_field(const oracle_domain* d, const oracle_params* p,
                      const double* f, const double* g, double* G);

int oracle_step(const oracle_domain* d, const oracle_params* p,
                const double* f, const double* g, double* f_out, double* g_out);

/* Pull streaming alone (the left-hand side of eq. lbe): fluid cells receive
 * f~_i(x - c_i) with the bounce-back rule; other cells copy their input. */
int oracle_stream(const oracle_domain* d, const double* f, const double* g,
                  double* f_out, double* g_out);

/* oracle_step evaluated only at the listed cells: f_out[i*n_cells + k]
 * receives the output of cell cells[k] (g_out likewise, 7 per cell). */
int oracle_step_cells(const oracle_domain* d, const oracle_params* p,
                      const double* f, const double* g,
                      const int64_t* cells, int64_t n_cells,
                      double* f_out, double* g_out);

/* Macroscopic fields of a post-collision state: rho, u = (sum c f~ - F/2)/rho,
 * s = sum g (s may be NULL; needs g). */
int oracle_macro(const oracle_domain* d, const oracle_params* p,
                 const double* f, const double* g,
                 double* rho, double* u, double* s);

/* ------------------------------------------------------------------------
 * Cross-scale exchange (sections "Mapping distribution functions" to
 * "Handling multiple scales").
 * ---------------------------------------------------------------------- */

/* Geometry and relaxation of one scale: lattice point (x, y, z) sits at the
 * physical position origin + (x, y, z) * dx. */
typedef struct {
    int32_t nx, ny, nz;
    int32_t periodic;      /* bit mask as in oracle_domain */
    double origin[3];
    double dx;             /* physical spacing of this scale */
    double nu;             /* shear viscosity in this scale's lattice units */
    double tau_s;          /* scalar relaxation time (0: no scalar) */
} oracle_scale;

/* Post-collision mapping from scale `src` to the cells `cells` of scale
 * `dst` (eq. s1_to_s2_mapping): the source state at the time weight w is
 * (1 - w) fA + w fB; it is interpolated trilinearly from the 8 corners of the
 * source cell that contains each target point, and the mapped populations
 * are T(m^eq + K^ m~^neq) with K^ = (I - S^dst) K (I - S^src)^-1, K = diag
 * with S_k^src / (alpha S_k^dst) for k = 4..8 and 1 elsewhere, alpha =
 * dx_src / dx_dst.  Only m4..m8 are rescaled (the higher-order rates are
 * the same lattice quantities on every scale).  The scalar (if gA != NULL
 * and g_out != NULL) is interpolated the same way and its non-equilibrium
 * part g - g^eq(s, u) scaled by (tau_dst - 1) / (alpha (tau_src - 1)).
 * Writes f_out[i*N_dst + cell] for the listed cells only.  fB may equal fA.
 * Returns -1 if a stencil leaves a non-periodic source box. */
int oracle_exchange(const oracle_scale* src, const double* fA, const double* fB,
                    const double* gA, const double* gB, double w,
                    const oracle_scale* dst, const int64_t* cells, int64_t n_cells,
                    double* f_out, double* g_out);

/* Lagrange quadratic through (t0, s0), (t1, s1), (t2, s2) evaluated at t:
 * out[k] for k < n (section "Temporal alignment and scale mapping"). */
/* The regularized no-slip wall node applied to one cell's pulled
 * populations f (the ORACLE_WALL rule of oracle_step, without the step):
 * n is the wall normal (a unit axis vector pointing into the wall), F the
 * body force at the node (may be NULL).  Returns -1 for a bad normal. */
int oracle_wall_regularize(const double f[27], const int32_t n[3], const double F[3],
                           double out[27]);

void oracle_time_interp(const double* s0, const double* s1, const double* s2,
                        double t0, double t1, double t2, double t, int64_t n, double* out);

#ifdef __cplusplus
}
#endif
#endif
