/*
 * cslbm.h -- C ABI of the continuous-scale central-moment lattice Boltzmann
 * library for AMD Instinct MI355X (gfx950).
 *
 * Method: Li, Bai & Liu, "Continuous-Scale Kinetic Fluid Simulation"
 * (arXiv 1807.02284).  The library evaluates the lattice Boltzmann update
 * (eq. lbe) on D3Q27 with the non-orthogonal central-moment collision
 * (eq. cmr_collision, appendix) and the adaptive relaxation of the
 * higher-order moments (section "Adaptive relaxation").
 *
 * General rules
 *   - Every pointer inside cslbm_level and every array argument is a DEVICE
 *     pointer unless stated otherwise.  All device memory is owned by the
 *     caller; the library keeps no pointer beyond a call.  Calls that need
 *     temporary device memory take it from the stream-ordered allocator and
 *     return it before they return.
 *   - Every call enqueues its kernels on the given stream and returns without
 *     synchronising, except calls that return values on the host
 *     (cslbm_conserved_f64, cslbm_check_finite), which synchronise the stream.
 *   - Return value: CSLBM_OK (0) or a negative CSLBM_ERR_* code.  Arguments
 *     are validated before any launch; a failed validation launches nothing.
 *     cslbm_last_error() returns a message for the last failure of the
 *     calling thread.  No C++ exception crosses this interface.
 *
 * Field layout
 *   - A level is a dense nx*ny*nz box; cell = x + nx*(y + ny*z) (x fastest).
 *   - Populations: 27 planes of `plane` elements each (plane >= nx*ny*nz),
 *     population i in the order of the appendix velocity list (entry 13 of
 *     c_z taken as -1).  Stored values are SHIFTED populations
 *     h_i = f_i - w_i with the product weights w = (2/3, 1/6, 1/6)^3:
 *     float for CSLBM_F32, IEEE binary16 (round to nearest even, subnormals
 *     kept) for CSLBM_F16S.  Arithmetic is FP32 in both cases.
 *   - The stored state at step n is the post-collision field f~(n); one
 *     step pulls f_i(x) = f~_i(x - c_i, n-1) and collides.
 *   - Passive scalar (optional): 7 float planes, D3Q7 velocities rest, +x,
 *     -x, +y, -y, +z, -z, unshifted.
 *   - Macroscopic arrays passed to init / read-back are dense (stride
 *     nx*ny*nz, not plane): rho[N], u[3][N], s[N].
 */
#ifndef CSLBM_H
#define CSLBM_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define CSLBM_OK 0
#define CSLBM_ERR_ARG (-1)          /* invalid pointer or parameter value */
#define CSLBM_ERR_SHAPE (-2)        /* inconsistent sizes / strides */
#define CSLBM_ERR_UNSUPPORTED (-3)  /* valid but not implemented combination */
#define CSLBM_ERR_HIP (-4)          /* a HIP runtime call or launch failed */
#define CSLBM_ERR_NONFINITE (-5)    /* NaN or Inf found in the state */

/* storage formats */
#define CSLBM_F32 0
#define CSLBM_F16S 1

/* cell kinds: low 3 bits of the per-cell flag byte.  Bits 3 (CSLBM_NEAR_WALL),
 * 4 (CSLBM_NEAR_FLUID) and 5-7 (the wall normal of a CSLBM_WALL cell) are
 * owned by the library and set by cslbm_prepare_flags. */
#define CSLBM_FLUID 0    /* collided */
#define CSLBM_SOLID 1    /* obstacle: halfway bounce-back for its neighbours;
                            its own output is the rest state (h = 0, g = 0) */
#define CSLBM_INLET 2    /* Dirichlet: output f^eq(1, u_in), g^eq(s_in, u_in) */
#define CSLBM_OUTFLOW 3  /* zero gradient: output = input of the x-1 neighbour */
#define CSLBM_GHOST 4    /* never collided; output = input (scale exchange writes it) */
#define CSLBM_NEUMANN 5  /* far-field zero gradient (section "Initialization and
                            boundary treatment"): output = input of the cell one
                            step inward along every non-periodic face it lies on */
#define CSLBM_WALL 6     /* no-slip wall through this node, the second-order
                            wall treatment of section "Initialization and
                            boundary treatment" (Latt et al.), written as the
                            regularized boundary condition of Latt & Chopard
                            (Math. Comput. Simul. 72, 2006; Latt et al., Phys.
                            Rev. E 77, 056703, 2008): the node is collided like
                            a fluid node after its populations are rebuilt as
                            f^eq(rho, u_w) + w/(2 cs^4) Q:Pi, with rho from
                            mass and normal momentum, the non-equilibrium of
                            the populations coming from the wall bounced from
                            the opposite ones, and u_w = -F/(2 rho) so that
                            the node's velocity (j + F/2)/rho is zero.  The
                            node must lie on one flat wall normal to a lattice
                            axis: exactly one of its 6 axis neighbours is
                            SOLID or outside a non-periodic face, and its
                            pull sources that are SOLID or outside are exactly
                            those of the 9 velocities pointing away from that
                            wall.  Otherwise cslbm_prepare_flags stores normal
                            code 7 and the step writes NaN at the cell, which
                            cslbm_check_finite reports. */
#define CSLBM_NEAR_WALL 8
#define CSLBM_NEAR_FLUID 16
#define CSLBM_WALL_NORMAL_SHIFT 5   /* flags >> 5 of a WALL cell: 1..6 = wall
                                       normal -x, +x, -y, +y, -z, +z (from the
                                       node into the wall); 7 = not on one
                                       flat axis-aligned wall */

/* floats in cslbm_level.gmax_buf */
#define CSLBM_GMAX_BUF 1025

/* Relaxation and model parameters (lattice units of the level). */
typedef struct cslbm_params {
    double nu;        /* shear viscosity: S4..S8 = 1/(3 nu + 1/2) (eq. viscosity) */
    double nu_hi[4];  /* artificial viscosities nu'_i of m9..m16, m17..m22,
                         m23..m25, m26 (appendix: 0.005, 0.007, 0.009, 0.01) */
    double a, b;      /* adaptive relaxation nu^'_i = (a G/g_max + b) nu'_i,
                         G clamped to g_max (paper: a = -4, b = 5) */
    double g_max;     /* gradient normalisation, > 0 */
    int32_t adaptive; /* 0: the factor is 1 (fixed nu'_i) */
    int32_t grad_mode; /* G of the adaptive factor: 0 = local strain-rate
                          magnitude sqrt(2 S^:S^) from the cell's own
                          non-equilibrium stress (eq. pi_1); 1 = |grad u|_F
                          of the stored velocity field by central differences
                          (one step lagged; needs vel/vel_next, fully
                          periodic levels without flags, cslbm_step only) */
    int32_t gmax_running; /* grad_mode 1 only: 0 = g_max is the constant
                          above; 1 = g_max is the maximum of the gradient
                          field of the step (section "Adaptive relaxation":
                          the maximum gradient magnitude for normalisation),
                          reduced before every step into gmax_buf */
    double tau_s;     /* scalar BGK relaxation time (> 1/2) */
    double beta;      /* buoyancy: F_z += beta (s - s_ref) */
    double s_ref;
    double u_in[3];   /* inlet velocity (CSLBM_INLET cells) */
    double s_in;      /* inlet scalar value */
} cslbm_params;

/* One uniform level (scale).  The library reads every field and writes only
 * f/f_next and g/g_next (swapped by cslbm_step). */
typedef struct cslbm_level {
    int32_t nx, ny, nz;
    int32_t storage;          /* CSLBM_F32 or CSLBM_F16S */
    int32_t periodic;         /* bit 0: x, bit 1: y, bit 2: z.  A non-periodic
                                 face is a halfway bounce-back wall; any
                                 non-periodic axis requires flags. */
    int32_t reserved0;
    int64_t plane;            /* elements per population plane, >= nx*ny*nz */
    void* f;                  /* [27][plane] current state (storage type) */
    void* f_next;             /* [27][plane] next state; must not alias f */
    float* g;                 /* [7][plane] scalar state, or NULL */
    float* g_next;            /* [7][plane], or NULL (both or neither) */
    uint8_t* flags;           /* [nx*ny*nz] cell kinds, or NULL = all fluid */
    uint32_t* links;          /* [nx*ny*nz] bounce-back masks written by
                                 cslbm_prepare_flags (bit i: the pull source
                                 x - c_i is solid or outside a non-periodic
                                 face), or NULL (computed per step instead) */
    const float* force;       /* [3][plane] body force field theta, or NULL */
    float* vel;               /* [3][nx*ny*nz] velocity read back from the
                                 current state (grad_mode 1), or NULL; written
                                 by cslbm_init_equilibrium and
                                 cslbm_set_populations, advanced by cslbm_step */
    float* vel_next;          /* [3][nx*ny*nz] next velocity (grad_mode 1) */
    float* gmax_buf;          /* [CSLBM_GMAX_BUF] work space of the running
                                 maximum (gmax_running 1): CSLBM_GMAX_BUF - 1
                                 partial slots, zeroed by the caller once and
                                 left zeroed by every step, then the field
                                 maximum of the last step in the last element */
    const int32_t* brick_table;  /* sparse brick storage, or NULL for a dense
                                 box: [nz/8][ny/8][nx/8] index of each 8x8x8
                                 brick of the box among the stored bricks, -1
                                 for a brick that is not stored */
    const int32_t* brick_origin; /* [n_bricks][3] brick coordinates (x, y, z,
                                 in bricks) of the stored bricks */
    int32_t n_bricks;         /* stored bricks (brick levels); cells are then
                                 stored brick after brick, 512 per brick in
                                 x-fastest order: index 512 b + lx + 8 ly + 64 lz,
                                 and every per-cell array (flags, links,
                                 states, lists) uses that order */
    int32_t wall_cells;       /* number of CSLBM_WALL cells in flags (0 when
                                 there are none); the caller keeps it in step
                                 with the flags.  The step handles wall cells
                                 in any case; the adjoint calls, which do not
                                 differentiate them, reject a level with
                                 wall_cells != 0 (CSLBM_ERR_UNSUPPORTED) */
    double origin[3];         /* physical position of cell (0,0,0) */
    double dx;                /* physical spacing of this scale */
    cslbm_params p;
} cslbm_level;

/* Brick levels (brick_table set; build addition for thin dynamic regions):
 * nx, ny, nz multiples of 8, no periodic axis, flags required, and every
 * FLUID cell's 26 neighbours stored (a GHOST or SOLID layer separates the
 * fluid from the bricks that are not stored).  Supported by the step (no
 * force field, grad_mode 0), the exchange on either side, the multi-scale
 * step and every per-cell call; not by cslbm_vorticity, the adjoints or the
 * gradient mode (CSLBM_ERR_UNSUPPORTED).  The plane stride of a brick level
 * is that of n_bricks * 512 cells: cslbm_plane_stride(512 * n_bricks, 1, 1). */

/* Recommended plane stride for a level: nx*ny*nz rounded up and padded so
 * that the 27 planes do not start at identical offsets modulo large powers
 * of two.  Returns a negative code for invalid sizes. */
int64_t cslbm_plane_stride(int32_t nx, int32_t ny, int32_t nz);

/* Bytes of ONE time level of state: 27 population planes (+7 scalar planes
 * when with_scalar) of cslbm_plane_stride elements.  Negative on error. */
int64_t cslbm_level_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t storage,
                          int32_t with_scalar);

/* Set bit CSLBM_NEAR_WALL of every fluid cell whose pull stencil reaches a
 * solid cell or leaves the box through a non-periodic face, and bit
 * CSLBM_NEAR_FLUID of every other cell with a fluid cell among its 26
 * neighbours (in a dense box taken with periodic wrap on every axis, in a
 * brick level only the stored ones); clear them
 * elsewhere, and (when L->links is set) write each cell's bounce-back mask.
 * Must be called after the kinds in L->flags change and before stepping. */
int cslbm_prepare_flags(const cslbm_level* L, hipStream_t stream);

/* Equilibrium initialisation (section "Initialization and boundary
 * treatment", f_0 = T m^eq(rho, u)).  Writes L->f (and L->g when present:
 * g^eq(s, u)).  rho may be NULL (rho = 1), s may be NULL (s = 0); u is
 * [3][N] dense. */
int cslbm_init_equilibrium(cslbm_level* L, const float* rho, const float* u, const float* s,
                           hipStream_t stream);

/* Copy populations into L->f from a dense [27][N] float array: physical f_i
 * when shifted == 0, f_i - w_i when shifted != 0.  g (dense [7][N], may be
 * NULL) goes to L->g. */
int cslbm_set_populations(cslbm_level* L, const float* f, const float* g, int32_t shifted,
                          hipStream_t stream);

/* Copy the state (f, and g when both carry the scalar) of the listed cells
 * of src to the listed cells of dst: dst cell dst_cells[k] receives src cell
 * src_cells[k] (device int32 lists of n_cells entries, each inside its
 * level; dst_cells distinct).  Both levels must use one storage format.
 * Used when a dynamic region is rebuilt (section "Scale construction",
 * dynamic scales): cells in both the old and the new box of a scale keep
 * their state.  Errors: CSLBM_ERR_UNSUPPORTED for mixed storage,
 * CSLBM_ERR_ARG for bad lists, aliasing states or a scalar on one side. */
int cslbm_copy_cells(const cslbm_level* src, const int32_t* src_cells, cslbm_level* dst,
                     const int32_t* dst_cells, int32_t n_cells, hipStream_t stream);

/* Copy L->f out to a dense [27][N] float array (physical f_i, or f_i - w_i
 * when shifted != 0), and L->g to g when both are non-NULL. */
int cslbm_get_populations(const cslbm_level* L, float* f, float* g, int32_t shifted,
                          hipStream_t stream);

/* n_steps lattice Boltzmann steps (eq. lbe with eq. cmr_collision): for
 * each step, pull-stream L->f into registers, collide, write L->f_next, and
 * swap L->f <-> L->f_next (and g) in *L.  After an even number of steps the
 * buffers are back in their original roles. */
int cslbm_step(cslbm_level* L, int32_t n_steps, hipStream_t stream);

/* Macroscopic fields of the stored state (the density and velocity that
 * follow eq. lbe: rho = sum_i f_i, u = sum_i c_i f_i / rho, read back after
 * the paper's iterations): rho = sum f~, u = (sum c f~ - F/2)/rho with the
 * body force F of the level (0 without one), s = sum g.  Outputs are dense
 * device float arrays of N = nx*ny*nz cells in storage order (u as
 * [3][N]); any output may be NULL.  Errors: CSLBM_ERR_ARG for a bad level,
 * CSLBM_ERR_HIP for a failed launch. */
int cslbm_read_macro(const cslbm_level* L, float* rho, float* u, float* s, hipStream_t stream);

/* Vorticity magnitude |curl u| of the stored state into omega (dense [N]),
 * and the speed |u| into speed (dense [N], may be NULL): u as in
 * cslbm_read_macro, central differences (periodic wrap on periodic axes,
 * one-sided at non-periodic faces).  The two thresholds of the dynamic
 * scale construction (section "Scale construction": gradient magnitude,
 * then velocity magnitude) are applied to these fields.  Takes its
 * temporary velocity field from the stream-ordered allocator. */
int cslbm_vorticity(const cslbm_level* L, float* omega, float* speed, hipStream_t stream);

/* Conserved totals over cells that are neither SOLID nor GHOST, accumulated
 * in FP64 with a fixed reduction order (bitwise reproducible):
 * out[0] = sum rho, out[1..3] = sum c f~ (momentum), out[4] = sum s (0
 * without scalar).  out is a HOST array; synchronises the stream. */
int cslbm_conserved_f64(const cslbm_level* L, double out[5], hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the totals
 * of cslbm_conserved_f64, same kernels and reduction order (bitwise equal
 * results), written to totals, a caller-owned DEVICE array of 5 doubles, on
 * the stream without synchronising.  The per-block partials live in a
 * library-held device array of 1024 x 6 doubles (48 KiB) per GPU, kept until
 * the process ends; the reduction grid is fixed, so every level size fits.
 * Calls no allocator.  Every call on one GPU shares that array: calls that
 * overlap in time on one GPU (different streams or threads) race.  The
 * current device must be the one the stream and the level belong to.
 * Errors: CSLBM_ERR_ARG for a bad level or NULL totals, CSLBM_ERR_HIP if the
 * scratch address cannot be looked up or a launch fails. */
int cslbm_conserved_f64_noalloc(const cslbm_level* L, double* totals, hipStream_t stream);

/* Count NaN/Inf values in L->f (and L->g).  *n_bad is a HOST int64.
 * Returns CSLBM_ERR_NONFINITE when the count is non-zero; synchronises. */
int cslbm_check_finite(const cslbm_level* L, int64_t* n_bad, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Continuous scales (sections "Mapping distribution functions",
 * "Spatial scale mapping", "Temporal alignment and scale mapping",
 * "Handling multiple scales", Algorithm 1).
 *
 * Every scale is a cslbm_level whose lattice point (x, y, z) sits at the
 * physical position origin + (x, y, z) * dx.  Its parameters are in its own
 * lattice units: a scale with spacing dx_i = dx_0 / alpha_i carries
 * nu_i = alpha_i nu_0 (invariant local Reynolds number, eq. S_relation).
 * ---------------------------------------------------------------------- */

/* Post-collision mapping from scale `src` onto the listed cells of scale
 * `dst` (eq. s1_to_s2_mapping with the trilinear interpolation of section
 * "Spatial scale mapping"):
 *   1. the source state at time weight w is (1 - w) fA + w fB (fB may be
 *      NULL when w == 0);
 *   2. it is interpolated trilinearly from the 8 corners of the source cell
 *      containing the target point (periodic wrap on periodic source axes);
 *   3. f~dst = T(m^eq + K^ m~neq) with K^ = (I - S^dst) K (I - S^src)^-1,
 *      K = S^src / (alpha S^dst) on the stress moments m4..m8 and 1 on every
 *      other moment; alpha = src->dx / dst->dx.
 * The scalar (gA and g_out non-NULL) is interpolated the same way and its
 * non-equilibrium part scaled by (tau_dst - 1) / (alpha (tau_src - 1)).
 * fA/fB/gA/gB use src's storage and plane stride; f_out/g_out use dst's.
 * cells: device int32 list of n_cells distinct dst cells; every stencil must
 * lie inside the source box on non-periodic axes (the caller's lists are
 * trusted; out-of-box corners are clamped, never read out of bounds).
 * Errors: CSLBM_ERR_ARG for NULL buffers, w outside [0, 1], a source
 * relaxation time of exactly 1 (singular (I - S)^-1). */
int cslbm_exchange(const cslbm_level* src, const void* fA, const void* fB, const float* gA,
                   const float* gB, double w, const cslbm_level* dst, void* f_out, float* g_out,
                   const int32_t* cells, int32_t n_cells, hipStream_t stream);

/* Quadratic Lagrange interpolation in time of three states of level L at
 * times t[0..2] (distinct), evaluated at t_eval, into out (and g_out from
 * g0..g2 when all are non-NULL); every plane element of every cell
 * (section "Temporal alignment and scale mapping"). */
int cslbm_time_interp(const cslbm_level* L, const void* s0, const void* s1, const void* s2,
                      const float* g0, const float* g1, const float* g2, const double t[3],
                      double t_eval, void* out, float* g_out, hipStream_t stream);

#define CSLBM_MAX_SCALES 8

/* One scale of a hierarchy.  level.f holds the scale's state at the current
 * reference time (read and written); level.f_next and work_f[0..1] (and the
 * scalar counterparts) are work space of the same size.  Scale 0 is the
 * reference scale: parent -1, no work buffers or lists needed. */
typedef struct cslbm_scale {
    cslbm_level level;
    void* work_f[2];                    /* [27][plane] each (finer scales) */
    float* work_g[2];                   /* [7][plane] each when level.g != NULL */
    int32_t parent;                     /* nearest coarser scale, or -1 */
    int32_t n_ghost;
    const int32_t* ghost_cells;         /* device: this scale's boundary cells
                                           (CSLBM_GHOST), written by prior-mapping */
    int32_t n_post[CSLBM_MAX_SCALES];
    const int32_t* post_cells[CSLBM_MAX_SCALES];  /* device: cells of coarser scale j
                                                     written by post-mapping */
    int32_t n_ghost_xlo, n_ghost_xhi;   /* the first n_ghost_xlo entries of
                                           ghost_cells lie on the plane x =
                                           ghost_xlo, the next n_ghost_xhi on
                                           x = ghost_xhi (0, 0: no such order) */
    int32_t ghost_xlo, ghost_xhi;       /* x indices of the two planes of the
                                           boundary shell normal to x (a box
                                           padded along x has its shell inside
                                           the box) */
    void* stage;                        /* device work space of
                                           cslbm_stage_bytes(parent, level,
                                           ghost_xlo, ghost_xhi) bytes, or
                                           NULL: with it (and the
                                           x-face counts above) the prior-
                                           mapping of the x-face ghosts reads a
                                           compact copy of the parent's few
                                           columns around each face, made once
                                           per reference step, instead of one
                                           cache line per parent row */
    int64_t stage_bytes;
    const int32_t* post_tiles[CSLBM_MAX_SCALES];  /* device, or NULL: post_cells[j]
                                           grouped into n_post_tiles[j] runs of
                                           consecutive entries, run t from entry
                                           post_tiles[j][t] to post_tiles[j][t+1]
                                           - 1 (n_post_tiles[j] + 1 ascending
                                           offsets, 0 first, n_post[j] last, at
                                           most 256 entries a run; a run outside
                                           these bounds is clipped to them).  When
                                           both scales are dense boxes, scale i
                                           has no periodic axis and scale j's
                                           cells are not all lattice points of
                                           scale i, each run is mapped by one
                                           workgroup that reads the scale-i cells
                                           its stencils reach once into LDS; with
                                           runs that are tiles of neighbouring
                                           cells (a few rows of one plane) that
                                           reads far fewer bytes than gathering
                                           every target's 8 corners.  The result
                                           is the same bit for bit. */
    int32_t n_post_tiles[CSLBM_MAX_SCALES];
    const int32_t* ghost_tiles;         /* device, or NULL: ghost_cells grouped
                                           into n_ghost_tiles runs of
                                           consecutive entries, run t from
                                           entry ghost_tiles[t] to
                                           ghost_tiles[t+1] - 1 (n_ghost_tiles
                                           + 1 ascending offsets, 0 first,
                                           n_ghost last, at most 256 entries a
                                           run; clipped to the list as above;
                                           a run that starts among the x-face
                                           entries of one plane must hold only
                                           entries of that plane, or its
                                           targets become NaN).  When this
                                           scale and its parent are dense boxes,
                                           the parent has no periodic axis and
                                           this scale's cells are not all
                                           parent lattice points, the prior-
                                           mapping (and its adjoint in
                                           cslbm_multiscale_adjoint_step) maps
                                           each run with one workgroup through
                                           LDS, as post_tiles does (x-face runs
                                           from the staged copies when there
                                           are any): with
                                           runs that are patches of one face of
                                           the shell the parent's cells are
                                           read once per patch instead of once
                                           per corner of every target.  The
                                           result is the same bit for bit. */
    int32_t n_ghost_tiles;
} cslbm_scale;

typedef struct cslbm_hierarchy {
    int32_t n_scales;                   /* 1..CSLBM_MAX_SCALES */
    int32_t reserved;
    cslbm_scale* scales;                /* HOST array of n_scales scales */
} cslbm_hierarchy;

/* n_ref_steps reference steps of Algorithm 1.  Per reference step:
 *   - scale 0 takes one step (its states at t_n and t_n + dt_0 stay in
 *     level.f_next and level.f);
 *   - with it, each far-field scale i (level.dx > scale 0's dx; alpha_i =
 *     dx_0 / dx_i < 1; parent 0; section "Temporal alignment and scale
 *     mapping" and the reversed rules of "Handling multiple scales"), in
 *     index order: its ghost cells (the whole region it shares with scale 0)
 *     are mapped from scale 0 at t_n; it takes one step of dt_i = dt_0 /
 *     alpha_i and is interpolated linearly back to t_n + dt_0,
 *     (1 - alpha_i) f(t_n) + alpha_i f(t_n + dt_i); its ghost cells are
 *     mapped again at t_n + dt_0; then post_cells[0] (scale 0's boundary
 *     shell, CSLBM_GHOST cells of scale 0) are mapped from it.  Its outer
 *     faces are normally CSLBM_NEUMANN cells;
 *   - then each finer scale i (in index order) with alpha_i = dx_0 / dx_i
 *     takes l = floor(alpha_i) + 1 sub-steps; before sub-step k < l its
 *     ghost cells are prior-mapped from the parent blended between its
 *     states at t_n and t_n + dt_0 with weight (k - 1) / alpha_i (the
 *     sub-step's start time), and before the final sub-step k = l from the
 *     parent at t_n + dt_0 (weight 1); the result is interpolated in time
 *     by the quadratic through 0, (l - 1)/alpha_i, l/alpha_i evaluated at 1;
 *     the ghosts are mapped again at weight 1; then the scale is post-mapped
 *     onto post_cells[j] of every larger scale j (j < i, or a far-field
 *     scale), in index order (at integer alpha_i the quadratic's weight on
 *     sub-step l is exactly 0 and that sub-step is not computed; the result
 *     is the same);
 *   - the interpolated states become the scales' level.f (pointer swap with
 *     work_f[1] / work_g[1]).
 * Every scale but scale 0 needs flags with CSLBM_GHOST cells; every scale
 * must carry the scalar or none; a finer scale's parent is never a far-field
 * scale.  Errors: CSLBM_ERR_ARG for an inconsistent hierarchy (parents,
 * spacings, buffers, lists, singular relaxation times). */
int cslbm_multiscale_step(cslbm_hierarchy* H, int32_t n_ref_steps, hipStream_t stream);

/* Bytes of the x-face staging work space (cslbm_scale.stage) of a finer
 * scale `level` whose parent is `parent` and whose boundary shell has its
 * planes normal to x at x = x_lo and x = x_hi: for each plane, the parent's
 * populations (and scalar) at both time levels over the columns and rows
 * the plane's trilinear stencils reach, with one cell of margin.  0 when
 * staging does not apply (a brick level on either side, or a stencil region
 * that wraps around a periodic parent axis or leaves the parent); negative
 * on invalid arguments.  The copy changes only where the prior-mapping
 * reads its corners: results are bitwise those of the unstaged mapping. */
int64_t cslbm_stage_bytes(const cslbm_level* parent, const cslbm_level* level, int32_t x_lo,
                          int32_t x_hi);

/* ------------------------------------------------------------------------
 * Differentiation (build addition; the paper has no adjoint).
 * ---------------------------------------------------------------------- */

/* n_steps forward steps that keep every state: step k reads (k == 0 ? L->f :
 * f_states[k-1]) and writes f_states[k] (likewise g from L->g into
 * g_states).  L->f and L->g are not modified.  f_states / g_states are HOST
 * arrays of n_steps DEVICE buffers of L's size; used to recompute a
 * checkpointed segment for the adjoint. */
int cslbm_step_store(const cslbm_level* L, int32_t n_steps, void* const* f_states,
                     float* const* g_states, hipStream_t stream);

/* Adjoint of one step (eq. lbe with eq. cmr_collision, the body force and
 * the scalar): with L->f (and L->g, L->force) the state f(n) that the
 * forward step read, lam_next = dL/df(n+1) [27][plane] and mu_next =
 * dL/dg(n+1) [7][plane], writes lam = dL/df(n) and mu = dL/dg(n) and adds
 * dL/dtheta to dtheta [3][plane] (may be NULL).  Adjoints are FP32 and refer
 * to the physical populations (a shift by w_i does not change them).  A
 * level without flags must be fully periodic (CSLBM_ERR_UNSUPPORTED
 * otherwise).  With flags: solid and inlet outputs do not depend on the
 * state; ghost, outflow and Neumann cells copy their source cell (identity
 * Jacobian); lam and mu are overwritten everywhere (zero where no output
 * depends on an element).  Non-smooth points of the adaptive factor take the
 * derivative of the branch they are on. */
int cslbm_adjoint_step(const cslbm_level* L, const float* lam_next, const float* mu_next,
                       float* lam, float* mu, float* dtheta, hipStream_t stream);

/* Adjoint of cslbm_exchange (sections "Spatial scale mapping" and
 * "Temporal alignment and scale mapping"): with the forward arguments (src,
 * fA, fB, gA, gB, w, dst, cells), lam_d [27][dst plane] (mu_d [7][..]) holds
 * dL/d(destination after the exchange); the listed cells' entries are routed
 * to the source states and then set to 0 (the exchange overwrote them):
 * lam_a += (1 - w) J^T lam_d and lam_b += w J^T lam_d (J the trilinear
 * interpolation followed by the central-moment rescaling of the target
 * state), likewise mu_a / mu_b.  A time level of weight 0 is not read or
 * touched and may be NULL.  FP32 source states only (CSLBM_ERR_UNSUPPORTED).
 * workspace NULL: targets sharing source corners are summed with atomic adds
 * (summation order not reproducible).  workspace DEVICE of at least
 * cslbm_exchange_adjoint_bytes(src, dst, n_cells) bytes (caller-owned,
 * contents overwritten): the gather form, where each source cell sums its
 * targets' contributions itself (reproducible; targets whose stencil wraps
 * or is clamped at the source faces still use atomic adds). */
int cslbm_exchange_adjoint(const cslbm_level* src, const void* fA, const void* fB, const float* gA,
                           const float* gB, double w, const cslbm_level* dst, float* lam_d,
                           float* mu_d, float* lam_a, float* lam_b, float* mu_a, float* mu_b,
                           const int32_t* cells, int32_t n_cells, void* workspace,
                           int64_t workspace_bytes, hipStream_t stream);

/* Workspace bytes of the gather form of cslbm_exchange_adjoint for n_cells
 * targets (a [34][n_cells] FP32 buffer, an int32 index map of the
 * destination box and a byte flag per source cell); -1 for NULL levels or a
 * negative count. */
int64_t cslbm_exchange_adjoint_bytes(const cslbm_level* src, const cslbm_level* dst, int32_t n_cells);

/* Workspace bytes that cslbm_multiscale_adjoint_step needs for H (the input
 * of every sub-step, the interpolated states and adjoint temporaries of all
 * scales), or -1 if H is not supported (message in cslbm_last_error). */
int64_t cslbm_multiscale_adjoint_bytes(const cslbm_hierarchy* H);

/* Adjoint of one reference step of cslbm_multiscale_step (Algorithm 1:
 * reference step, prior-mapping of each finer scale's ghost shell at the
 * sub-step times, sub-steps with the quadratic time interpolation, ghost
 * remap at weight 1, post-mapping into every coarser scale).
 *   f_in[i], g_in[i]  DEVICE states of scale i at t_n (HOST arrays of
 *                     n_scales pointers; g_in NULL without scalar).  The
 *                     GHOST cells of the finer scales' states are rewritten
 *                     with their prior-mapped values, as the forward step
 *                     does (their old values never enter the step); all
 *                     other elements are read only
 *   lam[i], mu[i]     in: dL/d(state of scale i at t_n + dt_0) [27|7][plane];
 *                     out: dL/d(state of scale i at t_n) (the elements of a
 *                     plane past its nx*ny*nz cells are no part of it and
 *                     are left unspecified)
 *   workspace         DEVICE, at least cslbm_multiscale_adjoint_bytes(H)
 * The forward step is recomputed from f_in into the workspace (the level
 * structs' own f / f_next / work buffers are not touched), the flags, lists,
 * force and parameters of H are used as in the forward step.  Supported:
 * FP32 storage, finer scales only (no far-field scale), every finer scale's
 * parent is the next coarser one (scale i's parent is i - 1); the force
 * field is held fixed (no dL/dtheta).  The exchange adjoints use the gather
 * form of cslbm_exchange_adjoint in the workspace (reproducible except for
 * targets whose stencil wraps at a periodic face).
 * Errors: CSLBM_ERR_UNSUPPORTED outside that scope, CSLBM_ERR_ARG for NULL
 * buffers or a short workspace, and the checks of cslbm_multiscale_step. */
int cslbm_multiscale_adjoint_step(const cslbm_hierarchy* H, const void* const* f_in,
                                  const float* const* g_in, float* const* lam, float* const* mu,
                                  void* workspace, int64_t workspace_bytes, hipStream_t stream);

/* sizeof(cslbm_params), sizeof(cslbm_level) and sizeof(cslbm_scale) as
 * compiled into the library (HOST pointers, each may be NULL), so that
 * bindings can verify their struct layout before the first call.  Always
 * CSLBM_OK. */
int cslbm_abi_sizes(int64_t* params_bytes, int64_t* level_bytes, int64_t* scale_bytes);

/* Message of the last failed call on this thread ("" if none). */
const char* cslbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CSLBM_H */
