/* Cell-centred multigrid solver and elliptic divergence cleaning for
 * MI355X (gfx950): C ABI.
 *
 * Cheong et al., "Gmunu" (arXiv 2012.07322), section 2.7 (non-linear
 * cell-centred multigrid: 3/5/7-point second-order operators, red-black
 * Newton-Gauss-Seidel smoothing, the same relaxation as the coarsest-level
 * solver, piecewise-constant restriction, Kwak prolongation) and section 2.2
 * (elliptic divergence cleaning).  The scalar equation solved is
 *     L(u) = Lap(u) - a (u + c)^p - a2 (u + c)^q = f,   p in {-1, 0, 1},
 * where Lap is the Laplacian of the flat reference metric in Cartesian,
 * cylindrical (R, z, phi) or spherical (r, theta, phi) coordinates.  The
 * scalar metric equations of section 2.6 in deviation form have this form
 * (conformal factor: p = -1, q = -7, c = 1, a = -2 pi U~,
 * a2 = -A~_ij A~^ij / 8, f = 0; lapse: p = 1 for u = alpha psi - 1), and so
 * has the Poisson equation of the cleaning (a = a2 = 0).  The vector
 * equation of the xCFC potential X and of the shift (section 2.6),
 *     L(X)^i = Lap X^i + (1/3) d_i d_j X^j = f^i,
 * is solved on Cartesian grids and on axisymmetric cylindrical (R, z) and
 * spherical (r, theta) grids in orthonormal components (second differences,
 * the four-point mixed difference of section 2.7 and the connection terms
 * of the reference metric; Newton-Gauss-Seidel over 2^ndim colours, or line
 * relaxation).
 *
 * Arrays: FP64 device memory, one ghost layer on each active axis, layout
 * [k][j][i] with i fastest: n[a] + 2 entries along an active axis, 1 along
 * an inactive one.  Vector fields are three such arrays back to back.  Ghost
 * entries of inputs are ignored; those of a solution are written from the
 * boundary conditions.  All calls are asynchronous on `stream` (NULL: the
 * default stream) unless stated; errors as in gmunu.h (GMUNU_E*).
 */
#ifndef GMUNU_MG_H
#define GMUNU_MG_H

#include "gmunu.h"

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GMUNU_MG_DIRICHLET = 0, /* u = 0 on the face */
  GMUNU_MG_NEUMANN = 1,   /* zero normal derivative (also: faces of zero area) */
  GMUNU_MG_PERIODIC = 2,
  GMUNU_MG_ROBIN = 3      /* d(r u)/dr = 0 (section 2.6): the outer r face (axis 0) of spherical grids, the R
                             and z faces of cylindrical ones (u + R du/dR + z du/dz = 0), any face of Cartesian
                             ones (u + x.grad u = 0); ghost value u_in r_in / r_ghost with r the distance of the
                             cell centres from the origin, exact for a 1/r fall-off */
};

typedef struct {
  int ndim;          /* 1..3 */
  int coord;         /* GMUNU_CART, GMUNU_CYL, GMUNU_SPH */
  int n[3];          /* interior cells of the finest level; inactive axes 1 */
  double xmin[3];    /* lower face coordinate per axis */
  double dx[3];      /* finest spacing per axis */
  int bc[3][2];      /* GMUNU_MG_* per axis and side */
  int levels;        /* levels in the hierarchy; 0: as many as the axes allow (see gmunu_mg_create) */
  int pre, post;     /* smoothing sweeps before and after the coarse correction (>= 0) */
  int coarse;        /* sweeps on the coarsest level (>= 1) */
  int power;         /* p: -1, 0 or 1 */
  double offset;     /* c */
  int power2;        /* q of the second term, -8..8; 0: no second term (a2 must be NULL) */
  int smoother;      /* GMUNU_MG_POINT or GMUNU_MG_LINE */
} gmunu_mg_desc;

/* Smoothers.  POINT: red-black Newton-Gauss-Seidel, one cell at a time
 * (section 2.7).  LINE: alternating zebra line relaxation, for the grids on
 * which section 2.7 notes that point smoothers converge slowly (spherical
 * polar cells, whose aspect r dtheta / dr runs from far below to far above
 * one): a sweep takes each active non-periodic axis in turn and relaxes
 * whole lines of cells along it, lines coloured by the parities of their
 * transverse indices and one colour after the other; each line takes one
 * Newton step of the equation with the couplings along the line solved
 * exactly (a tridiagonal system, parallel cyclic reduction, the face ghosts
 * at its two ends folded into the boundary cells through the boundary
 * rule) and the transverse neighbours held at their current values.  The
 * vector equations relax the components of a line one after the other.
 * Lines may be at most 1024 cells long (longer non-periodic axes: EINVAL);
 * with every active axis periodic LINE relaxes points.  The line systems
 * must be non-singular: a problem with no Dirichlet or Robin face, a = 0
 * and one active axis is not. */
enum { GMUNU_MG_POINT = 0, GMUNU_MG_LINE = 1 };

typedef struct gmunu_mg gmunu_mg;

/* Validate (each active n divisible by 2^(levels-1), at least 2 cells per
 * axis on the coarsest level and an even number on periodic axes, Robin
 * only where GMUNU_MG_ROBIN allows it,
 * fewer than 2^31 entries per array),
 * build the level hierarchy on the current device and allocate its arrays
 * (5 arrays per coarse level, 6 with power2 != 0; 1 on the finest; the
 * vector equations add 12 per coarse level on their first use).
 * Synchronous. */
int gmunu_mg_create(const gmunu_mg_desc *desc, gmunu_mg **out);
int gmunu_mg_destroy(gmunu_mg *mg);
/* Levels actually used. */
int gmunu_mg_levels(const gmunu_mg *mg);
/* Entries of one array of level l (l = levels - 1 is the finest). */
long gmunu_mg_size(const gmunu_mg *mg, int level);

/* Solve L(u) = f on the finest level in place (with the point smoother, on
 * a large finest level the first call allocates colour-split copies of f,
 * a and a2 that the red-black sweeps read): an FAS full-multigrid cycle
 * from the current u first when fmg != 0, then FAS V-cycles until
 * max |f - L(u)| <= tol or max_cycles cycles were done (the FMG cycle
 * counts as one).  a and a2 may be NULL (zero); a2 needs power2 != 0
 * (else EINVAL).  res_host (max_cycles + 1 doubles, nullable) receives the
 * residual norm before and after each cycle; *cycles_out the cycles done.
 * Synchronises `stream` once per cycle to read the norm.  The V-cycle is
 * replayed from a graph captured for the arrays (u, f, a, a2) of the call;
 * four such graphs are kept per hierarchy. */
int gmunu_mg_solve(gmunu_mg *mg, double *u, const double *f, const double *a, const double *a2, double tol,
                   int max_cycles, int fmg, double *res_host, int *cycles_out, void *stream);
/* max |f - L(u)| on the finest level (boundary rule inline).  Synchronous. */
int gmunu_mg_residual_norm(gmunu_mg *mg, double *u, const double *f, const double *a, const double *a2,
                           double *norm_out, void *stream);

/* Building blocks (finest level unless a level is given), for checking:
 * out = L(u) on the interior with u's ghosts as given; ghost fill; `sweeps`
 * sweeps of the descriptor's smoother (red-black: on a large finest level f,
 * a and a2 are first copied into colour-split buffers of the hierarchy, as
 * in the solve; line relaxation), then the ghost fill; restriction
 * of level l into level l - 1 (volume-weighted mean of children); Kwak
 * prolongation of level l - 1 (ghosts as given) into level l. */
int gmunu_mg_apply(gmunu_mg *mg, const double *u, const double *a, const double *a2, double *out, void *stream);
int gmunu_mg_fill_ghosts(gmunu_mg *mg, int level, double *u, void *stream);
int gmunu_mg_smooth(gmunu_mg *mg, double *u, const double *f, const double *a, const double *a2, int sweeps,
                    void *stream);
int gmunu_mg_restrict(gmunu_mg *mg, int level, const double *fine, double *coarse, void *stream);
int gmunu_mg_prolong(gmunu_mg *mg, int level, const double *coarse, double *fine, void *stream);

/* Divergence cleaning (section 2.2) of a vector field q (three arrays):
 * div = (1/sqrt g) d_i (sqrt g q^i) by centred differences (q's ghosts must
 * be set), then Lap(Phi) = div solved like gmunu_mg_solve (phi: initial
 * guess in, solution out; the descriptor's power must be 0 and a = 0), then
 * q^i -= g^ii d_i Phi (centred) on the interior.  div (nullable) receives
 * the divergence before cleaning.  Needs p = 0. */
int gmunu_mg_divergence(gmunu_mg *mg, const double *q, double *div, void *stream);
int gmunu_mg_subtract_gradient(gmunu_mg *mg, const double *phi, double *q, void *stream);
int gmunu_mg_clean(gmunu_mg *mg, double *q, double *phi, double *div, double tol, int max_cycles, double *res_host,
                   int *cycles_out, void *stream);

/* The same cleaning applied to a GRMHD state (layout of include/gmunu.h)
 * whose descriptor `hydro` has the multigrid's finest grid as its interior:
 * q_B = q[5..7] (interior; the ghost layer from psi^6 times the primitive
 * field, so prim's ghosts must be filled) is cleaned and written back to the
 * interior of q.  The caller then recovers the primitives (gmunu_c2p) and
 * fills their ghosts, as after any update of q.  Scratch of six finest-level
 * arrays is allocated on the first call.  Needs p = 0. */
int gmunu_mg_clean_state(gmunu_mg *mg, const gmunu_grid_desc *hydro, double *q, const double *prim,
                         const double *metric, double tol, int max_cycles, double *res_host, int *cycles_out,
                         void *stream);

/* The scalar CFC metric equations of section 2.6 solved for a GRMHD state
 * (steps 3 and 5 of the xCFC sequence, with the vector potential X and the
 * shift left as they are, i.e. A^ij = 0: exact for static configurations):
 *   Lap(psi - 1) = -2 pi U~ / psi,          U~ = q_tau + q_D,
 *   Lap(alpha psi - 1) = alpha psi 2 pi (U~ + 2 S~) / psi^2,
 *   S~ = psi^6 (rho h W^2 v^2 + 3 p) (fluid part, from prim and the new psi).
 * mpsi must have p = -1, c = 1 and malpha p = 1, c = 1, both on the
 * interior grid of `hydro` (boundary conditions: Robin on the outer radial
 * face, as section 2.6 prescribes, for spherical grids).  Starts from the
 * metric's psi and alpha; writes psi and alpha (metric variables 0 and 1) to
 * every cell of the GRMHD layout, ghost layers extended by the multigrid
 * boundary rule applied per layer.  cycles_out (2 ints, nullable): cycles of
 * each solve. */
int gmunu_mg_cfc_solve(gmunu_mg *mpsi, gmunu_mg *malpha, const gmunu_grid_desc *hydro, const double *q,
                       const double *prim, double *metric, double tol, int max_cycles, int *cycles_out,
                       void *stream);

/* Vector equation L(X) = f of section 2.6 on Cartesian grids, and on
 * cylindrical and spherical grids with at most two active axes
 * (axisymmetric: d/dphi = 0) in orthonormal components (X^R, X^z, X^phi;
 * X^r, X^theta, X^phi).  EINVAL for Robin faces, for curvilinear grids with
 * three active axes, and for spherical grids reaching r = 0 unless theta
 * is active and ends at pi/2 (equatorial symmetry); the descriptor's
 * power, offset and power2 are not used.  X and f: three arrays back to
 * back.  Values across the boundary come from each axis's rule with
 * per-component parity: Dirichlet faces flip every component, symmetry
 * (Neumann) faces the normal one, and the cylindrical axis and polar axis
 * also the phi component, the spherical centre every component; ghost
 * entries of X are not read.  vapply: out = L(X) on the interior.
 * vsmooth: `sweeps` sweeps of the descriptor's smoother (the 2^ndim
 * colours, or line relaxation), then X's ghosts filled.  vsolve: as
 * gmunu_mg_solve (per-component maximum norm); X's ghosts filled on
 * return.  The first vector call allocates the coarse levels' vector
 * arrays. */
int gmunu_mg_vapply(gmunu_mg *mg, const double *X, double *out, void *stream);
int gmunu_mg_vsmooth(gmunu_mg *mg, double *X, const double *f, int sweeps, void *stream);
int gmunu_mg_vsolve(gmunu_mg *mg, double *X, const double *f, double tol, int max_cycles, int fmg, double *res_host,
                    int *cycles_out, void *stream);

/* Section 2.6: A~^ij = D_i X^j + D_j X^i - (2/3) gamma^ij D_k X^k of the flat
 * reference metric, by centred differences (values across the boundary by
 * the vector rules) plus the connection terms in curvilinear coordinates,
 * on the interior, in orthonormal components as six arrays (11, 22, 33,
 * 12, 13, 23; Cartesian xx, yy, zz, xy, xz, yz) in A6, and A~_ij A~^ij in
 * A2.  Grids as for the vector equation. */
int gmunu_mg_xcfc_aij(gmunu_mg *mg, const double *X, double *A6, double *A2, void *stream);
/* Source of the shift equation, 16 pi w S_i + 2 A~^ij d_j w with
 * w = alpha psi^-6 (centred gradient from w's stored ghost entries, in
 * orthonormal components on curvilinear grids), S = S~_i (three arrays,
 * orthonormal), A6 as above; out: three arrays, interior. */
int gmunu_mg_xcfc_beta_rhs(gmunu_mg *mg, const double *w, const double *S, const double *A6, double *out,
                           void *stream);

/* The xCFC metric solve of section 2.6 (steps 1 to 6) for a GRMHD state on a
 * grid the vector equation accepts: X from L(X) = 8 pi S~_i (S~_i = q_{S_i},
 * covariant, divided by the scale factor h_i on curvilinear grids to give
 * orthonormal components; X in/out: initial guess and solution, three
 * multigrid arrays of mvec, orthonormal), A~^ij from X, psi
 * from its equation with both terms (mpsi: p = -1, q = -7, c = 1), S~ with
 * the new psi as in gmunu_mg_cfc_solve, alpha psi (malpha: p = 1, c = 1,
 * its coefficient with the (7/8) A~_ij A~^ij psi^-8 term), then the shift
 * from L(beta) = 16 pi alpha psi^-6 S~_i + 2 A~^ij d_j(alpha psi^-6)
 * starting from the metric's shift.  psi, alpha and the contravariant
 * coordinate components beta^i = beta^(i) / h_i (metric variables 0..4)
 * are written to every cell of the GRMHD layout, ghost layers extended by
 * the boundary rules (per-component parity for the shift).  mvec, mpsi
 * and malpha: hierarchies on the interior grid of `hydro` (mvec without
 * Robin faces: X = beta = 0 on outer Dirichlet faces).  cycles_out (4 ints,
 * nullable): cycles of the X, psi, alpha psi and beta solves.  Scratch of
 * 17 finest arrays is allocated in mvec on the first call. */
int gmunu_mg_xcfc_solve(gmunu_mg *mvec, gmunu_mg *mpsi, gmunu_mg *malpha, const gmunu_grid_desc *hydro,
                        const double *q, const double *prim, double *metric, double *X, double tol, int max_cycles,
                        int *cycles_out, void *stream);

/* max |L(psi - 1)| of the conformal-factor equation of section 2.6 with the
 * current metric and the state's conserved variables (U~ = q_tau + q_D;
 * with mvec and X the A~_ij A~^ij psi^-7 term from X as well):
 * the constraint residual that decides when the metric is re-solved during
 * an evolution (section 2.6, frequency of solving the metric).  mpsi: p =
 * -1, c = 1 (q = -7 with mvec).  Synchronous. */
int gmunu_mg_psi_residual(gmunu_mg *mvec, gmunu_mg *mpsi, const gmunu_grid_desc *hydro, const double *q,
                          const double *metric, const double *X, double *norm_out, void *stream);

/* A metric update inside a GRMHD evolution (lifting the frozen-metric
 * restriction, section 2.6 with the recovery of section 2.5): the metric
 * re-solved from the state's conserved variables -- the xCFC sequence of
 * gmunu_mg_xcfc_solve when mvec is given (X in/out), else
 * the scalar equations of gmunu_mg_cfc_solve (shift unchanged) -- then
 * gmunu_c2p of q on the new metric (q corrected where the recovery says so,
 * flags and nfatal_dev as there) and gmunu_fill_ghosts of prim.  ctx and
 * hydro describe the same grid (the context's and the descriptor it was
 * created from).  cycles_out (4 ints, nullable): cycles of the X, psi,
 * alpha psi and beta solves (0 for those not run). */
int gmunu_mg_metric_update(gmunu_mg *mvec, gmunu_mg *mpsi, gmunu_mg *malpha, gmunu_ctx *ctx,
                           const gmunu_grid_desc *hydro, double *q, double *prim, double *metric, double *X,
                           uint8_t *flags, unsigned int *nfatal_dev, double tol, int max_cycles, int *cycles_out,
                           void *stream);

/* Up to nsteps GRMHD steps on the current metric, as an evolution with a
 * dynamical metric takes them between re-solves (section 2.6, frequency of
 * solving the metric): each step is gmunu_step (K_ij from the shift) followed
 * by the conformal-factor residual of gmunu_mg_psi_residual, both on the
 * device.  After the first step whose residual exceeds eps the remaining
 * steps of the call change nothing (their dt is 0; *t_dev is restored at
 * the end), so the states equal those of the loop that checks the residual
 * on the host after every step and stops at the first trigger -- with one
 * host synchronisation per call instead of one per step.  *steps_out: the
 * steps taken (the trigger step when *triggered_out is 1, else nsteps).
 * t_end must be finite; t_dev and dt_dev are required.  The caller then
 * re-solves the metric (gmunu_mg_metric_update) when triggered or when its
 * step count since the last re-solve is reached.  Synchronous; the step
 * and residual arguments as for gmunu_step and gmunu_mg_psi_residual. */
int gmunu_mg_dynamical_steps(gmunu_mg *mvec, gmunu_mg *mpsi, gmunu_ctx *ctx, const gmunu_grid_desc *hydro,
                             double *q_n, double *q_s, double *prim, const double *metric, const double *X,
                             double cfl, double t_end, double *t_dev, double *dt_dev, uint8_t *flags,
                             unsigned int *nfatal_dev, int nsteps, double eps, int *steps_out, int *triggered_out,
                             void *stream);

#ifdef __cplusplus
}
#endif

#endif
