/*
 * Gmunu GRMHD finite-volume step -- CPU ORACLE (test infrastructure only).
 *
 * This file is the slow, plain, obviously-correct FP64 statement of what the
 * GPU path computes.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  The GPU library never links, includes or
 * calls anything here, and this file includes nothing from the GPU library.
 *
 * Source: Cheong, Lam, Ng, Li et al., "Gmunu: paralleled, grid-adaptive,
 * general-relativistic magnetohydrodynamics in curvilinear geometries in
 * dynamical space-times" (arXiv 2012.07322).  Every function cites the section
 * or equation it follows.  Where the paper is silent or garbled, the reading
 * taken is stated at the spot (and listed in the design notes).
 *
 * Conventions
 *   - Arrays are structure-of-arrays [var][k][j][i], i fastest, including
 *     ghost cells: nt[a] = n[a] + 2*g[a], g[a] = ng on active axes, 0 else.
 *   - prim = (rho, W v^1, W v^2, W v^3, p, B^1, B^2, B^3)  (contravariant,
 *     coordinate basis, B undensitised).
 *   - q    = psi^6 (D, S_1, S_2, S_3, tau, B^1, B^2, B^3)  (S covariant).
 *   - metric = (psi, alpha, beta^1, beta^2, beta^3) at cell centres, ghosts
 *     supplied by the caller.
 *   - coordinates: 0 Cartesian (x,y,z); 1 cylindrical (R,z,phi);
 *     2 spherical (r,theta,phi).
 *
 * Every part is pinned by a test independent of this file: the
 * gravitational sources (extrinsic-curvature and shift terms included)
 * against the covariant conservation law of a stationary 4-metric, the whole
 * discrete right-hand side against a 50-digit brute-force evaluation on
 * 8-cell grids, the shift in fluxes and speeds against the translated exact
 * Riemann solution, plus the closed forms, exact solutions and conservation
 * laws listed in the tests.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NV 8

enum { RHO = 0, WV1 = 1, PRS = 4, BB1 = 5 };
enum { QD = 0, QS1 = 1, QTAU = 4, QB1 = 5 };
enum { CART = 0, CYL = 1, SPH = 2 };
enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_REFLECT = 2, BC_AXIS = 3, BC_CENTER = 4, BC_NONE = 5 };
enum {
  F_ATMO = 1, F_EPS_CLAMP = 2, F_V_CLAMP = 4, F_FATAL_RHO = 8,
  F_FATAL_EPS = 16, F_FATAL_V = 32, F_NOCONV = 64
};
#define F_FATAL_MASK (F_FATAL_RHO | F_FATAL_EPS | F_FATAL_V | F_NOCONV)

typedef struct {
  int ndim, coord, n[3], ng;
  double xmin[3], dx[3];
  int bc[3][2];
  double gamma;
  double rho_atmo, k_atmo, gamma_atmo;
  double rho_low_factor, alpha_bh;
  double rho_max, eps_max, w_max;
  int c2p_maxit;
  double c2p_tol;
  int rk;
  int recon, riemann, pp, c2p;  /* scheme options: recon 0 MC, 1 MP5, 2 PPM; riemann 0 HLLE, 1 TVDLF;
                                 pp 0 off, 1 on; c2p 0 GRMHD, 1 GRHD z-scheme */
} og_desc;

/* ------------------------------------------------------------------ grid */

static int gh(const og_desc *d, int a) { return a < d->ndim ? d->ng : 0; }
static int ntl(const og_desc *d, int a) { return d->n[a] + 2 * gh(d, a); }
static long ntot(const og_desc *d) { return (long)ntl(d, 0) * ntl(d, 1) * ntl(d, 2); }

/* linear index of cell (i,j,k); interior indices run 0..n-1, ghosts outside */
static long at(const og_desc *d, int i, int j, int k) {
  return ((long)(k + gh(d, 2)) * ntl(d, 1) + (j + gh(d, 1))) * ntl(d, 0) + (i + gh(d, 0));
}

static double centre(const og_desc *d, int a, int i) { return d->xmin[a] + (i + 0.5) * d->dx[a]; }
static double face_pos(const og_desc *d, int a, int f) { return d->xmin[a] + f * d->dx[a]; }

/* Diagonal of the reference (flat) metric at a point (Appendix A:
 * cylindrical diag(1,1,R^2), spherical diag(1,r^2,r^2 sin^2 theta)). */
static void ref_metric(int coord, double x1, double x2, double g[3]) {
  g[0] = 1.0; g[1] = 1.0; g[2] = 1.0;
  if (coord == CYL) {
    g[2] = x1 * x1;
  } else if (coord == SPH) {
    double s = sin(x2);
    g[1] = x1 * x1;
    g[2] = x1 * x1 * s * s;
  }
}

/* Cell volume Delta V = integral of sqrt(ref det) over the cell
 * (Appendix A, cylindrical and spherical cell volumes). */
static double cell_volume(const og_desc *d, int i, int j, int k) {
  double x1 = centre(d, 0, i), x2 = centre(d, 1, j);
  double d1 = d->dx[0], d2 = d->dx[1], d3 = d->dx[2];
  (void)k;
  if (d->coord == CYL) return x1 * d1 * d2 * d3;
  if (d->coord == SPH) return (x1 * x1 + d1 * d1 / 12.0) * d1 * (2.0 * sin(x2) * sin(0.5 * d2)) * d3;
  return d1 * d2 * d3;
}

/* Area of the face of index f along axis a (face between cells f-1 and f),
 * at transverse cell (i,j,k) -- the other index along a is ignored
 * (Appendix A, cylindrical and spherical cell surfaces). */
static double face_area(const og_desc *d, int a, int f, int i, int j, int k) {
  double d1 = d->dx[0], d2 = d->dx[1], d3 = d->dx[2];
  (void)k;
  if (d->coord == CART) {
    if (a == 0) return d2 * d3;
    if (a == 1) return d1 * d3;
    return d1 * d2;
  }
  if (d->coord == CYL) {
    if (a == 0) return face_pos(d, 0, f) * d2 * d3;
    double R = centre(d, 0, i);
    if (a == 1) return R * d1 * d3;
    return R * d1 * d2;
  }
  /* spherical */
  if (a == 0) {
    double rf = face_pos(d, 0, f), th = centre(d, 1, j);
    return rf * rf * (2.0 * sin(th) * sin(0.5 * d2)) * d3;
  }
  {
    double r = centre(d, 0, i);
    double radial = (r * r + d1 * d1 / 12.0) * d1;
    if (a == 1) return radial * sin(face_pos(d, 1, f)) * d3;
    return radial * (2.0 * sin(centre(d, 1, j)) * sin(0.5 * d2));
  }
}

/* ------------------------------------------------------------ point state */

/* Everything the conserved variables, fluxes and wave speeds need at one
 * point, from the primitives and the CFC metric (section 2.1, magnetic
 * four-vector and energy-momentum tensor). */
typedef struct {
  double gd[3], gu[3];           /* gamma_ii = psi^4 ref_ii and its inverse */
  double psi6, alpha, beta[3];
  double rho, p, eps, h, W;
  double vu[3], vd[3];           /* Eulerian 3-velocity */
  double Bu[3], Bd[3], Bv, B2;
  double b0, bd[3], b2;
  double rhohs, ps;              /* rho h*, p* */
  double vhat[3];                /* alpha v^i - beta^i */
} pstate;

static void point_state(double gam, const double pr[NV], double psi, double alpha,
                        const double beta[3], const double ref[3], pstate *s) {
  double psi2 = psi * psi, psi4 = psi2 * psi2;
  s->psi6 = psi4 * psi2;
  s->alpha = alpha;
  for (int i = 0; i < 3; i++) {
    s->gd[i] = psi4 * ref[i];
    s->gu[i] = 1.0 / s->gd[i];
    s->beta[i] = beta[i];
  }
  s->rho = pr[RHO];
  s->p = pr[PRS];
  double u2 = 0.0;
  for (int i = 0; i < 3; i++) u2 += s->gd[i] * pr[WV1 + i] * pr[WV1 + i];
  s->W = sqrt(1.0 + u2);
  s->Bv = 0.0;
  s->B2 = 0.0;
  for (int i = 0; i < 3; i++) {
    s->vu[i] = pr[WV1 + i] / s->W;
    s->vd[i] = s->gd[i] * s->vu[i];
    s->Bu[i] = pr[BB1 + i];
    s->Bd[i] = s->gd[i] * s->Bu[i];
    s->Bv += s->Bu[i] * s->vd[i];
    s->B2 += s->Bu[i] * s->Bd[i];
  }
  /* b^0 = W B^k v_k / alpha ; b_i = B_i / W + alpha b^0 v_i ;
   * b^2 = B^i B_i / W^2 + (B^k v_k)^2 */
  s->b0 = s->W * s->Bv / alpha;
  for (int i = 0; i < 3; i++) s->bd[i] = s->Bd[i] / s->W + alpha * s->b0 * s->vd[i];
  s->b2 = s->B2 / (s->W * s->W) + s->Bv * s->Bv;
  /* ideal gas p = (Gamma-1) rho eps (section 3.1.1) */
  s->eps = s->p / ((gam - 1.0) * s->rho);
  s->h = 1.0 + s->eps + s->p / s->rho;
  s->rhohs = s->rho * s->h + s->b2;
  s->ps = s->p + 0.5 * s->b2;
  for (int i = 0; i < 3; i++) s->vhat[i] = alpha * s->vu[i] - beta[i];
}

/* Densitised conserved variables (section 2.1, definitions of q). */
static void cons_from_state(const pstate *s, double q[NV]) {
  double D = s->rho * s->W;
  double ab0 = s->alpha * s->b0;
  q[QD] = s->psi6 * D;
  for (int j = 0; j < 3; j++) q[QS1 + j] = s->psi6 * (s->rhohs * s->W * s->W * s->vd[j] - ab0 * s->bd[j]);
  q[QTAU] = s->psi6 * (s->rhohs * s->W * s->W - s->ps - ab0 * ab0 - D);
  for (int j = 0; j < 3; j++) q[QB1 + j] = s->psi6 * s->Bu[j];
}

/* Densitised flux along direction a (section 2.1, fluxes f^i).  The
 * induction flux with j == a is identically zero and is set to zero rather
 * than evaluated as a difference of equal products. */
static void flux_from_state(const pstate *s, int a, double f[NV]) {
  double D = s->rho * s->W;
  double ab0 = s->alpha * s->b0;
  double W2 = s->W * s->W;
  double va = s->vhat[a];
  double Ba = s->Bu[a];
  f[QD] = s->psi6 * D * va;
  for (int j = 0; j < 3; j++) {
    double Sj = s->rhohs * W2 * s->vd[j] - ab0 * s->bd[j];
    double fj = Sj * va - s->alpha * s->bd[j] * Ba / s->W;
    if (j == a) fj += s->alpha * s->ps;
    f[QS1 + j] = s->psi6 * fj;
  }
  {
    double tau = s->rhohs * W2 - s->ps - ab0 * ab0 - D;
    f[QTAU] = s->psi6 * (tau * va + s->alpha * s->ps * s->vu[a] - s->alpha * ab0 * Ba / s->W);
  }
  for (int j = 0; j < 3; j++)
    f[QB1 + j] = (j == a) ? 0.0 : s->psi6 * (va * s->Bu[j] - s->vhat[j] * Ba);
}

/* Magnitudes of the terms that make up each conserved variable and each
 * flux component along a (error scale for tests; tau and its flux are
 * differences of much larger terms in cold or static gas). */
static void abs_terms_from_state(const pstate *s, int a, double Ua[NV], double Fa[NV]) {
  double D = s->rho * s->W, W2 = s->W * s->W, ab0 = fabs(s->alpha * s->b0);
  double vh = fabs(s->alpha * s->vu[a]) + fabs(s->beta[a]);
  double Ba = fabs(s->Bu[a]);
  Ua[QD] = s->psi6 * D;
  for (int j = 0; j < 3; j++) Ua[QS1 + j] = s->psi6 * (fabs(s->rhohs * W2 * s->vd[j]) + ab0 * fabs(s->bd[j]));
  Ua[QTAU] = s->psi6 * (s->rhohs * W2 + s->ps + ab0 * ab0 + D);
  for (int j = 0; j < 3; j++) Ua[QB1 + j] = s->psi6 * fabs(s->Bu[j]);
  Fa[QD] = Ua[QD] * vh;
  for (int j = 0; j < 3; j++)
    Fa[QS1 + j] = Ua[QS1 + j] * vh + s->psi6 * (fabs(s->alpha * s->bd[j] * Ba / s->W) + (j == a ? s->alpha * s->ps : 0.0));
  Fa[QTAU] = Ua[QTAU] * vh + s->psi6 * (s->alpha * s->ps * fabs(s->vu[a]) + ab0 * s->alpha * Ba / s->W);
  for (int j = 0; j < 3; j++)
    Fa[QB1 + j] = (j == a) ? 0.0
                           : s->psi6 * (vh * fabs(s->Bu[j]) + (fabs(s->alpha * s->vu[j]) + fabs(s->beta[j])) * Ba);
}

/* Bounds of the characteristic speeds along a (section 2.3). */
static void speeds_from_state(double gam, const pstate *s, int a, double *lm, double *lp) {
  double cs2 = gam * s->p / (s->rho * s->h);
  double ca2 = s->b2 / s->rhohs;
  double a2 = cs2 + ca2 - cs2 * ca2;
  double v2 = 0.0;
  for (int i = 0; i < 3; i++) v2 += s->vu[i] * s->vd[i];
  double va = s->vu[a];
  double disc = a2 * (1.0 - v2) * ((1.0 - v2 * a2) * s->gu[a] - (1.0 - a2) * va * va);
  double sq = sqrt(disc > 0.0 ? disc : 0.0);
  double den = 1.0 - v2 * a2;
  double lbm = ((1.0 - a2) * va - sq) / den;
  double lbp = ((1.0 - a2) * va + sq) / den;
  *lm = s->alpha * lbm - s->beta[a];
  *lp = s->alpha * lbp - s->beta[a];
}

/* ------------------------------------------------------------------- c2p */

typedef struct {
  double D, qq, r2, B2c, rB, rperp2B2, h0, v0sq;
  double rho_min, rho_max, eps_min, eps_max, gam;
} c2p_consts;

typedef struct {
  double chi, rbar2, qbar, vhat2, What, rho, eps;
} c2p_eval;

/* Master function of the GRMHD recovery (section 2.5.2, step 3):
 * f(mu) = mu - 1/(nu_hat + mu rbar^2), with rho and eps limited to the EOS
 * validity range inside every evaluation. */
static double c2p_f(const c2p_consts *c, double mu, c2p_eval *e) {
  double chi = 1.0 / (1.0 + mu * c->B2c);
  double rbar2 = c->r2 * chi * chi + mu * chi * (1.0 + chi) * c->rB * c->rB;
  double qbar = c->qq - 0.5 * c->B2c - 0.5 * mu * mu * chi * chi * c->rperp2B2;
  double vh2 = mu * mu * rbar2;
  if (vh2 > c->v0sq) vh2 = c->v0sq;
  double What = 1.0 / sqrt(1.0 - vh2);
  double rho = c->D / What;
  double eps = What * (qbar - mu * rbar2) + vh2 * What * What / (1.0 + What);
  if (e) { e->chi = chi; e->rbar2 = rbar2; e->qbar = qbar; e->vhat2 = vh2; e->What = What; e->rho = rho; e->eps = eps; }
  rho = fmax(fmin(c->rho_max, rho), c->rho_min);
  eps = fmax(fmin(c->eps_max, eps), c->eps_min);
  double p = (c->gam - 1.0) * rho * eps;
  double ahat = p / (rho * (1.0 + eps));
  double nuA = (1.0 + ahat) * (1.0 + eps) / What;
  double nuB = (1.0 + ahat) * (1.0 + qbar - mu * rbar2);
  double nu = nuA > nuB ? nuA : nuB;
  return mu - 1.0 / (nu + mu * rbar2);
}

/* f_a(mu) = mu sqrt(h0^2 + rbar^2(mu)) - 1 and its derivative (section 2.5.2,
 * step 2), whose root mu_+ bounds the root of the master function. */
static double c2p_fa(const c2p_consts *c, double mu, double *dfa) {
  double chi = 1.0 / (1.0 + mu * c->B2c);
  double dchi = -c->B2c * chi * chi;
  double rB2 = c->rB * c->rB;
  double rbar2 = c->r2 * chi * chi + mu * chi * (1.0 + chi) * rB2;
  double drbar2 = 2.0 * c->r2 * chi * dchi + rB2 * (chi * (1.0 + chi) + mu * dchi * (1.0 + 2.0 * chi));
  double s = sqrt(c->h0 * c->h0 + rbar2);
  if (dfa) *dfa = s + mu * drbar2 / (2.0 * s);
  return mu * s - 1.0;
}

/* Illinois (modified regula falsi) root of g on the bracket [a, b] with
 * g(a) < 0 < g(b) (Dowell & Jarratt 1971, as used in section 2.5). */
typedef double (*scalar_fn)(const void *, double);
static double fa_only(const void *c, double mu) { return c2p_fa((const c2p_consts *)c, mu, NULL); }
static double f_only(const void *c, double mu) { return c2p_f((const c2p_consts *)c, mu, NULL); }

static double illinois(const void *c, scalar_fn g, double a, double b, double tol, int maxit, int *iters, int *ok) {
  double fa = g(c, a), fb = g(c, b);
  *ok = 1;
  *iters = 0;
  if (fb == 0.0) return b;
  if (fa == 0.0) return a;
  if (fa * fb > 0.0) { *ok = 0; return fabs(fa) < fabs(fb) ? a : b; }
  for (int it = 0; it < maxit; it++) {
    double cc = b - fb * (b - a) / (fb - fa);
    double fc = g(c, cc);
    *iters = it + 1;
    if (fc == 0.0) return cc;
    if (fc * fb < 0.0) {
      a = b;
      fa = fb;
    } else {
      fa *= 0.5;
    }
    b = cc;
    fb = fc;
    if (fabs(b - a) <= tol * fabs(b)) return b;
  }
  *ok = 0;
  return b;
}

static void atmosphere_prim(const og_desc *d, double B[3], double pr[NV]) {
  pr[RHO] = d->rho_atmo;
  pr[WV1] = pr[WV1 + 1] = pr[WV1 + 2] = 0.0;
  pr[PRS] = d->k_atmo * pow(d->rho_atmo, d->gamma_atmo);
  for (int i = 0; i < 3; i++) pr[BB1 + i] = B[i];
}

/* Error handling after a recovery (section 2.5.3), shared by both schemes:
 * atmosphere below rho_min, EOS limits, the velocity limit W_max (rescaled
 * only in the low-density or black-hole region, else fatal).  capped: the
 * recovery already had to cap the velocity (z-scheme, reading of the
 * bracket when S >= tau + D), treated like W > W_max. */
static int finish_recovery(const og_desc *d, double D, double rho, double eps, double W, double vu[3],
                           const double gd[3], double alpha, double Bu[3], double pr[NV], int flags, int capped) {
  double rho_min = d->rho_atmo;
  double rho_low = d->rho_low_factor * d->rho_atmo;
  if (rho < rho_min) {
    atmosphere_prim(d, Bu, pr);
    return flags | F_ATMO;
  }
  if (rho > d->rho_max) {
    flags |= F_FATAL_RHO;
    rho = d->rho_max;
  }
  int soft = (rho < rho_low) || (alpha < d->alpha_bh);
  if (eps < 0.0) {
    eps = 0.0;
    flags |= F_EPS_CLAMP;
  }
  if (eps > d->eps_max) {
    eps = d->eps_max;
    flags |= soft ? F_EPS_CLAMP : F_FATAL_EPS;
  }
  if (capped) flags |= soft ? F_V_CLAMP : F_FATAL_V;
  if (W > d->w_max) {
    if (soft) {
      /* rescale v to v_max keeping D: rho = D / W_max, then re-limit */
      double vmax2 = 1.0 - 1.0 / (d->w_max * d->w_max);
      double v2 = 0.0;
      for (int i = 0; i < 3; i++) v2 += vu[i] * gd[i] * vu[i];
      double sc = sqrt(vmax2 / v2);
      for (int i = 0; i < 3; i++) vu[i] *= sc;
      W = d->w_max;
      rho = D / W;
      if (rho < rho_min) rho = rho_min;
      if (rho > d->rho_max) rho = d->rho_max;
      if (eps < 0.0) eps = 0.0;
      if (eps > d->eps_max) eps = d->eps_max;
      flags |= F_V_CLAMP;
    } else {
      flags |= F_FATAL_V;
    }
  }
  pr[RHO] = rho;
  for (int i = 0; i < 3; i++) pr[WV1 + i] = W * vu[i];
  pr[PRS] = (d->gamma - 1.0) * rho * eps;
  for (int i = 0; i < 3; i++) pr[BB1 + i] = Bu[i];
  return flags;
}

/* --- GRHD recovery (section 2.5.1): the z = W v root on [z_-, z_+] --- */

typedef struct {
  double D, r, q, rho_min, rho_max, eps_min, eps_max, gam;
} z_consts;

/* f(z) = z - r / h(z) with rho(z) = D / W(z), eps(z) = W q - z r +
 * z^2 / (1 + W), both limited to the EOS range inside every evaluation,
 * W(z) = sqrt(1 + z^2).  On request: W, the raw rho and eps, and the h used. */
static double z_f(const z_consts *c, double z, double *W_out, double *rho_out, double *eps_out, double *h_out) {
  double W = sqrt(1.0 + z * z);
  double rho = c->D / W;
  double eps = W * c->q - z * c->r + z * z / (1.0 + W);
  if (W_out) { *W_out = W; *rho_out = rho; *eps_out = eps; }
  rho = fmax(fmin(c->rho_max, rho), c->rho_min);
  eps = fmax(fmin(c->eps_max, eps), c->eps_min);
  double p = (c->gam - 1.0) * rho * eps;
  double a = p / (rho * (1.0 + eps));
  double h = (1.0 + eps) * (1.0 + a);
  if (h_out) *h_out = h;
  return z - c->r / h;
}
static double zf_only(const void *c, double z) { return z_f((const z_consts *)c, z, NULL, NULL, NULL, NULL); }

static int c2p_point_z(const og_desc *d, const double qc[NV], double psi, double alpha, const double ref[3],
                       double pr[NV], int *iters_out) {
  double psi2 = psi * psi, psi4 = psi2 * psi2, psi6 = psi4 * psi2;
  double gd[3], gu[3];
  for (int i = 0; i < 3; i++) { gd[i] = psi4 * ref[i]; gu[i] = 1.0 / gd[i]; }
  double D = qc[QD] / psi6, tau = qc[QTAU] / psi6;
  double Sd[3], Bu[3];
  for (int i = 0; i < 3; i++) { Sd[i] = qc[QS1 + i] / psi6; Bu[i] = qc[QB1 + i] / psi6; }
  if (iters_out) *iters_out = 0;
  if (!(D >= d->rho_atmo)) {
    atmosphere_prim(d, Bu, pr);
    return F_ATMO;
  }
  /* step 1 */
  double S2 = 0.0;
  for (int i = 0; i < 3; i++) S2 += gu[i] * Sd[i] * Sd[i];
  double S = sqrt(S2);
  z_consts c;
  c.D = D;
  c.r = S / D;
  c.q = tau / D;
  c.rho_min = d->rho_atmo;
  c.rho_max = d->rho_max;
  c.eps_min = 0.0;
  c.eps_max = d->eps_max;
  c.gam = d->gamma;
  double k = S / (tau + D);
  /* a state with k beyond the one of W = W_max (or k >= 1, no finite W)
   * is recovered with k at that limit and flagged like W > W_max */
  double kmax = sqrt(1.0 - 1.0 / (d->w_max * d->w_max));
  int capped = 0;
  if (!(k <= kmax)) {
    k = kmax;
    capped = 1;
  }
  /* step 2 */
  double zm = 0.5 * k / sqrt(1.0 - 0.25 * k * k);
  double zp = k / sqrt(1.0 - k * k);
  /* step 3 */
  int iters = 0, ok = 1, flags = 0;
  double z = illinois(&c, zf_only, zm, zp, d->c2p_tol, d->c2p_maxit, &iters, &ok);
  if (iters_out) *iters_out = iters;
  if (!ok) flags |= F_NOCONV;
  /* step 4 */
  double W, rho, eps, h;
  z_f(&c, z, &W, &rho, &eps, &h);
  double vu[3];
  for (int i = 0; i < 3; i++) vu[i] = (gu[i] * Sd[i] / D) / (h * W);
  return finish_recovery(d, D, rho, eps, W, vu, gd, alpha, Bu, pr, flags, capped);
}

/* Recovery of the primitives from the densitised conserved variables at one
 * cell (section 2.5.2 steps 1-4; with c2p = 1 the GRHD z-scheme of section
 * 2.5.1) followed by the error handling of section 2.5.3.  Returns the flag
 * bits; *iters receives the root-finder iteration count. */
int og_c2p_point(const og_desc *d, const double qc[NV], double psi, double alpha,
                 const double ref[3], double pr[NV], int *iters_out) {
  if (d->c2p == 1) return c2p_point_z(d, qc, psi, alpha, ref, pr, iters_out);
  double psi2 = psi * psi, psi4 = psi2 * psi2, psi6 = psi4 * psi2;
  double gd[3], gu[3];
  for (int i = 0; i < 3; i++) { gd[i] = psi4 * ref[i]; gu[i] = 1.0 / gd[i]; }
  double D = qc[QD] / psi6, tau = qc[QTAU] / psi6;
  double Sd[3], Bu[3];
  for (int i = 0; i < 3; i++) { Sd[i] = qc[QS1 + i] / psi6; Bu[i] = qc[QB1 + i] / psi6; }
  int flags = 0;
  if (iters_out) *iters_out = 0;
  double rho_min = d->rho_atmo;

  /* rho = D / W <= D, so D below rho_min already means rho < rho_min */
  if (!(D >= rho_min)) {
    atmosphere_prim(d, Bu, pr);
    return F_ATMO;
  }

  /* step 1: rescaled variables */
  c2p_consts c;
  c.D = D;
  c.qq = tau / D;
  double ru[3], rd[3], Bcu[3];
  double sqD = sqrt(D);
  c.r2 = 0.0; c.B2c = 0.0; c.rB = 0.0;
  for (int i = 0; i < 3; i++) {
    rd[i] = Sd[i] / D;
    ru[i] = gu[i] * rd[i];
    Bcu[i] = Bu[i] / sqD;
    c.r2 += ru[i] * rd[i];
    c.B2c += gd[i] * Bcu[i] * Bcu[i];
    c.rB += rd[i] * Bcu[i];
  }
  c.rperp2B2 = c.B2c * c.r2 - c.rB * c.rB;
  if (c.rperp2B2 < 0.0) c.rperp2B2 = 0.0;
  c.h0 = 1.0; /* ideal gas: h = 1 + eps + p/rho >= 1 over eps >= 0 */
  c.v0sq = c.r2 / (c.h0 * c.h0 + c.r2);
  c.rho_min = rho_min;
  c.rho_max = d->rho_max;
  c.eps_min = 0.0;
  c.eps_max = d->eps_max;
  c.gam = d->gamma;

  /* step 2: mu_+ by Newton-Raphson from 1/h0, Illinois if that fails */
  double muplus = 1.0 / c.h0;
  {
    double mu = 1.0 / c.h0;
    int good = 0;
    for (int it = 0; it < 60; it++) {
      double dfa;
      double fa = c2p_fa(&c, mu, &dfa);
      if (fa == 0.0) { good = 1; break; }
      double mn = mu - fa / dfa;
      if (!(mn > 0.0 && mn <= 1.0 / c.h0)) break;
      if (fabs(mn - mu) <= 1e-15 * mn) { mu = mn; good = 1; break; }
      mu = mn;
    }
    if (!good) {
      int it2, ok2;
      mu = illinois(&c, fa_only, 0.0, 1.0 / c.h0, 1e-15, 200, &it2, &ok2);
    }
    muplus = mu;
  }

  /* step 3: the master function root on (0, mu_+] */
  int iters = 0, ok = 1;
  double mu;
  {
    double fb = c2p_f(&c, muplus, NULL);
    if (fb <= 0.0) {
      mu = muplus;
    } else {
      mu = illinois(&c, f_only, 0.0, muplus, d->c2p_tol, d->c2p_maxit, &iters, &ok);
    }
  }
  if (iters_out) *iters_out = iters;
  if (!ok) flags |= F_NOCONV;

  /* step 4: primitives from mu (raw values, before the limits) */
  c2p_eval e;
  c2p_f(&c, mu, &e);
  double W = e.What;
  double rho = e.rho;
  double eps = e.eps;
  double vu[3];
  for (int i = 0; i < 3; i++) vu[i] = mu * e.chi * (ru[i] + mu * c.rB * Bcu[i]);

  return finish_recovery(d, D, rho, eps, W, vu, gd, alpha, Bu, pr, flags, 0);
}

/* --------------------------------------------------- exported point calls */

void og_point_prim2con(double gam, const double pr[NV], const double met[5], const double ref[3], double q[NV]) {
  pstate s;
  point_state(gam, pr, met[0], met[1], met + 2, ref, &s);
  cons_from_state(&s, q);
}

void og_point_flux(double gam, const double pr[NV], const double met[5], const double ref[3], int a,
                   double f[NV], double lam[2]) {
  pstate s;
  point_state(gam, pr, met[0], met[1], met + 2, ref, &s);
  flux_from_state(&s, a, f);
  speeds_from_state(gam, &s, a, &lam[0], &lam[1]);
}

/* --------------------------------------------------------- reconstruction */

/* Monotonised-central slope (van Leer 1977, the "MC" limiter of section 3):
 * minmod(2 dl, (dl+dr)/2, 2 dr), zero where dl and dr differ in sign. */
static double mc_slope(double um, double u0, double up) {
  double dl = u0 - um, dr = up - u0;
  if (dl * dr <= 0.0) return 0.0;
  double c = 0.5 * (dl + dr);
  double m = fmin(fmin(fabs(2.0 * dl), fabs(c)), fabs(2.0 * dr));
  return dl > 0.0 ? m : -m;
}

/* MP5 (Suresh & Huynh 1997), the fifth-order monotonicity-preserving
 * reconstruction named in section 3: the interface value at i+1/2 from the
 * cell values u_{i-2..i+2} (a..e), left-biased.  The fifth-order value is
 * kept when it lies between u_i and the monotonicity bound u_mp (alpha = 4);
 * otherwise it is brought into [u_min, u_max] built from the curvature
 * (M4 minmod of second differences). */
static double minmod2(double x, double y) {
  if (x * y <= 0.0) return 0.0;
  return fabs(x) < fabs(y) ? x : y;
}
static double minmod4(double w, double x, double y, double z) {
  if (w > 0.0 && x > 0.0 && y > 0.0 && z > 0.0) return fmin(fmin(w, x), fmin(y, z));
  if (w < 0.0 && x < 0.0 && y < 0.0 && z < 0.0) return fmax(fmax(w, x), fmax(y, z));
  return 0.0;
}
static double mp5_face(double a, double b, double c, double d, double e) {
  const double alpha = 4.0;
  double uor = (2.0 * a - 13.0 * b + 47.0 * c + 27.0 * d - 3.0 * e) / 60.0;
  double ump = c + minmod2(d - c, alpha * (c - b));
  if ((uor - c) * (uor - ump) <= 0.0) return uor;
  double dm = a - 2.0 * b + c, d0 = b - 2.0 * c + d, dp = c - 2.0 * d + e;
  double dm4p = minmod4(4.0 * d0 - dp, 4.0 * dp - d0, d0, dp);
  double dm4m = minmod4(4.0 * dm - d0, 4.0 * d0 - dm, dm, d0);
  double uul = c + alpha * (c - b);
  double uav = 0.5 * (c + d);
  double umd = uav - 0.5 * dm4p;
  double ulc = c + 0.5 * (c - b) + (4.0 / 3.0) * dm4m;
  double umin = fmax(fmin(fmin(c, d), umd), fmin(fmin(c, uul), ulc));
  double umax = fmin(fmax(fmax(c, d), umd), fmax(fmax(c, uul), ulc));
  return uor + minmod2(umin - uor, umax - uor);
}

/* PPM (Colella & Woodward 1984), the third-order reconstruction named in
 * section 3, on a uniform grid without steepening or flattening: the value
 * of cell c (neighbours a, b | d, e) at its face toward d.  The interface
 * values between b, c and between c, d are the fourth-order interpolants
 * corrected by the difference of the limited (MC) slopes of the two cells;
 * the parabola through them is then made monotone: flat at a local extremum,
 * and the value at the far face (toward b) moved so that the parabola does
 * not overshoot, which changes the value toward d only when the overshoot is
 * on that side. */
static double ppm_face(double a, double b, double c, double d, double e) {
  double sb = mc_slope(a, b, c), sc = mc_slope(b, c, d), sd = mc_slope(c, d, e);
  double al = b + 0.5 * (c - b) - (sc - sb) / 6.0;
  double ar = c + 0.5 * (d - c) - (sd - sc) / 6.0;
  if ((ar - c) * (c - al) <= 0.0) return c;
  double dq = ar - al, m = c - 0.5 * (al + ar);
  if (-dq * dq / 6.0 > dq * m) return 3.0 * c - 2.0 * al;
  return ar;
}

/* HLLE flux (Harten, Lax & van Leer 1983; Einfeldt 1988), with the signal
 * speeds bounded by zero.  If both bounds vanish the average is used. */
static void hlle(const double fl[NV], const double fr[NV], const double ql[NV], const double qr[NV],
                 double lm, double lp, double f[NV]) {
  double ap = fmax(0.0, lp), am = fmin(0.0, lm);
  double den = ap - am;
  if (den < 1e-300) {
    for (int v = 0; v < NV; v++) f[v] = 0.5 * (fl[v] + fr[v]);
    return;
  }
  for (int v = 0; v < NV; v++) f[v] = (ap * fl[v] - am * fr[v] + ap * am * (qr[v] - ql[v])) / den;
}

static void load_metric(const og_desc *d, const double *met, long c, double m[5]) {
  long nt = ntot(d);
  for (int v = 0; v < 5; v++) m[v] = met[v * nt + c];
}

/* Flux times area through face f along axis a of the transverse cell
 * (i,j,k): MC-reconstructed left/right primitives, face metric as the mean
 * of the two neighbouring centres, then HLLE (section 2.1 discretised
 * equation; section 3 solver settings). */
/* Local Lax-Friedrichs (Rusanov) flux, the solver named TVDLF in section 3:
 * the mean of the two fluxes minus the largest speed magnitude c times half
 * the jump of the conserved variables. */
static void tvdlf(const double fl[NV], const double fr[NV], const double ql[NV], const double qr[NV], double c,
                  double f[NV]) {
  for (int v = 0; v < NV; v++) f[v] = 0.5 * (fl[v] + fr[v]) - 0.5 * c * (qr[v] - ql[v]);
}

/* What the positivity-preserving limiter needs besides the states: the
 * stage's time step and the state the stage's Euler step starts from. */
typedef struct {
  double dt;
  const double *qbase;
} pp_ctx;

/* theta of one conserved component and one side of a face (section 2.4):
 * the largest blend weight of the high-order flux that keeps the one-sided
 * Euler update u -/+ 2 dt/dV (f dA) above eps; 1 when the high-order flux
 * already does.  sgn = -1 for the cell below the face (u^-), +1 above (u^+);
 * fho, flf are flux times face area. */
static double pp_theta(double u, double dV, double dt, double fho, double flf, double sgn) {
  const double eps = 1e-16;
  if (u + sgn * 2.0 * dt / dV * fho > eps) return 1.0;
  double den = sgn * (flf - fho);
  if (den == 0.0) return 1.0;
  return (dV / (2.0 * dt) * (u - eps) + sgn * flf) / den;
}

static void face_flux_pp(const og_desc *d, const double *prim, const double *met, int a, int f,
                         int i, int j, int k, double out[NV], double *absterms, const pp_ctx *pp);

static void face_flux_x(const og_desc *d, const double *prim, const double *met, int a, int f,
                        int i, int j, int k, double out[NV], double *absterms) {
  face_flux_pp(d, prim, met, a, f, i, j, k, out, absterms, NULL);
}

static void face_flux_pp(const og_desc *d, const double *prim, const double *met, int a, int f,
                         int i, int j, int k, double out[NV], double *absterms, const pp_ctx *pp) {
  int cell[3] = {i, j, k};
  double area = face_area(d, a, f, i, j, k);
  if (area == 0.0) {
    for (int v = 0; v < NV; v++) out[v] = 0.0;
    if (absterms)
      for (int v = 0; v < NV; v++) absterms[v] = 0.0;
    return;
  }
  long nt = ntot(d);
  /* stencil cells f-3 .. f+2 along a (MC uses f-2 .. f+1) */
  long idx[6];
  for (int s = 0; s < 6; s++) {
    int c[3] = {cell[0], cell[1], cell[2]};
    c[a] = f - 3 + s;
    idx[s] = (s == 0 || s == 5) && d->recon == 0 ? -1 : at(d, c[0], c[1], c[2]);
  }
  double pl[NV], pr[NV];
  for (int v = 0; v < NV; v++) {
    double u[6];
    for (int s = 0; s < 6; s++) u[s] = idx[s] < 0 ? 0.0 : prim[v * nt + idx[s]];
    if (d->recon == 1) {
      pl[v] = mp5_face(u[0], u[1], u[2], u[3], u[4]);
      pr[v] = mp5_face(u[5], u[4], u[3], u[2], u[1]);
    } else if (d->recon == 2) {
      pl[v] = ppm_face(u[0], u[1], u[2], u[3], u[4]);
      pr[v] = ppm_face(u[5], u[4], u[3], u[2], u[1]);
    } else {
      pl[v] = u[2] + 0.5 * mc_slope(u[1], u[2], u[3]);
      pr[v] = u[3] - 0.5 * mc_slope(u[2], u[3], u[4]);
    }
  }
  if (d->recon != 0 && !(pl[RHO] > 0.0 && pl[PRS] > 0.0 && pr[RHO] > 0.0 && pr[PRS] > 0.0)) {
    /* a reconstructed state without positive density and pressure: both
     * sides of this face fall back to the adjacent cell values */
    for (int v = 0; v < NV; v++) {
      pl[v] = prim[v * nt + idx[2]];
      pr[v] = prim[v * nt + idx[3]];
    }
  }
  double m1[5], m2[5], mf[5];
  load_metric(d, met, idx[2], m1);
  load_metric(d, met, idx[3], m2);
  for (int v = 0; v < 5; v++) mf[v] = 0.5 * (m1[v] + m2[v]);
  double x[3] = {centre(d, 0, i), centre(d, 1, j), centre(d, 2, k)};
  x[a] = face_pos(d, a, f);
  double ref[3];
  ref_metric(d->coord, x[0], x[1], ref);
  pstate sl, sr;
  point_state(d->gamma, pl, mf[0], mf[1], mf + 2, ref, &sl);
  point_state(d->gamma, pr, mf[0], mf[1], mf + 2, ref, &sr);
  double ql[NV], qr[NV], fl[NV], fr[NV], lml, lpl, lmr, lpr;
  cons_from_state(&sl, ql);
  cons_from_state(&sr, qr);
  flux_from_state(&sl, a, fl);
  flux_from_state(&sr, a, fr);
  speeds_from_state(d->gamma, &sl, a, &lml, &lpl);
  speeds_from_state(d->gamma, &sr, a, &lmr, &lpr);
  double fh[NV];
  if (d->riemann == 1) {
    tvdlf(fl, fr, ql, qr, fmax(fmax(fabs(lml), fabs(lpl)), fmax(fabs(lmr), fabs(lpr))), fh);
  } else {
    hlle(fl, fr, ql, qr, fmin(lml, lmr), fmax(lpl, lpr), fh);
  }
  for (int v = 0; v < NV; v++) out[v] = fh[v] * area;
  if (pp && d->pp) {
    /* positivity-preserving limiter (section 2.4): blend with the
     * first-order Lax-Friedrichs flux of the two adjacent cell states (face
     * metric), theta from D and tau on both sides, the smaller one kept
     * (the largest theta for which both stay positive) */
    double p0[NV], p1[NV];
    for (int v = 0; v < NV; v++) {
      p0[v] = prim[v * nt + idx[2]];
      p1[v] = prim[v * nt + idx[3]];
    }
    pstate s0, s1;
    point_state(d->gamma, p0, mf[0], mf[1], mf + 2, ref, &s0);
    point_state(d->gamma, p1, mf[0], mf[1], mf + 2, ref, &s1);
    double q0[NV], q1[NV], f0[NV], f1[NV], lm0, lp0, lm1, lp1, flf[NV];
    cons_from_state(&s0, q0);
    cons_from_state(&s1, q1);
    flux_from_state(&s0, a, f0);
    flux_from_state(&s1, a, f1);
    speeds_from_state(d->gamma, &s0, a, &lm0, &lp0);
    speeds_from_state(d->gamma, &s1, a, &lm1, &lp1);
    tvdlf(f0, f1, q0, q1, fmax(fmax(fabs(lm0), fabs(lp0)), fmax(fabs(lm1), fabs(lp1))), flf);
    int c0[3] = {cell[0], cell[1], cell[2]}, c1[3] = {cell[0], cell[1], cell[2]};
    c0[a] = f - 1;
    c1[a] = f;
    double dV0 = cell_volume(d, c0[0], c0[1], c0[2]), dV1 = cell_volume(d, c1[0], c1[1], c1[2]);
    /* only the sides that are interior cells count: a ghost cell is not
     * advanced by the step, so its positivity is not at stake (and its
     * conserved state is not maintained) */
    int in0 = c0[a] >= 0, in1 = c1[a] < d->n[a];
    double theta = 1.0;
    const int comp[2] = {QD, QTAU};
    for (int m = 0; m < 2; m++) {
      int v = comp[m];
      double fho = out[v], fl = flf[v] * area;
      if (in0) theta = fmin(theta, pp_theta(pp->qbase[v * nt + idx[2]], dV0, pp->dt, fho, fl, -1.0));
      if (in1) theta = fmin(theta, pp_theta(pp->qbase[v * nt + idx[3]], dV1, pp->dt, fho, fl, +1.0));
    }
    theta = fmin(fmax(theta, 0.0), 1.0);
    if (theta < 1.0)
      for (int v = 0; v < NV; v++) out[v] = theta * out[v] + (1.0 - theta) * flf[v] * area;
  }
  if (absterms) {
    /* magnitude of the terms summed by the HLLE formula, with the states'
     * and fluxes' own term magnitudes (error scale) */
    double ual[NV], fal[NV], uar[NV], far_[NV];
    abs_terms_from_state(&sl, a, ual, fal);
    abs_terms_from_state(&sr, a, uar, far_);
    double ap = fmax(0.0, fmax(lpl, lpr)), am = fmin(0.0, fmin(lml, lmr)), den = ap - am;
    double cmax = fmax(fmax(fabs(lml), fabs(lpl)), fmax(fabs(lmr), fabs(lpr)));
    for (int v = 0; v < NV; v++) {
      double t;
      if (d->riemann == 1)
        t = 0.5 * (fal[v] + far_[v]) + 0.5 * cmax * (uar[v] + ual[v]);
      else
        t = den < 1e-300 ? 0.5 * (fal[v] + far_[v])
                         : (ap * fal[v] - am * far_[v] - ap * am * (uar[v] + ual[v])) / den;
      absterms[v] = t * area;
    }
  }
}

/* -------------------------------------------------------------- sources */

/* Point value of the reference-metric Christoffel symbols G[l][i][k]
 * (Appendix A). */
static void christoffel_point(int coord, double x1, double x2, double G[3][3][3]) {
  memset(G, 0, sizeof(double) * 27);
  if (coord == CYL) {
    G[0][2][2] = -x1;
    G[2][0][2] = G[2][2][0] = 1.0 / x1;
  } else if (coord == SPH) {
    double s = sin(x2), c = cos(x2);
    G[0][1][1] = -x1;
    G[0][2][2] = -x1 * s * s;
    G[1][0][1] = G[1][1][0] = 1.0 / x1;
    G[1][2][2] = -s * c;
    G[2][0][2] = G[2][2][0] = 1.0 / x1;
    G[2][1][2] = G[2][2][1] = c / s;
  }
}

/* Gravitational sources s_S_i and s_tau at the centre of cell (i,j,k)
 * (section 2.1, source terms), with centred differences of the metric
 * (second-order, as the derivative stencils of section 2.7) and K_ij of the
 * CFC metric under maximal slicing from the shift (section 2.6).  The result
 * is added to s[]. */
static void grav_sources_x(const og_desc *d, const double *met, const double *kij, const pstate *st, double psi,
                           int i, int j, int k, const double ref[3], double x1, double x2, double s[NV],
                           int absmode) {
#define TERM(x) (absmode ? fabs(x) : (x))
  int cell[3] = {i, j, k};
  double dalpha[3] = {0, 0, 0}, dpsi[3] = {0, 0, 0}, dbeta[3][3] = {{0}};
  long nt = ntot(d);
  for (int a = 0; a < d->ndim; a++) {
    int cp[3] = {cell[0], cell[1], cell[2]}, cm[3] = {cell[0], cell[1], cell[2]};
    cp[a] += 1;
    cm[a] -= 1;
    long ip = at(d, cp[0], cp[1], cp[2]), im = at(d, cm[0], cm[1], cm[2]);
    double inv = 1.0 / (2.0 * d->dx[a]);
    dpsi[a] = (met[0 * nt + ip] - met[0 * nt + im]) * inv;
    dalpha[a] = (met[1 * nt + ip] - met[1 * nt + im]) * inv;
    for (int m = 0; m < 3; m++) dbeta[a][m] = (met[(2 + m) * nt + ip] - met[(2 + m) * nt + im]) * inv;
  }
  double alpha = st->alpha;
  const double *beta = st->beta;
  double G[3][3][3];
  christoffel_point(d->coord, x1, x2, G);
  /* covariant derivative of the shift, nb[i][k] = d_i beta^k + G^k_il beta^l */
  double nb[3][3];
  for (int a = 0; a < 3; a++)
    for (int m = 0; m < 3; m++) {
      double v = dbeta[a][m];
      for (int l = 0; l < 3; l++) v += G[m][a][l] * beta[l];
      nb[a][m] = v;
    }
  /* K_ij given by the caller (6 arrays xx, xy, xz, yy, yz, zz), else
   * K_ij = psi^4/(2 alpha) (nb_i beta_j + nb_j beta_i - 2/3 ref_ij div beta) */
  double K[3][3];
  if (kij) {
    static const int comp[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    long c = at(d, i, j, k);
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) K[a][b] = kij[comp[a][b] * nt + c];
  } else {
    double divb = nb[0][0] + nb[1][1] + nb[2][2];
    double psi4 = psi * psi * psi * psi;
    for (int a = 0; a < 3; a++)
      for (int b = 0; b < 3; b++) {
        double v = ref[b] * nb[a][b] + ref[a] * nb[b][a];
        if (a == b) v -= 2.0 / 3.0 * ref[a] * divb;
        K[a][b] = psi4 / (2.0 * alpha) * v;
      }
  }
  /* T^{mu nu} = rho h* u^mu u^nu + p* g^{mu nu} - b^mu b^nu */
  double W = st->W;
  double u[4], bu[4];
  u[0] = W / alpha;
  for (int m = 0; m < 3; m++) u[1 + m] = W * (st->vu[m] - beta[m] / alpha);
  bu[0] = st->b0;
  for (int m = 0; m < 3; m++) bu[1 + m] = st->Bu[m] / W + st->b0 * st->vhat[m];
  double ginv[4][4];
  double ia2 = 1.0 / (alpha * alpha);
  ginv[0][0] = -ia2;
  for (int m = 0; m < 3; m++) { ginv[0][1 + m] = ginv[1 + m][0] = beta[m] * ia2; }
  for (int m = 0; m < 3; m++)
    for (int l = 0; l < 3; l++) ginv[1 + m][1 + l] = (m == l ? st->gu[m] : 0.0) - beta[m] * beta[l] * ia2;
  double T[4][4];
  for (int m = 0; m < 4; m++)
    for (int l = 0; l < 4; l++) T[m][l] = st->rhohs * u[m] * u[l] + st->ps * ginv[m][l] - bu[m] * bu[l];
  /* T^0_k = T^00 beta_k + T^0j gamma_jk */
  double T0d[3];
  for (int m = 0; m < 3; m++) T0d[m] = T[0][0] * st->gd[m] * beta[m] + T[0][1 + m] * st->gd[m];
  double pre = alpha * st->psi6;
  for (int a = 0; a < 3; a++) {
    double v = TERM(-T[0][0] * alpha * dalpha[a]);
    for (int m = 0; m < 3; m++) v += TERM(T0d[m] * nb[a][m]);
    /* nabla_i gamma_jk = 4 psi^3 d_i psi ref_jk (diagonal) */
    double dg = 4.0 * psi * psi * psi * dpsi[a];
    for (int m = 0; m < 3; m++) {
      double Tjk = T[0][0] * beta[m] * beta[m] + 2.0 * T[0][1 + m] * beta[m] + T[1 + m][1 + m];
      v += TERM(0.5 * Tjk * dg * ref[m]);
    }
    s[QS1 + a] += TERM(pre * v);
  }
  {
    double Kbb = 0.0, bda = 0.0, TK = 0.0, T0K = 0.0;
    for (int a = 0; a < 3; a++) {
      bda += TERM(beta[a] * dalpha[a]);
      for (int b = 0; b < 3; b++) {
        Kbb += TERM(K[a][b] * beta[a] * beta[b]);
        TK += TERM(T[1 + a][1 + b] * K[a][b]);
      }
    }
    for (int a = 0; a < 3; a++) {
      double Kb = 0.0;
      for (int b = 0; b < 3; b++) Kb += TERM(K[a][b] * beta[b]);
      T0K += TERM(T[0][1 + a] * (2.0 * Kb - TERM(dalpha[a])));
    }
    if (absmode)
      s[QTAU] += fabs(pre) * (fabs(T[0][0]) * (Kbb + bda) + T0K + TK);
    else
      s[QTAU] += pre * (T[0][0] * (Kbb - bda) + T0K + TK);
  }
#undef TERM
}

static void grav_sources(const og_desc *d, const double *met, const double *kij, const pstate *st, double psi, int i,
                         int j, int k, const double ref[3], double x1, double x2, double s[NV]) {
  grav_sources_x(d, met, kij, st, psi, i, j, k, ref, x1, x2, s, 0);
}

/* Geometric sources <Gamma^l_ik> (f_S_l)^k with the fluxes taken at the cell
 * centre (section 2.1 and Appendix A).  The row of the ignorable phi
 * coordinate is zero by construction.  The spherical <Gamma^phi_theta phi>
 * is taken as the exact cell average, (A_theta+ - A_theta-)/dV, of which the
 * printed cot(theta) is the point value. */
static void geom_sources_x(const og_desc *d, const pstate *st, int i, int j, int k, double s[NV], int absmode) {
  if (d->coord == CART) return;
  double f[3][NV];
  for (int a = 0; a < 3; a++) flux_from_state(st, a, f[a]);
  double dV = cell_volume(d, i, j, k);
  if (absmode)
    for (int a = 0; a < 3; a++)
      for (int v = 0; v < NV; v++) f[a][v] = fabs(f[a][v]);
  if (d->coord == CYL) {
    double R = centre(d, 0, i);
    s[QS1 + 0] += (absmode ? fabs(1.0 / R) : 1.0 / R) * f[2][QS1 + 2];
    return;
  }
  double rp = face_pos(d, 0, i + 1), rm = face_pos(d, 0, i);
  double Arp = face_area(d, 0, i + 1, i, j, k), Arm = face_area(d, 0, i, i, j, k);
  double Atp = face_area(d, 1, j + 1, i, j, k), Atm = face_area(d, 1, j, i, j, k);
  double g_th_rth = 0.5 * (Arp - Arm) / dV;          /* <G^th_r th> = <G^ph_r ph> */
  double g_r_thth = -0.25 * (rp * rp * Arp - rm * rm * Arm) / dV; /* <G^r_th th> */
  double g_ph_thph = (Atp - Atm) / dV;                /* <G^ph_th ph> */
  if (absmode) {
    g_th_rth = fabs(g_th_rth);
    g_r_thth = fabs(g_r_thth);
    g_ph_thph = fabs(g_ph_thph);
  }
  s[QS1 + 0] += g_th_rth * f[1][QS1 + 1] + g_th_rth * f[2][QS1 + 2];
  s[QS1 + 1] += g_r_thth * f[1][QS1 + 0] + g_th_rth * f[0][QS1 + 1] + g_ph_thph * f[2][QS1 + 2];
}

static void geom_sources(const og_desc *d, const pstate *st, int i, int j, int k, double s[NV]) {
  geom_sources_x(d, st, i, j, k, s, 0);
}

/* ------------------------------------------------------------------- RHS */

/* d<q>/dt at interior cell (i,j,k): minus the flux-area divergence over the
 * cell volume plus the gravitational and geometric sources (section 2.1,
 * the discretised equation; the minus sign on the flux bracket follows from
 * the conservation law and the positivity-limiter form of section 2.4). */
static void rhs_cell_pp(const og_desc *d, const double *prim, const double *met, const double *kij, int i, int j,
                        int k, double dq[NV], const pp_ctx *pp);

void og_rhs_cell(const og_desc *d, const double *prim, const double *met, int i, int j, int k, double dq[NV]) {
  rhs_cell_pp(d, prim, met, NULL, i, j, k, dq, NULL);
}

/* The same with the positivity-preserving limiter on the face fluxes when
 * the descriptor asks for it and pp is given. */
static void rhs_cell_pp(const og_desc *d, const double *prim, const double *met, const double *kij, int i, int j,
                        int k, double dq[NV], const pp_ctx *pp) {
  int cell[3] = {i, j, k};
  for (int v = 0; v < NV; v++) dq[v] = 0.0;
  double dV = cell_volume(d, i, j, k);
  for (int a = 0; a < d->ndim; a++) {
    double fm[NV], fp[NV];
    face_flux_pp(d, prim, met, a, cell[a], i, j, k, fm, NULL, pp);
    face_flux_pp(d, prim, met, a, cell[a] + 1, i, j, k, fp, NULL, pp);
    for (int v = 0; v < NV; v++) dq[v] -= (fp[v] - fm[v]) / dV;
  }
  long nt = ntot(d), c = at(d, i, j, k);
  double pr[NV], m[5];
  for (int v = 0; v < NV; v++) pr[v] = prim[v * nt + c];
  load_metric(d, met, c, m);
  double x1 = centre(d, 0, i), x2 = centre(d, 1, j);
  double ref[3];
  ref_metric(d->coord, x1, x2, ref);
  pstate st;
  point_state(d->gamma, pr, m[0], m[1], m + 2, ref, &st);
  double s[NV] = {0};
  grav_sources(d, met, kij, &st, m[0], i, j, k, ref, x1, x2, s);
  geom_sources(d, &st, i, j, k, s);
  for (int v = 0; v < NV; v++) dq[v] += s[v];
}

/* The RHS on every interior cell; kij (nullable): K_ij per cell, 6 arrays in
 * the grid's layout (xx, xy, xz, yy, yz, zz), else K_ij from the shift. */
void og_rhs_k(const og_desc *d, const double *prim, const double *met, const double *kij, double *dqdt) {
  long nt = ntot(d);
  for (int k = 0; k < d->n[2]; k++)
    for (int j = 0; j < d->n[1]; j++)
      for (int i = 0; i < d->n[0]; i++) {
        double dq[NV];
        rhs_cell_pp(d, prim, met, kij, i, j, k, dq, NULL);
        long c = at(d, i, j, k);
        for (int v = 0; v < NV; v++) dqdt[v * nt + c] = dq[v];
      }
}

void og_rhs(const og_desc *d, const double *prim, const double *met, double *dqdt) {
  og_rhs_k(d, prim, met, NULL, dqdt);
}

/* RHS at a list of interior cells given as (i,j,k) triples; out is [n][8];
 * kij as in og_rhs_k. */
void og_rhs_cells_k(const og_desc *d, const double *prim, const double *met, const double *kij, long ncell,
                    const int *ijk, double *out) {
  for (long c = 0; c < ncell; c++)
    rhs_cell_pp(d, prim, met, kij, ijk[3 * c], ijk[3 * c + 1], ijk[3 * c + 2], out + NV * c, NULL);
}

void og_rhs_cells(const og_desc *d, const double *prim, const double *met, long ncell, const int *ijk, double *out) {
  og_rhs_cells_k(d, prim, met, NULL, ncell, ijk, out);
}

/* The gravitational and the geometric source terms of interior cell
 * (i,j,k) separately (section 2.1, Appendix A), for checks; kij as in
 * og_rhs_k. */
void og_sources_cell(const og_desc *d, const double *prim, const double *met, const double *kij, int i, int j, int k,
                     double grav[NV], double geom[NV]) {
  long nt = ntot(d), c = at(d, i, j, k);
  double pr[NV], m[5];
  for (int v = 0; v < NV; v++) pr[v] = prim[v * nt + c];
  load_metric(d, met, c, m);
  double x1 = centre(d, 0, i), x2 = centre(d, 1, j);
  double ref[3];
  ref_metric(d->coord, x1, x2, ref);
  pstate st;
  point_state(d->gamma, pr, m[0], m[1], m + 2, ref, &st);
  for (int v = 0; v < NV; v++) grav[v] = geom[v] = 0.0;
  grav_sources(d, met, kij, &st, m[0], i, j, k, ref, x1, x2, grav);
  geom_sources(d, &st, i, j, k, geom);
}

/* Error scale of each cell's RHS (test helper): the sum over the cell's
 * faces of the magnitudes of the terms the HLLE flux adds up, times area over
 * volume, plus the summed magnitudes of every source term.  A floating-point
 * evaluation of the RHS is accurate relative to this sum, not to the RHS
 * itself, which cancels to near zero in smooth or static regions. */
void og_rhs_scale_cells_k(const og_desc *d, const double *prim, const double *met, const double *kij, long ncell,
                          const int *ijk, double *out) {
  long nt = ntot(d);
  for (long c = 0; c < ncell; c++) {
    int i = ijk[3 * c], j = ijk[3 * c + 1], k = ijk[3 * c + 2];
    int cell[3] = {i, j, k};
    double *o = out + NV * c;
    for (int v = 0; v < NV; v++) o[v] = 0.0;
    double dV = cell_volume(d, i, j, k);
    for (int a = 0; a < d->ndim; a++) {
      double fm[NV], fp[NV], am[NV], ap[NV];
      face_flux_x(d, prim, met, a, cell[a], i, j, k, fm, am);
      face_flux_x(d, prim, met, a, cell[a] + 1, i, j, k, fp, ap);
      for (int v = 0; v < NV; v++) o[v] += (ap[v] + am[v]) / dV;
    }
    long cc = at(d, i, j, k);
    double pr[NV], m[5];
    for (int v = 0; v < NV; v++) pr[v] = prim[v * nt + cc];
    load_metric(d, met, cc, m);
    double x1 = centre(d, 0, i), x2 = centre(d, 1, j);
    double ref[3];
    ref_metric(d->coord, x1, x2, ref);
    pstate st;
    point_state(d->gamma, pr, m[0], m[1], m + 2, ref, &st);
    double s1[NV] = {0}, s2[NV] = {0};
    grav_sources_x(d, met, kij, &st, m[0], i, j, k, ref, x1, x2, s1, 1);
    geom_sources_x(d, &st, i, j, k, s2, 1);
    for (int v = 0; v < NV; v++) o[v] += s1[v] + s2[v];
  }
}

void og_rhs_scale_cells(const og_desc *d, const double *prim, const double *met, long ncell, const int *ijk, double *out) {
  og_rhs_scale_cells_k(d, prim, met, NULL, ncell, ijk, out);
}

/* ------------------------------------------------------ prim2con / c2p */

void og_prim2con(const og_desc *d, const double *prim, const double *met, double *q) {
  long nt = ntot(d);
  for (int k = -gh(d, 2); k < d->n[2] + gh(d, 2); k++)
    for (int j = -gh(d, 1); j < d->n[1] + gh(d, 1); j++)
      for (int i = -gh(d, 0); i < d->n[0] + gh(d, 0); i++) {
        long c = at(d, i, j, k);
        double pr[NV], m[5], ref[3], qq[NV];
        for (int v = 0; v < NV; v++) pr[v] = prim[v * nt + c];
        load_metric(d, met, c, m);
        ref_metric(d->coord, centre(d, 0, i), centre(d, 1, j), ref);
        og_point_prim2con(d->gamma, pr, m, ref, qq);
        for (int v = 0; v < NV; v++) q[v * nt + c] = qq[v];
      }
}

/* c2p over interior cells.  Cells whose primitives were corrected (atmosphere
 * or clamps) get q rewritten from the corrected primitives.  Returns the
 * number of cells with a fatal flag. */
long og_c2p(const og_desc *d, double *q, const double *met, double *prim, uint8_t *flags) {
  long nt = ntot(d), nfatal = 0;
  /* cells are independent; the pragma only acts in the all-cores timing
   * build (-fopenmp) */
#pragma omp parallel for collapse(2) reduction(+ : nfatal)
  for (int k = 0; k < d->n[2]; k++)
    for (int j = 0; j < d->n[1]; j++)
      for (int i = 0; i < d->n[0]; i++) {
        long c = at(d, i, j, k);
        double qc[NV], pr[NV], m[5], ref[3];
        for (int v = 0; v < NV; v++) qc[v] = q[v * nt + c];
        load_metric(d, met, c, m);
        ref_metric(d->coord, centre(d, 0, i), centre(d, 1, j), ref);
        int fl = og_c2p_point(d, qc, m[0], m[1], ref, pr, NULL);
        for (int v = 0; v < NV; v++) prim[v * nt + c] = pr[v];
        if (fl & (F_ATMO | F_EPS_CLAMP | F_V_CLAMP)) {
          double qn[NV];
          og_point_prim2con(d->gamma, pr, m, ref, qn);
          for (int v = 0; v < NV; v++) q[v * nt + c] = qn[v];
        }
        if (fl & F_FATAL_MASK) nfatal++;
        if (flags) flags[c] = (uint8_t)fl;
      }
  return nfatal;
}

/* ----------------------------------------------------------- ghost fill */

/* Sign of variable v when mirrored through a boundary of type bc on axis a.
 * Vectors are contravariant coordinate components, so the parities follow
 * from continuing the coordinates through the boundary: the ghost at the
 * formal position (-R, z) or (r, -theta) is the point at phi + pi, the ghost
 * at (-r, theta) is the point (r, pi - theta, phi + pi).
 *   REFLECT (a wall): the normal component is odd.
 *   AXIS (R = 0, theta = 0 or pi): the normal component is odd; the phi
 *     component (an angular rate) is even.
 *   CENTER (r = 0): the r and theta components are odd, phi is even. */
static double mirror_sign(int bc, int a, int v) {
  int comp = -1;
  if (v >= WV1 && v < WV1 + 3) comp = v - WV1;
  if (v >= BB1 && v < BB1 + 3) comp = v - BB1;
  if (comp < 0) return 1.0;
  if (bc == BC_REFLECT || bc == BC_AXIS) return comp == a ? -1.0 : 1.0;
  if (bc == BC_CENTER) return (comp == 0 || comp == 1) ? -1.0 : 1.0;
  return 1.0;
}

/* Fill the ghost cells that share a face-normal line with the interior (the
 * only ghosts any stencil of the scheme reads). */
void og_fill_ghosts(const og_desc *d, double *prim) {
  long nt = ntot(d);
  for (int a = 0; a < d->ndim; a++) {
    int g = d->ng, n = d->n[a];
    int lo[3] = {0, 0, 0}, hi[3] = {d->n[0], d->n[1], d->n[2]};
    for (int side = 0; side < 2; side++) {
      int bc = d->bc[a][side];
      if (bc == BC_NONE) continue;
      lo[a] = 0; hi[a] = 1;
      for (int k = lo[2]; k < hi[2]; k++)
        for (int j = lo[1]; j < hi[1]; j++)
          for (int i = lo[0]; i < hi[0]; i++)
            for (int l = 0; l < g; l++) {
              int dst[3] = {i, j, k}, src[3] = {i, j, k};
              int gi = side == 0 ? -1 - l : n + l;   /* ghost index along a */
              dst[a] = gi;
              double sgn[NV];
              for (int v = 0; v < NV; v++) sgn[v] = 1.0;
              if (bc == BC_PERIODIC) {
                src[a] = side == 0 ? gi + n : gi - n;
              } else if (bc == BC_OUTFLOW) {
                src[a] = side == 0 ? 0 : n - 1;
              } else {
                src[a] = side == 0 ? -1 - gi : 2 * n - 1 - gi;
                for (int v = 0; v < NV; v++) sgn[v] = mirror_sign(bc, a, v);
                if (bc == BC_CENTER && d->ndim > 1) src[1] = d->n[1] - 1 - src[1];
                if ((bc == BC_CENTER || bc == BC_AXIS) && d->ndim > 2) src[2] = (src[2] + d->n[2] / 2) % d->n[2];
              }
              long cd = at(d, dst[0], dst[1], dst[2]), cs = at(d, src[0], src[1], src[2]);
              for (int v = 0; v < NV; v++) prim[v * nt + cd] = sgn[v] * prim[v * nt + cs];
            }
      lo[a] = 0; hi[a] = d->n[a];
    }
  }
}

/* ------------------------------------------------------------------ CFL */

/* Time step by the "maxsum" rule (section 2.9): dt = c / max over cells of
 * sum over active axes of max|lambda|/dx, with coordinate speeds and
 * coordinate spacings; dt is capped at t_end - t. */
double og_cfl_dt(const og_desc *d, const double *prim, const double *met, double cfl, double t, double t_end) {
  long nt = ntot(d);
  double mx = 0.0;
#pragma omp parallel for collapse(2) reduction(max : mx)
  for (int k = 0; k < d->n[2]; k++)
    for (int j = 0; j < d->n[1]; j++)
      for (int i = 0; i < d->n[0]; i++) {
        long c = at(d, i, j, k);
        double pr[NV], m[5], ref[3];
        for (int v = 0; v < NV; v++) pr[v] = prim[v * nt + c];
        load_metric(d, met, c, m);
        ref_metric(d->coord, centre(d, 0, i), centre(d, 1, j), ref);
        pstate st;
        point_state(d->gamma, pr, m[0], m[1], m + 2, ref, &st);
        double sum = 0.0;
        for (int a = 0; a < d->ndim; a++) {
          double lm, lp;
          speeds_from_state(d->gamma, &st, a, &lm, &lp);
          sum += fmax(fabs(lm), fabs(lp)) / d->dx[a];
        }
        if (sum > mx) mx = sum;
      }
  double dt = mx > 0.0 ? cfl / mx : t_end - t;
  if (t + dt > t_end) dt = t_end - t;
  /* at or past the end (t may land an ulp beyond t_end after the capped
   * step): no step */
  return dt > 0.0 ? dt : 0.0;
}

/* -------------------------------------------------------------- stepping */

/* One stage of the strong-stability-preserving Runge-Kutta integrators
 * (SSPRK3 is the default of section 3; SSPRK2 the setting of the convergence
 * tests).  Shu-Osher form:
 *   SSPRK3: u1 = un + dt L(un); u2 = 3/4 un + 1/4 (u1 + dt L(u1));
 *           un+1 = 1/3 un + 2/3 (u2 + dt L(u2))
 *   SSPRK2: u1 = un + dt L(un); un+1 = 1/2 un + 1/2 (u1 + dt L(u1)).
 * prim must hold the primitives of the current stage state with ghosts.
 * og_rk_update leaves the new stage state in qs (interior cells) before any
 * recovery; og_rk_stage then recovers prim (c2p, which may rewrite q of
 * corrected cells) and fills its ghosts, and returns the number of fatal c2p
 * cells. */
void og_rk_update_k(const og_desc *d, int stage, double dt, const double *qn, double *qs, const double *prim,
                    const double *met, const double *kij) {
  long nt = ntot(d);
  double a, b;
  if (stage == 0) { a = 0.0; b = 1.0; }
  else if (d->rk == 2) { a = 0.5; b = 0.5; }
  else if (stage == 1) { a = 0.75; b = 0.25; }
  else { a = 1.0 / 3.0; b = 2.0 / 3.0; }
  double *L = (double *)malloc(sizeof(double) * NV * nt);
  /* the stage's Euler step starts from q_n in stage 0, from q_s after */
  pp_ctx pp = {dt, stage == 0 ? qn : qs};
#pragma omp parallel for collapse(2)
  for (int k = 0; k < d->n[2]; k++)
    for (int j = 0; j < d->n[1]; j++)
      for (int i = 0; i < d->n[0]; i++) {
        double dq[NV];
        rhs_cell_pp(d, prim, met, kij, i, j, k, dq, &pp);
        long c = at(d, i, j, k);
        for (int v = 0; v < NV; v++) L[v * nt + c] = dq[v];
      }
#pragma omp parallel for collapse(2)
  for (int k = 0; k < d->n[2]; k++)
    for (int j = 0; j < d->n[1]; j++)
      for (int i = 0; i < d->n[0]; i++) {
        long c = at(d, i, j, k);
        for (int v = 0; v < NV; v++) {
          long o = v * nt + c;
          double us = stage == 0 ? qn[o] : qs[o];
          qs[o] = a * qn[o] + b * (us + dt * L[o]);
        }
      }
  free(L);
}

void og_rk_update(const og_desc *d, int stage, double dt, const double *qn, double *qs, const double *prim,
                  const double *met) {
  og_rk_update_k(d, stage, dt, qn, qs, prim, met, NULL);
}

long og_rk_stage_k(const og_desc *d, int stage, double dt, const double *qn, double *qs, double *prim,
                   const double *met, const double *kij, uint8_t *flags) {
  og_rk_update_k(d, stage, dt, qn, qs, prim, met, kij);
  long nf = og_c2p(d, qs, met, prim, flags);
  og_fill_ghosts(d, prim);
  return nf;
}

long og_rk_stage(const og_desc *d, int stage, double dt, const double *qn, double *qs, double *prim,
                 const double *met, uint8_t *flags) {
  og_rk_update(d, stage, dt, qn, qs, prim, met);
  long nf = og_c2p(d, qs, met, prim, flags);
  og_fill_ghosts(d, prim);
  return nf;
}

/* Advance q (and prim, which must be consistent with q, ghosts filled) by up
 * to nsteps steps or until t_end.  Returns the number of steps taken; *t is
 * advanced.  *nfatal accumulates fatal c2p cells. */
long og_evolve(const og_desc *d, double *q, double *prim, const double *met, double cfl, double *t,
               double t_end, long nsteps, long *nfatal) {
  long nt = ntot(d);
  double *qs = (double *)malloc(sizeof(double) * NV * nt);
  memcpy(qs, q, sizeof(double) * NV * nt);
  long s = 0;
  int nst = d->rk == 2 ? 2 : 3;
  while (s < nsteps && *t < t_end) {
    double dt = og_cfl_dt(d, prim, met, cfl, *t, t_end);
    if (!(dt > 0.0)) break;
    for (int st = 0; st < nst; st++) *nfatal += og_rk_stage(d, st, dt, q, qs, prim, met, NULL);
    memcpy(q, qs, sizeof(double) * NV * nt);
    *t += dt;
    s++;
  }
  free(qs);
  return s;
}

/* ---------------------------------------------------------- diagnostics */

/* Cell volumes of the interior (for volume-weighted norms and the rest-mass
 * integral of section 3.3). */
void og_cell_volumes(const og_desc *d, double *out) {
  long nt = ntot(d);
  for (long c = 0; c < nt; c++) out[c] = 0.0;
  for (int k = 0; k < d->n[2]; k++)
    for (int j = 0; j < d->n[1]; j++)
      for (int i = 0; i < d->n[0]; i++) out[at(d, i, j, k)] = cell_volume(d, i, j, k);
}

/* Geometry exported for checks: cell volume, the two face areas along each
 * axis, and the averaged Christoffel symbols of cell (i,j,k):
 * out = [dV, A0-, A0+, A1-, A1+, A2-, A2+, <G^th_r th>, <G^r_th th>,
 *        <G^ph_th ph>, <G^R_ph ph>, <G^ph_R ph>] */
void og_cell_geometry(const og_desc *d, int i, int j, int k, double out[12]) {
  int cell[3] = {i, j, k};
  double dV = cell_volume(d, i, j, k);
  out[0] = dV;
  for (int a = 0; a < 3; a++) {
    out[1 + 2 * a] = face_area(d, a, cell[a], i, j, k);
    out[2 + 2 * a] = face_area(d, a, cell[a] + 1, i, j, k);
  }
  for (int v = 7; v < 12; v++) out[v] = 0.0;
  if (d->coord == SPH) {
    double rp = face_pos(d, 0, i + 1), rm = face_pos(d, 0, i);
    out[7] = 0.5 * (out[2] - out[1]) / dV;
    out[8] = -0.25 * (rp * rp * out[2] - rm * rm * out[1]) / dV;
    out[9] = (out[4] - out[3]) / dV;
  } else if (d->coord == CYL) {
    double R = centre(d, 0, i), dR = d->dx[0];
    out[10] = -(R * R + dR * dR / 12.0) / R;
    out[11] = 1.0 / R;
  }
}

/* Threads the per-cell loops use (1 unless built with -fopenmp). */
#ifdef _OPENMP
#include <omp.h>
int og_threads(void) { return omp_get_max_threads(); }
#else
int og_threads(void) { return 1; }
#endif

long og_ntot(const og_desc *d) { return ntot(d); }
long og_index(const og_desc *d, int i, int j, int k) { return at(d, i, j, k); }
int og_desc_size(void) { return (int)sizeof(og_desc); }

/* MC-reconstructed face values of one variable on a line: for each face
 * f = 1..n-3 between cells f and f+1 of u[0..n-1], left value from cell f,
 * right value from cell f+1.  out_l/out_r have n-3 entries. */
/* MP5 face values of a 1D sequence: out_l[f - 2], out_r[f - 2] are the left
 * and right states at the face between u[f] and u[f + 1], f = 2 .. n-4. */
void og_mp5_faces(int n, const double *u, double *out_l, double *out_r) {
  for (int f = 2; f + 3 < n; f++) {
    out_l[f - 2] = mp5_face(u[f - 2], u[f - 1], u[f], u[f + 1], u[f + 2]);
    out_r[f - 2] = mp5_face(u[f + 3], u[f + 2], u[f + 1], u[f], u[f - 1]);
  }
}

void og_ppm_faces(int n, const double *u, double *out_l, double *out_r) {
  for (int f = 2; f + 3 < n; f++) {
    out_l[f - 2] = ppm_face(u[f - 2], u[f - 1], u[f], u[f + 1], u[f + 2]);
    out_r[f - 2] = ppm_face(u[f + 3], u[f + 2], u[f + 1], u[f], u[f - 1]);
  }
}

void og_mc_faces(int n, const double *u, double *out_l, double *out_r) {
  for (int f = 1; f + 2 < n; f++) {
    out_l[f - 1] = u[f] + 0.5 * mc_slope(u[f - 1], u[f], u[f + 1]);
    out_r[f - 1] = u[f + 1] - 0.5 * mc_slope(u[f], u[f + 1], u[f + 2]);
  }
}

/* HLLE flux between two primitive states at one point (flux, not times area). */
void og_point_hlle(double gam, const double pl[NV], const double pr[NV], const double met[5], const double ref[3],
                   int a, double f[NV]) {
  pstate sl, sr;
  point_state(gam, pl, met[0], met[1], met + 2, ref, &sl);
  point_state(gam, pr, met[0], met[1], met + 2, ref, &sr);
  double ql[NV], qr[NV], fl[NV], fr[NV], lml, lpl, lmr, lpr;
  cons_from_state(&sl, ql);
  cons_from_state(&sr, qr);
  flux_from_state(&sl, a, fl);
  flux_from_state(&sr, a, fr);
  speeds_from_state(gam, &sl, a, &lml, &lpl);
  speeds_from_state(gam, &sr, a, &lmr, &lpr);
  hlle(fl, fr, ql, qr, fmin(lml, lmr), fmax(lpl, lpr), f);
}

/* The local Lax-Friedrichs flux between two primitive states at one point. */
void og_point_tvdlf(double gam, const double pl[NV], const double pr[NV], const double met[5], const double ref[3],
                    int a, double f[NV]) {
  pstate sl, sr;
  point_state(gam, pl, met[0], met[1], met + 2, ref, &sl);
  point_state(gam, pr, met[0], met[1], met + 2, ref, &sr);
  double ql[NV], qr[NV], fl[NV], fr[NV], lml, lpl, lmr, lpr;
  cons_from_state(&sl, ql);
  cons_from_state(&sr, qr);
  flux_from_state(&sl, a, fl);
  flux_from_state(&sr, a, fr);
  speeds_from_state(gam, &sl, a, &lml, &lpl);
  speeds_from_state(gam, &sr, a, &lmr, &lpr);
  tvdlf(fl, fr, ql, qr, fmax(fmax(fabs(lml), fabs(lpl)), fmax(fabs(lmr), fabs(lpr))), f);
}
