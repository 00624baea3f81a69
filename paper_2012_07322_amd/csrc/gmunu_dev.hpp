// Device-side physics of the GRMHD finite-volume step on gfx950.
//
// Cheong et al., "Gmunu" (arXiv 2012.07322): conserved variables, fluxes and
// sources of section 2.1, wave-speed bounds of section 2.3, primitive
// recovery of section 2.5, geometry of Appendix A.  All FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gmunu.h"

namespace gm {

constexpr int NV = 8;
constexpr int NT = 256;  // threads per workgroup of the cell kernels

enum { CART = 0, CYL = 1, SPH = 2 };
enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_REFLECT = 2, BC_AXIS = 3, BC_CENTER = 4, BC_NONE = 5 };
enum {
  FL_ATMO = 1, FL_EPS = 2, FL_V = 4, FL_FRHO = 8, FL_FEPS = 16, FL_FV = 32, FL_NOCONV = 64,
  FL_FATAL = FL_FRHO | FL_FEPS | FL_FV | FL_NOCONV,
  FL_REWRITE = FL_ATMO | FL_EPS | FL_V
};

// Per-axis 1D geometry.  Every cell volume and face area of Appendix A is a
// product of one factor per axis: dV = cv0 cv1 cv2 and the area of an
// axis-a face is fa_a * prod_{b != a} cv_b, so (F dA)_+ - (F dA)_-) / dV
// reduces to (F fa)_+ - (F fa)_-) / cv_a.  Indices include ghosts: cell I in
// [0, nt), face F in [0, nt] between cells F-1 and F.
struct Geo {
  const double *icv[3];  // 1 / cv per cell
  const double *fa[3];   // face factor per face
  const double *r2c;     // axis-0 coordinate squared at centres
  const double *r2f;     // ... at faces
  const double *s2c;     // sin^2 of axis-1 coordinate at centres (spherical)
  const double *s2f;     // ... at faces
  const double *xc0;     // axis-0 centre coordinate
  const double *sc1, *cc1;  // sin, cos of axis-1 centre coordinate
  const double *gA;      // per axis-0 cell: sph <G^th_r th> = <G^ph_r ph>, cyl <G^ph_R ph>
  const double *gB;      // per axis-0 cell: sph <G^r_th th>
  const double *gC;      // per axis-1 cell: sph <G^ph_th ph>
};

struct Grid {
  int ndim, coord;
  int n[3], g[3], nt[3];
  long s[3];   // element strides of the three axes
  long nv;     // stride between variables (cells per array)
  double dx[3];
  double i2dx[3];   // 1 / (2 dx) for centred metric derivatives
  double idx[3];    // 1 / dx for the CFL rate
  double gam, gfac;  // Gamma and Gamma / (Gamma - 1)
  double gm1;        // Gamma - 1
  double rho_atmo, p_atmo, rho_low, alpha_bh, rho_max, eps_max, w_max;
  int maxit;
  double tol;
  int recon;    // GMUNU_RECON_*
  int riemann;  // GMUNU_RIEMANN_*
  int c2p;      // GMUNU_C2P_*
  int pp;       // positivity-preserving flux limiter on (single grids)
  int bc[3][2];
  Geo geo;
};

__device__ __forceinline__ long cell_offset(const Grid &G, int i, int j, int k) {
  return (long)(k + G.g[2]) * G.s[2] + (long)(j + G.g[1]) * G.s[1] + (i + G.g[0]);
}

// Diagonal of the reference metric from the squared axis-0 coordinate and
// sin^2 of the axis-1 coordinate at the evaluation point.
__device__ __forceinline__ void ref_diag(int coord, double r2, double s2, double &g1, double &g2) {
  if (coord == SPH) {
    g1 = r2;
    g2 = r2 * s2;
  } else if (coord == CYL) {
    g1 = 1.0;
    g2 = r2;
  } else {
    g1 = 1.0;
    g2 = 1.0;
  }
}

// 1/x: hardware reciprocal estimate refined by two Newton steps (matches the
// correctly rounded quotient on measured samples; finite non-zero x).
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// 1/sqrt(x) for finite x > 0: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rsq(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  double e = fma(-h * y, y, 0.5);
  y = fma(y, e, y);
  e = fma(-h * y, y, 0.5);
  return fma(y, e, y);
}

// sqrt(x) for x >= 0 (0 below 1e-300).
__device__ __forceinline__ double sqrt_pos(double x) { return x > 1e-300 ? x * rsq(x) : 0.0; }

// Monotonised-central limited slope: minmod(2 dl, (dl + dr) / 2, 2 dr).
__device__ __forceinline__ double mc_slope(double a, double b, double c) {
  double dl = b - a, dr = c - b;
  double cen = 0.5 * (dl + dr);
  double m = fmin(fmin(fabs(2.0 * dl), fabs(cen)), fabs(2.0 * dr));
  return (dl * dr > 0.0) ? copysign(m, cen) : 0.0;
}

// Half the monotonised-central slope, written minmod(dl, (dl + dr) / 4, dr):
// scaling by powers of two is exact, so this is bit for bit 0.5 *
// mc_slope(a, b, c), with two multiplications fewer.
__device__ __forceinline__ double mc_half_slope(double a, double b, double c) {
  const double dl = b - a, dr = c - b;
  const double q = 0.25 * (dl + dr);
  const double m = fmin(fmin(fabs(dl), fabs(q)), fabs(dr));
  return (dl * dr > 0.0) ? copysign(m, q) : 0.0;
}

// MP5 (Suresh & Huynh 1997; the default reconstruction of section 3): the
// left-biased interface value at i+1/2 from u_{i-2..i+2} = a..e.  The
// fifth-order value is kept when it lies between u_i and the monotonicity
// bound (alpha = 4), else it is brought into [u_min, u_max] built from the
// M4 minmod of second differences.
__device__ __forceinline__ double minmod2(double x, double y) {
  return x * y <= 0.0 ? 0.0 : (fabs(x) < fabs(y) ? x : y);
}
__device__ __forceinline__ double minmod4(double w, double x, double y, double z) {
  if (w > 0.0 && x > 0.0 && y > 0.0 && z > 0.0) return fmin(fmin(w, x), fmin(y, z));
  if (w < 0.0 && x < 0.0 && y < 0.0 && z < 0.0) return fmax(fmax(w, x), fmax(y, z));
  return 0.0;
}
__device__ __forceinline__ double mp5_face(double a, double b, double c, double d, double e) {
  constexpr double alpha = 4.0;
  const double uor = (2.0 * a - 13.0 * b + 47.0 * c + 27.0 * d - 3.0 * e) * (1.0 / 60.0);
  const double ump = c + minmod2(d - c, alpha * (c - b));
  if ((uor - c) * (uor - ump) <= 0.0) return uor;
  const double dm = a - 2.0 * b + c, d0 = b - 2.0 * c + d, dp = c - 2.0 * d + e;
  const double dm4p = minmod4(4.0 * d0 - dp, 4.0 * dp - d0, d0, dp);
  const double dm4m = minmod4(4.0 * dm - d0, 4.0 * d0 - dm, dm, d0);
  const double uul = c + alpha * (c - b);
  const double uav = 0.5 * (c + d);
  const double umd = uav - 0.5 * dm4p;
  const double ulc = c + 0.5 * (c - b) + (4.0 / 3.0) * dm4m;
  const double umin = fmax(fmin(fmin(c, d), umd), fmin(fmin(c, uul), ulc));
  const double umax = fmin(fmax(fmax(c, d), umd), fmax(fmax(c, uul), ulc));
  return uor + minmod2(umin - uor, umax - uor);
}

// PPM (Colella & Woodward 1984; named in section 3), uniform grid, no
// steepening or flattening: the value of cell c (neighbours a, b and d, e)
// at its face toward d.  Interfaces b|c and c|d from the fourth-order
// interpolant with MC slopes; the parabola is flat at a local extremum, and
// where it would overshoot on the d side its b-side value is what moves the
// d-side value (to 3c - 2 a_L).
__device__ __forceinline__ double ppm_face(double a, double b, double c, double d, double e) {
  const double sb = mc_slope(a, b, c), sc = mc_slope(b, c, d), sd = mc_slope(c, d, e);
  const double aL = 0.5 * (b + c) - (sc - sb) * (1.0 / 6.0);
  const double aR = 0.5 * (c + d) - (sd - sc) * (1.0 / 6.0);
  const double dq = aR - aL, m = c - 0.5 * (aL + aR);
  const double r = (dq * dq * (-1.0 / 6.0) > dq * m) ? 3.0 * c - 2.0 * aL : aR;
  return ((aR - c) * (c - aL) <= 0.0) ? c : r;
}

// Conserved vector U, flux F along direction D and the two wave-speed bounds
// of one primitive state at one point (section 2.1 and 2.3).  g1, g2: the
// reference metric diagonal (the first entry is 1 in every coordinate
// system used here).
template <int D>
__device__ __forceinline__ void state_flux(const double gam, const double gfac, const double *pr, double psi4,
                                           double psi6, double alpha, const double *beta, double g1, double g2,
                                           double gud, double *U, double *F, double &lm, double &lp) {
  const double gd[3] = {psi4, psi4 * g1, psi4 * g2};
  const double u2 = gd[0] * pr[1] * pr[1] + gd[1] * pr[2] * pr[2] + gd[2] * pr[3] * pr[3];
  const double W2 = 1.0 + u2;
  const double iW = rsq(W2);
  const double W = W2 * iW;
  double v[3], vd[3], Bd[3];
  double Bv = 0.0, BB = 0.0;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    v[a] = pr[1 + a] * iW;
    vd[a] = gd[a] * v[a];
    Bd[a] = gd[a] * pr[5 + a];
    Bv += pr[5 + a] * vd[a];
    BB += pr[5 + a] * Bd[a];
  }
  const double ab0 = W * Bv;  // alpha b^0
  double bd[3];
#pragma unroll
  for (int a = 0; a < 3; a++) bd[a] = Bd[a] * iW + ab0 * vd[a];
  const double b2 = BB * iW * iW + Bv * Bv;
  const double rho = pr[0], p = pr[4];
  const double rhoh = rho + gfac * p;
  const double rhohs = rhoh + b2;
  const double ps = p + 0.5 * b2;
  const double E = rhohs * W2;
  const double Dn = rho * W;
  U[0] = psi6 * Dn;
#pragma unroll
  for (int a = 0; a < 3; a++) U[1 + a] = psi6 * (E * vd[a] - ab0 * bd[a]);
  U[4] = psi6 * (E - ps - ab0 * ab0 - Dn);
#pragma unroll
  for (int a = 0; a < 3; a++) U[5 + a] = psi6 * pr[5 + a];

  const double vhd = alpha * v[D] - beta[D];
  const double Bdir = pr[5 + D];
  const double aBW = alpha * Bdir * iW;
  F[0] = U[0] * vhd;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    double f = U[1 + a] * vhd - psi6 * aBW * bd[a];
    if (a == D) f += psi6 * alpha * ps;
    F[1 + a] = f;
  }
  F[4] = U[4] * vhd + psi6 * (alpha * ps * v[D] - ab0 * aBW);
#pragma unroll
  for (int a = 0; a < 3; a++) {
    const double vha = alpha * v[a] - beta[a];
    F[5 + a] = (a == D) ? 0.0 : psi6 * (vhd * pr[5 + a] - vha * Bdir);
  }

  // wave-speed bounds: a^2 = cs^2 + ca^2 - cs^2 ca^2 (section 2.3), with
  // cs^2 = Gamma p / (rho h) and ca^2 = b^2 / (rho h*) from one reciprocal
  const double t = rcp(rhoh * rhohs);
  const double c_s2 = gam * p * rhohs * t;
  const double c_a2 = b2 * rhoh * t;
  const double a2 = c_s2 + c_a2 - c_s2 * c_a2;
  const double v2 = v[0] * vd[0] + v[1] * vd[1] + v[2] * vd[2];
  const double one_a2 = 1.0 - a2;
  const double va = v[D];
  const double va2a = 1.0 - v2 * a2;
  const double sq = sqrt_pos(a2 * (1.0 - v2) * (va2a * gud - one_a2 * va * va));
  const double iden = rcp(va2a);
  lm = alpha * ((one_a2 * va - sq) * iden) - beta[D];
  lp = alpha * ((one_a2 * va + sq) * iden) - beta[D];
}

// Conserved vector of one point (prim2con), with the same arithmetic.
__device__ __forceinline__ void prim_to_cons(double gam, double gfac, const double *pr, double psi, double alpha,
                                             const double *beta, double g1, double g2, double *U) {
  const double psi2 = psi * psi, psi4 = psi2 * psi2;
  double F[NV], lm, lp;
  state_flux<0>(gam, gfac, pr, psi4, psi4 * psi2, alpha, beta, g1, g2, rcp(psi4), U, F, lm, lp);
}

// CFL rate of one cell: sum over the active axes of max|lambda_a| / dx_a
// (section 2.9, maxsum), wave speeds as in section 2.3.
__device__ __forceinline__ double cfl_rate(const double gam, const double gfac, const double *pr, double psi,
                                           double alpha, const double *beta, double g1, double g2, int ndim,
                                           const double *idx) {
  const double psi2 = psi * psi, psi4 = psi2 * psi2;
  const double gd[3] = {psi4, psi4 * g1, psi4 * g2};
  const double W2 = 1.0 + gd[0] * pr[1] * pr[1] + gd[1] * pr[2] * pr[2] + gd[2] * pr[3] * pr[3];
  const double iW = rsq(W2);
  double v[3], Bv = 0.0, BB = 0.0, v2 = 0.0;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    v[a] = pr[1 + a] * iW;
    Bv += pr[5 + a] * gd[a] * v[a];
    BB += pr[5 + a] * gd[a] * pr[5 + a];
    v2 += v[a] * gd[a] * v[a];
  }
  const double b2 = BB * iW * iW + Bv * Bv;
  const double rhoh = pr[0] + gfac * pr[4];
  const double t = rcp(rhoh * (rhoh + b2));
  const double c_s2 = gam * pr[4] * (rhoh + b2) * t;
  const double c_a2 = b2 * rhoh * t;
  const double a2 = c_s2 + c_a2 - c_s2 * c_a2;
  const double one_a2 = 1.0 - a2;
  const double va2a = 1.0 - v2 * a2;
  const double iden = rcp(va2a);
  double rate = 0.0;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    if (a < ndim) {
      const double sq = sqrt_pos(a2 * (1.0 - v2) * (va2a * rcp(gd[a]) - one_a2 * v[a] * v[a]));
      const double lm = alpha * ((one_a2 * v[a] - sq) * iden) - beta[a];
      const double lp = alpha * ((one_a2 * v[a] + sq) * iden) - beta[a];
      rate += fmax(fabs(lm), fabs(lp)) * idx[a];
    }
  }
  return rate;
}

}  // namespace gm

namespace gm {

// Rescaled conserved quantities of one cell (section 2.5.2, step 1).
struct C2PConst {
  double D, q, r2, b2, rb, rpb2, v0sq;
};

// Evaluation of the master function at mu (section 2.5.2, step 3), with
// rho and eps limited to the EOS range inside the evaluation.  Optionally
// returns W and the unlimited rho, eps.
__device__ __forceinline__ double c2p_master(const Grid &G, const C2PConst &c, double mu, double *Wout,
                                             double *rho_raw, double *eps_raw, double *chi_out) {
  const double chi = rcp(1.0 + mu * c.b2);
  const double rbar2 = c.r2 * chi * chi + mu * chi * (1.0 + chi) * c.rb * c.rb;
  const double qbar = c.q - 0.5 * c.b2 - 0.5 * mu * mu * chi * chi * c.rpb2;
  const double vh2 = fmin(mu * mu * rbar2, c.v0sq);
  const double iWh = sqrt_pos(1.0 - vh2);  // 1 / W_hat
  const double Wh = rcp(iWh);
  const double rho_r = c.D * iWh;
  const double eps_r = Wh * (qbar - mu * rbar2) + vh2 * Wh * Wh * rcp(1.0 + Wh);
  if (Wout) {
    *Wout = Wh;
    *rho_raw = rho_r;
    *eps_raw = eps_r;
    *chi_out = chi;
  }
  const double rho = fmax(fmin(G.rho_max, rho_r), G.rho_atmo);
  const double eps = fmax(fmin(G.eps_max, eps_r), 0.0);
  // ideal gas: a = p / (rho (1 + eps)) = (Gamma - 1) eps / (1 + eps)
  const double ah = G.gm1 * eps * rcp(1.0 + eps);
  const double nuA = (1.0 + ah) * (1.0 + eps) * iWh;
  const double nuB = (1.0 + ah) * (1.0 + qbar - mu * rbar2);
  const double nu = fmax(nuA, nuB);
  (void)rho;
  return mu - rcp(nu + mu * rbar2);
}

// f_a(mu) = mu sqrt(1 + rbar^2(mu)) - 1 (h0 = 1 for the ideal gas) and its
// derivative (section 2.5.2, step 2).
__device__ __forceinline__ double c2p_fa(const C2PConst &c, double mu, double &df) {
  const double chi = rcp(1.0 + mu * c.b2);
  const double dchi = -c.b2 * chi * chi;
  const double rb2 = c.rb * c.rb;
  const double rbar2 = c.r2 * chi * chi + mu * chi * (1.0 + chi) * rb2;
  const double drbar2 = 2.0 * c.r2 * chi * dchi + rb2 * (chi + chi * chi + mu * dchi * (1.0 + 2.0 * chi));
  const double isq = rsq(1.0 + rbar2);
  const double sq = (1.0 + rbar2) * isq;
  df = sq + 0.5 * mu * drbar2 * isq;
  return mu * sq - 1.0;
}

// Regula falsi with the Illinois modification on a sign-changing bracket.
// Returns the final iterate; sets ok = false when maxit is reached.
template <typename Fn>
__device__ __forceinline__ double illinois_root(Fn f, double lo, double hi, double flo, double fhi, double tol,
                                                int maxit, int &iters, bool &ok) {
  // invariant: f(x_old) and f(x_new) bracket the root
  double xa = lo, fa = flo, xb = hi, fb = fhi;
  ok = true;
  iters = 0;
  for (int it = 0; it < maxit; ++it) {
    const double xc = xb - fb * (xb - xa) * rcp(fb - fa);
    const double fc = f(xc);
    iters = it + 1;
    if (fc == 0.0) return xc;
    if ((fc < 0.0) != (fb < 0.0)) {
      xa = xb;
      fa = fb;
    } else {
      fa *= 0.5;
    }
    xb = xc;
    fb = fc;
    if (fabs(xb - xa) <= tol * fabs(xb)) return xb;
  }
  ok = false;
  return xb;
}

// Error handling after a recovery (section 2.5.3), shared by both schemes:
// atmosphere below rho_min, EOS limits, the velocity limit W_max (rescaled
// only in the low-density or black-hole region, else fatal).  capped: the
// recovery already had to cap the velocity, treated like W > W_max.  Writes
// pr[0..4] (pr[5..7] hold B already).
__device__ __forceinline__ int c2p_finish(const Grid &G, double D, double rho, double eps, double W, double *v,
                                          const double *gd, double alpha, int flags, bool capped, double *pr) {
  if (rho < G.rho_atmo) {
    pr[0] = G.rho_atmo;
    pr[1] = pr[2] = pr[3] = 0.0;
    pr[4] = G.p_atmo;
    return flags | FL_ATMO;
  }
  if (rho > G.rho_max) {
    flags |= FL_FRHO;
    rho = G.rho_max;
  }
  const bool soft = (rho < G.rho_low) || (alpha < G.alpha_bh);
  if (eps < 0.0) {
    eps = 0.0;
    flags |= FL_EPS;
  }
  if (eps > G.eps_max) {
    eps = G.eps_max;
    flags |= soft ? FL_EPS : FL_FEPS;
  }
  if (capped) flags |= soft ? FL_V : FL_FV;
  if (W > G.w_max) {
    if (soft) {
      const double vmax2 = 1.0 - rcp(G.w_max * G.w_max);
      const double v2 = gd[0] * v[0] * v[0] + gd[1] * v[1] * v[1] + gd[2] * v[2] * v[2];
      const double sc = sqrt(vmax2 * rcp(v2));
#pragma unroll
      for (int a = 0; a < 3; a++) v[a] *= sc;
      W = G.w_max;
      rho = fmax(fmin(D / W, G.rho_max), G.rho_atmo);
      eps = fmax(fmin(eps, G.eps_max), 0.0);
      flags |= FL_V;
    } else {
      flags |= FL_FV;
    }
  }
  pr[0] = rho;
  pr[1] = W * v[0];
  pr[2] = W * v[1];
  pr[3] = W * v[2];
  pr[4] = G.gm1 * rho * eps;
  return flags;
}

// Primitive recovery of one cell from densitised q (section 2.5.2) and the
// error handling of section 2.5.3.  Returns flag bits; pr receives the
// primitives (atmosphere / limited values where flagged).
__device__ __forceinline__ int c2p_cell(const Grid &G, const double *qc, double psi, double alpha, double g1,
                                        double g2, double *pr) {
  const double psi2 = psi * psi, psi4 = psi2 * psi2;
  const double ipsi6 = rcp(psi4 * psi2);
  const double gd[3] = {psi4, psi4 * g1, psi4 * g2};
  const double D = qc[0] * ipsi6;
  double B[3];
#pragma unroll
  for (int a = 0; a < 3; a++) B[a] = qc[5 + a] * ipsi6;
  pr[5] = B[0];
  pr[6] = B[1];
  pr[7] = B[2];
  if (!(D >= G.rho_atmo)) {  // rho <= D, so rho < rho_min already
    pr[0] = G.rho_atmo;
    pr[1] = pr[2] = pr[3] = 0.0;
    pr[4] = G.p_atmo;
    return FL_ATMO;
  }
  const double iD = rcp(D);
  const double isD = rsq(D);
  C2PConst c;
  c.D = D;
  c.q = qc[4] * ipsi6 * iD;
  double ru[3], Bc[3];
  c.r2 = 0.0;
  c.b2 = 0.0;
  c.rb = 0.0;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    const double rd = qc[1 + a] * ipsi6 * iD;
    ru[a] = rd * rcp(gd[a]);
    Bc[a] = B[a] * isD;
    c.r2 += ru[a] * rd;
    c.b2 += gd[a] * Bc[a] * Bc[a];
    c.rb += rd * Bc[a];
  }
  c.rpb2 = fmax(c.b2 * c.r2 - c.rb * c.rb, 0.0);
  c.v0sq = c.r2 * rcp(1.0 + c.r2);

  // step 2: mu_+ by Newton-Raphson from 1/h0 = 1, Illinois as the fallback
  double mup = 1.0;
  {
    double mu = 1.0;
    bool good = false;
    for (int it = 0; it < 60; ++it) {
      double df;
      const double fv = c2p_fa(c, mu, df);
      if (fv == 0.0) {
        good = true;
        break;
      }
      const double mn = mu - fv * rcp(df);
      if (!(mn > 0.0 && mn <= 1.0)) break;
      if (fabs(mn - mu) <= 1e-15 * mn) {
        mu = mn;
        good = true;
        break;
      }
      mu = mn;
    }
    if (!good) {
      int its;
      bool ok;
      double dd;
      auto fa = [&](double x) { return c2p_fa(c, x, dd); };
      mu = illinois_root(fa, 0.0, 1.0, -1.0, fa(1.0), 1e-15, 200, its, ok);
    }
    mup = mu;
  }

  // step 3: root of the master function on (0, mu_+]
  int flags = 0;
  double mu;
  {
    auto f = [&](double x) { return c2p_master(G, c, x, nullptr, nullptr, nullptr, nullptr); };
    const double fhi = f(mup);
    if (fhi <= 0.0) {
      mu = mup;
    } else {
      const double flo = f(0.0);
      int its;
      bool ok;
      mu = illinois_root(f, 0.0, mup, flo, fhi, G.tol, G.maxit, its, ok);
      if (!ok) flags |= FL_NOCONV;
    }
  }

  // step 4: primitives at the root
  double W, rho, eps, chi;
  c2p_master(G, c, mu, &W, &rho, &eps, &chi);
  double v[3];
#pragma unroll
  for (int a = 0; a < 3; a++) v[a] = mu * chi * (ru[a] + mu * c.rb * Bc[a]);
  return c2p_finish(G, D, rho, eps, W, v, gd, alpha, flags, false, pr);
}

// GRHD recovery (section 2.5.1): f(z) = z - r / h(z) with z = W v,
// W = sqrt(1 + z^2), rho = D / W, eps = W q - z r + z^2 / (1 + W) limited
// to the EOS range inside each evaluation; for the ideal gas
// h = (1 + eps)(1 + a) = 1 + Gamma eps.
__device__ __forceinline__ double z_master(const Grid &G, double D, double r, double q, double z, double *Wout,
                                           double *rho_raw, double *eps_raw, double *h_out) {
  const double z2 = z * z;
  const double iW = rsq(1.0 + z2);
  const double W = (1.0 + z2) * iW;
  const double eps_r = W * q - z * r + z2 * rcp(1.0 + W);
  const double eps = fmax(fmin(G.eps_max, eps_r), 0.0);
  const double h = 1.0 + G.gam * eps;
  if (Wout) {
    *Wout = W;
    *rho_raw = D * iW;
    *eps_raw = eps_r;
    *h_out = h;
  }
  return z - r * rcp(h);
}

// Primitive recovery of one cell by the z-scheme (B is passed through: the
// scheme is for B = 0) and the error handling of section 2.5.3.
__device__ __forceinline__ int c2p_cell_z(const Grid &G, const double *qc, double psi, double alpha, double g1,
                                          double g2, double *pr) {
  const double psi2 = psi * psi, psi4 = psi2 * psi2;
  const double ipsi6 = rcp(psi4 * psi2);
  const double gd[3] = {psi4, psi4 * g1, psi4 * g2};
  const double D = qc[0] * ipsi6;
#pragma unroll
  for (int a = 0; a < 3; a++) pr[5 + a] = qc[5 + a] * ipsi6;
  if (!(D >= G.rho_atmo)) {
    pr[0] = G.rho_atmo;
    pr[1] = pr[2] = pr[3] = 0.0;
    pr[4] = G.p_atmo;
    return FL_ATMO;
  }
  const double tau = qc[4] * ipsi6;
  double Su[3], S2 = 0.0;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    const double Sd = qc[1 + a] * ipsi6;
    Su[a] = Sd * rcp(gd[a]);
    S2 += Su[a] * Sd;
  }
  const double S = sqrt_pos(S2);
  const double iD = rcp(D);
  const double r = S * iD, q = tau * iD;
  double k = S * rcp(tau + D);
  // beyond the k of W = W_max (or k >= 1: no finite W) the state is taken at
  // that limit and flagged like W > W_max
  const double kmax = sqrt_pos(1.0 - rcp(G.w_max * G.w_max));
  const bool capped = !(k <= kmax);
  if (capped) k = kmax;
  const double zm = 0.5 * k * rsq(1.0 - 0.25 * k * k);
  const double zp = k * rsq(1.0 - k * k);
  auto f = [&](double z) { return z_master(G, D, r, q, z, nullptr, nullptr, nullptr, nullptr); };
  int flags = 0;
  double z;
  const double fm = f(zm), fp = f(zp);
  if (fp == 0.0) {
    z = zp;
  } else if (fm == 0.0) {
    z = zm;
  } else if ((fm < 0.0) == (fp < 0.0)) {
    flags |= FL_NOCONV;
    z = fabs(fm) < fabs(fp) ? zm : zp;
  } else {
    int its;
    bool ok;
    z = illinois_root(f, zm, zp, fm, fp, G.tol, G.maxit, its, ok);
    if (!ok) flags |= FL_NOCONV;
  }
  double W, rho, eps, h;
  z_master(G, D, r, q, z, &W, &rho, &eps, &h);
  const double s = iD * rcp(h * W);
  double v[3] = {Su[0] * s, Su[1] * s, Su[2] * s};
  return c2p_finish(G, D, rho, eps, W, v, gd, alpha, flags, capped, pr);
}

// Recovery by the scheme the grid selects.
__device__ __forceinline__ int c2p_any(const Grid &G, const double *qc, double psi, double alpha, double g1,
                                       double g2, double *pr) {
  return G.c2p == GMUNU_C2P_GRHD_Z ? c2p_cell_z(G, qc, psi, alpha, g1, g2, pr)
                                   : c2p_cell(G, qc, psi, alpha, g1, g2, pr);
}

}  // namespace gm
