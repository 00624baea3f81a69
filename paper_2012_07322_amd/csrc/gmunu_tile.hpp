// Tile-level device routines shared by the single-grid and batched kernels:
// face fluxes (MC, MP5 or PPM reconstruction; HLLE or TVDLF; the
// positivity-preserving limiter), sources, the fused stage on one tile, and
// the per-cell recovery, ghost fill and CFL rate.  Cheong et al., "Gmunu"
// (arXiv 2012.07322): section 2.1 (fluxes, sources, update), section 2.3,
// section 2.4, section 2.5, section 2.9, section 3 (solver settings),
// Appendix A.
#pragma once

#include <hip/hip_runtime.h>

#include "gmunu_dev.hpp"

namespace gm {

constexpr double kTiny = 1e-300;
constexpr int kCflParts = 2048;  // workgroups of the CFL reduction

// Stencil halo of a reconstruction: cells on each side of a face that its
// states depend on (MC 2; MP5 and PPM 3).
constexpr int recon_halo(int rec) { return rec == GMUNU_RECON_MC ? 2 : 3; }

// Load variable v at byte offset ob from a tile base (scalar base, 32-bit
// per-lane offset).
__device__ __forceinline__ double ld(const double *__restrict__ base, long nv, int v, unsigned ob) {
  return *reinterpret_cast<const double *>(reinterpret_cast<const char *>(base + v * nv) + ob);
}

// What the positivity-preserving limiter needs besides the staged states:
// the conserved state the stage's Euler step starts from and the step.
struct PPBase {
  const double *q;  // base conserved state (q_n in the first stage, q_s after)
  double dt;
};

// theta of one conserved component on one side of a face (section 2.4): the
// largest weight of the high-order flux for which the one-sided Euler update
// u + sgn w F stays above eps, 1 when the high-order flux already keeps it
// there.  w = 2 dt / cv_D of the cell, sgn = -1 below the face, +1 above; fho,
// flf are the high-order and Lax-Friedrichs fluxes times the face factor.
__device__ __forceinline__ double pp_side(double u, double w, double fho, double flf, double sgn) {
  constexpr double eps = 1e-16;
  if (u + sgn * w * fho > eps) return 1.0;
  const double den = sgn * w * (flf - fho);
  if (den == 0.0) return 1.0;
  return ((u - eps) + sgn * w * flf) / den;
}

// Where the stage kernel takes the metric from: staged in LDS with the
// primitives (kMetLds), or read from memory by each face and cell; and
// whether the conserved state of the RK combination is loaded at the start
// of a tile (kPrefetchQ) or at its end.
#ifndef GM_MET_LDS
#define GM_MET_LDS 1
#endif
#ifndef GM_PREFETCH_Q
#define GM_PREFETCH_Q 0
#endif
constexpr bool kMetLds = GM_MET_LDS;
constexpr bool kPrefetchQ = GM_PREFETCH_Q;

// Plus-shaped staged region of a TX x TY x TZ tile: the tile's cells and,
// along each active axis, H cells on both sides of the tile (no edge or
// corner cells: the face fluxes have no transverse stencil and the metric
// derivatives are centred along one axis).  Seven boxes, each x-fastest:
// centre (TX, TY, TZ), x-lo and x-hi (H, TY, TZ), y-lo and y-hi (TX, H, TZ),
// z-lo and z-hi (TX, TY, H).  LDS holds the NV primitives of every region
// cell, variable-major, then (kMetLds) the 5 metric variables of the region
// of halo met_halo() (met_index).
template <int TX, int TY, int TZ, int ND, int H>
struct Plus {
  static constexpr int HY = ND > 1 ? H : 0, HZ = ND > 2 ? H : 0;
  static constexpr int NC = TX * TY * TZ, NXB = H * TY * TZ, NYB = TX * HY * TZ, NZB = TX * TY * HZ;
  static constexpr int XL = NC, XH = XL + NXB, YL = XH + NXB, YH = YL + NYB, ZL = YH + NYB, ZH = ZL + NZB;
  static constexpr int N = ZH + NZB;
};

// Tile-relative coordinates of region cell c.
template <int TX, int TY, int TZ, int ND, int H>
__device__ __forceinline__ void plus_cell(int c, int &x, int &y, int &z) {
  using P = Plus<TX, TY, TZ, ND, H>;
  if (c < P::XL) {
    x = c % TX;
    y = (c / TX) % TY;
    z = c / (TX * TY);
  } else if (c < P::YL) {
    const bool hi = c >= P::XH;
    const int l = c - (hi ? P::XH : P::XL);
    x = l % H + (hi ? TX : -H);
    y = (l / H) % TY;
    z = l / (H * TY);
  } else if (c < P::ZL) {
    const bool hi = c >= P::YH;
    const int l = c - (hi ? P::YH : P::YL);
    x = l % TX;
    y = (l / TX) % H + (hi ? TY : -H);
    z = l / (TX * H);
  } else {
    const bool hi = c >= P::ZH;
    const int l = c - (hi ? P::ZH : P::ZL);
    x = l % TX;
    y = (l / TX) % TY;
    z = l / (TX * TY) + (hi ? TZ : -H);
  }
}

// Region index of the cell at tile-relative position s along D, with the
// other two coordinates of (x, y, z) inside the tile.
template <int TX, int TY, int TZ, int ND, int H, int D>
__device__ __forceinline__ int plus_line(int s, int x, int y, int z) {
  using P = Plus<TX, TY, TZ, ND, H>;
  if constexpr (D == 0) {
    const int t = y + TY * z;
    return s < 0 ? P::XL + (s + H) + H * t : s < TX ? s + TX * t : P::XH + (s - TX) + H * t;
  } else if constexpr (D == 1) {
    return s < 0 ? P::YL + x + TX * ((s + H) + H * z)
                 : s < TY ? x + TX * (s + TY * z) : P::YH + x + TX * ((s - TY) + H * z);
  } else {
    return s < 0 ? P::ZL + x + TX * (y + TY * (s + H))
                 : s < TZ ? x + TX * (y + TY * s) : P::ZH + x + TX * (y + TY * (s - TZ));
  }
}

// The metric is staged on the plus region of halo MH: MH = H (the
// primitives' region, same indices) or MH = 1, which is all that is read (a
// face takes the metric of its two adjacent cells and the sources'
// derivatives are centred).  Index in the metric's region of region cell c
// at tile-relative (x, y, z), or -1 for a cell beyond MH; the centre box has
// the same indices in both regions.
template <int TX, int TY, int TZ, int ND, int H, int MH>
__device__ __forceinline__ int met_index(int c, int x, int y, int z) {
  static_assert(MH == H || MH == 1, "the metric is staged on the primitives' region or on halo 1");
  if constexpr (MH == H) {
    return c;
  } else {
    if (x >= 0 && x < TX && y >= 0 && y < TY && z >= 0 && z < TZ) return x + TX * (y + TY * z);
    if (x == -1 || x == TX) return plus_line<TX, TY, TZ, ND, 1, 0>(x, x, y, z);
    if (y == -1 || y == TY) return plus_line<TX, TY, TZ, ND, 1, 1>(y, x, y, z);
    if (z == -1 || z == TZ) return plus_line<TX, TY, TZ, ND, 1, 2>(z, x, y, z);
    return -1;
  }
}

// Face flux times face factor through the lower face (along D) of cell
// (i,j,k): reconstruction REC from the cells across the face (MC from four
// cells, halo H = 2; MP5 or PPM from six, H = 3), metric as the mean of the
// two adjacent centres, HLLE (R = 0) or TVDLF (R = 1).  The stencil comes
// from the workgroup's staged region S (NP cells per variable, primitive
// variables 0-7): ix[m], m = 0 .. 2H-1, is the region index of the cell
// H - m below the face (ix[H-1], ix[H] are the two adjacent cells, whose
// metric (psi, alpha, beta^1..3) is ma, mb).  nonflat is set when the two
// adjacent cells differ in psi or alpha or either has a non-zero shift.
//
// P = 1 applies the positivity-preserving limiter (section 2.4): the flux is
// blended with the first-order Lax-Friedrichs flux of the two adjacent cell
// states, with the largest theta that keeps D and tau of the Euler update of
// both adjacent interior cells above eps (ghost cells are not advanced and do
// not take part).
template <int D, int REC, int R, int P = 0>
__device__ __forceinline__ void face_flux(const Grid &G, const double *S, int NP, const int *ix, const double *ma,
                                          const double *mb, int i, int j, int k, double *Fo, bool &nonflat,
                                          const PPBase &pb = PPBase{nullptr, 0.0}) {
  constexpr int H = recon_halo(REC);
  const int cd = (D == 0 ? i : D == 1 ? j : k) + G.g[D];
  // zero-area faces (r = 0, theta = 0 or pi) are evaluated like any other
  // and their flux replaced by 0 at the end; no load-dependent branch here
  const double fa = G.geo.fa[D][cd];
  const int r1 = ix[H - 1], r2 = ix[H];
  double pl[NV], pr[NV];
  if constexpr (REC == GMUNU_RECON_MC) {
#pragma unroll
    for (int v = 0; v < NV; v++) {
      const double *Sv = S + v * NP;
      const double a = Sv[ix[0]], b = Sv[r1], e = Sv[r2], f = Sv[ix[3]];
      pl[v] = b + mc_half_slope(a, b, e);
      pr[v] = e - mc_half_slope(b, e, f);
    }
  } else {
#pragma unroll
    for (int v = 0; v < NV; v++) {
      const double *Sv = S + v * NP;
      const double u0 = Sv[ix[0]], u1 = Sv[ix[1]], u2 = Sv[ix[2]], u3 = Sv[ix[3]], u4 = Sv[ix[4]], u5 = Sv[ix[5]];
      if constexpr (REC == GMUNU_RECON_MP5) {
        pl[v] = mp5_face(u0, u1, u2, u3, u4);
        pr[v] = mp5_face(u5, u4, u3, u2, u1);
      } else {
        pl[v] = ppm_face(u0, u1, u2, u3, u4);
        pr[v] = ppm_face(u5, u4, u3, u2, u1);
      }
    }
    // a reconstructed state without positive density and pressure: both
    // sides fall back to the adjacent cell values
    if (!(pl[0] > 0.0 && pl[4] > 0.0 && pr[0] > 0.0 && pr[4] > 0.0)) {
#pragma unroll
      for (int v = 0; v < NV; v++) {
        pl[v] = S[v * NP + r1];
        pr[v] = S[v * NP + r2];
      }
    }
  }
  const double psi = 0.5 * (ma[0] + mb[0]);
  const double alpha = 0.5 * (ma[1] + mb[1]);
  double beta[3];
  bool shift = false;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    beta[a] = 0.5 * (ma[2 + a] + mb[2 + a]);
    shift = shift || ma[2 + a] != 0.0 || mb[2 + a] != 0.0;
  }
  nonflat = nonflat || shift || ma[0] != mb[0] || ma[1] != mb[1];
  double g1 = 1.0, g2 = 1.0;
  if (G.coord != CART) {
    const double r2c = (D == 0) ? G.geo.r2f[i + G.g[0]] : G.geo.r2c[i + G.g[0]];
    const double s2 = (D == 1) ? G.geo.s2f[j + G.g[1]] : G.geo.s2c[j + G.g[1]];
    ref_diag(G.coord, r2c, s2, g1, g2);
  }
  const double psi2 = psi * psi, psi4 = psi2 * psi2, psi6 = psi4 * psi2;
  const double gD = D == 0 ? 1.0 : D == 1 ? g1 : g2;
  const double gud = rcp(psi4 * gD);
  // both sides share the face metric, so the densitising factor psi^6 of U
  // and F is taken out of the two states and applied once to the flux,
  // together with the face factor
  const double fs = fa * psi6;
  double UL[NV], FL[NV], UR[NV], FR[NV], lmL, lpL, lmR, lpR;
  state_flux<D>(G.gam, G.gfac, pl, psi4, 1.0, alpha, beta, g1, g2, gud, UL, FL, lmL, lpL);
  state_flux<D>(G.gam, G.gfac, pr, psi4, 1.0, alpha, beta, g1, g2, gud, UR, FR, lmR, lpR);
  if constexpr (R == GMUNU_RIEMANN_TVDLF) {
    // local Lax-Friedrichs: the largest speed magnitude of both states
    const double c = fmax(fmax(fabs(lmL), fabs(lpL)), fmax(fabs(lmR), fabs(lpR)));
    const double h = 0.5 * fs, hc = h * c;
#pragma unroll
    for (int v = 0; v < NV; v++) {
      const double f = h * (FL[v] + FR[v]) - hc * (UR[v] - UL[v]);
      Fo[v] = fa == 0.0 ? 0.0 : f;
    }
  } else {
    // HLLE as three weights: F = cL F_L + cR F_R + cU (U_R - U_L), with
    // cL = ap/(ap-am), cR = -am/(ap-am), cU = ap am/(ap-am); the mean of the
    // two fluxes when both speed bounds vanish
    const double ap = fmax(0.0, fmax(lpL, lpR));
    const double am = fmin(0.0, fmin(lmL, lmR));
    const double den = ap - am;
    const bool avg = den < kTiny;
    const double w = fs * rcp(avg ? 1.0 : den);
    const double cL = avg ? 0.5 * fs : ap * w;
    const double cR = avg ? 0.5 * fs : -am * w;
    const double cU = avg ? 0.0 : ap * am * w;
#pragma unroll
    for (int v = 0; v < NV; v++) {
      const double f = cL * FL[v] + cR * FR[v] + cU * (UR[v] - UL[v]);
      Fo[v] = fa == 0.0 ? 0.0 : f;
    }
  }
  if constexpr (P) {
    // zero-area faces carry no flux either way
    if (fa == 0.0) return;
    double p0[NV], p1[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) {
      p0[v] = S[v * NP + r1];
      p1[v] = S[v * NP + r2];
    }
    double U0[NV], F0[NV], U1[NV], F1[NV], lm0, lp0, lm1, lp1;
    state_flux<D>(G.gam, G.gfac, p0, psi4, psi6, alpha, beta, g1, g2, gud, U0, F0, lm0, lp0);
    state_flux<D>(G.gam, G.gfac, p1, psi4, psi6, alpha, beta, g1, g2, gud, U1, F1, lm1, lp1);
    const double c = fmax(fmax(fabs(lm0), fabs(lp0)), fmax(fabs(lm1), fabs(lp1)));
    double Fl[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) Fl[v] = (0.5 * (F0[v] + F1[v]) - 0.5 * c * (U1[v] - U0[v])) * fa;
    // the cells below (interior index cd - 1) and above (cd) the face
    const int cd = D == 0 ? i : D == 1 ? j : k;
    const bool in0 = cd >= 1, in1 = cd < G.n[D];
    const long o1 = cell_offset(G, i, j, k), o0 = o1 - G.s[D];
    const double w0 = in0 ? 2.0 * pb.dt * G.geo.icv[D][cd - 1 + G.g[D]] : 0.0;
    const double w1 = in1 ? 2.0 * pb.dt * G.geo.icv[D][cd + G.g[D]] : 0.0;
    double theta = 1.0;
#pragma unroll
    for (int m = 0; m < 2; m++) {
      const int v = m == 0 ? 0 : 4;  // D and tau
      if (in0) theta = fmin(theta, pp_side(pb.q[v * G.nv + o0], w0, Fo[v], Fl[v], -1.0));
      if (in1) theta = fmin(theta, pp_side(pb.q[v * G.nv + o1], w1, Fo[v], Fl[v], 1.0));
    }
    theta = fmin(fmax(theta, 0.0), 1.0);
    if (theta < 1.0) {
#pragma unroll
      for (int v = 0; v < NV; v++) Fo[v] = theta * Fo[v] + (1.0 - theta) * Fl[v];
    }
  }
}

// Gravitational sources (section 2.1) with centred metric derivatives, and
// geometric sources <Gamma^l_ik> (f_S_l)^k with cell-centre fluxes
// (Appendix A), added into s[].  pr: the cell's primitives; m(v, a, o): the
// metric variable v at the cell (a < 0) or at its neighbour o = -1 / +1
// along axis a.  flat: the caller knows every metric derivative of the cell
// is 0 and its shift is 0, so the gravitational sources vanish.  kij
// (nullable): the extrinsic curvature K_ij of the cell (6 components xx, xy,
// xz, yy, yz, zz, covariant; component m at kij[m * kst]); when null it
// follows from the shift by the CFC relation under maximal slicing.
template <typename MetFn>
__device__ __forceinline__ void cell_sources(const Grid &G, const double *pr, MetFn m, bool flat, const double *kij,
                                             long kst, int i, int j, double *s) {
  const bool geom = G.coord != CART;
  if (flat && !geom) return;
  const double psi = m(0, -1, 0), alpha = m(1, -1, 0);
  double beta[3];
#pragma unroll
  for (int a = 0; a < 3; a++) beta[a] = m(2 + a, -1, 0);
  double dpsi[3] = {0, 0, 0}, dal[3] = {0, 0, 0}, db[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  bool grav = !flat;
  if (grav) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
      if (a < G.ndim) {
        dpsi[a] = (m(0, a, 1) - m(0, a, -1)) * G.i2dx[a];
        dal[a] = (m(1, a, 1) - m(1, a, -1)) * G.i2dx[a];
#pragma unroll
        for (int c = 0; c < 3; c++) db[a][c] = (m(2 + c, a, 1) - m(2 + c, a, -1)) * G.i2dx[a];
      }
    }
  }

  double g1 = 1.0, g2 = 1.0;
  if (geom) ref_diag(G.coord, G.geo.r2c[i + G.g[0]], G.geo.s2c[j + G.g[1]], g1, g2);
  const double ref[3] = {1.0, g1, g2};
  const double psi2 = psi * psi, psi4 = psi2 * psi2, psi6 = psi4 * psi2;
  const double gd[3] = {psi4, psi4 * g1, psi4 * g2};
  const double W2 = 1.0 + gd[0] * pr[1] * pr[1] + gd[1] * pr[2] * pr[2] + gd[2] * pr[3] * pr[3];
  const double iW = rsq(W2), W = W2 * iW;
  double v[3], vd[3], vh[3];
  double Bv = 0.0, BB = 0.0;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    v[a] = pr[1 + a] * iW;
    vd[a] = gd[a] * v[a];
    vh[a] = alpha * v[a] - beta[a];
    Bv += pr[5 + a] * vd[a];
    BB += pr[5 + a] * gd[a] * pr[5 + a];
  }
  const double b2 = BB * iW * iW + Bv * Bv;
  const double rhohs = pr[0] + G.gfac * pr[4] + b2;
  const double ps = pr[4] + 0.5 * b2;
  const double ia = rcp(alpha);
  const double b0 = W * Bv * ia;

  if (grav) {
    // T^{mu nu} = rho h* u u + p* g^{mu nu} - b b in the coordinate basis
    const double u0 = W * ia;
    double ui[3], bi[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      ui[a] = W * vh[a] * ia;
      bi[a] = pr[5 + a] * iW + b0 * vh[a];
    }
    const double ia2 = ia * ia;
    const double T00 = rhohs * u0 * u0 - ps * ia2 - b0 * b0;
    double T0[3], T[3][3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      T0[a] = rhohs * u0 * ui[a] + ps * beta[a] * ia2 - b0 * bi[a];
#pragma unroll
      for (int c = 0; c < 3; c++)
        T[a][c] = rhohs * ui[a] * ui[c] + ps * ((a == c ? rcp(gd[a]) : 0.0) - beta[a] * beta[c] * ia2) -
                  bi[a] * bi[c];
    }
    // covariant derivative of the shift, nb[i][k] = d_i beta^k + Gamma^k_il
    // beta^l, with the non-zero point Christoffel symbols of the coordinate
    // system: cylindrical Gamma^R_phiphi = -R, Gamma^phi_Rphi = 1/R;
    // spherical Gamma^r_thth = -r, Gamma^r_phph = -r sin^2, Gamma^th_rth =
    // Gamma^ph_rph = 1/r, Gamma^th_phph = -sin cos, Gamma^ph_thph = cot
    double nb[3][3];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
      for (int c = 0; c < 3; c++) nb[a][c] = db[a][c];
    if (G.coord == CYL) {
      const double R = G.geo.xc0[i + G.g[0]], iR = rcp(R);
      nb[2][0] += -R * beta[2];
      nb[0][2] += iR * beta[2];
      nb[2][2] += iR * beta[0];
    } else if (G.coord == SPH) {
      const double r = G.geo.xc0[i + G.g[0]], ir = rcp(r);
      const double sn = G.geo.sc1[j + G.g[1]], cs = G.geo.cc1[j + G.g[1]], ct = cs * rcp(sn);
      nb[1][0] += -r * beta[1];
      nb[2][0] += -r * sn * sn * beta[2];
      nb[0][1] += ir * beta[1];
      nb[1][1] += ir * beta[0];
      nb[2][1] += -sn * cs * beta[2];
      nb[0][2] += ir * beta[2];
      nb[2][2] += ir * beta[0];
      nb[1][2] += ct * beta[2];
      nb[2][2] += ct * beta[1];
    }
    double K[3][3];
    if (kij) {
      const int map[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
#pragma unroll
      for (int a = 0; a < 3; a++)
#pragma unroll
        for (int c = 0; c < 3; c++) K[a][c] = kij[map[a][c] * kst];
    } else {
      const double divb = nb[0][0] + nb[1][1] + nb[2][2];
      const double kf = psi4 * 0.5 * ia;
#pragma unroll
      for (int a = 0; a < 3; a++)
#pragma unroll
        for (int c = 0; c < 3; c++)
          K[a][c] = kf * (ref[c] * nb[a][c] + ref[a] * nb[c][a] - (a == c ? (2.0 / 3.0) * ref[a] * divb : 0.0));
    }
    const double pre = alpha * psi6;
    const double fourpsi3 = 4.0 * psi2 * psi;
#pragma unroll
    for (int a = 0; a < 3; a++) {
      double sv = -T00 * alpha * dal[a];
#pragma unroll
      for (int c = 0; c < 3; c++) {
        const double T0low = gd[c] * (T00 * beta[c] + T0[c]);  // T^0_c
        sv += T0low * nb[a][c];
        sv += 0.5 * (T00 * beta[c] * beta[c] + 2.0 * T0[c] * beta[c] + T[c][c]) * fourpsi3 * dpsi[a] * ref[c];
      }
      s[1 + a] += pre * sv;
    }
    double Kbb = 0.0, bda = 0.0, TK = 0.0, T0K = 0.0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
      bda += beta[a] * dal[a];
      double Kb = 0.0;
#pragma unroll
      for (int c = 0; c < 3; c++) {
        Kbb += K[a][c] * beta[a] * beta[c];
        TK += T[a][c] * K[a][c];
        Kb += K[a][c] * beta[c];
      }
      T0K += T0[a] * (2.0 * Kb - dal[a]);
    }
    s[4] += pre * (T00 * (Kbb - bda) + T0K + TK);
  }

  if (geom) {
    // cell-centre momentum fluxes (f_S_l)^k = S_l vhat^k + delta alpha p* - alpha b_l B^k / W
    const double E = rhohs * W2;
    const double ab0 = alpha * b0;
    double bd[3], Sl[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      bd[a] = gd[a] * pr[5 + a] * iW + ab0 * vd[a];
      Sl[a] = E * vd[a] - ab0 * bd[a];
    }
    auto fS = [&](int l, int kk) {
      double f = Sl[l] * vh[kk] - alpha * bd[l] * pr[5 + kk] * iW;
      if (l == kk) f += alpha * ps;
      return psi6 * f;
    };
    // (branch-free accumulation keeps s[] in registers)
    const double gA = G.geo.gA[i + G.g[0]];
    const bool sph = G.coord == SPH;
    const double gB = sph ? G.geo.gB[i + G.g[0]] : 0.0, gC = sph ? G.geo.gC[j + G.g[1]] : 0.0;
    const double add1 = sph ? gA * fS(1, 1) + gA * fS(2, 2) : gA * fS(2, 2);
    const double add2 = sph ? gB * fS(0, 1) + gA * fS(1, 0) + gC * fS(2, 2) : 0.0;
    s[1] += add1;
    s[2] += add2;
  }
}

// Faces of the pass along D (the tile's lower faces plus the upper layer).
template <int TX, int TY, int TZ, int D>
constexpr int pass_faces() {
  return (TX + (D == 0)) * (TY + (D == 1)) * (TZ + (D == 2));
}

template <int TX, int TY, int TZ, int ND>
constexpr int max_faces() {
  constexpr int f0 = pass_faces<TX, TY, TZ, 0>(), f1 = ND > 1 ? pass_faces<TX, TY, TZ, 1>() : 0,
                f2 = ND > 2 ? pass_faces<TX, TY, TZ, 2>() : 0;
  return f0 > f1 ? (f0 > f2 ? f0 : f2) : (f1 > f2 ? f1 : f2);
}

// LDS doubles per workgroup: the staged region's primitives, the metric on
// the region of halo MH (kMetLds), and the face fluxes of one pass.
template <int TX, int TY, int TZ, int ND, int H, int MH>
constexpr int stage_lds_mh() {
  return NV * Plus<TX, TY, TZ, ND, H>::N + (kMetLds ? 5 * Plus<TX, TY, TZ, ND, MH>::N : 0) +
         NV * max_faces<TX, TY, TZ, ND>();
}

// The metric's halo: the primitives' (no index arithmetic of its own) when
// two workgroups then fit the 160 KB of LDS of a CU, else 1 (the 8x8x3 and
// 16x4x3 tiles among others, whose full regions would leave one workgroup
// per CU).
template <int TX, int TY, int TZ, int ND, int H>
constexpr int met_halo() {
  return stage_lds_mh<TX, TY, TZ, ND, H, H>() * 8 * 2 <= 160 * 1024 ? H : 1;
}

template <int TX, int TY, int TZ, int ND, int H = 2>
constexpr int stage_lds() {
  return stage_lds_mh<TX, TY, TZ, ND, H, met_halo<TX, TY, TZ, ND, H>()>();
}

// Workgroups per CU that the LDS of a tile shape allows (160 KB per CU), at
// most GM_MAX_OCC.
#ifndef GM_MAX_OCC
#define GM_MAX_OCC 2
#endif
template <int TX, int TY, int TZ, int ND, int H = 2>
constexpr int stage_occupancy() {
  constexpr int per = stage_lds<TX, TY, TZ, ND, H>() * 8;
  constexpr int n = (160 * 1024) / per;
  return n > GM_MAX_OCC ? GM_MAX_OCC : n < 1 ? 1 : n;
}

// Tile shapes whose passes have at most one face per thread.
template <int TX, int TY, int TZ, int ND>
constexpr bool tile_fits() {
  return pass_faces<TX, TY, TZ, 0>() <= NT && (ND < 2 || pass_faces<TX, TY, TZ, 1>() <= NT) &&
         (ND < 3 || pass_faces<TX, TY, TZ, 2>() <= NT) && TX * TY * TZ <= NT;
}

// The primitives (and with kMetLds the metric) of a tile's region in
// registers on their way to LDS: loaded for the whole region at once, so
// that it costs one memory latency, and possibly while the workgroup still
// computes the previous tile.
template <int TX, int TY, int TZ, int ND, int H>
struct RegionRegs {
  static constexpr int NP = Plus<TX, TY, TZ, ND, H>::N;
  static constexpr int NIT = (NP + NT - 1) / NT;
  static constexpr int NW = NV + (kMetLds ? 5 : 0);
  double val[NIT][NW];
  bool in[NIT];
};

// Load the region of the tile with origin (i0, j0, k0), coalesced, each
// value read once from memory.
template <int TX, int TY, int TZ, int ND, int H>
__device__ __forceinline__ void region_load(const Grid &G, const double *__restrict__ prim,
                                            const double *__restrict__ met, int i0, int j0, int k0,
                                            RegionRegs<TX, TY, TZ, ND, H> &R) {
  using RR = RegionRegs<TX, TY, TZ, ND, H>;
#pragma unroll
  for (int it = 0; it < RR::NIT; it++) {
    const int c = threadIdx.x + it * NT;
    int x, y, z;
    plus_cell<TX, TY, TZ, ND, H>(c, x, y, z);
    const int gi = i0 + x, gj = j0 + y, gk = k0 + z;
    // cells outside the array (ragged tiles) are not needed by any valid face
    R.in[it] = c < RR::NP && gi < G.n[0] + G.g[0] && gj < G.n[1] + G.g[1] && gk < G.n[2] + G.g[2];
    // every path defines every register, so that no earlier value of R
    // stays live across a caller's loop
    if (R.in[it]) {
      const long o = cell_offset(G, gi, gj, gk);
#pragma unroll
      for (int v = 0; v < NV; v++) R.val[it][v] = prim[v * G.nv + o];
      if constexpr (kMetLds) {
        const bool m = met_index<TX, TY, TZ, ND, H, met_halo<TX, TY, TZ, ND, H>()>(c, x, y, z) >= 0;
#pragma unroll
        for (int w = 0; w < 5; w++) R.val[it][NV + w] = m ? met[w * G.nv + o] : 0.0;
      }
    } else {
#pragma unroll
      for (int v = 0; v < RR::NW; v++) R.val[it][v] = 0.0;
    }
  }
}

// Write a loaded region into the workgroup's LDS buffer S.
template <int TX, int TY, int TZ, int ND, int H>
__device__ __forceinline__ void region_store(const RegionRegs<TX, TY, TZ, ND, H> &R, double *S) {
  using RR = RegionRegs<TX, TY, TZ, ND, H>;
  constexpr int MH = met_halo<TX, TY, TZ, ND, H>();
  constexpr int NPM = Plus<TX, TY, TZ, ND, MH>::N;
#pragma unroll
  for (int it = 0; it < RR::NIT; it++) {
    const int c = threadIdx.x + it * NT;
    if (R.in[it]) {
#pragma unroll
      for (int v = 0; v < NV; v++) S[v * RR::NP + c] = R.val[it][v];
      if constexpr (kMetLds) {
        int x = 0, y = 0, z = 0;
        if constexpr (MH != H) plus_cell<TX, TY, TZ, ND, H>(c, x, y, z);
        const int m = met_index<TX, TY, TZ, ND, H, MH>(c, x, y, z);
        if (m >= 0) {
#pragma unroll
          for (int w = 0; w < 5; w++) S[NV * RR::NP + w * NPM + m] = R.val[it][NV + w];
        }
      }
    }
  }
}

// Face fluxes of the pass along D into registers (one face per thread; zero
// for threads without a valid face).
template <int TX, int TY, int TZ, int ND, int D, int REC, int R, int P>
__device__ __forceinline__ void pass_fluxes(const Grid &G, const double *S, const double *__restrict__ met, int i0,
                                            int j0, int k0, double *Fo, bool &nonflat, const PPBase &pb) {
  constexpr int H = recon_halo(REC);
  constexpr int NP = Plus<TX, TY, TZ, ND, H>::N;
  constexpr int FX = TX + (D == 0), FY = TY + (D == 1), FZ = TZ + (D == 2), NF = FX * FY * FZ;
  const int f = threadIdx.x;
  const int fx = f % FX, fy = (f / FX) % FY, fz = f / (FX * FY);
  const int ci = i0 + fx, cj = j0 + fy, ck = k0 + fz;
  const bool ok = f < NF && (D == 0 ? ci <= G.n[0] : ci < G.n[0]) && (D == 1 ? cj <= G.n[1] : cj < G.n[1]) &&
                  (D == 2 ? ck <= G.n[2] : ck < G.n[2]);
  if (ok) {
    const int sd = D == 0 ? fx : D == 1 ? fy : fz;
    int ix[2 * H];
#pragma unroll
    for (int m = 0; m < 2 * H; m++) ix[m] = plus_line<TX, TY, TZ, ND, H, D>(sd - H + m, fx, fy, fz);
    double ma[5], mb[5];
    if constexpr (kMetLds) {
      constexpr int MH = met_halo<TX, TY, TZ, ND, H>();
      constexpr int NPM = Plus<TX, TY, TZ, ND, MH>::N;
      const double *Sm = S + NV * NP;
      const int ja = MH == H ? ix[H - 1] : plus_line<TX, TY, TZ, ND, MH, D>(sd - 1, fx, fy, fz);
      const int jb = MH == H ? ix[H] : plus_line<TX, TY, TZ, ND, MH, D>(sd, fx, fy, fz);
#pragma unroll
      for (int w = 0; w < 5; w++) {
        ma[w] = Sm[w * NPM + ja];
        mb[w] = Sm[w * NPM + jb];
      }
    } else {
      const long ob = cell_offset(G, ci, cj, ck), oa = ob - G.s[D];
#pragma unroll
      for (int w = 0; w < 5; w++) {
        ma[w] = met[w * G.nv + oa];
        mb[w] = met[w * G.nv + ob];
      }
    }
    face_flux<D, REC, R, P>(G, S, NP, ix, ma, mb, ci, cj, ck, Fo, nonflat, pb);
  } else {
#pragma unroll
    for (int v = 0; v < NV; v++) Fo[v] = 0.0;
  }
}

// The pass's fluxes through LDS (SF) into the flux divergence acc of the
// thread's cell.  On entry every thread has finished reading SF of the
// previous pass (the caller's barrier); on return other threads may still
// read SF.
template <int TX, int TY, int TZ, int D>
__device__ __forceinline__ void pass_divergence(const Grid &G, double *SF, const double *Fo, int i0, int j0, int k0,
                                                int tx, int ty, int tz, bool valid, double *acc) {
  constexpr int FX = TX + (D == 0), FY = TY + (D == 1), FZ = TZ + (D == 2), NF = FX * FY * FZ;
  const int f = threadIdx.x;
  if (f < NF) {
#pragma unroll
    for (int v = 0; v < NV; v++) SF[v * NF + f] = Fo[v];
  }
  __syncthreads();
  if (valid) {
    const int fl = tx + FX * (ty + FY * tz);
    const int fu = fl + (D == 0 ? 1 : D == 1 ? FX : FX * FY);
    const int cd = (D == 0 ? i0 + tx : D == 1 ? j0 + ty : k0 + tz) + G.g[D];
    const double icv = G.geo.icv[D][cd];
#pragma unroll
    for (int v = 0; v < NV; v++) acc[v] -= (SF[v * NF + fu] - SF[v * NF + fl]) * icv;
  }
}

// One RK stage (MODE 1: q_out = ca q_n + cb (q_s + dt L)) or the RHS alone
// (MODE 0: out = L) on the tile of TX x TY x TZ cells with origin (i0,j0,k0),
// whose region (the tile plus REC's halo along each active axis) the
// workgroup has just staged in sF (stage_lds<TX,TY,TZ,ND,recon_halo(REC)>()
// doubles; the staging ordered by a barrier).  The three face passes run
// from LDS, each followed by the exchange of its fluxes.  Every thread of the
// workgroup (NT threads) must call it (it synchronises; on return sF may be
// restaged).  kij (nullable): K_ij per cell, 6 arrays in the grid's layout.
// prefetch: called by every thread after the sources, before the loads of
// the RK combination (a persistent caller loads its next tile there).
struct NoPrefetch {
  __device__ void operator()() const {}
};

// Outputs of the primitive recovery when a stage does it in its epilogue
// (MODE 2): prim must not be the primitives the stage reads (neighbouring
// tiles still read those).
struct FusedC2P {
  double *prim;
  uint8_t *flags;         // nullable
  unsigned int *nfatal;   // nullable
};

template <int TX, int TY, int TZ, int ND, int MODE, int REC = 0, int R = 0, int P = 0, typename Pre = NoPrefetch>
__device__ __forceinline__ void stage_staged(const Grid &G, int i0, int j0, int k0, const double *__restrict__ met,
                                             const double *qn, const double *qs, double *out,
                                             const double *__restrict__ dtp, double ca, double cb, double *sF,
                                             const double *__restrict__ kij = nullptr, Pre prefetch = Pre{},
                                             FusedC2P fc = FusedC2P{nullptr, nullptr, nullptr}) {
  static_assert(tile_fits<TX, TY, TZ, ND>(), "tile passes must have at most one face per thread");
  static_assert(P == 0 || MODE == 1, "the limiter needs the stage's Euler step");
  static_assert(MODE != 2 || kMetLds, "the fused recovery takes psi and alpha from the staged region");
  constexpr int H = recon_halo(REC);
  constexpr int NP = Plus<TX, TY, TZ, ND, H>::N;
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = (tid / TX) % TY, tz = tid / (TX * TY);
  const int i = i0 + tx, j = j0 + ty, k = k0 + tz;
  const bool valid = tid < TX * TY * TZ && (i < G.n[0]) && (j < G.n[1]) && (k < G.n[2]);
  const long oc = valid ? cell_offset(G, i, j, k) : 0;
  // the conserved state of the RK combination (kPrefetchQ: loaded first)
  double un[NV], us[NV];
  if (MODE != 0 && kPrefetchQ && valid) {
#pragma unroll
    for (int v = 0; v < NV; v++) {
      un[v] = qn[v * G.nv + oc];
      us[v] = ca == 0.0 ? 0.0 : qs[v * G.nv + oc];
    }
  }
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; v++) acc[v] = 0.0;
  PPBase pp{nullptr, 0.0};
  if constexpr (P) pp = PPBase{ca == 0.0 ? qn : qs, *dtp};
  constexpr int MH = met_halo<TX, TY, TZ, ND, H>();
  constexpr int NPM = Plus<TX, TY, TZ, ND, MH>::N;
  double *SF = sF + NV * NP + (kMetLds ? 5 * NPM : 0);
  bool nonflat = false;
  double Fo[NV];
  pass_fluxes<TX, TY, TZ, ND, 0, REC, R, P>(G, sF, met, i0, j0, k0, Fo, nonflat, pp);
  pass_divergence<TX, TY, TZ, 0>(G, SF, Fo, i0, j0, k0, tx, ty, tz, valid, acc);
  if constexpr (ND > 1) {
    pass_fluxes<TX, TY, TZ, ND, 1, REC, R, P>(G, sF, met, i0, j0, k0, Fo, nonflat, pp);
    __syncthreads();  // every thread has summed the previous pass's fluxes
    pass_divergence<TX, TY, TZ, 1>(G, SF, Fo, i0, j0, k0, tx, ty, tz, valid, acc);
  }
  if constexpr (ND > 2) {
    pass_fluxes<TX, TY, TZ, ND, 2, REC, R, P>(G, sF, met, i0, j0, k0, Fo, nonflat, pp);
    __syncthreads();
    pass_divergence<TX, TY, TZ, 2>(G, SF, Fo, i0, j0, k0, tx, ty, tz, valid, acc);
  }
  // flat: no face of the tile joins cells of different psi or alpha, and no
  // cell has a shift, so every centred metric derivative of its cells is 0
  const bool flat = !__syncthreads_or(nonflat);
  if (valid) {
    const int c = tx + TX * (ty + TY * tz);
    double prc[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) prc[v] = sF[v * NP + c];
    const double *Sm = sF + NV * NP;
    auto metv = [&](int w, int a, int o) -> double {
      if (a >= ND) return 0.0;
      if constexpr (kMetLds) {
        if (a < 0) return Sm[w * NPM + c];
        const int p = a == 0 ? plus_line<TX, TY, TZ, ND, MH, 0>(tx + o, tx, ty, tz)
                             : a == 1 ? plus_line<TX, TY, TZ, ND, MH, 1>(ty + o, tx, ty, tz)
                                      : plus_line<TX, TY, TZ, ND, MH, 2>(tz + o, tx, ty, tz);
        return Sm[w * NPM + p];
      } else {
        return met[w * G.nv + oc + (a < 0 ? 0 : o * G.s[a])];
      }
    };
    cell_sources(G, prc, metv, flat && !kij, kij ? kij + oc : nullptr, G.nv, i, j, acc);
  }
  // the caller's loads (the next tile's region) go out together with the
  // loads of the RK combination, so that their latencies overlap
  prefetch();
  if (valid) {
    if (MODE == 0) {
#pragma unroll
      for (int v = 0; v < NV; v++) out[v * G.nv + oc] = acc[v];
    } else {
      if constexpr (!kPrefetchQ) {
#pragma unroll
        for (int v = 0; v < NV; v++) {
          un[v] = qn[v * G.nv + oc];
          us[v] = ca == 0.0 ? 0.0 : qs[v * G.nv + oc];
        }
      }
      const double dt = *dtp;
      double qo[NV];
#pragma unroll
      for (int v = 0; v < NV; v++)
        qo[v] = ca == 0.0 ? cb * (un[v] + dt * acc[v]) : ca * un[v] + cb * (us[v] + dt * acc[v]);
      if constexpr (MODE == 2) {
        // the recovery of the new state (c2p_one's arithmetic on the same
        // values: q from registers, psi and alpha from the staged region)
        const int c = tx + TX * (ty + TY * tz);
        const double *Sm = sF + NV * NP;
        const double psi = Sm[c], alpha = Sm[NPM + c];
        double g1 = 1.0, g2 = 1.0;
        if (G.coord != CART) ref_diag(G.coord, G.geo.r2c[i + G.g[0]], G.geo.s2c[j + G.g[1]], g1, g2);
        double pr[NV];
        const int fl = c2p_any(G, qo, psi, alpha, g1, g2, pr);
#pragma unroll
        for (int v = 0; v < NV; v++) fc.prim[v * G.nv + oc] = pr[v];
        if (fl & FL_REWRITE) {
          const double beta[3] = {Sm[2 * NPM + c], Sm[3 * NPM + c], Sm[4 * NPM + c]};
          prim_to_cons(G.gam, G.gfac, pr, psi, alpha, beta, g1, g2, qo);
        }
        if (fc.flags) fc.flags[oc] = (uint8_t)fl;
        if ((fl & FL_FATAL) && fc.nfatal) atomicAdd(fc.nfatal, 1u);
      }
#pragma unroll
      for (int v = 0; v < NV; v++) out[v * G.nv + oc] = qo[v];
    }
  }
  // a workgroup that takes another tile next restages sF: every thread must
  // have finished reading it
  __syncthreads();
}

// The same for a tile whose region is not staged yet: stage it, then the
// stage.
template <int TX, int TY, int TZ, int ND, int MODE, int REC = 0, int R = 0, int P = 0>
__device__ __forceinline__ void stage_tile(const Grid &G, int i0, int j0, int k0, const double *__restrict__ prim,
                                           const double *__restrict__ met, const double *qn, const double *qs,
                                           double *out, const double *__restrict__ dtp, double ca, double cb,
                                           double *sF, const double *__restrict__ kij = nullptr,
                                           FusedC2P fc = FusedC2P{nullptr, nullptr, nullptr}) {
  constexpr int H = recon_halo(REC);
  RegionRegs<TX, TY, TZ, ND, H> Rg;
  region_load<TX, TY, TZ, ND, H>(G, prim, met, i0, j0, k0, Rg);
  region_store<TX, TY, TZ, ND, H>(Rg, sF);
  __syncthreads();
  stage_staged<TX, TY, TZ, ND, MODE, REC, R, P>(G, i0, j0, k0, met, qn, qs, out, dtp, ca, cb, sF, kij, NoPrefetch{},
                                               fc);
}

// The face-adjacent ghosts of the first `axes` axes whose source is interior
// cell (i, j, k), written from that cell's primitives pr by ghost_one's
// rules: an outflow face copies its end cell into every layer, a periodic
// face takes layer l from the cell l in from the other end, a reflecting
// face from the cell l in from its own end with the axis's components of
// velocity and field negated.  Only for axes whose faces are periodic,
// outflow or reflecting and that hold at least ng cells (every source
// interior); each ghost has one source, so one thread writes it.
__device__ __forceinline__ void face_ghosts_from(const Grid &G, double *prim, const double *pr, int i, int j, int k,
                                                 int axes) {
  const long nv = G.nv;
  const int cell[3] = {i, j, k};
  for (int a = 0; a < axes; a++) {
    const int na = G.n[a], ng = G.g[a], ca = cell[a];
    for (int side = 0; side < 2; side++) {
      const int bc = G.bc[a][side];
      if (bc != BC_OUTFLOW && bc != BC_PERIODIC && bc != BC_REFLECT) continue;
      int l0, l1;  // layers [l0, l1) of this side sourced by the cell
      if (bc == BC_OUTFLOW) {
        if (ca != (side == 0 ? 0 : na - 1)) continue;
        l0 = 0;
        l1 = ng;
      } else {
        l0 = (bc == BC_PERIODIC) == (side == 0) ? na - 1 - ca : ca;
        if (l0 >= ng) continue;
        l1 = l0 + 1;
      }
      const double s = bc == BC_REFLECT ? -1.0 : 1.0;
      for (int l = l0; l < l1; l++) {
        const int gi = side == 0 ? -1 - l : na + l;
        const long cd = cell_offset(G, a == 0 ? gi : i, a == 1 ? gi : j, a == 2 ? gi : k);
        prim[cd] = pr[0];
        prim[4 * nv + cd] = pr[4];
#pragma unroll
        for (int m = 0; m < 3; m++) {
          prim[(1 + m) * nv + cd] = m == a ? s * pr[1 + m] : pr[1 + m];
          prim[(5 + m) * nv + cd] = m == a ? s * pr[5 + m] : pr[5 + m];
        }
      }
    }
  }
}

// Primitive recovery of interior cell number t (x fastest) of grid G; a
// fatal outcome increments *nfatal and *nfatal2 (each nullable).  gaxes:
// also write the face ghosts of the first gaxes axes that this cell is the
// source of (face_ghosts_from; 0: none).
__device__ __forceinline__ void c2p_one(const Grid &G, double *q, const double *__restrict__ met, double *prim,
                                        uint8_t *flags, unsigned int *nfatal, long t,
                                        unsigned int *nfatal2 = nullptr, int gaxes = 0) {
  const int i = (int)(t % G.n[0]);
  const int j = (int)((t / G.n[0]) % G.n[1]);
  const int k = (int)(t / ((long)G.n[0] * G.n[1]));
  const long c = cell_offset(G, i, j, k);
  double qc[NV], pr[NV];
#pragma unroll
  for (int v = 0; v < NV; v++) qc[v] = q[v * G.nv + c];
  double g1 = 1.0, g2 = 1.0;
  if (G.coord != CART) ref_diag(G.coord, G.geo.r2c[i + G.g[0]], G.geo.s2c[j + G.g[1]], g1, g2);
  const double psi = met[c], alpha = met[G.nv + c];
  const int fl = c2p_any(G, qc, psi, alpha, g1, g2, pr);
#pragma unroll
  for (int v = 0; v < NV; v++) prim[v * G.nv + c] = pr[v];
  if (gaxes > 0) face_ghosts_from(G, prim, pr, i, j, k, gaxes);
  if (fl & FL_REWRITE) {
    double U[NV];
    const double beta[3] = {met[2 * G.nv + c], met[3 * G.nv + c], met[4 * G.nv + c]};
    prim_to_cons(G.gam, G.gfac, pr, psi, alpha, beta, g1, g2, U);
#pragma unroll
    for (int v = 0; v < NV; v++) q[v * G.nv + c] = U[v];
  }
  if (flags) flags[c] = (uint8_t)fl;
  if ((fl & FL_FATAL) && nfatal) atomicAdd(nfatal, 1u);
  if ((fl & FL_FATAL) && nfatal2) atomicAdd(nfatal2, 1u);
}

// Conserved variables of cell c (linear index, ghosts included) of grid G.
__device__ __forceinline__ void prim2con_one(const Grid &G, const double *__restrict__ prim,
                                             const double *__restrict__ met, double *q, long c) {
  const int I = (int)(c % G.nt[0]);
  const int J = (int)((c / G.nt[0]) % G.nt[1]);
  double pr[NV];
#pragma unroll
  for (int v = 0; v < NV; v++) pr[v] = prim[v * G.nv + c];
  double g1 = 1.0, g2 = 1.0;
  if (G.coord != CART) ref_diag(G.coord, G.geo.r2c[I], G.geo.s2c[J], g1, g2);
  const double beta[3] = {met[2 * G.nv + c], met[3 * G.nv + c], met[4 * G.nv + c]};
  double U[NV];
  prim_to_cons(G.gam, G.gfac, pr, met[c], met[G.nv + c], beta, g1, g2, U);
#pragma unroll
  for (int v = 0; v < NV; v++) q[v * G.nv + c] = U[v];
}

// Ghost fill of face-adjacent ghost number t of grid G (numbered axis by
// axis, lower side then upper side, layer, transverse index).
__device__ __forceinline__ void ghost_one(const Grid &G, double *prim, long t) {
  int a = 0;
  long per = 0;
  for (a = 0; a < G.ndim; a++) {
    per = 2L * G.g[a] * ((long)G.n[0] * G.n[1] * G.n[2] / G.n[a]);
    if (t < per) break;
    t -= per;
  }
  if (a >= G.ndim) return;
  const int ng = G.g[a];
  const int na = G.n[a];
  const long ntr = per / (2L * ng);
  const int side = (int)(t / (ng * ntr));
  long r = t % (ng * ntr);
  const int l = (int)(r / ntr);
  long tr = r % ntr;
  const int bc = G.bc[a][side];
  if (bc == BC_NONE) return;
  // transverse interior indices
  int idx[3];
  const int b1 = (a == 0) ? 1 : 0, b2 = (a == 2) ? 1 : 2;
  idx[b1] = (int)(tr % G.n[b1]);
  idx[b2] = (int)(tr / G.n[b1]);
  const int gi = side == 0 ? -1 - l : na + l;
  int src[3] = {idx[0], idx[1], idx[2]};
  idx[a] = gi;
  double sg[3] = {1.0, 1.0, 1.0};
  if (bc == BC_PERIODIC) {
    src[a] = side == 0 ? gi + na : gi - na;
  } else if (bc == BC_OUTFLOW) {
    src[a] = side == 0 ? 0 : na - 1;
  } else {
    src[a] = side == 0 ? -1 - gi : 2 * na - 1 - gi;
    if (bc == BC_REFLECT || bc == BC_AXIS) {
      sg[a] = -1.0;
    } else {  // CENTER: r and theta components odd
      sg[0] = -1.0;
      sg[1] = -1.0;
      if (G.ndim > 1) src[1] = G.n[1] - 1 - src[1];
    }
    if ((bc == BC_CENTER || bc == BC_AXIS) && G.ndim > 2) src[2] = (src[2] + G.n[2] / 2) % G.n[2];
  }
  const long cd = cell_offset(G, idx[0], idx[1], idx[2]);
  const long cs = cell_offset(G, src[0], src[1], src[2]);
  prim[cd] = prim[cs];
  prim[4 * G.nv + cd] = prim[4 * G.nv + cs];
#pragma unroll
  for (int m = 0; m < 3; m++) {
    prim[(1 + m) * G.nv + cd] = sg[m] * prim[(1 + m) * G.nv + cs];
    prim[(5 + m) * G.nv + cd] = sg[m] * prim[(5 + m) * G.nv + cs];
  }
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}

__device__ __forceinline__ long interior_count(const Grid &G) { return (long)G.n[0] * G.n[1] * G.n[2]; }

__device__ __forceinline__ long ghost_count(const Grid &G) {
  long tot = 0;
  for (int a = 0; a < G.ndim; a++) tot += 2L * G.g[a] * (interior_count(G) / G.n[a]);
  return tot;
}

// Maximum over the NT threads of a workgroup (result valid in thread 0).
__device__ __forceinline__ double block_max(double x) {
  x = wave_max(x);
  __shared__ double red[NT / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  double m = red[0];
#pragma unroll
  for (int w = 1; w < NT / 64; w++) m = fmax(m, red[w]);
  __syncthreads();
  return m;
}

// dt = cfl / max rate, capped at t_end - t (section 2.9); 0 at or past the
// end (the capped step may leave t an ulp beyond t_end, and a caller may pass
// t_end < t), so that such a step changes nothing.
__device__ __forceinline__ double dt_from_rate(double mx, double cfl, double t, double t_end) {
  double dt = mx > 0.0 ? cfl / mx : t_end - t;
  if (t + dt > t_end) dt = t_end - t;
  return dt > 0.0 ? dt : 0.0;
}

// CFL rate (section 2.9, maxsum) of interior cell number t of grid G.
__device__ __forceinline__ double cfl_one(const Grid &G, const double *__restrict__ prim,
                                          const double *__restrict__ met, long t) {
    const int i = (int)(t % G.n[0]);
    const int j = (int)((t / G.n[0]) % G.n[1]);
    const int k = (int)(t / ((long)G.n[0] * G.n[1]));
    const long c = cell_offset(G, i, j, k);
    double pr[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) pr[v] = prim[v * G.nv + c];
    double g1 = 1.0, g2 = 1.0;
    if (G.coord != CART) ref_diag(G.coord, G.geo.r2c[i + G.g[0]], G.geo.s2c[j + G.g[1]], g1, g2);
    const double beta[3] = {met[2 * G.nv + c], met[3 * G.nv + c], met[4 * G.nv + c]};
    return cfl_rate(G.gam, G.gfac, pr, met[c], met[G.nv + c], beta, g1, g2, G.ndim, G.idx);
}

}  // namespace gm
