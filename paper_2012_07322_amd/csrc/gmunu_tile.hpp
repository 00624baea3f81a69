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

// Face flux times face factor through the lower face (along D) of cell
// (i,j,k): reconstruction REC from the cells across the face (MC from four
// cells, halo H = 2; MP5 or PPM from six, H = 3), metric as the mean of the
// two adjacent centres, HLLE (R = 0) or TVDLF (R = 1).  The stencil comes
// from the workgroup's staged region S (RC cells per variable, prim
// variables 0-7, metric 8-12): r0 is the region index of the cell H below
// the face, rs the region stride along D.
//
// P = 1 applies the positivity-preserving limiter (section 2.4): the flux is
// blended with the first-order Lax-Friedrichs flux of the two adjacent cell
// states, with the largest theta that keeps D and tau of the Euler update of
// both adjacent interior cells above eps (ghost cells are not advanced and do
// not take part).
template <int D, int REC, int R, int P = 0>
__device__ __forceinline__ void face_flux(const Grid &G, const double *S, int RC, int r0, int rs, int i, int j,
                                          int k, double *Fo, const PPBase &pb = PPBase{nullptr, 0.0}) {
  constexpr int H = recon_halo(REC);
  const int cd = (D == 0 ? i : D == 1 ? j : k) + G.g[D];
  // zero-area faces (r = 0, theta = 0 or pi) are evaluated like any other
  // and their flux replaced by 0 at the end; no load-dependent branch here
  const double fa = G.geo.fa[D][cd];
  // the two cells adjacent to the face
  const int r1 = r0 + (H - 1) * rs, r2 = r1 + rs;
  double pl[NV], pr[NV];
  if constexpr (REC == GMUNU_RECON_MC) {
    const int r3 = r2 + rs;
#pragma unroll
    for (int v = 0; v < NV; v++) {
      const double *Sv = S + v * RC;
      const double a = Sv[r0], b = Sv[r1], e = Sv[r2], f = Sv[r3];
      pl[v] = b + 0.5 * mc_slope(a, b, e);
      pr[v] = e - 0.5 * mc_slope(b, e, f);
    }
  } else {
#pragma unroll
    for (int v = 0; v < NV; v++) {
      const double *Sv = S + v * RC;
      const double u0 = Sv[r0], u1 = Sv[r0 + rs], u2 = Sv[r1], u3 = Sv[r2], u4 = Sv[r2 + rs],
                   u5 = Sv[r2 + 2 * rs];
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
        pl[v] = S[v * RC + r1];
        pr[v] = S[v * RC + r2];
      }
    }
  }
  const double *Sm = S + NV * RC;
  const double psi = 0.5 * (Sm[r1] + Sm[r2]);
  const double alpha = 0.5 * (Sm[RC + r1] + Sm[RC + r2]);
  double beta[3];
#pragma unroll
  for (int a = 0; a < 3; a++) beta[a] = 0.5 * (Sm[(2 + a) * RC + r1] + Sm[(2 + a) * RC + r2]);
  double g1 = 1.0, g2 = 1.0;
  if (G.coord != CART) {
    const double r2c = (D == 0) ? G.geo.r2f[i + G.g[0]] : G.geo.r2c[i + G.g[0]];
    const double s2 = (D == 1) ? G.geo.s2f[j + G.g[1]] : G.geo.s2c[j + G.g[1]];
    ref_diag(G.coord, r2c, s2, g1, g2);
  }
  const double psi2 = psi * psi, psi4 = psi2 * psi2, psi6 = psi4 * psi2;
  const double gD = D == 0 ? 1.0 : D == 1 ? g1 : g2;
  const double gud = rcp(psi4 * gD);
  double UL[NV], FL[NV], UR[NV], FR[NV], lmL, lpL, lmR, lpR;
  state_flux<D>(G.gam, G.gfac, pl, psi4, psi6, alpha, beta, g1, g2, gud, UL, FL, lmL, lpL);
  state_flux<D>(G.gam, G.gfac, pr, psi4, psi6, alpha, beta, g1, g2, gud, UR, FR, lmR, lpR);
  if constexpr (R == GMUNU_RIEMANN_TVDLF) {
    // local Lax-Friedrichs: the largest speed magnitude of both states
    const double c = fmax(fmax(fabs(lmL), fabs(lpL)), fmax(fabs(lmR), fabs(lpR)));
#pragma unroll
    for (int v = 0; v < NV; v++) {
      const double f = (0.5 * (FL[v] + FR[v]) - 0.5 * c * (UR[v] - UL[v])) * fa;
      Fo[v] = fa == 0.0 ? 0.0 : f;
    }
  } else {
    const double ap = fmax(0.0, fmax(lpL, lpR));
    const double am = fmin(0.0, fmin(lmL, lmR));
    const double den = ap - am;
    const bool avg = den < kTiny;
    const double s = fa * rcp(avg ? 1.0 : den);
#pragma unroll
    for (int v = 0; v < NV; v++) {
      const double f =
          avg ? 0.5 * (FL[v] + FR[v]) * fa : (ap * FL[v] - am * FR[v] + ap * am * (UR[v] - UL[v])) * s;
      Fo[v] = fa == 0.0 ? 0.0 : f;
    }
  }
  if constexpr (P) {
    // zero-area faces carry no flux either way
    if (fa == 0.0) return;
    double p0[NV], p1[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) {
      p0[v] = S[v * RC + r1];
      p1[v] = S[v * RC + r2];
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
// (Appendix A), added into s[].
__device__ __forceinline__ void cell_sources(const Grid &G, const double *__restrict__ pb,
                                             const double *__restrict__ mb, int i, int j, int k, unsigned rel,
                                             double *s) {
  const unsigned oc = rel * 8u;
  const double psi = ld(mb, G.nv, 0, oc), alpha = ld(mb, G.nv, 1, oc);
  double beta[3];
#pragma unroll
  for (int a = 0; a < 3; a++) beta[a] = ld(mb, G.nv, 2 + a, oc);
  double dpsi[3] = {0, 0, 0}, dal[3] = {0, 0, 0}, db[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  bool grav = (beta[0] != 0.0) || (beta[1] != 0.0) || (beta[2] != 0.0);
#pragma unroll
  for (int a = 0; a < 3; a++) {
    if (a < G.ndim) {
      const unsigned op = oc + (unsigned)G.s[a] * 8u, om = oc - (unsigned)G.s[a] * 8u;
      dpsi[a] = (ld(mb, G.nv, 0, op) - ld(mb, G.nv, 0, om)) * G.i2dx[a];
      dal[a] = (ld(mb, G.nv, 1, op) - ld(mb, G.nv, 1, om)) * G.i2dx[a];
#pragma unroll
      for (int m = 0; m < 3; m++) db[a][m] = (ld(mb, G.nv, 2 + m, op) - ld(mb, G.nv, 2 + m, om)) * G.i2dx[a];
      grav = grav || dpsi[a] != 0.0 || dal[a] != 0.0 || db[a][0] != 0.0 || db[a][1] != 0.0 || db[a][2] != 0.0;
    }
  }
  const bool geom = G.coord != CART;
  if (!grav && !geom) return;
  double pr[NV];
#pragma unroll
  for (int v = 0; v < NV; v++) pr[v] = ld(pb, G.nv, v, oc);

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
      for (int m = 0; m < 3; m++)
        T[a][m] = rhohs * ui[a] * ui[m] + ps * ((a == m ? rcp(gd[a]) : 0.0) - beta[a] * beta[m] * ia2) -
                  bi[a] * bi[m];
    }
    // covariant derivative of the shift with point Christoffel symbols
    double Gm[3][3][3];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
      for (int b = 0; b < 3; b++)
#pragma unroll
        for (int m = 0; m < 3; m++) Gm[a][b][m] = 0.0;
    if (G.coord == CYL) {
      const double R = G.geo.xc0[i + G.g[0]];
      Gm[0][2][2] = -R;
      Gm[2][0][2] = Gm[2][2][0] = rcp(R);
    } else if (G.coord == SPH) {
      const double r = G.geo.xc0[i + G.g[0]];
      const double sn = G.geo.sc1[j + G.g[1]], cs = G.geo.cc1[j + G.g[1]];
      Gm[0][1][1] = -r;
      Gm[0][2][2] = -r * sn * sn;
      Gm[1][0][1] = Gm[1][1][0] = rcp(r);
      Gm[1][2][2] = -sn * cs;
      Gm[2][0][2] = Gm[2][2][0] = rcp(r);
      Gm[2][1][2] = Gm[2][2][1] = cs * rcp(sn);
    }
    double nb[3][3];  // nb[i][k] = d_i beta^k + Gamma^k_il beta^l
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
      for (int m = 0; m < 3; m++) nb[a][m] = db[a][m] + Gm[m][a][0] * beta[0] + Gm[m][a][1] * beta[1] + Gm[m][a][2] * beta[2];
    const double divb = nb[0][0] + nb[1][1] + nb[2][2];
    double K[3][3];
    const double kf = psi4 * 0.5 * ia;
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
      for (int m = 0; m < 3; m++)
        K[a][m] = kf * (ref[m] * nb[a][m] + ref[a] * nb[m][a] - (a == m ? (2.0 / 3.0) * ref[a] * divb : 0.0));
    const double pre = alpha * psi6;
    const double fourpsi3 = 4.0 * psi2 * psi;
#pragma unroll
    for (int a = 0; a < 3; a++) {
      double sv = -T00 * alpha * dal[a];
#pragma unroll
      for (int m = 0; m < 3; m++) {
        const double T0low = gd[m] * (T00 * beta[m] + T0[m]);  // T^0_m
        sv += T0low * nb[a][m];
        sv += 0.5 * (T00 * beta[m] * beta[m] + 2.0 * T0[m] * beta[m] + T[m][m]) * fourpsi3 * dpsi[a] * ref[m];
      }
      s[1 + a] += pre * sv;
    }
    double Kbb = 0.0, bda = 0.0, TK = 0.0, T0K = 0.0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
      bda += beta[a] * dal[a];
      double Kb = 0.0;
#pragma unroll
      for (int m = 0; m < 3; m++) {
        Kbb += K[a][m] * beta[a] * beta[m];
        TK += T[a][m] * K[a][m];
        Kb += K[a][m] * beta[m];
      }
      T0K += T0[a] * (2.0 * Kb - dal[a]);
    }
    s[4] += pre * (T00 * (Kbb - bda) + T0K + TK);
  }

  if (geom) {
    // cell-centre momentum fluxes (f_S_l)^k = S_l vhat^k + delta alpha p* - alpha b_l B^k / W
    const double E = rhohs * W2;
    const double ab0 = alpha * b0;
    double bd[3], S[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      bd[a] = gd[a] * pr[5 + a] * iW + ab0 * vd[a];
      S[a] = E * vd[a] - ab0 * bd[a];
    }
    auto fS = [&](int l, int kk) {
      double f = S[l] * vh[kk] - alpha * bd[l] * pr[5 + kk] * iW;
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

// Staged region of the face pass along D of a TX x TY x TZ tile: the tile's
// cells plus H on each side along D (H = 2 for MC, 3 for MP5 and PPM).
template <int TX, int TY, int TZ, int D, int H>
constexpr int region_cells() {
  return (TX + 2 * H * (D == 0)) * (TY + 2 * H * (D == 1)) * (TZ + 2 * H * (D == 2));
}

// Faces of the pass along D (the tile's lower faces plus the upper layer).
template <int TX, int TY, int TZ, int D>
constexpr int pass_faces() {
  return (TX + (D == 0)) * (TY + (D == 1)) * (TZ + (D == 2));
}

template <int TX, int TY, int TZ, int ND, int H>
constexpr int max_region() {
  constexpr int r0 = region_cells<TX, TY, TZ, 0, H>(), r1 = ND > 1 ? region_cells<TX, TY, TZ, 1, H>() : 0,
                r2 = ND > 2 ? region_cells<TX, TY, TZ, 2, H>() : 0;
  return r0 > r1 ? (r0 > r2 ? r0 : r2) : (r1 > r2 ? r1 : r2);
}

template <int TX, int TY, int TZ, int ND>
constexpr int max_faces() {
  constexpr int f0 = pass_faces<TX, TY, TZ, 0>(), f1 = ND > 1 ? pass_faces<TX, TY, TZ, 1>() : 0,
                f2 = ND > 2 ? pass_faces<TX, TY, TZ, 2>() : 0;
  return f0 > f1 ? (f0 > f2 ? f0 : f2) : (f1 > f2 ? f1 : f2);
}

// Separate flux buffer: when the staged region and the face fluxes both fit
// in LDS for three workgroups per CU (160 KB), the fluxes get their own
// buffer, so that one pass's fluxes are summed while the next pass's region
// is staged (two barriers per pass instead of four).
template <int TX, int TY, int TZ, int ND, int H>
constexpr bool split_lds() {
  return ((NV + 5) * max_region<TX, TY, TZ, ND, H>() + NV * max_faces<TX, TY, TZ, ND>()) * 8 * 3 <= 160 * 1024;
}

// LDS doubles per workgroup: the staged region (prim and metric) of the
// largest pass, and the face fluxes (in a buffer of their own, or over the
// region once it has been used).
template <int TX, int TY, int TZ, int ND, int H = 2>
constexpr int stage_lds() {
  return (NV + 5) * max_region<TX, TY, TZ, ND, H>() +
         (split_lds<TX, TY, TZ, ND, H>() ? NV * max_faces<TX, TY, TZ, ND>() : 0);
}

// Tile shapes whose passes have at most one face per thread.
template <int TX, int TY, int TZ, int ND>
constexpr bool tile_fits() {
  return pass_faces<TX, TY, TZ, 0>() <= NT && (ND < 2 || pass_faces<TX, TY, TZ, 1>() <= NT) &&
         (ND < 3 || pass_faces<TX, TY, TZ, 2>() <= NT) && TX * TY * TZ <= NT;
}

// Stage prim and metric of the pass's region (the tile plus H cells each
// side along D) into S, coalesced, each value read once from memory.
template <int TX, int TY, int TZ, int D, int H>
__device__ __forceinline__ void stage_region(const Grid &G, const double *__restrict__ prim,
                                             const double *__restrict__ met, double *S, int i0, int j0, int k0) {
  constexpr int RX = TX + 2 * H * (D == 0), RY = TY + 2 * H * (D == 1), RZ = TZ + 2 * H * (D == 2),
                RC = RX * RY * RZ;
  // region origin: the tile origin moved H cells down along D
  const int ai = i0 - H * (D == 0), aj = j0 - H * (D == 1), ak = k0 - H * (D == 2);
  for (int c = threadIdx.x; c < RC; c += NT) {
    const int ri = c % RX, rj = (c / RX) % RY, rk = c / (RX * RY);
    const int gi = ai + ri, gj = aj + rj, gk = ak + rk;
    // cells outside the array (ragged tiles) are not needed by any valid face
    if (gi < G.n[0] + G.g[0] && gj < G.n[1] + G.g[1] && gk < G.n[2] + G.g[2]) {
      const long o = cell_offset(G, gi, gj, gk);
#pragma unroll
      for (int v = 0; v < NV; v++) S[v * RC + c] = prim[v * G.nv + o];
#pragma unroll
      for (int w = 0; w < 5; w++) S[(NV + w) * RC + c] = met[w * G.nv + o];
    }
  }
}

// Flux divergence along D accumulated into acc of the thread's cell, from
// the pass's region staged in S: (1) one face per thread, (2) the fluxes
// through LDS (SF; SF == S reuses the region once every face is done) to the
// cells on both sides of each face.  Begins after a barrier that follows the
// staging; on return other threads may still read SF.
template <int TX, int TY, int TZ, int D, int REC, int R, int P>
__device__ __forceinline__ void face_pass(const Grid &G, const double *S, double *SF, int i0, int j0, int k0,
                                          int tx, int ty, int tz, bool valid, double *acc, const PPBase &pb) {
  constexpr int H = recon_halo(REC);
  constexpr int RX = TX + 2 * H * (D == 0), RY = TY + 2 * H * (D == 1), RZ = TZ + 2 * H * (D == 2),
                RC = RX * RY * RZ;
  constexpr int FX = TX + (D == 0), FY = TY + (D == 1), FZ = TZ + (D == 2), NF = FX * FY * FZ;
  const int tid = threadIdx.x;
  // (1) face tid: region index of the cell H below it along D
  double Fo[NV];
  const int f = tid;
  const int fx = f % FX, fy = (f / FX) % FY, fz = f / (FX * FY);
  const int ci = i0 + fx, cj = j0 + fy, ck = k0 + fz;
  const bool ok = f < NF && (D == 0 ? ci <= G.n[0] : ci < G.n[0]) && (D == 1 ? cj <= G.n[1] : cj < G.n[1]) &&
                  (D == 2 ? ck <= G.n[2] : ck < G.n[2]);
  if (ok) {
    constexpr int rs = D == 0 ? 1 : D == 1 ? RX : RX * RY;
    const int r0 = fx + RX * (fy + RY * fz);  // region coordinate = face coordinate - H + H along D
    face_flux<D, REC, R, P>(G, S, RC, r0, rs, ci, cj, ck, Fo, pb);
  } else {
#pragma unroll
    for (int v = 0; v < NV; v++) Fo[v] = 0.0;
  }
  if (SF == S) __syncthreads();  // every face has read the region
  // (2) fluxes through LDS
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
// (MODE 0: out = L) on the tile of TX x TY x TZ cells with origin (i0,j0,k0).
// Every thread of the workgroup (NT threads) must call it (it synchronises);
// sF is the workgroup's LDS buffer of stage_lds<TX,TY,TZ,ND,recon_halo(REC)>()
// doubles.
template <int TX, int TY, int TZ, int ND, int MODE, int REC = 0, int R = 0, int P = 0>
__device__ __forceinline__ void stage_tile(const Grid &G, int i0, int j0, int k0, const double *__restrict__ prim,
                                           const double *__restrict__ met, const double *qn, const double *qs,
                                           double *out, const double *__restrict__ dtp, double ca, double cb,
                                           double *sF) {
  static_assert(tile_fits<TX, TY, TZ, ND>(), "tile passes must have at most one face per thread");
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = (tid / TX) % TY, tz = tid / (TX * TY);
  const int i = i0 + tx, j = j0 + ty, k = k0 + tz;
  const bool valid = tid < TX * TY * TZ && (i < G.n[0]) && (j < G.n[1]) && (k < G.n[2]);
  // tile base: the cell (i0 - g0, j0 - g1, k0 - g2); every access of this
  // workgroup is at a non-negative offset from it
  const long lo = cell_offset(G, i0 - G.g[0], j0 - G.g[1], k0 - G.g[2]);
  const double *__restrict__ pb = prim + lo;
  const double *__restrict__ mb = met + lo;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; v++) acc[v] = 0.0;
  static_assert(P == 0 || MODE == 1, "the limiter needs the stage's Euler step");
  PPBase pp{nullptr, 0.0};
  if constexpr (P) pp = PPBase{ca == 0.0 ? qn : qs, *dtp};
  // with a separate flux buffer a pass's fluxes are summed while the next
  // region is staged; with a shared one the summation must end first
  constexpr int H = recon_halo(REC);
  constexpr bool split = split_lds<TX, TY, TZ, ND, H>();
  double *SF = split ? sF + (NV + 5) * max_region<TX, TY, TZ, ND, H>() : sF;
  stage_region<TX, TY, TZ, 0, H>(G, prim, met, sF, i0, j0, k0);
  __syncthreads();
  face_pass<TX, TY, TZ, 0, REC, R, P>(G, sF, SF, i0, j0, k0, tx, ty, tz, valid, acc, pp);
  if constexpr (ND > 1) {
    if constexpr (!split) __syncthreads();
    stage_region<TX, TY, TZ, 1, H>(G, prim, met, sF, i0, j0, k0);
    __syncthreads();
    face_pass<TX, TY, TZ, 1, REC, R, P>(G, sF, SF, i0, j0, k0, tx, ty, tz, valid, acc, pp);
  }
  if constexpr (ND > 2) {
    if constexpr (!split) __syncthreads();
    stage_region<TX, TY, TZ, 2, H>(G, prim, met, sF, i0, j0, k0);
    __syncthreads();
    face_pass<TX, TY, TZ, 2, REC, R, P>(G, sF, SF, i0, j0, k0, tx, ty, tz, valid, acc, pp);
  }
  // a workgroup that takes another tile next restages sF: with a shared
  // buffer the summation must end first (with a separate one the next
  // tile's first barrier orders the flux buffer)
  if constexpr (!split) __syncthreads();
  if (!valid) return;
  const unsigned rel = (unsigned)((tz + G.g[2]) * G.s[2] + (ty + G.g[1]) * G.s[1] + (tx + G.g[0]));
  cell_sources(G, pb, mb, i, j, k, rel, acc);
  const unsigned oc = rel * 8u;
  if (MODE == 0) {
#pragma unroll
    for (int v = 0; v < NV; v++)
      *reinterpret_cast<double *>(reinterpret_cast<char *>(out + lo + v * G.nv) + oc) = acc[v];
  } else {
    const double dt = *dtp;
    const double *qnb = qn + lo;
#pragma unroll
    for (int v = 0; v < NV; v++) {
      double *o = reinterpret_cast<double *>(reinterpret_cast<char *>(out + lo + v * G.nv) + oc);
      const double un = ld(qnb, G.nv, v, oc);
      if (ca == 0.0) {
        *o = cb * (un + dt * acc[v]);
      } else {
        const double us = ld(qs + lo, G.nv, v, oc);
        *o = ca * un + cb * (us + dt * acc[v]);
      }
    }
  }
}

// Primitive recovery of interior cell number t (x fastest) of grid G; a
// fatal outcome increments *nfatal and *nfatal2 (each nullable).
__device__ __forceinline__ void c2p_one(const Grid &G, double *q, const double *__restrict__ met, double *prim,
                                        uint8_t *flags, unsigned int *nfatal, long t,
                                        unsigned int *nfatal2 = nullptr) {
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
