// GRMHD finite-volume step for MI355X (gfx950): kernels and the C ABI.
//
// One RK stage is three launches on the caller's stream:
//   k_stage   per tile of cells: MC reconstruction, HLLE face fluxes (each
//             face computed once and exchanged through LDS), flux-area
//             divergence, gravitational + geometric sources, RK combination;
//   k_c2p     per interior cell: primitive recovery with error handling;
//   k_ghosts  per face-adjacent ghost cell: boundary fill of the primitives.
// The time step is a per-cell rate reduced by wavefront shuffles to one
// maximum per workgroup (a fixed number of grid-stride workgroups), then by
// one workgroup that writes dt: no atomics, no memset, graph-capturable.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/gmunu.h"
#include "gmunu_dev.hpp"

using namespace gm;

struct gmunu_ctx {
  gmunu_grid_desc d;
  Grid G;
  int device;
  double *geo;                 // packed 1D geometry tables (device)
  double *acc;                 // CFL partial maxima (device, kCflParts words)
  // launch timing (measurement only)
  int prof;
  std::vector<hipEvent_t> ev;  // pairs
  std::vector<int> kind;
  size_t nrec;
};

namespace {
// Brackets one launch with events when profiling is on.
struct ProfScope {
  gmunu_ctx *c;
  hipStream_t s;
  size_t slot;
  ProfScope(gmunu_ctx *ctx, hipStream_t st, int k) : c(ctx), s(st), slot((size_t)-1) {
    if (c->prof && c->nrec < c->kind.size()) {
      slot = c->nrec++;
      c->kind[slot] = k;
      (void)hipEventRecord(c->ev[2 * slot], s);
    }
  }
  ~ProfScope() {
    if (slot != (size_t)-1) (void)hipEventRecord(c->ev[2 * slot + 1], s);
  }
};
}  // namespace

// ------------------------------------------------------------------ kernels

namespace {

constexpr double kTiny = 1e-300;
constexpr int kCflParts = 2048;  // workgroups of the CFL reduction

// Face flux times face factor through the lower face (along D) of cell
// (i,j,k): MC reconstruction from the four cells across the face, metric as
// the mean of the two adjacent centres, HLLE.
// Load variable v at byte offset ob from a tile base (scalar base, 32-bit
// per-lane offset).
__device__ __forceinline__ double ld(const double *__restrict__ base, long nv, int v, unsigned ob) {
  return *reinterpret_cast<const double *>(reinterpret_cast<const char *>(base + v * nv) + ob);
}

// Face flux times face factor through the lower face (along D) of cell
// (i,j,k): MC reconstruction from the four cells across the face, metric as
// the mean of the two adjacent centres, HLLE.  pb, mb: prim and metric
// bases of the tile; rel: offset of cell (i,j,k) from them (in cells).
template <int D>
__device__ __forceinline__ void face_flux(const Grid &G, const double *__restrict__ pb,
                                          const double *__restrict__ mb, int i, int j, int k, unsigned rel,
                                          double *Fo) {
  const int cd = (D == 0 ? i : D == 1 ? j : k) + G.g[D];
  // zero-area faces (r = 0, theta = 0 or pi) are evaluated like any other
  // and their flux replaced by 0 at the end; no load-dependent branch here
  const double fa = G.geo.fa[D][cd];
  const unsigned sd8 = (unsigned)G.s[D] * 8u;
  const unsigned o2 = rel * 8u;  // cell f (right of the face)
  const unsigned o1 = o2 - sd8, o0 = o1 - sd8, o3 = o2 + sd8;
  double pl[NV], pr[NV];
#pragma unroll
  for (int v = 0; v < NV; v++) {
    const double a = ld(pb, G.nv, v, o0), b = ld(pb, G.nv, v, o1), e = ld(pb, G.nv, v, o2),
                 f = ld(pb, G.nv, v, o3);
    pl[v] = b + 0.5 * mc_slope(a, b, e);
    pr[v] = e - 0.5 * mc_slope(b, e, f);
  }
  const double psi = 0.5 * (ld(mb, G.nv, 0, o1) + ld(mb, G.nv, 0, o2));
  const double alpha = 0.5 * (ld(mb, G.nv, 1, o1) + ld(mb, G.nv, 1, o2));
  double beta[3];
#pragma unroll
  for (int a = 0; a < 3; a++) beta[a] = 0.5 * (ld(mb, G.nv, 2 + a, o1) + ld(mb, G.nv, 2 + a, o2));
  double g1 = 1.0, g2 = 1.0;
  if (G.coord != CART) {
    const double r2 = (D == 0) ? G.geo.r2f[i + G.g[0]] : G.geo.r2c[i + G.g[0]];
    const double s2 = (D == 1) ? G.geo.s2f[j + G.g[1]] : G.geo.s2c[j + G.g[1]];
    ref_diag(G.coord, r2, s2, g1, g2);
  }
  const double psi2 = psi * psi, psi4 = psi2 * psi2, psi6 = psi4 * psi2;
  const double gD = D == 0 ? 1.0 : D == 1 ? g1 : g2;
  const double gud = rcp(psi4 * gD);
  double UL[NV], FL[NV], UR[NV], FR[NV], lmL, lpL, lmR, lpR;
  state_flux<D>(G.gam, G.gfac, pl, psi4, psi6, alpha, beta, g1, g2, gud, UL, FL, lmL, lpL);
  state_flux<D>(G.gam, G.gfac, pr, psi4, psi6, alpha, beta, g1, g2, gud, UR, FR, lmR, lpR);
  const double ap = fmax(0.0, fmax(lpL, lpR));
  const double am = fmin(0.0, fmin(lmL, lmR));
  const double den = ap - am;
  const bool avg = den < kTiny;
  const double s = fa * rcp(avg ? 1.0 : den);
#pragma unroll
  for (int v = 0; v < NV; v++) {
    const double f = avg ? 0.5 * (FL[v] + FR[v]) * fa : (ap * FL[v] - am * FR[v] + ap * am * (UR[v] - UL[v])) * s;
    Fo[v] = fa == 0.0 ? 0.0 : f;
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

template <int TX, int TY, int TZ, int D>
__device__ __forceinline__ void face_pass(const Grid &G, const double *__restrict__ pb,
                                          const double *__restrict__ mb, double *sF, int i0, int j0, int k0,
                                          int tx, int ty, int tz, bool valid, double *acc) {
  constexpr int FX = TX + (D == 0), FY = TY + (D == 1), FZ = TZ + (D == 2);
  constexpr int NF = FX * FY * FZ;
  const int tid = threadIdx.x;
  for (int f = tid; f < NF; f += TX * TY * TZ) {
    const int fx = f % FX, fy = (f / FX) % FY, fz = f / (FX * FY);
    const int ci = i0 + fx, cj = j0 + fy, ck = k0 + fz;
    const bool ok = (D == 0 ? ci <= G.n[0] : ci < G.n[0]) && (D == 1 ? cj <= G.n[1] : cj < G.n[1]) &&
                    (D == 2 ? ck <= G.n[2] : ck < G.n[2]);
    double Fo[NV];
    if (ok) {
      // offset from the tile base (the cell at i0 - g0, j0 - g1, k0 - g2)
      const unsigned rel = (unsigned)((ck - k0 + G.g[2]) * G.s[2] + (cj - j0 + G.g[1]) * G.s[1] + (ci - i0 + G.g[0]));
      face_flux<D>(G, pb, mb, ci, cj, ck, rel, Fo);
    } else {
#pragma unroll
      for (int v = 0; v < NV; v++) Fo[v] = 0.0;
    }
#pragma unroll
    for (int v = 0; v < NV; v++) sF[v * NF + f] = Fo[v];
  }
  __syncthreads();
  if (valid) {
    const int fl = tx + FX * (ty + FY * tz);
    const int fu = fl + (D == 0 ? 1 : D == 1 ? FX : FX * FY);
    const int cd = (D == 0 ? i0 + tx : D == 1 ? j0 + ty : k0 + tz) + G.g[D];
    const double icv = G.geo.icv[D][cd];
#pragma unroll
    for (int v = 0; v < NV; v++) acc[v] -= (sF[v * NF + fu] - sF[v * NF + fl]) * icv;
  }
  __syncthreads();
}

// Tile of this workgroup.  Workgroups are dispatched round-robin over the
// eight XCDs (each with its own L2), so the linear block index is remapped
// to give each XCD one contiguous run of tiles (x fastest, then y, then z):
// neighbouring tiles, whose stencils overlap, then share an L2.
__device__ __forceinline__ void xcd_tile(const Grid &G, int TX, int TY, int TZ, int &bx, int &by, int &bz) {
  const int gx = (G.n[0] + TX - 1) / TX, gy = (G.n[1] + TY - 1) / TY, gz = (G.n[2] + TZ - 1) / TZ;
  const int nb = gx * gy * gz;
  const int b = blockIdx.x, x = b % 8, ii = b / 8, q = nb / 8, r = nb % 8;
  const int L = x * q + (x < r ? x : r) + ii;
  bx = L % gx;
  by = (L / gx) % gy;
  bz = L / (gx * gy);
}

template <int TX, int TY, int TZ, int ND>
constexpr int max_faces() {
  constexpr int a = (TX + 1) * TY * TZ;
  constexpr int b = ND > 1 ? TX * (TY + 1) * TZ : 0;
  constexpr int c = ND > 2 ? TX * TY * (TZ + 1) : 0;
  return a > b ? (a > c ? a : c) : (b > c ? b : c);
}

// MODE 0: dqdt = L(prim).  MODE 1: q_out = ca q_n + cb (q_s + dt L(prim)).
template <int TX, int TY, int TZ, int ND, int MODE>
__global__ __launch_bounds__(TX *TY *TZ, 3) void k_stage(const Grid G, const double *__restrict__ prim,
                                                      const double *__restrict__ met, const double *qn,
                                                      const double *qs, double *out,
                                                      const double *__restrict__ dtp, double ca, double cb) {
  __shared__ double sF[NV * max_faces<TX, TY, TZ, ND>()];
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = (tid / TX) % TY, tz = tid / (TX * TY);
  int bx, by, bz;
  xcd_tile(G, TX, TY, TZ, bx, by, bz);
  const int i0 = bx * TX, j0 = by * TY, k0 = bz * TZ;
  const int i = i0 + tx, j = j0 + ty, k = k0 + tz;
  const bool valid = (i < G.n[0]) && (j < G.n[1]) && (k < G.n[2]);
  // tile base: the cell (i0 - g0, j0 - g1, k0 - g2); every access of this
  // workgroup is at a non-negative offset from it
  const long lo = cell_offset(G, i0 - G.g[0], j0 - G.g[1], k0 - G.g[2]);
  const double *__restrict__ pb = prim + lo;
  const double *__restrict__ mb = met + lo;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; v++) acc[v] = 0.0;
  face_pass<TX, TY, TZ, 0>(G, pb, mb, sF, i0, j0, k0, tx, ty, tz, valid, acc);
  if constexpr (ND > 1) face_pass<TX, TY, TZ, 1>(G, pb, mb, sF, i0, j0, k0, tx, ty, tz, valid, acc);
  if constexpr (ND > 2) face_pass<TX, TY, TZ, 2>(G, pb, mb, sF, i0, j0, k0, tx, ty, tz, valid, acc);
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

__global__ __launch_bounds__(NT) void k_c2p(const Grid G, double *q, const double *__restrict__ met, double *prim,
                                            uint8_t *flags, unsigned int *nfatal) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  const long nin = (long)G.n[0] * G.n[1] * G.n[2];
  if (t >= nin) return;
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
  const int fl = c2p_cell(G, qc, psi, alpha, g1, g2, pr);
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
}

__global__ __launch_bounds__(NT) void k_prim2con(const Grid G, const double *__restrict__ prim,
                                                 const double *__restrict__ met, double *q) {
  const long c = (long)blockIdx.x * NT + threadIdx.x;
  if (c >= G.nv) return;
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

// Ghost fill on the face-adjacent ghost cells of every active axis.
__global__ __launch_bounds__(NT) void k_ghosts(const Grid G, double *prim, long total) {
  long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= total) return;
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

// Per-workgroup maxima of the CFL rate over a grid-stride range of interior
// cells, written to part[blockIdx] (no atomics).
__global__ __launch_bounds__(NT) void k_cfl(const Grid G, const double *__restrict__ prim,
                                            const double *__restrict__ met, double *part) {
  const long nin = (long)G.n[0] * G.n[1] * G.n[2];
  double rate = 0.0;
  for (long t = (long)blockIdx.x * NT + threadIdx.x; t < nin; t += (long)gridDim.x * NT) {
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
    rate = fmax(rate, cfl_rate(G.gam, G.gfac, pr, met[c], met[G.nv + c], beta, g1, g2, G.ndim, G.idx));
  }
  rate = wave_max(rate);
  __shared__ double red[NT / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = rate;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int w = 1; w < NT / 64; w++) m = fmax(m, red[w]);
    part[blockIdx.x] = m;
  }
}

// dt = cfl / max(part), capped at t_end - t.
__global__ __launch_bounds__(NT) void k_cfl_finish(const double *part, int nparts, double cfl, double t_end,
                                                   const double *tp, double *dtp) {
  double m = 0.0;
  for (int b = threadIdx.x; b < nparts; b += NT) m = fmax(m, part[b]);
  m = wave_max(m);
  __shared__ double red[NT / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mx = red[0];
    for (int w = 1; w < NT / 64; w++) mx = fmax(mx, red[w]);
    const double t = tp ? *tp : 0.0;
    double dt = mx > 0.0 ? cfl / mx : t_end - t;
    if (t + dt > t_end) dt = t_end - t;
    *dtp = dt;
  }
}

__global__ void k_advance(double *tp, const double *dtp) { *tp += *dtp; }

// ------------------------------------------------------------ host helpers

inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

int launch_status() { return hipGetLastError() == hipSuccess ? GMUNU_OK : GMUNU_EHIP; }

template <int TX, int TY, int TZ, int ND, int MODE>
void launch_stage_t(const gmunu_ctx *ctx, const double *prim, const double *met, const double *qn,
                    const double *qs, double *out, const double *dtp, double ca, double cb, hipStream_t st) {
  const Grid &G = ctx->G;
  dim3 grid(((G.n[0] + TX - 1) / TX) * ((G.n[1] + TY - 1) / TY) * ((G.n[2] + TZ - 1) / TZ));
  hipLaunchKernelGGL((k_stage<TX, TY, TZ, ND, MODE>), grid, dim3(TX * TY * TZ), 0, st, G, prim, met, qn, qs, out,
                     dtp, ca, cb);
}

template <int MODE>
void launch_stage(const gmunu_ctx *ctx, const double *prim, const double *met, const double *qn,
                  const double *qs, double *out, const double *dtp, double ca, double cb, hipStream_t st) {
  if (ctx->G.ndim == 1)
    launch_stage_t<256, 1, 1, 1, MODE>(ctx, prim, met, qn, qs, out, dtp, ca, cb, st);
  else if (ctx->G.ndim == 2)
    launch_stage_t<32, 8, 1, 2, MODE>(ctx, prim, met, qn, qs, out, dtp, ca, cb, st);
  else
    launch_stage_t<16, 4, 4, 3, MODE>(ctx, prim, met, qn, qs, out, dtp, ca, cb, st);
}

long interior_cells(const Grid &G) { return (long)G.n[0] * G.n[1] * G.n[2]; }

long ghost_total(const Grid &G) {
  long tot = 0;
  for (int a = 0; a < G.ndim; a++) tot += 2L * G.g[a] * (interior_cells(G) / G.n[a]);
  return tot;
}

unsigned blocks(long n) { return (unsigned)((n + NT - 1) / NT); }

}  // namespace

// --------------------------------------------------------------------- API

extern "C" {

int gmunu_create(const gmunu_grid_desc *desc, gmunu_ctx **out) {
  if (!desc || !out) return GMUNU_ENULL;
  const gmunu_grid_desc &d = *desc;
  if (d.ndim < 1 || d.ndim > 3 || d.coord < 0 || d.coord > 2) return GMUNU_EINVAL;
  if (d.ng < 2) return GMUNU_EINVAL;
  for (int a = 0; a < 3; a++) {
    if (d.n[a] < 1 || !(d.dx[a] > 0.0) || !std::isfinite(d.xmin[a])) return GMUNU_EINVAL;
    if (a >= d.ndim && d.n[a] != 1) return GMUNU_EINVAL;
    if (a < d.ndim && d.n[a] < 1) return GMUNU_EINVAL;
    for (int s = 0; s < 2; s++)
      if (a < d.ndim && (d.bc[a][s] < 0 || d.bc[a][s] > 5)) return GMUNU_EINVAL;
  }
  for (int a = 0; a < d.ndim; a++) {
    const bool per0 = d.bc[a][0] == GMUNU_BC_PERIODIC, per1 = d.bc[a][1] == GMUNU_BC_PERIODIC;
    if (per0 != per1) return GMUNU_EINVAL;
    if (per0 && d.n[a] < d.ng) return GMUNU_EINVAL;
    for (int s = 0; s < 2; s++) {
      const int b = d.bc[a][s];
      if ((b == GMUNU_BC_REFLECT || b == GMUNU_BC_AXIS || b == GMUNU_BC_CENTER) && d.n[a] < d.ng)
        return GMUNU_EINVAL;
      if ((b == GMUNU_BC_AXIS || b == GMUNU_BC_CENTER) && d.ndim > 2 && (d.n[2] % 2) != 0) return GMUNU_EINVAL;
    }
  }
  if (!(d.gamma > 1.0) || !(d.rho_atmo > 0.0) || !(d.w_max > 1.0) || d.c2p_maxit < 1 || !(d.c2p_tol > 0.0))
    return GMUNU_EINVAL;
  if (d.rk != 2 && d.rk != 3) return GMUNU_EINVAL;

  gmunu_ctx *ctx = new (std::nothrow) gmunu_ctx();
  if (!ctx) return GMUNU_ENOMEM;
  ctx->d = d;
  ctx->prof = 0;
  ctx->nrec = 0;
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    delete ctx;
    return GMUNU_EHIP;
  }
  Grid &G = ctx->G;
  std::memset(&G, 0, sizeof(G));
  G.ndim = d.ndim;
  G.coord = d.coord;
  for (int a = 0; a < 3; a++) {
    G.n[a] = d.n[a];
    G.g[a] = a < d.ndim ? d.ng : 0;
    G.nt[a] = d.n[a] + 2 * G.g[a];
    G.dx[a] = d.dx[a];
    G.i2dx[a] = 1.0 / (2.0 * d.dx[a]);
    G.idx[a] = 1.0 / d.dx[a];
    G.bc[a][0] = d.bc[a][0];
    G.bc[a][1] = d.bc[a][1];
  }
  G.s[0] = 1;
  G.s[1] = G.nt[0];
  G.s[2] = (long)G.nt[0] * G.nt[1];
  G.nv = G.s[2] * G.nt[2];
  G.gam = d.gamma;
  G.gm1 = d.gamma - 1.0;
  G.gfac = d.gamma / (d.gamma - 1.0);
  G.rho_atmo = d.rho_atmo;
  G.p_atmo = d.k_atmo * std::pow(d.rho_atmo, d.gamma_atmo);
  G.rho_low = d.rho_low_factor * d.rho_atmo;
  G.alpha_bh = d.alpha_bh;
  G.rho_max = d.rho_max;
  G.eps_max = d.eps_max;
  G.w_max = d.w_max;
  G.maxit = d.c2p_maxit;
  G.tol = d.c2p_tol;

  // 1D geometry tables (Appendix A), host FP64
  std::vector<double> tab;
  auto put = [&](const std::vector<double> &v) {
    size_t off = tab.size();
    tab.insert(tab.end(), v.begin(), v.end());
    return off;
  };
  size_t o_icv[3], o_fa[3];
  std::vector<double> xc[3], xf[3], cv[3];
  for (int a = 0; a < 3; a++) {
    xc[a].resize(G.nt[a]);
    xf[a].resize(G.nt[a] + 1);
    for (int I = 0; I < G.nt[a]; I++) xc[a][I] = d.xmin[a] + (I - G.g[a] + 0.5) * d.dx[a];
    for (int F = 0; F <= G.nt[a]; F++) xf[a][F] = d.xmin[a] + (F - G.g[a]) * d.dx[a];
    cv[a].resize(G.nt[a]);
    std::vector<double> icv(G.nt[a]), fa(G.nt[a] + 1, 1.0);
    for (int I = 0; I < G.nt[a]; I++) {
      double v = d.dx[a];
      if (d.coord == GMUNU_CYL && a == 0) v = xc[a][I] * d.dx[a];
      if (d.coord == GMUNU_SPH && a == 0) v = (xc[a][I] * xc[a][I] + d.dx[a] * d.dx[a] / 12.0) * d.dx[a];
      if (d.coord == GMUNU_SPH && a == 1) v = 2.0 * std::sin(xc[a][I]) * std::sin(0.5 * d.dx[a]);
      cv[a][I] = v;
      icv[I] = 1.0 / v;
    }
    for (int F = 0; F <= G.nt[a]; F++) {
      if (d.coord == GMUNU_CYL && a == 0) fa[F] = xf[a][F];
      if (d.coord == GMUNU_SPH && a == 0) fa[F] = xf[a][F] * xf[a][F];
      if (d.coord == GMUNU_SPH && a == 1) fa[F] = std::sin(xf[a][F]);
    }
    o_icv[a] = put(icv);
    o_fa[a] = put(fa);
  }
  std::vector<double> r2c(G.nt[0]), r2f(G.nt[0] + 1), s2c(G.nt[1]), s2f(G.nt[1] + 1), sc(G.nt[1]), cc(G.nt[1]);
  std::vector<double> gA(G.nt[0], 0.0), gB(G.nt[0], 0.0), gC(G.nt[1], 0.0);
  for (int I = 0; I < G.nt[0]; I++) r2c[I] = xc[0][I] * xc[0][I];
  for (int F = 0; F <= G.nt[0]; F++) r2f[F] = xf[0][F] * xf[0][F];
  for (int J = 0; J < G.nt[1]; J++) {
    sc[J] = std::sin(xc[1][J]);
    cc[J] = std::cos(xc[1][J]);
    s2c[J] = sc[J] * sc[J];
  }
  for (int F = 0; F <= G.nt[1]; F++) {
    const double s = std::sin(xf[1][F]);
    s2f[F] = s * s;
  }
  if (d.coord == GMUNU_SPH) {
    for (int I = 0; I < G.nt[0]; I++) {
      const double p2 = r2f[I + 1], m2 = r2f[I];
      gA[I] = 0.5 * (p2 - m2) / cv[0][I];
      gB[I] = -0.25 * (p2 * p2 - m2 * m2) / cv[0][I];
    }
    for (int J = 0; J < G.nt[1]; J++) gC[J] = (std::sin(xf[1][J + 1]) - std::sin(xf[1][J])) / cv[1][J];
  } else if (d.coord == GMUNU_CYL) {
    for (int I = 0; I < G.nt[0]; I++) gA[I] = 1.0 / xc[0][I];
  }
  const size_t o_r2c = put(r2c), o_r2f = put(r2f), o_s2c = put(s2c), o_s2f = put(s2f), o_xc0 = put(xc[0]),
               o_sc = put(sc), o_cc = put(cc), o_gA = put(gA), o_gB = put(gB), o_gC = put(gC);

  if (hipMalloc(&ctx->geo, tab.size() * sizeof(double)) != hipSuccess) {
    delete ctx;
    return GMUNU_ENOMEM;
  }
  if (hipMalloc(&ctx->acc, kCflParts * sizeof(double)) != hipSuccess) {
    (void)hipFree(ctx->geo);
    delete ctx;
    return GMUNU_ENOMEM;
  }
  if (hipMemcpy(ctx->geo, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(ctx->acc, 0, kCflParts * sizeof(double)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(ctx->geo);
    (void)hipFree(ctx->acc);
    delete ctx;
    return GMUNU_EHIP;
  }
  const double *g = ctx->geo;
  for (int a = 0; a < 3; a++) {
    G.geo.icv[a] = g + o_icv[a];
    G.geo.fa[a] = g + o_fa[a];
  }
  G.geo.r2c = g + o_r2c;
  G.geo.r2f = g + o_r2f;
  G.geo.s2c = g + o_s2c;
  G.geo.s2f = g + o_s2f;
  G.geo.xc0 = g + o_xc0;
  G.geo.sc1 = g + o_sc;
  G.geo.cc1 = g + o_cc;
  G.geo.gA = g + o_gA;
  G.geo.gB = g + o_gB;
  G.geo.gC = g + o_gC;
  *out = ctx;
  return GMUNU_OK;
}

int gmunu_destroy(gmunu_ctx *ctx) {
  if (!ctx) return GMUNU_ENULL;
  int rc = GMUNU_OK;
  for (auto e : ctx->ev) (void)hipEventDestroy(e);
  if (hipFree(ctx->geo) != hipSuccess) rc = GMUNU_EHIP;
  if (hipFree(ctx->acc) != hipSuccess) rc = GMUNU_EHIP;
  delete ctx;
  return rc;
}

long gmunu_ntot(const gmunu_ctx *ctx) { return ctx ? ctx->G.nv : -1; }

int gmunu_prim2con(gmunu_ctx *ctx, const double *prim, const double *metric, double *q, void *stream) {
  if (!ctx || !prim || !metric || !q) return GMUNU_ENULL;
  if (!aligned8(prim) || !aligned8(metric) || !aligned8(q)) return GMUNU_EALIGN;
  ProfScope ps(ctx, S(stream), GMUNU_K_OTHER);
  hipLaunchKernelGGL(k_prim2con, dim3(blocks(ctx->G.nv)), dim3(NT), 0, S(stream), ctx->G, prim, metric, q);
  return launch_status();
}

int gmunu_c2p(gmunu_ctx *ctx, double *q, const double *metric, double *prim, uint8_t *flags,
              unsigned int *nfatal_dev, void *stream) {
  if (!ctx || !q || !metric || !prim) return GMUNU_ENULL;
  if (!aligned8(prim) || !aligned8(metric) || !aligned8(q)) return GMUNU_EALIGN;
  ProfScope ps(ctx, S(stream), GMUNU_K_C2P);
  hipLaunchKernelGGL(k_c2p, dim3(blocks(interior_cells(ctx->G))), dim3(NT), 0, S(stream), ctx->G, q, metric, prim,
                     flags, nfatal_dev);
  return launch_status();
}

int gmunu_fill_ghosts(gmunu_ctx *ctx, double *prim, void *stream) {
  if (!ctx || !prim) return GMUNU_ENULL;
  if (!aligned8(prim)) return GMUNU_EALIGN;
  const long tot = ghost_total(ctx->G);
  if (tot == 0) return GMUNU_OK;
  ProfScope ps(ctx, S(stream), GMUNU_K_GHOSTS);
  hipLaunchKernelGGL(k_ghosts, dim3(blocks(tot)), dim3(NT), 0, S(stream), ctx->G, prim, tot);
  return launch_status();
}

int gmunu_rhs(gmunu_ctx *ctx, const double *prim, const double *metric, double *dqdt, void *stream) {
  if (!ctx || !prim || !metric || !dqdt) return GMUNU_ENULL;
  if (!aligned8(prim) || !aligned8(metric) || !aligned8(dqdt)) return GMUNU_EALIGN;
  {
    ProfScope ps(ctx, S(stream), GMUNU_K_STAGE);
    launch_stage<0>(ctx, prim, metric, nullptr, nullptr, dqdt, nullptr, 0.0, 0.0, S(stream));
  }
  return launch_status();
}

int gmunu_cfl_dt(gmunu_ctx *ctx, const double *prim, const double *metric, double cfl, double t_end,
                 const double *t_dev, double *dt_dev, void *stream) {
  if (!ctx || !prim || !metric || !dt_dev) return GMUNU_ENULL;
  if (!aligned8(prim) || !aligned8(metric) || !aligned8(dt_dev)) return GMUNU_EALIGN;
  if (!(cfl > 0.0)) return GMUNU_EINVAL;
  const long nb = blocks(interior_cells(ctx->G));
  const int nparts = (int)(nb < kCflParts ? nb : kCflParts);
  {
    ProfScope ps(ctx, S(stream), GMUNU_K_CFL);
    hipLaunchKernelGGL(k_cfl, dim3(nparts), dim3(NT), 0, S(stream), ctx->G, prim, metric, ctx->acc);
  }
  {
    ProfScope ps(ctx, S(stream), GMUNU_K_OTHER);
    hipLaunchKernelGGL(k_cfl_finish, dim3(1), dim3(NT), 0, S(stream), ctx->acc, nparts, cfl, t_end, t_dev, dt_dev);
  }
  return launch_status();
}

int gmunu_rk_stage(gmunu_ctx *ctx, int stage, const double *dt_dev, const double *q_n, const double *q_s,
                   double *q_out, const double *prim_in, double *prim_out, const double *metric, uint8_t *flags,
                   unsigned int *nfatal_dev, void *stream) {
  if (!ctx || !dt_dev || !q_n || !q_out || !prim_in || !prim_out || !metric) return GMUNU_ENULL;
  if (stage > 0 && !q_s) return GMUNU_ENULL;
  const int nst = ctx->d.rk;
  if (stage < 0 || stage >= nst) return GMUNU_EINVAL;
  double ca = 0.0, cb = 1.0;
  if (stage > 0) {
    if (nst == 2) {
      ca = 0.5;
      cb = 0.5;
    } else if (stage == 1) {
      ca = 0.75;
      cb = 0.25;
    } else {
      ca = 1.0 / 3.0;
      cb = 2.0 / 3.0;
    }
  }
  hipStream_t st = S(stream);
  {
    ProfScope ps(ctx, st, GMUNU_K_STAGE);
    launch_stage<1>(ctx, prim_in, metric, q_n, q_s, q_out, dt_dev, ca, cb, st);
  }
  int rc = launch_status();
  if (rc) return rc;
  rc = gmunu_c2p(ctx, q_out, metric, prim_out, flags, nfatal_dev, stream);
  if (rc) return rc;
  return gmunu_fill_ghosts(ctx, prim_out, stream);
}

int gmunu_step(gmunu_ctx *ctx, double *q_n, double *q_s, double *prim, const double *metric, double cfl,
               double t_end, double *t_dev, double *dt_dev, uint8_t *flags, unsigned int *nfatal_dev,
               void *stream) {
  if (!ctx || !q_n || !q_s || !prim || !metric || !t_dev || !dt_dev) return GMUNU_ENULL;
  int rc = gmunu_cfl_dt(ctx, prim, metric, cfl, t_end, t_dev, dt_dev, stream);
  if (rc) return rc;
  const int nst = ctx->d.rk;
  for (int s = 0; s < nst; s++) {
    double *out = (s == nst - 1) ? q_n : q_s;
    rc = gmunu_rk_stage(ctx, s, dt_dev, q_n, q_s, out, prim, prim, metric, flags, nfatal_dev, stream);
    if (rc) return rc;
  }
  {
    ProfScope ps(ctx, S(stream), GMUNU_K_OTHER);
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, S(stream), t_dev, dt_dev);
  }
  return launch_status();
}

int gmunu_profile(gmunu_ctx *ctx, int enable, int max_launches) {
  if (!ctx) return GMUNU_ENULL;
  for (auto e : ctx->ev) (void)hipEventDestroy(e);
  ctx->ev.clear();
  ctx->kind.clear();
  ctx->nrec = 0;
  ctx->prof = 0;
  if (!enable) return GMUNU_OK;
  if (max_launches < 1) return GMUNU_EINVAL;
  ctx->ev.resize(2 * (size_t)max_launches);
  ctx->kind.assign(max_launches, 0);
  for (auto &e : ctx->ev)
    if (hipEventCreate(&e) != hipSuccess) return GMUNU_EHIP;
  ctx->prof = 1;
  return GMUNU_OK;
}

int gmunu_profile_read(gmunu_ctx *ctx, double *ms_out, long *count_out) {
  if (!ctx || !ms_out || !count_out) return GMUNU_ENULL;
  for (int k = 0; k < GMUNU_NK; k++) {
    ms_out[k] = 0.0;
    count_out[k] = 0;
  }
  for (size_t i = 0; i < ctx->nrec; i++) {
    float ms = 0.f;
    if (hipEventSynchronize(ctx->ev[2 * i + 1]) != hipSuccess) return GMUNU_EHIP;
    if (hipEventElapsedTime(&ms, ctx->ev[2 * i], ctx->ev[2 * i + 1]) != hipSuccess) return GMUNU_EHIP;
    ms_out[ctx->kind[i]] += ms;
    count_out[ctx->kind[i]] += 1;
  }
  ctx->nrec = 0;
  return GMUNU_OK;
}

}  // extern "C"
