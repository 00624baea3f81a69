// Host-side grid setup shared by the single-grid context and the batch:
// descriptor validation, the Grid parameters, and the per-axis geometry
// tables of Appendix A (cell volumes, face areas, averaged Christoffel
// symbols of cylindrical and spherical coordinates).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/gmunu.h"
#include "gmunu_dev.hpp"

namespace gm {

// Largest x-y plane (ghosts included): the stage kernel addresses a tile's
// stencil with 32-bit byte offsets from the tile's base, spanning at most
// eight planes.
constexpr long kMaxPlane = 1L << 25;

inline int validate_desc(const gmunu_grid_desc &d) {
  if (d.ndim < 1 || d.ndim > 3 || d.coord < 0 || d.coord > 2) return GMUNU_EINVAL;
  if (d.ng < 2) return GMUNU_EINVAL;
  for (int a = 0; a < 3; a++) {
    if (d.n[a] < 1 || !(d.dx[a] > 0.0) || !std::isfinite(d.xmin[a])) return GMUNU_EINVAL;
    if (a >= d.ndim && d.n[a] != 1) return GMUNU_EINVAL;
    for (int s = 0; s < 2; s++)
      if (a < d.ndim && (d.bc[a][s] < 0 || d.bc[a][s] > 5)) return GMUNU_EINVAL;
  }
  if ((long)(d.n[0] + 2L * d.ng) * (d.n[1] + (d.ndim > 1 ? 2L * d.ng : 0L)) > kMaxPlane) return GMUNU_EINVAL;
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
  if (d.recon != GMUNU_RECON_MC && d.recon != GMUNU_RECON_MP5 && d.recon != GMUNU_RECON_PPM) return GMUNU_EINVAL;
  if (d.recon != GMUNU_RECON_MC && d.ng < 3) return GMUNU_EINVAL;
  if (d.riemann != GMUNU_RIEMANN_HLLE && d.riemann != GMUNU_RIEMANN_TVDLF) return GMUNU_EINVAL;
  if (d.pp_limiter != 0 && d.pp_limiter != 1) return GMUNU_EINVAL;
  if (d.c2p != GMUNU_C2P_GRMHD && d.c2p != GMUNU_C2P_GRHD_Z) return GMUNU_EINVAL;
  return GMUNU_OK;
}

// Offsets of the geometry tables of one grid inside a packed table.
struct GeoOffsets {
  size_t icv[3], fa[3], r2c, r2f, s2c, s2f, xc0, sc, cc, gA, gB, gC;
};

// Fill G's scalar parameters (all but the geometry pointers).
inline void grid_scalars(const gmunu_grid_desc &d, Grid &G) {
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
  G.recon = d.recon;
  G.riemann = d.riemann;
  G.c2p = d.c2p;
  G.pp = d.pp_limiter;
}

// Offsets of the geometry tables of a grid with nt cells per axis (ghosts
// included) in the packed order setup_grid writes them; total: the table's
// length in doubles.
inline GeoOffsets geo_layout(const int nt[3], size_t &total) {
  GeoOffsets o;
  size_t at = 0;
  auto take = [&](size_t n) {
    const size_t off = at;
    at += n;
    return off;
  };
  for (int a = 0; a < 3; a++) {
    o.icv[a] = take(nt[a]);
    o.fa[a] = take(nt[a] + 1);
  }
  o.r2c = take(nt[0]);
  o.r2f = take(nt[0] + 1);
  o.s2c = take(nt[1]);
  o.s2f = take(nt[1] + 1);
  o.xc0 = take(nt[0]);
  o.sc = take(nt[1]);
  o.cc = take(nt[1]);
  o.gA = take(nt[0]);
  o.gB = take(nt[0]);
  o.gC = take(nt[1]);
  total = at;
  return o;
}

// Fill G (all but the geometry pointers) and append the grid's 1D geometry
// tables to tab.
inline GeoOffsets setup_grid(const gmunu_grid_desc &d, Grid &G, std::vector<double> &tab) {
  grid_scalars(d, G);

  auto put = [&](const std::vector<double> &v) {
    size_t off = tab.size();
    tab.insert(tab.end(), v.begin(), v.end());
    return off;
  };
  GeoOffsets o;
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
    o.icv[a] = put(icv);
    o.fa[a] = put(fa);
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
    // <G^th_r th> = <G^ph_r ph> = (A_r+ - A_r-)/(2 dV); <G^r_th th> = -(r+^2 A_r+ - r-^2 A_r-)/(4 dV);
    // <G^ph_th ph> = (A_th+ - A_th-)/dV (the exact average of cot theta)
    for (int I = 0; I < G.nt[0]; I++) {
      const double p2 = r2f[I + 1], m2 = r2f[I];
      gA[I] = 0.5 * (p2 - m2) / cv[0][I];
      gB[I] = -0.25 * (p2 * p2 - m2 * m2) / cv[0][I];
    }
    for (int J = 0; J < G.nt[1]; J++) gC[J] = (std::sin(xf[1][J + 1]) - std::sin(xf[1][J])) / cv[1][J];
  } else if (d.coord == GMUNU_CYL) {
    for (int I = 0; I < G.nt[0]; I++) gA[I] = 1.0 / xc[0][I];  // <G^ph_R ph> = 1/R
  }
  o.r2c = put(r2c);
  o.r2f = put(r2f);
  o.s2c = put(s2c);
  o.s2f = put(s2f);
  o.xc0 = put(xc[0]);
  o.sc = put(sc);
  o.cc = put(cc);
  o.gA = put(gA);
  o.gB = put(gB);
  o.gC = put(gC);
  return o;
}

// Point G's geometry tables into the device copy of the packed table.
inline void bind_geo(Grid &G, const double *g, const GeoOffsets &o) {
  for (int a = 0; a < 3; a++) {
    G.geo.icv[a] = g + o.icv[a];
    G.geo.fa[a] = g + o.fa[a];
  }
  G.geo.r2c = g + o.r2c;
  G.geo.r2f = g + o.r2f;
  G.geo.s2c = g + o.s2c;
  G.geo.s2f = g + o.s2f;
  G.geo.xc0 = g + o.xc0;
  G.geo.sc1 = g + o.sc;
  G.geo.cc1 = g + o.cc;
  G.geo.gA = g + o.gA;
  G.geo.gB = g + o.gB;
  G.geo.gC = g + o.gC;
}

inline long interior_cells(const Grid &G) { return (long)G.n[0] * G.n[1] * G.n[2]; }

inline long ghost_total(const Grid &G) {
  long tot = 0;
  for (int a = 0; a < G.ndim; a++) tot += 2L * G.g[a] * (interior_cells(G) / G.n[a]);
  return tot;
}

inline unsigned nblocks(long n) { return (unsigned)((n + NT - 1) / NT); }

// Face ghosts that the recovery kernel of a step writes from the cells it
// recovers (else 0; the ghost kernel then skips them, as they come first in
// ghost_one's numbering): those of the leading axes (x; x and y; all three)
// whose faces are periodic, outflow or reflecting (each ghost a copy of one
// cell of its own line, sign-flipped for reflection) and that hold at least
// ng cells (every source interior).  *axes: how many axes.  The recovering
// thread stores them from its registers, into cache lines its line's
// primitives already occupy along x, and as whole rows along y and z; a
// ghost kernel would read every source again (and gather x-face ghosts one
// cache line per variable per ghost).
inline long recovery_ghosts(const gmunu_grid_desc &d, int *axes) {
  const long nin = (long)d.n[0] * d.n[1] * d.n[2];
  long tot = 0;
  int a = 0;
  for (; a < d.ndim; a++) {
    bool ok = d.n[a] >= d.ng;
    for (int s = 0; s < 2; s++) {
      const int bc = d.bc[a][s];
      ok = ok && (bc == GMUNU_BC_PERIODIC || bc == GMUNU_BC_OUTFLOW || bc == GMUNU_BC_REFLECT);
    }
    if (!ok) break;
    tot += 2L * d.ng * (nin / d.n[a]);
  }
  *axes = a;
  return tot;
}

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

inline bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

inline int launch_status() { return hipGetLastError() == hipSuccess ? GMUNU_OK : GMUNU_EHIP; }

}  // namespace gm
