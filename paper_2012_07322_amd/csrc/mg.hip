// Cell-centred multigrid solver and elliptic divergence cleaning for MI355X
// (gfx950): level hierarchy, kernels and the C ABI of include/gmunu_mg.h.
//
// Cheong et al., "Gmunu" (arXiv 2012.07322), section 2.7 and section 2.2.
// Every operation of a cycle is one launch over the cells (or ghosts) of one
// level, one thread per cell: the smoother updates one colour of the
// red-black ordering per launch (i + j + k even first), the residual, the
// restriction (volume-weighted mean of the children), the FAS coarse
// right-hand side and the Kwak prolongation of the coarse correction.  The
// geometry of the reference-metric Laplacian factorises into per-axis 1D
// tables per level (weights toward the lower and upper neighbour, the
// metric factors of the transverse terms, cell volumes), so a cell's
// operator is a handful of table reads and FMAs.  The residual norm is a
// grid-stride maximum with wavefront shuffles, one partial per workgroup and
// one finishing workgroup: no atomics, no memset.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <vector>

#include "../../include/gmunu.h"
#include "../../include/gmunu_mg.h"
#include "gmunu_dev.hpp"
#include "gmunu_host.hpp"
#include "gmunu_tile.hpp"

using namespace gm;

namespace {

constexpr int kMaxLevels = 16;
constexpr int kNormParts = 16384;
// after the norm's result: the state of a chunk of dynamical-metric steps
// (gmunu_mg_dynamical_steps: trigger step, time at that step)
constexpr int kGateSlots = 2;

// One level as the kernels see it.
struct MgGeo {
  int ndim, coord;
  int n[3], g[3];
  long s1, s2, nt;  // strides of axes 1 and 2, entries
  double ih2_2;     // 1 / h^2 along axis 2
  double h[3];
  // per axis-0 index (ghosts included)
  const double *a0m, *a0p, *g1, *g2, *vol0, *sg0;
  // per axis-1 index
  const double *a1m, *a1p, *s2t, *vol1, *sg1;
  int bc[3][2];
  double rob_lo, rob_hi;  // Robin ghost factors on axis 0 (centre inside / centre of the ghost)
  double x0[3];           // lower face coordinate per axis (Cartesian Robin factors)
  unsigned vodd[3][2];    // vector equations: components odd across each mirror face (bit q)
  int power, power2;
  double offset;
  int line;  // smoother: alternating zebra line relaxation (else red-black points)
  // vector operator (Cartesian): 1/h_a^2, 1/(4 h_a h_b) for the axis pairs
  // (0,1), (0,2), (1,2), and the inverse diagonal of each component's row
  double vih2[3], vmix[3], vidg[3];
};

// Running maximum of |v|; a NaN counts as infinite, so that a solution gone
// NaN never reads as converged.
__device__ __forceinline__ double mg_absmax(double m, double v) { return v != v ? INFINITY : fmax(m, fabs(v)); }

__device__ __forceinline__ long mg_off(const MgGeo &G, int i, int j, int k) {
  return (long)(k + G.g[2]) * G.s2 + (long)(j + G.g[1]) * G.s1 + (i + G.g[0]);
}

__device__ __forceinline__ double mg_ipow(double w, int q) {
  double r = 1.0;
  for (int e = q < 0 ? -q : q; e > 0; e--) r *= w;
  return q < 0 ? 1.0 / r : r;
}

// a (u + c)^p + a2 (u + c)^q and its derivative in u.
__device__ __forceinline__ double mg_nl(const MgGeo &G, double a, double a2, double u) {
  const double w = u + G.offset;
  const double t = G.power == 0 ? a : G.power == 1 ? a * w : a / w;
  return a2 != 0.0 ? t + a2 * mg_ipow(w, G.power2) : t;
}
__device__ __forceinline__ double mg_nl_du(const MgGeo &G, double a, double a2, double u) {
  const double w = u + G.offset;
  const double t = G.power == 0 ? 0.0 : G.power == 1 ? a : -a / (w * w);
  return a2 != 0.0 ? t + a2 * G.power2 * mg_ipow(w, G.power2 - 1) : t;
}

// Robin ghost factor r_in / r_ghost for the ghost of boundary cell c across
// face (a, up): on spherical grids (axis 0) the level's constants; on
// Cartesian and cylindrical grids r is the distance of the cell centres
// from the origin (x, y, z; or R, z) -- the conditions u + x.grad u = 0 and
// u + R du/dR + z du/dz = 0 of section 2.6 as a 1/r fall-off between the
// cell and its ghost.
__device__ __forceinline__ double mg_rob(const MgGeo &G, int i, int j, int k, int a, bool up) {
  if (G.coord == GMUNU_SPH) return up ? G.rob_hi : G.rob_lo;
  const int c[3] = {i, j, k};
  const int nb = G.coord == GMUNU_CYL ? 2 : 3;
  double ri = 0.0, rg = 0.0;
#pragma unroll
  for (int b = 0; b < 3; b++) {
    if (b >= G.ndim || b >= nb) continue;
    const double xi = G.x0[b] + (c[b] + 0.5) * G.h[b];
    const double xg = b == a ? G.x0[b] + (c[b] + (up ? 1 : -1) + 0.5) * G.h[b] : xi;
    ri += xi * xi;
    rg += xg * xg;
  }
  return sqrt(ri) / sqrt(rg);
}

// Neighbour of interior cell (i, j, k) along axis a (stride S) on the side
// `up`: the stored value inside, else the boundary rule applied to the cell
// itself (the value a ghost fill would store there).
__device__ __forceinline__ double mg_nb(const MgGeo &G, const double *__restrict__ u, long o, int i, int j, int k,
                                        int a, long S, bool up) {
  const int n = G.n[a], c = a == 0 ? i : a == 1 ? j : k;
  if (up ? c < n - 1 : c > 0) return u[up ? o + S : o - S];
  const int kind = G.bc[a][up ? 1 : 0];
  if (kind == GMUNU_MG_PERIODIC) return u[up ? o - (long)(n - 1) * S : o + (long)(n - 1) * S];
  const double ui = u[o];
  return kind == GMUNU_MG_DIRICHLET ? -ui : kind == GMUNU_MG_NEUMANN ? ui : ui * mg_rob(G, i, j, k, a, up);
}

// L(u) at interior cell (i,j,k) (linear offset o) and dL/du there.  GH:
// neighbours across the boundary from u's ghost entries as stored; else
// from the boundary rule (mg_nb), so that no ghost fill is needed.
template <bool GH>
__device__ __forceinline__ double mg_L(const MgGeo &G, const double *__restrict__ u, double av, double a2v, int i,
                                       int j, int k, long o, double *dg) {
  const int I = i + G.g[0], J = j + G.g[1];
  const double uc = u[o];
  double wm = G.a0m[I], wp = G.a0p[I];
  double um = GH ? u[o - 1] : mg_nb(G, u, o, i, j, k, 0, 1, false);
  double up = GH ? u[o + 1] : mg_nb(G, u, o, i, j, k, 0, 1, true);
  double lap = wp * (up - uc) - wm * (uc - um);
  double d = -(wm + wp);
  if (G.ndim > 1) {
    const double gi = G.g1[I];
    wm = gi * G.a1m[J];
    wp = gi * G.a1p[J];
    um = GH ? u[o - G.s1] : mg_nb(G, u, o, i, j, k, 1, G.s1, false);
    up = GH ? u[o + G.s1] : mg_nb(G, u, o, i, j, k, 1, G.s1, true);
    lap += wp * (up - uc) - wm * (uc - um);
    d -= wm + wp;
  }
  if (G.ndim > 2) {
    const double w = G.g2[I] * G.s2t[J] * G.ih2_2;
    um = GH ? u[o - G.s2] : mg_nb(G, u, o, i, j, k, 2, G.s2, false);
    up = GH ? u[o + G.s2] : mg_nb(G, u, o, i, j, k, 2, G.s2, true);
    lap += w * (up - uc) - w * (uc - um);
    d -= 2.0 * w;
  }
  if (dg) *dg = d - mg_nl_du(G, av, a2v, uc);
  return lap - mg_nl(G, av, a2v, uc);
}

// Interior cell number t (x fastest); 32-bit arithmetic (a level has fewer
// than 2^32 cells, which validation ensures).
__device__ __forceinline__ void mg_cell(const MgGeo &G, long t, int &i, int &j, int &k) {
  const unsigned u = (unsigned)t, n0 = (unsigned)G.n[0], n1 = (unsigned)G.n[1];
  const unsigned r = u / n0;
  i = (int)(u - r * n0);
  k = (int)(r / n1);
  j = (int)(r - (unsigned)k * n1);
}

__device__ __forceinline__ long mg_cells(const MgGeo &G) { return (long)G.n[0] * G.n[1] * G.n[2]; }

// Face-adjacent ghost number t: axis, side, transverse cell.
__device__ __forceinline__ void mg_ghost_one(const MgGeo &G, double *u, long t) {
  for (int a = 0; a < G.ndim; a++) {
    const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
    const long per = 2L * G.n[b1] * G.n[b2];
    if (t >= per) {
      t -= per;
      continue;
    }
    const int side = (int)(t & 1);
    const long tr = t >> 1;
    int gc[3], sc[3];
    gc[b1] = sc[b1] = (int)(tr % G.n[b1]);
    gc[b2] = sc[b2] = (int)(tr / G.n[b1]);
    gc[a] = side == 0 ? -1 : G.n[a];
    const int kind = G.bc[a][side];
    double v;
    if (kind == GMUNU_MG_PERIODIC) {
      sc[a] = side == 0 ? G.n[a] - 1 : 0;
      v = u[mg_off(G, sc[0], sc[1], sc[2])];
    } else {
      sc[a] = side == 0 ? 0 : G.n[a] - 1;
      const double ui = u[mg_off(G, sc[0], sc[1], sc[2])];
      v = kind == GMUNU_MG_DIRICHLET ? -ui
          : kind == GMUNU_MG_NEUMANN ? ui
                                     : ui * mg_rob(G, sc[0], sc[1], sc[2], a, side == 1);
    }
    u[mg_off(G, gc[0], gc[1], gc[2])] = v;
    return;
  }
}

__device__ __forceinline__ long mg_ghost_count(const MgGeo &G) {
  long s = 0;
  for (int a = 0; a < G.ndim; a++) {
    const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
    s += 2L * G.n[b1] * G.n[b2];
  }
  return s;
}

// Face ghost t of component q of a vector field: periodic wrap or mirror
// with the component's parity across that face.
__device__ __forceinline__ void mgv_ghost_one(const MgGeo &G, double *u, int q, long t) {
  for (int a = 0; a < G.ndim; a++) {
    const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
    const long per = 2L * G.n[b1] * G.n[b2];
    if (t >= per) {
      t -= per;
      continue;
    }
    const int side = (int)(t & 1);
    const long tr = t >> 1;
    int gc[3], sc[3];
    gc[b1] = sc[b1] = (int)(tr % G.n[b1]);
    gc[b2] = sc[b2] = (int)(tr / G.n[b1]);
    gc[a] = side == 0 ? -1 : G.n[a];
    double v;
    if (G.bc[a][side] == GMUNU_MG_PERIODIC) {
      sc[a] = side == 0 ? G.n[a] - 1 : 0;
      v = u[mg_off(G, sc[0], sc[1], sc[2])];
    } else {
      sc[a] = side == 0 ? 0 : G.n[a] - 1;
      const double ui = u[mg_off(G, sc[0], sc[1], sc[2])];
      v = (G.vodd[a][side] >> q) & 1 ? -ui : ui;
    }
    u[mg_off(G, gc[0], gc[1], gc[2])] = v;
    return;
  }
}

template <int NC>
__global__ __launch_bounds__(NT) void k_mg_ghosts(const MgGeo G, double *u) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
#pragma unroll
  for (int q = 0; q < NC; q++) {
    if (NC == 1)
      mg_ghost_one(G, u, t);
    else
      mgv_ghost_one(G, u + q * G.nt, q, t);
  }
}

// One colour of red-black Newton-Gauss-Seidel: thread t -> the t-th cell of
// that colour (every other cell of a row).  With fs non-null, f, a and a2
// are read from colour-split copies (per row the even-i cells, then the odd
// ones), so that a colour reads them contiguously.
__device__ __forceinline__ void mg_smooth_one(const MgGeo &G, double *u, const double *__restrict__ f,
                                              const double *__restrict__ a, const double *__restrict__ a2, int colour,
                                              long t, const double *__restrict__ fs = nullptr,
                                              const double *__restrict__ as = nullptr,
                                              const double *__restrict__ a2s = nullptr) {
  const unsigned hrow = (unsigned)(G.n[0] + 1) >> 1, n1 = (unsigned)G.n[1];
  if (t >= (long)hrow * G.n[1] * G.n[2]) return;
  const unsigned row = (unsigned)t / hrow;
  const int k = (int)(row / n1), j = (int)(row - (unsigned)k * n1);
  const int i = (int)((unsigned)t - row * hrow) * 2 + ((j + k + colour) & 1);
  if (i >= G.n[0]) return;
  const long o = mg_off(G, i, j, k);
  double fv, av, a2v;
  if (fs) {
    const long si = (long)row * G.n[0] + (long)(i & 1) * hrow + (i >> 1);
    fv = fs[si];
    av = as ? as[si] : 0.0;
    a2v = a2s ? a2s[si] : 0.0;
  } else {
    fv = f[o];
    av = a ? a[o] : 0.0;
    a2v = a2 ? a2[o] : 0.0;
  }
  double dg;
  const double Lu = mg_L<false>(G, u, av, a2v, i, j, k, o, &dg);
  u[o] -= (Lu - fv) / dg;
}

__global__ __launch_bounds__(NT) void k_mg_smooth(const MgGeo G, double *u, const double *__restrict__ f,
                                                  const double *__restrict__ a, const double *__restrict__ a2,
                                                  int colour, const double *__restrict__ fs,
                                                  const double *__restrict__ as, const double *__restrict__ a2s) {
  mg_smooth_one(G, u, f, a, a2, colour, (long)blockIdx.x * NT + threadIdx.x, fs, as, a2s);
}

// Colour-split copy of an interior array: per row the even-i cells, then
// the odd-i cells (the layout mg_smooth_one reads with fs).
__global__ __launch_bounds__(NT) void k_mg_split(const MgGeo G, const double *__restrict__ src,
                                                 double *__restrict__ dst) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= mg_cells(G)) return;
  int i, j, k;
  mg_cell(G, t, i, j, k);
  const long row = (long)k * G.n[1] + j, hrow = (G.n[0] + 1) >> 1;
  dst[row * G.n[0] + (i & 1) * hrow + (i >> 1)] = src[mg_off(G, i, j, k)];
}

// The coarsest-level solver: `sweeps` red-black sweeps by one workgroup,
// the colours separated by workgroup barriers instead of launches.  With
// lds != 0 the level's arrays (u, f and the given a, a2) are first copied
// into dynamic LDS, relaxed there and u copied back: the sweeps are then
// bound by LDS rather than global-memory latency.
__global__ __launch_bounds__(NT) void k_mg_coarse(const MgGeo G, double *u, const double *__restrict__ f,
                                                  const double *__restrict__ a, const double *__restrict__ a2,
                                                  int sweeps, int lds) {
  extern __shared__ double sm[];
  double *uu = u;
  const double *ff = f, *aa = a, *aa2 = a2;
  if (lds) {
    double *p = sm;
    for (long e = threadIdx.x; e < G.nt; e += NT) p[e] = u[e];
    uu = p;
    p += G.nt;
    for (long e = threadIdx.x; e < G.nt; e += NT) p[e] = f[e];
    ff = p;
    p += G.nt;
    if (a) {
      for (long e = threadIdx.x; e < G.nt; e += NT) p[e] = a[e];
      aa = p;
      p += G.nt;
    }
    if (a2) {
      for (long e = threadIdx.x; e < G.nt; e += NT) p[e] = a2[e];
      aa2 = p;
    }
    __syncthreads();
  }
  const long nc = (long)((G.n[0] + 1) >> 1) * G.n[1] * G.n[2];
  for (int s = 0; s < sweeps; s++)
    for (int c = 0; c < 2; c++) {
      for (long t = threadIdx.x; t < nc; t += NT) mg_smooth_one(G, uu, ff, aa, aa2, c, t);
      __syncthreads();
    }
  if (lds)
    for (long e = threadIdx.x; e < G.nt; e += NT) u[e] = uu[e];
}

// ---- Line relaxation --------------------------------------------------------
// An alternative to the paper's point smoother for the anisotropic cells on
// which section 2.7 notes that point smoothers converge slowly (spherical
// polar grids).  One workgroup per line (up to kLineThreads lanes, one or
// more cells per lane).  The line's tridiagonal system (couplings toward the
// lower and upper neighbour along the line, diagonal, right-hand side) is
// built in LDS by the lanes, cell by cell, and solved by parallel cyclic
// reduction: at stride s every row eliminates its couplings to the rows s
// below and s above, so after ceil(log2 n) doublings each row holds one
// unknown.  Two copies of the four arrays alternate between doublings.

constexpr int kLineWave = 64;
constexpr int kLineThreads = 512;
constexpr int kCoarseLineThreads = 1024;  // one-workgroup coarsest-level line solvers
constexpr int kMaxLine = 1024;

// Weights of the flux-form Laplacian from cell (I, J) (ghost-inclusive
// indices) toward its lower and upper neighbour along axis a: the terms
// of mg_L.
__device__ __forceinline__ void mg_w(const MgGeo &G, int I, int J, int a, double &wm, double &wp) {
  if (a == 0) {
    wm = G.a0m[I];
    wp = G.a0p[I];
  } else if (a == 1) {
    wm = G.g1[I] * G.a1m[J];
    wp = G.g1[I] * G.a1p[J];
  } else {
    wm = wp = G.g2[I] * G.s2t[J] * G.ih2_2;
  }
}

// Factor s of the boundary rule ghost = s u_cell across the non-periodic
// face (a, up) of boundary cell c.
__device__ __forceinline__ double mg_fold(const MgGeo &G, const int c[3], int a, bool up) {
  const int kind = G.bc[a][up ? 1 : 0];
  return kind == GMUNU_MG_DIRICHLET ? -1.0 : kind == GMUNU_MG_NEUMANN ? 1.0 : mg_rob(G, c[0], c[1], c[2], a, up);
}

// First cell of line t of colour `colour` along axis a: the transverse
// axes b1 < b2, each active one coloured by its index parity (bit 0: b1,
// bit 1: b2).  False past the last line.
__device__ __forceinline__ bool mg_line(const MgGeo &G, int a, int colour, long t, int c[3]) {
  const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
  const int p1 = colour & 1, p2 = (colour >> 1) & 1;
  const long h1 = b1 < G.ndim ? (G.n[b1] - p1 + 1) >> 1 : 1;
  const long h2 = b2 < G.ndim ? (G.n[b2] - p2 + 1) >> 1 : 1;
  if (t >= h1 * h2) return false;
  const int t1 = b1 < G.ndim ? 2 * (int)(t % h1) + p1 : 0;
  const int t2 = b2 < G.ndim ? 2 * (int)(t / h1) + p2 : 0;
  // (b1, b2) = (1, 2), (0, 2), (0, 1) for a = 0, 1, 2 (no dynamic indexing of c)
  c[0] = a == 0 ? 0 : t1;
  c[1] = a == 0 ? t1 : a == 1 ? 0 : t2;
  c[2] = a == 2 ? 0 : t2;
  return true;
}

// Parallel cyclic reduction of the system in sm (A: lower couplings, B:
// diagonal, C: upper couplings, D: right-hand side, n entries each, A[0] =
// C[n-1] = 0) by nl lanes (this one: ln); returns the copy (0 or 1)
// holding the decoupled rows, whose solution is D / B.  The doublings are
// separated by workgroup barriers, so every thread of the workgroup calls
// this with the same n.
__device__ __forceinline__ int mg_pcr(double *sm, int n, int ln, int nl) {
  int p = 0;
  for (int s = 1; s < n; s <<= 1) {
    const double *A = sm + p * 4 * n, *B = A + n, *C = B + n, *D = C + n;
    double *A2 = sm + (1 - p) * 4 * n, *B2 = A2 + n, *C2 = B2 + n, *D2 = C2 + n;
    for (int m = ln; m < n; m += nl) {
      double b = B[m], d = D[m], na = 0.0, nc = 0.0;
      if (m >= s) {
        const double al = -A[m] / B[m - s];
        na = al * A[m - s];
        b += al * C[m - s];
        d += al * D[m - s];
      }
      if (m + s < n) {
        const double ga = -C[m] / B[m + s];
        nc = ga * C[m + s];
        b += ga * A[m + s];
        d += ga * D[m + s];
      }
      A2[m] = na;
      B2[m] = b;
      C2[m] = nc;
      D2[m] = d;
    }
    __syncthreads();
    p ^= 1;
  }
  return p;
}

// One Newton step of the line from cell c along axis ax by nl lanes (this
// one: ln; LDS sm of 8 n doubles; live = false: lanes with no line that
// only keep the workgroup's barriers) with the exact Jacobian with
// respect to the line's cells: the couplings along the line, on the
// diagonal mg_L's dL/du plus, across each non-periodic boundary face of
// the cell, the weight toward the ghost times its boundary-rule factor (the
// ghost follows the cell); right-hand side f - L(u); u += the solution.
__device__ __forceinline__ void mg_line_step(const MgGeo &G, double *u, const double *__restrict__ f,
                                             const double *__restrict__ a, const double *__restrict__ a2, int ax,
                                             const int c[3], bool live, double *sm, int ln, int nl) {
  const int n = G.n[ax];
  for (int m = ln; live && m < n; m += nl) {
    const int cc[3] = {ax == 0 ? m : c[0], ax == 1 ? m : c[1], ax == 2 ? m : c[2]};
    const long o = mg_off(G, cc[0], cc[1], cc[2]);
    double dg, wm, wp;
    const double Lu = mg_L<false>(G, u, a ? a[o] : 0.0, a2 ? a2[o] : 0.0, cc[0], cc[1], cc[2], o, &dg);
#pragma unroll
    for (int b = 0; b < 3; b++) {
      if (b >= G.ndim || G.bc[b][0] == GMUNU_MG_PERIODIC || (cc[b] > 0 && cc[b] < G.n[b] - 1)) continue;
      mg_w(G, cc[0] + G.g[0], cc[1] + G.g[1], b, wm, wp);
      if (cc[b] == 0) dg += wm * mg_fold(G, cc, b, false);
      if (cc[b] == G.n[b] - 1) dg += wp * mg_fold(G, cc, b, true);
    }
    mg_w(G, cc[0] + G.g[0], cc[1] + G.g[1], ax, wm, wp);
    if (m == 0) wm = 0.0;
    if (m == n - 1) wp = 0.0;
    sm[m] = wm;
    sm[n + m] = dg;
    sm[2 * n + m] = wp;
    sm[3 * n + m] = f[o] - Lu;
  }
  __syncthreads();
  const double *R = sm + mg_pcr(sm, n, ln, nl) * 4 * n;
  for (int m = ln; live && m < n; m += nl) {
    const int cc[3] = {ax == 0 ? m : c[0], ax == 1 ? m : c[1], ax == 2 ? m : c[2]};
    u[mg_off(G, cc[0], cc[1], cc[2])] += R[3 * n + m] / R[n + m];
  }
}

// Lines of one colour along axis ax, one workgroup per line.
__global__ __launch_bounds__(kLineThreads) void k_mg_line(const MgGeo G, double *u, const double *__restrict__ f,
                                                          const double *__restrict__ a,
                                                          const double *__restrict__ a2, int ax, int colour) {
  extern __shared__ double sm[];
  int c[3];
  if (!mg_line(G, ax, colour, blockIdx.x, c)) return;
  mg_line_step(G, u, f, a, a2, ax, c, true, sm, threadIdx.x, blockDim.x);
}

// Number of lines of colour `colour` along axis a.
__host__ __device__ __forceinline__ long mg_line_count(const MgGeo &G, int a, int colour) {
  const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
  const long h1 = b1 < G.ndim ? (G.n[b1] - (colour & 1) + 1) >> 1 : 1;
  const long h2 = b2 < G.ndim ? (G.n[b2] - ((colour >> 1) & 1) + 1) >> 1 : 1;
  return h1 * h2;
}

// The coarsest-level solver of the line smoother: `sweeps` line sweeps by
// one workgroup of kCoarseLineThreads threads, its wavefronts taking a
// colour's lines in rounds, colours and axes separated by barriers.
// Dynamic LDS: the level's u, f (and the given a, a2) copied in and u
// copied back, then 8 nmax doubles per wavefront for the line systems.
__global__ __launch_bounds__(kCoarseLineThreads) void k_mg_line_coarse(const MgGeo G, double *u,
                                                                       const double *__restrict__ f,
                                                                       const double *__restrict__ a,
                                                                       const double *__restrict__ a2, int sweeps,
                                                                       int nmax) {
  extern __shared__ double sm[];
  double *p = sm, *uu = p;
  for (long e = threadIdx.x; e < G.nt; e += kCoarseLineThreads) p[e] = u[e];
  p += G.nt;
  for (long e = threadIdx.x; e < G.nt; e += kCoarseLineThreads) p[e] = f[e];
  const double *ff = p, *aa = nullptr, *aa2 = nullptr;
  p += G.nt;
  if (a) {
    for (long e = threadIdx.x; e < G.nt; e += kCoarseLineThreads) p[e] = a[e];
    aa = p;
    p += G.nt;
  }
  if (a2) {
    for (long e = threadIdx.x; e < G.nt; e += kCoarseLineThreads) p[e] = a2[e];
    aa2 = p;
    p += G.nt;
  }
  __syncthreads();
  const int w = threadIdx.x / kLineWave, ln = threadIdx.x % kLineWave, nw = kCoarseLineThreads / kLineWave;
  for (int s = 0; s < sweeps; s++)
    for (int ax = 0; ax < G.ndim; ax++) {
      if (G.bc[ax][0] == GMUNU_MG_PERIODIC) continue;
      for (int col = 0; col < 1 << (G.ndim - 1); col++) {
        const long nl = mg_line_count(G, ax, col);
        for (long t0 = 0; t0 < nl; t0 += nw) {
          int c[3] = {0, 0, 0};
          const bool live = mg_line(G, ax, col, t0 + w, c);
          mg_line_step(G, uu, ff, aa, aa2, ax, c, live, p + (long)w * 8 * nmax, ln, kLineWave);
          __syncthreads();
        }
      }
    }
  for (long e = threadIdx.x; e < G.nt; e += kCoarseLineThreads) u[e] = uu[e];
}

// out = L(u) on the interior.
__global__ __launch_bounds__(NT) void k_mg_apply(const MgGeo G, const double *__restrict__ u,
                                                 const double *__restrict__ a, const double *__restrict__ a2,
                                                 double *__restrict__ out) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= mg_cells(G)) return;
  int i, j, k;
  mg_cell(G, t, i, j, k);
  const long o = mg_off(G, i, j, k);
  out[o] = mg_L<true>(G, u, a ? a[o] : 0.0, a2 ? a2[o] : 0.0, i, j, k, o, nullptr);
}

// Per-workgroup maxima of |f - L(u)| over a grid-stride range of cells.
__global__ __launch_bounds__(NT) void k_mg_norm(const MgGeo G, const double *__restrict__ u,
                                                const double *__restrict__ f, const double *__restrict__ a,
                                                const double *__restrict__ a2, double *part) {
  double m = 0.0;
  for (long t = (long)blockIdx.x * NT + threadIdx.x; t < mg_cells(G); t += (long)gridDim.x * NT) {
    int i, j, k;
    mg_cell(G, t, i, j, k);
    const long o = mg_off(G, i, j, k);
    m = mg_absmax(m, f[o] - mg_L<false>(G, u, a ? a[o] : 0.0, a2 ? a2[o] : 0.0, i, j, k, o, nullptr));
  }
  m = block_max(m);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

__global__ __launch_bounds__(NT) void k_mg_norm_finish(double *part, int nparts) {
  double m = 0.0;
  for (int b = threadIdx.x; b < nparts; b += NT) m = fmax(m, part[b]);
  m = block_max(m);
  if (threadIdx.x == 0) part[kNormParts] = m;
}

// coarse = volume-weighted mean of the children (F: fine level, C: coarse).
__global__ __launch_bounds__(NT) void k_mg_restrict(const MgGeo F, const MgGeo C, const double *__restrict__ fine,
                                                    double *__restrict__ coarse) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= mg_cells(C)) return;
  int i, j, k;
  mg_cell(C, t, i, j, k);
  double s = 0.0, w = 0.0;
  const int nch = 1 << F.ndim;
  for (int ch = 0; ch < nch; ch++) {
    const int fi = 2 * i + (ch & 1);
    const int fj = F.ndim > 1 ? 2 * j + ((ch >> 1) & 1) : j;
    const int fk = F.ndim > 2 ? 2 * k + ((ch >> 2) & 1) : k;
    const double v = F.vol0[fi + F.g[0]] * F.vol1[fj + F.g[1]];
    s += v * fine[mg_off(F, fi, fj, fk)];
    w += v;
  }
  coarse[mg_off(C, i, j, k)] = s / w;
}

// FAS coarse problem: f_c = L_c(u_c) + r_c, and uo_c = u_c (u_c's ghosts set).
__global__ __launch_bounds__(NT) void k_mg_fas_rhs(const MgGeo C, const double *__restrict__ u,
                                                   const double *__restrict__ a, const double *__restrict__ a2,
                                                   const double *__restrict__ r, double *__restrict__ f,
                                                   double *__restrict__ uo) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= mg_cells(C)) return;
  int i, j, k;
  mg_cell(C, t, i, j, k);
  const long o = mg_off(C, i, j, k);
  f[o] = mg_L<false>(C, u, a ? a[o] : 0.0, a2 ? a2[o] : 0.0, i, j, k, o, nullptr) + r[o];
  uo[o] = u[o];
}

// Coarse problem of a fine level in one pass over the coarse cells: the
// residual f - L(u) of each child (boundary rule inline) and the
// volume-weighted means of u and of the residual into the coarse u and r.
__global__ __launch_bounds__(NT) void k_mg_restrict_res(const MgGeo F, const MgGeo C, const double *__restrict__ u,
                                                        const double *__restrict__ f, const double *__restrict__ a,
                                                        const double *__restrict__ a2, double *__restrict__ uc,
                                                        double *__restrict__ rc) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= mg_cells(C)) return;
  int i, j, k;
  mg_cell(C, t, i, j, k);
  double su = 0.0, sr = 0.0, w = 0.0;
  const int nch = 1 << F.ndim;
  for (int ch = 0; ch < nch; ch++) {
    const int fi = 2 * i + (ch & 1);
    const int fj = F.ndim > 1 ? 2 * j + ((ch >> 1) & 1) : j;
    const int fk = F.ndim > 2 ? 2 * k + ((ch >> 2) & 1) : k;
    const double v = F.vol0[fi + F.g[0]] * F.vol1[fj + F.g[1]];
    const long o = mg_off(F, fi, fj, fk);
    su += v * u[o];
    sr += v * (f[o] - mg_L<false>(F, u, a ? a[o] : 0.0, a2 ? a2[o] : 0.0, fi, fj, fk, o, nullptr));
    w += v;
  }
  const long oc = mg_off(C, i, j, k);
  uc[oc] = su / w;
  rc[oc] = sr / w;
}

// u_F += P (u_C - uo_C): Kwak prolongation of the coarse correction, whose
// values across the boundary follow the boundary rule (it is homogeneous,
// so the correction obeys it too); NC components back to back.
__device__ __forceinline__ double mg_corr(const MgGeo &C, const double *__restrict__ u,
                                          const double *__restrict__ uo, long o) {
  return u[o] - uo[o];
}

template <int NC>
__global__ __launch_bounds__(NT) void k_mg_correct(const MgGeo C, const MgGeo F, const double *__restrict__ uc0,
                                                   const double *__restrict__ uoc0, double *__restrict__ fine0) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= mg_cells(F)) return;
  int fc[3];
  mg_cell(F, t, fc[0], fc[1], fc[2]);
  int cc[3];
#pragma unroll
  for (int a = 0; a < 3; a++) cc[a] = a < F.ndim ? fc[a] >> 1 : fc[a];
  const double w0 = F.ndim == 1 ? 0.75 : F.ndim == 2 ? 0.5 : 0.25;
  const long oc = mg_off(C, cc[0], cc[1], cc[2]);
  const long S[3] = {1, C.s1, C.s2};
#pragma unroll
  for (int q = 0; q < NC; q++) {
    const double *uc = uc0 + q * C.nt, *uoc = uoc0 + q * C.nt;
    double *fine = fine0 + q * F.nt;
    const double e0 = mg_corr(C, uc, uoc, oc);
    double s = w0 * e0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
      if (a >= F.ndim) continue;
      const bool up = fc[a] & 1;
      const int c = cc[a], n = C.n[a];
      double e;
      if (up ? c < n - 1 : c > 0) {
        e = mg_corr(C, uc, uoc, up ? oc + S[a] : oc - S[a]);
      } else {
        const int kind = C.bc[a][up ? 1 : 0];
        if (kind == GMUNU_MG_PERIODIC)
          e = mg_corr(C, uc, uoc, up ? oc - (long)(n - 1) * S[a] : oc + (long)(n - 1) * S[a]);
        else if (NC == 3)  // vector components: their parity across the face
          e = (C.vodd[a][up ? 1 : 0] >> q) & 1 ? -e0 : e0;
        else
          e = kind == GMUNU_MG_DIRICHLET ? -e0
            : kind == GMUNU_MG_NEUMANN ? e0
                                       : e0 * mg_rob(C, cc[0], cc[1], cc[2], a, up);
      }
      s += 0.25 * e;
    }
    fine[mg_off(F, fc[0], fc[1], fc[2])] += s;
  }
}

// Kwak prolongation of v (coarse, ghosts set) into the fine interior:
// fine = P v (add = 0) or fine += P v (add = 1).
__global__ __launch_bounds__(NT) void k_mg_prolong(const MgGeo C, const MgGeo F, const double *__restrict__ v,
                                                   double *__restrict__ fine, int add) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= mg_cells(F)) return;
  int fc[3];
  mg_cell(F, t, fc[0], fc[1], fc[2]);
  int cc[3];
#pragma unroll
  for (int a = 0; a < 3; a++) cc[a] = a < F.ndim ? fc[a] >> 1 : fc[a];
  const double w0 = F.ndim == 1 ? 0.75 : F.ndim == 2 ? 0.5 : 0.25;
  const long oc = mg_off(C, cc[0], cc[1], cc[2]);
  double s = w0 * v[oc];
  s += 0.25 * v[oc + ((fc[0] & 1) ? 1 : -1)];
  if (F.ndim > 1) s += 0.25 * v[oc + ((fc[1] & 1) ? C.s1 : -C.s1)];
  if (F.ndim > 2) s += 0.25 * v[oc + ((fc[2] & 1) ? C.s2 : -C.s2)];
  const long of = mg_off(F, fc[0], fc[1], fc[2]);
  fine[of] = add ? fine[of] + s : s;
}

// (1/sqrt g) d_i (sqrt g q^i), centred.
__global__ __launch_bounds__(NT) void k_mg_div(const MgGeo G, const double *__restrict__ q, double *__restrict__ out) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= mg_cells(G)) return;
  int i, j, k;
  mg_cell(G, t, i, j, k);
  const int I = i + G.g[0], J = j + G.g[1];
  const long o = mg_off(G, i, j, k);
  const double sgc = G.sg0[I] * G.sg1[J];
  double s = (G.sg0[I + 1] * q[o + 1] - G.sg0[I - 1] * q[o - 1]) * G.sg1[J] / (2.0 * G.h[0]);
  if (G.ndim > 1)
    s += (G.sg1[J + 1] * q[G.nt + o + G.s1] - G.sg1[J - 1] * q[G.nt + o - G.s1]) * G.sg0[I] / (2.0 * G.h[1]);
  if (G.ndim > 2) s += (q[2 * G.nt + o + G.s2] - q[2 * G.nt + o - G.s2]) * sgc / (2.0 * G.h[2]);
  out[o] = s / sgc;
}

// q^i -= g^ii d_i phi, centred, on the interior.
__global__ __launch_bounds__(NT) void k_mg_subgrad(const MgGeo G, const double *__restrict__ phi,
                                                   double *__restrict__ q) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= mg_cells(G)) return;
  int i, j, k;
  mg_cell(G, t, i, j, k);
  const int I = i + G.g[0], J = j + G.g[1];
  const long o = mg_off(G, i, j, k);
  q[o] -= (phi[o + 1] - phi[o - 1]) / (2.0 * G.h[0]);
  if (G.ndim > 1) q[G.nt + o] -= G.g1[I] * (phi[o + G.s1] - phi[o - G.s1]) / (2.0 * G.h[1]);
  if (G.ndim > 2) q[2 * G.nt + o] -= G.g2[I] * G.s2t[J] * (phi[o + G.s2] - phi[o - G.s2]) / (2.0 * G.h[2]);
}

// ------------------------------------------- vector equations of xCFC
//
// L(X)^i = Lap X^i + (1/3) d_i d_j X^j on Cartesian grids (section 2.6),
// second differences and the four-point mixed difference of section 2.7.
// The mixed stencil couples diagonal neighbours, so the Newton-Gauss-Seidel
// smoother visits 2^ndim colours (i mod 2, j mod 2, k mod 2), one launch
// each; cells of one colour are never neighbours, and the three components
// of a cell do not enter each other's diagonal, so a colour updates all its
// cells and components at once.  Across the boundary every axis applies its
// own rule (mirror times -1 or +1, periodic wrap): a step from a cell along
// an axis is an offset and a sign, and a diagonal neighbour takes the
// product of the two steps' signs.

struct VStep {
  int dm[3], dp[3];  // offsets of the minus / plus neighbour along each axis
  unsigned neg;      // bit 6 q + a: the minus step negates component q; 6 q + 3 + a: the plus step
};

__device__ __forceinline__ void mgv_axis(const MgGeo &G, int c, int a, int S, bool up, int &d, unsigned &neg) {
  const int n = G.n[a];
  if (up ? c < n - 1 : c > 0) {
    d = up ? S : -S;
    return;
  }
  if (G.bc[a][up ? 1 : 0] == GMUNU_MG_PERIODIC) {
    d = up ? -(n - 1) * S : (n - 1) * S;
    return;
  }
  d = 0;
  const unsigned odd = G.vodd[a][up ? 1 : 0];
#pragma unroll
  for (int q = 0; q < 3; q++)
    if ((odd >> q) & 1) neg |= 1u << (6 * q + (up ? 3 : 0) + a);
}

__device__ __forceinline__ VStep mgv_steps(const MgGeo &G, int i, int j, int k) {
  VStep s;
  s.neg = 0;
  const int c[3] = {i, j, k};
  const int S[3] = {1, (int)G.s1, (int)G.s2};
#pragma unroll
  for (int a = 0; a < 3; a++) {
    s.dm[a] = s.dp[a] = 0;
    if (a >= G.ndim) continue;
    mgv_axis(G, c[a], a, S[a], false, s.dm[a], s.neg);
    mgv_axis(G, c[a], a, S[a], true, s.dp[a], s.neg);
  }
  return s;
}

__device__ __forceinline__ double mgv_sgn(unsigned neg, int bits, double v) { return (neg >> bits) & 1 ? -v : v; }

// Component b at the diagonal neighbour (sq along axis qa, sb along axis
// ab; +1 or -1): the sign is the product of its two steps' signs.
__device__ __forceinline__ double mgv_corner(const double *__restrict__ ub, const VStep &s, long o, int b, int qa,
                                             int sq, int ab, int sb) {
  const unsigned n1 = s.neg >> (6 * b + (sq > 0 ? 3 : 0) + qa), n2 = s.neg >> (6 * b + (sb > 0 ? 3 : 0) + ab);
  return mgv_sgn(n1 ^ n2, 0, ub[o + (sq > 0 ? s.dp[qa] : s.dm[qa]) + (sb > 0 ? s.dp[ab] : s.dm[ab])]);
}

// L(X) at interior cell (i, j) (offset o) on a Cartesian level, all three
// components, and the inverse diagonals (level constants: 1/h_a^2,
// 1/(4 h_a h_b) and the inverse diagonals are precomputed in MgGeo).
__device__ __forceinline__ void mgv_L_cart(const MgGeo &G, const double *__restrict__ u, const VStep &s, long o,
                                           double L[3], double idg[3]) {
  const long nt = G.nt;
#pragma unroll
  for (int q = 0; q < 3; q++) {
    const double *uq = u + q * nt;
    const double u0 = uq[o];
    double lap = 0.0, self = 0.0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
      if (a >= G.ndim) continue;
      const double up = mgv_sgn(s.neg, 6 * q + 3 + a, uq[o + s.dp[a]]);
      const double um = mgv_sgn(s.neg, 6 * q + a, uq[o + s.dm[a]]);
      const double d2 = (up - 2.0 * u0 + um) * G.vih2[a];
      lap += d2;
      if (a == q) self = d2;
    }
    double gd = self;
#pragma unroll
    for (int b = 0; b < 3; b++) {
      if (q >= G.ndim || b == q || b >= G.ndim) continue;
      const double *ub = u + b * nt;
      const double pp = mgv_corner(ub, s, o, b, q, 1, b, 1), pm = mgv_corner(ub, s, o, b, q, 1, b, -1);
      const double mp = mgv_corner(ub, s, o, b, q, -1, b, 1), mm = mgv_corner(ub, s, o, b, q, -1, b, -1);
      gd += (pp - pm - mp + mm) * G.vmix[q + b - 1];
    }
    L[q] = lap + gd * (1.0 / 3.0);
    idg[q] = G.vidg[q];
  }
}

// The same on an axisymmetric cylindrical (R, z) or spherical (r, theta)
// level in orthonormal components: the flux-form Laplacian of each
// component (the scalar operator's tables), the connection terms of the
// vector Laplacian and of grad div, mixed differences by the four-point
// formula with signed corner coordinates; diagonals per cell.
__device__ __forceinline__ void mgv_L_curv(const MgGeo &G, const double *__restrict__ u, const VStep &s, long o,
                                           int i, int j, double L[3], double idg[3]) {
  const long nt = G.nt;
  const bool two = G.ndim > 1;
  const int I = i + G.g[0], J = j + G.g[1];
  const double h0 = G.h[0], h1 = G.h[1];
  const double r = G.x0[0] + (i + 0.5) * h0, ir2 = 1.0 / (r * r);
  const double wm0 = G.a0m[I], wp0 = G.a0p[I];
  const double wm1 = two ? G.g1[I] * G.a1m[J] : 0.0, wp1 = two ? G.g1[I] * G.a1p[J] : 0.0;
  const double i4h = two ? 1.0 / (4.0 * h0 * h1) : 0.0;
  double l0[3], l1[3], u0[3];
#pragma unroll
  for (int q = 0; q < 3; q++) {
    const double *uq = u + q * nt;
    u0[q] = uq[o];
    l0[q] = wp0 * (mgv_sgn(s.neg, 6 * q + 3, uq[o + s.dp[0]]) - u0[q]) -
            wm0 * (u0[q] - mgv_sgn(s.neg, 6 * q, uq[o + s.dm[0]]));
    l1[q] = two ? wp1 * (mgv_sgn(s.neg, 6 * q + 4, uq[o + s.dp[1]]) - u0[q]) -
                      wm1 * (u0[q] - mgv_sgn(s.neg, 6 * q + 1, uq[o + s.dm[1]]))
                : 0.0;
  }
  const double dl0 = -(wm0 + wp0), dl1 = -(wm1 + wp1), dlap = dl0 + dl1;
  const double *u0p = u, *u1p = u + nt;
  if (G.coord == GMUNU_CYL) {
    double mixz = 0.0, mixR = 0.0;
    if (two) {
#pragma unroll
      for (int di = -1; di <= 1; di += 2)
#pragma unroll
        for (int dj = -1; dj <= 1; dj += 2) {
          mixz += di * dj * mgv_corner(u1p, s, o, 1, 0, di, 1, dj);
          mixR += di * dj * (r + di * h0) * mgv_corner(u0p, s, o, 0, 0, di, 1, dj);
        }
      mixz *= i4h;
      mixR *= i4h / r;
    }
    L[0] = l0[0] + l1[0] - u0[0] * ir2 + (l0[0] - u0[0] * ir2 + mixz) * (1.0 / 3.0);
    idg[0] = 1.0 / (dlap - ir2 + (dl0 - ir2) * (1.0 / 3.0));
    L[1] = l0[1] + l1[1] + (mixR + l1[1]) * (1.0 / 3.0);
    idg[1] = 1.0 / (dlap + dl1 * (1.0 / 3.0));
    L[2] = l0[2] + l1[2] - u0[2] * ir2;
    idg[2] = 1.0 / (dlap - ir2);
  } else {
    const double sn = G.sg1[J], is2 = 1.0 / (sn * sn);
    double dth = 0.0, dr = 0.0, mixt = 0.0, mixr = 0.0;
    if (two) {
      dth = (G.sg1[J + 1] * mgv_sgn(s.neg, 6 + 4, u1p[o + s.dp[1]]) -
             G.sg1[J - 1] * mgv_sgn(s.neg, 6 + 1, u1p[o + s.dm[1]])) /
            (2.0 * h1);
      dr = (mgv_sgn(s.neg, 4, u0p[o + s.dp[1]]) - mgv_sgn(s.neg, 1, u0p[o + s.dm[1]])) / (2.0 * h1);
#pragma unroll
      for (int di = -1; di <= 1; di += 2)
#pragma unroll
        for (int dj = -1; dj <= 1; dj += 2) {
          const double rc = r + di * h0;
          mixt += di * dj * G.sg1[J + dj] * mgv_corner(u1p, s, o, 1, 0, di, 1, dj);
          mixr += di * dj * (rc * rc) * mgv_corner(u0p, s, o, 0, 0, di, 1, dj);
        }
      // (1/sin) d_r d_th (sin A_th / r) without dividing by a corner radius
      mixt = (mixt * i4h / r - dth * ir2) / sn;
      mixr *= i4h * ir2 / r;
    }
    L[0] = l0[0] + l1[0] - 2.0 * u0[0] * ir2 - 2.0 * ir2 / sn * dth +
           (l0[0] - 2.0 * u0[0] * ir2 + mixt) * (1.0 / 3.0);
    idg[0] = 1.0 / (dlap - 2.0 * ir2 + (dl0 - 2.0 * ir2) * (1.0 / 3.0));
    L[1] = l0[1] + l1[1] - u0[1] * ir2 * is2 + 2.0 * ir2 * dr + (mixr + l1[1] - u0[1] * ir2 * is2) * (1.0 / 3.0);
    idg[1] = 1.0 / (dlap - ir2 * is2 + (dl1 - ir2 * is2) * (1.0 / 3.0));
    L[2] = l0[2] + l1[2] - u0[2] * ir2 * is2;
    idg[2] = 1.0 / (dlap - ir2 * is2);
  }
}

__device__ __forceinline__ void mgv_L(const MgGeo &G, const double *__restrict__ u, long o, int i, int j, int k,
                                      double L[3], double idg[3]) {
  const VStep s = mgv_steps(G, i, j, k);
  if (G.coord == GMUNU_CART)
    mgv_L_cart(G, u, s, o, L, idg);
  else
    mgv_L_curv(G, u, s, o, i, j, L, idg);
}

// Cells of colour `colour` (bit a: parity along axis a) on a level.
__device__ __forceinline__ long mgv_colour_cells(const MgGeo &G, int colour) {
  long n = 1;
#pragma unroll
  for (int a = 0; a < 3; a++) n *= a < G.ndim ? (G.n[a] - ((colour >> a) & 1) + 1) >> 1 : G.n[a];
  return n;
}

__device__ __forceinline__ void mgv_smooth_one(const MgGeo &G, double *u, const double *__restrict__ f, int colour,
                                               long t) {
  const int ci = colour & 1, cj = (colour >> 1) & 1, ck = (colour >> 2) & 1;
  const unsigned hx = (unsigned)(G.n[0] - ci + 1) >> 1;
  const unsigned hy = G.ndim > 1 ? (unsigned)(G.n[1] - cj + 1) >> 1 : 1u;
  const unsigned hz = G.ndim > 2 ? (unsigned)(G.n[2] - ck + 1) >> 1 : 1u;
  if (t >= (long)hx * hy * hz) return;
  const unsigned tt = (unsigned)t, r = tt / hx;
  const int i = 2 * (int)(tt - r * hx) + ci;
  const unsigned kk = r / hy;
  const int j = G.ndim > 1 ? 2 * (int)(r - kk * hy) + cj : 0;
  const int k = G.ndim > 2 ? 2 * (int)kk + ck : 0;
  const long o = mg_off(G, i, j, k);
  double L[3], idg[3];
  mgv_L(G, u, o, i, j, k, L, idg);
#pragma unroll
  for (int q = 0; q < 3; q++) u[q * G.nt + o] -= (L[q] - f[q * G.nt + o]) * idg[q];
}

__global__ __launch_bounds__(NT) void k_mgv_smooth(const MgGeo G, double *u, const double *__restrict__ f,
                                                   int colour) {
  mgv_smooth_one(G, u, f, colour, (long)blockIdx.x * NT + threadIdx.x);
}

// Two consecutive colours in one launch: (i even, j, k parities of `pair`)
// then (i odd, same j, k parities).  Within such a pair a cell depends only
// on its x-neighbours in the same row (the other rows it reads have other
// j or k parities), so a workgroup owns whole rows (rpw of them) and
// separates the halves by a barrier.  Same order and arithmetic as two
// single-colour launches.
__global__ __launch_bounds__(NT) void k_mgv_smooth2(const MgGeo G, double *u, const double *__restrict__ f,
                                                    int pair, int rpw) {
  const int cj = pair & 1, ck = (pair >> 1) & 1;
  const unsigned hy = G.ndim > 1 ? (unsigned)(G.n[1] - cj + 1) >> 1 : 1u;
  const unsigned hz = G.ndim > 2 ? (unsigned)(G.n[2] - ck + 1) >> 1 : 1u;
  const unsigned rows = hy * hz, row0 = blockIdx.x * (unsigned)rpw;
  for (int ci = 0; ci < 2; ci++) {
    const unsigned hx = (unsigned)(G.n[0] - ci + 1) >> 1;
    for (unsigned idx = threadIdx.x; idx < (unsigned)rpw * hx; idx += NT) {
      const unsigned rr = idx / hx, row = row0 + rr;
      if (row >= rows) break;
      const int i = 2 * (int)(idx - rr * hx) + ci;
      const unsigned kk = row / hy;
      const int j = G.ndim > 1 ? 2 * (int)(row - kk * hy) + cj : 0;
      const int k = G.ndim > 2 ? 2 * (int)kk + ck : 0;
      const long o = mg_off(G, i, j, k);
      double L[3], idg[3];
      mgv_L(G, u, o, i, j, k, L, idg);
#pragma unroll
      for (int q = 0; q < 3; q++) u[q * G.nt + o] -= (L[q] - f[q * G.nt + o]) * idg[q];
    }
    __syncthreads();
  }
}

// Coarsest level: all sweeps in one workgroup, colours separated by
// barriers; with lds != 0 on copies of X and f in dynamic LDS.
__global__ __launch_bounds__(NT) void k_mgv_coarse(const MgGeo G, double *u, const double *__restrict__ f,
                                                   int sweeps, int lds) {
  extern __shared__ double sm[];
  double *uu = u;
  const double *ff = f;
  const long n3 = 3 * G.nt;
  if (lds) {
    for (long e = threadIdx.x; e < n3; e += NT) {
      sm[e] = u[e];
      sm[n3 + e] = f[e];
    }
    __syncthreads();
    uu = sm;
    ff = sm + n3;
  }
  const int ncol = 1 << G.ndim;
  for (int s = 0; s < sweeps; s++)
    for (int c = 0; c < ncol; c++) {
      const long nc = mgv_colour_cells(G, c);
      for (long t = threadIdx.x; t < nc; t += NT) mgv_smooth_one(G, uu, ff, c, t);
      __syncthreads();
    }
  if (lds)
    for (long e = threadIdx.x; e < n3; e += NT) u[e] = uu[e];
}

// Line relaxation of the vector equations, the line from cell c along
// axis ax by one wavefront (as mg_line_step): the components one after the
// other, each a Newton step of its own equation with its exact Jacobian
// with respect to that component on the line -- the couplings of the
// component's flux-form Laplacian, times 4/3 along the component's own
// axis through the grad-div term; on the diagonal the point smoother's
// plus, across each non-periodic boundary face, the weight toward the
// mirror ghost times the component's sign there -- and everything else
// (the other components included) at its current value.
__device__ __forceinline__ void mgv_line_step(const MgGeo &G, double *u, const double *__restrict__ f, int ax,
                                              const int c[3], bool live, double *sm, int ln, int nl) {
  const int n = G.n[ax];
  for (int q = 0; q < 3; q++) {
    const double kap = ax == q && q < G.ndim ? 4.0 / 3.0 : 1.0;
    for (int m = ln; live && m < n; m += nl) {
      const int cc[3] = {ax == 0 ? m : c[0], ax == 1 ? m : c[1], ax == 2 ? m : c[2]};
      const long o = mg_off(G, cc[0], cc[1], cc[2]);
      double L[3], idg[3], wm, wp;
      mgv_L(G, u, o, cc[0], cc[1], cc[2], L, idg);
      double dg = 1.0 / idg[q];
#pragma unroll
      for (int b = 0; b < 3; b++) {
        if (b >= G.ndim || G.bc[b][0] == GMUNU_MG_PERIODIC || (cc[b] > 0 && cc[b] < G.n[b] - 1)) continue;
        const double kb = b == q ? 4.0 / 3.0 : 1.0;
        mg_w(G, cc[0] + G.g[0], cc[1] + G.g[1], b, wm, wp);
        if (cc[b] == 0) dg += (G.vodd[b][0] >> q) & 1 ? -kb * wm : kb * wm;
        if (cc[b] == G.n[b] - 1) dg += (G.vodd[b][1] >> q) & 1 ? -kb * wp : kb * wp;
      }
      mg_w(G, cc[0] + G.g[0], cc[1] + G.g[1], ax, wm, wp);
      wm = m == 0 ? 0.0 : kap * wm;
      wp = m == n - 1 ? 0.0 : kap * wp;
      sm[m] = wm;
      sm[n + m] = dg;
      sm[2 * n + m] = wp;
      sm[3 * n + m] = f[q * G.nt + o] - L[q];
    }
    __syncthreads();
    const double *R = sm + mg_pcr(sm, n, ln, nl) * 4 * n;
    for (int m = ln; live && m < n; m += nl) {
      const int cc[3] = {ax == 0 ? m : c[0], ax == 1 ? m : c[1], ax == 2 ? m : c[2]};
      u[q * G.nt + mg_off(G, cc[0], cc[1], cc[2])] += R[3 * n + m] / R[n + m];
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kLineThreads) void k_mgv_line(const MgGeo G, double *u, const double *__restrict__ f,
                                                           int ax, int colour) {
  extern __shared__ double sm[];
  int c[3];
  if (!mg_line(G, ax, colour, blockIdx.x, c)) return;
  mgv_line_step(G, u, f, ax, c, true, sm, threadIdx.x, blockDim.x);
}

// Coarsest level of the vector equations (as k_mg_line_coarse): X and f
// staged in LDS, then 8 nmax doubles per wavefront.
__global__ __launch_bounds__(kCoarseLineThreads) void k_mgv_line_coarse(const MgGeo G, double *u,
                                                                        const double *__restrict__ f, int sweeps,
                                                                        int nmax) {
  extern __shared__ double sm[];
  const long n3 = 3 * G.nt;
  for (long e = threadIdx.x; e < n3; e += kCoarseLineThreads) {
    sm[e] = u[e];
    sm[n3 + e] = f[e];
  }
  __syncthreads();
  double *lines = sm + 2 * n3;
  const int w = threadIdx.x / kLineWave, ln = threadIdx.x % kLineWave, nw = kCoarseLineThreads / kLineWave;
  for (int s = 0; s < sweeps; s++)
    for (int ax = 0; ax < G.ndim; ax++) {
      if (G.bc[ax][0] == GMUNU_MG_PERIODIC) continue;
      for (int col = 0; col < 1 << (G.ndim - 1); col++) {
        const long nl = mg_line_count(G, ax, col);
        for (long t0 = 0; t0 < nl; t0 += nw) {
          int c[3] = {0, 0, 0};
          const bool live = mg_line(G, ax, col, t0 + w, c);
          mgv_line_step(G, sm, sm + n3, ax, c, live, lines + (long)w * 8 * nmax, ln, kLineWave);
        }
      }
    }
  for (long e = threadIdx.x; e < n3; e += kCoarseLineThreads) u[e] = sm[e];
}

__global__ __launch_bounds__(NT) void k_mgv_apply(const MgGeo G, const double *__restrict__ u,
                                                  double *__restrict__ out) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= mg_cells(G)) return;
  int i, j, k;
  mg_cell(G, t, i, j, k);
  const long o = mg_off(G, i, j, k);
  double L[3], idg[3];
  mgv_L(G, u, o, i, j, k, L, idg);
#pragma unroll
  for (int q = 0; q < 3; q++) out[q * G.nt + o] = L[q];
}

__global__ __launch_bounds__(NT) void k_mgv_norm(const MgGeo G, const double *__restrict__ u,
                                                 const double *__restrict__ f, double *part) {
  double m = 0.0;
  for (long t = (long)blockIdx.x * NT + threadIdx.x; t < mg_cells(G); t += (long)gridDim.x * NT) {
    int i, j, k;
    mg_cell(G, t, i, j, k);
    const long o = mg_off(G, i, j, k);
    double L[3], idg[3];
    mgv_L(G, u, o, i, j, k, L, idg);
#pragma unroll
    for (int q = 0; q < 3; q++) m = mg_absmax(m, f[q * G.nt + o] - L[q]);
  }
  m = block_max(m);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// Coarse problem of a fine level for the vector equation: the children's
// residuals and values, volume-weighted means into the coarse r and u.
__global__ __launch_bounds__(NT) void k_mgv_restrict_res(const MgGeo F, const MgGeo C, const double *__restrict__ u,
                                                         const double *__restrict__ f, double *__restrict__ uc,
                                                         double *__restrict__ rc) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= mg_cells(C)) return;
  int i, j, k;
  mg_cell(C, t, i, j, k);
  double su[3] = {0.0, 0.0, 0.0}, sr[3] = {0.0, 0.0, 0.0}, w = 0.0;
  const int nch = 1 << F.ndim;
  for (int ch = 0; ch < nch; ch++) {
    const int fi = 2 * i + (ch & 1);
    const int fj = F.ndim > 1 ? 2 * j + ((ch >> 1) & 1) : j;
    const int fk = F.ndim > 2 ? 2 * k + ((ch >> 2) & 1) : k;
    const long o = mg_off(F, fi, fj, fk);
    const double v = F.vol0[fi + F.g[0]] * F.vol1[fj + F.g[1]];
    double L[3], idg[3];
    mgv_L(F, u, o, fi, fj, fk, L, idg);
#pragma unroll
    for (int q = 0; q < 3; q++) {
      su[q] += v * u[q * F.nt + o];
      sr[q] += v * (f[q * F.nt + o] - L[q]);
    }
    w += v;
  }
  const long oc = mg_off(C, i, j, k);
#pragma unroll
  for (int q = 0; q < 3; q++) {
    uc[q * C.nt + oc] = su[q] / w;
    rc[q * C.nt + oc] = sr[q] / w;
  }
}

// f_c = L_c(u_c) + r_c and uo_c = u_c.
__global__ __launch_bounds__(NT) void k_mgv_fas_rhs(const MgGeo C, const double *__restrict__ u,
                                                    const double *__restrict__ r, double *__restrict__ f,
                                                    double *__restrict__ uo) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= mg_cells(C)) return;
  int i, j, k;
  mg_cell(C, t, i, j, k);
  const long o = mg_off(C, i, j, k);
  double L[3], idg[3];
  mgv_L(C, u, o, i, j, k, L, idg);
#pragma unroll
  for (int q = 0; q < 3; q++) {
    f[q * C.nt + o] = L[q] + r[q * C.nt + o];
    uo[q * C.nt + o] = u[q * C.nt + o];
  }
}

// A~^ij = grad^i X^j + grad^j X^i - (2/3) delta^ij div X in orthonormal
// components (centred, boundary rule across the boundary; the connection
// terms of cylindrical and spherical coordinates, d/dphi = 0) as six
// components (xx yy zz xy xz yz in the order of the axes), and A~_ij A~^ij.
__global__ __launch_bounds__(NT) void k_mgv_aij(const MgGeo G, const double *__restrict__ X, double *__restrict__ A6,
                                                double *__restrict__ A2) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= mg_cells(G)) return;
  int i, j, k;
  mg_cell(G, t, i, j, k);
  const long o = mg_off(G, i, j, k);
  const VStep s = mgv_steps(G, i, j, k);
  double g[3][3];  // g[a][b] = grad_a X_b in orthonormal components
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) {
      const double *xb = X + b * G.nt;
      g[a][b] = a < G.ndim ? (mgv_sgn(s.neg, 6 * b + 3 + a, xb[o + s.dp[a]]) -
                              mgv_sgn(s.neg, 6 * b + a, xb[o + s.dm[a]])) /
                                 (2.0 * G.h[a])
                           : 0.0;
    }
  // connection terms (d/dphi = 0)
  const double x0v = X[o], x1v = X[G.nt + o], x2v = X[2 * G.nt + o];
  if (G.coord == GMUNU_CYL) {
    const double R = G.x0[0] + (i + 0.5) * G.h[0];
    g[2][0] = -x2v / R;
    g[2][1] = 0.0;
    g[2][2] = x0v / R;
  } else if (G.coord == GMUNU_SPH) {
    const double r = G.x0[0] + (i + 0.5) * G.h[0], th = G.x0[1] + (j + 0.5) * G.h[1];
    const double ct = cos(th) / sin(th);
    g[1][0] = (g[1][0] - x1v) / r;
    g[1][1] = (g[1][1] + x0v) / r;
    g[1][2] = g[1][2] / r;
    g[2][0] = -x2v / r;
    g[2][1] = -ct * x2v / r;
    g[2][2] = (x0v + ct * x1v) / r;
  }
  const double dv = g[0][0] + g[1][1] + g[2][2];
  double A[3][3], a2 = 0.0;
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) {
      A[a][b] = g[a][b] + g[b][a] - (a == b ? 2.0 / 3.0 * dv : 0.0);
      a2 += A[a][b] * A[a][b];
    }
  if (A6) {  // null: A2 alone (the residual check)
    A6[o] = A[0][0];
    A6[G.nt + o] = A[1][1];
    A6[2 * G.nt + o] = A[2][2];
    A6[3 * G.nt + o] = A[0][1];
    A6[4 * G.nt + o] = A[0][2];
    A6[5 * G.nt + o] = A[1][2];
  }
  A2[o] = a2;
}

// Source of the shift equation: 16 pi w S_i + 2 A~^ij grad_j w, w = alpha
// psi^-6 with its ghost entries as stored (centred orthonormal gradient).
__global__ __launch_bounds__(NT) void k_mgv_beta_rhs(const MgGeo G, const double *__restrict__ w,
                                                     const double *__restrict__ S, const double *__restrict__ A6,
                                                     double *__restrict__ out) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= mg_cells(G)) return;
  int i, j, k;
  mg_cell(G, t, i, j, k);
  const long o = mg_off(G, i, j, k);
  const long St[3] = {1, G.s1, G.s2};
  double gw[3];
#pragma unroll
  for (int a = 0; a < 3; a++) gw[a] = a < G.ndim ? (w[o + St[a]] - w[o - St[a]]) / (2.0 * G.h[a]) : 0.0;
  if (G.coord == GMUNU_SPH) gw[1] /= G.x0[0] + (i + 0.5) * G.h[0];  // orthonormal theta component
  const long nt = G.nt;
  const double axx = A6[o], ayy = A6[nt + o], azz = A6[2 * nt + o];
  const double axy = A6[3 * nt + o], axz = A6[4 * nt + o], ayz = A6[5 * nt + o];
  const double wc = 16.0 * M_PI * w[o];
  out[o] = wc * S[o] + 2.0 * (axx * gw[0] + axy * gw[1] + axz * gw[2]);
  out[nt + o] = wc * S[nt + o] + 2.0 * (axy * gw[0] + ayy * gw[1] + ayz * gw[2]);
  out[2 * nt + o] = wc * S[2 * nt + o] + 2.0 * (axz * gw[0] + ayz * gw[1] + azz * gw[2]);
}

// ------------------------------------------------- bridge to the GRMHD state

// Layout of a GRMHD state array (include/gmunu.h: [var][k][j][i], ng ghost
// layers on active axes) on the multigrid grid's interior.
struct Hydro {
  int ng[3];
  long T0, T1, nv;  // cells per row, per plane, per variable
  double gam;
};

__device__ __forceinline__ long hy_off(const Hydro &H, int i, int j, int k) {
  return (long)(k + H.ng[2]) * H.T1 + (long)(j + H.ng[1]) * H.T0 + (i + H.ng[0]);
}

// q_B of every entry of the multigrid vector layout (interior from q, the
// ghost layer from psi^6 times the primitive field, which the GRMHD ghost
// fill maintains).
__global__ __launch_bounds__(NT) void k_br_gather_qb(const MgGeo G, const Hydro H, const double *__restrict__ q,
                                                     const double *__restrict__ prim, const double *__restrict__ met,
                                                     double *__restrict__ qb) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= G.nt) return;
  const int I = (int)(t % G.s1), J = (int)((t / G.s1) % (G.s2 / G.s1)), K = (int)(t / G.s2);
  const int i = I - G.g[0], j = J - G.g[1], k = K - G.g[2];
  const long o = hy_off(H, i, j, k);
  const bool inside = i >= 0 && i < G.n[0] && j >= 0 && j < G.n[1] && k >= 0 && k < G.n[2];
  const double psi = met[o], psi2 = psi * psi, psi6 = psi2 * psi2 * psi2;
#pragma unroll
  for (int c = 0; c < 3; c++) qb[c * G.nt + t] = inside ? q[(5 + c) * H.nv + o] : psi6 * prim[(5 + c) * H.nv + o];
}

__global__ __launch_bounds__(NT) void k_br_scatter_qb(const MgGeo G, const Hydro H, const double *__restrict__ qb,
                                                      double *__restrict__ q) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= mg_cells(G)) return;
  int i, j, k;
  mg_cell(G, t, i, j, k);
  const long o = hy_off(H, i, j, k), m = mg_off(G, i, j, k);
#pragma unroll
  for (int c = 0; c < 3; c++) q[(5 + c) * H.nv + o] = qb[c * G.nt + m];
}

// Coefficients of the scalar CFC equations (section 2.6) on the interior:
// which 0 (conformal factor): a = -2 pi U~ with U~ = q_tau + q_D, and with
// A2 = A~_ij A~^ij given, a2 = -A2 / 8 (the term in psi^-7);
// which 1 (lapse): a = 2 pi (U~ + 2 S~) / psi^2 (+ (7/8) A2 psi^-8) with
// S~ = psi^6 (rho h W^2 v^2 + 3 p) from the primitives (fluid part) and psi
// from the metric.  u: the initial guess u = psi - 1, or alpha psi - 1, from
// the metric.
__global__ __launch_bounds__(NT) void k_br_cfc_coef(const MgGeo G, const Hydro H, const double *__restrict__ q,
                                                    const double *__restrict__ prim, const double *__restrict__ met,
                                                    int which, const double *__restrict__ A2, double *__restrict__ a,
                                                    double *__restrict__ a2, double *__restrict__ u) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= mg_cells(G)) return;
  int i, j, k;
  mg_cell(G, t, i, j, k);
  const long o = hy_off(H, i, j, k), m = mg_off(G, i, j, k);
  const double Ut = q[4 * H.nv + o] + q[o];
  const double psi = met[o];
  if (which == 0) {
    a[m] = -2.0 * M_PI * Ut;
    if (A2) a2[m] = -A2[m] / 8.0;
    u[m] = psi - 1.0;
    return;
  }
  const double psi2 = psi * psi, psi4 = psi2 * psi2;
  // gamma_ij = psi^4 gamma^_ij with the reference metric of the grid
  const int I = i + G.g[0], J = j + G.g[1];
  double g1 = 1.0, g2 = 1.0;
  if (G.coord == GMUNU_CYL) g2 = 1.0 / G.g2[I];
  if (G.coord == GMUNU_SPH) {
    g1 = 1.0 / G.g1[I];
    g2 = g1 / G.s2t[J];
  }
  const double u1 = prim[H.nv + o], u2 = prim[2 * H.nv + o], u3 = prim[3 * H.nv + o];
  const double w2v2 = psi4 * (u1 * u1 + g1 * u2 * u2 + g2 * u3 * u3);
  const double rho = prim[o], p = prim[4 * H.nv + o];
  const double rhoh = rho + H.gam / (H.gam - 1.0) * p;
  const double St = psi4 * psi2 * (rhoh * w2v2 + 3.0 * p);
  double av = 2.0 * M_PI * (Ut + 2.0 * St) / psi2;
  if (A2) av += 7.0 / 8.0 * A2[m] / (psi4 * psi4);
  a[m] = av;
  u[m] = met[H.nv + o] * psi - 1.0;
}

// Scale factors of the reference metric at signed cell-centre coordinates
// (x0, x1): orthonormal component = h_c times the contravariant one, and
// the covariant one divided by h_c.
__device__ __forceinline__ double mg_hscale(int coord, int c, double x0, double x1) {
  if (coord == GMUNU_CYL) return c == 2 ? x0 : 1.0;
  if (coord == GMUNU_SPH) return c == 0 ? 1.0 : c == 1 ? x0 : x0 * sin(x1);
  return 1.0;
}

// Momentum source of the vector equations in orthonormal components:
// S[c] = q_{S_c} / h_c (q_S = psi^6 S_c covariant, the rescaled S~_c of
// section 2.6) and fX = 8 pi S, on the interior.
__global__ __launch_bounds__(NT) void k_bx_src(const MgGeo G, const Hydro H, const double *__restrict__ q,
                                               double *__restrict__ S, double *__restrict__ fX) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= mg_cells(G)) return;
  int i, j, k;
  mg_cell(G, t, i, j, k);
  const long o = hy_off(H, i, j, k), m = mg_off(G, i, j, k);
  const double x0 = G.x0[0] + (i + 0.5) * G.h[0], x1 = G.x0[1] + (j + 0.5) * G.h[1];
#pragma unroll
  for (int c = 0; c < 3; c++) {
    const double v = q[(1 + c) * H.nv + o] / mg_hscale(G.coord, c, x0, x1);
    S[c * G.nt + m] = v;
    fX[c * G.nt + m] = 8.0 * M_PI * v;
  }
}

// w = alpha psi^-6 on every entry of the multigrid layout (its ghost layer
// from the metric's first ghost layer).
__global__ __launch_bounds__(NT) void k_bx_w(const MgGeo G, const Hydro H, const double *__restrict__ met,
                                             double *__restrict__ w) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= G.nt) return;
  const int I = (int)(t % G.s1), J = (int)((t / G.s1) % (G.s2 / G.s1)), K = (int)(t / G.s2);
  const long o = hy_off(H, I - G.g[0], J - G.g[1], K - G.g[2]);
  const double psi = met[o], psi2 = psi * psi;
  w[t] = met[H.nv + o] / (psi2 * psi2 * psi2);
}

// The metric's shift on the interior (orthonormal components) as the
// initial guess of its solve.
__global__ __launch_bounds__(NT) void k_bx_beta_in(const MgGeo G, const Hydro H, const double *__restrict__ met,
                                                   double *__restrict__ beta) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= mg_cells(G)) return;
  int i, j, k;
  mg_cell(G, t, i, j, k);
  const long o = hy_off(H, i, j, k), m = mg_off(G, i, j, k);
  const double x0 = G.x0[0] + (i + 0.5) * G.h[0], x1 = G.x0[1] + (j + 0.5) * G.h[1];
#pragma unroll
  for (int c = 0; c < 3; c++) beta[c * G.nt + m] = met[(2 + c) * H.nv + o] * mg_hscale(G.coord, c, x0, x1);
}

// Metric of every GRMHD cell (ng ghost layers included) from the solution u
// of level G, ghost layers extended by the multigrid boundary rule applied
// per layer (mirror about the face times -1, +1 or r_in / r_ghost; periodic
// wrap): which 0 writes psi = 1 + u, which 1 alpha = (1 + u) / psi, which
// 2..4 the shift component c = which - 2 from its orthonormal value u
// (mirrored with the component's parity, then divided by h_c at the
// cell's signed coordinates).
__global__ __launch_bounds__(NT) void k_br_store(const MgGeo G, const Hydro H, const double *__restrict__ u,
                                                 double xmin0, int which, double *__restrict__ met) {
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  if (t >= H.nv) return;
  int c[3] = {(int)(t % H.T0) - H.ng[0], (int)((t / H.T0) % (H.T1 / H.T0)) - H.ng[1], (int)(t / H.T1) - H.ng[2]};
  const double xc0 = G.x0[0] + (c[0] + 0.5) * G.h[0], xc1 = G.x0[1] + (c[1] + 0.5) * G.h[1];
  double fac = 1.0;
  // axes from the last to the first: an edge or corner ghost takes the
  // factor of each axis at the other coordinates not yet mapped inside
#pragma unroll
  for (int a = 2; a >= 0; a--) {
    if (a >= G.ndim) continue;
    const int n = G.n[a];
    if (c[a] >= 0 && c[a] < n) continue;
    const int side = c[a] < 0 ? 0 : 1;
    const int kind = G.bc[a][side];
    if (kind == GMUNU_MG_PERIODIC) {
      c[a] = side == 0 ? c[a] + n : c[a] - n;
      continue;
    }
    const int in = side == 0 ? -1 - c[a] : 2 * n - 1 - c[a];
    if (which >= 2) {
      if ((G.vodd[a][side] >> (which - 2)) & 1) fac = -fac;
    } else if (kind == GMUNU_MG_DIRICHLET) {
      fac = -fac;
    }
    if (which < 2 && kind == GMUNU_MG_ROBIN) {
      if (G.coord == GMUNU_SPH) {
        fac *= (xmin0 + (in + 0.5) * G.h[0]) / (xmin0 + (c[a] + 0.5) * G.h[0]);
      } else {
        const int nb = G.coord == GMUNU_CYL ? 2 : 3;
        double ri = 0.0, rg = 0.0;
#pragma unroll
        for (int b = 0; b < 3; b++) {
          if (b >= G.ndim || b >= nb) continue;
          const double xg = G.x0[b] + (c[b] + 0.5) * G.h[b];
          const double xi = b == a ? G.x0[b] + (in + 0.5) * G.h[b] : xg;
          ri += xi * xi;
          rg += xg * xg;
        }
        fac *= sqrt(ri) / sqrt(rg);
      }
    }
    c[a] = in;
  }
  const double v = fac * u[mg_off(G, c[0], c[1], c[2])];
  if (which == 0)
    met[t] = 1.0 + v;
  else if (which == 1)
    met[H.nv + t] = (1.0 + v) / met[t];
  else
    met[which * H.nv + t] = v / mg_hscale(G.coord, which - 2, xc0, xc1);
}

}  // namespace

struct gmunu_mg {
  gmunu_mg_desc d;
  int levels;
  MgGeo geo[kMaxLevels];
  double *tab;  // geometry tables of all levels (device)
  // per level: u, f, a, r, uo (the finest level's u, f, a are the caller's;
  // a[l] is NULL when the equation has no a)
  double *u[kMaxLevels], *f[kMaxLevels], *a[kMaxLevels], *r[kMaxLevels], *uo[kMaxLevels];
  double *aown[kMaxLevels];  // coarse-level storage of a
  double *a2[kMaxLevels], *a2own[kMaxLevels];  // the same for a2 (allocated when power2 != 0)
  // colour-split copies of the finest f, a, a2 for the red-black sweeps
  // (allocated by the first solve of a large enough level; fs == NULL: none)
  double *fs, *as, *a2s;
  const double *sf, *sa, *sa2;  // the split copies' sources in the cycles being run
  double *part;  // norm partials + result
  double *br;    // state bridge scratch (6 arrays of the finest level), allocated on first use
  // vector equations (Cartesian): per coarse level u, f, r, uo of three
  // components each, allocated on first use; xs: scratch of the xCFC
  // sequence (17 finest arrays), allocated on first use
  double *vu[kMaxLevels], *vf[kMaxLevels], *vr[kMaxLevels], *vuo[kMaxLevels];
  bool vready;
  double *xs;
  std::vector<double *> owned;
  // V-cycles are replayed from graphs captured on a private stream, each for
  // the finest arrays it was captured with (two per kind of equation)
  hipStream_t gs;
  hipEvent_t ev;
  struct Slot {
    hipGraphExec_t exec;
    bool vec;
    const double *u, *f, *a, *a2;
  } slot[4];
  int next_slot;
};

namespace {

// Axis a after L halvings: divisible, at least two cells, and an even count
// on a periodic axis (an odd count would give the cells on either side of
// the wrap the same colour, and a colour's cells would not be independent).
bool coarsens(const gmunu_mg_desc &d, int a, int L) {
  const int n = d.n[a] >> L;
  return d.n[a] % (1 << L) == 0 && n >= 2 && (d.bc[a][0] != GMUNU_MG_PERIODIC || n % 2 == 0);
}

int auto_levels(const gmunu_mg_desc &d) {
  int L = 1;
  for (;;) {
    bool ok = L < kMaxLevels;
    for (int a = 0; a < d.ndim && ok; a++) ok = coarsens(d, a, L);
    if (!ok) return L;
    L++;
  }
}

int validate(const gmunu_mg_desc &d, int levels) {
  if (d.ndim < 1 || d.ndim > 3 || d.coord < GMUNU_CART || d.coord > GMUNU_SPH) return GMUNU_EINVAL;
  if (levels < 1 || levels > kMaxLevels) return GMUNU_EINVAL;
  for (int a = 0; a < 3; a++) {
    if (a >= d.ndim) {
      if (d.n[a] != 1) return GMUNU_EINVAL;
      continue;
    }
    if (d.n[a] < 1 || !(d.dx[a] > 0.0) || !coarsens(d, a, levels - 1)) return GMUNU_EINVAL;
    for (int s = 0; s < 2; s++) {
      const int b = d.bc[a][s];
      if (b < GMUNU_MG_DIRICHLET || b > GMUNU_MG_ROBIN) return GMUNU_EINVAL;
      if (b == GMUNU_MG_ROBIN && ((d.coord == GMUNU_SPH && a != 0) || (d.coord == GMUNU_CYL && a == 2)))
        return GMUNU_EINVAL;
      if ((b == GMUNU_MG_PERIODIC) != (d.bc[a][1 - s] == GMUNU_MG_PERIODIC)) return GMUNU_EINVAL;
    }
  }
  if (d.coord != GMUNU_CART && d.xmin[0] < 0.0) return GMUNU_EINVAL;
  if (d.coord == GMUNU_SPH && d.ndim > 1 && (d.xmin[1] < 0.0 || d.xmin[1] + d.n[1] * d.dx[1] > M_PI + 1e-12))
    return GMUNU_EINVAL;
  if (d.power < -1 || d.power > 1 || d.pre < 0 || d.post < 0 || d.coarse < 1) return GMUNU_EINVAL;
  if (d.power2 < -8 || d.power2 > 8) return GMUNU_EINVAL;
  if (d.smoother != GMUNU_MG_POINT && d.smoother != GMUNU_MG_LINE) return GMUNU_EINVAL;
  for (int a = 0; a < d.ndim; a++)
    if (d.smoother == GMUNU_MG_LINE && d.bc[a][0] != GMUNU_MG_PERIODIC && d.n[a] > kMaxLine) return GMUNU_EINVAL;
  // cell numbers of a level fit 32-bit kernel arithmetic
  if ((double)(d.n[0] + 2) * (d.n[1] + 2) * (d.n[2] + 2) >= 2147483647.0) return GMUNU_EINVAL;
  return GMUNU_OK;
}

// Host tables of one level: 6 per axis-0 index, 5 per axis-1 index.
void level_tables(const gmunu_mg_desc &d, int s, std::vector<double> &tab, size_t off[11], MgGeo &G) {
  for (int a = 0; a < 3; a++) {
    G.g[a] = a < d.ndim ? 1 : 0;
    G.n[a] = a < d.ndim ? d.n[a] >> s : 1;
    G.h[a] = a < d.ndim ? d.dx[a] * (double)(1 << s) : d.dx[a];
  }
  const int t0 = G.n[0] + 2 * G.g[0], t1 = G.n[1] + 2 * G.g[1], t2 = G.n[2] + 2 * G.g[2];
  G.s1 = t0;
  G.s2 = (long)t0 * t1;
  G.nt = G.s2 * t2;
  G.ndim = d.ndim;
  G.coord = d.coord;
  G.ih2_2 = 1.0 / (G.h[2] * G.h[2]);
  const bool cyl = d.coord == GMUNU_CYL, sph = d.coord == GMUNU_SPH;
  std::vector<double> a0m(t0), a0p(t0), g1(t0), g2(t0), vol0(t0), sg0(t0);
  const double h0 = G.h[0], h02 = h0 * h0;
  for (int I = 0; I < t0; I++) {
    const double x = d.xmin[0] + (I - G.g[0] + 0.5) * h0;
    const double fm = d.xmin[0] + (I - G.g[0]) * h0, fp = fm + h0;
    a0m[I] = a0p[I] = 1.0 / h02;
    g1[I] = g2[I] = vol0[I] = sg0[I] = 1.0;
    if (cyl) {
      a0m[I] = fm / (x * h02);
      a0p[I] = fp / (x * h02);
      g2[I] = 1.0 / (x * x);
      vol0[I] = sg0[I] = x;
    } else if (sph) {
      a0m[I] = fm * fm / (x * x * h02);
      a0p[I] = fp * fp / (x * x * h02);
      g1[I] = g2[I] = 1.0 / (x * x);
      vol0[I] = x * x + h02 / 12.0;
      sg0[I] = x * x;
    }
  }
  std::vector<double> a1m(t1), a1p(t1), s2t(t1), vol1(t1), sg1(t1);
  const double h1 = G.h[1], h12 = h1 * h1;
  for (int J = 0; J < t1; J++) {
    const double y = d.xmin[1] + (J - G.g[1] + 0.5) * h1;
    const double fm = d.xmin[1] + (J - G.g[1]) * h1, fp = fm + h1;
    a1m[J] = a1p[J] = 1.0 / h12;
    s2t[J] = vol1[J] = sg1[J] = 1.0;
    if (sph) {
      const double sy = std::sin(y);
      a1m[J] = std::sin(fm) / (sy * h12);
      a1p[J] = std::sin(fp) / (sy * h12);
      s2t[J] = 1.0 / (sy * sy);
      vol1[J] = d.ndim > 1 ? sy : 1.0;
      sg1[J] = sy;
    }
  }
  const std::vector<double> *all[11] = {&a0m, &a0p, &g1, &g2, &vol0, &sg0, &a1m, &a1p, &s2t, &vol1, &sg1};
  for (int q = 0; q < 11; q++) {
    while (tab.size() % 32) tab.push_back(0.0);
    off[q] = tab.size();
    tab.insert(tab.end(), all[q]->begin(), all[q]->end());
  }
  for (int a = 0; a < 3; a++)
    for (int sd = 0; sd < 2; sd++) G.bc[a][sd] = d.bc[a][sd];
  // Robin ghost factors: centre of the boundary cell / centre of its ghost
  const double xin_lo = d.xmin[0] + 0.5 * h0, xg_lo = d.xmin[0] - 0.5 * h0;
  const double xin_hi = d.xmin[0] + (G.n[0] - 0.5) * h0, xg_hi = d.xmin[0] + (G.n[0] + 0.5) * h0;
  G.rob_lo = xin_lo / xg_lo;
  G.rob_hi = xin_hi / xg_hi;
  for (int a = 0; a < 3; a++) G.x0[a] = d.xmin[a];
  // per-component parity across each non-periodic face for the vector
  // equations: Dirichlet all odd; Neumann a symmetry face (normal component
  // odd), plus phi at the cylindrical and polar axes and every component at
  // the spherical centre (equatorially symmetric grids)
  for (int a = 0; a < 3; a++)
    for (int sd = 0; sd < 2; sd++) {
      const double fpos = sd == 0 ? d.xmin[a] : d.xmin[a] + d.n[a] * d.dx[a];
      unsigned odd = d.bc[a][sd] == GMUNU_MG_DIRICHLET ? 7u : 1u << a;
      if (d.bc[a][sd] == GMUNU_MG_NEUMANN) {
        if (d.coord == GMUNU_CYL && a == 0 && std::fabs(fpos) < 1e-12) odd |= 4u;
        if (d.coord == GMUNU_SPH && a == 0 && std::fabs(fpos) < 1e-12) odd = 7u;
        if (d.coord == GMUNU_SPH && a == 1 && (std::fabs(fpos) < 1e-12 || std::fabs(fpos - M_PI) < 1e-12)) odd |= 4u;
      }
      G.vodd[a][sd] = odd;
    }
  G.power = d.power;
  G.power2 = d.power2;
  G.offset = d.offset;
  G.line = 0;
  for (int a = 0; a < d.ndim; a++)
    if (d.smoother == GMUNU_MG_LINE && d.bc[a][0] != GMUNU_MG_PERIODIC) G.line = 1;
  double dsum = 0.0;
  for (int a = 0; a < 3; a++) {
    G.vih2[a] = a < d.ndim ? 1.0 / (G.h[a] * G.h[a]) : 0.0;
    dsum -= 2.0 * G.vih2[a];
  }
  const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
  for (int q = 0; q < 3; q++) {
    G.vmix[q] = pb[q] < d.ndim ? 1.0 / (4.0 * G.h[pa[q]] * G.h[pb[q]]) : 0.0;
    G.vidg[q] = 1.0 / (q < d.ndim ? dsum - (2.0 / 3.0) * G.vih2[q] : dsum);
  }
}

long ghost_count(const MgGeo &G) {
  long s = 0;
  for (int a = 0; a < G.ndim; a++) {
    const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
    s += 2L * G.n[b1] * G.n[b2];
  }
  return s;
}

long cells(const MgGeo &G) { return (long)G.n[0] * G.n[1] * G.n[2]; }

void ghosts(const MgGeo &G, double *u, hipStream_t st) {
  const long gc = ghost_count(G);
  if (gc) hipLaunchKernelGGL(k_mg_ghosts<1>, dim3(nblocks(gc)), dim3(NT), 0, st, G, u);
}

// Threads per line workgroup: a lane per cell up to kLineThreads.
int line_threads(int n) {
  const int t = (n + kLineWave - 1) / kLineWave * kLineWave;
  return t < kLineThreads ? t : kLineThreads;
}

// Line sweeps: per sweep every non-periodic axis, per axis its colours.
void line_sweeps(const MgGeo &G, double *u, const double *f, const double *a, const double *a2, int sweeps,
                 hipStream_t st) {
  for (int s = 0; s < sweeps; s++)
    for (int ax = 0; ax < G.ndim; ax++) {
      if (G.bc[ax][0] == GMUNU_MG_PERIODIC) continue;
      const size_t lds = 8 * (size_t)G.n[ax] * sizeof(double);
      for (int c = 0; c < 1 << (G.ndim - 1); c++)
        hipLaunchKernelGGL(k_mg_line, dim3(mg_line_count(G, ax, c)), dim3(line_threads(G.n[ax])), lds, st, G, u, f,
                           a, a2, ax, c);
    }
}

// Longest line of a level.
int line_nmax(const MgGeo &G) {
  int nmax = 1;
  for (int ax = 0; ax < G.ndim; ax++)
    if (G.bc[ax][0] != GMUNU_MG_PERIODIC) nmax = G.n[ax] > nmax ? G.n[ax] : nmax;
  return nmax;
}

// Dynamic LDS of a one-workgroup coarsest line solve staging `arrays`
// level arrays (0: does not fit).
size_t line_coarse_lds(const MgGeo &G, int arrays) {
  const size_t b =
      ((size_t)arrays * G.nt + (size_t)(kCoarseLineThreads / kLineWave) * 8 * line_nmax(G)) * sizeof(double);
  return b <= 64 * 1024 ? b : 0;
}

// Smoothing sweeps (boundary rule inline: no ghost fill between colours):
// line sweeps for the line smoother, else red-black.
void sweeps_raw(const MgGeo &G, double *u, const double *f, const double *a, const double *a2, int sweeps,
                hipStream_t st, const double *fs = nullptr, const double *as = nullptr, const double *a2s = nullptr) {
  if (G.line) {
    line_sweeps(G, u, f, a, a2, sweeps, st);
    return;
  }
  const long threads = (long)((G.n[0] + 1) / 2) * G.n[1] * G.n[2];
  for (int s = 0; s < sweeps; s++)
    for (int c = 0; c < 2; c++)
      hipLaunchKernelGGL(k_mg_smooth, dim3(nblocks(threads)), dim3(NT), 0, st, G, u, f, a, a2, c, fs, as, a2s);
}

// The same, then u's ghost entries from the boundary rule.
void smooth(const MgGeo &G, double *u, const double *f, const double *a, const double *a2, int sweeps,
            hipStream_t st) {
  sweeps_raw(G, u, f, a, a2, sweeps, st);
  ghosts(G, u, st);
}

// Coarse problem of level l: u_{l-1} = R u_l (kept in uo_{l-1}),
// f_{l-1} = L_{l-1}(R u_l) + R (f_l - L_l(u_l)).
void coarse_problem(gmunu_mg *m, int l, hipStream_t st) {
  const MgGeo &F = m->geo[l], &C = m->geo[l - 1];
  hipLaunchKernelGGL(k_mg_restrict_res, dim3(nblocks(cells(C))), dim3(NT), 0, st, F, C, m->u[l], m->f[l], m->a[l],
                     m->a2[l], m->u[l - 1], m->r[l - 1]);
  hipLaunchKernelGGL(k_mg_fas_rhs, dim3(nblocks(cells(C))), dim3(NT), 0, st, C, m->u[l - 1], m->a[l - 1],
                     m->a2[l - 1], m->r[l - 1], m->f[l - 1], m->uo[l - 1]);
}

// u_l += P(u_{l-1} - uo_{l-1})
void correct(gmunu_mg *m, int l, hipStream_t st) {
  const MgGeo &F = m->geo[l], &C = m->geo[l - 1];
  hipLaunchKernelGGL(k_mg_correct<1>, dim3(nblocks(cells(F))), dim3(NT), 0, st, C, F, m->u[l - 1], m->uo[l - 1],
                     m->u[l]);
}

// The coarsest level: one workgroup when it is small, else launches.
// Dynamic LDS a one-workgroup coarsest solve may stage (bytes).
constexpr long kCoarseLds = 64L * 1024;

void coarse_solve(gmunu_mg *m, hipStream_t st) {
  const MgGeo &G = m->geo[0];
  if (G.line) {
    const size_t lds = line_coarse_lds(G, 2 + (m->a[0] ? 1 : 0) + (m->a2[0] ? 1 : 0));
    if (cells(G) <= 64L * NT && lds)
      hipLaunchKernelGGL(k_mg_line_coarse, dim3(1), dim3(kCoarseLineThreads), lds, st, G, m->u[0], m->f[0],
                         m->a[0], m->a2[0], m->d.coarse, line_nmax(G));
    else
      line_sweeps(G, m->u[0], m->f[0], m->a[0], m->a2[0], m->d.coarse, st);
    return;
  }
  if (cells(G) <= 64L * NT) {
    const long bytes = (2 + (m->a[0] ? 1 : 0) + (m->a2[0] ? 1 : 0)) * G.nt * (long)sizeof(double);
    const int lds = bytes <= kCoarseLds;
    hipLaunchKernelGGL(k_mg_coarse, dim3(1), dim3(NT), lds ? bytes : 0, st, G, m->u[0], m->f[0], m->a[0], m->a2[0],
                       m->d.coarse, lds);
  } else
    sweeps_raw(G, m->u[0], m->f[0], m->a[0], m->a2[0], m->d.coarse, st);
}

void vcycle(gmunu_mg *m, int l, hipStream_t st) {
  if (l == 0) {
    coarse_solve(m, st);
    return;
  }
  const bool sp = l == m->levels - 1 && m->sf;  // finest level: colour-split f, a, a2
  sweeps_raw(m->geo[l], m->u[l], m->f[l], m->a[l], m->a2[l], m->d.pre, st, sp ? m->fs : nullptr,
             sp && m->sa ? m->as : nullptr, sp && m->sa2 ? m->a2s : nullptr);
  coarse_problem(m, l, st);
  vcycle(m, l - 1, st);
  correct(m, l, st);
  sweeps_raw(m->geo[l], m->u[l], m->f[l], m->a[l], m->a2[l], m->d.post, st, sp ? m->fs : nullptr,
             sp && m->sa ? m->as : nullptr, sp && m->sa2 ? m->a2s : nullptr);
}

void fmg(gmunu_mg *m, hipStream_t st) {
  const int top = m->levels - 1;
  for (int l = top; l > 0; l--) coarse_problem(m, l, st);
  coarse_solve(m, st);
  for (int l = 1; l <= top; l++) {
    correct(m, l, st);
    vcycle(m, l, st);
  }
}

// The finest-level residual norm's kernels: the result lands in
// part[kNormParts].
void norm_enqueue(gmunu_mg *m, hipStream_t st) {
  const int top = m->levels - 1;
  const MgGeo &G = m->geo[top];
  const long nb = nblocks(cells(G));
  const int np = (int)(nb < kNormParts ? nb : kNormParts);
  hipLaunchKernelGGL(k_mg_norm, dim3(np), dim3(NT), 0, st, G, m->u[top], m->f[top], m->a[top], m->a2[top],
                     m->part);
  hipLaunchKernelGGL(k_mg_norm_finish, dim3(1), dim3(NT), 0, st, m->part, np);
}

int norm(gmunu_mg *m, double *out, hipStream_t st) {
  norm_enqueue(m, st);
  if (hipMemcpyAsync(out, m->part + kNormParts, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return GMUNU_EHIP;
  return launch_status();
}

void split_copies(gmunu_mg *m, const double *f, const double *a, const double *a2, hipStream_t st);

// Bind the caller's finest-level arrays, restrict a and a2 to the coarse
// levels and refresh the colour-split copies.
void bind(gmunu_mg *m, double *u, const double *f, const double *a, const double *a2, hipStream_t st) {
  const int top = m->levels - 1;
  m->u[top] = u;
  m->f[top] = const_cast<double *>(f);
  m->a[top] = const_cast<double *>(a);
  m->a2[top] = const_cast<double *>(a2);
  for (int l = top; l > 0; l--) {
    m->a[l - 1] = a ? m->aown[l - 1] : nullptr;
    m->a2[l - 1] = a2 ? m->a2own[l - 1] : nullptr;
    if (a)
      hipLaunchKernelGGL(k_mg_restrict, dim3(nblocks(cells(m->geo[l - 1]))), dim3(NT), 0, st, m->geo[l],
                         m->geo[l - 1], m->a[l], m->a[l - 1]);
    if (a2)
      hipLaunchKernelGGL(k_mg_restrict, dim3(nblocks(cells(m->geo[l - 1]))), dim3(NT), 0, st, m->geo[l],
                         m->geo[l - 1], m->a2[l], m->a2[l - 1]);
  }
  split_copies(m, f, a, a2, st);
}

// Colour-split copies of the finest f, a, a2 for the red-black sweeps
// (large levels only: the copies cost one pass and save one per sweep).
void split_copies(gmunu_mg *m, const double *f, const double *a, const double *a2, hipStream_t st) {
  const MgGeo &G = m->geo[m->levels - 1];
  m->sf = m->sa = m->sa2 = nullptr;
  if (G.line || cells(G) < 32768 || G.n[0] < 16) return;
  const size_t bytes = (size_t)cells(G) * sizeof(double);
  auto get = [&](double *&p) {
    if (!p && hipMalloc(&p, bytes) == hipSuccess) m->owned.push_back(p);
    return p != nullptr;
  };
  if (!get(m->fs) || (a && !get(m->as)) || (a2 && !get(m->a2s))) return;
  const dim3 gr(nblocks(cells(G)));
  hipLaunchKernelGGL(k_mg_split, gr, dim3(NT), 0, st, G, f, m->fs);
  if (a) hipLaunchKernelGGL(k_mg_split, gr, dim3(NT), 0, st, G, a, m->as);
  if (a2) hipLaunchKernelGGL(k_mg_split, gr, dim3(NT), 0, st, G, a2, m->a2s);
  m->sf = f;
  m->sa = a;
  m->sa2 = a2;
}

// a2 is accepted only by a hierarchy whose equation has the second term.
bool a2_ok(const gmunu_mg *m, const double *a2) { return !a2 || (m->d.power2 != 0 && aligned8(a2)); }

bool ok_ptr(const void *p) { return p && aligned8(p); }

// The vector equations: Cartesian grids, or axisymmetric cylindrical and
// spherical ones (at most two active axes), faces Dirichlet, Neumann or
// periodic; a spherical grid reaching r = 0 must end at theta = pi/2.
bool vector_ok(const gmunu_mg *m) {
  const gmunu_mg_desc &d = m->d;
  for (int a = 0; a < 3; a++)
    for (int sd = 0; sd < 2; sd++)
      if (d.bc[a][sd] == GMUNU_MG_ROBIN) return false;
  if (d.coord != GMUNU_CART && d.ndim > 2) return false;
  if (d.coord == GMUNU_SPH && std::fabs(d.xmin[0]) < 1e-12 &&
      (d.ndim < 2 || std::fabs(d.xmin[1] + d.n[1] * d.dx[1] - M_PI / 2) > 1e-12))
    return false;
  return true;
}

// ----------------------------------------------- vector-equation cycles

long colour_cells(const MgGeo &G, int c) {
  long n = 1;
  for (int a = 0; a < 3; a++) n *= a < G.ndim ? (G.n[a] - ((c >> a) & 1) + 1) >> 1 : G.n[a];
  return n;
}

// Sweeps over the 2^ndim colours: two colours per launch (k_mgv_smooth2)
// when a row's half fits in 4 passes of a workgroup, else one per launch.
void vsweeps(const MgGeo &G, double *u, const double *f, int sweeps, hipStream_t st) {
  if (G.line) {
    for (int s = 0; s < sweeps; s++)
      for (int ax = 0; ax < G.ndim; ax++) {
        if (G.bc[ax][0] == GMUNU_MG_PERIODIC) continue;
        const size_t lds = 8 * (size_t)G.n[ax] * sizeof(double);
        for (int c = 0; c < 1 << (G.ndim - 1); c++)
          hipLaunchKernelGGL(k_mgv_line, dim3(mg_line_count(G, ax, c)), dim3(line_threads(G.n[ax])), lds, st, G, u,
                             f, ax, c);
      }
    return;
  }
  const int ncol = 1 << G.ndim;
  const long hx0 = (G.n[0] + 1) >> 1;
  const bool paired = hx0 <= 4L * NT;
  const int rpw = hx0 >= NT ? 1 : (int)(NT / hx0);
  for (int s = 0; s < sweeps; s++)
    for (int c = 0; c < ncol; c += paired ? 2 : 1) {
      if (paired) {
        const long rows = colour_cells(G, c) / ((G.n[0] + 1) >> 1);
        hipLaunchKernelGGL(k_mgv_smooth2, dim3((rows + rpw - 1) / rpw), dim3(NT), 0, st, G, u, f, c >> 1, rpw);
      } else {
        hipLaunchKernelGGL(k_mgv_smooth, dim3(nblocks(colour_cells(G, c))), dim3(NT), 0, st, G, u, f, c);
      }
    }
}

void vghosts(const MgGeo &G, double *u, hipStream_t st) {
  const long gc = ghost_count(G);
  if (gc) hipLaunchKernelGGL(k_mg_ghosts<3>, dim3(nblocks(gc)), dim3(NT), 0, st, G, u);
}

void vcoarse_problem(gmunu_mg *m, int l, hipStream_t st) {
  const MgGeo &F = m->geo[l], &C = m->geo[l - 1];
  hipLaunchKernelGGL(k_mgv_restrict_res, dim3(nblocks(cells(C))), dim3(NT), 0, st, F, C, m->vu[l], m->vf[l],
                     m->vu[l - 1], m->vr[l - 1]);
  hipLaunchKernelGGL(k_mgv_fas_rhs, dim3(nblocks(cells(C))), dim3(NT), 0, st, C, m->vu[l - 1], m->vr[l - 1],
                     m->vf[l - 1], m->vuo[l - 1]);
}

void vcorrect(gmunu_mg *m, int l, hipStream_t st) {
  const MgGeo &F = m->geo[l], &C = m->geo[l - 1];
  hipLaunchKernelGGL(k_mg_correct<3>, dim3(nblocks(cells(F))), dim3(NT), 0, st, C, F, m->vu[l - 1], m->vuo[l - 1],
                     m->vu[l]);
}

void vcoarse_solve(gmunu_mg *m, hipStream_t st) {
  const MgGeo &G = m->geo[0];
  if (G.line) {
    const size_t lds = line_coarse_lds(G, 6);
    if (cells(G) <= 64L * NT && lds)
      hipLaunchKernelGGL(k_mgv_line_coarse, dim3(1), dim3(kCoarseLineThreads), lds, st, G, m->vu[0], m->vf[0],
                         m->d.coarse, line_nmax(G));
    else
      vsweeps(G, m->vu[0], m->vf[0], m->d.coarse, st);
    return;
  }
  if (cells(G) <= 64L * NT) {
    const long bytes = 6 * G.nt * (long)sizeof(double);
    const int lds = bytes <= kCoarseLds;
    hipLaunchKernelGGL(k_mgv_coarse, dim3(1), dim3(NT), lds ? bytes : 0, st, G, m->vu[0], m->vf[0], m->d.coarse,
                       lds);
  } else
    vsweeps(G, m->vu[0], m->vf[0], m->d.coarse, st);
}

void vvcycle(gmunu_mg *m, int l, hipStream_t st) {
  if (l == 0) {
    vcoarse_solve(m, st);
    return;
  }
  vsweeps(m->geo[l], m->vu[l], m->vf[l], m->d.pre, st);
  vcoarse_problem(m, l, st);
  vvcycle(m, l - 1, st);
  vcorrect(m, l, st);
  vsweeps(m->geo[l], m->vu[l], m->vf[l], m->d.post, st);
}

void vfmg(gmunu_mg *m, hipStream_t st) {
  const int top = m->levels - 1;
  for (int l = top; l > 0; l--) vcoarse_problem(m, l, st);
  vcoarse_solve(m, st);
  for (int l = 1; l <= top; l++) {
    vcorrect(m, l, st);
    vvcycle(m, l, st);
  }
}

int vnorm(gmunu_mg *m, double *out, hipStream_t st) {
  const int top = m->levels - 1;
  const MgGeo &G = m->geo[top];
  const long nb = nblocks(cells(G));
  const int np = (int)(nb < kNormParts ? nb : kNormParts);
  hipLaunchKernelGGL(k_mgv_norm, dim3(np), dim3(NT), 0, st, G, m->vu[top], m->vf[top], m->part);
  hipLaunchKernelGGL(k_mg_norm_finish, dim3(1), dim3(NT), 0, st, m->part, np);
  if (hipMemcpyAsync(out, m->part + kNormParts, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return GMUNU_EHIP;
  return launch_status();
}

bool alloc_zeroed(gmunu_mg *m, size_t n, double **out) {
  double *p = nullptr;
  if (hipMalloc(&p, n * sizeof(double)) != hipSuccess) return false;
  if (hipMemset(p, 0, n * sizeof(double)) != hipSuccess) {
    (void)hipFree(p);
    return false;
  }
  m->owned.push_back(p);
  *out = p;
  return true;
}

bool vector_storage(gmunu_mg *m) {
  if (m->vready) return true;
  for (int l = 0; l < m->levels - 1; l++) {
    const size_t n = 3 * (size_t)m->geo[l].nt;
    if (!alloc_zeroed(m, n, &m->vu[l]) || !alloc_zeroed(m, n, &m->vf[l]) || !alloc_zeroed(m, n, &m->vr[l]) ||
        !alloc_zeroed(m, n, &m->vuo[l]))
      return false;
  }
  m->vready = true;
  return true;
}

// ------------------------------------------------- solve driver

// The private stream is ordered after the caller's work on entry and the
// caller's stream after the private one on exit.
int enter(gmunu_mg *m, hipStream_t cst) {
  if (!m->gs && hipStreamCreateWithFlags(&m->gs, hipStreamNonBlocking) != hipSuccess) return GMUNU_EHIP;
  if (!m->ev && hipEventCreateWithFlags(&m->ev, hipEventDisableTiming) != hipSuccess) return GMUNU_EHIP;
  if (hipEventRecord(m->ev, cst) != hipSuccess || hipStreamWaitEvent(m->gs, m->ev, 0) != hipSuccess)
    return GMUNU_EHIP;
  return GMUNU_OK;
}

int leave(gmunu_mg *m, hipStream_t cst) {
  if (hipEventRecord(m->ev, m->gs) != hipSuccess || hipStreamWaitEvent(cst, m->ev, 0) != hipSuccess)
    return GMUNU_EHIP;
  return launch_status();
}

// The graph of one V-cycle over the bound arrays: a cached one, else
// captured now into the least recently made slot (launches only: no
// memset, no host synchronisation inside).
hipGraphExec_t cycle_graph(gmunu_mg *m, bool vec, const double *u, const double *f, const double *a,
                           const double *a2) {
  for (auto &sl : m->slot)
    if (sl.exec && sl.vec == vec && sl.u == u && sl.f == f && sl.a == a && sl.a2 == a2) return sl.exec;
  auto &sl = m->slot[m->next_slot];
  m->next_slot = (m->next_slot + 1) % 4;
  if (sl.exec) {
    (void)hipGraphExecDestroy(sl.exec);
    sl.exec = nullptr;
  }
  hipStream_t st = m->gs;
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
  if (vec)
    vvcycle(m, m->levels - 1, st);
  else
    vcycle(m, m->levels - 1, st);
  if (hipStreamEndCapture(st, &g) != hipSuccess) return nullptr;
  const bool ok = hipGraphInstantiate(&sl.exec, g, nullptr, nullptr, 0) == hipSuccess;
  (void)hipGraphDestroy(g);
  if (!ok) {
    sl.exec = nullptr;
    return nullptr;
  }
  sl.vec = vec;
  sl.u = u;
  sl.f = f;
  sl.a = a;
  sl.a2 = a2;
  return sl.exec;
}

// Cycles until the norm is at most tol (arrays bound); the first one an FMG
// cycle when use_fmg.
int cycles(gmunu_mg *m, bool vec, hipGraphExec_t exec, double tol, int max_cycles, int use_fmg, double *res_host,
           int *cycles_out) {
  hipStream_t st = m->gs;
  double r;
  int rc = vec ? vnorm(m, &r, st) : norm(m, &r, st);
  if (rc) return rc;
  if (res_host) res_host[0] = r;
  int c = 0;
  while (c < max_cycles && r > tol) {
    if (c == 0 && use_fmg) {
      if (vec)
        vfmg(m, st);
      else
        fmg(m, st);
    } else if (hipGraphLaunch(exec, st) != hipSuccess) {
      return GMUNU_EHIP;
    }
    c++;
    rc = vec ? vnorm(m, &r, st) : norm(m, &r, st);
    if (rc) return rc;
    if (res_host) res_host[c] = r;
  }
  if (cycles_out) *cycles_out = c;
  return GMUNU_OK;
}

}  // namespace

// --------------------------------------------------------------------- API

extern "C" {

int gmunu_mg_create(const gmunu_mg_desc *desc, gmunu_mg **out) {
  if (!desc || !out) return GMUNU_ENULL;
  const int levels = desc->levels > 0 ? desc->levels : auto_levels(*desc);
  int rc = validate(*desc, levels);
  if (rc) return rc;
  gmunu_mg *m = new (std::nothrow) gmunu_mg();
  if (!m) return GMUNU_ENOMEM;
  m->d = *desc;
  m->levels = levels;
  std::vector<double> tab;
  size_t off[kMaxLevels][11];
  for (int l = 0; l < levels; l++) level_tables(*desc, levels - 1 - l, tab, off[l], m->geo[l]);
  auto alloc = [&](size_t n) -> double * {
    double *p = nullptr;
    if (hipMalloc(&p, n * sizeof(double)) != hipSuccess) return nullptr;
    m->owned.push_back(p);
    return p;
  };
  m->br = nullptr;
  m->xs = nullptr;
  m->fs = m->as = m->a2s = nullptr;
  m->sf = m->sa = m->sa2 = nullptr;
  m->vready = false;
  m->gs = nullptr;
  m->ev = nullptr;
  for (auto &sl : m->slot) sl = gmunu_mg::Slot{nullptr, false, nullptr, nullptr, nullptr, nullptr};
  m->next_slot = 0;
  bool ok = (m->tab = alloc(tab.size())) != nullptr && (m->part = alloc(kNormParts + 1 + kGateSlots)) != nullptr;
  // coarse levels: u, f, a, r (restricted residual) and uo (restricted u);
  // the finest level only uo (the cleaning's divergence when the caller
  // passes none)
  for (int l = 0; l < levels && ok; l++) {
    const size_t nt = (size_t)m->geo[l].nt;
    ok = (m->uo[l] = alloc(nt)) != nullptr;
    m->r[l] = nullptr;
    m->a2own[l] = nullptr;
    if (ok && l < levels - 1)
      ok = (m->r[l] = alloc(nt)) && (m->u[l] = alloc(nt)) && (m->f[l] = alloc(nt)) && (m->aown[l] = alloc(nt));
    if (ok && l < levels - 1 && desc->power2 != 0) ok = (m->a2own[l] = alloc(nt)) != nullptr;
  }
  ok = ok && hipMemcpy(m->tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
  // zero every owned level array (ghosts of coarse arrays are then defined)
  for (int l = 0; l < levels && ok; l++) {
    const size_t b = (size_t)m->geo[l].nt * sizeof(double);
    ok = hipMemset(m->uo[l], 0, b) == hipSuccess;
    if (ok && l < levels - 1)
      ok = hipMemset(m->r[l], 0, b) == hipSuccess && hipMemset(m->u[l], 0, b) == hipSuccess &&
           hipMemset(m->f[l], 0, b) == hipSuccess && hipMemset(m->aown[l], 0, b) == hipSuccess &&
           (!m->a2own[l] || hipMemset(m->a2own[l], 0, b) == hipSuccess);
  }
  ok = ok && hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    for (double *p : m->owned) (void)hipFree(p);
    delete m;
    return GMUNU_ENOMEM;
  }
  for (int l = 0; l < levels; l++) {
    MgGeo &G = m->geo[l];
    const double *b = m->tab;
    G.a0m = b + off[l][0];
    G.a0p = b + off[l][1];
    G.g1 = b + off[l][2];
    G.g2 = b + off[l][3];
    G.vol0 = b + off[l][4];
    G.sg0 = b + off[l][5];
    G.a1m = b + off[l][6];
    G.a1p = b + off[l][7];
    G.s2t = b + off[l][8];
    G.vol1 = b + off[l][9];
    G.sg1 = b + off[l][10];
  }
  *out = m;
  return GMUNU_OK;
}

int gmunu_mg_destroy(gmunu_mg *m) {
  if (!m) return GMUNU_ENULL;
  int rc = GMUNU_OK;
  for (auto &sl : m->slot)
    if (sl.exec && hipGraphExecDestroy(sl.exec) != hipSuccess) rc = GMUNU_EHIP;
  if (m->ev && hipEventDestroy(m->ev) != hipSuccess) rc = GMUNU_EHIP;
  if (m->gs && hipStreamDestroy(m->gs) != hipSuccess) rc = GMUNU_EHIP;
  for (double *p : m->owned)
    if (hipFree(p) != hipSuccess) rc = GMUNU_EHIP;
  delete m;
  return rc;
}

int gmunu_mg_levels(const gmunu_mg *m) { return m ? m->levels : GMUNU_ENULL; }

long gmunu_mg_size(const gmunu_mg *m, int level) {
  if (!m || level < 0 || level >= m->levels) return -1;
  return m->geo[level].nt;
}

int gmunu_mg_solve(gmunu_mg *m, double *u, const double *f, const double *a, const double *a2, double tol,
                   int max_cycles, int use_fmg, double *res_host, int *cycles_out, void *stream) {
  if (!m || !u || !f) return GMUNU_ENULL;
  if (!ok_ptr(u) || !ok_ptr(f) || (a && !aligned8(a))) return GMUNU_EALIGN;
  if (max_cycles < 0 || !(tol >= 0.0) || !a2_ok(m, a2)) return GMUNU_EINVAL;
  // the cycles run on the context's stream, ordered after the caller's work
  hipStream_t cst = as_stream(stream);
  int rc = enter(m, cst);
  if (rc) return rc;
  bind(m, u, f, a, a2, m->gs);
  hipGraphExec_t exec = cycle_graph(m, false, u, f, a, a2);
  if (!exec) return GMUNU_EHIP;
  rc = cycles(m, false, exec, tol, max_cycles, use_fmg, res_host, cycles_out);
  if (rc) return rc;
  ghosts(m->geo[m->levels - 1], u, m->gs);
  return leave(m, cst);
}

int gmunu_mg_residual_norm(gmunu_mg *m, double *u, const double *f, const double *a, const double *a2,
                           double *norm_out, void *stream) {
  if (!m || !u || !f || !norm_out) return GMUNU_ENULL;
  if (!ok_ptr(u) || !ok_ptr(f) || (a && !aligned8(a))) return GMUNU_EALIGN;
  if (!a2_ok(m, a2)) return GMUNU_EINVAL;
  hipStream_t st = as_stream(stream);
  const int top = m->levels - 1;
  m->u[top] = u;
  m->f[top] = const_cast<double *>(f);
  m->a[top] = const_cast<double *>(a);
  m->a2[top] = const_cast<double *>(a2);
  return norm(m, norm_out, st);
}

int gmunu_mg_apply(gmunu_mg *m, const double *u, const double *a, const double *a2, double *out, void *stream) {
  if (!m || !u || !out) return GMUNU_ENULL;
  if (!ok_ptr(u) || !ok_ptr(out) || (a && !aligned8(a))) return GMUNU_EALIGN;
  if (!a2_ok(m, a2)) return GMUNU_EINVAL;
  const MgGeo &G = m->geo[m->levels - 1];
  hipLaunchKernelGGL(k_mg_apply, dim3(nblocks(cells(G))), dim3(NT), 0, as_stream(stream), G, u, a, a2, out);
  return launch_status();
}

int gmunu_mg_fill_ghosts(gmunu_mg *m, int level, double *u, void *stream) {
  if (!m || !u) return GMUNU_ENULL;
  if (!aligned8(u)) return GMUNU_EALIGN;
  if (level < 0 || level >= m->levels) return GMUNU_EINVAL;
  ghosts(m->geo[level], u, as_stream(stream));
  return launch_status();
}

int gmunu_mg_smooth(gmunu_mg *m, double *u, const double *f, const double *a, const double *a2, int sweeps,
                    void *stream) {
  if (!m || !u || !f) return GMUNU_ENULL;
  if (!ok_ptr(u) || !ok_ptr(f) || (a && !aligned8(a))) return GMUNU_EALIGN;
  if (sweeps < 0 || !a2_ok(m, a2)) return GMUNU_EINVAL;
  hipStream_t st = as_stream(stream);
  const MgGeo &G = m->geo[m->levels - 1];
  split_copies(m, f, a, a2, st);
  const bool sp = m->sf != nullptr;
  sweeps_raw(G, u, f, a, a2, sweeps, st, sp ? m->fs : nullptr, sp && a ? m->as : nullptr,
             sp && a2 ? m->a2s : nullptr);
  ghosts(G, u, st);
  return launch_status();
}

int gmunu_mg_restrict(gmunu_mg *m, int level, const double *fine, double *coarse, void *stream) {
  if (!m || !fine || !coarse) return GMUNU_ENULL;
  if (!ok_ptr(fine) || !ok_ptr(coarse)) return GMUNU_EALIGN;
  if (level < 1 || level >= m->levels) return GMUNU_EINVAL;
  const MgGeo &C = m->geo[level - 1];
  hipLaunchKernelGGL(k_mg_restrict, dim3(nblocks(cells(C))), dim3(NT), 0, as_stream(stream), m->geo[level], C, fine,
                     coarse);
  return launch_status();
}

int gmunu_mg_prolong(gmunu_mg *m, int level, const double *coarse, double *fine, void *stream) {
  if (!m || !fine || !coarse) return GMUNU_ENULL;
  if (!ok_ptr(fine) || !ok_ptr(coarse)) return GMUNU_EALIGN;
  if (level < 1 || level >= m->levels) return GMUNU_EINVAL;
  const MgGeo &F = m->geo[level];
  hipLaunchKernelGGL(k_mg_prolong, dim3(nblocks(cells(F))), dim3(NT), 0, as_stream(stream), m->geo[level - 1], F,
                     coarse, fine, 0);
  return launch_status();
}

int gmunu_mg_divergence(gmunu_mg *m, const double *q, double *div, void *stream) {
  if (!m || !q || !div) return GMUNU_ENULL;
  if (!ok_ptr(q) || !ok_ptr(div)) return GMUNU_EALIGN;
  const MgGeo &G = m->geo[m->levels - 1];
  hipLaunchKernelGGL(k_mg_div, dim3(nblocks(cells(G))), dim3(NT), 0, as_stream(stream), G, q, div);
  return launch_status();
}

int gmunu_mg_subtract_gradient(gmunu_mg *m, const double *phi, double *q, void *stream) {
  if (!m || !q || !phi) return GMUNU_ENULL;
  if (!ok_ptr(q) || !ok_ptr(phi)) return GMUNU_EALIGN;
  const MgGeo &G = m->geo[m->levels - 1];
  hipLaunchKernelGGL(k_mg_subgrad, dim3(nblocks(cells(G))), dim3(NT), 0, as_stream(stream), G, phi, q);
  return launch_status();
}

int gmunu_mg_clean(gmunu_mg *m, double *q, double *phi, double *div, double tol, int max_cycles, double *res_host,
                   int *cycles_out, void *stream) {
  if (!m || !q || !phi) return GMUNU_ENULL;
  if (m->d.power != 0) return GMUNU_EINVAL;
  if (!ok_ptr(q) || !ok_ptr(phi) || (div && !aligned8(div))) return GMUNU_EALIGN;
  const int top = m->levels - 1;
  // the divergence goes into the caller's div, else into the finest uo buffer
  double *f = div ? div : m->uo[top];
  int rc = gmunu_mg_divergence(m, q, f, stream);
  if (rc) return rc;
  rc = gmunu_mg_solve(m, phi, f, nullptr, nullptr, tol, max_cycles, 1, res_host, cycles_out, stream);
  if (rc) return rc;
  ghosts(m->geo[top], phi, as_stream(stream));
  return gmunu_mg_subtract_gradient(m, phi, q, stream);
}

// ------------------------------------------------ vector equations (xCFC)

int gmunu_mg_vapply(gmunu_mg *m, const double *X, double *out, void *stream) {
  if (!m || !X || !out) return GMUNU_ENULL;
  if (!ok_ptr(X) || !ok_ptr(out)) return GMUNU_EALIGN;
  if (!vector_ok(m)) return GMUNU_EINVAL;
  const MgGeo &G = m->geo[m->levels - 1];
  hipLaunchKernelGGL(k_mgv_apply, dim3(nblocks(cells(G))), dim3(NT), 0, as_stream(stream), G, X, out);
  return launch_status();
}

int gmunu_mg_vsmooth(gmunu_mg *m, double *X, const double *f, int sweeps, void *stream) {
  if (!m || !X || !f) return GMUNU_ENULL;
  if (!ok_ptr(X) || !ok_ptr(f)) return GMUNU_EALIGN;
  if (!vector_ok(m) || sweeps < 0) return GMUNU_EINVAL;
  const MgGeo &G = m->geo[m->levels - 1];
  hipStream_t st = as_stream(stream);
  vsweeps(G, X, f, sweeps, st);
  vghosts(G, X, st);
  return launch_status();
}

int gmunu_mg_vsolve(gmunu_mg *m, double *X, const double *f, double tol, int max_cycles, int use_fmg,
                    double *res_host, int *cycles_out, void *stream) {
  if (!m || !X || !f) return GMUNU_ENULL;
  if (!ok_ptr(X) || !ok_ptr(f)) return GMUNU_EALIGN;
  if (!vector_ok(m) || max_cycles < 0 || !(tol >= 0.0)) return GMUNU_EINVAL;
  if (!vector_storage(m)) return GMUNU_ENOMEM;
  hipStream_t cst = as_stream(stream);
  int rc = enter(m, cst);
  if (rc) return rc;
  const int top = m->levels - 1;
  m->vu[top] = X;
  m->vf[top] = const_cast<double *>(f);
  hipGraphExec_t exec = cycle_graph(m, true, X, f, nullptr, nullptr);
  if (!exec) return GMUNU_EHIP;
  rc = cycles(m, true, exec, tol, max_cycles, use_fmg, res_host, cycles_out);
  if (rc) return rc;
  vghosts(m->geo[top], X, m->gs);
  return leave(m, cst);
}

int gmunu_mg_xcfc_aij(gmunu_mg *m, const double *X, double *A6, double *A2, void *stream) {
  if (!m || !X || !A6 || !A2) return GMUNU_ENULL;
  if (!ok_ptr(X) || !ok_ptr(A6) || !ok_ptr(A2)) return GMUNU_EALIGN;
  if (!vector_ok(m)) return GMUNU_EINVAL;
  const MgGeo &G = m->geo[m->levels - 1];
  hipLaunchKernelGGL(k_mgv_aij, dim3(nblocks(cells(G))), dim3(NT), 0, as_stream(stream), G, X, A6, A2);
  return launch_status();
}

int gmunu_mg_xcfc_beta_rhs(gmunu_mg *m, const double *w, const double *S, const double *A6, double *out,
                           void *stream) {
  if (!m || !w || !S || !A6 || !out) return GMUNU_ENULL;
  if (!ok_ptr(w) || !ok_ptr(S) || !ok_ptr(A6) || !ok_ptr(out)) return GMUNU_EALIGN;
  if (!vector_ok(m)) return GMUNU_EINVAL;
  const MgGeo &G = m->geo[m->levels - 1];
  hipLaunchKernelGGL(k_mgv_beta_rhs, dim3(nblocks(cells(G))), dim3(NT), 0, as_stream(stream), G, w, S, A6, out);
  return launch_status();
}

}  // extern "C"

namespace {

// The GRMHD layout of a descriptor whose interior is the multigrid's finest
// grid (same dimensions, coordinates, spacing and origin), else EINVAL.
int hydro_of(const gmunu_mg *m, const gmunu_grid_desc *hd, Hydro &H) {
  const gmunu_mg_desc &d = m->d;
  if (hd->ndim != d.ndim || hd->coord != d.coord || hd->ng < 1) return GMUNU_EINVAL;
  long T[3];
  for (int a = 0; a < 3; a++) {
    if (hd->n[a] != d.n[a]) return GMUNU_EINVAL;
    if (a < d.ndim && (std::fabs(hd->dx[a] - d.dx[a]) > 1e-12 * d.dx[a] ||
                       std::fabs(hd->xmin[a] - d.xmin[a]) > 1e-12 * (std::fabs(d.xmin[a]) + d.dx[a])))
      return GMUNU_EINVAL;
    H.ng[a] = a < d.ndim ? hd->ng : 0;
    T[a] = d.n[a] + 2 * H.ng[a];
  }
  H.T0 = T[0];
  H.T1 = T[0] * T[1];
  H.nv = H.T1 * T[2];
  H.gam = hd->gamma;
  return GMUNU_OK;
}

bool bridge_scratch(gmunu_mg *m);

// Steps 3 to 5 of the xCFC sequence (A2 = A~_ij A~^ij, or NULL for the
// scalar CFC equations alone): psi from its equation, S~ with the new psi,
// then alpha psi; psi and alpha written to the metric.  cyc: 2 ints.
int scalar_cfc(gmunu_mg *mpsi, gmunu_mg *malpha, const Hydro &H, const double *q, const double *prim,
               double *metric, const double *A2, double tol, int max_cycles, int *cyc, hipStream_t st) {
  gmunu_mg *ms[2] = {mpsi, malpha};
  const MgGeo &G0 = mpsi->geo[mpsi->levels - 1];
  double *u = mpsi->br, *a = mpsi->br + G0.nt, *f = mpsi->br + 2 * G0.nt, *a2 = mpsi->br + 3 * G0.nt;
  for (int w = 0; w < 2; w++) {
    gmunu_mg *m = ms[w];
    const MgGeo &G = m->geo[m->levels - 1];
    if (hipMemsetAsync(f, 0, (size_t)G0.nt * sizeof(double), st) != hipSuccess) return GMUNU_EHIP;
    hipLaunchKernelGGL(k_br_cfc_coef, dim3(nblocks(cells(G))), dim3(NT), 0, st, G, H, q, prim, metric, w, A2, a, a2,
                       u);
    const int rc = gmunu_mg_solve(m, u, f, a, w == 0 && A2 ? a2 : nullptr, tol, max_cycles, 1, nullptr, &cyc[w],
                                  (void *)st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_br_store, dim3(nblocks(H.nv)), dim3(NT), 0, st, G, H, u, m->d.xmin[0], w, metric);
  }
  return launch_status();
}

bool bridge_scratch(gmunu_mg *m) {
  if (m->br) return true;
  double *p = nullptr;
  if (hipMalloc(&p, 6 * (size_t)m->geo[m->levels - 1].nt * sizeof(double)) != hipSuccess) return false;
  if (hipMemset(p, 0, 6 * (size_t)m->geo[m->levels - 1].nt * sizeof(double)) != hipSuccess) {
    (void)hipFree(p);
    return false;
  }
  m->owned.push_back(p);
  m->br = p;
  return true;
}

}  // namespace

extern "C" {

int gmunu_mg_clean_state(gmunu_mg *m, const gmunu_grid_desc *hydro, double *q, const double *prim,
                         const double *metric, double tol, int max_cycles, double *res_host, int *cycles_out,
                         void *stream) {
  if (!m || !hydro || !q || !prim || !metric) return GMUNU_ENULL;
  if (!aligned8(q) || !aligned8(prim) || !aligned8(metric)) return GMUNU_EALIGN;
  Hydro H;
  int rc = hydro_of(m, hydro, H);
  if (rc) return rc;
  if (m->d.power != 0) return GMUNU_EINVAL;
  if (!bridge_scratch(m)) return GMUNU_ENOMEM;
  const MgGeo &G = m->geo[m->levels - 1];
  hipStream_t st = as_stream(stream);
  double *qb = m->br, *phi = m->br + 3 * G.nt, *div = m->br + 4 * G.nt;
  hipLaunchKernelGGL(k_br_gather_qb, dim3(nblocks(G.nt)), dim3(NT), 0, st, G, H, q, prim, metric, qb);
  if (hipMemsetAsync(phi, 0, (size_t)G.nt * sizeof(double), st) != hipSuccess) return GMUNU_EHIP;
  rc = gmunu_mg_clean(m, qb, phi, div, tol, max_cycles, res_host, cycles_out, stream);
  if (rc) return rc;
  hipLaunchKernelGGL(k_br_scatter_qb, dim3(nblocks(cells(G))), dim3(NT), 0, st, G, H, qb, q);
  return launch_status();
}

int gmunu_mg_cfc_solve(gmunu_mg *mpsi, gmunu_mg *malpha, const gmunu_grid_desc *hydro, const double *q,
                       const double *prim, double *metric, double tol, int max_cycles, int *cycles_out,
                       void *stream) {
  if (!mpsi || !malpha || !hydro || !q || !prim || !metric) return GMUNU_ENULL;
  if (!aligned8(q) || !aligned8(prim) || !aligned8(metric)) return GMUNU_EALIGN;
  Hydro H, H2;
  int rc = hydro_of(mpsi, hydro, H);
  if (!rc) rc = hydro_of(malpha, hydro, H2);
  if (rc) return rc;
  if (mpsi->d.power != -1 || mpsi->d.offset != 1.0 || malpha->d.power != 1 || malpha->d.offset != 1.0)
    return GMUNU_EINVAL;
  if (!bridge_scratch(mpsi)) return GMUNU_ENOMEM;
  int cyc[2] = {0, 0};
  rc = scalar_cfc(mpsi, malpha, H, q, prim, metric, nullptr, tol, max_cycles, cyc, as_stream(stream));
  if (!rc && cycles_out) {
    cycles_out[0] = cyc[0];
    cycles_out[1] = cyc[1];
  }
  return rc;
}

int gmunu_mg_xcfc_solve(gmunu_mg *mvec, gmunu_mg *mpsi, gmunu_mg *malpha, const gmunu_grid_desc *hydro,
                        const double *q, const double *prim, double *metric, double *X, double tol, int max_cycles,
                        int *cycles_out, void *stream) {
  if (!mvec || !mpsi || !malpha || !hydro || !q || !prim || !metric || !X) return GMUNU_ENULL;
  if (!aligned8(q) || !aligned8(prim) || !aligned8(metric) || !aligned8(X)) return GMUNU_EALIGN;
  Hydro H, H2, H3;
  int rc = hydro_of(mpsi, hydro, H);
  if (!rc) rc = hydro_of(malpha, hydro, H2);
  if (!rc) rc = hydro_of(mvec, hydro, H3);
  if (rc) return rc;
  if (!vector_ok(mvec) || mpsi->d.power != -1 || mpsi->d.offset != 1.0 || mpsi->d.power2 != -7 ||
      malpha->d.power != 1 || malpha->d.offset != 1.0)
    return GMUNU_EINVAL;
  if (!bridge_scratch(mpsi) || !vector_storage(mvec)) return GMUNU_ENOMEM;
  const MgGeo &G = mvec->geo[mvec->levels - 1];
  if (!mvec->xs && !alloc_zeroed(mvec, 17 * (size_t)G.nt, &mvec->xs)) return GMUNU_ENOMEM;
  hipStream_t st = as_stream(stream);
  double *S = mvec->xs, *fv = S + 3 * G.nt, *beta = S + 6 * G.nt, *A6 = S + 9 * G.nt, *A2 = S + 15 * G.nt,
         *w = S + 16 * G.nt;
  int cyc[4] = {0, 0, 0, 0};
  // step 1: the vector potential
  hipLaunchKernelGGL(k_bx_src, dim3(nblocks(cells(G))), dim3(NT), 0, st, G, H, q, S, fv);
  rc = gmunu_mg_vsolve(mvec, X, fv, tol, max_cycles, 1, nullptr, &cyc[0], stream);
  if (rc) return rc;
  // step 2: A~^ij
  hipLaunchKernelGGL(k_mgv_aij, dim3(nblocks(cells(G))), dim3(NT), 0, st, G, X, A6, A2);
  // steps 3 to 5: conformal factor and lapse
  rc = scalar_cfc(mpsi, malpha, H, q, prim, metric, A2, tol, max_cycles, &cyc[1], st);
  if (rc) return rc;
  // step 6: the shift
  hipLaunchKernelGGL(k_bx_w, dim3(nblocks(G.nt)), dim3(NT), 0, st, G, H, metric, w);
  hipLaunchKernelGGL(k_mgv_beta_rhs, dim3(nblocks(cells(G))), dim3(NT), 0, st, G, w, S, A6, fv);
  hipLaunchKernelGGL(k_bx_beta_in, dim3(nblocks(cells(G))), dim3(NT), 0, st, G, H, metric, beta);
  rc = gmunu_mg_vsolve(mvec, beta, fv, tol, max_cycles, 1, nullptr, &cyc[3], stream);
  if (rc) return rc;
  for (int c = 0; c < 3; c++)
    hipLaunchKernelGGL(k_br_store, dim3(nblocks(H.nv)), dim3(NT), 0, st, G, H, beta + c * G.nt, mvec->d.xmin[0],
                       2 + c, metric);
  if (cycles_out)
    for (int c = 0; c < 4; c++) cycles_out[c] = cyc[c];
  return launch_status();
}

}  // extern "C"

namespace {

// The kernels of gmunu_mg_psi_residual: the residual lands in
// mpsi->part[kNormParts].
int psi_residual_enqueue(gmunu_mg *mvec, gmunu_mg *mpsi, const gmunu_grid_desc *hydro, const double *q,
                         const double *metric, const double *X, hipStream_t st) {
  if (!mpsi || !hydro || !q || !metric || (mvec && !X)) return GMUNU_ENULL;
  if (!aligned8(q) || !aligned8(metric) || (X && !aligned8(X))) return GMUNU_EALIGN;
  Hydro H;
  int rc = hydro_of(mpsi, hydro, H);
  if (!rc && mvec) rc = hydro_of(mvec, hydro, H);
  if (rc) return rc;
  if (mpsi->d.power != -1 || mpsi->d.offset != 1.0 || (mvec && (!vector_ok(mvec) || mpsi->d.power2 != -7)))
    return GMUNU_EINVAL;
  if (!bridge_scratch(mpsi)) return GMUNU_ENOMEM;
  if (mvec && !mvec->xs && !alloc_zeroed(mvec, 17 * (size_t)mvec->geo[mvec->levels - 1].nt, &mvec->xs))
    return GMUNU_ENOMEM;
  const MgGeo &G = mpsi->geo[mpsi->levels - 1];
  double *u = mpsi->br, *a = mpsi->br + G.nt, *f = mpsi->br + 2 * G.nt, *a2 = mpsi->br + 3 * G.nt;
  const double *A2 = nullptr;
  if (mvec) {
    const MgGeo &V = mvec->geo[mvec->levels - 1];
    double *A2v = mvec->xs + 15 * V.nt;
    hipLaunchKernelGGL(k_mgv_aij, dim3(nblocks(cells(V))), dim3(NT), 0, st, V, X, nullptr, A2v);
    A2 = A2v;
  }
  if (hipMemsetAsync(f, 0, (size_t)G.nt * sizeof(double), st) != hipSuccess) return GMUNU_EHIP;
  // which 0 (the conformal factor) reads no primitives
  hipLaunchKernelGGL(k_br_cfc_coef, dim3(nblocks(cells(G))), dim3(NT), 0, st, G, H, q, nullptr, metric, 0, A2, a, a2,
                     u);
  const int top = mpsi->levels - 1;
  mpsi->u[top] = u;
  mpsi->f[top] = f;
  mpsi->a[top] = a;
  mpsi->a2[top] = A2 ? a2 : nullptr;
  norm_enqueue(mpsi, st);
  return launch_status();
}

__global__ void k_dyn_reset(double *g) {
  g[0] = 0.0;
  g[1] = 0.0;
}

// After step `step` of a chunk: the first step whose residual exceeds eps
// is recorded (g[0]) with the time after it (g[1]), and t becomes +inf, so
// that every later step of the chunk computes dt = 0 (its cap t_end - t,
// t_end finite, is negative) and changes nothing.
__global__ void k_dyn_gate(const double *res, double eps, double step, double *t, double *g) {
  if (g[0] == 0.0 && *res > eps) {
    g[0] = step;
    g[1] = *t;
    *t = INFINITY;
  }
}

__global__ void k_dyn_restore(double *t, const double *g) {
  if (g[0] != 0.0) *t = g[1];
}

}  // namespace

extern "C" {

int gmunu_mg_psi_residual(gmunu_mg *mvec, gmunu_mg *mpsi, const gmunu_grid_desc *hydro, const double *q,
                          const double *metric, const double *X, double *norm_out, void *stream) {
  if (!norm_out) return GMUNU_ENULL;
  hipStream_t st = as_stream(stream);
  const int rc = psi_residual_enqueue(mvec, mpsi, hydro, q, metric, X, st);
  if (rc) return rc;
  if (hipMemcpyAsync(norm_out, mpsi->part + kNormParts, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return GMUNU_EHIP;
  return launch_status();
}

int gmunu_mg_dynamical_steps(gmunu_mg *mvec, gmunu_mg *mpsi, gmunu_ctx *ctx, const gmunu_grid_desc *hydro,
                             double *q_n, double *q_s, double *prim, const double *metric, const double *X,
                             double cfl, double t_end, double *t_dev, double *dt_dev, uint8_t *flags,
                             unsigned int *nfatal_dev, int nsteps, double eps, int *steps_out, int *triggered_out,
                             void *stream) {
  if (!ctx || !mpsi || !hydro || !t_dev || !dt_dev || !steps_out || !triggered_out) return GMUNU_ENULL;
  if (nsteps < 1 || !std::isfinite(t_end)) return GMUNU_EINVAL;
  hipStream_t st = as_stream(stream);
  double *g = mpsi->part + kNormParts + 1;
  hipLaunchKernelGGL(k_dyn_reset, dim3(1), dim3(1), 0, st, g);
  for (int s = 1; s <= nsteps; s++) {
    int rc = gmunu_step(ctx, q_n, q_s, prim, metric, nullptr, cfl, t_end, t_dev, dt_dev, flags, nfatal_dev, stream);
    if (!rc) rc = psi_residual_enqueue(mvec, mpsi, hydro, q_n, metric, X, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_dyn_gate, dim3(1), dim3(1), 0, st, mpsi->part + kNormParts, eps, (double)s, t_dev, g);
  }
  hipLaunchKernelGGL(k_dyn_restore, dim3(1), dim3(1), 0, st, t_dev, g);
  double h[2];
  if (hipMemcpyAsync(h, g, sizeof h, hipMemcpyDeviceToHost, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
    return GMUNU_EHIP;
  *triggered_out = h[0] != 0.0;
  *steps_out = h[0] != 0.0 ? (int)h[0] : nsteps;
  return launch_status();
}

int gmunu_mg_metric_update(gmunu_mg *mvec, gmunu_mg *mpsi, gmunu_mg *malpha, gmunu_ctx *ctx,
                           const gmunu_grid_desc *hydro, double *q, double *prim, double *metric, double *X,
                           uint8_t *flags, unsigned int *nfatal_dev, double tol, int max_cycles, int *cycles_out,
                           void *stream) {
  if (!ctx || (mvec && !X)) return GMUNU_ENULL;
  int cyc[4] = {0, 0, 0, 0};
  int rc = mvec ? gmunu_mg_xcfc_solve(mvec, mpsi, malpha, hydro, q, prim, metric, X, tol, max_cycles, cyc, stream)
                : gmunu_mg_cfc_solve(mpsi, malpha, hydro, q, prim, metric, tol, max_cycles, cyc + 1, stream);
  if (rc) return rc;
  rc = gmunu_c2p(ctx, q, metric, prim, flags, nfatal_dev, stream);
  if (rc) return rc;
  rc = gmunu_fill_ghosts(ctx, prim, stream);
  if (rc) return rc;
  if (cycles_out)
    for (int c = 0; c < 4; c++) cycles_out[c] = cyc[c];
  return GMUNU_OK;
}

}  // extern "C"
