/* CPU oracle of the cell-centred multigrid solver (test infrastructure only:
 * only the tests, the smoke check and the benchmark's CPU-baseline leg use
 * it; the GPU path never does).
 *
 * Cheong et al., "Gmunu" (arXiv 2012.07322), section 2.7 (non-linear
 * cell-centred multigrid) and section 2.2 (elliptic divergence cleaning).
 * Plain C, FP64, one cell at a time, in the order the paper describes:
 *   - the equation L(u) = f with L(u) = Lap(u) - a (u + c)^p - a2 (u + c)^q,
 *     p in {-1, 0, 1}, q an integer (the scalar metric equations of section
 *     2.6 in deviation form, with q = -7 for the extrinsic-curvature term of
 *     the conformal-factor equation, and the Poisson equation of the
 *     divergence cleaning are all of this form);
 *   - Lap: the standard 3/5/7-point second-order Laplacian of the reference
 *     metric in Cartesian, cylindrical (R, z, phi) or spherical
 *     (r, theta, phi) coordinates, exactly as the paper writes it (with the
 *     second differences read as u+ - 2u + u-, see below);
 *   - smoother: Newton-Gauss-Seidel in red-black ordering (cells with
 *     i + j + k even first);
 *   - coarsest level: the same relaxation, repeated, as the solver;
 *   - restriction: piecewise constant (weighted mean of the 2^ndim
 *     children);
 *   - prolongation: Kwak's scheme (2D: (2 u_c + u_x + u_y) / 4 toward the
 *     child's side), generalised to 1D as (3 u_c + u_x) / 4 and to 3D as
 *     (u_c + u_x + u_y + u_z) / 4, the weights that keep the scheme's
 *     property of reproducing linear functions;
 *   - cycles: full-approximation-scheme V-cycles and an FAS full-multigrid
 *     cycle that starts from the current solution;
 *   - beside the paper's point smoother, alternating zebra line relaxation
 *     (line_smooth, vline_smooth), the standard remedy for the anisotropic
 *     cells on which the paper notes point smoothers converge slowly; it
 *     is defined by its steps there and changes the iteration, not the
 *     discrete solution.
 *
 * Readings where the paper is silent or garbled:
 *   - the cylindrical and spherical second differences are printed as
 *     u+ - 2u - u-; the Laplacian they discretise needs u+ - 2u + u-;
 *   - boundary conditions by ghost values: Dirichlet (u = 0 on the face),
 *     Neumann (zero normal derivative), periodic, and on the outer radial
 *     face the Robin condition d(r u)/dr = 0 of section 2.6 (ghost value
 *     u_in r_in / r_ghost, exact for a 1/r fall-off); on Cartesian and
 *     cylindrical grids the same condition (u + x.grad u = 0, and
 *     u + R du/dR + z du/dz = 0) on any face (cylindrical: the R and z
 *     faces), through the same ghost rule with r the distance of the cell
 *     centres from the origin (the paper imposes it at the outermost cell
 *     centres; the ghost form holds the 1/r fall-off the condition
 *     expresses between each boundary cell and its ghost); faces of zero
 *     area (r = 0, R = 0, theta = 0 or pi) need none;
 *   - on a periodic axis every level keeps an even number of cells (the
 *     caller chooses the levels so): with an odd count the cells on either
 *     side of the wrap share a colour, and the red-black and multi-colour
 *     orderings would no longer separate neighbours;
 *   - restriction is the volume-weighted mean of the children (the paper
 *     gives the piecewise constant stencil only; weighting by the cell
 *     volumes of the reference metric keeps the coarse problem consistent
 *     next to r = 0 and R = 0, and reduces to the plain mean on Cartesian
 *     grids).
 *
 * Arrays: one ghost layer on each active axis, layout [k][j][i], i fastest.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OM_PI 3.14159265358979323846

enum { OM_CART = 0, OM_CYL = 1, OM_SPH = 2 };
enum { OM_DIRICHLET = 0, OM_NEUMANN = 1, OM_PERIODIC = 2, OM_ROBIN = 3 };

typedef struct {
  int ndim, coord;
  int n[3];          /* interior cells of the finest level */
  double xmin[3];
  double dx[3];      /* finest spacing */
  int bc[3][2];
  int levels;        /* levels in the hierarchy (finest = levels - 1) */
  int pre, post;     /* red-black sweeps before / after the coarse correction */
  int coarse;        /* sweeps on the coarsest level */
  int power;         /* p */
  double offset;     /* c */
  int power2;        /* q of the optional second term a2 (u + c)^q */
  int smoother;      /* 0: red-black points (the paper's); 1: line relaxation */
} om_desc;

/* one level of the hierarchy */
typedef struct {
  int n[3], t[3];    /* interior cells, cells with ghosts */
  double dx[3];
  long nt;
} lvl;

static int gh(const om_desc *d, int a) { return a < d->ndim ? 1 : 0; }

static lvl level_of(const om_desc *d, int l) {
  lvl L;
  int s = d->levels - 1 - l;
  for (int a = 0; a < 3; a++) {
    L.n[a] = a < d->ndim ? d->n[a] >> s : 1;
    L.t[a] = L.n[a] + 2 * gh(d, a);
    L.dx[a] = a < d->ndim ? d->dx[a] * (double)(1 << s) : d->dx[a];
  }
  L.nt = (long)L.t[0] * L.t[1] * L.t[2];
  return L;
}

static long idx(const om_desc *d, const lvl *L, int i, int j, int k) {
  return ((long)(k + gh(d, 2)) * L->t[1] + (j + gh(d, 1))) * L->t[0] + (i + gh(d, 0));
}

static double centre(const om_desc *d, const lvl *L, int a, int i) { return d->xmin[a] + (i + 0.5) * L->dx[a]; }
static double face(const om_desc *d, const lvl *L, int a, int i) { return d->xmin[a] + i * L->dx[a]; }

/* Weights of the Laplacian at cell (i,j,k) along axis a toward the lower
 * (wm) and upper (wp) neighbour: Lap u = sum_a wp (u+ - u) - wm (u - u-). */
static void weights(const om_desc *d, const lvl *L, int a, int i, int j, int k, double *wm, double *wp) {
  double h2 = L->dx[a] * L->dx[a];
  double r = centre(d, L, 0, i), th = centre(d, L, 1, j);
  (void)k;
  *wm = *wp = 1.0 / h2;
  if (d->coord == OM_CYL) {
    if (a == 0) {
      *wm = face(d, L, 0, i) / (r * h2);
      *wp = face(d, L, 0, i + 1) / (r * h2);
    } else if (a == 2) {
      *wm = *wp = 1.0 / (r * r * h2);
    }
  } else if (d->coord == OM_SPH) {
    if (a == 0) {
      double fm = face(d, L, 0, i), fp = face(d, L, 0, i + 1);
      *wm = fm * fm / (r * r * h2);
      *wp = fp * fp / (r * r * h2);
    } else if (a == 1) {
      *wm = sin(face(d, L, 1, j)) / (r * r * sin(th) * h2);
      *wp = sin(face(d, L, 1, j + 1)) / (r * r * sin(th) * h2);
    } else {
      double s = sin(th);
      *wm = *wp = 1.0 / (r * r * s * s * h2);
    }
  }
}

/* running maximum of |v|; a NaN counts as infinite, so that a solution
 * gone NaN never reads as converged */
static double om_absmax(double m, double v) { return v != v ? INFINITY : fmax(m, fabs(v)); }

static double ipow(double w, int q) {
  double r = 1.0;
  for (int e = q < 0 ? -q : q; e > 0; e--) r *= w;
  return q < 0 ? 1.0 / r : r;
}

/* a (u + c)^p + a2 (u + c)^q and its derivative in u */
static double nonlin(const om_desc *d, double a, double a2, double u) {
  double w = u + d->offset, t;
  if (d->power == 0) t = a;
  else if (d->power == 1) t = a * w;
  else t = a / w;
  return a2 != 0.0 ? t + a2 * ipow(w, d->power2) : t;
}
static double nonlin_du(const om_desc *d, double a, double a2, double u) {
  double w = u + d->offset, t;
  if (d->power == 0) t = 0.0;
  else if (d->power == 1) t = a;
  else t = -a / (w * w);
  return a2 != 0.0 ? t + a2 * d->power2 * ipow(w, d->power2 - 1) : t;
}

/* L(u) at interior cell (i,j,k) and its derivative with respect to u there. */
static double apply_cell(const om_desc *d, const lvl *L, const double *u, const double *ac, const double *a2c,
                         int i, int j, int k, double *diag) {
  long c = idx(d, L, i, j, k);
  double lap = 0.0, dg = 0.0;
  int cell[3] = {i, j, k};
  for (int a = 0; a < d->ndim; a++) {
    int m[3] = {cell[0], cell[1], cell[2]}, p[3] = {cell[0], cell[1], cell[2]};
    m[a]--;
    p[a]++;
    double wm, wp;
    weights(d, L, a, i, j, k, &wm, &wp);
    double um = u[idx(d, L, m[0], m[1], m[2])], up = u[idx(d, L, p[0], p[1], p[2])];
    lap += wp * (up - u[c]) - wm * (u[c] - um);
    dg -= wp + wm;
  }
  double av = ac ? ac[c] : 0.0, a2v = a2c ? a2c[c] : 0.0;
  if (diag) *diag = dg - nonlin_du(d, av, a2v, u[c]);
  return lap - nonlin(d, av, a2v, u[c]);
}

/* Ratio ghost / boundary cell of the non-periodic face (a, side): cell s,
 * ghost g (s with index -1 or n along a). */
static double ghost_factor(const om_desc *d, const lvl *L, int a, int side, const int s[3], const int g[3]) {
  int kind = d->bc[a][side];
  if (kind == OM_DIRICHLET) return -1.0;
  if (kind == OM_NEUMANN) return 1.0;
  if (d->coord != OM_SPH) {
    /* 1/r falloff between the boundary cell and its ghost, r the distance
     * of the cell centres from the origin (Cartesian: the active axes;
     * cylindrical: R and z) */
    double ri = 0.0, rg = 0.0;
    for (int b = 0; b < d->ndim && b < (d->coord == OM_CYL ? 2 : 3); b++) {
      double xi = centre(d, L, b, s[b]), xg = centre(d, L, b, g[b]);
      ri += xi * xi;
      rg += xg * xg;
    }
    return sqrt(ri) / sqrt(rg);
  }
  return centre(d, L, a, s[a]) / centre(d, L, a, g[a]);
}

/* Ghost values of u on level L from its boundary conditions (face-adjacent
 * ghosts only: the stencils use no edge or corner ghost). */
static void fill_ghosts(const om_desc *d, const lvl *L, double *u) {
  for (int a = 0; a < d->ndim; a++) {
    int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
    for (int t2 = 0; t2 < L->n[b2]; t2++)
      for (int t1 = 0; t1 < L->n[b1]; t1++)
        for (int side = 0; side < 2; side++) {
          int g[3], s[3];
          g[b1] = s[b1] = t1;
          g[b2] = s[b2] = t2;
          g[a] = side == 0 ? -1 : L->n[a];
          int kind = d->bc[a][side];
          double v;
          if (kind == OM_PERIODIC) {
            s[a] = side == 0 ? L->n[a] - 1 : 0;
            v = u[idx(d, L, s[0], s[1], s[2])];
          } else {
            s[a] = side == 0 ? 0 : L->n[a] - 1;
            double ui = u[idx(d, L, s[0], s[1], s[2])];
            v = kind == OM_DIRICHLET ? -ui : kind == OM_NEUMANN ? ui : ui * ghost_factor(d, L, a, side, s, g);
          }
          u[idx(d, L, g[0], g[1], g[2])] = v;
        }
  }
}

/* Red-black Newton-Gauss-Seidel: colour 0 (i + j + k even), then colour 1,
 * ghosts refreshed before each colour. */
static void smooth(const om_desc *d, const lvl *L, double *u, const double *f, const double *ac, const double *a2c,
                   int sweeps) {
  for (int s = 0; s < sweeps; s++)
    for (int col = 0; col < 2; col++) {
      fill_ghosts(d, L, u);
      for (int k = 0; k < L->n[2]; k++)
        for (int j = 0; j < L->n[1]; j++)
          for (int i = 0; i < L->n[0]; i++) {
            if (((i + j + k) & 1) != col) continue;
            double dg;
            double Lu = apply_cell(d, L, u, ac, a2c, i, j, k, &dg);
            long c = idx(d, L, i, j, k);
            u[c] -= (Lu - f[c]) / dg;
          }
    }
  fill_ghosts(d, L, u);
}

/* Solve the tridiagonal system lo[m] x[m-1] + dg[m] x[m] + up[m] x[m+1] =
 * rhs[m] (m = 0..n-1; lo[0], up[n-1] unused) by Gaussian elimination
 * without pivoting (the Thomas algorithm); x overwrites rhs, up is
 * overwritten. */
static void thomas(int n, const double *lo, const double *dg, double *up, double *rhs) {
  double piv = dg[0];
  up[0] /= piv;
  rhs[0] /= piv;
  for (int m = 1; m < n; m++) {
    piv = dg[m] - lo[m] * up[m - 1];
    if (m < n - 1) up[m] /= piv;
    rhs[m] = (rhs[m] - lo[m] * rhs[m - 1]) / piv;
  }
  for (int m = n - 2; m >= 0; m--) rhs[m] -= up[m] * rhs[m + 1];
}

/* Lines of colour col along axis a: the transverse axes b1 < b2, colour
 * bit 0 the parity of the index along b1, bit 1 along b2 (active axes
 * only).  Calls back for each line's first cell. */
static int line_colours(const om_desc *d) { return 1 << (d->ndim - 1); }
static int on_line_colour(const om_desc *d, int a, int col, const int c[3]) {
  int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
  int p1 = b1 < d->ndim ? c[b1] & 1 : 0, p2 = b2 < d->ndim ? c[b2] & 1 : 0;
  return (p1 | (p2 << 1)) == col;
}

/* Alternating zebra line relaxation (an alternative to the paper's point
 * smoother for strongly anisotropic cells): per sweep each active
 * non-periodic axis in turn, per axis the line colours in order, per line
 * one Newton step of the line's equations with their exact Jacobian with
 * respect to the line's own cells -- the Laplacian weights toward the two
 * neighbours along the line, and on the diagonal dL/du plus, for every
 * face of the cell that is a non-periodic boundary, the weight toward that
 * face's ghost times ghost_factor (the ghost follows the cell) -- while
 * every other cell holds its current value.  For a linear L one sweep is
 * block Gauss-Seidel over the lines.  With every active axis periodic,
 * red-black point sweeps. */
static void line_smooth(const om_desc *d, const lvl *L, double *u, const double *f, const double *ac,
                        const double *a2c, int sweeps) {
  int any = 0;
  for (int a = 0; a < d->ndim; a++) any |= d->bc[a][0] != OM_PERIODIC;
  if (!any) {
    smooth(d, L, u, f, ac, a2c, sweeps);
    return;
  }
  int nmax = L->n[0] > L->n[1] ? L->n[0] : L->n[1];
  nmax = nmax > L->n[2] ? nmax : L->n[2];
  double *lo = malloc(sizeof(double) * nmax), *dg = malloc(sizeof(double) * nmax);
  double *up = malloc(sizeof(double) * nmax), *rhs = malloc(sizeof(double) * nmax);
  for (int s = 0; s < sweeps; s++)
    for (int a = 0; a < d->ndim; a++) {
      if (d->bc[a][0] == OM_PERIODIC) continue;
      int n = L->n[a];
      for (int col = 0; col < line_colours(d); col++) {
        fill_ghosts(d, L, u);
        for (int k = 0; k < (a == 2 ? 1 : L->n[2]); k++)
          for (int j = 0; j < (a == 1 ? 1 : L->n[1]); j++)
            for (int i = 0; i < (a == 0 ? 1 : L->n[0]); i++) {
              int c0[3] = {i, j, k};
              if (!on_line_colour(d, a, col, c0)) continue;
              for (int m = 0; m < n; m++) {
                int c[3] = {i, j, k};
                c[a] = m;
                double dgm, wm, wp;
                double Lu = apply_cell(d, L, u, ac, a2c, c[0], c[1], c[2], &dgm);
                for (int b = 0; b < d->ndim; b++) {
                  if (d->bc[b][0] == OM_PERIODIC) continue;
                  weights(d, L, b, c[0], c[1], c[2], &wm, &wp);
                  int g[3] = {c[0], c[1], c[2]};
                  if (c[b] == 0) {
                    g[b] = -1;
                    dgm += wm * ghost_factor(d, L, b, 0, c, g);
                  }
                  if (c[b] == L->n[b] - 1) {
                    g[b] = L->n[b];
                    dgm += wp * ghost_factor(d, L, b, 1, c, g);
                  }
                }
                weights(d, L, a, c[0], c[1], c[2], &wm, &wp);
                lo[m] = wm;
                up[m] = wp;
                dg[m] = dgm;
                rhs[m] = f[idx(d, L, c[0], c[1], c[2])] - Lu;
              }
              thomas(n, lo, dg, up, rhs);
              for (int m = 0; m < n; m++) {
                int c[3] = {i, j, k};
                c[a] = m;
                u[idx(d, L, c[0], c[1], c[2])] += rhs[m];
              }
            }
      }
    }
  free(lo);
  free(dg);
  free(up);
  free(rhs);
  fill_ghosts(d, L, u);
}

/* The descriptor's smoother. */
static void relax(const om_desc *d, const lvl *L, double *u, const double *f, const double *ac, const double *a2c,
                  int sweeps) {
  if (d->smoother)
    line_smooth(d, L, u, f, ac, a2c, sweeps);
  else
    smooth(d, L, u, f, ac, a2c, sweeps);
}

/* r = f - L(u) on the interior (u's ghosts must be current). */
static void residual(const om_desc *d, const lvl *L, const double *u, const double *f, const double *ac,
                     const double *a2c, double *r) {
  for (int k = 0; k < L->n[2]; k++)
    for (int j = 0; j < L->n[1]; j++)
      for (int i = 0; i < L->n[0]; i++) {
        long c = idx(d, L, i, j, k);
        r[c] = f[c] - apply_cell(d, L, u, ac, a2c, i, j, k, NULL);
      }
}

/* Volume of fine cell (i,j,k) up to a factor common to all cells of the
 * level (Appendix A): 1 (Cartesian), R (cylindrical), (r^2 + dr^2/12) sin
 * theta (spherical, exact shell and cone volumes). */
static double cell_vol(const om_desc *d, const lvl *L, int i, int j) {
  double r = centre(d, L, 0, i);
  if (d->coord == OM_CYL) return r;
  if (d->coord == OM_SPH) {
    double v = r * r + L->dx[0] * L->dx[0] / 12.0;
    if (d->ndim > 1) v *= sin(centre(d, L, 1, j));
    return v;
  }
  return 1.0;
}

/* coarse = volume-weighted mean of the 2^ndim fine children (interior):
 * the piecewise-constant coarse value with the children's integral. */
static void restrict_pc(const om_desc *d, const lvl *C, const lvl *F, const double *fine, double *coarse) {
  int nch = 1 << d->ndim;
  for (int k = 0; k < C->n[2]; k++)
    for (int j = 0; j < C->n[1]; j++)
      for (int i = 0; i < C->n[0]; i++) {
        double s = 0.0, w = 0.0;
        for (int ch = 0; ch < nch; ch++) {
          int fi = 2 * i + (ch & 1);
          int fj = d->ndim > 1 ? 2 * j + ((ch >> 1) & 1) : j;
          int fk = d->ndim > 2 ? 2 * k + ((ch >> 2) & 1) : k;
          double v = cell_vol(d, F, fi, fj);
          s += v * fine[idx(d, F, fi, fj, fk)];
          w += v;
        }
        coarse[idx(d, C, i, j, k)] = s / w;
      }
}

/* Kwak prolongation of the coarse field v (ghosts current) into the fine
 * interior: add (mode 1) or set (mode 0). */
static void prolong(const om_desc *d, const lvl *C, const lvl *F, const double *v, double *fine, int add) {
  const double w0 = d->ndim == 1 ? 0.75 : d->ndim == 2 ? 0.5 : 0.25;
  for (int k = 0; k < F->n[2]; k++)
    for (int j = 0; j < F->n[1]; j++)
      for (int i = 0; i < F->n[0]; i++) {
        int fc[3] = {i, j, k}, cc[3];
        for (int a = 0; a < 3; a++) cc[a] = a < d->ndim ? fc[a] >> 1 : fc[a];
        double s = w0 * v[idx(d, C, cc[0], cc[1], cc[2])];
        for (int a = 0; a < d->ndim; a++) {
          int nb[3] = {cc[0], cc[1], cc[2]};
          nb[a] += (fc[a] & 1) ? 1 : -1;
          s += 0.25 * v[idx(d, C, nb[0], nb[1], nb[2])];
        }
        long o = idx(d, F, i, j, k);
        fine[o] = add ? fine[o] + s : s;
      }
}

typedef struct {
  lvl L[16];
  double *u[16], *f[16], *a[16], *a2[16], *r[16], *uo[16];
} hier;

static void hier_init(const om_desc *d, hier *H, double *u_fine, const double *f_fine, const double *a_fine,
                      const double *a2_fine) {
  int top = d->levels - 1;
  for (int l = 0; l < d->levels; l++) {
    H->L[l] = level_of(d, l);
    long nt = H->L[l].nt;
    H->r[l] = (double *)calloc(nt, sizeof(double));
    H->uo[l] = (double *)calloc(nt, sizeof(double));
    if (l == top) {
      H->u[l] = u_fine;
      H->f[l] = (double *)f_fine;
      H->a[l] = (double *)a_fine;
      H->a2[l] = (double *)a2_fine;
    } else {
      H->u[l] = (double *)calloc(nt, sizeof(double));
      H->f[l] = (double *)calloc(nt, sizeof(double));
      H->a[l] = a_fine ? (double *)calloc(nt, sizeof(double)) : NULL;
      H->a2[l] = a2_fine ? (double *)calloc(nt, sizeof(double)) : NULL;
    }
  }
  for (int l = top; l > 0; l--) {
    if (a_fine) restrict_pc(d, &H->L[l - 1], &H->L[l], H->a[l], H->a[l - 1]);
    if (a2_fine) restrict_pc(d, &H->L[l - 1], &H->L[l], H->a2[l], H->a2[l - 1]);
  }
}

static void hier_free(const om_desc *d, hier *H) {
  int top = d->levels - 1;
  for (int l = 0; l < d->levels; l++) {
    free(H->r[l]);
    free(H->uo[l]);
    if (l != top) {
      free(H->u[l]);
      free(H->f[l]);
      free(H->a[l]);
      free(H->a2[l]);
    }
  }
}

/* Coarse problem of level l: u_{l-1} = R u_l (kept in uo_{l-1}),
 * f_{l-1} = L_{l-1}(R u_l) + R (f_l - L_l(u_l)). */
static void coarse_problem(const om_desc *d, hier *H, int l) {
  const lvl *F = &H->L[l], *C = &H->L[l - 1];
  fill_ghosts(d, F, H->u[l]);
  residual(d, F, H->u[l], H->f[l], H->a[l], H->a2[l], H->r[l]);
  restrict_pc(d, C, F, H->u[l], H->u[l - 1]);
  restrict_pc(d, C, F, H->r[l], H->r[l - 1]);
  fill_ghosts(d, C, H->u[l - 1]);
  memcpy(H->uo[l - 1], H->u[l - 1], sizeof(double) * C->nt);
  for (int k = 0; k < C->n[2]; k++)
    for (int j = 0; j < C->n[1]; j++)
      for (int i = 0; i < C->n[0]; i++) {
        long c = idx(d, C, i, j, k);
        H->f[l - 1][c] = apply_cell(d, C, H->u[l - 1], H->a[l - 1], H->a2[l - 1], i, j, k, NULL) + H->r[l - 1][c];
      }
}

/* u_l += P(u_{l-1} - uo_{l-1}) */
static void correct(const om_desc *d, hier *H, int l) {
  const lvl *C = &H->L[l - 1];
  for (long c = 0; c < C->nt; c++) H->uo[l - 1][c] = H->u[l - 1][c] - H->uo[l - 1][c];
  fill_ghosts(d, C, H->uo[l - 1]);
  prolong(d, C, &H->L[l], H->uo[l - 1], H->u[l], 1);
}

static void vcycle(const om_desc *d, hier *H, int l) {
  if (l == 0) {
    relax(d, &H->L[0], H->u[0], H->f[0], H->a[0], H->a2[0], d->coarse);
    return;
  }
  relax(d, &H->L[l], H->u[l], H->f[l], H->a[l], H->a2[l], d->pre);
  coarse_problem(d, H, l);
  vcycle(d, H, l - 1);
  correct(d, H, l);
  relax(d, &H->L[l], H->u[l], H->f[l], H->a[l], H->a2[l], d->post);
}

/* FAS full multigrid from the current solution: coarse problems down to
 * the coarsest level, solve there, then on the way up correct each level
 * from the one below and do one V-cycle on it. */
static void fmg(const om_desc *d, hier *H) {
  int top = d->levels - 1;
  for (int l = top; l > 0; l--) coarse_problem(d, H, l);
  relax(d, &H->L[0], H->u[0], H->f[0], H->a[0], H->a2[0], d->coarse);
  for (int l = 1; l <= top; l++) {
    correct(d, H, l);
    vcycle(d, H, l);
  }
}

static double max_residual(const om_desc *d, hier *H) {
  int top = d->levels - 1;
  const lvl *L = &H->L[top];
  fill_ghosts(d, L, H->u[top]);
  residual(d, L, H->u[top], H->f[top], H->a[top], H->a2[top], H->r[top]);
  double m = 0.0;
  for (int k = 0; k < L->n[2]; k++)
    for (int j = 0; j < L->n[1]; j++)
      for (int i = 0; i < L->n[0]; i++) m = om_absmax(m, H->r[top][idx(d, L, i, j, k)]);
  return m;
}

/* ------------------------------------------------------------------ API */

int om_desc_size(void) { return (int)sizeof(om_desc); }

/* L(u) on the finest level's interior; u's ghosts as the caller set them. */
void om_apply(const om_desc *d, const double *u, const double *a, const double *a2, double *out) {
  lvl L = level_of(d, d->levels - 1);
  for (int k = 0; k < L.n[2]; k++)
    for (int j = 0; j < L.n[1]; j++)
      for (int i = 0; i < L.n[0]; i++) {
        long c = idx(d, &L, i, j, k);
        out[c] = apply_cell(d, &L, u, a, a2, i, j, k, NULL);
      }
}

void om_fill_ghosts(const om_desc *d, int level, double *u) {
  lvl L = level_of(d, level);
  fill_ghosts(d, &L, u);
}

void om_smooth(const om_desc *d, double *u, const double *f, const double *a, const double *a2, int sweeps) {
  lvl L = level_of(d, d->levels - 1);
  smooth(d, &L, u, f, a, a2, sweeps);
}

/* `sweeps` line-relaxation sweeps on the finest level (line_smooth). */
void om_line_smooth(const om_desc *d, double *u, const double *f, const double *a, const double *a2, int sweeps) {
  lvl L = level_of(d, d->levels - 1);
  line_smooth(d, &L, u, f, a, a2, sweeps);
}

/* fine level l, coarse level l - 1 */
void om_restrict(const om_desc *d, int l, const double *fine, double *coarse) {
  lvl F = level_of(d, l), C = level_of(d, l - 1);
  restrict_pc(d, &C, &F, fine, coarse);
}

/* Kwak prolongation of coarse (level l - 1, ghosts as the caller set them)
 * into the interior of fine (level l). */
void om_prolong(const om_desc *d, int l, const double *coarse, double *fine) {
  lvl F = level_of(d, l), C = level_of(d, l - 1);
  prolong(d, &C, &F, coarse, fine, 0);
}

/* Solve L(u) = f on the finest level: an FAS-FMG cycle first when fmg is
 * set, then FAS V-cycles until max |f - L(u)| <= tol or max_cycles cycles
 * (the FMG cycle counts as one).  res[] (max_cycles + 1 entries) receives
 * the residual norm before and after each cycle.  Returns the cycles done. */
int om_solve(const om_desc *d, double *u, const double *f, const double *a, const double *a2, double tol,
             int max_cycles, int use_fmg, double *res) {
  hier H;
  hier_init(d, &H, u, f, a, a2);
  int top = d->levels - 1, c = 0;
  res[0] = max_residual(d, &H);
  while (c < max_cycles && res[c] > tol) {
    if (c == 0 && use_fmg)
      fmg(d, &H);
    else
      vcycle(d, &H, top);
    c++;
    res[c] = max_residual(d, &H);
  }
  fill_ghosts(d, &H.L[top], u);
  hier_free(d, &H);
  return c;
}

/* Divergence of a contravariant vector field q (3 components, same layout)
 * with respect to the reference metric, (1/sqrt(g)) d_i (sqrt(g) q^i) by
 * centred differences of sqrt(g) q^i at the neighbouring centres (the first
 * derivative of section 2.7), on the interior; q's ghosts must be set. */
static double sqrt_g(const om_desc *d, double r, double th) {
  if (d->coord == OM_CYL) return r;
  if (d->coord == OM_SPH) return r * r * sin(th);
  return 1.0;
}

void om_divergence(const om_desc *d, const double *q, double *out) {
  lvl L = level_of(d, d->levels - 1);
  for (int k = 0; k < L.n[2]; k++)
    for (int j = 0; j < L.n[1]; j++)
      for (int i = 0; i < L.n[0]; i++) {
        double s = 0.0;
        int cell[3] = {i, j, k};
        for (int a = 0; a < d->ndim; a++) {
          int m[3] = {i, j, k}, p[3] = {i, j, k};
          m[a]--;
          p[a]++;
          double gm = sqrt_g(d, centre(d, &L, 0, m[0]), centre(d, &L, 1, m[1]));
          double gp = sqrt_g(d, centre(d, &L, 0, p[0]), centre(d, &L, 1, p[1]));
          s += (gp * q[a * L.nt + idx(d, &L, p[0], p[1], p[2])] - gm * q[a * L.nt + idx(d, &L, m[0], m[1], m[2])]) /
               (2.0 * L.dx[a]);
        }
        (void)cell;
        out[idx(d, &L, i, j, k)] = s / sqrt_g(d, centre(d, &L, 0, i), centre(d, &L, 1, j));
      }
}

/* Contravariant gradient (g^{ii} d_i u, centred) of u, whose ghosts must be
 * set, subtracted from q on the interior: the cleaning update of section
 * 2.2. */
void om_subtract_gradient(const om_desc *d, const double *u, double *q) {
  lvl L = level_of(d, d->levels - 1);
  for (int k = 0; k < L.n[2]; k++)
    for (int j = 0; j < L.n[1]; j++)
      for (int i = 0; i < L.n[0]; i++) {
        double r = centre(d, &L, 0, i), th = centre(d, &L, 1, j);
        double gi[3] = {1.0, 1.0, 1.0};
        if (d->coord == OM_CYL) gi[2] = 1.0 / (r * r);
        if (d->coord == OM_SPH) {
          gi[1] = 1.0 / (r * r);
          gi[2] = 1.0 / (r * r * sin(th) * sin(th));
        }
        for (int a = 0; a < d->ndim; a++) {
          int m[3] = {i, j, k}, p[3] = {i, j, k};
          m[a]--;
          p[a]++;
          double g = (u[idx(d, &L, p[0], p[1], p[2])] - u[idx(d, &L, m[0], m[1], m[2])]) / (2.0 * L.dx[a]);
          q[a * L.nt + idx(d, &L, i, j, k)] -= gi[a] * g;
        }
      }
}

/* ------------------------------------------------------------------------
 * Vector equations of the xCFC scheme (section 2.6):
 *     L(X)^i = Lap X^i + (1/3) grad_i (div X) = f^i,
 * in orthonormal components (Cartesian x, y, z; cylindrical R, z, phi;
 * spherical r, theta, phi; curvilinear grids axisymmetric, d/dphi = 0, at
 * most two active axes).  Second derivatives by the standard second-order
 * differences (the flux form of the scalar Laplacian of each system), the
 * mixed ones by the four-point corner formula of section 2.7, first ones
 * centred.  In curvilinear coordinates the vector Laplacian and grad div of
 * orthonormal components carry the connection terms:
 *   cylindrical: L_R = Lap A_R - A_R/R^2 + (1/3) d_R D,
 *                L_z = Lap A_z + (1/3) d_z D,  L_phi = Lap A_phi - A_phi/R^2,
 *                D = (1/R) d_R (R A_R) + d_z A_z,
 *                d_R D = (1/R) d_R (R d_R A_R) - A_R/R^2 + d_R d_z A_z,
 *                d_z D = (1/R) d_R d_z (R A_R) + d_z^2 A_z;
 *   spherical:   L_r = Lap A_r - 2 A_r/r^2 - 2/(r^2 sin) d_th (sin A_th)
 *                      + (1/3) d_r D,
 *                L_th = Lap A_th - A_th/(r^2 sin^2) + (2/r^2) d_th A_r
 *                      + (1/3) (1/r) d_th D,
 *                L_phi = Lap A_phi - A_phi/(r^2 sin^2),
 *                D = (1/r^2) d_r (r^2 A_r) + 1/(r sin) d_th (sin A_th),
 *                d_r D = (1/r^2) d_r (r^2 d_r A_r) - 2 A_r/r^2
 *                        + (1/sin) [(1/r) d_r d_th (sin A_th) - d_th (sin A_th) / r^2]
 *                (the last written so that no corner radius divides: a
 *                coarse level's ghost centre can lie at r = 0),
 *                (1/r) d_th D = (1/r^3) d_r d_th (r^2 A_r)
 *                        + 1/(r^2 sin) d_th (sin d_th A_th) - A_th/(r^2 sin^2).
 * The mixed stencil couples diagonal neighbours, which share a colour in
 * the red-black ordering, so the Gauss-Seidel sweep visits the 2^ndim
 * colours (i mod 2, j mod 2, k mod 2) in turn; a colour's cells, and the
 * three components of each cell, are updated together from the values
 * before the colour's update.  Values across the boundary, edges and
 * corners included, come from each axis's rule applied to each component:
 * periodic wrap, or a mirror with a sign per component -- Dirichlet: all
 * odd; Neumann (a symmetry face): the normal component odd, and also the
 * phi component at the cylindrical axis and at the polar axis, and every
 * component at the spherical centre (whose mirror image at theta -> pi -
 * theta is the cell itself on equatorially symmetric grids, which the
 * centre therefore requires).  Coordinates enter the corner weights with
 * their signs, so across a mirror they extend the field's parity.  Same
 * level hierarchy, volume-weighted restriction, Kwak prolongation and FAS
 * cycles as the scalar solver, per component.  Vector arrays: three
 * component arrays back to back. */

static double vsign(const om_desc *d, const lvl *L, int a, int side, int comp) {
  if (d->bc[a][side] == OM_DIRICHLET) return -1.0;
  int odd = comp == a;
  double fpos = side == 0 ? d->xmin[a] : d->xmin[a] + L->n[a] * L->dx[a];
  if (d->coord == OM_CYL && a == 0 && fabs(fpos) < 1e-12 && comp == 2) odd = 1;
  if (d->coord == OM_SPH && a == 0 && fabs(fpos) < 1e-12) odd = 1;
  if (d->coord == OM_SPH && a == 1 && (fabs(fpos) < 1e-12 || fabs(fpos - OM_PI) < 1e-12) && comp == 2) odd = 1;
  return odd ? -1.0 : 1.0;
}

/* component comp of u at cell (i,j,k), inside or across the boundary */
static double vval(const om_desc *d, const lvl *L, const double *u, int comp, int i, int j, int k) {
  int c[3] = {i, j, k};
  double fac = 1.0;
  for (int a = 0; a < d->ndim; a++) {
    int n = L->n[a];
    if (c[a] >= 0 && c[a] < n) continue;
    int side = c[a] < 0 ? 0 : 1;
    if (d->bc[a][side] == OM_PERIODIC) {
      c[a] = side == 0 ? c[a] + n : c[a] - n;
      continue;
    }
    fac *= vsign(d, L, a, side, comp);
    c[a] = side == 0 ? -1 - c[a] : 2 * n - 1 - c[a];
  }
  return fac * u[comp * L->nt + idx(d, L, c[0], c[1], c[2])];
}

/* face ghosts of every component from the rule above */
static void vfill_ghosts(const om_desc *d, const lvl *L, double *u) {
  for (int comp = 0; comp < 3; comp++)
    for (int a = 0; a < d->ndim; a++) {
      int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
      for (int t2 = 0; t2 < L->n[b2]; t2++)
        for (int t1 = 0; t1 < L->n[b1]; t1++)
          for (int side = 0; side < 2; side++) {
            int g[3];
            g[b1] = t1;
            g[b2] = t2;
            g[a] = side == 0 ? -1 : L->n[a];
            u[comp * L->nt + idx(d, L, g[0], g[1], g[2])] = vval(d, L, u, comp, g[0], g[1], g[2]);
          }
    }
}

/* axis-a term of the flux-form Laplacian of component comp, and its
 * diagonal */
static double vlap_axis(const om_desc *d, const lvl *L, const double *u, int comp, int a, int i, int j, int k,
                        double *dg) {
  int m[3] = {i, j, k}, p[3] = {i, j, k};
  m[a]--;
  p[a]++;
  double wm, wp;
  weights(d, L, a, i, j, k, &wm, &wp);
  double u0 = u[comp * L->nt + idx(d, L, i, j, k)];
  *dg = -(wm + wp);
  return wp * (vval(d, L, u, comp, p[0], p[1], p[2]) - u0) - wm * (u0 - vval(d, L, u, comp, m[0], m[1], m[2]));
}

enum { W_ONE, W_R, W_SIN, W_R2 };

/* four-point mixed difference d_0 d_1 of g = w(corner) * component b */
static double vmix01(const om_desc *d, const lvl *L, const double *u, int b, int i, int j, int k, int wk) {
  double s = 0.0;
  for (int di = -1; di <= 1; di += 2)
    for (int dj = -1; dj <= 1; dj += 2) {
      double r = centre(d, L, 0, i + di), th = centre(d, L, 1, j + dj);
      double w = wk == W_ONE ? 1.0 : wk == W_R ? r : wk == W_R2 ? r * r : sin(th);
      s += di * dj * w * vval(d, L, u, b, i + di, j + dj, k);
    }
  return s / (4.0 * L->dx[0] * L->dx[1]);
}

static double vapply_cart(const om_desc *d, const lvl *L, const double *u, int comp, int i, int j, int k,
                          double *diag) {
  const double u0 = u[comp * L->nt + idx(d, L, i, j, k)];
  double lap = 0.0, dg = 0.0;
  for (int a = 0; a < d->ndim; a++) {
    int m[3] = {i, j, k}, p[3] = {i, j, k};
    m[a]--;
    p[a]++;
    double h2 = L->dx[a] * L->dx[a];
    lap += (vval(d, L, u, comp, p[0], p[1], p[2]) - 2.0 * u0 + vval(d, L, u, comp, m[0], m[1], m[2])) / h2;
    dg -= 2.0 / h2;
  }
  double gd = 0.0;
  if (comp < d->ndim) {
    for (int b = 0; b < d->ndim; b++) {
      if (b == comp) {
        int m[3] = {i, j, k}, p[3] = {i, j, k};
        m[b]--;
        p[b]++;
        double h2 = L->dx[b] * L->dx[b];
        gd += (vval(d, L, u, b, p[0], p[1], p[2]) - 2.0 * u0 + vval(d, L, u, b, m[0], m[1], m[2])) / h2;
        dg -= (2.0 / 3.0) / h2;
      } else {
        int pp[3] = {i, j, k}, pm[3] = {i, j, k}, mp[3] = {i, j, k}, mm[3] = {i, j, k};
        pp[comp]++; pp[b]++;
        pm[comp]++; pm[b]--;
        mp[comp]--; mp[b]++;
        mm[comp]--; mm[b]--;
        gd += (vval(d, L, u, b, pp[0], pp[1], pp[2]) - vval(d, L, u, b, pm[0], pm[1], pm[2]) -
               vval(d, L, u, b, mp[0], mp[1], mp[2]) + vval(d, L, u, b, mm[0], mm[1], mm[2])) /
              (4.0 * L->dx[comp] * L->dx[b]);
      }
    }
  }
  if (diag) *diag = dg;
  return lap + gd / 3.0;
}

static double vapply_curv(const om_desc *d, const lvl *L, const double *u, int comp, int i, int j, int k,
                          double *diag) {
  const double u0 = u[comp * L->nt + idx(d, L, i, j, k)];
  const int two = d->ndim > 1;
  double dl0, dl1 = 0.0;
  const double l0 = vlap_axis(d, L, u, comp, 0, i, j, k, &dl0);
  const double l1 = two ? vlap_axis(d, L, u, comp, 1, i, j, k, &dl1) : 0.0;
  const double lap = l0 + l1, dlap = dl0 + dl1;
  const double r = centre(d, L, 0, i), ir2 = 1.0 / (r * r);
  double Lq, dg;
  if (d->coord == OM_CYL) {
    if (comp == 0) {
      const double mix = two ? vmix01(d, L, u, 1, i, j, k, W_ONE) : 0.0;
      Lq = lap - u0 * ir2 + (l0 - u0 * ir2 + mix) / 3.0;
      dg = dlap - ir2 + (dl0 - ir2) / 3.0;
    } else if (comp == 1) {
      const double mix = two ? vmix01(d, L, u, 0, i, j, k, W_R) / r : 0.0;
      Lq = lap + (mix + l1) / 3.0;
      dg = dlap + dl1 / 3.0;
    } else {
      Lq = lap - u0 * ir2;
      dg = dlap - ir2;
    }
  } else {
    const double s = sin(centre(d, L, 1, j)), is2 = 1.0 / (s * s);
    if (comp == 0) {
      double dth = 0.0, mix = 0.0;
      if (two) {
        dth = (sin(centre(d, L, 1, j + 1)) * vval(d, L, u, 1, i, j + 1, k) -
               sin(centre(d, L, 1, j - 1)) * vval(d, L, u, 1, i, j - 1, k)) /
              (2.0 * L->dx[1]);
        mix = (vmix01(d, L, u, 1, i, j, k, W_SIN) / r - dth * ir2) / s;
      }
      Lq = lap - 2.0 * u0 * ir2 - 2.0 * ir2 / s * dth + (l0 - 2.0 * u0 * ir2 + mix) / 3.0;
      dg = dlap - 2.0 * ir2 + (dl0 - 2.0 * ir2) / 3.0;
    } else if (comp == 1) {
      double dr = 0.0, mix = 0.0;
      if (two) {
        dr = (vval(d, L, u, 0, i, j + 1, k) - vval(d, L, u, 0, i, j - 1, k)) / (2.0 * L->dx[1]);
        mix = vmix01(d, L, u, 0, i, j, k, W_R2) / (r * r * r);
      }
      Lq = lap - u0 * ir2 * is2 + 2.0 * ir2 * dr + (mix + l1 - u0 * ir2 * is2) / 3.0;
      dg = dlap - ir2 * is2 + (dl1 - ir2 * is2) / 3.0;
    } else {
      Lq = lap - u0 * ir2 * is2;
      dg = dlap - ir2 * is2;
    }
  }
  if (diag) *diag = dg;
  return Lq;
}

static double vapply_cell(const om_desc *d, const lvl *L, const double *u, int comp, int i, int j, int k,
                          double *diag) {
  return d->coord == OM_CART ? vapply_cart(d, L, u, comp, i, j, k, diag) : vapply_curv(d, L, u, comp, i, j, k, diag);
}

static void vsmooth(const om_desc *d, const lvl *L, double *u, const double *f, int sweeps) {
  const int ncol = 1 << d->ndim;
  for (int s = 0; s < sweeps; s++)
    for (int col = 0; col < ncol; col++)
      for (int k = 0; k < L->n[2]; k++)
        for (int j = 0; j < L->n[1]; j++)
          for (int i = 0; i < L->n[0]; i++) {
            int cc = (i & 1) | ((j & 1) << 1) | ((k & 1) << 2);
            if (cc != col) continue;
            long c = idx(d, L, i, j, k);
            double Lu[3], dg[3];
            for (int comp = 0; comp < 3; comp++) Lu[comp] = vapply_cell(d, L, u, comp, i, j, k, &dg[comp]);
            for (int comp = 0; comp < 3; comp++) u[comp * L->nt + c] -= (Lu[comp] - f[comp * L->nt + c]) / dg[comp];
          }
}

/* Line relaxation of the vector equations (as line_smooth): per line the
 * components one after the other, each a Newton step of its own equation
 * with its exact Jacobian with respect to that component on the line's
 * cells -- the flux-form Laplacian weights along the line, times 4/3 for
 * the component along the line's axis (the grad-div term adds (1/3)
 * d^2/dx_a^2 of the a-th component); on the diagonal the point smoother's
 * dL/du plus, for every non-periodic boundary face of the cell, the
 * weight toward its mirror ghost (times 4/3 across a face normal to the
 * component) times the component's sign there -- everything else at its
 * current value (the other components included). */
static void vline_smooth(const om_desc *d, const lvl *L, double *u, const double *f, int sweeps) {
  int any = 0;
  for (int a = 0; a < d->ndim; a++) any |= d->bc[a][0] != OM_PERIODIC;
  if (!any) {
    vsmooth(d, L, u, f, sweeps);
    return;
  }
  int nmax = L->n[0] > L->n[1] ? L->n[0] : L->n[1];
  nmax = nmax > L->n[2] ? nmax : L->n[2];
  double *lo = malloc(sizeof(double) * nmax), *dg = malloc(sizeof(double) * nmax);
  double *up = malloc(sizeof(double) * nmax), *rhs = malloc(sizeof(double) * nmax);
  for (int s = 0; s < sweeps; s++)
    for (int a = 0; a < d->ndim; a++) {
      if (d->bc[a][0] == OM_PERIODIC) continue;
      int n = L->n[a];
      for (int col = 0; col < line_colours(d); col++)
        for (int k = 0; k < (a == 2 ? 1 : L->n[2]); k++)
          for (int j = 0; j < (a == 1 ? 1 : L->n[1]); j++)
            for (int i = 0; i < (a == 0 ? 1 : L->n[0]); i++) {
              int c0[3] = {i, j, k};
              if (!on_line_colour(d, a, col, c0)) continue;
              for (int comp = 0; comp < 3; comp++) {
                double kap = comp == a ? 4.0 / 3.0 : 1.0;
                for (int m = 0; m < n; m++) {
                  int c[3] = {i, j, k};
                  c[a] = m;
                  double dgm, wm, wp;
                  double Lu = vapply_cell(d, L, u, comp, c[0], c[1], c[2], &dgm);
                  for (int b = 0; b < d->ndim; b++) {
                    if (d->bc[b][0] == OM_PERIODIC) continue;
                    double kb = comp == b ? 4.0 / 3.0 : 1.0;
                    weights(d, L, b, c[0], c[1], c[2], &wm, &wp);
                    if (c[b] == 0) dgm += kb * wm * vsign(d, L, b, 0, comp);
                    if (c[b] == L->n[b] - 1) dgm += kb * wp * vsign(d, L, b, 1, comp);
                  }
                  weights(d, L, a, c[0], c[1], c[2], &wm, &wp);
                  lo[m] = kap * wm;
                  up[m] = kap * wp;
                  dg[m] = dgm;
                  rhs[m] = f[comp * L->nt + idx(d, L, c[0], c[1], c[2])] - Lu;
                }
                thomas(n, lo, dg, up, rhs);
                for (int m = 0; m < n; m++) {
                  int c[3] = {i, j, k};
                  c[a] = m;
                  u[comp * L->nt + idx(d, L, c[0], c[1], c[2])] += rhs[m];
                }
              }
            }
    }
  free(lo);
  free(dg);
  free(up);
  free(rhs);
}

static void vrelax(const om_desc *d, const lvl *L, double *u, const double *f, int sweeps) {
  if (d->smoother)
    vline_smooth(d, L, u, f, sweeps);
  else
    vsmooth(d, L, u, f, sweeps);
}

static void vresidual(const om_desc *d, const lvl *L, const double *u, const double *f, double *r) {
  for (int k = 0; k < L->n[2]; k++)
    for (int j = 0; j < L->n[1]; j++)
      for (int i = 0; i < L->n[0]; i++) {
        long c = idx(d, L, i, j, k);
        for (int comp = 0; comp < 3; comp++)
          r[comp * L->nt + c] = f[comp * L->nt + c] - vapply_cell(d, L, u, comp, i, j, k, NULL);
      }
}

typedef struct {
  lvl L[16];
  double *u[16], *f[16], *r[16], *uo[16];
} vhier;

static void vhier_init(const om_desc *d, vhier *H, double *u, const double *f) {
  int top = d->levels - 1;
  for (int l = 0; l < d->levels; l++) {
    H->L[l] = level_of(d, l);
    long nt = 3 * H->L[l].nt;
    H->r[l] = (double *)calloc(nt, sizeof(double));
    H->uo[l] = (double *)calloc(nt, sizeof(double));
    H->u[l] = l == top ? u : (double *)calloc(nt, sizeof(double));
    H->f[l] = l == top ? (double *)f : (double *)calloc(nt, sizeof(double));
  }
}

static void vhier_free(const om_desc *d, vhier *H) {
  int top = d->levels - 1;
  for (int l = 0; l < d->levels; l++) {
    free(H->r[l]);
    free(H->uo[l]);
    if (l != top) {
      free(H->u[l]);
      free(H->f[l]);
    }
  }
}

static void vcoarse_problem(const om_desc *d, vhier *H, int l) {
  const lvl *F = &H->L[l], *C = &H->L[l - 1];
  vresidual(d, F, H->u[l], H->f[l], H->r[l]);
  for (int comp = 0; comp < 3; comp++) {
    restrict_pc(d, C, F, H->u[l] + comp * F->nt, H->u[l - 1] + comp * C->nt);
    restrict_pc(d, C, F, H->r[l] + comp * F->nt, H->r[l - 1] + comp * C->nt);
  }
  memcpy(H->uo[l - 1], H->u[l - 1], sizeof(double) * 3 * C->nt);
  for (int k = 0; k < C->n[2]; k++)
    for (int j = 0; j < C->n[1]; j++)
      for (int i = 0; i < C->n[0]; i++) {
        long c = idx(d, C, i, j, k);
        for (int comp = 0; comp < 3; comp++)
          H->f[l - 1][comp * C->nt + c] = vapply_cell(d, C, H->u[l - 1], comp, i, j, k, NULL) +
                                          H->r[l - 1][comp * C->nt + c];
      }
}

static void vcorrect(const om_desc *d, vhier *H, int l) {
  const lvl *C = &H->L[l - 1], *F = &H->L[l];
  for (long c = 0; c < 3 * C->nt; c++) H->uo[l - 1][c] = H->u[l - 1][c] - H->uo[l - 1][c];
  vfill_ghosts(d, C, H->uo[l - 1]);
  for (int comp = 0; comp < 3; comp++) prolong(d, C, F, H->uo[l - 1] + comp * C->nt, H->u[l] + comp * F->nt, 1);
}

static void vvcycle(const om_desc *d, vhier *H, int l) {
  if (l == 0) {
    vrelax(d, &H->L[0], H->u[0], H->f[0], d->coarse);
    return;
  }
  vrelax(d, &H->L[l], H->u[l], H->f[l], d->pre);
  vcoarse_problem(d, H, l);
  vvcycle(d, H, l - 1);
  vcorrect(d, H, l);
  vrelax(d, &H->L[l], H->u[l], H->f[l], d->post);
}

static void vfmg(const om_desc *d, vhier *H) {
  int top = d->levels - 1;
  for (int l = top; l > 0; l--) vcoarse_problem(d, H, l);
  vrelax(d, &H->L[0], H->u[0], H->f[0], d->coarse);
  for (int l = 1; l <= top; l++) {
    vcorrect(d, H, l);
    vvcycle(d, H, l);
  }
}

static double vmax_residual(const om_desc *d, vhier *H) {
  int top = d->levels - 1;
  const lvl *L = &H->L[top];
  vresidual(d, L, H->u[top], H->f[top], H->r[top]);
  double m = 0.0;
  for (int comp = 0; comp < 3; comp++)
    for (int k = 0; k < L->n[2]; k++)
      for (int j = 0; j < L->n[1]; j++)
        for (int i = 0; i < L->n[0]; i++) m = om_absmax(m, H->r[top][comp * L->nt + idx(d, L, i, j, k)]);
  return m;
}

/* L(X) on the interior of the finest level (Cartesian). */
void om_vapply(const om_desc *d, const double *u, double *out) {
  lvl L = level_of(d, d->levels - 1);
  for (int k = 0; k < L.n[2]; k++)
    for (int j = 0; j < L.n[1]; j++)
      for (int i = 0; i < L.n[0]; i++)
        for (int comp = 0; comp < 3; comp++)
          out[comp * L.nt + idx(d, &L, i, j, k)] = vapply_cell(d, &L, u, comp, i, j, k, NULL);
}

void om_vsmooth(const om_desc *d, double *u, const double *f, int sweeps) {
  lvl L = level_of(d, d->levels - 1);
  vsmooth(d, &L, u, f, sweeps);
}

void om_vline_smooth(const om_desc *d, double *u, const double *f, int sweeps) {
  lvl L = level_of(d, d->levels - 1);
  vline_smooth(d, &L, u, f, sweeps);
}

/* Face ghosts of the three components of X on the finest level from the
 * vector boundary rule (per-component parity). */
void om_vfill_ghosts(const om_desc *d, double *u) {
  lvl L = level_of(d, d->levels - 1);
  vfill_ghosts(d, &L, u);
}

/* Solve L(X) = f like om_solve; the ghost entries of X are left zero. */
int om_vsolve(const om_desc *d, double *u, const double *f, double tol, int max_cycles, int use_fmg, double *res) {
  vhier H;
  vhier_init(d, &H, u, f);
  int top = d->levels - 1, c = 0;
  res[0] = vmax_residual(d, &H);
  while (c < max_cycles && res[c] > tol) {
    if (c == 0 && use_fmg)
      vfmg(d, &H);
    else
      vvcycle(d, &H, top);
    c++;
    res[c] = vmax_residual(d, &H);
  }
  vhier_free(d, &H);
  return c;
}

/* A~^ij = grad^i X^j + grad^j X^i - (2/3) delta^ij div X (section 2.6) in
 * orthonormal components, centred first derivatives with the boundary rule
 * across the boundary, and the connection terms of cylindrical and
 * spherical coordinates (d/dphi = 0):
 *   cylindrical: grad_phi X_R = -X_phi/R, grad_phi X_phi = X_R/R;
 *   spherical:   grad_th X_r = (d_th X_r - X_th)/r, grad_th X_th = (d_th X_th + X_r)/r,
 *                grad_th X_phi = d_th X_phi / r, grad_phi X_r = -X_phi/r,
 *                grad_phi X_th = -cot X_phi / r, grad_phi X_phi = (X_r + cot X_th)/r.
 * On the interior: the six components (xx, yy, zz, xy, xz, yz, in the
 * order of the axes) into A6 and A~_ij A~^ij into a2. */
void om_xcfc_aij(const om_desc *d, const double *X, double *A6, double *a2) {
  lvl L = level_of(d, d->levels - 1);
  for (int k = 0; k < L.n[2]; k++)
    for (int j = 0; j < L.n[1]; j++)
      for (int i = 0; i < L.n[0]; i++) {
        double g[3][3];  /* g[a][b] = d_a X^b (coordinate derivative of component b) */
        for (int a = 0; a < 3; a++)
          for (int b = 0; b < 3; b++) {
            g[a][b] = 0.0;
            if (a >= d->ndim) continue;
            int m[3] = {i, j, k}, p[3] = {i, j, k};
            m[a]--;
            p[a]++;
            g[a][b] = (vval(d, &L, X, b, p[0], p[1], p[2]) - vval(d, &L, X, b, m[0], m[1], m[2])) / (2.0 * L.dx[a]);
          }
        long c = idx(d, &L, i, j, k);
        double x[3] = {X[c], X[L.nt + c], X[2 * L.nt + c]};
        double G[3][3];  /* G[a][b] = grad_a X_b, orthonormal */
        for (int a = 0; a < 3; a++)
          for (int b = 0; b < 3; b++) G[a][b] = g[a][b];
        if (d->coord == OM_CYL) {
          double R = centre(d, &L, 0, i);
          G[2][0] = -x[2] / R;
          G[2][1] = 0.0;
          G[2][2] = x[0] / R;
        } else if (d->coord == OM_SPH) {
          double r = centre(d, &L, 0, i), th = centre(d, &L, 1, j), ct = cos(th) / sin(th);
          G[1][0] = (g[1][0] - x[1]) / r;
          G[1][1] = (g[1][1] + x[0]) / r;
          G[1][2] = g[1][2] / r;
          G[2][0] = -x[2] / r;
          G[2][1] = -ct * x[2] / r;
          G[2][2] = (x[0] + ct * x[1]) / r;
        }
        double dv = G[0][0] + G[1][1] + G[2][2];
        double A[3][3];
        for (int a = 0; a < 3; a++)
          for (int b = 0; b < 3; b++) A[a][b] = G[a][b] + G[b][a] - (a == b ? 2.0 / 3.0 * dv : 0.0);
        const int pa[6] = {0, 1, 2, 0, 0, 1}, pb[6] = {0, 1, 2, 1, 2, 2};
        for (int q = 0; q < 6; q++) A6[q * L.nt + c] = A[pa[q]][pb[q]];
        double sum = 0.0;
        for (int a = 0; a < 3; a++)
          for (int b = 0; b < 3; b++) sum += A[a][b] * A[a][b];
        a2[c] = sum;
      }
}

/* Right-hand side of the shift equation (section 2.6), orthonormal
 * components: 16 pi w S_i + 2 A~^ij grad_j w with w = alpha psi^-6 (its
 * ghosts set by the caller; grad_theta w = d_theta w / r in spherical
 * coordinates), S = psi^6 S_i the rescaled momentum density and A6 from
 * om_xcfc_aij, on the interior. */
void om_xcfc_beta_rhs(const om_desc *d, const double *w, const double *S, const double *A6, double *out) {
  lvl L = level_of(d, d->levels - 1);
  const int qi[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
  for (int k = 0; k < L.n[2]; k++)
    for (int j = 0; j < L.n[1]; j++)
      for (int i = 0; i < L.n[0]; i++) {
        long c = idx(d, &L, i, j, k);
        double gw[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < d->ndim; a++) {
          int m[3] = {i, j, k}, p[3] = {i, j, k};
          m[a]--;
          p[a]++;
          gw[a] = (w[idx(d, &L, p[0], p[1], p[2])] - w[idx(d, &L, m[0], m[1], m[2])]) / (2.0 * L.dx[a]);
        }
        if (d->coord == OM_SPH) gw[1] /= centre(d, &L, 0, i);
        for (int a = 0; a < 3; a++) {
          double t = 0.0;
          for (int b = 0; b < 3; b++) t += A6[qi[a][b] * L.nt + c] * gw[b];
          out[a * L.nt + c] = 16.0 * OM_PI * w[c] * S[a * L.nt + c] + 2.0 * t;
        }
      }
}
