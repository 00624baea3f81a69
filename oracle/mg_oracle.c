/* CPU oracle of the cell-centred multigrid solver (test infrastructure only:
 * only the tests, the smoke check and the benchmark's CPU-baseline leg use
 * it; the GPU path never does).
 *
 * Cheong et al., "Gmunu" (arXiv 2012.07322), section 2.7 (non-linear
 * cell-centred multigrid) and section 2.2 (elliptic divergence cleaning).
 * Plain C, FP64, one cell at a time, in the order the paper describes:
 *   - the equation L(u) = f with L(u) = Lap(u) - a (u + c)^p, p in {-1, 0, 1}
 *     (the scalar metric equations of section 2.6 in deviation form and the
 *     Poisson equation of the divergence cleaning are all of this form);
 *   - Lap: the standard 3/5/7-point second-order Laplacian of the reference
 *     metric in Cartesian, cylindrical (R, z, phi) or spherical
 *     (r, theta, phi) coordinates, exactly as the paper writes it (with the
 *     second differences read as u+ - 2u + u-, see below);
 *   - smoother: Newton-Gauss-Seidel in red-black ordering (cells with
 *     i + j + k even first);
 *   - coarsest level: the same relaxation, repeated, as the solver;
 *   - restriction: piecewise constant (mean of the 2^ndim children);
 *   - prolongation: Kwak's scheme (2D: (2 u_c + u_x + u_y) / 4 toward the
 *     child's side), generalised to 1D as (3 u_c + u_x) / 4 and to 3D as
 *     (u_c + u_x + u_y + u_z) / 4, the weights that keep the scheme's
 *     property of reproducing linear functions;
 *   - cycles: full-approximation-scheme V-cycles and an FAS full-multigrid
 *     cycle that starts from the current solution.
 *
 * Readings where the paper is silent or garbled:
 *   - the cylindrical and spherical second differences are printed as
 *     u+ - 2u - u-; the Laplacian they discretise needs u+ - 2u + u-;
 *   - boundary conditions by ghost values: Dirichlet (u = 0 on the face),
 *     Neumann (zero normal derivative), periodic, and on the outer radial
 *     face the Robin condition d(r u)/dr = 0 of section 2.6 (ghost value
 *     u_in r_in / r_ghost, exact for a 1/r fall-off); faces of zero area
 *     (r = 0, R = 0, theta = 0 or pi) need none;
 *   - restriction is an unweighted mean of the children in every
 *     coordinate system (the paper gives the piecewise constant stencil
 *     only).
 *
 * Arrays: one ghost layer on each active axis, layout [k][j][i], i fastest.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

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

static double nonlin(const om_desc *d, double a, double u) {
  if (d->power == 0) return a;
  if (d->power == 1) return a * (u + d->offset);
  return a / (u + d->offset);
}
static double nonlin_du(const om_desc *d, double a, double u) {
  if (d->power == 0) return 0.0;
  if (d->power == 1) return a;
  return -a / ((u + d->offset) * (u + d->offset));
}

/* L(u) at interior cell (i,j,k) and its derivative with respect to u there. */
static double apply_cell(const om_desc *d, const lvl *L, const double *u, const double *ac, int i, int j, int k,
                         double *diag) {
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
  double av = ac ? ac[c] : 0.0;
  if (diag) *diag = dg - nonlin_du(d, av, u[c]);
  return lap - nonlin(d, av, u[c]);
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
            if (kind == OM_DIRICHLET) {
              v = -ui;
            } else if (kind == OM_NEUMANN) {
              v = ui;
            } else {
              v = ui * centre(d, L, a, s[a]) / centre(d, L, a, g[a]);
            }
          }
          u[idx(d, L, g[0], g[1], g[2])] = v;
        }
  }
}

/* Red-black Newton-Gauss-Seidel: colour 0 (i + j + k even), then colour 1,
 * ghosts refreshed before each colour. */
static void smooth(const om_desc *d, const lvl *L, double *u, const double *f, const double *ac, int sweeps) {
  for (int s = 0; s < sweeps; s++)
    for (int col = 0; col < 2; col++) {
      fill_ghosts(d, L, u);
      for (int k = 0; k < L->n[2]; k++)
        for (int j = 0; j < L->n[1]; j++)
          for (int i = 0; i < L->n[0]; i++) {
            if (((i + j + k) & 1) != col) continue;
            double dg;
            double Lu = apply_cell(d, L, u, ac, i, j, k, &dg);
            long c = idx(d, L, i, j, k);
            u[c] -= (Lu - f[c]) / dg;
          }
    }
  fill_ghosts(d, L, u);
}

/* r = f - L(u) on the interior (u's ghosts must be current). */
static void residual(const om_desc *d, const lvl *L, const double *u, const double *f, const double *ac, double *r) {
  for (int k = 0; k < L->n[2]; k++)
    for (int j = 0; j < L->n[1]; j++)
      for (int i = 0; i < L->n[0]; i++) {
        long c = idx(d, L, i, j, k);
        r[c] = f[c] - apply_cell(d, L, u, ac, i, j, k, NULL);
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
  double *u[16], *f[16], *a[16], *r[16], *uo[16];
} hier;

static void hier_init(const om_desc *d, hier *H, double *u_fine, const double *f_fine, const double *a_fine) {
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
    } else {
      H->u[l] = (double *)calloc(nt, sizeof(double));
      H->f[l] = (double *)calloc(nt, sizeof(double));
      H->a[l] = a_fine ? (double *)calloc(nt, sizeof(double)) : NULL;
    }
  }
  for (int l = top; l > 0; l--)
    if (a_fine) restrict_pc(d, &H->L[l - 1], &H->L[l], H->a[l], H->a[l - 1]);
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
    }
  }
}

/* Coarse problem of level l: u_{l-1} = R u_l (kept in uo_{l-1}),
 * f_{l-1} = L_{l-1}(R u_l) + R (f_l - L_l(u_l)). */
static void coarse_problem(const om_desc *d, hier *H, int l) {
  const lvl *F = &H->L[l], *C = &H->L[l - 1];
  fill_ghosts(d, F, H->u[l]);
  residual(d, F, H->u[l], H->f[l], H->a[l], H->r[l]);
  restrict_pc(d, C, F, H->u[l], H->u[l - 1]);
  restrict_pc(d, C, F, H->r[l], H->r[l - 1]);
  fill_ghosts(d, C, H->u[l - 1]);
  memcpy(H->uo[l - 1], H->u[l - 1], sizeof(double) * C->nt);
  for (int k = 0; k < C->n[2]; k++)
    for (int j = 0; j < C->n[1]; j++)
      for (int i = 0; i < C->n[0]; i++) {
        long c = idx(d, C, i, j, k);
        H->f[l - 1][c] = apply_cell(d, C, H->u[l - 1], H->a[l - 1], i, j, k, NULL) + H->r[l - 1][c];
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
    smooth(d, &H->L[0], H->u[0], H->f[0], H->a[0], d->coarse);
    return;
  }
  smooth(d, &H->L[l], H->u[l], H->f[l], H->a[l], d->pre);
  coarse_problem(d, H, l);
  vcycle(d, H, l - 1);
  correct(d, H, l);
  smooth(d, &H->L[l], H->u[l], H->f[l], H->a[l], d->post);
}

/* FAS full multigrid from the current solution: coarse problems down to
 * the coarsest level, solve there, then on the way up correct each level
 * from the one below and do one V-cycle on it. */
static void fmg(const om_desc *d, hier *H) {
  int top = d->levels - 1;
  for (int l = top; l > 0; l--) coarse_problem(d, H, l);
  smooth(d, &H->L[0], H->u[0], H->f[0], H->a[0], d->coarse);
  for (int l = 1; l <= top; l++) {
    correct(d, H, l);
    vcycle(d, H, l);
  }
}

static double max_residual(const om_desc *d, hier *H) {
  int top = d->levels - 1;
  const lvl *L = &H->L[top];
  fill_ghosts(d, L, H->u[top]);
  residual(d, L, H->u[top], H->f[top], H->a[top], H->r[top]);
  double m = 0.0;
  for (int k = 0; k < L->n[2]; k++)
    for (int j = 0; j < L->n[1]; j++)
      for (int i = 0; i < L->n[0]; i++) m = fmax(m, fabs(H->r[top][idx(d, L, i, j, k)]));
  return m;
}

/* ------------------------------------------------------------------ API */

int om_desc_size(void) { return (int)sizeof(om_desc); }

/* L(u) on the finest level's interior; u's ghosts as the caller set them. */
void om_apply(const om_desc *d, const double *u, const double *a, double *out) {
  lvl L = level_of(d, d->levels - 1);
  for (int k = 0; k < L.n[2]; k++)
    for (int j = 0; j < L.n[1]; j++)
      for (int i = 0; i < L.n[0]; i++) {
        long c = idx(d, &L, i, j, k);
        out[c] = apply_cell(d, &L, u, a, i, j, k, NULL);
      }
}

void om_fill_ghosts(const om_desc *d, int level, double *u) {
  lvl L = level_of(d, level);
  fill_ghosts(d, &L, u);
}

void om_smooth(const om_desc *d, double *u, const double *f, const double *a, int sweeps) {
  lvl L = level_of(d, d->levels - 1);
  smooth(d, &L, u, f, a, sweeps);
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
int om_solve(const om_desc *d, double *u, const double *f, const double *a, double tol, int max_cycles, int use_fmg,
             double *res) {
  hier H;
  hier_init(d, &H, u, f, a);
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
