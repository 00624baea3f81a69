// GRMHD finite-volume step for MI355X (gfx950): single-grid kernels and the
// C ABI.
//
// One RK stage is up to three launches on the caller's stream:
//   k_stage   per tile of cells (16x4x3 in 3D, 16x15 in 2D, 255 in 1D, so
//             that each direction's faces fit one per thread): the tile's
//             plus-shaped region of prim and metric is staged in LDS once,
//             then per direction each face is reconstructed (MC, MP5 or
//             PPM) and its HLLE or TVDLF flux (optionally positivity-limited)
//             computed once, fluxes exchanged through LDS into the flux-area
//             divergence; then gravitational + geometric sources and the RK
//             combination;
//   k_c2p     per interior cell: primitive recovery with error handling,
//             writing the face ghosts its cell is the source of on the axes
//             whose boundary rules copy a cell of the line;
//   k_ghosts  per remaining face-adjacent ghost cell: boundary fill.
// The time step is a per-cell rate reduced by wavefront shuffles to one
// maximum per workgroup (a fixed number of grid-stride workgroups, or in
// gmunu_steps the previous step's last recovery), then by one workgroup that
// writes dt: no atomics, no memset, graph-capturable.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/gmunu.h"
#include "gmunu_dev.hpp"
#include "gmunu_host.hpp"
#include "gmunu_tile.hpp"

using namespace gm;

struct gmunu_ctx {
  gmunu_grid_desc d;
  Grid G;
  int device;
  double *geo;                 // packed 1D geometry tables (device)
  double *acc;                 // CFL partial maxima (device, kCflParts words)
  double *c2pmax;              // CFL maxima per recovery workgroup (gmunu_steps; null in gmunu_step_static)
  long rghosts;                // face ghosts the recovery of a step writes (recovery_ghosts)
  int raxes;                   // on that many leading axes
  double *qt;                  // limiter only: third conserved state for the middle SSPRK3 stage
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

// MODE 0: dqdt = L(prim).  MODE 1: q_out = ca q_n + cb (q_s + dt L(prim)),
// with the positivity-preserving flux limiter when P = 1.  MODE 2: MODE 1
// and then the primitive recovery of q_out into fc.prim (another array
// than prim).  skipp (nullable): nothing is done when *skipp == 0 (a step
// past t_end).  One workgroup per tile.
template <int TX, int TY, int TZ, int ND, int MODE, int REC, int R, int P>
__global__ __launch_bounds__(NT, (stage_occupancy<TX, TY, TZ, ND, recon_halo(REC)>())) void k_stage(
    const Grid G, const double *__restrict__ prim, const double *__restrict__ met, const double *qn, const double *qs,
    double *out, const double *__restrict__ dtp, double ca, double cb, const double *__restrict__ skipp,
    const double *__restrict__ kij, FusedC2P fc) {
  __shared__ double sF[stage_lds<TX, TY, TZ, ND, recon_halo(REC)>()];
  if (skipp && *skipp == 0.0) return;
  int bx, by, bz;
  xcd_tile(G, TX, TY, TZ, bx, by, bz);
  stage_tile<TX, TY, TZ, ND, MODE, REC, R, P>(G, bx * TX, by * TY, bz * TZ, prim, met, qn, qs, out, dtp, ca, cb, sF,
                                            kij, fc);
}

// Recovery of one interior cell per thread.  gaxes: also write the face
// ghosts of the first gaxes axes copied from the recovered cells.  part
// (nullable): the workgroup's maximum CFL rate of the primitives just
// recovered, at part[blockIdx.x] (the next step's CFL maxima, when nothing
// changes the interior primitives before it).
__global__ __launch_bounds__(NT) void k_c2p(const Grid G, double *q, const double *__restrict__ met, double *prim,
                                            uint8_t *flags, unsigned int *nfatal, const double *__restrict__ skipp,
                                            int gaxes, double *part) {
  if (skipp && *skipp == 0.0) return;
  const long t = (long)blockIdx.x * NT + threadIdx.x;
  const bool in = t < interior_count(G);
  if (in) c2p_one(G, q, met, prim, flags, nfatal, t, nullptr, gaxes);
  if (part) {
    const double m = block_max(in ? cfl_one(G, prim, met, t) : 0.0);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
  }
}

__global__ __launch_bounds__(NT) void k_prim2con(const Grid G, const double *__restrict__ prim,
                                                 const double *__restrict__ met, double *q) {
  const long c = (long)blockIdx.x * NT + threadIdx.x;
  if (c < G.nv) prim2con_one(G, prim, met, q, c);
}

// Ghost fill, one ghost per thread, from ghost number `skip` on (ghosts are
// numbered axis by axis; the recovery may have written those of the
// leading axes).
__global__ __launch_bounds__(NT) void k_ghosts(const Grid G, double *prim, long total,
                                               const double *__restrict__ skipp, long skip) {
  if (skipp && *skipp == 0.0) return;
  const long t = (long)blockIdx.x * NT + threadIdx.x + skip;
  if (t < total) ghost_one(G, prim, t);
}

// Per-workgroup maxima of the CFL rate over a grid-stride range of interior
// cells, written to part[blockIdx] (no atomics).
__global__ __launch_bounds__(NT) void k_cfl(const Grid G, const double *__restrict__ prim,
                                            const double *__restrict__ met, double *part) {
  const long nin = interior_count(G);
  double rate = 0.0;
  for (long t = (long)blockIdx.x * NT + threadIdx.x; t < nin; t += (long)gridDim.x * NT)
    rate = fmax(rate, cfl_one(G, prim, met, t));
  const double m = block_max(rate);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// dt = cfl / max(part), capped at t_end - t.
// Eight independent maxima per thread keep eight loads in flight (the
// partials of gmunu_steps are one per recovery workgroup: 65536 at 256^3);
// the maximum does not depend on the order.
__global__ __launch_bounds__(NT) void k_cfl_finish(const double *part, int nparts, double cfl, double t_end,
                                                   const double *tp, double *dtp) {
  double mu[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int b = threadIdx.x;
  for (; b + 7 * NT < nparts; b += 8 * NT) {
#pragma unroll
    for (int u = 0; u < 8; u++) mu[u] = fmax(mu[u], part[b + u * NT]);
  }
  for (; b < nparts; b += NT) mu[0] = fmax(mu[0], part[b]);
  double m = 0.0;
#pragma unroll
  for (int u = 0; u < 8; u++) m = fmax(m, mu[u]);
  m = block_max(m);
  if (threadIdx.x == 0) *dtp = dt_from_rate(m, cfl, tp ? *tp : 0.0, t_end);
}

__global__ void k_advance(double *tp, const double *dtp) { *tp += *dtp; }

template <int TX, int TY, int TZ, int ND, int MODE, int REC, int R, int P>
void launch_stage_t(const gmunu_ctx *ctx, const double *prim, const double *met, const double *kij,
                    const double *qn, const double *qs, double *out, const double *dtp, double ca, double cb,
                    const double *skipp, FusedC2P fc, hipStream_t st) {
  const Grid &G = ctx->G;
  dim3 grid(((G.n[0] + TX - 1) / TX) * ((G.n[1] + TY - 1) / TY) * ((G.n[2] + TZ - 1) / TZ));
  hipLaunchKernelGGL((k_stage<TX, TY, TZ, ND, MODE, REC, R, P>), grid, dim3(NT), 0, st, G, prim, met, qn, qs, out,
                     dtp, ca, cb, skipp, kij, fc);
}

template <int MODE>
void launch_stage(const gmunu_ctx *ctx, const double *prim, const double *met, const double *kij,
                  const double *qn, const double *qs, double *out, const double *dtp, double ca, double cb,
                  const double *skipp, hipStream_t st, FusedC2P fc = FusedC2P{nullptr, nullptr, nullptr}) {
  const int rec = ctx->G.recon, lf = ctx->G.riemann == GMUNU_RIEMANN_TVDLF;
  // the limiter acts on the stage's Euler step, so the RHS alone (MODE 0) is unlimited
  const int pp = MODE != 0 && ctx->G.pp;
  switch (ctx->G.ndim * 16 + rec * 4 + lf * 2 + pp) {
#define GM_CASE(NDIM, TX, TY, TZ, M, L, P)                                                                      \
  case NDIM * 16 + M * 4 + L * 2 + P:                                                                            \
    launch_stage_t<TX, TY, TZ, NDIM, MODE, M, L, MODE == 1 && P>(ctx, prim, met, kij, qn, qs, out, dtp, ca, cb,  \
                                                                 skipp, fc, st);                                  \
    break;
#define GM_CASES_R(NDIM, TX, TY, TZ, M) \
  GM_CASE(NDIM, TX, TY, TZ, M, 0, 0)    \
  GM_CASE(NDIM, TX, TY, TZ, M, 0, 1)    \
  GM_CASE(NDIM, TX, TY, TZ, M, 1, 0)    \
  GM_CASE(NDIM, TX, TY, TZ, M, 1, 1)
#define GM_CASES(NDIM, TX, TY, TZ)  \
  GM_CASES_R(NDIM, TX, TY, TZ, 0) \
  GM_CASES_R(NDIM, TX, TY, TZ, 1) \
  GM_CASES_R(NDIM, TX, TY, TZ, 2)
    GM_CASES(1, 255, 1, 1)
    GM_CASES(2, 16, 15, 1)
    GM_CASES(3, 16, 4, 3)
#undef GM_CASES
#undef GM_CASES_R
#undef GM_CASE
    default:
      break;
  }
}

int launch_c2p(gmunu_ctx *ctx, double *q, const double *metric, double *prim, uint8_t *flags,
               unsigned int *nfatal_dev, const double *skipp, hipStream_t st, int gaxes = 0, double *part = nullptr) {
  ProfScope ps(ctx, st, GMUNU_K_C2P);
  hipLaunchKernelGGL(k_c2p, dim3(nblocks(interior_cells(ctx->G))), dim3(NT), 0, st, ctx->G, q, metric, prim, flags,
                     nfatal_dev, skipp, gaxes, part);
  return launch_status();
}

int launch_ghosts(gmunu_ctx *ctx, double *prim, const double *skipp, hipStream_t st, long skip = 0) {
  const long tot = ghost_total(ctx->G);
  if (tot - skip <= 0) return GMUNU_OK;
  ProfScope ps(ctx, st, GMUNU_K_GHOSTS);
  hipLaunchKernelGGL(k_ghosts, dim3(nblocks(tot - skip)), dim3(NT), 0, st, ctx->G, prim, tot, skipp, skip);
  return launch_status();
}

// One RK stage; with skipp non-null nothing is changed when *skipp == 0.
// part (nullable, separate recovery only): the recovery also writes the
// next step's CFL maxima there (k_c2p).
int rk_stage_impl(gmunu_ctx *ctx, int stage, const double *dt_dev, const double *q_n, const double *q_s,
                  double *q_out, const double *prim_in, double *prim_out, const double *metric, const double *kij,
                  uint8_t *flags, unsigned int *nfatal_dev, const double *skipp, hipStream_t st,
                  double *part = nullptr) {
  const int nst = ctx->d.rk;
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
  // with separate input and output primitives (and no limiter) the stage
  // kernel recovers the primitives itself; otherwise the recovery is its
  // own kernel after the stage
  const bool fuse = prim_out != prim_in && !ctx->G.pp;
  {
    ProfScope ps(ctx, st, GMUNU_K_STAGE);
    if (fuse)
      launch_stage<2>(ctx, prim_in, metric, kij, q_n, q_s, q_out, dt_dev, ca, cb, skipp, st,
                      FusedC2P{prim_out, flags, nfatal_dev});
    else
      launch_stage<1>(ctx, prim_in, metric, kij, q_n, q_s, q_out, dt_dev, ca, cb, skipp, st);
  }
  int rc = launch_status();
  if (rc) return rc;
  if (fuse) return launch_ghosts(ctx, prim_out, skipp, st);
  rc = launch_c2p(ctx, q_out, metric, prim_out, flags, nfatal_dev, skipp, st, ctx->raxes, part);
  if (rc) return rc;
  return launch_ghosts(ctx, prim_out, skipp, st, ctx->rghosts);
}

int step_impl(gmunu_ctx *ctx, double *q_n, double *q_s, double *prim, const double *metric, const double *kij,
              double cfl, double t_end, double *t_dev, double *dt_dev, uint8_t *flags, unsigned int *nfatal_dev,
              void *stream, bool cfl_from_part = false, double *part_out = nullptr);

}  // namespace

// --------------------------------------------------------------------- API

extern "C" {

int gmunu_create(const gmunu_grid_desc *desc, gmunu_ctx **out) {
  if (!desc || !out) return GMUNU_ENULL;
  const int rc = validate_desc(*desc);
  if (rc) return rc;
  gmunu_ctx *ctx = new (std::nothrow) gmunu_ctx();
  if (!ctx) return GMUNU_ENOMEM;
  ctx->d = *desc;
  ctx->prof = 0;
  ctx->nrec = 0;
  ctx->c2pmax = nullptr;
  ctx->rghosts = recovery_ghosts(*desc, &ctx->raxes);
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    delete ctx;
    return GMUNU_EHIP;
  }
  std::vector<double> tab;
  const GeoOffsets off = setup_grid(*desc, ctx->G, tab);
  if (hipMalloc(&ctx->geo, tab.size() * sizeof(double)) != hipSuccess) {
    delete ctx;
    return GMUNU_ENOMEM;
  }
  if (hipMalloc(&ctx->acc, kCflParts * sizeof(double)) != hipSuccess) {
    (void)hipFree(ctx->geo);
    delete ctx;
    return GMUNU_ENOMEM;
  }
  if (hipMalloc(&ctx->c2pmax, nblocks(interior_cells(ctx->G)) * sizeof(double)) != hipSuccess) {
    (void)hipFree(ctx->geo);
    (void)hipFree(ctx->acc);
    delete ctx;
    return GMUNU_ENOMEM;
  }
  // with the limiter a stage reads the base state of neighbouring cells, so
  // its output may not overwrite its base: the step needs a third state
  ctx->qt = nullptr;
  if (desc->pp_limiter && desc->rk == 3 &&
      hipMalloc(&ctx->qt, (size_t)NV * ctx->G.nv * sizeof(double)) != hipSuccess) {
    (void)hipFree(ctx->geo);
    (void)hipFree(ctx->acc);
    (void)hipFree(ctx->c2pmax);
    delete ctx;
    return GMUNU_ENOMEM;
  }
  if (hipMemcpy(ctx->geo, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(ctx->acc, 0, kCflParts * sizeof(double)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(ctx->geo);
    (void)hipFree(ctx->acc);
    (void)hipFree(ctx->c2pmax);
    if (ctx->qt) (void)hipFree(ctx->qt);
    delete ctx;
    return GMUNU_EHIP;
  }
  bind_geo(ctx->G, ctx->geo, off);
  *out = ctx;
  return GMUNU_OK;
}

int gmunu_destroy(gmunu_ctx *ctx) {
  if (!ctx) return GMUNU_ENULL;
  int rc = GMUNU_OK;
  for (auto e : ctx->ev) (void)hipEventDestroy(e);
  if (hipFree(ctx->geo) != hipSuccess) rc = GMUNU_EHIP;
  if (hipFree(ctx->acc) != hipSuccess) rc = GMUNU_EHIP;
  if (hipFree(ctx->c2pmax) != hipSuccess) rc = GMUNU_EHIP;
  if (ctx->qt && hipFree(ctx->qt) != hipSuccess) rc = GMUNU_EHIP;
  delete ctx;
  return rc;
}

long gmunu_ntot(const gmunu_ctx *ctx) { return ctx ? ctx->G.nv : -1; }

int gmunu_prim2con(gmunu_ctx *ctx, const double *prim, const double *metric, double *q, void *stream) {
  if (!ctx || !prim || !metric || !q) return GMUNU_ENULL;
  if (!aligned8(prim) || !aligned8(metric) || !aligned8(q)) return GMUNU_EALIGN;
  ProfScope ps(ctx, as_stream(stream), GMUNU_K_OTHER);
  hipLaunchKernelGGL(k_prim2con, dim3(nblocks(ctx->G.nv)), dim3(NT), 0, as_stream(stream), ctx->G, prim, metric, q);
  return launch_status();
}

int gmunu_c2p(gmunu_ctx *ctx, double *q, const double *metric, double *prim, uint8_t *flags,
              unsigned int *nfatal_dev, void *stream) {
  if (!ctx || !q || !metric || !prim) return GMUNU_ENULL;
  if (!aligned8(prim) || !aligned8(metric) || !aligned8(q)) return GMUNU_EALIGN;
  return launch_c2p(ctx, q, metric, prim, flags, nfatal_dev, nullptr, as_stream(stream));
}

int gmunu_fill_ghosts(gmunu_ctx *ctx, double *prim, void *stream) {
  if (!ctx || !prim) return GMUNU_ENULL;
  if (!aligned8(prim)) return GMUNU_EALIGN;
  return launch_ghosts(ctx, prim, nullptr, as_stream(stream));
}

int gmunu_rhs(gmunu_ctx *ctx, const double *prim, const double *metric, const double *kij, double *dqdt,
              void *stream) {
  if (!ctx || !prim || !metric || !dqdt) return GMUNU_ENULL;
  if (!aligned8(prim) || !aligned8(metric) || !aligned8(dqdt) || !aligned8(kij)) return GMUNU_EALIGN;
  {
    ProfScope ps(ctx, as_stream(stream), GMUNU_K_STAGE);
    launch_stage<0>(ctx, prim, metric, kij, nullptr, nullptr, dqdt, nullptr, 0.0, 0.0, nullptr, as_stream(stream));
  }
  return launch_status();
}

int gmunu_cfl_dt(gmunu_ctx *ctx, const double *prim, const double *metric, double cfl, double t_end,
                 const double *t_dev, double *dt_dev, void *stream) {
  if (!ctx || !prim || !metric || !dt_dev) return GMUNU_ENULL;
  if (!aligned8(prim) || !aligned8(metric) || !aligned8(dt_dev)) return GMUNU_EALIGN;
  if (!(cfl > 0.0)) return GMUNU_EINVAL;
  const long nb = nblocks(interior_cells(ctx->G));
  const int nparts = (int)(nb < kCflParts ? nb : kCflParts);
  {
    ProfScope ps(ctx, as_stream(stream), GMUNU_K_CFL);
    hipLaunchKernelGGL(k_cfl, dim3(nparts), dim3(NT), 0, as_stream(stream), ctx->G, prim, metric, ctx->acc);
  }
  {
    ProfScope ps(ctx, as_stream(stream), GMUNU_K_OTHER);
    hipLaunchKernelGGL(k_cfl_finish, dim3(1), dim3(NT), 0, as_stream(stream), ctx->acc, nparts, cfl, t_end, t_dev, dt_dev);
  }
  return launch_status();
}

int gmunu_rk_stage(gmunu_ctx *ctx, int stage, const double *dt_dev, const double *q_n, const double *q_s,
                   double *q_out, const double *prim_in, double *prim_out, const double *metric, const double *kij,
                   uint8_t *flags, unsigned int *nfatal_dev, void *stream) {
  if (!ctx || !dt_dev || !q_n || !q_out || !prim_in || !prim_out || !metric) return GMUNU_ENULL;
  if (!aligned8(kij)) return GMUNU_EALIGN;
  if (stage > 0 && !q_s) return GMUNU_ENULL;
  if (stage < 0 || stage >= ctx->d.rk) return GMUNU_EINVAL;
  if (ctx->d.pp_limiter && q_out == (stage == 0 ? q_n : q_s)) return GMUNU_EINVAL;
  return rk_stage_impl(ctx, stage, dt_dev, q_n, q_s, q_out, prim_in, prim_out, metric, kij, flags, nfatal_dev,
                       nullptr, as_stream(stream));
}

int gmunu_step(gmunu_ctx *ctx, double *q_n, double *q_s, double *prim, const double *metric, const double *kij,
               double cfl, double t_end, double *t_dev, double *dt_dev, uint8_t *flags, unsigned int *nfatal_dev,
               void *stream) {
  if (!ctx || !q_n || !q_s || !prim || !metric || !t_dev || !dt_dev) return GMUNU_ENULL;
  if (!aligned8(kij)) return GMUNU_EALIGN;
  return step_impl(ctx, q_n, q_s, prim, metric, kij, cfl, t_end, t_dev, dt_dev, flags, nfatal_dev, stream);
}

int gmunu_steps(gmunu_ctx *ctx, double *q_n, double *q_s, double *prim, const double *metric, const double *kij,
                double cfl, double t_end, double *t_dev, double *dt_dev, uint8_t *flags, unsigned int *nfatal_dev,
                int nsteps, void *stream) {
  if (!ctx || !q_n || !q_s || !prim || !metric || !t_dev || !dt_dev) return GMUNU_ENULL;
  if (!aligned8(kij)) return GMUNU_EALIGN;
  if (nsteps < 1) return GMUNU_EINVAL;
  for (int k = 0; k < nsteps; k++) {
    const int rc = step_impl(ctx, q_n, q_s, prim, metric, kij, cfl, t_end, t_dev, dt_dev, flags, nfatal_dev, stream,
                             k > 0, k + 1 < nsteps ? ctx->c2pmax : nullptr);
    if (rc) return rc;
  }
  return GMUNU_OK;
}

}  // extern "C"

namespace {

// The launches of one step (gmunu_step), on a context whose geometry tables
// and CFL partials are in place.  cfl_from_part: the CFL maxima are those
// the previous step's last recovery wrote to ctx->c2pmax (no CFL kernel);
// part_out (nullable): this step's last recovery writes the next step's
// maxima there.
int step_impl(gmunu_ctx *ctx, double *q_n, double *q_s, double *prim, const double *metric, const double *kij,
              double cfl, double t_end, double *t_dev, double *dt_dev, uint8_t *flags, unsigned int *nfatal_dev,
              void *stream, bool cfl_from_part, double *part_out) {
  int rc;
  if (cfl_from_part) {
    if (!(cfl > 0.0)) return GMUNU_EINVAL;
    ProfScope ps(ctx, as_stream(stream), GMUNU_K_OTHER);
    hipLaunchKernelGGL(k_cfl_finish, dim3(1), dim3(NT), 0, as_stream(stream), ctx->c2pmax,
                       (int)nblocks(interior_cells(ctx->G)), cfl, t_end, t_dev, dt_dev);
    rc = launch_status();
  } else {
    rc = gmunu_cfl_dt(ctx, prim, metric, cfl, t_end, t_dev, dt_dev, stream);
  }
  if (rc) return rc;
  const int nst = ctx->d.rk;
  // stage s reads base[s] and writes base[s + 1] (q_n last); without the
  // limiter a stage reads only its own cell's base, so the middle SSPRK3
  // stage may update q_s in place
  double *base[4] = {q_n, q_s, q_s, q_n};
  if (nst == 2) base[2] = q_n;
  if (nst == 3 && ctx->qt) base[2] = ctx->qt;
  for (int s = 0; s < nst; s++) {
    rc = rk_stage_impl(ctx, s, dt_dev, q_n, base[s], base[s + 1], prim, prim, metric, kij, flags, nfatal_dev,
                       dt_dev, as_stream(stream), s == nst - 1 ? part_out : nullptr);
    if (rc) return rc;
  }
  {
    ProfScope ps(ctx, as_stream(stream), GMUNU_K_OTHER);
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, as_stream(stream), t_dev, dt_dev);
  }
  return launch_status();
}

}  // namespace

extern "C" {

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

// ------------------------------------------------- allocation-free step

namespace {

// Capacity of the file-scope scratch: geometry tables of grids with at most
// kStaticAxis cells per axis (ghosts included), then the CFL partials.
constexpr int kStaticAxis = 8192;
constexpr size_t kStaticGeo = 16 * (size_t)(kStaticAxis + 1);
constexpr size_t kStaticWords = kStaticGeo + kCflParts;

}  // namespace

// The scratch of gmunu_step_static (one copy per GPU, held until the process
// ends).  In host code this name is a stand-in, not a device address: host
// code uses only the address hipGetSymbolAddress gives for the current
// device (static_scratch()).
static __device__ __align__(256) double scratch[kStaticWords];

namespace {

struct GeoParams {
  int coord, nt[3], g[3];
  double xmin[3], dx[3];
};

// The geometry tables of setup_grid (Appendix A), computed on the device:
// one thread per table index.  The products and sums are rounded one at a
// time as on the host; sines and cosines are the device's.
__global__ __launch_bounds__(NT) void k_geo(const GeoParams p, double *tab, const GeoOffsets o) {
  const int t = blockIdx.x * NT + threadIdx.x;
  auto xc = [&](int a, int I) { return __dadd_rn(p.xmin[a], __dmul_rn((double)(I - p.g[a]) + 0.5, p.dx[a])); };
  auto xf = [&](int a, int F) { return __dadd_rn(p.xmin[a], __dmul_rn((double)(F - p.g[a]), p.dx[a])); };
  auto cv = [&](int a, int I) {
    const double x = xc(a, I), d = p.dx[a];
    if (p.coord == GMUNU_CYL && a == 0) return __dmul_rn(x, d);
    if (p.coord == GMUNU_SPH && a == 0) return __dmul_rn(__dadd_rn(__dmul_rn(x, x), __ddiv_rn(__dmul_rn(d, d), 12.0)), d);
    if (p.coord == GMUNU_SPH && a == 1) return __dmul_rn(__dmul_rn(2.0, sin(x)), sin(__dmul_rn(0.5, d)));
    return d;
  };
  for (int a = 0; a < 3; a++) {
    if (t < p.nt[a]) tab[o.icv[a] + t] = __ddiv_rn(1.0, cv(a, t));
    if (t <= p.nt[a]) {
      const double x = xf(a, t);
      double f = 1.0;
      if (p.coord == GMUNU_CYL && a == 0) f = x;
      if (p.coord == GMUNU_SPH && a == 0) f = __dmul_rn(x, x);
      if (p.coord == GMUNU_SPH && a == 1) f = sin(x);
      tab[o.fa[a] + t] = f;
    }
  }
  if (t < p.nt[0]) {
    const double x = xc(0, t);
    tab[o.r2c + t] = __dmul_rn(x, x);
    tab[o.xc0 + t] = x;
    double gA = 0.0, gB = 0.0;
    if (p.coord == GMUNU_SPH) {
      const double xp = xf(0, t + 1), xm = xf(0, t);
      const double p2 = __dmul_rn(xp, xp), m2 = __dmul_rn(xm, xm), v = cv(0, t);
      gA = __ddiv_rn(__dmul_rn(0.5, __dsub_rn(p2, m2)), v);
      gB = __ddiv_rn(__dmul_rn(-0.25, __dsub_rn(__dmul_rn(p2, p2), __dmul_rn(m2, m2))), v);
    } else if (p.coord == GMUNU_CYL) {
      gA = __ddiv_rn(1.0, x);
    }
    tab[o.gA + t] = gA;
    tab[o.gB + t] = gB;
  }
  if (t <= p.nt[0]) {
    const double x = xf(0, t);
    tab[o.r2f + t] = __dmul_rn(x, x);
  }
  if (t < p.nt[1]) {
    const double x = xc(1, t), sn = sin(x);
    tab[o.sc + t] = sn;
    tab[o.cc + t] = cos(x);
    tab[o.s2c + t] = __dmul_rn(sn, sn);
    tab[o.gC + t] = p.coord == GMUNU_SPH ? __ddiv_rn(__dsub_rn(sin(xf(1, t + 1)), sin(xf(1, t))), cv(1, t)) : 0.0;
  }
  if (t <= p.nt[1]) {
    const double sn = sin(xf(1, t));
    tab[o.s2f + t] = __dmul_rn(sn, sn);
  }
}

// Device address of the scratch on each device, taken once per device (the
// first call with that device current).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

int static_scratch(double **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return GMUNU_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return GMUNU_EINVAL;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return GMUNU_EHIP;
    g_scratch[dev] = static_cast<double *>(ptr);
  }
  *out = g_scratch[dev];
  return GMUNU_OK;
}

}  // namespace

extern "C" {

int gmunu_step_static(const gmunu_grid_desc *desc, double *q_n, double *q_s, double *prim, const double *metric,
                      const double *kij, double cfl, double t_end, double *t_dev, double *dt_dev, uint8_t *flags,
                      unsigned int *nfatal_dev, void *stream) {
  if (!desc || !q_n || !q_s || !prim || !metric || !t_dev || !dt_dev) return GMUNU_ENULL;
  if (!aligned8(q_n) || !aligned8(q_s) || !aligned8(prim) || !aligned8(metric) || !aligned8(kij) ||
      !aligned8(t_dev) || !aligned8(dt_dev))
    return GMUNU_EALIGN;
  int rc = validate_desc(*desc);
  if (rc) return rc;
  // the limiter's middle SSPRK3 stage needs a third state, which a context
  // would hold
  if (desc->pp_limiter) return GMUNU_EINVAL;
  if (!(cfl > 0.0)) return GMUNU_EINVAL;
  // a context on the stack: its vectors stay empty (no allocation)
  gmunu_ctx ctx;
  ctx.d = *desc;
  ctx.prof = 0;
  ctx.nrec = 0;
  ctx.qt = nullptr;
  ctx.c2pmax = nullptr;
  ctx.rghosts = recovery_ghosts(*desc, &ctx.raxes);
  grid_scalars(*desc, ctx.G);
  for (int a = 0; a < 3; a++)
    if (ctx.G.nt[a] > kStaticAxis) return GMUNU_EINVAL;  // beyond the scratch's tables
  double *sp = nullptr;
  rc = static_scratch(&sp);
  if (rc) return rc;
  size_t words = 0;
  const GeoOffsets off = geo_layout(ctx.G.nt, words);
  if (words > kStaticGeo) return GMUNU_EINVAL;
  ctx.geo = sp;
  ctx.acc = sp + kStaticGeo;
  if (hipGetDevice(&ctx.device) != hipSuccess) return GMUNU_EHIP;
  bind_geo(ctx.G, ctx.geo, off);
  GeoParams gp;
  gp.coord = desc->coord;
  for (int a = 0; a < 3; a++) {
    gp.nt[a] = ctx.G.nt[a];
    gp.g[a] = ctx.G.g[a];
    gp.xmin[a] = desc->xmin[a];
    gp.dx[a] = desc->dx[a];
  }
  int len = 0;
  for (int a = 0; a < 3; a++) len = ctx.G.nt[a] + 1 > len ? ctx.G.nt[a] + 1 : len;
  hipLaunchKernelGGL(k_geo, dim3(nblocks(len)), dim3(NT), 0, as_stream(stream), gp, ctx.geo, off);
  rc = launch_status();
  if (rc) return rc;
  return step_impl(&ctx, q_n, q_s, prim, metric, kij, cfl, t_end, t_dev, dt_dev, flags, nfatal_dev, stream);
}

}  // extern "C"
