// Batched stage for many independent grids ("blocks") on one GPU.
//
// Work is cut into uniform items: a stage item is one tile (at most 256
// cells) of one block, a recovery / CFL item is 256 interior cells of one
// block, a ghost item 256 ghost cells.  Persistent kernels walk the item
// lists; each XCD takes one contiguous run of items so that the tiles of a
// block share that XCD's L2.  Item counts, block records and group times
// live in device memory, so a step captured into a HIP graph stays valid
// when blocks are added or removed between steps.  Per-cell arithmetic is
// the single-grid path's (gmunu_tile.hpp): a block advanced here is bitwise
// equal to the same block advanced alone, whatever tile shape is used.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/gmunu.h"
#include "gmunu_dev.hpp"
#include "gmunu_host.hpp"
#include "gmunu_tile.hpp"

using namespace gm;

namespace {

struct BlockRec {
  Grid G;
  double *qn, *qs, *prim;
  const double *met;
  uint8_t *flags;
  int group;
  int active;
};

// Compiled tile shapes (all 256 threads).
struct Variant {
  int tx, ty, tz, nd;
};
constexpr int NVAR = 8;
constexpr Variant kVar[NVAR] = {{8, 8, 4, 3},  {16, 4, 4, 3}, {32, 4, 2, 3}, {8, 4, 8, 3},
                                {32, 8, 1, 2}, {16, 16, 1, 2}, {64, 4, 1, 2}, {256, 1, 1, 1}};
enum { L_C2P = NVAR, L_GH = NVAR + 1, L_CFL = NVAR + 2, L_IC2P = NVAR + 3, L_IGH = NVAR + 4, NLIST = NVAR + 5 };

// Item range of this workgroup: a contiguous share of the list per XCD
// (workgroups are dispatched round-robin over the eight XCDs).
__device__ __forceinline__ void xcd_range(int n, int &first, int &end, int &stride) {
  const int G = gridDim.x, x = blockIdx.x % 8, l = blockIdx.x / 8;
  const int gx = (G - x + 7) / 8;
  const int lo = (int)((long)n * x / 8), hi = (int)((long)n * (x + 1) / 8);
  first = lo + l;
  end = hi;
  stride = gx;
}

template <int TX, int TY, int TZ, int ND, int MODE>
__global__ __launch_bounds__(TX *TY *TZ, 3) void k_bstage(const BlockRec *__restrict__ B,
                                                          const int4 *__restrict__ items,
                                                          const int *__restrict__ count, const double *dts,
                                                          double ca, double cb, int out_qn) {
  __shared__ double sF[NV * max_faces<TX, TY, TZ, ND>()];
  int it, end, stride;
  xcd_range(*count, it, end, stride);
  for (; it < end; it += stride) {
    const int4 w = items[it];
    const BlockRec &b = B[w.x];
    const double *dtp = dts + b.group;
    if (MODE == 1 && *dtp == 0.0) continue;
    double *out = (MODE == 0 || !out_qn) ? b.qs : b.qn;
    stage_tile<TX, TY, TZ, ND, MODE>(b.G, w.y, w.z, w.w, b.prim, b.met, b.qn, b.qs, out, dtp, ca, cb, sF);
  }
}

// Recovery on 256-cell items: from q_n (use_qn) or q_s.  force: ignore dt.
__global__ __launch_bounds__(NT) void k_bc2p(const BlockRec *__restrict__ B, const int2 *__restrict__ items,
                                             const int *__restrict__ count, const double *dts, int use_qn,
                                             int force, unsigned int *nfatal) {
  const int n = *count;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int2 w = items[it];
    const BlockRec &b = B[w.x];
    if (!force && dts[b.group] == 0.0) continue;
    const long t = (long)w.y + threadIdx.x;
    if (t < interior_count(b.G)) c2p_one(b.G, use_qn ? b.qn : b.qs, b.met, b.prim, b.flags, nfatal, t);
  }
}

__global__ __launch_bounds__(NT) void k_bprim2con(const BlockRec *__restrict__ B, const int2 *__restrict__ items,
                                                  const int *__restrict__ count) {
  const int n = *count;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int2 w = items[it];
    const BlockRec &b = B[w.x];
    const long t = (long)w.y + threadIdx.x;
    if (t < interior_count(b.G)) {
      const int i = (int)(t % b.G.n[0]), j = (int)((t / b.G.n[0]) % b.G.n[1]);
      const int k = (int)(t / ((long)b.G.n[0] * b.G.n[1]));
      prim2con_one(b.G, b.prim, b.met, b.qn, cell_offset(b.G, i, j, k));
    }
  }
}

__global__ __launch_bounds__(NT) void k_bghosts(const BlockRec *__restrict__ B, const int2 *__restrict__ items,
                                                const int *__restrict__ count, const double *dts, int force) {
  const int n = *count;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int2 w = items[it];
    const BlockRec &b = B[w.x];
    if (!force && dts[b.group] == 0.0) continue;
    const long t = (long)w.y + threadIdx.x;
    if (t < ghost_count(b.G)) ghost_one(b.G, b.prim, t);
  }
}

// Per-item maxima of the CFL rate (items ordered by group).
__global__ __launch_bounds__(NT) void k_bcfl(const BlockRec *__restrict__ B, const int2 *__restrict__ items,
                                             const int *__restrict__ count, double *part) {
  const int n = *count;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int2 w = items[it];
    const BlockRec &b = B[w.x];
    const long t = (long)w.y + threadIdx.x;
    const double r = t < interior_count(b.G) ? cfl_one(b.G, b.prim, b.met, t) : 0.0;
    const double m = block_max(r);
    if (threadIdx.x == 0) part[it] = m;
  }
}

// dt of each group: cfl / max rate over its items, capped at t_end - t,
// zero for a group without blocks or past its end.
__global__ __launch_bounds__(NT) void k_bcfl_finish(const int *__restrict__ gfirst, const int *__restrict__ gcount,
                                                    const double *__restrict__ part, int ngroups, double cfl,
                                                    const double *t, const double *t_end, double *dt) {
  for (int g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const int f = gfirst[g], c = gcount[g];
    double m = 0.0;
    for (int k = threadIdx.x; k < c; k += NT) m = fmax(m, part[f + k]);
    m = block_max(m);
    if (threadIdx.x == 0) {
      const double d = c > 0 ? dt_from_rate(m, cfl, t[g], t_end[g]) : 0.0;
      dt[g] = d > 0.0 ? d : 0.0;
    }
  }
}

__global__ void k_badvance(double *t, const double *dt, int ngroups) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < ngroups) t[g] += dt[g];
}

template <int V, int MODE>
void launch_variant(const BlockRec *B, const int4 *items, const int *count, const double *dts, double ca, double cb,
                    int out_qn, int grid, hipStream_t st) {
  constexpr Variant v = kVar[V];
  hipLaunchKernelGGL((k_bstage<v.tx, v.ty, v.tz, v.nd, MODE>), dim3(grid), dim3(NT), 0, st, B, items, count, dts, ca,
                     cb, out_qn);
}

template <int MODE>
void launch_variant_any(int v, const BlockRec *B, const int4 *items, const int *count, const double *dts, double ca,
                        double cb, int out_qn, int grid, hipStream_t st) {
  switch (v) {
    case 0: launch_variant<0, MODE>(B, items, count, dts, ca, cb, out_qn, grid, st); break;
    case 1: launch_variant<1, MODE>(B, items, count, dts, ca, cb, out_qn, grid, st); break;
    case 2: launch_variant<2, MODE>(B, items, count, dts, ca, cb, out_qn, grid, st); break;
    case 3: launch_variant<3, MODE>(B, items, count, dts, ca, cb, out_qn, grid, st); break;
    case 4: launch_variant<4, MODE>(B, items, count, dts, ca, cb, out_qn, grid, st); break;
    case 5: launch_variant<5, MODE>(B, items, count, dts, ca, cb, out_qn, grid, st); break;
    case 6: launch_variant<6, MODE>(B, items, count, dts, ca, cb, out_qn, grid, st); break;
    default: launch_variant<7, MODE>(B, items, count, dts, ca, cb, out_qn, grid, st); break;
  }
}

// Default tile for a block before (or without) tuning.
int default_variant(const gmunu_grid_desc &d) {
  if (d.ndim == 1) return 7;
  if (d.ndim == 2) return 4;
  return (d.n[0] <= 8 || d.n[1] <= 4) ? 0 : 1;
}

std::tuple<int, int, int, int> bucket_of(const gmunu_grid_desc &d) { return {d.ndim, d.n[0], d.n[1], d.n[2]}; }

}  // namespace

struct gmunu_batch {
  int maxb, maxg;
  long maxi;
  int ncu;
  std::vector<gmunu_block> blk;
  std::vector<char> used;
  std::vector<BlockRec> rec;
  std::vector<double *> geo;
  std::vector<int> var;
  std::map<std::tuple<int, int, int, int>, int> tuned;
  std::vector<std::pair<int, std::pair<double, double>>> time_set;
  long counts[NLIST];
  unsigned var_mask;
  // device tables
  BlockRec *d_rec;
  int4 *d_items[NVAR];
  int2 *d_list[5];  // c2p, ghosts, cfl, and the c2p / ghost items of an init
  int *d_count;
  int *d_gfirst, *d_gcount;
  double *d_part, *d_t, *d_dt, *d_tend;
  // captured step, replayed on a private stream ordered against the
  // caller's stream by events (capture is not possible on the null stream)
  hipStream_t pstream;
  hipEvent_t ev_in, ev_out;
  bool have_stream;
  hipGraphExec_t exec;
  bool have_graph;
  double graph_cfl;
  unsigned graph_mask;
  unsigned int *graph_nfatal;
};

namespace {

void free_batch(gmunu_batch *b) {
  if (b->have_graph) (void)hipGraphExecDestroy(b->exec);
  if (b->have_stream) {
    (void)hipStreamDestroy(b->pstream);
    (void)hipEventDestroy(b->ev_in);
    (void)hipEventDestroy(b->ev_out);
  }
  for (auto g : b->geo)
    if (g) (void)hipFree(g);
  (void)hipFree(b->d_rec);
  for (int v = 0; v < NVAR; v++) (void)hipFree(b->d_items[v]);
  for (int l = 0; l < 5; l++) (void)hipFree(b->d_list[l]);
  (void)hipFree(b->d_count);
  (void)hipFree(b->d_gfirst);
  (void)hipFree(b->d_gcount);
  (void)hipFree(b->d_part);
  (void)hipFree(b->d_t);
  (void)hipFree(b->d_dt);
  (void)hipFree(b->d_tend);
  delete b;
}

int persist_grid(const gmunu_batch *b, long items, int per_cu) {
  const long g = (long)b->ncu * per_cu;
  return (int)std::max(1L, std::min(g, std::max(items, 1L)));
}

// Enqueue one full step (cfl, stages, advance) on st.
int enqueue_step(gmunu_batch *b, double cfl, unsigned int *nfatal, hipStream_t st) {
  const int gsm = persist_grid(b, b->maxi, 8);
  const int gst = b->ncu * 4;
  hipLaunchKernelGGL(k_bcfl, dim3(gsm), dim3(NT), 0, st, b->d_rec, b->d_list[2], b->d_count + L_CFL, b->d_part);
  hipLaunchKernelGGL(k_bcfl_finish, dim3(std::min(b->maxg, 4096)), dim3(NT), 0, st, b->d_gfirst, b->d_gcount,
                     b->d_part, b->maxg, cfl, b->d_t, b->d_tend, b->d_dt);
  // RK stages (same coefficients as gmunu_rk_stage); blocks of a batch may
  // mix SSPRK2 and SSPRK3 only by group, so use the first block's choice
  int nst = 3;
  for (size_t s = 0; s < b->blk.size(); s++)
    if (b->used[s]) {
      nst = b->blk[s].desc.rk;
      break;
    }
  for (int s = 0; s < nst; s++) {
    double ca = 0.0, cb = 1.0;
    if (s > 0) {
      if (nst == 2) {
        ca = 0.5;
        cb = 0.5;
      } else if (s == 1) {
        ca = 0.75;
        cb = 0.25;
      } else {
        ca = 1.0 / 3.0;
        cb = 2.0 / 3.0;
      }
    }
    const int last = s == nst - 1;
    for (int v = 0; v < NVAR; v++)
      if (b->var_mask & (1u << v))
        launch_variant_any<1>(v, b->d_rec, b->d_items[v], b->d_count + v, b->d_dt, ca, cb, last, gst, st);
    hipLaunchKernelGGL(k_bc2p, dim3(gsm), dim3(NT), 0, st, b->d_rec, b->d_list[0], b->d_count + L_C2P, b->d_dt,
                       last, 0, nfatal);
    hipLaunchKernelGGL(k_bghosts, dim3(gsm), dim3(NT), 0, st, b->d_rec, b->d_list[1], b->d_count + L_GH, b->d_dt, 0);
  }
  hipLaunchKernelGGL(k_badvance, dim3((b->maxg + NT - 1) / NT), dim3(NT), 0, st, b->d_t, b->d_dt, b->maxg);
  return launch_status();
}

}  // namespace

extern "C" {

int gmunu_batch_create(int max_blocks, int max_groups, long max_items, gmunu_batch **out) {
  if (!out) return GMUNU_ENULL;
  if (max_blocks < 1 || max_groups < 1 || max_items < 1 || max_items > (1L << 30)) return GMUNU_EINVAL;
  gmunu_batch *b = new (std::nothrow) gmunu_batch();
  if (!b) return GMUNU_ENOMEM;
  b->maxb = max_blocks;
  b->maxg = max_groups;
  b->maxi = max_items;
  b->blk.resize(max_blocks);
  b->used.assign(max_blocks, 0);
  b->rec.resize(max_blocks);
  std::memset(b->rec.data(), 0, sizeof(BlockRec) * max_blocks);
  b->geo.assign(max_blocks, nullptr);
  b->var.assign(max_blocks, -1);
  for (long &c : b->counts) c = 0;
  b->var_mask = 0;
  b->have_graph = false;
  b->have_stream = false;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess) {
    delete b;
    return GMUNU_EHIP;
  }
  bool ok = hipMalloc(&b->d_rec, sizeof(BlockRec) * max_blocks) == hipSuccess;
  for (int v = 0; v < NVAR; v++) ok = ok && hipMalloc(&b->d_items[v], sizeof(int4) * max_items) == hipSuccess;
  for (int l = 0; l < 5; l++) ok = ok && hipMalloc(&b->d_list[l], sizeof(int2) * max_items) == hipSuccess;
  ok = ok && hipMalloc(&b->d_count, sizeof(int) * NLIST) == hipSuccess;
  ok = ok && hipMalloc(&b->d_gfirst, sizeof(int) * max_groups) == hipSuccess;
  ok = ok && hipMalloc(&b->d_gcount, sizeof(int) * max_groups) == hipSuccess;
  ok = ok && hipMalloc(&b->d_part, sizeof(double) * max_items) == hipSuccess;
  ok = ok && hipMalloc(&b->d_t, sizeof(double) * max_groups) == hipSuccess;
  ok = ok && hipMalloc(&b->d_dt, sizeof(double) * max_groups) == hipSuccess;
  ok = ok && hipMalloc(&b->d_tend, sizeof(double) * max_groups) == hipSuccess;
  if (!ok) {
    free_batch(b);
    return GMUNU_ENOMEM;
  }
  ok = hipMemset(b->d_rec, 0, sizeof(BlockRec) * max_blocks) == hipSuccess &&
       hipMemset(b->d_count, 0, sizeof(int) * NLIST) == hipSuccess &&
       hipMemset(b->d_gcount, 0, sizeof(int) * max_groups) == hipSuccess &&
       hipMemset(b->d_gfirst, 0, sizeof(int) * max_groups) == hipSuccess &&
       hipMemset(b->d_t, 0, sizeof(double) * max_groups) == hipSuccess &&
       hipMemset(b->d_dt, 0, sizeof(double) * max_groups) == hipSuccess &&
       hipMemset(b->d_tend, 0, sizeof(double) * max_groups) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    free_batch(b);
    return GMUNU_EHIP;
  }
  if (hipStreamCreateWithFlags(&b->pstream, hipStreamNonBlocking) != hipSuccess) {
    free_batch(b);
    return GMUNU_EHIP;
  }
  if (hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess) {
    (void)hipStreamDestroy(b->pstream);
    free_batch(b);
    return GMUNU_EHIP;
  }
  if (hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess) {
    (void)hipStreamDestroy(b->pstream);
    (void)hipEventDestroy(b->ev_in);
    free_batch(b);
    return GMUNU_EHIP;
  }
  b->have_stream = true;
  *out = b;
  return GMUNU_OK;
}

int gmunu_batch_destroy(gmunu_batch *b) {
  if (!b) return GMUNU_ENULL;
  free_batch(b);
  return GMUNU_OK;
}

int gmunu_batch_set_block(gmunu_batch *b, int slot, const gmunu_block *blk) {
  if (!b || !blk) return GMUNU_ENULL;
  if (slot < 0 || slot >= b->maxb || blk->group < 0 || blk->group >= b->maxg) return GMUNU_EINVAL;
  const int rc = validate_desc(blk->desc);
  if (rc) return rc;
  if (!blk->q_n || !blk->q_s || !blk->prim || !blk->metric) return GMUNU_ENULL;
  if (!aligned8(blk->q_n) || !aligned8(blk->q_s) || !aligned8(blk->prim) || !aligned8(blk->metric))
    return GMUNU_EALIGN;
  std::vector<double> tab;
  BlockRec r;
  std::memset(&r, 0, sizeof(r));
  const GeoOffsets off = setup_grid(blk->desc, r.G, tab);
  double *g = nullptr;
  if (hipMalloc(&g, tab.size() * sizeof(double)) != hipSuccess) return GMUNU_ENOMEM;
  if (hipMemcpy(g, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(g);
    return GMUNU_EHIP;
  }
  bind_geo(r.G, g, off);
  r.qn = blk->q_n;
  r.qs = blk->q_s;
  r.prim = blk->prim;
  r.met = blk->metric;
  r.flags = blk->flags;
  r.group = blk->group;
  r.active = 1;
  if (b->geo[slot]) (void)hipFree(b->geo[slot]);
  b->geo[slot] = g;
  b->rec[slot] = r;
  b->blk[slot] = *blk;
  b->used[slot] = 1;
  auto it = b->tuned.find(bucket_of(blk->desc));
  b->var[slot] = it != b->tuned.end() ? it->second : default_variant(blk->desc);
  return GMUNU_OK;
}

int gmunu_batch_clear_block(gmunu_batch *b, int slot) {
  if (!b) return GMUNU_ENULL;
  if (slot < 0 || slot >= b->maxb) return GMUNU_EINVAL;
  b->used[slot] = 0;
  b->rec[slot].active = 0;
  b->var[slot] = -1;
  return GMUNU_OK;
}

int gmunu_batch_set_group(gmunu_batch *b, int group, double t, double t_end) {
  if (!b) return GMUNU_ENULL;
  if (group < 0 || group >= b->maxg || !(t_end >= t)) return GMUNU_EINVAL;
  b->time_set.push_back({group, {t, t_end}});
  return GMUNU_OK;
}

int gmunu_batch_commit(gmunu_batch *b, void *stream) {
  if (!b) return GMUNU_ENULL;
  hipStream_t st = as_stream(stream);
  int rk = 0;
  for (int s = 0; s < b->maxb; s++)
    if (b->used[s]) {
      if (rk && b->blk[s].desc.rk != rk) return GMUNU_EINVAL;  // one integrator per batch
      rk = b->blk[s].desc.rk;
    }
  std::vector<int4> items[NVAR];
  std::vector<int2> lc2p, lgh;
  std::vector<std::vector<int2>> cfl_by_group(b->maxg);
  for (int s = 0; s < b->maxb; s++) {
    if (!b->used[s]) continue;
    const Grid &G = b->rec[s].G;
    const Variant v = kVar[b->var[s]];
    for (int k0 = 0; k0 < G.n[2]; k0 += v.tz)
      for (int j0 = 0; j0 < G.n[1]; j0 += v.ty)
        for (int i0 = 0; i0 < G.n[0]; i0 += v.tx) items[b->var[s]].push_back(make_int4(s, i0, j0, k0));
    const long nin = interior_cells(G), ngh = ghost_total(G);
    for (long f = 0; f < nin; f += NT) {
      lc2p.push_back(make_int2(s, (int)f));
      cfl_by_group[b->rec[s].group].push_back(make_int2(s, (int)f));
    }
    for (long f = 0; f < ngh; f += NT) lgh.push_back(make_int2(s, (int)f));
  }
  std::vector<int2> lcfl;
  std::vector<int> gfirst(b->maxg), gcount(b->maxg);
  for (int g = 0; g < b->maxg; g++) {
    gfirst[g] = (int)lcfl.size();
    gcount[g] = (int)cfl_by_group[g].size();
    lcfl.insert(lcfl.end(), cfl_by_group[g].begin(), cfl_by_group[g].end());
  }
  int cnt[NLIST];
  unsigned mask = 0;
  for (int v = 0; v < NVAR; v++) {
    if ((long)items[v].size() > b->maxi) return GMUNU_EINVAL;
    cnt[v] = (int)items[v].size();
    if (cnt[v]) mask |= 1u << v;
  }
  if ((long)lc2p.size() > b->maxi || (long)lgh.size() > b->maxi) return GMUNU_EINVAL;
  cnt[L_C2P] = (int)lc2p.size();
  cnt[L_GH] = (int)lgh.size();
  cnt[L_CFL] = (int)lcfl.size();
  bool ok = hipMemcpyAsync(b->d_rec, b->rec.data(), sizeof(BlockRec) * b->maxb, hipMemcpyHostToDevice, st) ==
            hipSuccess;
  for (int v = 0; v < NVAR; v++)
    if (cnt[v])
      ok = ok && hipMemcpyAsync(b->d_items[v], items[v].data(), sizeof(int4) * cnt[v], hipMemcpyHostToDevice, st) ==
                     hipSuccess;
  if (cnt[L_C2P])
    ok = ok && hipMemcpyAsync(b->d_list[0], lc2p.data(), sizeof(int2) * cnt[L_C2P], hipMemcpyHostToDevice, st) ==
                   hipSuccess;
  if (cnt[L_GH])
    ok = ok &&
         hipMemcpyAsync(b->d_list[1], lgh.data(), sizeof(int2) * cnt[L_GH], hipMemcpyHostToDevice, st) == hipSuccess;
  if (cnt[L_CFL])
    ok = ok && hipMemcpyAsync(b->d_list[2], lcfl.data(), sizeof(int2) * cnt[L_CFL], hipMemcpyHostToDevice, st) ==
                   hipSuccess;
  ok = ok && hipMemcpyAsync(b->d_gfirst, gfirst.data(), sizeof(int) * b->maxg, hipMemcpyHostToDevice, st) == hipSuccess;
  ok = ok && hipMemcpyAsync(b->d_gcount, gcount.data(), sizeof(int) * b->maxg, hipMemcpyHostToDevice, st) == hipSuccess;
  ok = ok && hipMemcpyAsync(b->d_count, cnt, sizeof(int) * L_IC2P, hipMemcpyHostToDevice, st) == hipSuccess;
  for (auto &ts : b->time_set) {
    ok = ok && hipMemcpyAsync(b->d_t + ts.first, &ts.second.first, sizeof(double), hipMemcpyHostToDevice, st) ==
                   hipSuccess;
    ok = ok && hipMemcpyAsync(b->d_tend + ts.first, &ts.second.second, sizeof(double), hipMemcpyHostToDevice, st) ==
                   hipSuccess;
  }
  ok = ok && hipStreamSynchronize(st) == hipSuccess;
  b->time_set.clear();
  if (!ok) return GMUNU_EHIP;
  for (int l = 0; l < L_IC2P; l++) b->counts[l] = cnt[l];
  b->var_mask = mask;
  return GMUNU_OK;
}

int gmunu_batch_init(gmunu_batch *b, const int *slots, int nslots, void *stream) {
  if (!b) return GMUNU_ENULL;
  hipStream_t st = as_stream(stream);
  // recovery and ghost items of the selected committed slots only
  std::vector<char> sel(b->maxb, slots ? 0 : 1);
  if (slots)
    for (int k = 0; k < nslots; k++) {
      if (slots[k] < 0 || slots[k] >= b->maxb) return GMUNU_EINVAL;
      sel[slots[k]] = 1;
    }
  std::vector<int2> lc, lg;
  for (int s = 0; s < b->maxb; s++) {
    if (!b->used[s] || !sel[s]) continue;
    const Grid &G = b->rec[s].G;
    for (long f = 0; f < interior_cells(G); f += NT) lc.push_back(make_int2(s, (int)f));
    for (long f = 0; f < ghost_total(G); f += NT) lg.push_back(make_int2(s, (int)f));
  }
  if ((long)lc.size() > b->maxi || (long)lg.size() > b->maxi) return GMUNU_EINVAL;
  const int cnt[2] = {(int)lc.size(), (int)lg.size()};
  bool ok = true;
  if (cnt[0])
    ok = hipMemcpyAsync(b->d_list[3], lc.data(), sizeof(int2) * cnt[0], hipMemcpyHostToDevice, st) == hipSuccess;
  if (cnt[1])
    ok = ok && hipMemcpyAsync(b->d_list[4], lg.data(), sizeof(int2) * cnt[1], hipMemcpyHostToDevice, st) == hipSuccess;
  ok = ok && hipMemcpyAsync(b->d_count + L_IC2P, cnt, sizeof(int) * 2, hipMemcpyHostToDevice, st) == hipSuccess;
  ok = ok && hipStreamSynchronize(st) == hipSuccess;
  if (!ok) return GMUNU_EHIP;
  const int gsm = persist_grid(b, b->maxi, 8);
  hipLaunchKernelGGL(k_bghosts, dim3(gsm), dim3(NT), 0, st, b->d_rec, b->d_list[4], b->d_count + L_IGH, b->d_dt, 1);
  hipLaunchKernelGGL(k_bprim2con, dim3(gsm), dim3(NT), 0, st, b->d_rec, b->d_list[3], b->d_count + L_IC2P);
  hipLaunchKernelGGL(k_bc2p, dim3(gsm), dim3(NT), 0, st, b->d_rec, b->d_list[3], b->d_count + L_IC2P, b->d_dt, 1, 1,
                     (unsigned int *)nullptr);
  hipLaunchKernelGGL(k_bghosts, dim3(gsm), dim3(NT), 0, st, b->d_rec, b->d_list[4], b->d_count + L_IGH, b->d_dt, 1);
  return launch_status();
}

int gmunu_batch_autotune(gmunu_batch *b, void *stream) {
  if (!b) return GMUNU_ENULL;
  hipStream_t st = as_stream(stream);
  std::map<std::tuple<int, int, int, int>, std::vector<int>> buckets;
  for (int s = 0; s < b->maxb; s++)
    if (b->used[s]) buckets[bucket_of(b->blk[s].desc)].push_back(s);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return GMUNU_EHIP;
  const std::vector<int> saved = b->var;
  int rc = GMUNU_OK;
  for (auto &bk : buckets) {
    const int nd = std::get<0>(bk.first);
    int best = -1;
    float best_ms = 0.f;
    for (int v = 0; v < NVAR; v++) {
      if (kVar[v].nd != nd) continue;
      // only this bucket's blocks, all on variant v
      for (int s = 0; s < b->maxb; s++)
        if (b->used[s]) b->var[s] = -2;
      for (int s : bk.second) b->var[s] = v;
      std::vector<int4> items;
      for (int s : bk.second) {
        const Grid &G = b->rec[s].G;
        for (int k0 = 0; k0 < G.n[2]; k0 += kVar[v].tz)
          for (int j0 = 0; j0 < G.n[1]; j0 += kVar[v].ty)
            for (int i0 = 0; i0 < G.n[0]; i0 += kVar[v].tx) items.push_back(make_int4(s, i0, j0, k0));
      }
      if ((long)items.size() > b->maxi) continue;
      const int n = (int)items.size();
      if (hipMemcpyAsync(b->d_items[v], items.data(), sizeof(int4) * n, hipMemcpyHostToDevice, st) != hipSuccess ||
          hipMemcpyAsync(b->d_count + v, &n, sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess ||
          hipMemcpyAsync(b->d_rec, b->rec.data(), sizeof(BlockRec) * b->maxb, hipMemcpyHostToDevice, st) !=
              hipSuccess) {
        rc = GMUNU_EHIP;
        break;
      }
      const int gst = b->ncu * 4;
      launch_variant_any<0>(v, b->d_rec, b->d_items[v], b->d_count + v, b->d_dt, 0.0, 1.0, 0, gst, st);  // warm-up
      (void)hipEventRecord(e0, st);
      for (int r = 0; r < 3; r++)
        launch_variant_any<0>(v, b->d_rec, b->d_items[v], b->d_count + v, b->d_dt, 0.0, 1.0, 0, gst, st);
      (void)hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess) {
        rc = GMUNU_EHIP;
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (best < 0 || ms < best_ms) {
        best = v;
        best_ms = ms;
      }
    }
    if (rc) break;
    if (best >= 0) b->tuned[bk.first] = best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->var = saved;
  if (rc) return rc;
  for (int s = 0; s < b->maxb; s++)
    if (b->used[s]) {
      auto it = b->tuned.find(bucket_of(b->blk[s].desc));
      if (it != b->tuned.end()) b->var[s] = it->second;
    }
  return gmunu_batch_commit(b, stream);
}

int gmunu_batch_step(gmunu_batch *b, double cfl, unsigned int *nfatal_dev, int use_graph, void *stream) {
  if (!b) return GMUNU_ENULL;
  if (!(cfl > 0.0)) return GMUNU_EINVAL;
  hipStream_t st = as_stream(stream);
  if (!use_graph) return enqueue_step(b, cfl, nfatal_dev, st);
  if (!b->have_graph || b->graph_cfl != cfl || b->graph_mask != b->var_mask || b->graph_nfatal != nfatal_dev) {
    if (b->have_graph) {
      (void)hipGraphExecDestroy(b->exec);
      b->have_graph = false;
    }
    hipGraph_t graph;
    if (hipStreamBeginCapture(b->pstream, hipStreamCaptureModeThreadLocal) != hipSuccess) return GMUNU_EHIP;
    const int rc = enqueue_step(b, cfl, nfatal_dev, b->pstream);
    const bool ended = hipStreamEndCapture(b->pstream, &graph) == hipSuccess;
    if (!ended || rc) {
      if (ended) (void)hipGraphDestroy(graph);
      return rc ? rc : GMUNU_EHIP;
    }
    const bool ok = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0) == hipSuccess;
    (void)hipGraphDestroy(graph);
    if (!ok) return GMUNU_EHIP;
    b->have_graph = true;
    b->graph_cfl = cfl;
    b->graph_mask = b->var_mask;
    b->graph_nfatal = nfatal_dev;
  }
  // order: caller's prior work -> replay on the private stream -> caller's later work
  bool ok = hipEventRecord(b->ev_in, st) == hipSuccess && hipStreamWaitEvent(b->pstream, b->ev_in, 0) == hipSuccess &&
            hipGraphLaunch(b->exec, b->pstream) == hipSuccess && hipEventRecord(b->ev_out, b->pstream) == hipSuccess &&
            hipStreamWaitEvent(st, b->ev_out, 0) == hipSuccess;
  return ok ? GMUNU_OK : GMUNU_EHIP;
}

int gmunu_batch_times(gmunu_batch *b, double *t_host, double *dt_host, void *stream) {
  if (!b) return GMUNU_ENULL;
  hipStream_t st = as_stream(stream);
  bool ok = true;
  if (t_host) ok = hipMemcpyAsync(t_host, b->d_t, sizeof(double) * b->maxg, hipMemcpyDeviceToHost, st) == hipSuccess;
  if (dt_host)
    ok = ok && hipMemcpyAsync(dt_host, b->d_dt, sizeof(double) * b->maxg, hipMemcpyDeviceToHost, st) == hipSuccess;
  ok = ok && hipStreamSynchronize(st) == hipSuccess;
  return ok ? GMUNU_OK : GMUNU_EHIP;
}

int gmunu_batch_info(gmunu_batch *b, long *items_out, int *out_variant) {
  if (!b) return GMUNU_ENULL;
  if (items_out) {
    long st = 0;
    for (int v = 0; v < NVAR; v++) st += b->counts[v];
    items_out[0] = st;
    items_out[1] = b->counts[L_C2P];
    items_out[2] = b->counts[L_GH];
  }
  if (out_variant)
    for (int s = 0; s < b->maxb; s++) out_variant[s] = b->used[s] ? b->var[s] : -1;
  return GMUNU_OK;
}

}  // extern "C"
