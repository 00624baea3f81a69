// Batched stage for many independent grids ("blocks") on one GPU.
//
// Work is cut into uniform items: a stage item is one tile (at most 256
// cells) of one block, a recovery / CFL item is 256 interior cells of one
// block, a ghost item 256 ghost cells.  Each work list is stored as a table
// of entries, one per block (the block's slot and the index of its first
// item); a workgroup finds the block of an item by search in that table and
// the tile from the item's rank inside the block.  Tables, block records and
// group times live in device memory, so a step captured into a HIP graph
// stays valid when blocks are added or removed, and a commit costs O(blocks)
// host work and upload.  Persistent kernels walk each list; each XCD takes
// one contiguous run of items so that the tiles of a block share that XCD's
// L2.  Per-cell arithmetic is the single-grid path's (gmunu_tile.hpp): a
// block advanced here is bitwise equal to the same block advanced alone,
// whatever tile shape is used.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/gmunu.h"
#include "batch_internal.hpp"
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
  // face ghosts of the first raxes axes (the first rghosts in ghost_one's
  // numbering) written by the recovery kernel of a step; the ghost kernel
  // fills the rest (recovery_ghosts)
  long rghosts;
  int raxes;
  int cfl_start;  // the block's first item in the CFL list (set at commit)
};

// Compiled tile shapes (256 threads; each pass has at most 256 faces) and
// reconstruction (GMUNU_RECON_*).
struct Variant {
  int tx, ty, tz, nd, rec;
};
constexpr int NVAR = 14;
constexpr Variant kVar[NVAR] = {{8, 8, 3, 3, 0},   {8, 5, 5, 3, 0},   {16, 4, 3, 3, 0}, {8, 6, 4, 3, 0},
                                {16, 15, 1, 2, 0}, {32, 7, 1, 2, 0},  {8, 28, 1, 2, 0}, {255, 1, 1, 1, 0},
                                {8, 5, 5, 3, 1},   {16, 15, 1, 2, 1}, {255, 1, 1, 1, 1}, {8, 5, 5, 3, 2},
                                {16, 15, 1, 2, 2}, {255, 1, 1, 1, 2}};
// Work lists: one per tile variant, then recovery, ghosts, CFL (entries
// ordered by group), and the recovery / ghost lists of an init.
// Stage lists: one per (tile variant, Riemann solver), list = variant +
// NVAR * riemann; then recovery, ghosts, CFL (entries ordered by group), and
// the recovery / ghost lists of an init.
constexpr int NSL = 2 * NVAR;
enum { L_C2P = NSL, L_GH, L_CFL, L_IC2P, L_IGH, NLIST };
static_assert(NSL <= kMaxVariants && NSL <= 32, "stage lists are counted in 32-bit masks and server counters");

// Entry table of one list on the device: blk[e] is the slot of entry e,
// start[e] the index of its first item (start[nent] = total), meta = {nent,
// total}.
struct DList {
  const int *blk, *start, *meta;
};

// Item range of this workgroup: a contiguous share of the list per XCD
// (workgroups are dispatched round-robin over the eight XCDs); a grid of
// fewer than eight workgroups strides over the whole list.
__device__ __forceinline__ void xcd_range(int n, int &first, int &end, int &stride) {
  if (gridDim.x < 8) {
    first = blockIdx.x;
    end = n;
    stride = gridDim.x;
    return;
  }
  const int G = gridDim.x, x = blockIdx.x % 8, l = blockIdx.x / 8;
  const int gx = (G - x + 7) / 8;
  const int lo = (int)((long)n * x / 8), hi = (int)((long)n * (x + 1) / 8);
  first = lo + l;
  end = hi;
  stride = gx;
}

// Entry holding item `it` (start[e] <= it < start[e+1]); e is the previous
// answer of this workgroup (items only increase) or -1.
__device__ __forceinline__ int find_entry(const int *start, int nent, int it, int e) {
  if (e >= 0 && it < start[e + 1]) return e;
  int lo = e < 0 ? 0 : e + 1, hi = nent - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= it)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <int TX, int TY, int TZ, int ND, int MODE, int REC, int R>
__global__ __launch_bounds__(NT, (stage_occupancy<TX, TY, TZ, ND, recon_halo(REC)>())) void k_bstage(const BlockRec *__restrict__ B, DList L,
                                                          const double *dts, double ca, double cb, int out_qn) {
  __shared__ double sF[stage_lds<TX, TY, TZ, ND, recon_halo(REC)>()];
  const int nent = L.meta[0];
  int it, end, stride;
  xcd_range(L.meta[1], it, end, stride);
  int e = -1;
  for (; it < end; it += stride) {
    e = find_entry(L.start, nent, it, e);
    const BlockRec &b = B[L.blk[e]];
    const double *dtp = dts + b.group;
    if (MODE == 1 && *dtp == 0.0) continue;
    const int l = it - L.start[e];
    const int gx = (b.G.n[0] + TX - 1) / TX, gy = (b.G.n[1] + TY - 1) / TY;
    const int i0 = (l % gx) * TX, j0 = ((l / gx) % gy) * TY, k0 = (l / (gx * gy)) * TZ;
    double *out = (MODE == 0 || !out_qn) ? b.qs : b.qn;
    stage_tile<TX, TY, TZ, ND, MODE, REC, R>(b.G, i0, j0, k0, b.prim, b.met, b.qn, b.qs, out, dtp, ca, cb, sF);
  }
}

// Recovery on 256-cell items: from q_n (use_qn) or q_s.  force: ignore dt.
// gfill: the thread that recovers a cell also writes the face ghosts of the
// block's first raxes axes copied from it (no barrier, no re-read).  part
// non-null (the last stage of a step followed by another step of the same
// launch sequence): the item's CFL rate maximum, from the primitives just
// recovered (nothing changes the interior primitives before the next step),
// at its place in the CFL list, so that the next step needs no CFL kernel.  Items skipped for dt = 0 write none:
// their group's dt stays 0 in the next step whatever its maxima.
__global__ __launch_bounds__(NT) void k_bc2p(const BlockRec *__restrict__ B, DList L, const double *dts, int use_qn,
                                             int force, unsigned int *nfatal, unsigned int *gfatal, int gfill,
                                             double *part) {
  const int nent = L.meta[0], n = L.meta[1];
  int e = -1;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    e = find_entry(L.start, nent, it, e);
    const BlockRec &b = B[L.blk[e]];
    if (!force && dts[b.group] == 0.0) continue;  // the same for the whole item
    const long t = (long)(it - L.start[e]) * NT + threadIdx.x;
    if (t < interior_count(b.G))
      c2p_one(b.G, use_qn ? b.qn : b.qs, b.met, b.prim, b.flags, nfatal, t, gfatal ? gfatal + b.group : nullptr,
              gfill ? b.raxes : 0);
    if (part) {
      const double r = t < interior_count(b.G) ? cfl_one(b.G, b.prim, b.met, t) : 0.0;
      const double m = block_max(r);
      if (threadIdx.x == 0) part[b.cfl_start + (it - L.start[e])] = m;
    }
  }
}

__global__ __launch_bounds__(NT) void k_bprim2con(const BlockRec *__restrict__ B, DList L) {
  const int nent = L.meta[0], n = L.meta[1];
  int e = -1;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    e = find_entry(L.start, nent, it, e);
    const BlockRec &b = B[L.blk[e]];
    const long t = (long)(it - L.start[e]) * NT + threadIdx.x;
    if (t < interior_count(b.G)) {
      const int i = (int)(t % b.G.n[0]), j = (int)((t / b.G.n[0]) % b.G.n[1]);
      const int k = (int)(t / ((long)b.G.n[0] * b.G.n[1]));
      prim2con_one(b.G, b.prim, b.met, b.qn, cell_offset(b.G, i, j, k));
    }
  }
}

// Ghost fill on 256-ghost items.  force: ignore dt, and fill every ghost
// (an init); otherwise a block's first rghosts ghosts (filled by the
// recovery kernel) are skipped.
__global__ __launch_bounds__(NT) void k_bghosts(const BlockRec *__restrict__ B, DList L, const double *dts,
                                                int force) {
  const int nent = L.meta[0], n = L.meta[1];
  int e = -1;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    e = find_entry(L.start, nent, it, e);
    const BlockRec &b = B[L.blk[e]];
    if (!force && dts[b.group] == 0.0) continue;
    const long t = (long)(it - L.start[e]) * NT + threadIdx.x + (force ? 0 : b.rghosts);
    if (t < ghost_count(b.G)) ghost_one(b.G, b.prim, t);
  }
}

// Per-item maxima of the CFL rate (entries ordered by group).
__global__ __launch_bounds__(NT) void k_bcfl(const BlockRec *__restrict__ B, DList L, double *part) {
  const int nent = L.meta[0], n = L.meta[1];
  int e = -1;
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    e = find_entry(L.start, nent, it, e);
    const BlockRec &b = B[L.blk[e]];
    const long t = (long)(it - L.start[e]) * NT + threadIdx.x;
    const double r = t < interior_count(b.G) ? cfl_one(b.G, b.prim, b.met, t) : 0.0;
    const double m = block_max(r);
    if (threadIdx.x == 0) part[it] = m;
  }
}

// dt of each group, one wavefront per group: cfl / max rate over its items,
// capped at t_end - t, zero for a group without blocks, past its end time or
// at its step limit.  A group with dt > 0 advances its time and step count
// here: nothing later in the step reads them.
__global__ __launch_bounds__(NT) void k_bcfl_finish(const int *__restrict__ gfirst, const int *__restrict__ gcount,
                                                    const double *__restrict__ part, int ngroups, double cfl,
                                                    double *t, const double *t_end, int *nstep, const int *maxstep,
                                                    double *dt) {
  const int g = blockIdx.x * (NT / 64) + (int)(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (g >= ngroups) return;  // uniform over the wavefront
  const int f = gfirst[g], c = gcount[g];
  double m = 0.0;
  for (int k = lane; k < c; k += 64) m = fmax(m, part[f + k]);
  m = wave_max(m);
  if (lane == 0) {
    const double d0 = (c > 0 && nstep[g] < maxstep[g]) ? dt_from_rate(m, cfl, t[g], t_end[g]) : 0.0;
    const double d = d0 > 0.0 ? d0 : 0.0;
    dt[g] = d;
    if (d > 0.0) {
      t[g] += d;
      nstep[g] += 1;
    }
  }
}

// Launch the stage kernel of list LI (variant LI % NVAR, Riemann solver
// LI / NVAR), or of the run-time list li by recursion over the lists.
template <int LI, int MODE>
void launch_list(const BlockRec *B, DList L, const double *dts, double ca, double cb, int out_qn, int grid,
                 hipStream_t st) {
  constexpr Variant v = kVar[LI % NVAR];
  hipLaunchKernelGGL((k_bstage<v.tx, v.ty, v.tz, v.nd, MODE, v.rec, LI / NVAR>), dim3(grid), dim3(NT), 0, st, B, L,
                     dts, ca, cb, out_qn);
}

template <int MODE, int LI = 0>
void launch_list_any(int li, const BlockRec *B, DList L, const double *dts, double ca, double cb, int out_qn,
                     int grid, hipStream_t st) {
  if constexpr (LI < NSL) {
    if (li == LI)
      launch_list<LI, MODE>(B, L, dts, ca, cb, out_qn, grid, st);
    else
      launch_list_any<MODE, LI + 1>(li, B, L, dts, ca, cb, out_qn, grid, st);
  }
}

// Default tile for a block before (or without) tuning.
int default_variant(const gmunu_grid_desc &d) {
  if (d.recon == GMUNU_RECON_MP5) return d.ndim == 1 ? 10 : d.ndim == 2 ? 9 : 8;
  if (d.recon == GMUNU_RECON_PPM) return d.ndim == 1 ? 13 : d.ndim == 2 ? 12 : 11;
  if (d.ndim == 1) return 7;
  if (d.ndim == 2) return 4;
  return d.n[0] <= 8 ? 0 : 1;
}


std::tuple<int, int, int, int, int, int> bucket_of(const gmunu_grid_desc &d) {
  return {d.ndim, d.n[0], d.n[1], d.n[2], d.recon, d.riemann};
}

int list_of(int variant, const gmunu_grid_desc &d) { return variant + NVAR * (d.riemann == GMUNU_RIEMANN_TVDLF); }

long ceil_div(long a, long b) { return (a + b - 1) / b; }

long stage_items(const gmunu_grid_desc &d, int v) {
  return ceil_div(d.n[0], kVar[v].tx) * ceil_div(d.n[1], kVar[v].ty) * ceil_div(d.n[2], kVar[v].tz);
}

long cell_items(const gmunu_grid_desc &d) { return ceil_div((long)d.n[0] * d.n[1] * d.n[2], NT); }

long ghost_cells(const gmunu_grid_desc &d) {
  const long nin = (long)d.n[0] * d.n[1] * d.n[2];
  long tot = 0;
  for (int a = 0; a < d.ndim; a++) tot += 2L * d.ng * (nin / d.n[a]);
  return tot;
}

// Items of the ghost list of a step (init: all ghosts).
long ghost_items(const gmunu_grid_desc &d) {
  int axes;
  return ceil_div(ghost_cells(d) - recovery_ghosts(d, &axes), NT);
}
long ghost_items_all(const gmunu_grid_desc &d) { return ceil_div(ghost_cells(d), NT); }

// Host copy of one list's entry table.
struct HList {
  std::vector<int> blk, start;
  long total = 0;
  void add(int slot, long items) {
    if (items <= 0) return;
    blk.push_back(slot);
    start.push_back((int)total);
    total += items;
  }
};

// Grid sizes of the kernels of one step: a persistent kernel gets about one
// workgroup per item of its list (a power of two, at most its cap), so that a
// step over a few small blocks does not launch thousands of idle workgroups.
struct Shape {
  int cfl = 1, c2p = 1, gh = 0;  // gh = 0: no ghost kernel (an empty ghost list)
  int st[NSL];
  Shape() {
    for (int &g : st) g = 1;
  }
};

int grid_for(long items, int cap) {
  int g = 1;
  while (g < items && g < cap) g <<= 1;
  return std::min(g, cap);
}

// A step captured with grids `have` serves lists that want `want` while no
// list outgrew its grid and none shrank below an eighth of a grid of more
// than 64 workgroups (any grid size gives the same results); a ghost list
// that emptied is still launched, empty.
bool shape_fits(const Shape &have, const Shape &want) {
  auto ok = [](int h, int w) { return w <= h && (8 * w > h || h <= 64); };
  if (!ok(have.cfl, want.cfl) || !ok(have.c2p, want.c2p)) return false;
  if (want.gh && !ok(have.gh, want.gh)) return false;
  for (int l = 0; l < NSL; l++)
    if (!ok(have.st[l], want.st[l])) return false;
  return true;
}

}  // namespace

struct gmunu_batch {
  int maxb, maxg;
  long maxi;
  int ncu;
  std::vector<gmunu_block> blk;
  std::vector<char> used;
  std::vector<BlockRec> rec;
  std::vector<double *> geo;  // per-slot geometry tables, grown, never shrunk
  std::vector<size_t> geo_cap;
  std::vector<int> var;
  std::map<std::tuple<int, int, int, int, int, int>, int> tuned;
  struct TimeSet {
    int group;
    double t, t_end;
    int max_steps;
  };
  std::vector<TimeSet> time_set;
  long counts[NLIST];
  unsigned var_mask;
  int rec_lo, rec_hi;  // slots whose records changed since the last upload
  // device tables
  BlockRec *d_rec;
  int *d_blk, *d_start, *d_meta;  // NLIST entry tables of maxb (+1) ints, meta 2 ints per list
  int *d_gfirst, *d_gcount;
  double *d_part, *d_t, *d_dt, *d_tend;
  int *d_nstep, *d_maxstep;
  unsigned int *d_gfatal;  // fatal recoveries per group since its set_group
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
  int graph_steps;
  Shape graph_shape;

  DList list(int l) const {
    return DList{d_blk + (size_t)l * maxb, d_start + (size_t)l * (maxb + 1), d_meta + 2 * l};
  }
  void touch(int s) {
    rec_lo = std::min(rec_lo, s);
    rec_hi = std::max(rec_hi, s + 1);
  }
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
  (void)hipFree(b->d_blk);
  (void)hipFree(b->d_start);
  (void)hipFree(b->d_meta);
  (void)hipFree(b->d_gfirst);
  (void)hipFree(b->d_gcount);
  (void)hipFree(b->d_part);
  (void)hipFree(b->d_t);
  (void)hipFree(b->d_dt);
  (void)hipFree(b->d_tend);
  (void)hipFree(b->d_nstep);
  (void)hipFree(b->d_maxstep);
  (void)hipFree(b->d_gfatal);
  delete b;
}

// Enqueue the upload of one list's entry table (host vectors must live until
// the stream is synchronised).
bool upload_list(gmunu_batch *b, int l, HList &h, int *meta_host, hipStream_t st) {
  const int nent = (int)h.blk.size();
  h.start.push_back((int)h.total);
  meta_host[0] = nent;
  meta_host[1] = (int)h.total;
  bool ok = true;
  if (nent) {
    ok = hipMemcpyAsync(b->d_blk + (size_t)l * b->maxb, h.blk.data(), sizeof(int) * nent, hipMemcpyHostToDevice,
                        st) == hipSuccess;
    ok = ok && hipMemcpyAsync(b->d_start + (size_t)l * (b->maxb + 1), h.start.data(), sizeof(int) * (nent + 1),
                              hipMemcpyHostToDevice, st) == hipSuccess;
  }
  return ok && hipMemcpyAsync(b->d_meta + 2 * l, meta_host, sizeof(int) * 2, hipMemcpyHostToDevice, st) == hipSuccess;
}

bool upload_records(gmunu_batch *b, hipStream_t st) {
  if (b->rec_hi <= b->rec_lo) return true;
  const bool ok = hipMemcpyAsync(b->d_rec + b->rec_lo, b->rec.data() + b->rec_lo,
                                 sizeof(BlockRec) * (b->rec_hi - b->rec_lo), hipMemcpyHostToDevice, st) == hipSuccess;
  b->rec_lo = INT_MAX;
  b->rec_hi = 0;
  return ok;
}

// Grids for the lists as last committed.  The caps keep each workgroup of a
// large list to a few items, so that workgroups retire often and kernels of
// other batches on the device (other streams) find free compute units.
constexpr int kGridPerCu = 16;

Shape step_shape(const gmunu_batch *b) {
  const int cap = kGridPerCu * b->ncu;
  Shape sh;
  sh.cfl = grid_for(b->counts[L_CFL], cap);
  sh.c2p = grid_for(b->counts[L_C2P], cap);
  sh.gh = b->counts[L_GH] ? grid_for(b->counts[L_GH], cap) : 0;
  for (int l = 0; l < NSL; l++) sh.st[l] = grid_for(b->counts[l], cap);
  return sh;
}

// Grids to capture for lists that want `w`: room to grow to twice the work
// (at least 64 workgroups) before the next capture.
Shape with_headroom(const gmunu_batch *b, const Shape &w) {
  const int cap = kGridPerCu * b->ncu;
  auto up = [cap](int g) { return std::min(cap, std::max(64, 2 * g)); };
  Shape sh;
  sh.cfl = up(w.cfl);
  sh.c2p = up(w.c2p);
  sh.gh = w.gh ? up(w.gh) : 0;
  for (int l = 0; l < NSL; l++) sh.st[l] = up(w.st[l]);
  return sh;
}

// Enqueue `steps` full steps (CFL and advance, stages) on st, with the stage
// kernels of the lists in `mask` and the grids of `sh`.
int enqueue_step(gmunu_batch *b, double cfl, unsigned int *nfatal, unsigned mask, const Shape &sh, int steps,
                 hipStream_t st) {
  // RK stages (same coefficients as gmunu_rk_stage); a batch holds one
  // integrator (checked at commit)
  int nst = 3;
  for (size_t s = 0; s < b->blk.size(); s++)
    if (b->used[s]) {
      nst = b->blk[s].desc.rk;
      break;
    }
  const int gfin = (b->maxg + NT / 64 - 1) / (NT / 64);
  for (int k = 0; k < steps; k++) {
    // CFL maxima: by the CFL kernel in the first step, by the last
    // recovery of the previous step after that
    if (k == 0) hipLaunchKernelGGL(k_bcfl, dim3(sh.cfl), dim3(NT), 0, st, b->d_rec, b->list(L_CFL), b->d_part);
    hipLaunchKernelGGL(k_bcfl_finish, dim3(gfin), dim3(NT), 0, st, b->d_gfirst, b->d_gcount, b->d_part, b->maxg,
                       cfl, b->d_t, b->d_tend, b->d_nstep, b->d_maxstep, b->d_dt);
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
      for (int l = 0; l < NSL; l++)
        if (mask & (1u << l)) launch_list_any<1>(l, b->d_rec, b->list(l), b->d_dt, ca, cb, last, sh.st[l], st);
      double *part = last && k + 1 < steps ? b->d_part : nullptr;
      hipLaunchKernelGGL(k_bc2p, dim3(sh.c2p), dim3(NT), 0, st, b->d_rec, b->list(L_C2P), b->d_dt, last, 0, nfatal,
                         b->d_gfatal, 1, part);
      if (sh.gh) hipLaunchKernelGGL(k_bghosts, dim3(sh.gh), dim3(NT), 0, st, b->d_rec, b->list(L_GH), b->d_dt, 0);
    }
  }
  return launch_status();
}

}  // namespace

namespace gm {

BatchItems batch_items_for(const gmunu_batch *b, const gmunu_grid_desc &d) {
  BatchItems r;
  int v = default_variant(d);
  if (b) {
    auto it = b->tuned.find(bucket_of(d));
    if (it != b->tuned.end()) v = it->second;
  }
  r.variant = list_of(v, d);
  r.stage = stage_items(d, v);
  r.cells = cell_items(d);
  r.ghosts = ghost_items(d);
  return r;
}

long batch_max_items(const gmunu_batch *b) { return b->maxi; }

hipStream_t batch_stream(const gmunu_batch *b) { return b->pstream; }

int batch_step_graph(gmunu_batch *b, double cfl, unsigned int *nfatal_dev, int steps, hipStream_t st) {
  if (!b) return GMUNU_ENULL;
  if (!(cfl > 0.0) || steps < 1) return GMUNU_EINVAL;
  // the captured step keeps the kernels of every variant used since the
  // capture (an empty list costs one short launch), so blocks of new shapes
  // coming and going do not force a capture each time
  const unsigned mask = b->var_mask | (b->have_graph ? b->graph_mask : 0u);
  const Shape want = step_shape(b);
  if (!b->have_graph || b->graph_cfl != cfl || b->graph_mask != mask || b->graph_nfatal != nfatal_dev ||
      b->graph_steps != steps || !shape_fits(b->graph_shape, want)) {
    if (b->have_graph) {
      (void)hipGraphExecDestroy(b->exec);
      b->have_graph = false;
    }
    hipGraph_t graph;
    if (hipStreamBeginCapture(b->pstream, hipStreamCaptureModeThreadLocal) != hipSuccess) return GMUNU_EHIP;
    const Shape cap = with_headroom(b, want);
    const int rc = enqueue_step(b, cfl, nfatal_dev, mask, cap, steps, b->pstream);
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
    b->graph_mask = mask;
    b->graph_nfatal = nfatal_dev;
    b->graph_steps = steps;
    b->graph_shape = cap;
  }
  if (st == b->pstream) return hipGraphLaunch(b->exec, b->pstream) == hipSuccess ? GMUNU_OK : GMUNU_EHIP;
  // order: caller's prior work -> replay on the private stream -> caller's later work
  bool ok = hipEventRecord(b->ev_in, st) == hipSuccess && hipStreamWaitEvent(b->pstream, b->ev_in, 0) == hipSuccess &&
            hipGraphLaunch(b->exec, b->pstream) == hipSuccess && hipEventRecord(b->ev_out, b->pstream) == hipSuccess &&
            hipStreamWaitEvent(st, b->ev_out, 0) == hipSuccess;
  return ok ? GMUNU_OK : GMUNU_EHIP;
}

}  // namespace gm

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
  b->geo_cap.assign(max_blocks, 0);
  b->var.assign(max_blocks, -1);
  for (long &c : b->counts) c = 0;
  b->var_mask = 0;
  b->rec_lo = INT_MAX;
  b->rec_hi = 0;
  b->have_graph = false;
  b->have_stream = false;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess) {
    delete b;
    return GMUNU_EHIP;
  }
  const size_t nb = max_blocks, ng = max_groups;
  bool ok = hipMalloc(&b->d_rec, sizeof(BlockRec) * nb) == hipSuccess;
  ok = ok && hipMalloc(&b->d_blk, sizeof(int) * NLIST * nb) == hipSuccess;
  ok = ok && hipMalloc(&b->d_start, sizeof(int) * NLIST * (nb + 1)) == hipSuccess;
  ok = ok && hipMalloc(&b->d_meta, sizeof(int) * 2 * NLIST) == hipSuccess;
  ok = ok && hipMalloc(&b->d_gfirst, sizeof(int) * ng) == hipSuccess;
  ok = ok && hipMalloc(&b->d_gcount, sizeof(int) * ng) == hipSuccess;
  ok = ok && hipMalloc(&b->d_part, sizeof(double) * max_items) == hipSuccess;
  ok = ok && hipMalloc(&b->d_t, sizeof(double) * ng) == hipSuccess;
  ok = ok && hipMalloc(&b->d_dt, sizeof(double) * ng) == hipSuccess;
  ok = ok && hipMalloc(&b->d_tend, sizeof(double) * ng) == hipSuccess;
  ok = ok && hipMalloc(&b->d_nstep, sizeof(int) * ng) == hipSuccess;
  ok = ok && hipMalloc(&b->d_maxstep, sizeof(int) * ng) == hipSuccess;
  ok = ok && hipMalloc(&b->d_gfatal, sizeof(unsigned int) * ng) == hipSuccess;
  if (!ok) {
    free_batch(b);
    return GMUNU_ENOMEM;
  }
  ok = hipMemset(b->d_rec, 0, sizeof(BlockRec) * nb) == hipSuccess &&
       hipMemset(b->d_meta, 0, sizeof(int) * 2 * NLIST) == hipSuccess &&
       hipMemset(b->d_gcount, 0, sizeof(int) * ng) == hipSuccess &&
       hipMemset(b->d_gfirst, 0, sizeof(int) * ng) == hipSuccess &&
       hipMemset(b->d_t, 0, sizeof(double) * ng) == hipSuccess &&
       hipMemset(b->d_dt, 0, sizeof(double) * ng) == hipSuccess &&
       hipMemset(b->d_tend, 0, sizeof(double) * ng) == hipSuccess &&
       hipMemset(b->d_nstep, 0, sizeof(int) * ng) == hipSuccess &&
       hipMemset(b->d_maxstep, 0, sizeof(int) * ng) == hipSuccess &&
       hipMemset(b->d_gfatal, 0, sizeof(unsigned int) * ng) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
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
  // the batched stage updates q_s in place, which the limiter (reading the
  // base state of neighbouring cells) does not allow
  if (blk->desc.pp_limiter) return GMUNU_EINVAL;
  if (!blk->q_n || !blk->q_s || !blk->prim || !blk->metric) return GMUNU_ENULL;
  if (!aligned8(blk->q_n) || !aligned8(blk->q_s) || !aligned8(blk->prim) || !aligned8(blk->metric))
    return GMUNU_EALIGN;
  std::vector<double> tab;
  BlockRec r;
  std::memset(&r, 0, sizeof(r));
  const GeoOffsets off = setup_grid(blk->desc, r.G, tab);
  // the slot's table buffer is reused when large enough (the slot is not in
  // use by a running step, so it may be overwritten)
  if (tab.size() > b->geo_cap[slot]) {
    double *g = nullptr;
    if (hipMalloc(&g, tab.size() * sizeof(double)) != hipSuccess) return GMUNU_ENOMEM;
    if (b->geo[slot]) (void)hipFree(b->geo[slot]);
    b->geo[slot] = g;
    b->geo_cap[slot] = tab.size();
  }
  double *g = b->geo[slot];
  if (hipMemcpy(g, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) return GMUNU_EHIP;
  bind_geo(r.G, g, off);
  r.qn = blk->q_n;
  r.qs = blk->q_s;
  r.prim = blk->prim;
  r.met = blk->metric;
  r.flags = blk->flags;
  r.group = blk->group;
  r.active = 1;
  r.rghosts = recovery_ghosts(blk->desc, &r.raxes);
  b->rec[slot] = r;
  b->blk[slot] = *blk;
  b->used[slot] = 1;
  b->touch(slot);
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
  b->touch(slot);
  return GMUNU_OK;
}

int gmunu_batch_set_tile(gmunu_batch *b, const gmunu_grid_desc *d, int tx, int ty, int tz) {
  if (!b || !d) return GMUNU_ENULL;
  int v = -1;
  for (int k = 0; k < NVAR; k++)
    if (kVar[k].tx == tx && kVar[k].ty == ty && kVar[k].tz == tz && kVar[k].nd == d->ndim &&
        kVar[k].rec == d->recon)
      v = k;
  if (v < 0) return GMUNU_EINVAL;
  const auto key = bucket_of(*d);
  b->tuned[key] = v;
  for (int s = 0; s < b->maxb; s++)
    if (b->used[s] && bucket_of(b->blk[s].desc) == key && b->var[s] != v) {
      b->var[s] = v;
      b->touch(s);
    }
  return GMUNU_OK;
}

int gmunu_batch_set_group(gmunu_batch *b, int group, double t, double t_end, int max_steps) {
  if (!b) return GMUNU_ENULL;
  if (group < 0 || group >= b->maxg || !(t_end >= t)) return GMUNU_EINVAL;
  b->time_set.push_back({group, t, t_end, max_steps > 0 ? max_steps : INT_MAX});
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
  HList h[L_IC2P];
  std::vector<std::vector<int>> by_group(b->maxg);
  for (int s = 0; s < b->maxb; s++) {
    if (!b->used[s]) continue;
    const gmunu_grid_desc &d = b->blk[s].desc;
    h[list_of(b->var[s], d)].add(s, stage_items(d, b->var[s]));
    h[L_C2P].add(s, cell_items(d));
    h[L_GH].add(s, ghost_items(d));
    by_group[b->rec[s].group].push_back(s);
  }
  std::vector<int> gfirst(b->maxg), gcount(b->maxg);
  for (int g = 0; g < b->maxg; g++) {
    gfirst[g] = (int)h[L_CFL].total;
    for (int s : by_group[g]) {
      if (b->rec[s].cfl_start != (int)h[L_CFL].total) {
        b->rec[s].cfl_start = (int)h[L_CFL].total;
        b->touch(s);
      }
      h[L_CFL].add(s, cell_items(b->blk[s].desc));
    }
    gcount[g] = (int)(h[L_CFL].total - gfirst[g]);
  }
  unsigned mask = 0;
  for (int l = 0; l < L_IC2P; l++)
    if (h[l].total > b->maxi) return GMUNU_EINVAL;
  for (int l = 0; l < NSL; l++)
    if (h[l].total) mask |= 1u << l;
  int meta[2 * L_IC2P];
  bool ok = upload_records(b, st);
  for (int l = 0; l < L_IC2P; l++) ok = ok && upload_list(b, l, h[l], meta + 2 * l, st);
  ok = ok && hipMemcpyAsync(b->d_gfirst, gfirst.data(), sizeof(int) * b->maxg, hipMemcpyHostToDevice, st) == hipSuccess;
  ok = ok && hipMemcpyAsync(b->d_gcount, gcount.data(), sizeof(int) * b->maxg, hipMemcpyHostToDevice, st) == hipSuccess;
  static const int zero = 0;
  for (auto &ts : b->time_set) {
    ok = ok && hipMemcpyAsync(b->d_t + ts.group, &ts.t, sizeof(double), hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(b->d_tend + ts.group, &ts.t_end, sizeof(double), hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(b->d_nstep + ts.group, &zero, sizeof(int), hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok &&
         hipMemcpyAsync(b->d_gfatal + ts.group, &zero, sizeof(unsigned int), hipMemcpyHostToDevice, st) == hipSuccess;
    ok = ok &&
         hipMemcpyAsync(b->d_maxstep + ts.group, &ts.max_steps, sizeof(int), hipMemcpyHostToDevice, st) == hipSuccess;
  }
  ok = ok && hipStreamSynchronize(st) == hipSuccess;
  b->time_set.clear();
  if (!ok) return GMUNU_EHIP;
  for (int l = 0; l < L_IC2P; l++) b->counts[l] = h[l].total;
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
  HList hc, hg;
  for (int s = 0; s < b->maxb; s++) {
    if (!b->used[s] || !sel[s]) continue;
    hc.add(s, cell_items(b->blk[s].desc));
    hg.add(s, ghost_items_all(b->blk[s].desc));
  }
  if (hc.total > b->maxi || hg.total > b->maxi) return GMUNU_EINVAL;
  int meta[4];
  bool ok = upload_records(b, st);
  ok = ok && upload_list(b, L_IC2P, hc, meta, st) && upload_list(b, L_IGH, hg, meta + 2, st);
  ok = ok && hipStreamSynchronize(st) == hipSuccess;
  if (!ok) return GMUNU_EHIP;
  const int gc = grid_for(hc.total, kGridPerCu * b->ncu), gg = grid_for(hg.total, kGridPerCu * b->ncu);
  hipLaunchKernelGGL(k_bghosts, dim3(gg), dim3(NT), 0, st, b->d_rec, b->list(L_IGH), b->d_dt, 1);
  hipLaunchKernelGGL(k_bprim2con, dim3(gc), dim3(NT), 0, st, b->d_rec, b->list(L_IC2P));
  hipLaunchKernelGGL(k_bc2p, dim3(gc), dim3(NT), 0, st, b->d_rec, b->list(L_IC2P), b->d_dt, 1, 1,
                     (unsigned int *)nullptr, (unsigned int *)nullptr, 0, (double *)nullptr);
  hipLaunchKernelGGL(k_bghosts, dim3(gg), dim3(NT), 0, st, b->d_rec, b->list(L_IGH), b->d_dt, 1);
  return launch_status();
}

int gmunu_batch_autotune(gmunu_batch *b, void *stream) {
  if (!b) return GMUNU_ENULL;
  hipStream_t st = as_stream(stream);
  std::map<std::tuple<int, int, int, int, int, int>, std::vector<int>> buckets;
  for (int s = 0; s < b->maxb; s++)
    if (b->used[s]) buckets[bucket_of(b->blk[s].desc)].push_back(s);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return GMUNU_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return GMUNU_EHIP;
  }
  int rc = upload_records(b, st) ? GMUNU_OK : GMUNU_EHIP;
  for (auto &bk : buckets) {
    if (rc) break;
    const int nd = std::get<0>(bk.first);
    const int rec = b->blk[bk.second[0]].desc.recon;
    int best = -1;
    float best_ms = 0.f;
    for (int v = 0; v < NVAR; v++) {
      if (kVar[v].nd != nd || kVar[v].rec != rec) continue;
      // only this bucket's blocks, all on variant v, in their stage list
      // (MODE 0 writes the right-hand side into q_s, which is scratch)
      const int li = list_of(v, b->blk[bk.second[0]].desc);
      HList h;
      for (int s : bk.second) h.add(s, stage_items(b->blk[s].desc, v));
      if (h.total > b->maxi) continue;
      int meta[2];
      if (!upload_list(b, li, h, meta, st) || hipStreamSynchronize(st) != hipSuccess) {
        rc = GMUNU_EHIP;
        break;
      }
      const int gst = grid_for(h.total, kGridPerCu * b->ncu);
      launch_list_any<0>(li, b->d_rec, b->list(li), b->d_dt, 0.0, 1.0, 0, gst, st);  // warm-up
      (void)hipEventRecord(e0, st);
      for (int r = 0; r < 3; r++) launch_list_any<0>(li, b->d_rec, b->list(li), b->d_dt, 0.0, 1.0, 0, gst, st);
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
    if (best >= 0) b->tuned[bk.first] = best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (int s = 0; s < b->maxb; s++)
    if (b->used[s]) {
      auto it = b->tuned.find(bucket_of(b->blk[s].desc));
      if (it != b->tuned.end()) b->var[s] = it->second;
    }
  // restore every list from the (re-chosen) variants, also after a failure
  const int rc2 = gmunu_batch_commit(b, stream);
  return rc ? rc : rc2;
}

int gmunu_batch_step(gmunu_batch *b, double cfl, unsigned int *nfatal_dev, int use_graph, void *stream) {
  if (!b) return GMUNU_ENULL;
  if (!(cfl > 0.0)) return GMUNU_EINVAL;
  hipStream_t st = as_stream(stream);
  if (!use_graph) return enqueue_step(b, cfl, nfatal_dev, b->var_mask, step_shape(b), 1, st);
  return batch_step_graph(b, cfl, nfatal_dev, 1, st);
}

int gmunu_batch_steps(gmunu_batch *b, double cfl, int nsteps, unsigned int *nfatal_dev, void *stream) {
  if (!b) return GMUNU_ENULL;
  if (!(cfl > 0.0) || nsteps < 1) return GMUNU_EINVAL;
  return batch_step_graph(b, cfl, nfatal_dev, nsteps, as_stream(stream));
}

int gmunu_batch_times(gmunu_batch *b, double *t_host, double *dt_host, int *nstep_host, unsigned int *nfatal_host,
                      void *stream) {
  if (!b) return GMUNU_ENULL;
  hipStream_t st = as_stream(stream);
  bool ok = true;
  if (t_host) ok = hipMemcpyAsync(t_host, b->d_t, sizeof(double) * b->maxg, hipMemcpyDeviceToHost, st) == hipSuccess;
  if (dt_host)
    ok = ok && hipMemcpyAsync(dt_host, b->d_dt, sizeof(double) * b->maxg, hipMemcpyDeviceToHost, st) == hipSuccess;
  if (nstep_host)
    ok = ok && hipMemcpyAsync(nstep_host, b->d_nstep, sizeof(int) * b->maxg, hipMemcpyDeviceToHost, st) == hipSuccess;
  if (nfatal_host)
    ok = ok && hipMemcpyAsync(nfatal_host, b->d_gfatal, sizeof(unsigned int) * b->maxg, hipMemcpyDeviceToHost, st) ==
                   hipSuccess;
  ok = ok && hipStreamSynchronize(st) == hipSuccess;
  return ok ? GMUNU_OK : GMUNU_EHIP;
}

int gmunu_batch_info(gmunu_batch *b, long *items_out, int *out_variant) {
  if (!b) return GMUNU_ENULL;
  if (items_out) {
    long st = 0;
    for (int l = 0; l < NSL; l++) st += b->counts[l];
    items_out[0] = st;
    items_out[1] = b->counts[L_C2P];
    items_out[2] = b->counts[L_GH];
  }
  if (out_variant)
    for (int s = 0; s < b->maxb; s++) out_variant[s] = b->used[s] ? b->var[s] : -1;
  return GMUNU_OK;
}

}  // extern "C"
