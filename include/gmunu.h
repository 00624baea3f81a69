/*
 * gmunu.h -- C ABI of the MI355X GRMHD finite-volume step.
 *
 * The library advances the ideal GRMHD equations in reference-metric form on
 * a given, frozen conformally flat (CFC) metric (psi, alpha, beta^i), as in
 * Cheong et al., "Gmunu" (arXiv 2012.07322), section 2.1 (equations,
 * conserved variables, fluxes, sources, discretised update), section 2.3
 * (wave speeds), section 2.5 (conservative-to-primitive recovery and its
 * error handling), section 2.9 (time step) and Appendix A (cell volumes,
 * face areas and averaged Christoffel symbols).  Reconstruction is MC, the
 * Riemann solver HLLE, the integrator SSPRK3 (or SSPRK2), as in section 3.
 *
 * Every array argument is a DEVICE pointer (HIP), FP64 unless stated, in
 * structure-of-arrays layout [var][k][j][i] with i fastest, ghost cells
 * included: nt[a] = n[a] + 2*g[a] cells along axis a, g[a] = ng on the active
 * axes (the first ndim) and 0 on the inactive ones.  The cell (i,j,k) of the
 * interior (0 <= i < n[0] ...) is at linear offset
 *     ((k+g[2]) * nt[1] + (j+g[1])) * nt[0] + (i+g[0]),
 * and variable v of an array is at v * ntot + offset, ntot = nt[0]nt[1]nt[2].
 *   prim   (8 vars): rho, W v^1, W v^2, W v^3, p, B^1, B^2, B^3
 *          (contravariant coordinate components; B not densitised)
 *   q      (8 vars): psi^6 (D, S_1, S_2, S_3, tau, B^1, B^2, B^3), S covariant
 *   metric (5 vars): psi, alpha, beta^1, beta^2, beta^3 at cell centres; the
 *          caller fills its ghost cells (it is never written).
 *   flags  (uint8, one per cell, nullable): c2p outcome bits GMUNU_FLAG_*.
 * Pointers must be 8-byte aligned (flags: any alignment).  The caller owns
 * all arrays and the stream; the context owns only geometry tables and small
 * scratch.  No call allocates or synchronises after gmunu_create, so a
 * sequence of calls can be captured into a HIP graph.
 *
 * Error convention: 0 on success; a negative GMUNU_E* code for invalid
 * arguments or HIP errors.  Physical failures of the recovery are never
 * return codes: they are per-cell flag bits and a device counter (nfatal)
 * the caller reads after synchronising.  The library never aborts (the
 * paper stops the code on a fatal recovery error, section 2.5.3).
 */
#ifndef GMUNU_H
#define GMUNU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { GMUNU_CART = 0, GMUNU_CYL = 1 /* (R, z, phi) */, GMUNU_SPH = 2 /* (r, theta, phi) */ };

/* Boundary kinds for the ghost fill of the primitives (the paper names the
 * ghost layers but not these rules; see gmunu_fill_ghosts). */
enum {
  GMUNU_BC_PERIODIC = 0,
  GMUNU_BC_OUTFLOW = 1, /* copy of the nearest interior cell */
  GMUNU_BC_REFLECT = 2, /* mirror; normal vector components odd */
  GMUNU_BC_AXIS = 3,    /* R = 0 or theta = 0, pi: mirror, normal component odd */
  GMUNU_BC_CENTER = 4,  /* r = 0: mirror to (r, pi - theta, phi + pi); r, theta comps odd */
  GMUNU_BC_NONE = 5     /* ghosts left as the caller set them */
};

enum {
  GMUNU_FLAG_ATMO = 1,      /* rho < rho_min: reset to atmosphere, q rewritten */
  GMUNU_FLAG_EPS_CLAMP = 2, /* eps limited to [0, eps_max], q rewritten */
  GMUNU_FLAG_V_CLAMP = 4,   /* velocity rescaled to W_max (low density), q rewritten */
  GMUNU_FLAG_FATAL_RHO = 8, /* rho > rho_max */
  GMUNU_FLAG_FATAL_EPS = 16,/* eps > eps_max at high density */
  GMUNU_FLAG_FATAL_V = 32,  /* W > W_max at high density */
  GMUNU_FLAG_NOCONV = 64    /* root finder did not converge */
};

enum {
  GMUNU_OK = 0,
  GMUNU_EINVAL = -1,  /* invalid descriptor or argument */
  GMUNU_ENULL = -2,   /* required pointer is NULL */
  GMUNU_EALIGN = -3,  /* pointer not 8-byte aligned */
  GMUNU_EHIP = -4,    /* a HIP runtime call failed */
  GMUNU_ENOMEM = -5,  /* device allocation at create time failed */
  GMUNU_ESTALL = -6,  /* a served solve stopped advancing (dt not positive
                         before its end, e.g. a non-finite wave speed) */
  GMUNU_ESTOP = -7    /* the server has stopped (after a HIP error) */
};

/* Grid and physics description (host struct, copied at create). */
typedef struct gmunu_grid_desc {
  int ndim;            /* 1, 2 or 3 active axes (the first ndim) */
  int coord;           /* GMUNU_CART / CYL / SPH */
  int n[3];            /* interior cells per axis (1 on inactive axes) */
  int ng;              /* ghost layers on active axes; MC needs >= 2 */
  double xmin[3];      /* lower edge of the interior, per axis */
  double dx[3];        /* uniform coordinate spacing (inactive phi: 2 pi) */
  int bc[3][2];        /* GMUNU_BC_* per axis and side (lower, upper) */
  double gamma;        /* ideal gas p = (Gamma - 1) rho eps */
  double rho_atmo;     /* atmosphere density; also the EOS floor rho_min */
  double k_atmo, gamma_atmo; /* atmosphere polytrope p = K rho^Gamma_atmo */
  double rho_low_factor;     /* low-density region rho < factor * rho_atmo (100) */
  double alpha_bh;           /* black-hole interior alpha < alpha_bh (1e-2) */
  double rho_max, eps_max;   /* EOS validity limits (may be +inf) */
  double w_max;              /* Lorentz factor limit */
  int c2p_maxit;             /* root-finder iteration limit */
  double c2p_tol;            /* relative tolerance of the recovered root */
  int rk;                    /* 3: SSPRK3, 2: SSPRK2 */
  int recon;                 /* GMUNU_RECON_* (reconstruction of the face states) */
  int riemann;               /* GMUNU_RIEMANN_* (approximate Riemann solver) */
  int pp_limiter;            /* 1: positivity-preserving flux limiter (section 2.4);
                                single grids only (gmunu_batch_set_block and
                                gmunu_server_submit reject it) */
  int c2p;                   /* GMUNU_C2P_* (primitive recovery scheme, section 2.5) */
} gmunu_grid_desc;

enum {
  GMUNU_RECON_MC = 0,        /* monotonised-central slopes (2 ghost layers) */
  GMUNU_RECON_MP5 = 1,       /* MP5, fifth order (3 ghost layers) */
  GMUNU_RECON_PPM = 2,       /* PPM, third order (3 ghost layers) */
  GMUNU_RIEMANN_HLLE = 0,    /* HLL with the two-speed bounds of section 2.3 */
  GMUNU_RIEMANN_TVDLF = 1,   /* local Lax-Friedrichs (Rusanov) */
  GMUNU_C2P_GRMHD = 0,       /* master-function recovery of section 2.5.2 (any B) */
  GMUNU_C2P_GRHD_Z = 1       /* z-scheme recovery of section 2.5.1 (B = 0 only; B passed through) */
};

typedef struct gmunu_ctx gmunu_ctx;

/* Validate the descriptor, build the geometry tables (Appendix A) on the
 * current HIP device and allocate the context's scratch.  Host call;
 * synchronous.  *out is set only on success. */
int gmunu_create(const gmunu_grid_desc *desc, gmunu_ctx **out);
int gmunu_destroy(gmunu_ctx *ctx);

/* Cells in one array (ntot) and the byte size of the 8-variable state. */
long gmunu_ntot(const gmunu_ctx *ctx);

/* q = prim2con(prim) on every cell including ghosts (section 2.1, the
 * definitions of the conserved variables).  Enqueued on `stream`
 * (a hipStream_t; NULL = default stream). */
int gmunu_prim2con(gmunu_ctx *ctx, const double *prim, const double *metric, double *q, void *stream);

/* Primitive recovery on the interior cells (section 2.5.2, then the error
 * handling of section 2.5.3).  Cells flagged ATMO, EPS_CLAMP or V_CLAMP get q
 * rewritten from the corrected primitives.  flags (nullable) receives the
 * bits per cell; nfatal_dev (nullable, one unsigned int) is incremented by
 * the number of cells with a fatal bit.  Ghost cells of prim are untouched. */
int gmunu_c2p(gmunu_ctx *ctx, double *q, const double *metric, double *prim, uint8_t *flags,
              unsigned int *nfatal_dev, void *stream);

/* Fill the ghost cells of prim that share a face-normal line with the
 * interior (edge and corner ghosts are never read by the scheme and are left
 * untouched), per the descriptor's boundary kinds. */
int gmunu_fill_ghosts(gmunu_ctx *ctx, double *prim, void *stream);

/* dq/dt on the interior cells: minus the flux-area divergence over the cell
 * volume plus gravitational and geometric sources (section 2.1, the
 * discretised equation), from primitives whose ghosts are filled.  Ghost
 * entries of dqdt are untouched.  The positivity-preserving limiter acts on
 * a stage's Euler step and is not applied here.
 *
 * kij (nullable, device): the extrinsic curvature K_ij that the energy and
 * momentum sources of section 2.1 contain, 6 arrays [6][layout] of the
 * covariant coordinate components (xx, xy, xz, yy, yz, zz in the grid's
 * axis order), read on the interior cells only; the caller owns it (e.g. from
 * its metric solver: section 2.6 approximates it by the traceless part of
 * the conformal vector X^i).  NULL: K_ij follows from the shift by the CFC
 * relation under maximal slicing, psi^4/(2 alpha) (D^_i beta_j + D^_j beta_i
 * - 2/3 gamma^_ij D^_k beta^k) with the flat covariant derivative D^ of the
 * reference metric gamma^ (not printed in the paper; zero for zero shift).
 * GMUNU_EALIGN if kij is not 8-byte aligned. */
int gmunu_rhs(gmunu_ctx *ctx, const double *prim, const double *metric, const double *kij, double *dqdt,
              void *stream);

/* Time step by the maxsum rule (section 2.9): dt = cfl / max over interior
 * cells of sum_axes max|lambda_a|/dx_a, capped at t_end - *t_dev, written to
 * dt_dev (one double).  t_dev may be NULL (then t = 0). */
int gmunu_cfl_dt(gmunu_ctx *ctx, const double *prim, const double *metric, double cfl, double t_end,
                 const double *t_dev, double *dt_dev, void *stream);

/* One Runge-Kutta stage (Shu-Osher form):
 *   q_out = a q_n + b (q_s + dt L(prim_in)),  (a,b) = (0,1) for stage 0,
 *   SSPRK3 stage 1 (3/4, 1/4), stage 2 (1/3, 2/3); SSPRK2 stage 1 (1/2, 1/2);
 * then q_out -> prim_out by gmunu_c2p and the ghost fill.  q_s is not read in
 * stage 0.  q_out may alias q_n or q_s (each cell reads only its own q),
 * except that with the positivity-preserving limiter (section 2.4) the stage
 * also reads the base state of the neighbouring cells (q_n in stage 0, q_s
 * after): then q_out must not overlap the base, and GMUNU_EINVAL is returned
 * when it is the same pointer.  prim_out may alias prim_in; when it is
 * another array (not overlapping prim_in) and the limiter is off, the stage
 * kernel does the recovery itself in its epilogue, with the same result bit
 * for bit (this saves the recovery's pass over q and the metric but runs the
 * iterative root finder at the stage kernel's occupancy: on a 256^3 blast it
 * is slower than the separate recovery, which gmunu_step uses).  dt is read
 * from dt_dev.  kij: as in gmunu_rhs (nullable). */
int gmunu_rk_stage(gmunu_ctx *ctx, int stage, const double *dt_dev, const double *q_n, const double *q_s,
                   double *q_out, const double *prim_in, double *prim_out, const double *metric,
                   const double *kij, uint8_t *flags, unsigned int *nfatal_dev, void *stream);

/* One full time step: dt = gmunu_cfl_dt(prim), the RK stages (q_n is
 * overwritten with q^{n+1}, q_s is scratch of the same size), prim ends
 * consistent with q^{n+1} with ghosts filled, and *t_dev += dt.  Device-side
 * time keeps the call graph-capturable.  Once *t_dev has reached t_end the
 * computed dt is 0 and the step changes nothing (q_n, q_s, prim and flags
 * are left as they are), so a caller may issue steps past the end.  With the
 * limiter and SSPRK3 the middle stage writes a third state that the context
 * holds (allocated by gmunu_create).  kij: as in gmunu_rhs (nullable), the
 * same for every stage of the step (the metric is frozen within a step). */
int gmunu_step(gmunu_ctx *ctx, double *q_n, double *q_s, double *prim, const double *metric, const double *kij,
               double cfl, double t_end, double *t_dev, double *dt_dev, uint8_t *flags, unsigned int *nfatal_dev,
               void *stream);

/* nsteps calls of gmunu_step with the same arguments, with the same result
 * bit for bit, in fewer launches: the last recovery of each step but the last
 * also writes the CFL maxima of the primitives it has just recovered (which
 * nothing changes before the next step's dt, section 2.9), so only the first
 * step launches the CFL kernel.  Time and dt stay on the device as in
 * gmunu_step (the call is capturable like it).  nsteps >= 1 (GMUNU_EINVAL
 * otherwise). */
int gmunu_steps(gmunu_ctx *ctx, double *q_n, double *q_s, double *prim, const double *metric, const double *kij,
                double cfl, double t_end, double *t_dev, double *dt_dev, uint8_t *flags, unsigned int *nfatal_dev,
                int nsteps, void *stream);

/* One step as gmunu_step, without a context and without allocating: for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc).  The grid's geometry
 * tables (computed on the device from desc at every call, with the device's
 * sine and cosine; the same values as a context's for Cartesian grids, within
 * an ulp for curvilinear ones) and the CFL partial maxima live in one
 * file-scope device array per GPU of about 1.1 MB, held until the process
 * ends.  Limit: at most 8192 cells per axis, ghosts included (GMUNU_EINVAL
 * beyond); the positivity-preserving limiter is not available here (its
 * middle SSPRK3 stage needs a third state: GMUNU_EINVAL).  Every call on one
 * GPU shares that array: calls that may overlap on one GPU (different
 * streams, or host threads) race and must be serialised by the caller.
 * Arguments, layouts and errors otherwise as gmunu_step. */
int gmunu_step_static(const gmunu_grid_desc *desc, double *q_n, double *q_s, double *prim, const double *metric,
                      const double *kij, double cfl, double t_end, double *t_dev, double *dt_dev, uint8_t *flags,
                      unsigned int *nfatal_dev, void *stream);

/* ------------------------------------------------------------------------
 * Batched stage: many independent grids ("blocks": uneven AMR-style blocks
 * of one simulation, or many simulations) advanced together by persistent
 * kernels over uniform (block, tile) work items, the whole step captured
 * once into a HIP graph and replayed.  The paper advances block-tree blocks
 * of N_grid^ndim cells with one time step for all blocks (section 2.8 and
 * 2.9); here blocks are grouped: all blocks of one group share one dt (the
 * minimum over the group's cells) and one time, groups are independent.
 *
 * Blocks live in slots.  gmunu_batch_set_block / clear_block edit the host
 * table; gmunu_batch_commit uploads it (synchronous on `stream`).  Kernels
 * read the item counts from device memory, so a captured step stays valid
 * across commits.  A step is the CFL kernel (maxima per item, then one
 * wavefront per group for its dt and time), and per RK stage the stage
 * kernels, the recovery kernel (whose threads also write the face ghosts
 * copied from the cells they recover, on the leading axes -- x, x and y, or
 * all three -- whose faces are periodic, outflow or reflecting and that hold
 * at least ng cells) and the ghost kernel for the rest (none when the
 * recovery writes every ghost).  A group whose dt is 0 (t >= t_end, or no time set) is
 * left untouched by a step.  Every block uses its own grid description and
 * arrays exactly as a single-grid context would.
 * ------------------------------------------------------------------------ */
typedef struct gmunu_batch gmunu_batch;

typedef struct gmunu_block {
  gmunu_grid_desc desc;  /* the block's grid */
  double *q_n, *q_s, *prim; /* device arrays, layout of the block's grid */
  const double *metric;     /* device, never written */
  uint8_t *flags;           /* nullable */
  int group;                /* 0 <= group < max_groups */
} gmunu_block;

/* Capacities: slots, groups, and work items per list (one item = one tile of
 * at most 256 cells, or 256 cells / ghosts).  Allocates device tables.
 * set_block, clear_block, set_group, commit, init and autotune must not be
 * called while a step of this batch may still run on the device (a slot's
 * geometry table is rewritten in place by set_block). */
int gmunu_batch_create(int max_blocks, int max_groups, long max_items, gmunu_batch **out);
int gmunu_batch_destroy(gmunu_batch *b);
/* GMUNU_EINVAL for an invalid descriptor or one with pp_limiter set (the
 * batched stage updates q_s in place, which the limiter's reads of
 * neighbouring base states rule out). */
int gmunu_batch_set_block(gmunu_batch *b, int slot, const gmunu_block *blk);
int gmunu_batch_clear_block(gmunu_batch *b, int slot);
/* Time, end time and step limit of a group (applied at the next commit,
 * which also resets the group's step count to 0).  A group stops (dt = 0)
 * when t reaches t_end or after max_steps steps; max_steps <= 0: no limit. */
int gmunu_batch_set_group(gmunu_batch *b, int group, double t, double t_end, int max_steps);
/* Rebuild the work lists and upload them; synchronises `stream`. */
int gmunu_batch_commit(gmunu_batch *b, void *stream);
/* Time the compiled tile shapes per block-size class on the committed
 * blocks and keep the fastest (writes q_s of the blocks as scratch);
 * recommits.  Results do not depend on the choice. */
int gmunu_batch_autotune(gmunu_batch *b, void *stream);
/* Pin the tile shape of the stage kernel for the class of blocks of
 * descriptor d (same ndim, n, recon and riemann), as the autotuner would:
 * blocks of that class already in the batch and those set later use it,
 * from the next commit on.  Compiled shapes (tx, ty, tz): MC in 3D 8x8x3,
 * 8x5x5, 16x4x3, 8x6x4, in 2D 16x15x1, 32x7x1, 8x28x1, in 1D 255x1x1; MP5
 * and PPM 8x5x5, 16x15x1, 255x1x1.  For reproducible timings and tests
 * (a tuning control, not in the paper); results do not depend on the shape.
 * GMUNU_EINVAL for a shape not compiled for d's ndim and reconstruction. */
int gmunu_batch_set_tile(gmunu_batch *b, const gmunu_grid_desc *d, int tx, int ty, int tz);
/* Initial data of the given committed slots (all if slots is NULL): fill the
 * ghosts of prim, q_n = prim2con(prim) on the interior, recover prim from
 * q_n, fill the ghosts again.  Other slots are not touched; synchronises
 * `stream` once (to upload the slot list). */
int gmunu_batch_init(gmunu_batch *b, const int *slots, int nslots, void *stream);
/* One step for every group with dt > 0: dt per group (section 2.9), the RK
 * stages (q_n <- q^{n+1}, q_s scratch, prim consistent, ghosts filled),
 * t += dt, step count += 1.  use_graph != 0: capture once and replay
 * (captured again when cfl, nfatal_dev or a new tile shape appears, or when
 * a work list outgrows, or shrinks well below, the grid it was captured
 * with: grids follow the committed work, so a batch of a few small blocks
 * launches few workgroups). */
int gmunu_batch_step(gmunu_batch *b, double cfl, unsigned int *nfatal_dev, int use_graph, void *stream);
/* nsteps >= 1 steps, each exactly as gmunu_batch_step with use_graph != 0,
 * replayed from one captured graph of nsteps steps (captured again when
 * nsteps changes).  Within the replay the CFL maxima of every step after
 * the first are computed by the previous step's last recovery from the
 * primitives it has just written, the values the CFL kernel would read:
 * the results equal nsteps calls of gmunu_batch_step bit for bit. */
int gmunu_batch_steps(gmunu_batch *b, double cfl, int nsteps, unsigned int *nfatal_dev, void *stream);
/* Copy the groups' t, last dt, step counts and fatal-recovery counts (cells
 * flagged FATAL_* summed over stages since the group's set_group) to host
 * arrays of max_groups entries (each nullable); synchronises `stream`. */
int gmunu_batch_times(gmunu_batch *b, double *t_host, double *dt_host, int *nstep_host, unsigned int *nfatal_host,
                      void *stream);
/* Number of committed items per list: [stage, c2p, ghosts] (ghosts of a
 * step: the ghosts that the recovery kernel writes are not counted);
 * tile variant chosen per block (out_variant[slot], -1 for empty slots). */
int gmunu_batch_info(gmunu_batch *b, long *items_out, int *out_variant);

/* Kernel timing, for measurement only (not for use under graph capture).
 * With enable != 0, every launch made through this context afterwards is
 * bracketed by HIP events on its stream (up to max_launches pairs; creating
 * them allocates, so enable outside any timed or captured region).
 * gmunu_profile_read synchronises those events and returns, per kernel kind
 * GMUNU_K_*, the summed milliseconds and the launch counts, then clears them. */
enum { GMUNU_K_STAGE = 0, GMUNU_K_C2P = 1, GMUNU_K_GHOSTS = 2, GMUNU_K_CFL = 3, GMUNU_K_OTHER = 4, GMUNU_NK = 5 };
int gmunu_profile(gmunu_ctx *ctx, int enable, int max_launches);
int gmunu_profile_read(gmunu_ctx *ctx, double *ms_out /* [GMUNU_NK] */, long *count_out /* [GMUNU_NK] */);

/* ------------------------------------------------------------------------
 * Request server: continuous batching of independent solves on one GPU.
 *
 * Callers submit solves (a grid, initial primitives and metric, an end time
 * and/or a step count) from any thread.  A worker thread admits them in
 * arrival order as soon as a slot and a contiguous range of the server's
 * device arena (its HBM budget, allocated once at create) are free, uploads
 * the initial data on a copy stream while the GPU keeps stepping the
 * resident solves, and adds the solve to a lane: a gmunu_batch with its own
 * stream (each solve its own group with its own dt), one lane per
 * integrator and kind (1D solves, other solves of at most 65536 interior
 * cells, larger ones), so small solves are not paced by large ones and the
 * lanes run concurrently.  Each lane replays its captured steps (8 per
 * replay for 1D solves, 2 for small, 1 for large) in rounds of about 2 ms
 * of device work (at least `steps_per_sync` steps).  A solve that reaches its end
 * is copied out (copy stream), removed from the batch and its memory
 * returned; its result is then available to gmunu_server_poll.  Each solve
 * is advanced by exactly the arithmetic of gmunu_step on its own grid, so a
 * served result equals the same solve advanced alone, bit for bit.  This
 * serving layer is not part of the paper; its numerics are the batch's.
 * ------------------------------------------------------------------------ */
typedef struct gmunu_server gmunu_server;

typedef struct gmunu_request {
  gmunu_grid_desc desc;  /* the solve's grid (validated at submit) */
  const double *prim;    /* initial primitives [8][layout of desc]; host or
                            device memory; ghost values are not used */
  const double *metric;  /* metric [5][layout], ghosts filled; host or device */
  double t_end;          /* the solve ends when t reaches t_end (>= 0; +inf:
                            no end time, then max_steps must be > 0) ... */
  int max_steps;         /* ... or after max_steps steps (<= 0: no limit) */
  double *q_out;         /* nullable, host or device: final q [8][layout]
                            (interior cells meaningful) */
  double *prim_out;      /* nullable, host or device: final primitives [8][layout]
                            with ghosts filled */
  unsigned long long tag; /* caller's label, returned in the result */
} gmunu_request;
/* prim and metric must stay valid and unchanged until the request's result
 * has been polled; q_out / prim_out are written before the result appears. */

typedef struct gmunu_result {
  unsigned long long id, tag;
  int status;     /* GMUNU_OK, GMUNU_ESTALL, GMUNU_ESTOP, or the GMUNU_E*
                     code with which the batch refused this one solve at
                     admission (the others go on) */
  int steps;      /* steps taken */
  unsigned int nfatal; /* fatal recoveries (cells x stages) during the solve */
  double t;       /* final time */
  double t_submit, t_admit, t_done; /* gmunu_server_clock(): submitted;
                                       memory granted (upload starts);
                                       outputs written */
  size_t bytes;   /* device footprint (q_n, q_s, prim, metric) */
} gmunu_result;

typedef struct gmunu_server_info {
  long submitted, admitted, completed, pending, resident;
  long replays;        /* batched steps issued (over all lanes) */
  size_t pool_bytes, pool_used, pool_peak;
  double busy_s;       /* worker time with at least one solve resident */
} gmunu_server_info;

/* Monotonic clock of the server, in seconds. */
double gmunu_server_clock(void);
/* hbm_bytes: arena for solve state (q_n, q_s, prim: 8 doubles per cell each,
 * metric 5; 232 bytes per cell with ghosts); max_slots: solves resident at
 * once per lane; cfl: Courant number of every solve; steps_per_sync >= 1:
 * least steps between completion checks.  Starts the worker on the
 * current device. */
int gmunu_server_create(size_t hbm_bytes, int max_slots, double cfl, int steps_per_sync, gmunu_server **out);
/* Queue a solve (non-blocking).  GMUNU_EINVAL if the descriptor is invalid
 * or asks for the limiter (solves run in a batch), if t_end is negative or
 * NaN, or +inf with no step limit, or if the solve can never fit the arena;
 * GMUNU_ESTOP after a worker error. */
int gmunu_server_submit(gmunu_server *s, const gmunu_request *req, unsigned long long *id_out);
/* Move up to `max` finished results into out; waits up to timeout_ms for the
 * first one if none is ready.  Returns the number moved (>= 0) or an error. */
int gmunu_server_poll(gmunu_server *s, gmunu_result *out, int max, int timeout_ms);
int gmunu_server_status(gmunu_server *s, gmunu_server_info *out);
/* Stop the worker (solves not finished are dropped) and free everything. */
int gmunu_server_destroy(gmunu_server *s);

#ifdef __cplusplus
}
#endif

#endif /* GMUNU_H */
