/*
 * hvpic.h -- C-ABI of the MI355X (gfx950) hybrid-PIC step library libhvpic.so.
 *
 * The library advances kinetic ions coupled to a massless electron fluid by
 * explicit time stepping, after Le et al., "Hybrid-VPIC: an open-source
 * kinetic/fluid hybrid particle-in-cell code" (arXiv 2305.05600):
 *   - ion push: leapfrog with the non-relativistic Boris method (Sec. II.B,
 *     eq:vadv and the position update that follows it);
 *   - particle shapes NGP (Sec. II.B, eq:ngp) and QS (App. B, eq:quad for the
 *     deposit, eq:quadFI + eq:quadF for the gather);
 *   - Ohm's law for massless electrons (Sec. II.A, eq:ohm) with the density
 *     floor, low-frequency Ampere, an isothermal/polytropic EOS or the
 *     electron energy equation (eq:dpdt with a heat flux -kappa0 grad T_e)
 *     and R_ei = eta J - eta_h lap J; Faraday's law (and the energy
 *     equation) subcycled inside the particle step; J_i extrapolated to the
 *     full step (Sec. II.B);
 *   - a stable counting sort of the particle store by cell (the store keeps a
 *     cell index plus in-cell offsets, Sec. II.B).
 *
 * Units: hybrid units with n0 = B0 = m_i = e = mu0 = 1 (lengths in d_i, time
 * in 1/Omega_i, speed in v_A).
 *
 * Data layout (all arrays are DEVICE memory owned by the caller):
 *   - cell index I = i + nx*(j + ny*k), 0 <= I < ncell = nx*ny*nz;
 *   - particles are structure-of-arrays: int32 cell[n]; float ox, oy[, oz][n]
 *     in-cell offsets in [-1, 1) in half-cell units about the cell centre
 *     (-1 is the left face; a particle on the right face belongs to the next
 *     cell); float ux, uy, uz[n] velocity; float w[n] weight.  2D runs use
 *     nz = 1 and pass oz = NULL;
 *   - grid fields are float [3][ncell] component-major (x block, y block,
 *     z block); densities are float [ncell];
 *   - cell_start is int32 [ncell+1]: particles of cell c occupy
 *     [cell_start[c], cell_start[c+1]) of a sorted store.
 *
 * Execution: every call validates its arguments on the host, then enqueues
 * kernels on the HIP stream given to hvpic_init and returns without waiting.
 * Only hvpic_sync_status blocks.  A context is not thread-safe; use one
 * context per stream.  The library allocates no device memory: every scratch
 * buffer lives in the caller-provided workspace.
 *
 * Errors: functions return HVPIC_OK (0) or a negative code.  Argument errors
 * return HVPIC_EINVAL and launch nothing.  Conditions found by kernels are
 * sticky status bits read (and cleared) by hvpic_sync_status.
 */
#ifndef HVPIC_H
#define HVPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HVPIC_OK = 0,
  HVPIC_EINVAL = -1, /* bad argument; nothing was launched            */
  HVPIC_ENOMEM = -2, /* workspace too small for the request           */
  HVPIC_EHIP = -3,   /* a HIP runtime call or kernel launch failed    */
  HVPIC_ESTATE = -4  /* context used before init or after finalize    */
};

enum { HVPIC_SHAPE_NGP = 0, HVPIC_SHAPE_QS = 1 };

/* Sticky status bits (hvpic_sync_status). */
enum {
  HVPIC_FLAG_MOVE_GT1 = 1,   /* a particle crossed more than one cell face in a
                                step; the neighbour-move sort fell back to the
                                full sort                                      */
  HVPIC_FLAG_FLOOR_HIT = 2,  /* n^{n+1/2} fell below n_floor in some cell      */
  HVPIC_FLAG_NONFINITE = 4,  /* non-finite or runaway displacement; the
                                particle was left in place                     */
  HVPIC_FLAG_BAD_INPUT = 8   /* a cell index outside [0, ncell) or an
                                inconsistent cell_start was met; the offending
                                entries were skipped                           */
};

typedef struct {
  int32_t ndim;              /* 2 or 3                                          */
  int32_t nx, ny, nz;        /* cells per axis; nz = 1 when ndim = 2            */
  double dx, dy, dz;         /* cell sizes (d_i); the cell volume is dx*dy*dz   */
  double dt;                 /* particle time step (1/Omega_i)                  */
  int32_t nsub;              /* Faraday substeps per particle step (Sec. II.A)  */
  int32_t shape;             /* HVPIC_SHAPE_NGP or HVPIC_SHAPE_QS               */
  int32_t nsmooth;           /* binomial passes applied by hvpic_smooth users   */
  double qs, ms;             /* ion species charge (Z e) and mass               */
  double te, gamma_e, n0;    /* EOS p_e = n0 te (n/n0)^gamma_e (Sec. II.A)      */
  double n_floor;            /* density floor n_f of the field solver           */
  double eta;                /* resistivity: R_ei = eta J - eta_h lap J         */
  double eta_h;              /* hyper-resistivity (>= 0)                        */
  int32_t energy_eq;         /* 0: p_e from the EOS; 1: p_e evolved by the
                                electron energy equation (gamma_e > 1), through
                                hvpic_field_advance_pe                          */
  double kappa0;             /* electron heat conductivity (>= 0; energy_eq)    */
  int32_t open_x;            /* 0: periodic in x; 1: open in x (Sec. II.C,
                                nx >= 3): the cells i = 0 and i = nx-1 are
                                ghosts, driven by the hvpic_open_* calls        */
  int32_t buffer_cells;      /* open_x: width w of the absorbing layer (>= 0)    */
  double eta_h_buffer;       /* open_x: eta_h added in the layer, ramping from
                                eta_h_buffer at the outermost interior column to
                                0 at depth w (>= 0)                             */
  int64_t np_capacity;       /* largest particle count any call will pass       */
} hvpic_params;

typedef struct {
  int64_t n;                 /* particle count, 0 <= n <= np_capacity            */
  int32_t* cell;
  float *ox, *oy, *oz;       /* oz NULL in 2D                                   */
  float *ux, *uy, *uz;
  float* w;
} hvpic_particles;

typedef struct hvpic_ctx hvpic_ctx;

/* Bytes of device workspace hvpic_init needs for these parameters.  Pure host
   computation; returns HVPIC_EINVAL for invalid parameters. */
int hvpic_workspace_bytes(const hvpic_params* params, size_t* bytes);

/* Creates a context bound to `hip_stream` (a hipStream_t; NULL = the null
   stream) and to `workspace` (device memory of at least
   hvpic_workspace_bytes, 256-byte aligned, owned by the caller and kept alive
   until hvpic_finalize).  Enqueues the clearing of the workspace's counters
   on the stream.  The context copies *params. */
int hvpic_init(const hvpic_params* params, void* hip_stream, void* workspace,
               hvpic_ctx** out);

/* Frees the host-side context only (never the caller's memory). */
int hvpic_finalize(hvpic_ctx* ctx);

/* Binds the context to another HIP stream (NULL = the null stream): later
   calls enqueue their kernels there.  Nothing already enqueued is waited
   for: ordering work between the old and the new stream (events) is the
   caller's.  Lets one context's calls that touch disjoint data run on two
   streams, e.g. the sort beside the field advance, while the move counts
   and the rest of the workspace stay with the context.  Returns
   HVPIC_ESTATE for an invalid context. */
int hvpic_set_stream(hvpic_ctx* ctx, void* hip_stream);

/* Gather + push (Sec. II.B eq:vadv, App. B eq:quadF): for each particle, E^n
   and B^n are interpolated at x^n with the context's shape, the velocity is
   advanced v^{n-1/2} -> v^{n+1/2} by the Boris method with
   a = (qs/ms) dt / 2 (half electric kick, rotation by t = a B,
   s = 2t/(1+t.t), half electric kick), and the particle moves
   x^{n+1} = x^n + v^{n+1/2} dt with its cell index and offsets renormalised
   into [-1, 1).  Updates p->cell, offsets and velocities in place.
   E, B: [3][ncell].  When n_mid and J_mid are both non-NULL, the moments at
   x^{n+1/2} = x^n + (dt/2) v^{n+1/2} are also deposited in the same pass
   (overwriting n_mid [ncell] and J_mid [3][ncell]; identical in value to
   hvpic_deposit with half_dt_back = dt/2 after the push), which saves one
   read of the particle store.  diag_out (device, may be NULL) receives 4
   doubles: K = sum 1/2 ms w v^{n-1/2}.v^{n+1/2} and
   P = sum ms w (v^{n-1/2}+v^{n+1/2})/2.
   cell_start (device int32 [ncell+1], may be NULL): when given, p must be
   sorted by cell with exactly this cell_start (as hvpic_sort writes it).
   The call then also counts, for every cell, its particles moving in each
   of the 3^ndim directions: the first pass of the neighbour-move sort, which
   the next hvpic_sort of the same store with cell_start_prev = cell_start
   uses instead of counting again (another push or sort in between discards
   the counts).  A particle whose place disagrees with cell_start, or a
   cell_start that is not a monotone partition of [0, n], raises
   HVPIC_FLAG_BAD_INPUT and sends that sort down the general path; the push
   itself is unaffected (every particle is pushed from its own cell).  With
   cell_start == NULL any order is accepted; a sorted order is the fast case. */
int hvpic_gather_push(hvpic_ctx* ctx, hvpic_particles* p, const int32_t* cell_start,
                      const float* E, const float* B, float* n_mid, float* J_mid,
                      double* diag_out);

/* Stable counting sort by cell index: out receives the particles of `in` in
   order of cell, equal cells in input order; cell_start [ncell+1] is written.
   `in` and `out` must not overlap and out->n is set to in->n (out's arrays
   must hold in->n entries; out->oz may be NULL in 2D).
   If full == 0 and cell_start_prev (the cell_start of `in` before its last
   push) is given, the neighbour-move path is used: it relies on every
   particle having moved at most one cell per axis since the store was sorted;
   particles that moved further are detected on the device and the call then
   completes with the general sort instead (HVPIC_FLAG_MOVE_GT1 is raised).
   full != 0 or cell_start_prev == NULL always runs the general sort (an
   LSD radix sort on the cell key).  Both paths give identical, bit-exact
   results. */
int hvpic_sort(hvpic_ctx* ctx, const hvpic_particles* in, hvpic_particles* out,
               const int32_t* cell_start_prev, int32_t* cell_start, int full);

/* The same sort given as a gather map instead of a moved store: perm
   (device int32 [in->n]) receives, for each position k of the stable order
   by cell, the index in `in` of the particle that goes there; cell_start
   [ncell+1] is written as hvpic_sort writes it.  Nothing else is written and
   `in` is only read (its cell array).  Same paths, checks and flags as
   hvpic_sort with full == 0 (cell_start_prev == NULL: the general sort).
   Together with hvpic_gather_push_perm this lets the next push read the
   store in sorted order, so the particles move once per step instead of
   twice. */
int hvpic_sort_perm(hvpic_ctx* ctx, const hvpic_particles* in, const int32_t* cell_start_prev,
                    int32_t* perm, int32_t* cell_start);

/* hvpic_gather_push of the store `in` read through a gather map: particle k
   of the step is element perm[k] of `in` (perm as hvpic_sort_perm writes
   it), and the pushed particle, weight included, is written to position k
   of `out` (out->n is set to in->n).  cell_start describes that order, as
   for hvpic_gather_push; the move counts it leaves are those of `out`.
   `in` and `out` must not overlap; in->w is always read.  Results are
   bit-identical to hvpic_sort into `out` followed by hvpic_gather_push on
   `out`. */
int hvpic_gather_push_perm(hvpic_ctx* ctx, const hvpic_particles* in, const int32_t* perm,
                           hvpic_particles* out, const int32_t* cell_start, const float* E,
                           const float* B, float* n_mid, float* J_mid, double* diag_out);

/* hvpic_gather_push_perm for a map that selects n_map (<= in->n) of the
   in->n ions of `in` (its entries index below in->n): pushes those n_map
   in map order into out (out->n = n_map).  The open step's map leaves
   absorbed ions out and takes the injected ones, which sit past the
   pushed ones in the store. */
int hvpic_gather_push_select(hvpic_ctx* ctx, const hvpic_particles* in, int64_t n_map,
                             const int32_t* perm, hvpic_particles* out,
                             const int32_t* cell_start, const float* E, const float* B,
                             float* n_mid, float* J_mid, double* diag_out);

/* Moments of the ion species (Sec. II.A n_e, J_i; eq:ngp / eq:quad) at
   x - half_dt_back * v (half_dt_back = dt/2 after a push gives
   x^{n+1/2}; 0 deposits at x).  Contributions per particle: n += qs w W/V_c,
   J += qs w W u/V_c with W the shape weight of each cell.  Overwrites
   n [ncell] and J [3][ncell].  Any particle order is accepted; a store
   sorted by cell is the fast case.  cell_start is not read (may be NULL). */
int hvpic_deposit(hvpic_ctx* ctx, const hvpic_particles* p, const int32_t* cell_start,
                  float half_dt_back, float* n, float* J);

/* Field advance (Sec. II.A eq:ohm + Faraday with subcycling, Sec. II.B
   extrapolation).  mode 0 (full step): with nbar = max(n_half, n_floor) and
   J_half held fixed, nsub explicit-midpoint substeps of h = dt/nsub
       Ea = Ohm(B), B* = B - (h/2) curl Ea, Eb = Ohm(B*), B <- B - h curl Eb,
   then n^{n+1} = 3/2 n_half - 1/2 n_prev, J^{n+1} likewise, and
   E_out = Ohm(B^{n+1}, n^{n+1}, J^{n+1}).  mode 1 (E only): E_out =
   Ohm(B, n_half, J_half); B, n_prev, J_prev are not touched (may be NULL).
   Ohm(B, n, J_i) = -u_i x B + (J x B)/n_f - grad(p_e)/n_f + eta J with
   J = curl B (centred differences), n_f = max(n, n_floor), u_i = J_i/n_f,
   p_e = n0 te (n_f/n0)^gamma_e; 1/n_f is formed in double precision.
   diag_out (device, may be NULL): 3 doubles {W_B, W_dB, W_e} =
   {1/2 sum |B|^2 V_c, 1/2 sum |B - <B>|^2 V_c} of the B left behind, and the
   electron internal energy of the density E_out was formed from (mode 0:
   n^{n+1}; mode 1: n_half), with n_f = max(n, n_floor):
   W_e = te sum n_f ln(n_f/n0) V_c for gamma_e = 1, else
   sum p_e V_c / (gamma_e - 1).  W_e is the electron term of the energy of
   the hybrid equations (Sec. II.A): with Ohm's law, Ampere and Faraday,
   d/dt (K_i + W_B + W_e) = eta sum (J.J_i - |J|^2) V_c.  All FP64.
   With eta_h > 0 Ohm's law gains -eta_h lap J, lap the compact
   (+1, -2, +1)/h^2 second difference summed over the axes, and the
   resistive work above becomes sum (eta J - eta_h lap J).(J_i - J) V_c.
   Returns HVPIC_EINVAL if the context's energy_eq is set (the pressure is
   then state: use hvpic_field_advance_pe). */
int hvpic_field_advance(hvpic_ctx* ctx, float* B, const float* n_half,
                        const float* J_half, const float* n_prev, const float* J_prev,
                        float* E_out, int mode, double* diag_out);

/* Field advance with the electron energy equation (Sec. II.A eq:dpdt with
   no collisional exchange and the heat flux Q_e = -kappa0 grad T_e), for a
   context with energy_eq = 1.  The electron pressure pe [ncell] is state:
   in mode 0 it is advanced in the same substeps as B,
       (B*, p*) = (B, p) + (h/2) rates(B, p),  (B, p) += h rates(B*, p*),
       dp/dt = -gamma div(p u_e) + (gamma-1) u_e.grad p
               + (gamma-1) kappa0 lap (p/n_f),  u_e = (J_i - curl B)/n_f,
   with n_half and J_half held fixed (centred div and grad, compact lap),
   and overwritten with the result; Ohm's law everywhere takes
   -grad(p)/n_f from the pressure instead of the EOS, and E_out is formed
   from the final B, p and the extrapolated moments.  mode 1: E_out from
   B, pe, n_half, J_half; nothing else is written.  diag_out as for
   hvpic_field_advance with W_e = sum p V_c/(gamma_e - 1) of the pressure
   E_out was formed from; then, with eta = eta_h = 0,
   d/dt (K_i + W_B + W_e) = 0 exactly in the spatially discrete equations.
   HVPIC_EINVAL unless energy_eq = 1, or for NULL arrays. */
int hvpic_field_advance_pe(hvpic_ctx* ctx, float* B, float* pe, const float* n_half,
                           const float* J_half, const float* n_prev, const float* J_prev,
                           float* E_out, int mode, double* diag_out);

/* The pressure of the equation of state, pe = n0 te (n_f/n0)^gamma_e with
   n_f = max(n, n_floor), into pe [ncell]: the starting value of the electron
   pressure for a run with the energy equation (Sec. II.A). */
int hvpic_eos_pressure(hvpic_ctx* ctx, const float* n, float* pe);

/* The deposit of hvpic_deposit, for callers that cannot allocate memory or
   create a context: code captured into a HIP graph, tight serving loops,
   harnesses that forbid allocation.  It takes the run parameters (as for
   hvpic_init; np_capacity is not used) and a HIP stream instead of a
   context, allocates nothing (no hipMalloc, no workspace: its scratch, the
   FP64 moment accumulators and a status word, is a device array of the
   library, one per GPU, held until the process ends) and enqueues on
   `hip_stream` the clearing of that scratch and the same kernels as
   hvpic_deposit: n [ncell] and J [3][ncell] are overwritten with the same
   moments (to rounding: the accumulation order of atomics differs).  Limit:
   nx*ny*nz <= HVPIC_NOALLOC_MAX_CELLS, else HVPIC_ENOMEM and nothing is
   launched; HVPIC_EINVAL for invalid parameters or pointers.  Particles
   whose cell lies outside [0, ncell) are skipped (no status is reported;
   use hvpic_deposit for that).  Every call on one GPU shares that GPU's
   scratch: calls that overlap on one GPU (several streams, or several host
   threads) race and must be ordered by the caller. */
#define HVPIC_NOALLOC_MAX_CELLS (1 << 20)
int hvpic_deposit_noalloc(const hvpic_params* params, void* hip_stream,
                          const hvpic_particles* p, float half_dt_back, float* n, float* J);

/* npasses of the binomial (1,2,1)/4 filter along every axis (Sec. II.B
   smoothing), in place on ncomp component-major grid arrays F. */
int hvpic_smooth(hvpic_ctx* ctx, float* F, int ncomp, int npasses);

/* Waits for the context's stream, returns the sticky status bits in *flags
   and, if counts is non-NULL, counts[0..2] = {particles moved more than one
   cell, non-finite/runaway particles, floor hits}; then clears them. */
int hvpic_sync_status(hvpic_ctx* ctx, uint32_t* flags, int64_t* counts);

/* Execution paths of the particle kernels (a test and tuning aid, not part of
   the method): waits for the context's stream, then stats[0] = blocks of the
   push and deposit kernels that worked through their LDS windows (a chunk of
   the sorted store spanning few enough cells) and stats[1] = blocks that fell
   back to global loads and atomics, counted since the context was created or
   the last call; then clears both. */
int hvpic_path_stats(hvpic_ctx* ctx, int64_t* stats);

/* Kernel timing on the context's stream (a measurement aid, not part of the
   method).  hvpic_timing_enable(ctx, max_launches, every) creates HIP event
   pairs for up to max_launches timed launches of each timed kernel
   (max_launches = 0 switches timing off and frees the events; at most 65536).
   While enabled, launch number 0, every, 2*every, ... of each timed kernel
   (counted from the enable call or the last read) is bracketed by events
   recorded on the context's stream, directly around that one kernel; the
   others run without them (each recorded event holds the stream a few
   microseconds, so sampling keeps the timed sequence close to an untimed
   one).  every = 1 times every launch.  hvpic_timing_read waits for the
   stream and returns, for kernel id `kernel`, the summed duration in
   milliseconds and the number of timed launches, then restarts the counts.
   Launches beyond max_launches timed ones are not timed.  Returns
   HVPIC_EINVAL for an unknown id, max_launches out of range or every < 1,
   HVPIC_EHIP if an event call fails. */
enum {
  HVPIC_KERNEL_GATHER_PUSH = 0,  /* fused gather + Boris push (+ deposit) */
  HVPIC_KERNEL_DEPOSIT = 1,      /* stand-alone moment deposit */
  HVPIC_KERNEL_SORT_SCATTER = 2, /* neighbour-move sort scatter */
  HVPIC_KERNEL_COUNT = 3
};
int hvpic_timing_enable(hvpic_ctx* ctx, int max_launches, int every);
int hvpic_timing_read(hvpic_ctx* ctx, int kernel, double* total_ms, int64_t* launches);

/* Static description of an error code. */
const char* hvpic_strerror(int code);

/* ------------------------------------------------------------ ensembles --
   Many independent 2D periodic runs stepped together (the batching form of
   the step).  Each run is the step of the calls above in the gather-map
   sequence: hvpic_gather_push_perm with the fused deposit and the move
   counts, hvpic_sort_perm, hvpic_field_advance (mode 0), with its own
   context, grid, particles and parameters.  Every phase of the step (push,
   moment output, the sort's three passes, each subcycle tile launch, the
   field diagnostics) is one persistent launch over the work items (run,
   chunk or tile) of all runs, so small runs share the GPU instead of each
   paying its launches.  The step's results per run are those of the plain
   calls (bit for bit but for the accumulation order of the atomics).

   A run's state rotates between two sets of buffers every step, as the plain
   sequence swaps them: at an even step count (store[0], cell_start[0],
   n[0], J[0]) hold the current sorted store (read through perm), its
   cell_start and the moments of level n-1/2; store[1], cell_start[1], n[1],
   J[1] are written; at an odd count the roles swap.  E, B and perm are
   updated in place.  Set up the even state with the plain calls (sort,
   deposit at x^n, field advance mode 1, an identity perm), or take the state
   a plain gather-map step left. */
typedef struct {
  hvpic_ctx* ctx;            /* the run's context: parameters and workspace   */
  hvpic_particles store[2];  /* two stores of the same n particles            */
  int32_t* perm;             /* [n] gather map over the current store         */
  int32_t* cell_start[2];    /* [ncell+1] each                                */
  float* E;                  /* [3][ncell] E^n                                */
  float* B;                  /* [3][ncell] B^n                                */
  float* n[2];               /* [ncell] each: n^{n-1/2} and the next level    */
  float* J[2];               /* [3][ncell] each                               */
  double* push_diag;         /* [4] {K, P} of the last step, or NULL          */
  double* field_diag;        /* [3] {W_B, W_dB, W_e}, or NULL                 */
} hvpic_run;

/* The choices the autotuner makes.  push_chunk[c]: particles per push block
   for runs of class c of particles per cell (c = 0: below 64, 1: below 128,
   2: more), 0/1/2 = 1024/2048/3072; a chunk must span few enough cells for
   the block's LDS windows.  field_tile[c]: subcycle tile for runs of grid
   class c (0: below 128^2 cells, 1: larger), 0 = 32x8, 1 = 16x16, 2 = 64x4.
   blocks_per_cu[k]: persistent workgroups per CU of the push, the moment
   output, the sort passes and the tile launches (1..64). */
typedef struct {
  int32_t push_chunk[3];
  int32_t field_tile[2];
  int32_t blocks_per_cu[4];
} hvpic_tuning;

typedef struct hvpic_ensemble hvpic_ensemble;

/* Device workspace the ensemble needs (tables of per-run arguments for both
   parities and the work-item lists).  HVPIC_EINVAL unless every run is 2D,
   periodic as all runs here are, without smoothing, hyper-resistivity or the
   energy equation, with 3 <= nsub <= 128 (the same for all runs), the same particle
   shape, 1 <= n < 2^30 particles in both stores, at most 512^2 cells, and all
   pointers set (the diagnostics may be NULL). */
int hvpic_ensemble_workspace_bytes(const hvpic_run* runs, int nruns, size_t* bytes);

/* The plain path's choices (3072-particle push blocks, 32x8 tiles). */
int hvpic_tuning_default(hvpic_tuning* t);

/* Creates an ensemble of nruns runs (the array is copied; the buffers and
   contexts are the caller's and must outlive it) on `hip_stream` with its
   tables in `workspace` (device memory of hvpic_ensemble_workspace_bytes,
   256-byte aligned).  tuning NULL: the defaults.  Uploads the tables with
   synchronous copies and enqueues the clearing of the runs' move counts. */
int hvpic_ensemble_init(const hvpic_run* runs, int nruns, void* hip_stream, void* workspace,
                        const hvpic_tuning* tuning, hvpic_ensemble** out);
int hvpic_ensemble_finalize(hvpic_ensemble* e);

/* One step of every run, enqueued on the ensemble's stream (by replaying
   the captured graph of the step's parity when capture is on). */
int hvpic_ensemble_step(hvpic_ensemble* e);

/* Steps taken so far (its parity says which buffers hold the state). */
int hvpic_ensemble_steps(const hvpic_ensemble* e, int64_t* steps);

/* enable = 1: captures the two parities of the step into HIP graphs (the
   ensemble's stream must not be the null stream), which later steps
   replay; 0: steps launch their kernels directly. */
int hvpic_ensemble_capture(hvpic_ensemble* e, int enable);

int hvpic_ensemble_get_tuning(const hvpic_ensemble* e, hvpic_tuning* t);
/* Waits for the ensemble's stream, then rebuilds the tables (and the graphs,
   if captured) for the new choices. */
int hvpic_ensemble_set_tuning(hvpic_ensemble* e, const hvpic_tuning* t);

/* The autotuner: tries the push chunk per class of particles per cell, the
   persistent grids and the tile shape per grid class, one knob at a time,
   keeping what takes least time; each candidate is timed with HIP events
   over `reps` REAL steps of the ensemble (all choices compute the same
   step, so the tuning steps advance the runs: hvpic_ensemble_steps counts
   them).  Leaves the best choices in force, returns them in *best (may be
   NULL) and the timed phases {push, moments + sort, fields} in ms[3] (may be
   NULL).  Waits for the stream. */
int hvpic_ensemble_autotune(hvpic_ensemble* e, int reps, hvpic_tuning* best, double* ms);

/* Runs `steps` real steps launching their kernels directly, with HIP events
   at the phase boundaries, waits for them, and returns the mean time per
   step of each phase in ms[3] = {push (all chunks of all runs), moment
   output + sort, field advance + diagnostics}. */
int hvpic_ensemble_time_phases(hvpic_ensemble* e, int steps, double* ms);

/* ------------------------------------------------- neural-operator surrogate --
   A small convolutional neural operator that proposes the result of the
   subcycled field advance of Sec. II.A on 2D periodic grids,
       B^{n+1} ~ B^n + out_std * NO((B^n, n^{n+1/2}, J_i^{n+1/2}) normalised),
   NO = four periodic 3x3 convolutions 7 -> 32 -> 32 -> 32 -> 3 with tanh
   between them, run on the matrix cores with BF16 operands and FP32
   accumulation, trained here on snapshots of the plain solver (MSE of the
   normalised increment, Adam).  The plain subcycle stays the reference: a
   proposal is used only if its residual against Faraday's law with Ohm's
   law at the midpoint,
       r = (B' - B^n)/dt + curl E((B^n + B')/2)   (moments held at n+1/2),
   satisfies ||r|| <= tol ||(B' - B^n)/dt||; otherwise the plain subcycle
   runs.  The decision is taken on the device (no host round trip).

   The parameter block (hvpic_no_params_bytes, device memory of the caller)
   holds the FP32 weights and biases, Adam's moments, the normalisation and
   the BF16 copies the kernels read.  Logical weight layout for load/store:
   the four layers concatenated, each [Cout][9][Cin] with tap t = 3(dy+1) +
   (dx+1) reading x[j+dy][i+dx] (periodic), biases concatenated, and the
   normalisation {mean[7], std[7], out_std[3]} of the input channels
   (B_x, B_y, B_z, n, J_x, J_y, J_z) and of the increment. */
int hvpic_no_params_bytes(size_t* bytes);
/* Device workspace (activations) for `batch` samples of an nx x ny grid. */
int hvpic_no_workspace_bytes(int nx, int ny, int batch, size_t* bytes);
/* Loads weights, biases and the normalisation (device arrays in the logical
   layout) into the block; clears Adam's state.  Enqueued on hip_stream. */
int hvpic_no_load(void* params, const float* w, const float* b, const float* norm,
                  void* hip_stream);
/* Copies the block's weights and biases out in the logical layout. */
int hvpic_no_store(const void* params, float* w, float* b, void* hip_stream);
/* The proposal B_out [3][nx*ny] for one state (B [3][P], n [P], J [3][P]). */
int hvpic_no_predict(const void* params, void* workspace, int nx, int ny, const float* B,
                     const float* n, const float* J, float* B_out, void* hip_stream);
/* One training step on the `batch` samples idx[0..batch) (device int32) of a
   data set B [S][3][P], n [S][P], J [S][3][P], B_target [S][3][P]: forward,
   the loss mean((d - (B_target - B)/out_std)^2) into *loss_out (device
   double, may be NULL), backward and one Adam step of rate lr. */
int hvpic_no_train_step(void* params, void* workspace, int nx, int ny, const float* B,
                        const float* n, const float* J, const float* B_target, const int32_t* idx,
                        int batch, float lr, double* loss_out, void* hip_stream);
/* The field advance (mode 0) with the operator's proposal in place of the
   subcycle when it passes the residual test (2D contexts without hyper-
   resistivity or the energy equation).  Same outputs as hvpic_field_advance;
   stats (device, may be NULL) <- {||r|| / ||rate||, 1 if accepted}.  The
   workspace is one of hvpic_no_workspace_bytes(nx, ny, 1). */
int hvpic_field_advance_no(hvpic_ctx* ctx, const void* params, void* workspace, float* B,
                           const float* n_half, const float* J_half, const float* n_prev,
                           const float* J_prev, float* E_out, double* diag_out, float tol,
                           double* stats);
/* One periodic 3x3 layer of the operator's kernels on nimg images (x: BF16
   [N][cinp], w: BF16 [coutp][9][cinp], bias FP32 [coutp]): mode 0 out = BF16
   tanh(conv + bias), 1 out = FP32 conv + bias, 2 out = BF16 conv * (1 - h^2)
   with h BF16 [N][coutp] (no bias).  (cinp, coutp, mode) in {(16,32,0),
   (32,32,0), (32,16,1), (16,32,2), (32,32,2)}. */
int hvpic_no_conv3x3(int nimg, int nx, int ny, int cinp, int coutp, int mode, const void* x,
                     const void* w, const float* bias, const void* h, void* out,
                     void* hip_stream);
/* Its weight gradient, added to dw [coutp][9][cinp] and db [coutp] (FP32):
   dw[o][t][c] += sum_p dz[p][o] x[p + off(t)][c], db[o] += sum_p dz[p][o].
   (cinp, coutp) in {(32,16), (32,32), (16,32)}; workspace as for a batch of
   nimg. */
int hvpic_no_conv3x3_wgrad(int nimg, int nx, int ny, int cinp, int coutp, const void* x,
                           const void* dz, float* dw, float* db, void* workspace,
                           void* hip_stream);

/* ---------------------------------------------------------------------------
 * Open boundaries in x (Sec. II.C), 2D or 3D, for a context with open_x = 1.
 * The grid's cells i = 0 and i = nx-1 (columns in 2D, planes in 3D; called
 * ghost columns below) lie outside the domain; the domain is i = 1 .. nx-2.
 * A face's rows are its ny nz cells (j, k), row r = j + ny k.  The magnetic
 * field is split B = B0 + B1:
 * B0 (device [3][ncell]) is a fixed external field with curl B0 = 0 that
 * the caller keeps, only B1 is advanced, and the plasma current of Ohm's
 * Hall and resistive terms is J = curl B1.  In a ghost cell B1 and the
 * moments equal their interior neighbour, and Ohm's law keeps the gradients
 * along the boundary and drops those normal to it (x-derivatives are zero
 * there).  A layer of buffer_cells cells at each boundary adds
 * eta_h_buffer (1 - d/buffer_cells) to eta_h, d = 0 at the outermost
 * interior column.  The push, the deposit and the sort run unchanged on this
 * grid (their periodic wrap only ever joins the two ghost columns).  One
 * step in the gather-map form: hvpic_gather_push_perm with E and B0 + B1
 * (counting moves, fused deposit) into the second store; hvpic_open_inject
 * appends the fresh ions to it; hvpic_sort_open_perm orders it, leaving the
 * absorbed ions out, and its info gives the live count; hvpic_open_fill of
 * the moments; hvpic_open_field_advance.  When the sort reports that it
 * could not take its neighbour path (far movers), hvpic_open_absorb and
 * hvpic_sort_open (the general radix path) order the store instead.
 * ------------------------------------------------------------------------- */

/* Drifting Maxwellian of the inflow: density n, drift (ux, uy, uz) (ux > 0
   flows in through the left face, out through the right), thermal speed
   vth (> 0), ppc ions per cell of density n; faces: bit 0 the left face,
   bit 1 the right. */
typedef struct {
  double n, ux, uy, uz, vth;
  int32_t ppc;
  int32_t faces;
} hvpic_inflow;

/* Copies column 1 into column 0 and column nx-2 into column nx-1, in every
   row (j, k), of the ncomp (1..16) component-major arrays F [ncomp][ncell]
   (the ghost rule of B1 and the moments). */
int hvpic_open_fill(hvpic_ctx* ctx, float* F, int ncomp);

/* hvpic_field_advance for open x: B1 (in/out [3][ncell]) advanced by the
   subcycled RK2 Faraday update (mode 0; the ghost columns refilled after
   each stage, only the interior updated by Faraday) with E from Ohm's law
   at the frozen n_half, J_half and B = B0 + B1; then E_out = E^{n+1} from
   B1 and the extrapolated moments 3/2 n_half - 1/2 n_prev (mode 0) or from
   n_half, J_half as given (mode 1: no advance, no ghost refill of B1), and
   Btot = B0 + B1 [3][ncell] for the next push.  The moments' ghost columns
   must be filled (hvpic_open_fill).  diag_out (device, may be NULL): W_B
   and W_dB of B0 + B1 and W_e, summed over the interior cells.  The count
   of n_half cells below n_floor goes to the status.  energy_eq is not
   supported here (HVPIC_EINVAL). */
int hvpic_open_field_advance(hvpic_ctx* ctx, const float* B0, float* B1, float* Btot,
                             const float* n_half, const float* J_half, const float* n_prev,
                             const float* J_prev, float* E_out, int mode, double* diag_out);

/* Absorption: every ion of p in a ghost column gets the key ncell (the
   general path's mark; hvpic_sort_open puts such ions last). */
int hvpic_open_absorb(hvpic_ctx* ctx, hvpic_particles* p);

/* Injection alone (hvpic_open_particles without the absorption), recorded
   for the next hvpic_sort_open_perm of the same store. */
int hvpic_open_inject(hvpic_ctx* ctx, hvpic_particles* p, const hvpic_inflow* in, uint64_t seed,
                      int64_t step);

/* The neighbour-move sort of the open step as a gather map (as
   hvpic_sort_perm): in's first n_pushed ions are the store that the
   counting push wrote in the order of cell_start_prev [ncell+1], moved by
   at most one cell; the ions after them (in->n - n_pushed) must be those
   the last hvpic_open_inject appended to this store.  Ions now in a ghost
   column are absorbed: left out of the order.  Writes perm[0 .. live) and
   cell_start [ncell+1] (cell_start[ncell] = live); each cell holds its
   moved ions in input order, then its injected ones.  info (device int32[2],
   may be NULL): info[0] = 1 when a far mover or an inconsistent
   cell_start_prev keeps the sort from its neighbour path (then nothing
   else is written and the caller takes the general path), else 0;
   info[1] = live. */
int hvpic_sort_open_perm(hvpic_ctx* ctx, const hvpic_particles* in, int64_t n_pushed,
                         const int32_t* cell_start_prev, int32_t* perm, int32_t* cell_start,
                         int32_t* info);

/* Absorption and injection of one step: every ion of p in a ghost column
   gets the key ncell (absorbed; hvpic_sort_open puts it last), then
   floor(N + U) fresh ions per row of each open face are appended at p->n
   (p->n grows on the host).  N = ppc dt/dx F(u, vth) with F the inward
   flux per unit density of the drifting Maxwellian and u the drift along
   the face's inward normal; U and every velocity and position draw are the
   counter-based uniforms mix(seed + mix(ctr)) of splitmix64's finaliser,
   the counter packing (step, face, row, ion, draw), so a run is repeatable.
   An injected ion sits in the first interior column at depth v dt U' from
   its face (v the inward normal speed, drawn from the flux-weighted
   distribution by inverting its distribution function), uniformly in y
   (and z in 3D: p->oz required), tangential velocities drifting
   Maxwellian, weight n dx dy dz / ppc.  0 <= step < 2^20, ny nz <= 65536,
   fewer than 2^20 ions per row.  p's arrays must hold np_capacity ions;
   HVPIC_ENOMEM (nothing launched) when the injected ions would exceed it. */
int hvpic_open_particles(hvpic_ctx* ctx, hvpic_particles* p, const hvpic_inflow* in,
                         uint64_t seed, int64_t step);

/* Stable sort of in by cell into out, the absorbed ions (key ncell) last.
   cell_start (device int32 [ncell+2]): cell_start[ncell] is the count of
   live ions (the caller's new n), cell_start[ncell+1] = in->n. */
int hvpic_sort_open(hvpic_ctx* ctx, const hvpic_particles* in, hvpic_particles* out,
                    int32_t* cell_start);

#ifdef __cplusplus
}
#endif
#endif
