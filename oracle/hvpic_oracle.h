/*
 * hvpic_oracle.h -- plain FP64 CPU oracle of the explicit kinetic-ion /
 * massless-fluid-electron hybrid PIC step (Le et al., "Hybrid-VPIC",
 * arXiv 2305.05600, Sec. II and App. B).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no source, header, table or helper with
 * the GPU library and the GPU library never calls it.
 *
 * Conventions (all of them restated in hvpic_oracle.c next to the code):
 *   - Hybrid units: n0 = B0 = m_i = e = mu0 = 1 (Sec. II.A, Alfvenic units).
 *   - Cell index I = i + nx*(j + ny*k)  (Sec. II.B: I <-> (i,j,k)).
 *   - In-cell offsets (dx,dy,dz) in [-1,1) in half-cell units about the
 *     cell centre (Sec. II.B gives [-1,1]^3; the right face belongs to the
 *     next cell).
 *   - Grid arrays are component-major: F[c + comp*ncell], comp 0..2.
 *   - 2D runs are 3D runs with nz = 1 (periodic, so k+-1 == k) and dz = 0
 *     offsets; dz (the cell depth) still enters the cell volume.
 *   - Every loop is single-threaded and in index order, so results are
 *     reproducible bit for bit.
 */
#ifndef HVPIC_ORACLE_H
#define HVPIC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_SHAPE_NGP = 0, ORC_SHAPE_QS = 1 };

typedef struct {
  int32_t ndim, nx, ny, nz;
  double dx, dy, dz, dt;
  int32_t nsub, shape, nsmooth;
  double qs, ms;                   /* species charge Z e and mass           */
  double te, gamma_e, n0, n_floor; /* p_e = n0 te (n/n0)^gamma, density floor */
  double eta;                      /* resistivity in R_ei = eta J - eta_h lap J */
  double eta_h;                    /* hyper-resistivity                    */
  int32_t energy_eq;               /* 1: p_e evolved by the energy equation */
  double kappa0;                   /* heat conductivity in Q_e = -kappa0 grad T_e */
  int32_t open_x;                  /* 1: x boundaries open (2D or 3D): the cells
                                      with i = 0 or nx-1 are ghost cells     */
  int32_t buffer_cells;            /* width of the enhanced eta_h layer        */
  double eta_h_buffer;             /* eta_h added at the open boundary (ramp)  */
} orc_params;

/* Plasma injected through the open faces (Sec. II.C): density, drift and
   per-component thermal speed; ppc particles per cell at that density; faces
   bit 0 = x-min face, bit 1 = x-max face. */
typedef struct {
  double n, ux, uy, uz, vth;
  int32_t ppc;
  int32_t faces;
} orc_inflow;

typedef struct {
  int64_t moved_gt1;  /* particles whose move crossed more than one cell face */
  int64_t nonfinite;  /* particles with a non-finite or runaway displacement  */
  int64_t floor_hits; /* cells with n below the density floor                 */
} orc_status;

/* Field value at a particle (eq:quadFI + eq:quadF for QS, cell value for NGP).
   F is one 3-component grid field; out[3] receives the interpolated vector. */
void orc_gather(const orc_params* p, const double* F, int32_t cell,
                double ox, double oy, double oz, double out[3]);

/* Non-relativistic Boris update of v (eq:vadv) with a = (q/m) dt / 2. */
void orc_boris(double a, const double E[3], const double B[3], double v[3]);

/* Leapfrog push of np particles: gather E^n, B^n at x^n, Boris to v^{n+1/2},
   move to x^{n+1} and re-index.  diag[4] = {K, Px, Py, Pz} with
   K = sum 1/2 m w v^{n-1/2}.v^{n+1/2} and P = sum m w (v^{n-1/2}+v^{n+1/2})/2. */
void orc_push(const orc_params* p, int64_t np, int32_t* cell, double* ox,
              double* oy, double* oz, double* ux, double* uy, double* uz,
              const double* w, const double* E, const double* B,
              double diag[4], orc_status* st);

/* Stable counting sort by cell key: perm[r] = index of the r-th particle in
   sorted order (ties kept in input order); cell_start[ncell+1]. */
void orc_sort(const orc_params* p, int64_t np, const int32_t* key,
              int64_t* perm, int32_t* cell_start);

/* Moments n and J_i (eq:ngp / eq:quad) deposited at x - half_dt_back * v.
   n[ncell] and J[3*ncell] are overwritten. */
void orc_deposit(const orc_params* p, int64_t np, const int32_t* cell,
                 const double* ox, const double* oy, const double* oz,
                 const double* ux, const double* uy, const double* uz,
                 const double* w, double half_dt_back, double* n, double* J);

/* npasses of the (1,2,1)/4 binomial filter along every axis, in place. */
void orc_smooth(const orc_params* p, double* F, int32_t ncomp, int32_t npasses);

/* Centred-difference curl, C = D x A. */
void orc_curl(const orc_params* p, const double* A, double* C);

/* Ohm's law (eq:ohm) with the density floor and p_e from the EOS;
   E[3*ncell] overwritten. */
void orc_ohm(const orc_params* p, const double* B, const double* n,
             const double* Ji, double* E);

/* The same with a given electron pressure pe[ncell] instead of the EOS. */
void orc_ohm_pe(const orc_params* p, const double* B, const double* n,
                const double* Ji, const double* pe, double* E);

/* Right-hand side of the electron energy equation (eq:dpdt, H_ei = 0):
   rate = -gamma div(p_e u_e) + (gamma-1) u_e.grad p_e + (gamma-1) kappa0 lap T_e,
   u_e = (J_i - curl B)/n_f, T_e = p_e/n_f; rate[ncell] overwritten. */
void orc_pe_rate(const orc_params* p, const double* B, const double* n,
                 const double* Ji, const double* pe, double* rate);

/* Field advance with the electron pressure evolved by eq:dpdt in the same
   RK2 subcycle as B (pe[ncell] in/out); otherwise as orc_field_advance, with
   E from the evolved p_e.  diag[3] = {W_B, W_dB, W_e = sum p_e V/(gamma-1)}. */
void orc_field_advance_pe(const orc_params* p, double* B, double* pe,
                          const double* n_half, const double* J_half,
                          const double* n_prev, const double* J_prev,
                          double* E_out, int32_t mode, double diag[3],
                          orc_status* st);

/* Field advance.  mode 0: nsub RK2-midpoint Faraday substeps of B with the
   moments frozen at n+1/2, then J_i, n extrapolated to n+1 and
   E_out = Ohm(B^{n+1}, n^{n+1}, J^{n+1}).  mode 1: E_out = Ohm(B, n_half,
   J_half) only.  diag[3] = {W_B, W_dB, W_e}: the magnetic energy and its
   fluctuation part for the B the call leaves behind, and the electron
   internal energy of the density E_out was formed from (floored). */
void orc_field_advance(const orc_params* p, double* B, const double* n_half,
                       const double* J_half, const double* n_prev,
                       const double* J_prev, double* E_out, int32_t mode,
                       double diag[3], orc_status* st);

/* ---- open boundaries in x (Sec. II.C), 2D, on a grid whose columns 0 and
   nx-1 are ghost columns ---- */

/* Ghost columns of ncomp component-major arrays set to their interior
   neighbours (B1 and the plasma moments). */
void orc_open_fill(const orc_params* p, double* F, int32_t ncomp);

/* curl with no x-derivatives in the ghost columns. */
void orc_open_curl(const orc_params* p, const double* A, double* C);

/* Ohm's law with B = B0 + B1 and J = curl B1 (the split of Sec. II.C), no
   gradients normal to an open boundary in the ghost columns, and eta_h
   raised over the buffer layer. */
void orc_open_ohm(const orc_params* p, const double* B0, const double* B1, const double* n,
                  const double* Ji, double* E);

/* The field advance of B1 (mode 0) or E only (mode 1) on the open grid;
   Btot = B0 + B1 afterwards; diag over the interior cells. */
void orc_open_field_advance(const orc_params* p, const double* B0, double* B1,
                            const double* n_half, const double* J_half, const double* n_prev,
                            const double* J_prev, double* E_out, double* Btot, int32_t mode,
                            double diag[3], orc_status* st);

/* Ions in the ghost columns are absorbed: their cell becomes ncell (the key
   that sorts them last); returns how many. */
int64_t orc_open_absorb(const orc_params* p, int64_t np, int32_t* cell);

/* Expected ions entering one boundary row of a face per step. */
double orc_inflow_expected(const orc_params* p, const orc_inflow* in, int32_t face);

/* Appends the ions injected this step (counter-based draws of seed and
   step) after the np stored ones; returns the new count (at most cap).  A
   face's rows are its (j, k) cells, row r = j + ny k (ny nz <= 65536); oz
   (3D) may be NULL in 2D. */
int64_t orc_open_inject(const orc_params* p, const orc_inflow* in, uint64_t seed, int64_t step,
                        int64_t np, int64_t cap, int32_t* cell, double* ox, double* oy,
                        double* oz, double* ux, double* uy, double* uz, double* w);

/* The uniform in [0, 1) of counter ctr and seed (splitmix64 mixing). */
double orc_uniform(uint64_t seed, uint64_t ctr);

#ifdef __cplusplus
}
#endif
#endif
