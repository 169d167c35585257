/*
 * hvpic_oracle.c -- plain FP64 CPU oracle of the Hybrid-VPIC step
 * (Le et al., arXiv 2305.05600).  TEST INFRASTRUCTURE ONLY: the GPU library
 * never calls this file and shares nothing with it.
 *
 * Each function follows one passage of the paper; readings of points the
 * paper leaves open are stated where they are used:
 *   gather ..... App. B, eq:quadFI and eq:quadF (QS); Sec. II.B (NGP)
 *   boris ...... Sec. II.B, eq:vadv and the Boris description after it
 *   move ....... Sec. II.B, position update and the (I, dx,dy,dz) store
 *   deposit .... Sec. II.B eq:ngp (NGP); App. B eq:quad (QS)
 *   ohm ........ Sec. II.A eq:ohm, density floor, Ampere, EOS, R_ei
 *   faraday .... Sec. II.A Faraday + subcycling; Sec. II.B extrapolation
 *   energy eq .. Sec. II.A eq:dpdt with Q_e = -kappa grad T_e (H_ei = 0)
 *   gradients .. Sec. II.B centred differences on the cell-centred grid
 *   smoothing .. Sec. II.B (binomial passes; the cited method is not in the
 *                paper, the (1,2,1)/4 reading is documented)
 *   sort ....... not in the paper: a stable counting sort by cell index
 */
#include "hvpic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- grid -- */

static int64_t ncell_of(const orc_params* p) {
  return (int64_t)p->nx * p->ny * p->nz;
}

static int wrap(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

/* I <-> (i,j,k), row-major with i fastest (Sec. II.B). */
static int64_t cell_of(const orc_params* p, int i, int j, int k) {
  return (int64_t)wrap(i, p->nx) +
         (int64_t)p->nx * ((int64_t)wrap(j, p->ny) + (int64_t)p->ny * wrap(k, p->nz));
}

static void ijk_of(const orc_params* p, int64_t c, int* i, int* j, int* k) {
  *i = (int)(c % p->nx);
  *j = (int)((c / p->nx) % p->ny);
  *k = (int)(c / ((int64_t)p->nx * p->ny));
}

static double cell_volume(const orc_params* p) { return p->dx * p->dy * p->dz; }

/* Centred difference of scalar Q along axis a at (i,j,k):
   (Q_{+1} - Q_{-1}) / (2 Delta_a)  (Sec. II.B gradient formula). */
static double dcentred(const orc_params* p, const double* Q, int a, int i, int j, int k) {
  int di = a == 0, dj = a == 1, dk = a == 2;
  double h = a == 0 ? p->dx : (a == 1 ? p->dy : p->dz);
  return (Q[cell_of(p, i + di, j + dj, k + dk)] - Q[cell_of(p, i - di, j - dj, k - dk)]) /
         (2.0 * h);
}

/* ---------------------------------------------------------- gather ----- */

/* QS interpolation (App. B).  The interpolants of eq:quadFI are built for the
   particle's cell and combined with eq:quadF:
     F = F0 + dx (Fx + dx Fxx) + dy (Fy + dy Fyy) + dz (Fz + dz Fzz).
   In 2D nz = 1, so k+1 and k-1 are cell k itself; Fz and Fzz then vanish. */
static double qs_interp(const orc_params* p, const double* Fc, int i, int j, int k,
                        double dx, double dy, double dz) {
  double F = Fc[cell_of(p, i, j, k)];
  double Fip = Fc[cell_of(p, i + 1, j, k)], Fim = Fc[cell_of(p, i - 1, j, k)];
  double Fjp = Fc[cell_of(p, i, j + 1, k)], Fjm = Fc[cell_of(p, i, j - 1, k)];
  double Fkp = Fc[cell_of(p, i, j, k + 1)], Fkm = Fc[cell_of(p, i, j, k - 1)];
  double F0 = (1.0 / 12.0) * (6.0 * F + Fip + Fjp + Fkp + Fim + Fjm + Fkm);
  double Fx = (1.0 / 6.0) * (Fip - Fim);
  double Fy = (1.0 / 6.0) * (Fjp - Fjm);
  double Fz = (1.0 / 6.0) * (Fkp - Fkm);
  double Fxx = (1.0 / 12.0) * (Fip + Fim - 2.0 * F);
  double Fyy = (1.0 / 12.0) * (Fjp + Fjm - 2.0 * F);
  double Fzz = (1.0 / 12.0) * (Fkp + Fkm - 2.0 * F);
  return F0 + dx * (Fx + dx * Fxx) + dy * (Fy + dy * Fyy) + dz * (Fz + dz * Fzz);
}

void orc_gather(const orc_params* p, const double* F, int32_t cell, double ox,
                double oy, double oz, double out[3]) {
  int64_t nc = ncell_of(p);
  int i, j, k;
  ijk_of(p, cell, &i, &j, &k);
  if (p->ndim == 2) oz = 0.0;
  for (int comp = 0; comp < 3; ++comp) {
    const double* Fc = F + comp * nc;
    if (p->shape == ORC_SHAPE_NGP)
      out[comp] = Fc[cell]; /* NGP: the local cell value (Sec. II.B) */
    else
      out[comp] = qs_interp(p, Fc, i, j, k, ox, oy, oz);
  }
}

/* ----------------------------------------------------------- Boris ----- */

/* v^{n+1/2} = v^{n-1/2} + (q/m)(E + vbar x B) dt with vbar the mean of the two
   half-step velocities (eq:vadv), solved by the standard Boris split: half
   electric kick, rotation about B, half electric kick.  a = (q/m) dt / 2;
   t = a B, s = 2 t / (1 + t.t). */
void orc_boris(double a, const double E[3], const double B[3], double v[3]) {
  double vm[3], vp[3], vprime[3], t[3], s[3];
  for (int c = 0; c < 3; ++c) vm[c] = v[c] + a * E[c];
  for (int c = 0; c < 3; ++c) t[c] = a * B[c];
  double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  for (int c = 0; c < 3; ++c) s[c] = 2.0 * t[c] / (1.0 + tt);
  vprime[0] = vm[0] + (vm[1] * t[2] - vm[2] * t[1]);
  vprime[1] = vm[1] + (vm[2] * t[0] - vm[0] * t[2]);
  vprime[2] = vm[2] + (vm[0] * t[1] - vm[1] * t[0]);
  vp[0] = vm[0] + (vprime[1] * s[2] - vprime[2] * s[1]);
  vp[1] = vm[1] + (vprime[2] * s[0] - vprime[0] * s[2]);
  vp[2] = vm[2] + (vprime[0] * s[1] - vprime[1] * s[0]);
  for (int c = 0; c < 3; ++c) v[c] = vp[c] + a * E[c];
}

/* ------------------------------------------------------------ move ----- */

/* Offsets live in [-1,1) in half-cell units.  After xi' = xi + displacement,
   the shift s is the unique integer with xi' - 2 s in [-1,1): a particle that
   lands exactly on the right face (+1) belongs to the next cell at -1.
   Returns s and updates *xi (which must be finite). */
static int reindex(double* xi, double disp) {
  double x = *xi + disp;
  int s;
  if (x >= 1.0) {
    s = x < 3.0 ? 1 : (int)floor((x + 1.0) * 0.5);
  } else if (x < -1.0) {
    s = x >= -3.0 ? -1 : (int)floor((x + 1.0) * 0.5);
  } else {
    s = 0;
  }
  x -= 2.0 * s;
  while (x >= 1.0) { x -= 2.0; ++s; }
  while (x < -1.0) { x += 2.0; --s; }
  *xi = x;
  return s;
}

/* Moves a point with offsets off[0..ndim) by disp (half-cell units) and
   writes the cell shifts to s.  If the new offset along any axis is
   non-finite or runaway (|xi'| >= 1e6 half-cells) the whole point stays
   where it was (shifts 0, offsets unchanged) and 0 is returned; else 1. */
static int move_point(int ndim, double off[3], const double disp[3], int s[3]) {
  s[0] = s[1] = s[2] = 0;
  for (int a = 0; a < ndim; ++a)
    if (!(fabs(off[a] + disp[a]) < 1.0e6)) return 0;
  for (int a = 0; a < ndim; ++a) s[a] = reindex(&off[a], disp[a]);
  return 1;
}

void orc_push(const orc_params* p, int64_t np, int32_t* cell, double* ox, double* oy,
              double* oz, double* ux, double* uy, double* uz, const double* w,
              const double* E, const double* B, double diag[4], orc_status* st) {
  double a = 0.5 * (p->qs / p->ms) * p->dt;
  double K = 0.0, P[3] = {0.0, 0.0, 0.0};
  int64_t gt1 = 0, bad = 0;
  for (int64_t n = 0; n < np; ++n) {
    double zoff = (p->ndim == 3) ? oz[n] : 0.0;
    double Ep[3], Bp[3];
    orc_gather(p, E, cell[n], ox[n], oy[n], zoff, Ep);
    orc_gather(p, B, cell[n], ox[n], oy[n], zoff, Bp);
    double vold[3] = {ux[n], uy[n], uz[n]};
    double v[3] = {ux[n], uy[n], uz[n]};
    orc_boris(a, Ep, Bp, v);
    K += 0.5 * p->ms * w[n] * (vold[0] * v[0] + vold[1] * v[1] + vold[2] * v[2]);
    for (int c = 0; c < 3; ++c) P[c] += p->ms * w[n] * 0.5 * (vold[c] + v[c]);
    ux[n] = v[0];
    uy[n] = v[1];
    uz[n] = v[2];
    /* x^{n+1} = x^n + v^{n+1/2} dt; in half-cell units the displacement
       along an axis of width h is 2 v dt / h.  A non-finite or runaway move
       leaves the particle where it was, counted once. */
    int i, j, k;
    ijk_of(p, cell[n], &i, &j, &k);
    double off[3] = {ox[n], oy[n], p->ndim == 3 ? oz[n] : 0.0};
    double disp[3] = {2.0 * v[0] * p->dt / p->dx, 2.0 * v[1] * p->dt / p->dy,
                      2.0 * v[2] * p->dt / p->dz};
    int s[3];
    if (!move_point(p->ndim, off, disp, s)) {
      ++bad;
      continue;
    }
    if (s[0] > 1 || s[0] < -1 || s[1] > 1 || s[1] < -1 || s[2] > 1 || s[2] < -1)
      ++gt1; /* counted once per particle */
    ox[n] = off[0];
    oy[n] = off[1];
    if (p->ndim == 3) oz[n] = off[2];
    cell[n] = (int32_t)cell_of(p, i + s[0], j + s[1], k + s[2]);
  }
  if (diag) {
    diag[0] = K;
    diag[1] = P[0];
    diag[2] = P[1];
    diag[3] = P[2];
  }
  if (st) {
    st->moved_gt1 += gt1;
    st->nonfinite += bad;
  }
}

/* ------------------------------------------------------------ sort ----- */

/* Counting sort: histogram of keys, exclusive prefix sum, then a scatter in
   input order so equal keys keep their input order (stable). */
void orc_sort(const orc_params* p, int64_t np, const int32_t* key, int64_t* perm,
              int32_t* cell_start) {
  int64_t nc = ncell_of(p);
  int64_t* count = (int64_t*)calloc((size_t)nc + 1, sizeof(int64_t));
  for (int64_t n = 0; n < np; ++n) count[key[n]] += 1;
  int64_t run = 0;
  for (int64_t c = 0; c < nc; ++c) {
    int64_t here = count[c];
    cell_start[c] = (int32_t)run;
    count[c] = run; /* becomes the write cursor of cell c */
    run += here;
  }
  cell_start[nc] = (int32_t)run;
  for (int64_t n = 0; n < np; ++n) perm[count[key[n]]++] = n;
  free(count);
}

/* --------------------------------------------------------- deposit ----- */

/* Adds weight W of a particle of charge weight qw and velocity u to cell c. */
static void accumulate(int64_t nc, double* n, double* J, int64_t c, double qwV, double W,
                       const double u[3]) {
  n[c] += qwV * W;
  J[c] += qwV * W * u[0];
  J[c + nc] += qwV * W * u[1];
  J[c + 2 * nc] += qwV * W * u[2];
}

/* Moments at x - half_dt_back v.  NGP (eq:ngp): n = q w / V_c in the cell,
   J = q w u / V_c.  QS (eq:quad, 7 cells):
     centre (3 - dx^2 - dy^2 - dz^2)/6, i+-1: (1 +- dx)^2/12, likewise j, k,
   each times q w / V_c for n and additionally times u for J (the current
   carries the density weight times the particle velocity).  In 2D the k+-1
   cells are the centre cell (nz = 1) and dz = 0. */
void orc_deposit(const orc_params* p, int64_t np, const int32_t* cell, const double* ox,
                 const double* oy, const double* oz, const double* ux, const double* uy,
                 const double* uz, const double* w, double half_dt_back, double* n,
                 double* J) {
  int64_t nc = ncell_of(p);
  memset(n, 0, sizeof(double) * (size_t)nc);
  memset(J, 0, sizeof(double) * 3 * (size_t)nc);
  double V = cell_volume(p);
  for (int64_t q = 0; q < np; ++q) {
    double u[3] = {ux[q], uy[q], uz[q]};
    int i, j, k;
    ijk_of(p, cell[q], &i, &j, &k);
    /* x^{n+1/2} = x^{n+1} - (dt/2) v^{n+1/2}, re-indexed like a move (a
       non-finite or runaway back step deposits at x itself). */
    double off[3] = {ox[q], oy[q], (p->ndim == 3) ? oz[q] : 0.0};
    double disp[3] = {-2.0 * half_dt_back * u[0] / p->dx, -2.0 * half_dt_back * u[1] / p->dy,
                      -2.0 * half_dt_back * u[2] / p->dz};
    int s[3];
    move_point(p->ndim, off, disp, s);
    i += s[0];
    j += s[1];
    k += s[2];
    double dx = off[0], dy = off[1], dz = off[2];
    double qwV = p->qs * w[q] / V;
    if (p->shape == ORC_SHAPE_NGP) {
      accumulate(nc, n, J, cell_of(p, i, j, k), qwV, 1.0, u);
      continue;
    }
    accumulate(nc, n, J, cell_of(p, i, j, k), qwV, (3.0 - dx * dx - dy * dy - dz * dz) / 6.0, u);
    accumulate(nc, n, J, cell_of(p, i + 1, j, k), qwV, (1.0 + dx) * (1.0 + dx) / 12.0, u);
    accumulate(nc, n, J, cell_of(p, i, j + 1, k), qwV, (1.0 + dy) * (1.0 + dy) / 12.0, u);
    accumulate(nc, n, J, cell_of(p, i, j, k + 1), qwV, (1.0 + dz) * (1.0 + dz) / 12.0, u);
    accumulate(nc, n, J, cell_of(p, i - 1, j, k), qwV, (1.0 - dx) * (1.0 - dx) / 12.0, u);
    accumulate(nc, n, J, cell_of(p, i, j - 1, k), qwV, (1.0 - dy) * (1.0 - dy) / 12.0, u);
    accumulate(nc, n, J, cell_of(p, i, j, k - 1), qwV, (1.0 - dz) * (1.0 - dz) / 12.0, u);
  }
}

/* ------------------------------------------------------- smoothing ----- */

/* One pass = the (1,2,1)/4 binomial filter along x, then y, then z (an axis of
   one cell is left unchanged, since its neighbours are the cell itself). */
void orc_smooth(const orc_params* p, double* F, int32_t ncomp, int32_t npasses) {
  int64_t nc = ncell_of(p);
  double* tmp = (double*)malloc(sizeof(double) * (size_t)nc);
  for (int pass = 0; pass < npasses; ++pass)
    for (int comp = 0; comp < ncomp; ++comp) {
      double* Q = F + comp * nc;
      for (int a = 0; a < 3; ++a) {
        int di = a == 0, dj = a == 1, dk = a == 2;
        for (int64_t c = 0; c < nc; ++c) {
          int i, j, k;
          ijk_of(p, c, &i, &j, &k);
          tmp[c] = 0.25 * (Q[cell_of(p, i - di, j - dj, k - dk)] + 2.0 * Q[c] +
                           Q[cell_of(p, i + di, j + dj, k + dk)]);
        }
        memcpy(Q, tmp, sizeof(double) * (size_t)nc);
      }
    }
  free(tmp);
}

/* ------------------------------------------------------------ fields --- */

void orc_curl(const orc_params* p, const double* A, double* C) {
  int64_t nc = ncell_of(p);
  const double *Ax = A, *Ay = A + nc, *Az = A + 2 * nc;
  for (int64_t c = 0; c < nc; ++c) {
    int i, j, k;
    ijk_of(p, c, &i, &j, &k);
    C[c] = dcentred(p, Az, 1, i, j, k) - dcentred(p, Ay, 2, i, j, k);
    C[c + nc] = dcentred(p, Ax, 2, i, j, k) - dcentred(p, Az, 0, i, j, k);
    C[c + 2 * nc] = dcentred(p, Ay, 0, i, j, k) - dcentred(p, Ax, 1, i, j, k);
  }
}

/* Compact second difference of scalar Q along axis a at (i,j,k):
   (Q_{+1} - 2 Q + Q_{-1}) / Delta_a^2 (an axis of one cell gives 0). */
static double d2(const orc_params* p, const double* Q, int a, int i, int j, int k) {
  int di = a == 0, dj = a == 1, dk = a == 2;
  double h = a == 0 ? p->dx : (a == 1 ? p->dy : p->dz);
  return (Q[cell_of(p, i + di, j + dj, k + dk)] - 2.0 * Q[cell_of(p, i, j, k)] +
          Q[cell_of(p, i - di, j - dj, k - dk)]) / (h * h);
}

/* Laplacian as the sum of the compact second differences (the reading of
   nabla^2 in the hyper-resistive term and in div(kappa grad T_e)). */
static double lap(const orc_params* p, const double* Q, int i, int j, int k) {
  return d2(p, Q, 0, i, j, k) + d2(p, Q, 1, i, j, k) + d2(p, Q, 2, i, j, k);
}

/* Ohm's law (eq:ohm) with mu0 J = curl B (low-frequency Ampere), the density
   floor n_e <- max(n_e, n_f) applied to every use of the density, a given
   electron pressure and R_ei = eta J - eta_h lap J:
     E = -grad(p_e)/n_e - u_i x B + (J x B)/n_e + eta J - eta_h lap J,
   u_i = J_i / n_e. */
void orc_ohm_pe(const orc_params* p, const double* B, const double* n, const double* Ji,
                const double* pe, double* E) {
  int64_t nc = ncell_of(p);
  double* J = (double*)malloc(sizeof(double) * 3 * (size_t)nc);
  orc_curl(p, B, J);
  for (int64_t c = 0; c < nc; ++c) {
    int i, j, k;
    ijk_of(p, c, &i, &j, &k);
    double ne = n[c] > p->n_floor ? n[c] : p->n_floor;
    double b[3] = {B[c], B[c + nc], B[c + 2 * nc]};
    double jt[3] = {J[c], J[c + nc], J[c + 2 * nc]};
    double ui[3] = {Ji[c] / ne, Ji[c + nc] / ne, Ji[c + 2 * nc] / ne};
    double gp[3] = {dcentred(p, pe, 0, i, j, k), dcentred(p, pe, 1, i, j, k),
                    dcentred(p, pe, 2, i, j, k)};
    double uxb[3] = {ui[1] * b[2] - ui[2] * b[1], ui[2] * b[0] - ui[0] * b[2],
                     ui[0] * b[1] - ui[1] * b[0]};
    double jxb[3] = {jt[1] * b[2] - jt[2] * b[1], jt[2] * b[0] - jt[0] * b[2],
                     jt[0] * b[1] - jt[1] * b[0]};
    for (int a = 0; a < 3; ++a) {
      double hyper = p->eta_h != 0.0 ? p->eta_h * lap(p, J + a * nc, i, j, k) : 0.0;
      E[c + a * nc] = -gp[a] / ne - uxb[a] + jxb[a] / ne + p->eta * jt[a] - hyper;
    }
  }
  free(J);
}

/* The EOS p_e = n0 te (n_e/n0)^gamma (Sec. II.A) of the floored density. */
static void eos_pressure(const orc_params* p, const double* n, double* pe) {
  int64_t nc = ncell_of(p);
  for (int64_t c = 0; c < nc; ++c) {
    double ne = n[c] > p->n_floor ? n[c] : p->n_floor;
    pe[c] = p->n0 * p->te * pow(ne / p->n0, p->gamma_e);
  }
}

void orc_ohm(const orc_params* p, const double* B, const double* n, const double* Ji,
             double* E) {
  int64_t nc = ncell_of(p);
  double* pe = (double*)malloc(sizeof(double) * (size_t)nc);
  eos_pressure(p, n, pe);
  orc_ohm_pe(p, B, n, Ji, pe, E);
  free(pe);
}

/* Electron energy equation (eq:dpdt) with H_ei = 0 and Q_e = -kappa0 grad T_e:
     dp_e/dt = -gamma div(p_e u_e) + (gamma-1) u_e.grad p_e
               + (gamma-1) kappa0 lap T_e,
   u_e = -(curl B - J_i)/n_e (massless electrons, e = mu0 = 1), T_e = p_e/n_e,
   n_e floored.  The divergence and gradient are centred differences, the
   conduction term the compact Laplacian (a constant kappa0 makes
   div(kappa0 grad T) = kappa0 lap T). */
void orc_pe_rate(const orc_params* p, const double* B, const double* n, const double* Ji,
                 const double* pe, double* rate) {
  int64_t nc = ncell_of(p);
  double g = p->gamma_e;
  double* J = (double*)malloc(sizeof(double) * 3 * (size_t)nc);
  double* ue = (double*)malloc(sizeof(double) * 3 * (size_t)nc);
  double* flux = (double*)malloc(sizeof(double) * 3 * (size_t)nc);
  double* T = (double*)malloc(sizeof(double) * (size_t)nc);
  orc_curl(p, B, J);
  for (int64_t c = 0; c < nc; ++c) {
    double ne = n[c] > p->n_floor ? n[c] : p->n_floor;
    for (int a = 0; a < 3; ++a) {
      ue[c + a * nc] = (Ji[c + a * nc] - J[c + a * nc]) / ne;
      flux[c + a * nc] = pe[c] * ue[c + a * nc];
    }
    T[c] = pe[c] / ne;
  }
  for (int64_t c = 0; c < nc; ++c) {
    int i, j, k;
    ijk_of(p, c, &i, &j, &k);
    double div = 0.0, adv = 0.0;
    for (int a = 0; a < 3; ++a) {
      div += dcentred(p, flux + a * nc, a, i, j, k);
      adv += ue[c + a * nc] * dcentred(p, pe, a, i, j, k);
    }
    rate[c] = -g * div + (g - 1.0) * adv + (g - 1.0) * p->kappa0 * lap(p, T, i, j, k);
  }
  free(J);
  free(ue);
  free(flux);
  free(T);
}

/* Field and electron energies of the state a field advance leaves behind:
     W_B  = 1/2 sum |B|^2 V_c               (magnetic energy, mu0 = 1)
     W_dB = 1/2 sum |B - <B>|^2 V_c          (energy of the fluctuations)
     W_e  = electron internal energy of the density n the call's E was formed
            from, with the floor applied as in Ohm's law:
              gamma = 1:  te sum n ln(n/n0) V_c   (isothermal free energy)
              else:       sum p_e V_c / (gamma - 1),  p_e = n0 te (n/n0)^gamma.
   W_e is the electron term of the energy budget of the hybrid equations
   (Sec. II.A): with eq:ohm, Ampere and Faraday the pressure work -u_e . grad p_e
   is the time derivative of exactly this energy (electron continuity).  With
   an evolved pressure pe (energy equation) W_e = sum p_e V / (gamma - 1). */
static void field_energy(const orc_params* p, const double* B, const double* n,
                         const double* pe, double diag[3]) {
  int64_t nc = ncell_of(p);
  double V = cell_volume(p);
  double mean[3] = {0, 0, 0}, wb = 0.0, wdb = 0.0, we = 0.0;
  for (int a = 0; a < 3; ++a) {
    for (int64_t c = 0; c < nc; ++c) mean[a] += B[c + a * nc];
    mean[a] /= (double)nc;
  }
  for (int a = 0; a < 3; ++a)
    for (int64_t c = 0; c < nc; ++c) {
      double b = B[c + a * nc];
      wb += 0.5 * b * b * V;
      wdb += 0.5 * (b - mean[a]) * (b - mean[a]) * V;
    }
  for (int64_t c = 0; c < nc; ++c) {
    double ne = n[c] > p->n_floor ? n[c] : p->n_floor;
    if (pe)
      we += pe[c] * V / (p->gamma_e - 1.0);
    else if (p->gamma_e == 1.0)
      we += p->te * ne * log(ne / p->n0) * V;
    else
      we += p->n0 * p->te * pow(ne / p->n0, p->gamma_e) * V / (p->gamma_e - 1.0);
  }
  diag[0] = wb;
  diag[1] = wdb;
  diag[2] = we;
}

/* Faraday dB/dt = -curl E, subcycled nsub times per particle step (Sec. II.A).
   Each substep of length h = dt/nsub is the explicit midpoint rule with the
   moments held at their n+1/2 values:
     Ea = Ohm(B),  B* = B - (h/2) curl Ea,  Eb = Ohm(B*),  B <- B - h curl Eb.
   After the subcycle J_i is extrapolated (Sec. II.B)
     J^{n+1} = 3/2 J^{n+1/2} - 1/2 J^{n-1/2}
   and n the same way, and E^{n+1} = Ohm(B^{n+1}, n^{n+1}, J^{n+1}). */
void orc_field_advance(const orc_params* p, double* B, const double* n_half,
                       const double* J_half, const double* n_prev, const double* J_prev,
                       double* E_out, int32_t mode, double diag[3], orc_status* st) {
  int64_t nc = ncell_of(p);
  if (st)
    for (int64_t c = 0; c < nc; ++c)
      if (n_half[c] < p->n_floor) st->floor_hits += 1;
  if (mode == 1) {
    orc_ohm(p, B, n_half, J_half, E_out);
    if (diag) field_energy(p, B, n_half, NULL, diag);
    return;
  }
  size_t v3 = sizeof(double) * 3 * (size_t)nc;
  double* Ea = (double*)malloc(v3);
  double* C = (double*)malloc(v3);
  double* Bs = (double*)malloc(v3);
  double h = p->dt / p->nsub;
  for (int m = 0; m < p->nsub; ++m) {
    orc_ohm(p, B, n_half, J_half, Ea);
    orc_curl(p, Ea, C);
    for (int64_t c = 0; c < 3 * nc; ++c) Bs[c] = B[c] - 0.5 * h * C[c];
    orc_ohm(p, Bs, n_half, J_half, Ea);
    orc_curl(p, Ea, C);
    for (int64_t c = 0; c < 3 * nc; ++c) B[c] = B[c] - h * C[c];
  }
  double* n1 = (double*)malloc(sizeof(double) * (size_t)nc);
  for (int64_t c = 0; c < nc; ++c) n1[c] = 1.5 * n_half[c] - 0.5 * n_prev[c];
  for (int64_t c = 0; c < 3 * nc; ++c) Bs[c] = 1.5 * J_half[c] - 0.5 * J_prev[c];
  orc_ohm(p, B, n1, Bs, E_out);
  if (diag) field_energy(p, B, n1, NULL, diag);
  free(n1);
  free(Ea);
  free(C);
  free(Bs);
}

/* Field advance with the electron energy equation: the state (B, p_e) is
   advanced by the same explicit midpoint rule per substep, with the moments
   held at n+1/2 (eq:dpdt is integrated within the loop of the magnetic
   field, Sec. II.A):
     Ea = Ohm(B, p_e), Ra = rate(B, p_e),
     B* = B - (h/2) curl Ea, p_e* = p_e + (h/2) Ra,
     Eb = Ohm(B*, p_e*), Rb = rate(B*, p_e*),
     B <- B - h curl Eb, p_e <- p_e + h Rb;
   then E^{n+1} = Ohm(B^{n+1}, n^{n+1}, J^{n+1}, p_e^{n+1}) with the moments
   extrapolated as in orc_field_advance. */
void orc_field_advance_pe(const orc_params* p, double* B, double* pe, const double* n_half,
                          const double* J_half, const double* n_prev, const double* J_prev,
                          double* E_out, int32_t mode, double diag[3], orc_status* st) {
  int64_t nc = ncell_of(p);
  if (st)
    for (int64_t c = 0; c < nc; ++c)
      if (n_half[c] < p->n_floor) st->floor_hits += 1;
  if (mode == 1) {
    orc_ohm_pe(p, B, n_half, J_half, pe, E_out);
    if (diag) field_energy(p, B, n_half, pe, diag);
    return;
  }
  size_t v3 = sizeof(double) * 3 * (size_t)nc, v1 = sizeof(double) * (size_t)nc;
  double* Ea = (double*)malloc(v3);
  double* C = (double*)malloc(v3);
  double* Bs = (double*)malloc(v3);
  double* R = (double*)malloc(v1);
  double* ps = (double*)malloc(v1);
  double h = p->dt / p->nsub;
  for (int m = 0; m < p->nsub; ++m) {
    orc_ohm_pe(p, B, n_half, J_half, pe, Ea);
    orc_pe_rate(p, B, n_half, J_half, pe, R);
    orc_curl(p, Ea, C);
    for (int64_t c = 0; c < 3 * nc; ++c) Bs[c] = B[c] - 0.5 * h * C[c];
    for (int64_t c = 0; c < nc; ++c) ps[c] = pe[c] + 0.5 * h * R[c];
    orc_ohm_pe(p, Bs, n_half, J_half, ps, Ea);
    orc_pe_rate(p, Bs, n_half, J_half, ps, R);
    orc_curl(p, Ea, C);
    for (int64_t c = 0; c < 3 * nc; ++c) B[c] = B[c] - h * C[c];
    for (int64_t c = 0; c < nc; ++c) pe[c] = pe[c] + h * R[c];
  }
  double* n1 = (double*)malloc(v1);
  for (int64_t c = 0; c < nc; ++c) n1[c] = 1.5 * n_half[c] - 0.5 * n_prev[c];
  for (int64_t c = 0; c < 3 * nc; ++c) Bs[c] = 1.5 * J_half[c] - 0.5 * J_prev[c];
  orc_ohm_pe(p, B, n1, Bs, pe, E_out);
  if (diag) field_energy(p, B, n1, pe, diag);
  free(n1);
  free(Ea);
  free(C);
  free(Bs);
  free(R);
  free(ps);
}

/* ------------------------------------------------------------------------
 * Open boundaries in x (Sec. II.C), 2D.  The grid's columns 0 and nx-1 are
 * ghost columns outside the domain.  B = B0 + B1 with B0 fixed (a vacuum
 * field: curl B0 = 0) and only B1 advanced; the plasma current of the Hall
 * and resistive terms is J = curl B1.  B1 and the moments in a ghost cell
 * equal their interior neighbour; Ohm's law in a ghost cell keeps the
 * gradients along the boundary and drops those normal to it.  A layer of
 * buffer_cells cells at each open boundary has eta_h raised by
 * eta_h_buffer, ramping linearly to zero inward.  Ions in a ghost column
 * are absorbed; fresh ions enter through the faces from a drifting
 * Maxwellian, with the flux-weighted distribution of the normal velocity.
 * ------------------------------------------------------------------------ */

static int ghost_col(const orc_params* p, int i) {
  return p->open_x && (i == 0 || i == p->nx - 1);
}

void orc_open_fill(const orc_params* p, double* F, int32_t ncomp) {
  if (!p->open_x) return;
  int64_t nc = ncell_of(p);
  for (int a = 0; a < ncomp; ++a)
    for (int k = 0; k < p->nz; ++k)
      for (int j = 0; j < p->ny; ++j) {
        double* f = F + a * nc;
        f[cell_of(p, 0, j, k)] = f[cell_of(p, 1, j, k)];
        f[cell_of(p, p->nx - 1, j, k)] = f[cell_of(p, p->nx - 2, j, k)];
      }
}

/* centred difference, zero along x in a ghost column */
static double dopen(const orc_params* p, const double* Q, int a, int i, int j, int k) {
  if (a == 0 && ghost_col(p, i)) return 0.0;
  return dcentred(p, Q, a, i, j, k);
}

static double lap_open(const orc_params* p, const double* Q, int i, int j, int k) {
  double r = d2(p, Q, 1, i, j, k) + d2(p, Q, 2, i, j, k);
  if (!ghost_col(p, i)) r += d2(p, Q, 0, i, j, k);
  return r;
}

void orc_open_curl(const orc_params* p, const double* A, double* C) {
  int64_t nc = ncell_of(p);
  const double *Ax = A, *Ay = A + nc, *Az = A + 2 * nc;
  for (int64_t c = 0; c < nc; ++c) {
    int i, j, k;
    ijk_of(p, c, &i, &j, &k);
    C[c] = dopen(p, Az, 1, i, j, k) - dopen(p, Ay, 2, i, j, k);
    C[c + nc] = dopen(p, Ax, 2, i, j, k) - dopen(p, Az, 0, i, j, k);
    C[c + 2 * nc] = dopen(p, Ay, 0, i, j, k) - dopen(p, Ax, 1, i, j, k);
  }
}

/* eta_h at column i: the buffer adds eta_h_buffer * (1 - d/w), d the
   column's distance in cells from the outermost interior column */
static double eta_h_at(const orc_params* p, int i) {
  double e = p->eta_h;
  if (p->open_x && p->buffer_cells > 0) {
    int d = i < p->nx - 1 - i ? i : p->nx - 1 - i;  /* ghost: 0, first interior: 1 */
    d = d > 0 ? d - 1 : 0;
    if (d < p->buffer_cells) e += p->eta_h_buffer * (1.0 - (double)d / p->buffer_cells);
  }
  return e;
}

void orc_open_ohm(const orc_params* p, const double* B0, const double* B1, const double* n,
                  const double* Ji, double* E) {
  int64_t nc = ncell_of(p);
  double* J = (double*)malloc(sizeof(double) * 3 * (size_t)nc);
  double* pe = (double*)malloc(sizeof(double) * (size_t)nc);
  orc_open_curl(p, B1, J);
  eos_pressure(p, n, pe);
  for (int64_t c = 0; c < nc; ++c) {
    int i, j, k;
    ijk_of(p, c, &i, &j, &k);
    double ne = n[c] > p->n_floor ? n[c] : p->n_floor;
    double b[3] = {B0[c] + B1[c], B0[c + nc] + B1[c + nc], B0[c + 2 * nc] + B1[c + 2 * nc]};
    double jt[3] = {J[c], J[c + nc], J[c + 2 * nc]};
    double ui[3] = {Ji[c] / ne, Ji[c + nc] / ne, Ji[c + 2 * nc] / ne};
    double gp[3] = {dopen(p, pe, 0, i, j, k), dopen(p, pe, 1, i, j, k), dopen(p, pe, 2, i, j, k)};
    double uxb[3] = {ui[1] * b[2] - ui[2] * b[1], ui[2] * b[0] - ui[0] * b[2],
                     ui[0] * b[1] - ui[1] * b[0]};
    double jxb[3] = {jt[1] * b[2] - jt[2] * b[1], jt[2] * b[0] - jt[0] * b[2],
                     jt[0] * b[1] - jt[1] * b[0]};
    double eh = eta_h_at(p, i);
    for (int a = 0; a < 3; ++a) {
      double hyper = eh != 0.0 ? eh * lap_open(p, J + a * nc, i, j, k) : 0.0;
      E[c + a * nc] = -gp[a] / ne - uxb[a] + jxb[a] / ne + p->eta * jt[a] - hyper;
    }
  }
  free(J);
  free(pe);
}

/* W_B, W_dB of the total B and W_e over the interior cells */
static void open_energy(const orc_params* p, const double* B, const double* n, double diag[3]) {
  int64_t nc = ncell_of(p);
  double V = cell_volume(p), wb = 0.0, we = 0.0, sum[3] = {0.0, 0.0, 0.0};
  int64_t cnt = 0;
  for (int64_t c = 0; c < nc; ++c) {
    int i, j, k;
    ijk_of(p, c, &i, &j, &k);
    if (ghost_col(p, i)) continue;
    ++cnt;
    for (int a = 0; a < 3; ++a) {
      wb += 0.5 * B[c + a * nc] * B[c + a * nc] * V;
      sum[a] += B[c + a * nc];
    }
    double ne = n[c] > p->n_floor ? n[c] : p->n_floor;
    if (p->gamma_e == 1.0)
      we += p->te * ne * log(ne / p->n0) * V;
    else
      we += p->n0 * p->te * pow(ne / p->n0, p->gamma_e) * V / (p->gamma_e - 1.0);
  }
  double m2 = sum[0] * sum[0] + sum[1] * sum[1] + sum[2] * sum[2];
  diag[0] = wb;
  diag[1] = wb - 0.5 * V * m2 / (double)cnt;
  diag[2] = we;
}

void orc_open_field_advance(const orc_params* p, const double* B0, double* B1,
                            const double* n_half, const double* J_half, const double* n_prev,
                            const double* J_prev, double* E_out, double* Btot, int32_t mode,
                            double diag[3], orc_status* st) {
  int64_t nc = ncell_of(p);
  if (st)
    for (int64_t c = 0; c < nc; ++c)
      if (n_half[c] < p->n_floor) st->floor_hits += 1;
  size_t v3 = sizeof(double) * 3 * (size_t)nc;
  double* n1 = (double*)malloc(sizeof(double) * (size_t)nc);
  double* J1 = (double*)malloc(v3);
  if (mode == 0) {
    double* Ea = (double*)malloc(v3);
    double* C = (double*)malloc(v3);
    double* Bs = (double*)malloc(v3);
    double h = p->dt / p->nsub;
    orc_open_fill(p, B1, 3);
    for (int m = 0; m < p->nsub; ++m) {
      orc_open_ohm(p, B0, B1, n_half, J_half, Ea);
      orc_open_curl(p, Ea, C);
      for (int64_t c = 0; c < 3 * nc; ++c) Bs[c] = B1[c] - 0.5 * h * C[c];
      orc_open_fill(p, Bs, 3);
      orc_open_ohm(p, B0, Bs, n_half, J_half, Ea);
      orc_open_curl(p, Ea, C);
      for (int64_t c = 0; c < 3 * nc; ++c) B1[c] = B1[c] - h * C[c];
      orc_open_fill(p, B1, 3);
    }
    for (int64_t c = 0; c < nc; ++c) n1[c] = 1.5 * n_half[c] - 0.5 * n_prev[c];
    for (int64_t c = 0; c < 3 * nc; ++c) J1[c] = 1.5 * J_half[c] - 0.5 * J_prev[c];
    free(Ea);
    free(C);
    free(Bs);
  } else {
    for (int64_t c = 0; c < nc; ++c) n1[c] = n_half[c];
    for (int64_t c = 0; c < 3 * nc; ++c) J1[c] = J_half[c];
  }
  orc_open_ohm(p, B0, B1, n1, J1, E_out);
  for (int64_t c = 0; c < 3 * nc; ++c) Btot[c] = B0[c] + B1[c];
  if (diag) open_energy(p, Btot, n1, diag);
  free(n1);
  free(J1);
}

int64_t orc_open_absorb(const orc_params* p, int64_t np, int32_t* cell) {
  int64_t nc = ncell_of(p), k = 0;
  for (int64_t q = 0; q < np; ++q) {
    int i, j, kk;
    ijk_of(p, cell[q], &i, &j, &kk);
    if (ghost_col(p, i)) {
      cell[q] = (int32_t)nc;
      ++k;
    }
  }
  return k;
}

/* splitmix64's finaliser (Steele, Lea & Flood 2014) */
static uint64_t mix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

double orc_uniform(uint64_t seed, uint64_t ctr) {
  return (double)(mix64(seed + mix64(ctr)) >> 11) * (1.0 / 9007199254740992.0);
}

/* counter of draw d of ion m of row r = j + ny k of face f at a step */
static uint64_t draw_ctr(int64_t step, int f, int j, int64_t m, int d) {
  return ((((uint64_t)step * 2u + (uint64_t)f) << 16 | (uint64_t)j) << 20 | (uint64_t)m) << 7 |
         (uint64_t)d;
}

/* a standard normal from draws d and d+1 (Box-Muller) */
static double normal_draw(uint64_t seed, int64_t step, int f, int j, int64_t m, int d) {
  double u1 = orc_uniform(seed, draw_ctr(step, f, j, m, d));
  double u2 = orc_uniform(seed, draw_ctr(step, f, j, m, d + 1));
  return sqrt(-2.0 * log(1.0 - u1)) * cos(6.283185307179586 * u2);
}

/* flux per unit density into the domain of a drifting Maxwellian with
   normal drift u (into the domain) and thermal speed vth:
   integral over v > 0 of v f(v) dv */
static double inflow_flux(double u, double vth) {
  return vth / sqrt(2.0 * 3.141592653589793) * exp(-0.5 * u * u / (vth * vth)) +
         0.5 * u * (1.0 + erf(u / (sqrt(2.0) * vth)));
}

/* integral over 0 < t < v of t exp(-(t-u)^2 / (2 vth^2)) dt, in closed form:
   with x = (t-u)/(sqrt(2) vth) it is
   vth u sqrt(pi/2) [erf(x1) - erf(x0)] + vth^2 [exp(-x0^2) - exp(-x1^2)] */
static double flux_integral(double u, double vth, double v) {
  double x0 = -u / (sqrt(2.0) * vth), x1 = (v - u) / (sqrt(2.0) * vth);
  return vth * u * sqrt(0.5 * 3.141592653589793) * (erf(x1) - erf(x0)) +
         vth * vth * (exp(-x0 * x0) - exp(-x1 * x1));
}

/* the speed v > 0 at which the distribution function of v exp(-(v-u)^2 /
   (2 vth^2)) reaches U: 60 bisection steps on [0, max(u, 0) + 10 vth] */
static double inflow_speed(double u, double vth, double U) {
  double lo = 0.0, hi = (u > 0.0 ? u : 0.0) + 10.0 * vth;
  double target = U * flux_integral(u, vth, hi);
  for (int it = 0; it < 60; ++it) {
    double mid = 0.5 * (lo + hi);
    if (flux_integral(u, vth, mid) < target)
      lo = mid;
    else
      hi = mid;
  }
  return 0.5 * (lo + hi);
}

double orc_inflow_expected(const orc_params* p, const orc_inflow* in, int32_t face) {
  double un = face == 0 ? in->ux : -in->ux;
  /* n F dt dy dz ions of weight n dx dy dz / ppc */
  return in->ppc * p->dt / p->dx * inflow_flux(un, in->vth);
}

int64_t orc_open_inject(const orc_params* p, const orc_inflow* in, uint64_t seed, int64_t step,
                        int64_t np, int64_t cap, int32_t* cell, double* ox, double* oy,
                        double* oz, double* ux, double* uy, double* uz, double* w) {
  double wb = in->n * p->dx * p->dy * p->dz / in->ppc;
  int rows = p->ny * p->nz;
  for (int f = 0; f < 2; ++f) {
    if (!((in->faces >> f) & 1)) continue;
    double un = f == 0 ? in->ux : -in->ux;
    double nexp = orc_inflow_expected(p, in, f);
    int col = f == 0 ? 1 : p->nx - 2;
    for (int r = 0; r < rows; ++r) {
      int j = r % p->ny, k = r / p->ny;
      int64_t cnt = (int64_t)floor(nexp + orc_uniform(seed, draw_ctr(step, f, r, 0, 127)));
      for (int64_t m = 0; m < cnt && np < cap; ++m) {
        /* normal speed: drifting Maxwellian weighted by v (v > 0), by
           inverting its distribution function at a uniform draw */
        double v = inflow_speed(un, in->vth, orc_uniform(seed, draw_ctr(step, f, r, m, 0)));
        double vy = in->uy + in->vth * normal_draw(seed, step, f, r, m, 96);
        double vz = in->uz + in->vth * normal_draw(seed, step, f, r, m, 98);
        /* entered at a uniform time within the step: depth v dt tau */
        double s = v * p->dt * orc_uniform(seed, draw_ctr(step, f, r, m, 100));
        double o = -1.0 + 2.0 * s / p->dx;
        if (o >= 1.0) o = 1.0 - 1e-7;
        /* the store holds FP32 values: the injected ion is what FP32 keeps */
        double xo = f == 0 ? o : -o;
        if (xo >= 1.0) xo = 1.0 - 1e-7;
        cell[np] = (int32_t)cell_of(p, col, j, k);
        ox[np] = (double)(float)xo;
        if (ox[np] >= 1.0) ox[np] = (double)nextafterf(1.0f, 0.0f);
        oy[np] = (double)(float)(-1.0 + 2.0 * orc_uniform(seed, draw_ctr(step, f, r, m, 101)));
        if (oy[np] >= 1.0) oy[np] = (double)nextafterf(1.0f, 0.0f);
        if (p->ndim == 3 && oz) {
          oz[np] = (double)(float)(-1.0 + 2.0 * orc_uniform(seed, draw_ctr(step, f, r, m, 102)));
          if (oz[np] >= 1.0) oz[np] = (double)nextafterf(1.0f, 0.0f);
        }
        ux[np] = (double)(float)(f == 0 ? v : -v);
        uy[np] = (double)(float)vy;
        uz[np] = (double)(float)vz;
        w[np] = (double)(float)wb;
        ++np;
      }
    }
  }
  return np;
}
