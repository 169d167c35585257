// Open boundaries in x for 2D runs (libhvpic.so, gfx950).
//
// Method (arXiv 2305.05600, Sec. II.C): the grid's first and last columns
// are ghost columns outside the domain.  The magnetic field is split
// B = B0 + B1: B0 is a fixed external vacuum field, only B1 is advanced, and
// the plasma current of the Hall and resistive terms is J = curl B1.  In a
// ghost cell B1 and the moments equal their interior neighbour, and Ohm's
// law keeps the gradients along the boundary while dropping those normal to
// it.  A layer of buffer_cells cells at each open boundary has the
// hyper-resistivity raised by eta_h_buffer, ramping to zero inward.  Ions in
// a ghost column are absorbed; fresh ions enter through the faces from a
// drifting Maxwellian with the flux-weighted distribution of the normal
// velocity.
//
// The particle kernels of the periodic step run unchanged on this grid (the
// ghost columns keep the two sides apart); absorbed ions get the key ncell
// and the open sort puts them last.  The field advance is the stencil-per-
// stage form: per RK2 stage the ghost columns are refilled, J = curl B1 (no
// x-derivatives in the ghosts), Ohm's law, then Faraday in the interior.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "fields_common.hpp"

namespace hvpic {
namespace {

struct OpenG {
  FGeo g;
  float ilx, ily, ilz;   // 1/dx^2, 1/dy^2, 1/dz^2
  float eta, eta_h, eta_hb;
  int nbuf;
};

__device__ __forceinline__ bool ghost_col(int i, int nx) { return i == 0 || i == nx - 1; }

__device__ __forceinline__ float eta_h_col(int i, const OpenG& o) {
  float e = o.eta_h;
  if (o.nbuf > 0) {
    int d = min(i, o.g.nx - 1 - i);
    d = d > 0 ? d - 1 : 0;
    if (d < o.nbuf) e += o.eta_hb * (1.0f - (float)d / (float)o.nbuf);
  }
  return e;
}

// ghost cells of ncomp component-major arrays <- their interior neighbours
// (rows = ny nz grid rows along x per component)
__global__ void k_open_fill(float* __restrict__ F, int ncomp, int nx, int rows, int ncell) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncomp * rows) return;
  const int a = t / rows, r = t - (t / rows) * rows;
  float* f = F + (int64_t)a * ncell + (int64_t)r * nx;
  f[0] = f[1];
  f[nx - 1] = f[nx - 2];
}

// 1/n_f, u_i and -grad(p_e)/n_f of the held moments (no x-component of the
// pressure gradient in a ghost cell)
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_open_prep(const float* __restrict__ n,
                                                      const float* __restrict__ Ji, FGeo g,
                                                      Eos eos, Aux aux) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= g.ncell) return;
  const int nc = g.ncell;
  int i, j, k;
  fijk(c, g, i, j, k);
  const Nbr nn = neighbours(c, i, j, k, g);
  const float nf = fmaxf(n[c], eos.nfloor);
  const float inv = (float)(1.0 / (double)nf);
  aux.inv[c] = inv;
  for (int a = 0; a < 3; ++a) aux.u[a * nc + c] = Ji[a * nc + c] * inv;
  auto pres = [&](int q) { return pressure(n[q], eos.nfloor, eos.te_n0, eos.n0, eos.gam, eos.iso); };
  aux.gp[c] = ghost_col(i, g.nx) ? 0.0f : -(pres(nn.xp) - pres(nn.xm)) * g.idx2 * inv;
  aux.gp[nc + c] = -(pres(nn.yp) - pres(nn.ym)) * g.idy2 * inv;
  aux.gp[2 * nc + c] = NDIM == 3 ? -(pres(nn.zp) - pres(nn.zm)) * g.idz2 * inv : 0.0f;
}

// J = curl B1 (B1 = hi + lo with HAS_LO), no x-derivatives in the ghosts
template <int NDIM, bool HAS_LO>
__global__ __launch_bounds__(kBlock) void k_open_curl(const float* __restrict__ Bh,
                                                      const float* __restrict__ Bl,
                                                      float* __restrict__ J, FGeo g) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= g.ncell) return;
  const int nc = g.ncell;
  int i, j, k;
  fijk(c, g, i, j, k);
  const Nbr n = neighbours(c, i, j, k, g);
  const BSum<HAS_LO> B{Bh, Bl};
  const bool gh = ghost_col(i, g.nx);
  const float dyBz = (B(2 * nc + n.yp) - B(2 * nc + n.ym)) * g.idy2;
  const float dyBx = (B(n.yp) - B(n.ym)) * g.idy2;
  const float dxBz = gh ? 0.0f : (B(2 * nc + n.xp) - B(2 * nc + n.xm)) * g.idx2;
  const float dxBy = gh ? 0.0f : (B(nc + n.xp) - B(nc + n.xm)) * g.idx2;
  float dzBy = 0.f, dzBx = 0.f;
  if (NDIM == 3) {
    dzBy = (B(nc + n.zp) - B(nc + n.zm)) * g.idz2;
    dzBx = (B(n.zp) - B(n.zm)) * g.idz2;
  }
  J[c] = dyBz - dzBy;
  J[nc + c] = dzBx - dxBz;
  J[2 * nc + c] = dxBy - dyBx;
}

// lap of component a of J at c (x part dropped in a ghost cell)
template <int NDIM>
__device__ __forceinline__ float lap_open(const float* __restrict__ J, int a, int c, int i,
                                          const Nbr& n, const OpenG& o) {
  const float* q = J + (int64_t)a * o.g.ncell;
  float r = (q[n.yp] + q[n.ym] - 2.0f * q[c]) * o.ily;
  if (!ghost_col(i, o.g.nx)) r += (q[n.xp] + q[n.xm] - 2.0f * q[c]) * o.ilx;
  if (NDIM == 3) r += (q[n.zp] + q[n.zm] - 2.0f * q[c]) * o.ilz;
  return r;
}

// E = (J/n_f - u_i) x (B0 + B1) - grad(p_e)/n_f + eta J - eta_h(x) lap J
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_open_ohm(const float* __restrict__ B0,
                                                     const float* __restrict__ B1,
                                                     const float* __restrict__ J, Aux aux,
                                                     float* __restrict__ E, OpenG o) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= o.g.ncell) return;
  const int nc = o.g.ncell;
  int i, j, k;
  fijk(c, o.g, i, j, k);
  const Nbr n = neighbours(c, i, j, k, o.g);
  const float b0 = B0[c] + B1[c], b1 = B0[nc + c] + B1[nc + c], b2 = B0[2 * nc + c] + B1[2 * nc + c];
  const float j0 = J[c], j1 = J[nc + c], j2 = J[2 * nc + c];
  const float inv = aux.inv[c];
  const float w0 = j0 * inv - aux.u[c], w1 = j1 * inv - aux.u[nc + c],
              w2 = j2 * inv - aux.u[2 * nc + c];
  const float eh = eta_h_col(i, o);
  float h0 = 0.f, h1 = 0.f, h2 = 0.f;
  if (eh != 0.0f) {
    h0 = eh * lap_open<NDIM>(J, 0, c, i, n, o);
    h1 = eh * lap_open<NDIM>(J, 1, c, i, n, o);
    h2 = eh * lap_open<NDIM>(J, 2, c, i, n, o);
  }
  E[c] = (w1 * b2 - w2 * b1) + aux.gp[c] + o.eta * j0 - h0;
  E[nc + c] = (w2 * b0 - w0 * b2) + aux.gp[nc + c] + o.eta * j1 - h1;
  E[2 * nc + c] = (w0 * b1 - w1 * b0) + aux.gp[2 * nc + c] + o.eta * j2 - h2;
}

// B1_dst = B1_base - coef curl E in the interior (compensated into lo_out
// when given, from lo_in, or from zero when lo_in is null), and the ghost
// rule: the threads of the outermost interior cells (i = 1, nx-2) also
// write their values into the ghost cell beside them.  base and lo_in are
// read at the thread's own cell only, and a ghost cell's thread reads and
// writes nothing, so dst may be base and lo_out may be lo_in.
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_open_faraday(const float* __restrict__ E,
                                                         const float* Bbase, float* Bdst,
                                                         const float* lo_in, float* lo_out,
                                                         float coef, FGeo g) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= g.ncell) return;
  int i, j, k;
  fijk(c, g, i, j, k);
  if (ghost_col(i, g.nx)) return;
  const BSum<false> Ea{E, nullptr};
  float ce[3];
  curl_at<NDIM>(Ea, c, g, ce);
  const bool left = i == 1, right = i == g.nx - 2;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int q = a * g.ncell + c;
    const float d = -coef * ce[a];
    const float hi = Bbase[q];
    float t, l = 0.0f;
    if (lo_out) {
      const float y = (lo_in ? lo_in[q] : 0.0f) + d;
      t = hi + y;
      l = y - (t - hi);
      lo_out[q] = l;
    } else {
      t = hi + d;
    }
    Bdst[q] = t;
    if (left) {
      Bdst[q - 1] = t;
      if (lo_out) lo_out[q - 1] = l;
    }
    if (right) {
      Bdst[q + 1] = t;
      if (lo_out) lo_out[q + 1] = l;
    }
  }
}

// E from B1 = Bh (+ Bl), J = curl B1 and the moments n_eff = ca*na + cb*nb,
// J_eff likewise (EXTRAP; otherwise na, Ja), with the open rules; B1out =
// B1 (when non-null), Btot = B0 + B1; per-block FP64 partials over the
// interior cells of {|Btot|^2, Btot, electron energy of n_eff}; the cells of
// na below the floor counted (all columns).
template <int NDIM, bool EXTRAP, bool HAS_LO>
__global__ __launch_bounds__(kBlock) void k_open_final(
    const float* __restrict__ Bh, const float* __restrict__ Bl, const float* __restrict__ J,
    const float* __restrict__ B0, float* __restrict__ B1out, float* __restrict__ Btot,
    const float* __restrict__ na, const float* __restrict__ nb, const float* __restrict__ Ja,
    const float* __restrict__ Jb, float ca, float cb, OpenG o, Eos eos, float* __restrict__ E,
    double* part, Status* st) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  const int nc = o.g.ncell;
  const bool live = c < nc;
  bool below = false;
  double v[kDiagNV] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (live) {
    int i, j, k;
    fijk(c, o.g, i, j, k);
    const Nbr n = neighbours(c, i, j, k, o.g);
    const bool gh = ghost_col(i, o.g.nx);
    auto dens = [&](int q) { return EXTRAP ? ca * na[q] + cb * nb[q] : na[q]; };
    const float n_c = dens(c);
    const BSum<HAS_LO> B1{Bh, Bl};
    const float c0 = B1(c), c1 = B1(nc + c), c2 = B1(2 * nc + c);
    const float b0 = B0[c] + c0, b1 = B0[nc + c] + c1, b2 = B0[2 * nc + c] + c2;
    below = na[c] < eos.nfloor;
    const float inv = (float)(1.0 / (double)fmaxf(n_c, eos.nfloor));
    float u[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      u[a] = (EXTRAP ? ca * Ja[a * nc + c] + cb * Jb[a * nc + c] : Ja[a * nc + c]) * inv;
    auto pres = [&](int q) {
      return pressure(dens(q), eos.nfloor, eos.te_n0, eos.n0, eos.gam, eos.iso);
    };
    const float gp0 = gh ? 0.0f : -(pres(n.xp) - pres(n.xm)) * o.g.idx2 * inv;
    const float gp1 = -(pres(n.yp) - pres(n.ym)) * o.g.idy2 * inv;
    const float gp2 = NDIM == 3 ? -(pres(n.zp) - pres(n.zm)) * o.g.idz2 * inv : 0.0f;
    const float j0 = J[c], j1 = J[nc + c], j2 = J[2 * nc + c];
    const float w0 = j0 * inv - u[0], w1 = j1 * inv - u[1], w2 = j2 * inv - u[2];
    const float eh = eta_h_col(i, o);
    float h0 = 0.f, h1 = 0.f, h2 = 0.f;
    if (eh != 0.0f) {
      h0 = eh * lap_open<NDIM>(J, 0, c, i, n, o);
      h1 = eh * lap_open<NDIM>(J, 1, c, i, n, o);
      h2 = eh * lap_open<NDIM>(J, 2, c, i, n, o);
    }
    E[c] = (w1 * b2 - w2 * b1) + gp0 + o.eta * j0 - h0;
    E[nc + c] = (w2 * b0 - w0 * b2) + gp1 + o.eta * j1 - h1;
    E[2 * nc + c] = (w0 * b1 - w1 * b0) + gp2 + o.eta * j2 - h2;
    if (B1out) {
      B1out[c] = c0;
      B1out[nc + c] = c1;
      B1out[2 * nc + c] = c2;
    }
    Btot[c] = b0;
    Btot[nc + c] = b1;
    Btot[2 * nc + c] = b2;
    if (part && !gh) {
      const double d0 = b0, d1 = b1, d2 = b2;
      v[0] = d0 * d0 + d1 * d1 + d2 * d2;
      v[1] = d0;
      v[2] = d1;
      v[3] = d2;
      v[4] = electron_energy(n_c, eos);
    }
  }
  const uint64_t m = __ballot(live && below);
  if ((threadIdx.x & 63) == 0 && m) {
    atomicOr(&st->flags, (uint32_t)HVPIC_FLAG_FLOOR_HIT);
    atomicAdd(&st->floor_hits, (unsigned long long)__builtin_popcountll(m));
  }
  if (part) block_partial<kDiagNV, kFieldPartStride>(v, part);
}

// ---------------------------------------------------------- particles --

__global__ void k_open_absorb(int32_t* __restrict__ cell, int64_t n, int nx, int ncell) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int c = cell[q];
  if ((unsigned)c >= (unsigned)ncell) return;
  const int i = c % nx;
  if (i == 0 || i == nx - 1) cell[q] = ncell;
}

// splitmix64's finaliser (Steele, Lea & Flood 2014), and the uniform in
// [0, 1) of a counter under a seed: the generator of the injection draws
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
__host__ __device__ __forceinline__ double uniform01(uint64_t seed, uint64_t ctr) {
  return (double)(mix64(seed + mix64(ctr)) >> 11) * (1.0 / 9007199254740992.0);
}
// counter of draw d of ion m of face row r (r = j + ny k) of face f at a step
__host__ __device__ __forceinline__ uint64_t draw_ctr(int64_t step, int f, int r, int64_t m,
                                                      int d) {
  return ((((uint64_t)step * 2u + (uint64_t)f) << 16 | (uint64_t)r) << 20 | (uint64_t)m) << 7 |
         (uint64_t)d;
}

__device__ double normal_draw(uint64_t seed, int64_t step, int f, int r, int64_t m, int d) {
  const double u1 = uniform01(seed, draw_ctr(step, f, r, m, d));
  const double u2 = uniform01(seed, draw_ctr(step, f, r, m, d + 1));
  return sqrt(-2.0 * log(1.0 - u1)) * cos(6.283185307179586 * u2);
}

// integral over 0 < t < v of t exp(-(t - u)^2 / (2 vth^2)) dt (closed form
// in erf and exp of x = (t - u)/(sqrt(2) vth))
__device__ double flux_integral(double u, double vth, double v) {
  const double s2 = 1.4142135623730951 * vth;
  const double x0 = -u / s2, x1 = (v - u) / s2;
  return vth * u * 1.2533141373155003 * (erf(x1) - erf(x0)) +
         vth * vth * (exp(-x0 * x0) - exp(-x1 * x1));
}

// the normal speed whose flux-weighted distribution function is U
__device__ double inflow_speed(double u, double vth, double U) {
  double lo = 0.0, hi = (u > 0.0 ? u : 0.0) + 10.0 * vth;
  const double target = U * flux_integral(u, vth, hi);
  for (int it = 0; it < 60; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (flux_integral(u, vth, mid) < target)
      lo = mid;
    else
      hi = mid;
  }
  return 0.5 * (lo + hi);
}

struct Inject {
  double nexp[2], un[2];
  double uy, uz, vth, dt, dx, w;
  int faces, nx, rows;  // rows = ny nz cells on a face
  uint64_t seed;
  int64_t step, n0;
};

// One block: per (face, row) the count floor(nexp + U) and its exclusive
// prefix over the rows in order (face-major): the injected ions of face f's
// row r are stored from n0 + off[f rows + r].
__global__ __launch_bounds__(1024) void k_open_inject_count(Inject P, int32_t* __restrict__ cnt,
                                                           int32_t* __restrict__ off) {
  __shared__ int32_t s_sum[1024];
  __shared__ int32_t s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  const int rows = 2 * P.rows;
  for (int r0 = 0; r0 < rows; r0 += 1024) {
    const int r = r0 + (int)threadIdx.x;
    int k = 0;
    if (r < rows) {
      const int f = r / P.rows, rr = r - f * P.rows;
      if ((P.faces >> f) & 1)
        k = (int)floor(P.nexp[f] + uniform01(P.seed, draw_ctr(P.step, f, rr, 0, 127)));
    }
    // inclusive scan over the block (Hillis-Steele in LDS)
    s_sum[threadIdx.x] = k;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int add = threadIdx.x >= (unsigned)o ? s_sum[threadIdx.x - o] : 0;
      __syncthreads();
      s_sum[threadIdx.x] += add;
      __syncthreads();
    }
    if (r < rows) {
      cnt[r] = k;
      off[r] = s_carry + s_sum[threadIdx.x] - k;
    }
    const int chunk = s_sum[1023];
    __syncthreads();
    if (threadIdx.x == 0) s_carry += chunk;
    __syncthreads();
  }
}

// One thread per injected ion t < total: its (face, row) slot s is the last
// with off[s] <= t (that slot holds it: off[s+1] = off[s] + cnt[s] > t), its
// rank m = t - off[s]; the ion's draws are those of (step, face, row, m).
// oz is written in 3D only (null in 2D).
__global__ __launch_bounds__(256) void k_open_inject_draw(Inject P, const int32_t* __restrict__ off,
                                                         int64_t total, int32_t* __restrict__ cell,
                                                         float* __restrict__ ox,
                                                         float* __restrict__ oy,
                                                         float* __restrict__ oz,
                                                         float* __restrict__ ux,
                                                         float* __restrict__ uy,
                                                         float* __restrict__ uz,
                                                         float* __restrict__ w) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  int lo = 0, hi = 2 * P.rows - 1;  // off[0] = 0 <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((int64_t)off[mid] <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int f = lo / P.rows, r = lo - f * P.rows;
  const int64_t m = t - off[lo];
  const double v = inflow_speed(P.un[f], P.vth, uniform01(P.seed, draw_ctr(P.step, f, r, m, 0)));
  const double vy = P.uy + P.vth * normal_draw(P.seed, P.step, f, r, m, 96);
  const double vz = P.uz + P.vth * normal_draw(P.seed, P.step, f, r, m, 98);
  const double s = v * P.dt * uniform01(P.seed, draw_ctr(P.step, f, r, m, 100));
  double o = -1.0 + 2.0 * s / P.dx;
  if (o >= 1.0) o = 1.0 - 1e-7;
  double xo = f == 0 ? o : -o;
  if (xo >= 1.0) xo = 1.0 - 1e-7;
  float fx = (float)xo;
  if (fx >= 1.0f) fx = 0.99999994f;
  float fy = (float)(-1.0 + 2.0 * uniform01(P.seed, draw_ctr(P.step, f, r, m, 101)));
  if (fy >= 1.0f) fy = 0.99999994f;
  const int64_t q = P.n0 + t;
  // cell (col, j, k) = col + nx (j + ny k) = col + nx r
  cell[q] = (f == 0 ? 1 : P.nx - 2) + P.nx * r;
  ox[q] = fx;
  oy[q] = fy;
  if (oz) {
    float fz = (float)(-1.0 + 2.0 * uniform01(P.seed, draw_ctr(P.step, f, r, m, 102)));
    if (fz >= 1.0f) fz = 0.99999994f;
    oz[q] = fz;
  }
  ux[q] = (float)(f == 0 ? v : -v);
  uy[q] = (float)vy;
  uz[q] = (float)vz;
  w[q] = (float)P.w;
}

// host: the expected count per row and step of a face, and the total of a
// step (the same draws as the kernel, in the same double arithmetic)
double inflow_flux_host(double u, double vth) {
  return vth / sqrt(2.0 * 3.141592653589793) * exp(-0.5 * u * u / (vth * vth)) +
         0.5 * u * (1.0 + erf(u / (sqrt(2.0) * vth)));
}

OpenG open_geo(const hvpic_ctx* c) {
  OpenG o;
  o.g = fgeo(c);
  o.ilx = (float)(1.0 / (c->p.dx * c->p.dx));
  o.ily = (float)(1.0 / (c->p.dy * c->p.dy));
  o.ilz = (float)(1.0 / (c->p.dz * c->p.dz));
  o.eta = (float)c->p.eta;
  o.eta_h = (float)c->p.eta_h;
  o.eta_hb = (float)c->p.eta_h_buffer;
  o.nbuf = c->p.buffer_cells;
  return o;
}

// cells on one open face: the grid rows along x
int face_rows(const hvpic_ctx* c) { return c->p.ny * (c->p.ndim == 3 ? c->p.nz : 1); }

void fill(hvpic_ctx* c, float* F, int ncomp) {
  const int rows = face_rows(c);
  const int t = ncomp * rows;
  hipLaunchKernelGGL(k_open_fill, dim3((unsigned)ceil_div(t, 256)), dim3(256), 0, c->stream, F,
                     ncomp, c->p.nx, rows, c->ncell);
}

bool open_ok(const hvpic_ctx* c) { return c && c->magic == kMagic && c->p.open_x == 1; }

// Checks and the host's count of an injection (the kernel draws the same
// counts): HVPIC_OK with the kernel arguments and the total, else the error
// (nothing launched).
int inject_plan(hvpic_ctx* c, const hvpic_particles* p, const hvpic_inflow* in, uint64_t seed,
                int64_t step, Inject& P, int64_t& total) {
  if (!open_ok(c) || !p || !in || step < 0 || step >= (int64_t(1) << 20)) return HVPIC_EINVAL;
  if (p->n < 0 || p->n > c->p.np_capacity || !p->cell || !p->ox || !p->oy || !p->ux || !p->uy ||
      !p->uz || !p->w || (c->p.ndim == 3 && !p->oz))
    return HVPIC_EINVAL;
  const int rows = face_rows(c);
  if (!(in->n > 0.0) || !(in->vth > 0.0) || !isfinite(in->n) || !isfinite(in->vth) ||
      in->ppc < 1 || !isfinite(in->ux) || !isfinite(in->uy) || !isfinite(in->uz) ||
      in->faces < 0 || in->faces > 3 || rows > 65536)
    return HVPIC_EINVAL;
  for (int f = 0; f < 2; ++f) {
    P.un[f] = f == 0 ? in->ux : -in->ux;
    P.nexp[f] = in->ppc * c->p.dt / c->p.dx * inflow_flux_host(P.un[f], in->vth);
  }
  P.uy = in->uy;
  P.uz = in->uz;
  P.vth = in->vth;
  P.dt = c->p.dt;
  P.dx = c->p.dx;
  P.w = in->n * c->p.dx * c->p.dy * c->p.dz / in->ppc;
  P.faces = in->faces;
  P.nx = c->p.nx;
  P.rows = rows;
  P.seed = seed;
  P.step = step;
  P.n0 = p->n;
  total = 0;
  for (int f = 0; f < 2; ++f) {
    if (!((in->faces >> f) & 1)) continue;
    for (int r = 0; r < rows; ++r) {
      const int64_t k = (int64_t)floor(P.nexp[f] + uniform01(seed, draw_ctr(step, f, r, 0, 127)));
      if (k >= (int64_t(1) << 20)) return HVPIC_EINVAL;  // beyond the counter's ion field
      total += k;
    }
  }
  if (p->n + total > c->p.np_capacity) return HVPIC_ENOMEM;
  return HVPIC_OK;
}

// Enqueues a planned injection and records it for hvpic_sort_open_perm.
void inject_launch(hvpic_ctx* c, hvpic_particles* p, const Inject& P, int64_t total) {
  c->inj_cell = p->cell;
  c->inj_n0 = p->n;
  c->inj_k = total;
  if (total > 0) {
    int32_t* cnt = c->open_rows;
    int32_t* off = c->open_rows + 2 * P.rows;
    float* oz = c->p.ndim == 3 ? p->oz : nullptr;
    hipLaunchKernelGGL(k_open_inject_count, dim3(1), dim3(1024), 0, c->stream, P, cnt, off);
    hipLaunchKernelGGL(k_open_inject_draw, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0,
                       c->stream, P, (const int32_t*)off, total, p->cell, p->ox, p->oy, oz, p->ux,
                       p->uy, p->uz, p->w);
  }
  p->n += total;
}

// the open field advance of one dimension (arguments checked by the caller)
template <int NDIM>
void open_advance(hvpic_ctx* c, const float* B0, float* B1, float* Btot, const float* n_half,
                  const float* J_half, const float* n_prev, const float* J_prev, float* E_out,
                  int mode, double* diag_out) {
  const OpenG o = open_geo(c);
  const FGeo& g = o.g;
  const int nc = c->ncell;
  const dim3 grid((unsigned)ceil_div(nc, kBlock)), blk(kBlock);
  hipStream_t s = c->stream;
  const Eos eos = make_eos(c);
  Aux aux;
  aux.inv = c->fscratch;
  aux.u = c->fscratch + nc;
  aux.gp = c->fscratch + 4ll * nc;
  float* Xh = c->fscratch + 7ll * nc;
  float* Xl = c->fscratch + 10ll * nc;
  float* Yh = c->fscratch + 13ll * nc;
  float* J = c->fscratch + 16ll * nc;
  float* E = c->fscratch + 19ll * nc;
  double* part = diag_out ? c->field_part : nullptr;
  const float* fh = B1;
  const float* fl = nullptr;
  if (mode == 0) fill(c, B1, 3);
  if (mode == 0 && c->p.nsub > 0) {
    const float h = (float)(c->p.dt / c->p.nsub);
    hipLaunchKernelGGL(k_open_prep<NDIM>, grid, blk, 0, s, n_half, J_half, g, eos, aux);
    for (int m = 0; m < c->p.nsub; ++m) {
      // B1 (hi + lo) of the substep: the caller's B1 (lo = 0) at the first
      const float* Xb = m == 0 ? (const float*)B1 : (const float*)Xh;
      const float* Xlb = m == 0 ? nullptr : (const float*)Xl;
      hipLaunchKernelGGL((k_open_curl<NDIM, false>), grid, blk, 0, s, Xb, (const float*)nullptr, J,
                         g);
      hipLaunchKernelGGL(k_open_ohm<NDIM>, grid, blk, 0, s, B0, Xb, (const float*)J, aux, E, o);
      hipLaunchKernelGGL(k_open_faraday<NDIM>, grid, blk, 0, s, (const float*)E, Xb, Yh,
                         (const float*)nullptr, (float*)nullptr, 0.5f * h, g);
      hipLaunchKernelGGL((k_open_curl<NDIM, false>), grid, blk, 0, s, (const float*)Yh,
                         (const float*)nullptr, J, g);
      hipLaunchKernelGGL(k_open_ohm<NDIM>, grid, blk, 0, s, B0, (const float*)Yh, (const float*)J,
                         aux, E, o);
      hipLaunchKernelGGL(k_open_faraday<NDIM>, grid, blk, 0, s, (const float*)E, Xb, Xh, Xlb, Xl,
                         h, g);
    }
    fh = Xh;
    fl = Xl;
  }
  if (fl)
    hipLaunchKernelGGL((k_open_curl<NDIM, true>), grid, blk, 0, s, fh, fl, J, g);
  else
    hipLaunchKernelGGL((k_open_curl<NDIM, false>), grid, blk, 0, s, fh, fl, J, g);
  float* B1out = fh == B1 ? nullptr : B1;
  if (mode == 0 && fl)
    hipLaunchKernelGGL((k_open_final<NDIM, true, true>), grid, blk, 0, s, fh, fl, (const float*)J,
                       B0, B1out, Btot, n_half, n_prev, J_half, J_prev, 1.5f, -0.5f, o, eos, E_out,
                       part, c->status);
  else if (mode == 0)
    hipLaunchKernelGGL((k_open_final<NDIM, true, false>), grid, blk, 0, s, fh, fl, (const float*)J,
                       B0, B1out, Btot, n_half, n_prev, J_half, J_prev, 1.5f, -0.5f, o, eos, E_out,
                       part, c->status);
  else
    hipLaunchKernelGGL((k_open_final<NDIM, false, false>), grid, blk, 0, s, fh, fl,
                       (const float*)J, B0, B1out, Btot, n_half, n_prev, J_half, J_prev, 1.5f,
                       -0.5f, o, eos, E_out, part, c->status);
  if (diag_out) {
    const double V = c->p.dx * c->p.dy * c->p.dz;
    const double we_scale = eos.iso ? V * c->p.te : V * c->p.n0 * c->p.te / (c->p.gamma_e - 1.0);
    const int interior = nc - 2 * face_rows(c);
    hipLaunchKernelGGL(k_field_diag_final, dim3(1), dim3(1024), 0, s, (const double*)part,
                       (int)grid.x, diag_out, 0.5 * V, 1.0 / (double)interior, we_scale);
  }
}

}  // namespace
}  // namespace hvpic

using namespace hvpic;

extern "C" {

int hvpic_open_fill(hvpic_ctx* ctx, float* F, int ncomp) {
  if (!ctx || ctx->magic != kMagic) return HVPIC_ESTATE;
  if (!open_ok(ctx) || !F || ncomp < 1 || ncomp > 16) return HVPIC_EINVAL;
  fill(ctx, F, ncomp);
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

int hvpic_open_field_advance(hvpic_ctx* ctx, const float* B0, float* B1, float* Btot,
                             const float* n_half, const float* J_half, const float* n_prev,
                             const float* J_prev, float* E_out, int mode, double* diag_out) {
  if (!ctx || ctx->magic != kMagic) return HVPIC_ESTATE;
  if (!open_ok(ctx) || ctx->p.energy_eq || !B0 || !B1 || !Btot || !n_half || !J_half || !E_out)
    return HVPIC_EINVAL;
  if (mode != 0 && mode != 1) return HVPIC_EINVAL;
  if (mode == 0 && (!n_prev || !J_prev)) return HVPIC_EINVAL;
  if (ctx->p.ndim == 3)
    open_advance<3>(ctx, B0, B1, Btot, n_half, J_half, n_prev, J_prev, E_out, mode, diag_out);
  else
    open_advance<2>(ctx, B0, B1, Btot, n_half, J_half, n_prev, J_prev, E_out, mode, diag_out);
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

int hvpic_open_absorb(hvpic_ctx* ctx, hvpic_particles* p) {
  if (!ctx || ctx->magic != kMagic) return HVPIC_ESTATE;
  if (!open_ok(ctx) || !p || p->n < 0 || p->n > ctx->p.np_capacity || (p->n > 0 && !p->cell))
    return HVPIC_EINVAL;
  if (p->n > 0)
    hipLaunchKernelGGL(k_open_absorb, dim3((unsigned)ceil_div(p->n, 256)), dim3(256), 0,
                       ctx->stream, p->cell, p->n, ctx->p.nx, ctx->ncell);
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

int hvpic_open_inject(hvpic_ctx* ctx, hvpic_particles* p, const hvpic_inflow* in, uint64_t seed,
                      int64_t step) {
  if (!ctx || ctx->magic != kMagic) return HVPIC_ESTATE;
  Inject P;
  int64_t total = 0;
  const int rc = inject_plan(ctx, p, in, seed, step, P, total);
  if (rc != HVPIC_OK) return rc;
  inject_launch(ctx, p, P, total);
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

int hvpic_open_particles(hvpic_ctx* ctx, hvpic_particles* p, const hvpic_inflow* in,
                         uint64_t seed, int64_t step) {
  if (!ctx || ctx->magic != kMagic) return HVPIC_ESTATE;
  Inject P;
  int64_t total = 0;
  const int rc = inject_plan(ctx, p, in, seed, step, P, total);
  if (rc != HVPIC_OK) return rc;
  if (p->n > 0)
    hipLaunchKernelGGL(k_open_absorb, dim3((unsigned)ceil_div(p->n, 256)), dim3(256), 0,
                       ctx->stream, p->cell, p->n, ctx->p.nx, ctx->ncell);
  inject_launch(ctx, p, P, total);
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

int hvpic_sort_open_perm(hvpic_ctx* ctx, const hvpic_particles* in, int64_t n_pushed,
                         const int32_t* cell_start_prev, int32_t* perm, int32_t* cell_start,
                         int32_t* info) {
  if (!ctx || ctx->magic != kMagic) return HVPIC_ESTATE;
  if (!open_ok(ctx) || !in || !cell_start_prev || !cell_start) return HVPIC_EINVAL;
  if (in->n < 0 || in->n > ctx->p.np_capacity || n_pushed < 0 || n_pushed > in->n)
    return HVPIC_EINVAL;
  if (in->n > 0 && (!in->cell || !perm)) return HVPIC_EINVAL;
  hvpic_ctx* c = ctx;
  const int32_t* inj_cnt = nullptr;
  if (in->n > n_pushed) {
    // the ions past n_pushed must be the last injection into this store
    if (c->inj_cell != in->cell || c->inj_n0 != n_pushed || c->inj_n0 + c->inj_k != in->n)
      return HVPIC_EINVAL;
    inj_cnt = c->open_rows;
  }
  const int rows = face_rows(c);
  return launch_sort_open_perm(c, in, n_pushed, cell_start_prev, perm, cell_start, info, inj_cnt,
                               c->open_rows + 2 * rows, c->open_rows + 4 * rows);
}

}  // extern "C"
