// Field solver kernels of libhvpic.so (gfx950).
//
// Method (arXiv 2305.05600, Sec. II.A and II.B):
//   Ohm's law (eq:ohm) for massless electrons, with mu0 J = curl B, the
//   density floor n_f = max(n, n_floor) used everywhere the density enters,
//   p_e = n0 te (n_f/n0)^gamma and R_ei = eta J:
//       E = -u_i x B + (J x B)/n_f - grad(p_e)/n_f + eta J,   u_i = J_i/n_f;
//   Faraday dB/dt = -curl E, subcycled: nsub explicit-midpoint substeps with
//   the moments held at their n+1/2 values; J_i (and n) extrapolated to the
//   full step as 3/2 (n+1/2) - 1/2 (n-1/2); gradients are centred differences
//   on the cell-centred grid.
//
// The moments are frozen during the subcycle, so one prep kernel forms
// 1/n_f (in FP64), u_i and -grad(p_e)/n_f once per step.  In 2D one kernel
// runs a whole RK2 substep on LDS tiles with a 4-cell halo (B -> Ea -> B* ->
// Eb -> B); in 3D each RK2 stage is one kernel that evaluates Ohm's law at the
// 2*ndim neighbours of a cell and takes the curl.  E is never stored inside
// the subcycle.  B is carried as an unevaluated sum hi + lo so that the many
// small substep updates keep their low bits.  The grids fit in the MI355X
// L2/MALL during the subcycle, so the substeps are latency-bound.
#include "hvpic_internal.hpp"

namespace hvpic {
namespace {

struct FGeo {
  int nx, ny, nz, ncell, nxny;
  float idx2, idy2, idz2;  // 1 / (2 dx) etc.
  FastDiv fnx, fny;
};

struct Aux {
  float* inv;  // 1/n_f
  float* u;    // [3][ncell] u_i
  float* gp;   // [3][ncell] -grad(p_e)/n_f
};

__device__ __forceinline__ void fijk(int c, const FGeo& g, int& i, int& j, int& k) {
  const uint32_t q = fdiv((uint32_t)c, g.fnx);
  i = c - (int)q * g.nx;
  const uint32_t q2 = fdiv(q, g.fny);
  j = (int)q - (int)q2 * g.ny;
  k = (int)q2;
}

// Linear indices of the +-x, +-y, +-z neighbours (periodic).
struct Nbr {
  int xm, xp, ym, yp, zm, zp;
};

__device__ __forceinline__ Nbr neighbours(int c, int i, int j, int k, const FGeo& g) {
  Nbr n;
  n.xm = i == 0 ? c + g.nx - 1 : c - 1;
  n.xp = i == g.nx - 1 ? c - g.nx + 1 : c + 1;
  n.ym = j == 0 ? c + g.nxny - g.nx : c - g.nx;
  n.yp = j == g.ny - 1 ? c - g.nxny + g.nx : c + g.nx;
  n.zm = k == 0 ? c + g.ncell - g.nxny : c - g.nxny;
  n.zp = k == g.nz - 1 ? c - g.ncell + g.nxny : c + g.nxny;
  return n;
}

// B held as an unevaluated sum hi + lo (lo may be null): the compensation
// term carries the low bits that the subcycle's small updates would round away.
struct BPair {
  const float* hi;
  const float* lo;
  __device__ __forceinline__ float operator()(int q) const { return lo ? hi[q] + lo[q] : hi[q]; }
};

template <int NDIM>
__device__ __forceinline__ void curl_at(BPair A, int c, const FGeo& g, float out[3]) {
  int i, j, k;
  fijk(c, g, i, j, k);
  const Nbr n = neighbours(c, i, j, k, g);
  const int nc = g.ncell;
  const float dyAz = (A(2 * nc + n.yp) - A(2 * nc + n.ym)) * g.idy2;
  const float dxAz = (A(2 * nc + n.xp) - A(2 * nc + n.xm)) * g.idx2;
  const float dxAy = (A(nc + n.xp) - A(nc + n.xm)) * g.idx2;
  const float dyAx = (A(n.yp) - A(n.ym)) * g.idy2;
  float dzAy = 0.f, dzAx = 0.f;
  if (NDIM == 3) {
    dzAy = (A(nc + n.zp) - A(nc + n.zm)) * g.idz2;
    dzAx = (A(n.zp) - A(n.zm)) * g.idz2;
  }
  out[0] = dyAz - dzAy;
  out[1] = dzAx - dxAz;
  out[2] = dxAy - dyAx;
}

// Ohm's law at cell c with the frozen-moment terms precomputed in aux.
template <int NDIM>
__device__ __forceinline__ void ohm_at(BPair B, const Aux& aux, float eta, int c, const FGeo& g,
                                       float E[3]) {
  const int nc = g.ncell;
  float J[3];
  curl_at<NDIM>(B, c, g, J);
  const float b0 = B(c), b1 = B(nc + c), b2 = B(2 * nc + c);
  const float inv = aux.inv[c];
  const float u0 = aux.u[c], u1 = aux.u[nc + c], u2 = aux.u[2 * nc + c];
  // (J - J_i) x B / n_f is -u_i x B + J x B / n_f
  const float w0 = J[0] * inv - u0, w1 = J[1] * inv - u1, w2 = J[2] * inv - u2;
  E[0] = (w1 * b2 - w2 * b1) + aux.gp[c] + eta * J[0];
  E[1] = (w2 * b0 - w0 * b2) + aux.gp[nc + c] + eta * J[1];
  E[2] = (w0 * b1 - w1 * b0) + aux.gp[2 * nc + c] + eta * J[2];
}

__device__ __forceinline__ float pressure(float n, float nfloor, float te_n0, float n0, float gam,
                                          bool iso) {
  const float nf = fmaxf(n, nfloor);
  return iso ? te_n0 / n0 * nf : te_n0 * powf(nf / n0, gam);
}

// Per-step frozen terms from n_eff = ca*na + cb*nb, J_eff = ca*Ja + cb*Jb.
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_field_prep(const float* __restrict__ na,
                                                       const float* __restrict__ nb,
                                                       const float* __restrict__ Ja,
                                                       const float* __restrict__ Jb, float ca,
                                                       float cb, FGeo g, float nfloor, float te_n0,
                                                       float n0, float gam, int iso, Aux aux,
                                                       Status* st, int count_floor) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  const bool live = c < g.ncell;
  bool below = false;
  if (live) {
    const int nc = g.ncell;
    int i, j, k;
    fijk(c, g, i, j, k);
    const Nbr nn = neighbours(c, i, j, k, g);
    auto dens = [&](int q) { return nb ? ca * na[q] + cb * nb[q] : na[q]; };
    const float n = dens(c);
    below = n < nfloor;
    const float nf = fmaxf(n, nfloor);
    const float inv = (float)(1.0 / (double)nf);
    aux.inv[c] = inv;
    for (int a = 0; a < 3; ++a) {
      const float J = Jb ? ca * Ja[a * nc + c] + cb * Jb[a * nc + c] : Ja[a * nc + c];
      aux.u[a * nc + c] = J * inv;
    }
    const float pxp = pressure(dens(nn.xp), nfloor, te_n0, n0, gam, iso);
    const float pxm = pressure(dens(nn.xm), nfloor, te_n0, n0, gam, iso);
    const float pyp = pressure(dens(nn.yp), nfloor, te_n0, n0, gam, iso);
    const float pym = pressure(dens(nn.ym), nfloor, te_n0, n0, gam, iso);
    aux.gp[c] = -(pxp - pxm) * g.idx2 * inv;
    aux.gp[nc + c] = -(pyp - pym) * g.idy2 * inv;
    float gz = 0.f;
    if (NDIM == 3) {
      const float pzp = pressure(dens(nn.zp), nfloor, te_n0, n0, gam, iso);
      const float pzm = pressure(dens(nn.zm), nfloor, te_n0, n0, gam, iso);
      gz = -(pzp - pzm) * g.idz2 * inv;
    }
    aux.gp[2 * nc + c] = gz;
  }
  if (count_floor) {
    const uint64_t m = __ballot(live && below);
    if ((threadIdx.x & 63) == 0 && m) {
      atomicOr(&st->flags, (uint32_t)HVPIC_FLAG_FLOOR_HIT);
      atomicAdd(&st->floor_hits, (unsigned long long)__builtin_popcountll(m));
    }
  }
}

// One RK2 stage: B_dst = B_base - coef * curl(Ohm(B_src)).  With lo non-null
// the update is compensated in place: (hi, lo) <- (hi, lo) - coef * curl E
// (Fast2Sum on the small increment); otherwise Bdst = hi - coef * curl E.
// Ohm's law is evaluated on B_src only, never on the array being written.
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_field_stage(const float* __restrict__ Bsrc,
                                                        const float* Bbase, float* Bdst,
                                                        float* lo, float coef, float eta,
                                                        FGeo g, Aux aux) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= g.ncell) return;
  const int nc = g.ncell;
  int i, j, k;
  fijk(c, g, i, j, k);
  const Nbr n = neighbours(c, i, j, k, g);
  float Exp[3], Exm[3], Eyp[3], Eym[3];
  const BPair Bp{Bsrc, nullptr};
  ohm_at<NDIM>(Bp, aux, eta, n.xp, g, Exp);
  ohm_at<NDIM>(Bp, aux, eta, n.xm, g, Exm);
  ohm_at<NDIM>(Bp, aux, eta, n.yp, g, Eyp);
  ohm_at<NDIM>(Bp, aux, eta, n.ym, g, Eym);
  float cx = (Eyp[2] - Eym[2]) * g.idy2;
  float cy = -(Exp[2] - Exm[2]) * g.idx2;
  float cz = (Exp[1] - Exm[1]) * g.idx2 - (Eyp[0] - Eym[0]) * g.idy2;
  if (NDIM == 3) {
    float Ezp[3], Ezm[3];
    ohm_at<NDIM>(Bp, aux, eta, n.zp, g, Ezp);
    ohm_at<NDIM>(Bp, aux, eta, n.zm, g, Ezm);
    cx -= (Ezp[1] - Ezm[1]) * g.idz2;
    cy += (Ezp[0] - Ezm[0]) * g.idz2;
  }
  const float d[3] = {-coef * cx, -coef * cy, -coef * cz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int q = a * nc + c;
    const float hi = Bbase[q];
    if (lo) {
      const float y = lo[q] + d[a];
      const float t = hi + y;
      lo[q] = y - (t - hi);
      Bdst[q] = t;
    } else {
      Bdst[q] = hi + d[a];
    }
  }
}


// One whole RK2 substep for a 2D tile of TX x TY cells with all intermediate
// fields in LDS: B (halo 4) -> Ea (halo 3) -> B* (halo 2) -> Eb (halo 1) ->
// B_new on the tile.  Reads Bin, writes Bout (distinct buffers: neighbouring
// tiles read the halo of Bin while this one writes).
constexpr int kTX = 32, kTY = 8;
constexpr int kSubBlock = 512;  // threads per substep tile (8 wavefronts hide the load latency)
constexpr int kBW = kTX + 8, kBH = kTY + 8;   // B with halo 4
constexpr int kAW = kTX + 6, kAH = kTY + 6;   // aux and Ea with halo 3
constexpr int kSW = kTX + 4, kSH = kTY + 4;   // B* with halo 2
constexpr int kFW = kTX + 2, kFH = kTY + 2;   // Eb with halo 1

__global__ __launch_bounds__(kSubBlock) void k_field_substep2d(const float* __restrict__ Bin,
                                                            const float* __restrict__ Lin,
                                                            float* __restrict__ Bout,
                                                            float* __restrict__ Lout, float h,
                                                            float eta, FGeo g, Aux aux) {
  __shared__ float sB[3][kBH * kBW];
  __shared__ float sA[7][kAH * kAW];
  __shared__ float sE[3][kAH * kAW];
  __shared__ float sS[3][kSH * kSW];
  const int nc = g.ncell;
  const int tx0 = blockIdx.x * kTX, ty0 = blockIdx.y * kTY;
  auto gidx = [&](int lx, int ly) {
    int x = tx0 + lx, y = ty0 + ly;
    x %= g.nx; if (x < 0) x += g.nx;
    y %= g.ny; if (y < 0) y += g.ny;
    return x + g.nx * y;
  };
  for (int t = threadIdx.x; t < kBH * kBW; t += kSubBlock) {
    const int ly = t / kBW - 4, lx = t % kBW - 4;
    const int c = gidx(lx, ly);
    sB[0][t] = Bin[c];
    sB[1][t] = Bin[nc + c];
    sB[2][t] = Bin[2 * nc + c];
  }
  for (int t = threadIdx.x; t < kAH * kAW; t += kSubBlock) {
    const int ly = t / kAW - 3, lx = t % kAW - 3;
    const int c = gidx(lx, ly);
    sA[0][t] = aux.inv[c];
    sA[1][t] = aux.u[c];
    sA[2][t] = aux.u[nc + c];
    sA[3][t] = aux.u[2 * nc + c];
    sA[4][t] = aux.gp[c];
    sA[5][t] = aux.gp[nc + c];
    sA[6][t] = aux.gp[2 * nc + c];
  }
  __syncthreads();
  // Ohm's law at a cell given B there, curl B there and the aux slot.
  auto ohm = [&](float b0, float b1, float b2, float j0, float j1, float j2, int a, float* e) {
    const float inv = sA[0][a];
    const float w0 = j0 * inv - sA[1][a], w1 = j1 * inv - sA[2][a], w2 = j2 * inv - sA[3][a];
    e[0] = (w1 * b2 - w2 * b1) + sA[4][a] + eta * j0;
    e[1] = (w2 * b0 - w0 * b2) + sA[5][a] + eta * j1;
    e[2] = (w0 * b1 - w1 * b0) + sA[6][a] + eta * j2;
  };
  // Ea on the tile with halo 3 (from B with halo 4)
  for (int t = threadIdx.x; t < kAH * kAW; t += kSubBlock) {
    const int ly = t / kAW, lx = t % kAW;      // B index = (ly+1, lx+1)
    const int b = (ly + 1) * kBW + lx + 1;
    const float j0 = (sB[2][b + kBW] - sB[2][b - kBW]) * g.idy2;
    const float j1 = -(sB[2][b + 1] - sB[2][b - 1]) * g.idx2;
    const float j2 = (sB[1][b + 1] - sB[1][b - 1]) * g.idx2 - (sB[0][b + kBW] - sB[0][b - kBW]) * g.idy2;
    float e[3];
    ohm(sB[0][b], sB[1][b], sB[2][b], j0, j1, j2, t, e);
    sE[0][t] = e[0];
    sE[1][t] = e[1];
    sE[2][t] = e[2];
  }
  __syncthreads();
  // B* = B - (h/2) curl Ea on the tile with halo 2
  const float hh = 0.5f * h;
  for (int t = threadIdx.x; t < kSH * kSW; t += kSubBlock) {
    const int ly = t / kSW, lx = t % kSW;
    const int e = (ly + 1) * kAW + lx + 1;     // Ea index
    const int b = (ly + 2) * kBW + lx + 2;     // B index
    const float c0 = (sE[2][e + kAW] - sE[2][e - kAW]) * g.idy2;
    const float c1 = -(sE[2][e + 1] - sE[2][e - 1]) * g.idx2;
    const float c2 = (sE[1][e + 1] - sE[1][e - 1]) * g.idx2 - (sE[0][e + kAW] - sE[0][e - kAW]) * g.idy2;
    sS[0][t] = sB[0][b] - hh * c0;
    sS[1][t] = sB[1][b] - hh * c1;
    sS[2][t] = sB[2][b] - hh * c2;
  }
  __syncthreads();
  // Eb on the tile with halo 1 (stored in sE with the Eb row width)
  for (int t = threadIdx.x; t < kFH * kFW; t += kSubBlock) {
    const int ly = t / kFW, lx = t % kFW;
    const int s = (ly + 1) * kSW + lx + 1;     // B* index
    const int a = (ly + 2) * kAW + lx + 2;     // aux index
    const float j0 = (sS[2][s + kSW] - sS[2][s - kSW]) * g.idy2;
    const float j1 = -(sS[2][s + 1] - sS[2][s - 1]) * g.idx2;
    const float j2 = (sS[1][s + 1] - sS[1][s - 1]) * g.idx2 - (sS[0][s + kSW] - sS[0][s - kSW]) * g.idy2;
    float e[3];
    ohm(sS[0][s], sS[1][s], sS[2][s], j0, j1, j2, a, e);
    // sE is free again (Ea was consumed before the last barrier)
    sE[0][t] = e[0];
    sE[1][t] = e[1];
    sE[2][t] = e[2];
  }
  __syncthreads();
  // B_new = B - h curl Eb on the tile
  for (int t = threadIdx.x; t < kTY * kTX; t += kSubBlock) {
    const int ly = t / kTX, lx = t % kTX;
    const int x = tx0 + lx, y = ty0 + ly;
    if (x >= g.nx || y >= g.ny) continue;
    const int e = (ly + 1) * kFW + lx + 1;
    const int b = (ly + 4) * kBW + lx + 4;
    const float c0 = (sE[2][e + kFW] - sE[2][e - kFW]) * g.idy2;
    const float c1 = -(sE[2][e + 1] - sE[2][e - 1]) * g.idx2;
    const float c2 = (sE[1][e + 1] - sE[1][e - 1]) * g.idx2 - (sE[0][e + kFW] - sE[0][e - kFW]) * g.idy2;
    const int c = x + g.nx * y;
    // compensated update (hi, lo) - h curl Eb; the increment is tiny next to B
    const float d[3] = {-h * c0, -h * c1, -h * c2};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float hi = sB[a][b];
      const float yv = (Lin ? Lin[a * nc + c] : 0.0f) + d[a];
      const float tv = hi + yv;
      Lout[a * nc + c] = yv - (tv - hi);
      Bout[a * nc + c] = tv;
    }
  }
}

// E = Ohm(B) written out, plus per-block FP64 partials {sum |B|^2, sum B}.
// With Bout non-null the final B = hi + lo is also written there (Bout is
// never one of the arrays read).
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_field_ohm_out(const float* __restrict__ Bh,
                                                          const float* __restrict__ Bl,
                                                          float* __restrict__ Bout, float eta,
                                                          FGeo g, Aux aux, float* __restrict__ E,
                                                          double* part) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  const int nc = g.ncell;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (c < nc) {
    const BPair B{Bh, Bl};
    float e[3];
    ohm_at<NDIM>(B, aux, eta, c, g, e);
    E[c] = e[0];
    E[nc + c] = e[1];
    E[2 * nc + c] = e[2];
    const float f0 = B(c), f1 = B(nc + c), f2 = B(2 * nc + c);
    if (Bout) {
      Bout[c] = f0;
      Bout[nc + c] = f1;
      Bout[2 * nc + c] = f2;
    }
    const double b0 = f0, b1 = f1, b2 = f2;
    v[0] = b0 * b0 + b1 * b1 + b2 * b2;
    v[1] = b0;
    v[2] = b1;
    v[3] = b2;
  }
  if (part) block_partial<4>(v, part);
}

// {W_B, W_dB} = {1/2 V sum |B|^2, 1/2 V (sum |B|^2 - |sum B|^2 / ncell)}.
__global__ __launch_bounds__(1024) void k_field_diag_final(const double* part, int nblocks,
                                                             double* out, double half_vol,
                                                             double inv_ncell) {
  double r[4];
  sum_partials<4>(part, nblocks, r);
  if (threadIdx.x == 0) {
    const double m2 = r[1] * r[1] + r[2] * r[2] + r[3] * r[3];
    out[0] = half_vol * r[0];
    out[1] = half_vol * (r[0] - m2 * inv_ncell);
  }
}

// One binomial (1,2,1)/4 pass along `axis` for ncomp component arrays.
__global__ __launch_bounds__(kBlock) void k_smooth_axis(const float* __restrict__ in,
                                                        float* __restrict__ out, int ncomp, int axis,
                                                        FGeo g) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (int64_t)ncomp * g.ncell) return;
  const int comp = (int)(t / g.ncell);
  const int c = (int)(t - (int64_t)comp * g.ncell);
  int i, j, k;
  fijk(c, g, i, j, k);
  const Nbr n = neighbours(c, i, j, k, g);
  const int m = axis == 0 ? n.xm : (axis == 1 ? n.ym : n.zm);
  const int p = axis == 0 ? n.xp : (axis == 1 ? n.yp : n.zp);
  const float* f = in + (int64_t)comp * g.ncell;
  out[(int64_t)comp * g.ncell + c] = 0.25f * (f[m] + 2.0f * f[c] + f[p]);
}

__global__ void k_copy(const float* __restrict__ in, float* __restrict__ out, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = in[i];
}

__global__ void k_fill(float* __restrict__ out, int64_t n, float v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = v;
}

FGeo fgeo(const hvpic_ctx* c) {
  FGeo g;
  g.nx = c->p.nx;
  g.ny = c->p.ny;
  g.nz = c->p.nz;
  g.ncell = c->ncell;
  g.nxny = c->p.nx * c->p.ny;
  g.idx2 = (float)(0.5 / c->p.dx);
  g.idy2 = (float)(0.5 / c->p.dy);
  g.idz2 = (float)(0.5 / c->p.dz);
  g.fnx = c->fnx;
  g.fny = c->fny;
  return g;
}

template <int NDIM>
int field_impl(hvpic_ctx* c, float* B, const float* n_half, const float* J_half,
               const float* n_prev, const float* J_prev, float* E_out, int mode,
               double* diag_out) {
  const FGeo g = fgeo(c);
  const int nc = c->ncell;
  const dim3 grid((unsigned)ceil_div(nc, kBlock)), blk(kBlock);
  hipStream_t s = c->stream;
  Aux aux;
  aux.inv = c->fscratch;
  aux.u = c->fscratch + nc;
  aux.gp = c->fscratch + 4ll * nc;
  // B pairs (hi, lo) for the compensated subcycle, ping-ponged in scratch
  float* Xh = c->fscratch + 7ll * nc;
  float* Xl = c->fscratch + 10ll * nc;
  float* Yh = c->fscratch + 13ll * nc;
  float* Yl = c->fscratch + 16ll * nc;
  const float nfloor = (float)c->p.n_floor, n0 = (float)c->p.n0;
  const float te_n0 = (float)(c->p.te * c->p.n0), gam = (float)c->p.gamma_e;
  const int iso = c->p.gamma_e == 1.0;
  const float eta = (float)c->p.eta;
  // frozen moments for the subcycle (mode 0) or the E-only evaluation (mode 1)
  hipLaunchKernelGGL((k_field_prep<NDIM>), grid, blk, 0, s, n_half, (const float*)nullptr, J_half,
                     (const float*)nullptr, 1.0f, 0.0f, g, nfloor, te_n0, n0, gam, iso, aux,
                     c->status, 1);
  const float* fh = B;        // final B = fh + fl
  const float* fl = nullptr;
  if (mode == 0 && c->p.nsub > 0) {
    const float h = (float)(c->p.dt / c->p.nsub);
    const int cblocks = (int)std::min<int64_t>(ceil_div(3ll * nc, kBlock), 1024);
    if (NDIM == 2) {
      // fused substeps; the caller's B is only read (first substep)
      const dim3 tiles((unsigned)ceil_div(c->p.nx, kTX), (unsigned)ceil_div(c->p.ny, kTY));
      const float* sh = B;
      const float* sl = nullptr;
      float* dh = Xh;
      float* dl = Xl;
      for (int m = 0; m < c->p.nsub; ++m) {
        hipLaunchKernelGGL(k_field_substep2d, tiles, dim3(kSubBlock), 0, s, sh, sl, dh, dl, h, eta, g,
                           aux);
        sh = dh;
        sl = dl;
        dh = dh == Xh ? Yh : Xh;
        dl = dl == Xl ? Yl : Xl;
      }
      fh = sh;
      fl = sl;
    } else {
      hipLaunchKernelGGL(k_copy, dim3(cblocks), blk, 0, s, (const float*)B, Xh, 3ll * nc);
      hipLaunchKernelGGL(k_fill, dim3(cblocks), blk, 0, s, Xl, 3ll * nc, 0.0f);
      for (int m = 0; m < c->p.nsub; ++m) {
        hipLaunchKernelGGL((k_field_stage<NDIM>), grid, blk, 0, s, (const float*)Xh,
                           (const float*)Xh, Yh, (float*)nullptr, 0.5f * h, eta, g, aux);
        hipLaunchKernelGGL((k_field_stage<NDIM>), grid, blk, 0, s, (const float*)Yh,
                           (const float*)Xh, Xh, Xl, h, eta, g, aux);
      }
      fh = Xh;
      fl = Xl;
    }
  }
  if (mode == 0) {
    // extrapolated moments for E^{n+1}
    hipLaunchKernelGGL((k_field_prep<NDIM>), grid, blk, 0, s, n_half, n_prev, J_half, J_prev, 1.5f,
                       -0.5f, g, nfloor, te_n0, n0, gam, iso, aux, c->status, 0);
  }
  hipLaunchKernelGGL((k_field_ohm_out<NDIM>), grid, blk, 0, s, fh, fl, fh == B ? nullptr : B, eta,
                     g, aux, E_out, diag_out ? c->field_part : nullptr);
  if (diag_out) {
    const double V = c->p.dx * c->p.dy * c->p.dz;
    hipLaunchKernelGGL(k_field_diag_final, dim3(1), dim3(1024), 0, s, (const double*)c->field_part,
                       (int)grid.x, diag_out, 0.5 * V, 1.0 / (double)nc);
  }
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

}  // namespace

int launch_field_advance(hvpic_ctx* c, float* B, const float* n_half, const float* J_half,
                         const float* n_prev, const float* J_prev, float* E_out, int mode,
                         double* diag_out) {
  if (c->p.ndim == 2)
    return field_impl<2>(c, B, n_half, J_half, n_prev, J_prev, E_out, mode, diag_out);
  return field_impl<3>(c, B, n_half, J_half, n_prev, J_prev, E_out, mode, diag_out);
}

int launch_smooth(hvpic_ctx* c, float* F, int ncomp, int npasses) {
  const FGeo g = fgeo(c);
  const int64_t total = (int64_t)ncomp * c->ncell;
  if (total == 0 || npasses == 0) return HVPIC_OK;
  const dim3 grid((unsigned)ceil_div(total, kBlock)), blk(kBlock);
  float* T = c->fscratch;
  for (int pass = 0; pass < npasses; ++pass) {
    hipLaunchKernelGGL(k_smooth_axis, grid, blk, 0, c->stream, (const float*)F, T, ncomp, 0, g);
    hipLaunchKernelGGL(k_smooth_axis, grid, blk, 0, c->stream, (const float*)T, F, ncomp, 1, g);
    if (c->p.ndim == 3) {
      hipLaunchKernelGGL(k_smooth_axis, grid, blk, 0, c->stream, (const float*)F, T, ncomp, 2, g);
      hipLaunchKernelGGL(k_copy, dim3(1024), blk, 0, c->stream, (const float*)T, F, total);
    }
  }
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

}  // namespace hvpic
