// Device helpers shared by the field-solver sources of libhvpic.so: grid
// geometry and periodic neighbours, centred curl, the equation of state, the
// frozen-moment terms of a field advance, the FP64 field diagnostics and
// plain copy/fill kernels.  Included by one translation unit per source; the
// definitions live in an anonymous namespace, one copy per unit.
#pragma once

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

// B held as an unevaluated sum hi + lo (HAS_LO; otherwise hi alone): the
// compensation term carries the low bits that the subcycle's small updates
// would round away.
template <bool HAS_LO>
struct BSum {
  const float* hi;
  const float* lo;
  __device__ __forceinline__ float operator()(int q) const { return HAS_LO ? hi[q] + lo[q] : hi[q]; }
};

template <int NDIM, class BA>
__device__ __forceinline__ void curl_at(BA A, int c, const FGeo& g, float out[3]) {
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
                                                       float n0, float gam, int iso, Aux aux) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c < g.ncell) {
    const int nc = g.ncell;
    int i, j, k;
    fijk(c, g, i, j, k);
    const Nbr nn = neighbours(c, i, j, k, g);
    auto dens = [&](int q) { return nb ? ca * na[q] + cb * nb[q] : na[q]; };
    const float n = dens(c);
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
}

// Equation of state and floor for the frozen-moment terms (FP32), and n0,
// gamma in FP64 for the electron energy diagnostic.
struct Eos {
  float nfloor, te_n0, n0, gam;
  int iso;
  double dn0, dgam, dfloor;
};

Eos make_eos(const hvpic_ctx* c) {
  Eos eos;
  eos.nfloor = (float)c->p.n_floor;
  eos.n0 = (float)c->p.n0;
  eos.te_n0 = (float)(c->p.te * c->p.n0);
  eos.gam = (float)c->p.gamma_e;
  eos.iso = c->p.gamma_e == 1.0;
  eos.dn0 = c->p.n0;
  eos.dgam = c->p.gamma_e;
  eos.dfloor = c->p.n_floor;
  return eos;
}

// Electron internal energy per unit volume of density n (floored), divided by
// te for gamma = 1 (n ln(n/n0)) and by n0 te / (gamma - 1) otherwise
// ((n/n0)^gamma); the factors are applied to the total (Sec. II.A EOS: the
// energy whose time derivative is the pressure work of the electrons).
__device__ __forceinline__ double electron_energy(float n, const Eos& eos) {
  const double nf = fmax((double)n, eos.dfloor);
  return eos.iso ? nf * log(nf / eos.dn0) : pow(nf / eos.dn0, eos.dgam);
}

// FP64 diagnostic values per block partial: sum |B|^2, sum B (three
// components) and the sum of the electron energy density.
constexpr int kDiagNV = 5;
// {W_B, W_dB, W_e} = {1/2 V sum |B|^2, 1/2 V (sum |B|^2 - |sum B|^2 / ncell),
// we_scale sum e(n)} with we_scale = V te (gamma = 1) or V n0 te / (gamma - 1).
// A kernel of its own: a last-block reduction inside k_field_final would need
// an agent-scope release per block, which writes back the L2.
struct DiagArgs {
  const double* part;
  int nblocks;
  double* out;
  double half_vol, inv_ncell, we_scale;
};

__device__ __forceinline__ void field_diag_body(const DiagArgs& D) {
  double r[kDiagNV];
  sum_partials<kDiagNV, kFieldPartStride>(D.part, D.nblocks, r);
  if (threadIdx.x == 0) {
    const double m2 = r[1] * r[1] + r[2] * r[2] + r[3] * r[3];
    D.out[0] = D.half_vol * r[0];
    D.out[1] = D.half_vol * (r[0] - m2 * D.inv_ncell);
    D.out[2] = D.we_scale * r[4];
  }
}

__global__ __launch_bounds__(1024) void k_field_diag_final(const double* part, int nblocks,
                                                             double* out, double half_vol,
                                                             double inv_ncell, double we_scale) {
  field_diag_body(DiagArgs{part, nblocks, out, half_vol, inv_ncell, we_scale});
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

}  // namespace
}  // namespace hvpic
