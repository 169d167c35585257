// Field advance with hyper-resistivity and the electron energy equation
// (libhvpic.so, gfx950).
//
// Method (arXiv 2305.05600, Sec. II.A): the resistive term of Ohm's law
// (eq:ohm) is R_ei = eta J - eta_h lap J, and with the energy equation the
// electron pressure obeys eq:dpdt with no collisional exchange (H_ei = 0) and
// the heat flux Q_e = -kappa0 grad T_e:
//   dp_e/dt = -gamma div(p_e u_e) + (gamma-1) u_e . grad p_e
//             + (gamma-1) kappa0 lap T_e,
//   u_e = (J_i - curl B)/n_f,  T_e = p_e/n_f,
// advanced in the same explicit-midpoint substeps as B, with the moments held
// at their n+1/2 values; Ohm's law then takes -grad(p_e)/n_f from the evolved
// pressure instead of the equation of state.  lap is the compact second
// difference (+1, -2, +1)/h^2 summed over the axes; div and grad are centred.
//
// Three whole-grid kernels per RK2 stage: J = curl B of the stage input; Ohm's
// law (needs lap J, so J at the neighbours) and, with the energy equation, the
// pressure update (needs u_e, p_e and T_e at the neighbours); B from curl E.
// Each is a stencil over arrays that stay in L2 during the subcycle.  B and
// p_e are carried as unevaluated sums hi + lo as on the plain path; the
// stage inputs are the hi parts.
#include "fields_common.hpp"

namespace hvpic {
namespace {

struct LapG {
  float ix, iy, iz;  // 1/dx^2, 1/dy^2, 1/dz^2
};

struct Phys {
  float eta, eta_h, gam, kappa0;
};

// a at the cell and its +-x, +-y, +-z neighbours (in 2D the z neighbours are
// the cell itself, so z differences vanish).
__device__ __forceinline__ void star(const float* __restrict__ a, int c, const Nbr& n,
                                     float v[7]) {
  v[0] = a[c];
  v[1] = a[n.xp];
  v[2] = a[n.xm];
  v[3] = a[n.yp];
  v[4] = a[n.ym];
  v[5] = a[n.zp];
  v[6] = a[n.zm];
}

template <class BA>
__device__ __forceinline__ void star_sum(BA a, int off, int c, const Nbr& n, float v[7]) {
  v[0] = a(off + c);
  v[1] = a(off + n.xp);
  v[2] = a(off + n.xm);
  v[3] = a(off + n.yp);
  v[4] = a(off + n.ym);
  v[5] = a(off + n.zp);
  v[6] = a(off + n.zm);
}

template <int NDIM>
__device__ __forceinline__ float lap7(const float v[7], const LapG& lg) {
  float r = (v[1] + v[2] - 2.0f * v[0]) * lg.ix + (v[3] + v[4] - 2.0f * v[0]) * lg.iy;
  if (NDIM == 3) r += (v[5] + v[6] - 2.0f * v[0]) * lg.iz;
  return r;
}

// J = curl B (B = hi + lo with HAS_LO).
template <int NDIM, bool HAS_LO>
__global__ __launch_bounds__(kBlock) void k_ext_curl(const float* __restrict__ Bh,
                                                     const float* __restrict__ Bl,
                                                     float* __restrict__ J, FGeo g) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= g.ncell) return;
  const BSum<HAS_LO> B{Bh, Bl};
  float j[3];
  curl_at<NDIM>(B, c, g, j);
  J[c] = j[0];
  J[g.ncell + c] = j[1];
  J[2 * g.ncell + c] = j[2];
}

// Ohm's law of the stage input (Bsrc, J = curl Bsrc, psrc) into E, with the
// frozen terms 1/n_f, u_i (and, without the energy equation, the EOS term
// -grad(p_e)/n_f) from aux.  With PE also the pressure update
// pdst = pbase + coef * rate (compensated into plo when non-null); pbase and
// pdst are read and written at the thread's own cell only, psrc is never
// written here.
template <int NDIM, bool PE>
__global__ __launch_bounds__(kBlock) void k_ext_ohm(const float* __restrict__ Bsrc,
                                                    const float* __restrict__ J,
                                                    const float* __restrict__ psrc,
                                                    const float* pbase, float* pdst, float* plo,
                                                    float coef, Aux aux, float* __restrict__ E,
                                                    FGeo g, LapG lg, Phys ph) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= g.ncell) return;
  const int nc = g.ncell;
  int i, j, k;
  fijk(c, g, i, j, k);
  const Nbr n = neighbours(c, i, j, k, g);
  float Js[3][7];
#pragma unroll
  for (int a = 0; a < 3; ++a) star(J + a * nc, c, n, Js[a]);
  const float inv = aux.inv[c];
  const float b0 = Bsrc[c], b1 = Bsrc[nc + c], b2 = Bsrc[2 * nc + c];
  const float u0 = aux.u[c], u1 = aux.u[nc + c], u2 = aux.u[2 * nc + c];
  float ps[7], gp[3];
  if (PE) {
    star(psrc, c, n, ps);
    gp[0] = -(ps[1] - ps[2]) * g.idx2 * inv;
    gp[1] = -(ps[3] - ps[4]) * g.idy2 * inv;
    gp[2] = NDIM == 3 ? -(ps[5] - ps[6]) * g.idz2 * inv : 0.0f;
  } else {
    gp[0] = aux.gp[c];
    gp[1] = aux.gp[nc + c];
    gp[2] = aux.gp[2 * nc + c];
  }
  const float j0 = Js[0][0], j1 = Js[1][0], j2 = Js[2][0];
  const float w0 = j0 * inv - u0, w1 = j1 * inv - u1, w2 = j2 * inv - u2;
  E[c] = (w1 * b2 - w2 * b1) + gp[0] + ph.eta * j0 - ph.eta_h * lap7<NDIM>(Js[0], lg);
  E[nc + c] = (w2 * b0 - w0 * b2) + gp[1] + ph.eta * j1 - ph.eta_h * lap7<NDIM>(Js[1], lg);
  E[2 * nc + c] = (w0 * b1 - w1 * b0) + gp[2] + ph.eta * j2 - ph.eta_h * lap7<NDIM>(Js[2], lg);
  if (PE) {
    float iv[7];
    star(aux.inv, c, n, iv);
    // u_e = u_i - J/n_f where the centred divergence and gradient need it
    const float uexp = aux.u[n.xp] - Js[0][1] * iv[1], uexm = aux.u[n.xm] - Js[0][2] * iv[2];
    const float ueyp = aux.u[nc + n.yp] - Js[1][3] * iv[3],
                ueym = aux.u[nc + n.ym] - Js[1][4] * iv[4];
    const float uex = u0 - j0 * inv, uey = u1 - j1 * inv, uez = u2 - j2 * inv;
    float div = (ps[1] * uexp - ps[2] * uexm) * g.idx2 + (ps[3] * ueyp - ps[4] * ueym) * g.idy2;
    float adv = uex * (ps[1] - ps[2]) * g.idx2 + uey * (ps[3] - ps[4]) * g.idy2;
    if (NDIM == 3) {
      const float uezp = aux.u[2 * nc + n.zp] - Js[2][5] * iv[5],
                  uezm = aux.u[2 * nc + n.zm] - Js[2][6] * iv[6];
      div += (ps[5] * uezp - ps[6] * uezm) * g.idz2;
      adv += uez * (ps[5] - ps[6]) * g.idz2;
    }
    float T[7];
#pragma unroll
    for (int s = 0; s < 7; ++s) T[s] = ps[s] * iv[s];
    const float gm1 = ph.gam - 1.0f;
    const float rate = -ph.gam * div + gm1 * adv + gm1 * ph.kappa0 * lap7<NDIM>(T, lg);
    const float d = coef * rate;
    const float hi = pbase[c];
    if (plo) {
      const float y = plo[c] + d;
      const float t = hi + y;
      plo[c] = y - (t - hi);
      pdst[c] = t;
    } else {
      pdst[c] = hi + d;
    }
  }
}

// B_dst = B_base - coef * curl E (compensated into lo when non-null); B_base
// and B_dst are read and written at the thread's own cell only.
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_ext_faraday(const float* __restrict__ E,
                                                        const float* Bbase, float* Bdst, float* lo,
                                                        float coef, FGeo g) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= g.ncell) return;
  const BSum<false> Ea{E, nullptr};
  float ce[3];
  curl_at<NDIM>(Ea, c, g, ce);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int q = a * g.ncell + c;
    const float d = -coef * ce[a];
    const float hi = Bbase[q];
    if (lo) {
      const float y = lo[q] + d;
      const float t = hi + y;
      lo[q] = y - (t - hi);
      Bdst[q] = t;
    } else {
      Bdst[q] = hi + d;
    }
  }
}

// E from B = Bh (+ Bl), J = curl B, the moments n_eff = ca*na + cb*nb,
// J_eff = ca*Ja + cb*Jb (EXTRAP; otherwise na, Ja) and the pressure p = ph (+ pl)
// (PE; otherwise the EOS of n_eff).  With Bout / pout non-null the final B and
// p go there (never among the arrays read).  Cells of na below the floor are
// counted when asked.  With part non-null, per-block FP64 partials {sum |B|^2,
// sum B, sum of the electron energy density} go to part: p (PE) or
// electron_energy(n_eff).
template <int NDIM, bool PE, bool EXTRAP, bool HAS_LO>
__global__ __launch_bounds__(kBlock) void k_ext_final(
    const float* __restrict__ Bh, const float* __restrict__ Bl, const float* __restrict__ Ph,
    const float* __restrict__ Pl, const float* __restrict__ J, float* __restrict__ Bout,
    float* __restrict__ pout, const float* __restrict__ na, const float* __restrict__ nb,
    const float* __restrict__ Ja, const float* __restrict__ Jb, float ca, float cb, Phys ph,
    FGeo g, LapG lg, Eos eos, float* __restrict__ E, double* part, Status* st,
    int count_floor) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  const int nc = g.ncell;
  const bool live = c < nc;
  bool below = false;
  double v[kDiagNV] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (live) {
    int i, j, k;
    fijk(c, g, i, j, k);
    const Nbr n = neighbours(c, i, j, k, g);
    auto dens = [&](int q) { return EXTRAP ? ca * na[q] + cb * nb[q] : na[q]; };
    const float n_c = dens(c);
    float Js[3][7];
#pragma unroll
    for (int a = 0; a < 3; ++a) star(J + a * nc, c, n, Js[a]);
    float Jv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      Jv[a] = EXTRAP ? ca * Ja[a * nc + c] + cb * Jb[a * nc + c] : Ja[a * nc + c];
    const BSum<HAS_LO> B{Bh, Bl};
    const float b0 = B(c), b1 = B(nc + c), b2 = B(2 * nc + c);
    below = na[c] < eos.nfloor;
    const float inv = (float)(1.0 / (double)fmaxf(n_c, eos.nfloor));
    float ps[7];
    if (PE) {
      const BSum<HAS_LO> P{Ph, Pl};
      star_sum(P, 0, c, n, ps);
    } else {
      auto pres = [&](int q) {
        return pressure(dens(q), eos.nfloor, eos.te_n0, eos.n0, eos.gam, eos.iso);
      };
      ps[0] = 0.0f;
      ps[1] = pres(n.xp);
      ps[2] = pres(n.xm);
      ps[3] = pres(n.yp);
      ps[4] = pres(n.ym);
      ps[5] = NDIM == 3 ? pres(n.zp) : 0.0f;
      ps[6] = NDIM == 3 ? pres(n.zm) : 0.0f;
    }
    const float gp0 = -(ps[1] - ps[2]) * g.idx2 * inv;
    const float gp1 = -(ps[3] - ps[4]) * g.idy2 * inv;
    const float gp2 = NDIM == 3 ? -(ps[5] - ps[6]) * g.idz2 * inv : 0.0f;
    const float j0 = Js[0][0], j1 = Js[1][0], j2 = Js[2][0];
    const float w0 = j0 * inv - Jv[0] * inv, w1 = j1 * inv - Jv[1] * inv,
                w2 = j2 * inv - Jv[2] * inv;
    E[c] = (w1 * b2 - w2 * b1) + gp0 + ph.eta * j0 - ph.eta_h * lap7<NDIM>(Js[0], lg);
    E[nc + c] = (w2 * b0 - w0 * b2) + gp1 + ph.eta * j1 - ph.eta_h * lap7<NDIM>(Js[1], lg);
    E[2 * nc + c] = (w0 * b1 - w1 * b0) + gp2 + ph.eta * j2 - ph.eta_h * lap7<NDIM>(Js[2], lg);
    if (Bout) {
      Bout[c] = b0;
      Bout[nc + c] = b1;
      Bout[2 * nc + c] = b2;
    }
    if (PE && pout) pout[c] = ps[0];
    const double d0 = b0, d1 = b1, d2 = b2;
    v[0] = d0 * d0 + d1 * d1 + d2 * d2;
    v[1] = d0;
    v[2] = d1;
    v[3] = d2;
    if (part) v[4] = PE ? (double)ps[0] : electron_energy(n_c, eos);
  }
  if (count_floor) {
    const uint64_t m = __ballot(live && below);
    if ((threadIdx.x & 63) == 0 && m) {
      atomicOr(&st->flags, (uint32_t)HVPIC_FLAG_FLOOR_HIT);
      atomicAdd(&st->floor_hits, (unsigned long long)__builtin_popcountll(m));
    }
  }
  if (part) block_partial<kDiagNV, kFieldPartStride>(v, part);
}

// p_e = n0 te (n_f/n0)^gamma of the floored density.
__global__ __launch_bounds__(kBlock) void k_eos_pressure(const float* __restrict__ n,
                                                         float* __restrict__ pe, int ncell,
                                                         Eos eos) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c < ncell) pe[c] = pressure(n[c], eos.nfloor, eos.te_n0, eos.n0, eos.gam, eos.iso);
}

template <int NDIM, bool PE>
int ext_impl(hvpic_ctx* c, float* B, float* pe, const float* n_half, const float* J_half,
             const float* n_prev, const float* J_prev, float* E_out, int mode, double* diag_out) {
  const FGeo g = fgeo(c);
  const int nc = c->ncell;
  const dim3 grid((unsigned)ceil_div(nc, kBlock)), blk(kBlock);
  hipStream_t s = c->stream;
  Aux aux;
  aux.inv = c->fscratch;
  aux.u = c->fscratch + nc;
  aux.gp = c->fscratch + 4ll * nc;
  float* Xh = c->fscratch + 7ll * nc;  // B (hi, lo) and the stage value
  float* Xl = c->fscratch + 10ll * nc;
  float* Yh = c->fscratch + 13ll * nc;
  float* J = c->fscratch + 16ll * nc;  // curl B of the stage
  float* E = c->fscratch + 19ll * nc;  // E of the stage
  float* Xp = c->fscratch + 22ll * nc; // p_e (hi, lo) and the stage value
  float* Xpl = c->fscratch + 23ll * nc;
  float* Yp = c->fscratch + 24ll * nc;
  const Eos eos = make_eos(c);
  const LapG lg{(float)(1.0 / (c->p.dx * c->p.dx)), (float)(1.0 / (c->p.dy * c->p.dy)),
                (float)(1.0 / (c->p.dz * c->p.dz))};
  const Phys ph{(float)c->p.eta, (float)c->p.eta_h, (float)c->p.gamma_e, (float)c->p.kappa0};
  const float* fh = B;
  const float* fl = nullptr;
  const float* fp = pe;
  const float* fpl = nullptr;
  if (mode == 0 && c->p.nsub > 0) {
    const float h = (float)(c->p.dt / c->p.nsub);
    hipLaunchKernelGGL((k_field_prep<NDIM>), grid, blk, 0, s, n_half, (const float*)nullptr,
                       J_half, (const float*)nullptr, 1.0f, 0.0f, g, eos.nfloor, eos.te_n0,
                       eos.n0, eos.gam, eos.iso, aux);
    const int cblocks = (int)std::min<int64_t>(ceil_div(3ll * nc, kBlock), 1024);
    hipLaunchKernelGGL(k_copy, dim3(cblocks), blk, 0, s, (const float*)B, Xh, 3ll * nc);
    hipLaunchKernelGGL(k_fill, dim3(cblocks), blk, 0, s, Xl, 3ll * nc, 0.0f);
    if (PE) {
      hipLaunchKernelGGL(k_copy, dim3(cblocks), blk, 0, s, (const float*)pe, Xp, (int64_t)nc);
      hipLaunchKernelGGL(k_fill, dim3(cblocks), blk, 0, s, Xpl, (int64_t)nc, 0.0f);
    }
    for (int m = 0; m < c->p.nsub; ++m) {
      // (B*, p*) = (B, p) + (h/2) rates of (B, p)
      hipLaunchKernelGGL((k_ext_curl<NDIM, false>), grid, blk, 0, s, (const float*)Xh,
                         (const float*)nullptr, J, g);
      hipLaunchKernelGGL((k_ext_ohm<NDIM, PE>), grid, blk, 0, s, (const float*)Xh,
                         (const float*)J, (const float*)Xp, (const float*)Xp, Yp, (float*)nullptr,
                         0.5f * h, aux, E, g, lg, ph);
      hipLaunchKernelGGL((k_ext_faraday<NDIM>), grid, blk, 0, s, (const float*)E,
                         (const float*)Xh, Yh, (float*)nullptr, 0.5f * h, g);
      // (B, p) += h rates of (B*, p*)
      hipLaunchKernelGGL((k_ext_curl<NDIM, false>), grid, blk, 0, s, (const float*)Yh,
                         (const float*)nullptr, J, g);
      hipLaunchKernelGGL((k_ext_ohm<NDIM, PE>), grid, blk, 0, s, (const float*)Yh,
                         (const float*)J, (const float*)Yp, (const float*)Xp, Xp, Xpl, h, aux, E,
                         g, lg, ph);
      hipLaunchKernelGGL((k_ext_faraday<NDIM>), grid, blk, 0, s, (const float*)E,
                         (const float*)Xh, Xh, Xl, h, g);
    }
    fh = Xh;
    fl = Xl;
    fp = Xp;
    fpl = Xpl;
  }
  if (fl)
    hipLaunchKernelGGL((k_ext_curl<NDIM, true>), grid, blk, 0, s, fh, fl, J, g);
  else
    hipLaunchKernelGGL((k_ext_curl<NDIM, false>), grid, blk, 0, s, fh, fl, J, g);
  float* Bout = fh == B ? nullptr : B;
  float* pout = fp == pe ? nullptr : pe;
  double* part = diag_out ? c->field_part : nullptr;
  auto final_kernel = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, blk, 0, s, fh, fl, fp, fpl, (const float*)J, Bout, pout,
                       n_half, n_prev, J_half, J_prev, 1.5f, -0.5f, ph, g, lg, eos, E_out, part,
                       c->status, 1);
  };
  if (mode == 0 && fl)
    final_kernel(k_ext_final<NDIM, PE, true, true>);
  else if (mode == 0)
    final_kernel(k_ext_final<NDIM, PE, true, false>);
  else
    final_kernel(k_ext_final<NDIM, PE, false, false>);
  if (diag_out) {
    const double V = c->p.dx * c->p.dy * c->p.dz;
    double we_scale;
    if (PE)
      we_scale = V / (c->p.gamma_e - 1.0);
    else
      we_scale = eos.iso ? V * c->p.te : V * c->p.n0 * c->p.te / (c->p.gamma_e - 1.0);
    hipLaunchKernelGGL(k_field_diag_final, dim3(1), dim3(1024), 0, s, (const double*)part,
                       (int)grid.x, diag_out, 0.5 * V, 1.0 / (double)nc, we_scale);
  }
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

}  // namespace

int launch_field_advance_ext(hvpic_ctx* c, float* B, float* pe, const float* n_half,
                             const float* J_half, const float* n_prev, const float* J_prev,
                             float* E_out, int mode, double* diag_out) {
  if (c->p.ndim == 2)
    return pe ? ext_impl<2, true>(c, B, pe, n_half, J_half, n_prev, J_prev, E_out, mode, diag_out)
              : ext_impl<2, false>(c, B, pe, n_half, J_half, n_prev, J_prev, E_out, mode,
                                   diag_out);
  return pe ? ext_impl<3, true>(c, B, pe, n_half, J_half, n_prev, J_prev, E_out, mode, diag_out)
            : ext_impl<3, false>(c, B, pe, n_half, J_half, n_prev, J_prev, E_out, mode, diag_out);
}

int launch_eos_pressure(hvpic_ctx* c, const float* n, float* pe) {
  if (c->ncell == 0) return HVPIC_OK;
  hipLaunchKernelGGL(k_eos_pressure, dim3((unsigned)ceil_div(c->ncell, kBlock)), dim3(kBlock), 0,
                     c->stream, n, pe, c->ncell, make_eos(c));
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

}  // namespace hvpic
