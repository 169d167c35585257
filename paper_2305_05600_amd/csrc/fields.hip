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
// The moments are frozen during the subcycle, so the terms that depend on them
// alone (1/n_f in FP64, u_i and -grad(p_e)/n_f) are formed once per cell.  In
// 2D one kernel runs two whole RK2 substeps on an LDS tile with an 8-cell halo
// (B -> Ea -> B* -> Eb -> B, twice), forming those terms on its own halo; in
// 3D a prep kernel stores them and each RK2 stage is one kernel that evaluates
// Ohm's law at the 2*ndim neighbours of a cell and takes the curl.  E is never
// stored inside the subcycle.  B is carried as an unevaluated sum hi + lo so
// that the many small substep updates keep their low bits.  One last kernel
// writes E from the extrapolated moments, the final B and the diagnostics.
// The grids fit in the MI355X L2/MALL during the subcycle, so the substeps are
// latency-bound: fewer, larger launches are what shortens them.
#include <string.h>

#include "fields_common.hpp"

namespace hvpic {
namespace {

// Ohm's law at cell c with the frozen-moment terms precomputed in aux.
template <int NDIM, class BA>
__device__ __forceinline__ void ohm_at(BA B, const Aux& aux, float eta, int c, const FGeo& g,
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
  const BSum<false> Bp{Bsrc, nullptr};
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

// The same stage in two passes: E = Ohm(B_src) once per cell, then the
// Faraday update from curl E.  Each cell's E is formed once instead of once
// per neighbour that needs it (2 NDIM times in k_field_stage), at the cost
// of writing E and reading it back.
template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_field_ohm_cells(const float* __restrict__ Bsrc,
                                                            float eta, FGeo g, Aux aux,
                                                            float* __restrict__ E) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= g.ncell) return;
  const int nc = g.ncell;
  float e[3];
  ohm_at<NDIM>(BSum<false>{Bsrc, nullptr}, aux, eta, c, g, e);
  E[c] = e[0];
  E[nc + c] = e[1];
  E[2 * nc + c] = e[2];
}

template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_field_curl_update(const float* __restrict__ E,
                                                              const float* Bbase, float* Bdst,
                                                              float* lo, float coef, FGeo g) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= g.ncell) return;
  const int nc = g.ncell;
  float ce[3];
  curl_at<NDIM>(BSum<false>{E, nullptr}, c, g, ce);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int q = a * nc + c;
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

// K whole RK2 substeps for a 2D tile of kTX x kTY cells, all intermediate
// fields in LDS.  Each substep needs B on a 4-cell halo (B -> Ea on halo 3 ->
// B* on halo 2 -> Eb on halo 1 -> B_new), so the tile reads B on a 4K halo and
// recomputes the overlap with its neighbours instead of a launch per substep.
// The frozen terms (1/n_f, u_i, -grad(p_e)/n_f) are formed here from the
// moments, on a halo of 4K - 1.  B enters as the sum hi + lo: Ohm's law sees
// hi only; each substep's increment goes to lo first (compensated sum), over
// the cells that the next substep reads.  Reads Bin/Lin, writes Bout/Lout
// (distinct buffers: neighbouring tiles read the halo of Bin while this one
// writes).
constexpr int kTX = 32, kTY = 8;
// 512 threads per tile.  The tile's LDS is sized at launch: with a static
// size the compiler would pad the VGPR allocation up to the occupancy that
// the LDS allows (169 per wave instead of the 64 used), and such tiles would
// rarely find room on CUs busy with a concurrently running particle kernel.
constexpr int kSubBlock = 512;

// One LDS plane: the tile with a halo of HALO cells, row-major.
template <int TX, int TY, int HALO>
struct Plane {
  static constexpr int W = TX + 2 * HALO, H = TY + 2 * HALO, N = W * H;
  __device__ static int at(int lx, int ly) { return (ly + HALO) * W + lx + HALO; }
};

template <int TX, int TY, int K, bool FINAL>
struct SubLds {
  // the final launch keeps its last substep's B on a 1-cell halo (for curl B)
  static constexpr int HB = 4 * K + (FINAL ? 1 : 0);
  using PB = Plane<TX, TY, HB>;      // B hi (and the pressure while the frozen terms are formed)
  using PA = Plane<TX, TY, HB - 1>;  // six frozen-term planes, then E (Ea, later Eb)
  using PS = Plane<TX, TY, HB - 2>;  // B*
  using PL = Plane<TX, TY, HB - 4>;  // lo over the output region of the first substep
  static constexpr int B0 = 0, A0 = 3 * PB::N, E0 = A0 + 6 * PA::N, S0 = E0 + 3 * PA::N,
                       L0 = S0 + 3 * PS::N, TOTAL = L0 + 3 * PL::N;
  static_assert(3 * PA::N + 3 * PS::N >= PB::N, "pressure plane overlays E and B*");
};

// FP64 sums of the five diagnostic values over a tile block (fixed order),
// thread 0 writes them to out[0..4].
__device__ void tile_partial(double* v, double* out) {
  __shared__ double s_red[kSubBlock / 64][kDiagNV];
#pragma unroll
  for (int k = 0; k < kDiagNV; ++k)
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o);
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < kDiagNV; ++k) s_red[wid][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < kDiagNV; ++k) {
      double t = 0.0;
      for (int w = 0; w < kSubBlock / 64; ++w) t += s_red[w][k];
      out[k] = t;
    }
}

// Per-step outputs of the final launch (FINAL): E from the moments
// extrapolated to the full step, n_eff = 1.5 nm - 0.5 np, J_eff = 1.5 Jm -
// 0.5 Jp, the final B = hi + lo into Bfin, the count of cells of nm below the
// floor, and per-tile FP64 partials {sum |B|^2, sum B, sum e(n_eff)} into
// part (e as in electron_energy).
struct SubFinal {
  const float* np;
  const float* Jp;
  float* E;
  float* Bfin;
  double* part;
  Status* st;
  const uint32_t* skip;  // non-null: the launch does nothing when *skip is set
};

template <int TX, int TY, int K, bool HAS_LIN, bool FINAL>
__device__ __forceinline__ void field_sub2d_body(
    const float* __restrict__ Bin, const float* __restrict__ Lin, float* __restrict__ Bout,
    float* __restrict__ Lout, const float* __restrict__ nm, const float* __restrict__ Jm, float h,
    float eta, const FGeo& g, const Eos& eos, const SubFinal& F, int bx, int by, int slot) {
  if (F.skip && *F.skip) return;  // uniform: the surrogate's proposal was accepted
  using L = SubLds<TX, TY, K, FINAL>;
  using PB = typename L::PB;
  using PA = typename L::PA;
  using PS = typename L::PS;
  using PL = typename L::PL;
  constexpr int HB = L::HB;
  extern __shared__ float sm[];  // L::TOTAL floats
  float* sB = sm + L::B0;
  float* sA = sm + L::A0;
  float* sE = sm + L::E0;
  float* sS = sm + L::S0;
  float* sL = sm + L::L0;
  float* sP = sE;  // pressure, only until the frozen terms are formed
  const int nc = g.ncell;
  const int tx0 = bx * TX, ty0 = by * TY;
  // periodic cell of tile-relative (lx, ly), for any halo width and grid size
  auto gidx = [&](int lx, int ly) {
    int x = tx0 + lx, y = ty0 + ly;
    x %= g.nx; if (x < 0) x += g.nx;
    y %= g.ny; if (y < 0) y += g.ny;
    return x + g.nx * y;
  };
  // The set-up loads of a thread are unrolled over clamped slots, with no
  // branch between them, and all issued before the first LDS store, so that
  // they are in flight together: B and n on halo HB, n and J on halo HB-1,
  // lo on halo HB-4 (the output region of the first substep).
  constexpr int IB = (PB::N + kSubBlock - 1) / kSubBlock;
  constexpr int IA = (PA::N + kSubBlock - 1) / kSubBlock;
  constexpr int IL = (PL::N + kSubBlock - 1) / kSubBlock;
  float vb[IB][4], va[IA][4], vl[IL][3];
  // final launch: each of the first TX*TY threads owns one tile cell and
  // loads its extrapolation inputs here, with the others (n at the cell and
  // its four neighbours, J at the cell)
  constexpr int NF = FINAL ? 16 : 1;
  float vf[NF];
  const int fx = (int)threadIdx.x % TX, fy = (int)threadIdx.x / TX;
  const bool fown = FINAL && (int)threadIdx.x < TX * TY;
  if (FINAL) {
    const int cf[5] = {gidx(fx, fy), gidx(fx + 1, fy), gidx(fx - 1, fy), gidx(fx, fy + 1),
                       gidx(fx, fy - 1)};
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      vf[q] = nm[cf[q]];
      vf[5 + q] = F.np[cf[q]];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      vf[10 + a] = Jm[a * nc + cf[0]];
      vf[13 + a] = F.Jp[a * nc + cf[0]];
    }
  }
#pragma unroll
  for (int u = 0; u < IB; ++u) {
    const int t = min((int)threadIdx.x + u * kSubBlock, PB::N - 1);
    const int c = gidx(t % PB::W - HB, t / PB::W - HB);
    vb[u][0] = Bin[c];
    vb[u][1] = Bin[nc + c];
    vb[u][2] = Bin[2 * nc + c];
    vb[u][3] = nm[c];
  }
#pragma unroll
  for (int u = 0; u < IA; ++u) {
    const int t = min((int)threadIdx.x + u * kSubBlock, PA::N - 1);
    const int c = gidx(t % PA::W - (HB - 1), t / PA::W - (HB - 1));
    va[u][0] = nm[c];
    va[u][1] = Jm[c];
    va[u][2] = Jm[nc + c];
    va[u][3] = Jm[2 * nc + c];
  }
#pragma unroll
  for (int u = 0; u < IL; ++u) {
    const int t = min((int)threadIdx.x + u * kSubBlock, PL::N - 1);
    const int c = gidx(t % PL::W - (HB - 4), t / PL::W - (HB - 4));
    vl[u][0] = HAS_LIN ? Lin[c] : 0.0f;
    vl[u][1] = HAS_LIN ? Lin[nc + c] : 0.0f;
    vl[u][2] = HAS_LIN ? Lin[2 * nc + c] : 0.0f;
  }
  // B and p_e on halo HB
#pragma unroll
  for (int u = 0; u < IB; ++u) {
    const int t = (int)threadIdx.x + u * kSubBlock;
    if (t < PB::N) {
      sB[t] = vb[u][0];
      sB[PB::N + t] = vb[u][1];
      sB[2 * PB::N + t] = vb[u][2];
      sP[t] = pressure(vb[u][3], eos.nfloor, eos.te_n0, eos.n0, eos.gam, eos.iso);
    }
  }
  // 1/n_f and u_i on halo HB-1
#pragma unroll
  for (int u = 0; u < IA; ++u) {
    const int t = (int)threadIdx.x + u * kSubBlock;
    if (t < PA::N) {
      const float inv = (float)(1.0 / (double)fmaxf(va[u][0], eos.nfloor));
      sA[t] = inv;
      sA[PA::N + t] = va[u][1] * inv;
      sA[2 * PA::N + t] = va[u][2] * inv;
      sA[3 * PA::N + t] = va[u][3] * inv;
    }
  }
#pragma unroll
  for (int u = 0; u < IL; ++u) {
    const int t = (int)threadIdx.x + u * kSubBlock;
    if (t < PL::N) {
      sL[t] = vl[u][0];
      sL[PL::N + t] = vl[u][1];
      sL[2 * PL::N + t] = vl[u][2];
    }
  }
  __syncthreads();
  // -grad(p_e)/n_f on halo HB-1 (its z component is zero in 2D)
  for (int t = threadIdx.x; t < PA::N; t += kSubBlock) {
    const int ly = t / PA::W - (HB - 1), lx = t % PA::W - (HB - 1);
    const int p = PB::at(lx, ly);
    const float inv = sA[t];
    sA[4 * PA::N + t] = -(sP[p + 1] - sP[p - 1]) * g.idx2 * inv;
    sA[5 * PA::N + t] = -(sP[p + PB::W] - sP[p - PB::W]) * g.idy2 * inv;
  }
  __syncthreads();
  // Ohm's law at a cell given B there, curl B there and the frozen-term slot.
  auto ohm = [&](float b0, float b1, float b2, float j0, float j1, float j2, int a, float* e) {
    const float inv = sA[a];
    const float w0 = j0 * inv - sA[PA::N + a], w1 = j1 * inv - sA[2 * PA::N + a],
                w2 = j2 * inv - sA[3 * PA::N + a];
    e[0] = (w1 * b2 - w2 * b1) + sA[4 * PA::N + a] + eta * j0;
    e[1] = (w2 * b0 - w0 * b2) + sA[5 * PA::N + a] + eta * j1;
    e[2] = (w0 * b1 - w1 * b0) + 0.0f + eta * j2;
  };
  const float hh = 0.5f * h;
#pragma unroll
  for (int s = 0; s < K; ++s) {
    const int hin = 4 * (K - s) + (FINAL ? 1 : 0);  // halo of this substep's input B
    // Ea on halo hin-1
    {
      const int r = hin - 1, W = TX + 2 * r, N = W * (TY + 2 * r);
      for (int t = threadIdx.x; t < N; t += kSubBlock) {
        const int ly = t / W - r, lx = t % W - r;
        const int b = PB::at(lx, ly), a = PA::at(lx, ly);
        const float j0 = (sB[2 * PB::N + b + PB::W] - sB[2 * PB::N + b - PB::W]) * g.idy2;
        const float j1 = -(sB[2 * PB::N + b + 1] - sB[2 * PB::N + b - 1]) * g.idx2;
        const float j2 = (sB[PB::N + b + 1] - sB[PB::N + b - 1]) * g.idx2 -
                         (sB[b + PB::W] - sB[b - PB::W]) * g.idy2;
        float e[3];
        ohm(sB[b], sB[PB::N + b], sB[2 * PB::N + b], j0, j1, j2, a, e);
        sE[a] = e[0];
        sE[PA::N + a] = e[1];
        sE[2 * PA::N + a] = e[2];
      }
    }
    __syncthreads();
    // B* = B - (h/2) curl Ea on halo hin-2
    {
      const int r = hin - 2, W = TX + 2 * r, N = W * (TY + 2 * r);
      for (int t = threadIdx.x; t < N; t += kSubBlock) {
        const int ly = t / W - r, lx = t % W - r;
        const int e = PA::at(lx, ly), b = PB::at(lx, ly), q = PS::at(lx, ly);
        const float c0 = (sE[2 * PA::N + e + PA::W] - sE[2 * PA::N + e - PA::W]) * g.idy2;
        const float c1 = -(sE[2 * PA::N + e + 1] - sE[2 * PA::N + e - 1]) * g.idx2;
        const float c2 = (sE[PA::N + e + 1] - sE[PA::N + e - 1]) * g.idx2 -
                         (sE[e + PA::W] - sE[e - PA::W]) * g.idy2;
        sS[q] = sB[b] - hh * c0;
        sS[PS::N + q] = sB[PB::N + b] - hh * c1;
        sS[2 * PS::N + q] = sB[2 * PB::N + b] - hh * c2;
      }
    }
    __syncthreads();
    // Eb on halo hin-3 (into the E planes: Ea was consumed before the barrier)
    {
      const int r = hin - 3, W = TX + 2 * r, N = W * (TY + 2 * r);
      for (int t = threadIdx.x; t < N; t += kSubBlock) {
        const int ly = t / W - r, lx = t % W - r;
        const int q = PS::at(lx, ly), a = PA::at(lx, ly);
        const float j0 = (sS[2 * PS::N + q + PS::W] - sS[2 * PS::N + q - PS::W]) * g.idy2;
        const float j1 = -(sS[2 * PS::N + q + 1] - sS[2 * PS::N + q - 1]) * g.idx2;
        const float j2 = (sS[PS::N + q + 1] - sS[PS::N + q - 1]) * g.idx2 -
                         (sS[q + PS::W] - sS[q - PS::W]) * g.idy2;
        float e[3];
        ohm(sS[q], sS[PS::N + q], sS[2 * PS::N + q], j0, j1, j2, a, e);
        sE[a] = e[0];
        sE[PA::N + a] = e[1];
        sE[2 * PA::N + a] = e[2];
      }
    }
    __syncthreads();
    // B_new = B - h curl Eb on halo hin-4, as the compensated sum
    // (hi, lo) - h curl Eb: the increment is tiny next to B
    {
      const int r = hin - 4, W = TX + 2 * r, N = W * (TY + 2 * r);
      for (int t = threadIdx.x; t < N; t += kSubBlock) {
        const int ly = t / W - r, lx = t % W - r;
        const int e = PA::at(lx, ly), b = PB::at(lx, ly), l = PL::at(lx, ly);
        const float c0 = (sE[2 * PA::N + e + PA::W] - sE[2 * PA::N + e - PA::W]) * g.idy2;
        const float c1 = -(sE[2 * PA::N + e + 1] - sE[2 * PA::N + e - 1]) * g.idx2;
        const float c2 = (sE[PA::N + e + 1] - sE[PA::N + e - 1]) * g.idx2 -
                         (sE[e + PA::W] - sE[e - PA::W]) * g.idy2;
        const float d[3] = {-h * c0, -h * c1, -h * c2};
        if (s + 1 < K || FINAL) {
          // next substep's input (or the final B on a 1-cell halo), in
          // place: this cell alone is read here
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const float hi = sB[a * PB::N + b];
            const float yv = sL[a * PL::N + l] + d[a];
            const float tv = hi + yv;
            sL[a * PL::N + l] = yv - (tv - hi);
            sB[a * PB::N + b] = tv;
          }
        } else {
          const int x = tx0 + lx, y = ty0 + ly;
          if (x >= g.nx || y >= g.ny) continue;
          const int c = x + g.nx * y;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const float hi = sB[a * PB::N + b];
            const float yv = sL[a * PL::N + l] + d[a];
            const float tv = hi + yv;
            Lout[a * nc + c] = yv - (tv - hi);
            Bout[a * nc + c] = tv;
          }
        }
      }
    }
    if (s + 1 < K || FINAL) __syncthreads();
  }
  if (FINAL) {
    // E at the tile's cells from the final B = hi + lo (curl on the 1-cell
    // halo) and the extrapolated frozen terms, as k_field_final forms them
    bool below = false;
    double v[kDiagNV] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const int x = tx0 + fx, y = ty0 + fy;
    const bool live = fown && x < g.nx && y < g.ny;
    if (live) {
      auto Bf = [&](int a, int lx, int ly) {
        const int b = PB::at(lx, ly), l = PL::at(lx, ly);
        return sB[a * PB::N + b] + sL[a * PL::N + l];
      };
      const float ca = 1.5f, cb = -0.5f;
      float ne[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) ne[q] = ca * vf[q] + cb * vf[5 + q];
      below = vf[0] < eos.nfloor;
      auto pres = [&](float n) {
        return pressure(n, eos.nfloor, eos.te_n0, eos.n0, eos.gam, eos.iso);
      };
      const float inv = (float)(1.0 / (double)fmaxf(ne[0], eos.nfloor));
      float u[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) u[a] = (ca * vf[10 + a] + cb * vf[13 + a]) * inv;
      const float gp0 = -(pres(ne[1]) - pres(ne[2])) * g.idx2 * inv;
      const float gp1 = -(pres(ne[3]) - pres(ne[4])) * g.idy2 * inv;
      // curl B at the cell (2D: no z derivatives)
      const float j0 = (Bf(2, fx, fy + 1) - Bf(2, fx, fy - 1)) * g.idy2;
      const float j1 = -(Bf(2, fx + 1, fy) - Bf(2, fx - 1, fy)) * g.idx2;
      const float j2 = (Bf(1, fx + 1, fy) - Bf(1, fx - 1, fy)) * g.idx2 -
                       (Bf(0, fx, fy + 1) - Bf(0, fx, fy - 1)) * g.idy2;
      const float b0 = Bf(0, fx, fy), b1 = Bf(1, fx, fy), b2 = Bf(2, fx, fy);
      const float w0 = j0 * inv - u[0], w1 = j1 * inv - u[1], w2 = j2 * inv - u[2];
      const int c = x + g.nx * y;
      F.E[c] = (w1 * b2 - w2 * b1) + gp0 + eta * j0;
      F.E[nc + c] = (w2 * b0 - w0 * b2) + gp1 + eta * j1;
      F.E[2 * nc + c] = (w0 * b1 - w1 * b0) + 0.f + eta * j2;
      F.Bfin[c] = b0;
      F.Bfin[nc + c] = b1;
      F.Bfin[2 * nc + c] = b2;
      const double d0 = b0, d1 = b1, d2 = b2;
      v[0] = d0 * d0 + d1 * d1 + d2 * d2;
      v[1] = d0;
      v[2] = d1;
      v[3] = d2;
      if (F.part) v[4] = electron_energy(ne[0], eos);
    }
    const uint64_t m = __ballot(live && below);
    if ((threadIdx.x & 63) == 0 && m) {
      atomicOr(&F.st->flags, (uint32_t)HVPIC_FLAG_FLOOR_HIT);
      atomicAdd(&F.st->floor_hits, (unsigned long long)__builtin_popcountll(m));
    }
    if (F.part)
      tile_partial(v, F.part + kFieldPartStride * (int64_t)slot);
  }
}

template <int K, bool HAS_LIN, bool FINAL>
__global__ __launch_bounds__(kSubBlock) void k_field_sub2d(
    const float* __restrict__ Bin, const float* __restrict__ Lin, float* __restrict__ Bout,
    float* __restrict__ Lout, const float* __restrict__ nm, const float* __restrict__ Jm, float h,
    float eta, FGeo g, Eos eos, SubFinal F) {
  field_sub2d_body<kTX, kTY, K, HAS_LIN, FINAL>(Bin, Lin, Bout, Lout, nm, Jm, h, eta, g, eos, F,
                                                blockIdx.x, blockIdx.y,
                                                blockIdx.y * gridDim.x + blockIdx.x);
}

// E at the end of the step from the moments n_eff = ca*na + cb*nb,
// J_eff = ca*Ja + cb*Jb (EXTRAP; otherwise na, Ja), with B = Bh + Bl (HAS_LO;
// otherwise Bh),
// with the frozen terms formed per cell as in k_field_prep.  With Bout
// non-null the final B = hi + lo is also written there (Bout is never one of
// the arrays read).  Cells of na below the floor are counted when asked
// (once per field advance).  With part non-null, per-block FP64 partials
// {sum |B|^2, sum B, sum e(n_eff)} go to part (e as in electron_energy).
template <int NDIM, bool EXTRAP, bool HAS_LO>
__global__ __launch_bounds__(kBlock) void k_field_final(
    const float* __restrict__ Bh, const float* __restrict__ Bl, float* __restrict__ Bout,
    const float* __restrict__ na, const float* __restrict__ nb, const float* __restrict__ Ja,
    const float* __restrict__ Jb, float ca, float cb, float eta, FGeo g, Eos eos,
    float* __restrict__ E, double* part, Status* st, int count_floor) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  const int nc = g.ncell;
  const bool live = c < nc;
  bool below = false;
  double v[kDiagNV] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (live) {
    int i, j, k;
    fijk(c, g, i, j, k);
    const Nbr nn = neighbours(c, i, j, k, g);
    // every load first (no branch between them), then the arithmetic
    auto dens = [&](int q) { return EXTRAP ? ca * na[q] + cb * nb[q] : na[q]; };
    const float n_c = dens(c);
    const float n_xp = dens(nn.xp), n_xm = dens(nn.xm), n_yp = dens(nn.yp), n_ym = dens(nn.ym);
    const float n_zp = NDIM == 3 ? dens(nn.zp) : 0.f, n_zm = NDIM == 3 ? dens(nn.zm) : 0.f;
    float Jv[3];
    for (int a = 0; a < 3; ++a)
      Jv[a] = EXTRAP ? ca * Ja[a * nc + c] + cb * Jb[a * nc + c] : Ja[a * nc + c];
    const BSum<HAS_LO> B{Bh, Bl};
    float J[3];
    curl_at<NDIM>(B, c, g, J);
    const float b0 = B(c), b1 = B(nc + c), b2 = B(2 * nc + c);
    below = na[c] < eos.nfloor;
    auto pres = [&](float n) {
      return pressure(n, eos.nfloor, eos.te_n0, eos.n0, eos.gam, eos.iso);
    };
    const float inv = (float)(1.0 / (double)fmaxf(n_c, eos.nfloor));
    float u[3];
    for (int a = 0; a < 3; ++a) u[a] = Jv[a] * inv;
    float gp[3];
    gp[0] = -(pres(n_xp) - pres(n_xm)) * g.idx2 * inv;
    gp[1] = -(pres(n_yp) - pres(n_ym)) * g.idy2 * inv;
    gp[2] = NDIM == 3 ? -(pres(n_zp) - pres(n_zm)) * g.idz2 * inv : 0.f;
    const float w0 = J[0] * inv - u[0], w1 = J[1] * inv - u[1], w2 = J[2] * inv - u[2];
    E[c] = (w1 * b2 - w2 * b1) + gp[0] + eta * J[0];
    E[nc + c] = (w2 * b0 - w0 * b2) + gp[1] + eta * J[1];
    E[2 * nc + c] = (w0 * b1 - w1 * b0) + gp[2] + eta * J[2];
    if (Bout) {
      Bout[c] = b0;
      Bout[nc + c] = b1;
      Bout[2 * nc + c] = b2;
    }
    const double d0 = b0, d1 = b1, d2 = b2;
    v[0] = d0 * d0 + d1 * d1 + d2 * d2;
    v[1] = d0;
    v[2] = d1;
    v[3] = d2;
    if (part) v[4] = electron_energy(n_c, eos);
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

// Binomial smoothing (Sec. II.B): one pass is the (1,2,1)/4 filter along x,
// then y, then z.  A block smooths one component on one tile: it loads the
// tile with a halo of kSmHalo cells (periodic indexing, so a grid smaller
// than the halo wraps as often as needed), runs up to kSmHalo passes in LDS
// (each axis filter is valid one cell further in, so after p passes the
// tile itself is), and writes the tile.  Reads `in`, writes `out` (distinct:
// neighbouring tiles read the halo of `in`).
constexpr int kSmHalo = 4;
template <int NDIM>
struct SmTile {
  static constexpr int TX = NDIM == 2 ? 32 : 8, TY = 8, TZ = NDIM == 2 ? 1 : 8;
  static constexpr int H = kSmHalo, HZ = NDIM == 2 ? 0 : kSmHalo;
  static constexpr int WX = TX + 2 * H, WY = TY + 2 * H, WZ = TZ + 2 * HZ;
  static constexpr int N = WX * WY * WZ;
};

template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_smooth_tile(const float* __restrict__ in,
                                                        float* __restrict__ out, int npasses,
                                                        FGeo g) {
  using T = SmTile<NDIM>;
  __shared__ float A[T::N], Bf[T::N];
  const int ntx = (g.nx + T::TX - 1) / T::TX, nty = (g.ny + T::TY - 1) / T::TY;
  const int tile = blockIdx.x;
  const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
  const int x0 = tx * T::TX - T::H, y0 = ty * T::TY - T::H, z0 = tz * T::TZ - T::HZ;
  const float* f = in + (int64_t)blockIdx.y * g.ncell;
  auto wrap = [](int a, int n) { a %= n; return a < 0 ? a + n : a; };
  for (int q = threadIdx.x; q < T::N; q += kBlock) {
    const int lx = q % T::WX, ly = (q / T::WX) % T::WY, lz = q / (T::WX * T::WY);
    const int x = wrap(x0 + lx, g.nx), y = wrap(y0 + ly, g.ny), z = wrap(z0 + lz, g.nz);
    A[q] = f[x + g.nx * (y + g.ny * z)];
  }
  __syncthreads();
  float* cur = A;
  float* nxt = Bf;
  for (int pass = 0; pass < npasses; ++pass) {
    for (int axis = 0; axis < NDIM; ++axis) {
      const int st = axis == 0 ? 1 : (axis == 1 ? T::WX : T::WX * T::WY);
      const int wa = axis == 0 ? T::WX : (axis == 1 ? T::WY : T::WZ);
      for (int q = threadIdx.x; q < T::N; q += kBlock) {
        const int la = axis == 0 ? q % T::WX : (axis == 1 ? (q / T::WX) % T::WY : q / (T::WX * T::WY));
        // the cells at the buffer edge along this axis keep their value; they
        // are outside the region still valid after this pass
        nxt[q] = la > 0 && la < wa - 1 ? 0.25f * (cur[q - st] + 2.0f * cur[q] + cur[q + st]) : cur[q];
      }
      __syncthreads();
      float* t = cur;
      cur = nxt;
      nxt = t;
    }
  }
  float* o = out + (int64_t)blockIdx.y * g.ncell;
  for (int q = threadIdx.x; q < T::TX * T::TY * T::TZ; q += kBlock) {
    const int lx = q % T::TX, ly = (q / T::TX) % T::TY, lz = q / (T::TX * T::TY);
    const int x = tx * T::TX + lx, y = ty * T::TY + ly, z = tz * T::TZ + lz;
    if (x < g.nx && y < g.ny && z < g.nz)
      o[x + g.nx * (y + g.ny * z)] =
          cur[(lx + T::H) + T::WX * ((ly + T::H) + T::WY * (lz + T::HZ))];
  }
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
  const Eos eos = make_eos(c);
  const float eta = (float)c->p.eta;
  const float* fh = B;        // final B = fh + fl
  const float* fl = nullptr;
  bool fused_final = false;   // the last 2D tile launch wrote E, B and the partials
  if (mode == 0 && c->p.nsub > 0) {
    const float h = (float)(c->p.dt / c->p.nsub);
    if (NDIM == 2) {
      // two substeps per launch (one for an odd last one), the frozen terms
      // formed in each tile; the caller's B is only read (first launch)
      const dim3 tiles((unsigned)ceil_div(c->p.nx, kTX), (unsigned)ceil_div(c->p.ny, kTY));
      const size_t lds2 = sizeof(float) * SubLds<kTX, kTY, 2, false>::TOTAL,
                   lds1 = sizeof(float) * SubLds<kTX, kTY, 1, false>::TOTAL,
                   lds2f = sizeof(float) * SubLds<kTX, kTY, 2, true>::TOTAL,
                   lds1f = sizeof(float) * SubLds<kTX, kTY, 1, true>::TOTAL;
      const float* sh = B;
      const float* sl = nullptr;
      float* dh = Xh;
      float* dl = Xl;
      // With two or more launches the last one also writes E, the final B
      // and the diagnostic partials (the first reads the caller's B, which
      // the final one writes: never the same launch).
      fused_final = c->p.nsub >= 3;
      SubFinal F{};
      F.np = n_prev;
      F.Jp = J_prev;
      F.E = E_out;
      F.Bfin = B;
      F.part = diag_out ? c->field_part : nullptr;
      F.st = c->status;
      const SubFinal none{};
      for (int m = 0; m < c->p.nsub;) {
        const bool two = c->p.nsub - m >= 2;
        const bool fin = fused_final && m + (two ? 2 : 1) >= c->p.nsub;
        if (fin && two)
          hipLaunchKernelGGL((k_field_sub2d<2, true, true>), tiles, dim3(kSubBlock), lds2f, s, sh,
                             sl, dh, dl, n_half, J_half, h, eta, g, eos, F);
        else if (fin)
          hipLaunchKernelGGL((k_field_sub2d<1, true, true>), tiles, dim3(kSubBlock), lds1f, s, sh,
                             sl, dh, dl, n_half, J_half, h, eta, g, eos, F);
        else if (two && sl)
          hipLaunchKernelGGL((k_field_sub2d<2, true, false>), tiles, dim3(kSubBlock), lds2, s, sh,
                             sl, dh, dl, n_half, J_half, h, eta, g, eos, none);
        else if (two)
          hipLaunchKernelGGL((k_field_sub2d<2, false, false>), tiles, dim3(kSubBlock), lds2, s, sh,
                             sl, dh, dl, n_half, J_half, h, eta, g, eos, none);
        else if (sl)
          hipLaunchKernelGGL((k_field_sub2d<1, true, false>), tiles, dim3(kSubBlock), lds1, s, sh,
                             sl, dh, dl, n_half, J_half, h, eta, g, eos, none);
        else
          hipLaunchKernelGGL((k_field_sub2d<1, false, false>), tiles, dim3(kSubBlock), lds1, s, sh,
                             sl, dh, dl, n_half, J_half, h, eta, g, eos, none);
        m += two ? 2 : 1;
        sh = dh;
        sl = dl;
        dh = dh == Xh ? Yh : Xh;
        dl = dl == Xl ? Yl : Xl;
      }
      fh = sh;
      fl = sl;
    } else {
      // frozen moments for the subcycle
      hipLaunchKernelGGL((k_field_prep<NDIM>), grid, blk, 0, s, n_half, (const float*)nullptr,
                         J_half, (const float*)nullptr, 1.0f, 0.0f, g, eos.nfloor, eos.te_n0,
                         eos.n0, eos.gam, eos.iso, aux);
      const int cblocks = (int)std::min<int64_t>(ceil_div(3ll * nc, kBlock), 1024);
      hipLaunchKernelGGL(k_copy, dim3(cblocks), blk, 0, s, (const float*)B, Xh, 3ll * nc);
      hipLaunchKernelGGL(k_fill, dim3(cblocks), blk, 0, s, Xl, 3ll * nc, 0.0f);
      float* Es = c->fscratch + 19ll * nc;  // E of a stage
      for (int m = 0; m < c->p.nsub; ++m) {
        hipLaunchKernelGGL((k_field_ohm_cells<NDIM>), grid, blk, 0, s, (const float*)Xh, eta, g,
                           aux, Es);
        hipLaunchKernelGGL((k_field_curl_update<NDIM>), grid, blk, 0, s, (const float*)Es,
                           (const float*)Xh, Yh, (float*)nullptr, 0.5f * h, g);
        hipLaunchKernelGGL((k_field_ohm_cells<NDIM>), grid, blk, 0, s, (const float*)Yh, eta, g,
                           aux, Es);
        hipLaunchKernelGGL((k_field_curl_update<NDIM>), grid, blk, 0, s, (const float*)Es,
                           (const float*)Xh, Xh, Xl, h, g);
      }
      fh = Xh;
      fl = Xl;
    }
  }
  // E^{n+1} from the extrapolated moments (mode 0) or E from the given ones
  // (mode 1), the final B, the floor count of n_half and the diagnostics
  const double V = c->p.dx * c->p.dy * c->p.dz;
  const double we_scale = eos.iso ? V * c->p.te : V * c->p.n0 * c->p.te / (c->p.gamma_e - 1.0);
  if (fused_final) {
    if (diag_out) {
      const dim3 tiles((unsigned)ceil_div(c->p.nx, kTX), (unsigned)ceil_div(c->p.ny, kTY));
      hipLaunchKernelGGL(k_field_diag_final, dim3(1), dim3(1024), 0, s,
                         (const double*)c->field_part, (int)(tiles.x * tiles.y), diag_out,
                         0.5 * V, 1.0 / (double)nc, we_scale);
    }
    return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
  }
  auto final_kernel = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, blk, 0, s, fh, fl, fh == B ? nullptr : B, n_half, n_prev,
                       J_half, J_prev, 1.5f, -0.5f, eta, g, eos, E_out,
                       diag_out ? c->field_part : nullptr, c->status, 1);
  };
  if (mode == 0 && fl)
    final_kernel(k_field_final<NDIM, true, true>);
  else if (mode == 0)
    final_kernel(k_field_final<NDIM, true, false>);
  else
    final_kernel(k_field_final<NDIM, false, false>);
  if (diag_out)
    hipLaunchKernelGGL(k_field_diag_final, dim3(1), dim3(1024), 0, s, (const double*)c->field_part,
                       (int)grid.x, diag_out, 0.5 * V, 1.0 / (double)nc, we_scale);
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

// Surrogate check: per-block FP64 partials of sum |Bno - T|^2 and
// sum |Bno - B|^2, where T = B - dt curl E((B + Bno)/2) (so that
// (Bno - T)/dt is the residual r and (Bno - B)/dt the proposed rate).
__global__ __launch_bounds__(kBlock) void k_no_resid(const float* __restrict__ Bno,
                                                     const float* __restrict__ T,
                                                     const float* __restrict__ B, int ncell,
                                                     double* part) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (c < ncell)
    for (int a = 0; a < 3; ++a) {
      const int q = a * ncell + c;
      const double r = (double)Bno[q] - (double)T[q], d = (double)Bno[q] - (double)B[q];
      v[0] += r * r;
      v[1] += d * d;
    }
  block_partial<2, kFieldPartStride>(v, part);
}

// The decision: accepted when ||r|| <= tol ||rate|| (finite, nonzero rate).
__global__ __launch_bounds__(1024) void k_no_decide(const double* part, int nblocks, float tol,
                                                    Status* st, double* stats) {
  double r[2];
  sum_partials<2, kFieldPartStride>(part, nblocks, r);
  if (threadIdx.x == 0) {
    const double ratio = r[1] > 0.0 ? sqrt(r[0] / r[1]) : INFINITY;
    const bool ok = isfinite(ratio) && ratio <= (double)tol;
    st->no_accept = ok ? 1u : 0u;
    if (stats) {
      stats[0] = ratio;
      stats[1] = ok ? 1.0 : 0.0;
    }
  }
}

__global__ void k_mid(const float* __restrict__ a, const float* __restrict__ b,
                      float* __restrict__ m, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) m[i] = 0.5f * (a[i] + b[i]);
}

// The accepted proposal becomes the subcycle's result (hi = Bno, lo = 0).
__global__ void k_no_take(const float* __restrict__ Bno, float* __restrict__ hi,
                          float* __restrict__ lo, int64_t n, const Status* st) {
  if (!st->no_accept) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    hi[i] = Bno[i];
    lo[i] = 0.0f;
  }
}

}  // namespace

int launch_field_advance_no(hvpic_ctx* c, float* B, const float* n_half, const float* J_half,
                            const float* n_prev, const float* J_prev, float* E_out,
                            double* diag_out, const float* Bno, float tol, double* stats) {
  const FGeo g = fgeo(c);
  const int nc = c->ncell;
  const dim3 grid((unsigned)ceil_div(nc, kBlock)), blk(kBlock);
  hipStream_t s = c->stream;
  const Eos eos = make_eos(c);
  const float eta = (float)c->p.eta;
  Aux aux;
  aux.inv = c->fscratch;
  aux.u = c->fscratch + nc;
  aux.gp = c->fscratch + 4ll * nc;
  float* Xh = c->fscratch + 7ll * nc;
  float* Xl = c->fscratch + 10ll * nc;
  float* Yh = c->fscratch + 13ll * nc;
  float* Yl = c->fscratch + 16ll * nc;
  float* Bmid = c->fscratch + 19ll * nc;
  float* T = Yl;  // consumed before the fallback's second launch writes Y
  const int64_t n3 = 3ll * nc;
  const unsigned g3 = (unsigned)ceil_div(n3, kBlock);
  // residual test of the proposal
  hipLaunchKernelGGL(k_mid, dim3(g3), blk, 0, s, (const float*)B, Bno, Bmid, n3);
  hipLaunchKernelGGL((k_field_prep<2>), grid, blk, 0, s, n_half, (const float*)nullptr, J_half,
                     (const float*)nullptr, 1.0f, 0.0f, g, eos.nfloor, eos.te_n0, eos.n0, eos.gam,
                     eos.iso, aux);
  hipLaunchKernelGGL((k_field_stage<2>), grid, blk, 0, s, (const float*)Bmid, (const float*)B, T,
                     (float*)nullptr, (float)c->p.dt, eta, g, aux);
  hipLaunchKernelGGL(k_no_resid, grid, blk, 0, s, Bno, (const float*)T, (const float*)B, nc,
                     c->field_part);
  hipLaunchKernelGGL(k_no_decide, dim3(1), dim3(1024), 0, s, (const double*)c->field_part,
                     (int)grid.x, tol, c->status, stats);
  // the plain subcycle, skipped by its kernels when the proposal was accepted
  const float h = (float)(c->p.dt / c->p.nsub);
  const dim3 tiles((unsigned)ceil_div(c->p.nx, kTX), (unsigned)ceil_div(c->p.ny, kTY));
  const size_t lds2 = sizeof(float) * SubLds<kTX, kTY, 2, false>::TOTAL,
               lds1 = sizeof(float) * SubLds<kTX, kTY, 1, false>::TOTAL;
  SubFinal guard{};
  guard.skip = &c->status->no_accept;
  const float* sh = B;
  const float* sl = nullptr;
  float* dh = Xh;
  float* dl = Xl;
  for (int m = 0; m < c->p.nsub;) {
    const bool two = c->p.nsub - m >= 2;
    if (two && sl)
      hipLaunchKernelGGL((k_field_sub2d<2, true, false>), tiles, dim3(kSubBlock), lds2, s, sh, sl,
                         dh, dl, n_half, J_half, h, eta, g, eos, guard);
    else if (two)
      hipLaunchKernelGGL((k_field_sub2d<2, false, false>), tiles, dim3(kSubBlock), lds2, s, sh, sl,
                         dh, dl, n_half, J_half, h, eta, g, eos, guard);
    else if (sl)
      hipLaunchKernelGGL((k_field_sub2d<1, true, false>), tiles, dim3(kSubBlock), lds1, s, sh, sl,
                         dh, dl, n_half, J_half, h, eta, g, eos, guard);
    else
      hipLaunchKernelGGL((k_field_sub2d<1, false, false>), tiles, dim3(kSubBlock), lds1, s, sh,
                         sl, dh, dl, n_half, J_half, h, eta, g, eos, guard);
    m += two ? 2 : 1;
    sh = dh;
    sl = dl;
    dh = dh == Xh ? Yh : Xh;
    dl = dl == Xl ? Yl : Xl;
  }
  float* fh = const_cast<float*>(sh);
  float* fl = const_cast<float*>(sl);
  hipLaunchKernelGGL(k_no_take, dim3(g3), blk, 0, s, Bno, fh, fl, n3,
                     (const Status*)c->status);
  // E^{n+1}, the final B, the floor count and the diagnostics
  hipLaunchKernelGGL((k_field_final<2, true, true>), grid, blk, 0, s, (const float*)fh,
                     (const float*)fl, B, n_half, n_prev, J_half, J_prev, 1.5f, -0.5f, eta, g, eos,
                     E_out, diag_out ? c->field_part : nullptr, c->status, 1);
  if (diag_out) {
    const double V = c->p.dx * c->p.dy * c->p.dz;
    const double we_scale =
        eos.iso ? V * c->p.te : V * c->p.n0 * c->p.te / (c->p.gamma_e - 1.0);
    hipLaunchKernelGGL(k_field_diag_final, dim3(1), dim3(1024), 0, s, (const double*)c->field_part,
                       (int)grid.x, diag_out, 0.5 * V, 1.0 / (double)nc, we_scale);
  }
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

// 2D tile shapes of the subcycle kernel: the plain path uses shape 0; the
// ensemble's tuner picks one per run.
constexpr int kTileW[kTileShapes] = {32, 16, 64};
constexpr int kTileH[kTileShapes] = {8, 16, 4};
static_assert(kTileW[0] == kTX && kTileH[0] == kTY, "shape 0 is the plain path's tile");

int64_t field_part_slots(const hvpic_params* p) {
  const int64_t nc = (int64_t)p->nx * p->ny * p->nz;
  int64_t slots = ceil_div(nc, kBlock);
  if (p->ndim == 2)
    for (int t = 0; t < kTileShapes; ++t)
      slots = std::max(slots, ceil_div(p->nx, kTileW[t]) * ceil_div(p->ny, kTileH[t]));
  return slots;
}

// ------------------------------------------------------------ ensembles --
// The 2D subcycle (tile launches of one or two substeps, the last also
// writing E, the final B and the diagnostic partials) and the diagnostics'
// final sums, batched over the runs of an ensemble: per launch one record
// per run, one persistent launch over the (run, tile) items.

namespace {

struct FieldArgs {
  const float* Bin;
  const float* Lin;
  float* Bout;
  float* Lout;
  const float* nm;
  const float* Jm;
  float h, eta;
  FGeo g;
  Eos eos;
  SubFinal F;
  int ntx;  // tiles along x
};

template <int TX, int TY, int K, bool HAS_LIN, bool FINAL>
__global__ __launch_bounds__(kSubBlock) void k_field_sub2d_batch(const FieldArgs* __restrict__ tab,
                                                                 const Item* __restrict__ items,
                                                                 int nitems) {
  for_items(nitems, [&](int it) {
    const Item item = items[it];
    const FieldArgs A = tab[item.run];
    field_sub2d_body<TX, TY, K, HAS_LIN, FINAL>(A.Bin, A.Lin, A.Bout, A.Lout, A.nm, A.Jm, A.h,
                                                A.eta, A.g, A.eos, A.F, item.idx % A.ntx,
                                                item.idx / A.ntx, item.idx);
    __syncthreads();
  });
}

__global__ __launch_bounds__(1024) void k_field_diag_batch(const DiagArgs* __restrict__ tab,
                                                           int nruns) {
  for (int r = blockIdx.x; r < nruns; r += gridDim.x) {
    const DiagArgs D = tab[r];
    if (D.out) field_diag_body(D);  // uniform per block
    __syncthreads();
  }
}

template <int TX, int TY>
int field_batch_shape(hipStream_t s, int K, bool has_lin, bool fin, const FieldArgs* t,
                      const Item* items, int nitems, int grid) {
  auto go = [&](auto kern, size_t lds) {
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kSubBlock), lds, s, t, items, nitems);
  };
  constexpr size_t f = sizeof(float);
  if (fin && K == 2)
    go(k_field_sub2d_batch<TX, TY, 2, true, true>, f * SubLds<TX, TY, 2, true>::TOTAL);
  else if (fin)
    go(k_field_sub2d_batch<TX, TY, 1, true, true>, f * SubLds<TX, TY, 1, true>::TOTAL);
  else if (K == 2 && has_lin)
    go(k_field_sub2d_batch<TX, TY, 2, true, false>, f * SubLds<TX, TY, 2, false>::TOTAL);
  else if (K == 2)
    go(k_field_sub2d_batch<TX, TY, 2, false, false>, f * SubLds<TX, TY, 2, false>::TOTAL);
  else if (has_lin)
    go(k_field_sub2d_batch<TX, TY, 1, true, false>, f * SubLds<TX, TY, 1, false>::TOTAL);
  else
    go(k_field_sub2d_batch<TX, TY, 1, false, false>, f * SubLds<TX, TY, 1, false>::TOTAL);
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

}  // namespace

int ens_field_tiles(const hvpic_ctx* c, int shape) {
  return (int)(ceil_div(c->p.nx, kTileW[shape]) * ceil_div(c->p.ny, kTileH[shape]));
}

int ens_field_launches(const hvpic_ctx* c, int* K, int* has_lin, int* fin) {
  int n = 0;
  for (int m = 0; m < c->p.nsub; ++n) {
    const bool two = c->p.nsub - m >= 2;
    if (K) K[n] = two ? 2 : 1;
    if (has_lin) has_lin[n] = m > 0;
    m += two ? 2 : 1;
    if (fin) fin[n] = m >= c->p.nsub;
  }
  return n;
}

size_t ens_field_record(hvpic_ctx* c, float* B, const float* n_half, const float* J_half,
                        const float* n_prev, const float* J_prev, float* E_out, bool diag,
                        int launch, int shape, void* dst) {
  if (dst) {
    const int nc = c->ncell;
    // the ping-pong of the (hi, lo) pairs as the plain path runs it: launch
    // 0 reads the caller's B, launch m writes X for even m and Y for odd m
    float* Xh = c->fscratch + 7ll * nc;
    float* Xl = c->fscratch + 10ll * nc;
    float* Yh = c->fscratch + 13ll * nc;
    float* Yl = c->fscratch + 16ll * nc;
    FieldArgs A{};
    A.Bin = launch == 0 ? B : (launch % 2 == 1 ? Xh : Yh);
    A.Lin = launch == 0 ? nullptr : (launch % 2 == 1 ? Xl : Yl);
    A.Bout = launch % 2 == 0 ? Xh : Yh;
    A.Lout = launch % 2 == 0 ? Xl : Yl;
    A.nm = n_half;
    A.Jm = J_half;
    A.h = (float)(c->p.dt / c->p.nsub);
    A.eta = (float)c->p.eta;
    A.g = fgeo(c);
    A.eos = make_eos(c);
    int fin[64];
    const int nl = ens_field_launches(c, nullptr, nullptr, fin);
    if (launch == nl - 1) {
      A.F.np = n_prev;
      A.F.Jp = J_prev;
      A.F.E = E_out;
      A.F.Bfin = B;
      A.F.part = diag ? c->field_part : nullptr;
      A.F.st = c->status;
    }
    A.ntx = (int)ceil_div(c->p.nx, kTileW[shape]);
    memcpy(dst, &A, sizeof(A));
  }
  return sizeof(FieldArgs);
}

size_t ens_field_diag_record(hvpic_ctx* c, double* out, int shape, void* dst) {
  if (dst) {
    const Eos eos = make_eos(c);
    const double V = c->p.dx * c->p.dy * c->p.dz;
    const double we_scale =
        eos.iso ? V * c->p.te : V * c->p.n0 * c->p.te / (c->p.gamma_e - 1.0);
    const DiagArgs D{c->field_part, ens_field_tiles(c, shape), out, 0.5 * V,
                     1.0 / (double)c->ncell, we_scale};
    memcpy(dst, &D, sizeof(D));
  }
  return sizeof(DiagArgs);
}

int ens_launch_field(hipStream_t s, int shape, int K, int has_lin, int fin, const void* tab,
                     const Item* items, int nitems, int grid) {
  if (nitems == 0) return HVPIC_OK;
  const FieldArgs* t = static_cast<const FieldArgs*>(tab);
  if (shape == 1) return field_batch_shape<16, 16>(s, K, has_lin, fin, t, items, nitems, grid);
  if (shape == 2) return field_batch_shape<64, 4>(s, K, has_lin, fin, t, items, nitems, grid);
  return field_batch_shape<32, 8>(s, K, has_lin, fin, t, items, nitems, grid);
}

int ens_launch_field_diag(hipStream_t s, const void* tab, int nruns) {
  if (nruns == 0) return HVPIC_OK;
  hipLaunchKernelGGL(k_field_diag_batch, dim3((unsigned)std::min(nruns, 1024)), dim3(1024), 0, s,
                     static_cast<const DiagArgs*>(tab), nruns);
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

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
  float* T = c->fscratch;  // [ncomp][ncell] staging of one launch's output
  auto tiles = [&](auto tile) {
    return (unsigned)(ceil_div(c->p.nx, tile.TX) * ceil_div(c->p.ny, tile.TY) *
                      ceil_div(c->p.nz, tile.TZ));
  };
  for (int done = 0; done < npasses; done += kSmHalo) {
    const int p = std::min(kSmHalo, npasses - done);
    if (c->p.ndim == 2)
      hipLaunchKernelGGL(k_smooth_tile<2>, dim3(tiles(SmTile<2>{}), ncomp), dim3(kBlock), 0,
                         c->stream, (const float*)F, T, p, g);
    else
      hipLaunchKernelGGL(k_smooth_tile<3>, dim3(tiles(SmTile<3>{}), ncomp), dim3(kBlock), 0,
                         c->stream, (const float*)F, T, p, g);
    hipLaunchKernelGGL(k_copy, dim3((unsigned)std::min<int64_t>(ceil_div(total, kBlock), 2048)),
                       dim3(kBlock), 0, c->stream, (const float*)T, F, total);
  }
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

}  // namespace hvpic
