// Particle kernels of libhvpic.so for gfx950: gather + Boris push + move
// (optionally with the moment deposit fused in) and the stand-alone deposit.
//
// Method (arXiv 2305.05600):
//   gather   App. B eq:quadFI/eq:quadF (QS), Sec. II.B (NGP); evaluated from
//            per-cell polynomial coefficients in the particle offsets.
//   push     Sec. II.B eq:vadv, non-relativistic Boris split.
//   move     Sec. II.B position update; offsets renormalised into [-1,1).
//   deposit  Sec. II.B eq:ngp, App. B eq:quad, at x^{n+1/2}.
//
// Data path.  Particles are structure-of-arrays and sorted by cell.  A block
// owns a contiguous chunk of particles; each wavefront walks its share in
// steps of 256, lane l taking four consecutive particles per step (16-byte
// accesses, 1 KiB per wavefront and array).  Sorted input means a lane's
// four particles nearly always share a cell, and the block's cells [c0, c1]
// form a short linear range.
//   * gather window (LDS): one record per cell c0..c1 with the interpolant's
//     polynomial coefficients for E and B and the cell's (i, j[, k]);
//   * deposit window (LDS, FP64 n, Jx, Jy, Jz): "bands" of cells
//     [c0 - 2, c1 + 2] shifted by by*nx (+ bz*nx*ny), by, bz in -3..3, so a
//     stencil cell that wraps around the x (3D: y) boundary lands one band
//     over, with no division;
//   * each lane keeps running FP32 sums of its particles that deposit into
//     the same cell and adds them to the window with FP64 LDS atomics when
//     that cell changes or the step ends (at the step end a quad of lanes
//     whose sums share a cell combines them first); the block then adds its
//     window to FP64 global
//     accumulators, and one pass converts those to the FP32 outputs.
// Particles outside the windows (unsorted or sparse input) use global loads
// and FP64 global atomics.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "hvpic_internal.hpp"

namespace hvpic {
namespace {

// Particles per lane and per block, and the largest deposit-window width
// (cells per band).  A 3D chunk spans more bands, so it is kept shorter.
template <int NDIM>
struct Chunk {
  static constexpr int PPT = NDIM == 2 ? 12 : 4;
  static constexpr int N = kBlock * PPT;
  static constexpr int WMAX = NDIM == 2 ? 64 : 24;
};
static_assert(Chunk<3>::N == kChunk3, "workspace sizing of the 3D chunk order");

struct Geo {
  int nx, ny, nz, ncell, nxny;
  FastDiv fnx, fny;
};

struct PushArgs {
  int64_t n;
  int32_t* __restrict__ cell;
  float* __restrict__ ox;
  float* __restrict__ oy;
  float* __restrict__ oz;
  float* __restrict__ ux;
  float* __restrict__ uy;
  float* __restrict__ uz;
  const float* __restrict__ w;
  const float* __restrict__ E;
  const float* __restrict__ B;
  double* __restrict__ acc;  // fused deposit: FP64 moments [4][ncell] (n, Jx, Jy, Jz)
  Geo g;
  float a;                  // (q/m) dt / 2
  float kx, ky, kz;         // full-step displacement per unit speed (half-cells)
  float qV;                 // q / V_c
  double ms;
  double* diag_part;        // per-block partials of {K, Px, Py, Pz}, or null
  Status* st;
  bool vec;                 // all particle arrays 16-byte aligned
  const int32_t* cs;        // cell_start of the sorted store, or null
  uint32_t* cnt;            // moves per (old cell, direction), written when cs is given
  // Read through a gather map: particle k of the step is element perm[k] of
  // the source arrays below, and the pushed store (weights included) goes to
  // the arrays above.  perm null: the store above is read and written in place.
  const int32_t* perm;
  int64_t nsrc;             // elements of the source arrays (map entries index below it)
  const int32_t* icell;
  const float *iox, *ioy, *ioz, *iux, *iuy, *iuz, *iw;
  float* wo;
  bool off32;               // every source byte offset fits 32 bits (n < 2^30)
  const int32_t* order;     // position -> chunk (a permutation of the chunks), or null
};

struct DepArgs {
  int64_t n;
  const int32_t* __restrict__ cell;
  const float* __restrict__ ox;
  const float* __restrict__ oy;
  const float* __restrict__ oz;
  const float* __restrict__ ux;
  const float* __restrict__ uy;
  const float* __restrict__ uz;
  const float* __restrict__ w;
  double* __restrict__ acc;  // FP64 moments [4][ncell]
  Geo g;
  float bx, by, bz;         // displacement of the deposit point per unit speed
  float qV;
  Status* st;
  bool vec;
};

// Chunk of the store for hardware block b of nb.  The GPU hands blocks out
// round-robin over its 8 XCDs, each with its own L2, so XCD x takes a
// contiguous eighth of the chunks: blocks working on neighbouring rows of
// cells (the stencil halos, the deposit windows, particles read from the
// next row over) then share one L2.  A bijection of [0, nb).
__device__ __forceinline__ int xcd_chunk(int b, int nb) {
  constexpr int X = 8;
  const int per = nb / X, rem = nb % X;
  const int x = b % X, i = b / X;
  return x * per + min(x, rem) + i;
}

__device__ __forceinline__ void decompose(int a, const Geo& g, int& i, int& j, int& k) {
  uint32_t q = fdiv((uint32_t)a, g.fnx);
  i = a - (int)q * g.nx;
  uint32_t q2 = fdiv(q, g.fny);
  j = (int)q - (int)q2 * g.ny;
  k = (int)q2;
}

__device__ __forceinline__ int wrapi(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// Shift s with x - 2s in [-1,1).  Exact compares for the common |s| <= 1 case
// (x - 2 is exact for x in [1,3) by Sterbenz); general floor beyond.  Returns
// false for a non-finite / runaway value (the caller keeps the particle).
__device__ __forceinline__ bool renorm(float& x, int& s) {
  if (!(fabsf(x) < 1.0e6f)) return false;
  s = 0;
  if (x >= 1.0f) {
    s = 1;
    if (x >= 3.0f) s = (int)floorf((x + 1.0f) * 0.5f);
  } else if (x < -1.0f) {
    s = -1;
    if (x < -3.0f) s = (int)floorf((x + 1.0f) * 0.5f);
  }
  x -= 2.0f * (float)s;
  while (x >= 1.0f) { x -= 2.0f; ++s; }
  while (x < -1.0f) { x += 2.0f; --s; }
  return true;
}

// ---------------------------------------------------------------- gather --

template <int NDIM, int SHAPE>
__device__ __forceinline__ void gather_eb(const float* __restrict__ E, const float* __restrict__ B,
                                          int a, int i, int j, int k, float x, float y, float z,
                                          const Geo& g, float Ep[3], float Bp[3]) {
  const int nc = g.ncell;
  if (SHAPE == HVPIC_SHAPE_NGP) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Ep[c] = __ldg(E + c * nc + a);
      Bp[c] = __ldg(B + c * nc + a);
    }
    return;
  }
  const int im = i == 0 ? a + g.nx - 1 : a - 1;
  const int ip = i == g.nx - 1 ? a - g.nx + 1 : a + 1;
  const int jm = j == 0 ? a + g.nxny - g.nx : a - g.nx;
  const int jp = j == g.ny - 1 ? a - g.nxny + g.nx : a + g.nx;
  const float c12 = 1.0f / 12.0f;
  const float xp = 1.0f + x, xm = 1.0f - x, yp = 1.0f + y, ym = 1.0f - y;
  const float wxp = xp * xp * c12, wxm = xm * xm * c12, wyp = yp * yp * c12, wym = ym * ym * c12;
  // centre weight as one minus the others (see dep_weights)
  if (NDIM == 2) {
    const float w0 = 1.0f - ((wxp + wxm) + (wyp + wym));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float* e = E + c * nc;
      const float* b = B + c * nc;
      Ep[c] = w0 * __ldg(e + a) + wxp * __ldg(e + ip) + wxm * __ldg(e + im) + wyp * __ldg(e + jp) +
              wym * __ldg(e + jm);
      Bp[c] = w0 * __ldg(b + a) + wxp * __ldg(b + ip) + wxm * __ldg(b + im) + wyp * __ldg(b + jp) +
              wym * __ldg(b + jm);
    }
  } else {
    const int km = k == 0 ? a + nc - g.nxny : a - g.nxny;
    const int kp = k == g.nz - 1 ? a - nc + g.nxny : a + g.nxny;
    const float zp = 1.0f + z, zm = 1.0f - z;
    const float wzp = zp * zp * c12, wzm = zm * zm * c12;
    const float w0 = 1.0f - ((wxp + wxm) + (wyp + wym) + (wzp + wzm));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float* e = E + c * nc;
      const float* b = B + c * nc;
      Ep[c] = w0 * __ldg(e + a) + wxp * __ldg(e + ip) + wxm * __ldg(e + im) + wyp * __ldg(e + jp) +
              wym * __ldg(e + jm) + wzp * __ldg(e + kp) + wzm * __ldg(e + km);
      Bp[c] = w0 * __ldg(b + a) + wxp * __ldg(b + ip) + wxm * __ldg(b + im) + wyp * __ldg(b + jp) +
              wym * __ldg(b + jm) + wzp * __ldg(b + kp) + wzm * __ldg(b + km);
    }
  }
}

// ---------------------------------------------------------------- windows --

// Gather record of one cell: the interpolated field as a polynomial in the
// particle's offsets (x, y[, z] in half-cell units), for the six components
// (Ex, Ey, Ez, Bx, By, Bz), followed by the cell's integer indices i, j[, k].
// Coefficient c of component f is stored at [c * 6 + f]:
//   2D QS: F = c0 + c1 x + c2 y + c3 x^2 + c4 y^2
//   3D QS: F = c0 + c1 x + c2 y + c3 z + c4 x^2 + c5 y^2 + c6 z^2
//   NGP:   F = c0
// For QS these are the App. B eq:quad weights (equivalently the
// eq:quadFI/eq:quadF interpolant) applied to the cell's 5- or 7-point
// neighbourhood and collected by powers of the offsets.
template <int NDIM, int SHAPE>
struct Rec {
  static constexpr int NC = SHAPE == HVPIC_SHAPE_NGP ? 1 : (NDIM == 2 ? 5 : 7);
  static constexpr int NF4 = (NC * 6 + NDIM + 3) / 4;  // float4 per record
};

template <int NDIM, int SHAPE>
struct Stencil {
  static constexpr int T = SHAPE == HVPIC_SHAPE_NGP ? 1 : (NDIM == 2 ? 5 : 7);
};

template <int NDIM>
__device__ __forceinline__ bool window_ok(int c0, int c1, const Geo& g, int& W) {
  W = c1 - c0 + 5;
  return c0 >= 0 && c1 < g.ncell && c1 >= c0 && W <= Chunk<NDIM>::WMAX && g.nx >= 4 &&
         (NDIM == 2 || g.ny >= 4);
}

// Linear cell of deposit-window column `off` in band (by, bz): the window
// starts two cells before c0; band (by, bz) is shifted by by*nx + bz*nx*ny.
// |by|, |bz| <= 2 and 0 <= c0 - 2 + off < ncell + WMAX, so the index is
// within a few grid lengths of the grid: wrapped by adds and subtracts
// instead of a 64-bit remainder.
__device__ __forceinline__ int64_t window_cell(int c0, int off, int by, int bz, const Geo& g) {
  int64_t c = (int64_t)c0 - 2 + off + (int64_t)by * g.nx + (int64_t)bz * g.nxny;
  while (c < 0) c += g.ncell;
  while (c >= g.ncell) c -= g.ncell;
  return c;
}

// Fills the gather records of cells c0 .. c0 + ncells - 1 (all inside the
// grid).  One thread per (cell, component).
template <int NDIM, int SHAPE>
__device__ void gwin_fill(float* gw, int ncells, int c0, const Geo& g,
                          const float* __restrict__ E, const float* __restrict__ B) {
  constexpr int NC = Rec<NDIM, SHAPE>::NC;
  constexpr int RL = Rec<NDIM, SHAPE>::NF4 * 4;
  const int nc = g.ncell;
  for (int s = threadIdx.x; s < ncells * 6; s += kBlock) {
    const int r = s / 6, comp = s - 6 * r;
    const int a = c0 + r;
    int i, j, k;
    decompose(a, g, i, j, k);
    const float* F = comp < 3 ? E + comp * nc : B + (comp - 3) * nc;
    float* rec = gw + r * RL;
    const float f0 = __ldg(F + a);
    if (SHAPE == HVPIC_SHAPE_NGP) {
      rec[comp] = f0;
    } else {
      const int im = i == 0 ? a + g.nx - 1 : a - 1;
      const int ip = i == g.nx - 1 ? a - g.nx + 1 : a + 1;
      const int jm = j == 0 ? a + g.nxny - g.nx : a - g.nx;
      const int jp = j == g.ny - 1 ? a - g.nxny + g.nx : a + g.nx;
      const float fxp = __ldg(F + ip), fxm = __ldg(F + im);
      const float fyp = __ldg(F + jp), fym = __ldg(F + jm);
      const float c6 = 1.0f / 6.0f, c12 = 1.0f / 12.0f;
      // written with the second differences, F0 = F + (sum of the
      // neighbours - 2 ndim F)/12 (the same value as (6F + sum)/12 in 3D):
      // a uniform field has zero differences and is gathered exactly, which
      // the FP32 roundings of 1/6 and 1/12 would otherwise bias by ~3e-8
      const float dxx = (fxp + fxm) - 2.0f * f0, dyy = (fyp + fym) - 2.0f * f0;
      if (NDIM == 2) {
        rec[0 * 6 + comp] = fmaf(dxx + dyy, c12, f0);
        rec[1 * 6 + comp] = (fxp - fxm) * c6;
        rec[2 * 6 + comp] = (fyp - fym) * c6;
        rec[3 * 6 + comp] = dxx * c12;
        rec[4 * 6 + comp] = dyy * c12;
      } else {
        const int km = k == 0 ? a + nc - g.nxny : a - g.nxny;
        const int kp = k == g.nz - 1 ? a - nc + g.nxny : a + g.nxny;
        const float fzp = __ldg(F + kp), fzm = __ldg(F + km);
        const float dzz = (fzp + fzm) - 2.0f * f0;
        rec[0 * 6 + comp] = fmaf((dxx + dyy) + dzz, c12, f0);
        rec[1 * 6 + comp] = (fxp - fxm) * c6;
        rec[2 * 6 + comp] = (fyp - fym) * c6;
        rec[3 * 6 + comp] = (fzp - fzm) * c6;
        rec[4 * 6 + comp] = dxx * c12;
        rec[5 * 6 + comp] = dyy * c12;
        rec[6 * 6 + comp] = dzz * c12;
      }
    }
    if (comp == 0) {
      int* ri = reinterpret_cast<int*>(rec + NC * 6);
      ri[0] = i;
      ri[1] = j;
      if (NDIM == 3) ri[2] = k;
    }
  }
}

// Field at a particle of window cell rel with offsets (x, y, z); also returns
// the cell's indices.
template <int NDIM, int SHAPE>
__device__ __forceinline__ void gather_rec(const float4* gw, int rel, float x, float y, float z,
                                           float Ep[3], float Bp[3], int& i, int& j, int& k) {
  constexpr int NF4 = Rec<NDIM, SHAPE>::NF4;
  constexpr int NC = Rec<NDIM, SHAPE>::NC;
  if (SHAPE == HVPIC_SHAPE_QS) {
    // the record's monomials, then coefficient by coefficient (8-byte reads
    // of its six components), so that few of the record's 30 (2D) or 42 (3D)
    // values are live at once: the 3D push then fits four wavefronts per
    // SIMD without spills
    const float* q = reinterpret_cast<const float*>(gw + rel * NF4);
    float m[NC];
    m[0] = 1.0f;
    m[1] = x;
    m[2] = y;
    if constexpr (NDIM == 2) {
      m[3] = x * x;
      m[4] = y * y;
    } else {
      m[3] = z;
      m[4] = x * x;
      m[5] = y * y;
      m[6] = z * z;
    }
    float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
      for (int h = 0; h < 3; ++h) {
        const float2 v = *reinterpret_cast<const float2*>(q + c * 6 + 2 * h);
        acc[2 * h] = fmaf(m[c], v.x, acc[2 * h]);
        acc[2 * h + 1] = fmaf(m[c], v.y, acc[2 * h + 1]);
      }
    }
    Ep[0] = acc[0];
    Ep[1] = acc[1];
    Ep[2] = acc[2];
    Bp[0] = acc[3];
    Bp[1] = acc[4];
    Bp[2] = acc[5];
    const int* ri = reinterpret_cast<const int*>(q + NC * 6);
    i = ri[0];
    j = ri[1];
    k = NDIM == 3 ? ri[2] : 0;
    return;
  }
  float r[NF4 * 4];
  const float4* p = gw + rel * NF4;
#pragma unroll
  for (int q = 0; q < NF4; ++q) {
    const float4 v = p[q];
    r[4 * q] = v.x;
    r[4 * q + 1] = v.y;
    r[4 * q + 2] = v.z;
    r[4 * q + 3] = v.w;
  }
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    float v;
    if (SHAPE == HVPIC_SHAPE_NGP)
      v = r[f];
    else if (NDIM == 2)
      v = fmaf(x, fmaf(x, r[18 + f], r[6 + f]), fmaf(y, fmaf(y, r[24 + f], r[12 + f]), r[f]));
    else
      v = fmaf(x, fmaf(x, r[24 + f], r[6 + f]),
               fmaf(y, fmaf(y, r[30 + f], r[12 + f]), fmaf(z, fmaf(z, r[36 + f], r[18 + f]), r[f])));
    if (f < 3)
      Ep[f] = v;
    else
      Bp[f - 3] = v;
  }
  i = __float_as_int(r[NC * 6]);
  j = __float_as_int(r[NC * 6 + 1]);
  k = NDIM == 3 ? __float_as_int(r[NC * 6 + 2]) : 0;
}

// ---------------------------------------------------------------- deposit --

// Stencil weights at deposit offsets (x, y, z): centre, +x, -x, +y, -y[, +z, -z]
// (Sec. II.B eq:ngp, App. B eq:quad).  The weights of eq:quad sum to one; the
// centre weight is taken as one minus the others (the same value as
// (3 - x^2 - y^2 - z^2)/6, or (4 - x^2 - y^2)/6 in 2D), so each particle
// deposits its whole charge in FP32 too: with the FP32 roundings of 1/6 and
// 1/12 the printed form deposits ~3e-8 too much, always in the same direction.
template <int NDIM, int SHAPE>
__device__ __forceinline__ void dep_weights(float x, float y, float z, float* wt) {
  if (SHAPE == HVPIC_SHAPE_NGP) {
    wt[0] = 1.0f;
    return;
  }
  const float c12 = 1.0f / 12.0f;
  const float xp = 1.0f + x, xm = 1.0f - x, yp = 1.0f + y, ym = 1.0f - y;
  wt[1] = xp * xp * c12;
  wt[2] = xm * xm * c12;
  wt[3] = yp * yp * c12;
  wt[4] = ym * ym * c12;
  float side = (wt[1] + wt[2]) + (wt[3] + wt[4]);
  if (NDIM == 3) {
    const float zp = 1.0f + z, zm = 1.0f - z;
    wt[5] = zp * zp * c12;
    wt[6] = zm * zm * c12;
    side += wt[5] + wt[6];
  }
  wt[0] = 1.0f - side;
}

// Deposit window: FP64 (n, Jx, Jy, Jz) per slot; slot = band * SW + column,
// band = (by + 2) [+ 5 (bz + 2)] for band offsets by, bz in -2..2.  A home
// cell (a particle's deposit cell) takes bands -1..1 only, so that its
// stencil stays inside; the rare deposit cell further out (a diagonal
// mid-point at a wrapped x or y edge) goes to the global accumulators.
template <int NDIM>
struct DWin {
  static constexpr int SW = Chunk<NDIM>::WMAX;  // slots per band
  static constexpr int BZ = 5 * SW;             // slots per z band row (3D)
  static constexpr int NB = NDIM == 2 ? 5 : 25;
  static constexpr int LEN = NB * SW * 4;       // doubles
};

// The block's deposit window in LDS: the FP64 sums, and per slot the wrap
// bits (as in stencil_slots) of that slot's cell.
struct WinLds {
  double* acc;
  const uint8_t* wrap;
};

// Window slots of the stencil cells of the cell at slot `key`; wrap bit 0/1:
// its +x/-x neighbour wraps around the x boundary, bit 2/3 the same for y (3D).
template <int NDIM, int SHAPE>
__device__ __forceinline__ void stencil_slots(int key, int wrap, int* s) {
  constexpr int SW = DWin<NDIM>::SW, BZ = DWin<NDIM>::BZ;
  s[0] = key;
  if (SHAPE == HVPIC_SHAPE_QS) {
    s[1] = key + 1 - ((wrap & 1) ? SW : 0);
    s[2] = key - 1 + ((wrap & 2) ? SW : 0);
    if (NDIM == 2) {
      s[3] = key + SW;
      s[4] = key - SW;
    } else {
      s[3] = key + SW - ((wrap & 4) ? BZ : 0);
      s[4] = key - SW + ((wrap & 8) ? BZ : 0);
      s[5] = key + BZ;
      s[6] = key - BZ;
    }
  }
}

// Wrap bits (as in stencil_slots) of the cell with indices (i, j).
template <int NDIM>
__device__ __forceinline__ int wrap_bits(int i, int j, const Geo& g) {
  int w = (i == g.nx - 1 ? 1 : 0) | (i == 0 ? 2 : 0);
  if (NDIM == 3) w |= (j == g.ny - 1 ? 4 : 0) | (j == 0 ? 8 : 0);
  return w;
}

// Window slot of the cell (mx, my, mz) away from the cell of window column
// `rel` with indices (i, j), as a home cell; -1 when its band offset is
// beyond -1..1 (the particle then deposits to the global accumulators).
template <int NDIM>
__device__ __forceinline__ int window_slot(int rel, int i, int j, int mx, int my, int mz,
                                           const Geo& g) {
  const int t1 = i + mx;
  const int wx = t1 < 0 ? 1 : (t1 >= g.nx ? -1 : 0);
  const int by = my + wx;
  int bz = 0;
  if (NDIM == 3) {
    const int t2 = j + my;
    const int wy = t2 < 0 ? 1 : (t2 >= g.ny ? -1 : 0);
    bz = mz + wy;
  }
  if (by < -1 || by > 1 || bz < -1 || bz > 1) return -1;
  const int band = NDIM == 3 ? (by + 2) + 5 * (bz + 2) : by + 2;
  return band * DWin<NDIM>::SW + rel + mx + 2;
}

// Deposit straight into the FP64 global accumulators (particles outside the
// windows).
template <int NDIM, int SHAPE>
__device__ __forceinline__ void deposit_global(int i, int j, int k, int mx, int my, int mz,
                                               const float* wt, float q, float vx, float vy,
                                               float vz, const Geo& g, double* __restrict__ acc) {
  constexpr int T = Stencil<NDIM, SHAPE>::T;
  const int nc = g.ncell;
  int sx[T], sy[T], sz[T];
  sx[0] = sy[0] = sz[0] = 0;
  if (SHAPE == HVPIC_SHAPE_QS) {
    sx[1] = 1; sy[1] = 0; sz[1] = 0;
    sx[2] = -1; sy[2] = 0; sz[2] = 0;
    sx[3] = 0; sy[3] = 1; sz[3] = 0;
    sx[4] = 0; sy[4] = -1; sz[4] = 0;
    if (NDIM == 3) {
      sx[5] = 0; sy[5] = 0; sz[5] = 1;
      sx[6] = 0; sy[6] = 0; sz[6] = -1;
    }
  }
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int c = wrapi(i + mx + sx[t], g.nx) +
                  g.nx * (wrapi(j + my + sy[t], g.ny) + g.ny * wrapi(k + mz + sz[t], g.nz));
    const float nq = q * wt[t];
    unsafeAtomicAdd(acc + c, (double)nq);
    unsafeAtomicAdd(acc + nc + c, (double)(nq * vx));
    unsafeAtomicAdd(acc + 2 * nc + c, (double)(nq * vy));
    unsafeAtomicAdd(acc + 3 * nc + c, (double)(nq * vz));
  }
}

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

__device__ __forceinline__ int lanes_below_count(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Orders the wavefront's LDS writes before its following LDS reads.
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-wavefront queue (LDS, structure-of-arrays of QCAP entries) of deposits
// that do not add to their lane's running sums: word 0 = window slot, then
// the deposit offsets, the charge factor and the velocity.
template <int NDIM>
struct Queue {
  static constexpr int QCAP = 64;
  static constexpr int QW = NDIM == 2 ? 7 : 8;  // words per entry
  float* base;
  int count;  // wavefront-uniform
};

// Adds every queued deposit to the window, lane e taking entry e.
template <int NDIM, int SHAPE>
__device__ __forceinline__ void queue_drain(Queue<NDIM>& Q, const WinLds& wl) {
  constexpr int T = Stencil<NDIM, SHAPE>::T;
  constexpr int QC = Queue<NDIM>::QCAP, o = NDIM == 3 ? 4 : 3;
  if (Q.count == 0) return;
  wave_sync_lds();
  const int e = threadIdx.x & 63;
  if (e < Q.count) {
    const float* b = Q.base;
    const int key = __float_as_int(b[e]);
    const float x = b[QC + e], y = b[2 * QC + e];
    const float z = NDIM == 3 ? b[3 * QC + e] : 0.0f;
    const float q = b[o * QC + e], vx = b[(o + 1) * QC + e];
    const float vy = b[(o + 2) * QC + e], vz = b[(o + 3) * QC + e];
    float wt[T];
    dep_weights<NDIM, SHAPE>(x, y, z, wt);
    int s[T];
    stencil_slots<NDIM, SHAPE>(key, wl.wrap[key], s);
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const float nq = q * wt[t];
      atomicAdd(wl.acc + s[t] * 4 + 0, (double)nq);
      atomicAdd(wl.acc + s[t] * 4 + 1, (double)(nq * vx));
      atomicAdd(wl.acc + s[t] * 4 + 2, (double)(nq * vy));
      atomicAdd(wl.acc + s[t] * 4 + 3, (double)(nq * vz));
    }
  }
  wave_sync_lds();
  Q.count = 0;
}

// Queues this lane's deposit when `exc`; every lane of the wavefront calls it.
template <int NDIM, int SHAPE>
__device__ __forceinline__ void queue_push(Queue<NDIM>& Q, const WinLds& wl, bool exc, int key,
                                           float x, float y, float z, float q, float vx,
                                           float vy, float vz) {
  constexpr int QC = Queue<NDIM>::QCAP, o = NDIM == 3 ? 4 : 3;
  const uint64_t m = __ballot(exc);
  if (m == 0) return;
  const int add = __builtin_popcountll(m);
  if (Q.count + add > QC) queue_drain<NDIM, SHAPE>(Q, wl);
  if (exc) {
    const int e = Q.count + lanes_below_count(m);
    float* b = Q.base;
    b[e] = __int_as_float(key);
    b[QC + e] = x;
    b[2 * QC + e] = y;
    if (NDIM == 3) b[3 * QC + e] = z;
    b[o * QC + e] = q;
    b[(o + 1) * QC + e] = vx;
    b[(o + 2) * QC + e] = vy;
    b[(o + 3) * QC + e] = vz;
  }
  Q.count += add;
}

// A lane's running FP32 moment sums for its home cell: the deposit cell of
// the first particle of its current group of four.
template <int NDIM, int SHAPE>
struct Home {
  float acc[Stencil<NDIM, SHAPE>::T][4];
  int key;  // window slot of the home cell, -1 if none yet
};

template <int NDIM, int SHAPE>
__device__ __forceinline__ void home_clear(Home<NDIM, SHAPE>& H) {
  H.key = -1;
#pragma unroll
  for (int t = 0; t < Stencil<NDIM, SHAPE>::T; ++t)
    H.acc[t][0] = H.acc[t][1] = H.acc[t][2] = H.acc[t][3] = 0.0f;
}

// Deposit of one particle: into the home sums when its deposit cell is the
// home cell, else into the queue (in the window) or the global accumulators.
// Every lane of the wavefront calls it.
template <int NDIM, int SHAPE>
__device__ __forceinline__ void deposit_particle(Home<NDIM, SHAPE>& H, Queue<NDIM>& Q,
                                                 const WinLds& wl, bool live, bool inwin, int rel,
                                                 int i, int j, int k, int mx, int my, int mz,
                                                 float x, float y, float z, float q, float vx,
                                                 float vy, float vz, const Geo& g,
                                                 double* __restrict__ acc) {
  constexpr int T = Stencil<NDIM, SHAPE>::T;
  const bool near = live && inwin && mx >= -1 && mx <= 1 && my >= -1 && my <= 1 &&
                    mz >= -1 && mz <= 1;
  const int key = near ? window_slot<NDIM>(rel, i, j, mx, my, mz, g) : -1;
  const bool use_win = key >= 0;
  if (use_win && H.key < 0) H.key = key;
  const bool stay = use_win && key == H.key;
  float wt[T];
  dep_weights<NDIM, SHAPE>(x, y, z, wt);
  const float qm = stay ? q : 0.0f;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const float a = qm * wt[t];
    H.acc[t][0] += a;
    H.acc[t][1] = fmaf(a, vx, H.acc[t][1]);
    H.acc[t][2] = fmaf(a, vy, H.acc[t][2]);
    H.acc[t][3] = fmaf(a, vz, H.acc[t][3]);
  }
  queue_push<NDIM, SHAPE>(Q, wl, use_win && !stay, key, x, y, z, q, vx, vy, vz);
  const bool global = live && !use_win;
  if (__ballot(global) != 0) {
    if (global) deposit_global<NDIM, SHAPE>(i, j, k, mx, my, mz, wt, q, vx, vy, vz, g, acc);
  }
}

// DPP move of v from `lane - D` within each 16-lane row (row_shr:D); lanes
// with no source get 0 (float) or `fill` (int).
template <int D>
__device__ __forceinline__ float shr_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                0x110 + D, 0xF, 0xF, true));
}
template <int D>
__device__ __forceinline__ int shr_i(int v, int fill) {
  return __builtin_amdgcn_update_dpp(fill, v, 0x110 + D, 0xF, 0xF, false);
}
// The same from `lane + 1` within the row (row_shl:1).
__device__ __forceinline__ int shl1_i(int v, int fill) {
  return __builtin_amdgcn_update_dpp(fill, v, 0x101, 0xF, 0xF, false);
}

// v += v[lane - D] * m for every home sum (lanes with no source add 0),
// within each 16-lane row.
template <int D, int T>
__device__ __forceinline__ void scan_level(float (&acc)[T][4], float m) {
  static_assert(D == 1 || D == 2 || D == 4 || D == 8, "row shift");
  asm volatile("s_nop 1");
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
      if (D == 1)
        asm volatile("v_fmac_f32_dpp %0, %0, %1 row_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
                     : "+v"(acc[t][ch]) : "v"(m));
      else if (D == 2)
        asm volatile("v_fmac_f32_dpp %0, %0, %1 row_shr:2 row_mask:0xf bank_mask:0xf bound_ctrl:1"
                     : "+v"(acc[t][ch]) : "v"(m));
      else if (D == 4)
        asm volatile("v_fmac_f32_dpp %0, %0, %1 row_shr:4 row_mask:0xf bank_mask:0xf bound_ctrl:1"
                     : "+v"(acc[t][ch]) : "v"(m));
      else
        asm volatile("v_fmac_f32_dpp %0, %0, %1 row_shr:8 row_mask:0xf bank_mask:0xf bound_ctrl:1"
                     : "+v"(acc[t][ch]) : "v"(m));
    }
}

// End of a group step: the home sums go to the window.  Consecutive lanes
// hold consecutive particles, so lanes with the same home cell form runs.
// An inclusive segmented scan within each 16-lane row (DPP, with segment-head
// flags, so runs are maximal stretches of equal adjacent keys whatever their
// order, cut at row ends) leaves each run's total in its last lane, which
// alone adds it to the window: a few active lanes per cell in each FP64 LDS
// atomic.  A level adds the neighbour's partial sum times 0 or 1, a DPP move
// and one FMA.  Every lane of the wavefront calls it.
template <int NDIM, int SHAPE>
__device__ __forceinline__ void home_flush(Home<NDIM, SHAPE>& H, const WinLds& wl) {
  constexpr int T = Stencil<NDIM, SHAPE>::T;
  const int r = threadIdx.x & 15;
  const int h = H.key;
  const int prev = shr_i<1>(h, -2), next = shl1_i(h, -2);
  const bool last = r == 15 || next != h;
  // f: a run starts at or after the first lane that v already covers
  int f = (r == 0 || prev != h) ? 1 : 0;
  float m1, m2, m4, m8;  // 1: add the partial sum d lanes back
  m1 = f ? 0.0f : 1.0f;
  f |= shr_i<1>(f, 1);
  m2 = f ? 0.0f : 1.0f;
  f |= shr_i<2>(f, 1);
  m4 = f ? 0.0f : 1.0f;
  f |= shr_i<4>(f, 1);
  m8 = f ? 0.0f : 1.0f;
  // One level for all sums at a time, each v += shr(v) * m as a single FMA
  // with the DPP move on its first operand (the compiler emits a separate
  // move for each).  A level's first read of a sum follows its last write by
  // all the other sums' instructions, except after the deposit's own writes:
  // the s_nop before each level covers the two wait states a DPP read needs
  // after a VALU write of its operand.
  scan_level<1, T>(H.acc, m1);
  scan_level<2, T>(H.acc, m2);
  scan_level<4, T>(H.acc, m4);
  scan_level<8, T>(H.acc, m8);
  if (h >= 0 && last) {
    int s[T];
    stencil_slots<NDIM, SHAPE>(h, wl.wrap[h], s);
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) atomicAdd(wl.acc + s[t] * 4 + ch, (double)H.acc[t][ch]);
  }
  home_clear(H);
}

// Clears the deposit window (every slot of every band, so that the loops
// divide by the compile-time band width only) and fills the wrap bits of the
// cells of columns [0, W) (column 0 = cell c0 - 2).
template <int NDIM>
__device__ void dwin_init(double* win, uint8_t* wrap, int W, int c0, const Geo& g) {
  constexpr int SW = DWin<NDIM>::SW, NB = DWin<NDIM>::NB;
  double2* w2 = reinterpret_cast<double2*>(win);
  for (int s = threadIdx.x; s < NB * SW * 2; s += kBlock) w2[s] = make_double2(0.0, 0.0);
  for (int s = threadIdx.x; s < NB * SW; s += kBlock) {
    const int band = s / SW, col = s - band * SW;
    if (col >= W) continue;
    const int c = (int)window_cell(c0, col, band % 5 - 2, NDIM == 3 ? band / 5 - 2 : 0, g);
    int i, j, k;
    decompose(c, g, i, j, k);
    wrap[s] = (uint8_t)wrap_bits<NDIM>(i, j, g);
  }
}

// Adds columns [0, W) of the block's deposit window (column 0 = cell c0 - 2)
// to the FP64 global accumulators.
template <int NDIM>
__device__ void dwin_flush(const double* win, int W, int c0, const Geo& g,
                           double* __restrict__ acc) {
  constexpr int SW = DWin<NDIM>::SW, NB = DWin<NDIM>::NB;
  for (int s = threadIdx.x; s < NB * SW * 4; s += kBlock) {
    const int band = s / (SW * 4), rest = s - band * (SW * 4);
    const int off = rest >> 2;
    if (off >= W) continue;
    const double v = win[s];
    if (v == 0.0) continue;
    const int ch = rest & 3;
    const int64_t c = window_cell(c0, off, band % 5 - 2, NDIM == 3 ? band / 5 - 2 : 0, g);
    unsafeAtomicAdd(acc + (int64_t)ch * g.ncell + c, v);
  }
}

// ------------------------------------------------------ particle I/O -----

// Four consecutive values at p + i as one 16-byte access (16-byte aligned).
template <typename T>
__device__ __forceinline__ void load4v(const T* __restrict__ p, int64_t i, T v[4]) {
  using V = typename std::conditional<std::is_same<T, int>::value, int4, float4>::type;
  const V u = *reinterpret_cast<const V*>(p + i);
  v[0] = u.x;
  v[1] = u.y;
  v[2] = u.z;
  v[3] = u.w;
}

// The same element by element up to end (zero beyond).
template <typename T>
__device__ __forceinline__ void load4e(const T* __restrict__ p, int64_t i, int64_t end, T v[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = i + q < end ? p[i + q] : T(0);
}

template <typename T>
__device__ __forceinline__ void store4(T* __restrict__ p, int64_t i, int64_t end, bool full,
                                       const T v[4]) {
  if (full) {
    using V = typename std::conditional<std::is_same<T, int>::value, int4, float4>::type;
    V u;
    u.x = v[0];
    u.y = v[1];
    u.z = v[2];
    u.w = v[3];
    *reinterpret_cast<V*>(p + i) = u;
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (i + q < end) p[i + q] = v[q];
  }
}

// One group step's particles of a lane: four consecutive ones.
template <int NDIM>
struct Group {
  int ca[4];
  float px[4], py[4], pz[4], ux[4], uy[4], uz[4], pw[4];
};

// Loads a lane's group at b4 from the particle arrays of A: 16-byte accesses
// when `full`, which must be the same on all lanes of the wavefront (one
// branch for the whole group, so that the compiler keeps the vector loads
// together and in flight at once), else element-wise ones.
template <int NDIM, typename Args>
__device__ __forceinline__ void load_group(const Args& A, int64_t b4, int64_t end, bool full,
                                           bool wq, Group<NDIM>& G) {
  if (full) {
    load4v(A.cell, b4, G.ca);
    load4v(A.ox, b4, G.px);
    load4v(A.oy, b4, G.py);
    if (NDIM == 3) load4v(A.oz, b4, G.pz);
    load4v(A.ux, b4, G.ux);
    load4v(A.uy, b4, G.uy);
    load4v(A.uz, b4, G.uz);
    if (wq) load4v(A.w, b4, G.pw);
  } else {
    load4e(A.cell, b4, end, G.ca);
    load4e(A.ox, b4, end, G.px);
    load4e(A.oy, b4, end, G.py);
    if (NDIM == 3) load4e(A.oz, b4, end, G.pz);
    load4e(A.ux, b4, end, G.ux);
    load4e(A.uy, b4, end, G.uy);
    load4e(A.uz, b4, end, G.uz);
    if (wq) load4e(A.w, b4, end, G.pw);
    // vmcnt(0): these loads are complete here, so that code after the branch
    // need not wait for them (nor for older loads in flight)
    __builtin_amdgcn_s_waitcnt(0x0F70);
  }
}

// The same through the gather map A.perm (16-byte aligned, like the
// destination store): four map entries, then element loads of the source.
template <int NDIM, int PM>
__device__ __forceinline__ void load_group_perm(const PushArgs& A, int64_t b4, int64_t end,
                                                bool full, Group<NDIM>& G) {
  int src[4];
  if (full)
    load4v(A.perm, b4, src);
  else
    load4e(A.perm, b4, end, src);
  // an entry outside [0, n) is read as element 0 and flagged (0 past the
  // end: a valid element, never stored)
  bool bad = false;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    bad |= (uint32_t)src[q] >= (uint32_t)A.nsrc;
    src[q] = (uint32_t)src[q] >= (uint32_t)A.nsrc ? 0 : src[q];
  }
  if (__ballot(bad) != 0) {
    if (bad) raise_flag(A.st, HVPIC_FLAG_BAD_INPUT, &A.st->bad_input);
  }
  if (PM == 1) {
    // one 32-bit byte offset per element shared by all arrays, whose bases
    // stay in scalar registers (no 64-bit address per load)
    auto at = [](const void* base, uint32_t o) {
      return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + o);
    };
    // a lane whose four entries are a run of the source (no mover among
    // them, the common case) takes each array's four values with one
    // 16-byte access at a 4-byte aligned address
    const bool run = src[1] == src[0] + 1 && src[2] == src[0] + 2 && src[3] == src[0] + 3;
    if (run) {
      typedef float F4u __attribute__((ext_vector_type(4), aligned(4)));
      const uint32_t o = (uint32_t)src[0] * 4u;
      auto at4 = [](const void* base, uint32_t o, float v[4]) {
        const F4u u = *reinterpret_cast<const F4u*>(reinterpret_cast<const char*>(base) + o);
        v[0] = u.x;
        v[1] = u.y;
        v[2] = u.z;
        v[3] = u.w;
      };
      float ci[4];
      at4(A.icell, o, ci);
#pragma unroll
      for (int q = 0; q < 4; ++q) G.ca[q] = __float_as_int(ci[q]);
      at4(A.iox, o, G.px);
      at4(A.ioy, o, G.py);
      if (NDIM == 3) at4(A.ioz, o, G.pz);
      at4(A.iux, o, G.ux);
      at4(A.iuy, o, G.uy);
      at4(A.iuz, o, G.uz);
      at4(A.iw, o, G.pw);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t o = (uint32_t)src[q] * 4u;
        G.ca[q] = __float_as_int(at(A.icell, o));
        G.px[q] = at(A.iox, o);
        G.py[q] = at(A.ioy, o);
        if (NDIM == 3) G.pz[q] = at(A.ioz, o);
        G.ux[q] = at(A.iux, o);
        G.uy[q] = at(A.iuy, o);
        G.uz[q] = at(A.iuz, o);
        G.pw[q] = at(A.iw, o);
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t e = src[q];
      G.ca[q] = A.icell[e];
      G.px[q] = A.iox[e];
      G.py[q] = A.ioy[e];
      if (NDIM == 3) G.pz[q] = A.ioz[e];
      G.ux[q] = A.iux[e];
      G.uy[q] = A.iuy[e];
      G.uz[q] = A.iuz[e];
      G.pw[q] = A.iw[e];
    }
  }
  if (!full) __builtin_amdgcn_s_waitcnt(0x0F70);  // as in load_group
}

// Shift s with x - 2s in [-1,1) for |x| < 3: one exact compare each way (x -/+
// 2 is exact there by Sterbenz), branch-free.  Callers send any other value
// down renorm.
__device__ __forceinline__ int near_shift(float x) {
  return (x >= 1.0f ? 1 : 0) - (x < -1.0f ? 1 : 0);
}

// Wrap of a cell index at most one cell outside [0, n).
__device__ __forceinline__ int wrap_near(int t, int n) {
  return t < 0 ? t + n : (t >= n ? t - n : t);
}

// Stand-alone shift (deposit kernel): the near case, else the general path.
__device__ __forceinline__ bool renorm_fast(float& x, int& s) {
  if (fabsf(x) < 3.0f) {
    s = near_shift(x);
    x = fmaf(-2.0f, (float)s, x);
    return true;
  }
  return renorm(x, s);
}

// ------------------------------------------------------------ move counts --
//
// With the store's cell_start given, the push also makes the first pass of
// the neighbour-move sort: for every old cell and each of the 3^ndim move
// directions, the number of its particles that moved that way.  A particle's
// old cell is its cell before the push, which must agree with its place in
// the store (checked).  Counts go to an LDS window over the block's cells
// (home-cell runs as for the deposit, other moves by LDS atomics); cells
// strictly inside the block's range hold no other block's particles and are
// stored plainly, the two end cells are added atomically, so the table must
// be zero beforehand (the sort's scatter leaves it zero).

template <int NDIM>
struct Moves {
  static constexpr int ND = NDIM == 2 ? 9 : 27;
  static constexpr int CENTRE = ND / 2;  // stayed in its cell
};

__device__ __forceinline__ void flag_far(Status* st, uint32_t bit, unsigned long long* counter) {
  raise_flag(st, bit, counter);
  __hip_atomic_store(&st->far_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int NDIM>
__device__ __forceinline__ void moves_window_init(const int32_t* __restrict__ cs, int c0, int span,
                                                  int32_t* s_cs, uint32_t* s_cnt) {
  for (int q = threadIdx.x; q <= span + 1; q += kBlock) s_cs[q] = cs[c0 + q];
  for (int q = threadIdx.x; q < (span + 1) * Moves<NDIM>::ND; q += kBlock) s_cnt[q] = 0;
}

// Each block checks its share of cell_start (a monotone partition of [0, n]);
// the scatter relies on it.  The shares are [f(bid), f(bid+1)) with
// f(b) = floor(b ncell / nb) in FP64 (monotone in b, f(0) = 0, f(nb) = ncell:
// a partition of the cells, without a 64-bit integer division).
__device__ __forceinline__ void check_cell_start(const int32_t* __restrict__ cs, int ncell,
                                                 int64_t n, Status* st, int bid, int nb) {
  const int64_t cb = (int64_t)((double)bid * (double)ncell / (double)nb);
  const int64_t ce = bid + 1 >= nb ? (int64_t)ncell
                                   : (int64_t)((double)(bid + 1) * (double)ncell / (double)nb);
  bool bad = false;
  for (int64_t c = cb + threadIdx.x; c < ce; c += kBlock) {
    const int32_t v0 = cs[c], v1 = cs[c + 1];
    bad |= v0 < 0 || v1 < v0 || (int64_t)v1 > n;
  }
  if (threadIdx.x == 0) {
    if (bid == 0) bad |= cs[0] != 0;
    if (bid == nb - 1) bad |= (int64_t)cs[ncell] != n;
  }
  if (bad) flag_far(st, HVPIC_FLAG_BAD_INPUT, &st->bad_input);
}

// Direction code of the move (i,j,k) -> (ni,nj,nk) (shift si,sj,sk) of
// particle idx of old cell a (window column rel; a is read only outside the
// window), classified as the sort does; -1 (and the sort sent down its
// general path) for a longer move or a particle out of place, and for a lane
// that is not live.  Every lane of the wavefront calls it: the rare cases
// take wavefront-uniform branches.
template <int NDIM, typename Args>
__device__ __forceinline__ int move_direction(const Args& A, int64_t idx, int a, int rel,
                                              bool live, bool inwin, const int32_t* s_cs, int i,
                                              int j, int k, int ni, int nj, int nk, int si,
                                              int sj, int sk) {
  const int rw = inwin ? rel : 0;
  int64_t lo = s_cs[rw], hi = s_cs[rw + 1];
  const bool outwin = live && !inwin;
  if (__ballot(outwin) != 0) {
    // the global table for a particle outside the window (relaxed atomics,
    // which the compiler cannot merge with the LDS reads into one flat read
    // through a select of the two addresses)
    if (outwin) {
      lo = __hip_atomic_load(A.cs + a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      hi = __hip_atomic_load(A.cs + a + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // vmcnt(0) here, so that the common path after the branch need not wait
    // for these (and with them for every older load in flight)
    __builtin_amdgcn_s_waitcnt(0x0F70);
  }
  const bool misplaced = live && (idx < lo || idx >= hi);
  const Geo& g = A.g;
  int di, dj, dk;
  if (g.nx >= 3 && g.ny >= 3 && (NDIM == 2 || g.nz >= 3)) {
    // with three or more cells per axis a shift of at most one cell is
    // exactly the wrapped index difference
    di = si < -1 || si > 1 ? 2 : si;
    dj = sj < -1 || sj > 1 ? 2 : sj;
    dk = sk < -1 || sk > 1 ? 2 : sk;
  } else {
    di = canon_move(ni - i, g.nx);
    dj = canon_move(nj - j, g.ny);
    dk = NDIM == 3 ? canon_move(nk - k, g.nz) : 0;
  }
  const bool far = live && !misplaced && (di == 2 || dj == 2 || dk == 2);
  if (__ballot(misplaced || far) != 0) {
    if (misplaced) flag_far(A.st, HVPIC_FLAG_BAD_INPUT, &A.st->bad_input);
    if (far) flag_far(A.st, HVPIC_FLAG_MOVE_GT1, nullptr);
  }
  return live && !misplaced && !far ? (di + 1) + 3 * (dj + 1) + (NDIM == 3 ? 9 * (dk + 1) : 0)
                                    : -1;
}

// Counts one move (d >= 0) of a particle of old cell a (window column rel; a
// is read only outside the window).  Every lane of the wavefront calls it.
template <int NDIM>
__device__ __forceinline__ void count_move(int d, bool inwin, int rel, int a, int& chome,
                                           uint32_t& nstay, uint32_t* s_cnt,
                                           uint32_t* __restrict__ cnt) {
  constexpr int ND = Moves<NDIM>::ND, CENTRE = Moves<NDIM>::CENTRE;
  const bool local = d >= 0 && inwin;
  if (local && chome < 0) chome = rel;
  const bool stays = local && rel == chome && d == CENTRE;
  nstay += stays ? 1u : 0u;
  const bool to_lds = local && !stays, to_global = d >= 0 && !inwin;
  if (__ballot(to_lds || to_global) != 0) {
    if (to_lds) atomicAdd(&s_cnt[rel * ND + d], 1u);
    if (to_global) atomicAdd(&cnt[(int64_t)a * ND + d], 1u);
  }
}

// End of a group step: home-cell stay counts go to the window, combined
// across a quad of lanes with the same home cell.  Every lane calls it.
template <int NDIM>
__device__ __forceinline__ void count_flush(int& chome, uint32_t& nstay, uint32_t* s_cnt) {
  const int h = chome;
  const bool same = h == dpp_i<0xB1>(h) && h == dpp_i<0x4E>(h) && h == dpp_i<0x1B>(h);
  uint32_t n = nstay;
  if (same) {
    n += (uint32_t)dpp_i<0xB1>((int)n);
    n += (uint32_t)dpp_i<0x4E>((int)n);
  }
  if (h >= 0 && n != 0 && (!same || (threadIdx.x & 3) == 0))
    atomicAdd(&s_cnt[h * Moves<NDIM>::ND + Moves<NDIM>::CENTRE], n);
  chome = -1;
  nstay = 0;
}

template <int NDIM>
__device__ void moves_window_flush(const uint32_t* s_cnt, int c0, int span,
                                   uint32_t* __restrict__ cnt) {
  constexpr int ND = Moves<NDIM>::ND;
  for (int q = threadIdx.x; q < (span + 1) * ND; q += kBlock) {
    const int rel = q / ND;
    const uint32_t v = s_cnt[q];
    uint32_t* dst = cnt + (int64_t)c0 * ND + q;
    if (rel == 0 || rel == span) {
      if (v) atomicAdd(dst, v);
    } else {
      *dst = v;
    }
  }
}

// The move of one lane outside the near case (an offset beyond three
// half-cells of the centre, or a non-finite one): the general shift, the
// status flags, the wrap of any shift, and the mid-point the same way (kept at
// x^n when it cannot be renormalised).  A non-finite position keeps the
// particle where it was.
template <int NDIM, bool DEP>
__device__ void move_general(const PushArgs& A, float x, float y, float z, float nvx, float nvy,
                             float nvz, int i, int j, int k, float& nx_, float& ny_, float& nz_,
                             int& si, int& sj, int& sk, int& ni, int& nj, int& nk, float& xm,
                             float& ym, float& zm, int& mx, int& my, int& mz) {
  const Geo& g = A.g;
  nx_ = fmaf(nvx, A.kx, x);
  ny_ = fmaf(nvy, A.ky, y);
  nz_ = NDIM == 3 ? fmaf(nvz, A.kz, z) : z;
  si = sj = sk = 0;
  bool ok = renorm(nx_, si);
  ok = renorm(ny_, sj) && ok;
  if (NDIM == 3) ok = renorm(nz_, sk) && ok;
  if (!ok) {
    raise_flag(A.st, HVPIC_FLAG_NONFINITE, &A.st->nonfinite);
    si = sj = sk = 0;
    nx_ = x;
    ny_ = y;
    nz_ = z;
  } else if (si > 1 || si < -1 || sj > 1 || sj < -1 || sk > 1 || sk < -1) {
    raise_flag(A.st, HVPIC_FLAG_MOVE_GT1, &A.st->moved_gt1);
  }
  ni = wrapi(i + si, g.nx);
  nj = wrapi(j + sj, g.ny);
  nk = NDIM == 3 ? wrapi(k + sk, g.nz) : 0;
  if (DEP) {
    xm = fmaf(nvx, 0.5f * A.kx, x);
    ym = fmaf(nvy, 0.5f * A.ky, y);
    zm = NDIM == 3 ? fmaf(nvz, 0.5f * A.kz, z) : 0.0f;
    mx = my = mz = 0;
    bool okm = ok && renorm(xm, mx);
    okm = okm && renorm(ym, my);
    if (NDIM == 3) okm = okm && renorm(zm, mz);
    if (!okm) {
      xm = x;
      ym = y;
      zm = z;
      mx = my = mz = 0;
    }
  }
}

// ---------------------------------------------------------------- kernels --

// Fused gather + Boris push + move (+ mid-point deposit when DEP).
// At most 128 VGPRs, so that four wavefronts per SIMD keep enough loads in
// flight (a 3D block's 35.8 KB of LDS allows four blocks per CU as well).
// PM: 0 reads and writes the store in place; 1 and 2 read it through the
// gather map A.perm (1: all byte offsets of the source arrays fit 32 bits).
// The push of one chunk of PPT*kBlock consecutive particles of the store
// (chunk `chunk` of the nb chunks of that store).  slot, a bijection of the
// launch's blocks onto [0, nb) that does not depend on the data, picks the
// block's share of the cell_start check and its diagnostic slot, so that
// the check covers every entry even where a chunk order built from a bad
// cell_start repeats a chunk.
template <int NDIM, int SHAPE, bool DEP, int PM, int PPT>
__device__ __forceinline__ void push_chunk(const PushArgs& A, int chunk, int slot, int nb) {
  constexpr int NF4 = Rec<NDIM, SHAPE>::NF4;
  constexpr int CN = kBlock * PPT;  // particles per chunk
  __shared__ float4 gw[Chunk<NDIM>::WMAX * NF4];
  __shared__ __attribute__((aligned(16))) double win[DEP ? DWin<NDIM>::LEN : 2];
  __shared__ uint8_t s_wrap[DEP ? DWin<NDIM>::NB * DWin<NDIM>::SW : 1];
  __shared__ float s_q[DEP ? kBlock / 64 * Queue<NDIM>::QCAP * Queue<NDIM>::QW : 1];
  __shared__ uint32_t s_cnt[Chunk<NDIM>::WMAX * Moves<NDIM>::ND];
  __shared__ int32_t s_cs[Chunk<NDIM>::WMAX + 1];
  __shared__ int s_c[2];
  const Geo& g = A.g;
  const int64_t base = (int64_t)chunk * CN;
  const int64_t end = min(base + (int64_t)CN, A.n);
  if (threadIdx.x == 0) {
    if (PM != 0) {
      // (entries outside [0, n) are flagged where the particles are loaded)
      const uint32_t e0 = (uint32_t)A.perm[base], e1 = (uint32_t)A.perm[end - 1];
      s_c[0] = A.icell[e0 < (uint32_t)A.nsrc ? e0 : 0];
      s_c[1] = A.icell[e1 < (uint32_t)A.nsrc ? e1 : 0];
    } else {
      s_c[0] = A.cell[base];
      s_c[1] = A.cell[end - 1];
    }
  }
  __syncthreads();
  const bool want_diag = A.diag_part != nullptr;
  const bool wq = DEP || want_diag || PM != 0;  // the weights are needed
  // Wavefront wv owns particles [base + wv*64*PPT, +64*PPT); in each group
  // step lane l takes four consecutive ones, so a step is one coalesced
  // 1 KiB access per array.  The first step's particles are loaded during the
  // set-up below, each later step's right after the previous step's stores.
  const int64_t wb = base + (int64_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * 64 * PPT;
  const int64_t lb = wb + 4 * (threadIdx.x & 63);
  // a step of the wavefront is all in range, or it takes element-wise accesses
  auto step_full = [&](int h) { return A.vec && wb + h * 64 + 256 <= end; };
  Group<NDIM> cur;
  if (PM != 0)
    load_group_perm<NDIM, PM>(A, lb, end, step_full(0), cur);
  else
    load_group<NDIM>(A, lb, end, step_full(0), wq, cur);
  const int c0 = s_c[0], span = s_c[1] - s_c[0];
  int W = 0;
  const bool wok = window_ok<NDIM>(c0, s_c[1], g, W);
  count_path(A.st, wok);
  const bool cnt_on = A.cs != nullptr;  // count the moves for the sort
  if (wok) {
    gwin_fill<NDIM, SHAPE>(reinterpret_cast<float*>(gw), span + 1, c0, g, A.E, A.B);
    if (DEP) dwin_init<NDIM>(win, s_wrap, W, c0, g);
    if (cnt_on) moves_window_init<NDIM>(A.cs, c0, span, s_cs, s_cnt);
  }
  if (cnt_on) check_cell_start(A.cs, g.ncell, A.n, A.st, slot, nb);
  __syncthreads();

  float dK = 0.f, dP0 = 0.f, dP1 = 0.f, dP2 = 0.f;
  const WinLds wl{win, s_wrap};
  Home<NDIM, SHAPE> H;
  home_clear(H);
  Queue<NDIM> Q;
  Q.base = s_q + (DEP ? (threadIdx.x >> 6) * Queue<NDIM>::QCAP * Queue<NDIM>::QW : 0);
  Q.count = 0;
  int chome = -1;      // window column of the lane's home cell for move counts
  uint32_t nstay = 0;  // home-cell particles that stay in their cell
#pragma unroll 1
  for (int h = 0; h < PPT; h += 4) {
    const int64_t b4 = lb + h * 64;
    const bool full = step_full(h);
    int* ca = cur.ca;
    float *px = cur.px, *py = cur.py, *pz = cur.pz, *ux = cur.ux, *uy = cur.uy, *uz = cur.uz;
    const float* pw = cur.pw;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // Every lane runs the common path; a lane past the end or with a bad
      // cell computes on finite stand-in values and has no effect.  Rare
      // cases (outside the windows, far or non-finite moves, flags) take
      // wavefront-uniform branches.
      const int a = ca[q];
      const float x = px[q], y = py[q], z = NDIM == 3 ? pz[q] : 0.f;
      const float vx = ux[q], vy = uy[q], vz = uz[q];
      const bool inrange = b4 + q < end;
      const bool badcell = inrange && (unsigned)a >= (unsigned)g.ncell;
      const bool live = inrange && !badcell;
      const float wgt = wq && live ? pw[q] : 0.f;
      if (__ballot(badcell) != 0) {
        if (badcell) raise_flag(A.st, HVPIC_FLAG_BAD_INPUT, &A.st->bad_input);
      }
      const int rel = a - c0;
      const bool inwin = wok && rel >= 0 && rel <= span;
      int i = 0, j = 0, k = 0;
      float Ep[3] = {0.f, 0.f, 0.f}, Bp[3] = {0.f, 0.f, 0.f};
      if (wok) gather_rec<NDIM, SHAPE>(gw, inwin ? rel : 0, x, y, z, Ep, Bp, i, j, k);
      // outside the windows: the cell index for the global tables, rebuilt
      // from its indices (a value of its own, so that the 64-bit address
      // arithmetic of this rare path does not move the loaded cells into
      // aligned register pairs on the common path)
      int ag = 0;
      const bool outwin = live && !inwin;
      if (__ballot(outwin) != 0) {
        if (outwin) {
          decompose(a, g, i, j, k);
          ag = i + g.nx * (j + g.ny * k);
          gather_eb<NDIM, SHAPE>(A.E, A.B, ag, i, j, k, x, y, z, g, Ep, Bp);
        }
      }
      // Boris: half kick, rotation, half kick.
      const float hh = A.a;
      const float vmx = fmaf(hh, Ep[0], vx), vmy = fmaf(hh, Ep[1], vy), vmz = fmaf(hh, Ep[2], vz);
      const float tx = hh * Bp[0], ty = hh * Bp[1], tz = hh * Bp[2];
      // 2 / (1 + |t|^2) through the hardware reciprocal (within 1 ulp; the
      // operand lies in [1, inf), so no denormals)
      const float f = 2.0f * __builtin_amdgcn_rcpf(1.0f + (tx * tx + ty * ty + tz * tz));
      const float sx = f * tx, sy = f * ty, sz = f * tz;
      const float qx = vmx + (vmy * tz - vmz * ty);
      const float qy = vmy + (vmz * tx - vmx * tz);
      const float qz = vmz + (vmx * ty - vmy * tx);
      const float nvx = fmaf(hh, Ep[0], vmx + (qy * sz - qz * sy));
      const float nvy = fmaf(hh, Ep[1], vmy + (qz * sx - qx * sz));
      const float nvz = fmaf(hh, Ep[2], vmz + (qx * sy - qy * sx));
      if (want_diag) {
        dK = fmaf(wgt, vx * nvx + vy * nvy + vz * nvz, dK);
        dP0 = fmaf(wgt, vx + nvx, dP0);
        dP1 = fmaf(wgt, vy + nvy, dP1);
        dP2 = fmaf(wgt, vz + nvz, dP2);
      }
      // Move: x^{n+1} = x^n + v^{n+1/2} dt, and for the deposit the mid-point
      // x^{n+1/2} = x^n + (dt/2) v^{n+1/2}, with renormalised offsets.
      float nx_ = fmaf(nvx, A.kx, x), ny_ = fmaf(nvy, A.ky, y);
      float nz_ = NDIM == 3 ? fmaf(nvz, A.kz, z) : z;
      float xm = 0.f, ym = 0.f, zm = 0.f;
      if (DEP) {
        xm = fmaf(nvx, 0.5f * A.kx, x);
        ym = fmaf(nvy, 0.5f * A.ky, y);
        zm = NDIM == 3 ? fmaf(nvz, 0.5f * A.kz, z) : 0.0f;
      }
      bool near = fabsf(nx_) < 3.0f && fabsf(ny_) < 3.0f && (NDIM == 2 || fabsf(nz_) < 3.0f);
      if (DEP)
        near = near && fabsf(xm) < 3.0f && fabsf(ym) < 3.0f && (NDIM == 2 || fabsf(zm) < 3.0f);
      int si = near_shift(nx_), sj = near_shift(ny_), sk = NDIM == 3 ? near_shift(nz_) : 0;
      nx_ = fmaf(-2.0f, (float)si, nx_);
      ny_ = fmaf(-2.0f, (float)sj, ny_);
      if (NDIM == 3) nz_ = fmaf(-2.0f, (float)sk, nz_);
      int mx = 0, my = 0, mz = 0;
      if (DEP) {
        mx = near_shift(xm);
        my = near_shift(ym);
        xm = fmaf(-2.0f, (float)mx, xm);
        ym = fmaf(-2.0f, (float)my, ym);
        if (NDIM == 3) {
          mz = near_shift(zm);
          zm = fmaf(-2.0f, (float)mz, zm);
        }
      }
      int ni = wrap_near(i + si, g.nx), nj = wrap_near(j + sj, g.ny);
      int nk = NDIM == 3 ? wrap_near(k + sk, g.nz) : 0;
      const bool general = live && !near;
      if (__ballot(general) != 0) {
        if (general)
          move_general<NDIM, DEP>(A, x, y, z, nvx, nvy, nvz, i, j, k, nx_, ny_, nz_, si, sj, sk,
                                  ni, nj, nk, xm, ym, zm, mx, my, mz);
      }
      // a lane that is not live keeps its values
      ca[q] = live ? ni + g.nx * (nj + g.ny * nk) : a;
      px[q] = live ? nx_ : x;
      py[q] = live ? ny_ : y;
      if (NDIM == 3) pz[q] = live ? nz_ : z;
      ux[q] = live ? nvx : vx;
      uy[q] = live ? nvy : vy;
      uz[q] = live ? nvz : vz;
      if (cnt_on) {
        const int d = move_direction<NDIM>(A, b4 + q, ag, rel, live, inwin, s_cs, i, j, k, ni, nj,
                                           nk, si, sj, sk);
        count_move<NDIM>(d, inwin, rel, ag, chome, nstay, s_cnt, A.cnt);
      }
      if (DEP)
        deposit_particle<NDIM, SHAPE>(H, Q, wl, live, inwin, rel, i, j, k, mx, my, mz, xm, ym,
                                      zm, A.qV * wgt, nvx, nvy, nvz, g, A.acc);
    }
    store4(A.cell, b4, end, full, ca);
    store4(A.ox, b4, end, full, px);
    store4(A.oy, b4, end, full, py);
    if (NDIM == 3) store4(A.oz, b4, end, full, pz);
    store4(A.ux, b4, end, full, ux);
    store4(A.uy, b4, end, full, uy);
    store4(A.uz, b4, end, full, uz);
    if (PM != 0) store4(A.wo, b4, end, full, pw);
    // the next step's particles arrive during the flushes below
    if (h + 4 < PPT) {
      if (PM != 0)
        load_group_perm<NDIM, PM>(A, b4 + 256, end, step_full(h + 4), cur);
      else
        load_group<NDIM>(A, b4 + 256, end, step_full(h + 4), wq, cur);
    }
    if (DEP) home_flush(H, wl);
    if (cnt_on) count_flush<NDIM>(chome, nstay, s_cnt);
  }
  if (DEP) queue_drain<NDIM, SHAPE>(Q, wl);
  if (want_diag) {
    const double hm = 0.5 * A.ms;
    double v[4] = {hm * dK, hm * dP0, hm * dP1, hm * dP2};
    block_partial<4>(v, A.diag_part, slot);
  }
  if (wok && (DEP || cnt_on)) {
    __syncthreads();
    if (DEP) dwin_flush<NDIM>(win, W, c0, g, A.acc);
    if (cnt_on) moves_window_flush<NDIM>(s_cnt, c0, span, A.cnt);
  }
}

template <int NDIM, int SHAPE, bool DEP, int PM>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
void k_gather_push(PushArgs A) {
  const int slot = xcd_chunk(blockIdx.x, gridDim.x);
  int chunk = slot;
  if (A.order) {
    const int o = A.order[slot];
    if ((unsigned)o < gridDim.x) chunk = o;
  }
  push_chunk<NDIM, SHAPE, DEP, PM, Chunk<NDIM>::PPT>(A, chunk, slot, gridDim.x);
}

// The order in which the 3D push takes its chunks.  The store is sorted by
// cell with x fastest, so a chunk lies in one grid row (j, k) of cells or
// straddles two.  In store order, an ion that moved in z in the last step
// is read from a plane (nx ny cells) away, long after its cache lines left
// the L2, while a y-neighbour row is only nx cells away.  Here the rows are
// visited in tiles of kOrderTj rows along y, plane after plane within a
// tile, so that both neighbours of a row are visited within kOrderTj rows
// of it (all but the rows at a tile's edge in y).  A chunk goes with the
// row of its first ion; the chunks of a row keep their order.  With
// F(r) = ceil(cs[r nx] / 1024), the first chunk that starts in row r, and
// K(r) = F(r+1) - F(r) the chunks that start there, position p of the
// order holds the chunk F(r) + p - P(t) for the row r at rank t, P the
// exclusive prefix sum of K over the ranks.  Three passes: per rank F and
// K, the scan of K, then per rank its entries.  Rows <= 65536.  This is a
// permutation of the nchunks chunks when cell_start does not decrease from
// row start to row start, starts at 0 and ends at n; otherwise (the push
// flags such a cell_start) the order is the store order, so that every
// chunk is still pushed once.
constexpr int kOrderTj = 16;
constexpr int kOrderPer = 16;  // ranks per thread per pass of the scan

// Workspace of the order: the order itself, then F, K, P per rank and the
// decision word.
struct OrderWs {
  int32_t *order, *F, *K, *P, *D;
};

// F and K of rank t's row; K = -1 marks a row start below the previous one.
__global__ void k_order_rows(const int32_t* __restrict__ cs, int nx, int ny, int nz,
                             int nchunks, OrderWs W) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ny * nz) return;
  const int tile = kOrderTj * nz;  // ranks per full tile
  const int jt = t / tile, local = t - jt * tile;
  const int T = min(kOrderTj, ny - jt * kOrderTj);  // rows of this tile
  const int k = local / T, j = jt * kOrderTj + (local - (local / T) * T);
  const int64_t r = (int64_t)j + (int64_t)ny * k;
  const int64_t a = cs[r * nx], b = cs[(r + 1) * nx];
  const int64_t fa = min<int64_t>(max<int64_t>((a + kChunk3 - 1) / kChunk3, 0), nchunks);
  const int64_t fb = min<int64_t>(max<int64_t>((b + kChunk3 - 1) / kChunk3, 0), nchunks);
  W.F[t] = (int)fa;
  W.K[t] = b < a ? -1 : (int)max<int64_t>(fb - fa, 0);
}

// One block: P = exclusive scan of K over the ranks, and the decision
// D = 1 (store order) for a bad cell_start, else 0.
__global__ __launch_bounds__(1024) void k_order_scan(const int32_t* __restrict__ cs, int nx,
                                                     int R, int64_t n, OrderWs W) {
  __shared__ int s_w[16];
  __shared__ int s_carry;
  bool bad = threadIdx.x == 0 && (cs[0] != 0 || (int64_t)cs[(int64_t)R * nx] != n);
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int t0 = 0; t0 < R; t0 += 1024 * kOrderPer) {
    int v[kOrderPer];
#pragma unroll
    for (int q = 0; q < kOrderPer; ++q) {
      const int t = t0 + q * 1024 + (int)threadIdx.x;
      v[q] = t < R ? W.K[t] : 0;
    }
#pragma unroll
    for (int q = 0; q < kOrderPer; ++q) {
      const int t = t0 + q * 1024 + (int)threadIdx.x;
      bad |= v[q] < 0;
      const int own = max(v[q], 0);
      int x = own;
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
      }
      if (lane == 63) s_w[wid] = x;
      __syncthreads();
      int before = s_carry, total = 0;
      for (int w = 0; w < 16; ++w) {
        if (w < wid) before += s_w[w];
        total += s_w[w];
      }
      if (t < R) W.P[t] = before + x - own;
      __syncthreads();
      if (threadIdx.x == 0) s_carry += total;
      __syncthreads();
    }
  }
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) W.D[0] = bad ? 1 : 0;
}

// Per rank its chunks at their positions, or (D = 1) the store order.
__global__ void k_order_write(int R, int nchunks, OrderWs W) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (W.D[0] != 0) {
    if (i < nchunks) W.order[i] = i;
    return;
  }
  if (i >= R) return;
  const int k = W.K[i], f = W.F[i], p = W.P[i];
  for (int m = 0; m < k; ++m)
    if (p + m < nchunks) W.order[p + m] = f + m;
}

// Stand-alone deposit at x - half_dt_back v (no push); same lane runs.
template <int NDIM, int SHAPE>
__global__ __launch_bounds__(kBlock) void k_deposit(DepArgs A) {
  constexpr int PPT = Chunk<NDIM>::PPT;
  __shared__ __attribute__((aligned(16))) double win[DWin<NDIM>::LEN];
  __shared__ uint8_t s_wrap[DWin<NDIM>::NB * DWin<NDIM>::SW];
  __shared__ float s_q[kBlock / 64 * Queue<NDIM>::QCAP * Queue<NDIM>::QW];
  __shared__ int s_c[2];
  const Geo& g = A.g;
  const int64_t base = (int64_t)xcd_chunk(blockIdx.x, gridDim.x) * Chunk<NDIM>::N;
  const int64_t end = min(base + (int64_t)Chunk<NDIM>::N, A.n);
  if (threadIdx.x == 0) {
    s_c[0] = A.cell[base];
    s_c[1] = A.cell[end - 1];
  }
  __syncthreads();
  const int c0 = s_c[0], span = s_c[1] - s_c[0];
  int W = 0;
  const bool wok = window_ok<NDIM>(c0, s_c[1], g, W);
  count_path(A.st, wok);
  if (wok) dwin_init<NDIM>(win, s_wrap, W, c0, g);
  __syncthreads();
  const WinLds wl{win, s_wrap};
  Home<NDIM, SHAPE> H;
  home_clear(H);
  Queue<NDIM> Q;
  Q.base = s_q + (threadIdx.x >> 6) * Queue<NDIM>::QCAP * Queue<NDIM>::QW;
  Q.count = 0;
  const int64_t wb = base + (int64_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * 64 * PPT;
  const int64_t lb = wb + 4 * (threadIdx.x & 63);
#pragma unroll 1
  for (int h = 0; h < PPT; h += 4) {
    const int64_t b4 = lb + h * 64;
    // the same on all lanes of the wavefront (see load_group)
    const bool full = A.vec && wb + h * 64 + 256 <= end;
    Group<NDIM> G;
    load_group<NDIM>(A, b4, end, full, true, G);
    const int* ca = G.ca;
    const float *px = G.px, *py = G.py, *pz = G.pz, *ux = G.ux, *uy = G.uy, *uz = G.uz;
    const float* pw = G.pw;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int a = ca[q];
      bool live = b4 + q < end;
      if (live && (unsigned)a >= (unsigned)g.ncell) {
        raise_flag(A.st, HVPIC_FLAG_BAD_INPUT, &A.st->bad_input);
        live = false;
      }
      if (!live) a = 0;
      int i = 0, j = 0, k = 0, mx = 0, my = 0, mz = 0;
      float x = px[q], y = py[q], z = NDIM == 3 ? pz[q] : 0.f;
      if (live) {
        decompose(a, g, i, j, k);
        float xm = fmaf(ux[q], A.bx, x), ym = fmaf(uy[q], A.by, y);
        float zm = NDIM == 3 ? fmaf(uz[q], A.bz, z) : 0.f;
        if (renorm_fast(xm, mx) && renorm_fast(ym, my) && (NDIM == 2 || renorm_fast(zm, mz))) {
          x = xm;
          y = ym;
          z = zm;
        } else {
          mx = my = mz = 0;
        }
      }
      const int rel = a - c0;
      const bool inwin = wok && rel >= 0 && rel <= span;
      deposit_particle<NDIM, SHAPE>(H, Q, wl, live, inwin, rel, i, j, k, mx, my, mz, x, y, z,
                                    A.qV * pw[q], ux[q], uy[q], uz[q], g, A.acc);
    }
    home_flush(H, wl);
  }
  queue_drain<NDIM, SHAPE>(Q, wl);
  if (wok) {
    __syncthreads();
    dwin_flush<NDIM>(win, W, c0, g, A.acc);
  }
}

__global__ void k_zero(float* __restrict__ a, int64_t na, float* __restrict__ b, int64_t nb) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < na + nb; i += stride) {
    if (i < na)
      a[i] = 0.0f;
    else
      b[i - na] = 0.0f;
  }
}

// FP64 moment accumulators -> FP32 outputs; leaves the accumulators at zero
// for the next deposit.  Blocks of 1024 threads, so that block 0 sums the
// push's per-block diagnostic partials in one round of loads.
constexpr int kMomBlock = 1024;
struct MomArgs {
  double* acc;
  int ncell;
  float* n;
  float* J;
  const double* part;
  int nparts;
  double* diag_out;
};

// Block bid of nb (blocks of kMomBlock threads) of the moment output.
__device__ __forceinline__ void moments_out_body(const MomArgs& M, int bid, int nb) {
  // block 0 also finishes the push diagnostics when asked (saves a launch)
  if (M.diag_out != nullptr && bid == 0) {
    double r[4];
    sum_partials<4>(M.part, M.nparts, r);
    if (threadIdx.x == 0)
      for (int k = 0; k < 4; ++k) M.diag_out[k] = r[k];
  }
  const int64_t stride = (int64_t)nb * kMomBlock;
  for (int64_t i = (int64_t)bid * kMomBlock + threadIdx.x; i < 4ll * M.ncell; i += stride) {
    const float v = (float)M.acc[i];
    M.acc[i] = 0.0;
    if (i < M.ncell)
      M.n[i] = v;
    else
      M.J[i - M.ncell] = v;
  }
}

__global__ __launch_bounds__(kMomBlock) void k_moments_out(MomArgs M) {
  moments_out_body(M, blockIdx.x, gridDim.x);
}

__global__ void k_write_zero_diag(double* out, int nv) {
  if (threadIdx.x < nv) out[threadIdx.x] = 0.0;
}

// One block of 1024 threads: up to 8192 partials in a single round of loads.
__global__ __launch_bounds__(1024) void k_push_diag_final(const double* part, int nblocks,
                                                          double* out) {
  double r[4];
  sum_partials<4>(part, nblocks, r);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) out[k] = r[k];
}

bool particles_aligned16(const hvpic_particles* p) {
  const void* ptrs[] = {p->cell, p->ox, p->oy, p->oz, p->ux, p->uy, p->uz, p->w};
  for (const void* q : ptrs)
    if (((uintptr_t)q & 15) != 0) return false;
  return true;
}

Geo make_geo(const hvpic_ctx* c) {
  Geo g;
  g.nx = c->p.nx;
  g.ny = c->p.ny;
  g.nz = c->p.nz;
  g.ncell = c->ncell;
  g.nxny = c->p.nx * c->p.ny;
  g.fnx = c->fnx;
  g.fny = c->fny;
  return g;
}

template <int NDIM, int SHAPE, int PM>
void push_dispatch_pm(bool dep, dim3 grid, hipStream_t s, const PushArgs& A) {
  if (dep)
    hipLaunchKernelGGL((k_gather_push<NDIM, SHAPE, true, PM>), grid, dim3(kBlock), 0, s, A);
  else
    hipLaunchKernelGGL((k_gather_push<NDIM, SHAPE, false, PM>), grid, dim3(kBlock), 0, s, A);
}

template <int NDIM, int SHAPE>
void push_dispatch(bool dep, dim3 grid, hipStream_t s, const PushArgs& A) {
  if (!A.perm)
    push_dispatch_pm<NDIM, SHAPE, 0>(dep, grid, s, A);
  else if (A.off32)
    push_dispatch_pm<NDIM, SHAPE, 1>(dep, grid, s, A);
  else
    push_dispatch_pm<NDIM, SHAPE, 2>(dep, grid, s, A);
}

int zero2(hvpic_ctx* c, float* a, int64_t na, float* b, int64_t nb) {
  const int64_t total = na + nb;
  if (total <= 0) return HVPIC_OK;
  const int blocks = (int)std::min<int64_t>(ceil_div(total, kBlock), 4096);
  hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(kBlock), 0, c->stream, a, na, b, nb);
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

}  // namespace

int launch_zero(hvpic_ctx* c, float* p, int64_t count) { return zero2(c, p, count, nullptr, 0); }

void zero_counts(hvpic_ctx* c) {
  const int64_t m = (int64_t)c->ncell * (c->p.ndim == 2 ? 9 : 27);
  zero2(c, reinterpret_cast<float*>(c->sort_cnt), m, nullptr, 0);
  c->cnt_clean = true;
}

// FP64 accumulators -> n, J; with diag_out also the push diagnostics from
// nparts per-block partials.
int moment_blocks(const hvpic_ctx* c) {
  return (int)std::min<int64_t>(ceil_div(4ll * c->ncell, kMomBlock), 512);
}

MomArgs mom_args(hvpic_ctx* c, float* n, float* J, int nparts, double* diag_out) {
  return MomArgs{c->mom_acc, c->ncell, n, J, (const double*)c->push_part, nparts, diag_out};
}

void moments_out(hvpic_ctx* c, float* n, float* J, int nparts = 0, double* diag_out = nullptr) {
  hipLaunchKernelGGL(k_moments_out, dim3(moment_blocks(c)), dim3(kMomBlock), 0, c->stream,
                     mom_args(c, n, J, nparts, diag_out));
}

namespace {

// The arguments of the push of store `in` read through `perm` (null: in
// place) into store `p`.
PushArgs push_args(hvpic_ctx* c, const hvpic_particles* in, const int32_t* perm,
                   hvpic_particles* p, const int32_t* cell_start, const float* E,
                   const float* B, double* diag_out) {
  PushArgs A;
  A.n = p->n;
  A.cell = p->cell;
  A.ox = p->ox;
  A.oy = p->oy;
  A.oz = p->oz;
  A.ux = p->ux;
  A.uy = p->uy;
  A.uz = p->uz;
  A.w = p->w;
  A.E = E;
  A.B = B;
  A.acc = c->mom_acc;
  A.g = make_geo(c);
  A.a = c->a;
  A.kx = c->kx;
  A.ky = c->ky;
  A.kz = c->kz;
  A.qV = c->qV;
  A.ms = c->p.ms;
  A.diag_part = diag_out ? c->push_part : nullptr;
  A.st = c->status;
  A.vec = particles_aligned16(p) && ((uintptr_t)perm & 15) == 0;
  A.off32 = in->n < (int64_t(1) << 30);
  A.cs = cell_start;
  A.cnt = c->sort_cnt;
  A.perm = perm;
  A.nsrc = in->n;
  A.icell = in->cell;
  A.iox = in->ox;
  A.ioy = in->oy;
  A.ioz = in->oz;
  A.iux = in->ux;
  A.iuy = in->uy;
  A.iuz = in->uz;
  A.iw = in->w;
  A.wo = p->w;
  A.order = nullptr;
  return A;
}

// The push of store `in` read through `perm` (null: in place, in == out) into
// store `out`.
int launch_push(hvpic_ctx* c, const hvpic_particles* in, const int32_t* perm,
                hvpic_particles* p, const int32_t* cell_start, const float* E, const float* B,
                float* n_mid, float* J_mid, double* diag_out) {
  const bool dep = n_mid != nullptr && J_mid != nullptr;
  c->cnt_ready = false;
  if (p->n == 0) {
    if (diag_out) hipLaunchKernelGGL(k_write_zero_diag, dim3(1), dim3(64), 0, c->stream, diag_out, 4);
    if (dep) moments_out(c, n_mid, J_mid);
    return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
  }
  PushArgs A = push_args(c, in, perm, p, cell_start, E, B, diag_out);
  if (cell_start != nullptr && !c->cnt_clean) zero_counts(c);
  const bool qs = c->p.shape == HVPIC_SHAPE_QS;
  int nblocks = 0;
  if (c->p.ndim == 3 && cell_start != nullptr && c->chunk_order &&
      (int64_t)c->p.ny * c->p.nz <= 65536) {
    // the chunk order (kernels of their own, outside the push's timing)
    const int R = c->p.ny * c->p.nz;
    const int nch = (int)ceil_div(p->n, Chunk<3>::N);
    OrderWs W;
    W.order = c->chunk_order;
    W.F = W.order + ceil_div(std::max<int64_t>(c->p.np_capacity, 1), kChunk3) + 1;
    W.K = W.F + R;
    W.P = W.K + R;
    W.D = W.P + R;
    hipLaunchKernelGGL(k_order_rows, dim3((unsigned)ceil_div(R, 256)), dim3(256), 0, c->stream,
                       cell_start, c->p.nx, c->p.ny, c->p.nz, nch, W);
    hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(1024), 0, c->stream, cell_start, c->p.nx, R,
                       p->n, W);
    hipLaunchKernelGGL(k_order_write, dim3((unsigned)ceil_div(std::max(R, nch), 256)), dim3(256),
                       0, c->stream, R, nch, W);
    A.order = W.order;
  }
  timing_begin(c, HVPIC_KERNEL_GATHER_PUSH);
  if (c->p.ndim == 2) {
    nblocks = (int)ceil_div(p->n, Chunk<2>::N);
    if (qs) push_dispatch<2, HVPIC_SHAPE_QS>(dep, dim3(nblocks), c->stream, A);
    else push_dispatch<2, HVPIC_SHAPE_NGP>(dep, dim3(nblocks), c->stream, A);
  } else {
    nblocks = (int)ceil_div(p->n, Chunk<3>::N);
    if (qs) push_dispatch<3, HVPIC_SHAPE_QS>(dep, dim3(nblocks), c->stream, A);
    else push_dispatch<3, HVPIC_SHAPE_NGP>(dep, dim3(nblocks), c->stream, A);
  }
  timing_end(c, HVPIC_KERNEL_GATHER_PUSH);
  if (cell_start != nullptr) {
    c->cnt_clean = false;
    c->cnt_ready = true;
    c->cnt_cell = p->cell;
    c->cnt_cs = cell_start;
    c->cnt_n = p->n;
  }
  if (dep)
    moments_out(c, n_mid, J_mid, nblocks, diag_out);
  else if (diag_out)
    hipLaunchKernelGGL(k_push_diag_final, dim3(1), dim3(1024), 0, c->stream,
                       (const double*)c->push_part, nblocks, diag_out);
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

}  // namespace


int launch_gather_push(hvpic_ctx* c, hvpic_particles* p, const int32_t* cell_start,
                       const float* E, const float* B, float* n_mid, float* J_mid,
                       double* diag_out) {
  return launch_push(c, p, nullptr, p, cell_start, E, B, n_mid, J_mid, diag_out);
}

int launch_gather_push_perm(hvpic_ctx* c, const hvpic_particles* in, const int32_t* perm,
                            hvpic_particles* out, const int32_t* cell_start, const float* E,
                            const float* B, float* n_mid, float* J_mid, double* diag_out) {
  out->n = in->n;
  return launch_push(c, in, perm, out, cell_start, E, B, n_mid, J_mid, diag_out);
}

int launch_gather_push_select(hvpic_ctx* c, const hvpic_particles* in, int64_t n_map,
                              const int32_t* perm, hvpic_particles* out,
                              const int32_t* cell_start, const float* E, const float* B,
                              float* n_mid, float* J_mid, double* diag_out) {
  out->n = n_map;
  return launch_push(c, in, perm, out, cell_start, E, B, n_mid, J_mid, diag_out);
}

int launch_deposit(hvpic_ctx* c, const hvpic_particles* p, const int32_t* cell_start,
                   float half_dt_back, float* n, float* J) {
  (void)cell_start;
  if (p->n == 0) {
    moments_out(c, n, J);
    return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
  }
  DepArgs A;
  A.n = p->n;
  A.cell = p->cell;
  A.ox = p->ox;
  A.oy = p->oy;
  A.oz = p->oz;
  A.ux = p->ux;
  A.uy = p->uy;
  A.uz = p->uz;
  A.w = p->w;
  A.acc = c->mom_acc;
  A.g = make_geo(c);
  // x - half_dt_back v in half-cell units: offset change -2 half_dt_back v / h.
  A.bx = (float)(-2.0 * (double)half_dt_back / c->p.dx);
  A.by = (float)(-2.0 * (double)half_dt_back / c->p.dy);
  A.bz = (float)(-2.0 * (double)half_dt_back / c->p.dz);
  A.qV = c->qV;
  A.st = c->status;
  A.vec = particles_aligned16(p);
  const bool qs = c->p.shape == HVPIC_SHAPE_QS;
  timing_begin(c, HVPIC_KERNEL_DEPOSIT);
  if (c->p.ndim == 2) {
    const dim3 grid((unsigned)ceil_div(p->n, Chunk<2>::N));
    if (qs) hipLaunchKernelGGL((k_deposit<2, HVPIC_SHAPE_QS>), grid, dim3(kBlock), 0, c->stream, A);
    else hipLaunchKernelGGL((k_deposit<2, HVPIC_SHAPE_NGP>), grid, dim3(kBlock), 0, c->stream, A);
  } else {
    const dim3 grid((unsigned)ceil_div(p->n, Chunk<3>::N));
    if (qs) hipLaunchKernelGGL((k_deposit<3, HVPIC_SHAPE_QS>), grid, dim3(kBlock), 0, c->stream, A);
    else hipLaunchKernelGGL((k_deposit<3, HVPIC_SHAPE_NGP>), grid, dim3(kBlock), 0, c->stream, A);
  }
  timing_end(c, HVPIC_KERNEL_DEPOSIT);
  moments_out(c, n, J);
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

// ------------------------------------------------------------ ensembles --
// Batched forms of the push (gather-map sequence, fused deposit, move counts,
// diagnostics) and of the moment output for an ensemble of independent 2D
// runs: one persistent launch covers the chunks of every run, each work item
// taking its run's arguments from a table in device memory.

namespace {

template <int SHAPE, int PPT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
void k_gather_push_batch(const PushArgs* __restrict__ tab, const Item* __restrict__ items,
                         int nitems) {
  for_items(nitems, [&](int it) {
    const Item item = items[it];
    const PushArgs A = tab[item.run];
    push_chunk<2, SHAPE, true, 1, PPT>(A, item.idx, item.idx, item.nb);
    __syncthreads();  // the next item reuses the LDS
  });
}

__global__ __launch_bounds__(kMomBlock) void k_moments_out_batch(const MomArgs* __restrict__ tab,
                                                                 const Item* __restrict__ items,
                                                                 int nitems) {
  for_items(nitems, [&](int it) {
    const Item item = items[it];
    const MomArgs M = tab[item.run];
    moments_out_body(M, item.idx, item.nb);
    __syncthreads();
  });
}

template <int SHAPE>
void push_batch_ppt(hipStream_t s, int ppt, const PushArgs* tab, const Item* items, int nitems,
                    int grid) {
  if (ppt == 4)
    hipLaunchKernelGGL((k_gather_push_batch<SHAPE, 4>), dim3(grid), dim3(kBlock), 0, s, tab, items,
                       nitems);
  else if (ppt == 8)
    hipLaunchKernelGGL((k_gather_push_batch<SHAPE, 8>), dim3(grid), dim3(kBlock), 0, s, tab, items,
                       nitems);
  else
    hipLaunchKernelGGL((k_gather_push_batch<SHAPE, 12>), dim3(grid), dim3(kBlock), 0, s, tab,
                       items, nitems);
}

}  // namespace

size_t ens_push_record(hvpic_ctx* c, const hvpic_particles* in, const int32_t* perm,
                       hvpic_particles* out, const int32_t* cs, const float* E, const float* B,
                       bool diag, void* dst) {
  if (dst) {
    const PushArgs A = push_args(c, in, perm, out, cs, E, B, diag ? c->push_part : nullptr);
    memcpy(dst, &A, sizeof(A));
  }
  return sizeof(PushArgs);
}

size_t ens_moments_record(hvpic_ctx* c, float* n, float* J, int nparts, double* diag_out,
                          void* dst) {
  if (dst) {
    const MomArgs M = mom_args(c, n, J, nparts, diag_out);
    memcpy(dst, &M, sizeof(M));
  }
  return sizeof(MomArgs);
}

int ens_moment_blocks(const hvpic_ctx* c) { return moment_blocks(c); }

int ens_launch_push(hipStream_t s, int shape, int ppt, const void* tab, const Item* items,
                    int nitems, int grid) {
  if (nitems == 0) return HVPIC_OK;
  const PushArgs* t = static_cast<const PushArgs*>(tab);
  if (shape == HVPIC_SHAPE_QS)
    push_batch_ppt<HVPIC_SHAPE_QS>(s, ppt, t, items, nitems, grid);
  else
    push_batch_ppt<HVPIC_SHAPE_NGP>(s, ppt, t, items, nitems, grid);
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

int ens_launch_moments(hipStream_t s, const void* tab, const Item* items, int nitems, int grid) {
  if (nitems == 0) return HVPIC_OK;
  hipLaunchKernelGGL(k_moments_out_batch, dim3(grid), dim3(kMomBlock), 0, s,
                     static_cast<const MomArgs*>(tab), items, nitems);
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

}  // namespace hvpic

// ------------------------------------------------- allocation-free deposit --
//
// hvpic_deposit_noalloc runs the same deposit kernels as hvpic_deposit with
// its scratch (the status word and the FP64 moment accumulators) in a
// file-scope device array instead of a context's workspace.  Each GPU the
// library runs on holds its own copy of the array until the process ends;
// host code reaches it only through the device address that
// hipGetSymbolAddress returns for the current device.

namespace hvpic {
namespace {

constexpr int64_t kNoAllocStatusBytes = 256;
constexpr int64_t kNoAllocBytes =
    kNoAllocStatusBytes + (int64_t)sizeof(double) * 4 * HVPIC_NOALLOC_MAX_CELLS;
static_assert(sizeof(Status) <= kNoAllocStatusBytes, "status block fits its slot");

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device

// The device address of this device's scratch array (looked up once).
int scratch_ptr(char** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return HVPIC_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return HVPIC_EHIP;
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return HVPIC_OK;
}

// Clears the status word and the first nacc accumulators.
__global__ void k_noalloc_clear(Status* st, double* acc, int64_t nacc) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nacc; i += stride)
    acc[i] = 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *st = Status{};
}

}  // namespace
}  // namespace hvpic

extern "C" int hvpic_deposit_noalloc(const hvpic_params* params, void* hip_stream,
                                     const hvpic_particles* p, float half_dt_back, float* n,
                                     float* J) {
  using namespace hvpic;
  if (!params_valid(params) || !p || !n || !J || !std::isfinite(half_dt_back)) return HVPIC_EINVAL;
  if (p->n < 0 || p->n >= (1ll << 31) - 1) return HVPIC_EINVAL;
  if (p->n > 0 && (!p->cell || !p->ox || !p->oy || !p->ux || !p->uy || !p->uz || !p->w ||
                   (params->ndim == 3 && !p->oz)))
    return HVPIC_EINVAL;
  const int64_t ncell = (int64_t)params->nx * params->ny * params->nz;
  if (ncell > HVPIC_NOALLOC_MAX_CELLS) return HVPIC_ENOMEM;
  char* base = nullptr;
  const int rc = scratch_ptr(&base);
  if (rc != HVPIC_OK) return rc;
  // A context on the stack carries what the launch wrappers read; its
  // workspace pointers are this device's scratch array.
  hvpic_ctx c;
  memset(&c, 0, sizeof(c));
  c.p = *params;
  c.stream = (hipStream_t)hip_stream;
  c.ncell = (int32_t)ncell;
  c.magic = kMagic;
  c.qV = (float)(params->qs / (params->dx * params->dy * params->dz));
  c.fnx = make_fastdiv((uint32_t)params->nx);
  c.fny = make_fastdiv((uint32_t)params->ny);
  c.status = reinterpret_cast<Status*>(base);
  c.mom_acc = reinterpret_cast<double*>(base + kNoAllocStatusBytes);
  hipLaunchKernelGGL(k_noalloc_clear, dim3((unsigned)std::min<int64_t>(ceil_div(4 * ncell, kBlock), 2048)),
                     dim3(kBlock), 0, c.stream, c.status, c.mom_acc, 4 * ncell);
  if (hipGetLastError() != hipSuccess) return HVPIC_EHIP;
  return launch_deposit(&c, p, nullptr, half_dt_back, n, J);
}

