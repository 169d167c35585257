// Particle kernels of libhvpic.so for gfx950: gather + Boris push + move
// (optionally with the moment deposit fused in) and the stand-alone deposit.
//
// Method (arXiv 2305.05600):
//   gather   App. B eq:quadFI/eq:quadF (QS) -- evaluated in the equivalent
//            weight form F(x_p) = sum_c W_c(dx,dy,dz) F_c with the eq:quad
//            weights, which the paper's consistency (no self-force) statement
//            makes identical to the interpolant form; Sec. II.B for NGP.
//   push     Sec. II.B eq:vadv, non-relativistic Boris split.
//   move     Sec. II.B position update; offsets renormalised into [-1,1).
//   deposit  Sec. II.B eq:ngp, App. B eq:quad, at x^{n+1/2}.
//
// Data path.  Particles are structure-of-arrays and sorted by cell.  A block
// owns a contiguous chunk of particles; each of its wavefronts walks a
// contiguous sub-range 64 particles at a time, so every load and store of the
// store is coalesced and consecutive iterations of a wavefront mostly stay in
// the same cell.  The chunk's cells [c0, c1] are covered by LDS windows laid
// out in "bands": band (by[, bz]) holds the linear cells
// [c0 + by*nx (+ bz*nx*ny) - m, c1 + ... + m] modulo ncell.  A stencil point
// that wraps around the x boundary lands one band over (and a y wrap in 3D one
// plane band over), so band index and offset follow from the particle's own
// cell with no division.
//   * gather window: bands -1..1, margin 1, E and B interleaved as two float4
//     per cell, so a stencil point costs two LDS reads;
//   * deposit window: bands -3..3, margin 2, FP64 (n, Jx, Jy, Jz) per cell.
// Deposit: each lane keeps running FP32 sums of its particles that belong to
// the wavefront's current mid-point cell; when the wavefront moves on to the
// next cell the sums are reduced over each 16-lane DPP row and added to the
// window in FP64.  Particles whose mid-point sits in another cell (movers) add
// straight into the window.  Each block flushes its window to FP64 global
// accumulators; one pass converts them to the FP32 outputs.  Particles outside
// the windows (unsorted or sparse input) use global loads / FP64 global atomics.
#include "hvpic_internal.hpp"

namespace hvpic {
namespace {

constexpr int kBands = 7;                 // deposit band offsets -3..3
constexpr int kGBands = 3;                // gather band offsets -1..1
constexpr int kGroupMin = 6;              // smallest lane group worth a DPP reduction

// Particles per thread and per block, and the window limits.  A 3D chunk
// spans more bands, so it is kept shorter to keep its windows small.
template <int NDIM>
struct Chunk {
  static constexpr int PPT = NDIM == 2 ? 8 : 4;
  static constexpr int N = kBlock * PPT;
  static constexpr int WMAX = NDIM == 2 ? 64 : 20;                 // deposit window width
  static constexpr int DB = NDIM == 2 ? kBands : kBands * kBands;  // deposit bands
  static constexpr int GB = NDIM == 2 ? kGBands : kGBands * kGBands;
  static constexpr int DEP_LEN = DB * WMAX * 4;                    // doubles
  static constexpr int G_LEN = GB * (WMAX - 2) * 2;                // float4
};


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
};

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
  const float c6 = 1.0f / 6.0f, c12 = 1.0f / 12.0f;
  const float xp = 1.0f + x, xm = 1.0f - x, yp = 1.0f + y, ym = 1.0f - y;
  const float wxp = xp * xp * c12, wxm = xm * xm * c12, wyp = yp * yp * c12, wym = ym * ym * c12;
  if (NDIM == 2) {
    const float w0 = (4.0f - x * x - y * y) * c6;
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
    const float w0 = (3.0f - x * x - y * y - z * z) * c6;
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

// ---------------------------------------------------------------- deposit --

template <int NDIM, int SHAPE>
struct Stencil {
  static constexpr int T = SHAPE == HVPIC_SHAPE_NGP ? 1 : (NDIM == 2 ? 5 : 7);
};

// Offsets (relative to the mid-point cell) and weights of the stencil cells.
template <int NDIM, int SHAPE>
__device__ __forceinline__ void stencil_weights(float x, float y, float z, float* wt, int* sx,
                                                int* sy, int* sz) {
  if (SHAPE == HVPIC_SHAPE_NGP) {
    wt[0] = 1.0f;
    sx[0] = sy[0] = sz[0] = 0;
    return;
  }
  const float c6 = 1.0f / 6.0f, c12 = 1.0f / 12.0f;
  const float xp = 1.0f + x, xm = 1.0f - x, yp = 1.0f + y, ym = 1.0f - y;
  wt[0] = (NDIM == 2 ? (4.0f - x * x - y * y) : (3.0f - x * x - y * y - z * z)) * c6;
  wt[1] = xp * xp * c12;
  wt[2] = xm * xm * c12;
  wt[3] = yp * yp * c12;
  wt[4] = ym * ym * c12;
  sx[0] = 0; sy[0] = 0; sz[0] = 0;
  sx[1] = 1; sy[1] = 0; sz[1] = 0;
  sx[2] = -1; sy[2] = 0; sz[2] = 0;
  sx[3] = 0; sy[3] = 1; sz[3] = 0;
  sx[4] = 0; sy[4] = -1; sz[4] = 0;
  if (NDIM == 3) {
    const float zp = 1.0f + z, zm = 1.0f - z;
    wt[5] = zp * zp * c12;
    wt[6] = zm * zm * c12;
    sx[5] = 0; sy[5] = 0; sz[5] = 1;
    sx[6] = 0; sy[6] = 0; sz[6] = -1;
  }
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

// Sum over the 16 lanes of each DPP row; every lane of the row gets the sum.
__device__ __forceinline__ float row_sum(float v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);  // row_half_mirror
  v += dpp<0x140>(v);  // row_mirror
  return v;
}

// Deposit slot (index of the (n, Jx, Jy, Jz) quadruple in the window) of each
// stencil cell of a particle of old cell (i,j,k) = c0 + rel whose mid-point
// sits (mx,my,mz) cells away.
template <int NDIM, int SHAPE>
__device__ __forceinline__ void deposit_slots(int rel, int i, int j, int mx, int my, int mz,
                                              const int* sx, const int* sy, const int* sz, int W,
                                              const Geo& g, int* slot) {
  constexpr int T = Stencil<NDIM, SHAPE>::T;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int dxt = mx + sx[t], dyt = my + sy[t], dzt = mz + sz[t];
    const int it = i + dxt;
    const int wx = it < 0 ? 1 : (it >= g.nx ? -1 : 0);
    int band = dyt + wx + 3;
    if (NDIM == 3) {
      const int jt = j + dyt;
      const int wy = jt < 0 ? 1 : (jt >= g.ny ? -1 : 0);
      band += kBands * (dzt + wy + 3);
    }
    slot[t] = (band * W + rel + dxt + 2) * 4;
  }
}

// Running per-lane moment sums of a wavefront for its current mid-point cell.
template <int T>
struct DepState {
  float acc[T][4];
  int cur;       // wavefront-uniform: deposit slot of the current cell's centre, -1 if none
  int cslot[T];  // wavefront-uniform: slots of the current cell's stencil
};

template <int T>
__device__ __forceinline__ void dep_init(DepState<T>& D) {
  D.cur = -1;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    D.cslot[t] = 0;
    D.acc[t][0] = D.acc[t][1] = D.acc[t][2] = D.acc[t][3] = 0.0f;
  }
}

template <int T>
__device__ __forceinline__ void dep_accumulate(DepState<T>& D, bool on, float q, const float* wt,
                                               float vx, float vy, float vz) {
  const float qm = on ? q : 0.0f;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const float a = qm * wt[t];
    D.acc[t][0] += a;
    D.acc[t][1] = fmaf(a, vx, D.acc[t][1]);
    D.acc[t][2] = fmaf(a, vy, D.acc[t][2]);
    D.acc[t][3] = fmaf(a, vz, D.acc[t][3]);
  }
}

// Adds the wavefront's sums for the current cell to the window (one FP64 LDS
// atomic per value from the first lane of each DPP row).  Uniform call.
template <int T>
__device__ __forceinline__ void dep_flush(DepState<T>& D, double* win) {
  if (D.cur < 0) return;
  const bool adder = (threadIdx.x & 15) == 0;
#pragma unroll
  for (int t = 0; t < T; ++t) {
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
      const float s = row_sum(D.acc[t][ch]);
      if (adder) atomicAdd(win + D.cslot[t] + ch, (double)s);
      D.acc[t][ch] = 0.0f;
    }
  }
  D.cur = -1;
}

// One particle per lane; every lane of the wavefront calls it (uniform
// control flow).  Lanes whose mid-point cell is the wavefront's current cell
// only add to their running sums; when enough lanes have moved on to another
// cell, the current sums are flushed and that cell becomes current; the
// remaining in-window lanes add directly into the window, and lanes outside
// the window add to the FP64 global accumulators.
template <int NDIM, int SHAPE>
__device__ __forceinline__ void dep_step(DepState<Stencil<NDIM, SHAPE>::T>& D, bool live,
                                         bool inwin, bool mover, const int* slot, const float* wt,
                                         float q, float vx, float vy, float vz, double* win,
                                         int i, int j, int k, int mx, int my, int mz,
                                         const int* sx, const int* sy, const int* sz,
                                         const Geo& g, double* __restrict__ acc) {
  constexpr int T = Stencil<NDIM, SHAPE>::T;
  const int lane = threadIdx.x & 63;
  const int key = (live && inwin) ? slot[0] : -1;
  const bool mine = key >= 0 && key == D.cur;
  dep_accumulate<T>(D, mine, q, wt, vx, vy, vz);
  uint64_t pend = __ballot(key >= 0 && !mine);
  if (pend) {
    const uint64_t settled = __ballot(key >= 0 && !mine && !mover);
    const int src = 63 - __builtin_clzll(settled ? settled : pend);
    const int nkey = __builtin_amdgcn_readlane(key, src);
    const uint64_t grp = __ballot(key == nkey) & pend;
    if (__builtin_popcountll(grp) >= kGroupMin) {
      dep_flush<T>(D, win);
      D.cur = nkey;
#pragma unroll
      for (int t = 0; t < T; ++t) D.cslot[t] = __builtin_amdgcn_readlane(slot[t], src);
      dep_accumulate<T>(D, (grp >> lane) & 1ull, q, wt, vx, vy, vz);
      pend &= ~grp;
    }
    if ((pend >> lane) & 1ull) {
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const float nq = q * wt[t];
        atomicAdd(win + slot[t] + 0, (double)nq);
        atomicAdd(win + slot[t] + 1, (double)(nq * vx));
        atomicAdd(win + slot[t] + 2, (double)(nq * vy));
        atomicAdd(win + slot[t] + 3, (double)(nq * vz));
      }
    }
  }
  if (live && !inwin) {
    const int nc = g.ncell;
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
}

// Window geometry for a chunk whose first and last particles sit in c0, c1:
// deposit window width W = span + 4, gather window width W - 2.
template <int NDIM>
__device__ __forceinline__ bool window_ok(int c0, int c1, const Geo& g, int& W) {
  W = c1 - c0 + 5;
  return c0 >= 0 && c1 < g.ncell && c1 >= c0 && W <= Chunk<NDIM>::WMAX && g.nx >= 4 &&
         (NDIM == 2 || g.ny >= 4);
}

__device__ __forceinline__ int64_t window_cell(int c0, int margin, int off, int by, int bz,
                                               const Geo& g) {
  int64_t c = (int64_t)c0 - margin + off + (int64_t)by * g.nx + (int64_t)bz * g.nxny;
  c %= g.ncell;
  return c < 0 ? c + g.ncell : c;
}

// E and B of the gather window, two float4 per cell: (Ex,Ey,Ez,0),(Bx,By,Bz,0).
template <int NDIM>
__device__ void gather_window_fill(float4* geb, int WG, int c0, const Geo& g,
                                   const float* __restrict__ E, const float* __restrict__ B) {
  const int len = Chunk<NDIM>::GB * WG;
  const int nc = g.ncell;
  for (int s = threadIdx.x; s < len; s += kBlock) {
    const int band = s / WG, off = s - band * WG;
    const int by = band % kGBands - 1, bz = band / kGBands - 1;
    const int64_t c = window_cell(c0, 1, off, by, bz, g);
    geb[2 * s] = make_float4(__ldg(E + c), __ldg(E + nc + c), __ldg(E + 2 * nc + c), 0.0f);
    geb[2 * s + 1] = make_float4(__ldg(B + c), __ldg(B + nc + c), __ldg(B + 2 * nc + c), 0.0f);
  }
}

// Gather from the window for a particle of cell c0 + rel.
template <int NDIM, int SHAPE>
__device__ __forceinline__ void gather_window(const float4* geb, int WG, int rel, int i, int j,
                                              float x, float y, float z, const Geo& g,
                                              float Ep[3], float Bp[3]) {
  constexpr int T = Stencil<NDIM, SHAPE>::T;
  float wt[T];
  int sx[T], sy[T], sz[T];
  stencil_weights<NDIM, SHAPE>(x, y, z, wt, sx, sy, sz);
  Ep[0] = Ep[1] = Ep[2] = Bp[0] = Bp[1] = Bp[2] = 0.0f;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int it = i + sx[t];
    const int wx = it < 0 ? 1 : (it >= g.nx ? -1 : 0);
    int band = sy[t] + wx + 1;
    if (NDIM == 3) {
      const int jt = j + sy[t];
      const int wy = jt < 0 ? 1 : (jt >= g.ny ? -1 : 0);
      band += kGBands * (sz[t] + wy + 1);
    }
    const int s = band * WG + rel + sx[t] + 1;
    const float4 e = geb[2 * s], b = geb[2 * s + 1];
    Ep[0] = fmaf(wt[t], e.x, Ep[0]);
    Ep[1] = fmaf(wt[t], e.y, Ep[1]);
    Ep[2] = fmaf(wt[t], e.z, Ep[2]);
    Bp[0] = fmaf(wt[t], b.x, Bp[0]);
    Bp[1] = fmaf(wt[t], b.y, Bp[1]);
    Bp[2] = fmaf(wt[t], b.z, Bp[2]);
  }
}

template <int NDIM>
__device__ void window_flush(const double* win, int W, int c0, const Geo& g,
                             double* __restrict__ acc) {
  const int len = Chunk<NDIM>::DB * W * 4;
  for (int s = threadIdx.x; s < len; s += kBlock) {
    const double v = win[s];
    if (v == 0.0) continue;
    const int ch = s & 3;
    const int cellslot = s >> 2;
    const int band = cellslot / W;
    const int off = cellslot - band * W;
    const int64_t c = window_cell(c0, 2, off, band % kBands - 3, band / kBands - 3, g);
    unsafeAtomicAdd(acc + (int64_t)ch * g.ncell + c, v);
  }
}

// ---------------------------------------------------------------- kernels --

template <int NDIM, int SHAPE, bool DEP>
__global__ __launch_bounds__(kBlock) void k_gather_push(PushArgs A) {
  constexpr int PPT = Chunk<NDIM>::PPT;
  constexpr int T = Stencil<NDIM, SHAPE>::T;
  __shared__ float4 geb[Chunk<NDIM>::G_LEN];
  __shared__ double win[DEP ? Chunk<NDIM>::DEP_LEN : 1];
  __shared__ int s_c[2];
  const Geo& g = A.g;
  const int64_t base = (int64_t)blockIdx.x * Chunk<NDIM>::N;
  const int64_t end = min(base + (int64_t)Chunk<NDIM>::N, A.n);
  if (threadIdx.x == 0) {
    s_c[0] = A.cell[base];
    s_c[1] = A.cell[end - 1];
  }
  __syncthreads();
  const int c0 = s_c[0], span = s_c[1] - s_c[0];
  int W = 0;
  const bool wok = window_ok<NDIM>(c0, s_c[1], g, W);
  if (wok) {
    gather_window_fill<NDIM>(geb, W - 2, c0, g, A.E, A.B);
    if (DEP)
      for (int s = threadIdx.x; s < Chunk<NDIM>::DB * W * 4; s += kBlock) win[s] = 0.0;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int64_t wbase = base + (int64_t)(threadIdx.x >> 6) * 64 * PPT;
  const bool want_diag = A.diag_part != nullptr;
  float dK = 0.f, dP0 = 0.f, dP1 = 0.f, dP2 = 0.f;
  DepState<T> D;
  if (DEP) dep_init<T>(D);
  for (int it = 0; it < PPT; ++it) {
    const int64_t idx = wbase + it * 64 + lane;
    bool live = idx < end;
    int a = 0;
    float x = 0.f, y = 0.f, z = 0.f, vx = 0.f, vy = 0.f, vz = 0.f, wq = 0.f;
    if (live) {
      a = A.cell[idx];
      x = A.ox[idx];
      y = A.oy[idx];
      if (NDIM == 3) z = A.oz[idx];
      vx = A.ux[idx];
      vy = A.uy[idx];
      vz = A.uz[idx];
      if (DEP || want_diag) wq = A.w[idx];
      if ((unsigned)a >= (unsigned)g.ncell) {
        raise_flag(A.st, HVPIC_FLAG_BAD_INPUT, &A.st->bad_input);
        live = false;
      }
    }
    const int rel = a - c0;
    const bool in_window = wok && rel >= 0 && rel <= span;
    int i = 0, j = 0, k = 0, mx = 0, my = 0, mz = 0;
    float xm = 0.f, ym = 0.f, zm = 0.f;
    if (live) {
      decompose(a, g, i, j, k);
      float Ep[3], Bp[3];
      if (in_window)
        gather_window<NDIM, SHAPE>(geb, W - 2, rel, i, j, x, y, z, g, Ep, Bp);
      else
        gather_eb<NDIM, SHAPE>(A.E, A.B, a, i, j, k, x, y, z, g, Ep, Bp);
      // Boris: half kick, rotation, half kick.
      const float h = A.a;
      const float vmx = fmaf(h, Ep[0], vx), vmy = fmaf(h, Ep[1], vy), vmz = fmaf(h, Ep[2], vz);
      const float tx = h * Bp[0], ty = h * Bp[1], tz = h * Bp[2];
      const float f = 2.0f / (1.0f + (tx * tx + ty * ty + tz * tz));
      const float sx = f * tx, sy = f * ty, sz = f * tz;
      const float px = vmx + (vmy * tz - vmz * ty);
      const float py = vmy + (vmz * tx - vmx * tz);
      const float pz = vmz + (vmx * ty - vmy * tx);
      const float nvx = fmaf(h, Ep[0], vmx + (py * sz - pz * sy));
      const float nvy = fmaf(h, Ep[1], vmy + (pz * sx - px * sz));
      const float nvz = fmaf(h, Ep[2], vmz + (px * sy - py * sx));
      if (want_diag) {
        dK = fmaf(wq, vx * nvx + vy * nvy + vz * nvz, dK);
        dP0 = fmaf(wq, vx + nvx, dP0);
        dP1 = fmaf(wq, vy + nvy, dP1);
        dP2 = fmaf(wq, vz + nvz, dP2);
      }
      // Move: x^{n+1} = x^n + v^{n+1/2} dt, renormalised offsets.
      float nx_ = fmaf(nvx, A.kx, x), ny_ = fmaf(nvy, A.ky, y), nz_ = z;
      int si = 0, sj = 0, sk = 0;
      bool ok = renorm(nx_, si) && renorm(ny_, sj);
      if (NDIM == 3) {
        nz_ = fmaf(nvz, A.kz, z);
        ok = ok && renorm(nz_, sk);
      }
      if (!ok) {
        raise_flag(A.st, HVPIC_FLAG_NONFINITE, &A.st->nonfinite);
        si = sj = sk = 0;
        nx_ = x;
        ny_ = y;
        nz_ = z;
      } else if (si > 1 || si < -1 || sj > 1 || sj < -1 || sk > 1 || sk < -1) {
        raise_flag(A.st, HVPIC_FLAG_MOVE_GT1, &A.st->moved_gt1);
      }
      int ni = i + si, nj = j + sj, nk = k + sk;
      if ((unsigned)ni >= (unsigned)g.nx) ni = wrapi(ni, g.nx);
      if ((unsigned)nj >= (unsigned)g.ny) nj = wrapi(nj, g.ny);
      if (NDIM == 3 && (unsigned)nk >= (unsigned)g.nz) nk = wrapi(nk, g.nz);
      A.cell[idx] = ni + g.nx * (nj + g.ny * nk);
      A.ox[idx] = nx_;
      A.oy[idx] = ny_;
      if (NDIM == 3) A.oz[idx] = nz_;
      A.ux[idx] = nvx;
      A.uy[idx] = nvy;
      A.uz[idx] = nvz;
      if (DEP) {
        // Mid-point x^{n+1/2} = x^n + (dt/2) v^{n+1/2}.
        xm = fmaf(nvx, 0.5f * A.kx, x);
        ym = fmaf(nvy, 0.5f * A.ky, y);
        zm = NDIM == 3 ? fmaf(nvz, 0.5f * A.kz, z) : 0.0f;
        if (!ok || !renorm(xm, mx) || !renorm(ym, my) || (NDIM == 3 && !renorm(zm, mz))) {
          xm = x; ym = y; zm = z; mx = my = mz = 0;
        }
        vx = nvx;
        vy = nvy;
        vz = nvz;
      }
    }
    if (DEP) {
      float wt[T];
      int sxs[T], sys[T], szs[T], slot[T];
      stencil_weights<NDIM, SHAPE>(xm, ym, zm, wt, sxs, sys, szs);
      const bool inwin = in_window && mx >= -1 && mx <= 1 && my >= -1 && my <= 1 && mz >= -1 &&
                         mz <= 1;
      deposit_slots<NDIM, SHAPE>(rel, i, j, mx, my, mz, sxs, sys, szs, W, g, slot);
      dep_step<NDIM, SHAPE>(D, live, inwin, (mx | my | mz) != 0, slot, wt, A.qV * wq, vx, vy, vz,
                            win, i, j, k, mx, my, mz, sxs, sys, szs, g, A.acc);
    }
  }
  if (DEP) dep_flush<T>(D, win);
  if (want_diag) {
    const double hm = 0.5 * A.ms;
    double v[4] = {hm * dK, hm * dP0, hm * dP1, hm * dP2};
    block_partial<4>(v, A.diag_part);
  }
  if (DEP && wok) {
    __syncthreads();
    window_flush<NDIM>(win, W, c0, g, A.acc);
  }
}

template <int NDIM, int SHAPE>
__global__ __launch_bounds__(kBlock) void k_deposit(DepArgs A) {
  constexpr int PPT = Chunk<NDIM>::PPT;
  constexpr int T = Stencil<NDIM, SHAPE>::T;
  __shared__ double win[Chunk<NDIM>::DEP_LEN];
  __shared__ int s_c[2];
  const Geo& g = A.g;
  const int64_t base = (int64_t)blockIdx.x * Chunk<NDIM>::N;
  const int64_t end = min(base + (int64_t)Chunk<NDIM>::N, A.n);
  if (threadIdx.x == 0) {
    s_c[0] = A.cell[base];
    s_c[1] = A.cell[end - 1];
  }
  __syncthreads();
  const int c0 = s_c[0], span = s_c[1] - s_c[0];
  int W = 0;
  const bool wok = window_ok<NDIM>(c0, s_c[1], g, W);
  if (wok)
    for (int s = threadIdx.x; s < Chunk<NDIM>::DB * W * 4; s += kBlock) win[s] = 0.0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t wbase = base + (int64_t)(threadIdx.x >> 6) * 64 * PPT;
  DepState<T> D;
  dep_init<T>(D);
  for (int it = 0; it < PPT; ++it) {
    const int64_t idx = wbase + it * 64 + lane;
    bool live = idx < end;
    int a = 0, i = 0, j = 0, k = 0, mx = 0, my = 0, mz = 0;
    float x = 0.f, y = 0.f, z = 0.f, vx = 0.f, vy = 0.f, vz = 0.f, q = 0.f;
    if (live) {
      a = A.cell[idx];
      x = A.ox[idx];
      y = A.oy[idx];
      if (NDIM == 3) z = A.oz[idx];
      vx = A.ux[idx];
      vy = A.uy[idx];
      vz = A.uz[idx];
      q = A.qV * A.w[idx];
      if ((unsigned)a >= (unsigned)g.ncell) {
        raise_flag(A.st, HVPIC_FLAG_BAD_INPUT, &A.st->bad_input);
        live = false;
        a = 0;
      }
    }
    if (live) {
      decompose(a, g, i, j, k);
      float xm = fmaf(vx, A.bx, x), ym = fmaf(vy, A.by, y), zm = NDIM == 3 ? fmaf(vz, A.bz, z) : 0.f;
      if (renorm(xm, mx) && renorm(ym, my) && (NDIM == 2 || renorm(zm, mz))) {
        x = xm;
        y = ym;
        z = zm;
      } else {
        mx = my = mz = 0;
      }
    }
    const int rel = a - c0;
    const bool inwin = wok && rel >= 0 && rel <= span && mx >= -1 && mx <= 1 && my >= -1 &&
                       my <= 1 && mz >= -1 && mz <= 1;
    float wt[T];
    int sxs[T], sys[T], szs[T], slot[T];
    stencil_weights<NDIM, SHAPE>(x, y, z, wt, sxs, sys, szs);
    deposit_slots<NDIM, SHAPE>(rel, i, j, mx, my, mz, sxs, sys, szs, W, g, slot);
    dep_step<NDIM, SHAPE>(D, live, inwin, (mx | my | mz) != 0, slot, wt, q, vx, vy, vz, win, i, j,
                          k, mx, my, mz, sxs, sys, szs, g, A.acc);
  }
  dep_flush<T>(D, win);
  if (wok) {
    __syncthreads();
    window_flush<NDIM>(win, W, c0, g, A.acc);
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
// for the next deposit.
__global__ void k_moments_out(double* __restrict__ acc, int ncell, float* __restrict__ n,
                              float* __restrict__ J) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 4ll * ncell; i += stride) {
    const float v = (float)acc[i];
    acc[i] = 0.0;
    if (i < ncell)
      n[i] = v;
    else
      J[i - ncell] = v;
  }
}

__global__ void k_write_zero_diag(double* out, int nv) {
  if (threadIdx.x < nv) out[threadIdx.x] = 0.0;
}

__global__ __launch_bounds__(kBlock) void k_push_diag_final(const double* part, int nblocks,
                                                            double* out) {
  double r[4];
  sum_partials<4>(part, nblocks, r);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) out[k] = r[k];
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

template <int NDIM, int SHAPE>
void push_dispatch(bool dep, dim3 grid, hipStream_t s, const PushArgs& A) {
  if (dep)
    hipLaunchKernelGGL((k_gather_push<NDIM, SHAPE, true>), grid, dim3(kBlock), 0, s, A);
  else
    hipLaunchKernelGGL((k_gather_push<NDIM, SHAPE, false>), grid, dim3(kBlock), 0, s, A);
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

void moments_out(hvpic_ctx* c, float* n, float* J) {
  const int blocks = (int)std::min<int64_t>(ceil_div(4ll * c->ncell, kBlock), 2048);
  hipLaunchKernelGGL(k_moments_out, dim3(blocks), dim3(kBlock), 0, c->stream, c->mom_acc,
                     c->ncell, n, J);
}

int launch_gather_push(hvpic_ctx* c, hvpic_particles* p, const float* E, const float* B,
                       float* n_mid, float* J_mid, double* diag_out) {
  const bool dep = n_mid != nullptr && J_mid != nullptr;
  if (p->n == 0) {
    if (diag_out) hipLaunchKernelGGL(k_write_zero_diag, dim3(1), dim3(64), 0, c->stream, diag_out, 4);
    if (dep) moments_out(c, n_mid, J_mid);
    return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
  }
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
  const bool qs = c->p.shape == HVPIC_SHAPE_QS;
  int nblocks = 0;
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
  if (dep) moments_out(c, n_mid, J_mid);
  if (diag_out)
    hipLaunchKernelGGL(k_push_diag_final, dim3(1), dim3(kBlock), 0, c->stream,
                       (const double*)c->push_part, nblocks, diag_out);
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

int launch_deposit(hvpic_ctx* c, const hvpic_particles* p, float half_dt_back, float* n,
                   float* J) {
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

}  // namespace hvpic
