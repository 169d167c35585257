// Stable counting sort of the particle store by cell index (gfx950).
//
// The paper keeps each particle as a cell index plus in-cell offsets (Sec.
// II.B); keeping the store ordered by cell is what makes the deposit's LDS
// windows and the gather's cache reuse work.  The result is the one stable
// order: by cell, equal cells in input order, plus cell_start[ncell+1].
//
// Neighbour-move path.  The input was sorted by the cells the particles held
// before the last push, and a push moves a particle by at most one cell per
// axis.  For an old cell a and a move direction d (3^ndim of them) let
// cnt[a][d] be the number of its particles that moved by d.  The particles
// landing in a new cell c come from the 3^ndim cells c - d; in the stable
// order they appear grouped by old cell index (the input order), and inside a
// group in input order.  So with cell_start[c] from the prefix sum of the
// per-new-cell totals, the first slot of group (a, d) is cell_start[c] plus the
// counts of the groups of c whose old cell index is smaller, and a particle's
// slot adds its rank among the earlier particles of its own group, found with
// wavefront ballots.  Kernels: count (one wavefront per old cell; skipped when
// the push already counted), tile totals of the new counts, per-cell prefix +
// group bases (each block adds up the tile totals before its own), scatter
// (one wavefront per two old cells).  A particle that moved further (or an
// inconsistent cell_start) is flagged by the count pass; the flag is handed
// to the scatter kernel, in which one block then runs the general sort on its
// own (slow, but it costs no extra launch in the common case and needs no host
// round trip).
//
// General path.  LSD radix sort of (cell, index) pairs with 8-bit digits;
// each pass is a per-tile digit histogram, a scan of the digit-major
// histogram, and a stable scatter whose in-tile ranks come from per-wavefront
// match masks.  The permutation then gathers the particle fields.  The same
// tile ranking drives the single-block fallback.
#include <string.h>

#include "hvpic_internal.hpp"

namespace hvpic {
namespace {

constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

struct SortGeo {
  int nx, ny, nz, ncell;
  FastDiv fnx, fny;
};

__device__ __forceinline__ void ijk(int c, const SortGeo& g, int& i, int& j, int& k) {
  const uint32_t q = fdiv((uint32_t)c, g.fnx);
  i = c - (int)q * g.nx;
  const uint32_t q2 = fdiv(q, g.fny);
  j = (int)q - (int)q2 * g.ny;
  k = (int)q2;
}

template <int NDIM>
struct Dirs {
  static constexpr int N = NDIM == 2 ? 9 : 27;
  static constexpr int BITS = NDIM == 2 ? 4 : 5;
};

// Direction code of a particle of old cell (i,j,k) now in cell key; -1 when it
// moved more than one cell along some axis (or the key is invalid).
template <int NDIM>
__device__ __forceinline__ int direction(int key, int i, int j, int k, const SortGeo& g) {
  if ((unsigned)key >= (unsigned)g.ncell) return -1;
  int i2, j2, k2;
  ijk(key, g, i2, j2, k2);
  const int di = canon_move(i2 - i, g.nx), dj = canon_move(j2 - j, g.ny);
  const int dk = NDIM == 3 ? canon_move(k2 - k, g.nz) : 0;
  if (di == 2 || dj == 2 || dk == 2) return -1;
  return (di + 1) + 3 * (dj + 1) + (NDIM == 3 ? 9 * (dk + 1) : 0);
}

// The same for a 2D old cell a whose neighbours need no wrap (an interior
// cell, one or more cells from every edge): from the index difference by two
// compares instead of two divisions.  The neighbours of such a cell are
// exactly the differences 0, +-1, +-nx, +-nx +- 1.
__device__ __forceinline__ int direction_interior2d(int key, int a, int nx) {
  const int delta = key - a;
  const int dj = delta >= nx - 1 ? 1 : (delta <= 1 - nx ? -1 : 0);
  const int di = delta - dj * nx;
  return di >= -1 && di <= 1 ? (di + 1) + 3 * (dj + 1) : -1;
}

// Whether the wavefront's old cells a0 .. a0+na-1 are all 2D interior cells.
template <int NDIM>
__device__ __forceinline__ bool wave_interior(int a0, int na, const SortGeo& g) {
  if (NDIM != 2 || g.nx < 3 || g.ny < 3) return false;
  int i0, j0, k0, i1, j1, k1;
  ijk(a0, g, i0, j0, k0);
  ijk(a0 + na - 1, g, i1, j1, k1);
  return i0 >= 1 && i1 <= g.nx - 2 && j0 >= 1 && j1 <= g.ny - 2 && j0 == j1;
}

// New cell reached from old cell a by direction d (wrapped).
template <int NDIM>
__device__ __forceinline__ int step_cell(int i, int j, int k, int d, const SortGeo& g) {
  const int di = d % 3 - 1, dj = (d / 3) % 3 - 1, dk = NDIM == 3 ? d / 9 - 1 : 0;
  int i2 = i + di, j2 = j + dj, k2 = k + dk;
  if (i2 < 0) i2 += g.nx; else if (i2 >= g.nx) i2 -= g.nx;
  if (j2 < 0) j2 += g.ny; else if (j2 >= g.ny) j2 -= g.ny;
  if (NDIM == 3) { if (k2 < 0) k2 += g.nz; else if (k2 >= g.nz) k2 -= g.nz; }
  return i2 + g.nx * (j2 + g.ny * k2);
}

// Mask of the lanes of `valid` whose code equals this lane's `code`, computed
// from one ballot per code bit.
template <int BITS>
__device__ __forceinline__ uint64_t match_code(int code, uint64_t valid, const uint64_t* bal) {
  uint64_t m = valid;
#pragma unroll
  for (int b = 0; b < BITS; ++b) m &= ((code >> b) & 1) ? bal[b] : ~bal[b];
  return m;
}

// ------------------------------------------------------- neighbour path --

// Each wavefront handles kCellsPerWave consecutive old cells and streams
// their particles in full 64-lane batches (a batch may straddle cells).
constexpr int kCellsPerWave = 2;
constexpr int kCellBits = 1;
constexpr int kCountBatches = 4;    // 64-particle batches whose keys are loaded together
// The scatter takes kScatterCells cells per wavefront.
constexpr int kScatterCells = 2;
constexpr int kScatterCellBits = 1;
constexpr int kScatterBatches = 4;  // batches whose fields are loaded together

// Boundaries of the wavefront's cells: b(m) = cs_prev[a0 + m], m = 0..na,
// held by lane m.  Returns false if they are not a monotone partition of
// [0, n] (then nothing of the wavefront is trusted).
__device__ __forceinline__ bool wave_bounds(const int32_t* cs_prev, int a0, int na, int64_t n,
                                            int lane, int& bnd) {
  bnd = lane <= na ? cs_prev[a0 + lane] : 0;
  const int prev = __shfl_up(bnd, 1);
  const bool bad = lane <= na && (bnd < 0 || bnd > n || (lane > 0 && bnd < prev));
  return __ballot(bad) == 0;
}

// Cell index m (0..na-1) within the wavefront of particle p, from the
// boundaries b(1..na-1) read from lanes 1..na-1 (all lanes must call it).
__device__ __forceinline__ int cell_in_wave(int64_t p, int bnd, int na) {
  int m = 0;
  for (int q = 1; q < na; ++q) m += p >= (int64_t)__builtin_amdgcn_readlane(bnd, q) ? 1 : 0;
  return m;
}
// The same for an unsigned 32-bit position (cell_start values are
// non-negative int32, checked by the caller).
__device__ __forceinline__ int cell_in_wave32(uint32_t p, int bnd, int na) {
  int m = 0;
  for (int q = 1; q < na; ++q) m += p >= (uint32_t)__builtin_amdgcn_readlane(bnd, q) ? 1 : 0;
  return m;
}

template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_nb_count(const int32_t* __restrict__ key,
                                                     const int32_t* __restrict__ cs_prev, int64_t n,
                                                     SortGeo g, uint32_t* __restrict__ cnt,
                                                     Status* st) {
  constexpr int ND = Dirs<NDIM>::N, NB = Dirs<NDIM>::BITS;
  constexpr int CODE_BITS = NB + kCellBits;
  __shared__ uint32_t s_cnt[kWaves][kCellsPerWave * ND];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int a0 = (blockIdx.x * kWaves + wid) * kCellsPerWave;
  const int na = a0 < g.ncell ? min(kCellsPerWave, g.ncell - a0) : 0;
  for (int q = lane; q < kCellsPerWave * ND; q += 64) s_cnt[wid][q] = 0;
  __syncthreads();
  if (na == 0) return;
  int bnd;
  if (!wave_bounds(cs_prev, a0, na, n, lane, bnd)) {
    if (lane == 0) {
      raise_flag(st, HVPIC_FLAG_BAD_INPUT, &st->bad_input);
      __hip_atomic_store(&st->far_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  const int64_t pb = __builtin_amdgcn_readlane(bnd, 0), pe = __builtin_amdgcn_readlane(bnd, na);
  bool far = false;
  for (int64_t q0 = pb; q0 < pe; q0 += 64 * kCountBatches) {
   int keys[kCountBatches];
#pragma unroll
   for (int b = 0; b < kCountBatches; ++b) {
     const int64_t p = q0 + b * 64 + lane;
     keys[b] = p < pe ? key[p] : 0;
   }
#pragma unroll
   for (int b = 0; b < kCountBatches; ++b) {
    const int64_t p = q0 + b * 64 + lane;
    const bool valid = p < pe;
    int code = 0;
    bool ok = false;
    const int m = cell_in_wave(p, bnd, na);
    if (valid) {
      int i, j, k;
      ijk(a0 + m, g, i, j, k);
      const int d = direction<NDIM>(keys[b], i, j, k, g);
      far |= d < 0;
      ok = d >= 0;
      code = (m << NB) | (ok ? d : 0);
    }
    uint64_t bal[CODE_BITS];
    const uint64_t vmask = __ballot(ok);
#pragma unroll
    for (int b = 0; b < CODE_BITS; ++b) bal[b] = __ballot(ok && ((code >> b) & 1));
    const uint64_t mine = match_code<CODE_BITS>(code, vmask, bal);
    if (ok && (mine & lanemask_lt()) == 0) {
      const int mm = code >> NB, d = code & ((1 << NB) - 1);
      s_cnt[wid][mm * ND + d] += (uint32_t)__builtin_popcountll(mine);
    }
    __builtin_amdgcn_wave_barrier();
   }
  }
  if (__ballot(far) && lane == 0) {
    atomicOr(&st->flags, (uint32_t)HVPIC_FLAG_MOVE_GT1);
    __hip_atomic_store(&st->far_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  for (int q = lane; q < na * ND; q += 64) cnt[(int64_t)a0 * ND + q] = s_cnt[wid][q];
}

// Block-level exclusive scan of TILE values held in LDS `s`; returns the
// tile total.  Thread t owns elements [t*PER, t*PER+PER).
template <int TILE = kScanTile>
__device__ uint32_t tile_exclusive_scan(uint32_t* s) {
  constexpr int PER = TILE / kBlock;
  __shared__ uint32_t wsum[kWaves];
  const int t = threadIdx.x;
  uint32_t v[PER], acc = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    v[q] = s[t * PER + q];
    acc += v[q];
  }
  // inclusive scan of acc over the block
  uint32_t x = acc;
  const int lane = t & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[t >> 6] = x;
  __syncthreads();
  uint32_t woff = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    if (w < (t >> 6)) woff += wsum[w];
    total += wsum[w];
  }
  uint32_t run = woff + x - acc;  // exclusive prefix of this thread
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    s[t * PER + q] = run;
    run += v[q];
  }
  __syncthreads();
  return total;
}

// Open x boundaries (Sec. II.C): the cells i = 0 and i = nx-1 are ghosts.
// Ions whose new cell is a ghost cell are absorbed (left out of the order);
// inj_cnt[f*rows + r] ions injected through face f into its row r = j + ny k
// (rows = ny nz) follow the pushed ions in the store and come last in their
// cell (i = 1 for f = 0, nx-2 for f = 1).  inj_base receives the first slot
// of each such group; info[0] = 1 when the neighbour path cannot be taken
// (far movers or an inconsistent cell_start: nothing else is then written).
struct OpenSort {
  const int32_t* inj_cnt;  // [2][rows] or null (no injection)
  int32_t* inj_base;       // [2][rows]
  int32_t* info;           // device int32[2] or null
  int rows;
};

// Per-new-cell totals, written to cs[c], and their per-tile sums (tiles of
// TILE cells).
template <int NDIM, int TILE, bool OPEN = false>
__device__ __forceinline__ void nb_newcount_body(const uint32_t* __restrict__ cnt, const SortGeo& g,
                                                 int32_t* __restrict__ cs,
                                                 uint32_t* __restrict__ blk, Status* st, int bid,
                                                 const OpenSort& os = OpenSort{}) {
  constexpr int ND = Dirs<NDIM>::N;
  __shared__ uint32_t wsum[kWaves];
  if (bid == 0 && threadIdx.x == 0) {
    const uint32_t f = __hip_atomic_load(&st->far_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&st->far_decision, f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&st->far_flag, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (OPEN && os.info) os.info[0] = f != 0u ? 1 : 0;
  }
  const int64_t t0 = (int64_t)bid * TILE;
  uint32_t local = 0;
  for (int q = 0; q < TILE / kBlock; ++q) {
    const int64_t c = t0 + q * kBlock + threadIdx.x;
    if (c >= g.ncell) break;
    int i, j, k;
    ijk((int)c, g, i, j, k);
    uint32_t s = 0;
    for (int d = 0; d < ND; ++d) {
      const int src = step_cell<NDIM>(i, j, k, ND - 1 - d, g);  // c - d == c + (ND-1-d)
      s += cnt[(int64_t)src * ND + d];
    }
    if (OPEN) {
      if (i == 0 || i == g.nx - 1) {
        s = 0;
      } else if (os.inj_cnt) {
        const int r = j + g.ny * k;
        if (i == 1) s += (uint32_t)os.inj_cnt[r];
        if (i == g.nx - 2) s += (uint32_t)os.inj_cnt[os.rows + r];
      }
    }
    cs[c] = (int32_t)s;
    local += s;
  }
  for (int o = 32; o > 0; o >>= 1) local += __shfl_xor(local, o);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = local;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (int w = 0; w < kWaves; ++w) s += wsum[w];
    blk[bid] = s;
  }
}

template <int NDIM, int TILE>
__global__ __launch_bounds__(kBlock) void k_nb_newcount(const uint32_t* __restrict__ cnt, SortGeo g,
                                                        int32_t* __restrict__ cs,
                                                        uint32_t* __restrict__ blk, Status* st) {
  nb_newcount_body<NDIM, TILE>(cnt, g, cs, blk, st, blockIdx.x);
}

// Exclusive scan of m tile totals in one block (in place); blk[m] = total.
__global__ __launch_bounds__(1024) void k_scan_tiles(uint32_t* blk, int m) {
  __shared__ uint32_t wsum[16];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int base = 0; base < m; base += 1024) {
    const int idx = base + threadIdx.x;
    const uint32_t v = idx < m ? blk[idx] : 0u;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    uint32_t woff = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
      if (w < wid) woff += wsum[w];
      tot += wsum[w];
    }
    const uint32_t c0 = carry;
    if (idx < m) blk[idx] = c0 + woff + x - v;
    __syncthreads();
    if (threadIdx.x == 0) carry = c0 + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) blk[m] = carry;
}

// Sum of v[0..m) by the whole block (every thread gets it).
__device__ uint32_t block_sum(const uint32_t* __restrict__ v, int m) {
  __shared__ uint32_t ws[kWaves];
  uint32_t x = 0;
  for (int i = threadIdx.x; i < m; i += kBlock) x += v[i];
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = x;
  __syncthreads();
  uint32_t t = 0;
  for (int w = 0; w < kWaves; ++w) t += ws[w];
  __syncthreads();
  return t;
}

// cell_start from the per-cell totals, and the first slot of every group
// (source cell, direction) of each new cell, written over cnt.  blk holds
// the tile totals; each block adds up those before it (a few hundred values
// at most), which spares a separate scan launch.
template <int NDIM, int TILE, bool OPEN = false>
__device__ __forceinline__ void nb_bases_body(uint32_t* __restrict__ cnt, const SortGeo& g,
                                              int32_t* __restrict__ cs,
                                              const uint32_t* __restrict__ blk, int bid,
                                              const OpenSort& os = OpenSort{}) {
  constexpr int ND = Dirs<NDIM>::N;
  __shared__ uint32_t s[TILE];
  const int64_t t0 = (int64_t)bid * TILE;
  for (int q = 0; q < TILE / kBlock; ++q) {
    const int64_t c = t0 + q * kBlock + threadIdx.x;
    s[q * kBlock + threadIdx.x] = c < g.ncell ? (uint32_t)cs[c] : 0u;
  }
  __syncthreads();
  const uint32_t tile_total = tile_exclusive_scan<TILE>(s);
  const uint32_t off = block_sum(blk, bid);
  for (int q = 0; q < TILE / kBlock; ++q) {
    const int64_t c = t0 + q * kBlock + threadIdx.x;
    if (c >= g.ncell) break;
    const uint32_t start = off + s[q * kBlock + threadIdx.x];
    cs[c] = (int32_t)start;
    if (c == g.ncell - 1) cs[g.ncell] = (int32_t)(off + tile_total);
    int i, j, k;
    ijk((int)c, g, i, j, k);
    int src[ND];
    uint32_t n[ND];
    for (int d = 0; d < ND; ++d) {
      src[d] = step_cell<NDIM>(i, j, k, ND - 1 - d, g);
      n[d] = cnt[(int64_t)src[d] * ND + d];
    }
    // groups in increasing old-cell index (ties only between empty groups).
    // For a cell whose neighbours need no wrap that order is d = ND-1 .. 0
    // (the source index falls as d rises), so the slots are a suffix sum.
    const bool interior = g.nx >= 3 && g.ny >= 3 && i >= 1 && i <= g.nx - 2 && j >= 1 &&
                          j <= g.ny - 2 &&
                          (NDIM == 2 || (g.nz >= 3 && k >= 1 && k <= g.nz - 2));
    if (OPEN && os.inj_cnt && (i == 1 || i == g.nx - 2)) {
      // the injected ions of the cell follow all the moved ones
      const int r = j + g.ny * k;
      uint32_t moved = 0;
      for (int d = 0; d < ND; ++d) moved += n[d];
      if (i == 1) os.inj_base[r] = (int32_t)(start + moved);
      if (i == g.nx - 2)
        os.inj_base[os.rows + r] =
            (int32_t)(start + moved + (i == 1 ? (uint32_t)os.inj_cnt[r] : 0u));
    }
    if (interior) {
      uint32_t before = 0;
#pragma unroll
      for (int d = ND - 1; d >= 0; --d) {
        cnt[(int64_t)src[d] * ND + d] = start + before;
        before += n[d];
      }
    } else {
      for (int d = 0; d < ND; ++d) {
        uint32_t before = 0;
        for (int e = 0; e < ND; ++e)
          if (src[e] < src[d] || (src[e] == src[d] && e < d)) before += n[e];
        cnt[(int64_t)src[d] * ND + d] = start + before;
      }
    }
  }
}

template <int NDIM, int TILE>
__global__ __launch_bounds__(kBlock) void k_nb_bases(uint32_t* __restrict__ cnt, SortGeo g,
                                                     int32_t* __restrict__ cs,
                                                     const uint32_t* __restrict__ blk) {
  nb_bases_body<NDIM, TILE>(cnt, g, cs, blk, blockIdx.x);
}


struct Fields {
  int32_t* cell;
  float* f[7];    // ox, oy, oz, ux, uy, uz, w (oz may be null)
  int32_t* perm;  // output only: if set, the order is written as this gather
                  // map (sorted position -> input index) and nothing else moves
};

// ------------------------------------------------------------- radix path --

// Stable destination of this thread's element in a block-wide tile whose
// elements are ordered by thread index.  run[b] is the first free slot of
// digit b and is advanced past the tile.  Every thread of the block calls it.
__device__ uint32_t tile_dest(bool valid, int digit, uint32_t (*wcnt)[kRadixBins], uint32_t* run) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  for (int b = threadIdx.x; b < nw * kRadixBins; b += blockDim.x) (&wcnt[0][0])[b] = 0;
  __syncthreads();
  uint64_t bal[kRadixBits];
  const uint64_t vmask = __ballot(valid);
#pragma unroll
  for (int b = 0; b < kRadixBits; ++b) bal[b] = __ballot(valid && ((digit >> b) & 1));
  const uint64_t mine = match_code<kRadixBits>(digit, vmask, bal);
  const uint32_t rank = (uint32_t)__builtin_popcountll(mine & lanemask_lt());
  if (valid && rank == 0) wcnt[wid][digit] = (uint32_t)__builtin_popcountll(mine);
  __syncthreads();
  uint32_t dst = 0;
  if (valid) {
    uint32_t before = run[digit];
    for (int w = 0; w < wid; ++w) before += wcnt[w][digit];
    dst = before + rank;
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kRadixBins; b += blockDim.x) {
    uint32_t s = 0;
    for (int w = 0; w < nw; ++w) s += wcnt[w][b];
    run[b] += s;
  }
  __syncthreads();
  return dst;
}

__device__ __forceinline__ uint32_t load_key(const uint32_t* kin, const int32_t* cells, int64_t i,
                                             int ncell) {
  uint32_t key = kin ? kin[i] : (uint32_t)cells[i];
  return key >= (uint32_t)ncell ? (uint32_t)ncell - 1 : key;  // invalid cells were flagged upstream
}

// Sorted-order gather of the particle fields plus cell_start from the sorted
// keys: the boundary between positions r-1 and r fills the starts of the cells
// in (key[r-1], key[r]].  Threads start at `first` and step by `stride`.
__device__ void gather_fields(const uint32_t* keys, const uint32_t* perm, int64_t n, Fields in,
                              Fields out, int32_t* cs, int ncell, int64_t first, int64_t stride) {
  for (int64_t r = first; r <= n; r += stride) {
    const int kprev = r == 0 ? -1 : (int)(keys ? keys[r - 1] : 0u);
    const int knext = r == n ? ncell : (int)(keys ? keys[r] : 0u);
    for (int c = kprev + 1; c <= knext && c <= ncell; ++c) cs[c] = (int32_t)r;
    if (r < n) {
      const uint32_t src = perm ? perm[r] : (uint32_t)r;
      if (out.perm) {
        out.perm[r] = (int32_t)src;
      } else {
        out.cell[r] = in.cell[src];
#pragma unroll
        for (int f = 0; f < 7; ++f)
          if (in.f[f]) out.f[f][r] = in.f[f][src];
      }
    }
  }
}

// Per-tile histogram of one digit; hist is digit-major [bin][tile].
__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                       const int32_t* __restrict__ cells, int64_t n,
                                                       int shift, uint32_t* __restrict__ hist,
                                                       int ntiles, int ncell) {
  __shared__ uint32_t h[kRadixBins];
  for (int b = threadIdx.x; b < kRadixBins; b += kBlock) h[b] = 0;
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * kRadixTile;
  for (int q = 0; q < kRadixItems; ++q) {
    const int64_t idx = t0 + q * kBlock + threadIdx.x;
    if (idx < n) atomicAdd(&h[(load_key(keys, cells, idx, ncell) >> shift) & (kRadixBins - 1)], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kRadixBins; b += kBlock) hist[(int64_t)b * ntiles + blockIdx.x] = h[b];
}

// Generic 3-kernel exclusive scan of a uint32 array (tile sums, scan of the
// tile sums in k_scan_tiles, tile scans plus offsets).
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t* __restrict__ v, int64_t m,
                                                        uint32_t* __restrict__ blk) {
  __shared__ uint32_t wsum[kWaves];
  const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
  uint32_t local = 0;
  for (int q = 0; q < kScanTile / kBlock; ++q) {
    const int64_t i = t0 + q * kBlock + threadIdx.x;
    if (i < m) local += v[i];
  }
  for (int o = 32; o > 0; o >>= 1) local += __shfl_xor(local, o);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = local;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (int w = 0; w < kWaves; ++w) s += wsum[w];
    blk[blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(uint32_t* __restrict__ v, int64_t m,
                                                       const uint32_t* __restrict__ blk) {
  __shared__ uint32_t s[kScanTile];
  const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
  for (int q = 0; q < kScanTile / kBlock; ++q) {
    const int64_t i = t0 + q * kBlock + threadIdx.x;
    s[q * kBlock + threadIdx.x] = i < m ? v[i] : 0u;
  }
  __syncthreads();
  tile_exclusive_scan(s);
  const uint32_t off = blk[blockIdx.x];
  for (int q = 0; q < kScanTile / kBlock; ++q) {
    const int64_t i = t0 + q * kBlock + threadIdx.x;
    if (i < m) v[i] = off + s[q * kBlock + threadIdx.x];
  }
}

// Stable scatter of one digit.  Within a tile the order is item-major:
// element (q, t) is tile[q*kBlock + t], matching the global index order.
__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    const int32_t* __restrict__ cells, int64_t n, int shift, const uint32_t* __restrict__ offs,
    int ntiles, uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, int ncell) {
  __shared__ uint32_t wcnt[kWaves][kRadixBins];
  __shared__ uint32_t run[kRadixBins];
  for (int b = threadIdx.x; b < kRadixBins; b += kBlock)
    run[b] = offs[(int64_t)b * ntiles + blockIdx.x];
  const int64_t t0 = (int64_t)blockIdx.x * kRadixTile;
  for (int q = 0; q < kRadixItems; ++q) {
    const int64_t idx = t0 + q * kBlock + threadIdx.x;
    const bool valid = idx < n;
    uint32_t key = 0, val = 0;
    if (valid) {
      key = load_key(kin, cells, idx, ncell);
      val = vin ? vin[idx] : (uint32_t)idx;
    }
    const uint32_t dst = tile_dest(valid, (key >> shift) & (kRadixBins - 1), wcnt, run);
    if (valid) {
      kout[dst] = key;
      vout[dst] = val;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_radix_final(const uint32_t* __restrict__ keys,
                                                        const uint32_t* __restrict__ perm, int64_t n,
                                                        Fields in, Fields out, int32_t* cs,
                                                        int ncell) {
  gather_fields(keys, perm, n, in, out, cs, ncell, (int64_t)blockIdx.x * kBlock + threadIdx.x,
                (int64_t)gridDim.x * kBlock);
}

// The whole stable sort by one block (fallback of the neighbour path).
__device__ void block_sort(int64_t n, int ncell, Fields in, Fields out, int32_t* cs,
                           uint32_t* const* rkey, uint32_t* const* rval) {
  __shared__ uint32_t wcnt[kWaves][kRadixBins];
  __shared__ uint32_t run[kRadixBins];
  int bits = 0;
  while (bits < 31 && (1ll << bits) < ncell) ++bits;
  const int passes = (bits + kRadixBits - 1) / kRadixBits;
  const uint32_t* kin = nullptr;
  const uint32_t* vin = nullptr;
  int cur = 0;
  for (int pass = 0; pass < passes && n > 0; ++pass) {
    const int shift = pass * kRadixBits;
    for (int b = threadIdx.x; b < kRadixBins; b += blockDim.x) run[b] = 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
      atomicAdd(&run[(load_key(kin, in.cell, i, ncell) >> shift) & (kRadixBins - 1)], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t acc = 0;
      for (int b = 0; b < kRadixBins; ++b) {
        const uint32_t v = run[b];
        run[b] = acc;
        acc += v;
      }
    }
    __syncthreads();
    for (int64_t t0 = 0; t0 < n; t0 += blockDim.x) {
      const int64_t idx = t0 + threadIdx.x;
      const bool valid = idx < n;
      uint32_t key = 0, val = 0;
      if (valid) {
        key = load_key(kin, in.cell, idx, ncell);
        val = vin ? vin[idx] : (uint32_t)idx;
      }
      const uint32_t dst = tile_dest(valid, (key >> shift) & (kRadixBins - 1), wcnt, run);
      if (valid) {
        rkey[cur][dst] = key;
        rval[cur][dst] = val;
      }
    }
    __threadfence();
    __syncthreads();
    kin = rkey[cur];
    vin = rval[cur];
    cur ^= 1;
  }
  gather_fields(kin, vin, n, in, out, cs, ncell, threadIdx.x, blockDim.x);
}

// PERM: write the gather map out.perm[dst] = p instead of moving the fields.
template <int NDIM, bool PERM, bool OPEN = false>
__device__ __forceinline__ void nb_scatter_body(const int32_t* __restrict__ cs_prev, int64_t n,
                                                const SortGeo& g, uint32_t* __restrict__ bases,
                                                const Fields& in, const Fields& out, int32_t* cs,
                                                const Status* st, uint32_t* rk0, uint32_t* rk1,
                                                uint32_t* rv0, uint32_t* rv1, int bid) {
  constexpr int ND = Dirs<NDIM>::N, NB = Dirs<NDIM>::BITS;
  constexpr int CODE_BITS = NB + kScatterCellBits;
  constexpr int NF = PERM ? 0 : 7;        // fields carried through registers
  constexpr int NG = kScatterCells * ND;  // groups of the wavefront
  constexpr int GPL = (NG + 63) / 64;     // groups per lane
  __shared__ uint32_t s_next[kWaves][NG];  // next free slot of each group
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int a0 = (bid * kWaves + wid) * kScatterCells;
  const int na = a0 < g.ncell ? min(kScatterCells, g.ncell - a0) : 0;
  // The far decision, the group bases and the cell bounds are independent:
  // their loads go out together.
  const uint32_t far = __hip_atomic_load(&st->far_decision, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
  uint32_t bv[GPL];
#pragma unroll
  for (int u = 0; u < GPL; ++u) {
    const int q = lane + 64 * u;
    bv[u] = q < na * ND ? bases[(int64_t)a0 * ND + q] : 0u;
  }
  const int bnd = lane <= na ? cs_prev[a0 + lane] : 0;
  // the group bases are used once: the table is left zero for the next
  // counting push
#pragma unroll
  for (int u = 0; u < GPL; ++u) {
    const int q = lane + 64 * u;
    if (q < na * ND) {
      s_next[wid][q] = bv[u];
      bases[(int64_t)a0 * ND + q] = 0u;
    }
  }
  if (far != 0) {
    // open boundaries: the caller takes the general path (info[0])
    if (!OPEN && bid == 0) {
      uint32_t* rkey[2] = {rk0, rk1};
      uint32_t* rval[2] = {rv0, rv1};
      block_sort(n, g.ncell, in, out, cs, rkey, rval);
    }
    return;
  }
  if (na == 0) return;
  {
    const int prev = __shfl_up(bnd, 1);
    const bool bad = lane <= na && (bnd < 0 || bnd > n || (lane > 0 && bnd < prev));
    if (__ballot(bad) != 0) return;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const bool interior = wave_interior<NDIM>(a0, na, g);
  // open: the column of the wave's first cell (an interior wave lies in one row)
  int col0 = 0;
  if (OPEN) {
    int j0, k0;
    ijk(a0, g, col0, j0, k0);
  }
  // positions in unsigned 32 bits: cell_start (and so n) is below 2^31, so
  // a batch's positions (up to 255 past pe) cannot wrap
  const uint32_t pb = (uint32_t)__builtin_amdgcn_readlane(bnd, 0);
  const uint32_t pe = (uint32_t)__builtin_amdgcn_readlane(bnd, na);
  const uint32_t n32 = (uint32_t)n;
  for (uint32_t q0 = pb; q0 < pe; q0 += 64 * kScatterBatches) {
   int keys[kScatterBatches];
   float vals[kScatterBatches][NF > 0 ? NF : 1];
#pragma unroll
   for (int b = 0; b < kScatterBatches; ++b) {
     const uint32_t p = q0 + b * 64 + lane;
     const bool v = p < pe;
     keys[b] = v ? in.cell[p] : 0;
#pragma unroll
     for (int f = 0; f < NF; ++f) vals[b][f] = (v && in.f[f]) ? in.f[f][p] : 0.0f;
   }
#pragma unroll
   for (int b = 0; b < kScatterBatches; ++b) {
    const uint32_t p = q0 + b * 64 + lane;
    const bool valid = p < pe;
    int code = 0;
    const int key = keys[b];
    bool ok = false;
    const int m = cell_in_wave32(p, bnd, na);
    if (valid) {
      int d;
      int iold = col0 + m;
      if (interior) {
        d = direction_interior2d(key, a0 + m, g.nx);
      } else {
        int i, j, k;
        ijk(a0 + m, g, i, j, k);
        d = direction<NDIM>(key, i, j, k, g);
        iold = i;
      }
      ok = d >= 0;
      if (OPEN && ok) {
        // absorbed: the new cell is in a ghost column
        int inew = iold + d % 3 - 1;
        if (inew < 0) inew += g.nx; else if (inew >= g.nx) inew -= g.nx;
        if (inew == 0 || inew == g.nx - 1) ok = false;
      }
      code = (m << NB) | (ok ? d : 0);
    }
    uint64_t bal[CODE_BITS];
    const uint64_t vmask = __ballot(ok);
#pragma unroll
    for (int b = 0; b < CODE_BITS; ++b) bal[b] = __ballot(ok && ((code >> b) & 1));
    const uint64_t mine = match_code<CODE_BITS>(code, vmask, bal);
    const uint64_t before = mine & lanemask_lt();
    const int slot = (code >> NB) * ND + (code & ((1 << NB) - 1));
    uint32_t dst = 0;
    if (ok) dst = s_next[wid][slot] + (uint32_t)__builtin_popcountll(before);
    __builtin_amdgcn_wave_barrier();
    if (ok && before == 0) s_next[wid][slot] += (uint32_t)__builtin_popcountll(mine);
    __builtin_amdgcn_wave_barrier();
    if (ok && dst < n32) {
      if (PERM) {
        out.perm[dst] = (int32_t)p;
      } else {
        out.cell[dst] = key;
#pragma unroll
        for (int f = 0; f < NF; ++f)
          if (in.f[f]) out.f[f][dst] = vals[b][f];
      }
    }
   }
  }
}

template <int NDIM, bool PERM>
__global__ __launch_bounds__(kBlock) void k_nb_scatter(const int32_t* __restrict__ cs_prev, int64_t n,
                                                       SortGeo g, uint32_t* __restrict__ bases,
                                                       Fields in, Fields out, int32_t* cs,
                                                       const Status* st, uint32_t* rk0, uint32_t* rk1,
                                                       uint32_t* rv0, uint32_t* rv1) {
  nb_scatter_body<NDIM, PERM>(cs_prev, n, g, bases, in, out, cs, st, rk0, rk1, rv0, rv1,
                              blockIdx.x);
}

// The open-boundary form (gather map): absorbed ions left out, injected
// ions appended to their cells.
template <int NDIM, int TILE>
__global__ __launch_bounds__(kBlock) void k_nb_newcount_open(const uint32_t* __restrict__ cnt,
                                                             SortGeo g, int32_t* __restrict__ cs,
                                                             uint32_t* __restrict__ blk,
                                                             Status* st, OpenSort os) {
  nb_newcount_body<NDIM, TILE, true>(cnt, g, cs, blk, st, blockIdx.x, os);
}

template <int NDIM, int TILE>
__global__ __launch_bounds__(kBlock) void k_nb_bases_open(uint32_t* __restrict__ cnt, SortGeo g,
                                                          int32_t* __restrict__ cs,
                                                          const uint32_t* __restrict__ blk,
                                                          OpenSort os) {
  nb_bases_body<NDIM, TILE, true>(cnt, g, cs, blk, blockIdx.x, os);
}

template <int NDIM>
__global__ __launch_bounds__(kBlock) void k_nb_scatter_open(const int32_t* __restrict__ cs_prev,
                                                            int64_t n, SortGeo g,
                                                            uint32_t* __restrict__ bases,
                                                            Fields in, Fields out, int32_t* cs,
                                                            const Status* st) {
  nb_scatter_body<NDIM, true, true>(cs_prev, n, g, bases, in, out, cs, st, nullptr, nullptr,
                                    nullptr, nullptr, blockIdx.x);
}

// The gather-map entries of the injected ions (slot r's ions, r over the
// face-major (face, row) pairs, are stored contiguously from
// n_pushed + inj_off[r]) and info[1] = the live count.
__global__ void k_open_inject_perm(const int32_t* __restrict__ inj_cnt,
                                   const int32_t* __restrict__ inj_off,
                                   const int32_t* __restrict__ inj_base, int rows, int64_t n_pushed,
                                   int32_t* __restrict__ perm, const Status* st,
                                   int32_t* __restrict__ info, const int32_t* __restrict__ cs,
                                   int ncell) {
  const uint32_t far = __hip_atomic_load(&st->far_decision, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
  if (far != 0) return;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (inj_cnt && r < rows) {
    const int k = inj_cnt[r], b = inj_base[r];
    const int64_t src = n_pushed + inj_off[r];
    for (int m = 0; m < k; ++m) perm[b + m] = (int32_t)(src + m);
  }
  if (r == 0 && info) info[1] = cs[ncell];
}

// Batched neighbour sort (gather-map form) over the runs of an ensemble:
// per run the arguments of the three passes, per pass one persistent launch.
struct NbArgs {
  const int32_t* cs_prev;
  int64_t n;
  SortGeo g;
  uint32_t* cnt;
  uint32_t* blk;
  Fields in, out;
  int32_t* cs;
  Status* st;
  uint32_t *rk0, *rk1, *rv0, *rv1;
};

__global__ __launch_bounds__(kBlock) void k_nb_newcount_batch(const NbArgs* __restrict__ tab,
                                                              const Item* __restrict__ items,
                                                              int nitems) {
  for_items(nitems, [&](int it) {
    const Item item = items[it];
    const NbArgs A = tab[item.run];
    nb_newcount_body<2, kNbTileSmall>(A.cnt, A.g, A.cs, A.blk, A.st, item.idx);
    __syncthreads();
  });
}

__global__ __launch_bounds__(kBlock) void k_nb_bases_batch(const NbArgs* __restrict__ tab,
                                                           const Item* __restrict__ items,
                                                           int nitems) {
  for_items(nitems, [&](int it) {
    const Item item = items[it];
    const NbArgs A = tab[item.run];
    nb_bases_body<2, kNbTileSmall>(A.cnt, A.g, A.cs, A.blk, item.idx);
    __syncthreads();
  });
}

__global__ __launch_bounds__(kBlock) void k_nb_scatter_batch(const NbArgs* __restrict__ tab,
                                                             const Item* __restrict__ items,
                                                             int nitems) {
  for_items(nitems, [&](int it) {
    const Item item = items[it];
    const NbArgs A = tab[item.run];
    nb_scatter_body<2, true>(A.cs_prev, A.n, A.g, A.cnt, A.in, A.out, A.cs, A.st, A.rk0, A.rk1,
                             A.rv0, A.rv1, item.idx);
    __syncthreads();
  });
}

Fields fields_of(const hvpic_particles* p) {
  Fields f;
  f.cell = p->cell;
  f.f[0] = p->ox;
  f.f[1] = p->oy;
  f.f[2] = p->oz;
  f.f[3] = p->ux;
  f.f[4] = p->uy;
  f.f[5] = p->uz;
  f.f[6] = p->w;
  f.perm = nullptr;
  return f;
}

SortGeo sort_geo(const hvpic_ctx* c) {
  SortGeo g;
  g.nx = c->p.nx;
  g.ny = c->p.ny;
  g.nz = c->p.nz;
  g.ncell = c->ncell;
  g.fnx = c->fnx;
  g.fny = c->fny;
  return g;
}

int radix_bits(int ncell) {
  int b = 0;
  while (b < 31 && (1ll << b) < ncell) ++b;
  return b;
}

// Radix sort by key; keys are the cells, clamped to nkeys - 1 (nkeys = ncell,
// or ncell + 1 where the key ncell marks absorbed ions, which go last);
// cs gets nkeys + 1 entries.
void enqueue_radix(hvpic_ctx* c, const hvpic_particles* in, const Fields& out, int32_t* cs,
                   int nkeys) {
  hipStream_t s = c->stream;
  const int64_t n = in->n;
  const int ncell = nkeys;
  const int ntiles = (int)ceil_div(std::max<int64_t>(n, 1), kRadixTile);
  const int passes = (radix_bits(ncell) + kRadixBits - 1) / kRadixBits;
  const uint32_t* kin = nullptr;
  const uint32_t* vin = nullptr;
  int cur = 0;
  const int64_t m = (int64_t)kRadixBins * ntiles;
  const int mtiles = (int)ceil_div(m, kScanTile);
  uint32_t* blk = (uint32_t*)c->sort_blk;
  for (int pass = 0; pass < passes && n > 0; ++pass) {
    const int shift = pass * kRadixBits;
    hipLaunchKernelGGL(k_radix_hist, dim3(ntiles), dim3(kBlock), 0, s, kin, in->cell, n, shift,
                       c->rhist, ntiles, ncell);
    hipLaunchKernelGGL(k_scan_reduce, dim3(mtiles), dim3(kBlock), 0, s, c->rhist, m, blk);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, blk, mtiles);
    hipLaunchKernelGGL(k_scan_apply, dim3(mtiles), dim3(kBlock), 0, s, c->rhist, m,
                       (const uint32_t*)blk);
    hipLaunchKernelGGL(k_radix_scatter, dim3(ntiles), dim3(kBlock), 0, s, kin, vin, in->cell, n,
                       shift, c->rhist, ntiles, c->rkey[cur], c->rval[cur], ncell);
    kin = c->rkey[cur];
    vin = c->rval[cur];
    cur ^= 1;
  }
  const int fblocks = (int)std::min<int64_t>(ceil_div(n + 1, kBlock), 65536);
  hipLaunchKernelGGL(k_radix_final, dim3(fblocks), dim3(kBlock), 0, s, kin, vin, n, fields_of(in),
                     out, cs, ncell);
}

template <int NDIM>
void enqueue_neighbour(hvpic_ctx* c, const hvpic_particles* in, const Fields& out,
                       const int32_t* cs_prev, int32_t* cs) {
  hipStream_t s = c->stream;
  const SortGeo g = sort_geo(c);
  const int cblocks = (int)ceil_div(c->ncell, kWaves * kCellsPerWave);
  uint32_t* blk = (uint32_t*)c->sort_blk;
  // A counting push of this same store already left the move counts.
  const bool counted = c->cnt_ready && c->cnt_cell == in->cell && c->cnt_cs == cs_prev &&
                       c->cnt_n == in->n;
  if (!counted)
    hipLaunchKernelGGL((k_nb_count<NDIM>), dim3(cblocks), dim3(kBlock), 0, s, in->cell, cs_prev,
                       in->n, g, c->sort_cnt, c->status);
  // small tiles spread the two short passes over more CUs while each block's
  // sum over the preceding tile totals stays short
  if (c->ncell <= kNbTileSmall * 512) {
    const int tiles = (int)ceil_div(c->ncell, kNbTileSmall);
    hipLaunchKernelGGL((k_nb_newcount<NDIM, kNbTileSmall>), dim3(tiles), dim3(kBlock), 0, s,
                       (const uint32_t*)c->sort_cnt, g, cs, blk, c->status);
    hipLaunchKernelGGL((k_nb_bases<NDIM, kNbTileSmall>), dim3(tiles), dim3(kBlock), 0, s,
                       c->sort_cnt, g, cs, (const uint32_t*)blk);
  } else {
    const int tiles = (int)ceil_div(c->ncell, kScanTile);
    hipLaunchKernelGGL((k_nb_newcount<NDIM, kScanTile>), dim3(tiles), dim3(kBlock), 0, s,
                       (const uint32_t*)c->sort_cnt, g, cs, blk, c->status);
    hipLaunchKernelGGL((k_nb_bases<NDIM, kScanTile>), dim3(tiles), dim3(kBlock), 0, s,
                       c->sort_cnt, g, cs, (const uint32_t*)blk);
  }
  timing_begin(c, HVPIC_KERNEL_SORT_SCATTER);
  const int sblocks = (int)ceil_div(c->ncell, kWaves * kScatterCells);
  if (out.perm)
    hipLaunchKernelGGL((k_nb_scatter<NDIM, true>), dim3(sblocks), dim3(kBlock), 0, s, cs_prev, in->n,
                       g, c->sort_cnt, fields_of(in), out, cs, (const Status*)c->status,
                       c->rkey[0], c->rkey[1], c->rval[0], c->rval[1]);
  else
    hipLaunchKernelGGL((k_nb_scatter<NDIM, false>), dim3(sblocks), dim3(kBlock), 0, s, cs_prev,
                       in->n, g, c->sort_cnt, fields_of(in), out, cs, (const Status*)c->status,
                       c->rkey[0], c->rkey[1], c->rval[0], c->rval[1]);
  timing_end(c, HVPIC_KERNEL_SORT_SCATTER);
}

}  // namespace

namespace {

int sort_to(hvpic_ctx* c, const hvpic_particles* in, const Fields& out, const int32_t* cs_prev,
            int32_t* cs, int full) {
  if (full || cs_prev == nullptr) {
    enqueue_radix(c, in, out, cs, c->ncell);
  } else if (c->p.ndim == 2) {
    enqueue_neighbour<2>(c, in, out, cs_prev, cs);
    c->cnt_clean = true;
  } else {
    enqueue_neighbour<3>(c, in, out, cs_prev, cs);
    c->cnt_clean = true;
  }
  c->cnt_ready = false;
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

}  // namespace

int launch_sort(hvpic_ctx* c, const hvpic_particles* in, hvpic_particles* out,
                const int32_t* cs_prev, int32_t* cs, int full) {
  out->n = in->n;
  return sort_to(c, in, fields_of(out), cs_prev, cs, full);
}

int launch_sort_open(hvpic_ctx* c, const hvpic_particles* in, hvpic_particles* out, int32_t* cs) {
  out->n = in->n;
  enqueue_radix(c, in, fields_of(out), cs, c->ncell + 1);
  c->cnt_ready = false;
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

namespace {

template <int NDIM>
void enqueue_sort_open_perm(hvpic_ctx* c, const hvpic_particles* in, int64_t n_pushed,
                            const int32_t* cs_prev, int32_t* perm, int32_t* cs, int32_t* info,
                            const int32_t* inj_cnt, const int32_t* inj_off, int32_t* inj_base,
                            int rows) {
  hipStream_t s = c->stream;
  const SortGeo g = sort_geo(c);
  uint32_t* blk = (uint32_t*)c->sort_blk;
  const bool counted = c->cnt_ready && c->cnt_cell == in->cell && c->cnt_cs == cs_prev &&
                       c->cnt_n == n_pushed;
  if (!counted) {
    const int cblocks = (int)ceil_div(c->ncell, kWaves * kCellsPerWave);
    hipLaunchKernelGGL((k_nb_count<NDIM>), dim3(cblocks), dim3(kBlock), 0, s, in->cell, cs_prev,
                       n_pushed, g, c->sort_cnt, c->status);
  }
  const OpenSort os{inj_cnt, inj_base, info, rows};
  if (c->ncell <= kNbTileSmall * 512) {
    const int tiles = (int)ceil_div(c->ncell, kNbTileSmall);
    hipLaunchKernelGGL((k_nb_newcount_open<NDIM, kNbTileSmall>), dim3(tiles), dim3(kBlock), 0, s,
                       (const uint32_t*)c->sort_cnt, g, cs, blk, c->status, os);
    hipLaunchKernelGGL((k_nb_bases_open<NDIM, kNbTileSmall>), dim3(tiles), dim3(kBlock), 0, s,
                       c->sort_cnt, g, cs, (const uint32_t*)blk, os);
  } else {
    const int tiles = (int)ceil_div(c->ncell, kScanTile);
    hipLaunchKernelGGL((k_nb_newcount_open<NDIM, kScanTile>), dim3(tiles), dim3(kBlock), 0, s,
                       (const uint32_t*)c->sort_cnt, g, cs, blk, c->status, os);
    hipLaunchKernelGGL((k_nb_bases_open<NDIM, kScanTile>), dim3(tiles), dim3(kBlock), 0, s,
                       c->sort_cnt, g, cs, (const uint32_t*)blk, os);
  }
  Fields out{};
  out.perm = perm;
  timing_begin(c, HVPIC_KERNEL_SORT_SCATTER);
  const int sblocks = (int)ceil_div(c->ncell, kWaves * kScatterCells);
  hipLaunchKernelGGL(k_nb_scatter_open<NDIM>, dim3(sblocks), dim3(kBlock), 0, s, cs_prev, in->n,
                     g, c->sort_cnt, fields_of(in), out, cs, (const Status*)c->status);
  timing_end(c, HVPIC_KERNEL_SORT_SCATTER);
  hipLaunchKernelGGL(k_open_inject_perm, dim3((unsigned)ceil_div(2 * rows, 256)), dim3(256), 0, s,
                     inj_cnt, inj_off, (const int32_t*)inj_base, 2 * rows, n_pushed, perm,
                     (const Status*)c->status, info, (const int32_t*)cs, c->ncell);
}

}  // namespace

int launch_sort_open_perm(hvpic_ctx* c, const hvpic_particles* in, int64_t n_pushed,
                          const int32_t* cs_prev, int32_t* perm, int32_t* cs, int32_t* info,
                          const int32_t* inj_cnt, const int32_t* inj_off, int32_t* inj_base) {
  const int rows = c->p.ny * (c->p.ndim == 3 ? c->p.nz : 1);
  if (c->p.ndim == 3)
    enqueue_sort_open_perm<3>(c, in, n_pushed, cs_prev, perm, cs, info, inj_cnt, inj_off,
                              inj_base, rows);
  else
    enqueue_sort_open_perm<2>(c, in, n_pushed, cs_prev, perm, cs, info, inj_cnt, inj_off,
                              inj_base, rows);
  c->cnt_clean = true;
  c->cnt_ready = false;
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

int launch_sort_perm(hvpic_ctx* c, const hvpic_particles* in, const int32_t* cs_prev,
                     int32_t* perm, int32_t* cs) {
  Fields out{};
  out.perm = perm;
  return sort_to(c, in, out, cs_prev, cs, 0);
}

size_t ens_sort_record(hvpic_ctx* c, const hvpic_particles* in, const int32_t* cs_prev,
                       int32_t* perm, int32_t* cs, void* dst) {
  if (dst) {
    NbArgs A;
    A.cs_prev = cs_prev;
    A.n = in->n;
    A.g = sort_geo(c);
    A.cnt = c->sort_cnt;
    A.blk = (uint32_t*)c->sort_blk;
    A.in = fields_of(in);
    A.out = Fields{};
    A.out.perm = perm;
    A.cs = cs;
    A.st = c->status;
    A.rk0 = c->rkey[0];
    A.rk1 = c->rkey[1];
    A.rv0 = c->rval[0];
    A.rv1 = c->rval[1];
    memcpy(dst, &A, sizeof(A));
  }
  return sizeof(NbArgs);
}

int ens_sort_tiles(const hvpic_ctx* c) { return (int)ceil_div(c->ncell, kNbTileSmall); }
int ens_sort_scatter_blocks(const hvpic_ctx* c) {
  return (int)ceil_div(c->ncell, kWaves * kScatterCells);
}
bool ens_sort_fits(const hvpic_ctx* c) { return c->ncell <= kNbTileSmall * 512; }

int ens_launch_sort(hipStream_t s, int pass, const void* tab, const Item* items, int nitems,
                    int grid) {
  if (nitems == 0) return HVPIC_OK;
  const NbArgs* t = static_cast<const NbArgs*>(tab);
  if (pass == 0)
    hipLaunchKernelGGL(k_nb_newcount_batch, dim3(grid), dim3(kBlock), 0, s, t, items, nitems);
  else if (pass == 1)
    hipLaunchKernelGGL(k_nb_bases_batch, dim3(grid), dim3(kBlock), 0, s, t, items, nitems);
  else
    hipLaunchKernelGGL(k_nb_scatter_batch, dim3(grid), dim3(kBlock), 0, s, t, items, nitems);
  return hipGetLastError() == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
}

}  // namespace hvpic
