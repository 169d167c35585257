// Internal declarations of libhvpic.so (gfx950).  Not part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hvpic.h"

namespace hvpic {

constexpr int kBlock = 256;      // threads per block for particle kernels

// Unsigned division by a runtime constant: q = mulhi(n, m) is floor(n/d) or
// one less, fixed by one compare.  Valid for n < 2^32.
struct FastDiv {
  uint32_t d, m;
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  f.m = d == 1 ? 0xFFFFFFFFu : (uint32_t)((1ull << 32) / d);
  return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv f) {
  uint32_t q = __umulhi(n, f.m);
  if (n - q * f.d >= f.d) ++q;
  return q;
}

// Device-side status block (first bytes of the workspace).
struct Status {
  uint32_t flags;
  uint32_t pad;
  unsigned long long moved_gt1;
  unsigned long long nonfinite;
  unsigned long long floor_hits;
  unsigned long long bad_input;
  uint32_t far_flag;        // set by the neighbour-move count kernel on a far mover
  uint32_t far_decision;    // far_flag handed to the scatter kernel (and far_flag cleared)
  // blocks of the particle kernels (push, deposit) that used the LDS windows
  // and that fell back to global loads and atomics (hvpic_path_stats)
  unsigned long long win_blocks;
  unsigned long long glob_blocks;
  // the surrogate field advance: 1 if the last proposal passed its residual
  // test (read by the kernels of the fallback and of the acceptance)
  uint32_t no_accept;
  uint32_t no_pad;
};

// One count per block of a particle kernel: whether it used the LDS windows.
__device__ __forceinline__ void count_path(Status* st, bool window) {
  if (threadIdx.x == 0) atomicAdd(window ? &st->win_blocks : &st->glob_blocks, 1ull);
}

// One work item of a batched launch over the runs of an ensemble: block idx
// of the nb blocks that run `run`'s share of the launch would take on its own.
struct Item {
  int32_t run, idx, nb;
};

// Calls f(it) for the items this block takes of a persistent launch over
// nitems items (gridDim.x a multiple of 8).  The GPU hands blocks out
// round-robin over its 8 XCDs, each with its own L2, so XCD x takes the
// contiguous x-th eighth of the item list (neighbouring chunks of one run
// share an L2) and its blocks stride through it.
template <class F>
__device__ __forceinline__ void for_items(int nitems, F f) {
  const int x = blockIdx.x & 7, l = blockIdx.x >> 3, g8 = gridDim.x >> 3;
  const int per = nitems >> 3, rem = nitems & 7;
  const int start = x * per + (x < rem ? x : rem), len = per + (x < rem ? 1 : 0);
  for (int j = l; j < len; j += g8) f(start + j);
}

// FP64 partial sums of NV values over a block, written by thread 0 to
// part[slot * STRIDE + k] (slot = blockIdx.x by default).  Fixed reduction
// order (deterministic).
template <int NV, int STRIDE = 4>
__device__ void block_partial(double* v, double* part, int64_t slot) {
  __shared__ double s_red[16][NV];
#pragma unroll
  for (int k = 0; k < NV; ++k)
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o);
  const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < NV; ++k) s_red[wid][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < NV; ++k) {
      double t = 0.0;
      for (int w = 0; w < nw; ++w) t += s_red[w][k];
      part[slot * STRIDE + k] = t;
    }
}

template <int NV, int STRIDE = 4>
__device__ void block_partial(double* v, double* part) {
  block_partial<NV, STRIDE>(v, part, blockIdx.x);
}

// Sum of nblocks partials (as written by block_partial) by one block, in a
// fixed order; thread 0 returns the totals in res.
template <int NV, int STRIDE = 4>
__device__ void sum_partials(const double* part, int nblocks, double* res) {
  __shared__ double s_red[16][NV];
  double t[NV];
  for (int k = 0; k < NV; ++k) t[k] = 0.0;
  // eight independent loads in flight per thread and step
  const int stride = blockDim.x;
  for (int b0 = threadIdx.x; b0 < nblocks; b0 += 8 * stride) {
    double v[8][NV];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int b = b0 + u * stride;
      for (int k = 0; k < NV; ++k) v[u][k] = b < nblocks ? part[(int64_t)b * STRIDE + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      for (int k = 0; k < NV; ++k) t[k] += v[u][k];
  }
  for (int k = 0; k < NV; ++k)
    for (int o = 32; o > 0; o >>= 1) t[k] += __shfl_xor(t[k], o);
  const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < NV; ++k) s_red[wid][k] = t[k];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < NV; ++k) {
      double r = 0.0;
      for (int w = 0; w < nw; ++w) r += s_red[w][k];
      res[k] = r;
    }
}

// Canonical move in {-1, 0, 1} between two indices along a periodic axis of
// n cells (delta = new - old), or 2 for a longer move.  Shared by the push
// (which counts moves for the sort) and the sort, so both classify alike.
__device__ __forceinline__ int canon_move(int delta, int n) {
  const int r = delta < 0 ? delta + n : delta;
  if (r == 0) return 0;
  if (r == 1) return 1;
  if (r == n - 1) return -1;
  return 2;
}

__device__ __forceinline__ void raise_flag(Status* st, uint32_t bit, unsigned long long* counter) {
  atomicOr(&st->flags, bit);
  if (counter) atomicAdd(counter, 1ull);
}

}  // namespace hvpic

// The context (opaque to C callers).
struct hvpic_ctx {
  hvpic_params p;
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  int32_t ncell;
  int32_t magic;
  // derived constants (FP32 as the kernels use them)
  float a;           // (qs/ms) dt / 2
  float kx, ky, kz;  // 2 dt / (dx, dy, dz): half-cells per unit speed per step
  float qV;          // qs / V_c
  hvpic::FastDiv fnx, fny;
  // workspace carve-out
  hvpic::Status* status;
  double* push_part;     // per-block FP64 partials of the push diagnostics [blocks][4]
  double* field_part;    // per-block FP64 partials of the field diagnostics [slots][8]
  uint32_t* sort_cnt;    // [ncell][3^ndim]
  int32_t* sort_blk;     // scan block sums
  uint32_t* rkey[2];     // radix keys   [np_capacity]
  uint32_t* rval[2];     // radix values [np_capacity]
  uint32_t* rhist;       // radix per-block digit counts
  float* fscratch;       // field scratch [20][ncell]
  double* mom_acc;       // FP64 moment accumulators [4][ncell], kept at zero between deposits
  // Move counts left in sort_cnt by a counting push, valid for the next
  // neighbour-move sort of the same store (cell array, cell_start, size).
  bool cnt_ready;
  bool cnt_clean;  // sort_cnt is all zero (a counting push needs that)
  const int32_t* cnt_cell;
  const int32_t* cnt_cs;
  int64_t cnt_n;
  // open boundaries: per face row the injected count, its offset within
  // the injected block and the first slot in the sorted order [3][2][ny nz]
  int32_t* open_rows;
  // 3D: the order in which the push takes its chunks [chunks + 1] and its
  // per-row workspace, or null
  int32_t* chunk_order;
  // the last injection: the store it appended to, its size before, count
  const int32_t* inj_cell;
  int64_t inj_n0, inj_k;
  // optional per-kernel timing: event pairs [kernel][slot][2]
  hipEvent_t* tev;
  int tmax;
  int tevery;                            // time launch 0, tevery, 2 tevery, ...
  int tcount[HVPIC_KERNEL_COUNT];        // timed launches
  int64_t tseen[HVPIC_KERNEL_COUNT];     // launches since enable / read
  bool tarmed[HVPIC_KERNEL_COUNT];       // the current launch has its begin event
};

namespace hvpic {

constexpr int32_t kMagic = 0x68767063;

// Launch wrappers, one per kernel family (implemented next to the kernels).
int launch_gather_push(hvpic_ctx* c, hvpic_particles* p, const int32_t* cell_start,
                       const float* E, const float* B, float* n_mid, float* J_mid,
                       double* diag_out);
int launch_gather_push_perm(hvpic_ctx* c, const hvpic_particles* in, const int32_t* perm,
                            hvpic_particles* out, const int32_t* cell_start, const float* E,
                            const float* B, float* n_mid, float* J_mid, double* diag_out);
int launch_gather_push_select(hvpic_ctx* c, const hvpic_particles* in, int64_t n_map,
                              const int32_t* perm, hvpic_particles* out,
                              const int32_t* cell_start, const float* E, const float* B,
                              float* n_mid, float* J_mid, double* diag_out);
int launch_deposit(hvpic_ctx* c, const hvpic_particles* p, const int32_t* cell_start,
                   float half_dt_back, float* n, float* J);
int launch_sort(hvpic_ctx* c, const hvpic_particles* in, hvpic_particles* out,
                const int32_t* cs_prev, int32_t* cs, int full);
int launch_sort_open(hvpic_ctx* c, const hvpic_particles* in, hvpic_particles* out, int32_t* cs);
int launch_sort_open_perm(hvpic_ctx* c, const hvpic_particles* in, int64_t n_pushed,
                          const int32_t* cs_prev, int32_t* perm, int32_t* cs, int32_t* info,
                          const int32_t* inj_cnt, const int32_t* inj_off, int32_t* inj_base);
int launch_sort_perm(hvpic_ctx* c, const hvpic_particles* in, const int32_t* cs_prev,
                     int32_t* perm, int32_t* cs);
int launch_field_advance(hvpic_ctx* c, float* B, const float* n_half, const float* J_half,
                         const float* n_prev, const float* J_prev, float* E_out, int mode,
                         double* diag_out);
// With hyper-resistivity and/or the energy equation (pe non-null): the
// stencil-per-stage path of fields_ext.hip.
int launch_field_advance_ext(hvpic_ctx* c, float* B, float* pe, const float* n_half,
                             const float* J_half, const float* n_prev, const float* J_prev,
                             float* E_out, int mode, double* diag_out);
int launch_eos_pressure(hvpic_ctx* c, const float* n, float* pe);
// The surrogate field advance (2D, mode 0): residual test of the proposal
// Bno, the plain subcycle as the fallback, then E, B and the diagnostics;
// stats (device, may be null) <- {residual ratio, accepted}.
int launch_field_advance_no(hvpic_ctx* c, float* B, const float* n_half, const float* J_half,
                            const float* n_prev, const float* J_prev, float* E_out,
                            double* diag_out, const float* Bno, float tol, double* stats);
// the operator's proposal for one sample (surrogate.hip)
size_t no_params_bytes();
int no_predict(hipStream_t s, const void* params, void* ws, int nx, int ny, const float* B,
               const float* n, const float* J, float* B_out);
int launch_smooth(hvpic_ctx* c, float* F, int ncomp, int npasses);

// Ensemble support: per-run argument records of the batched kernels, built on
// the host into `dst` (returning the record size; dst may be null to ask
// it), and the batched launches over work items (tables and items in device
// memory, grid a multiple of 8).  2D, gather-map sequence, fused deposit.
size_t ens_push_record(hvpic_ctx* c, const hvpic_particles* in, const int32_t* perm,
                       hvpic_particles* out, const int32_t* cs, const float* E, const float* B,
                       bool diag, void* dst);
size_t ens_moments_record(hvpic_ctx* c, float* n, float* J, int nparts, double* diag_out,
                          void* dst);
int ens_moment_blocks(const hvpic_ctx* c);
int ens_launch_push(hipStream_t s, int shape, int ppt, const void* tab, const Item* items,
                    int nitems, int grid);
int ens_launch_moments(hipStream_t s, const void* tab, const Item* items, int nitems, int grid);
size_t ens_sort_record(hvpic_ctx* c, const hvpic_particles* in, const int32_t* cs_prev,
                       int32_t* perm, int32_t* cs, void* dst);
int ens_sort_tiles(const hvpic_ctx* c);          // items of passes 0 and 1
int ens_sort_scatter_blocks(const hvpic_ctx* c); // items of pass 2
bool ens_sort_fits(const hvpic_ctx* c);          // the batched sort's tile size suits the grid
int ens_launch_sort(hipStream_t s, int pass, const void* tab, const Item* items, int nitems,
                    int grid);
constexpr int kTileShapes = 3;  // 2D subcycle tiles: 0 = 32x8, 1 = 16x16, 2 = 64x4
int ens_field_tiles(const hvpic_ctx* c, int shape);
// tile launches of a field advance; per launch its substeps K, whether it
// reads a lo part and whether it is the final one (arrays of >= 64 or null)
int ens_field_launches(const hvpic_ctx* c, int* K, int* has_lin, int* fin);
size_t ens_field_record(hvpic_ctx* c, float* B, const float* n_half, const float* J_half,
                        const float* n_prev, const float* J_prev, float* E_out, bool diag,
                        int launch, int shape, void* dst);
size_t ens_field_diag_record(hvpic_ctx* c, double* out, int shape, void* dst);
int ens_launch_field(hipStream_t s, int shape, int K, int has_lin, int fin, const void* tab,
                     const Item* items, int nitems, int grid);
int ens_launch_field_diag(hipStream_t s, const void* tab, int nruns);
// particles per chunk of the 2D push for ppt particles per lane
constexpr int ens_chunk(int ppt) { return 256 * ppt; }
// Per-block partial slots the field diagnostics need (the larger of the
// output kernel's blocks and the 2D subcycle's tiles); kFieldPartStride
// doubles each.
int64_t field_part_slots(const hvpic_params* p);
constexpr int kFieldPartStride = 8;
int launch_zero(hvpic_ctx* c, float* p, int64_t count);
bool params_valid(const hvpic_params* p);  // the checks hvpic_init applies
void zero_counts(hvpic_ctx* c);  // enqueues the clearing of sort_cnt

// Event bracket around one launch of kernel id k (no-op unless timing is on
// and the launch is one of the sampled ones).
inline void timing_begin(hvpic_ctx* c, int k) {
  c->tarmed[k] = false;
  if (!c->tev || c->tcount[k] >= c->tmax) return;
  const bool take = c->tseen[k] % c->tevery == 0;
  ++c->tseen[k];
  if (!take) return;
  (void)hipEventRecord(c->tev[((int64_t)k * c->tmax + c->tcount[k]) * 2], c->stream);
  c->tarmed[k] = true;
}
inline void timing_end(hvpic_ctx* c, int k) {
  if (!c->tarmed[k]) return;
  (void)hipEventRecord(c->tev[((int64_t)k * c->tmax + c->tcount[k]) * 2 + 1], c->stream);
  ++c->tcount[k];
  c->tarmed[k] = false;
}
int launch_init_workspace(hvpic_ctx* c);

// Workspace layout (bytes from the start; each region 256-byte aligned).
struct Layout {
  size_t status, push_part, field_part, sort_cnt, sort_blk, rkey0, rkey1, rval0, rval1, rhist,
      fscratch, mom_acc, open_rows, chunk_order, total;
};
Layout workspace_layout(const hvpic_params* p);

constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kRadixItems = 8;  // keys per thread per radix tile
constexpr int kRadixTile = kBlock * kRadixItems;
constexpr int kScanTile = 2048;  // elements per block of the prefix scans
constexpr int kNbTileSmall = 512;  // cells per block of the neighbour sort's scans (small grids)
constexpr int kChunk3 = 1024;      // ions per block of the 3D push

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace hvpic
