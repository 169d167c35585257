// C-ABI entry points of libhvpic.so: argument validation, the context and the
// workspace layout.  Every compute step runs in the kernels of particles.hip,
// sort.hip and fields.hip on the context's stream.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "hvpic_internal.hpp"

namespace hvpic {
namespace {

bool finite_pos(double x) { return isfinite(x) && x > 0.0; }

bool params_ok(const hvpic_params* p) {
  if (!p) return false;
  if (p->ndim != 2 && p->ndim != 3) return false;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return false;
  if (p->ndim == 2 && p->nz != 1) return false;
  const int64_t nc = (int64_t)p->nx * p->ny * p->nz;
  if (nc >= (1ll << 31) - 1) return false;
  if (!finite_pos(p->dx) || !finite_pos(p->dy) || !finite_pos(p->dz) || !finite_pos(p->dt))
    return false;
  if (p->nsub < 0 || p->nsmooth < 0) return false;
  if (p->shape != HVPIC_SHAPE_NGP && p->shape != HVPIC_SHAPE_QS) return false;
  if (!isfinite(p->qs) || !finite_pos(p->ms)) return false;
  if (!isfinite(p->te) || p->te < 0.0 || !finite_pos(p->gamma_e) || !finite_pos(p->n0) ||
      !finite_pos(p->n_floor))
    return false;
  if (!isfinite(p->eta) || p->eta < 0.0) return false;
  if (!isfinite(p->eta_h) || p->eta_h < 0.0) return false;
  if (p->energy_eq != 0 && p->energy_eq != 1) return false;
  if (p->energy_eq && !(p->gamma_e > 1.0)) return false;  // W_e = sum p V/(gamma-1)
  if (!isfinite(p->kappa0) || p->kappa0 < 0.0) return false;
  if (p->open_x != 0 && p->open_x != 1) return false;
  if (p->open_x && p->nx < 3) return false;
  if (p->buffer_cells < 0 || !isfinite(p->eta_h_buffer) || p->eta_h_buffer < 0.0) return false;
  if (p->np_capacity < 0 || p->np_capacity >= (1ll << 31) - 1) return false;
  return true;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool parts_ok(const hvpic_ctx* c, const hvpic_particles* q, bool need_w) {
  if (!q || q->n < 0 || q->n > c->p.np_capacity) return false;
  if (q->n == 0) return true;
  if (!q->cell || !q->ox || !q->oy || !q->ux || !q->uy || !q->uz) return false;
  if (need_w && !q->w) return false;
  if (c->p.ndim == 3 && !q->oz) return false;
  return true;
}

bool ctx_ok(const hvpic_ctx* c) { return c && c->magic == kMagic; }

}  // namespace

bool params_valid(const hvpic_params* p) { return params_ok(p); }

namespace {

__global__ void k_init_ws(Status* st, double* mom, int64_t nmom, uint32_t* cnt, int64_t ncnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t q = i; q < nmom; q += (int64_t)gridDim.x * blockDim.x) mom[q] = 0.0;
  for (int64_t q = i; q < ncnt; q += (int64_t)gridDim.x * blockDim.x) cnt[q] = 0u;
  if (i == 0) {
    st->flags = 0;
    st->moved_gt1 = st->nonfinite = st->floor_hits = st->bad_input = 0;
    st->far_flag = 0;
    st->far_decision = 0;
    st->win_blocks = st->glob_blocks = 0;
  }
}

__global__ void k_clear_paths(Status* st) {
  if (threadIdx.x == 0) st->win_blocks = st->glob_blocks = 0;
}

__global__ void k_clear_status(Status* st) {
  if (threadIdx.x == 0) {
    st->flags = 0;
    st->moved_gt1 = st->nonfinite = st->floor_hits = st->bad_input = 0;
  }
}

}  // namespace

Layout workspace_layout(const hvpic_params* p) {
  Layout L;
  const int64_t nc = (int64_t)p->nx * p->ny * p->nz;
  const int64_t cap = std::max<int64_t>(p->np_capacity, 1);
  const int ndir = p->ndim == 2 ? 9 : 27;
  const int64_t ntiles = ceil_div(cap, kRadixTile);
  const int64_t nblk = std::max(ceil_div(nc, kNbTileSmall), ceil_div(kRadixBins * ntiles, kScanTile)) + 1;
  size_t off = 0;
  L.status = off;    off += align256(sizeof(Status));
  // per-block partials: particle-chunk blocks (>= 1024 particles each) or
  // cell-row blocks (>= 16 cells each)
  L.push_part = off;
  off += align256(sizeof(double) * 4 * std::max(ceil_div(cap, 1024), ceil_div(nc, 16)));
  L.field_part = off; off += align256(sizeof(double) * kFieldPartStride * field_part_slots(p));
  L.sort_cnt = off;  off += align256(sizeof(uint32_t) * ndir * nc);
  L.sort_blk = off;  off += align256(sizeof(uint32_t) * nblk);
  L.rkey0 = off;     off += align256(sizeof(uint32_t) * cap);
  L.rkey1 = off;     off += align256(sizeof(uint32_t) * cap);
  L.rval0 = off;     off += align256(sizeof(uint32_t) * cap);
  L.rval1 = off;     off += align256(sizeof(uint32_t) * cap);
  L.rhist = off;     off += align256(sizeof(uint32_t) * kRadixBins * ntiles);
  L.fscratch = off;  off += align256(sizeof(float) * 25 * nc);
  L.mom_acc = off;   off += align256(sizeof(double) * 4 * nc);
  L.open_rows = off;
  off += align256(p->open_x ? sizeof(int32_t) * 3 * 2 * (size_t)p->ny * (size_t)p->nz : 0);
  L.chunk_order = off;
  // the order, then per grid row (j, k) F, K, P and one decision word
  off += align256(p->ndim == 3 ? sizeof(int32_t) * (size_t)(ceil_div(cap, kChunk3) + 1 +
                                                           3 * (int64_t)p->ny * p->nz + 1)
                               : 0);
  L.total = off;
  return L;
}

}  // namespace hvpic

using namespace hvpic;

extern "C" {

int hvpic_workspace_bytes(const hvpic_params* params, size_t* bytes) {
  if (!params_ok(params) || !bytes) return HVPIC_EINVAL;
  *bytes = workspace_layout(params).total;
  return HVPIC_OK;
}

int hvpic_init(const hvpic_params* params, void* hip_stream, void* workspace, hvpic_ctx** out) {
  if (!params_ok(params) || !workspace || !out) return HVPIC_EINVAL;
  if (((uintptr_t)workspace & 255) != 0) return HVPIC_EINVAL;
  hvpic_ctx* c = new (std::nothrow) hvpic_ctx;
  if (!c) return HVPIC_ENOMEM;
  memset(c, 0, sizeof(*c));
  c->p = *params;
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)workspace;
  const Layout L = workspace_layout(params);
  c->ws_bytes = L.total;
  c->ncell = params->nx * params->ny * params->nz;
  c->magic = kMagic;
  const double qm = params->qs / params->ms;
  c->a = (float)(0.5 * qm * params->dt);
  c->kx = (float)(2.0 * params->dt / params->dx);
  c->ky = (float)(2.0 * params->dt / params->dy);
  c->kz = (float)(2.0 * params->dt / params->dz);
  c->qV = (float)(params->qs / (params->dx * params->dy * params->dz));
  c->fnx = make_fastdiv((uint32_t)params->nx);
  c->fny = make_fastdiv((uint32_t)params->ny);
  c->status = (Status*)(c->ws + L.status);
  c->push_part = (double*)(c->ws + L.push_part);
  c->field_part = (double*)(c->ws + L.field_part);
  c->sort_cnt = (uint32_t*)(c->ws + L.sort_cnt);
  c->sort_blk = (int32_t*)(c->ws + L.sort_blk);
  c->rkey[0] = (uint32_t*)(c->ws + L.rkey0);
  c->rkey[1] = (uint32_t*)(c->ws + L.rkey1);
  c->rval[0] = (uint32_t*)(c->ws + L.rval0);
  c->rval[1] = (uint32_t*)(c->ws + L.rval1);
  c->rhist = (uint32_t*)(c->ws + L.rhist);
  c->fscratch = (float*)(c->ws + L.fscratch);
  c->mom_acc = (double*)(c->ws + L.mom_acc);
  c->open_rows = params->open_x ? (int32_t*)(c->ws + L.open_rows) : nullptr;
  c->chunk_order = params->ndim == 3 ? (int32_t*)(c->ws + L.chunk_order) : nullptr;
  hipLaunchKernelGGL(k_init_ws, dim3(256), dim3(256), 0, c->stream, c->status, c->mom_acc,
                     4ll * c->ncell, c->sort_cnt,
                     (int64_t)c->ncell * (params->ndim == 2 ? 9 : 27));
  c->cnt_clean = true;
  if (hipGetLastError() != hipSuccess) {
    delete c;
    return HVPIC_EHIP;
  }
  *out = c;
  return HVPIC_OK;
}

int hvpic_finalize(hvpic_ctx* ctx) {
  if (!ctx_ok(ctx)) return HVPIC_ESTATE;
  hvpic_timing_enable(ctx, 0, 1);
  ctx->magic = 0;
  delete ctx;
  return HVPIC_OK;
}

int hvpic_gather_push(hvpic_ctx* ctx, hvpic_particles* p, const int32_t* cell_start,
                      const float* E, const float* B, float* n_mid, float* J_mid,
                      double* diag_out) {
  if (!ctx_ok(ctx)) return HVPIC_ESTATE;
  const bool need_w = (n_mid && J_mid) || diag_out;
  if (!parts_ok(ctx, p, need_w) || !E || !B) return HVPIC_EINVAL;
  if ((n_mid == nullptr) != (J_mid == nullptr)) return HVPIC_EINVAL;
  return launch_gather_push(ctx, p, cell_start, E, B, n_mid, J_mid, diag_out);
}

int hvpic_gather_push_perm(hvpic_ctx* ctx, const hvpic_particles* in, const int32_t* perm,
                           hvpic_particles* out, const int32_t* cell_start, const float* E,
                           const float* B, float* n_mid, float* J_mid, double* diag_out) {
  if (!ctx_ok(ctx)) return HVPIC_ESTATE;
  if (!parts_ok(ctx, in, true) || !out || !E || !B) return HVPIC_EINVAL;
  if ((n_mid == nullptr) != (J_mid == nullptr)) return HVPIC_EINVAL;
  if (in->n > 0) {
    if (!perm || !out->cell || !out->ox || !out->oy || !out->ux || !out->uy || !out->uz ||
        !out->w)
      return HVPIC_EINVAL;
    if (ctx->p.ndim == 3 && !out->oz) return HVPIC_EINVAL;
    if (out->cell == in->cell || out->ox == in->ox || out->ux == in->ux || out->w == in->w)
      return HVPIC_EINVAL;
  }
  return launch_gather_push_perm(ctx, in, perm, out, cell_start, E, B, n_mid, J_mid, diag_out);
}
int hvpic_gather_push_select(hvpic_ctx* ctx, const hvpic_particles* in, int64_t n_map,
                             const int32_t* perm, hvpic_particles* out,
                             const int32_t* cell_start, const float* E, const float* B,
                             float* n_mid, float* J_mid, double* diag_out) {
  if (!ctx_ok(ctx)) return HVPIC_ESTATE;
  if (!parts_ok(ctx, in, true) || !out || !E || !B) return HVPIC_EINVAL;
  if (n_map < 0 || n_map > in->n) return HVPIC_EINVAL;
  if ((n_mid == nullptr) != (J_mid == nullptr)) return HVPIC_EINVAL;
  if (n_map > 0) {
    if (!perm || !out->cell || !out->ox || !out->oy || !out->ux || !out->uy || !out->uz ||
        !out->w)
      return HVPIC_EINVAL;
    if (ctx->p.ndim == 3 && !out->oz) return HVPIC_EINVAL;
    if (out->cell == in->cell || out->ox == in->ox || out->ux == in->ux || out->w == in->w)
      return HVPIC_EINVAL;
  }
  return launch_gather_push_select(ctx, in, n_map, perm, out, cell_start, E, B, n_mid, J_mid,
                                   diag_out);
}
int hvpic_sort_perm(hvpic_ctx* ctx, const hvpic_particles* in, const int32_t* cell_start_prev,
                    int32_t* perm, int32_t* cell_start) {
  if (!ctx_ok(ctx)) return HVPIC_ESTATE;
  if (!parts_ok(ctx, in, false) || !cell_start) return HVPIC_EINVAL;
  if (in->n > 0 && !perm) return HVPIC_EINVAL;
  return launch_sort_perm(ctx, in, cell_start_prev, perm, cell_start);
}
int hvpic_sort(hvpic_ctx* ctx, const hvpic_particles* in, hvpic_particles* out,
               const int32_t* cell_start_prev, int32_t* cell_start, int full) {
  if (!ctx_ok(ctx)) return HVPIC_ESTATE;
  if (!parts_ok(ctx, in, true) || !out || !cell_start) return HVPIC_EINVAL;
  if (in->n > 0) {
    if (!out->cell || !out->ox || !out->oy || !out->ux || !out->uy || !out->uz || !out->w)
      return HVPIC_EINVAL;
    if (ctx->p.ndim == 3 && !out->oz) return HVPIC_EINVAL;
    if (out->cell == in->cell || out->ox == in->ox || out->ux == in->ux || out->w == in->w)
      return HVPIC_EINVAL;
  }
  return launch_sort(ctx, in, out, cell_start_prev, cell_start, full);
}

int hvpic_sort_open(hvpic_ctx* ctx, const hvpic_particles* in, hvpic_particles* out,
                    int32_t* cell_start) {
  if (!ctx_ok(ctx)) return HVPIC_ESTATE;
  if (!ctx->p.open_x) return HVPIC_EINVAL;
  if (!parts_ok(ctx, in, true) || !out || !cell_start) return HVPIC_EINVAL;
  if (in->n > 0) {
    if (!out->cell || !out->ox || !out->oy || !out->ux || !out->uy || !out->uz || !out->w)
      return HVPIC_EINVAL;
    if (out->cell == in->cell || out->ox == in->ox || out->ux == in->ux || out->w == in->w)
      return HVPIC_EINVAL;
  }
  return launch_sort_open(ctx, in, out, cell_start);
}

int hvpic_deposit(hvpic_ctx* ctx, const hvpic_particles* p, const int32_t* cell_start,
                  float half_dt_back, float* n, float* J) {
  if (!ctx_ok(ctx)) return HVPIC_ESTATE;
  if (!parts_ok(ctx, p, true) || !n || !J || !isfinite(half_dt_back)) return HVPIC_EINVAL;
  return launch_deposit(ctx, p, cell_start, half_dt_back, n, J);
}

int hvpic_field_advance(hvpic_ctx* ctx, float* B, const float* n_half, const float* J_half,
                        const float* n_prev, const float* J_prev, float* E_out, int mode,
                        double* diag_out) {
  if (!ctx_ok(ctx)) return HVPIC_ESTATE;
  if (!B || !n_half || !J_half || !E_out) return HVPIC_EINVAL;
  if (mode != 0 && mode != 1) return HVPIC_EINVAL;
  if (mode == 0 && (!n_prev || !J_prev)) return HVPIC_EINVAL;
  if (ctx->p.energy_eq || ctx->p.open_x) return HVPIC_EINVAL;
  if (ctx->p.eta_h != 0.0)
    return launch_field_advance_ext(ctx, B, nullptr, n_half, J_half, n_prev, J_prev, E_out, mode,
                                    diag_out);
  return launch_field_advance(ctx, B, n_half, J_half, n_prev, J_prev, E_out, mode, diag_out);
}

int hvpic_field_advance_pe(hvpic_ctx* ctx, float* B, float* pe, const float* n_half,
                           const float* J_half, const float* n_prev, const float* J_prev,
                           float* E_out, int mode, double* diag_out) {
  if (!ctx_ok(ctx)) return HVPIC_ESTATE;
  if (!ctx->p.energy_eq || ctx->p.open_x) return HVPIC_EINVAL;
  if (!B || !pe || !n_half || !J_half || !E_out) return HVPIC_EINVAL;
  if (mode != 0 && mode != 1) return HVPIC_EINVAL;
  if (mode == 0 && (!n_prev || !J_prev)) return HVPIC_EINVAL;
  return launch_field_advance_ext(ctx, B, pe, n_half, J_half, n_prev, J_prev, E_out, mode,
                                  diag_out);
}

int hvpic_eos_pressure(hvpic_ctx* ctx, const float* n, float* pe) {
  if (!ctx_ok(ctx)) return HVPIC_ESTATE;
  if (!n || !pe) return HVPIC_EINVAL;
  return launch_eos_pressure(ctx, n, pe);
}

int hvpic_set_stream(hvpic_ctx* ctx, void* hip_stream) {
  if (!ctx_ok(ctx)) return HVPIC_ESTATE;
  ctx->stream = (hipStream_t)hip_stream;
  return HVPIC_OK;
}

int hvpic_smooth(hvpic_ctx* ctx, float* F, int ncomp, int npasses) {
  if (!ctx_ok(ctx)) return HVPIC_ESTATE;
  if (!F || ncomp < 1 || ncomp > 3 || npasses < 0) return HVPIC_EINVAL;
  return launch_smooth(ctx, F, ncomp, npasses);
}

int hvpic_sync_status(hvpic_ctx* ctx, uint32_t* flags, int64_t* counts) {
  if (!ctx_ok(ctx)) return HVPIC_ESTATE;
  if (!flags) return HVPIC_EINVAL;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return HVPIC_EHIP;
  Status h;
  if (hipMemcpy(&h, ctx->status, sizeof(Status), hipMemcpyDeviceToHost) != hipSuccess)
    return HVPIC_EHIP;
  *flags = h.flags;
  if (counts) {
    counts[0] = (int64_t)h.moved_gt1;
    counts[1] = (int64_t)h.nonfinite;
    counts[2] = (int64_t)h.floor_hits;
  }
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(64), 0, ctx->stream, ctx->status);
  if (hipGetLastError() != hipSuccess) return HVPIC_EHIP;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return HVPIC_EHIP;
  return HVPIC_OK;
}

int hvpic_path_stats(hvpic_ctx* ctx, int64_t* stats) {
  if (!ctx_ok(ctx)) return HVPIC_ESTATE;
  if (!stats) return HVPIC_EINVAL;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return HVPIC_EHIP;
  Status h;
  if (hipMemcpy(&h, ctx->status, sizeof(Status), hipMemcpyDeviceToHost) != hipSuccess)
    return HVPIC_EHIP;
  stats[0] = (int64_t)h.win_blocks;
  stats[1] = (int64_t)h.glob_blocks;
  hipLaunchKernelGGL(k_clear_paths, dim3(1), dim3(64), 0, ctx->stream, ctx->status);
  if (hipGetLastError() != hipSuccess) return HVPIC_EHIP;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return HVPIC_EHIP;
  return HVPIC_OK;
}

int hvpic_timing_enable(hvpic_ctx* ctx, int max_launches, int every) {
  if (!ctx_ok(ctx)) return HVPIC_ESTATE;
  if (max_launches < 0 || max_launches > 65536 || every < 1) return HVPIC_EINVAL;
  int rc = HVPIC_OK;
  if (ctx->tev) {
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) rc = HVPIC_EHIP;
    const int64_t ne = (int64_t)HVPIC_KERNEL_COUNT * ctx->tmax * 2;
    for (int64_t i = 0; i < ne; ++i)
      if (ctx->tev[i]) (void)hipEventDestroy(ctx->tev[i]);
    delete[] ctx->tev;
    ctx->tev = nullptr;
  }
  ctx->tmax = 0;
  ctx->tevery = every;
  for (int k = 0; k < HVPIC_KERNEL_COUNT; ++k) {
    ctx->tcount[k] = 0;
    ctx->tseen[k] = 0;
    ctx->tarmed[k] = false;
  }
  if (max_launches == 0 || rc != HVPIC_OK) return rc;
  const int64_t ne = (int64_t)HVPIC_KERNEL_COUNT * max_launches * 2;
  hipEvent_t* ev = new (std::nothrow) hipEvent_t[ne];
  if (!ev) return HVPIC_ENOMEM;
  for (int64_t i = 0; i < ne; ++i) ev[i] = nullptr;
  // Timing only: no system-scope fence when an event is recorded (that fence
  // writes back and invalidates the caches, a few microseconds of stall
  // between the bracketed kernel and the next one).  hvpic_timing_read
  // synchronises the stream before it reads them.
  for (int64_t i = 0; i < ne; ++i)
    if (hipEventCreateWithFlags(&ev[i], hipEventDisableSystemFence) != hipSuccess) {
      for (int64_t j = 0; j < i; ++j) (void)hipEventDestroy(ev[j]);
      delete[] ev;
      return HVPIC_EHIP;
    }
  ctx->tev = ev;
  ctx->tmax = max_launches;
  return HVPIC_OK;
}

int hvpic_timing_read(hvpic_ctx* ctx, int kernel, double* total_ms, int64_t* launches) {
  if (!ctx_ok(ctx)) return HVPIC_ESTATE;
  if (kernel < 0 || kernel >= HVPIC_KERNEL_COUNT || !total_ms || !launches) return HVPIC_EINVAL;
  *total_ms = 0.0;
  *launches = 0;
  if (!ctx->tev) return HVPIC_OK;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) return HVPIC_EHIP;
  double t = 0.0;
  for (int i = 0; i < ctx->tcount[kernel]; ++i) {
    float ms = 0.f;
    const int64_t e = ((int64_t)kernel * ctx->tmax + i) * 2;
    if (hipEventElapsedTime(&ms, ctx->tev[e], ctx->tev[e + 1]) != hipSuccess) return HVPIC_EHIP;
    t += ms;
  }
  *total_ms = t;
  *launches = ctx->tcount[kernel];
  ctx->tcount[kernel] = 0;
  ctx->tseen[kernel] = 0;
  return HVPIC_OK;
}

const char* hvpic_strerror(int code) {
  switch (code) {
    case HVPIC_OK: return "ok";
    case HVPIC_EINVAL: return "invalid argument";
    case HVPIC_ENOMEM: return "out of memory or workspace too small";
    case HVPIC_EHIP: return "HIP runtime error";
    case HVPIC_ESTATE: return "context not initialised";
    default: return "unknown error";
  }
}

}  // extern "C"
