// Ensembles of independent 2D runs stepped together (libhvpic.so, gfx950).
//
// Each run is a full hybrid-PIC step of its own (arXiv 2305.05600, Sec. II:
// gather + Boris push + fused mid-point deposit, neighbour-move sort left as
// a gather map, RK2-subcycled field advance), with its own grid, particles,
// parameters and context.  Small runs leave most of the GPU idle and pay a
// launch per kernel; here every phase of the step is ONE persistent launch
// over the work items (run, chunk or tile) of all runs, each item taking its
// run's arguments from a table in device memory.  Both parities of the
// step's buffer rotation have their tables built once, so a step is a fixed
// sequence of about ten launches that a hipGraph can capture.
//
// Tuning: the push's chunk length (particles per lane) is chosen per class of
// particles per cell, the subcycle's tile shape per class of grid size, and
// the persistent grid per phase, by timing real steps (every choice computes
// the same step, so the tuning steps are steps of the simulation).
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "hvpic_internal.hpp"

namespace hvpic {
namespace {

constexpr uint32_t kEnsMagic = 0x454e5331u;  // "ENS1"
constexpr int kPpt[3] = {4, 8, 12};           // push particles per lane, by choice 0..2
constexpr int kMaxLaunches = 64;
constexpr int kCUs = 256;

int ppc_class(const hvpic_ctx* c, int64_t n) {
  const double ppc = (double)n / (double)c->ncell;
  return ppc < 64.0 ? 0 : (ppc < 128.0 ? 1 : 2);
}
int grid_class(const hvpic_ctx* c) { return c->ncell < 128 * 128 ? 0 : 1; }

// grid of a persistent launch over nitems items: a multiple of 8 (one stride
// per XCD), at most blocks_per_cu blocks per CU and no more than the items
int persistent_grid(int nitems, int blocks_per_cu) {
  const int cap = std::max(8, blocks_per_cu * kCUs);
  const int g = std::min(cap, (int)ceil_div(std::max(nitems, 1), 8) * 8);
  return std::max(8, g / 8 * 8);
}

}  // namespace
}  // namespace hvpic

struct hvpic_ensemble {
  uint32_t magic;
  int nruns;
  hipStream_t stream;
  std::vector<hvpic_run> runs;
  hvpic_tuning tune;
  std::vector<int> pclass, gclass;
  char* ws;
  size_t ws_bytes;
  // tables (device) per parity
  char* push_tab[2];
  char* mom_tab[2];
  char* sort_tab[2];
  char* field_tab[2];  // [launch][run] records
  char* diag_tab[2];
  size_t push_rec, mom_rec, sort_rec, field_rec, diag_rec;
  // item lists (device)
  hvpic::Item* push_items;  // groups by push choice 0..2
  int push_off[4];
  hvpic::Item* mom_items;
  int n_mom;
  hvpic::Item* tile_items;
  int n_tiles;
  hvpic::Item* scat_items;
  int n_scat;
  hvpic::Item* field_items;  // groups by tile shape 0..2
  int field_off[4];
  int64_t push_cap, field_cap;  // item capacity of the two tuned lists
  int nlaunch;
  int K[hvpic::kMaxLaunches], has_lin[hvpic::kMaxLaunches], fin[hvpic::kMaxLaunches];
  int64_t steps;
  bool graph;
  hipGraphExec_t exec[2];
};

namespace hvpic {
namespace {

bool ens_ok(const hvpic_ensemble* e) { return e && e->magic == kEnsMagic; }

struct EnsLayout {
  size_t push_tab, mom_tab, sort_tab, field_tab, diag_tab, push_items, mom_items, tile_items,
      scat_items, field_items, total;
  int64_t push_cap, field_cap, n_mom, n_tiles, n_scat;
};

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

EnsLayout layout(const hvpic_run* runs, int nruns) {
  EnsLayout L{};
  size_t off = 0;
  const size_t pr = ens_push_record(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                    nullptr, false, nullptr);
  const size_t mr = ens_moments_record(nullptr, nullptr, nullptr, 0, nullptr, nullptr);
  const size_t sr = ens_sort_record(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
  const size_t fr = ens_field_record(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                     nullptr, false, 0, 0, nullptr);
  const size_t dr = ens_field_diag_record(nullptr, nullptr, 0, nullptr);
  int nl = 0;
  for (int r = 0; r < nruns; ++r) {
    hvpic_ctx* c = runs[r].ctx;
    const int64_t n = runs[r].store[0].n;
    L.push_cap += ceil_div(n, ens_chunk(kPpt[0]));
    L.n_mom += ens_moment_blocks(c);
    L.n_tiles += ens_sort_tiles(c);
    L.n_scat += ens_sort_scatter_blocks(c);
    int t = 0;
    for (int s = 0; s < kTileShapes; ++s) t = std::max(t, ens_field_tiles(c, s));
    L.field_cap += t;
    nl = ens_field_launches(c, nullptr, nullptr, nullptr);
  }
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += a256(bytes);
    return at;
  };
  L.push_tab = take(2 * pr * nruns);
  L.mom_tab = take(2 * mr * nruns);
  L.sort_tab = take(2 * sr * nruns);
  L.field_tab = take(2 * fr * nruns * (size_t)std::max(nl, 1));
  L.diag_tab = take(2 * dr * nruns);
  L.push_items = take(sizeof(Item) * L.push_cap);
  L.mom_items = take(sizeof(Item) * L.n_mom);
  L.tile_items = take(sizeof(Item) * L.n_tiles);
  L.scat_items = take(sizeof(Item) * L.n_scat);
  L.field_items = take(sizeof(Item) * L.field_cap);
  L.total = off;
  return L;
}

bool runs_ok(const hvpic_run* runs, int nruns) {
  if (!runs || nruns < 1 || nruns > (1 << 20)) return false;
  int nsub = -1, shape = -1;
  for (int r = 0; r < nruns; ++r) {
    const hvpic_run& R = runs[r];
    const hvpic_ctx* c = R.ctx;
    if (!c || c->magic != kMagic) return false;
    const hvpic_params& p = c->p;
    if (p.ndim != 2 || p.nsmooth != 0 || p.energy_eq != 0 || p.open_x != 0 || p.eta_h != 0.0 ||
        p.nsub < 3 ||
        p.nsub > 2 * kMaxLaunches)
      return false;
    if ((nsub >= 0 && p.nsub != nsub) || (shape >= 0 && p.shape != shape)) return false;
    nsub = p.nsub;
    shape = p.shape;
    if (!ens_sort_fits(c)) return false;
    const int64_t n = R.store[0].n;
    if (n < 1 || n != R.store[1].n || n > p.np_capacity || n >= (int64_t(1) << 30)) return false;
    for (int k = 0; k < 2; ++k) {
      const hvpic_particles& q = R.store[k];
      if (!q.cell || !q.ox || !q.oy || !q.ux || !q.uy || !q.uz || !q.w) return false;
      if (!R.cell_start[k] || !R.n[k] || !R.J[k]) return false;
    }
    if (!R.perm || !R.E || !R.B) return false;
  }
  return true;
}

bool tuning_ok(const hvpic_tuning* t) {
  if (!t) return false;
  for (int k = 0; k < 3; ++k)
    if (t->push_chunk[k] < 0 || t->push_chunk[k] > 2) return false;
  for (int k = 0; k < 2; ++k)
    if (t->field_tile[k] < 0 || t->field_tile[k] >= kTileShapes) return false;
  for (int k = 0; k < 4; ++k)
    if (t->blocks_per_cu[k] < 1 || t->blocks_per_cu[k] > 64) return false;
  return true;
}

// The item lists and both parities' tables for the current tuning, uploaded
// with synchronous copies (never inside a capture).
int build(hvpic_ensemble* e) {
  const int R = e->nruns;
  auto upload = [&](char* dst, const std::vector<char>& src) {
    return src.empty() || hipMemcpy(dst, src.data(), src.size(), hipMemcpyHostToDevice) == hipSuccess;
  };
  // items
  std::vector<Item> push, field, mom, tiles, scat;
  for (int g = 0; g < 3; ++g) {
    e->push_off[g] = (int)push.size();
    for (int r = 0; r < R; ++r) {
      if (e->tune.push_chunk[e->pclass[r]] != g) continue;
      const int nb = (int)ceil_div(e->runs[r].store[0].n, ens_chunk(kPpt[g]));
      for (int b = 0; b < nb; ++b) push.push_back(Item{r, b, nb});
    }
  }
  e->push_off[3] = (int)push.size();
  for (int g = 0; g < kTileShapes; ++g) {
    e->field_off[g] = (int)field.size();
    for (int r = 0; r < R; ++r) {
      if (e->tune.field_tile[e->gclass[r]] != g) continue;
      const int nb = ens_field_tiles(e->runs[r].ctx, g);
      for (int b = 0; b < nb; ++b) field.push_back(Item{r, b, nb});
    }
  }
  e->field_off[3] = (int)field.size();
  for (int r = 0; r < R; ++r) {
    hvpic_ctx* c = e->runs[r].ctx;
    const int nm = ens_moment_blocks(c), nt = ens_sort_tiles(c), ns = ens_sort_scatter_blocks(c);
    for (int b = 0; b < nm; ++b) mom.push_back(Item{r, b, nm});
    for (int b = 0; b < nt; ++b) tiles.push_back(Item{r, b, nt});
    for (int b = 0; b < ns; ++b) scat.push_back(Item{r, b, ns});
  }
  if ((int64_t)push.size() > e->push_cap || (int64_t)field.size() > e->field_cap) return HVPIC_EINVAL;
  auto up_items = [&](Item* dst, const std::vector<Item>& v) {
    return v.empty() ||
           hipMemcpy(dst, v.data(), sizeof(Item) * v.size(), hipMemcpyHostToDevice) == hipSuccess;
  };
  if (!up_items(e->push_items, push) || !up_items(e->field_items, field) ||
      !up_items(e->mom_items, mom) || !up_items(e->tile_items, tiles) ||
      !up_items(e->scat_items, scat))
    return HVPIC_EHIP;
  e->n_mom = (int)mom.size();
  e->n_tiles = (int)tiles.size();
  e->n_scat = (int)scat.size();
  // tables
  for (int par = 0; par < 2; ++par) {
    const int a = par, b = 1 - par;  // current store / moments level n-1/2, and the other
    std::vector<char> pt(e->push_rec * R), mt(e->mom_rec * R), st(e->sort_rec * R),
        ft(e->field_rec * R * e->nlaunch), dt(e->diag_rec * R);
    for (int r = 0; r < R; ++r) {
      hvpic_run& U = e->runs[r];
      hvpic_ctx* c = U.ctx;
      const int g = e->tune.push_chunk[e->pclass[r]];
      const int shape = e->tune.field_tile[e->gclass[r]];
      ens_push_record(c, &U.store[a], U.perm, &U.store[b], U.cell_start[a], U.E, U.B,
                      U.push_diag != nullptr, pt.data() + e->push_rec * r);
      ens_moments_record(c, U.n[b], U.J[b], (int)ceil_div(U.store[a].n, ens_chunk(kPpt[g])),
                         U.push_diag, mt.data() + e->mom_rec * r);
      ens_sort_record(c, &U.store[b], U.cell_start[a], U.perm, U.cell_start[b],
                      st.data() + e->sort_rec * r);
      for (int m = 0; m < e->nlaunch; ++m)
        ens_field_record(c, U.B, U.n[b], U.J[b], U.n[a], U.J[a], U.E, U.field_diag != nullptr, m,
                         shape, ft.data() + e->field_rec * ((size_t)m * R + r));
      // (a run without field diagnostics has a record with no output: skipped)
      ens_field_diag_record(c, U.field_diag, shape, dt.data() + e->diag_rec * r);
    }
    if (!upload(e->push_tab[par], pt) || !upload(e->mom_tab[par], mt) ||
        !upload(e->sort_tab[par], st) || !upload(e->field_tab[par], ft) ||
        !upload(e->diag_tab[par], dt))
      return HVPIC_EHIP;
  }
  return HVPIC_OK;
}

// One step of every run, parity par of the buffer rotation; with ev non-null
// the phase boundaries are recorded (push, moments + sort, fields).
int enqueue(hvpic_ensemble* e, int par, hipEvent_t* ev) {
  hipStream_t s = e->stream;
  int rc = HVPIC_OK;
  auto ok = [&](int v) {
    if (rc == HVPIC_OK) rc = v;
  };
  if (ev) (void)hipEventRecord(ev[0], s);
  for (int g = 0; g < 3; ++g) {
    const int n = e->push_off[g + 1] - e->push_off[g];
    ok(ens_launch_push(s, e->runs[0].ctx->p.shape, kPpt[g], e->push_tab[par],
                       e->push_items + e->push_off[g], n,
                       persistent_grid(n, e->tune.blocks_per_cu[0])));
  }
  if (ev) (void)hipEventRecord(ev[1], s);
  ok(ens_launch_moments(s, e->mom_tab[par], e->mom_items, e->n_mom,
                        persistent_grid(e->n_mom, e->tune.blocks_per_cu[1])));
  const int gs = e->tune.blocks_per_cu[2];
  ok(ens_launch_sort(s, 0, e->sort_tab[par], e->tile_items, e->n_tiles,
                     persistent_grid(e->n_tiles, gs)));
  ok(ens_launch_sort(s, 1, e->sort_tab[par], e->tile_items, e->n_tiles,
                     persistent_grid(e->n_tiles, gs)));
  ok(ens_launch_sort(s, 2, e->sort_tab[par], e->scat_items, e->n_scat,
                     persistent_grid(e->n_scat, gs)));
  if (ev) (void)hipEventRecord(ev[2], s);
  for (int m = 0; m < e->nlaunch; ++m)
    for (int g = 0; g < kTileShapes; ++g) {
      const int n = e->field_off[g + 1] - e->field_off[g];
      ok(ens_launch_field(s, g, e->K[m], e->has_lin[m], e->fin[m],
                          e->field_tab[par] + e->field_rec * (size_t)m * e->nruns,
                          e->field_items + e->field_off[g], n,
                          persistent_grid(n, e->tune.blocks_per_cu[3])));
    }
  ok(ens_launch_field_diag(s, e->diag_tab[par], e->nruns));
  if (ev) (void)hipEventRecord(ev[3], s);
  return rc;
}

void drop_graph(hvpic_ensemble* e) {
  if (!e->graph) return;
  for (int k = 0; k < 2; ++k) (void)hipGraphExecDestroy(e->exec[k]);
  e->graph = false;
}

}  // namespace
}  // namespace hvpic

using namespace hvpic;

extern "C" {

int hvpic_ensemble_workspace_bytes(const hvpic_run* runs, int nruns, size_t* bytes) {
  if (!bytes || !runs_ok(runs, nruns)) return HVPIC_EINVAL;
  *bytes = layout(runs, nruns).total;
  return HVPIC_OK;
}

int hvpic_tuning_default(hvpic_tuning* t) {
  if (!t) return HVPIC_EINVAL;
  // the plain path's choices: 12 particles per lane, 32x8 tiles
  for (int k = 0; k < 3; ++k) t->push_chunk[k] = 2;
  for (int k = 0; k < 2; ++k) t->field_tile[k] = 0;
  t->blocks_per_cu[0] = 4;
  t->blocks_per_cu[1] = 2;
  t->blocks_per_cu[2] = 4;
  t->blocks_per_cu[3] = 2;
  return HVPIC_OK;
}

int hvpic_ensemble_init(const hvpic_run* runs, int nruns, void* hip_stream, void* workspace,
                        const hvpic_tuning* tuning, hvpic_ensemble** out) {
  if (!out || !runs_ok(runs, nruns) || !workspace || ((uintptr_t)workspace & 255) != 0)
    return HVPIC_EINVAL;
  hvpic_tuning t;
  if (tuning) {
    if (!tuning_ok(tuning)) return HVPIC_EINVAL;
    t = *tuning;
  } else {
    hvpic_tuning_default(&t);
  }
  hvpic_ensemble* e = new (std::nothrow) hvpic_ensemble();
  if (!e) return HVPIC_ENOMEM;
  e->magic = kEnsMagic;
  e->nruns = nruns;
  e->stream = static_cast<hipStream_t>(hip_stream);
  e->runs.assign(runs, runs + nruns);
  e->tune = t;
  const EnsLayout L = layout(runs, nruns);
  char* ws = static_cast<char*>(workspace);
  e->ws = ws;
  e->ws_bytes = L.total;
  e->push_rec = ens_push_record(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                false, nullptr);
  e->mom_rec = ens_moments_record(nullptr, nullptr, nullptr, 0, nullptr, nullptr);
  e->sort_rec = ens_sort_record(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
  e->field_rec = ens_field_record(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                  false, 0, 0, nullptr);
  e->diag_rec = ens_field_diag_record(nullptr, nullptr, 0, nullptr);
  e->nlaunch = ens_field_launches(runs[0].ctx, e->K, e->has_lin, e->fin);
  for (int k = 0; k < 2; ++k) {
    e->push_tab[k] = ws + L.push_tab + k * e->push_rec * nruns;
    e->mom_tab[k] = ws + L.mom_tab + k * e->mom_rec * nruns;
    e->sort_tab[k] = ws + L.sort_tab + k * e->sort_rec * nruns;
    e->field_tab[k] = ws + L.field_tab + k * e->field_rec * nruns * e->nlaunch;
    e->diag_tab[k] = ws + L.diag_tab + k * e->diag_rec * nruns;
  }
  e->push_items = reinterpret_cast<Item*>(ws + L.push_items);
  e->mom_items = reinterpret_cast<Item*>(ws + L.mom_items);
  e->tile_items = reinterpret_cast<Item*>(ws + L.tile_items);
  e->scat_items = reinterpret_cast<Item*>(ws + L.scat_items);
  e->field_items = reinterpret_cast<Item*>(ws + L.field_items);
  e->push_cap = L.push_cap;
  e->field_cap = L.field_cap;
  e->pclass.resize(nruns);
  e->gclass.resize(nruns);
  for (int r = 0; r < nruns; ++r) {
    e->pclass[r] = ppc_class(runs[r].ctx, runs[r].store[0].n);
    e->gclass[r] = grid_class(runs[r].ctx);
  }
  e->steps = 0;
  e->graph = false;
  // The move counts the first push adds to start from zero; the contexts'
  // earlier calls may have left them otherwise.  The rest of the state is
  // the runs' own (a step of the gather-map sequence left it).
  for (int r = 0; r < nruns; ++r) {
    hvpic_ctx* c = runs[r].ctx;
    hipStream_t old = c->stream;
    c->stream = e->stream;
    zero_counts(c);
    c->stream = old;
  }
  const int rc = build(e);
  if (rc != HVPIC_OK) {
    e->magic = 0;
    delete e;
    return rc;
  }
  *out = e;
  return HVPIC_OK;
}

int hvpic_ensemble_finalize(hvpic_ensemble* e) {
  if (!ens_ok(e)) return HVPIC_ESTATE;
  drop_graph(e);
  e->magic = 0;
  delete e;
  return HVPIC_OK;
}

int hvpic_ensemble_step(hvpic_ensemble* e) {
  if (!ens_ok(e)) return HVPIC_ESTATE;
  const int par = (int)(e->steps & 1);
  int rc;
  if (e->graph)
    rc = hipGraphLaunch(e->exec[par], e->stream) == hipSuccess ? HVPIC_OK : HVPIC_EHIP;
  else
    rc = enqueue(e, par, nullptr);
  if (rc == HVPIC_OK) ++e->steps;
  return rc;
}

int hvpic_ensemble_steps(const hvpic_ensemble* e, int64_t* steps) {
  if (!ens_ok(e)) return HVPIC_ESTATE;
  if (!steps) return HVPIC_EINVAL;
  *steps = e->steps;
  return HVPIC_OK;
}

int hvpic_ensemble_capture(hvpic_ensemble* e, int enable) {
  if (!ens_ok(e)) return HVPIC_ESTATE;
  drop_graph(e);
  if (!enable) return HVPIC_OK;
  if (e->stream == nullptr) return HVPIC_EINVAL;  // the null stream cannot be captured
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  for (int par = 0; par < 2; ++par) {
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return HVPIC_EHIP;
    const int rc = enqueue(e, par, nullptr);
    const hipError_t ec = hipStreamEndCapture(e->stream, &g);
    if (rc != HVPIC_OK || ec != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      if (par == 1) (void)hipGraphExecDestroy(exec[0]);
      return HVPIC_EHIP;
    }
    const hipError_t ei = hipGraphInstantiate(&exec[par], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      if (par == 1) (void)hipGraphExecDestroy(exec[0]);
      return HVPIC_EHIP;
    }
  }
  e->exec[0] = exec[0];
  e->exec[1] = exec[1];
  e->graph = true;
  return HVPIC_OK;
}

int hvpic_ensemble_get_tuning(const hvpic_ensemble* e, hvpic_tuning* t) {
  if (!ens_ok(e)) return HVPIC_ESTATE;
  if (!t) return HVPIC_EINVAL;
  *t = e->tune;
  return HVPIC_OK;
}

int hvpic_ensemble_set_tuning(hvpic_ensemble* e, const hvpic_tuning* t) {
  if (!ens_ok(e)) return HVPIC_ESTATE;
  if (!tuning_ok(t)) return HVPIC_EINVAL;
  const bool had_graph = e->graph;
  drop_graph(e);
  // the tables are rewritten: nothing queued may still read them
  if (hipStreamSynchronize(e->stream) != hipSuccess) return HVPIC_EHIP;
  e->tune = *t;
  int rc = build(e);
  if (rc == HVPIC_OK && had_graph) rc = hvpic_ensemble_capture(e, 1);
  return rc;
}

int hvpic_ensemble_autotune(hvpic_ensemble* e, int reps, hvpic_tuning* best_out,
                            double* ms_out) {
  if (!ens_ok(e)) return HVPIC_ESTATE;
  if (reps < 1 || reps > 100) return HVPIC_EINVAL;
  const bool had_graph = e->graph;
  drop_graph(e);
  hipEvent_t ev[4];
  for (int k = 0; k < 4; ++k)
    if (hipEventCreate(&ev[k]) != hipSuccess) return HVPIC_EHIP;
  int rc = HVPIC_OK;
  // time of phase `ph` (0 push, 1 moments + sort, 2 fields) of a candidate:
  // the least over reps real steps
  auto trial = [&](const hvpic_tuning& t, int ph, double* ms) -> int {
    if (hipStreamSynchronize(e->stream) != hipSuccess) return HVPIC_EHIP;
    e->tune = t;
    int r = build(e);
    if (r != HVPIC_OK) return r;
    double best = 1e30;
    for (int k = 0; k < reps; ++k) {
      r = enqueue(e, (int)(e->steps & 1), ev);
      if (r != HVPIC_OK) return r;
      ++e->steps;
      if (hipEventSynchronize(ev[3]) != hipSuccess) return HVPIC_EHIP;
      float a = 0.f;
      (void)hipEventElapsedTime(&a, ev[ph], ev[ph + 1]);
      best = std::min(best, (double)a);
    }
    *ms = best;
    return HVPIC_OK;
  };
  hvpic_tuning cur = e->tune;
  double tms[3] = {0.0, 0.0, 0.0};
  // push: chunk length per ppc class, then the persistent grid
  for (int cls = 0; cls < 3 && rc == HVPIC_OK; ++cls) {
    bool present = false;
    for (int r = 0; r < e->nruns; ++r) present |= e->pclass[r] == cls;
    if (!present) continue;
    double best = 1e30;
    int arg = cur.push_chunk[cls];
    for (int g = 0; g < 3 && rc == HVPIC_OK; ++g) {
      hvpic_tuning t = cur;
      t.push_chunk[cls] = g;
      double ms = 0.0;
      rc = trial(t, 0, &ms);
      if (ms < best) best = ms, arg = g;
    }
    cur.push_chunk[cls] = arg;
    tms[0] = best;
  }
  const int grids[3] = {2, 4, 8};
  for (int ph = 0; ph < 3 && rc == HVPIC_OK; ++ph) {
    const int knob = ph == 0 ? 0 : (ph == 1 ? 2 : 3);
    double best = 1e30;
    int arg = cur.blocks_per_cu[knob];
    for (int q = 0; q < 3 && rc == HVPIC_OK; ++q) {
      hvpic_tuning t = cur;
      t.blocks_per_cu[knob] = ph == 2 ? grids[q] / 2 : grids[q];
      double ms = 0.0;
      rc = trial(t, ph, &ms);
      if (ms < best) best = ms, arg = t.blocks_per_cu[knob];
    }
    cur.blocks_per_cu[knob] = arg;
    tms[ph] = best;
  }
  // field: tile shape per grid class
  for (int cls = 0; cls < 2 && rc == HVPIC_OK; ++cls) {
    bool present = false;
    for (int r = 0; r < e->nruns; ++r) present |= e->gclass[r] == cls;
    if (!present) continue;
    double best = 1e30;
    int arg = cur.field_tile[cls];
    for (int s = 0; s < kTileShapes && rc == HVPIC_OK; ++s) {
      hvpic_tuning t = cur;
      t.field_tile[cls] = s;
      double ms = 0.0;
      rc = trial(t, 2, &ms);
      if (ms < best) best = ms, arg = s;
    }
    cur.field_tile[cls] = arg;
    tms[2] = best;
  }
  if (rc == HVPIC_OK) {
    (void)hipStreamSynchronize(e->stream);
    e->tune = cur;
    rc = build(e);
  }
  for (int k = 0; k < 4; ++k) (void)hipEventDestroy(ev[k]);
  if (rc == HVPIC_OK && had_graph) rc = hvpic_ensemble_capture(e, 1);
  if (rc == HVPIC_OK) {
    if (best_out) *best_out = e->tune;
    if (ms_out)
      for (int k = 0; k < 3; ++k) ms_out[k] = tms[k];
  }
  return rc;
}

int hvpic_ensemble_time_phases(hvpic_ensemble* e, int steps, double* ms) {
  if (!ens_ok(e)) return HVPIC_ESTATE;
  if (steps < 1 || steps > 100000 || !ms) return HVPIC_EINVAL;
  std::vector<hipEvent_t> ev(4 * (size_t)steps);
  for (auto& x : ev)
    if (hipEventCreate(&x) != hipSuccess) return HVPIC_EHIP;
  int rc = HVPIC_OK;
  for (int k = 0; k < steps && rc == HVPIC_OK; ++k) {
    rc = enqueue(e, (int)(e->steps & 1), ev.data() + 4 * (size_t)k);
    if (rc == HVPIC_OK) ++e->steps;
  }
  double sum[3] = {0.0, 0.0, 0.0};
  if (rc == HVPIC_OK && hipStreamSynchronize(e->stream) != hipSuccess) rc = HVPIC_EHIP;
  for (int k = 0; k < steps && rc == HVPIC_OK; ++k)
    for (int ph = 0; ph < 3; ++ph) {
      float a = 0.f;
      if (hipEventElapsedTime(&a, ev[4 * (size_t)k + ph], ev[4 * (size_t)k + ph + 1]) != hipSuccess)
        rc = HVPIC_EHIP;
      sum[ph] += a;
    }
  for (auto& x : ev) (void)hipEventDestroy(x);
  if (rc == HVPIC_OK)
    for (int ph = 0; ph < 3; ++ph) ms[ph] = sum[ph] / steps;
  return rc;
}

}  // extern "C"
