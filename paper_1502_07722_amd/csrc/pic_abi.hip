// C ABI of the PIC pair-potential library (declared in include/pic.h):
// argument validation, unit conversion, workspace carving, stream-ordered
// launches and device-error reporting.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pic_internal.h"

using namespace pic;

namespace {

constexpr size_t kAlign = 256;
constexpr int kDiagCap = 1024;  // device diag entries buffered between host copies

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int64_t blocks_of(int64_t n) { return (n + 255) / 256; }

struct Sizes {
  int64_t ncells = 0, nnodes = 0;
};

bool grid_sizes(const pic_grid_t *g, Sizes *s, std::string *why) {
  if (!g) { if (why) *why = "grid is NULL"; return false; }
  if (g->ndim != 2 && g->ndim != 3) { if (why) *why = "ndim must be 2 or 3"; return false; }
  int64_t nc = 1, nn = 1;
  for (int d = 0; d < g->ndim; ++d) {
    if (g->n[d] < 1) { if (why) *why = "cells per axis must be >= 1"; return false; }
    if (!(g->h[d] > 0.0) || !std::isfinite(g->h[d])) { if (why) *why = "cell size must be > 0"; return false; }
    if (g->bc[d] != 0 && g->bc[d] != 1) { if (why) *why = "bc must be 0 or 1"; return false; }
    nc *= g->n[d];
    nn *= g->n[d] + g->bc[d];
    if (nc >= (int64_t(1) << 31) || nn >= (int64_t(1) << 31)) {
      if (why) *why = "grid too large (cells and nodes must be < 2^31)";
      return false;
    }
  }
  s->ncells = nc;
  s->nnodes = nn;
  return true;
}

// Tiled fast path limits: packed cell coordinates and tile sizes.
bool tiled_supported(const pic_grid_t *g, int64_t max_n) {
  if (max_n >= (int64_t(1) << 30)) return false;  // 32-bit byte offsets into the store
  if (g->ndim == 2) return g->n[0] <= 65536 && g->n[1] <= 32768;
  return g->n[0] <= 2048 && g->n[1] <= 2048 && g->n[2] <= 512;
}

int min_tile_log2(int ndim) { return ndim == 2 ? 3 : 2; }  // smallest tiles: 8^2, 4^3
int max_tile_log2(int ndim) { return ndim == 2 ? 5 : 3; }  // largest: 32^2, 8^3 (LDS)

int64_t tiles_for(const pic_grid_t *g, int lt) {
  int64_t t = 1;
  for (int d = 0; d < g->ndim; ++d) t *= (g->n[d] + (1 << lt) - 1) >> lt;
  return t;
}

int64_t max_items_for(const pic_grid_t *g, int lt, int64_t max_n, int chunk) {
  return tiles_for(g, lt) + (max_n + chunk - 1) / chunk;
}

constexpr int kMinChunk = 1024;
constexpr int kDriftCheck = 32;      // adaptive re-binning looks at the drifter count this often
constexpr int kDriftFraction = 2048; // and re-bins once drifters exceed n / kDriftFraction
constexpr int kMaxBinPeriod = 1024;  // or after this many steps
constexpr int kMaxChunkHost = 32768;  // the fused kernel keeps a per-item outlier bitmask in LDS

struct Layout {
  size_t err, diag, partial, partial_pe, node, dens, G, total;
  bool tiled;
  size_t store[2], bins, items, n3[3], drift;
  int64_t tiles_max, items_max;
};

size_t store_bytes(int ndim, int64_t cap) { return align_up((size_t)cap * 4 * (4 + ndim + 3)); }

Layout make_layout(const pic_grid_t *g, const Sizes &s, int ndim, int64_t max_n) {
  Layout L{};
  size_t o = 0;
  L.tiled = tiled_supported(g, max_n);
  L.tiles_max = L.tiled ? tiles_for(g, min_tile_log2(ndim)) : 0;
  L.items_max = L.tiled ? max_items_for(g, min_tile_log2(ndim), max_n, kMinChunk) : 0;
  const int64_t partial_blocks =
      std::max<int64_t>(std::max<int64_t>(blocks_of(max_n), L.items_max + kDriftBlocks), 1);
  L.err = o; o = align_up(o + sizeof(uint32_t));
  L.diag = o; o = align_up(o + sizeof(pic_diag_t) * kDiagCap);
  L.partial = o; o = align_up(o + sizeof(double) * 8 * (size_t)partial_blocks);
  L.partial_pe = o; o = align_up(o + sizeof(double) * 8 * (size_t)std::max<int64_t>(blocks_of(s.nnodes), 1));
  L.node = o; o = align_up(o + sizeof(long long) * (size_t)s.nnodes);
  L.dens = o; o = align_up(o + sizeof(float) * (size_t)s.nnodes);
  L.G = o; o = align_up(o + sizeof(float) * (size_t)s.ncells * ndim);
  if (L.tiled) {
    for (int k = 0; k < 2; ++k) { L.store[k] = o; o += store_bytes(ndim, std::max<int64_t>(max_n, 1)); }
    L.bins = o; o = align_up(o + sizeof(int) * (size_t)(4 * L.tiles_max + 2));
    L.items = o; o = align_up(o + sizeof(Item) * (size_t)L.items_max);
    for (int k = 0; k < 3; ++k) { L.n3[k] = o; o = align_up(o + sizeof(long long) * (size_t)s.nnodes); }
    L.drift = o; o = align_up(o + sizeof(int) * (size_t)(std::max<int64_t>(max_n, 1) + 2));
  }
  L.total = o;
  return L;
}

}  // namespace

struct pic_ctx {
  pic_grid_t grid;
  pic_potential_t pot;
  double dt;
  int64_t max_n;
  Sizes sz;
  char *ws;
  hipStream_t stream;
  Geo geo;
  Pot P;
  DiagC dc;
  uint32_t *err;
  pic_diag_t *diag_dev;
  double *partial;
  double *partial_pe;
  long long *node;
  float *dens;
  float *G;
  std::string last_error;
  // tiled fast path
  bool tiled = false;
  TileGeo tg{};
  Store st[2]{};
  BinBufs bb{};
  long long *n3[3]{};
  int *drift = nullptr;  // [2 counters][max_n list]
  int64_t tiles_cap = 0, items_cap = 0;
  int sort_every = 0;           // > 0 fixed period, 0 never, < 0 adaptive
  int *h_drift = nullptr;       // pinned host copy of a drifter count (adaptive re-binning)
  hipEvent_t drift_ev = nullptr;
  bool drift_pending = false;
  bool force_untiled = false;
  long long *last_nodes = nullptr;
  int last_step = 0;
  // event timing of pic_step phases
  bool timing = false;
  pic_timing_t tacc{};
  std::vector<hipEvent_t> ev_pool;           // free events
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
};

static hipEvent_t take_event(pic_ctx_t *c) {
  if (c->ev_pool.empty()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  hipEvent_t e = c->ev_pool.back();
  c->ev_pool.pop_back();
  return e;
}

static void harvest_events(pic_ctx_t *c) {
  if (c->ev_pending.empty()) return;
  (void)hipStreamSynchronize(c->stream);
  for (auto &pe : c->ev_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pe.second.first, pe.second.second) == hipSuccess) {
      c->tacc.ms[pe.first] += ms;
      c->tacc.launches[pe.first] += 1;
    }
    c->ev_pool.push_back(pe.second.first);
    c->ev_pool.push_back(pe.second.second);
  }
  c->ev_pending.clear();
}

// RAII bracket: records an event pair around the launches of one phase.
struct PhaseTimer {
  pic_ctx_t *c;
  int phase;
  hipEvent_t a = nullptr;
  PhaseTimer(pic_ctx_t *ctx, int ph) : c(ctx), phase(ph) {
    if (c->timing && (a = take_event(c))) (void)hipEventRecord(a, c->stream);
  }
  ~PhaseTimer() {
    if (!a) return;
    hipEvent_t b = take_event(c);
    if (!b) return;
    (void)hipEventRecord(b, c->stream);
    c->ev_pending.push_back({phase, {a, b}});
    if (c->ev_pending.size() >= 512) harvest_events(c);
  }
};

static int fail(pic_ctx_t *ctx, int code, const std::string &msg) {
  if (ctx) ctx->last_error = msg;
  return code;
}

static int hip_check(pic_ctx_t *ctx, hipError_t e, const char *what) {
  if (e == hipSuccess) return PIC_OK;
  return fail(ctx, PIC_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

static int check_launch(pic_ctx_t *ctx, const char *what) {
  return hip_check(ctx, hipGetLastError(), what);
}

static int check_particles(pic_ctx_t *ctx, const pic_particles_t *p, bool need_vel, bool need_wq) {
  if (!p) return fail(ctx, PIC_EINVAL, "particles is NULL");
  if (p->n < 0) return fail(ctx, PIC_EINVAL, "particle count is negative");
  if (p->n > ctx->max_n) return fail(ctx, PIC_ENOSPACE, "particle count exceeds max_n of the context");
  if (p->n == 0) return PIC_OK;
  if (!p->cell || !p->off) return fail(ctx, PIC_EINVAL, "cell or off is NULL");
  if (need_vel && !p->vel) return fail(ctx, PIC_EINVAL, "vel is NULL");
  if (need_wq && !p->wq) return fail(ctx, PIC_EINVAL, "wq is NULL");
  return PIC_OK;
}

static PartPtrs ptrs(const pic_particles_t *p) {
  return PartPtrs{p->n, p->cell, p->off, p->vel, p->wq};
}

// Read and clear the device error word; map it to a status.
static int read_device_error(pic_ctx_t *ctx) {
  uint32_t h = 0;
  int rc = hip_check(ctx, hipMemcpyAsync(&h, ctx->err, sizeof(h), hipMemcpyDeviceToHost, ctx->stream),
                     "reading the device error word");
  if (rc) return rc;
  rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "stream synchronize");
  if (rc) return rc;
  if (h) {
    launch_clear_word(ctx->stream, ctx->err);
    rc = check_launch(ctx, "clearing the device error word");
    if (rc) return rc;
    rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "stream synchronize");
    if (rc) return rc;
  }
  if (h & ERR_RANGE) return fail(ctx, PIC_ERANGE, "a particle had a cell outside the grid or an offset outside [0,1)");
  if (h & ERR_WEIGHT) return fail(ctx, PIC_EOVERFLOW, "a particle had a negative fixed-point weight");
  if (h & ERR_CFL) return fail(ctx, PIC_ECFL, "a particle moved one cell or more in one step");
  return PIC_OK;
}

// Apply a tiling (tile edge 2^lt cells, halo, chunk, binning period).
static int apply_tiling(pic_ctx_t *c, int lt, int halo, int chunk, int sort_every) {
  const int nd = c->grid.ndim;
  if (lt < min_tile_log2(nd) || lt > max_tile_log2(nd)) return fail(c, PIC_EINVAL, "tile edge out of range");
  if (halo < 1 || halo > 4) return fail(c, PIC_EINVAL, "halo must be 1..4 cells");
  if (chunk < kMinChunk || chunk > kMaxChunkHost) return fail(c, PIC_EINVAL, "chunk out of range");
  if (sort_every < -1) return fail(c, PIC_EINVAL, "sort_every must be >= -1");
  TileGeo &T = c->tg;
  T.ntiles = 1;
  for (int d = 0; d < 3; ++d) {
    T.lt[d] = d < nd ? lt : 0;
    T.tn[d] = d < nd ? (c->grid.n[d] + (1 << lt) - 1) >> lt : 1;
    T.ntiles *= T.tn[d];
  }
  T.H = halo;
  T.chunk = chunk;
  TileGeo probe = T;
  if (window_lds_bytes(probe, nd) > 64 * 1024) return fail(c, PIC_EINVAL, "tile window does not fit in LDS");
  for (int d = 0; d < nd; ++d)  // periodic axes must hold a whole window (single-wrap window coordinates)
    if (!c->grid.bc[d] && c->grid.n[d] < (1 << lt) + 2 * halo + 3)
      return fail(c, PIC_EINVAL, "a periodic axis is shorter than the tile window");
  c->sort_every = sort_every;
  return PIC_OK;
}

static int64_t max_items_now(const pic_ctx_t *c, int64_t n) {
  return (int64_t)c->tg.ntiles + (n + c->tg.chunk - 1) / c->tg.chunk;
}

extern "C" {

int64_t pic_num_nodes(const pic_grid_t *grid) {
  Sizes s;
  return grid_sizes(grid, &s, nullptr) ? s.nnodes : 0;
}

size_t pic_workspace_bytes(const pic_grid_t *grid, int64_t max_n) {
  Sizes s;
  if (!grid_sizes(grid, &s, nullptr) || max_n < 0) return 0;
  return make_layout(grid, s, grid->ndim, max_n).total;
}

int pic_init(pic_ctx_t **out, const pic_grid_t *grid, const pic_potential_t *pot, double dt, int64_t max_n,
             void *ws, size_t ws_bytes, void *stream) {
  if (!out) return PIC_EINVAL;
  *out = nullptr;
  Sizes s;
  std::string why;
  if (!grid_sizes(grid, &s, &why)) return PIC_EINVAL;
  if (!pot) return PIC_EINVAL;
  const pic_potential_t &P = *pot;
  if (!(P.D > 0) || !(P.r0 > 0) || !(P.s_rep > 0) || !(P.c_att > 0) || !(P.g_clamp > 0) || !(P.g_clamp < 2) ||
      !(P.n_floor >= 0) || !(P.mass > 0) || !std::isfinite(P.s_rep) || !std::isfinite(P.c_att))
    return PIC_EINVAL;
  if (!(dt > 0) || !std::isfinite(dt)) return PIC_EINVAL;
  if (max_n < 0 || max_n >= (int64_t(1) << 40)) return PIC_EINVAL;
  Layout L = make_layout(grid, s, grid->ndim, max_n);
  if (!ws || ws_bytes < L.total) return PIC_ENOSPACE;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return PIC_EINVAL;

  pic_ctx_t *c = new pic_ctx_t();
  c->grid = *grid;
  if (c->grid.ndim == 2) {
    c->grid.n[2] = 1;
    c->grid.bc[2] = 0;
    c->grid.h[2] = c->grid.depth2d > 0 ? c->grid.depth2d : c->grid.h[0];
    c->grid.depth2d = c->grid.h[2];
  }
  c->pot = P;
  c->dt = dt;
  c->max_n = max_n;
  c->sz = s;
  c->ws = static_cast<char *>(ws);
  c->stream = static_cast<hipStream_t>(stream);

  const pic_grid_t &g = c->grid;
  const double V = g.h[0] * g.h[1] * g.h[2];
  const double r3 = P.r0 * P.r0 * P.r0;
  Geo &G = c->geo;
  std::memset(&G, 0, sizeof(G));
  G.ndim = g.ndim;
  for (int d = 0; d < 3; ++d) {
    G.n[d] = d < g.ndim ? g.n[d] : 1;
    G.bc[d] = d < g.ndim ? g.bc[d] : 0;
    G.nn[d] = d < g.ndim ? g.n[d] + g.bc[d] : 1;
    G.gam[d] = d < g.ndim ? (float)(P.r0 / ((g.ndim == 2 ? 2.0 : 4.0) * g.h[d])) : 0.0f;
    G.tau[d] = d < g.ndim ? (float)(dt / g.h[d]) : 0.0f;
  }
  G.ncells = (int)s.ncells;
  G.nnodes = (int)s.nnodes;
  G.inv_n0 = 1.0 / G.n[0];
  G.inv_n1 = 1.0 / G.n[1];
  G.kappa = (float)(std::ldexp(1.0, -20) * r3 / V);
  Pot &K = c->P;
  K.nfloor = (float)(P.n_floor * r3);
  K.gclamp = (float)P.g_clamp;
  K.s_rep = (float)P.s_rep;
  K.c_att = (float)P.c_att;
  K.beta = (float)(12.0 * P.D / P.r0);
  K.gv = (float)(dt / P.mass);
  c->dc = DiagC{P.D, P.mass, 0.5 * P.mass, std::ldexp(1.0, -20), V, r3, P.s_rep, P.c_att};

  c->err = reinterpret_cast<uint32_t *>(c->ws + L.err);
  c->diag_dev = reinterpret_cast<pic_diag_t *>(c->ws + L.diag);
  c->partial = reinterpret_cast<double *>(c->ws + L.partial);
  c->partial_pe = reinterpret_cast<double *>(c->ws + L.partial_pe);
  c->node = reinterpret_cast<long long *>(c->ws + L.node);
  c->dens = reinterpret_cast<float *>(c->ws + L.dens);
  c->G = reinterpret_cast<float *>(c->ws + L.G);
  c->tiled = L.tiled;
  if (L.tiled) {
    const int64_t cap = std::max<int64_t>(max_n, 1);
    for (int k = 0; k < 2; ++k) {
      char *b = c->ws + L.store[k];
      Store &S = c->st[k];
      S.cap = cap;
      S.pc = reinterpret_cast<int *>(b);
      S.off = reinterpret_cast<float *>(b + 4 * cap);
      S.vel = reinterpret_cast<float *>(b + 4 * cap * (1 + g.ndim));
      S.wq = reinterpret_cast<int *>(b + 4 * cap * (4 + g.ndim));
      S.oidx = reinterpret_cast<int *>(b + 4 * cap * (5 + g.ndim));
    }
    int *bi = reinterpret_cast<int *>(c->ws + L.bins);
    c->bb.counts = bi;
    c->bb.starts = bi + L.tiles_max;
    c->bb.cursors = bi + 2 * L.tiles_max + 1;
    c->bb.item_start = bi + 3 * L.tiles_max + 1;
    c->bb.num_items = bi + 4 * L.tiles_max + 1;
    c->bb.items = reinterpret_cast<Item *>(c->ws + L.items);
    for (int k = 0; k < 3; ++k) c->n3[k] = reinterpret_cast<long long *>(c->ws + L.n3[k]);
    c->drift = reinterpret_cast<int *>(c->ws + L.drift);
    c->tiles_cap = L.tiles_max;
    c->items_cap = L.items_max;
    TileGeo &T = c->tg;
    T.pshift[0] = 0;
    T.pshift[1] = g.ndim == 2 ? 16 : 11;
    T.pshift[2] = g.ndim == 2 ? 31 : 22;
    T.pmask[0] = g.ndim == 2 ? 0xFFFF : 0x7FF;
    T.pmask[1] = g.ndim == 2 ? 0x7FFF : 0x7FF;
    T.pmask[2] = g.ndim == 2 ? 0 : 0x1FF;
  }
  launch_clear_word(c->stream, c->err);
  if (hipGetLastError() != hipSuccess) {
    delete c;
    return PIC_EHIP;
  }
  if (c->tiled) {
    // default tiling; smaller tiles for small periodic grids; untiled if none fits
    int rc = PIC_EINVAL;
    if (g.ndim == 2) {
      for (int lt = 4; lt >= 3 && rc; --lt) rc = apply_tiling(c, lt, 2, 8192, -1);
      if (rc) rc = apply_tiling(c, 3, 1, 8192, -1);
    } else {
      for (int lt = 3; lt >= 2 && rc; --lt) rc = apply_tiling(c, lt, 1, 4096, -1);
    }
    if (rc) c->tiled = false;
    c->last_error.clear();
    if (c->tiled && (hipHostMalloc((void **)&c->h_drift, 16, hipHostMallocDefault) != hipSuccess ||
                     hipEventCreateWithFlags(&c->drift_ev, hipEventDisableTiming) != hipSuccess)) {
      c->h_drift = nullptr;
      c->tiled = false;
    }
  }
  *out = c;
  return PIC_OK;
}

int pic_set_tiling(pic_ctx_t *ctx, int32_t tile, int32_t halo, int32_t chunk, int32_t sort_every) {
  if (!ctx) return PIC_EINVAL;
  if (!ctx->tiled) return fail(ctx, PIC_EINVAL, "this grid uses the untiled path");
  int lt = 0;
  while ((1 << lt) < tile) ++lt;
  if ((1 << lt) != tile) return fail(ctx, PIC_EINVAL, "tile edge must be a power of two");
  return apply_tiling(ctx, lt, halo, chunk, sort_every);
}

int pic_destroy(pic_ctx_t *ctx) {
  if (!ctx) return PIC_OK;
  if (ctx->drift_ev) (void)hipEventSynchronize(ctx->drift_ev);
  if (ctx->drift_ev) (void)hipEventDestroy(ctx->drift_ev);
  if (ctx->h_drift) (void)hipHostFree(ctx->h_drift);
  harvest_events(ctx);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  delete ctx;
  return PIC_OK;
}

int pic_set_timing(pic_ctx_t *ctx, int32_t on) {
  if (!ctx) return PIC_EINVAL;
  harvest_events(ctx);
  ctx->timing = on != 0;
  if (on) ctx->tacc = pic_timing_t{};
  return PIC_OK;
}

int pic_get_timing(pic_ctx_t *ctx, pic_timing_t *out) {
  if (!ctx || !out) return PIC_EINVAL;
  harvest_events(ctx);
  *out = ctx->tacc;
  out->drifters_last = out->items_last = 0;
  if (ctx->tiled && ctx->last_nodes) {
    int h[3] = {0, 0, 0};
    (void)hipMemcpyAsync(&h[0], ctx->drift, 2 * sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
    (void)hipMemcpyAsync(&h[2], ctx->bb.num_items, sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
    int rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "stream synchronize");
    if (rc) return rc;
    out->drifters_last = h[(ctx->last_step + 1) & 1];
    out->items_last = h[2];
  }
  return PIC_OK;
}

const char *pic_last_error(const pic_ctx_t *ctx) {
  return ctx ? ctx->last_error.c_str() : "context is NULL";
}

int pic_sync(pic_ctx_t *ctx) {
  if (!ctx) return PIC_EINVAL;
  return read_device_error(ctx);
}

int pic_deposit(pic_ctx_t *ctx, const pic_particles_t *p, int64_t *node_w) {
  if (!ctx) return PIC_EINVAL;
  int rc = check_particles(ctx, p, false, true);
  if (rc) return rc;
  if (!node_w) return fail(ctx, PIC_EINVAL, "node_w is NULL");
  launch_fill64(ctx->stream, reinterpret_cast<long long *>(node_w), ctx->sz.nnodes);
  launch_deposit_atomic(ctx->stream, ctx->geo, ptrs(p), reinterpret_cast<long long *>(node_w), ctx->err);
  return check_launch(ctx, "deposit");
}

int pic_force(pic_ctx_t *ctx, const pic_particles_t *p, const int64_t *node_w, float *force,
              pic_diag_t *pe_or_null) {
  if (!ctx) return PIC_EINVAL;
  int rc = check_particles(ctx, p, false, false);
  if (rc) return rc;
  if (!node_w) return fail(ctx, PIC_EINVAL, "node_w is NULL");
  if (p->n > 0 && !force) return fail(ctx, PIC_EINVAL, "force is NULL");
  const long long *nw = reinterpret_cast<const long long *>(node_w);
  launch_grid(ctx->stream, ctx->geo, nw, ctx->dens, ctx->G);
  launch_force(ctx->stream, ctx->geo, ctx->P, ptrs(p), ctx->dens, ctx->G, force, ctx->err);
  rc = check_launch(ctx, "force");
  if (rc || !pe_or_null) return rc;
  int nb = launch_pe_nodes(ctx->stream, ctx->geo, ctx->dc, nw, ctx->partial_pe);
  launch_reduce_diag(ctx->stream, ctx->partial, 0, ctx->partial_pe, nb, ctx->diag_dev, 0);
  rc = check_launch(ctx, "potential energy");
  if (rc) return rc;
  pic_diag_t h;
  rc = hip_check(ctx, hipMemcpyAsync(&h, ctx->diag_dev, sizeof(h), hipMemcpyDeviceToHost, ctx->stream),
                 "copy diagnostics");
  if (rc) return rc;
  rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "stream synchronize");
  if (rc) return rc;
  std::memset(pe_or_null, 0, sizeof(*pe_or_null));
  pe_or_null->pe = h.pe;
  return PIC_OK;
}

int pic_kick(pic_ctx_t *ctx, pic_particles_t *p, const float *force, double frac) {
  if (!ctx) return PIC_EINVAL;
  int rc = check_particles(ctx, p, true, false);
  if (rc) return rc;
  if (p->n > 0 && !force) return fail(ctx, PIC_EINVAL, "force is NULL");
  if (!std::isfinite(frac)) return fail(ctx, PIC_EINVAL, "frac must be finite");
  launch_kick(ctx->stream, ctx->geo, ctx->P, ptrs(p), force, (float)frac);
  return check_launch(ctx, "kick");
}

int pic_push(pic_ctx_t *ctx, pic_particles_t *p, const float *force) {
  if (!ctx) return PIC_EINVAL;
  int rc = check_particles(ctx, p, true, false);
  if (rc) return rc;
  if (p->n > 0 && !force) return fail(ctx, PIC_EINVAL, "force is NULL");
  launch_push(ctx->stream, ctx->geo, ctx->P, ptrs(p), force, ctx->err);
  return check_launch(ctx, "push");
}

namespace {

struct DiagSink {
  pic_ctx_t *ctx;
  pic_diag_t *host;
  int slot = 0;
  int64_t copied = 0;
  int flush() {
    if (!slot) return PIC_OK;
    int r = hip_check(ctx, hipMemcpyAsync(host + copied, ctx->diag_dev, sizeof(pic_diag_t) * slot,
                                          hipMemcpyDeviceToHost, ctx->stream),
                      "copy diagnostics");
    if (r) return r;
    r = hip_check(ctx, hipStreamSynchronize(ctx->stream), "stream synchronize");
    copied += slot;
    slot = 0;
    return r;
  }
  pic_diag_t *next() { return ctx->diag_dev + slot; }
  int advance() {
    ++slot;
    return slot == kDiagCap ? flush() : PIC_OK;
  }
};

int step_untiled(pic_ctx_t *ctx, const PartPtrs &pp, int32_t nsteps, DiagSink &ds, int32_t diag_every) {
  for (int32_t s = 0; s < nsteps; ++s) {
    const bool want = ds.host && (s % diag_every) == 0;
    {
      PhaseTimer t(ctx, 0);
      launch_fill64(ctx->stream, ctx->node, ctx->sz.nnodes);
      launch_deposit_atomic(ctx->stream, ctx->geo, pp, ctx->node, ctx->err);
    }
    {
      PhaseTimer t(ctx, 1);
      launch_grid(ctx->stream, ctx->geo, ctx->node, ctx->dens, ctx->G);
    }
    int nbg = 0, nbp = 0;
    if (want) {
      PhaseTimer t(ctx, 4);
      nbg = launch_pe_nodes(ctx->stream, ctx->geo, ctx->dc, ctx->node, ctx->partial_pe);
    }
    {
      PhaseTimer t(ctx, 2);
      nbp = launch_force_push(ctx->stream, ctx->geo, ctx->P, ctx->dc, pp, ctx->dens, ctx->G, ctx->partial, want,
                              ctx->err);
    }
    if (want) {
      PhaseTimer t(ctx, 4);
      launch_reduce_diag(ctx->stream, ctx->partial, nbp, ctx->partial_pe, nbg, ds.next(), s);
    }
    int rc = check_launch(ctx, "step");
    if (rc) return rc;
    if (want && (rc = ds.advance())) return rc;
  }
  return PIC_OK;
}

int step_tiled(pic_ctx_t *ctx, const PartPtrs &pp, int32_t nsteps, DiagSink &ds, int32_t diag_every) {
  const Geo &g = ctx->geo;
  const int64_t n = pp.n;
  int cur = 0;
  const Store none{};
  // bring the caller's particles into the binned store; stop on invalid input
  {
    PhaseTimer t(ctx, 5);
    launch_bin(ctx->stream, g, ctx->tg, pp, none, ctx->st[cur], n, ctx->bb, true, ctx->err);
  }
  int rc = check_launch(ctx, "binning");
  if (rc) return rc;
  if ((rc = read_device_error(ctx))) return rc;
  const int64_t max_items = max_items_now(ctx, n);
  launch_fill64(ctx->stream, ctx->n3[0], ctx->sz.nnodes);
  launch_fill64(ctx->stream, ctx->n3[1], ctx->sz.nnodes);
  launch_fill32(ctx->stream, ctx->drift, 2);
  {
    PhaseTimer t(ctx, 0);
    launch_deposit_tiled(ctx->stream, g, ctx->tg, ctx->st[cur], ctx->bb, (int)max_items, ctx->n3[0]);
  }
  int since_bin = 0;
  ctx->drift_pending = false;
  for (int32_t s = 0; s < nsteps; ++s) {
    bool rebin = false;
    if (ctx->sort_every > 0) {
      rebin = s > 0 && s % ctx->sort_every == 0;
    } else if (ctx->sort_every < 0 && s > 0 && s % kDriftCheck == 0) {
      // adaptive: look at the drifter count copied kDriftCheck steps ago (long
      // finished, so the host does not stall), then post a copy of this one
      if (ctx->drift_pending) {
        (void)hipEventSynchronize(ctx->drift_ev);
        rebin = (int64_t)ctx->h_drift[0] * kDriftFraction > n || since_bin >= kMaxBinPeriod;
      }
      const int last = (s - 1) & 1;  // counter of the previous step
      (void)hipMemcpyAsync(ctx->h_drift, ctx->drift + last, sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
      (void)hipEventRecord(ctx->drift_ev, ctx->stream);
      ctx->drift_pending = true;
    }
    ++since_bin;
    if (rebin) {
      PhaseTimer t(ctx, 3);
      launch_bin(ctx->stream, g, ctx->tg, pp, ctx->st[cur], ctx->st[1 - cur], n, ctx->bb, false, ctx->err);
      cur = 1 - cur;
      since_bin = 0;
    }
    const bool want = ds.host && (s % diag_every) == 0;
    long long *Nc = ctx->n3[s % 3], *Nn = ctx->n3[(s + 1) % 3], *Nz = ctx->n3[(s + 2) % 3];
    const Drift dr{ctx->drift + 2, ctx->drift + (s & 1), ctx->drift + ((s + 1) & 1), (int)ctx->items_cap};
    int nbg = 0;
    if (want) {
      PhaseTimer t(ctx, 4);
      nbg = launch_pe_nodes(ctx->stream, g, ctx->dc, Nc, ctx->partial_pe);
    }
    {
      PhaseTimer t(ctx, 2);
      launch_step_tiled(ctx->stream, g, ctx->P, ctx->dc, ctx->tg, ctx->st[cur], ctx->bb, (int)max_items, Nc, Nn,
                        Nz, dr, ctx->partial, want, ctx->err);
    }
    {
      PhaseTimer t(ctx, 6);
      launch_drifters(ctx->stream, g, ctx->P, ctx->dc, ctx->tg, ctx->st[cur], Nc, Nn, dr, ctx->partial, want,
                      ctx->err);
    }
    if (want) {
      PhaseTimer t(ctx, 4);
      launch_reduce_diag_dev(ctx->stream, ctx->partial, ctx->bb.num_items, dr, ctx->partial_pe, nbg, ds.next(), s);
    }
    if ((rc = check_launch(ctx, "tiled step"))) return rc;
    if (want && (rc = ds.advance())) return rc;
  }
  {
    PhaseTimer t(ctx, 5);
    launch_export(ctx->stream, g, ctx->tg, ctx->st[cur], n, pp);
  }
  ctx->last_nodes = ctx->n3[nsteps % 3];
  ctx->last_step = nsteps - 1;
  return check_launch(ctx, "export");
}

}  // namespace

int pic_step(pic_ctx_t *ctx, pic_particles_t *p, int32_t nsteps, pic_diag_t *diag, int32_t diag_every) {
  if (!ctx) return PIC_EINVAL;
  int rc = check_particles(ctx, p, true, true);
  if (rc) return rc;
  if (nsteps < 0) return fail(ctx, PIC_EINVAL, "nsteps is negative");
  if (diag && diag_every < 1) return fail(ctx, PIC_EINVAL, "diag_every must be >= 1");
  DiagSink ds{ctx, diag};
  const PartPtrs pp = ptrs(p);
  ctx->last_nodes = nullptr;
  rc = (ctx->tiled && !ctx->force_untiled) ? step_tiled(ctx, pp, nsteps, ds, diag_every)
                                           : step_untiled(ctx, pp, nsteps, ds, diag_every);
  if (rc) return rc;
  if (diag && (rc = ds.flush())) return rc;
  return read_device_error(ctx);
}

int pic_step_nodes(pic_ctx_t *ctx, int64_t *node_w) {
  if (!ctx || !node_w) return PIC_EINVAL;
  if (!ctx->last_nodes) return fail(ctx, PIC_EINVAL, "no tiled pic_step has run on this context");
  return hip_check(ctx, hipMemcpyAsync(node_w, ctx->last_nodes, sizeof(long long) * (size_t)ctx->sz.nnodes,
                                       hipMemcpyDeviceToDevice, ctx->stream),
                   "copy node sums");
}

int pic_set_path(pic_ctx_t *ctx, int32_t untiled) {
  if (!ctx) return PIC_EINVAL;
  ctx->force_untiled = untiled != 0;
  return PIC_OK;
}

// ---------------------------------------------------------------------------
// Host calibration of the attractive correction factor (FP64).  The slab's
// node densities are those a flat commensurate lattice deposits: n_solid at
// every node inside, half of it on the surface node, zero beyond; the
// reflecting bottom wall keeps n_solid (half weight, half volume).
// ---------------------------------------------------------------------------
namespace {

struct Slab {
  int L;
  double h, nsolid;
  pic_potential_t pot;
  double node(int j) const { return j < 0 ? node(-j) : j < L ? nsolid : j == L ? 0.5 * nsolid : 0.0; }
  double centre_grad(int m) const {  // centre between nodes m and m+1 (mirror below the wall)
    if (m < 0) return -centre_grad(-1 - m);
    return (node(m + 1) - node(m)) / h;
  }
  double dphi(double r) const {
    double x6 = std::pow(pot.r0 / r, 6);
    double u = 12.0 * pot.D / r * (x6 - x6 * x6);
    return r < pot.r0 ? pot.s_rep * u : u;  // unit attractive multiplier
  }
  // normal force on a zero-weight atom at normal coordinate y (cells)
  double force(double y) const {
    int j = (int)std::floor(y);
    double f = y - j;
    double n = (1.0 - f) * node(j) + f * node(j + 1);
    int c0 = f >= 0.5 ? j : j - 1;
    double t = f >= 0.5 ? f - 0.5 : f + 0.5;
    double G = (1.0 - t) * centre_grad(c0) + t * centre_grad(c0 + 1);
    if (!(n > pot.n_floor)) return 0.0;
    double rbar = std::cbrt(1.0 / n);
    double g = -G / (3.0 * n) * rbar;  // d rbar/dx = -(1/3) n^(-4/3) dn/dx
    g = std::min(std::max(g, -pot.g_clamp), pot.g_clamp);
    return dphi(rbar / (1.0 - 0.5 * g)) - dphi(rbar / (1.0 + 0.5 * g));
  }
};

// Adaptive Simpson with an absolute tolerance proportional to the interval
// length (tol_per_len), so the recursion always terminates.
double simpson(const Slab &s, double a, double b, double fa, double fm, double fb, double whole,
               double tol_per_len, int depth) {
  double m = 0.5 * (a + b), lm = 0.5 * (a + m), rm = 0.5 * (m + b);
  double flm = s.force(lm), frm = s.force(rm);
  double left = (m - a) / 6.0 * (fa + 4.0 * flm + fm), right = (b - m) / 6.0 * (fm + 4.0 * frm + fb);
  double diff = left + right - whole;
  if (depth >= 50 || std::fabs(diff) <= 15.0 * tol_per_len * (b - a)) return left + right + diff / 15.0;
  return simpson(s, a, m, fa, flm, fm, left, tol_per_len, depth + 1) +
         simpson(s, m, b, fm, frm, fb, right, tol_per_len, depth + 1);
}

}  // namespace

int pic_calibrate_catt(const pic_grid_t *grid, const pic_potential_t *pot, double n_solid, int32_t slab_layers,
                       double *c_att, double *work) {
  Sizes sz;
  if (!grid_sizes(grid, &sz, nullptr) || !pot || !(n_solid > 0) || slab_layers < 2 || !c_att) return PIC_EINVAL;
  Slab s{slab_layers, grid->h[grid->ndim - 1], n_solid, *pot};
  const double y0 = 0.5 * slab_layers, y1 = slab_layers + 1.0;
  const int nscan = 8192;
  double ystar = -1.0, prev = s.force(y0);
  for (int k = 1; k <= nscan; ++k) {
    double y = y0 + (y1 - y0) * k / nscan, cur = s.force(y);
    if (prev > 0.0 && cur <= 0.0) {
      double a = y - (y1 - y0) / nscan, b = y;
      for (int it = 0; it < 200 && b - a > 0; ++it) {
        double m = 0.5 * (a + b);
        (s.force(m) > 0.0 ? a : b) = m;
      }
      ystar = 0.5 * (a + b);
    }
    prev = cur;
  }
  if (ystar < 0.0) return PIC_EINVAL;
  double fmax = 0.0;
  for (int k = 0; k <= nscan; ++k) fmax = std::max(fmax, std::fabs(s.force(y0 + (y1 - y0) * k / nscan)));
  const double tol = 1e-14 * fmax;
  double total = 0.0;
  for (double a = ystar; a < y1;) {  // split at the kinks: nodes and centres
    double b = std::min(std::floor(2.0 * a + 1.0) * 0.5, y1);
    double fa = s.force(a), fb = s.force(b), fm = s.force(0.5 * (a + b));
    total += simpson(s, a, b, fa, fm, fb, (b - a) / 6.0 * (fa + 4.0 * fm + fb), tol, 0);
    a = b;
  }
  double W = -total * s.h;
  if (!(W > 0)) return PIC_EINVAL;
  *c_att = pot->D / W;
  if (work) *work = W;
  return PIC_OK;
}

}  // extern "C"
