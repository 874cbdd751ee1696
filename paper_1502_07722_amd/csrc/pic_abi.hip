// C ABI of the PIC pair-potential library (declared in include/pic.h):
// argument validation, unit conversion, workspace carving, stream-ordered
// launches, graph replay and device-error reporting.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pic_crater.h"
#include "pic_internal.h"

using namespace pic;

// The static device array of pic_force_noalloc: node sums, node densities,
// cell-centred gradients and an error word for one grid.  Each GPU the
// library runs on holds its own copy until the process ends.  Host code never
// uses the array's name as an address: noalloc_scratch() looks the device
// address up once per device (hipGetSymbolAddress, with that device current)
// and keeps it.
static __device__ __align__(256) unsigned char scratch[PIC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kAlign = 256;
constexpr int kDiagCap = 1024;        // device diag entries buffered between host copies
constexpr int kMinChunk = 512;
constexpr int kMaxChunk = 32768;
constexpr int kDriftCheck = 48;       // adaptive re-binning looks at the drifter count this often
constexpr int kDriftFraction = 2048;  // and re-bins once drifters exceed n / kDriftFraction
constexpr int kMaxBinPeriod = 1024;   // or after this many steps
constexpr int kGraphSteps = 6;        // a replayed graph holds this many steps (node buffers x counters)
constexpr int kMaxSlabs = 1024;

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

pic_grid_t normalised(const pic_grid_t &in) {
  pic_grid_t g = in;
  if (g.ndim == 2) {
    g.n[2] = 1;
    g.bc[2] = 0;
    g.h[2] = g.depth2d > 0 ? g.depth2d : g.h[0];
    g.depth2d = g.h[2];
  }
  return g;
}

// Tiled path limits: packed cell coordinates.
bool tiled_supported(const pic_grid_t *g) {
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

struct Layout {
  size_t err, diag, partial, partial_pe, red, node, dens, G, Gbar, total;
  bool tiled;
  size_t store[2], bins, items, n3[3], drift, dacc, amax, slabs, offs;
  int64_t tiles_max, items_max, cap, nodes, pe_blocks;
};

size_t store_bytes(int ndim, int64_t cap) { return align_up((size_t)cap * 4 * (4 + ndim + 3)); }

// Workspace of a context of nslab slabs (the untiled single-slab buffers only
// when nslab == 1).
Layout make_layout(const pic_grid_t *grids, int nslab, const int64_t *max_n) {
  Layout L{};
  const int nd = grids[0].ndim;
  L.tiled = true;
  int64_t cells1 = 0;
  for (int k = 0; k < nslab; ++k) {
    Sizes s;
    grid_sizes(&grids[k], &s, nullptr);
    L.nodes += s.nnodes;
    L.cap += max_n[k];
    L.pe_blocks += std::max<int64_t>(blocks_of(s.nnodes), 1);
    L.tiles_max += tiles_for(&grids[k], min_tile_log2(nd));
    L.tiled = L.tiled && tiled_supported(&grids[k]);
    cells1 = s.ncells;
  }
  // 32-bit store slots and byte offsets, 32-bit node indices
  L.tiled = L.tiled && L.cap < (int64_t(1) << 30) && L.nodes < (int64_t(1) << 31);
  L.items_max = L.tiled ? L.tiles_max + (L.cap + kMinChunk - 1) / kMinChunk + nslab : 0;
  const int64_t partial_blocks = std::max<int64_t>(std::max<int64_t>(blocks_of(L.cap), L.items_max), 1);
  size_t o = 0;
  L.err = o; o = align_up(o + sizeof(uint32_t));
  L.diag = o; o = align_up(o + sizeof(pic_diag_t) * kDiagCap);
  L.partial = o; o = align_up(o + sizeof(double) * 8 * (size_t)partial_blocks);
  L.partial_pe = o; o = align_up(o + sizeof(double) * 8 * (size_t)L.pe_blocks);
  L.red = o; o = align_up(o + sizeof(double) * kDiagRedDoubles);
  if (nslab == 1) {
    L.node = o; o = align_up(o + sizeof(long long) * (size_t)L.nodes);
    L.dens = o; o = align_up(o + sizeof(float) * (size_t)L.nodes);
    L.G = o; o = align_up(o + sizeof(float) * (size_t)cells1 * nd);
    L.Gbar = o; o = align_up(o + sizeof(float) * (size_t)cells1 * nd);
  }
  if (L.tiled) {
    const int64_t cap = std::max<int64_t>(L.cap, 1);
    for (int k = 0; k < 2; ++k) { L.store[k] = o; o += store_bytes(nd, cap); }
    L.bins = o; o = align_up(o + sizeof(int) * (size_t)(4 * L.tiles_max + 4));
    L.items = o; o = align_up(o + sizeof(Item) * (size_t)L.items_max);
    for (int k = 0; k < 3; ++k) { L.n3[k] = o; o = align_up(o + sizeof(long long) * (size_t)L.nodes); }
    L.drift = o; o = align_up(o + sizeof(int) * (size_t)(cap + 4));
    L.dacc = o; o = align_up(o + sizeof(double) * 8 * (size_t)nslab);
    L.amax = o; o = align_up(o + sizeof(uint32_t) * 2);
    L.slabs = o; o = align_up(o + sizeof(SlabDesc) * (size_t)nslab);
    L.offs = o; o = align_up(o + sizeof(int) * (size_t)(2 * (nslab + 1)));
  }
  L.total = o;
  return L;
}

bool valid_potential(const pic_potential_t *pot) {
  if (!pot) return false;
  const pic_potential_t &P = *pot;
  if (P.kind != PIC_POT_LJ && P.kind != PIC_POT_MORSE) return false;
  if (P.lattice != PIC_LATTICE_CUBIC && P.lattice != PIC_LATTICE_HCP) return false;
  if (P.kind == PIC_POT_MORSE && !(P.alpha > 0 && std::isfinite(P.alpha))) return false;
  return P.D > 0 && P.r0 > 0 && P.s_rep > 0 && P.c_att > 0 && P.g_clamp > 0 && P.g_clamp < 2 &&
         P.n_floor >= 0 && P.mass > 0 && std::isfinite(P.s_rep) && std::isfinite(P.c_att) &&
         std::isfinite(P.D) && std::isfinite(P.r0) && std::isfinite(P.mass);
}

// Work items of a tiling at a given chunk: sum over tiles of ceil(count / chunk).
int64_t items_at(const std::vector<int> &counts, int chunk) {
  int64_t n = 0;
  for (int c : counts) n += (c + chunk - 1) / chunk;
  return n;
}

// Chunks (multiples of 64 in [kMinChunk, kMaxChunk]) whose item count is at
// most r whole rounds of the persistent grid and fills at least 90 % of the
// last round, r = 1..8: the smallest such chunk per r.
std::vector<int> balanced_chunks(const std::vector<int> &counts, int slots) {
  std::vector<int> out;
  if (slots < 1) return out;
  for (int r = 1; r <= 8; ++r) {
    int lo = kMinChunk, hi = kMaxChunk;
    if (items_at(counts, hi) > (int64_t)r * slots) continue;
    while (hi - lo > 64) {  // smallest chunk with items <= r * slots
      const int mid = (lo + hi) / 2 / 64 * 64;
      if (mid <= lo) break;
      (items_at(counts, mid) <= (int64_t)r * slots ? hi : lo) = mid;
    }
    const int64_t n = items_at(counts, hi);
    if (n * 10 >= (int64_t)r * slots * 9 && n > (int64_t)(r - 1) * slots) out.push_back(hi);
  }
  return out;
}

// Nodes and weights of the 16-point Gauss-Legendre rule: the roots of P_16
// by Newton's method from the usual cosine estimates, w = 2 / ((1 - x^2) P'^2).
Quad16 gauss_legendre16() {
  Quad16 q{};
  const int n = 16;
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;  // Legendre recurrence up to P_n
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    q.x[i] = x;
    q.w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  return q;
}

// Grid constants in the kernels' reduced units.
Geo make_geo(const pic_grid_t &g, const pic_potential_t &P, double dt, const Sizes &s) {
  Geo G;
  std::memset(&G, 0, sizeof(G));
  const double V = g.h[0] * g.h[1] * g.h[2];
  const double r3 = P.r0 * P.r0 * P.r0;
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
  return G;
}

// Potential constants in the kernels' reduced units (length r0, energy D).
Pot make_pot(const pic_potential_t &P, double dt) {
  Pot Q{};
  const double r3 = P.r0 * P.r0 * P.r0;
  Q.nfloor = (float)(P.n_floor * r3);
  Q.gclamp = (float)P.g_clamp;
  Q.hgclamp = 0.5f * Q.gclamp;
  Q.s_rep = (float)P.s_rep;
  Q.c_att = (float)P.c_att;
  Q.beta = (float)(12.0 * P.D / P.r0);
  Q.gv = (float)(dt / P.mass);
  Q.kind = P.kind;
  Q.mAl2 = P.kind == PIC_POT_MORSE ? (float)(P.alpha * P.r0 * M_LOG2E) : 0.0f;
  Q.mA6 = P.kind == PIC_POT_MORSE ? (float)(P.alpha * P.r0 / 6.0) : 0.0f;
  Q.mAt = 6.0f * Q.mA6 * Q.mA6;
  Q.lattice = P.lattice;
  Q.ks = 1.0f;
  return Q;
}

// The device address of the static scratch array on each device (see its
// definition at the top of the file).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The current device's address of the array (out may be NULL: look up only).
int noalloc_scratch(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PIC_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(::scratch)) != hipSuccess || !ptr) return PIC_EHIP;
    g_scratch_ptr[dev] = ptr;
  }
  if (out) *out = g_scratch_ptr[dev];
  return PIC_OK;
}

DiagC make_diag(const pic_grid_t &g, const pic_potential_t &P) {
  const double V = g.h[0] * g.h[1] * g.h[2];
  return DiagC{P.D, P.mass, 0.5 * P.mass, std::ldexp(1.0, -20), V, P.r0 * P.r0 * P.r0, P.s_rep, P.c_att,
               P.kind, P.kind == PIC_POT_MORSE ? P.alpha * P.r0 : 0.0, P.lattice};
}

}  // namespace

struct pic_ctx {
  // problem
  int nslab = 1;
  int ndim = 2;
  std::vector<pic_grid_t> grids;
  std::vector<int64_t> max_n;
  std::vector<Sizes> sizes;
  pic_potential_t pot{};
  double dt = 0;
  char *ws = nullptr;
  hipStream_t stream = nullptr;
  Pot P{};
  std::vector<DiagC> dcs;  // per slab (cell volume)
  Quad16 quad{};           // Gauss-Legendre rule of the Morse energy density
  // shared buffers
  uint32_t *err = nullptr;
  pic_diag_t *diag_dev = nullptr;
  double *partial = nullptr;
  double *partial_pe = nullptr;
  double *red = nullptr;  // second-level diagnostics sums
  std::vector<int> pe_off;  // first energy-partial block of each slab
  std::string last_error;
  // untiled single-slab path
  Geo geo{};
  long long *node = nullptr;
  float *dens = nullptr;
  float *G = nullptr;
  float *Gbar = nullptr;  // centre-gradient cotangent (reverse mode)
  bool force_untiled = false;
  // tiled path
  bool tiled = false;
  int lt = 4, ltl = 4, halo = 2, chunk = 8192, sort_every = -1;  // ltl: tile edge exponent, last axis
  std::vector<SlabDesc> sd;  // host copy of the slab table
  SlabDesc *sd_dev = nullptr;
  int *part_offs_dev = nullptr, *tile_offs_dev = nullptr;
  int ntiles = 0, nnodes = 0;
  int64_t cap = 0, items_cap = 0;
  Store st[2]{};
  BinBufs bb{};
  long long *n3[3]{};
  int *drift = nullptr;  // [count0, count1, work0, work1][list]
  double *dacc = nullptr;
  uint32_t *amax = nullptr;  // [2] largest node-cotangent contribution, this / previous reverse step
  int grid_blocks = 0;   // persistent grid of the fused kernel
  int *h_drift = nullptr;
  hipEvent_t drift_ev = nullptr;
  bool drift_pending = false;
  long long *last_nodes = nullptr;
  int last_step = 0;
  // recorded trajectories (reverse mode)
  std::vector<int64_t> rec_key;  // configuration of the last pic_forward_record
  std::vector<char> rec_rebinned;  // checkpoints whose binning differs from the previous one
  bool rec_all = false;            // records keep every state and node sum (no recompute)
  // graph replay of steady steps
  bool use_graph = true;
  hipGraphExec_t graph[2]{};
  std::vector<int64_t> graph_key;
  // event timing of pic_step phases
  bool timing = false;
  pic_timing_t tacc{};
  std::vector<hipEvent_t> ev_pool;
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

static int check_launch(pic_ctx_t *ctx, const char *what) { return hip_check(ctx, hipGetLastError(), what); }

static int check_particles(pic_ctx_t *ctx, const pic_particles_t *p, int64_t max_n, bool need_vel, bool need_wq) {
  if (!p) return fail(ctx, PIC_EINVAL, "particles is NULL");
  if (p->n < 0) return fail(ctx, PIC_EINVAL, "particle count is negative");
  if (p->n > max_n) return fail(ctx, PIC_ENOSPACE, "particle count exceeds max_n of the context");
  if (p->n == 0) return PIC_OK;
  if (!p->cell || !p->off) return fail(ctx, PIC_EINVAL, "cell or off is NULL");
  if (need_vel && !p->vel) return fail(ctx, PIC_EINVAL, "vel is NULL");
  if (need_wq && !p->wq) return fail(ctx, PIC_EINVAL, "wq is NULL");
  return PIC_OK;
}

static PartPtrs ptrs(const pic_particles_t *p) { return PartPtrs{p->n, p->cell, p->off, p->vel, p->wq}; }

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

static void drop_graphs(pic_ctx_t *c) {
  for (auto &g : c->graph)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  c->graph_key.clear();
}

// Apply a tiling to every slab (tiles of 2^lt cells along every axis but the
// last and 2^ltl along the last, halo, chunk, re-binning period) and upload
// the slab table.
static int apply_tiling(pic_ctx_t *c, int lt, int ltl, int halo, int chunk, int sort_every) {
  const int nd = c->ndim;
  if (lt < min_tile_log2(nd) || lt > max_tile_log2(nd)) return fail(c, PIC_EINVAL, "tile edge out of range");
  if (ltl < min_tile_log2(nd) || ltl > lt)
    return fail(c, PIC_EINVAL, "last-axis tile edge out of range (smallest tile edge .. tile)");
  if (halo < 1 || halo > 4) return fail(c, PIC_EINVAL, "halo must be 1..4 cells");
  if (chunk < kMinChunk || chunk > kMaxChunk) return fail(c, PIC_EINVAL, "chunk out of range");
  if (sort_every < -1) return fail(c, PIC_EINVAL, "sort_every must be >= -1");
  TileGeo T{};
  for (int d = 0; d < 3; ++d) T.lt[d] = d < nd - 1 ? lt : (d == nd - 1 ? ltl : 0);
  T.H = halo;
  T.chunk = chunk;
  T.pshift[0] = 0;
  T.pshift[1] = nd == 2 ? 16 : 11;
  T.pshift[2] = nd == 2 ? 31 : 22;
  T.pmask[0] = nd == 2 ? 0xFFFF : 0x7FF;
  T.pmask[1] = nd == 2 ? 0x7FFF : 0x7FF;
  T.pmask[2] = nd == 2 ? 0 : 0x1FF;
  if (window_lds_bytes(T, nd) > 64 * 1024) return fail(c, PIC_EINVAL, "tile window does not fit in LDS");
  std::vector<SlabDesc> sd(c->nslab);
  int tiles = 0, nodes = 0;
  for (int k = 0; k < c->nslab; ++k) {
    const pic_grid_t &g = c->grids[k];
    for (int d = 0; d < nd; ++d)  // periodic axes must hold a whole window (single-wrap window coordinates)
      if (!g.bc[d] && g.n[d] < (1 << T.lt[d]) + 2 * halo + 3)
        return fail(c, PIC_EINVAL, "a periodic axis is shorter than the tile window");
    SlabDesc &s = sd[k];
    s.g = make_geo(g, c->pot, c->dt, c->sizes[k]);
    s.tg = T;
    s.tg.ntiles = 1;
    for (int d = 0; d < 3; ++d) {
      s.tg.tn[d] = d < nd ? (g.n[d] + (1 << T.lt[d]) - 1) >> T.lt[d] : 1;
      s.tg.ntiles *= s.tg.tn[d];
    }
    s.node_off = nodes;
    s.tile_off = tiles;
    s.part_off = k < (int)c->sd.size() ? c->sd[k].part_off : 0;
    s.part_n = k < (int)c->sd.size() ? c->sd[k].part_n : 0;
    nodes += (int)c->sizes[k].nnodes;
    tiles += s.tg.ntiles;
  }
  c->sd = sd;
  c->ntiles = tiles;
  c->nnodes = nodes;
  c->lt = lt;
  c->ltl = ltl;
  c->halo = halo;
  c->chunk = chunk;
  c->sort_every = sort_every;
  std::vector<int> toffs(c->nslab + 1);
  for (int k = 0; k < c->nslab; ++k) toffs[k] = sd[k].tile_off;
  toffs[c->nslab] = tiles;
  int rc = hip_check(c, hipMemcpy(c->sd_dev, sd.data(), sizeof(SlabDesc) * c->nslab, hipMemcpyHostToDevice),
                     "upload slab table");
  if (!rc)
    rc = hip_check(c, hipMemcpy(c->tile_offs_dev, toffs.data(), sizeof(int) * toffs.size(), hipMemcpyHostToDevice),
                   "upload tile offsets");
  if (rc) return rc;
  c->grid_blocks = 0;
  drop_graphs(c);
  return PIC_OK;
}

// Per-call store layout: slab k owns slots [part_off_k, part_off_k + n_k).
static int bind_counts(pic_ctx_t *c, const pic_particles_t *parts) {
  std::vector<int> poffs(c->nslab + 1);
  int64_t off = 0;
  for (int k = 0; k < c->nslab; ++k) {
    c->sd[k].part_off = (int)off;
    c->sd[k].part_n = (int)parts[k].n;
    poffs[k] = (int)off;
    off += parts[k].n;
  }
  poffs[c->nslab] = (int)off;
  int rc = hip_check(c, hipMemcpyAsync(c->sd_dev, c->sd.data(), sizeof(SlabDesc) * c->nslab,
                                       hipMemcpyHostToDevice, c->stream),
                     "upload slab table");
  if (!rc)
    rc = hip_check(c, hipMemcpyAsync(c->part_offs_dev, poffs.data(), sizeof(int) * poffs.size(),
                                     hipMemcpyHostToDevice, c->stream),
                   "upload slot offsets");
  if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "stream synchronize");
  return rc;
}

static Batch batch_of(const pic_ctx_t *c, int64_t nparts) {
  return Batch{c->sd_dev, c->part_offs_dev, c->tile_offs_dev, c->nslab, c->ntiles, c->nnodes, (int)nparts};
}

// Create a context for nslab slabs; shared by pic_init and pic_init_batch.
static int init_common(pic_ctx_t **out, const pic_grid_t *grids_in, int nslab, const pic_potential_t *pot,
                       double dt, const int64_t *max_n, void *ws, size_t ws_bytes, void *stream) {
  if (!out) return PIC_EINVAL;
  *out = nullptr;
  if (!grids_in || !max_n || nslab < 1 || nslab > kMaxSlabs) return PIC_EINVAL;
  std::vector<pic_grid_t> grids(nslab);
  std::vector<Sizes> sizes(nslab);
  for (int k = 0; k < nslab; ++k) {
    if (!grid_sizes(&grids_in[k], &sizes[k], nullptr)) return PIC_EINVAL;
    if (grids_in[k].ndim != grids_in[0].ndim) return PIC_EINVAL;
    if (max_n[k] < 0 || max_n[k] >= (int64_t(1) << 40)) return PIC_EINVAL;
    grids[k] = normalised(grids_in[k]);
  }
  if (!valid_potential(pot)) return PIC_EINVAL;
  if (!(dt > 0) || !std::isfinite(dt)) return PIC_EINVAL;
  Layout L = make_layout(grids.data(), nslab, max_n);
  if (nslab > 1 && !L.tiled) return PIC_EINVAL;  // batches need the tiled path
  if (!ws || ws_bytes < L.total) return PIC_ENOSPACE;
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return PIC_EINVAL;

  pic_ctx_t *c = new pic_ctx_t();
  c->nslab = nslab;
  c->ndim = grids[0].ndim;
  c->grids = grids;
  c->max_n.assign(max_n, max_n + nslab);
  c->sizes = sizes;
  c->pot = *pot;
  c->dt = dt;
  c->ws = static_cast<char *>(ws);
  c->stream = static_cast<hipStream_t>(stream);
  const pic_potential_t &P = *pot;
  c->P = make_pot(P, dt);
  (void)noalloc_scratch(nullptr);  // look the static scratch array up on this device now
  c->quad = gauss_legendre16();
  int pe = 0;
  for (int k = 0; k < nslab; ++k) {
    c->dcs.push_back(make_diag(grids[k], P));
    c->pe_off.push_back(pe);
    pe += (int)std::max<int64_t>(blocks_of(sizes[k].nnodes), 1);
  }
  c->err = reinterpret_cast<uint32_t *>(c->ws + L.err);
  c->diag_dev = reinterpret_cast<pic_diag_t *>(c->ws + L.diag);
  c->partial = reinterpret_cast<double *>(c->ws + L.partial);
  c->partial_pe = reinterpret_cast<double *>(c->ws + L.partial_pe);
  c->red = reinterpret_cast<double *>(c->ws + L.red);
  if (nslab == 1) {
    c->geo = make_geo(grids[0], P, dt, sizes[0]);
    c->node = reinterpret_cast<long long *>(c->ws + L.node);
    c->dens = reinterpret_cast<float *>(c->ws + L.dens);
    c->G = reinterpret_cast<float *>(c->ws + L.G);
    c->Gbar = reinterpret_cast<float *>(c->ws + L.Gbar);
  }
  c->tiled = L.tiled;
  if (L.tiled) {
    const int64_t cap = std::max<int64_t>(L.cap, 1);
    c->cap = cap;
    c->items_cap = L.items_max;
    for (int k = 0; k < 2; ++k) {
      char *b = c->ws + L.store[k];
      Store &S = c->st[k];
      S.cap = cap;
      S.pc = reinterpret_cast<int *>(b);
      S.off = reinterpret_cast<float *>(b + 4 * cap);
      S.vel = reinterpret_cast<float *>(b + 4 * cap * (1 + c->ndim));
      S.wq = reinterpret_cast<int *>(b + 4 * cap * (4 + c->ndim));
      S.oidx = reinterpret_cast<int *>(b + 4 * cap * (5 + c->ndim));
    }
    int *bi = reinterpret_cast<int *>(c->ws + L.bins);
    const int64_t T = L.tiles_max;
    c->bb.counts = bi;
    c->bb.starts = bi + T;
    c->bb.cursors = bi + 2 * T + 1;
    c->bb.item_start = bi + 3 * T + 1;
    c->bb.num_items = bi + 4 * T + 2;
    c->bb.items = reinterpret_cast<Item *>(c->ws + L.items);
    for (int k = 0; k < 3; ++k) c->n3[k] = reinterpret_cast<long long *>(c->ws + L.n3[k]);
    c->drift = reinterpret_cast<int *>(c->ws + L.drift);
    c->dacc = reinterpret_cast<double *>(c->ws + L.dacc);
    c->amax = reinterpret_cast<uint32_t *>(c->ws + L.amax);
    c->sd_dev = reinterpret_cast<SlabDesc *>(c->ws + L.slabs);
    c->part_offs_dev = reinterpret_cast<int *>(c->ws + L.offs);
    c->tile_offs_dev = c->part_offs_dev + nslab + 1;
    // default tiling: 16^2 (2D) / 8^3 (3D) tiles, smaller where a periodic axis is short
    int rc = PIC_EINVAL;
    if (c->ndim == 2) {
      for (int lt = 4; lt >= 3 && rc && rc != PIC_EHIP; --lt) rc = apply_tiling(c, lt, lt, 2, 8192, -1);
      if (rc && rc != PIC_EHIP) rc = apply_tiling(c, 3, 3, 1, 8192, -1);
    } else {
      for (int lt = 3; lt >= 2 && rc && rc != PIC_EHIP; --lt) rc = apply_tiling(c, lt, lt, 1, 4096, -1);
    }
    if (rc == PIC_EHIP) {
      delete c;
      return PIC_EHIP;
    }
    if (rc) c->tiled = false;
    c->last_error.clear();
    if (c->tiled && (hipHostMalloc((void **)&c->h_drift, 16, hipHostMallocDefault) != hipSuccess ||
                     hipEventCreateWithFlags(&c->drift_ev, hipEventDisableTiming) != hipSuccess)) {
      c->h_drift = nullptr;
      c->tiled = false;
    }
    if (!c->tiled && nslab > 1) {
      delete c;
      return PIC_EINVAL;
    }
  }
  launch_clear_word(c->stream, c->err);
  if (c->tiled) launch_fill64(c->stream, reinterpret_cast<long long *>(c->dacc), 8 * nslab);
  if (hipGetLastError() != hipSuccess) {
    delete c;
    return PIC_EHIP;
  }
  *out = c;
  return PIC_OK;
}

namespace {

// Diagnostics: device entries (step-major, slab-minor) copied out in blocks
// into the caller's [nslab][ndiag] array.
struct DiagSink {
  pic_ctx_t *ctx;
  pic_diag_t *host;
  int64_t ndiag;
  int slot = 0;
  int64_t step_index = 0;  // diag steps already copied
  std::vector<pic_diag_t> stage;
  int flush() {
    if (!slot) return PIC_OK;
    stage.resize(slot);
    int r = hip_check(ctx, hipMemcpyAsync(stage.data(), ctx->diag_dev, sizeof(pic_diag_t) * slot,
                                          hipMemcpyDeviceToHost, ctx->stream),
                      "copy diagnostics");
    if (r) return r;
    r = hip_check(ctx, hipStreamSynchronize(ctx->stream), "stream synchronize");
    if (r) return r;
    const int ns = ctx->nslab;
    for (int e = 0; e < slot; ++e) host[(int64_t)(e % ns) * ndiag + step_index + e / ns] = stage[e];
    step_index += slot / ns;
    slot = 0;
    return PIC_OK;
  }
  pic_diag_t *next() { return ctx->diag_dev + slot; }
  int advance(int entries) {
    slot += entries;
    return slot + ctx->nslab > kDiagCap ? flush() : PIC_OK;
  }
};

int step_untiled(pic_ctx_t *ctx, const PartPtrs &pp, int32_t nsteps, DiagSink &ds, int32_t diag_every) {
  for (int32_t s = 0; s < nsteps; ++s) {
    const bool want = ds.host && (s % diag_every) == 0;
    {
      PhaseTimer t(ctx, 0);
      launch_fill64(ctx->stream, ctx->node, ctx->sizes[0].nnodes);
      launch_deposit_atomic(ctx->stream, ctx->geo, pp, ctx->node, ctx->err);
    }
    {
      PhaseTimer t(ctx, 1);
      launch_grid(ctx->stream, ctx->geo, ctx->node, ctx->dens, ctx->G);
    }
    int nbg = 0, nbp = 0;
    if (want) {
      PhaseTimer t(ctx, 4);
      nbg = launch_pe_nodes(ctx->stream, ctx->geo, ctx->dcs[0], ctx->quad, ctx->node, ctx->partial_pe);
    }
    {
      PhaseTimer t(ctx, 2);
      nbp = launch_force_push(ctx->stream, ctx->geo, ctx->P, ctx->dcs[0], pp, ctx->dens, ctx->G, ctx->partial, want,
                              ctx->err);
    }
    if (want) {
      PhaseTimer t(ctx, 4);
      launch_reduce_diag(ctx->stream, ctx->partial, nbp, ctx->partial_pe, nbg, ds.next(), s);
    }
    int rc = check_launch(ctx, "step");
    if (rc) return rc;
    if (want && (rc = ds.advance(1))) return rc;
  }
  return PIC_OK;
}

void ensure_grid_blocks(pic_ctx_t *c) {
  if (c->grid_blocks) return;
  int dev = 0, ncu = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0) ncu = 256;
  c->grid_blocks = ncu * step_kernel_blocks_per_cu(c->ndim, c->sd[0].tg);
}

Drift drift_of(pic_ctx_t *c, int s) {
  return Drift{c->drift + 4, c->drift + (s & 1), c->drift + ((s + 1) & 1), c->drift + 2 + (s & 1),
               c->drift + 2 + ((s + 1) & 1)};
}

// Most work items of a binning of n particles: one per tile plus one per chunk.
int64_t max_items_of(const pic_ctx_t *c, int64_t n) { return (int64_t)c->ntiles + (n + c->chunk - 1) / c->chunk; }

// Persistent grid of the fused kernel for n particles: the full grid, or
// fewer blocks when the step cannot have that many work items; extra blocks
// would only find the queue empty, and launching them costs more than the
// step on a small grid.
int step_grid(const pic_ctx_t *c, int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(c->grid_blocks, max_items_of(c, n)));
}

// The launch of one tiled step: one fused kernel (drifters included).
void enqueue_step(pic_ctx_t *c, const Batch &b, const Store &st, int s, bool diag) {
  long long *Nc = c->n3[s % 3], *Nn = c->n3[(s + 1) % 3], *Nz = c->n3[(s + 2) % 3];
  const Drift dr = drift_of(c, s);
  PhaseTimer t(c, 2);
  launch_step_tiled(c->stream, c->ndim, c->sd[0].tg, c->P, c->dcs[0], b, st, st, c->bb, step_grid(c, b.nparts), Nc,
                    Nn, Nz, dr, c->partial, diag, c->err);
}

// Graph of kGraphSteps plain steps starting at a step index that is a
// multiple of kGraphSteps (node buffers cycle with period 3, counters 2).
int graph_for(pic_ctx_t *c, const Batch &b, int cur, hipGraphExec_t *out) {
  std::vector<int64_t> key = {b.nparts, c->lt, c->ltl, c->halo, c->chunk, c->grid_blocks, c->nslab};
  for (const SlabDesc &s : c->sd) {
    key.push_back(s.part_off);
    key.push_back(s.part_n);
  }
  if (c->graph_key != key) {
    drop_graphs(c);
    c->graph_key = key;
  }
  if (c->graph[cur]) {
    *out = c->graph[cur];
    return PIC_OK;
  }
  const bool timing = c->timing;
  c->timing = false;  // no event records inside a capture
  hipGraph_t g = nullptr;
  int rc = hip_check(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal), "begin capture");
  if (rc) {
    c->timing = timing;
    return rc;
  }
  for (int s = 0; s < kGraphSteps; ++s) enqueue_step(c, b, c->st[cur], s, false);
  rc = hip_check(c, hipStreamEndCapture(c->stream, &g), "end capture");
  c->timing = timing;
  if (rc) return rc;
  rc = hip_check(c, hipGraphInstantiate(&c->graph[cur], g, nullptr, nullptr, 0), "instantiate graph");
  (void)hipGraphDestroy(g);
  if (rc) return rc;
  *out = c->graph[cur];
  return PIC_OK;
}

// Steps [s, s + kGraphSteps) are plain: no diagnostics, no re-binning and no
// adaptive check inside, and s is a multiple of kGraphSteps.
bool plain_block(const pic_ctx_t *c, int s, int nsteps, int since_bin, bool diag, int diag_every) {
  if (s % kGraphSteps || s + kGraphSteps > nsteps) return false;
  if (since_bin + kGraphSteps >= kMaxBinPeriod) return false;
  for (int k = 0; k < kGraphSteps; ++k) {
    const int t = s + k;
    if (diag && t % diag_every == 0) return false;
    if (c->sort_every > 0 && t > 0 && t % c->sort_every == 0) return false;
    if (c->sort_every < 0 && t > 0 && t % kDriftCheck == 0) return false;
  }
  return true;
}

int step_tiled(pic_ctx_t *ctx, const pic_particles_t *parts, int32_t nsteps, DiagSink &ds, int32_t diag_every,
               bool export_back = true, float *probe_ms = nullptr) {
  const int nd = ctx->ndim;
  int rc = bind_counts(ctx, parts);
  if (rc) return rc;
  int64_t n = 0;
  std::vector<PartPtrs> cps(ctx->nslab);
  for (int k = 0; k < ctx->nslab; ++k) {
    cps[k] = ptrs(&parts[k]);
    n += parts[k].n;
  }
  const Batch b = batch_of(ctx, n);
  ensure_grid_blocks(ctx);
  int cur = 0;
  // bring the caller's particles into the binned store; stop on invalid input
  {
    PhaseTimer t(ctx, 5);
    launch_import(ctx->stream, nd, ctx->sd.data(), cps.data(), ctx->nslab, ctx->bb, b, ctx->chunk, ctx->st[cur],
                  ctx->st[1 - cur].oidx, ctx->err);
  }
  if ((rc = check_launch(ctx, "binning"))) return rc;
  if ((rc = read_device_error(ctx))) return rc;
  const int64_t max_items = max_items_of(ctx, n);
  launch_fill64(ctx->stream, ctx->n3[0], ctx->nnodes);
  launch_fill64(ctx->stream, ctx->n3[1], ctx->nnodes);
  launch_fill32(ctx->stream, ctx->drift, 4);
  {
    PhaseTimer t(ctx, 0);
    launch_deposit_tiled(ctx->stream, nd, ctx->sd[0].tg, b, ctx->st[cur], ctx->bb, (int)max_items, ctx->n3[0]);
  }
  int since_bin = 0;
  ctx->drift_pending = false;
  hipEvent_t pa = nullptr, pb = nullptr;
  if (probe_ms) {
    pa = take_event(ctx);
    pb = take_event(ctx);
    if (!pa || !pb) return fail(ctx, PIC_EHIP, "event creation failed");
    (void)hipEventRecord(pa, ctx->stream);
  }
  for (int32_t s = 0; s < nsteps;) {
    // graphs need a capturable stream: never the legacy default (NULL) stream
    if (ctx->use_graph && !ctx->timing && ctx->stream != nullptr &&
        plain_block(ctx, s, nsteps, since_bin, ds.host != nullptr, diag_every)) {
      hipGraphExec_t ge = nullptr;
      if ((rc = graph_for(ctx, b, cur, &ge))) return rc;
      {
        PhaseTimer t(ctx, 7);
        rc = hip_check(ctx, hipGraphLaunch(ge, ctx->stream), "graph launch");
      }
      if (rc) return rc;
      s += kGraphSteps;
      since_bin += kGraphSteps;
      continue;
    }
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
      const int last = (s - 1) & 1;  // drifter counter of the previous step
      (void)hipMemcpyAsync(ctx->h_drift, ctx->drift + last, sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
      (void)hipEventRecord(ctx->drift_ev, ctx->stream);
      ctx->drift_pending = true;
    }
    if (rebin) {
      PhaseTimer t(ctx, 3);
      launch_rebin(ctx->stream, nd, ctx->bb, b, ctx->chunk, ctx->st[cur], ctx->st[1 - cur]);
      cur = 1 - cur;
      since_bin = 0;
    }
    const bool want = ds.host && (s % diag_every) == 0;
    if (want) {
      PhaseTimer t(ctx, 4);
      for (int k = 0; k < ctx->nslab; ++k)
        launch_pe_nodes(ctx->stream, ctx->sd[k].g, ctx->dcs[k], ctx->quad, ctx->n3[s % 3] + ctx->sd[k].node_off,
                        ctx->partial_pe + (int64_t)ctx->pe_off[k] * 8);
    }
    enqueue_step(ctx, b, ctx->st[cur], s, want);
    if (want) {
      PhaseTimer t(ctx, 4);
      for (int k = 0; k < ctx->nslab; ++k) {
        const int nbg = (int)std::max<int64_t>(blocks_of(ctx->sizes[k].nnodes), 1);
        launch_reduce_diag_slab(ctx->stream, ctx->partial, ctx->bb.item_start, ctx->sd[k].tile_off,
                                ctx->sd[k].tile_off + ctx->sd[k].tg.ntiles,
                                ctx->partial_pe + (int64_t)ctx->pe_off[k] * 8, nbg, ctx->red, ds.next() + k, s);
      }
    }
    if ((rc = check_launch(ctx, "tiled step"))) return rc;
    if (want && (rc = ds.advance(ctx->nslab))) return rc;
    ++s;
    ++since_bin;
  }
  if (probe_ms) {
    (void)hipEventRecord(pb, ctx->stream);
    rc = hip_check(ctx, hipEventSynchronize(pb), "probe sync");
    if (!rc) rc = hip_check(ctx, hipEventElapsedTime(probe_ms, pa, pb), "probe time");
    ctx->ev_pool.push_back(pa);
    ctx->ev_pool.push_back(pb);
    if (rc) return rc;
  }
  if (export_back) {
    PhaseTimer t(ctx, 5);
    for (int k = 0; k < ctx->nslab; ++k) launch_export(ctx->stream, nd, ctx->sd[k], ctx->st[cur], ctx->bb, cps[k]);
  }
  ctx->last_nodes = ctx->n3[nsteps % 3];
  ctx->last_step = nsteps - 1;
  return check_launch(ctx, "export");
}

}  // namespace

extern "C" {

int64_t pic_num_nodes(const pic_grid_t *grid) {
  Sizes s;
  return grid_sizes(grid, &s, nullptr) ? s.nnodes : 0;
}

size_t pic_workspace_bytes_batch(const pic_grid_t *grids, int32_t nslab, const int64_t *max_n) {
  if (!grids || !max_n || nslab < 1 || nslab > kMaxSlabs) return 0;
  std::vector<pic_grid_t> g(nslab);
  for (int k = 0; k < nslab; ++k) {
    Sizes s;
    if (!grid_sizes(&grids[k], &s, nullptr) || max_n[k] < 0 || grids[k].ndim != grids[0].ndim) return 0;
    g[k] = normalised(grids[k]);
  }
  Layout L = make_layout(g.data(), nslab, max_n);
  if (nslab > 1 && !L.tiled) return 0;
  return L.total;
}

size_t pic_workspace_bytes(const pic_grid_t *grid, int64_t max_n) {
  return pic_workspace_bytes_batch(grid, 1, &max_n);
}

int pic_init(pic_ctx_t **out, const pic_grid_t *grid, const pic_potential_t *pot, double dt, int64_t max_n,
             void *ws, size_t ws_bytes, void *stream) {
  return init_common(out, grid, 1, pot, dt, &max_n, ws, ws_bytes, stream);
}

int pic_init_batch(pic_ctx_t **out, const pic_grid_t *grids, int32_t nslab, const pic_potential_t *pot, double dt,
                   const int64_t *max_n, void *ws, size_t ws_bytes, void *stream) {
  return init_common(out, grids, nslab, pot, dt, max_n, ws, ws_bytes, stream);
}

int pic_destroy(pic_ctx_t *ctx) {
  if (!ctx) return PIC_OK;
  if (ctx->drift_ev) (void)hipEventSynchronize(ctx->drift_ev);
  if (ctx->drift_ev) (void)hipEventDestroy(ctx->drift_ev);
  if (ctx->h_drift) (void)hipHostFree(ctx->h_drift);
  drop_graphs(ctx);
  harvest_events(ctx);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  delete ctx;
  return PIC_OK;
}

const char *pic_last_error(const pic_ctx_t *ctx) { return ctx ? ctx->last_error.c_str() : "context is NULL"; }

int pic_sync(pic_ctx_t *ctx) {
  if (!ctx) return PIC_EINVAL;
  return read_device_error(ctx);
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
    out->drifters_last = h[ctx->last_step & 1];
    out->items_last = h[2];
  }
  return PIC_OK;
}

static int edge_log2(int32_t e) {
  int l = 0;
  while (l < 30 && (1 << l) < e) ++l;
  return e >= 1 && (1 << l) == e ? l : -1;
}

int pic_set_tile_shape(pic_ctx_t *ctx, int32_t tile, int32_t tile_last, int32_t halo, int32_t chunk,
                       int32_t sort_every) {
  if (!ctx) return PIC_EINVAL;
  if (!ctx->tiled) return fail(ctx, PIC_EINVAL, "this grid uses the untiled path");
  const int lt = edge_log2(tile), ltl = edge_log2(tile_last);
  if (lt < 0 || ltl < 0) return fail(ctx, PIC_EINVAL, "tile edges must be powers of two");
  const int old_lt = ctx->lt, old_l = ctx->ltl, old_h = ctx->halo, old_c = ctx->chunk, old_s = ctx->sort_every;
  int rc = apply_tiling(ctx, lt, ltl, halo, chunk, sort_every);
  if (rc && rc != PIC_EHIP) {
    std::string why = ctx->last_error;
    apply_tiling(ctx, old_lt, old_l, old_h, old_c, old_s);  // keep the previous (valid) tiling
    ctx->last_error = why;
  }
  return rc;
}

int pic_set_tiling(pic_ctx_t *ctx, int32_t tile, int32_t halo, int32_t chunk, int32_t sort_every) {
  return pic_set_tile_shape(ctx, tile, tile, halo, chunk, sort_every);
}

int pic_get_tiling(pic_ctx_t *ctx, int32_t *tile, int32_t *halo, int32_t *chunk, int32_t *sort_every) {
  if (!ctx) return PIC_EINVAL;
  if (!ctx->tiled) return fail(ctx, PIC_EINVAL, "this grid uses the untiled path");
  if (tile) *tile = 1 << ctx->lt;
  if (halo) *halo = ctx->halo;
  if (chunk) *chunk = ctx->chunk;
  if (sort_every) *sort_every = ctx->sort_every;
  return PIC_OK;
}

int pic_get_tile_shape(pic_ctx_t *ctx, int32_t *tile, int32_t *tile_last) {
  if (!ctx) return PIC_EINVAL;
  if (!ctx->tiled) return fail(ctx, PIC_EINVAL, "this grid uses the untiled path");
  if (tile) *tile = 1 << ctx->lt;
  if (tile_last) *tile_last = 1 << ctx->ltl;
  return PIC_OK;
}

int pic_set_path(pic_ctx_t *ctx, int32_t untiled) {
  if (!ctx) return PIC_EINVAL;
  if (untiled && ctx->nslab > 1) return fail(ctx, PIC_EINVAL, "batched contexts have only the tiled path");
  ctx->force_untiled = untiled != 0;
  return PIC_OK;
}

int pic_set_graph(pic_ctx_t *ctx, int32_t on) {
  if (!ctx) return PIC_EINVAL;
  ctx->use_graph = on != 0;
  if (!on) drop_graphs(ctx);
  return PIC_OK;
}

int pic_set_record_states(pic_ctx_t *ctx, int32_t all) {
  if (!ctx) return PIC_EINVAL;
  ctx->rec_all = all != 0;
  return PIC_OK;
}

static int single_slab(pic_ctx_t *ctx) {
  return ctx->nslab == 1 ? PIC_OK : fail(ctx, PIC_EINVAL, "this call needs a single-slab context");
}

int pic_deposit(pic_ctx_t *ctx, const pic_particles_t *p, int64_t *node_w) {
  if (!ctx) return PIC_EINVAL;
  int rc = single_slab(ctx);
  if (!rc) rc = check_particles(ctx, p, ctx->max_n[0], false, true);
  if (rc) return rc;
  if (!node_w) return fail(ctx, PIC_EINVAL, "node_w is NULL");
  launch_fill64(ctx->stream, reinterpret_cast<long long *>(node_w), ctx->sizes[0].nnodes);
  launch_deposit_atomic(ctx->stream, ctx->geo, ptrs(p), reinterpret_cast<long long *>(node_w), ctx->err);
  return check_launch(ctx, "deposit");
}

int pic_force(pic_ctx_t *ctx, const pic_particles_t *p, const int64_t *node_w, float *force,
              pic_diag_t *pe_or_null) {
  if (!ctx) return PIC_EINVAL;
  int rc = single_slab(ctx);
  if (!rc) rc = check_particles(ctx, p, ctx->max_n[0], false, false);
  if (rc) return rc;
  if (!node_w) return fail(ctx, PIC_EINVAL, "node_w is NULL");
  if (p->n > 0 && !force) return fail(ctx, PIC_EINVAL, "force is NULL");
  const long long *nw = reinterpret_cast<const long long *>(node_w);
  launch_grid(ctx->stream, ctx->geo, nw, ctx->dens, ctx->G);
  launch_force(ctx->stream, ctx->geo, ctx->P, ptrs(p), ctx->dens, ctx->G, force, ctx->err);
  rc = check_launch(ctx, "force");
  if (rc || !pe_or_null) return rc;
  int nb = launch_pe_nodes(ctx->stream, ctx->geo, ctx->dcs[0], ctx->quad, nw, ctx->partial_pe);
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

int pic_force_noalloc(const pic_grid_t *grid_in, const pic_potential_t *pot, const pic_particles_t *p,
                      float *force, uint32_t *device_error, void *stream) {
  Sizes sz;
  if (!grid_sizes(grid_in, &sz, nullptr) || !valid_potential(pot) || !p || p->n < 0) return PIC_EINVAL;
  if (p->n > 0 && (!p->cell || !p->off || !p->wq || !force)) return PIC_EINVAL;
  const pic_grid_t grid = normalised(*grid_in);
  // node sums (int64), node densities (float), cell-centred gradient planes
  // (float, ndim of them), error word
  const size_t o_dens = align_up(sizeof(long long) * (size_t)sz.nnodes);
  const size_t o_G = o_dens + align_up(sizeof(float) * (size_t)sz.nnodes);
  const size_t o_err = o_G + align_up(sizeof(float) * (size_t)sz.ncells * grid.ndim);
  if (o_err + kAlign > (size_t)PIC_NOALLOC_SCRATCH_BYTES) return PIC_ENOSPACE;
  void *base = nullptr;
  int rc = noalloc_scratch(&base);
  if (rc) return rc;
  char *b = static_cast<char *>(base);
  long long *node = reinterpret_cast<long long *>(b);
  float *dens = reinterpret_cast<float *>(b + o_dens);
  float *G = reinterpret_cast<float *>(b + o_G);
  uint32_t *err = device_error ? device_error : reinterpret_cast<uint32_t *>(b + o_err);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const Geo geo = make_geo(grid, *pot, 0.0, sz);
  const Pot P = make_pot(*pot, 0.0);
  const PartPtrs pp = ptrs(p);
  // the array keeps the previous call's contents: the node sums start at zero
  // (a fill kernel, so the call can also be captured into a graph)
  launch_fill64(st, node, sz.nnodes);
  if (!device_error) launch_clear_word(st, err);
  launch_deposit_atomic(st, geo, pp, node, err);
  launch_grid(st, geo, node, dens, G);
  launch_force(st, geo, P, pp, dens, G, force, err);
  return hipGetLastError() == hipSuccess ? PIC_OK : PIC_EHIP;
}

int pic_kick(pic_ctx_t *ctx, pic_particles_t *p, const float *force, double frac) {
  if (!ctx) return PIC_EINVAL;
  int rc = single_slab(ctx);
  if (!rc) rc = check_particles(ctx, p, ctx->max_n[0], true, false);
  if (rc) return rc;
  if (p->n > 0 && !force) return fail(ctx, PIC_EINVAL, "force is NULL");
  if (!std::isfinite(frac)) return fail(ctx, PIC_EINVAL, "frac must be finite");
  launch_kick(ctx->stream, ctx->geo, ctx->P, ptrs(p), force, (float)frac);
  return check_launch(ctx, "kick");
}

int pic_push(pic_ctx_t *ctx, pic_particles_t *p, const float *force) {
  if (!ctx) return PIC_EINVAL;
  int rc = single_slab(ctx);
  if (!rc) rc = check_particles(ctx, p, ctx->max_n[0], true, false);
  if (rc) return rc;
  if (p->n > 0 && !force) return fail(ctx, PIC_EINVAL, "force is NULL");
  launch_push(ctx->stream, ctx->geo, ctx->P, ptrs(p), force, ctx->err);
  return check_launch(ctx, "push");
}

// ---------------------------------------------------------------------------
// Reverse mode on caller arrays
// ---------------------------------------------------------------------------
// Slot scales of the parameter partials: the kernels accumulate D dJ/dD,
// r0 dJ/dr0, dJ/ds_rep, dJ/dc_att and alpha dJ/dalpha (zero under
// Lennard-Jones, whose alpha is unused).
static ThetaScale theta_scale(const pic_ctx_t *ctx) {
  const pic_potential_t &P = ctx->pot;
  return ThetaScale{{1.0 / P.D, 1.0 / P.r0, 1.0, 1.0, P.kind == PIC_POT_MORSE ? 1.0 / P.alpha : 0.0}};
}

// Shared tail of the two particle VJPs: nbar gets the gradient transpose, the
// per-block parameter partials are summed into dtheta.
static int adjoint_common(pic_ctx_t *ctx, const pic_particles_t *p, const int64_t *node_w, const float *nbar_next,
                          const float *fbar, float *lam_x, float *lam_v, float *nbar, double *dtheta,
                          bool force_only, const char *what) {
  if (!node_w) return fail(ctx, PIC_EINVAL, "node_w is NULL");
  if (!nbar) return fail(ctx, PIC_EINVAL, "nbar is NULL");
  if (!dtheta) return fail(ctx, PIC_EINVAL, "dtheta is NULL");
  if (p->n > 0 && (!lam_x || (!force_only && !lam_v) || (force_only && !fbar)))
    return fail(ctx, PIC_EINVAL, "a cotangent array is NULL");
  const Geo &g = ctx->geo;
  launch_grid(ctx->stream, g, reinterpret_cast<const long long *>(node_w), ctx->dens, ctx->G);
  launch_fillf(ctx->stream, nbar, g.nnodes);
  launch_fillf(ctx->stream, ctx->Gbar, (int64_t)g.ncells * g.ndim);
  const int nb = launch_adjoint(ctx->stream, g, ctx->P, ptrs(p), ctx->dens, ctx->G, nbar_next, fbar, lam_x, lam_v,
                                nbar, ctx->Gbar, ctx->partial, ctx->err, force_only);
  launch_gradient_vjp(ctx->stream, g, ctx->Gbar, nbar);
  if (nb > 0) launch_reduce_theta(ctx->stream, ctx->partial, nb, theta_scale(ctx), dtheta);
  return check_launch(ctx, what);
}

int pic_adjoint_step(pic_ctx_t *ctx, const pic_particles_t *state, const int64_t *node_w, const float *nbar_next,
                     float *lam_x, float *lam_v, float *nbar, double *dtheta) {
  if (!ctx) return PIC_EINVAL;
  int rc = single_slab(ctx);
  if (!rc) rc = check_particles(ctx, state, ctx->max_n[0], true, true);
  if (rc) return rc;
  return adjoint_common(ctx, state, node_w, nbar_next, nullptr, lam_x, lam_v, nbar, dtheta, false, "adjoint step");
}

int pic_force_vjp(pic_ctx_t *ctx, const pic_particles_t *state, const int64_t *node_w, const float *force_bar,
                  float *lam_x, float *nbar, double *dtheta) {
  if (!ctx) return PIC_EINVAL;
  int rc = single_slab(ctx);
  if (!rc) rc = check_particles(ctx, state, ctx->max_n[0], false, false);
  if (rc) return rc;
  return adjoint_common(ctx, state, node_w, nullptr, force_bar, lam_x, nullptr, nbar, dtheta, true, "force vjp");
}

int pic_deposit_vjp(pic_ctx_t *ctx, const pic_particles_t *state, const float *nbar, float *lam_x) {
  if (!ctx) return PIC_EINVAL;
  int rc = single_slab(ctx);
  if (!rc) rc = check_particles(ctx, state, ctx->max_n[0], false, true);
  if (rc) return rc;
  if (!nbar) return fail(ctx, PIC_EINVAL, "nbar is NULL");
  if (state->n > 0 && !lam_x) return fail(ctx, PIC_EINVAL, "lam_x is NULL");
  launch_deposit_vjp(ctx->stream, ctx->geo, ptrs(state), nbar, lam_x, ctx->err);
  return check_launch(ctx, "deposit vjp");
}

// ---------------------------------------------------------------------------
// Recorded trajectories: forward with checkpoints in the store's order, and
// the reverse sweep that recomputes each segment out of place and runs the
// tiled reverse kernel over it.
// ---------------------------------------------------------------------------
// Record (device, caller-owned): one entry per checkpoint, each with the
// state (pc, off, vel), the binning it was taken under (wq, oidx, work items,
// their count).  Recorded runs re-bin only at checkpoints, so every segment
// between two checkpoints keeps one binning.  A record that keeps every
// state holds the states of each checkpoint's whole segment (seg of them,
// the first being the checkpoint's), and after the entries the node sums of
// every step (nsteps + 2: the last two are the final step's deposit and
// clear targets), so that the reverse sweep recomputes nothing.
struct RecLayout {
  size_t state, wq, oidx, items, nitems, stride, nodes, node_stride, total;
  int nck, seg;
};

static size_t state_bytes_of(int nd, int64_t cap) { return align_up((size_t)cap * 4 * (1 + nd + 3)); }

static RecLayout rec_layout(const pic_ctx_t *c, int nsteps, int every) {
  RecLayout R{};
  const int64_t cap = c->cap;
  R.nck = (nsteps + every - 1) / every;
  R.seg = c->rec_all ? std::min(every, nsteps) : 1;
  size_t o = 0;
  R.state = o; o += state_bytes_of(c->ndim, cap) * (size_t)R.seg;
  R.wq = o; o = align_up(o + 4 * (size_t)cap);
  R.oidx = o; o = align_up(o + 4 * (size_t)cap);
  R.items = o; o = align_up(o + sizeof(Item) * (size_t)c->items_cap);
  R.nitems = o; o = align_up(o + sizeof(int));
  R.stride = o;
  R.nodes = o * (size_t)R.nck;
  R.node_stride = align_up(8 * (size_t)c->nnodes);
  R.total = R.nodes + (c->rec_all ? R.node_stride * (size_t)(nsteps + 2) : 0);
  return R;
}

// A store whose per-particle state lives at base (wq / oidx from ref).
static Store state_at(const pic_ctx_t *c, char *base, const Store &ref) {
  Store S = ref;
  const int64_t cap = c->cap;
  S.pc = reinterpret_cast<int *>(base);
  S.off = reinterpret_cast<float *>(base + 4 * cap);
  S.vel = reinterpret_cast<float *>(base + 4 * cap * (1 + c->ndim));
  return S;
}

static int copy_state(pic_ctx_t *c, const Store &dst, const Store &src) {
  const size_t cap = (size_t)c->cap;
  hipError_t e = hipMemcpyAsync(dst.pc, src.pc, 4 * cap, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dst.off, src.off, 4 * cap * c->ndim, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(dst.vel, src.vel, 4 * cap * 3, hipMemcpyDeviceToDevice, c->stream);
  return hip_check(c, e, "copy state");
}

static int recorded_ok(pic_ctx_t *c, const pic_particles_t *p, int nsteps, int every) {
  if (!c->tiled || c->nslab != 1 || c->force_untiled)
    return fail(c, PIC_EINVAL, "recorded trajectories need a single-slab context on the tiled path");
  if (nsteps < 1 || every < 1) return fail(c, PIC_EINVAL, "nsteps and every must be >= 1");
  return check_particles(c, p, c->max_n[0], true, true);
}

static std::vector<int64_t> rec_key_of(const pic_ctx_t *c, int64_t n, int nsteps, int every, const void *rec) {
  return {n,        nsteps,   every, c->lt, c->ltl, c->halo, c->chunk, (int64_t)reinterpret_cast<uintptr_t>(rec),
          c->rec_all};
}

size_t pic_record_bytes(pic_ctx_t *ctx, int32_t nsteps, int32_t every) {
  if (!ctx || !ctx->tiled || ctx->nslab != 1 || nsteps < 1 || every < 1) return 0;
  return rec_layout(ctx, nsteps, every).total;
}

// Backward scratch: a segment's recomputed states and node sums (not with a
// record that keeps every state), then the cotangents.
static size_t segment_scratch_bytes(const pic_ctx_t *c, int every) {
  if (c->rec_all) return 0;
  return state_bytes_of(c->ndim, c->cap) * (size_t)every + align_up(8 * (size_t)c->nnodes) * (size_t)(every + 1);
}

size_t pic_backward_bytes(pic_ctx_t *ctx, int32_t every) {
  if (!ctx || !ctx->tiled || ctx->nslab != 1 || every < 1) return 0;
  const size_t cap = (size_t)ctx->cap, nn = (size_t)ctx->nnodes;
  return segment_scratch_bytes(ctx, every) + align_up(4 * cap * ctx->ndim) + align_up(4 * cap * 3) +
         3 * align_up(4 * nn);
}

int pic_forward_record(pic_ctx_t *ctx, pic_particles_t *p, int32_t nsteps, int32_t every, void *record,
                       size_t record_bytes) {
  if (!ctx) return PIC_EINVAL;
  int rc = recorded_ok(ctx, p, nsteps, every);
  if (rc) return rc;
  const RecLayout R = rec_layout(ctx, nsteps, every);
  if (!record || record_bytes < R.total) return fail(ctx, PIC_ENOSPACE, "record buffer too small");
  if (reinterpret_cast<uintptr_t>(record) % kAlign) return fail(ctx, PIC_EINVAL, "record must be 256-byte aligned");
  char *rec = static_cast<char *>(record);
  const int nd = ctx->ndim;
  if ((rc = bind_counts(ctx, p))) return rc;
  const int64_t n = p->n;
  const Batch b = batch_of(ctx, n);
  ensure_grid_blocks(ctx);
  const PartPtrs cp = ptrs(p);
  launch_import(ctx->stream, nd, ctx->sd.data(), &cp, 1, ctx->bb, b, ctx->chunk, ctx->st[0], ctx->st[1].oidx,
                ctx->err);
  if ((rc = check_launch(ctx, "binning"))) return rc;
  if ((rc = read_device_error(ctx))) return rc;
  int cur = 0;
  const int64_t max_items = max_items_of(ctx, n);
  // node sums of step s: the three rotating buffers, or the record's own
  auto Ns = [&](int s) {
    return ctx->rec_all ? reinterpret_cast<long long *>(rec + R.nodes + R.node_stride * (size_t)s)
                        : ctx->n3[s % 3];
  };
  launch_fill64(ctx->stream, Ns(0), ctx->nnodes);
  launch_fill64(ctx->stream, Ns(1), ctx->nnodes);
  launch_fill32(ctx->stream, ctx->drift, 4);
  launch_deposit_tiled(ctx->stream, nd, ctx->sd[0].tg, b, ctx->st[cur], ctx->bb, (int)max_items, Ns(0));
  const size_t sb = state_bytes_of(nd, ctx->cap);
  std::vector<char> rebinned(R.nck, 0);
  int since_bin = 0;
  // state s of a record that keeps every state: slot k of checkpoint j's
  // segment (s = j every + k), with the binning of the working store
  auto rec_state = [&](int s) {
    const int j = s / every;
    return state_at(ctx, rec + R.stride * j + R.state + sb * (size_t)(s - j * every), ctx->st[cur]);
  };
  for (int32_t s = 0; s < nsteps; ++s) {
    if (s % every == 0) {
      const int j = s / every;
      // the state before step s: the working store, or (every state kept,
      // s > 0) already the record's, written there by step s - 1
      const bool in_rec = ctx->rec_all && s > 0;
      const Store src = in_rec ? rec_state(s) : ctx->st[cur];
      // re-bin at a checkpoint: always with a fixed re-binning period, and
      // with the adaptive one once more than n / kDriftFraction particles
      // left their window in the previous step
      bool rebin = false;
      if (s > 0 && ctx->sort_every > 0) {
        rebin = true;
      } else if (s > 0 && ctx->sort_every < 0) {
        int h = 0;
        if ((rc = hip_check(ctx, hipMemcpyAsync(&h, ctx->drift + ((s - 1) & 1), sizeof(int),
                                                hipMemcpyDeviceToHost, ctx->stream), "drifter count")))
          return rc;
        if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "stream synchronize"))) return rc;
        rebin = (int64_t)h * kDriftFraction > n || since_bin >= kMaxBinPeriod;
      }
      if (rebin) {
        launch_rebin(ctx->stream, nd, ctx->bb, b, ctx->chunk, src, ctx->st[1 - cur]);
        cur = 1 - cur;
        since_bin = 0;
        rebinned[j] = 1;
      }
      char *ck = rec + R.stride * j;
      const Store &S = ctx->st[cur];
      // the checkpoint's state: copied unless step s - 1 wrote it there and
      // the binning is unchanged
      if ((!in_rec || rebin) && (rc = copy_state(ctx, state_at(ctx, ck + R.state, S), S))) return rc;
      hipError_t e = hipMemcpyAsync(ck + R.wq, S.wq, 4 * (size_t)ctx->cap, hipMemcpyDeviceToDevice, ctx->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(ck + R.oidx, S.oidx, 4 * (size_t)ctx->cap, hipMemcpyDeviceToDevice, ctx->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(ck + R.items, ctx->bb.items, sizeof(Item) * (size_t)ctx->items_cap,
                           hipMemcpyDeviceToDevice, ctx->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(ck + R.nitems, ctx->bb.num_items, sizeof(int), hipMemcpyDeviceToDevice, ctx->stream);
      if ((rc = hip_check(ctx, e, "save checkpoint"))) return rc;
    }
    if (ctx->rec_all) {
      // step s reads state s from the record and writes state s + 1 there
      // (the next checkpoint re-bins it in place of a copy when it must);
      // the last step writes the working store, which is exported
      const Store out = s + 1 < nsteps ? rec_state(s + 1) : ctx->st[cur];
      launch_step_tiled(ctx->stream, nd, ctx->sd[0].tg, ctx->P, ctx->dcs[0], b, rec_state(s), out, ctx->bb,
                        step_grid(ctx, n), Ns(s), Ns(s + 1), Ns(s + 2), drift_of(ctx, s), ctx->partial, false,
                        ctx->err);
    } else {
      enqueue_step(ctx, b, ctx->st[cur], s, false);
    }
    if ((rc = check_launch(ctx, "recorded step"))) return rc;
    ++since_bin;
  }
  const Store &S = ctx->st[cur];
  launch_export(ctx->stream, nd, ctx->sd[0], S, ctx->bb, cp);
  if (ctx->rec_all &&
      (rc = hip_check(ctx, hipMemcpyAsync(ctx->n3[nsteps % 3], Ns(nsteps), 8 * (size_t)ctx->nnodes,
                                          hipMemcpyDeviceToDevice, ctx->stream), "final node sums")))
    return rc;
  ctx->last_nodes = ctx->n3[nsteps % 3];
  ctx->last_step = nsteps - 1;
  if ((rc = check_launch(ctx, "export"))) return rc;
  if ((rc = read_device_error(ctx))) return rc;
  ctx->rec_key = rec_key_of(ctx, n, nsteps, every, record);
  ctx->rec_rebinned = rebinned;
  return PIC_OK;
}

int pic_backward_record(pic_ctx_t *ctx, const pic_particles_t *p, int32_t nsteps, int32_t every,
                        const void *record, size_t record_bytes, void *scratch, size_t scratch_bytes, float *lam_x,
                        float *lam_v, double *dtheta, double start_kick) {
  if (!ctx) return PIC_EINVAL;
  if (!std::isfinite(start_kick)) return fail(ctx, PIC_EINVAL, "start_kick must be finite");
  int rc = recorded_ok(ctx, p, nsteps, every);
  if (rc) return rc;
  const RecLayout R = rec_layout(ctx, nsteps, every);
  if (!record || record_bytes < R.total) return fail(ctx, PIC_ENOSPACE, "record buffer too small");
  if (ctx->rec_key != rec_key_of(ctx, p->n, nsteps, every, record))
    return fail(ctx, PIC_EINVAL, "record was not written by pic_forward_record with these arguments and tiling");
  const size_t need = pic_backward_bytes(ctx, every);
  if (!scratch || scratch_bytes < need) return fail(ctx, PIC_ENOSPACE, "scratch buffer too small");
  if (reinterpret_cast<uintptr_t>(scratch) % kAlign) return fail(ctx, PIC_EINVAL, "scratch must be 256-byte aligned");
  if (!dtheta) return fail(ctx, PIC_EINVAL, "dtheta is NULL");
  if (p->n > 0 && (!lam_x || !lam_v)) return fail(ctx, PIC_EINVAL, "lam_x or lam_v is NULL");
  const int nd = ctx->ndim;
  const int64_t n = p->n, cap = ctx->cap;
  const size_t nn = (size_t)ctx->nnodes;
  char *rec = const_cast<char *>(static_cast<const char *>(record));
  char *scr = static_cast<char *>(scratch);
  // scratch: states of one segment, node sums of one segment (+1) (neither
  // with a record that keeps every state), cotangents
  const size_t sb = state_bytes_of(nd, cap);
  char *traj = scr;
  char *N0 = traj + sb * (size_t)every;
  float *lx = reinterpret_cast<float *>(scr + segment_scratch_bytes(ctx, every));
  float *lv = reinterpret_cast<float *>(reinterpret_cast<char *>(lx) + align_up(4 * (size_t)cap * nd));
  // node cotangents of three consecutive reverse steps: each step reads the
  // later step's, accumulates its own and clears the earlier step's
  float *nb3[3];
  nb3[0] = reinterpret_cast<float *>(reinterpret_cast<char *>(lv) + align_up(4 * (size_t)cap * 3));
  nb3[1] = reinterpret_cast<float *>(reinterpret_cast<char *>(nb3[0]) + align_up(4 * nn));
  nb3[2] = reinterpret_cast<float *>(reinterpret_cast<char *>(nb3[1]) + align_up(4 * nn));
  if ((rc = bind_counts(ctx, p))) return rc;
  const Batch b = batch_of(ctx, n);
  ensure_grid_blocks(ctx);
  ctx->last_nodes = nullptr;
  drop_graphs(ctx);
  const int64_t max_items = max_items_of(ctx, n);
  // checkpoint j's binning: a store whose wq / oidx are the record's, and its items
  auto ref_of = [&](int j) {
    Store S = ctx->st[0];
    char *ck = rec + R.stride * j;
    S.wq = reinterpret_cast<int *>(ck + R.wq);
    S.oidx = reinterpret_cast<int *>(ck + R.oidx);
    return S;
  };
  auto bins_of = [&](int j) {
    BinBufs bb = ctx->bb;
    char *ck = rec + R.stride * j;
    bb.items = reinterpret_cast<Item *>(ck + R.items);
    bb.num_items = reinterpret_cast<int *>(ck + R.nitems);
    return bb;
  };
  launch_to_store(ctx->stream, b, ref_of(R.nck - 1), nd, lam_x, n, lx);
  launch_to_store(ctx->stream, b, ref_of(R.nck - 1), 3, lam_v, n, lv);
  launch_fill64(ctx->stream, reinterpret_cast<long long *>(ctx->dacc), 8);
  launch_fill64(ctx->stream, reinterpret_cast<long long *>(ctx->partial), 8 * max_items);
  const Geo &g = ctx->geo;
  const float *nbar_next = nullptr;
  // the first reverse step's node cotangents and counters start at zero; each
  // later step's are cleared by the step before it
  launch_clear_reverse(ctx->stream, nb3[(nsteps - 1) % 3], ctx->nnodes, ctx->drift, ctx->amax + (nsteps & 1));
  launch_fill32(ctx->stream, ctx->drift + 1, 1);
  for (int j = R.nck - 1; j >= 0; --j) {
    const int s0 = j * every, len = std::min(every, nsteps - s0);
    const Store ref = ref_of(j);
    const BinBufs bb = bins_of(j);
    char *seg = rec + R.stride * j + R.state;
    auto slot = [&](int k) {
      return k == 0 || ctx->rec_all ? state_at(ctx, seg + sb * (size_t)k, ref) : state_at(ctx, traj + sb * k, ref);
    };
    auto Nk = [&](int k) {
      return reinterpret_cast<long long *>(ctx->rec_all ? rec + R.nodes + R.node_stride * (size_t)(s0 + k)
                                                        : N0 + align_up(8 * nn) * k);
    };
    if (!ctx->rec_all) {
      // recompute the segment's states (out of place) and node sums
      launch_fill64(ctx->stream, Nk(0), ctx->nnodes);
      if (len > 1) launch_fill64(ctx->stream, Nk(1), ctx->nnodes);
      launch_fill32(ctx->stream, ctx->drift, 4);
      launch_deposit_tiled(ctx->stream, nd, ctx->sd[0].tg, b, slot(0), bb, (int)max_items, Nk(0));
      for (int k = 0; k + 1 < len; ++k) {
        const Drift dr = drift_of(ctx, k);
        const Store in = slot(k), out = slot(k + 1);
        launch_step_tiled(ctx->stream, nd, ctx->sd[0].tg, ctx->P, ctx->dcs[0], b, in, out, bb, step_grid(ctx, n),
                          Nk(k), Nk(k + 1), Nk(k + 2), dr, ctx->partial, false, ctx->err);
      }
      // the recompute's drifter counters are the reverse steps' too
      launch_fill32(ctx->stream, ctx->drift, 2);
      if ((rc = check_launch(ctx, "recompute"))) return rc;
    }
    // reverse steps of the segment
    for (int k = len - 1; k >= 0; --k) {
      const int step = s0 + k;
      uint32_t *amax_prev = ctx->amax + (step & 1), *amax_cur = ctx->amax + ((step + 1) & 1);
      // the first step's kick also reverses the start kick of the same state:
      // its force cotangent is (1 + start_kick) times the step's own
      Pot P = ctx->P;
      if (step == 0) P.ks = (float)(1.0 + start_kick);
      if (step == nsteps - 1)  // seed the fixed-point scale of the first reverse step
        launch_adjoint_scale(ctx->stream, nd, ctx->sd[0].tg, P, b, slot(k), bb, (int)max_items, Nk(k), nbar_next, lx,
                             lv, amax_prev);
      float *nb_cur = nb3[step % 3];
      int *dcount = ctx->drift + (step & 1);
      // the state after this step in this segment's binning: the segment's
      // next slot, or the next checkpoint's state unless that one was re-binned
      Store after;
      const Store *known = nullptr;
      if (k + 1 < len) {
        after = slot(k + 1);
        known = &after;
      } else if (j + 1 < R.nck && !ctx->rec_rebinned[j + 1]) {
        after = state_at(ctx, rec + R.stride * (j + 1) + R.state, ref);
        known = &after;
      }
      const bool more = step > 0;  // the next reverse step's buffers: cleared by this one
      launch_adjoint_tiled(ctx->stream, nd, ctx->sd[0].tg, P, b, slot(k), bb, (int)max_items, Nk(k), nbar_next, lx, lv,
                           nb_cur, ctx->drift + 4, dcount, amax_prev, amax_cur, ctx->partial, ctx->dacc, ctx->err,
                           known, more ? nb3[(step + 2) % 3] : nullptr, ctx->nnodes,
                           more ? ctx->drift + ((step + 1) & 1) : nullptr, more ? amax_prev : nullptr);
      nbar_next = nb_cur;
      if ((rc = check_launch(ctx, "reverse step"))) return rc;
    }
    // into the previous segment's order (through the caller's order, with
    // lam_x / lam_v as the staging arrays) where the binning changed
    if (j > 0 && ctx->rec_rebinned[j]) {
      launch_from_store(ctx->stream, b, ref, nd, lx, n, lam_x);
      launch_from_store(ctx->stream, b, ref, 3, lv, n, lam_v);
      launch_to_store(ctx->stream, b, ref_of(j - 1), nd, lam_x, n, lx);
      launch_to_store(ctx->stream, b, ref_of(j - 1), 3, lam_v, n, lv);
    }
  }
  // parameter terms summed over the sweep (fixed order over the items)
  launch_reduce_theta(ctx->stream, ctx->partial, (int)max_items, theta_scale(ctx), dtheta, ctx->dacc);
  // deposit term of the initial positions, back to the caller's order
  const Store ref0 = ref_of(0);
  launch_deposit_vjp_store(ctx->stream, nd, b, state_at(ctx, rec + R.state, ref0), nbar_next, lx);
  launch_from_store(ctx->stream, b, ref0, nd, lx, n, lam_x);
  launch_from_store(ctx->stream, b, ref0, 3, lv, n, lam_v);
  if ((rc = check_launch(ctx, "reverse sweep"))) return rc;
  return read_device_error(ctx);
}

int pic_step_batch(pic_ctx_t *ctx, pic_particles_t *parts, int32_t nsteps, pic_diag_t *diag, int32_t diag_every) {
  if (!ctx) return PIC_EINVAL;
  if (!parts) return fail(ctx, PIC_EINVAL, "particles is NULL");
  int rc = PIC_OK;
  for (int k = 0; k < ctx->nslab && !rc; ++k) rc = check_particles(ctx, &parts[k], ctx->max_n[k], true, true);
  if (rc) return rc;
  if (nsteps < 0) return fail(ctx, PIC_EINVAL, "nsteps is negative");
  if (diag && diag_every < 1) return fail(ctx, PIC_EINVAL, "diag_every must be >= 1");
  const int64_t ndiag = diag ? (nsteps + diag_every - 1) / diag_every : 0;
  DiagSink ds{ctx, diag, ndiag};
  ctx->last_nodes = nullptr;
  if (ctx->tiled && !ctx->force_untiled) rc = step_tiled(ctx, parts, nsteps, ds, diag_every);
  else rc = step_untiled(ctx, ptrs(&parts[0]), nsteps, ds, diag_every);
  if (rc) return rc;
  if (diag && (rc = ds.flush())) return rc;
  return read_device_error(ctx);
}

int pic_step(pic_ctx_t *ctx, pic_particles_t *p, int32_t nsteps, pic_diag_t *diag, int32_t diag_every) {
  if (!ctx) return PIC_EINVAL;
  int rc = single_slab(ctx);
  if (rc) return rc;
  return pic_step_batch(ctx, p, nsteps, diag, diag_every);
}

int pic_autotune(pic_ctx_t *ctx, const pic_particles_t *parts, int32_t probe_steps, pic_tuning_t *out) {
  if (!ctx) return PIC_EINVAL;
  if (!ctx->tiled) return fail(ctx, PIC_EINVAL, "this grid uses the untiled path");
  if (!parts || probe_steps < 1) return fail(ctx, PIC_EINVAL, "need particles and probe_steps >= 1");
  int rc = PIC_OK;
  for (int k = 0; k < ctx->nslab && !rc; ++k) rc = check_particles(ctx, &parts[k], ctx->max_n[k], true, true);
  if (rc) return rc;
  const int nd = ctx->ndim;
  const int halo = nd == 2 ? 2 : 1;
  // tile shapes (edge exponents: all axes but the last, last axis): square
  // 8, 16, 32 in 2D; 4^3, 8^3 and 8 x 8 x 4 in 3D (a flatter window that
  // leaves LDS for more blocks per CU)
  struct Shape {
    int lt, ltl;
  };
  const Shape shapes2[3] = {{3, 3}, {4, 4}, {5, 5}}, shapes3[3] = {{2, 2}, {3, 3}, {3, 2}};
  const Shape *shapes = nd == 2 ? shapes2 : shapes3;
  const int chunks[6] = {512, 1024, 2048, 4096, 8192, 16384};
  const int old_lt = ctx->lt, old_l = ctx->ltl, old_h = ctx->halo, old_c = ctx->chunk, old_s = ctx->sort_every;
  const bool old_timing = ctx->timing, old_graph = ctx->use_graph;
  ctx->timing = false;
  ctx->use_graph = false;  // a graph capture per candidate would land inside its timed probe
  float best = 1e30f;
  int best_c = old_c, tried = 0;
  Shape best_s{old_lt, old_l};
  struct Probe {
    float ms;
    Shape sh;
    int c;
  };
  std::vector<Probe> probes;
  pic_particles_t *pp = const_cast<pic_particles_t *>(parts);
  for (int i = 0; i < 3; ++i) {
    const Shape sh = shapes[i];
    std::vector<int> cand(chunks, chunks + 6);
    for (size_t ci = 0; ci < cand.size(); ++ci) {
      const int c = cand[ci];
      if (apply_tiling(ctx, sh.lt, sh.ltl, halo, c, old_s)) continue;  // does not fit this grid
      DiagSink ds{ctx, nullptr, 0};
      float ms = 0.f;
      // the store is scratch: the caller's arrays are read, never written
      rc = step_tiled(ctx, pp, probe_steps, ds, 1, false, &ms);
      if (rc) break;
      ++tried;
      probes.push_back({ms, sh, c});
      if (ms < best) {
        best = ms;
        best_s = sh;
        best_c = c;
      }
      if (ci == 0) {
        // chunks whose item count fills whole rounds of the persistent grid,
        // from this tiling's particle counts per tile
        std::vector<int> counts(ctx->ntiles);
        rc = hip_check(ctx, hipMemcpy(counts.data(), ctx->bb.counts, sizeof(int) * counts.size(),
                                      hipMemcpyDeviceToHost), "tile counts");
        if (rc) break;
        for (int extra : balanced_chunks(counts, ctx->grid_blocks))
          if (std::find(cand.begin(), cand.end(), extra) == cand.end()) cand.push_back(extra);
      }
    }
    if (rc) break;
  }
  // Among the probes within 1 % of the fastest, take the largest items: the
  // forward steps cannot tell them apart, while a reverse sweep pays per item
  // (each flushes its window's node cotangents).
  float sel = best;
  for (const Probe &q : probes) {
    if (q.ms > best * 1.01f) continue;
    if (q.c > best_c || (q.c == best_c && q.ms < sel)) {
      best_c = q.c;
      best_s = q.sh;
      sel = q.ms;
    }
  }
  ctx->timing = old_timing;
  ctx->use_graph = old_graph;
  ctx->last_nodes = nullptr;
  const bool keep_old = rc || !tried;
  int rc2 = apply_tiling(ctx, keep_old ? old_lt : best_s.lt, keep_old ? old_l : best_s.ltl, keep_old ? old_h : halo,
                         keep_old ? old_c : best_c, old_s);
  if (rc) return rc;
  if (rc2) return rc2;
  if (!tried) return fail(ctx, PIC_EINVAL, "no tiling fits this grid");
  if (out) {
    out->tile = 1 << best_s.lt;
    out->halo = halo;
    out->chunk = best_c;
    out->candidates = tried;
    out->ms_per_step = sel / probe_steps;
    out->tile_last = 1 << best_s.ltl;
  }
  return read_device_error(ctx);
}

int pic_step_nodes(pic_ctx_t *ctx, int64_t *node_w) {
  if (!ctx || !node_w) return PIC_EINVAL;
  if (!ctx->last_nodes) return fail(ctx, PIC_EINVAL, "no tiled pic_step has run on this context");
  return hip_check(ctx, hipMemcpyAsync(node_w, ctx->last_nodes, sizeof(long long) * (size_t)ctx->nnodes,
                                       hipMemcpyDeviceToDevice, ctx->stream),
                   "copy node sums");
}

}  // extern "C"

namespace {

// Smallest node sum N >= 0 whose FP64 density (N * 2^-20 / V) / n_solid is
// at least cut, or -1 when it would pass 2^52 (beyond any node sum, and
// where N is no longer exact in a double).  The density grows with N, so
// the step from a close estimate to the exact edge is a few units.
long long cut_threshold(double V, double n_solid, double cut) {
  auto kept = [&](long long N) { return ((double)N * 0x1p-20 / V) / n_solid >= cut; };
  if (kept(0)) return 0;
  const double est = std::ceil(cut * n_solid * V * 0x1p20);
  if (!(est < 0x1p52)) return -1;
  long long N = (long long)est;
  for (int i = 0; i < 1024 && N > 0 && kept(N - 1); ++i) --N;
  for (int i = 0; i < 1024 && !kept(N); ++i) ++N;
  return kept(N) && (N == 0 || !kept(N - 1)) ? N : -1;
}

}  // namespace

extern "C" {

int64_t pic_num_columns(const pic_grid_t *grid) {
  Sizes s;
  if (!grid_sizes(grid, &s, nullptr)) return 0;
  int64_t c = 1;
  for (int d = 0; d < grid->ndim - 1; ++d) c *= grid->n[d] + grid->bc[d];
  return c;
}

int pic_crater(pic_ctx_t *ctx, const int64_t *node_w, const pic_crater_spec_t *spec, const double *y_s,
               const double *fluence, const double *beam_d, float *rho, int64_t *col_w, pic_crater_t *out) {
  if (!ctx) return PIC_EINVAL;
  if (!node_w || !spec || !y_s || !col_w || !out) return fail(ctx, PIC_EINVAL, "pic_crater: NULL argument");
  if (!(spec->n_solid > 0) || !std::isfinite(spec->n_solid) || !(spec->cut >= 0) || !std::isfinite(spec->cut) ||
      !(spec->depth_min > 0) || !std::isfinite(spec->depth_min))
    return fail(ctx, PIC_EINVAL, "pic_crater: n_solid and depth_min must be > 0, cut >= 0");
  if ((fluence == nullptr) != (beam_d == nullptr))
    return fail(ctx, PIC_EINVAL, "pic_crater: fluence and beam_d go together");
  std::vector<CraterSlab> tab(ctx->nslab);
  long long node_off = 0, col_off = 0;
  for (int k = 0; k < ctx->nslab; ++k) {
    const pic_grid_t &g = ctx->grids[k];  // normalised: h[2] is the 2D depth
    CraterSlab &c = tab[k];
    c = CraterSlab{};
    c.ndim = g.ndim;
    for (int d = 0; d < 3; ++d) {
      c.nn[d] = d < g.ndim ? g.n[d] + g.bc[d] : 1;
      c.bc[d] = d < g.ndim ? g.bc[d] : 0;
    }
    c.rows = c.nn[g.ndim - 1];
    c.ncols = (int)(ctx->sizes[k].nnodes / c.rows);
    c.node_off = node_off;
    c.col_off = col_off;
    const double V = g.h[0] * g.h[1] * g.h[2];
    double Vw = V;
    for (int w = 0; w < 4; ++w, Vw *= 0.5) {
      c.keep_min[w] = cut_threshold(Vw, spec->n_solid, spec->cut);
      if (c.keep_min[w] < 0) return fail(ctx, PIC_EINVAL, "pic_crater: cut is too large for int64 node sums");
      c.map_scale[w] = (float)(0x1p-20 / Vw / spec->n_solid);
    }
    const double area = g.ndim == 2 ? g.h[0] * g.h[2] : g.h[0] * g.h[1];
    c.t_scale = 0x1p-20 / (spec->n_solid * area);
    c.lat = g.ndim == 2 ? g.h[0] : g.h[0] * g.h[1];
    if (!std::isfinite(y_s[k])) return fail(ctx, PIC_EINVAL, "pic_crater: y_s must be finite");
    c.y_s = y_s[k];
    c.fluence = fluence ? fluence[k] : 0.0;
    c.beam_d = beam_d ? beam_d[k] : 0.0;
    if (!(c.fluence >= 0) || !(c.beam_d >= 0) || !std::isfinite(c.fluence) || !std::isfinite(c.beam_d))
      return fail(ctx, PIC_EINVAL, "pic_crater: fluence and beam_d must be finite and >= 0");
    node_off += ctx->sizes[k].nnodes;
    col_off += c.ncols;
  }
  const CraterArgs a{spec->n_solid, spec->cut, spec->depth_min};
  launch_fill64(ctx->stream, reinterpret_cast<long long *>(col_w), col_off);
  for (int k0 = 0; k0 < ctx->nslab; k0 += kCraterSlabs) {
    CraterBatch b{};
    b.n = std::min(kCraterSlabs, ctx->nslab - k0);
    int max_cols = 0, max_rows = 0;
    for (int i = 0; i < b.n; ++i) {
      b.s[i] = tab[k0 + i];
      max_cols = std::max(max_cols, b.s[i].ncols);
      max_rows = std::max(max_rows, b.s[i].rows);
    }
    launch_crater_columns(ctx->stream, b, max_cols, max_rows, a, reinterpret_cast<const long long *>(node_w), rho,
                          reinterpret_cast<long long *>(col_w));
    launch_crater_reduce(ctx->stream, b, a, reinterpret_cast<const long long *>(col_w), out + k0);
  }
  return check_launch(ctx, "crater kernels");
}

int pic_threshold_fit(int32_t n, const double *fluence, const double *width, double beam_d, double *f_th_fixed,
                      double *f_th_fit, double *beam_d_fit) {
  if (n < 0 || (n > 0 && (!fluence || !width)) || !f_th_fixed || !f_th_fit || !beam_d_fit) return PIC_EINVAL;
  const double nan = std::nan("");
  *f_th_fixed = *f_th_fit = *beam_d_fit = nan;
  std::vector<double> x, y;
  for (int i = 0; i < n; ++i) {
    if (!(width[i] > 0)) continue;
    if (!(fluence[i] > 0)) return PIC_EINVAL;
    x.push_back(std::log(fluence[i]));
    y.push_back(width[i] * width[i]);
  }
  const size_t m = x.size();
  if (m >= 1 && beam_d > 0) {
    // mean of ln F_th,i = ln F_i - Gamma_i^2 / a^2
    double s = 0;
    for (size_t i = 0; i < m; ++i) s += x[i] - y[i] / (beam_d * beam_d);
    *f_th_fixed = std::exp(s / (double)m);
  }
  if (m >= 2) {
    double xm = 0, ym = 0;
    for (size_t i = 0; i < m; ++i) {
      xm += x[i];
      ym += y[i];
    }
    xm /= (double)m;
    ym /= (double)m;
    double sxx = 0, sxy = 0;
    for (size_t i = 0; i < m; ++i) {
      sxx += (x[i] - xm) * (x[i] - xm);
      sxy += (x[i] - xm) * (y[i] - ym);
    }
    if (sxx > 0) {
      const double slope = sxy / sxx, icpt = ym - slope * xm;
      if (slope > 0) {
        *beam_d_fit = std::sqrt(slope);
        *f_th_fit = std::exp(-icpt / slope);
      }
    }
  }
  return PIC_OK;
}

}  // extern "C"

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
    double u;
    if (pot.kind == PIC_POT_MORSE) {
      const double e = std::exp(-pot.alpha * (r - pot.r0));
      u = 2.0 * pot.alpha * pot.D * (e - e * e);
    } else {
      const double x6 = std::pow(pot.r0 / r, 6);
      u = 12.0 * pot.D / r * (x6 - x6 * x6);
    }
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
    if (pot.lattice == PIC_LATTICE_HCP) {
      // 3 neighbours at +sqrt(2/3) along the normal and 3 at -sqrt(2/3); the
      // 6 basal neighbours add nothing along it
      const double c = std::cbrt(std::sqrt(2.0)), sn = std::sqrt(2.0 / 3.0);
      const double q = std::min(std::max(c * g * sn, -pot.g_clamp), pot.g_clamp);
      return 3.0 * sn * (dphi(c * rbar / (1.0 - 0.5 * q)) - dphi(c * rbar / (1.0 + 0.5 * q)));
    }
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

extern "C" int pic_calibrate_catt(const pic_grid_t *grid, const pic_potential_t *pot, double n_solid,
                                  int32_t slab_layers, double *c_att, double *work) {
  Sizes sz;
  if (!grid_sizes(grid, &sz, nullptr) || !valid_potential(pot) || !(n_solid > 0) || slab_layers < 2 || !c_att)
    return PIC_EINVAL;
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
