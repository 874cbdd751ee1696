// Tiled, fused time step of the PIC pair-potential cycle (arXiv 1502.07722)
// for gfx950.
//
// A context advances one or more independent slabs (grids).  Particles live
// in an internal structure-of-arrays store binned by tile (a block of cells
// of one slab, shorter along the last axis if the tiling asks for it).
// Within a tile the order is permuted once, at import (2D: a multiplicative
// scramble; 3D: layers of one particle per cell), so that the lanes of a
// wavefront hold particles of different cells (few same-address LDS atomics
// in the deposit).  A work item is a chunk of one tile's particles.  Each
// step is one persistent launch: block k starts with item k and takes the
// rest from an atomic counter; per item:
//   1. stage the node densities of the tile plus a halo (window) from the
//      int64 node sums of this step into LDS, and the cell-centred gradients;
//   2. for each particle: gather density and gradient (LDS), eq. (1)-(3)
//      force, leapfrog push, write the state back, and deposit the new
//      position into an LDS int64 accumulator;
//   3. flush the accumulator into the next step's node sums (global int64
//      atomics); every block also clears its share of the node buffer of the
//      step after next.
// Particles that drifted outside their window since the last binning go to
// the item's drifter list, which the block advances at the end of the item
// through the global node sums with the same arithmetic (same bits).  The
// int64 sums make the result independent of order, tiling, binning period
// and batching.
#include "pic_internal.h"
#include "pic_adjoint_dev.h"

#include <type_traits>

namespace pic {

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int fold_node(const Geo &g, int d, int a) {
  // node coordinate -> stored node: periodic wrap, mirror across reflecting
  // walls.  Callers stay within a few cells of the domain, so conditional
  // wraps replace integer division.
  const int n = g.n[d];
  if (!g.bc[d]) {
    while (a < 0) a += n;
    while (a >= n) a -= n;
    return a;
  }
  while (a < 0 || a > n) a = a < 0 ? -a : 2 * n - a;
  return a;
}

template <int ND>
__device__ __forceinline__ void unpack_cell(const TileGeo &tg, int pc, int idx[3]) {
  idx[0] = pc & tg.pmask[0];
  idx[1] = (pc >> tg.pshift[1]) & tg.pmask[1];
  idx[2] = ND == 3 ? (pc >> tg.pshift[2]) : 0;
}

template <int ND>
__device__ __forceinline__ int pack_cell(const TileGeo &tg, const int idx[3]) {
  int pc = idx[0] | (idx[1] << tg.pshift[1]);
  if (ND == 3) pc |= idx[2] << tg.pshift[2];
  return pc;
}

template <int ND>
__device__ __forceinline__ int tile_of(const TileGeo &tg, const int idx[3]) {
  int t = (idx[0] >> tg.lt[0]) + tg.tn[0] * (idx[1] >> tg.lt[1]);
  if (ND == 3) t += tg.tn[0] * tg.tn[1] * (idx[2] >> tg.lt[2]);
  return t;
}

// Window coordinate of cell / node coordinate c along axis d for a window whose
// first node is at coordinate o: periodic axes pick the representative in
// [lo, lo + n).  The tiled path only runs when every periodic axis is at least
// as long as the window, so c - o lies in [lo - n, lo + 2n) and one
// conditional add or subtract is enough.
__device__ __forceinline__ int window_coord(const Geo &g, int d, int c, int o, int lo) {
  int l = c - o;
  if (!g.bc[d]) {
    const int n = g.n[d];
    l = l < lo ? l + n : l;
    l = l >= lo + n ? l - n : l;
  }
  return l;
}

// Wave-aggregated atomic add of 1 per lane on counter[key]; returns this lane's
// rank (old value + position among lanes with the same key).  Every lane of
// the wavefront must call it; lanes with active == false take part but get -1.
__device__ __forceinline__ int wave_rank(int *counter, int key, bool active) {
  const int lane = threadIdx.x & 63;
  unsigned long long todo = __ballot(active);
  int out = -1;
  while (todo) {
    int leader = __ffsll((long long)todo) - 1;
    int lkey = __shfl(key, leader, 64);
    unsigned long long same = __ballot(active && key == lkey) & todo;
    int base = 0;
    if (lane == leader) base = atomicAdd(&counter[lkey], __popcll(same));
    base = __shfl(base, leader, 64);
    if ((same >> lane) & 1ull) out = base + __popcll(same & ((1ull << lane) - 1ull));
    todo &= ~same;
  }
  return out;
}

// q = k / d, r = k - q d for 0 <= k < 2^22 and 0 < d < 2^10, from a float
// reciprocal estimate (off by at most one) and one correction: exact.
__device__ __forceinline__ int div_small(int k, int d, float inv, int &r) {
  int q = (int)((float)k * inv);
  r = k - __umul24(q, d);
  if (r < 0) {
    q -= 1;
    r += d;
  } else if (r >= d) {
    q += 1;
    r -= d;
  }
  return q;
}

// Order of the particles inside a tile: ranks (arrival order at import) are
// taken in groups of kScrGroup consecutive ranks, and a group of len ranks is
// permuted by r -> (r * P) mod len with a prime P that does not divide len
// (a bijection that spreads same-cell runs, so that a wavefront's lanes hold
// particles of different cells); groups of at most 64 keep their order.  A
// group fits in LDS, so import and export can permute it there and touch HBM
// only in whole lines.
constexpr int kScrGroup = 4096;

__device__ __forceinline__ uint32_t scramble_prime(uint32_t L) {
  const uint32_t primes[3] = {40009u, 50021u, 60013u};
  uint32_t P = primes[0];
  if (L % P == 0) P = primes[1];
  if (L % P == 0) P = primes[2];
  return P;
}

// The group's positions of ranks r0, r0 + stride, r0 + 2 stride, ... (r0 <
// len): q advances by (stride * P) mod len, with one conditional subtraction.
struct ScrWalk {
  uint32_t q, step, len;
  __device__ __forceinline__ ScrWalk(int r0, int stride, int len_) : len((uint32_t)len_) {
    if (len <= 64) {
      q = (uint32_t)r0;
      step = (uint32_t)stride;
    } else {
      const uint64_t P = scramble_prime(len);
      q = (uint32_t)((uint64_t)(uint32_t)r0 * P % len);
      step = (uint32_t)((uint64_t)(uint32_t)stride * P % len);
    }
  }
  __device__ __forceinline__ void next() {
    q += step;
    if (len > 64 && q >= len) q -= len;
  }
};

// 3D tiles take the ranks of a group in layers instead: rank r goes to the
// column-major position of a row-major matrix of k columns, k the tile's
// mean particles per cell.  With ranks in cell order (a caller order that
// keeps a cell's particles together), layer c holds the c-th particle of
// each cell, cells in rank order, so the 64 lanes of a wavefront hold
// particles of 64 different, neighbouring cells: the window gathers touch
// nearby words and no two lanes of a deposit atomic share an address.  (In
// 2D, with 32 particles per cell, the multiplicative scramble measured
// faster.)  Any other caller order gives some other bijection: the results
// never depend on the order.
template <int ND>
struct TileOrder {
  ScrWalk w;
  int r, stride, k, m, rem;
  float ik;
  __device__ __forceinline__ TileOrder(int r0, int stride_, int len, int tile_count, int tile_cells)
      : w(r0, stride_, len), r(r0), stride(stride_) {
    k = len <= 64 ? 1 : max(1, min(1023, (tile_count + tile_cells / 2) / tile_cells));
    m = len / k;
    rem = len - m * k;
    ik = 1.0f / (float)k;
  }
  __device__ __forceinline__ int pos() const {
    if (ND == 2) return (int)w.q;
    int col;
    const int row = div_small(r, k, ik, col);  // r = row k + col
    return col * m + min(col, rem) + row;
  }
  __device__ __forceinline__ void next() {
    if (ND == 2) w.next();
    else r += stride;
  }
};

// ---------------------------------------------------------------------------
// Fused step
// ---------------------------------------------------------------------------
struct Window {
  int o[3];   // node coordinate of window node 0 per axis
  int wn[3];  // window nodes per axis (T + 2H + 3)
  int nW, nC; // window nodes, window centres
  int sy, sz; // node strides along y and z (wn0, wn0 wn1)
  int cy, cz; // centre strides along y and z ((wn0 - 1), (wn0 - 1)(wn1 - 1))
};

// Window indices (coordinates are non-negative and small: 24-bit multiplies).
template <int ND>
__device__ __forceinline__ int win_node(const Window &w, int a0, int a1, int a2) {
  return ND == 2 ? a0 + __umul24(w.sy, a1) : a0 + __umul24(w.sy, a1) + __umul24(w.sz, a2);
}
template <int ND>
__device__ __forceinline__ int win_centre(const Window &w, int m0, int m1, int m2) {
  return ND == 2 ? m0 + __umul24(w.cy, m1) : m0 + __umul24(w.cy, m1) + __umul24(w.cz, m2);
}
// Offset of corner k (bit d set = upper along d) from a cell's lower node /
// from the lower centre of a centre cube.
template <int ND>
__device__ __forceinline__ int node_corner(const Window &w, int k) {
  return (k & 1) + ((k >> 1) & 1) * w.sy + (ND == 3 ? ((k >> 2) & 1) * w.sz : 0);
}
template <int ND>
__device__ __forceinline__ int centre_corner(const Window &w, int k) {
  return (k & 1) + ((k >> 1) & 1) * w.cy + (ND == 3 ? ((k >> 2) & 1) * w.cz : 0);
}


// Index in a 3^ND block of nodes (per-axis offsets 0..2).
template <int ND>
__device__ __forceinline__ constexpr int b3(int a0, int a1, int a2) {
  return ND == 2 ? a0 + 3 * a1 : a0 + 3 * (a1 + 3 * a2);
}

// Global (window-free) density and gradient at a particle, folded like the
// window (so the values are the same bits as the window's).  All nodes come
// from one 3^ND block, from the lower centre's lower node c0 (folded once
// per axis): G from the 2^ND nearest centres, whose corners the block holds,
// and n from the own cell's corners, at block offsets idx - c0 (0 or 1 per
// axis).  Only particles that left their tile window since the last binning
// come here.
template <int ND>
__device__ __forceinline__ void gather_nodes_global(const Geo &g, const long long *__restrict__ N, const int idx[3],
                                                    const float f[3], float &nh, float Gp[3]) {
  int c0[3] = {0, 0, 0};
  float t[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int e = 0; e < ND; ++e) centre_stencil(idx[e], f[e], c0[e], t[e]);
  // a block away from the domain's edges needs no fold and no wall factor
  bool plain = true;
#pragma unroll
  for (int e = 0; e < ND; ++e) plain = plain && c0[e] >= 1 && c0[e] + 2 < g.n[e];
  constexpr int K3 = ND == 2 ? 9 : 27;
  float d3[K3];
  if (plain) {
    const int b = node_index<ND>(g, c0[0], c0[1], c0[2]);
#pragma unroll
    for (int a = 0; a < K3; ++a) {
      const int o = a % 3 + g.nn[0] * ((a / 3) % 3 + (ND == 3 ? g.nn[1] * (a / 9) : 0));
      d3[a] = wsum_float(N[b + o]) * g.kappa;
    }
  } else {
    int ax[3][3];
#pragma unroll
    for (int e = 0; e < 3; ++e)
#pragma unroll
      for (int j = 0; j < 3; ++j) ax[e][j] = e < ND ? fold_node(g, e, c0[e] + j) : 0;
#pragma unroll
    for (int a = 0; a < K3; ++a) {
      const int x = ax[0][a % 3], y = ax[1][(a / 3) % 3], z = ND == 3 ? ax[2][a / 9] : 0;
      d3[a] = node_density(g, N[node_index<ND>(g, x, y, z)], x, y, z);
    }
  }
  // all-ones masks of the offsets: the corners are picked by bitwise blends of
  // values, so the block stays in registers (no indexing by a run-time offset)
  const uint32_t m0 = idx[0] != c0[0] ? ~0u : 0u, m1 = idx[1] != c0[1] ? ~0u : 0u;
  const uint32_t m2 = ND == 3 && idx[2] != c0[2] ? ~0u : 0u;
  auto blend = [](float a, float b, uint32_t m) {  // m ? b : a
    return __uint_as_float((__float_as_uint(a) & ~m) | (__float_as_uint(b) & m));
  };
  float cr[8];
#pragma unroll
  for (int k = 0; k < (1 << ND); ++k) {
    const int b0 = k & 1, b1 = (k >> 1) & 1, b2 = ND == 3 ? (k >> 2) & 1 : 0;
    const float lo = blend(blend(d3[b3<ND>(b0, b1, b2)], d3[b3<ND>(b0 + 1, b1, b2)], m0),
                           blend(d3[b3<ND>(b0, b1 + 1, b2)], d3[b3<ND>(b0 + 1, b1 + 1, b2)], m0), m1);
    if (ND == 3) {
      const float hi = blend(blend(d3[b3<ND>(b0, b1, b2 + 1)], d3[b3<ND>(b0 + 1, b1, b2 + 1)], m0),
                             blend(d3[b3<ND>(b0, b1 + 1, b2 + 1)], d3[b3<ND>(b0 + 1, b1 + 1, b2 + 1)], m0), m1);
      cr[k] = blend(lo, hi, m2);
    } else {
      cr[k] = lo;
    }
  }
  nh = interp<ND>(cr, f);
  float vv[3][8];
#pragma unroll
  for (int m = 0; m < (1 << ND); ++m) {
    float c[8], Gc[3];
#pragma unroll
    for (int j = 0; j < (1 << ND); ++j)
      c[j] = d3[b3<ND>((m & 1) + (j & 1), ((m >> 1) & 1) + ((j >> 1) & 1), ND == 3 ? ((m >> 2) & 1) + ((j >> 2) & 1) : 0)];
    centre_gradient<ND>(g, c, Gc);
#pragma unroll
    for (int d = 0; d < ND; ++d) vv[d][m] = Gc[d];
  }
  Gp[2] = 0.0f;
#pragma unroll
  for (int d = 0; d < ND; ++d) Gp[d] = interp<ND>(vv[d], t);
}

template <int ND>
__device__ __forceinline__ void deposit_global(const Geo &g, unsigned long long *__restrict__ N, const int idx[3],
                                               const uint32_t t[8]) {
#pragma unroll
  for (int k = 0; k < (1 << ND); ++k) {
    if (!t[k]) continue;
    int x = node_axis(g, 0, idx[0] + (k & 1)), y = node_axis(g, 1, idx[1] + ((k >> 1) & 1));
    int z = ND == 3 ? node_axis(g, 2, idx[2] + ((k >> 2) & 1)) : 0;
    atomicAdd(&N[node_index<ND>(g, x, y, z)], (unsigned long long)t[k]);
  }
}

template <int ND>
__device__ __forceinline__ Window make_window(const TileGeo &tg, int tile) {
  Window w;
  int tx = tile % tg.tn[0];
  int r = tile / tg.tn[0];
  int ty = ND == 2 ? r : r % tg.tn[1];
  int tz = ND == 2 ? 0 : r / tg.tn[1];
  w.o[0] = (tx << tg.lt[0]) - tg.H - 1;
  w.o[1] = (ty << tg.lt[1]) - tg.H - 1;
  w.o[2] = ND == 3 ? (tz << tg.lt[2]) - tg.H - 1 : 0;
  w.nW = 1;
  w.nC = 1;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    w.wn[d] = d < ND ? (1 << tg.lt[d]) + 2 * tg.H + 3 : 1;
    w.nW *= w.wn[d];
    w.nC *= d < ND ? w.wn[d] - 1 : 1;
  }
  w.sy = w.wn[0];
  w.sz = w.wn[0] * w.wn[1];
  w.cy = w.wn[0] - 1;
  w.cz = (w.wn[0] - 1) * (w.wn[1] - 1);
  return w;
}

// Mixed-radix digits (a0, a1, a2) of k = k0, k0 + stride, k0 + 2 stride, ...
// over radices (r0, r1): each step adds the stride's digits with one
// conditional carry per digit (k0, stride < 2^22; r0, r1 < 2^10).
template <int ND>
struct Walk {
  int a[3], s[3], r0, r1;
  __device__ __forceinline__ Walk(int k0, int stride, int r0_, int r1_) : r0(r0_), r1(r1_) {
    const float i0 = 1.0f / (float)r0, i1 = 1.0f / (float)r1;
    int q = div_small(k0, r0, i0, a[0]);
    int t = div_small(stride, r0, i0, s[0]);
    if (ND == 2) {
      a[1] = q;
      s[1] = t;
      a[2] = s[2] = 0;
    } else {
      a[2] = div_small(q, r1, i1, a[1]);
      s[2] = div_small(t, r1, i1, s[1]);
    }
  }
  __device__ __forceinline__ void next() {
    a[0] += s[0];
    const int c0 = a[0] >= r0 ? 1 : 0;
    a[0] -= c0 ? r0 : 0;
    a[1] += s[1] + c0;
    if (ND == 3) {
      const int c1 = a[1] >= r1 ? 1 : 0;
      a[1] -= c1 ? r1 : 0;
      a[2] += s[2] + c1;
    }
  }
};

// Uniform properties of a window: every window node is a stored node as it
// stands (no periodic wrap or mirror), and none lies on a reflecting wall.
template <int ND>
__device__ __forceinline__ void window_flags(const Geo &g, const Window &w, bool &nofold, bool &nowall) {
  nofold = true;
  nowall = true;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    nofold = nofold && w.o[d] >= 0 && w.o[d] + w.wn[d] <= g.nn[d];
    nowall = nowall && (!g.bc[d] || (w.o[d] > 0 && w.o[d] + w.wn[d] - 1 < g.n[d]));
  }
}

// Stored node of window node a (folded like the global path).
template <int ND>
__device__ __forceinline__ void window_node(const Geo &g, const Window &w, const int a[3], bool nofold, int x[3]) {
  if (nofold) {
#pragma unroll
    for (int d = 0; d < 3; ++d) x[d] = d < ND ? w.o[d] + a[d] : 0;
  } else {
#pragma unroll
    for (int d = 0; d < 3; ++d) x[d] = d < ND ? fold_node(g, d, w.o[d] + a[d]) : 0;
  }
}

// The centre gradients of a staged window (the same function and inputs as
// every other path: the same bits), one plane per component; ends with a
// barrier.
template <int ND>
__device__ __forceinline__ void stage_gradients(const Geo &g, const Window &w, const float *dens, float *Gs) {
  Walk<ND> ic((int)threadIdx.x, (int)blockDim.x, w.cy, w.wn[1] - 1);
  for (int m = threadIdx.x; m < w.nC; m += blockDim.x, ic.next()) {
    const int nb = win_node<ND>(w, ic.a[0], ic.a[1], ic.a[2]);
    float c[8], G[3];
#pragma unroll
    for (int k = 0; k < (1 << ND); ++k) c[k] = dens[nb + node_corner<ND>(w, k)];
    centre_gradient<ND>(g, c, G);
#pragma unroll
    for (int d = 0; d < ND; ++d) Gs[d * w.nC + m] = G[d];  // one plane per component
  }
  __syncthreads();
}

// Stage the window: densities of the window nodes (folded like the global
// path) and the centre gradients between them; clear the accumulator.
template <int ND>
__device__ __forceinline__ void stage_window(const Geo &g, const Window &w, const long long *__restrict__ N,
                                             float *dens, float *Gs, unsigned long long *acc) {
  bool nofold, nowall;
  window_flags<ND>(g, w, nofold, nowall);
  Walk<ND> it((int)threadIdx.x, (int)blockDim.x, w.wn[0], w.wn[1]);
  for (int k = threadIdx.x; k < w.nW; k += blockDim.x, it.next()) {
    int x[3];
    window_node<ND>(g, w, it.a, nofold, x);
    const long long v = N[node_index<ND>(g, x[0], x[1], x[2])];
    dens[k] = nowall ? wsum_float(v) * g.kappa : node_density(g, v, x[0], x[1], x[2]);
    if (acc) acc[k] = 0ull;
  }
  __syncthreads();
  if (Gs) stage_gradients<ND>(g, w, dens, Gs);
}

template <int ND>
__device__ __forceinline__ void flush_window(const Geo &g, const Window &w, const unsigned long long *acc,
                                             unsigned long long *__restrict__ N) {
  bool nofold, nowall;
  window_flags<ND>(g, w, nofold, nowall);
  Walk<ND> it((int)threadIdx.x, (int)blockDim.x, w.wn[0], w.wn[1]);
  for (int k = threadIdx.x; k < w.nW; k += blockDim.x, it.next()) {
    const unsigned long long v = acc[k];
    if (!v) continue;
    // deposits only ever land on nodes inside the domain; wrap periodic axes
    int x[3];
    window_node<ND>(g, w, it.a, nofold, x);
    atomicAdd(&N[node_index<ND>(g, x[0], x[1], x[2])], v);
  }
}

__device__ __forceinline__ void clear_share(long long *__restrict__ Z, int nnodes) {
  if (!Z) return;
  int share = (nnodes + gridDim.x - 1) / gridDim.x;
  int lo = blockIdx.x * share, hi = min(nnodes, lo + share);
  for (int k = lo + threadIdx.x; k < hi; k += blockDim.x) Z[k] = 0;
}

// Window coordinates of a cell; returns true if inside [lo, hi] on every axis.
// edges: bit d clear = the window does not reach the periodic seam along d,
// where a plain difference is then exact.
template <int ND>
__device__ __forceinline__ bool in_window(const Geo &g, const Window &w, const int idx[3], int lo, int hi_off,
                                          int l[3], uint32_t edges = 7u) {
  bool ok = true;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    l[d] = ((edges >> d) & 1u) ? window_coord(g, d, idx[d], w.o[d], lo) : idx[d] - w.o[d];
    ok = ok && l[d] >= lo && l[d] <= w.wn[d] - hi_off;
  }
  return ok;
}

// Axes along which a tile window reaches a reflecting wall or the periodic
// seam (bit d): a particle of the item loop stays a cell away from both along
// the other axes, so it never mirrors or wraps there.
template <int ND>
__device__ __forceinline__ uint32_t window_edges(const Geo &g, const Window &w) {
  uint32_t e = 0;
#pragma unroll
  for (int d = 0; d < ND; ++d)
    if (!(w.o[d] >= 0 && w.o[d] + w.wn[d] <= g.n[d] + 1)) e |= 1u << d;
  return e;
}


// Per-array views of the store with 32-bit element offsets (the tiled path
// keeps max_n < 2^30, so byte offsets fit in 32 bits).
struct StoreView {
  const int *pc;
  const float *off[3];
  const float *vel[3];
  const int *wq;
  int *pc_o;           // outputs: the same arrays (in place) or the next
  float *off_o[3];     // state's arrays (out of place, when a trajectory
  float *vel_o[3];     // is recorded)
};

// OUT false: in place (o is s), so the outputs are the inputs' own pointers
// (one set of pointer registers).
template <bool OUT = true>
__device__ __forceinline__ StoreView view_of(const Store &s, const Store &o) {
  const Store &w = OUT ? o : s;
  StoreView v;
  v.pc = s.pc;
  v.wq = s.wq;
  v.pc_o = w.pc;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    v.off[d] = s.off + d * s.cap;
    v.vel[d] = s.vel + d * s.cap;
    v.off_o[d] = w.off + d * w.cap;
    v.vel_o[d] = w.vel + d * w.cap;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T &at(T *base, int p) {
  return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + (uint32_t)p * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ const T &at(const T *base, int p) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + (uint32_t)p * (uint32_t)sizeof(T));
}

// One particle's state in registers.
struct PState {
  int pc;
  float f[3];
  float v[3];
  int W;
};

// Loads of a slot inside the store (lanes past the item's end read its last
// slot and ignore it): no branch.
template <int ND, bool DIAG>
__device__ __forceinline__ void load_state_any(const StoreView &sv, int p, PState &q) {
  q.pc = at(sv.pc, p);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    q.f[d] = d < ND ? at(sv.off[d], p) : 0.0f;
    q.v[d] = d < ND || (ND == 2 && DIAG) ? at(sv.vel[d], p) : 0.0f;
  }
  q.W = at(sv.wq, p);
}

template <int ND, bool DIAG>
__device__ __forceinline__ void load_state(const StoreView &sv, int p, bool live, PState &q) {
  q.pc = 0;
  q.W = 0;
  q.f[0] = q.f[1] = q.f[2] = 0.0f;
  q.v[0] = q.v[1] = q.v[2] = 0.0f;
  if (live) {
    q.pc = at(sv.pc, p);
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      q.f[d] = at(sv.off[d], p);
      q.v[d] = at(sv.vel[d], p);
    }
    if (ND == 2 && DIAG) q.v[2] = at(sv.vel[2], p);
    q.W = at(sv.wq, p);
  }
}

// Force, push, state write-back and the new position's deposit shares of one
// particle, given its gathered density and gradient.
// OUT: the next state goes to the view's output arrays (a recorded
// trajectory); otherwise in place.
template <int ND, bool DIAG, bool INTERIOR, bool OUT, bool GEN>
__device__ __forceinline__ void advance_particle(const Geo &g, const Pot &P, const DiagC &dc, const TileGeo &tg,
                                                 const StoreView &sv, int p, int pc, int idx[3], float f[3],
                                                 float v[3], int W, float nh, const float Gp[3], uint32_t tq[8],
                                                 uint32_t &err, double acc6[6], uint32_t edges = 7u) {
  float Fh[3], bond = 0.0f;
  pair_force<ND, GEN>(P, nh, Gp, Fh, DIAG ? &bond : nullptr);
  float F[3] = {Fh[0] * P.beta, Fh[1] * P.beta, ND == 3 ? Fh[2] * P.beta : 0.0f};
  if (DIAG) {
    double wgt = (double)W * dc.wunit, vo2 = 0.0, vn2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      float vn = d < ND ? __builtin_fmaf(F[d], P.gv, v[d]) : v[d];
      vo2 += (double)v[d] * v[d];
      vn2 += (double)vn * vn;
      acc6[1 + d] += wgt * dc.mass * 0.5 * ((double)v[d] + (double)vn);
    }
    acc6[0] += wgt * dc.half_m * 0.5 * (vo2 + vn2);
    acc6[4] += wgt;
    acc6[5] += wgt * (double)bond * dc.D;
  }
  err |= push_particle<ND, INTERIOR>(g, P, F, idx, f, v, edges);
  const int pc2 = pack_cell<ND>(tg, idx);
  if (pc2 != pc || OUT) at(sv.pc_o, p) = pc2;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    at(sv.off_o[d], p) = f[d];
    at(sv.vel_o[d], p) = v[d];
  }
  // 2D: v_z is never changed; an out-of-place step still carries it over
  if (ND == 2 && OUT) at(sv.vel_o[2], p) = DIAG ? v[2] : at(sv.vel[2], p);
  deposit_shares<ND>((uint32_t)W, f, tq);
}

// ---------------------------------------------------------------------------
// Slab tables: a context advances one or more independent slabs (grids) in the
// same launches.  Store slots, tiles and node arrays of the slabs are
// concatenated; small offset tables map a slot or tile back to its slab.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_slab(const int *__restrict__ offs, int nslab, int x) {
  int lo = 0, hi = nslab - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (offs[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Binning: histogram by tile, scan, items, scatter.
// ---------------------------------------------------------------------------
// Import of the caller's arrays of one slab, in three passes: tile counts;
// each particle's caller index at the next free rank of its tile (arrival
// order: a wavefront's lanes of one tile take consecutive ranks, so these
// writes, and the reads of the last pass, are whole lines whenever the
// caller's order keeps a tile's particles together); and one block per tile
// that reads the particles in rank order, permutes each group of ranks in LDS
// and writes the tile's store slots in order.
//
// Only the cell decides the tile: a cell outside the grid is an error and its
// particle is left out; offsets and weights are checked in the last pass.
template <int ND>
__device__ __forceinline__ int import_tile(const SlabDesc &sd, const PartPtrs &cp, int64_t p, int idx[3],
                                           uint32_t *err) {
  const int c = cp.cell[p];
  if (c < 0 || c >= sd.g.ncells) {
    if (err) atomicOr(err, ERR_RANGE);
    return -1;
  }
  decode_cell<ND>(sd.g, c, idx);
  return sd.tile_off + tile_of<ND>(sd.tg, idx);
}

// The first two passes give each wavefront kWaveRuns x 64 consecutive
// particles (lane l takes particles c * 64 + l).  When all of them share one
// tile -- the common case for a caller order that keeps a tile's particles
// together -- a single atomic counts them or reserves their ranks; otherwise
// each 64-particle chunk goes through wave_rank (one atomic per distinct
// tile in the chunk).
constexpr int kWaveRuns = 4;

__device__ __forceinline__ int64_t import_wave_base() {
  return ((int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63)) * kWaveRuns;
}

__device__ __forceinline__ bool one_tile(const int t[kWaveRuns]) {
  const int t0 = __shfl(t[0], 0, 64);
  bool same = t0 >= 0;
#pragma unroll
  for (int c = 0; c < kWaveRuns; ++c) same = same && t[c] == t0;
  return __ballot(!same) == 0ull;
}

template <int ND>
__global__ void __launch_bounds__(256) k_import_hist(SlabDesc sd, PartPtrs cp, int *__restrict__ counts,
                                                     uint32_t *__restrict__ err) {
  const int64_t p0 = import_wave_base() + (threadIdx.x & 63);
  int t[kWaveRuns], idx[3];
#pragma unroll
  for (int c = 0; c < kWaveRuns; ++c) {
    const int64_t p = p0 + c * 64;
    t[c] = p < cp.n ? import_tile<ND>(sd, cp, p, idx, err) : -1;
  }
  if (one_tile(t)) {
    if ((threadIdx.x & 63) == 0) atomicAdd(&counts[t[0]], 64 * kWaveRuns);
    return;
  }
#pragma unroll
  for (int c = 0; c < kWaveRuns; ++c) wave_rank(counts, t[c] < 0 ? 0 : t[c], t[c] >= 0);
}

template <int ND>
__global__ void __launch_bounds__(256) k_import_index(SlabDesc sd, PartPtrs cp, const int *__restrict__ starts,
                                                      int *__restrict__ cursors, int *__restrict__ stage) {
  const int lane = threadIdx.x & 63;
  const int64_t p0 = import_wave_base() + lane;
  int t[kWaveRuns], idx[3];
#pragma unroll
  for (int c = 0; c < kWaveRuns; ++c) {
    const int64_t p = p0 + c * 64;
    t[c] = p < cp.n ? import_tile<ND>(sd, cp, p, idx, nullptr) : -1;
  }
  if (one_tile(t)) {
    int base = 0;
    if (lane == 0) base = atomicAdd(&cursors[t[0]], 64 * kWaveRuns);
    base = __shfl(base, 0, 64) + starts[t[0]];
#pragma unroll
    for (int c = 0; c < kWaveRuns; ++c) stage[base + c * 64 + lane] = (int)(p0 + c * 64);
    return;
  }
#pragma unroll
  for (int c = 0; c < kWaveRuns; ++c) {
    const int r = wave_rank(cursors, t[c] < 0 ? 0 : t[c], t[c] >= 0);
    if (t[c] >= 0) stage[starts[t[c]] + r] = (int)(p0 + c * 64);
  }
}

// One block per tile of the slab (blockIdx.x = tile within the slab), 1024
// threads.  The fields go through LDS four at a time: each thread loads four
// fields of each of its ranks before it stores any of them, and a group of
// 4096 ranks takes two (2D) or three (3D) passes with two barriers each.
constexpr int kGatherThreads = 1024;
constexpr int kFieldsPerPass = 4;

template <int ND>
__device__ __forceinline__ int import_field(const SlabDesc &sd, const PartPtrs &cp, int k, int64_t p, uint32_t &e) {
  // field k: 0 packed cell, 1..ND offsets, ND+1..ND+3 velocity, ND+4 weight,
  // ND+5 caller index
  if (k == 0) {
    int idx[3];
    decode_cell<ND>(sd.g, cp.cell[p], idx);
    return pack_cell<ND>(sd.tg, idx);
  }
  if (k <= ND) {
    const float f = cp.off[(int64_t)(k - 1) * cp.n + p];
    if (!(f >= 0.0f && f < 1.0f)) e |= ERR_RANGE;
    return __float_as_int(f);
  }
  if (k <= ND + 3) return __float_as_int(cp.vel[(int64_t)(k - ND - 1) * cp.n + p]);
  if (k == ND + 4) {
    const int W = cp.wq[p];
    if (W < 0) e |= ERR_WEIGHT;
    return W;
  }
  return (int)p;
}

template <int ND>
__global__ void __launch_bounds__(kGatherThreads) k_import_gather(SlabDesc sd, PartPtrs cp, Store d,
                                                                  const int *__restrict__ counts,
                                                                  const int *__restrict__ starts,
                                                                  const int *__restrict__ stage,
                                                                  uint32_t *__restrict__ err) {
  __shared__ int s_v[kFieldsPerPass][kScrGroup];
  constexpr int NF = ND + 6;
  const int t = sd.tile_off + (int)blockIdx.x;
  const int L = counts[t], s0 = starts[t];
  const int tile_cells = 1 << (sd.tg.lt[0] + sd.tg.lt[1] + (ND == 3 ? sd.tg.lt[2] : 0));
  const int tid = threadIdx.x, B = blockDim.x;
  uint32_t e = 0;
  for (int g0 = 0; g0 < L; g0 += kScrGroup) {
    const int len = min(kScrGroup, L - g0);
    const int64_t base = (int64_t)s0 + g0;
    for (int k0 = 0; k0 < NF; k0 += kFieldsPerPass) {
      // gathered in rank order, permuted in LDS ...
      TileOrder<ND> w(tid, B, len, L, tile_cells);
      for (int r = tid; r < len; r += B, w.next()) {
        const int64_t p = stage[base + r];
        int v[kFieldsPerPass];
#pragma unroll
        for (int j = 0; j < kFieldsPerPass; ++j) v[j] = k0 + j < NF ? import_field<ND>(sd, cp, k0 + j, p, e) : 0;
        const int q = w.pos();
#pragma unroll
        for (int j = 0; j < kFieldsPerPass; ++j) s_v[j][q] = v[j];
      }
      __syncthreads();
      // ... and written in slot order
#pragma unroll
      for (int j = 0; j < kFieldsPerPass; ++j) {
        const int k = k0 + j;
        if (k >= NF) break;
        int *dst = k == 0 ? d.pc
                   : k <= ND ? reinterpret_cast<int *>(d.off) + (int64_t)(k - 1) * d.cap
                   : k <= ND + 3 ? reinterpret_cast<int *>(d.vel) + (int64_t)(k - ND - 1) * d.cap
                   : k == ND + 4 ? d.wq : d.oidx;
        for (int q = tid; q < len; q += B) dst[base + q] = s_v[j][q];
      }
      __syncthreads();
    }
  }
  if (e) atomicOr(err, e);
}

// Re-binning of the store: the slab of a slot comes from the slot ranges.
template <int ND>
__device__ __forceinline__ int store_tile(const Batch &b, const Store &s, int p, int idx[3]) {
  const int k = find_slab(b.part_offs, b.nslab, p);
  const TileGeo tg = b.slabs[k].tg;
  unpack_cell<ND>(tg, s.pc[p], idx);
  return b.slabs[k].tile_off + tile_of<ND>(tg, idx);
}

template <int ND>
__global__ void __launch_bounds__(256) k_rebin_hist(Batch b, Store s, int *__restrict__ counts) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  int idx[3];
  int t = p < b.nparts ? store_tile<ND>(b, s, p, idx) : -1;
  wave_rank(counts, t < 0 ? 0 : t, t >= 0);
}

template <int ND>
__global__ void __launch_bounds__(256) k_rebin_scatter(Batch b, Store s, Store d, const int *__restrict__ starts,
                                                       int *__restrict__ cursors) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  int idx[3];
  int t = p < b.nparts ? store_tile<ND>(b, s, p, idx) : -1;
  // ranks keep the (already scrambled) order of each wavefront's run: coalesced writes
  int r = wave_rank(cursors, t < 0 ? 0 : t, t >= 0);
  if (t < 0) return;
  const int64_t q = starts[t] + r;
  d.pc[q] = s.pc[p];
#pragma unroll
  for (int k = 0; k < ND; ++k) d.off[k * d.cap + q] = s.off[k * s.cap + p];
#pragma unroll
  for (int k = 0; k < 3; ++k) d.vel[k * d.cap + q] = s.vel[k * s.cap + p];
  d.wq[q] = s.wq[p];
  d.oidx[q] = s.oidx[p];
}

// Exclusive scans of the tile counts -> starts and of the items per tile
// (ceil(count / chunk)) -> item_start, both with a final total entry, in
// three launches: per-block sums of 1024 tiles, one block scanning those
// sums, then per-block scans offset by them (which also clear the cursors).
// aux: two ints per block of 1024 tiles.
constexpr int kScanBlock = 1024;

__device__ __forceinline__ int tile_item_count(int c, int chunk) { return (c + chunk - 1) / chunk; }

// Inclusive scan of one value per thread over a block of kScanBlock threads
// (wavefront prefix sums, then the wavefront totals).
__device__ __forceinline__ int block_inclusive_scan(int v, int *s_w) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  if (lane == 63) s_w[wv] = v;
  __syncthreads();
  if (wv == 0) {
    int t = lane < kScanBlock / 64 ? s_w[lane] : 0;
#pragma unroll
    for (int o = 1; o < kScanBlock / 64; o <<= 1) {
      const int u = __shfl_up(t, o, 64);
      if (lane >= o) t += u;
    }
    if (lane < kScanBlock / 64) s_w[lane] = t;
  }
  __syncthreads();
  const int r = v + (wv > 0 ? s_w[wv - 1] : 0);
  __syncthreads();  // s_w is reused by the next scan
  return r;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_sums(int ntiles, int chunk, const int *__restrict__ counts,
                                                          int *__restrict__ aux) {
  __shared__ int s_w[kScanBlock / 64];
  const int t = blockIdx.x * kScanBlock + threadIdx.x;
  const int c = t < ntiles ? counts[t] : 0;
  const int a = block_inclusive_scan(c, s_w);
  const int b = block_inclusive_scan(tile_item_count(c, chunk), s_w);
  if (threadIdx.x == kScanBlock - 1) {
    aux[2 * blockIdx.x] = a;
    aux[2 * blockIdx.x + 1] = b;
  }
}

// One block: exclusive scan of the per-block sums in place, and the totals.
__global__ void __launch_bounds__(kScanBlock) k_scan_totals(int nblocks, int ntiles, int *__restrict__ aux,
                                                            int *__restrict__ starts, int *__restrict__ item_start,
                                                            int *__restrict__ num_items) {
  __shared__ int s_w[kScanBlock / 64];
  __shared__ int s_tot[2];
  int ca = 0, cb = 0;  // carried over chunks of kScanBlock block sums
  for (int k0 = 0; k0 < nblocks; k0 += kScanBlock) {
    const int k = k0 + (int)threadIdx.x;
    const int a = k < nblocks ? aux[2 * k] : 0, b = k < nblocks ? aux[2 * k + 1] : 0;
    const int ia = block_inclusive_scan(a, s_w), ib = block_inclusive_scan(b, s_w);
    if (k < nblocks) {
      aux[2 * k] = ca + ia - a;
      aux[2 * k + 1] = cb + ib - b;
    }
    if (threadIdx.x == kScanBlock - 1) {
      s_tot[0] = ia;
      s_tot[1] = ib;
    }
    __syncthreads();
    ca += s_tot[0];
    cb += s_tot[1];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    starts[ntiles] = ca;
    item_start[ntiles] = cb;
    *num_items = cb;
  }
}

__global__ void __launch_bounds__(kScanBlock) k_scan_apply(int ntiles, int chunk, const int *__restrict__ counts,
                                                           const int *__restrict__ aux, int *__restrict__ starts,
                                                           int *__restrict__ item_start, int *__restrict__ cursors) {
  __shared__ int s_w[kScanBlock / 64];
  const int t = blockIdx.x * kScanBlock + threadIdx.x;
  const int c = t < ntiles ? counts[t] : 0, m = tile_item_count(c, chunk);
  const int ia = block_inclusive_scan(c, s_w), ib = block_inclusive_scan(m, s_w);
  if (t < ntiles) {
    starts[t] = aux[2 * blockIdx.x] + ia - c;
    item_start[t] = aux[2 * blockIdx.x + 1] + ib - m;
    cursors[t] = 0;
  }
}

// The three launches; aux lives in the item buffer, which k_tile_items
// overwrites afterwards (it holds at least one item per tile).
static void launch_tile_scan(hipStream_t st, int ntiles, int chunk, const BinBufs &bb) {
  const int nb = std::max(1, (ntiles + kScanBlock - 1) / kScanBlock);
  int *aux = reinterpret_cast<int *>(bb.items);
  k_scan_sums<<<nb, kScanBlock, 0, st>>>(ntiles, chunk, bb.counts, aux);
  k_scan_totals<<<1, kScanBlock, 0, st>>>(nb, ntiles, aux, bb.starts, bb.item_start, bb.num_items);
  k_scan_apply<<<nb, kScanBlock, 0, st>>>(ntiles, chunk, bb.counts, aux, bb.starts, bb.item_start, bb.cursors);
}

__global__ void __launch_bounds__(256) k_tile_items(Batch b, const int *__restrict__ counts,
                                                    const int *__restrict__ starts,
                                                    const int *__restrict__ item_start, Item *__restrict__ items) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= b.ntiles) return;
  const int slab = find_slab(b.tile_offs, b.nslab, t);
  // ceil(c / chunk) items of near-equal size (each at most chunk; the scan
  // counted them): equal items let the persistent grid finish its rounds
  // together
  const int c = counts[t], s = starts[t], i0 = item_start[t];
  const int m = item_start[t + 1] - i0;
  for (int k = 0; k < m; ++k)
    items[i0 + k] = Item{t, s + (int)((long long)k * c / m), s + (int)((long long)(k + 1) * c / m), slab};
}

// The inverse of the import gather: one 1024-thread block per tile, four
// fields per pass through LDS, each group's caller indices loaded once.
template <int ND>
__global__ void __launch_bounds__(kGatherThreads) k_export(SlabDesc sd, Store s, const int *__restrict__ starts,
                                                           PartPtrs cp) {
  __shared__ int s_o[kScrGroup];
  __shared__ int s_v[kFieldsPerPass][kScrGroup];
  constexpr int NF = ND + 4;  // field k: 0 cell, 1..ND offsets, ND+1..ND+3 velocity
  const int t = sd.tile_off + (int)blockIdx.x;
  const int s0 = starts[t], L = starts[t + 1] - s0;
  const int tile_cells = 1 << (sd.tg.lt[0] + sd.tg.lt[1] + (ND == 3 ? sd.tg.lt[2] : 0));
  const int tid = threadIdx.x, B = blockDim.x;
  for (int g0 = 0; g0 < L; g0 += kScrGroup) {
    const int len = min(kScrGroup, L - g0);
    const int64_t base = (int64_t)s0 + g0;
    for (int q = tid; q < len; q += B) s_o[q] = s.oidx[base + q];
    for (int k0 = 0; k0 < NF; k0 += kFieldsPerPass) {
      // slots read in order ...
      for (int q = tid; q < len; q += B) {
        int v[kFieldsPerPass];
#pragma unroll
        for (int j = 0; j < kFieldsPerPass; ++j) {
          const int k = k0 + j;
          const int *src = k == 0 ? s.pc
                           : k <= ND ? reinterpret_cast<const int *>(s.off) + (int64_t)(k - 1) * s.cap
                                     : reinterpret_cast<const int *>(s.vel) + (int64_t)(k - ND - 1) * s.cap;
          v[j] = k < NF ? src[base + q] : 0;
        }
#pragma unroll
        for (int j = 0; j < kFieldsPerPass; ++j) s_v[j][q] = v[j];
      }
      __syncthreads();
      // ... and written in rank order, i.e. in runs of caller indices
      TileOrder<ND> w(tid, B, len, L, tile_cells);
      for (int r = tid; r < len; r += B, w.next()) {
        const int q = w.pos();
        const int64_t o = s_o[q];
#pragma unroll
        for (int j = 0; j < kFieldsPerPass; ++j) {
          const int k = k0 + j, v = s_v[j][q];
          if (k >= NF) break;
          if (k == 0) {
            int idx[3];
            unpack_cell<ND>(sd.tg, v, idx);
            cp.cell[o] = encode_cell<ND>(sd.g, idx);
          } else if (k <= ND) {
            reinterpret_cast<int *>(cp.off)[(int64_t)(k - 1) * cp.n + o] = v;
          } else {
            reinterpret_cast<int *>(cp.vel)[(int64_t)(k - ND - 1) * cp.n + o] = v;
          }
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// The fused step kernel
// ---------------------------------------------------------------------------
// Wave-aggregated append of the active lanes' values to a global list.
__device__ __forceinline__ void wave_append(int *list, int *count, int value, bool active) {
  const int lane = threadIdx.x & 63;
  unsigned long long m = __ballot(active);
  if (!m) return;
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(count, __popcll(m));
  base = __shfl(base, leader, 64);
  if (active) list[base + __popcll(m & ((1ull << lane) - 1ull))] = value;
}

// Window coordinates of a cell for the item loop: an interior window never
// touches the periodic seam, so a plain difference is exact there.
template <int ND, bool INTERIOR>
__device__ __forceinline__ bool item_window(const Geo &g, const Window &w, const int idx[3], int lo, int hi_off,
                                            int l[3], uint32_t edges) {
  if (!INTERIOR) return in_window<ND>(g, w, idx, lo, hi_off, l, edges);
  bool ok = true;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    l[d] = idx[d] - w.o[d];
    ok = ok && l[d] >= lo && l[d] <= w.wn[d] - hi_off;
  }
  return ok;
}

// The particles of one item whose cells lie in the tile window; the others
// (drifters) are appended to dlist, the item's own region of the drifter list
// (as long as the item: it cannot overflow), counted in ndrift (LDS).  Loads
// for the next round are issued before the current round is computed.
template <int ND, bool DIAG, bool INTERIOR, bool OUT, bool GEN>
__device__ __forceinline__ void run_item(const Geo &g, const Pot &P, const DiagC &dc, const TileGeo &tg,
                                         const StoreView &sv, const Item &it, const Window &w, const float *dens,
                                         const float *Gs, unsigned long long *acc,
                                         unsigned long long *__restrict__ Nnext, int *__restrict__ dlist,
                                         int *ndrift, uint32_t &e_all, double acc6[6], uint32_t edges) {
  PState cur, nxt;
  int p = it.start + (int)threadIdx.x;
  const int last = it.end - 1;
  load_state_any<ND, DIAG>(sv, min(p, last), cur);
  for (int base = it.start; base < it.end; base += blockDim.x) {
    const int pn = p + (int)blockDim.x;
    load_state_any<ND, DIAG>(sv, min(pn, last), nxt);
    const bool live = p < it.end;
    int idx[3], l[3];
    unpack_cell<ND>(tg, cur.pc, idx);
    const bool inside = live && item_window<ND, INTERIOR>(g, w, idx, 1, 3, l, edges);
    wave_append(dlist, ndrift, p, live && !inside);
    if (inside) {
      float cr[8];
      const int nb = win_node<ND>(w, l[0], l[1], l[2]);
#pragma unroll
      for (int k = 0; k < (1 << ND); ++k) cr[k] = dens[nb + node_corner<ND>(w, k)];
      const float nh = interp<ND>(cr, cur.f);
      int c0[3] = {0, 0, 0};
      float t[3] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int e = 0; e < ND; ++e) centre_stencil(l[e], cur.f[e], c0[e], t[e]);
      float Gp[3] = {0.f, 0.f, 0.f};
      float vv[3][8];
      const int cb = win_centre<ND>(w, c0[0], c0[1], c0[2]);
#pragma unroll
      for (int k = 0; k < (1 << ND); ++k) {
        const int m = cb + centre_corner<ND>(w, k);
        // component planes: the x-neighbour centres m, m + 1 are adjacent words
        // (one two-address LDS read per component and corner pair)
#pragma unroll
        for (int d = 0; d < ND; ++d) vv[d][k] = Gs[d * w.nC + m];
      }
#pragma unroll
      for (int d = 0; d < ND; ++d) Gp[d] = interp<ND>(vv[d], t);
      uint32_t tq[8];
      advance_particle<ND, DIAG, INTERIOR, OUT, GEN>(g, P, dc, tg, sv, p, cur.pc, idx, cur.f, cur.v, cur.W, nh, Gp, tq,
                                                     e_all, acc6, edges);
      // a sub-cell move keeps the new cell inside the deposit window
      if (item_window<ND, INTERIOR>(g, w, idx, 0, 2, l, edges)) {
        const int db = win_node<ND>(w, l[0], l[1], l[2]);
#pragma unroll
        for (int k = 0; k < (1 << ND); ++k) atomicAdd(&acc[db + node_corner<ND>(w, k)], (unsigned long long)tq[k]);
      } else {
        deposit_global<ND>(g, Nnext, idx, tq);
      }
    }
    cur = nxt;
    p = pn;
  }
}

// A drifter (a particle outside its tile window since the last binning): the
// same cycle through the global node sums of its slab, folded like the
// window, so its result is the same bits as inside a window.
template <int ND, bool DIAG, bool OUT, bool GEN>
__device__ __forceinline__ void advance_drifter(const Geo &g, const Pot &P, const DiagC &dc, const TileGeo &tg,
                                                const StoreView &sv, int p, const long long *__restrict__ N,
                                                unsigned long long *__restrict__ Nn, uint32_t &e_all,
                                                double acc6[6]) {
  PState q;
  load_state<ND, DIAG>(sv, p, true, q);
  int idx[3];
  unpack_cell<ND>(tg, q.pc, idx);
  float nh, Gp[3];
  gather_nodes_global<ND>(g, N, idx, q.f, nh, Gp);
  uint32_t tq[8];
  advance_particle<ND, DIAG, false, OUT, GEN>(g, P, dc, tg, sv, p, q.pc, idx, q.f, q.v, q.W, nh, Gp, tq, e_all,
                                              acc6);
  deposit_global<ND>(g, Nn, idx, tq);
}

// Persistent: a fixed grid works through the step's work items (chunks of
// one tile of one slab) until they are done.  Each item ends with its own
// drifters (a few per item: the context re-bins once they exceed a small
// fraction of the particles), so one launch is the whole step.  Every block
// also clears its share of the node buffer two steps ahead.
// The occupancy bound (waves per SIMD: 7 in 2D; 4 in 3D, where the window's
// LDS allows 3-5 blocks per CU and more waves would spill registers in the
// item loop) is what the item loop needs alone; it keeps the rarely taken
// drifter path from raising the register count of the whole kernel.
template <int ND, bool DIAG, bool OUT, bool GEN>
__global__ void __launch_bounds__(256, ND == 2 ? 7 : 4) k_step_tiled(Pot P, DiagC dc, Batch b, Store s, Store o,
                                                    const Item *__restrict__ items,
                                                    const int *__restrict__ num_items,
                                                    const long long *__restrict__ Ncur,
                                                    unsigned long long *__restrict__ Nnext,
                                                    long long *__restrict__ Nclear, Drift dr,
                                                    double *__restrict__ partial, uint32_t *__restrict__ err) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_item[2], s_ndrift;
  clear_share(Nclear, b.nnodes);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *dr.count_next = 0;  // the next step's drifter count and work counter
    *dr.work_next = 0;
  }
  const int nit = *num_items;
  const StoreView sv = view_of<OUT>(s, o);
  uint32_t e_all = 0;
  // The first item of block k is item k (no atomic at the start of the
  // launch, when every block would ask at once); the following ones come
  // from the counter (offset by the grid), each fetched before the flush of
  // the item before it.  The fetched index alternates between two LDS slots
  // (a slot is rewritten only after every thread has passed the barrier that
  // follows its read).
  int pick = blockIdx.x;
  for (int round = 0;; ++round) {
    if (pick >= nit) break;
    if (threadIdx.x == 0) s_ndrift = 0;  // visible after the window staging's barriers
    const Item it = items[pick];
    const SlabDesc &sd = b.slabs[it.slab];
    const Geo g = sd.g;
    const TileGeo tg = sd.tg;
    const Window w = make_window<ND>(tg, it.tile - sd.tile_off);
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(smem);
    float *dens = reinterpret_cast<float *>(acc + w.nW);
    float *Gs = dens + w.nW;
    unsigned long long *Nn = Nnext + sd.node_off;
    stage_window<ND>(g, w, Ncur + sd.node_off, dens, Gs, acc);  // ends with a barrier
    // interior windows: no wall and no periodic seam within reach of any
    // particle the item loop handles; otherwise only the axes in edges
    // need the wall and wrap code
    const uint32_t edges = __builtin_amdgcn_readfirstlane(window_edges<ND>(g, w));
    double acc6[6] = {0, 0, 0, 0, 0, 0};
    int *dlist = dr.list + it.start;  // slots [start, end) of the item
    if (!edges)
      run_item<ND, DIAG, true, OUT, GEN>(g, P, dc, tg, sv, it, w, dens, Gs, acc, Nn, dlist, &s_ndrift, e_all, acc6,
                                         edges);
    else
      run_item<ND, DIAG, false, OUT, GEN>(g, P, dc, tg, sv, it, w, dens, Gs, acc, Nn, dlist, &s_ndrift, e_all, acc6,
                                          edges);
    __syncthreads();  // the window's sums and the item's drifter list are complete
    // the next index, fetched before this item's flush and drifters, which
    // overlap the atomic's latency
    int next = 0;
    if (threadIdx.x == 0) next = (int)gridDim.x + atomicAdd(dr.work, 1);
    flush_window<ND>(g, w, acc, Nn);
    const int ndr = __builtin_amdgcn_readfirstlane(s_ndrift);
    if (ndr > 0) {
      if (threadIdx.x == 0) atomicAdd(dr.count, ndr);  // the step's total, for the re-binning policy
      for (int k = threadIdx.x; k < ndr; k += blockDim.x)
        advance_drifter<ND, DIAG, OUT, GEN>(g, P, dc, tg, sv, dlist[k], Ncur + sd.node_off, Nn, e_all, acc6);
    }
    if (DIAG) block_reduce_store<6>(acc6, partial + (int64_t)pick * 8);
    if (threadIdx.x == 0) s_item[round & 1] = next;
    __syncthreads();  // LDS is reused by the next item; the next index is visible
    pick = __builtin_amdgcn_readfirstlane(s_item[round & 1]);
  }
  if (e_all) atomicOr(err, e_all);
}

// Node sums of the current positions (the first step's input), same tiling.
template <int ND>
__global__ void __launch_bounds__(256) k_deposit_tiled(Batch b, Store s, const Item *__restrict__ items,
                                                       const int *__restrict__ num_items,
                                                       unsigned long long *__restrict__ N) {
  extern __shared__ __align__(16) unsigned char smem[];
  if ((int)blockIdx.x >= *num_items) return;
  const Item it = items[blockIdx.x];
  const SlabDesc &sd = b.slabs[it.slab];
  const Geo g = sd.g;
  const TileGeo tg = sd.tg;
  const Window w = make_window<ND>(tg, it.tile - sd.tile_off);
  unsigned long long *Ns = N + sd.node_off;
  unsigned long long *acc = reinterpret_cast<unsigned long long *>(smem);
  for (int k = threadIdx.x; k < w.nW; k += blockDim.x) acc[k] = 0ull;
  __syncthreads();
  const int64_t cap = s.cap;
  for (int p = it.start + threadIdx.x; p < it.end; p += blockDim.x) {
    float f[3] = {s.off[p], s.off[cap + p], ND == 3 ? s.off[2 * cap + p] : 0.0f};
    int idx[3], l[3];
    unpack_cell<ND>(tg, s.pc[p], idx);
    uint32_t tq[8];
    deposit_shares<ND>((uint32_t)s.wq[p], f, tq);
    if (in_window<ND>(g, w, idx, 0, 2, l)) {
#pragma unroll
      for (int k = 0; k < (1 << ND); ++k)
        if (tq[k])
          atomicAdd(&acc[win_node<ND>(w, l[0] + (k & 1), l[1] + ((k >> 1) & 1), ND == 3 ? l[2] + ((k >> 2) & 1) : 0)],
                    (unsigned long long)tq[k]);
    } else {
      deposit_global<ND>(g, Ns, idx, tq);
    }
  }
  __syncthreads();
  flush_window<ND>(g, w, acc, Ns);
}

// One slab's diagnostics: its items' block partials (a contiguous item range;
// each item's drifters are in its partial) and its node energy partials, in
// two launches: kRedBlocks blocks each sum a fixed share of both lists into
// red, then one block sums red in a fixed order (deterministic).
constexpr int kRedBlocks = kDiagRedDoubles / 8;

__global__ void __launch_bounds__(256) k_reduce_diag_part(const double *__restrict__ part_p,
                                                          const int *__restrict__ item_start, int tile_lo,
                                                          int tile_hi, const double *__restrict__ part_g, int nblk_g,
                                                          double *__restrict__ red) {
  const int lo = item_start[tile_lo], hi = item_start[tile_hi];
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  const int stride = gridDim.x * blockDim.x;
  for (int b = lo + blockIdx.x * blockDim.x + threadIdx.x; b < hi; b += stride)
#pragma unroll
    for (int i = 0; i < 6; ++i) acc[i] += part_p[(int64_t)b * 8 + i];
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nblk_g; b += stride) acc[6] += part_g[(int64_t)b * 8];
  block_reduce_store<7>(acc, red + (int64_t)blockIdx.x * 8);
}

__global__ void __launch_bounds__(256) k_reduce_diag_slab(const double *__restrict__ red, pic_diag_t *__restrict__ out,
                                                          int64_t step) {
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < kRedBlocks; b += blockDim.x)
#pragma unroll
    for (int i = 0; i < 7; ++i) acc[i] += red[(int64_t)b * 8 + i];
  __shared__ double res[8];
  block_reduce_store<7>(acc, res);
  __syncthreads();
  if (threadIdx.x == 0) {
    out->ke = res[0];
    out->px = res[1];
    out->py = res[2];
    out->pz = res[3];
    out->wsum = res[4];
    out->bond = res[5];
    out->pe = res[6];
    out->step = step;
  }
}

// ---------------------------------------------------------------------------
// Reverse mode in the store (recorded trajectories).  One block per item.
// The item's window (same origin and folding as the forward window) is
// staged in LDS twice: the node densities of step n, and the next step's node
// cotangent times the node's density factor.  Per particle, the 3^ND window
// nodes around its centre stencil give the 2^ND centre gradients through the
// forward's own centre_gradient (same bits as the forward), and the
// cotangents of the gathered density and gradient go back to those 3^ND
// nodes (the transpose of that stencil) in registers, then into an LDS node
// accumulator; the accumulator is flushed into the global node cotangent with
// the window's fold (periodic wrap, mirror across reflecting walls): the
// exact transpose of the forward's window staging.  Particles outside their
// window take the global path (global density / gradient grids, scatters to
// the global node and centre cotangents).
// ---------------------------------------------------------------------------
template <int ND>
__device__ __forceinline__ void load_adjoint_state(const StoreView &sv, const float *__restrict__ lx,
                                                   const float *__restrict__ lv, int cap, int p, bool on, PState &st,
                                                   float a[3], float c[3]) {
  load_state<ND, true>(sv, p, on, st);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    a[d] = (on && d < ND) ? lx[d * cap + p] : 0.0f;
    c[d] = on ? lv[d * cap + p] : 0.0f;
  }
}

// A particle's state and cotangents, loaded from a slot inside the store
// (lanes past the item's end read its last slot and ignore it).
struct AdjLoad {
  PState q;
  float ln[3], lv[3];
  int pcn;      // KNOWN: the next state's cell word and offsets
  float fn[3];
};
template <int ND, bool KNOWN = false>
__device__ __forceinline__ void load_adjoint_any(const StoreView &sv, const float *__restrict__ lx,
                                                 const float *__restrict__ lv, int cap, int p, AdjLoad &a,
                                                 const int *__restrict__ pc_next = nullptr,
                                                 const float *__restrict__ off_next = nullptr) {
  load_state_any<ND, true>(sv, p, a.q);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    a.ln[d] = d < ND ? lx[d * cap + p] : 0.0f;
    a.lv[d] = lv[d * cap + p];
  }
  if (KNOWN) {
    a.pcn = pc_next[p];
#pragma unroll
    for (int d = 0; d < 3; ++d) a.fn[d] = d < ND ? off_next[d * cap + p] : 0.0f;
  }
}

// Node cotangents accumulate in LDS as int64 fixed point: float atomic adds
// on LDS are more than an order of magnitude slower than integer ones on this
// chip.  The scale is a power of two set from the largest single contribution
// of the previous reverse step (amax_prev, float bits): values up to 128
// times that fit with 2^12 of headroom for the sum of a node's contributions
// and a resolution of 2^-44 of it; a larger value (a sudden jump) takes a
// global float atomic instead.  MAXONLY: only measure the largest
// contribution (seeds the scale of the first reverse step).
__device__ __forceinline__ int adj_scale_exp(uint32_t amax_bits) {
  const float m = __uint_as_float(amax_bits);
  if (!(m > 0.0f)) return 100;  // nothing seen: every nonzero value takes the float path
  int e;
  (void)frexpf(m, &e);  // m < 2^e
  return min(max(44 - e, -100), 100);
}

// v rounded to the nearest int64 (ties to even) for |v| < 2^51, exactly: the
// FP64 sum with 1.5 * 2^52 holds the integer in its low mantissa bits (three
// instructions where the generic float-to-int64 conversion takes eleven).
__device__ __forceinline__ long long fix64(float v) {
  return __double_as_longlong((double)v + 6755399441055744.0) - 0x4338000000000000ll;
}

// Node values at frame coordinates: an LDS window (frame = window), or the
// global node arrays (frame = global node coordinates, folded like the
// window: periodic wrap, mirror across reflecting walls).
template <int ND>
struct WinRead {
  const float *a;
  int s1, s2;  // window strides
  __device__ __forceinline__ float operator()(int x, int y, int z) const {
    return a[x + s1 * y + (ND == 3 ? s2 * z : 0)];
  }
};

template <int ND>
__device__ __forceinline__ int folded_node(const Geo &g, int x, int y, int z) {
  return node_index<ND>(g, fold_node(g, 0, x), fold_node(g, 1, y), ND == 3 ? fold_node(g, 2, z) : 0);
}

// Centre gradients of the 2^ND nearest centres: read from the window's planes
// (kPlanes), or built by the reverse step from its 3^ND node block.
template <int ND>
struct WinCentres {
  static constexpr bool kPlanes = true;
  const float *G;
  int nC, cy, cz;
  __device__ __forceinline__ float operator()(int d, int m0, int m1, int m2) const {
    return G[d * nC + m0 + cy * m1 + (ND == 3 ? cz * m2 : 0)];
  }
};
struct NoCentres {
  static constexpr bool kPlanes = false;
  __device__ __forceinline__ float operator()(int, int, int, int) const { return 0.0f; }
};

template <int ND>
struct GlobalDens {  // node density of step n from the node sums (the window's bits)
  const long long *N;
  const Geo *g;
  __device__ __forceinline__ float operator()(int x, int y, int z) const {
    const int a = fold_node(*g, 0, x), b = fold_node(*g, 1, y), c = ND == 3 ? fold_node(*g, 2, z) : 0;
    return node_density(*g, N[node_index<ND>(*g, a, b, c)], a, b, c);
  }
};

template <int ND>
struct GlobalNext {  // kfac * nbar of step n+1 at a (real) node
  const float *nb;
  const Geo *g;
  __device__ __forceinline__ float operator()(int x, int y, int z) const {
    const int a = fold_node(*g, 0, x), b = fold_node(*g, 1, y), c = ND == 3 ? fold_node(*g, 2, z) : 0;
    return node_density(*g, 1ll, a, b, c) * nb[node_index<ND>(*g, a, b, c)];
  }
};

// The reverse step of one particle from a 3^ND block of node densities (the
// nodes around its 2^ND nearest cell centres).  l: frame coordinates of the
// own cell's lower node.  The 2^ND centre gradients come from the block
// through the forward's own centre_gradient (same bits as the forward's
// window), the forward step is recomputed, the deposit term of step n+1 is
// read at the new position through `next` when has_next, and the cotangents
// of the gathered density and gradient go back to the block: a3 (node
// cotangents of the block, first node at frame coordinates B).  GEN: the
// potential chosen at run time (Lennard-Jones or Morse).
template <int ND, bool GEN, class Dens, class Next, class Cent = NoCentres>
__device__ __forceinline__ uint32_t adjoint_on_block(const Geo &g, const Pot &P, const int idx[3], const int l[3],
                                                     const PState &q, const Dens &dens, bool has_next,
                                                     const Next &next, float ln[3], float lvv[3], float lf[3],
                                                     float th[5], int B[3], float t[3], float &an, float aG[3],
                                                     uint32_t edges = 7u, const Cent &cent = Cent{},
                                                     const PushRecord *known = nullptr) {
  constexpr int K3 = ND == 2 ? 9 : 27;
  float cr[8];
#pragma unroll
  for (int k = 0; k < (1 << ND); ++k)
    cr[k] = dens(l[0] + (k & 1), l[1] + ((k >> 1) & 1), ND == 3 ? l[2] + ((k >> 2) & 1) : 0);
  const float nh = interp<ND>(cr, q.f);
  float dn[3];  // d nh / d offset, taken now so that cr dies here
  interp_grad<ND>(cr, q.f, dn);
  t[0] = t[1] = t[2] = 0.0f;
  B[2] = 0;
#pragma unroll
  for (int e = 0; e < ND; ++e) centre_stencil(l[e], q.f[e], B[e], t[e]);
  float Gp[3] = {0.f, 0.f, 0.f}, dG[3][3];
  {
    float vv[3][8];
    if constexpr (Cent::kPlanes) {
#pragma unroll
      for (int k = 0; k < (1 << ND); ++k)
#pragma unroll
        for (int d = 0; d < ND; ++d)
          vv[d][k] = cent(d, B[0] + (k & 1), B[1] + ((k >> 1) & 1), ND == 3 ? B[2] + ((k >> 2) & 1) : 0);
    } else {
      float d3[K3];
#pragma unroll
      for (int a = 0; a < K3; ++a) d3[a] = dens(B[0] + a % 3, B[1] + (a / 3) % 3, ND == 3 ? B[2] + a / 9 : 0);
#pragma unroll
      for (int k = 0; k < (1 << ND); ++k) {
        float c[8], Gc[3];
#pragma unroll
        for (int j = 0; j < (1 << ND); ++j)
          c[j] = d3[b3<ND>((k & 1) + (j & 1), ((k >> 1) & 1) + ((j >> 1) & 1),
                           ND == 3 ? ((k >> 2) & 1) + ((j >> 2) & 1) : 0)];
        centre_gradient<ND>(g, c, Gc);
#pragma unroll
        for (int d = 0; d < ND; ++d) vv[d][k] = Gc[d];
      }
    }
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      Gp[d] = interp<ND>(vv[d], t);
      interp_grad<ND>(vv[d], t, dG[d]);  // d Gp / d offset; vv dies here
    }
  }
  PushRecord r;
  uint32_t e_push = 0;
  if (known) r = *known;  // the forward's own result, read from the next state
  else e_push = recompute_push<ND, GEN>(g, P, idx, q.f, q.v, nh, Gp, r, edges);
  if (has_next) {
    int l2[3] = {0, 0, 0};
#pragma unroll
    for (int e = 0; e < ND; ++e) {
      int dlt = r.idx2[e] - idx[e];
      dlt = dlt > 1 ? dlt - g.n[e] : (dlt < -1 ? dlt + g.n[e] : dlt);  // across the periodic seam
      l2[e] = l[e] + dlt;
    }
    float c[8], dd[3];
#pragma unroll
    for (int k = 0; k < (1 << ND); ++k)
      c[k] = next(l2[0] + (k & 1), l2[1] + ((k >> 1) & 1), ND == 3 ? l2[2] + ((k >> 2) & 1) : 0);
    interp_grad<ND>(c, r.f2, dd);
    const float wgt = (float)q.W;
#pragma unroll
    for (int e = 0; e < ND; ++e) ln[e] = __builtin_fmaf(wgt, dd[e], ln[e]);
  }
  float mu[3] = {0.f, 0.f, 0.f};
  reverse_drift_kick<ND>(g, P, r, ln, lvv, lf, mu);
  pair_force_vjp<ND, GEN>(P, nh, Gp, mu, an, aG, th);
#pragma unroll
  for (int e = 0; e < ND; ++e) lf[e] = __builtin_fmaf(an, dn[e], lf[e]);
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int e = 0; e < ND; ++e) lf[e] = __builtin_fmaf(aG[d], dG[d][e], lf[e]);
  return e_push;
}

// The cotangents of a particle's gathered density (an) and gradient (aG) on
// its 3^ND node block: the transpose of the centre-gradient stencil
// (weights t), then the own cell's corners (offsets f, own lower node l).
// Both maps are separable over the axes: along axis e a node at block offset
// a enters the gradient component e with the difference weights
// D_e = (-(1 - t_e), (1 - t_e) - t_e, t_e) and the other components with the
// sum weights S_e = (1 - t_e, 1, t_e) (the centre-gradient stencil, then the
// interpolation between the two nearest centres), and the density with the
// own cell's linear weights U_e.
template <int ND>
__device__ __forceinline__ void block_cotangents(const Geo &g, const int l[3], const int B[3], const float f[3],
                                                 const float t[3], float an, const float aG[3],
                                                 float a3[ND == 2 ? 9 : 27]) {
  float D[3][3], S[3][3], U[3][3];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const float te = e < ND ? t[e] : 0.0f, ue = 1.0f - te;
    D[e][0] = -ue;
    D[e][1] = ue - te;
    D[e][2] = te;
    S[e][0] = ue;
    S[e][1] = 1.0f;
    S[e][2] = te;
    const int o = e < ND ? l[e] - B[e] : 0;  // own cell's lower node in the block: 0 or 1
    const float fe = e < ND ? f[e] : 0.0f;
    U[e][0] = o == 0 ? 1.0f - fe : 0.0f;
    U[e][1] = o == 0 ? fe : 1.0f - fe;
    U[e][2] = o == 0 ? 0.0f : fe;
  }
  const float cx = aG[0] * g.gam[0], cy = aG[1] * g.gam[1], cz = ND == 3 ? aG[2] * g.gam[2] : 0.0f;
#pragma unroll
  for (int bc = 0; bc < (ND == 2 ? 3 : 9); ++bc) {
    const int b = bc % 3, c = bc / 3;
    const float sz = ND == 3 ? S[2][c] : 1.0f, uz = ND == 3 ? U[2][c] : 1.0f;
    const float px = cx * (S[1][b] * sz);
    float pyz = cy * (D[1][b] * sz);
    if (ND == 3) pyz = __builtin_fmaf(cz, S[1][b] * D[2][c], pyz);
    const float pn = an * (U[1][b] * uz);
#pragma unroll
    for (int a = 0; a < 3; ++a)
      a3[a + 3 * bc] = __builtin_fmaf(px, D[0][a], __builtin_fmaf(pyz, S[0][a], pn * U[0][a]));
  }
}

// Adds NF per-thread values, summed over the block, into out[0..NF).
template <int NF>
__device__ __forceinline__ void block_reduce_add(double v[NF], double *__restrict__ out) {
  __shared__ double red[NF][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int i = 0; i < NF; ++i)
    for (int o = 32; o > 0; o >>= 1) v[i] += __shfl_down(v[i], o, 64);
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NF; ++i) red[i][wave] = v[i];
  __syncthreads();
  if (threadIdx.x < NF) {
    double s = 0.0;
    for (int w = 0; w < nwaves; ++w) s += red[threadIdx.x][w];
    out[threadIdx.x] += s;
  }
}

// PLANES: the window also holds the centre-gradient planes (staged once per
// item, as in the forward step) and each particle reads its 2^ND centres'
// gradients from them instead of building them from its 3^ND node block.
// nbar_clear (nclear floats, or null): the next reverse step's node
// cotangents, zeroed here a share per block (nothing of this step reads them).
// pc_next, off_next: the state after the step in the same binning, or null.
// Given, the items whose window reaches no reflecting wall (where nothing can
// reflect) read each particle's push from it instead of recomputing it: the
// new cell and offset are the forward's own bits.  The two kinds of item run
// separate copies of the particle loop, so that neither carries the other's
// registers.
template <int ND, bool MAXONLY, bool GEN, bool PLANES>
__global__ void __launch_bounds__(256, 4) k_adjoint_tiled(Pot P, Batch b, Store s, const Item *__restrict__ items,
                                                       const int *__restrict__ num_items,
                                                       const long long *__restrict__ Ncur,
                                                       const float *__restrict__ nbar_next, float *__restrict__ lx,
                                                       float *__restrict__ lv, float *__restrict__ nbar,
                                                       int *__restrict__ dlist, int *__restrict__ dcount,
                                                       const uint32_t *__restrict__ amax_prev,
                                                       uint32_t *__restrict__ amax_cur,
                                                       double *__restrict__ partial, uint32_t *__restrict__ err,
                                                       const int *__restrict__ pc_next,
                                                       const float *__restrict__ off_next,
                                                       float *__restrict__ nbar_clear, int64_t nclear) {
  constexpr int K3 = ND == 2 ? 9 : 27;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t s_amax;
  if (nbar_clear) {
    const int64_t share = (nclear + gridDim.x - 1) / gridDim.x, lo = (int64_t)blockIdx.x * share;
    const int64_t hi = min(nclear, lo + share);
    for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) nbar_clear[k] = 0.0f;
  }
  if ((int)blockIdx.x >= *num_items) return;
  const int sexp = MAXONLY ? 0 : adj_scale_exp(*amax_prev);
  const float to_fix = ldexpf(1.0f, sexp);    // exact power of two (sexp within float range)
  const float lim = ldexpf(1.0f, 51 - sexp);  // larger values: global float atomics
  // the block cotangents are built from inputs scaled by to_fix, which scales
  // every contribution exactly (a power of two): fixed point without a
  // multiply per node; lim_s = lim * to_fix
  constexpr float lim_s = 2251799813685248.0f;  // 2^51
  float vmax = 0.0f;    // largest contribution, scaled by to_fix (fixed-point particles)
  float vmax_u = 0.0f;  // largest contribution, unscaled (the other particles)
  const Item it = items[blockIdx.x];
  const SlabDesc &sd = b.slabs[it.slab];
  const Geo g = sd.g;
  const TileGeo tg = sd.tg;
  const Window w = make_window<ND>(tg, it.tile - sd.tile_off);
  // axes along which the window reaches a wall or the periodic seam (uniform)
  const uint32_t edges = __builtin_amdgcn_readfirstlane(window_edges<ND>(g, w));
  uint32_t walls = 0;
#pragma unroll
  for (int d = 0; d < ND; ++d) walls |= g.bc[d] ? (1u << d) : 0u;
  const bool known = !MAXONLY && pc_next != nullptr && (edges & walls) == 0u;
  unsigned long long *acc = reinterpret_cast<unsigned long long *>(smem);  // [nW] node cotangent, fixed point
  float *dw = reinterpret_cast<float *>(acc + w.nW);  // [nW] node densities of step n
  float *nx = dw + w.nW;                              // [nW] kfac * nbar of step n+1
  if (threadIdx.x == 0) s_amax = 0u;
  const long long *N = Ncur + sd.node_off;
  const float *nbn = nbar_next ? nbar_next + sd.node_off : nullptr;
  bool nofold, nowall;
  window_flags<ND>(g, w, nofold, nowall);
  {
    Walk<ND> wk((int)threadIdx.x, (int)blockDim.x, w.wn[0], w.wn[1]);
    for (int k = threadIdx.x; k < w.nW; k += blockDim.x, wk.next()) {
      int x[3];
      window_node<ND>(g, w, wk.a, nofold, x);
      const int node = node_index<ND>(g, x[0], x[1], x[2]);
      const float kf = nowall ? g.kappa : node_density(g, 1ll, x[0], x[1], x[2]);
      dw[k] = nowall ? wsum_float(N[node]) * g.kappa : node_density(g, N[node], x[0], x[1], x[2]);
      nx[k] = nbn ? kf * nbn[node] : 0.0f;
      acc[k] = 0ull;
    }
  }
  __syncthreads();
  float *Gs = nx + w.nW;  // [ND][nC] when PLANES
  if (PLANES) stage_gradients<ND>(g, w, dw, Gs);
  const WinRead<ND> dens{dw, w.wn[0], w.wn[0] * w.wn[1]};
  const WinRead<ND> next{nx, w.wn[0], w.wn[0] * w.wn[1]};
  const WinCentres<ND> cent{Gs, w.nC, w.cy, w.cz};
  const int cap = (int)s.cap;
  const StoreView sv = view_of(s, s);
  uint32_t e_all = 0;
  float thf[5] = {0.f, 0.f, 0.f, 0.f, 0.f};  // this thread's parameter terms (chunk / 256 particles at most)
  // loads for the next round are issued before the current round is computed
  const int last = it.end - 1;
  auto particle_loop = [&](auto known_tag) {
  constexpr bool KNOWN = decltype(known_tag)::value;
  AdjLoad cur, nxt;
  load_adjoint_any<ND, KNOWN>(sv, lx, lv, cap, min(it.start + (int)threadIdx.x, last), cur, pc_next, off_next);
  for (int base = it.start; base < it.end; base += blockDim.x) {
    const int p = base + (int)threadIdx.x;
    const bool live = p < it.end;
    load_adjoint_any<ND, KNOWN>(sv, lx, lv, cap, min(p + (int)blockDim.x, last), nxt, pc_next, off_next);
    const PState q = cur.q;
    float ln[3] = {cur.ln[0], cur.ln[1], cur.ln[2]}, lvv[3] = {cur.lv[0], cur.lv[1], cur.lv[2]};
    const int pcn = cur.pcn;
    const float fn[3] = {cur.fn[0], cur.fn[1], cur.fn[2]};
    cur = nxt;
    int idx[3], l[3];
    unpack_cell<ND>(tg, q.pc, idx);
    const bool inside = live && in_window<ND>(g, w, idx, 1, 3, l, edges);
    if (!MAXONLY) wave_append(dlist, dcount, p, live && !inside);  // the global path, in a kernel of its own
    if (inside) {
      float lf[3] = {0.f, 0.f, 0.f}, th[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, t[3], an, aG[3];
      int B[3];
      // KNOWN: the new cell and offset are the forward's own bits, and
      // nothing reflects
      PushRecord kr;
      if (KNOWN) {
        unpack_cell<ND>(tg, pcn, kr.idx2);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          kr.f2[d] = fn[d];
          kr.sgn[d] = 1.0f;
        }
      }
      if (PLANES)
        e_all |= adjoint_on_block<ND, GEN>(g, P, idx, l, q, dens, nbn != nullptr, next, ln, lvv, lf, th, B, t, an, aG,
                                           edges, cent, KNOWN ? &kr : nullptr);
      else
        e_all |= adjoint_on_block<ND, GEN>(g, P, idx, l, q, dens, nbn != nullptr, next, ln, lvv, lf, th, B, t, an, aG,
                                           edges, NoCentres{}, KNOWN ? &kr : nullptr);
      if (!MAXONLY) {  // the particle's cotangents and parameter terms, before its node block
#pragma unroll
        for (int d = 0; d < ND; ++d) lx[d * cap + p] = lf[d];
#pragma unroll
        for (int d = 0; d < 3; ++d) lv[d * cap + p] = lvv[d];
#pragma unroll
        for (int i = 0; i < 5; ++i) thf[i] += th[i];
      }
      float a3[K3];
      {
        const float aGs[3] = {aG[0] * to_fix, aG[1] * to_fix, aG[2] * to_fix};
        block_cotangents<ND>(g, l, B, q.f, t, an * to_fix, aGs, a3);
      }
      float pmax = 0.0f;  // this particle's largest contribution (scaled; inf when the scaling overflowed)
#pragma unroll
      for (int a = 0; a < K3; ++a) pmax = fmaxf(pmax, fabsf(a3[a]));
      if (MAXONLY) {
        vmax = fmaxf(vmax, pmax);  // to_fix = 1
      } else if (pmax < lim_s) {  // the common case: every contribution in fixed point, no branch per node
        vmax = fmaxf(vmax, pmax);
        const int nb = win_node<ND>(w, B[0], B[1], B[2]);
#pragma unroll
        for (int a = 0; a < K3; ++a)
          atomicAdd(&acc[nb + win_node<ND>(w, a % 3, (a / 3) % 3, ND == 3 ? a / 9 : 0)],
                    (unsigned long long)fix64(a3[a]));
      } else {
        // the contributions again, unscaled: some exceed the fixed-point range
        block_cotangents<ND>(g, l, B, q.f, t, an, aG, a3);
#pragma unroll
        for (int a = 0; a < K3; ++a) {
          vmax_u = fmaxf(vmax_u, fabsf(a3[a]));
          const int ax = B[0] + a % 3, ay = B[1] + (a / 3) % 3, az = ND == 3 ? B[2] + a / 9 : 0;
          if (fabsf(a3[a]) < lim) {
            atomicAdd(&acc[win_node<ND>(w, ax, ay, az)], (unsigned long long)fix64(a3[a] * to_fix));
          } else {
            atomicAdd(&nbar[sd.node_off + folded_node<ND>(g, w.o[0] + ax, w.o[1] + ay, w.o[2] + az)], a3[a]);
          }
        }
      }
    }
  }
  };
  if (known) particle_loop(std::true_type{});
  else particle_loop(std::false_type{});
  // largest single contribution of this block (the next step's scale)
  vmax = fmaxf(vmax * ldexpf(1.0f, -sexp), vmax_u);
  for (int o = 32; o > 0; o >>= 1) vmax = fmaxf(vmax, __shfl_xor(vmax, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(&s_amax, __float_as_uint(vmax));
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(amax_cur, s_amax);
  if (MAXONLY) return;
  const double from_fix = ldexp(1.0, -sexp);
  Walk<ND> wk((int)threadIdx.x, (int)blockDim.x, w.wn[0], w.wn[1]);
  for (int k = threadIdx.x; k < w.nW; k += blockDim.x, wk.next()) {
    const long long iv = (long long)acc[k];
    if (iv == 0) continue;
    int x[3];
    window_node<ND>(g, w, wk.a, nofold, x);
    atomicAdd(&nbar[sd.node_off + node_index<ND>(g, x[0], x[1], x[2])], (float)((double)iv * from_fix));
  }
  if (e_all) atomicOr(err, e_all);
  double thd[5] = {thf[0], thf[1], thf[2], thf[3], thf[4]};
  block_reduce_add<5>(thd, partial + (int64_t)blockIdx.x * 8);  // accumulates over the sweep
}

// The reverse step of the particles outside their window: the same block
// computation on the node sums (densities folded like the window's), scatters
// as global float atomics; parameter terms into dacc[0..4].
template <int ND, bool GEN>
// dcount_clear, amax_clear (or null): the next reverse step's drifter count
// and largest-contribution slot, zeroed here (neither is read in this launch).
__global__ void __launch_bounds__(256) k_adjoint_drifters(Pot P, Batch b, Store s, const int *__restrict__ dlist,
                                                          const int *__restrict__ dcount,
                                                          const long long *__restrict__ Ncur,
                                                          const float *__restrict__ nbar_next,
                                                          float *__restrict__ lx, float *__restrict__ lv,
                                                          float *__restrict__ nbar, double *__restrict__ dacc,
                                                          uint32_t *__restrict__ err, int *__restrict__ dcount_clear,
                                                          uint32_t *__restrict__ amax_clear) {
  constexpr int K3 = ND == 2 ? 9 : 27;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (dcount_clear) *dcount_clear = 0;
    if (amax_clear) *amax_clear = 0u;
  }
  const int n = *dcount;
  const int cap = (int)s.cap;
  const StoreView sv = view_of(s, s);
  uint32_t e_all = 0;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int p = dlist[k];
    const SlabDesc &sd = b.slabs[find_slab(b.part_offs, b.nslab, p)];
    const Geo g = sd.g;
    PState q;
    float ln[3], lvv[3];
    load_adjoint_state<ND>(sv, lx, lv, cap, p, true, q, ln, lvv);
    int idx[3];
    unpack_cell<ND>(sd.tg, q.pc, idx);
    const GlobalDens<ND> dens{Ncur + sd.node_off, &g};
    const GlobalNext<ND> next{nbar_next ? nbar_next + sd.node_off : nullptr, &g};
    float lf[3] = {0.f, 0.f, 0.f}, th[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, t[3], an, aG[3], a3[K3];
    int B[3];
    e_all |= adjoint_on_block<ND, GEN>(g, P, idx, idx, q, dens, nbar_next != nullptr, next, ln, lvv, lf, th, B, t, an,
                                       aG);
    block_cotangents<ND>(g, idx, B, q.f, t, an, aG, a3);
#pragma unroll
    for (int a = 0; a < K3; ++a)
      if (a3[a] != 0.0f)
        atomicAdd(&nbar[sd.node_off + folded_node<ND>(g, B[0] + a % 3, B[1] + (a / 3) % 3, ND == 3 ? B[2] + a / 9 : 0)],
                  a3[a]);
#pragma unroll
    for (int d = 0; d < ND; ++d) lx[d * cap + p] = lf[d];
#pragma unroll
    for (int d = 0; d < 3; ++d) lv[d * cap + p] = lvv[d];
#pragma unroll
    for (int i = 0; i < 5; ++i) atomicAdd(&dacc[i], (double)th[i]);
  }
  if (e_all) atomicOr(err, e_all);
}

// lam_x += the deposit term at the store's positions (the last reverse step).
template <int ND>
__global__ void __launch_bounds__(256) k_deposit_vjp_store(Batch b, Store s, const float *__restrict__ nbar,
                                                           float *__restrict__ lx) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= b.nparts) return;
  const SlabDesc &sd = b.slabs[find_slab(b.part_offs, b.nslab, p)];
  const int cap = (int)s.cap;
  const StoreView sv = view_of(s, s);
  PState q;
  load_state<ND, false>(sv, p, true, q);
  int idx[3];
  unpack_cell<ND>(sd.tg, q.pc, idx);
  float lf[3] = {lx[p], lx[cap + p], ND == 3 ? lx[2 * cap + p] : 0.0f};
  deposit_term<ND>(sd.g, nbar + sd.node_off, idx, q.f, q.W, lf);
#pragma unroll
  for (int d = 0; d < ND; ++d) lx[d * cap + p] = lf[d];
}

// Cotangents between the caller's order and the store's: slot p of the store
// holds caller particle part_off + oidx[p] of its slab (k arrays of stride
// cap in the store, stride n in the caller's arrays).
__global__ void __launch_bounds__(256) k_to_store(Batch b, Store s, int k, const float *__restrict__ src, int64_t n,
                                                  float *__restrict__ dst) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= b.nparts) return;
  const int o = s.oidx[p];
  for (int d = 0; d < k; ++d) dst[(int64_t)d * s.cap + p] = src[(int64_t)d * n + o];
}

__global__ void __launch_bounds__(256) k_from_store(Batch b, Store s, int k, const float *__restrict__ src, int64_t n,
                                                    float *__restrict__ dst) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= b.nparts) return;
  const int o = s.oidx[p];
  for (int d = 0; d < k; ++d) dst[(int64_t)d * n + o] = src[(int64_t)d * s.cap + p];
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

size_t window_lds_bytes(const TileGeo &tg, int ndim) {
  size_t nW = 1, nC = 1;
  for (int d = 0; d < ndim; ++d) {
    size_t wn = (size_t)(1 << tg.lt[d]) + 2 * tg.H + 3;
    nW *= wn;
    nC *= wn - 1;
  }
  return nW * 8 + nW * 4 + nC * 4 * ndim;
}

#define PIC_ND(nd_, ...)    \
  do {                      \
    if ((nd_) == 2) {       \
      constexpr int ND = 2; \
      __VA_ARGS__;          \
    } else {                \
      constexpr int ND = 3; \
      __VA_ARGS__;          \
    }                       \
  } while (0)

void launch_import(hipStream_t st, int ndim, const SlabDesc *sd_host, const PartPtrs *cp, int nslab,
                   const BinBufs &bb, const Batch &b, int chunk, const Store &dst, int *stage, uint32_t *err) {
  launch_fill32(st, bb.counts, b.ntiles);
  for (int k = 0; k < nslab; ++k)
    if (cp[k].n > 0)
      PIC_ND(ndim, (k_import_hist<ND><<<nblk(cp[k].n, 256 * kWaveRuns), 256, 0, st>>>(sd_host[k], cp[k], bb.counts,
                                                                                     err)));
  launch_tile_scan(st, b.ntiles, chunk, bb);
  k_tile_items<<<nblk(b.ntiles), 256, 0, st>>>(b, bb.counts, bb.starts, bb.item_start, bb.items);
  for (int k = 0; k < nslab; ++k)
    if (cp[k].n > 0)
      PIC_ND(ndim, (k_import_index<ND><<<nblk(cp[k].n, 256 * kWaveRuns), 256, 0, st>>>(sd_host[k], cp[k], bb.starts,
                                                                                      bb.cursors, stage)));
  for (int k = 0; k < nslab; ++k)
    if (cp[k].n > 0 && sd_host[k].tg.ntiles > 0)
      PIC_ND(ndim, (k_import_gather<ND><<<sd_host[k].tg.ntiles, kGatherThreads, 0, st>>>(sd_host[k], cp[k], dst,
                                                                                         bb.counts, bb.starts, stage,
                                                                                         err)));
}

void launch_rebin(hipStream_t st, int ndim, const BinBufs &bb, const Batch &b, int chunk, const Store &src,
                  const Store &dst) {
  launch_fill32(st, bb.counts, b.ntiles);
  if (b.nparts > 0) PIC_ND(ndim, (k_rebin_hist<ND><<<nblk(b.nparts), 256, 0, st>>>(b, src, bb.counts)));
  launch_tile_scan(st, b.ntiles, chunk, bb);
  k_tile_items<<<nblk(b.ntiles), 256, 0, st>>>(b, bb.counts, bb.starts, bb.item_start, bb.items);
  if (b.nparts > 0)
    PIC_ND(ndim, (k_rebin_scatter<ND><<<nblk(b.nparts), 256, 0, st>>>(b, src, dst, bb.starts, bb.cursors)));
}

void launch_export(hipStream_t st, int ndim, const SlabDesc &sd, const Store &s, const BinBufs &bb,
                   const PartPtrs &cp) {
  if (sd.part_n <= 0 || sd.tg.ntiles <= 0) return;
  PIC_ND(ndim, (k_export<ND><<<sd.tg.ntiles, kGatherThreads, 0, st>>>(sd, s, bb.starts, cp)));
}

void launch_deposit_tiled(hipStream_t st, int ndim, const TileGeo &tg, const Batch &b, const Store &s,
                          const BinBufs &bb, int max_items, long long *N) {
  if (max_items <= 0) return;
  size_t nW = 1;
  for (int d = 0; d < ndim; ++d) nW *= (size_t)(1 << tg.lt[d]) + 2 * tg.H + 3;
  PIC_ND(ndim, (k_deposit_tiled<ND><<<max_items, 256, nW * 8, st>>>(b, s, bb.items, bb.num_items,
                                                                      (unsigned long long *)N)));
}

void launch_step_tiled(hipStream_t st, int ndim, const TileGeo &tg, const Pot &P, const DiagC &dc, const Batch &b,
                       const Store &s, const Store &o, const BinBufs &bb, int grid, const long long *Ncur,
                       long long *Nnext, long long *Nclear, const Drift &dr, double *partial, bool diag,
                       uint32_t *err) {
  if (grid <= 0) return;
  const size_t lds = window_lds_bytes(tg, ndim);
  unsigned long long *nn = (unsigned long long *)Nnext;
  const bool out = s.pc != o.pc;
  // GEN: the Morse potential or the hexagonal lattice (runtime choice); the
  // Lennard-Jones cubic step compiles without either
  const bool gen = P.kind != 0 || P.lattice != 0;
#define PIC_STEP(DG, OT, GN)                                                                                      \
  PIC_ND(ndim, (k_step_tiled<ND, DG, OT, GN><<<grid, 256, lds, st>>>(P, dc, b, s, o, bb.items, bb.num_items, Ncur, \
                                                                     nn, Nclear, dr, partial, err)))
  if (out) {
    if (gen) PIC_STEP(false, true, true);
    else PIC_STEP(false, true, false);
  } else if (diag) {
    if (gen) PIC_STEP(true, false, true);
    else PIC_STEP(true, false, false);
  } else {
    if (gen) PIC_STEP(false, false, true);
    else PIC_STEP(false, false, false);
  }
#undef PIC_STEP
}

void launch_reduce_diag_slab(hipStream_t st, const double *part_p, const int *item_start, int tile_lo, int tile_hi,
                             const double *part_g, int nblk_g, double *red, pic_diag_t *out, int64_t step) {
  k_reduce_diag_part<<<kRedBlocks, 256, 0, st>>>(part_p, item_start, tile_lo, tile_hi, part_g, nblk_g, red);
  k_reduce_diag_slab<<<1, 256, 0, st>>>(red, out, step);
}

size_t adjoint_lds_bytes(const TileGeo &tg, int ndim, bool planes) {
  size_t nW = 1, nC = 1;
  for (int d = 0; d < ndim; ++d) {
    size_t wn = (size_t)(1 << tg.lt[d]) + 2 * tg.H + 3;
    nW *= wn;
    nC *= wn - 1;
  }
  return nW * (8 + 4 + 4) + (planes ? nC * 4 * (size_t)ndim : 0);
}

// The reverse step reads centre planes when they still leave room for 4
// blocks per CU (the kernel's occupancy bound); a larger window keeps its
// occupancy and builds the gradients from each particle's node block.
static bool adjoint_planes(const TileGeo &tg, int ndim) { return adjoint_lds_bytes(tg, ndim, true) <= 40 * 1024; }

void launch_adjoint_tiled(hipStream_t st, int ndim, const TileGeo &tg, const Pot &P, const Batch &b, const Store &s,
                          const BinBufs &bb, int max_items, const long long *N, const float *nbar_next,
                          float *lx, float *lv, float *nbar, int *dlist, int *dcount,
                          const uint32_t *amax_prev, uint32_t *amax_cur, double *partial, double *dacc,
                          uint32_t *err, const Store *next, float *nbar_clear, int64_t nclear, int *dcount_clear,
                          uint32_t *amax_clear) {
  const int *pc_next = next ? next->pc : nullptr;
  const float *off_next = next ? next->off : nullptr;
  if (max_items <= 0) return;
  const bool planes = adjoint_planes(tg, ndim);
  const size_t lds = adjoint_lds_bytes(tg, ndim, planes);
  // dcount and amax_cur start at zero: the caller clears them (with nbar)
  // GEN: the Morse potential or the hexagonal lattice (runtime choice)
#define PIC_ADJT(GN, PL)                                                                                          \
  PIC_ND(ndim, (k_adjoint_tiled<ND, false, GN, PL><<<max_items, 256, lds, st>>>(P, b, s, bb.items, bb.num_items, \
                                                                                  N, nbar_next, lx, lv, nbar,    \
                                                                                  dlist, dcount, amax_prev,      \
                                                                                  amax_cur, partial, err,        \
                                                                                  pc_next, off_next, nbar_clear, \
                                                                                  nclear)))
  if (P.kind != 0 || P.lattice != 0) {
    if (planes) PIC_ADJT(true, true);
    else PIC_ADJT(true, false);
    PIC_ND(ndim, (k_adjoint_drifters<ND, true><<<kDriftBlocks, 256, 0, st>>>(P, b, s, dlist, dcount, N, nbar_next, lx,
                                                                             lv, nbar, dacc, err, dcount_clear,
                                                                             amax_clear)));
  } else {
    if (planes) PIC_ADJT(false, true);
    else PIC_ADJT(false, false);
    PIC_ND(ndim, (k_adjoint_drifters<ND, false><<<kDriftBlocks, 256, 0, st>>>(P, b, s, dlist, dcount, N, nbar_next,
                                                                              lx, lv, nbar, dacc, err, dcount_clear,
                                                                              amax_clear)));
  }
#undef PIC_ADJT
}

void launch_adjoint_scale(hipStream_t st, int ndim, const TileGeo &tg, const Pot &P, const Batch &b, const Store &s,
                          const BinBufs &bb, int max_items, const long long *N, const float *nbar_next, float *lx,
                          float *lv, uint32_t *amax) {
  if (max_items <= 0) return;
  const size_t lds = adjoint_lds_bytes(tg, ndim, false);
  launch_fill32(st, reinterpret_cast<int *>(amax), 1);
#define PIC_ADJS(GN)                                                                                                \
  PIC_ND(ndim, (k_adjoint_tiled<ND, true, GN, false><<<max_items, 256, lds, st>>>(P, b, s, bb.items, bb.num_items, \
                                                                                    N, nbar_next, lx, lv, nullptr,  \
                                                                                    nullptr, nullptr, amax, amax,   \
                                                                                    nullptr, nullptr, nullptr,      \
                                                                                    nullptr, nullptr, 0)))
  if (P.kind != 0 || P.lattice != 0) PIC_ADJS(true);
  else PIC_ADJS(false);
#undef PIC_ADJS
}

void launch_deposit_vjp_store(hipStream_t st, int ndim, const Batch &b, const Store &s, const float *nbar,
                              float *lx) {
  if (b.nparts <= 0) return;
  PIC_ND(ndim, (k_deposit_vjp_store<ND><<<nblk(b.nparts), 256, 0, st>>>(b, s, nbar, lx)));
}

void launch_to_store(hipStream_t st, const Batch &b, const Store &s, int k, const float *src, int64_t n,
                     float *dst) {
  if (b.nparts > 0) k_to_store<<<nblk(b.nparts), 256, 0, st>>>(b, s, k, src, n, dst);
}

void launch_from_store(hipStream_t st, const Batch &b, const Store &s, int k, const float *src, int64_t n,
                       float *dst) {
  if (b.nparts > 0) k_from_store<<<nblk(b.nparts), 256, 0, st>>>(b, s, k, src, n, dst);
}

int step_kernel_blocks_per_cu(int ndim, const TileGeo &tg) {
  int nb = 0;
  const size_t lds = window_lds_bytes(tg, ndim);
  hipError_t e;
  if (ndim == 2) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step_tiled<2, false, false, false>, 256, lds);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step_tiled<3, false, false, false>, 256, lds);
  return e == hipSuccess && nb > 0 ? nb : 4;
}

}  // namespace pic
