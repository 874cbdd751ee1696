// Internal declarations shared by the C-ABI layer and the kernel files.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/pic.h"
#include "pic_device.h"

namespace pic {

// FP64 constants of the diagnostics (SI).
struct DiagC {
  double D, mass, half_m, wunit, vcell, r0cube, s_rep, c_att;
  int kind;     // pair potential: 0 Lennard-Jones (closed-form energy density), 1 Morse
  double mA;    // Morse: alpha r0
  int lattice;  // 0 cubic, 1 hexagonal close-packed
};

// 16-point Gauss-Legendre rule on [-1, 1] (the Morse energy density is an
// integral with no closed form).
struct Quad16 {
  double x[16], w[16];
};

struct PartPtrs {
  int64_t n;
  int *cell;
  float *off;
  float *vel;
  int *wq;
};

// Internal particle store of the tiled step: binned by tile, packed cell
// coordinates (2D: i | j << 16; 3D: i | j << 11 | k << 22), SoA with stride cap.
struct Store {
  int *pc;
  float *off;   // [ndim][cap]
  float *vel;   // [3][cap]
  int *wq;
  int *oidx;    // index of the particle in the caller's arrays
  int64_t cap;
};

// Tiling of the grid: tiles of 2^lt[d] cells per axis, halo H cells.
struct TileGeo {
  int lt[3];
  int tn[3];
  int ntiles;
  int H;
  int chunk;      // most particles per work item
  int pshift[3];  // packed-coordinate bit offsets
  int pmask[3];
};

// One slab of a (possibly batched) context: grid, tiling, and where its
// nodes, tiles and store slots start in the concatenated arrays.
struct SlabDesc {
  Geo g;
  TileGeo tg;
  int node_off;
  int tile_off;
  int part_off;
  int part_n;
};

// Device-side slab tables, passed by value to the kernels.
struct Batch {
  const SlabDesc *slabs;  // [nslab]
  const int *part_offs;   // [nslab + 1] first store slot of each slab
  const int *tile_offs;   // [nslab + 1] first tile of each slab
  int nslab;
  int ntiles;
  int nnodes;
  int nparts;
};

struct Item {
  int tile, start, end, slab;
};

// Drifter list of the fused step: particle slots outside their tile window,
// and the persistent kernel's work counter.  Counters alternate between
// steps; a step clears the next step's pair.
constexpr int kDriftBlocks = 256;
struct Drift {
  int *list;        // [store capacity]
  int *count;       // this step's drifter counter
  int *count_next;  // next step's
  int *work;        // this step's work-item counter
  int *work_next;   // next step's
};

struct BinBufs {
  int *counts;      // [ntiles]
  int *starts;      // [ntiles + 1]
  int *cursors;     // [ntiles]
  int *item_start;  // [ntiles + 1]
  Item *items;      // [max_items]
  int *num_items;   // [1]
};

void launch_fill64(hipStream_t s, long long *a, int64_t n);
void launch_clear_word(hipStream_t s, uint32_t *w);
void launch_deposit_atomic(hipStream_t s, const Geo &g, const PartPtrs &pp, long long *node, uint32_t *err);
void launch_grid(hipStream_t s, const Geo &g, const long long *node, float *dens, float *G);
void launch_force(hipStream_t s, const Geo &g, const Pot &P, const PartPtrs &pp, const float *dens,
                  const float *G, float *force, uint32_t *err);
void launch_push(hipStream_t s, const Geo &g, const Pot &P, const PartPtrs &pp, const float *force,
                 uint32_t *err);
void launch_kick(hipStream_t s, const Geo &g, const Pot &P, const PartPtrs &pp, const float *force, float frac);
int launch_force_push(hipStream_t s, const Geo &g, const Pot &P, const DiagC &dc, const PartPtrs &pp,
                      const float *dens, const float *G, double *partial, bool diag, uint32_t *err);
int launch_pe_nodes(hipStream_t s, const Geo &g, const DiagC &dc, const Quad16 &q, const long long *node,
                    double *partial);
void launch_reduce_diag(hipStream_t s, const double *part_p, int nblk_p, const double *part_g, int nblk_g,
                        pic_diag_t *out, int64_t step);

// tiled path (pic_tiled.hip)
size_t window_lds_bytes(const TileGeo &tg, int ndim);
// stage: int[store capacity] scratch (not dst's arrays)
void launch_import(hipStream_t st, int ndim, const SlabDesc *sd_host, const PartPtrs *cp, int nslab,
                   const BinBufs &bb, const Batch &b, int chunk, const Store &dst, int *stage, uint32_t *err);
void launch_rebin(hipStream_t st, int ndim, const BinBufs &bb, const Batch &b, int chunk, const Store &src,
                  const Store &dst);
// s must be binned as bb says (the last import or re-binning)
void launch_export(hipStream_t st, int ndim, const SlabDesc &sd, const Store &s, const BinBufs &bb,
                   const PartPtrs &cp);
void launch_deposit_tiled(hipStream_t st, int ndim, const TileGeo &tg, const Batch &b, const Store &s,
                          const BinBufs &bb, int max_items, long long *N);
// s: the state read; o: where the next state is written (o == s: in place)
void launch_step_tiled(hipStream_t st, int ndim, const TileGeo &tg, const Pot &P, const DiagC &dc, const Batch &b,
                       const Store &s, const Store &o, const BinBufs &bb, int grid, const long long *Ncur,
                       long long *Nnext, long long *Nclear, const Drift &dr, double *partial, bool diag,
                       uint32_t *err);
// red: kDiagRedDoubles doubles of scratch
constexpr int kDiagRedDoubles = 256 * 8;
void launch_reduce_diag_slab(hipStream_t st, const double *part_p, const int *item_start, int tile_lo, int tile_hi,
                             const double *part_g, int nblk_g, double *red, pic_diag_t *out, int64_t step);
int step_kernel_blocks_per_cu(int ndim, const TileGeo &tg);
void launch_fill32(hipStream_t s, int *a, int64_t n);

// reverse mode in the store (pic_tiled.hip); lx [ndim][cap], lv [3][cap]
size_t adjoint_lds_bytes(const TileGeo &tg, int ndim, bool planes);
// partial: per-item parameter sums, ACCUMULATED over the calls (clear once);
// N: the step's node sums; nbar, dcount and amax_cur must be zero on entry
// (launch_clear_reverse, or the previous reverse step's clears below)
// next: the state after this step in the same binning (its cells and
// offsets, written by the forward), or null: the push is then recomputed
// nbar_clear [nclear], dcount_clear, amax_clear (or null): the next reverse
// step's nbar, dcount and amax_cur, zeroed by this step's kernels; none may
// alias a buffer this step reads or writes
void launch_adjoint_tiled(hipStream_t st, int ndim, const TileGeo &tg, const Pot &P, const Batch &b, const Store &s,
                          const BinBufs &bb, int max_items, const long long *N, const float *nbar_next, float *lx,
                          float *lv, float *nbar, int *dlist, int *dcount, const uint32_t *amax_prev,
                          uint32_t *amax_cur, double *partial, double *dacc, uint32_t *err,
                          const Store *next = nullptr, float *nbar_clear = nullptr, int64_t nclear = 0,
                          int *dcount_clear = nullptr, uint32_t *amax_clear = nullptr);
// largest node-cotangent contribution of a reverse step, measured only (the
// fixed-point scale of the first reverse step); lx, lv are read only
void launch_adjoint_scale(hipStream_t st, int ndim, const TileGeo &tg, const Pot &P, const Batch &b, const Store &s,
                          const BinBufs &bb, int max_items, const long long *N, const float *nbar_next, float *lx,
                          float *lv, uint32_t *amax);
void launch_deposit_vjp_store(hipStream_t st, int ndim, const Batch &b, const Store &s, const float *nbar,
                              float *lx);
void launch_to_store(hipStream_t st, const Batch &b, const Store &s, int k, const float *src, int64_t n,
                     float *dst);
void launch_from_store(hipStream_t st, const Batch &b, const Store &s, int k, const float *src, int64_t n,
                       float *dst);

// reverse mode on caller arrays (pic_adjoint.hip)
void launch_fillf(hipStream_t st, float *a, int64_t n);
// a[0..n) = 0, *c1 = 0, *c2 = 0 in one launch
void launch_clear_reverse(hipStream_t st, float *a, int64_t n, int *c1, uint32_t *c2);
int launch_adjoint(hipStream_t st, const Geo &g, const Pot &P, const PartPtrs &p, const float *dens, const float *G,
                   const float *nbar_next, const float *fbar, float *lam_x, float *lam_v, float *nbar, float *Gbar,
                   double *partial, uint32_t *err, bool force_only);
void launch_gradient_vjp(hipStream_t st, const Geo &g, const float *Gbar, float *nbar);
void launch_deposit_vjp(hipStream_t st, const Geo &g, const PartPtrs &p, const float *nbar, float *lam_x,
                        uint32_t *err);
// Parameters of the reverse mode: D, r0, s_rep, c_att, alpha (Morse width).
constexpr int kTheta = 5;
struct ThetaScale {
  double s[kTheta];
};
// dtheta[i] += s[i] * (sum of the block partials + extra[i]), i < kTheta;
// extra (nullable) is cleared
void launch_reduce_theta(hipStream_t st, const double *partial, int nblocks, const ThetaScale &sc, double *dtheta,
                         double *extra = nullptr);

}  // namespace pic
