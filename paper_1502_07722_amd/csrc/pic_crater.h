// Crater measurement on node sums: per-slab tables and launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/pic.h"

namespace pic {

// One slab as the crater kernels see it.  Columns are the node lines along
// the normal (last) axis; a slab's nodes are node_off + col + ncols * row.
struct CraterSlab {
  long long node_off;  // first node of the slab in the caller's node array
  long long col_off;   // first column of the slab in the column array
  int nn[3];           // nodes per axis, fastest first (nn[ndim - 1] = rows)
  int bc[3];           // 1: reflecting walls on that axis (their nodes have half volume)
  int ndim, ncols, rows, pad;
  long long keep_min[4];  // by walls touched (0-3): smallest node sum at or above the cut-off
  float map_scale[4];     // by walls touched: density map = node sum * this (units of n_solid)
  double t_scale;         // thickness = column sum * t_scale * 2^(lateral walls), m
  double lat;             // lateral measure of a column away from walls: dx (2D), dx*dy (3D)
  double y_s;          // initial surface height, m
  double fluence;      // peak absorbed fluence for eq. (5), J/m^2 (0: none)
  double beam_d;       // beam diameter for eq. (5), m (0: none)
};

constexpr int kCraterSlabs = 16;  // slabs per launch (the table travels as a kernel argument)
constexpr int kCraterRows = 16;   // node rows per thread in the column pass (a launch-shape sweep's best)
constexpr int kCraterReduceThreads = 1024;

struct CraterBatch {
  CraterSlab s[kCraterSlabs];
  int n;
};

struct CraterArgs {
  double n_solid, cut, depth_min;
};

// Column pass: cut-off density map (rho may be NULL) and per-column sums of
// the kept node weights, added into col_w (cleared by the caller).
void launch_crater_columns(hipStream_t st, const CraterBatch &b, int max_ncols, int max_rows, CraterArgs a,
                           const long long *node_w, float *rho, long long *col_w);
// Per-slab reduction of the column sums into out[slab].
void launch_crater_reduce(hipStream_t st, const CraterBatch &b, CraterArgs a, const long long *col_w,
                          pic_crater_t *out);

}  // namespace pic
