// Crater measurement on the node sums of a finished run (results section,
// Figs. 3-4 and eq. 5).  Two passes, HBM-bound:
//
//  * column pass: every node's density in units of the solid density, set to
//    zero below the cut-off, optionally written out as the float map, and the
//    kept node weights summed per column (int64, so the sums are exact and
//    independent of order);
//  * reduction: per slab, each column's equivalent solid thickness
//    t = sum * 2^-20 / (n_solid * cross-section), its deficit y_s - t below
//    the initial surface, the deepest deficit, the cratered columns (deficit
//    >= depth_min), the crater diameter, and eq. (5).
//
// The cut-off is defined on the FP64 density (N * 2^-20 / V) / n_solid, V
// the node volume (halved once per wall the node lies on).  That value
// grows with the integer node sum N, so the host turns the decision into the
// smallest kept N per wall count and the kernel compares integers: the same
// decision, with no FP64 division per node.  The float map is N times a
// float scale (two roundings).
#include <cmath>

#include "pic_crater.h"

namespace pic {

namespace {

__device__ inline int lateral_walls(const CraterSlab &s, int col) {
  int w = 0;
  for (int d = 0; d < s.ndim - 1; ++d) {
    const int i = col % s.nn[d];
    col /= s.nn[d];
    if (s.bc[d] && (i == 0 || i == s.nn[d] - 1)) ++w;
  }
  return w;
}

// grid: x = blocks of 256 columns, y = chunks of kCraterRows rows, z = slab
// of the batch.  A thread owns one column's rows of its chunk: adjacent
// threads read adjacent nodes of a row.
__global__ void __launch_bounds__(256) k_crater_columns(CraterBatch b, CraterArgs a, const long long *node_w,
                                                         float *rho, unsigned long long *col_w) {
  const CraterSlab &s = b.s[blockIdx.z];
  const int col = blockIdx.x * 256 + threadIdx.x;
  const int r0 = blockIdx.y * kCraterRows;
  if (col >= s.ncols || r0 >= s.rows) return;
  const int r1 = min(r0 + kCraterRows, s.rows);
  const int ax = s.ndim - 1;
  const int lw = lateral_walls(s, col);
  const long long *src = node_w + s.node_off + col;
  // all of the chunk's loads first, so they are in flight together
  long long Nv[kCraterRows];
#pragma unroll
  for (int q = 0; q < kCraterRows; ++q)
    Nv[q] = r0 + q < r1 ? src[(long long)s.ncols * (r0 + q)] : 0;
  long long sum = 0;
#pragma unroll
  for (int q = 0; q < kCraterRows; ++q) {
    const int r = r0 + q;
    if (r >= r1) break;
    const long long N = Nv[q];
    const int walls = lw + ((s.bc[ax] && (r == 0 || r == s.rows - 1)) ? 1 : 0);
    const bool keep = N >= s.keep_min[walls];
    if (rho) rho[s.node_off + col + (long long)s.ncols * r] = keep ? (float)N * s.map_scale[walls] : 0.f;
    if (keep) sum += N;
  }
  if (sum) atomicAdd(col_w + s.col_off + col, (unsigned long long)sum);
}

template <typename T, typename Op>
__device__ inline T block_reduce(T v, T *lds, Op op) {
  lds[threadIdx.x] = v;
  __syncthreads();
  for (int w = kCraterReduceThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) lds[threadIdx.x] = op(lds[threadIdx.x], lds[threadIdx.x + w]);
    __syncthreads();
  }
  const T r = lds[0];
  __syncthreads();
  return r;
}

// One block per slab of the batch.
__global__ void __launch_bounds__(kCraterReduceThreads) k_crater_reduce(CraterBatch b, CraterArgs a,
                                                                         const long long *col_w, pic_crater_t *out) {
  __shared__ double ld[kCraterReduceThreads];
  __shared__ long long ll[kCraterReduceThreads];
  const CraterSlab &s = b.s[blockIdx.x];
  double tmin = INFINITY, tmax = -INFINITY;
  long long hits = 0, units = 0;  // units: quarter columns (lateral wall columns count half, corners a quarter)
  const long long *cw = col_w + s.col_off;
#pragma unroll 4
  for (int c = threadIdx.x; c < s.ncols; c += kCraterReduceThreads) {
    const int lw = lateral_walls(s, c);
    const double t = (double)cw[c] * s.t_scale * (double)(1 << lw);
    tmin = fmin(tmin, t);
    tmax = fmax(tmax, t);
    if (s.y_s - t >= a.depth_min) {
      ++hits;
      units += 4 >> lw;
    }
  }
  tmin = block_reduce(tmin, ld, [](double x, double y) { return fmin(x, y); });
  tmax = block_reduce(tmax, ld, [](double x, double y) { return fmax(x, y); });
  hits = block_reduce(hits, ll, [](long long x, long long y) { return x + y; });
  units = block_reduce(units, ll, [](long long x, long long y) { return x + y; });
  if (threadIdx.x == 0) {
    const double measure = (double)units * 0.25 * s.lat;
    const double width = s.ndim == 2 ? measure : 2.0 * sqrt(measure / M_PI);
    pic_crater_t r;
    r.depth = s.y_s - tmin;
    r.width = width;
    r.t_min = tmin;
    r.t_max = tmax;
    if (s.fluence > 0 && s.beam_d > 0) {
      const double q = width / s.beam_d;
      r.f_th = s.fluence * exp(-(q * q));
    } else {
      r.f_th = 0.0;
    }
    r.ncols = hits;
    out[blockIdx.x] = r;
  }
}

}  // namespace

void launch_crater_columns(hipStream_t st, const CraterBatch &b, int max_ncols, int max_rows, CraterArgs a,
                           const long long *node_w, float *rho, long long *col_w) {
  if (b.n < 1 || max_ncols < 1 || max_rows < 1) return;
  const dim3 grid((max_ncols + 255) / 256, (max_rows + kCraterRows - 1) / kCraterRows, b.n);
  k_crater_columns<<<grid, 256, 0, st>>>(b, a, node_w, rho, reinterpret_cast<unsigned long long *>(col_w));
}

void launch_crater_reduce(hipStream_t st, const CraterBatch &b, CraterArgs a, const long long *col_w,
                          pic_crater_t *out) {
  if (b.n < 1) return;
  k_crater_reduce<<<b.n, kCraterReduceThreads, 0, st>>>(b, a, col_w, out);
}

}  // namespace pic
