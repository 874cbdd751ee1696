// Reverse mode of the PIC pair-potential cycle (arXiv 1502.07722, Sec. 2):
// hand-written adjoints of deposit -> density/gradient -> gather -> eq. (1)-(3)
// -> leapfrog push, on caller arrays (one thread per particle).
//
// Cotangents carried per particle: lam_x = dJ/d(offset) per axis (per cell of
// displacement) and lam_v = dJ/dv (s/m).  Per node: nbar = dJ/d(n r0^3), the
// cotangent of the reduced node density.  Per cell centre (scratch): Gbar =
// dJ/d(dn/dx r0^4).  Parameters theta = (D, r0, s_rep, c_att, alpha); alpha,
// the Morse width, has a zero cotangent under Lennard-Jones.
//
// One reverse step n (forward: x(n), v(n-1/2) -> x(n+1), v(n+1/2)):
//   1. recompute the particle's forward step from x(n) (bit-identical to the
//      forward kernels: same device functions, same node sums);
//   2. complete lam_x(n+1) with the deposit term of step n+1:
//      lam_x += W kappa sum_k nbar(n+1)_k dS_k/dx at x(n+1);
//   3. reverse drift (mirror walls negate) and kick: lam_v += tau lam_x,
//      force cotangent mu = (dt/m) lam_v;
//   4. force VJP through eq. (3), (2), (1): cotangents of the gathered n and G
//      and of theta;
//   5. gather VJP: direct lam_x term, and scatters of the n and G cotangents to
//      nodes and cell centres; a grid pass then maps Gbar back to nodes
//      (transpose of the edge-difference stencil).
// The deposit term of step n itself is added by the next reverse step (2.),
// or by the deposit VJP at the end.  The fixed-point deposit is
// differentiated as the plain CIC deposit it approximates to 2^-16 cells.
#include "pic_internal.h"
#include "pic_adjoint_dev.h"

namespace pic {

// ---------------------------------------------------------------------------
// Kernels on caller arrays
// ---------------------------------------------------------------------------
// MODE 0: one full reverse step (lam_x, lam_v in/out).  MODE 1: VJP of the
// force alone, given the force cotangent fbar (1/N); lam_x accumulates.
template <int ND, int MODE>
__global__ void __launch_bounds__(256) k_adjoint(Geo g, Pot P, int64_t n, const int *__restrict__ cell,
                                                 const float *__restrict__ off, const float *__restrict__ vel,
                                                 const int *__restrict__ wq, const float *__restrict__ dens,
                                                 const float *__restrict__ G, const float *__restrict__ nbar_next,
                                                 const float *__restrict__ fbar, float *__restrict__ lam_x,
                                                 float *__restrict__ lam_v, float *__restrict__ nbar,
                                                 float *__restrict__ Gbar, double *__restrict__ partial,
                                                 uint32_t *__restrict__ err) {
  // Each wave takes every fourth particle of the block's 256 (blocks are
  // always 256 threads): particles next to each other in the caller's order,
  // often of one cell, land in different waves, so fewer lanes of a wave add
  // into the same node or cell at once.
  const int t = (int)threadIdx.x;
  const int64_t p = (int64_t)blockIdx.x * 256 + ((t & 63) << 2 | t >> 6);
  double thd[5] = {0, 0, 0, 0, 0};
  if (p < n) {
    int c = cell[p];
    float f[3] = {off[p], off[n + p], ND == 3 ? off[2 * n + p] : 0.0f};
    uint32_t e = (c < 0 || c >= g.ncells) ? ERR_RANGE : 0u;
#pragma unroll
    for (int d = 0; d < ND; ++d) e |= (f[d] >= 0.0f && f[d] < 1.0f) ? 0u : ERR_RANGE;
    if (e) {
      atomicOr(err, e);
    } else {
      int idx[3];
      decode_cell<ND>(g, c, idx);
      GatherState<ND> gs;
      gather_for_vjp<ND>(g, dens, G, idx, f, gs);
      float mu[3] = {0.f, 0.f, 0.f}, lf[3] = {0.f, 0.f, 0.f};
      if (MODE == 0) {
        const float v[3] = {vel[p], vel[n + p], vel[2 * n + p]};
        float ln[3] = {lam_x[p], lam_x[n + p], ND == 3 ? lam_x[2 * n + p] : 0.0f};
        float lv[3] = {lam_v[p], lam_v[n + p], lam_v[2 * n + p]};
        e = reverse_push<ND, true>(g, P, idx, f, v, nbar_next ? wq[p] : 0, gs.nh, gs.Gp, nbar_next, ln, lv, lf,
                                   mu);
        if (e) atomicOr(err, e);
#pragma unroll
        for (int d = 0; d < 3; ++d) lam_v[(int64_t)d * n + p] = lv[d];
      } else {
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          mu[d] = fbar[(int64_t)d * n + p] * P.beta;
          lf[d] = lam_x[(int64_t)d * n + p];
        }
      }
      float an, aG[3], th[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
      pair_force_vjp<ND, true>(P, gs.nh, gs.Gp, mu, an, aG, th);
      gather_vjp<ND>(g, idx, f, gs, an, aG, lf, nbar, Gbar);
#pragma unroll
      for (int d = 0; d < ND; ++d) lam_x[(int64_t)d * n + p] = lf[d];
#pragma unroll
      for (int i = 0; i < 5; ++i) thd[i] = th[i];
    }
  }
  block_reduce_store<5>(thd, partial + (int64_t)blockIdx.x * 8);
}

// nbar_k += sum over the cells c touching node k of gam_d Gbar_c[d] (+1 if k is
// an upper corner of c along d, else -1): the transpose of the gradient.
template <int ND>
__global__ void __launch_bounds__(256) k_gradient_vjp(Geo g, const float *__restrict__ Gbar,
                                                      float *__restrict__ nbar) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.nnodes) return;
  int a[3];
  a[0] = k % g.nn[0];
  const int r = k / g.nn[0];
  a[1] = ND == 2 ? r : r % g.nn[1];
  a[2] = ND == 2 ? 0 : r / g.nn[1];
  float acc = 0.0f;
#pragma unroll
  for (int b = 0; b < (1 << ND); ++b) {
    int m[3] = {0, 0, 0};
    bool ok = true;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      int md = a[d] - ((b >> d) & 1);
      if (g.bc[d]) ok = ok && md >= 0 && md < g.n[d];
      else md = md < 0 ? md + g.n[d] : md;
      m[d] = md;
    }
    if (!ok) continue;
    const int cc = encode_cell<ND>(g, m);
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const float v = g.gam[d] * Gbar[(int64_t)d * g.ncells + cc];
      acc += ((b >> d) & 1) ? v : -v;
    }
  }
  nbar[k] += acc;
}

template <int ND>
__global__ void __launch_bounds__(256) k_deposit_vjp(Geo g, int64_t n, const int *__restrict__ cell,
                                                     const float *__restrict__ off, const int *__restrict__ wq,
                                                     const float *__restrict__ nbar, float *__restrict__ lam_x,
                                                     uint32_t *__restrict__ err) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int c = cell[p];
  float f[3] = {off[p], off[n + p], ND == 3 ? off[2 * n + p] : 0.0f};
  uint32_t e = (c < 0 || c >= g.ncells) ? ERR_RANGE : 0u;
#pragma unroll
  for (int d = 0; d < ND; ++d) e |= (f[d] >= 0.0f && f[d] < 1.0f) ? 0u : ERR_RANGE;
  if (e) {
    atomicOr(err, e);
    return;
  }
  int idx[3];
  decode_cell<ND>(g, c, idx);
  float lf[3] = {lam_x[p], lam_x[n + p], ND == 3 ? lam_x[2 * n + p] : 0.0f};
  deposit_term<ND>(g, nbar, idx, f, wq[p], lf);
#pragma unroll
  for (int d = 0; d < ND; ++d) lam_x[(int64_t)d * n + p] = lf[d];
}

__global__ void k_fillf(float *__restrict__ a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0f;
}

// The clears of one reverse step in one launch: the step's node cotangents
// and two counters (drifters, largest contribution).
__global__ void k_clear_reverse(float *__restrict__ a, int64_t n, int *__restrict__ c1,
                                uint32_t *__restrict__ c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0f;
  if (i == 0) {
    *c1 = 0;
    *c2 = 0u;
  }
}

// Fixed-order sum of the per-block parameter partials into dtheta (+=);
// scale[i] turns slot i into dJ/dtheta_i (1/D, 1/r0, 1, 1, 1/alpha or 0).
__global__ void __launch_bounds__(256) k_reduce_theta(const double *__restrict__ partial, int nblocks, ThetaScale sc,
                                                      double *__restrict__ dtheta, double *__restrict__ extra) {
  __shared__ double red[kTheta][256];
  double acc[kTheta] = {0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
#pragma unroll
    for (int i = 0; i < kTheta; ++i) acc[i] += partial[(int64_t)b * 8 + i];
#pragma unroll
  for (int i = 0; i < kTheta; ++i) red[i][threadIdx.x] = acc[i];
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
#pragma unroll
      for (int i = 0; i < kTheta; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < kTheta) {
    const double scale = sc.s[threadIdx.x];
    double v = red[threadIdx.x][0];
    if (extra) {
      v += extra[threadIdx.x];
      extra[threadIdx.x] = 0.0;
    }
    dtheta[threadIdx.x] += v * scale;
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

void launch_fillf(hipStream_t st, float *a, int64_t n) {
  if (n > 0) hipLaunchKernelGGL(k_fillf, dim3(blocks_for(n)), dim3(256), 0, st, a, n);
}

void launch_clear_reverse(hipStream_t st, float *a, int64_t n, int *c1, uint32_t *c2) {
  hipLaunchKernelGGL(k_clear_reverse, dim3(blocks_for(n > 0 ? n : 1)), dim3(256), 0, st, a, n, c1, c2);
}

int launch_adjoint(hipStream_t st, const Geo &g, const Pot &P, const PartPtrs &p, const float *dens, const float *G,
                   const float *nbar_next, const float *fbar, float *lam_x, float *lam_v, float *nbar, float *Gbar,
                   double *partial, uint32_t *err, bool force_only) {
  if (p.n <= 0) return 0;
  const unsigned nb = blocks_for(p.n);
#define PIC_ADJ(ND, M)                                                                                         \
  hipLaunchKernelGGL((k_adjoint<ND, M>), dim3(nb), dim3(256), 0, st, g, P, p.n, p.cell, p.off, p.vel, p.wq, dens, \
                     G, nbar_next, fbar, lam_x, lam_v, nbar, Gbar, partial, err)
  if (g.ndim == 2) {
    if (force_only) PIC_ADJ(2, 1);
    else PIC_ADJ(2, 0);
  } else {
    if (force_only) PIC_ADJ(3, 1);
    else PIC_ADJ(3, 0);
  }
#undef PIC_ADJ
  return (int)nb;
}

void launch_gradient_vjp(hipStream_t st, const Geo &g, const float *Gbar, float *nbar) {
  if (g.nnodes <= 0) return;
  if (g.ndim == 2) hipLaunchKernelGGL(k_gradient_vjp<2>, dim3(blocks_for(g.nnodes)), dim3(256), 0, st, g, Gbar, nbar);
  else hipLaunchKernelGGL(k_gradient_vjp<3>, dim3(blocks_for(g.nnodes)), dim3(256), 0, st, g, Gbar, nbar);
}

void launch_deposit_vjp(hipStream_t st, const Geo &g, const PartPtrs &p, const float *nbar, float *lam_x,
                        uint32_t *err) {
  if (p.n <= 0) return;
  if (g.ndim == 2)
    hipLaunchKernelGGL(k_deposit_vjp<2>, dim3(blocks_for(p.n)), dim3(256), 0, st, g, p.n, p.cell, p.off, p.wq, nbar,
                       lam_x, err);
  else
    hipLaunchKernelGGL(k_deposit_vjp<3>, dim3(blocks_for(p.n)), dim3(256), 0, st, g, p.n, p.cell, p.off, p.wq, nbar,
                       lam_x, err);
}

void launch_reduce_theta(hipStream_t st, const double *partial, int nblocks, const ThetaScale &sc, double *dtheta,
                         double *extra) {
  hipLaunchKernelGGL(k_reduce_theta, dim3(1), dim3(256), 0, st, partial, nblocks, sc, dtheta, extra);
}

}  // namespace pic
