// Per-particle and per-grid HIP kernels of the PIC pair-potential cycle
// (arXiv 1502.07722) for gfx950, plus their host launchers.
//
//   k_deposit_atomic  step 1, one thread per particle, int64 global atomics
//   k_density         node sums -> reduced node density (FP32)
//   k_gradient        cell-centred gradient (FP32) from the node densities
//   k_force           steps 3-5: gather + eq. (1)-(3) -> force in newtons
//   k_push / k_kick   step 6 on caller arrays
//   k_force_push      steps 3-6 fused, optional FP64 diagnostics
//   k_pe_nodes        grid potential energy sum V eps(n) (FP64 diagnostic)
//   k_reduce_diag     fixed-order final reduction of the block partials
#include "pic_internal.h"

namespace pic {

// ---------------------------------------------------------------------------
// Deposit
// ---------------------------------------------------------------------------
template <int ND>
__device__ __forceinline__ uint32_t load_particle(const Geo &g, int64_t n, int64_t p, const int *cell,
                                                  const float *off, int &c, float f[3]) {
  c = cell[p];
  f[0] = off[p];
  f[1] = off[n + p];
  f[2] = ND == 3 ? off[2 * n + p] : 0.0f;
  uint32_t e = 0;
  if (c < 0 || c >= g.ncells) e |= ERR_RANGE;
#pragma unroll
  for (int d = 0; d < ND; ++d)
    if (!(f[d] >= 0.0f && f[d] < 1.0f)) e |= ERR_RANGE;
  return e;
}

template <int ND>
__global__ void __launch_bounds__(256) k_deposit_atomic(Geo g, int64_t n, const int *__restrict__ cell,
                                                        const float *__restrict__ off,
                                                        const int *__restrict__ wq,
                                                        unsigned long long *__restrict__ node,
                                                        uint32_t *__restrict__ err) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int c;
  float f[3];
  uint32_t e = load_particle<ND>(g, n, p, cell, off, c, f);
  int W = wq[p];
  if (W < 0) e |= ERR_WEIGHT;
  if (e) {
    atomicOr(err, e);
    return;
  }
  int idx[3];
  decode_cell<ND>(g, c, idx);
  uint32_t t[8];
  deposit_shares<ND>((uint32_t)W, f, t);
#pragma unroll
  for (int k = 0; k < (1 << ND); ++k) {
    int a0 = node_axis(g, 0, idx[0] + (k & 1));
    int a1 = node_axis(g, 1, idx[1] + ((k >> 1) & 1));
    int a2 = ND == 3 ? node_axis(g, 2, idx[2] + ((k >> 2) & 1)) : 0;
    if (t[k]) atomicAdd(&node[node_index<ND>(g, a0, a1, a2)], (unsigned long long)t[k]);
  }
}

__global__ void k_fill64(unsigned long long *__restrict__ a, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0ull;
}

__global__ void k_fill32(int *__restrict__ a, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

__global__ void k_clear_word(uint32_t *w) { *w = 0u; }

// ---------------------------------------------------------------------------
// Grid pass: density at nodes, gradient at cell centres
// ---------------------------------------------------------------------------
template <int ND>
__global__ void __launch_bounds__(256) k_density(Geo g, const long long *__restrict__ node,
                                                 float *__restrict__ dens) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= g.nnodes) return;
  int a0 = k % g.nn[0];
  int r = k / g.nn[0];
  int a1 = ND == 2 ? r : r % g.nn[1];
  int a2 = ND == 2 ? 0 : r / g.nn[1];
  dens[k] = node_density(g, node[k], a0, a1, a2);
}

template <int ND>
__device__ __forceinline__ void cell_corners(const Geo &g, const float *__restrict__ dens, const int idx[3],
                                             float c[8]) {
  int x0 = idx[0], x1 = node_axis(g, 0, idx[0] + 1);
  int y0 = idx[1], y1 = node_axis(g, 1, idx[1] + 1);
  if (ND == 2) {
    c[0] = dens[node_index<2>(g, x0, y0, 0)];
    c[1] = dens[node_index<2>(g, x1, y0, 0)];
    c[2] = dens[node_index<2>(g, x0, y1, 0)];
    c[3] = dens[node_index<2>(g, x1, y1, 0)];
  } else {
    int z0 = idx[2], z1 = node_axis(g, 2, idx[2] + 1);
    c[0] = dens[node_index<3>(g, x0, y0, z0)];
    c[1] = dens[node_index<3>(g, x1, y0, z0)];
    c[2] = dens[node_index<3>(g, x0, y1, z0)];
    c[3] = dens[node_index<3>(g, x1, y1, z0)];
    c[4] = dens[node_index<3>(g, x0, y0, z1)];
    c[5] = dens[node_index<3>(g, x1, y0, z1)];
    c[6] = dens[node_index<3>(g, x0, y1, z1)];
    c[7] = dens[node_index<3>(g, x1, y1, z1)];
  }
}

template <int ND>
__global__ void __launch_bounds__(256) k_gradient(Geo g, const float *__restrict__ dens, float *__restrict__ G) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ncells) return;
  int idx[3];
  decode_cell<ND>(g, c, idx);
  float cr[8], Gc[3];
  cell_corners<ND>(g, dens, idx, cr);
  centre_gradient<ND>(g, cr, Gc);
#pragma unroll
  for (int d = 0; d < ND; ++d) G[(int64_t)d * g.ncells + c] = Gc[d];
}

// ---------------------------------------------------------------------------
// Gather from the global density / gradient grids
// ---------------------------------------------------------------------------
// Centre value of component d at (possibly ghost) centre m: periodic axes wrap,
// reflecting axes mirror the first interior centre and negate the normal part.
template <int ND>
__device__ __forceinline__ float centre_value(const Geo &g, const float *__restrict__ G, int d, int m0, int m1,
                                              int m2) {
  int m[3] = {m0, m1, m2};
  bool flip = false;
#pragma unroll
  for (int e = 0; e < ND; ++e) {
    if (m[e] < 0) {
      if (g.bc[e]) { m[e] = 0; flip ^= (e == d); }
      else m[e] += g.n[e];
    } else if (m[e] >= g.n[e]) {
      if (g.bc[e]) { m[e] = g.n[e] - 1; flip ^= (e == d); }
      else m[e] -= g.n[e];
    }
  }
  float v = G[(int64_t)d * g.ncells + encode_cell<ND>(g, m)];
  return flip ? -v : v;
}

template <int ND>
__device__ __forceinline__ void gather_global(const Geo &g, const float *__restrict__ dens,
                                              const float *__restrict__ G, const int idx[3], const float f[3],
                                              float &nh, float Gp[3]) {
  float cr[8];
  cell_corners<ND>(g, dens, idx, cr);
  nh = interp<ND>(cr, f);
  int c0[3] = {0, 0, 0};
  float t[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int e = 0; e < ND; ++e) centre_stencil(idx[e], f[e], c0[e], t[e]);
  Gp[2] = 0.0f;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    float v[8];
#pragma unroll
    for (int k = 0; k < (1 << ND); ++k)
      v[k] = centre_value<ND>(g, G, d, c0[0] + (k & 1), c0[1] + ((k >> 1) & 1),
                              ND == 3 ? c0[2] + ((k >> 2) & 1) : 0);
    Gp[d] = interp<ND>(v, t);
  }
}

template <int ND>
__global__ void __launch_bounds__(256) k_force(Geo g, Pot P, int64_t n, const int *__restrict__ cell,
                                               const float *__restrict__ off, const float *__restrict__ dens,
                                               const float *__restrict__ G, float *__restrict__ force,
                                               uint32_t *__restrict__ err) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int c;
  float f[3];
  uint32_t e = load_particle<ND>(g, n, p, cell, off, c, f);
  float F[3] = {0.f, 0.f, 0.f};
  if (e) {
    atomicOr(err, e);
  } else {
    int idx[3];
    decode_cell<ND>(g, c, idx);
    float nh, Gp[3];
    gather_global<ND>(g, dens, G, idx, f, nh, Gp);
    pair_force<ND, true>(P, nh, Gp, F);
  }
#pragma unroll
  for (int d = 0; d < ND; ++d) force[(int64_t)d * n + p] = F[d] * P.beta;
}

// ---------------------------------------------------------------------------
// Push / kick on caller arrays
// ---------------------------------------------------------------------------
template <int ND>
__global__ void __launch_bounds__(256) k_push(Geo g, Pot P, int64_t n, int *__restrict__ cell,
                                              float *__restrict__ off, float *__restrict__ vel,
                                              const float *__restrict__ force, uint32_t *__restrict__ err) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int c;
  float f[3];
  uint32_t e = load_particle<ND>(g, n, p, cell, off, c, f);
  if (e) {
    atomicOr(err, e);
    return;
  }
  int idx[3];
  decode_cell<ND>(g, c, idx);
  float v[3] = {vel[p], vel[n + p], vel[2 * n + p]};
  float F[3] = {force[p], force[n + p], ND == 3 ? force[2 * n + p] : 0.0f};
  e = push_particle<ND>(g, P, F, idx, f, v);
  if (e) atomicOr(err, e);
  cell[p] = encode_cell<ND>(g, idx);
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    off[(int64_t)d * n + p] = f[d];
    vel[(int64_t)d * n + p] = v[d];
  }
}

template <int ND>
__global__ void __launch_bounds__(256) k_kick(Pot P, int64_t n, float *__restrict__ vel,
                                              const float *__restrict__ force, float frac) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
#pragma unroll
  for (int d = 0; d < ND; ++d)
    vel[(int64_t)d * n + p] = __builtin_fmaf(force[(int64_t)d * n + p] * frac, P.gv, vel[(int64_t)d * n + p]);
}

// ---------------------------------------------------------------------------
// Fused gather + force + push on caller arrays (steps 3-6), optional diagnostics
// (KE, momentum, weight, bond energy) as per-block FP64 partials.
// ---------------------------------------------------------------------------
template <int ND, bool DIAG>
__global__ void __launch_bounds__(256) k_force_push(Geo g, Pot P, DiagC dc, int64_t n, int *__restrict__ cell,
                                                    float *__restrict__ off, float *__restrict__ vel,
                                                    const int *__restrict__ wq, const float *__restrict__ dens,
                                                    const float *__restrict__ G, double *__restrict__ partial,
                                                    uint32_t *__restrict__ err) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  if (p < n) {
    int c;
    float f[3];
    uint32_t e = load_particle<ND>(g, n, p, cell, off, c, f);
    if (e) {
      atomicOr(err, e);
    } else {
      int idx[3];
      decode_cell<ND>(g, c, idx);
      float nh, Gp[3], Fh[3], bond = 0.0f;
      gather_global<ND>(g, dens, G, idx, f, nh, Gp);
      pair_force<ND, true>(P, nh, Gp, Fh, DIAG ? &bond : nullptr);
      float F[3] = {Fh[0] * P.beta, Fh[1] * P.beta, ND == 3 ? Fh[2] * P.beta : 0.0f};
      float v[3] = {vel[p], vel[n + p], vel[2 * n + p]};
      if (DIAG) {
        double w = (double)wq[p] * dc.wunit;
        double vo2 = 0.0, vn2 = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          float vn = d < ND ? __builtin_fmaf(F[d], P.gv, v[d]) : v[d];
          vo2 += (double)v[d] * v[d];
          vn2 += (double)vn * vn;
          acc[1 + d] = w * dc.mass * 0.5 * ((double)v[d] + (double)vn);
        }
        acc[0] = w * dc.half_m * 0.5 * (vo2 + vn2);
        acc[4] = w;
        acc[5] = w * (double)bond * dc.D;
      }
      e = push_particle<ND>(g, P, F, idx, f, v);
      if (e) atomicOr(err, e);
      cell[p] = encode_cell<ND>(g, idx);
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        off[(int64_t)d * n + p] = f[d];
        vel[(int64_t)d * n + p] = v[d];
      }
    }
  }
  if (DIAG) block_reduce_store<6>(acc, partial + (int64_t)blockIdx.x * 8);
}

// Chemical potential mu / D of the Morse potential at reduced density x > 0,
// given t = x^(1/3).  Cubic: rho = 1 / t = rbar / r0, mu = M (U - rbar U') / D
// plus the altered branch's constant above x = 1 (M = c_att below, s_rep
// above).  Hexagonal: twice that at the neighbour distance a = 2^(1/6) rbar,
// kink at x = sqrt(2).
__device__ __forceinline__ double mu_morse_t(const DiagC &dc, double t) {
  const bool hcp = dc.lattice == 1;
  const double rho = (hcp ? 1.122462048309373 : 1.0) / t;
  const double e = exp(-dc.mA * (rho - 1.0));
  const double u = e * (e - 2.0);                 // U / D
  const double du = 2.0 * dc.mA * e * (1.0 - e);  // r0 U'(r) / D
  const double m = (hcp ? 2.0 : 1.0);
  return rho >= 1.0 ? m * dc.c_att * (u - rho * du) : m * (dc.s_rep * (u - rho * du) + (dc.s_rep - dc.c_att));
}

// Integral of mu over [a, b] in x, one 16-point Gauss-Legendre panel.
__device__ __forceinline__ double gauss16(const DiagC &dc, const Quad16 &q, double a, double b) {
  const double h = 0.5 * (b - a), m = 0.5 * (a + b);
  double acc = 0.0;
  for (int i = 0; i < 16; ++i) acc += q.w[i] * mu_morse_t(dc, cbrt(m + h * q.x[i]));
  return h * acc;
}

// Integral of mu over [0, b] in t = x^(1/3) (dx = 3 t^2 dt), two 16-point
// Gauss-Legendre panels: in x the integrand is flat near 0 and turns sharply
// where the neighbour distance nears r0 (one panel in x is only good to about
// 1e-6); in t it is smooth (two panels: 4e-13 relative).
__device__ __forceinline__ double gauss16_cbrt(const DiagC &dc, const Quad16 &q, double b) {
  const double h = 0.25 * cbrt(b);
  double acc = 0.0;
  for (int k = 0; k < 2; ++k) {
    const double m = (2 * k + 1) * h;
    for (int i = 0; i < 16; ++i) {
      const double t = m + h * q.x[i];
      acc += q.w[i] * 3.0 * t * t * mu_morse_t(dc, t);
    }
  }
  return h * acc;
}

// Energy density of the pair potential in units of D r0^-3 at reduced density x:
// e'(x) = mu: plain L-J e(x) = 13/5 x^5 - 14/3 x^3, branches switch at x = 1;
// Morse: the integral of mu from 0 to x, split at x = 1 where mu has a kink.
__device__ __forceinline__ double eps_hat(const DiagC &dc, const Quad16 &q, double x) {
  const bool hcp = dc.lattice == 1;
  const double xk = hcp ? 1.4142135623730951 : 1.0;  // where the neighbour distance is r0
  if (dc.kind == 1) {
    if (!(x > 0.0)) return 0.0;
    double e = gauss16_cbrt(dc, q, fmin(x, xk));
    if (x > xk) e += gauss16(dc, q, xk, x);
    return e;
  }
  // L-J: cubic e(x) = 13/5 x^5 - 14/3 x^3; hexagonal 13/10 x^5 - 14/3 x^3
  const double c5 = hcp ? 13.0 / 10.0 : 13.0 / 5.0, m = hcp ? 2.0 : 1.0;
  auto lj = [c5](double y) { return c5 * y * y * y * y * y - (14.0 / 3.0) * y * y * y; };
  if (x <= xk) return dc.c_att * lj(x);
  return dc.c_att * lj(xk) + dc.s_rep * (lj(x) - lj(xk)) + m * (dc.s_rep - dc.c_att) * (x - xk);
}

template <int ND>
__global__ void __launch_bounds__(256) k_pe_nodes(Geo g, DiagC dc, Quad16 q, const long long *__restrict__ node,
                                                  double *__restrict__ partial) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  double acc[1] = {0.0};
  if (k < g.nnodes) {
    int a0 = k % g.nn[0];
    int r = k / g.nn[0];
    int a1 = ND == 2 ? r : r % g.nn[1];
    int a2 = ND == 2 ? 0 : r / g.nn[1];
    double V = dc.vcell;
    if (g.bc[0] && (a0 == 0 || a0 == g.n[0])) V *= 0.5;
    if (g.bc[1] && (a1 == 0 || a1 == g.n[1])) V *= 0.5;
    if (ND == 3 && g.bc[2] && (a2 == 0 || a2 == g.n[2])) V *= 0.5;
    double x = (double)node[k] * dc.wunit * dc.r0cube / V;
    acc[0] = V * eps_hat(dc, q, x) * dc.D / dc.r0cube;
  }
  block_reduce_store<1>(acc, partial + (int64_t)blockIdx.x * 8);
}

// Single block: sum block partials in a fixed order into one diag entry.
__global__ void __launch_bounds__(256) k_reduce_diag(const double *__restrict__ part_p, int nblk_p,
                                                     const double *__restrict__ part_g, int nblk_g,
                                                     pic_diag_t *__restrict__ out, int64_t step) {
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblk_p; b += blockDim.x)
#pragma unroll
    for (int i = 0; i < 6; ++i) acc[i] += part_p[(int64_t)b * 8 + i];
  for (int b = threadIdx.x; b < nblk_g; b += blockDim.x) acc[6] += part_g[(int64_t)b * 8];
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
// Host launchers
// ---------------------------------------------------------------------------
static inline unsigned nblocks(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

#define PIC_DISPATCH(ND_, ...) \
  do {                         \
    if ((ND_) == 2) {          \
      constexpr int ND = 2;    \
      __VA_ARGS__;             \
    } else {                   \
      constexpr int ND = 3;    \
      __VA_ARGS__;             \
    }                          \
  } while (0)

void launch_fill64(hipStream_t s, long long *a, int64_t n) {
  if (n > 0) k_fill64<<<nblocks(n), 256, 0, s>>>((unsigned long long *)a, n);
}

void launch_clear_word(hipStream_t s, uint32_t *w) { k_clear_word<<<1, 1, 0, s>>>(w); }

void launch_fill32(hipStream_t s, int *a, int64_t n) {
  if (n > 0) k_fill32<<<nblocks(n), 256, 0, s>>>(a, n);
}

void launch_deposit_atomic(hipStream_t s, const Geo &g, const PartPtrs &pp, long long *node, uint32_t *err) {
  if (pp.n <= 0) return;
  PIC_DISPATCH(g.ndim, (k_deposit_atomic<ND><<<nblocks(pp.n), 256, 0, s>>>(
                           g, pp.n, pp.cell, pp.off, pp.wq, (unsigned long long *)node, err)));
}

void launch_grid(hipStream_t s, const Geo &g, const long long *node, float *dens, float *G) {
  PIC_DISPATCH(g.ndim, (k_density<ND><<<nblocks(g.nnodes), 256, 0, s>>>(g, node, dens)));
  PIC_DISPATCH(g.ndim, (k_gradient<ND><<<nblocks(g.ncells), 256, 0, s>>>(g, dens, G)));
}

void launch_force(hipStream_t s, const Geo &g, const Pot &P, const PartPtrs &pp, const float *dens,
                  const float *G, float *force, uint32_t *err) {
  if (pp.n <= 0) return;
  PIC_DISPATCH(g.ndim, (k_force<ND><<<nblocks(pp.n), 256, 0, s>>>(g, P, pp.n, pp.cell, pp.off, dens, G,
                                                                   force, err)));
}

void launch_push(hipStream_t s, const Geo &g, const Pot &P, const PartPtrs &pp, const float *force,
                 uint32_t *err) {
  if (pp.n <= 0) return;
  PIC_DISPATCH(g.ndim, (k_push<ND><<<nblocks(pp.n), 256, 0, s>>>(g, P, pp.n, pp.cell, pp.off, pp.vel,
                                                                  force, err)));
}

void launch_kick(hipStream_t s, const Geo &g, const Pot &P, const PartPtrs &pp, const float *force,
                 float frac) {
  if (pp.n <= 0) return;
  PIC_DISPATCH(g.ndim, (k_kick<ND><<<nblocks(pp.n), 256, 0, s>>>(P, pp.n, pp.vel, force, frac)));
}

int launch_force_push(hipStream_t s, const Geo &g, const Pot &P, const DiagC &dc, const PartPtrs &pp,
                      const float *dens, const float *G, double *partial, bool diag, uint32_t *err) {
  if (pp.n <= 0) return 0;
  unsigned nb = nblocks(pp.n);
  if (diag)
    PIC_DISPATCH(g.ndim, (k_force_push<ND, true><<<nb, 256, 0, s>>>(g, P, dc, pp.n, pp.cell, pp.off, pp.vel,
                                                                     pp.wq, dens, G, partial, err)));
  else
    PIC_DISPATCH(g.ndim, (k_force_push<ND, false><<<nb, 256, 0, s>>>(g, P, dc, pp.n, pp.cell, pp.off,
                                                                      pp.vel, pp.wq, dens, G, partial, err)));
  return (int)nb;
}

int launch_pe_nodes(hipStream_t s, const Geo &g, const DiagC &dc, const Quad16 &q, const long long *node,
                    double *partial) {
  unsigned nb = nblocks(g.nnodes);
  PIC_DISPATCH(g.ndim, (k_pe_nodes<ND><<<nb, 256, 0, s>>>(g, dc, q, node, partial)));
  return (int)nb;
}

void launch_reduce_diag(hipStream_t s, const double *part_p, int nblk_p, const double *part_g, int nblk_g,
                        pic_diag_t *out, int64_t step) {
  k_reduce_diag<<<1, 256, 0, s>>>(part_p, nblk_p, part_g, nblk_g, out, step);
}

}  // namespace pic
