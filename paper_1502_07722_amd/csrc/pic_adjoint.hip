// Reverse mode of the PIC pair-potential cycle (arXiv 1502.07722, Sec. 2):
// hand-written adjoints of deposit -> density/gradient -> gather -> eq. (1)-(3)
// -> leapfrog push, on caller arrays (one thread per particle).
//
// Cotangents carried per particle: lam_x = dJ/d(offset) per axis (per cell of
// displacement) and lam_v = dJ/dv (s/m).  Per node: nbar = dJ/d(n r0^3), the
// cotangent of the reduced node density.  Per cell centre (scratch): Gbar =
// dJ/d(dn/dx r0^4).  Parameters theta = (D, r0, s_rep, c_att).
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

namespace pic {

// ---------------------------------------------------------------------------
// Derivative helpers
// ---------------------------------------------------------------------------
// d/dw_e of the multilinear interpolation interp<ND>(c, w).
template <int ND>
__device__ __forceinline__ void interp_grad(const float c[8], const float w[3], float dv[3]) {
  const float d01 = c[1] - c[0], d23 = c[3] - c[2];
  const float a = lerpf(c[0], c[1], w[0]), b = lerpf(c[2], c[3], w[0]);
  if (ND == 2) {
    dv[0] = lerpf(d01, d23, w[1]);
    dv[1] = b - a;
    dv[2] = 0.0f;
  } else {
    const float d45 = c[5] - c[4], d67 = c[7] - c[6];
    const float e = lerpf(c[4], c[5], w[0]), f = lerpf(c[6], c[7], w[0]);
    dv[0] = lerpf(lerpf(d01, d23, w[1]), lerpf(d45, d67, w[1]), w[2]);
    dv[1] = lerpf(b - a, f - e, w[2]);
    dv[2] = lerpf(e, f, w[1]) - lerpf(a, b, w[1]);
  }
}

// Corner weights of the multilinear interpolation (corner bit d = upper along d).
template <int ND>
__device__ __forceinline__ void corner_weights(const float w[3], float S[8]) {
#pragma unroll
  for (int k = 0; k < (1 << ND); ++k) {
    float s = (k & 1) ? w[0] : 1.0f - w[0];
    s *= ((k >> 1) & 1) ? w[1] : 1.0f - w[1];
    if (ND == 3) s *= ((k >> 2) & 1) ? w[2] : 1.0f - w[2];
    S[k] = s;
  }
}

// Stored cell and sign of the (possibly ghost) centre m for component d:
// periodic axes wrap, reflecting axes mirror and negate the normal part.
template <int ND>
__device__ __forceinline__ int centre_ref(const Geo &g, int d, int m0, int m1, int m2, float &sign) {
  int m[3] = {m0, m1, m2};
  sign = 1.0f;
#pragma unroll
  for (int e = 0; e < ND; ++e) {
    if (m[e] < 0) {
      if (g.bc[e]) { m[e] = 0; sign = (e == d) ? -sign : sign; }
      else m[e] += g.n[e];
    } else if (m[e] >= g.n[e]) {
      if (g.bc[e]) { m[e] = g.n[e] - 1; sign = (e == d) ? -sign : sign; }
      else m[e] -= g.n[e];
    }
  }
  return encode_cell<ND>(g, m);
}

template <int ND>
__device__ __forceinline__ int corner_node(const Geo &g, const int idx[3], int k, float &kfac) {
  const int a0 = node_axis(g, 0, idx[0] + (k & 1));
  const int a1 = node_axis(g, 1, idx[1] + ((k >> 1) & 1));
  const int a2 = ND == 3 ? node_axis(g, 2, idx[2] + ((k >> 2) & 1)) : 0;
  kfac = node_density(g, 1ll, a0, a1, a2);  // kappa, doubled per wall
  return node_index<ND>(g, a0, a1, a2);
}

// Eq. (1)-(3) reversed.  mu: cotangent of the reduced force Fh per axis.
// Returns the cotangents of the gathered reduced density (an) and gradient
// (aG), and adds the parameter terms: th[0] = sum mu Fh (-> dJ/dD = th0 / D),
// th[1] = sum mu (s dFh/ds - Fh) (-> dJ/dr0 = th1 / r0), th[2] = dJ/ds_rep,
// th[3] = dJ/dc_att.  The clamp of g and the density floor have zero
// derivative where they act.
template <int ND>
__device__ __forceinline__ void pair_force_vjp(const Pot &P, float nh, const float G[3], const float mu[3],
                                               float &an, float aG[3], float th[4]) {
  an = 0.0f;
  aG[0] = aG[1] = aG[2] = 0.0f;
  if (!(nh > P.nfloor)) return;
  const float q = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(nh) * (1.0f / 3.0f));
  const float rinv = __builtin_amdgcn_rcpf(nh * q);
  const float inv_n = __builtin_amdgcn_rcpf(nh);
  const float dqdn = q * inv_n * (1.0f / 3.0f);
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const float graw = (G[d] * rinv) * (-1.0f / 3.0f);
    const float g = fminf(fmaxf(graw, -P.gclamp), P.gclamp);
    const bool free_g = graw > -P.gclamp && graw < P.gclamp;
    const float hq = 0.5f * q * g;
    const float sp = q - hq, sm = q + hq;
    float k_p, dk_p, k_m, dk_m;
    {
      const float s2 = sp * sp, s6 = s2 * s2 * s2, s7 = s6 * sp, s12 = s6 * s6;
      k_p = __builtin_fmaf(-s7, s6, s7);
      dk_p = __builtin_fmaf(-13.0f, s12, 7.0f * s6);
    }
    {
      const float s2 = sm * sm, s6 = s2 * s2 * s2, s7 = s6 * sm, s12 = s6 * s6;
      k_m = __builtin_fmaf(-s7, s6, s7);
      dk_m = __builtin_fmaf(-13.0f, s12, 7.0f * s6);
    }
    const bool rp = sp > 1.0f, rm = sm > 1.0f;  // repulsive branch (r < r0)
    const float Mp = rp ? P.s_rep : P.c_att, Mm = rm ? P.s_rep : P.c_att;
    const float A = Mp * dk_p, B = Mm * dk_m;
    const float Fh = Mp * k_p - Mm * k_m;
    const float dFdq = A * (1.0f - 0.5f * g) - B * (1.0f + 0.5f * g);
    const float dFdg = -0.5f * q * (A + B);
    const float dgdn = free_g ? (-4.0f / 3.0f) * g * inv_n : 0.0f;
    const float dgdG = free_g ? (-1.0f / 3.0f) * rinv : 0.0f;
    const float m = mu[d];
    an += m * (dFdq * dqdn + dFdg * dgdn);
    aG[d] = m * dFdg * dgdG;
    th[0] += m * Fh;
    th[1] += m * (A * sp - B * sm - Fh);
    th[2] += m * ((rp ? k_p : 0.0f) - (rm ? k_m : 0.0f));
    th[3] += m * ((rp ? 0.0f : k_p) - (rm ? 0.0f : k_m));
  }
}

// Gather of n and G at (idx, f) with the corner values kept for the VJP.
template <int ND>
struct GatherState {
  float cr[8];      // node densities at the cell corners
  float vv[3][8];   // centre values per component
  int cidx[8];      // stored cell of each stencil centre
  float csign[3][8];
  float t[3];       // centre-stencil weights
  int c0[3];
  float nh, Gp[3];
};

template <int ND>
__device__ __forceinline__ void gather_for_vjp(const Geo &g, const float *__restrict__ dens,
                                               const float *__restrict__ G, const int idx[3], const float f[3],
                                               GatherState<ND> &s) {
  const int x1 = node_axis(g, 0, idx[0] + 1), y1 = node_axis(g, 1, idx[1] + 1);
  if (ND == 2) {
    s.cr[0] = dens[node_index<2>(g, idx[0], idx[1], 0)];
    s.cr[1] = dens[node_index<2>(g, x1, idx[1], 0)];
    s.cr[2] = dens[node_index<2>(g, idx[0], y1, 0)];
    s.cr[3] = dens[node_index<2>(g, x1, y1, 0)];
  } else {
    const int z1 = node_axis(g, 2, idx[2] + 1);
    s.cr[0] = dens[node_index<3>(g, idx[0], idx[1], idx[2])];
    s.cr[1] = dens[node_index<3>(g, x1, idx[1], idx[2])];
    s.cr[2] = dens[node_index<3>(g, idx[0], y1, idx[2])];
    s.cr[3] = dens[node_index<3>(g, x1, y1, idx[2])];
    s.cr[4] = dens[node_index<3>(g, idx[0], idx[1], z1)];
    s.cr[5] = dens[node_index<3>(g, x1, idx[1], z1)];
    s.cr[6] = dens[node_index<3>(g, idx[0], y1, z1)];
    s.cr[7] = dens[node_index<3>(g, x1, y1, z1)];
  }
  s.nh = interp<ND>(s.cr, f);
  s.c0[2] = 0;
  s.t[2] = 0.0f;
#pragma unroll
  for (int e = 0; e < ND; ++e) centre_stencil(idx[e], f[e], s.c0[e], s.t[e]);
  s.Gp[2] = 0.0f;
#pragma unroll
  for (int k = 0; k < (1 << ND); ++k) {
    const int m0 = s.c0[0] + (k & 1), m1 = s.c0[1] + ((k >> 1) & 1), m2 = ND == 3 ? s.c0[2] + ((k >> 2) & 1) : 0;
    float sg;
    s.cidx[k] = centre_ref<ND>(g, 0, m0, m1, m2, sg);
    s.csign[0][k] = sg;
#pragma unroll
    for (int d = 1; d < ND; ++d) {
      (void)centre_ref<ND>(g, d, m0, m1, m2, sg);
      s.csign[d][k] = sg;
    }
#pragma unroll
    for (int d = 0; d < ND; ++d) s.vv[d][k] = s.csign[d][k] * G[(int64_t)d * g.ncells + s.cidx[k]];
  }
#pragma unroll
  for (int d = 0; d < ND; ++d) s.Gp[d] = interp<ND>(s.vv[d], s.t);
}

// Direct position term and scatters of the gather VJP.
template <int ND>
__device__ __forceinline__ void gather_vjp(const Geo &g, const int idx[3], const float f[3], const GatherState<ND> &s,
                                           float an, const float aG[3], float lf[3], float *__restrict__ nbar,
                                           float *__restrict__ Gbar) {
  float dn[3];
  interp_grad<ND>(s.cr, f, dn);
#pragma unroll
  for (int e = 0; e < ND; ++e) lf[e] = __builtin_fmaf(an, dn[e], lf[e]);
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    float dg[3];
    interp_grad<ND>(s.vv[d], s.t, dg);
#pragma unroll
    for (int e = 0; e < ND; ++e) lf[e] = __builtin_fmaf(aG[d], dg[e], lf[e]);
  }
  float S[8];
  if (an != 0.0f) {
    corner_weights<ND>(f, S);
#pragma unroll
    for (int k = 0; k < (1 << ND); ++k) {
      float kf;
      const int node = corner_node<ND>(g, idx, k, kf);
      atomicAdd(&nbar[node], an * S[k]);
    }
  }
  corner_weights<ND>(s.t, S);
#pragma unroll
  for (int d = 0; d < ND; ++d)
    if (aG[d] != 0.0f)
#pragma unroll
      for (int k = 0; k < (1 << ND); ++k)
        atomicAdd(&Gbar[(int64_t)d * g.ncells + s.cidx[k]], aG[d] * S[k] * s.csign[d][k]);
}

// Deposit term: lam_x += W sum_k kfac_k nbar_k dS_k/dx at (idx, f).
template <int ND>
__device__ __forceinline__ void deposit_term(const Geo &g, const float *__restrict__ nbar, const int idx[3],
                                             const float f[3], int W, float lf[3]) {
  float c[8];
#pragma unroll
  for (int k = 0; k < (1 << ND); ++k) {
    float kf;
    const int node = corner_node<ND>(g, idx, k, kf);
    c[k] = kf * nbar[node];
  }
  float dd[3];
  interp_grad<ND>(c, f, dd);
  const float w = (float)W;
#pragma unroll
  for (int e = 0; e < ND; ++e) lf[e] = __builtin_fmaf(w, dd[e], lf[e]);
}

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
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double thd[4] = {0, 0, 0, 0};
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
        float v[3] = {vel[p], vel[n + p], vel[2 * n + p]};
        float Fh[3];
        pair_force<ND>(P, gs.nh, gs.Gp, Fh);
        const float F[3] = {Fh[0] * P.beta, Fh[1] * P.beta, ND == 3 ? Fh[2] * P.beta : 0.0f};
        float vpre[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) vpre[d] = d < ND ? __builtin_fmaf(F[d], P.gv, v[d]) : v[d];
        int idx2[3] = {idx[0], idx[1], idx[2]};
        float f2[3] = {f[0], f[1], f[2]}, v2[3] = {v[0], v[1], v[2]};
        e = push_particle<ND>(g, P, F, idx2, f2, v2);
        if (e) atomicOr(err, e);
        float ln[3] = {lam_x[p], lam_x[n + p], ND == 3 ? lam_x[2 * n + p] : 0.0f};
        if (nbar_next) deposit_term<ND>(g, nbar_next, idx2, f2, wq[p], ln);
        float lv[3] = {lam_v[p], lam_v[n + p], lam_v[2 * n + p]};
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          const float s = (v2[d] == vpre[d]) ? 1.0f : -1.0f;  // mirrored at a wall
          lv[d] = s * __builtin_fmaf(g.tau[d], ln[d], lv[d]);
          lf[d] = s * ln[d];
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) lam_v[(int64_t)d * n + p] = lv[d];
#pragma unroll
        for (int d = 0; d < ND; ++d) mu[d] = (lv[d] * P.gv) * P.beta;
      } else {
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          mu[d] = fbar[(int64_t)d * n + p] * P.beta;
          lf[d] = lam_x[(int64_t)d * n + p];
        }
      }
      float an, aG[3], th[4] = {0.f, 0.f, 0.f, 0.f};
      pair_force_vjp<ND>(P, gs.nh, gs.Gp, mu, an, aG, th);
      gather_vjp<ND>(g, idx, f, gs, an, aG, lf, nbar, Gbar);
#pragma unroll
      for (int d = 0; d < ND; ++d) lam_x[(int64_t)d * n + p] = lf[d];
#pragma unroll
      for (int i = 0; i < 4; ++i) thd[i] = th[i];
    }
  }
  block_reduce_store<4>(thd, partial + (int64_t)blockIdx.x * 8);
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

// Fixed-order sum of the per-block parameter partials into dtheta (+=).
__global__ void __launch_bounds__(256) k_reduce_theta(const double *__restrict__ partial, int nblocks,
                                                      double s0, double s1, double *__restrict__ dtheta) {
  __shared__ double red[4][256];
  double acc[4] = {0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += partial[(int64_t)b * 8 + i];
#pragma unroll
  for (int i = 0; i < 4; ++i) red[i][threadIdx.x] = acc[i];
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
#pragma unroll
      for (int i = 0; i < 4; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 4) {
    const double scale = threadIdx.x == 0 ? s0 : (threadIdx.x == 1 ? s1 : 1.0);
    dtheta[threadIdx.x] += red[threadIdx.x][0] * scale;
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

void launch_fillf(hipStream_t st, float *a, int64_t n) {
  if (n > 0) hipLaunchKernelGGL(k_fillf, dim3(blocks_for(n)), dim3(256), 0, st, a, n);
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

void launch_reduce_theta(hipStream_t st, const double *partial, int nblocks, double s0, double s1, double *dtheta) {
  hipLaunchKernelGGL(k_reduce_theta, dim3(1), dim3(256), 0, st, partial, nblocks, s0, s1, dtheta);
}

}  // namespace pic
