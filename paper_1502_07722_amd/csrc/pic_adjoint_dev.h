// Device-side building blocks of the reverse mode of the PIC pair-potential
// cycle (arXiv 1502.07722, Sec. 2, eqs. (1)-(3)), shared by the kernels on
// caller arrays and the tiled kernels so that both use the same arithmetic.
//
// Cotangents: lam_x = dJ/d(offset) per axis, lam_v = dJ/dv (s/m), nbar =
// dJ/d(n r0^3) per node, Gbar = dJ/d(dn/dx r0^4) per cell centre.
#pragma once
#include "pic_device.h"

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
// (aG), and adds the parameter terms as logarithmic derivatives of the
// force F = (12 D / r0) Fh taken at fixed physical distances, in units of
// 12 D / r0: th[0] = sum mu Fh (-> dJ/dD = th0 / D), th[1] = sum mu r0 dF/dr0
// (-> dJ/dr0 = th1 / r0), th[2] = dJ/ds_rep, th[3] = dJ/dc_att, th[4] = sum mu
// alpha dF/dalpha (-> dJ/dalpha = th4 / alpha; Morse only).  The clamp of g
// and the density floor have zero derivative where they act.
//
// Per neighbour, with s = r0 / r and the branch multiplier M fixed, r0 dF/dr0
// = M (s k' + A dk/dA) - Fh.  The Lennard-Jones k = s^7 - s^13 has no A; the
// Morse k = (A/6)(E - E^2), E = exp(A (1 - 1/s)), A = alpha r0: with t =
// (A^2/6)(E - 2E^2), k' = t / s^2, A dk/dA = k + t (1 - 1/s), so s k' +
// A dk/dA = k + t.
// Per-neighbour terms of eq. (3) for the reverse mode: k (reduced U' without
// the branch multiplier), dk = dk/ds, and t = s^2 dk/ds for Morse (zero for
// Lennard-Jones, whose r0 term is s k' - k).
template <bool GEN>
__device__ __forceinline__ void pair_terms(const Pot &P, float s, float &k, float &dk, float &t) {
  if (GEN && P.kind == 1) {
    const float E = morse_e(P, s), is = __builtin_amdgcn_rcpf(s);
    k = P.mA6 * __builtin_fmaf(-E, E, E);
    t = P.mAt * __builtin_fmaf(-2.0f * E, E, E);
    dk = t * is * is;
  } else {
    const float s2 = s * s, s6 = s2 * s2 * s2, s7 = s6 * s, s12 = s6 * s6;
    k = __builtin_fmaf(-s7, s6, s7);
    dk = __builtin_fmaf(-13.0f, s12, 7.0f * s6);
    t = 0.0f;
  }
}

// The hexagonal close-packed force reversed: per neighbour direction v
// (weight w), q_k = clamp(c g.v), s = (q / c)(1 - q_k / 2), F += w phi'(s) v
// (c = 2^(1/6); the clamp has zero derivative where it acts).  Same outputs
// and parameter terms as the cubic case below.  The loop keeps only the sums
// the outputs need (w_m = w mu.v, A = M dk/ds, M the branch multiplier):
//   S = sum w_m A s, E = sum of w_m A v over the unclamped q_k,
//   K_r, K_a = sum w_m k over the repulsive and the attractive branch,
//   T = sum w_m M t (Morse).
// s is linear in q (ds/dq = s / q) and dq/dn = q / (3 n), so the density
// term is S / (3 n); ds/dg = -(q / 2) v on the unclamped directions;
// sum w_m M k = s_rep K_r + c_att K_a; the Lennard-Jones r0 term
// M (s dk - k) sums to S - K; for Morse dk = t / s^2, so the width term
// M (k + t - t / s) sums to K + T - S.
template <int ND>
__device__ __forceinline__ void hcp_force_vjp(const Pot &P, float q, float rinv, float inv_n, const float G[3],
                                              const float mu[3], float &an, float aG[3], float th[5]) {
  const float c6 = 1.12246204831f, qc = q * 0.890898718140339f;  // q / 2^(1/6)
  float g[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int d = 0; d < ND; ++d) g[d] = (G[d] * rinv) * (-1.0f / 3.0f);
  const bool morse = P.kind == 1;
  float S = 0.0f, T = 0.0f, Kr = 0.0f, Ka = 0.0f, E[3] = {0.0f, 0.0f, 0.0f};
  const int n = ND == 3 ? 12 : 10;
#pragma unroll 1
  for (int j = 0; j < n; ++j) {
    const float *v = ND == 3 ? kHcp3[j] : kHcp2[j];
    float gu = g[0] * v[0] + g[1] * v[1], mk = mu[0] * v[0] + mu[1] * v[1];
    if (ND == 3) {
      gu = __builtin_fmaf(g[2], v[2], gu);
      mk = __builtin_fmaf(mu[2], v[2], mk);
    }
    const float cq = c6 * gu;
    const float qk = fminf(fmaxf(cq, -P.gclamp), P.gclamp);
    const bool free_q = cq > -P.gclamp && cq < P.gclamp;
    const float s = qc * __builtin_fmaf(-0.5f, qk, 1.0f);
    float k, dk, t;
    pair_terms<true>(P, s, k, dk, t);
    const bool rep = s > 1.0f;  // repulsive branch (r < r0)
    const float M = rep ? P.s_rep : P.c_att;
    const float wm = v[3] * mk, wA = wm * (M * dk), wk = wm * k;
    S = __builtin_fmaf(wA, s, S);
    const float wAf = free_q ? wA : 0.0f;
#pragma unroll
    for (int d = 0; d < ND; ++d) E[d] = __builtin_fmaf(wAf, v[d], E[d]);
    Kr += rep ? wk : 0.0f;
    Ka += rep ? 0.0f : wk;
    if (morse) T = __builtin_fmaf(wm * M, t, T);
  }
  an = S * inv_n * (1.0f / 3.0f);
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const float dg = (-0.5f * q) * E[d];
    an = __builtin_fmaf(dg, (-4.0f / 3.0f) * g[d] * inv_n, an);
    aG[d] = dg * (-1.0f / 3.0f) * rinv;
  }
  const float K = __builtin_fmaf(P.s_rep, Kr, P.c_att * Ka);
  // every slot takes one unconditional add (a branch between slots would
  // make the caller's array addressable memory)
  th[0] += K;
  th[1] += morse ? T : S - K;
  th[2] += Kr;
  th[3] += Ka;
  th[4] += morse ? (K + T) - S : 0.0f;
}

template <int ND, bool GEN = false>
__device__ __forceinline__ void pair_force_vjp(const Pot &P, float nh, const float G[3], const float mu[3],
                                               float &an, float aG[3], float th[5]) {
  an = 0.0f;
  aG[0] = aG[1] = aG[2] = 0.0f;
  if (!(nh > P.nfloor)) return;
  const bool morse = GEN && P.kind == 1;
  const float q = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(nh) * (1.0f / 3.0f));
  const float rinv = __builtin_amdgcn_rcpf(nh * q);
  const float inv_n = __builtin_amdgcn_rcpf(nh);
  const float dqdn = q * inv_n * (1.0f / 3.0f);
  if (GEN && P.lattice == 1) {
    hcp_force_vjp<ND>(P, q, rinv, inv_n, G, mu, an, aG, th);
    return;
  }
  // the forward's algebra: s+- = q -+ hq with hq = q g / 2 = -Gh / (6 nh),
  // clamped at +-hc, hc = q gclamp / 2.  F(q, hq) = M+ k(s+) - M- k(s-):
  // dF/dq = A - B and dF/dhq = -(A + B) with A = M+ k'(s+), B = M- k'(s-).
  // Free hq: dhq/dnh = -hq / nh, dhq/dGh = -1 / (6 nh); clamped hq = +-hc:
  // dhq/dnh = (hq / q) dq/dnh, dhq/dGh = 0.
  const float rn6 = inv_n * (-1.0f / 6.0f);
  const float hc = q * P.hgclamp;
  const float dqq = inv_n * (1.0f / 3.0f);  // (dq/dnh) / q
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const float hraw = G[d] * rn6;
    const float hq = fminf(fmaxf(hraw, -hc), hc);
    const bool free_h = hraw > -hc && hraw < hc;
    const float sp = q - hq, sm = q + hq;
    float k_p, dk_p, k_m, dk_m, t_p = 0.0f, t_m = 0.0f;
    if (morse) {
      const float Ep = morse_e(P, sp), Em = morse_e(P, sm);
      k_p = P.mA6 * __builtin_fmaf(-Ep, Ep, Ep);
      k_m = P.mA6 * __builtin_fmaf(-Em, Em, Em);
      t_p = P.mAt * __builtin_fmaf(-2.0f * Ep, Ep, Ep);
      t_m = P.mAt * __builtin_fmaf(-2.0f * Em, Em, Em);
      const float ip = __builtin_amdgcn_rcpf(sp), im = __builtin_amdgcn_rcpf(sm);
      dk_p = t_p * ip * ip;
      dk_m = t_m * im * im;
    } else {
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
    }
    const bool rp = sp > 1.0f, rm = sm > 1.0f;  // repulsive branch (r < r0)
    const float Mp = rp ? P.s_rep : P.c_att, Mm = rm ? P.s_rep : P.c_att;
    const float A = Mp * dk_p, B = Mm * dk_m;
    const float Fh = __builtin_fmaf(Mp, k_p, -(Mm * k_m));
    const float ApB = A + B, AmB = A - B;
    const float dhdn = free_h ? -hq * inv_n : hq * dqq;
    const float m = mu[d];
    an = __builtin_fmaf(m, __builtin_fmaf(AmB, dqdn, -(ApB * dhdn)), an);
    aG[d] = free_h ? (m * -ApB) * rn6 : 0.0f;
    th[0] = __builtin_fmaf(m, Fh, th[0]);
    const float Ws = __builtin_fmaf(A, sp, -(B * sm));  // M s dk/ds, + side minus - side
    if (morse) {
      // r0: M (k + t) per side; alpha: M A dk/dA = M (k + t - t / s), t / s = s dk/ds
      const float tpm = Mp * t_p - Mm * t_m;
      th[1] = __builtin_fmaf(m, tpm, th[1]);
      th[4] = __builtin_fmaf(m, (Fh + tpm) - Ws, th[4]);
    } else {
      th[1] = __builtin_fmaf(m, Ws - Fh, th[1]);
    }
    // the repulsive and attractive shares of k+ - k-
    const float krep = (rp ? k_p : 0.0f) - (rm ? k_m : 0.0f);
    th[2] = __builtin_fmaf(m, krep, th[2]);
    th[3] = __builtin_fmaf(m, (k_p - k_m) - krep, th[3]);
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

// The forward step of one particle recomputed from (idx, f, v) with the
// gathered (nh, Gp): same bits as the forward push, and which axes a wall
// mirrored (sign -1).
struct PushRecord {
  int idx2[3];
  float f2[3];
  float sgn[3];
};

// edges: as push_particle's (bit d clear = no wall or wrap within reach along d)
template <int ND, bool GEN = false>
__device__ __forceinline__ uint32_t recompute_push(const Geo &g, const Pot &P, const int idx[3], const float f[3],
                                                   const float v[3], float nh, const float Gp[3], PushRecord &r,
                                                   uint32_t edges = 7u) {
  float Fh[3];
  pair_force<ND, GEN>(P, nh, Gp, Fh);
  const float F[3] = {Fh[0] * P.beta, Fh[1] * P.beta, ND == 3 ? Fh[2] * P.beta : 0.0f};
  float vpre[3], v2[3] = {v[0], v[1], v[2]};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    vpre[d] = d < ND ? __builtin_fmaf(F[d], P.gv, v[d]) : v[d];
    r.idx2[d] = idx[d];
    r.f2[d] = f[d];
  }
  const uint32_t e = push_particle<ND>(g, P, F, r.idx2, r.f2, v2, edges);
#pragma unroll
  for (int d = 0; d < 3; ++d) r.sgn[d] = (d < ND && v2[d] != vpre[d]) ? -1.0f : 1.0f;
  return e;
}

// Reverse drift and kick: ln = complete lam_x(n+1), lv = lam_v(n+1/2) in,
// lam_v(n-1/2) out; lf = position term of lam_x(n); mu = cotangent of the
// reduced force.
template <int ND>
__device__ __forceinline__ void reverse_drift_kick(const Geo &g, const Pot &P, const PushRecord &r, const float ln[3],
                                                   float lv[3], float lf[3], float mu[3]) {
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    lv[d] = r.sgn[d] * __builtin_fmaf(g.tau[d], ln[d], lv[d]);
    lf[d] = r.sgn[d] * ln[d];
    mu[d] = ((lv[d] * P.gv) * P.beta) * P.ks;
  }
}

// Both, with the deposit term of step n+1 taken from the global nbar_next.
template <int ND, bool GEN = false>
__device__ __forceinline__ uint32_t reverse_push(const Geo &g, const Pot &P, const int idx[3], const float f[3],
                                                 const float v[3], int W, float nh, const float Gp[3],
                                                 const float *__restrict__ nbar_next, float ln[3], float lv[3],
                                                 float lf[3], float mu[3]) {
  PushRecord r;
  const uint32_t e = recompute_push<ND, GEN>(g, P, idx, f, v, nh, Gp, r);
  if (nbar_next) deposit_term<ND>(g, nbar_next, r.idx2, r.f2, W, ln);
  reverse_drift_kick<ND>(g, P, r, ln, lv, lf, mu);
  return e;
}

}  // namespace pic
