// Device-side building blocks of the PIC pair-potential cycle (arXiv 1502.07722)
// for gfx950.  Every kernel -- the separate deposit / force / push kernels and
// the fused step kernels -- evaluates the method through these functions, so
// that all paths produce the same bits.  The library is compiled with
// -ffp-contract=off: every fused multiply-add below is written explicitly.
//
// Reduced units inside the kernels: density nh = n r0^3, gradient Gh = dn/dx
// r0^4, force Fh in units of 12 D / r0.  Positions are (cell, offset in [0,1)).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

enum : uint32_t { ERR_RANGE = 1u, ERR_CFL = 2u, ERR_WEIGHT = 4u };

// Grid constants as the kernels need them.
struct Geo {
  int ndim;
  int n[3];        // cells per axis
  int nn[3];       // nodes per axis
  int bc[3];       // 0 periodic, 1 reflecting
  int ncells;
  int nnodes;
  double inv_n0;   // 1 / n[0], for decoding linear cell ids
  double inv_n1;   // 1 / n[1]
  float kappa;     // 2^-20 r0^3 / V_cell: weight units -> reduced density
  float gam[3];    // r0 / (2^(ndim-1) h_d): summed edge differences -> gradient
  float tau[3];    // dt / h_d: velocity (m/s) -> offset change per step
};

// Potential constants (reduced units) and the force / velocity scales.
struct Pot {
  float nfloor;    // n_floor r0^3
  float gclamp;
  float hgclamp;   // gclamp / 2
  float s_rep;
  float c_att;
  float beta;      // 12 D / r0: reduced force -> newtons
  float gv;        // dt / m: newtons -> velocity change per step
  int kind;        // pair potential: 0 Lennard-Jones eq. (3), 1 Morse
  float mAl2;      // Morse: alpha r0 log2(e)
  float mA6;       // Morse: alpha r0 / 6
  float mAt;       // Morse: 6 mA6^2 = (alpha r0)^2 / 6
  int lattice;     // 0 cubic (eqs. (1)-(2) per axis), 1 hexagonal close-packed
  float ks;        // reverse mode only: scale of the force cotangent of the
                   // step's kick (1; 1 + f when the step also reverses a start
                   // kick v(-1/2) = v(0) + f F(x0) dt / m of the same state)
};

// ---------------------------------------------------------------------------
// Cell ids
// ---------------------------------------------------------------------------
__device__ __forceinline__ int div_floor_pos(int c, int n, double inv) {
  // c >= 0; exact floor(c / n) from a double estimate plus one correction
  int q = (int)((double)c * inv);
  int r = c - q * n;
  if (r < 0) q -= 1;
  else if (r >= n) q += 1;
  return q;
}

template <int ND>
__device__ __forceinline__ void decode_cell(const Geo &g, int c, int idx[3]) {
  int q = div_floor_pos(c, g.n[0], g.inv_n0);
  idx[0] = c - q * g.n[0];
  if (ND == 2) {
    idx[1] = q;
    idx[2] = 0;
  } else {
    int q2 = div_floor_pos(q, g.n[1], g.inv_n1);
    idx[1] = q - q2 * g.n[1];
    idx[2] = q2;
  }
}

template <int ND>
__device__ __forceinline__ int encode_cell(const Geo &g, const int idx[3]) {
  return ND == 2 ? idx[0] + g.n[0] * idx[1] : idx[0] + g.n[0] * (idx[1] + g.n[1] * idx[2]);
}

// Stored node along axis d for node coordinate a in [0, n_d]: periodic axes wrap
// n_d -> 0 (deposit / gather never need other ghosts).
__device__ __forceinline__ int node_axis(const Geo &g, int d, int a) {
  return (!g.bc[d] && a == g.n[d]) ? 0 : a;
}

template <int ND>
__device__ __forceinline__ int node_index(const Geo &g, int a0, int a1, int a2) {
  return ND == 2 ? a0 + g.nn[0] * a1 : a0 + g.nn[0] * (a1 + g.nn[1] * a2);
}

// Node weight sum as a float: through double, where the sum of the two
// 32-bit halves is exact below 2^53, so the value is rounded once (and every
// path converts node sums here, so they all agree beyond that too).
__device__ __forceinline__ float wsum_float(long long wsum) { return (float)(double)wsum; }

// Reduced density of a stored node: weight sum * kappa, doubled for each
// reflecting wall the node lies on (half volume there).
__device__ __forceinline__ float node_density(const Geo &g, long long wsum, int a0, int a1, int a2) {
  float k = g.kappa;
  if (g.bc[0] && (a0 == 0 || a0 == g.n[0])) k *= 2.0f;
  if (g.bc[1] && (a1 == 0 || a1 == g.n[1])) k *= 2.0f;
  if (g.ndim == 3 && g.bc[2] && (a2 == 0 || a2 == g.n[2])) k *= 2.0f;
  return wsum_float(wsum) * k;
}

// ---------------------------------------------------------------------------
// Fixed-point deposit: offsets quantised to 16 bits, weight split axis by axis,
// upper node gets floor(part * u / 2^16), the lower node the rest.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t quant16(float f) {
  int u = (int)(f * 65536.0f);  // exact scaling; truncation = floor for f >= 0
  return (uint32_t)min(max(u, 0), 65535);
}

// floor(part * u / 2^16) for part < 2^31, u < 2^16, from two 16 x 16-bit
// products (full-rate 24-bit multiplies): part * u = ph u 2^16 + pl u, and the
// first term is a multiple of 2^16, so the floor splits exactly.
__device__ __forceinline__ uint32_t split_upper(uint32_t part, uint32_t u) {
  const uint32_t ph = part >> 16, pl = part & 0xffffu;
  const uint32_t hi = (uint32_t)__umul24(ph, u);  // < 2^31
  const uint32_t lo = (uint32_t)__umul24(pl, u);  // < 2^32: unsigned before the shift
  return hi + (lo >> 16);
}

// Shares of the 2^ND corner nodes; corner bit d set = upper node along d.
template <int ND>
__device__ __forceinline__ void deposit_shares(uint32_t W, const float f[3], uint32_t t[8]) {
  uint32_t ux = quant16(f[0]), uy = quant16(f[1]);
  uint32_t x1 = split_upper(W, ux), x0 = W - x1;
  uint32_t t01 = split_upper(x0, uy), t11 = split_upper(x1, uy);
  uint32_t t00 = x0 - t01, t10 = x1 - t11;
  if (ND == 2) {
    t[0] = t00; t[1] = t10; t[2] = t01; t[3] = t11;
  } else {
    uint32_t uz = quant16(f[2]);
    uint32_t a = split_upper(t00, uz), b = split_upper(t10, uz);
    uint32_t c = split_upper(t01, uz), d = split_upper(t11, uz);
    t[0] = t00 - a; t[1] = t10 - b; t[2] = t01 - c; t[3] = t11 - d;
    t[4] = a; t[5] = b; t[6] = c; t[7] = d;
  }
}

// ---------------------------------------------------------------------------
// Cell-centred gradient from the cell's 2^ND corner densities (corner bit d =
// upper along d): mean of the edge differences along d, in reduced units.
// ---------------------------------------------------------------------------
template <int ND>
__device__ __forceinline__ void centre_gradient(const Geo &g, const float c[8], float G[3]) {
  if (ND == 2) {
    G[0] = g.gam[0] * ((c[1] - c[0]) + (c[3] - c[2]));
    G[1] = g.gam[1] * ((c[2] - c[0]) + (c[3] - c[1]));
    G[2] = 0.0f;
  } else {
    G[0] = g.gam[0] * (((c[1] - c[0]) + (c[3] - c[2])) + ((c[5] - c[4]) + (c[7] - c[6])));
    G[1] = g.gam[1] * (((c[2] - c[0]) + (c[3] - c[1])) + ((c[6] - c[4]) + (c[7] - c[5])));
    G[2] = g.gam[2] * (((c[4] - c[0]) + (c[5] - c[1])) + ((c[6] - c[2]) + (c[7] - c[3])));
  }
}

__device__ __forceinline__ float lerpf(float a, float b, float t) { return __builtin_fmaf(t, b - a, a); }

// Multilinear interpolation of 2^ND corner values (corner bit d = upper along d).
template <int ND>
__device__ __forceinline__ float interp(const float c[8], const float w[3]) {
  float a = lerpf(c[0], c[1], w[0]);
  float b = lerpf(c[2], c[3], w[0]);
  float lo = lerpf(a, b, w[1]);
  if (ND == 2) return lo;
  float e = lerpf(c[4], c[5], w[0]);
  float f = lerpf(c[6], c[7], w[0]);
  return lerpf(lo, lerpf(e, f, w[1]), w[2]);
}

// Centre-interpolation base and weight along one axis: the two nearest centres
// are at (c0 + 1/2) and (c0 + 3/2) with weight t on the upper one.
__device__ __forceinline__ void centre_stencil(int i, float f, int &c0, float &t) {
  if (f >= 0.5f) { c0 = i; t = f - 0.5f; }
  else { c0 = i - 1; t = f + 0.5f; }
}

// ---------------------------------------------------------------------------
// Eq. (1)-(3).  q = n^(1/3) = r0 / rbar;  g = d rbar/dx = -(1/3) Gh / (nh q);
// s+- = r0 / r+- = q (1 -+ g/2);  phi'(s) = (12 D / r0) M(s) (s^7 - s^13),
// M = s_rep for r < r0 (s > 1), c_att otherwise;  F = phi'(s+) - phi'(s-).
// ---------------------------------------------------------------------------
// Morse in the same units: r / r0 = 1/s, e = exp(-alpha r0 (1/s - 1)),
// U'(r) / (12 D / r0) = (alpha r0 / 6) e (1 - e), U / D = e (e - 2).  GEN
// false compiles the Lennard-Jones cubic path alone (the kernels' default
// instantiation); GEN true adds the runtime choice of potential and lattice
// (kernel arguments, so the branches are uniform across the wavefront).
__device__ __forceinline__ float morse_e(const Pot &P, float s) {
  return __builtin_amdgcn_exp2f(__builtin_fmaf(-P.mAl2, __builtin_amdgcn_rcpf(s), P.mAl2));
}

// phi'(s) / (12 D / r0) as the branch factor M (s_rep for s > 1, c_att
// otherwise), returned, times the shape v.
template <bool GEN = false>
__device__ __forceinline__ float dphi_split(const Pot &P, float s, float &v) {
  if (GEN && P.kind == 1) {
    const float e = morse_e(P, s);
    v = P.mA6 * __builtin_fmaf(-e, e, e);  // (alpha r0 / 6) (e - e^2)
  } else {
    float s2 = s * s;
    float s3 = s2 * s;
    float s6 = s3 * s3;
    float s7 = s6 * s;
    v = __builtin_fmaf(-s7, s6, s7);  // s^7 - s^13
  }
  return s > 1.0f ? P.s_rep : P.c_att;
}

template <bool GEN = false>
__device__ __forceinline__ float dphi_hat(const Pot &P, float s) {
  float v;
  const float M = dphi_split<GEN>(P, s, v);
  return M * v;
}

template <bool GEN = false>
__device__ __forceinline__ float phi_hat(const Pot &P, float s) {
  // U / D; altered branches stay continuous at r0
  float u;
  if (GEN && P.kind == 1) {
    const float e = morse_e(P, s);
    u = e * (e - 2.0f);
  } else {
    float s6 = s * s * s;
    s6 = s6 * s6;
    u = __builtin_fmaf(s6, s6, -2.0f * s6);  // s^12 - 2 s^6
  }
  return s > 1.0f ? __builtin_fmaf(P.s_rep, u, P.s_rep - P.c_att) : P.c_att * u;
}


// The 12 neighbours in grid axes: 3D (basal 1, basal 2, c) = (x, y, z); 2D
// (basal 1, c) = (x, y), the basal-2 axis unresolved, so neighbours that
// differ only there merge (weights 2) and their out-of-plane forces cancel.
// Rows: v0, v1, v2, weight.  The loop over the table is unrolled: the
// kernels that carry this path are instantiations of their own (the general
// potential / lattice switch), and the 2D step still fits the item loop's
// occupancy (72 VGPRs, 7 waves per SIMD).
static __constant__ float kHcp3[12][4] = {
    {1.0f, 0.0f, 0.0f, 1.0f},
    {0.5f, 0.866025403784439f, 0.0f, 1.0f},
    {-0.5f, 0.866025403784439f, 0.0f, 1.0f},
    {-1.0f, 0.0f, 0.0f, 1.0f},
    {-0.5f, -0.866025403784439f, 0.0f, 1.0f},
    {0.5f, -0.866025403784439f, 0.0f, 1.0f},
    {0.5f, 0.288675134594813f, 0.816496580927726f, 1.0f},
    {-0.5f, 0.288675134594813f, 0.816496580927726f, 1.0f},
    {0.0f, -0.577350269189626f, 0.816496580927726f, 1.0f},
    {0.5f, 0.288675134594813f, -0.816496580927726f, 1.0f},
    {-0.5f, 0.288675134594813f, -0.816496580927726f, 1.0f},
    {0.0f, -0.577350269189626f, -0.816496580927726f, 1.0f}};
static __constant__ float kHcp2[10][4] = {
    {1.0f, 0.0f, 0.0f, 1.0f},  {-1.0f, 0.0f, 0.0f, 1.0f},
    {0.5f, 0.0f, 0.0f, 2.0f},  {-0.5f, 0.0f, 0.0f, 2.0f},
    {0.5f, 0.816496580927726f, 0.0f, 1.0f},   {-0.5f, 0.816496580927726f, 0.0f, 1.0f},
    {0.0f, 0.816496580927726f, 0.0f, 1.0f},   {0.5f, -0.816496580927726f, 0.0f, 1.0f},
    {-0.5f, -0.816496580927726f, 0.0f, 1.0f}, {0.0f, -0.816496580927726f, 0.0f, 1.0f}};

// Hexagonal close-packed neighbour k along grid direction v (weight w: the
// number of the 12 neighbours with this in-plane direction): q_k = c g.v with
// c = 2^(1/6), clamped; s = r0 / d = (q / c) (1 - q_k / 2).
template <int ND>
__device__ __forceinline__ void hcp_force(const Pot &P, float q, const float g[3], float F[3], float &e, bool bond) {
  const float qc = q * 0.890898718140339f;  // q / 2^(1/6)
  // The neighbours come in pairs that share most of their arithmetic: v and
  // -v (2D, and the basal plane in 3D), whose projections are opposite and
  // whose forces add as (f+ - f-) v; and, out of the 3D basal plane, mirror
  // images (v0, v1, +-v2), which share g0 v0 + g1 v1 and add as
  // ((f+ + f-) v0, (f+ + f-) v1, (f+ - f-) v2).  The first rows of the pairs:
  // 3D 0, 1, 2 (partners 3, 4, 5: -v), 6, 7, 8 (partners 9, 10, 11: mirror);
  // 2D 0, 2, 4, 5, 6 (partners 1, 3, 8, 7, 9: -v).
  const int npairs = ND == 3 ? 6 : 5;
#pragma unroll
  for (int k = 0; k < npairs; ++k) {
    const float *v = ND == 3 ? kHcp3[k < 3 ? k : k + 3] : kHcp2[k < 2 ? 2 * k : k + 2];
    const float w = v[3];
    const bool mirror = ND == 3 && k >= 3;  // v2 != 0: the partner is (v0, v1, -v2)
    const float a = g[0] * v[0] + g[1] * v[1];
    const float c = ND == 3 ? g[2] * v[2] : 0.0f;
    const float gp = mirror ? a + c : a, gm = mirror ? a - c : -a;
    const float qp = fminf(fmaxf(1.12246204831f * gp, -P.gclamp), P.gclamp);
    const float qm = fminf(fmaxf(1.12246204831f * gm, -P.gclamp), P.gclamp);
    const float sp = qc * __builtin_fmaf(-0.5f, qp, 1.0f), sm = qc * __builtin_fmaf(-0.5f, qm, 1.0f);
    const float fp = w * dphi_hat<true>(P, sp), fm = w * dphi_hat<true>(P, sm);
    if (mirror) {
      const float fs = fp + fm;
      F[0] = __builtin_fmaf(fs, v[0], F[0]);
      F[1] = __builtin_fmaf(fs, v[1], F[1]);
      F[2] = __builtin_fmaf(fp - fm, v[2], F[2]);
    } else {
      const float fd = fp - fm;
      F[0] = __builtin_fmaf(fd, v[0], F[0]);
      F[1] = __builtin_fmaf(fd, v[1], F[1]);
    }
    if (bond) e = __builtin_fmaf(0.5f * w, phi_hat<true>(P, sp) + phi_hat<true>(P, sm), e);
  }
}

template <int ND, bool GEN = false>
__device__ __forceinline__ void pair_force(const Pot &P, float nh, const float G[3], float F[3],
                                           float *bond = nullptr) {
  F[0] = F[1] = F[2] = 0.0f;
  if (bond) *bond = 0.0f;
  if (!(nh > P.nfloor)) return;
  float q = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(nh) * (1.0f / 3.0f));
  if (GEN && P.lattice == 1) {
    const float rinv = __builtin_amdgcn_rcpf(nh * q);
    float g[3] = {0.0f, 0.0f, 0.0f}, e = 0.0f;
#pragma unroll
    for (int d = 0; d < ND; ++d) g[d] = (G[d] * rinv) * (-1.0f / 3.0f);
    hcp_force<ND>(P, q, g, F, e, bond != nullptr);
    if (bond) *bond = e;
    return;
  }
  // s+- = q (1 -+ g/2) with g = -(1/3) Gh / (nh q):  q g / 2 = -Gh / (6 nh),
  // and |g| <= gclamp is |q g / 2| <= q gclamp / 2
  const float rn6 = __builtin_amdgcn_rcpf(nh) * (-1.0f / 6.0f);
  const float hc = q * P.hgclamp;
  float e = 0.0f;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const float hq = fminf(fmaxf(G[d] * rn6, -hc), hc);
    const float sp = q - hq;  // +d neighbour (farther when rbar grows towards +d)
    const float sm = q + hq;  // -d neighbour
    float vp, vm;
    const float Mp = dphi_split<GEN>(P, sp, vp), Mm = dphi_split<GEN>(P, sm, vm);
    F[d] = __builtin_fmaf(Mp, vp, -(Mm * vm));
    if (bond) e += 0.5f * (phi_hat<GEN>(P, sp) + phi_hat<GEN>(P, sm));
  }
  if (bond) *bond = e;
}

// ---------------------------------------------------------------------------
// Leapfrog push of one particle (kick with the force in newtons, then drift,
// carry, wrap / mirror).  Returns device error bits.
// ---------------------------------------------------------------------------
// INTERIOR: the caller guarantees the particle is at least one cell away from
// every wall and from the periodic seam, so no mirror or wrap can occur; the
// carry arithmetic is the same, so both variants give the same bits.  edges
// (uniform across the wavefront): bit d clear = the same guarantee along axis
// d alone, whose wall and wrap code is then skipped.
template <int ND, bool INTERIOR = false>
__device__ __forceinline__ uint32_t push_particle(const Geo &g, const Pot &P, const float F[3],
                                                  int idx[3], float f[3], float v[3], uint32_t edges = 7u) {
  uint32_t err = 0;
#pragma unroll
  for (int d = 0; d < ND; ++d) v[d] = __builtin_fmaf(F[d], P.gv, v[d]);
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    float df = v[d] * g.tau[d];
    const bool cfl = !(fabsf(df) < 1.0f);
    err |= cfl ? ERR_CFL : 0u;
    df = cfl ? 0.0f : df;
    const float x = f[d] + df;  // in (-1, 2)
    // carry one cell: x - floor(x) is exact on [0, 2); on (-1, 0) it is x + 1,
    // which a tiny negative x rounds up to 1: that is the node itself
    const float fl = floorf(x);
    float xc = x - fl;
    int ic = idx[d] + (int)fl;
    const bool tie = xc >= 1.0f;
    xc = tie ? 0.0f : xc;
    ic = tie ? idx[d] : ic;
    float xn = xc;
    if (!INTERIOR && ((edges >> d) & 1u)) {
      const int n = g.n[d];
      const bool up = x >= 1.0f, down = x < 0.0f;
      const bool wall_lo = g.bc[d] && idx[d] == 0 && down;
      const bool wall_hi = g.bc[d] && idx[d] == n - 1 && up;
      if (!g.bc[d]) ic = ic < 0 ? ic + n : (ic >= n ? ic - n : ic);
      // mirror at reflecting walls (2 - x is exact for x in [1, 2))
      float xm = wall_lo ? -x : 2.0f - x;
      xm = (wall_hi && xm >= 1.0f) ? 0x1.fffffep-1f : xm;  // exactly on the top wall
      const bool wall = wall_lo || wall_hi;
      xn = wall ? xm : xc;
      ic = wall ? idx[d] : ic;
      v[d] = wall ? -v[d] : v[d];
    }
    idx[d] = ic;
    // xn is never -0 (x - x is +0), so one unsigned compare tests [0, 1) and NaN
    const bool bad = __float_as_uint(xn) >= 0x3f800000u;
    err |= bad ? ERR_RANGE : 0u;
    f[d] = bad ? 0.0f : xn;
  }
  return err;
}

// ---------------------------------------------------------------------------
// FP64 block reduction of NF values (wave64 shuffles, then LDS across waves)
// ---------------------------------------------------------------------------
template <int NF>
__device__ __forceinline__ void block_reduce_store(double v[NF], double *__restrict__ out) {
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
    out[threadIdx.x] = s;
  }
}

}  // namespace pic
