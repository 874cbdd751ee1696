/*
 * FP64 CPU oracle for the PIC pair-potential cycle (arXiv 1502.07722).
 * TEST INFRASTRUCTURE ONLY -- see pic_oracle.h.  Plain single-threaded loops in
 * SI units; every function follows one step of the paper's cycle in the
 * paper's order.  Readings of points the paper leaves open are marked
 * "reading:".
 */
#include "pic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_WSHIFT 20
static const double ORC_WUNIT = 1.0 / 1048576.0; /* atoms per weight unit, 2^-20 */

/* ------------------------------------------------------------------------- */
/* Grid geometry: cells and nodes (Fig. 1A).  Nodes sit at integer positions; */
/* a periodic axis has n nodes, a reflecting axis n+1 (the walls included).   */
/* ------------------------------------------------------------------------- */

static int nodes_on_axis(const orc_grid *g, int d) { return g->n[d] + (g->bc[d] ? 1 : 0); }

int64_t orc_num_nodes(const orc_grid *g) {
  int64_t t = 1;
  for (int d = 0; d < g->ndim; ++d) t *= nodes_on_axis(g, d);
  return t;
}

int64_t orc_num_cells(const orc_grid *g) {
  int64_t t = 1;
  for (int d = 0; d < g->ndim; ++d) t *= g->n[d];
  return t;
}

static void cell_to_index(const orc_grid *g, int32_t c, int idx[3]) {
  idx[0] = idx[1] = idx[2] = 0;
  int64_t r = c;
  for (int d = 0; d < g->ndim; ++d) {
    idx[d] = (int)(r % g->n[d]);
    r /= g->n[d];
  }
}

static int32_t index_to_cell(const orc_grid *g, const int idx[3]) {
  int64_t c = 0, stride = 1;
  for (int d = 0; d < g->ndim; ++d) {
    c += (int64_t)idx[d] * stride;
    stride *= g->n[d];
  }
  return (int32_t)c;
}

/* Node coordinate along axis d -> stored node: wrap on periodic axes, mirror
 * across the wall on reflecting axes (reading: reflecting walls act as mirrors,
 * so a ghost node beyond a wall equals its mirror image). */
static int node_coord(const orc_grid *g, int d, int i) {
  int n = g->n[d];
  if (!g->bc[d]) {
    i %= n;
    if (i < 0) i += n;
    return i;
  }
  if (i < 0) i = -i;
  if (i > n) i = 2 * n - i;
  return i;
}

static int64_t node_at(const orc_grid *g, const int a[3]) {
  int64_t k = 0, stride = 1;
  for (int d = 0; d < g->ndim; ++d) {
    k += (int64_t)node_coord(g, d, a[d]) * stride;
    stride *= nodes_on_axis(g, d);
  }
  return k;
}

/* Volume a node represents: cell volume, halved for each reflecting wall the
 * node lies on.  2D: the grid stands for a slab of thickness depth2d (the
 * paper treats its 2D targets as unbounded along the third axis). */
static double node_volume(const orc_grid *g, int64_t k) {
  double V = g->h[0] * g->h[1] * (g->ndim == 3 ? g->h[2] : g->depth2d);
  for (int d = 0; d < g->ndim; ++d) {
    int nd = nodes_on_axis(g, d);
    int a = (int)(k % nd);
    k /= nd;
    if (g->bc[d] && (a == 0 || a == g->n[d])) V *= 0.5;
  }
  return V;
}

/* ------------------------------------------------------------------------- */
/* Deposit (method section, Fig. 1A): each macroparticle's weight -- the     */
/* number of atoms it stands for -- is shared among the nodes around it.     */
/* Reading: linear (cloud-in-cell) weights, 2^d nodes.  Quantized mode is the */
/* fixed-point rule: 16-bit offsets u = floor(f * 2^16), and the weight is    */
/* split axis by axis, upper part = floor(part * u / 2^16), lower = the rest, */
/* so every particle deposits exactly its integer weight.                     */
/* ------------------------------------------------------------------------- */

int orc_deposit(const orc_grid *g, int64_t np, const int32_t *cell, const double *off,
                const int32_t *wq, int64_t *node_q, double *node_f) {
  const int64_t nn = orc_num_nodes(g), nc = orc_num_cells(g);
  const int nd = g->ndim, ncorner = 1 << nd;
  int64_t *acc = node_q;
  int own = 0;
  if (g->quantized && !acc) {
    acc = (int64_t *)calloc((size_t)nn, sizeof(int64_t));
    if (!acc) return ORC_EINVAL;
    own = 1;
  }
  if (acc) memset(acc, 0, sizeof(int64_t) * (size_t)nn);
  memset(node_f, 0, sizeof(double) * (size_t)nn);

  for (int64_t p = 0; p < np; ++p) {
    if (cell[p] < 0 || cell[p] >= nc) { if (own) free(acc); return ORC_ERANGE; }
    if (wq[p] < 0) { if (own) free(acc); return ORC_EOVERFLOW; }
    for (int d = 0; d < nd; ++d) {
      double f = off[(int64_t)d * np + p];
      if (!(f >= 0.0 && f < 1.0)) { if (own) free(acc); return ORC_ERANGE; }
    }
  }
  /* Threaded build only (-fopenmp; the pragmas are inert otherwise): integer
   * sums are order free, so particles may be split over threads; the FP64
   * unquantized sums stay in particle order. */
#pragma omp parallel for schedule(static) if (g->quantized)
  for (int64_t p = 0; p < np; ++p) {
    int idx[3];
    cell_to_index(g, cell[p], idx);
    double f[3];
    for (int d = 0; d < nd; ++d) f[d] = off[(int64_t)d * np + p];
    for (int k = 0; k < ncorner; ++k) {
      int a[3] = {idx[0], idx[1], idx[2]};
      for (int d = 0; d < nd; ++d) a[d] += (k >> d) & 1;
      int64_t node = node_at(g, a);
      if (g->quantized) {
        /* recompute this corner's share by walking the split x, then y, then z */
        int64_t part = wq[p];
        for (int d = 0; d < nd; ++d) {
          double s = floor(f[d] * 65536.0);
          int64_t u = (int64_t)s;
          if (u < 0) u = 0;
          if (u > 65535) u = 65535;
          int64_t upper = (part * u) >> 16;
          part = ((k >> d) & 1) ? upper : part - upper;
        }
#pragma omp atomic
        acc[node] += part;
      } else {
        double wgt = (double)wq[p];
        for (int d = 0; d < nd; ++d) wgt *= ((k >> d) & 1) ? f[d] : 1.0 - f[d];
        node_f[node] += wgt;
      }
    }
  }
  if (g->quantized)
    for (int64_t k = 0; k < nn; ++k) node_f[k] = (double)acc[k];
  if (own) free(acc);
  return ORC_OK;
}

void orc_density(const orc_grid *g, const double *node_f, double *dens) {
  const int64_t nn = orc_num_nodes(g);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < nn; ++k) dens[k] = node_f[k] * ORC_WUNIT / node_volume(g, k);
}

/* ------------------------------------------------------------------------- */
/* Gradient (method section): from the node densities the method forms a    */
/* density gradient at the cell centres, half a node spacing from the nodes. */
/* Reading: component d at a cell                                             */
/* centre is the mean of the node differences along the cell's 2^(d-1) edges  */
/* parallel to d, divided by the cell edge.                                   */
/* ------------------------------------------------------------------------- */

void orc_gradient(const orc_grid *g, const double *dens, double *G) {
  const int64_t nc = orc_num_cells(g);
  const int nd = g->ndim, ncorner = 1 << nd;
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nc; ++c) {
    int idx[3];
    cell_to_index(g, (int32_t)c, idx);
    for (int d = 0; d < nd; ++d) {
      double sum = 0.0;
      for (int k = 0; k < ncorner; ++k) {
        if ((k >> d) & 1) continue; /* lower end of an edge along d */
        int lo[3] = {idx[0], idx[1], idx[2]}, hi[3];
        for (int e = 0; e < nd; ++e) lo[e] += (k >> e) & 1;
        memcpy(hi, lo, sizeof(hi));
        hi[d] += 1;
        sum += dens[node_at(g, hi)] - dens[node_at(g, lo)];
      }
      G[(int64_t)d * nc + c] = sum / ((double)(ncorner / 2) * g->h[d]);
    }
  }
}

/* Gradient component d at cell centre with (possibly ghost) index m.  Reading:
 * a ghost centre beyond a reflecting wall is the mirror of the first interior
 * centre, with the normal component negated and tangential ones kept. */
static double centre_gradient(const orc_grid *g, const double *G, int d, const int m_in[3]) {
  int m[3] = {m_in[0], m_in[1], m_in[2]};
  double sign = 1.0;
  for (int e = 0; e < g->ndim; ++e) {
    int n = g->n[e];
    if (!g->bc[e]) {
      m[e] %= n;
      if (m[e] < 0) m[e] += n;
    } else if (m[e] < 0) {
      m[e] = -1 - m[e];
      if (e == d) sign = -sign;
    } else if (m[e] >= n) {
      m[e] = 2 * n - 1 - m[e];
      if (e == d) sign = -sign;
    }
  }
  return sign * G[(int64_t)d * orc_num_cells(g) + index_to_cell(g, m)];
}

/* ------------------------------------------------------------------------- */
/* Gather (method section): density and gradient go back to each           */
/* macroparticle with the same shape that deposited it.  Reading: the linear */
/* shape as the deposit -- node density from the cell's 2^d corner nodes, the */
/* gradient from the 2^d nearest cell centres.                                */
/* ------------------------------------------------------------------------- */

void orc_gather(const orc_grid *g, const double *dens, const double *G, int32_t cell,
                const double *f, double *n_p, double *G_p) {
  const int nd = g->ndim, ncorner = 1 << nd;
  int idx[3];
  cell_to_index(g, cell, idx);
  double n = 0.0;
  for (int k = 0; k < ncorner; ++k) {
    int a[3] = {idx[0], idx[1], idx[2]};
    double wgt = 1.0;
    for (int d = 0; d < nd; ++d) {
      int b = (k >> d) & 1;
      a[d] += b;
      wgt *= b ? f[d] : 1.0 - f[d];
    }
    n += wgt * dens[node_at(g, a)];
  }
  *n_p = n;

  int c0[3] = {0, 0, 0};
  double t[3] = {0, 0, 0};
  for (int e = 0; e < nd; ++e) {
    if (f[e] >= 0.5) { c0[e] = idx[e]; t[e] = f[e] - 0.5; }
    else { c0[e] = idx[e] - 1; t[e] = f[e] + 0.5; }
  }
  for (int d = 0; d < nd; ++d) {
    double s = 0.0;
    for (int k = 0; k < ncorner; ++k) {
      int m[3] = {c0[0], c0[1], c0[2]};
      double wgt = 1.0;
      for (int e = 0; e < nd; ++e) {
        int b = (k >> e) & 1;
        m[e] += b;
        wgt *= b ? t[e] : 1.0 - t[e];
      }
      s += wgt * centre_gradient(g, G, d, m);
    }
    G_p[d] = s;
  }
}

/* ------------------------------------------------------------------------- */
/* Eq. (3): U(r) = D((r0/r)^12 - 2 (r0/r)^6).  The method works with any pair */
/* potential (the paper names the Morse potential among them); kind 1 is     */
/* Morse, U(r) = D(e^2 - 2e), e = exp(-a (r - r0)): the same well depth D at  */
/* the same equilibrium distance r0.  The altered potential: the repulsive   */
/* branch (r < r0) is scaled by s_rep (the paper's infinite wall is the      */
/* s_rep -> infinity limit), the attractive branch (r >= r0) by the          */
/* correction factor c_att.  U'(r0) = 0, so the force is continuous at r0.   */
/* ------------------------------------------------------------------------- */

static double base_u(const orc_pot *p, double r) {
  if (p->kind == 1) {
    double e = exp(-p->alpha * (r - p->r0));
    return p->D * (e * e - 2.0 * e);
  }
  double x = p->r0 / r;
  return p->D * (pow(x, 12.0) - 2.0 * pow(x, 6.0));
}

static double base_du(const orc_pot *p, double r) {
  if (p->kind == 1) {
    double e = exp(-p->alpha * (r - p->r0));
    return -2.0 * p->alpha * p->D * (e * e - e);
  }
  double x = p->r0 / r;
  return -(12.0 * p->D / r) * (pow(x, 12.0) - pow(x, 6.0));
}

double orc_phi_prime(const orc_pot *p, double r) {
  return (r < p->r0 ? p->s_rep : p->c_att) * base_du(p, r);
}

double orc_phi(const orc_pot *p, double r) {
  double u = base_u(p, r);
  if (r >= p->r0) return p->c_att * u;
  /* continuous at r0: s*U(r) + (s - c)*D */
  return p->s_rep * u + (p->s_rep - p->c_att) * p->D;
}

/* Local geometry and force at one macroparticle.
 *   rbar = n^(-1/3);  eq. (1): d rbar/dx_d = -(1/3) (dn/dx_d) n^(-4/3).
 *   eq. (2) from its midpoint rule: the +d neighbour sits at
 *   r+ = rbar / (1 - g/2) and the -d neighbour at r- = rbar / (1 + g/2),
 *   g = d rbar/dx_d (rbar evaluated half-way equals the pair distance).
 *   Force along d: phi'(r+) - phi'(r-), the two neighbours' pair forces
 *   (cubic lattice: one neighbour pair per evolved axis).
 * Reading: g is clamped to [-g_clamp, g_clamp] and the force is zero at
 * densities n <= n_floor, where eq. (2) stops describing a lattice. */
void orc_neighbour_distances(const orc_pot *p, double n_p, double G_pd, double *r_plus,
                             double *r_minus) {
  double rbar = pow(n_p, -1.0 / 3.0);
  double g = -(1.0 / 3.0) * G_pd * pow(n_p, -4.0 / 3.0); /* eq. (1) */
  if (g > p->g_clamp) g = p->g_clamp;
  if (g < -p->g_clamp) g = -p->g_clamp;
  *r_plus = rbar / (1.0 - 0.5 * g);  /* eq. (2), neighbour on the +d side */
  *r_minus = rbar / (1.0 + 0.5 * g); /* eq. (2), neighbour on the -d side */
}

/* Hexagonal close-packed lattice (the paper notes the construction adapts to
 * it).  Reading: the 12 nearest neighbours of the ideal lattice (c/a =
 * sqrt(8/3)), c axis along the normal (last) axis, a basal axis along x;
 * nearest-neighbour distance a = 2^(1/6) rbar (atomic volume a^3/sqrt(2)).
 * The midpoint rule of eq. (2) along neighbour direction u: the pair
 * distance equals the local spacing half-way, d = 2^(1/6) (rbar + (d/2)
 * grad(rbar).u), so d = 2^(1/6) rbar / (1 - q/2) with q = 2^(1/6) grad(rbar).u
 * clamped to [-g_clamp, g_clamp] (the cubic rule is c = 1, u = +-e_d).  The
 * force is the sum of the 12 pair forces phi'(d) u.  In 2D the second basal
 * axis is the one the plane does not resolve: its density gradient is zero
 * and its force component is dropped (the lattice and its mirror image in
 * that axis give the same in-plane force and opposite out-of-plane ones). */
#define HCP_C 1.1224620483093730 /* 2^(1/6) */
void orc_hcp_direction(int k, double u[3]) { /* basal 1, basal 2, c */
  if (k < 6) {
    double t = acos(-1.0) / 3.0 * k;
    u[0] = cos(t); u[1] = sin(t); u[2] = 0.0;
  } else {
    double t = acos(-1.0) * (1.0 / 6.0 + 2.0 / 3.0 * ((k - 6) % 3));
    u[0] = cos(t) / sqrt(3.0); u[1] = sin(t) / sqrt(3.0); u[2] = (k < 9 ? 1.0 : -1.0) * sqrt(2.0 / 3.0);
  }
}

/* neighbour k's direction in grid axes (evolved components; 2D: x, normal) */
static void hcp_grid_direction(int ndim, int k, double v[3]) {
  double u[3];
  orc_hcp_direction(k, u);
  if (ndim == 3) { v[0] = u[0]; v[1] = u[1]; v[2] = u[2]; }
  else { v[0] = u[0]; v[1] = u[2]; v[2] = 0.0; }
}

static double hcp_distance(const orc_pot *p, int ndim, double n_p, const double *G_p, const double *v) {
  double rbar = pow(n_p, -1.0 / 3.0), gu = 0.0;
  for (int d = 0; d < ndim; ++d) gu += -(1.0 / 3.0) * G_p[d] * pow(n_p, -4.0 / 3.0) * v[d]; /* eq. (1) */
  double q = HCP_C * gu;
  if (q > p->g_clamp) q = p->g_clamp;
  if (q < -p->g_clamp) q = -p->g_clamp;
  return HCP_C * rbar / (1.0 - 0.5 * q);
}

void orc_local_force(const orc_pot *p, int ndim, double n_p, const double *G_p, double *F) {
  for (int d = 0; d < ndim; ++d) F[d] = 0.0;
  if (!(n_p > p->n_floor)) return;
  if (p->lattice == 1) {
    for (int k = 0; k < 12; ++k) {
      double v[3];
      hcp_grid_direction(ndim, k, v);
      double f = orc_phi_prime(p, hcp_distance(p, ndim, n_p, G_p, v));
      for (int d = 0; d < ndim; ++d) F[d] += f * v[d];
    }
    return;
  }
  for (int d = 0; d < ndim; ++d) {
    double r_plus, r_minus;
    orc_neighbour_distances(p, n_p, G_p[d], &r_plus, &r_minus);
    F[d] = orc_phi_prime(p, r_plus) - orc_phi_prime(p, r_minus);
  }
}

/* Per-atom bond energy of the same construction: (1/2) sum over the
 * neighbour pairs of phi(r) (cubic: 2*ndim, hexagonal: 12). */
static double local_bond_energy(const orc_pot *p, int ndim, double n_p, const double *G_p) {
  if (!(n_p > p->n_floor)) return 0.0;
  double e = 0.0;
  if (p->lattice == 1) {
    for (int k = 0; k < 12; ++k) {
      double v[3];
      hcp_grid_direction(ndim, k, v);
      e += 0.5 * orc_phi(p, hcp_distance(p, ndim, n_p, G_p, v));
    }
    return e;
  }
  for (int d = 0; d < ndim; ++d) {
    double r_plus, r_minus;
    orc_neighbour_distances(p, n_p, G_p[d], &r_plus, &r_minus);
    e += 0.5 * (orc_phi(p, r_plus) + orc_phi(p, r_minus));
  }
  return e;
}

/* Energy density whose density derivative is the per-atom chemical potential
 * mu(n) = phi(rbar) - rbar phi'(rbar), rbar = n^(-1/3) (so that in a slowly
 * varying density the force above is -grad mu).  For the plain L-J branch
 * eps(n) = D (13/5 r0^12 n^5 - 14/3 r0^6 n^3); the branch multipliers switch
 * at n0 = r0^-3 with continuity of eps and its slope. */
/* mu(n) = phi(rbar) - rbar phi'(rbar), rbar = n^(-1/3); hexagonal lattice:
 * mu = 2 (phi(a) - a phi'(a)), a = 2^(1/6) rbar: the 12 bonds (sum of u u^T
 * = 4 I) give the small-gradient force 2^(4/3) rbar phi''(a) grad(rbar),
 * which is -grad mu. */
static double chem_potential(const orc_pot *p, double n) {
  if (!(n > 0.0)) return 0.0;
  double rb = pow(n, -1.0 / 3.0);
  if (p->lattice == 1) {
    double a = HCP_C * rb;
    return 2.0 * (orc_phi(p, a) - a * orc_phi_prime(p, a));
  }
  return orc_phi(p, rb) - rb * orc_phi_prime(p, rb);
}

static double simpson_step(const orc_pot *p, double a, double b, double fa, double fm, double fb, double whole,
                           double tol, int depth) {
  double m = 0.5 * (a + b);
  double lm = chem_potential(p, 0.5 * (a + m)), rm = chem_potential(p, 0.5 * (m + b));
  double left = (m - a) / 6.0 * (fa + 4.0 * lm + fm), right = (b - m) / 6.0 * (fm + 4.0 * rm + fb);
  double diff = left + right - whole;
  if (depth <= 0 || fabs(diff) <= 15.0 * tol) return left + right + diff / 15.0;
  return simpson_step(p, a, m, fa, lm, fm, left, 0.5 * tol, depth - 1) +
         simpson_step(p, m, b, fm, rm, fb, right, 0.5 * tol, depth - 1);
}

static double integrate_mu(const orc_pot *p, double a, double b) {
  if (!(b > a)) return 0.0;
  double fa = chem_potential(p, a), fb = chem_potential(p, b), fm = chem_potential(p, 0.5 * (a + b));
  double whole = (b - a) / 6.0 * (fa + 4.0 * fm + fb);
  /* tolerance relative to the integrand's size on the interval, so that the
   * recursion ends where mu grows steeply (compressed densities) */
  double big = fmax(fmax(fabs(fa), fabs(fb)), fmax(fabs(fm), p->D));
  return simpson_step(p, a, b, fa, fm, fb, whole, 1e-14 * big * (b - a), 40);
}

/* The integral of mu from 0 to n, split where the branch multiplier switches
 * (n0 = r0^-3, sqrt(2) r0^-3 on the hexagonal lattice; mu has a kink). */
double orc_energy_density_quad(const orc_pot *p, double n) {
  const double n0 = (p->lattice == 1 ? sqrt(2.0) : 1.0) / (p->r0 * p->r0 * p->r0);
  if (n <= n0) return integrate_mu(p, 0.0, n);
  return integrate_mu(p, 0.0, n0) + integrate_mu(p, n0, n);
}

double orc_energy_density(const orc_pot *p, double n) {
  if (p->kind != 0 || p->lattice != 0) return orc_energy_density_quad(p, n);
  const double r6 = pow(p->r0, 6.0), r12 = r6 * r6;
  const double n0 = 1.0 / (p->r0 * p->r0 * p->r0);
  double lj = p->D * (13.0 / 5.0 * r12 * pow(n, 5.0) - 14.0 / 3.0 * r6 * pow(n, 3.0));
  if (n <= n0) return p->c_att * lj;
  double lj0 = p->D * (13.0 / 5.0 * r12 * pow(n0, 5.0) - 14.0 / 3.0 * r6 * pow(n0, 3.0));
  return p->c_att * lj0 + p->s_rep * (lj - lj0) + (p->s_rep - p->c_att) * p->D * (n - n0);
}

void orc_forces(const orc_grid *g, const orc_pot *p, const double *node_f, int64_t np,
                const int32_t *cell, const double *off, double *F) {
  const int64_t nn = orc_num_nodes(g), nc = orc_num_cells(g);
  double *dens = (double *)malloc(sizeof(double) * (size_t)nn);
  double *G = (double *)malloc(sizeof(double) * (size_t)(nc * g->ndim));
  orc_density(g, node_f, dens);
  orc_gradient(g, dens, G);
  for (int64_t i = 0; i < np; ++i) {
    double f[3], n_p, G_p[3], Fi[3];
    for (int d = 0; d < g->ndim; ++d) f[d] = off[(int64_t)d * np + i];
    orc_gather(g, dens, G, cell[i], f, &n_p, G_p);
    orc_local_force(p, g->ndim, n_p, G_p, Fi);
    for (int d = 0; d < g->ndim; ++d) F[(int64_t)d * np + i] = Fi[d];
  }
  free(dens);
  free(G);
}

/* ------------------------------------------------------------------------- */
/* Push.  Reading: standard PIC leapfrog with half-step velocities,           */
/*   v(n+1/2) = v(n-1/2) + F(n)/m dt,   x(n+1) = x(n) + v(n+1/2) dt,           */
/* 2D moves only the two in-plane coordinates (all three velocity components  */
/* are kept; F_z = 0).  The position is (cell, offset in [0,1)): carry whole  */
/* cells, wrap periodic axes, mirror at reflecting walls (v_d -> -v_d).  A     */
/* step that moves a particle a whole cell or more is an error (CFL).          */
/* ------------------------------------------------------------------------- */

int orc_push_one(const orc_grid *g, const orc_pot *p, double dt, const double *F, int32_t *cell,
                 double *f, double *v) {
  int idx[3];
  cell_to_index(g, *cell, idx);
  for (int d = 0; d < g->ndim; ++d) v[d] += F[d] / p->mass * dt;
  for (int d = 0; d < g->ndim; ++d) {
    double df = v[d] * dt / g->h[d];
    if (!(fabs(df) < 1.0)) return ORC_ECFL;
    double x = f[d] + df;
    int n = g->n[d];
    if (g->bc[d] && idx[d] == 0 && x < 0.0) {
      x = -x;
      v[d] = -v[d];
    } else if (g->bc[d] && idx[d] == n - 1 && x >= 1.0) {
      x = 2.0 - x;
      v[d] = -v[d];
      if (x >= 1.0) x = nextafter(1.0, 0.0); /* exactly on the wall */
    } else if (x >= 1.0) {
      x -= 1.0;
      idx[d] += 1;
    } else if (x < 0.0) {
      x += 1.0;
      idx[d] -= 1;
      if (x >= 1.0) { /* rounded up: the particle sits on the node itself */
        x = 0.0;
        idx[d] += 1;
      }
    }
    if (!g->bc[d]) {
      if (idx[d] < 0) idx[d] += n;
      if (idx[d] >= n) idx[d] -= n;
    }
    f[d] = x;
  }
  *cell = index_to_cell(g, idx);
  return ORC_OK;
}

void orc_kick(const orc_grid *g, const orc_pot *p, double dt, double frac, int64_t np,
              const double *F, double *vel) {
  for (int64_t i = 0; i < np; ++i)
    for (int d = 0; d < g->ndim; ++d) vel[(int64_t)d * np + i] += frac * F[(int64_t)d * np + i] / p->mass * dt;
}

/* ------------------------------------------------------------------------- */
/* Full cycle, with diagnostics at the requested steps:                        */
/*   KE(n) = sum w m/2 (|v(n-1/2)|^2 + |v(n+1/2)|^2)/2,                          */
/*   P(n)  = sum w m (v(n-1/2) + v(n+1/2))/2,                                    */
/*   PE(n) = sum over nodes V_node eps(n_node),  bond = sum w e_bond.            */
/* ------------------------------------------------------------------------- */

int orc_run(const orc_grid *g, const orc_pot *p, double dt, int64_t np, int32_t *cell, double *off,
            double *vel, const int32_t *wq, int nsteps, int diag_every, orc_diag *diag) {
  const int64_t nn = orc_num_nodes(g), nc = orc_num_cells(g);
  const int nd = g->ndim;
  double *node_f = (double *)malloc(sizeof(double) * (size_t)(nn > 0 ? nn : 1));
  double *dens = (double *)malloc(sizeof(double) * (size_t)(nn > 0 ? nn : 1));
  double *G = (double *)malloc(sizeof(double) * (size_t)(nc * nd > 0 ? nc * nd : 1));
  int rc = ORC_OK, di = 0;
  for (int s = 0; s < nsteps && rc == ORC_OK; ++s) {
    rc = orc_deposit(g, np, cell, off, wq, NULL, node_f);
    if (rc) break;
    orc_density(g, node_f, dens);
    orc_gradient(g, dens, G);
    int want = diag && diag_every > 0 && (s % diag_every) == 0;
    double ke = 0, px = 0, py = 0, pz = 0, ws = 0, bond = 0;
    int64_t first_bad = np;
#pragma omp parallel for schedule(static) reduction(+ : ke, px, py, pz, ws, bond) reduction(min : first_bad)
    for (int64_t i = 0; i < np; ++i) {
      double f[3] = {0, 0, 0}, v[3], n_p, G_p[3] = {0, 0, 0}, Fi[3] = {0, 0, 0};
      for (int d = 0; d < nd; ++d) f[d] = off[(int64_t)d * np + i];
      for (int d = 0; d < 3; ++d) v[d] = vel[(int64_t)d * np + i];
      orc_gather(g, dens, G, cell[i], f, &n_p, G_p);
      orc_local_force(p, nd, n_p, G_p, Fi);
      if (want) {
        double w = wq[i] * ORC_WUNIT, v2o = 0, v2n = 0, vn[3];
        for (int d = 0; d < 3; ++d) {
          vn[d] = v[d] + (d < nd ? Fi[d] / p->mass * dt : 0.0);
          v2o += v[d] * v[d];
          v2n += vn[d] * vn[d];
        }
        ke += w * 0.5 * p->mass * 0.5 * (v2o + v2n);
        px += w * p->mass * 0.5 * (v[0] + vn[0]);
        py += w * p->mass * 0.5 * (v[1] + vn[1]);
        pz += w * p->mass * 0.5 * (v[2] + vn[2]);
        ws += w;
        bond += w * local_bond_energy(p, nd, n_p, G_p);
      }
      if (orc_push_one(g, p, dt, Fi, &cell[i], f, v) != ORC_OK) {
        if (i < first_bad) first_bad = i;
        continue;
      }
      for (int d = 0; d < nd; ++d) off[(int64_t)d * np + i] = f[d];
      for (int d = 0; d < 3; ++d) vel[(int64_t)d * np + i] = v[d];
    }
    if (first_bad < np) rc = ORC_ECFL;
    if (want && rc == ORC_OK) {
      double pe = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : pe)
      for (int64_t k = 0; k < nn; ++k) pe += node_volume(g, k) * orc_energy_density(p, dens[k]);
      orc_diag *o = &diag[di++];
      o->ke = ke; o->pe = pe; o->px = px; o->py = py; o->pz = pz; o->wsum = ws; o->bond = bond;
      o->step = s;
    }
  }
  free(node_f);
  free(dens);
  free(G);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Attractive correction (method section, after eq. 3): a factor on the     */
/* attractive force, set from the work the force does on one atom that      */
/* leaves the target and goes to infinity.  Reading: build a flat            */
/* slab of solid density as a commensurate lattice (lattice_k^d particles per */
/* cell) on a grid of the given cell size, move a zero-weight test atom along */
/* the surface normal with unit attractive multiplier, take W = -integral of  */
/* its normal force from the outermost repulsive-to-attractive sign change to */
/* infinity (zero beyond the first empty node), and set c_att = D / W.        */
/* ------------------------------------------------------------------------- */

typedef struct {
  const orc_grid *g;
  const orc_pot *p;
  const double *dens, *G;
  int nd;
} calib_ctx;

static double calib_force(const calib_ctx *c, double y_cells) {
  int idx[3] = {0, 0, 0};
  double f[3] = {0.25, 0.25, 0.25};
  int nd = c->nd, ax = nd - 1;
  double fl = floor(y_cells);
  idx[ax] = (int)fl;
  f[ax] = y_cells - fl;
  double n_p, G_p[3], F[3];
  orc_gather(c->g, c->dens, c->G, index_to_cell(c->g, idx), f, &n_p, G_p);
  orc_local_force(c->p, nd, n_p, G_p, F);
  return F[ax];
}

static double gauss_legendre16(const calib_ctx *c, double a, double b) {
  static const double x[8] = {0.0950125098376374, 0.2816035507792589, 0.4580167776572274,
                              0.6178762444026438, 0.7554044083550030, 0.8656312023878318,
                              0.9445750230732326, 0.9894009349916499};
  static const double w[8] = {0.1894506104550685, 0.1826034150449236, 0.1691565193950025,
                              0.1495959888165767, 0.1246289712555339, 0.0951585116824928,
                              0.0622535239386479, 0.0271524594117541};
  double m = 0.5 * (a + b), r = 0.5 * (b - a), s = 0.0;
  for (int i = 0; i < 8; ++i) s += w[i] * (calib_force(c, m - r * x[i]) + calib_force(c, m + r * x[i]));
  return r * s;
}

/* Interval halving until the two halves agree with the whole to 1e-12 of
 * their magnitudes (at most 18 halvings). */
static double adaptive_gl(const calib_ctx *c, double a, double b, double whole, int depth) {
  double m = 0.5 * (a + b);
  double l = gauss_legendre16(c, a, m), r = gauss_legendre16(c, m, b);
  if (depth >= 18 || fabs(l + r - whole) <= 1e-12 * (fabs(l) + fabs(r)) + 1e-300) return l + r;
  return adaptive_gl(c, a, m, l, depth + 1) + adaptive_gl(c, m, b, r, depth + 1);
}

int orc_calibrate_catt(const orc_grid *gin, const orc_pot *pin, double n_solid, int slab_layers,
                       int lattice_k, double *c_att, double *work, double *y_star) {
  if (slab_layers < 2 || lattice_k < 1) return ORC_EINVAL;
  const int nd = gin->ndim, ax = nd - 1;
  orc_grid g = *gin;
  for (int d = 0; d < nd; ++d) { g.n[d] = 2; g.bc[d] = 0; }
  g.n[ax] = slab_layers + 4;
  g.bc[ax] = 1;
  g.quantized = 0;
  orc_pot p = *pin;
  p.c_att = 1.0;

  /* the lattice: lattice_k^nd particles per slab cell at (a + 1/2)/k */
  int64_t lateral = 1;
  for (int d = 0; d < ax; ++d) lateral *= g.n[d];
  int64_t per = 1;
  for (int d = 0; d < nd; ++d) per *= lattice_k;
  int64_t np = lateral * slab_layers * per;
  int32_t *cell = (int32_t *)malloc(sizeof(int32_t) * (size_t)np);
  int32_t *wq = (int32_t *)malloc(sizeof(int32_t) * (size_t)np);
  double *off = (double *)malloc(sizeof(double) * (size_t)(np * nd));
  /* unquantized deposit: weight unit chosen so node density is exactly n_solid */
  double V = g.h[0] * g.h[1] * (nd == 3 ? g.h[2] : g.depth2d);
  int64_t i = 0;
  for (int64_t c = 0; c < lateral * slab_layers; ++c)
    for (int64_t s = 0; s < per; ++s, ++i) {
      cell[i] = (int32_t)c;
      wq[i] = 1;
      int64_t r = s;
      for (int d = 0; d < nd; ++d) {
        off[(int64_t)d * np + i] = ((double)(r % lattice_k) + 0.5) / lattice_k;
        r /= lattice_k;
      }
    }
  const int64_t nn = orc_num_nodes(&g), nc = orc_num_cells(&g);
  double *node_f = (double *)malloc(sizeof(double) * (size_t)nn);
  double *dens = (double *)malloc(sizeof(double) * (size_t)nn);
  double *G = (double *)malloc(sizeof(double) * (size_t)(nc * nd));
  orc_deposit(&g, np, cell, off, wq, NULL, node_f);
  /* each particle carries n_solid V / per atoms */
  for (int64_t k = 0; k < nn; ++k) node_f[k] *= (n_solid * V / (double)per) / ORC_WUNIT;
  orc_density(&g, node_f, dens);
  orc_gradient(&g, dens, G);
  calib_ctx cx = {&g, &p, dens, G, nd};

  /* outermost repulsive (outward, F > 0) -> attractive (F <= 0) sign change
   * between the middle of the slab and the first empty node */
  double y_lo = 0.5 * slab_layers, y_end = slab_layers + 1.0;
  const int nscan = 4096;
  double ys = -1.0;
  double prev = calib_force(&cx, y_lo);
  for (int k = 1; k <= nscan; ++k) {
    double y = y_lo + (y_end - y_lo) * k / nscan;
    double cur = calib_force(&cx, y);
    if (prev > 0.0 && cur <= 0.0) {
      double a = y - (y_end - y_lo) / nscan, b = y;
      for (int it = 0; it < 200; ++it) {
        double m = 0.5 * (a + b);
        if (calib_force(&cx, m) > 0.0) a = m; else b = m;
      }
      ys = 0.5 * (a + b);
    }
    prev = cur;
  }
  int rc = ORC_OK;
  if (ys < 0.0) {
    rc = ORC_EINVAL;
  } else {
    /* integrate piecewise between the kinks (nodes and centres: every half cell) */
    double total = 0.0, a = ys;
    while (a < y_end) {
      double b = floor(a * 2.0 + 1.0) * 0.5;
      if (b > y_end) b = y_end;
      if (b > a) total += adaptive_gl(&cx, a, b, gauss_legendre16(&cx, a, b), 0);
      a = b;
    }
    double W = -total * g.h[ax]; /* y in cells -> metres */
    if (work) *work = W;
    if (y_star) *y_star = ys;
    if (c_att) *c_att = p.D / W;
  }
  free(cell); free(wq); free(off); free(node_f); free(dens); free(G);
  return rc;
}

double orc_functional(const orc_grid *g, int64_t np, const int32_t *cell, const double *off,
                      const int32_t *wq, double y_s, double tau) {
  const int ax = g->ndim - 1;
  double J = 0.0;
  for (int64_t i = 0; i < np; ++i) {
    int idx[3];
    cell_to_index(g, cell[i], idx);
    double y = ((double)idx[ax] + off[(int64_t)ax * np + i]) * g->h[ax];
    J += wq[i] * ORC_WUNIT / (1.0 + exp(-(y - y_s) / tau));
  }
  return J;
}
