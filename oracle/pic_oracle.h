/*
 * FP64 CPU oracle for the PIC pair-potential cycle of Mitchell, Schumacher and
 * Chowdhury, "Modeling crater formation in femtosecond-pulse laser damage from
 * basic principles" (arXiv 1502.07722).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this code; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no source with the HIP library: its own types, its
 * own index arithmetic, SI units throughout, plain loops, no blocking or fusion.
 *
 * What it computes, per time step (the paper's PIC cycle, Fig. 1):
 *   deposit   each macroparticle weight onto the surrounding nodes (linear
 *             cloud-in-cell), in int64 fixed point (exact, order-free);
 *   density   node weight / node volume (half volume on reflecting walls);
 *   gradient  density gradient at the half-node (cell-centred) positions;
 *   gather    node density and centre gradient back to each particle with the
 *             same linear shape ("self-consistent" interpolation);
 *   geometry  rbar = n^(-1/3), eq. (1) for d rbar/dx, eq. (2) for the two
 *             nearest-neighbour distances per axis (cubic lattice);
 *   force     pair force from the altered L-J potential, eq. (3), with a
 *             multiplier on the repulsive branch and the attractive correction;
 *   push      leapfrog ("the PIC cycle ... evaluated for each time step as
 *             usual"), 2D keeps three velocity components.
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int ndim;        /* 2 or 3 */
  int n[3];        /* cells per axis */
  double h[3];     /* cell edge per axis, m */
  int bc[3];       /* 0 periodic, 1 reflecting */
  double depth2d;  /* 2D: thickness represented by the grid, m */
  int quantized;   /* 1: int64 fixed-point deposit; 0: plain FP64 CIC */
} orc_grid;

typedef struct {
  double D, r0, s_rep, c_att, g_clamp, n_floor, mass;
  int kind;      /* pair potential U: 0 eq. (3) Lennard-Jones, 1 Morse */
  int lattice;   /* assumed lattice: 0 cubic (eq. 1-2 per axis), 1 hexagonal close-packed */
  double alpha;  /* Morse width a, 1/m (kind 1) */
} orc_pot;

typedef struct {
  double ke, pe, px, py, pz, wsum, bond;
  int64_t step;
} orc_diag;

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_ERANGE = 2, ORC_ECFL = 3, ORC_EOVERFLOW = 4 };

int64_t orc_num_nodes(const orc_grid *g);
int64_t orc_num_cells(const orc_grid *g);

/* Fixed-point deposit (quantized) or plain FP64 deposit (g->quantized == 0).
 * off is [ndim][np] (axis-major), weights are wq = w * 2^20.
 * node_q receives int64 sums (quantized) and node_f FP64 sums in units of
 * 2^-20 atoms (both modes fill node_f; node_q may be NULL). */
int orc_deposit(const orc_grid *g, int64_t np, const int32_t *cell, const double *off,
                const int32_t *wq, int64_t *node_q, double *node_f);
void orc_density(const orc_grid *g, const double *node_f, double *dens);
void orc_gradient(const orc_grid *g, const double *dens, double *G /* [ndim][ncells] */);
void orc_gather(const orc_grid *g, const double *dens, const double *G, int32_t cell,
                const double *f, double *n_p, double *G_p);
/* eq. (1)-(2): distances to the +d and -d nearest neighbours (clamped g). */
void orc_neighbour_distances(const orc_pot *p, double n_p, double G_pd, double *r_plus,
                             double *r_minus);
void orc_local_force(const orc_pot *p, int ndim, double n_p, const double *G_p, double *F);
double orc_phi_prime(const orc_pot *p, double r);
double orc_phi(const orc_pot *p, double r);
double orc_energy_density(const orc_pot *p, double n);
/* Unit vector to nearest neighbour k (0-11) of the ideal hexagonal
 * close-packed lattice, in (basal 1, basal 2, c) axes. */
void orc_hcp_direction(int k, double u[3]);
/* The same energy density by adaptive quadrature of mu from 0 to n, for any
 * kind (the Morse energy density has no closed form). */
double orc_energy_density_quad(const orc_pot *p, double n);

/* Forces on np particles for a given deposit (node_f in 2^-20 atom units). */
void orc_forces(const orc_grid *g, const orc_pot *p, const double *node_f, int64_t np,
                const int32_t *cell, const double *off, double *F /* [ndim][np] */);

/* One leapfrog kick+drift for one particle; returns ORC_OK or ORC_ECFL. */
int orc_push_one(const orc_grid *g, const orc_pot *p, double dt, const double *F,
                 int32_t *cell, double *f /* [ndim] */, double *v /* [3] */);

/* v += frac * F/m * dt (used to start leapfrog: frac = -1/2). */
void orc_kick(const orc_grid *g, const orc_pot *p, double dt, double frac, int64_t np,
              const double *F, double *vel /* [3][np] */);

/* nsteps full cycles.  diag (optional) receives one entry per step whose index
 * is a multiple of diag_every.  Returns ORC_OK or the first error. */
int orc_run(const orc_grid *g, const orc_pot *p, double dt, int64_t np, int32_t *cell,
            double *off, double *vel, const int32_t *wq, int nsteps, int diag_every,
            orc_diag *diag);

/* Attractive correction factor: C_att = D / W, W the work to take a surface
 * atom of a flat solid-density slab out to infinity with unit multiplier. */
int orc_calibrate_catt(const orc_grid *g, const orc_pot *p, double n_solid, int slab_layers,
                       int lattice_k, double *c_att, double *work, double *y_star);

/* Smoothed removed-weight functional: sum_p w_p sigmoid((y_p - y_s)/tau). */
double orc_functional(const orc_grid *g, int64_t np, const int32_t *cell, const double *off,
                      const int32_t *wq, double y_s, double tau);

#ifdef __cplusplus
}
#endif
#endif
