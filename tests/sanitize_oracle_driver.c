/* Drives the FP64 oracle through its entry points under AddressSanitizer
 * and UndefinedBehaviorSanitizer (built and run by test_sanitizers.py):
 * deposits, forces and runs with diagnostics in 2D and 3D for both pair
 * potentials and both lattices, calibration, and the error paths. */
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/pic_oracle.h"

static unsigned long long lcg = 12345;
static double urand(void) {
  lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
  return (double)(lcg >> 11) / 9007199254740992.0;
}

static int run_case(int ndim, int kind, int lattice) {
  orc_grid g = {0};
  g.ndim = ndim;
  g.n[0] = 8; g.n[1] = 7; g.n[2] = ndim == 3 ? 6 : 1;
  for (int d = 0; d < 3; ++d) g.h[d] = 2e-9;
  g.bc[ndim - 1] = 1;
  g.depth2d = ndim == 2 ? 2e-9 : 0.0;
  g.quantized = 1;
  orc_pot p = {6.5577e-20, 2.2754e-10 * (lattice ? 1.12246 : 1.0), 1.0, 0.3, 1.0, 8.49e22, 1.0552e-25,
               kind, lattice, 1.3588e10};
  const int layers = 3, ppc = 4;
  int64_t lateral = ndim == 3 ? 8 * 7 : 8;
  int64_t np = lateral * layers * ppc;
  int32_t *cell = malloc(sizeof(int32_t) * np);
  int32_t *wq = malloc(sizeof(int32_t) * np);
  double *off = malloc(sizeof(double) * ndim * np);
  double *vel = malloc(sizeof(double) * 3 * np);
  for (int64_t i = 0; i < np; ++i) {
    cell[i] = (int32_t)(i / ppc);
    wq[i] = (int32_t)(150.0 * 1048576.0);
    for (int d = 0; d < ndim; ++d) off[d * np + i] = 0.05 + 0.9 * urand();
    for (int d = 0; d < 3; ++d) vel[d * np + i] = 300.0 * (urand() - 0.5);
  }
  int64_t nn = orc_num_nodes(&g);
  int64_t *nq = malloc(sizeof(int64_t) * nn);
  double *nf = malloc(sizeof(double) * nn);
  double *F = malloc(sizeof(double) * ndim * np);
  int bad = 0;
  if (orc_deposit(&g, np, cell, off, wq, nq, nf) != ORC_OK) bad |= 1;
  orc_forces(&g, &p, nf, np, cell, off, F);
  orc_diag diag[4];
  if (orc_run(&g, &p, 1e-15, np, cell, off, vel, wq, 20, 5, diag) != ORC_OK) bad |= 2;
  double c_att = 0, work = 0, ys = 0;
  orc_grid gc = g;
  gc.quantized = 0;
  if (orc_calibrate_catt(&gc, &p, 8.49e28, 8, 2, &c_att, &work, &ys) != ORC_OK || !(c_att > 0)) bad |= 4;
  /* error paths: a cell outside the grid, an offset outside [0, 1) */
  int32_t keep = cell[0];
  cell[0] = (int32_t)orc_num_cells(&g);
  if (orc_deposit(&g, np, cell, off, wq, nq, nf) != ORC_ERANGE) bad |= 8;
  cell[0] = keep;
  off[0] = 1.5;
  if (orc_deposit(&g, np, cell, off, wq, nq, nf) != ORC_ERANGE) bad |= 16;
  free(cell); free(wq); free(off); free(vel); free(nq); free(nf); free(F);
  return bad;
}

int main(void) {
  int bad = 0;
  for (int nd = 2; nd <= 3; ++nd)
    for (int kind = 0; kind <= 1; ++kind)
      for (int lat = 0; lat <= 1; ++lat) {
        int b = run_case(nd, kind, lat);
        if (b) fprintf(stderr, "case %dD kind %d lattice %d: flags %d\n", nd, kind, lat, b);
        bad |= b;
      }
  printf("oracle sanitizer driver %s\n", bad ? "FAILED" : "ok");
  return bad ? 1 : 0;
}
