/* Test driver (not part of the library): runs the FP64 oracle on small
 * grids so that a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * sees every code path of the grid step: periodic grids down to 1 x 1,
 * walls with a body force, the closure hook, the three-dimensional lattice
 * and the single-node entry points.  Prints "ok" and exits 0 when every
 * result is finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct orc orc;
typedef struct orc3d orc3d;
orc *orc_create(int nx, int ny, double tau_f, double tau_m, int walls, double Gx, double Gy,
                double bwx, double bwy, int feq_option);
void orc_destroy(orc *h);
void orc_init(orc *h, const double *u, const double *b);
void orc_step(orc *h, long n);
void orc_moments(const orc *h, double *rho, double *u, double *b);
void orc_diagnostics(const orc *h, double out[3]);
void orc_current_vorticity(const orc *h, double *jz, double *wz);
int orc_closure_nparams(void);
int orc_set_closure(orc *h, const double *params, const double *norm);
orc3d *orc3d_create(int nx, int ny, int nz, double tau_f, double tau_m);
void orc3d_destroy(orc3d *h);
void orc3d_init(orc3d *h, const double *u, const double *b);
void orc3d_step(orc3d *h, long n);
void orc3d_moments(const orc3d *h, double *rho, double *u, double *b);

static unsigned long long state = 88172645463325252ull;
static double rnd(void) {  /* xorshift64, uniform in [-1, 1) */
  state ^= state << 13;
  state ^= state >> 7;
  state ^= state << 17;
  return (double)(state >> 11) * 0x1.0p-52 - 1.0;
}

static int finite_all(const double *a, long n) {
  for (long i = 0; i < n; ++i)
    if (!isfinite(a[i])) return 0;
  return 1;
}

static int run2d(int nx, int ny, int walls, double G, int feq, int closure, long steps) {
  const long N = (long)nx * ny;
  double *u = malloc(2 * N * sizeof *u), *b = malloc(2 * N * sizeof *b);
  double *rho = malloc(N * sizeof *rho), *jz = malloc(N * sizeof *jz), *wz = malloc(N * sizeof *wz);
  for (long i = 0; i < 2 * N; ++i) u[i] = 0.03 * rnd(), b[i] = 0.03 * rnd();
  orc *h = orc_create(nx, ny, 0.53, 0.57, walls, G, 0.0, 0.0, walls ? 0.01 : 0.0, feq);
  if (!h) return 0;
  if (closure) {
    const int np = orc_closure_nparams();
    double *p = malloc(np * sizeof *p), norm[19];
    for (int k = 0; k < np; ++k) p[k] = 0.1 * rnd();
    for (int k = 0; k < 8; ++k) norm[k] = 0.0, norm[8 + k] = 0.05;
    norm[0] = 1.0;
    for (int k = 16; k < 19; ++k) norm[k] = 1e-5;
    if (orc_set_closure(h, p, norm) != 0) return 0;
    free(p);
  }
  orc_init(h, u, b);
  orc_step(h, steps);
  double d[3];
  orc_moments(h, rho, u, b);
  orc_diagnostics(h, d);
  int ok = finite_all(rho, N) && finite_all(u, 2 * N) && finite_all(b, 2 * N) && finite_all(d, 3);
  if (!walls) {
    orc_current_vorticity(h, jz, wz);
    ok = ok && finite_all(jz, N) && finite_all(wz, N);
  }
  orc_destroy(h);
  free(u), free(b), free(rho), free(jz), free(wz);
  return ok;
}

static int run3d(int nx, int ny, int nz, long steps) {
  const long N = (long)nx * ny * nz;
  double *u = malloc(3 * N * sizeof *u), *b = malloc(3 * N * sizeof *b), *rho = malloc(N * sizeof *rho);
  for (long i = 0; i < 3 * N; ++i) u[i] = 0.03 * rnd(), b[i] = 0.03 * rnd();
  orc3d *h = orc3d_create(nx, ny, nz, 0.55, 0.6);
  if (!h) return 0;
  orc3d_init(h, u, b);
  orc3d_step(h, steps);
  orc3d_moments(h, rho, u, b);
  int ok = finite_all(rho, N) && finite_all(u, 3 * N) && finite_all(b, 3 * N);
  orc3d_destroy(h);
  free(u), free(b), free(rho);
  return ok;
}

int main(void) {
  int ok = 1;
  ok = ok && run2d(7, 5, 0, 0.0, 0, 0, 20);
  ok = ok && run2d(1, 1, 0, 0.0, 0, 0, 5);
  ok = ok && run2d(2, 1, 0, 0.0, 1, 0, 5);
  ok = ok && run2d(6, 9, 1, 1e-5, 0, 0, 20);
  ok = ok && run2d(5, 2, 1, 1e-5, 0, 0, 5);
  ok = ok && run2d(8, 8, 0, 0.0, 0, 1, 5);
  ok = ok && run3d(3, 4, 5, 5);
  ok = ok && run3d(1, 1, 1, 3);
  puts(ok ? "ok" : "FAILED");
  return ok ? 0 : 1;
}
