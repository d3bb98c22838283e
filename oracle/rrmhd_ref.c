/*
 * The boundary's C-ABI over the FP64 oracle, with HOST pointers.
 *
 * TEST INFRASTRUCTURE ONLY (see rrmhd_oracle.c).  It exports the same entry
 * points and argument layouts as the HIP library's boundary -- create, init,
 * step, moments, diagnostics, invariants, step count, destroy, strerror --
 * so one test script can drive either backend; every array here is host
 * memory, and the arithmetic is the oracle's.  The structures below repeat
 * the boundary's published layouts field for field (an interface has to be
 * alike); nothing is shared with the HIP library's sources.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct orc orc;
orc *orc_create(int nx, int ny, double tau_f, double tau_m, int walls, double Gx, double Gy,
                double bwx, double bwy, int feq_option);
void orc_destroy(orc *h);
void orc_init(orc *h, const double *u, const double *b);
void orc_step(orc *h, long n);
long orc_step_count(const orc *h);
void orc_moments(const orc *h, double *rho, double *u, double *b);
void orc_diagnostics(const orc *h, double out[3]);
void orc_invariants(const orc *h, double out[5]);

/* the boundary's codes and layouts */
enum { REF_OK = 0, REF_EINVAL = -1, REF_ENOMEM = -2, REF_ENONFINITE = -4, REF_ESTATE = -5 };
enum { REF_STORE_F32 = 0, REF_STORE_F16 = 1, REF_STORE_F16_SR = 2, REF_STORE_INPLACE = 0x100 };
enum { REF_BC_PERIODIC = 0, REF_BC_WALLS_Y = 1 };
typedef struct {
  int32_t nx, ny;
  int32_t storage;
  float codec_scale;
} ref_grid;
typedef struct {
  int32_t kind;
  double force[2];
  double b_wall[2];
} ref_bc;

typedef struct {
  orc *o;
  int nx, ny;
  int ready;
} ref_handle;

/* The storage kind is accepted as the boundary accepts it; the oracle keeps
 * FP64 populations whatever it says.  The stream argument is ignored: every
 * call completes before it returns. */
int rrmhd_create(const ref_grid *g, double tau_f, double tau_m, const ref_bc *bc,
                 void *stream, ref_handle **out) {
  (void)stream;
  if (!out) return REF_EINVAL;
  *out = NULL;
  if (!g || g->nx < 1 || g->ny < 1) return REF_EINVAL;
  const int kind = g->storage & 0xff, flags = g->storage & ~0xff;
  if ((kind != REF_STORE_F32 && kind != REF_STORE_F16 && kind != REF_STORE_F16_SR) ||
      (flags != 0 && flags != REF_STORE_INPLACE))
    return REF_EINVAL;
  if (!isfinite(tau_f) || !isfinite(tau_m) || tau_f <= 0.5 || tau_m <= 0.5) return REF_EINVAL;
  ref_bc b = {REF_BC_PERIODIC, {0.0, 0.0}, {0.0, 0.0}};
  if (bc) b = *bc;
  if (b.kind != REF_BC_PERIODIC && b.kind != REF_BC_WALLS_Y) return REF_EINVAL;
  if (b.kind == REF_BC_WALLS_Y && g->ny < 2) return REF_EINVAL;
  for (int k = 0; k < 2; ++k)
    if (!isfinite(b.force[k]) || !isfinite(b.b_wall[k])) return REF_EINVAL;
  ref_handle *h = (ref_handle *)calloc(1, sizeof(ref_handle));
  if (!h) return REF_ENOMEM;
  h->o = orc_create(g->nx, g->ny, tau_f, tau_m, b.kind == REF_BC_WALLS_Y, b.force[0],
                    b.force[1], b.b_wall[0], b.b_wall[1], 0);
  if (!h->o) {
    free(h);
    return REF_ENOMEM;
  }
  h->nx = g->nx;
  h->ny = g->ny;
  *out = h;
  return REF_OK;
}

int rrmhd_init(ref_handle *h, const double *u, const double *b) {
  if (!h || !u || !b) return REF_EINVAL;
  orc_init(h->o, u, b);
  h->ready = 1;
  return REF_OK;
}

int rrmhd_step(ref_handle *h, int64_t n) {
  if (!h || n < 0) return REF_EINVAL;
  if (!h->ready) return REF_ESTATE;
  orc_step(h->o, (long)n);
  return REF_OK;
}

int rrmhd_moments(ref_handle *h, double *rho, double *u, double *b) {
  if (!h) return REF_EINVAL;
  if (!h->ready) return REF_ESTATE;
  orc_moments(h->o, rho, u, b);
  return REF_OK;
}

int rrmhd_diagnostics(ref_handle *h, double *E_kin, double *E_mag, double *max_div_b) {
  if (!h) return REF_EINVAL;
  if (!h->ready) return REF_ESTATE;
  double r[3];
  orc_diagnostics(h->o, r);
  const int bad = !(isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]));
  if (E_kin) *E_kin = bad ? NAN : r[0];
  if (E_mag) *E_mag = bad ? NAN : r[1];
  if (max_div_b) *max_div_b = bad ? NAN : r[2];
  return bad ? REF_ENONFINITE : REF_OK;
}

int rrmhd_invariants(ref_handle *h, double out[5]) {
  if (!h || !out) return REF_EINVAL;
  if (!h->ready) return REF_ESTATE;
  orc_invariants(h->o, out);
  return REF_OK;
}

int rrmhd_step_count(const ref_handle *h, int64_t *out) {
  if (!h || !out) return REF_EINVAL;
  *out = h->ready ? (int64_t)orc_step_count(h->o) : 0;
  return REF_OK;
}

int rrmhd_destroy(ref_handle *h) {
  if (!h) return REF_OK;
  orc_destroy(h->o);
  free(h);
  return REF_OK;
}

const char *rrmhd_strerror(int code) {
  switch (code) {
    case REF_OK: return "ok";
    case REF_EINVAL: return "invalid argument";
    case REF_ENOMEM: return "out of memory";
    case REF_ENONFINITE: return "non-finite diagnostic";
    case REF_ESTATE: return "invalid state (not initialised)";
    default: return "unknown error";
  }
}
