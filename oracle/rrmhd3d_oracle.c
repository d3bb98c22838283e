/* rrmhd3d_oracle.c -- plain FP64 CPU oracle of the three-dimensional
 * extension of the recursive regularised LB-MHD step.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): used by tests/ and by
 * nothing on the product path; shares no code with the HIP library.
 *
 * The paper treats two dimensions (D2Q9 fluid, D2Q5 magnetic lattice) and
 * names the extension to three-dimensional lattices as the next step
 * (Conclusions) without giving its equations.  This oracle takes the direct
 * generalisation of the algorithm of Sec. II.B, each step written in general
 * tensor form:
 *   - fluid lattice D3Q27 (the tensor product of three D1Q3 lattices, weights
 *     2/3 and 1/6 per direction, c_s^2 = 1/3);
 *   - equilibrium: the Hermite series w_i sum_n a0^(n):H^(n)/(n! c_s^2n)
 *     (Eq. fistar_acoeff) over every D3Q27-supported component up to sixth
 *     order, with a0^(n) = rho u...u and the Maxwell stress
 *     M = |b|^2/2 I - b b added at second order only, as task 2 of the
 *     algorithm does in two dimensions;
 *   - non-equilibrium: a1^(2) = sum_i H^(2)_i (f_i - f_eq,i) (projection, task
 *     3), then for n = 3..6 the recursion
 *       a1^(n)_{a1..an} = u_an a1^(n-1)_{a1..a(n-1)}
 *                         + sum_{j<n} (prod_{k != j, n} u_ak) a1^(2)_{aj an}
 *     (the recursion of task 3 in its general form), restricted to supported
 *     components in the reconstruction (task 4);
 *   - collision f* = f_eq + (1 - omega) f_neq,reg (task 5);
 *   - magnetic lattice D3Q7 with weights psi_0 = 1/4, psi_j = 1/8 (so
 *     sum_j psi_j e_ja e_jb = c_m^2 delta_ab with c_m^2 = 1/4), vector BGK with
 *     g_eq,j = psi_j [b + e_j.(u b - b u) / c_m^2] (the equilibrium of
 *     Sec. II.A with the lattice's own c_m^2);
 *   - push streaming with periodic wrap in x, y and z (task 6).
 * A D3Q27-supported component is an index tuple in which no direction occurs
 * more than twice (H_xxx and higher powers alias on the lattice).
 *
 * Velocity order: i = 9 (c_x + 1) + 3 (c_y + 1) + (c_z + 1).  Magnetic order:
 * j = 0 rest, 1 +x, 2 -x, 3 +y, 4 -y, 5 +z, 6 -z.  Layout of the grid:
 * f[i][z][y][x], g[j][component][z][y][x].
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q3 27
#define QM3 7
#define CS2 (1.0 / 3.0)
#define CM2 0.25

static int C3[Q3][3];
static double W3[Q3];
static const int E3[QM3][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0},
                               {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
static const double PSI3[QM3] = {0.25, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125};

/* supported index tuples of each order n = 0..6, as base-3 codes */
#define MAXN 6
static int ntup[MAXN + 1];
static int tup[MAXN + 1][729][MAXN];
/* H^(n) of every velocity at every supported tuple */
static double Htab[MAXN + 1][729][Q3];
static int tables_ready = 0;

static double w1(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }

/* H^(n)_{idx}(c): sum over sets of disjoint pairs of index positions of
 * (-c_s^2)^(pairs) prod_pairs delta prod_unpaired c (the Hermite tensor
 * polynomial of the lattice Boltzmann expansion). */
static double herm_rec(const int *idx, int n, int used, const int c[3]) {
  int p = 0;
  while (p < n && (used >> p & 1)) ++p;
  if (p == n) return 1.0;
  const int u1 = used | (1 << p);
  double s = (double)c[idx[p]] * herm_rec(idx, n, u1, c);
  for (int q = p + 1; q < n; ++q) {
    if (u1 >> q & 1) continue;
    if (idx[p] != idx[q]) continue;
    s += -CS2 * herm_rec(idx, n, u1 | (1 << q), c);
  }
  return s;
}

double orc3d_hermite(int n, const int *idx, int i) { return herm_rec(idx, n, 0, C3[i]); }

static int is_supported(const int *idx, int n) {
  int cnt[3] = {0, 0, 0};
  for (int k = 0; k < n; ++k) cnt[idx[k]]++;
  return cnt[0] <= 2 && cnt[1] <= 2 && cnt[2] <= 2;
}

static double fact(int n) {
  double f = 1.0;
  for (int k = 2; k <= n; ++k) f *= k;
  return f;
}

static void build_tables(void) {
  if (tables_ready) return;
  for (int i = 0; i < Q3; ++i) {
    C3[i][0] = i / 9 - 1;
    C3[i][1] = (i / 3) % 3 - 1;
    C3[i][2] = i % 3 - 1;
    W3[i] = w1(C3[i][0]) * w1(C3[i][1]) * w1(C3[i][2]);
  }
  for (int n = 0; n <= MAXN; ++n) {
    int total = 1;
    for (int k = 0; k < n; ++k) total *= 3;
    ntup[n] = 0;
    for (int code = 0; code < total; ++code) {
      int idx[MAXN];
      int v = code;
      for (int k = n - 1; k >= 0; --k) {
        idx[k] = v % 3;
        v /= 3;
      }
      if (!is_supported(idx, n)) continue;
      const int t = ntup[n]++;
      memcpy(tup[n][t], idx, sizeof(int) * (size_t)(n ? n : 1));
      for (int i = 0; i < Q3; ++i) Htab[n][t][i] = herm_rec(idx, n, 0, C3[i]);
    }
  }
  tables_ready = 1;
}

void orc3d_lattice(int *c, double *w) {
  build_tables();
  for (int i = 0; i < Q3; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = C3[i][a];
    w[i] = W3[i];
  }
}

static void maxwell3(const double b[3], double M[3][3]) {
  const double b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) M[a][c] = (a == c ? 0.5 * b2 : 0.0) - b[a] * b[c];
}

/* equilibrium as the Hermite series over supported components */
static void feq3(double rho, const double u[3], const double b[3], double feq[Q3]) {
  double M[3][3];
  maxwell3(b, M);
  for (int i = 0; i < Q3; ++i) {
    double s = 0.0;
    for (int n = 0; n <= MAXN; ++n) {
      double sn = 0.0;
      for (int t = 0; t < ntup[n]; ++t) {
        double a0 = rho;
        for (int k = 0; k < n; ++k) a0 *= u[tup[n][t][k]];
        if (n == 2) a0 += M[tup[n][t][0]][tup[n][t][1]];
        sn += a0 * Htab[n][t][i];
      }
      s += sn / (fact(n) * pow(CS2, n));
    }
    feq[i] = W3[i] * s;
  }
}

static void geq3(const double u[3], const double b[3], double geq[3 * QM3]) {
  for (int j = 0; j < QM3; ++j)
    for (int a = 0; a < 3; ++a) {
      double s = b[a];
      for (int c = 0; c < 3; ++c) s += E3[j][c] * (u[c] * b[a] - u[a] * b[c]) / CM2;
      geq[3 * j + a] = PSI3[j] * s;
    }
}

/* aux layout (for the node API): rho, u[3], b[3], a2[9], a3[27], a4[81],
 * a5[243], a6[729], feq[27], geq[21], fneq_reg[27] */
#define AUX3 (1 + 3 + 3 + 9 + 27 + 81 + 243 + 729 + 27 + 21 + 27)

static void collide3(const double *f, const double *g, double omega, double omega_m, double *fs,
                     double *gs, double *aux) {
  double rho = 0.0, j[3] = {0, 0, 0}, b[3] = {0, 0, 0};
  for (int i = 0; i < Q3; ++i) {
    rho += f[i];
    for (int a = 0; a < 3; ++a) j[a] += C3[i][a] * f[i];
  }
  double u[3];
  for (int a = 0; a < 3; ++a) u[a] = j[a] / rho;
  for (int q = 0; q < QM3; ++q)
    for (int a = 0; a < 3; ++a) b[a] += g[3 * q + a];
  double feq[Q3], geq[3 * QM3];
  feq3(rho, u, b, feq);
  geq3(u, b, geq);
  /* a1^(n) as full tensors, n = 2..6 (index code in base 3) */
  static const int sizes[MAXN + 1] = {1, 3, 9, 27, 81, 243, 729};
  double *an[MAXN + 1];
  double buf[9 + 27 + 81 + 243 + 729];
  an[2] = buf;
  an[3] = an[2] + 9;
  an[4] = an[3] + 27;
  an[5] = an[4] + 81;
  an[6] = an[5] + 243;
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) {
      int idx[2] = {a, c};
      double s = 0.0;
      for (int i = 0; i < Q3; ++i) s += herm_rec(idx, 2, 0, C3[i]) * (f[i] - feq[i]);
      an[2][3 * a + c] = s;
    }
  for (int n = 3; n <= MAXN; ++n) {
    for (int code = 0; code < sizes[n]; ++code) {
      int idx[MAXN];
      int v = code;
      for (int k = n - 1; k >= 0; --k) {
        idx[k] = v % 3;
        v /= 3;
      }
      const int last = idx[n - 1];
      double s = u[last] * an[n - 1][code / 3];
      for (int jj = 0; jj < n - 1; ++jj) {
        double p = 1.0;
        for (int k = 0; k < n - 1; ++k)
          if (k != jj) p *= u[idx[k]];
        s += p * an[2][3 * idx[jj] + last];
      }
      an[n][code] = s;
    }
  }
  double fneq[Q3];
  for (int i = 0; i < Q3; ++i) {
    double s = 0.0;
    for (int n = 2; n <= MAXN; ++n) {
      double sn = 0.0;
      for (int t = 0; t < ntup[n]; ++t) {
        int code = 0;
        for (int k = 0; k < n; ++k) code = 3 * code + tup[n][t][k];
        sn += an[n][code] * Htab[n][t][i];
      }
      s += sn / (fact(n) * pow(CS2, n));
    }
    fneq[i] = W3[i] * s;
  }
  for (int i = 0; i < Q3; ++i) fs[i] = feq[i] + (1.0 - omega) * fneq[i];
  for (int k = 0; k < 3 * QM3; ++k) gs[k] = geq[k] + (1.0 - omega_m) * (g[k] - geq[k]);
  if (aux) {
    double *p = aux;
    *p++ = rho;
    for (int a = 0; a < 3; ++a) *p++ = u[a];
    for (int a = 0; a < 3; ++a) *p++ = b[a];
    for (int n = 2; n <= MAXN; ++n)
      for (int k = 0; k < sizes[n]; ++k) *p++ = an[n][k];
    for (int i = 0; i < Q3; ++i) *p++ = feq[i];
    for (int k = 0; k < 3 * QM3; ++k) *p++ = geq[k];
    for (int i = 0; i < Q3; ++i) *p++ = fneq[i];
  }
}

int orc3d_aux_size(void) { return AUX3; }

void orc3d_node_equilibrium(double rho, const double u[3], const double b[3], double feq[Q3],
                            double geq[3 * QM3]) {
  build_tables();
  feq3(rho, u, b, feq);
  geq3(u, b, geq);
}

void orc3d_node_collide(const double f[Q3], const double g[3 * QM3], double omega,
                        double omega_m, double fs[Q3], double gs[3 * QM3], double *aux) {
  build_tables();
  collide3(f, g, omega, omega_m, fs, gs, aux);
}

/* ---- grid ------------------------------------------------------------------ */
typedef struct {
  int nx, ny, nz;
  long n;
  double omega, omega_m;
  double *f, *g, *f2, *g2;
  long step;
} orc3d;

orc3d *orc3d_create(int nx, int ny, int nz, double tau_f, double tau_m) {
  if (nx < 1 || ny < 1 || nz < 1 || !(tau_f > 0.5) || !(tau_m > 0.5)) return NULL;
  build_tables();
  orc3d *h = (orc3d *)calloc(1, sizeof(orc3d));
  h->nx = nx;
  h->ny = ny;
  h->nz = nz;
  h->n = (long)nx * ny * nz;
  h->omega = 1.0 / tau_f;
  h->omega_m = 1.0 / tau_m;
  h->f = (double *)calloc((size_t)(Q3 * h->n), sizeof(double));
  h->f2 = (double *)calloc((size_t)(Q3 * h->n), sizeof(double));
  h->g = (double *)calloc((size_t)(3 * QM3 * h->n), sizeof(double));
  h->g2 = (double *)calloc((size_t)(3 * QM3 * h->n), sizeof(double));
  return h;
}

void orc3d_destroy(orc3d *h) {
  if (!h) return;
  free(h->f);
  free(h->f2);
  free(h->g);
  free(h->g2);
  free(h);
}

/* u, b: [3][nz][ny][nx]; rho = 1, populations at equilibrium */
void orc3d_init(orc3d *h, const double *u, const double *b) {
  const long N = h->n;
#pragma omp parallel for schedule(static)
  for (long p = 0; p < N; ++p) {
    double uu[3] = {u[p], u[N + p], u[2 * N + p]}, bb[3] = {b[p], b[N + p], b[2 * N + p]};
    double feq[Q3], geq[3 * QM3];
    feq3(1.0, uu, bb, feq);
    geq3(uu, bb, geq);
    for (int i = 0; i < Q3; ++i) h->f[i * N + p] = feq[i];
    for (int k = 0; k < 3 * QM3; ++k) h->g[k * N + p] = geq[k];
  }
  h->step = 0;
}

static int wrap3(int v, int n) { return ((v % n) + n) % n; }

static void one_step3(orc3d *h) {
  const long N = h->n;
  const int nx = h->nx, ny = h->ny, nz = h->nz;
#pragma omp parallel for schedule(static)
  for (long p = 0; p < N; ++p) {
    const int x = (int)(p % nx), y = (int)((p / nx) % ny), z = (int)(p / ((long)nx * ny));
    double f[Q3], g[3 * QM3], fs[Q3], gs[3 * QM3];
    for (int i = 0; i < Q3; ++i) f[i] = h->f[i * N + p];
    for (int k = 0; k < 3 * QM3; ++k) g[k] = h->g[k * N + p];
    collide3(f, g, h->omega, h->omega_m, fs, gs, NULL);
    for (int i = 0; i < Q3; ++i) {
      const long q = ((long)wrap3(z + C3[i][2], nz) * ny + wrap3(y + C3[i][1], ny)) * nx +
                     wrap3(x + C3[i][0], nx);
      h->f2[i * N + q] = fs[i];
    }
    for (int jj = 0; jj < QM3; ++jj) {
      const long q = ((long)wrap3(z + E3[jj][2], nz) * ny + wrap3(y + E3[jj][1], ny)) * nx +
                     wrap3(x + E3[jj][0], nx);
      for (int a = 0; a < 3; ++a) h->g2[(3 * jj + a) * N + q] = gs[3 * jj + a];
    }
  }
  double *t = h->f;
  h->f = h->f2;
  h->f2 = t;
  t = h->g;
  h->g = h->g2;
  h->g2 = t;
  h->step++;
}

void orc3d_step(orc3d *h, long n) {
  for (long k = 0; k < n; ++k) one_step3(h);
}

long orc3d_step_count(const orc3d *h) { return h->step; }

/* rho [nz][ny][nx]; u, b [3][nz][ny][nx]; any may be NULL */
void orc3d_moments(const orc3d *h, double *rho, double *u, double *b) {
  const long N = h->n;
#pragma omp parallel for schedule(static)
  for (long p = 0; p < N; ++p) {
    double r = 0.0, j[3] = {0, 0, 0}, bb[3] = {0, 0, 0};
    for (int i = 0; i < Q3; ++i) {
      const double v = h->f[i * N + p];
      r += v;
      for (int a = 0; a < 3; ++a) j[a] += C3[i][a] * v;
    }
    for (int q = 0; q < QM3; ++q)
      for (int a = 0; a < 3; ++a) bb[a] += h->g[(3 * q + a) * N + p];
    if (rho) rho[p] = r;
    for (int a = 0; a < 3; ++a) {
      if (u) u[a * N + p] = j[a] / r;
      if (b) b[a * N + p] = bb[a];
    }
  }
}

/* E_kin = sum |u|^2 / (2N), E_mag = sum |b|^2 / (2N), max |div b| with the
 * isotropic lattice gradient d_a phi = (1/c_s^2) sum_i w_i c_ia phi(x + c_i)
 * (the gradient of Sec. III on D3Q27). */
void orc3d_diagnostics(const orc3d *h, double out[3]) {
  const long N = h->n;
  double *rho = (double *)malloc(sizeof(double) * (size_t)N);
  double *u = (double *)malloc(sizeof(double) * (size_t)(3 * N));
  double *b = (double *)malloc(sizeof(double) * (size_t)(3 * N));
  orc3d_moments(h, rho, u, b);
  double ek = 0.0, em = 0.0, mx = 0.0;
  for (long p = 0; p < N; ++p)
    for (int a = 0; a < 3; ++a) {
      ek += u[a * N + p] * u[a * N + p];
      em += b[a * N + p] * b[a * N + p];
    }
  for (long p = 0; p < N; ++p) {
    const int x = (int)(p % h->nx), y = (int)((p / h->nx) % h->ny),
              z = (int)(p / ((long)h->nx * h->ny));
    double s = 0.0;
    for (int i = 0; i < Q3; ++i) {
      const long q = ((long)wrap3(z + C3[i][2], h->nz) * h->ny + wrap3(y + C3[i][1], h->ny)) *
                         h->nx + wrap3(x + C3[i][0], h->nx);
      for (int a = 0; a < 3; ++a) s += W3[i] * C3[i][a] * b[a * N + q];
    }
    const double d = fabs(s / CS2);
    if (d > mx || d != d) mx = d;
  }
  out[0] = ek / (2.0 * N);
  out[1] = em / (2.0 * N);
  out[2] = mx;
  free(rho);
  free(u);
  free(b);
}

/* mass, sum rho u (3), sum b (3) */
void orc3d_invariants(const orc3d *h, double out[7]) {
  const long N = h->n;
  for (int k = 0; k < 7; ++k) out[k] = 0.0;
  for (long p = 0; p < N; ++p) {
    for (int i = 0; i < Q3; ++i) {
      const double v = h->f[i * N + p];
      out[0] += v;
      for (int a = 0; a < 3; ++a) out[1 + a] += C3[i][a] * v;
    }
    for (int q = 0; q < QM3; ++q)
      for (int a = 0; a < 3; ++a) out[4 + a] += h->g[(3 * q + a) * N + p];
  }
}
