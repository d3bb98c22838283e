/*
 * Plain FP64 CPU oracle for the recursive regularised lattice Boltzmann
 * method for 2D incompressible MHD (De Rosis, "Recursive regularised lattice
 * Boltzmann method for magnetohydrodynamics", arXiv 2602.14667).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so and may
 * be loaded only by the test-suite, by the smoke check and by the benchmark's
 * CPU-baseline leg.  It shares no code, header, table or constant with the HIP
 * library, and nothing on the product path calls it.
 *
 * The code follows the paper's "Algorithm of computation" (Sec. II.B) task by
 * task, with generic Hermite tensors over {x,y}^n taken from their definition
 * (Sec. II.A) and an explicit D2Q9 support mask.  It is deliberately slow and
 * plain: no fusion, no blocking, no precision tricks.
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *   - the fourth-order equilibrium term H_xxyy u_x^2 u_y^2 carries the factor
 *     1/(4 c_s^8) that the general series w_i sum_n a:H/(n! c_s^{2n}) gives
 *     (the printed equilibrium shows no coefficient);
 *   - the Maxwell stress enters the equilibrium at second order only, as in
 *     the equilibrium used by the algorithm (task 2); the full series with the
 *     u.M cross terms of the equilibrium Hermite coefficients is available as
 *     FEQ_SERIES_FULL for ablations only;
 *   - the regularised third/fourth-order sums keep only the tensor components
 *     that D2Q9 supports (no index repeated three or more times), i.e. the
 *     xxy, xyy and xxyy families that the printed equilibrium keeps;
 *   - the state is the pre-collision population set; a step is collide then
 *     stream; initialisation is the equilibrium of (rho=1, u, b);
 *   - walls and forcing (not in the paper): half-way bounce-back for f,
 *     anti-bounce-back with a prescribed wall field for g, Guo-type forcing
 *     with the first-order non-equilibrium coefficient kept in the
 *     reconstruction.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- Sec. II.A: lattices ------------------------------------------------ */
/* D2Q9 velocities in Latt's ordering and their weights. */
static const int CI[9][2] = {{0, 0},  {-1, 1}, {-1, 0}, {-1, -1}, {0, -1},
                             {1, -1}, {1, 0},  {1, 1},  {0, 1}};
static const double WI[9] = {4.0 / 9.0,  1.0 / 36.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 9.0,  1.0 / 36.0, 1.0 / 9.0};
/* D2Q5 velocities for the vector magnetic populations and their weights. */
static const int EJ[5][2] = {{0, 0}, {-1, 0}, {0, -1}, {1, 0}, {0, 1}};
static const double PSI[5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0,
                              1.0 / 6.0};
/* Lattice sound speed squared, c_s = 1/sqrt(3). */
static const double CS2 = 1.0 / 3.0;

enum { FEQ_ALGORITHM = 0, FEQ_SERIES_FULL = 1 };

static int delta(int a, int b) { return a == b ? 1 : 0; }

/* Index of the D2Q9 velocity opposite to c_i, found by search. */
static int opposite_f(int i) {
  for (int k = 0; k < 9; ++k)
    if (CI[k][0] == -CI[i][0] && CI[k][1] == -CI[i][1]) return k;
  return -1;
}

/* Index of the D2Q5 velocity opposite to e_j, found by search. */
static int opposite_g(int j) {
  for (int k = 0; k < 5; ++k)
    if (EJ[k][0] == -EJ[j][0] && EJ[k][1] == -EJ[j][1]) return k;
  return -1;
}

/* ---- Sec. II.A: Hermite tensors from their definition ------------------- */
/* H^(n)_{i, idx[0..n-1]} for n = 0..4; idx entries are 0 (x) or 1 (y). */
double orc_hermite(int n, const int *idx, int i) {
  const int *c = CI[i];
  if (n == 0) return 1.0;
  if (n == 1) return c[idx[0]];
  if (n == 2) {
    int a = idx[0], b = idx[1];
    return c[a] * c[b] - CS2 * delta(a, b);
  }
  if (n == 3) {
    int a = idx[0], b = idx[1], g = idx[2];
    return c[a] * c[b] * c[g] -
           CS2 * (c[a] * delta(b, g) + c[b] * delta(a, g) + c[g] * delta(a, b));
  }
  if (n == 4) {
    int a = idx[0], b = idx[1], g = idx[2], d = idx[3];
    /* the six ways of pairing two indices into a Kronecker delta */
    double cc_delta = c[a] * c[b] * delta(g, d) + c[a] * c[g] * delta(b, d) +
                      c[a] * c[d] * delta(b, g) + c[b] * c[g] * delta(a, d) +
                      c[b] * c[d] * delta(a, g) + c[g] * c[d] * delta(a, b);
    /* the three pairings of four indices into two deltas */
    double dd = delta(a, b) * delta(g, d) + delta(a, g) * delta(b, d) +
                delta(a, d) * delta(b, g);
    return (double)(c[a] * c[b] * c[g] * c[d]) - CS2 * cc_delta +
           CS2 * CS2 * dd;
  }
  return 0.0;
}

/* D2Q9 support mask: a tensor component is kept when no Cartesian direction
 * is repeated three or more times (c^3 = c on D2Q9, so such components are
 * aliases of lower orders). */
static int supported(int n, const int *idx) {
  int nx = 0, ny = 0;
  for (int k = 0; k < n; ++k) {
    if (idx[k] == 0)
      ++nx;
    else
      ++ny;
  }
  return nx <= 2 && ny <= 2;
}

/* Tables of H^(2), H^(3), H^(4) for every velocity and index tuple, filled
 * once from orc_hermite so that the per-node loops stay readable. */
static double H2T[9][2][2], H3T[9][2][2][2], H4T[9][2][2][2][2];
static int tables_ready = 0;

static void build_tables(void) {
  if (tables_ready) return;
  for (int i = 0; i < 9; ++i)
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        int i2[2] = {a, b};
        H2T[i][a][b] = orc_hermite(2, i2, i);
        for (int g = 0; g < 2; ++g) {
          int i3[3] = {a, b, g};
          H3T[i][a][b][g] = orc_hermite(3, i3, i);
          for (int d = 0; d < 2; ++d) {
            int i4[4] = {a, b, g, d};
            H4T[i][a][b][g][d] = orc_hermite(4, i4, i);
          }
        }
      }
  tables_ready = 1;
}

static double fact(int n) {
  double r = 1.0;
  for (int k = 2; k <= n; ++k) r *= k;
  return r;
}

/* ---- Maxwell stress tensor M = |b|^2 delta / 2 - b b (Sec. II.B) -------- */
static void maxwell(const double b[2], double M[2][2]) {
  double b2 = b[0] * b[0] + b[1] * b[1];
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 2; ++c) M[a][c] = 0.5 * b2 * delta(a, c) - b[a] * b[c];
}

/* ---- Algorithm task 2: equilibria --------------------------------------- */
/* Fourth-order fluid equilibrium in the form the algorithm uses (Eq. feq_4th
 * with the 1/(4 c_s^8) reading), Maxwell stress at second order. */
static void feq_algorithm(double rho, const double u[2], const double b[2],
                          double feq[9]) {
  const int ixxy[3] = {0, 0, 1}, ixyy[3] = {0, 1, 1}, ixxyy[4] = {0, 0, 1, 1};
  double b2 = b[0] * b[0] + b[1] * b[1];
  for (int i = 0; i < 9; ++i) {
    double cu = 0.0, H2uu = 0.0;
    for (int a = 0; a < 2; ++a) {
      cu += orc_hermite(1, &a, i) * u[a];
      for (int c = 0; c < 2; ++c) H2uu += H2T[i][a][c] * u[a] * u[c];
    }
    double third = (orc_hermite(3, ixxy, i) * u[0] * u[0] * u[1] +
                    orc_hermite(3, ixyy, i) * u[0] * u[1] * u[1]) /
                   (2.0 * CS2 * CS2 * CS2);
    double fourth = orc_hermite(4, ixxyy, i) * u[0] * u[0] * u[1] * u[1] /
                    (4.0 * CS2 * CS2 * CS2 * CS2);
    double bracket =
        1.0 + cu / CS2 + H2uu / (2.0 * CS2 * CS2) + third + fourth;
    double c2 = (double)(CI[i][0] * CI[i][0] + CI[i][1] * CI[i][1]);
    double cb = CI[i][0] * b[0] + CI[i][1] * b[1];
    double mx = WI[i] / (2.0 * CS2 * CS2) * (0.5 * b2 * c2 - cb * cb);
    feq[i] = WI[i] * rho * bracket + mx;
  }
}

/* Equilibrium as the Hermite series w_i sum_n a0^(n):H^(n)/(n! c_s^{2n})
 * (the equilibrium part of Eq. fistar_acoeff) over the supported components,
 * with the equilibrium coefficients of Eq. eq:a0_4.  With full = 0 the Maxwell
 * tensor enters a0^(2) only; with full = 1 the u.M cross terms of a0^(3) and
 * a0^(4) are included as well. */
static void feq_series(double rho, const double u[2], const double b[2],
                       int full, double feq[9]) {
  double M[2][2];
  maxwell(b, M);
  double mfull = full ? 1.0 : 0.0;
  for (int i = 0; i < 9; ++i) {
    double s = rho; /* n = 0 */
    for (int a = 0; a < 2; ++a) s += rho * u[a] * CI[i][a] / CS2;
    double s2 = 0.0, s3 = 0.0, s4 = 0.0;
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 2; ++c) {
        s2 += (rho * u[a] * u[c] + M[a][c]) * H2T[i][a][c];
        for (int g = 0; g < 2; ++g) {
          int i3[3] = {a, c, g};
          if (supported(3, i3)) {
            double a3 = rho * u[a] * u[c] * u[g] +
                        mfull * (u[a] * M[c][g] + u[c] * M[a][g] +
                                 u[g] * M[a][c]);
            s3 += a3 * H3T[i][a][c][g];
          }
          for (int d = 0; d < 2; ++d) {
            int i4[4] = {a, c, g, d};
            if (!supported(4, i4)) continue;
            double a4 = rho * u[a] * u[c] * u[g] * u[d] +
                        mfull * (u[a] * u[c] * M[g][d] + u[a] * u[g] * M[c][d] +
                                 u[a] * u[d] * M[c][g] + u[c] * u[g] * M[a][d] +
                                 u[c] * u[d] * M[a][g] + u[g] * u[d] * M[a][c]);
            s4 += a4 * H4T[i][a][c][g][d];
          }
        }
      }
    s += s2 / (fact(2) * CS2 * CS2) + s3 / (fact(3) * CS2 * CS2 * CS2) +
         s4 / (fact(4) * CS2 * CS2 * CS2 * CS2);
    feq[i] = WI[i] * s;
  }
}

/* Magnetic equilibrium g_eq,j,alpha = psi_j [b_alpha + e_j,beta (u_beta
 * b_alpha - u_alpha b_beta) / c_s^2] (Sec. II.A, algorithm task 2). */
static void geq_vector(const double u[2], const double b[2], double geq[10]) {
  for (int j = 0; j < 5; ++j)
    for (int a = 0; a < 2; ++a) {
      double s = b[a];
      for (int c = 0; c < 2; ++c)
        s += EJ[j][c] * (u[c] * b[a] - u[a] * b[c]) / CS2;
      geq[2 * j + a] = PSI[j] * s;
    }
}

/* Auxiliary per-node quantities exposed for single-node tests. */
typedef struct {
  double rho, u[2], b[2];
  double a1[2];          /* first-order non-equilibrium coefficient */
  double a2[2][2];       /* second-order coefficient a_1^(2) */
  double a3[2][2][2];    /* recursive third-order coefficient */
  double a4[2][2][2][2]; /* recursive fourth-order coefficient */
  double feq[9], geq[10], fneq_reg[9];
} node_aux;

/* One collision at one node: algorithm tasks 1-5.  f[9], g[10] (g[2j+c]) are
 * the pre-collision populations; G is the body force per unit mass (zero in
 * the paper).  Outputs the post-collision populations fs, gs. */
/* Learned closure (a project addition; the paper has none): an MLP maps the
 * node's pre-collision (rho, u, b, a_1^(2)) to a correction of a_1^(2) that
 * is added before the recursion of task 3.  Defined further below. */
typedef struct closure closure;
static void closure_apply(const closure *c, double rho, const double u[2],
                          const double b[2], double a2[2][2]);

static void collide_node_c(const double *f, const double *g, double omega,
                           double omega_m, const double G[2], int feq_option,
                           const closure *cl, const double *dnode, double *fs,
                           double *gs, node_aux *ax);

static void collide_node(const double *f, const double *g, double omega,
                         double omega_m, const double G[2], int feq_option,
                         double *fs, double *gs, node_aux *ax) {
  collide_node_c(f, g, omega, omega_m, G, feq_option, NULL, NULL, fs, gs, ax);
}

/* Tasks 3 (recursion) and 4 without the weight: r[i] such that the
 * regularised non-equilibrium population is w_i r[i], from the velocity and
 * a_1^(2); a3, a4 receive the recursive coefficients.  Only the
 * D2Q9-supported index sets enter the sums. */
static void reg_expand(const double u[2], const double a2[2][2],
                       double a3[2][2][2], double a4[2][2][2][2], double r[9]) {
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 2; ++c)
      for (int g3 = 0; g3 < 2; ++g3)
        a3[a][c][g3] = u[a] * a2[c][g3] + u[c] * a2[a][g3] + u[g3] * a2[a][c];
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 2; ++c)
      for (int g3 = 0; g3 < 2; ++g3)
        for (int d = 0; d < 2; ++d)
          a4[a][c][g3][d] =
              u[a] * a3[c][g3][d] + u[c] * a3[a][g3][d] + u[g3] * a3[a][c][d] +
              u[d] * a3[a][c][g3] -
              (u[a] * u[c] * a2[g3][d] + u[a] * u[g3] * a2[c][d] +
               u[a] * u[d] * a2[c][g3] + u[c] * u[g3] * a2[a][d] +
               u[c] * u[d] * a2[a][g3] + u[g3] * u[d] * a2[a][c]);
  for (int i = 0; i < 9; ++i) {
    double s2 = 0.0, s3 = 0.0, s4 = 0.0;
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 2; ++c) {
        s2 += a2[a][c] * H2T[i][a][c];
        for (int g3 = 0; g3 < 2; ++g3) {
          int i3[3] = {a, c, g3};
          if (supported(3, i3)) s3 += a3[a][c][g3] * H3T[i][a][c][g3];
          for (int d = 0; d < 2; ++d) {
            int i4[4] = {a, c, g3, d};
            if (supported(4, i4)) s4 += a4[a][c][g3][d] * H4T[i][a][c][g3][d];
          }
        }
      }
    r[i] = s2 / (2.0 * CS2 * CS2) + s3 / (6.0 * CS2 * CS2 * CS2) +
           s4 / (24.0 * CS2 * CS2 * CS2 * CS2);
  }
}

static void collide_node_c(const double *f, const double *g, double omega,
                           double omega_m, const double G[2], int feq_option,
                           const closure *cl, const double *dnode, double *fs,
                           double *gs, node_aux *ax) {
  node_aux local;
  node_aux *A = ax ? ax : &local;
  /* task 1: macroscopic variables */
  double rho = 0.0, j[2] = {0.0, 0.0}, b[2] = {0.0, 0.0};
  for (int i = 0; i < 9; ++i) {
    rho += f[i];
    for (int a = 0; a < 2; ++a) j[a] += f[i] * CI[i][a];
  }
  for (int q = 0; q < 5; ++q)
    for (int a = 0; a < 2; ++a) b[a] += g[2 * q + a];
  double F[2] = {rho * G[0], rho * G[1]};
  int forced = (G[0] != 0.0 || G[1] != 0.0);
  double u[2];
  /* forcing reading: the velocity carries half the force impulse */
  for (int a = 0; a < 2; ++a) u[a] = (j[a] + 0.5 * F[a]) / rho;

  /* task 2: equilibria */
  double feq[9], geq[10];
  if (feq_option == FEQ_SERIES_FULL)
    feq_series(rho, u, b, 1, feq);
  else
    feq_algorithm(rho, u, b, feq);
  geq_vector(u, b, geq);

  /* task 3: non-equilibrium Hermite coefficients */
  double a1[2] = {0.0, 0.0}, a2[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int i = 0; i < 9; ++i) {
    double fn = f[i] - feq[i];
    for (int a = 0; a < 2; ++a) {
      a1[a] += CI[i][a] * fn;
      for (int c = 0; c < 2; ++c) a2[a][c] += H2T[i][a][c] * fn;
    }
  }
  if (cl) closure_apply(cl, rho, u, b, a2);
  if (dnode) {
    /* a prescribed correction (dxx, dxy, dyy) of this node */
    a2[0][0] += dnode[0];
    a2[0][1] += dnode[1];
    a2[1][0] += dnode[1];
    a2[1][1] += dnode[2];
  }
  double a3[2][2][2], a4[2][2][2][2], rr[9];
  reg_expand(u, (const double(*)[2])a2, a3, a4, rr);

  /* task 4: regularised non-equilibrium populations (Eq. fineq_reg) */
  double fneq[9];
  for (int i = 0; i < 9; ++i) {
    double r = rr[i];
    /* forcing reading: the first-order term of the series, which vanishes
     * without a force, is kept when a force acts */
    if (forced) r += (CI[i][0] * a1[0] + CI[i][1] * a1[1]) / CS2;
    fneq[i] = WI[i] * r;
  }

  /* task 5: collision */
  for (int i = 0; i < 9; ++i) {
    fs[i] = feq[i] + (1.0 - omega) * fneq[i];
    if (forced) {
      /* Guo-type source (1 - omega/2) S_i with
       * S_i = w_i [c_i.F / c_s^2 + H2_i:(uF + Fu) / (2 c_s^4)] */
      double cF = CI[i][0] * F[0] + CI[i][1] * F[1];
      double HuF = 0.0;
      for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c)
          HuF += H2T[i][a][c] * (u[a] * F[c] + F[a] * u[c]);
      double S = WI[i] * (cF / CS2 + HuF / (2.0 * CS2 * CS2));
      fs[i] += (1.0 - 0.5 * omega) * S;
    }
  }
  for (int k = 0; k < 10; ++k) gs[k] = geq[k] + (1.0 - omega_m) * (g[k] - geq[k]);

  if (A) {
    A->rho = rho;
    memcpy(A->u, u, sizeof u);
    memcpy(A->b, b, sizeof b);
    memcpy(A->a1, a1, sizeof a1);
    memcpy(A->a2, a2, sizeof a2);
    memcpy(A->a3, a3, sizeof a3);
    memcpy(A->a4, a4, sizeof a4);
    memcpy(A->feq, feq, sizeof feq);
    memcpy(A->geq, geq, sizeof geq);
    memcpy(A->fneq_reg, fneq, sizeof fneq);
  }
}

/* ======================================================================== */
/* Grid state                                                                */
/* ======================================================================== */
typedef struct orc {
  int nx, ny;
  double tau_f, tau_m;
  int walls;       /* 0: doubly periodic; 1: walls at y = -1/2, ny - 1/2 */
  double G[2];     /* body force per unit mass */
  double bwall[2]; /* wall magnetic field for the anti-bounce-back */
  int feq_option;
  closure *cl;    /* NULL: plain method */
  const double *delta; /* NULL, or a prescribed a_1^(2) correction [ny][nx][3] */
  long step;
  double *f, *g;       /* f[i][y][x], g[j][c][y][x]: pre-collision state */
  double *fn, *gn;     /* scratch for the next state */
} orc;

#define FIDX(h, i, y, x) (((size_t)(i) * (h)->ny + (y)) * (h)->nx + (x))
#define GIDX(h, j, c, y, x) \
  ((((size_t)(j) * 2 + (c)) * (h)->ny + (y)) * (h)->nx + (x))

orc *orc_create(int nx, int ny, double tau_f, double tau_m, int walls,
                double Gx, double Gy, double bwx, double bwy, int feq_option) {
  if (nx < 1 || ny < 1 || tau_f <= 0.5 || tau_m <= 0.5) return NULL;
  if (walls && ny < 2) return NULL;
  build_tables();
  orc *h = (orc *)calloc(1, sizeof(orc));
  if (!h) return NULL;
  h->nx = nx;
  h->ny = ny;
  h->tau_f = tau_f;
  h->tau_m = tau_m;
  h->walls = walls;
  h->G[0] = Gx;
  h->G[1] = Gy;
  h->bwall[0] = bwx;
  h->bwall[1] = bwy;
  h->feq_option = feq_option;
  size_t n = (size_t)nx * ny;
  h->f = (double *)calloc(9 * n, sizeof(double));
  h->fn = (double *)calloc(9 * n, sizeof(double));
  h->g = (double *)calloc(10 * n, sizeof(double));
  h->gn = (double *)calloc(10 * n, sizeof(double));
  if (!h->f || !h->fn || !h->g || !h->gn) {
    free(h->f);
    free(h->fn);
    free(h->g);
    free(h->gn);
    free(h);
    return NULL;
  }
  return h;
}

void orc_destroy(orc *h) {
  if (!h) return;
  free(h->cl);
  free(h->f);
  free(h->fn);
  free(h->g);
  free(h->gn);
  free(h);
}

/* Initial state: equilibrium of (rho = 1, u, b); u, b are [2][ny][nx]. */
void orc_init(orc *h, const double *u, const double *b) {
  size_t n = (size_t)h->nx * h->ny;
  for (int y = 0; y < h->ny; ++y)
    for (int x = 0; x < h->nx; ++x) {
      size_t p = (size_t)y * h->nx + x;
      double uu[2] = {u[p], u[n + p]}, bb[2] = {b[p], b[n + p]};
      double feq[9], geq[10];
      if (h->feq_option == FEQ_SERIES_FULL)
        feq_series(1.0, uu, bb, 1, feq);
      else
        feq_algorithm(1.0, uu, bb, feq);
      geq_vector(uu, bb, geq);
      for (int i = 0; i < 9; ++i) h->f[FIDX(h, i, y, x)] = feq[i];
      for (int j = 0; j < 5; ++j)
        for (int c = 0; c < 2; ++c) h->g[GIDX(h, j, c, y, x)] = geq[2 * j + c];
    }
  h->step = 0;
}

static int wrap(int v, int n) { return ((v % n) + n) % n; }

/* One time step: collide every node (tasks 1-5) and push the post-collision
 * populations to their neighbours (task 6).  Walls reflect what would leave
 * the domain back into the node it came from. */
static void one_step(orc *h) {
  const int nx = h->nx, ny = h->ny;
  const double omega = 1.0 / h->tau_f, omega_m = 1.0 / h->tau_m;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y) {
    for (int x = 0; x < nx; ++x) {
      double f[9], g[10], fs[9], gs[10];
      for (int i = 0; i < 9; ++i) f[i] = h->f[FIDX(h, i, y, x)];
      for (int j = 0; j < 5; ++j)
        for (int c = 0; c < 2; ++c) g[2 * j + c] = h->g[GIDX(h, j, c, y, x)];
      const double *dn = h->delta ? h->delta + 3 * ((size_t)y * nx + x) : NULL;
      collide_node_c(f, g, omega, omega_m, h->G, h->feq_option, h->cl, dn, fs,
                     gs, NULL);
      for (int i = 0; i < 9; ++i) {
        int ty = y + CI[i][1];
        int tx = wrap(x + CI[i][0], nx);
        if (h->walls && (ty < 0 || ty >= ny)) {
          /* half-way bounce-back: returns reversed to the same node */
          int o = opposite_f(i);
          h->fn[FIDX(h, o, y, x)] = fs[i];
        } else {
          h->fn[FIDX(h, i, wrap(ty, ny), tx)] = fs[i];
        }
      }
      for (int j = 0; j < 5; ++j) {
        int ty = y + EJ[j][1];
        int tx = wrap(x + EJ[j][0], nx);
        if (h->walls && (ty < 0 || ty >= ny)) {
          /* anti-bounce-back imposing the wall field */
          int o = opposite_g(j);
          for (int c = 0; c < 2; ++c)
            h->gn[GIDX(h, o, c, y, x)] =
                -gs[2 * j + c] + 2.0 * PSI[o] * h->bwall[c];
        } else {
          for (int c = 0; c < 2; ++c)
            h->gn[GIDX(h, j, c, wrap(ty, ny), tx)] = gs[2 * j + c];
        }
      }
    }
  }
  double *t = h->f;
  h->f = h->fn;
  h->fn = t;
  t = h->g;
  h->g = h->gn;
  h->gn = t;
  h->step++;
}

void orc_step(orc *h, long n) {
  for (long k = 0; k < n; ++k) one_step(h);
}

long orc_step_count(const orc *h) { return h->step; }

/* Macroscopic fields of the current (pre-collision) state, algorithm task 1.
 * rho is [ny][nx]; u and b are [2][ny][nx]; any may be NULL. */
void orc_moments(const orc *h, double *rho, double *u, double *b) {
  size_t n = (size_t)h->nx * h->ny;
  for (int y = 0; y < h->ny; ++y)
    for (int x = 0; x < h->nx; ++x) {
      size_t p = (size_t)y * h->nx + x;
      double r = 0.0, j[2] = {0.0, 0.0}, bb[2] = {0.0, 0.0};
      for (int i = 0; i < 9; ++i) {
        double fi = h->f[FIDX(h, i, y, x)];
        r += fi;
        j[0] += fi * CI[i][0];
        j[1] += fi * CI[i][1];
      }
      for (int q = 0; q < 5; ++q)
        for (int c = 0; c < 2; ++c) bb[c] += h->g[GIDX(h, q, c, y, x)];
      if (rho) rho[p] = r;
      if (u) {
        u[p] = (j[0] + 0.5 * r * h->G[0]) / r;
        u[n + p] = (j[1] + 0.5 * r * h->G[1]) / r;
      }
      if (b) {
        b[p] = bb[0];
        b[n + p] = bb[1];
      }
    }
}

/* Isotropic lattice gradient d_alpha phi(x) = c_s^-2 sum_i w_i phi(x + c_i)
 * c_i,alpha (Sec. III); returns d_x (comp 0) or d_y (comp 1) of field phi at
 * (x, y) with periodic wrap. */
static double iso_grad(const orc *h, const double *phi, int x, int y,
                       int comp) {
  double s = 0.0;
  for (int i = 0; i < 9; ++i) {
    int xx = wrap(x + CI[i][0], h->nx), yy = wrap(y + CI[i][1], h->ny);
    s += WI[i] * phi[(size_t)yy * h->nx + xx] * CI[i][comp];
  }
  return s / CS2;
}

/* Diagnostics: out[0] = E_kin = sum |u|^2 / (2 N), out[1] = E_mag likewise
 * (the averaged energies of Sec. III with the integral as a node sum),
 * out[2] = max |div b| with the isotropic gradient; with walls the maximum
 * runs over the interior rows 1..ny-2. */
void orc_diagnostics(const orc *h, double out[3]) {
  size_t n = (size_t)h->nx * h->ny;
  double *u = (double *)malloc(2 * n * sizeof(double));
  double *b = (double *)malloc(2 * n * sizeof(double));
  orc_moments(h, NULL, u, b);
  double ek = 0.0, em = 0.0, dmax = 0.0;
  for (size_t p = 0; p < n; ++p) {
    ek += u[p] * u[p] + u[n + p] * u[n + p];
    em += b[p] * b[p] + b[n + p] * b[n + p];
  }
  int y0 = h->walls ? 1 : 0, y1 = h->walls ? h->ny - 1 : h->ny;
  for (int y = y0; y < y1; ++y)
    for (int x = 0; x < h->nx; ++x) {
      double d = iso_grad(h, b, x, y, 0) + iso_grad(h, b + n, x, y, 1);
      if (fabs(d) > dmax || isnan(d)) dmax = isnan(d) ? d : fabs(d);
    }
  out[0] = ek / (2.0 * (double)n);
  out[1] = em / (2.0 * (double)n);
  out[2] = dmax;
  free(u);
  free(b);
}

/* Conserved sums: mass, total momentum sum_i c_i f_i, total field sum b. */
void orc_invariants(const orc *h, double out[5]) {
  double s[5] = {0, 0, 0, 0, 0};
  for (int y = 0; y < h->ny; ++y)
    for (int x = 0; x < h->nx; ++x) {
      for (int i = 0; i < 9; ++i) {
        double fi = h->f[FIDX(h, i, y, x)];
        s[0] += fi;
        s[1] += fi * CI[i][0];
        s[2] += fi * CI[i][1];
      }
      for (int q = 0; q < 5; ++q) {
        s[3] += h->g[GIDX(h, q, 0, y, x)];
        s[4] += h->g[GIDX(h, q, 1, y, x)];
      }
    }
  memcpy(out, s, sizeof s);
}

/* Local current density from the populations (Eq. current), evaluated with
 * g - g_eq directly, and vorticity d_x u_y - d_y u_x with the isotropic
 * gradient.  Both are [ny][nx]; either may be NULL. */
void orc_current_vorticity(const orc *h, double *jz, double *wz) {
  size_t n = (size_t)h->nx * h->ny;
  double *u = (double *)malloc(2 * n * sizeof(double));
  double *b = (double *)malloc(2 * n * sizeof(double));
  orc_moments(h, NULL, u, b);
  const double omega_m = 1.0 / h->tau_m;
  for (int y = 0; y < h->ny; ++y)
    for (int x = 0; x < h->nx; ++x) {
      size_t p = (size_t)y * h->nx + x;
      if (jz) {
        double uu[2] = {u[p], u[n + p]}, bb[2] = {b[p], b[n + p]}, geq[10];
        geq_vector(uu, bb, geq);
        /* eps_ab sum_j e_j,a (g_j,b - geq_j,b), eps_xy = 1, eps_yx = -1 */
        double s = 0.0;
        for (int j = 0; j < 5; ++j) {
          double gx = h->g[GIDX(h, j, 0, y, x)] - geq[2 * j];
          double gy = h->g[GIDX(h, j, 1, y, x)] - geq[2 * j + 1];
          s += EJ[j][0] * gy - EJ[j][1] * gx;
        }
        jz[p] = -omega_m / CS2 * s;
      }
      if (wz) wz[p] = iso_grad(h, u + n, x, y, 0) - iso_grad(h, u, x, y, 1);
    }
  free(u);
  free(b);
}

/* Raw access to the pre-collision populations, f[9][ny][nx] and
 * g[5][2][ny][nx]. */
void orc_get_state(const orc *h, double *f, double *g) {
  size_t n = (size_t)h->nx * h->ny;
  if (f) memcpy(f, h->f, 9 * n * sizeof(double));
  if (g) memcpy(g, h->g, 10 * n * sizeof(double));
}

void orc_set_state(orc *h, const double *f, const double *g) {
  size_t n = (size_t)h->nx * h->ny;
  if (f) memcpy(h->f, f, 9 * n * sizeof(double));
  if (g) memcpy(h->g, g, 10 * n * sizeof(double));
}

/* Storage-precision model (a test of the arithmetic, not of the method):
 * rounds the current state to what FP32 storage keeps, i.e. the offsets
 * f_i - w_i and the magnetic populations g_j, each to the nearest FP32 value
 * (round to nearest even, the C cast), while every step stays in FP64.  A GPU
 * run whose arithmetic is exact up to its storage rounding stays as close to
 * the FP64 run as this model does. */
void orc_round_state_f32(orc *h) {
  size_t n = (size_t)h->nx * h->ny;
  for (int i = 0; i < 9; ++i)
    for (size_t p = 0; p < n; ++p) {
      double *v = &h->f[(size_t)i * n + p];
      *v = WI[i] + (double)(float)(*v - WI[i]);
    }
  for (size_t p = 0; p < 10 * n; ++p) h->g[p] = (double)(float)h->g[p];
}

/* n steps, each followed by the FP32 storage rounding above. */
void orc_step_rounded_f32(orc *h, long n) {
  for (long k = 0; k < n; ++k) {
    one_step(h);
    orc_round_state_f32(h);
  }
}

/* ---- single-node entry points for tests --------------------------------- */
void orc_node_equilibrium(double rho, const double u[2], const double b[2],
                          int option, double feq[9], double geq[10]) {
  build_tables();
  if (option == FEQ_SERIES_FULL)
    feq_series(rho, u, b, 1, feq);
  else
    feq_algorithm(rho, u, b, feq);
  if (geq) geq_vector(u, b, geq);
}

/* Equilibrium written as the plain Hermite series with the Maxwell tensor at
 * second order only (full = 0) or with all cross terms (full = 1). */
void orc_node_feq_series(double rho, const double u[2], const double b[2],
                         int full, double feq[9]) {
  build_tables();
  feq_series(rho, u, b, full, feq);
}

/* Collide one node.  aux (may be NULL) receives, in order: rho, u[2], b[2],
 * a1[2], a2[4] (xx, xy, yx, yy), a3[8], a4[16], feq[9], geq[10],
 * fneq_reg[9] -- 63 doubles. */
void orc_node_collide(const double f[9], const double g[10], double omega,
                      double omega_m, const double G[2], int option,
                      double fs[9], double gs[10], double *aux) {
  build_tables();
  node_aux A;
  double zero[2] = {0.0, 0.0};
  collide_node(f, g, omega, omega_m, G ? G : zero, option, fs, gs, &A);
  if (aux) {
    double *p = aux;
    *p++ = A.rho;
    *p++ = A.u[0];
    *p++ = A.u[1];
    *p++ = A.b[0];
    *p++ = A.b[1];
    *p++ = A.a1[0];
    *p++ = A.a1[1];
    memcpy(p, A.a2, sizeof A.a2);
    p += 4;
    memcpy(p, A.a3, sizeof A.a3);
    p += 8;
    memcpy(p, A.a4, sizeof A.a4);
    p += 16;
    memcpy(p, A.feq, sizeof A.feq);
    p += 9;
    memcpy(p, A.geq, sizeof A.geq);
    p += 10;
    memcpy(p, A.fneq_reg, sizeof A.fneq_reg);
  }
}

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Thread count of later grid loops (timing only; n >= 1). */
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ======================================================================== */
/* Learned closure (project addition): MLP 8 -> 64 -> 64 -> 3 with GELU      */
/* ======================================================================== */
/* Parameter vector (4931 values): W1[64][8], b1[64], W2[64][64], b2[64],
 * W3[3][64], b3[3].  Normalisation (19 values): mu[8], sigma[8],
 * sigma_out[3].  Features x = (rho, u_x, u_y, b_x, b_y, a_xx, a_xy, a_yy);
 * x_hat = (x - mu) / sigma; h1 = GELU(W1 x_hat + b1); h2 = GELU(W2 h1 + b2);
 * y = W3 h2 + b3; correction = sigma_out * y added to (a_xx, a_xy, a_yy). */
enum { NH = 64, NIN = 8, NOUT = 3 };
enum {
  OFF_W1 = 0,
  OFF_B1 = OFF_W1 + NH * NIN,
  OFF_W2 = OFF_B1 + NH,
  OFF_B2 = OFF_W2 + NH * NH,
  OFF_W3 = OFF_B2 + NH,
  OFF_B3 = OFF_W3 + NOUT * NH,
  NPARAM = OFF_B3 + NOUT
};

struct closure {
  double p[NPARAM];
  double norm[2 * NIN + NOUT];
};

/* GELU in the tanh form of Hendrycks & Gimpel (2016). */
static double gelu(double z) {
  const double k = 0.7978845608028654; /* sqrt(2/pi) */
  return 0.5 * z * (1.0 + tanh(k * (z + 0.044715 * z * z * z)));
}

static double gelu_grad(double z) {
  const double k = 0.7978845608028654;
  const double t = tanh(k * (z + 0.044715 * z * z * z));
  return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * k * (1.0 + 3.0 * 0.044715 * z * z);
}

typedef struct {
  double xh[NIN], z1[NH], h1[NH], z2[NH], h2[NH], y[NOUT];
} mlp_cache;

static void mlp_forward(const double *p, const double *norm, const double *x,
                        mlp_cache *c) {
  for (int k = 0; k < NIN; ++k) c->xh[k] = (x[k] - norm[k]) / norm[NIN + k];
  for (int i = 0; i < NH; ++i) {
    double s = p[OFF_B1 + i];
    for (int k = 0; k < NIN; ++k) s += p[OFF_W1 + i * NIN + k] * c->xh[k];
    c->z1[i] = s;
    c->h1[i] = gelu(s);
  }
  for (int i = 0; i < NH; ++i) {
    double s = p[OFF_B2 + i];
    for (int k = 0; k < NH; ++k) s += p[OFF_W2 + i * NH + k] * c->h1[k];
    c->z2[i] = s;
    c->h2[i] = gelu(s);
  }
  for (int o = 0; o < NOUT; ++o) {
    double s = p[OFF_B3 + o];
    for (int k = 0; k < NH; ++k) s += p[OFF_W3 + o * NH + k] * c->h2[k];
    c->y[o] = s;
  }
}

static void closure_apply(const closure *c, double rho, const double u[2],
                          const double b[2], double a2[2][2]) {
  const double x[NIN] = {rho, u[0], u[1], b[0], b[1], a2[0][0], a2[0][1], a2[1][1]};
  mlp_cache m;
  mlp_forward(c->p, c->norm, x, &m);
  const double *so = c->norm + 2 * NIN;
  a2[0][0] += so[0] * m.y[0];
  a2[0][1] += so[1] * m.y[1];
  a2[1][0] += so[1] * m.y[1];
  a2[1][1] += so[2] * m.y[2];
}

int orc_closure_nparams(void) { return NPARAM; }

/* Install (params, norm) on a grid solver; params == NULL removes it. */
int orc_set_closure(orc *h, const double *params, const double *norm) {
  free(h->cl);
  h->cl = NULL;
  if (!params) return 0;
  h->cl = (closure *)malloc(sizeof(closure));
  if (!h->cl) return -1;
  memcpy(h->cl->p, params, sizeof h->cl->p);
  memcpy(h->cl->norm, norm, sizeof h->cl->norm);
  return 0;
}

/* Network output y[n][3] (normalised units) for inputs x[n][8]. */
void orc_mlp_forward(const double *params, const double *norm, const double *x,
                     int n, double *y) {
  for (int s = 0; s < n; ++s) {
    mlp_cache m;
    mlp_forward(params, norm, x + (size_t)s * NIN, &m);
    for (int o = 0; o < NOUT; ++o) y[(size_t)s * NOUT + o] = m.y[o];
  }
}

/* Reverse mode through one forward pass: adds d(dy . y)/d(params) to grad. */
static void mlp_backprop(const double *p, const mlp_cache *m, const double dy[NOUT],
                         double *grad) {
  double dz2[NH], dz1[NH];
  for (int o = 0; o < NOUT; ++o) {
    grad[OFF_B3 + o] += dy[o];
    for (int k = 0; k < NH; ++k) grad[OFF_W3 + o * NH + k] += dy[o] * m->h2[k];
  }
  for (int k = 0; k < NH; ++k) {
    double sacc = 0.0;
    for (int o = 0; o < NOUT; ++o) sacc += p[OFF_W3 + o * NH + k] * dy[o];
    dz2[k] = sacc * gelu_grad(m->z2[k]);
    grad[OFF_B2 + k] += dz2[k];
  }
  for (int i = 0; i < NH; ++i)
    for (int k = 0; k < NH; ++k) grad[OFF_W2 + i * NH + k] += dz2[i] * m->h1[k];
  for (int k = 0; k < NH; ++k) {
    double sacc = 0.0;
    for (int i = 0; i < NH; ++i) sacc += p[OFF_W2 + i * NH + k] * dz2[i];
    dz1[k] = sacc * gelu_grad(m->z1[k]);
    grad[OFF_B1 + k] += dz1[k];
  }
  for (int i = 0; i < NH; ++i)
    for (int k = 0; k < NIN; ++k) grad[OFF_W1 + i * NIN + k] += dz1[i] * m->xh[k];
}

/* Mean squared error L = (1/n) sum_s sum_o (y_o(x_s) - t_so)^2 and its
 * gradient with respect to every parameter, by reverse-mode
 * differentiation of the forward pass. */
double orc_mlp_loss_grad(const double *params, const double *norm,
                         const double *x, const double *t, int n,
                         double *grad) {
  memset(grad, 0, sizeof(double) * NPARAM);
  double loss = 0.0;
  for (int s = 0; s < n; ++s) {
    mlp_cache m;
    mlp_forward(params, norm, x + (size_t)s * NIN, &m);
    double dy[NOUT];
    for (int o = 0; o < NOUT; ++o) {
      const double r = m.y[o] - t[(size_t)s * NOUT + o];
      loss += r * r;
      dy[o] = 2.0 * r / n;
    }
    mlp_backprop(params, &m, dy, grad);
  }
  return loss / n;
}

/* Input gradient: gx[s] = d/dx_s (dy[s] . y(x_s)) for raw features x[n][8]. */
void orc_mlp_vjp_input(const double *params, const double *norm, const double *x,
                       const double *dy, int n, double *gx) {
  const double *p = params;
  for (int s = 0; s < n; ++s) {
    mlp_cache m;
    mlp_forward(p, norm, x + (size_t)s * NIN, &m);
    double dz2[NH], dz1[NH];
    for (int k = 0; k < NH; ++k) {
      double a = 0.0;
      for (int o = 0; o < NOUT; ++o) a += p[OFF_W3 + o * NH + k] * dy[(size_t)s * NOUT + o];
      dz2[k] = a * gelu_grad(m.z2[k]);
    }
    for (int k = 0; k < NH; ++k) {
      double a = 0.0;
      for (int i = 0; i < NH; ++i) a += p[OFF_W2 + i * NH + k] * dz2[i];
      dz1[k] = a * gelu_grad(m.z1[k]);
    }
    for (int k = 0; k < NIN; ++k) {
      double a = 0.0;
      for (int i = 0; i < NH; ++i) a += p[OFF_W1 + i * NIN + k] * dz1[i];
      gx[(size_t)s * NIN + k] = a / norm[NIN + k];
    }
  }
}

/* Vector-Jacobian product: grad = d/d(params) sum_s dy[s] . y(x_s), for
 * dy[n][3] (normalised output units). */
void orc_mlp_vjp(const double *params, const double *norm, const double *x,
                 const double *dy, int n, double *grad) {
  memset(grad, 0, sizeof(double) * NPARAM);
  for (int s = 0; s < n; ++s) {
    mlp_cache m;
    mlp_forward(params, norm, x + (size_t)s * NIN, &m);
    mlp_backprop(params, &m, dy + (size_t)s * NOUT, grad);
  }
}

/* One Adam step (Kingma & Ba 2015) at step number t >= 1. */
void orc_adam_step(double *params, double *m, double *v, const double *grad,
                   int n, double lr, double beta1, double beta2, double eps,
                   int t) {
  const double c1 = 1.0 - pow(beta1, t), c2 = 1.0 - pow(beta2, t);
  for (int k = 0; k < n; ++k) {
    m[k] = beta1 * m[k] + (1.0 - beta1) * grad[k];
    v[k] = beta2 * v[k] + (1.0 - beta2) * grad[k] * grad[k];
    const double mh = m[k] / c1, vh = v[k] / c2;
    params[k] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* Training samples of the closure (project addition) from fine moments
 * rho[nf][nf], u[2][nf][nf], b[2][nf][nf]: box filter over fac x fac blocks;
 * features (rho_bar, u_bar = (rho u)_bar / rho_bar, b_bar, a_CE) with
 * a_CE = -rho_bar c_s^2 tau_c (grad u_bar + grad u_bar^T), the gradient being
 * the isotropic lattice gradient of Sec. III on the coarse grid; target
 * tau_sgs / (tau_c - 1), tau_sgs = (rho u u)_bar - rho_bar u_bar u_bar
 * + M(b)_bar - M(b_bar).  x[nc*nc][8], t[nc*nc][3]. */
void orc_train_samples(const double *rho, const double *u, const double *b,
                       int nf, int fac, double tau_c, double *x, double *t) {
  const int nc = nf / fac;
  const size_t Nf = (size_t)nf * nf, Nc = (size_t)nc * nc;
  double *R = calloc(Nc, sizeof(double)), *JX = calloc(Nc, sizeof(double)),
         *JY = calloc(Nc, sizeof(double)), *BX = calloc(Nc, sizeof(double)),
         *BY = calloc(Nc, sizeof(double)), *PXX = calloc(Nc, sizeof(double)),
         *PXY = calloc(Nc, sizeof(double)), *PYY = calloc(Nc, sizeof(double)),
         *MXX = calloc(Nc, sizeof(double)), *MXY = calloc(Nc, sizeof(double)),
         *MYY = calloc(Nc, sizeof(double));
  for (int y = 0; y < nf; ++y)
    for (int xx = 0; xx < nf; ++xx) {
      const size_t f = (size_t)y * nf + xx, c = (size_t)(y / fac) * nc + xx / fac;
      const double r = rho[f], ux = u[f], uy = u[Nf + f], bx = b[f], by = b[Nf + f];
      double bb[2] = {bx, by}, M[2][2];
      maxwell(bb, M);
      R[c] += r;
      JX[c] += r * ux;
      JY[c] += r * uy;
      BX[c] += bx;
      BY[c] += by;
      PXX[c] += r * ux * ux;
      PXY[c] += r * ux * uy;
      PYY[c] += r * uy * uy;
      MXX[c] += M[0][0];
      MXY[c] += M[0][1];
      MYY[c] += M[1][1];
    }
  const double a = 1.0 / ((double)fac * fac);
  double *arrs[11] = {R, JX, JY, BX, BY, PXX, PXY, PYY, MXX, MXY, MYY};
  for (int k = 0; k < 11; ++k)
    for (size_t c = 0; c < Nc; ++c) arrs[k][c] *= a;
  double *UX = malloc(Nc * sizeof(double)), *UY = malloc(Nc * sizeof(double));
  for (size_t c = 0; c < Nc; ++c) {
    UX[c] = JX[c] / R[c];
    UY[c] = JY[c] / R[c];
  }
  for (int cy = 0; cy < nc; ++cy)
    for (int cx = 0; cx < nc; ++cx) {
      const size_t c = (size_t)cy * nc + cx;
      double g[2][2]; /* g[a][b] = d_a u_b */
      for (int aa = 0; aa < 2; ++aa) {
        double sx = 0.0, sy = 0.0;
        for (int i = 0; i < 9; ++i) {
          const size_t q = (size_t)wrap(cy + CI[i][1], nc) * nc + wrap(cx + CI[i][0], nc);
          sx += WI[i] * UX[q] * CI[i][aa];
          sy += WI[i] * UY[q] * CI[i][aa];
        }
        g[aa][0] = sx / CS2;
        g[aa][1] = sy / CS2;
      }
      const double r = R[c], ux = UX[c], uy = UY[c];
      double bb[2] = {BX[c], BY[c]}, Mb[2][2];
      maxwell(bb, Mb);
      const double k = -r * CS2 * tau_c;
      x[c * 8 + 0] = r;
      x[c * 8 + 1] = ux;
      x[c * 8 + 2] = uy;
      x[c * 8 + 3] = BX[c];
      x[c * 8 + 4] = BY[c];
      x[c * 8 + 5] = k * (g[0][0] + g[0][0]);
      x[c * 8 + 6] = k * (g[0][1] + g[1][0]);
      x[c * 8 + 7] = k * (g[1][1] + g[1][1]);
      const double sxx = PXX[c] - r * ux * ux + MXX[c] - Mb[0][0];
      const double sxy = PXY[c] - r * ux * uy + MXY[c] - Mb[0][1];
      const double syy = PYY[c] - r * uy * uy + MYY[c] - Mb[1][1];
      t[c * 3 + 0] = sxx / (tau_c - 1.0);
      t[c * 3 + 1] = sxy / (tau_c - 1.0);
      t[c * 3 + 2] = syy / (tau_c - 1.0);
    }
  for (int k = 0; k < 11; ++k) free(arrs[k]);
  free(UX);
  free(UY);
}

/* ======================================================================== */
/* One-step solver-in-the-loop objective of the closure (project addition) */
/* ======================================================================== */
/* Coarse node X of an nc x nc grid covers the fine block fac X .. fac X +
 * fac - 1 (both axes); coarse step n corresponds to fine step fac n
 * (acoustic scaling, tau_c = 1/2 + (tau_f - 1/2) / fac).
 *
 * Restart at fine time t: box-filter rho, rho u and b; u_bar = (rho u)_bar /
 * rho_bar; a_CE = -rho_bar c_s^2 tau_c (grad u_bar + grad u_bar^T) with the
 * isotropic gradient of Sec. III on the coarse grid; f = f_eq(rho_bar, u_bar,
 * b_bar) + f_neq,reg(u_bar, a_CE) (tasks 2-4); g = g_eq(u_bar, b_bar).
 * One coarse step of this state with delta(X) added to a_1^(2) at every node
 * before the recursion gives the momentum j_c(X) = sum_i c_i f_i(X) at coarse
 * time 1.  Objective
 *   L = sum_X |j_c(X) - j_bar(X, t + fac)|^2 / sum_X |j_bar(t + fac) - j_bar(t)|^2. */

/* Box filter of rho, rho u_x, rho u_y, b_x, b_y: out[5][nc][nc]. */
static void filter_rjb(const double *rho, const double *u, const double *b,
                       int nf, int fac, double *out) {
  const int nc = nf / fac;
  const size_t Nf = (size_t)nf * nf, Nc = (size_t)nc * nc;
  memset(out, 0, 5 * Nc * sizeof(double));
  for (int y = 0; y < nf; ++y)
    for (int x = 0; x < nf; ++x) {
      const size_t f = (size_t)y * nf + x, c = (size_t)(y / fac) * nc + x / fac;
      out[c] += rho[f];
      out[Nc + c] += rho[f] * u[f];
      out[2 * Nc + c] += rho[f] * u[Nf + f];
      out[3 * Nc + c] += b[f];
      out[4 * Nc + c] += b[Nf + f];
    }
  const double a = 1.0 / ((double)fac * fac);
  for (size_t k = 0; k < 5 * Nc; ++k) out[k] *= a;
}

/* Restart populations (solver layout f[9][nc][nc], g[5][2][nc][nc]) from
 * filtered fields F[5][nc][nc]; q[Nc][3] (may be NULL) is an extra
 * non-equilibrium (xx, xy, yy) added to a_CE. */
static void restart_state(const double *F, int nc, double tau_c, const double *q,
                          double *f, double *g) {
  const size_t Nc = (size_t)nc * nc;
  double *U = malloc(2 * Nc * sizeof(double));
  for (size_t c = 0; c < Nc; ++c) {
    U[c] = F[Nc + c] / F[c];
    U[Nc + c] = F[2 * Nc + c] / F[c];
  }
  for (int cy = 0; cy < nc; ++cy)
    for (int cx = 0; cx < nc; ++cx) {
      const size_t c = (size_t)cy * nc + cx;
      double gr[2][2] = {{0.0, 0.0}, {0.0, 0.0}}; /* gr[a][b] = d_a u_b */
      for (int i = 0; i < 9; ++i) {
        const size_t q = (size_t)wrap(cy + CI[i][1], nc) * nc + wrap(cx + CI[i][0], nc);
        for (int a = 0; a < 2; ++a)
          for (int bb = 0; bb < 2; ++bb) gr[a][bb] += WI[i] * CI[i][a] * U[bb * Nc + q] / CS2;
      }
      const double rho = F[c], u[2] = {U[c], U[Nc + c]}, b[2] = {F[3 * Nc + c], F[4 * Nc + c]};
      double a2[2][2];
      for (int a = 0; a < 2; ++a)
        for (int bb = 0; bb < 2; ++bb) a2[a][bb] = -rho * CS2 * tau_c * (gr[a][bb] + gr[bb][a]);
      if (q) {
        a2[0][0] += q[3 * c];
        a2[0][1] += q[3 * c + 1];
        a2[1][0] += q[3 * c + 1];
        a2[1][1] += q[3 * c + 2];
      }
      double feq[9], geq[10], a3[2][2][2], a4[2][2][2][2], r[9];
      feq_algorithm(rho, u, b, feq);
      geq_vector(u, b, geq);
      reg_expand(u, (const double(*)[2])a2, a3, a4, r);
      for (int i = 0; i < 9; ++i) f[(size_t)i * Nc + c] = feq[i] + WI[i] * r[i];
      for (int j = 0; j < 5; ++j)
        for (int k = 0; k < 2; ++k) g[((size_t)j * 2 + k) * Nc + c] = geq[2 * j + k];
    }
  free(U);
}

/* The objective for fine moments (rho0, u0, b0) at t and (rho1, u1, b1) at
 * t + fac (rho [nf][nf], u and b [2][nf][nf]), an extra restart
 * non-equilibrium q[Nc][3] (NULL: none; the closure's own steady response
 * (tau_c - 1) D in the feedback form of the objective) and a correction
 * delta[Nc][3] (NULL: none).  Returns L; optional outputs: resid[Nc][2] = j_c - j_bar(t +
 * fac), x[Nc][8] = the restart state's features (rho, u, b, a_1^(2)) computed
 * from its populations as the collision computes them, *den. */
double orc_onestep_objective(const double *rho0, const double *u0, const double *b0,
                             const double *rho1, const double *u1, const double *b1,
                             int nf, int fac, double tau_c, const double *q,
                             const double *delta, double *resid, double *x,
                             double *den_out) {
  build_tables();
  const int nc = nf / fac;
  const size_t Nc = (size_t)nc * nc;
  double *F0 = malloc(5 * Nc * sizeof(double)), *F1 = malloc(5 * Nc * sizeof(double));
  double *f = malloc(9 * Nc * sizeof(double)), *g = malloc(10 * Nc * sizeof(double));
  filter_rjb(rho0, u0, b0, nf, fac, F0);
  filter_rjb(rho1, u1, b1, nf, fac, F1);
  restart_state(F0, nc, tau_c, q, f, g);
  orc *h = orc_create(nc, nc, tau_c, tau_c, 0, 0.0, 0.0, 0.0, 0.0, FEQ_ALGORITHM);
  orc_set_state(h, f, g);
  if (x) {
    const double G0[2] = {0.0, 0.0};
    for (size_t c = 0; c < Nc; ++c) {
      double fl[9], gl[10], fs[9], gs[10];
      node_aux ax;
      for (int i = 0; i < 9; ++i) fl[i] = f[(size_t)i * Nc + c];
      for (int k = 0; k < 10; ++k) gl[k] = g[(size_t)k * Nc + c];
      collide_node(fl, gl, 1.0 / tau_c, 1.0 / tau_c, G0, FEQ_ALGORITHM, fs, gs, &ax);
      const double v[8] = {ax.rho, ax.u[0], ax.u[1], ax.b[0], ax.b[1],
                           ax.a2[0][0], ax.a2[0][1], ax.a2[1][1]};
      memcpy(x + 8 * c, v, sizeof v);
    }
  }
  h->delta = delta;
  one_step(h);
  h->delta = NULL;
  double num = 0.0, den = 0.0;
  for (size_t c = 0; c < Nc; ++c) {
    double j[2] = {0.0, 0.0};
    for (int i = 0; i < 9; ++i)
      for (int a = 0; a < 2; ++a) j[a] += CI[i][a] * h->f[(size_t)i * Nc + c];
    for (int a = 0; a < 2; ++a) {
      const double r = j[a] - F1[(1 + a) * Nc + c];
      const double d = F1[(1 + a) * Nc + c] - F0[(1 + a) * Nc + c];
      if (resid) resid[2 * c + a] = r;
      num += r * r;
      den += d * d;
    }
  }
  if (den_out) *den_out = den;
  orc_destroy(h);
  free(F0);
  free(F1);
  free(f);
  free(g);
  return num / den;
}

/* Transpose of the linear part of delta -> j_c of the objective, applied to
 * w[Nc][2]: out[Y][k] = sum_i (c_i . w(Y + c_i)) d fs_i(Y) / d delta_k(Y).
 * At the restart velocity u(Y) (x[Y][1..2]) the post-collision populations
 * depend on delta only through (1 - 1/tau_c) f_neq,reg(u, a_1^(2) + delta),
 * which is linear in a_1^(2); its columns are the regularised populations of
 * the unit corrections (the xy unit sets both off-diagonal entries). */
void orc_onestep_adjoint(const double *x, int nc, double tau_c, const double *w,
                         double *out) {
  build_tables();
  const double E[3][2][2] = {{{1, 0}, {0, 0}}, {{0, 1}, {1, 0}}, {{0, 0}, {0, 1}}};
  for (int cy = 0; cy < nc; ++cy)
    for (int cx = 0; cx < nc; ++cx) {
      const size_t c = (size_t)cy * nc + cx;
      const double u[2] = {x[8 * c + 1], x[8 * c + 2]};
      double m[9];
      for (int i = 0; i < 9; ++i) {
        const size_t q = (size_t)wrap(cy + CI[i][1], nc) * nc + wrap(cx + CI[i][0], nc);
        m[i] = CI[i][0] * w[2 * q] + CI[i][1] * w[2 * q + 1];
      }
      for (int k = 0; k < 3; ++k) {
        double a3[2][2][2], a4[2][2][2][2], r[9], s = 0.0;
        reg_expand(u, E[k], a3, a4, r);
        for (int i = 0; i < 9; ++i) s += m[i] * (1.0 - 1.0 / tau_c) * WI[i] * r[i];
        out[3 * c + k] = s;
      }
    }
}
