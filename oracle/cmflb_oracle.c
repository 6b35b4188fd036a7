/*
 * cmflb_oracle.c -- plain, slow, FP64 CPU oracle of the fluctuating
 * orthogonal-central-moment lattice Boltzmann method (CM-FLBM) of
 * De Rosis & Zhou, "A fluctuating lattice Boltzmann formulation based on
 * orthogonal central moments" (arXiv 2602.16486).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP implementation.
 *
 * What it computes, in the paper's order (Sec. 2, "Algorithm of
 * computation"): for every site, (1) density and velocity (eq. macro),
 * (2) standard normals for the noisy modes, (3) pre-collision central
 * moments k = T(u) f with T built densely from the basis polynomials
 * evaluated at the shifted velocities c_i - u (Sec. 2.2 and 2.3),
 * (4) the collision k* = (I - Lambda) k + Lambda k_eq + I~ phi eta
 * (eq. cm_collision) with k_eq = T(u) f_eq(rho, u) evaluated literally and
 * phi from eq. phi_general using the local density, (5)+(6) the back
 * transformation f* = T(u)^-1 k* by an LU solve with partial pivoting (or,
 * as a second path, f* = M^-1 N(-u) k* with M^-1 = W M^T B^-1), and (7) the
 * streaming f_i(x + c_i, t + 1) = f*_i(x, t) with periodic wrap
 * (eq. streaming).  Everything is FP64; there is no blocking, fusion or
 * reordering beyond that.
 *
 * Readings of the paper taken here (each listed with its reason in the
 * design notes of the repository):
 *  - D2Q9 equilibrium: the compact form prints the H_xxyy u_x^2 u_y^2 term
 *    without its 1/(4 c_s^8) factor; the general Hermite form (eq. feq) is
 *    used, keeping the terms in which each Cartesian index appears at most
 *    twice, each with coefficient 1/(n_x! n_y! n_z! c_s^(2n)).
 *  - D3Q27 basis row 15 is (c_y^2 - c_s^2) c_z (the printed c_s^2 c_y term
 *    breaks orthogonality and contradicts the printed b_15 = 2/27).
 *  - D3Q19 (Sec. 2.4): the velocities are taken in the D3Q27 order of
 *    Sec. 2.3 with the eight corners left out (the paper lists the set, not
 *    an order).  Its printed equilibrium does not conserve mass; the paper
 *    also states that the equilibrium's central moments are (rho, 0, ..., 0),
 *    which fixes it uniquely: k_eq = rho e_0 is used in the collision and
 *    f_eq = T(u)^-1 rho e_0 (LU solve) as the equilibrium.  The second
 *    reconstruction path does not apply on D3Q19 (N(u)^-1 != N(-u) there).
 *  - Noise: eta comes from Philox4x32-10 (Salmon et al., SC'11) keyed by the
 *    64-bit seed, counter (site, step, replica, block) -- for steps of 2^32
 *    and beyond (site, step mod 2^32, replica, block + 2^8 floor(step /
 *    2^32)), so that no two steps below 2^56 share a counter -- mapped to
 *    normals by the Box-Muller transform (details at normals()).  The paper
 *    asks only for independent standard normal variables.
 *
 * Parity pins: see the test suite (tests/test_oracle_*.py).  The Philox
 * generator has no published known-answer vector in this repository; it is
 * pinned by inversion of its round function, by bijectivity and by
 * statistical checks.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_QMAX 27
#define ORC_CS2 (1.0 / 3.0)
#define ORC_NSTAT 12

/* ---- lattices, in the paper's velocity order --------------------------- */

/* D2Q9 (Sec. 2.2): c_x = [0,1,0,-1,0,1,-1,-1,1], c_y = [0,0,1,0,-1,1,1,-1,-1]. */
static const int d2q9_c[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const double d2q9_w[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                                 1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                                 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* D3Q27 (Sec. 2.3), listed component-wise in the paper. */
static const int d3q27_cx[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1,
                                 -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
static const int d3q27_cy[27] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0,
                                 0, 1, -1, 1, -1, 1, 1, -1, -1, 1, 1, -1, -1};
static const int d3q27_cz[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1,
                                 -1, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1};

static double d3q27_weight(int i) {
  if (i == 0) return 8.0 / 27.0;
  if (i <= 6) return 2.0 / 27.0;
  if (i <= 18) return 1.0 / 54.0;
  return 1.0 / 216.0;
}

static int lattice_ok(int q) { return q == 9 || q == 19 || q == 27; }

static void velocity(int q, int i, double c[3]) {
  if (q == 9) {
    c[0] = d2q9_c[i][0];
    c[1] = d2q9_c[i][1];
    c[2] = 0.0;
  } else {
    c[0] = d3q27_cx[i];
    c[1] = d3q27_cy[i];
    c[2] = d3q27_cz[i];
  }
}

/* D3Q19 weights (Sec. 2.4): 1/3, 1/18 (|c|^2 = 1), 1/36 (|c|^2 = 2). */
static double d3q19_weight(int i) {
  if (i == 0) return 1.0 / 3.0;
  return i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0;
}

static double weight(int q, int i) {
  if (q == 9) return d2q9_w[i];
  return q == 19 ? d3q19_weight(i) : d3q27_weight(i);
}

/* ---- moment bases ------------------------------------------------------- */

/* Row v of the D2Q9 orthogonal basis (Sec. 2.2), evaluated at (x, y). */
static double d2q9_orth_row(int v, double x, double y) {
  const double s = ORC_CS2;
  switch (v) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return x * x + y * y - 2.0 * s;
    case 4: return x * x - y * y;
    case 5: return x * y;
    case 6: return (x * x - s) * y;
    case 7: return x * (y * y - s);
    case 8: return (x * x - s) * (y * y - s);
  }
  return 0.0;
}

/* Row v of the D2Q9 non-orthogonal basis (Sec. 2.2, first basis). */
static double d2q9_nonorth_row(int v, double x, double y) {
  switch (v) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return x * x + y * y;
    case 4: return x * x - y * y;
    case 5: return x * y;
    case 6: return x * x * y;
    case 7: return x * y * y;
    case 8: return x * x * y * y;
  }
  return 0.0;
}

/* Row v of the D3Q27 orthogonal basis (Sec. 2.3), written as printed except
 * row 15, which is read as (c_y^2 - c_s^2) c_z. */
static double d3q27_row(int v, double x, double y, double z) {
  const double s = ORC_CS2, s2 = s * s, s3 = s * s * s;
  switch (v) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * x - s;
    case 5: return y * y - s;
    case 6: return z * z - s;
    case 7: return x * y;
    case 8: return x * z;
    case 9: return y * z;
    case 10: return x * x * y - s * y;
    case 11: return x * x * z - s * z;
    case 12: return x * y * y - s * x;
    case 13: return x * z * z - s * x;
    case 14: return y * z * z - s * y;
    case 15: return y * y * z - s * z;
    case 16: return x * y * z;
    case 17: return x * x * y * y - s * (x * x + y * y) + s2;
    case 18: return x * x * z * z - s * (x * x + z * z) + s2;
    case 19: return y * y * z * z - s * (y * y + z * z) + s2;
    case 20: return x * y * z * z - s * x * y;
    case 21: return x * y * y * z - s * x * z;
    case 22: return x * x * y * z - s * y * z;
    case 23: return x * x * y * z * z - s * (x * x * y + y * z * z) + s2 * y;
    case 24: return x * x * y * y * z - s * (x * x * z + y * y * z) + s2 * z;
    case 25: return x * y * y * z * z - s * (x * y * y + x * z * z) + s2 * x;
    case 26:
      return x * x * y * y * z * z -
             s * (x * x * y * y + x * x * z * z + y * y * z * z) +
             s2 * (x * x + y * y + z * z) - s3;
  }
  return 0.0;
}

/* Row v of the D3Q19 basis (Sec. 2.4), with c^2 = x^2 + y^2 + z^2. */
static double d3q19_row(int v, double x, double y, double z) {
  const double c2 = x * x + y * y + z * z;
  switch (v) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return c2 - 1.0;
    case 5: return 3.0 * x * x - c2;
    case 6: return y * y - z * z;
    case 7: return x * y;
    case 8: return y * z;
    case 9: return x * z;
    case 10: return x * (3.0 * c2 - 5.0);
    case 11: return y * (3.0 * c2 - 5.0);
    case 12: return z * (3.0 * c2 - 5.0);
    case 13: return x * (y * y - z * z);
    case 14: return y * (z * z - x * x);
    case 15: return z * (x * x - y * y);
    case 16: return 3.0 * c2 * c2 - 6.0 * c2 + 1.0;
    case 17: return (2.0 * c2 - 3.0) * (3.0 * x * x - c2);
    case 18: return (2.0 * c2 - 3.0) * (y * y - z * z);
  }
  return 0.0;
}

static double basis_row(int q, int basis, int v, const double c[3]) {
  if (q == 9)
    return basis == 1 ? d2q9_nonorth_row(v, c[0], c[1])
                      : d2q9_orth_row(v, c[0], c[1]);
  if (q == 19) return d3q19_row(v, c[0], c[1], c[2]);
  return d3q27_row(v, c[0], c[1], c[2]);
}

/* T_vi = P_v(c_i - u): the central-moment transformation (Sec. 2.2).  With
 * u = 0 this is the raw-moment matrix M. */
static void build_T(int q, int basis, const double u[3], double *T) {
  for (int i = 0; i < q; ++i) {
    double c[3];
    velocity(q, i, c);
    double cb[3] = {c[0] - u[0], c[1] - u[1], c[2] - u[2]};
    for (int v = 0; v < q; ++v) T[v * q + i] = basis_row(q, basis, v, cb);
  }
}

/* b_v = sum_i w_i M_vi^2 (the normalisation factor below eq. Xi_pop). */
static void build_norms(int q, int basis, double *b) {
  double M[ORC_QMAX * ORC_QMAX];
  const double zero[3] = {0, 0, 0};
  build_T(q, basis, zero, M);
  for (int v = 0; v < q; ++v) {
    double s = 0.0;
    for (int i = 0; i < q; ++i) s += weight(q, i) * M[v * q + i] * M[v * q + i];
    b[v] = s;
  }
}

/* ---- Hermite equilibrium (eq. feq) -------------------------------------- */

/* Hermite tensor component H^(n)_{a_1..a_n}(c) from the recursive
 * definition H^(n+1)_{a B} = c_a H^(n)_B - c_s^2 sum_j delta_{a b_j}
 * H^(n-1)_{B without b_j}, which reproduces the tensors printed for
 * n <= 4 (Sec. 2.2). */
static double hermite(const double c[3], const int *idx, int n) {
  if (n == 0) return 1.0;
  const int a = idx[0];
  const int *rest = idx + 1;
  double h = c[a] * hermite(c, rest, n - 1);
  for (int j = 0; j < n - 1; ++j) {
    if (rest[j] != a) continue;
    int red[8];
    int m = 0;
    for (int l = 0; l < n - 1; ++l)
      if (l != j) red[m++] = rest[l];
    h -= ORC_CS2 * hermite(c, red, n - 2);
  }
  return h;
}

static double factorial(int n) {
  double f = 1.0;
  for (int k = 2; k <= n; ++k) f *= k;
  return f;
}

/* Tables that depend only on the lattice and basis, built once per call:
 * velocities, weights, M, b_v and the Hermite terms of the equilibrium. */
typedef struct {
  int q, basis, nm;
  double c[ORC_QMAX][3], w[ORC_QMAX];
  double M[ORC_QMAX * ORC_QMAX], b[ORC_QMAX];
  int mexp[ORC_QMAX][3];
  double herm[ORC_QMAX][ORC_QMAX]; /* H_m(c_i) / (m_x! m_y! m_z! c_s^(2|m|)) */
} ctx_t;

static void build_norms(int q, int basis, double *b);

static void ctx_init(ctx_t *x, int q, int basis) {
  const double zero[3] = {0, 0, 0};
  x->q = q;
  x->basis = basis;
  for (int i = 0; i < q; ++i) {
    velocity(q, i, x->c[i]);
    x->w[i] = weight(q, i);
  }
  build_T(q, basis, zero, x->M);
  build_norms(q, basis, x->b);
  const int dims = q == 9 ? 2 : 3;
  int nm = 0;
  for (int mx = 0; mx <= 2; ++mx)
    for (int my = 0; my <= 2; ++my)
      for (int mz = 0; mz <= (dims == 3 ? 2 : 0); ++mz) {
        x->mexp[nm][0] = mx;
        x->mexp[nm][1] = my;
        x->mexp[nm][2] = mz;
        int idx[8];
        int n = 0;
        for (int k = 0; k < mx; ++k) idx[n++] = 0;
        for (int k = 0; k < my; ++k) idx[n++] = 1;
        for (int k = 0; k < mz; ++k) idx[n++] = 2;
        double coef = 1.0 / (factorial(mx) * factorial(my) * factorial(mz) *
                             pow(ORC_CS2, n));
        for (int i = 0; i < q; ++i)
          x->herm[i][nm] = coef * hermite(x->c[i], idx, n);
        ++nm;
      }
  x->nm = nm;
}

static int lu_solve(int q, const double *A_in, const double *b_in, double *x);

/* f_eq_i = w_i rho sum_m H_m(c_i) u^m / (m_x! m_y! m_z! c_s^(2|m|)) over
 * multi-indices m with every m_a <= 2 (the terms kept by the paper's D2Q9
 * and D3Q27 equilibria; a full tensor contraction groups each multi-index
 * with multiplicity n!/(m_x! m_y! m_z!)).  D3Q19: the state whose central
 * moments are (rho, 0, ..., 0), f_eq = T(u)^-1 rho e_0. */
static void equilibrium(const ctx_t *x, double rho, const double u[3],
                        double *feq) {
  if (x->q == 19) {
    double T[ORC_QMAX * ORC_QMAX], k[ORC_QMAX] = {0};
    build_T(19, 0, u, T);
    k[0] = rho;
    if (lu_solve(19, T, k, feq) != 0)
      for (int i = 0; i < 19; ++i) feq[i] = NAN;
    return;
  }
  double um[ORC_QMAX];
  for (int m = 0; m < x->nm; ++m) {
    double p = 1.0;
    for (int a = 0; a < 3; ++a)
      for (int e = 0; e < x->mexp[m][a]; ++e) p *= u[a];
    um[m] = p;
  }
  for (int i = 0; i < x->q; ++i) {
    double sum = 0.0;
    for (int m = 0; m < x->nm; ++m) sum += x->herm[i][m] * um[m];
    feq[i] = x->w[i] * rho * sum;
  }
}

/* ---- Philox4x32-10 and Box-Muller --------------------------------------- */

/* Philox4x32 with 10 rounds as defined by Salmon, Moraes, Dror and Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3" (SC'11): each round
 * multiplies words 0 and 2 by 0xD2511F53 and 0xCD9E8D57 (64-bit products),
 * outputs (hi2 ^ x1 ^ k0, lo2, hi0 ^ x3 ^ k1, lo0), and the key is advanced
 * by the Weyl constants (0x9E3779B9, 0xBB67AE85) between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0;
    x1 = y1;
    x2 = y2;
    x3 = y3;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

static int first_noisy_mode(int q) { return q == 9 ? 3 : 4; }

/* Standard normals eta_v for the noisy modes v = first..q-1 (Sec. 2.2:
 * I~ = diag[0,0,0,1,..]; Sec. 2.3: I~_0-3 = 0).  Normal n = v - first; pair
 * p = n / 2 draws Philox block p / 2 with counter (site, step mod 2^32,
 * replica, block + 2^8 floor(step / 2^32)) and key (seed low word, seed
 * high word), using words
 * (2 (p mod 2), 2 (p mod 2) + 1) = (a, b);
 * u1 = ((a >> 8) + 1) 2^-24 in (0, 1], u2 = (b >> 8) 2^-24 in [0, 1),
 * r = sqrt(-2 ln u1), theta = 2 pi u2; even n takes r cos(theta), odd n
 * r sin(theta).  eta[v] = 0 for the conserved modes. */
static void normals(int q, uint64_t seed, uint32_t replica, uint64_t step,
                    uint32_t site, double *eta) {
  const int first = first_noisy_mode(q);
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int v = 0; v < q; ++v) eta[v] = 0.0;
  for (int v = first; v < q; ++v) {
    int n = v - first, p = n / 2, blk = p / 2, wsel = 2 * (p % 2);
    uint32_t ctr[4] = {site, (uint32_t)step, replica,
                       (uint32_t)blk + ((uint32_t)(step >> 32) << 8)}, out[4];
    orc_philox4x32_10(ctr, key, out);
    uint32_t a = out[wsel], b = out[wsel + 1];
    double u1 = ((double)(a >> 8) + 1.0) * ldexp(1.0, -24);
    double u2 = (double)(b >> 8) * ldexp(1.0, -24);
    double r = sqrt(-2.0 * log(u1));
    double th = 2.0 * M_PI * u2;
    eta[v] = (n % 2 == 0) ? r * cos(th) : r * sin(th);
  }
}

/* ---- dense linear algebra ------------------------------------------------ */

static void matvec(int q, const double *A, const double *x, double *y) {
  for (int r = 0; r < q; ++r) {
    double s = 0.0;
    for (int c = 0; c < q; ++c) s += A[r * q + c] * x[c];
    y[r] = s;
  }
}

/* Solve A x = b by Gaussian elimination with partial pivoting (A and b are
 * copied).  Returns 0, or -1 for a singular matrix. */
static int lu_solve(int q, const double *A_in, const double *b_in, double *x) {
  double A[ORC_QMAX * ORC_QMAX], b[ORC_QMAX];
  memcpy(A, A_in, sizeof(double) * q * q);
  memcpy(b, b_in, sizeof(double) * q);
  for (int k = 0; k < q; ++k) {
    int piv = k;
    double best = fabs(A[k * q + k]);
    for (int r = k + 1; r < q; ++r)
      if (fabs(A[r * q + k]) > best) {
        best = fabs(A[r * q + k]);
        piv = r;
      }
    if (best == 0.0) return -1;
    if (piv != k) {
      for (int c = 0; c < q; ++c) {
        double t = A[k * q + c];
        A[k * q + c] = A[piv * q + c];
        A[piv * q + c] = t;
      }
      double t = b[k];
      b[k] = b[piv];
      b[piv] = t;
    }
    for (int r = k + 1; r < q; ++r) {
      double m = A[r * q + k] / A[k * q + k];
      if (m == 0.0) continue;
      for (int c = k; c < q; ++c) A[r * q + c] -= m * A[k * q + c];
      b[r] -= m * b[k];
    }
  }
  for (int r = q - 1; r >= 0; --r) {
    double s = b[r];
    for (int c = r + 1; c < q; ++c) s -= A[r * q + c] * x[c];
    x[r] = s / A[r * q + r];
  }
  return 0;
}

/* f* = M^-1 N(-u) k*, with N(-u) = T(-u) M^-1 and M^-1 = W M^T B^-1 (valid
 * for the orthogonal bases only). */
static void reconstruct_shift(const ctx_t *x, const double u[3],
                              const double *kstar, double *fstar) {
  const int q = x->q;
  double Tm[ORC_QMAX * ORC_QMAX], r[ORC_QMAX], tmp[ORC_QMAX];
  const double mu[3] = {-u[0], -u[1], -u[2]};
  build_T(q, x->basis, mu, Tm);
  /* tmp = M^-1 k* = W M^T B^-1 k* */
  for (int i = 0; i < q; ++i) {
    double s = 0.0;
    for (int v = 0; v < q; ++v) s += x->M[v * q + i] * kstar[v] / x->b[v];
    tmp[i] = x->w[i] * s;
  }
  /* r = T(-u) tmp = N(-u) k* (post-collision raw moments) */
  matvec(q, Tm, tmp, r);
  /* f* = M^-1 r */
  for (int i = 0; i < q; ++i) {
    double s = 0.0;
    for (int v = 0; v < q; ++v) s += x->M[v * q + i] * r[v] / x->b[v];
    fstar[i] = x->w[i] * s;
  }
}

/* ---- one site ------------------------------------------------------------ */

typedef struct {
  double rho, u[3];
} macro_t;

/* Collision at one site.  f: q pre-collision populations; eta: q normals
 * (ignored for the conserved modes); lambda: q relaxation rates; outputs
 * kpre and kstar (may be NULL) and fstar.  Returns 0, or -1 when T(u) is
 * singular. */
static int collide_site(const ctx_t *x, int method, double kT,
                        const double *lambda, const double *f,
                        const double *eta, macro_t *mac, double *kpre_out,
                        double *kstar_out, double *fstar) {
  const int q = x->q;
  double T[ORC_QMAX * ORC_QMAX], k[ORC_QMAX], feq[ORC_QMAX], keq[ORC_QMAX];
  double kstar[ORC_QMAX];
  /* step 1: rho = sum f, rho u = sum c f (eq. macro) */
  double rho = 0.0, j[3] = {0, 0, 0};
  for (int i = 0; i < q; ++i) {
    rho += f[i];
    j[0] += x->c[i][0] * f[i];
    j[1] += x->c[i][1] * f[i];
    j[2] += x->c[i][2] * f[i];
  }
  double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
  if (mac) {
    mac->rho = rho;
    mac->u[0] = u[0];
    mac->u[1] = u[1];
    mac->u[2] = u[2];
  }
  /* step 3: k = T(u) f */
  build_T(q, x->basis, u, T);
  matvec(q, T, f, k);
  /* k_eq = T(u) f_eq(rho, u); D3Q19: k_eq = (rho, 0, ..., 0) as stated */
  if (q == 19) {
    for (int v = 0; v < q; ++v) keq[v] = 0.0;
    keq[0] = rho;
  } else {
    equilibrium(x, rho, u, feq);
    matvec(q, T, feq, keq);
  }
  /* step 4: eq. cm_collision, phi from eq. phi_general with the local rho */
  const int first = first_noisy_mode(q);
  for (int v = 0; v < q; ++v) {
    double L = lambda[v];
    double noise = 0.0;
    if (v >= first) {
      double phi = sqrt(rho * kT * L * (2.0 - L) * x->b[v] / ORC_CS2);
      noise = phi * eta[v];
    }
    kstar[v] = (1.0 - L) * k[v] + L * keq[v] + noise;
  }
  if (kpre_out) memcpy(kpre_out, k, sizeof(double) * q);
  if (kstar_out) memcpy(kstar_out, kstar, sizeof(double) * q);
  /* steps 5-6: f* = T(u)^-1 k* */
  if (method == 1) {
    reconstruct_shift(x, u, kstar, fstar);
    return 0;
  }
  return lu_solve(q, T, kstar, fstar);
}

/* ---- exported API -------------------------------------------------------- */

static int args_ok(int q, int basis) {
  return lattice_ok(q) && (basis == 0 || (basis == 1 && q == 9));
}

/* the second reconstruction path needs N(u)^-1 = N(-u) (not on D3Q19) */
static int method_ok(int q, int method) { return method == 0 || (method == 1 && q != 19); }

int orc_lattice(int q, int32_t *c, double *w) {
  if (!lattice_ok(q)) return -1;
  for (int i = 0; i < q; ++i) {
    double cv[3];
    velocity(q, i, cv);
    c[3 * i + 0] = (int32_t)cv[0];
    c[3 * i + 1] = (int32_t)cv[1];
    c[3 * i + 2] = (int32_t)cv[2];
    w[i] = weight(q, i);
  }
  return 0;
}

/* T(u) for the chosen basis (0 = the paper's orthogonal basis, 1 = the D2Q9
 * non-orthogonal basis).  u = NULL gives the raw-moment matrix M.  Row-major,
 * T[v * q + i]. */
int orc_transform(int q, int basis, const double *u, double *T) {
  if (!args_ok(q, basis)) return -1;
  const double zero[3] = {0, 0, 0};
  build_T(q, basis, u ? u : zero, T);
  return 0;
}

int orc_norms(int q, int basis, double *b) {
  if (!args_ok(q, basis)) return -1;
  build_norms(q, basis, b);
  return 0;
}

int orc_equilibrium(int q, double rho, const double *u, double *feq) {
  if (!lattice_ok(q)) return -1;
  ctx_t x;
  ctx_init(&x, q, 0);
  equilibrium(&x, rho, u, feq);
  return 0;
}

/* Relaxation rates of the paper: D2Q9 Lambda = diag[1,1,1,1,w,w,1,1,1]
 * (Sec. 2.2); D3Q27 Lambda_0-6 = Lambda_10-26 = 1, Lambda_7-9 = w
 * (Sec. 2.3); D3Q19 Lambda_7-9 = w, the rest 1 (Sec. 2.4); w = 1/tau. */
int orc_paper_lambda(int q, double omega, double *lambda) {
  if (!lattice_ok(q)) return -1;
  for (int v = 0; v < q; ++v) lambda[v] = 1.0;
  if (q == 9) {
    lambda[4] = omega;
    lambda[5] = omega;
  } else {
    lambda[7] = omega;
    lambda[8] = omega;
    lambda[9] = omega;
  }
  return 0;
}

int orc_normals(int q, uint64_t seed, uint32_t replica, uint64_t step,
                uint32_t site, double *eta) {
  if (!lattice_ok(q)) return -1;
  normals(q, seed, replica, step, site, eta);
  return 0;
}

/* One collision at one site with caller-given normals.  out_macro receives
 * (rho, u_x, u_y, u_z); every output pointer except fstar may be NULL. */
int orc_collide_site(int q, int basis, int method, double kT,
                     const double *lambda, const double *f, const double *eta,
                     double *out_macro, double *kpre, double *kstar,
                     double *fstar) {
  if (!args_ok(q, basis) || !method_ok(q, method)) return -1;
  ctx_t x;
  ctx_init(&x, q, basis);
  macro_t m;
  int rc = collide_site(&x, method, kT, lambda, f, eta, &m, kpre, kstar, fstar);
  if (out_macro) {
    out_macro[0] = m.rho;
    out_macro[1] = m.u[0];
    out_macro[2] = m.u[1];
    out_macro[3] = m.u[2];
  }
  return rc;
}

/*
 * Advance a periodic lattice by nsteps.
 *   f      : q x N pre-collision populations, SoA, site s = x + nx (y + ny z);
 *            overwritten with the state after the last step.
 *   step0  : index of the first step (the noise counter of that step).
 *   stats  : nsteps x 12 doubles, row t = [step, sum rho, sum rho u (3),
 *            sum u (3), sum u^2 (3), count of sites with non-finite rho or
 *            u], taken from the pre-collision state of that step; may be
 *            NULL.
 * The per-step order is the paper's: macro, noise, collide, reconstruct,
 * stream.  Returns 0, -1 for bad arguments, -2 when some T(u) was singular.
 */
int orc_run(int q, int basis, int method, int nx, int ny, int nz, double kT,
            const double *lambda, uint64_t seed, uint32_t replica, double *f,
            int64_t step0, int64_t nsteps, double *stats, int nthreads) {
  if (!args_ok(q, basis) || !method_ok(q, method) || nx < 1 || ny < 1 || nz < 1) return -1;
  if (q == 9 && nz != 1) return -1;
  ctx_t x;
  ctx_init(&x, q, basis);
  const int64_t N = (int64_t)nx * ny * nz;
  const int64_t nrows = (int64_t)ny * nz;
  double *fstar = (double *)malloc(sizeof(double) * q * N);
  double *rowstat = (double *)malloc(sizeof(double) * nrows * 11);
  if (!fstar || !rowstat) {
    free(fstar);
    free(rowstat);
    return -1;
  }
  int status = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  for (int64_t t = 0; t < nsteps; ++t) {
    const uint64_t step = (uint64_t)(step0 + t);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int64_t row = 0; row < nrows; ++row) {
      double acc[11] = {0};
      const int y = (int)(row % ny), z = (int)(row / ny);
      for (int xi = 0; xi < nx; ++xi) {
        const int64_t s = xi + (int64_t)nx * (y + (int64_t)ny * z);
        double fl[ORC_QMAX], fs[ORC_QMAX], eta[ORC_QMAX];
        for (int i = 0; i < q; ++i) fl[i] = f[i * N + s];
        /* step 2: the normals of this site and step */
        normals(q, seed, replica, step, (uint32_t)s, eta);
        macro_t m;
        if (collide_site(&x, method, kT, lambda, fl, eta, &m, NULL, NULL, fs) !=
            0)
          bad = 1;
        acc[0] += m.rho;
        for (int a = 0; a < 3; ++a) {
          acc[1 + a] += m.rho * m.u[a];
          acc[4 + a] += m.u[a];
          acc[7 + a] += m.u[a] * m.u[a];
        }
        if (!isfinite(m.rho) || !isfinite(m.u[0]) || !isfinite(m.u[1]) ||
            !isfinite(m.u[2]))
          acc[10] += 1.0;
        for (int i = 0; i < q; ++i) fstar[i * N + s] = fs[i];
      }
      memcpy(rowstat + row * 11, acc, sizeof acc);
    }
    if (bad) status = -2;
    if (stats) {
      double *st = stats + t * ORC_NSTAT;
      memset(st, 0, sizeof(double) * ORC_NSTAT);
      st[0] = (double)step;
      for (int64_t row = 0; row < nrows; ++row)
        for (int k = 0; k < 11; ++k) st[1 + k] += rowstat[row * 11 + k];
    }
    /* step 7: f_i(x + c_i, t + 1) = f*_i(x, t), periodic (eq. streaming) */
#pragma omp parallel for schedule(static)
    for (int64_t row = 0; row < nrows; ++row) {
      const int y = (int)(row % ny), z = (int)(row / ny);
      for (int i = 0; i < q; ++i) {
        const int cx = (int)x.c[i][0], cy = (int)x.c[i][1], cz = (int)x.c[i][2];
        const int yd = ((y + cy) % ny + ny) % ny;
        const int zd = ((z + cz) % nz + nz) % nz;
        for (int xi = 0; xi < nx; ++xi) {
          const int xd = ((xi + cx) % nx + nx) % nx;
          const int64_t s = xi + (int64_t)nx * (y + (int64_t)ny * z);
          const int64_t d = xd + (int64_t)nx * (yd + (int64_t)ny * zd);
          f[i * N + d] = fstar[i * N + s];
        }
      }
    }
  }
  free(fstar);
  free(rowstat);
  return status;
}

/* Fill q x N populations with the equilibrium of per-site rho (N values, or
 * NULL for rho0) and u (3 x N values, SoA, or NULL for rest). */
int orc_init_equilibrium(int q, int64_t N, double rho0, const double *rho,
                         const double *u, double *f) {
  if (!lattice_ok(q) || N < 0) return -1;
  ctx_t x;
  ctx_init(&x, q, 0);
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < N; ++s) {
    double uu[3] = {0, 0, 0}, feq[ORC_QMAX];
    if (u) {
      uu[0] = u[s];
      uu[1] = u[N + s];
      uu[2] = u[2 * N + s];
    }
    equilibrium(&x, rho ? rho[s] : rho0, uu, feq);
    for (int i = 0; i < q; ++i) f[i * N + s] = feq[i];
  }
  return 0;
}

int orc_nstat(void) { return ORC_NSTAT; }

/* Hermite tensor component H^(n)_{idx[0..n-1]}(c), idx entries 0=x 1=y 2=z. */
double orc_hermite(const double *c, const int32_t *idx, int n) {
  int local[8];
  if (n < 0 || n > 8) return NAN;
  for (int k = 0; k < n; ++k) local[k] = idx[k];
  return hermite(c, local, n);
}
