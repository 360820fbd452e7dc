/*
 * CPU oracle for the balanced-tree FMM evaluation pass (1/r kernel, 3D).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this code:
 * it is used by the test-suite, by the smoke check and by the benchmark's
 * CPU-baseline leg.  It shares no code with the GPU library.
 *
 * Plain, slow and written to be checked by eye against the paper
 * (Bull & Engblom, "Distributed and adaptive fast multipole method in three
 * dimensions") and against the textbook expansion theorems the paper defers
 * to (Greengard-Rokhlin spherical-harmonic expansions, its reference
 * "greengardshortcourse").  All arithmetic is IEEE binary64; build with
 * -O2 -ffp-contract=off and without -ffast-math.
 *
 * Conventions (readings of the paper, listed in the design notes):
 *  - Kernel: G(x_i, x_j) = q_j / |x_i - x_j|; field E = -grad(phi).
 *    Pairs at distance 0 contribute nothing (this covers j == i, eq. (2.1)).
 *  - "levels" L = number of 8-way splits; leaves are the 8^L boxes of level L.
 *  - Root cell = tight axis-aligned bounding box of the points (Section 2.1).
 *  - Every box of level l < L is split into 8 by three successive median
 *    bisections (Section 2.1.2, eta = 1), each along the longest edge of the
 *    current cell (ties: x before y before z).  The low side receives
 *    floor(n/2) points in the total order (coordinate, original index), the
 *    split plane is the midpoint of the two middle coordinates (the point's
 *    own coordinate when n = 1, the cell midpoint when n = 0), and the
 *    partition is stable (points keep ascending original
 *    index inside every box).  Child number = 4*b1 + 2*b2 + b3 with b_i = 1
 *    for the high side of bisection i; global index 8*parent + child.
 *    Coordinates are read through x + 0.0, which maps -0.0 to +0.0.
 *  - Box centre = cell centre, box radius = half the cell diagonal.
 *  - theta-criterion, eq. (2.2): distinct boxes with centre distance d > 0
 *    are weakly connected iff R + theta*r <= theta*d (R, r = larger, smaller
 *    radius); otherwise strongly connected.  Connections are inherited as in
 *    Section 2.1.1: only children of strongly connected parents are tested.
 *  - Expansion order p = highest degree kept, (p+1)^2 complex terms.
 *  - M2L at every level 1..L, L2L for levels 1..L-1 (reading of Algorithm 3).
 *  - M2L has two forms with the same result up to rounding: the basic
 *    O(p^4) translation theorem (default) and the rotational O(p^3) form the
 *    paper uses (Section 2.1.3), selected by orc_set_m2l_form.  The test-suite
 *    pins each against the other.
 *  - OpenMP threads share out independent boxes, leaves and targets only;
 *    every sum runs in the same order as with one thread.
 *
 * Pins: the test-suite checks every function here against closed forms,
 * hand-derived golden trees and lists, exactness identities of the
 * translations, the published truncation bounds, and the reductions of the
 * whole method to the direct sum (L = 0, theta = 0).  The paper prints no
 * error values for its convergence experiment (Section 3.1), so the error
 * levels of the whole method are parity unpinned against numbers of the
 * paper's own: they are pinned only to the shape of its bound.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>


#define ORC_PMAX 20
#define NTERMS(p) (((p) + 1) * ((p) + 1))
#define IDX(n, m) ((n) * (n) + (n) + (m))

typedef double complex cplx;

/* Allocation that stops the process with a message when memory runs out
 * (the lists of very large trees can exceed the host's memory). */
static void* xmalloc(size_t bytes) {
  void* p = malloc(bytes);
  if (!p) {
    fprintf(stderr, "oracle: out of host memory allocating %zu bytes\n", bytes);
    abort();
  }
  return p;
}
static void* xcalloc(size_t count, size_t size) {
  void* p = calloc(count, size);
  if (!p) {
    fprintf(stderr, "oracle: out of host memory allocating %zu x %zu bytes\n", count, size);
    abort();
  }
  return p;
}

/* ------------------------------------------------------------------------ */
/* Direct sum, eq. (2.1).                                                   */
/* ------------------------------------------------------------------------ */

/* Neumaier-compensated accumulator. */
typedef struct { double s, c; } acc_t;
static void acc_add(acc_t* a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
  else a->c += (v - t) + a->s;
  a->s = t;
}
static double acc_get(const acc_t* a) { return a->s + a->c; }

/* phi_i = sum_{j != i, r_ij > 0} q_j / r_ij,  E_i = sum q_j (x_i - x_j) / r_ij^3,
 * for the nt targets listed in `targets` (or all n when targets == NULL).
 * Outputs are indexed by target slot (0..nt-1). */
void orc_direct(int64_t n, const double* x, const double* y, const double* z, const double* q,
                int64_t nt, const int64_t* targets, double* phi, double* ex, double* ey, double* ez) {
  if (targets == NULL) nt = n;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < nt; ++k) {
    int64_t i = targets ? targets[k] : k;
    acc_t ap = {0, 0}, ax = {0, 0}, ay = {0, 0}, az = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
      double r2 = dx * dx + dy * dy + dz * dz;
      if (r2 == 0.0) continue;
      double r = sqrt(r2);
      double inv = 1.0 / r;
      double inv3 = inv / r2;
      acc_add(&ap, q[j] * inv);
      acc_add(&ax, q[j] * dx * inv3);
      acc_add(&ay, q[j] * dy * inv3);
      acc_add(&az, q[j] * dz * inv3);
    }
    phi[k] = acc_get(&ap);
    ex[k] = acc_get(&ax);
    ey[k] = acc_get(&ay);
    ez[k] = acc_get(&az);
  }
}

/* ------------------------------------------------------------------------ */
/* Spherical harmonics (Greengard-Rokhlin normalisation, no Condon-Shortley   */
/* phase):  Y_n^m(a,b) = sqrt((n-|m|)!/(n+|m|)!) P_n^|m|(cos a) e^{i m b}.    */
/* ------------------------------------------------------------------------ */

static double g_fact[2 * 2 * ORC_PMAX + 2];
static void init_fact(void) {
  if (g_fact[0] == 1.0) return;
  g_fact[0] = 1.0;
  for (int i = 1; i < (int)(sizeof(g_fact) / sizeof(g_fact[0])); ++i) g_fact[i] = g_fact[i - 1] * (double)i;
}

/* Regular solid harmonics S_n^m(u) = |u|^n Y_n^m(angles of u), n <= nmax,
 * together with their Cartesian gradients (when grad != NULL).  Built from
 * Q_n^m = r^n P_n^m(cos t) e^{i m f} (m >= 0), which obeys the Legendre
 * recurrences multiplied by r^n:
 *   Q_m^m = (2m-1) (x + i y) Q_{m-1}^{m-1},
 *   Q_{m+1}^m = (2m+1) z Q_m^m,
 *   (n-m) Q_n^m = (2n-1) z Q_{n-1}^m - (n+m-1) r^2 Q_{n-2}^m;
 * gradients follow by the product rule.  S_n^{-m} = conj(S_n^m). */
static void solid_harmonics(int nmax, double ux, double uy, double uz, cplx* S, cplx (*grad)[3]) {
  static __thread cplx Q[(2 * ORC_PMAX + 1) * (2 * ORC_PMAX + 1)];
  static __thread cplx G[(2 * ORC_PMAX + 1) * (2 * ORC_PMAX + 1)][3];
  init_fact();
  const double r2 = ux * ux + uy * uy + uz * uz;
  const cplx w = ux + I * uy;
  const int want_grad = grad != NULL;
#define QI(n, m) ((n) * ((n) + 1) / 2 + (m))
  Q[QI(0, 0)] = 1.0;
  if (want_grad) G[QI(0, 0)][0] = G[QI(0, 0)][1] = G[QI(0, 0)][2] = 0.0;
  for (int m = 0; m <= nmax; ++m) {
    if (m > 0) {
      const cplx prev = Q[QI(m - 1, m - 1)];
      Q[QI(m, m)] = (double)(2 * m - 1) * w * prev;
      if (want_grad) {
        G[QI(m, m)][0] = (double)(2 * m - 1) * (prev + w * G[QI(m - 1, m - 1)][0]);
        G[QI(m, m)][1] = (double)(2 * m - 1) * (I * prev + w * G[QI(m - 1, m - 1)][1]);
        G[QI(m, m)][2] = (double)(2 * m - 1) * (w * G[QI(m - 1, m - 1)][2]);
      }
    }
    if (m + 1 <= nmax) {
      const cplx qm = Q[QI(m, m)];
      Q[QI(m + 1, m)] = (double)(2 * m + 1) * uz * qm;
      if (want_grad) {
        G[QI(m + 1, m)][0] = (double)(2 * m + 1) * uz * G[QI(m, m)][0];
        G[QI(m + 1, m)][1] = (double)(2 * m + 1) * uz * G[QI(m, m)][1];
        G[QI(m + 1, m)][2] = (double)(2 * m + 1) * (qm + uz * G[QI(m, m)][2]);
      }
    }
    for (int n = m + 2; n <= nmax; ++n) {
      const cplx a = Q[QI(n - 1, m)], b = Q[QI(n - 2, m)];
      const double c1 = (double)(2 * n - 1), c2 = (double)(n + m - 1), inv = 1.0 / (double)(n - m);
      Q[QI(n, m)] = (c1 * uz * a - c2 * r2 * b) * inv;
      if (want_grad) {
        const double du[3] = {ux, uy, uz};
        for (int d = 0; d < 3; ++d) {
          cplx t = c1 * uz * G[QI(n - 1, m)][d] - c2 * r2 * G[QI(n - 2, m)][d] - c2 * (2.0 * du[d]) * b;
          if (d == 2) t += c1 * a;
          G[QI(n, m)][d] = t * inv;
        }
      }
    }
  }
  for (int n = 0; n <= nmax; ++n) {
    for (int m = 0; m <= n; ++m) {
      const double nrm = sqrt(g_fact[n - m] / g_fact[n + m]);
      const cplx s = nrm * Q[QI(n, m)];
      S[IDX(n, m)] = s;
      S[IDX(n, -m)] = conj(s);
      if (want_grad) {
        for (int d = 0; d < 3; ++d) {
          const cplx g = nrm * G[QI(n, m)][d];
          grad[IDX(n, m)][d] = g;
          grad[IDX(n, -m)][d] = conj(g);
        }
      }
    }
  }
#undef QI
}

/* Y_n^m at the direction of v (unit-sphere values), n <= nmax; also |v|. */
static double sph_harmonics(int nmax, double vx, double vy, double vz, cplx* Y) {
  const double rho = sqrt(vx * vx + vy * vy + vz * vz);
  solid_harmonics(nmax, vx / rho, vy / rho, vz / rho, Y, NULL);
  return rho;
}

/* A_n^m = (-1)^n / sqrt((n-m)!(n+m)!), tabulated once for n <= 2*ORC_PMAX */
static double g_A[2 * ORC_PMAX + 1][2 * ORC_PMAX + 1];
static int g_A_ready;
static double Acoef(int n, int m) {
  if (!g_A_ready) {
    init_fact();
    for (int a = 0; a <= 2 * ORC_PMAX; ++a)
      for (int b = 0; b <= a; ++b) g_A[a][b] = ((a & 1) ? -1.0 : 1.0) / sqrt(g_fact[a - b] * g_fact[a + b]);
    g_A_ready = 1;
  }
  return g_A[n][m];
}

/* Tables that are filled lazily; filled before any parallel region. */
static void orc_init(void) {
  init_fact();
  (void)Acoef(0, 0);
}

/* i^e for any integer e */
static cplx ipow(int e) {
  switch (((e % 4) + 4) % 4) {
    case 0: return 1.0;
    case 1: return I;
    case 2: return -1.0;
    default: return -I;
  }
}

/* ------------------------------------------------------------------------ */
/* Expansion operators (Section 2.1; Algorithm 1 for their order of use).   */
/* Coefficients are stored at IDX(n,m) = n^2 + n + m, -n <= m <= n.          */
/* ------------------------------------------------------------------------ */

/* P2M: multipole about centre c of charges q_i at x_i (Algorithm 1, P2M):
 *   M_n^m = sum_i q_i rho_i^n Y_n^{-m}(alpha_i, beta_i),
 * (rho_i, alpha_i, beta_i) = spherical coordinates of x_i - c. */
void orc_p2m(int p, double cx, double cy, double cz, int64_t n, const double* x, const double* y,
             const double* z, const double* q, cplx* M) {
  cplx S[NTERMS(ORC_PMAX)];
  for (int k = 0; k < NTERMS(p); ++k) M[k] = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    solid_harmonics(p, x[i] - cx, y[i] - cy, z[i] - cz, S, NULL);
    for (int nn = 0; nn <= p; ++nn)
      for (int m = -nn; m <= nn; ++m) M[IDX(nn, m)] += q[i] * S[IDX(nn, -m)];
  }
}

/* M2M: multipole O about an old centre at (rho, alpha, beta) relative to the
 * new centre -> multipole about the new centre (Algorithm 1, M2M):
 *   M_j^k = sum_{n=0}^{j} sum_{m=-n}^{n} O_{j-n}^{k-m} i^{|k|-|m|-|k-m|}
 *           A_n^m A_{j-n}^{k-m} rho^n Y_n^{-m}(alpha, beta) / A_j^k.
 * d = old centre - new centre. */
void orc_m2m(int p, const cplx* O, double dx, double dy, double dz, cplx* M) {
  cplx Y[NTERMS(ORC_PMAX)];
  init_fact();
  for (int k = 0; k < NTERMS(p); ++k) M[k] = 0.0;
  const double rho2 = dx * dx + dy * dy + dz * dz;
  if (rho2 == 0.0) {
    for (int k = 0; k < NTERMS(p); ++k) M[k] = O[k];
    return;
  }
  const double rho = sph_harmonics(p, dx, dy, dz, Y);
  for (int j = 0; j <= p; ++j)
    for (int k = -j; k <= j; ++k) {
      cplx acc = 0.0;
      for (int n = 0; n <= j; ++n) {
        const double rn = pow(rho, (double)n);
        for (int m = -n; m <= n; ++m) {
          const int jn = j - n, km = k - m;
          if (abs(km) > jn) continue;
          acc += O[IDX(jn, km)] * ipow(abs(k) - abs(m) - abs(km)) * Acoef(n, abs(m)) * Acoef(jn, abs(km)) * rn *
                 Y[IDX(n, -m)];
        }
      }
      M[IDX(j, k)] = acc / Acoef(j, abs(k));
    }
}

/* M2L: multipole O about a source centre at (rho, alpha, beta) relative to the
 * target centre -> local expansion about the target centre (the M2L shift of
 * Section 2.1.3 and Algorithm 3, in its basic O(p^4) form):
 *   L_j^k = sum_{n=0}^{p} sum_{m=-n}^{n} O_n^m i^{|k-m|-|k|-|m|} A_n^m A_j^k
 *           Y_{j+n}^{m-k}(alpha, beta) / ((-1)^n A_{j+n}^{m-k} rho^{j+n+1}).
 * d = source centre - target centre.  The result is added to L. */
void orc_m2l_add(int p, const cplx* O, double dx, double dy, double dz, cplx* L) {
  cplx Y[NTERMS(2 * ORC_PMAX)];
  init_fact();
  const double rho = sph_harmonics(2 * p, dx, dy, dz, Y);
  for (int j = 0; j <= p; ++j)
    for (int k = -j; k <= j; ++k) {
      cplx acc = 0.0;
      for (int n = 0; n <= p; ++n) {
        const double sgn_n = (n & 1) ? -1.0 : 1.0;
        const double rpow = pow(rho, (double)(j + n + 1));
        for (int m = -n; m <= n; ++m) {
          const int mk = m - k;
          acc += O[IDX(n, m)] * ipow(abs(k - m) - abs(k) - abs(m)) * Acoef(n, abs(m)) * Acoef(j, abs(k)) *
                 Y[IDX(j + n, mk)] / (sgn_n * Acoef(j + n, abs(mk)) * rpow);
        }
      }
      L[IDX(j, k)] += acc;
    }
}

/* ------------------------------------------------------------------------ */
/* M2L in rotational form (Section 2.1.3: the z-axis of the expansion is    */
/* turned onto the vector between the two centres, O(p^3) per pair).        */
/* ------------------------------------------------------------------------ */

/* For a rotation R let D_n(R) be defined by Y_n^m(R u) = sum_m' D[m][m']
 * Y_n^m'(u) for unit u.  Then D(R1 R2) = D(R1) D(R2), D(Rz(g)) = diag(e^{i m g}),
 * and D is unitary (all Y_n^m have the same norm 4 pi / (2n+1) over the
 * sphere).  Only D_n(K) for the fixed quarter turn K = Rx(-pi/2) (K z = y) is
 * tabulated, by projection:
 *   D[m][m'] = (2n+1)/(4 pi) * integral Y_n^m(K u) conj(Y_n^m'(u)) du,
 * with a product rule exact for these integrands: Gauss-Legendre in cos(t)
 * with n+1 nodes (exact to degree 2n+1) and 2n+1 equispaced azimuths (which
 * cancel every azimuthal frequency 0 < |f| <= 2n). */
static cplx* g_dk[ORC_PMAX + 1];

/* P_k(t) and P_{k-1}(t) by the three-term Legendre recurrence */
static void legendre_pair(int k, double t, double* pk, double* pkm1) {
  double p0 = 1.0, p1 = t;
  for (int j = 2; j <= k; ++j) {
    const double p2 = ((2.0 * j - 1.0) * t * p1 - (j - 1.0) * p0) / j;
    p0 = p1;
    p1 = p2;
  }
  *pk = p1;
  *pkm1 = p0;
}

/* Gauss-Legendre nodes and weights on [-1, 1] (npts >= 1): Newton's method
 * on P_npts from the usual cosine guesses; w = 2 / ((1 - t^2) P'(t)^2). */
static void gauss_legendre_nodes(int npts, double* x, double* w) {
  for (int i = 0; i < npts; ++i) {
    double t = cos(M_PI * (i + 0.75) / (npts + 0.5));
    for (int it = 0; it < 100; ++it) {
      double pk, pm;
      legendre_pair(npts, t, &pk, &pm);
      const double dp = npts * (t * pk - pm) / (t * t - 1.0);
      const double dt = pk / dp;
      t -= dt;
      if (fabs(dt) <= 1e-15 * fabs(t) + 1e-300) break;
    }
    double pk, pm;
    legendre_pair(npts, t, &pk, &pm);
    const double dp = npts * (t * pk - pm) / (t * t - 1.0);
    x[i] = t;
    w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

static void rot_tables(int p) {
  init_fact();
  for (int n = 0; n <= p; ++n) {
    if (g_dk[n]) continue;
    const int w2 = 2 * n + 1;
    cplx* D = (cplx*)xcalloc((size_t)w2 * w2, sizeof(cplx));
    double xs[ORC_PMAX + 1], ws[ORC_PMAX + 1];
    gauss_legendre_nodes(n + 1, xs, ws);
    cplx Yu[NTERMS(ORC_PMAX)], Yk[NTERMS(ORC_PMAX)];
    for (int i = 0; i <= n; ++i) {
      const double ct = xs[i], st = sqrt(1.0 - ct * ct);
      for (int k = 0; k < w2; ++k) {
        const double ph = 2.0 * M_PI * k / w2;
        const double ux = st * cos(ph), uy = st * sin(ph), uz = ct;
        solid_harmonics(n, ux, uy, uz, Yu, NULL);
        solid_harmonics(n, ux, uz, -uy, Yk, NULL); /* K u = (x, z, -y) */
        const double wt = ws[i] * (2.0 * M_PI / w2) * (2.0 * n + 1.0) / (4.0 * M_PI);
        for (int m = -n; m <= n; ++m)
          for (int mp = -n; mp <= n; ++mp) D[(m + n) * w2 + (mp + n)] += wt * Yk[IDX(n, m)] * conj(Yu[IDX(n, mp)]);
      }
    }
    g_dk[n] = D;
  }
}

/* The same result as orc_m2l_add (up to rounding), computed by rotation.
 * With d = rho (sin a cos b, sin a sin b, cos a) and Q = Rz(b) K Rz(a) K^-1
 * (Q z = d/rho), the far field about the source centre, written in the frame
 * x = Q x', has coefficients O' = D(Q)^T O per degree, i.e.
 *   O' = conj(D(K)) Dz(a) D(K)^T Dz(b) O;
 * along the z-axis the translation theorem keeps the order k:
 *   L'_j^k = sum_{n >= |k|} O'_n^k (-1)^|k| A_n^k A_j^k / ((-1)^n A_{j+n}^0 rho^{j+n+1});
 * and the local expansion returns to the original frame by the inverse of
 * D(Q)^T, which is conj(D(Q)):
 *   L = Dz(-b) conj(D(K)) Dz(-a) D(K)^T L'.
 * d = source centre - target centre.  The result is added to L.  The tables
 * of order p must exist (orc_rot_prepare) before parallel use. */
void orc_m2l_rot_add(int p, const cplx* O, double dx, double dy, double dz, cplx* L) {
  rot_tables(p);
  const double rxy = sqrt(dx * dx + dy * dy);
  const double rho = sqrt(dx * dx + dy * dy + dz * dz);
  const double a = atan2(rxy, dz), b = atan2(dy, dx);
  cplx Op[NTERMS(ORC_PMAX)], Lp[NTERMS(ORC_PMAX)];
  cplx w[2 * ORC_PMAX + 1], v[2 * ORC_PMAX + 1];
  for (int n = 0; n <= p; ++n) {
    const cplx* D = g_dk[n];
    const int w2 = 2 * n + 1;
    for (int m = -n; m <= n; ++m) w[m + n] = cexp(I * (double)m * b) * O[IDX(n, m)];
    for (int mp = -n; mp <= n; ++mp) {
      cplx acc = 0.0;
      for (int m = -n; m <= n; ++m) acc += D[(m + n) * w2 + (mp + n)] * w[m + n];
      v[mp + n] = cexp(I * (double)mp * a) * acc;
    }
    for (int m = -n; m <= n; ++m) {
      cplx acc = 0.0;
      for (int q = -n; q <= n; ++q) acc += conj(D[(m + n) * w2 + (q + n)]) * v[q + n];
      Op[IDX(n, m)] = acc;
    }
  }
  for (int j = 0; j <= p; ++j)
    for (int k = -j; k <= j; ++k) {
      const int ak = abs(k);
      cplx acc = 0.0;
      for (int n = ak; n <= p; ++n) {
        const double sgn = (((n + ak) & 1) ? -1.0 : 1.0);
        acc += Op[IDX(n, k)] * (sgn * Acoef(n, ak) * Acoef(j, ak) / (Acoef(j + n, 0) * pow(rho, (double)(j + n + 1))));
      }
      Lp[IDX(j, k)] = acc;
    }
  for (int j = 0; j <= p; ++j) {
    const cplx* D = g_dk[j];
    const int w2 = 2 * j + 1;
    for (int mp = -j; mp <= j; ++mp) {
      cplx acc = 0.0;
      for (int m = -j; m <= j; ++m) acc += D[(m + j) * w2 + (mp + j)] * Lp[IDX(j, m)];
      w[mp + j] = cexp(-I * (double)mp * a) * acc;
    }
    for (int m = -j; m <= j; ++m) {
      cplx acc = 0.0;
      for (int q = -j; q <= j; ++q) acc += conj(D[(m + j) * w2 + (q + j)]) * w[q + j];
      L[IDX(j, m)] += cexp(-I * (double)m * b) * acc;
    }
  }
}

/* Which M2L form the whole-method evaluation uses: 0 = the basic O(p^4)
 * translation theorem (default), 1 = the rotational form. */
static int g_m2l_rot = 0;
void orc_set_m2l_form(int rotational) { g_m2l_rot = rotational != 0; }
/* Threads of the parallel loops (0 or less: the OpenMP default); returns the
 * number the next parallel region will use. */
int orc_set_threads(int nthreads) {
  if (nthreads > 0) omp_set_num_threads(nthreads);
  return omp_get_max_threads();
}
void orc_rot_prepare(int p) { orc_init(); rot_tables(p); }

static void m2l_add(int p, const cplx* O, double dx, double dy, double dz, cplx* L) {
  if (g_m2l_rot) orc_m2l_rot_add(p, O, dx, dy, dz, L);
  else orc_m2l_add(p, O, dx, dy, dz, L);
}

/* L2L: local expansion O about an old centre at (rho, alpha, beta) relative to
 * the new centre -> local expansion about the new centre (Algorithm 3, L2L):
 *   L_j^k = sum_{n=j}^{p} sum_{m=-n}^{n} O_n^m i^{|m|-|m-k|-|k|} A_{n-j}^{m-k}
 *           A_j^k rho^{n-j} Y_{n-j}^{m-k}(alpha, beta) / ((-1)^{n+j} A_n^m).
 * d = old centre - new centre.  The result is added to L. */
void orc_l2l_add(int p, const cplx* O, double dx, double dy, double dz, cplx* L) {
  cplx Y[NTERMS(ORC_PMAX)];
  init_fact();
  const double rho2 = dx * dx + dy * dy + dz * dz;
  if (rho2 == 0.0) {
    for (int k = 0; k < NTERMS(p); ++k) L[k] += O[k];
    return;
  }
  const double rho = sph_harmonics(p, dx, dy, dz, Y);
  for (int j = 0; j <= p; ++j)
    for (int k = -j; k <= j; ++k) {
      cplx acc = 0.0;
      for (int n = j; n <= p; ++n) {
        const double sgn = ((n + j) & 1) ? -1.0 : 1.0;
        const double rn = pow(rho, (double)(n - j));
        for (int m = -n; m <= n; ++m) {
          const int mk = m - k, nj = n - j;
          if (abs(mk) > nj) continue;
          acc += O[IDX(n, m)] * ipow(abs(m) - abs(mk) - abs(k)) * Acoef(nj, abs(mk)) * Acoef(j, abs(k)) * rn *
                 Y[IDX(nj, mk)] / (sgn * Acoef(n, abs(m)));
        }
      }
      L[IDX(j, k)] += acc;
    }
}

/* L2P: phi(x) = sum_j sum_k L_j^k Y_j^k(theta, phi) r^j about centre c, and
 * E = -grad(phi) (Algorithm 4, L2P).  Results are added to the outputs. */
void orc_l2p_add(int p, const cplx* L, double cx, double cy, double cz, double x, double y, double z,
                 double* phi, double* ex, double* ey, double* ez) {
  cplx S[NTERMS(ORC_PMAX)];
  cplx G[NTERMS(ORC_PMAX)][3];
  solid_harmonics(p, x - cx, y - cy, z - cz, S, G);
  cplx f = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
  for (int k = 0; k < NTERMS(p); ++k) {
    f += L[k] * S[k];
    gx += L[k] * G[k][0];
    gy += L[k] * G[k][1];
    gz += L[k] * G[k][2];
  }
  *phi += creal(f);
  *ex -= creal(gx);
  *ey -= creal(gy);
  *ez -= creal(gz);
}

/* Far-field evaluation of a multipole expansion (used by the tests only):
 * phi(x) = sum_n sum_m M_n^m Y_n^m(theta, phi) / r^{n+1}. */
void orc_m2p(int p, const cplx* M, double cx, double cy, double cz, double x, double y, double z, double* phi) {
  cplx S[NTERMS(ORC_PMAX)];
  const double ux = x - cx, uy = y - cy, uz = z - cz;
  const double r = sqrt(ux * ux + uy * uy + uz * uz);
  solid_harmonics(p, ux, uy, uz, S, NULL);
  cplx f = 0.0;
  for (int n = 0; n <= p; ++n) {
    const double rr = pow(r, (double)(2 * n + 1));
    for (int m = -n; m <= n; ++m) f += M[IDX(n, m)] * S[IDX(n, m)] / rr;
  }
  *phi = creal(f);
}

/* Local expansion of point charges about centre c (used by the tests only):
 * L_j^k = sum_i q_i Y_j^{-k}(alpha_i, beta_i) / rho_i^{j+1}. */
void orc_p2l(int p, double cx, double cy, double cz, int64_t n, const double* x, const double* y,
             const double* z, const double* q, cplx* L) {
  cplx Y[NTERMS(ORC_PMAX)];
  for (int k = 0; k < NTERMS(p); ++k) L[k] = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double rho = sph_harmonics(p, x[i] - cx, y[i] - cy, z[i] - cz, Y);
    for (int j = 0; j <= p; ++j) {
      const double rr = pow(rho, (double)(j + 1));
      for (int k = -j; k <= j; ++k) L[IDX(j, k)] += q[i] * Y[IDX(j, -k)] / rr;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Balanced tree by median splits (Section 2.1.2, eta = 1; Algorithm 2).     */
/* ------------------------------------------------------------------------ */

typedef struct {
  int64_t nbox;     /* 8^l */
  double* geom;     /* nbox x 10: lo[3], hi[3], centre[3], radius */
  int64_t* start;   /* nbox + 1: point range of each box in tree order */
  int64_t* s_off;   /* strong list, CSR by target box: nbox + 1 offsets */
  int32_t* s_idx;
  int64_t* w_off;   /* weak list, CSR by target box */
  int32_t* w_idx;
} orc_level;

typedef struct {
  int64_t n;
  int L;
  double theta;
  double eta;              /* split parameter, Section 2.1.2 */
  const double *x, *y, *z; /* caller's arrays, input order */
  int64_t m;               /* separate evaluation targets (may be 0) */
  const double *tx, *ty, *tz;
  int32_t* perm;           /* tree order -> original index */
  orc_level* lev;          /* levels 0..L */
  char* listed;            /* targeted mode: leaves whose chains have lists (NULL: all) */
} orc_tree;

typedef struct { double key; int32_t idx; } kv_t;

/* total order (coordinate, original index) */
static int kv_cmp(const void* a, const void* b) {
  const kv_t* u = (const kv_t*)a;
  const kv_t* v = (const kv_t*)b;
  if (u->key < v->key) return -1;
  if (u->key > v->key) return 1;
  return (u->idx > v->idx) - (u->idx < v->idx);
}

static double coord(const orc_tree* t, int axis, int32_t i) {
  const double* c = axis == 0 ? t->x : axis == 1 ? t->y : t->z;
  return c[i] + 0.0; /* -0.0 -> +0.0 */
}

/* One bisection of the points perm[s..e) inside cell (lo, hi): chooses the
 * axis, reorders perm[s..e) stably into low | high and returns the size of
 * the low side; writes the split plane coordinate and axis.
 * eta = 1: the median split below.  eta < 1 (Section 2.1.2): the plane is the
 * weighted average (1 - eta) * (cell midpoint) + eta * (the eta = 1 plane),
 * and the points whose coordinate lies below it form the low side. */
static int64_t bisect_median(const orc_tree* t, int32_t* perm, int64_t s, int64_t e, const double lo[3],
                             const double hi[3], int* axis_out, double* plane_out, kv_t* kv, int32_t* tmp);

static int64_t bisect(const orc_tree* t, int32_t* perm, int64_t s, int64_t e, const double lo[3],
                      const double hi[3], int* axis_out, double* plane_out, kv_t* kv, int32_t* tmp,
                      int32_t* scratch) {
  if (t->eta == 1.0) return bisect_median(t, perm, s, e, lo, hi, axis_out, plane_out, kv, tmp);
  /* the eta = 1 plane, found on a copy so that perm keeps its order */
  memcpy(scratch, perm + s, (size_t)(e - s) * sizeof(int32_t));
  double plane1;
  bisect_median(t, scratch, 0, e - s, lo, hi, axis_out, &plane1, kv, tmp);
  const int axis = *axis_out;
  const double mid = 0.5 * (lo[axis] + hi[axis]);
  const double plane = (1.0 - t->eta) * mid + t->eta * plane1;
  int64_t nl = 0, nh = 0;
  for (int64_t i = s; i < e; ++i) {
    if (coord(t, axis, perm[i]) < plane) scratch[nl++] = perm[i];
    else tmp[nh++] = perm[i];
  }
  memcpy(perm + s, scratch, (size_t)nl * sizeof(int32_t));
  memcpy(perm + s + nl, tmp, (size_t)nh * sizeof(int32_t));
  *plane_out = plane;
  return nl;
}

static int64_t bisect_median(const orc_tree* t, int32_t* perm, int64_t s, int64_t e, const double lo[3],
                             const double hi[3], int* axis_out, double* plane_out, kv_t* kv, int32_t* tmp) {
  int axis = 0;
  double ext = hi[0] - lo[0];
  for (int a = 1; a < 3; ++a)
    if (hi[a] - lo[a] > ext) { ext = hi[a] - lo[a]; axis = a; }
  const int64_t n = e - s;
  const int64_t m = n / 2;
  double plane;
  if (n == 0) {
    plane = 0.5 * (lo[axis] + hi[axis]);
  } else if (n == 1) {
    /* the single point goes to the high side (the low side gets floor(1/2) = 0
     * points) and the plane passes through it, so it stays inside its cell */
    plane = coord(t, axis, perm[s]);
  } else {
    for (int64_t i = 0; i < n; ++i) { kv[i].key = coord(t, axis, perm[s + i]); kv[i].idx = perm[s + i]; }
    qsort(kv, (size_t)n, sizeof(kv_t), kv_cmp);
    plane = 0.5 * (kv[m - 1].key + kv[m].key);
    const kv_t piv = kv[m];
    int64_t nl = 0, nh = 0;
    for (int64_t i = 0; i < n; ++i) {
      kv_t me = {coord(t, axis, perm[s + i]), perm[s + i]};
      if (kv_cmp(&me, &piv) < 0) perm[s + nl++] = me.idx;
      else tmp[nh++] = me.idx;
    }
    memcpy(perm + s + nl, tmp, (size_t)nh * sizeof(int32_t));
  }
  *axis_out = axis;
  *plane_out = plane;
  return m;
}

static void build_tree(orc_tree* t) {
  const int L = t->L;
  const int64_t n = t->n;
  t->perm = (int32_t*)xmalloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  for (int64_t i = 0; i < n; ++i) t->perm[i] = (int32_t)i;
  t->lev = (orc_level*)xcalloc((size_t)L + 1, sizeof(orc_level));
  int64_t nb = 1;
  for (int l = 0; l <= L; ++l, nb *= 8) {
    t->lev[l].nbox = nb;
    t->lev[l].geom = (double*)xcalloc((size_t)nb * 10, sizeof(double));
    t->lev[l].start = (int64_t*)xcalloc((size_t)nb + 1, sizeof(int64_t));
  }
  /* root: tight bounding box of the sources and of the separate targets */
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int a = 0; a < 3; ++a) {
    if (n > 0) { lo[a] = hi[a] = coord(t, a, 0); }
    for (int64_t i = 1; i < n; ++i) {
      const double c = coord(t, a, (int32_t)i);
      if (c < lo[a]) lo[a] = c;
      if (c > hi[a]) hi[a] = c;
    }
    const double* tc = a == 0 ? t->tx : a == 1 ? t->ty : t->tz;
    for (int64_t i = 0; i < t->m; ++i) {
      const double c = tc[i] + 0.0;
      if (c < lo[a]) lo[a] = c;
      if (c > hi[a]) hi[a] = c;
    }
  }
  double* g0 = t->lev[0].geom;
  for (int a = 0; a < 3; ++a) { g0[a] = lo[a]; g0[3 + a] = hi[a]; }
  t->lev[0].start[0] = 0;
  t->lev[0].start[1] = n;

  kv_t* kv = (kv_t*)xmalloc((size_t)(n > 0 ? n : 1) * sizeof(kv_t));
  int32_t* tmp = (int32_t*)xmalloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  int32_t* scratch = (int32_t*)xmalloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  for (int l = 0; l < L; ++l) {
    orc_level* P = &t->lev[l];
    orc_level* C = &t->lev[l + 1];
    /* boxes are independent: each works on its own range of perm and of the
     * buffers kv, tmp, scratch */
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < P->nbox; ++b) {
      const int64_t base = P->start[b];
      kv_t* kvb = kv + base;
      int32_t* tmpb = tmp + base;
      int32_t* scrb = scratch + base;
      /* three successive bisections; sub-cells indexed by the bits so far */
      double clo[8][3], chi[8][3];
      int64_t cs[8], ce[8];
      for (int a = 0; a < 3; ++a) { clo[0][a] = P->geom[b * 10 + a]; chi[0][a] = P->geom[b * 10 + 3 + a]; }
      cs[0] = P->start[b];
      ce[0] = P->start[b + 1];
      int cnt = 1;
      for (int k = 0; k < 3; ++k) {
        double nlo[8][3], nhi[8][3];
        int64_t ns[8], ne[8];
        for (int c = 0; c < cnt; ++c) {
          int axis;
          double plane;
          const int64_t m = bisect(t, t->perm, cs[c], ce[c], clo[c], chi[c], &axis, &plane, kvb, tmpb, scrb);
          for (int h = 0; h < 2; ++h) {
            const int o = 2 * c + h;
            memcpy(nlo[o], clo[c], sizeof(nlo[o]));
            memcpy(nhi[o], chi[c], sizeof(nhi[o]));
          }
          nhi[2 * c][axis] = plane;
          nlo[2 * c + 1][axis] = plane;
          ns[2 * c] = cs[c];
          ne[2 * c] = cs[c] + m;
          ns[2 * c + 1] = cs[c] + m;
          ne[2 * c + 1] = ce[c];
        }
        cnt *= 2;
        memcpy(clo, nlo, sizeof(clo));
        memcpy(chi, nhi, sizeof(chi));
        memcpy(cs, ns, sizeof(cs));
        memcpy(ce, ne, sizeof(ce));
      }
      for (int c = 0; c < 8; ++c) {
        const int64_t j = 8 * b + c;
        for (int a = 0; a < 3; ++a) { C->geom[j * 10 + a] = clo[c][a]; C->geom[j * 10 + 3 + a] = chi[c][a]; }
        C->start[j] = cs[c];
      }
    }
    C->start[C->nbox] = n;
  }
  free(kv);
  free(tmp);
  free(scratch);
  /* centres and radii, Section 2.1.1 */
  for (int l = 0; l <= L; ++l) {
    orc_level* V = &t->lev[l];
    for (int64_t b = 0; b < V->nbox; ++b) {
      double* g = V->geom + b * 10;
      double d[3];
      for (int a = 0; a < 3; ++a) {
        g[6 + a] = 0.5 * (g[a] + g[3 + a]);
        d[a] = g[3 + a] - g[a];
      }
      g[9] = 0.5 * sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
    }
  }
}

/* theta-criterion, eq. (2.2): 1 = weak, 0 = strong */
static int is_weak(const double* gi, const double* gj, double theta) {
  const double dx = gi[6] - gj[6], dy = gi[7] - gj[7], dz = gi[8] - gj[8];
  const double d = sqrt((dx * dx + dy * dy) + dz * dz);
  if (!(d > 0.0)) return 0;
  const double R = gi[9] > gj[9] ? gi[9] : gj[9];
  const double r = gi[9] > gj[9] ? gj[9] : gi[9];
  return R + theta * r <= theta * d;
}

/* Connectivity per level (Section 2.1.1 inheritance; Algorithm 2): the
 * candidates of box i are the children of every box strongly connected to
 * the parent of i, in ascending order.  need[l][i] = 0 leaves the rows of box
 * i empty (targeted mode: only the ancestors of chosen leaves get lists; a
 * needed box always has a needed parent); need == NULL builds every row. */
static void build_lists_masked(orc_tree* t, char* const* need) {
  orc_level* V0 = &t->lev[0];
  V0->s_off = (int64_t*)xmalloc(2 * sizeof(int64_t));
  V0->s_idx = (int32_t*)xmalloc(sizeof(int32_t));
  V0->w_off = (int64_t*)xcalloc(2, sizeof(int64_t));
  V0->w_idx = (int32_t*)xmalloc(sizeof(int32_t));
  V0->s_off[0] = 0;
  V0->s_off[1] = 1;
  V0->s_idx[0] = 0;
  for (int l = 1; l <= t->L; ++l) {
    orc_level* P = &t->lev[l - 1];
    orc_level* V = &t->lev[l];
    const char* nd = need ? need[l] : NULL;
    int64_t* cs = (int64_t*)xcalloc((size_t)V->nbox + 1, sizeof(int64_t));
    int64_t* cw = (int64_t*)xcalloc((size_t)V->nbox + 1, sizeof(int64_t));
    /* count, then fill: the same candidate loop twice */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < V->nbox; ++i) {
      if (nd && !nd[i]) continue;
      const int64_t par = i / 8;
      int64_t ns = 0, nw = 0;
      for (int64_t e = P->s_off[par]; e < P->s_off[par + 1]; ++e) {
        const int64_t J = P->s_idx[e];
        for (int c = 0; c < 8; ++c) {
          const int64_t j = 8 * J + c;
          if (j != i && is_weak(V->geom + i * 10, V->geom + j * 10, t->theta)) ++nw;
          else ++ns;
        }
      }
      cs[i] = ns;
      cw[i] = nw;
    }
    V->s_off = (int64_t*)xmalloc((size_t)(V->nbox + 1) * sizeof(int64_t));
    V->w_off = (int64_t*)xmalloc((size_t)(V->nbox + 1) * sizeof(int64_t));
    int64_t ts = 0, tw = 0;
    for (int64_t i = 0; i < V->nbox; ++i) {
      V->s_off[i] = ts;
      V->w_off[i] = tw;
      ts += cs[i];
      tw += cw[i];
    }
    V->s_off[V->nbox] = ts;
    V->w_off[V->nbox] = tw;
    free(cs);
    free(cw);
    V->s_idx = (int32_t*)xmalloc((size_t)(ts > 0 ? ts : 1) * sizeof(int32_t));
    V->w_idx = (int32_t*)xmalloc((size_t)(tw > 0 ? tw : 1) * sizeof(int32_t));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < V->nbox; ++i) {
      if (nd && !nd[i]) continue;
      const int64_t par = i / 8;
      int64_t ns = V->s_off[i], nw = V->w_off[i];
      for (int64_t e = P->s_off[par]; e < P->s_off[par + 1]; ++e) {
        const int64_t J = P->s_idx[e];
        for (int c = 0; c < 8; ++c) {
          const int64_t j = 8 * J + c;
          if (j != i && is_weak(V->geom + i * 10, V->geom + j * 10, t->theta)) V->w_idx[nw++] = (int32_t)j;
          else V->s_idx[ns++] = (int32_t)j;
        }
      }
    }
  }
}

static void build_lists(orc_tree* t) { build_lists_masked(t, NULL); }

/* ------------------------------------------------------------------------ */
/* Public tree API                                                          */
/* ------------------------------------------------------------------------ */

/* Tree over n sources; the m separate targets (m may be 0) only widen the
 * root cell so that every target lies in some leaf cell.  eta as in bisect. */
void* orc_create_ex(int64_t n, const double* x, const double* y, const double* z, int64_t m, const double* tx,
                    const double* ty, const double* tz, int L, double theta, double eta) {
  orc_init();
  orc_tree* t = (orc_tree*)xcalloc(1, sizeof(orc_tree));
  t->n = n;
  t->L = L;
  t->theta = theta;
  t->eta = eta;
  t->x = x;
  t->y = y;
  t->z = z;
  t->m = m;
  t->tx = tx;
  t->ty = ty;
  t->tz = tz;
  build_tree(t);
  build_lists(t);
  return t;
}

/* Targeted mode, for trees whose full lists do not fit in host memory: the
 * tree is built in full, but the strong and weak lists only for the
 * ancestors of the nleaves listed leaves (every other row is empty).  The
 * tree can then be evaluated at (a subset of) those leaves only: the
 * upward pass is complete, M2L and L2L run along the chains of the listed
 * leaves, P2P over their strong lists -- the same arithmetic as a full tree
 * evaluated at those leaves. */
void* orc_create_targeted(int64_t n, const double* x, const double* y, const double* z, int L, double theta,
                          int64_t nleaves, const int64_t* leaves) {
  orc_init();
  orc_tree* t = (orc_tree*)xcalloc(1, sizeof(orc_tree));
  t->n = n;
  t->L = L;
  t->theta = theta;
  t->eta = 1.0;
  t->x = x;
  t->y = y;
  t->z = z;
  build_tree(t);
  char** need = (char**)xcalloc((size_t)L + 1, sizeof(char*));
  for (int l = 0; l <= L; ++l) need[l] = (char*)xcalloc((size_t)t->lev[l].nbox, 1);
  for (int64_t s = 0; s < nleaves; ++s) {
    int64_t b = leaves[s];
    for (int l = L; l >= 0; --l, b /= 8) need[l][b] = 1;
  }
  build_lists_masked(t, need);
  t->listed = need[L];
  for (int l = 0; l < L; ++l) free(need[l]);
  free(need);
  return t;
}

/* Rebuilds the lists of a tree for another theta (the tree does not depend
 * on theta); a targeted tree keeps its chosen leaves. */
void orc_set_theta(void* h, double theta) {
  orc_tree* t = (orc_tree*)h;
  for (int l = 0; l <= t->L; ++l) {
    orc_level* V = &t->lev[l];
    free(V->s_off); free(V->s_idx); free(V->w_off); free(V->w_idx);
    V->s_off = V->w_off = NULL;
    V->s_idx = V->w_idx = NULL;
  }
  t->theta = theta;
  if (!t->listed) {
    build_lists(t);
    return;
  }
  const int L = t->L;
  char** need = (char**)xcalloc((size_t)L + 1, sizeof(char*));
  for (int l = 0; l < L; ++l) need[l] = (char*)xcalloc((size_t)t->lev[l].nbox, 1);
  need[L] = t->listed;
  for (int64_t b = 0; b < t->lev[L].nbox; ++b) {
    if (!t->listed[b]) continue;
    int64_t a = b / 8;
    for (int l = L - 1; l >= 0; --l, a /= 8) need[l][a] = 1;
  }
  build_lists_masked(t, need);
  for (int l = 0; l < L; ++l) free(need[l]);
  free(need);
}

void* orc_create(int64_t n, const double* x, const double* y, const double* z, int L, double theta) {
  return orc_create_ex(n, x, y, z, 0, NULL, NULL, NULL, L, theta, 1.0);
}

void orc_destroy(void* h) {
  orc_tree* t = (orc_tree*)h;
  if (!t) return;
  for (int l = 0; l <= t->L; ++l) {
    orc_level* V = &t->lev[l];
    free(V->geom); free(V->start); free(V->s_off); free(V->s_idx); free(V->w_off); free(V->w_idx);
  }
  free(t->lev);
  free(t->perm);
  free(t->listed);
  free(t);
}

void orc_get_perm(void* h, int32_t* perm) {
  const orc_tree* t = (const orc_tree*)h;
  memcpy(perm, t->perm, (size_t)t->n * sizeof(int32_t));
}

void orc_get_geom(void* h, int l, double* geom) {
  const orc_tree* t = (const orc_tree*)h;
  memcpy(geom, t->lev[l].geom, (size_t)t->lev[l].nbox * 10 * sizeof(double));
}

void orc_get_start(void* h, int l, int64_t* start) {
  const orc_tree* t = (const orc_tree*)h;
  memcpy(start, t->lev[l].start, (size_t)(t->lev[l].nbox + 1) * sizeof(int64_t));
}

int64_t orc_list_nnz(void* h, int l, int kind) {
  const orc_tree* t = (const orc_tree*)h;
  const orc_level* V = &t->lev[l];
  return kind == 0 ? V->s_off[V->nbox] : V->w_off[V->nbox];
}

void orc_get_list(void* h, int l, int kind, int64_t* off, int32_t* idx) {
  const orc_tree* t = (const orc_tree*)h;
  const orc_level* V = &t->lev[l];
  const int64_t* o = kind == 0 ? V->s_off : V->w_off;
  const int32_t* ix = kind == 0 ? V->s_idx : V->w_idx;
  memcpy(off, o, (size_t)(V->nbox + 1) * sizeof(int64_t));
  memcpy(idx, ix, (size_t)o[V->nbox] * sizeof(int32_t));
}

/* ------------------------------------------------------------------------ */
/* Evaluation (Algorithm 1: P2M, M2M, then Algorithm 3: M2L, L2L, then       */
/* Algorithm 4: L2P, P2P), for the points of the listed leaves.              */
/* ------------------------------------------------------------------------ */

/* Upward and downward passes (Algorithm 1: P2M, M2M; Algorithm 3: M2L,
 * L2L) on point data in tree order.  Local expansions are formed for the
 * leaves flagged in need_leaf and their ancestors; returns them per level
 * (Lx[l], l = 1..L; free with free_levels). */
static void free_levels(cplx** X, int L) {
  if (!X) return;
  for (int l = 0; l <= L; ++l) free(X[l]);
  free(X);
}

static cplx** far_pass(const orc_tree* t, const double* px, const double* py, const double* pz, const double* pq,
                       int p, const char* need_leaf) {
  const int L = t->L;
  const int nt = NTERMS(p);
  const orc_level* leaf = &t->lev[L];
  char** need = (char**)xcalloc((size_t)L + 1, sizeof(char*));
  for (int l = 0; l <= L; ++l) need[l] = (char*)xcalloc((size_t)t->lev[l].nbox, 1);
  for (int64_t s = 0; s < leaf->nbox; ++s) {
    if (!need_leaf[s]) continue;
    int64_t b = s;
    for (int l = L; l >= 0; --l, b /= 8) need[l][b] = 1;
  }

  cplx** Mx = (cplx**)xcalloc((size_t)L + 1, sizeof(cplx*));
  cplx** Lx = (cplx**)xcalloc((size_t)L + 1, sizeof(cplx*));
  orc_init();
  if (g_m2l_rot) rot_tables(p);
  {
    for (int l = 1; l <= L; ++l) {
      Mx[l] = (cplx*)xcalloc((size_t)t->lev[l].nbox * nt, sizeof(cplx));
      Lx[l] = (cplx*)xcalloc((size_t)t->lev[l].nbox * nt, sizeof(cplx));
    }
    /* P2M on level L */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < leaf->nbox; ++b) {
      const double* g = leaf->geom + b * 10;
      const int64_t s = leaf->start[b], e = leaf->start[b + 1];
      orc_p2m(p, g[6], g[7], g[8], e - s, px + s, py + s, pz + s, pq + s, Mx[L] + b * nt);
    }
    /* M2M, l = L .. 2: parents on level l-1 from their 8 children */
    for (int l = L; l >= 2; --l) {
      const orc_level* C = &t->lev[l];
      const orc_level* P = &t->lev[l - 1];
#pragma omp parallel for schedule(dynamic, 64)
      for (int64_t b = 0; b < P->nbox; ++b) {
        cplx tmpM[NTERMS(ORC_PMAX)];
        const double* gp = P->geom + b * 10;
        cplx* dst = Mx[l - 1] + b * nt;
        for (int c = 0; c < 8; ++c) {
          const int64_t j = 8 * b + c;
          const double* gc = C->geom + j * 10;
          orc_m2m(p, Mx[l] + j * nt, gc[6] - gp[6], gc[7] - gp[7], gc[8] - gp[8], tmpM);
          for (int k = 0; k < nt; ++k) dst[k] += tmpM[k];
        }
      }
    }
    /* downward pass over the needed boxes: M2L at every level, then L2L */
    for (int l = 1; l <= L; ++l) {
      const orc_level* V = &t->lev[l];
#pragma omp parallel for schedule(dynamic, 1)
      for (int64_t i = 0; i < V->nbox; ++i) {
        if (!need[l][i]) continue;
        cplx* dst = Lx[l] + i * nt;
        if (l >= 2) {
          const orc_level* P = &t->lev[l - 1];
          const int64_t par = i / 8;
          const double* gp = P->geom + par * 10;
          const double* gi = V->geom + i * 10;
          orc_l2l_add(p, Lx[l - 1] + par * nt, gp[6] - gi[6], gp[7] - gi[7], gp[8] - gi[8], dst);
        }
        const double* gi = V->geom + i * 10;
        for (int64_t e = V->w_off[i]; e < V->w_off[i + 1]; ++e) {
          const int64_t j = V->w_idx[e];
          const double* gj = V->geom + j * 10;
          m2l_add(p, Mx[l] + j * nt, gj[6] - gi[6], gj[7] - gi[7], gj[8] - gi[8], dst);
        }
      }
    }
  }

  for (int l = 0; l <= L; ++l) free(need[l]);
  free(need);
  free_levels(Mx, L);
  return Lx;
}

/* parts: bit 0 = near field (P2P), bit 1 = far field (L2P).
 * leaves == NULL means every leaf.  Outputs are written at the original
 * point index of every point of the listed leaves; other entries untouched.
 * Returns 0 on success. */
int orc_evaluate(void* h, const double* q, int p, int parts, int64_t nleaves, const int64_t* leaves, double* phi,
                 double* ex, double* ey, double* ez) {
  orc_tree* t = (orc_tree*)h;
  if (p < 0 || p > ORC_PMAX) return -1;
  const int L = t->L;
  const int nt = NTERMS(p);
  const orc_level* leaf = &t->lev[L];
  if (leaves == NULL) nleaves = leaf->nbox;
  if (t->listed) /* targeted mode: only leaves whose chains have lists */
    for (int64_t s = 0; s < nleaves; ++s)
      if (!leaves || !t->listed[leaves[s]]) return -3;

  /* point data in tree order */
  const int64_t n = t->n;
  double* px = (double*)xmalloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double* py = (double*)xmalloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double* pz = (double*)xmalloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double* pq = (double*)xmalloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  for (int64_t i = 0; i < n; ++i) {
    const int32_t o = t->perm[i];
    px[i] = t->x[o]; py[i] = t->y[o]; pz[i] = t->z[o]; pq[i] = q[o];
  }

  /* which boxes need a local expansion: ancestors of the listed leaves */
  char* need_leaf = (char*)xcalloc((size_t)leaf->nbox, 1);
  for (int64_t s = 0; s < nleaves; ++s) need_leaf[leaves ? leaves[s] : s] = 1;
  cplx** Lx = ((parts & 2) && L >= 1) ? far_pass(t, px, py, pz, pq, p, need_leaf) : NULL;
  free(need_leaf);

#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t s = 0; s < nleaves; ++s) {
    const int64_t b = leaves ? leaves[s] : s;
    const double* g = leaf->geom + b * 10;
    const int64_t s0 = leaf->start[b], s1 = leaf->start[b + 1];
    for (int64_t ti = s0; ti < s1; ++ti) {
      double f = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
      if ((parts & 2) && L >= 1) orc_l2p_add(p, Lx[L] + b * nt, g[6], g[7], g[8], px[ti], py[ti], pz[ti], &f, &fx, &fy, &fz);
      if (parts & 1) {
        /* P2P over the strongly connected leaves, Algorithm 4 */
        for (int64_t e = leaf->s_off[b]; e < leaf->s_off[b + 1]; ++e) {
          const int64_t j = leaf->s_idx[e];
          for (int64_t si = leaf->start[j]; si < leaf->start[j + 1]; ++si) {
            const double dx = px[ti] - px[si], dy = py[ti] - py[si], dz = pz[ti] - pz[si];
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            const double r = sqrt(r2);
            const double inv = 1.0 / r;
            const double inv3 = inv / r2;
            f += pq[si] * inv;
            fx += pq[si] * dx * inv3;
            fy += pq[si] * dy * inv3;
            fz += pq[si] * dz * inv3;
          }
        }
      }
      const int32_t o = t->perm[ti];
      phi[o] = f;
      ex[o] = fx;
      ey[o] = fy;
      ez[o] = fz;
    }
  }

  free_levels(Lx, L);
  free(px); free(py); free(pz); free(pq);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Evaluation at separate targets (the convergence test of Section 3.1      */
/* evaluates at points that are not sources).                               */
/* ------------------------------------------------------------------------ */

/* The leaf whose cell holds target (x, y, z): from the root, at every level
 * the first of the eight children (in child order) whose closed cell
 * contains the point.  The children's cells tile the parent's cell, so one
 * always does for a point inside the root cell; -1 outside it. */
int64_t orc_locate(void* h, double x, double y, double z) {
  const orc_tree* t = (const orc_tree*)h;
  const double v[3] = {x + 0.0, y + 0.0, z + 0.0};
  const double* g0 = t->lev[0].geom;
  for (int a = 0; a < 3; ++a)
    if (!(v[a] >= g0[a] && v[a] <= g0[3 + a])) return -1;
  int64_t b = 0;
  for (int l = 1; l <= t->L; ++l) {
    const double* g = t->lev[l].geom;
    int64_t found = -1;
    for (int c = 0; c < 8 && found < 0; ++c) {
      const int64_t j = 8 * b + c;
      int in = 1;
      for (int a = 0; a < 3; ++a)
        if (!(v[a] >= g[j * 10 + a] && v[a] <= g[j * 10 + 3 + a])) in = 0;
      if (in) found = j;
    }
    if (found < 0) return -1;
    b = found;
  }
  return b;
}

/* phi and E = -grad phi at the tree's m separate targets (input order):
 * far field from the local expansion of the target's leaf (L2P), near field
 * from the sources of the leaves strongly connected to it (P2P; a source at
 * the target's own position contributes nothing).  parts as in
 * orc_evaluate.  Returns 0, or -1 for a bad order, -2 for a target outside
 * the root cell. */
int orc_evaluate_targets(void* h, const double* q, int p, int parts, double* phi, double* ex, double* ey,
                         double* ez) {
  orc_tree* t = (orc_tree*)h;
  if (p < 0 || p > ORC_PMAX) return -1;
  if (t->listed) return -3;
  const int L = t->L;
  const int nt = NTERMS(p);
  const orc_level* leaf = &t->lev[L];
  const int64_t n = t->n, m = t->m;
  int64_t* tleaf = (int64_t*)xmalloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
  for (int64_t k = 0; k < m; ++k) {
    tleaf[k] = orc_locate(h, t->tx[k], t->ty[k], t->tz[k]);
    if (tleaf[k] < 0) { free(tleaf); return -2; }
  }
  double* px = (double*)xmalloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double* py = (double*)xmalloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double* pz = (double*)xmalloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  double* pq = (double*)xmalloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  for (int64_t i = 0; i < n; ++i) {
    const int32_t o = t->perm[i];
    px[i] = t->x[o]; py[i] = t->y[o]; pz[i] = t->z[o]; pq[i] = q[o];
  }
  char* need_leaf = (char*)xcalloc((size_t)leaf->nbox, 1);
  for (int64_t k = 0; k < m; ++k) need_leaf[tleaf[k]] = 1;
  cplx** Lx = ((parts & 2) && L >= 1) ? far_pass(t, px, py, pz, pq, p, need_leaf) : NULL;
  free(need_leaf);

#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < m; ++k) {
    const int64_t b = tleaf[k];
    const double x = t->tx[k] + 0.0, y = t->ty[k] + 0.0, z = t->tz[k] + 0.0;
    double f = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    if (Lx) {
      const double* g = leaf->geom + b * 10;
      orc_l2p_add(p, Lx[L] + b * nt, g[6], g[7], g[8], x, y, z, &f, &fx, &fy, &fz);
    }
    if (parts & 1) {
      for (int64_t e = leaf->s_off[b]; e < leaf->s_off[b + 1]; ++e) {
        const int64_t j = leaf->s_idx[e];
        for (int64_t si = leaf->start[j]; si < leaf->start[j + 1]; ++si) {
          const double dx = x - px[si], dy = y - py[si], dz = z - pz[si];
          const double r2 = dx * dx + dy * dy + dz * dz;
          if (r2 == 0.0) continue;
          const double r = sqrt(r2);
          const double inv = 1.0 / r;
          const double inv3 = inv / r2;
          f += pq[si] * inv;
          fx += pq[si] * dx * inv3;
          fy += pq[si] * dy * inv3;
          fz += pq[si] * dz * inv3;
        }
      }
    }
    phi[k] = f;
    ex[k] = fx;
    ey[k] = fy;
    ez[k] = fz;
  }
  free_levels(Lx, L);
  free(tleaf);
  free(px); free(py); free(pz); free(pq);
  return 0;
}
