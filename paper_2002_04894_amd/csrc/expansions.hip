// Multipole / local expansions on the GPU (Section 2.1: spherical-harmonic
// expansions of order p about box centres; Algorithm 1 P2M and M2M,
// Algorithm 3 M2L and L2L, Algorithm 4 L2P).
//
// Basis.  Real regular solid harmonics R_b(u) = |u|^n Y_b(u/|u|), where Y_b
// are the Schmidt semi-normalised real harmonics of degree n (b runs over
// c_0, c_1, s_1, ..., c_n, s_n; storage index n^2, n^2 + 2m - 1, n^2 + 2m).
// Within one degree they are orthogonal with equal norms, so a rotation acts
// on the 2n+1 coefficients of degree n by an orthogonal matrix, and
//   1/|x - y| = sum_b R_b(y) I_b(x),  I_b(x) = R_b(x) / |x|^(2n+1),  |y| < |x|.
// Hence the multipole M_b = sum_i q_i R_b(x_i - c) and the local expansion
// Phi(x) = sum_b L_b R_b(x - c).  With G_n^m = sqrt((n-m)!/(n+m)!) r^n P_n^m
// e^{i m phi} (no Condon-Shortley phase), R_{n,m,c} + i R_{n,m,s} =
// sqrt(2 - delta_m0) G_n^m, and G obeys
//   G_m^m     = sqrt((2m-1)/(2m)) (x + i y) G_{m-1}^{m-1},
//   G_{m+1}^m = sqrt(2m+1) z G_m^m,
//   G_n^m     = [(2n-1) z G_{n-1}^m - sqrt((n+m-1)(n-m-1)) r^2 G_{n-2}^m] / sqrt((n+m)(n-m)).
//
// Translations use the rotational form the paper adopts for M2L (Section
// 2.1.3): rotate the expansion so that the translation vector is the +z axis,
// translate along z, rotate back; O(p^3) per translation.  A rotation
// Ry(g) equals J Rz(g) J^T with J the fixed matrix of a quarter turn about x
// (tabulated per degree by exact quadrature), and z-rotations mix the
// (c_m, s_m) pairs, so no per-pair rotation matrix is generated.  Along z the
// translations are, with rho the distance:
//   M2L:  L'_{j,m} = sum_n (-1)^(n+m) (n+j)! / (rho^(n+j+1) sqrt((n+m)!(n-m)!(j+m)!(j-m)!)) M'_{n,m}
//   M2M:  M'_{n,m} = sum_{j<=n} rho^(n-j)/(n-j)! sqrt((n+m)!(n-m)!/((j+m)!(j-m)!)) M_{j,m}
//   L2L:  L'_{j,m} = sum_{n>=j} (same coefficient) L_{n,m}
// (identical for the c and s parts of each m).
#include <math.h>

#include <map>
#include <mutex>

#include "fmm_internal.h"
#include "tile_layout.h"
#include "lane_ops.h"

namespace fmm {

// ----------------------------------------------------------------------------
// host: fixed tables
// ----------------------------------------------------------------------------
namespace {

// real regular solid harmonics at v, degrees <= p (host, for the quadrature)
void host_R(int p, const double v[3], double* out) {
  const double x = v[0], y = v[1], z = v[2];
  const double r2 = x * x + y * y + z * z;
  std::vector<double> gr((p + 1) * (p + 1)), gi((p + 1) * (p + 1));
  auto at = [&](int n, int m) { return n * (p + 1) + m; };
  gr[at(0, 0)] = 1.0;
  gi[at(0, 0)] = 0.0;
  for (int m = 0; m <= p; ++m) {
    if (m > 0) {
      const double a = sqrt((2.0 * m - 1.0) / (2.0 * m));
      const double pr = gr[at(m - 1, m - 1)], pi = gi[at(m - 1, m - 1)];
      gr[at(m, m)] = a * (x * pr - y * pi);
      gi[at(m, m)] = a * (x * pi + y * pr);
    }
    if (m + 1 <= p) {
      const double b = sqrt(2.0 * m + 1.0);
      gr[at(m + 1, m)] = b * z * gr[at(m, m)];
      gi[at(m + 1, m)] = b * z * gi[at(m, m)];
    }
    for (int n = m + 2; n <= p; ++n) {
      const double d = sqrt((double)(n + m) * (n - m));
      const double c1 = (2.0 * n - 1.0) / d;
      const double c2 = sqrt((double)(n + m - 1) * (n - m - 1)) / d;
      gr[at(n, m)] = c1 * z * gr[at(n - 1, m)] - c2 * r2 * gr[at(n - 2, m)];
      gi[at(n, m)] = c1 * z * gi[at(n - 1, m)] - c2 * r2 * gi[at(n - 2, m)];
    }
  }
  const double s2 = sqrt(2.0);
  for (int n = 0; n <= p; ++n) {
    out[n * n] = gr[at(n, 0)];
    for (int m = 1; m <= n; ++m) {
      out[n * n + 2 * m - 1] = s2 * gr[at(n, m)];
      out[n * n + 2 * m] = s2 * gi[at(n, m)];
    }
  }
}

// Gauss-Legendre nodes / weights on [-1, 1] by Newton iteration
void gauss_legendre(int N, std::vector<double>& xs, std::vector<double>& ws) {
  xs.resize(N);
  ws.resize(N);
  for (int i = 0; i < N; ++i) {
    double x = cos(M_PI * (i + 0.75) / (N + 0.5));
    double dp = 0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= N; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      // p1 = P_N(x), p0 = P_{N-1}(x)
      dp = N * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    xs[i] = x;
    ws[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
}

long double f_all(int k) {
  long double f = 1.0L;
  for (int i = 2; i <= k; ++i) f *= i;
  return f;
}

// x-parity class of local index i within a degree: c_m (i = 2m-1) and s_m
// (i = 2m) are even under x -> -x iff m + [s] is even.
int parity_class(int i) {
  if (i == 0) return 0;
  const int m = (i + 1) >> 1, s = (i & 1) ? 0 : 1;
  return (m + s) & 1;
}

struct HostTables {
  std::vector<double> J, A, B, rc, mtab;
  std::vector<float> mtab32;
  std::vector<int> joff, pos, ipos;
  std::vector<int8_t> sdeg;
  int stride = 0;
  bool tiled = false;
};

// Rotation matrices by exact quadrature: J^n_{bb'} with
// R_b(K v) = sum_b' J^n_{bb'} R_b'(v) for a fixed rotation K (kv = K v).
std::vector<double> quarter_turn(int p, const std::vector<int>& joff, void (*K)(const double*, double*)) {
  const int nth = p + 2, nph = 2 * p + 2;
  std::vector<double> gx, gw;
  gauss_legendre(nth, gx, gw);
  const int nt = nterms(p);
  std::vector<double> Rv(nt), RK(nt);
  std::vector<long double> acc(joff[p + 1], 0.0L);
  for (int a = 0; a < nth; ++a) {
    const double ct = gx[a];
    const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    for (int k = 0; k < nph; ++k) {
      const double ph = 2.0 * M_PI * k / nph;
      const double v[3] = {st * cos(ph), st * sin(ph), ct};
      double kv[3];
      K(v, kv);
      host_R(p, v, Rv.data());
      host_R(p, kv, RK.data());
      const long double w = (long double)gw[a] * (2.0L * M_PI / nph);
      for (int n = 0; n <= p; ++n) {
        const int s = 2 * n + 1;
        for (int i = 0; i < s; ++i)
          for (int j = 0; j < s; ++j)
            acc[joff[n] + i * s + j] += w * (long double)RK[n * n + i] * (long double)Rv[n * n + j];
      }
    }
  }
  std::vector<double> J(joff[p + 1]);
  for (int n = 0; n <= p; ++n) {
    const int s = 2 * n + 1;
    for (int i = 0; i < s * s; ++i) J[joff[n] + i] = (double)(acc[joff[n] + i] * (2.0L * n + 1.0L) / (4.0L * M_PI));
  }
  return J;
}

void quarter_x(const double* v, double* kv) {  // quarter turn about x: (x, y, z) -> (x, z, -y)
  kv[0] = v[0];
  kv[1] = v[2];
  kv[2] = -v[1];
}
void quarter_y(const double* v, double* kv) {  // quarter turn about y: (x, y, z) -> (z, y, -x)
  kv[0] = v[2];
  kv[1] = v[1];
  kv[2] = -v[0];
}

HostTables make_host_tables(int p) {
  HostTables h;
  // J: R_b(K v) = sum_b' J_bb' R_b'(v), K = quarter turn about x: (x,y,z) -> (x, z, -y);
  // entries between the two x-parity classes vanish and are set to 0
  h.joff.resize(p + 2);
  h.joff[0] = 0;
  for (int n = 0; n <= p; ++n) h.joff[n + 1] = h.joff[n] + (2 * n + 1) * (2 * n + 1);
  h.J = quarter_turn(p, h.joff, quarter_x);
  for (int n = 0; n <= p; ++n) {
    const int s = 2 * n + 1;
    for (int i = 0; i < s; ++i)
      for (int j = 0; j < s; ++j)
        if (parity_class(i) != parity_class(j)) h.J[h.joff[n] + i * s + j] = 0.0;
  }
  // factorials
  std::vector<long double> f(2 * p + 2);
  f[0] = 1.0L;
  for (int i = 1; i < (int)f.size(); ++i) f[i] = f[i - 1] * i;
  const int P1 = p + 1;
  h.A.assign((size_t)P1 * P1 * P1, 0.0);
  h.B.assign((size_t)P1 * P1 * P1, 0.0);
  for (int m = 0; m <= p; ++m)
    for (int j = m; j <= p; ++j)
      for (int n = m; n <= p; ++n) {
        const long double sgn = ((n + m) & 1) ? -1.0L : 1.0L;
        h.A[((size_t)m * P1 + j) * P1 + n] =
            (double)(sgn * f[n + j] / sqrtl(f[n + m] * f[n - m] * f[j + m] * f[j - m]));
        if (j <= n)
          h.B[((size_t)m * P1 + n) * P1 + j] =
              (double)(sqrtl(f[n + m] * f[n - m] / (f[j + m] * f[j - m])) / f[n - j]);
      }
  // recurrence constants: am[m], bm[m], c1[n][m], c2[n][m]
  h.rc.assign(2 * P1 + 2 * P1 * P1, 0.0);
  for (int m = 1; m <= p; ++m) h.rc[m] = sqrt((2.0 * m - 1.0) / (2.0 * m));
  for (int m = 0; m <= p; ++m) h.rc[P1 + m] = sqrt(2.0 * m + 1.0);
  for (int n = 0; n <= p; ++n)
    for (int m = 0; m + 2 <= n; ++m) {
      const double d = sqrt((double)(n + m) * (n - m));
      h.rc[2 * P1 + n * P1 + m] = (2.0 * n - 1.0) / d;
      h.rc[2 * P1 + P1 * P1 + n * P1 + m] = sqrt((double)(n + m - 1) * (n - m - 1)) / d;
    }
  // storage layout
  const int nt = nterms(p);
  h.tiled = p <= tl::kMaxP;
  h.stride = h.tiled ? tl::stride(p) : nt;
  h.pos.assign(nt, -1);
  h.ipos.assign(h.stride, -1);
  if (!h.tiled) {
    for (int k = 0; k < nt; ++k) h.pos[k] = h.ipos[k] = k;
    return h;
  }
  h.sdeg.assign(h.stride, -1);
  for (int t = 0; t < tl::ntiles(p); ++t)
    for (int sl = 0; sl < 16; ++sl) {
      const tl::Slot d = tl::decode(p, t, sl);
      if (!d.valid) continue;
      const int k = d.n * d.n + (d.m == 0 ? 0 : 2 * d.m - 1 + d.sine);
      h.pos[k] = tl::spos(t, sl);
      h.ipos[tl::spos(t, sl)] = k;
      h.sdeg[tl::spos(t, sl)] = (int8_t)d.n;
    }
  // MFMA tables, stored as operand fragments (entry [step][lane] is what lane
  // `lane` feeds to the k-step `step` of a 16x16x4 chain: row lane % 16,
  // column 4 step + lane / 16):
  //  - per tile, the matrix of the quarter turn about y restricted to the
  //    tile (its cosine and sine blocks; cross entries vanish);
  //  - per order m, the z-axis translation without its distance powers,
  //    H_m[a][b] = (-1)^(m+b) (2m+a+b)! u_{m+a,m} u_{m+b,m},
  //    u_{n,m} = 1/sqrt((n+m)!(n-m)!), a, b < p + 1 - m.
  const std::vector<double> Jy = quarter_turn(p, h.joff, quarter_y);
  const int T = tl::ntiles(p);
  std::vector<double> W((size_t)T * 256, 0.0);
  for (int t = 0; t < T; ++t)
    for (int r = 0; r < 16; ++r)
      for (int c = 0; c < 16; ++c) {
        const tl::Slot a = tl::decode(p, t, r), b = tl::decode(p, t, c);
        if (!a.valid || !b.valid || a.n != b.n || a.sine != b.sine) continue;
        const int n = a.n, sdim = 2 * n + 1;
        const int ia = a.m == 0 ? 0 : 2 * a.m - 1 + a.sine;
        const int ib = b.m == 0 ? 0 : 2 * b.m - 1 + b.sine;
        W[(size_t)t * 256 + r * 16 + c] = Jy[h.joff[n] + ia * sdim + ib];
      }
  const int H = tl::hoff(p, p + 1);
  h.mtab.assign((size_t)T * 4 * 64 + (size_t)H * 64, 0.0);
  for (int t = 0; t < T; ++t)
    for (int st = 0; st < 4; ++st)
      for (int lane = 0; lane < 64; ++lane)
        h.mtab[((size_t)t * 4 + st) * 64 + lane] = W[(size_t)t * 256 + (lane % 16) * 16 + 4 * st + lane / 16];
  double* hf = h.mtab.data() + (size_t)T * 4 * 64;
  for (int m = 0; m <= p; ++m) {
    const int K = p + 1 - m;
    for (int st = 0; st < tl::hsteps(p, m); ++st)
      for (int lane = 0; lane < 64; ++lane) {
        const int a = lane % 16, b = 4 * st + lane / 16;
        if (a >= K || b >= K) continue;
        const long double u = 1.0L / sqrtl(f_all(2 * m + a) * f_all(a) * f_all(2 * m + b) * f_all(b));
        const long double sg = ((m + b) & 1) ? -1.0L : 1.0L;
        hf[((size_t)tl::hoff(p, m) + st) * 64 + lane] = (double)(sg * f_all(2 * m + a + b) * u);
      }
  }
  // binary32 fragments for v_mfma_f32_16x16x4f32, whose result rows are
  // 4 (lane / 16) + i (against 4 i + lane / 16 for the binary64 one): the
  // same fragments with the operand row r read from row 4 (r % 4) + r / 4,
  // so that the binary32 chains see the same slot order as the binary64 ones
  h.mtab32.resize(h.mtab.size());
  const size_t nfrag = h.mtab.size() / 64;
  for (size_t f = 0; f < nfrag; ++f)
    for (int lane = 0; lane < 64; ++lane) {
      const int r = lane % 16, src_lane = (4 * (r % 4) + r / 4) + 16 * (lane / 16);
      h.mtab32[f * 64 + lane] = (float)h.mtab[f * 64 + src_lane];
    }
  return h;
}

// The operands of the per-lane M2L kernel on the 4x4x1 matrix instruction, in
// the order of lane_ops.h: J, J^T and the z-translation core, each as whole
// groups of 64 values.
std::vector<float> lane_tables(const HostTables& h, int p) {
  using namespace lops;
  std::vector<float> out((size_t)table_floats(p), 0.0f);
  size_t base = 0;
  for (int trans = 0; trans < 2; ++trans) {
    int u = 0;
    for (int n = 0; n <= p; ++n) {
      const int sd = 2 * n + 1;
      for (int cls = 0; cls < 2; ++cls) {
        const int s = cls_size(n, cls);
        for (int k = 0; k < s; ++k)
          for (int c = 0; c < chunks(s); ++c, ++u)
            for (int i = 0; i < 4; ++i) {
              const int r = 4 * c + i;
              if (r >= s) continue;
              const int a = cls_member(n, cls, r), b = cls_member(n, cls, k);
              const double v = trans ? h.J[h.joff[n] + b * sd + a] : h.J[h.joff[n] + a * sd + b];
              out[base + (size_t)(u / 16) * 64 + 4 * (u % 16) + i] = (float)v;
            }
      }
    }
    base += (size_t)64 * groups(n_j(p));
  }
  const int P1 = p + 1;
  int u = 0;
  for (int m = 0; m <= p; ++m) {
    const int s = p + 1 - m;
    for (int k = 0; k < s; ++k)
      for (int c = 0; c < chunks(s); ++c, ++u)
        for (int i = 0; i < 4; ++i) {
          const int r = 4 * c + i;
          if (r >= s) continue;
          out[base + (size_t)(u / 16) * 64 + 4 * (u % 16) + i] = (float)h.A[((size_t)m * P1 + m + r) * P1 + m + k];
        }
  }
  return out;
}

// The operands of the binary64 per-quad kernels (lane_ops.h): J and, where it
// fits, J^T as 4x4 parts in instruction order, then the z-translation core
// Z[m][d][n] (output degree d, input degree n) of the given kind: for M2L
// A[m][d][n]; for M2M B[m][d][n] (n <= d) and for L2L B[m][n][d] (n >= d),
// the powers of the distance applied apart.
enum QuadKind { kQuadM2L = 0, kQuadM2M = 1, kQuadL2L = 2 };
std::vector<double> quad_tables(const HostTables& h, int p, int kind) {
  using namespace lops;
  std::vector<double> out((size_t)qtable_doubles(p), 0.0);
  const int ntab = qtable_has_jt(p) ? 2 : 1;
  for (int trans = 0; trans < ntab; ++trans) {
    double* T = out.data() + (size_t)trans * 16 * qj_count(p);
    for (int d = 0; d <= p; ++d) {
      const int sd = 2 * d + 1, nr = qreg(d);
      for (int x = 0; x < 2; ++x)
        for (int g = 0; g < nr; ++g)
          for (int c = 0; c < nr; ++c) {
            const int u = qj_offset(d, x) + g * nr + c;
            for (int k = 0; k < 4; ++k)
              for (int i = 0; i < 4; ++i) {
                const int a = qmember(d, x, 4 * c + i), b = qmember(d, x, 4 * g + k);
                if (a < 0 || b < 0) continue;
                T[16 * u + 4 * k + i] = trans ? h.J[h.joff[d] + b * sd + a] : h.J[h.joff[d] + a * sd + b];
              }
          }
    }
  }
  double* Z = out.data() + (size_t)ntab * 16 * qj_count(p);
  const size_t P1 = (size_t)p + 1;
  for (int m = 0; m <= p; ++m)
    for (int d = m; d <= p; ++d)
      for (int n = m; n <= p; ++n) {
        double v;
        if (kind == kQuadM2L)
          v = h.A[((size_t)m * P1 + d) * P1 + n];
        else if (kind == kQuadM2M)
          v = n <= d ? h.B[((size_t)m * P1 + d) * P1 + n] : 0.0;
        else
          v = n >= d ? h.B[((size_t)m * P1 + n) * P1 + d] : 0.0;
        Z[((size_t)m * P1 + d) * P1 + n] = v;
      }
  return out;
}

std::mutex g_tab_mu;
std::map<std::pair<int, int>, Tables> g_tabs;  // (device, p) -> tables

// copy enqueued on stream s; the caller waits for s before the tables are
// used anywhere else
template <class T>
T* upload(const std::vector<T>& v, hipStream_t s) {
  T* d = nullptr;
  const size_t bytes = std::max<size_t>(1, v.size()) * sizeof(T);
  if (hipMalloc((void**)&d, bytes) != hipSuccess) fail(FMM_ENOMEM, "hipMalloc failed for operator tables");
  if (!v.empty()) HIPCHECK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return d;
}

}  // namespace

bool tables_ready(int p) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  std::lock_guard<std::mutex> g(g_tab_mu);
  return g_tabs.count({dev, p}) != 0;
}

// The tables of order p on the current device, made on first use.  Later
// calls use them from any stream, also non-blocking ones that do not order
// after the null stream, and a synchronous copy from pageable memory may
// return before its data has reached the device: so the uploads go on the
// caller's stream and are waited for before the tables are published.
const Tables& tables_for(int p, hipStream_t s) {
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_tab_mu);
  auto it = g_tabs.find({dev, p});
  if (it != g_tabs.end()) return it->second;
  if (capturing(s))
    fail(FMM_EUNSUPPORTED, "the operator tables of order " + std::to_string(p) +
                               " must be made (one evaluation at this order) before graph capture");
  HostTables h = make_host_tables(p);
  Tables t;
  t.p = p;
  t.J = upload(h.J, s);
  t.joff = upload(h.joff, s);
  t.B = upload(h.B, s);
  t.rc = upload(h.rc, s);
  t.stride = h.stride;
  t.pos = upload(h.pos, s);
  t.ipos = upload(h.ipos, s);
  t.tiled = h.tiled;
  t.quad = upload(quad_tables(h, p, kQuadM2L), s);
  if (p <= kQuadXlateMaxP) {
    t.quad_m2m = upload(quad_tables(h, p, kQuadM2M), s);
    t.quad_l2l = upload(quad_tables(h, p, kQuadL2L), s);
  }
  if (h.tiled) {
    t.mtab = upload(h.mtab, s);
    t.mtab32 = upload(h.mtab32, s);
    t.sdeg = upload(h.sdeg, s);
    t.lane = upload(lane_tables(h, p), s);
  }
  HIPCHECK(hipStreamSynchronize(s));  // also keeps h alive until the copies are done
  return g_tabs.emplace(std::make_pair(dev, p), t).first->second;
}

// ----------------------------------------------------------------------------
// device
// ----------------------------------------------------------------------------
namespace {

struct XT {
  int p;
  int nt;
  int stride;
  const int* __restrict__ pos;
  const int* __restrict__ ipos;
  const double* __restrict__ J;
  const int* __restrict__ joff;
  const double* __restrict__ B;
  const double* __restrict__ rc;
};

XT make_xt(const Tables& t) { return XT{t.p, nterms(t.p), t.stride, t.pos, t.ipos, t.J, t.joff, t.B, t.rc}; }

enum Kind { kM2M = 0, kL2L = 2 };

__device__ __forceinline__ void decode(int k, int& n, int& i) {
  n = (int)sqrtf((float)k);
  while (n * n > k) --n;
  while ((n + 1) * (n + 1) <= k) ++n;
  i = k - n * n;
}

// Per-wave scratch for one translation.
struct XScratch {
  double ca[kMaxOrder + 1], sa[kMaxOrder + 1];  // cos/sin(m alpha)
  double cb[kMaxOrder + 1], sb[kMaxOrder + 1];  // cos/sin(m beta)
  double pw[2 * kMaxOrder + 2];                 // rho^k
};

// dst = Rz(sign * gamma) src   (per (c_m, s_m) pair)
__device__ __forceinline__ void rotz(const double* src, double* dst, int nt, const double* cs, const double* sn,
                                     double sign) {
  const int lane = threadIdx.x & 63;
  for (int k = lane; k < nt; k += 64) {
    int n, i;
    decode(k, n, i);
    if (i == 0) {
      dst[k] = src[k];
    } else {
      const int m = (i + 1) >> 1;
      const double c = cs[m], s = sign * sn[m];
      if (i & 1)
        dst[k] = c * src[k] - s * src[k + 1];
      else
        dst[k] = s * src[k - 1] + c * src[k];
    }
  }
}

// dst = J src (trans = false) or J^T src (trans = true), per degree
__device__ __forceinline__ void applyJ(const double* src, double* dst, const XT& tb, bool trans) {
  const int lane = threadIdx.x & 63;
  for (int k = lane; k < tb.nt; k += 64) {
    int n, i;
    decode(k, n, i);
    const int s = 2 * n + 1;
    const double* Jn = tb.J + tb.joff[n];
    const double* x = src + n * n;
    double acc = 0.0;
    if (!trans) {
      for (int q = 0; q < s; ++q) acc += Jn[i * s + q] * x[q];
    } else {
      for (int q = 0; q < s; ++q) acc += Jn[q * s + i] * x[q];
    }
    dst[k] = acc;
  }
}

__device__ __forceinline__ int cidx(int n, int m, int t) { return n * n + (m == 0 ? 0 : 2 * m - 1 + t); }

__device__ __forceinline__ void ztrans(const double* src, double* dst, const XT& tb, const double* pw, int kind) {
  const int lane = threadIdx.x & 63;
  const int p = tb.p, P1 = p + 1;
  for (int k = lane; k < tb.nt; k += 64) {
    int d, i;
    decode(k, d, i);
    const int m = (i + 1) >> 1;
    const int t = (i == 0) ? 0 : ((i & 1) ? 0 : 1);
    double acc = 0.0;
    if (kind == kM2M) {
      const double* Br = tb.B + ((size_t)m * P1 + d) * P1;
      for (int j = m; j <= d; ++j) acc += Br[j] * (pw[d - j] * src[cidx(j, m, t)]);
    } else {
      for (int n = d; n <= p; ++n) acc += tb.B[((size_t)m * P1 + n) * P1 + d] * (pw[n - d] * src[cidx(n, m, t)]);
    }
    dst[k] = acc;
  }
}

// acc += T(d) X for one M2M or L2L translation, d = (dx, dy, dz) = child
// centre - parent centre.  X is overwritten.  Called by a whole 64-lane
// workgroup.
__device__ void translate(int kind, double dx, double dy, double dz, double* X, double* T, double* acc,
                          const XT& tb, XScratch& sc) {
  const int lane = threadIdx.x & 63;
  const int nt = tb.nt, p = tb.p;
  const double rxy2 = dx * dx + dy * dy;
  const double rho2 = rxy2 + dz * dz;
  if (rho2 == 0.0) {  // coincident centres: identity
    for (int k = lane; k < nt; k += 64) acc[k] += X[k];
    __syncthreads();
    return;
  }
  const double rho = sqrt(rho2), rxy = sqrt(rxy2);
  const double ca1 = dz / rho, sa1 = rxy / rho;
  const double cb1 = rxy > 0.0 ? dx / rxy : 1.0, sb1 = rxy > 0.0 ? dy / rxy : 0.0;
  if (lane <= p) {
    double c = 1.0, s = 0.0, c2 = 1.0, s2 = 0.0;
    for (int q = 0; q < lane; ++q) {
      const double cn = c * ca1 - s * sa1, sn = s * ca1 + c * sa1;
      c = cn;
      s = sn;
      const double cn2 = c2 * cb1 - s2 * sb1, sn2 = s2 * cb1 + c2 * sb1;
      c2 = cn2;
      s2 = sn2;
    }
    sc.ca[lane] = c;
    sc.sa[lane] = s;
    sc.cb[lane] = c2;
    sc.sb[lane] = s2;
  }
  if (lane <= 2 * p + 1) {
    double v = 1.0;
    for (int q = 0; q < lane; ++q) v *= rho;
    sc.pw[lane] = v;
  }
  __syncthreads();
  rotz(X, T, nt, sc.cb, sc.sb, -1.0);
  __syncthreads();
  applyJ(T, X, tb, true);
  __syncthreads();
  rotz(X, T, nt, sc.ca, sc.sa, -1.0);
  __syncthreads();
  applyJ(T, X, tb, false);
  __syncthreads();
  ztrans(X, T, tb, sc.pw, kind);
  __syncthreads();
  applyJ(T, X, tb, true);
  __syncthreads();
  rotz(X, T, nt, sc.ca, sc.sa, 1.0);
  __syncthreads();
  applyJ(T, X, tb, false);
  __syncthreads();
  // acc += Rz(beta) X
  for (int k = lane; k < nt; k += 64) {
    int n, i;
    decode(k, n, i);
    double v;
    if (i == 0) {
      v = X[k];
    } else {
      const int m = (i + 1) >> 1;
      const double c = sc.cb[m], s = sc.sb[m];
      v = (i & 1) ? (c * X[k] - s * X[k + 1]) : (s * X[k - 1] + c * X[k]);
    }
    acc[k] += v;
  }
  __syncthreads();
}

// coefficient vector (standard order, LDS) <-> storage layout (global)
__device__ __forceinline__ void load_coefs(const double* __restrict__ src, double* dst, const XT& tb) {
  for (int k = threadIdx.x & 63; k < tb.nt; k += 64) dst[k] = src[tb.pos[k]];
}
__device__ __forceinline__ void store_coefs(const double* src, double* __restrict__ dst, const XT& tb) {
  for (int q = threadIdx.x & 63; q < tb.stride; q += 64) {
    const int k = tb.ipos[q];
    dst[q] = k >= 0 ? src[k] : 0.0;
  }
}

__device__ __forceinline__ int level_of(const LevelView& lv, int64_t gid) {
  int l = 0;
  while (l < lv.L && gid >= lv.gofs[l + 1]) ++l;
  return l;
}

// ---- M2M: parents of level l-1 from their 8 children on level l ----
// The three coefficient vectors of a translation (X, T, acc) live in dynamic
// LDS sized for the order, tb.nt doubles each (4 KB at p 12 instead of 10.3 KB
// for the highest order), so more workgroups fit on a CU.
__global__ __launch_bounds__(64) void k_m2m(LevelView lv, int l, XT tb, double* __restrict__ Mx) {
  extern __shared__ double xs[];
  double* X = xs;
  double* T = xs + tb.nt;
  double* acc = xs + 2 * tb.nt;
  __shared__ XScratch sc;
  const int lane = threadIdx.x;
  const int nt = tb.nt;
  const int64_t par = blockIdx.x;
  for (int k = lane; k < nt; k += 64) acc[k] = 0.0;
  const double* gp = lv.geom[l - 1] + par * 10;
  for (int c = 0; c < 8; ++c) {
    const int64_t ch = 8 * par + c;
    const double* gc = lv.geom[l] + ch * 10;
    load_coefs(Mx + (size_t)(lv.gofs[l] + ch) * tb.stride, X, tb);
    __syncthreads();
    translate(kM2M, gc[6] - gp[6], gc[7] - gp[7], gc[8] - gp[8], X, T, acc, tb, sc);
  }
  __syncthreads();
  store_coefs(acc, Mx + (size_t)(lv.gofs[l - 1] + par) * tb.stride, tb);
}

// ---- L2L: children of level l receive their parent's local expansion ----
// One workgroup per child; the workgroups are dealt to the eight XCDs in
// turn, so child (b mod 8) ceil(nbox / 8) + floor(b / 8) goes to block b:
// siblings, which read the same parent expansion, share an XCD's L2.
__global__ __launch_bounds__(64) void k_l2l(LevelView lv, int l, int64_t nbox, XT tb, double* __restrict__ Lx) {
  extern __shared__ double xs[];
  double* X = xs;
  double* T = xs + tb.nt;
  double* acc = xs + 2 * tb.nt;
  __shared__ XScratch sc;
  const int64_t ch = (int64_t)(blockIdx.x % 8) * ((nbox + 7) / 8) + blockIdx.x / 8;
  if (ch >= nbox) return;
  const int64_t par = ch >> 3;
  const double* gc = lv.geom[l] + ch * 10;
  const double* gp = lv.geom[l - 1] + par * 10;
  double* dst = Lx + (size_t)(lv.gofs[l] + ch) * tb.stride;
  load_coefs(dst, acc, tb);
  load_coefs(Lx + (size_t)(lv.gofs[l - 1] + par) * tb.stride, X, tb);
  __syncthreads();
  translate(kL2L, gc[6] - gp[6], gc[7] - gp[7], gc[8] - gp[8], X, T, acc, tb, sc);
  store_coefs(acc, dst, tb);
}

// ---- P2M: one 64-lane workgroup per leaf, lanes over points ----
// For each order m every lane puts its point's terms of degrees m..p (cosine
// and sine parts: the columns) into one LDS row; then each column is summed
// over the 64 rows in a fixed order by g lanes (g the largest power of two
// with g * columns <= 64), each adding every g-th row, and g - 1 exchanges
// add their partial sums.  The row stride p2m_stride(p) is odd, so the row
// writes and the column reads are free of bank conflicts.
__host__ __device__ constexpr int p2m_stride(int p) { return 2 * (p + 1) + 1; }

__global__ __launch_bounds__(64) void k_p2m(LevelView lv, XT tb, const double* __restrict__ px,
                                            const double* __restrict__ py, const double* __restrict__ pz,
                                            const double* __restrict__ qt, double* __restrict__ Mx) {
  extern __shared__ double rows[];  // 64 x p2m_stride(p), then the sums (tb.nt)
  const int lane = threadIdx.x;
  const int L = lv.L, p = tb.p, P1 = p + 1, nt = tb.nt;
  const int64_t b = blockIdx.x;
  const double* g = lv.geom[L] + b * 10;
  const double cx = g[6], cy = g[7], cz = g[8];
  const int s0 = lv.start[L][b], s1 = lv.start[L][b + 1];
  const double* am = tb.rc;
  const double* bm = tb.rc + P1;
  const double* c1 = tb.rc + 2 * P1;
  const double* c2 = tb.rc + 2 * P1 + P1 * P1;
  const double s2 = 1.4142135623730951;
  const int SP = p2m_stride(p);
  double* row = rows + lane * SP;
  double* acc = rows + 64 * SP;
  for (int k = lane; k < nt; k += 64) acc[k] = 0.0;
  __syncthreads();
  for (int c0 = s0; c0 < s1; c0 += 64) {
    const int t = c0 + lane;
    const bool valid = t < s1;
    const double x = valid ? px[t] - cx : 0.0;
    const double y = valid ? py[t] - cy : 0.0;
    const double z = valid ? pz[t] - cz : 0.0;
    const double q = valid ? qt[t] : 0.0;
    const double r2 = x * x + y * y + z * z;
    double mr = 1.0, mi = 0.0;  // G_m^m
    for (int m = 0; m <= p; ++m) {
      if (m > 0) {
        const double nr = am[m] * (x * mr - y * mi);
        const double ni = am[m] * (x * mi + y * mr);
        mr = nr;
        mi = ni;
      }
      // degrees m and m + 1, then the three-term recurrence two degrees per
      // pass: (ar, ai) holds G_{n-2} and receives G_n, (br, bi) holds G_{n-1}
      const double cq = (m == 0 ? 1.0 : s2) * q, sq = s2 * q;
      double ar = mr, ai = mi;
      row[0] = cq * ar;
      row[1] = sq * ai;
      if (m < p) {
        double br = bm[m] * z * mr, bi = bm[m] * z * mi;
        row[2] = cq * br;
        row[3] = sq * bi;
        int n = m + 2;
        for (; n + 1 <= p; n += 2) {
          ar = c1[n * P1 + m] * z * br - c2[n * P1 + m] * r2 * ar;
          ai = c1[n * P1 + m] * z * bi - c2[n * P1 + m] * r2 * ai;
          row[2 * (n - m)] = cq * ar;
          row[2 * (n - m) + 1] = sq * ai;
          br = c1[(n + 1) * P1 + m] * z * ar - c2[(n + 1) * P1 + m] * r2 * br;
          bi = c1[(n + 1) * P1 + m] * z * ai - c2[(n + 1) * P1 + m] * r2 * bi;
          row[2 * (n + 1 - m)] = cq * br;
          row[2 * (n + 1 - m) + 1] = sq * bi;
        }
        if (n <= p) {
          ar = c1[n * P1 + m] * z * br - c2[n * P1 + m] * r2 * ar;
          ai = c1[n * P1 + m] * z * bi - c2[n * P1 + m] * r2 * ai;
          row[2 * (n - m)] = cq * ar;
          row[2 * (n - m) + 1] = sq * ai;
        }
      }
      __syncthreads();
      // column col = 2 (n - m) + part of every row; g lanes per column
      const int ncol = 2 * (P1 - m);
      int g = 1;
      while (2 * g * ncol <= 64) g *= 2;
      const int col = lane / g, sub = lane % g;
      double v = 0.0;
      if (col < ncol)
        for (int r = sub; r < 64; r += g) v += rows[r * SP + col];
      for (int d = 1; d < g; d <<= 1) v += __shfl_xor(v, d);
      const int n = m + (col >> 1), part = col & 1;
      if (col < ncol && sub == 0 && (m > 0 || part == 0)) acc[cidx(n, m, part)] += v;
      __syncthreads();
    }
  }
  __syncthreads();
  store_coefs(acc, Mx + (size_t)(lv.gofs[L] + b) * tb.stride, tb);
}

// ---- L2P: far field at the points of each leaf (phi and E = -grad phi) ----
// The evaluation points of leaf b are [start[b], start[b+1]) of (px, py, pz):
// the leaf's own sources, or the separate targets grouped by leaf.
__global__ __launch_bounds__(64) void k_l2p(LevelView lv, XT tb, const int32_t* __restrict__ start,
                                            const double* __restrict__ px, const double* __restrict__ py,
                                            const double* __restrict__ pz, const double* __restrict__ Lx,
                                            double* __restrict__ fphi, double* __restrict__ fex,
                                            double* __restrict__ fey, double* __restrict__ fez) {
  const int lane = threadIdx.x;
  const int L = lv.L, p = tb.p, P1 = p + 1;
  const int64_t b = blockIdx.x;
  const double* g = lv.geom[L] + b * 10;
  const double cx = g[6], cy = g[7], cz = g[8];
  const int s0 = start[b], s1 = start[b + 1];
  const double* Lc = Lx + (size_t)(lv.gofs[L] + b) * tb.stride;
  const int* pos = tb.pos;
  const double* am = tb.rc;
  const double* bm = tb.rc + P1;
  const double* c1 = tb.rc + 2 * P1;
  const double* c2 = tb.rc + 2 * P1 + P1 * P1;
  const double s2 = 1.4142135623730951;
  for (int c0 = s0; c0 < s1; c0 += 64) {
    const int t = c0 + lane;
    if (t >= s1) break;
    const double x = px[t] - cx, y = py[t] - cy, z = pz[t] - cz;
    const double r2 = x * x + y * y + z * z;
    // G and its gradient (complex): value, d/dx, d/dy, d/dz
    double mr = 1.0, mi = 0.0, mxr = 0, mxi = 0, myr = 0, myi = 0, mzr = 0, mzi = 0;
    double f = 0, fx = 0, fy = 0, fz = 0;
    for (int m = 0; m <= p; ++m) {
      if (m > 0) {
        const double a = am[m];
        // G = a (x + i y) Gp;  dG = a [(1, i, 0) Gp + (x + i y) dGp]
        const double nr = a * (x * mr - y * mi), ni = a * (x * mi + y * mr);
        const double nxr = a * (mr + x * mxr - y * mxi), nxi = a * (mi + x * mxi + y * mxr);
        const double nyr = a * (-mi + x * myr - y * myi), nyi = a * (mr + x * myi + y * myr);
        const double nzr = a * (x * mzr - y * mzi), nzi = a * (x * mzi + y * mzr);
        mr = nr; mi = ni; mxr = nxr; mxi = nxi; myr = nyr; myi = nyi; mzr = nzr; mzi = nzi;
      }
      // degree n = m, then n = m + 1, then the three-term recurrence, two
      // degrees per pass so that the two history arrays alternate roles
      // instead of being copied: ga holds G_{n-2} and receives G_n, gb holds
      // G_{n-1}
      const double msc = m == 0 ? 1.0 : s2;
      auto add = [&](const double* g, int n) __attribute__((always_inline)) {
        const double lc = Lc[pos[cidx(n, m, 0)]] * msc;
        const double ls = m == 0 ? 0.0 : Lc[pos[cidx(n, m, 1)]] * s2;
        f += lc * g[0] + ls * g[1];
        fx += lc * g[2] + ls * g[3];
        fy += lc * g[4] + ls * g[5];
        fz += lc * g[6] + ls * g[7];
      };
      // G_n from G_{n-1} (gb) and G_{n-2} (ga, overwritten; its components 0
      // and 1 are read by the gradient terms, so they are replaced last)
      auto rec = [&](double* ga, const double* gb, int n) __attribute__((always_inline)) {
        const double a1 = c1[n * P1 + m], a2 = c2[n * P1 + m];
        const double g0 = ga[0], g1v = ga[1];
        ga[2] = a1 * z * gb[2] - a2 * (r2 * ga[2] + 2.0 * x * g0);
        ga[3] = a1 * z * gb[3] - a2 * (r2 * ga[3] + 2.0 * x * g1v);
        ga[4] = a1 * z * gb[4] - a2 * (r2 * ga[4] + 2.0 * y * g0);
        ga[5] = a1 * z * gb[5] - a2 * (r2 * ga[5] + 2.0 * y * g1v);
        ga[6] = a1 * (gb[0] + z * gb[6]) - a2 * (r2 * ga[6] + 2.0 * z * g0);
        ga[7] = a1 * (gb[1] + z * gb[7]) - a2 * (r2 * ga[7] + 2.0 * z * g1v);
        ga[0] = a1 * z * gb[0] - a2 * r2 * g0;
        ga[1] = a1 * z * gb[1] - a2 * r2 * g1v;
      };
      double gA[8] = {mr, mi, mxr, mxi, myr, myi, mzr, mzi};  // G_m^m
      add(gA, m);
      if (m < p) {
        const double bb = bm[m];
        double gB[8] = {bb * z * mr,  bb * z * mi,  bb * z * mxr,         bb * z * mxi,
                        bb * z * myr, bb * z * myi, bb * (mr + z * mzr), bb * (mi + z * mzi)};  // G_{m+1}^m
        add(gB, m + 1);
        int n = m + 2;
        for (; n + 1 <= p; n += 2) {
          rec(gA, gB, n);
          add(gA, n);
          rec(gB, gA, n + 1);
          add(gB, n + 1);
        }
        if (n <= p) {
          rec(gA, gB, n);
          add(gA, n);
        }
      }
    }
    fphi[t] = f;
    fex[t] = -fx;
    fey[t] = -fy;
    fez[t] = -fz;
  }
}

}  // namespace

// launch helpers used by evaluate() (p2p.hip)
void launch_p2m(const Tree& t, const Tables& tb, const double* qt, double* Mx, hipStream_t s) {
  const size_t lds = ((size_t)64 * p2m_stride(tb.p) + nterms(tb.p)) * sizeof(double);
  k_p2m<<<(unsigned)t.lev[t.L].nbox, 64, lds, s>>>(t.view(), make_xt(tb), t.px, t.py, t.pz, qt, Mx);
  HIPCHECK(hipGetLastError());
}
bool launch_m2m_quad64(const Tree& t, int l, const Tables& tb, double* Mx, hipStream_t s);
bool launch_l2l_quad64(const Tree& t, int l, const Tables& tb, double* Lx, hipStream_t s);

// M2M and L2L four lanes per translation on the matrix cores up to order
// kQuadXlateMaxP, the generic translation above
void launch_m2m(const Tree& t, int l, const Tables& tb, double* Mx, hipStream_t s) {
  if (launch_m2m_quad64(t, l, tb, Mx, s)) return;
  const size_t lds = 3 * (size_t)nterms(tb.p) * sizeof(double);
  k_m2m<<<(unsigned)t.lev[l - 1].nbox, 64, lds, s>>>(t.view(), l, make_xt(tb), Mx);
  HIPCHECK(hipGetLastError());
}
bool launch_m2l_mfma(const Tree& t, const Tables& tb, const double* Mx, double* Lx, hipStream_t s);
bool launch_m2l_mfma_mixed(const Tree& t, const Tables& tb, const double* Mx, double* Lx, hipStream_t s);
bool launch_m2l_quad64(const Tree& t, const Tables& tb, const double* Mx, double* Lx, hipStream_t s);

// M2L on the matrix cores: binary32 on scaled expansions for orders up to 15
// unless binary64 is asked for (one pair per lane up to 14, 16-pair tiles at
// 15), else binary64 (four lanes per pair at orders up to 13 and 16..20,
// 16-pair tiles at 14 and 15)
void launch_m2l(const Tree& t, const Tables& tb, const double* Mx, double* Lx, int prec, hipStream_t s) {
  if (prec != FMM_PREC_F64 && launch_m2l_mfma_mixed(t, tb, Mx, Lx, s)) return;
  if (launch_m2l_quad64(t, tb, Mx, Lx, s)) return;
  if (launch_m2l_mfma(t, tb, Mx, Lx, s)) return;
  fail(FMM_EUNSUPPORTED, "no M2L kernel for order " + std::to_string(tb.p));
}
void launch_l2l(const Tree& t, int l, const Tables& tb, double* Lx, hipStream_t s) {
  if (launch_l2l_quad64(t, l, tb, Lx, s)) return;
  const int64_t nbox = t.lev[l].nbox;
  const size_t lds = 3 * (size_t)nterms(tb.p) * sizeof(double);
  k_l2l<<<(unsigned)(8 * ((nbox + 7) / 8)), 64, lds, s>>>(t.view(), l, nbox, make_xt(tb), Lx);
  HIPCHECK(hipGetLastError());
}
void launch_l2p(const Tree& t, const Tables& tb, const double* Lx, const int32_t* start, const double* px,
                const double* py, const double* pz, double* f0, double* f1, double* f2, double* f3, hipStream_t s) {
  k_l2p<<<(unsigned)t.lev[t.L].nbox, 64, 0, s>>>(t.view(), make_xt(tb), start, px, py, pz, Lx, f0, f1, f2, f3);
  HIPCHECK(hipGetLastError());
}

}  // namespace fmm
