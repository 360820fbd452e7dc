// M2L in binary64 (Algorithm 3, M2L; rotational form of Section 2.1.3), four
// lanes per weak pair, the fixed quarter turns on the matrix cores.
//
// The translation is the sequence of the other M2L kernels:
//   Rz(-beta), J^T, Rz(-alpha), J, z-axis translation, J^T, Rz(alpha), J, Rz(beta),
// with J the fixed quarter turn about x and (alpha, beta) the polar and
// azimuthal angles of d = c_source - c_target, on radius-scaled expansions
// (M~_n = M_n / r_s^n in, the factors (r_s/rho)^n and (r_t/rho)^j / rho, the
// result unscaled by r_t^-n), here all in binary64.
//
// A wave takes 16 pairs of one target box; lane 16 k + q holds phase k of
// pair q, i.e. the members m = k (mod 4) of every block (lane_ops.h: per
// degree two blocks indexed by the order m, the two parity classes of J).
// Hence:
//   - a J block is a chain of v_mfma_f64_4x4x4f64, one per (k-step, output
//     chunk of 4 rows): the instruction's k index runs over the four phase
//     lanes of a pair, and its output row i lands in phase i of the same pair,
//     so every step's result is the next step's operand in place; the
//     operator values come from LDS (binary64 instructions take no broadcast
//     of one block's operand, so every lane reads its value); J^T has a
//     table of its own up to order 18 and above reads the table of J with
//     the two chunk indices swapped and each 4x4 part transposed;
//   - a z-turn multiplies the (cosine, sine) parts of (d, m), which share a
//     lane and register, by the lane's own e^{i m theta};
//   - the z translation of order m involves only order-m coefficients of
//     all degrees, which share a lane: each lane runs it for its orders on the
//     vector units (binary64 vector and matrix peaks are equal on this part);
//   - the 16 pair results are summed across the lanes by halving exchanges
//     through DPP (fixed order: deterministic) and the batches in binary64.
// Padding is per 4x4 part of a block: 1.57x the algorithmic J products at
// order 12, against 2.42x for the 16x16 tiles of m2l_mfma.hip.  Orders 16..20
// run here too (one wave per SIMD), where the tiles stop.
//
// The same steps with the M2M or L2L core along z make k_xlate_quad (end of
// the file), which runs M2M and L2L up to order 13.
#include <type_traits>

#include "fmm_internal.h"
#include "lane_ops.h"
#include "tile_layout.h"

namespace fmm {
namespace {

template <int B, int E, class F>
__device__ __forceinline__ void qfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    qfor<B + 1, E>(f);
  }
}

// sizes of the halving exchanges over the 16 pairs of a wave
__host__ __device__ constexpr int qlvl(int nt, int s) {
  int v = nt;
  for (int k = 0; k < s; ++k) v = (v + 1) / 2;
  return v;
}

// degree of register R
__host__ __device__ constexpr int qdeg(int R) {
  int d = 0;
  while (lops::qbase(d + 1, 0) <= R) ++d;
  return d;
}

__device__ __forceinline__ double mfma64(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// One block (d, x) of a J application: NR = qreg(d) k-steps times NR output
// chunks; tl = the lane's slot in a 16-value operand, 4 k + i, or with T
// (J^T from the table of J, whose part (c, g) transposed is part (g, c) of
// J^T) 4 i + k
template <int D, int X>
struct QBlk {
  static constexpr int NR = lops::qreg(D);
  static constexpr int R0 = lops::qbase(D, X);
  static constexpr int U0 = lops::qj_offset(D, X);
  double acc[NR];
  __device__ __forceinline__ QBlk() {
    qfor<0, NR>([&](auto c) __attribute__((always_inline)) { acc[c] = 0.0; });
  }
  template <bool T, int G>
  __device__ __forceinline__ void step(const double* X_, const double* tab, int tl) {
    if constexpr (G < NR) {
      const double xg = X_[R0 + G];
      qfor<0, NR>([&](auto c) __attribute__((always_inline)) {
        constexpr int C = decltype(c)::value;
        constexpr int u = U0 + (T ? C * NR + G : G * NR + C);
        acc[c] = mfma64(tab[16 * u + tl], xg, acc[c]);
      });
    }
  }
  __device__ __forceinline__ void store(double* X_) {
    qfor<0, NR>([&](auto c) __attribute__((always_inline)) { X_[R0 + decltype(c)::value] = acc[c]; });
  }
};

// X <- J X (or J^T X from its own table; T: J^T X from the table of J, tl the
// lane's slot for that case): degree d beside degree P - d, both blocks each,
// in lock-step over the k-steps (independent chains in flight)
template <int P, bool T>
__device__ __forceinline__ void qjapply(double* X, const double* tab, int tl) {
  qfor<0, P / 2 + 1>([&](auto dI) __attribute__((always_inline)) {
    constexpr int d = decltype(dI)::value, d2 = P - d;
    QBlk<d, 0> a0;
    QBlk<d, 1> a1;
    if constexpr (d2 > d) {
      QBlk<d2, 0> b0;
      QBlk<d2, 1> b1;
      qfor<0, lops::qreg(d2)>([&](auto g) __attribute__((always_inline)) {
        constexpr int G = decltype(g)::value;
        a0.template step<T, G>(X, tab, tl);
        a1.template step<T, G>(X, tab, tl);
        b0.template step<T, G>(X, tab, tl);
        b1.template step<T, G>(X, tab, tl);
      });
      b0.store(X);
      b1.store(X);
    } else {
      qfor<0, lops::qreg(d)>([&](auto g) __attribute__((always_inline)) {
        constexpr int G = decltype(g)::value;
        a0.template step<T, G>(X, tab, tl);
        a1.template step<T, G>(X, tab, tl);
      });
    }
    a0.store(X);
    a1.store(X);
    __builtin_amdgcn_sched_barrier(0);
  });
}

// X <- Rz(sign * theta) X with (c1, s1) = (cos theta, sin theta): the lane's
// members m = 4 g + k turn by e^{i m theta}; with block 0 holding c_m for
// even m and s_m for odd m, the turn of (b0, b1) is (C b0 - S' b1, S' b0 +
// C b1) with S' = S for even m and -S for odd m
template <int P>
__device__ __forceinline__ void qrotz(double* X, double c1, double s1, double sign, int k) {
  constexpr int NG = P / 4 + 1;
  // e^{i k theta} and e^{i 4 theta}
  const double c2 = c1 * c1 - s1 * s1, s2 = 2.0 * s1 * c1;
  const double c3 = c2 * c1 - s2 * s1, s3 = s2 * c1 + c2 * s1;
  const double c4 = c2 * c2 - s2 * s2, s4 = 2.0 * s2 * c2;
  double cc = k == 0 ? 1.0 : k == 1 ? c1 : k == 2 ? c2 : c3;
  double ss = k == 0 ? 0.0 : k == 1 ? s1 : k == 2 ? s2 : s3;
  const double par = (k & 1) ? -sign : sign;
  double C[NG], S[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    C[g] = cc;
    S[g] = par * ss;
    const double nc = cc * c4 - ss * s4, ns = ss * c4 + cc * s4;
    cc = nc;
    ss = ns;
  }
  qfor<0, P + 1>([&](auto dI) __attribute__((always_inline)) {
    constexpr int d = decltype(dI)::value;
    qfor<0, lops::qreg(d)>([&](auto g) __attribute__((always_inline)) {
      constexpr int G = decltype(g)::value;
      constexpr int r0 = lops::qbase(d, 0) + G, r1 = lops::qbase(d, 1) + G;
      const double b0 = X[r0], b1 = X[r1];
      X[r0] = C[G] * b0 - S[G] * b1;
      X[r1] = S[G] * b0 + C[G] * b1;
    });
  });
}

// the z-axis translation: the lane's orders m = 4 g + k, both blocks, with
// the core A[m][d][n] of its own order (Az, orders above P zero).  Input
// degree n is first multiplied by in_base^n and output degree d by out_mult
// out_base^d; with EXP also by 2^(in_exp n) and 2^(out_exp d) (ldexp: exact,
// and saturating only where the scaled value itself leaves the range)
template <int P, bool EXP = false>
__device__ __forceinline__ void qztrans(double* X, const double* __restrict__ Az, int k, double in_base,
                                        double out_base, double out_mult, int in_exp = 0, int out_exp = 0) {
  constexpr int P1 = P + 1;
  {
    double w = 1.0;
    qfor<0, P + 1>([&](auto dI) __attribute__((always_inline)) {
      constexpr int d = decltype(dI)::value;
      qfor<0, 2 * lops::qreg(d)>([&](auto r) __attribute__((always_inline)) {
        if constexpr (EXP)
          X[lops::qbase(d, 0) + decltype(r)::value] = ldexp(X[lops::qbase(d, 0) + decltype(r)::value] * w, in_exp * d);
        else
          X[lops::qbase(d, 0) + decltype(r)::value] *= w;
      });
      w *= in_base;
    });
  }
  qfor<0, P / 4 + 1>([&](auto gI) __attribute__((always_inline)) {
    constexpr int G = decltype(gI)::value;
    constexpr int N0 = 4 * G;  // lowest degree holding register G
    // the lane's order, orders above P reading the zero slot P + 1
    const double* Am = Az + (4 * G + k <= P ? 4 * G + k : P + 1) * P1 * P1;
    double y0[P1 - N0], y1[P1 - N0];
    qfor<0, P1 - N0>([&](auto r) __attribute__((always_inline)) { y0[r] = y1[r] = 0.0; });
    // input degree by input degree: only one column of the core is loaded
    // at a time (all of them at once would not fit the registers)
    qfor<N0, P1>([&](auto nI) __attribute__((always_inline)) {
      constexpr int n = decltype(nI)::value;
      const double x0 = X[lops::qbase(n, 0) + G], x1 = X[lops::qbase(n, 1) + G];
      qfor<N0, P1>([&](auto dI) __attribute__((always_inline)) {
        constexpr int d = decltype(dI)::value;
        const double a = Am[d * P1 + n];
        y0[d - N0] += a * x0;
        y1[d - N0] += a * x1;
      });
      __builtin_amdgcn_sched_barrier(0);
    });
    qfor<N0, P1>([&](auto dI) __attribute__((always_inline)) {
      constexpr int d = decltype(dI)::value;
      X[lops::qbase(d, 0) + G] = y0[d - N0];
      X[lops::qbase(d, 1) + G] = y1[d - N0];
    });
  });
  {
    double w = out_mult;
    qfor<0, P + 1>([&](auto dI) __attribute__((always_inline)) {
      constexpr int d = decltype(dI)::value;
      qfor<0, 2 * lops::qreg(d)>([&](auto r) __attribute__((always_inline)) {
        if constexpr (EXP)
          X[lops::qbase(d, 0) + decltype(r)::value] = ldexp(X[lops::qbase(d, 0) + decltype(r)::value] * w, out_exp * d);
        else
          X[lops::qbase(d, 0) + decltype(r)::value] *= w;
      });
      w *= out_base;
    });
  }
}

__device__ __forceinline__ int qlevel_of(const LevelView& lv, int64_t gid) {
  int l = 0;
  while (l < lv.L && gid >= lv.gofs[l + 1]) ++l;
  return l;
}

// Waves per SIMD: 2 up to order 13, 1 from 16 on.  One block per CU (512
// threads for two waves per SIMD, 256 for one), so that the tables (J, J^T up
// to order 18, the z core: 55 KB at order 12, 158 KB at 18, 143 KB at 20) are
// staged into LDS once per CU.
template <int P>
struct QuadCfg {
  static constexpr int kWaves = P <= 13 ? 2 : 1;
  static constexpr int kThreads = 256 * kWaves;
  static constexpr int kJ = 16 * lops::qj_count(P);  // doubles of the J table
  static constexpr int kLds = lops::qtable_doubles(P);
  static_assert(kLds * 8 <= 160 * 1024, "the tables must fit in LDS");
};

// One step of the translation, kept apart from its neighbours by the
// scheduler (bounds the registers in flight)
#define FMM_QSTEP(x) \
  x;                 \
  __builtin_amdgcn_sched_barrier(0)

// A halving exchange over lanes at distance D (8, 4, 2 or 1: within a row of
// 16 lanes) of a wave whose lanes hold NS values src: lanes with that lane bit
// clear keep the lower ND values and add their partner's, the others the
// upper ones (zero-padded).  The partner's value is a DPP read (row_ror:8,
// quad_perm [2,3,0,1] or [1,0,3,2]; distance 4 as two shifts, row_shl:4 and
// row_shr:4), vector work instead of LDS permutes, which the operand reads
// already load.
template <int CTRL>
__device__ __forceinline__ double qdpp(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, 0xf, 0xf, true),
                          __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xf, 0xf, true));
}
template <int NS, int ND, int D>
__device__ __forceinline__ void qhalve(const double* src, double* dst, int lane) {
  const bool up = (lane & D) != 0;
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    const double lo = src[i];
    const double hi = ND + i < NS ? src[ND + i] : 0.0;
    if constexpr (D == 4) {
      const double t0 = lo + qdpp<0x104>(lo), t1 = hi + qdpp<0x114>(hi);
      dst[i] = up ? t1 : t0;
    } else {
      constexpr int C = D == 8 ? 0x128 : D == 2 ? 0x4E : 0xB1;
      const double send = up ? lo : hi, keep = up ? hi : lo;
      dst[i] = keep + qdpp<C>(send);
    }
    if ((i & 7) == 7) __builtin_amdgcn_sched_barrier(0);
  }
}

template <int P>
__global__ __launch_bounds__(QuadCfg<P>::kThreads)
__attribute__((amdgpu_waves_per_eu(QuadCfg<P>::kWaves, QuadCfg<P>::kWaves))) void
k_m2l_quad(LevelView lv, const double* __restrict__ qtab, const int* __restrict__ pos, int S,
           const double* __restrict__ Mq, double* __restrict__ Lx, int64_t ntarget, const int32_t* __restrict__ order,
           int* __restrict__ queue) {
  constexpr int NQ = lops::nq(P);
  constexpr int NJ = QuadCfg<P>::kJ;
  constexpr int NF = qlvl(NQ, 4);  // values a lane holds after the exchanges
  constexpr int NL = QuadCfg<P>::kLds;
  __shared__ double tabs[NL];
  for (int i = threadIdx.x; i < NL; i += blockDim.x) tabs[i] = qtab[i];
  __syncthreads();
  constexpr bool HJT = lops::qtable_has_jt(P);
  const double* Az = tabs + (HJT ? 2 : 1) * NJ;
  const int lane = threadIdx.x & 63;
  const int k = lane >> 4, q = lane & 15;
  const int tl = 4 * k + (lane & 3);   // this lane's value in a 4x4 part of J
  const int tlt = 4 * (lane & 3) + k;  // and of J^T
  for (;;) {
    int kq = 0;
    if (lane == 0) kq = atomicAdd(queue, 1);
    kq = __builtin_amdgcn_readfirstlane(kq);
    if (kq >= ntarget) break;
    const int64_t gid = lv.gofs[1] + order[kq];
    const int l = qlevel_of(lv, gid);
    const int64_t bi = gid - lv.gofs[l];
    const double* geo = lv.geom[l];
    const double cix = geo[bi * 10 + 6], ciy = geo[bi * 10 + 7], ciz = geo[bi * 10 + 8];
    const double rt = geo[bi * 10 + 9] > 0.0 ? geo[bi * 10 + 9] : 1.0;
    const int64_t e0 = lv.w_off[l][bi], e1 = lv.w_off[l][bi + 1];
    const int32_t* widx = lv.w_idx[l];
    const double* Mlev = Mq + (size_t)lv.gofs[l] * NQ * 4;
    double acc[NF];
#pragma unroll
    for (int i = 0; i < NF; ++i) acc[i] = 0.0;

    for (int64_t eb = e0; eb < e1; eb += 16) {
      const int64_t e = eb + q;
      const bool valid = e < e1;
      const int64_t j = widx[valid ? e : e0];
      const double dx = geo[j * 10 + 6] - cix, dy = geo[j * 10 + 7] - ciy, dz = geo[j * 10 + 8] - ciz;
      const double rs = geo[j * 10 + 9] > 0.0 ? geo[j * 10 + 9] : 1.0;
      const double rxy2 = dx * dx + dy * dy;
      const double rho = sqrt(rxy2 + dz * dz), rxy = sqrt(rxy2);
      const double irho = 1.0 / rho;
      const double ca = dz * irho, sa = rxy * irho;
      const double cb = rxy > 0.0 ? dx / rxy : 1.0, sb = rxy > 0.0 ? dy / rxy : 0.0;
      // a pair past the end of the list translates the first source with zero factors
      const double in_base = valid ? rs * irho : 0.0;
      const double out_base = valid ? rt * irho : 0.0;
      const double out_mult = valid ? irho : 0.0;

      double X[NQ];
      const double* src = Mlev + (size_t)j * NQ * 4 + k;
#pragma unroll
      for (int r = 0; r < NQ; ++r) X[r] = src[4 * r];

      FMM_QSTEP(qrotz<P>(X, cb, sb, -1.0, k));
      FMM_QSTEP((qjapply<P, !HJT>(X, HJT ? tabs + NJ : tabs, HJT ? tl : tlt)));
      FMM_QSTEP(qrotz<P>(X, ca, sa, -1.0, k));
      FMM_QSTEP((qjapply<P, false>(X, tabs, tl)));
      FMM_QSTEP(qztrans<P>(X, Az, k, in_base, out_base, out_mult));
      FMM_QSTEP((qjapply<P, !HJT>(X, HJT ? tabs + NJ : tabs, HJT ? tl : tlt)));
      FMM_QSTEP(qrotz<P>(X, ca, sa, 1.0, k));
      FMM_QSTEP((qjapply<P, false>(X, tabs, tl)));
      FMM_QSTEP(qrotz<P>(X, cb, sb, 1.0, k));

      // sum over the 16 pairs (lane bits 0..3): four halving exchanges
      double h1[qlvl(NQ, 1)], h2[qlvl(NQ, 2)], h3[qlvl(NQ, 3)], h4[qlvl(NQ, 4)];
      qhalve<NQ, qlvl(NQ, 1), 8>(X, h1, lane);
      qhalve<qlvl(NQ, 1), qlvl(NQ, 2), 4>(h1, h2, lane);
      qhalve<qlvl(NQ, 2), qlvl(NQ, 3), 2>(h2, h3, lane);
      qhalve<qlvl(NQ, 3), qlvl(NQ, 4), 1>(h3, h4, lane);
#pragma unroll
      for (int i = 0; i < NF; ++i) acc[i] += h4[i];
    }
    // lane's values: registers base + i of phase k, where each exchange
    // added the kept half's offset; entries past a half's end are padding
    int base = 0, len = NQ;
#pragma unroll
    for (int sidx = 1; sidx <= 4; ++sidx) {
      const int half = qlvl(NQ, sidx);
      const int dist = 16 >> sidx;
      if (lane & dist) {
        base += half;
        len = len - half > 0 ? len - half : 0;
      } else {
        len = len < half ? len : half;
      }
    }
    double* dst = Lx + (size_t)gid * S;
    const double irt = 1.0 / rt;
    qfor<0, NF>([&](auto iI) __attribute__((always_inline)) {
      constexpr int i = decltype(iI)::value;
      if (i < len) {
        const int R = base + i;
        const int d = qdeg(R);
        const int x = R - lops::qbase(d, 0) >= lops::qreg(d) ? 1 : 0;
        const int g = R - lops::qbase(d, x);
        const int mi = lops::qmember(d, x, 4 * g + k);
        if (mi >= 0) {
          double v = acc[i];
          for (int t = 0; t < d; ++t) v *= irt;
          dst[pos[d * d + mi]] = v;
        }
      }
    });
  }
}

// The multipoles of levels 1..L in the quad layout, scaled by r^-n (r the box
// radius, 1 for a box of zero extent): per box NQ registers x 4 phases.
template <int P>
__global__ void k_quad_copy(LevelView lv, int S, const int* __restrict__ pos, const double* __restrict__ Mx,
                            double* __restrict__ Mq, int64_t nbox_total) {
  constexpr int NQ = lops::nq(P);
  const int64_t gid = 1 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (gid >= nbox_total) return;
  int l = 1;
  while (l < lv.L && gid >= lv.gofs[l + 1]) ++l;
  const double r = lv.geom[l][(gid - lv.gofs[l]) * 10 + 9];
  const double is = r > 0.0 ? 1.0 / r : 1.0;
  for (int t = threadIdx.x & 63; t < 4 * NQ; t += 64) {
    const int R = t >> 2, k = t & 3;
    const int d = qdeg(R);
    const int x = R - lops::qbase(d, 0) >= lops::qreg(d) ? 1 : 0;
    const int g = R - lops::qbase(d, x);
    const int mi = lops::qmember(d, x, 4 * g + k);
    double v = 0.0;
    if (mi >= 0) {
      v = Mx[(size_t)gid * S + pos[d * d + mi]];
      for (int u = 0; u < d; ++u) v *= is;
    }
    Mq[(size_t)gid * NQ * 4 + t] = v;
  }
}

__global__ void k_zero_queue_q(int* queue) {
  if (threadIdx.x == 0) *queue = 0;
}

template <int P>
void launch_one_quad(const Tree& t, const Tables& tb, const double* Mx, double* Lx, hipStream_t s) {
  const int64_t ntarget = t.nbox_total - 1;
  if (ntarget <= 0) return;
  constexpr int NQ = lops::nq(P);
  double* Mq = (double*)dalloc((size_t)t.nbox_total * NQ * 4 * sizeof(double), s);
  k_quad_copy<P><<<(unsigned)((ntarget + 3) / 4), 256, 0, s>>>(t.view(), tb.stride, tb.pos, Mx, Mq, t.nbox_total);
  HIPCHECK(hipGetLastError());
  static const int grid_max = [] {
    int dev = 0, ncu = 0, per = 0;
    HIPCHECK(hipGetDevice(&dev));
    HIPCHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_m2l_quad<P>, QuadCfg<P>::kThreads, 0));
    return ncu * (per > 0 ? per : 1);
  }();
  const int64_t need = (ntarget + QuadCfg<P>::kThreads / 64 - 1) / (QuadCfg<P>::kThreads / 64);
  const unsigned grid = (unsigned)(need < grid_max ? need : grid_max);
  int* queue = (int*)dalloc(sizeof(int), s);
  k_zero_queue_q<<<1, 64, 0, s>>>(queue);
  HIPCHECK(hipGetLastError());
  k_m2l_quad<P><<<grid, QuadCfg<P>::kThreads, 0, s>>>(t.view(), tb.quad, tb.pos, tb.stride, Mq, Lx, ntarget,
                                                       t.m2l_order, queue);
  HIPCHECK(hipGetLastError());
  dfree(queue, s);
  dfree(Mq, s);
}

// ---- M2M and L2L, four lanes per translation (Algorithm 1 M2M, Algorithm 3
// L2L; orders up to kQuadXlateMaxP) ----
// The rotations and quarter turns of the M2L kernel with the M2M or L2L core
// along z; the distance powers are applied apart (M2M: input degree n times
// rho^-n, output degree d times rho^d; L2L the reverse), in binary64 without
// radius scaling, each power split into one of mu in [1, 2) and an exact
// power-of-two scaling.  A wave takes 16 children of level l, the children of two
// parents: M2M sums each parent's eight translated children by three halving
// exchanges and writes the parent (and zeroes its storage's padding slots);
// L2L adds the parent's translated expansion into each child.  The vector is
// child centre - parent centre for both, as in the generic translation, and
// a pair at distance zero is the identity (its input is added back).
template <int P, bool L2L>
__global__ __launch_bounds__(QuadCfg<P>::kThreads)
__attribute__((amdgpu_waves_per_eu(QuadCfg<P>::kWaves, QuadCfg<P>::kWaves))) void
k_xlate_quad(LevelView lv, int l, const double* __restrict__ qtab, const int* __restrict__ pos,
             const int* __restrict__ ipos, int S, double* __restrict__ E, int64_t ngroup) {
  constexpr int NQ = lops::nq(P);
  constexpr int NJ = QuadCfg<P>::kJ;
  constexpr int NL = QuadCfg<P>::kLds;
  constexpr int NF = qlvl(NQ, 3);  // values a lane holds after the M2M exchanges
  static_assert(lops::qtable_has_jt(P), "orders whose table holds J^T");
  __shared__ double tabs[NL];
  __shared__ int spos[NQ * 4];  // storage position of (register, phase); -1: zero slot
  for (int i = threadIdx.x; i < NL; i += blockDim.x) tabs[i] = qtab[i];
  for (int t = threadIdx.x; t < NQ * 4; t += blockDim.x) {
    const int R = t >> 2, ph = t & 3;
    const int d = qdeg(R);
    const int x = R - lops::qbase(d, 0) >= lops::qreg(d) ? 1 : 0;
    const int mi = lops::qmember(d, x, 4 * (R - lops::qbase(d, x)) + ph);
    spos[t] = mi >= 0 ? pos[d * d + mi] : -1;
  }
  __syncthreads();
  const double* Az = tabs + 2 * NJ;
  const int lane = threadIdx.x & 63;
  const int k = lane >> 4, q = lane & 15;
  const int tl = 4 * k + (lane & 3);
  const double* gch = lv.geom[l];
  const double* gpa = lv.geom[l - 1];
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t cg = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); cg < ngroup; cg += nw) {
    const int64_t ch = 16 * cg + q, par = ch >> 3;
    const double dx = gch[ch * 10 + 6] - gpa[par * 10 + 6];
    const double dy = gch[ch * 10 + 7] - gpa[par * 10 + 7];
    const double dz = gch[ch * 10 + 8] - gpa[par * 10 + 8];
    const double rxy2 = dx * dx + dy * dy;
    const double rho = sqrt(rxy2 + dz * dz), rxy = sqrt(rxy2);
    const bool zero = !(rho > 0.0);
    const double ca = zero ? 1.0 : dz / rho, sa = zero ? 0.0 : rxy / rho;
    const double cb = rxy > 0.0 ? dx / rxy : 1.0, sb = rxy > 0.0 ? dy / rxy : 0.0;
    // rho = 2^e mu with mu in [1, 2): the powers of mu stay in range and
    // those of 2^e are exact ldexp scalings, so no partial product leaves the
    // binary64 range unless the scaled coefficient does.  A pair at distance
    // zero translates to zero here; its identity is added below.
    const int e = zero ? 0 : ilogb(rho);
    const double mu = zero ? 0.0 : ldexp(rho, -e);
    const double in_base = zero ? 0.0 : (L2L ? mu : 1.0 / mu);
    const double out_base = zero ? 0.0 : (L2L ? 1.0 / mu : mu);
    const double out_mult = zero ? 0.0 : 1.0;
    const int in_exp = L2L ? e : -e, out_exp = -in_exp;
    const double* src = E + (size_t)(L2L ? lv.gofs[l - 1] + par : lv.gofs[l] + ch) * S;

    double X[NQ];
    qfor<0, NQ>([&](auto rI) __attribute__((always_inline)) {
      const int sp = spos[4 * decltype(rI)::value + k];
      X[decltype(rI)::value] = sp >= 0 ? src[sp] : 0.0;
    });
    FMM_QSTEP(qrotz<P>(X, cb, sb, -1.0, k));
    FMM_QSTEP((qjapply<P, false>(X, tabs + NJ, tl)));
    FMM_QSTEP(qrotz<P>(X, ca, sa, -1.0, k));
    FMM_QSTEP((qjapply<P, false>(X, tabs, tl)));
    FMM_QSTEP((qztrans<P, true>(X, Az, k, in_base, out_base, out_mult, in_exp, out_exp)));
    FMM_QSTEP((qjapply<P, false>(X, tabs + NJ, tl)));
    FMM_QSTEP(qrotz<P>(X, ca, sa, 1.0, k));
    FMM_QSTEP((qjapply<P, false>(X, tabs, tl)));
    FMM_QSTEP(qrotz<P>(X, cb, sb, 1.0, k));
    if (__ballot(zero)) {
      qfor<0, NQ>([&](auto rI) __attribute__((always_inline)) {
        const int sp = spos[4 * decltype(rI)::value + k];
        if (zero && sp >= 0) X[decltype(rI)::value] += src[sp];
      });
    }

    if constexpr (L2L) {
      double* dst = E + (size_t)(lv.gofs[l] + ch) * S;
      qfor<0, NQ>([&](auto rI) __attribute__((always_inline)) {
        const int sp = spos[4 * decltype(rI)::value + k];
        if (sp >= 0) dst[sp] += X[decltype(rI)::value];
      });
    } else {
      // sum over the eight children of each parent (lane bits 0..2)
      double h1[qlvl(NQ, 1)], h2[qlvl(NQ, 2)], h3[qlvl(NQ, 3)];
      qhalve<NQ, qlvl(NQ, 1), 4>(X, h1, lane);
      qhalve<qlvl(NQ, 1), qlvl(NQ, 2), 2>(h1, h2, lane);
      qhalve<qlvl(NQ, 2), qlvl(NQ, 3), 1>(h2, h3, lane);
      // lane's values: registers base + i of phase k of parent 2 cg + (q >> 3)
      int base = 0, len = NQ;
#pragma unroll
      for (int sidx = 1; sidx <= 3; ++sidx) {
        const int half = qlvl(NQ, sidx);
        if (lane & (8 >> sidx)) {
          base += half;
          len = len - half > 0 ? len - half : 0;
        } else {
          len = len < half ? len : half;
        }
      }
      double* dst = E + (size_t)(lv.gofs[l - 1] + 2 * cg + (q >> 3)) * S;
      qfor<0, NF>([&](auto iI) __attribute__((always_inline)) {
        constexpr int i = decltype(iI)::value;
        if (i < len) {
          const int sp = spos[4 * (base + i) + k];
          if (sp >= 0) dst[sp] = h3[i];
        }
      });
      double* pdst = E + (size_t)(lv.gofs[l - 1] + 2 * cg) * S;
      for (int t = lane; t < 2 * S; t += 64)
        if (ipos[t % S] < 0) pdst[t] = 0.0;
    }
  }
}

template <int P, bool L2L>
void launch_one_xlate(const Tree& t, int l, const Tables& tb, double* E, hipStream_t s) {
  const int64_t ngroup = t.lev[l].nbox / 16;
  if (ngroup <= 0) return;
  static const int grid_max = [] {
    int dev = 0, ncu = 0, per = 0;
    HIPCHECK(hipGetDevice(&dev));
    HIPCHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_xlate_quad<P, L2L>, QuadCfg<P>::kThreads, 0));
    return ncu * (per > 0 ? per : 1);
  }();
  const int64_t need = (ngroup + QuadCfg<P>::kThreads / 64 - 1) / (QuadCfg<P>::kThreads / 64);
  const unsigned grid = (unsigned)(need < grid_max ? need : grid_max);
  k_xlate_quad<P, L2L><<<grid, QuadCfg<P>::kThreads, 0, s>>>(t.view(), l, L2L ? tb.quad_l2l : tb.quad_m2m, tb.pos,
                                                              tb.ipos, tb.stride, E, ngroup);
  HIPCHECK(hipGetLastError());
}

template <bool L2L>
bool launch_xlate(const Tree& t, int l, const Tables& tb, double* E, hipStream_t s) {
  switch (tb.p) {
    case 0: launch_one_xlate<0, L2L>(t, l, tb, E, s); break;
    case 1: launch_one_xlate<1, L2L>(t, l, tb, E, s); break;
    case 2: launch_one_xlate<2, L2L>(t, l, tb, E, s); break;
    case 3: launch_one_xlate<3, L2L>(t, l, tb, E, s); break;
    case 4: launch_one_xlate<4, L2L>(t, l, tb, E, s); break;
    case 5: launch_one_xlate<5, L2L>(t, l, tb, E, s); break;
    case 6: launch_one_xlate<6, L2L>(t, l, tb, E, s); break;
    case 7: launch_one_xlate<7, L2L>(t, l, tb, E, s); break;
    case 8: launch_one_xlate<8, L2L>(t, l, tb, E, s); break;
    case 9: launch_one_xlate<9, L2L>(t, l, tb, E, s); break;
    case 10: launch_one_xlate<10, L2L>(t, l, tb, E, s); break;
    case 11: launch_one_xlate<11, L2L>(t, l, tb, E, s); break;
    case 12: launch_one_xlate<12, L2L>(t, l, tb, E, s); break;
    case 13: launch_one_xlate<13, L2L>(t, l, tb, E, s); break;
    default: return false;
  }
  static_assert(kQuadXlateMaxP == 13, "the cases above cover orders 0 .. kQuadXlateMaxP");
  return true;
}

}  // namespace

// binary64 M2L with this kernel: orders up to 13 and 16..20; false for 14
// and 15 (the 16x16 tile kernel is faster there, the two-wave quad kernel
// spills)
bool launch_m2l_quad64(const Tree& t, const Tables& tb, const double* Mx, double* Lx, hipStream_t s) {
  switch (tb.p) {
    case 0: launch_one_quad<0>(t, tb, Mx, Lx, s); break;
    case 1: launch_one_quad<1>(t, tb, Mx, Lx, s); break;
    case 2: launch_one_quad<2>(t, tb, Mx, Lx, s); break;
    case 3: launch_one_quad<3>(t, tb, Mx, Lx, s); break;
    case 4: launch_one_quad<4>(t, tb, Mx, Lx, s); break;
    case 5: launch_one_quad<5>(t, tb, Mx, Lx, s); break;
    case 6: launch_one_quad<6>(t, tb, Mx, Lx, s); break;
    case 7: launch_one_quad<7>(t, tb, Mx, Lx, s); break;
    case 8: launch_one_quad<8>(t, tb, Mx, Lx, s); break;
    case 9: launch_one_quad<9>(t, tb, Mx, Lx, s); break;
    case 10: launch_one_quad<10>(t, tb, Mx, Lx, s); break;
    case 11: launch_one_quad<11>(t, tb, Mx, Lx, s); break;
    case 12: launch_one_quad<12>(t, tb, Mx, Lx, s); break;
    case 13: launch_one_quad<13>(t, tb, Mx, Lx, s); break;
    case 16: launch_one_quad<16>(t, tb, Mx, Lx, s); break;
    case 17: launch_one_quad<17>(t, tb, Mx, Lx, s); break;
    case 18: launch_one_quad<18>(t, tb, Mx, Lx, s); break;
    case 19: launch_one_quad<19>(t, tb, Mx, Lx, s); break;
    case 20: launch_one_quad<20>(t, tb, Mx, Lx, s); break;
    default: return false;
  }
  return true;
}

// M2M from level l into level l - 1, or L2L from level l - 1 into level l,
// four lanes per translation: orders up to kQuadXlateMaxP with the tables
// made; false for the others (the generic translation then runs)
bool launch_m2m_quad64(const Tree& t, int l, const Tables& tb, double* Mx, hipStream_t s) {
  return tb.quad_m2m != nullptr && t.lev[l].nbox % 16 == 0 && launch_xlate<false>(t, l, tb, Mx, s);
}
bool launch_l2l_quad64(const Tree& t, int l, const Tables& tb, double* Lx, hipStream_t s) {
  return tb.quad_l2l != nullptr && t.lev[l].nbox % 16 == 0 && launch_xlate<true>(t, l, tb, Lx, s);
}

}  // namespace fmm
