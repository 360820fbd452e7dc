// M2L for the mixed-precision mode (Algorithm 3, M2L; rotational form of
// Section 2.1.3), one weak pair per lane, at orders p <= 14: binary32 on
// radius-scaled expansions, the fixed operators on the matrix cores.
//
// Every lane of a wave takes one pair of the same target box, 64 pairs at a
// time, and holds its pair's whole expansion in registers in the standard
// order (c_{n,0}, c_{n,1}, s_{n,1}, ..., per degree n).  The translation is
// the same sequence as in the binary64 kernels:
//   Rz(-beta), J^T, Rz(-alpha), J, z-axis translation, J^T, Rz(alpha), J, Rz(beta),
// with J the fixed quarter turn about x (block-diagonal in two parity classes
// per degree) and (alpha, beta) the polar and azimuthal angles of
// d = c_source - c_target.  J, J^T and the z-translation core are the same
// for every pair, so each of their blocks acts on all 64 lanes at once as a
// chain of 4x4x1 matrix instructions (16 blocks of 4 lanes): one instruction
// multiplies four operator rows by one coefficient of every lane, and its
// four results land in that lane's registers -- lane = pair, register = row,
// no data moves between lanes.  The operator values of 16 instructions share
// one register (one block's values broadcast to all blocks, lane_ops.h),
// read from a table in LDS.  Only rows of a block are padded to a multiple
// of 4 (1.17x the algorithmic products at p = 12, against 2.42x for 16x16
// tiles of two degree blocks each).  The z-turns and the radius powers run on
// the vector units.  The 64 pair results are summed across the lanes by
// halving exchanges (a fixed order: deterministic) and the batch sums are
// added in binary64.  The expansions are scaled as for the binary32 tile
// kernel: M~_n = M_n / r_s^n on the way in, so the factors (r_s/rho)^n and
// (r_t/rho)^j / rho stay below one, and the result is unscaled by r_t^-n
// into binary64.
#include <type_traits>

#include "fmm_internal.h"
#include "lane_ops.h"
#include "tile_layout.h"

namespace fmm {
namespace {

__host__ __device__ constexpr int deg_of(int k) {
  int n = 0;
  while ((n + 1) * (n + 1) <= k) ++n;
  return n;
}
// index of c_{n,m} (t = 0) or s_{n,m} (t = 1) in the standard order
__host__ __device__ constexpr int cidx(int n, int m, int t) { return n * n + (m == 0 ? 0 : 2 * m - 1 + t); }
// sizes of the halving exchanges: level 0 holds all NT values, each of the
// six levels keeps the lane's half (rounded up)
__host__ __device__ constexpr int lvl(int nt, int s) {
  int v = nt;
  for (int k = 0; k < s; ++k) v = (v + 1) / 2;
  return v;
}

typedef float f4 __attribute__((ext_vector_type(4)));

// D + A_ab * b on the 16-block 4x4x1 instruction, the A operand of block AB
// broadcast to all blocks: lane 4q + j receives rows i = 0..3 of
// A_AB[i] * b(lane)
template <int AB>
__device__ __forceinline__ f4 mfma_bc(float a, float b, f4 d) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, d, 4, AB, 0);
}

// f(integral_constant<int, I>) for I = B .. E-1, as straight-line code
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Blocks on the matrix cores.  A block of S rows computes
// D_c += Op[4c .. 4c+3][k] x_k over its S inputs x_k = X[in(k)], then sets
// X[in(r)] = row r; its instruction U0 + k * chunks(S) + c takes its operand
// values from group (U0 + ...) / 16 of tab.  Up to four blocks with disjoint
// inputs run in lock-step over k, so that their accumulator chains are
// independent instructions in flight; S = 0 is an absent block.
template <int S, int U0>
struct Blk {
  static constexpr int kS = S;
  static constexpr int kNC = S > 0 ? lops::chunks(S) : 1;
  f4 D[kNC];
  float av = 0.f;
  __device__ __forceinline__ Blk() {
    static_for<0, kNC>([&](auto c) __attribute__((always_inline)) { D[c] = f4{0.f, 0.f, 0.f, 0.f}; });
  }
  template <int K, class In>
  __device__ __forceinline__ void step(const float* X, const float* tab, int lane, In in) {
    if constexpr (K < S) {
      const float xk = X[in(std::integral_constant<int, K>{})];
      static_for<0, kNC>([&](auto c) __attribute__((always_inline)) {
        constexpr int u = U0 + K * kNC + decltype(c)::value;
        if constexpr (u % 16 == 0 || (K == 0 && decltype(c)::value == 0)) av = tab[(u / 16) * 64 + lane];
        D[c] = mfma_bc<u % 16>(av, xk, D[c]);
      });
    }
  }
  template <class In>
  __device__ __forceinline__ void store(float* X, In in) {
    static_for<0, S>([&](auto r) __attribute__((always_inline)) {
      X[in(r)] = D[decltype(r)::value / 4][decltype(r)::value % 4];
    });
  }
};

template <int S0, int U0, int S1, int U1, int S2, int U2, int S3, int U3, class I0, class I1, class I2, class I3>
__device__ __forceinline__ void blocks_mf(float* X, const float* t0, const float* t1, const float* t2,
                                          const float* t3, int lane, I0 in0, I1 in1, I2 in2, I3 in3) {
  constexpr int SM01 = S0 > S1 ? S0 : S1, SM23 = S2 > S3 ? S2 : S3;
  constexpr int SM = SM01 > SM23 ? SM01 : SM23;
  Blk<S0, U0> b0;
  Blk<S1, U1> b1;
  Blk<S2, U2> b2;
  Blk<S3, U3> b3;
  static_for<0, SM>([&](auto k) __attribute__((always_inline)) {
    constexpr int K = decltype(k)::value;
    b0.template step<K>(X, t0, lane, in0);
    b1.template step<K>(X, t1, lane, in1);
    b2.template step<K>(X, t2, lane, in2);
    b3.template step<K>(X, t3, lane, in3);
  });
  b0.store(X, in0);
  b1.store(X, in1);
  b2.store(X, in2);
  b3.store(X, in3);
}

// the class members of degree N (standard indices), and the order-M part T
template <int N, int CLS>
struct JIn {
  template <class R>
  __device__ constexpr int operator()(R) const { return N * N + lops::cls_member(N, CLS, R::value); }
};
template <int M, int T>
struct ZIn {
  template <class R>
  __device__ constexpr int operator()(R) const { return cidx(M + R::value, M, T); }
};

// X <- J X or J^T X on the matrix cores: per degree and parity class, the
// class block times the lane's class members (lane_ops.h), degree n beside
// degree P - n; tab: the operator's groups in LDS
template <int P>
__device__ __forceinline__ void japply_mf(float* X, const float* tab, int lane) {
  static_for<0, P / 2 + 1>([&](auto nI) __attribute__((always_inline)) {
    constexpr int n = decltype(nI)::value, n2 = P - n;
    constexpr bool two = n2 > n;
    constexpr int s2 = two ? lops::cls_size(n2, 0) : 0, s3 = two ? lops::cls_size(n2, 1) : 0;
    blocks_mf<lops::cls_size(n, 0), lops::j_offset(n, 0), lops::cls_size(n, 1), lops::j_offset(n, 1), s2,
              lops::j_offset(n2, 0), s3, lops::j_offset(n2, 1)>(X, tab, tab, tab, tab, lane, JIn<n, 0>{},
                                                                  JIn<n, 1>{}, JIn<n2, 0>{}, JIn<n2, 1>{});
    // a few blocks at a time: bounded registers
    __builtin_amdgcn_sched_barrier(0);
  });
}

// X <- Rz(sign * g) X, with (c1, s1) = (cos g, sin g); the multiples by the
// angle-addition recurrence in binary64
// FRESH: the recurrence is not shared with the other turn by the same angle
// (shared, its 2P binary64 values stay live through the whole translation;
// where registers are short that costs more than running it again)
template <int P, bool FRESH>
__device__ __forceinline__ void rotz(float* X, double c1, double s1, double sign) {
  if constexpr (FRESH) asm volatile("" : "+v"(c1), "+v"(s1));
  double c = 1.0, s = 0.0;
#pragma unroll
  for (int m = 1; m <= P; ++m) {
    const double nc = c * c1 - s * s1, ns = s * c1 + c * s1;
    c = nc;
    s = ns;
    const float cm = (float)c, sm = (float)(sign * s);
#pragma unroll
    for (int n = m; n <= P; ++n) {
      const float a = X[cidx(n, m, 0)], b = X[cidx(n, m, 1)];
      X[cidx(n, m, 0)] = cm * a - sm * b;
      X[cidx(n, m, 1)] = sm * a + cm * b;
    }
  }
}

// the z-axis translation with the core products on the matrix cores: per
// order m the block A[m][d][n] (d, n = m .. P) times the lane's cosine and
// sine parts of order m (one operand table for both)
template <int P>
__device__ __forceinline__ void ztrans_mf(float* X, const float* tab, int lane, float in_base, float out_base,
                                          float out_mult) {
  {
    float w = in_base;
#pragma unroll
    for (int n = 1; n <= P; ++n) {
#pragma unroll
      for (int i = 0; i < 2 * n + 1; ++i) X[n * n + i] *= w;
      w *= in_base;
    }
  }
  // order m beside order P - m, cosine and sine parts each
  static_for<0, P / 2 + 1>([&](auto mI) __attribute__((always_inline)) {
    constexpr int m = decltype(mI)::value, m2 = P - m;
    constexpr bool two = m2 > m;
    constexpr int s1 = m > 0 ? P + 1 - m : 0, s2 = two ? P + 1 - m2 : 0;
    constexpr int s3 = (two && m2 > 0) ? P + 1 - m2 : 0;
    blocks_mf<P + 1 - m, lops::z_offset(P, m), s1, lops::z_offset(P, m), s2, lops::z_offset(P, m2), s3,
              lops::z_offset(P, m2)>(
        X, tab, tab, tab, tab, lane, ZIn<m, 0>{}, ZIn<m, 1>{}, ZIn<m2, 0>{}, ZIn<m2, 1>{});
    __builtin_amdgcn_sched_barrier(0);
  });
  float w = out_mult;
#pragma unroll
  for (int d = 0; d <= P; ++d) {
#pragma unroll
    for (int i = 0; i < 2 * d + 1; ++i) X[d * d + i] *= w;
    w *= out_base;
  }
}

// One halving exchange of the sum over the lanes, ND = ceil(NS / 2): dst[i]
// = src[i] of this lane and of its partner at lane distance D (lanes with
// bit D clear) or src[ND + i] of both (bit set); the upper half of an odd
// count is padded with zero.  Distances 32 and 16 are permlane swaps (the swap of (lower,
// upper) leaves each lane the two terms of its own sum), 8, 2 and 1 a DPP
// read of the partner, 4 two DPP shifts.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}
template <int NS, int D>
__device__ __forceinline__ void halve(const float* src, float* dst, int lane) {
  constexpr int ND = (NS + 1) / 2;
  const bool up = (lane & D) != 0;
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    const float lo = src[i];
    const float hi = ND + i < NS ? src[ND + i] : 0.f;
    if constexpr (D == 32 || D == 16) {
      const auto r = D == 32 ? __builtin_amdgcn_permlane32_swap(__float_as_uint(lo), __float_as_uint(hi), false, false)
                             : __builtin_amdgcn_permlane16_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
      dst[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    } else if constexpr (D == 4) {
      // row_shl:4 reads lane + 4, row_shr:4 lane - 4 (within rows of 16)
      const float t0 = lo + dpp<0x104>(lo), t1 = hi + dpp<0x114>(hi);
      dst[i] = up ? t1 : t0;
    } else {
      // the partner lane^D: row_ror:8, quad_perm [2,3,0,1], [1,0,3,2]
      constexpr int C = D == 8 ? 0x128 : D == 2 ? 0x4E : 0xB1;
      const float send = up ? lo : hi, keep = up ? hi : lo;
      dst[i] = keep + dpp<C>(send);
    }
    if ((i & 7) == 7) __builtin_amdgcn_sched_barrier(0);  // a few in flight: bounded registers
  }
}

__device__ __forceinline__ int level_of3(const LevelView& lv, int64_t gid) {
  int l = 0;
  while (l < lv.L && gid >= lv.gofs[l + 1]) ++l;
  return l;
}

// Waves per SIMD: 2 up to order 12 (256 registers; at orders 11 and 12 a
// few values spill, which costs less than halving the waves), 1 above.
// kFresh (the z-turns recompute their recurrence) from order 11: measured on
// 2^24 Plummer points, sharing it is 2 % faster at order 10 and 2 % and 22 %
// slower at 11 and 12.
template <int P>
struct LaneCfg {
  static constexpr int kWaves = P <= 12 ? 2 : 1;
  static constexpr bool kFresh = kWaves == 2 && P >= 11;
};

// Persistent waves: each takes the next target of the longest-first order.
template <int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(LaneCfg<P>::kWaves, LaneCfg<P>::kWaves))) void
k_m2l_lane(LevelView lv, const float* __restrict__ ltab, const int* __restrict__ pos, const float* __restrict__ Mf,
           double* __restrict__ Lx, int64_t ntarget, const int32_t* __restrict__ order, int* __restrict__ queue) {
  constexpr int NT = (P + 1) * (P + 1);
  constexpr int S = tl::stride(P);
  constexpr int SD = lops::dense_stride(P);
  constexpr int NF = lvl(NT, 6);  // values a lane holds after the exchanges
  constexpr bool FR = LaneCfg<P>::kFresh;
  constexpr int GJ = 64 * lops::groups(lops::n_j(P));  // table: J, J^T, z core
  __shared__ float tabs[lops::table_floats(P)];
  for (int i = threadIdx.x; i < lops::table_floats(P); i += blockDim.x) tabs[i] = ltab[i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  for (;;) {
    int kq = 0;
    if (lane == 0) kq = atomicAdd(queue, 1);
    kq = __builtin_amdgcn_readfirstlane(kq);  // uniform: the target's values in scalar registers
    if (kq >= ntarget) break;
    const int64_t gid = lv.gofs[1] + order[kq];
    const int l = level_of3(lv, gid);
    const int64_t bi = gid - lv.gofs[l];
    const double* geo = lv.geom[l];
    const double cix = geo[bi * 10 + 6], ciy = geo[bi * 10 + 7], ciz = geo[bi * 10 + 8];
    const double rt = geo[bi * 10 + 9] > 0.0 ? geo[bi * 10 + 9] : 1.0;
    const int64_t e0 = lv.w_off[l][bi], e1 = lv.w_off[l][bi + 1];
    const int32_t* widx = lv.w_idx[l];
    const float* Mlev = Mf + (size_t)lv.gofs[l] * SD;
    double acc[NF];
#pragma unroll
    for (int i = 0; i < NF; ++i) acc[i] = 0.0;

    for (int64_t eb = e0; eb < e1; eb += 64) {
      const int64_t e = eb + lane;
      const bool valid = e < e1;
      const int64_t j = widx[valid ? e : e0];
      const double dx = geo[j * 10 + 6] - cix, dy = geo[j * 10 + 7] - ciy, dz = geo[j * 10 + 8] - ciz;
      const double rs = geo[j * 10 + 9] > 0.0 ? geo[j * 10 + 9] : 1.0;
      const double rxy2 = dx * dx + dy * dy;
      const double rho = sqrt(rxy2 + dz * dz), rxy = sqrt(rxy2);
      const double irho = 1.0 / rho;
      const double ca = dz * irho, sa = rxy * irho;
      const double cb = rxy > 0.0 ? dx / rxy : 1.0, sb = rxy > 0.0 ? dy / rxy : 0.0;
      // a lane past the end of the list translates the first source with zero factors
      const float in_base = valid ? (float)(rs * irho) : 0.f;
      const float out_base = valid ? (float)(rt * irho) : 0.f;
      const float out_mult = valid ? (float)irho : 0.f;

      float X[NT];
      const float4* src = (const float4*)(Mlev + (size_t)j * SD);
#pragma unroll
      for (int q = 0; q < SD / 4; ++q) {
        const float4 v = src[q];
        if (4 * q + 0 < NT) X[4 * q + 0] = v.x;
        if (4 * q + 1 < NT) X[4 * q + 1] = v.y;
        if (4 * q + 2 < NT) X[4 * q + 2] = v.z;
        if (4 * q + 3 < NT) X[4 * q + 3] = v.w;
      }

      // the steps are kept apart in the schedule (interleaving them only
      // raises the number of live values)
#define FMM_STEP(x)                      \
  x;                                     \
  __builtin_amdgcn_sched_barrier(0)
      FMM_STEP((rotz<P, FR>(X, cb, sb, -1.0)));
      FMM_STEP(japply_mf<P>(X, tabs + GJ, lane));
      FMM_STEP((rotz<P, FR>(X, ca, sa, -1.0)));
      FMM_STEP(japply_mf<P>(X, tabs, lane));
      FMM_STEP(ztrans_mf<P>(X, tabs + 2 * GJ, lane, in_base, out_base, out_mult));
      FMM_STEP(japply_mf<P>(X, tabs + GJ, lane));
      FMM_STEP((rotz<P, FR>(X, ca, sa, 1.0)));
      FMM_STEP(japply_mf<P>(X, tabs, lane));
      FMM_STEP((rotz<P, FR>(X, cb, sb, 1.0)));
#undef FMM_STEP

      // sum over the 64 lanes: six halving exchanges; at the exchange with
      // lane distance d the lanes with bit d clear keep the lower half
      float h1[lvl(NT, 1)], h2[lvl(NT, 2)], h3[lvl(NT, 3)], h4[lvl(NT, 4)], h5[lvl(NT, 5)], h6[lvl(NT, 6)];
      halve<NT, 32>(X, h1, lane);
      halve<lvl(NT, 1), 16>(h1, h2, lane);
      halve<lvl(NT, 2), 8>(h2, h3, lane);
      halve<lvl(NT, 3), 4>(h3, h4, lane);
      halve<lvl(NT, 4), 2>(h4, h5, lane);
      halve<lvl(NT, 5), 1>(h5, h6, lane);
#pragma unroll
      for (int i = 0; i < NF; ++i) acc[i] += (double)h6[i];
    }
    // lane's values: standard index base + i, where each exchange added the
    // kept half's offset; entries past a half's end are padding
    int base = 0, len = NT;
#pragma unroll
    for (int sidx = 1; sidx <= 6; ++sidx) {
      const int half = lvl(NT, sidx);
      const int dist = 64 >> sidx;
      if (lane & dist) {
        base += half;
        len = len - half > 0 ? len - half : 0;
      } else {
        len = len < half ? len : half;
      }
    }
    double* dst = Lx + (size_t)gid * S;
    const double irt = 1.0 / rt;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      if (i >= len) continue;
      const int k = base + i;
      const int n = deg_of(k);
      double v = acc[i];
      for (int q = 0; q < n; ++q) v *= irt;
      dst[pos[k]] = v;
    }
  }
}

// The binary32 multipoles of levels 1..L for this kernel, from the binary64
// ones (tile layout, S per box): standard order, scaled by r^-n (r the box
// radius, 1 for a box of zero extent; the same products as for the tile
// kernel's copy), lops::dense_stride(P) floats per box with a zero tail.
template <int P>
__global__ void k_scale_lane(LevelView lv, int S, const int* __restrict__ pos, const double* __restrict__ Mx,
                             float* __restrict__ Mf, int64_t nbox_total) {
  constexpr int NT = (P + 1) * (P + 1), SD = lops::dense_stride(P);
  const int64_t gid = 1 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (gid >= nbox_total) return;
  int l = 1;
  while (l < lv.L && gid >= lv.gofs[l + 1]) ++l;
  const double r = lv.geom[l][(gid - lv.gofs[l]) * 10 + 9];
  const double is = r > 0.0 ? 1.0 / r : 1.0;
  for (int k = threadIdx.x & 63; k < SD; k += 64) {
    float v = 0.f;
    if (k < NT) {
      const int n = deg_of(k);
      double d = Mx[(size_t)gid * S + pos[k]];
      for (int q = 0; q < n; ++q) d *= is;
      v = (float)d;
    }
    Mf[(size_t)gid * SD + k] = v;
  }
}

__global__ void k_zero_queue_l(int* queue) {
  if (threadIdx.x == 0) *queue = 0;
}

template <int P>
void launch_one_lane(const Tree& t, const Tables& tb, const double* Mx, double* Lx, hipStream_t s) {
  const int64_t ntarget = t.nbox_total - 1;
  if (ntarget <= 0) return;
  float* Mf = (float*)dalloc((size_t)t.nbox_total * lops::dense_stride(P) * sizeof(float), s);
  k_scale_lane<P><<<(unsigned)((ntarget + 3) / 4), 256, 0, s>>>(t.view(), tb.stride, tb.pos, Mx, Mf, t.nbox_total);
  HIPCHECK(hipGetLastError());
  static const int grid_max = [] {
    int dev = 0, ncu = 0, per = 0;
    HIPCHECK(hipGetDevice(&dev));
    HIPCHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_m2l_lane<P>, 256, 0));
    return ncu * (per > 0 ? per : 1);
  }();
  const int64_t need = (ntarget + 3) / 4;
  const unsigned grid = (unsigned)(need < grid_max ? need : grid_max);
  int* queue = (int*)dalloc(sizeof(int), s);
  k_zero_queue_l<<<1, 64, 0, s>>>(queue);
  HIPCHECK(hipGetLastError());
  k_m2l_lane<P><<<grid, 256, 0, s>>>(t.view(), tb.lane, tb.pos, Mf, Lx, ntarget, t.m2l_order, queue);
  HIPCHECK(hipGetLastError());
  dfree(queue, s);
  dfree(Mf, s);
}

}  // namespace

// mixed-precision M2L with this kernel from the binary64 multipoles Mx (tile
// layout); false above order 14, where the 16x16 tile kernel is as fast
bool launch_m2l_lane32(const Tree& t, const Tables& tb, const double* Mx, double* Lx, hipStream_t s) {
  switch (tb.p) {
    case 0: launch_one_lane<0>(t, tb, Mx, Lx, s); break;
    case 1: launch_one_lane<1>(t, tb, Mx, Lx, s); break;
    case 2: launch_one_lane<2>(t, tb, Mx, Lx, s); break;
    case 3: launch_one_lane<3>(t, tb, Mx, Lx, s); break;
    case 4: launch_one_lane<4>(t, tb, Mx, Lx, s); break;
    case 5: launch_one_lane<5>(t, tb, Mx, Lx, s); break;
    case 6: launch_one_lane<6>(t, tb, Mx, Lx, s); break;
    case 7: launch_one_lane<7>(t, tb, Mx, Lx, s); break;
    case 8: launch_one_lane<8>(t, tb, Mx, Lx, s); break;
    case 9: launch_one_lane<9>(t, tb, Mx, Lx, s); break;
    case 10: launch_one_lane<10>(t, tb, Mx, Lx, s); break;
    case 11: launch_one_lane<11>(t, tb, Mx, Lx, s); break;
    case 12: launch_one_lane<12>(t, tb, Mx, Lx, s); break;
    case 13: launch_one_lane<13>(t, tb, Mx, Lx, s); break;
    case 14: launch_one_lane<14>(t, tb, Mx, Lx, s); break;
    default: return false;
  }
  return true;
}

}  // namespace fmm
