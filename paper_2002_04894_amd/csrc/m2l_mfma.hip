// M2L on the matrix cores (Algorithm 3, M2L; rotational form of Section
// 2.1.3), for expansion orders p <= 15, in FP64 (v_mfma_f64_16x16x4f64).
//
// One wave computes the local expansion of one target box i:
//   L_i = sum over weak pairs j of  O(Q)^T Z(rho) O(Q) M_j,
// where Q turns d = c_j - c_i onto the +z axis.  With K the quarter turn
// about y and J = O(K) (fixed; block-diagonal in the cosine/sine blocks),
// Q = Rx(alpha) Rz(pi/2 - beta) and Rx(g) = K Rz(g) K^T give
//   O(Q) = J Rz(alpha) J^T Rz(theta),  theta = pi/2 - beta,
// alpha, beta the polar and azimuthal angles of d.  The sign flip
// D = diag((-1)^m) is the z-turn by pi and satisfies J^T = D J D, so only J
// is needed:
//   O(Q)   = J Rz(alpha + pi) J Rz(theta + pi),
//   O(Q)^T = D Rz(-theta - pi) J Rz(-alpha - pi) J D,
// and the last D (a fixed sign per coefficient) is applied once per target
// after the sum over pairs; the inner D turns the z-axis translation sign
// (-1)^(n+m) into (-1)^n:
//   L'_{j,m} = sum_n (-1)^n (n+j)! u_{n,m} u_{j,m} rho^-(n+j+1) M'_{n,m},
//   u_{n,m} = 1/sqrt((n+m)!(n-m)!).
// The weak list is taken 16 pairs at a time: the coefficients of the 16 pairs
// are the columns of 16x16 tiles (tile_layout.h), so each J product is one
// MFMA chain per tile with the same fixed operand for every pair, and its
// result is already laid out as the next operand.  z-rotations act lane by
// lane on (cosine, sine) partners.  For the z translation the coefficients
// are moved to order-major rows through LDS; per order m it is a fixed
// matrix (factorials and u folded in) between two diagonal scalings by
// powers of 1/rho.  The 16 pair results of a batch are summed through LDS
// into one accumulator per coefficient: no atomics, deterministic.
#include "fmm_internal.h"
#include "tile_layout.h"

namespace fmm {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

// Orders this wave's LDS accesses around a point (other lanes of the wave
// read what this lane wrote): a compiler barrier only, since the LDS unit
// executes one wave's instructions in order.
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int P>
struct Cfg {
  static constexpr int T = tl::ntiles(P);
  static constexpr int NP = tl::npairs(P);
  static constexpr int S = tl::stride(P);
  static constexpr int ZR = tl::zrows(P);
  static constexpr int H = tl::hoff(P, P + 1);
  // z buffer rows: ZR coefficient rows, then a write-only row (also read past
  // the last order by the zero-padded tail of its last k-step), two more such
  // rows, and a row that stays zero
  static constexpr int ZDUMMY = ZR;
  static constexpr int ZZERO = ZR + 3;
  static constexpr int RSTRIDE = 18;  // row stride of the pair-sum buffer (no bank conflicts)
  // the pair-sum rounds reuse the z buffer
  static constexpr int ZBUF = 16 * (ZR + 4) > 64 * RSTRIDE ? 16 * (ZR + 4) : 64 * RSTRIDE;
  // per pair: (cos, sin)(m (theta + pi)), (cos, sin)(m (alpha + pi)), m = 0..P
  static constexpr int TRIG = 4 * (P + 1);
  static constexpr int SHARED = T * 256 + H * 64;
  static constexpr int PERWAVE = 16 * TRIG + ZBUF;
  static constexpr int LDS = SHARED + 4 * PERWAVE;
  static constexpr int NR = (T + 3) / 4;  // pair-sum rounds of four tiles
};

__device__ __forceinline__ int level_of2(const LevelView& lv, int64_t gid) {
  int l = 0;
  while (l < lv.L && gid >= lv.gofs[l + 1]) ++l;
  return l;
}

// order m of slot s of tile t, clamped to P for padding slots
template <int P>
__device__ __forceinline__ int slot_m(int t, int s) {
  constexpr int NP = tl::npairs(P);
  int m;
  if (t < 2 * NP) {
    const int a = t < NP ? t : t - NP;
    m = s <= a ? s : s - a - 1;
  } else if (tl::has_mixed(P) && t == tl::mixed_tile(P)) {
    m = s < 8 ? s : s - 8;
  } else {
    m = s;
  }
  return m < P ? m : P;
}

// 1 if register i of tile t holds sine-block slots (fixed per (t, i))
template <int P>
__host__ __device__ constexpr int reg_sine(int t, int i) {
  constexpr int NP = tl::npairs(P);
  if (t < NP) return 0;
  if (t < 2 * NP) return 1;
  if (tl::has_mixed(P) && t == tl::mixed_tile(P)) return i >= 2 ? 1 : 0;
  return t == tl::top_s(P) ? 1 : 0;
}

// (c, s) <- (cos c - sgn sin s, sgn sin c + cos s) for every (cosine, sine)
// partner pair; cs points at the (cos m g, sin m g) pairs of this lane's pair
template <int P>
__device__ __forceinline__ void rotz(d4* st, const double* cs, double sgn, int g) {
  constexpr int NP = tl::npairs(P);
  auto rot = [&](double& c, double& s, int m) {
    const d2 v = *(const d2*)(cs + 2 * m);
    const double co = v.x, si = sgn * v.y;
    const double nc = co * c - si * s;
    const double ns = si * c + co * s;
    c = nc;
    s = ns;
  };
#pragma unroll
  for (int a = 0; a < NP; ++a) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double c = st[a][i], s = st[NP + a][i];
      rot(c, s, slot_m<P>(a, 4 * i + g));
      st[a][i] = c;
      st[NP + a][i] = s;
    }
  }
  if constexpr (tl::has_mixed(P)) {
    constexpr int t = tl::mixed_tile(P);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      double c = st[t][i], s = st[t][i + 2];
      rot(c, s, slot_m<P>(t, 4 * i + g));
      st[t][i] = c;
      st[t][i + 2] = s;
    }
  }
  {
    constexpr int tc = tl::top_c(P), ts = tl::top_s(P);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double c = st[tc][i], s = st[ts][i];
      rot(c, s, slot_m<P>(tc, 4 * i + g));
      st[tc][i] = c;
      st[ts][i] = s;
    }
  }
}

// st[t] <- J_t st[t] for every tile; jf holds the operand fragments
template <int P>
__device__ __forceinline__ void japply(d4* st, const double* jf, int lane) {
  constexpr int T = tl::ntiles(P);
#pragma unroll
  for (int t = 0; t < T; ++t) {
    d4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 4; ++k) d = mfma(jf[(t * 4 + k) * 64 + lane], st[t][k], d);
    st[t] = d;
  }
}

// z-buffer row of slot s of tile t: the row (m, n) of a coefficient, or
// `other` for a padding slot or an always-zero sine slot
template <int P>
__device__ __forceinline__ int zrow(int t, int s, int other) {
  const tl::Slot d = tl::decode(P, t, s);
  return d.valid ? tl::zoff(P, d.m) + d.n - d.m : other;
}

// z-axis translation of the cosine (SINE = 0) or sine blocks
template <int P, int SINE>
__device__ __forceinline__ void ztrans_part(d4* st, double* zb, const double* hf, double ir, int lane) {
  using C = Cfg<P>;
  constexpr int T = C::T;
  const int r16 = lane & 15, g = lane >> 4;
  // to order-major rows
#pragma unroll
  for (int t = 0; t < T; ++t) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (reg_sine<P>(t, i) != SINE) continue;
      zb[zrow<P>(t, 4 * i + g, C::ZDUMMY) * 16 + r16] = st[t][i];
    }
  }
  wave_lds_fence();
  // per order m: L'(m + a) = ir^(m + a + 1) sum_b H_m[a][b] ir^(m + b) M'(m + b)
  double irg = 1.0;  // ir^g
  for (int k = 0; k < g; ++k) irg *= ir;
  const double ir2 = ir * ir, ir4 = ir2 * ir2;
  double pm = SINE ? ir : 1.0;  // ir^m
#pragma unroll
  for (int m = SINE; m <= P; ++m) {
    const int K = P + 1 - m;
    const int zo = tl::zoff(P, m);
    const int ho = tl::hoff(P, m);
    d4 d = {0.0, 0.0, 0.0, 0.0};
    double w = pm * irg;  // ir^(m + 4k + g)
#pragma unroll
    for (int k = 0; k < tl::hsteps(P, m); ++k) {
      const double bv = zb[(zo + 4 * k + g) * 16 + r16] * w;
      d = mfma(hf[(ho + k) * 64 + lane], bv, d);
      w *= ir4;
    }
    double wo = pm * irg * ir;  // ir^(m + 4i + g + 1)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (4 * i < K) {
        const int row = (4 * i + 3 < K || 4 * i + g < K) ? zo + 4 * i + g : C::ZDUMMY;
        zb[row * 16 + r16] = d[i] * wo;
      }
      wo *= ir4;
    }
    pm *= ir;
  }
  wave_lds_fence();
  // back to tiles
#pragma unroll
  for (int t = 0; t < T; ++t) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (reg_sine<P>(t, i) != SINE) continue;
      st[t][i] = zb[zrow<P>(t, 4 * i + g, C::ZZERO) * 16 + r16];
    }
  }
  wave_lds_fence();
}

template <int P>
__global__ __launch_bounds__(256, 1) void k_m2l_mfma(LevelView lv, const double* __restrict__ mtab,
                                                     const double* __restrict__ Mx, double* __restrict__ Lx,
                                                     int64_t ntarget, const int32_t* __restrict__ order,
                                                     int* __restrict__ queue) {
  using C = Cfg<P>;
  constexpr int T = C::T;
  constexpr int S = C::S;
  __shared__ double smem[C::LDS];
  const double* jf = smem;
  const double* hf = smem + T * 256;
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r16 = lane & 15, g = lane >> 4;
  double* trig = smem + C::SHARED + wid * C::PERWAVE;
  double* zb = trig + 16 * C::TRIG;
  // every LDS word starts finite: buffer tails are read (and multiplied by 0)
  for (int k = threadIdx.x; k < C::LDS; k += 256) smem[k] = k < C::SHARED ? mtab[k] : 0.0;
  __syncthreads();

  double* tp = trig + r16 * C::TRIG;  // this lane's pair
  const double* cs_t = tp;
  const double* cs_a = tp + 2 * (P + 1);
  // the coefficient each lane accumulates in round r: slot lane % 16 of tile
  // 4 r + lane / 16, stored with the sign (-1)^m of the final D
  double sgn_out[C::NR];
#pragma unroll
  for (int r = 0; r < C::NR; ++r) {
    const int t = 4 * r + (lane >> 4);
    const tl::Slot d = tl::decode(P, t < T ? t : 0, lane & 15);
    sgn_out[r] = (d.m & 1) ? -1.0 : 1.0;
  }

  // persistent waves: each takes the next target of the longest-first order
  // until the queue is empty (no block-wide barrier below this point)
  for (;;) {
    int k_next = 0;
    if (lane == 0) k_next = atomicAdd(queue, 1);
    k_next = __shfl(k_next, 0);
    if (k_next >= ntarget) break;
    const int64_t tgt = order[k_next];
    const int64_t gid = lv.gofs[1] + tgt;
    const int l = level_of2(lv, gid);
    const int64_t bi = gid - lv.gofs[l];
    const double* geo = lv.geom[l];
    const double cix = geo[bi * 10 + 6], ciy = geo[bi * 10 + 7], ciz = geo[bi * 10 + 8];
    const int64_t e0 = lv.w_off[l][bi], e1 = lv.w_off[l][bi + 1];
    const int32_t* widx = lv.w_idx[l];
    const double* Mlev = Mx + (size_t)lv.gofs[l] * S;

    double acc[C::NR];
#pragma unroll
    for (int r = 0; r < C::NR; ++r) acc[r] = 0.0;

    for (int64_t eb = e0; eb < e1; eb += 16) {
      // pair of this lane's column; past the end of the list the column
      // repeats the first source with 1/rho = 0, which zeroes its result
      const int64_t e = eb + r16;
      const bool valid = e < e1;
      const int j = widx[valid ? e : e0];
      double dx = geo[(int64_t)j * 10 + 6] - cix, dy = geo[(int64_t)j * 10 + 7] - ciy,
             dz = geo[(int64_t)j * 10 + 8] - ciz;
      if (!valid) {
        dx = 0.0;
        dy = 0.0;
        dz = 1.0;
      }
      const double rxy2 = dx * dx + dy * dy;
      const double rho = sqrt(rxy2 + dz * dz), rxy = sqrt(rxy2);
      const double ir = valid ? 1.0 / rho : 0.0;
      // (cos, sin)(m (angle + pi)) by the angle-addition recurrence; lane
      // groups 0, 2 build the theta table and 1, 3 the alpha table (groups 2
      // and 3 write the same values to the same words as 0 and 1)
      {
        const bool ta = (g & 1) != 0;
        const double c1 = ta ? -dz / rho : (rxy > 0.0 ? -dy / rxy : 0.0);
        const double s1 = ta ? -rxy / rho : (rxy > 0.0 ? -dx / rxy : -1.0);
        double* dst = tp + (ta ? 2 * (P + 1) : 0);
        double c = 1.0, s = 0.0;
#pragma unroll
        for (int m = 0; m <= P; ++m) {
          *(d2*)(dst + 2 * m) = d2{c, s};
          const double nc = c * c1 - s * s1, ns = s * c1 + c * s1;
          c = nc;
          s = ns;
        }
      }
      d4 st[T];
      const double* src = Mlev + (size_t)j * S + 4 * g;
#pragma unroll
      for (int t = 0; t < T; ++t) st[t] = *(const d4*)(src + 16 * t);
      wave_lds_fence();

      rotz<P>(st, cs_t, 1.0, g);
      japply<P>(st, jf, lane);
      rotz<P>(st, cs_a, 1.0, g);
      japply<P>(st, jf, lane);
      ztrans_part<P, 0>(st, zb, hf, ir, lane);
      ztrans_part<P, 1>(st, zb, hf, ir, lane);
      japply<P>(st, jf, lane);
      rotz<P>(st, cs_a, -1.0, g);
      japply<P>(st, jf, lane);
      rotz<P>(st, cs_t, -1.0, g);

      // sum over the 16 pairs: four tiles per round through LDS; lane L adds
      // up row L (slot L % 16 of tile 4 r + L / 16)
#pragma unroll
      for (int r = 0; r < C::NR; ++r) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int t = 4 * r + q;
          if (t >= T) continue;
#pragma unroll
          for (int i = 0; i < 4; ++i) zb[(q * 16 + 4 * i + g) * C::RSTRIDE + r16] = st[t][i];
        }
        wave_lds_fence();
        if (4 * r + 3 < T || 4 * r + (lane >> 4) < T) {
          const double* row = zb + lane * C::RSTRIDE;
          d2 v = *(const d2*)row;
#pragma unroll
          for (int k = 1; k < 8; ++k) v += *(const d2*)(row + 2 * k);
          acc[r] += v.x + v.y;
        }
        wave_lds_fence();
      }
    }
    double* dst = Lx + (size_t)gid * S;
#pragma unroll
    for (int r = 0; r < C::NR; ++r) {
      const int t = 4 * r + (lane >> 4);
      if (t < T) dst[tl::spos(t, lane & 15)] = sgn_out[r] * acc[r];
    }
  }
}

template <int P>
void launch_one(const Tree& t, const Tables& tb, const double* Mx, double* Lx, hipStream_t s) {
  const int64_t ntarget = t.nbox_total - 1;
  static int grid_max = 0;  // resident blocks of this instantiation on the device
  if (grid_max == 0) {
    int dev = 0, ncu = 0, per = 0;
    HIPCHECK(hipGetDevice(&dev));
    HIPCHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_m2l_mfma<P>, 256, 0));
    grid_max = ncu * (per > 0 ? per : 1);
  }
  const int64_t need = (ntarget + 3) / 4;
  const unsigned grid = (unsigned)(need < grid_max ? need : grid_max);
  int* queue = (int*)dalloc(sizeof(int), s);
  HIPCHECK(hipMemsetAsync(queue, 0, sizeof(int), s));
  k_m2l_mfma<P><<<grid, 256, 0, s>>>(t.view(), tb.mtab, Mx, Lx, ntarget, t.m2l_order, queue);
  HIPCHECK(hipGetLastError());
  dfree(queue, s);
}

}  // namespace

bool launch_m2l_mfma(const Tree& t, const Tables& tb, const double* Mx, double* Lx, hipStream_t s) {
  if (!tb.tiled) return false;
  switch (tb.p) {
    case 0: launch_one<0>(t, tb, Mx, Lx, s); break;
    case 1: launch_one<1>(t, tb, Mx, Lx, s); break;
    case 2: launch_one<2>(t, tb, Mx, Lx, s); break;
    case 3: launch_one<3>(t, tb, Mx, Lx, s); break;
    case 4: launch_one<4>(t, tb, Mx, Lx, s); break;
    case 5: launch_one<5>(t, tb, Mx, Lx, s); break;
    case 6: launch_one<6>(t, tb, Mx, Lx, s); break;
    case 7: launch_one<7>(t, tb, Mx, Lx, s); break;
    case 8: launch_one<8>(t, tb, Mx, Lx, s); break;
    case 9: launch_one<9>(t, tb, Mx, Lx, s); break;
    case 10: launch_one<10>(t, tb, Mx, Lx, s); break;
    case 11: launch_one<11>(t, tb, Mx, Lx, s); break;
    case 12: launch_one<12>(t, tb, Mx, Lx, s); break;
    case 13: launch_one<13>(t, tb, Mx, Lx, s); break;
    case 14: launch_one<14>(t, tb, Mx, Lx, s); break;
    case 15: launch_one<15>(t, tb, Mx, Lx, s); break;
    default: return false;
  }
  return true;
}

}  // namespace fmm
