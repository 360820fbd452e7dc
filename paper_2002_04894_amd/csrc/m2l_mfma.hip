// M2L on the matrix cores (Algorithm 3, M2L; rotational form of Section
// 2.1.3), for expansion orders p <= 15, in FP64 (v_mfma_f64_16x16x4f64).
//
// One wave computes the local expansion of one target box i:
//   L_i = sum over weak pairs j of  O(Q)^T Z(rho) O(Q) M_j,
// where Q turns d = c_j - c_i onto the +z axis.  With K the quarter turn
// about y and J = O(K) (fixed, block-diagonal in the cosine/sine blocks),
// Q = Rx(alpha) Rz(pi/2 - beta) and Rx(g) = K Rz(g) K^T give
//   O(Q)   = J Rz(alpha) J^T Rz(pi/2 - beta),
//   O(Q)^T = Rz(beta - pi/2) J Rz(-alpha) J^T,
// with alpha, beta the polar and azimuthal angles of d.  The weak list is
// taken 16 pairs at a time: the coefficients of the 16 pairs form the
// columns of 16x16 tiles (see tile_layout.h), so every J or J^T product is
// one MFMA chain per tile with the same fixed matrix for all pairs, and each
// MFMA result is already laid out as the next MFMA operand.  z-rotations act
// lane by lane on (cosine, sine) partners.  The z-axis translation
//   L'_{j,m} = sum_n (-1)^(n+m) (n+j)! u_{n,m} u_{j,m} rho^-(n+j+1) M'_{n,m},
//   u_{n,m} = 1/sqrt((n+m)!(n-m)!),
// is a Hankel product H_{ab} = (a+b+2m)! between diagonal scalings; the
// coefficients are transposed to order-major rows through LDS for it.  The
// 16 per-pair results are summed in registers and reduced across lanes once
// per target: no atomics, deterministic.
#include "fmm_internal.h"
#include "tile_layout.h"

namespace fmm {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): this wave's LDS traffic has landed
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// sum over the 16 lanes of a DPP row (the 16 pair columns), by rotations
template <int CTRL>
__device__ __forceinline__ double dpp_ror(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double row_sum16(double v) {
  v += dpp_ror<0x128>(v);  // row_ror:8
  v += dpp_ror<0x124>(v);  // row_ror:4
  v += dpp_ror<0x122>(v);  // row_ror:2
  v += dpp_ror<0x121>(v);  // row_ror:1
  return v;
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
  // (cos,sin)(m alpha), (cos,sin)(m theta2), rho^-k; even, so (cos,sin) pairs are 16-byte aligned
  static constexpr int TRIG = 4 * (P + 1) + (P + 2) + ((P + 2) & 1);
  static constexpr int SHARED = T * 272 + 32 + 256;
  static constexpr int PERWAVE = 16 * TRIG + 16 * ZR;
  static constexpr int LDS = SHARED + 4 * PERWAVE;
};

__device__ __forceinline__ int level_of2(const LevelView& lv, int64_t gid) {
  int l = 0;
  while (l < lv.L && gid >= lv.gofs[l + 1]) ++l;
  return l;
}

// order m of slot (4i + g) of tile t
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

// (c, s) <- (cos c - sgn sin s, sgn sin c + cos s) for every (cosine, sine)
// partner pair; cs points at (cos m g, sin m g) pairs of this lane's pair
template <int P>
__device__ __forceinline__ void rotz(d4* st, const double* cs, double sgn, int g) {
  constexpr int NP = tl::npairs(P);
  auto rot = [&](double& c, double& s, int m) {
    const double co = cs[2 * m], si = sgn * cs[2 * m + 1];
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

// st[t] <- W_t st[t] (TR = false) or W_t^T st[t] (TR = true) for every tile
template <int P, bool TR>
__device__ __forceinline__ void japply(d4* st, const double* Jt, int r16, int g) {
  constexpr int T = tl::ntiles(P);
#pragma unroll
  for (int t = 0; t < T; ++t) {
    d4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const double a = TR ? Jt[t * 272 + (4 * s + g) * 17 + r16] : Jt[t * 272 + r16 * 17 + 4 * s + g];
      d = mfma(a, st[t][s], d);
    }
    st[t] = d;
  }
}

// z-axis M2L of one part (cosine or sine blocks) through the LDS buffer zb
template <int P, int SINE>
__device__ __forceinline__ void ztrans_part(d4* st, double* zb, const double* fct, const double* uz,
                                            const double* rp, int r16, int g) {
  constexpr int T = tl::ntiles(P);
  // scatter into order-major rows, scaled by (-1)^n u_{n,m} rho^-n
#pragma unroll
  for (int t = 0; t < T; ++t) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const tl::Slot d = tl::decode(P, t, 4 * i + g);
      if (d.valid && d.sine == SINE) {
        const double sc = ((d.n & 1) ? -1.0 : 1.0) * uz[16 * d.m + d.n] * rp[d.n];
        zb[(tl::zoff(P, d.m) + d.n - d.m) * 16 + r16] = st[t][i] * sc;
      }
    }
  }
  wave_lds_sync();
#pragma unroll
  for (int m = SINE; m <= P; ++m) {
    const int K = P + 1 - m;
    const int zo = tl::zoff(P, m);
    d4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < (K + 3) / 4; ++s) {
      const int b = 4 * s + g;
      const double bv = b < K ? zb[(zo + b) * 16 + r16] : 0.0;
      const double av = (r16 < K && b < K) ? fct[r16 + b + 2 * m] : 0.0;
      d = mfma(av, bv, d);
    }
    const double sg = (m & 1) ? -1.0 : 1.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int a = 4 * i + g;
      if (a < K) {
        const int j = m + a;
        zb[(zo + a) * 16 + r16] = d[i] * sg * uz[16 * m + j] * rp[j + 1];
      }
    }
  }
  wave_lds_sync();
#pragma unroll
  for (int t = 0; t < T; ++t) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const tl::Slot d = tl::decode(P, t, 4 * i + g);
      if (d.valid && d.sine == SINE) st[t][i] = zb[(tl::zoff(P, d.m) + d.n - d.m) * 16 + r16];
    }
  }
  wave_lds_sync();
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
  double* Jt = smem;
  double* fct = Jt + T * 272;
  double* uz = fct + 32;
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* trig = smem + C::SHARED + wid * C::PERWAVE;
  double* zb = trig + 16 * C::TRIG;
  for (int k = threadIdx.x; k < C::SHARED; k += 256) smem[k] = mtab[k];
  __syncthreads();

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
    const int r16 = lane & 15, g = lane >> 4;
    const double* geo = lv.geom[l];
    const double cix = geo[bi * 10 + 6], ciy = geo[bi * 10 + 7], ciz = geo[bi * 10 + 8];
    const int64_t e0 = lv.w_off[l][bi], e1 = lv.w_off[l][bi + 1];
    const int32_t* widx = lv.w_idx[l];
    const double* Mlev = Mx + (size_t)lv.gofs[l] * S;
    double* tp = trig + r16 * C::TRIG;  // this lane's pair
    const double* cs_a = tp;
    const double* cs_t = tp + 2 * (P + 1);
    const double* rp = tp + 4 * (P + 1);

    // compact accumulator: lane r16 owns the tiles t with t % 16 == r16
    constexpr int NA = (T + 15) / 16;
    d4 acc[NA];
#pragma unroll
    for (int k = 0; k < NA; ++k) acc[k] = d4{0.0, 0.0, 0.0, 0.0};

    for (int64_t eb = e0; eb < e1; eb += 16) {
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
      // trig and power tables of this pair, split over the 4 lanes of the pair
      if (g == 0) {
        const double ca = dz / rho, sa = rxy / rho;
        double c = 1.0, s = 0.0;
        for (int m = 0; m <= P; ++m) {
          tp[2 * m] = c;
          tp[2 * m + 1] = s;
          const double nc = c * ca - s * sa, ns = s * ca + c * sa;
          c = nc;
          s = ns;
        }
      } else if (g == 1) {
        // theta2 = pi/2 - beta: cos = sin(beta), sin = cos(beta)
        const double ct = rxy > 0.0 ? dy / rxy : 0.0, st2 = rxy > 0.0 ? dx / rxy : 1.0;
        double c = 1.0, s = 0.0;
        for (int m = 0; m <= P; ++m) {
          tp[2 * (P + 1) + 2 * m] = c;
          tp[2 * (P + 1) + 2 * m + 1] = s;
          const double nc = c * ct - s * st2, ns = s * ct + c * st2;
          c = nc;
          s = ns;
        }
      } else if (g == 2) {
        const double ir = 1.0 / rho;
        double v = 1.0;
        for (int k = 0; k <= P + 1; ++k) {
          tp[4 * (P + 1) + k] = v;
          v *= ir;
        }
      }
      d4 st[T];
      const double* src = Mlev + (size_t)j * S + 4 * g;
#pragma unroll
      for (int t = 0; t < T; ++t) st[t] = valid ? *(const d4*)(src + 16 * t) : d4{0.0, 0.0, 0.0, 0.0};
      wave_lds_sync();

      rotz<P>(st, cs_t, 1.0, g);
      japply<P, true>(st, Jt, r16, g);
      rotz<P>(st, cs_a, 1.0, g);
      japply<P, false>(st, Jt, r16, g);
      ztrans_part<P, 0>(st, zb, fct, uz, rp, r16, g);
      ztrans_part<P, 1>(st, zb, fct, uz, rp, r16, g);
      japply<P, true>(st, Jt, r16, g);
      rotz<P>(st, cs_a, -1.0, g);
      japply<P, false>(st, Jt, r16, g);
      rotz<P>(st, cs_t, -1.0, g);
      // sum this batch over its 16 pairs; the owner lane of each tile keeps it
#pragma unroll
      for (int t = 0; t < T; ++t) {
        d4 v;
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = row_sum16(st[t][i]);
        if (r16 == (t & 15)) acc[t >> 4] += v;
      }
      wave_lds_sync();  // trig table is rewritten by the next batch
    }
    double* dst = Lx + (size_t)gid * S + 4 * g;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      const int t = 16 * k + r16;
      if (t < T) *(d4*)(dst + 16 * t) = acc[k];
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
