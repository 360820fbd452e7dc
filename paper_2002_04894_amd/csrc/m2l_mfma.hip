// M2L on the matrix cores (Algorithm 3, M2L; rotational form of Section
// 2.1.3), for expansion orders p <= 15, in FP64 (v_mfma_f64_16x16x4f64).
//
// A block of two waves computes the local expansion of one target box i:
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
// powers of 1/rho.  The two waves of a block share each batch: each owns
// half of the tiles and half of the orders m of the z translation, and they
// meet at block barriers around the exchanges through LDS; with two such
// waves on every SIMD, one wave's vector and LDS work runs while the other's
// matrix products do.  The 16 pair results of a batch are summed through LDS
// into one accumulator per coefficient: no atomics, deterministic.
#include "fmm_internal.h"
#include "tile_layout.h"

namespace fmm {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

// The kernel runs in binary64, or (mixed precision) in binary32 on
// radius-scaled expansions: R is the arithmetic type of the translations.
template <class R>
struct Ar;
template <>
struct Ar<double> {
  typedef d4 v4;
  typedef d2 v2;
  static constexpr int kRowStride = 18;  // pair-sum rows: 144 B, no bank conflicts
};
template <>
struct Ar<float> {
  typedef f4 v4;
  typedef f2 v2;
  static constexpr int kRowStride = 20;
};

// Waves per SIMD the kernel is compiled for (the register budget per lane
// is 512 / that).  binary64: 2 (its operand fragments already spill a little
// at 256 registers).  binary32: 4 up to order 8, 3 above; measured on the
// 2^24-point Plummer cloud at theta 0.6 against 2 waves: 131 / 137.6 / 159.3
// ms at order 8, 156.6 / 175.2 ms (3 / 2 waves) at order 10, 220.5 / 232.5 at
// 12, 232.2 / 259.6 at 13 (4 waves lost above order 8, on spills).
template <int P, class R>
struct Occ {
  static constexpr int kWavesPerEu = 2;
};
template <int P>
struct Occ<P, float> {
  static constexpr int kWavesPerEu = P <= 8 ? 4 : 3;
};

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
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int P, class R>
struct Cfg {
  static constexpr int T = tl::ntiles(P);
  static constexpr int NP = tl::npairs(P);
  static constexpr int S = tl::stride(P);
  static constexpr int ZR = tl::zrows(P);
  static constexpr int H = tl::hoff(P, P + 1);
  // z buffer: ZR coefficient rows, a write-only row (also read past the last
  // order by the zero-padded tail of its last k-step) and two more such rows;
  // the two waves' pair-sum rounds reuse it
  static constexpr int ZDUMMY = ZR;
  static constexpr int RSTRIDE = Ar<R>::kRowStride;
  static constexpr int ZBUF = 16 * (ZR + 3) > 2 * 64 * RSTRIDE ? 16 * (ZR + 3) : 2 * 64 * RSTRIDE;
  // per pair: (cos, sin)(m (theta + pi)), (cos, sin)(m (alpha + pi)), m = 0..P;
  // 16 more bytes per pair so that the 16 pair columns hit different banks
  static constexpr int TRIG = 4 * (P + 1) + 2;
  // per block: two trig tables (alternate batches), the z buffer, a row that
  // stays zero, and the slot that hands out targets (elements of R)
  static constexpr int LDS = 2 * 16 * TRIG + ZBUF + 16 + 2;
};

// Work split between the two waves of a block.  Wave 0 owns the degree pairs
// a < NA (both their cosine and sine tiles) and the mixed tile, wave 1 the
// other pairs and the two tiles of degree P; the orders m of the z
// translation go to the wave with the smaller matrix-core load so far.
template <int P>
__host__ __device__ constexpr int split_na() {
  constexpr int NP = tl::npairs(P), MX = tl::has_mixed(P) ? 1 : 0;
  const int na = (2 * NP + 2 - MX + 2) / 4;
  return na < NP ? na : NP;
}
template <int P>
__host__ __device__ constexpr int tile_owner(int t) {
  constexpr int NP = tl::npairs(P);
  if (t < 2 * NP) return (t < NP ? t : t - NP) < split_na<P>() ? 0 : 1;
  if (tl::has_mixed(P) && t == tl::mixed_tile(P)) return 0;
  return 1;
}
template <int P>
__host__ __device__ constexpr int tiles_of(int w) {
  int c = 0;
  for (int t = 0; t < tl::ntiles(P); ++t) c += tile_owner<P>(t) == w ? 1 : 0;
  return c;
}
// k-th tile (in tile order) owned by wave w
template <int P>
__host__ __device__ constexpr int owned_tile(int w, int k) {
  for (int t = 0; t < tl::ntiles(P); ++t)
    if (tile_owner<P>(t) == w && k-- == 0) return t;
  return 0;
}
struct MSplit {
  int owner[tl::kMaxP + 1];
};
template <int P>
__host__ __device__ constexpr MSplit m_split() {
  MSplit r{};
  int load[2] = {16 * tiles_of<P>(0), 16 * tiles_of<P>(1)};  // four J products of four steps per tile
  // orders by decreasing work: low m first (more rows)
  for (int m = 0; m <= P; ++m) {
    const int w = load[0] <= load[1] ? 0 : 1;
    r.owner[m] = w;
    load[w] += tl::hsteps(P, m) * (m == 0 ? 1 : 2);
  }
  return r;
}

__device__ __forceinline__ int level_of2(const LevelView& lv, int64_t gid) {
  int l = 0;
  while (l < lv.L && gid >= lv.gofs[l + 1]) ++l;
  return l;
}

// Slot s of tile t as a coefficient position (degree n, order m), or a
// padding slot (pos = 0).  The always-zero sine slot of order 0 counts as a
// position: it is carried along like any coefficient.
struct Pos {
  int pos, n, m;
};
template <int P>
__host__ __device__ constexpr Pos slot_pos(int t, int s) {
  constexpr int NP = tl::npairs(P);
  if (t < 2 * NP) {
    const int a = t < NP ? t : t - NP, b = P - 1 - a;
    if (s <= a) return Pos{1, a, s};
    if (s <= a + 1 + b) return Pos{1, b, s - a - 1};
    return Pos{0, 0, 0};
  }
  if (tl::has_mixed(P) && t == tl::mixed_tile(P)) {
    const int h = (P - 1) / 2;
    if (s <= h) return Pos{1, h, s};
    if (s >= 8 && s <= 8 + h) return Pos{1, h, s - 8};
    return Pos{0, 0, 0};
  }
  return s <= P ? Pos{1, P, s} : Pos{0, 0, 0};
}

// 1 if k-step k of tile t (slots 4k .. 4k+3) holds a coefficient position.
// A step of padding slots only multiplies zero operator columns, so the J
// products skip it (below order 12 the last step of every pair tile).
template <int P>
__host__ __device__ constexpr bool kstep_used(int t, int k) {
  for (int g = 0; g < 4; ++g)
    if (slot_pos<P>(t, 4 * k + g).pos) return true;
  return false;
}

// 1 if register i of tile t holds padding slots only (then the J products
// give it zeros, and the rotations and the z translation leave it alone).
template <int P>
__host__ __device__ constexpr bool all_pad(int t, int i) {
  return !kstep_used<P>(t, i);
}

// The four lanes groups g = 0..3 hold slots 4i + g of register i.  Along g
// they form at most three runs: within a run either padding, or one degree n
// with orders m = m0 + g.
struct Quad {
  int nseg;
  int end[3];  // run k covers g < end[k]
  int pad[3], n[3], m0[3];
};
template <int P>
__host__ __device__ constexpr Quad quad(int t, int i) {
  Quad q{0, {4, 4, 4}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int g = 0; g < 4; ++g) {
    const Pos d = slot_pos<P>(t, 4 * i + g);
    const int k = q.nseg - 1;
    const bool same = q.nseg > 0 && ((q.pad[k] && !d.pos) ||
                                    (!q.pad[k] && d.pos && d.n == q.n[k] && d.m == q.m0[k] + g));
    if (!same) {
      if (q.nseg > 0) q.end[q.nseg - 1] = g;
      q.pad[q.nseg] = d.pos ? 0 : 1;
      q.n[q.nseg] = d.n;
      q.m0[q.nseg] = d.m - g;
      ++q.nseg;
    }
  }
  q.end[q.nseg - 1] = 4;
  return q;
}

// pick v[k] for this lane's run of q
__device__ __forceinline__ int pick(const Quad& q, int g, int v0, int v1, int v2) {
  if (q.nseg == 1) return v0;
  const int w = g < q.end[0] ? v0 : v1;
  return q.nseg == 2 ? w : (g < q.end[1] ? w : v2);
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

// (c, s) <- f (cos c - sgn sin s, sgn sin c + cos s) for every (cosine, sine)
// partner pair, f = mult * base^n for a slot of degree n (SCALE) or 1; cs:
// this lane's (cos, sin) table shifted by 2 (g - 4)
template <int P, int W, bool SCALE, class R>
__device__ __forceinline__ void rotz(typename Ar<R>::v4* st, const R* cs, R sgn, int g, R base, R mult) {
  typedef typename Ar<R>::v2 v2;
  constexpr int NP = tl::npairs(P);
  R pw[SCALE ? P + 1 : 1];  // mult * base^n, built here to keep it short-lived
  pw[0] = mult;
  if constexpr (SCALE) {
#pragma unroll
    for (int n = 1; n <= P; ++n) pw[n] = pw[n - 1] * base;
  }
  auto rot = [&](R& c, R& s, int t, int i) {
    const Quad q = quad<P>(t, i);
    if (q.nseg == 1 && q.pad[0]) return;  // padding only: nothing to rotate
    const int k0 = 2 * (q.m0[0] + 4), k1 = 2 * (q.m0[1] + 4), k2 = 2 * (q.m0[2] + 4);
    // a padding run reads any finite entry: its coefficients are zero
    const v2 v = *(const v2*)(cs + pick(q, g, q.pad[0] ? 8 : k0, q.pad[1] ? 8 : k1, q.pad[2] ? 8 : k2));
    R co = v.x, si = sgn * v.y;
    if constexpr (SCALE) {
      const R f = q.nseg == 1 ? pw[q.n[0]]
                              : (g < q.end[0] ? pw[q.n[0]]
                                              : (q.nseg == 2 || g < q.end[1] ? pw[q.n[1]] : pw[q.n[2]]));
      co *= f;
      si *= f;
    }
    const R nc = co * c - si * s;
    const R ns = si * c + co * s;
    c = nc;
    s = ns;
  };
#pragma unroll
  for (int a = 0; a < NP; ++a) {
    if (tile_owner<P>(a) != W) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      R c = st[a][i], s = st[NP + a][i];
      rot(c, s, a, i);
      st[a][i] = c;
      st[NP + a][i] = s;
    }
  }
  if constexpr (tl::has_mixed(P) && tile_owner<P>(tl::mixed_tile(P)) == W) {
    constexpr int t = tl::mixed_tile(P);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      R c = st[t][i], s = st[t][i + 2];
      rot(c, s, t, i);
      st[t][i] = c;
      st[t][i + 2] = s;
    }
  }
  if constexpr (tile_owner<P>(tl::top_c(P)) == W) {
    constexpr int tc = tl::top_c(P), ts = tl::top_s(P);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      R c = st[tc][i], s = st[ts][i];
      rot(c, s, tc, i);
      st[tc][i] = c;
      st[ts][i] = s;
    }
  }
}

// st[t] <- J_t st[t] for the tiles of wave W; jr: this lane's operand
// fragments of J (in registers)
template <int P, int W, class R>
__device__ __forceinline__ void japply(typename Ar<R>::v4* st, const R* jr) {
  constexpr int T = tl::ntiles(P);
#pragma unroll
  for (int t = 0; t < T; ++t) {
    if (tile_owner<P>(t) != W) continue;
    typename Ar<R>::v4 d = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (kstep_used<P>(t, k)) d = mfma(jr[t * 4 + k], st[t][k], d);
    st[t] = d;
  }
}

// z buffer addressing: zl[k] points at row zoff(m) - m of this lane's column
// for m = k - 4 + g (so that row (m, n) is zl[k] + 16 n), zd at the
// write-only row, zz at the zero row
template <class R>
struct ZView {
  R* zl[20];
  R* zd;
  const R* zz;
};

template <int P, class R>
__device__ __forceinline__ R* zslot(const ZView<R>& z, int t, int i, int g, bool for_read) {
  const Quad q = quad<P>(t, i);
  R* other = for_read ? (R*)z.zz : z.zd;
  R* a0 = q.pad[0] ? other : z.zl[q.m0[0] + 4] + 16 * q.n[0];
  if (q.nseg == 1) return a0;
  R* a1 = q.pad[1] ? other : z.zl[q.m0[1] + 4] + 16 * q.n[1];
  R* w = g < q.end[0] ? a0 : a1;
  if (q.nseg == 2) return w;
  R* a2 = q.pad[2] ? other : z.zl[q.m0[2] + 4] + 16 * q.n[2];
  return g < q.end[1] ? w : a2;
}

// z-axis translation of the cosine (SINE = 0) or sine blocks; the input is
// already scaled by (1/rho)^n and the output by (1/rho)^(j+1) is applied by
// the next rotation.  Both waves move their tiles to the order-major rows
// and back; each computes its own orders.  hr: this lane's operand fragments
// of the order-m matrices (in registers).
template <int P, int W, int SINE, class R>
__device__ __forceinline__ void ztrans_part(typename Ar<R>::v4* st, const ZView<R>& z, R* zcol, const R* hr,
                                            int lane) {
  constexpr int T = tl::ntiles(P);
  constexpr MSplit ms = m_split<P>();
  const int g = lane >> 4;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    if (tile_owner<P>(t) != W) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (reg_sine<P>(t, i) != SINE || all_pad<P>(t, i)) continue;
      *zslot<P, R>(z, t, i, g, false) = st[t][i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = SINE; m <= P; ++m) {
    if (ms.owner[m] != W) continue;
    const int K = P + 1 - m;
    const int zo = tl::zoff(P, m);
    const int ho = tl::hoff(P, m);
    typename Ar<R>::v4 d = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < tl::hsteps(P, m); ++k) d = mfma(hr[ho + k], zcol[(zo + 4 * k) * 16], d);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (4 * i >= K) continue;
      R* dst = (4 * i + 3 < K || 4 * i + g < K) ? zcol + (zo + 4 * i) * 16 : z.zd;
      *dst = d[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < T; ++t) {
    if (tile_owner<P>(t) != W) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (reg_sine<P>(t, i) != SINE || all_pad<P>(t, i)) continue;
      st[t][i] = *zslot<P, R>(z, t, i, g, true);
    }
  }
  __syncthreads();
}

// the work of wave W of the block (both waves run the same loop structure
// and meet at the same barriers).  R = double: Mx holds the multipoles
// (binary64).  R = float: Mx holds them in binary32, scaled as
// M~_n = M_n / s^n with s the box radius (1 for a box of zero extent), and
// the result is unscaled into binary64 at the store.
template <int P, int W, class R>
__device__ __forceinline__ void m2l_wave(R* smem, const LevelView& lv, const R* __restrict__ mtab,
                                         const R* __restrict__ Mx, double* __restrict__ Lx, int64_t ntarget,
                                         const int32_t* __restrict__ order, int* __restrict__ queue) {
  using C = Cfg<P, R>;
  typedef typename Ar<R>::v4 v4;
  typedef typename Ar<R>::v2 v2;
  constexpr bool MIXED = sizeof(R) == 4;
  constexpr int T = C::T;
  constexpr int S = C::S;
  constexpr int NTW = tiles_of<P>(W);
  constexpr int NRW = (NTW + 3) / 4;  // pair-sum rounds of four tiles
  constexpr MSplit ms = m_split<P>();
  const int lane = threadIdx.x & 63;
  const int r16 = lane & 15, g = lane >> 4;
  R* trig = smem;                       // two tables, alternate batches
  R* zb = smem + 2 * 16 * C::TRIG;
  R* zero_row = zb + C::ZBUF;           // stays zero
  int* slot = (int*)(zero_row + 16);    // target handed to the block

  // operand fragments of this wave's J tiles and orders, kept in registers
  R jr[T * 4];
#pragma unroll
  for (int t = 0; t < T; ++t)
    if (tile_owner<P>(t) == W)
#pragma unroll
      for (int k = 0; k < 4; ++k) jr[t * 4 + k] = kstep_used<P>(t, k) ? mtab[(t * 4 + k) * 64 + lane] : (R)0;
  R hr[C::H];
#pragma unroll
  for (int m = 0; m <= P; ++m)
    if (ms.owner[m] == W)
#pragma unroll
      for (int k = 0; k < tl::hsteps(P, m); ++k)
        hr[tl::hoff(P, m) + k] = mtab[T * 256 + (tl::hoff(P, m) + k) * 64 + lane];

  ZView<R> z;
#pragma unroll
  for (int k = 0; k < 20; ++k) {
    const int m = k - 4 + g;
    z.zl[k] = zb + 16 * (tl::zoff(P, m) - m) + r16;
  }
  z.zd = zb + 16 * C::ZDUMMY + r16;
  z.zz = zero_row + r16;
  R* zcol = zb + 16 * g + r16;
  R* red = zb + W * 64 * C::RSTRIDE;  // this wave's pair-sum rows

  // persistent blocks: each takes the next target of the longest-first order
  // until the queue is empty
  for (;;) {
    if (W == 0 && lane == 0) *slot = atomicAdd(queue, 1);
    __syncthreads();
    const int k_next = *slot;
    __syncthreads();
    if (k_next >= ntarget) break;
    const int64_t tgt = order[k_next];
    const int64_t gid = lv.gofs[1] + tgt;
    const int l = level_of2(lv, gid);
    const int64_t bi = gid - lv.gofs[l];
    const double* geo = lv.geom[l];
    const double cix = geo[bi * 10 + 6], ciy = geo[bi * 10 + 7], ciz = geo[bi * 10 + 8];
    const double rt = geo[bi * 10 + 9] > 0.0 ? geo[bi * 10 + 9] : 1.0;  // target scale (MIXED)
    const int64_t e0 = lv.w_off[l][bi], e1 = lv.w_off[l][bi + 1];
    const int32_t* widx = lv.w_idx[l];
    const R* Mlev = Mx + (size_t)lv.gofs[l] * S;

    double acc[NRW > 0 ? NRW : 1];
#pragma unroll
    for (int r = 0; r < NRW; ++r) acc[r] = 0.0;

    int buf = 0;
    for (int64_t eb = e0; eb < e1; eb += 16, buf ^= 1) {
      // pair of this lane's column; past the end of the list the column
      // repeats the first source with zero factors, which zeroes its result
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
      const double irho = 1.0 / rho;
      // scalings: M'(n) (1/rho)^n into the z translation, its output times
      // (1/rho)^(j+1); with scaled expansions (s/rho)^n and (rt/rho)^j / rho
      R in_base, out_base, out_mult;
      if constexpr (MIXED) {
        const double rs = geo[(int64_t)j * 10 + 9] > 0.0 ? geo[(int64_t)j * 10 + 9] : 1.0;
        in_base = valid ? (R)(rs * irho) : (R)0;
        out_base = valid ? (R)(rt * irho) : (R)0;
        out_mult = valid ? (R)irho : (R)0;
      } else {
        in_base = valid ? irho : 0.0;
        out_base = in_base;
        out_mult = in_base;
      }
      R* tp = trig + buf * 16 * C::TRIG + r16 * C::TRIG;  // this lane's pair
      // (cos, sin)(m (angle + pi)) by the angle-addition recurrence (binary64):
      // wave 0 builds the theta table, wave 1 the alpha table (the four lane
      // groups write the same values to the same words)
      {
        double c1, s1;
        if (W == 0) {
          const double irxy = rxy > 0.0 ? 1.0 / rxy : 0.0;
          c1 = -dy * irxy;
          s1 = rxy > 0.0 ? -dx * irxy : -1.0;
        } else {
          c1 = -dz * irho;
          s1 = -rxy * irho;
        }
        R* dst = tp + (W == 0 ? 0 : 2 * (P + 1));
        double c = 1.0, s = 0.0;
#pragma unroll
        for (int m = 0; m <= P; ++m) {
          *(v2*)(dst + 2 * m) = v2{(R)c, (R)s};
          const double nc = c * c1 - s * s1, ns = s * c1 + c * s1;
          c = nc;
          s = ns;
        }
      }
      v4 st[T];
      const R* src = Mlev + (size_t)j * S + 4 * g;
#pragma unroll
      for (int t = 0; t < T; ++t)
        if (tile_owner<P>(t) == W) st[t] = *(const v4*)(src + 16 * t);
      __syncthreads();  // both tables written

      // (cos, sin) tables shifted so that entry 2 (m0 + 4) is order m0 + g
      const R* cs_t = tp + 2 * (g - 4);
      const R* cs_a = tp + 2 * (P + 1) + 2 * (g - 4);
      // scheduling strategy for the long barrier-free stretches
      __builtin_amdgcn_iglp_opt(0);
      rotz<P, W, false, R>(st, cs_t, (R)1, g, (R)0, (R)1);
      japply<P, W, R>(st, jr);
      rotz<P, W, true, R>(st, cs_a, (R)1, g, in_base, (R)1);
      japply<P, W, R>(st, jr);
      ztrans_part<P, W, 0, R>(st, z, zcol, hr, lane);
      ztrans_part<P, W, 1, R>(st, z, zcol, hr, lane);
      __builtin_amdgcn_iglp_opt(0);
      japply<P, W, R>(st, jr);
      rotz<P, W, true, R>(st, cs_a, (R)-1, g, out_base, out_mult);
      japply<P, W, R>(st, jr);
      rotz<P, W, false, R>(st, cs_t, (R)-1, g, (R)0, (R)1);

      // sum over the 16 pairs, four of this wave's tiles per round; lane L
      // adds up row L (slot L % 16 of its tile 4 r + L / 16); each batch sum
      // is added into binary64
#pragma unroll
      for (int r = 0; r < NRW; ++r) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (4 * r + q >= NTW) continue;
          const int t = owned_tile<P>(W, 4 * r + q);
#pragma unroll
          for (int i = 0; i < 4; ++i) red[(q * 16 + 4 * i + g) * C::RSTRIDE + r16] = st[t][i];
        }
        wave_lds_fence();
        if (4 * r + 3 < NTW || 4 * r + (lane >> 4) < NTW) {
          const R* row = red + lane * C::RSTRIDE;
          if constexpr (MIXED) {
            // the 16 binary32 pair results are summed in binary64 (exact for
            // all but extreme exponent spreads)
            double sum = 0.0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              const v2 v = *(const v2*)(row + 2 * k);
              sum += (double)v.x;
              sum += (double)v.y;
            }
            acc[r] += sum;
          } else {
            v2 v = *(const v2*)row;
#pragma unroll
            for (int k = 1; k < 8; ++k) v += *(const v2*)(row + 2 * k);
            acc[r] += (double)(v.x + v.y);
          }
        }
        wave_lds_fence();
      }
    }
    // lane L holds slot L % 16 of the wave's tile 4 r + L / 16; the final D is
    // the sign (-1)^m, and scaled expansions are unscaled by rt^-n
    double* dst = Lx + (size_t)gid * S;
#pragma unroll
    for (int r = 0; r < NRW; ++r) {
      const int k = 4 * r + (lane >> 4);
      if (k < NTW) {
        const int t = owned_tile<P>(W, k);
        const Pos d = slot_pos<P>(t, lane & 15);
        double v = (d.m & 1) ? -acc[r] : acc[r];
        if (MIXED) {
          const double irt = 1.0 / rt;
          for (int n = 0; n < d.n; ++n) v *= irt;
        }
        dst[tl::spos(t, lane & 15)] = v;
      }
    }
  }
}

template <int P, class R>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(Occ<P, R>::kWavesPerEu,
                                                                     Occ<P, R>::kWavesPerEu))) void k_m2l_mfma(
    LevelView lv, const R* __restrict__ mtab, const R* __restrict__ Mx, double* __restrict__ Lx,
    int64_t ntarget, const int32_t* __restrict__ order, int* __restrict__ queue) {
  __shared__ R smem[Cfg<P, R>::LDS];
  // every LDS word starts finite: buffer tails are read (and multiplied by 0)
  for (int k = threadIdx.x; k < Cfg<P, R>::LDS; k += 128) smem[k] = (R)0;
  __syncthreads();
  if (threadIdx.x < 64)
    m2l_wave<P, 0, R>(smem, lv, mtab, Mx, Lx, ntarget, order, queue);
  else
    m2l_wave<P, 1, R>(smem, lv, mtab, Mx, Lx, ntarget, order, queue);
}

// binary32 copy of the multipoles of levels 1..L, scaled by s^-n (s the box
// radius, 1 for a box of zero extent); padding positions stay zero
__global__ void k_scale_m32(LevelView lv, int S, const int8_t* __restrict__ sdeg, const double* __restrict__ Mx,
                            float* __restrict__ Mf, int64_t nbox_total) {
  const int64_t gid = 1 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (gid >= nbox_total) return;
  int l = 1;
  while (l < lv.L && gid >= lv.gofs[l + 1]) ++l;
  const double r = lv.geom[l][(gid - lv.gofs[l]) * 10 + 9];
  const double is = r > 0.0 ? 1.0 / r : 1.0;
  for (int q = threadIdx.x & 63; q < S; q += 64) {
    const int n = sdeg[q];
    double v = Mx[(size_t)gid * S + q];
    for (int k = 0; k < n; ++k) v *= is;
    Mf[(size_t)gid * S + q] = n >= 0 ? (float)v : 0.f;
  }
}

__global__ void k_zero_queue(int* queue) {
  if (threadIdx.x == 0) *queue = 0;
}

template <int P, class R>
void launch_one(const Tree& t, const Tables& tb, const R* Mx, double* Lx, hipStream_t s) {
  const int64_t ntarget = t.nbox_total - 1;
  // resident blocks of this instantiation on the device (initialised once,
  // thread-safe)
  static const int grid_max = [] {
    int dev = 0, ncu = 0, per = 0;
    HIPCHECK(hipGetDevice(&dev));
    HIPCHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_m2l_mfma<P, R>, 128, 0));
    return ncu * (per > 0 ? per : 1);
  }();
  const int64_t need = ntarget;
  const unsigned grid = (unsigned)(need < grid_max ? need : grid_max);
  int* queue = (int*)dalloc(sizeof(int), s);
  // cleared by a kernel, not a memset node, so that the launch may be captured in a graph
  k_zero_queue<<<1, 64, 0, s>>>(queue);
  HIPCHECK(hipGetLastError());
  const R* mt;
  if constexpr (sizeof(R) == 4)
    mt = tb.mtab32;
  else
    mt = tb.mtab;
  k_m2l_mfma<P, R><<<grid, 128, 0, s>>>(t.view(), mt, Mx, Lx, ntarget, t.m2l_order, queue);
  HIPCHECK(hipGetLastError());
  dfree(queue, s);
}

template <class R>
bool launch_any(const Tree& t, const Tables& tb, const R* Mx, double* Lx, hipStream_t s) {
  switch (tb.p) {
    case 0: launch_one<0, R>(t, tb, Mx, Lx, s); break;
    case 1: launch_one<1, R>(t, tb, Mx, Lx, s); break;
    case 2: launch_one<2, R>(t, tb, Mx, Lx, s); break;
    case 3: launch_one<3, R>(t, tb, Mx, Lx, s); break;
    case 4: launch_one<4, R>(t, tb, Mx, Lx, s); break;
    case 5: launch_one<5, R>(t, tb, Mx, Lx, s); break;
    case 6: launch_one<6, R>(t, tb, Mx, Lx, s); break;
    case 7: launch_one<7, R>(t, tb, Mx, Lx, s); break;
    case 8: launch_one<8, R>(t, tb, Mx, Lx, s); break;
    case 9: launch_one<9, R>(t, tb, Mx, Lx, s); break;
    case 10: launch_one<10, R>(t, tb, Mx, Lx, s); break;
    case 11: launch_one<11, R>(t, tb, Mx, Lx, s); break;
    case 12: launch_one<12, R>(t, tb, Mx, Lx, s); break;
    case 13: launch_one<13, R>(t, tb, Mx, Lx, s); break;
    case 14: launch_one<14, R>(t, tb, Mx, Lx, s); break;
    case 15: launch_one<15, R>(t, tb, Mx, Lx, s); break;
    default: return false;
  }
  return true;
}

}  // namespace

bool launch_m2l_mfma(const Tree& t, const Tables& tb, const double* Mx, double* Lx, hipStream_t s) {
  if (!tb.tiled) return false;
  return launch_any<double>(t, tb, Mx, Lx, s);
}

bool launch_m2l_lane32(const Tree& t, const Tables& tb, const double* Mx, double* Lx, hipStream_t s);

bool launch_m2l_mfma_mixed(const Tree& t, const Tables& tb, const double* Mx, double* Lx, hipStream_t s) {
  if (!tb.tiled) return false;
  // orders up to 14 one pair per lane (m2l_lane.hip), 15 in 16x16 tiles
  if (launch_m2l_lane32(t, tb, Mx, Lx, s)) return true;
  float* Mf = (float*)dalloc((size_t)t.nbox_total * tb.stride * sizeof(float), s);
  if (t.nbox_total > 1) {
    k_scale_m32<<<(unsigned)((t.nbox_total - 1 + 3) / 4), 256, 0, s>>>(t.view(), tb.stride, tb.sdeg, Mx, Mf,
                                                                      t.nbox_total);
    HIPCHECK(hipGetLastError());
  }
  const bool ok = launch_any<float>(t, tb, Mf, Lx, s);
  dfree(Mf, s);
  return ok;
}

}  // namespace fmm
