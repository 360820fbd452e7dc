// M2L on the vector units (Algorithm 3, M2L; rotational form of Section
// 2.1.3), one weak pair per lane, for the mixed-precision mode (binary32 on
// radius-scaled expansions) at orders p <= 9.
//
// Every lane of a wave takes one pair of the same target box, 64 pairs at a
// time, and holds its pair's whole expansion in registers in the standard
// order (c_{n,0}, c_{n,1}, s_{n,1}, ..., per degree n).  The translation is
// the same sequence as the binary64 vector kernel k_m2l:
//   Rz(-beta), J^T, Rz(-alpha), J, z-axis translation, J^T, Rz(alpha), J, Rz(beta),
// with J the fixed quarter turn about x (block-diagonal in two parity classes
// per degree) and (alpha, beta) the polar and azimuthal angles of
// d = c_source - c_target.  Every operand of the fixed matrices (J and the
// z-translation core A) is the same for all lanes, so it is read once per
// wave as a scalar operand; no work is padded, unlike 16x16 matrix tiles of
// two degree blocks each.  The 64 pair results are summed across the lanes by
// halving exchanges (a fixed order: deterministic) and the batch sums are
// added in binary64.  The expansions are scaled as for the binary32 matrix
// kernel: M~_n = M_n / r_s^n on the way in, so the factors (r_s/rho)^n and
// (r_t/rho)^j / rho stay below one, and the result is unscaled by r_t^-n
// into binary64.
#include "fmm_internal.h"
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
// 0 / 1: the two classes of the standard index i within a degree that the
// quarter turn about x keeps apart (its other entries vanish)
__host__ __device__ constexpr int parity_cls(int i) {
  return i == 0 ? 0 : ((((i + 1) >> 1) + ((i & 1) ? 0 : 1)) & 1);
}
// storage position of standard index k in the tile layout of order P
template <int P>
__host__ __device__ constexpr int tpos(int k) {
  const int n = deg_of(k), i = k - n * n, m = (i + 1) >> 1, sine = (i != 0 && (i & 1) == 0) ? 1 : 0;
  for (int t = 0; t < tl::ntiles(P); ++t)
    for (int s = 0; s < 16; ++s) {
      const tl::Slot d = tl::decode(P, t, s);
      if (d.valid && d.n == n && d.m == m && d.sine == sine) return tl::spos(t, s);
    }
  return -1;
}
// the whole map, built at compile time (indexing a constant table keeps the
// expansion in registers after unrolling)
template <int P>
struct PosTab {
  int v[(P + 1) * (P + 1)];
};
template <int P>
__host__ __device__ constexpr PosTab<P> make_pos() {
  PosTab<P> t{};
  for (int k = 0; k < (P + 1) * (P + 1); ++k) t.v[k] = tpos<P>(k);
  return t;
}

// sizes of the halving exchanges: level 0 holds all NT values, each of the
// six levels keeps the lane's half (rounded up)
__host__ __device__ constexpr int lvl(int nt, int s) {
  int v = nt;
  for (int k = 0; k < s; ++k) v = (v + 1) / 2;
  return v;
}

// The operator entries are the same for every pair, so the compiler would
// keep all of them in scalar registers across the pair loop (thousands of
// values: they spill).  Passing the table pointer through an opaque move
// makes every use load its entries again, from the scalar cache, where they
// are needed.
// The tables never change while a kernel runs, so they are read through the
// constant address space, which lets the loads be scalar.
typedef const __attribute__((address_space(4))) float cfloat;
__device__ __forceinline__ cfloat* opaque(const float* p) {
  asm volatile("" : "+s"(p));
  return (cfloat*)(uintptr_t)p;
}

// X <- Rz(sign * g) X, with (c1, s1) = (cos g, sin g); the multiples by the
// angle-addition recurrence in binary64
template <int P>
__device__ __forceinline__ void rotz(float* X, double c1, double s1, double sign) {
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

// X <- J X (TRANS = false) or J^T X (TRANS = true), degree by degree; J
// entries are uniform loads (scalar operands), the vanishing ones skipped
// Jc: the nonzero entries of J (TRANS = false) or J^T (TRANS = true) in the
// order they are used -- per degree, per parity class, row by row -- so that
// consecutive uses are consecutive words (wide scalar loads); see
// compact_j in expansions.hip
template <int P, bool TRANS>
__device__ __forceinline__ void japply(float* X, const float* __restrict__ Jc) {
  int off = 0;
#pragma unroll
  for (int n = 0; n <= P; ++n) {
    const int sd = 2 * n + 1;
    // one parity class at a time: the other's values stay untouched meanwhile
#pragma unroll
    for (int cls = 0; cls < 2; ++cls) {
      cfloat* J = opaque(Jc + off);
      float tmp[P + 1];
      int c = 0, u = 0;
#pragma unroll
      for (int i = 0; i < sd; ++i) {
        if (parity_cls(i) != cls) continue;
        float acc = 0.f;
#pragma unroll
        for (int q = 0; q < sd; ++q) {
          if (parity_cls(q) != cls) continue;
          acc += J[u++] * X[n * n + q];
        }
        tmp[c++] = acc;
      }
      off += u;
      c = 0;
#pragma unroll
      for (int i = 0; i < sd; ++i) {
        if (parity_cls(i) != cls) continue;
        X[n * n + i] = tmp[c++];
      }
    }
  }
}

// z-axis translation (M2L): X_{d,m} <- out(d) sum_{n >= m} A[m][d][n] in(n) X_{n,m},
// in(n) = in_base^n, out(d) = out_mult * out_base^d, cosine and sine parts
// alike; the input powers are applied first, in place, so that only one
// order's results are held apart
template <int P>
__device__ __forceinline__ void ztrans(float* X, const float* __restrict__ At, float in_base, float out_base,
                                       float out_mult) {
  constexpr int P1 = P + 1;
  {
    float w = in_base;
#pragma unroll
    for (int n = 1; n <= P; ++n) {
#pragma unroll
      for (int i = 0; i < 2 * n + 1; ++i) X[n * n + i] *= w;
      w *= in_base;
    }
  }
#pragma unroll
  for (int m = 0; m <= P; ++m) {
#pragma unroll
    for (int t = 0; t < (m == 0 ? 1 : 2); ++t) {
      cfloat* A = opaque(At);
      float out[P1];
#pragma unroll
      for (int d = m; d <= P; ++d) {
        float acc = 0.f;
#pragma unroll
        for (int n = m; n <= P; ++n) acc += A[(m * P1 + d) * P1 + n] * X[cidx(n, m, t)];
        out[d] = acc;
      }
#pragma unroll
      for (int d = m; d <= P; ++d) X[cidx(d, m, t)] = out[d];
    }
  }
  float w = out_mult;
#pragma unroll
  for (int d = 0; d <= P; ++d) {
#pragma unroll
    for (int i = 0; i < 2 * d + 1; ++i) X[d * d + i] *= w;
    w *= out_base;
  }
}

__device__ __forceinline__ int level_of3(const LevelView& lv, int64_t gid) {
  int l = 0;
  while (l < lv.L && gid >= lv.gofs[l + 1]) ++l;
  return l;
}

// Persistent waves: each takes the next target of the longest-first order.
// Two waves per SIMD: a pair's expansion and its temporaries fit in 256
// registers up to order 9; order 10 does not fit, and at one wave per SIMD
// the kernel is slower than the matrix-core one
template <int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void
k_m2l_valu(
    LevelView lv, const float* __restrict__ Jn, const float* __restrict__ Jt, const float* __restrict__ A,
    const int* __restrict__ pos,
    const float* __restrict__ Mx, double* __restrict__ Lx, int64_t ntarget, const int32_t* __restrict__ order,
    int* __restrict__ queue) {
  constexpr int NT = (P + 1) * (P + 1);
  constexpr int S = tl::stride(P);
  constexpr int NF = lvl(NT, 6);  // values a lane holds after the exchanges
  const int lane = threadIdx.x & 63;
  for (;;) {
    int kq = 0;
    if (lane == 0) kq = atomicAdd(queue, 1);
    kq = __shfl(kq, 0);
    if (kq >= ntarget) break;
    const int64_t gid = lv.gofs[1] + order[kq];
    const int l = level_of3(lv, gid);
    const int64_t bi = gid - lv.gofs[l];
    const double* geo = lv.geom[l];
    const double cix = geo[bi * 10 + 6], ciy = geo[bi * 10 + 7], ciz = geo[bi * 10 + 8];
    const double rt = geo[bi * 10 + 9] > 0.0 ? geo[bi * 10 + 9] : 1.0;
    const int64_t e0 = lv.w_off[l][bi], e1 = lv.w_off[l][bi + 1];
    const int32_t* widx = lv.w_idx[l];
    const float* Mlev = Mx + (size_t)lv.gofs[l] * S;
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
      const float* src = Mlev + (size_t)j * S;
      constexpr PosTab<P> kPos = make_pos<P>();
      static_assert(kPos.v[0] >= 0, "tile layout map");
#pragma unroll
      for (int k = 0; k < NT; ++k) X[k] = src[kPos.v[k]];

      // the steps are kept apart in the schedule (interleaving them only
      // raises the number of live values)
#define FMM_STEP(x)                      \
  x;                                     \
  __builtin_amdgcn_sched_barrier(0)
      FMM_STEP(rotz<P>(X, cb, sb, -1.0));
      FMM_STEP((japply<P, true>(X, Jt)));
      FMM_STEP(rotz<P>(X, ca, sa, -1.0));
      FMM_STEP((japply<P, false>(X, Jn)));
      FMM_STEP(ztrans<P>(X, A, in_base, out_base, out_mult));
      FMM_STEP((japply<P, true>(X, Jt)));
      FMM_STEP(rotz<P>(X, ca, sa, 1.0));
      FMM_STEP((japply<P, false>(X, Jn)));
      FMM_STEP(rotz<P>(X, cb, sb, 1.0));
#undef FMM_STEP

      // sum over the 64 lanes: six halving exchanges; at the exchange with
      // lane distance d the lanes with bit d clear keep the lower half
#define FMM_HALVE(SRC, N_SRC, DST, N_DST, DIST)                          \
  float DST[N_DST];                                                     \
  {                                                                     \
    const bool up = (lane & (DIST)) != 0;                               \
    _Pragma("unroll") for (int i = 0; i < (N_DST); ++i) {               \
      const int ih = (N_DST) + i < (N_SRC) ? (N_DST) + i : (N_SRC) - 1; \
      const float lo = SRC[i];                                          \
      const float hi = (N_DST) + i < (N_SRC) ? SRC[ih] : 0.f;           \
      const float send = up ? lo : hi;                                  \
      const float keep = up ? hi : lo;                                  \
      DST[i] = keep + __shfl_xor(send, (DIST));                         \
      /* a few exchanges in flight at a time: bounded registers */      \
      if ((i & 7) == 7) __builtin_amdgcn_sched_barrier(0);              \
    }                                                                   \
  }
      FMM_HALVE(X, NT, h1, lvl(NT, 1), 32)
      FMM_HALVE(h1, lvl(NT, 1), h2, lvl(NT, 2), 16)
      FMM_HALVE(h2, lvl(NT, 2), h3, lvl(NT, 3), 8)
      FMM_HALVE(h3, lvl(NT, 3), h4, lvl(NT, 4), 4)
      FMM_HALVE(h4, lvl(NT, 4), h5, lvl(NT, 5), 2)
      FMM_HALVE(h5, lvl(NT, 5), h6, lvl(NT, 6), 1)
#undef FMM_HALVE
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

__global__ void k_zero_queue_v(int* queue) {
  if (threadIdx.x == 0) *queue = 0;
}

template <int P>
void launch_one_valu(const Tree& t, const Tables& tb, const float* Mf, double* Lx, hipStream_t s) {
  const int64_t ntarget = t.nbox_total - 1;
  static const int grid_max = [] {
    int dev = 0, ncu = 0, per = 0;
    HIPCHECK(hipGetDevice(&dev));
    HIPCHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_m2l_valu<P>, 256, 0));
    return ncu * (per > 0 ? per : 1);
  }();
  const int64_t need = (ntarget + 3) / 4;
  const unsigned grid = (unsigned)(need < grid_max ? need : grid_max);
  int* queue = (int*)dalloc(sizeof(int), s);
  k_zero_queue_v<<<1, 64, 0, s>>>(queue);
  HIPCHECK(hipGetLastError());
  k_m2l_valu<P><<<grid, 256, 0, s>>>(t.view(), tb.J32, tb.JT32, tb.A32, tb.pos, Mf, Lx, ntarget, t.m2l_order,
                                     queue);
  HIPCHECK(hipGetLastError());
  dfree(queue, s);
}

}  // namespace

// the vector kernel for the scaled binary32 multipoles Mf (tile layout);
// false above order 9, where the matrix-core kernel is the faster one
bool launch_m2l_valu32(const Tree& t, const Tables& tb, const float* Mf, double* Lx, hipStream_t s) {
  switch (tb.p) {
    case 0: launch_one_valu<0>(t, tb, Mf, Lx, s); break;
    case 1: launch_one_valu<1>(t, tb, Mf, Lx, s); break;
    case 2: launch_one_valu<2>(t, tb, Mf, Lx, s); break;
    case 3: launch_one_valu<3>(t, tb, Mf, Lx, s); break;
    case 4: launch_one_valu<4>(t, tb, Mf, Lx, s); break;
    case 5: launch_one_valu<5>(t, tb, Mf, Lx, s); break;
    case 6: launch_one_valu<6>(t, tb, Mf, Lx, s); break;
    case 7: launch_one_valu<7>(t, tb, Mf, Lx, s); break;
    case 8: launch_one_valu<8>(t, tb, Mf, Lx, s); break;
    case 9: launch_one_valu<9>(t, tb, Mf, Lx, s); break;
    default: return false;
  }
  return true;
}

}  // namespace fmm
