// Balanced tree by median splits (Section 2.1.2 with eta = 1, Algorithm 2 on
// one process), built on the GPU.
//
// Every box of level l < L is split into 8 by three successive bisections;
// bisection round k (k = 0 .. 3L-1) works on the 2^k segments of depth k.
// A segment is one contiguous range of points in tree order.  Per segment:
//   * axis = longest edge of its cell (ties: x, then y, then z);
//   * the rank-floor(n/2) point in the total order (coordinate, original
//     index) is found by an MSB radix select on order-preserving 64-bit keys
//     of the coordinate (the bits shared by the cell's two bounds are skipped;
//     ties are broken by position, which is ascending original index because
//     every partition is stable);
//   * a stable partition moves the low side in front of the high side;
//   * the split plane is the midpoint of the two middle coordinates (the
//     point's coordinate for one point, the cell midpoint for none).
// Child cells are the parent cell cut at the plane; the child number is
// 4*b1 + 2*b2 + b3 with b = 1 for the high side, so the segment index at
// depth 3l is the box index at level l.
#include <algorithm>
#include <vector>

#include "fmm_internal.h"

namespace fmm {
namespace {

__device__ __forceinline__ uint64_t okey(double c) {
  // order-preserving bit pattern; -0.0 is read as +0.0
  const uint64_t b = (uint64_t)__double_as_longlong(c + 0.0);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ void k_canon_copy(const double* __restrict__ x, const double* __restrict__ y,
                             const double* __restrict__ z, double* __restrict__ ox, double* __restrict__ oy,
                             double* __restrict__ oz, int32_t* __restrict__ oid, int64_t n, int* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = x[i] + 0.0, b = y[i] + 0.0, c = z[i] + 0.0;
  const double lim = 1e300;
  if (!(fabs(a) <= lim && fabs(b) <= lim && fabs(c) <= lim)) atomicOr(bad, 1);
  ox[i] = a;
  oy[i] = b;
  oz[i] = c;
  oid[i] = (int32_t)i;
}

// min / max of the three coordinates: per-block partials, then one block
__global__ void k_bbox_partial(const double* __restrict__ x, const double* __restrict__ y,
                               const double* __restrict__ z, int64_t n, double* __restrict__ part) {
  __shared__ double sm[6][4];
  double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double a = x[i], b = y[i], c = z[i];
    v[0] = fmin(v[0], a); v[1] = fmin(v[1], b); v[2] = fmin(v[2], c);
    v[3] = fmax(v[3], a); v[4] = fmax(v[4], b); v[5] = fmax(v[5], c);
  }
  for (int d = 32; d >= 1; d >>= 1)
    for (int k = 0; k < 6; ++k) {
      const double o = __shfl_xor(v[k], d);
      v[k] = k < 3 ? fmin(v[k], o) : fmax(v[k], o);
    }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0)
    for (int k = 0; k < 6; ++k) sm[k][wid] = v[k];
  __syncthreads();
  if (threadIdx.x < 6) {
    const int k = threadIdx.x;
    double r = sm[k][0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = k < 3 ? fmin(r, sm[k][w]) : fmax(r, sm[k][w]);
    part[blockIdx.x * 6 + k] = r;
  }
}

__global__ void k_bbox_final(const double* __restrict__ part, int nparts, int64_t n, double* __restrict__ cells,
                             int32_t* __restrict__ seg_start, int32_t* __restrict__ seg_n) {
  if (threadIdx.x < 6) {
    const int k = threadIdx.x;
    double r = part[k];
    for (int i = 1; i < nparts; ++i) r = k < 3 ? fmin(r, part[i * 6 + k]) : fmax(r, part[i * 6 + k]);
    cells[k] = r;
  }
  if (threadIdx.x == 0) {
    seg_start[0] = 0;
    seg_n[0] = (int32_t)n;
  }
}

// exclusive block scan of ints; also returns the block total
template <int BS>
__device__ __forceinline__ int block_excl_scan(int v, int* sm, int& total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(inc, d);
    if (lane >= d) inc += t;
  }
  if constexpr (BS == 64) {
    total = __shfl(inc, 63);
    return inc - v;
  } else {
    if (lane == 63) sm[wid] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < BS / 64; ++w) {
      const int s = sm[w];
      off += (w < wid) ? s : 0;
      tot += s;
    }
    __syncthreads();
    total = tot;
    return off + inc - v;
  }
}

template <int BS>
__device__ __forceinline__ double block_reduce(double v, bool is_max, double* sm) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const double o = __shfl_xor(v, d);
    v = is_max ? fmax(v, o) : fmin(v, o);
  }
  if constexpr (BS == 64) {
    return v;
  } else {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sm[wid] = v;
    __syncthreads();
    double r = sm[0];
#pragma unroll
    for (int w = 1; w < BS / 64; ++w) r = is_max ? fmax(r, sm[w]) : fmin(r, sm[w]);
    __syncthreads();
    return r;
  }
}

struct SelState {
  uint64_t prefix;
  int shift;
  int rank;
  int cnt;
};

// One bisection round: block b handles segment b of depth `depth`.
template <int BS>
__global__ __launch_bounds__(BS) void k_orb_round(
    const double* __restrict__ xin, const double* __restrict__ yin, const double* __restrict__ zin,
    const int32_t* __restrict__ iin, double* __restrict__ xout, double* __restrict__ yout, double* __restrict__ zout,
    int32_t* __restrict__ iout, double* __restrict__ cells, int32_t* __restrict__ seg_start,
    int32_t* __restrict__ seg_n, int depth) {
#pragma clang fp contract(off)
  __shared__ unsigned hist[256];
  __shared__ SelState st;
  __shared__ int scan_sm[BS / 64 + 1];
  __shared__ double red_sm[BS / 64 + 1];
  const int tid = threadIdx.x;
  const int64_t base = ((int64_t)1 << depth) - 1;
  const int64_t seg = base + blockIdx.x;
  const int start = seg_start[seg];
  const int n = seg_n[seg];
  double lo[3], hi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = cells[seg * 6 + a];
    hi[a] = cells[seg * 6 + 3 + a];
  }
  int axis = 0;
  double ext = hi[0] - lo[0];
  if (hi[1] - lo[1] > ext) { ext = hi[1] - lo[1]; axis = 1; }
  if (hi[2] - lo[2] > ext) { ext = hi[2] - lo[2]; axis = 2; }
  const double* cin = axis == 0 ? xin : (axis == 1 ? yin : zin);
  const int m = n / 2;
  double plane;

  if (n < 2) {
    if (n == 1) {
      // lone point: goes to the high side, the plane passes through it
      if (tid == 0) {
        xout[start] = xin[start];
        yout[start] = yin[start];
        zout[start] = zin[start];
        iout[start] = iin[start];
      }
      plane = cin[start];
    } else {
      plane = 0.5 * (lo[axis] + hi[axis]);
    }
  } else {
    // ---- radix select of the rank-m key ----
    if (tid == 0) {
      const uint64_t klo = okey(lo[axis]), khi = okey(hi[axis]);
      const uint64_t dif = klo ^ khi;
      const int sh = dif ? __clzll((long long)dif) : 64;
      st.shift = sh;
      st.prefix = sh == 0 ? 0ull : (klo >> (64 - sh));
      st.rank = m;
      st.cnt = n;
    }
    __syncthreads();
    while (true) {
      const int shift = st.shift;
      const int cnt = st.cnt;
      const uint64_t prefix = st.prefix;
      if (cnt <= 1 || shift >= 64) break;
      const int D = min(8, 64 - shift);
      for (int i = tid; i < 256; i += BS) hist[i] = 0u;
      __syncthreads();
      for (int i = tid; i < n; i += BS) {
        const uint64_t k = okey(cin[start + i]);
        const bool match = (shift == 0) || ((k >> (64 - shift)) == prefix);
        if (match) atomicAdd(&hist[(unsigned)((k << shift) >> (64 - D))], 1u);
      }
      __syncthreads();
      if (tid < 64) {
        const int lane = tid;
        unsigned h[4];
        unsigned s = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          h[q] = hist[lane * 4 + q];
          s += h[q];
        }
        unsigned inc = s;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          const unsigned t = __shfl_up(inc, d);
          if (lane >= d) inc += t;
        }
        const unsigned exc = inc - s;
        const unsigned r = (unsigned)st.rank;
        if (s > 0 && exc <= r && r < inc) {
          unsigned before = exc;
          int q = 0;
          while (before + h[q] <= r) {
            before += h[q];
            ++q;
          }
          st.prefix = (prefix << D) | (uint64_t)(lane * 4 + q);
          st.shift = shift + D;
          st.rank = (int)(r - before);
          st.cnt = (int)h[q];
        }
      }
      __syncthreads();
    }
    const int shift = st.shift;
    const uint64_t prefix = st.prefix;
    const int rank = st.rank;

    // ---- stable partition: low = key-prefix below, or equal and early ----
    int low_base = 0, eq_base = 0;
    double cmax_low = -INFINITY, cmin_high = INFINITY;
    for (int c0 = 0; c0 < n; c0 += BS) {
      const int i = c0 + tid;
      const bool valid = i < n;
      double cx = 0, cy = 0, cz = 0, cc = 0;
      int id = 0;
      bool less = false, match = false;
      if (valid) {
        cx = xin[start + i];
        cy = yin[start + i];
        cz = zin[start + i];
        id = iin[start + i];
        cc = axis == 0 ? cx : (axis == 1 ? cy : cz);
        const uint64_t k = okey(cc);
        const uint64_t top = k >> (64 - shift);  // shift >= 1 here
        less = top < prefix;
        match = top == prefix;
      }
      int eq_tot;
      const int eqr = block_excl_scan<BS>(match ? 1 : 0, scan_sm, eq_tot);
      const bool low = valid && (less || (match && (eq_base + eqr) < rank));
      int low_tot;
      const int lr = block_excl_scan<BS>(low ? 1 : 0, scan_sm, low_tot);
      if (valid) {
        int dst;
        if (low) {
          dst = start + low_base + lr;
          cmax_low = fmax(cmax_low, cc);
        } else {
          dst = start + m + (i - (low_base + lr));
          cmin_high = fmin(cmin_high, cc);
        }
        // low positions stay below start + m and high ones below start + n
        // whenever the selection is right; the guard keeps a wrong selection
        // from writing outside this segment (parity tests would flag it)
        if ((low && dst < start + m) || (!low && dst < start + n)) {
          xout[dst] = cx;
          yout[dst] = cy;
          zout[dst] = cz;
          iout[dst] = id;
        }
      }
      low_base += low_tot;
      eq_base += eq_tot;
    }
    cmax_low = block_reduce<BS>(cmax_low, true, red_sm);
    cmin_high = block_reduce<BS>(cmin_high, false, red_sm);
    plane = 0.5 * (cmax_low + cmin_high);
  }

  if (tid == 0) {
    const int64_t cb = ((int64_t)1 << (depth + 1)) - 1 + 2 * (int64_t)blockIdx.x;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cells[cb * 6 + a] = lo[a];
      cells[cb * 6 + 3 + a] = hi[a];
      cells[(cb + 1) * 6 + a] = lo[a];
      cells[(cb + 1) * 6 + 3 + a] = hi[a];
    }
    cells[cb * 6 + 3 + axis] = plane;
    cells[(cb + 1) * 6 + axis] = plane;
    seg_start[cb] = start;
    seg_n[cb] = m;
    seg_start[cb + 1] = start + m;
    seg_n[cb + 1] = n - m;
  }
}

// ---- the same bisection round for few, large segments: every segment is
// cut into chunks of kChunk points, one block per chunk, and the select /
// partition steps go through per-segment state in global memory ----
constexpr int kChunk = 2048;
constexpr int kChunkBS = 256;
constexpr int kSelPasses = 8;  // 8-bit digits cover the 64-bit key

struct SegSel {
  uint64_t prefix;
  int shift;
  int rank;
  int cnt;
  int axis;
};

__device__ __forceinline__ int seg_axis(const double* lo, const double* hi) {
  int axis = 0;
  double ext = hi[0] - lo[0];
  if (hi[1] - lo[1] > ext) { ext = hi[1] - lo[1]; axis = 1; }
  if (hi[2] - lo[2] > ext) { axis = 2; }
  return axis;
}

// state of segment blockIdx.x; clears its global histogram
__global__ __launch_bounds__(256) void k_mb_init(const double* __restrict__ cells, const int32_t* __restrict__ seg_n,
                                                 int depth, SegSel* __restrict__ sel, unsigned* __restrict__ ghist) {
  const int64_t seg = ((int64_t)1 << depth) - 1 + blockIdx.x;
  ghist[(size_t)blockIdx.x * 256 + threadIdx.x] = 0u;
  if (threadIdx.x != 0) return;
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = cells[seg * 6 + a];
    hi[a] = cells[seg * 6 + 3 + a];
  }
  const int axis = seg_axis(lo, hi);
  const uint64_t klo = okey(lo[axis]), khi = okey(hi[axis]);
  const uint64_t dif = klo ^ khi;
  const int sh = dif ? __clzll((long long)dif) : 64;
  SegSel st;
  st.shift = sh;
  st.prefix = sh == 0 ? 0ull : (klo >> (64 - sh));
  st.rank = seg_n[seg] / 2;
  st.cnt = seg_n[seg];
  st.axis = axis;
  sel[blockIdx.x] = st;
}

// digit histogram of the keys that still match the selected prefix
__global__ __launch_bounds__(kChunkBS) void k_mb_hist(const double* __restrict__ xin, const double* __restrict__ yin,
                                                      const double* __restrict__ zin,
                                                      const int32_t* __restrict__ seg_start,
                                                      const int32_t* __restrict__ seg_n, int depth, int nchunk,
                                                      const SegSel* __restrict__ sel, unsigned* __restrict__ ghist) {
  __shared__ unsigned hist[256];
  const int sg = blockIdx.x / nchunk, c = blockIdx.x % nchunk;
  const SegSel st = sel[sg];
  if (st.cnt <= 1 || st.shift >= 64) return;  // selection finished
  const int64_t seg = ((int64_t)1 << depth) - 1 + sg;
  const int start = seg_start[seg], n = seg_n[seg];
  const int i0 = c * kChunk, i1 = min(n, i0 + kChunk);
  if (i0 >= i1) return;
  const double* cin = st.axis == 0 ? xin : (st.axis == 1 ? yin : zin);
  const int shift = st.shift;
  const int D = min(8, 64 - shift);
  hist[threadIdx.x] = 0u;
  __syncthreads();
  for (int i = i0 + threadIdx.x; i < i1; i += kChunkBS) {
    const uint64_t k = okey(cin[start + i]);
    const bool match = (shift == 0) || ((k >> (64 - shift)) == st.prefix);
    if (match) atomicAdd(&hist[(unsigned)((k << shift) >> (64 - D))], 1u);
  }
  __syncthreads();
  const unsigned h = hist[threadIdx.x];
  if (h) atomicAdd(&ghist[(size_t)sg * 256 + threadIdx.x], h);
}

// pick the digit that holds the wanted rank (one wave per segment)
__global__ __launch_bounds__(64) void k_mb_select(SegSel* __restrict__ sel, unsigned* __restrict__ ghist) {
  const int lane = threadIdx.x;
  SegSel st = sel[blockIdx.x];
  if (st.cnt <= 1 || st.shift >= 64) return;
  const int D = min(8, 64 - st.shift);
  unsigned* hg = ghist + (size_t)blockIdx.x * 256;
  unsigned h[4];
  unsigned s = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    h[q] = hg[lane * 4 + q];
    s += h[q];
    hg[lane * 4 + q] = 0u;
  }
  unsigned inc = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const unsigned t = __shfl_up(inc, d);
    if (lane >= d) inc += t;
  }
  const unsigned exc = inc - s;
  const unsigned r = (unsigned)st.rank;
  if (s > 0 && exc <= r && r < inc) {
    unsigned before = exc;
    int q = 0;
    while (before + h[q] <= r) {
      before += h[q];
      ++q;
    }
    st.prefix = (st.prefix << D) | (uint64_t)(lane * 4 + q);
    st.shift = st.shift + D;
    st.rank = (int)(r - before);
    st.cnt = (int)h[q];
    sel[blockIdx.x] = st;
  }
}

__device__ __forceinline__ void mb_flags(const SegSel& st, double c, bool& less, bool& match) {
  const uint64_t top = okey(c) >> (64 - st.shift);  // shift >= 1 once a pass has run
  less = top < st.prefix;
  match = top == st.prefix;
}

// per chunk: points below the selected prefix, and points matching it
__global__ __launch_bounds__(kChunkBS) void k_mb_count(const double* __restrict__ xin, const double* __restrict__ yin,
                                                       const double* __restrict__ zin,
                                                       const int32_t* __restrict__ seg_start,
                                                       const int32_t* __restrict__ seg_n, int depth, int nchunk,
                                                       const SegSel* __restrict__ sel, int2* __restrict__ ccount) {
  __shared__ int sm[kChunkBS / 64][2];
  const int sg = blockIdx.x / nchunk, c = blockIdx.x % nchunk;
  const SegSel st = sel[sg];
  const int64_t seg = ((int64_t)1 << depth) - 1 + sg;
  const int start = seg_start[seg], n = seg_n[seg];
  const int i0 = c * kChunk, i1 = min(n, i0 + kChunk);
  const double* cin = st.axis == 0 ? xin : (st.axis == 1 ? yin : zin);
  int nl = 0, ne = 0;
  for (int i = i0 + threadIdx.x; i < i1; i += kChunkBS) {
    bool less, match;
    mb_flags(st, cin[start + i], less, match);
    nl += less;
    ne += match;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    nl += __shfl_xor(nl, d);
    ne += __shfl_xor(ne, d);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sm[wid][0] = nl;
    sm[wid][1] = ne;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int a = 0, b = 0;
    for (int w = 0; w < kChunkBS / 64; ++w) {
      a += sm[w][0];
      b += sm[w][1];
    }
    ccount[blockIdx.x] = make_int2(a, b);
  }
}

// per segment: where each chunk's low and equal points start (one wave)
__global__ __launch_bounds__(64) void k_mb_scan(const SegSel* __restrict__ sel, int nchunk,
                                                const int2* __restrict__ ccount, int2* __restrict__ cbase) {
  const int lane = threadIdx.x;
  const int rank = sel[blockIdx.x].rank;
  int low_base = 0, eq_base = 0;
  for (int c0 = 0; c0 < nchunk; c0 += 64) {
    const int c = c0 + lane;
    const int2 v = c < nchunk ? ccount[(size_t)blockIdx.x * nchunk + c] : make_int2(0, 0);
    int e = v.y;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int t = __shfl_up(e, d);
      if (lane >= d) e += t;
    }
    const int eq_exc = eq_base + e - v.y;
    const int take = min(v.y, max(0, rank - eq_exc));  // equal points of this chunk on the low side
    const int lowc = v.x + take;
    int lw = lowc;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int t = __shfl_up(lw, d);
      if (lane >= d) lw += t;
    }
    if (c < nchunk) cbase[(size_t)blockIdx.x * nchunk + c] = make_int2(low_base + lw - lowc, eq_exc);
    low_base += __shfl(lw, 63);
    eq_base += __shfl(e, 63);
  }
}

// stable scatter of one chunk; partial max of the low and min of the high side
__global__ __launch_bounds__(kChunkBS) void k_mb_scatter(
    const double* __restrict__ xin, const double* __restrict__ yin, const double* __restrict__ zin,
    const int32_t* __restrict__ iin, double* __restrict__ xout, double* __restrict__ yout, double* __restrict__ zout,
    int32_t* __restrict__ iout, const int32_t* __restrict__ seg_start, const int32_t* __restrict__ seg_n, int depth,
    int nchunk, const SegSel* __restrict__ sel, const int2* __restrict__ cbase, double2* __restrict__ cpart) {
  __shared__ int scan_sm[kChunkBS / 64 + 1];
  __shared__ double red_sm[kChunkBS / 64 + 1];
  const int sg = blockIdx.x / nchunk, c = blockIdx.x % nchunk;
  const SegSel st = sel[sg];
  const int64_t seg = ((int64_t)1 << depth) - 1 + sg;
  const int start = seg_start[seg], n = seg_n[seg];
  const int m = n / 2;
  const int i0 = c * kChunk, i1 = min(n, i0 + kChunk);
  const int2 bs = cbase[blockIdx.x];
  int low_base = bs.x, eq_base = bs.y;
  double cmax_low = -INFINITY, cmin_high = INFINITY;
  for (int c0 = i0; c0 < i1; c0 += kChunkBS) {  // block-uniform trip count
    const int i = c0 + threadIdx.x;
    const bool valid = i < i1;
    double cx = 0, cy = 0, cz = 0, cc = 0;
    int id = 0;
    bool less = false, match = false;
    if (valid) {
      cx = xin[start + i];
      cy = yin[start + i];
      cz = zin[start + i];
      id = iin[start + i];
      cc = st.axis == 0 ? cx : (st.axis == 1 ? cy : cz);
      mb_flags(st, cc, less, match);
    }
    int eq_tot;
    const int eqr = block_excl_scan<kChunkBS>(match ? 1 : 0, scan_sm, eq_tot);
    const bool low = valid && (less || (match && (eq_base + eqr) < st.rank));
    int low_tot;
    const int lr = block_excl_scan<kChunkBS>(low ? 1 : 0, scan_sm, low_tot);
    if (valid) {
      int dst;
      if (low) {
        dst = start + low_base + lr;
        cmax_low = fmax(cmax_low, cc);
      } else {
        dst = start + m + (i - (low_base + lr));
        cmin_high = fmin(cmin_high, cc);
      }
      // as in the one-block round: a wrong selection cannot write outside
      // the segment
      if ((low && dst < start + m) || (!low && dst >= start + m && dst < start + n)) {
        xout[dst] = cx;
        yout[dst] = cy;
        zout[dst] = cz;
        iout[dst] = id;
      }
    }
    low_base += low_tot;
    eq_base += eq_tot;
  }
  cmax_low = block_reduce<kChunkBS>(cmax_low, true, red_sm);
  cmin_high = block_reduce<kChunkBS>(cmin_high, false, red_sm);
  if (threadIdx.x == 0) cpart[blockIdx.x] = make_double2(cmax_low, cmin_high);
}

// split plane and the two child cells / ranges (one wave per segment)
__global__ __launch_bounds__(64) void k_mb_final(const SegSel* __restrict__ sel, int nchunk,
                                                 const double2* __restrict__ cpart, double* __restrict__ cells,
                                                 int32_t* __restrict__ seg_start, int32_t* __restrict__ seg_n,
                                                 int depth) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x;
  double a = -INFINITY, b = INFINITY;
  for (int c = lane; c < nchunk; c += 64) {
    const double2 v = cpart[(size_t)blockIdx.x * nchunk + c];
    a = fmax(a, v.x);
    b = fmin(b, v.y);
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    a = fmax(a, __shfl_xor(a, d));
    b = fmin(b, __shfl_xor(b, d));
  }
  if (lane != 0) return;
  const int axis = sel[blockIdx.x].axis;
  const double plane = 0.5 * (a + b);
  const int64_t seg = ((int64_t)1 << depth) - 1 + blockIdx.x;
  const int start = seg_start[seg], n = seg_n[seg], m = n / 2;
  const int64_t cb = ((int64_t)1 << (depth + 1)) - 1 + 2 * (int64_t)blockIdx.x;
  for (int k = 0; k < 3; ++k) {
    const double lo = cells[seg * 6 + k], hi = cells[seg * 6 + 3 + k];
    cells[cb * 6 + k] = lo;
    cells[cb * 6 + 3 + k] = hi;
    cells[(cb + 1) * 6 + k] = lo;
    cells[(cb + 1) * 6 + 3 + k] = hi;
  }
  cells[cb * 6 + 3 + axis] = plane;
  cells[(cb + 1) * 6 + axis] = plane;
  seg_start[cb] = start;
  seg_n[cb] = m;
  seg_start[cb + 1] = start + m;
  seg_n[cb + 1] = n - m;
}

// ---- eta < 1 (Section 2.1.2): each split plane of a depth moves from the
// median plane found by the round above to (1 - eta) * (cell midpoint) +
// eta * (median plane), and the depth's points are partitioned again, stably,
// by which side of it they lie on (below = low side) ----
__global__ void k_eta_planes(int64_t nsegd, int depth, double eta, double* __restrict__ cells,
                             double* __restrict__ plane, int* __restrict__ axis_of) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsegd) return;
  const int64_t seg = ((int64_t)1 << depth) - 1 + i;
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = cells[seg * 6 + a];
    hi[a] = cells[seg * 6 + 3 + a];
  }
  int axis = 0;
  double ext = hi[0] - lo[0];
  if (hi[1] - lo[1] > ext) { ext = hi[1] - lo[1]; axis = 1; }
  if (hi[2] - lo[2] > ext) { ext = hi[2] - lo[2]; axis = 2; }
  const int64_t cb = ((int64_t)1 << (depth + 1)) - 1 + 2 * i;
  const double median = cells[cb * 6 + 3 + axis];
  const double mid = 0.5 * (lo[axis] + hi[axis]);
  const double pl = (1.0 - eta) * mid + eta * median;
  cells[cb * 6 + 3 + axis] = pl;
  cells[(cb + 1) * 6 + axis] = pl;
  plane[i] = pl;
  axis_of[i] = axis;
}

// per point of the depth's (pre-split) order: its segment (the last one
// starting at or before it; the segments tile [0, n) in order) and whether it
// lies below that segment's plane
__global__ void k_eta_flags(int64_t n, int depth, int64_t nsegd, const int32_t* __restrict__ seg_start,
                            const double* __restrict__ plane, const int* __restrict__ axis_of,
                            const double* __restrict__ xin, const double* __restrict__ yin,
                            const double* __restrict__ zin, int32_t* __restrict__ flag, int32_t* __restrict__ segof) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t* st = seg_start + ((int64_t)1 << depth) - 1;
  int64_t lo = 0, hi = nsegd - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (st[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  const int a = axis_of[lo];
  const double c = a == 0 ? xin[i] : (a == 1 ? yin[i] : zin[i]);
  flag[i] = c < plane[lo] ? 1 : 0;
  segof[i] = (int32_t)lo;
}

// stable partition by the flags: low side first, each side in its old order
__global__ void k_eta_scatter(int64_t n, int depth, const int32_t* __restrict__ seg_start,
                              const int32_t* __restrict__ seg_n, const int32_t* __restrict__ segof,
                              const int32_t* __restrict__ flag, const int64_t* __restrict__ below,
                              const double* __restrict__ xin, const double* __restrict__ yin,
                              const double* __restrict__ zin, const int32_t* __restrict__ iin,
                              double* __restrict__ xout, double* __restrict__ yout, double* __restrict__ zout,
                              int32_t* __restrict__ iout) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t seg = ((int64_t)1 << depth) - 1 + segof[i];
  const int64_t st = seg_start[seg], ns = seg_n[seg];
  const int64_t b = below[i] - below[st];
  const int64_t nlow = below[st + ns] - below[st];
  const int64_t dst = flag[i] ? st + b : st + nlow + (i - st - b);
  xout[dst] = xin[i];
  yout[dst] = yin[i];
  zout[dst] = zin[i];
  iout[dst] = iin[i];
}

__global__ void k_eta_counts(int64_t nsegd, int depth, const int64_t* __restrict__ below,
                             int32_t* __restrict__ seg_start, int32_t* __restrict__ seg_n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsegd) return;
  const int64_t seg = ((int64_t)1 << depth) - 1 + i;
  const int32_t st = seg_start[seg], ns = seg_n[seg];
  const int32_t nlow = (int32_t)(below[st + ns] - below[st]);
  const int64_t cb = ((int64_t)1 << (depth + 1)) - 1 + 2 * i;
  seg_start[cb] = st;
  seg_n[cb] = nlow;
  seg_start[cb + 1] = st + nlow;
  seg_n[cb + 1] = ns - nlow;
}

// ---- separate targets: the leaf whose cell holds each target (from the
// root, the first of the eight children in child order whose closed cell
// contains it), then the targets grouped by leaf ----
__global__ void k_locate(int64_t m, LevelView lv, const double* __restrict__ tx, const double* __restrict__ ty,
                         const double* __restrict__ tz, int32_t* __restrict__ tleaf, int* __restrict__ bad) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const double v[3] = {tx[k], ty[k], tz[k]};
  int64_t b = 0;
  bool ok = true;
  for (int a = 0; a < 3; ++a) ok = ok && v[a] >= lv.geom[0][a] && v[a] <= lv.geom[0][3 + a];
  for (int l = 1; l <= lv.L && ok; ++l) {
    const double* g = lv.geom[l];
    int64_t found = -1;
    for (int c = 0; c < 8 && found < 0; ++c) {
      const int64_t j = 8 * b + c;
      bool in = true;
      for (int a = 0; a < 3; ++a) in = in && v[a] >= g[j * 10 + a] && v[a] <= g[j * 10 + 3 + a];
      if (in) found = j;
    }
    if (found < 0) ok = false;
    else b = found;
  }
  if (!ok) atomicOr(bad, 1);
  tleaf[k] = ok ? (int32_t)b : 0;
}

__global__ void k_tcount(int64_t m, const int32_t* __restrict__ tleaf, int32_t* __restrict__ cnt) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) atomicAdd(&cnt[tleaf[k]], 1);
}

// targets into their leaf's range; the order inside a leaf is not fixed
// (every target's result depends only on its own position and leaf)
__global__ void k_tscatter(int64_t m, const int32_t* __restrict__ tleaf, const int64_t* __restrict__ off,
                           int32_t* __restrict__ cursor, const double* __restrict__ tx, const double* __restrict__ ty,
                           const double* __restrict__ tz, double* __restrict__ gx, double* __restrict__ gy,
                           double* __restrict__ gz, int32_t* __restrict__ tperm) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const int32_t b = tleaf[k];
  const int64_t dst = off[b] + atomicAdd(&cursor[b], 1);
  gx[dst] = tx[k];
  gy[dst] = ty[k];
  gz[dst] = tz[k];
  tperm[dst] = (int32_t)k;
}

__global__ void k_to_int32(int64_t n, const int64_t* __restrict__ in, int32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= n) out[i] = (int32_t)in[i];
}

// centre = cell centre, radius = half the cell diagonal (Section 2.1.1)
__global__ void k_box_geom(const double* __restrict__ cells, const int32_t* __restrict__ seg_start, int depth,
                           int64_t nbox, double* __restrict__ geom, int32_t* __restrict__ start, int32_t n) {
#pragma clang fp contract(off)
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b > nbox) return;
  if (b == nbox) {
    start[nbox] = n;
    return;
  }
  const int64_t c = ((int64_t)1 << depth) - 1 + b;
  double d[3];
  for (int a = 0; a < 3; ++a) {
    const double lo = cells[c * 6 + a], hi = cells[c * 6 + 3 + a];
    geom[b * 10 + a] = lo;
    geom[b * 10 + 3 + a] = hi;
    geom[b * 10 + 6 + a] = 0.5 * (lo + hi);
    d[a] = hi - lo;
  }
  geom[b * 10 + 9] = 0.5 * sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
  start[b] = seg_start[c];
}

}  // namespace

void tree_build(Tree& t, const double* x, const double* y, const double* z, const double* tx, const double* ty,
                const double* tz, hipStream_t s) {
  const int64_t n = t.n;
  const int L = t.L;
  double* xs[2];
  double* ys[2];
  double* zs[2];
  int32_t* ids[2];
  for (int k = 0; k < 2; ++k) {
    xs[k] = (double*)dalloc(n * sizeof(double), s);
    ys[k] = (double*)dalloc(n * sizeof(double), s);
    zs[k] = (double*)dalloc(n * sizeof(double), s);
    ids[k] = (int32_t*)dalloc(n * sizeof(int32_t), s);
  }
  const int64_t nseg = ((int64_t)2 << (3 * L)) - 1;  // depths 0 .. 3L
  double* cells = (double*)dalloc(nseg * 6 * sizeof(double), s);
  int32_t* seg_start = (int32_t*)dalloc(nseg * sizeof(int32_t), s);
  int32_t* seg_n = (int32_t*)dalloc(nseg * sizeof(int32_t), s);
  int* bad = (int*)dalloc(sizeof(int), s);
  HIPCHECK(hipMemsetAsync(bad, 0, sizeof(int), s));

  const int nb = (int)((n + 255) / 256);
  k_canon_copy<<<nb, 256, 0, s>>>(x, y, z, xs[0], ys[0], zs[0], ids[0], n, bad);
  HIPCHECK(hipGetLastError());
  const int nparts = (int)std::min<int64_t>(1024, (n + 255) / 256);
  const int64_t m = t.m;
  const int nparts_t = m > 0 ? (int)std::min<int64_t>(1024, (m + 255) / 256) : 0;
  double* part = (double*)dalloc((size_t)(nparts + nparts_t) * 6 * sizeof(double), s);
  k_bbox_partial<<<nparts, 256, 0, s>>>(xs[0], ys[0], zs[0], n, part);
  HIPCHECK(hipGetLastError());
  if (m > 0) {
    // canonical copies of the targets (caller's order); they widen the root
    int32_t* tid = (int32_t*)dalloc(m * sizeof(int32_t), s);
    t.tx = (double*)dalloc(m * sizeof(double), s);
    t.ty = (double*)dalloc(m * sizeof(double), s);
    t.tz = (double*)dalloc(m * sizeof(double), s);
    k_canon_copy<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(tx, ty, tz, t.tx, t.ty, t.tz, tid, m, bad);
    HIPCHECK(hipGetLastError());
    dfree(tid, s);
    k_bbox_partial<<<nparts_t, 256, 0, s>>>(t.tx, t.ty, t.tz, m, part + (size_t)nparts * 6);
    HIPCHECK(hipGetLastError());
  }
  k_bbox_final<<<1, 64, 0, s>>>(part, nparts + nparts_t, n, cells, seg_start, seg_n);
  HIPCHECK(hipGetLastError());
  dfree(part, s);
  // eta < 1: per-depth plane and segment scratch for the re-partition
  const bool blend = t.eta < 1.0;
  const int64_t maxsegd = L > 0 ? ((int64_t)1 << (3 * L - 1)) : 1;
  double* eplane = blend ? (double*)dalloc(maxsegd * sizeof(double), s) : nullptr;
  int* eaxis = blend ? (int*)dalloc(maxsegd * sizeof(int), s) : nullptr;
  int32_t* eflag = blend ? (int32_t*)dalloc(n * sizeof(int32_t), s) : nullptr;
  int32_t* esegof = blend ? (int32_t*)dalloc(n * sizeof(int32_t), s) : nullptr;
  int64_t* ebelow = blend ? (int64_t*)dalloc((n + 1) * sizeof(int64_t), s) : nullptr;

  // rounds whose segments all hold at least kMultiMin points (and are few)
  // go through the chunked kernels; the rest run one block per segment
  constexpr int64_t kMultiMin = 4 * kChunk;
  constexpr int64_t kMultiMaxSeg = 512;
  SegSel* sel = nullptr;
  unsigned* ghist = nullptr;
  int2* ccount = nullptr;
  int2* cbase = nullptr;
  double2* cpart = nullptr;
  // the chunked rounds' state, allocated under the condition that selects
  // them below: a round is chunked when it has at most kMultiMaxSeg segments,
  // every one holds at least kMultiMin points and the chunks fit in nblk_cap
  // (the first round, a single segment, whenever n >= kMultiMin).  With
  // eta = 1 the segment sizes follow from n; with eta < 1 children may be
  // unequal, so each round's sizes are read back until a segment is smaller
  // than kMultiMin (its children are no larger, so no later round qualifies).
  const bool any_multi = n >= kMultiMin;
  const int64_t nblk_cap = 2 * ((n + kChunk - 1) / kChunk + kMultiMaxSeg);
  if (any_multi) {
    sel = (SegSel*)dalloc(kMultiMaxSeg * sizeof(SegSel), s);
    ghist = (unsigned*)dalloc(kMultiMaxSeg * 256 * sizeof(unsigned), s);
    ccount = (int2*)dalloc(nblk_cap * sizeof(int2), s);
    cbase = (int2*)dalloc(nblk_cap * sizeof(int2), s);
    cpart = (double2*)dalloc(nblk_cap * sizeof(double2), s);
  }
  std::vector<int32_t> hseg_n;
  bool sizes_ok = true;  // eta < 1: no earlier round had a segment below kMultiMin

  int cur = 0;
  for (int depth = 0; depth < 3 * L; ++depth) {
    const int64_t nsegd = (int64_t)1 << depth;
    const int64_t maxn = (n + nsegd - 1) / nsegd;
    const int64_t minn = n / nsegd;
    const int o = cur ^ 1;
    bool multi = false;
    int64_t seg_max = maxn;
    if (any_multi && nsegd <= kMultiMaxSeg) {
      if (!blend || depth == 0) {
        multi = minn >= kMultiMin;
      } else if (sizes_ok) {
        hseg_n.resize((size_t)nsegd);
        HIPCHECK(hipMemcpyAsync(hseg_n.data(), seg_n + (nsegd - 1), nsegd * sizeof(int32_t), hipMemcpyDeviceToHost,
                                s));
        HIPCHECK(hipStreamSynchronize(s));
        const auto mm = std::minmax_element(hseg_n.begin(), hseg_n.end());
        sizes_ok = *mm.first >= kMultiMin;
        seg_max = *mm.second;
        multi = sizes_ok && nsegd * ((seg_max + kChunk - 1) / kChunk) <= nblk_cap;
      }
    }
    if (multi) {
      const int nchunk = (int)((seg_max + kChunk - 1) / kChunk);
      const unsigned nseg = (unsigned)nsegd, nblk = (unsigned)(nsegd * nchunk);
      k_mb_init<<<nseg, 256, 0, s>>>(cells, seg_n, depth, sel, ghist);
      HIPCHECK(hipGetLastError());
      for (int pass = 0; pass < kSelPasses; ++pass) {
        k_mb_hist<<<nblk, kChunkBS, 0, s>>>(xs[cur], ys[cur], zs[cur], seg_start, seg_n, depth, nchunk, sel, ghist);
        HIPCHECK(hipGetLastError());
        k_mb_select<<<nseg, 64, 0, s>>>(sel, ghist);
        HIPCHECK(hipGetLastError());
      }
      k_mb_count<<<nblk, kChunkBS, 0, s>>>(xs[cur], ys[cur], zs[cur], seg_start, seg_n, depth, nchunk, sel, ccount);
      HIPCHECK(hipGetLastError());
      k_mb_scan<<<nseg, 64, 0, s>>>(sel, nchunk, ccount, cbase);
      HIPCHECK(hipGetLastError());
      k_mb_scatter<<<nblk, kChunkBS, 0, s>>>(xs[cur], ys[cur], zs[cur], ids[cur], xs[o], ys[o], zs[o], ids[o],
                                             seg_start, seg_n, depth, nchunk, sel, cbase, cpart);
      HIPCHECK(hipGetLastError());
      k_mb_final<<<nseg, 64, 0, s>>>(sel, nchunk, cpart, cells, seg_start, seg_n, depth);
      HIPCHECK(hipGetLastError());
    } else if (blend || maxn > 128) {
      k_orb_round<256><<<(unsigned)nsegd, 256, 0, s>>>(xs[cur], ys[cur], zs[cur], ids[cur], xs[o], ys[o], zs[o],
                                                       ids[o], cells, seg_start, seg_n, depth);
    } else {
      k_orb_round<64><<<(unsigned)nsegd, 64, 0, s>>>(xs[cur], ys[cur], zs[cur], ids[cur], xs[o], ys[o], zs[o],
                                                     ids[o], cells, seg_start, seg_n, depth);
    }
    HIPCHECK(hipGetLastError());
    if (blend) {
      const unsigned gs = (unsigned)((nsegd + 255) / 256), gp = (unsigned)((n + 255) / 256);
      k_eta_planes<<<gs, 256, 0, s>>>(nsegd, depth, t.eta, cells, eplane, eaxis);
      HIPCHECK(hipGetLastError());
      k_eta_flags<<<gp, 256, 0, s>>>(n, depth, nsegd, seg_start, eplane, eaxis, xs[cur], ys[cur], zs[cur], eflag,
                                     esegof);
      HIPCHECK(hipGetLastError());
      scan_counts(eflag, ebelow, n, 0, s);
      k_eta_scatter<<<gp, 256, 0, s>>>(n, depth, seg_start, seg_n, esegof, eflag, ebelow, xs[cur], ys[cur], zs[cur],
                                       ids[cur], xs[o], ys[o], zs[o], ids[o]);
      HIPCHECK(hipGetLastError());
      k_eta_counts<<<gs, 256, 0, s>>>(nsegd, depth, ebelow, seg_start, seg_n);
      HIPCHECK(hipGetLastError());
    }
    cur = o;
  }
  if (blend) {
    dfree(eplane, s);
    dfree(eaxis, s);
    dfree(eflag, s);
    dfree(esegof, s);
    dfree(ebelow, s);
  }
  if (sel) {
    dfree(sel, s);
    dfree(ghist, s);
    dfree(ccount, s);
    dfree(cbase, s);
    dfree(cpart, s);
  }

  t.lev.assign(L + 1, Level());
  int64_t g = 0;
  for (int l = 0; l <= L; ++l) {
    Level& V = t.lev[l];
    V.nbox = (int64_t)1 << (3 * l);
    V.gofs = g;
    g += V.nbox;
    V.geom = (double*)dalloc(V.nbox * 10 * sizeof(double), s);
    V.start = (int32_t*)dalloc((V.nbox + 1) * sizeof(int32_t), s);
    k_box_geom<<<(unsigned)((V.nbox + 1 + 255) / 256), 256, 0, s>>>(cells, seg_start, 3 * l, V.nbox, V.geom,
                                                                    V.start, (int32_t)n);
    HIPCHECK(hipGetLastError());
  }
  t.nbox_total = g;
  t.px = xs[cur];
  t.py = ys[cur];
  t.pz = zs[cur];
  t.perm = ids[cur];
  dfree(xs[cur ^ 1], s);
  dfree(ys[cur ^ 1], s);
  dfree(zs[cur ^ 1], s);
  dfree(ids[cur ^ 1], s);
  dfree(cells, s);
  dfree(seg_start, s);
  dfree(seg_n, s);

  int hbad = 0;
  HIPCHECK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  dfree(bad, s);
  if (hbad) fail(FMM_EINVAL, "non-finite coordinate or |coordinate| > 1e300");
}

void targets_build(Tree& t, hipStream_t s) {
  const int64_t m = t.m;
  const int L = t.L;
  const int64_t nleaf = t.lev[L].nbox;
  t.tleaf = (int32_t*)dalloc(std::max<int64_t>(1, m) * sizeof(int32_t), s);
  t.tstart = (int32_t*)dalloc((nleaf + 1) * sizeof(int32_t), s);
  int* bad = (int*)dalloc(sizeof(int), s);
  int32_t* cnt = (int32_t*)dalloc(nleaf * sizeof(int32_t), s);
  int64_t* off = (int64_t*)dalloc((nleaf + 1) * sizeof(int64_t), s);
  HIPCHECK(hipMemsetAsync(bad, 0, sizeof(int), s));
  HIPCHECK(hipMemsetAsync(cnt, 0, nleaf * sizeof(int32_t), s));
  const unsigned gm = (unsigned)((m + 255) / 256);
  if (m > 0) {
    k_locate<<<gm, 256, 0, s>>>(m, t.view(), t.tx, t.ty, t.tz, t.tleaf, bad);
    HIPCHECK(hipGetLastError());
    k_tcount<<<gm, 256, 0, s>>>(m, t.tleaf, cnt);
    HIPCHECK(hipGetLastError());
  }
  scan_counts(cnt, off, nleaf, 0, s);
  k_to_int32<<<(unsigned)((nleaf + 1 + 255) / 256), 256, 0, s>>>(nleaf, off, t.tstart);
  HIPCHECK(hipGetLastError());
  double* gx = (double*)dalloc(std::max<int64_t>(1, m) * sizeof(double), s);
  double* gy = (double*)dalloc(std::max<int64_t>(1, m) * sizeof(double), s);
  double* gz = (double*)dalloc(std::max<int64_t>(1, m) * sizeof(double), s);
  t.tperm = (int32_t*)dalloc(std::max<int64_t>(1, m) * sizeof(int32_t), s);
  if (m > 0) {
    HIPCHECK(hipMemsetAsync(cnt, 0, nleaf * sizeof(int32_t), s));
    k_tscatter<<<gm, 256, 0, s>>>(m, t.tleaf, off, cnt, t.tx, t.ty, t.tz, gx, gy, gz, t.tperm);
    HIPCHECK(hipGetLastError());
  }
  dfree(t.tx, s);
  dfree(t.ty, s);
  dfree(t.tz, s);
  t.tx = gx;
  t.ty = gy;
  t.tz = gz;
  dfree(cnt, s);
  dfree(off, s);
  int hbad = 0;
  HIPCHECK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  dfree(bad, s);
  // every target lies in the root cell, which is widened to hold them
  if (hbad) fail(FMM_EDEVICE, "a target was not found in any leaf cell");
}

}  // namespace fmm
