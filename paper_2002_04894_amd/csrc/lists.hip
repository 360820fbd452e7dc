// theta-criterion connectivity (Section 2.1.1, eq. (2.2); Algorithm 2 on one
// process).  Level 0: the root is strongly connected to itself.  On level l
// the candidates of box i are the eight children of every box strongly
// connected to the parent of i, in ascending order; a distinct candidate j
// with centre distance d > 0 is weakly connected iff R + theta*r <= theta*d
// (R, r the larger and smaller radius), otherwise strongly connected.  The
// lists are CSR by target box: a count pass, a scan, and a fill pass (the
// same loop writing indices), so each row comes out in ascending order.
#include <algorithm>
#include <numeric>

#include "fmm_internal.h"

namespace fmm {
namespace {

__device__ __forceinline__ bool is_weak(const double* gi, const double* gj, double theta) {
#pragma clang fp contract(off)
  const double dx = gi[6] - gj[6], dy = gi[7] - gj[7], dz = gi[8] - gj[8];
  const double d = sqrt((dx * dx + dy * dy) + dz * dz);
  if (!(d > 0.0)) return false;
  const double ri = gi[9], rj = gj[9];
  const double R = ri > rj ? ri : rj;
  const double r = ri > rj ? rj : ri;
  return R + theta * r <= theta * d;
}

template <bool FILL>
__global__ void k_lists(int64_t nbox, const double* __restrict__ geom, const int64_t* __restrict__ ps_off,
                        const int32_t* __restrict__ ps_idx, double theta, int32_t* __restrict__ ns,
                        int32_t* __restrict__ nw, const int64_t* __restrict__ s_off, int32_t* __restrict__ s_idx,
                        const int64_t* __restrict__ w_off, int32_t* __restrict__ w_idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nbox) return;
  const int64_t par = i >> 3;
  const double* gi = geom + i * 10;
  int cs = 0, cw = 0;
  int64_t so = 0, wo = 0;
  if (FILL) {
    so = s_off[i];
    wo = w_off[i];
  }
  for (int64_t e = ps_off[par]; e < ps_off[par + 1]; ++e) {
    const int64_t J = ps_idx[e];
    for (int c = 0; c < 8; ++c) {
      const int64_t j = 8 * J + c;
      const bool weak = (j != i) && is_weak(gi, geom + j * 10, theta);
      if (weak) {
        if (FILL) w_idx[wo + cw] = (int32_t)j;
        ++cw;
      } else {
        if (FILL) s_idx[so + cs] = (int32_t)j;
        ++cs;
      }
    }
  }
  if (!FILL) {
    ns[i] = cs;
    nw[i] = cw;
  }
}

// ---- exclusive scan: per-block scan, scan of block sums, add ----
constexpr int kScanBS = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanBS * kScanItems;

__device__ __forceinline__ int64_t wave_incl_scan(int64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t t = __shfl_up(v, d);
    if (lane >= d) v += t;
  }
  return v;
}

__device__ __forceinline__ int64_t block_excl_scan64(int64_t v, int64_t* sm, int64_t& total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t inc = wave_incl_scan(v);
  if (lane == 63) sm[wid] = inc;
  __syncthreads();
  int64_t off = 0, tot = 0;
  for (int w = 0; w < kScanBS / 64; ++w) {
    off += (w < wid) ? sm[w] : 0;
    tot += sm[w];
  }
  __syncthreads();
  total = tot;
  return off + inc - v;
}

__global__ void k_scan_tiles(const int32_t* __restrict__ in, int64_t* __restrict__ out, int64_t n,
                             int64_t* __restrict__ tile_sums) {
  __shared__ int64_t sm[kScanBS / 64];
  const int64_t t0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (t0 + k < n) ? in[t0 + k] : 0;
    s += v[k];
  }
  int64_t tot;
  int64_t ex = block_excl_scan64(s, sm, tot);
  for (int k = 0; k < kScanItems; ++k) {
    if (t0 + k < n) out[t0 + k] = ex;
    ex += v[k];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

__global__ void k_scan_sums(int64_t* __restrict__ sums, int64_t ntiles, int64_t base, int64_t* __restrict__ total_out) {
  __shared__ int64_t sm[kScanBS / 64];
  int64_t carry = base;
  for (int64_t c0 = 0; c0 < ntiles; c0 += kScanBS) {
    const int64_t i = c0 + threadIdx.x;
    const int64_t v = i < ntiles ? sums[i] : 0;
    int64_t tot;
    const int64_t ex = block_excl_scan64(v, sm, tot);
    if (i < ntiles) sums[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *total_out = carry;
}

__global__ void k_scan_add(int64_t* __restrict__ out, int64_t n, const int64_t* __restrict__ tile_off) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += tile_off[i / kScanTile];
}

// P2P work count: sum over leaves of n_i * sum_{j in strong(i)} n_j
__global__ void k_p2p_count(int64_t nleaf, const int32_t* __restrict__ start, const int64_t* __restrict__ s_off,
                            const int32_t* __restrict__ s_idx, unsigned long long* __restrict__ acc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long v = 0;
  if (i < nleaf) {
    int64_t src = 0;
    for (int64_t e = s_off[i]; e < s_off[i + 1]; ++e) {
      const int j = s_idx[e];
      src += start[j + 1] - start[j];
    }
    v = (unsigned long long)((int64_t)(start[i + 1] - start[i]) * src);
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
  if ((threadIdx.x & 63) == 0) atomicAdd(acc, v);
}

}  // namespace

void scan_counts(const int32_t* in, int64_t* out, int64_t n, int64_t base, hipStream_t s) {
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  int64_t* sums = (int64_t*)dalloc((ntiles + 1) * sizeof(int64_t), s);
  if (ntiles > 0) {
    k_scan_tiles<<<(unsigned)ntiles, kScanBS, 0, s>>>(in, out, n, sums);
    HIPCHECK(hipGetLastError());
  }
  k_scan_sums<<<1, kScanBS, 0, s>>>(sums, ntiles, base, out + n);
  HIPCHECK(hipGetLastError());
  if (n > 0) {
    k_scan_add<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(out, n, sums);
    HIPCHECK(hipGetLastError());
  }
  dfree(sums, s);
}

void lists_build(Tree& t, hipStream_t s) {
  const int L = t.L;
  // level 0: root strongly connected to itself
  {
    Level& V = t.lev[0];
    const int64_t h_off[2] = {0, 1};
    const int64_t h_woff[2] = {0, 0};
    const int32_t h_idx[1] = {0};
    V.s_off = (int64_t*)dalloc(2 * sizeof(int64_t), s);
    V.w_off = (int64_t*)dalloc(2 * sizeof(int64_t), s);
    V.s_idx = (int32_t*)dalloc(sizeof(int32_t), s);
    V.w_idx = nullptr;
    HIPCHECK(hipMemcpyAsync(V.s_off, h_off, sizeof(h_off), hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(V.w_off, h_woff, sizeof(h_woff), hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(V.s_idx, h_idx, sizeof(h_idx), hipMemcpyHostToDevice, s));
    V.s_nnz = 1;
    V.w_nnz = 0;
    HIPCHECK(hipStreamSynchronize(s));  // host sources above are on the stack
  }
  int64_t* tot = nullptr;
  HIPCHECK(hipHostMalloc((void**)&tot, 2 * sizeof(int64_t), hipHostMallocDefault));
  int64_t m2l = 0;
  for (int l = 1; l <= L; ++l) {
    Level& P = t.lev[l - 1];
    Level& V = t.lev[l];
    const int64_t nb = V.nbox;
    int32_t* ns = (int32_t*)dalloc(nb * sizeof(int32_t), s);
    int32_t* nw = (int32_t*)dalloc(nb * sizeof(int32_t), s);
    const unsigned grid = (unsigned)((nb + 255) / 256);
    k_lists<false><<<grid, 256, 0, s>>>(nb, V.geom, P.s_off, P.s_idx, t.theta, ns, nw, nullptr, nullptr, nullptr,
                                        nullptr);
    HIPCHECK(hipGetLastError());
    V.s_off = (int64_t*)dalloc((nb + 1) * sizeof(int64_t), s);
    V.w_off = (int64_t*)dalloc((nb + 1) * sizeof(int64_t), s);
    scan_counts(ns, V.s_off, nb, 0, s);
    scan_counts(nw, V.w_off, nb, 0, s);
    HIPCHECK(hipMemcpyAsync(&tot[0], V.s_off + nb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(&tot[1], V.w_off + nb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    V.s_nnz = tot[0];
    V.w_nnz = tot[1];
    m2l += V.w_nnz;
    V.s_idx = (int32_t*)dalloc(std::max<int64_t>(1, V.s_nnz) * sizeof(int32_t), s);
    V.w_idx = (int32_t*)dalloc(std::max<int64_t>(1, V.w_nnz) * sizeof(int32_t), s);
    k_lists<true><<<grid, 256, 0, s>>>(nb, V.geom, P.s_off, P.s_idx, t.theta, nullptr, nullptr, V.s_off, V.s_idx,
                                       V.w_off, V.w_idx);
    HIPCHECK(hipGetLastError());
    dfree(ns, s);
    dfree(nw, s);
  }
  HIPCHECK(hipHostFree(tot));
  t.m2l_pairs = m2l;

  // M2L work order: targets of levels 1..L by decreasing weak-list length
  // (ties by box id), so that long lists start first and the tail is short
  const int64_t ntarget = t.nbox_total - 1;
  if (ntarget > 0) {
    std::vector<int64_t> cnt(ntarget);
    std::vector<int64_t> off;
    for (int l = 1; l <= L; ++l) {
      const Level& V = t.lev[l];
      off.resize(V.nbox + 1);
      HIPCHECK(hipMemcpyAsync(off.data(), V.w_off, (V.nbox + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
      HIPCHECK(hipStreamSynchronize(s));
      for (int64_t i = 0; i < V.nbox; ++i) cnt[V.gofs - 1 + i] = off[i + 1] - off[i];
    }
    std::vector<int32_t> ord(ntarget);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return cnt[a] > cnt[b]; });
    t.m2l_order = (int32_t*)dalloc(ntarget * sizeof(int32_t), s);
    HIPCHECK(hipMemcpyAsync(t.m2l_order, ord.data(), ntarget * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIPCHECK(hipStreamSynchronize(s));  // ord is a host temporary
  }
}

void tree_compute_stats(Tree& t, hipStream_t s) {
  const Level& V = t.lev[t.L];
  unsigned long long* acc = (unsigned long long*)dalloc(sizeof(unsigned long long), s);
  HIPCHECK(hipMemsetAsync(acc, 0, sizeof(unsigned long long), s));
  k_p2p_count<<<(unsigned)((V.nbox + 255) / 256), 256, 0, s>>>(V.nbox, V.start, V.s_off, V.s_idx, acc);
  HIPCHECK(hipGetLastError());
  unsigned long long h = 0;
  HIPCHECK(hipMemcpyAsync(&h, acc, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  dfree(acc, s);
  t.p2p_pairs = (int64_t)h - t.n;
}

}  // namespace fmm
