// theta-criterion connectivity (Section 2.1.1, eq. (2.2); Algorithm 2 on one
// process).  Level 0: the root is strongly connected to itself.  On level l
// the candidates of box i are the eight children of every box strongly
// connected to the parent of i, in ascending order; a distinct candidate j
// with centre distance d > 0 is weakly connected iff R + theta*r <= theta*d
// (R, r the larger and smaller radius), otherwise strongly connected.  The
// lists are CSR by target box: a count pass (which keeps every outcome as a
// bit), a scan, and a fill pass over the same candidates in the same order,
// so each row comes out in ascending order.
#include <algorithm>

#include "fmm_internal.h"

namespace fmm {
namespace {

// eq. (2.2) for box i (geometry gi) and a candidate with centre (cjx, cjy,
// cjz) and radius rj; evaluated as written, without FMA contraction
__device__ __forceinline__ bool is_weak(const double* gi, double cjx, double cjy, double cjz, double rj,
                                        double theta) {
#pragma clang fp contract(off)
  const double dx = gi[6] - cjx, dy = gi[7] - cjy, dz = gi[8] - cjz;
  const double d = sqrt((dx * dx + dy * dy) + dz * dz);
  if (!(d > 0.0)) return false;
  const double ri = gi[9];
  const double R = ri > rj ? ri : rj;
  const double r = ri > rj ? rj : ri;
  return R + theta * r <= theta * d;
}

// One wave per target box i; lanes take 64 consecutive candidates at a time
// and a ballot compacts them, so each row keeps ascending candidate order.
// kListGroups groups of 64 candidates are in flight together: their index and
// geometry loads are issued before any of them is tested.
constexpr int kListGroups = 4;

// A block (one wave) takes one box.  Blocks are dispatched to the eight XCDs
// in turn; they are mapped to boxes so that each XCD takes a contiguous run
// of boxes in tree order, whose candidates (children of nearby parents'
// strong lists) overlap and stay in that XCD's L2.  The grid is
// 8 ceil(nbox / 8) blocks; indexes past the last box return.
__device__ __forceinline__ int64_t xcd_box(int64_t nbox) {
  const int64_t per = (nbox + 7) / 8;
  return (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
}

// Candidate centre and radius as one 32-byte record per box (one load per
// candidate instead of four at the 80-byte stride of the box geometry).
__global__ void k_centre_radius(int64_t nbox, const double* __restrict__ geom, double4* __restrict__ cr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nbox) cr[i] = make_double4(geom[i * 10 + 6], geom[i * 10 + 7], geom[i * 10 + 8], geom[i * 10 + 9]);
}

// 64-bit mask words per child of each parent: ceil(8 |strong(parent)| / 64)
__global__ void k_mask_words(int64_t npar, const int64_t* __restrict__ ps_off, int32_t* __restrict__ words) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < npar) words[p] = (int32_t)((ps_off[p + 1] - ps_off[p] + 7) / 8);
}

// Count pass: the theta test of every candidate of box i; the weak outcome
// of each group of 64 candidates is kept as one mask word (box i's words
// start at 8 wofs[parent] + child * words[parent]), and the counts of the
// row are written.
__global__ __launch_bounds__(64) void k_lists_count(int64_t nbox, const double* __restrict__ geom,
                                                     const double4* __restrict__ cr,
                                                     const int64_t* __restrict__ ps_off,
                                                     const int32_t* __restrict__ ps_idx, double theta,
                                                     const int64_t* __restrict__ wofs,
                                                     const int32_t* __restrict__ words,
                                                     uint64_t* __restrict__ mask, int32_t* __restrict__ ns,
                                                     int32_t* __restrict__ nw) {
  const int lane = threadIdx.x & 63;
  const int64_t i = xcd_box(nbox);
  if (i >= nbox) return;
  const int64_t par = i >> 3;
  const double* gi = geom + i * 10;
  const int64_t e0 = ps_off[par];
  const int64_t ncand = 8 * (ps_off[par + 1] - e0);
  uint64_t* mrow = mask + 8 * wofs[par] + (i & 7) * (int64_t)words[par];
  int64_t cs = 0, cw = 0;
  for (int64_t k0 = 0; k0 < ncand; k0 += 64 * kListGroups) {
    int64_t j[kListGroups];
    bool valid[kListGroups];
#pragma unroll
    for (int u = 0; u < kListGroups; ++u) {
      const int64_t k = k0 + 64 * u + lane;
      valid[u] = k < ncand;
      j[u] = valid[u] ? 8 * (int64_t)ps_idx[e0 + (k >> 3)] + (k & 7) : i;
    }
    double4 c[kListGroups];
#pragma unroll
    for (int u = 0; u < kListGroups; ++u) c[u] = cr[j[u]];
#pragma unroll
    for (int u = 0; u < kListGroups; ++u) {
      const bool weak = valid[u] && (j[u] != i) && is_weak(gi, c[u].x, c[u].y, c[u].z, c[u].w, theta);
      const bool strong = valid[u] && !weak;
      const uint64_t mw = __ballot(weak), ms = __ballot(strong);
      const int64_t g = k0 / 64 + u;
      if (lane == 0 && 64 * g < ncand) mrow[g] = mw;
      cw += __popcll(mw);
      cs += __popcll(ms);
    }
  }
  if (lane == 0) {
    ns[i] = (int32_t)cs;
    nw[i] = (int32_t)cw;
  }
}

// Fill pass: the candidates again, in the same order, sorted into the rows
// by the count pass's mask words (no geometry, no test).
__global__ __launch_bounds__(64) void k_lists_fill(int64_t nbox, const int64_t* __restrict__ ps_off,
                                                    const int32_t* __restrict__ ps_idx,
                                                    const int64_t* __restrict__ wofs,
                                                    const int32_t* __restrict__ words,
                                                    const uint64_t* __restrict__ mask,
                                                    const int64_t* __restrict__ s_off, int32_t* __restrict__ s_idx,
                                                    const int64_t* __restrict__ w_off, int32_t* __restrict__ w_idx) {
  const int lane = threadIdx.x & 63;
  const int64_t i = xcd_box(nbox);
  if (i >= nbox) return;
  const int64_t par = i >> 3;
  const int64_t e0 = ps_off[par];
  const int64_t ncand = 8 * (ps_off[par + 1] - e0);
  const uint64_t* mrow = mask + 8 * wofs[par] + (i & 7) * (int64_t)words[par];
  const uint64_t below = (1ull << lane) - 1ull;
  const int64_t so = s_off[i], wo = w_off[i];
  int64_t cs = 0, cw = 0;
  for (int64_t k0 = 0; k0 < ncand; k0 += 64 * kListGroups) {
    int32_t j[kListGroups];
#pragma unroll
    for (int u = 0; u < kListGroups; ++u) {
      const int64_t k = k0 + 64 * u + lane;
      j[u] = k < ncand ? 8 * ps_idx[e0 + (k >> 3)] + (int32_t)(k & 7) : 0;
    }
#pragma unroll
    for (int u = 0; u < kListGroups; ++u) {
      const int64_t g = k0 / 64 + u;
      if (64 * g >= ncand) break;
      const int64_t left = ncand - 64 * g;
      const uint64_t vm = left >= 64 ? ~0ull : ((1ull << left) - 1ull);
      const uint64_t mw = mrow[g], ms = vm & ~mw;
      if ((mw >> lane) & 1ull) w_idx[wo + cw + __popcll(mw & below)] = j[u];
      if ((ms >> lane) & 1ull) s_idx[so + cs + __popcll(ms & below)] = j[u];
      cw += __popcll(mw);
      cs += __popcll(ms);
    }
  }
}

// M2L work order, longest weak list first: targets are binned by list length
// (bin 0 = longest), the bins scanned, then scattered.  The order within a
// bin is not fixed; it only schedules work, every target's result is the same.
constexpr int kOrderBins = 4096;
// A workgroup takes kOrderChunk consecutive boxes and counts them per bin in
// LDS, then makes one global atomic per nonzero bin: most lists of a deep
// level can fall into one bin (the longest), where an atomic per box would
// serialise.
constexpr int64_t kOrderChunk = 16384;

__device__ __forceinline__ int order_bin(int64_t c) {
  return kOrderBins - 1 - (int)(c < kOrderBins - 1 ? c : kOrderBins - 1);
}

__global__ __launch_bounds__(256) void k_order_hist(int64_t nbox, const int64_t* __restrict__ w_off,
                                                    int32_t* __restrict__ hist) {
  __shared__ int32_t h[kOrderBins];
  for (int b = threadIdx.x; b < kOrderBins; b += blockDim.x) h[b] = 0;
  __syncthreads();
  const int64_t i0 = (int64_t)blockIdx.x * kOrderChunk;
  const int64_t i1 = nbox < i0 + kOrderChunk ? nbox : i0 + kOrderChunk;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) atomicAdd(&h[order_bin(w_off[i + 1] - w_off[i])], 1);
  __syncthreads();
  for (int b = threadIdx.x; b < kOrderBins; b += blockDim.x)
    if (h[b] != 0) atomicAdd(&hist[b], h[b]);
}

// The same chunks: the workgroup reserves its run of slots in each bin with
// one global atomic, then hands the slots out from LDS.
__global__ __launch_bounds__(256) void k_order_scatter(int64_t nbox, int64_t gofs, const int64_t* __restrict__ w_off,
                                                       unsigned long long* __restrict__ cursor,
                                                       int32_t* __restrict__ order) {
  __shared__ unsigned long long h[kOrderBins];
  for (int b = threadIdx.x; b < kOrderBins; b += blockDim.x) h[b] = 0;
  __syncthreads();
  const int64_t i0 = (int64_t)blockIdx.x * kOrderChunk;
  const int64_t i1 = nbox < i0 + kOrderChunk ? nbox : i0 + kOrderChunk;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) atomicAdd(&h[order_bin(w_off[i + 1] - w_off[i])], 1ull);
  __syncthreads();
  for (int b = threadIdx.x; b < kOrderBins; b += blockDim.x)
    if (h[b] != 0) h[b] = atomicAdd(&cursor[b], h[b]);
  __syncthreads();
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const unsigned long long pos = atomicAdd(&h[order_bin(w_off[i + 1] - w_off[i])], 1ull);
    order[pos] = (int32_t)(gofs - 1 + i);
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

template <class TIn>
__global__ void k_scan_tiles(const TIn* __restrict__ in, int64_t* __restrict__ out, int64_t n,
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

}  // namespace

namespace {
// level 0: the root is strongly connected to itself and to nothing else
__global__ void k_root_lists(int64_t* __restrict__ s_off, int64_t* __restrict__ w_off, int32_t* __restrict__ s_idx) {
  if (threadIdx.x == 0) {
    s_off[0] = 0;
    s_off[1] = 1;
    w_off[0] = 0;
    w_off[1] = 0;
    s_idx[0] = 0;
  }
}

template <class TIn>
void scan_any(const TIn* in, int64_t* out, int64_t n, int64_t base, hipStream_t s) {
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  int64_t* sums = (int64_t*)dalloc((ntiles + 1) * sizeof(int64_t), s);
  if (ntiles > 0) {
    k_scan_tiles<TIn><<<(unsigned)ntiles, kScanBS, 0, s>>>(in, out, n, sums);
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
}  // namespace

void scan_counts(const int32_t* in, int64_t* out, int64_t n, int64_t base, hipStream_t s) {
  scan_any(in, out, n, base, s);
}
void scan_counts(const int64_t* in, int64_t* out, int64_t n, int64_t base, hipStream_t s) {
  scan_any(in, out, n, base, s);
}

void lists_build(Tree& t, hipStream_t s) {
  const int L = t.L;
  // level 0: root strongly connected to itself
  {
    Level& V = t.lev[0];
    V.s_off = (int64_t*)dalloc(2 * sizeof(int64_t), s);
    V.w_off = (int64_t*)dalloc(2 * sizeof(int64_t), s);
    V.s_idx = (int32_t*)dalloc(sizeof(int32_t), s);
    V.w_idx = nullptr;
    k_root_lists<<<1, 64, 0, s>>>(V.s_off, V.w_off, V.s_idx);
    HIPCHECK(hipGetLastError());
    V.s_nnz = 1;
    V.w_nnz = 0;
  }
  int64_t* tot = host_stage();
  int64_t m2l = 0;
  for (int l = 1; l <= L; ++l) {
    Level& P = t.lev[l - 1];
    Level& V = t.lev[l];
    const int64_t nb = V.nbox;
    const int64_t npar = P.nbox;
    int32_t* ns = (int32_t*)dalloc(nb * sizeof(int32_t), s);
    int32_t* nw = (int32_t*)dalloc(nb * sizeof(int32_t), s);
    double4* cr = (double4*)dalloc(nb * sizeof(double4), s);
    int32_t* words = (int32_t*)dalloc(npar * sizeof(int32_t), s);
    int64_t* wofs = (int64_t*)dalloc((npar + 1) * sizeof(int64_t), s);
    k_centre_radius<<<(unsigned)((nb + 255) / 256), 256, 0, s>>>(nb, V.geom, cr);
    HIPCHECK(hipGetLastError());
    k_mask_words<<<(unsigned)((npar + 255) / 256), 256, 0, s>>>(npar, P.s_off, words);
    HIPCHECK(hipGetLastError());
    scan_counts(words, wofs, npar, 0, s);
    // mask words in all: 8 sum_p ceil(S_p / 8) <= (the parents' strong
    // entries) + 8 npar, known on the host without a read-back
    const int64_t nwords = P.s_nnz + 8 * npar;
    uint64_t* mask = (uint64_t*)dalloc(std::max<int64_t>(1, nwords) * sizeof(uint64_t), s);
    const unsigned grid = (unsigned)(8 * ((nb + 7) / 8));
    k_lists_count<<<grid, 64, 0, s>>>(nb, V.geom, cr, P.s_off, P.s_idx, t.theta, wofs, words, mask, ns, nw);
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
    k_lists_fill<<<grid, 64, 0, s>>>(nb, P.s_off, P.s_idx, wofs, words, mask, V.s_off, V.s_idx, V.w_off,
                                      V.w_idx);
    HIPCHECK(hipGetLastError());
    dfree(mask, s);
    dfree(wofs, s);
    dfree(words, s);
    dfree(cr, s);
    dfree(ns, s);
    dfree(nw, s);
  }
  t.m2l_pairs = m2l;

  // M2L work order over the targets of levels 1..L (box id - 1)
  const int64_t ntarget = t.nbox_total - 1;
  if (ntarget > 0) {
    int32_t* hist = (int32_t*)dalloc(kOrderBins * sizeof(int32_t), s);
    int64_t* cursor = (int64_t*)dalloc((kOrderBins + 1) * sizeof(int64_t), s);
    HIPCHECK(hipMemsetAsync(hist, 0, kOrderBins * sizeof(int32_t), s));
    for (int l = 1; l <= L; ++l) {
      const Level& V = t.lev[l];
      k_order_hist<<<(unsigned)((V.nbox + kOrderChunk - 1) / kOrderChunk), 256, 0, s>>>(V.nbox, V.w_off, hist);
      HIPCHECK(hipGetLastError());
    }
    scan_counts(hist, cursor, kOrderBins, 0, s);
    t.m2l_order = (int32_t*)dalloc(ntarget * sizeof(int32_t), s);
    for (int l = 1; l <= L; ++l) {
      const Level& V = t.lev[l];
      k_order_scatter<<<(unsigned)((V.nbox + kOrderChunk - 1) / kOrderChunk), 256, 0, s>>>(
          V.nbox, V.gofs, V.w_off, (unsigned long long*)cursor, t.m2l_order);
      HIPCHECK(hipGetLastError());
    }
    dfree(hist, s);
    dfree(cursor, s);
  }
}

}  // namespace fmm
