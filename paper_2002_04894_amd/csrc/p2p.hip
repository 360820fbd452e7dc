// Near field (P2P, Algorithm 4) and the evaluation driver (Algorithm 1:
// P2M, M2M; Algorithm 3: M2L, L2L; Algorithm 4: L2P, P2P).
//
// P2P: for every target point t of leaf i and every source s of a leaf j
// strongly connected to i (i itself included), phi_t += q_s / r and
// E_t += q_s (x_t - x_s) / r^3, skipping pairs at distance 0 (this removes
// the self term j = i of eq. (2.1)).  Each target pulls from its full list
// (gather form: no atomics, deterministic).  On clustered data the strong
// lists of a few leaves hold far more sources than the rest, so each list is
// cut into segments of about kP2PSeg source points (a plan made once per
// tree); one 64-lane workgroup takes one segment.  A leaf with one segment
// writes its result directly; the segments of a split leaf write partial sums
// that a second pass adds up in segment order.
#include <algorithm>

#include "fmm_internal.h"
#include "lane_ops.h"
#include "tile_layout.h"

namespace fmm {

void launch_p2m(const Tree& t, const Tables& tb, const double* qt, double* Mx, hipStream_t s);
void launch_m2m(const Tree& t, int l, const Tables& tb, double* Mx, hipStream_t s);
void launch_m2l(const Tree& t, const Tables& tb, const double* Mx, double* Lx, int prec, hipStream_t s);
void launch_l2l(const Tree& t, int l, const Tables& tb, double* Lx, hipStream_t s);
void launch_l2p(const Tree& t, const Tables& tb, const double* Lx, const int32_t* start, const double* px,
                const double* py, const double* pz, double* f0, double* f1, double* f2, double* f3, hipStream_t s);

namespace {

__global__ void k_gather(const double* __restrict__ q, const int32_t* __restrict__ perm, double* __restrict__ qt,
                         int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) qt[i] = q[perm[i]];
}

// 1/sqrt(r2) to full double precision: hardware estimate + one Newton step
// (relative error below 5e-15); 0 for r2 == 0.  The estimate of +0 is +inf,
// whose low word is zero, so clearing its high word gives +0 and the Newton
// step then keeps 0: one select of one word instead of two on the result.
__device__ __forceinline__ double rsqrt_nr(double r2) {
  const double e = __builtin_amdgcn_rsq(r2);
  const long long b = __double_as_longlong(e);
  const int hi = r2 > 0.0 ? (int)(b >> 32) : 0;
  const double y0 = __hiloint2double(hi, (int)b);
  return y0 * (1.5 - 0.5 * r2 * y0 * y0);
}

// Work items (segments, in leaf order) are mapped to blocks so that
// consecutive ones, whose sources overlap, run on the same XCD and share its
// L2.
__device__ __forceinline__ int64_t xcd_leaf(int64_t nleaf) {
  const int64_t per = (nleaf + 7) / 8;
  return (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
}

constexpr int kP2PBuf = 256;     // source points staged per chunk (x, y, z, q): 8 KB of LDS, 3 waves per SIMD
constexpr int64_t kP2PSeg = 8192;  // source points per work item (about)

// ---- the plan: one wave per leaf walks its strong list 64 entries at a
// time.  Entry e starts a segment when it is the first of the list or when
// floor(sources before e / kP2PSeg) changes at e.
__device__ __forceinline__ int64_t wave_incl_scan64(int64_t v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t t = __shfl_up(v, d);
    if (lane >= d) v += t;
  }
  return v;
}

template <bool FILL>
__global__ __launch_bounds__(256) void k_seg_plan(int64_t nleaf, const int32_t* __restrict__ start,
                                                  const int64_t* __restrict__ s_off, const int32_t* __restrict__ s_idx,
                                                  int32_t* __restrict__ nseg, int64_t* __restrict__ work,
                                                  const int64_t* __restrict__ leaf_seg, int32_t* __restrict__ seg_leaf,
                                                  int64_t* __restrict__ seg_e0) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= nleaf) return;
  const int64_t e0 = s_off[i], e1 = s_off[i + 1];
  const uint64_t below = (1ull << lane) - 1ull;
  int64_t carry = 0;  // sources of the entries before this chunk
  int prev_last = 0;  // sources of the entry just before this chunk
  int64_t flags = 0;  // segments started so far
  const int64_t base = FILL ? leaf_seg[i] : 0;
  for (int64_t k0 = e0; k0 < e1; k0 += 64) {
    const int64_t e = k0 + lane;
    const bool valid = e < e1;
    int cnt = 0;
    if (valid) {
      const int j = s_idx[e];
      cnt = start[j + 1] - start[j];
    }
    const int64_t incl = wave_incl_scan64(cnt, lane);
    const int64_t excl = carry + incl - cnt;
    const int up = __shfl_up(cnt, 1);
    const int prev = lane == 0 ? prev_last : up;
    const bool flag = valid && (e == e0 || excl / kP2PSeg != (excl - prev) / kP2PSeg);
    const uint64_t m = __ballot(flag);
    if (FILL && flag) {
      const int64_t pos = base + flags + __popcll(m & below);
      seg_leaf[pos] = (int32_t)i;
      seg_e0[pos] = e;
    }
    flags += __popcll(m);
    carry += __shfl(incl, 63);
    prev_last = __shfl(cnt, 63);
  }
  if (!FILL && lane == 0) {
    nseg[i] = (int32_t)flags;
    work[i] = (int64_t)(start[i + 1] - start[i]) * carry;  // interactions of this leaf
  }
}

// partial sums needed by leaf i: one per target and segment when split
__global__ void k_part_count(int64_t nleaf, const int32_t* __restrict__ start, const int32_t* __restrict__ nseg,
                             int64_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nleaf) cnt[i] = nseg[i] > 1 ? (int64_t)nseg[i] * (start[i + 1] - start[i]) : 0;
}

__global__ void k_sum64(int64_t n, const int64_t* __restrict__ v, unsigned long long* __restrict__ acc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long x = i < n ? (unsigned long long)v[i] : 0ull;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
  if ((threadIdx.x & 63) == 0) atomicAdd(acc, x);
}

// One 64-lane workgroup per segment.  Each lane holds two targets, t and
// t + TT, and one of R = 64 / TT source streams, so every source read from
// LDS serves two interactions.  Sources are staged in chunks of up to kP2PBuf
// points gathered from consecutive entries of the segment: the lanes take the
// chunk's points in a flat order, so all their loads are in flight together.
// The targets of leaf b are [tstart[b], tstart[b+1]) of (tx, ty, tz), written
// to index tperm[.] of the outputs: the leaf's own sources (tstart = start,
// tx = px, tperm = perm) or the separate targets grouped by leaf.
// Binary32 near field (F32): coordinates are taken relative to the target
// leaf's cell centre in binary64 and rounded to binary32, so that the
// differences of nearby points keep binary32 accuracy; 1/r is the hardware
// binary32 reciprocal square root; each lane sums the interactions of one
// staged chunk in binary32 and adds the chunk sums into compensated binary32
// accumulators (Kahan); the results are widened to binary64 before the far
// field is added.  Two distinct points whose relative coordinates round to
// the same binary32 values count as coincident (contribute nothing).
struct Kahan {
  float s = 0.f, c = 0.f;
  __device__ __forceinline__ void add(float v) {
    const float y = v - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
  }
  __device__ __forceinline__ double get() const { return (double)s - (double)c; }
};

template <bool F32>
__global__ __launch_bounds__(64) void k_p2p(int64_t nseg, const int32_t* __restrict__ seg_leaf,
                                            const int64_t* __restrict__ seg_e0, const int64_t* __restrict__ leaf_seg,
                                            const int64_t* __restrict__ leaf_part, const int32_t* __restrict__ start,
                                            const int64_t* __restrict__ s_off, const int32_t* __restrict__ s_idx,
                                            const double* __restrict__ px, const double* __restrict__ py,
                                            const double* __restrict__ pz, const double* __restrict__ qt,
                                            const int32_t* __restrict__ tstart, const double* __restrict__ tx,
                                            const double* __restrict__ ty, const double* __restrict__ tz,
                                            const int32_t* __restrict__ perm, const double* __restrict__ f0,
                                            const double* __restrict__ f1, const double* __restrict__ f2,
                                            const double* __restrict__ f3, double4* __restrict__ part,
                                            double* __restrict__ pot, double* __restrict__ ex,
                                            double* __restrict__ ey, double* __restrict__ ez,
                                            const double* __restrict__ lgeom) {
  __shared__ double4 buf[F32 ? 1 : kP2PBuf];
  __shared__ float4 bufs[F32 ? kP2PBuf : 1];
  const int64_t g = xcd_leaf(nseg);
  if (g >= nseg) return;
  const int lane = threadIdx.x;
  const int64_t b = seg_leaf[g];
  const int64_t sb = leaf_seg[b], ns = leaf_seg[b + 1] - sb, r = g - sb;
  const int64_t e0 = seg_e0[g], e1 = r + 1 < ns ? seg_e0[g + 1] : s_off[b + 1];
  const int t0 = tstart[b], t1 = tstart[b + 1];
  const int nt = t1 - t0;
  double4* pout = ns > 1 ? part + leaf_part[b] + r * nt : nullptr;  // partial sums, by target - t0
  // lanes = (target pair, source stream)
  const int TT = nt <= 16 ? 8 : (nt <= 32 ? 16 : (nt <= 64 ? 32 : 64));
  const int R = 64 / TT;
  const int tl = lane % TT, h = lane / TT;
  double ccx = 0.0, ccy = 0.0, ccz = 0.0;  // binary32 mode: the target leaf's centre
  if (F32) {
    ccx = lgeom[b * 10 + 6];
    ccy = lgeom[b * 10 + 7];
    ccz = lgeom[b * 10 + 8];
  }
  for (int c0 = t0; c0 < t1; c0 += 2 * TT) {
    const int ta = c0 + tl, tb = c0 + tl + TT;
    const bool va = ta < t1, vb = tb < t1;
    const int ua = va ? ta : t0, ub = vb ? tb : t0;
    const double xa = tx[ua], ya = ty[ua], za = tz[ua];
    const double xb = tx[ub], yb = ty[ub], zb = tz[ub];
    double fa = 0.0, gxa = 0.0, gya = 0.0, gza = 0.0;
    double fb = 0.0, gxb = 0.0, gyb = 0.0, gzb = 0.0;
    // binary32: relative target coordinates, chunk sums, compensated totals
    const float xfa = (float)(xa - ccx), yfa = (float)(ya - ccy), zfa = (float)(za - ccz);
    const float xfb = (float)(xb - ccx), yfb = (float)(yb - ccy), zfb = (float)(zb - ccz);
    float sa[4] = {0.f, 0.f, 0.f, 0.f}, sb[4] = {0.f, 0.f, 0.f, 0.f};
    Kahan ka[4], kb[4];
    auto interact32 = [&](const float4 s) {
      {
        const float dx = xfa - s.x, dy = yfa - s.y, dz = zfa - s.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float inv = r2 > 0.f ? __builtin_amdgcn_rsqf(r2) : 0.f;
        const float qi = s.w * inv;
        const float qi3 = qi * inv * inv;
        sa[0] += qi;
        sa[1] += qi3 * dx;
        sa[2] += qi3 * dy;
        sa[3] += qi3 * dz;
      }
      {
        const float dx = xfb - s.x, dy = yfb - s.y, dz = zfb - s.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float inv = r2 > 0.f ? __builtin_amdgcn_rsqf(r2) : 0.f;
        const float qi = s.w * inv;
        const float qi3 = qi * inv * inv;
        sb[0] += qi;
        sb[1] += qi3 * dx;
        sb[2] += qi3 * dy;
        sb[3] += qi3 * dz;
      }
    };
    auto interact = [&](const double4 s) {
      {
        const double dx = xa - s.x, dy = ya - s.y, dz = za - s.z;
        const double inv = rsqrt_nr(dx * dx + dy * dy + dz * dz);
        const double qi = s.w * inv;
        const double qi3 = qi * inv * inv;
        fa += qi;
        gxa += qi3 * dx;
        gya += qi3 * dy;
        gza += qi3 * dz;
      }
      {
        const double dx = xb - s.x, dy = yb - s.y, dz = zb - s.z;
        const double inv = rsqrt_nr(dx * dx + dy * dy + dz * dz);
        const double qi = s.w * inv;
        const double qi3 = qi * inv * inv;
        fb += qi;
        gxb += qi3 * dx;
        gyb += qi3 * dy;
        gzb += qi3 * dz;
      }
    };
    int64_t e = e0;  // next entry
    int off = 0;     // points of entry e already staged
    while (e < e1) {
      // up to 16 entries from e on: lane q < 16 takes entry e + q
      int base = 0, cnt = 0;
      if (lane < 16 && e + lane < e1) {
        const int j = s_idx[e + lane];
        base = start[j] + (lane == 0 ? off : 0);
        cnt = start[j + 1] - base;
      }
      int pre = cnt;  // inclusive prefix over lanes 0..15
#pragma unroll
      for (int d = 1; d < 16; d <<= 1) {
        const int v = __shfl_up(pre, d, 16);
        if ((lane & 15) >= d) pre += v;
      }
      const int all = __shfl(pre, 15);
      const int fill = all < kP2PBuf ? all : kP2PBuf;
      const int avail = (int)(e1 - e < 16 ? e1 - e : 16);
      // flat point f of the chunk lies in entry q: pre[q-1] <= f < pre[q];
      // all loads of the chunk are issued before the LDS stores
      constexpr int kIt = kP2PBuf / 64;
      double4 v[kIt];
#pragma unroll
      for (int it = 0; it < kIt; ++it) {
        const int f = it * 64 + lane;
        int q = 0;
#pragma unroll
        for (int k = 0; k < 15; ++k) q += (__shfl(pre, k) <= f) ? 1 : 0;
        const int lo = __shfl(pre, q) - __shfl(cnt, q);
        const int u = __shfl(base, q) + (f - lo);
        if (f < fill) v[it] = make_double4(px[u], py[u], pz[u], qt[u]);
      }
#pragma unroll
      for (int it = 0; it < kIt; ++it) {
        const int f = it * 64 + lane;
        if (f < fill) {
          if (F32)
            bufs[f] = make_float4((float)(v[it].x - ccx), (float)(v[it].y - ccy), (float)(v[it].z - ccz),
                                  (float)v[it].w);
          else
            buf[f] = v[it];
        }
      }
      // entries staged completely, and how far into the next one
      int done = 0;
#pragma unroll
      for (int k = 0; k < 16; ++k) done += (k < avail && __shfl(pre, k) <= fill) ? 1 : 0;
      if (done < avail) {
        const int prev = done == 0 ? 0 : __shfl(pre, done - 1);
        off = (done == 0 ? off : 0) + (fill - prev);
      } else {
        off = 0;
      }
      e += done;
      __syncthreads();
      int u = h;
      if (F32) {
        for (; u + 3 * R < fill; u += 4 * R) {
          const float4 s0 = bufs[u], s1 = bufs[u + R], s2 = bufs[u + 2 * R], s3 = bufs[u + 3 * R];
          interact32(s0);
          interact32(s1);
          interact32(s2);
          interact32(s3);
        }
        for (; u < fill; u += R) interact32(bufs[u]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          ka[k].add(sa[k]);
          kb[k].add(sb[k]);
          sa[k] = 0.f;
          sb[k] = 0.f;
        }
      } else {
        for (; u + 3 * R < fill; u += 4 * R) {
          const double4 s0 = buf[u], s1 = buf[u + R], s2 = buf[u + 2 * R], s3 = buf[u + 3 * R];
          interact(s0);
          interact(s1);
          interact(s2);
          interact(s3);
        }
        for (; u < fill; u += R) interact(buf[u]);
      }
      __syncthreads();
    }
    if (F32) {
      fa = ka[0].get();
      gxa = ka[1].get();
      gya = ka[2].get();
      gza = ka[3].get();
      fb = kb[0].get();
      gxb = kb[1].get();
      gyb = kb[2].get();
      gzb = kb[3].get();
    }
    // sum the source streams (fixed order)
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      if (d >= TT) {
        fa += __shfl_xor(fa, d);
        gxa += __shfl_xor(gxa, d);
        gya += __shfl_xor(gya, d);
        gza += __shfl_xor(gza, d);
        fb += __shfl_xor(fb, d);
        gxb += __shfl_xor(gxb, d);
        gyb += __shfl_xor(gyb, d);
        gzb += __shfl_xor(gzb, d);
      }
    }
    if (h == 0) {
      auto put = [&](int t, double f, double gx, double gy, double gz) {
        if (pout) {
          pout[t - t0] = make_double4(f, gx, gy, gz);
          return;
        }
        if (f0) {
          f += f0[t];
          gx += f1[t];
          gy += f2[t];
          gz += f3[t];
        }
        const int o = perm[t];
        pot[o] = f;
        ex[o] = gx;
        ey[o] = gy;
        ez[o] = gz;
      };
      if (va) put(ta, fa, gxa, gya, gza);
      if (vb) put(tb, fb, gxb, gyb, gzb);
    }
  }
}

// Results of the leaves not written by k_p2p: with partial sums (NEAR = 1)
// the split leaves, their segments added in order; without the near field
// (NEAR = 0) every leaf.  One wave per leaf, lanes over targets.
template <int NEAR>
__global__ __launch_bounds__(256) void k_p2p_final(int64_t nleaf, const int32_t* __restrict__ start,
                                                   const int64_t* __restrict__ leaf_seg,
                                                   const int64_t* __restrict__ leaf_part,
                                                   const double4* __restrict__ part,
                                                   const int32_t* __restrict__ perm, const double* __restrict__ f0,
                                                   const double* __restrict__ f1, const double* __restrict__ f2,
                                                   const double* __restrict__ f3, double* __restrict__ pot,
                                                   double* __restrict__ ex, double* __restrict__ ey,
                                                   double* __restrict__ ez) {
  const int lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= nleaf) return;
  const int64_t ns = NEAR ? leaf_seg[b + 1] - leaf_seg[b] : 0;
  if (NEAR && ns <= 1) return;
  const int t0 = start[b], t1 = start[b + 1], nt = t1 - t0;
  for (int t = t0 + lane; t < t1; t += 64) {
    double f = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    if (NEAR) {
      const double4* pp = part + leaf_part[b] + (t - t0);
      for (int64_t r = 0; r < ns; ++r) {
        const double4 v = pp[r * nt];
        f += v.x;
        gx += v.y;
        gy += v.z;
        gz += v.w;
      }
    }
    if (f0) {
      f += f0[t];
      gx += f1[t];
      gy += f2[t];
      gz += f3[t];
    }
    const int o = perm[t];
    pot[o] = f;
    ex[o] = gx;
    ey[o] = gy;
    ez[o] = gz;
  }
}

// partial sums needed for the separate targets of leaf i
__global__ void k_tpart_count(int64_t nleaf, const int32_t* __restrict__ tstart, const int64_t* __restrict__ leaf_seg,
                              int64_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nleaf) return;
  const int64_t ns = leaf_seg[i + 1] - leaf_seg[i];
  cnt[i] = ns > 1 ? ns * (int64_t)(tstart[i + 1] - tstart[i]) : 0;
}

}  // namespace

void p2p_plan_targets(Tree& t, hipStream_t s) {
  const int64_t nleaf = t.lev[t.L].nbox;
  int64_t* pcnt = (int64_t*)dalloc(nleaf * sizeof(int64_t), s);
  k_tpart_count<<<(unsigned)((nleaf + 255) / 256), 256, 0, s>>>(nleaf, t.tstart, t.p2p_leaf_seg, pcnt);
  HIPCHECK(hipGetLastError());
  t.p2p_leaf_tpart = (int64_t*)dalloc((nleaf + 1) * sizeof(int64_t), s);
  scan_counts(pcnt, t.p2p_leaf_tpart, nleaf, 0, s);
  int64_t* h = host_stage();
  HIPCHECK(hipMemcpyAsync(h, t.p2p_leaf_tpart + nleaf, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  t.p2p_ntpart = *h;
  dfree(pcnt, s);
}

void p2p_plan(Tree& t, hipStream_t s) {
  const Level& V = t.lev[t.L];
  const int64_t nleaf = V.nbox;
  int32_t* nseg = (int32_t*)dalloc(nleaf * sizeof(int32_t), s);
  int64_t* work = (int64_t*)dalloc(nleaf * sizeof(int64_t), s);
  int64_t* pcnt = (int64_t*)dalloc(nleaf * sizeof(int64_t), s);
  unsigned long long* acc = (unsigned long long*)dalloc(sizeof(unsigned long long), s);
  HIPCHECK(hipMemsetAsync(acc, 0, sizeof(unsigned long long), s));
  const unsigned gw = (unsigned)((nleaf + 3) / 4);
  k_seg_plan<false><<<gw, 256, 0, s>>>(nleaf, V.start, V.s_off, V.s_idx, nseg, work, nullptr, nullptr, nullptr);
  HIPCHECK(hipGetLastError());
  t.p2p_leaf_seg = (int64_t*)dalloc((nleaf + 1) * sizeof(int64_t), s);
  t.p2p_leaf_part = (int64_t*)dalloc((nleaf + 1) * sizeof(int64_t), s);
  scan_counts(nseg, t.p2p_leaf_seg, nleaf, 0, s);
  k_part_count<<<(unsigned)((nleaf + 255) / 256), 256, 0, s>>>(nleaf, V.start, nseg, pcnt);
  HIPCHECK(hipGetLastError());
  scan_counts(pcnt, t.p2p_leaf_part, nleaf, 0, s);
  k_sum64<<<(unsigned)((nleaf + 255) / 256), 256, 0, s>>>(nleaf, work, acc);
  HIPCHECK(hipGetLastError());
  int64_t* h = host_stage();
  HIPCHECK(hipMemcpyAsync(&h[0], t.p2p_leaf_seg + nleaf, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(&h[1], t.p2p_leaf_part + nleaf, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(&h[2], acc, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  t.p2p_nseg = h[0];
  t.p2p_npart = h[1];
  t.p2p_pairs = h[2] - t.n;  // minus the n self pairs
  t.p2p_seg_leaf = (int32_t*)dalloc(std::max<int64_t>(1, t.p2p_nseg) * sizeof(int32_t), s);
  t.p2p_seg_e0 = (int64_t*)dalloc(std::max<int64_t>(1, t.p2p_nseg) * sizeof(int64_t), s);
  k_seg_plan<true><<<gw, 256, 0, s>>>(nleaf, V.start, V.s_off, V.s_idx, nullptr, nullptr, t.p2p_leaf_seg,
                                      t.p2p_seg_leaf, t.p2p_seg_e0);
  HIPCHECK(hipGetLastError());
  dfree(nseg, s);
  dfree(work, s);
  dfree(pcnt, s);
  dfree(acc, s);
}

// prec: FMM_PREC_F64; FMM_PREC_MIXED for the binary32 M2L; FMM_PREC_F32 for
// the binary32 M2L and the binary32 near field (k_p2p<true>: its field loses
// up to a few 1e-5 relative on clustered clouds, through the cancellation among
// near contributions, so it serves loose tolerances only)
namespace {

// Upward and downward passes (Algorithm 1: P2M, M2M; Algorithm 3: M2L, L2L)
// for charges qt in tree order, then L2P at the points (px, py, pz) grouped by
// leaf as [start[b], start[b+1]) into far[0..3] (allocated here).
void far_field(const Tree& t, const double* qt, int p, int prec, const int32_t* start, const double* px,
               const double* py, const double* pz, int64_t npts, double* far[4], hipStream_t s) {
  const int L = t.L;
  PhaseTimer& tm = timer();
  const Tables& tb = tables_for(p, s);
  double* Mx = (double*)dalloc((size_t)t.nbox_total * tb.stride * sizeof(double), s);
  double* Lx = (double*)dalloc((size_t)t.nbox_total * tb.stride * sizeof(double), s);
  for (int k = 0; k < 4; ++k) far[k] = (double*)dalloc(std::max<int64_t>(1, npts) * sizeof(double), s);
  tm.begin(FMM_PH_P2M, s);
  launch_p2m(t, tb, qt, Mx, s);
  tm.end(FMM_PH_P2M, s);
  tm.begin(FMM_PH_M2M, s);
  for (int l = L; l >= 2; --l) launch_m2m(t, l, tb, Mx, s);
  tm.end(FMM_PH_M2M, s);
  tm.begin(FMM_PH_M2L, s);
  launch_m2l(t, tb, Mx, Lx, prec, s);
  tm.end(FMM_PH_M2L, s);
  tm.begin(FMM_PH_L2L, s);
  for (int l = 2; l <= L; ++l) launch_l2l(t, l, tb, Lx, s);
  tm.end(FMM_PH_L2L, s);
  tm.begin(FMM_PH_L2P, s);
  launch_l2p(t, tb, Lx, start, px, py, pz, far[0], far[1], far[2], far[3], s);
  tm.end(FMM_PH_L2P, s);
  dfree(Mx, s);
  dfree(Lx, s);
}

// Near field (P2P) at the points grouped by leaf as [start[b], start[b+1]) of
// (px, py, pz), plus the far field when far[0] is set; results go to index
// perm[.] of the outputs.  leaf_part / npart: partial-sum layout of the split
// leaves for these points.
void near_field_and_store(const Tree& t, const double* qt, int parts, int prec, const int32_t* start,
                          const double* px, const double* py, const double* pz, const int32_t* perm,
                          const int64_t* leaf_part, int64_t npart, double* const far[4], double* pot, double* ex,
                          double* ey, double* ez, hipStream_t s) {
  PhaseTimer& tm = timer();
  const Level& V = t.lev[t.L];
  tm.begin(FMM_PH_P2P, s);
  const unsigned gfin = (unsigned)((V.nbox + 3) / 4);
  if (parts & FMM_PART_NEAR) {
    double4* part = npart > 0 ? (double4*)dalloc(npart * sizeof(double4), s) : nullptr;
    const unsigned grid = (unsigned)(8 * ((t.p2p_nseg + 7) / 8));
    if (prec == FMM_PREC_F32)
      k_p2p<true><<<grid, 64, 0, s>>>(t.p2p_nseg, t.p2p_seg_leaf, t.p2p_seg_e0, t.p2p_leaf_seg, leaf_part, V.start,
                                      V.s_off, V.s_idx, t.px, t.py, t.pz, qt, start, px, py, pz, perm, far[0], far[1],
                                      far[2], far[3], part, pot, ex, ey, ez, V.geom);
    else
      k_p2p<false><<<grid, 64, 0, s>>>(t.p2p_nseg, t.p2p_seg_leaf, t.p2p_seg_e0, t.p2p_leaf_seg, leaf_part, V.start,
                                       V.s_off, V.s_idx, t.px, t.py, t.pz, qt, start, px, py, pz, perm, far[0],
                                       far[1], far[2], far[3], part, pot, ex, ey, ez, V.geom);
    HIPCHECK(hipGetLastError());
    if (part) {
      k_p2p_final<1><<<gfin, 256, 0, s>>>(V.nbox, start, t.p2p_leaf_seg, leaf_part, part, perm, far[0], far[1],
                                         far[2], far[3], pot, ex, ey, ez);
      HIPCHECK(hipGetLastError());
      dfree(part, s);
    }
  } else {
    k_p2p_final<0><<<gfin, 256, 0, s>>>(V.nbox, start, nullptr, nullptr, nullptr, perm, far[0], far[1], far[2],
                                       far[3], pot, ex, ey, ez);
    HIPCHECK(hipGetLastError());
  }
  tm.end(FMM_PH_P2P, s);
}

double* gather_charges(const Tree& t, const double* q, hipStream_t s) {
  double* qt = (double*)dalloc(t.n * sizeof(double), s);
  k_gather<<<(unsigned)((t.n + 255) / 256), 256, 0, s>>>(q, t.perm, qt, t.n);
  HIPCHECK(hipGetLastError());
  return qt;
}

}  // namespace

void evaluate(const Tree& t, const double* q, int p, int parts, int prec, double* pot, double* ex, double* ey,
              double* ez, hipStream_t s) {
  double* qt = gather_charges(t, q, s);
  double* far[4] = {nullptr, nullptr, nullptr, nullptr};
  const Level& V = t.lev[t.L];
  if ((parts & FMM_PART_FAR) && t.L >= 1) far_field(t, qt, p, prec, V.start, t.px, t.py, t.pz, t.n, far, s);
  near_field_and_store(t, qt, parts, prec, V.start, t.px, t.py, t.pz, t.perm, t.p2p_leaf_part, t.p2p_npart, far, pot, ex,
                       ey, ez, s);
  for (int k = 0; k < 4; ++k)
    if (far[k]) dfree(far[k], s);
  dfree(qt, s);
}

size_t eval_scratch_bytes(const Tree& t, int p, int prec) {
  // what evaluate() allocates, at its peak (far_field inside the charges'
  // lifetime, then the near field's partial sums while the far field lives)
  const size_t stride = p <= tl::kMaxP ? (size_t)tl::stride(p) : (size_t)nterms(p);
  const size_t nbox = (size_t)t.nbox_total;
  auto one = [&](int64_t npts, int64_t npart) {
    const size_t qt = (size_t)t.n * 8;
    const size_t far = t.L >= 1 ? 4 * (size_t)std::max<int64_t>(1, npts) * 8 : 0;
    // the M2L kernel's own copy of the multipoles, per box: binary32 dense
    // (per-lane kernel, orders up to 14) or tiled (order 15), else binary64
    // in the quad layout (orders up to 13 and 16..20)
    size_t copy = 0;
    if (prec != FMM_PREC_F64 && p <= 14) copy = (size_t)lops::dense_stride(p) * 4;
    else if (prec != FMM_PREC_F64 && p <= tl::kMaxP) copy = stride * 4;
    else if (p <= 13 || p >= 16) copy = (size_t)lops::nq(p) * 4 * 8;
    size_t expn = 0;
    if (t.L >= 1) expn = 2 * nbox * stride * 8 + 256 + nbox * copy;  // multipoles, locals, M2L queue, copy
    const size_t part = (size_t)std::max<int64_t>(0, npart) * 32;
    return qt + far + std::max(expn, part);
  };
  size_t b = one(t.n, t.p2p_npart);
  if (t.m > 0) b = std::max(b, one(t.m, t.p2p_ntpart));
  return b;
}

// phi and E at the tree's separate targets (outputs in the caller's target
// order): the same passes, with L2P and P2P at the targets grouped by leaf
void evaluate_targets(const Tree& t, const double* q, int p, int parts, int prec, double* pot, double* ex, double* ey,
                      double* ez, hipStream_t s) {
  if (t.m == 0) return;
  double* qt = gather_charges(t, q, s);
  double* far[4] = {nullptr, nullptr, nullptr, nullptr};
  if ((parts & FMM_PART_FAR) && t.L >= 1) far_field(t, qt, p, prec, t.tstart, t.tx, t.ty, t.tz, t.m, far, s);
  near_field_and_store(t, qt, parts, prec, t.tstart, t.tx, t.ty, t.tz, t.tperm, t.p2p_leaf_tpart, t.p2p_ntpart, far, pot,
                       ex, ey, ez, s);
  for (int k = 0; k < 4; ++k)
    if (far[k]) dfree(far[k], s);
  dfree(qt, s);
}

}  // namespace fmm
