// Near field (P2P, Algorithm 4) and the evaluation driver (Algorithm 1:
// P2M, M2M; Algorithm 3: M2L, L2L; Algorithm 4: L2P, P2P).
//
// P2P: for every target point t of leaf i and every source s of a leaf j
// strongly connected to i (i itself included), phi_t += q_s / r and
// E_t += q_s (x_t - x_s) / r^3, skipping pairs at distance 0 (this removes
// the self term j = i of eq. (2.1)).  Each target pulls from its full list
// (gather form: no atomics, deterministic).  One 64-lane workgroup per leaf,
// lanes over targets (and over 2 or 4 source streams for small leaves);
// source points are staged through LDS and read back as broadcasts.
#include "fmm_internal.h"

namespace fmm {

void launch_p2m(const Tree& t, const Tables& tb, const double* qt, double* Mx, hipStream_t s);
void launch_m2m(const Tree& t, int l, const Tables& tb, double* Mx, hipStream_t s);
void launch_m2l(const Tree& t, const Tables& tb, const double* Mx, double* Lx, hipStream_t s);
void launch_l2l(const Tree& t, int l, const Tables& tb, double* Lx, hipStream_t s);
void launch_l2p(const Tree& t, const Tables& tb, const double* Lx, double* f0, double* f1, double* f2, double* f3,
                hipStream_t s);

namespace {

__global__ void k_gather(const double* __restrict__ q, const int32_t* __restrict__ perm, double* __restrict__ qt,
                         int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) qt[i] = q[perm[i]];
}

// 1/sqrt(r2) to full double precision: hardware estimate + one Newton step
// (relative error below 5e-15); 0 for r2 == 0.
__device__ __forceinline__ double rsqrt_nr(double r2) {
  const double y0 = __builtin_amdgcn_rsq(r2);
  const double y1 = y0 * (1.5 - 0.5 * r2 * y0 * y0);
  return r2 > 0.0 ? y1 : 0.0;
}

// Leaves are mapped to blocks so that consecutive leaves (whose strong
// lists overlap) run on the same XCD and share its L2.
__device__ __forceinline__ int64_t xcd_leaf(int64_t nleaf) {
  const int64_t per = (nleaf + 7) / 8;
  return (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
}

constexpr int kP2PBuf = 512;  // source points staged per round (x, y, z, q)

__global__ __launch_bounds__(64) void k_p2p(int64_t nleaf, const int32_t* __restrict__ start,
                                            const int64_t* __restrict__ s_off, const int32_t* __restrict__ s_idx,
                                            const double* __restrict__ px, const double* __restrict__ py,
                                            const double* __restrict__ pz, const double* __restrict__ qt,
                                            const int32_t* __restrict__ perm, int near,
                                            const double* __restrict__ f0, const double* __restrict__ f1,
                                            const double* __restrict__ f2, const double* __restrict__ f3,
                                            double* __restrict__ pot, double* __restrict__ ex,
                                            double* __restrict__ ey, double* __restrict__ ez) {
  __shared__ double4 buf[kP2PBuf];
  const int64_t b = xcd_leaf(nleaf);
  if (b >= nleaf) return;
  const int lane = threadIdx.x;
  const int t0 = start[b], t1 = start[b + 1];
  const int nt = t1 - t0;
  const int64_t e0 = s_off[b], e1 = s_off[b + 1];
  // lanes = (target, split): small leaves split the sources over 2 or 4 lane groups
  const int TT = nt <= 16 ? 16 : (nt <= 32 ? 32 : 64);
  const int R = 64 / TT;
  const int tl = lane % TT, h = lane / TT;
  for (int c0 = t0; c0 < t1; c0 += TT) {
    const int t = c0 + tl;
    const bool valid = t < t1;
    const int tt = valid ? t : t0;
    const double xt = px[tt], yt = py[tt], zt = pz[tt];
    double f = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    auto interact = [&](const double4 s) {
      const double dx = xt - s.x, dy = yt - s.y, dz = zt - s.z;
      const double r2 = dx * dx + dy * dy + dz * dz;
      const double inv = rsqrt_nr(r2);
      const double qi = s.w * inv;
      const double qi3 = qi * inv * inv;
      f += qi;
      gx += qi3 * dx;
      gy += qi3 * dy;
      gz += qi3 * dz;
    };
    auto flush = [&](int fill) {
      __syncthreads();
      int u = h;
      for (; u + 3 * R < fill; u += 4 * R) {
        const double4 a = buf[u], bb = buf[u + R], c = buf[u + 2 * R], d = buf[u + 3 * R];
        interact(a);
        interact(bb);
        interact(c);
        interact(d);
      }
      for (; u < fill; u += R) interact(buf[u]);
      __syncthreads();
    };
    if (near) {
      int fill = 0;
      for (int64_t e = e0; e < e1; ++e) {
        const int j = s_idx[e];
        int u0 = start[j];
        const int u1 = start[j + 1];
        while (u0 < u1) {
          const int cnt = min(u1 - u0, kP2PBuf - fill);
          for (int k = lane; k < cnt; k += 64)
            buf[fill + k] = make_double4(px[u0 + k], py[u0 + k], pz[u0 + k], qt[u0 + k]);
          fill += cnt;
          u0 += cnt;
          if (fill == kP2PBuf) {
            flush(fill);
            fill = 0;
          }
        }
      }
      if (fill > 0) flush(fill);
    }
    // sum the source splits (fixed order)
    if (R >= 4) {
      f += __shfl_xor(f, 16);
      gx += __shfl_xor(gx, 16);
      gy += __shfl_xor(gy, 16);
      gz += __shfl_xor(gz, 16);
    }
    if (R >= 2) {
      f += __shfl_xor(f, 32);
      gx += __shfl_xor(gx, 32);
      gy += __shfl_xor(gy, 32);
      gz += __shfl_xor(gz, 32);
    }
    if (valid && h == 0) {
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
}

}  // namespace

void evaluate(const Tree& t, const double* q, int p, int parts, double* pot, double* ex, double* ey, double* ez,
              hipStream_t s) {
  const int64_t n = t.n;
  const int L = t.L;
  PhaseTimer& tm = timer();
  double* qt = (double*)dalloc(n * sizeof(double), s);
  k_gather<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(q, t.perm, qt, n);
  HIPCHECK(hipGetLastError());

  double* far[4] = {nullptr, nullptr, nullptr, nullptr};
  const bool do_far = (parts & FMM_PART_FAR) && L >= 1;
  if (do_far) {
    const Tables& tb = tables_for(p, s);
    double* Mx = (double*)dalloc((size_t)t.nbox_total * tb.stride * sizeof(double), s);
    double* Lx = (double*)dalloc((size_t)t.nbox_total * tb.stride * sizeof(double), s);
    for (int k = 0; k < 4; ++k) far[k] = (double*)dalloc(n * sizeof(double), s);
    tm.begin(FMM_PH_P2M, s);
    launch_p2m(t, tb, qt, Mx, s);
    tm.end(FMM_PH_P2M, s);
    tm.begin(FMM_PH_M2M, s);
    for (int l = L; l >= 2; --l) launch_m2m(t, l, tb, Mx, s);
    tm.end(FMM_PH_M2M, s);
    tm.begin(FMM_PH_M2L, s);
    launch_m2l(t, tb, Mx, Lx, s);
    tm.end(FMM_PH_M2L, s);
    tm.begin(FMM_PH_L2L, s);
    for (int l = 2; l <= L; ++l) launch_l2l(t, l, tb, Lx, s);
    tm.end(FMM_PH_L2L, s);
    tm.begin(FMM_PH_L2P, s);
    launch_l2p(t, tb, Lx, far[0], far[1], far[2], far[3], s);
    tm.end(FMM_PH_L2P, s);
    dfree(Mx, s);
    dfree(Lx, s);
  }
  const Level& V = t.lev[L];
  tm.begin(FMM_PH_P2P, s);
  k_p2p<<<(unsigned)(8 * ((V.nbox + 7) / 8)), 64, 0, s>>>(V.nbox, V.start, V.s_off, V.s_idx, t.px, t.py, t.pz, qt, t.perm,
                                        (parts & FMM_PART_NEAR) ? 1 : 0, far[0], far[1], far[2], far[3], pot, ex, ey,
                                        ez);
  HIPCHECK(hipGetLastError());
  tm.end(FMM_PH_P2P, s);
  for (int k = 0; k < 4; ++k)
    if (far[k]) dfree(far[k], s);
  dfree(qt, s);
}

}  // namespace fmm
