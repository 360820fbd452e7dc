// Tile layout of one expansion (orders p <= 15) for the MFMA translation
// kernel.
//
// The (p+1)^2 real coefficients are split per degree n into a cosine block
// c_n = (c_{n,0..n}) and a sine block s_n = (s_{n,0..n}) (s_{n,0} is an
// always-zero slot), and the blocks are packed into tiles of 16 slots:
//   pair tiles    {c_a at slots 0..a, c_b at a+1..p} and the same for s,
//                 b = p-1-a, for a = 0 .. npairs-1 (a < b);
//   a mixed tile  {c_h at 0..h, s_h at 8..8+h}, h = (p-1)/2, when p is odd;
//   top tiles     {c_p at 0..p} and {s_p at 0..p}.
// A rotation about y keeps c and s blocks apart and a rotation about z mixes
// c_{n,m} with s_{n,m}; with this packing the two always sit at the same slot
// of the partner tile (or 8 slots further in the mixed tile), i.e. in the same
// lane of the 16x16x4 MFMA layout, where lane (pair P, group g) holds the
// slots 4i + g, i = 0..3.  In memory a tile is stored as [g][i] so that each
// lane reads 4 consecutive doubles.
#pragma once

namespace fmm {
namespace tl {

constexpr int kMaxP = 15;

__host__ __device__ constexpr int npairs(int p) { return p / 2; }
__host__ __device__ constexpr bool has_mixed(int p) { return (p & 1) != 0; }
__host__ __device__ constexpr int ntiles(int p) { return 2 * npairs(p) + (has_mixed(p) ? 1 : 0) + 2; }
__host__ __device__ constexpr int stride(int p) { return 16 * ntiles(p); }
__host__ __device__ constexpr int mixed_tile(int p) { return 2 * npairs(p); }
__host__ __device__ constexpr int top_c(int p) { return 2 * npairs(p) + (has_mixed(p) ? 1 : 0); }
__host__ __device__ constexpr int top_s(int p) { return top_c(p) + 1; }
// storage position of slot s of tile t
__host__ __device__ constexpr int spos(int t, int s) { return 16 * t + 4 * (s & 3) + (s >> 2); }
// first row of order m in the z-translation buffer (rows (m, n), n = m..p)
__host__ __device__ constexpr int zoff(int p, int m) { return m * (p + 1) - m * (m - 1) / 2; }
__host__ __device__ constexpr int zrows(int p) { return zoff(p, p + 1); }
// k-steps of 4 of the order-m z-translation (p + 1 - m rows), and the first
// step of order m in the operator table
__host__ __device__ constexpr int hsteps(int p, int m) { return (p + 1 - m + 3) / 4; }
__host__ __device__ constexpr int hoff(int p, int m) {
  int o = 0;
  for (int k = 0; k < m; ++k) o += hsteps(p, k);
  return o;
}

struct Slot {
  int n, m;
  int sine;   // 0 = cosine block, 1 = sine block
  int valid;  // 1 if the slot holds a real coefficient
};

__host__ __device__ constexpr Slot decode(int p, int t, int s) {
  const int np = npairs(p);
  if (t < 2 * np) {
    const int a = t < np ? t : t - np;
    const int b = p - 1 - a;
    const int sine = t < np ? 0 : 1;
    int n = -1, m = 0;
    if (s <= a) {
      n = a;
      m = s;
    } else if (s <= a + 1 + b) {
      n = b;
      m = s - a - 1;
    }
    return Slot{n < 0 ? 0 : n, m, sine, (n >= 0 && !(sine && m == 0)) ? 1 : 0};
  }
  if (has_mixed(p) && t == mixed_tile(p)) {
    const int h = (p - 1) / 2;
    if (s <= h) return Slot{h, s, 0, 1};
    if (s >= 8 && s <= 8 + h) return Slot{h, s - 8, 1, (s - 8) > 0 ? 1 : 0};
    return Slot{0, 0, 0, 0};
  }
  const int sine = (t == top_s(p)) ? 1 : 0;
  if (s <= p) return Slot{p, s, sine, (sine && s == 0) ? 0 : 1};
  return Slot{0, 0, 0, 0};
}

}  // namespace tl
}  // namespace fmm
