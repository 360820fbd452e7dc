// Operand order of the per-lane M2L kernel (m2l_lane.hip) on the 16-block
// 4x4x1 matrix instruction, shared by the kernel and by the host code that
// packs its operator tables.
//
// Each lane holds one pair's expansion; a fixed operator block B (s x s) acts
// on s of the lane's coefficients as a sequence of instructions, one per
// (input column k, output chunk c of 4 rows): D_c += B[4c .. 4c+3][k] * x_k.
// The 4 operator values of an instruction are the A operand of one block,
// broadcast to all 16 blocks, so 16 consecutive instructions take theirs from
// one register: the table holds, per group of 16 instructions, 64 values,
// value 4 * (u mod 16) + i = row i of instruction u (zero past the block).
//
// Blocks, in order:
//   J or J^T: per degree n, per parity class cls (0: n+1 members, 1: n), the
//             class members in standard order (the quarter turn about x
//             keeps the classes apart);
//   z core:   per order m, rows d and columns n = m .. P (one table for the
//             cosine and the sine parts, which share it).
#pragma once

namespace fmm {
namespace lops {

// 0 / 1: the two classes of the standard index i within a degree (c_m at
// i = 2m-1, s_m at i = 2m) that the quarter turn about x keeps apart
__host__ __device__ constexpr int parity_cls(int i) {
  return i == 0 ? 0 : ((((i + 1) >> 1) + ((i & 1) ? 0 : 1)) & 1);
}
__host__ __device__ constexpr int cls_size(int n, int cls) { return cls == 0 ? n + 1 : n; }
// r-th member (standard index within degree n) of class cls
__host__ __device__ constexpr int cls_member(int n, int cls, int r) {
  for (int i = 0; i < 2 * n + 1; ++i)
    if (parity_cls(i) == cls && r-- == 0) return i;
  return -1;
}
__host__ __device__ constexpr int chunks(int s) { return (s + 3) / 4; }
// first instruction of block (n, cls) of a J application, and of order m of
// the z translation at expansion order p (its blocks have p + 1 - m rows)
__host__ __device__ constexpr int j_offset(int n, int cls) {
  int u = 0;
  for (int a = 0; a < n; ++a)
    for (int c = 0; c < 2; ++c) u += cls_size(a, c) * chunks(cls_size(a, c));
  return cls == 0 ? u : u + cls_size(n, 0) * chunks(cls_size(n, 0));
}
__host__ __device__ constexpr int z_offset(int p, int m) {
  int u = 0;
  for (int a = 0; a < m; ++a) u += (p + 1 - a) * chunks(p + 1 - a);
  return u;
}
// instructions of one J application and of the z translation (per part)
__host__ __device__ constexpr int n_j(int p) { return j_offset(p + 1, 0); }
__host__ __device__ constexpr int n_z(int p) { return z_offset(p, p + 1); }
__host__ __device__ constexpr int groups(int u) { return (u + 15) / 16; }
// floats per box of the binary32 multipoles the per-lane kernel reads: the
// (p+1)^2 coefficients in the standard order, padded to whole 16-byte loads
__host__ __device__ constexpr int dense_stride(int p) { return ((p + 1) * (p + 1) + 3) & ~3; }
// table floats: J, J^T, z core, each padded to whole groups
__host__ __device__ constexpr int table_floats(int p) { return 64 * (2 * groups(n_j(p)) + groups(n_z(p))); }

// ---- the binary64 per-quad M2L kernel (m2l_quad.hip) on v_mfma_f64_4x4x4f64 ----
//
// A wave takes 16 pairs; lane 16 k + q holds phase k (0..3) of pair q.  Per
// degree d the coefficients form two blocks indexed by the order m = 0..d:
// block 0 holds c_m for even m and s_m for odd m, block 1 the others (its
// member 0, s_0, is a zero slot) -- the two classes that the quarter turn
// about x keeps apart, ordered by m.  Member m of a block sits in phase
// m mod 4, register m / 4 of the block, so that the cosine and sine parts of
// (d, m) share a lane and register index, and all degrees of order m share a
// lane.  A block product takes ceil((d+1)/4)^2 instructions, one per (k-step
// g, output chunk c): D_c += Op[4c .. 4c+3][4g .. 4g+3] X_g; the operand of
// instruction u is 16 values, row i and column k of its 4x4 part at 16 u +
// 4 k + i (the lane layout of the instruction: lane 16 k + 4 b + i holds
// A[i][k] of block b, for every b).
__host__ __device__ constexpr int qreg(int d) { return d / 4 + 1; }
// first register of block (d, x)
__host__ __device__ constexpr int qbase(int d, int x) {
  int r = 0;
  for (int a = 0; a < d; ++a) r += 2 * qreg(a);
  return r + x * qreg(d);
}
__host__ __device__ constexpr int nq(int p) { return qbase(p + 1, 0); }
// standard index within degree d of member m of block x, or -1 for a zero slot
__host__ __device__ constexpr int qmember(int d, int x, int m) {
  if (m > d) return -1;
  if ((m & 1) == x) return m == 0 ? 0 : 2 * m - 1;  // c_m
  return m == 0 ? -1 : 2 * m;                       // s_m
}
// first instruction of block (d, x) in one J application
__host__ __device__ constexpr int qj_offset(int d, int x) {
  int u = 0;
  for (int a = 0; a < d; ++a) u += 2 * qreg(a) * qreg(a);
  return u + x * qreg(d) * qreg(d);
}
__host__ __device__ constexpr int qj_count(int p) { return qj_offset(p + 1, 0); }
// z-translation core A[m][d][n] for m = 0 .. p + 1 (order p + 1 all zero: the
// slot of the lanes whose order exceeds p)
__host__ __device__ constexpr int qcore_doubles(int p) { return (p + 2) * (p + 1) * (p + 1); }
// whether the table holds J^T beside J: where both fit in 160 KB of LDS with
// the core (orders up to 18); above, the kernel reads J^T from J transposed
__host__ __device__ constexpr bool qtable_has_jt(int p) {
  return (2 * 16 * qj_count(p) + qcore_doubles(p)) * 8 <= 160 * 1024;
}
// table: J (16 values per instruction), J^T in the same form if it fits, then
// the z-translation core
__host__ __device__ constexpr int qtable_doubles(int p) {
  return (qtable_has_jt(p) ? 2 : 1) * 16 * qj_count(p) + qcore_doubles(p);
}

}  // namespace lops
}  // namespace fmm
