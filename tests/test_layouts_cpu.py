"""Host logic of the operand and register layouts that the two per-pair M2L
kernels and the host code packing their operator tables share (the header
paper_2002_04894_amd/csrc/lane_ops.h), compiled for the host with g++ and
checked without a GPU:

  - per-lane kernel: per degree n the two parity classes of the quarter turn
    about x partition the 2n+1 standard indices, class 0 holds n+1 members
    and class 1 n, members ascend, the instruction offsets of the blocks are
    consecutive and the table holds whole groups of 16 instructions;
  - per-quad kernel: every standard coefficient (d, i) of every order up to
    18 sits in exactly one (block, member) slot, the only empty slots are s_0
    and members above d, block 0 holds c_m for even m, the register offsets
    and instruction offsets are consecutive, the table holds J^T beside J up
    to order 18 only, and the tables fit in LDS (160 KB) at every order up to
    20, the highest;
  - the dense binary32 stride covers (p+1)^2 in whole 16-byte loads.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2002_04894_amd", "csrc", "lane_ops.h")

PROGRAM = r"""
#define __host__
#define __device__
#include <cstdio>
#include <vector>
#include "lane_ops.h"
using namespace fmm::lops;
static int fails = 0;
#define CHECK(c, ...) do { if (!(c)) { ++fails; std::printf("FAIL " __VA_ARGS__); std::printf("\n"); } } while (0)
int main() {
  for (int p = 0; p <= 20; ++p) {
    // per-lane kernel
    int u = 0;
    for (int n = 0; n <= p; ++n) {
      std::vector<int> seen(2 * n + 1, 0);
      for (int cls = 0; cls < 2; ++cls) {
        CHECK(j_offset(n, cls) == u, "j_offset p=%d n=%d cls=%d", p, n, cls);
        const int s = cls_size(n, cls);
        CHECK(s == (cls == 0 ? n + 1 : n), "cls_size");
        int prev = -1;
        for (int r = 0; r < s; ++r) {
          const int i = cls_member(n, cls, r);
          CHECK(i >= 0 && i <= 2 * n, "member range n=%d cls=%d r=%d", n, cls, r);
          if (i < 0 || i > 2 * n) continue;
          CHECK(parity_cls(i) == cls, "member class");
          CHECK(i > prev, "members ascend");
          prev = i;
          ++seen[i];
        }
        CHECK(cls_member(n, cls, s) == -1, "no member past the class");
        u += s * chunks(s);
      }
      for (int i = 0; i <= 2 * n; ++i) CHECK(seen[i] == 1, "standard index %d of degree %d covered once", i, n);
    }
    CHECK(n_j(p) == u, "n_j p=%d", p);
    int z = 0;
    for (int m = 0; m <= p; ++m) {
      CHECK(z_offset(p, m) == z, "z_offset");
      z += (p + 1 - m) * chunks(p + 1 - m);
    }
    CHECK(n_z(p) == z, "n_z");
    CHECK(table_floats(p) == 64 * (2 * groups(n_j(p)) + groups(n_z(p))), "table_floats");
    CHECK(table_floats(p) % 64 == 0 && 16 * groups(n_j(p)) >= n_j(p), "whole groups");
    CHECK(dense_stride(p) >= (p + 1) * (p + 1) && dense_stride(p) % 4 == 0 && dense_stride(p) - (p + 1) * (p + 1) < 4,
          "dense_stride p=%d", p);
    // per-quad kernel
    int r = 0, uq = 0;
    for (int d = 0; d <= p; ++d) {
      std::vector<int> seen(2 * d + 1, 0);
      for (int x = 0; x < 2; ++x) {
        CHECK(qbase(d, x) == r, "qbase p=%d d=%d x=%d", p, d, x);
        CHECK(qj_offset(d, x) == uq, "qj_offset");
        r += qreg(d);
        uq += qreg(d) * qreg(d);
        CHECK(4 * qreg(d) >= d + 1 && 4 * (qreg(d) - 1) <= d, "qreg covers the members");
        for (int m = 0; m < 4 * qreg(d); ++m) {
          const int i = qmember(d, x, m);
          if (i < 0) {
            CHECK(m > d || (m == 0 && x == 1), "zero slot d=%d x=%d m=%d", d, x, m);
            continue;
          }
          CHECK(m <= d && i <= 2 * d, "member range");
          // block 0: c_m for even m, s_m for odd m
          const bool cosine = (i == 0) || (i & 1);
          CHECK(cosine == ((m & 1) == x), "block parity d=%d x=%d m=%d", d, x, m);
          CHECK((i == 0 ? 0 : (i + 1) >> 1) == m, "order of the member");
          ++seen[i];
        }
      }
      for (int i = 0; i <= 2 * d; ++i) CHECK(seen[i] == 1, "quad: index %d of degree %d covered once", i, d);
    }
    CHECK(nq(p) == r, "nq");
    CHECK(qj_count(p) == uq, "qj_count");
    CHECK(qtable_has_jt(p) == (p <= 18), "J^T table up to order 18 (p=%d)", p);
    CHECK(qtable_doubles(p) == (p <= 18 ? 2 : 1) * 16 * qj_count(p) + (p + 2) * (p + 1) * (p + 1), "qtable_doubles");
    if (p <= 20) CHECK(qtable_doubles(p) * 8 <= 160 * 1024, "quad tables in LDS (p=%d)", p);
  }
  std::printf(fails ? "%d failures\n" : "ok\n", fails);
  return fails != 0;
}
"""


def test_lane_and_quad_layouts(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    src = tmp_path / "layouts.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "layouts"
    subprocess.run([gxx, "-std=c++17", "-O1", "-I", os.path.dirname(HDR), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok"), out.stdout[-2000:]
