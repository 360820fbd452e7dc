// Internal declarations of the gfx950 FMM library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/fmm.h"

namespace fmm {

constexpr int kWave = 64;
constexpr int kMaxLevels = FMM_MAX_LEVELS;
constexpr int kMaxOrder = FMM_MAX_ORDER;
// M2M and L2L run four lanes per translation on the matrix cores up to this
// order (two waves per SIMD), the generic binary64 translation above
constexpr int kQuadXlateMaxP = 13;

inline int nterms(int p) { return (p + 1) * (p + 1); }

// Error carrying a status code; caught at the ABI boundary.
struct Error {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg);
void check_hip(hipError_t e, const char* what);
#define HIPCHECK(x) ::fmm::check_hip((x), #x)

// Device allocator: the hook set by fmm_set_allocator, or (all NULL) the
// device's default stream-ordered pool.
struct Allocator {
  fmm_alloc_fn alloc = nullptr;
  fmm_free_fn free = nullptr;
  void* user = nullptr;
};

// Stream-ordered device allocation through the allocator of the current
// entry-point call.  Every allocation is entered in the call's ledger until
// it is freed, so that a call that fails frees what it allocated.
void* dalloc(size_t bytes, hipStream_t s);
void dfree(void* p, hipStream_t s);

// Evaluation scratch carved from one fixed device buffer (the entry point
// that allocates nothing): while an arena is set on this thread, dalloc hands
// out 256-byte aligned slices of it (FMM_EINVAL when it runs out) and dfree
// does nothing.
struct Arena {
  char* base = nullptr;
  size_t size = 0;
  size_t used = 0;
};
void set_arena(Arena* a);  // nullptr: back to the allocator

// 1 if work enqueued on s is being captured into a graph
bool capturing(hipStream_t s);

// Per-thread pinned host words for small device-to-host read-backs (made
// once per thread; kStageWords int64 values).
constexpr int kStageWords = 64;
int64_t* host_stage();

// Per-level box geometry / lists in device memory.
struct Level {
  int64_t nbox = 0;
  int64_t gofs = 0;           // global box id of box 0 of this level
  double* geom = nullptr;     // nbox x 10: lo[3], hi[3], centre[3], radius
  int32_t* start = nullptr;   // nbox + 1 point offsets (tree order)
  int64_t* s_off = nullptr;   // strong CSR (local box indices)
  int32_t* s_idx = nullptr;
  int64_t s_nnz = 0;
  int64_t* w_off = nullptr;   // weak CSR (local box indices)
  int32_t* w_idx = nullptr;
  int64_t w_nnz = 0;
};

// Device-side view of all levels, passed by value to kernels.
struct LevelView {
  int L;
  int64_t gofs[kMaxLevels + 2];
  const double* geom[kMaxLevels + 1];
  const int32_t* start[kMaxLevels + 1];
  const int64_t* s_off[kMaxLevels + 1];
  const int32_t* s_idx[kMaxLevels + 1];
  const int64_t* w_off[kMaxLevels + 1];
  const int32_t* w_idx[kMaxLevels + 1];
};

struct Tree {
  int64_t n = 0;
  int L = 0;
  double theta = 0;
  double eta = 1.0;  // split parameter (Section 2.1.2): 1 = median planes
  hipStream_t stream = nullptr;
  // points in tree order
  double* px = nullptr;
  double* py = nullptr;
  double* pz = nullptr;
  int32_t* perm = nullptr;
  std::vector<Level> lev;     // 0..L
  int64_t nbox_total = 0;     // sum over levels 0..L
  int32_t* m2l_order = nullptr;  // M2L targets (box id - 1), longest weak list first
  int64_t m2l_pairs = 0;
  int64_t p2p_pairs = 0;
  // near-field work items: each leaf's strong list cut into segments of about
  // the same number of source points
  int64_t p2p_nseg = 0;
  int32_t* p2p_seg_leaf = nullptr;   // [nseg] target leaf
  int64_t* p2p_seg_e0 = nullptr;     // [nseg] first strong-list entry
  int64_t* p2p_leaf_seg = nullptr;   // [nleaf + 1] first segment of each leaf
  int64_t* p2p_leaf_part = nullptr;  // [nleaf + 1] first partial sum of each split leaf
  int64_t p2p_npart = 0;             // partial sums (target x segment) of split leaves
  // separate evaluation targets (m may be 0), grouped by the leaf that holds
  // them; before targets_build the coordinate arrays hold the caller's order
  int64_t m = 0;
  double* tx = nullptr;
  double* ty = nullptr;
  double* tz = nullptr;
  int32_t* tperm = nullptr;           // [m] grouped order -> caller's index
  int32_t* tleaf = nullptr;           // [m] leaf of each target, caller's order
  int32_t* tstart = nullptr;          // [nleaf + 1] target range of each leaf
  int64_t* p2p_leaf_tpart = nullptr;  // [nleaf + 1] first partial sum of each split leaf (targets)
  int64_t p2p_ntpart = 0;
  // memory and stream bookkeeping (api.hip)
  Allocator alloc;                 // allocator of the tree's own device memory
  size_t bytes = 0;                // device bytes the tree owns
  hipEvent_t built = nullptr;      // recorded on the build stream when the build is enqueued
  hipStream_t build_stream = nullptr;
  std::vector<std::pair<hipStream_t, hipEvent_t>> uses;  // last evaluation enqueued on each stream
  LevelView view() const;
};

// Fixed operator tables of one expansion order p (device memory).
struct Tables {
  int p = -1;
  double* J = nullptr;     // per degree n a (2n+1)^2 row-major block at joff[n]
  int* joff = nullptr;     // p + 2 offsets
  double* B = nullptr;     // M2M / L2L along z: B[(m*(p+1) + n)*(p+1) + j]
  double* rc = nullptr;    // recurrence constants, see expansions.hip
  // storage of one expansion: `stride` doubles per box; coefficient k
  // (k = n^2, n^2+2m-1, n^2+2m for c_{n,0}, c_{n,m}, s_{n,m}) lives at pos[k];
  // ipos[q] is the coefficient at storage position q, or -1 for a zero slot
  int stride = 0;
  int* pos = nullptr;
  int* ipos = nullptr;
  // MFMA translation tables (p <= 15), as operand fragments [step][lane]:
  // the y-quarter-turn tile matrices [ntiles * 4][64], then the z-translation
  // matrices per order [sum_m hsteps][64]
  double* mtab = nullptr;
  float* mtab32 = nullptr;  // the same in binary32, rows ordered for the binary32 MFMA
  int8_t* sdeg = nullptr;  // degree of each storage position, -1 for a zero slot
  // J, J^T and the z-translation core as operands of the per-lane M2L
  // kernel's 4x4x1 matrix instructions (lane_ops.h), binary32
  float* lane = nullptr;
  // J, J^T (where it fits in LDS) and the z-translation core for the
  // binary64 per-quad M2L kernel (lane_ops.h), and the same with the M2M and
  // L2L cores for the per-quad translation kernel (orders up to
  // kQuadXlateMaxP)
  double* quad = nullptr;
  double* quad_m2m = nullptr;
  double* quad_l2l = nullptr;
  bool tiled = false;
};
const Tables& tables_for(int p, hipStream_t s);
// the tables of order p exist on the current device (no allocation, no wait)
bool tables_ready(int p);

// Phase timer (HIP events), per thread.
struct PhaseTimer {
  void begin(int phase, hipStream_t s);
  void end(int phase, hipStream_t s);
  void reset();
  bool set_enabled(bool on);  // returns the previous setting
};
PhaseTimer& timer();

// ---- launch wrappers ----
// t.n, t.L, t.eta and, when t.m > 0, the targets (tx, ty, tz, caller's
// order) are inputs; the targets only widen the root cell
void tree_build(Tree& t, const double* x, const double* y, const double* z, const double* tx, const double* ty,
                const double* tz, hipStream_t s);
// locates the targets in the leaves and groups them by leaf (after lists)
void targets_build(Tree& t, hipStream_t s);
void lists_build(Tree& t, hipStream_t s);
void p2p_plan(Tree& t, hipStream_t s);
// partial-sum layout of the split leaves for the separate targets
void p2p_plan_targets(Tree& t, hipStream_t s);
void evaluate_targets(const Tree& t, const double* q, int p, int parts, int prec, double* pot, double* ex, double* ey,
                      double* ez, hipStream_t s);
void evaluate(const Tree& t, const double* q, int p, int parts, int prec, double* pot, double* ex, double* ey, double* ez,
              hipStream_t s);

// evaluate() with its scratch in the device's fixed scratch array (no
// allocation, no event, no host wait); FMM_EINVAL beyond the array's size,
// FMM_EUNSUPPORTED when the order's tables are not made yet
void evaluate_noalloc(const Tree& t, const double* q, int p, int parts, int prec, double* pot, double* ex,
                      double* ey, double* ez, hipStream_t s);
size_t noalloc_scratch_bytes();

// peak scratch bytes of one evaluation (evaluate, plus evaluate_targets when
// the tree has targets) at order p and precision prec
size_t eval_scratch_bytes(const Tree& t, int p, int prec);

// exclusive scan of int32 counts into int64 offsets (out[n] = total + base)
void scan_counts(const int32_t* in, int64_t* out, int64_t n, int64_t base, hipStream_t s);
void scan_counts(const int64_t* in, int64_t* out, int64_t n, int64_t base, hipStream_t s);

}  // namespace fmm
