// C ABI of the library (declared in include/fmm.h): argument validation,
// error reporting, stream-ordered allocation, phase timing and the
// introspection exports.  No exception crosses this layer.
#include <math.h>
#include <string.h>

#include <cstdint>
#include <cstdio>
#include <memory>
#include <mutex>

#include "fmm_internal.h"

struct fmm_tree {
  fmm::Tree t;
};

namespace fmm {

// 1 if work enqueued on s is being captured into a graph
bool capturing(hipStream_t s) {
  if (!s) return false;  // the null stream is never captured
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return st != hipStreamCaptureStatusNone;
}

namespace {
thread_local std::string g_err;

void set_err(const std::string& m) { g_err = m; }

std::once_flag g_pool_once;
void init_pool() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
}

// the process-wide allocator hook (fmm_set_allocator)
std::mutex g_alloc_mu;
Allocator g_alloc;

Allocator current_allocator() {
  std::lock_guard<std::mutex> g(g_alloc_mu);
  return g_alloc;
}

void* raw_alloc(const Allocator& a, size_t bytes, hipStream_t s) {
  void* p = nullptr;
  if (a.alloc) {
    p = a.alloc(bytes, (void*)s, a.user);
  } else {
    std::call_once(g_pool_once, init_pool);
    if (hipMallocAsync(&p, bytes, s) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
  }
  return p;
}

void raw_free(const Allocator& a, void* p, hipStream_t s) {
  if (!p) return;
  if (a.free)
    a.free(p, (void*)s, a.user);
  else
    (void)hipFreeAsync(p, s);
}

// The allocations of one entry-point call: a failed call frees those still
// live; a successful build hands them to its tree.
struct Ledger {
  Allocator a;
  std::vector<std::pair<void*, size_t>> live;
};
thread_local Ledger* g_ledger = nullptr;

class CallScope {
 public:
  CallScope(const Allocator& a, hipStream_t s) : s_(s), prev_(g_ledger) {
    led_.a = a;
    g_ledger = &led_;
  }
  ~CallScope() {
    if (!kept_)
      for (auto it = led_.live.rbegin(); it != led_.live.rend(); ++it) raw_free(led_.a, it->first, s_);
    g_ledger = prev_;
  }
  // the live allocations now belong to the caller (a tree); returns their bytes
  size_t keep() {
    kept_ = true;
    size_t b = 0;
    for (auto& e : led_.live) b += e.second;
    return b;
  }

 private:
  Ledger led_;
  hipStream_t s_;
  Ledger* prev_;
  bool kept_ = false;
};

template <class F>
fmm_status guarded(F&& f) {
  try {
    f();
    g_err.clear();
    return FMM_OK;
  } catch (const Error& e) {
    set_err(e.msg);
    return (fmm_status)e.code;
  } catch (const std::bad_alloc&) {
    set_err("host allocation failed");
    return FMM_ENOMEM;
  } catch (...) {
    set_err("unexpected internal error");
    return FMM_EDEVICE;
  }
}

// Frees the tree's memory through its allocator on the stream of its last
// use, after that stream has waited for every other stream that used it.
void release(Tree& t) {
  hipStream_t s = t.stream;
  for (auto& u : t.uses) {
    if (u.first != s) (void)hipStreamWaitEvent(s, u.second, 0);
    (void)hipEventDestroy(u.second);
  }
  t.uses.clear();
  if (t.built) {
    if (t.build_stream != s) (void)hipStreamWaitEvent(s, t.built, 0);
    (void)hipEventDestroy(t.built);
    t.built = nullptr;
  }
  auto f = [&](void* p) { raw_free(t.alloc, p, s); };
  f(t.px);
  f(t.py);
  f(t.pz);
  f(t.perm);
  f(t.m2l_order);
  f(t.p2p_seg_leaf);
  f(t.p2p_seg_e0);
  f(t.p2p_leaf_seg);
  f(t.p2p_leaf_part);
  f(t.tx);
  f(t.ty);
  f(t.tz);
  f(t.tperm);
  f(t.tleaf);
  f(t.tstart);
  f(t.p2p_leaf_tpart);
  for (Level& V : t.lev) {
    f(V.geom);
    f(V.start);
    f(V.s_off);
    f(V.s_idx);
    f(V.w_off);
    f(V.w_idx);
  }
  t.lev.clear();
  t.px = t.py = t.pz = nullptr;
  t.perm = nullptr;
  t.m2l_order = nullptr;
  t.p2p_seg_leaf = nullptr;
  t.p2p_seg_e0 = nullptr;
  t.p2p_leaf_seg = nullptr;
  t.p2p_leaf_part = nullptr;
  t.tx = t.ty = t.tz = nullptr;
  t.tperm = t.tleaf = t.tstart = nullptr;
  t.p2p_leaf_tpart = nullptr;
}

// An evaluation on stream s: s first waits for the build when it is another
// stream; afterwards the evaluation is recorded so that fmm_free can wait.
// Under graph capture neither happens (no event may cross the capture): the
// caller orders the build before the capture and keeps the tree alive while
// the graph may run.
void begin_use(Tree& t, hipStream_t s) {
  if (capturing(s)) return;
  if (t.built && s != t.build_stream) HIPCHECK(hipStreamWaitEvent(s, t.built, 0));
}
void end_use(Tree& t, hipStream_t s) {
  if (capturing(s)) return;
  hipEvent_t ev = nullptr;
  for (auto& u : t.uses)
    if (u.first == s) ev = u.second;
  if (!ev) {
    HIPCHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    t.uses.emplace_back(s, ev);
  }
  HIPCHECK(hipEventRecord(ev, s));
  t.stream = s;
}

// ---- phase timer ----
struct TimerState {
  bool on = false;
  hipEvent_t ev[FMM_NUM_PHASES][2] = {};
  bool used[FMM_NUM_PHASES] = {};
  bool created = false;
};
thread_local TimerState g_tm;

}  // namespace

[[noreturn]] void fail(int code, const std::string& msg) { throw Error{code, msg}; }

void check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  const int code = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? FMM_ENOMEM : FMM_EDEVICE;
  fail(code, std::string(what) + ": " + hipGetErrorString(e));
}

thread_local Arena* g_arena = nullptr;
void set_arena(Arena* a) { g_arena = a; }

void* dalloc(size_t bytes, hipStream_t s) {
  if (bytes == 0) bytes = 8;
  if (g_arena) {
    const size_t off = (g_arena->used + 255) & ~(size_t)255;
    if (off > g_arena->size || bytes > g_arena->size - off)
      fail(FMM_EINVAL, "evaluation scratch exceeds the fixed buffer of " + std::to_string(g_arena->size) + " bytes");
    g_arena->used = off + bytes;
    return g_arena->base + off;
  }
  const Allocator a = g_ledger ? g_ledger->a : Allocator{};
  void* p = raw_alloc(a, bytes, s);
  if (!p) fail(FMM_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  if (g_ledger) {
    try {
      g_ledger->live.emplace_back(p, bytes);
    } catch (...) {
      raw_free(a, p, s);
      throw;
    }
  }
  return p;
}

void dfree(void* p, hipStream_t s) {
  if (!p || g_arena) return;
  const Allocator a = g_ledger ? g_ledger->a : Allocator{};
  if (g_ledger) {
    auto& v = g_ledger->live;
    for (size_t k = v.size(); k-- > 0;)
      if (v[k].first == p) {
        v.erase(v.begin() + (long)k);
        break;
      }
  }
  raw_free(a, p, s);
}

int64_t* host_stage() {
  thread_local int64_t* h = nullptr;
  if (!h) {
    void* p = nullptr;
    HIPCHECK(hipHostMalloc(&p, kStageWords * sizeof(int64_t), hipHostMallocDefault));
    h = (int64_t*)p;
  }
  return h;
}

LevelView Tree::view() const {
  LevelView v{};
  v.L = L;
  for (int l = 0; l <= L; ++l) {
    const Level& V = lev[l];
    v.gofs[l] = V.gofs;
    v.geom[l] = V.geom;
    v.start[l] = V.start;
    v.s_off[l] = V.s_off;
    v.s_idx[l] = V.s_idx;
    v.w_off[l] = V.w_off;
    v.w_idx[l] = V.w_idx;
  }
  v.gofs[L + 1] = nbox_total;
  return v;
}

PhaseTimer& timer() {
  static thread_local PhaseTimer t;
  return t;
}

bool PhaseTimer::set_enabled(bool on) {
  const bool was = g_tm.on;
  g_tm.on = on;
  return was;
}

void PhaseTimer::reset() {
  for (bool& u : g_tm.used) u = false;
}

void PhaseTimer::begin(int ph, hipStream_t s) {
  if (!g_tm.on) return;
  if (!g_tm.created) {
    for (auto& e : g_tm.ev) {
      HIPCHECK(hipEventCreate(&e[0]));
      HIPCHECK(hipEventCreate(&e[1]));
    }
    g_tm.created = true;
  }
  HIPCHECK(hipEventRecord(g_tm.ev[ph][0], s));
  g_tm.used[ph] = true;
}

void PhaseTimer::end(int ph, hipStream_t s) {
  if (!g_tm.on) return;
  HIPCHECK(hipEventRecord(g_tm.ev[ph][1], s));
}

}  // namespace fmm

using fmm::Error;
using fmm::fail;

namespace {

void validate_points(const void* x, const void* y, const void* z, int64_t n) {
  if (!x || !y || !z) fail(FMM_EINVAL, "coordinate pointer is NULL");
  if (n < 1 || n > FMM_MAX_POINTS) fail(FMM_EINVAL, "n must be in [1, 2^31-1]");
}

void validate_tree_args(int levels, double theta) {
  if (levels < 0 || levels > FMM_MAX_LEVELS) fail(FMM_EINVAL, "levels must be in [0, 8]");
  if (!(theta >= 0.0 && theta < 1.0)) fail(FMM_EINVAL, "theta must be in [0, 1)");
}

void validate_eval_args(const void* q, int p, const void* a, const void* b, const void* c, const void* d) {
  if (!q) fail(FMM_EINVAL, "charge pointer is NULL");
  if (!a || !b || !c || !d) fail(FMM_EINVAL, "output pointer is NULL");
  if (p < 0 || p > FMM_MAX_ORDER) fail(FMM_EINVAL, "p must be in [0, 20]");
}

void ensure_device() {
  int cnt = 0;
  const hipError_t e = hipGetDeviceCount(&cnt);
  if (e != hipSuccess || cnt < 1) {
    (void)hipGetLastError();
    fail(FMM_EDEVICE, "no HIP device available");
  }
}

fmm_tree* build_impl(const double* x, const double* y, const double* z, int64_t n, const double* tx,
                     const double* ty, const double* tz, int64_t m, int levels, double theta, double eta,
                     hipStream_t s) {
  validate_points(x, y, z, n);
  validate_tree_args(levels, theta);
  if (!(eta >= 0.0 && eta <= 1.0)) fail(FMM_EINVAL, "eta must be in [0, 1]");
  if (m < 0 || m > FMM_MAX_POINTS) fail(FMM_EINVAL, "m must be in [0, 2^31-1]");
  if (m > 0 && (!tx || !ty || !tz)) fail(FMM_EINVAL, "target pointer is NULL");
  ensure_device();
  std::unique_ptr<fmm_tree> h(new fmm_tree());
  fmm::Tree& t = h->t;
  t.n = n;
  t.L = levels;
  t.theta = theta;
  t.eta = eta;
  t.m = m;
  t.stream = s;
  t.build_stream = s;
  t.alloc = fmm::current_allocator();
  fmm::CallScope scope(t.alloc, s);  // frees everything allocated here if the build fails
  fmm::timer().reset();
  fmm::timer().begin(FMM_PH_TREE, s);
  fmm::tree_build(t, x, y, z, tx, ty, tz, s);
  fmm::timer().end(FMM_PH_TREE, s);
  fmm::timer().begin(FMM_PH_LISTS, s);
  fmm::lists_build(t, s);
  fmm::p2p_plan(t, s);
  if (m > 0) {
    fmm::targets_build(t, s);
    fmm::p2p_plan_targets(t, s);
  }
  fmm::timer().end(FMM_PH_LISTS, s);
  HIPCHECK(hipEventCreateWithFlags(&t.built, hipEventDisableTiming));
  HIPCHECK(hipEventRecord(t.built, s));
  t.bytes = scope.keep();
  return h.release();
}

// Runs one evaluation of tree t on stream s with its scratch memory in a
// call scope (freed if the evaluation fails; the tree stays valid).
template <class F>
void run_evaluation(fmm::Tree& t, hipStream_t s, F&& f) {
  fmm::begin_use(t, s);
  // recorded also when the evaluation fails part-way: work may be enqueued
  struct Use {
    fmm::Tree& t;
    hipStream_t s;
    ~Use() {
      try {
        fmm::end_use(t, s);
      } catch (...) {
      }
    }
  } use{t, s};
  struct Timer {
    bool was;
    bool cap;
    explicit Timer(hipStream_t s) : was(false), cap(fmm::capturing(s)) {
      if (cap) was = fmm::timer().set_enabled(false);  // no timing events inside a graph
    }
    ~Timer() {
      if (cap) fmm::timer().set_enabled(was);
    }
  } tm{s};
  fmm::CallScope scope(fmm::current_allocator(), s);
  f();
}

const fmm::Tree& get(const fmm_tree* h) {
  if (!h) fail(FMM_EINVAL, "tree handle is NULL");
  return h->t;
}

}  // namespace

extern "C" {

fmm_status fmm_build(const double* x, const double* y, const double* z, int64_t n, int levels, double theta, void* stream,
              fmm_tree** out) {
  return fmm::guarded([&] {
    if (!out) fail(FMM_EINVAL, "out is NULL");
    *out = nullptr;
    *out = build_impl(x, y, z, n, nullptr, nullptr, nullptr, 0, levels, theta, 1.0, (hipStream_t)stream);
  });
}

fmm_status fmm_build_ex(const double* x, const double* y, const double* z, int64_t n, const double* tx, const double* ty,
                 const double* tz, int64_t m, int levels, double theta, double eta, void* stream, fmm_tree** out) {
  return fmm::guarded([&] {
    if (!out) fail(FMM_EINVAL, "out is NULL");
    *out = nullptr;
    *out = build_impl(x, y, z, n, tx, ty, tz, m, levels, theta, eta, (hipStream_t)stream);
  });
}

fmm_status fmm_evaluate_targets(fmm_tree* tree, const double* q, int p, int parts, int precision, double* pot, double* ex,
                         double* ey, double* ez, void* stream) {
  return fmm::guarded([&] {
    fmm::Tree& t = const_cast<fmm::Tree&>(get(tree));
    if (!q) fail(FMM_EINVAL, "charge pointer is NULL");
    if (p < 0 || p > FMM_MAX_ORDER) fail(FMM_EINVAL, "p must be in [0, 20]");
    if (t.m > 0 && (!pot || !ex || !ey || !ez)) fail(FMM_EINVAL, "output pointer is NULL");
    if (parts < 1 || parts > 3) fail(FMM_EINVAL, "parts must be 1, 2 or 3");
    if (precision != FMM_PREC_F64 && precision != FMM_PREC_MIXED && precision != FMM_PREC_F32)
      fail(FMM_EINVAL, "unknown precision");
    hipStream_t s = (hipStream_t)stream;
    run_evaluation(t, s, [&] { fmm::evaluate_targets(t, q, p, parts, precision, pot, ex, ey, ez, s); });
  });
}

fmm_status fmm_tree_targets(const fmm_tree* tree, int64_t* m, int32_t* leaf) {
  return fmm::guarded([&] {
    const fmm::Tree& t = get(tree);
    if (m) *m = t.m;
    if (leaf && t.m > 0) {
      HIPCHECK(hipStreamSynchronize(t.stream));
      HIPCHECK(hipMemcpy(leaf, t.tleaf, t.m * sizeof(int32_t), hipMemcpyDeviceToHost));
    }
  });
}

fmm_status fmm_evaluate_tree_ex(fmm_tree* tree, const double* q, int p, int parts, int precision, double* pot, double* ex,
                         double* ey, double* ez, void* stream) {
  return fmm::guarded([&] {
    fmm::Tree& t = const_cast<fmm::Tree&>(get(tree));
    validate_eval_args(q, p, pot, ex, ey, ez);
    if (parts < 1 || parts > 3) fail(FMM_EINVAL, "parts must be 1, 2 or 3");
    if (precision != FMM_PREC_F64 && precision != FMM_PREC_MIXED && precision != FMM_PREC_F32)
      fail(FMM_EINVAL, "unknown precision");
    hipStream_t s = (hipStream_t)stream;
    run_evaluation(t, s, [&] { fmm::evaluate(t, q, p, parts, precision, pot, ex, ey, ez, s); });
  });
}

fmm_status fmm_evaluate_tree_noalloc(fmm_tree* tree, const double* q, int p, int parts, int precision, double* pot,
                                     double* ex, double* ey, double* ez, void* stream) {
  return fmm::guarded([&] {
    fmm::Tree& t = const_cast<fmm::Tree&>(get(tree));
    validate_eval_args(q, p, pot, ex, ey, ez);
    if (parts < 1 || parts > 3) fail(FMM_EINVAL, "parts must be 1, 2 or 3");
    if (precision != FMM_PREC_F64 && precision != FMM_PREC_MIXED && precision != FMM_PREC_F32)
      fail(FMM_EINVAL, "unknown precision");
    fmm::evaluate_noalloc(t, q, p, parts, precision, pot, ex, ey, ez, (hipStream_t)stream);
  });
}

fmm_status fmm_evaluate_tree_parts(fmm_tree* tree, const double* q, int p, int parts, double* pot, double* ex, double* ey,
                            double* ez, void* stream) {
  return fmm_evaluate_tree_ex(tree, q, p, parts, FMM_PREC_F64, pot, ex, ey, ez, stream);
}

fmm_status fmm_evaluate_tree(fmm_tree* tree, const double* q, int p, double* pot, double* ex, double* ey, double* ez,
                      void* stream) {
  return fmm_evaluate_tree_parts(tree, q, p, FMM_PART_ALL, pot, ex, ey, ez, stream);
}

fmm_status fmm_evaluate(const double* x, const double* y, const double* z, const double* q, int64_t n, double theta, int p,
                 int levels, double* pot, double* ex, double* ey, double* ez, void* stream) {
  return fmm::guarded([&] {
    validate_points(x, y, z, n);
    validate_tree_args(levels, theta);
    validate_eval_args(q, p, pot, ex, ey, ez);
    hipStream_t s = (hipStream_t)stream;
    std::unique_ptr<fmm_tree> h(build_impl(x, y, z, n, nullptr, nullptr, nullptr, 0, levels, theta, 1.0, s));
    struct Rel {
      fmm::Tree& t;
      ~Rel() { fmm::release(t); }
    } rel{h->t};
    run_evaluation(h->t, s, [&] { fmm::evaluate(h->t, q, p, FMM_PART_ALL, FMM_PREC_F64, pot, ex, ey, ez, s); });
  });
}

fmm_status fmm_free(fmm_tree* tree) {
  return fmm::guarded([&] {
    if (!tree) return;
    fmm::release(tree->t);
    delete tree;
  });
}

const char* fmm_last_error(void) { return fmm::g_err.c_str(); }

fmm_status fmm_tree_info(const fmm_tree* tree, int64_t* n, int* levels, double* theta) {
  return fmm::guarded([&] {
    const fmm::Tree& t = get(tree);
    if (n) *n = t.n;
    if (levels) *levels = t.L;
    if (theta) *theta = t.theta;
  });
}

fmm_status fmm_tree_perm(const fmm_tree* tree, int32_t* perm) {
  return fmm::guarded([&] {
    const fmm::Tree& t = get(tree);
    if (!perm) fail(FMM_EINVAL, "perm is NULL");
    HIPCHECK(hipStreamSynchronize(t.stream));
    HIPCHECK(hipMemcpy(perm, t.perm, t.n * sizeof(int32_t), hipMemcpyDeviceToHost));
  });
}

fmm_status fmm_tree_boxes(const fmm_tree* tree, int level, double* geom, int64_t* start) {
  return fmm::guarded([&] {
    const fmm::Tree& t = get(tree);
    if (level < 0 || level > t.L) fail(FMM_EINVAL, "level out of range");
    const fmm::Level& V = t.lev[level];
    HIPCHECK(hipStreamSynchronize(t.stream));
    if (geom) HIPCHECK(hipMemcpy(geom, V.geom, V.nbox * 10 * sizeof(double), hipMemcpyDeviceToHost));
    if (start) {
      std::vector<int32_t> tmp(V.nbox + 1);
      HIPCHECK(hipMemcpy(tmp.data(), V.start, (V.nbox + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
      for (int64_t i = 0; i <= V.nbox; ++i) start[i] = tmp[i];
    }
  });
}

fmm_status fmm_tree_lists(const fmm_tree* tree, int level, int kind, int64_t* nnz, int64_t* offsets, int32_t* idx) {
  return fmm::guarded([&] {
    const fmm::Tree& t = get(tree);
    if (level < 0 || level > t.L) fail(FMM_EINVAL, "level out of range");
    if (kind != 0 && kind != 1) fail(FMM_EINVAL, "kind must be 0 (strong) or 1 (weak)");
    const fmm::Level& V = t.lev[level];
    const int64_t cnt = kind == 0 ? V.s_nnz : V.w_nnz;
    if (nnz) *nnz = cnt;
    HIPCHECK(hipStreamSynchronize(t.stream));
    if (offsets)
      HIPCHECK(hipMemcpy(offsets, kind == 0 ? V.s_off : V.w_off, (V.nbox + 1) * sizeof(int64_t),
                         hipMemcpyDeviceToHost));
    if (idx && cnt > 0)
      HIPCHECK(hipMemcpy(idx, kind == 0 ? V.s_idx : V.w_idx, cnt * sizeof(int32_t), hipMemcpyDeviceToHost));
  });
}

fmm_status fmm_tree_stats(const fmm_tree* tree, int64_t* m2l_pairs, int64_t* p2p_pairs) {
  return fmm::guarded([&] {
    const fmm::Tree& t = get(tree);
    if (m2l_pairs) *m2l_pairs = t.m2l_pairs;
    if (p2p_pairs) *p2p_pairs = t.p2p_pairs;
  });
}

fmm_status fmm_set_allocator(fmm_alloc_fn alloc, fmm_free_fn free_fn, void* user) {
  return fmm::guarded([&] {
    if ((alloc == nullptr) != (free_fn == nullptr)) fail(FMM_EINVAL, "alloc and free must both be set or both NULL");
    std::lock_guard<std::mutex> g(fmm::g_alloc_mu);
    fmm::g_alloc = fmm::Allocator{alloc, free_fn, alloc ? user : nullptr};
  });
}

fmm_status fmm_tree_bytes(const fmm_tree* tree, int p, int precision, size_t* tree_bytes, size_t* eval_bytes) {
  return fmm::guarded([&] {
    const fmm::Tree& t = get(tree);
    if (p < 0 || p > FMM_MAX_ORDER) fail(FMM_EINVAL, "p must be in [0, 20]");
    if (precision != FMM_PREC_F64 && precision != FMM_PREC_MIXED && precision != FMM_PREC_F32)
      fail(FMM_EINVAL, "unknown precision");
    if (tree_bytes) *tree_bytes = t.bytes;
    if (eval_bytes) *eval_bytes = fmm::eval_scratch_bytes(t, p, precision);
  });
}

fmm_status fmm_set_profiling(int on) {
  fmm::g_tm.on = on != 0;
  return FMM_OK;
}

fmm_status fmm_last_timings(double* ms) {
  return fmm::guarded([&] {
    if (!ms) fail(FMM_EINVAL, "ms is NULL");
    for (int k = 0; k < FMM_NUM_PHASES; ++k) {
      ms[k] = 0.0;
      if (!fmm::g_tm.on || !fmm::g_tm.created || !fmm::g_tm.used[k]) continue;
      HIPCHECK(hipEventSynchronize(fmm::g_tm.ev[k][1]));
      float v = 0.f;
      HIPCHECK(hipEventElapsedTime(&v, fmm::g_tm.ev[k][0], fmm::g_tm.ev[k][1]));
      ms[k] = v;
    }
  });
}

size_t fmm_bytes_estimate(int64_t n, int levels, double theta, int p) {
  if (n < 1 || levels < 0 || levels > FMM_MAX_LEVELS || p < 0 || p > FMM_MAX_ORDER) return 0;
  if (!(theta >= 0.0 && theta < 1.0)) return 0;
  int64_t nbox = 0;
  for (int l = 0; l <= levels; ++l) nbox += (int64_t)1 << (3 * l);
  const double th = theta > 0.05 ? theta : 0.05;
  // weak and strong links per box on a uniform lattice grow like theta^-3
  const double links = 650.0 * (0.125 / (th * th * th)) + 100.0;
  // points: coordinates (two copies during the build), permutation, charges,
  // far field, and an allowance for the near-field partial sums
  const size_t pts = (size_t)n * (2 * 28 + 8 + 4 * 8 + 8 + 32);
  const size_t geo = (size_t)nbox * (10 * 8 + 4 + 16) + ((size_t)2 << (3 * levels)) * (6 * 8 + 8);
  const size_t lists = (size_t)((double)nbox * links * 4.0);
  const size_t expn = (size_t)nbox * (size_t)(p + 1) * (p + 1) * 8 * 2;
  return pts + geo + lists + expn + ((size_t)64 << 20);
}

}  // extern "C"
