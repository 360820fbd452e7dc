// The evaluation entry point that allocates nothing (fmm_evaluate_tree_noalloc
// in include/fmm.h), for callers that cannot allocate device memory: code
// under HIP graph capture, tight serving loops.  Its scratch memory is one
// fixed device array per GPU, carved into the same buffers the ordinary
// evaluation takes from its allocator.
#include <mutex>

#include "fmm_internal.h"

namespace fmm {
namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;

// The scratch array.  In host code its name is only a stand-in for the
// symbol: its device address (a different one on every GPU) comes from
// hipGetSymbolAddress, made once per device and kept in scratch_ptr.
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

char* scratch_on_current_device() {
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(FMM_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPCHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) fail(FMM_EDEVICE, "no device address for the scratch array");
    g_scratch_ptr[dev] = (char*)ptr;
  }
  return g_scratch_ptr[dev];
}

struct ArenaScope {
  explicit ArenaScope(Arena* a) { set_arena(a); }
  ~ArenaScope() { set_arena(nullptr); }
};

struct TimerOff {
  bool was;
  TimerOff() : was(timer().set_enabled(false)) {}
  ~TimerOff() { timer().set_enabled(was); }
};

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

// One evaluation of tree t with every scratch buffer in the device's scratch
// array: the buffers are laid out as evaluate() requests them, 256-byte
// aligned; the limit is checked before anything is enqueued.
void evaluate_noalloc(const Tree& t, const double* q, int p, int parts, int prec, double* pot, double* ex,
                      double* ey, double* ez, hipStream_t s) {
  // evaluate() requests at most 12 buffers; each may lose 255 bytes to alignment
  const size_t need = eval_scratch_bytes(t, p, prec) + 12 * 256;
  if (need > kScratchBytes)
    fail(FMM_EINVAL, "this evaluation needs " + std::to_string(need) + " bytes of scratch; the fixed buffer holds " +
                         std::to_string(kScratchBytes));
  if (t.L >= 1 && (parts & FMM_PART_FAR) && !tables_ready(p))
    fail(FMM_EUNSUPPORTED, "the operator tables of order " + std::to_string(p) +
                               " are not on this device yet: evaluate once at this order with an allocating entry point");
  Arena a;
  a.base = scratch_on_current_device();
  a.size = kScratchBytes;
  ArenaScope as(&a);
  TimerOff off;
  evaluate(t, q, p, parts, prec, pot, ex, ey, ez, s);
}

}  // namespace fmm
