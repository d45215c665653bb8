// Batched dot products that allocate nothing: fdot_modp_many_noalloc.
//
// The same computation and kernels as fdot_modp_many_algo (the dot product
// of each pair over GF(p), Sec. 1 and Sec. 3), for callers that cannot
// allocate device memory at the call (code under graph capture, tight serving
// loops, harnesses that forbid allocation).  The batched kernels' scratch --
// one combination word per pair, the plan of the batch (pair positions and
// unit counts, first pair of each range, the range totals) -- lives in one
// file-scope device array of fixed size instead of a per-stream workspace.
// Each GPU holds its own copy of the array until the process ends; its
// device address is looked up once per device and used for every launch.
#include <mutex>

#include "fdot_internal.h"

namespace {

constexpr size_t kPairs = FDOT_NOALLOC_MAX_PAIRS;
// Layout (the Workspace view below): combination words, pair positions, unit
// counts, range starts, range totals.
constexpr size_t kAccBytes = kPairs * 8;
constexpr size_t kFirstBytes = kPairs * 8;
constexpr size_t kUnitsBytes = kPairs * 4;
constexpr size_t kStartBytes = (size_t)kMaxRanges * 4;
constexpr size_t kTqBytes = 64;
constexpr size_t kScratchBytes =
    (kAccBytes + kFirstBytes + kUnitsBytes + kStartBytes + kTqBytes + 255) & ~(size_t)255;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_ptr[kMaxDevices] = {nullptr};

// Device address of this device's copy of `scratch` (looked up once per
// device, with that device current).
fdot_status_t scratch_ptr(unsigned char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FDOT_E_DEVICE;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FDOT_E_DEVICE;
    g_ptr[dev] = (unsigned char*)p;
  }
  *out = g_ptr[dev];
  return FDOT_OK;
}

}  // namespace

extern "C" fdot_status_t fdot_modp_many_noalloc(fdot_field_t f, fdot_algo_t algo, size_t count,
                                                const fdot_desc_t* desc, void* results,
                                                void* stream) {
  if (!f) return FDOT_E_INVALID_ARG;
  if (f->host_only) return FDOT_E_UNSUPPORTED;
  if ((int)algo < FDOT_ALGO_AUTO || (int)algo > FDOT_ALGO_HYBRID) return FDOT_E_INVALID_ARG;
  if (count > kPairs) return FDOT_E_INVALID_ARG;
  if (f->degree > 1) {
    // GF(p^d): the batched kernel keeps every sum in registers and LDS and
    // takes no scratch; the schedule rules are those of fdot_modp_many_algo.
    const bool char2 = f->info.p == 2;
    bool xor_values = false;
    if (algo == FDOT_ALGO_AUTO || (algo == FDOT_ALGO_ZECH_EXP && char2))
      xor_values = char2;
    else if (algo != FDOT_ALGO_ZECH_TPLUS1)
      return FDOT_E_UNSUPPORTED;
    if (count == 0) return FDOT_OK;
    if (!desc || !results || ((uintptr_t)desc % 8) || ((uintptr_t)results % 2))
      return FDOT_E_INVALID_ARG;
    return fd_launch_ext_many(f, xor_values, count, desc, (uint16_t*)results,
                              (hipStream_t)stream);
  }
  if (count == 0) return FDOT_OK;
  if (!desc || !results || ((uintptr_t)desc % 8) || ((uintptr_t)results % f->info.elem_bytes))
    return FDOT_E_INVALID_ARG;
  unsigned char* base = nullptr;
  fdot_status_t st = scratch_ptr(&base);
  if (st != FDOT_OK) return st;
  Workspace w;
  w.device = -1;
  w.cap = kPairs;
  w.base = base;
  w.acc = (unsigned long long*)base;
  w.first = (uint64_t*)(base + kAccBytes);
  w.units = (uint32_t*)(base + kAccBytes + kFirstBytes);
  w.start = (uint32_t*)(base + kAccBytes + kFirstBytes + kUnitsBytes);
  w.tq = (uint64_t*)(base + kAccBytes + kFirstBytes + kUnitsBytes + kStartBytes);
  if (f->opt.validate) {
    // the check word of the fixed array: no workspace is taken
    st = fd_validate_call(f, (hipStream_t)stream, nullptr, 0, desc, count,
                          (unsigned long long*)(w.tq + kTqCheckWord));
    if (st != FDOT_OK) return st;
  }
  // The combination words must start at zero.  The kernels return each word
  // to zero when its pair completes, but the array is shared by every call on
  // this GPU: clear this batch's words with a kernel (not a memset node, so
  // the call may be captured into a graph).
  const hipStream_t s = (hipStream_t)stream;
  st = fd_launch_zero(w.acc, count * 8, s);
  if (st != FDOT_OK) return st;
  return fd_launch_many(f, algo, count, desc, results, &w, s);
}
