// C-ABI layer of libfdot: argument checks, per-stream workspace, the tuned
// parameter table and the public compute calls.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "fdot_internal.h"

namespace {

std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;
std::vector<void*> g_ws_retired;  // workspaces a captured graph may still use

std::mutex g_tune_mu;
std::map<std::string, int64_t> g_tune;
bool g_tune_loaded = false;

// Optional "key=value" lines from the file named by FDOT_TUNE_FILE (the table
// an install-time tuning run writes), read once.
void load_tune_file_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = getenv("FDOT_TUNE_FILE");
  if (!path || !*path) return;
  FILE* fp = fopen(path, "r");
  if (!fp) return;
  char line[256];
  while (fgets(line, sizeof line, fp)) {
    char* eq = strchr(line, '=');
    if (!eq || line[0] == '#') continue;
    *eq = 0;
    char* k = line;
    while (*k == ' ' || *k == '\t') ++k;
    char* end = eq - 1;
    while (end >= k && (*end == ' ' || *end == '\t')) *end-- = 0;
    g_tune[k] = strtoll(eq + 1, nullptr, 10);
  }
  fclose(fp);
}

bool aligned_to(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Kernel trace: a pool of event pairs, reused from the start at every enable.
constexpr size_t kTraceMax = 1u << 16;
std::mutex g_tr_mu;
bool g_tr_on = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_tr_pool;
size_t g_tr_used = 0;
bool g_tr_lost = false;

}  // namespace

int fd_trace_begin(hipStream_t s) {
  std::lock_guard<std::mutex> g(g_tr_mu);
  if (!g_tr_on) return -1;
  if (g_tr_used == g_tr_pool.size()) {
    hipEvent_t a = nullptr, b = nullptr;
    if (g_tr_pool.size() >= kTraceMax || hipEventCreate(&a) != hipSuccess) {
      g_tr_lost = true;
      return -1;
    }
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      g_tr_lost = true;
      return -1;
    }
    g_tr_pool.emplace_back(a, b);
  }
  const int slot = (int)g_tr_used++;
  if (hipEventRecord(g_tr_pool[slot].first, s) != hipSuccess) g_tr_lost = true;
  return slot;
}

void fd_trace_end(hipStream_t s, int slot) {
  if (slot < 0) return;
  std::lock_guard<std::mutex> g(g_tr_mu);
  if ((size_t)slot < g_tr_pool.size() && hipEventRecord(g_tr_pool[slot].second, s) != hipSuccess)
    g_tr_lost = true;
}

int64_t fd_tune(const char* key, int64_t fallback) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  load_tune_file_locked();
  auto it = g_tune.find(key);
  return it == g_tune.end() ? fallback : it->second;
}

int fd_cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

hipError_t fd_alloc_async(void** p, size_t bytes, hipStream_t s) {
  // Freed blocks stay in the device's default pool for the next growth
  // instead of going back to the driver at every synchronisation.
  static bool pool_set[64] = {false};
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64 && !pool_set[dev]) {
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
      uint64_t keep = ~0ull;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    pool_set[dev] = true;
  }
  return hipMallocAsync(p, bytes, s);
}

void fd_workspace_release(hipStream_t s) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  std::lock_guard<std::mutex> g(g_ws_mu);
  auto it = g_ws.find(std::make_pair(dev, s));
  if (it == g_ws.end()) return;
  Workspace* w = it->second;
  if (w) {
    if (w->captured)
      g_ws_retired.push_back(w->base);
    else
      (void)hipFreeAsync(w->base, s);
    delete w;
  }
  g_ws.erase(it);
}

fdot_status_t fd_workspace_get(hipStream_t s, size_t count, Workspace** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return FDOT_E_DEVICE;
  std::lock_guard<std::mutex> g(g_ws_mu);
  Workspace*& w = g_ws[std::make_pair(dev, s)];
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const bool capturing =
      hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
  if (w && w->cap >= count) {
    // A captured graph keeps this buffer's address: later growth must not
    // free it while such a graph may still be replayed.
    if (capturing) w->captured = true;
    *out = w;
    return FDOT_OK;
  }
  // Growing allocates, which a stream under graph capture cannot do.
  if (capturing) return FDOT_E_BUSY;
  size_t cap = count < 4096 ? 4096 : count;
  if (w) cap = std::max(cap, w->cap + w->cap / 2);  // geometric growth
  const size_t bytes_acc = cap * 8, bytes_first = cap * 8, bytes_units = (cap * 4 + 7) / 8 * 8,
               bytes_start = (size_t)kMaxRanges * 4;
  const size_t bytes = bytes_acc + bytes_first + bytes_units + bytes_start + 64;
  void* base = nullptr;
  if (fd_alloc_async(&base, bytes, s) != hipSuccess) return FDOT_E_NOMEM;
  if (fd_launch_zero(base, bytes, s) != FDOT_OK) {
    (void)hipFreeAsync(base, s);
    return FDOT_E_DEVICE;
  }
  if (w) {  // freed in stream order, after the work already queued on s
    if (w->captured)
      g_ws_retired.push_back(w->base);  // kept until the process ends
    else
      (void)hipFreeAsync(w->base, s);
    w->captured = false;
  } else {
    w = new Workspace;
  }
  w->device = dev;
  w->cap = cap;
  w->base = base;
  char* b = (char*)base;
  w->acc = (unsigned long long*)b;
  w->first = (uint64_t*)(b + bytes_acc);
  w->units = (uint32_t*)(b + bytes_acc + bytes_first);
  w->start = (uint32_t*)(b + bytes_acc + bytes_first + bytes_units);
  w->tq = (uint64_t*)(b + bytes_acc + bytes_first + bytes_units + bytes_start);
  *out = w;
  return FDOT_OK;
}

extern "C" {

const char* fdot_status_string(int status) {
  switch (status) {
    case FDOT_OK: return "ok";
    case FDOT_E_INVALID_ARG: return "invalid argument";
    case FDOT_E_NOT_PRIME: return "modulus is not prime";
    case FDOT_E_BOUND: return "prime outside the representation bound";
    case FDOT_E_UNSUPPORTED: return "unsupported for this representation or algorithm";
    case FDOT_E_DEVICE: return "device (HIP) error";
    case FDOT_E_NOMEM: return "out of memory";
    case FDOT_E_BUSY: return "busy";
    case FDOT_E_NOT_FOUND: return "not found";
    case FDOT_E_NONCANON: return "input not canonical in its representation";
  }
  return "unknown status";
}

int fdot_version(void) { return 1; }

fdot_status_t fdot_tune_set(const char* key, int64_t value) {
  if (!key || !*key) return FDOT_E_INVALID_ARG;
  std::lock_guard<std::mutex> g(g_tune_mu);
  load_tune_file_locked();
  if (value == INT64_MIN)
    g_tune.erase(key);
  else
    g_tune[key] = value;
  return FDOT_OK;
}

fdot_status_t fdot_tune_get(const char* key, int64_t* value) {
  if (!key || !value) return FDOT_E_INVALID_ARG;
  std::lock_guard<std::mutex> g(g_tune_mu);
  load_tune_file_locked();
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return FDOT_E_NOT_FOUND;
  *value = it->second;
  return FDOT_OK;
}

fdot_status_t fdot_trace_enable(int on) {
  std::lock_guard<std::mutex> g(g_tr_mu);
  g_tr_on = on != 0;
  if (g_tr_on) {
    g_tr_used = 0;
    g_tr_lost = false;
  }
  return FDOT_OK;
}

fdot_status_t fdot_trace_read(double* ms, size_t cap, size_t* count) {
  if (!count || (cap && !ms)) return FDOT_E_INVALID_ARG;
  std::lock_guard<std::mutex> g(g_tr_mu);
  if (g_tr_lost) return FDOT_E_NOMEM;
  *count = g_tr_used;
  for (size_t i = 0; i < g_tr_used && i < cap; ++i) {
    if (hipEventSynchronize(g_tr_pool[i].second) != hipSuccess) return FDOT_E_DEVICE;
    float t = 0.f;
    if (hipEventElapsedTime(&t, g_tr_pool[i].first, g_tr_pool[i].second) != hipSuccess)
      return FDOT_E_DEVICE;
    ms[i] = t;
  }
  return FDOT_OK;
}

fdot_status_t fdot_workspace_reserve(void* stream, size_t count) {
  Workspace* w = nullptr;
  return fd_workspace_get((hipStream_t)stream, count ? count : 1, &w);
}

fdot_status_t fdot_encode(fdot_field_t f, const uint32_t* canon, void* rep, size_t n, void* stream) {
  if (!f) return FDOT_E_INVALID_ARG;
  if (f->host_only) return FDOT_E_UNSUPPORTED;
  if (n && (!canon || !rep || !aligned_to(rep, f->info.elem_bytes) || !aligned_to(canon, 4)))
    return FDOT_E_INVALID_ARG;
  return fd_launch_encode(f, canon, rep, n, (hipStream_t)stream);
}

fdot_status_t fdot_decode(fdot_field_t f, const void* rep, uint32_t* canon, size_t n, void* stream) {
  if (!f) return FDOT_E_INVALID_ARG;
  if (f->host_only) return FDOT_E_UNSUPPORTED;
  if (n && (!canon || !rep || !aligned_to(rep, f->info.elem_bytes) || !aligned_to(canon, 4)))
    return FDOT_E_INVALID_ARG;
  return fd_launch_decode(f, rep, canon, n, (hipStream_t)stream);
}

// Schedules of a GF(p^d) dot product: the plus-one table (any p), or in
// characteristic 2 the products' values accumulated by exclusive or
// (FDOT_ALGO_ZECH_EXP, the default there).
static fdot_status_t ext_schedule(const fdot_field_s* f, fdot_algo_t algo, bool* xor_values) {
  const bool char2 = f->info.p == 2;
  *xor_values = false;
  if (algo == FDOT_ALGO_AUTO || (algo == FDOT_ALGO_ZECH_EXP && char2)) {
    *xor_values = char2;
    return FDOT_OK;
  }
  return algo == FDOT_ALGO_ZECH_TPLUS1 ? FDOT_OK : FDOT_E_UNSUPPORTED;
}

fdot_status_t fdot_elementwise(fdot_field_t f, fdot_ew_op_t op, size_t n, const void* alpha,
                               const void* x, const void* y, void* r, void* stream) {
  if (!f) return FDOT_E_INVALID_ARG;
  if (f->host_only) return FDOT_E_UNSUPPORTED;
  if ((int)op < FDOT_EW_ADD || (int)op > FDOT_EW_AXPYIN) return FDOT_E_INVALID_ARG;
  if (n == 0) return FDOT_OK;
  const size_t es = f->info.elem_bytes;
  const bool needs_y = op != FDOT_EW_NEG && op != FDOT_EW_AXPYIN;
  const bool needs_a = op == FDOT_EW_AXPY || op == FDOT_EW_AXPYIN;
  if (!x || !r || !aligned_to(x, es) || !aligned_to(r, es)) return FDOT_E_INVALID_ARG;
  if (needs_y && (!y || !aligned_to(y, es))) return FDOT_E_INVALID_ARG;
  if (needs_a && !alpha) return FDOT_E_INVALID_ARG;
  if (f->opt.validate) {
    if (needs_a && !fd_canonical_host(f, alpha)) return FDOT_E_NONCANON;
    FdCheck c[3];
    int k = 0;
    c[k++] = {x, 1, n, n};
    if (needs_y) c[k++] = {y, 1, n, n};
    if (op == FDOT_EW_AXPYIN) c[k++] = {r, 1, n, n};
    const fdot_status_t st = fd_validate_call(f, (hipStream_t)stream, c, k, nullptr, 0, nullptr);
    if (st != FDOT_OK) return st;
  }
  return fd_launch_elementwise(f, op, n, needs_a ? alpha : nullptr, x, needs_y ? y : nullptr, r,
                               (hipStream_t)stream);
}

fdot_status_t fdot_modp_algo(fdot_field_t f, fdot_algo_t algo, const void* x, const void* y,
                             size_t n, void* result, void* stream) {
  if (!f || !result) return FDOT_E_INVALID_ARG;
  if (f->host_only) return FDOT_E_UNSUPPORTED;
  if ((int)algo < FDOT_ALGO_AUTO || (int)algo > FDOT_ALGO_HYBRID) return FDOT_E_INVALID_ARG;
  const size_t es = f->info.elem_bytes;
  if (!aligned_to(result, es)) return FDOT_E_INVALID_ARG;
  if (n && (!x || !y || !aligned_to(x, es) || !aligned_to(y, es))) return FDOT_E_INVALID_ARG;
  if (f->opt.validate && n) {
    const FdCheck c[2] = {{x, 1, n, n}, {y, 1, n, n}};
    const fdot_status_t st = fd_validate_call(f, (hipStream_t)stream, c, 2, nullptr, 0, nullptr);
    if (st != FDOT_OK) return st;
  }
  if (f->degree > 1) {
    bool xv = false;
    const fdot_status_t st = ext_schedule(f, algo, &xv);
    if (st != FDOT_OK) return st;
    return fd_launch_ext_dot(f, xv, (const uint16_t*)x, (const uint16_t*)y, n,
                             (uint16_t*)result, (hipStream_t)stream);
  }
  Workspace* w = nullptr;
  fdot_status_t st = fd_workspace_get((hipStream_t)stream, 1, &w);
  if (st != FDOT_OK) return st;
  return fd_launch_dot(f, algo, x, y, n, result, w, (hipStream_t)stream);
}

fdot_status_t fdot_modp(fdot_field_t f, const void* x, const void* y, size_t n, void* result,
                        void* stream) {
  return fdot_modp_algo(f, FDOT_ALGO_AUTO, x, y, n, result, stream);
}

fdot_status_t fdot_modp_many_algo(fdot_field_t f, fdot_algo_t algo, size_t count,
                                  const fdot_desc_t* desc, void* results, void* stream) {
  if (!f) return FDOT_E_INVALID_ARG;
  if (f->host_only) return FDOT_E_UNSUPPORTED;
  if ((int)algo < FDOT_ALGO_AUTO || (int)algo > FDOT_ALGO_HYBRID) return FDOT_E_INVALID_ARG;
  bool xv = false;
  if (f->degree > 1) {
    const fdot_status_t st = ext_schedule(f, algo, &xv);
    if (st != FDOT_OK) return st;
  }
  if (count == 0) return FDOT_OK;
  if (!desc || !results || !aligned_to(desc, 8) || !aligned_to(results, f->info.elem_bytes))
    return FDOT_E_INVALID_ARG;
  if (count > (1ull << 31)) return FDOT_E_INVALID_ARG;
  if (f->opt.validate) {
    const fdot_status_t st =
        fd_validate_call(f, (hipStream_t)stream, nullptr, 0, desc, count, nullptr);
    if (st != FDOT_OK) return st;
  }
  if (f->degree > 1)
    return fd_launch_ext_many(f, xv, count, desc, (uint16_t*)results, (hipStream_t)stream);
  Workspace* w = nullptr;
  fdot_status_t st = fd_workspace_get((hipStream_t)stream, count, &w);
  if (st != FDOT_OK) return st;
  return fd_launch_many(f, algo, count, desc, results, w, (hipStream_t)stream);
}

fdot_status_t fdot_modp_many_mixed(size_t count, const fdot_mixed_desc_t* desc,
                                   const fdot_field_t* fields, size_t nfields, void* results,
                                   void* stream) {
  if (!fields || nfields == 0 || nfields > 0xFFFFFFFFull) return FDOT_E_INVALID_ARG;
  for (size_t i = 0; i < nfields; ++i) {
    const fdot_field_t f = fields[i];
    if (!f || f->degree > 1 || f->info.rep != fields[0]->info.rep) return FDOT_E_INVALID_ARG;
    if (f->host_only) return FDOT_E_UNSUPPORTED;
  }
  if (count == 0) return FDOT_OK;
  if (!desc || !results || !aligned_to(desc, 8) || !aligned_to(results, fields[0]->info.elem_bytes))
    return FDOT_E_INVALID_ARG;
  if (count > (1ull << 31)) return FDOT_E_INVALID_ARG;
  return fd_launch_many_mixed(count, desc, fields, nfields, results, (hipStream_t)stream);
}

fdot_status_t fdot_modp_many(fdot_field_t f, size_t count, const fdot_desc_t* desc, void* results,
                             void* stream) {
  return fdot_modp_many_algo(f, FDOT_ALGO_AUTO, count, desc, results, stream);
}

fdot_status_t fgemv_modp(fdot_field_t f, size_t m, size_t n, const void* A, size_t lda,
                         const void* x, void* y, void* stream) {
  if (!f) return FDOT_E_INVALID_ARG;
  if (f->host_only) return FDOT_E_UNSUPPORTED;
  if (f->degree > 1) return FDOT_E_UNSUPPORTED;
  if (m == 0) return FDOT_OK;
  const size_t es = f->info.elem_bytes;
  if (!A || !y || (n && !x) || lda < n) return FDOT_E_INVALID_ARG;
  if (!aligned_to(A, es) || !aligned_to(y, es) || (x && !aligned_to(x, es)))
    return FDOT_E_INVALID_ARG;
  if (f->opt.validate && n) {
    const FdCheck c[2] = {{A, m, n, lda}, {x, 1, n, n}};
    const fdot_status_t st = fd_validate_call(f, (hipStream_t)stream, c, 2, nullptr, 0, nullptr);
    if (st != FDOT_OK) return st;
  }
  return fd_launch_gemv(f, m, n, A, lda, x, y, (hipStream_t)stream);
}

fdot_status_t fgemm_modp(fdot_field_t f, size_t M, size_t N, size_t K, const void* A, size_t lda,
                         const void* B, size_t ldb, void* C, size_t ldc, void* stream) {
  if (!f) return FDOT_E_INVALID_ARG;
  if (f->host_only) return FDOT_E_UNSUPPORTED;
  if (f->degree > 1) return FDOT_E_UNSUPPORTED;
  if (M == 0 || N == 0) return FDOT_OK;
  const size_t es = f->info.elem_bytes;
  if (!C || ldc < N || (K && (!A || !B || lda < K || ldb < N))) return FDOT_E_INVALID_ARG;
  if (!aligned_to(C, es) || (A && !aligned_to(A, es)) || (B && !aligned_to(B, es)))
    return FDOT_E_INVALID_ARG;
  if (f->opt.validate && K) {
    const FdCheck c[2] = {{A, M, K, lda}, {B, K, N, ldb}};
    const fdot_status_t st = fd_validate_call(f, (hipStream_t)stream, c, 2, nullptr, 0, nullptr);
    if (st != FDOT_OK) return st;
  }
  return fd_launch_gemm(f, M, N, K, A, lda, B, ldb, C, ldc, (hipStream_t)stream);
}

}  // extern "C"
