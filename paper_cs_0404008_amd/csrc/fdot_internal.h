// Internal declarations of libfdot: the field object, the per-stream
// workspace, the tuning table and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "fdot.h"
#include "fdot_arith.h"

struct fdot_field_s {
  fdot_field_info_t info;
  fdot_options_t opt;   // creation options (all zero: defaults)
  FieldK k;             // device-ready constants (table pointers on device)
  int device;
  bool host_only;       // constants only: no device tables, no compute
  uint32_t degree;      // 1: GF(p); d > 1: GF(p^d) in discrete logs (k.p holds q)
  uint16_t* d_zval;     // Zech tables on the device (owned)
  uint16_t* d_zplus1;
  uint16_t* d_zidx;
  uint16_t* d_zpk;     // Zech, q <= 32768: plus-one table of the packed step (owned)
  int8_t* d_cinv;       // centred residues: table of inverses (owned)
};

// Most ranges of one batched launch (one per group of resident wavefronts).
constexpr uint32_t kMaxRanges = 1u << 16;

// Device scratch owned per stream: one combination word per pair (residue
// sum and finished-unit count, returned to zero by the wavefront that
// finishes the pair, so no clearing happens between calls), and the plan of
// a batch (pair positions and unit counts, first pair of each range, total
// and range length), rewritten by every batched call.

struct Workspace {
  int device = -1;
  size_t cap = 0;                     // pairs
  void* base = nullptr;
  unsigned long long* acc = nullptr;  // cap: combination words
  uint64_t* first = nullptr;          // cap: position of each pair in the padded sequence
  uint32_t* units = nullptr;          // cap: units of each pair
  uint32_t* start = nullptr;          // kMaxRanges: first pair of each range
  uint64_t* tq = nullptr;             // 8 words: the batch's range totals (0..2); word
                                      // kTqCheckWord counts non-canonical inputs
  bool captured = false;  // handed to a graph capture: never freed on growth
};

// Word of Workspace::tq that input validation counts into.
constexpr int kTqCheckWord = 4;

// One operand of a call to validate: rows x cols elements, row stride ld.
struct FdCheck {
  const void* x;
  uint64_t rows, cols, ld;
};

// Validation (validate.hip).  fd_validate_call counts the non-canonical
// elements of the listed operands (and of every pair of desc, if given)
// into `word` (NULL: the stream's workspace word), waits for the stream and
// returns FDOT_E_NONCANON if there are any.
fdot_status_t fd_validate_call(const fdot_field_s* f, hipStream_t s, const FdCheck* parts,
                               int nparts, const fdot_desc_t* desc, uint64_t count_pairs,
                               unsigned long long* word);
// Host check of a scalar operand (elementwise alpha) in the representation.
bool fd_canonical_host(const fdot_field_s* f, const void* value);

// Host-side helpers (host_field.cpp).
int fd_is_prime_u64(uint64_t n);
uint32_t fd_primitive_root(uint64_t p);
fdot_status_t fd_fill_params(uint64_t p, fdot_rep_t rep, fdot_field_info_t* out);
void fd_fieldk_from_info(const fdot_field_info_t* info, FieldK* k);
int fd_zech_build(uint64_t p, uint32_t g, uint16_t* value, uint16_t* index, uint16_t* plus1);
uint64_t fd_zech_packed_bytes(uint64_t q);
fdot_status_t fd_zech_packed_upload(const uint16_t* plus1, uint32_t q, fdot_field_s* f);

// Runtime (runtime.cpp).
fdot_status_t fd_workspace_get(hipStream_t s, size_t count, Workspace** out);
// Releases (stream-ordered) the workspace and the matrix scratch of stream s;
// called before a library-owned stream is destroyed.
void fd_workspace_release(hipStream_t s);
void fd_scratch_release(hipStream_t s);
// Per-stream device scratch of at least `bytes` (stream-ordered growth; under
// graph capture only an existing buffer that is large enough).
fdot_status_t fd_scratch_get(hipStream_t s, size_t bytes, void** out);
// Stream-ordered device allocation from the default pool, which keeps freed
// blocks for reuse.
hipError_t fd_alloc_async(void** p, size_t bytes, hipStream_t s);
int64_t fd_tune(const char* key, int64_t fallback);
// Kernel trace (fdot_trace_enable): fd_trace_begin records the start event of
// a traced kernel on s and returns its slot (-1 when tracing is off or the
// pool is full); fd_trace_end records its end.
int fd_trace_begin(hipStream_t s);
void fd_trace_end(hipStream_t s, int slot);
int fd_cu_count();

// Launchers (dot_kernels.hip, gemm_kernels.hip).  All validate nothing: the
// C-ABI layer has checked arguments.
fdot_status_t fd_launch_dot(const fdot_field_s* f, fdot_algo_t algo, const void* x,
                            const void* y, uint64_t n, void* result, Workspace* ws,
                            hipStream_t s);
fdot_status_t fd_launch_many(const fdot_field_s* f, fdot_algo_t algo, size_t count,
                             const fdot_desc_t* desc, void* results, Workspace* ws,
                             hipStream_t s);
fdot_status_t fd_launch_encode(const fdot_field_s* f, const uint32_t* canon, void* rep,
                               size_t n, hipStream_t s);
fdot_status_t fd_launch_decode(const fdot_field_s* f, const void* rep, uint32_t* canon,
                               size_t n, hipStream_t s);
fdot_status_t fd_launch_gemv(const fdot_field_s* f, size_t m, size_t n, const void* A,
                             size_t lda, const void* x, void* y, hipStream_t s);
fdot_status_t fd_launch_gemm(const fdot_field_s* f, size_t M, size_t N, size_t K,
                             const void* A, size_t lda, const void* B, size_t ldb,
                             void* C, size_t ldc, hipStream_t s);
fdot_status_t fd_launch_zero(void* ptr, size_t bytes, hipStream_t s);
fdot_status_t fd_launch_many_mixed(uint64_t count, const fdot_mixed_desc_t* desc,
                                   const fdot_field_s* const* fields, size_t nfields,
                                   void* results, hipStream_t s);
// GF(p^d) dot products; xor_values (characteristic 2 only): accumulate the
// products' values by exclusive or instead of their codes by the plus-one
// table.
fdot_status_t fd_launch_ext_many(const fdot_field_s* f, bool xor_values, uint64_t count,
                                 const fdot_desc_t* desc, uint16_t* results, hipStream_t s);
fdot_status_t fd_launch_ext_dot(const fdot_field_s* f, bool xor_values, const uint16_t* x,
                                const uint16_t* y, uint64_t n, uint16_t* result, hipStream_t s);
fdot_status_t fd_launch_elementwise(const fdot_field_s* f, fdot_ew_op_t op, uint64_t n,
                                    const void* alpha, const void* x, const void* y, void* r,
                                    hipStream_t s);
fdot_algo_t fd_default_algo(const fdot_field_s* f, uint64_t n);
