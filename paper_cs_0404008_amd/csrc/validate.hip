// Input validation: counts of stored values that are not canonical in the
// field's representation.  The representations of Sec. 2 hold an element as
// a residue in [0, p) (classical and Montgomery), an integral double in
// [0, p) (Sec. 2.3), a discrete-log code in [0, q-1] (Sec. 2.4) or a centred
// residue in [-(p-1)/2, (p-1)/2] (Sec. 3.2.2); the dot-product kernels assume
// this and do not check it.  The public check (fdot_validate) adds the count
// to a caller's device word; a field created with the validate option runs
// the same kernels before every compute call and refuses non-canonical input.
#include <algorithm>

#include "fdot_internal.h"

namespace {

constexpr int VT = 256;

__device__ __forceinline__ bool canon(uint32_t v, const FieldK& F) { return v < F.p; }
__device__ __forceinline__ bool canon(double v, const FieldK& F) {
  return v >= 0.0 && v < F.P && v == floor(v);  // NaN fails the first test
}
__device__ __forceinline__ bool canon(uint16_t v, const FieldK& F) { return v < F.p; }
__device__ __forceinline__ bool canon(int8_t v, const FieldK& F) {
  return (int32_t)v >= -F.half && (int32_t)v <= F.half;
}

__device__ __forceinline__ void add_count(uint32_t bad, unsigned long long* count) {
  uint64_t b = bad;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) b += __shfl_xor(b, o, 64);
  if ((threadIdx.x & 63u) == 0 && b) atomicAdd(count, (unsigned long long)b);
}

// rows x cols elements at x with row stride ld (a vector: rows = 1).
template <typename E>
__global__ __launch_bounds__(VT) void noncanon_kernel(const FieldK F, const E* x, uint64_t rows,
                                                      uint64_t cols, uint64_t ld,
                                                      unsigned long long* count) {
  const uint64_t total = rows * cols;
  uint32_t bad = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * VT + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * VT) {
    const uint64_t r = i / cols, c = i - r * cols;
    bad += canon(x[r * ld + c], F) ? 0u : 1u;
  }
  add_count(bad, count);
}

// Both operands of every pair of a batch; workgroups take pairs in turn.
template <typename E>
__global__ __launch_bounds__(VT) void noncanon_many_kernel(const FieldK F, const fdot_desc_t* desc,
                                                           uint64_t count_pairs,
                                                           unsigned long long* count) {
  uint32_t bad = 0;
  for (uint64_t k = blockIdx.x; k < count_pairs; k += gridDim.x) {
    const E* x = (const E*)desc[k].x;
    const E* y = (const E*)desc[k].y;
    const uint64_t n = desc[k].n;
    for (uint64_t i = threadIdx.x; i < n; i += VT)
      bad += (canon(x[i], F) ? 0u : 1u) + (canon(y[i], F) ? 0u : 1u);
  }
  add_count(bad, count);
}

__global__ void clear_count_kernel(unsigned long long* w) { *w = 0; }

unsigned grid_for(uint64_t work) {
  const uint64_t cap = (uint64_t)fd_cu_count() * 8;
  const uint64_t g = (work + VT - 1) / VT;
  return (unsigned)(g < 1 ? 1 : g > cap ? cap : g);
}

fdot_status_t launch_count(const fdot_field_s* f, const void* x, uint64_t rows, uint64_t cols,
                           uint64_t ld, unsigned long long* count, hipStream_t s) {
  if (rows == 0 || cols == 0) return FDOT_OK;
  const unsigned g = grid_for(rows * cols);
  switch (f->info.rep) {
    case FDOT_REP_ZPZ_U32:
    case FDOT_REP_MONT_U32:
      hipLaunchKernelGGL(noncanon_kernel<uint32_t>, dim3(g), dim3(VT), 0, s, f->k,
                         (const uint32_t*)x, rows, cols, ld, count);
      break;
    case FDOT_REP_FP64:
      hipLaunchKernelGGL(noncanon_kernel<double>, dim3(g), dim3(VT), 0, s, f->k,
                         (const double*)x, rows, cols, ld, count);
      break;
    case FDOT_REP_ZECH_U16:
      hipLaunchKernelGGL(noncanon_kernel<uint16_t>, dim3(g), dim3(VT), 0, s, f->k,
                         (const uint16_t*)x, rows, cols, ld, count);
      break;
    case FDOT_REP_CENTRED_I8:
      hipLaunchKernelGGL(noncanon_kernel<int8_t>, dim3(g), dim3(VT), 0, s, f->k,
                         (const int8_t*)x, rows, cols, ld, count);
      break;
    default: return FDOT_E_INVALID_ARG;
  }
  return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
}

fdot_status_t count_many(const fdot_field_s* f, const fdot_desc_t* desc,
                                     uint64_t count_pairs, unsigned long long* count,
                                     hipStream_t s) {
  if (count_pairs == 0) return FDOT_OK;
  const unsigned g = (unsigned)std::min<uint64_t>(count_pairs, (uint64_t)fd_cu_count() * 8);
  switch (f->info.rep) {
    case FDOT_REP_ZPZ_U32:
    case FDOT_REP_MONT_U32:
      hipLaunchKernelGGL(noncanon_many_kernel<uint32_t>, dim3(g), dim3(VT), 0, s, f->k, desc,
                         count_pairs, count);
      break;
    case FDOT_REP_FP64:
      hipLaunchKernelGGL(noncanon_many_kernel<double>, dim3(g), dim3(VT), 0, s, f->k, desc,
                         count_pairs, count);
      break;
    case FDOT_REP_ZECH_U16:
      hipLaunchKernelGGL(noncanon_many_kernel<uint16_t>, dim3(g), dim3(VT), 0, s, f->k, desc,
                         count_pairs, count);
      break;
    case FDOT_REP_CENTRED_I8:
      hipLaunchKernelGGL(noncanon_many_kernel<int8_t>, dim3(g), dim3(VT), 0, s, f->k, desc,
                         count_pairs, count);
      break;
    default: return FDOT_E_INVALID_ARG;
  }
  return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
}

fdot_status_t clear_count(unsigned long long* count, hipStream_t s) {
  hipLaunchKernelGGL(clear_count_kernel, dim3(1), dim3(1), 0, s, count);
  return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
}

}  // namespace

// Validation of a call's inputs for a field created with the validate
// option: the operands' non-canonical elements are counted into the
// stream's check word, which the host then reads (the call waits for the
// stream); FDOT_E_NONCANON when any is found.  A stream under graph capture
// cannot be waited for: FDOT_E_UNSUPPORTED.
fdot_status_t fd_validate_call(const fdot_field_s* f, hipStream_t s, const FdCheck* parts,
                               int nparts, const fdot_desc_t* desc, uint64_t count_pairs,
                               unsigned long long* word) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return FDOT_E_UNSUPPORTED;
  fdot_status_t st = FDOT_OK;
  if (!word) {
    Workspace* w = nullptr;
    st = fd_workspace_get(s, 1, &w);
    if (st != FDOT_OK) return st;
    word = (unsigned long long*)(w->tq + kTqCheckWord);
  }
  st = clear_count(word, s);
  for (int i = 0; i < nparts && st == FDOT_OK; ++i)
    st = launch_count(f, parts[i].x, parts[i].rows, parts[i].cols, parts[i].ld, word, s);
  if (st == FDOT_OK && desc) st = count_many(f, desc, count_pairs, word, s);
  if (st != FDOT_OK) return st;
  unsigned long long bad = 0;
  if (hipMemcpyAsync(&bad, word, sizeof bad, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FDOT_E_DEVICE;
  return bad ? FDOT_E_NONCANON : FDOT_OK;
}

extern "C" fdot_status_t fdot_validate(fdot_field_t f, const void* x, size_t n, uint64_t* count,
                                       void* stream) {
  if (!f || !count || ((uintptr_t)count & 7u)) return FDOT_E_INVALID_ARG;
  if (f->host_only) return FDOT_E_UNSUPPORTED;
  if (n == 0) return FDOT_OK;
  if (!x || ((uintptr_t)x % f->info.elem_bytes)) return FDOT_E_INVALID_ARG;
  return launch_count(f, x, 1, n, n, (unsigned long long*)count, (hipStream_t)stream);
}
