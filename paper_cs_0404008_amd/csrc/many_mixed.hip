// Batched dot products over several prime fields in one call: for each
// field, the pairs of the other fields are masked to length 0 (the batched
// path then spends no range on them and writes their encoded zero), the
// batched path of that field runs, and a merge copies each pair's own result
// into place.  Per-stream scratch holds the masked descriptors and one
// field's results; it grows stream-ordered, outside graph capture.
#include <algorithm>
#include <map>
#include <mutex>
#include <set>

#include "fdot_internal.h"

namespace {

__global__ void mask_desc_kernel(const fdot_mixed_desc_t* in, uint64_t count, uint32_t field,
                                 fdot_desc_t* out) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const fdot_mixed_desc_t d = in[i];
    out[i].x = d.x;
    out[i].y = d.y;
    out[i].n = d.field == field ? d.n : 0;
  }
}

template <typename E>
__global__ void merge_kernel(const E* field_results, const fdot_mixed_desc_t* desc, uint64_t count,
                             uint32_t field, E* results) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * blockDim.x)
    if (desc[i].field == field) results[i] = field_results[i];
}

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, std::pair<void*, size_t>> g_buf;
std::set<void*> g_captured;  // held by a captured graph: never freed

fdot_status_t buffer_for(hipStream_t s, size_t bytes, void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return FDOT_E_DEVICE;
  std::lock_guard<std::mutex> g(g_mu);
  auto& e = g_buf[std::make_pair(dev, s)];
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const bool capturing =
      hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
  if (e.second >= bytes) {
    if (capturing) g_captured.insert(e.first);
    *out = e.first;
    return FDOT_OK;
  }
  if (capturing) return FDOT_E_BUSY;  // growing allocates
  bytes = std::max(bytes, e.second + e.second / 2);
  void* p = nullptr;
  if (fd_alloc_async(&p, bytes, s) != hipSuccess) return FDOT_E_NOMEM;
  if (e.first && !g_captured.count(e.first)) (void)hipFreeAsync(e.first, s);
  e = std::make_pair(p, bytes);
  *out = p;
  return FDOT_OK;
}

}  // namespace

fdot_status_t fd_launch_many_mixed(uint64_t count, const fdot_mixed_desc_t* desc,
                                   const fdot_field_s* const* fields, size_t nfields,
                                   void* results, hipStream_t s) {
  const size_t es = fields[0]->info.elem_bytes;
  const size_t desc_bytes = (count * sizeof(fdot_desc_t) + 255) / 256 * 256;
  void* buf = nullptr;
  fdot_status_t st = buffer_for(s, desc_bytes + count * es + 16, &buf);
  if (st != FDOT_OK) return st;
  fdot_desc_t* masked = (fdot_desc_t*)buf;
  void* field_results = (char*)buf + desc_bytes;
  Workspace* w = nullptr;
  st = fd_workspace_get(s, count, &w);
  if (st != FDOT_OK) return st;
  const unsigned grid = (unsigned)std::min<uint64_t>((count + 255) / 256, 4096);
  for (size_t f = 0; f < nfields; ++f) {
    hipLaunchKernelGGL(mask_desc_kernel, dim3(grid), dim3(256), 0, s, desc, count, (uint32_t)f,
                       masked);
    if (hipGetLastError() != hipSuccess) return FDOT_E_DEVICE;
    st = fd_launch_many(fields[f], FDOT_ALGO_AUTO, count, masked, field_results, w, s);
    if (st != FDOT_OK) return st;
    switch (es) {
      case 1: hipLaunchKernelGGL(merge_kernel<uint8_t>, dim3(grid), dim3(256), 0, s,
                                 (const uint8_t*)field_results, desc, count, (uint32_t)f,
                                 (uint8_t*)results); break;
      case 2: hipLaunchKernelGGL(merge_kernel<uint16_t>, dim3(grid), dim3(256), 0, s,
                                 (const uint16_t*)field_results, desc, count, (uint32_t)f,
                                 (uint16_t*)results); break;
      case 4: hipLaunchKernelGGL(merge_kernel<uint32_t>, dim3(grid), dim3(256), 0, s,
                                 (const uint32_t*)field_results, desc, count, (uint32_t)f,
                                 (uint32_t*)results); break;
      default: hipLaunchKernelGGL(merge_kernel<uint64_t>, dim3(grid), dim3(256), 0, s,
                                  (const uint64_t*)field_results, desc, count, (uint32_t)f,
                                  (uint64_t*)results); break;
    }
    if (hipGetLastError() != hipSuccess) return FDOT_E_DEVICE;
  }
  return FDOT_OK;
}
