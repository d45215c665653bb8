// Device twin of the host input generator (synth/__init__.py): the same
// SplitMix64 counter stream and Lemire multiply-shift range reduction, so that
// inputs too large to build on the host are written straight into HBM with the
// same bits.  Input generation only; nothing of the dot-product method.
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GOLDEN_GAMMA 0x9E3779B97F4A7C15ull

__host__ __device__ static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return mix64(mix64(seed + GOLDEN_GAMMA) + stream * GOLDEN_GAMMA);
}

// dtype: 0 = uint32, 1 = uint16, 2 = double, 3 = int8, 4 = int64
template <typename T>
__global__ void synth_fill_kernel(uint64_t k, uint64_t offset, uint64_t n,
                                  uint64_t m, int64_t lo, T* out) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    uint64_t z = mix64(k + (offset + i + 1) * GOLDEN_GAMMA);
    uint64_t u = ((z >> 32) * m) >> 32;
    out[i] = (T)((int64_t)u + lo);
  }
}

extern "C" int synth_fill(uint64_t seed, uint64_t stream, uint64_t offset,
                          uint64_t n, uint64_t m, int64_t lo, int dtype,
                          void* out, void* stream_handle) {
  if (n == 0) return 0;
  if (m == 0 || m > (1ull << 32) || out == nullptr) return -1;
  hipStream_t s = (hipStream_t)stream_handle;
  uint64_t k = stream_key(seed, stream);
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  dim3 grid((unsigned)blocks), block(256);
  switch (dtype) {
    case 0: hipLaunchKernelGGL(synth_fill_kernel<uint32_t>, grid, block, 0, s, k, offset, n, m, lo, (uint32_t*)out); break;
    case 1: hipLaunchKernelGGL(synth_fill_kernel<uint16_t>, grid, block, 0, s, k, offset, n, m, lo, (uint16_t*)out); break;
    case 2: hipLaunchKernelGGL(synth_fill_kernel<double>, grid, block, 0, s, k, offset, n, m, lo, (double*)out); break;
    case 3: hipLaunchKernelGGL(synth_fill_kernel<int8_t>, grid, block, 0, s, k, offset, n, m, lo, (int8_t*)out); break;
    case 4: hipLaunchKernelGGL(synth_fill_kernel<int64_t>, grid, block, 0, s, k, offset, n, m, lo, (int64_t*)out); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}
