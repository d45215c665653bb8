// Measured peaks, reported beside the datasheet figures: a plain read-only
// reduction (the rate at which HBM feeds a kernel that does nothing but read
// and add), and back-to-back matrix instructions on register operands (the
// rate at which the matrix cores retire work with no memory traffic; for
// int8 on constant and on pseudo-random operands).  No
// part of the method runs here; the roofline fractions of the library's
// kernels are quoted against both kinds of peak.
#include "fdot_internal.h"

namespace {

typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int RT = 256;  // threads per workgroup of the read kernel
constexpr int MT = 512;  // threads per workgroup of the matrix loops (8 wavefronts)
constexpr int CH = 4;    // independent accumulator chains per wavefront

__global__ void clear_word_kernel(unsigned long long* w) { *w = 0; }

// Sum of all 32-bit words mod 2^64; U 16-byte loads in flight per lane.
template <int U>
__global__ __launch_bounds__(RT) void read_sum_kernel(const v4u* x, uint64_t nv,
                                                      unsigned long long* result) {
  const uint64_t stride = (uint64_t)gridDim.x * RT;
  uint64_t i = (uint64_t)blockIdx.x * RT + threadIdx.x;
  uint64_t s0 = 0, s1 = 0;
  for (; i + (uint64_t)(U - 1) * stride < nv; i += (uint64_t)U * stride) {
    v4u a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) a[u] = __builtin_nontemporal_load(x + i + (uint64_t)u * stride);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      s0 += (uint64_t)a[u].x + a[u].z;
      s1 += (uint64_t)a[u].y + a[u].w;
    }
  }
  for (; i < nv; i += stride) {
    const v4u a = x[i];
    s0 += (uint64_t)a.x + a.z;
    s1 += (uint64_t)a.y + a.w;
  }
  uint64_t s = s0 + s1;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63u) == 0) atomicAdd(result, (unsigned long long)s);
}

// iters rounds of CH independent int8 products 32x32x32 per wavefront.  Every
// operand byte is a (resp. b), so each accumulator element gains 32ab per
// product; element 0 of chain 0 of the first wavefront is written out.
__global__ __launch_bounds__(MT) void mfma_i8_loop_kernel(uint32_t iters, int a, int b,
                                                          int32_t* result) {
  const uint32_t ra = (uint32_t)(a & 0xFF) * 0x01010101u;
  const uint32_t rb = (uint32_t)(b & 0xFF) * 0x01010101u;
  const v4i va = {(int)ra, (int)ra, (int)ra, (int)ra};
  const v4i vb = {(int)rb, (int)rb, (int)rb, (int)rb};
  v16i acc[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[c][e] = 0;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(va, vb, acc[c], 0, 0, 0);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) result[0] = acc[0][0];
  // keep the other chains live: three equal accumulators of 32ab per round
  // sum to a multiple of 32, never to this odd value
  int32_t other = 0;
#pragma unroll
  for (int c = 1; c < CH; ++c) other += acc[c][0];
  if (other == INT32_MIN + 1) result[1] = other;
}

// Operand words of the random-operand loop: the "lowbias32" integer hash
// (C. Wellons) of (lane, chain, word), mixed with the seed.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// The int8 loop on operands that look like data: every lane holds its own
// pseudo-random bytes (chain c of A: words mix(seed ^ mix(lane 256 + 4c + w)),
// B: words mix(seed ^ mix(lane 256 + 128 + w)), w < 4).  Matrix-core power,
// hence the clock the chip holds, depends on the operand bits: constant
// operands measure the issue rate, these the rate a product of random
// residues can reach with no memory traffic at all.  Element 0 of chain 0
// of the first wavefront gains sum_k A[0][k] B[k][0] per product, i.e. the
// bytewise dot products of lanes 0 and 32.
__global__ __launch_bounds__(MT) void mfma_i8_rand_loop_kernel(uint32_t iters, uint32_t seed,
                                                               int32_t* result) {
  const uint32_t lane = threadIdx.x & 63u;
  v4i va[CH], vb;
#pragma unroll
  for (int c = 0; c < CH; ++c)
#pragma unroll
    for (int w = 0; w < 4; ++w) va[c][w] = (int)mix32(seed ^ mix32(lane * 256u + 4u * c + w));
#pragma unroll
  for (int w = 0; w < 4; ++w) vb[w] = (int)mix32(seed ^ mix32(lane * 256u + 128u + w));
  v16i acc[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[c][e] = 0;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(va[c], vb, acc[c], 0, 0, 0);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) result[0] = acc[0][0];
  int32_t other = 0;
#pragma unroll
  for (int c = 1; c < CH; ++c) other ^= acc[c][0] ^ acc[c][15];
  if (other == 0x7FFFFFFF && blockIdx.x == 0 && threadIdx.x == 0) result[1] = other;
}

// The same with FP64 products 16x16x4: each element gains 4ab per product.
__global__ __launch_bounds__(MT) void mfma_f64_loop_kernel(uint32_t iters, double a, double b,
                                                           double* result) {
  v4d acc[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) acc[c] = (v4d){0.0, 0.0, 0.0, 0.0};
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) result[0] = acc[0][0];
  double other = 0.0;
#pragma unroll
  for (int c = 1; c < CH; ++c) other += acc[c][0];
  if (other != other) result[1] = other;  // NaN only from non-finite operands
}

}  // namespace

extern "C" fdot_status_t fdot_calib_read(const void* x, size_t n_words, uint32_t blocks,
                                         uint32_t unroll, uint64_t* result, void* stream) {
  if (!result || (n_words & 3u) || ((uintptr_t)result & 7u)) return FDOT_E_INVALID_ARG;
  if (n_words && (!x || ((uintptr_t)x & 15u))) return FDOT_E_INVALID_ARG;
  if (unroll != 4 && unroll != 8) return FDOT_E_INVALID_ARG;
  const hipStream_t s = (hipStream_t)stream;
  const uint32_t grid = blocks ? blocks : (uint32_t)fd_cu_count() * 8u;
  const uint64_t nv = n_words / 4;
  hipLaunchKernelGGL(clear_word_kernel, dim3(1), dim3(1), 0, s, (unsigned long long*)result);
  if (nv) {
    if (unroll == 8)
      hipLaunchKernelGGL(read_sum_kernel<8>, dim3(grid), dim3(RT), 0, s, (const v4u*)x, nv,
                         (unsigned long long*)result);
    else
      hipLaunchKernelGGL(read_sum_kernel<4>, dim3(grid), dim3(RT), 0, s, (const v4u*)x, nv,
                         (unsigned long long*)result);
  }
  return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
}

extern "C" fdot_status_t fdot_calib_mfma(int kind, uint32_t blocks, uint32_t iters, double a,
                                         double b, void* result, uint64_t* ops, void* stream) {
  if (!result || kind < 0 || kind > 2 || ((uintptr_t)result & 7u)) return FDOT_E_INVALID_ARG;
  if (kind == 0 && !(a >= -128.0 && a <= 127.0 && b >= -128.0 && b <= 127.0 &&
                     a == (double)(int)a && b == (double)(int)b))
    return FDOT_E_INVALID_ARG;
  if (kind == 2 && !(a >= 0.0 && a <= 4294967295.0 && a == (double)(uint32_t)a))
    return FDOT_E_INVALID_ARG;
  const hipStream_t s = (hipStream_t)stream;
  const uint32_t grid = blocks ? blocks : (uint32_t)fd_cu_count() * 2u;
  const uint64_t per_product = kind != 1 ? 2ull * 32 * 32 * 32 : 2ull * 16 * 16 * 4;
  if (ops) *ops = (uint64_t)grid * (MT / 64) * iters * CH * per_product;
  if (kind == 2)
    hipLaunchKernelGGL(mfma_i8_rand_loop_kernel, dim3(grid), dim3(MT), 0, s, iters,
                       (uint32_t)a, (int32_t*)result);
  else if (kind == 0)
    hipLaunchKernelGGL(mfma_i8_loop_kernel, dim3(grid), dim3(MT), 0, s, iters, (int)a, (int)b,
                       (int32_t*)result);
  else
    hipLaunchKernelGGL(mfma_f64_loop_kernel, dim3(grid), dim3(MT), 0, s, iters, a, b,
                       (double*)result);
  return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
}
