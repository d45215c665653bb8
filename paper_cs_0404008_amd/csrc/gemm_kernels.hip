// Matrix product C = A B over GF(p).
//
// Every entry of C is a dot product of a row of A with a column of B (Sec. 1:
// the dot product is the core of matrix multiplication), so the exactness
// argument of Sec. 3 carries over entry by entry.  This file holds the exact
// general kernel that serves every representation on the vector ALUs; the
// matrix-core kernels live in gemm_mfma.hip.
#include <string.h>

#include "fdot_internal.h"

namespace {

// Term value of one stored element: the residue for classical, floating,
// Zech and centred storage, the raw Montgomery residue X = x*B for
// Montgomery storage (its products carry B^2; one REDC at the end).
__device__ __forceinline__ uint32_t load_term(const FieldK& F, int rep, const void* base, size_t i) {
  switch (rep) {
    case FDOT_REP_ZPZ_U32:
    case FDOT_REP_MONT_U32: return ((const uint32_t*)base)[i];
    case FDOT_REP_FP64: return (uint32_t)((const double*)base)[i];
    case FDOT_REP_ZECH_U16: return F.zval[((const uint16_t*)base)[i]];
    case FDOT_REP_CENTRED_I8: {
      const int32_t c = ((const int8_t*)base)[i];
      return (uint32_t)(c < 0 ? c + (int32_t)F.p32 : c);
    }
  }
  return 0;
}

__device__ __forceinline__ void store_rep(const FieldK& F, int rep, void* base, size_t i, uint32_t r) {
  switch (rep) {
    case FDOT_REP_ZPZ_U32: ((uint32_t*)base)[i] = r; break;
    case FDOT_REP_MONT_U32: ((uint32_t*)base)[i] = redc(r, F); break;
    case FDOT_REP_FP64: ((double*)base)[i] = (double)r; break;
    case FDOT_REP_ZECH_U16: ((uint16_t*)base)[i] = F.zidx[r]; break;
    case FDOT_REP_CENTRED_I8:
      ((int8_t*)base)[i] = (int8_t)((int32_t)r > F.half ? (int32_t)r - (int32_t)F.p32 : (int32_t)r);
      break;
  }
}

// 64x64 output tile per workgroup, 4x4 entries per thread, K staged through
// LDS 16 at a time.  Each entry accumulates with the on-demand correction of
// Sec. 3.3 (64-bit sum, CORR = 2^64 mod p added on wrap), exact for any
// p < 2^32 and any K.
constexpr int VT = 64, VK = 16;
__global__ __launch_bounds__(256) void gemm_valu_kernel(const FieldK F, int rep, uint64_t M,
                                                        uint64_t N, uint64_t K, const void* A,
                                                        uint64_t lda, const void* B, uint64_t ldb,
                                                        void* C, uint64_t ldc) {
  __shared__ uint32_t As[VK][VT + 1];
  __shared__ uint32_t Bs[VK][VT + 1];
  const uint32_t tid = threadIdx.x;
  const uint32_t tx = tid & 15u, ty = tid >> 4;
  const uint64_t row0 = (uint64_t)blockIdx.y * VT, col0 = (uint64_t)blockIdx.x * VT;
  uint64_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0;
  for (uint64_t k0 = 0; k0 < K; k0 += VK) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const uint32_t e = tid + 256u * t;           // 0..1023
      const uint32_t ar = e / VK, ak = e % VK;     // A tile: 64 rows x 16 k
      const uint64_t gr = row0 + ar, gk = k0 + ak;
      As[ak][ar] = (gr < M && gk < K) ? load_term(F, rep, A, gr * lda + gk) : 0u;
      const uint32_t bk = e / VT, bc = e % VT;     // B tile: 16 k x 64 cols
      const uint64_t gk2 = k0 + bk, gc = col0 + bc;
      Bs[bk][bc] = (gk2 < K && gc < N) ? load_term(F, rep, B, gk2 * ldb + gc) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < VK; ++kk) {
      uint32_t a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint64_t prod = (uint64_t)a[i] * b[j];
          acc[i][j] += prod;
          if (acc[i][j] < prod) acc[i][j] += F.corr;
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint64_t r = row0 + ty + 16 * i, c = col0 + tx + 16 * j;
      if (r < M && c < N) store_rep(F, rep, C, r * ldc + c, mod_u64(acc[i][j], F));
    }
}

}  // namespace

fdot_status_t fd_launch_gemm_mfma(const fdot_field_s* f, size_t M, size_t N, size_t K,
                                  const void* A, size_t lda, const void* B, size_t ldb, void* C,
                                  size_t ldc, hipStream_t s, bool* handled);

fdot_status_t fd_launch_gemm_valu(const fdot_field_s* f, size_t M, size_t N, size_t K,
                                  const void* A, size_t lda, const void* B, size_t ldb, void* C,
                                  size_t ldc, hipStream_t s) {
  const dim3 grid((unsigned)((N + VT - 1) / VT), (unsigned)((M + VT - 1) / VT));
  if (grid.y > 65535) return FDOT_E_INVALID_ARG;
  hipLaunchKernelGGL(gemm_valu_kernel, grid, dim3(256), 0, s, f->k, f->info.rep, (uint64_t)M,
                     (uint64_t)N, (uint64_t)K, A, (uint64_t)lda, B, (uint64_t)ldb, C, (uint64_t)ldc);
  return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
}

fdot_status_t fd_launch_gemm(const fdot_field_s* f, size_t M, size_t N, size_t K, const void* A,
                             size_t lda, const void* B, size_t ldb, void* C, size_t ldc,
                             hipStream_t s) {
  if (fd_tune("gemm.force_valu", 0) == 0) {
    bool handled = false;
    fdot_status_t st = fd_launch_gemm_mfma(f, M, N, K, A, lda, B, ldb, C, ldc, s, &handled);
    if (handled) return st;
  }
  return fd_launch_gemm_valu(f, M, N, K, A, lda, B, ldb, C, ldc, s);
}
