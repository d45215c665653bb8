// Matrix-core (MFMA) kernels for the exact matrix product C = A B over GF(p).
//
// Exactness.  Every entry of C is a dot product (Sec. 1), so the delayed
// reduction of Sec. 3.1 applies to the K loop: products of residues are
// accumulated on the matrix cores and the accumulator is folded back to a
// residue every K-block, with the block chosen so that no partial sum can
// leave the exact range of the accumulator:
//  * FP64: integral doubles are exact up to 2^53 (Eq. 1 with m = 53), and a
//    sum of exact integers below 2^53 is the same whatever order the matrix
//    core adds them in.  Residues are used as stored, or centred
//    (Sec. 3.2.2) for primes whose squares leave too little room.
//  * int8: centred residues of p < 2^8, 32-bit integer accumulation, folded
//    before |sum| could reach 2^31 (the centred bound of Sec. 3.2.2).
//
// Operand layouts of the gfx950 instructions used (one wavefront):
//  v_mfma_f64_16x16x4_f64: lane l holds A[l%16][l/16] and B[l/16][l%16]; its
//    four results are D[4r + l/16][l%16], r = 0..3.
//  v_mfma_i32_32x32x32_i8: lane l holds 16 int8 of row l%32 of A and of
//    column l%32 of B, for the k-slots 16*(l/32) .. 16*(l/32)+15 (any
//    assignment of k-slots works as long as A and B use the same one); its 16
//    results are D[8(r/4) + 4(l/32) + r%4][l%32].
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <set>
#include <type_traits>
#include <utility>

#include "fdot_internal.h"

typedef double v4d __attribute__((ext_vector_type(4)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

namespace {

// Global-memory load through an address-space-1 pointer (a global load, not
// a flat one the compiler would have to wait for together with LDS traffic).
template <typename T>
__device__ __forceinline__ T gld(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}

// Workgroups are dispatched to the 8 XCDs round-robin (block b runs on XCD
// b mod 8).  Remap so that each XCD gets a contiguous range of output tiles,
// then walk tiles in bands of kBand tile-rows, so the tiles sharing A and B
// panels run on the same XCD, close in time, and hit its L2.
constexpr int kXcds = 8;
constexpr int kBand = 8;
__device__ __forceinline__ void tile_of(uint32_t b, uint32_t nblocks, uint32_t tiles_m,
                                        uint32_t tiles_n, uint32_t* tm, uint32_t* tn) {
  uint32_t t = b;
  if (nblocks % kXcds == 0) t = (b % kXcds) * (nblocks / kXcds) + b / kXcds;
  const uint32_t band_tiles = kBand * tiles_n;
  const uint32_t band = t / band_tiles;
  const uint32_t in_band = t % band_tiles;
  const uint32_t rows = (tiles_m - band * kBand) < kBand ? (tiles_m - band * kBand) : kBand;
  *tm = band * kBand + in_band % rows;
  *tn = in_band / rows;
}

// ------------------------------------------------------------------ FP64
constexpr int FM = 128, FN = 128, FK = 16;

template <typename E, bool CENTRE>
__device__ __forceinline__ double to_term(E v, const FieldK& F) {
  double d = (double)v;
  if (CENTRE) d = d > (double)F.half ? d - F.P : d;
  return d;
}

__device__ __forceinline__ double fold_keep(double acc, const FieldK& F, bool centre) {
  double r = fold_f64(acc, F);
  if (centre) r = r > (double)F.half ? r - F.P : r;
  return r;
}

// Two consecutive elements of a row as terms.  VEC: one 16-byte (double) or
// 8-byte (uint32) load, the caller having checked alignment and bounds.
template <typename E, bool CENTRE, bool VEC>
__device__ __forceinline__ void load_pair(const E* base, uint64_t off, bool in0, bool in1,
                                          const FieldK& F, double& t0, double& t1) {
  if (VEC && in1) {
    if constexpr (sizeof(E) == 8) {
      typedef double d2 __attribute__((ext_vector_type(2)));
      const d2 v = gld((const d2*)(base + off));
      t0 = to_term<E, CENTRE>((E)v.x, F);
      t1 = to_term<E, CENTRE>((E)v.y, F);
    } else {
      typedef unsigned int u2 __attribute__((ext_vector_type(2)));
      const u2 v = gld((const u2*)(base + off));
      t0 = to_term<E, CENTRE>((E)v.x, F);
      t1 = to_term<E, CENTRE>((E)v.y, F);
    }
  } else {
    t0 = in0 ? to_term<E, CENTRE>(gld(base + off), F) : 0.0;
    t1 = in1 ? to_term<E, CENTRE>(gld(base + off + 1), F) : 0.0;
  }
}

// C tile 128 x 128 per workgroup; wavefront w owns rows 64*(w/2).., columns
// 64*(w%2).. as 4 x 4 blocks of 16 x 16.  K is staged through two LDS
// buffers 16 at a time (A row-major with a padded pitch, B as stored),
// consumed in 4 steps of one MFMA K (4); the next K-tile is fetched into
// registers while the current one is multiplied and staged into LDS halfway
// through it.  The accumulators are folded after every fold_sub MFMA
// steps (SUBFOLD, for block lengths below one K-tile) or K-tiles.
constexpr int FAP = FK + 1;    // A pitch in LDS (doubles): conflict-free column reads
constexpr int FBP = FN + 2;    // B pitch in LDS (doubles): keeps 16-byte alignment
constexpr size_t kF64Lds = (size_t)2 * (FM * FAP + FK * FBP) * sizeof(double);  // two buffers
// With four wavefronts the register budget is held to two wavefronts per
// SIMD (256 registers a lane), so that two workgroups share a CU; left to
// itself the compiler takes about 340 and only one fits.
template <typename E, bool CENTRE, bool VEC, bool SUBFOLD, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW == 4 ? 2 : 1)))
void gemm_f64_kernel(const FieldK F, int rep, uint32_t M, uint32_t N, uint32_t K, const E* A,
                     uint64_t lda, const E* B, uint64_t ldb, void* C, uint64_t ldc,
                     uint32_t fold_sub) {
  extern __shared__ __attribute__((aligned(16))) double s_f64[];
  double* const As0 = s_f64;                   // [2][FM * FAP]
  double* const Bs0 = s_f64 + 2 * FM * FAP;    // [2][FK * FBP]
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  const uint32_t tiles_m = (M + FM - 1) / FM, tiles_n = (N + FN - 1) / FN;
  uint32_t tm, tn;
  tile_of(blockIdx.x, gridDim.x, tiles_m, tiles_n, &tm, &tn);
  const uint32_t m0 = tm * FM, n0 = tn * FN;
  // NW = 4: wavefront w owns a 64 x 64 sub-tile (4 x 4 blocks of 16 x 16);
  // NW = 8: a 32 x 64 sub-tile (2 x 4 blocks), two wavefronts per SIMD;
  // NW = 16: a 16 x 64 sub-tile, four per SIMD.
  constexpr int NT = 64 * NW, BI = 16 / NW, QN = 1024 / NT;
  const uint32_t wm = (w >> 1) * (16 * BI), wn = (w & 1) * 64;
  // This thread's share of a K-tile: QN pairs of A (row ar + (NT/8) q,
  // columns ak, ak+1) and QN pairs of B (row bk + NW q, columns bc, bc+1).
  const uint32_t ar = tid / 8, ak = 2 * (tid % 8);
  const uint32_t bk = tid / 64, bc = 2 * (tid % 64);
  // VEC: every fetch is one unconditional load of an element pair (rows
  // start on a pair boundary and K and N are even, so a pair whose first
  // element is inside the matrix lies inside it; pairs outside are read from
  // the matrix's first pair), masked and converted when staged: no
  // branch separates a load from its use, so a K-tile's loads stay in flight
  // together.  Otherwise element loads under bounds checks.
  typedef typename std::conditional<sizeof(E) == 8, double, unsigned int>::type S1;
  typedef S1 S2 __attribute__((ext_vector_type(2)));
  S2 xa[QN], xb[QN];
  uint32_t oka = 0, okb = 0;
  double ra[QN][2], rb[QN][2];
  auto fetch = [&](uint32_t k0) {
    if constexpr (VEC) {
      oka = okb = 0;
#pragma unroll
      for (int q = 0; q < QN; ++q) {
        const uint32_t gm = m0 + ar + (NT / 8) * q, gk = k0 + ak;
        const bool a0 = gm < M && gk < K, a1 = a0 && gk + 1 < K;
        xa[q] = gld((const S2*)(A + (a0 ? (uint64_t)gm * lda + gk : 0)));
        oka |= ((uint32_t)a0 | (uint32_t)a1 << 1) << (2 * q);
        const uint32_t gk2 = k0 + bk + NW * q, gn = n0 + bc;
        const bool b0 = gk2 < K && gn < N, b1 = b0 && gn + 1 < N;
        xb[q] = gld((const S2*)(B + (b0 ? (uint64_t)gk2 * ldb + gn : 0)));
        okb |= ((uint32_t)b0 | (uint32_t)b1 << 1) << (2 * q);
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      const uint32_t gm = m0 + ar + (NT / 8) * q, gk = k0 + ak;
      const bool rin = gm < M;
      load_pair<E, CENTRE, VEC>(A, (uint64_t)gm * lda + gk, rin && gk < K, rin && gk + 1 < K, F,
                                ra[q][0], ra[q][1]);
      const uint32_t gk2 = k0 + bk + NW * q, gn = n0 + bc;
      const bool kin = gk2 < K;
      load_pair<E, CENTRE, VEC>(B, (uint64_t)gk2 * ldb + gn, kin && gn < N, kin && gn + 1 < N, F,
                                rb[q][0], rb[q][1]);
    }
  };
  v4d acc[BI][4];
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};
  auto stage = [&](int buf) {
    double* As = As0 + buf * FM * FAP;
    double* Bs = Bs0 + buf * FK * FBP;
    if constexpr (VEC) {
#pragma unroll
      for (int q = 0; q < QN; ++q) {
        ra[q][0] = (oka >> (2 * q)) & 1u ? to_term<E, CENTRE>((E)xa[q].x, F) : 0.0;
        ra[q][1] = (oka >> (2 * q + 1)) & 1u ? to_term<E, CENTRE>((E)xa[q].y, F) : 0.0;
        rb[q][0] = (okb >> (2 * q)) & 1u ? to_term<E, CENTRE>((E)xb[q].x, F) : 0.0;
        rb[q][1] = (okb >> (2 * q + 1)) & 1u ? to_term<E, CENTRE>((E)xb[q].y, F) : 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < QN; ++q) {
      As[(ar + (NT / 8) * q) * FAP + ak] = ra[q][0];
      As[(ar + (NT / 8) * q) * FAP + ak + 1] = ra[q][1];
      Bs[(bk + NW * q) * FBP + bc] = rb[q][0];
      Bs[(bk + NW * q) * FBP + bc + 1] = rb[q][1];
    }
  };
  auto fold_all = [&]() {
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][j][r] = fold_keep(acc[i][j][r], F, CENTRE);
  };
  // Two LDS buffers: the next K-tile, fetched into registers during the
  // current one's products, is staged into the other buffer, so one barrier
  // per K-tile suffices.
  uint32_t sub = 0;
  if (K > 0) {
    fetch(0);
    stage(0);
    __syncthreads();
    if (FK < K) fetch(FK);
  }
  uint32_t t = 0;
  for (uint32_t k0 = 0; k0 < K; k0 += FK, ++t) {
    const int buf = t & 1;
    const double* As = As0 + buf * FM * FAP;
    const double* Bs = Bs0 + buf * FK * FBP;
#pragma unroll
    for (int s = 0; s < FK / 4; ++s) {
      const uint32_t kr = 4 * s + lane / 16;
      double a[BI], b[4];
#pragma unroll
      for (int i = 0; i < BI; ++i) a[i] = As[(wm + 16 * i + lane % 16) * FAP + kr];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kr * FBP + wn + 16 * j + lane % 16];
#pragma unroll
      for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
      if (SUBFOLD && ++sub == fold_sub) {
        fold_all();
        sub = 0;
      }
      // The next K-tile goes into the other buffer halfway through this
      // one's products (nobody reads that buffer since the last barrier),
      // so its waits and LDS writes overlap the remaining matrix products
      // instead of sitting between the last product and the barrier.
      if (s == 1 && k0 + FK < K) stage(buf ^ 1);
    }
    __syncthreads();  // the other buffer is complete; nobody reads this one any more
    if (k0 + 2 * FK < K) fetch(k0 + 2 * FK);
    // Without SUBFOLD, fold_sub counts whole K-tiles.
    if (!SUBFOLD && ++sub == fold_sub) {
      fold_all();
      sub = 0;
    }
  }
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t gm = m0 + wm + 16 * i + 4 * r + lane / 16;
        const uint32_t gn = n0 + wn + 16 * j + lane % 16;
        if (gm < M && gn < N) {
          const uint32_t v = (uint32_t)fold_f64(acc[i][j][r], F);
          const uint64_t o = (uint64_t)gm * ldc + gn;
          if (rep == FDOT_REP_FP64) ((double*)C)[o] = (double)v;
          else if (rep == FDOT_REP_MONT_U32) ((uint32_t*)C)[o] = redc(v, F);
          else ((uint32_t*)C)[o] = v;
        }
      }
}

// ------------------------------------------------------------------ int8
constexpr int IPAD = 16;

// Signed 32-bit value to its centred residue, through a double quotient.
__device__ __forceinline__ int32_t centred_mod(int32_t v, const FieldK& F) {
  const double q = floor((double)v * F.invP);
  int32_t r = v - (int32_t)q * (int32_t)F.p32;
  r = r >= (int32_t)F.p32 ? r - (int32_t)F.p32 : r;
  r = r < 0 ? r + (int32_t)F.p32 : r;
  return r > F.half ? r - (int32_t)F.p32 : r;
}

// C tile (64 BI) x (64 BJ) per workgroup from A (M x K, int8 row-major) and
// Bt = B^T (N x K, int8 row-major); wavefront w owns a (32 BI) x (32 BJ)
// sub-tile as BI x BJ blocks of 32 x 32.  K is staged IK at a time (rows
// padded by 16 bytes in LDS, so the 16-byte fragment reads of 16 lanes hit
// distinct banks) and consumed in MFMA steps of 32; the next K-tile is
// fetched into registers while the current one is multiplied.  Accumulators
// are folded (to centred residues) after every fold_steps stagings.
// Output of one int8 product.  Centred residues: the int8 result.  SPLIT
// (digit products of larger residues): Cu += (acc mod p) w, mod p, for the
// digit pair's weight w < p (each output is owned by one lane of one launch,
// and the launches of a product run in order on one stream).
// Centred residue of a finished int8 tile entry.
__device__ __forceinline__ void i8_store(int8_t* C, uint64_t o, int32_t acc, const FieldK& F) {
  C[o] = (int8_t)centred_mod(acc, F);
}

// x * w mod p for any x < 2^32 by Shoup's method: wgt holds w < p in its low
// half and floor(w 2^32 / p) in its high half, so the quotient estimate is
// one multiply-high and falls short of the true quotient by at most one.
__device__ __forceinline__ uint32_t mulmod_pre(uint32_t x, uint64_t wgt, const FieldK& F) {
  const uint64_t q = ((uint64_t)x * (wgt >> 32)) >> 32;
  const uint64_t r = (uint64_t)x * (uint32_t)wgt - q * F.p;
  return (uint32_t)(r >= F.p ? r - F.p : r);
}

// Digit-product epilogue for one 32-row block of a wavefront's tile:
// Cu = (Cu + acc * w) mod p for its 32 x 32*BJ entries, or Cu = acc * w mod
// p for the first product of a sum (fresh: Cu is not read, so it needs no
// clearing beforehand).  A negative acc is
// first lifted by pm, the least multiple of p that is at least 2^31, so that
// the multiplier sees a value in [0, 2^32).  The products replace the
// accumulators in place; then every load of Cu is issued before the first
// store, so their latencies overlap.  Requires M, N >= 1.
template <int BJ>
__device__ __forceinline__ void split_rows(uint32_t* Cu, uint64_t ldc, uint64_t wgt, v16i* acc,
                                           uint32_t row0, uint32_t col0, uint32_t lane,
                                           uint32_t M, uint32_t N, uint64_t pm,
                                           const FieldK& F, uint32_t fresh) {
#pragma unroll
  for (int j = 0; j < BJ; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t a = acc[j][r];
      acc[j][r] = (int32_t)mulmod_pre((uint32_t)(a < 0 ? a + (int64_t)pm : a), wgt, F);
    }
  uint32_t old[BJ][16] = {};
  if (!fresh) {
#pragma unroll
    for (int j = 0; j < BJ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const uint32_t gm = row0 + 8 * (r / 4) + 4 * (lane / 32) + r % 4;
        const uint32_t gn = col0 + 32 * j + lane % 32;
        // clamped (always valid) addresses keep the loads unconditional, so
        // they are all in flight together; entries outside C are not stored
        old[j][r] = Cu[(uint64_t)min(gm, M - 1) * ldc + min(gn, N - 1)];
      }
  }
#pragma unroll
  for (int j = 0; j < BJ; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const uint32_t gm = row0 + 8 * (r / 4) + 4 * (lane / 32) + r % 4;
      const uint32_t gn = col0 + 32 * j + lane % 32;
      if (gm < M && gn < N) {
        const uint64_t t = (uint64_t)old[j][r] + (uint32_t)acc[j][r];
        Cu[(uint64_t)gm * ldc + gn] = (uint32_t)(t >= F.p ? t - F.p : t);
      }
    }
}

template <int BI, int BJ, int IK, bool VEC, bool SPLIT = false>
__global__ __launch_bounds__(256) void gemm_i8_kernel(const FieldK F, uint32_t M, uint32_t N,
                                                      uint32_t K, const int8_t* A, uint64_t lda,
                                                      const int8_t* Bt, uint64_t ldbt, int8_t* C,
                                                      uint64_t ldc, uint32_t fold_steps,
                                                      uint32_t* Cu = nullptr, uint64_t wgt = 0,
                        uint32_t fresh = 0) {
  constexpr int TM = 64 * BI, TN = 64 * BJ;
  constexpr int NA = TM * IK / 16 / 256, NB = TN * IK / 16 / 256;  // 16-byte vectors per thread
  // Two LDS buffers where both fit in 64 KiB: the next K-tile is written to
  // the other buffer halfway through this one's products, one barrier per
  // K-tile.  Otherwise one buffer, written between two barriers.
  constexpr bool DB = 2 * (TM + TN) * (IK + IPAD) <= 65536;
  constexpr int NBUF = DB ? 2 : 1;
  __shared__ __attribute__((aligned(16))) int8_t As[NBUF][TM][IK + IPAD];
  __shared__ __attribute__((aligned(16))) int8_t Bs[NBUF][TN][IK + IPAD];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  const uint32_t tiles_m = (M + TM - 1) / TM, tiles_n = (N + TN - 1) / TN;
  uint32_t tm, tn;
  tile_of(blockIdx.x, gridDim.x, tiles_m, tiles_n, &tm, &tn);
  const uint32_t m0 = tm * TM, n0 = tn * TN;
  const uint32_t wm = (w >> 1) * 32 * BI, wn = (w & 1) * 32 * BJ;
  v4i pa[NA], pb[NB];
  auto fetch_row = [&](const int8_t* base, uint64_t ld, uint32_t row, uint32_t rows, uint32_t gk) {
    v4i v = {0, 0, 0, 0};
    if (row >= rows) return v;
    if (VEC && gk + 16 <= K) return gld((const v4i*)(base + (uint64_t)row * ld + gk));
    int8_t t[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) t[i] = gk + i < K ? gld(base + (uint64_t)row * ld + gk + i) : (int8_t)0;
    __builtin_memcpy(&v, t, 16);
    return v;
  };
  auto fetch = [&](uint32_t k0) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const uint32_t e = tid + 256u * q;
      pa[q] = fetch_row(A, lda, m0 + e / (IK / 16), M, k0 + (e % (IK / 16)) * 16);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const uint32_t e = tid + 256u * q;
      pb[q] = fetch_row(Bt, ldbt, n0 + e / (IK / 16), N, k0 + (e % (IK / 16)) * 16);
    }
  };
  v16i acc[BI][BJ];
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;
  auto stage = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const uint32_t e = tid + 256u * q;
      *(v4i*)&As[buf][e / (IK / 16)][(e % (IK / 16)) * 16] = pa[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const uint32_t e = tid + 256u * q;
      *(v4i*)&Bs[buf][e / (IK / 16)][(e % (IK / 16)) * 16] = pb[q];
    }
  };
  uint32_t steps = 0;
  if (K > 0) fetch(0);
  if (DB && K > 0) {
    stage(0);
    __syncthreads();
    if (IK < K) fetch(IK);
  }
  uint32_t t = 0;
  for (uint32_t k0 = 0; k0 < K; k0 += IK, ++t) {
    const int buf = DB ? (int)(t & 1) : 0;
    if (!DB) {
      __syncthreads();
      stage(0);
      __syncthreads();
      if (k0 + IK < K) fetch(k0 + IK);
    }
#pragma unroll
    for (int s = 0; s < IK / 32; ++s) {
      const uint32_t kc = 32 * s + 16 * (lane / 32);
      v4i a[BI], b[BJ];
#pragma unroll
      for (int i = 0; i < BI; ++i) a[i] = *(const v4i*)&As[buf][wm + 32 * i + lane % 32][kc];
#pragma unroll
      for (int j = 0; j < BJ; ++j) b[j] = *(const v4i*)&Bs[buf][wn + 32 * j + lane % 32][kc];
#pragma unroll
      for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[j], acc[i][j], 0, 0, 0);
      // the other buffer has had no reader since the last barrier
      if (DB && s == IK / 64 && k0 + IK < K) stage(buf ^ 1);
    }
    if (DB) {
      __syncthreads();  // the other buffer is complete; nobody reads this one any more
      if (k0 + 2 * IK < K) fetch(k0 + 2 * IK);
    }
    if (++steps == fold_steps) {
#pragma unroll
      for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[i][j][r] = centred_mod(acc[i][j][r], F);
      steps = 0;
    }
  }
  if constexpr (SPLIT) {
    const uint64_t pm = (0x80000000ull + F.p - 1) / F.p * F.p;
#pragma unroll
    for (int i = 0; i < BI; ++i)
      split_rows<BJ>(Cu, ldc, wgt, acc[i], m0 + wm + 32 * i, n0 + wn, lane, M, N, pm, F,
                     fresh);
    return;
  }
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const uint32_t gm = m0 + wm + 32 * i + 8 * (r / 4) + 4 * (lane / 32) + r % 4;
        const uint32_t gn = n0 + wn + 32 * j + lane % 32;
        if (gm < M && gn < N) i8_store(C, (uint64_t)gm * ldc + gn, acc[i][j][r], F);
      }
}

// Large-tile int8 kernel: C tile 256 x 256 per workgroup, each wavefront a
// 128 x 128 sub-tile as 4 x 4 blocks of 32 x 32 (the accumulators, 256
// registers per lane, live in the accumulation registers; one wavefront per
// SIMD).  Per MFMA the wavefront reads half as many LDS bytes as with 2 x 2
// blocks.  K is staged IK at a time through two LDS buffers: the next
// K-tile, fetched into registers during the current one's products, is
// written to the other buffer, so one barrier per K-tile suffices.  FOLDS:
// the accumulators are folded inside the loop, which keeps them in ordinary
// registers and spills; the launcher uses this kernel only when K fits one
// fold block (FOLDS false: accumulators read once, at the end).
template <int IK, int BJ, bool VEC, bool FOLDS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BJ == 4 ? 1 : 2, BJ == 4 ? 1 : 2)))
void gemm_i8_big_kernel(const FieldK F, uint32_t M, uint32_t N, uint32_t K, const int8_t* A,
                        uint64_t lda, const int8_t* Bt, uint64_t ldbt, int8_t* C, uint64_t ldc,
                        uint32_t fold_steps) {
  constexpr int TM = 256, TN = 64 * BJ, P = IK;  // rows unpadded, chunks swizzled
  constexpr int CPR = IK / 16;                    // 16-byte chunks per row
  constexpr int SW = CPR == 4 ? 2 : 1;            // log2(16 / CPR)
  constexpr int NV = TM * IK / 16 / 256;   // 16-byte vectors of A per thread
  constexpr int NVB = TN * IK / 16 / 256;  // and of B
  extern __shared__ __attribute__((aligned(16))) int8_t s_i8[];
  int8_t* As = s_i8;                      // [2][TM][P]
  int8_t* Bs = s_i8 + 2 * TM * P;         // [2][TN][P]
  const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
  const uint32_t tiles_m = (M + TM - 1) / TM, tiles_n = (N + TN - 1) / TN;
  uint32_t tm, tn;
  tile_of(blockIdx.x, gridDim.x, tiles_m, tiles_n, &tm, &tn);
  const uint32_t m0 = tm * TM, n0 = tn * TN;
  const uint32_t wm = (w >> 1) * 128, wn = (w & 1) * 32 * BJ;
  // Operand rows are 16-byte aligned and K is a multiple of 16 (the launcher
  // checks): every fetch is one unconditional 16-byte load from a clamped
  // address, zeroed when staged if it lies outside the matrix, so no branch
  // separates a load from its use and the loads of a K-tile stay in flight
  // together.
  static_assert(VEC, "the large-tile kernel needs 16-byte rows");
  struct Regs {
    v4i a[NV], b[NVB];
    uint32_t okA, okB;
  };
  auto fetch = [&](Regs& R, uint32_t k0) {
    R.okA = R.okB = 0;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const uint32_t e = tid + 256u * q;
      const uint32_t r = e / (IK / 16), gk = k0 + (e % (IK / 16)) * 16;
      const uint32_t kc = gk < K ? gk : K - 16;
      const uint32_t ra = m0 + r < M ? m0 + r : M - 1;
      R.a[q] = gld((const v4i*)(A + (uint64_t)ra * lda + kc));
      R.okA |= (uint32_t)(m0 + r < M && gk < K) << q;
    }
#pragma unroll
    for (int q = 0; q < NVB; ++q) {
      const uint32_t e = tid + 256u * q;
      const uint32_t r = e / (IK / 16), gk = k0 + (e % (IK / 16)) * 16;
      const uint32_t kc = gk < K ? gk : K - 16;
      const uint32_t rb = n0 + r < N ? n0 + r : N - 1;
      R.b[q] = gld((const v4i*)(Bt + (uint64_t)rb * ldbt + kc));
      R.okB |= (uint32_t)(n0 + r < N && gk < K) << q;
    }
  };
  // LDS layout: chunk c of row r is stored at chunk c ^ ((r >> SW) mod CPR)
  // of that row, so that the 16 lanes of one LDS access (a column of 16
  // rows when the MFMA operands are read, CPR chunks of 16 / CPR rows when a
  // K-tile is written) touch 16 distinct 16-byte bank groups.
  auto swz = [](uint32_t r, uint32_t c) -> uint32_t {
    return (((c >> 4) ^ (r >> SW)) & (CPR - 1)) << 4;
  };
  auto stage = [&](const Regs& R, int buf) {
    const v4i zero = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const uint32_t e = tid + 256u * q;
      const uint32_t r = e / (IK / 16), c = (e % (IK / 16)) * 16;
      *(v4i*)&As[(buf * TM + r) * P + swz(r, c)] = ((R.okA >> q) & 1u) ? R.a[q] : zero;
    }
#pragma unroll
    for (int q = 0; q < NVB; ++q) {
      const uint32_t e = tid + 256u * q;
      const uint32_t r = e / (IK / 16), c = (e % (IK / 16)) * 16;
      *(v4i*)&Bs[(buf * TN + r) * P + swz(r, c)] = ((R.okB >> q) & 1u) ? R.b[q] : zero;
    }
  };
  v16i acc[4][BJ];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;
  auto compute = [&](int buf) {
#pragma unroll
    for (int s = 0; s < IK / 32; ++s) {
      const uint32_t kc = 32 * s + 16 * (lane / 32);
      v4i a[4], b[BJ];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t r = wm + 32 * i + lane % 32;
        a[i] = *(const v4i*)&As[(buf * TM + r) * P + swz(r, kc)];
      }
#pragma unroll
      for (int j = 0; j < BJ; ++j) {
        const uint32_t r = wn + 32 * j + lane % 32;
        b[j] = *(const v4i*)&Bs[(buf * TN + r) * P + swz(r, kc)];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  };
  uint32_t steps = 0;
  auto fold = [&]() {
    if (FOLDS && ++steps == fold_steps) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[i][j][r] = centred_mod(acc[i][j][r], F);
      steps = 0;
    }
  };
  // One register set, fetched one K-tile ahead.
  const uint32_t tiles_k = (K + IK - 1) / IK;
  Regs R;
  if (tiles_k > 0) {
    fetch(R, 0);
    stage(R, 0);
    __syncthreads();
    if (tiles_k > 1) fetch(R, IK);
  }
  for (uint32_t t = 0; t < tiles_k; ++t) {
    const int buf = t & 1;
    compute(buf);
    if (t + 1 < tiles_k) stage(R, buf ^ 1);
    __syncthreads();  // the other buffer is complete; nobody reads this one any more
    if (t + 2 < tiles_k) fetch(R, (t + 2) * IK);
    fold();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const uint32_t gm = m0 + wm + 32 * i + 8 * (r / 4) + 4 * (lane / 32) + r % 4;
        const uint32_t gn = n0 + wn + 32 * j + lane % 32;
        if (gm < M && gn < N) C[(uint64_t)gm * ldc + gn] = (int8_t)centred_mod(acc[i][j][r], F);
      }
}

// s_waitcnt for "at most N vector-memory operations outstanding", leaving the
// other counters alone (gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt
// 6:4, lgkmcnt 11:8).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Workgroup barrier without a memory fence: a fence would wait for every
// outstanding load, including the K-tiles still being prefetched.  Callers
// wait for the loads they need themselves; the empty asm statements keep the
// compiler from moving LDS accesses across the barrier.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// int8 kernel fed by direct global-to-LDS loads (global_load_lds_dwordx4:
// each lane's 16 bytes land at LDS base + 16 x lane, no registers involved),
// so K-tiles can be prefetched NS-1 tiles ahead through NS LDS stages.  C
// tile 256 x (64 BJ); each wavefront a 128 x (32 BJ) sub-tile as 4 x BJ
// blocks of 32 x 32; K-tiles of 64.  Rows of a stage are 64 bytes, chunk c
// of row r stored at chunk c ^ ((r >> 2) mod 4) (the lane that fills a
// chunk position fetches the chunk that belongs there), so LDS reads and
// writes touch 16 distinct 16-byte bank groups.  Needs K a multiple of 64
// (no zero fill is possible on this path) and 16-byte rows; rows of A and
// B^T past M and N are read from the last row and only reach outputs that
// are not stored.
template <int BJ, int NS, int NW, bool SPLIT = false, int IKT = 64>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(BJ == 4 ? 1 : 2, BJ == 4 ? 1 : 2)))
void gemm_i8_dma_kernel(const FieldK F, uint32_t M, uint32_t N, uint32_t K, const int8_t* A,
                        uint64_t lda, const int8_t* Bt, uint64_t ldbt, int8_t* C, uint64_t ldc,
                        uint32_t* Cu = nullptr, uint64_t wgt = 0,
                        uint32_t fresh = 0) {
  // NW = 4 wavefronts as 2 x 2, or 8 as 2 x 4 (the workgroup tile twice as
  // wide); each wavefront a 128 x (32 BJ) sub-tile.
  // IKT = 64: rows of 64 bytes, four 16-byte chunks; IKT = 128: rows of
  // 128 bytes (whole cache lines per row in every load), eight chunks.
  constexpr int IK = IKT, TM = 256, TN = 64 * BJ * (NW / 4), WC = NW / 2;
  constexpr int CH = IK / 16, RPI = 64 / CH;  // chunks per row, rows per load
  constexpr int SA = TM * IK, SB = TN * IK, SS = SA + SB;    // bytes per stage
  constexpr int NIA = SA / 1024 / NW, NIB = SB / 1024 / NW;  // DMA instructions per wave
  constexpr int PER = NIA + NIB;
  extern __shared__ __attribute__((aligned(16))) int8_t s_dma[];
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const uint32_t w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t tiles_m = (M + TM - 1) / TM, tiles_n = (N + TN - 1) / TN;
  uint32_t tm, tn;
  tile_of(blockIdx.x, gridDim.x, tiles_m, tiles_n, &tm, &tn);
  const uint32_t m0 = tm * TM, n0 = tn * TN;
  const uint32_t wm = (w / WC) * 128, wn = (w % WC) * 32 * BJ;
  // this lane's part of every DMA instruction: row lane/CH of an RPI-row
  // band, chunk position lane%CH; chunk c of row r is stored at position
  // c ^ f(r), f(r) = (r/4) mod 4 for four chunks, (r/2) mod 8 for eight, so
  // that any 16 lanes reading one chunk of 16 consecutive rows hit 16
  // distinct 16-byte bank groups
  const uint32_t lr = lane / CH, lp = lane % CH;
  auto fsw = [](uint32_t r) -> uint32_t { return CH == 4 ? ((r >> 2) & 3u) : ((r >> 1) & 7u); };
  const uint8_t* gA[NIA];
  const uint8_t* gB[NIB];
#pragma unroll
  for (int j = 0; j < NIA; ++j) {
    const uint32_t r = RPI * (NIA * w + j) + lr;
    const uint32_t row = m0 + r < M ? m0 + r : M - 1;
    gA[j] = (const uint8_t*)A + (uint64_t)row * lda + 16 * (lp ^ fsw(r));
  }
#pragma unroll
  for (int j = 0; j < NIB; ++j) {
    const uint32_t r = RPI * (NIB * w + j) + lr;
    const uint32_t row = n0 + r < N ? n0 + r : N - 1;
    gB[j] = (const uint8_t*)Bt + (uint64_t)row * ldbt + 16 * (lp ^ fsw(r));
  }
  auto issue = [&](uint32_t t, uint32_t stage) {
    int8_t* base = s_dma + stage * SS;
    const uint64_t k0 = (uint64_t)t * IK;
#pragma unroll
    for (int j = 0; j < NIA; ++j)
      __builtin_amdgcn_global_load_lds(
          (const __attribute__((address_space(1))) void*)(gA[j] + k0),
          (__attribute__((address_space(3))) void*)(base + 1024 * (NIA * w + j)), 16, 0, 0);
#pragma unroll
    for (int j = 0; j < NIB; ++j)
      __builtin_amdgcn_global_load_lds(
          (const __attribute__((address_space(1))) void*)(gB[j] + k0),
          (__attribute__((address_space(3))) void*)(base + SA + 1024 * (NIB * w + j)), 16, 0, 0);
  };
  auto swz = [&](uint32_t r, uint32_t c) -> uint32_t { return ((c >> 4) ^ fsw(r)) << 4; };
  v16i acc[4][BJ];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;
  const uint32_t tiles_k = K / IK;
#pragma unroll
  for (int st = 0; st < NS - 1; ++st)
    if ((uint32_t)st < tiles_k) issue(st, st);
  for (uint32_t t = 0; t < tiles_k; ++t) {
    // this wave's loads of tile t are done (later tiles may still be in
    // flight), then everybody's are, and everybody has finished tile t-1
    if (t + NS - 2 < tiles_k) wait_vmcnt<(NS - 2) * PER>(); else wait_vmcnt<0>();
    lds_barrier();
    if (t + NS - 1 < tiles_k) issue(t + NS - 1, (t + NS - 1) % NS);
    const int8_t* As = s_dma + (t % NS) * SS;
    const int8_t* Bs = As + SA;
#pragma unroll
    for (int s = 0; s < IK / 32; ++s) {
      const uint32_t kc = 32 * s + 16 * (lane / 32);
      v4i a[4], b[BJ];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t r = wm + 32 * i + lane % 32;
        a[i] = *(const v4i*)&As[r * IK + swz(r, kc)];
      }
#pragma unroll
      for (int j = 0; j < BJ; ++j) {
        const uint32_t r = wn + 32 * j + lane % 32;
        b[j] = *(const v4i*)&Bs[r * IK + swz(r, kc)];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  if constexpr (SPLIT) {
    const uint64_t pm = (0x80000000ull + F.p - 1) / F.p * F.p;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      split_rows<BJ>(Cu, ldc, wgt, acc[i], m0 + wm + 32 * i, n0 + wn, lane, M, N, pm, F,
                     fresh);
    return;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const uint32_t gm = m0 + wm + 32 * i + 8 * (r / 4) + 4 * (lane / 32) + r % 4;
        const uint32_t gn = n0 + wn + 32 * j + lane % 32;
        if (gm < M && gn < N) i8_store(C, (uint64_t)gm * ldc + gn, acc[i][j][r], F);
      }
}

// Bt = B^T for int8 matrices, 64 x 64 tiles through LDS.  Each thread
// moves 16 bytes each way: one 16-byte load of a row segment of B (when the
// segment is inside B and aligned), sixteen LDS byte reads down a column, one
// 16-byte store of a row segment of Bt; bytewise at the edges.
__global__ __launch_bounds__(256) void transpose_i8_kernel(const int8_t* B, uint64_t ldb, uint32_t K,
                                                           uint32_t N, int8_t* Bt, uint64_t ldbt,
                                                           uint32_t Kout) {
  __shared__ int8_t t[64][65];
  const uint32_t k0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const uint32_t r = threadIdx.x / 4, c = (threadIdx.x % 4) * 16;  // 64 rows x 4 segments
  const bool vin = ((ldb | ldbt | (uintptr_t)B | (uintptr_t)Bt) & 15u) == 0;
  if (vin && k0 + r < K && n0 + c + 16 <= N) {
    const v4i v = gld((const v4i*)(B + (uint64_t)(k0 + r) * ldb + n0 + c));
    int8_t b[16];
    __builtin_memcpy(b, &v, 16);
#pragma unroll
    for (int i = 0; i < 16; ++i) t[r][c + i] = b[i];
  } else {
#pragma unroll
    for (int i = 0; i < 16; ++i)
      t[r][c + i] = (k0 + r < K && n0 + c + i < N) ? B[(uint64_t)(k0 + r) * ldb + n0 + c + i] : (int8_t)0;
  }
  __syncthreads();
  // row r of this Bt tile is column r of the B tile: k = c .. c+15
  int8_t b[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) b[i] = t[c + i][r];
  if (n0 + r >= N) return;
  // columns K .. Kout-1 of Bt (zero in the tile) are the zero padding
  if (vin && k0 + c + 16 <= Kout) {
    v4i v;
    __builtin_memcpy(&v, b, 16);
    *(v4i*)(Bt + (uint64_t)(n0 + r) * ldbt + k0 + c) = v;
  } else {
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (k0 + c + i < Kout) Bt[(uint64_t)(n0 + r) * ldbt + k0 + c + i] = b[i];
  }
}

// dst = src (rows x cols, row stride ld) with each row padded by zeros to
// ldd elements: one workgroup per row at a time, coalesced along the row.
template <typename T>
__global__ __launch_bounds__(256) void pad_copy_kernel(const T* src, uint64_t ld, uint32_t rows,
                                                       uint32_t cols, T* dst, uint32_t ldd) {
  for (uint32_t row = blockIdx.x; row < rows; row += gridDim.x)
    for (uint32_t c = threadIdx.x; c < ldd; c += 256)
      dst[(uint64_t)row * ldd + c] = c < cols ? src[(uint64_t)row * ld + c] : (T)0;
}

template <typename T>
hipError_t pad_copy(const void* src, size_t ld, size_t rows, size_t cols, void* dst, size_t ldd,
                    hipStream_t s) {
  hipLaunchKernelGGL(pad_copy_kernel<T>, dim3((unsigned)std::min<size_t>(rows, 65536)), dim3(256),
                     0, s, (const T*)src, (uint64_t)ld, (uint32_t)rows, (uint32_t)cols, (T*)dst,
                     (uint32_t)ldd);
  return hipGetLastError();
}

// Ap = A with rows padded by zeros from K to Kp (a multiple of 64), row
// stride Kp: one 16-byte segment of Ap per thread.
__global__ __launch_bounds__(256) void pad_rows_i8_kernel(const int8_t* A, uint64_t lda, uint32_t M,
                                                          uint32_t K, int8_t* Ap, uint32_t Kp) {
  const uint64_t segs = (uint64_t)M * (Kp / 16);
  for (uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x; e < segs;
       e += (uint64_t)gridDim.x * 256) {
    const uint64_t row = e / (Kp / 16);
    const uint32_t k = (uint32_t)(e % (Kp / 16)) * 16;
    const int8_t* src = A + row * lda + k;
    v4i v = {0, 0, 0, 0};
    if (k + 16 <= K && ((uintptr_t)src & 15u) == 0) {
      v = gld((const v4i*)src);
    } else {
      int8_t t[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) t[i] = k + i < K ? src[i] : (int8_t)0;
      __builtin_memcpy(&v, t, 16);
    }
    *(v4i*)(Ap + row * Kp + k) = v;
  }
}

// Scratch for the transposed B, one buffer per (device, stream), grown on
// demand (outside graph capture).
std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, std::pair<void*, size_t>> g_scratch;
std::set<void*> g_scratch_captured;

fdot_status_t scratch_for(hipStream_t s, size_t bytes, void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return FDOT_E_DEVICE;
  std::lock_guard<std::mutex> g(g_mu);
  auto& e = g_scratch[std::make_pair(dev, s)];
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const bool capturing =
      hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
  if (e.second >= bytes) {
    if (capturing) g_scratch_captured.insert(e.first);
    *out = e.first;
    return FDOT_OK;
  }
  if (capturing) return FDOT_E_BUSY;  // growing allocates
  // Stream-ordered allocation and release: the old buffer is freed after the
  // work already queued on s, and the host never waits for the device.
  // Growth is geometric, so a stream of rising sizes reallocates rarely.
  bytes = std::max(bytes, e.second + e.second / 2);
  void* p = nullptr;
  if (fd_alloc_async(&p, bytes, s) != hipSuccess) return FDOT_E_NOMEM;
  // a buffer that a captured graph holds stays allocated until the process ends
  if (e.first && !g_scratch_captured.count(e.first)) (void)hipFreeAsync(e.first, s);
  e = std::make_pair(p, bytes);
  *out = p;
  return FDOT_OK;
}

}  // namespace

fdot_status_t fd_scratch_get(hipStream_t s, size_t bytes, void** out) {
  return scratch_for(s, bytes, out);
}

void fd_scratch_release(hipStream_t s) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  std::lock_guard<std::mutex> g(g_mu);
  auto it = g_scratch.find(std::make_pair(dev, s));
  if (it == g_scratch.end()) return;
  if (it->second.first && !g_scratch_captured.count(it->second.first))
    (void)hipFreeAsync(it->second.first, s);
  g_scratch.erase(it);
}

namespace {

// Largest lambda with carry + lambda*h^2 <= limit (h = largest |term|).
uint64_t lambda_carried(uint64_t limit, uint64_t h, uint64_t carry) {
  if (h == 0) return ~0ull;
  const unsigned __int128 hh = (unsigned __int128)h * h;
  if (limit < carry) return 0;
  const unsigned __int128 l = (limit - carry) / hh;
  return l > 0xFFFFFFFFull ? 0xFFFFFFFFull : (uint64_t)l;
}

// ------------------------------------------------- large primes on int8 cores
// A residue below p < 2^32 is centred (|c| <= (p-1)/2) and written with D <= 4
// balanced base-256 digits in [-128, 127]: c = d0 + 256 d1 + 2^16 d2 + 2^24 d3,
// four of which cover |c| <= 2139062143.  Then A B = sum over digit pairs
// (i, j) of 256^(i+j) A_i B_j, D^2 exact int8 products with int32
// accumulation (|d d'| <= 2^14, so up to 131071 terms need no fold), each
// reduced mod p and added with its weight 256^(i+j) mod p (times B^-1 for
// Montgomery residues, whose products carry B^2) -- the operand-splitting
// counterpart of the delayed reduction of Sec. 3.1 on matrix cores.
constexpr uint64_t kSplitMaxHalf = 2139062143ull;  // 127 (1 + 2^8 + 2^16 + 2^24)

// Residue of a stored value: uint32 residues and integral doubles as they
// are, discrete-log codes (uint16) through the field's table of powers.
template <typename E>
__device__ __forceinline__ uint32_t stored_residue(E v, const FieldK& F) {
  if constexpr (std::is_same<E, uint16_t>::value) return F.zval[v];
  else return (uint32_t)v;
}

// Balanced base-256 digits needed for centred residues |c| <= h: D digits
// in [-128, 127] reach 127 (256^D - 1) / 255.
int split_digits(uint64_t h) {
  if (h <= 127ull) return 1;
  if (h <= 32639ull) return 2;
  if (h <= 8355711ull) return 3;
  return 4;
}
constexpr uint32_t kSplitMaxK = 131071;            // (2^31 - 1) / 2^14

__device__ __forceinline__ void balanced_digits(uint32_t v, const FieldK& F, int8_t d[4]) {
  int64_t c = v > (uint32_t)F.half ? (int64_t)v - (int64_t)F.p : (int64_t)v;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int64_t t = c & 255;
    if (t >= 128) t -= 256;
    d[i] = (int8_t)t;
    c = (c - t) / 256;
  }
}

// A (M x K residues, row stride lda; uint32 or integral doubles) to its nd
// digits: row r of the result is digit 0 of row r of A, then digit 1, ...,
// each ldk long with zeros in columns K .. ldk-1.
template <typename E>
__global__ __launch_bounds__(256) void digits_rows_kernel(const E* A, uint64_t lda,
                                                          uint32_t M, uint32_t K, uint32_t ldk,
                                                          int8_t* D, int nd, const FieldK F) {
  const uint64_t total = (uint64_t)M * (ldk / 4);
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t row = e / (ldk / 4);
    const uint32_t k = (uint32_t)(e % (ldk / 4)) * 4;
    int8_t d[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (k + q < K) {
        balanced_digits(stored_residue(A[row * lda + k + q], F), F, d[q]);
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) d[q][i] = 0;
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (i >= nd) break;  // the digits above nd are zero for |c| <= h
      const uint32_t packed = (uint32_t)(uint8_t)d[0][i] | (uint32_t)(uint8_t)d[1][i] << 8 |
                              (uint32_t)(uint8_t)d[2][i] << 16 | (uint32_t)(uint8_t)d[3][i] << 24;
      *(uint32_t*)(D + row * (nd * (uint64_t)ldk) + i * (uint64_t)ldk + k) = packed;
    }
  }
}

// B (K x N residues, row stride ldb) to the digits of B^T: row n of the
// result is digit nd-1 of column n of B, then digit nd-2, ..., digit 0, each
// ldk long (zeros in columns K .. ldk-1); 64 x 64 tiles through LDS.  With
// A's digits in rising and B's in falling order, the pairs (i, e - i) of one
// weight 256^e sit side by side along k in both.
template <typename E>
__global__ __launch_bounds__(256) void digits_cols_kernel(const E* B, uint64_t ldb,
                                                          uint32_t K, uint32_t N, uint32_t ldk,
                                                          int8_t* D, int nd, const FieldK F) {
  __shared__ uint32_t t[64][65];
  const uint32_t k0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  for (uint32_t e = threadIdx.x; e < 64 * 64; e += 256) {
    const uint32_t r = e / 64, c = e % 64;  // r: k, c: n
    t[r][c] = (k0 + r < K && n0 + c < N) ? stored_residue(B[(uint64_t)(k0 + r) * ldb + n0 + c], F) : 0u;
  }
  __syncthreads();
  const uint32_t r = threadIdx.x / 4, c = (threadIdx.x % 4) * 16;  // r: n, c: first k
  if (n0 + r >= N || k0 + c >= ldk) return;
  int8_t d[16][4];
#pragma unroll
  for (int q = 0; q < 16; ++q) balanced_digits(t[c + q][r], F, d[q]);  // zero residue: zero digits
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (i >= nd) break;
    int8_t row[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) row[q] = d[q][i];
    v4i v;
    __builtin_memcpy(&v, row, 16);
    *(v4i*)(D + (uint64_t)(n0 + r) * (nd * (uint64_t)ldk) + (uint64_t)(nd - 1 - i) * ldk + k0 + c) = v;
  }
}

// C (M x N discrete-log codes, row stride ldc) = codes of Cu (dense residues).
__global__ __launch_bounds__(256) void residues_to_codes_kernel(const FieldK F, const uint32_t* Cu,
                                                                uint32_t M, uint32_t N,
                                                                uint16_t* C, uint64_t ldc) {
  const uint64_t total = (uint64_t)M * N;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * blockDim.x)
    C[(e / N) * ldc + e % N] = F.zidx[Cu[e]];
}

// C (M x N integral doubles, row stride ldc) = Cu (M x N residues, dense).
__global__ __launch_bounds__(256) void residues_to_f64_kernel(const uint32_t* Cu, uint32_t M,
                                                              uint32_t N, double* C, uint64_t ldc) {
  const uint64_t total = (uint64_t)M * N;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * blockDim.x)
    C[(e / N) * ldc + e % N] = (double)Cu[e];
}

fdot_status_t gemm_split(const fdot_field_s* f, size_t M, size_t N, size_t K, const void* A,
                         size_t lda, const void* B, size_t ldb, void* C, size_t ldc,
                         hipStream_t s) {
  const fdot_field_info_t& I = f->info;
  const bool f64 = I.rep == FDOT_REP_FP64;  // doubles in and out; residues summed in scratch
  const bool zech = I.rep == FDOT_REP_ZECH_U16;  // codes in and out; residues summed in scratch
  // 256 x 256 direct-to-LDS tiles (K-tiles of 128, whole 128-byte rows per
  // load) once they fill half the chip, else 128 x 128
  const int64_t small = fd_tune("gemm.split.small", -1);
  const bool big = M >= 256 && N >= 256 &&
                   (small == 0 || (small < 0 && ((M + 255) / 256) * ((N + 255) / 256) >= 128));
  const uint32_t ldk = (uint32_t)(big ? (K + 127) / 128 * 128 : (K + 63) / 64 * 64);
  const int nd = split_digits((I.p - 1) / 2);
  const size_t planes = (size_t)nd * ((size_t)M + N) * ldk + 256;
  const size_t bytes = planes + ((f64 || zech) ? (size_t)4 * M * N : 0);
  void* scr = nullptr;
  fdot_status_t st = scratch_for(s, bytes, &scr);
  if (st != FDOT_OK) return st;
  int8_t* Ad = (int8_t*)scr;
  int8_t* Bd = Ad + (size_t)nd * M * ldk;
  void* Cf = C;
  const size_t ldcf = ldc;
  if (f64 || zech) {
    C = (char*)scr + planes;
    ldc = N;
  }
  const uint64_t cells = (uint64_t)M * N;
  const unsigned zg = (unsigned)std::min<uint64_t>((cells + 255) / 256, 65536);
  // C is not cleared: the first launch (weight 256^0) writes every entry
  const uint64_t ag = std::min<uint64_t>(((uint64_t)M * (ldk / 4) + 255) / 256, 65536);
  const dim3 cg((unsigned)((N + 63) / 64), (unsigned)(ldk / 64));
  if (f64) {
    hipLaunchKernelGGL(digits_rows_kernel<double>, dim3((unsigned)ag), dim3(256), 0, s,
                       (const double*)A, (uint64_t)lda, (uint32_t)M, (uint32_t)K, ldk, Ad, nd, f->k);
    hipLaunchKernelGGL(digits_cols_kernel<double>, cg, dim3(256), 0, s, (const double*)B,
                       (uint64_t)ldb, (uint32_t)K, (uint32_t)N, ldk, Bd, nd, f->k);
  } else if (zech) {
    hipLaunchKernelGGL(digits_rows_kernel<uint16_t>, dim3((unsigned)ag), dim3(256), 0, s,
                       (const uint16_t*)A, (uint64_t)lda, (uint32_t)M, (uint32_t)K, ldk, Ad, nd, f->k);
    hipLaunchKernelGGL(digits_cols_kernel<uint16_t>, cg, dim3(256), 0, s, (const uint16_t*)B,
                       (uint64_t)ldb, (uint32_t)K, (uint32_t)N, ldk, Bd, nd, f->k);
  } else {
    hipLaunchKernelGGL(digits_rows_kernel<uint32_t>, dim3((unsigned)ag), dim3(256), 0, s,
                       (const uint32_t*)A, (uint64_t)lda, (uint32_t)M, (uint32_t)K, ldk, Ad, nd, f->k);
    hipLaunchKernelGGL(digits_cols_kernel<uint32_t>, cg, dim3(256), 0, s, (const uint32_t*)B,
                       (uint64_t)ldb, (uint32_t)K, (uint32_t)N, ldk, Bd, nd, f->k);
  }
  if (hipGetLastError() != hipSuccess) return FDOT_E_DEVICE;
  const unsigned __int128 p = I.p;
  uint64_t base = I.rep == FDOT_REP_MONT_U32 ? I.binv_mod_p : 1;  // Montgomery: one factor B^-1
  const size_t lds = (size_t)2 * (256 + 256) * 128;
  if (big) {
    static bool attr_set = false;
    if (!attr_set) {
      (void)hipFuncSetAttribute((const void*)gemm_i8_dma_kernel<2, 2, 8, true, 128>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      attr_set = true;
    }
  }
  // One product per weight: the pairs (i, e - i) of weight 256^e are adjacent
  // along k in both digit layouts, so they form one int8 product of length
  // (pairs) * ldk, in as few launches as the int32 bound allows (at most
  // 131071 terms of |d d'| <= 2^14 each): 2D - 1 epilogues instead of D^2.
  const uint64_t ld_all = (uint64_t)nd * ldk;
  const int per_launch = (int)std::max<uint64_t>(1, (uint64_t)kSplitMaxK / ldk);
  for (int e = 0; e <= 2 * nd - 2; ++e) {
    // 256^e (B^-1) mod p with its precomputed quotient for the epilogue
    const uint64_t w = base | ((uint64_t)(((unsigned __int128)base << 32) / p) << 32);
    const int i_lo = std::max(0, e - nd + 1), i_hi = std::min(e, nd - 1);
    for (int c = i_lo; c <= i_hi; c += per_launch) {
      const int cnt = std::min(per_launch, i_hi - c + 1);
      const int8_t* Ai = Ad + (size_t)c * ldk;                    // digits c .. c+cnt-1 of A
      const int8_t* Bj = Bd + (size_t)(nd - 1 - (e - c)) * ldk;   // digits e-c .. down of B
      const uint32_t Kx = (uint32_t)cnt * ldk;
      const uint32_t fresh = e == 0 && c == i_lo ? 1u : 0u;  // the first launch
      if (big) {
        const uint64_t tiles = ((M + 255) / 256) * ((N + 255) / 256);
        hipLaunchKernelGGL((gemm_i8_dma_kernel<2, 2, 8, true, 128>), dim3((unsigned)tiles), dim3(512),
                           lds, s, f->k, (uint32_t)M, (uint32_t)N, Kx, Ai, ld_all, Bj, ld_all,
                           (int8_t*)nullptr, (uint64_t)ldc, (uint32_t*)C, w, fresh);
      } else {
        const uint64_t tiles = ((M + 127) / 128) * ((N + 127) / 128);
        hipLaunchKernelGGL((gemm_i8_kernel<2, 2, 64, true, true>), dim3((unsigned)tiles),
                           dim3(256), 0, s, f->k, (uint32_t)M, (uint32_t)N, Kx, Ai, ld_all, Bj,
                           ld_all, (int8_t*)nullptr, (uint64_t)ldc, 0xFFFFFFFFu, (uint32_t*)C, w,
                           fresh);
      }
      if (hipGetLastError() != hipSuccess) return FDOT_E_DEVICE;
    }
    base = (uint64_t)(((unsigned __int128)base * 256u) % p);
  }
  if (f64) {
    hipLaunchKernelGGL(residues_to_f64_kernel, dim3(zg), dim3(256), 0, s, (const uint32_t*)C,
                       (uint32_t)M, (uint32_t)N, (double*)Cf, (uint64_t)ldcf);
    if (hipGetLastError() != hipSuccess) return FDOT_E_DEVICE;
  }
  if (zech) {
    hipLaunchKernelGGL(residues_to_codes_kernel, dim3(zg), dim3(256), 0, s, f->k,
                       (const uint32_t*)C, (uint32_t)M, (uint32_t)N, (uint16_t*)Cf, (uint64_t)ldcf);
    if (hipGetLastError() != hipSuccess) return FDOT_E_DEVICE;
  }
  return FDOT_OK;
}

}  // namespace

fdot_status_t fd_launch_gemm_mfma(const fdot_field_s* f, size_t M, size_t N, size_t K,
                                  const void* A, size_t lda, const void* B, size_t ldb, void* C,
                                  size_t ldc, hipStream_t s, bool* handled) {
  *handled = false;
  const fdot_field_info_t& I = f->info;
  if (M > 0x7FFFFFFFull || N > 0x7FFFFFFFull || K > 0x7FFFFFFFull) return FDOT_E_UNSUPPORTED;
  const uint64_t p = I.p, h = (p - 1) / 2;
  if (I.rep == FDOT_REP_CENTRED_I8) {
    // |centred residue| <= h; carried residue after a fold also <= h.
    const uint64_t lam = lambda_carried(0x7FFFFFFFull, h, h);
    if (lam < 128 || fd_tune("gemm.i8.disable", 0)) return FDOT_E_UNSUPPORTED;
    *handled = true;
    int64_t shape = fd_tune("gemm.i8.tile", M >= 1024 && N >= 1024 ? 8 : 2);
    // The direct-to-LDS tilings need K a multiple of 64 and 16-byte rows of A;
    // other shapes get zero-padded copies (zero terms leave every sum as it
    // is, so the fold bound still applies to the true K).
    const uint64_t kmul = shape >= 8 ? 128 : 64;  // K-tile of the direct-to-LDS kernel
    const uint64_t Kp = (K + kmul - 1) / kmul * kmul;
    const bool dma = (shape >= 5 && shape <= 9) && K > 0 &&
                     (uint64_t)K <= (lam / 128) * 128 && M >= 256 && N >= 256 &&
                     Kp <= 0xFFFFFFFFull && fd_tune("gemm.i8.pad", 1) != 0;
    const bool pad_a = dma && (K % kmul != 0 || lda % 16 != 0 || ((uintptr_t)A) % 16 != 0);
    const uint64_t ldbt = dma ? Kp : K;
    void* bt = nullptr;
    fdot_status_t st =
        scratch_for(s, (size_t)N * ldbt + (pad_a ? (size_t)M * Kp : 0) + 16, &bt);
    if (st != FDOT_OK) return st;
    if (K > 0) {
      hipLaunchKernelGGL(transpose_i8_kernel, dim3((unsigned)((N + 63) / 64), (unsigned)((ldbt + 63) / 64)),
                         dim3(256), 0, s, (const int8_t*)B, (uint64_t)ldb, (uint32_t)K, (uint32_t)N,
                         (int8_t*)bt, ldbt, (uint32_t)ldbt);
      if (hipGetLastError() != hipSuccess) return FDOT_E_DEVICE;
    }
    if (pad_a) {
      int8_t* ap = (int8_t*)bt + (size_t)N * ldbt;
      const uint64_t segs = (uint64_t)M * (Kp / 16);
      hipLaunchKernelGGL(pad_rows_i8_kernel, dim3((unsigned)std::min<uint64_t>((segs + 255) / 256, 65536)),
                         dim3(256), 0, s, (const int8_t*)A, (uint64_t)lda, (uint32_t)M, (uint32_t)K,
                         ap, (uint32_t)Kp);
      if (hipGetLastError() != hipSuccess) return FDOT_E_DEVICE;
      A = ap;
      lda = Kp;
    }
    if (dma) K = Kp;
    // Kernel and workgroup tile (tune key gemm.i8.tile): large matrices use 8 by
    // default.  Direct-to-LDS loads: 8 = 256 x 256 with eight wavefronts and
    // two stages of K-tiles of 128, 9 = the same with four wavefronts of
    // 128 x 128; K-tiles of 64: 7 = 256 x 256 with eight wavefronts and four
    // stages, 5 = 256 x 128 with three stages, 6 = 256 x 256 with four
    // wavefronts and four stages.  Register-staged,
    // double-buffered: 4 = 256 x 128, 3 = 256 x 256.  Register-staged with
    // in-loop folds (any K): 2 = 128 x 128 (small matrices), 1 = 256 x 128,
    // 0 = 256 x 256.  A tiling whose conditions fail falls back to the next
    // one that applies.
    // the large tile keeps its accumulators unfolded (only when K fits one fold
    // block) and needs 16-byte rows
    if ((shape >= 3 && shape <= 9) &&
        ((uint64_t)K > (lam / 128) * 128 || K % 16 != 0 || lda % 16 != 0 ||
                       ((uintptr_t)A) % 16 != 0 || M < 256 || N < 256))
      shape = 2;
    const int64_t kt = fd_tune("gemm.i8.ktile", 128) == 64 ? 64 : 128;
    const uint32_t fold_steps = (uint32_t)(lam / (uint64_t)kt);
    const bool vec = (lda % 16 == 0) && (((uintptr_t)A) % 16 == 0) && (K % 16 == 0);
    const uint32_t TM = shape == 2 ? 128 : 256, TN = (shape == 0 || shape == 3) ? 256 : 128;
    const uint64_t tiles = ((M + TM - 1) / TM) * ((N + TN - 1) / TN);
    if (tiles > 0x7FFFFFFFull) return FDOT_E_INVALID_ARG;
#define FD_I8_LAUNCH(BI, BJ, KT, V)                                                               \
  hipLaunchKernelGGL((gemm_i8_kernel<BI, BJ, KT, V>), dim3((unsigned)tiles), dim3(256), 0, s,     \
                     f->k, (uint32_t)M, (uint32_t)N, (uint32_t)K, (const int8_t*)A,                \
                     (uint64_t)lda, (const int8_t*)bt, (uint64_t)K, (int8_t*)C, (uint64_t)ldc,    \
                     fold_steps)
#define FD_I8_SHAPE(KT)                                                                            \
  if (shape == 2) { if (vec) FD_I8_LAUNCH(2, 2, KT, true); else FD_I8_LAUNCH(2, 2, KT, false); }  \
  else if (shape == 1) { if (vec) FD_I8_LAUNCH(4, 2, KT, true); else FD_I8_LAUNCH(4, 2, KT, false); } \
  else { if (vec) FD_I8_LAUNCH(4, 4, KT, true); else FD_I8_LAUNCH(4, 4, KT, false); }
    if ((shape >= 5 && shape <= 9) && K % kmul == 0) {
#define FD_I8_DMA(BJ, NS, NW, IKT)                                                                 \
  {                                                                                                \
    constexpr int DTN = 64 * BJ * (NW / 4);                                                        \
    const size_t lds = (size_t)NS * (256 + DTN) * IKT;                                             \
    static bool attr_set = false;                                                                  \
    if (!attr_set) {                                                                               \
      (void)hipFuncSetAttribute((const void*)gemm_i8_dma_kernel<BJ, NS, NW, false, IKT>,          \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);             \
      attr_set = true;                                                                             \
    }                                                                                              \
    const uint64_t dma_tiles = ((M + 255) / 256) * ((N + DTN - 1) / DTN);                          \
    hipLaunchKernelGGL((gemm_i8_dma_kernel<BJ, NS, NW, false, IKT>), dim3((unsigned)dma_tiles),    \
                       dim3(64 * NW), lds, s, f->k, (uint32_t)M, (uint32_t)N, (uint32_t)K,         \
                       (const int8_t*)A, (uint64_t)lda, (const int8_t*)bt, ldbt, (int8_t*)C,       \
                       (uint64_t)ldc);                                                             \
  }
      // 8: K-tiles of 128 (whole 128-byte rows per load), two stages
      if (shape == 5) FD_I8_DMA(2, 3, 4, 64) else if (shape == 6) FD_I8_DMA(4, 4, 4, 64)
      else if (shape == 8) FD_I8_DMA(2, 2, 8, 128) else if (shape == 9) FD_I8_DMA(4, 2, 4, 128)
      else FD_I8_DMA(2, 4, 8, 64)
#undef FD_I8_DMA
    } else if (shape >= 3 && shape <= 9) {
      // 3: 256 x 256 tile, one wavefront per SIMD; 4: 256 x 128, two
      const int64_t bkt = (shape == 4 || shape == 5 || shape >= 7) ? 64 : (fd_tune("gemm.i8.big.ktile", 128) == 64 ? 64 : 128);
      const uint32_t big_fold = (uint32_t)(lam / (uint64_t)bkt);
#define FD_I8_BIG(KT, BJ)                                                                          \
  {                                                                                                \
    const size_t lds = (size_t)2 * (256 + 64 * BJ) * KT;                                           \
    static bool attr_set = false;                                                                  \
    if (!attr_set) {                                                                               \
      (void)hipFuncSetAttribute((const void*)gemm_i8_big_kernel<KT, BJ, true, false>,            \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);             \
      attr_set = true;                                                                             \
    }                                                                                              \
    const uint64_t big_tiles = ((M + 255) / 256) * ((N + 64 * BJ - 1) / (64 * BJ));                \
    hipLaunchKernelGGL((gemm_i8_big_kernel<KT, BJ, true, false>), dim3((unsigned)big_tiles),       \
                       dim3(256), lds, s, f->k, (uint32_t)M, (uint32_t)N, (uint32_t)K,             \
                       (const int8_t*)A, (uint64_t)lda, (const int8_t*)bt, (uint64_t)K,            \
                       (int8_t*)C, (uint64_t)ldc, big_fold);                                       \
  }
      if (shape == 4 || shape == 5 || shape >= 7) FD_I8_BIG(64, 2) else if (bkt == 64) FD_I8_BIG(64, 4) else FD_I8_BIG(128, 4)
#undef FD_I8_BIG
    } else if (kt == 64) { FD_I8_SHAPE(64) } else { FD_I8_SHAPE(128) }
#undef FD_I8_SHAPE
#undef FD_I8_LAUNCH
    return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
  }
  if (I.rep == FDOT_REP_ZECH_U16) {
    // discrete logs: the digit products on the int8 matrix cores, from the
    // codes' residues, above a size (tune key gemm.split.zech_min_work); the
    // exact vector-ALU kernel below it
    const bool ok = f->degree == 1 && K >= 1 && K <= kSplitMaxK - 63 && M > 0 && N > 0 &&
                    fd_tune("gemm.split.disable", 0) == 0 &&
                    (double)M * (double)N * (double)K >=
                        (double)fd_tune("gemm.split.zech_min_work", 1ll << 24);
    if (!ok) return FDOT_E_UNSUPPORTED;
    *handled = true;
    return gemm_split(f, M, N, K, A, lda, B, ldb, C, ldc, s);
  }
  if (I.rep != FDOT_REP_FP64 && I.rep != FDOT_REP_ZPZ_U32 && I.rep != FDOT_REP_MONT_U32)
    return FDOT_E_UNSUPPORTED;
  if (fd_tune("gemm.f64.disable", 0)) return FDOT_E_UNSUPPORTED;
  // Exact double sums up to 2^53.  Residues as stored: terms <= (p-1)^2,
  // carried residue <= p-1.  Centred: terms <= h^2, carried |residue| <= h.
  const uint64_t lim = 1ull << 53;
  const uint64_t lam_plain = lambda_carried(lim, p - 1, p - 1);
  const uint64_t lam_centre = lambda_carried(lim, h, h);
  bool centre;
  uint64_t lam;
  if (lam_plain >= 64 || lam_plain >= lam_centre) {
    centre = false;
    lam = lam_plain;
  } else {
    centre = true;
    lam = lam_centre;
  }
  // Digit products on the int8 matrix cores: the only matrix-core path for
  // larger primes (lambda < 4), and faster than the FP64 matrix cores for
  // every prime once the product is large enough to amortise its D^2
  // launches (D = 2, 3 or 4 digits by the size of p; tune key
  // gemm.split.min_work, in M*N*K; gemm.split.disable keeps the FP64 path).
  const bool split_ok = h <= kSplitMaxHalf && K >= 1 && K <= kSplitMaxK - 63 && M > 0 && N > 0 &&
                        fd_tune("gemm.split.disable", 0) == 0;
  // Crossovers measured at square shapes (the autotuner's split sweep): two
  // digits (3 products per weight) and four digits (7, against FP64 products
  // folded every few terms) beat the FP64 cores from about 512^3, three
  // digits (5, against unfolded FP64 products) between 2048^3 and 3072^3.
  const int nd = split_digits(h);
  const int64_t min_work = nd == 3 ? (1ll << 34) : (1ll << 27);
  // measured crossover for this digit count (autotuner), else the default;
  // gemm.split.min_work overrides both
  char key[32];
  snprintf(key, sizeof key, "gemm.split.min_work.d%d", nd);
  const bool split_wins = (double)M * (double)N * (double)K >=
                          (double)fd_tune("gemm.split.min_work", fd_tune(key, min_work));
  if (split_ok && (lam < 4 || split_wins)) {
    *handled = true;
    return gemm_split(f, M, N, K, A, lda, B, ldb, C, ldc, s);
  }
  if (lam < 4) return FDOT_E_UNSUPPORTED;
  *handled = true;
  const uint64_t tiles = ((M + FM - 1) / FM) * ((N + FN - 1) / FN);
  if (tiles > 0x7FFFFFFFull) return FDOT_E_INVALID_ARG;
  const bool subfold = lam < FK;
  const uint32_t fold_sub = (uint32_t)(subfold ? lam / 4 : lam / FK);
  const dim3 grid((unsigned)tiles);
  // wavefronts per workgroup: 8 of 32 x 64 (two per SIMD, default), 16 of
  // 16 x 64 or 4 of 64 x 64
  const int64_t nw = fd_tune("gemm.f64.waves", 8);
#define FD_F64_LAUNCH_NW(E, CEN, V, SF, NW)                                                       \
  do {                                                                                             \
    static bool attr_set = false;                                                                  \
    if (!attr_set) {                                                                               \
      (void)hipFuncSetAttribute((const void*)gemm_f64_kernel<E, CEN, V, SF, NW>,                 \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kF64Lds);         \
      attr_set = true;                                                                             \
    }                                                                                              \
    hipLaunchKernelGGL((gemm_f64_kernel<E, CEN, V, SF, NW>), grid, dim3(64 * NW), kF64Lds, s, f->k,\
                       I.rep, (uint32_t)M, (uint32_t)N, (uint32_t)K, (const E*)A, (uint64_t)lda,  \
                       (const E*)B, (uint64_t)ldb, C, (uint64_t)ldc, fold_sub);                    \
  } while (0)
#define FD_F64_LAUNCH(E, CEN, V, SF)                                                              \
  do {                                                                                             \
    if (nw == 8) FD_F64_LAUNCH_NW(E, CEN, V, SF, 8);                                              \
    else if (nw == 16) FD_F64_LAUNCH_NW(E, CEN, V, SF, 16);                                        \
    else FD_F64_LAUNCH_NW(E, CEN, V, SF, 4);                                                       \
  } while (0)
#define FD_F64_PICK(E, CEN)                                                                        \
  if (vec) { if (subfold) FD_F64_LAUNCH(E, CEN, true, true); else FD_F64_LAUNCH(E, CEN, true, false); } \
  else { if (subfold) FD_F64_LAUNCH(E, CEN, false, true); else FD_F64_LAUNCH(E, CEN, false, false); }
  const size_t esz = I.elem_bytes, pair = 2 * esz;
  // Pair loads need both rows of A and B to start on a pair boundary, and K
  // and N even so that no pair reaches past the end of a row.
  bool vec = lda % 2 == 0 && ldb % 2 == 0 && K % 2 == 0 && N % 2 == 0 &&
             ((uintptr_t)A) % pair == 0 && ((uintptr_t)B) % pair == 0;
  // Any other shape or layout: A and B are copied into scratch with rows
  // padded by zeros to an even length, so every pair load stays inside its
  // padded row; the kernel's masks by K and N still drop the padding.
  if (!vec && K > 0 && M > 0 && N > 0 && fd_tune("gemm.f64.pad", 1) != 0) {
    const size_t Kp = K + (K & 1), Np = N + (N & 1);
    const size_t a_bytes = (M * Kp * esz + 255) / 256 * 256;
    void* scr = nullptr;
    fdot_status_t st = scratch_for(s, a_bytes + K * Np * esz, &scr);
    if (st != FDOT_OK) return st;
    char* ap = (char*)scr;
    char* bp = ap + a_bytes;
    const hipError_t ea = esz == 8 ? pad_copy<uint64_t>(A, lda, M, K, ap, Kp, s)
                                   : pad_copy<uint32_t>(A, lda, M, K, ap, Kp, s);
    const hipError_t eb = esz == 8 ? pad_copy<uint64_t>(B, ldb, K, N, bp, Np, s)
                                   : pad_copy<uint32_t>(B, ldb, K, N, bp, Np, s);
    if (ea != hipSuccess || eb != hipSuccess) return FDOT_E_DEVICE;
    A = ap;
    lda = Kp;
    B = bp;
    ldb = Np;
    vec = true;
  }
  if (I.rep == FDOT_REP_FP64) {
    if (centre) { FD_F64_PICK(double, true) } else { FD_F64_PICK(double, false) }
  } else {
    if (centre) { FD_F64_PICK(uint32_t, true) } else { FD_F64_PICK(uint32_t, false) }
  }
#undef FD_F64_PICK
#undef FD_F64_LAUNCH
#undef FD_F64_LAUNCH_NW
  return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
}
