// Streaming dot products over GF(p): the single form (one vector pair) and the
// batched form (many pairs of uneven length in one launch), plus the
// representation conversions and the matrix-vector product.
//
// Work decomposition.  A vector pair is cut into chunks of `chunk` elements;
// a workgroup streams one chunk with 16-byte loads, every lane accumulating
// its share in registers (the delayed reduction of Sec. 3.1-3.2, the on-demand
// correction of Sec. 3.3, or a per-term reduction), then folds its
// accumulators to a residue below p.  The workgroup sums its lanes' residues,
// folds once more and adds the result (< p) to the pair's 64-bit accumulator
// with one atomic; the workgroup that completes a pair's last chunk reads the
// accumulator, reduces it, encodes the result in the pair's representation and
// puts the accumulator and its ticket back to zero for the next call.  Integer
// sums are exact and associative, so the result is the same bit pattern
// whatever the order in which chunks finish.
#include <stdio.h>
#include <string.h>

#include <type_traits>

#include "fdot_internal.h"

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

namespace {

struct Job {
  const void* x;             // single form
  const void* y;
  uint64_t n;
  const fdot_desc_t* desc;   // batched form
  uint64_t count;
  const uint64_t* offsets;   // chunk prefix sums (count + 1)
  const uint64_t* total;     // number of chunks of the batch
  uint64_t chunk;            // elements per chunk
  unsigned long long* acc;
  unsigned int* done;
  void* results;
  uint32_t fold_vecs;        // vectors between two folds (folding policies)
  uint32_t pad;
};

__device__ __forceinline__ uint32_t lo16(uint32_t w) { return w & 0xFFFFu; }
__device__ __forceinline__ uint32_t hi16(uint32_t w) { return w >> 16; }

struct D2 {
  double x, y;
};
__device__ __forceinline__ D2 as_d2(const u32x4& v) {
  D2 d;
  __builtin_memcpy(&d, &v, sizeof(d));
  return d;
}

// ------------------------------------------------------------------ policies
// Each lane policy keeps a lane's accumulators and knows how to consume one
// 16-byte vector pair, one scalar pair, how to fold its state to a residue in
// [0, p) and how to encode a final residue in its representation.

// Classical residues, 64-bit accumulators, one reduction per block of at most
// lambda products (Sec. 3.1 Eq. 1, Sec. 3.2).  With FOLD = false the host has
// checked that a lane never receives more than lambda products per chunk.
template <bool FOLD>
struct PZpzDelayed {
  using E = uint32_t;
  static constexpr int VW = 4;
  static constexpr int U = 4;
  uint64_t s0, s1;
  uint32_t cnt;
  __device__ void init(const FieldK&) { s0 = s1 = 0; cnt = 0; }
  __device__ void vec(const u32x4& a, const u32x4& b, const FieldK& F, const Job& J) {
    s0 += (uint64_t)a.x * b.x;
    s1 += (uint64_t)a.y * b.y;
    s0 += (uint64_t)a.z * b.z;
    s1 += (uint64_t)a.w * b.w;
    if (FOLD && ++cnt == J.fold_vecs) {
      s0 = mod_u64(s0, F);
      s1 = mod_u64(s1, F);
      cnt = 0;
    }
  }
  __device__ void one(E a, E b, const FieldK& F, const Job&) {
    s0 += (uint64_t)a * b;
    if (FOLD) s0 = mod_u64(s0, F);
  }
  __device__ uint32_t finish(const FieldK& F) {
    return mod_u64((uint64_t)mod_u64(s0, F) + mod_u64(s1, F), F);
  }
  __device__ static void store(void* out, uint64_t k, uint32_t r, const FieldK&) {
    ((uint32_t*)out)[k] = r;
  }
};

// Classical residues reduced after every product (the AXPY of Sec. 2.1):
// acc + a*b < p*2^32, so one 2-by-1 division step per term.  Four independent
// accumulators per lane keep the dependency chains short.
struct PZpzPerTerm {
  using E = uint32_t;
  static constexpr int VW = 4;
  static constexpr int U = 4;
  uint32_t a0, a1, a2, a3;
  __device__ void init(const FieldK&) { a0 = a1 = a2 = a3 = 0; }
  __device__ void vec(const u32x4& a, const u32x4& b, const FieldK& F, const Job&) {
    a0 = mod_small((uint64_t)a.x * b.x + a0, F);
    a1 = mod_small((uint64_t)a.y * b.y + a1, F);
    a2 = mod_small((uint64_t)a.z * b.z + a2, F);
    a3 = mod_small((uint64_t)a.w * b.w + a3, F);
  }
  __device__ void one(E a, E b, const FieldK& F, const Job&) {
    a0 = mod_small((uint64_t)a * b + a0, F);
  }
  __device__ uint32_t finish(const FieldK& F) {
    return mod_u64((uint64_t)a0 + a1 + a2 + a3, F);
  }
  __device__ static void store(void* out, uint64_t k, uint32_t r, const FieldK&) {
    ((uint32_t*)out)[k] = r;
  }
};

// Division on demand (Sec. 3.3): the 64-bit sum may wrap; a wrap happened
// iff the new sum is below the product just added, and then 2^64 mod p is
// added back.  After a wrap the sum is below the product, so adding the
// correction (< p) cannot wrap again.
__device__ __forceinline__ void ovf_add(uint64_t& s, uint64_t prod, uint64_t corr) {
  s += prod;
  if (s < prod) s += corr;
}

// MONT = false: classical residues.  MONT = true: Montgomery residues, whose
// products X*Y carry a factor B^2, so the folded sum is (sum x*y) B^2 and one
// final reduction REDC brings it to the Montgomery form (sum x*y) B: the
// "k+1 reductions" of overflow-Montgomery (Sec. 3.3).
template <bool MONT>
struct POverflow {
  using E = uint32_t;
  static constexpr int VW = 4;
  static constexpr int U = 4;
  uint64_t s0, s1;
  __device__ void init(const FieldK&) { s0 = s1 = 0; }
  __device__ void vec(const u32x4& a, const u32x4& b, const FieldK& F, const Job&) {
    ovf_add(s0, (uint64_t)a.x * b.x, F.corr);
    ovf_add(s1, (uint64_t)a.y * b.y, F.corr);
    ovf_add(s0, (uint64_t)a.z * b.z, F.corr);
    ovf_add(s1, (uint64_t)a.w * b.w, F.corr);
  }
  __device__ void one(E a, E b, const FieldK& F, const Job&) {
    ovf_add(s0, (uint64_t)a * b, F.corr);
  }
  __device__ uint32_t finish(const FieldK& F) {
    return mod_u64((uint64_t)mod_u64(s0, F) + mod_u64(s1, F), F);
  }
  __device__ static void store(void* out, uint64_t k, uint32_t r, const FieldK& F) {
    ((uint32_t*)out)[k] = MONT ? redc(r, F) : r;
  }
};

// Montgomery residues (B = 2^32) with one REDC per block (Sec. 3.2.1): a
// block sums at most lambda_redc products X*Y, each carrying B^2, and stays
// below p*B, so REDC returns (block sum)*B^-1 mod p, which is already in
// Montgomery form.  The REDC outputs of the blocks are added as plain
// residues and reduced once at the end.
template <bool FOLD>
struct PMontDelayed {
  using E = uint32_t;
  static constexpr int VW = 4;
  static constexpr int U = 4;
  uint64_t t0, t1, tot;
  uint32_t cnt;
  __device__ void init(const FieldK&) { t0 = t1 = tot = 0; cnt = 0; }
  __device__ void vec(const u32x4& a, const u32x4& b, const FieldK& F, const Job& J) {
    t0 += (uint64_t)a.x * b.x;
    t1 += (uint64_t)a.y * b.y;
    t0 += (uint64_t)a.z * b.z;
    t1 += (uint64_t)a.w * b.w;
    if (FOLD && ++cnt == J.fold_vecs) {
      tot += (uint64_t)redc(t0, F) + redc(t1, F);
      t0 = t1 = 0;
      cnt = 0;
    }
  }
  __device__ void one(E a, E b, const FieldK& F, const Job&) {
    t0 += (uint64_t)a * b;
    if (FOLD) {
      tot += redc(t0, F);
      t0 = 0;
    }
  }
  __device__ uint32_t finish(const FieldK& F) {
    return mod_u64(tot + redc(t0, F) + redc(t1, F), F);
  }
  __device__ static void store(void* out, uint64_t k, uint32_t r, const FieldK&) {
    ((uint32_t*)out)[k] = r;
  }
};

// Montgomery residues, one REDC per product (a Montgomery multiplication per
// term, Sec. 2.2), for primes so close to 2^32 that two products overflow
// p*B.
struct PMontPerTerm {
  using E = uint32_t;
  static constexpr int VW = 4;
  static constexpr int U = 4;
  uint64_t t0, t1;
  __device__ void init(const FieldK&) { t0 = t1 = 0; }
  __device__ void vec(const u32x4& a, const u32x4& b, const FieldK& F, const Job&) {
    t0 += redc((uint64_t)a.x * b.x, F);
    t1 += redc((uint64_t)a.y * b.y, F);
    t0 += redc((uint64_t)a.z * b.z, F);
    t1 += redc((uint64_t)a.w * b.w, F);
  }
  __device__ void one(E a, E b, const FieldK& F, const Job&) { t0 += redc((uint64_t)a * b, F); }
  __device__ uint32_t finish(const FieldK& F) {
    return mod_u64((uint64_t)mod_u64(t0, F) + mod_u64(t1, F), F);
  }
  __device__ static void store(void* out, uint64_t k, uint32_t r, const FieldK&) {
    ((uint32_t*)out)[k] = r;
  }
};

// Residues held in doubles (Sec. 2.3 with the delayed division of Sec. 3.1,
// m = 53): fused multiply-adds are exact while the integral sum stays at or
// below 2^53; the floating-point remainder folds every lambda_f64 products.
template <bool FOLD>
struct PF64 {
  using E = double;
  static constexpr int VW = 2;
  static constexpr int U = 4;
  double a0, a1;
  uint32_t cnt;
  __device__ void init(const FieldK&) { a0 = a1 = 0.0; cnt = 0; }
  __device__ void vec(const u32x4& av, const u32x4& bv, const FieldK& F, const Job& J) {
    const D2 a = as_d2(av), b = as_d2(bv);
    a0 = fma(a.x, b.x, a0);
    a1 = fma(a.y, b.y, a1);
    if (FOLD && ++cnt == J.fold_vecs) {
      a0 = fold_f64(a0, F);
      a1 = fold_f64(a1, F);
      cnt = 0;
    }
  }
  __device__ void one(E a, E b, const FieldK& F, const Job&) {
    a0 = fma(a, b, a0);
    if (FOLD) a0 = fold_f64(a0, F);
  }
  __device__ uint32_t finish(const FieldK& F) {
    const uint64_t r = (uint64_t)fold_f64(a0, F) + (uint64_t)fold_f64(a1, F);
    return (uint32_t)(r >= F.p ? r - F.p : r);
  }
  __device__ static void store(void* out, uint64_t k, uint32_t r, const FieldK&) {
    ((double*)out)[k] = (double)r;
  }
};

// Zech product: index addition modulo q-1 (Sec. 2.4), code 0 is the zero
// element and absorbs.
__device__ __forceinline__ uint32_t zech_mul(uint32_t a, uint32_t b, uint32_t qbar) {
  uint32_t t = a + b;
  t = t > qbar ? t - qbar : t;
  return (a == 0u || b == 0u) ? 0u : t;
}

// Zech codes; products by index addition, then the value table (in LDS) turns
// each product into a classical residue that is summed with delayed
// reduction (the host checks that a lane's 32-bit sum cannot overflow).
struct PZechExp {
  using E = uint16_t;
  static constexpr int VW = 8;
  static constexpr int U = 2;
  static constexpr bool kTable = true;
  uint32_t s0, s1;
  const uint16_t* tab;  // value table in LDS
  __device__ void init(const FieldK&) { s0 = s1 = 0; }
  __device__ void term(uint32_t& s, uint32_t a, uint32_t b, const FieldK& F) {
    uint32_t t = a + b;
    t = t > F.qbar ? t - F.qbar : t;
    const uint32_t v = tab[t];
    s += (a == 0u || b == 0u) ? 0u : v;
  }
  __device__ void vec(const u32x4& a, const u32x4& b, const FieldK& F, const Job&) {
    term(s0, lo16(a.x), lo16(b.x), F); term(s1, hi16(a.x), hi16(b.x), F);
    term(s0, lo16(a.y), lo16(b.y), F); term(s1, hi16(a.y), hi16(b.y), F);
    term(s0, lo16(a.z), lo16(b.z), F); term(s1, hi16(a.z), hi16(b.z), F);
    term(s0, lo16(a.w), lo16(b.w), F); term(s1, hi16(a.w), hi16(b.w), F);
  }
  __device__ void one(E a, E b, const FieldK& F, const Job&) { term(s0, a, b, F); }
  __device__ uint32_t finish(const FieldK& F) { return mod_u64((uint64_t)s0 + s1, F); }
  __device__ static void store(void* out, uint64_t k, uint32_t r, const FieldK& F) {
    ((uint16_t*)out)[k] = F.zidx[r];
  }
};

// Zech codes with Zech addition (Sec. 2.4): g^u + g^t = g^u (1 + g^(t-u)),
// the exponent of 1 + g^k read from the plus-one table (in LDS), 0 when
// 1 + g^k = 0.  Eight independent Zech accumulators per lane (one per
// element of a 16-byte vector).
struct PZechTplus1 {
  using E = uint16_t;
  static constexpr int VW = 8;
  static constexpr int U = 2;
  static constexpr bool kTable = true;
  uint32_t z[8];
  const uint16_t* tab;  // plus-one table in LDS
  __device__ void init(const FieldK&) {
#pragma unroll
    for (int j = 0; j < 8; ++j) z[j] = 0;
  }
  __device__ uint32_t zadd(uint32_t u, uint32_t t, const FieldK& F) {
    int k = (int)t - (int)u;
    k += (k <= 0) ? (int)F.qbar : 0;  // k in [1, q-1]
    const uint32_t h = tab[k];
    uint32_t w = u + h;
    w = w > F.qbar ? w - F.qbar : w;
    w = (h == 0u) ? 0u : w;
    w = (u == 0u) ? t : w;
    return (t == 0u) ? u : w;
  }
  __device__ void term(int j, uint32_t a, uint32_t b, const FieldK& F) {
    z[j] = zadd(z[j], zech_mul(a, b, F.qbar), F);
  }
  __device__ void vec(const u32x4& a, const u32x4& b, const FieldK& F, const Job&) {
    term(0, lo16(a.x), lo16(b.x), F); term(1, hi16(a.x), hi16(b.x), F);
    term(2, lo16(a.y), lo16(b.y), F); term(3, hi16(a.y), hi16(b.y), F);
    term(4, lo16(a.z), lo16(b.z), F); term(5, hi16(a.z), hi16(b.z), F);
    term(6, lo16(a.w), lo16(b.w), F); term(7, hi16(a.w), hi16(b.w), F);
  }
  __device__ void one(E a, E b, const FieldK& F, const Job&) { term(0, a, b, F); }
  __device__ uint32_t finish(const FieldK& F) {
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += F.zval[z[j]];
    return mod_u64(s, F);
  }
  __device__ static void store(void* out, uint64_t k, uint32_t r, const FieldK& F) {
    ((uint16_t*)out)[k] = F.zidx[r];
  }
};

// Centred residues in int8 (Sec. 3.2.2): four-way int8 dot products into a
// 32-bit accumulator, flushed to 64 bits every lambda_i32c products.
template <bool FOLD>
struct PCentred {
  using E = int8_t;
  static constexpr int VW = 16;
  static constexpr int U = 4;
  int32_t a;
  int64_t acc;
  uint32_t cnt;
  __device__ void init(const FieldK&) { a = 0; acc = 0; cnt = 0; }
  __device__ void vec(const u32x4& x, const u32x4& y, const FieldK&, const Job& J) {
    a = __builtin_amdgcn_sdot4((int)x.x, (int)y.x, a, false);
    a = __builtin_amdgcn_sdot4((int)x.y, (int)y.y, a, false);
    a = __builtin_amdgcn_sdot4((int)x.z, (int)y.z, a, false);
    a = __builtin_amdgcn_sdot4((int)x.w, (int)y.w, a, false);
    if (FOLD && ++cnt == J.fold_vecs) {
      acc += a;
      a = 0;
      cnt = 0;
    }
  }
  __device__ void one(E x, E y, const FieldK&, const Job&) {
    a += (int32_t)x * (int32_t)y;
    if (FOLD) {
      acc += a;
      a = 0;
    }
  }
  __device__ uint32_t finish(const FieldK& F) { return mod_i64(acc + a, F); }
  __device__ static void store(void* out, uint64_t k, uint32_t r, const FieldK& F) {
    const int32_t c = (int32_t)r > F.half ? (int32_t)r - (int32_t)F.p32 : (int32_t)r;
    ((int8_t*)out)[k] = (int8_t)c;
  }
};

template <class P, class = void>
struct HasTable { static constexpr bool value = false; };
template <class P>
struct HasTable<P, decltype((void)P::kTable)> { static constexpr bool value = P::kTable; };

// --------------------------------------------------------------- the driver

// Stream [x, x+len) against [y, y+len) through one lane policy.  16-byte
// vector loads when both pointers share the same offset modulo 16 (a short
// scalar head aligns them); scalar loads otherwise.
template <class Pol, int NTH>
__device__ __forceinline__ void run_range(Pol& L, const typename Pol::E* x,
                                          const typename Pol::E* y, uint64_t len,
                                          const FieldK& F, const Job& J) {
  using E = typename Pol::E;
  constexpr int VW = Pol::VW, U = Pol::U;
  const uint32_t tid = threadIdx.x;
  const uintptr_t ax = (uintptr_t)x & 15u, ay = (uintptr_t)y & 15u;
  if (ax != ay) {
    for (uint64_t i = tid; i < len; i += NTH) L.one(x[i], y[i], F, J);
    return;
  }
  uint64_t head = ax ? (16u - ax) / sizeof(E) : 0;
  if (head > len) head = len;
  if (tid < head) L.one(x[tid], y[tid], F, J);
  const u32x4* xv = (const u32x4*)(x + head);
  const u32x4* yv = (const u32x4*)(y + head);
  const uint64_t nv = (len - head) / VW;
  uint64_t i = tid;
  for (; i + (uint64_t)(U - 1) * NTH < nv; i += (uint64_t)U * NTH) {
    u32x4 a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      a[u] = __builtin_nontemporal_load(xv + i + (uint64_t)u * NTH);
      b[u] = __builtin_nontemporal_load(yv + i + (uint64_t)u * NTH);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) L.vec(a[u], b[u], F, J);
  }
  for (; i < nv; i += NTH) L.vec(xv[i], yv[i], F, J);
  const uint64_t t0 = head + nv * VW;
  if (tid < len - t0) L.one(x[t0 + tid], y[t0 + tid], F, J);
}

// Sum of one 64-bit value per thread; the result is valid in thread 0.
template <int NTH>
__device__ __forceinline__ uint64_t block_sum(uint64_t v, unsigned long long* s) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();  // the previous chunk's reader of s is done
  if ((threadIdx.x & 63u) == 0) s[threadIdx.x >> 6] = v;
  __syncthreads();
  uint64_t t = 0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < NTH / 64; ++w) t += s[w];
  }
  return t;
}

// Largest k with offsets[k] <= c (skips empty instances).
__device__ __forceinline__ uint64_t find_instance(const uint64_t* offsets, uint64_t count,
                                                  uint64_t c) {
  uint64_t lo = 0, hi = count;
  while (lo < hi) {
    const uint64_t mid = (lo + hi + 1) >> 1;
    if (offsets[mid] <= c) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <class Pol, int NTH, bool MANY>
__global__ __launch_bounds__(NTH) void dot_kernel(const FieldK F, const Job J) {
  using E = typename Pol::E;
  extern __shared__ uint16_t s_tab[];
  __shared__ unsigned long long s_red[NTH / 64];
  constexpr bool kTab = HasTable<Pol>::value;
  if (kTab) {
    // The policy's table (p entries of 16 bits) is copied once per workgroup.
    const uint16_t* src = nullptr;
    if constexpr (kTab) src = std::is_same<Pol, PZechExp>::value ? F.zval : F.zplus1;
    for (uint32_t i = threadIdx.x; i < F.p32; i += NTH) s_tab[i] = src[i];
    __syncthreads();
  }
  const uint64_t total = MANY ? *J.total : (J.n + J.chunk - 1) / J.chunk;
  for (uint64_t c = blockIdx.x; c < total; c += gridDim.x) {
    uint64_t k, nck, len;
    const E* x;
    const E* y;
    if (MANY) {
      k = find_instance(J.offsets, J.count, c);
      const uint64_t first = J.offsets[k];
      nck = J.offsets[k + 1] - first;
      const fdot_desc_t d = J.desc[k];
      const uint64_t beg = (c - first) * J.chunk;
      len = d.n - beg < J.chunk ? d.n - beg : J.chunk;
      x = (const E*)d.x + beg;
      y = (const E*)d.y + beg;
    } else {
      k = 0;
      nck = total;
      const uint64_t beg = c * J.chunk;
      len = J.n - beg < J.chunk ? J.n - beg : J.chunk;
      x = (const E*)J.x + beg;
      y = (const E*)J.y + beg;
    }
    Pol L;
    L.init(F);
    if constexpr (kTab) L.tab = s_tab;
    run_range<Pol, NTH>(L, x, y, len, F, J);
    const uint64_t wsum = block_sum<NTH>(L.finish(F), s_red);
    if (threadIdx.x == 0) {
      atomicAdd(J.acc + k, (unsigned long long)mod_u64(wsum, F));
      __threadfence();
      const unsigned prev = atomicAdd(J.done + k, 1u);
      if (prev + 1 == nck) {
        __threadfence();
        const unsigned long long tot = atomicExch(J.acc + k, 0ull);
        atomicExch(J.done + k, 0u);
        Pol::store(J.results, k, mod_u64(tot, F), F);
      }
    }
  }
}

// Chunk plan of a batch: offsets[k] = sum_{j<k} ceil(n_j / chunk),
// offsets[count] = total.  Empty instances get the zero element (all-zero
// bits in every representation) at once, since no chunk will finish them.
constexpr int PLAN_NT = 1024;
__global__ __launch_bounds__(PLAN_NT) void plan_kernel(const fdot_desc_t* desc, uint64_t count,
                                                       uint64_t chunk, uint64_t* offsets,
                                                       uint64_t* total, void* results,
                                                       uint32_t elem_bytes) {
  __shared__ uint64_t s[PLAN_NT];
  const uint32_t t = threadIdx.x;
  const uint64_t seg = (count + PLAN_NT - 1) / PLAN_NT;
  const uint64_t b = t * seg < count ? t * seg : count;
  const uint64_t e = b + seg < count ? b + seg : count;
  uint64_t local = 0;
  for (uint64_t k = b; k < e; ++k) local += (desc[k].n + chunk - 1) / chunk;
  s[t] = local;
  __syncthreads();
  for (uint32_t o = 1; o < PLAN_NT; o <<= 1) {  // inclusive scan
    const uint64_t v = t >= o ? s[t - o] : 0;
    __syncthreads();
    s[t] += v;
    __syncthreads();
  }
  uint64_t run = s[t] - local;
  for (uint64_t k = b; k < e; ++k) {
    offsets[k] = run;
    const uint64_t n = desc[k].n;
    run += (n + chunk - 1) / chunk;
    if (n == 0) {
      uint8_t* r = (uint8_t*)results + k * elem_bytes;
      for (uint32_t i = 0; i < elem_bytes; ++i) r[i] = 0;
    }
  }
  if (t == PLAN_NT - 1) {
    offsets[count] = s[t];
    *total = s[t];
  }
}

__global__ void zero_kernel(uint8_t* p, size_t bytes) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < bytes;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// Zero element for a dot of length 0 in the single form.
__global__ void store_zero_kernel(uint8_t* r, uint32_t bytes) {
  if (threadIdx.x < bytes) r[threadIdx.x] = 0;
}

// -------------------------------------------------------------- conversions
__global__ void encode_kernel(const FieldK F, int rep, const uint32_t* canon, void* out,
                              size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const uint32_t r = canon[i];
    switch (rep) {
      case FDOT_REP_ZPZ_U32: ((uint32_t*)out)[i] = r; break;
      case FDOT_REP_MONT_U32: ((uint32_t*)out)[i] = mod_u64((uint64_t)r << 32, F); break;
      case FDOT_REP_FP64: ((double*)out)[i] = (double)r; break;
      case FDOT_REP_ZECH_U16: ((uint16_t*)out)[i] = F.zidx[r]; break;
      case FDOT_REP_CENTRED_I8:
        ((int8_t*)out)[i] = (int8_t)((int32_t)r > F.half ? (int32_t)r - (int32_t)F.p32 : (int32_t)r);
        break;
    }
  }
}

__global__ void decode_kernel(const FieldK F, int rep, const void* in, uint32_t* canon,
                              size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    uint32_t r = 0;
    switch (rep) {
      case FDOT_REP_ZPZ_U32: r = ((const uint32_t*)in)[i]; break;
      case FDOT_REP_MONT_U32: r = redc(((const uint32_t*)in)[i], F); break;
      case FDOT_REP_FP64: r = (uint32_t)((const double*)in)[i]; break;
      case FDOT_REP_ZECH_U16: r = F.zval[((const uint16_t*)in)[i]]; break;
      case FDOT_REP_CENTRED_I8: {
        const int32_t c = ((const int8_t*)in)[i];
        r = (uint32_t)(c < 0 ? c + (int32_t)F.p32 : c);
        break;
      }
    }
    canon[i] = r;
  }
}

// ------------------------------------------------------------------ gemv
// y = A x: one wavefront per row, the row streamed with the same lane
// policies as the dot product; x is re-read by every row from L2.
template <class Pol>
__global__ __launch_bounds__(256) void gemv_kernel(const FieldK F, const Job J, uint64_t m,
                                                   uint64_t n, uint64_t lda, const void* A,
                                                   const void* x, void* y) {
  using E = typename Pol::E;
  extern __shared__ uint16_t s_tab[];
  constexpr bool kTab = HasTable<Pol>::value;
  if (kTab) {
    const uint16_t* src = nullptr;
    if constexpr (kTab) src = std::is_same<Pol, PZechExp>::value ? F.zval : F.zplus1;
    for (uint32_t i = threadIdx.x; i < F.p32; i += 256) s_tab[i] = src[i];
    __syncthreads();
  }
  const uint64_t row = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= m) return;
  const uint32_t lane = threadIdx.x & 63u;
  const E* a = (const E*)A + row * lda;
  const E* xv = (const E*)x;
  Pol L;
  L.init(F);
  if constexpr (kTab) L.tab = s_tab;
  constexpr int VW = Pol::VW;
  const uintptr_t aa = (uintptr_t)a & 15u, ax = (uintptr_t)xv & 15u;
  if (aa != ax) {
    for (uint64_t i = lane; i < n; i += 64) L.one(a[i], xv[i], F, J);
  } else {
    uint64_t head = aa ? (16u - aa) / sizeof(E) : 0;
    if (head > n) head = n;
    if (lane < head) L.one(a[lane], xv[lane], F, J);
    const u32x4* av = (const u32x4*)(a + head);
    const u32x4* bv = (const u32x4*)(xv + head);
    const uint64_t nv = (n - head) / VW;
    uint64_t i = lane;
    for (; i + 64 < nv; i += 128) {
      const u32x4 a0 = av[i], b0 = bv[i], a1 = av[i + 64], b1 = bv[i + 64];
      L.vec(a0, b0, F, J);
      L.vec(a1, b1, F, J);
    }
    for (; i < nv; i += 64) L.vec(av[i], bv[i], F, J);
    const uint64_t t0 = head + nv * VW;
    if (lane < n - t0) L.one(a[t0 + lane], xv[t0 + lane], F, J);
  }
  uint64_t v = L.finish(F);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  if (lane == 0) Pol::store(y, row, mod_u64(v, F), F);
}

// ---------------------------------------------------------------- launching
enum class Kind {
  ZpzDelayed, ZpzDelayedFold, ZpzPerTerm, ZpzOverflow,
  MontDelayed, MontDelayedFold, MontPerTerm, MontOverflow,
  F64, F64Fold, ZechExp, ZechTplus1, Centred, CentredFold
};

struct Plan {
  Kind kind;
  uint32_t fold_vecs;
  int nth;
  size_t lds;
};

// Products one accumulator of a lane can receive from one chunk (or row):
// ppv per vector, plus at most one head and one tail product.
static uint64_t lane_products(uint64_t chunk, int vw, int nth, uint64_t ppv) {
  const uint64_t vecs = (chunk + (uint64_t)vw * nth - 1) / ((uint64_t)vw * nth);
  return vecs * ppv + 2;
}

static fdot_status_t make_plan(const fdot_field_s* f, fdot_algo_t algo, uint64_t chunk,
                               int nth, Plan* pl) {
  const fdot_field_info_t& I = f->info;
  if (algo == FDOT_ALGO_AUTO) algo = fd_default_algo(f, chunk);
  pl->fold_vecs = 0;
  pl->nth = nth;
  pl->lds = 0;
  switch (I.rep) {
    case FDOT_REP_ZPZ_U32:
      if (algo == FDOT_ALGO_OVERFLOW) { pl->kind = Kind::ZpzOverflow; return FDOT_OK; }
      if (algo == FDOT_ALGO_PERTERM || (algo == FDOT_ALGO_DELAYED && I.lambda_u64 < 2)) {
        pl->kind = Kind::ZpzPerTerm;
        return FDOT_OK;
      }
      if (algo != FDOT_ALGO_DELAYED) return FDOT_E_UNSUPPORTED;
      if (I.lambda_u64 >= lane_products(chunk, 4, nth, 2)) {
        pl->kind = Kind::ZpzDelayed;
      } else {
        pl->kind = Kind::ZpzDelayedFold;
        pl->fold_vecs = (uint32_t)(I.lambda_u64 / 2);
      }
      return FDOT_OK;
    case FDOT_REP_MONT_U32:
      if (algo == FDOT_ALGO_OVERFLOW) { pl->kind = Kind::MontOverflow; return FDOT_OK; }
      if (algo == FDOT_ALGO_PERTERM || (algo == FDOT_ALGO_DELAYED && I.lambda_redc < 2)) {
        pl->kind = Kind::MontPerTerm;
        return FDOT_OK;
      }
      if (algo != FDOT_ALGO_DELAYED) return FDOT_E_UNSUPPORTED;
      if (I.lambda_redc >= lane_products(chunk, 4, nth, 2)) {
        pl->kind = Kind::MontDelayed;
      } else {
        pl->kind = Kind::MontDelayedFold;
        pl->fold_vecs = (uint32_t)(I.lambda_redc / 2);
      }
      return FDOT_OK;
    case FDOT_REP_FP64:
      if (algo == FDOT_ALGO_PERTERM) {
        pl->kind = Kind::F64Fold;
        pl->fold_vecs = 1;
        return FDOT_OK;
      }
      if (algo != FDOT_ALGO_DELAYED) return FDOT_E_UNSUPPORTED;
      if (I.lambda_f64 >= lane_products(chunk, 2, nth, 1)) {
        pl->kind = Kind::F64;
      } else {
        pl->kind = Kind::F64Fold;
        pl->fold_vecs = (uint32_t)(I.lambda_f64 < 0xFFFFFFFFull ? I.lambda_f64 : 0xFFFFFFFFull);
      }
      return FDOT_OK;
    case FDOT_REP_ZECH_U16:
      pl->lds = (size_t)((I.p + 1) / 2) * 4;
      if (algo == FDOT_ALGO_ZECH_TPLUS1) { pl->kind = Kind::ZechTplus1; return FDOT_OK; }
      if (algo != FDOT_ALGO_ZECH_EXP) return FDOT_E_UNSUPPORTED;
      // Each lane sums up to lane_products values below p in 32 bits.
      if (lane_products(chunk, 8, nth, 4) * (I.p - 1) > 0xFFFFFFFFull) return FDOT_E_UNSUPPORTED;
      pl->kind = Kind::ZechExp;
      return FDOT_OK;
    case FDOT_REP_CENTRED_I8:
      if (algo != FDOT_ALGO_DELAYED) return FDOT_E_UNSUPPORTED;
      if (I.lambda_i32c >= lane_products(chunk, 16, nth, 16)) {
        pl->kind = Kind::Centred;
      } else {
        if (I.lambda_i32c < 16) return FDOT_E_UNSUPPORTED;
        pl->kind = Kind::CentredFold;
        pl->fold_vecs = (uint32_t)(I.lambda_i32c / 16);
      }
      return FDOT_OK;
  }
  return FDOT_E_UNSUPPORTED;
}

template <class Pol, int NTH>
static fdot_status_t launch_dot_t(const FieldK& F, const Job& J, bool many, unsigned grid,
                                  size_t lds, hipStream_t s) {
  if (many) {
    auto fn = dot_kernel<Pol, NTH, true>;
    if (lds > 65536) hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(NTH), lds, s, F, J);
  } else {
    auto fn = dot_kernel<Pol, NTH, false>;
    if (lds > 65536) hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(NTH), lds, s, F, J);
  }
  return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
}

static fdot_status_t dispatch(const Plan& pl, const FieldK& F, const Job& J, bool many,
                              unsigned grid, hipStream_t s) {
  switch (pl.kind) {
    case Kind::ZpzDelayed: return launch_dot_t<PZpzDelayed<false>, 256>(F, J, many, grid, 0, s);
    case Kind::ZpzDelayedFold: return launch_dot_t<PZpzDelayed<true>, 256>(F, J, many, grid, 0, s);
    case Kind::ZpzPerTerm: return launch_dot_t<PZpzPerTerm, 256>(F, J, many, grid, 0, s);
    case Kind::ZpzOverflow: return launch_dot_t<POverflow<false>, 256>(F, J, many, grid, 0, s);
    case Kind::MontDelayed: return launch_dot_t<PMontDelayed<false>, 256>(F, J, many, grid, 0, s);
    case Kind::MontDelayedFold: return launch_dot_t<PMontDelayed<true>, 256>(F, J, many, grid, 0, s);
    case Kind::MontPerTerm: return launch_dot_t<PMontPerTerm, 256>(F, J, many, grid, 0, s);
    case Kind::MontOverflow: return launch_dot_t<POverflow<true>, 256>(F, J, many, grid, 0, s);
    case Kind::F64: return launch_dot_t<PF64<false>, 256>(F, J, many, grid, 0, s);
    case Kind::F64Fold: return launch_dot_t<PF64<true>, 256>(F, J, many, grid, 0, s);
    case Kind::ZechExp: return launch_dot_t<PZechExp, 1024>(F, J, many, grid, pl.lds, s);
    case Kind::ZechTplus1: return launch_dot_t<PZechTplus1, 1024>(F, J, many, grid, pl.lds, s);
    case Kind::Centred: return launch_dot_t<PCentred<false>, 256>(F, J, many, grid, 0, s);
    case Kind::CentredFold: return launch_dot_t<PCentred<true>, 256>(F, J, many, grid, 0, s);
  }
  return FDOT_E_UNSUPPORTED;
}

static const char* rep_key(int rep) {
  switch (rep) {
    case FDOT_REP_ZPZ_U32: return "zpz";
    case FDOT_REP_MONT_U32: return "mont";
    case FDOT_REP_FP64: return "fp64";
    case FDOT_REP_ZECH_U16: return "zech";
    case FDOT_REP_CENTRED_I8: return "centred";
  }
  return "zpz";
}

struct LaunchShape {
  uint64_t chunk;
  int nth;
  unsigned max_grid;
};

static LaunchShape shape_for(const fdot_field_s* f) {
  char key[64];
  const char* r = rep_key(f->info.rep);
  const bool zech = f->info.rep == FDOT_REP_ZECH_U16;
  // Defaults: 256 KiB per operand per chunk for 16-byte-vector policies.
  const int64_t dflt_chunk = (int64_t)(262144 / f->info.elem_bytes);
  snprintf(key, sizeof key, "chunk.%s", r);
  int64_t chunk = fd_tune(key, dflt_chunk);
  chunk = (chunk + 15) / 16 * 16;
  if (chunk < 1024) chunk = 1024;
  snprintf(key, sizeof key, "wg_per_cu.%s", r);
  int64_t wpc = fd_tune(key, zech ? (f->info.p <= 40000 ? 2 : 1) : 8);
  if (wpc < 1) wpc = 1;
  LaunchShape sh;
  sh.chunk = (uint64_t)chunk;
  sh.nth = zech ? 1024 : 256;
  sh.max_grid = (unsigned)(fd_cu_count() * wpc);
  return sh;
}

}  // namespace

fdot_algo_t fd_default_algo(const fdot_field_s* f, uint64_t) {
  const fdot_field_info_t& I = f->info;
  switch (I.rep) {
    case FDOT_REP_ZPZ_U32:
      if (I.lambda_u64 >= 2) return FDOT_ALGO_DELAYED;
      return (fdot_algo_t)fd_tune("auto.zpz.lambda1", FDOT_ALGO_PERTERM);
    case FDOT_REP_MONT_U32: return (fdot_algo_t)fd_tune("auto.mont", FDOT_ALGO_DELAYED);
    case FDOT_REP_FP64: return FDOT_ALGO_DELAYED;
    case FDOT_REP_ZECH_U16: return (fdot_algo_t)fd_tune("auto.zech", FDOT_ALGO_ZECH_EXP);
    case FDOT_REP_CENTRED_I8: return FDOT_ALGO_DELAYED;
  }
  return FDOT_ALGO_DELAYED;
}

fdot_status_t fd_launch_dot(const fdot_field_s* f, fdot_algo_t algo, const void* x, const void* y,
                            uint64_t n, void* result, Workspace* ws, hipStream_t s) {
  if (n == 0) {
    hipLaunchKernelGGL(store_zero_kernel, dim3(1), dim3(64), 0, s, (uint8_t*)result,
                       f->info.elem_bytes);
    return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
  }
  const LaunchShape sh = shape_for(f);
  Plan pl;
  fdot_status_t st = make_plan(f, algo, sh.chunk, sh.nth, &pl);
  if (st != FDOT_OK) return st;
  Job J;
  memset(&J, 0, sizeof J);
  J.x = x;
  J.y = y;
  J.n = n;
  J.chunk = sh.chunk;
  J.acc = ws->acc;
  J.done = ws->done;
  J.results = result;
  J.fold_vecs = pl.fold_vecs;
  const uint64_t chunks = (n + sh.chunk - 1) / sh.chunk;
  const unsigned grid = (unsigned)(chunks < sh.max_grid ? chunks : sh.max_grid);
  return dispatch(pl, f->k, J, false, grid, s);
}

fdot_status_t fd_launch_many(const fdot_field_s* f, fdot_algo_t algo, size_t count,
                             const fdot_desc_t* desc, void* results, Workspace* ws,
                             hipStream_t s) {
  if (count == 0) return FDOT_OK;
  const LaunchShape sh = shape_for(f);
  Plan pl;
  fdot_status_t st = make_plan(f, algo, sh.chunk, sh.nth, &pl);
  if (st != FDOT_OK) return st;
  hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(PLAN_NT), 0, s, desc, (uint64_t)count, sh.chunk,
                     ws->offsets, ws->total, results, f->info.elem_bytes);
  if (hipGetLastError() != hipSuccess) return FDOT_E_DEVICE;
  Job J;
  memset(&J, 0, sizeof J);
  J.desc = desc;
  J.count = count;
  J.offsets = ws->offsets;
  J.total = ws->total;
  J.chunk = sh.chunk;
  J.acc = ws->acc;
  J.done = ws->done;
  J.results = results;
  J.fold_vecs = pl.fold_vecs;
  return dispatch(pl, f->k, J, true, sh.max_grid, s);
}

fdot_status_t fd_launch_encode(const fdot_field_s* f, const uint32_t* canon, void* rep, size_t n,
                               hipStream_t s) {
  if (n == 0) return FDOT_OK;
  const size_t blocks = (n + 255) / 256 < 16384 ? (n + 255) / 256 : 16384;
  hipLaunchKernelGGL(encode_kernel, dim3((unsigned)blocks), dim3(256), 0, s, f->k, f->info.rep,
                     canon, rep, n);
  return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
}

fdot_status_t fd_launch_decode(const fdot_field_s* f, const void* rep, uint32_t* canon, size_t n,
                               hipStream_t s) {
  if (n == 0) return FDOT_OK;
  const size_t blocks = (n + 255) / 256 < 16384 ? (n + 255) / 256 : 16384;
  hipLaunchKernelGGL(decode_kernel, dim3((unsigned)blocks), dim3(256), 0, s, f->k, f->info.rep,
                     rep, canon, n);
  return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
}

fdot_status_t fd_launch_zero(void* ptr, size_t bytes, hipStream_t s) {
  if (bytes == 0) return FDOT_OK;
  const size_t blocks = (bytes + 255) / 256 < 4096 ? (bytes + 255) / 256 : 4096;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (uint8_t*)ptr, bytes);
  return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
}

template <class Pol>
static fdot_status_t launch_gemv_t(const fdot_field_s* f, const Job& J, size_t m, size_t n,
                                   const void* A, size_t lda, const void* x, void* y, size_t lds,
                                   hipStream_t s) {
  auto fn = gemv_kernel<Pol>;
  if (lds > 65536) hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(fn, dim3((unsigned)((m + 3) / 4)), dim3(256), lds, s, f->k, J, (uint64_t)m,
                     (uint64_t)n, (uint64_t)lda, A, x, y);
  return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
}

fdot_status_t fd_launch_gemv(const fdot_field_s* f, size_t m, size_t n, const void* A, size_t lda,
                             const void* x, void* y, hipStream_t s) {
  if (m == 0) return FDOT_OK;
  // A row is one "chunk" streamed by one wavefront (64 lanes).
  Plan pl;
  fdot_algo_t algo = fd_default_algo(f, n);
  if (f->info.rep == FDOT_REP_ZECH_U16) algo = FDOT_ALGO_ZECH_EXP;
  fdot_status_t st = make_plan(f, algo, n ? n : 1, 64, &pl);
  if (st != FDOT_OK) return st;
  if (pl.lds) pl.lds = (size_t)f->info.p * 2;
  Job J;
  memset(&J, 0, sizeof J);
  J.fold_vecs = pl.fold_vecs;
  switch (pl.kind) {
    case Kind::ZpzDelayed: return launch_gemv_t<PZpzDelayed<false>>(f, J, m, n, A, lda, x, y, 0, s);
    case Kind::ZpzDelayedFold: return launch_gemv_t<PZpzDelayed<true>>(f, J, m, n, A, lda, x, y, 0, s);
    case Kind::ZpzPerTerm: return launch_gemv_t<PZpzPerTerm>(f, J, m, n, A, lda, x, y, 0, s);
    case Kind::ZpzOverflow: return launch_gemv_t<POverflow<false>>(f, J, m, n, A, lda, x, y, 0, s);
    case Kind::MontDelayed: return launch_gemv_t<PMontDelayed<false>>(f, J, m, n, A, lda, x, y, 0, s);
    case Kind::MontDelayedFold: return launch_gemv_t<PMontDelayed<true>>(f, J, m, n, A, lda, x, y, 0, s);
    case Kind::MontPerTerm: return launch_gemv_t<PMontPerTerm>(f, J, m, n, A, lda, x, y, 0, s);
    case Kind::MontOverflow: return launch_gemv_t<POverflow<true>>(f, J, m, n, A, lda, x, y, 0, s);
    case Kind::F64: return launch_gemv_t<PF64<false>>(f, J, m, n, A, lda, x, y, 0, s);
    case Kind::F64Fold: return launch_gemv_t<PF64<true>>(f, J, m, n, A, lda, x, y, 0, s);
    case Kind::ZechExp: return launch_gemv_t<PZechExp>(f, J, m, n, A, lda, x, y, pl.lds, s);
    case Kind::ZechTplus1: return launch_gemv_t<PZechTplus1>(f, J, m, n, A, lda, x, y, pl.lds, s);
    case Kind::Centred: return launch_gemv_t<PCentred<false>>(f, J, m, n, A, lda, x, y, 0, s);
    case Kind::CentredFold: return launch_gemv_t<PCentred<true>>(f, J, m, n, A, lda, x, y, 0, s);
  }
  return FDOT_E_UNSUPPORTED;
}
