// Streaming dot products over GF(p): the single form (one vector pair) and the
// batched form (many pairs of uneven length in one launch), plus the
// representation conversions and the matrix-vector product.
//
// Work decomposition.  The unit of work is one wavefront streaming a slice of
// one pair with 16-byte loads, each lane accumulating its share in registers
// (the delayed reduction of Sec. 3.1-3.2, the on-demand correction of
// Sec. 3.3, or a per-term reduction) and folding to a residue below p at the
// end.  The single form cuts its pair into chunks, about one per resident
// wavefront.  The batched form lays the pairs end to end (each padded to a
// multiple of 64 elements) and cuts that sequence into equal ranges, one per
// group of S wavefronts, so that every wavefront streams the same number of
// bytes whatever the lengths of the pairs: a range covers the tail of one
// pair, whole pairs and the head of the next, and each piece is one unit.
//
// Combination.  The wavefront sums its lanes' residues with cross-lane
// shuffles, folds once more, and adds the result r < p to the pair's
// combination word with one 64-bit atomic: the low 48 bits collect the
// residues, the high 16 bits count finished units.  A pair has at most 65535
// units, so the low field cannot overflow into the count, and the wavefront
// whose atomic returns count = units-1 holds the complete sum: it reduces it,
// encodes the result in the pair's representation and puts the word back to
// zero for the next call.  No workgroup barrier, no memory fence: waves never
// wait for one another.  Integer sums are exact and associative, so the
// result is the same bit pattern whatever order the units finish in.
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "fdot_internal.h"
#include "zech_packed.h"

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// 16-byte loads issued per operand before they are consumed (per lane).
#ifndef FDOT_UNROLL
#define FDOT_UNROLL 4
#endif

// Operand pointers reach the kernels through descriptors, so the compiler
// cannot tell they address global memory and would emit flat loads, which
// it must wait for all at once.  These casts make every streaming load a
// global load, so a wavefront keeps all of its loads in flight.
typedef __attribute__((address_space(1))) const u32x4 gvec_t;
template <typename T>
using gptr_t = __attribute__((address_space(1))) const T*;

__device__ __forceinline__ u32x4 load_nt(const u32x4* p) {
  return __builtin_nontemporal_load((gvec_t*)p);
}
__device__ __forceinline__ u32x4 load_v(const u32x4* p) { return *(gvec_t*)p; }
template <typename T>
__device__ __forceinline__ T load_s(const T* p) {
  return *(gptr_t<T>)p;
}

namespace {

constexpr uint64_t kCountOne = 1ull << 48;
constexpr uint64_t kSumMask = kCountOne - 1;
constexpr uint64_t kMaxUnits = 65535;  // per pair: the 16-bit count field

struct Job {
  const void* x;             // single form
  const void* y;
  uint64_t n;
  uint64_t chunk;            // single form: elements per chunk (at least; see chunk_of)
  const fdot_desc_t* desc;   // batched form
  uint64_t count;
  const uint64_t* first;     // batched: position of each pair in the padded sequence
  const uint32_t* units;     // batched: units of each pair
  const uint32_t* start;     // batched: first pair of each range
  const uint64_t* tq;        // batched: padded total T, range length Q, ranges R
  uint64_t q_target;         // batched: elements per range (target)
  uint32_t groups;           // batched: groups of S wavefronts
  uint32_t max_ranges;       // batched: most ranges
  unsigned long long* acc;   // combination words, one per pair
  void* results;
  uint32_t fold_vecs;        // vectors between two folds
  uint32_t slice_shift;      // log2 of the wavefronts sharing one chunk or range
  uint32_t elem_bytes;       // bytes of one result
  uint32_t spread;           // single form: first-level combination words (<= 1: one word)
};

// Single form: first-level combination word j sits kSpreadStride words
// after the previous one, so that the words fall in distinct cache lines
// and memory channels and their atomics proceed in parallel.
constexpr uint32_t kSpreadStride = 32;
constexpr uint32_t kSpreadMax = 64;

// Chunk length used for a pair of length n: the configured chunk, or longer
// when the pair would otherwise need more than 65535 work units (chunks x
// slices), the most the 16-bit count of its combination word can hold.
__host__ __device__ __forceinline__ uint64_t chunk_of(uint64_t n, uint64_t chunk,
                                                      uint32_t slice_shift) {
  const uint64_t max_chunks = kMaxUnits >> slice_shift;
  const uint64_t need = (n + max_chunks - 1) / max_chunks;
  const uint64_t c = (need + 15) / 16 * 16;
  return c > chunk ? c : chunk;
}

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
// A lane policy keeps one lane's accumulators and knows how to consume one
// 16-byte vector pair, one scalar pair, how to fold its state to a residue in
// [0, p) and how to encode a final residue in its representation.  Policies
// with a block bound count vectors and fold every J.fold_vecs of them; the
// host sets fold_vecs from lambda so that no accumulator can overflow, and to
// 2^32-1 (never reached) when lambda is out of reach.

// Classical residues, 64-bit accumulators, one reduction per block of at most
// lambda products (Sec. 3.1 Eq. 1 with the carried residue, Sec. 3.2).  Two
// accumulators, each taking two products per vector.
struct PZpzDelayed {
  using E = uint32_t;
  static constexpr int VW = 4;
  static constexpr int U = FDOT_UNROLL;
  static constexpr bool kFolds = true;
  uint64_t s0, s1;
  __device__ void init(const FieldK&) { s0 = s1 = 0; }
  __device__ void vec(const u32x4& a, const u32x4& b, const FieldK&) {
    s0 += (uint64_t)a.x * b.x;
    s1 += (uint64_t)a.y * b.y;
    s0 += (uint64_t)a.z * b.z;
    s1 += (uint64_t)a.w * b.w;
  }
  __device__ void fold(const FieldK& F) {
    s0 = mod_u64(s0, F);
    s1 = mod_u64(s1, F);
  }
  __device__ void one(E a, E b, const FieldK& F, const Job&) {
    s0 = mod_u64(s0 + (uint64_t)a * b, F);
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
  static constexpr int U = FDOT_UNROLL;
  uint32_t a0, a1, a2, a3;
  __device__ void init(const FieldK&) { a0 = a1 = a2 = a3 = 0; }
  __device__ void vec(const u32x4& a, const u32x4& b, const FieldK& F) {
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
  static constexpr int U = FDOT_UNROLL;
  uint64_t s0, s1;
  __device__ void init(const FieldK&) { s0 = s1 = 0; }
  __device__ void vec(const u32x4& a, const u32x4& b, const FieldK& F) {
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

// Block-overflow (Sec. 3.4): products are added without a test for blocks of
// at most lambda of them, lambda p (p-1) < 2^64, so a block wraps the sum at
// most once; the wrap shows as a sum below the block's starting value and is
// corrected with CORR = 2^64 mod p, which cannot wrap again (the sum after a
// wrap is below lambda (p-1)^2).  Two accumulators, each taking two products
// per vector; fold() closes the blocks.  MONT as in POverflow.
template <bool MONT>
struct PHybrid {
  using E = uint32_t;
  static constexpr int VW = 4;
  static constexpr int U = FDOT_UNROLL;
  static constexpr bool kFolds = true;
  uint64_t s0, s1, b0, b1;
  uint64_t corr;
  __device__ void init(const FieldK& F) {
    s0 = s1 = b0 = b1 = 0;
    corr = F.corr;
  }
  __device__ void vec(const u32x4& a, const u32x4& b, const FieldK&) {
    s0 += (uint64_t)a.x * b.x;
    s1 += (uint64_t)a.y * b.y;
    s0 += (uint64_t)a.z * b.z;
    s1 += (uint64_t)a.w * b.w;
  }
  __device__ void fold(const FieldK&) {
    s0 += s0 < b0 ? corr : 0;
    s1 += s1 < b1 ? corr : 0;
    b0 = s0;
    b1 = s1;
  }
  __device__ void one(E a, E b, const FieldK& F, const Job&) {
    fold(F);
    ovf_add(s0, (uint64_t)a * b, corr);
    b0 = s0;
  }
  __device__ uint32_t finish(const FieldK& F) {
    fold(F);
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
struct PMontDelayed {
  using E = uint32_t;
  static constexpr int VW = 4;
  static constexpr int U = FDOT_UNROLL;
  static constexpr bool kFolds = true;
  uint64_t t0, t1, tot;
  __device__ void init(const FieldK&) { t0 = t1 = tot = 0; }
  __device__ void vec(const u32x4& a, const u32x4& b, const FieldK&) {
    t0 += (uint64_t)a.x * b.x;
    t1 += (uint64_t)a.y * b.y;
    t0 += (uint64_t)a.z * b.z;
    t1 += (uint64_t)a.w * b.w;
  }
  __device__ void fold(const FieldK& F) {
    tot += (uint64_t)redc(t0, F) + redc(t1, F);
    t0 = t1 = 0;
  }
  __device__ void one(E a, E b, const FieldK& F, const Job&) {
    tot += redc((uint64_t)a * b, F);
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
  static constexpr int U = FDOT_UNROLL;
  uint64_t t0, t1;
  __device__ void init(const FieldK&) { t0 = t1 = 0; }
  __device__ void vec(const u32x4& a, const u32x4& b, const FieldK& F) {
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
struct PF64 {
  using E = double;
  static constexpr int VW = 2;
  static constexpr int U = FDOT_UNROLL;
  static constexpr bool kFolds = true;
  double a0, a1;
  __device__ void init(const FieldK&) { a0 = a1 = 0.0; }
  __device__ void vec(const u32x4& av, const u32x4& bv, const FieldK&) {
    const D2 a = as_d2(av), b = as_d2(bv);
    a0 = fma(a.x, b.x, a0);
    a1 = fma(a.y, b.y, a1);
  }
  __device__ void fold(const FieldK& F) {
    a0 = fold_f64(a0, F);
    a1 = fold_f64(a1, F);
  }
  __device__ void one(E a, E b, const FieldK& F, const Job&) { a0 = fold_f64(fma(a, b, a0), F); }
  __device__ uint32_t finish(const FieldK& F) {
    const uint64_t r = (uint64_t)fold_f64(a0, F) + (uint64_t)fold_f64(a1, F);
    return (uint32_t)(r >= F.p ? r - F.p : r);
  }
  __device__ static void store(void* out, uint64_t k, uint32_t r, const FieldK&) {
    ((double*)out)[k] = (double)r;
  }
};

// Zech product: index addition modulo q-1 (Sec. 2.4); code 0 is the zero
// element and absorbs.
__device__ __forceinline__ uint32_t zech_mul(uint32_t a, uint32_t b, uint32_t qbar) {
  uint32_t t = a + b;
  t = t > qbar ? t - qbar : t;
  return (a == 0u || b == 0u) ? 0u : t;
}

// Zech codes; products by index addition, then the value table (in LDS) turns
// each product into a classical residue that is summed with delayed
// reduction: two 32-bit sums, each taking four values per vector, flushed to
// 64 bits every fold_vecs vectors.
struct PZechExp {
  using E = uint16_t;
  static constexpr int VW = 8;
  static constexpr int U = 2;
  static constexpr bool kTable = true;
  static constexpr bool kPrefetch = true;
  static constexpr bool kFolds = true;
  uint32_t s0, s1;
  uint64_t tot;
  const uint16_t* tab;  // value table in LDS
  __device__ void init(const FieldK&) { s0 = s1 = 0; tot = 0; }
  __device__ void term(uint32_t& s, uint32_t a, uint32_t b, const FieldK& F) {
    uint32_t t = a + b;
    t = t > F.qbar ? t - F.qbar : t;
    const uint32_t v = tab[t];
    s += (a == 0u || b == 0u) ? 0u : v;
  }
  __device__ void vec(const u32x4& a, const u32x4& b, const FieldK& F) {
    term(s0, lo16(a.x), lo16(b.x), F); term(s1, hi16(a.x), hi16(b.x), F);
    term(s0, lo16(a.y), lo16(b.y), F); term(s1, hi16(a.y), hi16(b.y), F);
    term(s0, lo16(a.z), lo16(b.z), F); term(s1, hi16(a.z), hi16(b.z), F);
    term(s0, lo16(a.w), lo16(b.w), F); term(s1, hi16(a.w), hi16(b.w), F);
  }
  __device__ void fold(const FieldK&) {
    tot += (uint64_t)s0 + s1;
    s0 = s1 = 0;
  }
  __device__ void one(E a, E b, const FieldK& F, const Job&) {
    uint32_t s = 0;
    term(s, a, b, F);
    tot += s;
  }
  __device__ uint32_t finish(const FieldK& F) { return mod_u64(tot + s0 + s1, F); }
  __device__ static void store(void* out, uint64_t k, uint32_t r, const FieldK& F) {
    ((uint16_t*)out)[k] = F.zidx[r];
  }
};

// The value table with two codes per register, for q <= 32768 (every code
// fits 15 bits, a sum of two fits 16): the product's index (a + b) mod q' is
// the minimum of s and s - q' in packed 16-bit arithmetic, in [0, q'], with
// the staged table's entry 0 set to entry q' (the value 1 of g^0); a zero
// factor is masked out of the loaded pair of values by a bit mask.  The
// values still go into two 32-bit sums (low and high halves), folded as
// PZechExp's.
struct PZechExpP {
  using E = uint16_t;
  static constexpr int VW = 8;
  static constexpr int U = 2;
  static constexpr bool kTable = true;
  static constexpr bool kPrefetch = true;
  static constexpr bool kFolds = true;
  static constexpr bool kEntry0 = true;
  uint32_t s0, s1;
  uint64_t tot;
  const uint16_t* tab;  // value table in LDS, entry 0 = entry q'
  ZechPacked C;
  __device__ void init(const FieldK& F) {
    s0 = s1 = 0;
    tot = 0;
    C = zech_packed_constants(F);
  }
  __device__ __forceinline__ void term2(uint32_t aw, uint32_t bw) {
    uint32_t S, Sq, t, t2, mn, m1, mp;
    FD_PK("v_pk_add_u16", S, aw, bw);
    FD_PKS("v_pk_sub_u16", Sq, S, C.qq);
    FD_PK("v_pk_min_u16", t, S, Sq);        // (a + b) mod q', in [0, q']
    FD_PK("v_pk_add_u16", t2, t, t);        // byte offsets of the two values
    FD_PK("v_pk_min_u16", mn, aw, bw);
    FD_PKS("v_pk_min_u16", m1, mn, C.k1);
    FD_PKNEG(mp, m1);                       // ones where the product is nonzero
    const char* tb = (const char*)tab;
    const uint32_t vw = ((uint32_t)*(const uint16_t*)(tb + (t2 & 0xFFFFu)) |
                         ((uint32_t)*(const uint16_t*)(tb + (t2 >> 16)) << 16)) & mp;
    s0 += vw & 0xFFFFu;
    s1 += vw >> 16;
  }
  __device__ void vec(const u32x4& a, const u32x4& b, const FieldK&) {
    term2(a.x, b.x);
    term2(a.y, b.y);
    term2(a.z, b.z);
    term2(a.w, b.w);
  }
  __device__ void fold(const FieldK&) {
    tot += (uint64_t)s0 + s1;
    s0 = s1 = 0;
  }
  __device__ void one(E a, E b, const FieldK&, const Job&) {
    term2(a, b);  // high halves: zero codes, masked
    tot += (uint64_t)s0 + s1;
    s0 = s1 = 0;
  }
  __device__ uint32_t finish(const FieldK& F) { return mod_u64(tot + s0 + s1, F); }
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
  static constexpr bool kPrefetch = true;
  static constexpr bool kEntry0 = true;
  // running forms of zech_acc1 (code - 1, zero as 0xFFFFFFFF)
  uint32_t z[8];
  const uint16_t* tab;  // plus-one table in LDS, entry 0 = entry q'
  __device__ void init(const FieldK&) {
#pragma unroll
    for (int j = 0; j < 8; ++j) z[j] = 0xFFFFFFFFu;
  }
  __device__ void term(int j, uint32_t a, uint32_t b, const FieldK& F) {
    z[j] = zech_acc1(z[j], a, b, tab, F.qbar);
  }
  __device__ void vec(const u32x4& a, const u32x4& b, const FieldK& F) {
    const uint32_t ca[8] = {lo16(a.x), hi16(a.x), lo16(a.y), hi16(a.y),
                            lo16(a.z), hi16(a.z), lo16(a.w), hi16(a.w)};
    const uint32_t cb[8] = {lo16(b.x), hi16(b.x), lo16(b.y), hi16(b.y),
                            lo16(b.z), hi16(b.z), lo16(b.w), hi16(b.w)};
    zech_acc1_x8(z, ca, cb, tab, F.qbar);  // the eight table reads overlap
  }
  __device__ void one(E a, E b, const FieldK& F, const Job&) { term(0, a, b, F); }
  __device__ uint32_t finish(const FieldK& F) {
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += F.zval[z[j] + 1u];  // stored codes (0xFFFFFFFF -> 0)
    return mod_u64(s, F);
  }
  __device__ static void store(void* out, uint64_t k, uint32_t r, const FieldK& F) {
    ((uint16_t*)out)[k] = F.zidx[r];
  }
};

// The same Zech addition for p <= 32768 with two accumulators per register:
// the packed step of zech_packed.h (index arithmetic of two codes per 16-bit
// instruction, the zero element by bit masks) on a plus-one table with a mark
// where 1 + g^k = 0; the accumulators stay in the step's running form.
struct PZechTplus1P {
  using E = uint16_t;
  static constexpr int VW = 8;
  static constexpr int U = 2;
  static constexpr bool kTable = true;
  static constexpr bool kPrefetch = true;
  static constexpr bool kPackedPlus1 = true;
  static constexpr bool kStepVecs = true;
  // accumulators in the running form of zech_acc2 (code - 1, zero as
  // 0xFFFF), two per register; one set of 8 per vector of a step, so that
  // the U vectors' dependent table reads overlap
  uint32_t z[4 * U];
  uint32_t zt;     // accumulator of the scalar head and tail
  const uint16_t* tab;
  ZechPacked C;
  __device__ void init(const FieldK& F) {
#pragma unroll
    for (int j = 0; j < 4 * U; ++j) z[j] = 0xFFFFFFFFu;
    zt = 0xFFFFFFFFu;
    C = zech_packed_constants(F);
  }
  __device__ __forceinline__ uint32_t step(uint32_t zv, uint32_t aw, uint32_t bw) const {
    return zech_acc2(zv, aw, bw, (const char*)tab, C);
  }
  __device__ void vec(const u32x4& a, const u32x4& b, const FieldK&) {
    z[0] = step(z[0], a.x, b.x);
    z[1] = step(z[1], a.y, b.y);
    z[2] = step(z[2], a.z, b.z);
    z[3] = step(z[3], a.w, b.w);
  }
  __device__ void vecs(const u32x4* a, const u32x4* b, const FieldK&) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      z[4 * u + 0] = step(z[4 * u + 0], a[u].x, b[u].x);
      z[4 * u + 1] = step(z[4 * u + 1], a[u].y, b[u].y);
      z[4 * u + 2] = step(z[4 * u + 2], a[u].z, b[u].z);
      z[4 * u + 3] = step(z[4 * u + 3], a[u].w, b[u].w);
    }
  }
  __device__ void one(E a, E b, const FieldK&, const Job&) {
    zt = step(zt, a, b);  // low half only: the high half adds zero and stays zero
  }
  // stored code of a running form: v + 1 (0xFFFF -> 0)
  __device__ static uint32_t code(uint32_t v) { return (v + 1) & 0xFFFFu; }
  __device__ uint32_t finish(const FieldK& F) {
    uint32_t s = F.zval[code(zt)];
#pragma unroll
    for (int j = 0; j < 4 * U; ++j) s += F.zval[code(z[j])] + F.zval[code(z[j] >> 16)];
    return mod_u64(s, F);
  }
  __device__ static void store(void* out, uint64_t k, uint32_t r, const FieldK& F) {
    ((uint16_t*)out)[k] = F.zidx[r];
  }
};

// The table a table policy stages in LDS: the value table, the plus-one
// table, or for the packed policy its plus-one table with the zero mark.
template <class Pol, class = void>
struct PackedPlus1 { static constexpr bool value = false; };
template <class P>
struct PackedPlus1<P, decltype((void)P::kPackedPlus1)> { static constexpr bool value = P::kPackedPlus1; };

// A policy whose staged plus-one table has entry q' copied to entry 0.
template <class Pol, class = void>
struct Entry0 { static constexpr bool value = false; };
template <class P>
struct Entry0<P, decltype((void)P::kEntry0)> { static constexpr bool value = P::kEntry0; };

template <class Pol>
__device__ __forceinline__ const uint16_t* table_source(const FieldK& F) {
  if constexpr (std::is_same<Pol, PZechExp>::value || std::is_same<Pol, PZechExpP>::value)
    return F.zval;
  if constexpr (PackedPlus1<Pol>::value) return F.zpk;
  return F.zplus1;
}

// Centred residues in int8 (Sec. 3.2.2): four-way int8 dot products into a
// 32-bit accumulator, flushed to 64 bits every lambda_i32c products.
struct PCentred {
  using E = int8_t;
  static constexpr int VW = 16;
  static constexpr int U = FDOT_UNROLL;
  static constexpr bool kFolds = true;
  int32_t a;
  int64_t acc;
  __device__ void init(const FieldK&) { a = 0; acc = 0; }
  __device__ void vec(const u32x4& x, const u32x4& y, const FieldK&) {
    a = __builtin_amdgcn_sdot4((int)x.x, (int)y.x, a, false);
    a = __builtin_amdgcn_sdot4((int)x.y, (int)y.y, a, false);
    a = __builtin_amdgcn_sdot4((int)x.z, (int)y.z, a, false);
    a = __builtin_amdgcn_sdot4((int)x.w, (int)y.w, a, false);
  }
  __device__ void fold(const FieldK&) {
    acc += a;
    a = 0;
  }
  __device__ void one(E x, E y, const FieldK&, const Job&) { acc += (int32_t)x * (int32_t)y; }
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

template <class P, class = void>
struct Prefetch { static constexpr bool value = false; };
template <class P>
struct Prefetch<P, decltype((void)P::kPrefetch)> { static constexpr bool value = P::kPrefetch; };

// A policy that takes all U vectors of a step at once (vecs), e.g. to keep
// one accumulator set per vector.
template <class P, class = void>
struct StepVecs { static constexpr bool value = false; };
template <class P>
struct StepVecs<P, decltype((void)P::kStepVecs)> { static constexpr bool value = P::kStepVecs; };

template <class P, class = void>
struct Folds { static constexpr bool value = false; };
template <class P>
struct Folds<P, decltype((void)P::kFolds)> { static constexpr bool value = P::kFolds; };

// --------------------------------------------------------------- the driver

// Sixteen-byte-aligned zeros: the address that masked-off loads read, so
// that loads near the end of a range can be issued unconditionally.
__device__ const u32x4 g_zero16[2] = {{0u, 0u, 0u, 0u}, {0u, 0u, 0u, 0u}};

// One wavefront streams its slice of [x, x+len) against [y, y+len) through a
// lane policy.  The range is read as 1 KiB blocks (64 lanes x 16 bytes); slice
// s of S takes blocks s, s+S, s+2S, ..., so the S wavefronts working on one
// chunk sweep it together as one contiguous stream.  Slice 0 also takes a
// short scalar head that aligns both pointers to 16 bytes when they share the
// same offset, and the scalar tail, whose loads are issued with the first
// step; pointers with different offsets are read with scalar loads.  The last
// partial step is one masked step (lanes past the end read zeros), so the
// end of a range costs one memory latency.  A folding policy folds before any
// accumulator can have taken more than fold_vecs vectors: once per step when
// fold_vecs >= U, after every vector otherwise.
template <class Pol>
__device__ __forceinline__ void wave_range(Pol& L, const typename Pol::E* x,
                                           const typename Pol::E* y, uint64_t len,
                                           uint32_t lane, uint32_t slice, uint32_t S,
                                           const FieldK& F, const Job& J) {
  using E = typename Pol::E;
  constexpr int VW = Pol::VW, U = Pol::U, W = 64;
  constexpr bool kF = Folds<Pol>::value;
  const uint32_t fv = J.fold_vecs;
  const uintptr_t ax = (uintptr_t)x & 15u, ay = (uintptr_t)y & 15u;
  if (ax != ay) {
    for (uint64_t i = (uint64_t)slice * W + lane; i < len; i += (uint64_t)S * W)
      L.one(load_s(x + i), load_s(y + i), F, J);
    return;
  }
  uint64_t head = ax ? (16u - ax) / sizeof(E) : 0;
  if (head > len) head = len;
  if (slice == 0 && lane < head) L.one(load_s(x + lane), load_s(y + lane), F, J);
  const u32x4* xv = (const u32x4*)(x + head);
  const u32x4* yv = (const u32x4*)(y + head);
  const uint64_t nv = (len - head) / VW;
  const uint64_t t0 = head + nv * VW;
  // the scalar tail, loaded now and consumed at the end
  const bool has_tail = slice == 0 && lane < len - t0;
  const E tx = load_s(has_tail ? x + t0 + lane : (const E*)g_zero16);
  const E ty = load_s(has_tail ? y + t0 + lane : (const E*)g_zero16);
  const uint64_t step = (uint64_t)S * W;  // vectors from one block of this slice to the next
  uint64_t i = (uint64_t)slice * W + lane;
  uint32_t pending = 0;                   // vectors taken since the last fold
  if constexpr (Prefetch<Pol>::value) {
    // the next step's loads are issued before this step is consumed, so
    // that a policy with a long per-vector computation keeps its loads in
    // flight while it computes
    if (i + (uint64_t)(U - 1) * step < nv) {
      u32x4 a[U], b[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        a[u] = load_nt(xv + i + (uint64_t)u * step);
        b[u] = load_nt(yv + i + (uint64_t)u * step);
      }
      for (;;) {
        const uint64_t in = i + (uint64_t)U * step;
        const bool more = in + (uint64_t)(U - 1) * step < nv;
        u32x4 an[U], bn[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          an[u] = load_nt(more ? xv + in + (uint64_t)u * step : g_zero16);
          bn[u] = load_nt(more ? yv + in + (uint64_t)u * step : g_zero16);
        }
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (StepVecs<Pol>::value) {
          L.vecs(a, b, F);
        } else {
#pragma unroll
          for (int u = 0; u < U; ++u) L.vec(a[u], b[u], F);
        }
        if constexpr (kF) {
          pending += U;
          if (pending > fv - U) {
            L.fold(F);
            pending = 0;
          }
        }
        i = in;
        if (!more) break;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          a[u] = an[u];
          b[u] = bn[u];
        }
      }
    }
  } else if (!kF || fv >= (uint32_t)U) {
    for (; i + (uint64_t)(U - 1) * step < nv; i += (uint64_t)U * step) {
      u32x4 a[U], b[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        a[u] = load_nt(xv + i + (uint64_t)u * step);
        b[u] = load_nt(yv + i + (uint64_t)u * step);
      }
      // issue every load of the step before consuming any of them
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < U; ++u) L.vec(a[u], b[u], F);
      if constexpr (kF) {
        pending += U;
        if (pending > fv - U) {
          L.fold(F);
          pending = 0;
        }
      }
    }
  } else {
    for (; i + (uint64_t)(U - 1) * step < nv; i += (uint64_t)U * step) {
      u32x4 a[U], b[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        a[u] = load_nt(xv + i + (uint64_t)u * step);
        b[u] = load_nt(yv + i + (uint64_t)u * step);
      }
      // issue every load of the step before consuming any of them
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        L.vec(a[u], b[u], F);
        if constexpr (kF) {
          if (++pending == fv) {
            L.fold(F);
            pending = 0;
          }
        }
      }
    }
  }
  // the last, partial step: fewer than U vectors are left for this lane
  if (i < nv) {
    const u32x4 zero = {0u, 0u, 0u, 0u};
    u32x4 a[U - 1], b[U - 1];
#pragma unroll
    for (int u = 0; u < U - 1; ++u) {
      const uint64_t idx = i + (uint64_t)u * step;
      a[u] = load_nt(idx < nv ? xv + idx : g_zero16);
      b[u] = load_nt(idx < nv ? yv + idx : g_zero16);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U - 1; ++u) {
      const bool ok = i + (uint64_t)u * step < nv;
      L.vec(ok ? a[u] : zero, ok ? b[u] : zero, F);
      if constexpr (kF) {
        if (++pending >= fv) {
          L.fold(F);
          pending = 0;
        }
      }
    }
  }
  if (has_tail) L.one(tx, ty, F, J);
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Copies the policy's table (p entries of 16 bits) into LDS, once per
// workgroup.
template <class Pol, int NTH>
__device__ __forceinline__ void load_table(const FieldK& F, uint16_t* s_tab) {
  fd_table_to_lds<NTH>(s_tab, table_source<Pol>(F), F.p32);
  if constexpr (Entry0<Pol>::value) {
    // the one-code step reads entry 0 for g^0, as entry q'
    if (threadIdx.x == 0) s_tab[0] = s_tab[F.qbar];
    __syncthreads();
  }
}

// Adds a unit's residue to its pair's combination word.  The returned old
// word is checked one unit later, so that the wavefront does not wait for the
// atomic before streaming its next unit; the wavefront that completes a pair
// stores its result.
template <class Pol>
struct Combiner {
  bool pending = false;
  uint64_t pk = 0, pnck = 0, pr = 0;
  unsigned long long pold = 0;
  __device__ __forceinline__ void settle(const FieldK& F, const Job& J) {
    if (pending && (pold >> 48) + 1 == pnck) {
      // Every other unit of that pair has been added: the word is ours.
      atomicExch(J.acc + pk, 0ull);
      Pol::store(J.results, pk, mod_u64((pold & kSumMask) + pr, F), F);
    }
    pending = false;
  }
  // lane 0 only
  __device__ __forceinline__ void add(uint64_t k, uint64_t nck, uint64_t wsum, const FieldK& F,
                                      const Job& J) {
    settle(F, J);
    pr = mod_u64(wsum, F);
    pold = atomicAdd(J.acc + k, (unsigned long long)(pr + kCountOne));
    pk = k;
    pnck = nck;
    pending = true;
  }
};

// Single form.  Every unit of one dot product adding to one word made the
// atomics queue on one address (about 12 ns each, serialised), which bounded
// a dot of a few hundred units.  Units are therefore spread over W words
// (unit u to word u mod W); the wavefront that completes a word adds that
// word's residue to word 0 and returns the word to zero; the wavefront that
// completes word 0 (W additions) stores the result.  W = 1 is the plain
// one-word combination.  Sums stay below 2^48: at most 65535 residues per
// word.
template <class Pol>
struct SpreadCombiner {
  bool pending = false;
  uint32_t pw = 0, pnck = 0;
  uint64_t pr = 0;
  unsigned long long pold = 0;
  __device__ __forceinline__ void settle(const FieldK& F, const Job& J, uint32_t W) {
    if (pending && (pold >> 48) + 1 == pnck) {
      const uint64_t r1 = mod_u64((pold & kSumMask) + pr, F);
      atomicExch(J.acc + pw, 0ull);
      if (W == 1) {
        Pol::store(J.results, 0, (uint32_t)r1, F);
      } else {
        const unsigned long long o2 = atomicAdd(J.acc, (unsigned long long)(r1 + kCountOne));
        if ((o2 >> 48) + 1 == W) {
          atomicExch(J.acc, 0ull);
          Pol::store(J.results, 0, mod_u64((o2 & kSumMask) + r1, F), F);
        }
      }
    }
    pending = false;
  }
  // lane 0 only; unit u of total, first-level words W
  __device__ __forceinline__ void add(uint32_t u, uint32_t total, uint32_t W, uint64_t wsum,
                                      const FieldK& F, const Job& J) {
    settle(F, J, W);
    const uint32_t j = u % W;
    pw = W == 1 ? 0u : (j + 1) * kSpreadStride;
    pnck = (total - j + W - 1) / W;  // units u' < total with u' mod W = j
    pr = mod_u64(wsum, F);
    pold = atomicAdd(J.acc + pw, (unsigned long long)(pr + kCountOne));
    pending = true;
  }
};

// Single form: unit u = slice (u mod S) of chunk (u / S), S = 2^slice_shift;
// consecutive waves of a workgroup take consecutive units, and the grid
// strides over the rest.
template <class Pol, int NTH>
__global__ __launch_bounds__(NTH) void dot_kernel(const FieldK F, const Job J) {
  using E = typename Pol::E;
  extern __shared__ uint16_t s_tab[];
  constexpr bool kTab = HasTable<Pol>::value;
  if constexpr (kTab) load_table<Pol, NTH>(F, s_tab);
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t sh = J.slice_shift;
  const uint32_t S = 1u << sh;
  const uint64_t cs = chunk_of(J.n, J.chunk, sh);
  const uint64_t total = ((J.n + cs - 1) / cs) << sh;
  const uint64_t wstride = (uint64_t)gridDim.x * (NTH / 64);
  const uint32_t W = J.spread <= 1 ? 1u : J.spread < total ? J.spread : (uint32_t)total;
  SpreadCombiner<Pol> C;
  for (uint64_t u = (uint64_t)blockIdx.x * (NTH / 64) + (threadIdx.x >> 6); u < total;
       u += wstride) {
    const uint64_t c = u >> sh;
    const uint32_t slice = (uint32_t)(u & (S - 1));
    const uint64_t beg = c * cs;
    const uint64_t len = J.n - beg < cs ? J.n - beg : cs;
    Pol L;
    L.init(F);
    if constexpr (kTab) L.tab = s_tab;
    wave_range<Pol>(L, (const E*)J.x + beg, (const E*)J.y + beg, len, lane, slice, S, F, J);
    const uint64_t wsum = wave_sum(L.finish(F));
    if (lane == 0) C.add((uint32_t)u, (uint32_t)total, W, wsum, F, J);
  }
  if (lane == 0) C.settle(F, J, W);
}

// Batched form.  The padded sequence [0, T) is cut into R ranges of Q
// elements (the last one shorter), dealt cyclically to G groups of S
// wavefronts: group g streams ranges g, g+G, g+2G, ..., each of its S
// wavefronts one interleaved slice.  Every group gets the same number of
// ranges (the plan picks Q so), and at any moment the groups work on
// neighbouring ranges, so the whole GPU sweeps one window of memory.

struct PairRef {
  uint64_t first;  // position in the padded sequence
  uint32_t units;
  fdot_desc_t d;
};

// Where a batch's plan lives: the tables written by plan_kernel, or the
// workgroup's own prefix sums in LDS (fused form, small batches).
struct PlanTables {
  const Job* J;
  __device__ __forceinline__ PairRef pair(uint64_t k) const {
    PairRef P;
    P.first = J->first[k];
    P.units = J->units[k];
    P.d = J->desc[k];
    return P;
  }
  __device__ __forceinline__ uint64_t start(uint64_t r, uint64_t) const { return J->start[r]; }
};

struct PlanLds {
  const Job* J;
  const uint64_t* pf;  // pf[k] = first[k], pf[count] = T
  uint64_t Q;
  uint32_t S;
  __device__ __forceinline__ PairRef pair(uint64_t k) const {
    PairRef P;
    P.first = pf[k];
    const uint64_t end = pf[k + 1];
    P.units = end > P.first ? (uint32_t)((end - 1) / Q - P.first / Q + 1) * S : 0u;
    P.d = J->desc[k];
    return P;
  }
  // the pair whose padded span holds lo: largest k with pf[k] <= lo
  __device__ __forceinline__ uint64_t start(uint64_t, uint64_t lo) const {
    uint64_t a = 0, b = J->count;
    while (a + 1 < b) {
      const uint64_t m = (a + b) >> 1;
      if (pf[m] <= lo) a = m; else b = m;
    }
    while (a + 1 < J->count && pf[a + 1] <= lo) ++a;
    return a;
  }
};

// Streams every piece of the padded sequence inside [lo, hi): pairs k, k+1,
// ... (P describes pair k) up to the first that begins at or after hi.  The
// next pair's descriptor is fetched while the current piece streams.
template <class Pol, class Src>
__device__ __forceinline__ void many_range(const FieldK& F, const Job& J, const Src& src,
                                           uint16_t* s_tab, uint64_t k, PairRef P, uint64_t lo,
                                           uint64_t hi, uint32_t lane, uint32_t slice, uint32_t S,
                                           Combiner<Pol>& C) {
  using E = typename Pol::E;
  while (P.first < hi) {
    const bool more = k + 1 < J.count;
    PairRef P2 = P;
    if (more) P2 = src.pair(k + 1);
    if (P.d.n) {
      const uint64_t a = P.first > lo ? P.first : lo;
      const uint64_t end = P.first + P.d.n;
      const uint64_t b = end < hi ? end : hi;
      Pol L;
      L.init(F);
      if constexpr (HasTable<Pol>::value) L.tab = s_tab;
      if (b > a)
        wave_range<Pol>(L, (const E*)P.d.x + (a - P.first), (const E*)P.d.y + (a - P.first), b - a,
                        lane, slice, S, F, J);
      const uint64_t wsum = wave_sum(L.finish(F));
      if (lane == 0) C.add(k, P.units, wsum, F, J);
    }
    if (!more) break;
    ++k;
    P = P2;
  }
}

// Range length and count of a batch of padded total T: a whole number of
// ranges per group, about q_target elements each, rounded up to a multiple
// of 64 so that a piece of a pair keeps the pair's alignment; at most
// max_ranges ranges (the longer Q then).
__host__ __device__ __forceinline__ void batch_ranges(uint64_t T, uint64_t groups,
                                                      uint64_t q_target, uint64_t max_ranges,
                                                      uint64_t* Q_out, uint64_t* R_out) {
  const uint64_t per_round = groups * (q_target < 64 ? 64 : q_target);
  uint64_t rounds = (T + per_round / 2) / per_round;
  if (rounds < 1) rounds = 1;
  const uint64_t slots = groups * rounds;
  uint64_t Q = ((T + slots - 1) / slots + 63) & ~63ull;
  if (Q == 0) Q = 64;
  if ((T + Q - 1) / Q > max_ranges) Q = ((T + max_ranges - 1) / max_ranges + 63) & ~63ull;
  *Q_out = Q;
  *R_out = (T + Q - 1) / Q;
}

// Batched kernel.  FUSED: the workgroup first builds the batch's prefix
// sums in LDS itself (batches of at most kFusedMax pairs), instead of
// reading the tables of a separate plan launch; workgroup 0 also writes
// the zero element of empty pairs.
constexpr uint32_t kFusedMax = 7680;  // LDS: (7680 + 1 + 256) x 8 bytes < 64 KiB

template <class Pol, int NTH, bool FUSED>
__global__ __launch_bounds__(NTH) void many_kernel(const FieldK F, const Job J) {
  extern __shared__ __align__(16) unsigned char s_raw[];
  uint16_t* s_tab = (uint16_t*)s_raw;
  if constexpr (HasTable<Pol>::value) load_table<Pol, NTH>(F, s_tab);
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t sh = J.slice_shift;
  const uint32_t S = 1u << sh;
  const uint32_t w = blockIdx.x * (NTH / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t G = J.groups;
  uint64_t T, Q, R;
  PlanLds lsrc;
  if constexpr (FUSED) {
    uint64_t* pf = (uint64_t*)s_raw;         // count + 1
    uint64_t* part = pf + J.count + 1;       // NTH
    const uint32_t t = threadIdx.x;
    for (uint64_t k = t; k < J.count; k += NTH) pf[k + 1] = (load_s(&J.desc[k].n) + 63) & ~63ull;
    if (t == 0) pf[0] = 0;
    __syncthreads();
    const uint64_t seg = (J.count + NTH - 1) / NTH;
    const uint64_t b = t * seg < J.count ? t * seg : J.count;
    const uint64_t e = b + seg < J.count ? b + seg : J.count;
    uint64_t run = 0;
    for (uint64_t k = b; k < e; ++k) {
      run += pf[k + 1];
      pf[k + 1] = run;
    }
    part[t] = run;
    __syncthreads();
    for (uint32_t o = 1; o < NTH; o <<= 1) {  // inclusive scan of the segment totals
      const uint64_t v = t >= o ? part[t - o] : 0;
      __syncthreads();
      part[t] += v;
      __syncthreads();
    }
    const uint64_t off = part[t] - run;
    for (uint64_t k = b; k < e; ++k) pf[k + 1] += off;
    __syncthreads();
    T = pf[J.count];
    batch_ranges(T, G, J.q_target, J.max_ranges, &Q, &R);
    if (blockIdx.x == 0) {
      for (uint64_t k = t; k < J.count; k += NTH)
        if (pf[k + 1] == pf[k]) {
          uint8_t* res = (uint8_t*)J.results + k * J.elem_bytes;
          for (uint32_t i = 0; i < J.elem_bytes; ++i) res[i] = 0;
        }
    }
    lsrc.J = &J;
    lsrc.pf = pf;
    lsrc.Q = Q;
    lsrc.S = S;
  } else {
    T = J.tq[0];
    Q = J.tq[1];
    R = J.tq[2];
  }
  uint64_t r = w >> sh;
  if (r >= R || r >= G) return;
  Combiner<Pol> C;
  auto run_ranges = [&](const auto& src) {
    // Two-deep prefetch over this group's ranges: while range r streams, the
    // first pair of range r+G is being described and the start of range
    // r+2G is being looked up.
    uint64_t k = src.start(r, r * Q);
    PairRef P = src.pair(k);
    uint64_t kn = r + G < R ? src.start(r + G, (r + G) * Q) : 0;
    for (;;) {
      const bool has_next = r + G < R;
      PairRef Pn = P;
      if (has_next) Pn = src.pair(kn);
      const uint64_t kn2 = r + 2 * G < R ? src.start(r + 2 * G, (r + 2 * G) * Q) : 0;
      const uint64_t lo = r * Q;
      const uint64_t hi = T - lo < Q ? T : lo + Q;
      many_range<Pol>(F, J, src, s_tab, k, P, lo, hi, lane, w & (S - 1), S, C);
      if (!has_next) break;
      r += G;
      k = kn;
      P = Pn;
      kn = kn2;
    }
  };
  if constexpr (FUSED) {
    run_ranges(lsrc);
  } else {
    PlanTables tsrc;
    tsrc.J = &J;
    run_ranges(tsrc);
  }
  if (lane == 0) C.settle(F, J);
}

// Plan of a batch (one workgroup).  first[k] = sum over j < k of n_j rounded
// up to a multiple of 64, T = first[count].  Q is T over a whole number of
// ranges per group (about q_target elements each), rounded up to a multiple
// of 64 so that a piece of a pair keeps the pair's alignment; R = ceil(T/Q),
// at most max_ranges (the longer Q then).  units[k] = S x (ranges meeting
// pair k's padded span); start[r] = the pair whose padded span holds r Q.
// Empty pairs get the zero element (all-zero bits in every representation)
// at once, since no unit will finish them.
constexpr int PLAN_NT = 1024;

__device__ __forceinline__ uint64_t pad64(uint64_t n) { return (n + 63) & ~63ull; }

__global__ __launch_bounds__(PLAN_NT) void plan_kernel(const fdot_desc_t* desc, uint64_t count,
                                                       uint32_t groups, uint32_t S,
                                                       uint64_t q_target, uint32_t max_ranges,
                                                       uint64_t* first, uint32_t* units,
                                                       uint32_t* start, uint64_t* tq,
                                                       void* results, uint32_t elem_bytes) {
  constexpr int kWaves = PLAN_NT / 64;
  constexpr int kRegs = 8;  // pairs per thread whose lengths stay in registers
  __shared__ uint64_t s_wave[kWaves];
  const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
  const uint64_t seg = (count + PLAN_NT - 1) / PLAN_NT;
  const uint64_t b = t * seg < count ? t * seg : count;
  const uint64_t e = b + seg < count ? b + seg : count;
  const bool in_regs = seg <= (uint64_t)kRegs;
  uint64_t pn[kRegs];
  uint64_t local = 0;
  if (in_regs) {
#pragma unroll
    for (int j = 0; j < kRegs; ++j) {  // independent loads, all in flight together
      pn[j] = b + j < e ? pad64(load_s(&desc[b + j].n)) : 0;
      local += pn[j];
    }
  } else {
    for (uint64_t k = b; k < e; ++k) local += pad64(load_s(&desc[k].n));
  }
  // inclusive scan of the segment totals: within each wavefront by shuffles,
  // then the wavefront totals through LDS (one barrier)
  unsigned long long incl = local;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long v = __shfl_up(incl, (unsigned)o, 64);
    if (lane >= (uint32_t)o) incl += v;
  }
  if (lane == 63) s_wave[w] = incl;
  __syncthreads();
  uint64_t T = 0, before = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    const uint64_t v = s_wave[i];
    before += (uint32_t)i < w ? v : 0;
    T += v;
  }
  uint64_t Q, R;
  batch_ranges(T, groups, q_target, max_ranges, &Q, &R);
  uint64_t run = before + incl - local;
  auto place = [&](uint64_t k, uint64_t n_pad) {
    first[k] = run;
    if (n_pad) {
      const uint64_t r0 = run / Q, r1 = (run + n_pad - 1) / Q;
      units[k] = (uint32_t)((r1 - r0 + 1) * S);
      for (uint64_t r = (run + Q - 1) / Q; r <= r1; ++r) start[r] = (uint32_t)k;
    } else {
      units[k] = 0;
      uint8_t* res = (uint8_t*)results + k * elem_bytes;
      for (uint32_t i = 0; i < elem_bytes; ++i) res[i] = 0;
    }
    run += n_pad;
  };
  if (in_regs) {
#pragma unroll
    for (int j = 0; j < kRegs; ++j)
      if (b + j < e) place(b + j, pn[j]);
  } else {
    for (uint64_t k = b; k < e; ++k) place(k, pad64(load_s(&desc[k].n)));
  }
  if (t == 0) {
    tq[0] = T;
    tq[1] = Q;
    tq[2] = R;
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
  if constexpr (kTab) {
    load_table<Pol, 256>(F, s_tab);
  }
  const uint64_t row = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= m) return;
  const uint32_t lane = threadIdx.x & 63u;
  Pol L;
  L.init(F);
  if constexpr (kTab) L.tab = s_tab;
  wave_range<Pol>(L, (const E*)A + row * lda, (const E*)x, n, lane, 0, 1, F, J);
  const uint64_t v = wave_sum(L.finish(F));
  if (lane == 0) Pol::store(y, row, mod_u64(v, F), F);
}

// y = A x, RB rows per wavefront: every 16-byte vector of x is loaded once
// for RB rows, so x's re-reads (from L2) cost 1/RB load per term instead of
// one.  The rows of one wavefront and the copy of x it reads share their
// 16-byte phase, so one head, one vector loop and one tail serve all RB rows.
// Row phases repeat with period P (P = 1 when a row is a whole number of
// 16-byte units): the rows of class c (r = c mod P) go RB at a time to a
// wavefront, which reads a copy of x placed at class c's phase (xbase +
// c xstride + phase); with P = 1 and x in phase, x itself.  Policies that
// fold do so once fold_vecs vectors have been added since the last fold, as
// in the dot product.
template <class Pol, int RB>
__global__ __launch_bounds__(256) void gemv_rows_kernel(const FieldK F, const Job J, uint64_t m,
                                                        uint64_t n, uint64_t lda, const void* A,
                                                        const void* x, void* y, uint32_t P,
                                                        const uint8_t* xbase, uint64_t xstride) {
  using E = typename Pol::E;
  constexpr int VW = Pol::VW, U = 2, W = 64;
  constexpr bool kF = Folds<Pol>::value;
  extern __shared__ uint16_t s_tab[];
  constexpr bool kTab = HasTable<Pol>::value;
  if constexpr (kTab) {
    load_table<Pol, 256>(F, s_tab);
  }
  const uint64_t wv = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const uint64_t c = wv % P, q = wv / P;
  const uint64_t r0 = c + (uint64_t)P * RB * q;  // rows r0 + P j, j < RB
  if (r0 >= m) return;
  const uint64_t rlast = c + (uint64_t)P * ((m - 1 - c) / P);  // last row of class c
  const uint32_t lane = threadIdx.x & 63u;
  const E* xs = P == 1 && xbase == nullptr
                    ? (const E*)x
                    : (const E*)(xbase + c * xstride +
                                 (((uintptr_t)A + c * lda * sizeof(E)) & 15u));
  const E* rows[RB];
  Pol L[RB];
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    // rows past the class's last repeat it; their sums are not stored
    const uint64_t r = r0 + (uint64_t)P * j <= rlast ? r0 + (uint64_t)P * j : rlast;
    rows[j] = (const E*)A + r * lda;
    L[j].init(F);
    if constexpr (kTab) L[j].tab = s_tab;
  }
  const uintptr_t ax = (uintptr_t)xs & 15u;
  uint64_t head = ax ? (16u - ax) / sizeof(E) : 0;
  if (head > n) head = n;
  if (lane < head) {
    const E xe = load_s(xs + lane);
#pragma unroll
    for (int j = 0; j < RB; ++j) L[j].one(load_s(rows[j] + lane), xe, F, J);
  }
  const u32x4* xv = (const u32x4*)(xs + head);
  const uint64_t nv = (n - head) / VW;
  const uint64_t t0 = head + nv * VW;
  const uint32_t fv = J.fold_vecs;
  uint32_t pending = 0;
  uint64_t i = lane;
  for (; i + (uint64_t)(U - 1) * W < nv; i += (uint64_t)U * W) {
    u32x4 b[U], a[RB][U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      b[u] = load_nt(xv + i + (uint64_t)u * W);
#pragma unroll
      for (int j = 0; j < RB; ++j) a[j][u] = load_nt((const u32x4*)(rows[j] + head) + i + (uint64_t)u * W);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int j = 0; j < RB; ++j) L[j].vec(a[j][u], b[u], F);
      if constexpr (kF) {
        if (++pending >= fv) {
#pragma unroll
          for (int j = 0; j < RB; ++j) L[j].fold(F);
          pending = 0;
        }
      }
    }
  }
  if (i < nv) {  // at most U - 1 = 1 vector left for this lane
    const u32x4 b = load_nt(xv + i);
#pragma unroll
    for (int j = 0; j < RB; ++j) L[j].vec(load_nt((const u32x4*)(rows[j] + head) + i), b, F);
    // at most fv vectors since the last fold: finish() folds the rest
  }
  if (lane < n - t0) {
    const E xe = load_s(xs + t0 + lane);
#pragma unroll
    for (int j = 0; j < RB; ++j) L[j].one(load_s(rows[j] + t0 + lane), xe, F, J);
  }
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    const uint64_t v = wave_sum(L[j].finish(F));
    const uint64_t r = r0 + (uint64_t)P * j;
    if (lane == 0 && r <= rlast) Pol::store(y, r, mod_u64(v, F), F);
  }
}

// Copies of x at the 16-byte phase of each row class c < P (gridDim.y = P).
template <typename E>
__global__ void x_phase_copies_kernel(const E* x, uint64_t n, uint8_t* xbase, uint64_t xstride,
                                      uintptr_t a_addr, uint64_t row_bytes) {
  const uint64_t c = blockIdx.y;
  E* dst = (E*)(xbase + c * xstride + ((a_addr + c * row_bytes) & 15u));
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
    dst[i] = x[i];
}

// ---------------------------------------------------------------- launching
enum class Kind {
  ZpzDelayed, ZpzPerTerm, ZpzOverflow, ZpzHybrid, MontDelayed, MontPerTerm, MontOverflow,
  MontHybrid, F64, ZechExp, ZechExpP, ZechTplus1, ZechTplus1P, Centred
};

// Sec. 3.4, Eq. 2 (strict reading): largest lambda with lambda p (p-1) < 2^64.
static uint64_t hybrid_lambda(uint64_t p) {
  const unsigned __int128 pp = (unsigned __int128)p * (p - 1);
  if (pp == 0) return ~0ull;
  const unsigned __int128 l = (~(unsigned __int128)0 >> 64) / pp;
  return l > ~0ull ? ~0ull : (uint64_t)l;
}

struct Plan {
  Kind kind;
  uint32_t fold_vecs;
  size_t lds;
};

static uint32_t clamp_vecs(uint64_t v) {
  return v == 0 ? 1u : (v > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)v);
}

// Choose the lane policy and its fold period from the field's block lengths.
static fdot_status_t make_plan_lambda(const fdot_field_s* f, fdot_algo_t algo, Plan* pl) {
  const fdot_field_info_t& I = f->info;
  if (algo == FDOT_ALGO_AUTO) algo = fd_default_algo(f, 0);
  pl->fold_vecs = 0xFFFFFFFFu;
  pl->lds = 0;
  switch (I.rep) {
    case FDOT_REP_ZPZ_U32:
      if (algo == FDOT_ALGO_OVERFLOW || (algo == FDOT_ALGO_HYBRID && hybrid_lambda(I.p) < 2)) {
        pl->kind = Kind::ZpzOverflow;
        return FDOT_OK;
      }
      if (algo == FDOT_ALGO_HYBRID) {
        pl->kind = Kind::ZpzHybrid;
        pl->fold_vecs = clamp_vecs(hybrid_lambda(I.p) / 2);  // two products per vector per sum
        return FDOT_OK;
      }
      if (algo == FDOT_ALGO_PERTERM || (algo == FDOT_ALGO_DELAYED && I.lambda_u64 < 2)) {
        pl->kind = Kind::ZpzPerTerm;
        return FDOT_OK;
      }
      if (algo != FDOT_ALGO_DELAYED) return FDOT_E_UNSUPPORTED;
      pl->kind = Kind::ZpzDelayed;
      pl->fold_vecs = clamp_vecs(I.lambda_u64 / 2);  // two products per vector per accumulator
      return FDOT_OK;
    case FDOT_REP_MONT_U32:
      if (algo == FDOT_ALGO_OVERFLOW || (algo == FDOT_ALGO_HYBRID && hybrid_lambda(I.p) < 2)) {
        pl->kind = Kind::MontOverflow;
        return FDOT_OK;
      }
      if (algo == FDOT_ALGO_HYBRID) {
        pl->kind = Kind::MontHybrid;
        pl->fold_vecs = clamp_vecs(hybrid_lambda(I.p) / 2);
        return FDOT_OK;
      }
      if (algo == FDOT_ALGO_PERTERM || (algo == FDOT_ALGO_DELAYED && I.lambda_redc < 2)) {
        pl->kind = Kind::MontPerTerm;
        return FDOT_OK;
      }
      if (algo != FDOT_ALGO_DELAYED) return FDOT_E_UNSUPPORTED;
      pl->kind = Kind::MontDelayed;
      pl->fold_vecs = clamp_vecs(I.lambda_redc / 2);
      return FDOT_OK;
    case FDOT_REP_FP64:
      if (algo != FDOT_ALGO_DELAYED && algo != FDOT_ALGO_PERTERM) return FDOT_E_UNSUPPORTED;
      pl->kind = Kind::F64;
      pl->fold_vecs = algo == FDOT_ALGO_PERTERM ? 1u : clamp_vecs(I.lambda_f64);
      return FDOT_OK;
    case FDOT_REP_ZECH_U16:
      pl->lds = (size_t)I.p * 2;
      if (algo == FDOT_ALGO_ZECH_TPLUS1) {
        // two codes per packed 16-bit instruction where a sum of two codes
        // fits 16 bits (tune key zech.packed = 0 keeps one code per lane)
        const bool packed = I.p <= 32768 && fd_tune("zech.packed", 1) != 0;
        pl->kind = packed ? Kind::ZechTplus1P : Kind::ZechTplus1;
        return FDOT_OK;
      }
      if (algo != FDOT_ALGO_ZECH_EXP) return FDOT_E_UNSUPPORTED;
      pl->kind = I.p <= 32768 && fd_tune("zech.packed", 1) != 0 ? Kind::ZechExpP : Kind::ZechExp;
      // each 32-bit sum takes four values below p per vector
      pl->fold_vecs = clamp_vecs(0xFFFFFFFFull / (4 * (I.p - 1)));
      return FDOT_OK;
    case FDOT_REP_CENTRED_I8:
      if (algo != FDOT_ALGO_DELAYED) return FDOT_E_UNSUPPORTED;
      if (I.lambda_i32c < 16) return FDOT_E_UNSUPPORTED;
      pl->kind = Kind::Centred;
      pl->fold_vecs = clamp_vecs(I.lambda_i32c / 16);  // sixteen products per vector
      return FDOT_OK;
  }
  return FDOT_E_UNSUPPORTED;
}

// The plan, with the field's block option applied: a delayed schedule folds
// after at most block products per accumulator (products per vector and
// accumulator: two for 32-bit residues, one for doubles, four discrete-log
// values per sum, sixteen centred int8 products), whole vectors, at least
// one.  A shorter block only folds more often, so exactness is kept.
static fdot_status_t make_plan(const fdot_field_s* f, fdot_algo_t algo, Plan* pl) {
  const fdot_status_t st = make_plan_lambda(f, algo, pl);
  if (st != FDOT_OK || f->opt.block == 0 || pl->fold_vecs == 0xFFFFFFFFu) return st;
  uint64_t per = 2;
  switch (pl->kind) {
    case Kind::F64: per = 1; break;
    case Kind::ZechExp:
    case Kind::ZechExpP: per = 4; break;
    case Kind::Centred: per = 16; break;
    default: break;
  }
  uint64_t v = f->opt.block / per;
  if (v < 1) v = 1;
  if (v < pl->fold_vecs) pl->fold_vecs = (uint32_t)v;
  return FDOT_OK;
}

// Workgroups of `fn` that can be resident on one CU with `lds` bytes of
// dynamic LDS (cached).  Grids are clamped to CUs x this: a larger grid would
// leave a second, short wave of workgroups at the end.
static int resident_per_cu(const void* fn, int nth, size_t lds) {
  static std::mutex mu;
  static std::map<std::pair<const void*, size_t>, int> cache;
  std::lock_guard<std::mutex> g(mu);
  auto key = std::make_pair(fn, lds);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  if (lds > 65536)
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, nth, lds) != hipSuccess || nb < 1) nb = 1;
  cache[key] = nb;
  return nb;
}

struct Launch {
  FieldK F;
  Job J;
  bool many;
  uint64_t work_waves;  // single form: units to cover
  unsigned wg_per_cu;
  size_t lds;
  hipStream_t s;
  const Workspace* ws;  // batched form
  uint32_t max_groups;  // batched form: most groups of S wavefronts
  uint64_t range;       // batched form: elements per range (target)
  uint32_t fused;       // batched form: largest batch planned inside the kernel
  uint32_t elem_bytes;
};

template <class Pol, int NTH>
static fdot_status_t launch_t(Launch A) {
  constexpr int WPW = NTH / 64;
  const bool fused = A.many && !HasTable<Pol>::value && A.J.count <= A.fused;
  const size_t lds = fused ? (size_t)(A.J.count + 1 + NTH) * sizeof(uint64_t) : A.lds;
  const void* fn = !A.many ? (const void*)dot_kernel<Pol, NTH>
                   : fused ? (const void*)many_kernel<Pol, NTH, true>
                           : (const void*)many_kernel<Pol, NTH, false>;
  unsigned per_cu = (unsigned)resident_per_cu(fn, NTH, (lds + 8191) & ~(size_t)8191);
  if (A.wg_per_cu < per_cu) per_cu = A.wg_per_cu;
  uint64_t grid = (uint64_t)fd_cu_count() * per_cu;
  if (!A.many) {
    const uint64_t need = (A.work_waves + WPW - 1) / WPW;
    if (need < grid) grid = need;
    if (grid < 1) grid = 1;
    const int tr = fd_trace_begin(A.s);
    hipLaunchKernelGGL((dot_kernel<Pol, NTH>), dim3((unsigned)grid), dim3(NTH), A.lds, A.s, A.F,
                       A.J);
    fd_trace_end(A.s, tr);
    return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
  }
  // Groups of S resident wavefronts; a pair meets at most R ranges, so
  // S x R must fit the 16-bit unit count of its combination word.
  const uint32_t S = 1u << A.J.slice_shift;
  uint64_t groups = grid * WPW / S;
  if (groups > A.max_groups) groups = A.max_groups;
  if (groups < 1) groups = 1;
  grid = (groups * S + WPW - 1) / WPW;
  uint64_t max_ranges = kMaxUnits / S;
  if (max_ranges > kMaxRanges) max_ranges = kMaxRanges;
  if (max_ranges < groups) max_ranges = groups;  // S x groups <= resident waves < 2^16
  Job J = A.J;
  J.first = A.ws->first;
  J.units = A.ws->units;
  J.start = A.ws->start;
  J.tq = A.ws->tq;
  J.q_target = A.range;
  J.groups = (uint32_t)groups;
  J.max_ranges = (uint32_t)max_ranges;
  if (fused) {
    const int tr = fd_trace_begin(A.s);
    hipLaunchKernelGGL((many_kernel<Pol, NTH, true>), dim3((unsigned)grid), dim3(NTH), lds, A.s,
                       A.F, J);
    fd_trace_end(A.s, tr);
  } else {
    hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(PLAN_NT), 0, A.s, J.desc, J.count,
                       (uint32_t)groups, S, A.range, (uint32_t)max_ranges, A.ws->first,
                       A.ws->units, A.ws->start, A.ws->tq, J.results, A.elem_bytes);
    if (hipGetLastError() != hipSuccess) return FDOT_E_DEVICE;
    const int tr = fd_trace_begin(A.s);
    hipLaunchKernelGGL((many_kernel<Pol, NTH, false>), dim3((unsigned)grid), dim3(NTH), A.lds,
                       A.s, A.F, J);
    fd_trace_end(A.s, tr);
  }
  return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
}

static fdot_status_t dispatch(const Plan& pl, const Launch& A0) {
  Launch A = A0;
  A.lds = pl.lds;
  switch (pl.kind) {
    case Kind::ZpzDelayed: return launch_t<PZpzDelayed, 256>(A);
    case Kind::ZpzPerTerm: return launch_t<PZpzPerTerm, 256>(A);
    case Kind::ZpzOverflow: return launch_t<POverflow<false>, 256>(A);
    case Kind::ZpzHybrid: return launch_t<PHybrid<false>, 256>(A);
    case Kind::MontHybrid: return launch_t<PHybrid<true>, 256>(A);
    case Kind::MontDelayed: return launch_t<PMontDelayed, 256>(A);
    case Kind::MontPerTerm: return launch_t<PMontPerTerm, 256>(A);
    case Kind::MontOverflow: return launch_t<POverflow<true>, 256>(A);
    case Kind::F64: return launch_t<PF64, 256>(A);
    case Kind::ZechExp: return launch_t<PZechExp, 1024>(A);
    case Kind::ZechTplus1: return launch_t<PZechTplus1, 1024>(A);
    case Kind::ZechTplus1P: return launch_t<PZechTplus1P, 1024>(A);
    case Kind::ZechExpP: return launch_t<PZechExpP, 1024>(A);
    case Kind::Centred: return launch_t<PCentred, 256>(A);
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

// Launch parameters from the tuning table.  slices.<rep>: wavefronts that
// share one chunk of the single form (1, 2, 4 or 8); many.slices.<rep>: the
// same for one range of the batched form (default 1);
// many.groups.<rep>: most groups of the batched form (default: all resident
// wavefronts / S); many.range.<rep>: bytes per operand of one range (default
// 512 KiB); many.fused.<rep>: largest batch whose plan is built inside the
// batched kernel (default 512, at most 7680; larger batches get a separate
// plan launch); chunk.<rep>: largest chunk of the single form (default 1
// MiB per operand); min_chunk.<rep>: smallest chunk of the single form, which
// otherwise spreads a vector over every resident wavefront; spread.<rep>:
// first-level combination words of the single form (default 32, at most
// 64); wg_per_cu.<rep>: workgroups per CU (further clamped by residency).
struct Shape {
  uint64_t chunk;
  unsigned wg_per_cu;
  int waves_per_wg;
  uint32_t slice_shift;
  uint32_t max_groups;
  uint64_t range;
  uint32_t fused;  // largest batch planned inside the kernel (0: never)
  uint32_t spread;  // single form: first-level combination words
};

static uint32_t log2_slices(int64_t sl) { return sl >= 8 ? 3 : sl >= 4 ? 2 : sl >= 2 ? 1 : 0; }

static Shape shape_for(const fdot_field_s* f, uint64_t n_single) {
  char key[64];
  const char* r = rep_key(f->info.rep);
  const bool zech = f->info.rep == FDOT_REP_ZECH_U16;
  const uint64_t eb = f->info.elem_bytes;
  Shape sh;
  sh.waves_per_wg = zech ? 16 : 4;
  snprintf(key, sizeof key, "wg_per_cu.%s", r);
  int64_t wpc = fd_tune(key, 2);
  sh.wg_per_cu = (unsigned)(wpc < 1 ? 1 : wpc);
  sh.max_groups = kMaxRanges;
  sh.range = 0;
  sh.fused = 0;
  sh.chunk = 0;
  snprintf(key, sizeof key, "spread.%s", r);
  const int64_t sp = fd_tune(key, 32);
  sh.spread = (uint32_t)(sp < 1 ? 1 : sp > (int64_t)kSpreadMax ? kSpreadMax : sp);
  if (!n_single) {
    snprintf(key, sizeof key, "many.slices.%s", r);
    sh.slice_shift = log2_slices(fd_tune(key, 1));
    snprintf(key, sizeof key, "many.groups.%s", r);
    const int64_t mg = fd_tune(key, (int64_t)kMaxRanges);
    sh.max_groups = (uint32_t)(mg < 1 ? 1 : mg > (int64_t)kMaxRanges ? kMaxRanges : mg);
    snprintf(key, sizeof key, "many.range.%s", r);
    const int64_t rb = fd_tune(key, 524288);
    sh.range = (uint64_t)(rb < 64 ? 64 : rb) / eb;
    snprintf(key, sizeof key, "many.fused.%s", r);
    const int64_t fz = fd_tune(key, 512);
    sh.fused = (uint32_t)(fz < 0 ? 0 : fz > (int64_t)kFusedMax ? kFusedMax : fz);
    return sh;
  }
  snprintf(key, sizeof key, "slices.%s", r);
  sh.slice_shift = log2_slices(fd_tune(key, 1));
  snprintf(key, sizeof key, "chunk.%s", r);
  int64_t chunk = fd_tune(key, (int64_t)(1048576 / eb));
  snprintf(key, sizeof key, "min_chunk.%s", r);
  int64_t mn = fd_tune(key, (int64_t)(4096 / eb));
  const uint64_t waves = (uint64_t)fd_cu_count() * sh.wg_per_cu * sh.waves_per_wg;
  const int64_t spread = (int64_t)((n_single + waves - 1) / waves);
  chunk = spread < chunk ? spread : chunk;
  if (chunk < mn) chunk = mn;
  chunk = (chunk + 15) / 16 * 16;
  if (chunk < 64) chunk = 64;
  sh.chunk = (uint64_t)chunk;
  return sh;
}

}  // namespace

fdot_algo_t fd_default_algo(const fdot_field_s* f, uint64_t) {
  const fdot_field_info_t& I = f->info;
  if (f->opt.algo != FDOT_ALGO_AUTO) return (fdot_algo_t)f->opt.algo;  // creation option
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
  const Shape sh = shape_for(f, n);
  Plan pl;
  fdot_status_t st = make_plan(f, algo, &pl);
  if (st != FDOT_OK) return st;
  Launch A;
  memset(&A, 0, sizeof A);
  A.F = f->k;
  A.J.x = x;
  A.J.y = y;
  A.J.n = n;
  A.J.chunk = sh.chunk;
  A.J.acc = ws->acc;
  A.J.results = result;
  A.J.fold_vecs = pl.fold_vecs;
  A.J.slice_shift = sh.slice_shift;
  A.J.spread = sh.spread;
  while (A.J.spread > 1 && (uint64_t)(A.J.spread + 1) * kSpreadStride > ws->cap) A.J.spread >>= 1;
  A.many = false;
  const uint64_t cs = chunk_of(n, sh.chunk, sh.slice_shift);
  A.work_waves = ((n + cs - 1) / cs) << sh.slice_shift;
  A.wg_per_cu = sh.wg_per_cu;
  A.s = s;
  return dispatch(pl, A);
}

fdot_status_t fd_launch_many(const fdot_field_s* f, fdot_algo_t algo, size_t count,
                             const fdot_desc_t* desc, void* results, Workspace* ws,
                             hipStream_t s) {
  if (count == 0) return FDOT_OK;
  const Shape sh = shape_for(f, 0);
  Plan pl;
  fdot_status_t st = make_plan(f, algo, &pl);
  if (st != FDOT_OK) return st;
  Launch A;
  memset(&A, 0, sizeof A);
  A.F = f->k;
  A.J.desc = desc;
  A.J.count = count;
  A.J.acc = ws->acc;
  A.J.results = results;
  A.J.fold_vecs = pl.fold_vecs;
  A.J.slice_shift = sh.slice_shift;
  A.many = true;
  A.wg_per_cu = sh.wg_per_cu;
  A.s = s;
  A.ws = ws;
  A.max_groups = sh.max_groups;
  A.range = sh.range;
  A.fused = sh.fused;
  A.elem_bytes = f->info.elem_bytes;
  A.J.elem_bytes = f->info.elem_bytes;
  return dispatch(pl, A);
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
static fdot_status_t launch_gemv_t(const fdot_field_s* f, const Job& J0, size_t m, size_t n,
                                   const void* A, size_t lda, const void* x, void* y, size_t lds,
                                   hipStream_t s) {
  // Rows go four to a wavefront, each wavefront's rows of one 16-byte phase
  // class, reading x itself when every row is in phase with it and otherwise
  // a copy of x per class (tune key gemv.rows = 1 keeps one wavefront per
  // row).
  const uint64_t eb = sizeof(typename Pol::E);
  const bool folds_ok = !Folds<Pol>::value || J0.fold_vecs >= 1;
  if (folds_ok && n >= 256 && fd_tune("gemv.rows", 4) == 4) {
    const uint64_t d = (lda * eb) % 16;
    const uint32_t P = d == 0 ? 1u : 16u / (uint32_t)(d & (~d + 1));  // 16 / gcd(d, 16)
    const uint8_t* xbase = nullptr;
    uint64_t xstride = 0;
    if (P > 1 || (uintptr_t)A % 16 != (uintptr_t)x % 16) {
      xstride = (n * eb + 16 + 255) & ~(uint64_t)255;
      void* scr = nullptr;
      fdot_status_t st = fd_scratch_get(s, (size_t)P * xstride, &scr);
      if (st != FDOT_OK) return st;
      xbase = (const uint8_t*)scr;
      const unsigned gx = (unsigned)std::min<uint64_t>((n + 255) / 256, 1024);
      hipLaunchKernelGGL(x_phase_copies_kernel<typename Pol::E>, dim3(gx, P), dim3(256), 0, s,
                         (const typename Pol::E*)x, (uint64_t)n, (uint8_t*)scr, xstride,
                         (uintptr_t)A, (uint64_t)(lda * eb));
      if (hipGetLastError() != hipSuccess) return FDOT_E_DEVICE;
    }
    auto fr = gemv_rows_kernel<Pol, 4>;
    if (lds > 65536)
      (void)hipFuncSetAttribute((const void*)fr, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
    const uint64_t per_class = ((m + P - 1) / P + 3) / 4;  // wavefronts per class
    const uint64_t waves = per_class * P;
    if ((waves + 3) / 4 > 0x7FFFFFFFull) return FDOT_E_INVALID_ARG;
    hipLaunchKernelGGL(fr, dim3((unsigned)((waves + 3) / 4)), dim3(256), lds, s, f->k, J0,
                       (uint64_t)m, (uint64_t)n, (uint64_t)lda, A, x, y, P, xbase, xstride);
    return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
  }
  const Job& J = J0;
  auto fn = gemv_kernel<Pol>;
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  hipLaunchKernelGGL(fn, dim3((unsigned)((m + 3) / 4)), dim3(256), lds, s, f->k, J, (uint64_t)m,
                     (uint64_t)n, (uint64_t)lda, A, x, y);
  return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
}

fdot_status_t fd_launch_gemv(const fdot_field_s* f, size_t m, size_t n, const void* A, size_t lda,
                             const void* x, void* y, hipStream_t s) {
  if (m == 0) return FDOT_OK;
  if ((m + 3) / 4 > 0x7FFFFFFFull) return FDOT_E_INVALID_ARG;
  Plan pl;
  fdot_algo_t algo = fd_default_algo(f, n);
  fdot_status_t st = make_plan(f, algo, &pl);
  if (st != FDOT_OK) return st;
  Job J;
  memset(&J, 0, sizeof J);
  J.fold_vecs = pl.fold_vecs;
  switch (pl.kind) {
    case Kind::ZpzDelayed: return launch_gemv_t<PZpzDelayed>(f, J, m, n, A, lda, x, y, 0, s);
    case Kind::ZpzPerTerm: return launch_gemv_t<PZpzPerTerm>(f, J, m, n, A, lda, x, y, 0, s);
    case Kind::ZpzOverflow: return launch_gemv_t<POverflow<false>>(f, J, m, n, A, lda, x, y, 0, s);
    case Kind::ZpzHybrid: return launch_gemv_t<PHybrid<false>>(f, J, m, n, A, lda, x, y, 0, s);
    case Kind::MontHybrid: return launch_gemv_t<PHybrid<true>>(f, J, m, n, A, lda, x, y, 0, s);
    case Kind::MontDelayed: return launch_gemv_t<PMontDelayed>(f, J, m, n, A, lda, x, y, 0, s);
    case Kind::MontPerTerm: return launch_gemv_t<PMontPerTerm>(f, J, m, n, A, lda, x, y, 0, s);
    case Kind::MontOverflow: return launch_gemv_t<POverflow<true>>(f, J, m, n, A, lda, x, y, 0, s);
    case Kind::F64: return launch_gemv_t<PF64>(f, J, m, n, A, lda, x, y, 0, s);
    case Kind::ZechExp: return launch_gemv_t<PZechExp>(f, J, m, n, A, lda, x, y, pl.lds, s);
    case Kind::ZechTplus1: return launch_gemv_t<PZechTplus1>(f, J, m, n, A, lda, x, y, pl.lds, s);
    case Kind::ZechTplus1P: return launch_gemv_t<PZechTplus1P>(f, J, m, n, A, lda, x, y, pl.lds, s);
    case Kind::ZechExpP: return launch_gemv_t<PZechExpP>(f, J, m, n, A, lda, x, y, pl.lds, s);
    case Kind::Centred: return launch_gemv_t<PCentred>(f, J, m, n, A, lda, x, y, 0, s);
  }
  return FDOT_E_UNSUPPORTED;
}

// Copy results[i] (elem_bytes each) to the output pointer dst[i]: used by the
// request server to hand each fused dot product its own output.
__global__ void scatter_kernel(const uint8_t* src, void* const* dst, uint64_t count, uint32_t eb) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint8_t* d = (uint8_t*)dst[i];
    for (uint32_t b = 0; b < eb; ++b) d[b] = src[i * eb + b];
  }
}

fdot_status_t fd_launch_scatter(const void* src, void* const* dst, size_t count, uint32_t elem_bytes,
                                hipStream_t s) {
  if (count == 0) return FDOT_OK;
  const unsigned blocks = (unsigned)((count + 255) / 256 < 1024 ? (count + 255) / 256 : 1024);
  hipLaunchKernelGGL(scatter_kernel, dim3(blocks), dim3(256), 0, s, (const uint8_t*)src, dst,
                     (uint64_t)count, elem_bytes);
  return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
}
