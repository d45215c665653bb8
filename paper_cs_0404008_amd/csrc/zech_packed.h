// Zech arithmetic on two discrete-logarithm codes per 32-bit register, for
// fields with q <= 32768 elements (Sec. 2.4, Table 1): every code then fits
// 15 bits and a sum of two codes fits 16, so the index arithmetic of two
// codes runs in one packed 16-bit instruction and the tests for the zero
// element become bit masks instead of per-code selects.
//
// Codes (as stored): 0 is the zero element, c in [1, q'] is g^c, q' = q - 1
// (q' itself codes g^0 = 1).  A running sum is held as v = code - 1 in
// [0, q' - 1], and the zero element as 0xFFFF (the stored code minus one,
// modulo 2^16).  zech_acc2(v, a, b) returns, per half, the running form of
// v + a b for codes a, b:
//  * product: s = a + b; its running form is (s - 1) mod q', the minimum of
//    s - 1 (saturating at 0) and s - 1 - q' in 16-bit wrap-around arithmetic;
//    a mask is all ones in each half where neither factor is zero;
//  * sum g^u + g^t = g^(u + h) with g^h = 1 + g^k, k = t - u: k is the
//    difference of the two running forms reduced the same way, the table
//    gives h (the code of 1 + g^k) or the mark 0xFFFF where 1 + g^k = 0, and
//    the running form of the sum is (v + h) mod q';
//  * the mark makes the result 0xFFFF (the sum is zero); a zero running sum
//    takes the product, a zero product leaves the running sum as it is.
// Every table index lies in [0, q'] (q' only for a zero running sum, whose
// lookup is discarded), so the table needs q entries.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fdot_arith.h"

// The packed 16-bit ALU instructions are written out one per statement (so
// that the compiler can still interleave independent chains): it otherwise
// turns the mask arithmetic back into per-half compares and selects.  They
// are pure register operations, no memory access.
#define FD_PK(op, d, a, b) asm(op " %0, %1, %2" : "=v"(d) : "v"(a), "v"(b))
// the same with a wave-uniform operand in a scalar register (second, or first)
#define FD_PKS(op, d, a, b) asm(op " %0, %1, %2" : "=v"(d) : "v"(a), "s"(b))
#define FD_PKS1(op, d, a, b) asm(op " %0, %1, %2" : "=v"(d) : "s"(a), "v"(b))
// 0 - a in both halves: all ones where a half is 1, zero where it is 0
#define FD_PKNEG(d, a) asm("v_pk_sub_u16 %0, 0, %1" : "=v"(d) : "v"(a))

typedef unsigned short fd_u16x2 __attribute__((ext_vector_type(2)));

// a - b per 16-bit half, saturating at 0 (the compiler's own saturating
// subtraction, one packed instruction).
__device__ __forceinline__ uint32_t fd_pk_sub_sat(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t,
                            __builtin_elementwise_sub_sat(__builtin_bit_cast(fd_u16x2, a),
                                                          __builtin_bit_cast(fd_u16x2, b)));
}

// Packed constants: 1, q' + 1, q' and 15 in both halves.
struct ZechPacked {
  uint32_t k1, q1, qq, f15;
};

__device__ __forceinline__ ZechPacked zech_packed_constants(const FieldK& F) {
  ZechPacked c;
  c.k1 = 0x00010001u;
  c.qq = F.qbar | (F.qbar << 16);
  c.q1 = (F.qbar + 1) | ((F.qbar + 1) << 16);
  c.f15 = 0x000F000Fu;
  return c;
}

// Copies n table entries from device memory into LDS (all threads of the
// workgroup, NTH of them), 16 bytes at a time when both sides are 16-byte
// aligned, and waits for the workgroup.
template <int NTH>
__device__ __forceinline__ void fd_table_to_lds(uint16_t* s, const uint16_t* g, uint32_t n) {
  uint32_t done = 0;
  if ((((uintptr_t)s | (uintptr_t)g) & 15u) == 0) {
    const uint32_t nv = n / 8;
    for (uint32_t i = threadIdx.x; i < nv; i += NTH) ((uint4*)s)[i] = ((const uint4*)g)[i];
    done = nv * 8;
  }
  for (uint32_t i = done + threadIdx.x; i < n; i += NTH) s[i] = g[i];
  __syncthreads();
}

// Running form v + a b per 16-bit half; tb: the packed step's plus-one
// table (FieldK::zpk, bytes, in LDS).
__device__ __forceinline__ uint32_t zech_acc2(uint32_t v, uint32_t aw, uint32_t bw,
                                              const char* tb, const ZechPacked& C) {
  uint32_t S, Sb, R, mn, m1, mp, D, Dq, K, K2, S1, S1q, Wm, hs, hz;
  FD_PK("v_pk_add_u16", S, aw, bw);
  const uint32_t Sa = fd_pk_sub_sat(S, C.k1);
  FD_PKS("v_pk_sub_u16", Sb, S, C.q1);
  FD_PK("v_pk_min_u16", R, Sa, Sb);        // product, running form
  FD_PK("v_pk_min_u16", mn, aw, bw);
  FD_PKS("v_pk_min_u16", m1, mn, C.k1);
  FD_PKNEG(mp, m1);                        // ones where the product is nonzero
  FD_PK("v_pk_sub_u16", D, R, v);
  FD_PKS("v_pk_add_u16", Dq, D, C.qq);
  FD_PK("v_pk_min_u16", K, D, Dq);         // k in [0, q']
  FD_PK("v_pk_add_u16", K2, K, K);         // byte offsets of the two table entries
  const uint32_t hw = (uint32_t)*(const uint16_t*)(tb + (K2 & 0xFFFFu)) |
                      ((uint32_t)*(const uint16_t*)(tb + (K2 >> 16)) << 16);
  FD_PK("v_pk_add_u16", S1, v, hw);
  FD_PKS("v_pk_sub_u16", S1q, S1, C.qq);
  FD_PK("v_pk_min_u16", Wm, S1, S1q);      // running form of the sum
  FD_PKS1("v_pk_ashrrev_i16", hs, C.f15, hw);  // ones where the sum is zero
  FD_PKS1("v_pk_ashrrev_i16", hz, C.f15, v);   // ones where the running sum is zero
  const uint32_t r1 = Wm | hs;
  const uint32_t r2 = (R & hz) | (r1 & ~hz);
  return (r2 & mp) | (v & ~mp);
}

// The same step on one code per 32-bit lane, for q <= 65536 (codes up to
// 65535, so no two share a register): running form v = code - 1, the zero
// element as 0xFFFFFFFF; tab is the plus-one table indexed by code with entry
// 0 replaced by entry q' (both stand for g^0 here), a zero entry marking
// 1 + g^k = 0.  Every index lies in [0, q'].
__device__ __forceinline__ uint32_t zech_acc1(uint32_t v, uint32_t a, uint32_t b,
                                              const uint16_t* tab, uint32_t qq) {
  const uint32_t S = a + b;
  const uint32_t Sa = __builtin_elementwise_sub_sat(S, 1u);
  const uint32_t R = min(Sa, S - (qq + 1));     // product, running form
  const uint32_t D = R - v;
  const uint32_t K = min(D, D + qq);
  const uint32_t h = tab[K];
  const uint32_t S1 = v + h;
  const uint32_t W = min(S1, S1 - qq);          // running form of the sum
  const uint32_t r1 = h == 0 ? 0xFFFFFFFFu : W;
  const uint32_t r2 = (int32_t)v < 0 ? R : r1;  // a zero running sum takes the product
  return (a == 0 || b == 0) ? v : r2;           // a zero product changes nothing
}

// Eight independent running forms v[j] + a[j] b[j] of zech_acc1 at once: the
// eight table indices first, then the eight table reads back to back, then
// the eight sums, so that the reads' latencies overlap instead of each sum
// waiting for its own read (the compiler otherwise keeps every step whole).
__device__ __forceinline__ void zech_acc1_x8(uint32_t (&v)[8], const uint32_t (&a)[8],
                                             const uint32_t (&b)[8], const uint16_t* tab,
                                             uint32_t qq) {
  uint32_t R[8], K[8], m[8], h[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const uint32_t S = a[j] + b[j];
    R[j] = min(__builtin_elementwise_sub_sat(S, 1u), S - (qq + 1));
    const uint32_t D = R[j] - v[j];
    K[j] = min(D, D + qq);
    m[j] = min(a[j], b[j]);  // 0 for a zero product
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int j = 0; j < 8; ++j) h[j] = tab[K[j]];
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const uint32_t S1 = v[j] + h[j];
    const uint32_t W = min(S1, S1 - qq);
    const uint32_t r1 = h[j] == 0 ? 0xFFFFFFFFu : W;
    const uint32_t r2 = (int32_t)v[j] < 0 ? R[j] : r1;
    v[j] = m[j] == 0 ? v[j] : r2;
  }
}

// Stored code z + a b per 16-bit half (codes in, code out).
__device__ __forceinline__ uint32_t zech_step2(uint32_t zw, uint32_t aw, uint32_t bw,
                                               const char* tb, const ZechPacked& C) {
  uint32_t v, out;
  FD_PKS("v_pk_sub_u16", v, zw, C.k1);
  const uint32_t r = zech_acc2(v, aw, bw, tb, C);
  FD_PKS("v_pk_add_u16", out, r, C.k1);
  return out;
}
