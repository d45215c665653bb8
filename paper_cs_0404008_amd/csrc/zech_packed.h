// Zech arithmetic on two discrete-logarithm codes per 32-bit register, for
// fields with q <= 32768 elements (Sec. 2.4, Table 1): every code then fits
// 15 bits and a sum of two codes fits 16, so the index arithmetic of two
// codes runs in one packed 16-bit instruction and the tests for the zero
// element become bit masks instead of per-code selects.
//
// Codes (as stored): 0 is the zero element, c in [1, q'] is g^c, q' = q - 1
// (q' itself codes g^0 = 1).  zech_step2(z, a, b) returns, per half, the code
// of z + a b:
//  * product: s = a + b; (s - 1) mod q' = min(s - 1, s - 1 - q') in 16-bit
//    wrap-around arithmetic; its code is that plus one, with a mask that is
//    all ones in each half where neither factor is zero;
//  * sum g^u + g^t = g^(u + h) with g^h = 1 + g^k, k = t - u: first
//    k - 1 = (t - 1 - u) mod q' by the same minimum, then the plus-one table
//    shifted by one index, tab[k - 1] = h - 1, or 0x8000 where 1 + g^k = 0
//    (built at field creation, FieldK::zsh1); the code of the sum is ((u + h - 1) mod q') + 1,
//    zeroed where the table holds the 0x8000 mark; a zero accumulator takes
//    the product, a zero product leaves the accumulator as it is.
// Every table index lies in [0, q' - 1] for any codes in [0, q'].
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

// z + a b per 16-bit half; tb: the shifted table (bytes, in LDS).
__device__ __forceinline__ uint32_t zech_step2(uint32_t zw, uint32_t aw, uint32_t bw,
                                               const char* tb, const ZechPacked& C) {
  uint32_t S, Sa, Sb, R, mn, m1, mp, Pc, D, Dq, K, K2, S1, S1q, Wm, W, hs, keep, mz, mu;
  FD_PK("v_pk_add_u16", S, aw, bw);
  FD_PKS("v_pk_sub_u16", Sa, S, C.k1);
  FD_PKS("v_pk_sub_u16", Sb, S, C.q1);
  FD_PK("v_pk_min_u16", R, Sa, Sb);        // (s - 1) mod q'
  FD_PK("v_pk_min_u16", mn, aw, bw);
  FD_PKS("v_pk_min_u16", m1, mn, C.k1);
  FD_PKNEG(mp, m1);                        // ones where the product is nonzero
  const uint32_t Pm = R & mp;              // product code - 1 (0 if zero)
  FD_PKS("v_pk_add_u16", Pc, Pm, C.k1);    // product code
  FD_PK("v_pk_sub_u16", D, Pm, zw);
  FD_PKS("v_pk_add_u16", Dq, D, C.qq);
  FD_PK("v_pk_min_u16", K, D, Dq);         // k - 1 in [0, q' - 1]
  FD_PK("v_pk_add_u16", K2, K, K);         // byte offsets of the two table entries
  const uint32_t hw = (uint32_t)*(const uint16_t*)(tb + (K2 & 0xFFFFu)) |
                      ((uint32_t)*(const uint16_t*)(tb + (K2 >> 16)) << 16);
  FD_PK("v_pk_add_u16", S1, zw, hw);       // u + h - 1
  FD_PKS("v_pk_sub_u16", S1q, S1, C.qq);
  FD_PK("v_pk_min_u16", Wm, S1, S1q);
  FD_PKS("v_pk_add_u16", W, Wm, C.k1);     // code of the sum
  FD_PKS1("v_pk_lshrrev_b16", hs, C.f15, hw);
  FD_PKS("v_pk_sub_u16", keep, hs, C.k1);  // zero where the sum is 0
  FD_PKS("v_pk_min_u16", mz, zw, C.k1);
  FD_PKNEG(mu, mz);                        // ones where u != 0
  const uint32_t r1 = W & keep;
  const uint32_t r2 = (r1 & mu) | (Pc & ~mu);
  return (r2 & mp) | (zw & ~mp);
}
