// Field arithmetic shared by the kernels and by the host-side fold check.
//
// The reductions are the ones the paper compares (Sec. 2): a machine-style
// remainder (GPUs have no integer divider, so the remainder is taken with a
// precomputed reciprocal: the 2-by-1 division by an invariant divisor of
// N. Moeller and T. Granlund, "Improved division by invariant integers", IEEE
// Trans. Computers 60(2), 2011, Algorithm 4), Montgomery's REDC with B = 2^32
// (Sec. 2.2), and the floating-point remainder T - floor(T/p)*p with one
// correction each way (Sec. 2.3).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#define FD_HD __host__ __device__ __forceinline__

// Everything a kernel needs to know about GF(p), passed by value.
struct FieldK {
  uint64_t p;
  uint64_t corr;      // 2^64 mod p
  double P;           // p as a double
  double invP;        // RN(1/p)
  uint32_t p32;
  uint32_t shift;     // s: 2^31 <= p*2^s < 2^32
  uint32_t dnorm;     // p*2^s
  uint32_t recip;     // floor((2^64-1)/dnorm) - 2^32
  uint32_t n_im;      // -p^-1 mod 2^32
  uint32_t qbar;      // p-1 (Zech index of the element 1)
  int32_t half;       // (p-1)/2 (centred range)
  uint32_t pad;
  const uint16_t* zval;    // Zech code -> value, p entries (zval[0] = 0)
  const uint16_t* zplus1;  // Zech plus-one table, p entries
  const uint16_t* zidx;    // value -> Zech code, p entries
  const int8_t* cinv;      // centred residues (p < 2^8): inverse of c at c + 128, 256 entries
  float invPf;             // 1/p in single precision (centred residues)
  uint32_t pad2;
  // Zech, q <= 32768: the plus-one table of the packed step, entry k = code
  // of 1 + g^k (k = 0 and k = q - 1 both for g^0), or 0xFFFF where that sum
  // is zero; q entries, zero-padded to a multiple of 8, 16-byte aligned
  // (null for larger q)
  const uint16_t* zpk;
};

// Remainder of the two-word number u1*2^32 + u0 by a normalised divisor d
// (2^31 <= d < 2^32) when u1 < d, using v = floor((2^64-1)/d) - 2^32.
// Candidate quotient from the reciprocal, then at most two corrections; all
// quotient arithmetic is modulo 2^32 as in the published algorithm.
FD_HD uint32_t rem_2by1(uint32_t u1, uint32_t u0, uint32_t d, uint32_t v) {
  uint64_t q = (uint64_t)v * u1 + ((((uint64_t)u1) << 32) | u0);
  uint32_t q1 = (uint32_t)(q >> 32) + 1u;
  uint32_t q0 = (uint32_t)q;
  uint32_t r = u0 - q1 * d;
  if (r > q0) r += d;
  if (r >= d) r -= d;
  return r;
}

// T mod p for any 64-bit T: T*2^s split into three 32-bit words, two 2-by-1
// steps, then undo the normalisation shift.
FD_HD uint32_t mod_u64(uint64_t T, const FieldK& F) {
  const uint32_t s = F.shift, d = F.dnorm, v = F.recip;
  if (s == 0) {
    uint32_t u1 = (uint32_t)(T >> 32);
    if (u1 >= d) u1 -= d;
    return rem_2by1(u1, (uint32_t)T, d, v);
  }
  uint32_t n2 = (uint32_t)(T >> (64 - s));
  uint32_t n1 = (uint32_t)(T >> (32 - s));
  uint32_t n0 = (uint32_t)(T << s);
  uint32_t r = rem_2by1(n2, n1, d, v);
  r = rem_2by1(r, n0, d, v);
  return r >> s;
}

// T mod p when T < p*2^32 (so T*2^s still fits 64 bits with a top word below
// the divisor): one 2-by-1 step.  This covers acc + a*b with acc, a, b < p.
FD_HD uint32_t mod_small(uint64_t T, const FieldK& F) {
  const uint64_t t = T << F.shift;
  return rem_2by1((uint32_t)(t >> 32), (uint32_t)t, F.dnorm, F.recip) >> F.shift;
}

// Montgomery reduction with B = 2^32 (Sec. 2.2): for T < p*B returns
// T*B^-1 mod p in [0, p).  U = T*n_im mod B makes T + U*p divisible by B; the
// sum can need 65 bits when p > 2^31, so its carry is kept.
FD_HD uint32_t redc(uint64_t T, const FieldK& F) {
  const uint32_t U = (uint32_t)T * F.n_im;
  const uint64_t S = T + (uint64_t)U * F.p32;
  const uint64_t carry = S < T ? 1ull : 0ull;
  const uint64_t r = (S >> 32) | (carry << 32);
  return (uint32_t)(r >= F.p ? r - F.p : r);
}

// Floating-point remainder of an integral T in [0, 2^53] (Sec. 2.3): the
// quotient from the rounded inverse is off by at most one, the remainder is
// computed exactly by one fused multiply-add and corrected once.
FD_HD double fold_f64(double T, const FieldK& F) {
  const double q = floor(T * F.invP);
  double r = fma(-q, F.P, T);
  r = (r >= F.P) ? r - F.P : r;
  r = (r < 0.0) ? r + F.P : r;
  return r;
}

// Residue of a signed 64-bit value.
FD_HD uint32_t mod_i64(int64_t T, const FieldK& F) {
  if (T >= 0) return mod_u64((uint64_t)T, F);
  const uint32_t r = mod_u64((uint64_t)(-(T + 1)) + 1u, F);
  return r == 0 ? 0u : F.p32 - r;
}
