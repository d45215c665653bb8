// Elementwise field operations (Sec. 2, opening): addition, subtraction,
// negation, multiplication, division, AXPY (r = a x + y) and AXPYIN
// (r = a x + r) on vectors of n stored values, in each representation:
//
//   classical residues (Sec. 2.1): one conditional correction for the sums,
//     one remainder for a product or for a whole AXPY (a x + y < p 2^32);
//   Montgomery residues (Sec. 2.2): sums as classical, products by REDC;
//   integral doubles (Sec. 2.3): sums with one correction, products and
//     AXPY by the floating-point remainder (exact: a x + y <= 2^53 is the
//     field's admission bound);
//   discrete logarithms (Sec. 2.4, Table 1): products and quotients are index
//     sums and differences modulo q-1, negation adds the index of -1,
//     addition goes through the plus-one table, g^i + g^j = g^i (1 + g^(j-i));
//   centred residues (Sec. 3.2.2): sums with one correction each way,
//     products by the nearest quotient in single precision (below).
//
// Division multiplies by the inverse.  For classical, Montgomery and double
// residues the inverse is b^(p-2) (Fermat), by sliding-window powering with
// the representation's own product: the same instruction stream for every lane,
// where the extended Euclidean algorithm of Sec. 2.1 would branch per lane.
// On the vector path one exponentiation serves the divisors of 16 elements
// per lane, 8 for doubles (simultaneous inversion).  Centred residues (p < 2^8) read their
// inverses from a 256-entry table built at field creation.  A zero divisor
// gives the zero element.
//
// Discrete-log addition, subtraction and AXPY are all z + a b (a = 1, a = -1,
// a = alpha): over fields of at most 32768 elements two codes per packed
// 16-bit step, above that one code per lane (zech_packed.h).
//
// Every lane handles 16 bytes of each operand (one vector load) when all
// pointers are 16-byte aligned, else one element, with as many workgroups as
// that takes (the discrete-log sums: resident workgroups with the table in
// LDS).  The kernels are bound by HBM except division for large primes
// (ALU-bound: one exponentiation, about 1.3 log2 p products, per 16 divisors).
#include <string.h>

#include <algorithm>
#include <type_traits>

#include "fdot_internal.h"
#include "zech_packed.h"

namespace {

struct RZpz {
  using E = uint32_t;
  static __device__ E zero() { return 0; }
  static __device__ E one(const FieldK&) { return 1; }
  static __device__ E add(E a, E b, const FieldK& F) {
    const uint64_t s = (uint64_t)a + b;
    return (E)(s >= F.p ? s - F.p : s);
  }
  static __device__ E sub(E a, E b, const FieldK& F) {
    return a >= b ? a - b : (E)((uint64_t)a + F.p - b);
  }
  static __device__ E neg(E a, const FieldK& F) { return a == 0 ? 0u : (E)(F.p - a); }
  static __device__ E mul(E a, E b, const FieldK& F) { return mod_small((uint64_t)a * b, F); }
  // one remainder for the whole a x + y (< p^2 < p 2^32)
  static __device__ E axpy(E a, E x, E y, const FieldK& F) {
    return mod_small((uint64_t)a * x + y, F);
  }
  static __device__ bool is_zero(E a) { return a == 0; }
};

struct RMont : RZpz {
  // Montgomery form of 1 is B mod p
  static __device__ E one(const FieldK& F) { return mod_u64(1ull << 32, F); }
  static __device__ E mul(E a, E b, const FieldK& F) { return redc((uint64_t)a * b, F); }
  static __device__ E axpy(E a, E x, E y, const FieldK& F) { return add(mul(a, x, F), y, F); }
};

struct RF64 {
  using E = double;
  static __device__ E zero() { return 0.0; }
  static __device__ E one(const FieldK&) { return 1.0; }
  static __device__ E add(E a, E b, const FieldK& F) {
    const double s = a + b;
    return s >= F.P ? s - F.P : s;
  }
  static __device__ E sub(E a, E b, const FieldK& F) { return a >= b ? a - b : (a - b) + F.P; }
  static __device__ E neg(E a, const FieldK& F) { return a == 0.0 ? 0.0 : F.P - a; }
  static __device__ E mul(E a, E b, const FieldK& F) { return fold_f64(a * b, F); }
  static __device__ E axpy(E a, E x, E y, const FieldK& F) { return fold_f64(fma(a, x, y), F); }
  static __device__ bool is_zero(E a) { return a == 0.0; }
};

// Codes: 0 is the zero element, i in [1, q-1] is g^i (q-1 codes the element 1);
// the same for prime fields and for extensions GF(p^d) (Sec. 2.4.2), whose
// constants hold q in place of p.
struct RZech {
  using E = uint16_t;
  static __device__ E zero() { return 0; }
  static __device__ E one(const FieldK& F) { return (E)F.qbar; }
  static __device__ E idx_add(uint32_t i, uint32_t j, const FieldK& F) {
    const uint32_t k = i + j;
    return (E)(k > F.qbar ? k - F.qbar : k);
  }
  static __device__ E idx_sub(uint32_t i, uint32_t j, const FieldK& F) {
    return (E)(i > j ? i - j : i + F.qbar - j);
  }
  static __device__ E mul(E a, E b, const FieldK& F) {
    return (a == 0 || b == 0) ? (E)0 : idx_add(a, b, F);
  }
  static __device__ E div(E a, E b, const FieldK& F) {
    return (a == 0 || b == 0) ? (E)0 : idx_sub(a, b, F);
  }
  // -1 = g^((q-1)/2) in odd characteristic (half holds (q-1)/2); in
  // characteristic 2, -1 = 1 and half holds 0
  static __device__ E neg(E a, const FieldK& F) {
    return a == 0 ? (E)0 : idx_add(a, (uint32_t)F.half, F);
  }
  // z + a b by the one-code step of zech_packed.h (running form code - 1);
  // F.zplus1 is the plus-one table staged in LDS with entry 0 = entry q'
  static __device__ E fma(E z, E a, E b, const FieldK& F) {
    return (E)(zech_acc1((uint32_t)z - 1u, a, b, F.zplus1, F.qbar) + 1u);
  }
  static __device__ E add(E a, E b, const FieldK& F) { return fma(a, b, (E)F.qbar, F); }
  static __device__ E sub(E a, E b, const FieldK& F) {
    return fma(a, (E)(F.half ? (uint32_t)F.half : F.qbar), b, F);  // a + (-1) b
  }
  static __device__ E axpy(E a, E x, E y, const FieldK& F) { return fma(y, a, x, F); }
  static __device__ bool is_zero(E a) { return a == 0; }
};

struct RCentred {
  using E = int8_t;
  static __device__ E zero() { return 0; }
  static __device__ E one(const FieldK&) { return 1; }
  static __device__ E centre(int32_t s, const FieldK& F) {
    s = s > F.half ? s - (int32_t)F.p32 : s;
    return (E)(s < -F.half ? s + (int32_t)F.p32 : s);
  }
  static __device__ E add(E a, E b, const FieldK& F) { return centre((int32_t)a + b, F); }
  static __device__ E sub(E a, E b, const FieldK& F) { return centre((int32_t)a - b, F); }
  static __device__ E neg(E a, const FieldK&) { return (E)-a; }
  // Centred remainder of |v| <= h^2 + h < 2^14 (a product, or a x + y):
  // v - p rint(v / p), the quotient rounded to nearest from v * RN(1/p) in
  // single precision.  Exact: the computed quotient is within 2^-17 of v/p,
  // and v/p (p odd) is never closer than 1/(2p) to a half-integer, so the
  // rounding picks the nearest integer and the remainder lies in [-h, h]
  // (the same FMA-free remainder as Sec. 2.3's doubles, in a format whose
  // 24-bit mantissa holds these values exactly).
  static __device__ E centre_mod(int32_t v, const FieldK& F) {
    const float q = __builtin_rintf((float)v * F.invPf);
    return (E)(v - (int32_t)F.p32 * (int32_t)q);
  }
  static __device__ E mul(E a, E b, const FieldK& F) { return centre_mod((int32_t)a * b, F); }
  static __device__ E axpy(E a, E x, E y, const FieldK& F) {
    return centre_mod((int32_t)a * x + y, F);
  }
  static __device__ bool is_zero(E a) { return a == 0; }
};

// 16-byte global accesses, marked nontemporal: every element is touched once.
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const v4u gv4_t;
typedef __attribute__((address_space(1))) v4u gv4w_t;

template <class V>
__device__ __forceinline__ V load16(const V* p) {
  const v4u raw = __builtin_nontemporal_load((gv4_t*)p);
  V v;
  __builtin_memcpy(&v, &raw, 16);
  return v;
}
template <class V>
__device__ __forceinline__ void store16(V* p, const V& v) {
  v4u raw;
  __builtin_memcpy(&raw, &v, 16);
  __builtin_nontemporal_store(raw, (gv4w_t*)p);
}

// Discrete-logarithm additions read the plus-one table at random; it is
// staged in LDS (2p bytes, at most 128 KiB) by workgroups that stay resident
// for the whole vector.
template <class R, int OP>
constexpr bool table_in_lds() {
  return std::is_same<R, RZech>::value &&
         (OP == FDOT_EW_ADD || OP == FDOT_EW_SUB || OP == FDOT_EW_AXPY);
}

// b^(p-2), left to right over the bits of p-2 with windows of up to three
// bits that end in a one (sliding windows): each window is one product by
// b, b^3, b^5 or b^7 (computed first, four products), after one squaring per
// bit.  For p = 2^31-1 that is 30 squarings and 14 products, against 30 and
// 30 bit by bit.  The exponent is the field's, the same for every lane, so
// the loop and its branches are uniform.
template <class R>
__device__ typename R::E inverse(typename R::E b, const FieldK& F) {
  using E = typename R::E;
  const uint64_t e = F.p - 2;
  if (e == 0) return R::one(F);  // p = 2: the only nonzero element is its own inverse
  const E b2 = R::mul(b, b, F);
  const E b3 = R::mul(b, b2, F), b5 = R::mul(b3, b2, F), b7 = R::mul(b5, b2, F);
  auto odd_power = [&](uint32_t w) { return w == 1 ? b : w == 3 ? b3 : w == 5 ? b5 : b7; };
  int bit = 63 - __builtin_clzll(e);
  // the top window starts the result without squarings
  int lo = bit >= 2 ? bit - 2 : 0;
  while (!((e >> lo) & 1)) ++lo;
  E r = odd_power((uint32_t)(e >> lo) & ((2u << (bit - lo)) - 1));
  bit = lo - 1;
  while (bit >= 0) {
    if (!((e >> bit) & 1)) {
      r = R::mul(r, r, F);
      --bit;
      continue;
    }
    lo = bit >= 2 ? bit - 2 : 0;
    while (!((e >> lo) & 1)) ++lo;
    for (int i = lo; i <= bit; ++i) r = R::mul(r, r, F);
    r = R::mul(r, odd_power((uint32_t)(e >> lo) & ((2u << (bit - lo)) - 1)), F);
    bit = lo - 1;
  }
  return r;
}

template <class R>
__device__ typename R::E divide(typename R::E a, typename R::E b, const FieldK& F) {
  if constexpr (std::is_same<R, RZech>::value) {
    return R::div(a, b, F);
  } else if constexpr (std::is_same<R, RCentred>::value) {
    // the table of inverses (in LDS), inverse of 0 stored as 0
    return R::mul(a, F.cinv[(int32_t)b + 128], F);
  } else {
    if (R::is_zero(b)) return R::zero();
    if (F.p == 2) return a;  // the only nonzero divisor is 1
    return R::mul(a, inverse<R>(b, F), F);
  }
}

// Division of W elements with one inversion (simultaneous inversion): the
// divisors' prefix products, one exponentiation for the inverse of the whole
// product, then each divisor's inverse peeled off with two products.  That is
// about 4 products per element plus one exponentiation per W elements,
// instead of one exponentiation per element.  A zero divisor enters the
// product as one and gives the zero element.
template <class R, int W>
__device__ __forceinline__ void divide_vec(const typename R::E* a, const typename R::E* b,
                                           typename R::E* out, const FieldK& F) {
  using E = typename R::E;
  E c[W], pre[W];
#pragma unroll
  for (int k = 0; k < W; ++k) c[k] = R::is_zero(b[k]) ? R::one(F) : b[k];
  pre[0] = c[0];
#pragma unroll
  for (int k = 1; k < W; ++k) pre[k] = R::mul(pre[k - 1], c[k], F);
  E inv = inverse<R>(pre[W - 1], F);  // inverse of c[0] ... c[k] while peeling
#pragma unroll
  for (int k = W - 1; k > 0; --k) {
    const E ik = R::mul(inv, pre[k - 1], F);  // 1 / c[k]
    inv = R::mul(inv, c[k], F);
    out[k] = R::is_zero(b[k]) ? R::zero() : R::mul(a[k], ik, F);
  }
  out[0] = R::is_zero(b[0]) ? R::zero() : R::mul(a[0], inv, F);
}

template <class R, int OP>
__device__ __forceinline__ typename R::E apply(typename R::E a, typename R::E x,
                                               typename R::E y, const FieldK& F) {
  switch (OP) {
    case FDOT_EW_ADD: return R::add(x, y, F);
    case FDOT_EW_SUB: return R::sub(x, y, F);
    case FDOT_EW_NEG: return R::neg(x, F);
    case FDOT_EW_MUL: return R::mul(x, y, F);
    case FDOT_EW_DIV: return divide<R>(x, y, F);
    default: return R::axpy(a, x, y, F);  // AXPY, and AXPYIN with y = r
  }
}

// y is read for the binary operations and AXPY; for AXPYIN it is r itself.
template <int OP>
constexpr bool reads_y() {
  return OP != FDOT_EW_NEG;
}

template <class R, int OP, bool VEC, int NT>
__global__ __launch_bounds__(NT) void ew_kernel(const FieldK Fin, uint64_t n,
                                                const typename R::E* x,
                                                const typename R::E* y, typename R::E* r,
                                                typename R::E a) {
  using E = typename R::E;
  FieldK F = Fin;
  if constexpr (std::is_same<R, RCentred>::value && OP == FDOT_EW_DIV) {
    __shared__ int8_t s_inv[256];
    for (uint32_t i = threadIdx.x; i < 256; i += NT) s_inv[i] = Fin.cinv[i];
    __syncthreads();
    F.cinv = s_inv;
  }
  if constexpr (table_in_lds<R, OP>()) {
    extern __shared__ uint16_t s_plus1[];
    fd_table_to_lds<NT>(s_plus1, Fin.zplus1, (uint32_t)Fin.p);
    if (threadIdx.x == 0) s_plus1[0] = s_plus1[Fin.qbar];  // g^0, for the one-code step
    __syncthreads();
    F.zplus1 = s_plus1;
  }
  const uint64_t tid = (uint64_t)blockIdx.x * NT + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * NT;
  if constexpr (VEC) {
    constexpr int W = 16 / (int)sizeof(E);
    struct alignas(16) V { E e[W]; };
    const uint64_t nv = n / W;
    uint64_t v = tid;
    for (; v < nv; v += stride) {
      const V xv = load16((const V*)x + v);
      V yv = {};
      if constexpr (reads_y<OP>()) yv = load16((const V*)y + v);
      V out;
      if constexpr (OP == FDOT_EW_DIV && !std::is_same<R, RZech>::value &&
                    !std::is_same<R, RCentred>::value) {
        divide_vec<R, W>(xv.e, yv.e, out.e, F);
      } else {
#pragma unroll
        for (int k = 0; k < W; ++k) out.e[k] = apply<R, OP>(a, xv.e[k], yv.e[k], F);
      }
      store16((V*)r + v, out);
    }
    for (uint64_t i = nv * W + tid; i < n; i += stride)
      r[i] = apply<R, OP>(a, x[i], reads_y<OP>() ? y[i] : E(0), F);
  } else {
    for (uint64_t i = tid; i < n; i += stride)
      r[i] = apply<R, OP>(a, x[i], reads_y<OP>() ? y[i] : E(0), F);
  }
}

// Division for classical, Montgomery and double residues on 16-byte aligned
// operands: each lane takes NE elements (NE / W vectors, NT vectors apart so
// that the loads stay coalesced) and inverts their divisors with one
// exponentiation (simultaneous inversion, as divide_vec, over NE elements
// instead of one vector's W): about 4 products per element plus an NE-th of
// an exponentiation.  A zero divisor counts as one in the product and gives
// zero.  The n mod W last elements are divided one by one.
template <class R, int NT, int NE>
__global__ __launch_bounds__(NT) void ew_div_kernel(const FieldK F, uint64_t n,
                                                    const typename R::E* x,
                                                    const typename R::E* y, typename R::E* r) {
  using E = typename R::E;
  constexpr int W = 16 / (int)sizeof(E);
  constexpr int G = NE / W;
  static_assert(G * W == NE, "whole vectors per lane");
  struct alignas(16) V { E e[W]; };
  const uint64_t nv = n / W;
  const uint64_t span = (uint64_t)NT * G;
  for (uint64_t b0 = (uint64_t)blockIdx.x * span; b0 < nv; b0 += (uint64_t)gridDim.x * span) {
    E a[NE], d[NE];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const uint64_t v = b0 + (uint64_t)g * NT + threadIdx.x;
      V xv = {}, yv = {};
      if (v < nv) {
        xv = load16((const V*)x + v);
        yv = load16((const V*)y + v);
      }
#pragma unroll
      for (int k = 0; k < W; ++k) {
        a[g * W + k] = xv.e[k];
        d[g * W + k] = yv.e[k];
      }
    }
    E pre[NE];
    pre[0] = R::is_zero(d[0]) ? R::one(F) : d[0];
#pragma unroll
    for (int k = 1; k < NE; ++k) pre[k] = R::mul(pre[k - 1], R::is_zero(d[k]) ? R::one(F) : d[k], F);
    E inv = inverse<R>(pre[NE - 1], F);  // of the divisors 0 .. k while peeling
#pragma unroll
    for (int k = NE - 1; k > 0; --k) {
      const E ik = R::mul(inv, pre[k - 1], F);
      inv = R::mul(inv, R::is_zero(d[k]) ? R::one(F) : d[k], F);
      a[k] = R::is_zero(d[k]) ? R::zero() : R::mul(a[k], ik, F);
    }
    a[0] = R::is_zero(d[0]) ? R::zero() : R::mul(a[0], inv, F);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const uint64_t v = b0 + (uint64_t)g * NT + threadIdx.x;
      if (v < nv) {
        V out;
#pragma unroll
        for (int k = 0; k < W; ++k) out.e[k] = a[g * W + k];
        store16((V*)r + v, out);
      }
    }
  }
  if (blockIdx.x == 0)
    for (uint64_t i = nv * W + threadIdx.x; i < n; i += NT) r[i] = divide<R>(x[i], y[i], F);
}

template <class R, int NE>
fdot_status_t launch_div(const fdot_field_s* f, uint64_t n, const void* x, const void* y, void* r,
                         hipStream_t s) {
  using E = typename R::E;
  constexpr int NT = 256, W = 16 / (int)sizeof(E);
  const uint64_t blocks = (n / W + (uint64_t)NT * (NE / W) - 1) / ((uint64_t)NT * (NE / W));
  const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(blocks, (1ull << 31) - 1));
  hipLaunchKernelGGL((ew_div_kernel<R, NT, NE>), dim3(grid), dim3(NT), 0, s, f->k, n,
                     (const E*)x, (const E*)y, (E*)r);
  return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
}

// Discrete-log addition, subtraction and AXPY for fields of at most 32768
// elements: each is z + a b per code (zech_packed.h) -- x + y with a = 1,
// x - y = x + (-1) y, a x + y -- on two codes per packed step, with the
// packed step's plus-one table in LDS.  aw: the code of a in both halves.
template <int OP, bool VEC, int NT>
__global__ __launch_bounds__(NT) void ew_zech2_kernel(const FieldK F, uint64_t n, const uint16_t* x,
                                                      const uint16_t* y, uint16_t* r, uint32_t aw) {
  extern __shared__ uint16_t s_tab[];
  fd_table_to_lds<NT>(s_tab, F.zpk, F.p32);
  const ZechPacked C = zech_packed_constants(F);
  const char* tb = (const char*)s_tab;
  // SUB accumulates into x (z = x, b = y); ADD and AXPY into y (z = y, b = x)
  const uint16_t* zs = OP == FDOT_EW_SUB ? x : y;
  const uint16_t* bs = OP == FDOT_EW_SUB ? y : x;
  const uint64_t tid = (uint64_t)blockIdx.x * NT + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * NT;
  uint64_t done = 0;
  if constexpr (VEC) {
    // two vectors per lane per step, all four loads issued before the table
    // lookups: the resident workgroups are few (the LDS holds few tables), so
    // each lane keeps more bytes in flight
    const uint64_t nv = n / 8;
    auto step4 = [&](const v4u& zv, const v4u& bv) {
      v4u out;
      out.x = zech_step2(zv.x, aw, bv.x, tb, C);
      out.y = zech_step2(zv.y, aw, bv.y, tb, C);
      out.z = zech_step2(zv.z, aw, bv.z, tb, C);
      out.w = zech_step2(zv.w, aw, bv.w, tb, C);
      return out;
    };
    uint64_t v = tid;
    for (; v + stride < nv; v += 2 * stride) {
      const v4u z0 = load16((const v4u*)zs + v), b0 = load16((const v4u*)bs + v);
      const v4u z1 = load16((const v4u*)zs + v + stride), b1 = load16((const v4u*)bs + v + stride);
      store16((v4u*)r + v, step4(z0, b0));
      store16((v4u*)r + v + stride, step4(z1, b1));
    }
    if (v < nv) store16((v4u*)r + v, step4(load16((const v4u*)zs + v), load16((const v4u*)bs + v)));
    done = nv * 8;
  }
  for (uint64_t i = done + tid; i < n; i += stride)  // low half only
    r[i] = (uint16_t)zech_step2(zs[i], aw & 0xFFFFu, bs[i], tb, C);
}

template <int OP>
fdot_status_t launch_zech2(const fdot_field_s* f, uint64_t n, uint16_t a, const void* x,
                           const void* y, void* r, hipStream_t s) {
  constexpr int NT = 1024;
  const FieldK& F = f->k;
  uint32_t code = a;                                  // AXPY
  if (OP == FDOT_EW_ADD) code = F.qbar;               // 1
  if (OP == FDOT_EW_SUB) code = F.half ? (uint32_t)F.half : F.qbar;  // -1 (= 1 in characteristic 2)
  const uint32_t aw = code | (code << 16);
  const bool vec = (((uintptr_t)x | (uintptr_t)y | (uintptr_t)r) & 15u) == 0;
  const uint64_t work = vec ? (n + 7) / 8 : n;
  const size_t lds = (size_t)F.p * sizeof(uint16_t);  // q entries
  const uint64_t per_cu = std::max<uint64_t>(1, (160u * 1024u) / lds);
  const unsigned grid = (unsigned)std::max<uint64_t>(
      1, std::min<uint64_t>((work + NT - 1) / NT, (uint64_t)fd_cu_count() * per_cu));
  if (vec)
    hipLaunchKernelGGL((ew_zech2_kernel<OP, true, NT>), dim3(grid), dim3(NT), lds, s, F, n,
                       (const uint16_t*)x, (const uint16_t*)y, (uint16_t*)r, aw);
  else
    hipLaunchKernelGGL((ew_zech2_kernel<OP, false, NT>), dim3(grid), dim3(NT), lds, s, F, n,
                       (const uint16_t*)x, (const uint16_t*)y, (uint16_t*)r, aw);
  return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
}

template <class R, int OP>
fdot_status_t launch_op(const fdot_field_s* f, uint64_t n, const void* alpha, const void* x,
                        const void* y, void* r, hipStream_t s) {
  using E = typename R::E;
  E a{};
  if (alpha) memcpy(&a, alpha, sizeof(E));
  if constexpr (table_in_lds<R, OP>()) {
    // q <= 32768: two codes per packed step (tune key zech.packed = 0: one per lane)
    if (f->k.p <= 32768 && fd_tune("zech.packed", 1) != 0)
      return launch_zech2<OP>(f, n, (uint16_t)a, x, y, r, s);
  }
  const uintptr_t bits = (uintptr_t)x | (uintptr_t)r | (reads_y<OP>() ? (uintptr_t)y : 0);
  const bool vec = (bits & 15u) == 0;
  if constexpr (OP == FDOT_EW_DIV && !std::is_same<R, RZech>::value &&
                !std::is_same<R, RCentred>::value) {
    // NE elements per exponentiation (tune key ew.div_elems: 8, 16 or 32):
    // 8 for doubles (fewer registers, more resident waves: 0.70 -> 0.76 of
    // HBM at p = 2^26-5), 16 for the 32-bit forms (8 measured 0.70 against
    // 0.74 classical and 0.52 against 0.69 Montgomery)
    if (vec) {
      const int64_t ne = fd_tune("ew.div_elems", std::is_same<R, RF64>::value ? 8 : 16);
      return ne == 32  ? launch_div<R, 32>(f, n, x, y, r, s)
             : ne == 8 ? launch_div<R, 8>(f, n, x, y, r, s)
                       : launch_div<R, 16>(f, n, x, y, r, s);
    }
  }
  const uint64_t per = vec ? 16 / sizeof(E) : 1;
  const uint64_t work = (n + per - 1) / per;
  if constexpr (table_in_lds<R, OP>()) {
    // 1024 threads per workgroup, as many resident workgroups as the LDS
    // holds tables (160 KiB per CU), and no more than the work needs
    constexpr int NT = 1024;
    const size_t lds = (size_t)f->k.p * sizeof(uint16_t);  // q entries
    const uint64_t per_cu = std::max<uint64_t>(1, (160u * 1024u) / lds);
    const unsigned grid = (unsigned)std::max<uint64_t>(
        1, std::min<uint64_t>((work + NT - 1) / NT, (uint64_t)fd_cu_count() * per_cu));
    static bool attr_set[2] = {false, false};
    if (!attr_set[vec]) {
      (void)hipFuncSetAttribute(vec ? (const void*)ew_kernel<R, OP, true, NT>
                                    : (const void*)ew_kernel<R, OP, false, NT>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
      attr_set[vec] = true;
    }
    if (vec)
      hipLaunchKernelGGL((ew_kernel<R, OP, true, NT>), dim3(grid), dim3(NT), lds, s, f->k, n,
                         (const E*)x, (const E*)y, (E*)r, a);
    else
      hipLaunchKernelGGL((ew_kernel<R, OP, false, NT>), dim3(grid), dim3(NT), lds, s, f->k, n,
                         (const E*)x, (const E*)y, (E*)r, a);
  } else {
    // One 16-byte vector per lane (tune key ew.wg_per_cu caps the workgroups
    // per CU instead, the lanes then striding): a grid-stride loop keeps one
    // load in flight per lane, since each store may alias the next loads,
    // and reached 0.58 of HBM against 0.81 for one vector per lane.
    const int64_t per_cu = fd_tune("ew.wg_per_cu", 0);
    const uint64_t cap = per_cu > 0 ? (uint64_t)fd_cu_count() * per_cu : (1ull << 31) - 1;
    const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((work + 255) / 256, cap));
    if (vec)
      hipLaunchKernelGGL((ew_kernel<R, OP, true, 256>), dim3(grid), dim3(256), 0, s, f->k, n,
                         (const E*)x, (const E*)y, (E*)r, a);
    else
      hipLaunchKernelGGL((ew_kernel<R, OP, false, 256>), dim3(grid), dim3(256), 0, s, f->k, n,
                         (const E*)x, (const E*)y, (E*)r, a);
  }
  return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
}

template <class R>
fdot_status_t launch_rep(const fdot_field_s* f, fdot_ew_op_t op, uint64_t n, const void* alpha,
                         const void* x, const void* y, void* r, hipStream_t s) {
  switch (op) {
    case FDOT_EW_ADD: return launch_op<R, FDOT_EW_ADD>(f, n, alpha, x, y, r, s);
    case FDOT_EW_SUB: return launch_op<R, FDOT_EW_SUB>(f, n, alpha, x, y, r, s);
    case FDOT_EW_NEG: return launch_op<R, FDOT_EW_NEG>(f, n, alpha, x, y, r, s);
    case FDOT_EW_MUL: return launch_op<R, FDOT_EW_MUL>(f, n, alpha, x, y, r, s);
    case FDOT_EW_DIV: return launch_op<R, FDOT_EW_DIV>(f, n, alpha, x, y, r, s);
    case FDOT_EW_AXPY: return launch_op<R, FDOT_EW_AXPY>(f, n, alpha, x, y, r, s);
    case FDOT_EW_AXPYIN: return launch_op<R, FDOT_EW_AXPY>(f, n, alpha, x, r, r, s);
  }
  return FDOT_E_INVALID_ARG;
}

}  // namespace

fdot_status_t fd_launch_elementwise(const fdot_field_s* f, fdot_ew_op_t op, uint64_t n,
                                    const void* alpha, const void* x, const void* y, void* r,
                                    hipStream_t s) {
  if (n == 0) return FDOT_OK;
  switch (f->info.rep) {
    case FDOT_REP_ZPZ_U32: return launch_rep<RZpz>(f, op, n, alpha, x, y, r, s);
    case FDOT_REP_MONT_U32: return launch_rep<RMont>(f, op, n, alpha, x, y, r, s);
    case FDOT_REP_FP64: return launch_rep<RF64>(f, op, n, alpha, x, y, r, s);
    case FDOT_REP_ZECH_U16: return launch_rep<RZech>(f, op, n, alpha, x, y, r, s);
    case FDOT_REP_CENTRED_I8: return launch_rep<RCentred>(f, op, n, alpha, x, y, r, s);
  }
  return FDOT_E_UNSUPPORTED;
}
