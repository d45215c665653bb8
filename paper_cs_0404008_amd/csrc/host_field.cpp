// Field set-up on the host: primality, representation bounds (Sec. 2), block
// lengths (Sec. 3.1 Eq. 1 and its variants), reduction constants and the Zech
// tables (Sec. 2.4).  Nothing here runs per element.
#include <stdio.h>
#include <string.h>

#include <new>

#include "fdot_internal.h"

typedef unsigned __int128 u128;

static uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m) {
  return (uint64_t)(((u128)a * b) % m);
}

static uint64_t powmod64(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  b %= m;
  while (e) {
    if (e & 1) r = mulmod64(r, b, m);
    b = mulmod64(b, b, m);
    e >>= 1;
  }
  return r;
}

// Deterministic Miller-Rabin for 64-bit integers: the first twelve prime
// bases are a witness set for every n < 3.3e24 (Sorenson & Webster 2015).
int fd_is_prime_u64(uint64_t n) {
  static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (uint64_t b : bases) {
    if (n == b) return 1;
    if (n % b == 0) return 0;
  }
  uint64_t d = n - 1;
  int r = 0;
  while ((d & 1) == 0) { d >>= 1; ++r; }
  for (uint64_t a : bases) {
    uint64_t x = powmod64(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < r; ++i) {
      x = mulmod64(x, x, n);
      if (x == n - 1) { comp = false; break; }
    }
    if (comp) return 0;
  }
  return 1;
}

// Smallest generator of GF(p)^*: g^((p-1)/f) != 1 for each prime f | p-1.
uint32_t fd_primitive_root(uint64_t p) {
  if (p == 2) return 1;
  uint64_t f[64];
  int nf = 0;
  uint64_t m = p - 1;
  for (uint64_t d = 2; d * d <= m; ++d)
    if (m % d == 0) {
      f[nf++] = d;
      while (m % d == 0) m /= d;
    }
  if (m > 1) f[nf++] = m;
  for (uint64_t g = 2; g < p; ++g) {
    bool ok = true;
    for (int i = 0; i < nf && ok; ++i) ok = powmod64(g, (p - 1) / f[i], p) != 1;
    if (ok) return (uint32_t)g;
  }
  return 0;
}

// Block lengths.  The blocked loop keeps the residue of the previous block
// in the accumulator, so a block of lambda products is safe when
// (p-1) + lambda (p-1)^2 fits (Eq. 1 with the carried term).
static uint64_t lambda_of(uint64_t p, fdot_acc_t acc) {
  if (p < 2) return 0;
  const u128 pm1 = p - 1, sq = pm1 * pm1;
  if (sq == 0) return ~0ull;  // p = 2: every product is 0 or 1 ... and sq = 1
  u128 lim;
  switch (acc) {
    case FDOT_ACC_U64: lim = ~(u128)0 >> 64; break;                   // 2^64-1
    case FDOT_ACC_U32: lim = 0xFFFFFFFFull; break;
    case FDOT_ACC_F64: lim = (u128)1 << 53; break;
    case FDOT_ACC_I32_CENTRED: {
      const u128 h = (p - 1) / 2;
      if (h == 0) return ~0ull;
      const u128 l = ((((u128)1) << 31) - 1) / (h * h);
      return l > ~0ull ? ~0ull : (uint64_t)l;
    }
    case FDOT_ACC_F64_CENTRED: {
      const u128 h = (p - 1) / 2;
      if (h == 0) return ~0ull;
      const u128 l = (((u128)1) << 53) / (h * h);
      return l > ~0ull ? ~0ull : (uint64_t)l;
    }
    case FDOT_ACC_MONT_REDC: {
      if (p >= (1ull << 32)) return 0;
      const u128 l = ((u128)p * ((u128)1 << 32) - 1) / sq;
      return l > ~0ull ? ~0ull : (uint64_t)l;
    }
    case FDOT_ACC_U64_HYBRID: {
      const u128 l = (~(u128)0 >> 64) / ((u128)p * (p - 1));
      return l > ~0ull ? ~0ull : (uint64_t)l;
    }
    default: return 0;
  }
  if (lim < pm1) return 0;
  const u128 l = (lim - pm1) / sq;
  return l > ~0ull ? ~0ull : (uint64_t)l;
}

fdot_status_t fd_fill_params(uint64_t p, fdot_rep_t rep, fdot_field_info_t* out) {
  if (!out) return FDOT_E_INVALID_ARG;
  if ((int)rep < FDOT_REP_ZPZ_U32 || (int)rep > FDOT_REP_CENTRED_I8) return FDOT_E_INVALID_ARG;
  if (p >= (1ull << 32)) return FDOT_E_BOUND;  // word-size: residues in 32 bits
  if (!fd_is_prime_u64(p)) return FDOT_E_NOT_PRIME;
  fdot_field_info_t I;
  memset(&I, 0, sizeof(I));
  I.p = p;
  I.rep = rep;
  I.lambda_u64 = lambda_of(p, FDOT_ACC_U64);
  I.lambda_f64 = lambda_of(p, FDOT_ACC_F64);
  I.lambda_i32c = (p & 1) ? lambda_of(p, FDOT_ACC_I32_CENTRED) : 0;
  I.lambda_redc = (p & 1) ? lambda_of(p, FDOT_ACC_MONT_REDC) : 0;
  I.corr = (uint64_t)((((u128)1) << 64) % p);
  uint32_t s = 0;
  while (((uint64_t)p << s) < (1ull << 31)) ++s;
  I.norm_shift = s;
  const uint64_t d = (uint64_t)p << s;
  I.recip = (uint32_t)((~(u128)0 >> 64) / d - ((u128)1 << 32));
  if (p & 1) {
    uint32_t inv = (uint32_t)p;  // Newton iteration for p^-1 mod 2^32
    for (int i = 0; i < 5; ++i) inv *= 2u - (uint32_t)p * inv;
    I.n_im = (uint32_t)(0u - inv);
    I.b_mod_p = (uint32_t)((1ull << 32) % p);
    I.binv_mod_p = (uint32_t)powmod64(I.b_mod_p, p - 2, p);
  }
  I.b2_mod_p = (uint32_t)I.corr;
  I.inv_p = 1.0 / (double)p;
  switch (rep) {
    case FDOT_REP_ZPZ_U32: I.elem_bytes = 4; break;
    case FDOT_REP_MONT_U32:
      I.elem_bytes = 4;
      if (p == 2) return FDOT_E_BOUND;  // B = 2^32 needs gcd(p, B) = 1
      break;
    case FDOT_REP_FP64:
      I.elem_bytes = 8;
      if (I.lambda_f64 < 1) return FDOT_E_BOUND;  // one product must be exact
      break;
    case FDOT_REP_ZECH_U16:
      I.elem_bytes = 2;
      if (p < 3 || p > 65536) return FDOT_E_BOUND;  // codes 0..p-1 in 16 bits
      I.g = fd_primitive_root(p);
      I.table_bytes = 3ull * p * sizeof(uint16_t) + fd_zech_packed_bytes(p);
      break;
    case FDOT_REP_CENTRED_I8:
      I.elem_bytes = 1;
      if (p < 3 || p > 255) return FDOT_E_BOUND;  // odd p, |a| <= 127
      I.table_bytes = 256;                          // inverses, for division
      break;
    default: return FDOT_E_INVALID_ARG;
  }
  I.degree = 1;
  I.q = p;
  *out = I;
  return FDOT_OK;
}

void fd_fieldk_from_info(const fdot_field_info_t* I, FieldK* k) {
  memset(k, 0, sizeof(*k));
  k->p = I->p;
  k->corr = I->corr;
  k->P = (double)I->p;
  k->invP = I->inv_p;
  k->p32 = (uint32_t)I->p;
  k->shift = I->norm_shift;
  k->dnorm = (uint32_t)(I->p << I->norm_shift);
  k->recip = I->recip;
  k->n_im = I->n_im;
  k->qbar = (uint32_t)(I->p - 1);
  k->half = (int32_t)((I->p - 1) / 2);
  k->invPf = (float)I->inv_p;
}

// Zech tables for the generator g (Sec. 2.4).  Codes: 0 for the zero element,
// i in [1, p-1] for g^i (so p-1 codes g^(p-1) = 1).
int fd_zech_build(uint64_t p, uint32_t g, uint16_t* value, uint16_t* index, uint16_t* plus1) {
  if (p < 3 || p > 65536 || g == 0) return -1;
  uint16_t* val = value;
  uint16_t* idx = index;
  uint16_t* tmpv = nullptr;
  uint16_t* tmpi = nullptr;
  if (!val) val = tmpv = new (std::nothrow) uint16_t[p];
  if (!idx) idx = tmpi = new (std::nothrow) uint16_t[p];
  if (!val || !idx) { delete[] tmpv; delete[] tmpi; return -1; }
  val[0] = 0;
  idx[0] = 0;
  uint64_t v = 1;
  for (uint64_t i = 1; i <= p - 1; ++i) {
    v = v * g % p;
    val[i] = (uint16_t)v;
    idx[v] = (uint16_t)i;
  }
  if (plus1) {
    // plus1[k] = code of 1 + g^k; k = 0 stands for the zero element.
    for (uint64_t k = 0; k <= p - 1; ++k) {
      const uint64_t gk = (k == 0) ? 0 : val[k];
      plus1[k] = idx[(gk + 1) % p];
    }
  }
  delete[] tmpv;
  delete[] tmpi;
  return 0;
}

// Largest block length of the representation's delayed schedule (the bound a
// block option may not exceed).
static uint64_t delayed_lambda(const fdot_field_info_t& I) {
  switch (I.rep) {
    case FDOT_REP_ZPZ_U32: return I.lambda_u64;
    case FDOT_REP_MONT_U32: return I.lambda_redc;
    case FDOT_REP_FP64: return I.lambda_f64;
    case FDOT_REP_ZECH_U16: return 0xFFFFFFFFull / (I.p - 1);
    case FDOT_REP_CENTRED_I8: return I.lambda_i32c;
  }
  return 0;
}

// Schedules each representation has (fdot_algo_t).
static bool algo_allowed(int rep, int algo) {
  if (algo == FDOT_ALGO_AUTO) return true;
  switch (rep) {
    case FDOT_REP_ZPZ_U32:
    case FDOT_REP_MONT_U32:
      return algo == FDOT_ALGO_DELAYED || algo == FDOT_ALGO_PERTERM ||
             algo == FDOT_ALGO_OVERFLOW || algo == FDOT_ALGO_HYBRID;
    case FDOT_REP_FP64: return algo == FDOT_ALGO_DELAYED || algo == FDOT_ALGO_PERTERM;
    case FDOT_REP_ZECH_U16: return algo == FDOT_ALGO_ZECH_EXP || algo == FDOT_ALGO_ZECH_TPLUS1;
    case FDOT_REP_CENTRED_I8: return algo == FDOT_ALGO_DELAYED;
  }
  return false;
}

// Bytes of the packed step's plus-one table (q <= 32768, padded to 16 bytes).
uint64_t fd_zech_packed_bytes(uint64_t q) {
  return q <= 32768 ? ((q + 7) & ~7ull) * sizeof(uint16_t) : 0;
}

// The plus-one table of the packed discrete-log step, from the plus-one
// table indexed by code (host copy, q entries; code q - 1 is g^0): entry k =
// plus1[k] for k in [1, q - 1], entry 0 = plus1[q - 1] (1 + g^0), and 0xFFFF
// in place of the zero code (1 + g^k = 0); the padding is 0.  Uploaded to
// f->d_zpk / f->k.zpk; nothing for q > 32768.
fdot_status_t fd_zech_packed_upload(const uint16_t* plus1, uint32_t q, fdot_field_s* f) {
  const uint64_t bytes = fd_zech_packed_bytes(q);
  if (!bytes) return FDOT_OK;
  const uint64_t n = bytes / sizeof(uint16_t);
  uint16_t* h = new (std::nothrow) uint16_t[n];
  if (!h) return FDOT_E_NOMEM;
  for (uint64_t i = 0; i < n; ++i) {
    const uint16_t v = i == 0 ? plus1[q - 1] : i < q ? plus1[i] : 1;
    h[i] = i >= q ? 0 : v == 0 ? (uint16_t)0xFFFFu : v;
  }
  uint16_t* d = nullptr;
  fdot_status_t st = FDOT_OK;
  if (hipMalloc((void**)&d, bytes) != hipSuccess) st = FDOT_E_NOMEM;
  else if (hipMemcpy(d, h, bytes, hipMemcpyHostToDevice) != hipSuccess) {
    hipFree(d);
    st = FDOT_E_DEVICE;
  }
  delete[] h;
  if (st == FDOT_OK) {
    f->d_zpk = d;
    f->k.zpk = d;
  }
  return st;
}

bool fd_canonical_host(const fdot_field_s* f, const void* value) {
  const uint64_t q = f->degree > 1 ? f->info.q : f->info.p;
  switch (f->info.rep) {
    case FDOT_REP_ZPZ_U32:
    case FDOT_REP_MONT_U32: return *(const uint32_t*)value < f->info.p;
    case FDOT_REP_FP64: {
      const double v = *(const double*)value;
      return v >= 0.0 && v < (double)f->info.p && v == floor(v);
    }
    case FDOT_REP_ZECH_U16: return *(const uint16_t*)value < q;
    case FDOT_REP_CENTRED_I8: {
      const int v = *(const int8_t*)value;
      const int h = (int)((f->info.p - 1) / 2);
      return v >= -h && v <= h;
    }
  }
  return false;
}

extern "C" {

fdot_status_t fdot_field_params(uint64_t p, fdot_rep_t rep, fdot_field_info_t* out) {
  return fd_fill_params(p, rep, out);
}

fdot_status_t fdot_lambda(uint64_t p, fdot_acc_t acc, uint64_t* lambda) {
  if (!lambda || p < 2) return FDOT_E_INVALID_ARG;
  if ((int)acc < FDOT_ACC_U64 || (int)acc > FDOT_ACC_U64_HYBRID) return FDOT_E_INVALID_ARG;
  *lambda = lambda_of(p, acc);
  return FDOT_OK;
}

fdot_status_t fdot_max_prime(fdot_bound_t kind, uint32_t bits, uint64_t* out) {
  if (!out || bits < 8 || bits > 64) return FDOT_E_INVALID_ARG;
  // Largest integer x satisfying the monotone bound, by bisection, then the
  // nearest prime at or below it.
  auto ok = [&](u128 x) -> bool {
    switch (kind) {
      case FDOT_BOUND_AXPY_SIGNED: return x * (x - 1) <= ((((u128)1) << (bits - 1)) - 1);
      case FDOT_BOUND_AXPY_UNSIGNED: return x * (x - 1) <= ((((u128)1) << bits) - 1);
      case FDOT_BOUND_MONTGOMERY: {
        if (bits > 32) return false;
        const u128 B = (u128)1 << bits;
        return (x - 1) * (x - 1) + x * (B - 1) < B * B;
      }
      case FDOT_BOUND_ZECH_INDEX: return 2 * (x - 1) <= ((((u128)1) << (bits - 1)) - 1);
      default: break;
    }
    return false;
  };
  if ((int)kind < 0 || (int)kind > FDOT_BOUND_ZECH_INDEX) return FDOT_E_INVALID_ARG;
  if (kind == FDOT_BOUND_MONTGOMERY && bits > 32) return FDOT_E_INVALID_ARG;
  u128 lo = 2, hi = (u128)1 << (bits < 64 ? bits : 63);
  if (bits == 64) hi = ((u128)1 << 64);
  while (lo < hi) {
    const u128 mid = (lo + hi + 1) / 2;
    if (ok(mid)) lo = mid; else hi = mid - 1;
  }
  for (u128 x = lo; x >= 2; --x)
    if (x < ((u128)1 << 64) && fd_is_prime_u64((uint64_t)x)) { *out = (uint64_t)x; return FDOT_OK; }
  return FDOT_E_NOT_FOUND;
}

fdot_status_t fdot_choose_rep(uint64_t p, uint64_t n, fdot_rep_t* rep) {
  if (!rep) return FDOT_E_INVALID_ARG;
  if (p < 2 || !fd_is_prime_u64(p)) return FDOT_E_NOT_PRIME;
  fdot_field_info_t info;
  int bits = 0;
  while (bits < 64 && (p >> bits) != 0) ++bits;
  int decade = 0;
  for (uint64_t t = n; t >= 10; t /= 10) ++decade;
  char key[64];
  snprintf(key, sizeof key, "auto.rep.b%d.n%d", bits, decade);
  int64_t tuned = fd_tune(key, -1);
  if (tuned < 0) {
    snprintf(key, sizeof key, "auto.rep.b%d", bits);
    tuned = fd_tune(key, -1);
  }
  if (tuned >= FDOT_REP_ZPZ_U32 && tuned <= FDOT_REP_CENTRED_I8 &&
      fd_fill_params(p, (fdot_rep_t)tuned, &info) == FDOT_OK) {
    *rep = (fdot_rep_t)tuned;
    return FDOT_OK;
  }
  static const fdot_rep_t by_bytes[] = {FDOT_REP_CENTRED_I8, FDOT_REP_ZECH_U16, FDOT_REP_ZPZ_U32,
                                        FDOT_REP_FP64};
  for (fdot_rep_t r : by_bytes)
    if (fd_fill_params(p, r, &info) == FDOT_OK) {
      *rep = r;
      return FDOT_OK;
    }
  return FDOT_E_BOUND;
}

fdot_status_t fdot_host_fold(const fdot_field_info_t* info, fdot_fold_t kind, uint64_t T,
                             uint64_t* out) {
  if (!info || !out) return FDOT_E_INVALID_ARG;
  FieldK k;
  fd_fieldk_from_info(info, &k);
  switch (kind) {
    case FDOT_FOLD_REMAINDER: *out = mod_u64(T, k); return FDOT_OK;
    case FDOT_FOLD_REDC:
      if (!(info->p & 1) || (u128)T >= (u128)info->p << 32) return FDOT_E_INVALID_ARG;
      *out = redc(T, k);
      return FDOT_OK;
    case FDOT_FOLD_FP64:
      if (T > (1ull << 53)) return FDOT_E_INVALID_ARG;
      *out = (uint64_t)fold_f64((double)T, k);
      return FDOT_OK;
    default: break;
  }
  return FDOT_E_INVALID_ARG;
}

fdot_status_t fdot_zech_tables(uint64_t p, uint16_t* value, uint16_t* index, uint16_t* plus1) {
  if (p < 3 || p > 65536) return FDOT_E_BOUND;
  if (!fd_is_prime_u64(p)) return FDOT_E_NOT_PRIME;
  return fd_zech_build(p, fd_primitive_root(p), value, index, plus1) == 0 ? FDOT_OK : FDOT_E_NOMEM;
}

fdot_status_t fdot_field_create(uint64_t p, fdot_rep_t rep, const fdot_options_t* opt,
                                fdot_field_t* out) {
  if (!out) return FDOT_E_INVALID_ARG;
  *out = nullptr;
  fdot_field_info_t I;
  fdot_status_t st = fd_fill_params(p, rep, &I);
  if (st != FDOT_OK) return st;
  fdot_options_t o;
  memset(&o, 0, sizeof o);
  if (opt) {
    o = *opt;
    if (o.reserved[0] || o.reserved[1]) return FDOT_E_INVALID_ARG;
    if (o.algo < FDOT_ALGO_AUTO || o.algo > FDOT_ALGO_HYBRID) return FDOT_E_INVALID_ARG;
    if (!algo_allowed(I.rep, o.algo)) return FDOT_E_UNSUPPORTED;
    if (o.block > delayed_lambda(I)) return FDOT_E_BOUND;
  }
  fdot_field_s* f = new (std::nothrow) fdot_field_s;
  if (!f) return FDOT_E_NOMEM;
  memset(f, 0, sizeof(*f));
  f->info = I;
  f->opt = o;
  f->degree = 1;
  fd_fieldk_from_info(&I, &f->k);
  if (hipGetDevice(&f->device) != hipSuccess) { delete f; return FDOT_E_DEVICE; }
  if (rep == FDOT_REP_ZECH_U16) {
    uint16_t* h = new (std::nothrow) uint16_t[3 * p];
    if (!h) { delete f; return FDOT_E_NOMEM; }
    fd_zech_build(p, I.g, h, h + p, h + 2 * p);
    uint16_t* d = nullptr;
    if (hipMalloc((void**)&d, 3 * p * sizeof(uint16_t)) != hipSuccess) {
      delete[] h; delete f; return FDOT_E_NOMEM;
    }
    if (hipMemcpy(d, h, 3 * p * sizeof(uint16_t), hipMemcpyHostToDevice) != hipSuccess) {
      hipFree(d); delete[] h; delete f; return FDOT_E_DEVICE;
    }
    const fdot_status_t st = fd_zech_packed_upload(h + 2 * p, p, f);
    delete[] h;
    if (st != FDOT_OK) { hipFree(d); delete f; return st; }
    f->d_zval = d;
    f->d_zidx = d + p;
    f->d_zplus1 = d + 2 * p;
    f->k.zval = f->d_zval;
    f->k.zidx = f->d_zidx;
    f->k.zplus1 = f->d_zplus1;
  }
  if (rep == FDOT_REP_CENTRED_I8) {
    // inverses of the centred residues, for elementwise division: c * c^-1
    // = 1 mod p, found by trying every candidate (p < 2^8); 0 maps to 0
    int8_t h[256];
    memset(h, 0, sizeof h);
    const int64_t pp = (int64_t)p, half = (pp - 1) / 2;
    for (int64_t c = -half; c <= half; ++c) {
      if (c == 0) continue;
      for (int64_t d = -half; d <= half; ++d)
        if ((((c * d) % pp) + pp) % pp == 1) { h[c + 128] = (int8_t)d; break; }
    }
    int8_t* d = nullptr;
    if (hipMalloc((void**)&d, sizeof h) != hipSuccess) { delete f; return FDOT_E_NOMEM; }
    if (hipMemcpy(d, h, sizeof h, hipMemcpyHostToDevice) != hipSuccess) {
      hipFree(d); delete f; return FDOT_E_DEVICE;
    }
    f->d_cinv = d;
    f->k.cinv = d;
  }
  *out = f;
  return FDOT_OK;
}

// GF(p^d) (Sec. 2.4.2).  Elements are coefficient vectors c_0..c_{d-1} over
// GF(p), valued c_0 + c_1 p + ...; the powers of X are stepped like a linear
// feedback shift register: multiplying by X shifts the coefficients up and
// folds the overflowing top coefficient back with X^d = -(f_0 + ... +
// f_{d-1} X^{d-1}).  A candidate modulus is primitive exactly when this
// sequence first returns to 1 after q-1 steps.
namespace {
struct ExtStepper {
  uint64_t p;
  int d;
  uint32_t f[16];
  uint32_t c[16];
  uint64_t value() const {
    uint64_t v = 0;
    for (int i = d - 1; i >= 0; --i) v = v * p + c[i];
    return v;
  }
  void times_x() {
    const uint64_t top = c[d - 1];
    for (int i = d - 1; i > 0; --i) c[i] = c[i - 1];
    c[0] = 0;
    if (top)
      for (int i = 0; i < d; ++i) c[i] = (uint32_t)((c[i] + (p - top) * f[i]) % p);
  }
};
}  // namespace

fdot_status_t fdot_field_create_ext(uint64_t p, uint32_t d, fdot_field_t* out) {
  if (!out) return FDOT_E_INVALID_ARG;
  *out = nullptr;
  if (d < 2 || d > 16) return FDOT_E_BOUND;
  if (!fd_is_prime_u64(p)) return FDOT_E_NOT_PRIME;
  uint64_t q = 1;
  for (uint32_t i = 0; i < d; ++i) {
    q *= p;
    if (q > 65536) return FDOT_E_BOUND;  // codes 0..q-1 in 16 bits
  }
  ExtStepper st{};
  st.p = p;
  st.d = (int)d;
  uint64_t low = 0;
  bool found = false;
  for (; low < q && !found; ++low) {
    uint64_t t = low;
    for (uint32_t i = 0; i < d; ++i) { st.f[i] = (uint32_t)(t % p); t /= p; }
    if (st.f[0] == 0) continue;  // X divides the candidate
    for (uint32_t i = 0; i < d; ++i) st.c[i] = 0;
    st.c[0] = 1;
    uint64_t k = 0;
    do { st.times_x(); ++k; } while (st.value() != 1 && k < q);
    found = (k == q - 1);
  }
  if (!found) return FDOT_E_BOUND;
  --low;
  uint16_t* h = new (std::nothrow) uint16_t[3 * q];
  if (!h) return FDOT_E_NOMEM;
  uint16_t *val = h, *idx = h + q, *plus1 = h + 2 * q;
  val[0] = 0;
  idx[0] = 0;
  for (uint32_t i = 0; i < d; ++i) st.c[i] = 0;
  st.c[0] = 1;
  for (uint64_t i = 1; i <= q - 1; ++i) {
    st.times_x();
    const uint64_t v = st.value();
    val[i] = (uint16_t)v;
    idx[v] = (uint16_t)i;
  }
  // plus1[k] = code of 1 + (element coded k): add 1 to the constant coefficient
  for (uint64_t k = 0; k <= q - 1; ++k) {
    const uint64_t v = k == 0 ? 0 : val[k];
    const uint64_t c0 = v % p;
    plus1[k] = idx[v - c0 + (c0 + 1) % p];
  }
  fdot_field_s* f = new (std::nothrow) fdot_field_s;
  if (!f) { delete[] h; return FDOT_E_NOMEM; }
  memset(f, 0, sizeof(*f));
  f->info.p = p;
  f->info.rep = FDOT_REP_ZECH_U16;
  f->info.elem_bytes = 2;
  f->info.table_bytes = 3ull * q * sizeof(uint16_t) + fd_zech_packed_bytes(q);
  f->info.degree = d;
  f->info.q = q;
  uint64_t pd = 1;
  for (uint32_t i = 0; i < d; ++i) pd *= p;
  f->info.modulus = pd + low;
  f->degree = d;
  // kernel constants: codes modulo q-1; -1 = X^((q-1)/2) in odd
  // characteristic, -1 = 1 (negation is the identity) in characteristic 2
  f->k.p = q;
  f->k.p32 = (uint32_t)q;
  f->k.qbar = (uint32_t)(q - 1);
  f->k.half = (p & 1) ? (int32_t)((q - 1) / 2) : 0;
  if (hipGetDevice(&f->device) != hipSuccess) { delete[] h; delete f; return FDOT_E_DEVICE; }
  uint16_t* dev = nullptr;
  if (hipMalloc((void**)&dev, 3 * q * sizeof(uint16_t)) != hipSuccess) {
    delete[] h; delete f; return FDOT_E_NOMEM;
  }
  if (hipMemcpy(dev, h, 3 * q * sizeof(uint16_t), hipMemcpyHostToDevice) != hipSuccess) {
    hipFree(dev); delete[] h; delete f; return FDOT_E_DEVICE;
  }
  const fdot_status_t ust = fd_zech_packed_upload(h + 2 * q, (uint32_t)q, f);
  delete[] h;
  if (ust != FDOT_OK) { hipFree(dev); delete f; return ust; }
  f->d_zval = dev;
  f->d_zidx = dev + q;
  f->d_zplus1 = dev + 2 * q;
  f->k.zval = f->d_zval;
  f->k.zidx = f->d_zidx;
  f->k.zplus1 = f->d_zplus1;
  *out = f;
  return FDOT_OK;
}

fdot_status_t fdot_field_destroy(fdot_field_t f) {
  if (!f) return FDOT_E_INVALID_ARG;
  if (f->d_zval) hipFree(f->d_zval);
  if (f->d_cinv) hipFree(f->d_cinv);
  if (f->d_zpk) hipFree(f->d_zpk);
  delete f;
  return FDOT_OK;
}

fdot_status_t fdot_field_info(fdot_field_t f, fdot_field_info_t* out) {
  if (!f || !out) return FDOT_E_INVALID_ARG;
  *out = f->info;
  return FDOT_OK;
}

}  // extern "C"

extern "C" fdot_status_t fdot_field_create_host(uint64_t p, fdot_rep_t rep, fdot_field_t* out) {
  if (!out) return FDOT_E_INVALID_ARG;
  *out = nullptr;
  fdot_field_info_t I;
  fdot_status_t st = fd_fill_params(p, rep, &I);
  if (st != FDOT_OK) return st;
  fdot_field_s* f = new (std::nothrow) fdot_field_s;
  if (!f) return FDOT_E_NOMEM;
  memset(f, 0, sizeof(*f));
  f->info = I;
  f->info.table_bytes = 0;
  fd_fieldk_from_info(&I, &f->k);
  f->device = -1;
  f->host_only = true;
  f->degree = 1;
  *out = f;
  return FDOT_OK;
}
