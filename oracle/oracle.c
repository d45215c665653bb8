/*
 * Reference oracle for the exact dot product over a word-size prime field
 * (J.-G. Dumas, "Efficient dot product over word-size finite fields").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include, link,
 * load or call this file; only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg use it.  It shares no code, header, table or
 * constant generator with the GPU path.
 *
 * What it computes is the plain definition that every method of the paper
 * reaches exactly (Sec. 3, the delayed, blocked and on-demand schedules all
 * return the same residue): for a representation R with decoding map D_R onto
 * Z/pZ and encoding map E_R its inverse,
 *
 *     dot(x, y) = E_R( sum_{i<n} D_R(x_i) * D_R(y_i)  mod p )
 *
 * with the sum reduced after every single term in 128-bit unsigned arithmetic
 * (acc = (acc + a*b) mod p).  No block length, no Montgomery reduction, no
 * table-driven addition: just the definition, slowly.
 *
 * Representations (Sec. 2):
 *   ZPZ     uint32  residue in [0, p)                      (Sec. 2.1)
 *   MONT    uint32  a*B mod p with B = 2^32                (Sec. 2.2)
 *   FP64    double  integral residue in [0, p)             (Sec. 2.3)
 *   ZECH    uint16  discrete-log index: 0 -> 0, 1 -> q-1,
 *                   g^i -> i for 1 <= i < q-1              (Sec. 2.4)
 *   CENTRED int8    residue in [-(p-1)/2, (p-1)/2]         (Sec. 3.2.2)
 * The Zech generator g is the smallest primitive root mod p (the paper does
 * not name one).
 *
 * Every entry point returns 0 on success and a negative code when an input is
 * not canonical for its representation, p is unsuitable, or memory runs out.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

enum { ORC_ZPZ = 0, ORC_MONT = 1, ORC_FP64 = 2, ORC_ZECH = 3, ORC_CENTRED = 4 };
enum { ORC_OK = 0, ORC_E_ARG = -1, ORC_E_PRIME = -2, ORC_E_NONCANON = -3, ORC_E_NOMEM = -4 };

/* ---------------------------------------------------------------- integers */

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t p) {
  return (uint64_t)(((u128)a * b) % p);
}

static uint64_t powmod(uint64_t b, uint64_t e, uint64_t p) {
  uint64_t r = 1 % p;
  b %= p;
  while (e) {
    if (e & 1) r = mulmod(r, b, p);
    b = mulmod(b, b, p);
    e >>= 1;
  }
  return r;
}

/* Primality by trial division: fine for every p the oracle accepts (< 2^32). */
int orc_is_prime(uint64_t p) {
  if (p < 2) return 0;
  if (p < 4) return 1;
  if (p % 2 == 0) return 0;
  for (uint64_t d = 3; d * d <= p; d += 2)
    if (p % d == 0) return 0;
  return 1;
}

/* Inverse of a modulo p by the extended Euclidean algorithm. */
uint64_t orc_inv_mod(uint64_t a, uint64_t p) {
  int64_t t0 = 0, t1 = 1;
  int64_t r0 = (int64_t)p, r1 = (int64_t)(a % p);
  while (r1 != 0) {
    int64_t q = r0 / r1, tmp;
    tmp = r0 - q * r1; r0 = r1; r1 = tmp;
    tmp = t0 - q * t1; t0 = t1; t1 = tmp;
  }
  if (r0 != 1) return 0; /* not invertible */
  if (t0 < 0) t0 += (int64_t)p;
  return (uint64_t)t0;
}

/* Smallest g whose multiplicative order is p-1: g^((p-1)/f) != 1 for every
 * prime factor f of p-1 (factors found by trial division). */
uint64_t orc_primitive_root(uint64_t p) {
  if (!orc_is_prime(p)) return 0;
  if (p == 2) return 1;
  uint64_t fac[64];
  int nf = 0;
  uint64_t m = p - 1;
  for (uint64_t d = 2; d * d <= m; ++d) {
    if (m % d == 0) {
      fac[nf++] = d;
      while (m % d == 0) m /= d;
    }
  }
  if (m > 1) fac[nf++] = m;
  for (uint64_t g = 2; g < p; ++g) {
    int ok = 1;
    for (int i = 0; i < nf && ok; ++i)
      if (powmod(g, (p - 1) / fac[i], p) == 1) ok = 0;
    if (ok) return g;
  }
  return 0;
}

/* ----------------------------------------------------------- field context */

typedef struct {
  uint64_t p;
  int rep;
  uint64_t g;         /* Zech generator */
  uint64_t b_mod_p;   /* 2^32 mod p   (Montgomery) */
  uint64_t binv;      /* 2^-32 mod p  (Montgomery) */
  uint32_t* zexp;     /* Zech: zexp[i] = g^i mod p for 1 <= i <= p-1 */
  uint32_t* zlog;     /* Zech: zlog[v] = index coding v (zlog[0] = 0)  */
} orc_field;

static void field_free(orc_field* f) {
  free(f->zexp);
  free(f->zlog);
  f->zexp = f->zlog = NULL;
}

static int field_init(orc_field* f, uint64_t p, int rep) {
  memset(f, 0, sizeof(*f));
  f->p = p;
  f->rep = rep;
  if (rep < ORC_ZPZ || rep > ORC_CENTRED) return ORC_E_ARG;
  if (!orc_is_prime(p) || p >= (1ull << 32)) return ORC_E_PRIME;
  if (rep == ORC_MONT) {
    if (p == 2) return ORC_E_PRIME;
    f->b_mod_p = (uint64_t)(((u128)1 << 32) % p);
    f->binv = orc_inv_mod(f->b_mod_p, p);
  } else if (rep == ORC_FP64) {
    if (p > (1ull << 26) * 2) return ORC_E_PRIME; /* residues far inside 2^53 */
  } else if (rep == ORC_ZECH) {
    if (p == 2 || p > 65536) return ORC_E_PRIME;
    f->g = orc_primitive_root(p);
    f->zexp = (uint32_t*)malloc(sizeof(uint32_t) * p);
    f->zlog = (uint32_t*)malloc(sizeof(uint32_t) * p);
    if (!f->zexp || !f->zlog) { field_free(f); return ORC_E_NOMEM; }
    f->zexp[0] = 0;
    f->zlog[0] = 0;
    uint64_t v = 1;
    for (uint64_t i = 1; i <= p - 1; ++i) {
      v = mulmod(v, f->g, p);
      f->zexp[i] = (uint32_t)v; /* g^(p-1) = 1 lands on index q-1 */
      f->zlog[v] = (uint32_t)i;
    }
  } else if (rep == ORC_CENTRED) {
    if (p == 2 || p > 255) return ORC_E_PRIME;
  }
  return ORC_OK;
}

/* Decode element i of array v to its residue in [0,p); -1 if not canonical. */
static int64_t decode(const orc_field* f, const void* v, size_t i) {
  uint64_t p = f->p;
  switch (f->rep) {
    case ORC_ZPZ: {
      uint64_t a = ((const uint32_t*)v)[i];
      return a < p ? (int64_t)a : -1;
    }
    case ORC_MONT: {
      uint64_t a = ((const uint32_t*)v)[i];
      if (a >= p) return -1;
      return (int64_t)mulmod(a, f->binv, p);
    }
    case ORC_FP64: {
      double d = ((const double*)v)[i];
      if (!(d >= 0.0) || d >= (double)p || d != floor(d)) return -1;
      return (int64_t)(uint64_t)d;
    }
    case ORC_ZECH: {
      uint64_t k = ((const uint16_t*)v)[i];
      if (k > p - 1) return -1;
      return (int64_t)f->zexp[k]; /* zexp[0] = 0 codes the zero element */
    }
    case ORC_CENTRED: {
      int64_t c = ((const int8_t*)v)[i];
      int64_t h = (int64_t)(p - 1) / 2;
      if (c < -h || c > h) return -1;
      return c < 0 ? c + (int64_t)p : c;
    }
  }
  return -1;
}

static void encode(const orc_field* f, uint64_t r, void* out, size_t i) {
  uint64_t p = f->p;
  switch (f->rep) {
    case ORC_ZPZ: ((uint32_t*)out)[i] = (uint32_t)r; break;
    case ORC_MONT: ((uint32_t*)out)[i] = (uint32_t)(((u128)r << 32) % p); break;
    case ORC_FP64: ((double*)out)[i] = (double)r; break;
    case ORC_ZECH: ((uint16_t*)out)[i] = (uint16_t)f->zlog[r]; break;
    case ORC_CENTRED:
      ((int8_t*)out)[i] = (int8_t)(r > (p - 1) / 2 ? (int64_t)r - (int64_t)p : (int64_t)r);
      break;
  }
}

/* ------------------------------------------------------------ entry points */

int orc_generator(uint64_t p, uint64_t* g) {
  *g = orc_primitive_root(p);
  return *g ? ORC_OK : ORC_E_PRIME;
}

/* canon[i] in [0,p) -> rep[i] */
int orc_encode_array(uint64_t p, int rep, const uint64_t* canon, void* out, size_t n) {
  orc_field f;
  int rc = field_init(&f, p, rep);
  if (rc) { field_free(&f); return rc; }
  for (size_t i = 0; i < n; ++i) {
    if (canon[i] >= p) { field_free(&f); return ORC_E_NONCANON; }
    encode(&f, canon[i], out, i);
  }
  field_free(&f);
  return ORC_OK;
}

/* rep[i] -> canon[i] in [0,p) */
int orc_decode_array(uint64_t p, int rep, const void* v, uint64_t* canon, size_t n) {
  orc_field f;
  int rc = field_init(&f, p, rep);
  if (rc) { field_free(&f); return rc; }
  for (size_t i = 0; i < n; ++i) {
    int64_t a = decode(&f, v, i);
    if (a < 0) { field_free(&f); return ORC_E_NONCANON; }
    canon[i] = (uint64_t)a;
  }
  field_free(&f);
  return ORC_OK;
}

static int dot_with(const orc_field* f, const void* x, const void* y, size_t n,
                    void* out, size_t out_index) {
  uint64_t acc = 0;
  for (size_t i = 0; i < n; ++i) {
    int64_t a = decode(f, x, i), b = decode(f, y, i);
    if (a < 0 || b < 0) return ORC_E_NONCANON;
    acc = (uint64_t)(((u128)acc + (u128)(uint64_t)a * (uint64_t)b) % f->p);
  }
  encode(f, acc, out, out_index);
  return ORC_OK;
}

/* One dot product; *out receives one element of the representation's type. */
int orc_dot(uint64_t p, int rep, const void* x, const void* y, size_t n, void* out) {
  orc_field f;
  int rc = field_init(&f, p, rep);
  if (rc == ORC_OK) rc = dot_with(&f, x, y, n, out, 0);
  field_free(&f);
  return rc;
}

/* count independent dot products (instance k: xs[k], ys[k], ns[k]) into
 * out[k]; instances are spread over threads, each one is computed exactly as
 * orc_dot computes it. */
int orc_dot_many(uint64_t p, int rep, size_t count, const void* const* xs,
                 const void* const* ys, const uint64_t* ns, void* out) {
  orc_field f;
  int rc = field_init(&f, p, rep);
  if (rc) { field_free(&f); return rc; }
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
  for (long k = 0; k < (long)count; ++k)
    bad |= dot_with(&f, xs[k], ys[k], (size_t)ns[k], out, (size_t)k) != ORC_OK;
  field_free(&f);
  return bad ? ORC_E_NONCANON : ORC_OK;
}

static size_t elem_size(int rep) {
  switch (rep) {
    case ORC_ZPZ: case ORC_MONT: return 4;
    case ORC_FP64: return 8;
    case ORC_ZECH: return 2;
    case ORC_CENTRED: return 1;
  }
  return 0;
}

/* One entry of C = A*B: A row-major M x K (leading dimension lda), B row-major
 * K x N (ldb); entry (i,j) = dot of row i of A with column j of B. */
static int gemm_entry(const orc_field* f, const char* A, size_t lda, const char* B,
                      size_t ldb, size_t K, size_t i, size_t j, uint64_t* r) {
  size_t es = elem_size(f->rep);
  uint64_t acc = 0;
  for (size_t k = 0; k < K; ++k) {
    int64_t a = decode(f, A + (i * lda + k) * es, 0);
    int64_t b = decode(f, B + (k * ldb + j) * es, 0);
    if (a < 0 || b < 0) return ORC_E_NONCANON;
    acc = (uint64_t)(((u128)acc + (u128)(uint64_t)a * (uint64_t)b) % f->p);
  }
  *r = acc;
  return ORC_OK;
}

/* C = A*B mod p, all in representation rep; C row-major with ldc. */
int orc_gemm(uint64_t p, int rep, size_t M, size_t N, size_t K, const void* A,
             size_t lda, const void* B, size_t ldb, void* C, size_t ldc) {
  orc_field f;
  int rc = field_init(&f, p, rep);
  if (rc) { field_free(&f); return rc; }
  size_t es = elem_size(rep);
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (long i = 0; i < (long)M; ++i)
    for (size_t j = 0; j < N; ++j) {
      uint64_t r = 0;
      bad |= gemm_entry(&f, (const char*)A, lda, (const char*)B, ldb, K, (size_t)i, j, &r) != ORC_OK;
      encode(&f, r, (char*)C + ((size_t)i * ldc + j) * es, 0);
    }
  field_free(&f);
  return bad ? ORC_E_NONCANON : ORC_OK;
}

/* Selected entries (rows[t], cols[t]) of C = A*B into out[t] (rep type). */
int orc_gemm_entries(uint64_t p, int rep, size_t K, const void* A, size_t lda,
                     const void* B, size_t ldb, size_t count, const uint64_t* rows,
                     const uint64_t* cols, void* out) {
  orc_field f;
  int rc = field_init(&f, p, rep);
  if (rc) { field_free(&f); return rc; }
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
  for (long t = 0; t < (long)count; ++t) {
    uint64_t r = 0;
    bad |= gemm_entry(&f, (const char*)A, lda, (const char*)B, ldb, K, rows[t], cols[t], &r) != ORC_OK;
    encode(&f, r, out, (size_t)t);
  }
  field_free(&f);
  return bad ? ORC_E_NONCANON : ORC_OK;
}

/* y = A*x mod p, A row-major m x n (lda). */
int orc_gemv(uint64_t p, int rep, size_t m, size_t n, const void* A, size_t lda,
             const void* x, void* y) {
  orc_field f;
  int rc = field_init(&f, p, rep);
  if (rc) { field_free(&f); return rc; }
  size_t es = elem_size(rep);
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (long i = 0; i < (long)m; ++i)
    bad |= dot_with(&f, (const char*)A + (size_t)i * lda * es, x, n, y, (size_t)i) != ORC_OK;
  field_free(&f);
  return bad ? ORC_E_NONCANON : ORC_OK;
}

/* ------------------------------------------------- elementwise operations */

/* The seven basic operations of Sec. 2 (opening), on every element i, by
 * their plain definitions on residues in [0,p):
 *   0 ADD    r = x + y          1 SUB    r = x - y        2 NEG  r = -x
 *   3 MUL    r = x * y          4 DIV    r = x * y^-1 (inverse by the
 *            extended Euclidean algorithm, as Sec. 2.1 does it; y = 0 gives
 *            the zero element, a convention: the paper leaves it undefined)
 *   5 AXPY   r = a * x + y      6 AXPYIN r = a * x + r (r read, then written)
 * each reduced mod p in 128-bit arithmetic, decoded from and encoded to the
 * representation as for the dot product.  a is one element of the
 * representation (read for AXPY and AXPYIN only). */
int orc_elementwise(uint64_t p, int rep, int op, size_t n, const void* a, const void* x,
                    const void* y, void* r) {
  if (op < 0 || op > 6) return ORC_E_ARG;
  orc_field f;
  int rc = field_init(&f, p, rep);
  if (rc) { field_free(&f); return rc; }
  int64_t av = 0;
  if (op == 5 || op == 6) {
    av = decode(&f, a, 0);
    if (av < 0) { field_free(&f); return ORC_E_NONCANON; }
  }
  for (size_t i = 0; i < n; ++i) {
    const int64_t xv = decode(&f, x, i);
    int64_t yv = 0;
    if (op == 0 || op == 1 || op == 3 || op == 4 || op == 5) yv = decode(&f, y, i);
    if (op == 6) yv = decode(&f, r, i);
    if (xv < 0 || yv < 0) { field_free(&f); return ORC_E_NONCANON; }
    const uint64_t u = (uint64_t)xv, v = (uint64_t)yv;
    uint64_t out = 0;
    switch (op) {
      case 0: out = (uint64_t)(((u128)u + v) % p); break;
      case 1: out = (uint64_t)(((u128)u + p - v) % p); break;
      case 2: out = (p - u) % p; break;
      case 3: out = mulmod(u, v, p); break;
      case 4: out = v == 0 ? 0 : mulmod(u, orc_inv_mod(v, p), p); break;
      case 5:
      case 6: out = (uint64_t)(((u128)(uint64_t)av * u + v) % p); break;
    }
    encode(&f, out, r, i);
  }
  field_free(&f);
  return ORC_OK;
}

/* ------------------------------------------- extension fields GF(p^d) */

/* Sec. 2.4.2: the discrete-logarithm representation is the same for a field
 * extension GF(q), q = p^d.  Here an element is a polynomial of degree < d
 * over GF(p), written as the integer c_0 + c_1 p + ... + c_{d-1} p^{d-1}
 * (its "value"), and arithmetic is polynomial arithmetic modulo a monic
 * primitive polynomial f of degree d: the one whose lower coefficients,
 * read as the same kind of integer, are smallest.  The generator is the
 * class of X; code 0 is the zero element, code i (1 <= i <= q-1) is X^i (so
 * q-1 codes 1), as for prime fields.  All arithmetic below works on
 * coefficient arrays; nothing is tabulated except the code <-> value maps,
 * which are built by repeated multiplication by X. */

#define EXT_MAXD 16

typedef struct {
  uint64_t p, q;
  int d;
  uint64_t f[EXT_MAXD + 1];  /* modulus coefficients, f[d] = 1 */
  uint32_t* exp;             /* code -> value (exp[0] = 0) */
  uint32_t* log;             /* value -> code */
} orc_ext;

static void ext_to_coef(const orc_ext* E, uint64_t v, uint64_t* c) {
  for (int i = 0; i < E->d; ++i) { c[i] = v % E->p; v /= E->p; }
}
static uint64_t ext_from_coef(const orc_ext* E, const uint64_t* c) {
  uint64_t v = 0;
  for (int i = E->d - 1; i >= 0; --i) v = v * E->p + c[i];
  return v;
}
static uint64_t ext_add(const orc_ext* E, uint64_t a, uint64_t b) {
  uint64_t ca[EXT_MAXD], cb[EXT_MAXD];
  ext_to_coef(E, a, ca); ext_to_coef(E, b, cb);
  for (int i = 0; i < E->d; ++i) ca[i] = (ca[i] + cb[i]) % E->p;
  return ext_from_coef(E, ca);
}
static uint64_t ext_neg(const orc_ext* E, uint64_t a) {
  uint64_t ca[EXT_MAXD];
  ext_to_coef(E, a, ca);
  for (int i = 0; i < E->d; ++i) ca[i] = (E->p - ca[i]) % E->p;
  return ext_from_coef(E, ca);
}
/* schoolbook product, then reduction by the monic modulus from the top */
static uint64_t ext_mul(const orc_ext* E, uint64_t a, uint64_t b) {
  uint64_t ca[EXT_MAXD], cb[EXT_MAXD], t[2 * EXT_MAXD] = {0};
  ext_to_coef(E, a, ca); ext_to_coef(E, b, cb);
  const int d = E->d;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) t[i + j] = (t[i + j] + ca[i] * cb[j]) % E->p;
  for (int k = 2 * d - 2; k >= d; --k) {
    const uint64_t c = t[k];
    if (!c) continue;
    for (int i = 0; i <= d; ++i) t[k - d + i] = (t[k - d + i] + (E->p - c) * E->f[i]) % E->p;
  }
  return ext_from_coef(E, t);
}
static uint64_t ext_pow(const orc_ext* E, uint64_t a, uint64_t e) {
  uint64_t r = 1;
  while (e) {
    if (e & 1) r = ext_mul(E, r, a);
    a = ext_mul(E, a, a);
    e >>= 1;
  }
  return r;
}

static void ext_free(orc_ext* E) {
  free(E->exp); free(E->log);
  E->exp = E->log = NULL;
}

/* Find the modulus: candidates in increasing order of their lower
 * coefficients; f is primitive exactly when X, multiplied by itself, first
 * returns to 1 after q-1 steps (X has order q-1). */
static int ext_init(orc_ext* E, uint64_t p, int d) {
  memset(E, 0, sizeof(*E));
  if (d < 2 || d > EXT_MAXD || !orc_is_prime(p)) return ORC_E_PRIME;
  uint64_t q = 1;
  for (int i = 0; i < d; ++i) { q *= p; if (q > 65536) return ORC_E_PRIME; }
  E->p = p; E->q = q; E->d = d;
  E->exp = (uint32_t*)malloc(sizeof(uint32_t) * q);
  E->log = (uint32_t*)malloc(sizeof(uint32_t) * q);
  if (!E->exp || !E->log) { ext_free(E); return ORC_E_NOMEM; }
  const uint64_t x = p;  /* the value of the polynomial X */
  for (uint64_t low = 0; low < q; ++low) {
    uint64_t c[EXT_MAXD];
    ext_to_coef(E, low, c);
    if (c[0] == 0) continue;  /* X divides f */
    for (int i = 0; i < d; ++i) E->f[i] = c[i];
    E->f[d] = 1;
    uint64_t v = 1, k = 0;
    do { v = ext_mul(E, v, x); ++k; } while (v != 1 && k < q);
    if (k != q - 1) continue;
    E->exp[0] = 0; E->log[0] = 0;
    v = 1;
    for (uint64_t i = 1; i <= q - 1; ++i) {
      v = ext_mul(E, v, x);
      E->exp[i] = (uint32_t)v;
      E->log[v] = (uint32_t)i;
    }
    return ORC_OK;
  }
  ext_free(E);
  return ORC_E_PRIME;
}

/* The modulus as an integer: f(p) = sum f_i p^i, including p^d. */
int orc_ext_modulus(uint64_t p, int d, uint64_t* modulus) {
  orc_ext E;
  int rc = ext_init(&E, p, d);
  if (rc == ORC_OK) {
    uint64_t v = 0;
    for (int i = d; i >= 0; --i) v = v * p + E.f[i];
    *modulus = v;
  }
  ext_free(&E);
  return rc;
}

/* Codes <-> values (uint16 codes, uint32 values). */
int orc_ext_encode(uint64_t p, int d, const uint32_t* values, uint16_t* codes, size_t n) {
  orc_ext E;
  int rc = ext_init(&E, p, d);
  for (size_t i = 0; rc == ORC_OK && i < n; ++i) {
    if (values[i] >= E.q) rc = ORC_E_NONCANON;
    else codes[i] = (uint16_t)E.log[values[i]];
  }
  ext_free(&E);
  return rc;
}
int orc_ext_decode(uint64_t p, int d, const uint16_t* codes, uint32_t* values, size_t n) {
  orc_ext E;
  int rc = ext_init(&E, p, d);
  for (size_t i = 0; rc == ORC_OK && i < n; ++i) {
    if (codes[i] >= E.q) rc = ORC_E_NONCANON;
    else values[i] = E.exp[codes[i]];
  }
  ext_free(&E);
  return rc;
}

/* sum x_i y_i in GF(q), on codes: every product and sum in polynomial
 * arithmetic, the result encoded to its code. */
int orc_ext_dot(uint64_t p, int d, const uint16_t* x, const uint16_t* y, size_t n,
                uint16_t* out) {
  orc_ext E;
  int rc = ext_init(&E, p, d);
  uint64_t acc = 0;
  for (size_t i = 0; rc == ORC_OK && i < n; ++i) {
    if (x[i] >= E.q || y[i] >= E.q) { rc = ORC_E_NONCANON; break; }
    acc = ext_add(&E, acc, ext_mul(&E, E.exp[x[i]], E.exp[y[i]]));
  }
  if (rc == ORC_OK) *out = (uint16_t)E.log[acc];
  ext_free(&E);
  return rc;
}

/* The seven elementwise operations of Sec. 2 in GF(q) on codes, numbered as
 * for prime fields; the inverse is a^(q-2); a zero divisor gives zero. */
int orc_ext_elementwise(uint64_t p, int d, int op, size_t n, const uint16_t* a,
                        const uint16_t* x, const uint16_t* y, uint16_t* r) {
  if (op < 0 || op > 6) return ORC_E_ARG;
  orc_ext E;
  int rc = ext_init(&E, p, d);
  if (rc) { ext_free(&E); return rc; }
  /* every code read must be canonical, in [0, q-1] (Sec. 2.4): refuse the
   * call before writing anything */
  const int reads_y = op == 0 || op == 1 || op == 3 || op == 4 || op == 5;
  if ((op == 5 || op == 6) && a[0] >= E.q) { ext_free(&E); return ORC_E_NONCANON; }
  for (size_t i = 0; i < n; ++i)
    if (x[i] >= E.q || (reads_y && y[i] >= E.q) || (op == 6 && r[i] >= E.q)) {
      ext_free(&E);
      return ORC_E_NONCANON;
    }
  const uint64_t av = (op == 5 || op == 6) ? E.exp[a[0]] : 0;
  for (size_t i = 0; i < n; ++i) {
    const uint64_t u = E.exp[x[i]];
    uint64_t v = 0;
    if (op == 0 || op == 1 || op == 3 || op == 4 || op == 5) v = E.exp[y[i]];
    if (op == 6) v = E.exp[r[i]];
    uint64_t out = 0;
    switch (op) {
      case 0: out = ext_add(&E, u, v); break;
      case 1: out = ext_add(&E, u, ext_neg(&E, v)); break;
      case 2: out = ext_neg(&E, u); break;
      case 3: out = ext_mul(&E, u, v); break;
      case 4: out = v == 0 ? 0 : ext_mul(&E, u, ext_pow(&E, v, E.q - 2)); break;
      case 5:
      case 6: out = ext_add(&E, ext_mul(&E, av, u), v); break;
    }
    r[i] = (uint16_t)E.log[out];
  }
  ext_free(&E);
  return ORC_OK;
}

int orc_version(void) { return 1; }

/* Threads of the batched entry points (for timing the oracle; every result is
 * computed the same way whatever the count).  n <= 0: one per processor. */
void orc_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
  (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
