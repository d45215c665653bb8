/*
 * fdot.h -- exact linear algebra over a word-size prime field GF(p) on AMD
 * Instinct MI355X (gfx950).
 *
 * The operation is the one studied in J.-G. Dumas, "Efficient dot product over
 * word-size finite fields": the exact dot product of two vectors over GF(p)
 * (Sec. 1), computed in one of the element representations of Sec. 2, with the
 * modular reduction delayed as long as the accumulator cannot overflow
 * (Sec. 3.1 Eq. 1 and the blocked loop of Sec. 3.2), or performed on demand
 * (Sec. 3.3).  Matrix-vector and matrix-matrix products are the same
 * contraction per output entry (Sec. 1 names them as the dot product's
 * users).
 *
 * Conventions for every call:
 *  - All functions are plain C, return fdot_status_t (0 = success, < 0 = error)
 *    and never throw.
 *  - "device" pointers are HIP device allocations owned by the caller; the
 *    library never frees them.  "host" pointers are ordinary host memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Compute calls only enqueue work on it and return; argument errors are
 *    reported synchronously, launch errors as FDOT_E_DEVICE.
 *  - Vectors and matrices are dense; matrices are row-major with a leading
 *    dimension counted in elements.
 *  - Inputs must be canonical in their representation (below).  The hot path
 *    does not check this; a non-canonical input gives an unspecified result.
 *  - Results are written in the input representation and in its canonical
 *    form, so exactly one bit pattern is correct (the conversions themselves
 *    are not part of a dot product, Sec. 3).
 */
#ifndef FDOT_H
#define FDOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FDOT_OK = 0,
  FDOT_E_INVALID_ARG = -1, /* null pointer, bad size, bad enum, misaligned ld */
  FDOT_E_NOT_PRIME = -2,   /* p is not prime */
  FDOT_E_BOUND = -3,       /* p outside the representation's bound */
  FDOT_E_UNSUPPORTED = -4, /* no such form for this representation/algorithm */
  FDOT_E_DEVICE = -5,      /* a HIP call failed */
  FDOT_E_NOMEM = -6,       /* device or host allocation failed */
  FDOT_E_BUSY = -7,        /* queue full / workspace cannot grow now */
  FDOT_E_NOT_FOUND = -8,   /* unknown ticket or key */
  FDOT_E_NONCANON = -9     /* an input is not canonical in its representation
                              (reported only where validation was asked for) */
} fdot_status_t;

/* Element representations (Sec. 2).  Storage type and canonical range:
 *  ZPZ_U32     uint32  a in [0, p), p < 2^32                    (Sec. 2.1)
 *  MONT_U32    uint32  a*B mod p, B = 2^32, odd p < 2^32         (Sec. 2.2)
 *  FP64        double  integral a in [0, p), (p-1)^2 <= 2^53    (Sec. 2.3)
 *  ZECH_U16    uint16  0 -> 0, 1 -> p-1, g^i -> i (1 <= i < p-1)
 *                      with g the smallest primitive root, p <= 65521
 *                                                                (Sec. 2.4)
 *  CENTRED_I8  int8    a in [-(p-1)/2, (p-1)/2], odd p < 256    (Sec. 3.2.2)
 */
typedef enum {
  FDOT_REP_ZPZ_U32 = 0,
  FDOT_REP_MONT_U32 = 1,
  FDOT_REP_FP64 = 2,
  FDOT_REP_ZECH_U16 = 3,
  FDOT_REP_CENTRED_I8 = 4,
  FDOT_REP_FORCE_INT32 = 0x7fffffff /* not a representation: every int32 value is a
                                       valid fdot_rep_t, so an unknown one can be
                                       checked and refused */
} fdot_rep_t;

/* Accumulation schedules of Sec. 3 (every one returns the same result). */
typedef enum {
  FDOT_ALGO_AUTO = 0,        /* the library's (tuned) choice */
  FDOT_ALGO_DELAYED = 1,     /* Sec. 3.1-3.2: reduce once per block of at most
                                lambda products (lambda from Eq. 1 with the
                                carried residue); for MONT_U32 one Montgomery
                                reduction per block (Sec. 3.2.1) */
  FDOT_ALGO_PERTERM = 2,     /* Sec. 2.1 AXPY: reduce after every product */
  FDOT_ALGO_OVERFLOW = 3,    /* Sec. 3.3: let the 64-bit sum wrap, detect the
                                wrap by t+ab < ab and add CORR = 2^64 mod p;
                                for MONT_U32 one extra reduction at the end */
  FDOT_ALGO_ZECH_TPLUS1 = 4, /* Sec. 2.4: products by index addition, sums by
                                Zech addition through the plus-one table */
  FDOT_ALGO_ZECH_EXP = 5,    /* Sec. 2.4 + 3.1: products by index addition,
                                then the value table and a delayed integer sum */
  FDOT_ALGO_HYBRID = 6,      /* Sec. 3.4: blocks of lambda products with
                                lambda p (p-1) < 2^64 (Eq. 2, strict reading)
                                added without a test, one wrap test and CORR
                                per block; ZPZ_U32 and MONT_U32 (one extra
                                reduction at the end); where lambda < 2 the
                                same as OVERFLOW */
  FDOT_ALGO_FORCE_INT32 = 0x7fffffff /* not a schedule (32-bit range, as above) */
} fdot_algo_t;

/* Accumulator kinds for the bound calculator. */
typedef enum {
  FDOT_ACC_U64 = 0,         /* unsigned 64-bit, carried residue  (Eq. 1)       */
  FDOT_ACC_U32 = 1,         /* unsigned 32-bit, carried residue  (Eq. 1)       */
  FDOT_ACC_F64 = 2,         /* double: exact integers up to 2^53 (Eq. 1, m=53) */
  FDOT_ACC_I32_CENTRED = 3, /* signed 32-bit, centred operands   (Sec. 3.2.2)  */
  FDOT_ACC_F64_CENTRED = 4, /* double, centred operands: |sum| <= 2^53        */
  FDOT_ACC_MONT_REDC = 5,   /* products summed before one Montgomery reduction
                               with B = 2^32: sum < p*B          (Sec. 2.2)   */
  FDOT_ACC_U64_HYBRID = 6,  /* Eq. 2 strict: lambda*p*(p-1) < 2^64 (Sec. 3.4) */
  FDOT_ACC_FORCE_INT32 = 0x7fffffff
} fdot_acc_t;

/* Prime bounds printed by the paper, for the bound calculator. */
typedef enum {
  FDOT_BOUND_AXPY_SIGNED = 0,   /* p(p-1) <= 2^(m-1)-1            (Sec. 2.1) */
  FDOT_BOUND_AXPY_UNSIGNED = 1, /* p(p-1) <= 2^m-1                (Sec. 2.1) */
  FDOT_BOUND_MONTGOMERY = 2,    /* (p-1)^2 + p(B-1) < B^2, B=2^m  (Sec. 2.2) */
  FDOT_BOUND_ZECH_INDEX = 3,    /* 2(p-1) <= 2^(m-1)-1            (Sec. 2.4) */
  FDOT_BOUND_FORCE_INT32 = 0x7fffffff
} fdot_bound_t;

/* Fold primitives (the reductions of Sec. 2), for host-side checks. */
typedef enum {
  FDOT_FOLD_REMAINDER = 0, /* T mod p by a precomputed reciprocal (2-by-1
                              division by an invariant divisor), any T < 2^64 */
  FDOT_FOLD_REDC = 1,      /* Montgomery: T * 2^-32 mod p, T < p*2^32 (Sec. 2.2) */
  FDOT_FOLD_FP64 = 2,      /* T - floor(T*invP)*P with one +-P correction,
                              T <= 2^53 (Sec. 2.3) */
  FDOT_FOLD_FORCE_INT32 = 0x7fffffff
} fdot_fold_t;

/* Constants of a field (all host values). */
typedef struct {
  uint64_t p;
  int32_t rep;               /* fdot_rep_t */
  uint32_t elem_bytes;       /* storage size of one element */
  uint64_t lambda_u64;       /* FDOT_ACC_U64 block length */
  uint64_t lambda_f64;       /* FDOT_ACC_F64 block length (0 if p too large) */
  uint64_t lambda_i32c;      /* FDOT_ACC_I32_CENTRED block length */
  uint64_t lambda_redc;      /* FDOT_ACC_MONT_REDC block length (odd p) */
  uint64_t corr;             /* 2^64 mod p (Sec. 3.3) */
  uint32_t norm_shift;       /* s with 2^31 <= p*2^s < 2^32 */
  uint32_t recip;            /* floor((2^64-1)/(p*2^s)) - 2^32 */
  uint32_t n_im;             /* -p^-1 mod 2^32 (odd p; Sec. 2.2) */
  uint32_t b_mod_p;          /* 2^32 mod p: Montgomery form of 1 */
  uint32_t binv_mod_p;       /* 2^-32 mod p (odd p) */
  uint32_t b2_mod_p;         /* 2^64 mod p */
  uint32_t g;                /* smallest primitive root (Zech; 0 otherwise) */
  uint32_t reserved;
  double inv_p;              /* 1.0/p rounded to nearest */
  uint64_t table_bytes;      /* device bytes held by the field's tables */
  uint32_t degree;           /* d: the field has q = p^d elements (1: prime field) */
  uint32_t reserved2;
  uint64_t q;                /* p^d */
  uint64_t modulus;          /* d > 1: the modulus polynomial f as f(p) */
} fdot_field_info_t;

/* One instance of a batched dot product (device-resident array). */
typedef struct {
  const void* x; /* device, n elements of the field's storage type */
  const void* y; /* device, n elements */
  uint64_t n;
} fdot_desc_t;

/* One instance of a batched dot product over one of several fields. */
typedef struct {
  const void* x;   /* device, n elements of the field's storage type */
  const void* y;   /* device, n elements */
  uint64_t n;
  uint32_t field;  /* index into the call's array of fields */
  uint32_t reserved;
} fdot_mixed_desc_t;

typedef struct fdot_field_s* fdot_field_t;

/* ------------------------------------------------------------------ host only
 * These touch no GPU. */

const char* fdot_status_string(int status);
int fdot_version(void);

/* Validate p for `rep` (prime; within the representation bound of Sec. 2)
 * and fill every constant of the field; no device tables are built. */
fdot_status_t fdot_field_params(uint64_t p, fdot_rep_t rep, fdot_field_info_t* out);

/* Largest block length lambda for accumulator `acc` (Sec. 3.1 Eq. 1 with the
 * residue carried between blocks, Sec. 3.2.2, Sec. 3.4 Eq. 2, Sec. 2.2).
 * 0 means not even one product fits. */
fdot_status_t fdot_lambda(uint64_t p, fdot_acc_t acc, uint64_t* lambda);

/* Largest prime below the bound `kind` for word size `bits` (Sec. 2.1, 2.2,
 * 2.4); bits in [8, 64]. */
fdot_status_t fdot_max_prime(fdot_bound_t kind, uint32_t bits, uint64_t* p);

/* The representation to hold GF(p) vectors in for dot products of length
 * about n on this device: the switch between representations by prime size,
 * vector size and architecture that the Conclusion calls for.  A measured
 * choice written by the autotuner at install time (tune keys
 * auto.rep.b<bits>.n<decade>, then auto.rep.b<bits>, bits = bit length of p,
 * decade = floor(log10 n)) wins when that representation admits p.
 * Otherwise the model for a device where the streaming dot is bound by HBM
 * bandwidth: the admissible representation with the fewest bytes per element
 * (centred int8, then discrete logarithms in 16 bits, then classical 32-bit
 * residues, then doubles).  Host only; FDOT_E_BOUND if no representation
 * admits p, FDOT_E_NOT_PRIME if p is not prime. */
fdot_status_t fdot_choose_rep(uint64_t p, uint64_t n, fdot_rep_t* rep);

/* Evaluate one fold primitive on the host with the field's constants, with
 * the same code the kernels run.  Returns FDOT_E_INVALID_ARG when T is
 * outside the primitive's input range. */
fdot_status_t fdot_host_fold(const fdot_field_info_t* info, fdot_fold_t kind,
                             uint64_t T, uint64_t* out);

/* The Zech tables for a prime p <= 65521 with the smallest primitive root g
 * (Sec. 2.4).  Each host array has p entries:
 *   value[i] = g^i mod p for 1 <= i <= p-1, value[0] = 0 (index 0 codes 0);
 *   index[v] = Zech code of v (index[0] = 0, index[1] = p-1);
 *   plus1[k] = h with g^h = 1 + g^k for 1 <= k <= p-1, 0 when 1 + g^k = 0;
 *              plus1[0] = p-1 (1 + 0 = 1).
 * Any pointer may be NULL. */
fdot_status_t fdot_zech_tables(uint64_t p, uint16_t* value, uint16_t* index,
                               uint16_t* plus1);

/* ----------------------------------------------------------------- fields */

/* Options of a field (fdot_field_create); NULL or all zero = defaults.
 *  validate: nonzero = every compute call on the field (fdot_modp*,
 *    fdot_modp_many*, fgemv_modp, fgemm_modp, fdot_elementwise) first counts
 *    the non-canonical elements of its inputs with a check kernel on the
 *    call's stream and waits for the result, so the call becomes synchronous;
 *    when any is found it returns FDOT_E_NONCANON and computes nothing.  A
 *    stream under graph capture cannot wait: FDOT_E_UNSUPPORTED there.
 *    Canonical ranges are those of fdot_rep_t (Sec. 2.1: a residue is an
 *    integer in [0, p)).  fdot_modp_many_mixed does not validate.
 *  algo: the schedule (fdot_algo_t) used where a dot-product call asks for
 *    FDOT_ALGO_AUTO; 0 = the library's choice.  FDOT_E_UNSUPPORTED at
 *    creation for a schedule the representation does not have.
 *  block: the delayed schedules of the dot-product, batched and
 *    matrix-vector forms fold each accumulator after at most block products
 *    (rounded down to the kernel's vectors, at least one vector) instead of
 *    lambda; 0 = lambda.  FDOT_E_BOUND above lambda of the representation's
 *    delayed schedule (lambda_u64, lambda_redc, lambda_f64, lambda_i32c, or
 *    (2^32-1)/(p-1) values per sum for discrete logarithms).  Matrix
 *    products keep their own K-blocks. */
typedef struct {
  uint32_t validate;
  int32_t algo;
  uint64_t block;
  uint64_t reserved[2]; /* zero */
} fdot_options_t;

/* Create a field: validates like fdot_field_params, then uploads its device
 * tables (Zech) to the current device.  opt may be NULL.  The handle is
 * immutable and may be shared by threads and streams; destroy it once no
 * enqueued work uses it. */
fdot_status_t fdot_field_create(uint64_t p, fdot_rep_t rep, const fdot_options_t* opt,
                                fdot_field_t* out);
/* A field handle with its constants only (no device tables, no GPU touched):
 * usable where only the field's description is needed (request planning, the
 * request server in fake-device mode); compute calls on it return
 * FDOT_E_UNSUPPORTED. */
fdot_status_t fdot_field_create_host(uint64_t p, fdot_rep_t rep, fdot_field_t* out);
fdot_status_t fdot_field_destroy(fdot_field_t f);

/* GF(q), q = p^d with d >= 2 and q <= 65536, in the discrete-logarithm
 * representation (Sec. 2.4.2: the representation is unchanged for field
 * extensions, where the classical one would need polynomial arithmetic).
 * An element is a polynomial c_0 + c_1 X + ... + c_{d-1} X^{d-1} over GF(p);
 * its canonical value (fdot_encode / fdot_decode) is the integer
 * c_0 + c_1 p + ... + c_{d-1} p^{d-1}.  Arithmetic is modulo the monic
 * primitive polynomial f of degree d whose lower coefficients, read the same
 * way, are smallest; the generator is the class of X, and codes are as for
 * prime fields (0 = zero, i = X^i, q-1 = 1).  Supported: encode, decode,
 * fdot_modp and fdot_modp_many, fdot_elementwise.  Dot-product schedules:
 * FDOT_ALGO_ZECH_TPLUS1, sums through the plus-one table (any p); and for
 * p = 2 FDOT_ALGO_ZECH_EXP, each product's value (its coefficient bits)
 * looked up and the values summed by exclusive or, which is polynomial
 * addition over GF(2).  FDOT_ALGO_AUTO is ZECH_EXP for p = 2 and
 * ZECH_TPLUS1 otherwise; other schedules return FDOT_E_UNSUPPORTED.  The
 * matrix forms and fdot_modp_many_mixed return FDOT_E_UNSUPPORTED /
 * FDOT_E_INVALID_ARG.  FDOT_E_NOT_PRIME / FDOT_E_BOUND for a p that is not
 * prime or a q out of range. */
fdot_status_t fdot_field_create_ext(uint64_t p, uint32_t d, fdot_field_t* out);
fdot_status_t fdot_field_info(fdot_field_t f, fdot_field_info_t* out);

/* Count the non-canonical elements of x[0 .. n-1] (stored values of the
 * field's representation, device, aligned to the element size) and add the
 * count to *count (device, 8-byte aligned; the caller clears it).  Enqueued
 * on the stream; no wait. */
fdot_status_t fdot_validate(fdot_field_t f, const void* x, size_t n, uint64_t* count,
                            void* stream);

/* Conversions (Sec. 2; untimed by the paper's convention, Sec. 3).
 * canon: device uint32 residues in [0, p); rep: device storage array. */
fdot_status_t fdot_encode(fdot_field_t f, const uint32_t* canon, void* rep,
                          size_t n, void* stream);
fdot_status_t fdot_decode(fdot_field_t f, const void* rep, uint32_t* canon,
                          size_t n, void* stream);

/* --------------------------------------------------- elementwise operations */

/* The seven basic operations of Sec. 2 (opening) on vectors, elementwise. */
typedef enum {
  FDOT_EW_ADD = 0,    /* r = x + y */
  FDOT_EW_SUB = 1,    /* r = x - y */
  FDOT_EW_NEG = 2,    /* r = -x */
  FDOT_EW_MUL = 3,    /* r = x * y */
  FDOT_EW_DIV = 4,    /* r = x / y; a zero divisor gives the zero element */
  FDOT_EW_AXPY = 5,   /* r = a * x + y */
  FDOT_EW_AXPYIN = 6, /* r = a * x + r */
  FDOT_EW_FORCE_INT32 = 0x7fffffff
} fdot_ew_op_t;

/* r[i] = op(x[i], y[i]) for i < n over GF(p) in the field's representation
 * (Sec. 2.1-2.4 give each operation per representation).  x, y and r are
 * device arrays of the representation's element type, aligned to its size;
 * y is read by ADD, SUB, MUL, DIV and AXPY (NULL allowed otherwise); r may be
 * the same array as x or y (not a partial overlap).  alpha points to one
 * element of the representation in host memory, read at the call, for AXPY
 * and AXPYIN (NULL allowed otherwise).  Inputs must be canonical.  n = 0
 * does nothing.  Enqueued on the stream. */
fdot_status_t fdot_elementwise(fdot_field_t f, fdot_ew_op_t op, size_t n, const void* alpha,
                               const void* x, const void* y, void* r, void* stream);

/* ------------------------------------------------------- measured peaks */

/* Calibration kernels, no part of the method: they measure the two roofs the
 * method's kernels are held against (HBM bandwidth for the streaming forms,
 * matrix-core rate for the matrix product), so that fractions can be quoted
 * against measured as well as datasheet peaks.
 *
 * fdot_calib_read: *result = the sum mod 2^64 of the n_words 32-bit words at
 * x, each read once by 16-byte nontemporal loads.  x: device, 16-byte
 * aligned (may be NULL when n_words is 0), n_words a multiple of 4; result: device, 8-byte aligned,
 * overwritten (cleared by a kernel first, so the call may be captured).
 * blocks: workgroups of 256 threads (0 = 8 per compute unit); unroll: loads
 * in flight per thread, 4 or 8.  FDOT_E_INVALID_ARG otherwise. */
fdot_status_t fdot_calib_read(const void* x, size_t n_words, uint32_t blocks, uint32_t unroll,
                              uint64_t* result, void* stream);

/* fdot_calib_mfma: each wavefront of `blocks` workgroups of 512 threads
 * (0 = 2 per compute unit) runs `iters` rounds of four independent matrix
 * products on register operands.  kind 0: int8 32x32x32 products with int32
 * accumulation, every left operand element a and right one b (integers in
 * [-128, 127]), result int32; kind 1: FP64 16x16x4 products, result double;
 * kind 2: int8 32x32x32 on pseudo-random operand bytes (a = seed, an integer
 * in [0, 2^32); b unused): chain c of lane l holds the words
 * h(a ^ h(256 l + 4 c + w)) of the left operand and h(a ^ h(256 l + 128 + w))
 * of the right one, w < 4, h the lowbias32 integer hash.  Matrix-core power,
 * and so the clock, depends on operand bits: kinds 0 and 1 measure the issue
 * rate, kind 2 what random data can reach.  result: device array of two
 * elements, 8-byte aligned; result[0] = element 0 of the first wavefront's
 * first accumulator, i.e. iters * 32 * a * b (kind 0, int32, wrapping),
 * iters * 4 * a * b (kind 1), iters * (bytewise dot of lanes 0 and 32)
 * (kind 2, wrapping); result[1] is a sink that keeps the other accumulators
 * live.  *ops (host, may be NULL) = operations executed, two per
 * multiply-add.  FDOT_E_INVALID_ARG for another kind or operand. */
fdot_status_t fdot_calib_mfma(int kind, uint32_t blocks, uint32_t iters, double a, double b,
                              void* result, uint64_t* ops, void* stream);

/* ------------------------------------------------------------ dot products */

/* result[0] = sum_{i<n} x_i*y_i over GF(p) (Sec. 1, Sec. 3), x, y, result on
 * the device in the field's representation.  n = 0 gives the encoded zero;
 * x == y is allowed.  Pointers must be aligned to the element size. */
fdot_status_t fdot_modp(fdot_field_t f, const void* x, const void* y, size_t n,
                        void* result, void* stream);
fdot_status_t fdot_modp_algo(fdot_field_t f, fdot_algo_t algo, const void* x,
                             const void* y, size_t n, void* result, void* stream);

/* results[k] = dot of desc[k] for k < count, one launch sequence for the whole
 * batch (uneven lengths allowed).  desc and results are device arrays. */
fdot_status_t fdot_modp_many(fdot_field_t f, size_t count, const fdot_desc_t* desc,
                             void* results, void* stream);
fdot_status_t fdot_modp_many_algo(fdot_field_t f, fdot_algo_t algo, size_t count,
                                  const fdot_desc_t* desc, void* results, void* stream);

/* For callers that cannot allocate device memory at the call: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, results and kernels as fdot_modp_many_algo, but the batch's
 * device scratch (a combination word per pair and the plan of the batch,
 * about 1.5 MiB) is a fixed array inside the library, one copy per GPU, held
 * until the process ends; the call makes no device allocation.  count may be
 * at most FDOT_NOALLOC_MAX_PAIRS (FDOT_E_INVALID_ARG above it).  Every call on
 * one GPU shares that GPU's array: calls that overlap on one GPU (on two
 * streams, or from two threads) race and their results are unspecified;
 * calls ordered on one stream are safe.  Each call first clears its pairs'
 * combination words with a kernel, so a call may be captured into a graph
 * and replayed. */
#define FDOT_NOALLOC_MAX_PAIRS 65536
fdot_status_t fdot_modp_many_noalloc(fdot_field_t f, fdot_algo_t algo, size_t count,
                                     const fdot_desc_t* desc, void* results, void* stream);

/* results[k] = dot of desc[k] over fields[desc[k].field], k < count: one batch
 * over several primes (Sec. 1: the dot product as a building block; a request
 * stream mixes fields).  fields is a host array of nfields prime fields of one
 * representation (the results array has its element type); desc and results
 * are device arrays.  For each field the batched path runs once with the
 * other fields' pairs masked to length 0, and a merge keeps each pair's own
 * result.  A pair whose field index is >= nfields has its result left
 * unwritten.  FDOT_E_INVALID_ARG for mixed representations or an extension
 * field. */
fdot_status_t fdot_modp_many_mixed(size_t count, const fdot_mixed_desc_t* desc,
                                   const fdot_field_t* fields, size_t nfields, void* results,
                                   void* stream);

/* ----------------------------------------------------------- matrix forms */

/* y = A x over GF(p): A is m x n row-major (lda >= n), x has n entries, y has
 * m entries; all on the device in the field's representation. */
fdot_status_t fgemv_modp(fdot_field_t f, size_t m, size_t n, const void* A,
                         size_t lda, const void* x, void* y, void* stream);

/* C = A B over GF(p): A M x K (lda >= K), B K x N (ldb >= N), C M x N
 * (ldc >= N), row-major device arrays in the field's representation.  The
 * contraction runs on matrix cores when exactness allows it (FP64 when the
 * field's residues fit an exact double block, int8 for CENTRED_I8), cut into
 * K-blocks that never exceed the exact range before a mod-p fold. */
fdot_status_t fgemm_modp(fdot_field_t f, size_t M, size_t N, size_t K, const void* A,
                         size_t lda, const void* B, size_t ldb, void* C, size_t ldc,
                         void* stream);

/* ------------------------------------------------------ runtime / tuning */

/* Pre-size the per-stream workspace for batches of up to `count` instances.
 * Call before capturing a stream into a HIP graph: a capture cannot allocate. */
fdot_status_t fdot_workspace_reserve(void* stream, size_t count);

/* Kernel trace, for measuring a streaming kernel apart from the launches
 * around it (a batched call is a plan launch and the streaming kernel).
 * While enabled, every streaming dot-product kernel (the single form of
 * fdot_modp*, the batched kernel of fdot_modp_many*) is bracketed by a pair
 * of HIP events recorded on the call's own stream.  fdot_trace_enable(1)
 * starts a new record (event pairs are created on first use and reused, at
 * most 65536 per record); fdot_trace_enable(0) stops recording.
 * fdot_trace_read waits for the recorded events and writes the device time
 * of each traced kernel in milliseconds, in launch order, to ms[0 ..
 * min(cap, *count) - 1]; *count = kernels recorded.  FDOT_E_NOMEM if the
 * record overflowed or an event could not be created.  Host only apart from
 * the event records; not for use while another thread is issuing traced
 * calls. */
fdot_status_t fdot_trace_enable(int on);
fdot_status_t fdot_trace_read(double* ms, size_t cap, size_t* count);

/* Tuned launch parameters, keyed by name (e.g. "chunk.zpz", "wg_per_cu.zpz").
 * fdot_tune_set with value INT64_MIN removes the key (back to the built-in
 * default); fdot_tune_get of a key that is not set gives FDOT_E_NOT_FOUND.
 * The file named by the environment variable FDOT_TUNE_FILE ("key=value"
 * lines) is read at the first tuning lookup. */
fdot_status_t fdot_tune_set(const char* key, int64_t value);
fdot_status_t fdot_tune_get(const char* key, int64_t* value);

/* ------------------------------------------------------------------ serving
 * A request server for streams of dot / matrix-vector / matrix products of
 * mixed primes and sizes (the dot product as the building block of higher
 * routines, Sec. 1, served continuously).  Requests arriving while others
 * run are admitted as soon as an in-flight slot and enough of the HBM
 * budget are free; at every scheduling step the admitted dot requests of one
 * field are fused into one batched launch, and launches are spread over
 * several HIP streams by estimated device time: long matrix products on one,
 * long streaming requests on another, everything shorter than short_ns on
 * the rest, so that short requests never wait behind long ones in a stream
 * and the work of different requests overlaps on the device.  Results are
 * exact, so a request's result is the same alone and in any mix.  Operands
 * stay device-resident and owned by the caller until the request is done;
 * the server never copies or frees them.  The server's launches run on its
 * own streams: operands must be complete on the device when the request is
 * submitted, or the request names a HIP event (ready) that its launch
 * waits for. */

typedef enum { FDOT_OP_DOT = 0, FDOT_OP_GEMV = 1, FDOT_OP_GEMM = 2,
               FDOT_OP_FORCE_INT32 = 0x7fffffff } fdot_op_t;

typedef struct {
  int32_t op;          /* fdot_op_t */
  int32_t reserved;
  fdot_field_t field;
  const void* a;       /* DOT: x (n);  GEMV: A (m x n);  GEMM: A (m x k) */
  const void* b;       /* DOT: y (n);  GEMV: x (n);      GEMM: B (k x n) */
  void* out;           /* DOT: 1 elem; GEMV: y (m);      GEMM: C (m x n) */
  uint64_t m, n, k;    /* dense row-major operands, leading dimension = row length */
  uint64_t footprint;  /* device bytes charged against the budget while the request
                          is admitted; 0 = its operand and result bytes plus the
                          library scratch it takes (an upper bound) */
  void* ready;         /* optional hipEvent_t recorded after the operands were
                          produced; the request's launch waits for it (NULL: the
                          operands are complete at submit) */
} fdot_request_t;

typedef struct {
  uint64_t hbm_budget;   /* admitted footprint allowed at once (bytes) */
  uint32_t max_inflight; /* admitted requests at once */
  uint32_t max_queue;    /* waiting requests before submit returns FDOT_E_BUSY */
  uint32_t streams;      /* HIP streams the launches are spread over */
  uint32_t max_batch;    /* dot requests fused into one launch */
  uint32_t fake_device;  /* 1: no GPU; completions are simulated (scheduler tests) */
  uint32_t plain;        /* 1: no batching: one launch per request, one stream,
                            arrival order (the comparison baseline) */
  uint64_t exclusive_ns; /* a request whose estimated device time exceeds this
                            runs alone: it is admitted when nothing is in
                            flight and nothing is admitted while it runs, so
                            overlap never slows the longest requests (0 = off:
                            on the mixed stream it cost more waiting behind
                            long requests than it saved) */
  uint64_t short_ns;     /* with three or more streams: matrix products run on
                            stream 0; streaming requests (or fused dot batches)
                            estimated below short_ns on streams 2.., longer ones
                            on stream 1; 0 = 100 us */
  uint32_t matrix_depth; /* at most this many matrix products outstanding on
                            stream 0; the others wait in the server, admitted, and
                            the shortest estimate goes next (the oldest once it has
                            waited four times its estimate, at least 2 ms); 0 = 2;
                            UINT32_MAX: no limit (each launched when admitted) */
  uint32_t reserved;
} fdot_server_cfg_t;

typedef struct {
  uint64_t submit_ns;    /* steady-clock times of the request's life */
  uint64_t admit_ns;
  uint64_t launch_ns;
  uint64_t done_ns;      /* when the scheduler saw its launch complete */
  int32_t status;        /* FDOT_OK, or the error of its launch */
  uint32_t batch_size;   /* requests carried by the same launch */
  uint32_t stream;       /* index of the server stream it was launched on */
  uint32_t reserved;
} fdot_timing_t;

typedef struct {
  uint64_t submitted, completed, rejected;
  uint64_t launches;            /* kernel launch groups issued */
  uint64_t peak_footprint;      /* largest admitted footprint seen */
  uint32_t peak_inflight;       /* largest number of admitted requests seen */
  uint32_t reserved;
} fdot_server_stats_t;

typedef struct fdot_server_s* fdot_server_t;

/* Start a server (its scheduling thread and streams) on the current device.
 * cfg NULL = defaults (64 GiB budget, 256 slots, 4096 queue, 4 streams,
 * 4096 per batch). */
fdot_status_t fdot_server_create(const fdot_server_cfg_t* cfg, fdot_server_t* out);
/* Queue a request; *ticket identifies it.  FDOT_E_BUSY: the queue is full;
 * FDOT_E_NOMEM: its footprint exceeds the whole budget; FDOT_E_INVALID_ARG:
 * malformed request.  Thread-safe. */
fdot_status_t fdot_server_submit(fdot_server_t s, const fdot_request_t* req, uint64_t* ticket);
/* *done = 1 once the request's result is in place (timing filled in). */
fdot_status_t fdot_server_poll(fdot_server_t s, uint64_t ticket, int* done, fdot_timing_t* t);
/* Block until every submitted request is done, or timeout_ms passes
 * (FDOT_E_BUSY on timeout). */
fdot_status_t fdot_server_drain(fdot_server_t s, uint64_t timeout_ms);
/* Load generator: submit reqs[i] when arrival_s[i] seconds (non-decreasing)
 * have passed since the call, wait for all, fill timings[i]; there submit_ns
 * is the scheduled arrival, so time spent blocked in submit counts as
 * waiting. */
fdot_status_t fdot_server_replay(fdot_server_t s, const fdot_request_t* reqs,
                                 const double* arrival_s, size_t count, fdot_timing_t* timings);
fdot_status_t fdot_server_stats(fdot_server_t s, fdot_server_stats_t* out);
/* Drain, stop the scheduling thread, release streams and buffers. */
fdot_status_t fdot_server_destroy(fdot_server_t s);

#ifdef __cplusplus
}
#endif

#endif /* FDOT_H */
