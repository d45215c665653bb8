// Dot products over extension fields GF(p^d), q = p^d <= 65536, in discrete
// logarithms (Sec. 2.4.2): the representation stays atomic, so the per-term
// work is the prime-field one -- a product is an index sum modulo q-1, a sum
// goes through the plus-one table (Sec. 2.4, Table 1).  No code stands for a
// residue mod p here, so partial sums are also combined by table addition:
// eight independent accumulators per lane (one per 16-bit slot of a 16-byte
// load, so consecutive terms do not wait on each other's table lookups),
// then across the wavefront by shuffles, across the workgroup through LDS,
// and across workgroups by a second, one-workgroup pass.  The plus-one table
// (2q bytes) is copied into LDS by workgroups that stay resident.  The
// batched form gives whole pairs to resident workgroups in turn.
//
// In characteristic 2 there is a cheaper schedule, the extension-field
// counterpart of converting codes to values (Sec. 2.4): the value of a code
// is its polynomial's coefficient bits, and adding polynomials over GF(2) is
// the exclusive or of those bits, exact and carry-free.  So each product code
// is looked up in the value table and XORed into the accumulator, with no
// plus-one chain; the final value goes back to a code through the index
// table.  That is about a third of the vector instructions per term.
#include <algorithm>
#include <type_traits>

#include "fdot_internal.h"
#include "zech_packed.h"

namespace {

constexpr int NT = 1024;
constexpr int EU = 4;  // vector pairs in flight per lane

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t zmul(uint32_t a, uint32_t b, uint32_t qbar) {
  if (a == 0 || b == 0) return 0;
  const uint32_t k = a + b;
  return k > qbar ? k - qbar : k;
}

// a + b = a (1 + b/a); tab[k] is the code of 1 + (element coded k)
__device__ __forceinline__ uint32_t zadd(uint32_t a, uint32_t b, uint32_t qbar,
                                         const uint16_t* tab) {
  if (a == 0) return b;
  if (b == 0) return a;
  const uint32_t k = b > a ? b - a : b + qbar - a;  // code of b / a, in [1, q-1]
  const uint32_t t = tab[k];
  if (t == 0) return 0;
  const uint32_t w = a + t;
  return w > qbar ? w - qbar : w;
}

// Accumulator of one lane.  XOR = false: Zech codes summed by the plus-one
// table (tab = plus-one table); XOR = true: polynomial values over GF(2)
// summed by exclusive or (tab = value table).
template <bool XOR>
struct Acc;

template <>
struct Acc<false> {
  // running forms (zech_acc1), one per 16-bit slot of a vector; the staged
  // table's entry 0 is entry q' (see the kernels)
  uint32_t z[8] = {~0u, ~0u, ~0u, ~0u, ~0u, ~0u, ~0u, ~0u};
  __device__ __forceinline__ void one(uint32_t a, uint32_t b, uint32_t qbar, const uint16_t* tab) {
    z[0] = zech_acc1(z[0], a, b, tab, qbar);
  }
  __device__ __forceinline__ void vec(const v4u& a, const v4u& b, uint32_t qbar,
                                      const uint16_t* tab, int) {
    uint32_t ca[8], cb[8];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      ca[2 * j] = a[j] & 0xFFFFu;
      ca[2 * j + 1] = a[j] >> 16;
      cb[2 * j] = b[j] & 0xFFFFu;
      cb[2 * j + 1] = b[j] >> 16;
    }
    zech_acc1_x8(z, ca, cb, tab, qbar);
  }
  __device__ __forceinline__ uint32_t total(uint32_t qbar, const uint16_t* tab) const {
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) acc = zadd(acc, z[j] + 1u, qbar, tab);  // codes
    return acc;
  }
};

template <>
struct Acc<true> {
  uint32_t v0 = 0, v1 = 0;
  __device__ __forceinline__ void one(uint32_t a, uint32_t b, uint32_t qbar, const uint16_t* tab) {
    v0 ^= tab[zmul(a, b, qbar)];  // the zero code's value is 0
  }
  __device__ __forceinline__ void vec(const v4u& a, const v4u& b, uint32_t qbar,
                                      const uint16_t* tab, int) {
    // the eight products' codes, then their eight value reads back to back
    // (so that the reads overlap), then the exclusive ors
    uint32_t k[8], h[8];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      k[2 * j] = zmul(a[j] & 0xFFFFu, b[j] & 0xFFFFu, qbar);
      k[2 * j + 1] = zmul(a[j] >> 16, b[j] >> 16, qbar);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < 8; ++j) h[j] = tab[k[j]];
    __builtin_amdgcn_sched_barrier(0);
    v0 ^= (h[0] ^ h[2]) ^ (h[4] ^ h[6]);
    v1 ^= (h[1] ^ h[3]) ^ (h[5] ^ h[7]);
  }
  __device__ __forceinline__ uint32_t total(uint32_t, const uint16_t*) const { return v0 ^ v1; }
};

// Packed accumulators for q <= 32768 (zech_packed.h): two codes per register
// in the running form, one set of eight per vector of a step, so the EU
// vectors' dependent table reads overlap; the step's plus-one table (with its
// zero mark) is in LDS.  total() folds the sets into one register with the
// same step (adding a running sum s to another is one step with a = the
// code of s, b = the code of 1) and returns the table sum of its two codes.
struct AccP {
  uint32_t z[EU][4];
  const char* tb;
  ZechPacked C;
  __device__ __forceinline__ void init(const FieldK& F, const uint16_t* s_tab) {
#pragma unroll
    for (int u = 0; u < EU; ++u)
#pragma unroll
      for (int j = 0; j < 4; ++j) z[u][j] = 0xFFFFFFFFu;
    tb = (const char*)s_tab;
    C = zech_packed_constants(F);
  }
  __device__ __forceinline__ void one(uint32_t a, uint32_t b, uint32_t, const uint16_t*) {
    z[0][0] = zech_acc2(z[0][0], a, b, tb, C);  // high halves: zero codes, a zero product
  }
  __device__ __forceinline__ void vec(const v4u& a, const v4u& b, uint32_t, const uint16_t*,
                                      int u) {
#pragma unroll
    for (int j = 0; j < 4; ++j) z[u][j] = zech_acc2(z[u][j], a[j], b[j], tb, C);
  }
  __device__ __forceinline__ uint32_t add(uint32_t v, uint32_t w) const {
    uint32_t code;
    FD_PKS("v_pk_add_u16", code, w, C.k1);  // running form -> code (0xFFFF -> 0)
    return zech_acc2(v, code, C.qq, tb, C);
  }
  __device__ __forceinline__ uint32_t total(uint32_t qbar, const uint16_t* plus1) const {
    uint32_t r[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      r[j] = z[0][j];
#pragma unroll
      for (int u = 1; u < EU; ++u) r[j] = add(r[j], z[u][j]);
    }
    const uint32_t v = add(add(r[0], r[1]), add(r[2], r[3]));
    return zadd((v + 1) & 0xFFFFu, ((v >> 16) + 1) & 0xFFFFu, qbar, plus1);
  }
};

// Combines two lane or workgroup sums: table addition of codes, or XOR of
// values.
template <bool XOR>
__device__ __forceinline__ uint32_t combine(uint32_t a, uint32_t b, uint32_t qbar,
                                            const uint16_t* tab) {
  if constexpr (XOR) return a ^ b;
  else return zadd(a, b, qbar, tab);
}

// Streams vectors v0, v0 + step, ... below nv of x and y into z, EU vector
// pairs loaded before any is consumed, so that enough bytes are in flight to
// cover the memory latency.
template <class AccT>
__device__ __forceinline__ void stream_vectors(const v4u* x, const v4u* y, uint64_t v0,
                                               uint64_t step, uint64_t nv, AccT& A,
                                               uint32_t qbar, const uint16_t* tab) {
  uint64_t v = v0;
  for (; v + (uint64_t)(EU - 1) * step < nv; v += (uint64_t)EU * step) {
    v4u a[EU], b[EU];
#pragma unroll
    for (int u = 0; u < EU; ++u) {
      a[u] = __builtin_nontemporal_load(x + v + (uint64_t)u * step);
      b[u] = __builtin_nontemporal_load(y + v + (uint64_t)u * step);
    }
#pragma unroll
    for (int u = 0; u < EU; ++u) A.vec(a[u], b[u], qbar, tab, u);
  }
  for (; v < nv; v += step) {
    const v4u a = __builtin_nontemporal_load(x + v);
    const v4u b = __builtin_nontemporal_load(y + v);
    A.vec(a, b, qbar, tab, 0);
  }
}

// Sum of the lane values of a workgroup of NT threads; valid in thread 0.
template <bool XOR>
__device__ uint32_t block_sum(uint32_t acc, uint32_t qbar, const uint16_t* tab, uint32_t* s_part) {
  for (int off = 32; off > 0; off >>= 1)
    acc = combine<XOR>(acc, (uint32_t)__shfl_xor((int)acc, off), qbar, tab);
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  if (lane == 0) s_part[w] = acc;
  __syncthreads();
  uint32_t s = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / 64; ++i) s = combine<XOR>(s, s_part[i], qbar, tab);
  return s;
}

template <bool XOR>
__device__ __forceinline__ const uint16_t* table_of(const FieldK& F) {
  return XOR ? F.zval : F.zplus1;
}

// The lane accumulator of a schedule: PK, the packed plus-one step
// (q <= 32768); otherwise table addition of codes or XOR of values.  The
// table staged in LDS is the step's own; sums across lanes and workgroups
// (combine) read the plus-one table indexed by code, which for PK is the
// one in device memory.
template <bool XOR, bool PK>
using AccOf = typename std::conditional<PK, AccP, Acc<XOR>>::type;

template <bool XOR, bool PK>
__device__ __forceinline__ const uint16_t* staged_table(const FieldK& F) {
  return PK ? F.zpk : table_of<XOR>(F);
}

template <bool XOR, bool PK>
__device__ __forceinline__ void init_acc(AccOf<XOR, PK>& A, const FieldK& F, const uint16_t* s_tab) {
  if constexpr (PK) A.init(F, s_tab);
}

template <bool XOR, bool PK>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8, 8))) void ext_dot_kernel(const FieldK F, const uint16_t* x,
                                                     const uint16_t* y, uint64_t n, int vec,
                                                     uint16_t* partial) {
  extern __shared__ uint16_t s_tab[];
  __shared__ uint32_t s_part[NT / 64];
  fd_table_to_lds<NT>(s_tab, staged_table<XOR, PK>(F), (uint32_t)F.p);
  if constexpr (!XOR && !PK) {
    // the one-code step reads entry 0 for g^0 (zadd never reads it)
    if (threadIdx.x == 0) s_tab[0] = s_tab[F.qbar];
    __syncthreads();
  }
  const uint16_t* ctab = PK ? F.zplus1 : s_tab;  // for combine
  const uint32_t qbar = F.qbar;
  const uint64_t tid = (uint64_t)blockIdx.x * NT + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * NT;
  AccOf<XOR, PK> A;
  init_acc<XOR, PK>(A, F, s_tab);
  uint64_t done = 0;
  if (vec) {
    const uint64_t nv = n / 8;
    stream_vectors((const v4u*)x, (const v4u*)y, tid, stride, nv, A, qbar, s_tab);
    done = nv * 8;
  }
  for (uint64_t i = done + tid; i < n; i += stride) A.one(x[i], y[i], qbar, s_tab);
  const uint32_t s = block_sum<XOR>(A.total(qbar, ctab), qbar, ctab, s_part);
  if (threadIdx.x == 0) partial[blockIdx.x] = (uint16_t)s;
}

// The partials live in the stream's workspace, whose combination words the
// prime-field dot kernels expect to find zero: each is cleared once read.
// XOR: the partials are values, and the result is the code of their sum.
template <bool XOR>
__global__ __launch_bounds__(NT) void ext_sum_kernel(const FieldK F, uint16_t* partial,
                                                     uint32_t count, uint16_t* result) {
  __shared__ uint32_t s_part[NT / 64];
  uint32_t acc = 0;
  for (uint32_t i = threadIdx.x; i < count; i += NT) {
    acc = combine<XOR>(acc, partial[i], F.qbar, F.zplus1);
    partial[i] = 0;
  }
  const uint32_t s = block_sum<XOR>(acc, F.qbar, F.zplus1, s_part);
  if (threadIdx.x == 0) result[0] = XOR ? F.zidx[s] : (uint16_t)s;
}

// Batched form: resident workgroups take whole pairs in turn (pair k goes to
// workgroup k mod grid), each reducing its pair with all its lanes and the
// table copied into LDS once.
template <bool XOR, bool PK>
__global__ __launch_bounds__(NT) void ext_many_kernel(const FieldK F, const fdot_desc_t* desc,
                                                      uint64_t count, uint16_t* results) {
  extern __shared__ uint16_t s_tab[];
  __shared__ uint32_t s_part[NT / 64];
  fd_table_to_lds<NT>(s_tab, staged_table<XOR, PK>(F), (uint32_t)F.p);
  if constexpr (!XOR && !PK) {
    // the one-code step reads entry 0 for g^0 (zadd never reads it)
    if (threadIdx.x == 0) s_tab[0] = s_tab[F.qbar];
    __syncthreads();
  }
  const uint16_t* ctab = PK ? F.zplus1 : s_tab;  // for combine
  const uint32_t qbar = F.qbar;
  for (uint64_t k = blockIdx.x; k < count; k += gridDim.x) {
    const fdot_desc_t d = desc[k];
    const uint16_t* x = (const uint16_t*)d.x;
    const uint16_t* y = (const uint16_t*)d.y;
    AccOf<XOR, PK> A;
    init_acc<XOR, PK>(A, F, s_tab);
    uint64_t done = 0;
    if (((((uintptr_t)x) | ((uintptr_t)y)) & 15u) == 0) {
      const uint64_t nv = d.n / 8;
      stream_vectors((const v4u*)x, (const v4u*)y, threadIdx.x, NT, nv, A, qbar, s_tab);
      done = nv * 8;
    }
    for (uint64_t i = done + threadIdx.x; i < d.n; i += NT) A.one(x[i], y[i], qbar, s_tab);
    const uint32_t sum = block_sum<XOR>(A.total(qbar, ctab), qbar, ctab, s_part);
    if (threadIdx.x == 0) results[k] = XOR ? F.zidx[sum] : (uint16_t)sum;
    __syncthreads();  // s_part is reused by the next pair
  }
}

}  // namespace

namespace {

// q <= 32768 (tune key zech.packed = 0: one code per lane)
bool use_packed(const fdot_field_s* f, bool xor_values) {
  return !xor_values && f->k.zpk != nullptr && fd_tune("zech.packed", 1) != 0;
}

template <class Fn>
void set_lds_limit(Fn* fn) {
  (void)hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                            128 * 1024);
}

}  // namespace

fdot_status_t fd_launch_ext_many(const fdot_field_s* f, bool xor_values, uint64_t count,
                                 const fdot_desc_t* desc, uint16_t* results, hipStream_t s) {
  const uint64_t q = f->k.p;
  const size_t lds = (size_t)q * sizeof(uint16_t);
  const uint64_t per_cu = std::max<uint64_t>(1, (160u * 1024u) / (lds + 1024));
  const uint32_t grid = (uint32_t)std::max<uint64_t>(
      1, std::min<uint64_t>(count, (uint64_t)fd_cu_count() * std::min<uint64_t>(per_cu, 2)));
  static bool attr_set = false;
  if (!attr_set) {
    set_lds_limit(ext_many_kernel<false, false>);
    set_lds_limit(ext_many_kernel<true, false>);
    set_lds_limit(ext_many_kernel<false, true>);
    attr_set = true;
  }
  if (xor_values)
    hipLaunchKernelGGL((ext_many_kernel<true, false>), dim3(grid), dim3(NT), lds, s, f->k, desc,
                       count, results);
  else if (use_packed(f, xor_values))
    hipLaunchKernelGGL((ext_many_kernel<false, true>), dim3(grid), dim3(NT), lds, s, f->k, desc,
                       count, results);
  else
    hipLaunchKernelGGL((ext_many_kernel<false, false>), dim3(grid), dim3(NT), lds, s, f->k, desc,
                       count, results);
  return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
}

fdot_status_t fd_launch_ext_dot(const fdot_field_s* f, bool xor_values, const uint16_t* x,
                                const uint16_t* y, uint64_t n, uint16_t* result, hipStream_t s) {
  const uint64_t q = f->k.p;
  const size_t lds = (size_t)q * sizeof(uint16_t);
  // resident workgroups per CU: as many as the table copies fit in LDS, and
  // at most two of NT threads (32 wavefronts per CU)
  const uint64_t per_cu =
      std::min<uint64_t>(2, std::max<uint64_t>(1, (160u * 1024u) / (lds + 1024)));
  const bool vec = ((((uintptr_t)x) | ((uintptr_t)y)) & 15u) == 0;
  const uint64_t work = vec ? n / 8 + 1 : n;
  const uint32_t grid = (uint32_t)std::max<uint64_t>(
      1, std::min<uint64_t>((work + NT - 1) / NT, (uint64_t)fd_cu_count() * per_cu));
  Workspace* w = nullptr;
  fdot_status_t st = fd_workspace_get(s, grid, &w);  // one 64-bit word per workgroup
  if (st != FDOT_OK) return st;
  uint16_t* partial = (uint16_t*)w->acc;
  static bool attr_set = false;
  if (!attr_set) {
    set_lds_limit(ext_dot_kernel<false, false>);
    set_lds_limit(ext_dot_kernel<true, false>);
    set_lds_limit(ext_dot_kernel<false, true>);
    attr_set = true;
  }
  const uint32_t parts = n > 0 ? grid : 0u;
  const int v = vec ? 1 : 0;
  if (xor_values) {
    if (n > 0)
      hipLaunchKernelGGL((ext_dot_kernel<true, false>), dim3(grid), dim3(NT), lds, s, f->k, x, y,
                         n, v, partial);
    hipLaunchKernelGGL(ext_sum_kernel<true>, dim3(1), dim3(NT), 0, s, f->k, partial, parts,
                       result);
  } else {
    if (n > 0) {
      if (use_packed(f, xor_values))
        hipLaunchKernelGGL((ext_dot_kernel<false, true>), dim3(grid), dim3(NT), lds, s, f->k, x,
                           y, n, v, partial);
      else
        hipLaunchKernelGGL((ext_dot_kernel<false, false>), dim3(grid), dim3(NT), lds, s, f->k, x,
                           y, n, v, partial);
    }
    hipLaunchKernelGGL(ext_sum_kernel<false>, dim3(1), dim3(NT), 0, s, f->k, partial, parts,
                       result);
  }
  return hipGetLastError() == hipSuccess ? FDOT_OK : FDOT_E_DEVICE;
}
