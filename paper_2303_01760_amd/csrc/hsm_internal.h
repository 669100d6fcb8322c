// Internal declarations of the HIP library behind include/hsm.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <climits>

#include <string>
#include <vector>

#include "../../include/hsm.h"

namespace hsm {

constexpr int kMaxBuckets = 16;
constexpr int kMaxDomainsInline = 0;  // domain tables always live in device memory

// bucket types (internal order is bucket-major)
enum BucketType : int32_t { B_REG = 0, B_SCAT = 1, B_DIR = 2, B_NEU = 3 };

// ---------------------------------------------------------------- errors --
void set_error(hsm_status code, const std::string &msg, int64_t node = -1);
hsm_status hip_fail(hipError_t e, const char *what);

#define HSM_HIP(call)                                  \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hsm::hip_fail(e_, #call); \
  } while (0)

// Error flags latched by build kernels: one bit per error kind and, per kind,
// the lowest offending node in caller numbering (INT64_MAX if none).
enum BuildErr : int32_t { BE_DUPLICATE = 0, BE_AMBIGUOUS = 1, BE_SINGULAR = 2, BE_SMALL_DOMAIN = 3, BE_NONFINITE = 4, BE_COUNT = 5 };
struct DevStatus {
  uint32_t bits;
  int32_t pad;
  unsigned long long node[BE_COUNT];
};
__device__ inline void latch(DevStatus *st, int kind, int64_t node) {
  atomicOr(&st->bits, 1u << kind);
  atomicMin(&st->node[kind], (unsigned long long)node);
}

// ------------------------------------------------------ device buffers ---
struct DBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  DBuf(DBuf &&o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DBuf &operator=(DBuf &&o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  hsm_status alloc(size_t n) {
    release();
    if (n == 0) n = 16;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      set_error(HSM_E_OOM, "device allocation of " + std::to_string(n) + " bytes failed");
      return HSM_E_OOM;
    }
    bytes = n;
    return HSM_OK;
  }
  template <class T> T *as() const { return static_cast<T *>(p); }
};

// Scratch memory of one call, from a stream-ordered pool of the library (one
// per device, created on first use).  Allocation and release are ordered on
// the stream, so temporaries need no synchronisation before they are freed,
// and the pool keeps up to kScratchPoolKeep bytes of released memory for the
// next call instead of returning it to the device.
constexpr uint64_t kScratchPoolKeep = 4ull << 30;
constexpr int kMaxDevices = 64;
hipMemPool_t scratch_pool(int device);

struct SBuf {
  void *p = nullptr;
  hipStream_t s = nullptr;
  SBuf() = default;
  SBuf(const SBuf &) = delete;
  SBuf &operator=(const SBuf &) = delete;
  ~SBuf() { release(); }
  void release() {
    if (p) (void)hipFreeAsync(p, s);
    p = nullptr;
  }
  hsm_status alloc(size_t n, hipStream_t stream) {
    release();
    if (n == 0) n = 16;
    int dev = 0;
    hipMemPool_t pool = nullptr;
    if (hipGetDevice(&dev) == hipSuccess) pool = scratch_pool(dev);
    if (!pool) {
      (void)hipGetLastError();
      set_error(HSM_E_HIP, "no scratch memory pool on this device");
      return HSM_E_HIP;
    }
    hipError_t e = hipMallocFromPoolAsync(&p, n, pool, stream);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      set_error(HSM_E_OOM, "scratch allocation of " + std::to_string(n) + " bytes failed");
      return HSM_E_OOM;
    }
    s = stream;
    return HSM_OK;
  }
  template <class T> T *as() const { return static_cast<T *>(p); }
};

// Bump allocation of several temporaries from one scratch-pool block: the
// caller adds up the 256-byte-rounded sizes, reserves, then takes them.
inline size_t round256(size_t b) { return ((b ? b : 1) + 255) & ~(size_t)255; }
struct Arena {
  SBuf buf;
  size_t off = 0, cap = 0;
  hsm_status reserve(size_t bytes, hipStream_t s) {
    off = 0;
    cap = bytes;
    return buf.alloc(bytes, s);
  }
  struct View {
    void *p = nullptr;
    template <class T> T *as() const { return static_cast<T *>(p); }
  };
  // the next `bytes` (NULL view when the reservation is exhausted)
  View take(size_t bytes) {
    View v;
    const size_t b = round256(bytes);
    if (off + b > cap) return v;
    v.p = static_cast<char *>(buf.p) + off;
    off += b;
    return v;
  }
};

// --------------------------------------------------------------- buckets --
struct Bucket {
  int32_t type = 0;    // BucketType
  int32_t width = 0;   // stencil width
  int32_t m = 0;       // RBF-FD degree (0 for MON)
  int32_t nops = 0;    // weight arrays stored: d+1, plus 1 (normal derivative) on wall buckets
  int64_t start = 0;   // first internal index
  int64_t count = 0;
  DBuf idx;            // int32 [width][count], internal numbering
  DBuf w;              // double [nops][width][count]
  DBuf w32;            // float  [nops][width][count] (made on first FP32 use)
};

// First block of each bucket, passed by value: the bucket index of a block
// follows from statically indexed kernel arguments (scalar registers), so
// the descriptor load is the only memory access and can start at once.
struct BlockMap {
  int64_t block0[kMaxBuckets];
  int32_t nb, pad;
};

}  // namespace hsm

struct hsm_stencils;
namespace hsm { struct BucketTable; }

struct hsm_stencils {
  int32_t d = 0, mode = 0, n_domains = 0;
  std::vector<int64_t> dom_off;   // [n_domains + 1] domain ranges, caller numbering (host)
  int64_t N = 0, nnz = 0, n_regular = 0, n_scattered = 0, n_boundary = 0;
  int64_t n_wall_fallback = 0;   // wall nodes solved with monomials of degree m-1
  hsm::DBuf fallback;            // int32 [1 + n_wall_fallback]: the count, then those nodes (internal numbering)
  std::vector<hsm::Bucket> buckets;
  hsm::DBuf perm;        // int32 [N] internal -> caller
  hsm::DBuf iperm;       // int32 [N] caller -> internal
  hsm::DBuf x;           // double [d][N] internal order
  hsm::DBuf kind;        // uint8 [N] internal order
  hsm::DBuf normal;      // double [d][N] internal order
  hsm::DBuf cls;         // uint8 [N] caller order
  int32_t device = 0;
  int32_t solve_groups = 0;      // RBF-FD systems per wave (0: the most that fit)
  double build_ms[4] = {0, 0, 0, 0};
  mutable bool w32_ready = false;
  mutable hsm::DBuf dtab[2];     // device copies of the apply bucket table (FP64, FP32 weights)
  mutable int64_t dtab_blocks[2] = {-1, -1};
  mutable hsm::BlockMap bmap[2];
  mutable hsm::DBuf dtab_sub;          // the table of the last bucket-masked apply
  mutable uint32_t dtab_sub_key = 0;   // its bucket mask and precision (bit 31: FP32); 0: none
  mutable int64_t dtab_sub_blocks = 0;
  mutable hsm::BlockMap bmap_sub;
  double bucket_solve_ms[16] = {};     // device time of each bucket's first solve pass
};

namespace hsm {

// Bucket table handed to kernels by value.
// Raw buffer loads: a resource (base address and byte size, in scalar
// registers), a 32-bit per-lane byte offset and a uniform 32-bit byte
// offset.  A load costs one vector register of address, and loads at uniform
// strides from one lane offset (the SoA stencil arrays) share it; the
// compiler also sees plain vector-memory loads it can keep in flight
// together (pointers read from device memory would otherwise compile to
// flat loads, which it can only await all at once).  Reads past the stated
// size return zero.  Each resource spans one row of a stencil array or one
// node vector, so every offset stays below 4 GiB (the node count is capped
// on the host).
struct Buf {
  __amdgpu_buffer_rsrc_t r;
};
constexpr int kBufDword3 = 0x00020000;   // gfx9 raw buffer: 32-bit data format, no swizzle
__device__ __forceinline__ Buf make_buf(const void *p, uint64_t bytes) {
  const uint32_t n = bytes > 0xffffffffull ? 0xffffffffu : (uint32_t)bytes;
  return Buf{__builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)n, kBufDword3)};
}
template <class T>
__device__ __forceinline__ T ld(const Buf &b, uint32_t voff);
template <>
__device__ __forceinline__ int32_t ld<int32_t>(const Buf &b, uint32_t voff) {
  return (int32_t)__builtin_amdgcn_raw_buffer_load_b32(b.r, voff, 0, 0);
}
template <>
__device__ __forceinline__ float ld<float>(const Buf &b, uint32_t voff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(b.r, voff, 0, 0));
}
template <>
__device__ __forceinline__ double ld<double>(const Buf &b, uint32_t voff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(b.r, voff, 0, 0));
}
template <>
__device__ __forceinline__ double2 ld<double2>(const Buf &b, uint32_t voff) {
  const auto q = __builtin_amdgcn_raw_buffer_load_b128(b.r, voff, 0, 0);
  return make_double2(__builtin_bit_cast(double, (uint64_t)q[0] | ((uint64_t)q[1] << 32)),
                      __builtin_bit_cast(double, (uint64_t)q[2] | ((uint64_t)q[3] << 32)));
}
// Row e (uniform) of an SoA array [rows][cnt], element t (per lane).
template <class T>
__device__ __forceinline__ T ld_soa(const void *base, uint32_t cnt, uint32_t e, uint32_t t) {
  const Buf b = make_buf(static_cast<const T *>(base) + (uint64_t)e * cnt, (uint64_t)cnt * sizeof(T));
  return ld<T>(b, t * (uint32_t)sizeof(T));
}
// Element nb (per lane) of a node vector held as a resource.
template <class T>
__device__ __forceinline__ T ld_at(const Buf &b, int32_t nb) {
  return ld<T>(b, (uint32_t)nb * (uint32_t)sizeof(T));
}
// Plane c (uniform) of a [planes][n] array as a resource.
template <class T>
__device__ __forceinline__ Buf plane(const T *base, int64_t n, int c) {
  return make_buf(base + (int64_t)c * n, (uint64_t)n * sizeof(T));
}

// Ties a register value to this point of the program (an empty asm
// statement that reads and writes it): the arithmetic producing it cannot be
// sunk below.
template <class T>
__device__ __forceinline__ void pin(T &x) {
  asm volatile("" : "+v"(x));
}

// Dot-product accumulators.  FMA in the working precision, or FP32 with
// compensated products and sums (Ogita, Rump, Oishi 2005, "Dot2":
// TwoProduct by FMA, Knuth's TwoSum), which evaluates an FP32 dot product as
// if in twice the working precision.  Sources are built with
// -ffp-contract=off, so the error-free transformations stay as written.
template <class T>
struct Acc {
  T s;
  __device__ __forceinline__ void init() { s = T(0); }
  __device__ __forceinline__ void add(T w, T u) { s = fma(w, u, s); }
  __device__ __forceinline__ void settle() { pin(s); }
  __device__ __forceinline__ T get() const { return s; }
  __device__ __forceinline__ double get_d() const { return (double)s; }
};
struct Dot2 {
  float s, c;
  __device__ __forceinline__ void init() { s = 0.f; c = 0.f; }
  __device__ __forceinline__ void add(float w, float u) {
    const float p = w * u;
    const float pe = fmaf(w, u, -p);          // TwoProduct error
    const float t = s + p;                     // TwoSum(s, p)
    const float z = t - s;
    const float se = (s - (t - z)) + (p - z);
    s = t;
    c = c + (pe + se);
  }
  __device__ __forceinline__ void settle() { pin(s); pin(c); }
  __device__ __forceinline__ float get() const { return s + c; }
  __device__ __forceinline__ double get_d() const { return (double)s + (double)c; }
};
// The accumulator of field applies for a field storage type: FP64 FMA, or
// Dot2 for FP32 fields.
template <class FT>
struct FieldAccT;
template <>
struct FieldAccT<double> {
  using type = Acc<double>;
};
template <>
struct FieldAccT<float> {
  using type = Dot2;
};
template <class FT>
using FieldAcc = typename FieldAccT<FT>::type;

// A fixed-size bundle of values loaded together.
template <class T, int K>
struct Pack {
  T v[K];
};

// Two bundles of different types loaded together.
template <class TA, int KA, class TB, int KB>
struct Pack2 {
  Pack<TA, KA> a;
  Pack<TB, KB> b;
};

// Largest divisor of W that is at most K.
constexpr int chunk_of(int W, int K) {
  for (int c = K < W ? K : W; c > 1; --c)
    if (W % c == 0) return c;
  return 1;
}

// Stencil gather of node t over its W entries, in chunks of C entries (the
// largest divisor of W not above K): a chunk's indices and weights are
// loaded, then its neighbour values, and only then consumed, in stencil
// order, by use(j, weights, values); settle() then pins the accumulators.
// The loads of a chunk are in flight together instead of one neighbour
// after another, and each chunk's values die with the chunk: the pins keep
// the accumulation from being sunk to the end, and a scheduling barrier
// keeps the next chunk's loads from being hoisted (either would hold every
// chunk's values live at once).  idx: the bucket's [W][cnt] neighbour indices.
// hook(): called once, after the first chunk's neighbour loads are issued and
// before any of them is consumed (work on values loaded before the gather,
// done while the gather is in flight).
struct NoHook {
  __device__ __forceinline__ void operator()() const {}
};
template <int W, int K = 12, class FW, class FV, class FU, class FS, class FH = NoHook>
__device__ __forceinline__ void gather_chunks(const void *idx, uint32_t cnt, uint32_t t, FW &&wload, FV &&vload,
                                              FU &&use, FS &&settle, FH &&hook = FH{}) {
  constexpr int C = chunk_of(W, K);
  // with two chunks, both chunks' indices in one round of loads: the second
  // chunk then waits for its values (and weights) only, not for its indices
  // first (more chunks would hold too many registers)
  constexpr bool pre = (W / C == 2);
  int32_t nb[pre ? W : C];
  if (pre) {
#pragma unroll
    for (int j = 0; j < (pre ? W : C); ++j) nb[j] = ld_soa<int32_t>(idx, cnt, j, t);
  }
#pragma unroll
  for (int j0 = 0; j0 < W; j0 += C) {
    decltype(wload(0)) wv[C];
    decltype(vload(0)) vv[C];
    if (!pre) {
#pragma unroll
      for (int c = 0; c < C; ++c) nb[c] = ld_soa<int32_t>(idx, cnt, j0 + c, t);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) wv[c] = wload(j0 + c);
#pragma unroll
    for (int c = 0; c < C; ++c) vv[c] = vload(nb[(pre ? j0 : 0) + c]);
    if (j0 == 0) hook();
#pragma unroll
    for (int c = 0; c < C; ++c) use(j0 + c, wv[c], vv[c]);
    if (j0 + C < W) {
      settle();
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

struct BucketDesc {
  int64_t start, count;
  int32_t type, width;
  int64_t block0;        // first block of this bucket in a multi-bucket launch
  const int32_t *idx;
  const void *w;         // [nops][width][count] of the launch's precision
  const void *aux;       // per-launch extra array (the stepper's pressure-operator weights)
  int32_t nops, pad;
};
struct BucketTable {
  BucketDesc b[kMaxBuckets];
  int32_t nb, pad;
  int64_t nblocks;
};

// The bucket a block belongs to.  The table lives in device memory (indexed
// kernel-argument arrays end up copied to scratch memory); all loads here
// are wave-uniform.
__device__ __forceinline__ BucketDesc select_bucket(const BucketTable *__restrict__ tab, int64_t block) {
  const int nb = tab->nb;
  int bi = 0;
  for (int k = 1; k < nb; ++k)
    if (block >= tab->b[k].block0) bi = k;
  return tab->b[bi];
}

__device__ __forceinline__ int bucket_index(const BlockMap &bm, int64_t block) {
  int bi = 0;
#pragma unroll
  for (int k = 1; k < kMaxBuckets; ++k)
    if (k < bm.nb && block >= bm.block0[k]) bi = k;
  return bi;
}
inline BlockMap make_blockmap(const BucketTable &tab) {
  BlockMap bm{};
  bm.nb = tab.nb;
  for (int k = 0; k < tab.nb; ++k) bm.block0[k] = tab.b[k].block0;
  for (int k = tab.nb; k < kMaxBuckets; ++k) bm.block0[k] = INT64_MAX;
  return bm;
}

// Fills tab for all buckets of st (or only those whose type bit is in type_mask),
// with `bs` threads per block and one node per thread.  fp32 selects w32.
void make_table(const hsm_stencils *st, BucketTable &tab, int bs, uint32_t type_mask, bool fp32,
                uint32_t bucket_mask = 0xFFFFFFFFu);

// ---------------------------------------------------------------- scan ----
// Exclusive prefix sum of n int32 values into int64 out[n+1] (out[n] = total).
// exclusive prefix sum of in[0..n) into out[0..n], out[n] = total; ws holds
// scan_i32_to_i64_ws(n) int64 of scratch (NULL: taken from the scratch pool)
hsm_status scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, hipStream_t s, int64_t *ws = nullptr);
int64_t scan_i32_to_i64_ws(int64_t n);

// ------------------------------------------------------------- builders ---
hsm_status build_stencils_impl(const hsm_nodeset *ns, int32_t mode, hipStream_t s, hsm_stencils **out);
hsm_status solve_bucket(const hsm_stencils *st, const Bucket &b, const double *x_int,
                        const double *normal_int, DevStatus *status, hipStream_t s, int32_t *retry = nullptr,
                        int32_t *nretry = nullptr);
hsm_status solve_bucket_list(const hsm_stencils *st, const Bucket &b, const double *x_int,
                             const double *normal_int, DevStatus *status, hipStream_t s, const int32_t *list,
                             int64_t nlist);
hsm_status cond_bucket(const hsm_stencils *st, const Bucket &b, double *kappa, hipStream_t s, const int32_t *list,
                       int64_t nlist);
hsm_status apply_impl(const hsm_stencils *st, uint32_t op_mask, int32_t dtype, const void *u, void *out,
                      hipStream_t s, uint32_t bucket_mask = 0xFFFFFFFFu);
hsm_status ensure_w32(const hsm_stencils *st, hipStream_t s);

inline int nmono(int d, int m) {
  int q = 1;
  for (int k = 1; k <= d; ++k) q = q * (m + k) / k;
  return q;
}

}  // namespace hsm
