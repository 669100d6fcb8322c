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
  int64_t N = 0, nnz = 0, n_regular = 0, n_scattered = 0, n_boundary = 0;
  std::vector<hsm::Bucket> buckets;
  hsm::DBuf perm;        // int32 [N] internal -> caller
  hsm::DBuf iperm;       // int32 [N] caller -> internal
  hsm::DBuf x;           // double [d][N] internal order
  hsm::DBuf kind;        // uint8 [N] internal order
  hsm::DBuf normal;      // double [d][N] internal order
  hsm::DBuf cls;         // uint8 [N] caller order
  int32_t device = 0;
  double build_ms[4] = {0, 0, 0, 0};
  mutable bool w32_ready = false;
  mutable hsm::DBuf dtab[2];     // device copies of the apply bucket table (FP64, FP32 weights)
  mutable int64_t dtab_blocks[2] = {-1, -1};
  mutable hsm::BlockMap bmap[2];
};

namespace hsm {

// Bucket table handed to kernels by value.
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
void make_table(const hsm_stencils *st, BucketTable &tab, int bs, uint32_t type_mask, bool fp32);

// ---------------------------------------------------------------- scan ----
// Exclusive prefix sum of n int32 values into int64 out[n+1] (out[n] = total).
hsm_status scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, hipStream_t s);

// ------------------------------------------------------------- builders ---
hsm_status build_stencils_impl(const hsm_nodeset *ns, int32_t mode, hipStream_t s, hsm_stencils **out);
hsm_status solve_bucket(const hsm_stencils *st, const Bucket &b, const double *x_int,
                        const double *normal_int, DevStatus *status, hipStream_t s);
hsm_status apply_impl(const hsm_stencils *st, uint32_t op_mask, int32_t dtype, const void *u, void *out,
                      hipStream_t s);
hsm_status ensure_w32(const hsm_stencils *st, hipStream_t s);

inline int nmono(int d, int m) {
  int q = 1;
  for (int k = 1; k <= d; ++k) q = q * (m + k) / k;
  return q;
}

}  // namespace hsm
