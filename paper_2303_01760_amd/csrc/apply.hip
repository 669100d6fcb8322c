// Operator application, Eq. (1): out(x_c) = sum_i w_i u(x_i), at every node.
//
// Nodes are stored bucket by bucket (one stencil width per bucket); stencil
// indices and weights are SoA [j][node] so consecutive threads read
// consecutive addresses.  One launch covers every bucket: each block looks up
// its bucket in a small table and runs the loop unrolled for that width.
// Several operators applied to one field share the index reads and the
// gathered values.
//
// Precisions: FP64 (fused multiply-add accumulation); FP32; FP32 with
// compensated products and sums (Ogita, Rump, Oishi 2005, "Dot2": TwoProduct
// by FMA, Knuth's TwoSum), which evaluates the FP32 dot product as if in
// twice the working precision.  Built with -ffp-contract=off; every FMA below
// is written out.
#include <hip/hip_runtime.h>

#include "hsm_internal.h"

namespace hsm {
namespace {

constexpr int kBS = 256;
constexpr int kMaxOps = 5;

struct ApplyArgs {
  const BucketTable *tab;
  BlockMap bm;
  const void *u;
  void *out;
  int64_t N;
  int nops;
  int op_store[kMaxOps];   // storage slot of each requested operator, -1 = not stored (write 0)
  int op_wall_only[kMaxOps];
};

template <class T>
struct Acc {
  T s;
  __device__ __forceinline__ void init() { s = T(0); }
  __device__ __forceinline__ void add(T w, T u) { s = fma(w, u, s); }
  __device__ __forceinline__ T get() const { return s; }
};

// Dot2 accumulator in FP32
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
  __device__ __forceinline__ float get() const { return s + c; }
};

// Operator selection of one launch, held in registers.
struct OpSel {
  int nops;
  int slot[kMaxOps];   // storage slot, -1 = operator not stored (writes 0)
  int wall_only[kMaxOps];
};

template <class T, class A, int W>
__device__ __forceinline__ void apply_node(const T *__restrict__ u, T *__restrict__ out, int64_t N, const OpSel &os,
                                           const BucketDesc &b, int64_t t) {
  const T *__restrict__ w = static_cast<const T *>(b.w);
  const int64_t cnt = b.count;
  const int width = (W > 0) ? W : b.width;
  const bool wall = (b.type == B_DIR || b.type == B_NEU);
  bool on[kMaxOps];
#pragma unroll
  for (int o = 0; o < kMaxOps; ++o) on[o] = o < os.nops && os.slot[o] >= 0 && (!os.wall_only[o] || wall);
  A acc[kMaxOps];
#pragma unroll
  for (int o = 0; o < kMaxOps; ++o) acc[o].init();
#pragma unroll
  for (int j = 0; j < width; ++j) {
    const int32_t nb = b.idx[(int64_t)j * cnt + t];
    const T uv = u[nb];
#pragma unroll
    for (int o = 0; o < kMaxOps; ++o)
      if (on[o]) acc[o].add(w[((int64_t)os.slot[o] * width + j) * cnt + t], uv);
  }
#pragma unroll
  for (int o = 0; o < kMaxOps; ++o)
    if (o < os.nops) out[(int64_t)o * N + b.start + t] = on[o] ? (T)acc[o].get() : T(0);
}

template <class T, class A>
__global__ __launch_bounds__(kBS) void k_apply(ApplyArgs a) {
  const BucketDesc b = a.tab->b[bucket_index(a.bm, blockIdx.x)];
  const int64_t t = ((int64_t)blockIdx.x - b.block0) * kBS + threadIdx.x;
  if (t >= b.count) return;
  OpSel os;
  os.nops = a.nops;
#pragma unroll
  for (int o = 0; o < kMaxOps; ++o) { os.slot[o] = a.op_store[o]; os.wall_only[o] = a.op_wall_only[o]; }
  const T *u = static_cast<const T *>(a.u);
  T *out = static_cast<T *>(a.out);
  const int64_t N = a.N;
  switch (b.width) {
    case 5: apply_node<T, A, 5>(u, out, N, os, b, t); break;
    case 7: apply_node<T, A, 7>(u, out, N, os, b, t); break;
    case 12: apply_node<T, A, 12>(u, out, N, os, b, t); break;
    case 20: apply_node<T, A, 20>(u, out, N, os, b, t); break;
    case 30: apply_node<T, A, 30>(u, out, N, os, b, t); break;
    default: apply_node<T, A, 0>(u, out, N, os, b, t); break;
  }
}

// Four independent 16-byte loads in flight per thread, nontemporal (streamed
// data is not reused), grid-stride over the buffer.
typedef int v4i __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_stream_copy(const v4i *__restrict__ src, v4i *__restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    v4i v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = __builtin_nontemporal_load(src + i + k * stride);
#pragma unroll
    for (int k = 0; k < 4; ++k) __builtin_nontemporal_store(v[k], dst + i + k * stride);
  }
  for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__global__ void k_to_f32(const double *src, float *dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

}  // namespace

void make_table(const hsm_stencils *st, BucketTable &tab, int bs, uint32_t type_mask, bool fp32) {
  tab.nb = 0;
  tab.nblocks = 0;
  for (const Bucket &B : st->buckets) {
    if (!((type_mask >> B.type) & 1u) || B.count == 0) continue;
    BucketDesc &d = tab.b[tab.nb++];
    d.start = B.start;
    d.count = B.count;
    d.type = B.type;
    d.width = B.width;
    d.block0 = tab.nblocks;
    d.idx = B.idx.as<int32_t>();
    d.w = fp32 ? B.w32.p : B.w.p;
    d.aux = nullptr;
    d.nops = B.nops;
    d.pad = 0;
    tab.nblocks += (B.count + bs - 1) / bs;
  }
}

hsm_status ensure_w32(const hsm_stencils *st, hipStream_t s) {
  if (st->w32_ready) return HSM_OK;
  for (const Bucket &B0 : st->buckets) {
    Bucket &B = const_cast<Bucket &>(B0);
    const int64_t n = (int64_t)B.nops * B.width * B.count;
    hsm_status rc = B.w32.alloc(sizeof(float) * (n > 0 ? n : 1));
    if (rc) return rc;
    if (n > 0) {
      hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, B.w.as<double>(),
                         B.w32.as<float>(), n);
      HSM_HIP(hipGetLastError());
    }
  }
  st->w32_ready = true;
  return HSM_OK;
}

hsm_status apply_impl(const hsm_stencils *st, uint32_t op_mask, int32_t dtype, const void *u, void *out,
                      hipStream_t s) {
  ApplyArgs a;
  const int d = st->d;
  a.nops = 0;
  const uint32_t bits[5] = {HSM_OP_DX, HSM_OP_DY, HSM_OP_DZ, HSM_OP_LAP, HSM_OP_DN};
  for (int k = 0; k < 5; ++k) {
    if (!(op_mask & bits[k])) continue;
    int slot, wall_only = 0;
    if (k < 3) slot = (k < d) ? k : -1;
    else if (k == 3) slot = d;
    else { slot = d + 1; wall_only = 1; }
    a.op_store[a.nops] = slot;
    a.op_wall_only[a.nops] = wall_only;
    a.nops++;
  }
  const bool fp32 = dtype != HSM_F64;
  if (fp32) {
    hsm_status rc = ensure_w32(st, s);
    if (rc) return rc;
  }
  const int which = fp32 ? 1 : 0;
  if (st->dtab_blocks[which] < 0) {
    BucketTable tab;
    make_table(st, tab, kBS, 0xFu, fp32);
    hsm_status rc = st->dtab[which].alloc(sizeof(BucketTable));
    if (rc) return rc;
    HSM_HIP(hipMemcpyAsync(st->dtab[which].p, &tab, sizeof(BucketTable), hipMemcpyHostToDevice, s));
    HSM_HIP(hipStreamSynchronize(s));
    st->dtab_blocks[which] = tab.nblocks;
    st->bmap[which] = make_blockmap(tab);
  }
  a.tab = st->dtab[which].as<BucketTable>();
  a.bm = st->bmap[which];
  a.u = u;
  a.out = out;
  a.N = st->N;
  const int64_t nblocks = st->dtab_blocks[which];
  if (nblocks == 0 || a.nops == 0) return HSM_OK;
  const dim3 g((unsigned)nblocks), b(kBS);
  if (dtype == HSM_F64) hipLaunchKernelGGL((k_apply<double, Acc<double>>), g, b, 0, s, a);
  else if (dtype == HSM_F32) hipLaunchKernelGGL((k_apply<float, Acc<float>>), g, b, 0, s, a);
  else hipLaunchKernelGGL((k_apply<float, Dot2>), g, b, 0, s, a);
  HSM_HIP(hipGetLastError());
  return HSM_OK;
}

}  // namespace hsm

extern "C" hsm_status hsm_stream_copy(const void *src, void *dst, int64_t bytes, void *stream) {
  using namespace hsm;
  if (!src || !dst || bytes < 0 || (bytes % 16) != 0) {
    set_error(HSM_E_INVALID, "hsm_stream_copy needs non-NULL buffers and a byte count that is a multiple of 16");
    return HSM_E_INVALID;
  }
  const int64_t n = bytes / 16;
  if (n == 0) return HSM_OK;
  // 256 CUs x 8 blocks of 256 threads resident; grid-stride beyond
  int64_t blocks = (n + 1023) / 1024;
  if (blocks > 256 * 8) blocks = 256 * 8;
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, (const v4i *)src,
                     (v4i *)dst, n);
  HSM_HIP(hipGetLastError());
  return HSM_OK;
}
