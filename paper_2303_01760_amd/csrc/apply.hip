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
// twice the working precision.  Both FP32 forms sum w_j (u_j - u_c) over the
// non-centre entries (equal to Eq. (1): the weights of every operator sum to
// zero), so the error of each rounded weight scales with a difference of
// nearby values, not with the field's magnitude.  Built with
// -ffp-contract=off; every FMA below is written out.
#include <hip/hip_runtime.h>

#include <type_traits>

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
  int nops;                  // requested operators = output planes
  int ld_slot[kMaxOps];      // storage slot of each stored operator that is computed
  int ld_wall_only[kMaxOps]; // 1: only wall buckets hold it (normal derivative); 0 elsewhere
  int out_src[kMaxOps];      // output plane o takes computed operator out_src[o]; -1: zero (not stored)
};

// One node: NL operators computed from one pass over the stencil (the
// indices and gathered values are shared), W entries (0: width known only
// at run time).
template <class T, class A, int NL, int W>
__device__ __forceinline__ void apply_node(const ApplyArgs &a, const BucketDesc &b, int64_t t) {
  const uint32_t cnt = (uint32_t)b.count, t32 = (uint32_t)t;
  const int width = (W > 0) ? W : b.width;
  const bool wall = (b.type == B_DIR || b.type == B_NEU);
  bool live[NL];
  uint32_t row0[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    live[k] = !a.ld_wall_only[k] || wall;
    row0[k] = (uint32_t)((live[k] ? a.ld_slot[k] : 0) * width);   // a present row keeps every load valid
  }
  // FP32: the difference form sum_{j>=1} w_j (u_j - u_c), u_c the centre
  // value (stencil entry 0).  Every operator annihilates constants, so its
  // weights sum to zero and this equals Eq. (1); but the rounding of each
  // FP32 weight then multiplies a difference of nearby values instead of the
  // value itself, and the centre weight is not read.
  constexpr bool kDiff = std::is_same<T, float>::value;
  A acc[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) acc[k].init();
  T uc = T(0);
  const Buf ub = plane(static_cast<const T *>(a.u), a.N, 0);
  const auto wl = [&](int j) __attribute__((always_inline)) {
    Pack<T, NL> r;
#pragma unroll
    for (int k = 0; k < NL; ++k) r.v[k] = (kDiff && j == 0) ? T(0) : ld_soa<T>(b.w, cnt, row0[k] + j, t32);
    return r;
  };
  const auto vl = [&](int32_t nb) __attribute__((always_inline)) { return ld_at<T>(ub, nb); };
  const auto use = [&](int j, const Pack<T, NL> &wv, T uv) __attribute__((always_inline)) {
    if (kDiff && j == 0) {
      uc = uv;
      return;
    }
    const T du = kDiff ? T(uv - uc) : uv;
#pragma unroll
    for (int k = 0; k < NL; ++k) acc[k].add(wv.v[k], du);
  };
  if constexpr (W > 0) {
    gather_chunks<W, 8>(b.idx, cnt, t32, wl, vl, use, [&]() __attribute__((always_inline)) {
#pragma unroll
      for (int k = 0; k < NL; ++k) acc[k].settle();
    });
  } else {
    for (int j = 0; j < width; ++j) use(j, wl(j), vl(ld_soa<int32_t>(b.idx, cnt, j, t32)));
  }
  T *out = static_cast<T *>(a.out);
  for (int o = 0; o < a.nops; ++o) {
    const int src = a.out_src[o];
    T val = T(0);
#pragma unroll
    for (int k = 0; k < NL; ++k)
      if (src == k && live[k]) val = (T)acc[k].get();
    out[(int64_t)o * a.N + b.start + t] = val;
  }
}

template <class T, class A, int NL>
__global__ __launch_bounds__(kBS) void k_apply(ApplyArgs a) {
  const BucketDesc b = a.tab->b[bucket_index(a.bm, blockIdx.x)];
  const int64_t t = ((int64_t)blockIdx.x - b.block0) * kBS + threadIdx.x;
  if (t >= b.count) return;
  switch (b.width) {
    case 5: apply_node<T, A, NL, 5>(a, b, t); break;
    case 6: apply_node<T, A, NL, 6>(a, b, t); break;
    case 7: apply_node<T, A, NL, 7>(a, b, t); break;
    case 8: apply_node<T, A, NL, 8>(a, b, t); break;
    case 12: apply_node<T, A, NL, 12>(a, b, t); break;
    case 20: apply_node<T, A, NL, 20>(a, b, t); break;
    case 30: apply_node<T, A, NL, 30>(a, b, t); break;
    case 40: apply_node<T, A, NL, 40>(a, b, t); break;
    default: apply_node<T, A, NL, 0>(a, b, t); break;
  }
}

// A launch with nl computed operators.
template <class T, class A>
void launch_apply(int nl, dim3 g, dim3 bs, hipStream_t s, const ApplyArgs &a) {
  switch (nl) {
    case 1: hipLaunchKernelGGL((k_apply<T, A, 1>), g, bs, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_apply<T, A, 2>), g, bs, 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_apply<T, A, 3>), g, bs, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_apply<T, A, 4>), g, bs, 0, s, a); break;
    default: hipLaunchKernelGGL((k_apply<T, A, 5>), g, bs, 0, s, a); break;
  }
}

template <class T>
__global__ void k_zero(T *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = T(0);
}

// One 16-byte element per thread, one thread per element: the simplest
// streaming pattern is also the fastest measured on this part (the
// hardware keeps enough loads in flight across the resident waves).
typedef int v4i __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_stream_copy(const v4i *__restrict__ src, v4i *__restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void k_to_f32(const double *src, float *dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

}  // namespace

void make_table(const hsm_stencils *st, BucketTable &tab, int bs, uint32_t type_mask, bool fp32,
                uint32_t bucket_mask) {
  tab.nb = 0;
  tab.nblocks = 0;
  for (size_t k = 0; k < st->buckets.size(); ++k) {
    const Bucket &B = st->buckets[k];
    if (!((type_mask >> B.type) & 1u) || B.count == 0) continue;
    if (k < 32 && !((bucket_mask >> k) & 1u)) continue;
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
                      hipStream_t s, uint32_t bucket_mask) {
  ApplyArgs a;
  const int d = st->d;
  a.nops = 0;
  int nl = 0;
  const uint32_t bits[5] = {HSM_OP_DX, HSM_OP_DY, HSM_OP_DZ, HSM_OP_LAP, HSM_OP_DN};
  for (int k = 0; k < 5; ++k) {
    if (!(op_mask & bits[k])) continue;
    int slot, wall_only = 0;
    if (k < 3) slot = (k < d) ? k : -1;
    else if (k == 3) slot = d;
    else { slot = d + 1; wall_only = 1; }
    if (slot >= 0) {
      a.ld_slot[nl] = slot;
      a.ld_wall_only[nl] = wall_only;
      a.out_src[a.nops] = nl++;
    } else {
      a.out_src[a.nops] = -1;
    }
    a.nops++;
  }
  for (int k = nl; k < kMaxOps; ++k) { a.ld_slot[k] = 0; a.ld_wall_only[k] = 0; }
  for (int o = a.nops; o < kMaxOps; ++o) a.out_src[o] = -1;
  const bool fp32 = dtype != HSM_F64;
  if (fp32) {
    hsm_status rc = ensure_w32(st, s);
    if (rc) return rc;
  }
  const int which = fp32 ? 1 : 0;
  const bool all = (bucket_mask | ~((st->buckets.size() >= 32) ? 0xFFFFFFFFu
                                                                : ((1u << st->buckets.size()) - 1u))) == 0xFFFFFFFFu;
  int64_t nblocks;
  if (all) {
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
    nblocks = st->dtab_blocks[which];
  } else {
    // a subset of the buckets: its own table (the last one is kept)
    const uint32_t key = (bucket_mask & 0x7FFFFFFFu) | (fp32 ? 0x80000000u : 0u);
    if (st->dtab_sub_key != key || !st->dtab_sub.p) {
      BucketTable tab;
      make_table(st, tab, kBS, 0xFu, fp32, bucket_mask);
      hsm_status rc = st->dtab_sub.alloc(sizeof(BucketTable));
      if (rc) return rc;
      HSM_HIP(hipMemcpyAsync(st->dtab_sub.p, &tab, sizeof(BucketTable), hipMemcpyHostToDevice, s));
      HSM_HIP(hipStreamSynchronize(s));
      st->dtab_sub_key = key;
      st->dtab_sub_blocks = tab.nblocks;
      st->bmap_sub = make_blockmap(tab);
    }
    a.tab = st->dtab_sub.as<BucketTable>();
    a.bm = st->bmap_sub;
    nblocks = st->dtab_sub_blocks;
  }
  a.u = u;
  a.out = out;
  a.N = st->N;
  if (nblocks == 0 || a.nops == 0) return HSM_OK;
  const dim3 g((unsigned)nblocks), b(kBS);
  if (nl == 0) {            // only operators that are not stored (d/dz in 2D): zeros on the selected rows
    for (size_t k = 0; k < st->buckets.size(); ++k) {
      const Bucket &B = st->buckets[k];
      if (B.count == 0 || (k < 32 && !((bucket_mask >> k) & 1u))) continue;
      const dim3 gz((unsigned)((B.count + 255) / 256));
      for (int o = 0; o < a.nops; ++o) {
        const int64_t off = (int64_t)o * a.N + B.start;
        if (dtype == HSM_F64)
          hipLaunchKernelGGL(k_zero<double>, gz, dim3(256), 0, s, static_cast<double *>(out) + off, B.count);
        else hipLaunchKernelGGL(k_zero<float>, gz, dim3(256), 0, s, static_cast<float *>(out) + off, B.count);
      }
    }
  } else if (dtype == HSM_F64) launch_apply<double, Acc<double>>(nl, g, b, s, a);
  else if (dtype == HSM_F32) launch_apply<float, Acc<float>>(nl, g, b, s, a);
  else launch_apply<float, Dot2>(nl, g, b, s, a);
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
  const int64_t blocks = (n + 255) / 256;
  if (blocks >= (1LL << 24)) { set_error(HSM_E_INVALID, "copy too large (at most 64 GiB per call)"); return HSM_E_INVALID; }
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, (const v4i *)src,
                     (v4i *)dst, n);
  HSM_HIP(hipGetLastError());
  return HSM_OK;
}
