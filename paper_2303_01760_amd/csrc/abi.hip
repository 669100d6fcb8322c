// C ABI entry points (include/hsm.h): argument checks, error reporting,
// export of stencils in the caller's numbering, and order conversion.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hsm_internal.h"

namespace hsm {

static thread_local std::string g_msg = "no error";
static thread_local int64_t g_node = -1;

void set_error(hsm_status code, const std::string &msg, int64_t node) {
  g_msg = "hsm error " + std::to_string(code) + ": " + msg;
  if (node >= 0) g_msg += " (node " + std::to_string(node) + ")";
  g_node = node;
}

hsm_status hip_fail(hipError_t e, const char *what) {
  (void)hipGetLastError();
  set_error(HSM_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return HSM_E_HIP;
}

bool rbffd_supported(int d, int m, int n);

namespace {

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <class T>
__global__ void k_permute(const T *src, T *dst, const int32_t *map, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[map[i]];
}

struct ExportArgs {
  BucketTable tab;
  const int32_t *perm, *iperm;
  int64_t N;
  int d;
  const int64_t *off;   // [N+1] caller numbering
  int32_t *width;       // [N]
  int32_t *idx;         // [nnz]
  double *w;            // [d+2][nnz]
  int64_t nnz;
  const void *wptr[kMaxBuckets];
};

__device__ int bucket_of(const BucketTable &tab, int64_t t) {
  int bi = 0;
  for (int k = 1; k < tab.nb; ++k)
    if (t >= tab.b[k].start) bi = k;
  return bi;
}

__global__ void k_export_width(ExportArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  const int64_t t = a.iperm[i];
  a.width[i] = a.tab.b[bucket_of(a.tab, t)].width;
}

__global__ void k_export_fill(ExportArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  const int64_t t = a.iperm[i];
  const int bi = bucket_of(a.tab, t);
  const BucketDesc &b = a.tab.b[bi];
  const int64_t tb = t - b.start, cnt = b.count;
  const int W = b.width;
  const double *w = static_cast<const double *>(a.wptr[bi]);
  const bool wall = (b.type == B_DIR || b.type == B_NEU);
  const int64_t o = a.off[i];
  for (int j = 0; j < W; ++j) {
    a.idx[o + j] = a.perm[b.idx[(int64_t)j * cnt + tb]];
    for (int q = 0; q <= a.d; ++q) a.w[q * a.nnz + o + j] = w[((int64_t)q * W + j) * cnt + tb];
    a.w[(a.d + 1) * a.nnz + o + j] = wall ? w[((int64_t)(a.d + 1) * W + j) * cnt + tb] : 0.0;
  }
}

bool check_ptr(const void *p, const char *name) {
  if (!p) { set_error(HSM_E_INVALID, std::string(name) + " is NULL"); return false; }
  return true;
}

// The fixed scratch array of hsm_stencils_export_noalloc.  Each GPU that
// loads the library holds its own copy until the process ends.  In host code
// `scratch` names a host-side stand-in, not device memory: kernels and copies
// take the device address that hipGetSymbolAddress returns for the current
// device (static_scratch), never the array's name.
constexpr size_t kStaticScratchBytes = (size_t)HSM_EXPORT_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
hsm_status static_scratch(void **out) {
  int dev = -1;
  HSM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error(HSM_E_HIP, "device index out of range");
    return HSM_E_HIP;
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) {
      set_error(HSM_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
      return HSM_E_HIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return HSM_OK;
}

// Device temporaries of an export: widths [N], offsets [N+1], indices
// [nnz], weights [d+2][nnz] and the prefix-sum workspace, each 256-byte aligned.
struct ExportScratch {
  int32_t *width;
  int64_t *off;
  int32_t *idx;
  double *w;
  int64_t *ws;
};
size_t export_scratch_bytes(const hsm_stencils *st) {
  const int64_t N = st->N, nnz = st->nnz;
  return round256(sizeof(int32_t) * N) + round256(sizeof(int64_t) * (N + 1)) + round256(sizeof(int32_t) * nnz) +
         round256(sizeof(double) * (st->d + 2) * nnz) + round256(sizeof(int64_t) * scan_i32_to_i64_ws(N));
}
ExportScratch carve_export_scratch(const hsm_stencils *st, void *base) {
  const int64_t N = st->N, nnz = st->nnz;
  char *p = static_cast<char *>(base);
  ExportScratch e;
  e.width = reinterpret_cast<int32_t *>(p); p += round256(sizeof(int32_t) * N);
  e.off = reinterpret_cast<int64_t *>(p); p += round256(sizeof(int64_t) * (N + 1));
  e.idx = reinterpret_cast<int32_t *>(p); p += round256(sizeof(int32_t) * nnz);
  e.w = reinterpret_cast<double *>(p); p += round256(sizeof(double) * (st->d + 2) * nnz);
  e.ws = reinterpret_cast<int64_t *>(p);
  return e;
}

// Stencils in the caller's numbering, copied to host memory.  scr: device
// scratch of export_scratch_bytes(st) bytes, or NULL to allocate it (device
// buffers for the arrays, the scratch pool for the prefix sum).  Every byte of
// scratch that is read is first written by this call.
hsm_status export_impl(const hsm_stencils *st, uint8_t *host_class, int64_t *host_offsets, int32_t *host_idx,
                       double *host_w, hipStream_t s, void *scr) {
  if (!check_ptr(st, "stencils")) return HSM_E_INVALID;
  const int64_t N = st->N;
  if (host_class && N > 0) HSM_HIP(hipMemcpyAsync(host_class, st->cls.p, N, hipMemcpyDeviceToHost, s));
  if (host_offsets || host_idx || host_w) {
    ExportArgs a;
    make_table(st, a.tab, 256, 0xFu, false);
    int k = 0;
    for (const Bucket &B : st->buckets)
      if (B.count) a.wptr[k++] = B.w.p;
    a.perm = st->perm.as<int32_t>(); a.iperm = st->iperm.as<int32_t>(); a.N = N; a.d = st->d; a.nnz = st->nnz;
    DBuf width, offs, idx, w;
    ExportScratch e{};
    hsm_status rc;
    if (scr) {
      e = carve_export_scratch(st, scr);
    } else {
      if ((rc = width.alloc(sizeof(int32_t) * N)) || (rc = offs.alloc(sizeof(int64_t) * (N + 1))) ||
          (rc = idx.alloc(sizeof(int32_t) * st->nnz)) || (rc = w.alloc(sizeof(double) * (st->d + 2) * st->nnz)))
        return rc;
      e = ExportScratch{width.as<int32_t>(), offs.as<int64_t>(), idx.as<int32_t>(), w.as<double>(), nullptr};
    }
    a.width = e.width; a.off = e.off; a.idx = e.idx; a.w = e.w;
    if (N > 0) {
      hipLaunchKernelGGL(k_export_width, dim3(nblk(N, 256)), dim3(256), 0, s, a);
      HSM_HIP(hipGetLastError());
    }
    if ((rc = scan_i32_to_i64(e.width, e.off, N, s, e.ws))) return rc;
    if (N > 0) {
      hipLaunchKernelGGL(k_export_fill, dim3(nblk(N, 256)), dim3(256), 0, s, a);
      HSM_HIP(hipGetLastError());
    }
    if (host_offsets) HSM_HIP(hipMemcpyAsync(host_offsets, e.off, sizeof(int64_t) * (N + 1), hipMemcpyDeviceToHost, s));
    if (host_idx) HSM_HIP(hipMemcpyAsync(host_idx, e.idx, sizeof(int32_t) * st->nnz, hipMemcpyDeviceToHost, s));
    if (host_w)
      HSM_HIP(hipMemcpyAsync(host_w, e.w, sizeof(double) * (st->d + 2) * st->nnz, hipMemcpyDeviceToHost, s));
    HSM_HIP(hipStreamSynchronize(s));
    return HSM_OK;
  }
  HSM_HIP(hipStreamSynchronize(s));
  return HSM_OK;
}

}  // namespace
}  // namespace hsm

using namespace hsm;

extern "C" {

const char *hsm_last_error(void) { return g_msg.c_str(); }
int64_t hsm_last_error_node(void) { return g_node; }
const char *hsm_version(void) { return "hsm 0.1 (gfx950)"; }

hsm_status hsm_build_stencils(const hsm_nodeset *ns, int32_t mode, void *stream, hsm_stencils **out) {
  if (!check_ptr(ns, "nodes") || !check_ptr(out, "out")) return HSM_E_INVALID;
  *out = nullptr;
  if (ns->d != 2 && ns->d != 3) { set_error(HSM_E_INVALID, "d must be 2 or 3"); return HSM_E_INVALID; }
  if (mode != HSM_MODE_HYBRID && mode != HSM_MODE_ALL_SCATTERED) {
    set_error(HSM_E_INVALID, "unknown mode");
    return HSM_E_INVALID;
  }
  if (ns->n_domains < 1 || ns->n_domains > (1 << 20)) { set_error(HSM_E_INVALID, "n_domains out of range"); return HSM_E_INVALID; }
  if (ns->tile_log2 < 0 || ns->tile_log2 > 5) { set_error(HSM_E_INVALID, "tile_log2 must be 0 (default) or 1..5"); return HSM_E_INVALID; }
  if (ns->solve_groups < 0 || ns->solve_groups > 3) { set_error(HSM_E_INVALID, "solve_groups must be 0 (auto), 1, 2 or 3"); return HSM_E_INVALID; }
  if (!check_ptr(ns->host_domain_offsets, "host_domain_offsets") || !check_ptr(ns->host_h_regular, "host_h_regular") ||
      !check_ptr(ns->host_m, "host_m"))
    return HSM_E_INVALID;
  const int64_t *off = ns->host_domain_offsets;
  if (off[0] != 0) { set_error(HSM_E_INVALID, "host_domain_offsets[0] must be 0"); return HSM_E_INVALID; }
  for (int k = 0; k < ns->n_domains; ++k) {
    const int m = ns->host_m[k];
    const int n = ns->host_n ? ns->host_n[k] : 2 * nmono(ns->d, m < 0 ? 0 : m);
    if (m < 1 || !rbffd_supported(ns->d, m, n)) {
      set_error(HSM_E_INVALID, "unsupported (d, m, n) = (" + std::to_string(ns->d) + ", " + std::to_string(m) + ", " +
                                   std::to_string(n) + ") in domain " + std::to_string(k));
      return HSM_E_INVALID;
    }
    if (!(ns->host_h_regular[k] > 0) || !std::isfinite(ns->host_h_regular[k])) {
      set_error(HSM_E_INVALID, "h_regular must be positive in domain " + std::to_string(k));
      return HSM_E_INVALID;
    }
    if (off[k + 1] - off[k] < std::max(n, 2 * ns->d + 1)) {
      set_error(HSM_E_INVALID, "domain " + std::to_string(k) + " has fewer nodes than its stencil size");
      return HSM_E_INVALID;
    }
  }
  const int64_t N = off[ns->n_domains];
  // kernels address node vectors of up to 16-byte elements with 32-bit byte offsets
  if (N > HSM_MAX_NODES) { set_error(HSM_E_INVALID, "too many nodes (at most HSM_MAX_NODES)"); return HSM_E_INVALID; }
  if (!check_ptr(ns->x, "x") || !check_ptr(ns->kind, "kind") || !check_ptr(ns->normal, "normal"))
    return HSM_E_INVALID;
  hsm_status rc = build_stencils_impl(ns, mode, (hipStream_t)stream, out);
  if (rc != HSM_OK) *out = nullptr;
  return rc;
}

hsm_status hsm_stencils_get_info(const hsm_stencils *st, hsm_stencils_info *o) {
  if (!check_ptr(st, "stencils") || !check_ptr(o, "out")) return HSM_E_INVALID;
  std::memset(o, 0, sizeof(*o));
  o->d = st->d; o->mode = st->mode; o->n_domains = st->n_domains;
  o->n_buckets = (int32_t)st->buckets.size();
  o->n_nodes = st->N; o->nnz = st->nnz; o->n_regular = st->n_regular; o->n_scattered = st->n_scattered;
  o->n_boundary = st->n_boundary;
  o->n_wall_fallback = st->n_wall_fallback;
  for (size_t k = 0; k < st->buckets.size() && k < 16; ++k) {
    o->bucket_width[k] = st->buckets[k].width;
    o->bucket_type[k] = st->buckets[k].type;
    o->bucket_count[k] = st->buckets[k].count;
  }
  for (int k = 0; k < 4; ++k) o->build_ms[k] = st->build_ms[k];
  for (int k = 0; k < 16; ++k) o->bucket_solve_ms[k] = st->bucket_solve_ms[k];
  return HSM_OK;
}

hsm_status hsm_stencils_export(const hsm_stencils *st, uint8_t *host_class, int64_t *host_offsets, int32_t *host_idx,
                               double *host_w, void *stream) {
  return export_impl(st, host_class, host_offsets, host_idx, host_w, (hipStream_t)stream, nullptr);
}

hsm_status hsm_stencils_export_noalloc(const hsm_stencils *st, uint8_t *host_class, int64_t *host_offsets,
                                       int32_t *host_idx, double *host_w, void *stream) {
  if (!check_ptr(st, "stencils")) return HSM_E_INVALID;
  const size_t need = export_scratch_bytes(st);
  if (need > kStaticScratchBytes) {
    set_error(HSM_E_INVALID, "hsm_stencils_export_noalloc needs " + std::to_string(need) +
                                 " bytes of scratch; its fixed device array holds " +
                                 std::to_string(kStaticScratchBytes) + " (use hsm_stencils_export)");
    return HSM_E_INVALID;
  }
  void *scr = nullptr;
  hsm_status rc = static_scratch(&scr);
  if (rc != HSM_OK) return rc;
  return export_impl(st, host_class, host_offsets, host_idx, host_w, (hipStream_t)stream, scr);
}

hsm_status hsm_permute(const hsm_stencils *st, int32_t direction, int32_t dtype, const void *src, void *dst,
                       void *stream) {
  if (!check_ptr(st, "stencils")) return HSM_E_INVALID;
  if (st->N == 0) return HSM_OK;
  if (!check_ptr(src, "src") || !check_ptr(dst, "dst")) return HSM_E_INVALID;
  if (src == dst) { set_error(HSM_E_INVALID, "src and dst must differ"); return HSM_E_INVALID; }
  if (direction != HSM_TO_INTERNAL && direction != HSM_TO_CALLER) { set_error(HSM_E_INVALID, "bad direction"); return HSM_E_INVALID; }
  const int32_t *map = direction == HSM_TO_INTERNAL ? st->perm.as<int32_t>() : st->iperm.as<int32_t>();
  hipStream_t s = (hipStream_t)stream;
  const dim3 g(nblk(st->N, 256)), b(256);
  if (dtype == HSM_F64) hipLaunchKernelGGL(k_permute<double>, g, b, 0, s, (const double *)src, (double *)dst, map, st->N);
  else if (dtype == HSM_F32) hipLaunchKernelGGL(k_permute<float>, g, b, 0, s, (const float *)src, (float *)dst, map, st->N);
  else { set_error(HSM_E_INVALID, "dtype must be HSM_F64 or HSM_F32"); return HSM_E_INVALID; }
  HSM_HIP(hipGetLastError());
  return HSM_OK;
}

hsm_status hsm_apply_operator(const hsm_stencils *st, uint32_t op_mask, int32_t dtype, const void *u, void *out,
                              void *stream) {
  if (!check_ptr(st, "stencils")) return HSM_E_INVALID;
  if (op_mask == 0 || (op_mask & ~31u)) { set_error(HSM_E_INVALID, "op_mask must be a nonzero set of HSM_OP_* bits"); return HSM_E_INVALID; }
  if (dtype != HSM_F64 && dtype != HSM_F32 && dtype != HSM_F32_COMP) { set_error(HSM_E_INVALID, "bad dtype"); return HSM_E_INVALID; }
  if ((op_mask & HSM_OP_DZ) && st->d < 3) { set_error(HSM_E_INVALID, "HSM_OP_DZ needs d = 3"); return HSM_E_INVALID; }
  if (st->N == 0) return HSM_OK;
  if (!check_ptr(u, "u") || !check_ptr(out, "out")) return HSM_E_INVALID;
  if (u == out) { set_error(HSM_E_INVALID, "u and out must not overlap"); return HSM_E_INVALID; }
  return apply_impl(st, op_mask, dtype, u, out, (hipStream_t)stream);
}

hsm_status hsm_apply_operator_buckets(const hsm_stencils *st, uint32_t op_mask, int32_t dtype, uint32_t bucket_mask,
                                      const void *u, void *out, void *stream) {
  if (bucket_mask == 0) { set_error(HSM_E_INVALID, "bucket_mask selects no bucket"); return HSM_E_INVALID; }
  if (!check_ptr(st, "stencils")) return HSM_E_INVALID;
  if (op_mask == 0 || (op_mask & ~31u)) { set_error(HSM_E_INVALID, "op_mask must be a nonzero set of HSM_OP_* bits"); return HSM_E_INVALID; }
  if (dtype != HSM_F64 && dtype != HSM_F32 && dtype != HSM_F32_COMP) { set_error(HSM_E_INVALID, "bad dtype"); return HSM_E_INVALID; }
  if ((op_mask & HSM_OP_DZ) && st->d < 3) { set_error(HSM_E_INVALID, "HSM_OP_DZ needs d = 3"); return HSM_E_INVALID; }
  if (st->N == 0) return HSM_OK;
  if (!check_ptr(u, "u") || !check_ptr(out, "out")) return HSM_E_INVALID;
  if (u == out) { set_error(HSM_E_INVALID, "u and out must not overlap"); return HSM_E_INVALID; }
  return apply_impl(st, op_mask, dtype, u, out, (hipStream_t)stream, bucket_mask);
}

int64_t hsm_apply_node_count(const hsm_stencils *st, uint32_t op_mask) {
  if (!st) return 0;
  int64_t total = 0;
  int nop_all = 0;
  for (uint32_t b : {HSM_OP_DX, HSM_OP_DY, HSM_OP_DZ, HSM_OP_LAP})
    if (op_mask & b) ++nop_all;
  for (const Bucket &B : st->buckets) {
    total += B.count * nop_all;
    if ((op_mask & HSM_OP_DN) && (B.type == B_DIR || B.type == B_NEU)) total += B.count;
  }
  return total;
}

hsm_status hsm_stencils_condition(const hsm_stencils *st, double *kappa, void *stream) {
  if (!check_ptr(st, "stencils")) return HSM_E_INVALID;
  if (st->N == 0) return HSM_OK;
  if (!check_ptr(kappa, "kappa")) return HSM_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  hsm_status rc;
  for (const Bucket &B : st->buckets)
    if ((rc = cond_bucket(st, B, kappa, s, nullptr, 0))) return rc;
  if (st->n_wall_fallback > 0) {
    // the wall nodes that were solved with degree m-1: their own system
    const int32_t *list = st->fallback.as<int32_t>() + 1;
    for (const Bucket &B : st->buckets)
      if (B.type == B_DIR || B.type == B_NEU)
        if ((rc = cond_bucket(st, B, kappa, s, list, st->n_wall_fallback))) return rc;
  }
  return HSM_OK;
}

void hsm_stencils_destroy(hsm_stencils *st) { delete st; }

}  // extern "C"
