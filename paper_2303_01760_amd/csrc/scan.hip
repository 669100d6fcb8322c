// Device-wide exclusive prefix sums (three passes: tile sums, scan of the
// tile sums, tile scans).  Deterministic: integer sums, fixed tiling.
#include <cstring>
#include <mutex>

#include "hsm_internal.h"

namespace hsm {
namespace {

constexpr int kBS = 256;     // threads per block
constexpr int kIPT = 8;      // items per thread
constexpr int kTile = kBS * kIPT;

__device__ int64_t block_exclusive_scan(int64_t v, int64_t *total) {
  __shared__ int64_t wsum[kBS / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wv] = x;
  __syncthreads();
  int64_t base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kBS / 64; ++k) {
    if (k < wv) base += wsum[k];
    tot += wsum[k];
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

template <class T>
__global__ __launch_bounds__(kBS) void k_tile_sums(const T *in, int64_t n, int64_t *sums) {
  const int64_t base = (int64_t)blockIdx.x * kTile;
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kIPT; ++k) {
    int64_t i = base + (int64_t)k * kBS + threadIdx.x;
    if (i < n) s += (int64_t)in[i];
  }
  int64_t tot;
  (void)block_exclusive_scan(s, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <class T>
__global__ __launch_bounds__(kBS) void k_tile_scan(const T *in, int64_t n, const int64_t *offs, int64_t *out,
                                                   int write_total) {
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kIPT;
  int64_t vals[kIPT];
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kIPT; ++k) {
    int64_t i = base + k;
    vals[k] = (i < n) ? (int64_t)in[i] : 0;
    s += vals[k];
  }
  int64_t tot;
  int64_t run = block_exclusive_scan(s, &tot) + (offs ? offs[blockIdx.x] : 0);
#pragma unroll
  for (int k = 0; k < kIPT; ++k) {
    int64_t i = base + k;
    if (i < n) out[i] = run;
    run += vals[k];
  }
  if (write_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kBS - 1) out[n] = run;
}

int64_t scan_ws(int64_t n) {
  if (n <= kTile) return 0;
  const int64_t nt = (n + kTile - 1) / kTile;
  return 2 * nt + 1 + scan_ws(nt);
}

// ws: scan_ws(n) int64 of scratch, or NULL to take it from the scratch pool
template <class T>
hsm_status scan_any(const T *in, int64_t *out, int64_t n, hipStream_t s, int64_t *ws) {
  if (n <= 0) {
    hipLaunchKernelGGL(k_tile_scan<T>, dim3(1), dim3(kBS), 0, s, in, (int64_t)0, (const int64_t *)nullptr,
                       out, 1);
    HSM_HIP(hipGetLastError());
    return HSM_OK;
  }
  const int64_t nt = (n + kTile - 1) / kTile;
  if (nt == 1) {
    hipLaunchKernelGGL(k_tile_scan<T>, dim3(1), dim3(kBS), 0, s, in, n, (const int64_t *)nullptr, out, 1);
    HSM_HIP(hipGetLastError());
    return HSM_OK;
  }
  SBuf own;
  hsm_status rc;
  if (!ws) {
    if ((rc = own.alloc(sizeof(int64_t) * scan_ws(n), s)) != HSM_OK) return rc;
    ws = own.as<int64_t>();
  }
  int64_t *sums = ws, *offs = ws + nt;
  hipLaunchKernelGGL(k_tile_sums<T>, dim3((unsigned)nt), dim3(kBS), 0, s, in, n, sums);
  HSM_HIP(hipGetLastError());
  if ((rc = scan_any<int64_t>(sums, offs, nt, s, ws + 2 * nt + 1)) != HSM_OK) return rc;
  hipLaunchKernelGGL(k_tile_scan<T>, dim3((unsigned)nt), dim3(kBS), 0, s, in, n, (const int64_t *)offs, out, 1);
  HSM_HIP(hipGetLastError());
  return HSM_OK;    // the temporaries are released in stream order
}

}  // namespace

hsm_status scan_i32_to_i64(const int32_t *in, int64_t *out, int64_t n, hipStream_t s, int64_t *ws) {
  return scan_any<int32_t>(in, out, n, s, ws);
}

int64_t scan_i32_to_i64_ws(int64_t n) { return scan_ws(n); }

hipMemPool_t scratch_pool(int device) {
  static std::mutex mu;
  static hipMemPool_t pools[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(mu);
  if (!pools[device]) {
    hipMemPoolProps props;
    std::memset(&props, 0, sizeof(props));
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = device;
    hipMemPool_t pool = nullptr;
    if (hipMemPoolCreate(&pool, &props) != hipSuccess) return nullptr;
    uint64_t keep = kScratchPoolKeep;
    if (hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess) {
      (void)hipMemPoolDestroy(pool);
      return nullptr;
    }
    pools[device] = pool;
  }
  return pools[device];
}

}  // namespace hsm
