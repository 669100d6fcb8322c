// Stencil construction on the GPU: per-domain cell grids, the
// regular/scattered classifier, exact k-nearest-neighbour search for the
// nodes that take RBF-FD stencils, the width-bucketed internal node order,
// and the per-bucket stencil index arrays.
//
// Compiled with -ffp-contract=off: squared distances and the axis-cross test
// are rounded step by step exactly as written, so neighbour lists and classes
// are bit-for-bit those of the definition (Section 2: stencils of n nearest
// nodes; MON on regular nodes, RBF-FD on scattered nodes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>

#include "hsm_internal.h"

namespace hsm {
namespace {

constexpr double kCrossTau = 1e-6;  // cross-detection tolerance in units of h_r

struct GridDesc {
  double origin[3];
  double cs;          // cell edge
  int32_t dims[3];    // cells per axis
  int32_t ntiles[3];  // tiles per axis
  int32_t tl;         // tile edge 2^tl cells (default 8x8 in 2D, 4x4x4 in 3D)
  int64_t cell_off;   // first global cell id of this domain
};

__device__ __forceinline__ int find_domain(int64_t i, const int64_t *off, int nd) {
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Cells are numbered tile by tile so that the cell-sorted node order is
// spatially compact (tiles of 2^tl cells per axis, row-major; by default
// 8x8 in 2D and 4x4x4 in 3D).
template <int D>
__device__ __forceinline__ int64_t cell_id(const GridDesc &g, const int *c) {
  const int L = g.tl, msk = (1 << L) - 1;
  if (D == 2) {
    const int64_t t = (int64_t)(c[1] >> L) * g.ntiles[0] + (c[0] >> L);
    return g.cell_off + (t << (2 * L)) + ((int64_t)(c[1] & msk) << L) + (c[0] & msk);
  } else {
    const int64_t t = ((int64_t)(c[2] >> L) * g.ntiles[1] + (c[1] >> L)) * g.ntiles[0] + (c[0] >> L);
    return g.cell_off + (t << (3 * L)) + ((int64_t)(c[2] & msk) << (2 * L)) + ((int64_t)(c[1] & msk) << L) +
           (c[0] & msk);
  }
}

template <int D>
__device__ __forceinline__ void cell_coords(const GridDesc &g, const double *p, int *c) {
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const double f = floor((p[a] - g.origin[a]) / g.cs);
    // NaN and negative values map to cell 0, values beyond the grid to the last cell
    c[a] = (f >= 0.0) ? ((f <= (double)(g.dims[a] - 1)) ? (int)f : g.dims[a] - 1) : 0;
  }
}

// ---------------------------------------------------------------- bbox ----
// Per-domain bounding boxes in two passes: block b covers chunk b % P of
// domain b / P (P chunks per domain) and writes its min and max; then one
// thread per (domain, bound component) folds the P partial values.
template <int D>
__global__ __launch_bounds__(256) void k_bbox_part(const double *x, int64_t N, const int64_t *off, int P,
                                                   double *part) {
  const int64_t b = blockIdx.x;
  const int64_t dm = b / P, j = b % P;
  const int64_t lo0 = off[dm], hi0 = off[dm + 1];
  const int64_t chunk = (hi0 - lo0 + P - 1) / P;
  const int64_t lo = lo0 + j * chunk, hi = min(lo + chunk, hi0);
  __shared__ double smin[256][D], smax[256][D];
  double mn[D], mx[D];
#pragma unroll
  for (int a = 0; a < D; ++a) { mn[a] = INFINITY; mx[a] = -INFINITY; }
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256)
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double v = x[a * N + i];
      mn[a] = fmin(mn[a], v);
      mx[a] = fmax(mx[a], v);
    }
#pragma unroll
  for (int a = 0; a < D; ++a) { smin[threadIdx.x][a] = mn[a]; smax[threadIdx.x][a] = mx[a]; }
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
#pragma unroll
      for (int a = 0; a < D; ++a) {
        smin[threadIdx.x][a] = fmin(smin[threadIdx.x][a], smin[threadIdx.x + st][a]);
        smax[threadIdx.x][a] = fmax(smax[threadIdx.x][a], smax[threadIdx.x + st][a]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 2 * D) {
    const int a = threadIdx.x % D, hiside = threadIdx.x / D;
    part[b * 6 + hiside * 3 + a] = hiside ? smax[0][a] : smin[0][a];
  }
}

// bbox[(dm * 2 + side) * 3 + a], a < D: side 0 the minimum, 1 the maximum;
// one wave per domain, lanes striding over the P partial boxes
template <int D>
__global__ __launch_bounds__(64) void k_bbox_fold(const double *part, int nd, int P, double *bbox) {
  const int64_t dm = blockIdx.x;
  const int lane = threadIdx.x;
  double mn[D], mx[D];
#pragma unroll
  for (int a = 0; a < D; ++a) { mn[a] = INFINITY; mx[a] = -INFINITY; }
  for (int j = lane; j < P; j += 64)
#pragma unroll
    for (int a = 0; a < D; ++a) {
      mn[a] = fmin(mn[a], part[(dm * P + j) * 6 + a]);
      mx[a] = fmax(mx[a], part[(dm * P + j) * 6 + 3 + a]);
    }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int a = 0; a < D; ++a) {
      mn[a] = fmin(mn[a], __shfl_xor(mn[a], o, 64));
      mx[a] = fmax(mx[a], __shfl_xor(mx[a], o, 64));
    }
  if (lane == 0)
#pragma unroll
    for (int a = 0; a < D; ++a) { bbox[(dm * 2 + 0) * 3 + a] = mn[a]; bbox[(dm * 2 + 1) * 3 + a] = mx[a]; }
}

// ------------------------------------------------------------ cell sort ---
template <int D>
__global__ void k_cell_of(const double *x, int64_t N, const int64_t *off, int nd, const GridDesc *grids,
                          int64_t *cell, int32_t *count, DevStatus *status) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int dm = find_domain(i, off, nd);
  double p[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    p[a] = x[a * N + i];
    if (!isfinite(p[a])) latch(status, BE_NONFINITE, i);
  }
  int c[3];
  cell_coords<D>(grids[dm], p, c);
  int64_t id = cell_id<D>(grids[dm], c);
  cell[i] = id;
  atomicAdd(&count[id], 1);
}

__global__ void k_cell_scatter(const int64_t *cell, int64_t N, const int64_t *start, int32_t *fill,
                               int32_t *nodes) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int64_t c = cell[i];
  int32_t k = atomicAdd(&fill[c], 1);
  nodes[start[c] + k] = (int32_t)i;
}

// each cell's list sorted by node index: the order of the cell-sorted node
// sequence (and so of the internal order) does not depend on atomics
__global__ void k_cell_sort(const int64_t *start, int64_t ncells, int32_t *nodes) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  int64_t lo = start[c], hi = start[c + 1];
  for (int64_t a = lo + 1; a < hi; ++a) {
    int32_t v = nodes[a];
    int64_t b = a - 1;
    while (b >= lo && nodes[b] > v) { nodes[b + 1] = nodes[b]; --b; }
    nodes[b + 1] = v;
  }
}

// positions and kinds in cell-sorted order
template <int D>
__global__ void k_sort_pos(const int32_t *nodes, int64_t N, const double *x, const uint8_t *kind, double *xs,
                           uint8_t *ks) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
  const int32_t j = nodes[s];
#pragma unroll
  for (int q = 0; q < D; ++q) xs[q * N + s] = x[q * N + j];
  ks[s] = kind[j];
}

// ------------------------------------------------- kNN + classifier -------
struct KnnArgs {
  const double *x;
  const uint8_t *kind;
  int64_t N;
  const int64_t *off;
  int nd;
  const GridDesc *grids;
  const int64_t *cell_start;
  const int32_t *cell_nodes;
  const int32_t *qlist;     // non-NULL: cell-sorted positions of the nodes that need neighbours
  const int64_t *nq;        // length of qlist (device)
  const double *xs;         // [D][N] positions in cell-sorted order (xs[s] = x[cell_nodes[s]])
  const uint8_t *ks;        // [N] kinds in cell-sorted order
  const int32_t *n_dom;     // stencil size per domain
  const double *h_dom;
  int hybrid;
  int32_t *knn;             // [K][N] caller numbering
  uint8_t *cls;             // [N]
  int32_t *cross;           // [2D][N]
  DevStatus *status;
};

template <int K>
__device__ __forceinline__ void topk_insert(double (&bd)[K], int32_t (&bj)[K], double d2, int32_t j) {
#pragma unroll
  for (int p = K - 1; p >= 0; --p) {
    const bool here = (d2 < bd[p]) || (d2 == bd[p] && j < bj[p]);
    bool prev = false;
    if (p > 0) prev = (d2 < bd[p - 1]) || (d2 == bd[p - 1] && j < bj[p - 1]);
    if (here) {
      bd[p] = prev ? bd[p - 1] : d2;
      bj[p] = prev ? bj[p - 1] : j;
    }
  }
}

// One thread per node, visited in cell order.  Cells are searched ring by
// ring (Chebyshev shells) until the k-th best squared distance is below a
// lower bound of every node in the unvisited cells.  The cells of a shell row
// that lie in one tile along x have consecutive ids, so their nodes form one
// contiguous range of the cell-sorted arrays: a row costs one pair of range
// loads per tile it crosses, and candidates are fetched four at a time (the
// best-k set under the order (distance, index) does not depend on the order
// in which candidates arrive).
template <int D, int K>
__global__ __launch_bounds__(128) void k_knn(KnnArgs a) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a.qlist) {
    if (t >= *a.nq) return;
    t = a.qlist[t];
  } else if (t >= a.N) {
    return;
  }
  const int64_t N = a.N;
  const int32_t i = a.cell_nodes[t];
  const int dm = find_domain(i, a.off, a.nd);
  const GridDesc g = a.grids[dm];
  const bool bnd = a.ks[t] != 0;               // a wall node draws from interior nodes only
  double xi[D];
#pragma unroll
  for (int q = 0; q < D; ++q) xi[q] = a.xs[q * N + t];
  int ci[3] = {0, 0, 0};
  cell_coords<D>(g, xi, ci);
  const int msk = (1 << g.tl) - 1;

  double bd[K];
  int32_t bj[K];
#pragma unroll
  for (int p = 0; p < K; ++p) { bd[p] = INFINITY; bj[p] = INT_MAX; }
  int filled = 0;
  bool dup = false;
  const double margin = 1e-6 * g.cs;

  // candidates s0 <= s < s1 of the cell-sorted arrays
  auto scan = [&](int64_t s0, int64_t s1) {
    for (int64_t s = s0; s < s1; s += 4) {
      double pq[4][D];
      int32_t jj[4];
      uint8_t kk[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t su = (s + u < s1) ? s + u : s;
        jj[u] = a.cell_nodes[su];
        kk[u] = a.ks[su];
#pragma unroll
        for (int q = 0; q < D; ++q) pq[u][q] = a.xs[q * N + su];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (s + u >= s1) break;
        const int32_t j = jj[u];
        if (bnd && j != i && kk[u] != 0) continue;
        double d2 = 0.0;
#pragma unroll
        for (int q = 0; q < D; ++q) {
          const double dq = pq[u][q] - xi[q];
          const double sq = dq * dq;
          d2 = (q == 0) ? sq : d2 + sq;
        }
        if (d2 == 0.0 && j != i) dup = true;
        if ((d2 < bd[K - 1]) || (d2 == bd[K - 1] && j < bj[K - 1])) {
          topk_insert<K>(bd, bj, d2, j);
          filled = min(filled + 1, K);
        }
      }
    }
  };
  // cells xa..xb of the row (c1, c2), split where the row leaves a tile.
  // Once k candidates are held, the row is cut to the cells that can reach
  // the current k-th distance: a lower bound of the distance across y (, z)
  // leaves a reach along x, widened by the margin (every skipped node lies
  // strictly beyond the k-th distance, so the best-k set is unchanged).
  auto visit_row = [&](int c1, int c2, int xa, int xb) {
    if (filled == K) {
      double dyz = 0.0;
      const int cc[3] = {0, c1, c2};
#pragma unroll
      for (int q = 1; q < D; ++q) {
        const double lo = g.origin[q] + (double)cc[q] * g.cs;
        const double e = fmax(0.0, fmax(lo - xi[q], xi[q] - (lo + g.cs)) - margin);
        dyz += e * e;
      }
      const double rem = bd[K - 1] * (1.0 + 1e-12) - dyz;
      if (rem < 0.0) return;
      const double reach = sqrt(rem) + margin;
      xa = max(xa, (int)fmax(floor((xi[0] - reach - g.origin[0]) / g.cs), -1.0));
      xb = min(xb, (int)fmin(floor((xi[0] + reach - g.origin[0]) / g.cs), (double)g.dims[0]));
    }
    int c[3] = {xa, c1, c2};
    while (c[0] <= xb) {
      const int xe = min(xb, c[0] | msk);
      const int64_t id = cell_id<D>(g, c);
      const int64_t s0 = a.cell_start[id], s1 = a.cell_start[id + (xe - c[0]) + 1];
      scan(s0, s1);
      c[0] = xe + 1;
    }
  };

  for (int r = 0;; ++r) {
    // visit the shell of Chebyshev radius r
    int lo[3], hi[3];
#pragma unroll
    for (int q = 0; q < D; ++q) {
      lo[q] = max(ci[q] - r, 0);
      hi[q] = min(ci[q] + r, g.dims[q] - 1);
    }
    const int zlo = (D == 3) ? lo[2] : 0, zhi = (D == 3) ? hi[2] : 0;
    for (int z = zlo; z <= zhi; ++z)
      for (int y = lo[1]; y <= hi[1]; ++y) {
        const bool full_row = (abs(y - ci[1]) == r) || (D == 3 && abs(z - ci[2]) == r);
        if (full_row) {
          visit_row(y, z, lo[0], hi[0]);
        } else {
          // rows strictly inside the shell contribute only their two end cells
          if (ci[0] - r >= 0) visit_row(y, z, ci[0] - r, ci[0] - r);
          if (r > 0 && ci[0] + r <= g.dims[0] - 1) visit_row(y, z, ci[0] + r, ci[0] + r);
        }
      }
    // lower bound of the distance to any node in an unvisited cell
    bool any = false;
    double b = INFINITY;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      if (ci[q] - r - 1 >= 0) {
        any = true;
        b = fmin(b, xi[q] - (g.origin[q] + (double)(ci[q] - r) * g.cs) - margin);
      }
      if (ci[q] + r + 1 <= g.dims[q] - 1) {
        any = true;
        b = fmin(b, (g.origin[q] + (double)(ci[q] + r + 1) * g.cs) - xi[q] - margin);
      }
    }
    if (!any) break;
    if (filled == K && b > 0.0 && bd[K - 1] < b * b * (1.0 - 1e-12)) break;
  }

  const int n_i = a.n_dom[dm];
  if (dup) latch(a.status, BE_DUPLICATE, i);
  if (filled < n_i) latch(a.status, BE_SMALL_DOMAIN, i);
#pragma unroll
  for (int p = 0; p < K; ++p) a.knn[(int64_t)p * N + i] = bj[p];
}

// The classifier, one thread per node in cell order.  An interior node of a
// hybrid set is regular when each of its 2d axis points x +- h_r e_a has
// exactly one node within kCrossTau h_r (max-norm); the count runs over
// every node of the cells that the tolerance box around the point touches
// (widened by the margin, so no matching node is missed).  Every node also
// looks for a coinciding node: one would lie in the cells around its own
// position.  Wall nodes, and every node of an all-scattered set, are
// scattered.
template <int D>
__global__ __launch_bounds__(128) void k_classify(KnnArgs a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.N) return;
  const int64_t N = a.N;
  const int32_t i = a.cell_nodes[t];
  const int dm = find_domain(i, a.off, a.nd);
  const GridDesc g = a.grids[dm];
  const bool bnd = a.ks[t] != 0;
  double xi[D];
#pragma unroll
  for (int q = 0; q < D; ++q) xi[q] = a.xs[q * N + t];
  const double margin = 1e-6 * g.cs;

  // every node of the cells meeting the box [p - w, p + w]
  auto each_in_box = [&](const double *p, double w, auto &&f) {
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    double pl[D], ph[D];
#pragma unroll
    for (int q = 0; q < D; ++q) { pl[q] = p[q] - w; ph[q] = p[q] + w; }
    cell_coords<D>(g, pl, lo);
    cell_coords<D>(g, ph, hi);
    int c[3] = {0, 0, 0};
    for (c[2] = (D == 3 ? lo[2] : 0); c[2] <= (D == 3 ? hi[2] : 0); ++c[2])
      for (c[1] = lo[1]; c[1] <= hi[1]; ++c[1])
        for (c[0] = lo[0]; c[0] <= hi[0]; ++c[0]) {
          const int64_t id = cell_id<D>(g, c);
          const int64_t s1 = a.cell_start[id + 1];
          for (int64_t s = a.cell_start[id]; s < s1; ++s) f(s);
        }
  };

  bool dup = false;
  each_in_box(xi, margin, [&](int64_t s) {
    const int32_t j = a.cell_nodes[s];
    double d2 = 0.0;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const double dq = a.xs[q * N + s] - xi[q];
      const double sq = dq * dq;
      d2 = (q == 0) ? sq : d2 + sq;
    }
    if (d2 == 0.0 && j != i) dup = true;
  });
  if (dup) latch(a.status, BE_DUPLICATE, i);

  uint8_t cl = 1;
  if (a.hybrid && !bnd) {
    const double h = a.h_dom[dm];
    const double tol = kCrossTau * h;
    bool reg = true;
#pragma unroll
    for (int ax = 0; ax < D; ++ax)
#pragma unroll
      for (int sg = 0; sg < 2; ++sg) {
        double pc[D];
#pragma unroll
        for (int q = 0; q < D; ++q) pc[q] = xi[q];
        pc[ax] = sg ? xi[ax] + h : xi[ax] - h;
        int cnt = 0;
        int32_t fnd = -1;
        each_in_box(pc, tol + margin, [&](int64_t s) {
          const int32_t j = a.cell_nodes[s];
          if (j == i) return;
          double tq[D];
#pragma unroll
          for (int q = 0; q < D; ++q) tq[q] = a.xs[q * N + s] - xi[q];
          const double e = sg ? tq[ax] - h : tq[ax] + h;
          bool ok = fabs(e) <= tol;
#pragma unroll
          for (int q = 0; q < D; ++q)
            if (q != ax && !(fabs(tq[q]) <= tol)) ok = false;
          if (ok) { ++cnt; fnd = j; }
        });
        reg = reg && (cnt == 1);
        a.cross[(int64_t)(2 * ax + sg) * N + i] = fnd;
      }
    cl = reg ? 0 : 1;
  }
  a.cls[i] = cl;
}

// cell-sorted positions of the scattered nodes, in cell order
__global__ void k_flag_scattered(const int32_t *nodes, const uint8_t *cls, int64_t N, int32_t *flag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  flag[t] = cls[nodes[t]] != 0 ? 1 : 0;
}

__global__ void k_compact(const int32_t *flag, const int64_t *pos, int64_t N, int32_t *out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  if (flag[t]) out[pos[t]] = (int32_t)t;
}

// ------------------------------------------------- buckets and ordering ---
// bucket index: regular 0; scattered 1+c; Dirichlet wall 1+nc+c; Neumann wall 1+2nc+c
__global__ void k_bucket_of(const uint8_t *cls, const uint8_t *kind, int64_t N, const int64_t *off, int nd,
                            const int32_t *combo, int nc, int32_t *bucket) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int dm = find_domain(i, off, nd);
  const int c = combo[dm];
  int b;
  if (kind[i] == 1) b = 1 + nc + c;
  else if (kind[i] == 2) b = 1 + 2 * nc + c;
  else b = cls[i] == 0 ? 0 : 1 + c;
  bucket[i] = b;
}

__global__ void k_flag(const int32_t *seq, const int32_t *bucket, int64_t N, int b, int32_t *flag) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  flag[t] = bucket[seq[t]] == b ? 1 : 0;
}

// bucket b's size (the flag total) into counts[b]; its nodes go after those
// of buckets 0..b-1
__global__ void k_bucket_total(const int64_t *pos, int64_t N, int b, int64_t *counts) {
  if (blockIdx.x == 0 && threadIdx.x == 0) counts[b] = pos[N];
}

__global__ void k_place(const int32_t *seq, const int32_t *flag, const int64_t *pos, int64_t N,
                        const int64_t *counts, int b, int32_t *perm) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  int64_t start = 0;
  for (int c = 0; c < b; ++c) start += counts[c];
  if (flag[t]) perm[start + pos[t]] = seq[t];
}

template <int D>
__global__ void k_gather_nodes(const int32_t *perm, int64_t N, const double *x, const uint8_t *kind,
                               const double *normal, int32_t *iperm, double *xi, uint8_t *ki, double *ni) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int32_t i = perm[t];
  iperm[i] = (int32_t)t;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    xi[a * N + t] = x[a * N + i];
    ni[a * N + t] = normal[a * N + i];
  }
  ki[t] = kind[i];
}

// stencil of each node of a bucket, in internal numbering, SoA [width][count]
__global__ void k_stencil_idx(const int32_t *perm, const int32_t *iperm, int64_t N, int64_t start, int64_t count,
                              int width, int regular, int D, const int32_t *knn, const int32_t *cross,
                              int32_t *idx) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int32_t i = perm[start + t];
  for (int j = 0; j < width; ++j) {
    int32_t src;
    if (regular) src = (j == 0) ? i : cross[(int64_t)(j - 1) * N + i];
    else src = knn[(int64_t)j * N + i];
    // an unfilled neighbour slot (domain too small, already latched) maps to the node itself
    idx[(int64_t)j * count + t] = (src >= 0 && src < N) ? iperm[src] : iperm[i];
  }
}

__global__ void k_init_status(DevStatus *st) {
  if (threadIdx.x == 0) {
    st->bits = 0;
    for (int k = 0; k < BE_COUNT; ++k) st->node[k] = ~0ull;
  }
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <int D, int K>
void launch_knn(const KnnArgs &a, hipStream_t s) {
  hipLaunchKernelGGL((k_knn<D, K>), dim3(nblk(a.N, 128)), dim3(128), 0, s, a);
}

template <int D>
bool dispatch_knn(int K, const KnnArgs &a, hipStream_t s) {
  switch (K) {
    case 8: launch_knn<D, 8>(a, s); return true;
    case 12: launch_knn<D, 12>(a, s); return true;
    case 20: launch_knn<D, 20>(a, s); return true;
    case 32: launch_knn<D, 32>(a, s); return true;
    case 40: launch_knn<D, 40>(a, s); return true;
    case 64: launch_knn<D, 64>(a, s); return true;
  }
  return false;
}

int knn_capacity(int k) {
  const int caps[] = {8, 12, 20, 32, 40, 64};
  for (int c : caps)
    if (k <= c) return c;
  return -1;
}

}  // namespace

// ====================================================================== //
hsm_status build_stencils_impl(const hsm_nodeset *ns, int32_t mode, hipStream_t s, hsm_stencils **out) {
  const int d = ns->d, nd = ns->n_domains;
  const int64_t N = ns->host_domain_offsets[nd];
  auto t_start = std::chrono::steady_clock::now();

  // ---- host-side tables
  std::vector<int32_t> n_dom(nd), m_dom(nd), combo(nd);
  std::vector<std::pair<int, int>> combos;  // (m, n)
  int kmax = 0;
  for (int k = 0; k < nd; ++k) {
    const int m = ns->host_m[k];
    const int Q = nmono(d, m);
    const int n = ns->host_n ? ns->host_n[k] : 2 * Q;
    n_dom[k] = n;
    m_dom[k] = m;
    auto key = std::make_pair(m, n);
    auto it = std::find(combos.begin(), combos.end(), key);
    if (it == combos.end()) { combos.push_back(key); combo[k] = (int)combos.size() - 1; }
    else combo[k] = (int)(it - combos.begin());
    kmax = std::max(kmax, n);
  }
  kmax = std::max(kmax, 2 * d + 1);
  const int nc = (int)combos.size();
  if (1 + 3 * nc > kMaxBuckets) {
    set_error(HSM_E_INVALID, "too many distinct (m, n) stencil kinds (at most 5)");
    return HSM_E_INVALID;
  }
  const int K = knn_capacity(kmax);
  if (K < 0) { set_error(HSM_E_INVALID, "stencil size too large"); return HSM_E_INVALID; }

  hsm_status rc;
  auto st = new hsm_stencils();
  std::unique_ptr<hsm_stencils> guard(st);
  st->d = d; st->mode = mode; st->n_domains = nd; st->N = N;
  st->solve_groups = ns->solve_groups;
  st->dom_off.assign(ns->host_domain_offsets, ns->host_domain_offsets + nd + 1);
  HSM_HIP(hipGetDevice(&st->device));

  // chunks per domain of the bounding-box pass: about 4096 nodes each
  int64_t max_cnt = 0;
  for (int k = 0; k < nd; ++k)
    max_cnt = std::max<int64_t>(max_cnt, ns->host_domain_offsets[k + 1] - ns->host_domain_offsets[k]);
  const int bbP = (int)std::min<int64_t>(256, std::max<int64_t>(1, (max_cnt + 4095) / 4096));
  // temporaries of the build: two blocks of the scratch pool (per-domain data
  // now, node and cell arrays once the grids are known), released in stream order
  const size_t b_off = sizeof(int64_t) * (nd + 1), b_h = sizeof(double) * nd, b_n = sizeof(int32_t) * nd,
               b_combo = sizeof(int32_t) * nd, b_bbox = sizeof(double) * nd * 6,
               b_bbpart = sizeof(double) * nd * bbP * 6, b_grid = sizeof(GridDesc) * nd, b_status = sizeof(DevStatus);
  Arena ar1;
  if ((rc = ar1.reserve(round256(b_off) + round256(b_h) + round256(b_n) + round256(b_combo) + round256(b_bbox) +
                            round256(b_bbpart) + round256(b_grid) + round256(b_status), s)))
    return rc;
  const Arena::View d_off = ar1.take(b_off), d_h = ar1.take(b_h), d_n = ar1.take(b_n), d_combo = ar1.take(b_combo),
                    d_bbox = ar1.take(b_bbox), d_bbpart = ar1.take(b_bbpart), d_grid = ar1.take(b_grid),
                    d_status = ar1.take(b_status);
  if (!d_status.p) { set_error(HSM_E_HIP, "scratch reservation too small"); return HSM_E_HIP; }
  HSM_HIP(hipMemcpyAsync(d_off.p, ns->host_domain_offsets, sizeof(int64_t) * (nd + 1), hipMemcpyHostToDevice, s));
  HSM_HIP(hipMemcpyAsync(d_h.p, ns->host_h_regular, sizeof(double) * nd, hipMemcpyHostToDevice, s));
  HSM_HIP(hipMemcpyAsync(d_n.p, n_dom.data(), sizeof(int32_t) * nd, hipMemcpyHostToDevice, s));
  HSM_HIP(hipMemcpyAsync(d_combo.p, combo.data(), sizeof(int32_t) * nd, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_init_status, dim3(1), dim3(64), 0, s, d_status.as<DevStatus>());

  hipEvent_t ev[4];
  for (auto &e : ev) HSM_HIP(hipEventCreate(&e));
  struct EvGuard { hipEvent_t *e; ~EvGuard() { for (int k = 0; k < 4; ++k) (void)hipEventDestroy(e[k]); } } evg{ev};
  HSM_HIP(hipEventRecord(ev[0], s));

  // ---- per-domain bounding boxes -> cell grids (about two nodes per cell)
  const unsigned bb_blocks = (unsigned)((int64_t)nd * bbP);
  if (d == 2) {
    hipLaunchKernelGGL(k_bbox_part<2>, dim3(bb_blocks), dim3(256), 0, s, ns->x, N, d_off.as<int64_t>(), bbP,
                       d_bbpart.as<double>());
    hipLaunchKernelGGL(k_bbox_fold<2>, dim3(nd), dim3(64), 0, s, d_bbpart.as<double>(), nd, bbP,
                       d_bbox.as<double>());
  } else {
    hipLaunchKernelGGL(k_bbox_part<3>, dim3(bb_blocks), dim3(256), 0, s, ns->x, N, d_off.as<int64_t>(), bbP,
                       d_bbpart.as<double>());
    hipLaunchKernelGGL(k_bbox_fold<3>, dim3(nd), dim3(64), 0, s, d_bbpart.as<double>(), nd, bbP,
                       d_bbox.as<double>());
  }
  HSM_HIP(hipGetLastError());
  std::vector<double> bbox(nd * 6);
  HSM_HIP(hipMemcpyAsync(bbox.data(), d_bbox.p, sizeof(double) * nd * 6, hipMemcpyDeviceToHost, s));
  HSM_HIP(hipStreamSynchronize(s));
  std::vector<GridDesc> grids(nd);
  int64_t ncells = 0;
  for (int k = 0; k < nd; ++k) {
    GridDesc &g = grids[k];
    g.tl = ns->tile_log2 > 0 ? ns->tile_log2 : (d == 2 ? 3 : 2);
    const int64_t cnt = ns->host_domain_offsets[k + 1] - ns->host_domain_offsets[k];
    double ext[3] = {0, 0, 0}, vol = 1.0;
    for (int a = 0; a < d; ++a) {
      if (!std::isfinite(bbox[(k * 2) * 3 + a]) || !std::isfinite(bbox[(k * 2 + 1) * 3 + a])) {
        set_error(HSM_E_INVALID, "non-finite node position in domain " + std::to_string(k));
        return HSM_E_INVALID;
      }
      ext[a] = bbox[(k * 2 + 1) * 3 + a] - bbox[(k * 2) * 3 + a];
      g.origin[a] = bbox[(k * 2) * 3 + a];
    }
    double emax = std::max(ext[0], std::max(ext[1], ext[2]));
    if (!(emax > 0)) emax = 1.0;
    for (int a = 0; a < d; ++a) vol *= std::max(ext[a], emax * 1e-3);
    double cs = std::pow(2.0 * vol / (double)std::max<int64_t>(cnt, 1), 1.0 / d);
    if (!(cs > 0)) cs = emax;
    int64_t cells;
    for (;;) {
      cells = 1;
      for (int a = 0; a < d; ++a) {
        g.dims[a] = (int32_t)std::floor(ext[a] / cs) + 1;
        const int tile = 1 << g.tl;
        g.ntiles[a] = (g.dims[a] + tile - 1) / tile;
        cells *= (int64_t)g.ntiles[a] * tile;
      }
      if (cells <= 8 * cnt + 4096 && g.dims[0] < (1 << 20)) break;
      cs *= 1.25;
    }
    for (int a = d; a < 3; ++a) { g.dims[a] = 1; g.ntiles[a] = 1; g.origin[a] = 0; }
    g.cs = cs;
    g.cell_off = ncells;
    ncells += cells;
  }
  HSM_HIP(hipMemcpyAsync(d_grid.p, grids.data(), sizeof(GridDesc) * nd, hipMemcpyHostToDevice, s));

  // ---- counting sort of nodes into cells
  const size_t b_cell = sizeof(int64_t) * N, b_count = sizeof(int32_t) * ncells,
               b_start = sizeof(int64_t) * (ncells + 1), b_fill = sizeof(int32_t) * ncells,
               b_cellnodes = sizeof(int32_t) * N, b_knn = sizeof(int32_t) * K * N,
               b_cross = sizeof(int32_t) * 2 * d * N, b_xs = sizeof(double) * d * N, b_ks = (size_t)N,
               b_bucket = sizeof(int32_t) * N, b_flag = sizeof(int32_t) * N, b_pos = sizeof(int64_t) * (N + 1),
               b_bcount = sizeof(int64_t) * kMaxBuckets,
               b_scan = sizeof(int64_t) * std::max(scan_i32_to_i64_ws(ncells), scan_i32_to_i64_ws(N));
  Arena ar2;
  if ((rc = ar2.reserve(round256(b_cell) + round256(b_count) + round256(b_start) + round256(b_fill) +
                            round256(b_cellnodes) + round256(b_knn) + round256(b_cross) + round256(b_xs) +
                            round256(b_ks) + round256(b_bucket) + round256(b_flag) + round256(b_pos) +
                            round256(b_bcount) + round256(b_scan), s)))
    return rc;
  const Arena::View d_cell = ar2.take(b_cell), d_count = ar2.take(b_count), d_start = ar2.take(b_start),
                    d_fill = ar2.take(b_fill), d_cellnodes = ar2.take(b_cellnodes), d_knn = ar2.take(b_knn),
                    d_cross = ar2.take(b_cross), d_xs = ar2.take(b_xs), d_ks = ar2.take(b_ks),
                    d_bucket = ar2.take(b_bucket), d_flag = ar2.take(b_flag), d_pos = ar2.take(b_pos),
                    d_bcount = ar2.take(b_bcount), d_scan = ar2.take(b_scan);
  if (!d_scan.p) { set_error(HSM_E_HIP, "scratch reservation too small"); return HSM_E_HIP; }
  HSM_HIP(hipMemsetAsync(d_count.p, 0, sizeof(int32_t) * ncells, s));
  HSM_HIP(hipMemsetAsync(d_fill.p, 0, sizeof(int32_t) * ncells, s));
  if (N > 0) {
    if (d == 2)
      hipLaunchKernelGGL(k_cell_of<2>, dim3(nblk(N, 256)), dim3(256), 0, s, ns->x, N, d_off.as<int64_t>(), nd,
                         d_grid.as<GridDesc>(), d_cell.as<int64_t>(), d_count.as<int32_t>(),
                         d_status.as<DevStatus>());
    else
      hipLaunchKernelGGL(k_cell_of<3>, dim3(nblk(N, 256)), dim3(256), 0, s, ns->x, N, d_off.as<int64_t>(), nd,
                         d_grid.as<GridDesc>(), d_cell.as<int64_t>(), d_count.as<int32_t>(),
                         d_status.as<DevStatus>());
    HSM_HIP(hipGetLastError());
  }
  if ((rc = scan_i32_to_i64(d_count.as<int32_t>(), d_start.as<int64_t>(), ncells, s, d_scan.as<int64_t>()))) return rc;
  if (N > 0) {
    hipLaunchKernelGGL(k_cell_scatter, dim3(nblk(N, 256)), dim3(256), 0, s, d_cell.as<int64_t>(), N,
                       d_start.as<int64_t>(), d_fill.as<int32_t>(), d_cellnodes.as<int32_t>());
    hipLaunchKernelGGL(k_cell_sort, dim3(nblk(ncells, 256)), dim3(256), 0, s, d_start.as<int64_t>(), ncells,
                       d_cellnodes.as<int32_t>());
    HSM_HIP(hipGetLastError());
  }

  // ---- k nearest neighbours and classes
  if ((rc = st->cls.alloc(N))) return rc;
  if (N > 0) {
    if (d == 2)
      hipLaunchKernelGGL(k_sort_pos<2>, dim3(nblk(N, 256)), dim3(256), 0, s, d_cellnodes.as<int32_t>(), N, ns->x,
                         ns->kind, d_xs.as<double>(), d_ks.as<uint8_t>());
    else
      hipLaunchKernelGGL(k_sort_pos<3>, dim3(nblk(N, 256)), dim3(256), 0, s, d_cellnodes.as<int32_t>(), N, ns->x,
                         ns->kind, d_xs.as<double>(), d_ks.as<uint8_t>());
    HSM_HIP(hipGetLastError());
  }
  KnnArgs ka;
  ka.x = ns->x; ka.kind = ns->kind; ka.N = N; ka.off = d_off.as<int64_t>(); ka.nd = nd;
  ka.grids = d_grid.as<GridDesc>(); ka.cell_start = d_start.as<int64_t>(); ka.cell_nodes = d_cellnodes.as<int32_t>();
  ka.xs = d_xs.as<double>(); ka.ks = d_ks.as<uint8_t>();
  ka.n_dom = d_n.as<int32_t>(); ka.h_dom = d_h.as<double>(); ka.hybrid = (mode == HSM_MODE_HYBRID);
  ka.knn = d_knn.as<int32_t>(); ka.cls = st->cls.as<uint8_t>(); ka.cross = d_cross.as<int32_t>();
  ka.status = d_status.as<DevStatus>();
  ka.qlist = nullptr;
  ka.nq = nullptr;
  // d_bucket holds the kNN query list until the buckets are formed

  if (N > 0) {
    // classes first; in a hybrid set only the scattered and wall nodes need neighbours
    if (d == 2) hipLaunchKernelGGL(k_classify<2>, dim3(nblk(N, 128)), dim3(128), 0, s, ka);
    else hipLaunchKernelGGL(k_classify<3>, dim3(nblk(N, 128)), dim3(128), 0, s, ka);
    HSM_HIP(hipGetLastError());
    if (mode == HSM_MODE_HYBRID) {
      hipLaunchKernelGGL(k_flag_scattered, dim3(nblk(N, 256)), dim3(256), 0, s, d_cellnodes.as<int32_t>(),
                         st->cls.as<uint8_t>(), N, d_flag.as<int32_t>());
      if ((rc = scan_i32_to_i64(d_flag.as<int32_t>(), d_pos.as<int64_t>(), N, s, d_scan.as<int64_t>()))) return rc;
      hipLaunchKernelGGL(k_compact, dim3(nblk(N, 256)), dim3(256), 0, s, d_flag.as<int32_t>(),
                         d_pos.as<int64_t>(), N, d_bucket.as<int32_t>());
      HSM_HIP(hipGetLastError());
      ka.qlist = d_bucket.as<int32_t>();
      ka.nq = d_pos.as<int64_t>() + N;
    }
    if (!(d == 2 ? dispatch_knn<2>(K, ka, s) : dispatch_knn<3>(K, ka, s))) {
      set_error(HSM_E_INVALID, "unsupported neighbour count");
      return HSM_E_INVALID;
    }
    HSM_HIP(hipGetLastError());
  }
  HSM_HIP(hipEventRecord(ev[1], s));

  // ---- width buckets and the internal order (bucket-major, cell order inside)
  const int NBall = 1 + 3 * nc;
  if ((rc = st->perm.alloc(sizeof(int32_t) * N)) || (rc = st->iperm.alloc(sizeof(int32_t) * N)) ||
      (rc = st->x.alloc(sizeof(double) * d * N)) || (rc = st->kind.alloc(N)) ||
      (rc = st->normal.alloc(sizeof(double) * d * N)))
    return rc;
  if (N > 0) {
    hipLaunchKernelGGL(k_bucket_of, dim3(nblk(N, 256)), dim3(256), 0, s, st->cls.as<uint8_t>(), ns->kind, N,
                       d_off.as<int64_t>(), nd, d_combo.as<int32_t>(), nc, d_bucket.as<int32_t>());
    HSM_HIP(hipGetLastError());
  }
  std::vector<int64_t> bcount(NBall, 0), bstart(NBall, 0);
  for (int b = 0; b < NBall; ++b) {
    if (N > 0) {
      hipLaunchKernelGGL(k_flag, dim3(nblk(N, 256)), dim3(256), 0, s, d_cellnodes.as<int32_t>(),
                         d_bucket.as<int32_t>(), N, b, d_flag.as<int32_t>());
      HSM_HIP(hipGetLastError());
    }
    if ((rc = scan_i32_to_i64(d_flag.as<int32_t>(), d_pos.as<int64_t>(), N, s, d_scan.as<int64_t>()))) return rc;
    hipLaunchKernelGGL(k_bucket_total, dim3(1), dim3(64), 0, s, d_pos.as<int64_t>(), N, b,
                       d_bcount.as<int64_t>());
    if (N > 0)
      hipLaunchKernelGGL(k_place, dim3(nblk(N, 256)), dim3(256), 0, s, d_cellnodes.as<int32_t>(),
                         d_flag.as<int32_t>(), d_pos.as<int64_t>(), N, d_bcount.as<int64_t>(), b,
                         st->perm.as<int32_t>());
    HSM_HIP(hipGetLastError());
  }
  HSM_HIP(hipMemcpyAsync(bcount.data(), d_bcount.p, sizeof(int64_t) * NBall, hipMemcpyDeviceToHost, s));
  HSM_HIP(hipStreamSynchronize(s));
  int64_t run = 0;
  for (int b = 0; b < NBall; ++b) {
    bstart[b] = run;
    run += bcount[b];
  }
  if (run != N) { set_error(HSM_E_HIP, "bucket partition lost nodes"); return HSM_E_HIP; }
  if (N > 0) {
    if (d == 2)
      hipLaunchKernelGGL(k_gather_nodes<2>, dim3(nblk(N, 256)), dim3(256), 0, s, st->perm.as<int32_t>(), N, ns->x,
                         ns->kind, ns->normal, st->iperm.as<int32_t>(), st->x.as<double>(), st->kind.as<uint8_t>(),
                         st->normal.as<double>());
    else
      hipLaunchKernelGGL(k_gather_nodes<3>, dim3(nblk(N, 256)), dim3(256), 0, s, st->perm.as<int32_t>(), N, ns->x,
                         ns->kind, ns->normal, st->iperm.as<int32_t>(), st->x.as<double>(), st->kind.as<uint8_t>(),
                         st->normal.as<double>());
    HSM_HIP(hipGetLastError());
  }

  // ---- per-bucket stencils
  for (int b = 0; b < NBall; ++b) {
    if (bcount[b] == 0) continue;
    Bucket B;
    B.start = bstart[b];
    B.count = bcount[b];
    if (b == 0) { B.type = B_REG; B.width = 2 * d + 1; B.m = 0; }
    else {
      const int c = (b - 1) % nc;
      B.type = 1 + (b - 1) / nc;
      B.m = combos[c].first;
      B.width = combos[c].second;
    }
    B.nops = d + 1 + ((B.type == B_DIR || B.type == B_NEU) ? 1 : 0);
    if ((rc = B.idx.alloc(sizeof(int32_t) * B.width * B.count)) ||
        (rc = B.w.alloc(sizeof(double) * B.nops * B.width * B.count)))
      return rc;
    hipLaunchKernelGGL(k_stencil_idx, dim3(nblk(B.count, 256)), dim3(256), 0, s, st->perm.as<int32_t>(),
                       st->iperm.as<int32_t>(), N, B.start, B.count, B.width, B.type == B_REG ? 1 : 0, d,
                       d_knn.as<int32_t>(), d_cross.as<int32_t>(), B.idx.as<int32_t>());
    HSM_HIP(hipGetLastError());
    st->nnz += (int64_t)B.width * B.count;
    if (B.type == B_REG) st->n_regular += B.count;
    else st->n_scattered += B.count;
    if (B.type == B_DIR || B.type == B_NEU) st->n_boundary += B.count;
    st->buckets.push_back(std::move(B));
  }
  // check neighbour-search errors before solving
  DevStatus hs;
  HSM_HIP(hipMemcpyAsync(&hs, d_status.p, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
  HSM_HIP(hipStreamSynchronize(s));
  // a domain with fewer nodes than its stencil size (every one of its nodes
  // offends; regular nodes take no neighbour search, so the host checks)
  for (int k = 0; k < nd; ++k)
    if (ns->host_domain_offsets[k + 1] - ns->host_domain_offsets[k] < n_dom[k]) {
      hs.bits |= 1u << BE_SMALL_DOMAIN;
      hs.node[BE_SMALL_DOMAIN] = std::min<unsigned long long>(hs.node[BE_SMALL_DOMAIN],
                                                              (unsigned long long)ns->host_domain_offsets[k]);
      break;
    }
  HSM_HIP(hipEventRecord(ev[2], s));
  if (!(hs.bits & ((1u << BE_DUPLICATE) | (1u << BE_SMALL_DOMAIN) | (1u << BE_AMBIGUOUS) | (1u << BE_NONFINITE)))) {
    // wall nodes whose degree-m system is singular are listed, not failed
    DBuf d_retry;
    if ((rc = d_retry.alloc(sizeof(int32_t) * (st->n_boundary + 1)))) return rc;
    int32_t *retry = d_retry.as<int32_t>();
    HSM_HIP(hipMemsetAsync(retry, 0, sizeof(int32_t), s));
    auto is_wall = [](const Bucket &B) { return B.type == B_DIR || B.type == B_NEU; };
    // each bucket's solves between events of their own (per-bucket solve rates)
    const size_t nbk = st->buckets.size() < 16 ? st->buckets.size() : 16;
    std::vector<hipEvent_t> bev(nbk + 1, nullptr);
    for (auto &e : bev) HSM_HIP(hipEventCreate(&e));
    for (size_t k = 0; k < st->buckets.size(); ++k) {
      const Bucket &B = st->buckets[k];
      if (k < nbk) HSM_HIP(hipEventRecord(bev[k], s));
      if ((rc = solve_bucket(st, B, st->x.as<double>(), st->normal.as<double>(), d_status.as<DevStatus>(), s,
                             is_wall(B) ? retry + 1 : nullptr, retry))) {
        for (auto &e : bev) (void)hipEventDestroy(e);
        return rc;
      }
    }
    HSM_HIP(hipEventRecord(bev[nbk], s));
    int32_t nretry = 0;
    HSM_HIP(hipMemcpyAsync(&nretry, retry, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HSM_HIP(hipMemcpyAsync(&hs, d_status.p, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    HSM_HIP(hipStreamSynchronize(s));
    for (size_t k = 0; k < nbk; ++k) {
      float ms_k = 0.0f;
      HSM_HIP(hipEventElapsedTime(&ms_k, bev[k], bev[k + 1]));
      st->bucket_solve_ms[k] = ms_k;
    }
    for (auto &e : bev) HSM_HIP(hipEventDestroy(e));
    if (nretry > 0 && !hs.bits) {
      // the fallback: those wall nodes take degree m-1 on the same stencil
      // (walls need first derivatives only); failures now latch
      for (const Bucket &B : st->buckets) {
        if (!is_wall(B)) continue;
        if ((rc = solve_bucket_list(st, B, st->x.as<double>(), st->normal.as<double>(), d_status.as<DevStatus>(), s,
                                    retry + 1, nretry)))
          return rc;
      }
      HSM_HIP(hipMemcpyAsync(&hs, d_status.p, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    }
    st->n_wall_fallback = nretry;
    st->fallback = std::move(d_retry);   // kept for the condition-number diagnostic
  }
  HSM_HIP(hipEventRecord(ev[3], s));
  HSM_HIP(hipStreamSynchronize(s));
  if (hs.bits) {
    struct { int bit; hsm_status code; const char *msg; } order[] = {
        {BE_NONFINITE, HSM_E_INVALID, "non-finite node position"},
        {BE_DUPLICATE, HSM_E_DUPLICATE_NODE, "two nodes of a domain coincide"},
        {BE_SMALL_DOMAIN, HSM_E_INVALID, "a domain has fewer nodes than the stencil size"},
        {BE_AMBIGUOUS, HSM_E_AMBIGUOUS, "too many nodes within h_r of a node to classify it"},
        {BE_SINGULAR, HSM_E_SINGULAR, "singular local system"}};
    for (auto &o : order)
      if (hs.bits & (1u << o.bit)) {
        set_error(o.code, o.msg, (int64_t)hs.node[o.bit]);
        return o.code;
      }
  }
  float ms[3] = {0, 0, 0};
  HSM_HIP(hipEventElapsedTime(&ms[0], ev[0], ev[1]));
  HSM_HIP(hipEventElapsedTime(&ms[1], ev[1], ev[2]));
  HSM_HIP(hipEventElapsedTime(&ms[2], ev[2], ev[3]));
  st->build_ms[0] = ms[0];
  st->build_ms[1] = ms[1];
  st->build_ms[2] = ms[2];
  st->build_ms[3] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  (void)m_dom;
  *out = guard.release();
  return HSM_OK;
}

}  // namespace hsm
