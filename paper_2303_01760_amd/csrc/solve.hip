// Batched local solves M w = l for the stencil weights (Section 2.1).
//
// RBF-FD (scattered nodes): M = [[A, P], [P^T, 0]] with A_jl = |y_j - y_l|^3
// (PHS of order 3) and P_ja = y_j^alpha for all monomials of degree <= m
// (Section 2 and the choice k = 3, m = 2 of Section 4), in coordinates y
// centred at the node and scaled by the stencil radius.  Right-hand sides
// are the operator applied to each basis function at the centre:
//   d/dx_a : -3 |y_j| y_j,a  and 1 on the monomial x_a
//   Lap    : 3 (d+1) |y_j|   and 2 on each monomial x_a^2.
// One wave64 per system, one matrix row per lane, so S = n + Q <= 64.
//
// MON (regular nodes): the 2d+1 monomials {1, x_a, x_a^2} on the 2d+1 node
// axis cross (Section 2 and its footnote); one thread per node.
//
// Both use LU with partial pivoting in one fixed form: in column k the pivot
// is the not-yet-used row of largest magnitude, the lowest row on ties; rows
// are not moved; back substitution runs columns from last to first.  The
// file is compiled with -ffp-contract=off, so every product and sum is
// rounded as written and the pivoting decisions are reproducible.
#include <hip/hip_runtime.h>

#include <cstring>

#include "hsm_internal.h"

namespace hsm {
namespace {

constexpr double kPivotRel = 1e-14;  // pivot below kPivotRel * max|M| => singular

template <int D, int M>
struct Monos {
  static constexpr int count() {
    int q = 1;
    for (int k = 1; k <= D; ++k) q = q * (M + k) / k;
    return q;
  }
  static constexpr int Q = count();
  int e[Q][3];
  // graded; inside a degree, descending power of x, then of y
  constexpr Monos() : e{} {
    int q = 0;
    for (int deg = 0; deg <= M; ++deg) {
      if (D == 2) {
        for (int ax = deg; ax >= 0; --ax) { e[q][0] = ax; e[q][1] = deg - ax; e[q][2] = 0; ++q; }
      } else {
        for (int ax = deg; ax >= 0; --ax)
          for (int ay = deg - ax; ay >= 0; --ay) { e[q][0] = ax; e[q][1] = ay; e[q][2] = deg - ax - ay; ++q; }
      }
    }
  }
};

__device__ __forceinline__ double rdlane(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Lanes per group when a wave holds G systems: 64, 32 or 21 (lane 63 idles
// with G = 3, counted in the last group).
template <int G>
constexpr int group_lanes() { return G == 3 ? 21 : 64 / G; }

// Maximum over the lanes of each group.  G = 1, 2: butterfly over aligned
// lane blocks.  G = 3: cyclic doubling inside the group of 21 (each lane
// ends with the maximum over 32 cyclically consecutive lanes, which covers
// the group); `lane` counts in the group, `base` is its first lane.
template <int G>
__device__ __forceinline__ double group_max(double v, int lane = 0, int base = 0) {
  if constexpr (G == 3) {
    constexpr int GL = group_lanes<3>();
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) {
      int l = lane + o;
      l = (l >= 2 * GL) ? l - 2 * GL : ((l >= GL) ? l - GL : l);
      v = fmax(v, __shfl(v, base + l, 64));
    }
    return v;
  } else {
#pragma unroll
    for (int o = 32 / G; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
  }
}

struct SolveArgs {
  const double *x;        // [D][N] internal order
  const double *normal;   // [D][N] internal order
  int64_t N;
  const int32_t *idx;     // [W][count]
  int64_t count, start;
  double *w;              // [nops][W][count]
  int wall;               // also write normal-derivative weights
  const int32_t *perm;
  DevStatus *status;
  int32_t *retry;         // non-NULL: list singular nodes here (internal numbering) instead of failing
  int32_t *nretry;        // length of that list
  const int32_t *list;    // non-NULL: block b solves internal node list[b] (if it is in this bucket)
  double *kappa;          // condition-number kernels: [N] caller order
};

// Row `lane` of the RBF-FD system of node t (Section 2.1): M = [[A, P],
// [P^T, 0]] and the right-hand sides of d/dx_a and the Laplacian, in local
// coordinates y_j = (x_j - x_c) / s; returns the centre c and the scale s.
// M is symmetric, so the row is also column `lane`.  The wave holds G
// systems, group `grp` of 64 / G lanes this one (lane counted in the group).
template <int D, int M, int NS, int G = 1>
__device__ __forceinline__ void rbffd_rows(const SolveArgs &a, int64_t t, int lane,
                                           double (&Rw)[NS + Monos<D, M>::Q], double (&B)[D + 1], int32_t &c,
                                           double &s, int grp = 0) {
  constexpr int Q = Monos<D, M>::Q;
  constexpr int S = NS + Q;
  constexpr int R = D + 1;
  const int64_t cnt = a.count, N = a.N;
  constexpr Monos<D, M> mono{};
  __shared__ double sy_[G][NS][D];
  __shared__ double smono_[G][NS][Q];
  double (&sy)[NS][D] = sy_[grp];
  double (&smono)[NS][Q] = smono_[grp];

  // local coordinates y_j = (x_j - x_c) / s, s = max_j |x_j - x_c|
  c = a.idx[t];
  double dxv[D], r = 0.0;
#pragma unroll
  for (int q = 0; q < D; ++q) dxv[q] = 0.0;
  if (lane < NS) {
    const int32_t nj = a.idx[(int64_t)lane * cnt + t];
    double sq = 0.0;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      dxv[q] = a.x[q * N + nj] - a.x[q * N + c];
      const double v = dxv[q] * dxv[q];
      sq = (q == 0) ? v : sq + v;
    }
    r = sqrt(sq);
  }
  s = group_max<G>(r, lane, grp * group_lanes<G>());
  double y[D];
#pragma unroll
  for (int q = 0; q < D; ++q) y[q] = dxv[q] / s;
  if (lane < NS) {
#pragma unroll
    for (int q = 0; q < D; ++q) sy[lane][q] = y[q];
#pragma unroll
    for (int al = 0; al < Q; ++al) {
      double p = 1.0;
#pragma unroll
      for (int q = 0; q < D; ++q)
#pragma unroll
        for (int e = 0; e < mono.e[al][q]; ++e) p = p * y[q];
      smono[lane][al] = p;
    }
  }
  __syncthreads();

  // this lane's row of M and of the right-hand sides
#pragma unroll
  for (int k = 0; k < S; ++k) Rw[k] = 0.0;
#pragma unroll
  for (int q = 0; q < R; ++q) B[q] = 0.0;
  if (lane < NS) {
#pragma unroll
    for (int l = 0; l < NS; ++l) {
      double sq = 0.0;
#pragma unroll
      for (int q = 0; q < D; ++q) {
        const double dv = y[q] - sy[l][q];
        const double v = dv * dv;
        sq = (q == 0) ? v : sq + v;
      }
      const double rr = sqrt(sq);
      Rw[l] = rr * rr * rr;
    }
#pragma unroll
    for (int al = 0; al < Q; ++al) Rw[NS + al] = smono[lane][al];
    double sq = 0.0;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const double v = y[q] * y[q];
      sq = (q == 0) ? v : sq + v;
    }
    const double rl = sqrt(sq);
#pragma unroll
    for (int q = 0; q < D; ++q) B[q] = -((3.0 * rl) * y[q]);
    B[D] = (3.0 * (D + 1)) * rl;
  } else if (lane < S) {
#pragma unroll
    for (int al = 0; al < Q; ++al) {
      if (lane - NS != al) continue;
#pragma unroll
      for (int l = 0; l < NS; ++l) Rw[l] = smono[l][al];
      const int deg = mono.e[al][0] + mono.e[al][1] + mono.e[al][2];
#pragma unroll
      for (int q = 0; q < D; ++q) {
        if (deg == 1 && mono.e[al][q] == 1) B[q] = 1.0;
        if (deg == 2 && mono.e[al][q] == 2) B[D] = 2.0;
      }
    }
  }

}

// G systems per wave (G = 3 when S <= 21, 2 when S <= 32): lanes
// GL g .. GL g + GL - 1 hold system G b + g of block b (GL = 21, 32).  Every
// system takes exactly the operations of the one-system form; the pivot row
// reaches its group by lane permutes.
template <int D, int M, int NS, int G>
__global__ __launch_bounds__(64) void k_rbffd(SolveArgs a) {
  constexpr int Q = Monos<D, M>::Q;
  constexpr int S = NS + Q;
  constexpr int R = D + 1;
  constexpr int GL = group_lanes<G>();
  static_assert(S <= GL, "one system row per lane");
  const int grp = (G == 1) ? 0 : min((int)threadIdx.x / GL, G - 1);
  const int lane = (int)threadIdx.x - grp * GL;      // lane 63 of G = 3: 21, past every row
  const int base = grp * GL;
  int64_t t;
  bool live = true;
  if (a.list) {
    // list mode: one system per block
    const int64_t g = a.list[blockIdx.x];
    if (G != 1 || g < a.start || g >= a.start + a.count) return;
    t = g - a.start;
  } else {
    t = (int64_t)blockIdx.x * G + grp;
    live = t < a.count;
    if (!live) t = a.count - 1;       // a group past the end repeats the last system and stores nothing
  }
  const int64_t cnt = a.count, N = a.N;
  double Rw[S], B[R];
  int32_t c;
  double s;
  rbffd_rows<D, M, NS, G>(a, t, lane, Rw, B, c, s, grp);

  // elimination.  One system per wave (G = 1): the pivot row is read lane by
  // lane into scalar registers (v_readlane) and used as a scalar operand.
  // Several systems per wave: the pivot row of each step reaches its group
  // through LDS: the pivot lane writes columns k..S-1 and the right-hand
  // sides to its group's row, and every lane reads them back as it
  // eliminates (a broadcast read: the group's lanes read the same address),
  // instead of two lane permutes per entry.  The arithmetic is the same
  // either way.
  constexpr int PW = (S + R + 1) & ~1;         // row length, even: 16-byte aligned rows
  __shared__ __align__(16) double prow_[G == 1 ? 1 : G][G == 1 ? 2 : PW];
  double *prow = prow_[G == 1 ? 0 : grp];
  double amax = 0.0;
#pragma unroll
  for (int k = 0; k < S; ++k) amax = fmax(amax, fabs(Rw[k]));
  amax = group_max<G>(amax, lane, base);
  const double thr = kPivotRel * amax;
  bool used = lane >= S;
  int pstep = used ? S : -1;
  int piv[S];
  bool singular = false;
#pragma unroll
  for (int k = 0; k < S; ++k) {
    const double cand = used ? -1.0 : fabs(Rw[k]);
    const double best = group_max<G>(cand, lane, base);
    if (!(best > thr)) singular = true;
    if (G == 1 && singular) break;
    const unsigned long long mask = __ballot(!used && cand == best);
    const unsigned long long gm = (G == 1) ? mask : ((mask >> base) & ((1ull << GL) - 1ull));
    const int p = gm ? __ffsll((long long)gm) - 1 : 0;
    piv[k] = p;
    if constexpr (G == 1) {
      (void)prow;
      double pr[S], pb[R];
      const double pk = rdlane(Rw[k], p);
#pragma unroll
      for (int j = k + 1; j < S; ++j) pr[j] = rdlane(Rw[j], p);
#pragma unroll
      for (int q = 0; q < R; ++q) pb[q] = rdlane(B[q], p);
      if (lane == p) {
        used = true;
        pstep = k;
      } else if (!used) {
        const double l = Rw[k] / pk;
#pragma unroll
        for (int j = k + 1; j < S; ++j) Rw[j] = Rw[j] - l * pr[j];
#pragma unroll
        for (int q = 0; q < R; ++q) B[q] = B[q] - l * pb[q];
      }
    } else {
      if (lane == p) {
#pragma unroll
        for (int j = k; j < S; ++j) prow[j] = Rw[j];
#pragma unroll
        for (int q = 0; q < R; ++q) prow[S + q] = B[q];
      }
      __syncthreads();                        // one wave per block: orders the LDS write before the reads
      if (!singular) {
        if (lane == p) {
          used = true;
          pstep = k;
        } else if (!used) {
          const double l = Rw[k] / prow[k];
#pragma unroll
          for (int j = k + 1; j < S; ++j) Rw[j] = Rw[j] - l * prow[j];
#pragma unroll
          for (int q = 0; q < R; ++q) B[q] = B[q] - l * prow[S + q];
        }
      }
      __syncthreads();                        // every read of this pivot row before the next is written
    }
  }
  if (G == 1 && singular) {
    if (lane == 0) {
      if (a.retry) a.retry[atomicAdd(a.nretry, 1)] = (int32_t)(a.start + t);
      else latch(a.status, BE_SINGULAR, a.perm[a.start + t]);
    }
    return;
  }
  // back substitution, last column first
  double myw[R];
#pragma unroll
  for (int q = 0; q < R; ++q) myw[q] = 0.0;
#pragma unroll
  for (int k = S - 1; k >= 0; --k) {
    const int p = piv[k];
    double den, xk[R];
    if (G == 1) {
      den = rdlane(Rw[k], p);
#pragma unroll
      for (int q = 0; q < R; ++q) xk[q] = rdlane(B[q], p) / den;
    } else {
      const int src = base + p;
      den = __shfl(Rw[k], src, 64);
#pragma unroll
      for (int q = 0; q < R; ++q) xk[q] = __shfl(B[q], src, 64) / den;
    }
    if (k < NS && lane == k) {
#pragma unroll
      for (int q = 0; q < R; ++q) myw[q] = xk[q];
    }
    if (pstep < k) {
#pragma unroll
      for (int q = 0; q < R; ++q) B[q] = B[q] - Rw[k] * xk[q];
    }
  }
  if (!live) return;
  if (singular) {
    if (lane == 0) {
      if (a.retry) a.retry[atomicAdd(a.nretry, 1)] = (int32_t)(a.start + t);
      else latch(a.status, BE_SINGULAR, a.perm[a.start + t]);
    }
    return;
  }
  if (lane < NS) {
    const int64_t WC = (int64_t)NS * cnt;
    const double s2 = s * s;
    double wv[R];
#pragma unroll
    for (int q = 0; q < D; ++q) wv[q] = myw[q] / s;
    wv[D] = myw[D] / s2;
#pragma unroll
    for (int q = 0; q < R; ++q) a.w[q * WC + (int64_t)lane * cnt + t] = wv[q];
    if (a.wall) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < D; ++q) {
        const double v = a.normal[q * N + c] * wv[q];
        acc = (q == 0) ? v : acc + v;
      }
      a.w[R * WC + (int64_t)lane * cnt + t] = acc;
    }
  }
}

// MON on the axis cross [c, -x, +x, -y, +y (, -z, +z)], one thread per node.
template <int D>
__global__ __launch_bounds__(128) void k_mon(SolveArgs a) {
  constexpr int S = 2 * D + 1, R = D + 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.count) return;
  const int64_t cnt = a.count, N = a.N;
  const int32_t c = a.idx[t];
  double y[S][D], s = 0.0;
#pragma unroll
  for (int j = 0; j < S; ++j) {
    const int32_t nj = a.idx[(int64_t)j * cnt + t];
    double sq = 0.0;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      y[j][q] = a.x[q * N + nj] - a.x[q * N + c];
      const double v = y[j][q] * y[j][q];
      sq = (q == 0) ? v : sq + v;
    }
    const double r = sqrt(sq);
    if (r > s) s = r;
  }
#pragma unroll
  for (int j = 0; j < S; ++j)
#pragma unroll
    for (int q = 0; q < D; ++q) y[j][q] = y[j][q] / s;
  // rows: basis functions 1, x_a (a < D), x_a^2; columns: stencil nodes
  double A[S][S], B[S][R];
#pragma unroll
  for (int j = 0; j < S; ++j) {
    A[0][j] = 1.0;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      A[1 + q][j] = y[j][q];
      A[1 + D + q][j] = y[j][q] * y[j][q];
    }
  }
#pragma unroll
  for (int r = 0; r < S; ++r)
#pragma unroll
    for (int q = 0; q < R; ++q) B[r][q] = 0.0;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    B[1 + q][q] = 1.0;
    B[1 + D + q][D] = 2.0;
  }
  double amax = 0.0;
#pragma unroll
  for (int r = 0; r < S; ++r)
#pragma unroll
    for (int j = 0; j < S; ++j) amax = fmax(amax, fabs(A[r][j]));
  const double thr = kPivotRel * amax;
  unsigned used = 0;
  int pivrow[S], stepof[S];
#pragma unroll
  for (int r = 0; r < S; ++r) stepof[r] = S;
#pragma unroll
  for (int k = 0; k < S; ++k) {
    double best = -1.0;
    int p = 0;
#pragma unroll
    for (int r = 0; r < S; ++r)
      if (!((used >> r) & 1u) && fabs(A[r][k]) > best) { best = fabs(A[r][k]); p = r; }
    if (!(best > thr)) {
      latch(a.status, BE_SINGULAR, a.perm[a.start + t]);
      return;
    }
    used |= 1u << p;
    pivrow[k] = p;
    double pv[S], pb[R];
#pragma unroll
    for (int j = 0; j < S; ++j) pv[j] = A[0][j];
#pragma unroll
    for (int q = 0; q < R; ++q) pb[q] = B[0][q];
#pragma unroll
    for (int r = 1; r < S; ++r)
      if (p == r) {
#pragma unroll
        for (int j = 0; j < S; ++j) pv[j] = A[r][j];
#pragma unroll
        for (int q = 0; q < R; ++q) pb[q] = B[r][q];
      }
#pragma unroll
    for (int r = 0; r < S; ++r) {
      if (r == p) stepof[r] = k;
      if ((used >> r) & 1u) continue;
      const double l = A[r][k] / pv[k];
#pragma unroll
      for (int j = k + 1; j < S; ++j) A[r][j] = A[r][j] - l * pv[j];
#pragma unroll
      for (int q = 0; q < R; ++q) B[r][q] = B[r][q] - l * pb[q];
    }
  }
  double xs[S][R];
#pragma unroll
  for (int k = S - 1; k >= 0; --k) {
    const int p = pivrow[k];
    double den = A[0][k], num[R];
#pragma unroll
    for (int q = 0; q < R; ++q) num[q] = B[0][q];
#pragma unroll
    for (int r = 1; r < S; ++r)
      if (p == r) {
        den = A[r][k];
#pragma unroll
        for (int q = 0; q < R; ++q) num[q] = B[r][q];
      }
#pragma unroll
    for (int q = 0; q < R; ++q) xs[k][q] = num[q] / den;
#pragma unroll
    for (int r = 0; r < S; ++r)
      if (stepof[r] < k)
#pragma unroll
        for (int q = 0; q < R; ++q) B[r][q] = B[r][q] - A[r][k] * xs[k][q];
  }
  const int64_t WC = (int64_t)S * cnt;
  const double s2 = s * s;
#pragma unroll
  for (int j = 0; j < S; ++j) {
#pragma unroll
    for (int q = 0; q < D; ++q) a.w[q * WC + (int64_t)j * cnt + t] = xs[j][q] / s;
    a.w[D * WC + (int64_t)j * cnt + t] = xs[j][D] / s2;
  }
}

// groups: systems per wave requested (0: the most that fit), capped at what
// fits (3 when S <= 21, 2 when S <= 32); the list mode solves one per wave.
template <int D, int M, int NS>
void launch_rbffd(const SolveArgs &a, hipStream_t s, int64_t nlist = -1, int groups = 0) {
  constexpr int S = NS + Monos<D, M>::Q;
  constexpr int Gmax = S <= 21 ? 3 : S <= 32 ? 2 : 1;
  const int G = nlist >= 0 ? 1 : (groups <= 0 || groups > Gmax) ? Gmax : groups;
  if constexpr (Gmax >= 3) {
    if (G == 3) {
      hipLaunchKernelGGL((k_rbffd<D, M, NS, 3>), dim3((unsigned)((a.count + 2) / 3)), dim3(64), 0, s, a);
      return;
    }
  }
  if constexpr (Gmax >= 2) {
    if (G == 2) {
      hipLaunchKernelGGL((k_rbffd<D, M, NS, 2>), dim3((unsigned)((a.count + 1) / 2)), dim3(64), 0, s, a);
      return;
    }
  }
  const int64_t g = nlist >= 0 ? nlist : a.count;
  hipLaunchKernelGGL((k_rbffd<D, M, NS, 1>), dim3((unsigned)g), dim3(64), 0, s, a);
}

// ------------------------------------------------- condition numbers --
// kappa(M) = |M|_2 |M^-1|_2 = sigma_max / sigma_min of a node's local system
// (Section 2.1, Fig. 2).  The singular values come from one-sided Jacobi
// (Hestenes 1958): plane rotations of column pairs until every pair is
// orthogonal to working precision; the column norms are then the singular
// values.  One wave per system, one column per lane; the S/2 disjoint pairs
// of a round-robin round rotate at once, each lane fetching its partner's
// column.  Both lanes of a pair form the same sums in the same order (lower
// column first), so they take identical rotations.

constexpr double kJacobiTol = 1e-15;   // rotate while |u.v| > tol |u| |v|
constexpr int kJacobiSweeps = 40;

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// The singular value of this lane's column (lanes >= S hold zero columns).
template <int S>
__device__ __forceinline__ double jacobi_sv(double (&col)[S], int lane) {
  constexpr int P = (S + 1) & ~1;      // players of the round-robin (even)
  static_assert(P <= 64, "one column per lane");
  for (int sweep = 0; sweep < kJacobiSweeps; ++sweep) {
    bool rotated = false;
    for (int r = 0; r < P - 1; ++r) {
      int partner;
      if (lane >= P) partner = lane;
      else if (lane == P - 1) partner = r;
      else if (lane == r) partner = P - 1;
      else partner = (2 * r - lane + 2 * (P - 1)) % (P - 1);
      double oth[S];
#pragma unroll
      for (int i = 0; i < S; ++i) oth[i] = __shfl(col[i], partner, 64);
      const bool lo = lane < partner;
      double a2 = 0.0, b2 = 0.0, g = 0.0;   // |u|^2, |v|^2, u.v with u the lower column
#pragma unroll
      for (int i = 0; i < S; ++i) {
        const double u = lo ? col[i] : oth[i], v = lo ? oth[i] : col[i];
        a2 = fma(u, u, a2);
        b2 = fma(v, v, b2);
        g = fma(u, v, g);
      }
      if (partner != lane && fabs(g) > kJacobiTol * sqrt(a2 * b2)) {
        const double zeta = (b2 - a2) / (2.0 * g);
        const double tn = copysign(1.0, zeta) / (fabs(zeta) + sqrt(fma(zeta, zeta, 1.0)));
        const double cs = 1.0 / sqrt(fma(tn, tn, 1.0)), sn = cs * tn;
#pragma unroll
        for (int i = 0; i < S; ++i) {
          const double u = lo ? col[i] : oth[i], v = lo ? oth[i] : col[i];
          col[i] = lo ? cs * u - sn * v : sn * u + cs * v;
        }
        rotated = true;
      }
    }
    if (!__any(rotated)) break;
  }
  double n2 = 0.0;
#pragma unroll
  for (int i = 0; i < S; ++i) n2 = fma(col[i], col[i], n2);
  return sqrt(n2);
}

template <int S>
__device__ __forceinline__ void store_kappa(const SolveArgs &a, int64_t t, int lane, double sv) {
  const double smax = wave_max(lane < S ? sv : 0.0);
  const double smin = wave_min(lane < S ? sv : INFINITY);
  if (lane == 0) a.kappa[a.perm[a.start + t]] = smin > 0.0 ? smax / smin : INFINITY;
}

// RBF-FD system of a scattered node (M is symmetric: row = column).
template <int D, int M, int NS>
__global__ __launch_bounds__(64) void k_cond_rbffd(SolveArgs a) {
  constexpr int S = NS + Monos<D, M>::Q;
  static_assert(S <= 63, "one column per lane, plus a zero column when S is odd");
  const int lane = threadIdx.x;
  int64_t t = blockIdx.x;
  if (a.list) {
    const int64_t g = a.list[blockIdx.x];
    if (g < a.start || g >= a.start + a.count) return;
    t = g - a.start;
  }
  double Rw[S], B[D + 1];
  int32_t c;
  double s;
  rbffd_rows<D, M, NS>(a, t, lane, Rw, B, c, s);
  store_kappa<S>(a, t, lane, jacobi_sv<S>(Rw, lane));
}

// MON system of a regular node: column j holds the basis {1, y_a, y_a^2} at
// cross node j, in the coordinates k_mon uses.
template <int D>
__global__ __launch_bounds__(64) void k_cond_mon(SolveArgs a) {
  constexpr int S = 2 * D + 1;
  const int lane = threadIdx.x;
  const int64_t t = blockIdx.x, cnt = a.count, N = a.N;
  const int32_t c = a.idx[t];
  double dx[D], r = 0.0;
#pragma unroll
  for (int q = 0; q < D; ++q) dx[q] = 0.0;
  if (lane < S) {
    const int32_t nj = a.idx[(int64_t)lane * cnt + t];
    double sq = 0.0;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      dx[q] = a.x[q * N + nj] - a.x[q * N + c];
      const double v = dx[q] * dx[q];
      sq = (q == 0) ? v : sq + v;
    }
    r = sqrt(sq);
  }
  const double s = wave_max(r);
  double col[S];
#pragma unroll
  for (int i = 0; i < S; ++i) col[i] = 0.0;
  if (lane < S) {
    col[0] = 1.0;
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const double y = dx[q] / s;
      col[1 + q] = y;
      col[1 + D + q] = y * y;
    }
  }
  store_kappa<S>(a, t, lane, jacobi_sv<S>(col, lane));
}

template <int D, int M, int NS>
void launch_cond(const SolveArgs &a, hipStream_t s, int64_t nlist = -1) {
  const int64_t g = nlist >= 0 ? nlist : a.count;
  hipLaunchKernelGGL((k_cond_rbffd<D, M, NS>), dim3((unsigned)g), dim3(64), 0, s, a);
}

}  // namespace

// (d, m, n) combinations with a compiled local-solve kernel
bool rbffd_supported(int d, int m, int n) {
  if (d == 2) return (m == 1 && n == 6) || (m == 2 && n == 12) || (m == 3 && n == 20) || (m == 4 && n == 30);
  if (d == 3) return (m == 1 && n == 8) || (m == 2 && n == 20) || (m == 2 && n == 30) || (m == 3 && n == 40);
  return false;
}

hsm_status solve_bucket(const hsm_stencils *st, const Bucket &b, const double *x_int, const double *normal_int,
                        DevStatus *status, hipStream_t s, int32_t *retry, int32_t *nretry) {
  if (b.count == 0) return HSM_OK;
  SolveArgs a;
  a.x = x_int; a.normal = normal_int; a.N = st->N; a.idx = b.idx.as<int32_t>(); a.count = b.count;
  a.start = b.start; a.w = b.w.as<double>(); a.wall = (b.type == B_DIR || b.type == B_NEU);
  a.perm = st->perm.as<int32_t>(); a.status = status;
  a.retry = retry; a.nretry = nretry; a.list = nullptr;
  const int d = st->d;
  if (b.type == B_REG) {
    const unsigned g = (unsigned)((b.count + 127) / 128);
    if (d == 2) hipLaunchKernelGGL(k_mon<2>, dim3(g), dim3(128), 0, s, a);
    else hipLaunchKernelGGL(k_mon<3>, dim3(g), dim3(128), 0, s, a);
  } else {
    const int m = b.m, n = b.width;
    if (d == 2 && m == 1 && n == 6) launch_rbffd<2, 1, 6>(a, s, -1, st->solve_groups);
    else if (d == 2 && m == 2 && n == 12) launch_rbffd<2, 2, 12>(a, s, -1, st->solve_groups);
    else if (d == 2 && m == 3 && n == 20) launch_rbffd<2, 3, 20>(a, s, -1, st->solve_groups);
    else if (d == 2 && m == 4 && n == 30) launch_rbffd<2, 4, 30>(a, s, -1, st->solve_groups);
    else if (d == 3 && m == 1 && n == 8) launch_rbffd<3, 1, 8>(a, s, -1, st->solve_groups);
    else if (d == 3 && m == 2 && n == 20) launch_rbffd<3, 2, 20>(a, s, -1, st->solve_groups);
    else if (d == 3 && m == 2 && n == 30) launch_rbffd<3, 2, 30>(a, s, -1, st->solve_groups);
    else if (d == 3 && m == 3 && n == 40) launch_rbffd<3, 3, 40>(a, s, -1, st->solve_groups);
    else {
      set_error(HSM_E_INVALID, "no local-solve kernel for this (d, m, n)");
      return HSM_E_INVALID;
    }
  }
  HSM_HIP(hipGetLastError());
  return HSM_OK;
}

// The wall fallback: the listed nodes of a wall bucket (internal numbering;
// nodes of other buckets are skipped) solved with monomials of degree m-1 on
// their stencil.  Supported where m >= 2.
hsm_status solve_bucket_list(const hsm_stencils *st, const Bucket &b, const double *x_int, const double *normal_int,
                             DevStatus *status, hipStream_t s, const int32_t *list, int64_t nlist) {
  if (b.count == 0 || nlist <= 0) return HSM_OK;
  SolveArgs a;
  a.x = x_int; a.normal = normal_int; a.N = st->N; a.idx = b.idx.as<int32_t>(); a.count = b.count;
  a.start = b.start; a.w = b.w.as<double>(); a.wall = (b.type == B_DIR || b.type == B_NEU);
  a.perm = st->perm.as<int32_t>(); a.status = status;
  a.retry = nullptr; a.nretry = nullptr; a.list = list;
  const int d = st->d, m = b.m, n = b.width;
  if (d == 2 && m == 2 && n == 12) launch_rbffd<2, 1, 12>(a, s, nlist);
  else if (d == 2 && m == 3 && n == 20) launch_rbffd<2, 2, 20>(a, s, nlist);
  else if (d == 2 && m == 4 && n == 30) launch_rbffd<2, 3, 30>(a, s, nlist);
  else if (d == 3 && m == 2 && n == 20) launch_rbffd<3, 1, 20>(a, s, nlist);
  else if (d == 3 && m == 2 && n == 30) launch_rbffd<3, 1, 30>(a, s, nlist);
  else if (d == 3 && m == 3 && n == 40) launch_rbffd<3, 2, 40>(a, s, nlist);
  else {
    // no reduced-degree kernel (m = 1): the singular system is an error
    set_error(HSM_E_SINGULAR, "singular local system at a wall node (no lower-degree fallback for m = 1)");
    return HSM_E_SINGULAR;
  }
  HSM_HIP(hipGetLastError());
  return HSM_OK;
}


// Condition numbers of every node of a bucket (the system solved for its
// weights), written to kappa [N] in caller order.  With a list, only the
// listed nodes of the bucket, with monomials of degree m-1 (the wall
// fallback).
hsm_status cond_bucket(const hsm_stencils *st, const Bucket &b, double *kappa, hipStream_t s, const int32_t *list,
                       int64_t nlist) {
  if (b.count == 0 || (list && nlist <= 0)) return HSM_OK;
  SolveArgs a;
  std::memset(&a, 0, sizeof(a));
  a.x = st->x.as<double>(); a.normal = st->normal.as<double>(); a.N = st->N; a.idx = b.idx.as<int32_t>();
  a.count = b.count; a.start = b.start; a.perm = st->perm.as<int32_t>(); a.list = list; a.kappa = kappa;
  const int d = st->d, m = b.m, n = b.width;
  const int64_t nl = list ? nlist : -1;
  if (b.type == B_REG) {
    if (list) return HSM_OK;
    if (d == 2) hipLaunchKernelGGL(k_cond_mon<2>, dim3((unsigned)b.count), dim3(64), 0, s, a);
    else hipLaunchKernelGGL(k_cond_mon<3>, dim3((unsigned)b.count), dim3(64), 0, s, a);
  } else if (!list) {
    if (d == 2 && m == 1 && n == 6) launch_cond<2, 1, 6>(a, s);
    else if (d == 2 && m == 2 && n == 12) launch_cond<2, 2, 12>(a, s);
    else if (d == 2 && m == 3 && n == 20) launch_cond<2, 3, 20>(a, s);
    else if (d == 2 && m == 4 && n == 30) launch_cond<2, 4, 30>(a, s);
    else if (d == 3 && m == 1 && n == 8) launch_cond<3, 1, 8>(a, s);
    else if (d == 3 && m == 2 && n == 20) launch_cond<3, 2, 20>(a, s);
    else if (d == 3 && m == 2 && n == 30) launch_cond<3, 2, 30>(a, s);
    else if (d == 3 && m == 3 && n == 40) launch_cond<3, 3, 40>(a, s);
    else { set_error(HSM_E_INVALID, "no condition-number kernel for this (d, m, n)"); return HSM_E_INVALID; }
  } else {
    if (d == 2 && m == 2 && n == 12) launch_cond<2, 1, 12>(a, s, nl);
    else if (d == 2 && m == 3 && n == 20) launch_cond<2, 2, 20>(a, s, nl);
    else if (d == 2 && m == 4 && n == 30) launch_cond<2, 3, 30>(a, s, nl);
    else if (d == 3 && m == 2 && n == 20) launch_cond<3, 1, 20>(a, s, nl);
    else if (d == 3 && m == 2 && n == 30) launch_cond<3, 1, 30>(a, s, nl);
    else if (d == 3 && m == 3 && n == 40) launch_cond<3, 2, 40>(a, s, nl);
    else { set_error(HSM_E_INVALID, "no reduced-degree condition-number kernel"); return HSM_E_INVALID; }
  }
  HSM_HIP(hipGetLastError());
  return HSM_OK;
}
}  // namespace hsm
