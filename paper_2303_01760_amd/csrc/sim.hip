// Explicit time stepping of the Boussinesq natural-convection equations
// (Eqs. (2)-(4)) with Chorin's projection (Section 3), on the width-bucketed
// stencils.  Per step, in internal node order:
//   pre : predictor v* (fused: all derivatives of all velocity components in
//         one pass over the stencils), pressure right-hand side and the
//         initial Krylov residual;
//   Krylov: BiCGSTAB on the bordered pressure system, three fused kernels per
//         iteration (each recomputes the combined vector it multiplies on the
//         fly at the neighbours, so a matrix-vector product and the vector
//         update before it are one pass);
//   post: projection v = v* - dt grad p fused with the heat update, then the
//         Neumann-wall temperatures.
// Reductions are deterministic: fixed per-block trees, then the last block to
// finish sums the block partials in block order.  The three phases are
// replayed from HIP graphs; the host only reads a convergence flag between
// batches of Krylov iterations.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <memory>
#include <type_traits>
#include <vector>

#include "hsm_internal.h"

namespace hsm {
namespace {

constexpr int kBS = 256;
constexpr int kNQ = 4;          // partial sums per block
constexpr int kMaxIterChunk = 256;

struct Scalars {
  double rho, alpha, omega, beta;
  double bnorm2, rr, ss, relres;
  int32_t done, first, zero_sol, early_s;
  int32_t iters, fail, nonfinite, ticket;
};

struct HostFlags {
  int32_t done, iters, fail, nonfinite;
  double relres;
  double pad;
};

struct SimArgs {
  const BucketTable *tab;          // device table; aux = row-scaled pressure weights [W][count]
  int64_t N;
  double dt, Ra, Pr, T_ref, tol;
  int32_t maxiter, pad;
  // fields
  const double *v;    // [D][N]
  double *vs;         // [D][N]
  const double *T;    // [N]
  double *Tn;         // [N]
  double *vout;       // [D][N]
  // Krylov vectors, each [N+1] (slot N: the border multiplier / zero-mean row)
  double *x, *r, *rh, *Pold, *Vold, *Pnew, *Vnew, *S, *Tv;
  double *partials;   // [nblocks][kNQ]
  Scalars *sc;
};

template <class F>
__device__ __forceinline__ void with_width2(int w, F &&f) {
  switch (w) {
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 12: f(std::integral_constant<int, 12>{}); break;
    case 20: f(std::integral_constant<int, 20>{}); break;
    case 30: f(std::integral_constant<int, 30>{}); break;
    default: break;
  }
}
template <class F>
__device__ __forceinline__ void with_width3(int w, F &&f) {
  switch (w) {
    case 7: f(std::integral_constant<int, 7>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 20: f(std::integral_constant<int, 20>{}); break;
    case 30: f(std::integral_constant<int, 30>{}); break;
    case 40: f(std::integral_constant<int, 40>{}); break;
    default: break;
  }
}
template <int D, class F>
__device__ __forceinline__ void with_width(int w, F &&f) {
  if constexpr (D == 2) with_width2(w, f);
  else with_width3(w, f);
}

// bucket fields as plain scalars
struct BScal {
  int64_t start, count, block0;
  int32_t type, width;
  const int32_t *idx;
  const double *w;
  const double *wP;
};

// Deterministic block sum of kNQ values; thread 0 gets the totals.
__device__ __forceinline__ void block_sum(double (&v)[kNQ]) {
  __shared__ double red[kBS / 64][kNQ];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kNQ; ++q) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
  }
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < kNQ; ++q) red[wv][q] = v[q];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kNQ; ++q) {
      double s = red[0][q];
#pragma unroll
      for (int k = 1; k < kBS / 64; ++k) s += red[k][q];
      v[q] = s;
    }
  }
  __syncthreads();
}

// Writes this block's partials; returns true in every thread of the last
// block to finish, which then holds the grid totals in tot (thread 0 only).
__device__ __forceinline__ bool grid_sum(double (&v)[kNQ], double *partials, Scalars *sc, double (&tot)[kNQ]) {
  __shared__ int last;
  block_sum(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kNQ; ++q) partials[(int64_t)blockIdx.x * kNQ + q] = v[q];
    __threadfence();
    const int tk = atomicAdd(&sc->ticket, 1);
    last = (tk == (int)gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  double acc[kNQ];
#pragma unroll
  for (int q = 0; q < kNQ; ++q) acc[q] = 0.0;
  for (int64_t b = threadIdx.x; b < gridDim.x; b += kBS)
#pragma unroll
    for (int q = 0; q < kNQ; ++q) acc[q] += __builtin_nontemporal_load(&partials[b * kNQ + q]);
  block_sum(acc);
#pragma unroll
  for (int q = 0; q < kNQ; ++q) tot[q] = acc[q];
  if (threadIdx.x == 0) sc->ticket = 0;
  return true;
}

// ------------------------------------------------------------- predictor --
template <int D>
__global__ __launch_bounds__(kBS) void k_predict(SimArgs a) {
  const BucketDesc bd = select_bucket(a.tab, blockIdx.x);
  const BScal b{bd.start, bd.count, bd.block0, bd.type, bd.width, bd.idx, static_cast<const double *>(bd.w),
                static_cast<const double *>(bd.aux)};
  const int64_t t = ((int64_t)blockIdx.x - b.block0) * kBS + threadIdx.x;
  if (t >= b.count) return;
  const int64_t N = a.N, i = b.start + t, cnt = b.count;
  if (b.type == B_DIR || b.type == B_NEU) {
#pragma unroll
    for (int c = 0; c < D; ++c) a.vs[c * N + i] = 0.0;
    return;
  }
  const double *__restrict__ w = b.w;
  const int32_t *__restrict__ idx = b.idx;
  const double *__restrict__ v = a.v;
  double *__restrict__ vs = a.vs;
  const double Ti = a.T[i], Tref = a.T_ref, Ra = a.Ra, Pr = a.Pr, dt = a.dt;
  with_width<D>(b.width, [&](auto wc) __attribute__((always_inline)) {
    constexpr int W = decltype(wc)::value;
    double g[D][D], L[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      L[c] = 0.0;
#pragma unroll
      for (int q = 0; q < D; ++q) g[c][q] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const int32_t nb = idx[(int64_t)j * cnt + t];
      double wq[D + 1];
#pragma unroll
      for (int q = 0; q <= D; ++q) wq[q] = w[((int64_t)q * W + j) * cnt + t];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const double u = v[c * N + nb];
#pragma unroll
        for (int q = 0; q < D; ++q) g[c][q] = fma(wq[q], u, g[c][q]);
        L[c] = fma(wq[D], u, L[c]);
      }
    }
    double vi[D];
#pragma unroll
    for (int q = 0; q < D; ++q) vi[q] = v[q * N + i];
    const double buoy = (Ra * Pr) * (Ti - Tref);
#pragma unroll
    for (int c = 0; c < D; ++c) {
      double adv = vi[0] * g[c][0];
#pragma unroll
      for (int q = 1; q < D; ++q) adv = fma(vi[q], g[c][q], adv);
      double f = fma(Pr, L[c], -adv);
      if (c == D - 1) f += buoy;
      vs[c * N + i] = fma(dt, f, vi[c]);
    }
  });
}

// ---------------------------------------- pressure rhs + initial residual --
template <int D>
__global__ __launch_bounds__(kBS) void k_rhs(SimArgs a) {
  const BucketDesc bd = select_bucket(a.tab, blockIdx.x);
  const BScal b{bd.start, bd.count, bd.block0, bd.type, bd.width, bd.idx, static_cast<const double *>(bd.w),
                static_cast<const double *>(bd.aux)};
  const int64_t t = ((int64_t)blockIdx.x - b.block0) * kBS + threadIdx.x;
  double part[kNQ] = {0.0, 0.0, 0.0, 0.0};  // b^2, r^2, sum p
  const int64_t N = a.N;
  const double lam = a.x[N];
  if (t < b.count) {
    const int64_t i = b.start + t, cnt = b.count;
    const double *w = b.w;
    const double *wP = b.wP;
    const bool wall = (b.type == B_DIR || b.type == B_NEU);
    with_width<D>(b.width, [&](auto wc) __attribute__((always_inline)) {
      constexpr int W = decltype(wc)::value;
      double div = 0.0, Ap = 0.0;
#pragma unroll
      for (int j = 0; j < W; ++j) {
        const int32_t nb = b.idx[(int64_t)j * cnt + t];
        Ap = fma(wP[(int64_t)j * cnt + t], a.x[nb], Ap);
        if (!wall)
#pragma unroll
          for (int q = 0; q < D; ++q) div = fma(w[((int64_t)q * W + j) * cnt + t], a.vs[q * N + nb], div);
      }
      double rhs = 0.0;
      if (!wall) rhs = (div / a.dt) / w[((int64_t)D * W + 0) * cnt + t];
      const double r = rhs - (Ap + lam);
      a.r[i] = r;
      a.rh[i] = r;
      part[0] = rhs * rhs;
      part[1] = r * r;
      part[2] = a.x[i];
    });
  }
  double tot[kNQ];
  if (grid_sum(part, a.partials, a.sc, tot) && threadIdx.x == 0) {
    Scalars *sc = a.sc;
    const double rN = -tot[2];    // border row: 0 - sum p
    a.r[N] = rN;
    a.rh[N] = rN;
    sc->bnorm2 = tot[0];
    sc->rr = tot[1] + rN * rN;
    sc->rho = sc->rr;
    sc->alpha = 1.0; sc->omega = 1.0; sc->beta = 0.0;
    sc->first = 1; sc->iters = 0; sc->fail = 0; sc->early_s = 0;
    sc->zero_sol = (tot[0] == 0.0) ? 1 : 0;
    const double bn = sqrt(tot[0]);
    sc->relres = bn > 0.0 ? sqrt(sc->rr) / bn : 0.0;
    sc->done = (bn == 0.0 || sqrt(sc->rr) <= a.tol * bn) ? 1 : 0;
  }
}

// ------------------------------------------------------- BiCGSTAB steps --
// (a) p = r + beta (p - omega v) on the fly, v = A p, (rh, v)
template <int D>
__global__ __launch_bounds__(kBS) void k_bicg_pv(SimArgs a) {
  const Scalars *scr = a.sc;
  if (scr->done) return;
  const BucketDesc bd = select_bucket(a.tab, blockIdx.x);
  const BScal b{bd.start, bd.count, bd.block0, bd.type, bd.width, bd.idx, static_cast<const double *>(bd.w),
                static_cast<const double *>(bd.aux)};
  const int64_t t = ((int64_t)blockIdx.x - b.block0) * kBS + threadIdx.x;
  const int64_t N = a.N;
  const bool first = scr->first != 0;
  const double beta = scr->beta, omega = scr->omega;
  const double *__restrict__ r = a.r;
  const double *__restrict__ Po = a.Pold;
  const double *__restrict__ Vo = a.Vold;
  auto pnew = [&](int64_t j) { return first ? r[j] : fma(beta, fma(-omega, Vo[j], Po[j]), r[j]); };
  const double pN = pnew(N);
  double part[kNQ] = {0.0, 0.0, 0.0, 0.0};  // (rh, v), sum p
  if (t < b.count) {
    const int64_t i = b.start + t, cnt = b.count;
    const double *wP = b.wP;
    with_width<D>(b.width, [&](auto wc) __attribute__((always_inline)) {
      constexpr int W = decltype(wc)::value;
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < W; ++j) {
        const int32_t nb = b.idx[(int64_t)j * cnt + t];
        acc = fma(wP[(int64_t)j * cnt + t], pnew(nb), acc);
      }
      const double vi = acc + pN;
      const double pi = pnew(i);
      a.Pnew[i] = pi;
      a.Vnew[i] = vi;
      part[0] = a.rh[i] * vi;
      part[1] = pi;
    });
  }
  double tot[kNQ];
  if (grid_sum(part, a.partials, a.sc, tot) && threadIdx.x == 0) {
    Scalars *sc = a.sc;
    const double vN = tot[1];
    a.Pnew[N] = pN;
    a.Vnew[N] = vN;
    const double rv = tot[0] + a.rh[N] * vN;
    if (rv == 0.0) { sc->fail = 1; sc->done = 1; }
    else sc->alpha = sc->rho / rv;
  }
}

// (b) s = r - alpha v on the fly, t = A s, (t, s), (t, t), sum s, (s, s)
template <int D>
__global__ __launch_bounds__(kBS) void k_bicg_st(SimArgs a) {
  const Scalars *scr = a.sc;
  if (scr->done) return;
  const BucketDesc bd = select_bucket(a.tab, blockIdx.x);
  const BScal b{bd.start, bd.count, bd.block0, bd.type, bd.width, bd.idx, static_cast<const double *>(bd.w),
                static_cast<const double *>(bd.aux)};
  const int64_t t = ((int64_t)blockIdx.x - b.block0) * kBS + threadIdx.x;
  const int64_t N = a.N;
  const double alpha = scr->alpha;
  const double *__restrict__ r = a.r;
  const double *__restrict__ V = a.Vnew;
  auto snew = [&](int64_t j) { return fma(-alpha, V[j], r[j]); };
  const double sN = snew(N);
  double part[kNQ] = {0.0, 0.0, 0.0, 0.0};
  if (t < b.count) {
    const int64_t i = b.start + t, cnt = b.count;
    const double *wP = b.wP;
    with_width<D>(b.width, [&](auto wc) __attribute__((always_inline)) {
      constexpr int W = decltype(wc)::value;
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < W; ++j) {
        const int32_t nb = b.idx[(int64_t)j * cnt + t];
        acc = fma(wP[(int64_t)j * cnt + t], snew(nb), acc);
      }
      const double ti = acc + sN;
      const double si = snew(i);
      a.S[i] = si;
      a.Tv[i] = ti;
      part[0] = ti * si;
      part[1] = ti * ti;
      part[2] = si;
      part[3] = si * si;
    });
  }
  double tot[kNQ];
  if (grid_sum(part, a.partials, a.sc, tot) && threadIdx.x == 0) {
    Scalars *sc = a.sc;
    const double tN = tot[2];
    a.S[N] = sN;
    a.Tv[N] = tN;
    const double ts = fma(tN, sN, tot[0]);
    const double tt = fma(tN, tN, tot[1]);
    const double ss = fma(sN, sN, tot[3]);
    sc->ss = ss;
    const double bn = sqrt(sc->bnorm2);
    if (sqrt(ss) <= a.tol * bn) sc->early_s = 1;
    else if (tt == 0.0) { sc->fail = 1; sc->done = 1; }
    else sc->omega = ts / tt;
  }
}

// (c) x += alpha p + omega s, r = s - omega t, (rh, r), (r, r); next beta
template <int D>
__global__ __launch_bounds__(kBS) void k_bicg_xr(SimArgs a) {
  const Scalars *scr = a.sc;
  if (scr->done) return;
  const int64_t N = a.N;
  const int64_t i = (int64_t)blockIdx.x * kBS + threadIdx.x;
  const double alpha = scr->alpha, omega = scr->omega;
  const bool early = scr->early_s != 0;
  double part[kNQ] = {0.0, 0.0, 0.0, 0.0};
  if (i < N) {
    if (early) {
      a.x[i] = fma(alpha, a.Pnew[i], a.x[i]);
    } else {
      const double si = a.S[i];
      a.x[i] = fma(omega, si, fma(alpha, a.Pnew[i], a.x[i]));
      const double ri = fma(-omega, a.Tv[i], si);
      a.r[i] = ri;
      part[0] = a.rh[i] * ri;
      part[1] = ri * ri;
    }
  }
  double tot[kNQ];
  if (grid_sum(part, a.partials, a.sc, tot) && threadIdx.x == 0) {
    Scalars *sc = a.sc;
    sc->iters += 1;
    const double bn = sqrt(sc->bnorm2);
    if (early) {
      a.x[N] = fma(alpha, a.Pnew[N], a.x[N]);
      sc->relres = sqrt(sc->ss) / bn;
      sc->done = 1;
    } else {
      const double sN = a.S[N];
      a.x[N] = fma(omega, sN, fma(alpha, a.Pnew[N], a.x[N]));
      const double rN = fma(-omega, a.Tv[N], sN);
      a.r[N] = rN;
      const double rho_new = fma(a.rh[N], rN, tot[0]);
      const double rr = fma(rN, rN, tot[1]);
      sc->rr = rr;
      sc->relres = sqrt(rr) / bn;
      if (sqrt(rr) <= a.tol * bn) sc->done = 1;
      else if (sc->iters >= a.maxiter) { sc->fail = 2; sc->done = 1; }
      else if (rho_new == 0.0 || omega == 0.0) { sc->fail = 1; sc->done = 1; }
      else {
        sc->beta = (rho_new / sc->rho) * (alpha / omega);
        sc->rho = rho_new;
        sc->first = 0;
      }
    }
  }
}

// -------------------------------------------- projection + heat transport --
template <int D>
__global__ __launch_bounds__(kBS) void k_correct_heat(SimArgs a) {
  const BucketDesc bd = select_bucket(a.tab, blockIdx.x);
  const BScal b{bd.start, bd.count, bd.block0, bd.type, bd.width, bd.idx, static_cast<const double *>(bd.w),
                static_cast<const double *>(bd.aux)};
  const int64_t t = ((int64_t)blockIdx.x - b.block0) * kBS + threadIdx.x;
  const int64_t N = a.N;
  const bool zero = a.sc->zero_sol != 0;
  if (zero && blockIdx.x == 0 && threadIdx.x == 0) a.x[N] = 0.0;
  if (t >= b.count) return;
  const int64_t i = b.start + t, cnt = b.count;
  bool bad = false;
  if (b.type == B_DIR || b.type == B_NEU) {
#pragma unroll
    for (int c = 0; c < D; ++c) a.vout[c * N + i] = 0.0;
    if (b.type == B_DIR) a.Tn[i] = a.T[i];
    if (zero) a.x[i] = 0.0;
    return;
  }
  const double *__restrict__ w = b.w;
  const int32_t *__restrict__ idx = b.idx;
  const double *__restrict__ px = a.x;
  const double *__restrict__ T = a.T;
  const double *__restrict__ vs = a.vs;
  double *__restrict__ vout = a.vout;
  double *__restrict__ Tnp = a.Tn;
  const double dt = a.dt;
  with_width<D>(b.width, [&](auto wc) __attribute__((always_inline)) {
    constexpr int W = decltype(wc)::value;
    double gp[D], gT[D], LT = 0.0;
#pragma unroll
    for (int q = 0; q < D; ++q) { gp[q] = 0.0; gT[q] = 0.0; }
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const int32_t nb = idx[(int64_t)j * cnt + t];
      const double pj = zero ? 0.0 : px[nb];
      const double Tj = T[nb];
#pragma unroll
      for (int q = 0; q < D; ++q) {
        const double wq = w[((int64_t)q * W + j) * cnt + t];
        gp[q] = fma(wq, pj, gp[q]);
        gT[q] = fma(wq, Tj, gT[q]);
      }
      LT = fma(w[((int64_t)D * W + j) * cnt + t], Tj, LT);
    }
    double vn[D];
#pragma unroll
    for (int q = 0; q < D; ++q) {
      vn[q] = fma(-dt, gp[q], vs[q * N + i]);
      vout[q * N + i] = vn[q];
      bad = bad || !isfinite(vn[q]);
    }
    double adv = vn[0] * gT[0];
#pragma unroll
    for (int q = 1; q < D; ++q) adv = fma(vn[q], gT[q], adv);
    const double Tn = fma(dt, LT - adv, T[i]);
    Tnp[i] = Tn;
    bad = bad || !isfinite(Tn);
  });
  if (zero) a.x[i] = 0.0;
  if (bad) atomicOr(&a.sc->nonfinite, 1);
}

// Neumann walls: the temperature that zeroes the normal derivative, from the
// new interior values (wall stencils hold the wall node and interior nodes).
template <int D>
__global__ __launch_bounds__(kBS) void k_neumann(SimArgs a) {
  const BucketDesc bd = select_bucket(a.tab, blockIdx.x);
  const BScal b{bd.start, bd.count, bd.block0, bd.type, bd.width, bd.idx, static_cast<const double *>(bd.w),
                static_cast<const double *>(bd.aux)};
  const int64_t t = ((int64_t)blockIdx.x - b.block0) * kBS + threadIdx.x;
  if (t >= b.count || b.type != B_NEU) return;
  const int64_t N = a.N, i = b.start + t, cnt = b.count;
  const double *__restrict__ w = b.w;
  const int32_t *__restrict__ idx = b.idx;
  double *Tn = a.Tn;
  Scalars *sc = a.sc;
  with_width<D>(b.width, [&](auto wc) __attribute__((always_inline)) {
    constexpr int W = decltype(wc)::value;
    const double *wn = w + (int64_t)(D + 1) * W * cnt;
    double acc = 0.0;
#pragma unroll
    for (int j = 1; j < W; ++j) acc = fma(wn[(int64_t)j * cnt + t], Tn[idx[(int64_t)j * cnt + t]], acc);
    const double Tb = -acc / wn[t];
    Tn[i] = Tb;
    if (!isfinite(Tb)) atomicOr(&sc->nonfinite, 1);
  });
  (void)N;
}

// pressure-operator rows: Laplacian (interior) or normal derivative (walls), divided by the centre weight
__global__ void k_scale_rows(const double *w, int64_t cnt, int W, int slot, double *wP) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt) return;
  const double *src = w + (int64_t)slot * W * cnt;
  const double dg = src[t];
  for (int j = 0; j < W; ++j) wP[(int64_t)j * cnt + t] = src[(int64_t)j * cnt + t] / dg;
}

__global__ void k_fill(double *p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_init_scalars(Scalars *sc) {
  if (threadIdx.x == 0) {
    memset(sc, 0, sizeof(Scalars));
    sc->done = 1;
  }
}

template <class T>
__global__ void k_gather(const T *src, T *dst, const int32_t *map, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[map[i]];
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace
}  // namespace hsm

using namespace hsm;

struct hsm_sim {
  const hsm_stencils *st = nullptr;
  hsm_sim_params prm{};
  int d = 0;
  int64_t N = 0;
  int chunk = 16;
  DBuf v, vs, T[2], vec[9], partials, sc, wP[kMaxBuckets];
  double *x = nullptr, *r = nullptr, *rh = nullptr, *P[2] = {nullptr, nullptr}, *V[2] = {nullptr, nullptr},
         *S = nullptr, *Tv = nullptr;
  int parity = 0;
  hipStream_t s = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_chunk[2] = {nullptr, nullptr};
  HostFlags *hflags = nullptr;   // pinned [2]
  bool graphs_ready = false;
  hipGraphExec_t g_pre[2] = {nullptr, nullptr}, g_kry[2] = {nullptr, nullptr}, g_post[2] = {nullptr, nullptr};
  hipGraph_t gr[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  hsm_sim_stats stats{};
  int64_t n_int = 0, n_neu = 0;
  BucketTable tab_all{};
  DBuf dtab;
  int64_t nblk_nodes = 0;

  ~hsm_sim() {
    if (s) (void)hipStreamSynchronize(s);
    for (auto &g : g_pre) if (g) (void)hipGraphExecDestroy(g);
    for (auto &g : g_kry) if (g) (void)hipGraphExecDestroy(g);
    for (auto &g : g_post) if (g) (void)hipGraphExecDestroy(g);
    for (auto &g : gr) if (g) (void)hipGraphDestroy(g);
    if (hflags) (void)hipHostFree(hflags);
    for (auto &e : ev_chunk) if (e) (void)hipEventDestroy(e);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (s) (void)hipStreamDestroy(s);
  }
};

namespace hsm {
namespace {

SimArgs make_args(hsm_sim *m, int par, int kpar) {
  SimArgs a;
  std::memset(&a, 0, sizeof(a));
  a.tab = m->dtab.as<BucketTable>();
  a.N = m->N;
  a.dt = m->prm.dt; a.Ra = m->prm.Ra; a.Pr = m->prm.Pr; a.T_ref = m->prm.T_ref; a.tol = m->prm.krylov_tol;
  a.maxiter = m->prm.krylov_maxiter;
  a.v = m->v.as<double>();
  a.vs = m->vs.as<double>();
  a.T = m->T[par].as<double>();
  a.Tn = m->T[par ^ 1].as<double>();
  a.vout = m->v.as<double>();
  a.x = m->x; a.r = m->r; a.rh = m->rh;
  a.Pold = m->P[kpar]; a.Vold = m->V[kpar]; a.Pnew = m->P[kpar ^ 1]; a.Vnew = m->V[kpar ^ 1];
  a.S = m->S; a.Tv = m->Tv;
  a.partials = m->partials.as<double>();
  a.sc = m->sc.as<Scalars>();
  return a;
}

template <int D>
hsm_status enqueue_pre(hsm_sim *m, int par, hipStream_t s) {
  SimArgs a = make_args(m, par, 0);
  hipLaunchKernelGGL(k_predict<D>, dim3((unsigned)m->tab_all.nblocks), dim3(kBS), 0, s, a);
  hipLaunchKernelGGL(k_rhs<D>, dim3((unsigned)m->tab_all.nblocks), dim3(kBS), 0, s, a);
  HSM_HIP(hipGetLastError());
  return HSM_OK;
}

template <int D>
hsm_status enqueue_krylov(hsm_sim *m, int slot, hipStream_t s) {
  for (int it = 0; it < m->chunk; ++it) {
    SimArgs a = make_args(m, 0, it & 1);
    hipLaunchKernelGGL(k_bicg_pv<D>, dim3((unsigned)m->tab_all.nblocks), dim3(kBS), 0, s, a);
    hipLaunchKernelGGL(k_bicg_st<D>, dim3((unsigned)m->tab_all.nblocks), dim3(kBS), 0, s, a);
    hipLaunchKernelGGL(k_bicg_xr<D>, dim3(nblk(m->N, kBS)), dim3(kBS), 0, s, a);
  }
  HSM_HIP(hipGetLastError());
  Scalars *sc = m->sc.as<Scalars>();
  // iters, fail and nonfinite are consecutive in both structs
  HSM_HIP(hipMemcpyAsync(&m->hflags[slot].iters, &sc->iters, sizeof(int32_t) * 3, hipMemcpyDeviceToHost, s));
  HSM_HIP(hipMemcpyAsync(&m->hflags[slot].relres, &sc->relres, sizeof(double), hipMemcpyDeviceToHost, s));
  HSM_HIP(hipMemcpyAsync(&m->hflags[slot].done, &sc->done, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  return HSM_OK;
}

template <int D>
hsm_status enqueue_post(hsm_sim *m, int par, hipStream_t s) {
  SimArgs a = make_args(m, par, 0);
  hipLaunchKernelGGL(k_correct_heat<D>, dim3((unsigned)m->tab_all.nblocks), dim3(kBS), 0, s, a);
  hipLaunchKernelGGL(k_neumann<D>, dim3((unsigned)m->tab_all.nblocks), dim3(kBS), 0, s, a);
  HSM_HIP(hipGetLastError());
  return HSM_OK;
}

template <class F>
hsm_status capture(hsm_sim *m, hipGraph_t &g, hipGraphExec_t &e, F &&f) {
  HSM_HIP(hipStreamBeginCapture(m->s, hipStreamCaptureModeRelaxed));
  hsm_status rc = f();
  hipGraph_t graph = nullptr;
  hipError_t ee = hipStreamEndCapture(m->s, &graph);
  if (rc) { if (graph) (void)hipGraphDestroy(graph); return rc; }
  if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
  g = graph;
  HSM_HIP(hipGraphInstantiate(&e, graph, nullptr, nullptr, 0));
  return HSM_OK;
}

template <int D>
hsm_status make_graphs(hsm_sim *m) {
  hsm_status rc;
  for (int par = 0; par < 2; ++par) {
    if ((rc = capture(m, m->gr[par], m->g_pre[par], [&] { return enqueue_pre<D>(m, par, m->s); }))) return rc;
    if ((rc = capture(m, m->gr[2 + par], m->g_kry[par], [&] { return enqueue_krylov<D>(m, par, m->s); }))) return rc;
    if ((rc = capture(m, m->gr[4 + par], m->g_post[par], [&] { return enqueue_post<D>(m, par, m->s); }))) return rc;
  }
  m->graphs_ready = true;
  return HSM_OK;
}

// Direct launches of the same work (launch_mode 1).
template <int D>
hsm_status launch_pre(hsm_sim *m, int par) { return enqueue_pre<D>(m, par, m->s); }
template <int D>
hsm_status launch_krylov(hsm_sim *m, int slot) { return enqueue_krylov<D>(m, slot, m->s); }
template <int D>
hsm_status launch_post(hsm_sim *m, int par) { return enqueue_post<D>(m, par, m->s); }

hsm_status do_pre(hsm_sim *m, int par) {
  if (m->prm.launch_mode == 1) return m->d == 2 ? launch_pre<2>(m, par) : launch_pre<3>(m, par);
  HSM_HIP(hipGraphLaunch(m->g_pre[par], m->s));
  return HSM_OK;
}
hsm_status do_krylov(hsm_sim *m, int slot) {
  if (m->prm.launch_mode == 1) return m->d == 2 ? launch_krylov<2>(m, slot) : launch_krylov<3>(m, slot);
  HSM_HIP(hipGraphLaunch(m->g_kry[slot], m->s));
  return HSM_OK;
}
hsm_status do_post(hsm_sim *m, int par) {
  if (m->prm.launch_mode == 1) return m->d == 2 ? launch_post<2>(m, par) : launch_post<3>(m, par);
  HSM_HIP(hipGraphLaunch(m->g_post[par], m->s));
  return HSM_OK;
}

hsm_status run_steps(hsm_sim *m, int nsteps) {
  hsm_status rc;
  if (!m->graphs_ready && m->prm.launch_mode == 0) {
    if ((rc = (m->d == 2 ? make_graphs<2>(m) : make_graphs<3>(m)))) return rc;
  }
  const int D = m->d;
  const int64_t per_iter = 2 * m->N;
  const int max_chunks = m->prm.krylov_maxiter / m->chunk + 2;
  for (int k = 0; k < nsteps; ++k) {
    const int par = m->parity;
    if ((rc = do_pre(m, par))) return rc;
    if ((rc = do_krylov(m, 0))) return rc;
    HSM_HIP(hipEventRecord(m->ev_chunk[0], m->s));
    int c = 0;
    HostFlags f{};
    for (;;) {
      const int nxt = (c + 1) & 1;
      if ((rc = do_krylov(m, nxt))) return rc;             // queued ahead; a no-op once converged
      HSM_HIP(hipEventRecord(m->ev_chunk[nxt], m->s));
      HSM_HIP(hipEventSynchronize(m->ev_chunk[c & 1]));
      f = m->hflags[c & 1];
      if (f.done || f.nonfinite) break;
      if (++c > max_chunks) { f.fail = 2; break; }
    }
    if ((rc = do_post(m, par))) return rc;
    m->parity ^= 1;
    m->stats.steps += 1;
    m->stats.krylov_iters_last = f.iters;
    m->stats.krylov_iters_total += f.iters;
    m->stats.last_relres = f.relres;
    m->stats.node_applies += m->n_int * (D * (D + 1) + D + 2 * D + 1) + m->N + per_iter * f.iters + m->n_neu;
    if (f.nonfinite) { m->stats.status = HSM_E_NONFINITE; break; }
    if (f.fail) { m->stats.status = HSM_E_NOT_CONVERGED; break; }
  }
  if (m->stats.status) {
    set_error(m->stats.status, m->stats.status == HSM_E_NONFINITE ? "non-finite field during stepping"
                                                                  : "pressure solve did not converge");
    return m->stats.status;
  }
  return HSM_OK;
}

}  // namespace
}  // namespace hsm

extern "C" {

hsm_status hsm_sim_create(const hsm_stencils *st, const hsm_sim_params *prm, const double *v, const double *T,
                          const double *p, void *stream, hsm_sim **out) {
  if (!out) { set_error(HSM_E_INVALID, "out is NULL"); return HSM_E_INVALID; }
  *out = nullptr;
  if (!st || !prm || !v || !T) { set_error(HSM_E_INVALID, "stencils, params, v and T are required"); return HSM_E_INVALID; }
  if (!(prm->dt > 0) || !std::isfinite(prm->dt) || !std::isfinite(prm->Ra) || !std::isfinite(prm->Pr) ||
      !std::isfinite(prm->T_ref) || !(prm->krylov_tol > 0) || prm->krylov_maxiter < 1) {
    set_error(HSM_E_INVALID, "bad simulation parameters");
    return HSM_E_INVALID;
  }
  if (prm->field_dtype != HSM_F64) { set_error(HSM_E_INVALID, "field_dtype must be HSM_F64"); return HSM_E_INVALID; }
  if (st->N < 1) { set_error(HSM_E_INVALID, "empty stencil set"); return HSM_E_INVALID; }
  if (prm->launch_mode != 0 && prm->launch_mode != 1) { set_error(HSM_E_INVALID, "launch_mode must be 0 or 1"); return HSM_E_INVALID; }
  if (prm->krylov_chunk < 0 || prm->krylov_chunk > kMaxIterChunk) {
    set_error(HSM_E_INVALID, "krylov_chunk out of range");
    return HSM_E_INVALID;
  }
  auto m = std::make_unique<hsm_sim>();
  m->st = st; m->prm = *prm; m->d = st->d; m->N = st->N;
  m->chunk = prm->krylov_chunk ? prm->krylov_chunk : 16;
  if (m->chunk & 1) m->chunk += 1;   // even: ping-pong buffers line up across batches
  const int64_t N = st->N, d = st->d;
  hipStream_t us = (hipStream_t)stream;
  hsm_status rc;
  if ((rc = m->v.alloc(sizeof(double) * d * N)) || (rc = m->vs.alloc(sizeof(double) * d * N)) ||
      (rc = m->T[0].alloc(sizeof(double) * N)) || (rc = m->T[1].alloc(sizeof(double) * N)) ||
      (rc = m->sc.alloc(sizeof(Scalars))))
    return rc;
  for (auto &b : m->vec)
    if ((rc = b.alloc(sizeof(double) * (N + 1)))) return rc;
  m->x = m->vec[0].as<double>(); m->r = m->vec[1].as<double>(); m->rh = m->vec[2].as<double>();
  m->P[0] = m->vec[3].as<double>(); m->P[1] = m->vec[4].as<double>();
  m->V[0] = m->vec[5].as<double>(); m->V[1] = m->vec[6].as<double>();
  m->S = m->vec[7].as<double>(); m->Tv = m->vec[8].as<double>();
  make_table(st, m->tab_all, kBS, 0xFu, false);
  if ((rc = m->partials.alloc(sizeof(double) * kNQ * (m->tab_all.nblocks + nblk(N, kBS) + 1)))) return rc;
  int k = 0;
  for (const Bucket &B : st->buckets) {
    if (B.count == 0) continue;
    if ((rc = m->wP[k].alloc(sizeof(double) * B.width * B.count))) return rc;
    const int slot = (B.type == B_DIR || B.type == B_NEU) ? st->d + 1 : st->d;
    hipLaunchKernelGGL(k_scale_rows, dim3(nblk(B.count, 256)), dim3(256), 0, us, B.w.as<double>(), B.count, B.width,
                       slot, m->wP[k].as<double>());
    if (B.type == B_REG || B.type == B_SCAT) m->n_int += B.count;
    if (B.type == B_NEU) m->n_neu += B.count;
    m->tab_all.b[k].aux = m->wP[k].p;
    ++k;
  }
  if ((rc = m->dtab.alloc(sizeof(BucketTable)))) return rc;
  HSM_HIP(hipMemcpyAsync(m->dtab.p, &m->tab_all, sizeof(BucketTable), hipMemcpyHostToDevice, us));
  const int32_t *perm = st->perm.as<int32_t>();
  for (int c = 0; c < d; ++c)
    hipLaunchKernelGGL(k_gather<double>, dim3(nblk(N, 256)), dim3(256), 0, us, v + c * N, m->v.as<double>() + c * N,
                       perm, N);
  hipLaunchKernelGGL(k_gather<double>, dim3(nblk(N, 256)), dim3(256), 0, us, T, m->T[0].as<double>(), perm, N);
  for (auto &b : m->vec) hipLaunchKernelGGL(k_fill, dim3(nblk(N + 1, 256)), dim3(256), 0, us, b.as<double>(), N + 1, 0.0);
  if (p) hipLaunchKernelGGL(k_gather<double>, dim3(nblk(N, 256)), dim3(256), 0, us, p, m->x, perm, N);
  hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(64), 0, us, m->sc.as<Scalars>());
  HSM_HIP(hipGetLastError());
  HSM_HIP(hipStreamSynchronize(us));
  HSM_HIP(hipStreamCreateWithFlags(&m->s, hipStreamNonBlocking));
  HSM_HIP(hipEventCreateWithFlags(&m->ev_in, hipEventDisableTiming));
  HSM_HIP(hipEventCreateWithFlags(&m->ev_out, hipEventDisableTiming));
  for (auto &e : m->ev_chunk) HSM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  HSM_HIP(hipHostMalloc((void **)&m->hflags, sizeof(HostFlags) * 2, hipHostMallocDefault));
  std::memset(m->hflags, 0, sizeof(HostFlags) * 2);
  *out = m.release();
  return HSM_OK;
}

hsm_status hsm_step(hsm_sim *m, int32_t nsteps, void *stream) {
  if (!m) { set_error(HSM_E_INVALID, "sim is NULL"); return HSM_E_INVALID; }
  if (nsteps < 0) { set_error(HSM_E_INVALID, "nsteps < 0"); return HSM_E_INVALID; }
  if (m->stats.status) { set_error(m->stats.status, "simulation already failed"); return m->stats.status; }
  if (nsteps == 0) return HSM_OK;
  hipStream_t us = (hipStream_t)stream;
  HSM_HIP(hipEventRecord(m->ev_in, us));
  HSM_HIP(hipStreamWaitEvent(m->s, m->ev_in, 0));
  hsm_status rc = run_steps(m, nsteps);
  HSM_HIP(hipEventRecord(m->ev_out, m->s));
  HSM_HIP(hipStreamWaitEvent(us, m->ev_out, 0));
  return rc;
}

hsm_status hsm_sim_get_stats(hsm_sim *m, hsm_sim_stats *out) {
  if (!m || !out) { set_error(HSM_E_INVALID, "NULL argument"); return HSM_E_INVALID; }
  HSM_HIP(hipStreamSynchronize(m->s));
  Scalars sc;
  HSM_HIP(hipMemcpy(&sc, m->sc.p, sizeof(Scalars), hipMemcpyDeviceToHost));
  if (sc.nonfinite && !m->stats.status) m->stats.status = HSM_E_NONFINITE;
  *out = m->stats;
  return m->stats.status;
}

hsm_status hsm_sim_read(hsm_sim *m, double *v, double *T, double *p, void *stream) {
  if (!m) { set_error(HSM_E_INVALID, "sim is NULL"); return HSM_E_INVALID; }
  hipStream_t us = (hipStream_t)stream;
  HSM_HIP(hipEventRecord(m->ev_out, m->s));
  HSM_HIP(hipStreamWaitEvent(us, m->ev_out, 0));
  const int64_t N = m->N;
  const int32_t *ip = m->st->iperm.as<int32_t>();
  if (v)
    for (int c = 0; c < m->d; ++c)
      hipLaunchKernelGGL(k_gather<double>, dim3(nblk(N, 256)), dim3(256), 0, us, m->v.as<double>() + c * N, v + c * N,
                         ip, N);
  if (T) hipLaunchKernelGGL(k_gather<double>, dim3(nblk(N, 256)), dim3(256), 0, us, m->T[m->parity].as<double>(), T, ip, N);
  if (p) hipLaunchKernelGGL(k_gather<double>, dim3(nblk(N, 256)), dim3(256), 0, us, (const double *)m->x, p, ip, N);
  HSM_HIP(hipGetLastError());
  return HSM_OK;
}

void hsm_sim_destroy(hsm_sim *m) { delete m; }

}  // extern "C"
