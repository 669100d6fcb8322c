// Explicit time stepping of the Boussinesq natural-convection equations
// (Eqs. (2)-(4)) with Chorin's projection (Section 3), on the width-bucketed
// stencils.  Per step, in internal node order:
//   pre : predictor v* (fused: all derivatives of all velocity components in
//         one pass over the stencils), pressure right-hand side and the
//         initial Krylov residual;
//   Krylov: BiCGSTAB on the bordered pressure system, two fused kernels per
//         iteration; each forms the vector it multiplies on the fly at the
//         neighbours, so the vector updates and the matrix-vector product are
//         one pass over the stencils;
//   post: projection v = v* - dt grad p fused with the heat update, then the
//         Neumann-wall temperatures.
// Reductions are deterministic and use no fences or atomics: each kernel
// writes one partial sum per block, and the next kernel reduces all of them
// in the same fixed order in every block.  The phases are replayed from HIP
// graphs; the host reads a convergence summary once per batch of iterations.
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
constexpr int kNR = 3;          // partial sums of the right-hand-side kernel
constexpr int kNA = 3;          // partial sums of the p/v kernel
constexpr int kNB = 6;          // partial sums of the s/t kernel
constexpr int kMaxIterChunk = 256;

// Host-visible summary written once per batch of Krylov iterations.
struct HostFlags {
  int32_t done, iters, fail, nonfinite;
  double relres;
  double pad;
};

// Krylov state.  Values a kernel computes for iteration k live in slot k & 1,
// so kernels of iteration k never overwrite what their own blocks still read.
struct Scalars {
  double rho[2], alpha[2];
  double bnorm2, relres;
  int32_t done, fail, zero_sol, nonfinite;
  int32_t it_base, iters, early[2];   // early: 1 = |s| converged, 2 = breakdown, 3 = zero right-hand side
  HostFlags mirror;
};

struct SimArgs {
  const BucketTable *tab;          // device table; aux = row-scaled pressure weights [W][count]
  int64_t N;
  double dt, Ra, Pr, T_ref, tol;
  int32_t maxiter, chunk;
  // fields
  const double *v;    // [D][N]
  double *vs;         // [D][N]
  const double *T;    // [N]
  double *Tn;         // [N]
  double *vout;       // [D][N]
  // Krylov vectors, each [N+1] (slot N: the border multiplier / zero-mean row)
  double *x, *r, *rh, *Pold, *Vold, *Pnew, *Vnew, *S, *Tv;
  double *partR, *partA, *partB;   // block partial sums [nblocks][kN*]
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

// Deterministic block sum of NQ values (fixed shuffle tree, then the waves in
// order); thread 0 writes the block's partials.  No fences or atomics: the
// consumer is a later kernel.
template <int NQ>
__device__ __forceinline__ void block_partials(double (&v)[NQ], double *part) {
  __shared__ double red[kBS / 64][NQ];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) red[wv][q] = v[q];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double s = red[0][q];
#pragma unroll
      for (int k = 1; k < kBS / 64; ++k) s += red[k][q];
      part[(int64_t)blockIdx.x * NQ + q] = s;
    }
}

// Grid totals of a previous kernel's block partials, reduced by every block
// in the same fixed order (so every block holds bit-identical totals).
template <int NQ>
__device__ __forceinline__ void reduce_prev(const double *__restrict__ part, int64_t nblk, double (&tot)[NQ]) {
  __shared__ double red[kBS / 64][NQ];
  __shared__ double res[NQ];
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  for (int64_t b = threadIdx.x; b < nblk; b += kBS)
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] += part[b * NQ + q];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o, 64);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) red[wv][q] = acc[q];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double s = red[0][q];
#pragma unroll
      for (int k = 1; k < kBS / 64; ++k) s += red[k][q];
      res[q] = s;
    }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) tot[q] = res[q];
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
// b = div(v*)/dt / diag at interior nodes, 0 at walls; r0 = b - A x; rh = r0.
template <int D>
__global__ __launch_bounds__(kBS) void k_rhs(SimArgs a) {
  const BucketDesc bd = select_bucket(a.tab, blockIdx.x);
  const BScal b{bd.start, bd.count, bd.block0, bd.type, bd.width, bd.idx, static_cast<const double *>(bd.w),
                static_cast<const double *>(bd.aux)};
  const int64_t t = ((int64_t)blockIdx.x - b.block0) * kBS + threadIdx.x;
  double part[kNR] = {0.0, 0.0, 0.0};  // b.b, r.r, sum x
  const int64_t N = a.N;
  const double lam = a.x[N];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Scalars *sc = a.sc;
    sc->done = 0; sc->fail = 0; sc->zero_sol = 0; sc->it_base = 0; sc->iters = 0;
    sc->early[0] = 0; sc->early[1] = 0;
  }
  if (t < b.count) {
    const int64_t i = b.start + t, cnt = b.count;
    const double *w = b.w;
    const double *wP = b.wP;
    const bool wall = (b.type == B_DIR || b.type == B_NEU);
    const double *__restrict__ x = a.x;
    const double *__restrict__ vs = a.vs;
    const int32_t *__restrict__ idx = b.idx;
    const double dt = a.dt;
    double r = 0.0, rhs = 0.0;
    with_width<D>(b.width, [&](auto wc) __attribute__((always_inline)) {
      constexpr int W = decltype(wc)::value;
      double div = 0.0, Ap = 0.0;
#pragma unroll
      for (int j = 0; j < W; ++j) {
        const int32_t nb = idx[(int64_t)j * cnt + t];
        Ap = fma(wP[(int64_t)j * cnt + t], x[nb], Ap);
        if (!wall)
#pragma unroll
          for (int q = 0; q < D; ++q) div = fma(w[((int64_t)q * W + j) * cnt + t], vs[q * N + nb], div);
      }
      if (!wall) rhs = (div / dt) / w[((int64_t)D * W + 0) * cnt + t];
      r = rhs - (Ap + lam);
    });
    a.r[i] = r;
    a.rh[i] = r;
    part[0] = rhs * rhs;
    part[1] = r * r;
    part[2] = x[i];
  }
  block_partials<kNR>(part, a.partR);
}

// ------------------------------------------------------- BiCGSTAB steps --
// Iteration k (k = it_base + it) in two kernels.
//   pv(k): from the s/t partials of iteration k-1: omega = (t,s)/(t,t),
//          r_k = s - omega t, x += alpha p + omega s, rho_k = (rh, r_k),
//          beta = (rho_k/rho_{k-1}) (alpha/omega); then p_k = r_k + beta (p - omega v)
//          formed on the fly at every neighbour, and v_k = A p_k.
//          (k = 0: p_0 = r_0 from the right-hand-side kernel.)
//   st(k): from the p/v partials: convergence test on |r_k|, alpha = rho_k/(rh, v_k);
//          then s = r_k - alpha v_k on the fly and t = A s.
// The border row and column (zero mean, multiplier) are the vectors' slot N.
template <int D>
__global__ __launch_bounds__(kBS) void k_bicg_pv(SimArgs a, int it) {
  Scalars *sc = a.sc;
  if (sc->done) return;
  const int64_t N = a.N, nblk = gridDim.x;
  const int k = sc->it_base + it;
  const int par = it & 1;
  const bool first = (k == 0);
  const double bn = sqrt(sc->bnorm2);
  double omega = 0.0, beta = 0.0, alpha_p = 0.0, rho_k = 0.0, rN, pN;
  int early = 0;
  if (first) {
    double tot[kNR];
    reduce_prev<kNR>(a.partR, nblk, tot);
    rN = -tot[2];                               // border row of r0: 0 - sum x
    rho_k = fma(rN, rN, tot[1]);                // (rh, r0) = |r0|^2
    pN = rN;
    if (tot[0] == 0.0) early = 3;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->bnorm2 = tot[0];
      a.r[N] = rN;
      a.rh[N] = rN;
      a.Pnew[N] = pN;
      sc->rho[par] = rho_k;
      sc->early[par] = early;
    }
    if (early) return;
  } else {
    double tot[kNB];
    reduce_prev<kNB>(a.partB, nblk, tot);
    const double sN = a.S[N], rhN = a.rh[N];
    const double tN = tot[5];                   // border row of t = A s: sum s
    const double ts = fma(tN, sN, tot[0]), tt = fma(tN, tN, tot[1]);
    const double rhs_ = fma(rhN, sN, tot[2]), rht = fma(rhN, tN, tot[3]);
    const double ss = fma(sN, sN, tot[4]);
    alpha_p = sc->alpha[par ^ 1];
    const double rho_p = sc->rho[par ^ 1];
    if (sqrt(ss) <= a.tol * bn) early = 1;
    else if (tt == 0.0) early = 2;
    else {
      omega = ts / tt;
      rho_k = fma(-omega, rht, rhs_);
      if (rho_k == 0.0 || omega == 0.0) early = 2;
      else beta = (rho_k / rho_p) * (alpha_p / omega);
    }
    rN = fma(-omega, tN, sN);
    pN = fma(beta, fma(-omega, a.Vold[N], a.Pold[N]), rN);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->early[par] = early;
      if (early == 1) {
        a.x[N] = fma(alpha_p, a.Pold[N], a.x[N]);
        sc->relres = sqrt(ss) / bn;
      } else if (early == 0) {
        a.x[N] = fma(omega, sN, fma(alpha_p, a.Pold[N], a.x[N]));
        a.r[N] = rN;
        a.Tv[N] = tN;
        a.Pnew[N] = pN;
        sc->rho[par] = rho_k;
      }
    }
    if (early == 2) return;
  }
  const BucketDesc bd = select_bucket(a.tab, blockIdx.x);
  const BScal b{bd.start, bd.count, bd.block0, bd.type, bd.width, bd.idx, static_cast<const double *>(bd.w),
                static_cast<const double *>(bd.aux)};
  const int64_t t = ((int64_t)blockIdx.x - b.block0) * kBS + threadIdx.x;
  const double *__restrict__ r = a.r;
  const double *__restrict__ S = a.S;
  const double *__restrict__ Tv = a.Tv;
  const double *__restrict__ Po = a.Pold;
  const double *__restrict__ Vo = a.Vold;
  if (early == 1) {                             // |s| converged: x += alpha p, nothing else
    if (t < b.count) {
      const int64_t i = b.start + t;
      a.x[i] = fma(alpha_p, Po[i], a.x[i]);
    }
    return;
  }
  double part[kNA] = {0.0, 0.0, 0.0};           // (rh, v), sum p, |r|^2
  if (t < b.count) {
    const int64_t i = b.start + t, cnt = b.count;
    const int32_t *__restrict__ idx = b.idx;
    const double *__restrict__ wP = b.wP;
    double ri;
    if (first) ri = r[i];
    else {
      const double si = S[i];
      a.x[i] = fma(omega, si, fma(alpha_p, Po[i], a.x[i]));
      ri = fma(-omega, Tv[i], si);
      a.r[i] = ri;
    }
    const double pi = first ? ri : fma(beta, fma(-omega, Vo[i], Po[i]), ri);
    double acc = 0.0;
    with_width<D>(b.width, [&](auto wc) __attribute__((always_inline)) {
      constexpr int W = decltype(wc)::value;
#pragma unroll
      for (int j = 0; j < W; ++j) {
        const int32_t nb = idx[(int64_t)j * cnt + t];
        const double pj = first ? r[nb] : fma(beta, fma(-omega, Vo[nb], Po[nb]), fma(-omega, Tv[nb], S[nb]));
        acc = fma(wP[(int64_t)j * cnt + t], pj, acc);
      }
    });
    const double vi = acc + pN;
    a.Pnew[i] = pi;
    a.Vnew[i] = vi;
    part[0] = a.rh[i] * vi;
    part[1] = pi;
    part[2] = ri * ri;
  }
  block_partials<kNA>(part, a.partA);
}

template <int D>
__global__ __launch_bounds__(kBS) void k_bicg_st(SimArgs a, int it) {
  Scalars *sc = a.sc;
  if (sc->done) return;
  const int64_t N = a.N, nblk = gridDim.x;
  const int k = sc->it_base + it;
  const int par = it & 1;
  const int early = sc->early[par];
  if (early) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->done = 1;
      sc->iters = (early == 3) ? 0 : k;
      if (early == 2) sc->fail = 1;
      if (early == 3) { sc->zero_sol = 1; sc->relres = 0.0; }
    }
    return;
  }
  double tot[kNA];
  reduce_prev<kNA>(a.partA, nblk, tot);
  const double bn = sqrt(sc->bnorm2);
  const double vN = tot[1];                     // border row of v = A p: sum p
  const double rN = a.r[N];
  const double rv = fma(a.rh[N], vN, tot[0]);
  const double rr = fma(rN, rN, tot[2]);
  const double relres = sqrt(rr) / bn;
  int stop = 0;
  if (sqrt(rr) <= a.tol * bn) stop = 1;
  else if (k >= a.maxiter) stop = 2;
  else if (rv == 0.0) stop = 3;
  const double alpha = stop ? 0.0 : sc->rho[par] / rv;
  const double sN = fma(-alpha, vN, rN);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->relres = relres;
    if (stop) {
      sc->done = 1;
      sc->iters = k;
      if (stop >= 2) sc->fail = stop == 2 ? 2 : 1;
    } else {
      sc->alpha[par] = alpha;
      a.Vnew[N] = vN;
      a.S[N] = sN;
    }
  }
  if (stop) return;
  const BucketDesc bd = select_bucket(a.tab, blockIdx.x);
  const BScal b{bd.start, bd.count, bd.block0, bd.type, bd.width, bd.idx, static_cast<const double *>(bd.w),
                static_cast<const double *>(bd.aux)};
  const int64_t t = ((int64_t)blockIdx.x - b.block0) * kBS + threadIdx.x;
  double part[kNB] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // (t,s), (t,t), (rh,s), (rh,t), (s,s), sum s
  if (t < b.count) {
    const int64_t i = b.start + t, cnt = b.count;
    const int32_t *__restrict__ idx = b.idx;
    const double *__restrict__ wP = b.wP;
    const double *__restrict__ r = a.r;
    const double *__restrict__ V = a.Vnew;
    double acc = 0.0;
    with_width<D>(b.width, [&](auto wc) __attribute__((always_inline)) {
      constexpr int W = decltype(wc)::value;
#pragma unroll
      for (int j = 0; j < W; ++j) {
        const int32_t nb = idx[(int64_t)j * cnt + t];
        acc = fma(wP[(int64_t)j * cnt + t], fma(-alpha, V[nb], r[nb]), acc);
      }
    });
    const double si = fma(-alpha, V[i], r[i]);
    const double ti = acc + sN;
    const double rhi = a.rh[i];
    a.S[i] = si;
    a.Tv[i] = ti;
    part[0] = ti * si;
    part[1] = ti * ti;
    part[2] = rhi * si;
    part[3] = rhi * ti;
    part[4] = si * si;
    part[5] = si;
  }
  block_partials<kNB>(part, a.partB);
}

// End of a batch of iterations: advance the iteration base and publish a
// summary for the host.
__global__ void k_chunk_end(SimArgs a) {
  if (threadIdx.x != 0) return;
  Scalars *sc = a.sc;
  if (!sc->done) sc->it_base += a.chunk;
  HostFlags &h = sc->mirror;
  h.done = sc->done;
  h.iters = sc->done ? sc->iters : sc->it_base;
  h.fail = sc->fail;
  h.nonfinite = sc->nonfinite;
  h.relres = sc->relres;
  h.pad = 0.0;
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
  DBuf v, vs, T[2], vec[9], partR, partA, partB, sc, wP[kMaxBuckets];
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
  // profiling: events captured around kernels (profile mode)
  hipEvent_t ep_pre[2][3] = {}, ep_kry[2][4] = {}, ep_post[2][3] = {};
  double k_sum_ms[HSM_K_COUNT] = {};
  int64_t k_cnt[HSM_K_COUNT] = {};
  int post_pending = -1;     // parity of a post phase whose events are not read yet
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
    for (auto &row : ep_pre) for (auto &e : row) if (e) (void)hipEventDestroy(e);
    for (auto &row : ep_kry) for (auto &e : row) if (e) (void)hipEventDestroy(e);
    for (auto &row : ep_post) for (auto &e : row) if (e) (void)hipEventDestroy(e);
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
  a.chunk = m->chunk;
  a.v = m->v.as<double>();
  a.vs = m->vs.as<double>();
  a.T = m->T[par].as<double>();
  a.Tn = m->T[par ^ 1].as<double>();
  a.vout = m->v.as<double>();
  a.x = m->x; a.r = m->r; a.rh = m->rh;
  a.Pold = m->P[kpar]; a.Vold = m->V[kpar]; a.Pnew = m->P[kpar ^ 1]; a.Vnew = m->V[kpar ^ 1];
  a.S = m->S; a.Tv = m->Tv;
  a.partR = m->partR.as<double>();
  a.partA = m->partA.as<double>();
  a.partB = m->partB.as<double>();
  a.sc = m->sc.as<Scalars>();
  return a;
}

// Kernel launches of each phase.  `timed` brackets the kernels with HIP
// events (direct launches only: events recorded inside a captured graph
// cannot be timed).
template <int D>
hsm_status enqueue_pre(hsm_sim *m, int par, hipStream_t s, bool timed) {
  SimArgs a = make_args(m, par, 0);
  if (timed) HSM_HIP(hipEventRecord(m->ep_pre[par][0], s));
  hipLaunchKernelGGL(k_predict<D>, dim3((unsigned)m->tab_all.nblocks), dim3(kBS), 0, s, a);
  if (timed) HSM_HIP(hipEventRecord(m->ep_pre[par][1], s));
  hipLaunchKernelGGL(k_rhs<D>, dim3((unsigned)m->tab_all.nblocks), dim3(kBS), 0, s, a);
  if (timed) HSM_HIP(hipEventRecord(m->ep_pre[par][2], s));
  HSM_HIP(hipGetLastError());
  return HSM_OK;
}

// Krylov iterations [it0, it1) of a batch; the ping-pong parity follows the
// iteration number, so a batch may be split across launch paths.
template <int D>
hsm_status enqueue_krylov(hsm_sim *m, int slot, hipStream_t s, int it0, int it1, bool timed, bool flags) {
  const dim3 g((unsigned)m->tab_all.nblocks), b(kBS);
  for (int it = it0; it < it1; ++it) {
    SimArgs a = make_args(m, 0, it & 1);
    const bool tm = timed && it == 0;
    if (tm) HSM_HIP(hipEventRecord(m->ep_kry[slot][0], s));
    hipLaunchKernelGGL(k_bicg_pv<D>, g, b, 0, s, a, it);
    if (tm) HSM_HIP(hipEventRecord(m->ep_kry[slot][1], s));
    hipLaunchKernelGGL(k_bicg_st<D>, g, b, 0, s, a, it);
    if (tm) HSM_HIP(hipEventRecord(m->ep_kry[slot][2], s));
  }
  HSM_HIP(hipGetLastError());
  if (flags) {
    SimArgs a = make_args(m, 0, 0);
    hipLaunchKernelGGL(k_chunk_end, dim3(1), dim3(64), 0, s, a);
    HSM_HIP(hipGetLastError());
    Scalars *sc = m->sc.as<Scalars>();
    HSM_HIP(hipMemcpyAsync(&m->hflags[slot], &sc->mirror, sizeof(HostFlags), hipMemcpyDeviceToHost, s));
  }
  return HSM_OK;
}

template <int D>
hsm_status enqueue_post(hsm_sim *m, int par, hipStream_t s, bool timed) {
  SimArgs a = make_args(m, par, 0);
  if (timed) HSM_HIP(hipEventRecord(m->ep_post[par][0], s));
  hipLaunchKernelGGL(k_correct_heat<D>, dim3((unsigned)m->tab_all.nblocks), dim3(kBS), 0, s, a);
  if (timed) HSM_HIP(hipEventRecord(m->ep_post[par][1], s));
  hipLaunchKernelGGL(k_neumann<D>, dim3((unsigned)m->tab_all.nblocks), dim3(kBS), 0, s, a);
  if (timed) HSM_HIP(hipEventRecord(m->ep_post[par][2], s));
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
  const bool prof = m->prm.profile != 0;
  for (int par = 0; par < 2; ++par) {
    if (!prof) {
      if ((rc = capture(m, m->gr[par], m->g_pre[par], [&] { return enqueue_pre<D>(m, par, m->s, false); }))) return rc;
      if ((rc = capture(m, m->gr[4 + par], m->g_post[par], [&] { return enqueue_post<D>(m, par, m->s, false); })))
        return rc;
    }
    // in profile mode the first iteration of a batch is launched directly (timed); the graph holds the rest
    const int it0 = prof ? 1 : 0;
    if ((rc = capture(m, m->gr[2 + par], m->g_kry[par],
                      [&] { return enqueue_krylov<D>(m, par, m->s, it0, m->chunk, false, true); })))
      return rc;
  }
  m->graphs_ready = true;
  return HSM_OK;
}

// Direct launches (launch_mode 1, or the timed parts of profile mode) and graph replays.
hsm_status do_pre(hsm_sim *m, int par) {
  const bool timed = m->prm.profile != 0;
  if (m->prm.launch_mode == 1 || timed)
    return m->d == 2 ? enqueue_pre<2>(m, par, m->s, timed) : enqueue_pre<3>(m, par, m->s, timed);
  HSM_HIP(hipGraphLaunch(m->g_pre[par], m->s));
  return HSM_OK;
}
hsm_status do_krylov(hsm_sim *m, int slot) {
  const bool timed = m->prm.profile != 0;
  if (m->prm.launch_mode == 1)
    return m->d == 2 ? enqueue_krylov<2>(m, slot, m->s, 0, m->chunk, timed, true)
                     : enqueue_krylov<3>(m, slot, m->s, 0, m->chunk, timed, true);
  if (timed) {
    hsm_status rc = m->d == 2 ? enqueue_krylov<2>(m, slot, m->s, 0, 1, true, false)
                              : enqueue_krylov<3>(m, slot, m->s, 0, 1, true, false);
    if (rc) return rc;
  }
  HSM_HIP(hipGraphLaunch(m->g_kry[slot], m->s));
  return HSM_OK;
}
hsm_status do_post(hsm_sim *m, int par) {
  const bool timed = m->prm.profile != 0;
  if (m->prm.launch_mode == 1 || timed)
    return m->d == 2 ? enqueue_post<2>(m, par, m->s, timed) : enqueue_post<3>(m, par, m->s, timed);
  HSM_HIP(hipGraphLaunch(m->g_post[par], m->s));
  return HSM_OK;
}

hsm_status add_time(hsm_sim *m, int k, hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  HSM_HIP(hipEventElapsedTime(&ms, a, b));
  m->k_sum_ms[k] += ms;
  m->k_cnt[k] += 1;
  return HSM_OK;
}

// post-phase events of an earlier step (complete once later work has synchronised)
hsm_status read_post(hsm_sim *m) {
  if (!m->prm.profile || m->post_pending < 0) return HSM_OK;
  const int p = m->post_pending;
  m->post_pending = -1;
  hsm_status rc;
  if ((rc = add_time(m, HSM_K_CORRECT_HEAT, m->ep_post[p][0], m->ep_post[p][1]))) return rc;
  return add_time(m, HSM_K_NEUMANN, m->ep_post[p][1], m->ep_post[p][2]);
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
    int prev_iters = 0;
    HostFlags f{};
    for (;;) {
      const int nxt = (c + 1) & 1;
      if ((rc = do_krylov(m, nxt))) return rc;             // queued ahead; a no-op once converged
      HSM_HIP(hipEventRecord(m->ev_chunk[nxt], m->s));
      HSM_HIP(hipEventSynchronize(m->ev_chunk[c & 1]));
      f = m->hflags[c & 1];
      if (m->prm.profile) {
        if (c == 0) {
          if ((rc = read_post(m))) return rc;
          if ((rc = add_time(m, HSM_K_PREDICT, m->ep_pre[par][0], m->ep_pre[par][1]))) return rc;
          if ((rc = add_time(m, HSM_K_RHS, m->ep_pre[par][1], m->ep_pre[par][2]))) return rc;
        }
        // the first iteration of this batch did real work only if the count moved past it
        if (f.iters > prev_iters) {
          hipEvent_t *e = m->ep_kry[c & 1];
          if ((rc = add_time(m, HSM_K_BICG_PV, e[0], e[1])) || (rc = add_time(m, HSM_K_BICG_ST, e[1], e[2])))
            return rc;
        }
        prev_iters = f.iters;
      }
      if (f.done || f.nonfinite) break;
      if (++c > max_chunks) { f.fail = 2; break; }
    }
    if ((rc = do_post(m, par))) return rc;
    if (m->prm.profile) m->post_pending = par;
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
  if (prm->profile != 0 && prm->profile != 1) { set_error(HSM_E_INVALID, "profile must be 0 or 1"); return HSM_E_INVALID; }
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
  if ((rc = m->partR.alloc(sizeof(double) * kNR * (m->tab_all.nblocks + 1))) ||
      (rc = m->partA.alloc(sizeof(double) * kNA * (m->tab_all.nblocks + 1))) ||
      (rc = m->partB.alloc(sizeof(double) * kNB * (m->tab_all.nblocks + 1))))
    return rc;
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
  if (prm->profile) {
    for (auto &row : m->ep_pre) for (auto &e : row) HSM_HIP(hipEventCreate(&e));
    for (auto &row : m->ep_kry) for (auto &e : row) HSM_HIP(hipEventCreate(&e));
    for (auto &row : m->ep_post) for (auto &e : row) HSM_HIP(hipEventCreate(&e));
  }
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

hsm_status hsm_sim_kernel_times(hsm_sim *m, double *host_mean_ms, int64_t *host_count) {
  if (!m || !host_mean_ms || !host_count) { set_error(HSM_E_INVALID, "NULL argument"); return HSM_E_INVALID; }
  if (!m->prm.profile) { set_error(HSM_E_INVALID, "simulation was not created with profile = 1"); return HSM_E_INVALID; }
  HSM_HIP(hipStreamSynchronize(m->s));
  hsm_status rc = read_post(m);
  if (rc) return rc;
  for (int k = 0; k < HSM_K_COUNT; ++k) {
    host_mean_ms[k] = m->k_cnt[k] ? m->k_sum_ms[k] / (double)m->k_cnt[k] : 0.0;
    host_count[k] = m->k_cnt[k];
  }
  return HSM_OK;
}

hsm_status hsm_sim_sizes(hsm_sim *m, int64_t *info) {
  if (!m || !info) { set_error(HSM_E_INVALID, "NULL argument"); return HSM_E_INVALID; }
  info[0] = m->N;
  info[1] = m->st->nnz;
  info[2] = m->n_int;
  info[3] = m->n_neu;
  return HSM_OK;
}

void hsm_sim_destroy(hsm_sim *m) { delete m; }

}  // extern "C"
