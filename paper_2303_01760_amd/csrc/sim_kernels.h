// Device code of the time-step driver: the kernels and the device-side
// Krylov state.  Included once, by sim.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <type_traits>

#include "hsm_internal.h"

namespace hsm {
namespace {

constexpr int kBS = 512;   // the largest block of the node kernels (block_nodes; 256 by default)
constexpr int kNR = 3;          // partial sums of the right-hand-side kernel
constexpr int kNA = 3;          // partial sums of the p/v kernel
constexpr int kNB = 6;          // partial sums of the s/t kernel
constexpr int kMaxIterChunk = 256;
constexpr int64_t kSepReduceBlocks = 1024;   // above this grid size, totals come from the reduction kernels
constexpr int kRedThreads = 1024;            // threads of a reduction kernel (one block)
// A regular bucket shares the lattice pressure row when every row deviates
// from it by at most this (the rows are O(1): divided by the centre weight).
// Regular nodes of an exact lattice deviate by rounding only (about 1e-16);
// the classifier admits cross nodes up to 1e-6 h_r off, whose rows then keep
// their own weights.
constexpr double kLatticeRowTol = 1e-12;

// Host-visible summary written once per batch of Krylov iterations.
struct HostFlags {
  int32_t done, iters, fail, nonfinite;
  double relres;
  double node_mv;      // node rows through a pressure matrix-vector product so far this step (per-domain path)
  int32_t nactive;     // blocks the Krylov kernels will run in the next batch (per-domain path)
  int32_t pad;
};

// Krylov state.  Values a kernel computes for iteration k live in slot k & 1,
// so kernels of iteration k never overwrite what their own blocks still read.
struct Scalars {
  double rho[2], alpha[2], omega[2], beta[2];
  double bnorm2, relres;
  double node_mv;      // per-domain path: node rows that went through a Krylov matvec this step
  // the four values every Krylov block reads first, in one 16-byte load
  int32_t nactive;     // per-domain path: entries of SimArgs::active
  int32_t list_sel;    // per-domain path: 0 = every block (SimArgs::lblk0), 1 = SimArgs::lblk1
  int32_t done, it_base;
  int32_t fail, zero_sol, nonfinite;
  int32_t iters, early[2];   // early: 1 = |s| converged, 2 = breakdown, 3 = zero right-hand side
  HostFlags mirror;
};

// Per-domain Krylov state (the reduction-kernel path): every domain runs its
// own BiCGSTAB, with its own scalars and stopping test, in the same launches;
// a block of a finished domain returns at once.  Slot conventions as above.
struct DomState {
  double rho[2], alpha[2], omega[2], beta[2];
  double bnorm2, relres;
  int64_t mv;          // node rows of this domain through a matvec in this solve
  int32_t early[2];    // decided for the iteration of that parity: 1 = |s| converged, 2 = breakdown
  int32_t done, fail, iters, zero_sol;
};

// What a Krylov node kernel of the per-domain path needs of its block's
// domain, written by the reduction kernel before it and read in one 64-byte
// load.  For k_bicg_pv: c = (omega, beta, alpha of the previous iteration,
// c_d times the border entry of p'); for k_bicg_st: c = (alpha, c_d times
// the border entry of s).  done: nothing to do for the domain (finished, or
// its right-hand side is zero); early: as DomState::early.
struct alignas(64) DomLaunch {
  double c[4];
  int32_t done, early;
  int32_t pad[6];
};
static_assert(sizeof(DomLaunch) == 64, "one 64-byte load per block");

// One block of a stepper launch: up to kBS consecutive nodes of one width
// bucket, all of one domain (so a block's partial sums are sums over part of
// one domain).
struct BlockDesc {
  const void *idx;     // the bucket's [width][count] int32 neighbour indices (internal numbering)
  const void *w;       // [nops][width][count] field weights, in the field storage type
  const void *wP;      // [width][count] FP64 pressure-operator rows (divided by the centre weight)
  int64_t bstart;      // the bucket's first node (internal numbering)
  int32_t first;       // this block's first node, counted from bstart
  int32_t nodes;       // nodes in this block (<= kBS)
  int32_t count;       // the bucket's node count: the SoA stride
  int32_t type, width;
  int32_t domain;      // the border row of this block's nodes is N + domain
  int32_t prow;        // row of this block's partial sums: its place in the per-domain block lists,
                       // so each domain's rows are contiguous
  int32_t wshared;     // 1: wP is one row of `width` doubles that every node of the block uses (regular
                       // nodes whose pressure rows all equal the lattice row); 0: wP is [width][count]
};
static_assert(sizeof(BlockDesc) == 64, "one 64-byte scalar load per block");

struct SimArgs {
  const BlockDesc *blk;            // [nblk]
  int64_t nblk;
  int64_t N;
  int32_t K;                       // domains: Krylov vectors hold N + K entries, slot N + k is domain k's border
  const int32_t *dom_blk_off;      // [K+1] per-domain ranges of dom_blk
  const int32_t *dom_blk;          // the blocks of each domain, ascending
  const int64_t *dom_nodes;        // [K] nodes per domain
  const double *bscale;            // [K] c_k = 1/sqrt(nodes of domain k): domain k's border row and column hold c_k
  int32_t *active;                 // [nblk] blocks of unfinished domains (per-domain path), rebuilt as domains finish
  // The Krylov kernels' blocks by list position, descriptors in full: every
  // block in dom_blk order, and the blocks of `active` (copied by
  // k_list_desc after each rebuild).  A workgroup reads both descriptors of
  // its position in the same round as the batch scalars, so the list choice
  // costs no dependent load.  Both hold at least the Krylov grid's entries.
  const BlockDesc *lblk0;
  BlockDesc *lblk1;
  // The Krylov node kernels' own partition of the nodes: blocks of bs / Q
  // nodes for a width with Q lanes per node (lanes_for); per-domain block
  // ranges and lists as for blk.  partA and partB hold one row per such block.
  const BlockDesc *kblk;           // [nkblk]
  int64_t nkblk;
  const int32_t *kdom_blk_off;     // [K+1]
  const int32_t *kdom_blk;
  DomLaunch *lpv, *lst;            // [K] per-domain records for k_bicg_pv and k_bicg_st
  double dt, Ra, Pr, T_ref, tol;
  int32_t maxiter, chunk;
  int32_t xcd_order;   // 1: the Krylov kernels hand each XCD one contiguous run of the block list (list_pos)
  int32_t sepred;      // 1: grid totals (border rows included) come from the reduction kernels;
                       // 0: one domain, each block reduces the partials and handles the border itself
  // fields, in the field storage type (double, or float in the FP32 form)
  const void *v;      // [D][N]
  void *vs;           // [D][N]
  const void *T;      // [N]
  void *Tn;           // [N]
  void *vout;         // [D][N]
  // Krylov vectors, each [N+K]
  double *x, *rh;
  double2 *ST, *PVo, *PVn, *RV;   // pairs (s,t), (p,v) previous/this iteration, (r,v)
  double *partR, *partA, *partB;   // block partial sums [nblk][kN*]
  Scalars *sc;
  DomState *dom;                   // [K] (reduction-kernel path)
};

// The pressure-operator rows of a block: per node (SoA [W][count]), or one
// row shared by every node of the block (read as uniform scalars).  f gets
// std::true_type for the shared row; only the regular width can have one.
template <int D, int W, class F>
__device__ __forceinline__ void with_rows(const BlockDesc &b, F &&f) {
  if constexpr (W == 2 * D + 1) {
    if (b.wshared) {
      f(std::true_type{});
      return;
    }
  }
  f(std::false_type{});
}
template <bool SH>
__device__ __forceinline__ double ld_prow(const BlockDesc &b, uint32_t cnt, int j, uint32_t t) {
  if constexpr (SH) return static_cast<const double *>(b.wP)[j];
  else return ld_soa<double>(b.wP, cnt, j, t);
}

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

// Position in the list of blocks to run that workgroup w takes.  Workgroups
// are dispatched to the XCDs round-robin (w on XCD w % kXcds), and each XCD
// has its own L2: with xcd_order, XCD x takes the contiguous run
// [x C, (x + 1) C) of the list, C = ceil(nact / kXcds), so the neighbours a
// block gathers are mostly in blocks its own L2 has just read; otherwise
// position w (consecutive blocks on different XCDs, all of them sweeping one
// window of the node arrays).  Positions >= nact have nothing to do; the
// grid holds at least kXcds C workgroups.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t list_pos(int64_t w, int64_t nact, int xcd_order) {
  if (!xcd_order) return w;
  const int64_t C = (nact + kXcds - 1) / kXcds, q = w / kXcds;
  return q < C ? (w % kXcds) * C + q : nact;
}

// Field operators of the FP32 form act on differences from the centre value,
// sum_{j>=1} w_j (u_j - u_c): equal to Eq. (1), because the weights of every
// operator (each annihilates constants) sum to zero, but the rounding of an
// FP32 weight then scales with a difference of nearby values rather than with
// the value itself.  That matters where a field is a large smooth part plus a
// small one: the pressure is nearly hydrostatic (its gradient balances the
// buoyancy), and the velocity is what is left after the projection removes
// that balance.  The FP64 form keeps Eq. (1) as written.
template <class FT>
constexpr bool kDiffForm = std::is_same<FT, float>::value;

// Cross-lane moves by DPP (data-parallel primitives: a VALU operand read
// from another lane of the same row of 16), on the two halves of a double.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32));
}
__device__ __forceinline__ double read_lane(double v, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return __builtin_bit_cast(double, (uint64_t)lo | ((uint64_t)hi << 32));
}
// Sum over the 64 lanes of a wave, the same value in every lane: swap
// neighbours, then pairs (quad_perm), mirror within 8 and within 16 lanes
// (each step adds two equal-sized partial sums, and a + b == b + a, so every
// lane of a row holds the identical row sum), then the four row sums in a
// fixed order.  Fixed order throughout: deterministic.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);   // row_half_mirror
  v += dpp_mov<0x140>(v);   // row_mirror
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Lanes that share one node's stencil in the Krylov node kernels (and the
// host's partition of their blocks): one for the regular width, whose
// lattice row may be one row shared by the block (read as uniform values);
// otherwise the fewest, a power of two up to 16, that leave each lane at most
// kLaneEntries entries.  A wide stencil's gather is then one round of loads
// per lane instead of a chain of chunks, each waiting for the last.  (At
// most 4, 6 and 8 entries a lane were measured; 8 was fastest in 2D and 3D.)
constexpr int kLaneEntries = 8;   // most stencil entries a lane takes
__host__ __device__ constexpr int lanes_for(int W, int D) {
  if (W == 2 * D + 1) return 1;
  int q = 1;
  while (q < 16 && (W + q - 1) / q > kLaneEntries) q *= 2;
  return q;
}

// Sum over each aligned group of Q lanes (Q a power of two up to 16, the
// same in every lane), the same value in every lane of the group, added in a
// fixed order.  Every lane of the wave must be active.
__device__ __forceinline__ double lane_sum(double v, int Q) {
  if (Q >= 2) v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
  if (Q >= 4) v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
  if (Q >= 8) v += dpp_mov<0x141>(v);   // row_half_mirror
  if (Q >= 16) v += dpp_mov<0x140>(v);  // row_mirror
  return v;
}

// Deterministic block sum of NQ values (wave sums, then the waves in order);
// the first NQ threads write the block's partials.  No fences or atomics:
// the consumer is a later kernel.
template <int NQ>
__device__ __forceinline__ void block_partials(double (&v)[NQ], double *part, int64_t row = -1, bool again = false) {
  __shared__ double red[kBS / 64][NQ];
  const int wv = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);   // blocks of 64 to kBS threads
#pragma unroll
  for (int q = 0; q < NQ; ++q) v[q] = wave_sum(v[q]);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) red[wv][q] = v[q];
  __syncthreads();
  if (threadIdx.x < NQ) {
    const int q = threadIdx.x;
    double s = red[0][q];
    for (int k = 1; k < nw; ++k) s += red[k][q];
    part[(row < 0 ? (int64_t)blockIdx.x : row) * NQ + q] = s;
  }
  if (again) __syncthreads();                  // the shared array is reused by this block's next row
}

// Grid totals of a previous kernel's block partials, reduced by every block
// (and every thread of it) in the same fixed order, so all hold bit-identical
// totals.
template <int NQ>
__device__ __forceinline__ void reduce_prev(const double *__restrict__ part, int64_t nblk, double (&tot)[NQ]) {
  __shared__ double red[kBS / 64][NQ];
  const int64_t bs = blockDim.x;               // 64 to kBS threads
  // all loads of the first four passes issued before any sum (same order as a plain loop)
  constexpr int U = 4;
  double vals[U][NQ];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t b = threadIdx.x + (int64_t)u * bs;
#pragma unroll
    for (int q = 0; q < NQ; ++q) vals[u][q] = (b < nblk) ? part[b * NQ + q] : 0.0;
  }
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    acc[q] = vals[0][q];
#pragma unroll
    for (int u = 1; u < U; ++u) acc[q] += vals[u][q];
  }
  for (int64_t b = threadIdx.x + (int64_t)U * bs; b < nblk; b += bs)
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] += part[b * NQ + q];
  const int wv = threadIdx.x >> 6, nw = (int)(bs >> 6);
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = wave_sum(acc[q]);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) red[wv][q] = acc[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double s = red[0][q];
    for (int k = 1; k < nw; ++k) s += red[k][q];
    tot[q] = s;
  }
}

// ------------------------------------------------------ reduction kernels --
// The per-domain reductions run as a grid over domains: G waves of a
// kRedThreads block sum one domain's block partials (G = 16 for one domain,
// down to 1 for sixteen or more domains, sixteen to a block).  Lanes stride
// over the domain's partial rows (contiguous: BlockDesc::prow), a DPP wave
// sum folds the lanes and the G wave sums are added in order: a fixed
// order, so the totals are deterministic.  Each domain's update touches
// only its own state, so the blocks need no fences or atomics between them:
// with several domains, the batch flags and the list of unfinished domains'
// blocks are gathered once per batch of iterations (k_chunk_end); with one
// domain (one block) they are published at once.
constexpr int kRedWaves = kRedThreads / 64;

// Waves per domain for K domains.
__host__ __device__ constexpr int red_group(int K) {
  int p = 1;
  while (p < K && p < kRedWaves) p <<= 1;
  return kRedWaves / p;
}
// Blocks of a reduction launch.
inline int64_t red_grid(int K) {
  const int dpb = kRedWaves / red_group(K);
  return (K + dpb - 1) / dpb;
}

struct RedSlot {
  int d;         // this wave's domain (>= K: none)
  int g;         // this wave's share of it, 0 .. G-1
  bool lead;     // the thread that updates the domain: share 0, lane 0
};
__device__ __forceinline__ RedSlot red_slot(int K) {
  const int G = red_group(K), wv = threadIdx.x >> 6;
  RedSlot r;
  r.d = (int)blockIdx.x * (kRedWaves / G) + wv / G;
  r.g = wv % G;
  r.lead = r.g == 0 && (threadIdx.x & 63) == 0 && r.d < K;
  return r;
}

// Totals of domain r.d's block partials (its rows [j0, j1)), valid in the
// lead thread.  `need` is the same in every lane of a wave.  Every thread of
// the block calls it.
template <int NQ>
__device__ __forceinline__ void domain_sums(const SimArgs &a, const double *__restrict__ part, const RedSlot &r,
                                            bool need, int j0, int j1, double (&tot)[NQ]) {
  __shared__ double red[kRedWaves][NQ];
  const int G = red_group(a.K), wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  if (need) {
    // four passes' loads issued before their sums (rows past the end read
    // as 0.0, which leaves every sum unchanged)
    constexpr int U = 4;
    const int step = G * 64;
    for (int j = j0 + r.g * 64 + lane; j < j1; j += U * step) {
      double vals[U][NQ];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool in = j + u * step < j1;
        const int64_t row = in ? (int64_t)(j + u * step) : (int64_t)j;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const double x = part[row * NQ + q];
          vals[u][q] = in ? x : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] += vals[u][q];
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = wave_sum(acc[q]);
  }
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) red[wv][q] = acc[q];
  __syncthreads();
  if (r.lead)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double t = red[wv][q];
      for (int k = 1; k < G; ++k) t += red[wv + k][q];
      tot[q] = t;
    }
}

struct BatchFlags {
  int32_t ndone, fail, iters;
  unsigned long long relres_bits;   // non-negative doubles order like their bit patterns
  unsigned long long mv;            // node rows through a matvec (integer sum: order-free)
};
__device__ __forceinline__ void batch_begin(BatchFlags &f) {
  if (threadIdx.x == 0) { f.ndone = 0; f.fail = 0; f.iters = 0; f.relres_bits = 0ull; f.mv = 0ull; }
  __syncthreads();
}
__device__ __forceinline__ void batch_add(BatchFlags &f, const DomState &ds) {
  if (ds.done) atomicAdd(&f.ndone, 1);
  if (ds.fail) atomicMax(&f.fail, ds.fail);
  atomicMax(&f.iters, ds.iters);
  atomicMax(&f.relres_bits, (unsigned long long)__double_as_longlong(ds.relres));
  atomicAdd(&f.mv, (unsigned long long)ds.mv);
}
// Thread 0 publishes the flags of every domain (every domain done: the
// batch is done); node_mv is this solve's running total.
__device__ __forceinline__ void batch_end(const SimArgs &a, BatchFlags &f) {
  __syncthreads();
  if (threadIdx.x == 0) {
    Scalars *sc = a.sc;
    sc->relres = __longlong_as_double((long long)f.relres_bits);
    sc->node_mv = (double)f.mv;
    if (f.ndone == a.K) {
      sc->done = 1;
      sc->iters = f.iters;
      sc->fail = f.fail;
    }
  }
}

// The list of blocks of unfinished domains, domain by domain in order (a
// block-wide scan of their block counts), for the per-domain Krylov kernels.
__device__ __forceinline__ void build_active(const SimArgs &a) {
  __shared__ int32_t scan[kRedThreads];
  __shared__ int32_t carry;
  const int tid = threadIdx.x;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int d0 = 0; d0 < a.K; d0 += kRedThreads) {
    const int d = d0 + tid;
    const int c = (d < a.K && !a.dom[d].done) ? a.kdom_blk_off[d + 1] - a.kdom_blk_off[d] : 0;
    scan[tid] = c;
    __syncthreads();
    for (int off = 1; off < kRedThreads; off <<= 1) {
      const int v = tid >= off ? scan[tid - off] : 0;
      __syncthreads();
      scan[tid] += v;
      __syncthreads();
    }
    // entry e of this chunk belongs to the first domain whose inclusive
    // count exceeds e
    const int total = scan[kRedThreads - 1], base = carry;
    for (int e = tid; e < total; e += kRedThreads) {
      int lo = 0, hi = kRedThreads - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (scan[mid] > e) hi = mid;
        else lo = mid + 1;
      }
      const int before = lo > 0 ? scan[lo - 1] : 0;
      a.active[base + e] = a.kdom_blk[a.kdom_blk_off[d0 + lo] + (e - before)];
    }
    __syncthreads();
    if (tid == 0) carry = base + total;
    __syncthreads();
  }
  if (tid == 0) {
    a.sc->nactive = carry;
    a.sc->list_sel = 1;
  }
}

// After the right-hand-side kernel, per domain: |b|^2; the border row of r0
// (0 - sum x over the domain: the border unknowns are the multipliers, whose
// rows have right-hand side 0); r^ = r0; rho_0 = |r0|^2.  A domain with a zero
// right-hand side is done at once with p = 0.
__global__ __launch_bounds__(kRedThreads) void k_reduce_r(SimArgs a) {
  __shared__ BatchFlags f;
  const bool one = a.K == 1;
  if (one) batch_begin(f);
  const int64_t N = a.N;
  const RedSlot rs = red_slot(a.K);
  const int d = rs.d;
  const int j0 = d < a.K ? a.dom_blk_off[d] : 0, j1 = d < a.K ? a.dom_blk_off[d + 1] : 0;
  const double cb = d < a.K ? a.bscale[d] : 0.0;
  double tot[kNR];
  domain_sums<kNR>(a, a.partR, rs, d < a.K, j0, j1, tot);
  if (rs.lead) {
    DomState &ds = a.dom[d];
    const double r = -(cb * tot[2]);
    a.RV[N + d] = make_double2(r, 0.0);
    a.rh[N + d] = r;
    const double rr = fma(r, r, tot[1]);
    ds.bnorm2 = tot[0];
    ds.rho[0] = rr;
    ds.early[0] = 0;
    ds.fail = 0;
    ds.iters = 0;
    ds.mv = 0;
    ds.zero_sol = tot[0] == 0.0;
    ds.done = ds.zero_sol;
    ds.relres = ds.zero_sol ? 0.0 : sqrt(rr / tot[0]);
    DomLaunch L{};
    L.c[3] = cb * r;                            // p0 = r0 on the border row
    L.done = ds.done;
    a.lpv[d] = L;
    L.c[3] = 0.0;
    a.lst[d] = L;
    if (one) batch_add(f, ds);
  }
  if (one) batch_end(a, f);
}

// After k_bicg_pv(it), per unfinished domain: the border rows of iteration
// k = it_base + it (r = s - omega t, x += alpha_prev p + omega s,
// p' = r + beta (p - omega v); k = 0: r from k_reduce_r, p' = r), then
// v' = sum_{i in d} p'_i; stores (p', v') and (r, v').  Then the stopping
// test on |r| and alpha = rho / (r^, v').  A domain whose |s| converged
// (early 1) only takes x += alpha_prev p on its border and is done; a
// breakdown (early 2) ends it as failed.
__global__ __launch_bounds__(kRedThreads) void k_reduce_a(SimArgs a, int it) {
  Scalars *sc = a.sc;
  const int par = it & 1;
  const int64_t N = a.N;
  const RedSlot rs = red_slot(a.K);
  const int d = rs.d;
  const bool has = d < a.K;
  // every load that depends on nothing else first (one round): the batch
  // state, the domain's state and block range, and the lead's border rows
  // and scalars, which it uses once the partials are summed
  const int all_done = sc->done, it_base = sc->it_base;
  int dd = 1, e = 0, j0 = 0, j1 = 0;
  if (has) {
    dd = a.dom[d].done;
    e = a.dom[d].early[par];
    j0 = a.kdom_blk_off[d];
    j1 = a.kdom_blk_off[d + 1];
  }
  double alpha_p = 0.0, omega = 0.0, beta = 0.0, bnorm2 = 0.0, rho = 0.0, xb = 0.0, rhb = 0.0;
  double2 rvb = make_double2(0.0, 0.0), stb = rvb, pvb = rvb;
  int64_t nodes = 0;
  double cb = 0.0;
  if (rs.lead) {
    const DomState &ds = a.dom[d];
    cb = a.bscale[d];
    alpha_p = ds.alpha[par ^ 1]; omega = ds.omega[par]; beta = ds.beta[par];
    bnorm2 = ds.bnorm2; rho = ds.rho[par];
    xb = a.x[N + d]; rhb = a.rh[N + d];
    rvb = a.RV[N + d]; stb = a.ST[N + d]; pvb = a.PVo[N + d];
    nodes = a.dom_nodes[d];
  }
  if (all_done) return;
  __shared__ BatchFlags f;
  const bool one = a.K == 1;
  if (one) batch_begin(f);
  const int k = it_base + it;
  const bool live = has && !dd;
  if (!live || k == 0) e = 0;
  double tot[kNA];
  domain_sums<kNA>(a, a.partA, rs, live && e == 0, j0, j1, tot);
  if (rs.lead) {
    DomState &ds = a.dom[d];
    if (live) {
      if (e == 1) {
        a.x[N + d] = fma(alpha_p, pvb.x, xb);
        ds.done = 1;
        ds.iters = k;
      } else if (e == 2) {
        ds.done = 1;
        ds.fail = 1;
        ds.iters = k;
      } else {
        // (the launch records are written below, from the outcome)
        ds.mv += nodes;                         // k_bicg_pv's matvec on this domain
        double r, p;
        if (k == 0) {
          r = rvb.x;
          p = r;
        } else {
          a.x[N + d] = fma(omega, stb.x, fma(alpha_p, pvb.x, xb));
          r = fma(-omega, stb.y, stb.x);
          p = fma(beta, fma(-omega, pvb.y, pvb.x), r);
        }
        const double vb = cb * tot[1];          // border row of v = A p': c_d sum of p' over the domain
        a.PVn[N + d] = make_double2(p, vb);
        a.RV[N + d] = make_double2(r, vb);
        const double rv = fma(rhb, vb, tot[0]);
        const double rr = fma(r, r, tot[2]);
        const double bn = sqrt(bnorm2);
        ds.relres = sqrt(rr) / bn;
        if (sqrt(rr) <= a.tol * bn) { ds.done = 1; ds.iters = k; }
        else if (k >= a.maxiter) { ds.done = 1; ds.fail = 2; ds.iters = k; }
        else if (rv == 0.0) { ds.done = 1; ds.fail = 1; ds.iters = k; }
        else {
          ds.alpha[par] = rho / rv;
          ds.mv += nodes;                       // k_bicg_st's matvec follows
          DomLaunch L{};
          L.c[0] = ds.alpha[par];
          L.c[1] = cb * fma(-ds.alpha[par], vb, r);   // c_d times the border entry of s = r - alpha v
          a.lst[d] = L;
        }
      }
      if (ds.done) {                            // no more node work for this domain in this solve
        a.lst[d].done = 1;
        a.lpv[d].done = 1;
      }
    }
    if (one) batch_add(f, ds);
  }
  if (one) batch_end(a, f);
}

// After k_bicg_st(it), per unfinished domain: s = r - alpha v and
// t = sum_{i in d} s_i on the border row (stored as (s, t)); then, for the
// next iteration: |s| converged (early 1), breakdown (early 2), or
// omega = (t,s)/(t,t), rho' = (r^,s) - omega (r^,t), beta = (rho'/rho)(alpha/omega).
__global__ __launch_bounds__(kRedThreads) void k_reduce_b(SimArgs a, int it) {
  Scalars *sc = a.sc;
  const int par = it & 1, nx = par ^ 1;
  const int64_t N = a.N;
  const RedSlot rs = red_slot(a.K);
  const int d = rs.d;
  const bool has = d < a.K;
  // independent loads first, as in k_reduce_a
  const int all_done = sc->done;
  int dd = 1, j0 = 0, j1 = 0;
  if (has) {
    dd = a.dom[d].done;
    j0 = a.kdom_blk_off[d];
    j1 = a.kdom_blk_off[d + 1];
  }
  double alpha = 0.0, rho = 0.0, bnorm2 = 0.0, rhb = 0.0, cb = 0.0;
  double2 rv = make_double2(0.0, 0.0), pvb = rv;
  if (rs.lead) {
    const DomState &ds = a.dom[d];
    cb = a.bscale[d];
    alpha = ds.alpha[par]; rho = ds.rho[par]; bnorm2 = ds.bnorm2;
    rv = a.RV[N + d];
    rhb = a.rh[N + d];
    pvb = a.PVn[N + d];                         // (p', v) of the border, stored by k_reduce_a
  }
  if (all_done) return;
  const bool live = has && !dd;
  double tot[kNB];
  domain_sums<kNB>(a, a.partB, rs, live, j0, j1, tot);
  if (!(rs.lead && live)) return;
  DomState &ds = a.dom[d];
  const double sb = fma(-alpha, rv.y, rv.x), tb = cb * tot[5];   // border row of t = A s: c_d sum s
  a.ST[N + d] = make_double2(sb, tb);
  const double ts = fma(tb, sb, tot[0]), tt = fma(tb, tb, tot[1]);
  const double rhs_ = fma(rhb, sb, tot[2]), rht = fma(rhb, tb, tot[3]);
  const double ss = fma(sb, sb, tot[4]);
  const double bn = sqrt(bnorm2);
  int e = 0;
  double omega = 0.0, beta = 0.0, rho_n = 0.0;
  if (sqrt(ss) <= a.tol * bn) { e = 1; ds.relres = sqrt(ss) / bn; }
  else if (tt == 0.0) e = 2;
  else {
    omega = ts / tt;
    rho_n = fma(-omega, rht, rhs_);
    if (rho_n == 0.0 || omega == 0.0) e = 2;
    else beta = (rho_n / rho) * (alpha / omega);
  }
  ds.early[nx] = e;
  ds.omega[nx] = omega;
  ds.beta[nx] = beta;
  ds.rho[nx] = rho_n;
  // the next k_bicg_pv's record (its border entry of p', as k_reduce_a will store it)
  DomLaunch L{};
  L.c[0] = omega;
  L.c[1] = beta;
  L.c[2] = alpha;
  L.c[3] = cb * fma(beta, fma(-omega, pvb.y, pvb.x), fma(-omega, tb, sb));
  L.early = e;
  a.lpv[d] = L;
}

// ------------------------------------------------------------- predictor --
// v* = v + dt (-(v.grad) v + Pr lap v - Ra Pr g (T - T_ref)) at interior nodes
// (Eq. (2) with the pressure term left out: Chorin's splitting, Section 3);
// 0 at walls.  FT: field and weight storage (double, or float with Dot2
// applies); the pointwise update is in FP64.
template <int D, class FT>
__global__ __launch_bounds__(kBS) void k_predict(SimArgs a) {
  const BlockDesc b = a.blk[blockIdx.x];
  const int64_t t = b.first + (int64_t)threadIdx.x;
  const bool live = (int)threadIdx.x < b.nodes;
  if (!live) return;
  const int64_t N = a.N, i = b.bstart + t;
  FT *__restrict__ vs = static_cast<FT *>(a.vs);
  if (b.type == B_DIR || b.type == B_NEU) {
#pragma unroll
    for (int c = 0; c < D; ++c) vs[c * N + i] = FT(0);
    return;
  }
  const FT *__restrict__ v = static_cast<const FT *>(a.v);
  const uint32_t cnt32 = (uint32_t)b.count, t32 = (uint32_t)t;
  Buf vb[D];
#pragma unroll
  for (int c = 0; c < D; ++c) vb[c] = plane(v, N, c);
  const double Ti = (double)static_cast<const FT *>(a.T)[i], Tref = a.T_ref, Ra = a.Ra, Pr = a.Pr, dt = a.dt;
  using AccT = FieldAcc<FT>;
  constexpr bool kDiff = kDiffForm<FT>;
  with_width<D>(b.width, [&](auto wc) __attribute__((always_inline)) {
    constexpr int W = decltype(wc)::value;
    AccT g[D][D], L[D];
    FT uc[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      L[c].init();
      uc[c] = FT(0);
#pragma unroll
      for (int q = 0; q < D; ++q) g[c][q].init();
    }
    gather_chunks<W>(
        b.idx, cnt32, t32,
        [&](int j) __attribute__((always_inline)) {
          Pack<FT, D + 1> r;
#pragma unroll
          for (int q = 0; q <= D; ++q) r.v[q] = (kDiff && j == 0) ? FT(0) : ld_soa<FT>(b.w, cnt32, q * W + j, t32);
          return r;
        },
        [&](int32_t nb) __attribute__((always_inline)) {
          Pack<FT, D> r;
#pragma unroll
          for (int c = 0; c < D; ++c) r.v[c] = ld_at<FT>(vb[c], nb);
          return r;
        },
        [&](int j, const Pack<FT, D + 1> &wq, const Pack<FT, D> &u) __attribute__((always_inline)) {
          if (kDiff && j == 0) {
#pragma unroll
            for (int c = 0; c < D; ++c) uc[c] = u.v[c];
            return;
          }
#pragma unroll
          for (int c = 0; c < D; ++c) {
            const FT du = kDiff ? FT(u.v[c] - uc[c]) : u.v[c];
#pragma unroll
            for (int q = 0; q < D; ++q) g[c][q].add(wq.v[q], du);
            L[c].add(wq.v[D], du);
          }
        },
        [&]() __attribute__((always_inline)) {
#pragma unroll
          for (int c = 0; c < D; ++c) {
            L[c].settle();
#pragma unroll
            for (int q = 0; q < D; ++q) g[c][q].settle();
          }
        });
    double vi[D];
#pragma unroll
    for (int q = 0; q < D; ++q) vi[q] = (double)v[q * N + i];
    const double buoy = (Ra * Pr) * (Ti - Tref);
#pragma unroll
    for (int c = 0; c < D; ++c) {
      double adv = vi[0] * g[c][0].get_d();
#pragma unroll
      for (int q = 1; q < D; ++q) adv = fma(vi[q], g[c][q].get_d(), adv);
      double f = fma(Pr, L[c].get_d(), -adv);
      if (c == D - 1) f += buoy;
      vs[c * N + i] = (FT)fma(dt, f, vi[c]);
    }
  });
}

// ---------------------------------------- pressure rhs + initial residual --
// b = div(v*)/dt / diag at interior nodes, 0 at walls; r0 = b - A x; rh = r0.
// The divergence is a field apply (FT); the pressure operator is FP64.
template <int D, class FT>
__global__ __launch_bounds__(kBS) void k_rhs(SimArgs a) {
  const BlockDesc b = a.blk[blockIdx.x];
  const int64_t t = b.first + (int64_t)threadIdx.x;
  const bool live = (int)threadIdx.x < b.nodes;
  double part[kNR] = {0.0, 0.0, 0.0};  // b.b, r.r, sum x
  const int64_t N = a.N;
  const double lam = a.bscale[b.domain] * a.x[N + b.domain];   // c_d times this domain's border multiplier
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Scalars *sc = a.sc;
    sc->done = 0; sc->fail = 0; sc->zero_sol = 0; sc->it_base = 0; sc->iters = 0; sc->node_mv = 0.0;
    sc->early[0] = 0; sc->early[1] = 0;
    sc->list_sel = 0;                           // a new solve starts from every block
    sc->nactive = (int32_t)a.nkblk;           // the Krylov kernels' list: every block
  }
  if (live) {
    const int64_t i = b.bstart + t;
    const uint32_t cnt32 = (uint32_t)b.count, t32 = (uint32_t)t;
    const bool wall = (b.type == B_DIR || b.type == B_NEU);
    const double *__restrict__ x = a.x;
    const Buf xb = plane(a.x, N + 1, 0);
    Buf vsb[D];
#pragma unroll
    for (int q = 0; q < D; ++q) vsb[q] = plane(static_cast<const FT *>(a.vs), N, q);
    const double dt = a.dt;
    double r = 0.0, rhs = 0.0;
    using AccT = FieldAcc<FT>;
    constexpr bool kDiff = kDiffForm<FT>;
    with_width<D>(b.width, [&](auto wc) __attribute__((always_inline)) {
      constexpr int W = decltype(wc)::value;
      with_rows<D, W>(b, [&](auto sh) __attribute__((always_inline)) {
      constexpr bool SH = decltype(sh)::value;
      double Ap = 0.0;
      AccT div;
      div.init();
      FT uc[D];
#pragma unroll
      for (int q = 0; q < D; ++q) uc[q] = FT(0);
      gather_chunks<W>(
          b.idx, cnt32, t32,
          [&](int j) __attribute__((always_inline)) {
            Pack<double, 1> wp;
            wp.v[0] = ld_prow<SH>(b, cnt32, j, t32);
            Pack<FT, D> wd;
#pragma unroll
            for (int q = 0; q < D; ++q)   // unused at walls
              wd.v[q] = (kDiff && j == 0) ? FT(0) : ld_soa<FT>(b.w, cnt32, q * W + j, t32);
            return Pack2<double, 1, FT, D>{wp, wd};
          },
          [&](int32_t nb) __attribute__((always_inline)) {
            Pack<double, 1> xp;
            xp.v[0] = ld_at<double>(xb, nb);
            Pack<FT, D> u;
#pragma unroll
            for (int q = 0; q < D; ++q) u.v[q] = ld_at<FT>(vsb[q], nb);
            return Pack2<double, 1, FT, D>{xp, u};
          },
          [&](int j, const Pack2<double, 1, FT, D> &wq, const Pack2<double, 1, FT, D> &u)
              __attribute__((always_inline)) {
                Ap = fma(wq.a.v[0], u.a.v[0], Ap);
                if (kDiff && j == 0) {
#pragma unroll
                  for (int q = 0; q < D; ++q) uc[q] = u.b.v[q];
                } else if (!wall) {
#pragma unroll
                  for (int q = 0; q < D; ++q) div.add(wq.b.v[q], kDiff ? FT(u.b.v[q] - uc[q]) : u.b.v[q]);
                }
              },
          [&]() __attribute__((always_inline)) { pin(Ap); div.settle(); });
      if (!wall) rhs = (div.get_d() / dt) / (double)ld_soa<FT>(b.w, cnt32, D * W, t32);
      r = rhs - (Ap + lam);
      });
    });
    a.RV[i] = make_double2(r, 0.0);
    a.rh[i] = r;
    part[0] = rhs * rhs;
    part[1] = r * r;
    part[2] = x[i];
  }
  block_partials<kNR>(part, a.partR, b.prow);
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
// Vectors gathered together are stored as pairs, one 16-byte load per
// neighbour: (s, t), (p, v) (two generations) and (r, v).  The border row
// and column (zero mean, multiplier) are slot N of every vector.
// The node rows of one block of k_bicg_pv (cpN: c_d times the border entry of
// p'), Q threads per node (Q = lanes_for(width) with LN, else 1; uniform in
// the block).  The node's own values are loaded first and used only once the
// neighbour loads are in flight (the gather's hook), so the block's loads go
// out in one round; the stores come last, from the node's first lane.  Only
// the gather is compiled per width.
template <int D, int KP, bool LN>
__device__ __forceinline__ void pv_rows(const SimArgs &a, const BlockDesc &b, bool again, bool first,
                                        int early, double omega, double beta, double alpha_p, double cpN) {
  const int64_t N = a.N;
  const double2 *__restrict__ ST = a.ST;
  const double2 *__restrict__ PVo = a.PVo;
  const double2 *__restrict__ RV = a.RV;
  const int Q = LN ? lanes_for(b.width, D) : 1;
  const int node = (int)threadIdx.x >> __builtin_ctz((unsigned)Q);
  const int sub = (int)threadIdx.x & (Q - 1);
  const int64_t t = b.first + (int64_t)node;
  const bool live = node < b.nodes;
  const bool lead = live && sub == 0;
  const int64_t i = b.bstart + t;
  if (early == 1) {                             // |s| converged: x += alpha p, nothing else
    if (lead) a.x[i] = fma(alpha_p, PVo[i].x, a.x[i]);
    return;
  }
  double2 sti = make_double2(0.0, 0.0), pvi = sti;
  double xi = 0.0, rhi = 0.0;
  if (live) {
    if (first) {
      sti = RV[i];                              // (r0, .)
    } else {
      sti = ST[i];
      pvi = PVo[i];
      xi = a.x[i];
    }
    rhi = a.rh[i];
  }
  double ri = 0.0, pi = 0.0, xn = 0.0, acc = 0.0;
  const auto own = [&]() __attribute__((always_inline)) {
    if (first) {
      ri = sti.x;
      pi = ri;
    } else {
      xn = fma(omega, sti.x, fma(alpha_p, pvi.x, xi));
      ri = fma(-omega, sti.y, sti.x);
      pi = fma(beta, fma(-omega, pvi.y, pvi.x), ri);
    }
  };
  if (live) {
    const uint32_t cnt32 = (uint32_t)b.count, t32 = (uint32_t)t;
    const Buf RVb = plane(RV, N + 1, 0), STb = plane(ST, N + 1, 0), PVb = plane(PVo, N + 1, 0);
    with_width<D>(b.width, [&](auto wc) __attribute__((always_inline)) {
      constexpr int W = decltype(wc)::value;
      constexpr int QW = LN ? lanes_for(W, D) : 1;
      with_rows<D, W>(b, [&](auto sh) __attribute__((always_inline)) {
        constexpr bool SH = decltype(sh)::value;
        const auto wl = [&](int j) __attribute__((always_inline)) {
          if constexpr (QW == 1) return ld_prow<SH>(b, cnt32, j, t32);
          else return static_cast<const double *>(b.wP)[(uint64_t)j * cnt32 + t32];
        };
        if (first) {
          gather_lanes<W, QW, 12>(
              b.idx, cnt32, t32, sub, wl,
              [&](int32_t nb) __attribute__((always_inline)) { return ld_at<double>(RVb, 2 * nb); },
              [&](int, double wj, double rj) __attribute__((always_inline)) { acc = fma(wj, rj, acc); },
              [&]() __attribute__((always_inline)) { pin(acc); }, own);
        } else {
          gather_lanes<W, QW, KP>(
              b.idx, cnt32, t32, sub, wl,
              [&](int32_t nb) __attribute__((always_inline)) {
                return Pack<double2, 2>{{ld_at<double2>(STb, nb), ld_at<double2>(PVb, nb)}};
              },
              [&](int, double wj, const Pack<double2, 2> &g) __attribute__((always_inline)) {
                const double pj = fma(beta, fma(-omega, g.v[1].y, g.v[1].x), fma(-omega, g.v[0].y, g.v[0].x));
                acc = fma(wj, pj, acc);
              },
              [&]() __attribute__((always_inline)) { pin(acc); }, own);
        }
      });
    });
  }
  if (LN) acc = lane_sum(acc, Q);
  double part[kNA] = {0.0, 0.0, 0.0};           // (rh, v), sum p, |r|^2
  if (lead) {
    if (!first) a.x[i] = xn;
    const double vi = acc + cpN;                // + c_d times the border entry of p'
    a.PVn[i] = make_double2(pi, vi);
    a.RV[i] = make_double2(ri, vi);
    part[0] = rhi * vi;
    part[1] = pi;
    part[2] = ri * ri;
  }
  block_partials<kNA>(part, a.partA, b.prow, again);
}

// The descriptor of list position w's block: the Krylov kernels of the
// per-domain path give each workgroup one position (directly, or in the
// XCD-contiguous order, which needs the list length first).  Returns false
// for a position past the list.
__device__ __forceinline__ bool listed_block(const SimArgs &a, int64_t w, int nact, int lsel, BlockDesc &b) {
  // both descriptors of position w, loaded with the batch scalars (no branch
  // before them, so no dependent round); w is below both arrays' length
  const BlockDesc b0 = a.lblk0[w], b1 = a.lblk1[w];
  b = lsel ? b1 : b0;
  if (!a.xcd_order) return w < nact;
  const int64_t v = list_pos(w, nact, 1);
  if (v >= nact) return false;
  b = lsel ? a.lblk1[v] : a.lblk0[v];
  return true;
}

// A domain's launch record as one 16-dword load (its fields are then in the
// same round of loads, whichever of them a test uses first).
__device__ __forceinline__ DomLaunch load_launch(const DomLaunch *p) {
  typedef int32_t v16 __attribute__((ext_vector_type(16)));
  const v16 v = *reinterpret_cast<const v16 *>(p);
  DomLaunch L;
  __builtin_memcpy(&L, &v, sizeof(L));
  return L;
}

// Node t's stencil gather, shared by Q lanes: lane `sub` takes entries sub,
// sub + Q, ... (the last round leaves lanes idle where Q does not divide W;
// their index and weight are not loaded and they add nothing).  Indices and
// weights are plain global loads (an entry's plane varies across lanes); all
// of a lane's neighbour loads go out in one round, then hook(), then use()
// in entry order.  Q == 1: gather_chunks.
template <int W, int Q, int K, class FW, class FV, class FU, class FS, class FH>
__device__ __forceinline__ void gather_lanes(const void *idx, uint32_t cnt, uint32_t t, int sub, FW &&wload,
                                             FV &&vload, FU &&use, FS &&settle, FH &&hook) {
  if constexpr (Q == 1) {
    gather_chunks<W, K>(idx, cnt, t, wload, vload, use, settle, hook);
  } else {
    constexpr int E = (W + Q - 1) / Q;
    const int last = W - (E - 1) * Q;           // lanes with an entry in the last round
    const int32_t *__restrict__ ix = static_cast<const int32_t *>(idx);
    int32_t nb[E];
    decltype(wload(0)) wv[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int j = k * Q + sub;
      nb[k] = 0;                                // an idle lane gathers node 0 (in bounds) and adds nothing
      wv[k] = 0;
      if (k < E - 1 || sub < last) {
        nb[k] = ix[(uint64_t)j * cnt + t];
        wv[k] = wload(j);
      }
    }
    decltype(vload(0)) vv[E];
#pragma unroll
    for (int k = 0; k < E; ++k) vv[k] = vload(nb[k]);
    hook();
#pragma unroll
    for (int k = 0; k < E; ++k)
      if (k < E - 1 || sub < last) use(k * Q + sub, wv[k], vv[k]);
    settle();
  }
}

// KP: entries per gather chunk (a tuning parameter: more loads in flight
// against more registers held).  SEP: the reduction-kernel path (a.sepred),
// a template parameter so that no branch on it separates the first round of
// loads.  LN: several lanes per node of a non-regular width (lanes_for).
template <int D, int KP, bool SEP, bool LN>
__global__ __launch_bounds__(kBS) void k_bicg_pv(SimArgs a, int it) {
  Scalars *sc = a.sc;
  const int par = it & 1;
  // independent loads first (one wait), then the early exit
  const int done = sc->done, it_base = sc->it_base, nact = sc->nactive, lsel = sc->list_sel;
  const double bnorm2 = sc->bnorm2, alpha_prev = sc->alpha[par ^ 1], rho_prev = sc->rho[par ^ 1];
  const int64_t N = a.N;
  const int k = it_base + it;
  const bool first = (k == 0);
  const double2 *__restrict__ ST = a.ST;
  const double2 *__restrict__ PVo = a.PVo;
  if constexpr (SEP) {
    // the listed blocks (every block, or those of domains unfinished at the
    // last batch end); each domain's scalars were decided by k_reduce_b (or
    // k_reduce_r)
    BlockDesc b;
    const bool in = listed_block(a, blockIdx.x, nact, lsel, b);
    if (done || !in) return;
    // the domain's record (decided by k_reduce_b, or k_reduce_r for the first iteration)
    const DomLaunch L = load_launch(a.lpv + b.domain);
    if (L.done || (!first && L.early == 2)) return;
    pv_rows<D, KP, LN>(a, b, true, first, first ? 0 : L.early, L.c[0], L.c[1], L.c[2], L.c[3]);
    return;
  }
  // one domain, small grid: every block reduces the partials and takes the same decisions
  if (done) return;
  const BlockDesc b = a.kblk[blockIdx.x];
  double omega = 0.0, beta = 0.0, alpha_p = 0.0, pN;
  int early = 0;
  if (first) {
    double tot[kNR];
    reduce_prev<kNR>(a.partR, a.nblk, tot);   // k_rhs: one row per node block
    const double rN = -(a.bscale[0] * tot[2]);  // border row of r0: 0 - c sum x
    const double rho_k = fma(rN, rN, tot[1]);   // (rh, r0) = |r0|^2
    pN = rN;
    if (tot[0] == 0.0) early = 3;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->bnorm2 = tot[0];
      a.RV[N] = make_double2(rN, 0.0);
      a.rh[N] = rN;
      a.PVn[N] = make_double2(pN, 0.0);
      sc->rho[par] = rho_k;
      sc->early[par] = early;
    }
    if (early) return;
  } else {
    double tot[kNB];
    reduce_prev<kNB>(a.partB, gridDim.x, tot);
    const double bn = sqrt(bnorm2);
    const double sN = ST[N].x, rhN = a.rh[N];
    const double2 pvN = PVo[N];
    const double tN = a.bscale[0] * tot[5];     // border row of t = A s: c sum s
    const double ts = fma(tN, sN, tot[0]), tt = fma(tN, tN, tot[1]);
    const double rhs_ = fma(rhN, sN, tot[2]), rht = fma(rhN, tN, tot[3]);
    const double ss = fma(sN, sN, tot[4]);
    alpha_p = alpha_prev;
    const double rho_p = rho_prev;
    double rho_k = 0.0;
    if (sqrt(ss) <= a.tol * bn) early = 1;
    else if (tt == 0.0) early = 2;
    else {
      omega = ts / tt;
      rho_k = fma(-omega, rht, rhs_);
      if (rho_k == 0.0 || omega == 0.0) early = 2;
      else beta = (rho_k / rho_p) * (alpha_p / omega);
    }
    const double rN = fma(-omega, tN, sN);
    pN = fma(beta, fma(-omega, pvN.y, pvN.x), rN);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->early[par] = early;
      if (early == 1) {
        a.x[N] = fma(alpha_p, pvN.x, a.x[N]);
        sc->relres = sqrt(ss) / bn;
      } else if (early == 0) {
        a.x[N] = fma(omega, sN, fma(alpha_p, pvN.x, a.x[N]));
        a.RV[N] = make_double2(rN, 0.0);
        a.PVn[N] = make_double2(pN, 0.0);
        sc->rho[par] = rho_k;
      }
    }
    if (early == 2) return;
  }
  pv_rows<D, KP, LN>(a, b, false, first, early, omega, beta, alpha_p, a.bscale[0] * pN);
}

// The node rows of one block of k_bicg_st (csN: c_d times the border entry of
// s), Q threads per node as in k_bicg_pv: own values first, used in the
// gather's hook; stores from the node's first lane.
template <int D, bool LN>
__device__ __forceinline__ void st_rows(const SimArgs &a, const BlockDesc &b, bool again, double alpha,
                                        double csN) {
  const int64_t N = a.N;
  const int Q = LN ? lanes_for(b.width, D) : 1;
  const int node = (int)threadIdx.x >> __builtin_ctz((unsigned)Q);
  const int sub = (int)threadIdx.x & (Q - 1);
  const int64_t t = b.first + (int64_t)node;
  const bool live = node < b.nodes;
  const bool lead = live && sub == 0;
  const int64_t i = b.bstart + t;
  const double2 *__restrict__ RV = a.RV;
  double2 rvi = make_double2(0.0, 0.0);
  double rhi = 0.0, si = 0.0, acc = 0.0;
  if (live) {
    rvi = RV[i];
    rhi = a.rh[i];
  }
  const auto own = [&]() __attribute__((always_inline)) { si = fma(-alpha, rvi.y, rvi.x); };
  if (live) {
    const uint32_t cnt32 = (uint32_t)b.count, t32 = (uint32_t)t;
    const Buf RVb = plane(RV, N + 1, 0);
    with_width<D>(b.width, [&](auto wc) __attribute__((always_inline)) {
      constexpr int W = decltype(wc)::value;
      constexpr int QW = LN ? lanes_for(W, D) : 1;
      with_rows<D, W>(b, [&](auto sh) __attribute__((always_inline)) {
        constexpr bool SH = decltype(sh)::value;
        const auto wl = [&](int j) __attribute__((always_inline)) {
          if constexpr (QW == 1) return ld_prow<SH>(b, cnt32, j, t32);
          else return static_cast<const double *>(b.wP)[(uint64_t)j * cnt32 + t32];
        };
        gather_lanes<W, QW, 12>(
            b.idx, cnt32, t32, sub, wl,
            [&](int32_t nb) __attribute__((always_inline)) { return ld_at<double2>(RVb, nb); },
            [&](int, double wj, const double2 &rv2) __attribute__((always_inline)) {
              acc = fma(wj, fma(-alpha, rv2.y, rv2.x), acc);
            },
            [&]() __attribute__((always_inline)) { pin(acc); }, own);
      });
    });
  }
  if (LN) acc = lane_sum(acc, Q);
  double part[kNB] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // (t,s), (t,t), (rh,s), (rh,t), (s,s), sum s
  if (lead) {
    const double ti = acc + csN;                // + c_d times the border entry of s
    a.ST[i] = make_double2(si, ti);
    part[0] = ti * si;
    part[1] = ti * ti;
    part[2] = rhi * si;
    part[3] = rhi * ti;
    part[4] = si * si;
    part[5] = si;
  }
  block_partials<kNB>(part, a.partB, b.prow, again);
}

template <int D, bool SEP, bool LN>
__global__ __launch_bounds__(kBS) void k_bicg_st(SimArgs a, int it) {
  Scalars *sc = a.sc;
  const int par = it & 1;
  const int done = sc->done, it_base = sc->it_base, early = sc->early[par], nact = sc->nactive, lsel = sc->list_sel;
  const double bnorm2 = sc->bnorm2, rho_k = sc->rho[par];
  const int64_t N = a.N;
  const int k = it_base + it;
  if constexpr (SEP) {
    // the listed blocks of domains unfinished at the last batch end; alpha
    // was decided by k_reduce_a
    BlockDesc b;
    const bool in = listed_block(a, blockIdx.x, nact, lsel, b);
    if (done || !in) return;
    const DomLaunch L = load_launch(a.lst + b.domain);   // decided by k_reduce_a
    if (L.done) return;
    st_rows<D, LN>(a, b, true, L.c[0], L.c[1]);
    return;
  }
  if (done) return;
  const BlockDesc b = a.kblk[blockIdx.x];
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
  reduce_prev<kNA>(a.partA, gridDim.x, tot);
  const double bn = sqrt(bnorm2);
  const double vN = a.bscale[0] * tot[1];       // border row of v = A p: c sum p
  const double rN = a.RV[N].x;
  const double rv = fma(a.rh[N], vN, tot[0]);
  const double rr = fma(rN, rN, tot[2]);
  const double relres = sqrt(rr) / bn;
  int stop = 0;
  if (sqrt(rr) <= a.tol * bn) stop = 1;
  else if (k >= a.maxiter) stop = 2;
  else if (rv == 0.0) stop = 3;
  const double alpha = stop ? 0.0 : rho_k / rv;
  const double sN = fma(-alpha, vN, rN);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->relres = relres;
    if (stop) {
      sc->done = 1;
      sc->iters = k;
      if (stop >= 2) sc->fail = stop == 2 ? 2 : 1;
    } else {
      sc->alpha[par] = alpha;
      a.PVn[N].y = vN;
      a.RV[N].y = vN;
      a.ST[N] = make_double2(sN, 0.0);
    }
  }
  if (stop) return;
  st_rows<D, LN>(a, b, false, alpha, a.bscale[0] * sN);
}

// End of a batch of iterations (one block of kRedThreads).  With several
// domains: the batch flags from every domain's state and the list of the
// blocks still to run.  Then: advance the iteration base and publish a
// summary for the host.
__global__ __launch_bounds__(kRedThreads) void k_chunk_end(SimArgs a) {
  Scalars *sc = a.sc;
  if (a.K > 1 && !sc->done) {
    __shared__ BatchFlags f;
    batch_begin(f);
    for (int d = threadIdx.x; d < a.K; d += kRedThreads) batch_add(f, a.dom[d]);
    batch_end(a, f);
    __syncthreads();
    if (!sc->done) build_active(a);
  }
  if (threadIdx.x != 0) return;
  if (!sc->done) sc->it_base += a.chunk;
  HostFlags &h = sc->mirror;
  h.done = sc->done;
  h.iters = sc->done ? sc->iters : sc->it_base;
  h.fail = sc->fail;
  h.nonfinite = sc->nonfinite;
  h.relres = sc->relres;
  h.node_mv = sc->node_mv;
  h.nactive = sc->nactive;
}

// After k_chunk_end rebuilt the list of unfinished domains' blocks: their
// descriptors in list order, one thread per position.
__global__ __launch_bounds__(kBS) void k_list_desc(SimArgs a) {
  const Scalars *sc = a.sc;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sc->done || !sc->list_sel || v >= sc->nactive) return;
  a.lblk1[v] = a.kblk[a.active[v]];
}

// -------------------------------------------- projection + heat transport --
// v = v* - dt grad p at interior nodes (0 at walls); T' = T + dt (lap T -
// v.grad T) with the new velocity (Eq. (4)); Dirichlet walls keep T.  The
// pressure gradient reads FP64 p with FT weights, accumulated in FP64 (in
// the FP32 form over FP64 differences p_j - p_c).
template <int D, class FT>
__global__ __launch_bounds__(kBS) void k_correct_heat(SimArgs a) {
  const BlockDesc b = a.blk[blockIdx.x];
  const int64_t t = b.first + (int64_t)threadIdx.x;
  const bool live = (int)threadIdx.x < b.nodes;
  const int64_t N = a.N;
  // a domain whose pressure problem had a zero right-hand side takes p = 0
  const bool zero = a.sepred ? a.dom[b.domain].zero_sol != 0 : a.sc->zero_sol != 0;
  if (blockIdx.x == 0)
    for (int d = threadIdx.x; d < a.K; d += blockDim.x)
      if (a.sepred ? a.dom[d].zero_sol != 0 : a.sc->zero_sol != 0) a.x[N + d] = 0.0;
  if (!live) return;
  const int64_t i = b.bstart + t;
  const FT *__restrict__ T = static_cast<const FT *>(a.T);
  FT *__restrict__ vout = static_cast<FT *>(a.vout);
  FT *__restrict__ Tnp = static_cast<FT *>(a.Tn);
  bool bad = false;
  if (b.type == B_DIR || b.type == B_NEU) {
#pragma unroll
    for (int c = 0; c < D; ++c) vout[c * N + i] = FT(0);
    if (b.type == B_DIR) Tnp[i] = T[i];
    if (zero) a.x[i] = 0.0;
    return;
  }
  const uint32_t cnt32 = (uint32_t)b.count, t32 = (uint32_t)t;
  const Buf xb = plane(a.x, N + 1, 0), Tb = plane(T, N, 0);
  const FT *__restrict__ vs = static_cast<const FT *>(a.vs);
  const double dt = a.dt;
  using AccT = FieldAcc<FT>;
  constexpr bool kDiff = kDiffForm<FT>;
  with_width<D>(b.width, [&](auto wc) __attribute__((always_inline)) {
    constexpr int W = decltype(wc)::value;
    double gp[D];
    AccT gT[D], LT;
    double pc = 0.0;
    FT Tc = FT(0);
    LT.init();
#pragma unroll
    for (int q = 0; q < D; ++q) { gp[q] = 0.0; gT[q].init(); }
    gather_chunks<W>(
        b.idx, cnt32, t32,
        [&](int j) __attribute__((always_inline)) {
          Pack<FT, D + 1> r;
#pragma unroll
          for (int q = 0; q <= D; ++q) r.v[q] = (kDiff && j == 0) ? FT(0) : ld_soa<FT>(b.w, cnt32, q * W + j, t32);
          return r;
        },
        [&](int32_t nb) __attribute__((always_inline)) {
          const double pj = ld_at<double>(xb, nb);
          Pack2<double, 1, FT, 1> r;
          r.a.v[0] = zero ? 0.0 : pj;
          r.b.v[0] = ld_at<FT>(Tb, nb);
          return r;
        },
        [&](int j, const Pack<FT, D + 1> &wq, const Pack2<double, 1, FT, 1> &u) __attribute__((always_inline)) {
          if (kDiff && j == 0) {
            pc = u.a.v[0];
            Tc = u.b.v[0];
            return;
          }
          // FP32 form: the pressure difference is taken in FP64, then weighted
          const double pj = kDiff ? u.a.v[0] - pc : u.a.v[0];
          const FT Tj = kDiff ? FT(u.b.v[0] - Tc) : u.b.v[0];
#pragma unroll
          for (int q = 0; q < D; ++q) {
            gp[q] = fma((double)wq.v[q], pj, gp[q]);
            gT[q].add(wq.v[q], Tj);
          }
          LT.add(wq.v[D], Tj);
        },
        [&]() __attribute__((always_inline)) {
          LT.settle();
#pragma unroll
          for (int q = 0; q < D; ++q) { pin(gp[q]); gT[q].settle(); }
        });
    double vn[D];
#pragma unroll
    for (int q = 0; q < D; ++q) {
      vn[q] = fma(-dt, gp[q], (double)vs[q * N + i]);
      const FT st = (FT)vn[q];
      vout[q * N + i] = st;
      vn[q] = (double)st;                    // the stored velocity advects T
      bad = bad || !isfinite(vn[q]);
    }
    double adv = vn[0] * gT[0].get_d();
#pragma unroll
    for (int q = 1; q < D; ++q) adv = fma(vn[q], gT[q].get_d(), adv);
    const double Tn = fma(dt, LT.get_d() - adv, (double)T[i]);
    Tnp[i] = (FT)Tn;
    bad = bad || !isfinite(Tn);
  });
  if (zero) a.x[i] = 0.0;
  if (bad) atomicOr(&a.sc->nonfinite, 1);
}

// Neumann walls: the temperature that zeroes the normal derivative, from the
// new interior values (wall stencils hold the wall node and interior nodes).
template <int D, class FT>
__global__ __launch_bounds__(kBS) void k_neumann(SimArgs a) {
  const BlockDesc b = a.blk[blockIdx.x];
  const int64_t t = b.first + (int64_t)threadIdx.x;
  const bool live = (int)threadIdx.x < b.nodes;
  if (!live || b.type != B_NEU) return;
  const int64_t N = a.N, i = b.bstart + t;
  const uint32_t cnt32 = (uint32_t)b.count, t32 = (uint32_t)t;
  FT *Tn = static_cast<FT *>(a.Tn);
  const Buf Tnb = plane(Tn, N, 0);
  Scalars *sc = a.sc;
  using AccT = FieldAcc<FT>;
  constexpr bool kDiff = kDiffForm<FT>;
  with_width<D>(b.width, [&](auto wc) __attribute__((always_inline)) {
    constexpr int W = decltype(wc)::value;
    AccT acc;
    acc.init();
    FT T1 = FT(0);
    gather_chunks<W>(
        b.idx, cnt32, t32,
        [&](int j) __attribute__((always_inline)) {
          return (kDiff && j == 1) ? FT(0) : ld_soa<FT>(b.w, cnt32, (D + 1) * W + j, t32);
        },
        [&](int32_t nb) __attribute__((always_inline)) { return ld_at<FT>(Tnb, nb); },
        [&](int j, FT wj, FT Tj) __attribute__((always_inline)) {
          // the wall node's own entry (j = 0) is the unknown
          if (kDiff && j == 1) T1 = Tj;
          else if (j > 0) acc.add(wj, kDiff ? FT(Tj - T1) : Tj);
        },
        [&]() __attribute__((always_inline)) { acc.settle(); });
    // FP32 form: the weights sum to zero, so sum_{j>=1} w_j (T_j - T_1) + w_0 (T_b - T_1) = 0
    const double w0 = (double)ld_soa<FT>(b.w, cnt32, (D + 1) * W, t32);
    const double Tb = kDiff ? (double)T1 - acc.get_d() / w0 : -acc.get_d() / w0;
    Tn[i] = (FT)Tb;
    if (!isfinite(Tb)) atomicOr(&sc->nonfinite, 1);
  });
}

// pressure-operator rows: Laplacian (interior) or normal derivative (walls), divided by the centre weight
__global__ void k_scale_rows(const double *w, int64_t cnt, int W, int slot, double *wP) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt) return;
  const double *src = w + (int64_t)slot * W * cnt;
  const double dg = src[t];
  for (int j = 0; j < W; ++j) wP[(int64_t)j * cnt + t] = src[(int64_t)j * cnt + t] / dg;
}

// Largest |wP[j][t] - L_j| over a regular bucket's pressure rows, L the
// lattice row (1 at the centre, -1/(2d) at each of the 2d cross nodes: the
// MON Laplacian on an exact lattice cross, divided by its centre weight).
// Non-negative doubles order as their bit patterns; a NaN deviation maps to
// the largest pattern.
__global__ void k_lattice_dev(const double *wP, int64_t cnt, int W, unsigned long long *dev) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt) return;
  const double off = -1.0 / (double)(W - 1);
  double m = 0.0;
  for (int j = 0; j < W; ++j) {
    const double e = fabs(wP[(int64_t)j * cnt + t] - (j == 0 ? 1.0 : off));
    m = (e > m || e != e) ? (e != e ? INFINITY : e) : m;
  }
  atomicMax(dev, (unsigned long long)__double_as_longlong(m));
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

template <class S, class T>
__global__ void k_gather(const S *src, T *dst, const int32_t *map, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (T)src[map[i]];
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace
}  // namespace hsm
