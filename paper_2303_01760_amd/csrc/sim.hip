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

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <string>
#include <memory>
#include <type_traits>
#include <vector>

#include "hsm_internal.h"

#include "sim_kernels.h"

using namespace hsm;

struct hsm_sim {
  const hsm_stencils *st = nullptr;
  hsm_sim_params prm{};
  int d = 0;
  int64_t N = 0;
  int chunk = 32;
  int bs = kBS;                // threads (and at most nodes) per block of the node kernels
  int kp = 8;                  // entries per gather chunk of the p/v kernel
  bool xcd = false;            // XCD-contiguous block order in the Krylov kernels (reduction-kernel path)
  DBuf v, vs, T[2], vec[2], pairs[4], partR, partA, partB, sc, wP[kMaxBuckets];
  double *x = nullptr, *rh = nullptr;
  double2 *ST = nullptr, *PV[2] = {nullptr, nullptr}, *RV = nullptr;
  int parity = 0;
  hipStream_t s = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_chunk[2] = {nullptr, nullptr};
  HostFlags *hflags = nullptr;   // pinned [2]
  bool graphs_ready = false;
  hipGraphExec_t g_pre[2] = {nullptr, nullptr}, g_post[2] = {nullptr, nullptr};
  hipGraph_t gr[4] = {nullptr, nullptr, nullptr, nullptr};
  // Krylov batches per host-flag slot and grid level: with several domains the
  // list of blocks to run shrinks as domains finish, and a batch is launched
  // with the smallest captured grid that still covers it (level L: the full
  // grid halved L times)
  static constexpr int kLevels = 8;
  hipGraphExec_t g_kry[2][kLevels] = {};
  hipGraph_t gr_kry[2][kLevels] = {};
  int nlev = 1;
  int64_t lev_grid[kLevels] = {};
  int64_t known_nact = 0;     // an upper bound of the blocks still to run (from the latest flags read)
  hsm_sim_stats stats{};
  int64_t n_int = 0, n_neu = 0;
  int64_t n_shared = 0, nnz_shared = 0;   // regular nodes (and their stencil entries) on the shared lattice row
  // profiling: events captured around kernels (profile mode)
  hipEvent_t ep_pre[2][2] = {}, ep_kry[2][2] = {}, ep_post[2][2] = {};  // start/stop around each phase
  double k_sum_ms[HSM_PH_COUNT] = {};
  int64_t k_cnt[HSM_PH_COUNT] = {};
  int post_pending = -1;     // parity of a post phase whose events are not read yet
  int32_t K = 1;              // domains (border rows)
  int64_t nblk = 0;           // blocks of every node launch
  DBuf blk, dom_blk_off, dom_blk;   // block descriptors; per-domain block lists
  DBuf dom;                          // per-domain Krylov state [K]
  DBuf dom_nodes;                    // int64 [K] nodes per domain
  DBuf bscale;                       // double [K] border scale 1/sqrt(nodes) per domain
  DBuf active;                       // int32 [nblk] blocks of unfinished domains
  DBuf lblk0, lblk1;                 // descriptors by list position: every block; the blocks of `active`
  DBuf kblk, kdom_blk_off, kdom_blk; // the Krylov node kernels' partition (bs / lanes nodes a block)
  int64_t nkblk = 0;
  bool lanes = false;                // several threads per node of a non-regular width (lanes_for)
  DBuf lpv, lst;                     // DomLaunch [K]: per-domain records of the Krylov node kernels
  int64_t kry_grid = 0;              // grid of the Krylov node kernels (every block descriptor)
  bool f32 = false;           // FP32 field form (HSM_F32_COMP)
  bool sepred = false;        // grid totals by a separate one-block kernel (large grids)

  ~hsm_sim() {
    if (s) (void)hipStreamSynchronize(s);
    for (auto &g : g_pre) if (g) (void)hipGraphExecDestroy(g);
    for (auto &row : g_kry) for (auto &g : row) if (g) (void)hipGraphExecDestroy(g);
    for (auto &g : g_post) if (g) (void)hipGraphExecDestroy(g);
    for (auto &g : gr) if (g) (void)hipGraphDestroy(g);
    for (auto &row : gr_kry) for (auto &g : row) if (g) (void)hipGraphDestroy(g);
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
  a.blk = m->blk.as<BlockDesc>();
  a.nblk = m->nblk;
  a.K = m->K;
  a.dom_blk_off = m->dom_blk_off.as<int32_t>();
  a.dom_blk = m->dom_blk.as<int32_t>();
  a.dom = m->dom.as<DomState>();
  a.dom_nodes = m->dom_nodes.as<int64_t>();
  a.bscale = m->bscale.as<double>();
  a.active = m->active.as<int32_t>();
  a.lblk0 = m->lblk0.as<BlockDesc>();
  a.lblk1 = m->lblk1.as<BlockDesc>();
  a.lpv = m->lpv.as<DomLaunch>();
  a.kblk = m->kblk.as<BlockDesc>();
  a.nkblk = m->nkblk;
  a.kdom_blk_off = m->kdom_blk_off.as<int32_t>();
  a.kdom_blk = m->kdom_blk.as<int32_t>();
  a.lst = m->lst.as<DomLaunch>();
  a.N = m->N;
  a.dt = m->prm.dt; a.Ra = m->prm.Ra; a.Pr = m->prm.Pr; a.T_ref = m->prm.T_ref; a.tol = m->prm.krylov_tol;
  a.maxiter = m->prm.krylov_maxiter;
  a.chunk = m->chunk;
  a.sepred = m->sepred ? 1 : 0;
  a.xcd_order = m->xcd ? 1 : 0;
  a.v = m->v.p;
  a.vs = m->vs.p;
  a.T = m->T[par].p;
  a.Tn = m->T[par ^ 1].p;
  a.vout = m->v.p;
  a.x = m->x; a.rh = m->rh;
  a.ST = m->ST; a.RV = m->RV;
  a.PVo = m->PV[kpar]; a.PVn = m->PV[kpar ^ 1];
  a.partR = m->partR.as<double>();
  a.partA = m->partA.as<double>();
  a.partB = m->partB.as<double>();
  a.sc = m->sc.as<Scalars>();
  return a;
}

// Kernel launches of each phase.
template <int D>
hsm_status enqueue_pre(hsm_sim *m, int par, hipStream_t s) {
  SimArgs a = make_args(m, par, 0);
  const dim3 g((unsigned)m->nblk), b((unsigned)m->bs);
  if (m->f32) {
    hipLaunchKernelGGL((k_predict<D, float>), g, b, 0, s, a);
    hipLaunchKernelGGL((k_rhs<D, float>), g, b, 0, s, a);
  } else {
    hipLaunchKernelGGL((k_predict<D, double>), g, b, 0, s, a);
    hipLaunchKernelGGL((k_rhs<D, double>), g, b, 0, s, a);
  }
  if (m->sepred) hipLaunchKernelGGL(k_reduce_r, dim3((unsigned)red_grid(m->K)), dim3(kRedThreads), 0, s, a);
  HSM_HIP(hipGetLastError());
  return HSM_OK;
}

template <int D, int KP, bool LN>
void launch_pv(bool sep, dim3 g, dim3 b, hipStream_t s, const SimArgs &a, int it) {
  if (sep) hipLaunchKernelGGL((k_bicg_pv<D, KP, true, LN>), g, b, 0, s, a, it);
  else hipLaunchKernelGGL((k_bicg_pv<D, KP, false, LN>), g, b, 0, s, a, it);
}
template <int D, bool LN>
void launch_st(bool sep, dim3 g, dim3 b, hipStream_t s, const SimArgs &a, int it) {
  if (sep) hipLaunchKernelGGL((k_bicg_st<D, true, LN>), g, b, 0, s, a, it);
  else hipLaunchKernelGGL((k_bicg_st<D, false, LN>), g, b, 0, s, a, it);
}

// Krylov iterations [it0, it1) of a batch; the ping-pong parity follows the
// iteration number, so a batch may be split across launch paths.
template <int D>
hsm_status enqueue_krylov(hsm_sim *m, int slot, hipStream_t s, int it0, int it1, bool flags, int lev = 0) {
  const dim3 g((unsigned)m->lev_grid[lev]), b((unsigned)m->bs);
  for (int it = it0; it < it1; ++it) {
    SimArgs a = make_args(m, 0, it & 1);
    switch (m->kp) {
      case 4: m->lanes ? launch_pv<D, 4, true>(m->sepred, g, b, s, a, it) : launch_pv<D, 4, false>(m->sepred, g, b, s, a, it); break;
      case 6: m->lanes ? launch_pv<D, 6, true>(m->sepred, g, b, s, a, it) : launch_pv<D, 6, false>(m->sepred, g, b, s, a, it); break;
      case 12: m->lanes ? launch_pv<D, 12, true>(m->sepred, g, b, s, a, it) : launch_pv<D, 12, false>(m->sepred, g, b, s, a, it); break;
      default: m->lanes ? launch_pv<D, 8, true>(m->sepred, g, b, s, a, it) : launch_pv<D, 8, false>(m->sepred, g, b, s, a, it); break;
    }
    if (m->sepred) hipLaunchKernelGGL(k_reduce_a, dim3((unsigned)red_grid(m->K)), dim3(kRedThreads), 0, s, a, it);
    if (m->lanes) launch_st<D, true>(m->sepred, g, b, s, a, it);
    else launch_st<D, false>(m->sepred, g, b, s, a, it);
    if (m->sepred) hipLaunchKernelGGL(k_reduce_b, dim3((unsigned)red_grid(m->K)), dim3(kRedThreads), 0, s, a, it);
  }
  HSM_HIP(hipGetLastError());
  if (flags) {
    SimArgs a = make_args(m, 0, 0);
    hipLaunchKernelGGL(k_chunk_end, dim3(1), dim3(kRedThreads), 0, s, a);
    if (m->sepred && m->K > 1)
      hipLaunchKernelGGL(k_list_desc, dim3((unsigned)((m->nkblk + kBS - 1) / kBS)), dim3(kBS), 0, s, a);
    HSM_HIP(hipGetLastError());
    Scalars *sc = m->sc.as<Scalars>();
    HSM_HIP(hipMemcpyAsync(&m->hflags[slot], &sc->mirror, sizeof(HostFlags), hipMemcpyDeviceToHost, s));
  }
  return HSM_OK;
}

template <int D>
hsm_status enqueue_post(hsm_sim *m, int par, hipStream_t s) {
  SimArgs a = make_args(m, par, 0);
  const dim3 g((unsigned)m->nblk), b((unsigned)m->bs);
  if (m->f32) {
    hipLaunchKernelGGL((k_correct_heat<D, float>), g, b, 0, s, a);
    hipLaunchKernelGGL((k_neumann<D, float>), g, b, 0, s, a);
  } else {
    hipLaunchKernelGGL((k_correct_heat<D, double>), g, b, 0, s, a);
    hipLaunchKernelGGL((k_neumann<D, double>), g, b, 0, s, a);
  }
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
    if ((rc = capture(m, m->gr[2 + par], m->g_post[par], [&] { return enqueue_post<D>(m, par, m->s); })))
      return rc;
    for (int lev = 0; lev < m->nlev; ++lev)
      if ((rc = capture(m, m->gr_kry[par][lev], m->g_kry[par][lev],
                        [&] { return enqueue_krylov<D>(m, par, m->s, 0, m->chunk, true, lev); })))
        return rc;
  }
  m->graphs_ready = true;
  return HSM_OK;
}

// Each phase is either replayed from its graph or launched directly
// (launch_mode 1); in profile mode start/stop events bracket the phase on the
// stepper's stream (events recorded inside a captured graph cannot be timed,
// so they sit around the graph launch).
hsm_status do_pre(hsm_sim *m, int par) {
  hsm_status rc = HSM_OK;
  if (m->prm.profile) HSM_HIP(hipEventRecord(m->ep_pre[par][0], m->s));
  if (m->prm.launch_mode == 1) rc = m->d == 2 ? enqueue_pre<2>(m, par, m->s) : enqueue_pre<3>(m, par, m->s);
  else HSM_HIP(hipGraphLaunch(m->g_pre[par], m->s));
  if (rc) return rc;
  if (m->prm.profile) HSM_HIP(hipEventRecord(m->ep_pre[par][1], m->s));
  return HSM_OK;
}
// The smallest captured grid level that covers `nact` blocks.
int level_for(const hsm_sim *m, int64_t nact) {
  int lev = 0;
  while (lev + 1 < m->nlev && m->lev_grid[lev + 1] >= nact) ++lev;
  return lev;
}
hsm_status do_krylov(hsm_sim *m, int slot) {
  hsm_status rc = HSM_OK;
  const int lev = level_for(m, m->known_nact);
  if (lev > 0) m->stats.krylov_reduced_batches += 1;
  if (m->prm.profile) HSM_HIP(hipEventRecord(m->ep_kry[slot][0], m->s));
  if (m->prm.launch_mode == 1)
    rc = m->d == 2 ? enqueue_krylov<2>(m, slot, m->s, 0, m->chunk, true, lev)
                   : enqueue_krylov<3>(m, slot, m->s, 0, m->chunk, true, lev);
  else HSM_HIP(hipGraphLaunch(m->g_kry[slot][lev], m->s));
  if (rc) return rc;
  if (m->prm.profile) HSM_HIP(hipEventRecord(m->ep_kry[slot][1], m->s));
  return HSM_OK;
}
hsm_status do_post(hsm_sim *m, int par) {
  hsm_status rc = HSM_OK;
  if (m->prm.profile) HSM_HIP(hipEventRecord(m->ep_post[par][0], m->s));
  if (m->prm.launch_mode == 1) rc = m->d == 2 ? enqueue_post<2>(m, par, m->s) : enqueue_post<3>(m, par, m->s);
  else HSM_HIP(hipGraphLaunch(m->g_post[par], m->s));
  if (rc) return rc;
  if (m->prm.profile) HSM_HIP(hipEventRecord(m->ep_post[par][1], m->s));
  return HSM_OK;
}

hsm_status add_time(hsm_sim *m, int k, hipEvent_t a, hipEvent_t b, int64_t units = 1) {
  float ms = 0.f;
  HSM_HIP(hipEventElapsedTime(&ms, a, b));
  m->k_sum_ms[k] += ms;
  m->k_cnt[k] += units;
  return HSM_OK;
}

// post-phase events of an earlier step (complete once later work has synchronised)
hsm_status read_post(hsm_sim *m) {
  if (!m->prm.profile || m->post_pending < 0) return HSM_OK;
  const int p = m->post_pending;
  m->post_pending = -1;
  return add_time(m, HSM_PH_POST, m->ep_post[p][0], m->ep_post[p][1]);
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
    m->known_nact = m->nkblk;                               // a new solve runs every block
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
      // blocks of unfinished domains after this batch: the batches queued
      // from here on run no more (the list only shrinks within a solve)
      if (m->sepred && m->K > 1) m->known_nact = std::min<int64_t>(m->known_nact, f.nactive);
      if (m->prm.profile) {
        if (c == 0) {
          if ((rc = read_post(m))) return rc;
          if ((rc = add_time(m, HSM_PH_PRE, m->ep_pre[par][0], m->ep_pre[par][1]))) return rc;
        }
        // batches in which every iteration did work: batch time per iteration
        if (!f.done && (rc = add_time(m, HSM_PH_KRYLOV_ITER, m->ep_kry[c & 1][0], m->ep_kry[c & 1][1], m->chunk)))
          return rc;
        if ((rc = add_time(m, HSM_PH_KRYLOV_TOTAL, m->ep_kry[c & 1][0], m->ep_kry[c & 1][1], 1))) return rc;
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
    // Krylov matvec rows: counted per domain on the reduction-kernel path (domains stop
    // separately), two per iteration over all nodes otherwise
    const int64_t mv = m->sepred ? (int64_t)f.node_mv : per_iter * f.iters;
    m->stats.krylov_node_matvecs += mv;
    m->stats.node_applies += m->n_int * (D * (D + 1) + D + 2 * D + 1) + m->N + mv + m->n_neu;
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
  if (prm->field_dtype != HSM_F64 && prm->field_dtype != HSM_F32_COMP) {
    set_error(HSM_E_INVALID, "field_dtype must be HSM_F64 or HSM_F32_COMP");
    return HSM_E_INVALID;
  }
  if (st->N < 1) { set_error(HSM_E_INVALID, "empty stencil set"); return HSM_E_INVALID; }
  if (prm->profile != 0 && prm->profile != 1) { set_error(HSM_E_INVALID, "profile must be 0 or 1"); return HSM_E_INVALID; }
  if (prm->launch_mode != 0 && prm->launch_mode != 1) { set_error(HSM_E_INVALID, "launch_mode must be 0 or 1"); return HSM_E_INVALID; }
  if (prm->reduce_mode < 0 || prm->reduce_mode > 2) {
    set_error(HSM_E_INVALID, "reduce_mode must be 0, 1 or 2");
    return HSM_E_INVALID;
  }
  if (prm->krylov_chunk < 0 || prm->krylov_chunk > kMaxIterChunk) {
    set_error(HSM_E_INVALID, "krylov_chunk out of range");
    return HSM_E_INVALID;
  }
  auto m = std::make_unique<hsm_sim>();
  m->st = st; m->prm = *prm; m->d = st->d; m->N = st->N;
  m->chunk = prm->krylov_chunk ? prm->krylov_chunk : 32;
  if (prm->block_nodes != 0 && prm->block_nodes != 64 && prm->block_nodes != 128 && prm->block_nodes != 256 &&
      prm->block_nodes != 512) {
    set_error(HSM_E_INVALID, "block_nodes must be 0 (256), 64, 128, 256 or 512");
    return HSM_E_INVALID;
  }
  if (prm->gather_chunk != 0 && prm->gather_chunk != 4 && prm->gather_chunk != 6 && prm->gather_chunk != 8 &&
      prm->gather_chunk != 12) {
    set_error(HSM_E_INVALID, "gather_chunk must be 0 (8), 4, 6, 8 or 12");
    return HSM_E_INVALID;
  }
  if (prm->lattice_rows != 0 && prm->lattice_rows != 1) {
    set_error(HSM_E_INVALID, "lattice_rows must be 0 or 1");
    return HSM_E_INVALID;
  }
  if (prm->wide_lanes < 0 || prm->wide_lanes > 2) {
    set_error(HSM_E_INVALID, "wide_lanes must be 0 (auto), 1 or 2");
    return HSM_E_INVALID;
  }
  if (prm->xcd_order != 0 && prm->xcd_order != 1) {
    set_error(HSM_E_INVALID, "xcd_order must be 0 or 1");
    return HSM_E_INVALID;
  }
  m->bs = prm->block_nodes ? prm->block_nodes : 256;
  m->kp = prm->gather_chunk ? prm->gather_chunk : 8;
  if (m->chunk & 1) m->chunk += 1;   // even: ping-pong buffers line up across batches
  const int64_t N = st->N, d = st->d;
  hipStream_t us = (hipStream_t)stream;
  hsm_status rc;
  m->f32 = prm->field_dtype == HSM_F32_COMP;
  const size_t fsz = m->f32 ? sizeof(float) : sizeof(double);
  if ((rc = m->v.alloc(fsz * d * N)) || (rc = m->vs.alloc(fsz * d * N)) || (rc = m->T[0].alloc(fsz * N)) ||
      (rc = m->T[1].alloc(fsz * N)) || (rc = m->sc.alloc(sizeof(Scalars))))
    return rc;
  if (m->f32 && (rc = ensure_w32(st, us))) return rc;
  // Krylov vectors: N node rows and one border row per domain
  m->K = st->n_domains;
  const int64_t NK = N + m->K;
  for (auto &b : m->vec)
    if ((rc = b.alloc(sizeof(double) * NK))) return rc;
  for (auto &b : m->pairs)
    if ((rc = b.alloc(sizeof(double2) * NK))) return rc;
  m->x = m->vec[0].as<double>(); m->rh = m->vec[1].as<double>();
  m->ST = m->pairs[0].as<double2>(); m->PV[0] = m->pairs[1].as<double2>(); m->PV[1] = m->pairs[2].as<double2>();
  m->RV = m->pairs[3].as<double2>();
  // pressure-operator rows, per bucket.  A regular bucket whose rows all
  // equal the lattice row (1 at the centre, -1/(2d) on the cross) to within
  // kLatticeRowTol keeps that one row instead of a row per node: the
  // Krylov kernels then read W uniform values instead of W per node.
  std::vector<const void *> wp_of(st->buckets.size(), nullptr);
  std::vector<int32_t> shared_of(st->buckets.size(), 0);
  {
    DBuf dev;
    if ((rc = dev.alloc(sizeof(unsigned long long)))) return rc;
    int k = 0;
    for (size_t kb = 0; kb < st->buckets.size(); ++kb) {
      const Bucket &B = st->buckets[kb];
      if (B.count == 0) continue;
      if ((rc = m->wP[k].alloc(sizeof(double) * B.width * B.count))) return rc;
      const int slot = (B.type == B_DIR || B.type == B_NEU) ? st->d + 1 : st->d;
      hipLaunchKernelGGL(k_scale_rows, dim3(nblk(B.count, 256)), dim3(256), 0, us, B.w.as<double>(), B.count,
                         B.width, slot, m->wP[k].as<double>());
      if (B.type == B_REG || B.type == B_SCAT) m->n_int += B.count;
      if (B.type == B_NEU) m->n_neu += B.count;
      wp_of[kb] = m->wP[k].p;
      if (B.type == B_REG && B.width == 2 * st->d + 1 && prm->lattice_rows == 0) {
        unsigned long long h = 0;
        HSM_HIP(hipMemsetAsync(dev.p, 0, sizeof(h), us));
        hipLaunchKernelGGL(k_lattice_dev, dim3(nblk(B.count, 256)), dim3(256), 0, us, m->wP[k].as<double>(),
                           B.count, B.width, dev.as<unsigned long long>());
        HSM_HIP(hipGetLastError());
        HSM_HIP(hipMemcpyAsync(&h, dev.p, sizeof(h), hipMemcpyDeviceToHost, us));
        HSM_HIP(hipStreamSynchronize(us));
        double worst;
        std::memcpy(&worst, &h, sizeof(worst));
        if (worst <= kLatticeRowTol) {
          std::vector<double> row(B.width, -1.0 / (double)(2 * st->d));
          row[0] = 1.0;
          if ((rc = m->wP[k].alloc(sizeof(double) * B.width))) return rc;
          HSM_HIP(hipMemcpyAsync(m->wP[k].p, row.data(), sizeof(double) * B.width, hipMemcpyHostToDevice, us));
          HSM_HIP(hipStreamSynchronize(us));
          wp_of[kb] = m->wP[k].p;
          shared_of[kb] = 1;
          m->n_shared += B.count;
          m->nnz_shared += B.count * B.width;
        }
      }
      ++k;
    }
  }
  // blocks: up to m->bs consecutive nodes of one bucket and one domain
  std::vector<int32_t> dom_int;
  if (m->K > 1) {
    std::vector<int32_t> hperm(N);
    HSM_HIP(hipMemcpyAsync(hperm.data(), st->perm.p, sizeof(int32_t) * N, hipMemcpyDeviceToHost, us));
    HSM_HIP(hipStreamSynchronize(us));
    dom_int.resize(N);
    for (int64_t i = 0; i < N; ++i)
      dom_int[i] = (int32_t)(std::upper_bound(st->dom_off.begin(), st->dom_off.end(), (int64_t)hperm[i]) -
                             st->dom_off.begin() - 1);
  }
  // a partition of the nodes into blocks of up to `per(width)` consecutive
  // nodes of one bucket and one domain, with the per-domain block lists (the
  // reduction kernels' rows: prow is a block's place in them)
  struct Partition {
    std::vector<BlockDesc> blocks;
    std::vector<int32_t> dbo, dbl;
  };
  const auto partition = [&](auto per) {
    Partition P;
    for (size_t kb = 0; kb < st->buckets.size(); ++kb) {
      const Bucket &B = st->buckets[kb];
      const int64_t cap = per(B.width);
      for (int64_t j = 0; j < B.count;) {
        const int32_t dom = m->K > 1 ? dom_int[B.start + j] : 0;
        int64_t e = j + 1;
        while (e < B.count && e - j < cap && (m->K == 1 || dom_int[B.start + e] == dom)) ++e;
        BlockDesc bd;
        std::memset(&bd, 0, sizeof(bd));
        bd.idx = B.idx.p;
        bd.w = m->f32 ? B.w32.p : B.w.p;         // field weights in the field storage type
        bd.wP = wp_of[kb];
        bd.wshared = shared_of[kb];
        bd.bstart = B.start;
        bd.first = (int32_t)j;
        bd.nodes = (int32_t)(e - j);
        bd.count = (int32_t)B.count;
        bd.type = B.type;
        bd.width = B.width;
        bd.domain = dom;
        P.blocks.push_back(bd);
        j = e;
      }
    }
    P.dbo.assign(m->K + 1, 0);
    P.dbl.resize(P.blocks.size());
    for (const BlockDesc &bd : P.blocks) P.dbo[bd.domain + 1] += 1;
    for (int32_t d2 = 0; d2 < m->K; ++d2) P.dbo[d2 + 1] += P.dbo[d2];
    std::vector<int32_t> fill(P.dbo.begin(), P.dbo.end() - 1);
    for (size_t b2 = 0; b2 < P.blocks.size(); ++b2) P.dbl[fill[P.blocks[b2].domain]++] = (int32_t)b2;
    for (size_t j2 = 0; j2 < P.dbl.size(); ++j2) P.blocks[P.dbl[j2]].prow = (int32_t)j2;   // one domain: prow = block
    return P;
  };
  const auto upload = [&](const Partition &P, DBuf &blk, DBuf &off, DBuf &lst) -> hsm_status {
    hsm_status r;
    if ((r = blk.alloc(sizeof(BlockDesc) * (P.blocks.size() + 1))) || (r = off.alloc(sizeof(int32_t) * P.dbo.size())) ||
        (r = lst.alloc(sizeof(int32_t) * (P.dbl.size() + 1))))
      return r;
    HSM_HIP(hipMemcpyAsync(blk.p, P.blocks.data(), sizeof(BlockDesc) * P.blocks.size(), hipMemcpyHostToDevice, us));
    HSM_HIP(hipMemcpyAsync(off.p, P.dbo.data(), sizeof(int32_t) * P.dbo.size(), hipMemcpyHostToDevice, us));
    HSM_HIP(hipMemcpyAsync(lst.p, P.dbl.data(), sizeof(int32_t) * P.dbl.size(), hipMemcpyHostToDevice, us));
    return HSM_OK;
  };
  // every node kernel but the Krylov ones: one node per thread
  const Partition base = partition([&](int) { return (int64_t)m->bs; });
  // the Krylov node kernels: lanes_for(width) threads per node, or one.
  // Several lanes shorten a wide stencil's chain of gather rounds; where most
  // nodes are wide, their redundant own loads and extra blocks cost more
  // (measured: 9 % faster Krylov batches on the 512 hybrid domains, 21 % and
  // 37 % slower in the all-scattered 2D and 3D layouts)
  if (prm->wide_lanes == 0) {
    int64_t wide = 0;
    for (const Bucket &B : st->buckets)
      if (lanes_for(B.width, st->d) > 1) wide += B.count;
    m->lanes = 2 * wide < N;
  } else {
    m->lanes = prm->wide_lanes == 2;
  }
  const Partition kry = partition([&](int w) { return (int64_t)(m->bs / (m->lanes ? lanes_for(w, st->d) : 1)); });
  m->nblk = (int64_t)base.blocks.size();
  m->nkblk = (int64_t)kry.blocks.size();
  if ((rc = upload(base, m->blk, m->dom_blk_off, m->dom_blk)) ||
      (rc = upload(kry, m->kblk, m->kdom_blk_off, m->kdom_blk)))
    return rc;
  // descriptors by list position (the Krylov kernels' workgroups): every
  // Krylov block in per-domain order, and room for the list of unfinished
  // domains' blocks (zeroed; rewritten before each use)
  std::vector<BlockDesc> listed(kry.dbl.size() + 8);
  std::memset(listed.data(), 0, sizeof(BlockDesc) * listed.size());
  for (size_t j2 = 0; j2 < kry.dbl.size(); ++j2) listed[j2] = kry.blocks[kry.dbl[j2]];
  if ((rc = m->lblk0.alloc(sizeof(BlockDesc) * listed.size())) ||
      (rc = m->lblk1.alloc(sizeof(BlockDesc) * listed.size())))
    return rc;
  HSM_HIP(hipMemcpyAsync(m->lblk0.p, listed.data(), sizeof(BlockDesc) * listed.size(), hipMemcpyHostToDevice, us));
  HSM_HIP(hipMemsetAsync(m->lblk1.p, 0, sizeof(BlockDesc) * listed.size(), us));
  HSM_HIP(hipStreamSynchronize(us));      // the host vectors above go out of scope
  // grid totals: in every block's prologue for one domain on a small grid;
  // otherwise by the reduction kernels, which also own the border rows (a
  // block reading every partial costs more than a launch near a thousand
  // blocks; many domains need per-domain sums)
  if (m->K > 1 && prm->reduce_mode == 1) {
    set_error(HSM_E_INVALID, "reduce_mode 1 (in-kernel reduction) needs a single domain");
    return HSM_E_INVALID;
  }
  m->sepred = m->K > 1 || prm->reduce_mode == 2 || (prm->reduce_mode == 0 && m->nkblk > kSepReduceBlocks);
  // Krylov node kernels: one block per descriptor; with many domains the
  // blocks past the list of unfinished domains' blocks return at once (a
  // grid of the blocks the device holds at once, walking the list, measured
  // 9 % slower on 512 domains: the hardware refills a full grid faster than
  // a block walks its share)
  // the XCD-contiguous order needs at least 8 ceil(nkblk / 8) workgroups (one grid slot per list position)
  m->xcd = m->sepred && prm->xcd_order != 0;
  m->kry_grid = m->xcd ? (m->nkblk + kXcds - 1) / kXcds * kXcds : m->nkblk;
  // grid levels of the Krylov batches: several domains only (their list of
  // blocks shrinks as domains finish); each level holds at least 8 workgroups
  // per XCD-order slot and at least 2048 workgroups
  m->lev_grid[0] = m->kry_grid;
  m->nlev = 1;
  if (m->sepred && m->K > 1)
    while (m->nlev < hsm_sim::kLevels && m->lev_grid[m->nlev - 1] / 2 >= 2048) {
      m->lev_grid[m->nlev] = (m->lev_grid[m->nlev - 1] / 2 + kXcds - 1) / kXcds * kXcds;
      ++m->nlev;
    }
  m->known_nact = m->nkblk;
  if ((rc = m->active.alloc(sizeof(int32_t) * (m->nkblk + 1)))) return rc;
  if ((rc = m->dom.alloc(sizeof(DomState) * m->K)) || (rc = m->dom_nodes.alloc(sizeof(int64_t) * m->K)) ||
      (rc = m->bscale.alloc(sizeof(double) * m->K)))
    return rc;
  HSM_HIP(hipMemsetAsync(m->dom.p, 0, sizeof(DomState) * m->K, us));
  if ((rc = m->lpv.alloc(sizeof(DomLaunch) * m->K)) || (rc = m->lst.alloc(sizeof(DomLaunch) * m->K))) return rc;
  HSM_HIP(hipMemsetAsync(m->lpv.p, 0, sizeof(DomLaunch) * m->K, us));
  HSM_HIP(hipMemsetAsync(m->lst.p, 0, sizeof(DomLaunch) * m->K, us));
  {
    // the zero-mean border of domain k holds c_k = 1/sqrt(N_k): the same
    // constraint as a border of ones, with the border's eigenvalue pair at
    // +-1 instead of +-sqrt(N_k)
    std::vector<int64_t> dn(m->K);
    std::vector<double> bs(m->K);
    for (int32_t d2 = 0; d2 < m->K; ++d2) {
      dn[d2] = st->dom_off[d2 + 1] - st->dom_off[d2];
      bs[d2] = 1.0 / std::sqrt((double)dn[d2]);
    }
    HSM_HIP(hipMemcpyAsync(m->dom_nodes.p, dn.data(), sizeof(int64_t) * m->K, hipMemcpyHostToDevice, us));
    HSM_HIP(hipMemcpyAsync(m->bscale.p, bs.data(), sizeof(double) * m->K, hipMemcpyHostToDevice, us));
    HSM_HIP(hipStreamSynchronize(us));
  }
  if ((rc = m->partR.alloc(sizeof(double) * kNR * (m->nblk + 1))) ||
      (rc = m->partA.alloc(sizeof(double) * kNA * (m->nkblk + 1))) ||
      (rc = m->partB.alloc(sizeof(double) * kNB * (m->nkblk + 1))))
    return rc;
  const int32_t *perm = st->perm.as<int32_t>();
  for (int c = 0; c < d; ++c) {
    if (m->f32)
      hipLaunchKernelGGL((k_gather<double, float>), dim3(nblk(N, 256)), dim3(256), 0, us, v + c * N,
                         m->v.as<float>() + c * N, perm, N);
    else
      hipLaunchKernelGGL((k_gather<double, double>), dim3(nblk(N, 256)), dim3(256), 0, us, v + c * N,
                         m->v.as<double>() + c * N, perm, N);
  }
  if (m->f32)
    hipLaunchKernelGGL((k_gather<double, float>), dim3(nblk(N, 256)), dim3(256), 0, us, T, m->T[0].as<float>(), perm, N);
  else
    hipLaunchKernelGGL((k_gather<double, double>), dim3(nblk(N, 256)), dim3(256), 0, us, T, m->T[0].as<double>(), perm,
                       N);
  for (auto &b : m->vec) hipLaunchKernelGGL(k_fill, dim3(nblk(NK, 256)), dim3(256), 0, us, b.as<double>(), NK, 0.0);
  for (auto &b : m->pairs)
    hipLaunchKernelGGL(k_fill, dim3(nblk(2 * NK, 256)), dim3(256), 0, us, b.as<double>(), 2 * NK, 0.0);
  if (p) hipLaunchKernelGGL((k_gather<double, double>), dim3(nblk(N, 256)), dim3(256), 0, us, p, m->x, perm, N);
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
  const dim3 g(nblk(N, 256)), b(256);
  if (v)
    for (int c = 0; c < m->d; ++c) {
      if (m->f32) hipLaunchKernelGGL((k_gather<float, double>), g, b, 0, us, m->v.as<float>() + c * N, v + c * N, ip, N);
      else hipLaunchKernelGGL((k_gather<double, double>), g, b, 0, us, m->v.as<double>() + c * N, v + c * N, ip, N);
    }
  if (T) {
    if (m->f32) hipLaunchKernelGGL((k_gather<float, double>), g, b, 0, us, m->T[m->parity].as<float>(), T, ip, N);
    else hipLaunchKernelGGL((k_gather<double, double>), g, b, 0, us, m->T[m->parity].as<double>(), T, ip, N);
  }
  if (p) hipLaunchKernelGGL((k_gather<double, double>), g, b, 0, us, (const double *)m->x, p, ip, N);
  HSM_HIP(hipGetLastError());
  return HSM_OK;
}

hsm_status hsm_sim_phase_times(hsm_sim *m, double *host_mean_ms, int64_t *host_count) {
  if (!m || !host_mean_ms || !host_count) { set_error(HSM_E_INVALID, "NULL argument"); return HSM_E_INVALID; }
  if (!m->prm.profile) { set_error(HSM_E_INVALID, "simulation was not created with profile = 1"); return HSM_E_INVALID; }
  HSM_HIP(hipStreamSynchronize(m->s));
  hsm_status rc = read_post(m);
  if (rc) return rc;
  for (int k = 0; k < HSM_PH_COUNT; ++k) {
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
  info[4] = m->n_shared;
  info[5] = m->nnz_shared;
  return HSM_OK;
}

void hsm_sim_destroy(hsm_sim *m) { delete m; }

}  // extern "C"
