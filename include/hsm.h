/*
 * hsm.h -- C ABI of the MI355X (gfx950) hybrid scattered-regular meshless library.
 *
 * The library implements the hot path of the hybrid method of Jancic, Rot and
 * Kosec, "Spatially-varying meshless approximation method for enhanced
 * computational efficiency" (arXiv 2303.01760):
 *   - per-node stencils and weights of d/dx, d/dy (, d/dz) and the Laplacian,
 *     built once: RBF-FD (PHS r^3 + monomials up to degree m over
 *     n = 2 C(m+d, m) nearest nodes) on scattered nodes, MON (monomials
 *     {1, x_k, x_k^2} over the 2d+1 node axis cross) on regular nodes
 *     (Section 2; Section 2.1 for the local system M w = l);
 *   - the operator approximation of Eq. (1), (L u)(x_c) ~ sum_i w_i u(x_i),
 *     applied many times inside explicit time steps;
 *   - explicit Euler steps of the Boussinesq natural-convection equations
 *     (Eqs. (2)-(4)) with Chorin's pressure projection (Section 3).
 *
 * Every computation runs in hand-written HIP kernels on one GPU.  There is no
 * CPU fallback: without a usable gfx950 device every call that computes
 * returns HSM_E_HIP.
 *
 * Conventions
 *   - Pointers named host_* are host memory; every other array pointer is
 *     device memory (e.g. from torch tensors).  The caller owns all arrays it
 *     passes and must keep them alive for the duration of the call.
 *   - Handles (hsm_stencils, hsm_sim) are owned by the library and released
 *     with the matching *_destroy function.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   - Functions return HSM_OK (0) or a negative hsm_status.  On error
 *     hsm_last_error() gives a message and hsm_last_error_node() the node
 *     (caller numbering) the error refers to, or -1; both are per thread.
 *   - Positions, normals and fields are SoA: component a of node i is at
 *     [a * N + i].
 *   - Node classes: 0 = regular (MON stencil), 1 = scattered (RBF-FD).
 *   - Node kinds (input): 0 = interior, 1 = Dirichlet-T wall, 2 = Neumann-T
 *     (adiabatic) wall.  Every wall node is no-slip for velocity.
 */
#ifndef HSM_H
#define HSM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hsm_status;
enum {
  HSM_OK = 0,
  HSM_E_INVALID = -1,        /* bad argument; nothing was computed */
  HSM_E_SINGULAR = -2,       /* a local system M w = l has no usable pivot */
  HSM_E_DUPLICATE_NODE = -3, /* two nodes of one domain coincide */
  HSM_E_NOT_CONVERGED = -4,  /* pressure Krylov solve hit its iteration cap */
  HSM_E_NONFINITE = -5,      /* a field became Inf/NaN during stepping */
  HSM_E_HIP = -6,            /* HIP runtime error (no device, launch failure) */
  HSM_E_OOM = -7,            /* device allocation failed */
  HSM_E_AMBIGUOUS = -8       /* reserved (no longer returned: crowded nodes are classified exactly) */
};

/* operator bits */
enum { HSM_OP_DX = 1, HSM_OP_DY = 2, HSM_OP_DZ = 4, HSM_OP_LAP = 8, HSM_OP_DN = 16 };
/* data types of fields and weights */
enum { HSM_F64 = 0, HSM_F32 = 1, HSM_F32_COMP = 2 };
/* approximation layout */
enum { HSM_MODE_HYBRID = 0, HSM_MODE_ALL_SCATTERED = 1 };
/* direction of hsm_permute */
enum { HSM_TO_INTERNAL = 0, HSM_TO_CALLER = 1 };

typedef struct hsm_stencils hsm_stencils;
typedef struct hsm_sim hsm_sim;

/* A node set: one or more independent domains stored back to back.
 * Stencils never cross a domain boundary. */
typedef struct {
  int32_t d;                           /* dimension, 2 or 3 */
  int32_t n_domains;                   /* >= 1 */
  const int64_t *host_domain_offsets;  /* [n_domains+1]; domain k = nodes [off[k], off[k+1]) */
  const double *x;                     /* device [d][N] positions */
  const uint8_t *kind;                 /* device [N] 0 interior, 1 Dirichlet-T, 2 Neumann-T */
  const double *normal;                /* device [d][N] outward unit normal (read at wall nodes) */
  const double *host_h_regular;        /* [n_domains] regular lattice spacing h_r (> 0) */
  const int32_t *host_m;               /* [n_domains] monomial degree of RBF-FD stencils */
  const int32_t *host_n;               /* [n_domains] RBF-FD stencil size, or NULL for 2 C(m+d, m) */
  int32_t tile_log2;                   /* internal node order: tiles of 2^tile_log2 search cells per axis
                                          (1..5); 0 for the default (8x8 in 2D, 4x4x4 in 3D) */
  int32_t solve_groups;                /* RBF-FD local systems per wave64: 0 for the most that fit (3 when
                                          the system size is <= 21, 2 when <= 32, else 1); 1, 2 or 3 (capped
                                          at what fits).  The weights do not depend on it. */
} hsm_nodeset;

/* Summary of a built stencil set. */
typedef struct {
  int32_t d, mode, n_domains, n_buckets;
  int64_t n_nodes, nnz;                /* nnz = total stencil entries over all nodes */
  int64_t n_regular, n_scattered;      /* by class */
  int64_t n_boundary;
  int64_t n_wall_fallback;             /* wall nodes solved with monomials of degree m-1 (see below) */
  int32_t bucket_width[16];            /* per width bucket, in internal order */
  int32_t bucket_type[16];             /* 0 regular, 1 scattered interior, 2 Dirichlet wall, 3 Neumann wall */
  int64_t bucket_count[16];
  double build_ms[4];                  /* device time of: neighbour search, classify+order, local solves, total */
  double bucket_solve_ms[16];          /* device time of each bucket's local solves (first pass) */
} hsm_stencils_info;

/*
 * hsm_build_stencils -- stencils and FP64 weights of d/dx_a and the Laplacian
 * at every node (Section 2; Eq. (1); Section 2.1).
 *
 * Stencil selection (text before Eq. (1)): an interior node takes the n nodes
 * of its domain nearest to it, ordered by (squared distance, caller index)
 * with squared distance dx*dx + dy*dy (+ dz*dz) rounded step by step in that
 * order; the node itself comes first.  A wall node takes itself and its n-1
 * nearest interior nodes; if that local system is singular (the interior
 * nodes leave the degree-m monomial block rank-deficient, e.g. all but the
 * wall node on two lattice planes), the wall node uses monomials of degree
 * m-1 on the same stencil (walls need first derivatives only; m >= 2).
 * Classification (Section 2, Fig. 1): in HSM_MODE_HYBRID an interior node is
 * regular if, for each axis a and sign s,
 * exactly one node lies within 1e-6 h_r (max-norm) of x + s h_r e_a; its
 * stencil is then [i, -x, +x, -y, +y (, -z, +z)] with MON weights.  All other
 * nodes (every node in HSM_MODE_ALL_SCATTERED) get RBF-FD weights.  Wall
 * nodes also get normal-derivative weights sum_a n_a w_a (HSM_OP_DN).
 * Weights solve the local system in coordinates centred at the node and
 * scaled by the stencil radius, by LU with partial pivoting.
 *
 * Supported: d = 2 with 1 <= m <= 4, d = 3 with 1 <= m <= 3, and
 * n + C(m+d, d) <= 64 (so 2D m=4 n=30 and 3D m=2 n=20 or 30 fit), and at
 * most HSM_MAX_NODES nodes in total.
 *
 * Scratch memory (cell lists, neighbour lists, prefix-sum workspace) comes
 * in two blocks from a stream-ordered memory pool that the library creates
 * per device on first use; released blocks stay in the pool, up to 4 GiB per
 * device, for the next build, until the process ends.
 *
 * Synchronises `stream`.  Errors: HSM_E_INVALID (arguments, a domain with
 * fewer than n usable nodes), HSM_E_DUPLICATE_NODE,
 * HSM_E_SINGULAR (hsm_last_error_node names the node), HSM_E_OOM, HSM_E_HIP.
 * On success *out is a new handle.
 */
#define HSM_MAX_NODES 268435454LL   /* (N + 1) * 16 bytes stay below 4 GiB */
hsm_status hsm_build_stencils(const hsm_nodeset *nodes, int32_t mode, void *stream, hsm_stencils **out);

hsm_status hsm_stencils_get_info(const hsm_stencils *st, hsm_stencils_info *out);

/*
 * hsm_stencils_export -- copy classes, stencils and weights to host memory in
 * the caller's node numbering (CSR).  host_offsets [N+1]; host_idx [nnz]
 * (caller indices, stencil order); host_w [d+2][nnz] holding d/dx_0..d/dx_{d-1},
 * the Laplacian and the normal derivative (0 at interior nodes).  Any output
 * pointer may be NULL.  Synchronises `stream`.
 */
hsm_status hsm_stencils_export(const hsm_stencils *st, uint8_t *host_class, int64_t *host_offsets,
                               int32_t *host_idx, double *host_w, void *stream);

/*
 * hsm_stencils_export_noalloc -- hsm_stencils_export with no device
 * allocation, for callers that cannot allocate (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Its device
 * temporaries (widths [N], offsets [N+1], indices [nnz], weights
 * [d+2][nnz], prefix-sum workspace; about 4N + 8N + 4 nnz + 8 (d+2) nnz
 * bytes) come from one fixed device array of
 * HSM_EXPORT_NOALLOC_SCRATCH_BYTES that every GPU using the library holds
 * until the process ends; a set needing more (about 1.8M stencil entries in
 * 2D, 1.4M in 3D) is HSM_E_INVALID.  All calls on one GPU share that GPU's
 * array: calls that overlap in time on the same GPU (several host threads
 * or streams) race, and the caller must serialise them.  Same arguments,
 * outputs, synchronisation and other errors as hsm_stencils_export.
 */
#define HSM_EXPORT_NOALLOC_SCRATCH_BYTES (64LL << 20)
hsm_status hsm_stencils_export_noalloc(const hsm_stencils *st, uint8_t *host_class, int64_t *host_offsets,
                                       int32_t *host_idx, double *host_w, void *stream);

/*
 * hsm_stencils_condition -- the stability diagnostic of Section 2.1 (Fig. 2):
 * for every node, the 2-norm condition number kappa(M) = |M|_2 |M^-1|_2 =
 * sigma_max / sigma_min of the local system solved for its weights (the
 * matrix is shared by every operator of the node): the RBF-FD matrix
 * [[A, P], [P^T, 0]] at scattered nodes (monomials of degree m-1 at wall
 * nodes that fell back), the MON matrix of the basis {1, x_a, x_a^2} on the
 * axis cross at regular nodes, both in the local coordinates of the solve
 * (centred at the node, scaled by its stencil radius).  Singular values by
 * one-sided Jacobi.  kappa: device [N] doubles, caller order, written in
 * full (+inf for a system with a zero singular value).  Asynchronous on
 * `stream`.  Errors: HSM_E_INVALID, HSM_E_HIP.
 */
hsm_status hsm_stencils_condition(const hsm_stencils *st, double *kappa, void *stream);

/*
 * hsm_permute -- move a field between the caller's node order and the
 * library's internal order (width buckets; spatially sorted inside each
 * bucket), in which hsm_apply_operator reads and writes fields.
 * dtype HSM_F64 or HSM_F32; src and dst are device [N] and must not overlap.
 * Asynchronous on `stream`.
 */
hsm_status hsm_permute(const hsm_stencils *st, int32_t direction, int32_t dtype, const void *src,
                       void *dst, void *stream);

/*
 * hsm_apply_operator -- Eq. (1) at every node: out_op[i] = sum_j w_op[i][j] u[idx[i][j]]
 * for every operator bit set in op_mask (HSM_OP_DX .. HSM_OP_LAP; HSM_OP_DN
 * only on wall nodes, 0 elsewhere).  u is device [N] and out device
 * [popcount(op_mask)][N], both in internal order, operators in ascending bit
 * order.  dtype: HSM_F64 (FP64 weights and fields), HSM_F32 (FP32 weights
 * and fields, FP32 sums) or HSM_F32_COMP (FP32 weights and fields, products
 * and sums compensated: Ogita-Rump-Oishi Dot2).  u and out must not overlap.
 * Asynchronous on `stream`; only argument errors are returned.
 */
hsm_status hsm_apply_operator(const hsm_stencils *st, uint32_t op_mask, int32_t dtype, const void *u,
                              void *out, void *stream);

/*
 * hsm_apply_operator_buckets -- hsm_apply_operator restricted to the width
 * buckets whose bit is set in bucket_mask (bit k = bucket k of
 * hsm_stencils_info, internal order); the output rows of the other buckets
 * are left as they were.  For per-bucket throughput, and for callers that
 * update one kind of node only.  Same arguments, layouts and errors
 * otherwise; bucket_mask 0 is HSM_E_INVALID.
 */
hsm_status hsm_apply_operator_buckets(const hsm_stencils *st, uint32_t op_mask, int32_t dtype,
                                      uint32_t bucket_mask, const void *u, void *out, void *stream);

/* Number of (operator, node) pairs one hsm_apply_operator call computes. */
int64_t hsm_apply_node_count(const hsm_stencils *st, uint32_t op_mask);

/* Simulation parameters (Section 3).  rho = 1; gravity points along the last
 * axis, g = -e_y (2D) or -e_z (3D); T_Delta = T - T_ref in Eq. (3). */
typedef struct {
  double Ra, Pr, dt, T_ref;
  double krylov_tol;       /* relative residual of the pressure solve, e.g. 1e-12 */
  int32_t krylov_maxiter;  /* iteration cap per step */
  int32_t field_dtype;     /* HSM_F64, or HSM_F32_COMP: see below */
  int32_t krylov_chunk;    /* iterations per device-side batch between convergence checks (0 = 32) */
  int32_t launch_mode;     /* 0: replay captured HIP graphs, 1: launch kernels directly (same kernels) */
  int32_t profile;         /* 1: bracket each phase (pre, Krylov batch, post) with HIP events; see hsm_sim_phase_times */
  int32_t reduce_mode;     /* Krylov dot products: 0 auto, 1 each block reduces all partials, 2 one-block kernel */
  int32_t block_nodes;     /* nodes (threads) per block of the node kernels: 0 (= 256), 64, 128, 256 or 512 */
  int32_t gather_chunk;    /* stencil entries per gather round of the BiCGSTAB p/v kernel: 0 (= 8), 4, 6, 8, 12 */
  int32_t xcd_order;       /* 1: where the dot products use the reduction kernels (several domains, or more
                              than 1024 blocks), each XCD runs one contiguous run of the Krylov kernels' blocks
                              (its L2 then holds the neighbours they gather); 0: consecutive blocks on
                              consecutive XCDs */
  int32_t lattice_rows;    /* 0: a regular bucket whose pressure rows all equal the lattice row (1 at the
                              centre, -1/(2d) on the cross) to 1e-12 stores that one row, read by every node;
                              1: every node keeps its own row (as built) */
  int32_t wide_lanes;      /* threads per node of the Krylov kernels for the non-regular widths: 0 (auto:
                              several, 2..16 so that each takes at most 8 stencil entries, when such nodes are
                              fewer than half of all nodes; else one), 1: one thread per node, 2: several */
} hsm_sim_params;

typedef struct {
  int64_t steps;                 /* steps completed */
  int64_t krylov_iters_total;    /* over all steps */
  int32_t krylov_iters_last;     /* of the last step */
  int32_t status;                /* latched hsm_status of the stepping */
  double last_relres;            /* relative residual reached in the last step */
  int64_t node_applies;          /* (operator, field, node) triples evaluated so far */
  int64_t krylov_node_matvecs;   /* node rows through a pressure matrix-vector product so far */
  int64_t krylov_reduced_batches; /* Krylov batches launched on a grid below the full one (several domains: the
                                     grid follows the shrinking list of unfinished domains' blocks) */
} hsm_sim_stats;

/*
 * Field forms.  HSM_F64: every field, weight and sum in FP64.  HSM_F32_COMP:
 * v, v*, T stored in FP32 and the field operators (advection, diffusion,
 * divergence, heat, Neumann walls) apply FP32 weights with compensated FP32
 * dot products (Dot2), pointwise updates in FP64 before the FP32 store; the
 * pressure problem (its operator, Krylov vectors, reductions and p itself)
 * stays FP64, and so does the pressure gradient's accumulation.  The caller's
 * arrays are FP64 in both forms (converted on create and read).
 */

/*
 * hsm_sim_create -- a simulation state on a stencil set.  v [d][N], T [N] and
 * p [N] (may be NULL for zero) are device arrays in the caller's numbering,
 * copied in; T at Dirichlet nodes is their wall temperature.  The pressure
 * problem of each step is the Poisson equation of the projection with
 * dp/dn = 0 at walls and zero mean in every domain: each domain k of the
 * stencil set has its own border row and column with entries 1/sqrt(N_k)
 * (the zero-mean constraint with a Lagrange multiplier, scaled so that the
 * bordered matrix keeps an O(1) eigenvalue pair), and all domains advance
 * together with the same dt.  Uses `stream` for the copies and synchronises
 * it.
 */
hsm_status hsm_sim_create(const hsm_stencils *st, const hsm_sim_params *prm, const double *v,
                          const double *T, const double *p, void *stream, hsm_sim **out);

/*
 * hsm_step -- advance nsteps explicit Euler steps (Section 3):
 *   v* = v + dt(-(v.grad)v + Pr Lap v - Ra Pr g T_Delta)  (interior), 0 at walls;
 *   Lap p = div(v*) / dt  (interior), dp/dn = 0 (walls), sum p = 0;
 *   v = v* - dt grad p; T = T + dt(-v.grad T + Lap T) with the new v;
 *   Dirichlet walls keep T; Neumann walls take the T that zeroes dT/dn.
 * Work is ordered on `stream` (device-side batches replayed from HIP graphs);
 * the call returns once the work is queued, except that it waits for each
 * step's Krylov convergence flag.  Numerical failures are latched and read
 * by hsm_sim_get_stats.
 */
hsm_status hsm_step(hsm_sim *sim, int32_t nsteps, void *stream);

/* Synchronises and returns the latched status (HSM_OK, HSM_E_NONFINITE, HSM_E_NOT_CONVERGED). */
hsm_status hsm_sim_get_stats(hsm_sim *sim, hsm_sim_stats *out);

/* Copy v [d][N], T [N], p [N] (caller numbering, FP64) out; NULL skips a field. */
hsm_status hsm_sim_read(hsm_sim *sim, double *v, double *T, double *p, void *stream);

/* Phases timed in profile mode, in this order. */
enum { HSM_PH_PRE = 0, HSM_PH_KRYLOV_ITER = 1, HSM_PH_POST = 2, HSM_PH_KRYLOV_TOTAL = 3, HSM_PH_COUNT = 4 };

/*
 * hsm_sim_phase_times -- in profile mode, mean device time (ms) of: the
 * pre-Krylov phase of a step (predictor, pressure right-hand side, initial
 * residual); one BiCGSTAB iteration (its two kernels), from the batches in
 * which every iteration did work (batch time / batch size); the post-Krylov
 * phase (projection, heat, walls); one Krylov batch, over every batch
 * (including the last, partly idle one: with many domains, batch time
 * against krylov_node_matvecs gives the work actually done).  host_count gets
 * the number of steps, iterations, steps and batches behind each mean.  Both arrays [HSM_PH_COUNT], host.
 * Start/stop events bracket each graph launch on the stepper's stream.
 * Synchronises.  HSM_E_INVALID unless created with profile = 1.
 */
hsm_status hsm_sim_phase_times(hsm_sim *sim, double *host_mean_ms, int64_t *host_count);

/* The per-step pressure-operator bytes and node counts behind the timings
 * (host_info: 6 entries): [0] = N, [1] = total stencil entries (nnz),
 * [2] = interior nodes, [3] = Neumann-wall nodes, [4] = regular nodes whose
 * pressure rows are the shared lattice row (see lattice_rows), [5] = their
 * stencil entries. */
hsm_status hsm_sim_sizes(hsm_sim *sim, int64_t *host_info);

void hsm_sim_destroy(hsm_sim *sim);

/*
 * hsm_stream_copy -- plain streaming copy of `bytes` (a multiple of 16, at
 * most 64 GiB) from src to dst on `stream`, one 16-byte element per thread.
 * A measurement aid:
 * it calibrates achievable HBM bandwidth and the hardware byte counters
 * against a kernel whose traffic is known exactly.
 */
hsm_status hsm_stream_copy(const void *src, void *dst, int64_t bytes, void *stream);
void hsm_stencils_destroy(hsm_stencils *st);

const char *hsm_last_error(void);
int64_t hsm_last_error_node(void);

/* Library version string. */
const char *hsm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HSM_H */
