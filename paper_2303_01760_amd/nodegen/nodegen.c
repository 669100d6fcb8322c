/*
 * Seeded synthetic node sets for the hybrid scattered-regular discretisation.
 *
 * This file places nodes and nothing else: it holds none of the method's
 * arithmetic (no neighbour search, no classification, no weights, no
 * operators).  Both the FP64 CPU oracle and the GPU library consume its
 * output, so it is deliberately kept apart from both.
 *
 * The construction follows the paper's description of how a hybrid node set
 * is made (Section 2): fill the box with a regular lattice, remove lattice
 * nodes close to the irregular boundaries, then fill those voids with a
 * scattered (Poisson-disk) node placement.  The paper's own scattered fill
 * algorithm is external to the paper; Bridson's 2007 Poisson-disk sampling
 * (radius h, 30 candidates per active point) stands in for it.  The paper's
 * duck-shaped obstacles exist only as a figure, so circles (2D) and spheres
 * (3D) stand in for them.
 *
 * Layout of the output: positions and normals are SoA [d][N] doubles.
 * Node kinds: 0 interior, 1 Dirichlet-T boundary, 2 Neumann-T boundary.
 * Normals point out of the fluid (into obstacles, away from the box).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t d;             /* 2 or 3 */
  int32_t n_obst;        /* number of circular / spherical obstacles */
  double h;              /* lattice spacing and Poisson-disk radius */
  double wall_band;      /* width of the scattered band along the box walls */
  double obst_band;      /* width of the scattered band around obstacles */
  double rmin, rmax;     /* obstacle radius range (uniform) */
  double gap;            /* minimum gap between obstacles and to the box, in units of h */
  int32_t wall_kind[6];  /* kind of each box face: x-, x+, y-, y+, z-, z+ */
  double wall_T[6];      /* Dirichlet value of each box face */
  double obst_T[2];      /* Dirichlet value of even / odd obstacles */
  int32_t obst_kind;     /* kind of obstacle boundary nodes (1 or 2) */
  int32_t n_candidates;  /* Poisson-disk candidates per active point (30) */
  uint64_t seed;
  int32_t quarters;      /* 2D only, 1: the quarters x<1/2,y<1/2 and x>1/2,y>1/2 are scattered too */
  int32_t split_axis;    /* >= 0: the part x[split_axis] < split_pos is scattered too */
  double split_pos;
  double h_s;            /* 0 < h_s < h: spacing at obstacle surfaces, growing linearly to h over obst_band */
} ng_params;

typedef struct {
  int64_t n, cap;
  int d;
  double *x;        /* [n][d] interleaved while building */
  double *nrm;      /* [n][d] */
  uint8_t *kind;
  double *tbc;
  int8_t *origin;   /* 0 lattice, 1 boundary, 2 scattered fill */
  int32_t *group;   /* -1 fluid, 0..5 box face, 6+i obstacle i */
  int32_t n_obst;
  double *obst;     /* [n_obst][d+1]: centre, radius */
} ng_set;

/* ---- PRNG: splitmix64 seeding, xoshiro256** stream ---- */
typedef struct { uint64_t s[4]; } rng_t;
static uint64_t splitmix64(uint64_t *z) {
  uint64_t r = (*z += 0x9E3779B97F4A7C15ULL);
  r = (r ^ (r >> 30)) * 0xBF58476D1CE4E5B9ULL;
  r = (r ^ (r >> 27)) * 0x94D049BB133111EBULL;
  return r ^ (r >> 31);
}
static void rng_seed(rng_t *g, uint64_t seed) {
  uint64_t z = seed;
  for (int i = 0; i < 4; ++i) g->s[i] = splitmix64(&z);
}
static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
static uint64_t rng_next(rng_t *g) {
  uint64_t *s = g->s;
  uint64_t r = rotl(s[1] * 5, 7) * 9, t = s[1] << 17;
  s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
  s[2] ^= t; s[3] = rotl(s[3], 45);
  return r;
}
static double rng_u01(rng_t *g) { return (double)(rng_next(g) >> 11) * (1.0 / 9007199254740992.0); }

static int push(ng_set *S, const double *p, const double *nrm, int kind, double tbc, int origin, int group) {
  if (S->n == S->cap) {
    int64_t c = S->cap ? S->cap * 2 : 4096;
    double *x = realloc(S->x, sizeof(double) * c * S->d);
    double *nn = realloc(S->nrm, sizeof(double) * c * S->d);
    uint8_t *k = realloc(S->kind, c);
    double *t = realloc(S->tbc, sizeof(double) * c);
    int8_t *o = realloc(S->origin, c);
    int32_t *gr = realloc(S->group, sizeof(int32_t) * c);
    if (!x || !nn || !k || !t || !o || !gr) return -1;
    S->x = x; S->nrm = nn; S->kind = k; S->tbc = t; S->origin = o; S->group = gr; S->cap = c;
  }
  int64_t i = S->n++;
  for (int a = 0; a < S->d; ++a) {
    S->x[i * S->d + a] = p[a];
    S->nrm[i * S->d + a] = nrm ? nrm[a] : 0.0;
  }
  S->kind[i] = (uint8_t)kind; S->tbc[i] = tbc; S->origin[i] = (int8_t)origin; S->group[i] = group;
  return 0;
}

static double dist_surface(const ng_set *S, const double *p, int *which) {
  /* signed distance to the nearest obstacle surface (negative inside) */
  double best = 1e300; int w = -1;
  for (int o = 0; o < S->n_obst; ++o) {
    const double *c = S->obst + o * (S->d + 1);
    double s = 0;
    for (int a = 0; a < S->d; ++a) s += (p[a] - c[a]) * (p[a] - c[a]);
    double v = sqrt(s) - c[S->d];
    if (v < best) { best = v; w = o; }
  }
  if (which) *which = w;
  return best;
}

/* Node spacing at p: h, or with refinement towards the obstacles (h_s > 0)
 * h_s on their surfaces growing linearly to h at distance obst_band. */
static double spacing(const ng_params *P, const ng_set *S, const double *p) {
  if (!(P->h_s > 0) || P->h_s >= P->h || S->n_obst == 0 || !(P->obst_band > 0)) return P->h;
  double f = dist_surface(S, p, NULL) / P->obst_band;
  if (f < 0) f = 0;
  if (f > 1) f = 1;
  return P->h_s + (P->h - P->h_s) * f;
}

/* ---- uniform cell list used only for Poisson-disk rejection ---- */
typedef struct { int d, nc; double cs; int64_t *head, *next; int64_t cap; int64_t ncell; } cgrid;
static void cg_cell(const cgrid *G, const double *p, int *ci) {
  for (int a = 0; a < G->d; ++a) {
    int c = (int)floor(p[a] / G->cs);
    if (c < 0) c = 0;
    if (c >= G->nc) c = G->nc - 1;
    ci[a] = c;
  }
}
static int64_t cg_id(const cgrid *G, const int *ci) {
  int64_t id = 0;
  for (int a = G->d - 1; a >= 0; --a) id = id * G->nc + ci[a];
  return id;
}
static int cg_insert(cgrid *G, int64_t i, const double *p) {
  if (i >= G->cap) {
    int64_t c = G->cap ? G->cap * 2 : 4096;
    while (c <= i) c *= 2;
    int64_t *nx = realloc(G->next, sizeof(int64_t) * c);
    if (!nx) return -1;
    G->next = nx; G->cap = c;
  }
  int ci[3];
  cg_cell(G, p, ci);
  int64_t id = cg_id(G, ci);
  G->next[i] = G->head[id];
  G->head[id] = i;
  return 0;
}
static int cg_far(const cgrid *G, const ng_set *S, const double *p, double r2) {
  int ci[3] = {0, 0, 0}, lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  cg_cell(G, p, ci);
  for (int a = 0; a < G->d; ++a) {
    lo[a] = ci[a] > 0 ? ci[a] - 1 : 0;
    hi[a] = ci[a] < G->nc - 1 ? ci[a] + 1 : G->nc - 1;
  }
  int c[3];
  for (c[2] = (G->d == 3 ? lo[2] : 0); c[2] <= (G->d == 3 ? hi[2] : 0); ++c[2])
    for (c[1] = lo[1]; c[1] <= hi[1]; ++c[1])
      for (c[0] = lo[0]; c[0] <= hi[0]; ++c[0]) {
        for (int64_t j = G->head[cg_id(G, c)]; j >= 0; j = G->next[j]) {
          double s = 0;
          for (int a = 0; a < G->d; ++a) {
            double t = S->x[j * S->d + a] - p[a];
            s += t * t;
          }
          if (s < r2) return 0;
        }
      }
  return 1;
}

static void free_set(ng_set *S) {
  free(S->x); free(S->nrm); free(S->kind); free(S->tbc); free(S->origin); free(S->group); free(S->obst);
  free(S);
}

/* Returns an opaque set, or NULL on invalid parameters / allocation failure. */
/* The two diagonal quarters of the unit square that the quarters layout
 * fills with scattered nodes (points on the dividing lines stay regular). */
static int in_quarters(const double *p) {
  return (p[0] < 0.5 && p[1] < 0.5) || (p[0] > 0.5 && p[1] > 0.5);
}

void *ng_generate(const ng_params *P, int64_t *n_out) {
  *n_out = 0;
  if (!P || (P->d != 2 && P->d != 3) || !(P->h > 0) || P->h > 0.5 || P->n_obst < 0) return NULL;
  if (P->quarters && P->d != 2) return NULL;
  if (P->split_axis < -1 || P->split_axis >= P->d) return NULL;
  if (P->h_s < 0 || P->h_s > P->h) return NULL;
  const int d = P->d;
  const double h = P->h;
  const int nl = (int)llround(1.0 / h); /* lattice: i*h, i = 1 .. nl-1 interior */
  if (fabs(nl * h - 1.0) > 1e-9 || nl < 4) return NULL;
  ng_set *S = calloc(1, sizeof(ng_set));
  if (!S) return NULL;
  S->d = d;
  rng_t g;
  rng_seed(&g, P->seed);

  /* obstacles: rejection-sampled so that they keep a gap to the box and to each other */
  S->obst = calloc((size_t)(P->n_obst > 0 ? P->n_obst : 1) * (d + 1), sizeof(double));
  const double gap = P->gap * h;
  for (int o = 0; o < P->n_obst; ++o) {
    int placed = 0;
    for (int attempt = 0; attempt < 200000 && !placed; ++attempt) {
      double r = P->rmin + (P->rmax - P->rmin) * rng_u01(&g);
      double c[3];
      for (int a = 0; a < d; ++a) c[a] = (r + gap) + (1.0 - 2.0 * (r + gap)) * rng_u01(&g);
      int ok = 1;
      for (int q = 0; q < o && ok; ++q) {
        const double *cq = S->obst + q * (d + 1);
        double s = 0;
        for (int a = 0; a < d; ++a) s += (c[a] - cq[a]) * (c[a] - cq[a]);
        if (sqrt(s) < r + cq[d] + gap) ok = 0;
      }
      if (ok) {
        for (int a = 0; a < d; ++a) S->obst[o * (d + 1) + a] = c[a];
        S->obst[o * (d + 1) + d] = r;
        placed = 1;
      }
    }
    if (!placed) { free_set(S); return NULL; }
    S->n_obst = o + 1;
  }

  /* box-wall boundary nodes: lattice positions on each face, edges and corners excluded */
  const int wall_band_i = (int)llround(P->wall_band / h);
  for (int face = 0; face < 2 * d; ++face) {
    int ax = face / 2, side = face % 2;
    double nrm[3] = {0, 0, 0};
    nrm[ax] = side ? 1.0 : -1.0;
    int other[2], no = 0;
    for (int a = 0; a < d; ++a) if (a != ax) other[no++] = a;
    int kmax = (d == 3) ? nl - 1 : 1;
    for (int k = 1; k <= kmax; ++k)
      for (int j = 1; j <= nl - 1; ++j) {
        double p[3];
        p[ax] = side ? 1.0 : 0.0;
        p[other[0]] = j * h;
        if (d == 3) p[other[1]] = k * h;
        int w;
        if (S->n_obst && dist_surface(S, p, &w) < 0) continue;
        int kind = P->wall_kind[face];
        if (push(S, p, nrm, kind, kind == 1 ? P->wall_T[face] : 0.0, 1, face)) { free_set(S); return NULL; }
      }
  }
  /* obstacle boundary nodes, at the surface spacing */
  const double hb = (P->h_s > 0 && P->h_s < h) ? P->h_s : h;
  for (int o = 0; o < S->n_obst; ++o) {
    const double *c = S->obst + o * (d + 1);
    const double r = c[d];
    double tb = P->obst_T[o % 2];
    if (d == 2) {
      int n = (int)ceil(2.0 * M_PI * r / hb);
      double ph = 2.0 * M_PI * rng_u01(&g);
      for (int k = 0; k < n; ++k) {
        double t = ph + 2.0 * M_PI * k / n;
        double u[2] = {cos(t), sin(t)};
        double p[2] = {c[0] + r * u[0], c[1] + r * u[1]};
        double nrm[2] = {-u[0], -u[1]};
        if (push(S, p, nrm, P->obst_kind, P->obst_kind == 1 ? tb : 0.0, 1, 6 + o)) { free_set(S); return NULL; }
      }
    } else {
      int n = (int)ceil(4.0 * M_PI * r * r / (hb * hb));
      double ph = 2.0 * M_PI * rng_u01(&g);
      const double ga = M_PI * (3.0 - sqrt(5.0));
      for (int k = 0; k < n; ++k) {
        double z = 1.0 - (2.0 * k + 1.0) / n;
        double rho = sqrt(fmax(0.0, 1.0 - z * z));
        double t = ph + ga * k;
        double u[3] = {rho * cos(t), rho * sin(t), z};
        double p[3] = {c[0] + r * u[0], c[1] + r * u[1], c[2] + r * u[2]};
        double nrm[3] = {-u[0], -u[1], -u[2]};
        if (push(S, p, nrm, P->obst_kind, P->obst_kind == 1 ? tb : 0.0, 1, 6 + o)) { free_set(S); return NULL; }
      }
    }
  }
  const int64_t n_boundary = S->n;

  /* regular lattice, minus the scattered bands and the obstacles */
  {
    int kmax = (d == 3) ? nl - 1 : 1;
    for (int k = 1; k <= kmax; ++k)
      for (int j = 1; j <= nl - 1; ++j)
        for (int i = 1; i <= nl - 1; ++i) {
          int idx[3] = {i, j, k};
          int inband = 0;
          for (int a = 0; a < d; ++a)
            if (idx[a] < wall_band_i || idx[a] > nl - wall_band_i) inband = 1;
          double p[3] = {i * h, j * h, k * h};
          if (P->quarters && in_quarters(p)) inband = 1;
          if (P->split_axis >= 0 && p[P->split_axis] < P->split_pos) inband = 1;
          if (inband) continue;
          if (S->n_obst && dist_surface(S, p, NULL) < P->obst_band) continue;
          if (push(S, p, NULL, 0, 0.0, 0, -1)) { free_set(S); return NULL; }
        }
  }

  /* Poisson-disk fill of the bands (Bridson 2007), seeded from the boundary nodes */
  cgrid G;
  memset(&G, 0, sizeof G);
  G.d = d;
  G.cs = h;
  G.nc = (int)ceil(1.0 / h) + 1;
  G.ncell = 1;
  for (int a = 0; a < d; ++a) G.ncell *= G.nc;
  G.head = malloc(sizeof(int64_t) * G.ncell);
  if (!G.head) { free_set(S); return NULL; }
  for (int64_t c = 0; c < G.ncell; ++c) G.head[c] = -1;
  for (int64_t i = 0; i < S->n; ++i)
    if (cg_insert(&G, i, S->x + i * d)) { free(G.head); free(G.next); free_set(S); return NULL; }
  int64_t *active = malloc(sizeof(int64_t) * (S->cap + 16));
  int64_t act_cap = S->cap + 16, nact = 0;
  for (int64_t i = 0; i < n_boundary; ++i) active[nact++] = i;
  const double wb = wall_band_i * h;
  while (nact > 0) {
    int64_t pick = (int64_t)(rng_u01(&g) * nact);
    if (pick >= nact) pick = nact - 1;
    int64_t a0 = active[pick];
    const double r0 = spacing(P, S, S->x + a0 * d);
    int found = 0;
    for (int t = 0; t < P->n_candidates; ++t) {
      double p[3], dir[3], s = 0;
      if (d == 2) {
        double th = 2.0 * M_PI * rng_u01(&g);
        double rr = r0 * sqrt(1.0 + 3.0 * rng_u01(&g));
        dir[0] = rr * cos(th); dir[1] = rr * sin(th);
      } else {
        double z = 2.0 * rng_u01(&g) - 1.0, th = 2.0 * M_PI * rng_u01(&g);
        double rho = sqrt(fmax(0.0, 1.0 - z * z));
        double rr = r0 * cbrt(1.0 + 7.0 * rng_u01(&g));
        dir[0] = rr * rho * cos(th); dir[1] = rr * rho * sin(th); dir[2] = rr * z;
      }
      int inside = 1;
      for (int a = 0; a < d; ++a) {
        p[a] = S->x[a0 * d + a] + dir[a];
        if (!(p[a] > 0.0 && p[a] < 1.0)) inside = 0;
      }
      (void)s;
      if (!inside) continue;
      /* at least half the local spacing from every box face: the face lattice
         keeps the fill away from the faces, but not along the edges where two
         faces meet (their edge nodes are left out), nor between face nodes
         where the local spacing is below the lattice spacing */
      const double rp0 = spacing(P, S, p);
      for (int a = 0; a < d; ++a)
        if (p[a] < 0.5 * rp0 || p[a] > 1.0 - 0.5 * rp0) inside = 0;
      if (!inside) continue;
      /* inside one of the scattered bands? */
      int inband = 0;
      for (int a = 0; a < d; ++a)
        if (p[a] < wb || p[a] > 1.0 - wb) inband = 1;
      if (P->quarters && in_quarters(p)) inband = 1;
      if (P->split_axis >= 0 && p[P->split_axis] < P->split_pos) inband = 1;
      if (S->n_obst) {
        double ds = dist_surface(S, p, NULL);
        if (ds <= 0.0) continue;              /* inside an obstacle */
        if (ds < P->obst_band) inband = 1;
      }
      if (!inband) continue;
      const double rp = spacing(P, S, p);
      if (!cg_far(&G, S, p, rp * rp)) continue;
      if (push(S, p, NULL, 0, 0.0, 2, -1)) { free(active); free(G.head); free(G.next); free_set(S); return NULL; }
      if (cg_insert(&G, S->n - 1, p)) { free(active); free(G.head); free(G.next); free_set(S); return NULL; }
      if (nact == act_cap) {
        act_cap *= 2;
        int64_t *na = realloc(active, sizeof(int64_t) * act_cap);
        if (!na) { free(active); free(G.head); free(G.next); free_set(S); return NULL; }
        active = na;
      }
      active[nact++] = S->n - 1;
      found = 1;
      break;
    }
    if (!found) active[pick] = active[--nact];
  }
  free(active); free(G.head); free(G.next);
  *n_out = S->n;
  return S;
}

/* Copies the generated set out in SoA form; any output pointer may be NULL. */
void ng_copy(void *h, double *x, uint8_t *kind, double *normal, double *tbc, int8_t *origin, int32_t *group) {
  ng_set *S = (ng_set *)h;
  const int64_t n = S->n;
  for (int64_t i = 0; i < n; ++i) {
    for (int a = 0; a < S->d; ++a) {
      if (x) x[a * n + i] = S->x[i * S->d + a];
      if (normal) normal[a * n + i] = S->nrm[i * S->d + a];
    }
    if (kind) kind[i] = S->kind[i];
    if (tbc) tbc[i] = S->tbc[i];
    if (origin) origin[i] = S->origin[i];
    if (group) group[i] = S->group[i];
  }
}

/* Obstacle table: [n_obst][d+1] (centre, radius). Returns n_obst. */
int32_t ng_obstacles(void *h, double *out) {
  ng_set *S = (ng_set *)h;
  if (out) memcpy(out, S->obst, sizeof(double) * S->n_obst * (S->d + 1));
  return S->n_obst;
}

void ng_free(void *h) {
  if (h) free_set((ng_set *)h);
}
