/*
 * bh_oracle.c -- CPU FP64 oracle for the Barnes-Hut tree method of
 * Nakasato, "Implementation of a Parallel Tree Method on a GPU" (arXiv:1112.4539).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or helper with the HIP library and includes nothing of it.
 *
 * Everything is IEEE binary64.  The file must be compiled with
 * -ffp-contract=off so that every a*b+c below is two roundings unless it is an
 * explicit fma() call.
 *
 * What each part follows:
 *   direct sum ............ Sec. 3, Eq. (1): softened pairwise gravity, j != i.
 *                           Sign conventions: the acceleration points from x_i
 *                           toward x_j (attractive; the appendix kernel forms
 *                           x_j - x_i), the potential is the physical -sum m/r.
 *   tree construction ..... Sec. 4.1: the enclosing cube is cut into eight equal
 *                           sub-cells recursively until a cell holds zero or one
 *                           particle.  Cells are cut on a 2^21 integer grid of the
 *                           root cube (the Morton grid of Sec. 5), so the cut
 *                           cannot go on forever for coincident particles: a
 *                           level-21 cell keeps all its particles (bucket leaf).
 *                           A cell whose particles all fall in one sub-cell is
 *                           replaced by that sub-cell (compressed octree).
 *   cell moments .......... Sec. 4.4: cell mass = total mass, cell position = the
 *                           centre of mass (monopole only).
 *   opening criterion ..... Sec. 4.4, Eq. (2) and the S_effective equation:
 *                           accept a cell iff d^2 > (l/theta + s)^2, l the side of
 *                           the cell, s the distance from the cell's geometric
 *                           centre to its centre of mass, d the distance from the
 *                           particle to the centre of mass.
 *   tree walk ............. Sec. 4.1, Fig. 3 (recursive treewalk): a one-particle
 *                           cell gives a particle-particle term, an accepted cell a
 *                           particle-cell term with the same softened kernel, any
 *                           other cell is opened and its sub-cells walked in order.
 *   next pointers ......... Sec. 4.4 (next/more): nodes are numbered in depth-first
 *                           preorder, children in octant order, so more(c) = c+1
 *                           and next(c) = the first node after c's subtree.
 *   error statistics ...... Sec. 5, Eq. (4) (mean relative error) and its RMS form.
 *   neighbour search ...... Sec. 4.3, Fig. 4 (general tree walk): proc_particle
 *                           records a particle within the search radius,
 *                           distance_test skips a cell whose cube lies wholly
 *                           outside the search ball, proc_cell does nothing.  The
 *                           per-neighbour work here is the SPH density sum with
 *                           the M4 cubic spline kernel (Monaghan & Lattanzio 1985).
 *   time loop ............. Sec. 1: forces, then orbit integration, repeated.  The
 *                           integrator is the kick-drift-kick leapfrog on the
 *                           direct-sum forces.
 *   quadrupole cell term .. Sec. 4.1 allows any higher moment in the particle-cell
 *                           term and Sec. 7 names higher multipoles as the next
 *                           step.  Order 2 here is the second-order Taylor
 *                           expansion, about the cell's centre of mass, of the
 *                           softened potential of Eq. (1) summed over the cell's
 *                           particles; it needs the cell's second moments
 *                           B_ab = sum_j m_j y_a y_b, y = x_j - com (definition
 *                           evaluated directly over the cell's particles).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_LEVELS 21                 /* bits per axis of the integer grid */
#define ORC_GRID (1u << ORC_LEVELS)   /* 2^21 cells per axis at the finest level */

/* ------------------------------------------------------------------------- */
/* Direct O(N^2) sum, Eq. (1).                                               */
/* ------------------------------------------------------------------------- */

/* One softened pair term: source (xj, mj) acting on target xi.
 * r2 = |xj - xi|^2 + eps^2, acc += mj (xj - xi) / r2^(3/2), pot -= mj / r2^(1/2).
 * A pair with r2 == 0 (coincident and unsoftened) contributes nothing.
 * amag accumulates |term| so callers can judge cancellation. */
static void orc_pair(const double *xi, const double *xj, double mj, double eps2,
                     double *acc, double *pot, double *amag) {
  double dx = xj[0] - xi[0];
  double dy = xj[1] - xi[1];
  double dz = xj[2] - xi[2];
  double r2 = dx * dx + dy * dy + dz * dz + eps2;
  if (r2 == 0.0) return;
  double rinv = 1.0 / sqrt(r2);
  double mr3 = mj * (rinv * rinv * rinv);
  acc[0] += mr3 * dx;
  acc[1] += mr3 * dy;
  acc[2] += mr3 * dz;
  *pot -= mj * rinv;
  *amag += fabs(mr3) * sqrt(dx * dx + dy * dy + dz * dz);
}

/* Particle-cell term to second order: the Taylor expansion about the centre of
 * mass `com` of sum_j m_j g(x_i - x_j), g(r) = -(|r|^2 + eps^2)^(-1/2), over
 * the cell's particles, with M = sum m_j, the first moment zero about com, and
 * second moments B (xx xy xz yy yz zz), T = trace B.  With d = com - x_i,
 * rho^2 = |d|^2 + eps^2, and dBd = d.B.d:
 *   pot = -M/rho + (T/rho^3 - 3 dBd/rho^5) / 2
 *   acc = M d/rho^3 - 3 (B d)/rho^5 + (15/2 dBd/rho^7 - 3/2 T/rho^5) d
 * (the second derivatives of g give delta_ab rho^-3 - 3 r_a r_b rho^-5; the
 * acceleration is minus the gradient of pot in x_i).  amag gets |acc|. */
static void orc_pair_quad(const double *xi, const double *cm, double M, const double *B, double eps2,
                          double *acc, double *pot, double *amag) {
  double d[3] = {cm[0] - xi[0], cm[1] - xi[1], cm[2] - xi[2]};
  double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2;
  if (r2 == 0.0) return;
  double ri = 1.0 / sqrt(r2);
  double ri2 = ri * ri;
  double ri3 = ri * ri2;
  double ri5 = ri3 * ri2;
  double ri7 = ri5 * ri2;
  double Bd[3] = {B[0] * d[0] + B[1] * d[1] + B[2] * d[2],
                  B[1] * d[0] + B[3] * d[1] + B[4] * d[2],
                  B[2] * d[0] + B[4] * d[1] + B[5] * d[2]};
  double dBd = d[0] * Bd[0] + d[1] * Bd[1] + d[2] * Bd[2];
  double T = B[0] + B[3] + B[5];
  double f[3];
  for (int k = 0; k < 3; ++k)
    f[k] = M * ri3 * d[k] - 3.0 * ri5 * Bd[k] + (7.5 * dBd * ri7 - 1.5 * T * ri5) * d[k];
  acc[0] += f[0];
  acc[1] += f[1];
  acc[2] += f[2];
  *pot += -M * ri + 0.5 * (T * ri3 - 3.0 * dBd * ri5);
  *amag += sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
}

/* One cell term of order 2 for a given centre of mass, mass and second moments
 * (no tree): used to test the expansion against the exact sum it approximates. */
void orc_cell_term(const double *xi, const double *cm, double M, const double *B, double eps, int order,
                   double *acc, double *pot) {
  double a[3] = {0, 0, 0}, p = 0, am = 0;
  if (order == 2) orc_pair_quad(xi, cm, M, B, eps * eps, a, &p, &am);
  else orc_pair(xi, cm, M, eps * eps, a, &p, &am);
  acc[0] = a[0]; acc[1] = a[1]; acc[2] = a[2];
  *pot = p;
}

/* Direct sum over all j != i (ascending original index) for each target.
 * pos: [n][3], mass: [n]; targets: nt indices (NULL = all n, in order).
 * acc: [nt][3], pot: [nt], amag: [nt] (may be NULL). */
int orc_direct(const double *pos, const double *mass, int64_t n,
               const int64_t *targets, int64_t nt, double eps,
               double *acc, double *pot, double *amag) {
  if (n < 0 || nt < 0 || eps < 0) return -1;
  double eps2 = eps * eps;
  int64_t t;
#pragma omp parallel for schedule(dynamic, 16)
  for (t = 0; t < nt; ++t) {
    int64_t i = targets ? targets[t] : t;
    double a[3] = {0, 0, 0}, p = 0, am = 0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      orc_pair(pos + 3 * i, pos + 3 * j, mass[j], eps2, a, &p, &am);
    }
    acc[3 * t] = a[0];
    acc[3 * t + 1] = a[1];
    acc[3 * t + 2] = a[2];
    pot[t] = p;
    if (amag) amag[t] = am;
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Tree construction (Sec. 4.1) and moments (Sec. 4.4).                       */
/* ------------------------------------------------------------------------- */

typedef struct {
  int64_t n, n_nodes, cap;
  double lo[3], L;
  const double *pos, *mass;  /* caller's arrays, original order */
  uint32_t *q;               /* [n][3] integer grid coordinates */
  /* per node, depth-first preorder */
  int32_t *level, *first, *count, *next;
  int8_t *leaf;
  int64_t *cell;             /* [node][3] integer cell coordinates at its level */
  double *com, *Mx;          /* [node][3] */
  double *B;                 /* [node][6] second moments about the centre of mass: xx xy xz yy yz zz */
  double *M, *s, *l;
  /* particle order */
  int64_t *perm;             /* sorted position -> original index (leaf order) */
  int64_t *rank;             /* original index -> sorted position */
  int64_t *tmp;              /* scratch for the stable partition */
  int64_t placed;            /* particles emitted into perm so far */
} otree;

static int orc_grow(otree *t) {
  if (t->n_nodes < t->cap) return 0;
  int64_t cap = t->cap ? 2 * t->cap : 64;
#define GROW(f, T, k) do { void *p_ = realloc(t->f, (size_t)cap * (k) * sizeof(T)); if (!p_) return -1; t->f = (T *)p_; } while (0)
  GROW(level, int32_t, 1); GROW(first, int32_t, 1); GROW(count, int32_t, 1);
  GROW(next, int32_t, 1); GROW(leaf, int8_t, 1); GROW(cell, int64_t, 3);
  GROW(com, double, 3); GROW(Mx, double, 3); GROW(M, double, 1); GROW(B, double, 6);
  GROW(s, double, 1); GROW(l, double, 1);
#undef GROW
  t->cap = cap;
  return 0;
}

/* octant of particle i among the children of a cell at `level`:
 * 4*bx + 2*by + bz, b_d the grid bit that selects the child half on axis d. */
static int orc_octant(const otree *t, int64_t i, int level) {
  int b = ORC_LEVELS - 1 - level;
  const uint32_t *q = t->q + 3 * i;
  return (int)(((q[0] >> b) & 1u) << 2 | ((q[1] >> b) & 1u) << 1 | ((q[2] >> b) & 1u));
}

/* Build the subtree for the particles idx[0..cnt) that lie in the cell
 * (level, c).  Returns the node id or -1 on allocation failure. */
static int64_t orc_build_rec(otree *t, int level, int64_t cx, int64_t cy, int64_t cz,
                             int64_t *idx, int64_t cnt) {
  /* A cell whose particles all lie in one sub-cell is replaced by that sub-cell. */
  while (cnt >= 2 && level < ORC_LEVELS) {
    int o0 = orc_octant(t, idx[0], level), same = 1;
    for (int64_t k = 1; k < cnt && same; ++k) same = orc_octant(t, idx[k], level) == o0;
    if (!same) break;
    cx = 2 * cx + ((o0 >> 2) & 1);
    cy = 2 * cy + ((o0 >> 1) & 1);
    cz = 2 * cz + (o0 & 1);
    ++level;
  }
  if (orc_grow(t)) return -1;
  int64_t id = t->n_nodes++;
  t->level[id] = level;
  t->cell[3 * id] = cx;
  t->cell[3 * id + 1] = cy;
  t->cell[3 * id + 2] = cz;
  t->first[id] = (int32_t)t->placed;
  t->count[id] = (int32_t)cnt;
  if (cnt == 1 || level == ORC_LEVELS) {
    /* leaf: one particle, or a finest-grid cell holding coincident keys */
    t->leaf[id] = 1;
    for (int64_t k = 0; k < cnt; ++k) t->perm[t->placed++] = idx[k];
    t->next[id] = (int32_t)(id + 1);
    return id;
  }
  t->leaf[id] = 0;
  /* stable partition of idx by octant (input order kept inside each octant) */
  int64_t start[9] = {0};
  for (int64_t k = 0; k < cnt; ++k) start[orc_octant(t, idx[k], level) + 1]++;
  for (int o = 0; o < 8; ++o) start[o + 1] += start[o];
  int64_t fill[8];
  for (int o = 0; o < 8; ++o) fill[o] = start[o];
  int64_t *scratch = t->tmp;  /* the caller guarantees it is at least cnt long */
  for (int64_t k = 0; k < cnt; ++k) scratch[fill[orc_octant(t, idx[k], level)]++] = idx[k];
  memcpy(idx, scratch, (size_t)cnt * sizeof(int64_t));
  for (int o = 0; o < 8; ++o) {
    int64_t c = start[o + 1] - start[o];
    if (c == 0) continue;
    if (orc_build_rec(t, level + 1, 2 * cx + ((o >> 2) & 1), 2 * cy + ((o >> 1) & 1),
                      2 * cz + (o & 1), idx + start[o], c) < 0)
      return -1;
  }
  t->next[id] = (int32_t)t->n_nodes;
  return id;
}

void orc_tree_free(otree *t) {
  if (!t) return;
  free(t->q); free(t->level); free(t->first); free(t->count); free(t->next);
  free(t->leaf); free(t->cell); free(t->com); free(t->Mx); free(t->M); free(t->B);
  free(t->s); free(t->l); free(t->perm); free(t->rank); free(t->tmp);
  free(t);
}

/* Build the tree of n particles.  pos [n][3] and mass [n] must stay alive for
 * as long as the tree is used (the walk reads them).  Returns NULL on failure. */
otree *orc_tree_build(const double *pos, const double *mass, int64_t n) {
  if (n < 0) return NULL;
  otree *t = (otree *)calloc(1, sizeof(otree));
  if (!t) return NULL;
  t->n = n;
  t->pos = pos;
  t->mass = mass;
  size_t nn = (size_t)(n > 0 ? n : 1);
  t->q = (uint32_t *)malloc(nn * 3 * sizeof(uint32_t));
  t->perm = (int64_t *)malloc(nn * sizeof(int64_t));
  t->rank = (int64_t *)malloc(nn * sizeof(int64_t));
  t->tmp = (int64_t *)malloc(nn * sizeof(int64_t));
  int64_t *idx = (int64_t *)malloc(nn * sizeof(int64_t));
  if (!t->q || !t->perm || !t->rank || !t->tmp || !idx) { free(idx); orc_tree_free(t); return NULL; }

  /* Root cube: lower corner = coordinate-wise minimum, side = largest extent
   * (1 when every particle coincides). */
  double hi[3];
  for (int d = 0; d < 3; ++d) { t->lo[d] = n ? pos[d] : 0.0; hi[d] = t->lo[d]; }
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) {
      double v = pos[3 * i + d];
      if (v < t->lo[d]) t->lo[d] = v;
      if (v > hi[d]) hi[d] = v;
    }
  double L = 0.0;
  for (int d = 0; d < 3; ++d) { double e = hi[d] - t->lo[d]; if (e > L) L = e; }
  if (L == 0.0) L = 1.0;
  t->L = L;

  /* Integer grid coordinate of every particle on the 2^21 grid of the cube. */
  double scale = (double)ORC_GRID / L;
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) {
      double v = floor((pos[3 * i + d] - t->lo[d]) * scale);
      if (v < 0.0) v = 0.0;
      if (v > (double)(ORC_GRID - 1)) v = (double)(ORC_GRID - 1);
      t->q[3 * i + d] = (uint32_t)v;
    }

  for (int64_t i = 0; i < n; ++i) idx[i] = i;
  if (n > 0 && orc_build_rec(t, 0, 0, 0, 0, idx, n) < 0) { free(idx); orc_tree_free(t); return NULL; }
  free(idx);
  for (int64_t k = 0; k < n; ++k) t->rank[t->perm[k]] = k;

  /* Moments, children before parents (reverse preorder).  Sums are left folds:
   * particles of a leaf in sorted order, children of a cell in octant order. */
  for (int64_t c = t->n_nodes - 1; c >= 0; --c) {
    double M = 0, X[3] = {0, 0, 0};
    if (t->leaf[c]) {
      for (int64_t k = t->first[c]; k < (int64_t)t->first[c] + t->count[c]; ++k) {
        int64_t j = t->perm[k];
        M += mass[j];
        for (int d = 0; d < 3; ++d) X[d] += mass[j] * pos[3 * j + d];
      }
    } else {
      for (int64_t ch = c + 1; ch < t->next[c]; ch = t->next[ch]) {
        M += t->M[ch];
        for (int d = 0; d < 3; ++d) X[d] += t->Mx[3 * ch + d];
      }
    }
    t->M[c] = M;
    for (int d = 0; d < 3; ++d) t->Mx[3 * c + d] = X[d];
    double l = ldexp(L, -t->level[c]);
    t->l[c] = l;
    double ctr[3];
    for (int d = 0; d < 3; ++d) ctr[d] = t->lo[d] + ((double)t->cell[3 * c + d] + 0.5) * l;
    if (t->leaf[c] && t->count[c] == 1) {
      /* a one-particle cell sits at its particle */
      int64_t j = t->perm[t->first[c]];
      for (int d = 0; d < 3; ++d) t->com[3 * c + d] = pos[3 * j + d];
    } else {
      for (int d = 0; d < 3; ++d) t->com[3 * c + d] = M != 0.0 ? X[d] / M : ctr[d];
    }
    if (t->leaf[c]) {
      t->s[c] = 0.0;
    } else {
      double dx = ctr[0] - t->com[3 * c];
      double dy = ctr[1] - t->com[3 * c + 1];
      double dz = ctr[2] - t->com[3 * c + 2];
      t->s[c] = sqrt(fma(dz, dz, fma(dy, dy, dx * dx)));
    }
  }
  /* Second moments about each node's centre of mass, straight from the
   * definition: B_ab = sum over the node's particles of m (x_a - com_a)(x_b - com_b),
   * particles in sorted order.  (A one-particle leaf has B = 0 exactly.) */
  int64_t cc;
#pragma omp parallel for schedule(dynamic, 256)
  for (cc = 0; cc < t->n_nodes; ++cc) {
    double b[6] = {0, 0, 0, 0, 0, 0};
    const double *cm = t->com + 3 * cc;
    for (int64_t k = t->first[cc]; k < (int64_t)t->first[cc] + t->count[cc]; ++k) {
      int64_t j = t->perm[k];
      double y0 = pos[3 * j] - cm[0], y1 = pos[3 * j + 1] - cm[1], y2 = pos[3 * j + 2] - cm[2];
      double m = mass[j];
      b[0] += m * y0 * y0; b[1] += m * y0 * y1; b[2] += m * y0 * y2;
      b[3] += m * y1 * y1; b[4] += m * y1 * y2; b[5] += m * y2 * y2;
    }
    if (t->leaf[cc] && t->count[cc] == 1) for (int a = 0; a < 6; ++a) b[a] = 0.0;
    for (int a = 0; a < 6; ++a) t->B[6 * cc + a] = b[a];
  }
  return t;
}

/* Second moments [n_nodes][6] (xx xy xz yy yz zz) about each node's centre of mass. */
void orc_tree_quad(const otree *t, double *B) {
  memcpy(B, t->B, (size_t)t->n_nodes * 6 * sizeof(double));
}

int64_t orc_tree_nodes(const otree *t) { return t ? t->n_nodes : -1; }

/* Root cube: lo[3], L. */
void orc_tree_cube(const otree *t, double *lo, double *L) {
  for (int d = 0; d < 3; ++d) lo[d] = t->lo[d];
  *L = t->L;
}

/* Copy the node arrays (preorder) and the particle order out.  Any pointer may
 * be NULL.  cell/com are [n_nodes][3]; perm is [n]. */
void orc_tree_export(const otree *t, int32_t *level, int32_t *first, int32_t *count,
                     int32_t *next, int8_t *leaf, int64_t *cell, double *com, double *M,
                     double *s, double *l, int64_t *perm) {
  int64_t m = t->n_nodes;
  if (level) memcpy(level, t->level, (size_t)m * sizeof(int32_t));
  if (first) memcpy(first, t->first, (size_t)m * sizeof(int32_t));
  if (count) memcpy(count, t->count, (size_t)m * sizeof(int32_t));
  if (next) memcpy(next, t->next, (size_t)m * sizeof(int32_t));
  if (leaf) memcpy(leaf, t->leaf, (size_t)m * sizeof(int8_t));
  if (cell) memcpy(cell, t->cell, (size_t)m * 3 * sizeof(int64_t));
  if (com) memcpy(com, t->com, (size_t)m * 3 * sizeof(double));
  if (M) memcpy(M, t->M, (size_t)m * sizeof(double));
  if (s) memcpy(s, t->s, (size_t)m * sizeof(double));
  if (l) memcpy(l, t->l, (size_t)m * sizeof(double));
  if (perm) memcpy(perm, t->perm, (size_t)t->n * sizeof(int64_t));
}

/* ------------------------------------------------------------------------- */
/* Tree walk, Fig. 3 with the opening test of Eq. (2)/(3).                    */
/* ------------------------------------------------------------------------- */

/* Interaction-list word: a particle-particle entry is (original index << 1),
 * a particle-cell entry is (preorder node id << 1) | 1.  The ordered list of a
 * particle is summarised by a 64-bit FNV-1a style hash taken over these words:
 * h = (h xor word) * 1099511628211, starting from 14695981039346656037. */
#define ORC_FNV_OFFSET 14695981039346656037ull
#define ORC_FNV_PRIME 1099511628211ull

typedef struct {
  const otree *t;
  int64_t i;           /* target, original index */
  int64_t ri;          /* its sorted position */
  const double *xi;
  double inv_theta, eps2;
  int order;           /* 1: monopole cell terms (Eq. (1)), 2: with the quadrupole correction */
  double a[3], p, amag;
  int64_t n_pp, n_pc;
  uint64_t hash;
  int64_t *list;       /* optional dump, entries as above (truncated to maxlen) */
  int64_t maxlen, len;
} orc_walker;

static void orc_record(orc_walker *w, uint64_t word) {
  w->hash = (w->hash ^ word) * ORC_FNV_PRIME;
  if (w->list && w->len < w->maxlen) w->list[w->len] = (int64_t)word;
  w->len++;
}

static void orc_treewalk(orc_walker *w, int64_t c) {
  const otree *t = w->t;
  if (t->leaf[c]) {
    /* particle-particle terms with every particle of the cell except i itself */
    for (int64_t k = t->first[c]; k < (int64_t)t->first[c] + t->count[c]; ++k) {
      int64_t j = t->perm[k];
      if (j == w->i) continue;
      orc_pair(w->xi, t->pos + 3 * j, t->mass[j], w->eps2, w->a, &w->p, &w->amag);
      w->n_pp++;
      orc_record(w, (uint64_t)j << 1);
    }
    return;
  }
  int inside = w->ri >= t->first[c] && w->ri < (int64_t)t->first[c] + t->count[c];
  if (!inside) {
    const double *cm = t->com + 3 * c;
    double dx = cm[0] - w->xi[0];
    double dy = cm[1] - w->xi[1];
    double dz = cm[2] - w->xi[2];
    double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
    double u = fma(t->l[c], w->inv_theta, t->s[c]);  /* l/theta + s */
    if (d2 > u * u) {
      if (w->order == 2)
        orc_pair_quad(w->xi, cm, t->M[c], t->B + 6 * c, w->eps2, w->a, &w->p, &w->amag);
      else
        orc_pair(w->xi, cm, t->M[c], w->eps2, w->a, &w->p, &w->amag);
      w->n_pc++;
      orc_record(w, ((uint64_t)c << 1) | 1u);
      return;
    }
  }
  for (int64_t ch = c + 1; ch < t->next[c]; ch = t->next[ch]) orc_treewalk(w, ch);
}

/* Walk the tree for each target (original indices; NULL = all n in order).
 * theta_per_target (nt values, may be NULL) overrides theta.  order 1 uses
 * monopole cell terms, order 2 adds the quadrupole correction (the opening
 * test and so the lists are the same for both).  Outputs per
 * target: acc [3], pot, amag (sum of |term|), n_pp, n_pc, hash; any may be
 * NULL.  lists (optional) is [nt][maxlen] of int64 words (truncated). */
int orc_walk(const otree *t, const int64_t *targets, int64_t nt, double theta,
             const double *theta_per_target, double eps, int order, double *acc, double *pot,
             double *amag, int64_t *n_pp, int64_t *n_pc, uint64_t *hash,
             int64_t *lists, int64_t maxlen) {
  if (!t || nt < 0 || eps < 0 || (order != 1 && order != 2)) return -1;
  int64_t k;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(| : bad)
  for (k = 0; k < nt; ++k) {
    orc_walker w;
    memset(&w, 0, sizeof w);
    w.t = t;
    w.i = targets ? targets[k] : k;
    if (w.i < 0 || w.i >= t->n) { bad = 1; continue; }
    w.ri = t->rank[w.i];
    w.xi = t->pos + 3 * w.i;
    double th = theta_per_target ? theta_per_target[k] : theta;
    w.inv_theta = 1.0 / th;
    w.eps2 = eps * eps;
    w.order = order;
    w.hash = ORC_FNV_OFFSET;
    w.list = lists ? lists + k * maxlen : NULL;
    w.maxlen = maxlen;
    if (t->n_nodes > 0) orc_treewalk(&w, 0);
    if (acc) { acc[3 * k] = w.a[0]; acc[3 * k + 1] = w.a[1]; acc[3 * k + 2] = w.a[2]; }
    if (pot) pot[k] = w.p;
    if (amag) amag[k] = w.amag;
    if (n_pp) n_pp[k] = w.n_pp;
    if (n_pc) n_pc[k] = w.n_pc;
    if (hash) hash[k] = w.hash;
  }
  return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------- */
/* Neighbour search: the general tree walk of Fig. 4.                        */
/* ------------------------------------------------------------------------- */

/* M4 cubic spline of compact support 2h in three dimensions (Monaghan &
 * Lattanzio 1985): W(r, h) = 1/(pi h^3) * {1 - 3/2 q^2 + 3/4 q^3 for q < 1,
 * (2 - q)^3 / 4 for 1 <= q < 2, 0 beyond}, q = r/h. */
double orc_sph_kernel(double r, double h) {
  double q = r / h;
  double sig = 1.0 / (M_PI * h * h * h);
  if (q < 1.0) return sig * (1.0 - 1.5 * q * q + 0.75 * q * q * q);
  if (q < 2.0) { double u = 2.0 - q; return sig * 0.25 * u * u * u; }
  return 0.0;
}

typedef struct {
  const otree *t;
  int64_t i;
  const double *xi;
  double r2;           /* squared search radius */
  double h;            /* kernel scale: radius / 2 */
  double rho;
  int64_t count;
  uint64_t hash;
  int64_t *list, maxlen, len;
} orc_nbr;

/* proc_particle: j (original index) is a neighbour of i iff j != i and
 * |x_j - x_i|^2 < radius^2 (squared distance as fma(dz,dz,fma(dy,dy,dx*dx))). */
static void orc_nbr_particle(orc_nbr *w, int64_t j) {
  if (j == w->i) return;
  const double *xj = w->t->pos + 3 * j;
  double dx = xj[0] - w->xi[0], dy = xj[1] - w->xi[1], dz = xj[2] - w->xi[2];
  double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
  if (!(d2 < w->r2)) return;
  w->count++;
  w->hash = (w->hash ^ ((uint64_t)j << 1)) * ORC_FNV_PRIME;
  if (w->list && w->len < w->maxlen) w->list[w->len] = (int64_t)j;
  w->len++;
  w->rho += w->t->mass[j] * orc_sph_kernel(sqrt(d2), w->h);
}

/* distance_test: the cell's cube [lo + cell l, lo + (cell + 1) l) cannot hold a
 * point within the radius iff its nearest point to x_i is at least the radius
 * away. */
static int orc_cell_far(const orc_nbr *w, int64_t c) {
  const otree *t = w->t;
  double l = t->l[c], d2 = 0.0;
  for (int d = 0; d < 3; ++d) {
    double lo = t->lo[d] + (double)t->cell[3 * c + d] * l, hi = lo + l, x = w->xi[d], e = 0.0;
    if (x < lo) e = lo - x;
    else if (x > hi) e = x - hi;
    d2 += e * e;
  }
  return d2 >= w->r2;
}

static void orc_nbrwalk(orc_nbr *w, int64_t c) {
  const otree *t = w->t;
  if (t->leaf[c]) {
    for (int64_t k = t->first[c]; k < (int64_t)t->first[c] + t->count[c]; ++k) orc_nbr_particle(w, t->perm[k]);
    return;
  }
  if (orc_cell_far(w, c)) return;
  for (int64_t ch = c + 1; ch < t->next[c]; ch = t->next[ch]) orc_nbrwalk(w, ch);
}

/* Neighbours within `radius` of each target (original indices; NULL = all):
 * count, ordered hash of the neighbours' original indices j (word j << 1, the
 * walk's depth-first order, FNV-1a as for interaction lists), optional lists
 * [nt][maxlen], and the SPH density rho_i = m_i W(0, h) + sum_j m_j W(r_ij, h)
 * with h = radius / 2 (any output may be NULL). */
int orc_neighbours(const otree *t, const int64_t *targets, int64_t nt, double radius, int64_t *count,
                   uint64_t *hash, int64_t *lists, int64_t maxlen, double *rho) {
  if (!t || nt < 0 || !(radius > 0.0)) return -1;
  int64_t k;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
  for (k = 0; k < nt; ++k) {
    orc_nbr w;
    memset(&w, 0, sizeof w);
    w.t = t;
    w.i = targets ? targets[k] : k;
    if (w.i < 0 || w.i >= t->n) { bad = 1; continue; }
    w.xi = t->pos + 3 * w.i;
    w.r2 = radius * radius;
    w.h = 0.5 * radius;
    w.rho = t->mass[w.i] * orc_sph_kernel(0.0, w.h);
    w.hash = ORC_FNV_OFFSET;
    w.list = lists ? lists + k * maxlen : NULL;
    w.maxlen = maxlen;
    if (t->n_nodes > 0) orc_nbrwalk(&w, 0);
    if (count) count[k] = w.count;
    if (hash) hash[k] = w.hash;
    if (rho) rho[k] = w.rho;
  }
  return bad ? -1 : 0;
}

/* Brute force over all pairs: neighbour counts and the density, for the pins. */
int orc_neighbours_brute(const double *pos, const double *mass, int64_t n, const int64_t *targets, int64_t nt,
                         double radius, int64_t *count, double *rho) {
  if (n < 0 || nt < 0 || !(radius > 0.0)) return -1;
  double r2 = radius * radius, h = 0.5 * radius;
  int64_t k;
#pragma omp parallel for schedule(dynamic, 16)
  for (k = 0; k < nt; ++k) {
    int64_t i = targets ? targets[k] : k;
    int64_t cnt = 0;
    double rh = mass[i] * orc_sph_kernel(0.0, h);
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double dx = pos[3 * j] - pos[3 * i], dy = pos[3 * j + 1] - pos[3 * i + 1], dz = pos[3 * j + 2] - pos[3 * i + 2];
      double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
      if (d2 < r2) {
        ++cnt;
        rh += mass[j] * orc_sph_kernel(sqrt(d2), h);
      }
    }
    if (count) count[k] = cnt;
    if (rho) rho[k] = rh;
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Time loop (Sec. 1): forces, orbit integration, repeat.                     */
/* ------------------------------------------------------------------------- */

/* `steps` kick-drift-kick leapfrog steps of size dt on the direct-sum forces
 * of Eq. (1): v += dt/2 a(x); x += dt v; v += dt/2 a(x).  pos, vel [n][3] are
 * advanced in place; acc [n][3] and pot [n] end as the forces at the final
 * positions (acc must hold a(x) of the initial positions on entry). */
int orc_leapfrog(double *pos, double *vel, const double *mass, int64_t n, double eps, double dt, int64_t steps,
                 double *acc, double *pot) {
  if (n < 0 || steps < 0 || eps < 0) return -1;
  for (int64_t s = 0; s < steps; ++s) {
    for (int64_t k = 0; k < 3 * n; ++k) {
      vel[k] += 0.5 * dt * acc[k];
      pos[k] += dt * vel[k];
    }
    if (orc_direct(pos, mass, n, NULL, n, eps, acc, pot, NULL) != 0) return -1;
    for (int64_t k = 0; k < 3 * n; ++k) vel[k] += 0.5 * dt * acc[k];
  }
  return 0;
}

/* Threads the parallel loops use from now on (n >= 1); for timing the oracle on
 * one core beside all of them. */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
