/*
 * bh_oracle.c -- FP64 CPU oracle for the grouped Barnes-Hut oct-tree force.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it; the product path never does.
 * It shares no code, header or constant generator with the GPU library.
 *
 * What it computes (N. Nakasato, "Oct-tree Method on GPU"):
 *   - direct summation of Eq. (1): softened potential and force, with the
 *     attractive sign convention acc_i = sum_j m_j (x_j - x_i)/(r^2+eps^2)^(3/2),
 *     pot_i = -sum_j m_j / (r^2+eps^2)^(1/2), j != i, G = 1;
 *   - the oct-tree of Sec. 3.1: the cube enclosing all particles is split into
 *     eight sub-cells recursively until a cell holds one particle (a cell at the
 *     finest key level, 21, that still holds several particles is a bucket that
 *     is always opened);
 *   - monopole cells (Sec. 3.1): total mass at the centre of mass;
 *   - the modified opening criterion of Eq. (2)/(3): a cell is far enough when
 *     d^2 > (l/theta + s)^2, with l the cell side, s the distance from the
 *     cell's geometric centre to its centre of mass, strict ">" as in the
 *     kernel of Fig. "treegpu";
 *   - Morton order (Sec. 3.5): particles sorted by their depth-first leaf order;
 *   - the grouped (vectorised) form of the walk (Sec. 1 and Sec. 3.2): particles
 *     are grouped, each group walks the tree once (Fig. "treewalk" applied to
 *     the group) to build one interaction list, and every member sums Eq. (1)
 *     over that list, skipping only its own particle entry.
 *
 * Everything is FP64, compiled without floating-point contraction, evaluated
 * in the order written.  The recursion follows Fig. "treewalk" directly.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_KEY_LEVELS 21                 /* bits per axis in a Morton key */
#define ORC_QMAX ((int64_t)((1 << ORC_KEY_LEVELS) - 1))

/* ------------------------------------------------------------------------- */
/* Direct summation, Eq. (1)                                                  */
/* ------------------------------------------------------------------------- */

/* One particle i against all j != i.  pos is [n][3], row-major. */
static void direct_one(int64_t n, const double *pos, const double *mass, double eps2,
                       int64_t i, double *acc3, double *pot1) {
  double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
  double ax = 0.0, ay = 0.0, az = 0.0, p = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    if (j == i) continue;
    double dx = pos[3 * j] - xi;
    double dy = pos[3 * j + 1] - yi;
    double dz = pos[3 * j + 2] - zi;
    double r2 = dx * dx + dy * dy + dz * dz + eps2;
    double rinv = 1.0 / sqrt(r2);
    double mr3 = mass[j] * rinv * rinv * rinv;
    ax += mr3 * dx;
    ay += mr3 * dy;
    az += mr3 * dz;
    p -= mass[j] * rinv;
  }
  acc3[0] = ax; acc3[1] = ay; acc3[2] = az;
  *pot1 = p;
}

/* Direct sum for the particles listed in idx (all particles if idx == NULL,
 * then ns must equal n).  Results are written row k for idx[k]. */
int oracle_direct(int64_t n, const double *pos, const double *mass, double eps,
                  int64_t ns, const int64_t *idx, double *acc, double *pot) {
  if (n < 0 || ns < 0 || (idx == NULL && ns != n)) return -1;
  double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < ns; ++k) {
    int64_t i = idx ? idx[k] : k;
    direct_one(n, pos, mass, eps2, i, acc + 3 * k, pot + k);
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Oct-tree                                                                   */
/* ------------------------------------------------------------------------- */

enum { ORC_CELL = 0, ORC_PARTICLE = 1, ORC_BUCKET = 2 };

typedef struct {
  int level;            /* 0 = root cube, cell side = side / 2^level */
  int kind;             /* ORC_CELL, ORC_PARTICLE or ORC_BUCKET */
  int64_t first, count; /* particle range in Morton order */
  int64_t cell[3];      /* integer cell coordinates at this level */
  int64_t child[8];     /* node ids of the non-empty sub-cells, octant order */
  int nchild;
  int64_t parent;
  double m, mx[3];      /* total mass and mass-weighted position sums */
  double com[3];        /* centre of mass */
  double l, s;          /* cell side, |geometric centre - centre of mass| */
  double q[6];          /* second moments about com: xx, yy, zz, xy, xz, yz (oracle_tree_quadrupoles) */
} orc_node;

typedef struct {
  int64_t n;
  double lo[3], side, scale;
  uint64_t *key;        /* sorted keys (Morton or Peano-Hilbert) */
  int64_t *q;           /* integer cell coordinates [n][3], sorted order */
  int64_t *perm;        /* perm[k] = input index of the k-th particle in Morton order */
  double *spos, *smass; /* positions and masses in Morton order */
  orc_node *node;
  int64_t nnode, cap;
  int64_t root;
  /* groups */
  int n_crit;
  int64_t ngroup, gcap;
  int64_t *gfirst, *gcount;
  double *glo, *ghi;    /* group bounding boxes [G][3] */
  int have_quad;        /* quadrupoles computed */
} orc_tree;

/* Bit b of the three cell coordinates, interleaved x, y, z (x most significant). */
static uint64_t morton_key(const int64_t q[3]) {
  uint64_t k = 0;
  for (int b = ORC_KEY_LEVELS - 1; b >= 0; --b) {
    k = (k << 3) | ((uint64_t)((q[0] >> b) & 1) << 2) | ((uint64_t)((q[1] >> b) & 1) << 1) |
        (uint64_t)((q[2] >> b) & 1);
  }
  return k;
}

/* Peano-Hilbert index of a cell, by J. Skilling's method ("Programming the
 * Hilbert curve", AIP Conf. Proc. 707, 2004): the coordinates are turned in
 * place into the "transpose" of the index -- walking the bits from the top,
 * each lower bit field is either inverted in x (when the current bit of an
 * axis is set) or exchanged between x and that axis, then the result is
 * Gray-decoded across the axes -- and the transpose's bits, read level by
 * level with x first, are the index.  The curve starts at the origin cell and
 * moves by one cell along one axis at every step; each octant of a cell is a
 * contiguous range of indices, so the index's octal digits name the octree's
 * cells as Morton digits do. */
static uint64_t hilbert_key(const int64_t q[3]) {
  uint32_t x[3] = {(uint32_t)q[0], (uint32_t)q[1], (uint32_t)q[2]};
  for (uint32_t bit = 1u << (ORC_KEY_LEVELS - 1); bit > 1; bit >>= 1) {
    const uint32_t low = bit - 1;
    for (int a = 0; a < 3; ++a) {
      if (x[a] & bit) {
        x[0] ^= low;
      } else {
        const uint32_t swap = (x[0] ^ x[a]) & low;
        x[0] ^= swap;
        x[a] ^= swap;
      }
    }
  }
  x[1] ^= x[0];
  x[2] ^= x[1];
  uint32_t flip = 0;
  for (uint32_t bit = 1u << (ORC_KEY_LEVELS - 1); bit > 1; bit >>= 1)
    if (x[2] & bit) flip ^= bit - 1;
  int64_t t[3];
  for (int a = 0; a < 3; ++a) t[a] = (int64_t)(x[a] ^ flip);
  return morton_key(t);
}

/* Octant (0..7) of a key at a given level (level 1 = first split of the root). */
static int key_digit(uint64_t key, int level) {
  return (int)((key >> (3 * (ORC_KEY_LEVELS - level))) & 7u);
}

static const uint64_t *g_sort_keys; /* used only by the qsort comparator below */

static int cmp_key_index(const void *pa, const void *pb) {
  int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
  uint64_t ka = g_sort_keys[a], kb = g_sort_keys[b];
  if (ka < kb) return -1;
  if (ka > kb) return 1;
  return (a < b) ? -1 : (a > b);
}

static int64_t new_node(orc_tree *t) {
  if (t->nnode == t->cap) {
    int64_t nc = t->cap ? 2 * t->cap : 1024;
    orc_node *p = (orc_node *)realloc(t->node, (size_t)nc * sizeof(orc_node));
    if (!p) return -1;
    t->node = p;
    t->cap = nc;
  }
  int64_t id = t->nnode++;
  memset(&t->node[id], 0, sizeof(orc_node));
  t->node[id].parent = -1;
  for (int k = 0; k < 8; ++k) t->node[id].child[k] = -1;
  return id;
}

/* Geometric quantities of a cell: side l and s = |centre - com|.  A cell with
 * zero mass has no centre of mass; its centre is used instead. */
static void finish_cell(orc_tree *t, orc_node *v) {
  for (int k = 0; k < 3; ++k) v->com[k] = (v->m > 0.0) ? v->mx[k] / v->m : 0.0;
  v->l = ldexp(t->side, -v->level);
  double c[3];
  for (int k = 0; k < 3; ++k) {
    double h = (double)v->cell[k] + 0.5;
    h = h * v->l;
    c[k] = t->lo[k] + h;
  }
  if (!(v->m > 0.0))
    for (int k = 0; k < 3; ++k) v->com[k] = c[k];
  double dx = c[0] - v->com[0], dy = c[1] - v->com[1], dz = c[2] - v->com[2];
  v->s = sqrt(dx * dx + dy * dy + dz * dz);
}

/* Build the sub-tree of the cell (level, cell coordinates) holding the Morton
 * range [first, first + count).  Sec. 3.1: subdivide into eight sub-cells until
 * a cell holds one particle.  Moments are summed from the children in octant
 * order (a particle contributes m and m*x). */
static int64_t build_rec(orc_tree *t, int level, int64_t first, int64_t count, const int64_t cell[3],
                         int64_t parent) {
  int64_t id = new_node(t);
  if (id < 0) return -1;
  orc_node *v = &t->node[id];
  v->level = level;
  v->first = first;
  v->count = count;
  v->parent = parent;
  for (int k = 0; k < 3; ++k) v->cell[k] = cell[k];

  if (count == 1) {
    v->kind = ORC_PARTICLE;
    double m = t->smass[first];
    v->m = m;
    for (int k = 0; k < 3; ++k) {
      v->mx[k] = m * t->spos[3 * first + k];
      v->com[k] = t->spos[3 * first + k];
    }
    v->l = 0.0;
    v->s = 0.0;
    return id;
  }
  if (level == ORC_KEY_LEVELS) {
    /* finest level: all keys equal; a bucket that the walk always opens */
    v->kind = ORC_BUCKET;
    v->m = 0.0;
    v->mx[0] = v->mx[1] = v->mx[2] = 0.0;
    for (int64_t p = first; p < first + count; ++p) {
      double m = t->smass[p];
      v->m = v->m + m;
      for (int k = 0; k < 3; ++k) v->mx[k] = v->mx[k] + m * t->spos[3 * p + k];
    }
    finish_cell(t, v);
    v->l = INFINITY; /* never far enough */
    return id;
  }
  v->kind = ORC_CELL;
  /* split the range by the octant digit of the next level */
  int64_t p = first, end = first + count;
  int nchild = 0;
  int64_t kids[8];
  while (p < end) {
    int d = key_digit(t->key[p], level + 1);
    int64_t q = p;
    while (q < end && key_digit(t->key[q], level + 1) == d) ++q;
    /* the sub-cell from a member's own cell coordinates (for either curve) */
    const int sh = ORC_KEY_LEVELS - (level + 1);
    int64_t sub[3] = {t->q[3 * p] >> sh, t->q[3 * p + 1] >> sh, t->q[3 * p + 2] >> sh};
    int64_t c = build_rec(t, level + 1, p, q - p, sub, id);
    if (c < 0) return -1;
    kids[nchild++] = c;
    p = q;
  }
  v = &t->node[id]; /* the array may have moved */
  v->nchild = nchild;
  v->m = 0.0;
  v->mx[0] = v->mx[1] = v->mx[2] = 0.0;
  for (int k = 0; k < nchild; ++k) {
    orc_node *c = &t->node[kids[k]];
    v->child[k] = kids[k];
    v->m = v->m + c->m;
    for (int a = 0; a < 3; ++a) v->mx[a] = v->mx[a] + c->mx[a];
  }
  finish_cell(t, v);
  return id;
}

void oracle_tree_free(void *h) {
  orc_tree *t = (orc_tree *)h;
  if (!t) return;
  free(t->key); free(t->q); free(t->perm); free(t->spos); free(t->smass); free(t->node);
  free(t->gfirst); free(t->gcount); free(t->glo); free(t->ghi);
  free(t);
}

/* Root cube, keys (curve 0: Morton, 1: Peano-Hilbert), sort and recursive
 * build.  Returns NULL on bad input. */
void *oracle_tree_build2(int64_t n, const double *pos, const double *mass, int curve) {
  if (n < 0) return NULL;
  orc_tree *t = (orc_tree *)calloc(1, sizeof(orc_tree));
  if (!t) return NULL;
  t->n = n;
  t->root = -1;
  if (n == 0) return t;
  for (int64_t i = 0; i < 3 * n; ++i)
    if (!isfinite(pos[i])) { oracle_tree_free(t); return NULL; }
  for (int64_t i = 0; i < n; ++i)
    if (!isfinite(mass[i]) || mass[i] < 0.0) { oracle_tree_free(t); return NULL; }

  /* the cube that encloses all particles: corner at the per-axis minimum,
   * side = largest extent, widened by 2^-20 so the maximum maps inside */
  double hi[3];
  for (int k = 0; k < 3; ++k) t->lo[k] = hi[k] = pos[k];
  for (int64_t i = 1; i < n; ++i)
    for (int k = 0; k < 3; ++k) {
      if (pos[3 * i + k] < t->lo[k]) t->lo[k] = pos[3 * i + k];
      if (pos[3 * i + k] > hi[k]) hi[k] = pos[3 * i + k];
    }
  double ext = 0.0;
  for (int k = 0; k < 3; ++k) {
    double e = hi[k] - t->lo[k];
    if (e > ext) ext = e;
  }
  t->side = (ext > 0.0) ? ext * (1.0 + 0x1p-20) : 1.0;
  t->scale = 0x1p21 / t->side;

  /* integer cell coordinates at the finest level and their Morton keys */
  uint64_t *rawkey = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
  int64_t *rawq = (int64_t *)malloc((size_t)n * 3 * sizeof(int64_t));
  t->key = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
  t->q = (int64_t *)malloc((size_t)n * 3 * sizeof(int64_t));
  t->perm = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  t->spos = (double *)malloc((size_t)n * 3 * sizeof(double));
  t->smass = (double *)malloc((size_t)n * sizeof(double));
  if (!rawkey || !rawq || !t->key || !t->q || !t->perm || !t->spos || !t->smass) {
    free(rawkey);
    free(rawq);
    oracle_tree_free(t);
    return NULL;
  }
  for (int64_t i = 0; i < n; ++i) {
    int64_t q[3];
    for (int k = 0; k < 3; ++k) {
      double u = pos[3 * i + k] - t->lo[k];
      u = u * t->scale;
      int64_t c;
      if (!(u >= 0.0)) c = 0;
      else if (u >= (double)ORC_QMAX) c = ORC_QMAX;
      else c = (int64_t)floor(u);
      q[k] = c;
    }
    rawkey[i] = curve ? hilbert_key(q) : morton_key(q);
    for (int k = 0; k < 3; ++k) rawq[3 * i + k] = q[k];
    t->perm[i] = i;
  }
  /* Morton order, ties kept in input order */
  g_sort_keys = rawkey;
  qsort(t->perm, (size_t)n, sizeof(int64_t), cmp_key_index);
  g_sort_keys = NULL;
  for (int64_t i = 0; i < n; ++i) {
    int64_t j = t->perm[i];
    t->key[i] = rawkey[j];
    for (int k = 0; k < 3; ++k) {
      t->spos[3 * i + k] = pos[3 * j + k];
      t->q[3 * i + k] = rawq[3 * j + k];
    }
    t->smass[i] = mass[j];
  }
  free(rawkey);
  free(rawq);

  int64_t root_cell[3] = {0, 0, 0};
  t->root = build_rec(t, 0, 0, n, root_cell, -1);
  if (t->root < 0) { oracle_tree_free(t); return NULL; }
  return t;
}

void *oracle_tree_build(int64_t n, const double *pos, const double *mass) {
  return oracle_tree_build2(n, pos, mass, 0);
}

/* The Peano-Hilbert index of integer cell coordinates q[0..3) (for pins). */
uint64_t oracle_hilbert_key(int64_t x, int64_t y, int64_t z) {
  const int64_t q[3] = {x, y, z};
  return hilbert_key(q);
}

/* ------------------------------------------------------------------------- */
/* Groups                                                                     */
/* ------------------------------------------------------------------------- */

static int add_group(orc_tree *t, int64_t first, int64_t count) {
  if (t->ngroup == t->gcap) {
    int64_t nc = t->gcap ? 2 * t->gcap : 256;
    int64_t *a = (int64_t *)realloc(t->gfirst, (size_t)nc * sizeof(int64_t));
    if (!a) return -1;
    t->gfirst = a;
    int64_t *b = (int64_t *)realloc(t->gcount, (size_t)nc * sizeof(int64_t));
    if (!b) return -1;
    t->gcount = b;
    t->gcap = nc;
  }
  t->gfirst[t->ngroup] = first;
  t->gcount[t->ngroup] = count;
  t->ngroup++;
  return 0;
}

/* A node with more than n_crit particles is not a group.  Its children are
 * visited in octant order: large children are split further, and runs of
 * consecutive small children (<= n_crit particles each) are packed greedily
 * into groups of at most n_crit particles.  A bucket's children are its
 * particles. */
static int groups_rec(orc_tree *t, int64_t id) {
  orc_node *v = &t->node[id];
  int64_t run_first = -1, run_count = 0;
  int64_t nk = (v->kind == ORC_BUCKET) ? v->count : v->nchild;
  for (int64_t k = 0; k < nk; ++k) {
    int64_t cf, cc, cid = -1;
    if (v->kind == ORC_BUCKET) {
      cf = v->first + k;
      cc = 1;
    } else {
      cid = v->child[k];
      cf = t->node[cid].first;
      cc = t->node[cid].count;
    }
    if (cc > t->n_crit) {
      if (run_count > 0 && add_group(t, run_first, run_count)) return -1;
      run_count = 0;
      if (groups_rec(t, cid)) return -1;
      v = &t->node[id];
      continue;
    }
    if (run_count > 0 && run_count + cc > t->n_crit) {
      if (add_group(t, run_first, run_count)) return -1;
      run_count = 0;
    }
    if (run_count == 0) run_first = cf;
    run_count += cc;
  }
  if (run_count > 0 && add_group(t, run_first, run_count)) return -1;
  return 0;
}

/* Build the groups for a critical size n_crit; returns G or -1. */
int64_t oracle_tree_groups(void *h, int n_crit) {
  orc_tree *t = (orc_tree *)h;
  if (!t || n_crit < 1) return -1;
  t->n_crit = n_crit;
  t->ngroup = 0;
  if (t->n == 0) return 0;
  if (t->node[t->root].count <= n_crit) {
    if (add_group(t, 0, t->n)) return -1;
  } else if (groups_rec(t, t->root)) {
    return -1;
  }
  free(t->glo); free(t->ghi);
  t->glo = (double *)malloc((size_t)t->ngroup * 3 * sizeof(double));
  t->ghi = (double *)malloc((size_t)t->ngroup * 3 * sizeof(double));
  if (!t->glo || !t->ghi) return -1;
  for (int64_t g = 0; g < t->ngroup; ++g) {
    int64_t a = t->gfirst[g], c = t->gcount[g];
    for (int k = 0; k < 3; ++k) t->glo[3 * g + k] = t->ghi[3 * g + k] = t->spos[3 * a + k];
    for (int64_t p = a + 1; p < a + c; ++p)
      for (int k = 0; k < 3; ++k) {
        double x = t->spos[3 * p + k];
        if (x < t->glo[3 * g + k]) t->glo[3 * g + k] = x;
        if (x > t->ghi[3 * g + k]) t->ghi[3 * g + k] = x;
      }
  }
  return t->ngroup;
}

/* ------------------------------------------------------------------------- */
/* Group walk (Fig. "treewalk" for a group) and force sum                     */
/* ------------------------------------------------------------------------- */

typedef struct {
  double x, y, z, m;
  int64_t particle; /* Morton index of a particle entry, -1 for a cell */
  int64_t node;     /* node the entry comes from (the bucket for its particles) */
} orc_entry;

typedef struct {
  orc_entry *e;
  int64_t n, cap;
} orc_list;

static int list_push(orc_list *L, double x, double y, double z, double m, int64_t particle, int64_t node) {
  if (L->n == L->cap) {
    int64_t nc = L->cap ? 2 * L->cap : 1024;
    orc_entry *p = (orc_entry *)realloc(L->e, (size_t)nc * sizeof(orc_entry));
    if (!p) return -1;
    L->e = p;
    L->cap = nc;
  }
  orc_entry *q = &L->e[L->n++];
  q->x = x; q->y = y; q->z = z; q->m = m; q->particle = particle; q->node = node;
  return 0;
}

/* Eq. (2)/(3) for a group: d is the distance from the cell's centre of mass to
 * the group's bounding box; the cell is far enough iff d^2 > (l/theta + s)^2. */
static int far_enough(const orc_node *v, const double *glo, const double *ghi, double theta) {
  double e[3];
  for (int k = 0; k < 3; ++k) {
    double below = glo[k] - v->com[k];
    double above = v->com[k] - ghi[k];
    double d = fmax(below, above);
    e[k] = fmax(0.0, d);
  }
  double d2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
  double r = v->l / theta;
  r = r + v->s;
  double seff = r * r;
  return d2 > seff;
}

static int walk_rec(const orc_tree *t, int64_t id, const double *glo, const double *ghi, double theta,
                    orc_list *L) {
  const orc_node *v = &t->node[id];
  if (v->kind == ORC_PARTICLE)
    return list_push(L, v->com[0], v->com[1], v->com[2], v->m, v->first, id);
  if (v->kind == ORC_BUCKET) {
    for (int64_t p = v->first; p < v->first + v->count; ++p)
      if (list_push(L, t->spos[3 * p], t->spos[3 * p + 1], t->spos[3 * p + 2], t->smass[p], p, id)) return -1;
    return 0;
  }
  if (far_enough(v, glo, ghi, theta))
    return list_push(L, v->com[0], v->com[1], v->com[2], v->m, -1, id);
  for (int k = 0; k < v->nchild; ++k)
    if (walk_rec(t, v->child[k], glo, ghi, theta, L)) return -1;
  return 0;
}

/* Second mass moments of every node about its centre of mass, from the
 * plain definition over the node's own particles: S_ab = sum m d_a d_b,
 * d = x - com (the traceless quadrupole is 3 S - tr(S) I).  A particle's are
 * zero.  The paper keeps only monopoles; the expansion one order further is
 * an extension of it. */
void oracle_tree_quadrupoles(void *h) {
  orc_tree *t = (orc_tree *)h;
  if (!t || t->have_quad) return;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t id = 0; id < t->nnode; ++id) {
    orc_node *v = &t->node[id];
    for (int k = 0; k < 6; ++k) v->q[k] = 0.0;
    if (v->kind == ORC_PARTICLE) continue;
    for (int64_t p = v->first; p < v->first + v->count; ++p) {
      const double m = t->smass[p];
      const double dx = t->spos[3 * p] - v->com[0], dy = t->spos[3 * p + 1] - v->com[1],
                   dz = t->spos[3 * p + 2] - v->com[2];
      v->q[0] += m * dx * dx;
      v->q[1] += m * dy * dy;
      v->q[2] += m * dz * dz;
      v->q[3] += m * dx * dy;
      v->q[4] += m * dx * dz;
      v->q[5] += m * dy * dz;
    }
  }
  t->have_quad = 1;
}

/* Second moments of node id (6 values as above); zeros before they are
 * computed. */
void oracle_tree_node_quadrupole(void *h, int64_t id, double *q6) {
  orc_tree *t = (orc_tree *)h;
  for (int k = 0; k < 6; ++k) q6[k] = (t && t->have_quad && id >= 0 && id < t->nnode) ? t->node[id].q[k] : 0.0;
}

/* Interaction list of group g; entries are written as (x, y, z, m) rows, the
 * Morton index of particle entries (-1 for cells) and the source node id.
 * Returns the list length (possibly larger than cap, in which case only cap
 * rows are written). */
int64_t oracle_tree_group_list(void *h, int64_t g, double theta, int64_t cap, double *xyzm, int64_t *particle,
                               int64_t *node) {
  orc_tree *t = (orc_tree *)h;
  if (!t || g < 0 || g >= t->ngroup) return -1;
  orc_list L = {0};
  if (walk_rec(t, t->root, t->glo + 3 * g, t->ghi + 3 * g, theta, &L)) { free(L.e); return -1; }
  for (int64_t k = 0; k < L.n && k < cap; ++k) {
    xyzm[4 * k] = L.e[k].x; xyzm[4 * k + 1] = L.e[k].y;
    xyzm[4 * k + 2] = L.e[k].z; xyzm[4 * k + 3] = L.e[k].m;
    if (particle) particle[k] = L.e[k].particle;
    if (node) node[k] = L.e[k].node;
  }
  int64_t n = L.n;
  free(L.e);
  return n;
}

/* Forces for the selected groups (all if gsel == NULL).  theta_g (per group,
 * nullable) overrides theta.  acc [n][3] and pot [n] are indexed in input
 * order; only members of selected groups are written; with acc == NULL only
 * the lists are built.  acc_abs [n] (nullable) receives the sum of the force
 * magnitudes of the individual terms, sum_e m_e r/(r^2+eps^2)^(3/2), the scale
 * against which cancellation in acc is measured.  Per selected group k:
 * list_len[k] = list length, list_mass[k] = sum of entry masses (nullable).
 * interactions (nullable) receives sum over members of (list length - 1). */
int oracle_tree_forces2(void *h, double eps, double theta, const double *theta_g, int64_t nsel,
                        const int64_t *gsel, int quadrupole, double *acc, double *pot, double *acc_abs,
                        int64_t *list_len, double *list_mass, int64_t *interactions);

int oracle_tree_forces(void *h, double eps, double theta, const double *theta_g, int64_t nsel,
                       const int64_t *gsel, double *acc, double *pot, double *acc_abs, int64_t *list_len,
                       double *list_mass, int64_t *interactions) {
  return oracle_tree_forces2(h, eps, theta, theta_g, nsel, gsel, 0, acc, pot, acc_abs, list_len, list_mass,
                             interactions);
}

/* As oracle_tree_forces; with quadrupole != 0 a cell entry adds the
 * second-order term of the Taylor expansion of the softened potential of its
 * particles about their centre of mass.  With u = com - x_i, R^2 = |u|^2 +
 * eps^2 and S the cell's second moments, T = tr S:
 *   pot = -M/R - 3 (u.S.u) / (2 R^5) + T / (2 R^3)
 * and the acceleration is its gradient in u,
 *   acc = M u/R^3 - 3 S u/R^5 + (15 (u.S.u) / (2 R^7) - 3 T / (2 R^5)) u.
 * (For eps = 0 this is the traceless quadrupole form.)  acc_abs still sums
 * the magnitudes of the monopole parts. */
int oracle_tree_forces2(void *h, double eps, double theta, const double *theta_g, int64_t nsel,
                        const int64_t *gsel, int quadrupole, double *acc, double *pot, double *acc_abs,
                        int64_t *list_len, double *list_mass, int64_t *interactions) {
  orc_tree *t = (orc_tree *)h;
  if (!t) return -1;
  if (quadrupole) oracle_tree_quadrupoles(t);
  if (gsel == NULL) nsel = t->ngroup;
  double eps2 = eps * eps;
  int64_t total = 0;
  int failed = 0;
#pragma omp parallel reduction(+ : total) reduction(| : failed)
  {
    orc_list L = {0};
#pragma omp for schedule(dynamic, 1)
    for (int64_t k = 0; k < nsel; ++k) {
      int64_t g = gsel ? gsel[k] : k;
      if (g < 0 || g >= t->ngroup) { failed |= 1; continue; }
      double th = theta_g ? theta_g[g] : theta;
      L.n = 0;
      if (walk_rec(t, t->root, t->glo + 3 * g, t->ghi + 3 * g, th, &L)) { failed |= 1; continue; }
      if (list_len) list_len[k] = L.n;
      if (list_mass) {
        double ms = 0.0;
        for (int64_t e = 0; e < L.n; ++e) ms += L.e[e].m;
        list_mass[k] = ms;
      }
      int64_t a = t->gfirst[g];
      total += t->gcount[g] * (L.n - 1);
      if (!acc) continue;
      for (int64_t i = a; i < a + t->gcount[g]; ++i) {
        double xi = t->spos[3 * i], yi = t->spos[3 * i + 1], zi = t->spos[3 * i + 2];
        double ax = 0.0, ay = 0.0, az = 0.0, p = 0.0, aa = 0.0;
        for (int64_t e = 0; e < L.n; ++e) {
          const orc_entry *q = &L.e[e];
          if (q->particle == i) continue; /* j != i in Eq. (1) */
          double dx = q->x - xi, dy = q->y - yi, dz = q->z - zi;
          double r2 = dx * dx + dy * dy + dz * dz + eps2;
          double rinv = 1.0 / sqrt(r2);
          double mr3 = q->m * rinv * rinv * rinv;
          ax += mr3 * dx;
          ay += mr3 * dy;
          az += mr3 * dz;
          p -= q->m * rinv;
          if (acc_abs) aa += mr3 * sqrt(dx * dx + dy * dy + dz * dz);
          if (quadrupole && q->particle < 0) {
            const double *S = t->node[q->node].q;
            const double sx = S[0] * dx + S[3] * dy + S[4] * dz;
            const double sy = S[3] * dx + S[1] * dy + S[5] * dz;
            const double sz = S[4] * dx + S[5] * dy + S[2] * dz;
            const double usu = dx * sx + dy * sy + dz * sz;
            const double tr = S[0] + S[1] + S[2];
            const double r3 = rinv * rinv * rinv;
            const double r5 = r3 * rinv * rinv;
            const double r7 = r5 * rinv * rinv;
            const double c = 7.5 * usu * r7 - 1.5 * tr * r5;
            ax += -3.0 * sx * r5 + c * dx;
            ay += -3.0 * sy * r5 + c * dy;
            az += -3.0 * sz * r5 + c * dz;
            p += -1.5 * usu * r5 + 0.5 * tr * r3;
          }
        }
        int64_t o = t->perm[i];
        acc[3 * o] = ax; acc[3 * o + 1] = ay; acc[3 * o + 2] = az;
        pot[o] = p;
        if (acc_abs) acc_abs[o] = aa;
      }
    }
    free(L.e);
  }
  if (interactions) *interactions = total;
  return failed ? -1 : 0;
}

/* ------------------------------------------------------------------------- */
/* Accessors for tests                                                        */
/* ------------------------------------------------------------------------- */

/* lo[3], side, number of nodes (all kinds, chain cells included), root id */
void oracle_tree_info(void *h, double *lo, double *side, int64_t *nnode, int64_t *root) {
  orc_tree *t = (orc_tree *)h;
  for (int k = 0; k < 3; ++k) lo[k] = t->lo[k];
  *side = t->side;
  *nnode = t->nnode;
  *root = t->root;
}

void oracle_tree_sorted(void *h, uint64_t *keys, int64_t *perm) {
  orc_tree *t = (orc_tree *)h;
  if (keys) memcpy(keys, t->key, (size_t)t->n * sizeof(uint64_t));
  if (perm) memcpy(perm, t->perm, (size_t)t->n * sizeof(int64_t));
}

/* Node table in creation (depth-first) order.  ints: [nnode][6] = level, kind,
 * first, count, nchild, parent.  reals: [nnode][6] = m, com x/y/z, l, s.
 * children: [nnode][8] child ids (-1 when absent). */
void oracle_tree_nodes(void *h, int64_t *ints, double *reals, int64_t *children) {
  orc_tree *t = (orc_tree *)h;
  for (int64_t i = 0; i < t->nnode; ++i) {
    const orc_node *v = &t->node[i];
    int64_t *a = ints + 6 * i;
    a[0] = v->level; a[1] = v->kind; a[2] = v->first; a[3] = v->count; a[4] = v->nchild; a[5] = v->parent;
    double *r = reals + 6 * i;
    r[0] = v->m; r[1] = v->com[0]; r[2] = v->com[1]; r[3] = v->com[2]; r[4] = v->l; r[5] = v->s;
    if (children)
      for (int k = 0; k < 8; ++k) children[8 * i + k] = v->child[k];
  }
}

/* Groups: first, count (Morton ranges), bounding boxes lo/hi [G][3]. */
void oracle_tree_group_info(void *h, int64_t *first, int64_t *count, double *lo, double *hi) {
  orc_tree *t = (orc_tree *)h;
  for (int64_t g = 0; g < t->ngroup; ++g) {
    if (first) first[g] = t->gfirst[g];
    if (count) count[g] = t->gcount[g];
    for (int k = 0; k < 3; ++k) {
      if (lo) lo[3 * g + k] = t->glo[3 * g + k];
      if (hi) hi[3 * g + k] = t->ghi[3 * g + k];
    }
  }
}

/* ---- neighbour search (the general treewalk of Sec. 3.3 applied to short-
 * range interactions, as in SPH) ------------------------------------------
 *
 * The plain definition, by brute force over all pairs: the neighbours of
 * particle i are the particles j != i with |x_j - x_i| < h_i (its own search
 * radius, the "gather" form), the distance squared evaluated as
 * (dx*dx + dy*dy) + dz*dz with dx = x_j - x_i.  The SPH density
 *   rho_i = m_i W(0, h_i) + sum over neighbours m_j W(|x_j - x_i|, h_i)
 * uses the cubic spline kernel of Monaghan and Lattanzio (1985) with compact
 * support h: q = r/h, W = 8/(pi h^3) (1 - 6 q^2 + 6 q^3) for q < 1/2,
 * 16/(pi h^3) (1 - q)^3 for q < 1, 0 beyond (a choice: the paper names SPH
 * as the application without fixing a kernel). */
double oracle_sph_kernel(double r, double h) {
  const double q = r / h;
  const double sigma = 8.0 / (M_PI * h * h * h);
  if (q < 0.5) return sigma * (1.0 - 6.0 * q * q + 6.0 * q * q * q);
  if (q < 1.0) {
    const double u = 1.0 - q;
    return sigma * 2.0 * u * u * u;
  }
  return 0.0;
}

/* count[i] (nullable), rho[i] (nullable) and, when offsets is given, the
 * neighbours of i (input indices, increasing) at nbr[offsets[i] ...]. */
int oracle_neighbors(int64_t n, const double *pos, const double *mass, const double *h, int64_t *count,
                     double *rho, const int64_t *offsets, int64_t *nbr) {
  if (n < 0 || (n > 0 && (!pos || !h))) return -1;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
    const double hi = h[i];
    const double h2 = hi * hi;
    int64_t c = 0;
    double r = mass ? mass[i] * oracle_sph_kernel(0.0, hi) : 0.0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      const double dx = pos[3 * j] - xi, dy = pos[3 * j + 1] - yi, dz = pos[3 * j + 2] - zi;
      const double r2 = (dx * dx + dy * dy) + dz * dz;
      if (!(r2 < h2)) continue;
      if (offsets && nbr) nbr[offsets[i] + c] = j;
      ++c;
      if (mass) r += mass[j] * oracle_sph_kernel(sqrt(r2), hi);
    }
    if (count) count[i] = c;
    if (rho) rho[i] = r;
  }
  return 0;
}

/* The same for the selected particles sel[0 .. nsel) only (count, rho in
 * selection order), by brute force over all n. */
int oracle_neighbors_sel(int64_t n, const double *pos, const double *mass, const double *h, int64_t nsel,
                         const int64_t *sel, int64_t *count, double *rho) {
  if (n < 0 || nsel < 0 || (nsel > 0 && (!pos || !h || !sel))) return -1;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(| : bad)
  for (int64_t k = 0; k < nsel; ++k) {
    const int64_t i = sel[k];
    if (i < 0 || i >= n) { bad |= 1; continue; }
    const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
    const double hi = h[i];
    const double h2 = hi * hi;
    int64_t c = 0;
    double r = mass ? mass[i] * oracle_sph_kernel(0.0, hi) : 0.0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      const double dx = pos[3 * j] - xi, dy = pos[3 * j + 1] - yi, dz = pos[3 * j + 2] - zi;
      const double r2 = (dx * dx + dy * dy) + dz * dz;
      if (!(r2 < h2)) continue;
      ++c;
      if (mass) r += mass[j] * oracle_sph_kernel(sqrt(r2), hi);
    }
    if (count) count[k] = c;
    if (rho) rho[k] = r;
  }
  return bad ? -1 : 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
