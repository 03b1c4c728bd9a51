/*
 * orc.c -- FP64 CPU oracle of the Barnes-Hut step of "Accelerated FDPS"
 * (Iwasawa et al. 2019): root cell, Morton keys, stable key sort, reorder,
 * octree link, multipole moments, particle groups, group-wise tree walk that
 * emits index interaction lists, list forces, direct forces, kick-drift.
 *
 * TEST INFRASTRUCTURE ONLY: only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the GPU library, and the GPU library never calls it.
 *
 * Plain and slow on purpose: every stage follows the paper's description in
 * its own order, in FP64, with no blocking or fusion.  Where the paper is
 * silent the reading used is stated at the function.  Built with
 * -ffp-contract=off so that every product and sum is rounded on its own.
 *
 * Readings of points the paper leaves open (all stated again in the design
 * notes of the repository):
 *   R1 root cell: cube anchored at the per-axis minimum, side L = 2^k, the
 *      smallest power of two strictly larger than the largest extent.
 *   R2 keys: 21 bits per axis, 63-bit key, x is the most significant bit of
 *      every 3-bit digit.
 *   R3 sort: stable, equal keys keep their input order.
 *   R4 link: a cell is split iff it holds more than n_leaf particles and its
 *      level is below 21; only non-empty octants become children; cells are
 *      numbered in DFS pre-order, children in octant order.
 *   R5 groups: a group is a cell that holds at most n_grp particles (or is a
 *      leaf) and whose parent holds more than n_grp particles (or is the
 *      root itself).
 *   R6 opening test: distance from the group's tight box to the geometric
 *      centre of the cell, accepted iff d^2 > (s/theta)^2 with s the side of
 *      the cell; a cell whose particle range contains the group's is opened.
 *   R7 softening: Plummer, also inside superparticle terms; the particle
 *      itself is skipped (its pull is exactly zero, its potential is
 *      excluded).
 *   R8 quadrupole: second-order Taylor expansion of the softened kernel about
 *      the centre of mass, with S_ab = sum m (x-X)_a (x-X)_b (not traceless).
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define KEY_BITS 21
#define MAX_LEVEL 21

struct orc_tree {
  int64_t n;
  int n_leaf, n_grp;
  double lo[3];
  int k;
  /* particles in sorted (Morton) order */
  uint64_t* key;
  uint32_t* perm; /* sorted position -> input index */
  double *x, *y, *z, *m;
  /* cells, DFS pre-order */
  int64_t n_cell, cap_cell;
  uint64_t* prefix;
  uint8_t* level;
  uint8_t* leaf;
  uint32_t *begin, *count, *parent, *skip;
  double* ctr; /* 3 per cell */
  double* mass;
  double* com;  /* 3 per cell */
  double* com0; /* 3 per cell: centres of mass at construction */
  double *bmin, *bmax; /* 3 per cell: box of the cell's particles now */
  int moved; /* 0 from construction until the first reuse step */
  double* quad; /* 6 per cell: xx yy zz xy xz yz */
  /* groups; g_lo/g_hi is the box the group's current list was walked
   * with (the construction-time box until a list refresh) */
  int64_t n_groups;
  uint32_t *g_cell, *g_begin, *g_count;
  double *g_lo, *g_hi, *g_ctr; /* 3 per group */
  double* g_tau0;              /* 3 per group: cell shift at that walk */
  double *g_sa, *g_so;         /* opening-test slacks of that walk */
  /* neighbour lists (short-range walk), every group */
  int have_nbr;
  int64_t* nb_off;
  uint32_t* nb;
  /* lists over the last walked selection */
  int have_lists;
  int64_t n_sel;
  int64_t* sel;
  int64_t *epj_off, *spj_off;
  uint32_t *epj, *spj;
};

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ---------------------------------------------------------------------- */
/* Root cell (section 4.3: the root cell is fixed from the positions of all
 * particles before the local tree is made).  Reading R1. */
int orc_root(int64_t n, const double* x, const double* y, const double* z,
             double lo[3], int* k) {
  if (n <= 0 || !x || !y || !z || !lo || !k) return -1;
  const double* p[3] = {x, y, z};
  double ext = 0.0;
  for (int a = 0; a < 3; ++a) {
    double mn = p[a][0], mx = p[a][0];
    for (int64_t i = 1; i < n; ++i) {
      if (p[a][i] < mn) mn = p[a][i];
      if (p[a][i] > mx) mx = p[a][i];
    }
    lo[a] = mn;
    double e = mx - mn;
    if (e > ext) ext = e;
  }
  if (!(ext >= 0.0) || isinf(ext)) return -1; /* NaN or inf input */
  if (ext == 0.0) {
    *k = 0;
    return 0;
  }
  /* smallest k with 2^k > ext */
  int kk;
  frexp(ext, &kk);
  while (ldexp(1.0, kk) <= ext) kk++;
  while (ldexp(1.0, kk - 1) > ext) kk--;
  *k = kk;
  return 0;
}

uint64_t orc_interleave(uint32_t qx, uint32_t qy, uint32_t qz) {
  uint64_t key = 0;
  for (int b = 0; b < KEY_BITS; ++b) {
    key |= (uint64_t)((qx >> b) & 1u) << (3 * b + 2);
    key |= (uint64_t)((qy >> b) & 1u) << (3 * b + 1);
    key |= (uint64_t)((qz >> b) & 1u) << (3 * b);
  }
  return key;
}

/* Integer cell coordinates (level bits per axis) of the level-`level` cell
 * that holds `key`. */
void orc_deinterleave(uint64_t key, int level, uint32_t q[3]) {
  uint64_t p = key >> (3 * (MAX_LEVEL - level));
  q[0] = q[1] = q[2] = 0;
  for (int b = 0; b < level; ++b) {
    q[0] |= (uint32_t)((p >> (3 * b + 2)) & 1u) << b;
    q[1] |= (uint32_t)((p >> (3 * b + 1)) & 1u) << b;
    q[2] |= (uint32_t)((p >> (3 * b)) & 1u) << b;
  }
}

/* Morton keys (section 4.3, local tree step 1).  Reading R2: quantise the
 * offset from the root corner to 21 bits per axis. */
int orc_keys(int64_t n, const double* x, const double* y, const double* z,
             const double lo[3], int k, uint64_t* key) {
  if (n < 0 || (n > 0 && (!x || !y || !z || !key))) return -1;
  const double scale = ldexp(1.0, KEY_BITS - k);
  const double qmax = (double)((1u << KEY_BITS) - 1u);
  const double* p[3] = {x, y, z};
  for (int64_t i = 0; i < n; ++i) {
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
      double d = p[a][i] - lo[a];
      double f = floor(d * scale);
      if (f < 0.0) f = 0.0;
      if (f > qmax) f = qmax;
      q[a] = (uint32_t)f;
    }
    key[i] = orc_interleave(q[0], q[1], q[2]);
  }
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Stable sort of key-index pairs (section 4.3, local tree step 2; reading
 * R3).  qsort on (key, input index) pairs is the stable order because the
 * second field breaks every tie. */
typedef struct {
  uint64_t key;
  uint32_t idx;
} kv_t;

static int kv_cmp(const void* a, const void* b) {
  const kv_t* u = (const kv_t*)a;
  const kv_t* v = (const kv_t*)b;
  if (u->key != v->key) return u->key < v->key ? -1 : 1;
  if (u->idx != v->idx) return u->idx < v->idx ? -1 : 1;
  return 0;
}

/* ---------------------------------------------------------------------- */
static int grow_cells(orc_tree* t) {
  int64_t cap = t->cap_cell ? 2 * t->cap_cell : 1024;
#define GROW(ptr, type, per)                                         \
  do {                                                               \
    void* np = realloc(t->ptr, (size_t)cap * (per) * sizeof(type));  \
    if (!np) return -1;                                              \
    t->ptr = (type*)np;                                              \
  } while (0)
  GROW(prefix, uint64_t, 1);
  GROW(level, uint8_t, 1);
  GROW(leaf, uint8_t, 1);
  GROW(begin, uint32_t, 1);
  GROW(count, uint32_t, 1);
  GROW(parent, uint32_t, 1);
  GROW(skip, uint32_t, 1);
  GROW(ctr, double, 3);
#undef GROW
  t->cap_cell = cap;
  return 0;
}

/* Geometric centre of a cell: root corner + (2q+1) * L * 2^-(level+1). */
static void cell_centre(const orc_tree* t, uint64_t first_key, int level,
                        double out[3]) {
  uint32_t q[3];
  orc_deinterleave(first_key, level, q);
  const double half = ldexp(1.0, t->k - level - 1);
  for (int a = 0; a < 3; ++a)
    out[a] = t->lo[a] + (2.0 * (double)q[a] + 1.0) * half;
}

/* Link (section 4.3, local tree step 4; reading R4): top-down, a cell over
 * the sorted range [b, e) at `level`; children are the runs of equal
 * next-level digit.  Recursion order gives DFS pre-order ids. */
static int link_cell(orc_tree* t, int level, int64_t b, int64_t e,
                     uint32_t parent_id) {
  if (t->n_cell == t->cap_cell && grow_cells(t)) return -1;
  const int64_t id = t->n_cell++;
  t->prefix[id] = t->key[b] >> (3 * (MAX_LEVEL - level));
  t->level[id] = (uint8_t)level;
  t->begin[id] = (uint32_t)b;
  t->count[id] = (uint32_t)(e - b);
  t->parent[id] = parent_id;
  cell_centre(t, t->key[b], level, &t->ctr[3 * id]);
  const int split = (e - b) > t->n_leaf && level < MAX_LEVEL;
  t->leaf[id] = (uint8_t)!split;
  if (split) {
    const int sh = 3 * (MAX_LEVEL - (level + 1));
    int64_t cb = b;
    for (uint64_t oct = 0; oct < 8; ++oct) {
      const uint64_t want = (t->prefix[id] << 3) | oct;
      int64_t ce = cb;
      while (ce < e && (t->key[ce] >> sh) == want) ce++;
      if (ce > cb) {
        if (link_cell(t, level + 1, cb, ce, (uint32_t)id)) return -1;
        cb = ce;
      }
    }
    if (cb != e) return -1; /* keys not sorted: cannot happen */
  }
  t->skip[id] = (uint32_t)t->n_cell;
  return 0;
}

/* Multipole moments of every cell over its particle range (section 4.3:
 * moments are recomputed at every step, reuse steps included). */
static void compute_moments(orc_tree* t) {
  for (int64_t c = 0; c < t->n_cell; ++c) {
    const int64_t b = t->begin[c], e = b + t->count[c];
    double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    for (int64_t i = b; i < e; ++i) {
      M += t->m[i];
      sx += t->m[i] * t->x[i];
      sy += t->m[i] * t->y[i];
      sz += t->m[i] * t->z[i];
    }
    double X[3];
    if (M > 0.0) {
      X[0] = sx / M;
      X[1] = sy / M;
      X[2] = sz / M;
    } else {
      X[0] = t->ctr[3 * c];
      X[1] = t->ctr[3 * c + 1];
      X[2] = t->ctr[3 * c + 2];
    }
    double S[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = b; i < e; ++i) {
      const double dx = t->x[i] - X[0], dy = t->y[i] - X[1],
                   dz = t->z[i] - X[2];
      S[0] += t->m[i] * dx * dx;
      S[1] += t->m[i] * dy * dy;
      S[2] += t->m[i] * dz * dz;
      S[3] += t->m[i] * dx * dy;
      S[4] += t->m[i] * dx * dz;
      S[5] += t->m[i] * dy * dz;
    }
    t->mass[c] = M;
    memcpy(&t->com[3 * c], X, sizeof X);
    memcpy(&t->quad[6 * c], S, sizeof S);
    const double* p[3] = {t->x, t->y, t->z};
    for (int a = 0; a < 3; ++a) {
      double mn = p[a][b], mx = p[a][b];
      for (int64_t i = b + 1; i < e; ++i) {
        if (p[a][i] < mn) mn = p[a][i];
        if (p[a][i] > mx) mx = p[a][i];
      }
      t->bmin[3 * c + a] = mn;
      t->bmax[3 * c + a] = mx;
    }
  }
}

/* Particle groups (Barnes' vectorisation, section 2; reading R5). */
static int make_groups(orc_tree* t) {
  int64_t ng = 0;
  for (int64_t c = 0; c < t->n_cell; ++c) {
    const int small = t->count[c] <= (uint32_t)t->n_grp || t->leaf[c];
    const int top = c == 0 || t->count[t->parent[c]] > (uint32_t)t->n_grp;
    if (small && top) ng++;
  }
  t->n_groups = ng;
  t->g_cell = (uint32_t*)malloc((size_t)(ng ? ng : 1) * sizeof(uint32_t));
  t->g_begin = (uint32_t*)malloc((size_t)(ng ? ng : 1) * sizeof(uint32_t));
  t->g_count = (uint32_t*)malloc((size_t)(ng ? ng : 1) * sizeof(uint32_t));
  t->g_lo = (double*)malloc((size_t)(ng ? ng : 1) * 3 * sizeof(double));
  t->g_hi = (double*)malloc((size_t)(ng ? ng : 1) * 3 * sizeof(double));
  t->g_ctr = (double*)malloc((size_t)(ng ? ng : 1) * 3 * sizeof(double));
  t->g_tau0 = (double*)calloc((size_t)(ng ? ng : 1) * 3, sizeof(double));
  t->g_sa = (double*)malloc((size_t)(ng ? ng : 1) * sizeof(double));
  t->g_so = (double*)malloc((size_t)(ng ? ng : 1) * sizeof(double));
  if (!t->g_cell || !t->g_begin || !t->g_count || !t->g_lo || !t->g_hi ||
      !t->g_ctr || !t->g_tau0 || !t->g_sa || !t->g_so)
    return -1;
  int64_t g = 0;
  for (int64_t c = 0; c < t->n_cell; ++c) {
    const int small = t->count[c] <= (uint32_t)t->n_grp || t->leaf[c];
    const int top = c == 0 || t->count[t->parent[c]] > (uint32_t)t->n_grp;
    if (!(small && top)) continue;
    t->g_cell[g] = (uint32_t)c;
    t->g_sa[g] = t->g_so[g] = INFINITY;
    t->g_begin[g] = t->begin[c];
    t->g_count[g] = t->count[c];
    const int64_t b = t->begin[c], e = b + t->count[c];
    const double* p[3] = {t->x, t->y, t->z};
    for (int a = 0; a < 3; ++a) {
      double mn = p[a][b], mx = p[a][b];
      for (int64_t i = b + 1; i < e; ++i) {
        if (p[a][i] < mn) mn = p[a][i];
        if (p[a][i] > mx) mx = p[a][i];
      }
      t->g_lo[3 * g + a] = mn;
      t->g_hi[3 * g + a] = mx;
      t->g_ctr[3 * g + a] = t->ctr[3 * c + a];
    }
    g++;
  }
  return 0;
}

static void free_lists(orc_tree* t) {
  free(t->sel);
  free(t->epj_off);
  free(t->spj_off);
  free(t->epj);
  free(t->spj);
  t->sel = NULL;
  t->epj_off = t->spj_off = NULL;
  t->epj = t->spj = NULL;
  t->have_lists = 0;
  t->n_sel = 0;
}

void orc_free(orc_tree* t) {
  if (!t) return;
  free(t->key);
  free(t->perm);
  free(t->x);
  free(t->y);
  free(t->z);
  free(t->m);
  free(t->prefix);
  free(t->level);
  free(t->leaf);
  free(t->begin);
  free(t->count);
  free(t->parent);
  free(t->skip);
  free(t->ctr);
  free(t->mass);
  free(t->com);
  free(t->com0);
  free(t->bmin);
  free(t->bmax);
  free(t->quad);
  free(t->g_cell);
  free(t->g_begin);
  free(t->g_count);
  free(t->g_lo);
  free(t->g_hi);
  free(t->g_ctr);
  free(t->g_tau0);
  free(t->g_sa);
  free(t->g_so);
  free_lists(t);
  free(t->nb_off);
  free(t->nb);
  free(t);
}

/* Construction step up to the groups: root, keys, sort, reorder, link,
 * moments, groups (section 4.3). */
orc_tree* orc_build(int64_t n, const double* x, const double* y,
                    const double* z, const double* m, int n_leaf, int n_grp) {
  if (n <= 0 || n > 0xFFFFFFF0LL || !x || !y || !z || !m || n_leaf < 1 ||
      n_grp < 1)
    return NULL;
  orc_tree* t = (orc_tree*)calloc(1, sizeof(orc_tree));
  if (!t) return NULL;
  t->n = n;
  t->n_leaf = n_leaf;
  t->n_grp = n_grp;
  if (orc_root(n, x, y, z, t->lo, &t->k)) goto fail;

  uint64_t* raw = (uint64_t*)malloc((size_t)n * sizeof(uint64_t));
  kv_t* kv = (kv_t*)malloc((size_t)n * sizeof(kv_t));
  if (!raw || !kv) {
    free(raw);
    free(kv);
    goto fail;
  }
  orc_keys(n, x, y, z, t->lo, t->k, raw);
  for (int64_t i = 0; i < n; ++i) {
    kv[i].key = raw[i];
    kv[i].idx = (uint32_t)i;
  }
  free(raw);
  qsort(kv, (size_t)n, sizeof(kv_t), kv_cmp);

  t->key = (uint64_t*)malloc((size_t)n * sizeof(uint64_t));
  t->perm = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
  t->x = (double*)malloc((size_t)n * sizeof(double));
  t->y = (double*)malloc((size_t)n * sizeof(double));
  t->z = (double*)malloc((size_t)n * sizeof(double));
  t->m = (double*)malloc((size_t)n * sizeof(double));
  if (!t->key || !t->perm || !t->x || !t->y || !t->z || !t->m) {
    free(kv);
    goto fail;
  }
  /* reorder (section 4.3, local tree step 3) */
  for (int64_t i = 0; i < n; ++i) {
    t->key[i] = kv[i].key;
    t->perm[i] = kv[i].idx;
    t->x[i] = x[kv[i].idx];
    t->y[i] = y[kv[i].idx];
    t->z[i] = z[kv[i].idx];
    t->m[i] = m[kv[i].idx];
  }
  free(kv);

  if (link_cell(t, 0, 0, n, 0xFFFFFFFFu)) goto fail;
  t->mass = (double*)malloc((size_t)t->n_cell * sizeof(double));
  t->com = (double*)malloc((size_t)t->n_cell * 3 * sizeof(double));
  t->com0 = (double*)malloc((size_t)t->n_cell * 3 * sizeof(double));
  t->bmin = (double*)malloc((size_t)t->n_cell * 3 * sizeof(double));
  t->bmax = (double*)malloc((size_t)t->n_cell * 3 * sizeof(double));
  t->quad = (double*)malloc((size_t)t->n_cell * 6 * sizeof(double));
  if (!t->mass || !t->com || !t->com0 || !t->bmin || !t->bmax || !t->quad)
    goto fail;
  compute_moments(t);
  memcpy(t->com0, t->com, (size_t)t->n_cell * 3 * sizeof(double));
  if (make_groups(t)) goto fail;
  return t;
fail:
  orc_free(t);
  return NULL;
}

int orc_info(const orc_tree* t, int64_t info[6], double lo[3]) {
  if (!t || !info) return -1;
  info[0] = t->n;
  info[1] = t->n_cell;
  info[2] = t->n_groups;
  info[3] = t->k;
  info[4] = t->n_leaf;
  info[5] = t->n_grp;
  if (lo) memcpy(lo, t->lo, 3 * sizeof(double));
  return 0;
}

int orc_get_keys(const orc_tree* t, uint64_t* key, uint32_t* perm) {
  if (!t) return -1;
  if (key) memcpy(key, t->key, (size_t)t->n * sizeof(uint64_t));
  if (perm) memcpy(perm, t->perm, (size_t)t->n * sizeof(uint32_t));
  return 0;
}

int orc_get_cells(const orc_tree* t, uint64_t* prefix, uint8_t* level,
                  uint32_t* begin, uint32_t* count, uint32_t* parent,
                  uint32_t* skip, uint8_t* leaf, double* ctr3) {
  if (!t) return -1;
  const size_t nc = (size_t)t->n_cell;
  if (prefix) memcpy(prefix, t->prefix, nc * sizeof(uint64_t));
  if (level) memcpy(level, t->level, nc);
  if (begin) memcpy(begin, t->begin, nc * sizeof(uint32_t));
  if (count) memcpy(count, t->count, nc * sizeof(uint32_t));
  if (parent) memcpy(parent, t->parent, nc * sizeof(uint32_t));
  if (skip) memcpy(skip, t->skip, nc * sizeof(uint32_t));
  if (leaf) memcpy(leaf, t->leaf, nc);
  if (ctr3) memcpy(ctr3, t->ctr, nc * 3 * sizeof(double));
  return 0;
}

int orc_get_moments(const orc_tree* t, double* mass, double* com3,
                    double* quad6) {
  if (!t) return -1;
  const size_t nc = (size_t)t->n_cell;
  if (mass) memcpy(mass, t->mass, nc * sizeof(double));
  if (com3) memcpy(com3, t->com, nc * 3 * sizeof(double));
  if (quad6) memcpy(quad6, t->quad, nc * 6 * sizeof(double));
  return 0;
}

int orc_get_groups(const orc_tree* t, uint32_t* cell, uint32_t* begin,
                   uint32_t* count, double* lo3, double* hi3, double* ctr3) {
  if (!t) return -1;
  const size_t ng = (size_t)t->n_groups;
  if (cell) memcpy(cell, t->g_cell, ng * sizeof(uint32_t));
  if (begin) memcpy(begin, t->g_begin, ng * sizeof(uint32_t));
  if (count) memcpy(count, t->g_count, ng * sizeof(uint32_t));
  if (lo3) memcpy(lo3, t->g_lo, ng * 3 * sizeof(double));
  if (hi3) memcpy(hi3, t->g_hi, ng * 3 * sizeof(double));
  if (ctr3) memcpy(ctr3, t->g_ctr, ng * 3 * sizeof(double));
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Opening-test slack of a walk, in length units: sa = the smallest
 * |box - centre| - rcrit over accepted cells, so = the smallest
 * rcrit - |box - centre| over opened cells that do not hold the group
 * (+inf when there is none).  No cell changes side before the box or a
 * centre has moved by the slack. */
typedef struct {
  double sa, so;
} orc_slack;

/* Centre of cell c for the opening test.  Reuse with per-group list
 * refresh (an extension; the paper reuses whole lists, section 4.2): cells
 * keep their particle ranges and each cell's geometric centre is carried
 * along by the displacement of its centre of mass since construction, so
 * that a rigid motion changes no list.  Right after construction the
 * displacement is exactly zero and the test is the plain one. */
static void cell_shift(const orc_tree* t, int64_t c, double tr[3]) {
  for (int a = 0; a < 3; ++a) tr[a] = t->com[3 * c + a] - t->com0[3 * c + a];
}

/* Moved centre of cell c (geometric centre + shift). */
static void moved_centre(const orc_tree* t, int64_t c, double cc[3]) {
  double tr[3];
  cell_shift(t, c, tr);
  for (int a = 0; a < 3; ++a) cc[a] = t->ctr[3 * c + a] + tr[a];
}

/* Side used in the opening test of a refresh walk for cell c: until the
 * first reuse step the geometric side (construction walks are the plain
 * test R6); after it the geometric side or twice the largest per-axis
 * distance from the moved centre cc to the box of the cell's current
 * particles, whichever is larger, so that a cell whose particles spread is
 * opened sooner.  (A particle can sit just outside its cube even at
 * construction, by the rounding of x - lo in the key, so the box rule is
 * not applied before anything has moved.) */
static double side_eff(const orc_tree* t, int64_t c, const double cc[3]) {
  const double s = ldexp(1.0, t->k - t->level[c]);
  if (!t->moved) return s;
  double h = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double up = t->bmax[3 * c + a] - cc[a];
    const double dn = cc[a] - t->bmin[3 * c + a];
    if (up > h) h = up;
    if (dn > h) h = dn;
  }
  const double w = 2.0 * h;
  return w > s ? w : s;
}

/* (side_eff / theta)^2: the squared opening radius of cell c. */
static double crit2(const orc_tree* t, int64_t c, const double cc[3],
                    double theta) {
  const double r = side_eff(t, c, cc) / theta;
  return r * r;
}

int orc_cell_sides(const orc_tree* t, double* side) {
  if (!t || !side) return -1;
  for (int64_t c = 0; c < t->n_cell; ++c) {
    double cc[3];
    moved_centre(t, c, cc);
    side[c] = side_eff(t, c, cc);
  }
  return 0;
}

/* Group tree walk (section 4.3 "construct the interaction lists"; indirect
 * addressing of section 4.1: the lists hold 32-bit indices).  Reading R6.
 * DFS from the root over the pre-order cell array; `skip` jumps over a
 * subtree.  When `fill` is zero only the list lengths are counted.
 * `plain` = 1 is the construction walk: the geometric centre of every cell
 * and its squared opening radius (s/theta)^2.  `plain` = 0 is a refresh
 * walk between construction steps (an extension of section 4.2): moved
 * centres and effective sides. */
static void walk_box(const orc_tree* t, int64_t g, const double* glo,
                     const double* ghi, double theta, int plain, int fill,
                     uint32_t* epj, uint32_t* spj, int64_t* n_epj,
                     int64_t* n_spj, orc_slack* mg) {
  const uint32_t gb = t->g_begin[g];
  const uint64_t ge = (uint64_t)gb + t->g_count[g];
  double sa = INFINITY, so = INFINITY;
  int64_t ne = 0, ns = 0;
  int64_t c = 0;
  while (c < t->n_cell) {
    const uint32_t cb = t->begin[c];
    const uint64_t ce = (uint64_t)cb + t->count[c];
    int open;
    if (cb <= gb && ce >= ge) {
      open = 1; /* the cell holds the group */
    } else {
      double cc[3], d[3], rc;
      if (plain) {
        const double r = ldexp(1.0, t->k - t->level[c]) / theta;
        for (int a = 0; a < 3; ++a) cc[a] = t->ctr[3 * c + a];
        rc = r * r;
      } else {
        moved_centre(t, c, cc);
        rc = crit2(t, c, cc, theta);
      }
      for (int a = 0; a < 3; ++a) {
        double v = 0.0;
        const double below = glo[a] - cc[a];
        const double above = cc[a] - ghi[a];
        if (below > v) v = below;
        if (above > v) v = above;
        d[a] = v;
      }
      const double d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
      open = !(d2 > rc);
      if (mg) {
        const double dd = sqrt(d2), rr = sqrt(rc);
        if (open) {
          if (rr - dd < so) so = rr - dd;
        } else if (dd - rr < sa) {
          sa = dd - rr;
        }
      }
    }
    if (!open) {
      if (fill) spj[ns] = (uint32_t)c;
      ns++;
      c = t->skip[c];
    } else if (t->leaf[c]) {
      for (uint64_t j = cb; j < ce; ++j) {
        if (fill) epj[ne] = (uint32_t)j;
        ne++;
      }
      c = t->skip[c];
    } else {
      c = c + 1;
    }
  }
  *n_epj = ne;
  *n_spj = ns;
  if (mg) {
    mg->sa = sa;
    mg->so = so;
  }
}

/* Tight box of group g's particles at their current positions. */
static void group_box(const orc_tree* t, int64_t g, double lo[3],
                      double hi[3]) {
  const int64_t b = t->g_begin[g], e = b + t->g_count[g];
  const double* p[3] = {t->x, t->y, t->z};
  for (int a = 0; a < 3; ++a) {
    lo[a] = hi[a] = p[a][b];
    for (int64_t i = b + 1; i < e; ++i) {
      if (p[a][i] < lo[a]) lo[a] = p[a][i];
      if (p[a][i] > hi[a]) hi[a] = p[a][i];
    }
  }
}

/* Walk group g with box (lo, hi) and record what the features need. */
static void walk_record(orc_tree* t, int64_t g, double theta, int plain,
                        int fill, uint32_t* epj, uint32_t* spj, int64_t* ne,
                        int64_t* ns) {
  orc_slack mg;
  walk_box(t, g, &t->g_lo[3 * g], &t->g_hi[3 * g], theta, plain, fill, epj,
           spj, ne, ns, &mg);
  if (!fill) {
    t->g_sa[g] = mg.sa;
    t->g_so[g] = mg.so;
    cell_shift(t, t->g_cell[g], &t->g_tau0[3 * g]);
  }
}

int orc_group_margins(const orc_tree* t, double* sa, double* so) {
  if (!t || !sa || !so) return -1;
  memcpy(sa, t->g_sa, (size_t)t->n_groups * sizeof(double));
  memcpy(so, t->g_so, (size_t)t->n_groups * sizeof(double));
  return 0;
}

static int full_lists(const orc_tree* t) {
  return t->have_lists && t->n_sel == t->n_groups;
}

/* Staleness of a kept list (reuse steps): a group's list is stale when one
 * of its superparticles no longer passes the opening test at the relaxed
 * angle theta (1 + tau), measured from the group's current tight box to the
 * cell's current centre (tau = 0: a fresh walk would open that cell).
 * Particles (EPJ) are exact and cells that a fresh walk would accept
 * higher up only cost work, so neither makes a list stale.  Needs lists of
 * every group; also returns the current boxes. */
int orc_group_stale(const orc_tree* t, double theta, double tau,
                    uint8_t* stale, double* lo3, double* hi3) {
  if (!t || !stale || !full_lists(t) || !(tau >= 0.0)) return -1;
  const double th = theta * (1.0 + tau);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t g = 0; g < t->n_groups; ++g) {
    double lo[3], hi[3];
    group_box(t, g, lo, hi);
    if (lo3) memcpy(&lo3[3 * g], lo, sizeof lo);
    if (hi3) memcpy(&hi3[3 * g], hi, sizeof hi);
    int bad = 0;
    for (int64_t j = t->spj_off[g]; j < t->spj_off[g + 1] && !bad; ++j) {
      const uint32_t c = t->spj[j];
      double cc[3], d[3];
      moved_centre(t, c, cc);
      for (int a = 0; a < 3; ++a) {
        double v = 0.0;
        const double below = lo[a] - cc[a];
        const double above = cc[a] - hi[a];
        if (below > v) v = below;
        if (above > v) v = above;
        d[a] = v;
      }
      const double d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
      bad = !(d2 > crit2(t, c, cc, th));
    }
    stale[g] = (uint8_t)bad;
  }
  return 0;
}

/* Per-group list refresh: the listed groups (ascending ids) get their box
 * set to the current tight box and their list walked again; every other
 * list is kept as it is. */
int orc_refresh_lists(orc_tree* t, double theta, int64_t n_sel,
                      const int64_t* sel, int64_t sizes[3]) {
  if (!t || !sizes || n_sel < 0 || (n_sel > 0 && !sel) || !full_lists(t))
    return -1;
  const int64_t G = t->n_groups;
  uint8_t* pick = (uint8_t*)calloc((size_t)(G ? G : 1), 1);
  int64_t* ne = (int64_t*)malloc((size_t)(G ? G : 1) * sizeof(int64_t));
  int64_t* ns = (int64_t*)malloc((size_t)(G ? G : 1) * sizeof(int64_t));
  int64_t* eo = (int64_t*)malloc((size_t)(G + 1) * sizeof(int64_t));
  int64_t* so = (int64_t*)malloc((size_t)(G + 1) * sizeof(int64_t));
  uint32_t *ee = NULL, *ss = NULL;
  int rc = -1;
  if (!pick || !ne || !ns || !eo || !so) goto out;
  for (int64_t i = 0; i < n_sel; ++i) {
    if (sel[i] < 0 || sel[i] >= G || (i > 0 && sel[i] <= sel[i - 1])) goto out;
    pick[sel[i]] = 1;
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t g = 0; g < G; ++g) {
    if (pick[g]) {
      group_box(t, g, &t->g_lo[3 * g], &t->g_hi[3 * g]);
      walk_record(t, g, theta, 0, 0, NULL, NULL, &ne[g], &ns[g]);
    } else {
      ne[g] = t->epj_off[g + 1] - t->epj_off[g];
      ns[g] = t->spj_off[g + 1] - t->spj_off[g];
    }
  }
  eo[0] = so[0] = 0;
  for (int64_t g = 0; g < G; ++g) {
    eo[g + 1] = eo[g] + ne[g];
    so[g + 1] = so[g] + ns[g];
  }
  ee = (uint32_t*)malloc((size_t)(eo[G] + 1) * sizeof(uint32_t));
  ss = (uint32_t*)malloc((size_t)(so[G] + 1) * sizeof(uint32_t));
  if (!ee || !ss) goto out;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t g = 0; g < G; ++g) {
    if (pick[g]) {
      int64_t a, b;
      walk_record(t, g, theta, 0, 1, ee + eo[g], ss + so[g], &a, &b);
    } else {
      memcpy(ee + eo[g], t->epj + t->epj_off[g], (size_t)ne[g] * 4);
      memcpy(ss + so[g], t->spj + t->spj_off[g], (size_t)ns[g] * 4);
    }
  }
  free(t->epj);
  free(t->spj);
  free(t->epj_off);
  free(t->spj_off);
  t->epj = ee;
  t->spj = ss;
  t->epj_off = eo;
  t->spj_off = so;
  ee = ss = NULL;
  eo = so = NULL;
  sizes[0] = G;
  sizes[1] = t->epj_off[G];
  sizes[2] = t->spj_off[G];
  rc = 0;
out:
  free(pick);
  free(ne);
  free(ns);
  free(eo);
  free(so);
  free(ee);
  free(ss);
  return rc;
}

/* Ratio a / b capped at 1e6 (0 / 0 = 0, x / 0 = cap). */
static double capped(double a, double b) {
  const double cap = 1e6;
  if (b > 0.0) {
    const double q = a / b;
    return q < cap ? q : cap;
  }
  return a > 0.0 ? cap : 0.0;
}

/* The 12 inputs of the rebuild predictor for every group (row-major,
 * 12 per group).  With s the side of the group's cell, (lo, hi) its current
 * box, (lo0, hi0), tau0, sa, so the box, cell shift and slacks of the walk
 * that made its list, dtau = (current cell shift) - tau0:
 *   e_a   = max(|lo_a - lo0_a - dtau_a|, |hi_a - hi0_a - dtau_a|)
 *   E = |e|, B = |dtau|, grow = max_a max(0, (hi - lo)_a - (hi0 - lo0)_a)
 *   f0 = min(age, kmax) / kmax
 *   f1..f4 = log1p of E/sa, E/so, B/sa, B/so   (ratios capped at 1e6)
 *   f5, f6 = log1p(E / s), log1p(B / s)
 *   f7, f8 = log1p of sa/s, so/s                (capped)
 *   f9 = log1p(grow / s)
 *   f10 = log2(n_i) / 6, f11 = log2(1 + list length) / 16 */
int orc_group_features(const orc_tree* t, int kmax, const int32_t* age,
                       double* feat) {
  if (!t || kmax < 1 || !age || !feat || !full_lists(t)) return -1;
  for (int64_t g = 0; g < t->n_groups; ++g) {
    const uint32_t c = t->g_cell[g];
    const double s = ldexp(1.0, t->k - t->level[c]);
    double lo[3], hi[3], tr[3], e[3], dt[3];
    group_box(t, g, lo, hi);
    cell_shift(t, c, tr);
    double grow = 0.0;
    for (int a = 0; a < 3; ++a) {
      dt[a] = tr[a] - t->g_tau0[3 * g + a];
      const double dl = fabs((lo[a] - t->g_lo[3 * g + a]) - dt[a]);
      const double dh = fabs((hi[a] - t->g_hi[3 * g + a]) - dt[a]);
      e[a] = dl > dh ? dl : dh;
      const double w = (hi[a] - lo[a]) - (t->g_hi[3 * g + a] - t->g_lo[3 * g + a]);
      if (w > grow) grow = w;
    }
    const double E = sqrt((e[0] * e[0] + e[1] * e[1]) + e[2] * e[2]);
    const double B = sqrt((dt[0] * dt[0] + dt[1] * dt[1]) + dt[2] * dt[2]);
    const double sa = t->g_sa[g], so = t->g_so[g];
    const int64_t nl = (t->epj_off[g + 1] - t->epj_off[g]) +
                       (t->spj_off[g + 1] - t->spj_off[g]);
    double* f = feat + 12 * g;
    f[0] = (double)(age[g] < kmax ? (age[g] > 0 ? age[g] : 0) : kmax) / kmax;
    f[1] = log1p(capped(E, sa));
    f[2] = log1p(capped(E, so));
    f[3] = log1p(capped(B, sa));
    f[4] = log1p(capped(B, so));
    f[5] = log1p(E / s);
    f[6] = log1p(B / s);
    f[7] = log1p(capped(sa, s));
    f[8] = log1p(capped(so, s));
    f[9] = log1p(grow / s);
    f[10] = log2((double)t->g_count[g]) / 6.0;
    f[11] = log2(1.0 + (double)nl) / 16.0;
  }
  return 0;
}

int orc_make_lists(orc_tree* t, double theta, int64_t n_sel,
                   const int64_t* sel, int64_t sizes[3]) {
  if (!t || theta < 0.0 || !sizes) return -1;
  free_lists(t);
  const int64_t ns_all = sel ? n_sel : t->n_groups;
  if (ns_all < 0) return -1;
  t->n_sel = ns_all;
  t->sel = (int64_t*)malloc((size_t)(ns_all ? ns_all : 1) * sizeof(int64_t));
  t->epj_off = (int64_t*)malloc((size_t)(ns_all + 1) * sizeof(int64_t));
  t->spj_off = (int64_t*)malloc((size_t)(ns_all + 1) * sizeof(int64_t));
  if (!t->sel || !t->epj_off || !t->spj_off) return -1;
  for (int64_t s = 0; s < ns_all; ++s) {
    const int64_t g = sel ? sel[s] : s;
    if (g < 0 || g >= t->n_groups) return -1;
    t->sel[s] = g;
  }
  /* count pass */
  int64_t* ne = (int64_t*)malloc((size_t)(ns_all ? ns_all : 1) * sizeof(int64_t));
  int64_t* ns = (int64_t*)malloc((size_t)(ns_all ? ns_all : 1) * sizeof(int64_t));
  if (!ne || !ns) {
    free(ne);
    free(ns);
    return -1;
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t s = 0; s < ns_all; ++s)
    walk_record(t, t->sel[s], theta, 1, 0, NULL, NULL, &ne[s], &ns[s]);
  t->epj_off[0] = t->spj_off[0] = 0;
  for (int64_t s = 0; s < ns_all; ++s) {
    t->epj_off[s + 1] = t->epj_off[s] + ne[s];
    t->spj_off[s + 1] = t->spj_off[s] + ns[s];
  }
  free(ne);
  free(ns);
  t->epj = (uint32_t*)malloc((size_t)(t->epj_off[ns_all] + 1) * sizeof(uint32_t));
  t->spj = (uint32_t*)malloc((size_t)(t->spj_off[ns_all] + 1) * sizeof(uint32_t));
  if (!t->epj || !t->spj) return -1;
  /* fill pass */
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t s = 0; s < ns_all; ++s) {
    int64_t a, b;
    walk_record(t, t->sel[s], theta, 1, 1, t->epj + t->epj_off[s],
                t->spj + t->spj_off[s], &a, &b);
  }
  sizes[0] = ns_all;
  sizes[1] = t->epj_off[ns_all];
  sizes[2] = t->spj_off[ns_all];
  t->have_lists = 1;
  return 0;
}

int orc_get_lists(const orc_tree* t, int64_t* epj_off, uint32_t* epj,
                  int64_t* spj_off, uint32_t* spj) {
  if (!t || !t->have_lists) return -1;
  const size_t s = (size_t)t->n_sel;
  if (epj_off) memcpy(epj_off, t->epj_off, (s + 1) * sizeof(int64_t));
  if (spj_off) memcpy(spj_off, t->spj_off, (s + 1) * sizeof(int64_t));
  if (epj) memcpy(epj, t->epj, (size_t)t->epj_off[s] * sizeof(uint32_t));
  if (spj) memcpy(spj, t->spj, (size_t)t->spj_off[s] * sizeof(uint32_t));
  return 0;
}

/* Reuse step (section 4.2): particle order, cells, groups and lists stay as
 * built; only the particle data and the moments are refreshed. */
int orc_refresh(orc_tree* t, const double* x, const double* y,
                const double* z, const double* m) {
  if (!t || !x || !y || !z || !m) return -1;
  for (int64_t i = 0; i < t->n; ++i) {
    const uint32_t s = t->perm[i];
    t->x[i] = x[s];
    t->y[i] = y[s];
    t->z[i] = z[s];
    t->m[i] = m[s];
  }
  compute_moments(t);
  t->moved = 1;
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Forces from the interaction lists (section 4.3: the kernel evaluates the
 * pull of the EPJ and SPJ of each list on the particles of its group).
 * Readings R7 and R8. */
int orc_force_lists(const orc_tree* t, int order, double eps, double G,
                    double* ax, double* ay, double* az, double* pot) {
  if (!t || !t->have_lists || !ax || !ay || !az || !pot) return -1;
  if (order != 1 && order != 2) return -1;
  const double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t s = 0; s < t->n_sel; ++s) {
    const int64_t g = t->sel[s];
    const int64_t b = t->g_begin[g], e = b + t->g_count[g];
    for (int64_t i = b; i < e; ++i) {
      const double xi = t->x[i], yi = t->y[i], zi = t->z[i];
      double fx = 0.0, fy = 0.0, fz = 0.0, ph = 0.0;
      for (int64_t q = t->epj_off[s]; q < t->epj_off[s + 1]; ++q) {
        const int64_t j = t->epj[q];
        if (j == i) continue;
        const double dx = t->x[j] - xi, dy = t->y[j] - yi, dz = t->z[j] - zi;
        const double r2 = dx * dx + dy * dy + dz * dz + eps2;
        const double rinv = 1.0 / sqrt(r2);
        const double mr = G * t->m[j] * rinv;
        const double mr3 = mr * rinv * rinv;
        fx += mr3 * dx;
        fy += mr3 * dy;
        fz += mr3 * dz;
        ph -= mr;
      }
      for (int64_t q = t->spj_off[s]; q < t->spj_off[s + 1]; ++q) {
        const int64_t c = t->spj[q];
        const double* X = &t->com[3 * c];
        const double M = t->mass[c];
        /* r points from the expansion centre to the particle */
        const double r[3] = {xi - X[0], yi - X[1], zi - X[2]};
        const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + eps2;
        const double f = 1.0 / sqrt(r2);
        const double f2 = f * f, f3 = f2 * f;
        double acc[3] = {-M * f3 * r[0], -M * f3 * r[1], -M * f3 * r[2]};
        double phi = -M * f;
        if (order == 2) {
          const double* S = &t->quad[6 * c];
          /* S r with S = [[xx,xy,xz],[xy,yy,yz],[xz,yz,zz]] */
          const double Sr[3] = {S[0] * r[0] + S[3] * r[1] + S[4] * r[2],
                                S[3] * r[0] + S[1] * r[1] + S[5] * r[2],
                                S[4] * r[0] + S[5] * r[1] + S[2] * r[2]};
          const double qq = r[0] * Sr[0] + r[1] * Sr[1] + r[2] * Sr[2];
          const double tr = S[0] + S[1] + S[2];
          const double f5 = f3 * f2, f7 = f5 * f2;
          phi -= (3.0 * qq * f2 - tr) * f3 / 2.0;
          for (int a = 0; a < 3; ++a)
            acc[a] += 3.0 * Sr[a] * f5 - 7.5 * qq * r[a] * f7 +
                      1.5 * tr * r[a] * f5;
        }
        fx += G * acc[0];
        fy += G * acc[1];
        fz += G * acc[2];
        ph += G * phi;
      }
      const uint32_t o = t->perm[i];
      ax[o] = fx;
      ay[o] = fy;
      az[o] = fz;
      pot[o] = ph;
    }
  }
  return 0;
}

/* Direct summation, the quantity the tree method approximates. */
int orc_force_direct(int64_t n, const double* x, const double* y,
                     const double* z, const double* m, double eps, double G,
                     int64_t n_tgt, const int64_t* tgt, double* ax,
                     double* ay, double* az, double* pot) {
  if (n < 0 || n_tgt < 0 || !x || !y || !z || !m || !tgt || !ax || !ay ||
      !az || !pot)
    return -1;
  const double eps2 = eps * eps;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
  for (int64_t s = 0; s < n_tgt; ++s) {
    const int64_t i = tgt[s];
    if (i < 0 || i >= n) {
      bad = 1;
      continue;
    }
    double fx = 0.0, fy = 0.0, fz = 0.0, ph = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      const double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
      const double r2 = dx * dx + dy * dy + dz * dz + eps2;
      const double rinv = 1.0 / sqrt(r2);
      const double mr = G * m[j] * rinv;
      const double mr3 = mr * rinv * rinv;
      fx += mr3 * dx;
      fy += mr3 * dy;
      fz += mr3 * dz;
      ph -= mr;
    }
    ax[s] = fx;
    ay[s] = fy;
    az[s] = fz;
    pot[s] = ph;
  }
  return bad ? -1 : 0;
}

/* Kick-drift (section 4.3: after the force the orbits are integrated; the
 * paper does not name the integrator -- KDK leapfrog is used, adjacent half
 * kicks merged into one call). */
int orc_kick_drift(int64_t n, double* x, double* y, double* z, double* vx,
                   double* vy, double* vz, const double* ax,
                   const double* ay, const double* az, double dt_kick,
                   double dt_drift, double ext_mass, double G) {
  if (n < 0 || !x || !y || !z || !vx || !vy || !vz || !ax || !ay || !az)
    return -1;
  for (int64_t i = 0; i < n; ++i) {
    double gx = ax[i], gy = ay[i], gz = az[i];
    if (ext_mass != 0.0) {
      const double r2 = x[i] * x[i] + y[i] * y[i] + z[i] * z[i];
      const double r = sqrt(r2);
      const double k = G * ext_mass / (r2 * r);
      gx -= k * x[i];
      gy -= k * y[i];
      gz -= k * z[i];
    }
    vx[i] += gx * dt_kick;
    vy[i] += gy * dt_kick;
    vz[i] += gz * dt_kick;
    x[i] += vx[i] * dt_drift;
    y[i] += vy[i] * dt_drift;
    z[i] += vz[i] * dt_drift;
  }
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Short-range interactions (section 2: the same group-wise walk with an
 * opening criterion other than the opening angle; section 4.2: such lists
 * are reused over several steps).  Reading R18: with one search radius h,
 * a cell that holds the group is opened; any other cell is opened when its
 * cube overlaps the group's tight box grown by h on every side, i.e. when
 * on every axis the gap between the box and the cell's centre is at most
 * half the side plus h, and is skipped with its subtree otherwise; an
 * opened leaf puts its particles on the list.  Every particle within h of a
 * member (max norm, hence also Euclidean) is on the group's list. */
static void nbr_walk(const orc_tree* t, int64_t g, double h, uint32_t* out,
                     int64_t* n_out) {
  const uint32_t gb = t->g_begin[g];
  const uint64_t ge = (uint64_t)gb + t->g_count[g];
  const double* lo = &t->g_lo[3 * g];
  const double* hi = &t->g_hi[3 * g];
  int64_t ne = 0;
  int64_t c = 0;
  while (c < t->n_cell) {
    const uint32_t cb = t->begin[c];
    const uint64_t ce = (uint64_t)cb + t->count[c];
    int open = 1;
    if (!(cb <= gb && ce >= ge)) {
      const double r = ldexp(1.0, t->k - t->level[c] - 1) + h;
      for (int a = 0; a < 3; ++a) {
        double v = 0.0;
        const double below = lo[a] - t->ctr[3 * c + a];
        const double above = t->ctr[3 * c + a] - hi[a];
        if (below > v) v = below;
        if (above > v) v = above;
        if (v > r) open = 0;
      }
    }
    if (!open) {
      c = t->skip[c];
    } else if (t->leaf[c]) {
      for (uint64_t j = cb; j < ce; ++j) {
        if (out) out[ne] = (uint32_t)j;
        ne++;
      }
      c = t->skip[c];
    } else {
      c = c + 1;
    }
  }
  *n_out = ne;
}

int orc_neighbour_lists(orc_tree* t, double h, int64_t* n_entries) {
  if (!t || !(h >= 0.0) || !isfinite(h) || !n_entries) return -1;
  free(t->nb_off);
  free(t->nb);
  t->nb = NULL;
  t->have_nbr = 0;
  const int64_t ng = t->n_groups;
  t->nb_off = (int64_t*)malloc((size_t)(ng + 1) * sizeof(int64_t));
  int64_t* cnt = (int64_t*)malloc((size_t)(ng ? ng : 1) * sizeof(int64_t));
  if (!t->nb_off || !cnt) {
    free(cnt);
    return -1;
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t g = 0; g < ng; ++g) nbr_walk(t, g, h, NULL, &cnt[g]);
  t->nb_off[0] = 0;
  for (int64_t g = 0; g < ng; ++g) t->nb_off[g + 1] = t->nb_off[g] + cnt[g];
  free(cnt);
  t->nb = (uint32_t*)malloc((size_t)(t->nb_off[ng] + 1) * sizeof(uint32_t));
  if (!t->nb) return -1;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t g = 0; g < ng; ++g) {
    int64_t k;
    nbr_walk(t, g, h, t->nb + t->nb_off[g], &k);
  }
  t->have_nbr = 1;
  *n_entries = t->nb_off[ng];
  return 0;
}

int orc_get_neighbour_lists(const orc_tree* t, int64_t* off, uint32_t* ids) {
  if (!t || !t->have_nbr) return -1;
  if (off) memcpy(off, t->nb_off, (size_t)(t->n_groups + 1) * sizeof(int64_t));
  if (ids) memcpy(ids, t->nb, (size_t)t->nb_off[t->n_groups] * sizeof(uint32_t));
  return 0;
}

/* The SPH kernel (reading R18): cubic spline of compact support h,
 * W(r, h) = 8 / (pi h^3) w(r / h), w(q) = 1 - 6 q^2 + 6 q^3 on [0, 1/2],
 * 2 (1 - q)^3 on (1/2, 1], 0 beyond. */
double orc_sph_w(double r, double h) {
  const double q = r / h;
  double w = 0.0;
  if (q <= 0.5) {
    w = 1.0 - 6.0 * q * q + 6.0 * q * q * q;
  } else if (q <= 1.0) {
    const double u = 1.0 - q;
    w = 2.0 * u * u * u;
  }
  return 8.0 / (3.14159265358979323846 * h * h * h) * w;
}

/* SPH density over the neighbour lists at the positions of the last
 * orc_build / orc_refresh: rho_i = sum over the list of i's group of
 * m_j W(|x_i - x_j|, h), the particle itself included.  Input order. */
int orc_sph_density(const orc_tree* t, double h, double* rho) {
  if (!t || !t->have_nbr || !rho || !(h > 0.0) || !isfinite(h)) return -1;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t g = 0; g < t->n_groups; ++g) {
    const int64_t b = t->g_begin[g], e = b + t->g_count[g];
    for (int64_t i = b; i < e; ++i) {
      double sum = 0.0;
      for (int64_t q = t->nb_off[g]; q < t->nb_off[g + 1]; ++q) {
        const int64_t j = t->nb[q];
        const double dx = t->x[j] - t->x[i], dy = t->y[j] - t->y[i],
                     dz = t->z[j] - t->z[i];
        sum += t->m[j] * orc_sph_w(sqrt(dx * dx + dy * dy + dz * dz), h);
      }
      rho[t->perm[i]] = sum;
    }
  }
  return 0;
}

/* The same density over all pairs (the quantity the lists must reproduce). */
int orc_sph_density_direct(int64_t n, const double* x, const double* y,
                           const double* z, const double* m, double h,
                           double* rho) {
  if (n < 0 || !x || !y || !z || !m || !rho || !(h > 0.0)) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double sum = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      const double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
      sum += m[j] * orc_sph_w(sqrt(dx * dx + dy * dy + dz * dz), h);
    }
    rho[i] = sum;
  }
  return 0;
}
