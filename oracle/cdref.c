/* cdref.c - FP64 CPU oracle of the Contact Dynamics contact-force solve.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Written to be
 * read against the paper (Shojaaee et al., Sec. 2-3): plain loops, no
 * blocking, no fusion, every step in the paper's order.  Built with
 * -O2 -ffp-contract=off so that every floating-point operation is the IEEE
 * operation written here.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *  - the gap entering the force law is max(g, 0) unless overlap_mode = 1
 *    (initial overlaps are not pushed apart in one step);
 *  - the order inside a domain is a greedy colouring in canonical order
 *    (instead of a random order), which is an exact sequential order;
 *  - |R| is the Euclidean norm of the contact force and R_avg the mean of
 *    |R| over all listed contacts; a relative test with 0/0 passes;
 *  - bisection cuts are placed by contact count at the k-th smallest
 *    contact position, k = floor(n L_left / (L_left + L_right)), with the
 *    cut axis along the longest side of the node's region.
 */
#include "cdref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* small vector helpers (component order fixed: 0, 1, 2)               */
/* ------------------------------------------------------------------ */

/* Tangent basis (t1, t2) of a unit normal in 3D, right-handed with
 * t1 x t2 = n.  Construction of Duff et al., "Building an orthonormal
 * basis, revisited", JCGT 6(1), 2017.  In 2D the tangent is t = z x n. */
static void tangent_basis3(const double n[3], double t1[3], double t2[3]) {
  double sign = copysign(1.0, n[2]);
  double a = -1.0 / (sign + n[2]);
  double b = n[0] * n[1] * a;
  t1[0] = 1.0 + sign * n[0] * n[0] * a;
  t1[1] = sign * b;
  t1[2] = -sign * n[0];
  t2[0] = b;
  t2[1] = sign + n[1] * n[1] * a;
  t2[2] = -n[1];
}

static void contact_frame(int dim, const double* normal, int64_t nc, int64_t c,
                          double n[3], double t1[3], double t2[3]) {
  for (int k = 0; k < 3; ++k) n[k] = t1[k] = t2[k] = 0.0;
  for (int k = 0; k < dim; ++k) n[k] = normal[k * nc + c];
  if (dim == 2) {
    t1[0] = -n[1];
    t1[1] = n[0];
    t2[2] = 1.0;
  } else {
    tangent_basis3(n, t1, t2);
  }
}

/* Separation along a periodic axis of length L (the benchmark boxes of
 * Sec. 4.1 are periodic in x): the nearest image, |d| <= L/2. */
static double min_image(double d, double L) {
  if (d > 0.5 * L) return d - L;
  if (d < -0.5 * L) return d + L;
  return d;
}

/* A coordinate back into [lo, lo + L) after it left by less than L. */
static double wrap_into(double q, double lo, double L) {
  if (q >= lo + L) return q - L;
  if (q < lo) return q + L;
  return q;
}

/* gap between particle i and body j (particle or wall), Sec. 2.1 / Fig. 1;
 * period (NULL: none) holds the length of each periodic axis, 0 for open
 * ones, and particle pairs are taken at their nearest image */
static double pair_gap(int dim, int64_t n, const double* x, const double* r,
                       const double* wall_normal, const double* wall_offset,
                       int64_t i, int64_t j, double nrm[3], const double* period) {
  if (j < n) {
    double delta[3] = {0, 0, 0};
    double d2 = 0.0;
    for (int k = 0; k < dim; ++k) {
      delta[k] = x[k * n + j] - x[k * n + i];
      if (period && period[k] > 0.0) delta[k] = min_image(delta[k], period[k]);
      d2 = d2 + delta[k] * delta[k];
    }
    double dist = sqrt(d2);
    if (nrm) for (int k = 0; k < dim; ++k) nrm[k] = delta[k] / dist;
    return (dist - r[i]) - r[j];
  } else {
    int64_t w = j - n;
    double proj = 0.0;
    for (int k = 0; k < dim; ++k) proj = proj + wall_normal[w * dim + k] * x[k * n + i];
    if (nrm) for (int k = 0; k < dim; ++k) nrm[k] = -wall_normal[w * dim + k];
    return (proj - wall_offset[w]) - r[i];
  }
}

/* ------------------------------------------------------------------ */
/* contact detection (Sec. 3.1 boundary width, Sec. 3.2 cell method)   */
/* ------------------------------------------------------------------ */

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

int cdref_detect(int dim, int64_t n, const double* x, const double* r,
                 int n_walls, const double* wall_normal, const double* wall_offset,
                 double skin, int use_cells, const double* box_lo, const double* box_hi,
                 int64_t cap, int32_t* ci, int32_t* cj, int64_t* nc) {
  return cdref_detect_bc(dim, n, x, r, n_walls, wall_normal, wall_offset, skin, use_cells,
                         box_lo, box_hi, NULL, cap, ci, cj, nc);
}

int cdref_detect_bc(int dim, int64_t n, const double* x, const double* r,
                    int n_walls, const double* wall_normal, const double* wall_offset,
                    double skin, int use_cells, const double* box_lo, const double* box_hi,
                    const double* period, int64_t cap, int32_t* ci, int32_t* cj, int64_t* nc) {
  int64_t count = 0;
  if (dim != 2 && dim != 3) return CDREF_EINVAL;
  if (!use_cells) {
    for (int64_t i = 0; i < n; ++i) {
      for (int64_t j = i + 1; j < n; ++j) {
        if (pair_gap(dim, n, x, r, wall_normal, wall_offset, i, j, NULL, period) <= skin) {
          if (count < cap) { ci[count] = (int32_t)i; cj[count] = (int32_t)j; }
          ++count;
        }
      }
      for (int w = 0; w < n_walls; ++w) {
        if (pair_gap(dim, n, x, r, wall_normal, wall_offset, i, n + w, NULL, period) <= skin) {
          if (count < cap) { ci[count] = (int32_t)i; cj[count] = (int32_t)(n + w); }
          ++count;
        }
      }
    }
    *nc = count;
    return count > cap ? CDREF_ECAPACITY : CDREF_OK;
  }
  /* cell method: mesh >= 2.2 r_max and >= the largest possible centre distance */
  double rmax = 0.0;
  for (int64_t i = 0; i < n; ++i) if (r[i] > rmax) rmax = r[i];
  double a = 2.2 * rmax;
  if (2.0 * rmax + skin > a) a = 2.0 * rmax + skin;
  int64_t ncell[3] = {1, 1, 1};
  double width[3] = {1, 1, 1};
  for (int k = 0; k < dim; ++k) {
    double len = box_hi[k] - box_lo[k];
    int64_t m = (int64_t)floor(len / a);
    if (m < 1) m = 1;
    if (m > 4096) m = 4096;
    ncell[k] = m;
    width[k] = len / (double)m;
    /* a periodic axis needs three cells so that the neighbour cells of a
       cell are distinct and a pair is seen at one image only */
    if (period && period[k] > 0.0 && m < 3) return CDREF_EINVAL;
  }
  int64_t total = ncell[0] * ncell[1] * ncell[2];
  int64_t* cell = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t* start = (int64_t*)calloc((size_t)(total + 1), sizeof(int64_t));
  int64_t* members = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(total + 1));
  int32_t* cand = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!cell || !start || !members || !fill || !cand) {
    free(cell); free(start); free(members); free(fill); free(cand);
    return CDREF_ENOMEM;
  }
  int64_t ic[3];
  for (int64_t i = 0; i < n; ++i) {
    for (int k = 0; k < 3; ++k) ic[k] = 0;
    for (int k = 0; k < dim; ++k) {
      double q = floor((x[k * n + i] - box_lo[k]) / width[k]);
      int64_t m = q < 0.0 ? 0 : (q > (double)(ncell[k] - 1) ? ncell[k] - 1 : (int64_t)q);
      ic[k] = m;
    }
    cell[i] = (ic[2] * ncell[1] + ic[1]) * ncell[0] + ic[0];
    start[cell[i] + 1] += 1;
  }
  for (int64_t c = 0; c < total; ++c) start[c + 1] += start[c];
  memcpy(fill, start, sizeof(int64_t) * (size_t)(total + 1));
  for (int64_t i = 0; i < n; ++i) members[fill[cell[i]]++] = i;

  for (int64_t i = 0; i < n; ++i) {
    int64_t c = cell[i];
    int64_t cx = c % ncell[0], cy = (c / ncell[0]) % ncell[1], cz = c / (ncell[0] * ncell[1]);
    int ncand = 0;
    for (int64_t dz = -1; dz <= 1; ++dz) {
      for (int64_t dy = -1; dy <= 1; ++dy) {
        for (int64_t dx = -1; dx <= 1; ++dx) {
          int64_t qx = cx + dx, qy = cy + dy, qz = cz + dz;
          /* periodic axes: the neighbour cells wrap around */
          if (period && period[0] > 0.0) qx = (qx + ncell[0]) % ncell[0];
          if (period && dim > 1 && period[1] > 0.0) qy = (qy + ncell[1]) % ncell[1];
          if (period && dim > 2 && period[2] > 0.0) qz = (qz + ncell[2]) % ncell[2];
          if (qx < 0 || qy < 0 || qz < 0 || qx >= ncell[0] || qy >= ncell[1] || qz >= ncell[2])
            continue;
          int64_t q = (qz * ncell[1] + qy) * ncell[0] + qx;
          for (int64_t s = start[q]; s < start[q + 1]; ++s) {
            int64_t j = members[s];
            if (j <= i) continue;
            if (pair_gap(dim, n, x, r, wall_normal, wall_offset, i, j, NULL, period) <= skin)
              cand[ncand++] = (int32_t)j;
          }
        }
      }
    }
    qsort(cand, (size_t)ncand, sizeof(int32_t), cmp_i32);
    for (int s = 0; s < ncand; ++s) {
      if (count < cap) { ci[count] = (int32_t)i; cj[count] = cand[s]; }
      ++count;
    }
    for (int w = 0; w < n_walls; ++w) {
      if (pair_gap(dim, n, x, r, wall_normal, wall_offset, i, n + w, NULL, period) <= skin) {
        if (count < cap) { ci[count] = (int32_t)i; cj[count] = (int32_t)(n + w); }
        ++count;
      }
    }
  }
  free(cell); free(start); free(members); free(fill); free(cand);
  *nc = count;
  return count > cap ? CDREF_ECAPACITY : CDREF_OK;
}

void cdref_geometry(int dim, int64_t n, const double* x, const double* r,
                    int n_walls, const double* wall_normal, const double* wall_offset,
                    int64_t nc, const int32_t* ci, const int32_t* cj,
                    double* normal, double* gap, double* xmid) {
  cdref_geometry_bc(dim, n, x, r, n_walls, wall_normal, wall_offset, NULL, NULL, nc, ci, cj,
                    normal, gap, xmid);
}

void cdref_geometry_bc(int dim, int64_t n, const double* x, const double* r,
                       int n_walls, const double* wall_normal, const double* wall_offset,
                       const double* period, const double* box_lo, int64_t nc,
                       const int32_t* ci, const int32_t* cj, double* normal, double* gap,
                       double* xmid) {
  (void)n_walls;
  for (int64_t c = 0; c < nc; ++c) {
    double nrm[3];
    int64_t i = ci[c], j = cj[c];
    double g = pair_gap(dim, n, x, r, wall_normal, wall_offset, i, j, nrm, period);
    gap[c] = g;
    double lever = r[i] + 0.5 * g;   /* middle of the gap, Sec. 3.1 */
    for (int k = 0; k < dim; ++k) {
      normal[k * nc + c] = nrm[k];
      xmid[k * nc + c] = x[k * n + i] + lever * nrm[k];
      /* on a periodic axis the position is taken back into the box */
      if (period && period[k] > 0.0)
        xmid[k * nc + c] = wrap_into(xmid[k * nc + c], box_lo[k], period[k]);
    }
  }
}

/* ------------------------------------------------------------------ */
/* hierarchical domain tree (Sec. 3.2, Fig. 8)                          */
/* ------------------------------------------------------------------ */

typedef struct {
  int count;
  int32_t* child;   /* 2 per node */
  int32_t* leaf;    /* domain id or -1 */
  int32_t* leaves;  /* leaf count below the node */
} tree_shape;

static int tree_shape_build(int P, tree_shape* t) {
  int total = 2 * P - 1;
  t->count = total;
  t->child = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)total);
  t->leaf = (int32_t*)malloc(sizeof(int32_t) * (size_t)total);
  t->leaves = (int32_t*)malloc(sizeof(int32_t) * (size_t)total);
  if (!t->child || !t->leaf || !t->leaves) return CDREF_ENOMEM;
  for (int k = 0; k < 2 * total; ++k) t->child[k] = -1;
  /* level by level: branch every node of a level until 2^l < P <= 2^(l+1),
     then branch only the first P - 2^l nodes of level l, left to right */
  int created = 1;
  int level_begin = 0, level_size = 1;
  if (P > 1) {
    int l = 0;
    while ((1 << (l + 1)) < P) ++l;      /* now 2^l < P <= 2^(l+1) */
    for (int m = 0; m < l; ++m) {
      for (int q = 0; q < level_size; ++q) {
        int node = level_begin + q;
        t->child[2 * node] = created++;
        t->child[2 * node + 1] = created++;
      }
      level_begin += level_size;
      level_size *= 2;
    }
    int extra = P - (1 << l);
    for (int q = 0; q < extra; ++q) {
      int node = level_begin + q;
      t->child[2 * node] = created++;
      t->child[2 * node + 1] = created++;
    }
  }
  if (created != total) return CDREF_EINVAL;
  /* leaves numbered left to right by a depth-first walk */
  int* stack = (int*)malloc(sizeof(int) * (size_t)total);
  int* post = (int*)malloc(sizeof(int) * (size_t)total);
  if (!stack || !post) { free(stack); free(post); return CDREF_ENOMEM; }
  int sp = 0, next_leaf = 0, npost = 0;
  stack[sp++] = 0;
  while (sp > 0) {
    int node = stack[--sp];
    post[npost++] = node;
    if (t->child[2 * node] < 0) {
      t->leaf[node] = next_leaf++;
    } else {
      t->leaf[node] = -1;
      stack[sp++] = t->child[2 * node + 1];   /* right pushed first: left visited first */
      stack[sp++] = t->child[2 * node];
    }
  }
  /* leaf counts: children are always created after their parent */
  for (int node = total - 1; node >= 0; --node) {
    if (t->child[2 * node] < 0) t->leaves[node] = 1;
    else t->leaves[node] = t->leaves[t->child[2 * node]] + t->leaves[t->child[2 * node + 1]];
  }
  free(stack); free(post);
  return CDREF_OK;
}

static void tree_shape_free(tree_shape* t) {
  free(t->child); free(t->leaf); free(t->leaves);
}

int cdref_tree_leaves(int P, int32_t* node_leaves) {
  if (P < 1) return CDREF_EINVAL;
  tree_shape t;
  int st = tree_shape_build(P, &t);
  if (st == CDREF_OK) memcpy(node_leaves, t.leaves, sizeof(int32_t) * (size_t)t.count);
  tree_shape_free(&t);
  return st;
}

static int cmp_f64(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

/* ------------------------------------------------------------------ */
/* mixed sequential/parallel update (Sec. 2.3)                          */
/* ------------------------------------------------------------------ */

/* SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014): the finaliser applied to x + golden gamma. */
static uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* A uniform number in [0, 1) for the pair (i, j): the top 53 bits of
 * SplitMix64(SplitMix64(SplitMix64(seed) ^ i) ^ j). */
double cdref_pair_uniform(uint64_t seed, int64_t i, int64_t j) {
  uint64_t h = splitmix64(splitmix64(splitmix64(seed) ^ (uint64_t)i) ^ (uint64_t)j);
  return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

/* The contacts updated in parallel: those whose pair number falls below p. */
void cdref_parallel_flags(int64_t nc, const int32_t* ci, const int32_t* cj, double p,
                          uint64_t seed, uint8_t* flags) {
  for (int64_t c = 0; c < nc; ++c)
    flags[c] = cdref_pair_uniform(seed, ci[c], cj[c]) < p ? 1 : 0;
}

/* ------------------------------------------------------------------ */
/* random sequential order (Sec. 2.1)                                   */
/* ------------------------------------------------------------------ */

/* The key of time step `step`: SplitMix64(SplitMix64(seed) ^ step). */
uint64_t cdref_random_step_key(uint64_t seed, int64_t step) {
  return splitmix64(splitmix64(seed) ^ (uint64_t)step);
}

/* The draw of slot s in sweep j (1-based) of the step with key k:
 * SplitMix64(SplitMix64(k ^ j) ^ s).  A domain updates its contacts in the
 * order of increasing draw, equal draws by slot. */
uint64_t cdref_random_slot_key(uint64_t step_key, int j, int64_t s) {
  return splitmix64(splitmix64(step_key ^ (uint64_t)j) ^ (uint64_t)s);
}

typedef struct {
  uint64_t key;
  int64_t slot;
} rand_slot;

/* threads over which the domains of a sweep are spread (1: serial) */
static int g_threads = 1;

void cdref_set_threads(int threads) { g_threads = threads > 1 ? threads : 1; }

static int rand_slot_cmp(const void* a, const void* b) {
  const rand_slot* x = (const rand_slot*)a;
  const rand_slot* y = (const rand_slot*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return x->slot < y->slot ? -1 : (x->slot > y->slot ? 1 : 0);
}

/* ------------------------------------------------------------------ */
/* adaptive load balancing (Sec. 3.3)                                   */
/* ------------------------------------------------------------------ */

/* Load imbalance of a step (Sec. 3.3): sigma_T = sqrt(<T^2> - <T>^2) / <T>,
 * the averages taken over the P domains' times. */
double cdref_sigma_t(int P, const double* T) {
  if (P < 1) return 0.0;
  double s = 0.0, s2 = 0.0;
  for (int i = 0; i < P; ++i) {
    s = s + T[i];
    s2 = s2 + T[i] * T[i];
  }
  double mean = s / (double)P, mean2 = s2 / (double)P;
  double var = mean2 - mean * mean;
  if (var < 0.0) var = 0.0;
  return mean > 0.0 ? sqrt(var) / mean : 0.0;
}

/* Share of its node's contacts that the left branch of every inner node
 * receives (Sec. 3.3): nu_L / (nu_L + nu_R), where nu of a branch sums the
 * capacities of the leaves below it (the paper's nu_j = sum V_i / T_i; here
 * a capacity is the contacts a domain handled per unit time).  A capacity
 * that is not positive and finite carries no measurement and counts as the
 * mean of the valid ones (1 when there are none).  node_frac has 2P-1
 * entries in creation order (0 for leaves). */
static int balance_fractions(const tree_shape* t, const double* capacity, double* node_frac) {
  double* nu = (double*)malloc(sizeof(double) * (size_t)t->count);
  if (!nu) return CDREF_ENOMEM;
  double sum = 0.0;
  int valid = 0;
  int P = (t->count + 1) / 2;
  for (int i = 0; i < P; ++i) {
    if (capacity[i] > 0.0 && isfinite(capacity[i])) {
      sum = sum + capacity[i];
      ++valid;
    }
  }
  double fill = valid > 0 ? sum / (double)valid : 1.0;
  /* children are created after their parents: reverse creation order is
     bottom-up */
  for (int node = t->count - 1; node >= 0; --node) {
    int left = t->child[2 * node], right = t->child[2 * node + 1];
    if (left < 0) {
      double c = capacity[t->leaf[node]];
      nu[node] = (c > 0.0 && isfinite(c)) ? c : fill;
      node_frac[node] = 0.0;
    } else {
      nu[node] = nu[left] + nu[right];
      node_frac[node] = nu[left] / nu[node];
    }
  }
  free(nu);
  return CDREF_OK;
}

int cdref_balance_fractions(int P, const double* capacity, double* node_frac) {
  if (P < 1) return CDREF_EINVAL;
  tree_shape t;
  int st = tree_shape_build(P, &t);
  if (st == CDREF_OK) st = balance_fractions(&t, capacity, node_frac);
  tree_shape_free(&t);
  return st;
}

/* split `node` owning contacts ids[0..cnt) in region [lo, hi]; frac (or
   NULL: leaf counts) gives the left branch's share of the contacts */
static void orb_split(int dim, const tree_shape* t, const double* frac, int node,
                      const double* lo, const double* hi, int64_t nc, const double* xmid,
                      int32_t* ids, int64_t cnt, int32_t* node_axis, double* node_cut,
                      int32_t* dom, double* scratch, int32_t* tmp_ids) {
  if (t->child[2 * node] < 0) {
    node_axis[node] = -1;
    node_cut[node] = 0.0;
    for (int64_t s = 0; s < cnt; ++s) dom[ids[s]] = t->leaf[node];
    return;
  }
  /* cut perpendicular to the longest side (shortest interface), ties to x,y,z */
  int axis = 0;
  double best = hi[0] - lo[0];
  for (int k = 1; k < dim; ++k) {
    if (hi[k] - lo[k] > best) { best = hi[k] - lo[k]; axis = k; }
  }
  int left = t->child[2 * node], right = t->child[2 * node + 1];
  int64_t ll = t->leaves[left], lr = t->leaves[right];
  double cut;
  if (cnt > 0) {
    for (int64_t s = 0; s < cnt; ++s) scratch[s] = xmid[(int64_t)axis * nc + ids[s]];
    qsort(scratch, (size_t)cnt, sizeof(double), cmp_f64);
    int64_t k;
    if (frac) {
      /* share of contacts = share of capacity (Sec. 3.3) */
      k = (int64_t)floor((double)cnt * frac[node]);
      if (k > cnt - 1) k = cnt - 1;
      if (k < 0) k = 0;
    } else {
      k = (cnt * ll) / (ll + lr);   /* share of contacts ~ share of leaves */
    }
    cut = scratch[k];
  } else {
    cut = 0.5 * (lo[axis] + hi[axis]);
  }
  node_axis[node] = axis;
  node_cut[node] = cut;
  /* stable partition: coordinate < cut goes left, ties go right */
  int64_t nl = 0, nr = 0;
  for (int64_t s = 0; s < cnt; ++s) {
    if (xmid[(int64_t)axis * nc + ids[s]] < cut) ids[nl++] = ids[s];
    else tmp_ids[nr++] = ids[s];
  }
  memcpy(ids + nl, tmp_ids, sizeof(int32_t) * (size_t)nr);
  double llo[3], lhi[3], rlo[3], rhi[3];
  for (int k = 0; k < dim; ++k) { llo[k] = rlo[k] = lo[k]; lhi[k] = rhi[k] = hi[k]; }
  lhi[axis] = cut;
  rlo[axis] = cut;
  orb_split(dim, t, frac, left, llo, lhi, nc, xmid, ids, nl, node_axis, node_cut, dom, scratch,
            tmp_ids);
  orb_split(dim, t, frac, right, rlo, rhi, nc, xmid, ids + nl, nr, node_axis, node_cut, dom,
            scratch, tmp_ids);
}

int cdref_orb(int dim, int P, const double* box_lo, const double* box_hi,
              int64_t nc, const double* xmid,
              int32_t* node_axis, double* node_cut, int32_t* node_child,
              int32_t* node_leaf, int32_t* node_leaves, int32_t* dom) {
  return cdref_orb_capacity(dim, P, box_lo, box_hi, nc, xmid, NULL, node_axis, node_cut,
                            node_child, node_leaf, node_leaves, dom);
}

int cdref_orb_capacity(int dim, int P, const double* box_lo, const double* box_hi,
                       int64_t nc, const double* xmid, const double* capacity,
                       int32_t* node_axis, double* node_cut, int32_t* node_child,
                       int32_t* node_leaf, int32_t* node_leaves, int32_t* dom) {
  if (P < 1 || (dim != 2 && dim != 3)) return CDREF_EINVAL;
  tree_shape t;
  int st = tree_shape_build(P, &t);
  if (st != CDREF_OK) { tree_shape_free(&t); return st; }
  double* frac = NULL;
  if (capacity) {
    frac = (double*)malloc(sizeof(double) * (size_t)t.count);
    if (!frac) { tree_shape_free(&t); return CDREF_ENOMEM; }
    st = balance_fractions(&t, capacity, frac);
    if (st != CDREF_OK) { free(frac); tree_shape_free(&t); return st; }
  }
  int32_t* ids = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
  int32_t* tmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
  double* scratch = (double*)malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
  if (!ids || !tmp || !scratch) {
    free(ids); free(tmp); free(scratch); free(frac); tree_shape_free(&t);
    return CDREF_ENOMEM;
  }
  for (int64_t c = 0; c < nc; ++c) ids[c] = (int32_t)c;
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int k = 0; k < dim; ++k) { lo[k] = box_lo[k]; hi[k] = box_hi[k]; }
  orb_split(dim, &t, frac, 0, lo, hi, nc, xmid, ids, nc, node_axis, node_cut, dom, scratch, tmp);
  memcpy(node_child, t.child, sizeof(int32_t) * 2 * (size_t)t.count);
  memcpy(node_leaf, t.leaf, sizeof(int32_t) * (size_t)t.count);
  if (node_leaves) memcpy(node_leaves, t.leaves, sizeof(int32_t) * (size_t)t.count);
  free(ids); free(tmp); free(scratch); free(frac); tree_shape_free(&t);
  return CDREF_OK;
}

void cdref_descend(int dim, int P, const int32_t* node_axis, const double* node_cut,
                   const int32_t* node_child, const int32_t* node_leaf,
                   int64_t nc, const double* xmid, int32_t* dom) {
  (void)dim; (void)P;
  for (int64_t c = 0; c < nc; ++c) {
    int node = 0;
    while (node_leaf[node] < 0) {
      int axis = node_axis[node];
      node = xmid[(int64_t)axis * nc + c] < node_cut[node] ? node_child[2 * node]
                                                            : node_child[2 * node + 1];
    }
    dom[c] = node_leaf[node];
  }
}

/* ------------------------------------------------------------------ */
/* update order inside a domain                                         */
/* ------------------------------------------------------------------ */

#define CDREF_MAX_COLORS 256

int cdref_order(int64_t n, int64_t nc, const int32_t* ci, const int32_t* cj,
                int P, const int32_t* dom, int32_t* color, int32_t* slot_contact,
                int64_t* dom_start) {
  return cdref_order_mixed(n, nc, ci, cj, P, dom, NULL, color, slot_contact, dom_start);
}

/* The same with the contacts flagged in `parallel` (NULL: none) updated in
 * parallel (Sec. 2.3): they take colour 0 and come first in their domain,
 * and the other contacts are coloured first-fit from colour 1. */
int cdref_order_mixed(int64_t n, int64_t nc, const int32_t* ci, const int32_t* cj,
                      int P, const int32_t* dom, const uint8_t* parallel, int32_t* color,
                      int32_t* slot_contact, int64_t* dom_start) {
  return cdref_order_bc(n, nc, ci, cj, P, dom, parallel, 0, color, slot_contact, dom_start);
}

int cdref_order_bc(int64_t n, int64_t nc, const int32_t* ci, const int32_t* cj, int P,
                   const int32_t* dom, const uint8_t* parallel, int mobile_mask, int32_t* color,
                   int32_t* slot_contact, int64_t* dom_start) {
  const int words = CDREF_MAX_COLORS / 64;
  const int first = parallel ? 1 : 0;   /* the first colour of a sequential contact */
  /* colour sets of the particles, then of the walls (a wall of finite mass
     is a body whose velocity the contacts change: its contacts conflict) */
  uint64_t* used =
      (uint64_t*)calloc((size_t)(n + CDREF_MAX_WALLS) * words, sizeof(uint64_t));
  int64_t* count = (int64_t*)calloc((size_t)P + 1, sizeof(int64_t));
  int64_t* members_start = (int64_t*)calloc((size_t)P + 1, sizeof(int64_t));
  int32_t* members = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
  if (!used || !count || !members_start || !members) {
    free(used); free(count); free(members_start); free(members);
    return CDREF_ENOMEM;
  }
  /* contacts of each domain in canonical order */
  for (int64_t c = 0; c < nc; ++c) members_start[dom[c] + 1] += 1;
  for (int d = 0; d < P; ++d) members_start[d + 1] += members_start[d];
  for (int d = 0; d <= P; ++d) count[d] = members_start[d];
  for (int64_t c = 0; c < nc; ++c) members[count[dom[c]]++] = (int32_t)c;

  int status = CDREF_OK;
  int64_t slot = 0;
  for (int d = 0; d < P; ++d) {
    dom_start[d] = slot;
    int maxcol = -1;
    /* greedy first-fit colouring in canonical order */
    for (int64_t s = members_start[d]; s < members_start[d + 1]; ++s) {
      int32_t c = members[s];
      int64_t a = ci[c], b = cj[c];
      if (parallel && parallel[c]) {
        color[c] = 0;
        if (maxcol < 0) maxcol = 0;
        continue;
      }
      const int b_body = b < n || ((mobile_mask >> (b - n)) & 1);
      int k = first;
      for (; k < CDREF_MAX_COLORS; ++k) {
        uint64_t bit = 1ull << (k % 64);
        int in_a = (used[a * words + k / 64] & bit) != 0;
        int in_b = b_body ? (used[b * words + k / 64] & bit) != 0 : 0;
        if (!in_a && !in_b) break;
      }
      if (k == CDREF_MAX_COLORS) { status = CDREF_ECAPACITY; k = CDREF_MAX_COLORS - 1; }
      color[c] = k;
      used[a * words + k / 64] |= 1ull << (k % 64);
      if (b_body) used[b * words + k / 64] |= 1ull << (k % 64);
      if (k > maxcol) maxcol = k;
    }
    /* order by (colour, canonical id) */
    for (int k = 0; k <= maxcol; ++k)
      for (int64_t s = members_start[d]; s < members_start[d + 1]; ++s)
        if (color[members[s]] == k) slot_contact[slot++] = members[s];
    /* clear the colour sets of this domain's particles */
    for (int64_t s = members_start[d]; s < members_start[d + 1]; ++s) {
      int32_t c = members[s];
      for (int w = 0; w < words; ++w) {
        used[(int64_t)ci[c] * words + w] = 0;
        used[(int64_t)cj[c] * words + w] = 0;
      }
    }
  }
  dom_start[P] = slot;
  free(used); free(count); free(members_start); free(members);
  return status;
}

/* ------------------------------------------------------------------ */
/* velocities from forces: Eq. (1) and its rotational analogue          */
/* ------------------------------------------------------------------ */

/* V = v + dt/m (F + sum of contact forces), W = w + dt/I (T + sum of torques),
 * the sums taken over the particle's contacts in ascending contact id. */
void cdref_velocities(int dim, int64_t n, double dt, const double* v, const double* w,
                      const double* m, const double* inertia, const double* r,
                      const double* f, const double* t, int64_t nc,
                      const int32_t* ci, const int32_t* cj, const double* normal,
                      const double* R, double* V, double* W) {
  int dr = dim == 2 ? 1 : 3;
  double* acc = (double*)malloc(sizeof(double) * (size_t)(dim * (n > 0 ? n : 1)));
  double* tacc = (double*)malloc(sizeof(double) * (size_t)(dr * (n > 0 ? n : 1)));
  for (int64_t i = 0; i < n; ++i) {
    for (int k = 0; k < dim; ++k) acc[k * n + i] = f[k * n + i];
    for (int k = 0; k < dr; ++k) tacc[k * n + i] = t[k * n + i];
  }
  for (int64_t c = 0; c < nc; ++c) {
    double nv[3], t1[3], t2[3];
    contact_frame(dim, normal, nc, c, nv, t1, t2);
    double rn = R[c], rt1 = R[nc + c], rt2 = dim == 3 ? R[2 * nc + c] : 0.0;
    double force[3], q[3];
    for (int k = 0; k < dim; ++k) {
      force[k] = rn * nv[k] + rt1 * t1[k];
      if (dim == 3) force[k] = force[k] + rt2 * t2[k];
    }
    /* n x R: the torque of the force about a lever along n, per unit lever */
    if (dim == 2) {
      q[0] = rt1;
    } else {
      for (int k = 0; k < 3; ++k) q[k] = rt1 * t2[k] - rt2 * t1[k];
    }
    int64_t a = ci[c], b = cj[c];
    /* body 1 receives -R at lever r_a n; body 2 receives R at lever -r_b n;
       both torques are -r (n x R) */
    for (int k = 0; k < dim; ++k) acc[k * n + a] = acc[k * n + a] - force[k];
    for (int k = 0; k < dr; ++k) tacc[k * n + a] = tacc[k * n + a] - r[a] * q[k];
    if (b < n) {
      for (int k = 0; k < dim; ++k) acc[k * n + b] = acc[k * n + b] + force[k];
      for (int k = 0; k < dr; ++k) tacc[k * n + b] = tacc[k * n + b] - r[b] * q[k];
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    double dtim = dt * (1.0 / m[i]);
    double dtii = dt * (1.0 / inertia[i]);
    for (int k = 0; k < dim; ++k) V[k * n + i] = v[k * n + i] + dtim * acc[k * n + i];
    for (int k = 0; k < dr; ++k) W[k * n + i] = w[k * n + i] + dtii * tacc[k * n + i];
  }
  free(acc); free(tacc);
}

/* ------------------------------------------------------------------ */
/* single-contact force law: Sec. 2.1, Eqs. (3)-(9), Fig. 2             */
/* ------------------------------------------------------------------ */

typedef struct {
  double gdt;        /* g_e / dt */
  double dwn, dwt;   /* dt w_n, dt w_t : M^-1 = w_n nn + w_t (1 - nn) */
  double kn, kt;     /* 1/(dt w_n), 1/(dt w_t) */
  double mu;
} contact_consts;

/* Given the velocities of both bodies (with every current force applied,
 * including this contact's own R), return the new force R' in the contact
 * frame.  Rold and Rnew: (R_n, R_t1[, R_t2]). */
static void local_force(int dim, const double n[3], const double t1[3], const double t2[3],
                        const contact_consts* k, double ra, double rb,
                        const double Va[3], const double Wa[3], const double Vb[3],
                        const double Wb[3], const double Rold[3], double Rnew[3]) {
  double dV[3] = {0, 0, 0};
  for (int q = 0; q < dim; ++q) dV[q] = Vb[q] - Va[q];
  double vn = 0.0, vt1 = 0.0, vt2 = 0.0;
  for (int q = 0; q < dim; ++q) vn = vn + dV[q] * n[q];
  if (dim == 2) {
    /* relative velocity of the contact points projected on t = z x n */
    double dvt = dV[0] * t1[0] + dV[1] * t1[1];
    double spin = ra * Wa[0] + rb * Wb[0];
    vt1 = dvt - spin;
  } else {
    double spin[3];
    for (int q = 0; q < 3; ++q) spin[q] = ra * Wa[q] + rb * Wb[q];
    double dvt1 = 0.0, dvt2 = 0.0, s2 = 0.0, s1 = 0.0;
    for (int q = 0; q < 3; ++q) {
      dvt1 = dvt1 + dV[q] * t1[q];
      dvt2 = dvt2 + dV[q] * t2[q];
      s2 = s2 + spin[q] * t2[q];
      s1 = s1 + spin[q] * t1[q];
    }
    vt1 = dvt1 - s2;
    vt2 = dvt2 + s1;
  }
  /* hypothetical relative velocity without this contact's force (R = 0) */
  double un = vn - k->dwn * Rold[0];
  double ut1 = vt1 - k->dwt * Rold[1];
  double ut2 = dim == 3 ? vt2 - k->dwt * Rold[2] : 0.0;
  /* predicted gap g + dt u_n (Eq. 3), divided by dt */
  double s = k->gdt + un;
  Rnew[0] = Rnew[1] = Rnew[2] = 0.0;
  if (s >= 0.0) return;                 /* contact stays open: R = 0 */
  /* sticking force from g(t+dt) = 0 and v_t(t+dt) = 0 (Eqs. 4-5) */
  double rn = -s * k->kn;
  double T1 = -ut1 * k->kt;
  double T2 = dim == 3 ? -ut2 * k->kt : 0.0;
  double lim = k->mu * rn;              /* Coulomb bound (Eq. 7) */
  Rnew[0] = rn;
  if (dim == 2) {
    if (fabs(T1) <= lim) Rnew[1] = T1;
    else Rnew[1] = T1 > 0.0 ? lim : -lim;   /* sliding (Eqs. 8-9) */
  } else {
    double tn = sqrt(T1 * T1 + T2 * T2);
    if (tn <= lim) {
      Rnew[1] = T1;
      Rnew[2] = T2;
    } else {
      /* sliding: R_t = -mu R_n v_t/|v_t|; with M diagonal in the contact
         frame the slip is parallel to the sticking force (Eqs. 8-9) */
      double fac = lim / tn;
      Rnew[1] = T1 * fac;
      Rnew[2] = T2 * fac;
    }
  }
}

/* ------------------------------------------------------------------ */
/* convergence tests (I) and (II), Sec. 2.1                             */
/* ------------------------------------------------------------------ */

int cdref_criterion(int dim, int64_t nc, const double* Rprev, const double* R, double ravg_prev,
                    double alpha, int criterion, int64_t* n_pass, double* max_d_fail,
                    double* r_avg, int* finite) {
  int64_t npass = 0;
  double maxd = 0.0, sum = 0.0;
  int any_fail = 0, ok = 1;
  for (int64_t c = 0; c < nc; ++c) {
    double d2 = 0.0, s2 = 0.0, q = 0.0;
    for (int k = 0; k < dim; ++k) {
      double a1 = R[k * nc + c], a0 = Rprev[k * nc + c];
      d2 = d2 + (a1 - a0) * (a1 - a0);
      s2 = s2 + (a1 + a0) * (a1 + a0);
      q = q + a1 * a1;
    }
    if (!isfinite(q)) ok = 0;
    sum = sum + sqrt(q);
    /* relative change (R^j - R^j-1)^2 / (R^j + R^j-1)^2 < alpha; 0/0 passes */
    if (d2 < alpha * s2 || d2 == 0.0) {
      ++npass;
    } else {
      if (!any_fail || d2 > maxd) maxd = d2;
      any_fail = 1;
    }
  }
  double ravg = nc > 0 ? sum / (double)nc : 0.0;
  int conv;
  if (criterion == 0) {
    /* (I): at least 90% pass the relative test and every other contact has
       (R^j - R^j-1)^2 < alpha R_avg^(j-1)^2 */
    conv = (10 * npass >= 9 * nc) && (!any_fail || maxd < alpha * (ravg_prev * ravg_prev));
  } else {
    /* (II): relative change of the average force */
    double dd = (ravg - ravg_prev) * (ravg - ravg_prev);
    double ss = (ravg + ravg_prev) * (ravg + ravg_prev);
    conv = dd < alpha * ss || dd == 0.0;
  }
  if (n_pass) *n_pass = npass;
  if (max_d_fail) *max_d_fail = maxd;
  if (r_avg) *r_avg = ravg;
  if (finite) *finite = ok;
  return conv;
}

/* ------------------------------------------------------------------ */
/* iterative solve with domain-wise sweeps (Sec. 2.1, Sec. 3.1)         */
/* ------------------------------------------------------------------ */

int cdref_solve(const cdref_params* p, int64_t n, const double* v, const double* w,
                const double* r, const double* m, const double* inertia,
                const double* f, const double* t, const double* wall_velocity,
                int64_t nc, const int32_t* ci, const int32_t* cj,
                const double* normal, const double* gap, const double* mu_c,
                int P, const int64_t* dom_start, const int32_t* slot_contact,
                double* R, cdref_info* info, double* history) {
  return cdref_solve_mixed(p, n, v, w, r, m, inertia, f, t, wall_velocity, nc, ci, cj, normal,
                           gap, mu_c, NULL, P, dom_start, slot_contact, R, info, history);
}

/* The solve; `parallel` (or NULL) flags contacts updated in parallel
 * (Sec. 2.3); with `step_key` non-NULL each domain instead updates its
 * contacts in the random order of cdref_random_slot_key, drawn afresh in
 * every sweep (Sec. 2.1). */
static int solve_impl(const cdref_params* p, int64_t n, const double* v, const double* w,
                      const double* r, const double* m, const double* inertia,
                      const double* f, const double* t, const double* wall_velocity,
                      int64_t nc, const int32_t* ci, const int32_t* cj,
                      const double* normal, const double* gap, const double* mu_c,
                      const uint8_t* parallel, const uint64_t* step_key, int P,
                      const int64_t* dom_start, const int32_t* slot_contact, double* R,
                      cdref_info* info, double* history, const cdref_mobile_walls* mw) {
  int dim = p->dim, dr = dim == 2 ? 1 : 3;
  /* walls whose normal motion follows from the forces (finite mass) */
  const int W = p->n_walls;
  double dtiM[CDREF_MAX_WALLS] = {0};
  int any_mobile = 0;
  if (mw && W > CDREF_MAX_WALLS) return CDREF_EINVAL;
  for (int q = 0; q < W && mw; ++q) {
    dtiM[q] = p->dt * mw->inv_mass[q];
    if (mw->inv_mass[q] != 0.0) any_mobile = 1;
  }
  int64_t nn = n > 0 ? n : 1, ncc = nc > 0 ? nc : 1;
  memset(info, 0, sizeof(*info));
  info->n_contacts = nc;
  if (nc == 0) return CDREF_OK;
  double dt = p->dt;
  contact_consts* cc = (contact_consts*)malloc(sizeof(contact_consts) * (size_t)ncc);
  double* Rprev = (double*)malloc(sizeof(double) * (size_t)(dim * ncc));
  double* Vg = (double*)malloc(sizeof(double) * (size_t)(dim * nn));
  double* Wg = (double*)malloc(sizeof(double) * (size_t)(dr * nn));
  /* one private velocity copy per thread (domains run on `threads` threads) */
  const int threads = g_threads;
  double* Vd = (double*)malloc(sizeof(double) * (size_t)(dim * nn) * (size_t)threads);
  double* Wd = (double*)malloc(sizeof(double) * (size_t)(dr * nn) * (size_t)threads);
  double* dtim = (double*)malloc(sizeof(double) * (size_t)nn);
  double* dtii = (double*)malloc(sizeof(double) * (size_t)nn);
  /* the walls' velocities: after the exchange (Uex) and each thread's
     private copy (Ut) that its domain's contacts update */
  double Uex[CDREF_MAX_WALLS * 3] = {0};
  double* Ut = (double*)malloc(sizeof(double) * (size_t)(CDREF_MAX_WALLS * 3) * (size_t)threads);
  rand_slot* ord =
      step_key ? (rand_slot*)malloc(sizeof(rand_slot) * (size_t)ncc * (size_t)threads) : NULL;
  if (!cc || !Rprev || !Vg || !Wg || !Vd || !Wd || !dtim || !dtii || !Ut ||
      (step_key && !ord)) {
    free(cc); free(Rprev); free(Vg); free(Wg); free(Vd); free(Wd); free(dtim); free(dtii);
    free(ord); free(Ut);
    return CDREF_ENOMEM;
  }
  for (int q = 0; q < W * dim; ++q) Uex[q] = wall_velocity ? wall_velocity[q] : 0.0;
  for (int64_t i = 0; i < n; ++i) {
    dtim[i] = dt * (1.0 / m[i]);
    dtii[i] = dt * (1.0 / inertia[i]);
  }
  /* per-contact constants of this step: the pair's inverse mass matrix in
     the contact frame (Eq. 5) and the (clamped) gap */
  for (int64_t c = 0; c < nc; ++c) {
    int64_t a = ci[c], b = cj[c];
    double wn = 1.0 / m[a] + (b < n ? 1.0 / m[b] : 0.0);
    double wt = wn + (r[a] * r[a]) * (1.0 / inertia[a]);
    wt = wt + (b < n ? (r[b] * r[b]) * (1.0 / inertia[b]) : 0.0);
    if (b >= n && mw && mw->inv_mass[b - n] != 0.0) {
      /* a wall of finite mass moves along its normal only: it adds 1/M to
         the normal term and nothing to the tangential one */
      wn = 1.0 / m[a] + mw->inv_mass[b - n];
      wt = 1.0 / m[a] + (r[a] * r[a]) * (1.0 / inertia[a]);
    }
    double ge = gap[c];
    if (p->overlap_mode == 0 && ge < 0.0) ge = 0.0;
    cc[c].gdt = ge / dt;
    cc[c].dwn = dt * wn;
    cc[c].dwt = dt * wt;
    cc[c].kn = 1.0 / cc[c].dwn;
    cc[c].kt = 1.0 / cc[c].dwt;
    cc[c].mu = mu_c ? mu_c[c] : p->mu;
  }
  int limit = p->fixed_iters > 0 ? p->fixed_iters : p->max_iter;
  double alpha = p->alpha;
  /* R_avg of the starting forces */
  double sum = 0.0;
  for (int64_t c = 0; c < nc; ++c) {
    double q = 0.0;
    for (int k = 0; k < dim; ++k) q = q + R[k * nc + c] * R[k * nc + c];
    sum = sum + sqrt(q);
  }
  double ravg_prev = sum / (double)nc;
  int status = CDREF_MAXITER;
  int j = 0;
  while (j < limit) {
    ++j;
    memcpy(Rprev, R, sizeof(double) * (size_t)(dim * nc));
    /* exchange: every particle's velocity from the forces of sweep j-1 */
    cdref_velocities(dim, n, dt, v, w, m, inertia, r, f, t, nc, ci, cj, normal, Rprev, Vg, Wg);
    /* ... and every wall's of finite mass */
    if (any_mobile) cdref_wall_velocities(dim, n, dt, W, wall_velocity, mw, nc, cj, Rprev, Uex);
    /* each domain sweeps its native contacts sequentially on a private copy
       of the velocities; other domains' contacts keep their sweep j-1 value.
       The domains of a sweep are independent: with threads > 1 they are
       spread over OpenMP threads, each with its own copy */
#ifdef _OPENMP
#pragma omp parallel for num_threads(threads) schedule(dynamic, 8) if (threads > 1)
#endif
    for (int d = 0; d < P; ++d) {
      int tid = 0;
#ifdef _OPENMP
      tid = omp_get_thread_num();
#endif
      double* Vt = Vd + (int64_t)tid * dim * nn;
      double* Wt = Wd + (int64_t)tid * dr * nn;
      /* the domain's own copy of the walls' velocities */
      double* Uw = Ut + (int64_t)tid * CDREF_MAX_WALLS * 3;
      for (int q = 0; q < W * dim; ++q) Uw[q] = Uex[q];
      rand_slot* od = ord ? ord + (int64_t)tid * ncc : NULL;
      const int64_t len = dom_start[d + 1] - dom_start[d];
      /* the domain starts from the exchanged velocities of its bodies */
      for (int64_t s = dom_start[d]; s < dom_start[d + 1]; ++s) {
        int64_t c = slot_contact[s];
        int64_t ends[2] = {ci[c], cj[c]};
        for (int e = 0; e < 2; ++e) {
          int64_t q = ends[e];
          if (q >= n) continue;
          for (int k = 0; k < dim; ++k) Vt[k * n + q] = Vg[k * n + q];
          for (int k = 0; k < dr; ++k) Wt[k * n + q] = Wg[k * n + q];
        }
      }
      if (step_key) {
        /* this sweep's random order of the domain's contacts */
        for (int64_t q = 0; q < len; ++q) {
          od[q].slot = dom_start[d] + q;
          od[q].key = cdref_random_slot_key(*step_key, j, od[q].slot);
        }
        qsort(od, (size_t)len, sizeof(rand_slot), rand_slot_cmp);
      }
      /* pass 0: the domain's parallel contacts (Sec. 2.3) from the velocities
         of the exchange, their changes not applied in this sweep (the other
         contacts see their old forces); pass 1: the sequential update, in
         slot order or in the sweep's random order */
      for (int pass = parallel ? 0 : 1; pass < 2; ++pass)
      for (int64_t q = 0; q < len; ++q) {
        int64_t s = step_key ? od[q].slot : dom_start[d] + q;
        int64_t c = slot_contact[s];
        const int par = parallel ? parallel[c] != 0 : 0;
        if (par != (pass == 0)) continue;
        int64_t a = ci[c], b = cj[c];
        double nv[3], t1[3], t2[3];
        contact_frame(dim, normal, nc, c, nv, t1, t2);
        double Va[3] = {0, 0, 0}, Wa[3] = {0, 0, 0}, Vb[3] = {0, 0, 0}, Wb[3] = {0, 0, 0};
        for (int k = 0; k < dim; ++k) Va[k] = Vt[k * n + a];
        for (int k = 0; k < dr; ++k) Wa[k] = Wt[k * n + a];
        double rb = 0.0;
        if (b < n) {
          for (int k = 0; k < dim; ++k) Vb[k] = Vt[k * n + b];
          for (int k = 0; k < dr; ++k) Wb[k] = Wt[k * n + b];
          rb = r[b];
        } else {
          for (int k = 0; k < dim; ++k) Vb[k] = Uw[(b - n) * dim + k];
        }
        double Rold[3] = {0, 0, 0}, Rnew[3];
        for (int k = 0; k < dim; ++k) Rold[k] = R[k * nc + c];
        local_force(dim, nv, t1, t2, &cc[c], r[a], rb, Va, Wa, Vb, Wb, Rold, Rnew);
        double dRn = Rnew[0] - Rold[0], dR1 = Rnew[1] - Rold[1];
        double dR2 = dim == 3 ? Rnew[2] - Rold[2] : 0.0;
        for (int k = 0; k < dim; ++k) R[k * nc + c] = Rnew[k];
        if (par) continue;
        /* apply the change to both bodies' private velocities */
        double dF[3], dq[3];
        for (int k = 0; k < dim; ++k) {
          dF[k] = dRn * nv[k] + dR1 * t1[k];
          if (dim == 3) dF[k] = dF[k] + dR2 * t2[k];
        }
        if (dim == 2) dq[0] = dR1;
        else for (int k = 0; k < 3; ++k) dq[k] = dR1 * t2[k] - dR2 * t1[k];
        for (int k = 0; k < dim; ++k) Vt[k * n + a] = Vt[k * n + a] - dtim[a] * dF[k];
        for (int k = 0; k < dr; ++k) Wt[k * n + a] = Wt[k * n + a] - dtii[a] * (r[a] * dq[k]);
        if (b < n) {
          for (int k = 0; k < dim; ++k) Vt[k * n + b] = Vt[k * n + b] + dtim[b] * dF[k];
          for (int k = 0; k < dr; ++k) Wt[k * n + b] = Wt[k * n + b] - dtii[b] * (r[b] * dq[k]);
        } else if (dtiM[b - n] != 0.0) {
          /* a wall of finite mass takes the normal part of the change */
          for (int k = 0; k < dim; ++k)
            Uw[(b - n) * dim + k] = Uw[(b - n) * dim + k] + dtiM[b - n] * (dRn * nv[k]);
        }
      }
    }
    /* convergence tests (Sec. 2.1) */
    int64_t npass = 0;
    double maxd = 0.0, ravg = 0.0;
    int finite = 1;
    int conv = cdref_criterion(dim, nc, Rprev, R, ravg_prev, alpha, p->criterion, &npass, &maxd,
                               &ravg, &finite);
    if (history) {
      history[0 * (int64_t)limit + (j - 1)] = (double)npass;
      history[1 * (int64_t)limit + (j - 1)] = maxd;
      history[2 * (int64_t)limit + (j - 1)] = ravg;
      history[3 * (int64_t)limit + (j - 1)] = (double)conv;
    }
    info->n_pass = npass;
    info->max_d_fail = maxd;
    info->r_avg = ravg;
    info->r_avg_prev = ravg_prev;
    info->iterations = j;
    ravg_prev = ravg;
    if (!finite) { status = CDREF_ENONFINITE; break; }
    if (p->fixed_iters > 0) {
      if (j == p->fixed_iters) { status = CDREF_OK; break; }
      continue;
    }
    if (conv) { status = CDREF_OK; break; }
  }
  info->status = status;
  free(cc); free(Rprev); free(Vg); free(Wg); free(Vd); free(Wd); free(dtim); free(dtii);
  free(ord); free(Ut);
  return status;
}

int cdref_solve_mixed(const cdref_params* p, int64_t n, const double* v, const double* w,
                      const double* r, const double* m, const double* inertia,
                      const double* f, const double* t, const double* wall_velocity,
                      int64_t nc, const int32_t* ci, const int32_t* cj,
                      const double* normal, const double* gap, const double* mu_c,
                      const uint8_t* parallel, int P, const int64_t* dom_start,
                      const int32_t* slot_contact, double* R, cdref_info* info,
                      double* history) {
  return solve_impl(p, n, v, w, r, m, inertia, f, t, wall_velocity, nc, ci, cj, normal, gap,
                    mu_c, parallel, NULL, P, dom_start, slot_contact, R, info, history, NULL);
}

int cdref_solve_random(const cdref_params* p, int64_t n, const double* v, const double* w,
                       const double* r, const double* m, const double* inertia,
                       const double* f, const double* t, const double* wall_velocity,
                       int64_t nc, const int32_t* ci, const int32_t* cj,
                       const double* normal, const double* gap, const double* mu_c, int P,
                       const int64_t* dom_start, const int32_t* slot_contact, uint64_t seed,
                       int64_t step, double* R, cdref_info* info, double* history) {
  const uint64_t key = cdref_random_step_key(seed, step);
  return solve_impl(p, n, v, w, r, m, inertia, f, t, wall_velocity, nc, ci, cj, normal, gap,
                    mu_c, NULL, &key, P, dom_start, slot_contact, R, info, history, NULL);
}

int cdref_solve_bc(const cdref_params* p, int64_t n, const double* v, const double* w,
                   const double* r, const double* m, const double* inertia,
                   const double* f, const double* t, const double* wall_velocity,
                   int64_t nc, const int32_t* ci, const int32_t* cj,
                   const double* normal, const double* gap, const double* mu_c,
                   const uint8_t* parallel, int P, const int64_t* dom_start,
                   const int32_t* slot_contact, const cdref_mobile_walls* mw, double* R,
                   cdref_info* info, double* history) {
  return solve_impl(p, n, v, w, r, m, inertia, f, t, wall_velocity, nc, ci, cj, normal, gap,
                    mu_c, parallel, NULL, P, dom_start, slot_contact, R, info, history, mw);
}

/* Velocities of the walls after forces R (Eq. 1 for a wall body): a wall of
 * finite mass M under the external force F along its normal nu has normal
 * velocity u_n + dt/M (F - sum of R_n over its contacts, ascending contact
 * id; the force on the wall along nu is -R_n since n = -nu), its tangential
 * velocity stays prescribed; other walls keep their velocity. */
void cdref_wall_velocities(int dim, int64_t n, double dt, int W, const double* wall_velocity,
                           const cdref_mobile_walls* mw, int64_t nc, const int32_t* cj,
                           const double* R, double* U) {
  for (int q = 0; q < W; ++q) {
    const double* u = wall_velocity + q * dim;
    if (!mw || mw->inv_mass[q] == 0.0) {
      for (int k = 0; k < dim; ++k) U[q * dim + k] = u[k];
      continue;
    }
    const double* nu = mw->normal + q * dim;
    double un = 0.0;
    for (int k = 0; k < dim; ++k) un = un + nu[k] * u[k];
    double acc = mw->force[q];
    for (int64_t c = 0; c < nc; ++c)
      if (cj[c] == n + q) acc = acc - R[c];
    const double un1 = un + (dt * mw->inv_mass[q]) * acc;
    for (int k = 0; k < dim; ++k) U[q * dim + k] = (u[k] - un * nu[k]) + un1 * nu[k];
  }
}

/* ------------------------------------------------------------------ */
/* whole time steps (Fig. 3 and Fig. 7)                                 */
/* ------------------------------------------------------------------ */

struct cdref_sim {
  cdref_params p;
  int64_t n;
  int dr;
  double *x, *v, *w, *r, *m, *I, *f, *t;
  double *wn, *wo, *wu;
  double lo[3], hi[3];
  int64_t step;
  /* tree */
  int32_t *axis, *child, *leaf;
  double* cut;
  int have_tree;
  double* capacity;   /* per-domain capacities for the tree rebuilds, or NULL */
  double mixed_p;     /* share of contacts updated in parallel (< 0: none) */
  uint64_t mixed_seed;
  int rand_on;        /* random sequential order (Sec. 2.1) */
  uint64_t rand_seed;
  /* boundary conditions of the benchmark setups (Sec. 4.1, Sec. 4.4) */
  double period[3];   /* > 0: periodic axis of this length */
  int has_period;
  double wall_inv_mass[CDREF_MAX_WALLS], wall_force[CDREF_MAX_WALLS];
  int has_mobile;
  /* contacts of the last step */
  int64_t nc, cap;
  int32_t *ci, *cj, *dom, *color, *slot;
  double *normal, *gap, *xmid, *R;
};

static double* dup_array(const double* a, int64_t count) {
  double* b = (double*)malloc(sizeof(double) * (size_t)(count > 0 ? count : 1));
  if (b && count > 0) memcpy(b, a, sizeof(double) * (size_t)count);
  return b;
}

cdref_sim* cdref_sim_create(const cdref_params* p, int64_t n, const double* x,
                            const double* v, const double* w, const double* r,
                            const double* m, const double* inertia, const double* f,
                            const double* t, const double* wall_normal,
                            const double* wall_offset, const double* wall_velocity,
                            const double* box_lo, const double* box_hi) {
  if (p->dim != 2 && p->dim != 3) return NULL;
  if (p->n_domains < 1 || n < 1) return NULL;
  cdref_sim* s = (cdref_sim*)calloc(1, sizeof(cdref_sim));
  if (s) s->mixed_p = -1.0;
  if (!s) return NULL;
  s->p = *p;
  if (s->p.repartition_every < 1) s->p.repartition_every = 1;
  s->n = n;
  int dim = p->dim;
  s->dr = dim == 2 ? 1 : 3;
  s->x = dup_array(x, dim * n);
  s->v = dup_array(v, dim * n);
  s->w = dup_array(w, s->dr * n);
  s->r = dup_array(r, n);
  s->m = dup_array(m, n);
  s->I = dup_array(inertia, n);
  s->f = dup_array(f, dim * n);
  s->t = dup_array(t, s->dr * n);
  s->wn = dup_array(wall_normal, (int64_t)p->n_walls * dim);
  s->wo = dup_array(wall_offset, p->n_walls);
  s->wu = dup_array(wall_velocity, (int64_t)p->n_walls * dim);
  for (int k = 0; k < 3; ++k) { s->lo[k] = k < dim ? box_lo[k] : 0.0; s->hi[k] = k < dim ? box_hi[k] : 0.0; }
  int nodes = 2 * p->n_domains - 1;
  s->axis = (int32_t*)calloc((size_t)nodes, sizeof(int32_t));
  s->child = (int32_t*)calloc(2 * (size_t)nodes, sizeof(int32_t));
  s->leaf = (int32_t*)calloc((size_t)nodes, sizeof(int32_t));
  s->cut = (double*)calloc((size_t)nodes, sizeof(double));
  return s;
}

void cdref_sim_destroy(cdref_sim* s) {
  if (!s) return;
  free(s->x); free(s->v); free(s->w); free(s->r); free(s->m); free(s->I); free(s->f);
  free(s->t); free(s->wn); free(s->wo); free(s->wu);
  free(s->axis); free(s->child); free(s->leaf); free(s->cut);
  free(s->ci); free(s->cj); free(s->dom); free(s->color); free(s->slot);
  free(s->normal); free(s->gap); free(s->xmid); free(s->R);
  free(s->capacity);
  free(s);
}

int cdref_sim_set_bc(cdref_sim* s, int periodic_mask, const double* wall_inv_mass,
                     const double* wall_force) {
  const int dim = s->p.dim, W = s->p.n_walls;
  if (W > CDREF_MAX_WALLS) return CDREF_EINVAL;
  s->has_period = 0;
  for (int k = 0; k < 3; ++k) {
    s->period[k] = 0.0;
    if (k < dim && (periodic_mask >> k) & 1) {
      s->period[k] = s->hi[k] - s->lo[k];
      s->has_period = 1;
      /* no wall may bound a periodic axis */
      for (int q = 0; q < W; ++q)
        if (s->wn[q * dim + k] != 0.0) return CDREF_EINVAL;
    }
  }
  s->has_mobile = 0;
  for (int q = 0; q < CDREF_MAX_WALLS; ++q) {
    s->wall_inv_mass[q] = (wall_inv_mass && q < W) ? wall_inv_mass[q] : 0.0;
    s->wall_force[q] = (wall_force && q < W) ? wall_force[q] : 0.0;
    if (s->wall_inv_mass[q] < 0.0) return CDREF_EINVAL;
    if (s->wall_inv_mass[q] != 0.0) s->has_mobile = 1;
  }
  return CDREF_OK;
}

void cdref_sim_wall_velocities(const cdref_sim* s, double* U) {
  for (int q = 0; q < s->p.n_walls * s->p.dim; ++q) U[q] = s->wu[q];
}

void cdref_sim_set_mixed(cdref_sim* s, double p, uint64_t seed) {
  s->mixed_p = p;
  s->mixed_seed = seed;
}

int cdref_sim_set_random(cdref_sim* s, int on, uint64_t seed) {
  s->rand_on = on != 0;
  s->rand_seed = seed;
  return CDREF_OK;
}

int cdref_sim_set_capacity(cdref_sim* s, const double* capacity) {
  int P = s->p.n_domains;
  if (!capacity) {
    free(s->capacity);
    s->capacity = NULL;
    return CDREF_OK;
  }
  if (!s->capacity) s->capacity = (double*)malloc(sizeof(double) * (size_t)P);
  if (!s->capacity) return CDREF_ENOMEM;
  memcpy(s->capacity, capacity, sizeof(double) * (size_t)P);
  return CDREF_OK;
}

/* contact arrays for at least `need` contacts: a quarter more than needed
 * when they grow, exactly `keep` (the previous capacity) otherwise */
static int ensure_capacity(cdref_sim* s, int64_t need, int64_t keep) {
  if (need <= s->cap) return CDREF_OK;
  int64_t cap = need > keep ? need + need / 4 + 64 : keep;
  int dim = s->p.dim;
  free(s->ci); free(s->cj); free(s->dom); free(s->color); free(s->slot);
  free(s->normal); free(s->gap); free(s->xmid);
  s->ci = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
  s->cj = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
  s->dom = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
  s->color = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
  s->slot = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
  s->normal = (double*)malloc(sizeof(double) * (size_t)(dim * cap));
  s->gap = (double*)malloc(sizeof(double) * (size_t)cap);
  s->xmid = (double*)malloc(sizeof(double) * (size_t)(dim * cap));
  if (!s->ci || !s->cj || !s->dom || !s->color || !s->slot || !s->normal || !s->gap || !s->xmid)
    return CDREF_ENOMEM;
  s->cap = cap;
  return CDREF_OK;
}

int cdref_sim_step(cdref_sim* s, cdref_info* info) {
  cdref_params* p = &s->p;
  int dim = p->dim, dr = s->dr;
  int64_t n = s->n;
  memset(info, 0, sizeof(*info));
  for (int64_t i = 0; i < n; ++i) {
    if (!(s->r[i] > 0.0) || !(s->m[i] > 0.0) || !(s->I[i] > 0.0)) return CDREF_EINVAL;
    for (int k = 0; k < dim; ++k)
      if (!isfinite(s->x[k * n + i]) || !isfinite(s->v[k * n + i])) return CDREF_ENONFINITE;
  }
  /* boundary width: two particles can touch within dt if their gap is below
     2 vmax dt (Sec. 3.1) */
  double vmax = 0.0, rmax = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double q = 0.0;
    for (int k = 0; k < dim; ++k) q = q + s->v[k * n + i] * s->v[k * n + i];
    double sp = sqrt(q);
    if (sp > vmax) vmax = sp;
    if (s->r[i] > rmax) rmax = s->r[i];
  }
  for (int wi = 0; wi < p->n_walls; ++wi) {
    double q = 0.0;
    for (int k = 0; k < dim; ++k) q = q + s->wu[wi * dim + k] * s->wu[wi * dim + k];
    double sp = sqrt(q);
    if (sp > vmax) vmax = sp;
  }
  double skin = p->skin >= 0.0 ? p->skin : 2.0 * vmax * p->dt;
  info->skin = skin;
  if (skin > 0.2 * rmax) return CDREF_EINVAL;   /* displacement bound 0.1 r_max */

  /* previous contacts for the warm start */
  int64_t old_nc = s->nc;
  int32_t* old_ci = s->ci;
  int32_t* old_cj = s->cj;
  double* old_R = s->R;
  s->ci = NULL; s->cj = NULL; s->R = NULL;
  /* detection */
  int64_t nc = 0;
  int st;
  {
    int64_t guess = s->cap > 0 ? s->cap : 4 * n + 64;
    int32_t* ci = (int32_t*)malloc(sizeof(int32_t) * (size_t)guess);
    int32_t* cj = (int32_t*)malloc(sizeof(int32_t) * (size_t)guess);
    const double* period = s->has_period ? s->period : NULL;
    st = cdref_detect_bc(dim, n, s->x, s->r, p->n_walls, s->wn, s->wo, skin, 1, s->lo, s->hi,
                         period, guess, ci, cj, &nc);
    if (st == CDREF_ECAPACITY) {
      free(ci); free(cj);
      ci = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
      cj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
      st = cdref_detect_bc(dim, n, s->x, s->r, p->n_walls, s->wn, s->wo, skin, 1, s->lo, s->hi,
                           period, nc, ci, cj, &nc);
    }
    if (st != CDREF_OK) { free(ci); free(cj); free(old_ci); free(old_cj); free(old_R); return st; }
    int64_t keep_cap = s->cap;
    free(s->dom); free(s->color); free(s->slot); free(s->normal); free(s->gap); free(s->xmid);
    s->dom = NULL; s->color = NULL; s->slot = NULL; s->normal = NULL; s->gap = NULL; s->xmid = NULL;
    s->cap = 0;
    st = ensure_capacity(s, nc, keep_cap);
    if (st != CDREF_OK) { free(ci); free(cj); return st; }
    memcpy(s->ci, ci, sizeof(int32_t) * (size_t)nc);
    memcpy(s->cj, cj, sizeof(int32_t) * (size_t)nc);
    free(ci); free(cj);
  }
  s->nc = nc;
  info->n_contacts = nc;
  cdref_geometry_bc(dim, n, s->x, s->r, p->n_walls, s->wn, s->wo,
                    s->has_period ? s->period : NULL, s->lo, nc, s->ci, s->cj, s->normal,
                    s->gap, s->xmid);
  /* warm start: forces of the same pair in the previous step, else zero */
  s->R = (double*)calloc((size_t)(dim * (nc > 0 ? nc : 1)), sizeof(double));
  if (p->warm_start && old_R) {
    for (int64_t c = 0; c < nc; ++c) {
      int64_t lo = 0, hi = old_nc;
      while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (old_ci[mid] < s->ci[c] || (old_ci[mid] == s->ci[c] && old_cj[mid] < s->cj[c]))
          lo = mid + 1;
        else
          hi = mid;
      }
      if (lo < old_nc && old_ci[lo] == s->ci[c] && old_cj[lo] == s->cj[c])
        for (int k = 0; k < dim; ++k) s->R[k * nc + c] = old_R[k * old_nc + lo];
    }
  }
  free(old_ci); free(old_cj); free(old_R);
  /* partition: rebuild the tree every repartition_every steps, otherwise
     descend the existing one (Sec. 3.2) */
  int P = p->n_domains;
  if (!s->have_tree || s->step % p->repartition_every == 0) {
    st = cdref_orb_capacity(dim, P, s->lo, s->hi, nc, s->xmid, s->capacity, s->axis, s->cut,
                            s->child, s->leaf, NULL, s->dom);
    if (st != CDREF_OK) return st;
    s->have_tree = 1;
  } else {
    cdref_descend(dim, P, s->axis, s->cut, s->child, s->leaf, nc, s->xmid, s->dom);
  }
  int64_t* dom_start = (int64_t*)malloc(sizeof(int64_t) * ((size_t)P + 1));
  /* mixed update (Sec. 2.3): the contacts whose pair draw falls below p */
  uint8_t* par = NULL;
  if (s->mixed_p >= 0.0) {
    par = (uint8_t*)malloc((size_t)(nc > 0 ? nc : 1));
    if (!par) { free(dom_start); return CDREF_ENOMEM; }
    cdref_parallel_flags(nc, s->ci, s->cj, s->mixed_p, s->mixed_seed, par);
  }
  int mobile_mask = 0;
  for (int q = 0; q < p->n_walls && s->has_mobile; ++q)
    if (s->wall_inv_mass[q] != 0.0) mobile_mask |= 1 << q;
  st = cdref_order_bc(n, nc, s->ci, s->cj, P, s->dom, par, mobile_mask, s->color, s->slot,
                      dom_start);
  if (st != CDREF_OK) { free(dom_start); free(par); return st; }
  cdref_mobile_walls mw = {s->wn, s->wall_inv_mass, s->wall_force};
  const cdref_mobile_walls* mwp = s->has_mobile ? &mw : NULL;
  if (s->rand_on && par) {
    st = CDREF_EINVAL;   /* the random order has no parallel contacts */
  } else if (s->rand_on) {
    const uint64_t key = cdref_random_step_key(s->rand_seed, s->step);
    st = solve_impl(p, n, s->v, s->w, s->r, s->m, s->I, s->f, s->t, s->wu, nc, s->ci, s->cj,
                    s->normal, s->gap, NULL, NULL, &key, P, dom_start, s->slot, s->R, info,
                    NULL, mwp);
  } else {
    st = solve_impl(p, n, s->v, s->w, s->r, s->m, s->I, s->f, s->t, s->wu, nc, s->ci, s->cj,
                    s->normal, s->gap, NULL, par, NULL, P, dom_start, s->slot, s->R, info, NULL,
                    mwp);
  }
  free(par);
  info->skin = skin;
  info->n_contacts = nc;
  free(dom_start);
  if (st < 0) return st;
  /* time stepping: Eqs. (1)-(2) with the final forces */
  double* V = (double*)malloc(sizeof(double) * (size_t)(dim * n));
  double* W = (double*)malloc(sizeof(double) * (size_t)(dr * n));
  cdref_velocities(dim, n, p->dt, s->v, s->w, s->m, s->I, s->r, s->f, s->t, nc, s->ci, s->cj,
                   s->normal, s->R, V, W);
  for (int64_t i = 0; i < n; ++i) {
    for (int k = 0; k < dim; ++k) {
      s->v[k * n + i] = V[k * n + i];
      s->x[k * n + i] = s->x[k * n + i] + V[k * n + i] * p->dt;
      /* a particle leaving a periodic box enters it on the other side */
      if (s->has_period && s->period[k] > 0.0)
        s->x[k * n + i] = wrap_into(s->x[k * n + i], s->lo[k], s->period[k]);
    }
    for (int k = 0; k < dr; ++k) s->w[k * n + i] = W[k * n + i];
  }
  free(V); free(W);
  /* walls of finite mass: their velocity from the final forces (Eq. 1) */
  if (s->has_mobile) {
    double U[CDREF_MAX_WALLS * 3];
    cdref_wall_velocities(dim, n, p->dt, p->n_walls, s->wu, mwp, nc, s->cj, s->R, U);
    for (int q = 0; q < p->n_walls * dim; ++q) s->wu[q] = U[q];
  }
  /* walls translate; a box face follows the wall lying on it */
  for (int wi = 0; wi < p->n_walls; ++wi) {
    double un = 0.0;
    for (int k = 0; k < dim; ++k) un = un + s->wn[wi * dim + k] * s->wu[wi * dim + k];
    s->wo[wi] = s->wo[wi] + p->dt * un;
    for (int k = 0; k < dim; ++k) {
      int unit = 1;
      for (int q = 0; q < dim; ++q)
        if (q != k && s->wn[wi * dim + q] != 0.0) unit = 0;
      if (!unit) continue;
      if (s->wn[wi * dim + k] == 1.0) s->lo[k] = s->wo[wi];
      if (s->wn[wi * dim + k] == -1.0) s->hi[k] = -s->wo[wi];
    }
  }
  s->step += 1;
  return st;
}

void cdref_sim_state(const cdref_sim* s, double* x, double* v, double* w, double* wall_offset) {
  int dim = s->p.dim;
  if (x) memcpy(x, s->x, sizeof(double) * (size_t)(dim * s->n));
  if (v) memcpy(v, s->v, sizeof(double) * (size_t)(dim * s->n));
  if (w) memcpy(w, s->w, sizeof(double) * (size_t)(s->dr * s->n));
  if (wall_offset && s->p.n_walls > 0)
    memcpy(wall_offset, s->wo, sizeof(double) * (size_t)s->p.n_walls);
}

int64_t cdref_sim_contacts(const cdref_sim* s, int64_t cap, int32_t* ci, int32_t* cj,
                           double* normal, double* gap, double* R, int32_t* dom,
                           int32_t* color, int32_t* slot_contact) {
  int64_t nc = s->nc;
  if (cap < nc) return nc;
  int dim = s->p.dim;
  if (ci) memcpy(ci, s->ci, sizeof(int32_t) * (size_t)nc);
  if (cj) memcpy(cj, s->cj, sizeof(int32_t) * (size_t)nc);
  if (normal) memcpy(normal, s->normal, sizeof(double) * (size_t)(dim * nc));
  if (gap) memcpy(gap, s->gap, sizeof(double) * (size_t)nc);
  if (R) memcpy(R, s->R, sizeof(double) * (size_t)(dim * nc));
  if (dom) memcpy(dom, s->dom, sizeof(int32_t) * (size_t)nc);
  if (color) memcpy(color, s->color, sizeof(int32_t) * (size_t)nc);
  if (slot_contact) memcpy(slot_contact, s->slot, sizeof(int32_t) * (size_t)nc);
  return nc;
}

void cdref_sim_box(const cdref_sim* s, double* lo, double* hi) {
  for (int k = 0; k < s->p.dim; ++k) {
    lo[k] = s->lo[k];
    hi[k] = s->hi[k];
  }
}

void cdref_sim_tree(const cdref_sim* s, int32_t* node_axis, double* node_cut,
                    int32_t* node_child, int32_t* node_leaf) {
  int nodes = 2 * s->p.n_domains - 1;
  memcpy(node_axis, s->axis, sizeof(int32_t) * (size_t)nodes);
  memcpy(node_cut, s->cut, sizeof(double) * (size_t)nodes);
  memcpy(node_child, s->child, sizeof(int32_t) * 2 * (size_t)nodes);
  memcpy(node_leaf, s->leaf, sizeof(int32_t) * (size_t)nodes);
}
