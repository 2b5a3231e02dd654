/*
 * pcc_oracle.c -- plain CPU reference of the cluster-preserving correction.
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the GPU library, with which it shares
 * no code.  Single-threaded, IEEE double precision, no contraction
 * (build with -ffp-contract=off).  Each function names the passage of the
 * paper it follows; readings of open points are stated in place.
 */
#include "pcc_oracle.h"

#include <dlfcn.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* small helpers                                                            */
/* ------------------------------------------------------------------------ */
void orc_free(void *ptr) { free(ptr); }

static void *xmalloc(size_t bytes) { return malloc(bytes ? bytes : 1); }

static void *xcalloc(size_t count, size_t size) {
  return calloc(count ? count : 1, size ? size : 1);
}

void orc_params_default(orc_params *p) {
  memset(p, 0, sizeof(*p));
  p->mode = ORC_HF;
  p->m_bits = 16;            /* Sec. 3.3: m = 16 is the default bit depth */
  p->optimizer = ORC_ADAM;   /* Sec. 4.2: Adam in every experiment */
  p->margin_policy = ORC_MARGIN_SAFE;
  p->lr = 1e-3;
  p->beta1 = 0.9;
  p->beta2 = 0.999;
  p->adam_eps = 1e-8;
  p->max_iters = 0;
  p->loss_tol = 0.0;
}

/* Spacing of float32 numbers at magnitude a > 0. */
static double ulp_f32(double a) {
  int e;
  frexp(a, &e); /* a = f * 2^e with f in [0.5, 1) */
  double s = ldexp(1.0, e - 24);
  double tiny = ldexp(1.0, -149);
  return s < tiny ? tiny : s;
}

/*
 * Constants of Alg. 1 and Sec. 3.3.
 *   r_s = b - 2 sqrt(3) xi  (safe links, Sec. 3.2)
 *   r_v = b + 2 sqrt(3) xi  (vulnerable pairs, Sec. 3.1)
 *   eps_q = 2 xi / (2^m - 1): the largest error of a quantised edit when the
 *   edit range [-2 xi, 2 xi] is split into 2^m - 1 steps of 4 xi / (2^m - 1).
 * PAPER margins: xi' = xi (1 - 2^-m) and a distance margin 2 sqrt(3) eps_q.
 * SAFE margins (default reading): the decoded coordinate also carries the
 * float32 rounding of x_hat + edit, at most half a float32 ulp u of the
 * largest magnitude, so the per-coordinate decode error is bounded by
 * delta_q = (eps_q + u)(1 + 2^-16); then xi' = xi - delta_q keeps every
 * decoded coordinate within xi, and the distance margin 2 sqrt(3) delta_q
 * keeps every satisfied active pair on the right side of b after decoding.
 */
void orc_constants(const orc_params *p, double maxabs, orc_consts *c) {
  double two_sqrt3 = 2.0 * sqrt(3.0);
  double levels = ldexp(1.0, p->m_bits) - 1.0;
  memset(c, 0, sizeof(*c));
  c->rs = p->b - two_sqrt3 * p->xi;
  c->rv = p->b + two_sqrt3 * p->xi;
  c->b2 = p->b * p->b;
  c->rs2 = c->rs > 0.0 ? c->rs * c->rs : -1.0;
  c->rv2 = c->rv * c->rv;
  c->eps_q = 2.0 * p->xi / levels;
  c->qstep = 4.0 * p->xi / levels;
  if (p->margin_policy == ORC_MARGIN_PAPER) {
    c->delta_q = c->eps_q;
    c->xi_p = p->xi * (1.0 - ldexp(1.0, -p->m_bits));
    c->delta_t = two_sqrt3 * c->eps_q;
  } else {
    double u = 0.5 * ulp_f32(maxabs + 2.0 * p->xi);
    c->delta_q = (c->eps_q + u) * (1.0 + ldexp(1.0, -16));
    c->xi_p = p->xi - c->delta_q;
    c->delta_t = two_sqrt3 * c->delta_q;
  }
  c->bm = p->b - c->delta_t;
  c->bp = p->b + c->delta_t;
  c->bm2 = c->bm * c->bm;
  c->bp2 = c->bp * c->bp;
}

double orc_max_abs(int64_t n, const float *const xyz[3], const float *const rec[3]) {
  double m = 0.0;
  for (int a = 0; a < 3; a++)
    for (int64_t k = 0; k < n; k++) {
      double u = fabs((double)xyz[a][k]), v = fabs((double)rec[a][k]);
      if (u > m) m = u;
      if (v > m) m = v;
    }
  return m;
}

/*
 * Difference along one axis.  The paper's domain is open (Sec. 3); for a
 * periodic axis of side L the minimum image is taken: the difference of two
 * coordinates is moved by one period when it exceeds half a period.
 */
static double axis_diff(double d, double L) {
  if (L > 0.0) {
    if (d > 0.5 * L)
      d -= L;
    else if (d < -0.5 * L)
      d += L;
  }
  return d;
}

/* Squared Euclidean distance in double precision, summed x, y, then z. */
double orc_dist2(const float *const xyz[3], int64_t i, int64_t j, const double box[3]) {
  double dx = axis_diff((double)xyz[0][i] - (double)xyz[0][j], box[0]);
  double dy = axis_diff((double)xyz[1][i] - (double)xyz[1][j], box[1]);
  double dz = axis_diff((double)xyz[2][i] - (double)xyz[2][j], box[2]);
  return (dx * dx + dy * dy) + dz * dz;
}

/*
 * Pair classes, Sec. 3.1 and 3.2, as comparisons of the squared distance
 * with squared thresholds:
 *   safe link                 d <= b - 2 sqrt(3) xi   (only if that is > 0)
 *   potentially broken (pb)   b - 2 sqrt(3) xi < d <= b
 *   potentially created (pc)  b < d <= b + 2 sqrt(3) xi
 */
int orc_classify(double d2, const orc_consts *c) {
  if (c->rs > 0.0 && d2 <= c->rs2) return ORC_SAFE;
  if (d2 <= c->b2) return ORC_PB;
  if (d2 <= c->rv2) return ORC_PC;
  return ORC_NONE;
}

/* ------------------------------------------------------------------------ */
/* fixed-radius pair search by cell linking (Sec. 2.4.1, Sec. 3.3)          */
/* ------------------------------------------------------------------------ */
static int cmp_pair(const void *a, const void *b) {
  const orc_pair *p = (const orc_pair *)a, *q = (const orc_pair *)b;
  if (p->i != q->i) return p->i < q->i ? -1 : 1;
  if (p->j != q->j) return p->j < q->j ? -1 : 1;
  return 0;
}

/*
 * Every unordered pair within radius sqrt(r2).  Cells have side at least the
 * radius, so both members of such a pair lie in the same or adjacent cells;
 * each particle is compared with every particle of its 27 surrounding cells
 * and a pair is kept once, from its lower index.
 */
int64_t orc_pairs(int64_t n, const float *const xyz[3], const double box[3],
                  double r2, orc_pair **out) {
  *out = NULL;
  if (n < 2 || !(r2 >= 0.0)) {
    *out = (orc_pair *)xmalloc(sizeof(orc_pair));
    return 0;
  }
  double r = sqrt(r2);
  double wmin = r * (1.0 + 1e-9) + 1e-300;
  double lo[3], ext[3];
  int64_t nc[3];
  for (int a = 0; a < 3; a++) {
    if (box[a] > 0.0) {
      lo[a] = 0.0;
      ext[a] = box[a];
    } else {
      double mn = xyz[a][0], mx = xyz[a][0];
      for (int64_t k = 1; k < n; k++) {
        if (xyz[a][k] < mn) mn = xyz[a][k];
        if (xyz[a][k] > mx) mx = xyz[a][k];
      }
      lo[a] = mn;
      ext[a] = mx - mn;
    }
  }
  /* cells no smaller than the radius; no more cells than about 4n */
  double grow = 1.0;
  for (;;) {
    double total = 1.0;
    for (int a = 0; a < 3; a++) {
      double f = floor(ext[a] / (wmin * grow));
      nc[a] = f < 1.0 ? 1 : (int64_t)f;
      if (box[a] > 0.0 && nc[a] < 3) nc[a] = 1; /* too few cells to wrap */
      total *= (double)nc[a];
    }
    if (total <= 4.0 * (double)n + 64.0) break;
    grow *= 1.25;
  }
  int64_t ncell = nc[0] * nc[1] * nc[2];
  int64_t *cell = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)n);
  int64_t *start = (int64_t *)xcalloc((size_t)ncell + 1, sizeof(int64_t));
  int64_t *members = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)n);
  int64_t *fill = (int64_t *)xcalloc((size_t)ncell, sizeof(int64_t));
  int64_t ci[3];
  for (int64_t k = 0; k < n; k++) {
    for (int a = 0; a < 3; a++) {
      int64_t c = 0;
      if (nc[a] > 1) {
        double w = ext[a] / (double)nc[a];
        c = (int64_t)floor(((double)xyz[a][k] - lo[a]) / w);
        if (box[a] > 0.0) {
          c %= nc[a];
          if (c < 0) c += nc[a];
        } else {
          if (c < 0) c = 0;
          if (c >= nc[a]) c = nc[a] - 1;
        }
      }
      ci[a] = c;
    }
    cell[k] = (ci[2] * nc[1] + ci[1]) * nc[0] + ci[0];
    start[cell[k] + 1]++;
  }
  for (int64_t c = 0; c < ncell; c++) start[c + 1] += start[c];
  for (int64_t k = 0; k < n; k++) members[start[cell[k]] + fill[cell[k]]++] = k;
  free(fill);

  int64_t cap = 1024, cnt = 0;
  orc_pair *pairs = (orc_pair *)xmalloc(sizeof(orc_pair) * (size_t)cap);
  for (int64_t i = 0; i < n; i++) {
    int64_t c = cell[i];
    int64_t cx = c % nc[0], cy = (c / nc[0]) % nc[1], cz = c / (nc[0] * nc[1]);
    for (int oz = -1; oz <= 1; oz++)
      for (int oy = -1; oy <= 1; oy++)
        for (int ox = -1; ox <= 1; ox++) {
          int64_t q[3] = {cx + ox, cy + oy, cz + oz};
          int o[3] = {ox, oy, oz};
          int skip = 0;
          for (int a = 0; a < 3; a++) {
            if (nc[a] == 1) {
              if (o[a] != 0) skip = 1;
            } else if (box[a] > 0.0) {
              q[a] = (q[a] + nc[a]) % nc[a];
            } else if (q[a] < 0 || q[a] >= nc[a]) {
              skip = 1;
            }
          }
          if (skip) continue;
          int64_t nb = (q[2] * nc[1] + q[1]) * nc[0] + q[0];
          for (int64_t s = start[nb]; s < start[nb + 1]; s++) {
            int64_t j = members[s];
            if (j <= i) continue;
            double d2 = orc_dist2(xyz, i, j, box);
            if (d2 <= r2) {
              if (cnt == cap) {
                cap *= 2;
                orc_pair *np = (orc_pair *)realloc(pairs, sizeof(orc_pair) * (size_t)cap);
                if (!np) {
                  free(pairs);
                  free(cell);
                  free(start);
                  free(members);
                  return -1;
                }
                pairs = np;
              }
              pairs[cnt].i = (uint32_t)i;
              pairs[cnt].j = (uint32_t)j;
              pairs[cnt].d2 = d2;
              cnt++;
            }
          }
        }
  }
  free(cell);
  free(start);
  free(members);
  qsort(pairs, (size_t)cnt, sizeof(orc_pair), cmp_pair);
  *out = pairs;
  return cnt;
}

/* ------------------------------------------------------------------------ */
/* union-find with minimum-index roots (Sec. 2.4.1)                         */
/* ------------------------------------------------------------------------ */
static int32_t uf_find(int32_t *parent, int32_t a) {
  while (parent[a] != a) {
    parent[a] = parent[parent[a]]; /* path halving */
    a = parent[a];
  }
  return a;
}

/* Links the larger root under the smaller one; 1 if two sets were merged. */
static int uf_union(int32_t *parent, int32_t a, int32_t b) {
  a = uf_find(parent, a);
  b = uf_find(parent, b);
  if (a == b) return 0;
  if (a < b)
    parent[b] = a;
  else
    parent[a] = b;
  return 1;
}

/*
 * Sec. 2.4: FoF clusters are the connected components of the graph of links
 * d <= b.  Sec. 3.2: safe components are those of the safe links.  Every
 * label is the smallest particle index of its component.
 */
void orc_components(int64_t n, const orc_pair *pairs, int64_t np,
                    const orc_consts *c, int which, int32_t *labels) {
  for (int64_t k = 0; k < n; k++) labels[k] = (int32_t)k;
  for (int64_t k = 0; k < np; k++) {
    int cls = orc_classify(pairs[k].d2, c);
    int take = which == 0 ? (cls == ORC_SAFE) : (cls == ORC_SAFE || cls == ORC_PB);
    if (take) uf_union(labels, (int32_t)pairs[k].i, (int32_t)pairs[k].j);
  }
  for (int64_t k = 0; k < n; k++) labels[k] = uf_find(labels, (int32_t)k);
}

/* ------------------------------------------------------------------------ */
/* constraint selection (Sec. 3.2, Sec. 3.3 "Active pair selection")         */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint64_t key;
  uint32_t i, j;
} orc_cand;

static int cmp_cand(const void *a, const void *b) {
  const orc_cand *p = (const orc_cand *)a, *q = (const orc_cand *)b;
  return p->key < q->key ? -1 : (p->key > q->key ? 1 : 0);
}

typedef struct {
  uint32_t i, j;
  uint8_t t;
} orc_act;

static int cmp_act(const void *a, const void *b) {
  const orc_act *p = (const orc_act *)a, *q = (const orc_act *)b;
  if (p->i != q->i) return p->i < q->i ? -1 : 1;
  if (p->j != q->j) return p->j < q->j ? -1 : 1;
  return 0;
}

/*
 * VP: A = V.
 * SC: drop vulnerable pairs whose ends share a safe component.
 * HF: contract safe components to supernodes; potentially-created pairs are
 * kept only between different original halos; of the potentially-broken
 * pairs between different supernodes a spanning forest is kept.  The paper
 * accepts any spanning forest; the reading here is the unique minimum
 * spanning forest under the key (already violated at the reconstruction,
 * smaller index, larger index), built by Kruskal's algorithm.  The original
 * halos of the supernode graph are exactly the FoF components, because every
 * link is either safe or potentially broken.
 */
int64_t orc_select(int mode, int64_t n, const orc_pair *pairs, int64_t np,
                   const orc_consts *c, const int32_t *safe_labels,
                   const int32_t *fof_labels, const float *const rec[3],
                   const double box[3], uint32_t **a_i, uint32_t **a_j,
                   uint8_t **a_type) {
  orc_act *act = (orc_act *)xmalloc(sizeof(orc_act) * (size_t)(np + 1));
  int64_t na = 0;
  if (mode == ORC_VP || mode == ORC_SC) {
    for (int64_t k = 0; k < np; k++) {
      int cls = orc_classify(pairs[k].d2, c);
      if (cls != ORC_PB && cls != ORC_PC) continue;
      if (mode == ORC_SC && safe_labels[pairs[k].i] == safe_labels[pairs[k].j]) continue;
      act[na].i = pairs[k].i;
      act[na].j = pairs[k].j;
      act[na].t = (uint8_t)cls;
      na++;
    }
  } else {
    orc_cand *cand = (orc_cand *)xmalloc(sizeof(orc_cand) * (size_t)(np + 1));
    int64_t nc = 0;
    for (int64_t k = 0; k < np; k++) {
      int cls = orc_classify(pairs[k].d2, c);
      uint32_t i = pairs[k].i, j = pairs[k].j;
      if (cls == ORC_PC && fof_labels[i] != fof_labels[j]) {
        act[na].i = i;
        act[na].j = j;
        act[na].t = ORC_PC;
        na++;
      } else if (cls == ORC_PB && safe_labels[i] != safe_labels[j]) {
        uint64_t viol0 = orc_dist2(rec, i, j, box) > c->bm2 ? 1u : 0u;
        cand[nc].key = (viol0 << 62) | ((uint64_t)i << 31) | (uint64_t)j;
        cand[nc].i = i;
        cand[nc].j = j;
        nc++;
      }
    }
    qsort(cand, (size_t)nc, sizeof(orc_cand), cmp_cand);
    int32_t *super = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    for (int64_t k = 0; k < n; k++) super[k] = (int32_t)k;
    for (int64_t k = 0; k < nc; k++) {
      if (uf_union(super, safe_labels[cand[k].i], safe_labels[cand[k].j])) {
        act[na].i = cand[k].i;
        act[na].j = cand[k].j;
        act[na].t = ORC_PB;
        na++;
      }
    }
    free(super);
    free(cand);
  }
  qsort(act, (size_t)na, sizeof(orc_act), cmp_act);
  *a_i = (uint32_t *)xmalloc(sizeof(uint32_t) * (size_t)na);
  *a_j = (uint32_t *)xmalloc(sizeof(uint32_t) * (size_t)na);
  *a_type = (uint8_t *)xmalloc((size_t)na);
  for (int64_t k = 0; k < na; k++) {
    (*a_i)[k] = act[k].i;
    (*a_j)[k] = act[k].j;
    (*a_type)[k] = act[k].t;
  }
  free(act);
  return na;
}

/* ------------------------------------------------------------------------ */
/* projected gradient descent on the tightened loss (Alg. 1, Eq. 3)          */
/* ------------------------------------------------------------------------ */
typedef struct {
  double loss;
  int64_t viol;
} orc_eval;

/*
 * Tightened loss at q (Eq. 3) and its gradient.  A potentially-broken pair
 * (an original link) is violated when its current distance exceeds
 * b - delta_t; a potentially-created pair (an original non-link) when its
 * current distance is at most b + delta_t.  Each violated pair adds the square
 * of its overshoot h; the gradient of h^2 is 2 h times the derivative of the
 * distance, (q_i - q_j) / d for particle i and the opposite for j.  When a
 * created pair sits at distance 0 the direction is undefined; the reading
 * here takes the direction of the original positions.
 */
static orc_eval evaluate(int64_t na, const uint32_t *a_i, const uint32_t *a_j,
                         const uint8_t *a_type, const uint8_t *a_thr, const int64_t *eidx,
                         double *const q[3], double *const g[3], int64_t ne,
                         const float *const xyz[3], const double box[3],
                         const orc_consts *cs) {
  orc_eval ev = {0.0, 0};
  for (int a = 0; a < 3; a++) memset(g[a], 0, sizeof(double) * (size_t)ne);
  for (int64_t k = 0; k < na; k++) {
    const orc_consts *c = cs + a_thr[k]; /* the pair's own threshold */
    int64_t ei = eidx[a_i[k]], ej = eidx[a_j[k]];
    double dv[3];
    for (int a = 0; a < 3; a++) dv[a] = axis_diff(q[a][ei] - q[a][ej], box[a]);
    double d2 = (dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2];
    if (a_type[k] == ORC_PB) {
      if (d2 > c->bm2) {
        double d = sqrt(d2);
        double h = d - c->bm;
        ev.viol++;
        ev.loss += h * h;
        for (int a = 0; a < 3; a++) {
          double u = dv[a] / d;
          g[a][ei] += 2.0 * h * u;
          g[a][ej] -= 2.0 * h * u;
        }
      }
    } else {
      if (d2 <= c->bp2) {
        double d = sqrt(d2);
        double h = c->bp - d;
        double u[3];
        ev.viol++;
        ev.loss += h * h;
        if (d > 0.0) {
          for (int a = 0; a < 3; a++) u[a] = dv[a] / d;
        } else {
          double ov[3];
          for (int a = 0; a < 3; a++)
            ov[a] = axis_diff((double)xyz[a][a_i[k]] - (double)xyz[a][a_j[k]], box[a]);
          double od = sqrt((ov[0] * ov[0] + ov[1] * ov[1]) + ov[2] * ov[2]);
          for (int a = 0; a < 3; a++) u[a] = ov[a] / od;
        }
        for (int a = 0; a < 3; a++) {
          g[a][ei] -= 2.0 * h * u[a];
          g[a][ej] += 2.0 * h * u[a];
        }
      }
    }
  }
  return ev;
}

/*
 * Alg. 1 loop with the readings:
 *   - the stopping test comes first in every iteration (Sec. 3.3 "Gradient
 *     descent and projection"); by default it stops when no active pair is
 *     violated, or when the loss is <= loss_tol if that is set;
 *   - the step is Adam (Sec. 4.2) with bias correction and t starting at 1,
 *     or plain gradient descent (the printed Alg. 1);
 *   - after each step every editable particle is clamped into the box of
 *     half-width xi' centred on its original position (Eq. 2).
 * Returns the number of steps; q holds the final coordinates.
 */
static int64_t pgd(int64_t na, const uint32_t *a_i, const uint32_t *a_j,
                   const uint8_t *a_type, const uint8_t *a_thr, int64_t ne,
                   const uint32_t *e_ids, int64_t n, const float *const xyz[3],
                   const double box[3], const orc_consts *c, const orc_params *p,
                   double *const q[3], orc_result *r) {
  int64_t *eidx = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)(n ? n : 1));
  for (int64_t k = 0; k < n; k++) eidx[k] = -1;
  for (int64_t e = 0; e < ne; e++) eidx[e_ids[e]] = e;
  double *m[3], *v[3], *g[3], *lo[3], *hi[3];
  for (int a = 0; a < 3; a++) {
    m[a] = (double *)xcalloc((size_t)ne, sizeof(double));
    v[a] = (double *)xcalloc((size_t)ne, sizeof(double));
    g[a] = (double *)xcalloc((size_t)ne, sizeof(double));
    lo[a] = (double *)xmalloc(sizeof(double) * (size_t)ne);
    hi[a] = (double *)xmalloc(sizeof(double) * (size_t)ne);
    for (int64_t e = 0; e < ne; e++) {
      double x = (double)xyz[a][e_ids[e]];
      lo[a][e] = x - c->xi_p;
      hi[a][e] = x + c->xi_p;
    }
  }
  int64_t tmax = p->max_iters > 0 ? p->max_iters : 100000;
  int64_t cap = 64;
  r->loss_hist = (double *)xmalloc(sizeof(double) * (size_t)cap);
  r->viol_hist = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)cap);
  int64_t t = 0;
  for (;;) {
    orc_eval ev = evaluate(na, a_i, a_j, a_type, a_thr, eidx, q, g, ne, xyz, box, c);
    if (t + 1 > cap) {
      cap *= 2;
      r->loss_hist = (double *)realloc(r->loss_hist, sizeof(double) * (size_t)cap);
      r->viol_hist = (int64_t *)realloc(r->viol_hist, sizeof(int64_t) * (size_t)cap);
    }
    r->loss_hist[t] = ev.loss;
    r->viol_hist[t] = ev.viol;
    if (t == 0) {
      r->loss0 = ev.loss;
      r->viol0 = ev.viol;
    }
    r->loss_final = ev.loss;
    r->viol_final = ev.viol;
    int done = p->loss_tol > 0.0 ? (ev.loss <= p->loss_tol) : (ev.viol == 0);
    if (done) {
      r->status = ORC_OK;
      break;
    }
    if (t == tmax) {
      r->status = ORC_NOT_CONVERGED;
      break;
    }
    const double lr = p->lr; /* the fixed step of Sec. 4.2 */
    t++;
    double bc1 = 1.0 - pow(p->beta1, (double)t);
    double bc2 = 1.0 - pow(p->beta2, (double)t);
    for (int a = 0; a < 3; a++)
      for (int64_t e = 0; e < ne; e++) {
        double gr = g[a][e];
        if (p->optimizer == ORC_SGD) {
          q[a][e] = q[a][e] - lr * gr;
        } else {
          m[a][e] = p->beta1 * m[a][e] + (1.0 - p->beta1) * gr;
          v[a][e] = p->beta2 * v[a][e] + (1.0 - p->beta2) * gr * gr;
          double mh = m[a][e] / bc1;
          double vh = v[a][e] / bc2;
          q[a][e] = q[a][e] - lr * mh / (sqrt(vh) + p->adam_eps);
        }
        q[a][e] = fmin(fmax(q[a][e], lo[a][e]), hi[a][e]);
      }
  }
  for (int a = 0; a < 3; a++) {
    free(m[a]);
    free(v[a]);
    free(g[a]);
    free(lo[a]);
    free(hi[a]);
  }
  free(eidx);
  return t;
}

/* ------------------------------------------------------------------------ */
/* edit stream: flags, quantised edits, Huffman, ZSTD (Alg. 1, Sec. 3.3)     */
/* ------------------------------------------------------------------------ */
/*
 * Byte layout (little-endian), shared with the GPU library by specification
 * only:
 *   header, 64 bytes:
 *     u32 magic 0x45434350 | u16 version 2 | u8 m | u8 flags
 *     (bit 0: payload is one ZSTD frame, bit 1: symbols are Huffman coded)
 *     u64 n | u64 flagged | f64 step | f64 offset | u64 raw payload bytes |
 *     u64 stored payload bytes | u32 symbol bits (8 or 16) | u32 0
 *   payload:
 *     ceil(n/8) flag bytes, particle k at bit (k mod 8) of byte (k div 8);
 *     the symbol sequence: for axis x, y, z, for each flagged particle in
 *     increasing index, its code (m = 32: low 16 bits, then high 16 bits);
 *     Huffman coded: u32 K, K u32 symbols, K u8 code lengths, u64 bit count,
 *     u32 C (symbols per chunk), u32 0, then for each chunk of C symbols
 *     (the last one may be shorter) the u64 stream bit at which its first
 *     code starts, then the bits; canonical codes in (length, symbol) order,
 *     each code emitted most significant bit first, stream bit q at bit
 *     (q mod 8) of byte (q div 8).  The chunk starts let a decoder begin at
 *     any chunk.  Otherwise the symbols as little-endian integers.
 *   decode: edit = code * step - offset; x' = float32(x_hat + edit).
 */
#define ORC_MAGIC 0x45434350u
#define ORC_VERSION 2
#define ORC_HDR 64
#define ORC_MAXLEN 24
#define ORC_CHUNK 4096

typedef size_t (*zbound_fn)(size_t);
typedef size_t (*zcomp_fn)(void *, size_t, const void *, size_t, int);
typedef size_t (*zdecomp_fn)(void *, size_t, const void *, size_t);
typedef unsigned (*ziserr_fn)(size_t);

typedef struct {
  int ok;
  zbound_fn bound;
  zcomp_fn comp;
  zdecomp_fn decomp;
  ziserr_fn iserr;
} orc_zstd;

static orc_zstd *zstd_lib(void) {
  static orc_zstd z;
  static int tried = 0;
  if (!tried) {
    tried = 1;
    void *h = dlopen("libzstd.so.1", RTLD_NOW | RTLD_LOCAL);
    if (h) {
      z.bound = (zbound_fn)dlsym(h, "ZSTD_compressBound");
      z.comp = (zcomp_fn)dlsym(h, "ZSTD_compress");
      z.decomp = (zdecomp_fn)dlsym(h, "ZSTD_decompress");
      z.iserr = (ziserr_fn)dlsym(h, "ZSTD_isError");
      z.ok = z.bound && z.comp && z.decomp && z.iserr;
    }
  }
  return &z;
}

static void put_u16(uint8_t *b, uint16_t v) { memcpy(b, &v, 2); }
static void put_u32(uint8_t *b, uint32_t v) { memcpy(b, &v, 4); }
static void put_u64(uint8_t *b, uint64_t v) { memcpy(b, &v, 8); }
static void put_f64(uint8_t *b, double v) { memcpy(b, &v, 8); }
static uint16_t get_u16(const uint8_t *b) { uint16_t v; memcpy(&v, b, 2); return v; }
static uint32_t get_u32(const uint8_t *b) { uint32_t v; memcpy(&v, b, 4); return v; }
static uint64_t get_u64(const uint8_t *b) { uint64_t v; memcpy(&v, b, 8); return v; }
static double get_f64(const uint8_t *b) { double v; memcpy(&v, b, 8); return v; }

typedef struct {
  uint64_t f;
  int64_t id;
} orc_leaf;

static int cmp_leaf(const void *a, const void *b) {
  const orc_leaf *p = (const orc_leaf *)a, *q = (const orc_leaf *)b;
  if (p->f != q->f) return p->f < q->f ? -1 : 1;
  return p->id < q->id ? -1 : (p->id > q->id ? 1 : 0);
}

/* Huffman code lengths, at most ORC_MAXLEN bits: the two-queue construction;
 * if the deepest leaf is too deep, the counts are halved and it is redone. */
static void huff_lengths(int64_t k, const uint64_t *freq, uint8_t *len) {
  if (k == 1) {
    len[0] = 1;
    return;
  }
  uint64_t *f = (uint64_t *)xmalloc(sizeof(uint64_t) * (size_t)k);
  memcpy(f, freq, sizeof(uint64_t) * (size_t)k);
  int64_t nn = 2 * k - 1;
  uint64_t *w = (uint64_t *)xmalloc(sizeof(uint64_t) * (size_t)nn);
  int64_t *parent = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)nn);
  int32_t *depth = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)nn);
  orc_leaf *leaves = (orc_leaf *)xmalloc(sizeof(orc_leaf) * (size_t)k);
  for (;;) {
    for (int64_t s = 0; s < k; s++) {
      leaves[s].f = f[s];
      leaves[s].id = s;
      w[s] = f[s];
    }
    qsort(leaves, (size_t)k, sizeof(orc_leaf), cmp_leaf);
    int64_t lq = 0, iq = k, made = k;
    for (int64_t step = 0; step < k - 1; step++) {
      int64_t pick[2];
      for (int t = 0; t < 2; t++) {
        int use_leaf;
        if (lq >= k)
          use_leaf = 0;
        else if (iq >= made)
          use_leaf = 1;
        else
          use_leaf = leaves[lq].f <= w[iq];
        pick[t] = use_leaf ? leaves[lq++].id : iq++;
      }
      w[made] = w[pick[0]] + w[pick[1]];
      parent[pick[0]] = made;
      parent[pick[1]] = made;
      made++;
    }
    depth[nn - 1] = 0;
    for (int64_t s = nn - 2; s >= 0; s--) depth[s] = depth[parent[s]] + 1;
    int32_t mx = 0;
    for (int64_t s = 0; s < k; s++)
      if (depth[s] > mx) mx = depth[s];
    if (mx <= ORC_MAXLEN) {
      for (int64_t s = 0; s < k; s++) len[s] = (uint8_t)depth[s];
      break;
    }
    for (int64_t s = 0; s < k; s++) f[s] = (f[s] + 1) / 2;
  }
  free(f);
  free(w);
  free(parent);
  free(depth);
  free(leaves);
}

typedef struct {
  uint8_t len;
  uint32_t sym;
} orc_cl;

static int cmp_cl(const void *a, const void *b) {
  const orc_cl *p = (const orc_cl *)a, *q = (const orc_cl *)b;
  if (p->len != q->len) return p->len < q->len ? -1 : 1;
  return p->sym < q->sym ? -1 : (p->sym > q->sym ? 1 : 0);
}

/* canonical codes: in (length, symbol) order, each code is the previous one
 * plus one, shifted left by the growth in length */
static void canonical_codes(int64_t k, orc_cl *cl, uint32_t *code) {
  qsort(cl, (size_t)k, sizeof(orc_cl), cmp_cl);
  uint32_t cur = 0;
  for (int64_t s = 0; s < k; s++) {
    if (s > 0) cur = (cur + 1) << (cl[s].len - cl[s - 1].len);
    code[s] = cur;
  }
}

/* Writes the stream for the final coordinates p; returns its length. */
static int64_t encode(int64_t n, const float *const rec[3], double *const p[3],
                      const orc_params *par, const orc_consts *c, uint8_t **out,
                      int64_t *n_flagged) {
  int m = par->m_bits;
  int sym_bits = m == 8 ? 8 : 16;
  int per_code = m == 32 ? 2 : 1;
  uint64_t maxcode = (uint64_t)(ldexp(1.0, m) - 1.0);
  double step = c->qstep, offset = 2.0 * par->xi;
  int64_t nb = (n + 7) / 8;
  uint8_t *flags = (uint8_t *)xcalloc((size_t)nb, 1);
  int64_t nf = 0;
  for (int64_t k = 0; k < n; k++) {
    int moved = 0;
    for (int a = 0; a < 3; a++)
      if (p[a][k] - (double)rec[a][k] != 0.0) moved = 1;
    if (moved) {
      flags[k >> 3] |= (uint8_t)(1u << (k & 7));
      nf++;
    }
  }
  /* quantised edits: code = clamp(rint((edit + 2 xi) / step), 0, 2^m - 1) */
  int64_t nsym = 3 * nf * per_code;
  uint32_t *sym = (uint32_t *)xmalloc(sizeof(uint32_t) * (size_t)(nsym ? nsym : 1));
  int64_t w = 0;
  for (int a = 0; a < 3; a++)
    for (int64_t k = 0; k < n; k++) {
      if (!(flags[k >> 3] >> (k & 7) & 1)) continue;
      double edit = p[a][k] - (double)rec[a][k];
      double qv = rint((edit + offset) / step);
      if (qv < 0.0) qv = 0.0;
      if (qv > (double)maxcode) qv = (double)maxcode;
      uint64_t code = (uint64_t)qv;
      if (per_code == 2) {
        sym[w++] = (uint32_t)(code & 0xffffu);
        sym[w++] = (uint32_t)(code >> 16);
      } else {
        sym[w++] = (uint32_t)code;
      }
    }
  /* Huffman over the symbol alphabet */
  int64_t alpha = (int64_t)1 << sym_bits;
  uint64_t *hist = (uint64_t *)xcalloc((size_t)alpha, sizeof(uint64_t));
  for (int64_t s = 0; s < nsym; s++) hist[sym[s]]++;
  int64_t k = 0;
  for (int64_t s = 0; s < alpha; s++)
    if (hist[s]) k++;
  int64_t raw_len = nb;
  uint8_t *payload;
  int use_huff = nsym > 0;
  if (use_huff) {
    uint64_t *freq = (uint64_t *)xmalloc(sizeof(uint64_t) * (size_t)k);
    uint32_t *syms = (uint32_t *)xmalloc(sizeof(uint32_t) * (size_t)k);
    uint8_t *len = (uint8_t *)xmalloc((size_t)k);
    int64_t t = 0;
    for (int64_t s = 0; s < alpha; s++)
      if (hist[s]) {
        freq[t] = hist[s];
        syms[t] = (uint32_t)s;
        t++;
      }
    huff_lengths(k, freq, len);
    orc_cl *cl = (orc_cl *)xmalloc(sizeof(orc_cl) * (size_t)k);
    for (int64_t s = 0; s < k; s++) {
      cl[s].len = len[s];
      cl[s].sym = syms[s];
    }
    uint32_t *code = (uint32_t *)xmalloc(sizeof(uint32_t) * (size_t)k);
    canonical_codes(k, cl, code);
    uint32_t *sym_code = (uint32_t *)xcalloc((size_t)alpha, sizeof(uint32_t));
    uint8_t *sym_len = (uint8_t *)xcalloc((size_t)alpha, 1);
    for (int64_t s = 0; s < k; s++) {
      sym_code[cl[s].sym] = code[s];
      sym_len[cl[s].sym] = cl[s].len;
    }
    uint64_t nbits = 0;
    for (int64_t s = 0; s < nsym; s++) nbits += sym_len[sym[s]];
    int64_t bbytes = (int64_t)((nbits + 7) / 8);
    int64_t nchunks = (nsym + ORC_CHUNK - 1) / ORC_CHUNK;
    raw_len = nb + 4 + 5 * k + 8 + 8 + 8 * nchunks + bbytes;
    payload = (uint8_t *)xcalloc((size_t)raw_len, 1);
    memcpy(payload, flags, (size_t)nb);
    uint8_t *q = payload + nb;
    put_u32(q, (uint32_t)k);
    q += 4;
    for (int64_t s = 0; s < k; s++) put_u32(q + 4 * s, cl[s].sym);
    q += 4 * k;
    for (int64_t s = 0; s < k; s++) q[s] = cl[s].len;
    q += k;
    put_u64(q, nbits);
    q += 8;
    put_u32(q, ORC_CHUNK);
    q += 8;
    uint8_t *index = q;
    q += 8 * nchunks;
    uint64_t pos = 0;
    for (int64_t s = 0; s < nsym; s++) {
      if (s % ORC_CHUNK == 0) put_u64(index + 8 * (s / ORC_CHUNK), pos);
      uint32_t cd = sym_code[sym[s]];
      int l = sym_len[sym[s]];
      for (int bit = l - 1; bit >= 0; bit--) {
        if ((cd >> bit) & 1u) q[pos >> 3] |= (uint8_t)(1u << (pos & 7));
        pos++;
      }
    }
    free(freq);
    free(syms);
    free(len);
    free(cl);
    free(code);
    free(sym_code);
    free(sym_len);
  } else {
    payload = (uint8_t *)xcalloc((size_t)raw_len, 1);
    memcpy(payload, flags, (size_t)nb);
  }
  free(hist);
  free(sym);
  free(flags);
  /* ZSTD over the whole payload when the runtime library is present */
  orc_zstd *z = zstd_lib();
  uint8_t *stored = payload;
  int64_t stored_len = raw_len;
  int zflag = 0;
  if (z->ok && raw_len > 0) {
    size_t cap = z->bound((size_t)raw_len);
    uint8_t *zb = (uint8_t *)xmalloc(cap);
    size_t got = z->comp(zb, cap, payload, (size_t)raw_len, 3);
    if (!z->iserr(got)) {
      stored = zb;
      stored_len = (int64_t)got;
      zflag = 1;
    } else {
      free(zb);
    }
  }
  uint8_t *s = (uint8_t *)xcalloc((size_t)(ORC_HDR + stored_len), 1);
  put_u32(s + 0, ORC_MAGIC);
  put_u16(s + 4, ORC_VERSION);
  s[6] = (uint8_t)m;
  s[7] = (uint8_t)((zflag ? 1 : 0) | (use_huff ? 2 : 0));
  put_u64(s + 8, (uint64_t)n);
  put_u64(s + 16, (uint64_t)nf);
  put_f64(s + 24, step);
  put_f64(s + 32, offset);
  put_u64(s + 40, (uint64_t)raw_len);
  put_u64(s + 48, (uint64_t)stored_len);
  put_u32(s + 56, (uint32_t)sym_bits);
  memcpy(s + ORC_HDR, stored, (size_t)stored_len);
  if (stored != payload) free(stored);
  free(payload);
  *out = s;
  *n_flagged = nf;
  return ORC_HDR + stored_len;
}

/* Reconstruction of the edited data (Sec. 3.3): undo ZSTD and Huffman, map
 * the dequantised edits to the flagged particles, add them to x_hat. */
int orc_decode(const uint8_t *stream, int64_t len, int64_t n,
               const float *const rec[3], float *const out[3]) {
  if (len < ORC_HDR || get_u32(stream) != ORC_MAGIC || get_u16(stream + 4) != ORC_VERSION)
    return -1;
  int m = stream[6], fl = stream[7];
  if ((int64_t)get_u64(stream + 8) != n) return -1;
  int64_t nf = (int64_t)get_u64(stream + 16);
  double step = get_f64(stream + 24), offset = get_f64(stream + 32);
  int64_t raw_len = (int64_t)get_u64(stream + 40);
  int64_t stored_len = (int64_t)get_u64(stream + 48);
  int sym_bits = (int)get_u32(stream + 56);
  if (stored_len != len - ORC_HDR) return -1;
  if (!(m == 8 || m == 16 || m == 32) || !(sym_bits == 8 || sym_bits == 16)) return -1;
  uint8_t *payload;
  if (fl & 1) {
    orc_zstd *z = zstd_lib();
    if (!z->ok) return -2;
    payload = (uint8_t *)xmalloc((size_t)raw_len);
    size_t got = z->decomp(payload, (size_t)raw_len, stream + ORC_HDR, (size_t)stored_len);
    if (z->iserr(got) || (int64_t)got != raw_len) {
      free(payload);
      return -1;
    }
  } else {
    if (raw_len != stored_len) return -1;
    payload = (uint8_t *)xmalloc((size_t)(raw_len ? raw_len : 1));
    memcpy(payload, stream + ORC_HDR, (size_t)raw_len);
  }
  int per_code = m == 32 ? 2 : 1;
  int64_t nb = (n + 7) / 8;
  int64_t nsym = 3 * nf * per_code;
  uint32_t *sym = (uint32_t *)xmalloc(sizeof(uint32_t) * (size_t)(nsym ? nsym : 1));
  const uint8_t *q = payload + nb;
  if (nsym > 0 && (fl & 2)) {
    uint32_t k = get_u32(q);
    q += 4;
    orc_cl *cl = (orc_cl *)xmalloc(sizeof(orc_cl) * (size_t)(k ? k : 1));
    for (uint32_t s = 0; s < k; s++) cl[s].sym = get_u32(q + 4 * s);
    q += 4 * (size_t)k;
    for (uint32_t s = 0; s < k; s++) cl[s].len = q[s];
    q += k;
    uint64_t nbits = get_u64(q);
    q += 8;
    uint32_t chunk = get_u32(q);
    q += 8;
    if (chunk == 0) {
      free(cl);
      free(sym);
      free(payload);
      return -1;
    }
    /* the chunk starts: checked against the positions the decoding reaches */
    const uint8_t *index = q;
    q += 8 * (size_t)((nsym + chunk - 1) / chunk);
    uint32_t *code = (uint32_t *)xmalloc(sizeof(uint32_t) * (size_t)(k ? k : 1));
    canonical_codes(k, cl, code);
    /* per length: first canonical code and index of its first symbol */
    int64_t first_idx[ORC_MAXLEN + 2], count[ORC_MAXLEN + 2];
    uint32_t first_code[ORC_MAXLEN + 2];
    for (int l = 0; l <= ORC_MAXLEN + 1; l++) {
      count[l] = 0;
      first_idx[l] = -1;
      first_code[l] = 0;
    }
    for (uint32_t s = 0; s < k; s++) {
      int l = cl[s].len;
      if (count[l] == 0) {
        first_idx[l] = s;
        first_code[l] = code[s];
      }
      count[l]++;
    }
    uint64_t pos = 0;
    for (int64_t s = 0; s < nsym; s++) {
      uint32_t cd = 0;
      int l = 0;
      if (s % chunk == 0 && get_u64(index + 8 * (size_t)(s / chunk)) != pos) {
        free(cl);
        free(code);
        free(sym);
        free(payload);
        return -1;
      }
      for (;;) {
        if (pos >= nbits || l >= ORC_MAXLEN) {
          free(cl);
          free(code);
          free(sym);
          free(payload);
          return -1;
        }
        cd = (cd << 1) | ((q[pos >> 3] >> (pos & 7)) & 1u);
        pos++;
        l++;
        if (count[l] && cd >= first_code[l] && (int64_t)(cd - first_code[l]) < count[l]) {
          sym[s] = cl[first_idx[l] + (cd - first_code[l])].sym;
          break;
        }
      }
    }
    free(cl);
    free(code);
  } else {
    int bytes = sym_bits / 8;
    for (int64_t s = 0; s < nsym; s++) {
      uint32_t v = 0;
      for (int t = 0; t < bytes; t++) v |= (uint32_t)q[bytes * s + t] << (8 * t);
      sym[s] = v;
    }
  }
  for (int a = 0; a < 3; a++) memcpy(out[a], rec[a], sizeof(float) * (size_t)n);
  int64_t r = 0;
  for (int a = 0; a < 3; a++)
    for (int64_t k = 0; k < n; k++) {
      if (!(payload[k >> 3] >> (k & 7) & 1)) continue;
      uint64_t code;
      if (per_code == 2) {
        code = (uint64_t)sym[r] | ((uint64_t)sym[r + 1] << 16);
        r += 2;
      } else {
        code = sym[r++];
      }
      double edit = (double)code * step - offset;
      out[a][k] = (float)((double)rec[a][k] + edit);
    }
  free(sym);
  free(payload);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* the whole correction                                                     */
/* ------------------------------------------------------------------------ */
/* union of the per-threshold active lists, ordered by (i, j, threshold) */
typedef struct {
  uint32_t i, j;
  uint8_t type, thr;
} orc_tagged;

static int cmp_tagged(const void *a, const void *b) {
  const orc_tagged *x = (const orc_tagged *)a, *y = (const orc_tagged *)b;
  if (x->i != y->i) return x->i < y->i ? -1 : 1;
  if (x->j != y->j) return x->j < y->j ? -1 : 1;
  return (int)x->thr - (int)y->thr;
}

/*
 * The correction for one or more linking lengths b_list[0..nb).  Every
 * threshold's constraints are selected exactly as for a single one (its own
 * pair classes, safe components, halos and forest); the active list is their
 * union, each pair tagged with its threshold (a pair selected for two
 * thresholds is two constraints), and the tightened loss sums every
 * constraint with its own b -+ delta_t.  The margins (delta_q, xi', delta_t)
 * depend on xi, m and the coordinates only, so they are shared.  labels_all,
 * if not NULL, receives the FoF labels at every b ([nb][n]); r->labels and
 * r->safe_labels are those of b_list[0].
 */
static int correct_impl(int64_t n, const float *const xyz[3], const float *const rec[3],
                        const orc_params *p, const double *b_list, int nb,
                        int32_t *labels_all, orc_result *r) {
  memset(r, 0, sizeof(*r));
  if (n < 0 || nb < 1 || nb > ORC_MAX_THRESHOLDS || !(p->xi >= 0.0) ||
      !(p->m_bits == 8 || p->m_bits == 16 || p->m_bits == 32))
    return r->status = ORC_E_INVALID;
  double bmax = 0.0;
  for (int k = 0; k < nb; k++) {
    if (!(b_list[k] > 0.0)) return r->status = ORC_E_INVALID;
    if (b_list[k] > bmax) bmax = b_list[k];
  }
  for (int a = 0; a < 3; a++) {
    if (!(p->box[a] >= 0.0)) return r->status = ORC_E_INVALID;
    if (p->box[a] > 0.0 && !(p->box[a] > 2.0 * (bmax + 2.0 * sqrt(3.0) * p->xi)))
      return r->status = ORC_E_INVALID;
  }
  for (int a = 0; a < 3; a++)
    for (int64_t k = 0; k < n; k++) {
      if (!isfinite(xyz[a][k]) || !isfinite(rec[a][k])) return r->status = ORC_E_INVALID;
      /* Sec. 3.1 assumes the base compressor honours the bound */
      if (fabs((double)rec[a][k] - (double)xyz[a][k]) > p->xi)
        return r->status = ORC_E_INPUT_BOUND;
    }
  const double maxabs = orc_max_abs(n, xyz, rec);
  orc_consts cs[ORC_MAX_THRESHOLDS];
  orc_tagged *all = NULL;
  int64_t n_all = 0;
  int32_t *lab = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
  int32_t *safe = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
  for (int t = 0; t < nb; t++) {
    orc_params pt = *p;
    pt.b = b_list[t];
    orc_constants(&pt, maxabs, &cs[t]);
    orc_pair *pairs = NULL;
    int64_t np = orc_pairs(n, xyz, p->box, cs[t].rv2, &pairs);
    if (t == 0) {
      r->n_pairs = np;
      for (int64_t k = 0; k < np; k++) {
        int cls = orc_classify(pairs[k].d2, &cs[0]);
        r->n_safe += cls == ORC_SAFE;
        r->n_pb += cls == ORC_PB;
        r->n_pc += cls == ORC_PC;
      }
    }
    orc_components(n, pairs, np, &cs[t], 1, lab);
    orc_components(n, pairs, np, &cs[t], 0, safe);
    if (labels_all) memcpy(labels_all + (size_t)t * (size_t)n, lab, sizeof(int32_t) * (size_t)n);
    if (t == 0) {
      r->labels = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
      r->safe_labels = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
      memcpy(r->labels, lab, sizeof(int32_t) * (size_t)n);
      memcpy(r->safe_labels, safe, sizeof(int32_t) * (size_t)n);
    }
    uint32_t *ai = NULL, *aj = NULL;
    uint8_t *at = NULL;
    int64_t na = orc_select(p->mode, n, pairs, np, &cs[t], safe, lab, rec, p->box, &ai, &aj, &at);
    free(pairs);
    all = (orc_tagged *)realloc(all, sizeof(orc_tagged) * (size_t)(n_all + na + 1));
    for (int64_t k = 0; k < na; k++) {
      all[n_all + k].i = ai[k];
      all[n_all + k].j = aj[k];
      all[n_all + k].type = at[k];
      all[n_all + k].thr = (uint8_t)t;
    }
    n_all += na;
    free(ai);
    free(aj);
    free(at);
  }
  free(lab);
  free(safe);
  qsort(all, (size_t)n_all, sizeof(orc_tagged), cmp_tagged);
  r->n_a = n_all;
  r->a_i = (uint32_t *)xmalloc(sizeof(uint32_t) * (size_t)(n_all ? n_all : 1));
  r->a_j = (uint32_t *)xmalloc(sizeof(uint32_t) * (size_t)(n_all ? n_all : 1));
  r->a_type = (uint8_t *)xmalloc((size_t)(n_all ? n_all : 1));
  r->a_thr = (uint8_t *)xmalloc((size_t)(n_all ? n_all : 1));
  for (int64_t k = 0; k < n_all; k++) {
    r->a_i[k] = all[k].i;
    r->a_j[k] = all[k].j;
    r->a_type[k] = all[k].type;
    r->a_thr[k] = all[k].thr;
  }
  free(all);
  r->n_active = r->n_a;

  /* E = endpoints(A), ascending */
  uint8_t *is_e = (uint8_t *)xcalloc((size_t)(n ? n : 1), 1);
  for (int64_t k = 0; k < r->n_a; k++) is_e[r->a_i[k]] = is_e[r->a_j[k]] = 1;
  r->n_e = 0;
  for (int64_t k = 0; k < n; k++) r->n_e += is_e[k];
  r->e_ids = (uint32_t *)xmalloc(sizeof(uint32_t) * (size_t)(r->n_e ? r->n_e : 1));
  for (int64_t k = 0, t = 0; k < n; k++)
    if (is_e[k]) r->e_ids[t++] = (uint32_t)k;
  free(is_e);
  r->n_editable = r->n_e;

  /* optimise the editable coordinates, starting from the reconstruction */
  double *q[3];
  for (int a = 0; a < 3; a++) {
    q[a] = (double *)xmalloc(sizeof(double) * (size_t)(r->n_e ? r->n_e : 1));
    for (int64_t e = 0; e < r->n_e; e++) q[a][e] = (double)rec[a][r->e_ids[e]];
  }
  r->iters = pgd(r->n_a, r->a_i, r->a_j, r->a_type, r->a_thr, r->n_e, r->e_ids, n, xyz,
                 p->box, cs, p, q, r);
  r->p = (double *)xmalloc(sizeof(double) * (size_t)(3 * n + 1));
  double *pp[3] = {r->p, r->p + n, r->p + 2 * n};
  for (int a = 0; a < 3; a++) {
    for (int64_t k = 0; k < n; k++) pp[a][k] = (double)rec[a][k];
    for (int64_t e = 0; e < r->n_e; e++) pp[a][r->e_ids[e]] = q[a][e];
    free(q[a]);
  }
  r->stream_len = encode(n, rec, pp, p, &cs[0], &r->stream, &r->n_flagged);
  return r->status;
}

int orc_correct(int64_t n, const float *const xyz[3], const float *const rec[3],
                const orc_params *p, orc_result *r) {
  return correct_impl(n, xyz, rec, p, &p->b, 1, NULL, r);
}

int orc_correct_multi(int64_t n, const float *const xyz[3], const float *const rec[3],
                      const orc_params *p, const double *b_list, int32_t nb,
                      int32_t *labels_all, orc_result *r) {
  return correct_impl(n, xyz, rec, p, b_list, nb, labels_all, r);
}

void orc_result_free(orc_result *r) {
  free(r->labels);
  free(r->safe_labels);
  free(r->a_i);
  free(r->a_j);
  free(r->a_type);
  free(r->a_thr);
  free(r->e_ids);
  free(r->p);
  free(r->loss_hist);
  free(r->viol_hist);
  free(r->stream);
  memset(r, 0, sizeof(*r));
}

int orc_fof_labels(int64_t n, const float *const xyz[3], double b,
                   const double box[3], int32_t *labels) {
  orc_pair *pairs = NULL;
  int64_t np = orc_pairs(n, xyz, box, b * b, &pairs);
  if (np < 0) return -1;
  for (int64_t k = 0; k < n; k++) labels[k] = (int32_t)k;
  for (int64_t k = 0; k < np; k++) uf_union(labels, (int32_t)pairs[k].i, (int32_t)pairs[k].j);
  for (int64_t k = 0; k < n; k++) labels[k] = uf_find(labels, (int32_t)k);
  free(pairs);
  return 0;
}
