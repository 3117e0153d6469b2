/*
 * vqhull_oracle.c -- plain CPU Quickhull, the ground truth that the HIP path is
 * checked against.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library, and the GPU library never calls
 * it.
 *
 * What it computes (VQhull paper, Section 2.1, Algorithm 1 "Quickhull
 * algorithm"): the vertices of the convex hull of a finite planar point set, in
 * clockwise order, by the recursive partition of Algorithm 1.  Quickhull on
 * binary64 inputs does not always return the exact hull (Section 5.2, the
 * Circle dataset: round-off makes near-collinear neighbours look concave), so
 * this file is the algorithm itself, step by step, with every floating-point
 * and tie decision fixed:
 *
 *   R1  orient(a,b,c) = (a.x-c.x)*(b.y-c.y) - (a.y-c.y)*(b.x-c.x) in binary64,
 *       round to nearest even, evaluated in exactly this order, with no fused
 *       multiply-add (this file must be compiled with -ffp-contract=off) and
 *       gradual underflow.  "u is left of a->b" is orient(a,b,u) > 0: this is
 *       the displayed left-of inequality of Section 2.1 with both products
 *       moved to one side (for finite products A > B iff fl(A-B) > 0).
 *   R2  "right of p->q" at the top level is "left of q->p", orient(q,p,u) > 0,
 *       which is exactly -orient(p,q,u).
 *   R3  the distance order of Section 2.1 is realised by the scalar key
 *       orient(a,b,u) for the edge a->b (|ab| times the signed distance in
 *       exact arithmetic, so the same order); argmax ties are broken by
 *       x ascending, then y ascending, then index ascending.
 *   R4  p is the lexicographic minimum of (x, y, index) and q the
 *       lexicographic maximum of (x, y), lowest index among equal points.
 *   R5  a point left of both a->r and r->b (possible only under rounding) goes
 *       to S1.
 *   R6  the tests are strict: points on an edge are dropped.
 *   R7  output order: [p] ++ Hull(S1,p,r1,q) ++ [q] ++ Hull(S2,q,r2,p) with
 *       Hull(P,a,r,b) = Hull(S1,a,r1,r) ++ [r] ++ Hull(S2,r,r2,b), which is
 *       clockwise from p with y pointing up.
 *   R8  n = 0 gives no vertex; all points equal gives [p]; NaN or infinity in
 *       the input is an error (status 3).
 *
 * The recursion is the plain recursive function of Algorithm 1; every call
 * allocates one buffer for its two subsets and frees it on return.
 *
 * A multithreaded form of the same function (vqhull_oracle_hull_mt, OpenMP)
 * serves as the all-core CPU baseline.  It computes exactly the same steps:
 * the extremes and every partition are split into chunks of consecutive
 * points whose partial results are combined in chunk order (so each subset
 * lists its points in the same order as the sequential scan), and the two
 * recursive calls of each step run as independent tasks whose vertex lists
 * are joined in the order of R7.  Its result is identical to
 * vqhull_oracle_hull's for any thread count.
 *
 * Octagon prefilter (Section 6: the Akl-Toussaint heuristic the paper proposes
 * as future work).  A variant of the method first drops the points that lie
 * strictly inside the octagon spanned by eight directional extremes, then runs
 * Algorithm 1 unchanged on the points that remain (keeping their indices).
 * The dropped points lie strictly inside the hull, so in exact arithmetic the
 * hull is the same; the rules below fix every rounding and tie:
 *
 *   F1  vertices, counter-clockwise: v0 = min y, v1 = max fl(x-y), v2 = q (R4),
 *       v3 = max fl(x+y), v4 = max y, v5 = min fl(x-y), v6 = p (R4),
 *       v7 = min fl(x+y); among equal values the lowest index.
 *   F2  D = fl(fl(x[v2] - x[v6]) + fl(y[v4] - y[v0])) bounds every coordinate
 *       difference |u - v| of the input (width plus height of its box).
 *   F3  coordinates are taken relative to the origin o = p: u' = (fl(u.x - o.x),
 *       fl(u.y - o.y)).  Edge i runs from a = v_i to b = v_(i+1 mod 8):
 *       ex = fl(b.x - a.x), ey = fl(b.y - a.y), and
 *         L_i(u) = fl(fl(ex * u'.y) - fl(ey * u'.x)),
 *         c_i    = L_i(a) (the same expression for the vertex a),
 *         M_i    = max(2^-44 * fl(fl(|ex| + |ey|) * D), 2^-900),
 *         T_i    = fl(c_i + M_i).
 *       L_i(u) - c_i is the cross product of the edge with u - a: positive on
 *       the inner, left side of a counter-clockwise polygon.
 *   F4  u is dropped iff L_i(u) > T_i for all eight edges.  The rounding
 *       errors of L_i(u), c_i and T_i together with the rounding of the edge
 *       direction stay below 10 ulp-units of (|ex| + |ey|) * D (and below
 *       2^-1070 in the gradual-underflow range), far under M_i, so a dropped
 *       point is strictly left of every edge in exact arithmetic: the closed
 *       polygon then winds around it, which puts it strictly inside the hull.
 *       An edge of zero length (ex = ey = 0: a repeated vertex) adds nothing
 *       to the winding and is skipped (T_i = -infinity); when all eight edges
 *       have zero length (all points equal) nothing is dropped.
 *   F5  the filter applies only to inputs of more than a given number of
 *       points (below it every point is kept).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_ERR_INVALID_ARGUMENT 1
#define ORACLE_ERR_OUT_OF_MEMORY 2
#define ORACLE_ERR_NONFINITE 3

/* R1: the orientation value; positive iff c is strictly left of a->b. */
double vqhull_oracle_orient(double ax, double ay, double bx, double by, double cx, double cy) {
  double t1 = ax - cx;
  double t2 = by - cy;
  double t3 = ay - cy;
  double t4 = bx - cx;
  double m1 = t1 * t2;
  double m2 = t3 * t4;
  return m1 - m2;
}

/* R3: is candidate (k, i) farther than the current best (bk, bi)?  best < 0
 * means "no best yet". */
static int farther(const double* x, const double* y, double k, int64_t i, double bk, int64_t bi) {
  if (bi < 0) return 1;
  if (k > bk) return 1;
  if (k < bk) return 0;
  if (x[i] < x[bi]) return 1;
  if (x[i] > x[bi]) return 0;
  if (y[i] < y[bi]) return 1;
  if (y[i] > y[bi]) return 0;
  return i < bi;
}

typedef struct {
  int64_t* idx;
  int64_t len;
} out_list;

/*
 * One partition step of Algorithm 1 for the triangle (a, r, b): every u of P
 * left of a->r goes to S1, else every u left of r->b goes to S2, else it is
 * dropped (R5, R6); r1 and r2 are the farthest points of S1 from a->r and of
 * S2 from r->b (R3).  S1 is written to s[0..n1) and S2 to s[m-n2..m).
 */
static void split(const double* x, const double* y, const int64_t* P, int64_t m, int64_t a, int64_t r, int64_t b,
                  int64_t* s, int64_t* n1_out, int64_t* n2_out, int64_t* r1_out, int64_t* r2_out) {
  int64_t n1 = 0, n2 = 0;
  int64_t r1 = -1, r2 = -1;
  double k1 = 0.0, k2 = 0.0;
  for (int64_t j = 0; j < m; ++j) {
    int64_t u = P[j];
    double o1 = vqhull_oracle_orient(x[a], y[a], x[r], y[r], x[u], y[u]);
    if (o1 > 0.0) {
      s[n1++] = u;
      if (farther(x, y, o1, u, k1, r1)) {
        k1 = o1;
        r1 = u;
      }
      continue;
    }
    double o2 = vqhull_oracle_orient(x[r], y[r], x[b], y[b], x[u], y[u]);
    if (o2 > 0.0) {
      s[m - 1 - n2++] = u;
      if (farther(x, y, o2, u, k2, r2)) {
        k2 = o2;
        r2 = u;
      }
    }
  }
  *n1_out = n1;
  *n2_out = n2;
  *r1_out = r1;
  *r2_out = r2;
}

/* Hull(P, a, r, b) of Algorithm 1, appending its vertices in order (R7). */
static int hull_rec(const double* x, const double* y, const int64_t* P, int64_t m, int64_t a, int64_t r, int64_t b,
                    out_list* out) {
  if (m <= 1) { /* base case: return P itself */
    if (m == 1) out->idx[out->len++] = P[0];
    return ORACLE_OK;
  }
  int64_t* s = (int64_t*)malloc((size_t)m * sizeof(int64_t));
  if (!s) return ORACLE_ERR_OUT_OF_MEMORY;
  int64_t n1, n2, r1, r2;
  split(x, y, P, m, a, r, b, s, &n1, &n2, &r1, &r2);
  int st = hull_rec(x, y, s, n1, a, r1, r, out);
  if (st == ORACLE_OK) {
    out->idx[out->len++] = r;
    st = hull_rec(x, y, s + (m - n2), n2, r, r2, b, out);
  }
  free(s);
  return st;
}

/* R1 on n triples: abc holds a.x, a.y, b.x, b.y, c.x, c.y per triple. */
int vqhull_oracle_orient_batch(const double* abc, int64_t n, double* out) {
  if (n < 0 || (n > 0 && (!abc || !out))) return ORACLE_ERR_INVALID_ARGUMENT;
  for (int64_t i = 0; i < n; ++i) {
    const double* t = abc + 6 * i;
    out[i] = vqhull_oracle_orient(t[0], t[1], t[2], t[3], t[4], t[5]);
  }
  return ORACLE_OK;
}

/* R4: p = lexmin (x, y, index); q = lexmax (x, y), lowest index among equals. */
int vqhull_oracle_extremes(const double* x, const double* y, int64_t n, int64_t* p_out, int64_t* q_out) {
  if (n < 1 || !x || !y || !p_out || !q_out) return ORACLE_ERR_INVALID_ARGUMENT;
  int64_t p = 0, q = 0;
  for (int64_t i = 1; i < n; ++i) {
    if (x[i] < x[p] || (x[i] == x[p] && y[i] < y[p])) p = i;
    if (x[i] > x[q] || (x[i] == x[q] && y[i] > y[q])) q = i;
  }
  *p_out = p;
  *q_out = q;
  return ORACLE_OK;
}

/*
 * One partition step on an explicit subset: P holds m point indices, (a, r, b)
 * the triangle.  s must hold m entries; on return S1 = s[0..n1) and
 * S2 = s[m-n2..m) (each in the scan order of P), and r1 / r2 are the argmax
 * points (-1 for an empty subset).  The top-level step of Algorithm 1 is
 * (a, r, b) = (p, q, p).
 */
int vqhull_oracle_split(const double* x, const double* y, const int64_t* P, int64_t m, int64_t a, int64_t r,
                        int64_t b, int64_t* s, int64_t* n1, int64_t* n2, int64_t* r1, int64_t* r2) {
  if (m < 0 || !x || !y || (m > 0 && (!P || !s)) || !n1 || !n2 || !r1 || !r2) return ORACLE_ERR_INVALID_ARGUMENT;
  split(x, y, P, m, a, r, b, s, n1, n2, r1, r2);
  return ORACLE_OK;
}

/*
 * Algorithm 1 on all n points: writes the hull vertices (indices into x, y)
 * in clockwise order from p to out_idx (capacity n) and their number to
 * *out_count.
 */
int vqhull_oracle_hull(const double* x, const double* y, int64_t n, int64_t* out_idx, int64_t* out_count) {
  if (n < 0 || !out_count || (n > 0 && (!x || !y || !out_idx))) return ORACLE_ERR_INVALID_ARGUMENT;
  *out_count = 0;
  if (n == 0) return ORACLE_OK;
  for (int64_t i = 0; i < n; ++i)
    if (!isfinite(x[i]) || !isfinite(y[i])) return ORACLE_ERR_NONFINITE;

  int64_t p, q;
  vqhull_oracle_extremes(x, y, n, &p, &q);
  out_list out = {out_idx, 0};
  out.idx[out.len++] = p;
  if (p == q) { /* every point equals p */
    *out_count = out.len;
    return ORACLE_OK;
  }

  int64_t* all = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int64_t* s = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  if (!all || !s) {
    free(all);
    free(s);
    return ORACLE_ERR_OUT_OF_MEMORY;
  }
  for (int64_t i = 0; i < n; ++i) all[i] = i;
  /* S1 = left of p->q, S2 = left of q->p (R2), r1 / r2 their farthest points:
   * the partition of the degenerate triangle (p, q, p). */
  int64_t n1, n2, r1, r2;
  split(x, y, all, n, p, q, p, s, &n1, &n2, &r1, &r2);
  free(all);
  int st = hull_rec(x, y, s, n1, p, r1, q, &out);
  if (st == ORACLE_OK) {
    out.idx[out.len++] = q;
    st = hull_rec(x, y, s + (n - n2), n2, q, r2, p, &out);
  }
  free(s);
  if (st == ORACLE_OK) *out_count = out.len;
  return st;
}

/* F1: v = argmin (sign * value(i)) with the lowest index among equal values. */
static int64_t oct_extreme(const double* x, const double* y, int64_t n, int dir) {
  int64_t best = 0;
  double bv = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double v;
    switch (dir) {
      case 0: v = y[i]; break;           /* min y */
      case 1: v = -(x[i] - y[i]); break; /* max fl(x-y): -fl(x-y) is exact */
      case 3: v = -(x[i] + y[i]); break; /* max fl(x+y) */
      case 4: v = -y[i]; break;          /* max y */
      case 5: v = x[i] - y[i]; break;    /* min fl(x-y) */
      default: v = x[i] + y[i]; break;   /* 7: min fl(x+y) */
    }
    if (i == 0 || v < bv) {
      best = i;
      bv = v;
    }
  }
  return best;
}

/*
 * F1-F4 on all n points (no size threshold): writes the eight vertices to
 * vert[0..8) and keep[i] = 0 for a dropped point, 1 otherwise.
 */
int vqhull_oracle_octagon(const double* x, const double* y, int64_t n, int64_t* vert, uint8_t* keep) {
  if (n < 1 || !x || !y || !vert || !keep) return ORACLE_ERR_INVALID_ARGUMENT;
  int64_t p, q;
  vqhull_oracle_extremes(x, y, n, &p, &q);
  for (int d = 0; d < 8; ++d) vert[d] = d == 2 ? q : d == 6 ? p : oct_extreme(x, y, n, d);
  double D = (x[q] - x[p]) + (y[vert[4]] - y[vert[0]]);
  double ox = x[p], oy = y[p];
  double ex[8], ey[8], T[8];
  int edges = 0;
  for (int i = 0; i < 8; ++i) {
    int64_t a = vert[i], b = vert[(i + 1) % 8];
    ex[i] = x[b] - x[a];
    ey[i] = y[b] - y[a];
    double ay = y[a] - oy;
    double ax = x[a] - ox;
    double c1 = ex[i] * ay;
    double c2 = ey[i] * ax;
    double c = c1 - c2;
    double s = fabs(ex[i]) + fabs(ey[i]);
    double sd = s * D;
    double M = fmax(0x1p-44 * sd, 0x1p-900);
    T[i] = c + M;
    if (ex[i] == 0.0 && ey[i] == 0.0) {
      T[i] = -INFINITY;
    } else {
      ++edges;
    }
  }
  for (int64_t u = 0; u < n; ++u) {
    if (edges == 0) {
      keep[u] = 1;
      continue;
    }
    double uy = y[u] - oy;
    double ux = x[u] - ox;
    int inside = 1;
    for (int i = 0; i < 8; ++i) {
      double l1 = ex[i] * uy;
      double l2 = ey[i] * ux;
      double L = l1 - l2;
      if (!(L > T[i])) inside = 0;
    }
    keep[u] = (uint8_t)!inside;
  }
  return ORACLE_OK;
}

/* ------------------------------------------------ multithreaded form (OpenMP)
 *
 * The all-core CPU baseline.  Same rules R1-R8, same partition order, same
 * result as vqhull_oracle_hull.  `grain` is the number of points per chunk of
 * a parallel scan and the smallest subproblem that is handed to a task of its
 * own (smaller ones run in the calling task).
 */
typedef struct {
  int64_t n1, n2, r1, r2;
} part_acc;

/* split() over chunks of `grain` points run as tasks: each chunk is split on
 * its own into its slice of `tmp` (S1 at the slice's front, S2 at its back),
 * then the chunks are combined in order -- sizes summed into offsets, farthest
 * points compared by R3 -- and each chunk's members are copied to the places
 * the sequential split would give them: the j-th member of S1 overall at
 * s[j], the j-th member of S2 at s[m - 1 - j]. */
static int split_mt(const double* x, const double* y, const int64_t* P, int64_t m, int64_t a, int64_t r, int64_t b,
                    int64_t* s, int64_t grain, int64_t* n1, int64_t* n2, int64_t* r1, int64_t* r2) {
  int64_t nch = (m + grain - 1) / grain;
  part_acc* acc = (part_acc*)malloc((size_t)nch * sizeof(part_acc));
  int64_t* tmp = (int64_t*)malloc((size_t)m * sizeof(int64_t));
  if (!acc || !tmp) {
    free(acc);
    free(tmp);
    return ORACLE_ERR_OUT_OF_MEMORY;
  }
#pragma omp taskloop grainsize(1)
  for (int64_t c = 0; c < nch; ++c) {
    int64_t lo = c * grain, hi = lo + grain < m ? lo + grain : m;
    split(x, y, P + lo, hi - lo, a, r, b, tmp + lo, &acc[c].n1, &acc[c].n2, &acc[c].r1, &acc[c].r2);
  }
  int64_t t1 = 0, t2 = 0, b1 = -1, b2 = -1;
  double k1 = 0.0, k2 = 0.0;
  int64_t* o1 = (int64_t*)malloc((size_t)nch * 2 * sizeof(int64_t));
  if (!o1) {
    free(acc);
    free(tmp);
    return ORACLE_ERR_OUT_OF_MEMORY;
  }
  for (int64_t c = 0; c < nch; ++c) {
    if (acc[c].r1 >= 0) {
      double k = vqhull_oracle_orient(x[a], y[a], x[r], y[r], x[acc[c].r1], y[acc[c].r1]);
      if (farther(x, y, k, acc[c].r1, k1, b1)) {
        k1 = k;
        b1 = acc[c].r1;
      }
    }
    if (acc[c].r2 >= 0) {
      double k = vqhull_oracle_orient(x[r], y[r], x[b], y[b], x[acc[c].r2], y[acc[c].r2]);
      if (farther(x, y, k, acc[c].r2, k2, b2)) {
        k2 = k;
        b2 = acc[c].r2;
      }
    }
    o1[2 * c] = t1;
    o1[2 * c + 1] = t2;
    t1 += acc[c].n1;
    t2 += acc[c].n2;
  }
#pragma omp taskloop grainsize(1)
  for (int64_t c = 0; c < nch; ++c) {
    int64_t lo = c * grain, len = (lo + grain < m ? lo + grain : m) - lo;
    memcpy(s + o1[2 * c], tmp + lo, (size_t)acc[c].n1 * sizeof(int64_t));
    memcpy(s + (m - o1[2 * c + 1] - acc[c].n2), tmp + lo + (len - acc[c].n2), (size_t)acc[c].n2 * sizeof(int64_t));
  }
  free(o1);
  free(acc);
  free(tmp);
  *n1 = t1;
  *n2 = t2;
  *r1 = b1;
  *r2 = b2;
  return ORACLE_OK;
}

/* Hull(P, a, r, b) into out[0 .. *len) (out has room for m entries): the two
 * recursive calls write into the two ends of out, then the list
 * Hull(S1) ++ [r] ++ Hull(S2) is joined at the front (R7).  S1 and S2 do not
 * contain r, so n1 + 1 + n2 <= m and the join only moves entries forward. */
static int hull_mt_rec(const double* x, const double* y, const int64_t* P, int64_t m, int64_t a, int64_t r,
                       int64_t b, int64_t grain, int64_t* out, int64_t* len) {
  *len = 0;
  if (m <= 1) {
    if (m == 1) out[(*len)++] = P[0];
    return ORACLE_OK;
  }
  int64_t* s = (int64_t*)malloc((size_t)m * sizeof(int64_t));
  if (!s) return ORACLE_ERR_OUT_OF_MEMORY;
  int64_t n1, n2, r1, r2;
  int st = ORACLE_OK, st1 = ORACLE_OK, st2 = ORACLE_OK;
  if (m > 2 * grain) {
    st = split_mt(x, y, P, m, a, r, b, s, grain, &n1, &n2, &r1, &r2);
  } else {
    split(x, y, P, m, a, r, b, s, &n1, &n2, &r1, &r2);
  }
  int64_t len1 = 0, len2 = 0;
  if (st == ORACLE_OK) {
    if (m > grain) {
#pragma omp task shared(st1, len1)
      st1 = hull_mt_rec(x, y, s, n1, a, r1, r, grain, out, &len1);
#pragma omp task shared(st2, len2)
      st2 = hull_mt_rec(x, y, s + (m - n2), n2, r, r2, b, grain, out + (m - n2), &len2);
#pragma omp taskwait
    } else {
      st1 = hull_mt_rec(x, y, s, n1, a, r1, r, grain, out, &len1);
      st2 = hull_mt_rec(x, y, s + (m - n2), n2, r, r2, b, grain, out + (m - n2), &len2);
    }
    st = st1 != ORACLE_OK ? st1 : st2;
  }
  free(s);
  if (st != ORACLE_OK) return st;
  out[len1] = r;
  memmove(out + len1 + 1, out + (m - n2), (size_t)len2 * sizeof(int64_t));
  *len = len1 + 1 + len2;
  return ORACLE_OK;
}

/* R4 over chunks, combined in chunk order with the same strict comparisons,
 * so the first of equal points wins as in the sequential scan. */
static void extremes_mt(const double* x, const double* y, int64_t n, int64_t grain, int64_t* p_out, int64_t* q_out) {
  int64_t nch = (n + grain - 1) / grain;
  int64_t* pq = (int64_t*)malloc((size_t)(2 * nch) * sizeof(int64_t));
  if (!pq) { /* fall back to one scan */
    vqhull_oracle_extremes(x, y, n, p_out, q_out);
    return;
  }
#pragma omp taskloop grainsize(1)
  for (int64_t c = 0; c < nch; ++c) {
    int64_t lo = c * grain, hi = lo + grain < n ? lo + grain : n;
    int64_t p, q; /* the sequential scan over the chunk */
    vqhull_oracle_extremes(x + lo, y + lo, hi - lo, &p, &q);
    pq[2 * c] = lo + p;
    pq[2 * c + 1] = lo + q;
  }
  int64_t p = pq[0], q = pq[1];
  for (int64_t c = 1; c < nch; ++c) {
    int64_t cp = pq[2 * c], cq = pq[2 * c + 1];
    if (x[cp] < x[p] || (x[cp] == x[p] && y[cp] < y[p])) p = cp;
    if (x[cq] > x[q] || (x[cq] == x[q] && y[cq] > y[q])) q = cq;
  }
  free(pq);
  *p_out = p;
  *q_out = q;
}

static int hull_mt_top(const double* x, const double* y, int64_t n, int64_t grain, int64_t* out_idx,
                       int64_t* out_count) {
  int nonfinite = 0;
#pragma omp taskloop grainsize(1) shared(nonfinite)
  for (int64_t c = 0; c < (n + grain - 1) / grain; ++c) {
    int64_t lo = c * grain, hi = lo + grain < n ? lo + grain : n;
    for (int64_t i = lo; i < hi; ++i)
      if (!isfinite(x[i]) || !isfinite(y[i])) {
#pragma omp atomic write
        nonfinite = 1;
      }
  }
  if (nonfinite) return ORACLE_ERR_NONFINITE;
  int64_t p, q;
  extremes_mt(x, y, n, grain, &p, &q);
  out_idx[0] = p;
  *out_count = 1;
  if (p == q) return ORACLE_OK;
  int64_t* all = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int64_t* s = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int64_t* tmp = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int st = ORACLE_ERR_OUT_OF_MEMORY;
  if (all && s && tmp) {
#pragma omp taskloop grainsize(1)
    for (int64_t c = 0; c < (n + grain - 1) / grain; ++c) {
      int64_t lo = c * grain, hi = lo + grain < n ? lo + grain : n;
      for (int64_t i = lo; i < hi; ++i) all[i] = i;
    }
    /* the degenerate triangle (p, q, p) (R2) */
    int64_t n1, n2, r1, r2;
    st = split_mt(x, y, all, n, p, q, p, s, grain, &n1, &n2, &r1, &r2);
    if (st == ORACLE_OK) {
      int64_t len1 = 0, len2 = 0;
      int st1 = ORACLE_OK, st2 = ORACLE_OK;
#pragma omp task shared(st1, len1)
      st1 = hull_mt_rec(x, y, s, n1, p, r1, q, grain, tmp, &len1);
#pragma omp task shared(st2, len2)
      st2 = hull_mt_rec(x, y, s + (n - n2), n2, q, r2, p, grain, tmp + (n - n2), &len2);
#pragma omp taskwait
      st = st1 != ORACLE_OK ? st1 : st2;
      if (st == ORACLE_OK) { /* [p] ++ Hull(S1) ++ [q] ++ Hull(S2) (R7) */
        int64_t k = 1;
        memcpy(out_idx + k, tmp, (size_t)len1 * sizeof(int64_t));
        k += len1;
        out_idx[k++] = q;
        memcpy(out_idx + k, tmp + (n - n2), (size_t)len2 * sizeof(int64_t));
        *out_count = k + len2;
      }
    }
  }
  free(all);
  free(s);
  free(tmp);
  return st;
}

/*
 * Algorithm 1 on all n points with `threads` OpenMP threads (<= 0: the
 * runtime's default); grain as above (<= 0: n / (8 threads), at least 2^18).  Same output as
 * vqhull_oracle_hull.
 */
int vqhull_oracle_hull_mt(const double* x, const double* y, int64_t n, int64_t* out_idx, int64_t* out_count,
                          int threads, int64_t grain) {
  if (n < 0 || !out_count || (n > 0 && (!x || !y || !out_idx))) return ORACLE_ERR_INVALID_ARGUMENT;
  *out_count = 0;
  if (n == 0) return ORACLE_OK;
  if (threads <= 0) threads = omp_get_max_threads();
  if (grain <= 0) { /* about eight chunks per thread over the whole input, at least 2^18 points */
    grain = n / (8 * (int64_t)threads);
    if (grain < ((int64_t)1 << 18)) grain = (int64_t)1 << 18;
  }
  int st = ORACLE_OK;
#pragma omp parallel num_threads(threads)
#pragma omp single
  st = hull_mt_top(x, y, n, grain, out_idx, out_count);
  if (st != ORACLE_OK) *out_count = 0;
  return st;
}
