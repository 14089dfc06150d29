/*
 * Oracle (test infrastructure only): index helpers of the weak-form operator
 * for a periodic tensor-product grid of affine box elements (Sec. 3.1: each
 * element is mapped to the reference cube; for a box of widths h_d the
 * Jacobian is prod h_d/2 and d/dx_d = (2/h_d) d/dxi_d).
 */
#ifndef NSK_ORACLE_GEOM_H
#define NSK_ORACLE_GEOM_H
#include <stdlib.h>
#include "oracle.h"

typedef struct {
  int dim, np, nnode, nf, nvar, nlift;
  int nel[3];
  long E;
  const double* xb[3];
  or_basis b;
} or_geom;

static inline int or_geom_init(or_geom* g, const or_prob* P) {
  if (P->dim < 1 || P->dim > 3 || P->N < 1 || P->N > OR_NMAX) return -1;
  g->dim = P->dim;
  g->np = P->N + 1;
  g->nnode = 1;
  g->nf = 1;
  for (int d = 0; d < g->dim; ++d) g->nnode *= g->np;
  for (int d = 1; d < g->dim; ++d) g->nf *= g->np;
  g->nvar = g->dim + 2;
  g->nlift = g->dim + 1;
  g->E = 1;
  for (int d = 0; d < 3; ++d) {
    g->nel[d] = d < g->dim ? P->nel[d] : 1;
    if (g->nel[d] < 1) return -1;
    g->E *= g->nel[d];
    g->xb[d] = d < g->dim ? P->xb[d] : NULL;
    if (d < g->dim && !g->xb[d]) return -1;
  }
  return or_make_basis(P->N, &g->b);
}

static inline void or_geom_free(or_geom* g) { (void)g; }

/* element index along direction d */
static inline int or_elem_index(const or_geom* g, long e, int d) {
  if (d == 0) return (int)(e % g->nel[0]);
  if (d == 1) return (int)((e / g->nel[0]) % g->nel[1]);
  return (int)(e / ((long)g->nel[0] * g->nel[1]));
}

/* periodic neighbour of element e in direction d, s = -1 or +1 */
static inline long or_neighbor(const or_geom* g, long e, int d, int s) {
  int idx[3] = {or_elem_index(g, e, 0), or_elem_index(g, e, 1), or_elem_index(g, e, 2)};
  idx[d] = (idx[d] + s + g->nel[d]) % g->nel[d];
  return idx[0] + (long)g->nel[0] * (idx[1] + (long)g->nel[1] * idx[2]);
}

static inline double or_width(const or_geom* g, long e, int d) {
  int k = or_elem_index(g, e, d);
  return g->xb[d][k + 1] - g->xb[d][k];
}

/* node on the line in direction d through face node f, at position l */
static inline int or_line_node(const or_geom* g, int d, int f, int l) {
  int idx[3] = {0, 0, 0};
  for (int dd = 0; dd < g->dim; ++dd) {
    if (dd == d) continue;
    idx[dd] = f % g->np;
    f /= g->np;
  }
  idx[d] = l;
  return idx[0] + g->np * (idx[1] + g->np * idx[2]);
}

/* inverse: node n -> (face node f, position i) for direction d */
static inline void or_node_line(const or_geom* g, int n, int d, int* f, int* i) {
  int idx[3] = {0, 0, 0};
  for (int dd = 0; dd < g->dim; ++dd) {
    idx[dd] = n % g->np;
    n /= g->np;
  }
  int ff = 0, mul = 1;
  for (int dd = 0; dd < g->dim; ++dd) {
    if (dd == d) continue;
    ff += idx[dd] * mul;
    mul *= g->np;
  }
  *f = ff;
  *i = idx[d];
}

/* J_e * omega_n: physical quadrature weight of node n of element e */
static inline double or_quad_weight(const or_geom* g, long e, int n) {
  double wq = 1.0;
  for (int d = 0; d < g->dim; ++d) {
    int f, i;
    or_node_line(g, n, d, &f, &i);
    wq *= 0.5 * or_width(g, e, d) * g->b.w[i];
  }
  return wq;
}
#endif
