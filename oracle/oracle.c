/*
 * Plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see oracle.h).
 *
 * Written for obviousness, not speed: every basis value is produced by the literal
 * Cox-de Boor recursion at every quadrature point, every element integral by the naive
 * per-quadrature-point double loop over (a, b), and every CSR slot by binary search.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXP 7            /* functions per axis per element (degree <= 6) */
#define ORC_MAXLOC 343        /* ORC_MAXP^3 */
#define ORC_MAXQ 12

/* ------------------------------------------------------------------------------------ */
/* Gauss-Legendre rule on [-1,1]: Newton iteration on P_n from the three-term recurrence  */
/* (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1}; weights 2 / ((1-x^2) P_n'(x)^2).              */
/* ------------------------------------------------------------------------------------ */
int orc_gauss_legendre(int n, double *x, double *w) {
  if (n < 1 || n > 64 || !x || !w) return 1;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5)), pn = 0.0, pm = 0.0, dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      pn = z;                               /* P_1 */
      pm = 1.0;                             /* P_0 */
      for (int k = 1; k < n; ++k) {
        double pk = ((2.0 * k + 1.0) * z * pn - k * pm) / (k + 1.0);
        pm = pn;
        pn = pk;
      }
      if (n == 1) { pn = z; pm = 1.0; }
      dp = n * (z * pn - pm) / (z * z - 1.0);    /* P_n'(z) */
      double dz = pn / dp;
      z -= dz;
      if (fabs(dz) <= 1e-17) break;
    }
    pn = z; pm = 1.0;
    for (int k = 1; k < n; ++k) {
      double pk = ((2.0 * k + 1.0) * z * pn - k * pm) / (k + 1.0);
      pm = pn;
      pn = pk;
    }
    dp = n * (z * pn - pm) / (z * z - 1.0);
    double wt = 2.0 / ((1.0 - z * z) * dp * dp);
    x[n - 1 - i] = z;  w[n - 1 - i] = wt;      /* ascending order, symmetric pairs */
    x[i] = -z;         w[i] = wt;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
  return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Cox-de Boor recursion taken literally (Sec. 2.1), with 0/0 := 0.  B_{i,0} is the       */
/* half-open indicator of [xi_i, xi_{i+1}); by convention the last non-empty span is also  */
/* closed on the right so that the basis is defined at the end of the patch.               */
/* ------------------------------------------------------------------------------------ */
static double cdb(const double *U, int nk, int i, int p, double xi) {
  if (p == 0) {
    if (U[i] <= xi && xi < U[i + 1]) return 1.0;
    if (xi == U[nk - 1] && U[i] < U[i + 1] && U[i + 1] == U[nk - 1]) return 1.0;
    return 0.0;
  }
  double a = U[i + p] - U[i];
  double b = U[i + p + 1] - U[i + 1];
  double left = 0.0, right = 0.0;
  if (a != 0.0) left = (xi - U[i]) / a * cdb(U, nk, i, p - 1, xi);
  if (b != 0.0) right = (U[i + p + 1] - xi) / b * cdb(U, nk, i + 1, p - 1, xi);
  return left + right;
}

/* First derivative: p/(xi_{i+p}-xi_i) B_{i,p-1} - p/(xi_{i+p+1}-xi_{i+1}) B_{i+1,p-1}.
 * (The paper prints a plus sign between the two terms; the minus sign is the one that
 * differentiates the recursion above, and it is what makes the derivatives sum to zero.) */
static double cdb_der(const double *U, int nk, int i, int p, double xi) {
  if (p == 0) return 0.0;
  double a = U[i + p] - U[i];
  double b = U[i + p + 1] - U[i + 1];
  double d = 0.0;
  if (a != 0.0) d += p / a * cdb(U, nk, i, p - 1, xi);
  if (b != 0.0) d -= p / b * cdb(U, nk, i + 1, p - 1, xi);
  return d;
}

/* Second derivative: the same derivative formula applied once more, to the first derivatives of
 * the two degree p-1 functions. */
static double cdb_der2(const double *U, int nk, int i, int p, double xi) {
  if (p <= 1) return 0.0;
  double a = U[i + p] - U[i];
  double b = U[i + p + 1] - U[i + 1];
  double d = 0.0;
  if (a != 0.0) d += p / a * cdb_der(U, nk, i, p - 1, xi);
  if (b != 0.0) d -= p / b * cdb_der(U, nk, i + 1, p - 1, xi);
  return d;
}

/* Third derivative: the derivative formula applied to the second derivatives of the two degree p-1
 * functions. */
static double cdb_der3(const double *U, int nk, int i, int p, double xi) {
  if (p <= 2) return 0.0;
  double a = U[i + p] - U[i];
  double b = U[i + p + 1] - U[i + 1];
  double d = 0.0;
  if (a != 0.0) d += p / a * cdb_der2(U, nk, i, p - 1, xi);
  if (b != 0.0) d -= p / b * cdb_der2(U, nk, i + 1, p - 1, xi);
  return d;
}

int orc_basis_1d_d3(int p, const double *U, int nk, int i, double xi, double *d3) {
  if (p < 0 || !U || !d3 || i < 0 || i + p + 1 >= nk) return 1;
  *d3 = cdb_der3(U, nk, i, p, xi);
  return 0;
}

int orc_basis_1d_d2(int p, const double *U, int nk, int i, double xi, double *d2) {
  if (p < 0 || !U || !d2 || i < 0 || i + p + 1 >= nk) return 1;
  *d2 = cdb_der2(U, nk, i, p, xi);
  return 0;
}

int orc_basis_1d(int p, const double *U, int nk, int i, double xi, double *val, double *der) {
  if (p < 0 || !U || i < 0 || i + p + 1 >= nk) return 1;
  if (val) *val = cdb(U, nk, i, p, xi);
  if (der) *der = cdb_der(U, nk, i, p, xi);
  return 0;
}

/* Algorithm 2: left-most and right-most indices of the functions whose support overlaps
 * the support of function i (clamped to the valid range). */
int orc_stencil(int p, const double *U, int nk, int i, int *l, int *r) {
  int n = nk - p - 1;
  if (i < 0 || i >= n) return 1;
  int j = i;
  while (j + 1 < nk && U[j] == U[j + 1]) j++;
  int ll = j - p;
  j = i + p + 1;
  while (j - 1 >= 0 && U[j] == U[j - 1]) j--;
  int rr = j - 1;
  if (ll < 0) ll = 0;
  if (rr > n - 1) rr = n - 1;
  *l = ll;
  *r = rr;
  return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Problem layout                                                                        */
/* ------------------------------------------------------------------------------------ */
typedef struct {
  int dim;
  int p[3], n[3], nq[3], ne[3];
  int *span[3];            /* span index s of each element: functions s-p..s are nonzero */
  int per[3];              /* periodic axis: continuity k + 1 across the seam; 0: not periodic */
  const double *kn[3];     /* knots in use (the unclamped copy on a periodic axis) */
  double *ukn[3];          /* owned unclamped copy, or NULL */
  double gx[3][ORC_MAXQ], gw[3][ORC_MAXQ];
  int64_t N, E;
} layout;

static void lay_free(layout *L) {
  for (int d = 0; d < 3; ++d) {
    free(L->span[d]);
    free(L->ukn[d]);
  }
}

/* ------------------------------------------------------------------------------------ */
/* Periodicity (Sec. 2.4): unclamp an open knot vector for C^k continuity across the seam  */
/* by redefining k+1 knots at each end (eq:unclamp-left, eq:unclamp-right), in place.       */
/* n is the index of the last basis function of the open vector (m = n + p + 1).           */
/* ------------------------------------------------------------------------------------ */
int orc_unclamp(int n, int p, int k, double *U) {
  if (k < 0 || k > p - 1 || n < p) return 1;
  int m = n + p + 1;
  for (int i = 0; i <= k; ++i) U[k - i] = U[p] - U[n + 1] + U[n - i];
  for (int i = 0; i <= k; ++i) U[m - k + i] = U[n + 1] - U[p] + U[p + i + 1];
  return 0;
}

/* eq:map-wrap: global index of a basis function on a periodic axis with nper functions */
static int wrap(int i, int nper) {
  int q = (int)floor((double)i / (double)nper);
  return i - nper * q;
}

/* global index of local function a (0..p) of the element with span s along axis d */
static int fn_index(const layout *L, int d, int s, int a) {
  int i = s - L->p[d] + a;
  return L->per[d] ? wrap(i, L->n[d]) : i;
}

/* sorted distinct functions sharing an element with function i along axis d */
static int axis_neighbors(const layout *L, int d, int i, int *out) {
  int c = 0;
  for (int e = 0; e < L->ne[d]; ++e) {
    int s = L->span[d][e], has = 0;
    for (int a = 0; a <= L->p[d]; ++a) has |= fn_index(L, d, s, a) == i;
    if (!has) continue;
    for (int b = 0; b <= L->p[d]; ++b) {
      int j = fn_index(L, d, s, b), k = 0;
      while (k < c && out[k] != j) ++k;
      if (k == c) out[c++] = j;
    }
  }
  for (int x = 1; x < c; ++x)     /* insertion sort */
    for (int y = x; y > 0 && out[y - 1] > out[y]; --y) {
      int t = out[y]; out[y] = out[y - 1]; out[y - 1] = t;
    }
  return c;
}

static int lay_init(const orc_problem *pb, layout *L) {
  memset(L, 0, sizeof(*L));
  if (!pb || pb->dim < 1 || pb->dim > 3) return 1;
  L->dim = pb->dim;
  L->N = 1;
  L->E = 1;
  for (int d = 0; d < 3; ++d) {
    if (d >= pb->dim) {
      L->p[d] = 0; L->n[d] = 1; L->nq[d] = 1; L->ne[d] = 1;
      L->span[d] = (int *)calloc(1, sizeof(int));
      L->gx[d][0] = 0.0; L->gw[d][0] = 2.0;
      continue;
    }
    int p = pb->degree[d], nk = pb->nknots[d];
    const double *U = pb->knots[d];
    if (p < 1 || p > ORC_MAXP - 1 || !U || nk < 2 * p + 2) { lay_free(L); return 1; }
    for (int k = 0; k + 1 < nk; ++k)
      if (!(U[k] <= U[k + 1])) { lay_free(L); return 1; }
    for (int k = 0; k < p; ++k)
      if (U[k] != U[k + 1] || U[nk - 1 - k] != U[nk - 2 - k]) { lay_free(L); return 1; }
    L->p[d] = p;
    L->n[d] = nk - p - 1;
    L->kn[d] = U;
    L->per[d] = pb->periodic[d];
    if (L->per[d]) {
      int k = L->per[d] - 1;
      /* the seam must not be a Dirichlet face, and n - k >= 2p + 1 keeps the wrapped stencil distinct */
      if (k < 0 || k > p - 1 || ((pb->dirichlet_mask >> (2 * d)) & 3u) || L->n[d] - 1 - k < 2 * p + 1) {
        lay_free(L);
        return 1;
      }
      L->ukn[d] = (double *)malloc(sizeof(double) * nk);
      memcpy(L->ukn[d], U, sizeof(double) * nk);
      orc_unclamp(L->n[d] - 1, p, k, L->ukn[d]);
      L->kn[d] = L->ukn[d];
    }
    L->nq[d] = pb->nquad[d] > 0 ? pb->nquad[d] : p + 1;
    if (L->nq[d] > ORC_MAXQ) { lay_free(L); return 1; }
    orc_gauss_legendre(L->nq[d], L->gx[d], L->gw[d]);
    L->span[d] = (int *)malloc(sizeof(int) * nk);
    int ne = 0;
    for (int s = p; s < L->n[d]; ++s)
      if (U[s] < U[s + 1]) L->span[d][ne++] = s;
    if (ne == 0) { lay_free(L); return 1; }
    L->ne[d] = ne;
    if (L->per[d]) L->n[d] -= L->per[d];   /* n - k distinct functions (n: index of the last) */
  }
  for (int d = 0; d < 3; ++d) { L->N *= L->n[d]; L->E *= L->ne[d]; }
  if (pb->weights)
    for (int64_t A = 0; A < L->N; ++A)
      if (!(pb->weights[A] > 0.0)) { lay_free(L); return 1; }
  if (pb->kappa_mode < 0 || pb->kappa_mode > 2) { lay_free(L); return 1; }
  if (pb->kappa_mode != 0 && !pb->kappa) { lay_free(L); return 1; }
  return 0;
}

static int is_dirichlet(const orc_problem *pb, const layout *L, int64_t A) {
  int64_t i[3] = {A % L->n[0], (A / L->n[0]) % L->n[1], A / ((int64_t)L->n[0] * L->n[1])};
  for (int d = 0; d < pb->dim; ++d) {
    if ((pb->dirichlet_mask >> (2 * d)) & 1u)
      if (i[d] == 0) return 1;
    if ((pb->dirichlet_mask >> (2 * d + 1)) & 1u)
      if (i[d] == L->n[d] - 1) return 1;
  }
  return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Shape functions at one quadrature point of one element (ShapeFuns in Algorithm 3)     */
/* ------------------------------------------------------------------------------------ */
typedef struct {
  int nloc;
  int64_t A[ORC_MAXLOC];     /* global index of each local function (a0 fastest) */
  double N[ORC_MAXLOC];      /* rational basis values */
  double dN[ORC_MAXLOC][3];  /* spatial gradients */
  double x[3];
  double W;                  /* quadrature weight * span factors * det J */
  double u, gu[3], kap, f;
} qpoint;

static int eval_qp(const orc_problem *pb, const layout *L, const int e[3], const int g[3],
                   const double *U, qpoint *q) {
  int dim = L->dim;
  double B[3][ORC_MAXP], dB[3][ORC_MAXP], wq = 1.0;
  for (int d = 0; d < 3; ++d) {
    if (d >= dim) { B[d][0] = 1.0; dB[d][0] = 0.0; continue; }
    const double *K = L->kn[d];
    int s = L->span[d][e[d]], p = L->p[d];
    double a = K[s], b = K[s + 1];
    double xi = 0.5 * ((a + b) + (b - a) * L->gx[d][g[d]]);
    wq *= L->gw[d][g[d]] * 0.5 * (b - a);
    for (int k = 0; k <= p; ++k)
      orc_basis_1d(p, K, pb->nknots[d], s - p + k, xi, &B[d][k], &dB[d][k]);
  }
  int P0 = L->p[0] + 1, P1 = L->p[1] + 1, P2 = L->p[2] + 1;
  int nloc = P0 * P1 * P2;
  q->nloc = nloc;
  double M[ORC_MAXLOC], dM[ORC_MAXLOC][3];
  for (int a2 = 0; a2 < P2; ++a2)
    for (int a1 = 0; a1 < P1; ++a1)
      for (int a0 = 0; a0 < P0; ++a0) {
        int a = a0 + P0 * (a1 + P1 * a2);
        int64_t i0 = fn_index(L, 0, L->span[0][e[0]], a0);
        int64_t i1 = fn_index(L, 1, L->span[1][e[1]], a1);
        int64_t i2 = fn_index(L, 2, L->span[2][e[2]], a2);
        q->A[a] = i0 + (int64_t)L->n[0] * (i1 + (int64_t)L->n[1] * i2);
        M[a] = B[0][a0] * B[1][a1] * B[2][a2];
        dM[a][0] = dB[0][a0] * B[1][a1] * B[2][a2];
        dM[a][1] = B[0][a0] * dB[1][a1] * B[2][a2];
        dM[a][2] = B[0][a0] * B[1][a1] * dB[2][a2];
      }
  /* rational basis (eq:rational) and parametric derivatives (eq:drational) */
  double dNp[ORC_MAXLOC][3];
  if (pb->weights) {
    double w = 0.0, dw[3] = {0, 0, 0};
    for (int a = 0; a < nloc; ++a) {
      double wa = pb->weights[q->A[a]];
      w += wa * M[a];
      for (int al = 0; al < 3; ++al) dw[al] += wa * dM[a][al];
    }
    for (int a = 0; a < nloc; ++a) {
      double wa = pb->weights[q->A[a]];
      q->N[a] = wa * M[a] / w;
      for (int al = 0; al < 3; ++al) dNp[a][al] = (wa * dM[a][al] - q->N[a] * dw[al]) / w;
    }
  } else {
    for (int a = 0; a < nloc; ++a) {
      q->N[a] = M[a];
      for (int al = 0; al < 3; ++al) dNp[a][al] = dM[a][al];
    }
  }
  /* geometry: x_{i,alpha} = sum_A x_{A,i} N_{A,alpha}; inverse via eq:identity */
  double J[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  double xi_phys[3] = {0, 0, 0};
  if (pb->ctrl) {
    for (int i = 0; i < dim; ++i)
      for (int al = 0; al < dim; ++al) J[i][al] = 0.0;
    for (int a = 0; a < nloc; ++a)
      for (int i = 0; i < dim; ++i) {
        double xa = pb->ctrl[q->A[a] * dim + i];
        xi_phys[i] += xa * q->N[a];
        for (int al = 0; al < dim; ++al) J[i][al] += xa * dNp[a][al];
      }
  } else {
    for (int d = 0; d < dim; ++d) {
      const double *K = L->kn[d];
      int s = L->span[d][e[d]];
      xi_phys[d] = 0.5 * ((K[s] + K[s + 1]) + (K[s + 1] - K[s]) * L->gx[d][g[d]]);
    }
  }
  double det, Ji[3][3];
  if (dim == 1) {
    det = J[0][0];
    Ji[0][0] = 1.0 / det;
  } else if (dim == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    Ji[0][0] = J[1][1] / det;  Ji[0][1] = -J[0][1] / det;
    Ji[1][0] = -J[1][0] / det; Ji[1][1] = J[0][0] / det;
  } else {
    det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
        - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
        + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  }
  if (!(det > 0.0)) return 2;
  /* Ji[alpha][i] = d xi_alpha / d x_i ; spatial gradient N_{A,i} = N_{A,alpha} xi_{alpha,i} */
  for (int a = 0; a < nloc; ++a)
    for (int i = 0; i < 3; ++i) {
      double s = 0.0;
      if (i < dim)
        for (int al = 0; al < dim; ++al) s += dNp[a][al] * Ji[al][i];
      q->dN[a][i] = s;
    }
  for (int i = 0; i < 3; ++i) q->x[i] = xi_phys[i];
  q->W = wq * det;
  /* state, coefficient and source at the point */
  q->u = 0.0;
  q->gu[0] = q->gu[1] = q->gu[2] = 0.0;
  for (int a = 0; a < nloc; ++a) {
    double Ua = U ? U[q->A[a]] : 0.0;
    q->u += Ua * q->N[a];
    for (int i = 0; i < 3; ++i) q->gu[i] += Ua * q->dN[a][i];
  }
  if (pb->kappa_mode == 0) {
    q->kap = 1.0;
  } else if (pb->kappa_mode == 1) {
    q->kap = 0.0;
    for (int a = 0; a < nloc; ++a) q->kap += pb->kappa[q->A[a]] * q->N[a];
  } else {
    int64_t ee = e[0] + (int64_t)L->ne[0] * (e[1] + (int64_t)L->ne[1] * e[2]);
    q->kap = pb->kappa[ee];
  }
  q->f = 0.0;
  if (pb->source)
    for (int a = 0; a < nloc; ++a) q->f += pb->source[q->A[a]] * q->N[a];
  return 0;
}

static void elem_multi(const layout *L, int64_t e, int em[3]) {
  em[0] = (int)(e % L->ne[0]);
  em[1] = (int)((e / L->ne[0]) % L->ne[1]);
  em[2] = (int)(e / ((int64_t)L->ne[0] * L->ne[1]));
}

static void qp_multi(const layout *L, int g, int gm[3]) {
  gm[0] = g % L->nq[0];
  gm[1] = (g / L->nq[0]) % L->nq[1];
  gm[2] = g / (L->nq[0] * L->nq[1]);
}

/* ------------------------------------------------------------------------------------ */
/* Sizes and the CSR pattern (Algorithm 2 per axis, tensor product, sorted columns)      */
/* ------------------------------------------------------------------------------------ */
int orc_sizes(const orc_problem *pb, int64_t *ndof, int64_t *nelem, int64_t *nnz) {
  layout L;
  if (lay_init(pb, &L)) return 1;
  int64_t cnt = 0;
  for (int64_t A = 0; A < L.N; ++A) {
    int64_t i[3] = {A % L.n[0], (A / L.n[0]) % L.n[1], A / ((int64_t)L.n[0] * L.n[1])};
    int64_t w = 1;
    for (int d = 0; d < pb->dim; ++d) {
      if (L.per[d]) {
        int nb[2 * ORC_MAXP + 8];
        w *= axis_neighbors(&L, d, (int)i[d], nb);
      } else {
        int l, r;
        orc_stencil(L.p[d], pb->knots[d], pb->nknots[d], (int)i[d], &l, &r);
        w *= (r - l + 1);
      }
    }
    cnt += w;
  }
  if (ndof) *ndof = L.N;
  if (nelem) *nelem = L.E;
  if (nnz) *nnz = cnt;
  lay_free(&L);
  return 0;
}

int orc_csr_pattern(const orc_problem *pb, int64_t *row_ptr, int32_t *col_idx) {
  layout L;
  if (lay_init(pb, &L)) return 1;
  int64_t pos = 0;
  row_ptr[0] = 0;
  for (int64_t A = 0; A < L.N; ++A) {
    int64_t i[3] = {A % L.n[0], (A / L.n[0]) % L.n[1], A / ((int64_t)L.n[0] * L.n[1])};
    /* per axis, the sorted functions sharing an element with i[d] (Algorithm 2 on an open axis) */
    int nb[3][2 * ORC_MAXP + 8], c[3] = {1, 1, 1};
    nb[1][0] = nb[2][0] = 0;
    for (int d = 0; d < pb->dim; ++d) {
      if (L.per[d]) {
        c[d] = axis_neighbors(&L, d, (int)i[d], nb[d]);
      } else {
        int l, r;
        orc_stencil(L.p[d], pb->knots[d], pb->nknots[d], (int)i[d], &l, &r);
        c[d] = r - l + 1;
        for (int j = l; j <= r; ++j) nb[d][j - l] = j;
      }
    }
    for (int x2 = 0; x2 < c[2]; ++x2)
      for (int x1 = 0; x1 < c[1]; ++x1)
        for (int x0 = 0; x0 < c[0]; ++x0)
          col_idx[pos++] = (int32_t)(nb[0][x0] + (int64_t)L.n[0] * (nb[1][x1] + (int64_t)L.n[1] * nb[2][x2]));
    row_ptr[A + 1] = pos;
  }
  lay_free(&L);
  return 0;
}

static int64_t csr_find(const int64_t *row_ptr, const int32_t *col_idx, int64_t A, int64_t B) {
  int64_t lo = row_ptr[A], hi = row_ptr[A + 1] - 1;
  while (lo <= hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (col_idx[mid] == B) return mid;
    if (col_idx[mid] < B) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

/* ------------------------------------------------------------------------------------ */
/* Integrands (eq:residual, eq:jacobian, with kappa and an optional source f)            */
/*   R_a += W ( kappa grad N_a . grad u - N_a (lambda e^u + f) )                          */
/*   K_ab += W ( kappa grad N_a . grad N_b - lambda e^u N_a N_b )                         */
/* ------------------------------------------------------------------------------------ */
static double res_term(const orc_problem *pb, const qpoint *q, int a) {
  double g = q->dN[a][0] * q->gu[0] + q->dN[a][1] * q->gu[1] + q->dN[a][2] * q->gu[2];
  return q->W * (q->kap * g - q->N[a] * (pb->lambda * exp(q->u) + q->f));
}

static double jac_term(const orc_problem *pb, const qpoint *q, int a, int b) {
  double g = q->dN[a][0] * q->dN[b][0] + q->dN[a][1] * q->dN[b][1] + q->dN[a][2] * q->dN[b][2];
  return q->W * (q->kap * g - pb->lambda * exp(q->u) * q->N[a] * q->N[b]);
}

int orc_residual(const orc_problem *pb, const double *U, double *R) {
  layout L;
  if (lay_init(pb, &L)) return 1;
  memset(R, 0, sizeof(double) * L.N);
  qpoint *q = (qpoint *)malloc(sizeof(qpoint));
  int nqe = L.nq[0] * L.nq[1] * L.nq[2], rc = 0;
  for (int64_t e = 0; e < L.E && !rc; ++e) {
    int em[3], gm[3];
    elem_multi(&L, e, em);
    for (int g = 0; g < nqe && !rc; ++g) {
      qp_multi(&L, g, gm);
      if ((rc = eval_qp(pb, &L, em, gm, U, q))) break;
      for (int a = 0; a < q->nloc; ++a) R[q->A[a]] += res_term(pb, q, a);
    }
  }
  for (int64_t A = 0; A < L.N; ++A)
    if (is_dirichlet(pb, &L, A)) R[A] = U[A];
  free(q);
  lay_free(&L);
  return rc;
}

static void jac_bc_rows(const orc_problem *pb, const layout *L, const int64_t *row_ptr,
                        const int32_t *col_idx, double *vals, int64_t A, double *rowvals) {
  int64_t base = row_ptr[A];
  double *v = rowvals ? rowvals : vals + base;
  if (is_dirichlet(pb, L, A)) {
    for (int64_t k = base; k < row_ptr[A + 1]; ++k) v[k - base] = (col_idx[k] == A) ? 1.0 : 0.0;
  } else {
    for (int64_t k = base; k < row_ptr[A + 1]; ++k)
      if (is_dirichlet(pb, L, col_idx[k])) v[k - base] = 0.0;
  }
}

int orc_jacobian(const orc_problem *pb, const double *U, const int64_t *row_ptr,
                 const int32_t *col_idx, double *vals) {
  layout L;
  if (lay_init(pb, &L)) return 1;
  memset(vals, 0, sizeof(double) * row_ptr[L.N]);
  qpoint *q = (qpoint *)malloc(sizeof(qpoint));
  int nqe = L.nq[0] * L.nq[1] * L.nq[2], rc = 0;
  for (int64_t e = 0; e < L.E && !rc; ++e) {
    int em[3], gm[3];
    elem_multi(&L, e, em);
    for (int g = 0; g < nqe && !rc; ++g) {
      qp_multi(&L, g, gm);
      if ((rc = eval_qp(pb, &L, em, gm, U, q))) break;
      for (int a = 0; a < q->nloc; ++a)
        for (int b = 0; b < q->nloc; ++b) {
          int64_t k = csr_find(row_ptr, col_idx, q->A[a], q->A[b]);
          if (k < 0) { rc = 3; break; }
          vals[k] += jac_term(pb, q, a, b);
        }
    }
  }
  if (!rc)
    for (int64_t A = 0; A < L.N; ++A) jac_bc_rows(pb, &L, row_ptr, col_idx, vals, A, NULL);
  free(q);
  lay_free(&L);
  return rc;
}

/* ------------------------------------------------------------------------------------ */
/* Local numerical differentiation (Sec. 2.8, eq:fdjac): at each quadrature point q of     */
/* element e, column k of dF_q/dU_e is (F_q(U_e + delta e_k) - F_q(U_e)) / delta, where     */
/* F_q[a] is the point's contribution to the element residual and                           */
/* delta = eta sqrt(1 + ||U_e||_2); eta <= 0 selects the default sqrt(machine epsilon).     */
/* The element matrices are summed into the CSR values, then the Dirichlet rows and columns  */
/* are treated as for the explicit Jacobian.                                                */
/* ------------------------------------------------------------------------------------ */
static void state_at(const qpoint *q, const double *Ue, qpoint *out) {
  *out = *q;
  out->u = 0.0;
  out->gu[0] = out->gu[1] = out->gu[2] = 0.0;
  for (int a = 0; a < q->nloc; ++a) {
    out->u += Ue[a] * q->N[a];
    for (int i = 0; i < 3; ++i) out->gu[i] += Ue[a] * q->dN[a][i];
  }
}

int orc_jacobian_nd(const orc_problem *pb, const double *U, const int64_t *row_ptr,
                    const int32_t *col_idx, double eta, double *vals) {
  layout L;
  if (lay_init(pb, &L)) return 1;
  if (!(eta > 0.0)) eta = sqrt(2.220446049250313e-16);
  memset(vals, 0, sizeof(double) * row_ptr[L.N]);
  qpoint *q = (qpoint *)malloc(3 * sizeof(qpoint));
  qpoint *qb = q + 1, *qk = q + 2;
  double *Ue = (double *)malloc(sizeof(double) * ORC_MAXLOC);
  double *F0 = (double *)malloc(sizeof(double) * ORC_MAXLOC);
  double *Ke = (double *)malloc(sizeof(double) * ORC_MAXLOC * ORC_MAXLOC);
  int nqe = L.nq[0] * L.nq[1] * L.nq[2], rc = 0;
  for (int64_t e = 0; e < L.E && !rc; ++e) {
    int em[3], gm[3];
    elem_multi(&L, e, em);
    int nloc = 0;
    memset(Ke, 0, sizeof(double) * ORC_MAXLOC * ORC_MAXLOC);
    double delta = 0.0;
    for (int g = 0; g < nqe && !rc; ++g) {
      qp_multi(&L, g, gm);
      if ((rc = eval_qp(pb, &L, em, gm, U, q))) break;
      nloc = q->nloc;
      if (g == 0) {
        double nrm = 0.0;
        for (int a = 0; a < nloc; ++a) {
          Ue[a] = U[q->A[a]];
          nrm += Ue[a] * Ue[a];
        }
        delta = eta * sqrt(1.0 + sqrt(nrm));
      }
      state_at(q, Ue, qb);
      for (int a = 0; a < nloc; ++a) F0[a] = res_term(pb, qb, a);
      for (int k = 0; k < nloc; ++k) {
        double keep = Ue[k];
        Ue[k] = keep + delta;
        state_at(q, Ue, qk);
        Ue[k] = keep;
        for (int a = 0; a < nloc; ++a) Ke[a * nloc + k] += (res_term(pb, qk, a) - F0[a]) / delta;
      }
    }
    for (int a = 0; a < nloc && !rc; ++a)
      for (int k = 0; k < nloc; ++k) {
        int64_t s = csr_find(row_ptr, col_idx, q->A[a], q->A[k]);
        if (s < 0) { rc = 3; break; }
        vals[s] += Ke[a * nloc + k];
      }
  }
  if (!rc)
    for (int64_t A = 0; A < L.N; ++A) jac_bc_rows(pb, &L, row_ptr, col_idx, vals, A, NULL);
  free(Ke);
  free(F0);
  free(Ue);
  free(q);
  lay_free(&L);
  return rc;
}

/* elements of one axis whose span contains function i */
static int elems_of_fn(const layout *L, int d, int i, int *out) {
  int c = 0;
  for (int e = 0; e < L->ne[d]; ++e) {
    int s = L->span[d][e], has = 0;
    for (int a = 0; a <= L->p[d]; ++a) has |= fn_index(L, d, s, a) == i;
    if (has) out[c++] = e;
  }
  return c;
}

static int row_contrib(const orc_problem *pb, const layout *L, const double *U, int64_t A,
                       int want_jac, const int64_t *row_ptr, const int32_t *col_idx,
                       double *rowvals, double *rval) {
  int64_t i[3] = {A % L->n[0], (A / L->n[0]) % L->n[1], A / ((int64_t)L->n[0] * L->n[1])};
  int el[3][ORC_MAXP + 8], ce[3];
  for (int d = 0; d < 3; ++d) {
    if (d >= L->dim) { el[d][0] = 0; ce[d] = 1; continue; }
    ce[d] = elems_of_fn(L, d, (int)i[d], el[d]);
  }
  int64_t len = want_jac ? row_ptr[A + 1] - row_ptr[A] : 0;
  if (want_jac) memset(rowvals, 0, sizeof(double) * len);
  double r = 0.0;
  qpoint *q = (qpoint *)malloc(sizeof(qpoint));
  int nqe = L->nq[0] * L->nq[1] * L->nq[2], rc = 0;
  for (int c2 = 0; c2 < ce[2] && !rc; ++c2)
    for (int c1 = 0; c1 < ce[1] && !rc; ++c1)
      for (int c0 = 0; c0 < ce[0] && !rc; ++c0) {
        int em[3] = {el[0][c0], el[1][c1], el[2][c2]}, gm[3];
        for (int g = 0; g < nqe && !rc; ++g) {
          qp_multi(L, g, gm);
          if ((rc = eval_qp(pb, L, em, gm, U, q))) break;
          int a = -1;
          for (int k = 0; k < q->nloc; ++k)
            if (q->A[k] == A) a = k;
          if (a < 0) continue;
          r += res_term(pb, q, a);
          if (want_jac)
            for (int b = 0; b < q->nloc; ++b) {
              int64_t k = csr_find(row_ptr, col_idx, A, q->A[b]);
              if (k < 0) { rc = 3; break; }
              rowvals[k - row_ptr[A]] += jac_term(pb, q, a, b);
            }
        }
      }
  free(q);
  if (rc) return rc;
  if (want_jac) jac_bc_rows(pb, L, row_ptr, col_idx, NULL, A, rowvals);
  if (rval) *rval = is_dirichlet(pb, L, A) ? U[A] : r;
  return 0;
}

int orc_residual_rows(const orc_problem *pb, const double *U, const int64_t *rows, int64_t nrows,
                      double *out) {
  layout L;
  if (lay_init(pb, &L)) return 1;
  int rc = 0;
  for (int64_t k = 0; k < nrows && !rc; ++k) {
    if (rows[k] < 0 || rows[k] >= L.N) { rc = 1; break; }
    rc = row_contrib(pb, &L, U, rows[k], 0, NULL, NULL, NULL, &out[k]);
  }
  lay_free(&L);
  return rc;
}

int orc_jacobian_rows(const orc_problem *pb, const double *U, const int64_t *rows, int64_t nrows,
                      const int64_t *row_ptr, const int32_t *col_idx, double *out) {
  layout L;
  if (lay_init(pb, &L)) return 1;
  int rc = 0;
  int64_t pos = 0;
  for (int64_t k = 0; k < nrows && !rc; ++k) {
    if (rows[k] < 0 || rows[k] >= L.N) { rc = 1; break; }
    rc = row_contrib(pb, &L, U, rows[k], 1, row_ptr, col_idx, out + pos, NULL);
    pos += row_ptr[rows[k] + 1] - row_ptr[rows[k]];
  }
  lay_free(&L);
  return rc;
}

int orc_element_matrix(const orc_problem *pb, const double *U, int64_t elem, double *Ke, double *Re) {
  layout L;
  if (lay_init(pb, &L)) return 1;
  if (elem < 0 || elem >= L.E) { lay_free(&L); return 1; }
  qpoint *q = (qpoint *)malloc(sizeof(qpoint));
  int em[3], gm[3], nqe = L.nq[0] * L.nq[1] * L.nq[2], rc = 0;
  int nloc = (L.p[0] + 1) * (L.p[1] + 1) * (L.p[2] + 1);
  if (Ke) memset(Ke, 0, sizeof(double) * nloc * nloc);
  if (Re) memset(Re, 0, sizeof(double) * nloc);
  elem_multi(&L, elem, em);
  for (int g = 0; g < nqe && !rc; ++g) {
    qp_multi(&L, g, gm);
    if ((rc = eval_qp(pb, &L, em, gm, U, q))) break;
    for (int a = 0; a < nloc; ++a) {
      if (Re) Re[a] += res_term(pb, q, a);
      if (Ke)
        for (int b = 0; b < nloc; ++b) Ke[a * nloc + b] += jac_term(pb, q, a, b);
    }
  }
  free(q);
  lay_free(&L);
  return rc;
}

int orc_jacobian_elements(const orc_problem *pb, const double *U, const int64_t *elems, int64_t n,
                          const int64_t *row_ptr, const int32_t *col_idx, double *vals) {
  layout L;
  if (lay_init(pb, &L)) return 1;
  qpoint *q = (qpoint *)malloc(sizeof(qpoint));
  int nqe = L.nq[0] * L.nq[1] * L.nq[2], rc = 0;
  for (int64_t k = 0; k < n && !rc; ++k) {
    int em[3], gm[3];
    if (elems[k] < 0 || elems[k] >= L.E) { rc = 1; break; }
    elem_multi(&L, elems[k], em);
    for (int g = 0; g < nqe && !rc; ++g) {
      qp_multi(&L, g, gm);
      if ((rc = eval_qp(pb, &L, em, gm, U, q))) break;
      for (int a = 0; a < q->nloc; ++a)
        for (int b = 0; b < q->nloc; ++b) {
          int64_t s = csr_find(row_ptr, col_idx, q->A[a], q->A[b]);
          if (s < 0) { rc = 3; break; }
          vals[s] += jac_term(pb, q, a, b);
        }
    }
  }
  free(q);
  lay_free(&L);
  return rc;
}

int orc_spmv(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const double *vals,
             const double *x, double *y) {
  for (int64_t A = 0; A < n; ++A) {
    double s = 0.0;
    for (int64_t k = row_ptr[A]; k < row_ptr[A + 1]; ++k) s += vals[k] * x[col_idx[k]];
    y[A] = s;
  }
  return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Linear solvers for Newton: banded LU without pivoting (the Jacobian is symmetric      */
/* positive definite on the lower solution branch) and Jacobi-preconditioned CG.          */
/* ------------------------------------------------------------------------------------ */
static int banded_solve(int64_t N, const int64_t *rp, const int32_t *ci, const double *v,
                        const double *rhs, double *x) {
  int64_t bw = 0;
  for (int64_t A = 0; A < N; ++A)
    for (int64_t k = rp[A]; k < rp[A + 1]; ++k) {
      int64_t d = ci[k] - A;
      if (d < 0) d = -d;
      if (d > bw) bw = d;
    }
  int64_t W = 2 * bw + 1;
  if (N <= 0 || N > INT64_MAX / W) return 2;
  double *band = (double *)calloc((size_t)(N * W), sizeof(double));
  if (!band) return 2;
#define BAND(i, j) band[(i) * W + ((j) - (i) + bw)]
  for (int64_t A = 0; A < N; ++A)
    for (int64_t k = rp[A]; k < rp[A + 1]; ++k) BAND(A, (int64_t)ci[k]) = v[k];
  for (int64_t k = 0; k < N; ++k) {
    double piv = BAND(k, k);
    if (piv == 0.0) { free(band); return 4; }
    int64_t iend = k + bw < N - 1 ? k + bw : N - 1;
    for (int64_t i = k + 1; i <= iend; ++i) {
      double l = BAND(i, k) / piv;
      if (l == 0.0) continue;
      BAND(i, k) = l;
      for (int64_t j = k + 1; j <= iend; ++j) BAND(i, j) -= l * BAND(k, j);
    }
  }
  for (int64_t i = 0; i < N; ++i) {
    double s = rhs[i];
    int64_t j0 = i - bw > 0 ? i - bw : 0;
    for (int64_t j = j0; j < i; ++j) s -= BAND(i, j) * x[j];
    x[i] = s;
  }
  for (int64_t i = N - 1; i >= 0; --i) {
    double s = x[i];
    int64_t j1 = i + bw < N - 1 ? i + bw : N - 1;
    for (int64_t j = i + 1; j <= j1; ++j) s -= BAND(i, j) * x[j];
    x[i] = s / BAND(i, i);
  }
#undef BAND
  free(band);
  return 0;
}

static int cg_solve(int64_t N, const int64_t *rp, const int32_t *ci, const double *v,
                    const double *b, double *x, double rtol, int maxit) {
  double *r = (double *)malloc(sizeof(double) * N), *z = (double *)malloc(sizeof(double) * N);
  double *p = (double *)malloc(sizeof(double) * N), *q = (double *)malloc(sizeof(double) * N);
  double *dinv = (double *)malloc(sizeof(double) * N);
  for (int64_t A = 0; A < N; ++A) {
    double d = 1.0;
    for (int64_t k = rp[A]; k < rp[A + 1]; ++k)
      if (ci[k] == A) d = v[k];
    dinv[A] = 1.0 / d;
    x[A] = 0.0;
    r[A] = b[A];
  }
  double bn = 0.0, rz = 0.0;
  for (int64_t A = 0; A < N; ++A) {
    z[A] = dinv[A] * r[A];
    p[A] = z[A];
    bn += b[A] * b[A];
    rz += r[A] * z[A];
  }
  bn = sqrt(bn);
  int rc = 4;
  for (int it = 0; it < maxit; ++it) {
    orc_spmv(N, rp, ci, v, p, q);
    double pq = 0.0;
    for (int64_t A = 0; A < N; ++A) pq += p[A] * q[A];
    double al = rz / pq, rn = 0.0;
    for (int64_t A = 0; A < N; ++A) {
      x[A] += al * p[A];
      r[A] -= al * q[A];
      rn += r[A] * r[A];
    }
    if (sqrt(rn) <= rtol * bn) { rc = 0; break; }
    double rz2 = 0.0;
    for (int64_t A = 0; A < N; ++A) {
      z[A] = dinv[A] * r[A];
      rz2 += r[A] * z[A];
    }
    double be = rz2 / rz;
    rz = rz2;
    for (int64_t A = 0; A < N; ++A) p[A] = z[A] + be * p[A];
  }
  free(r); free(z); free(p); free(q); free(dinv);
  return rc;
}

int orc_newton(const orc_problem *pb, double *U, double atol, double rtol, int maxit,
               int linear_solver, double cg_rtol, double *hist, int *iters) {
  layout L;
  if (lay_init(pb, &L)) return 1;
  int64_t N = L.N, nnz;
  orc_sizes(pb, NULL, NULL, &nnz);
  int64_t *rp = (int64_t *)malloc(sizeof(int64_t) * (N + 1));
  int32_t *ci = (int32_t *)malloc(sizeof(int32_t) * nnz);
  double *v = (double *)malloc(sizeof(double) * nnz);
  double *R = (double *)malloc(sizeof(double) * N), *d = (double *)malloc(sizeof(double) * N);
  orc_csr_pattern(pb, rp, ci);
  for (int64_t A = 0; A < N; ++A)
    if (is_dirichlet(pb, &L, A)) U[A] = 0.0;
  int rc = 4, k;
  double r0 = -1.0;
  for (k = 0; k <= maxit; ++k) {
    if (orc_residual(pb, U, R)) { rc = 2; break; }
    double nr = 0.0;
    for (int64_t A = 0; A < N; ++A) nr += R[A] * R[A];
    nr = sqrt(nr);
    if (hist) hist[k] = nr;
    if (r0 < 0) r0 = nr;
    if (!(nr == nr)) { rc = 4; break; }
    if (nr < atol || nr <= rtol * r0) { rc = 0; break; }
    if (k == maxit) break;
    if (orc_jacobian(pb, U, rp, ci, v)) { rc = 2; break; }
    for (int64_t A = 0; A < N; ++A) R[A] = -R[A];
    int ls = linear_solver;
    if (ls == 0) ls = (pb->dim <= 2 && N <= 200000) ? 1 : 2;
    int lrc = (ls == 1) ? banded_solve(N, rp, ci, v, R, d) : cg_solve(N, rp, ci, v, R, d, cg_rtol, 20000);
    if (lrc) { rc = 5; break; }
    for (int64_t A = 0; A < N; ++A) U[A] += d[A];
  }
  if (iters) *iters = k;
  free(rp); free(ci); free(v); free(R); free(d);
  lay_free(&L);
  return rc;
}

/* ------------------------------------------------------------------------------------ */
/* Quadrature-point data, load vectors and mass matrices (for convergence tests)         */
/* ------------------------------------------------------------------------------------ */
int64_t orc_nqp(const orc_problem *pb) {
  layout L;
  if (lay_init(pb, &L)) return -1;
  int64_t n = L.E * L.nq[0] * L.nq[1] * L.nq[2];
  lay_free(&L);
  return n;
}

int orc_qp_data(const orc_problem *pb, const double *U, double *xq, double *Wq, double *uq,
                double *gradu) {
  layout L;
  if (lay_init(pb, &L)) return 1;
  qpoint *q = (qpoint *)malloc(sizeof(qpoint));
  int nqe = L.nq[0] * L.nq[1] * L.nq[2], rc = 0, dim = pb->dim;
  int64_t k = 0;
  for (int64_t e = 0; e < L.E && !rc; ++e) {
    int em[3], gm[3];
    elem_multi(&L, e, em);
    for (int g = 0; g < nqe && !rc; ++g, ++k) {
      qp_multi(&L, g, gm);
      if ((rc = eval_qp(pb, &L, em, gm, U, q))) break;
      for (int i = 0; i < dim; ++i) {
        if (xq) xq[k * dim + i] = q->x[i];
        if (gradu) gradu[k * dim + i] = q->gu[i];
      }
      if (Wq) Wq[k] = q->W;
      if (uq) uq[k] = q->u;
    }
  }
  free(q);
  lay_free(&L);
  return rc;
}

int orc_load_vector(const orc_problem *pb, const double *fq, double *b) {
  layout L;
  if (lay_init(pb, &L)) return 1;
  memset(b, 0, sizeof(double) * L.N);
  qpoint *q = (qpoint *)malloc(sizeof(qpoint));
  int nqe = L.nq[0] * L.nq[1] * L.nq[2], rc = 0;
  int64_t k = 0;
  for (int64_t e = 0; e < L.E && !rc; ++e) {
    int em[3], gm[3];
    elem_multi(&L, e, em);
    for (int g = 0; g < nqe && !rc; ++g, ++k) {
      qp_multi(&L, g, gm);
      if ((rc = eval_qp(pb, &L, em, gm, NULL, q))) break;
      for (int a = 0; a < q->nloc; ++a) b[q->A[a]] += q->W * q->N[a] * fq[k];
    }
  }
  free(q);
  lay_free(&L);
  return rc;
}

int orc_mass_matrix(const orc_problem *pb, const int64_t *row_ptr, const int32_t *col_idx,
                    double *vals) {
  layout L;
  if (lay_init(pb, &L)) return 1;
  memset(vals, 0, sizeof(double) * row_ptr[L.N]);
  qpoint *q = (qpoint *)malloc(sizeof(qpoint));
  int nqe = L.nq[0] * L.nq[1] * L.nq[2], rc = 0;
  for (int64_t e = 0; e < L.E && !rc; ++e) {
    int em[3], gm[3];
    elem_multi(&L, e, em);
    for (int g = 0; g < nqe && !rc; ++g) {
      qp_multi(&L, g, gm);
      if ((rc = eval_qp(pb, &L, em, gm, NULL, q))) break;
      for (int a = 0; a < q->nloc; ++a)
        for (int b = 0; b < q->nloc; ++b) {
          int64_t s = csr_find(row_ptr, col_idx, q->A[a], q->A[b]);
          if (s < 0) { rc = 3; break; }
          vals[s] += q->W * q->N[a] * q->N[b];
        }
    }
  }
  free(q);
  lay_free(&L);
  return rc;
}

/* ------------------------------------------------------------------------------------ */
/* Second spatial derivatives (Sec. 2.3 eq:ddrational; App. A eq:identity, eq:ddimap,     */
/* eq:ddspatial) at local coordinates t in [-1,1]^dim of one element, and the fourth-order */
/* operator R_A = sum_e sum_q W (Lap N_A)(Lap u_h) built from them.                        */
/* ------------------------------------------------------------------------------------ */
typedef struct {
  int nloc;
  int64_t A[ORC_MAXLOC];
  double N[ORC_MAXLOC], dN[ORC_MAXLOC][3], d2N[ORC_MAXLOC][3][3];   /* spatial */
  double d3N[ORC_MAXLOC][3][3][3];                                  /* spatial third derivatives */
  double x[3];
  double detJ;      /* det of the map xi -> x (the parametric span factors excluded) */
  double span;      /* product of the span factors (xi_{s+1} - xi_s) / 2 */
} hpoint;

static int eval_hess(const orc_problem *pb, const layout *L, const int e[3], const double t[3], hpoint *h) {
  const int dim = L->dim;
  double B[3][ORC_MAXP], dB[3][ORC_MAXP], d2B[3][ORC_MAXP], d3B[3][ORC_MAXP];
  h->span = 1.0;
  for (int d = 0; d < 3; ++d) {
    if (d >= dim) { B[d][0] = 1.0; dB[d][0] = 0.0; d2B[d][0] = 0.0; d3B[d][0] = 0.0; continue; }
    const double *K = L->kn[d];
    int s = L->span[d][e[d]], p = L->p[d];
    double a = K[s], b = K[s + 1];
    double xi = 0.5 * ((a + b) + (b - a) * t[d]);
    h->span *= 0.5 * (b - a);
    for (int k = 0; k <= p; ++k) {
      orc_basis_1d(p, K, pb->nknots[d], s - p + k, xi, &B[d][k], &dB[d][k]);
      orc_basis_1d_d2(p, K, pb->nknots[d], s - p + k, xi, &d2B[d][k]);
      orc_basis_1d_d3(p, K, pb->nknots[d], s - p + k, xi, &d3B[d][k]);
    }
  }
  const int P0 = L->p[0] + 1, P1 = L->p[1] + 1, P2 = L->p[2] + 1, nloc = P0 * P1 * P2;
  h->nloc = nloc;
  static double M[ORC_MAXLOC], dM[ORC_MAXLOC][3], d2M[ORC_MAXLOC][3][3], d3M[ORC_MAXLOC][3][3][3];
  static double Np[ORC_MAXLOC], dNp[ORC_MAXLOC][3], d2Np[ORC_MAXLOC][3][3], d3Np[ORC_MAXLOC][3][3][3];
  for (int a2 = 0; a2 < P2; ++a2)
    for (int a1 = 0; a1 < P1; ++a1)
      for (int a0 = 0; a0 < P0; ++a0) {
        int a = a0 + P0 * (a1 + P1 * a2), ai[3] = {a0, a1, a2};
        int64_t i0 = fn_index(L, 0, L->span[0][e[0]], a0);
        int64_t i1 = fn_index(L, 1, L->span[1][e[1]], a1);
        int64_t i2 = fn_index(L, 2, L->span[2][e[2]], a2);
        h->A[a] = i0 + (int64_t)L->n[0] * (i1 + (int64_t)L->n[1] * i2);
        /* tensor product (Sec. 2.2): differentiate the factor of each axis named by the index */
        for (int al = 0; al < 3; ++al) {
          double v = 1.0;
          for (int d = 0; d < 3; ++d) v *= (d == al) ? dB[d][ai[d]] : B[d][ai[d]];
          dM[a][al] = v;
          for (int be = 0; be < 3; ++be) {
            double w2 = 1.0;
            for (int d = 0; d < 3; ++d) {
              int order = (d == al) + (d == be);
              w2 *= order == 0 ? B[d][ai[d]] : order == 1 ? dB[d][ai[d]] : d2B[d][ai[d]];
            }
            d2M[a][al][be] = w2;
            for (int ga = 0; ga < 3; ++ga) {
              double w3 = 1.0;
              for (int d = 0; d < 3; ++d) {
                int order = (d == al) + (d == be) + (d == ga);
                w3 *= order == 0 ? B[d][ai[d]] : order == 1 ? dB[d][ai[d]] : order == 2 ? d2B[d][ai[d]] : d3B[d][ai[d]];
              }
              d3M[a][al][be][ga] = w3;
            }
          }
        }
        M[a] = B[0][a0] * B[1][a1] * B[2][a2];
      }
  /* rational basis and its first and second parametric derivatives (eq:rational, eq:drational,
   * eq:ddrational); without weights N_A = M_A */
  if (pb->weights) {
    double w = 0.0, dw[3] = {0, 0, 0}, d2w[3][3] = {{0}}, d3w[3][3][3] = {{{0}}};
    for (int a = 0; a < nloc; ++a) {
      double wa = pb->weights[h->A[a]];
      w += wa * M[a];
      for (int al = 0; al < 3; ++al) {
        dw[al] += wa * dM[a][al];
        for (int be = 0; be < 3; ++be) {
          d2w[al][be] += wa * d2M[a][al][be];
          for (int ga = 0; ga < 3; ++ga) d3w[al][be][ga] += wa * d3M[a][al][be][ga];
        }
      }
    }
    for (int a = 0; a < nloc; ++a) {
      double wa = pb->weights[h->A[a]];
      Np[a] = wa * M[a] / w;
      for (int al = 0; al < 3; ++al) dNp[a][al] = (wa * dM[a][al] - Np[a] * dw[al]) / w;
      for (int al = 0; al < 3; ++al)
        for (int be = 0; be < 3; ++be)
          d2Np[a][al][be] = (wa * d2M[a][al][be] - Np[a] * d2w[al][be]) / w
                            - (dNp[a][be] * dw[al] + dNp[a][al] * dw[be]) / w;
      /* eq:dddrational */
      for (int al = 0; al < 3; ++al)
        for (int be = 0; be < 3; ++be)
          for (int ga = 0; ga < 3; ++ga)
            d3Np[a][al][be][ga] = (wa * d3M[a][al][be][ga] - Np[a] * d3w[al][be][ga]) / w
                                  - (dNp[a][al] * d2w[be][ga] + dNp[a][be] * d2w[al][ga] + dNp[a][ga] * d2w[al][be]) / w
                                  - (d2Np[a][be][ga] * dw[al] + d2Np[a][al][ga] * dw[be] + d2Np[a][al][be] * dw[ga]) / w;
    }
  } else {
    for (int a = 0; a < nloc; ++a) {
      Np[a] = M[a];
      for (int al = 0; al < 3; ++al) {
        dNp[a][al] = dM[a][al];
        for (int be = 0; be < 3; ++be) {
          d2Np[a][al][be] = d2M[a][al][be];
          for (int ga = 0; ga < 3; ++ga) d3Np[a][al][be][ga] = d3M[a][al][be][ga];
        }
      }
    }
  }
  /* geometry and its parametric derivatives (App. A): x_{i,alpha}, x_{i,alpha beta} */
  double J[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}, H[3][3][3] = {{{0}}}, T[3][3][3][3] = {{{{0}}}};
  for (int i = 0; i < 3; ++i) h->x[i] = 0.0;
  if (pb->ctrl) {
    for (int i = 0; i < dim; ++i)
      for (int al = 0; al < dim; ++al) J[i][al] = 0.0;
    for (int a = 0; a < nloc; ++a)
      for (int i = 0; i < dim; ++i) {
        double xa = pb->ctrl[h->A[a] * dim + i];
        h->x[i] += xa * Np[a];
        for (int al = 0; al < dim; ++al) {
          J[i][al] += xa * dNp[a][al];
          for (int be = 0; be < dim; ++be) {
            H[i][al][be] += xa * d2Np[a][al][be];
            for (int ga = 0; ga < dim; ++ga) T[i][al][be][ga] += xa * d3Np[a][al][be][ga];
          }
        }
      }
  } else {
    for (int d = 0; d < dim; ++d) {
      const double *K = L->kn[d];
      int sp = L->span[d][e[d]];
      h->x[d] = 0.5 * ((K[sp] + K[sp + 1]) + (K[sp + 1] - K[sp]) * t[d]);
    }
  }
  /* first derivatives of the inverse map from eq:identity (matrix inverse, by cofactors) */
  double det, Ji[3][3] = {{0}};
  if (dim == 1) {
    det = J[0][0];
    Ji[0][0] = 1.0 / det;
  } else if (dim == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    Ji[0][0] = J[1][1] / det;  Ji[0][1] = -J[0][1] / det;
    Ji[1][0] = -J[1][0] / det; Ji[1][1] = J[0][0] / det;
  } else {
    det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
        - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
        + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        /* cofactor of J[c][r], over det: (J^-1)[r][c] */
        int r1 = (c + 1) % 3, r2 = (c + 2) % 3, c1 = (r + 1) % 3, c2 = (r + 2) % 3;
        Ji[r][c] = (J[r1][c1] * J[r2][c2] - J[r1][c2] * J[r2][c1]) / det;
      }
  }
  if (!(det > 0.0)) return 2;
  h->detJ = det;
  /* eq:ddimap, with the sign that differentiating eq:identity gives:
   * xi_{alpha,ij} = - xi_{alpha,m} x_{m,eps mu} xi_{eps,i} xi_{mu,j} */
  double X2[3][3][3] = {{{0}}};   /* [alpha][i][j] */
  for (int al = 0; al < dim; ++al)
    for (int i = 0; i < dim; ++i)
      for (int j = 0; j < dim; ++j) {
        double sum = 0.0;
        for (int m = 0; m < dim; ++m)
          for (int ep = 0; ep < dim; ++ep)
            for (int mu = 0; mu < dim; ++mu) sum += Ji[al][m] * H[m][ep][mu] * Ji[ep][i] * Ji[mu][j];
        X2[al][i][j] = -sum;
      }
  /* eq:dspatial and eq:ddspatial */
  for (int a = 0; a < nloc; ++a) {
    h->N[a] = Np[a];
    for (int i = 0; i < 3; ++i) {
      double g = 0.0;
      if (i < dim)
        for (int al = 0; al < dim; ++al) g += dNp[a][al] * Ji[al][i];
      h->dN[a][i] = g;
      for (int j = 0; j < 3; ++j) {
        double v = 0.0;
        if (i < dim && j < dim) {
          for (int al = 0; al < dim; ++al)
            for (int be = 0; be < dim; ++be) v += d2Np[a][al][be] * Ji[al][i] * Ji[be][j];
          for (int al = 0; al < dim; ++al) v += dNp[a][al] * X2[al][i][j];
        }
        h->d2N[a][i][j] = v;
      }
    }
  }
  /* eq:dddimap: xi_{alpha,ijk} = - x_{m,eps mu om} xi_{alpha,m} xi_{eps,i} xi_{mu,j} xi_{om,k}
   *   - x_{m,eps mu} (xi_{alpha,mk} xi_{eps,i} xi_{mu,j} + xi_{alpha,m} xi_{eps,ik} xi_{mu,j}
   *                   + xi_{alpha,m} xi_{eps,i} xi_{mu,jk}) */
  static double X3[3][3][3][3];   /* [alpha][i][j][k] */
  for (int al = 0; al < 3; ++al)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) {
          double sum = 0.0;
          if (al < dim && i < dim && j < dim && k < dim)
            for (int m = 0; m < dim; ++m)
              for (int ep = 0; ep < dim; ++ep)
                for (int mu = 0; mu < dim; ++mu) {
                  for (int om = 0; om < dim; ++om)
                    sum += T[m][ep][mu][om] * Ji[al][m] * Ji[ep][i] * Ji[mu][j] * Ji[om][k];
                  sum += H[m][ep][mu] * (X2[al][m][k] * Ji[ep][i] * Ji[mu][j] + Ji[al][m] * X2[ep][i][k] * Ji[mu][j] +
                                         Ji[al][m] * Ji[ep][i] * X2[mu][j][k]);
                }
          X3[al][i][j][k] = -sum;
        }
  /* eq:dddspatial: N_{A,ijk} = N_{A,abc} xi_{a,i} xi_{b,j} xi_{c,k}
   *   + N_{A,ab} (xi_{a,ik} xi_{b,j} + xi_{a,i} xi_{b,jk} + xi_{a,ij} xi_{b,k}) + N_{A,a} xi_{a,ijk} */
  for (int a = 0; a < nloc; ++a)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) {
          double v = 0.0;
          if (i < dim && j < dim && k < dim) {
            for (int al = 0; al < dim; ++al)
              for (int be = 0; be < dim; ++be) {
                for (int ga = 0; ga < dim; ++ga) v += d3Np[a][al][be][ga] * Ji[al][i] * Ji[be][j] * Ji[ga][k];
                v += d2Np[a][al][be] * (X2[al][i][k] * Ji[be][j] + Ji[al][i] * X2[be][j][k] + X2[al][i][j] * Ji[be][k]);
              }
            for (int al = 0; al < dim; ++al) v += dNp[a][al] * X3[al][i][j][k];
          }
          h->d3N[a][i][j][k] = v;
        }
  return 0;
}

int orc_basis_third(const orc_problem *pb, int64_t elem, const double *t, int64_t *A, double *d3N) {
  layout L;
  if (!pb || !t || lay_init(pb, &L)) return 1;
  int64_t ne = (int64_t)L.ne[0] * L.ne[1] * L.ne[2];
  if (elem < 0 || elem >= ne) { lay_free(&L); return 1; }
  int em[3];
  elem_multi(&L, elem, em);
  static hpoint h;
  double tt[3] = {t[0], L.dim > 1 ? t[1] : 0.0, L.dim > 2 ? t[2] : 0.0};
  int rc = eval_hess(pb, &L, em, tt, &h);
  if (!rc)
    for (int a = 0; a < h.nloc; ++a) {
      if (A) A[a] = h.A[a];
      if (d3N)
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) d3N[((a * 3 + i) * 3 + j) * 3 + k] = h.d3N[a][i][j][k];
    }
  lay_free(&L);
  return rc;
}

/* R_A = sum over elements and Gauss points of W grad N_A . grad(Lap u_h), with
 * d_i Lap u_h = sum_B U_B sum_j N_{B,ijj} (eq:dddspatial), W as for the fourth-order operator below:
 * the fourth-order operator in the form integrated by parts once (gradient of the Laplacian against
 * the gradient of the test function). */
int orc_grad_laplacian_residual(const orc_problem *pb, const double *U, double *R) {
  layout L;
  if (!pb || !U || !R || lay_init(pb, &L)) return 1;
  int64_t N = (int64_t)L.n[0] * L.n[1] * L.n[2], ne = (int64_t)L.ne[0] * L.ne[1] * L.ne[2];
  for (int64_t A = 0; A < N; ++A) R[A] = 0.0;
  int nqt = L.nq[0] * L.nq[1] * L.nq[2];
  static hpoint h;
  for (int64_t e = 0; e < ne; ++e) {
    int em[3];
    elem_multi(&L, e, em);
    for (int g = 0; g < nqt; ++g) {
      int gm[3];
      qp_multi(&L, g, gm);
      double t[3], wq = 1.0;
      for (int d = 0; d < 3; ++d) {
        t[d] = d < L.dim ? L.gx[d][gm[d]] : 0.0;
        if (d < L.dim) wq *= L.gw[d][gm[d]];
      }
      int rc = eval_hess(pb, &L, em, t, &h);
      if (rc) { lay_free(&L); return rc; }
      double W = wq * h.span * h.detJ, glu[3] = {0, 0, 0};
      for (int a = 0; a < h.nloc; ++a)
        for (int i = 0; i < L.dim; ++i)
          for (int j = 0; j < L.dim; ++j) glu[i] += U[h.A[a]] * h.d3N[a][i][j][j];
      for (int a = 0; a < h.nloc; ++a) {
        double s = 0.0;
        for (int i = 0; i < L.dim; ++i) s += h.dN[a][i] * glu[i];
        R[h.A[a]] += W * s;
      }
    }
  }
  lay_free(&L);
  return 0;
}

int orc_basis_hessian(const orc_problem *pb, int64_t elem, const double *t, int64_t *A, double *N,
                      double *dN, double *d2N, double *x) {
  layout L;
  if (!pb || !t || lay_init(pb, &L)) return 1;
  int64_t ne = (int64_t)L.ne[0] * L.ne[1] * L.ne[2];
  if (elem < 0 || elem >= ne) { lay_free(&L); return 1; }
  int em[3];
  elem_multi(&L, elem, em);
  static hpoint h;
  double tt[3] = {t[0], L.dim > 1 ? t[1] : 0.0, L.dim > 2 ? t[2] : 0.0};
  int rc = eval_hess(pb, &L, em, tt, &h);
  if (!rc) {
    for (int a = 0; a < h.nloc; ++a) {
      if (A) A[a] = h.A[a];
      if (N) N[a] = h.N[a];
      for (int i = 0; i < 3; ++i) {
        if (dN) dN[a * 3 + i] = h.dN[a][i];
        for (int j = 0; j < 3; ++j)
          if (d2N) d2N[(a * 3 + i) * 3 + j] = h.d2N[a][i][j];
      }
    }
    if (x) for (int i = 0; i < 3; ++i) x[i] = h.x[i];
  }
  lay_free(&L);
  return rc;
}

/* R_A = sum over elements and Gauss points of W (Lap N_A)(Lap u_h), Lap the spatial Laplacian
 * (trace of eq:ddspatial), W = Gauss weights * span factors * det J; all functions, no boundary
 * rows: the fourth-order operator of a primal biharmonic / Cahn-Hilliard-type weak form. */
int orc_biharmonic_residual(const orc_problem *pb, const double *U, double *R) {
  layout L;
  if (!pb || !U || !R || lay_init(pb, &L)) return 1;
  int64_t N = (int64_t)L.n[0] * L.n[1] * L.n[2], ne = (int64_t)L.ne[0] * L.ne[1] * L.ne[2];
  for (int64_t A = 0; A < N; ++A) R[A] = 0.0;
  int nqt = L.nq[0] * L.nq[1] * L.nq[2];
  static hpoint h;
  static double lap[ORC_MAXLOC];
  for (int64_t e = 0; e < ne; ++e) {
    int em[3];
    elem_multi(&L, e, em);
    for (int g = 0; g < nqt; ++g) {
      int gm[3];
      qp_multi(&L, g, gm);
      double t[3], wq = 1.0;
      for (int d = 0; d < 3; ++d) {
        t[d] = d < L.dim ? L.gx[d][gm[d]] : 0.0;
        if (d < L.dim) wq *= L.gw[d][gm[d]];
      }
      int rc = eval_hess(pb, &L, em, t, &h);
      if (rc) { lay_free(&L); return rc; }
      double W = wq * h.span * h.detJ, lu = 0.0;
      for (int a = 0; a < h.nloc; ++a) {
        lap[a] = 0.0;
        for (int i = 0; i < L.dim; ++i) lap[a] += h.d2N[a][i][i];
        lu += U[h.A[a]] * lap[a];
      }
      for (int a = 0; a < h.nloc; ++a) R[h.A[a]] += W * lap[a] * lu;
    }
  }
  lay_free(&L);
  return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Generalized-alpha time stepping (eq:ga) for first-order systems R(Udot, U) = 0         */
/* ------------------------------------------------------------------------------------ */
int orc_gen_alpha_params(double rho, double *am, double *af, double *gamma) {
  if (!(rho >= 0.0 && rho <= 1.0) || !am || !af || !gamma) return 1;
  *am = 0.5 * (3.0 - rho) / (1.0 + rho);
  *af = 1.0 / (1.0 + rho);
  *gamma = 0.5 + *am - *af;
  return 0;
}

/* One step for R(Udot, U) = M0 Udot + R_B(U): R_B the residual of eq:residual (Dirichlet rows U_A),
 * M0 the mass matrix with the rows and columns of Dirichlet functions removed.  Unknown Udot_{n+1},
 * by Newton on G = M0 Udot_{n+am} + R_B(U_{n+af}) (eq:ga), dG/dUdot_{n+1} = am M0 + af gamma dt
 * J(U_{n+af}), each linear system solved exactly (banded LU in 2D, CG to 1e-14 in 3D); starts from
 * Udot_{n+1} = Udot_n (zero on Dirichlet functions); stops when ||G||_2 < atol. */
int orc_gen_alpha_step(const orc_problem *pb, const double *U0, const double *V0, double dt, double rho,
                       double atol, int maxit, double *U1, double *V1, int *iters) {
  double am, af, gm;
  if (!pb || !U0 || !V0 || !U1 || !V1 || !(dt > 0.0) || orc_gen_alpha_params(rho, &am, &af, &gm)) return 1;
  layout L;
  if (lay_init(pb, &L)) return 1;
  int64_t N = L.N, nnz;
  orc_sizes(pb, NULL, NULL, &nnz);
  int64_t *rp = (int64_t *)malloc(sizeof(int64_t) * (N + 1));
  int32_t *ci = (int32_t *)malloc(sizeof(int32_t) * nnz);
  double *Mv = (double *)malloc(sizeof(double) * nnz), *Jv = (double *)malloc(sizeof(double) * nnz);
  double *Ua = (double *)malloc(sizeof(double) * N), *Va = (double *)malloc(sizeof(double) * N);
  double *G = (double *)malloc(sizeof(double) * N), *d = (double *)malloc(sizeof(double) * N);
  char *dir = (char *)malloc((size_t)N);
  orc_csr_pattern(pb, rp, ci);
  int rc = orc_mass_matrix(pb, rp, ci, Mv);
  for (int64_t A = 0; A < N; ++A) dir[A] = (char)is_dirichlet(pb, &L, A);
  for (int64_t A = 0; A < N; ++A)
    for (int64_t k = rp[A]; k < rp[A + 1]; ++k)
      if (dir[A] || dir[ci[k]]) Mv[k] = 0.0;
  for (int64_t A = 0; A < N; ++A) V1[A] = dir[A] ? 0.0 : V0[A];
  int k = 0;
  if (!rc) rc = 4;
  for (k = 0; k <= maxit && rc != 0 && rc != 2 && rc != 5; ++k) {
    for (int64_t A = 0; A < N; ++A) {
      Ua[A] = U0[A] + af * dt * (gm * V1[A] + (1.0 - gm) * V0[A]);
      Va[A] = V0[A] + am * (V1[A] - V0[A]);
    }
    if (orc_residual(pb, Ua, G)) { rc = 2; break; }
    double nr = 0.0;
    for (int64_t A = 0; A < N; ++A) {
      double s = 0.0;
      for (int64_t q = rp[A]; q < rp[A + 1]; ++q) s += Mv[q] * Va[ci[q]];
      G[A] += s;
      nr += G[A] * G[A];
    }
    if (!(nr == nr)) { rc = 4; break; }
    if (sqrt(nr) < atol) { rc = 0; break; }
    if (k == maxit) break;
    if (orc_jacobian(pb, Ua, rp, ci, Jv)) { rc = 2; break; }
    for (int64_t q = 0; q < nnz; ++q) Jv[q] = am * Mv[q] + af * gm * dt * Jv[q];
    for (int64_t A = 0; A < N; ++A) G[A] = -G[A];
    int lrc = (pb->dim <= 2 && N <= 200000) ? banded_solve(N, rp, ci, Jv, G, d) : cg_solve(N, rp, ci, Jv, G, d, 1e-14, 20000);
    if (lrc) { rc = 5; break; }
    for (int64_t A = 0; A < N; ++A) V1[A] += d[A];
  }
  for (int64_t A = 0; A < N; ++A) U1[A] = U0[A] + dt * (gm * V1[A] + (1.0 - gm) * V0[A]);
  if (iters) *iters = k;
  free(rp); free(ci); free(Mv); free(Jv); free(Ua); free(Va); free(G); free(d); free(dir);
  lay_free(&L);
  return rc;
}

/* ------------------------------------------------------------------------------------ */
/* Cahn-Hilliard residual (the paper's strong form, D = 1), primal weak form:            */
/*   R_A = sum_e sum_q W [ N_A cdot + M mu' grad N_A . grad c                             */
/*                         + lam (M Lap N_A + M' grad c . grad N_A) Lap c ]               */
/* M = c (1 - c), M' = 1 - 2c, mu' = 1 / (2 theta c (1 - c)) - 2 (derivative of the       */
/* chemical potential); boundary terms dropped (periodic axes, or the natural conditions).*/
/* ------------------------------------------------------------------------------------ */
int orc_cahn_hilliard_residual(const orc_problem *pb, const double *Cv, const double *Cd, double theta,
                               double lam, double *R) {
  layout L;
  if (!pb || !Cv || !Cd || !R || !(theta > 0.0) || lay_init(pb, &L)) return 1;
  int64_t N = (int64_t)L.n[0] * L.n[1] * L.n[2], ne = (int64_t)L.ne[0] * L.ne[1] * L.ne[2];
  for (int64_t A = 0; A < N; ++A) R[A] = 0.0;
  int nqt = L.nq[0] * L.nq[1] * L.nq[2];
  static hpoint h;
  static double lap[ORC_MAXLOC];
  for (int64_t e = 0; e < ne; ++e) {
    int em[3];
    elem_multi(&L, e, em);
    for (int g = 0; g < nqt; ++g) {
      int gm[3];
      qp_multi(&L, g, gm);
      double t[3], wq = 1.0;
      for (int d = 0; d < 3; ++d) {
        t[d] = d < L.dim ? L.gx[d][gm[d]] : 0.0;
        if (d < L.dim) wq *= L.gw[d][gm[d]];
      }
      int rc = eval_hess(pb, &L, em, t, &h);
      if (rc) { lay_free(&L); return rc; }
      double W = wq * h.span * h.detJ, c = 0.0, cd = 0.0, gc[3] = {0, 0, 0}, lc = 0.0;
      for (int a = 0; a < h.nloc; ++a) {
        lap[a] = 0.0;
        for (int i = 0; i < L.dim; ++i) lap[a] += h.d2N[a][i][i];
        c += Cv[h.A[a]] * h.N[a];
        cd += Cd[h.A[a]] * h.N[a];
        for (int i = 0; i < 3; ++i) gc[i] += Cv[h.A[a]] * h.dN[a][i];
        lc += Cv[h.A[a]] * lap[a];
      }
      double M = c * (1.0 - c), dM = 1.0 - 2.0 * c, dmu = 1.0 / (2.0 * theta * c * (1.0 - c)) - 2.0;
      for (int a = 0; a < h.nloc; ++a) {
        double gg = 0.0;
        for (int i = 0; i < 3; ++i) gg += h.dN[a][i] * gc[i];
        R[h.A[a]] += W * (h.N[a] * cd + M * dmu * gg + lam * (M * lap[a] + dM * gg) * lc);
      }
    }
  }
  lay_free(&L);
  return 0;
}
