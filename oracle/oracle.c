/*
 * CPU oracle for the space-charge field path.  TEST INFRASTRUCTURE ONLY: the
 * tests, the smoke check and the CPU-baseline leg of the benchmark are its
 * only users; the product library never links or calls it.
 *
 * Plain, slow and direct: every sum is a brute-force loop over all pairs,
 * accumulated in x87 long double, and every cell integral is evaluated in
 * long double from its closed form.  Nothing here is blocked, fused or
 * reordered.  Each function names the passage of the paper it follows
 * (OuroborosBEM, arXiv 2110.09214).
 *
 * Conventions (shared with the Python wrapper, oracle/__init__.py):
 *   positions are AoS row-major (n, 3) float64; panels are three (N, 3)
 *   vertex arrays a, b, c (counter-clockwise about the normal
 *   n = (b-a)x(c-a)/|..|); kind 0 = electrode cell (ed), 1 = dielectric
 *   interface cell (dd); eps1 on the -n side, eps2 on the +n side.
 *   Units SI.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef long double real;

/* CODATA 2018. */
#define EPS0 8.8541878128e-12L
#define QE 1.602176634e-19L
#define ME 9.1093837015e-31L
#define KB 1.380649e-23L
#define AMU 1.66053906660e-27L
#define PI_L 3.141592653589793238462643383279502884L

static real k_e(void) { return 1.0L / (4.0L * PI_L * EPS0); }

void oc_constants(double *out) {
  out[0] = (double)EPS0;
  out[1] = (double)k_e();
  out[2] = (double)QE;
  out[3] = (double)ME;
  out[4] = (double)KB;
  out[5] = (double)AMU;
}

/* ------------------------------------------------------------------------- */
/* small vector helpers                                                       */
/* ------------------------------------------------------------------------- */
typedef struct { real x, y, z; } v3;
static v3 mk(real x, real y, real z) { v3 r = {x, y, z}; return r; }
static v3 ld(const double *p) { return mk(p[0], p[1], p[2]); }
static v3 sub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 add(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 scl(v3 a, real s) { return mk(a.x * s, a.y * s, a.z * s); }
static real dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 crs(v3 a, v3 b) { return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
static real nrm(v3 a) { return sqrtl(dot(a, a)); }

/* ------------------------------------------------------------------------- */
/* Cell geometry (section 2.2: flat cells with constant sigma, collocation    */
/* at the cell centre r_i).                                                   */
/* ------------------------------------------------------------------------- */
typedef struct {
  v3 p[3];    /* vertices a, b, c */
  v3 N2;      /* (b-a)x(c-a) = 2 * area * n */
  v3 n;       /* unit normal */
  real area;
  v3 t[3];    /* unit tangent of edge e: p[e] -> p[e+1] */
  v3 m[3];    /* outward in-plane unit normal of edge e: t x n */
  real L[3];  /* edge lengths */
  v3 cen;     /* centroid */
  real diam;  /* longest edge */
} tri_t;

static void tri_setup(const double *a, const double *b, const double *c, tri_t *T) {
  T->p[0] = ld(a); T->p[1] = ld(b); T->p[2] = ld(c);
  T->N2 = crs(sub(T->p[1], T->p[0]), sub(T->p[2], T->p[0]));
  real n2 = nrm(T->N2);
  T->area = 0.5L * n2;
  T->n = scl(T->N2, 1.0L / n2);
  T->diam = 0;
  for (int e = 0; e < 3; ++e) {
    v3 d = sub(T->p[(e + 1) % 3], T->p[e]);
    T->L[e] = nrm(d);
    T->t[e] = scl(d, 1.0L / T->L[e]);
    T->m[e] = crs(T->t[e], T->n);
    if (T->L[e] > T->diam) T->diam = T->L[e];
  }
  T->cen = scl(add(add(T->p[0], T->p[1]), T->p[2]), 1.0L / 3.0L);
}

/* Per-edge quantities of the line integral f_e = int_e dl' / |r - r'|.
 * l- , l+ : signed abscissae of the endpoints along t measured from the foot
 *           of r on the edge line (l = t.(p - r)), R-, R+ : endpoint distances,
 *           R0sq : squared distance of r from the edge line, d : r - foot. */
typedef struct { real lm, lp, Rm, Rp, R0sq, f; v3 d; } edge_t;

static edge_t edge_eval(const tri_t *T, int e, v3 r) {
  edge_t E;
  v3 pm = T->p[e];
  v3 dm = sub(r, pm);
  E.lm = -dot(T->t[e], dm);
  E.lp = E.lm + T->L[e];
  E.Rm = nrm(dm);
  E.Rp = nrm(sub(r, T->p[(e + 1) % 3]));
  v3 tx = crs(T->t[e], dm);
  E.R0sq = dot(tx, tx);
  E.d = add(dm, scl(T->t[e], E.lm));
  /* f = ln((R+ + l+)/(R- + l-)) = ln((R- - l-)/(R+ - l+)); written as log1p of
   * a ratio whose numerator has no cancellation: R+ - R- = L (l+ + l-)/(R+ + R-). */
  real s = E.lp + E.lm, L = T->L[e], Rs = E.Rp + E.Rm;
  if (s >= 0) {
    real den = (E.lm >= 0) ? (E.Rm + E.lm) : E.R0sq / (E.Rm - E.lm);
    E.f = log1pl(L * (1.0L + s / Rs) / den);
  } else {
    real den = (E.lp <= 0) ? (E.Rp - E.lp) : E.R0sq / (E.Rp + E.lp);
    E.f = log1pl(L * (1.0L - s / Rs) / den);
  }
  return E;
}

/* Signed solid angle subtended by the cell at r, positive on the +n side
 * (van Oosterom & Strackee); the numerator A.(BxC) is formed as
 * -(r - a).((b - a)x(c - a)), which is the same determinant without the
 * cancellation of the B x C product.  A point exactly in the cell plane gets 0
 * (principal value: the +-2 pi jump of the normal field is carried by the
 * diagonal term of the Neumann rows, eq. (BEMfld)). */
static real solid_angle(const tri_t *T, v3 r) {
  v3 A = sub(T->p[0], r), B = sub(T->p[1], r), C = sub(T->p[2], r);
  real num = dot(sub(r, T->p[0]), T->N2);
  if (num == 0) return 0;
  real a = nrm(A), b = nrm(B), c = nrm(C);
  real den = a * b * c + dot(A, B) * c + dot(A, C) * b + dot(B, C) * a;
  return 2.0L * atan2l(num, den);
}

/* Unit-density cell integrals at r (the integrals of eqs. (BEM2), (BEM3)):
 *   IV = int_C dS' / |r - r'|,  IE = int_C (r - r') / |r - r'|^3 dS'.
 * Closed forms from the divergence theorem on the flat cell:
 *   IE = sum_e m_e f_e + n Omega,   IV = sum_e (m_e.(p_e - r)) f_e - h Omega,
 * with h = n.(r - a). */
static void tri_IV_IE(const tri_t *T, v3 r, real *IV, v3 *IE) {
  real Om = solid_angle(T, r);
  real h = dot(T->n, sub(r, T->p[0]));
  v3 ie = scl(T->n, Om);
  real iv = -h * Om;
  for (int e = 0; e < 3; ++e) {
    edge_t E = edge_eval(T, e, r);
    ie = add(ie, scl(T->m[e], E.f));
    iv += dot(T->m[e], sub(T->p[e], r)) * E.f;
  }
  if (IV) *IV = iv;
  if (IE) *IE = ie;
}

/* (l+/R+ - l-/R-)/R0^2 without cancellation when r is near the edge line. */
static real lr_diff(const edge_t *E) {
  if (E->lm >= 0)
    return 1.0L / (E->Rm * (E->Rm + E->lm)) - 1.0L / (E->Rp * (E->Rp + E->lp));
  if (E->lp <= 0)
    return 1.0L / (E->Rp * (E->Rp - E->lp)) - 1.0L / (E->Rm * (E->Rm - E->lm));
  return (E->lp / E->Rp - E->lm / E->Rm) / E->R0sq;
}

/* Jacobian G[j][k] = d IE_j / d r_k of the unit-density cell field (for the
 * adjoint; not in the paper).  IE = sum_e m_e f_e + n Omega gives
 *   G = sum_e m_e (x) grad f_e + n (x) grad Omega,
 *   grad f_e   = -d_e D_e - t_e (1/R+ - 1/R-),   D_e = (l+/R+ - l-/R-)/R0^2,
 *   grad Omega = -sum_e (t_e x d_e) D_e.                                  */
static void tri_grad(const tri_t *T, v3 r, real G[3][3]) {
  v3 gO = mk(0, 0, 0);
  for (int j = 0; j < 3; ++j)
    for (int k = 0; k < 3; ++k) G[j][k] = 0;
  for (int e = 0; e < 3; ++e) {
    edge_t E = edge_eval(T, e, r);
    real D = lr_diff(&E);
    real inv_diff = -T->L[e] * (E.lp + E.lm) / ((E.Rp + E.Rm) * E.Rp * E.Rm); /* 1/R+ - 1/R- */
    v3 gf = add(scl(E.d, -D), scl(T->t[e], -inv_diff));
    real mv[3] = {T->m[e].x, T->m[e].y, T->m[e].z};
    real gv[3] = {gf.x, gf.y, gf.z};
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) G[j][k] += mv[j] * gv[k];
    gO = add(gO, scl(crs(T->t[e], E.d), -D));
  }
  real nv[3] = {T->n.x, T->n.y, T->n.z};
  real ov[3] = {gO.x, gO.y, gO.z};
  for (int j = 0; j < 3; ++j)
    for (int k = 0; k < 3; ++k) G[j][k] += nv[j] * ov[k];
}

/* Exported single-cell evaluations (for the pins). */
void oc_tri_integrals(const double *a, const double *b, const double *c, const double *r, double *IV,
                      double *IE) {
  tri_t T;
  tri_setup(a, b, c, &T);
  real iv;
  v3 ie;
  tri_IV_IE(&T, ld(r), &iv, &ie);
  *IV = (double)iv;
  IE[0] = (double)ie.x; IE[1] = (double)ie.y; IE[2] = (double)ie.z;
}

void oc_tri_grad(const double *a, const double *b, const double *c, const double *r, double *G) {
  tri_t T;
  tri_setup(a, b, c, &T);
  real g[3][3];
  tri_grad(&T, ld(r), g);
  for (int j = 0; j < 3; ++j)
    for (int k = 0; k < 3; ++k) G[3 * j + k] = (double)g[j][k];
}

void oc_tri_geometry(int64_t N, const double *a, const double *b, const double *c, double *normal,
                     double *area, double *centroid, double *diam) {
  for (int64_t i = 0; i < N; ++i) {
    tri_t T;
    tri_setup(a + 3 * i, b + 3 * i, c + 3 * i, &T);
    normal[3 * i] = (double)T.n.x; normal[3 * i + 1] = (double)T.n.y; normal[3 * i + 2] = (double)T.n.z;
    area[i] = (double)T.area;
    centroid[3 * i] = (double)T.cen.x; centroid[3 * i + 1] = (double)T.cen.y;
    centroid[3 * i + 2] = (double)T.cen.z;
    diam[i] = (double)T.diam;
  }
}

/* ------------------------------------------------------------------------- */
/* Panel field, eqs. (BEM2), (BEM3): V and E at targets from constant sigma   */
/* per cell.                                                                   */
/* ------------------------------------------------------------------------- */
void oc_panel_field(int64_t nt, const double *x, int64_t N, const double *a, const double *b,
                    const double *c, const double *sigma, double *E, double *V) {
  tri_t *T = (tri_t *)malloc(sizeof(tri_t) * (size_t)(N > 0 ? N : 1));
  for (int64_t k = 0; k < N; ++k) tri_setup(a + 3 * k, b + 3 * k, c + 3 * k, &T[k]);
  real ke = k_e();
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < nt; ++i) {
    v3 r = ld(x + 3 * i);
    real ex = 0, ey = 0, ez = 0, vv = 0;
    for (int64_t k = 0; k < N; ++k) {
      real iv;
      v3 ie;
      tri_IV_IE(&T[k], r, &iv, &ie);
      real s = sigma[k];
      ex += s * ie.x; ey += s * ie.y; ez += s * ie.z; vv += s * iv;
    }
    E[3 * i] = (double)(ke * ex); E[3 * i + 1] = (double)(ke * ey); E[3 * i + 2] = (double)(ke * ez);
    if (V) V[i] = (double)(ke * vv);
  }
  free(T);
}

/* ------------------------------------------------------------------------- */
/* Direct pairwise field, eq. (nbody), with Plummer softening s:              */
/*   E_i = k_e sum_{j != i} q_j (x_i - x_j) / (|x_i - x_j|^2 + s^2)^{3/2}      */
/*   V_i = k_e sum_{j != i} q_j / (|x_i - x_j|^2 + s^2)^{1/2}                  */
/* tgt_is_src: targets are the sources (same arrays), j = i skipped by index. */
/* Optionally, for each target of species e- (0) or cation (1), the nearest    */
/* source of the opposite one of these two species (distance^2 unsoftened,    */
/* ties to the lower source index), as used by the recombination test         */
/* (section 3.3.6: distances from the N-body evaluation).                     */
/* ------------------------------------------------------------------------- */
void oc_pair_field(int64_t nt, const double *xt, int64_t ns, const double *xs, const double *q,
                   double soft, int tgt_is_src, double *E, double *V, const int8_t *sp_t,
                   const int8_t *sp_s, int64_t *nn_idx, double *nn_d2) {
  real ke = k_e(), s2 = (real)soft * (real)soft;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < nt; ++i) {
    v3 r = ld(xt + 3 * i);
    real ex = 0, ey = 0, ez = 0, vv = 0;
    int want = -1;
    if (nn_idx && sp_t) want = (sp_t[i] == 0) ? 1 : (sp_t[i] == 1 ? 0 : -1);
    double best = INFINITY;
    int64_t bi = -1;
    for (int64_t j = 0; j < ns; ++j) {
      if (tgt_is_src && j == i) continue;
      v3 d = sub(r, ld(xs + 3 * j));
      real d2 = dot(d, d);
      real S2 = d2 + s2;
      real inv = 1.0L / sqrtl(S2);
      real w = q[j] * inv * inv * inv;
      ex += w * d.x; ey += w * d.y; ez += w * d.z;
      vv += q[j] * inv;
      if (want >= 0 && sp_s[j] == want) {
        double dd = (double)d2;
        if (dd < best) { best = dd; bi = j; }
      }
    }
    E[3 * i] = (double)(ke * ex); E[3 * i + 1] = (double)(ke * ey); E[3 * i + 2] = (double)(ke * ez);
    if (V) V[i] = (double)(ke * vv);
    if (nn_idx) { nn_idx[i] = bi; nn_d2[i] = best; }
  }
}

/* ------------------------------------------------------------------------- */
/* Collocation system, eqs. (BEMpot), (BEMfld), (matrixBEM).  Row-major A.    */
/*   ed row i: A_ij = k_e IV(j, r_i)                                          */
/*   dd row i: A_ii = (eps1 + eps2)/2,                                         */
/*             A_ij = (eps2 - eps1)/(4 pi) n_i . IE(j, r_i)   (j != i)         */
/* (eq. (BEMfld) divided by eps0; r_i = centroid of cell i.)                  */
/* ------------------------------------------------------------------------- */
static real bem_entry(const tri_t *T, const int8_t *kind, const double *eps1, const double *eps2,
                      int64_t i, int64_t j) {
  real iv;
  v3 ie;
  if (kind[i] == 0) {
    tri_IV_IE(&T[j], T[i].cen, &iv, NULL);
    return k_e() * iv;
  }
  if (i == j) return 0.5L * ((real)eps1[i] + (real)eps2[i]);
  tri_IV_IE(&T[j], T[i].cen, NULL, &ie);
  return ((real)eps2[i] - (real)eps1[i]) / (4.0L * PI_L) * dot(T[i].n, ie);
}

void oc_bem_assemble(int64_t N, const double *a, const double *b, const double *c, const int8_t *kind,
                     const double *eps1, const double *eps2, double *A) {
  tri_t *T = (tri_t *)malloc(sizeof(tri_t) * (size_t)N);
  for (int64_t k = 0; k < N; ++k) tri_setup(a + 3 * k, b + 3 * k, c + 3 * k, &T[k]);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < N; ++i)
    for (int64_t j = 0; j < N; ++j) A[i * N + j] = (double)bem_entry(T, kind, eps1, eps2, i, j);
  free(T);
}

/* Residual r_i = rhs_i - sum_j A_ij sigma_j for the listed rows, with A
 * regenerated on the fly (no stored matrix) and long double accumulation. */
void oc_bem_residual_rows(int64_t N, const double *a, const double *b, const double *c, const int8_t *kind,
                          const double *eps1, const double *eps2, const double *sigma, const double *rhs,
                          int64_t nrows, const int64_t *rows, double *res, double *absrow) {
  tri_t *T = (tri_t *)malloc(sizeof(tri_t) * (size_t)N);
  for (int64_t k = 0; k < N; ++k) tri_setup(a + 3 * k, b + 3 * k, c + 3 * k, &T[k]);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t r = 0; r < nrows; ++r) {
    int64_t i = rows[r];
    real acc = rhs[i], aa = 0;
    for (int64_t j = 0; j < N; ++j) {
      real Aij = (real)(double)bem_entry(T, kind, eps1, eps2, i, j);
      acc -= Aij * (real)sigma[j];
      aa += fabsl(Aij);
    }
    res[r] = (double)acc;
    if (absrow) absrow[r] = (double)aa;
  }
  free(T);
}

/* Residual of a stored row-major system in long double. */
void oc_residual_dense(int64_t N, const double *A, const double *x, const double *b, double *r) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    real acc = b[i];
    for (int64_t j = 0; j < N; ++j) acc -= (real)A[i * N + j] * (real)x[j];
    r[i] = (double)acc;
  }
}

/* ------------------------------------------------------------------------- */
/* Adjoint of the field evaluation for L = sum_i w_i . E(x_i) (not in the     */
/* paper).                                                                     */
/*   dL/dsigma_k = k_e sum_i w_i . IE(k, x_i)                                  */
/*   dL/dx_i    += k_e sum_k sigma_k G_k(x_i)^T w_i                            */
/* ------------------------------------------------------------------------- */
void oc_panel_backward(int64_t nt, const double *x, int64_t N, const double *a, const double *b,
                       const double *c, const double *sigma, const double *w, double *g_sigma, double *g_x) {
  tri_t *T = (tri_t *)malloc(sizeof(tri_t) * (size_t)(N > 0 ? N : 1));
  for (int64_t k = 0; k < N; ++k) tri_setup(a + 3 * k, b + 3 * k, c + 3 * k, &T[k]);
  real ke = k_e();
  if (g_sigma) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < N; ++k) {
      real acc = 0;
      for (int64_t i = 0; i < nt; ++i) {
        v3 ie;
        tri_IV_IE(&T[k], ld(x + 3 * i), NULL, &ie);
        acc += w[3 * i] * ie.x + w[3 * i + 1] * ie.y + w[3 * i + 2] * ie.z;
      }
      g_sigma[k] = (double)(ke * acc);
    }
  }
  if (g_x) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i) {
      v3 r = ld(x + 3 * i);
      real gx = 0, gy = 0, gz = 0;
      real wv[3] = {w[3 * i], w[3 * i + 1], w[3 * i + 2]};
      for (int64_t k = 0; k < N; ++k) {
        real G[3][3];
        tri_grad(&T[k], r, G);
        real s = sigma[k];
        gx += s * (G[0][0] * wv[0] + G[1][0] * wv[1] + G[2][0] * wv[2]);
        gy += s * (G[0][1] * wv[0] + G[1][1] * wv[1] + G[2][1] * wv[2]);
        gz += s * (G[0][2] * wv[0] + G[1][2] * wv[1] + G[2][2] * wv[2]);
      }
      g_x[3 * i] = (double)(ke * gx); g_x[3 * i + 1] = (double)(ke * gy); g_x[3 * i + 2] = (double)(ke * gz);
    }
  }
  free(T);
}

/* Pairwise adjoint.  With K(d) = d / S^3, S^2 = |d|^2 + s^2, and its Jacobian
 * J(d) = I/S^3 - 3 d d^T / S^5 (symmetric, even in d):
 *   target part  g_t[i] = k_e sum_j q_j J(x_i - x_j) w_i
 *   source part  g_s[j] = -k_e q_j sum_i J(x_i - x_j) w_i
 * With tgt_is_src the two parts are summed into g_t (g_s unused). */
void oc_pair_backward(int64_t nt, const double *xt, int64_t ns, const double *xs, const double *q,
                      double soft, int tgt_is_src, const double *w, double *g_t, double *g_s) {
  real ke = k_e(), s2 = (real)soft * (real)soft;
  if (g_t) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < nt; ++i) {
      v3 r = ld(xt + 3 * i);
      v3 wi = ld(w + 3 * i);
      real gx = 0, gy = 0, gz = 0;
      for (int64_t j = 0; j < ns; ++j) {
        if (tgt_is_src && j == i) continue;
        v3 d = sub(r, ld(xs + 3 * j));
        real S2 = dot(d, d) + s2;
        real inv = 1.0L / sqrtl(S2);
        real i3 = inv * inv * inv, i5 = i3 * inv * inv;
        /* a = q_j w_i (target role) - q_i w_j (source role, if shared) */
        v3 av = scl(wi, (real)q[j]);
        if (tgt_is_src) av = sub(av, scl(ld(w + 3 * j), (real)q[i]));
        real da = dot(d, av);
        gx += av.x * i3 - 3.0L * d.x * da * i5;
        gy += av.y * i3 - 3.0L * d.y * da * i5;
        gz += av.z * i3 - 3.0L * d.z * da * i5;
      }
      g_t[3 * i] = (double)(ke * gx); g_t[3 * i + 1] = (double)(ke * gy); g_t[3 * i + 2] = (double)(ke * gz);
    }
  }
  if (g_s && !tgt_is_src) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < ns; ++j) {
      v3 xj = ld(xs + 3 * j);
      real gx = 0, gy = 0, gz = 0;
      for (int64_t i = 0; i < nt; ++i) {
        v3 d = sub(ld(xt + 3 * i), xj);
        real S2 = dot(d, d) + s2;
        real inv = 1.0L / sqrtl(S2);
        real i3 = inv * inv * inv, i5 = i3 * inv * inv;
        v3 wi = ld(w + 3 * i);
        real dw = dot(d, wi);
        gx += wi.x * i3 - 3.0L * d.x * dw * i5;
        gy += wi.y * i3 - 3.0L * d.y * dw * i5;
        gz += wi.z * i3 - 3.0L * d.z * dw * i5;
      }
      real f = -ke * (real)q[j];
      g_s[3 * j] = (double)(f * gx); g_s[3 * j + 1] = (double)(f * gy); g_s[3 * j + 2] = (double)(f * gz);
    }
  }
}

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the        */
/* 4x32 Philox S-P network, multipliers 0xD2511F53 / 0xCD9E8D57, key Weyl     */
/* increments 0x9E3779B9 / 0xBB67AE85.                                         */
/* ------------------------------------------------------------------------- */
void oc_philox4x32_10(const uint32_t *ctr_in, const uint32_t *key_in, uint32_t *out) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double u01(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

/* ------------------------------------------------------------------------- */
/* Transport step: constant-field flights (Euler with one field evaluation   */
/* per step, section 3.3.5), null-collision Monte Carlo against the gas      */
/* tables (section 3.4; the null-collision variant the paper contrasts with), */
/* absorption on cells (section 2.3) and ionisation pair creation (eq.       */
/* (distIoni)).                                                               */
/* ------------------------------------------------------------------------- */
typedef struct {
  int32_t n_nodes;
  double e_min, e_max;     /* eV */
  const double *xs;        /* [5][n_nodes] m^2 */
  double thr[5];           /* eV */
  double density, temperature, m_gas, m_cation, m_anion, ion_xs_iso, ion_xs_back;
  const double *xi;        /* [n_nodes] anisotropy xi(E) of eq. (anisotrop), or NULL (isotropic) */
  double penning_prob;     /* Penning transfer probability (section 3.4.4), 0 = off */
  double penning_level;    /* ionisation potential of the quenching species, eV */
} oc_gas;

typedef struct {
  double dt;
  uint32_t step;
  uint64_t seed;
  int32_t max_coll;
  int32_t max_ion_per_step;  /* ionisations with children per particle per step */
  double ion_v_cap;          /* speed bound used for the ion null-collision rate */
  double box_lo[3], box_hi[3];
} oc_step;

/* Per-particle outcome. */
enum { OC_ALIVE = 0, OC_ABSORBED = 1, OC_LEFT = 2 };

/* Cross section k at energy eps (eV), linear in the normalised lethargy of
 * eq. (leth) between log-spaced nodes, clamped to the end nodes. */
static double xs_at(const oc_gas *g, int k, double eps) {
  int n = g->n_nodes;
  if (!(eps > g->e_min)) return g->xs[k * n];
  if (eps >= g->e_max) return g->xs[k * n + n - 1];
  double p = (double)(n - 1) * (log(eps / g->e_min) / log(g->e_max / g->e_min));
  int i = (int)floor(p);
  if (i >= n - 1) i = n - 2;
  double fr = p - (double)i;
  return g->xs[k * n + i] * (1.0 - fr) + g->xs[k * n + i + 1] * fr;
}

double oc_xs_at(const oc_gas *g, int k, double eps) { return xs_at(g, k, eps); }

/* Electron null-collision rate bound: N max_b max(sig_b, sig_b+1) v(E_b+1). */
double oc_nu_max_electron(const oc_gas *g) {
  int n = g->n_nodes;
  double best = 0;
  for (int b = 0; b + 1 < n; ++b) {
    double E1 = g->e_min * pow(g->e_max / g->e_min, (double)(b + 1) / (double)(n - 1));
    double s0 = 0, s1 = 0;
    for (int k = 0; k < 5; ++k) { s0 += g->xs[k * n + b]; s1 += g->xs[k * n + b + 1]; }
    double v1 = sqrt(2.0 * E1 * (double)QE / (double)ME);
    double nu = g->density * (s0 > s1 ? s0 : s1) * v1;
    if (nu > best) best = nu;
  }
  return best;
}

/* First crossing of segment p0 -> p1 with any cell (Moller-Trumbore), smallest
 * parameter t in (0, 1]; returns the cell index or -1. */
static int64_t first_hit(int64_t N, const tri_t *T, const double *p0, const double *p1, double *t_hit) {
  real ox = p0[0], oy = p0[1], oz = p0[2];
  v3 o = mk(ox, oy, oz);
  v3 dir = sub(ld(p1), o);
  int64_t best = -1;
  real bt = 2.0L;
  for (int64_t k = 0; k < N; ++k) {
    v3 e1 = sub(T[k].p[1], T[k].p[0]), e2 = sub(T[k].p[2], T[k].p[0]);
    v3 pv = crs(dir, e2);
    real det = dot(e1, pv);
    if (det == 0) continue;
    real inv = 1.0L / det;
    v3 tv = sub(o, T[k].p[0]);
    real u = dot(tv, pv) * inv;
    if (u < 0 || u > 1) continue;
    v3 qv = crs(tv, e1);
    real v = dot(dir, qv) * inv;
    if (v < 0 || u + v > 1) continue;
    real t = dot(e2, qv) * inv;
    if (t > 0 && t <= 1 && t < bt) { bt = t; best = k; }
  }
  *t_hit = (double)bt;
  return best;
}

static void isotropic(double u2, double u3, double *d) {
  double ct = 1.0 - 2.0 * u2, st = sqrt(fmax(0.0, 1.0 - ct * ct)), ph = 2.0 * M_PI * u3;
  d[0] = st * cos(ph); d[1] = st * sin(ph); d[2] = ct;
}

/* Table value at eps (eV), linear in the normalised lethargy of eq. (leth)
 * between log-spaced nodes, clamped to the end nodes (as xs_at). */
static double table_at(const oc_gas *g, const double *tab, double eps) {
  int n = g->n_nodes;
  if (!(eps > g->e_min)) return tab[0];
  if (eps >= g->e_max) return tab[n - 1];
  double p = (double)(n - 1) * (log(eps / g->e_min) / log(g->e_max / g->e_min));
  int i = (int)floor(p);
  if (i >= n - 1) i = n - 2;
  double fr = p - (double)i;
  return tab[i] * (1.0 - fr) + tab[i + 1] * fr;
}

/* Scattering angle of eq. (anisotrop) for a uniform R in [0, 1):
 * cos theta = 1 - 2R(1 - xi)/(1 + xi(1 - 2R)). */
double oc_aniso_cos(double xi, double R) { return 1.0 - 2.0 * R * (1.0 - xi) / (1.0 + xi * (1.0 - 2.0 * R)); }

/* Unit vector at polar angle theta (cos ct) and azimuth 2 pi u about the unit
 * vector d: basis e1 = (a x d)/|a x d| with a the z axis (x axis when d is
 * within 25.8 degrees of z), e2 = d x e1. */
static void rotate_about(const double *d, double ct, double u, double *out) {
  double a[3] = {0.0, 0.0, 1.0};
  if (fabs(d[2]) >= 0.9) { a[0] = 1.0; a[2] = 0.0; }
  double e1[3] = {a[1] * d[2] - a[2] * d[1], a[2] * d[0] - a[0] * d[2], a[0] * d[1] - a[1] * d[0]};
  double l = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  for (int k = 0; k < 3; ++k) e1[k] /= l;
  double e2[3] = {d[1] * e1[2] - d[2] * e1[1], d[2] * e1[0] - d[0] * e1[2], d[0] * e1[1] - d[1] * e1[0]};
  double st = sqrt(fmax(0.0, 1.0 - ct * ct)), ph = 2.0 * M_PI * u;
  double cp = cos(ph), sp = sin(ph);
  for (int k = 0; k < 3; ++k) out[k] = ct * d[k] + st * (cp * e1[k] + sp * e2[k]);
}

/* Children of one particle and step: pairs (electron, cation) in slots
 * [(i*mi + c)*2 + {0, 1}]. */
typedef struct {
  int64_t i;
  int mi;
  int32_t *n_child;
  double *child_x, *child_v;
} oc_kids;

static int add_pair(oc_kids *K, const double *xe, const double *ve, const double *xc, const double *vc) {
  int nc = K->n_child[K->i];
  if (nc >= K->mi) return 0;
  double *ce = K->child_x + ((K->i * K->mi + nc) * 2 + 0) * 3, *cv = K->child_v + ((K->i * K->mi + nc) * 2 + 0) * 3;
  double *ix = K->child_x + ((K->i * K->mi + nc) * 2 + 1) * 3, *iv = K->child_v + ((K->i * K->mi + nc) * 2 + 1) * 3;
  for (int d = 0; d < 3; ++d) { ce[d] = xe[d]; cv[d] = ve[d]; ix[d] = xc[d]; iv[d] = vc[d]; }
  K->n_child[K->i] = nc + 1;
  return 1;
}

/* Counter slots (shared by both collision models). */
enum { CN_EL = 0, CN_NULL = 5, CN_ION = 6, CN_OVF = 7, CN_CAP = 8, CN_DROP = 9, CN_PEN = 10, CN_COUNT = 11 };

/* Real interaction `proc` (elastic, exc1, exc2, ionisation, attachment) of an
 * electron of energy eps (eV) at X with velocity V (section 3.4.3).  u2, u3:
 * the collision's own uniforms; c4 (counter word 3 free) and key give the
 * extra draws: word 3 = 2k + 1 for the ionisation / Penning words, 0x80000000
 * | k for the Penning cation.  Returns 1 when the electron became an anion. */
static int electron_interaction(const oc_gas *g, int proc, double eps, double *X, double *Vv, double u2, double u3,
                                uint32_t *c4, const uint32_t *key, uint32_t k, oc_kids *K, int64_t *cnt) {
  const double qe = (double)QE, me = (double)ME, ke = (double)k_e();
  const double e_therm = 1.5 * (double)KB * g->temperature; /* J */
  double v2 = Vv[0] * Vv[0] + Vv[1] * Vv[1] + Vv[2] * Vv[2];
  double vm = sqrt(v2);
  double dir[3];
  if (proc == 0) { /* elastic, recoil loss 2 m_e/M (1 - cos theta) */
    double ct;
    if (g->xi && vm > 0) { /* eq. (anisotrop) about the incident direction */
      double xi = table_at(g, g->xi, eps);
      ct = oc_aniso_cos(xi, u2);
      double d0[3] = {Vv[0] / vm, Vv[1] / vm, Vv[2] / vm};
      rotate_about(d0, ct, u3, dir);
    } else {
      isotropic(u2, u3, dir);
      ct = (vm > 0) ? (dir[0] * Vv[0] + dir[1] * Vv[1] + dir[2] * Vv[2]) / vm : 1.0;
    }
    double e2 = eps * (1.0 - 2.0 * me / g->m_gas * (1.0 - ct));
    double s = sqrt(2.0 * e2 * qe / me);
    for (int d = 0; d < 3; ++d) Vv[d] = s * dir[d];
    return 0;
  }
  if (proc == 1 || proc == 2 || proc == 3) {
    double e_res = (proc == 3) ? eps - g->thr[3] - e_therm / qe : -1.0;
    if (proc != 3 || e_res <= 0.0) { /* excitation (or sub-threshold ionisation) */
      double e2 = eps - g->thr[proc];
      if (e2 < 0) e2 = 0;
      isotropic(u2, u3, dir);
      double s = sqrt(2.0 * e2 * qe / me);
      for (int d = 0; d < 3; ++d) Vv[d] = s * dir[d];
      if (proc != 3 && g->penning_prob > 0.0 && g->thr[proc] >= g->penning_level) {
        /* Penning transfer (section 3.4.4): the excited state ionises the
         * quencher with probability penning_prob; the released electron
         * takes the excess energy thr - penning_level, the cation a thermal
         * speed, both isotropic, at the collision point */
        uint32_t w2[4], w3[4];
        c4[3] = 2u * k + 1u;
        oc_philox4x32_10(c4, key, w2);
        if (u01(w2[0]) < g->penning_prob) {
          c4[3] = 0x80000000u | k;
          oc_philox4x32_10(c4, key, w3);
          double de[3], dc[3], ve[3], vc[3];
          isotropic(u01(w2[1]), u01(w2[2]), de);
          isotropic(u01(w3[0]), u01(w3[1]), dc);
          double se = sqrt(2.0 * (g->thr[proc] - g->penning_level) * qe / me);
          double si = sqrt(2.0 * e_therm / g->m_cation);
          for (int d = 0; d < 3; ++d) { ve[d] = se * de[d]; vc[d] = si * dc[d]; }
          cnt[CN_PEN] += 1;
          if (!add_pair(K, X, ve, X, vc)) cnt[CN_DROP] += 2;
        }
      }
      return 0;
    }
    /* ionisation, eq. (distIoni) */
    uint32_t w2[4];
    c4[3] = 2u * k + 1u;
    oc_philox4x32_10(c4, key, w2);
    double uh[3], ud[3];
    isotropic(u01(w2[0]), u01(w2[1]), uh);
    isotropic(u01(w2[2]), u01(w2[3]), ud);
    double eres_j = e_res * qe;
    /* eq. (distIoni) with the energy in eV (volts): r = k_e e / (2 E_res[eV]),
     * i.e. the separation at which the pair's Coulomb energy k_e e^2 / r is
     * 2 E_res (the same convention gives 4.59e-11 m for eq. (distRecomb)
     * at 15.7 eV). */
    double r = ke * qe * qe / (2.0 * eres_j);
    double s = sqrt(2.0 * (0.5 * eres_j) / me);
    double si = sqrt(2.0 * e_therm / g->m_cation);
    double xe[3], ve[3], vc[3];
    for (int d = 0; d < 3; ++d) { xe[d] = X[d] - r * uh[d]; ve[d] = -s * uh[d]; vc[d] = si * ud[d]; }
    if (!add_pair(K, xe, ve, X, vc)) cnt[CN_DROP] += 2;
    for (int d = 0; d < 3; ++d) { X[d] += r * uh[d]; Vv[d] = s * uh[d]; }
    return 0;
  }
  /* attachment: anion, momentum conserved with the gas at rest */
  for (int d = 0; d < 3; ++d) Vv[d] *= me / g->m_anion;
  return 1;
}

/* Ion collision: 0 = isotropic in the centre of mass (gas at rest), 1 =
 * backscatter (charge exchange: the ion takes a thermal gas velocity). */
static void ion_interaction(const oc_gas *g, int sp, int proc, double *Vv, double u2, double u3, uint32_t *c4,
                            const uint32_t *key, uint32_t k) {
  double vm = sqrt(Vv[0] * Vv[0] + Vv[1] * Vv[1] + Vv[2] * Vv[2]);
  if (proc == 0) {
    double mion = (sp == 1) ? g->m_cation : g->m_anion;
    double fm = mion / (mion + g->m_gas), fM = g->m_gas / (mion + g->m_gas);
    double dir[3];
    isotropic(u2, u3, dir);
    for (int d = 0; d < 3; ++d) Vv[d] = fm * Vv[d] + fM * vm * dir[d];
  } else {
    uint32_t w2[4];
    c4[3] = 2u * k + 1u;
    oc_philox4x32_10(c4, key, w2);
    double sd = sqrt((double)KB * g->temperature / g->m_gas);
    double r1 = sqrt(-2.0 * log(u01(w2[0]))), r2 = sqrt(-2.0 * log(u01(w2[2])));
    Vv[0] = sd * r1 * cos(2.0 * M_PI * u01(w2[1]));
    Vv[1] = sd * r1 * sin(2.0 * M_PI * u01(w2[1]));
    Vv[2] = sd * r2 * cos(2.0 * M_PI * u01(w2[3]));
  }
}

static int outside_box(const oc_step *p, const double *X) {
  return X[0] < p->box_lo[0] || X[0] > p->box_hi[0] || X[1] < p->box_lo[1] || X[1] > p->box_hi[1] ||
         X[2] < p->box_lo[2] || X[2] > p->box_hi[2];
}

/* Outputs per particle i (arrays of n): new state in place (x, v), species in
 * place, status (OC_*), hit cell (or -1), event counters, and up to
 * max_ion_per_step child pairs: child_x/child_v [(i*max_ion + c)*2 + {0 e-, 1
 * cation}][3], n_child[i].  counters (CN_*): real collisions by electron
 * process (5 slots), null, ion collisions, rate overflows, flight cap
 * reached, children dropped, Penning transfers.  */
void oc_mc_step(int64_t n, double *x, double *v, int8_t *species, const int64_t *id, const double *E,
                const uint8_t *skip, const oc_gas *g, const oc_step *p, int64_t N, const double *a,
                const double *b, const double *c, int8_t *status, int64_t *hit, int32_t *n_child,
                double *child_x, double *child_v, int64_t *counters) {
  tri_t *T = (tri_t *)malloc(sizeof(tri_t) * (size_t)(N > 0 ? N : 1));
  for (int64_t k = 0; k < N; ++k) tri_setup(a + 3 * k, b + 3 * k, c + 3 * k, &T[k]);
  const double qe = (double)QE, me = (double)ME;
  double nu_e = oc_nu_max_electron(g);
  double nu_i = g->density * (g->ion_xs_iso + g->ion_xs_back) * p->ion_v_cap;
  int64_t cnt[CN_COUNT] = {0};
  uint32_t key[2] = {(uint32_t)(p->seed & 0xffffffffu), (uint32_t)(p->seed >> 32)};

#pragma omp parallel for schedule(dynamic, 64) reduction(+ : cnt[:CN_COUNT])
  for (int64_t i = 0; i < n; ++i) {
    status[i] = OC_ALIVE;
    hit[i] = -1;
    n_child[i] = 0;
    if (skip && skip[i]) continue;
    oc_kids K = {i, p->max_ion_per_step, n_child, child_x, child_v};
    double X[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
    double Vv[3] = {v[3 * i], v[3 * i + 1], v[3 * i + 2]};
    int sp = species[i];
    double t = 0.0;
    int ballistic = 0;
    uint32_t c4[4] = {(uint32_t)((uint64_t)id[i] & 0xffffffffu), (uint32_t)((uint64_t)id[i] >> 32), p->step, 0};
    for (int k = 0;; ++k) {
      double m = (sp == 0) ? me : (sp == 1 ? g->m_cation : g->m_anion);
      double q = (sp == 1) ? qe : -qe;
      double acc[3] = {q * E[3 * i] / m, q * E[3 * i + 1] / m, q * E[3 * i + 2] / m};
      double numax = (sp == 0) ? nu_e : nu_i;
      double tau;
      uint32_t w[4];
      int last = 0;
      if (ballistic || k >= p->max_coll || numax <= 0) {
        if (!ballistic && numax > 0 && k >= p->max_coll) cnt[CN_CAP] += 1;
        tau = p->dt - t;
        last = 1;
      } else {
        c4[3] = 2u * (uint32_t)k;
        oc_philox4x32_10(c4, key, w);
        tau = -log(u01(w[0])) / numax;
        if (t + tau >= p->dt) { tau = p->dt - t; last = 1; }
      }
      /* constant-field flight over tau; chord tested for absorption */
      double X1[3], V1[3];
      for (int d = 0; d < 3; ++d) {
        X1[d] = X[d] + Vv[d] * tau + 0.5 * acc[d] * tau * tau;
        V1[d] = Vv[d] + acc[d] * tau;
      }
      double th;
      int64_t h = (N > 0) ? first_hit(N, T, X, X1, &th) : -1;
      if (h >= 0) { status[i] = OC_ABSORBED; hit[i] = h; break; }
      for (int d = 0; d < 3; ++d) { X[d] = X1[d]; Vv[d] = V1[d]; }
      if (outside_box(p, X)) { status[i] = OC_LEFT; break; }
      if (last) break;
      t += tau;
      double v2 = Vv[0] * Vv[0] + Vv[1] * Vv[1] + Vv[2] * Vv[2];
      double vm = sqrt(v2);
      double u1 = u01(w[1]), u2 = u01(w[2]), u3 = u01(w[3]);
      if (sp == 0) {
        double eps = 0.5 * me * v2 / qe; /* eV */
        double nuk[5], tot = 0;
        for (int kk = 0; kk < 5; ++kk) { nuk[kk] = g->density * xs_at(g, kk, eps) * vm; tot += nuk[kk]; }
        double lim = numax;
        if (tot > numax) { cnt[CN_OVF] += 1; lim = tot; }
        double sel = u1 * lim, cum = 0;
        int proc = -1;
        for (int kk = 0; kk < 5; ++kk) { cum += nuk[kk]; if (sel < cum) { proc = kk; break; } }
        if (proc < 0) { cnt[CN_NULL] += 1; continue; }
        cnt[CN_EL + proc] += 1;
        if (electron_interaction(g, proc, eps, X, Vv, u2, u3, c4, key, (uint32_t)k, &K, cnt)) {
          sp = 2;
          ballistic = 1;
        }
      } else {
        double nui = g->density * g->ion_xs_iso * vm, nub = g->density * g->ion_xs_back * vm;
        double lim = numax;
        if (nui + nub > numax) { cnt[CN_OVF] += 1; lim = nui + nub; }
        double sel = u1 * lim;
        if (sel < nui + nub) {
          ion_interaction(g, sp, sel < nui ? 0 : 1, Vv, u2, u3, c4, key, (uint32_t)k);
          cnt[CN_ION] += 1;
        } else {
          cnt[CN_NULL] += 1;
        }
      }
    }
    x[3 * i] = X[0]; x[3 * i + 1] = X[1]; x[3 * i + 2] = X[2];
    v[3 * i] = Vv[0]; v[3 * i + 1] = Vv[1]; v[3 * i + 2] = Vv[2];
    species[i] = (int8_t)sp;
  }
  for (int k = 0; k < CN_COUNT; ++k) counters[k] += cnt[k];
  free(T);
}

/* Flight of duration tau for the particles with skip[i] == 0 and status[i]
 * == OC_ALIVE: constant acceleration q E / m (E may be NULL: straight drift),
 * chord tested for absorption, then the world box.  Used by the Euler and
 * PEFRL steppers of section 3.3.5 (a drift is one PEFRL position update). */
void oc_flight(int64_t n, double *x, double *v, const int8_t *species, const double *E, const uint8_t *skip,
               const oc_gas *g, const oc_step *p, double tau, int64_t N, const double *a, const double *b,
               const double *c, int8_t *status, int64_t *hit) {
  tri_t *T = (tri_t *)malloc(sizeof(tri_t) * (size_t)(N > 0 ? N : 1));
  for (int64_t k = 0; k < N; ++k) tri_setup(a + 3 * k, b + 3 * k, c + 3 * k, &T[k]);
  const double qe = (double)QE, me = (double)ME;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    if ((skip && skip[i]) || status[i] != OC_ALIVE) continue;
    int sp = species[i];
    double m = (sp == 0) ? me : (sp == 1 ? g->m_cation : g->m_anion);
    double q = (sp == 1) ? qe : -qe;
    double X1[3], V1[3];
    for (int d = 0; d < 3; ++d) {
      double acc = E ? q * E[3 * i + d] / m : 0.0;
      X1[d] = x[3 * i + d] + v[3 * i + d] * tau + 0.5 * acc * tau * tau;
      V1[d] = v[3 * i + d] + acc * tau;
    }
    double th;
    int64_t h = (N > 0) ? first_hit(N, T, x + 3 * i, X1, &th) : -1;
    if (h >= 0) { status[i] = OC_ABSORBED; hit[i] = h; continue; }
    for (int d = 0; d < 3; ++d) { x[3 * i + d] = X1[d]; v[3 * i + d] = V1[d]; }
    if (outside_box(p, x + 3 * i)) status[i] = OC_LEFT;
  }
  free(T);
}

/* Per-step collision model of section 3.4.2: after the drift over dt, each
 * live particle collides with probability 1 - exp(-nu_tot dt) (nu_tot = N
 * sigma_tot(E) v, gas at rest), the process chosen with probabilities
 * nu_k / nu_tot (one draw: counter (id, step, 0)), then the same
 * interactions as above at the end point.  At most one collision per step. */
void oc_collide_step(int64_t n, double *x, double *v, int8_t *species, const int64_t *id, const uint8_t *skip,
                     const oc_gas *g, const oc_step *p, const int8_t *status, int32_t *n_child, double *child_x,
                     double *child_v, int64_t *counters) {
  const double qe = (double)QE, me = (double)ME;
  int64_t cnt[CN_COUNT] = {0};
  uint32_t key[2] = {(uint32_t)(p->seed & 0xffffffffu), (uint32_t)(p->seed >> 32)};
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : cnt[:CN_COUNT])
  for (int64_t i = 0; i < n; ++i) {
    n_child[i] = 0;
    if ((skip && skip[i]) || status[i] != OC_ALIVE) continue;
    oc_kids K = {i, p->max_ion_per_step, n_child, child_x, child_v};
    double *X = x + 3 * i, *Vv = v + 3 * i;
    int sp = species[i];
    uint32_t c4[4] = {(uint32_t)((uint64_t)id[i] & 0xffffffffu), (uint32_t)((uint64_t)id[i] >> 32), p->step, 0};
    uint32_t w[4];
    oc_philox4x32_10(c4, key, w);
    double v2 = Vv[0] * Vv[0] + Vv[1] * Vv[1] + Vv[2] * Vv[2];
    double vm = sqrt(v2);
    double u0 = u01(w[0]), u1 = u01(w[1]), u2 = u01(w[2]), u3 = u01(w[3]);
    if (sp == 0) {
      double eps = 0.5 * me * v2 / qe;
      double nuk[5], tot = 0;
      for (int kk = 0; kk < 5; ++kk) { nuk[kk] = g->density * xs_at(g, kk, eps) * vm; tot += nuk[kk]; }
      if (!(u0 < -expm1(-tot * p->dt))) { cnt[CN_NULL] += 1; continue; }
      double sel = u1 * tot, cum = 0;
      int proc = 4;
      for (int kk = 0; kk < 5; ++kk) { cum += nuk[kk]; if (sel < cum) { proc = kk; break; } }
      cnt[CN_EL + proc] += 1;
      if (electron_interaction(g, proc, eps, X, Vv, u2, u3, c4, key, 0u, &K, cnt)) species[i] = 2;
    } else {
      double nui = g->density * g->ion_xs_iso * vm, nub = g->density * g->ion_xs_back * vm;
      if (!(u0 < -expm1(-(nui + nub) * p->dt))) { cnt[CN_NULL] += 1; continue; }
      ion_interaction(g, sp, (u1 * (nui + nub) < nui) ? 0 : 1, Vv, u2, u3, c4, key, 0u);
      cnt[CN_ION] += 1;
    }
  }
  for (int k = 0; k < CN_COUNT; ++k) counters[k] += cnt[k];
}

/* Central difference of L = sum_i w_i . E(x_i) (targets = sources = the n
 * particles, cells with sigma) with respect to coordinate `axis` of particle
 * m, step h.  Only the terms that involve particle m change, so they are
 * re-summed directly (pairwise differences of the kernel), which keeps the
 * difference accurate at any n. */
double oc_fd_particle(int64_t n, const double *x, const double *q, const double *w, double soft, int64_t N,
                      const double *a, const double *b, const double *c, const double *sigma, int64_t m, int axis,
                      double h) {
  real ke = k_e(), s2 = (real)soft * (real)soft;
  v3 xm = ld(x + 3 * m);
  v3 dp = mk(axis == 0 ? h : 0, axis == 1 ? h : 0, axis == 2 ? h : 0);
  v3 xp = add(xm, dp), xn = sub(xm, dp);
  real acc = 0;
  /* source role: other targets see particle m move */
#pragma omp parallel for reduction(+ : acc) schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    if (i == m) continue;
    v3 xi = ld(x + 3 * i);
    v3 d1 = sub(xi, xp), d2 = sub(xi, xn);
    real S1 = dot(d1, d1) + s2, S2 = dot(d2, d2) + s2;
    real i1 = 1.0L / (S1 * sqrtl(S1)), i2 = 1.0L / (S2 * sqrtl(S2));
    v3 dK = sub(scl(d1, i1), scl(d2, i2));
    acc += (real)q[m] * dot(ld(w + 3 * i), dK);
  }
  /* target role: the field at particle m itself */
  real acc2 = 0;
#pragma omp parallel for reduction(+ : acc2) schedule(static)
  for (int64_t j = 0; j < n; ++j) {
    if (j == m) continue;
    v3 xj = ld(x + 3 * j);
    v3 d1 = sub(xp, xj), d2 = sub(xn, xj);
    real S1 = dot(d1, d1) + s2, S2 = dot(d2, d2) + s2;
    real i1 = 1.0L / (S1 * sqrtl(S1)), i2 = 1.0L / (S2 * sqrtl(S2));
    v3 dK = sub(scl(d1, i1), scl(d2, i2));
    acc2 += (real)q[j] * dot(ld(w + 3 * m), dK);
  }
  real acc3 = 0;
  if (N > 0) {
#pragma omp parallel for reduction(+ : acc3) schedule(static)
    for (int64_t k = 0; k < N; ++k) {
      tri_t T;
      tri_setup(a + 3 * k, b + 3 * k, c + 3 * k, &T);
      v3 e1, e2;
      tri_IV_IE(&T, xp, NULL, &e1);
      tri_IV_IE(&T, xn, NULL, &e2);
      acc3 += (real)sigma[k] * dot(ld(w + 3 * m), sub(e1, e2));
    }
  }
  return (double)(ke * (acc + acc2 + acc3) / (2.0L * (real)h));
}

/* Influence of point charges on the collocation equations (section 3.3.2,
 * eqs. (potpart), (fldpart), (BEMpotpart), (BEMfldpart)).  The charges'
 * potential and field averaged over cell i,
 *   Vbar_i = k_e / A_i sum_p q_p int_{C_i} dS / |r - x_p|      = k_e/A_i sum_p q_p IV_i(x_p)
 *   Ebar_i = k_e / A_i sum_p q_p int_{C_i} (r - x_p)/|r - x_p|^3 dS = -k_e/A_i sum_p q_p IE_i(x_p)
 * modify the left-hand side: ed rows V_i - Vbar_i, dd rows
 * sigma_F,i - (eps_2 - eps_1) Ebar_i . n_i with absolute permittivities
 * eps = eps0 eps_r. */
void oc_influence(int64_t N, const double *a, const double *b, const double *c, const int8_t *kind,
                  const double *eps1, const double *eps2, const double *rhs, int64_t n, const double *x,
                  const double *q, double *rhs_out, double *vbar, double *ebar) {
  real ke = k_e();
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < N; ++i) {
    tri_t T;
    tri_setup(a + 3 * i, b + 3 * i, c + 3 * i, &T);
    real sv = 0, ex = 0, ey = 0, ez = 0;
    for (int64_t p = 0; p < n; ++p) {
      real iv;
      v3 ie;
      tri_IV_IE(&T, ld(x + 3 * p), &iv, &ie);
      real qp = q[p];
      sv += qp * iv;
      ex += qp * ie.x; ey += qp * ie.y; ez += qp * ie.z;
    }
    real vb = ke * sv / T.area;
    v3 eb = scl(mk(ex, ey, ez), -ke / T.area);
    if (vbar) vbar[i] = (double)vb;
    if (ebar) { ebar[3 * i] = (double)eb.x; ebar[3 * i + 1] = (double)eb.y; ebar[3 * i + 2] = (double)eb.z; }
    if (kind[i] == 0)
      rhs_out[i] = (double)((real)rhs[i] - vb);
    else
      rhs_out[i] = (double)((real)rhs[i] - EPS0 * ((real)eps2[i] - (real)eps1[i]) * dot(eb, T.n));
  }
}
