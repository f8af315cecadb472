/*
 * bssn_oracle.c -- TEST INFRASTRUCTURE: the plain CPU oracle.
 *
 * A deliberately direct evaluation of the discretised BSSN evolution of
 * arXiv:2505.00097. Every quantity is built with full 3x3(x3x3) index loops in
 * the order and notation of the paper's equations, with no blocking, fusion
 * or symmetry tricks, so that each step can be compared with the paper by
 * eye. It is used only by tests/, the smoke check and the CPU baseline of the
 * benchmark, to check the HIP library; it shares no source with that library.
 *
 * Discretisation (the plain definition the GPU path must reproduce):
 *   - cell-centred logical grid, N_G ghost layers (Sec. 3);
 *   - every partial derivative of an evolved rescaled variable is a finite
 *     difference of order N_FD = 2 (N_G - 1) (Sec. 3: N_G = N_FD/2 + 1 ghost
 *     layers; the benchmark runs use N_FD = 4, the production head-on run of
 *     Sec. 4.1 N_FD = 8): centred (N_FD + 1)-point stencils, their tensor
 *     product for mixed derivatives, and for the advection terms beta^k d_k
 *     the same width of stencil shifted one point upwind (Sec. 3, second
 *     paragraph);
 *   - every reference-metric quantity (S_i, its derivatives, Gammahat and its
 *     derivatives) is evaluated analytically (Sec. 2.2, Eq. 22);
 *   - RHS = Eqs. 7-15 with Eq. 12 (Sec. 2.1), unrescaled/rescaled per Sec. 2.2;
 *   - optional Kreiss-Oliger dissipation added to each rescaled right-hand
 *     side (Sec. 4.1, strengths for gauge and metric variables);
 *   - boundary fill after every RK substage: outer extrapolation, then inner
 *     parity copies (Sec. 3, ordered boundary steps); or, with the radiation
 *     outer boundary, the pure-outer points evolved by a Sommerfeld condition
 *     and only the inner copies refilled;
 *   - classical RK4 (Sec. 4.2.1 footnote), or the three-stage strong-
 *     stability-preserving Runge-Kutta scheme the production head-on run of
 *     Sec. 4.1 uses (SSPRK3 of Gottlieb, Shu and Tadmor, cited there).
 * Readings where the paper is silent or garbled are marked "Reading:".
 *
 * Precision: every quantity has the type `real` (oracle_real): double in the
 * FP64 oracle (liboracle.so); the same source compiled with
 * -DORACLE_REAL="long double" (liboracle_ld.so) is the extended-precision
 * reference against which both the FP64 oracle and the GPU are measured at
 * ill-conditioned points. Literal fractions are written as (real)a / b so
 * that they are rounded in the build's own precision.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared [-DORACLE_REAL="long double"].
 */
#include "bssn_oracle.h"

#include <tgmath.h> /* math routines chosen by argument type: double or long double */
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NGF ORACLE_NGF

typedef oracle_real real; /* double, or long double in the reference build */

/* gridfunction order (alphabetical names of the rescaled variables) */
enum {
  ADD00, ADD01, ADD02, ADD11, ADD12, ADD22, ALPHA, BETU0, BETU1, BETU2, CF,
  HDD00, HDD01, HDD02, HDD11, HDD12, HDD22, LAMU0, LAMU1, LAMU2, TRK,
  VETU0, VETU1, VETU2
};

/* position of the symmetric pair (i,j) in the 00,01,02,11,12,22 order */
static const int SYM[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

/* tensor type of each gridfunction: 0 scalar, 1 vector (index in vidx),
 * 2 symmetric rank-2 (indices in tidx) */
static const int GF_TYPE[NGF] = {2, 2, 2, 2, 2, 2, 0, 1, 1, 1, 0,
                                 2, 2, 2, 2, 2, 2, 1, 1, 1, 0, 1, 1, 1};
static const int GF_I[NGF] = {0, 0, 0, 1, 1, 2, 0, 0, 1, 2, 0,
                              0, 0, 0, 1, 1, 2, 0, 1, 2, 0, 0, 1, 2};
static const int GF_J[NGF] = {0, 1, 2, 1, 2, 2, 0, 0, 0, 0, 0,
                              0, 1, 2, 1, 2, 2, 0, 0, 0, 0, 0, 0, 0};

/* ------------------------------------------------------------------------ */
/* Grid (Sec. 3, first paragraph): logical domain [xxmin, xxmax], N cells,
 * cell-centred points xxmin + (j - ng + 1/2) dxx.                           */
#define MAXR 5 /* centred stencil radius up to 5: N_FD up to 10 */

/* Finite-difference weights for N_FD = 2R (R = N_G - 1), unit spacing:
 *   D f  = sum_{j=1..R} d1[j] (f_j - f_-j)
 *   D2 f = sum_{j=1..R} d2[j] ((f_j - f_0) + (f_-j - f_0))
 *   U+ f = sum_{m != 1} up[m + R - 1] (f_m - f_1),  m = -(R-1) .. R+1
 *   KO f = sum_{j=1..R+1} ko[j] ((f_j - f_0) + (f_-j - f_0))
 * The sums are grouped into differences (the weights of each stencil add up
 * to zero), so a constant field has exactly zero derivatives.               */
typedef struct {
  int R;
  real d1[MAXR + 1], d2[MAXR + 1], up[2 * MAXR + 1], ko[MAXR + 2];
} Sten;

typedef struct {
  oracle_params p;
  int n[3];
  long long np;     /* points incl. ghosts */
  long long st[3];  /* flat-index strides */
  real xxmin[3], xxmax[3], dxx[3];
  Sten fd;
} Grid;

int oracle_check(const oracle_params* p) {
  if (!p) return -1;
  if (p->coord < 0 || p->coord > 2) return -1;
  if (p->ng < 3 || p->ng > MAXR + 1) return -1;
  if (p->bc_kind != 0 && p->bc_kind != 1) return -1;
  /* the periodic phi direction may have fewer cells than ghost layers (its
   * ghosts wrap around as often as needed); the others need N >= ng */
  const int dphi = p->coord == 1 ? 1 : 2;
  for (int d = 0; d < 3; d++)
    if (d != dphi && p->N[d] < p->ng) return -1;
  if (p->N[dphi] < 2) return -1;
  if (p->coord == 1) {
    if (p->N[1] % 2) return -1;
    if (!(p->ampl[0] > 0) || !(p->ampl[2] > 0) || !(p->sinhw[0] > 0) || !(p->sinhw[2] > 0))
      return -1;
  } else {
    if (p->N[2] % 2) return -1;
    if (!(p->ampl[0] > 0)) return -1;
    if (p->coord == 0 && !(p->sinhw[0] > 0)) return -1;
  }
  return 0;
}

/* w[j] with f^(der)(0) ~ sum_j w[j] f(m[j]) (der = 1 or 2): the weights are
 * the derivatives at 0 of the Lagrange basis polynomials through the n
 * integer nodes m[], L_j(x) = prod_{i != j} (x - m_i)/(m_j - m_i).          */
static void lagrange_weights(int n, const int* m, int der, real* w) {
  for (int j = 0; j < n; j++) {
    real s = 0.0;
    for (int k = 0; k < n; k++) {
      if (k == j) continue;
      if (der == 1) {
        real prod = 1.0 / (real)(m[j] - m[k]);
        for (int i = 0; i < n; i++)
          if (i != j && i != k) prod *= (0.0 - m[i]) / (real)(m[j] - m[i]);
        s += prod;
      } else {
        for (int l = 0; l < n; l++) {
          if (l == j || l == k) continue;
          real prod = 1.0 / ((real)(m[j] - m[k]) * (real)(m[j] - m[l]));
          for (int i = 0; i < n; i++)
            if (i != j && i != k && i != l) prod *= (0.0 - m[i]) / (real)(m[j] - m[i]);
          s += prod;
        }
      }
    }
    w[j] = s;
  }
}

/* Kreiss-Oliger dissipation of order 2R + 1 (Sec. 4.1 runs N_FD = 8 with
 * ninth-order dissipation operators). Reading: the operator is the
 * difference of order 2p = 2R + 2, radius p = N_G, scaled to
 * (-1)^(p+1) delta^2p f / (4^p h), whose Fourier symbol is -sin^2p(theta/2)/h
 * (it damps the grid-scale modes and is O(h^(2p-1)) on smooth data); with
 * delta^2p f = sum_j (-1)^(j+p) C(2p, p+j) f_j the grouped weight of the
 * pair +-j is (-1)^(j+1) C(2p, p+j) / 4^p.                                  */
static void build_stencils(int R, Sten* S) {
  int m[2 * MAXR + 3];
  real w[2 * MAXR + 3];
  S->R = R;
  for (int j = 0; j <= 2 * R; j++) m[j] = j - R; /* centred nodes -R..R */
  lagrange_weights(2 * R + 1, m, 1, w);
  for (int j = 0; j <= R; j++) S->d1[j] = w[R + j];
  lagrange_weights(2 * R + 1, m, 2, w);
  for (int j = 0; j <= R; j++) S->d2[j] = w[R + j];
  for (int j = 0; j <= 2 * R; j++) m[j] = j - R + 1; /* shifted nodes -(R-1)..R+1 */
  lagrange_weights(2 * R + 1, m, 1, w);
  for (int j = 0; j <= 2 * R; j++) S->up[j] = w[j];
  const int p = R + 1;
  real binom = 1.0, scale = 1.0; /* C(2p, p + j), 4^-p */
  for (int k = 0; k < p; k++) scale /= 4.0;
  for (int j = p; j >= 0; j--) {
    if (j < p) binom = binom * (real)(p + j + 1) / (real)(p - j); /* C(2p,p+j) from C(2p,p+j+1) */
    S->ko[j] = ((j + 1) % 2 == 0 ? 1.0 : -1.0) * binom * scale;
  }
}

static int grid_setup(const oracle_params* p, Grid* G) {
  if (oracle_check(p)) return -1;
  G->p = *p;
  const real PI = (real)3.14159265358979323846264338327950288L;
  if (p->coord == 1) { /* SinhCylindrical: (xx0, phi, xx2) */
    G->xxmin[0] = 0.0; G->xxmax[0] = 1.0;
    G->xxmin[1] = -PI; G->xxmax[1] = PI;
    G->xxmin[2] = -1.0; G->xxmax[2] = 1.0;
  } else { /* (Sinh)Spherical: (xx0, theta, phi) */
    G->xxmin[0] = 0.0; G->xxmax[0] = 1.0;
    G->xxmin[1] = 0.0; G->xxmax[1] = PI;
    G->xxmin[2] = -PI; G->xxmax[2] = PI;
  }
  for (int d = 0; d < 3; d++) {
    G->n[d] = p->N[d] + 2 * p->ng;
    G->dxx[d] = (G->xxmax[d] - G->xxmin[d]) / (real)p->N[d];
  }
  G->st[0] = 1;
  G->st[1] = G->n[0];
  G->st[2] = (long long)G->n[0] * G->n[1];
  G->np = G->st[2] * G->n[2];
  build_stencils(p->ng - 1, &G->fd);
  return 0;
}

static real xx_of(const Grid* G, int d, int j) {
  return G->xxmin[d] + ((real)(j - G->p.ng) + 0.5) * G->dxx[d];
}

real oracle_xx(const oracle_params* p, int d, int j) {
  Grid G;
  if (grid_setup(p, &G)) return NAN;
  return xx_of(&G, d, j);
}

/* ------------------------------------------------------------------------ */
/* Radial map of Eq. 22: x' = A sinh(x/w)/sinh(1/w), with its first three
 * derivatives; the uniform map x' = A x for plain Spherical.               */
static void radial_map(int linear, real A, real w, real x, real out[4]) {
  if (linear) {
    out[0] = A * x; out[1] = A; out[2] = 0.0; out[3] = 0.0;
    return;
  }
  const real s = sinh(1.0 / w);
  out[0] = A * sinh(x / w) / s;
  out[1] = A * cosh(x / w) / (w * s);
  out[2] = A * sinh(x / w) / (w * w * s);
  out[3] = A * cosh(x / w) / (w * w * w * s);
}

/* inverse of radial_map's value */
static real radial_map_inv(int linear, real A, real w, real r) {
  if (linear) return r / A;
  return w * asinh(r * sinh(1.0 / w) / A);
}

/* Scale factors S_(i) = sqrt(gammahat_ii) of the flat reference metric in the
 * logical coordinates (Sec. 2.2), with analytic sign, and their first and
 * second logical derivatives: dS[i][k] = d_k S_i, ddS[i][k][l] = d_k d_l S_i.
 *   (Sinh)Spherical: gammahat = diag(r'^2, r^2, r^2 sin^2 theta)
 *   SinhCylindrical: gammahat = diag(rho'^2, rho^2, z'^2)                  */
static void scale_factors(const Grid* G, const real xx[3], real S[3], real dS[3][3],
                          real ddS[3][3][3]) {
  memset(dS, 0, 9 * sizeof(real));
  memset(ddS, 0, 27 * sizeof(real));
  const oracle_params* p = &G->p;
  if (p->coord == 1) {
    real R[4], Z[4];
    radial_map(0, p->ampl[0], p->sinhw[0], xx[0], R);
    radial_map(0, p->ampl[2], p->sinhw[2], xx[2], Z);
    S[0] = R[1]; S[1] = R[0]; S[2] = Z[1];
    dS[0][0] = R[2]; dS[1][0] = R[1]; dS[2][2] = Z[2];
    ddS[0][0][0] = R[3]; ddS[1][0][0] = R[2]; ddS[2][2][2] = Z[3];
  } else {
    real R[4];
    radial_map(p->coord == 2, p->ampl[0], p->sinhw[0], xx[0], R);
    const real st = sin(xx[1]), ct = cos(xx[1]);
    S[0] = R[1]; S[1] = R[0]; S[2] = R[0] * st;
    dS[0][0] = R[2];
    dS[1][0] = R[1];
    dS[2][0] = R[1] * st; dS[2][1] = R[0] * ct;
    ddS[0][0][0] = R[3];
    ddS[1][0][0] = R[2];
    ddS[2][0][0] = R[2] * st;
    ddS[2][0][1] = ddS[2][1][0] = R[1] * ct;
    ddS[2][1][1] = -R[0] * st;
  }
}

void oracle_scalefactors(const oracle_params* p, const real xx[3], real S[3], real dS[9],
                         real ddS[27]) {
  Grid G;
  if (grid_setup(p, &G)) return;
  real a[3][3], b[3][3][3];
  scale_factors(&G, xx, S, a, b);
  memcpy(dS, a, sizeof a);
  memcpy(ddS, b, sizeof b);
}

/* Cartesian position (Eqs. 18-20 for the spherical family; x = rho cos phi,
 * y = rho sin phi, z for the cylindrical one).                              */
static void xx_to_cart(const Grid* G, const real xx[3], real x[3]) {
  const oracle_params* p = &G->p;
  real R[4];
  if (p->coord == 1) {
    real Z[4];
    radial_map(0, p->ampl[0], p->sinhw[0], xx[0], R);
    radial_map(0, p->ampl[2], p->sinhw[2], xx[2], Z);
    x[0] = R[0] * cos(xx[1]);
    x[1] = R[0] * sin(xx[1]);
    x[2] = Z[0];
  } else {
    radial_map(p->coord == 2, p->ampl[0], p->sinhw[0], xx[0], R);
    x[0] = R[0] * sin(xx[1]) * cos(xx[2]);
    x[1] = R[0] * sin(xx[1]) * sin(xx[2]);
    x[2] = R[0] * cos(xx[1]);
  }
}

void oracle_xx_to_cart(const oracle_params* p, const real xx[3], real x[3]) {
  Grid G;
  if (grid_setup(p, &G)) return;
  xx_to_cart(&G, xx, x);
}

/* Jacobian J[i][a] = d x^a / d xx^i of the Cartesian map above. */
static void jacobian(const Grid* G, const real xx[3], real J[3][3]) {
  const oracle_params* p = &G->p;
  real R[4];
  if (p->coord == 1) {
    real Z[4];
    radial_map(0, p->ampl[0], p->sinhw[0], xx[0], R);
    radial_map(0, p->ampl[2], p->sinhw[2], xx[2], Z);
    const real cp = cos(xx[1]), sp = sin(xx[1]);
    J[0][0] = R[1] * cp;  J[0][1] = R[1] * sp; J[0][2] = 0.0;
    J[1][0] = -R[0] * sp; J[1][1] = R[0] * cp; J[1][2] = 0.0;
    J[2][0] = 0.0;        J[2][1] = 0.0;       J[2][2] = Z[1];
  } else {
    radial_map(p->coord == 2, p->ampl[0], p->sinhw[0], xx[0], R);
    const real st = sin(xx[1]), ct = cos(xx[1]), sp = sin(xx[2]), cp = cos(xx[2]);
    J[0][0] = R[1] * st * cp; J[0][1] = R[1] * st * sp; J[0][2] = R[1] * ct;
    J[1][0] = R[0] * ct * cp; J[1][1] = R[0] * ct * sp; J[1][2] = -R[0] * st;
    J[2][0] = -R[0] * st * sp; J[2][1] = R[0] * st * cp; J[2][2] = 0.0;
  }
}

/* Rescaled basis e~_(i) = e^_(i) / S_(i) with e^_(i) = d x / d xx^i (Sec. 2.2),
 * e[i][a] = Cartesian component a of e~_(i).                                */
static void rescaled_basis(const Grid* G, const real xx[3], real e[3][3]) {
  real S[3], dS[3][3], ddS[3][3][3];
  scale_factors(G, xx, S, dS, ddS);
  real J[3][3];
  jacobian(G, xx, J);
  for (int i = 0; i < 3; i++)
    for (int a = 0; a < 3; a++) e[i][a] = J[i][a] / S[i];
}

void oracle_rescaled_basis(const oracle_params* p, const real xx[3], real ebasis[9]) {
  Grid G;
  if (grid_setup(p, &G)) return;
  real e[3][3];
  rescaled_basis(&G, xx, e);
  memcpy(ebasis, e, sizeof e);
}

/* ------------------------------------------------------------------------ */
/* CFL time step. Reading: dt = CFL * min over interior points and directions
 * of S_i dxx^i (the proper grid spacing); with CFL = 0.5 (Sec. 4.1) this
 * reproduces the 8428 iterations quoted for 7.5 M in Sec. 4.2.1.            */
real oracle_dt(const oracle_params* p) {
  Grid G;
  if (grid_setup(p, &G)) return NAN;
  real dsmin = INFINITY;
  for (int i2 = p->ng; i2 < p->ng + p->N[2]; i2++)
    for (int i1 = p->ng; i1 < p->ng + p->N[1]; i1++)
      for (int i0 = p->ng; i0 < p->ng + p->N[0]; i0++) {
        real xx[3] = {xx_of(&G, 0, i0), xx_of(&G, 1, i1), xx_of(&G, 2, i2)};
        real S[3], dS[3][3], ddS[3][3][3];
        scale_factors(&G, xx, S, dS, ddS);
        for (int d = 0; d < 3; d++) {
          real ds = fabs(S[d]) * G.dxx[d];
          if (ds < dsmin) dsmin = ds;
        }
      }
  return p->cfl * dsmin;
}

/* ------------------------------------------------------------------------ */
/* Boundary maps (Sec. 3, Fig. 1): a ghost point is mapped to Cartesian
 * coordinates and back to the canonical coordinate range; the nearest cell
 * is its source. If that is the point itself it is an outer-boundary point,
 * otherwise an inner-boundary point whose value is copied from the source
 * with the parity of the rescaled basis vectors, e~(dst).e~(src) = +-1.     */
static long long flat(const Grid* G, int i0, int i1, int i2) {
  return (long long)i0 + G->st[1] * i1 + G->st[2] * i2;
}

static int is_interior(const Grid* G, int i0, int i1, int i2) {
  const int ng = G->p.ng;
  return i0 >= ng && i0 < ng + G->p.N[0] && i1 >= ng && i1 < ng + G->p.N[1] && i2 >= ng &&
         i2 < ng + G->p.N[2];
}

static int nearest_cell(const Grid* G, int d, real xx) {
  return (int)floor((xx - G->xxmin[d]) / G->dxx[d] + (real)G->p.ng);
}

static int wrap_periodic(const Grid* G, int d, int j) {
  const int ng = G->p.ng, N = G->p.N[d];
  int m = (j - ng) % N;
  if (m < 0) m += N;
  return ng + m;
}

/* Cartesian -> canonical logical coordinates -> nearest cell indices. */
static void cart_to_cell(const Grid* G, const real x[3], int c[3]) {
  const oracle_params* p = &G->p;
  if (p->coord == 1) {
    const real rho = sqrt(x[0] * x[0] + x[1] * x[1]);
    const real phi = atan2(x[1], x[0]);
    c[0] = nearest_cell(G, 0, radial_map_inv(0, p->ampl[0], p->sinhw[0], rho));
    c[1] = wrap_periodic(G, 1, nearest_cell(G, 1, phi));
    c[2] = nearest_cell(G, 2, radial_map_inv(0, p->ampl[2], p->sinhw[2], x[2]));
  } else {
    const real r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    const real th = acos(x[2] / r);
    const real phi = atan2(x[1], x[0]);
    c[0] = nearest_cell(G, 0, radial_map_inv(p->coord == 2, p->ampl[0], p->sinhw[0], r));
    c[1] = nearest_cell(G, 1, th);
    c[2] = wrap_periodic(G, 2, nearest_cell(G, 2, phi));
  }
}

static int build_maps(const Grid* G, int* kind, int* src, int* parity) {
  int bad = 0;
  for (int i2 = 0; i2 < G->n[2]; i2++)
    for (int i1 = 0; i1 < G->n[1]; i1++)
      for (int i0 = 0; i0 < G->n[0]; i0++) {
        const long long q = flat(G, i0, i1, i2);
        src[q] = (int)q;
        parity[q] = 0;
        if (is_interior(G, i0, i1, i2)) { kind[q] = 0; continue; }
        real xx[3] = {xx_of(G, 0, i0), xx_of(G, 1, i1), xx_of(G, 2, i2)};
        real x[3];
        xx_to_cart(G, xx, x);
        int c[3];
        cart_to_cell(G, x, c);
        if (c[0] == i0 && c[1] == i1 && c[2] == i2) { kind[q] = 1; continue; }
        kind[q] = 2;
        if (c[0] < 0 || c[0] >= G->n[0] || c[1] < 0 || c[1] >= G->n[1] || c[2] < 0 ||
            c[2] >= G->n[2]) { bad = 1; kind[q] = -1; continue; }
        src[q] = (int)flat(G, c[0], c[1], c[2]);
        real xs[3] = {xx_of(G, 0, c[0]), xx_of(G, 1, c[1]), xx_of(G, 2, c[2])};
        real ed[3][3], es[3][3];
        rescaled_basis(G, xx, ed);
        rescaled_basis(G, xs, es);
        for (int d = 0; d < 3; d++) {
          const real dot = ed[d][0] * es[d][0] + ed[d][1] * es[d][1] + ed[d][2] * es[d][2];
          if (fabs(fabs(dot) - 1.0) > 1e-10) bad = 1;
          if (dot < 0) parity[q] |= 1 << d;
        }
      }
  /* every source must be an interior or an outer-boundary point */
  for (long long q = 0; q < G->np; q++)
    if (kind[q] == 2) {
      const int k = kind[src[q]];
      if (k != 0 && k != 1) bad = 1;
    }
  return bad ? -1 : 0;
}

int oracle_bc_maps(const oracle_params* p, int* kind, int* src, int* parity) {
  Grid G;
  if (grid_setup(p, &G)) return -1;
  return build_maps(&G, kind, src, parity);
}

/* sign picked up by gridfunction g under the per-direction parities */
static real gf_sign(int g, int parity) {
  real s = 1.0;
  if (GF_TYPE[g] >= 1 && (parity >> GF_I[g] & 1)) s = -s;
  if (GF_TYPE[g] == 2 && (parity >> GF_J[g] & 1)) s = -s;
  return s;
}

/* Ghost fill (Sec. 3, ordered boundary steps 1 and 2).
 * Step 1, outer boundary. Reading: quadratic extrapolation along the inward
 * face normal, f(g) = 3 f(g-1) - 3 f(g-2) + f(g-3), done layer by layer; in
 * each layer the x0 faces, then the x1 faces, then the x2 faces, each face's
 * transverse range widened by the faces already done. Only outer-boundary
 * points (those the round trip maps to themselves) are written.
 * Step 2, inner boundary: copy from the mapped source with parity signs.   */
/* outer = 1: extrapolate the pure-outer points in shell order, then copy the
 * inner ghosts; outer = 0 (radiation boundary inside the time integrator):
 * the inner copies only.                                                    */
static void apply_bcs_with_maps(const Grid* G, const int* kind, const int* src,
                                const int* parity, real* y, int outer) {
  const int ng = G->p.ng;
  int lo[3], hi[3]; /* current face ranges, [lo, hi) */
  for (int d = 0; d < 3; d++) { lo[d] = ng; hi[d] = ng + G->p.N[d]; }
  for (int layer = 0; layer < (outer ? ng : 0); layer++) {
    for (int d = 0; d < 3; d++) {
      for (int side = 0; side < 2; side++) {
        const int face = side == 0 ? lo[d] - 1 : hi[d];
        const int inward = side == 0 ? +1 : -1;
        int a0 = lo[0], b0 = hi[0], a1 = lo[1], b1 = hi[1], a2 = lo[2], b2 = hi[2];
        if (d == 0) { a0 = face; b0 = face + 1; }
        if (d == 1) { a1 = face; b1 = face + 1; }
        if (d == 2) { a2 = face; b2 = face + 1; }
        const long long step = inward * G->st[d];
        for (int i2 = a2; i2 < b2; i2++)
          for (int i1 = a1; i1 < b1; i1++)
            for (int i0 = a0; i0 < b0; i0++) {
              const long long q = flat(G, i0, i1, i2);
              if (kind[q] != 1) continue;
              for (int g = 0; g < NGF; g++) {
                real* f = y + g * G->np + q;
                f[0] = 3.0 * f[step] - 3.0 * f[2 * step] + f[3 * step];
              }
            }
      }
      lo[d]--;
      hi[d]++;
    }
  }
  for (long long q = 0; q < G->np; q++)
    if (kind[q] == 2)
      for (int g = 0; g < NGF; g++)
        y[g * G->np + q] = gf_sign(g, parity[q]) * y[g * G->np + src[q]];
}

int oracle_apply_bcs(const oracle_params* p, real* y) {
  Grid G;
  if (grid_setup(p, &G)) return -1;
  int* kind = (int*)malloc(sizeof(int) * G.np);
  int* src = (int*)malloc(sizeof(int) * G.np);
  int* par = (int*)malloc(sizeof(int) * G.np);
  int rc = build_maps(&G, kind, src, par);
  if (rc == 0) apply_bcs_with_maps(&G, kind, src, par, y, 1);
  free(kind); free(src); free(par);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Brill-Lindquist punctures (analytic stand-in for the TwoPunctures data of
 * the head-on run, Sec. 4.1): conformally flat, time symmetric (K_ij = 0),
 * psi = 1 + sum m_n / (2 |x - x_n|), gamma_ij = psi^4 delta_ij, so
 * W = psi^-2, eps = Abar = K = Lambdabar = 0; precollapsed lapse psi^-2
 * (or 1), zero shift and B. Interior points, then the ghost fill.           */
int oracle_id_brill_lindquist(const oracle_params* p, int np, const real* m,
                              const real* pos, int lapse_kind, real* y) {
  Grid G;
  if (grid_setup(p, &G)) return -1;
  memset(y, 0, sizeof(real) * NGF * G.np);
  for (int i2 = p->ng; i2 < p->ng + p->N[2]; i2++)
    for (int i1 = p->ng; i1 < p->ng + p->N[1]; i1++)
      for (int i0 = p->ng; i0 < p->ng + p->N[0]; i0++) {
        real xx[3] = {xx_of(&G, 0, i0), xx_of(&G, 1, i1), xx_of(&G, 2, i2)};
        real x[3];
        xx_to_cart(&G, xx, x);
        real psi = 1.0;
        for (int n = 0; n < np; n++) {
          const real dx = x[0] - pos[3 * n], dy = x[1] - pos[3 * n + 1],
                       dz = x[2] - pos[3 * n + 2];
          psi += m[n] / (2.0 * sqrt(dx * dx + dy * dy + dz * dz));
        }
        const long long q = flat(&G, i0, i1, i2);
        y[CF * G.np + q] = 1.0 / (psi * psi);
        y[ALPHA * G.np + q] = lapse_kind == 0 ? 1.0 / (psi * psi) : 1.0;
      }
  return oracle_apply_bcs(p, y);
}

/* ------------------------------------------------------------------------ */
/* Finite differences along a direction with stride s and spacing h (f
 * points at the centre), with the weights above. U+ is the stencil shifted
 * one point toward +s, U- its mirror image (shifted toward -s); for N_FD = 4
 * they are
 *   D f  = [8 (f1 - f-1) - (f2 - f-2)] / 12h
 *   D2 f = [-f-2 + 16 f-1 - 30 f0 + 16 f1 - f2] / 12h^2
 *   U+ f = [-3 f-1 - 10 f0 + 18 f1 - 6 f2 + f3] / 12h
 *   U- f = [3 f1 + 10 f0 - 18 f-1 + 6 f-2 - f-3] / 12h.                     */
static real fd_d1(const Sten* S, const real* f, long long s, real h) {
  real a = 0.0;
  for (int j = S->R; j >= 1; j--) a += S->d1[j] * (f[j * s] - f[-j * s]);
  return a / h;
}
static real fd_d2(const Sten* S, const real* f, long long s, real h) {
  real a = 0.0;
  for (int j = S->R; j >= 1; j--) a += S->d2[j] * ((f[j * s] - f[0]) + (f[-j * s] - f[0]));
  return a / (h * h);
}
/* D_k D_l f (k != l): the tensor product of two centred first differences */
static real fd_d11(const Sten* S, const real* f, long long sk, long long sl, real hk, real hl) {
  real a = 0.0;
  for (int j = S->R; j >= 1; j--)
    a += S->d1[j] * (fd_d1(S, f + j * sk, sl, hl) - fd_d1(S, f - j * sk, sl, hl));
  return a / hk;
}
static real fd_up(const Sten* S, const real* f, long long s, real h) {
  real a = 0.0;
  for (int m = S->R + 1; m >= -(S->R - 1); m--)
    if (m != 1) a += S->up[m + S->R - 1] * (f[m * s] - f[s]);
  return a / h;
}
static real fd_dn(const Sten* S, const real* f, long long s, real h) {
  return -fd_up(S, f, -s, h);
}
static real fd_ko(const Sten* S, const real* f, long long s, real h) {
  real a = 0.0;
  for (int j = S->R + 1; j >= 1; j--) a += S->ko[j] * ((f[j * s] - f[0]) + (f[-j * s] - f[0]));
  return a / h;
}

int oracle_fd_point(const oracle_params* p, const real* f, long long idx, real d1[3],
                    real d2[9], real uplus[3], real uminus[3]) {
  Grid G;
  if (grid_setup(p, &G)) return -1;
  const real* c = f + idx;
  for (int k = 0; k < 3; k++) {
    d1[k] = fd_d1(&G.fd, c, G.st[k], G.dxx[k]);
    uplus[k] = fd_up(&G.fd, c, G.st[k], G.dxx[k]);
    uminus[k] = fd_dn(&G.fd, c, G.st[k], G.dxx[k]);
    for (int l = 0; l < 3; l++)
      d2[3 * k + l] = k == l ? fd_d2(&G.fd, c, G.st[k], G.dxx[k])
                             : fd_d11(&G.fd, c, G.st[k], G.st[l], G.dxx[k], G.dxx[l]);
  }
  return 0;
}

int oracle_ko_point(const oracle_params* p, const real* f, long long idx, real ko[3]) {
  Grid G;
  if (grid_setup(p, &G)) return -1;
  for (int k = 0; k < 3; k++) ko[k] = fd_ko(&G.fd, f + idx, G.st[k], G.dxx[k]);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* general symmetric 3x3 inverse */
static void inverse3(const real a[3][3], real inv[3][3]) {
  const real det = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
                     a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
                     a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
  inv[0][0] = (a[1][1] * a[2][2] - a[1][2] * a[2][1]) / det;
  inv[0][1] = (a[0][2] * a[2][1] - a[0][1] * a[2][2]) / det;
  inv[0][2] = (a[0][1] * a[1][2] - a[0][2] * a[1][1]) / det;
  inv[1][0] = (a[1][2] * a[2][0] - a[1][0] * a[2][2]) / det;
  inv[1][1] = (a[0][0] * a[2][2] - a[0][2] * a[2][0]) / det;
  inv[1][2] = (a[0][2] * a[1][0] - a[0][0] * a[1][2]) / det;
  inv[2][0] = (a[1][0] * a[2][1] - a[1][1] * a[2][0]) / det;
  inv[2][1] = (a[0][1] * a[2][0] - a[0][0] * a[2][1]) / det;
  inv[2][2] = (a[0][0] * a[1][1] - a[0][1] * a[1][0]) / det;
}

/* Everything the RHS, the Ricci tensor and the constraints need at a point. */
typedef struct {
  real rhs[NGF];
  real ricci_resc[6];
  real H, M_resc[3], C_resc[3];
} PointOut;

static void bssn_point(const Grid* G, real eta, const real* y, int i0, int i1, int i2,
                       PointOut* out) {
  const long long q = flat(G, i0, i1, i2);
  const long long np = G->np;
  const real xx[3] = {xx_of(G, 0, i0), xx_of(G, 1, i1), xx_of(G, 2, i2)};

  /* ---- 1. finite differences of the rescaled evolved variables --------- */
  real v[NGF], d1[NGF][3], d2[NGF][3][3], up[NGF][3];
  for (int g = 0; g < NGF; g++) {
    const real* f = y + g * np + q;
    v[g] = f[0];
    for (int k = 0; k < 3; k++) d1[g][k] = fd_d1(&G->fd, f, G->st[k], G->dxx[k]);
    for (int k = 0; k < 3; k++)
      for (int l = k; l < 3; l++) {
        d2[g][k][l] = k == l ? fd_d2(&G->fd, f, G->st[k], G->dxx[k])
                             : fd_d11(&G->fd, f, G->st[k], G->st[l], G->dxx[k], G->dxx[l]);
        d2[g][l][k] = d2[g][k][l];
      }
  }
  /* Reading: the upwind side is chosen by the sign of the shift component
   * (vet^k > 0: stencil shifted toward +k, else toward -k).                 */
  for (int g = 0; g < NGF; g++) {
    const real* f = y + g * np + q;
    for (int k = 0; k < 3; k++)
      up[g][k] = v[VETU0 + k] > 0.0 ? fd_up(&G->fd, f, G->st[k], G->dxx[k])
                                    : fd_dn(&G->fd, f, G->st[k], G->dxx[k]);
  }

  /* ---- 2. reference metric (analytic): gammahat_ij = S_i^2 delta_ij ---- */
  real S[3], dS[3][3], ddS[3][3][3];
  scale_factors(G, xx, S, dS, ddS);
  real gh[3][3] = {{0}}, dgh[3][3][3] = {{{0}}}, ddgh[3][3][3][3] = {{{{0}}}};
  for (int i = 0; i < 3; i++) {
    gh[i][i] = S[i] * S[i];
    for (int k = 0; k < 3; k++) {
      dgh[i][i][k] = 2.0 * S[i] * dS[i][k];
      for (int l = 0; l < 3; l++)
        ddgh[i][i][k][l] = 2.0 * (dS[i][l] * dS[i][k] + S[i] * ddS[i][k][l]);
    }
  }
  real ghUU[3][3];
  inverse3(gh, ghUU);
  /* Christoffel symbols of gammahat and their derivatives:
   * Gh[i][j][k] = Gammahat^i_jk, dGh[i][j][k][l] = d_l Gammahat^i_jk       */
  real Gh[3][3][3], dGh[3][3][3][3];
  real dghUU[3][3][3]; /* d_l gammahat^ij */
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      for (int l = 0; l < 3; l++) {
        real s = 0.0;
        for (int a = 0; a < 3; a++)
          for (int b = 0; b < 3; b++) s -= ghUU[i][a] * dgh[a][b][l] * ghUU[b][j];
        dghUU[i][j][l] = s;
      }
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      for (int k = 0; k < 3; k++) {
        real s = 0.0;
        for (int m = 0; m < 3; m++)
          s += 0.5 * ghUU[i][m] * (dgh[m][k][j] + dgh[m][j][k] - dgh[j][k][m]);
        Gh[i][j][k] = s;
        for (int l = 0; l < 3; l++) {
          real t = 0.0;
          for (int m = 0; m < 3; m++)
            t += 0.5 * dghUU[i][m][l] * (dgh[m][k][j] + dgh[m][j][k] - dgh[j][k][m]) +
                 0.5 * ghUU[i][m] * (ddgh[m][k][j][l] + ddgh[m][j][k][l] - ddgh[j][k][m][l]);
          dGh[i][j][k][l] = t;
        }
      }

  /* ---- 3. unrescale (Sec. 2.2): eps_ij = h_ij S_i S_j, Abar likewise,
   *      Lambdabar^i = lambda^i / S_i, beta^i = vet^i / S_i, B^i = bet^i / S_i,
   *      derivatives by the product rule with analytic derivatives of S.   */
  real ReDD[3][3], dReDD[3][3][3], ddReDD[3][3][3][3];
  real ReU[3], dReU[3][3], ddReU[3][3][3];
  for (int i = 0; i < 3; i++) {
    ReU[i] = 1.0 / S[i];
    for (int k = 0; k < 3; k++) {
      dReU[i][k] = -dS[i][k] / (S[i] * S[i]);
      for (int l = 0; l < 3; l++)
        ddReU[i][k][l] = -ddS[i][k][l] / (S[i] * S[i]) +
                         2.0 * dS[i][k] * dS[i][l] / (S[i] * S[i] * S[i]);
    }
    for (int j = 0; j < 3; j++) {
      ReDD[i][j] = S[i] * S[j];
      for (int k = 0; k < 3; k++) {
        dReDD[i][j][k] = dS[i][k] * S[j] + S[i] * dS[j][k];
        for (int l = 0; l < 3; l++)
          ddReDD[i][j][k][l] = ddS[i][k][l] * S[j] + dS[i][k] * dS[j][l] +
                               dS[i][l] * dS[j][k] + S[i] * ddS[j][k][l];
      }
    }
  }
  real eps[3][3], deps[3][3][3], ddeps[3][3][3][3], deps_up[3][3][3];
  real Abar[3][3], dAbar[3][3][3], dAbar_up[3][3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      const int gh_ = HDD00 + SYM[i][j], ga = ADD00 + SYM[i][j];
      eps[i][j] = v[gh_] * ReDD[i][j];
      Abar[i][j] = v[ga] * ReDD[i][j];
      for (int k = 0; k < 3; k++) {
        deps[i][j][k] = d1[gh_][k] * ReDD[i][j] + v[gh_] * dReDD[i][j][k];
        deps_up[i][j][k] = up[gh_][k] * ReDD[i][j] + v[gh_] * dReDD[i][j][k];
        dAbar[i][j][k] = d1[ga][k] * ReDD[i][j] + v[ga] * dReDD[i][j][k];
        dAbar_up[i][j][k] = up[ga][k] * ReDD[i][j] + v[ga] * dReDD[i][j][k];
        for (int l = 0; l < 3; l++)
          ddeps[i][j][k][l] = d2[gh_][k][l] * ReDD[i][j] + d1[gh_][k] * dReDD[i][j][l] +
                              d1[gh_][l] * dReDD[i][j][k] + v[gh_] * ddReDD[i][j][k][l];
      }
    }
  real Lam[3], dLam[3][3], dLam_up[3][3];
  real beta[3], dbeta[3][3], ddbeta[3][3][3], dbeta_up[3][3];
  real B[3], dB_up[3][3];
  for (int i = 0; i < 3; i++) {
    const int gl = LAMU0 + i, gv = VETU0 + i, gb = BETU0 + i;
    Lam[i] = v[gl] * ReU[i];
    beta[i] = v[gv] * ReU[i];
    B[i] = v[gb] * ReU[i];
    for (int k = 0; k < 3; k++) {
      dLam[i][k] = d1[gl][k] * ReU[i] + v[gl] * dReU[i][k];
      dLam_up[i][k] = up[gl][k] * ReU[i] + v[gl] * dReU[i][k];
      dbeta[i][k] = d1[gv][k] * ReU[i] + v[gv] * dReU[i][k];
      dbeta_up[i][k] = up[gv][k] * ReU[i] + v[gv] * dReU[i][k];
      dB_up[i][k] = up[gb][k] * ReU[i] + v[gb] * dReU[i][k];
      for (int l = 0; l < 3; l++)
        ddbeta[i][k][l] = d2[gv][k][l] * ReU[i] + d1[gv][k] * dReU[i][l] +
                          d1[gv][l] * dReU[i][k] + v[gv] * ddReU[i][k][l];
    }
  }
  const real W = v[CF], K = v[TRK], alpha = v[ALPHA];
  real dW[3], ddW[3][3], dW_up[3], dK[3], dK_up[3], dalpha[3], ddalpha[3][3], dalpha_up[3];
  for (int k = 0; k < 3; k++) {
    dW[k] = d1[CF][k]; dW_up[k] = up[CF][k];
    dK[k] = d1[TRK][k]; dK_up[k] = up[TRK][k];
    dalpha[k] = d1[ALPHA][k]; dalpha_up[k] = up[ALPHA][k];
    for (int l = 0; l < 3; l++) { ddW[k][l] = d2[CF][k][l]; ddalpha[k][l] = d2[ALPHA][k][l]; }
  }

  /* ---- 4. conformal metric, Eq. 3: gammabar_ij = gammahat_ij + eps_ij --- */
  real gb[3][3], gbUU[3][3], dgb[3][3][3], ddgb[3][3][3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      gb[i][j] = gh[i][j] + eps[i][j];
      for (int k = 0; k < 3; k++) {
        dgb[i][j][k] = dgh[i][j][k] + deps[i][j][k];
        for (int l = 0; l < 3; l++) ddgb[i][j][k][l] = ddgh[i][j][k][l] + ddeps[i][j][k][l];
      }
    }
  inverse3(gb, gbUU);

  /* ---- 5. connection difference, Eqs. 4-5. Eq. 4 is evaluated in the
   * equivalent reference-covariant form
   *   Delta^k_ij = 1/2 gammabar^kl (Dhat_i eps_lj + Dhat_j eps_il - Dhat_l eps_ij),
   * Dhat_k eps_ij = d_k eps_ij - Gammahat^m_ki eps_mj - Gammahat^m_kj eps_im
   * (Dhat gammahat = 0), which vanishes exactly when eps does.             */
  real Dhat_eps[3][3][3]; /* [i][j][k] = Dhat_k eps_ij */
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      for (int k = 0; k < 3; k++) {
        real s = deps[i][j][k];
        for (int m = 0; m < 3; m++) s -= Gh[m][k][i] * eps[m][j] + Gh[m][k][j] * eps[i][m];
        Dhat_eps[i][j][k] = s;
      }
  real DeltaUDD[3][3][3], DeltaU[3], DeltaDDD[3][3][3], Gb[3][3][3];
  for (int k = 0; k < 3; k++)
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) {
        real s = 0.0;
        for (int l = 0; l < 3; l++)
          s += 0.5 * gbUU[k][l] * (Dhat_eps[l][j][i] + Dhat_eps[i][l][j] - Dhat_eps[i][j][l]);
        DeltaUDD[k][i][j] = s;
        Gb[k][i][j] = Gh[k][i][j] + s; /* Gammabar = Gammahat + Delta (Eq. 4) */
      }
  for (int k = 0; k < 3; k++) {
    real s = 0.0;
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) s += gbUU[i][j] * DeltaUDD[k][i][j];
    DeltaU[k] = s; /* Eq. 5 */
  }
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      for (int k = 0; k < 3; k++) {
        real s = 0.0;
        for (int l = 0; l < 3; l++) s += gb[i][l] * DeltaUDD[l][j][k];
        DeltaDDD[i][j][k] = s; /* Delta_ijk = gammabar_il Delta^l_jk */
      }

  /* ---- 6. conformal Ricci tensor, Eq. 12 ------------------------------- */
  /* d_k (Dhat_l eps_ij) and Dhat_k Dhat_l eps_ij (= Dhat_k Dhat_l gammabar_ij) */
  real DDeps[3][3][3][3]; /* [i][j][l][k] = Dhat_k Dhat_l eps_ij */
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      for (int l = 0; l < 3; l++)
        for (int k = 0; k < 3; k++) {
          real dD = ddeps[i][j][l][k];
          for (int m = 0; m < 3; m++)
            dD -= dGh[m][l][i][k] * eps[m][j] + Gh[m][l][i] * deps[m][j][k] +
                  dGh[m][l][j][k] * eps[i][m] + Gh[m][l][j] * deps[i][m][k];
          real s = dD;
          for (int m = 0; m < 3; m++)
            s -= Gh[m][k][l] * Dhat_eps[i][j][m] + Gh[m][k][i] * Dhat_eps[m][j][l] +
                 Gh[m][k][j] * Dhat_eps[i][m][l];
          DDeps[i][j][l][k] = s;
        }
  real DhatLam[3][3]; /* [k][j] = Dhat_j Lambdabar^k */
  for (int k = 0; k < 3; k++)
    for (int j = 0; j < 3; j++) {
      real s = dLam[k][j];
      for (int m = 0; m < 3; m++) s += Gh[k][j][m] * Lam[m];
      DhatLam[k][j] = s;
    }
  real R[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      real s = 0.0;
      for (int k = 0; k < 3; k++)
        for (int l = 0; l < 3; l++) s += -0.5 * gbUU[k][l] * DDeps[i][j][l][k];
      for (int k = 0; k < 3; k++)
        s += 0.5 * (gb[k][i] * DhatLam[k][j] + gb[k][j] * DhatLam[k][i]);
      for (int k = 0; k < 3; k++) s += 0.5 * DeltaU[k] * (DeltaDDD[i][j][k] + DeltaDDD[j][i][k]);
      for (int k = 0; k < 3; k++)
        for (int l = 0; l < 3; l++)
          for (int m = 0; m < 3; m++)
            s += gbUU[k][l] * (DeltaUDD[m][k][i] * DeltaDDD[j][m][l] +
                               DeltaUDD[m][k][j] * DeltaDDD[i][m][l] +
                               DeltaUDD[m][i][k] * DeltaDDD[m][j][l]);
      R[i][j] = s;
    }

  /* ---- 7. conformal factor: W = exp(-2 phi) (Sec. 2.1 after Eq. 2) ----- */
  real phi_d[3], phi_dd[3][3];
  for (int i = 0; i < 3; i++) phi_d[i] = -dW[i] / (2.0 * W);
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) phi_dd[i][j] = -ddW[i][j] / (2.0 * W) + dW[i] * dW[j] / (2.0 * W * W);
  const real em4phi = W * W; /* exp(-4 phi) */

  /* ---- 8. covariant derivatives and contractions ----------------------- */
  real DbDb_alpha[3][3], DbDb_phi[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      real a = ddalpha[i][j], b = phi_dd[i][j];
      for (int k = 0; k < 3; k++) { a -= Gb[k][i][j] * dalpha[k]; b -= Gb[k][i][j] * phi_d[k]; }
      DbDb_alpha[i][j] = a;
      DbDb_phi[i][j] = b;
    }
  real Dbar_beta = 0.0; /* Dbar_k beta^k = d_k beta^k + Gammabar^k_km beta^m */
  for (int k = 0; k < 3; k++) {
    Dbar_beta += dbeta[k][k];
    for (int m = 0; m < 3; m++) Dbar_beta += Gb[k][k][m] * beta[m];
  }
  real Dhat_betaU[3][3]; /* [i][j] = Dhat_j beta^i */
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      real s = dbeta[i][j];
      for (int m = 0; m < 3; m++) s += Gh[i][j][m] * beta[m];
      Dhat_betaU[i][j] = s;
    }
  real Dhat_betaD[3][3]; /* [i][j] = Dhat_i beta_j, beta_j = gammahat_jm beta^m */
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      real s = 0.0;
      for (int m = 0; m < 3; m++) s += gh[j][m] * Dhat_betaU[m][i];
      Dhat_betaD[i][j] = s;
    }
  real AbarUD[3][3], AbarUU[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      real s = 0.0;
      for (int k = 0; k < 3; k++) s += gbUU[i][k] * Abar[k][j];
      AbarUD[i][j] = s;
    }
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      real s = 0.0;
      for (int k = 0; k < 3; k++)
        for (int l = 0; l < 3; l++) s += gbUU[i][k] * gbUU[j][l] * Abar[k][l];
      AbarUU[i][j] = s;
    }
  real trAbar = 0.0, AbarAbar = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      trAbar += gbUU[i][j] * Abar[i][j];
      AbarAbar += Abar[i][j] * AbarUU[i][j];
    }

  /* ---- 9. Eq. 7: d_perp eps_ij; d_t = d_perp + Lie_beta ----------------
   * Reading: beta_j in Eq. 7 is lowered with gammahat, so that
   * 2 Dhat_(i beta_j) = Lie_beta gammahat_ij.                              */
  real rhs_eps[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      const real dperp = (real)2 / 3 * gb[i][j] * (alpha * trAbar - Dbar_beta) +
                           Dhat_betaD[i][j] + Dhat_betaD[j][i] - 2.0 * alpha * Abar[i][j];
      real lie = 0.0;
      for (int k = 0; k < 3; k++)
        lie += beta[k] * deps_up[i][j][k] + eps[k][j] * dbeta[k][i] + eps[i][k] * dbeta[k][j];
      rhs_eps[i][j] = dperp + lie;
    }

  /* ---- 10. Eq. 8: d_perp Abar_ij --------------------------------------- */
  real X[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      X[i][j] = -2.0 * alpha * DbDb_phi[i][j] + 4.0 * alpha * phi_d[i] * phi_d[j] +
                2.0 * (dalpha[i] * phi_d[j] + dalpha[j] * phi_d[i]) - DbDb_alpha[i][j] +
                alpha * R[i][j];
  real trX = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) trX += gbUU[i][j] * X[i][j];
  real rhs_Abar[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      const real XTF = X[i][j] - (real)1 / 3 * gb[i][j] * trX;
      real AA = 0.0;
      for (int k = 0; k < 3; k++) AA += Abar[i][k] * AbarUD[k][j];
      const real dperp = -(real)2 / 3 * Abar[i][j] * Dbar_beta - 2.0 * alpha * AA +
                           alpha * Abar[i][j] * K + em4phi * XTF;
      real lie = 0.0;
      for (int k = 0; k < 3; k++)
        lie += beta[k] * dAbar_up[i][j][k] + Abar[k][j] * dbeta[k][i] + Abar[i][k] * dbeta[k][j];
      rhs_Abar[i][j] = dperp + lie;
    }

  /* ---- 11. Eq. 9: d_perp W;  Eq. 10: d_perp K ------------------------- */
  real advW = 0.0, advK = 0.0, advAlpha = 0.0;
  for (int k = 0; k < 3; k++) {
    advW += beta[k] * dW_up[k];
    advK += beta[k] * dK_up[k];
    advAlpha += beta[k] * dalpha_up[k];
  }
  const real rhs_W = -(real)1 / 3 * W * (Dbar_beta - alpha * K) + advW;
  real lap_alpha = 0.0, dalpha_dphi = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      lap_alpha += gbUU[i][j] * DbDb_alpha[i][j];
      dalpha_dphi += gbUU[i][j] * dalpha[i] * phi_d[j];
    }
  const real rhs_K = (real)1 / 3 * alpha * K * K + alpha * AbarAbar -
                       em4phi * (lap_alpha + 2.0 * dalpha_dphi) + advK;

  /* ---- 12. Eq. 11: d_perp Lambdabar^i ---------------------------------
   * Reading: the printed equation lacks lapse factors; the terms are
   * -2 Abar^ij (d_j alpha - 6 alpha d_j phi) + 2 alpha Abar^jk Delta^i_jk,
   * the form that follows from adding alpha times the momentum constraint
   * (Eq. 17) and the only one under which the constraints are preserved.   */
  real DhatDhat_beta[3][3][3]; /* [i][k][j] = Dhat_j Dhat_k beta^i */
  for (int i = 0; i < 3; i++)
    for (int k = 0; k < 3; k++)
      for (int j = 0; j < 3; j++) {
        real s = ddbeta[i][k][j]; /* d_j (Dhat_k beta^i) */
        for (int m = 0; m < 3; m++) s += dGh[i][k][m][j] * beta[m] + Gh[i][k][m] * dbeta[m][j];
        for (int m = 0; m < 3; m++)
          s += Gh[i][j][m] * Dhat_betaU[m][k] - Gh[m][j][k] * Dhat_betaU[i][m];
        DhatDhat_beta[i][k][j] = s;
      }
  /* d_k Gammabar^j_jm = 1/2 d_k (gammabar^jl d_m gammabar_jl)             */
  real dGbc[3][3]; /* [m][k] */
  for (int m = 0; m < 3; m++)
    for (int k = 0; k < 3; k++) {
      real s = 0.0;
      for (int j = 0; j < 3; j++)
        for (int l = 0; l < 3; l++) {
          real dUU = 0.0; /* d_k gammabar^jl */
          for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) dUU -= gbUU[j][a] * gbUU[l][b] * dgb[a][b][k];
          s += 0.5 * (dUU * dgb[j][l][m] + gbUU[j][l] * ddgb[j][l][k][m]);
        }
      dGbc[m][k] = s;
    }
  real Gbc[3]; /* Gammabar^j_jm */
  for (int m = 0; m < 3; m++) {
    Gbc[m] = 0.0;
    for (int j = 0; j < 3; j++) Gbc[m] += Gb[j][j][m];
  }
  real dDbar_beta[3]; /* d_k (Dbar_j beta^j) */
  for (int k = 0; k < 3; k++) {
    real s = 0.0;
    for (int j = 0; j < 3; j++) s += ddbeta[j][j][k];
    for (int m = 0; m < 3; m++) s += dGbc[m][k] * beta[m] + Gbc[m] * dbeta[m][k];
    dDbar_beta[k] = s;
  }
  real rhs_Lam[3];
  for (int i = 0; i < 3; i++) {
    real t2 = 0.0, t4 = 0.0, t5 = 0.0, t6 = 0.0, t7 = 0.0;
    for (int j = 0; j < 3; j++)
      for (int k = 0; k < 3; k++) t2 += gbUU[j][k] * DhatDhat_beta[i][k][j];
    const real t3 = (real)2 / 3 * DeltaU[i] * Dbar_beta;
    for (int k = 0; k < 3; k++) t4 += gbUU[i][k] * dDbar_beta[k];
    t4 *= (real)1 / 3;
    for (int j = 0; j < 3; j++) t5 += -2.0 * AbarUU[i][j] * (dalpha[j] - 6.0 * alpha * phi_d[j]);
    for (int j = 0; j < 3; j++)
      for (int k = 0; k < 3; k++) t6 += 2.0 * alpha * AbarUU[j][k] * DeltaUDD[i][j][k];
    for (int j = 0; j < 3; j++) t7 += -(real)4 / 3 * alpha * gbUU[i][j] * dK[j];
    real lie = 0.0; /* Lie_beta Lambdabar^i = beta^k d_k Lambdabar^i - Lambdabar^k d_k beta^i */
    for (int k = 0; k < 3; k++) lie += beta[k] * dLam_up[i][k] - Lam[k] * dbeta[i][k];
    rhs_Lam[i] = t2 + t3 + t4 + t5 + t6 + t7 + lie;
  }

  /* ---- 13. gauge, Eqs. 13-15. Reading: d_t Lambdabar^i in Eq. 15 is the
   * full right-hand side of Lambdabar^i just computed.                     */
  const real rhs_alpha = -2.0 * alpha * K + advAlpha;
  real rhs_beta[3], rhs_B[3];
  for (int i = 0; i < 3; i++) {
    real ab = 0.0, aB = 0.0;
    for (int j = 0; j < 3; j++) { ab += beta[j] * dbeta_up[i][j]; aB += beta[j] * dB_up[i][j]; }
    rhs_beta[i] = B[i] + ab;
    rhs_B[i] = 0.75 * rhs_Lam[i] - eta * B[i] + aB;
  }

  /* ---- 14. rescale the right-hand sides (Sec. 2.2) -------------------- */
  for (int i = 0; i < 3; i++)
    for (int j = i; j < 3; j++) {
      out->rhs[HDD00 + SYM[i][j]] = rhs_eps[i][j] / ReDD[i][j];
      out->rhs[ADD00 + SYM[i][j]] = rhs_Abar[i][j] / ReDD[i][j];
      out->ricci_resc[SYM[i][j]] = R[i][j] / ReDD[i][j];
    }
  for (int i = 0; i < 3; i++) {
    out->rhs[LAMU0 + i] = rhs_Lam[i] / ReU[i];
    out->rhs[VETU0 + i] = rhs_beta[i] / ReU[i];
    out->rhs[BETU0 + i] = rhs_B[i] / ReU[i];
  }
  out->rhs[CF] = rhs_W;
  out->rhs[TRK] = rhs_K;
  out->rhs[ALPHA] = rhs_alpha;

  /* ---- 14b. Kreiss-Oliger dissipation (Sec. 4.1) ---------------------- */
  /* Reading: the dissipation is added to each rescaled right-hand side after
   * the equations, with the gauge strength for alpha, vet^i and bet^i and
   * the metric strength for the rest; the 3/4 d_t lambda^i inside bet^i's
   * right-hand side above is the undissipated one.                          */
  if (G->p.diss_gauge != 0.0 || G->p.diss_metric != 0.0)
    for (int g = 0; g < NGF; g++) {
      const int gauge = g == ALPHA || (g >= BETU0 && g <= BETU2) || (g >= VETU0 && g <= VETU2);
      const real eps = gauge ? G->p.diss_gauge : G->p.diss_metric;
      const real* f = y + g * np + q;
      for (int k = 0; k < 3; k++) out->rhs[g] += eps * fd_ko(&G->fd, f, G->st[k], G->dxx[k]);
    }

  /* ---- 15. constraints: Eq. 16 (H), Eq. 17 (M^i), C^i ------------------ */
  real Rtr = 0.0, dphi2 = 0.0, lap_phi = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      Rtr += gbUU[i][j] * R[i][j];
      dphi2 += gbUU[i][j] * phi_d[i] * phi_d[j];
      lap_phi += gbUU[i][j] * DbDb_phi[i][j];
    }
  out->H = (real)2 / 3 * K * K - AbarAbar + em4phi * (Rtr - 8.0 * dphi2 - 8.0 * lap_phi);

  real dgbUU[3][3][3]; /* d_k gammabar^ij */
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      for (int k = 0; k < 3; k++) {
        real s = 0.0;
        for (int a = 0; a < 3; a++)
          for (int b = 0; b < 3; b++) s -= gbUU[i][a] * dgb[a][b][k] * gbUU[b][j];
        dgbUU[i][j][k] = s;
      }
  real dAbarUU[3][3][3]; /* d_k Abar^ij */
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      for (int k = 0; k < 3; k++) {
        real s = 0.0;
        for (int a = 0; a < 3; a++)
          for (int b = 0; b < 3; b++)
            s += dgbUU[i][a][k] * gbUU[j][b] * Abar[a][b] + gbUU[i][a] * dgbUU[j][b][k] * Abar[a][b] +
                 gbUU[i][a] * gbUU[j][b] * dAbar[a][b][k];
        dAbarUU[i][j][k] = s;
      }
  for (int i = 0; i < 3; i++) {
    real div = 0.0; /* Dhat_j Abar^ij */
    for (int j = 0; j < 3; j++) {
      div += dAbarUU[i][j][j];
      for (int m = 0; m < 3; m++) div += Gh[i][j][m] * AbarUU[m][j] + Gh[j][j][m] * AbarUU[i][m];
    }
    real sym = 0.0; /* 2 Abar^k(i Delta^j)_jk */
    for (int j = 0; j < 3; j++)
      for (int k = 0; k < 3; k++)
        sym += AbarUU[k][i] * DeltaUDD[j][j][k] + AbarUU[k][j] * DeltaUDD[i][j][k];
    real t6 = 0.0, tK = 0.0;
    for (int j = 0; j < 3; j++) {
      t6 += 6.0 * AbarUU[i][j] * phi_d[j];
      tK += -(real)2 / 3 * gbUU[i][j] * dK[j];
    }
    out->M_resc[i] = em4phi * (div + sym + t6 + tK) * S[i];
    out->C_resc[i] = (Lam[i] - DeltaU[i]) * S[i];
  }
}

/* ------------------------------------------------------------------------ */
static void interior_index(const Grid* G, long long t, int* i0, int* i1, int* i2) {
  const int ng = G->p.ng;
  const long long N0 = G->p.N[0], N1 = G->p.N[1];
  *i0 = ng + (int)(t % N0);
  *i1 = ng + (int)((t / N0) % N1);
  *i2 = ng + (int)(t / (N0 * N1));
}

/* ------------------------------------------------------------------------ */
/* Sommerfeld radiation outer boundary. Sec. 3 names Sommerfeld radiation
 * conditions for the outer ghost points but gives no form. Reading: near the
 * outer boundary every rescaled gridfunction is an outgoing spherical wave
 * about its asymptotic value, f = f_inf + u(t - r/v)/r, which any such u
 * satisfies through
 *   d_t f = -v (f - f_inf)/r - v rhat.grad f
 * at each pure-outer ghost point; f_inf = 1 for alpha and W, 0 otherwise;
 * v = sqrt(2) for alpha (the asymptotic gauge speed of 1+log slicing), 1
 * otherwise. rhat.grad f = sum_i (x/r . grad xx^i) df/dxx^i, each logical
 * derivative the (N_FD + 1)-point one of the grid's order (Sec. 4.1 pairs
 * eighth-order differencing with an eighth-order radiation condition),
 * centred where the array allows and shifted to stay inside it otherwise. The pure-outer points are then
 * advanced by the time integrator like interior points, and the inner ghosts
 * are copies as before.                                                     */
static real somm_finf(int g) { return (g == ALPHA || g == CF) ? 1.0 : 0.0; }
static real somm_speed(int g) { return g == ALPHA ? sqrt((real)2) : 1.0; }

static void radiation_point(const Grid* G, const real* y, int i0, int i1, int i2, real rhs[NGF]) {
  const int idx[3] = {i0, i1, i2};
  const real xx[3] = {xx_of(G, 0, i0), xx_of(G, 1, i1), xx_of(G, 2, i2)};
  real x[3], J[3][3], K[3][3];
  xx_to_cart(G, xx, x);
  const real r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  jacobian(G, xx, J);
  inverse3(J, K); /* K[a][i] = d xx^i / d x^a */
  real rd[3];    /* rhat . grad xx^i */
  for (int i = 0; i < 3; i++) {
    rd[i] = 0.0;
    for (int a = 0; a < 3; a++) rd[i] += x[a] / r * K[a][i];
  }
  const int R = G->fd.R, W = 2 * R + 1; /* stencil width of the FD order */
  int s[3];
  real w[3][2 * MAXR + 1];
  for (int d = 0; d < 3; d++) {
    s[d] = -R;
    if (idx[d] - R < 0) s[d] = -idx[d];
    if (idx[d] + R > G->n[d] - 1) s[d] = G->n[d] - 1 - idx[d] - 2 * R;
    int m[2 * MAXR + 1];
    for (int j = 0; j < W; j++) m[j] = s[d] + j;
    lagrange_weights(W, m, 1, w[d]);
  }
  const long long q = flat(G, i0, i1, i2);
  for (int g = 0; g < NGF; g++) {
    const real* f = y + g * G->np + q;
    real drf = 0.0;
    for (int d = 0; d < 3; d++) {
      real D = 0.0;
      for (int j = 0; j < W; j++) D += w[d][j] * f[(s[d] + j) * G->st[d]];
      drf += rd[d] * D / G->dxx[d];
    }
    const real v = somm_speed(g);
    rhs[g] = -v * (f[0] - somm_finf(g)) / r - v * drf;
  }
}

int oracle_rhs(const oracle_params* p, real eta, const real* y, real* rhs) {
  Grid G;
  if (grid_setup(p, &G)) return -1;
  const long long nint = (long long)p->N[0] * p->N[1] * p->N[2];
#pragma omp parallel for schedule(static)
  for (long long t = 0; t < nint; t++) {
    int i0, i1, i2;
    interior_index(&G, t, &i0, &i1, &i2);
    PointOut o;
    bssn_point(&G, eta, y, i0, i1, i2, &o);
    const long long q = flat(&G, i0, i1, i2);
    for (int g = 0; g < NGF; g++) rhs[g * G.np + q] = o.rhs[g];
  }
  if (p->bc_kind == 1) { /* the radiation condition at the pure-outer points */
    int* kind = (int*)malloc(sizeof(int) * G.np);
    int* src = (int*)malloc(sizeof(int) * G.np);
    int* par = (int*)malloc(sizeof(int) * G.np);
    const int rc = build_maps(&G, kind, src, par);
    if (rc == 0)
      for (long long q = 0; q < G.np; q++) {
        if (kind[q] != 1) continue;
        const int i0 = (int)(q % G.n[0]), i1 = (int)((q / G.n[0]) % G.n[1]),
                  i2 = (int)(q / ((long long)G.n[0] * G.n[1]));
        real r[NGF];
        radiation_point(&G, y, i0, i1, i2, r);
        for (int g = 0; g < NGF; g++) rhs[g * G.np + q] = r[g];
      }
    free(kind); free(src); free(par);
    if (rc) return rc;
  }
  return 0;
}

int oracle_rhs_points(const oracle_params* p, real eta, const real* y, int npts,
                      const long long* idx, real* out, real* ricci) {
  Grid G;
  if (grid_setup(p, &G)) return -1;
  for (int t = 0; t < npts; t++) {
    const long long q = idx[t];
    const int i0 = (int)(q % G.n[0]), i1 = (int)((q / G.n[0]) % G.n[1]),
              i2 = (int)(q / ((long long)G.n[0] * G.n[1]));
    if (!is_interior(&G, i0, i1, i2)) return -1;
  }
#pragma omp parallel for schedule(static)
  for (int t = 0; t < npts; t++) {
    const long long q = idx[t];
    const int i0 = (int)(q % G.n[0]), i1 = (int)((q / G.n[0]) % G.n[1]),
              i2 = (int)(q / ((long long)G.n[0] * G.n[1]));
    PointOut o;
    bssn_point(&G, eta, y, i0, i1, i2, &o);
    for (int g = 0; g < NGF; g++) out[(long long)NGF * t + g] = o.rhs[g];
    if (ricci)
      for (int c = 0; c < 6; c++) ricci[6LL * t + c] = o.ricci_resc[c];
  }
  return 0;
}

int oracle_constraints(const oracle_params* p, const real* y, real* H, real* M, real* C) {
  Grid G;
  if (grid_setup(p, &G)) return -1;
  const long long nint = (long long)p->N[0] * p->N[1] * p->N[2];
#pragma omp parallel for schedule(static)
  for (long long t = 0; t < nint; t++) {
    int i0, i1, i2;
    interior_index(&G, t, &i0, &i1, &i2);
    PointOut o;
    bssn_point(&G, 0.0, y, i0, i1, i2, &o);
    const long long q = flat(&G, i0, i1, i2);
    if (H) H[q] = o.H;
    for (int i = 0; i < 3; i++) {
      if (M) M[i * G.np + q] = o.M_resc[i];
      if (C) C[i * G.np + q] = o.C_resc[i];
    }
  }
  return 0;
}

/* Classical RK4 (Sec. 4.2.1 footnote) with the ghost fill after each stage
 * and after the final combination (Sec. 3, boundary steps per substage):
 *   k1 = f(y_n), y1 = y_n + dt/2 k1; k2 = f(y1), y2 = y_n + dt/2 k2;
 *   k3 = f(y2), y3 = y_n + dt k3;    k4 = f(y3);
 *   y_n+1 = y_n + dt/6 (k1 + 2 k2 + 2 k3 + k4). Interior points only.      */
int oracle_rk4_step(const oracle_params* p, real eta, real dt, real* y) {
  Grid G;
  if (grid_setup(p, &G)) return -1;
  const long long n = NGF * G.np;
  real* k[4];
  for (int s = 0; s < 4; s++) k[s] = (real*)calloc((size_t)n, sizeof(real));
  real* ys = (real*)malloc(sizeof(real) * n);
  int* kind = (int*)malloc(sizeof(int) * G.np);
  int* src = (int*)malloc(sizeof(int) * G.np);
  int* par = (int*)malloc(sizeof(int) * G.np);
  int rc = build_maps(&G, kind, src, par);
  const int rad = p->bc_kind == 1;
  if (rc == 0) {
    const real c[3] = {0.5, 0.5, 1.0};
    memcpy(ys, y, sizeof(real) * n);
    for (int s = 0; s < 4; s++) {
      oracle_rhs(p, eta, ys, k[s]);
      if (s == 3) break;
      for (long long t = 0; t < G.np; t++)
        if (kind[t] == 0 || (rad && kind[t] == 1))
          for (int g = 0; g < NGF; g++)
            ys[g * G.np + t] = y[g * G.np + t] + c[s] * dt * k[s][g * G.np + t];
      apply_bcs_with_maps(&G, kind, src, par, ys, !rad);
    }
    for (long long t = 0; t < G.np; t++)
      if (kind[t] == 0 || (rad && kind[t] == 1))
        for (int g = 0; g < NGF; g++) {
          const long long e = g * G.np + t;
          y[e] = y[e] + dt / 6.0 * (k[0][e] + 2.0 * k[1][e] + 2.0 * k[2][e] + k[3][e]);
        }
    apply_bcs_with_maps(&G, kind, src, par, y, !rad);
  }
  for (int s = 0; s < 4; s++) free(k[s]);
  free(ys); free(kind); free(src); free(par);
  return rc;
}

/* SSPRK3 (Sec. 4.1, the scheme of the Gottlieb-Shu-Tadmor reference), in
 * its convex-combination form of forward-Euler steps, with the ghost fill
 * after each stage as for RK4:
 *   y1 = y_n + dt f(y_n);
 *   y2 = 3/4 y_n + 1/4 (y1 + dt f(y1));
 *   y_n+1 = 1/3 y_n + 2/3 (y2 + dt f(y2)).  Interior points only.          */
int oracle_ssprk3_step(const oracle_params* p, real eta, real dt, real* y) {
  Grid G;
  if (grid_setup(p, &G)) return -1;
  const long long n = NGF * G.np;
  real* k = (real*)calloc((size_t)n, sizeof(real));
  real* y1 = (real*)malloc(sizeof(real) * n);
  real* y2 = (real*)malloc(sizeof(real) * n);
  int* kind = (int*)malloc(sizeof(int) * G.np);
  int* src = (int*)malloc(sizeof(int) * G.np);
  int* par = (int*)malloc(sizeof(int) * G.np);
  int rc = build_maps(&G, kind, src, par);
  const int rad = p->bc_kind == 1;
  if (rc == 0) {
    /* stage 1: forward Euler from y_n */
    memcpy(y1, y, sizeof(real) * n);
    oracle_rhs(p, eta, y, k);
    for (long long t = 0; t < G.np; t++)
      if (kind[t] == 0 || (rad && kind[t] == 1))
        for (int g = 0; g < NGF; g++) {
          const long long e = g * G.np + t;
          y1[e] = y[e] + dt * k[e];
        }
    apply_bcs_with_maps(&G, kind, src, par, y1, !rad);
    /* stage 2: average of y_n and a forward-Euler step from y1 */
    memcpy(y2, y1, sizeof(real) * n);
    oracle_rhs(p, eta, y1, k);
    for (long long t = 0; t < G.np; t++)
      if (kind[t] == 0 || (rad && kind[t] == 1))
        for (int g = 0; g < NGF; g++) {
          const long long e = g * G.np + t;
          y2[e] = 0.75 * y[e] + 0.25 * (y1[e] + dt * k[e]);
        }
    apply_bcs_with_maps(&G, kind, src, par, y2, !rad);
    /* stage 3: average of y_n and a forward-Euler step from y2 */
    oracle_rhs(p, eta, y2, k);
    for (long long t = 0; t < G.np; t++)
      if (kind[t] == 0 || (rad && kind[t] == 1))
        for (int g = 0; g < NGF; g++) {
          const long long e = g * G.np + t;
          y[e] = ((real)1 / 3) * y[e] + ((real)2 / 3) * (y2[e] + dt * k[e]);
        }
    apply_bcs_with_maps(&G, kind, src, par, y, !rad);
  }
  free(k); free(y1); free(y2); free(kind); free(src); free(par);
  return rc;
}

void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
