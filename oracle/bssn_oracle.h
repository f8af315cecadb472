/*
 * bssn_oracle.h -- TEST INFRASTRUCTURE. Interface of the plain CPU oracle.
 *
 * The oracle is a slow, direct evaluation (FP64, or extended precision in
 * its second build) of the discretised BSSN
 * evolution of arXiv:2505.00097 (Sec. 2.1 Eqs. 4-17, Sec. 2.2 rescaling,
 * Sec. 3 grid and ghost zones, Eq. 22 sinh map, RK4 of Sec. 4.2.1). It exists
 * only to check the HIP library: only tests/, the smoke check and the CPU
 * baseline of the benchmark may call it. It shares no source with the HIP
 * library and reads no output of it.
 *
 * Arrays use the same layout as the library: y[g][i2][i1][i0], i0 fastest,
 * n[d] = N[d] + 2*ng points per direction, gridfunction order
 *   aDD00 aDD01 aDD02 aDD11 aDD12 aDD22 alpha betU0 betU1 betU2 cf
 *   hDD00 hDD01 hDD02 hDD11 hDD12 hDD22 lambdaU0 lambdaU1 lambdaU2 trK
 *   vetU0 vetU1 vetU2
 * All pointers are host pointers.
 */
#ifndef BSSN_ORACLE_H
#define BSSN_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_NGF 24

/* The floating-point type of every computation and of every array and
 * scalar of the interface below: double in the FP64 oracle; the
 * extended-precision reference is this same source compiled with
 * -DORACLE_REAL="long double" (x87 80-bit on x86-64), the yardstick for
 * the rounding error of FP64 evaluations at ill-conditioned points. The
 * parameter struct stays double in both builds, so both evaluate the same
 * problem. */
#ifndef ORACLE_REAL
#define ORACLE_REAL double
#endif
typedef ORACLE_REAL oracle_real;

typedef struct {
  int coord;       /* 0 SinhSpherical, 1 SinhCylindrical, 2 Spherical */
  int N[3];        /* interior points per direction */
  int ng;          /* ghost layers N_G, 3..6: finite differences of order 2 (N_G - 1) */
  double ampl[3];  /* outer extent of the sinh (or linear) maps */
  double sinhw[3]; /* sinh widths */
  double cfl;
  /* Kreiss-Oliger dissipation strengths (Sec. 4.1), 0 = off: diss_gauge for
   * alpha, vet^i, bet^i; diss_metric for every other gridfunction. */
  double diss_gauge, diss_metric;
  /* outer boundary (Sec. 3): 0 quadratic extrapolation, 1 Sommerfeld
   * radiation condition evolved at the pure-outer ghost points */
  int bc_kind;
} oracle_params;

/* 0 if the parameters describe a grid the oracle supports, -1 otherwise. */
int oracle_check(const oracle_params* p);

/* Logical coordinate of cell j in direction d (cell-centred, Sec. 3). */
oracle_real oracle_xx(const oracle_params* p, int d, int j);

/* Scale factors S_i, d_k S_i (dS[3*i+k]) and d_k d_l S_i (ddS[9*i+3*k+l])
 * at logical coordinates xx. */
void oracle_scalefactors(const oracle_params* p, const oracle_real xx[3], oracle_real S[3],
                         oracle_real dS[9], oracle_real ddS[27]);

/* Cartesian position of logical coordinates xx. */
void oracle_xx_to_cart(const oracle_params* p, const oracle_real xx[3], oracle_real x[3]);

/* Rescaled basis vectors e~_(i) = (d x / d xx^i) / S_i, ebasis[3*i+a]. */
void oracle_rescaled_basis(const oracle_params* p, const oracle_real xx[3], oracle_real ebasis[9]);

/* CFL time step: cfl * min over interior points of min_i S_i dxx^i. */
oracle_real oracle_dt(const oracle_params* p);

/* Ghost classification by the Cartesian round trip. Arrays of n_points ints:
 * kind 0 interior / 1 pure outer / 2 inner, src flat index, parity bit d set
 * when e~_(d) flips sign. Returns 0, or -1 if some inner ghost does not map
 * to an interior or pure-outer point or a basis dot product is not +-1. */
int oracle_bc_maps(const oracle_params* p, int* kind, int* src, int* parity);

/* Ghost fill in place: extrapolation in shell order, then parity copies. */
int oracle_apply_bcs(const oracle_params* p, oracle_real* y);

/* Brill-Lindquist data on interior points, then oracle_apply_bcs.
 * lapse_kind 0: alpha = psi^-2, 1: alpha = 1. */
int oracle_id_brill_lindquist(const oracle_params* p, int np, const oracle_real* m,
                              const oracle_real* pos, int lapse_kind, oracle_real* y);

/* Rescaled right-hand sides at every interior point (ghost entries of rhs
 * untouched; with bc_kind 1 also at every pure-outer ghost point, from the
 * radiation condition). eta: Gamma-driver damping. */
int oracle_rhs(const oracle_params* p, oracle_real eta, const oracle_real* y, oracle_real* rhs);

/* Right-hand sides at a list of interior points (flat indices). out[24*q+g].
 * ricci (may be NULL) receives the rescaled Rbar_ij, ricci[6*q + (00,01,02,
 * 11,12,22)]. */
int oracle_rhs_points(const oracle_params* p, oracle_real eta, const oracle_real* y, int npts,
                      const long long* idx, oracle_real* out, oracle_real* ricci);

/* Constraints at every interior point: H (Eq. 16), rescaled momentum
 * constraint S_i M^i (Eq. 17, 3 gridfunctions) and rescaled C^i = Lambdabar^i
 * - Delta^i times S_i (3 gridfunctions). Any output may be NULL. */
int oracle_constraints(const oracle_params* p, const oracle_real* y, oracle_real* H, oracle_real* M,
                       oracle_real* C);

/* One classical RK4 step in place (ghosts refilled after each stage; with
 * bc_kind 1 the pure-outer points are advanced like interior points and only
 * the inner ghosts are refilled). */
int oracle_rk4_step(const oracle_params* p, oracle_real eta, oracle_real dt, oracle_real* y);

/* One SSPRK3 step in place (ghosts refilled after each stage). */
int oracle_ssprk3_step(const oracle_params* p, oracle_real eta, oracle_real dt, oracle_real* y);

/* Finite-difference operators applied to a single gridfunction f (n_points
 * values) at flat index idx: d1[k], d2[3*k+l], upwinded U+[k], U-[k]. */
int oracle_fd_point(const oracle_params* p, const oracle_real* f, long long idx, oracle_real d1[3],
                    oracle_real d2[9], oracle_real uplus[3], oracle_real uminus[3]);

/* Kreiss-Oliger operator (without the strength) of f at flat index idx
 * along each direction k: ko[k]. */
int oracle_ko_point(const oracle_params* p, const oracle_real* f, long long idx, oracle_real ko[3]);

/* Set the number of OpenMP threads the oracle runs with (n > 0). */
void oracle_set_num_threads(int n);

/* Number of OpenMP threads the oracle runs with. */
int oracle_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
