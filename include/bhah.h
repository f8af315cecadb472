/*
 * bhah.h -- C ABI of the MI355X-native BSSN evolution core.
 *
 * What the library computes (paper: "superB/NRPy: Scalable, Task-Based
 * Numerical Relativity for 3G Gravitational Wave Science", arXiv:2505.00097):
 *   - the right-hand sides of the covariant BSSN system with 1+log slicing and
 *     the Gamma-driver shift (Sec. 2.1, Eqs. 7-15, Ricci tensor Eq. 12), for
 *     the 24 rescaled evolved variables (Sec. 2.2) on cell-centred curvilinear
 *     grids (Sec. 3, first paragraphs; sinh radial map Eq. 22);
 *   - classical RK4 time stepping (Sec. 4.2.1, footnote on the integrator);
 *   - the ghost-zone fill: outer-boundary ghosts first, then inner-boundary
 *     (parity) ghosts, after every Runge-Kutta substage (Sec. 3, ghost-point
 *     classes and the ordered list of boundary steps);
 *   - Brill-Lindquist puncture initial data (analytic, conformally flat,
 *     time-symmetric: the stand-in for the TwoPunctures data of the head-on
 *     run, Sec. 4.1, which needs a third-party elliptic solver) and the
 *     Hamiltonian constraint (Eq. 16) as a diagnostic.
 *
 * Conventions shared by every entry point
 *   Return codes : BHAH_OK (0) or a negative BHAH_E* code. A message for the
 *                  last failure on the calling thread is in bhah_last_error().
 *                  No C++ exception crosses this boundary and nothing aborts.
 *   Precision    : IEEE FP64 everywhere.
 *   State layout : y[g][i2][i1][i0], i0 fastest, gridfunction-major, with
 *                  n_total[d] = N[d] + 2*nghosts points per direction and no
 *                  padding: element (g,i0,i1,i2) is at
 *                  ((g*n_total[2] + i2)*n_total[1] + i1)*n_total[0] + i0.
 *                  The 24 gridfunctions are ordered as in enum bhah_gf.
 *   Pointers     : pointers named y, rhs, aux, H, M, C, workspace are DEVICE
 *                  pointers owned by the caller, on the device that was
 *                  current when the grid was created; they must be 8-byte
 *                  aligned (BHAH_EINVAL otherwise). Pointers named host_* or
 *                  taken as parameters structs are host pointers.
 *   Streams      : `stream` is a hipStream_t passed as void*; NULL means the
 *                  null stream. Every call that takes a stream only enqueues
 *                  work and returns; results are ready when the stream is.
 *   Memory       : calls on a grid that take a stream allocate no device
 *                  memory; all temporaries live in the caller's `workspace`.
 *                  Ensembles hold a work description that bhah_batch_step
 *                  grows with the job set; the server holds its job states;
 *                  bhah_probe_peaks allocates and frees its test arrays.
 */
#ifndef BHAH_H
#define BHAH_H

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
enum {
  BHAH_OK = 0,
  BHAH_EINVAL = -1,  /* bad argument: NULL pointer, unsupported parameter,
                        grid too small, odd N_phi where a pi shift is needed */
  BHAH_EDEVICE = -2, /* a HIP runtime call failed (text in bhah_last_error) */
  BHAH_ENOMEM = -3   /* a host or device allocation inside a *_create failed */
};

/* ---- coordinate systems (Sec. 3 first paragraph; Eq. 22) ---------------- *
 * Logical coordinates xx^i are uniform and cell-centred (Sec. 3): point j of
 * direction i sits at xx^i_min + (j - nghosts + 1/2) * dxx^i with
 * dxx^i = (xx^i_max - xx^i_min) / N[i].
 *   BHAH_SINH_SPHERICAL  : xx0 in [0,1] -> r = ampl[0] sinh(xx0/w0)/sinh(1/w0),
 *                          xx1 = theta in [0,pi], xx2 = phi in [-pi,pi].
 *   BHAH_SINH_CYLINDRICAL: xx0 in [0,1] -> rho = ampl[0] sinh(xx0/w0)/sinh(1/w0),
 *                          xx1 = phi in [-pi,pi],
 *                          xx2 in [-1,1] -> z = ampl[2] sinh(xx2/w2)/sinh(1/w2).
 *   BHAH_SPHERICAL       : xx0 in [0,1] -> r = ampl[0] * xx0 (uniform radius,
 *                          the grid of the paper's single-node benchmark),
 *                          xx1 = theta, xx2 = phi.
 * Scale factors S_(i) = sqrt(gammahat_ii) (Sec. 2.2) are taken with their
 * analytic sign: (r', r, r sin(theta)) and (rho', rho, z').                  */
enum { BHAH_SINH_SPHERICAL = 0, BHAH_SINH_CYLINDRICAL = 1, BHAH_SPHERICAL = 2 };

/* ---- outer boundary condition (Sec. 3, outer boundary points) ---------- *
 * BHAH_BC_EXTRAP: quadratic extrapolation along the face normal,
 * f(g) = 3 f(g-1) - 3 f(g-2) + f(g-3), applied ghost layer by ghost layer in
 * the order x0 faces, x1 faces, x2 faces, each face range growing by the
 * layers already filled.
 * BHAH_BC_RADIATION: Sommerfeld radiation condition (Sec. 3 names it; its
 * form here is an outgoing spherical wave about the asymptotic value):
 * every pure-outer ghost point is an evolved point with
 *   d_t f = -v (f - f_inf)/r - v df/dr,
 * f_inf = 1 for alpha and cf, 0 otherwise; v = sqrt(2) for alpha, 1
 * otherwise; df/dr through the logical derivatives along the mapped radial
 * directions (xx0, and xx2 on SinhCylindrical grids), (N_FD + 1)-point
 * stencils of the grid's order centred where the array allows, shifted
 * inward otherwise. The
 * time integrators advance those points like interior ones and refill only
 * the inner ghosts (parity copies of interior or outer points).
 * bhah_apply_bcs always uses the extrapolation (initial fill of any grid). */
enum { BHAH_BC_EXTRAP = 0, BHAH_BC_RADIATION = 1 };

/* ---- time integrators of ensembles and the server ---------------------- *
 * BHAH_RK4: as bhah_rk4_step; BHAH_SSPRK3: as bhah_ssprk3_step.            */
enum { BHAH_RK4 = 0, BHAH_SSPRK3 = 1 };

/* ---- the 24 evolved rescaled gridfunctions (Sec. 2.1 last gauge paragraph;
 * rescaling Sec. 2.2): h_ij = eps_ij/(S_i S_j), a_ij = Abar_ij/(S_i S_j),
 * lambda^i = S_i Lambdabar^i, vet^i = S_i beta^i, bet^i = S_i B^i,
 * cf = W = exp(-2 phi), trK = K, alpha = lapse.                              */
enum bhah_gf {
  BHAH_ADD00 = 0, BHAH_ADD01, BHAH_ADD02, BHAH_ADD11, BHAH_ADD12, BHAH_ADD22,
  BHAH_ALPHA, BHAH_BETU0, BHAH_BETU1, BHAH_BETU2, BHAH_CF,
  BHAH_HDD00, BHAH_HDD01, BHAH_HDD02, BHAH_HDD11, BHAH_HDD12, BHAH_HDD22,
  BHAH_LAMBDAU0, BHAH_LAMBDAU1, BHAH_LAMBDAU2, BHAH_TRK,
  BHAH_VETU0, BHAH_VETU1, BHAH_VETU2,
  BHAH_NUM_GFS /* = 24 */
};

/* Number of gridfunctions in the `aux` array of bhah_bssn_rhs: the rescaled
 * conformal Ricci tensor Rbar_ij/(S_i S_j) (00,01,02,11,12,22), then
 * Q_k = (d_k Gammabar^j_jm) beta^m (k = 0,1,2).                              */
#define BHAH_NUM_AUX_GFS 9

typedef struct bhah_grid bhah_grid;   /* opaque, immutable after create */
typedef struct bhah_batch bhah_batch; /* opaque ensemble of grids        */

/* Grid parameters. nghosts selects the finite-difference order N_FD =
 * 2 (nghosts - 1): 3 for 4th order (the benchmark runs of Sec. 4.2.1) or 5
 * for 8th order (the production head-on run of Sec. 4.1); upwinded advection
 * needs N_FD/2 + 1 ghost layers (Sec. 3). The order applies to every
 * derivative, to the Kreiss-Oliger operator (order N_FD + 1) and to the
 * radiation condition's stencils, in solo calls, ensembles (which may mix
 * both orders) and the server. ampl[]/sinhw[] entries for directions without
 * a map are ignored. cfl scales the time step (Sec. 4.1 uses 0.5). bc_kind:
 * BHAH_BC_EXTRAP or BHAH_BC_RADIATION (both in solo calls, ensembles and the
 * server).                                                                   */
typedef struct {
  int coord;
  int N[3];
  int nghosts;
  double ampl[3];
  double sinhw[3];
  double cfl;
  int bc_kind;
} bhah_grid_params;

/* Gauge parameters: eta is the Gamma-driver damping of Eq. 15 (Sec. 4.1 uses
 * 2.0). shift_variant must be 0: dB^i/dt uses the full dLambdabar^i/dt of
 * Eq. 11 including its advection term.
 * diss_gauge, diss_metric: Kreiss-Oliger dissipation strengths (Sec. 4.1
 * uses 0.99 and 0.3), >= 0, 0 = off. The term eps/(4^N_G dxx^k) sum_k
 * delta_k^(2 N_G) f (the difference of order 2 N_G and radius N_G along each
 * logical direction: the sixth over 64 with 3 ghost layers, the tenth over
 * 1024 with 5), with the sign that makes its Fourier symbol
 * -sin^(2 N_G)(theta/2)/dxx^k, is added to each rescaled right-hand side
 * after Eqs. 7-15: diss_gauge for
 * alpha, vet^i, bet^i, diss_metric for the other gridfunctions; bet^i's
 * 3/4 dlambda^i/dt is the undissipated one.                                 */
typedef struct {
  double eta;
  int shift_variant;
  double diss_gauge;
  double diss_metric;
} bhah_gauge_params;

typedef struct {
  int n_total[3];              /* N[d] + 2*nghosts                           */
  long long n_points;          /* n_total[0]*n_total[1]*n_total[2]          */
  long long n_interior;        /* N[0]*N[1]*N[2]                            */
  long long state_doubles;     /* 24 * n_points: size of one state array    */
  long long aux_doubles;       /* BHAH_NUM_AUX_GFS * n_points               */
  long long workspace_doubles; /* size of the rk4_step workspace (3 states)  */
  long long n_pure_outer;      /* ghost points filled by extrapolation      */
  long long n_inner;           /* ghost points filled by a parity copy      */
  double dxx[3];
  double xxmin[3];
  double dt;                   /* cfl * min over interior of min_i S_i dxx^i */
} bhah_grid_info;

/* Create a grid: validates the parameters, builds the 1-D reference-metric
 * tables and the boundary maps on the host and copies them to the current
 * device. Host-synchronous. Returns BHAH_EINVAL for coord/nghosts/bc_kind out
 * of range, any N[d] < nghosts, or an odd N_phi (the inner maps shift phi by
 * pi); BHAH_ENOMEM / BHAH_EDEVICE on allocation failure. *out is set only on
 * success. (Sec. 3: grid and ghost points; Sec. 2.2: rescaling.)            */
int bhah_grid_create(const bhah_grid_params* params, bhah_grid** out);

/* Free the grid and its device tables. NULL is accepted. The caller must
 * make sure no enqueued work still uses the grid.                           */
void bhah_grid_destroy(bhah_grid* g);

/* Sizes, spacing and the CFL time step of a grid (host, synchronous).       */
int bhah_grid_get_info(const bhah_grid* g, bhah_grid_info* info);

/* Copy the boundary maps to host arrays (host, synchronous). Each pointer may
 * be NULL to skip it; non-NULL arrays must hold n_points ints.
 *   host_kind[p]   : 0 interior, 1 pure outer (filled by extrapolation),
 *                    2 inner (filled by a parity copy)
 *   host_src[p]    : flat index of the source point of an inner ghost,
 *                    p itself for the other kinds
 *   host_parity[p] : bit d set means the rescaled basis vector e~_(d) flips
 *                    sign between source and destination (p_d = -1); 0 for
 *                    non-inner points.
 * (Sec. 3: inner boundary points copy mapped values with tensor parity.)    */
int bhah_grid_get_bc_maps(const bhah_grid* g, int* host_kind, int* host_src,
                          int* host_parity);

/* Brill-Lindquist puncture data, the analytic stand-in for the TwoPunctures
 * initial data of Sec. 4.1 (both conformally flat with K = 0 at the
 * punctures' rest): psi = 1 + sum_n m_n / (2 |x - x_n|),
 * W = psi^-2, alpha = psi^-2 (lapse_kind 0) or 1 (lapse_kind 1), all other
 * variables zero; interior points are set, then bhah_apply_bcs fills the
 * ghosts. host_masses[n_punct] and host_pos[3*n_punct] (Cartesian x,y,z) are
 * host arrays read before the call returns. n_punct may be 0 (flat space).  */
int bhah_set_initial_data_brill_lindquist(const bhah_grid* g, int n_punct,
                                          const double* host_masses,
                                          const double* host_pos,
                                          int lapse_kind, double* y,
                                          void* stream);

/* Ghost-zone fill in place (Sec. 3, boundary steps 1 and 2): every pure-outer
 * ghost by quadratic extrapolation in shell order, then every inner ghost as
 * y_g[dst] = s_g * y_g[src] with s_g = product of p_d over the gridfunction's
 * tensor indices. Interior points are not modified.                          */
int bhah_apply_bcs(const bhah_grid* g, double* y, void* stream);

/* BSSN + gauge right-hand sides (Eqs. 7-15 with Eq. 12) of the rescaled
 * variables at every interior point. y must have valid ghosts. rhs has the
 * state layout; only its interior points are written (and, on a
 * BHAH_BC_RADIATION grid, its pure-outer points, with the radiation
 * condition's right-hand side). aux receives
 * BHAH_NUM_AUX_GFS gridfunctions (state layout, interior points) computed on
 * the way, or may be NULL to skip them. Finite differences of the grid's
 * order (4th or 8th), advection terms beta^k d_k upwinded (Sec. 3 second
 * paragraph).                                                               */
int bhah_bssn_rhs(const bhah_grid* g, const bhah_gauge_params* gp,
                  const double* y, double* rhs, double* aux, void* stream);

/* One classical RK4 step of size dt, in place on y (RK4 per Sec. 4.2.1; the
 * boundary fill of Sec. 3 after every stage and after the final combine).
 * On return every ghost of y is valid, exactly as bhah_apply_bcs leaves it.
 * The intermediate stage arrays get only the ghosts the stencils read: phi
 * ghost planes are exact periodic copies that the stencils never read (they
 * wrap the phi index onto the interior), so they are filled once, after the
 * final combine; the result is the same. workspace must hold
 * info.workspace_doubles doubles and must not alias y.                       */
int bhah_rk4_step(const bhah_grid* g, const bhah_gauge_params* gp, double dt,
                  double* y, double* workspace, void* stream);

/* One step of size dt of the three-stage strong-stability-preserving
 * Runge-Kutta scheme that the production head-on run of Sec. 4.1 uses
 * (Gottlieb, Shu and Tadmor), in place on y:
 *   A = y + dt f(y); B = 3/4 y + 1/4 (A + dt f(A));
 *   y <- 1/3 y + 2/3 (B + dt f(B)),
 * with the boundary fill of Sec. 3 after every stage. Ghost handling,
 * workspace (the first two thirds of info.workspace_doubles are used) and
 * errors are as for bhah_rk4_step.                                          */
int bhah_ssprk3_step(const bhah_grid* g, const bhah_gauge_params* gp, double dt,
                     double* y, double* workspace, void* stream);

/* nsteps steps of bhah_rk4_step (integrator BHAH_RK4) or bhah_ssprk3_step
 * (BHAH_SSPRK3) in one call, the same arithmetic stage by stage, so the
 * state on return equals that of nsteps single-step calls bit for bit, and
 * every ghost of y is valid on return. Between the steps only the ghosts
 * the stencils read are refilled: the phi ghost planes (exact periodic
 * copies, never read by the stencils, which wrap the phi index onto the
 * interior) are filled once, after the last step, instead of after every
 * step (on the head-on grid they are most of the 215k ghost points).
 * nsteps = 0 does nothing; nsteps < 0, an unknown integrator or the
 * arguments rejected by bhah_rk4_step give BHAH_EINVAL.                     */
int bhah_evolve(const bhah_grid* g, const bhah_gauge_params* gp, int integrator,
                double dt, int nsteps, double* y, double* workspace, void* stream);

/* ---- allocation-free RK4 step ---------------------------------------------
 * For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid allocation): one
 * bhah_rk4_step whose workspace is a library-owned file-scope device array
 * instead of a caller buffer. The array holds three states of at most
 * BHAH_NOALLOC_MAX_POINTS points (ghosts included): 3 x 24 x 294912 doubles,
 * about 162 MiB, on every device the library runs on, from the library's
 * load until the process ends. A grid with more points (info.n_points) gets
 * BHAH_EINVAL; other arguments and errors are as for bhah_rk4_step, and the
 * result is the same, bit for bit. The call allocates nothing; its first
 * call on a device (the device current at the call, which must be the
 * grid's) looks up the array's device address once. Every call on one
 * device shares that device's array: calls that overlap on one GPU (two
 * streams, two host threads) race and must be serialised by the caller.
 * No part of the array needs clearing: every workspace value a step reads
 * is written earlier in the same step.                                      */
#define BHAH_NOALLOC_MAX_POINTS 294912
int bhah_rk4_step_noalloc(const bhah_grid* g, const bhah_gauge_params* gp, double dt,
                          double* y, void* stream);

/* All three constraints at every interior point, centred differences of
 * the grid's order: H of Eq. 16 (one gridfunction), the momentum constraint M^i of
 * Eq. 17 and C^i = Lambdabar^i - Delta^i (three gridfunctions each, rescaled
 * like lambda^i: times S_i). Same layout as the state, interior points only;
 * any of H, M, C may be NULL (skipped). y must have valid ghosts.           */
int bhah_constraints(const bhah_grid* g, const double* y, double* H, double* M,
                     double* C, void* stream);

/* Tile shape of this grid's right-hand-side kernel (bhah_bssn_rhs,
 * bhah_rk4_step, bhah_ssprk3_step, bhah_evolve): 64 points, 2^lx along i0,
 * 2^ly along i1, 64 >> (lx + ly) along i2, walked in bands of `band` tile
 * rows of i1. The extent along phi (i1 on SinhCylindrical grids, i2
 * otherwise) must be 1. Default (6, 0, 4). The shape changes speed only:
 * every point's arithmetic is the same, and with one wave per tile the
 * results are bitwise equal across shapes. With row tiles (lx = 6) the one-wave kernel brings
 * stencil rows shared by the tile's points into LDS with a few wide loads
 * (at 4th order; at 8th order on two-phi-plane grids without
 * dissipation). Setting a shape keeps the number of waves per tile
 * (below).                                                                  */
int bhah_grid_set_tile(bhah_grid* g, int lx, int ly, int band);
int bhah_grid_get_tile(const bhah_grid* g, int* lx, int* ly, int* band);

/* Waves per tile of this grid's right-hand-side kernel: 1 (default: one
 * wave computes all of a point's right-hand sides) or 2 (two waves of one
 * block share each point, one the metric part of Eqs. 7-15 with the Ricci
 * tensor of Eq. 12, the other the gauge part, exchanging intermediates
 * through LDS; each wave runs on its own SIMD). Two waves shorten a step on
 * grids with at most half as many tiles as the device has SIMDs; the
 * results agree with one wave to rounding (the sums are grouped
 * differently), not bit for bit. The two-wave kernel exists at 4th order
 * (nghosts = 3) without dissipation for every family and phi extent except
 * the general SinhSpherical one, and with dissipation for SinhCylindrical
 * grids of two phi planes; elsewhere the one-wave kernel runs whatever this
 * is set to. Any value other than 1 or 2 gets BHAH_EINVAL. The ensemble
 * engine and the server always use one wave per tile.                       */
int bhah_grid_set_waves_per_tile(bhah_grid* g, int waves);
int bhah_grid_get_waves_per_tile(const bhah_grid* g, int* waves);

/* Time every allowed tile shape for this grid on state y (valid ghosts),
 * with one and with two waves per tile, writing right-hand sides into rhs
 * (state layout, caller-owned scratch), after a few warm-up launches, in
 * two passes; keep the first candidate within 2% of the fastest, one-wave
 * shapes before two-wave ones and larger extents along i0 first (so two
 * waves are chosen only when more than 2% faster than every one-wave
 * shape). Synchronises stream.                                              */
int bhah_grid_tune(bhah_grid* g, const bhah_gauge_params* gp, const double* y,
                   double* rhs, void* stream);

/* Hamiltonian constraint H of Eq. 16 at every interior point (centred
 * differences of the grid's order), written into H (one gridfunction, state point
 * layout, interior points only). y must have valid ghosts.                  */
int bhah_hamiltonian_constraint(const bhah_grid* g, const double* y, double* H,
                                void* stream);

/* ---- ensembles: many independent grids advanced together ---------------- *
 * A batch advances n independent grids (jobs) that share gauge parameters.
 * It is the ensemble form of bhah_rk4_step: per stage, one persistent
 * right-hand-side kernel per kernel variant (coordinate family, two phi
 * planes or more) strides over a (job, tile) work list covering every active
 * job, one kernel evolves the outer points of radiation-boundary jobs, and
 * one ghost-fill kernel runs over a (job, ghost chunk) list; the grids may
 * mix both outer-boundary kinds. A step count's worth of stages is captured once
 * in a hipGraph and replayed. The per-point arithmetic is the same device
 * code as bhah_rk4_step, so each job's result equals its solo evolution
 * bit for bit. Tile shapes are chosen per size class (coordinate family and
 * interior extents) by timing the candidates on the jobs' own data the first
 * time the class is seen (right-hand side written into workspace, which
 * every step overwrites anyway). tune_cache_path may be NULL; if it names a
 * file, choices are read from it and written back (JSON, one entry per
 * line). The same grid may appear several times (jobs of one resolution).
 * Device memory held by the batch: a work description of roughly
 * 750 B per job + 8 B per tile + 8 B per 256 ghost or radiation points.
 * Errors: BHAH_EINVAL for NULL or inconsistent arguments, BHAH_EDEVICE /
 * BHAH_ENOMEM from the runtime. Calls on one batch must not overlap and must
 * be ordered on one stream (or the caller orders them).                      */
int bhah_batch_create(const bhah_grid* const* grids, int n,
                      const bhah_gauge_params* gp, const char* tune_cache_path,
                      bhah_batch** out);

/* Advance the jobs with host_active[j] != 0 (host_active may be NULL: all)
 * by nsteps RK4 steps each, job j at its own step host_dt[j], on y[j]
 * (state, valid ghosts) with workspace ws[j] (info.workspace_doubles).
 * On return every ghost of y[j] is valid again. Between the steps inside
 * one captured graph only the ghosts the stencils read are refilled (phi
 * ghost planes are exact periodic copies that the stencils never read);
 * the results are the same as nsteps calls of bhah_rk4_step, bit for bit.
 * y, ws and host_dt are host arrays of n entries (device pointers in y, ws).
 * Asynchronous on stream; the first call for a new size class also times
 * tile candidates (synchronising the stream).                               */
int bhah_batch_step(bhah_batch* b, double* const* y, double* const* ws,
                    const double* host_dt, const unsigned char* host_active,
                    int nsteps, void* stream);

/* RK4 steps captured per graph (default 10; larger step counts replay it). */
int bhah_batch_set_graph_steps(bhah_batch* b, int steps);

/* Time integrator of the batch's steps: BHAH_RK4 (the default) or
 * BHAH_SSPRK3. Each job then equals its solo bhah_rk4_step /
 * bhah_ssprk3_step evolution bit for bit. Takes effect at the next
 * bhah_batch_step (the captured graphs are rebuilt). BHAH_EINVAL otherwise. */
int bhah_batch_set_integrator(bhah_batch* b, int integrator);

/* Launch shape of the right-hand-side kernel: blocks_per_cu > 0 runs that
 * many persistent 64-lane blocks per compute unit striding over the work
 * list (default 4: one wave per SIMD); 0 launches one block per tile.       */
int bhah_batch_set_blocks_per_cu(bhah_batch* b, int blocks_per_cu);

typedef struct {
  int n_active;          /* jobs in the current work lists                   */
  int n_tiles;           /* (job, tile) entries, 64 points each              */
  int n_chunks;          /* (job, 256 ghost points) entries                  */
  int graph_steps;       /* RK4 steps per captured graph                     */
  int rhs_blocks;        /* persistent blocks of the right-hand-side kernel  */
  int n_classes_tuned;   /* size classes with a tile choice                  */
  double tune_seconds;   /* wall time spent timing tile candidates           */
  int blocks_per_cu;     /* persistent RHS blocks per CU (0: one per tile)   */
  /* launch tuning (bhah_batch_set_launch_tuning) for the current job set:
   * microseconds per step of the chosen graph steps / blocks per CU and of
   * the default (10, 4), candidates timed, seconds spent, and 1 if the
   * choice came from the cache file (then nothing was timed)              */
  double launch_us_per_step, launch_default_us_per_step, launch_tune_seconds;
  int launch_candidates, launch_from_cache;
} bhah_batch_info;

int bhah_batch_get_info(const bhah_batch* b, bhah_batch_info* info);

/* Launch tuning (off by default): with on != 0, the first bhah_batch_step
 * on a job set not seen before times every pair of graph steps {4, 10, 25}
 * and persistent blocks per CU {2, 4, 8, one per tile} on device copies of
 * the jobs' states (the caller's states are untouched; the results are the
 * same bit for bit whatever the pair), keeps the fastest (the default
 * (10, 4) unless another is more than 2% faster) and stores it per job-set
 * signature (the multiset of grid shapes, numerics and the integrator) in
 * the tile cache file. The copies need one state per job of device memory
 * for the duration of the tuning (BHAH_ENOMEM otherwise).                   */
int bhah_batch_set_launch_tuning(bhah_batch* b, int on);

/* Tile choice for job j's size class: log2 extents along i0 and i1 (the
 * extent along i2 is 64 >> (lx + ly)) and band (tile rows of i1 walked
 * together). Defaults (6, 0, 4) before the class is tuned.                  */
int bhah_batch_get_tile(const bhah_batch* b, int j, int* lx, int* ly, int* band);

void bhah_batch_destroy(bhah_batch* b);

/* ---- serving: continuous batching of evolution jobs ---------------------- *
 * A server accepts head-on (or any Brill-Lindquist) evolution jobs as they
 * arrive, admits them while a job slot is free and the device memory it
 * holds for job states stays within budget_bytes, keeps every admitted
 * job's state (state + RK4 workspace, 4 x info.state_doubles doubles) in
 * device memory, and on each tick advances all running jobs together
 * through one ensemble engine (bhah_batch's kernels and graphs), each job
 * taking min(its steps left, steps_per_tick) steps. Jobs of one grid shape
 * share one bhah_grid; freed state slots are reused by later jobs of the
 * same shape, and free slots of other shapes are given back to the device
 * when a queued job would not fit the budget otherwise. Times are seconds
 * since bhah_server_create on the host steady clock; device-side times
 * (a job's completion, busy time, step latency) come from events on the
 * server's stream mapped onto that clock.                                  */
typedef struct bhah_server bhah_server;

typedef struct {
  double budget_bytes;      /* device memory for job states                   */
  int max_jobs;             /* running jobs at most                           */
  int steps_per_tick;       /* RK4 steps per tick at most                     */
  int keep_results;         /* 1: a finished job's state stays until fetched  */
  long long target_points;  /* admit while running jobs hold fewer interior
                               points than this (0: no limit); about four
                               64-point tiles per SIMD fill the GPU, more only
                               lengthens every running job's step           */
  bhah_gauge_params gauge;
  const char* tune_cache_path; /* may be NULL                                 */
  int integrator;           /* BHAH_RK4 or BHAH_SSPRK3                        */
} bhah_server_params;

typedef struct {
  bhah_grid_params grid;
  int n_punct;              /* <= 16                                          */
  double masses[16];
  double pos[16][3];        /* Cartesian positions                            */
  int lapse_kind;           /* 0 or 1, as bhah_set_initial_data_brill_lindquist */
  long long nsteps;         /* RK4 steps at the grid's CFL dt (info.dt)       */
} bhah_job_desc;

/* DONE: finished, state kept for bhah_server_fetch (keep_results);
 * RELEASED: finished and its memory reused; FAILED: its initial data could
 * not be set at admission (it left the queue, other jobs go on).           */
enum { BHAH_JOB_QUEUED = 0, BHAH_JOB_RUNNING = 1, BHAH_JOB_DONE = 2, BHAH_JOB_RELEASED = 3, BHAH_JOB_FAILED = 4 };

typedef struct {
  int state;                /* BHAH_JOB_*                                      */
  long long steps_done;
  long long interior_points;
  double t_submit, t_admit, t_done;   /* -1 while not reached               */
} bhah_job_status;

typedef struct {
  long long submitted, done, running, queued;
  long long point_steps;    /* interior point RK4 updates done                */
  double busy_seconds;      /* summed wall time of ticks that ran work        */
  double elapsed_seconds;   /* since create                                   */
  double step_ms_p50, step_ms_p99;  /* per job-step latency over all steps    */
  double job_s_p50, job_s_p99;      /* submit -> done of finished jobs        */
  double held_bytes, peak_held_bytes;
  int peak_running;
  long long failed;         /* jobs that failed at admission                  */
} bhah_server_stats;

/* stream: the stream every device operation of the server runs on.          */
int bhah_server_create(const bhah_server_params* p, void* stream, bhah_server** out);
/* Queue a job (arrival time = now); *id receives its handle. BHAH_EINVAL
 * for a NULL argument, n_punct outside 0..16, nsteps < 0, lapse_kind not 0
 * or 1, invalid grid parameters, or a job larger than the whole budget.     */
int bhah_server_submit(bhah_server* s, const bhah_job_desc* job, long long* id);
/* Admit queued jobs that fit (their initial data is set on the stream),
 * enqueue one graph launch in which every running job takes
 * min(steps_per_tick, its steps left) steps, then wait for the previous
 * tick's device work: at most one tick is in flight, so the host's
 * admission and bookkeeping overlap the device's steps. Jobs whose last
 * steps complete become DONE (keep_results) or RELEASED; a job's results
 * are final once its status says so. With nothing left running or queued
 * the tick also waits for its own work, so a tick that reports no job
 * running and none queued has completed everything. *running (jobs with
 * steps still to enqueue) and *queued (may be NULL) receive the counts
 * after the tick; bhah_server_get_stats counts as running also the jobs
 * whose last steps are still in flight.                                     */
int bhah_server_tick(bhah_server* s, int* running, int* queued);
int bhah_server_job_status(const bhah_server* s, long long id, bhah_job_status* st);
/* Copy a finished job's state (info.state_doubles doubles, device pointer
 * dst, ordered on the server's stream and completed on return) and release
 * its memory. BHAH_EINVAL if the job is unknown, not done or released.      */
int bhah_server_fetch(bhah_server* s, long long id, double* dst);
int bhah_server_get_stats(const bhah_server* s, bhah_server_stats* st);
void bhah_server_destroy(bhah_server* s);

/* ---- machine peaks --------------------------------------------------------
 * Measured ceilings of the current device, for reading the kernels' roofline
 * fractions against what the card sustains as well as against its published
 * figures. *fp64_tflops: independent FP64 FMA chains (2 flops per FMA) at
 * full occupancy. *hbm_gbps: a streaming triad a = b + s*c over three 2 GiB
 * arrays, 48 bytes moved per pair of doubles. Outputs are host pointers.
 * Allocates about 6 GiB of device memory for the duration of the call and
 * frees it; returns after the stream has drained. BHAH_EINVAL on NULL
 * outputs, BHAH_EDEVICE on a HIP failure.                                   */
int bhah_probe_peaks(double* fp64_tflops, double* hbm_gbps, void* stream);

/* Message describing the last failed call on this thread ("" if none).      */
const char* bhah_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BHAH_H */
