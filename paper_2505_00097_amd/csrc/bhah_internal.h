// bhah_internal.h -- internal types of the HIP library (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bhah.h"

namespace bhah {

constexpr int NG = 3;     // ghost layers of the 4th-order grids (5 for 8th order)
constexpr int NGF = 24;   // evolved gridfunctions
constexpr int NAUX = 9;   // rescaled Ricci (6) + contracted d Gammabar term (3)

// Per-direction 1-D tables, one row per grid index (ghosts included), TAB_W
// doubles per row. Mapped directions (r or rho, and z): [map, d map, d2 map,
// d3 map, 1/map, 1/d map] (derivatives with respect to the logical
// coordinate). Angles (theta, phi): [sin, cos, 1/sin].
constexpr int TAB_W = 8;

#ifndef BHAH_DEFAULT_BAND
#define BHAH_DEFAULT_BAND 4
#endif
#ifndef BHAH_NXCD
#define BHAH_NXCD 8
#endif

// Everything a kernel needs to address one grid. Passed by value.
struct GridDev {
  int coord;
  int N0, N1, N2;      // interior points
  int n0, n1, n2;      // incl. ghosts
  int s1, s2;          // flat strides of i1, i2 (s0 = 1)
  int ng;              // ghost layers N_G (3 or 5): differences of order 2 (N_G - 1)
  long long sgf;       // gridfunction stride = n0*n1*n2
  double inv_dx[3];    // 1/dxx
  const double* tab0;  // [n0][TAB_W]
  const double* tab1;  // [n1][TAB_W]
  const double* tab2;  // [n2][TAB_W]
};

// sign flip of gridfunction g under the parity bits par (bit d: the
// direction-d basis vector reverses); tensor type per gridfunction: scalar,
// vector (index i) or rank 2 (indices i, j). The flip is the parity of the
// reversed directions among the gridfunction's indices: a mask of them per
// gridfunction (a direction that appears twice cancels), four bits each,
// packed into two 64-bit constants so that the lookup needs no memory.
__host__ __device__ constexpr unsigned long long gf_flip_masks(int first) {
  constexpr int I[NGF] = {0, 0, 0, 1, 1, 2, -1, 0, 1, 2, -1, 0, 0, 0, 1, 1, 2, 0, 1, 2, -1, 0, 1, 2};
  constexpr int J[NGF] = {0, 1, 2, 1, 2, 2, -1, -1, -1, -1, -1, 0, 1, 2, 1, 2, 2, -1, -1, -1, -1, -1, -1, -1};
  unsigned long long m = 0;
  for (int g = first; g < first + 16 && g < NGF; g++) {
    unsigned long long b = 0;
    if (I[g] >= 0) b ^= 1ull << I[g];
    if (J[g] >= 0) b ^= 1ull << J[g];
    m |= b << (4 * (g - first));
  }
  return m;
}
__host__ __device__ __forceinline__ int gf_flip(int g, int par) {
  constexpr unsigned long long LO = gf_flip_masks(0), HI = gf_flip_masks(16);
  const unsigned m = (unsigned)((g < 16 ? LO >> (4 * g) : HI >> (4 * (g - 16))) & 0xFull);
  return __builtin_popcount((unsigned)par & m) & 1;
}

// Ghost fill list: every ghost point p receives
//   y_g[p] = sign_g(parity_p) * sum_t w_t * y_g[src_t]
// over interior sources only (outer extrapolation composed in exact integer
// arithmetic on the host; inner copies carry their source's combination).
struct GhostDev {
  int n_ghost;
  const int* dst;       // [n_ghost]
  const int* start;     // [n_ghost + 1] offsets into src/w
  const int* parity;    // [n_ghost] bit d: e~_(d) flips
  const int* src;       // [n_terms]
  const double* w;      // [n_terms]
};

// Pure-outer ghost points evolved by the radiation condition: flat index,
// packed stencil starts (s0 + 2R) | (s2 + 2R) << 4 of the (2R+1)-point
// logical derivatives along xx0 and xx2 (s in -2R..0, R = N_G - 1), and per
// point 1/r and
// (rhat . grad xx^k) / dxx^k for k = 0, 2 (zero where r does not depend on
// xx^k).
struct RadDev {
  int n;
  const int* q;       // [n]
  const int* shift;   // [n]
  const double* coef;  // [n][3]
  int R;              // stencil radius N_G - 1
  const double* w;    // [2R+1][2R+1]: row s + 2R holds the weights of nodes s..s+2R
};
// host copy of a ghost list in the GhostDev layout
struct HostGhosts {
  std::vector<int> dst, start, par, src;
  std::vector<double> w;
};

// RK stage epilogue of the right-hand-side kernel: with rhs != nullptr the
// right-hand side k is stored; otherwise out1 = base1 + c1 k and, if out2 is
// set, out2 = base2 + c2 k, gridfunction by gridfunction. With base2 set but
// no out2 the stage mixes two states: out1 = m1 base1 + m2 base2 + c1 k.
struct StageArgs {
  double* rhs;
  const double* base1;
  double* out1;
  double c1;
  const double* base2;
  double* out2;
  double c2;
  double m1, m2;
};

// Gauge and dissipation parameters as the right-hand-side kernel takes them:
// eta of Eq. 15, Kreiss-Oliger strengths for gauge and metric variables.
struct Gauge {
  double eta, dg, dm;
  bool ko() const { return dg != 0.0 || dm != 0.0; }
};
inline Gauge gauge_of(const bhah_gauge_params& p) { return Gauge{p.eta, p.diss_gauge, p.diss_metric}; }
// BHAH_OK, or BHAH_EINVAL with a message naming the caller
int check_gauge(const bhah_gauge_params* gp, const char* who);

// Tile shape and walk of the right-hand-side kernel over one grid: tiles of
// 64 points, 2^lx along i0, 2^ly along i1 and 64 >> (lx + ly) along i2,
// walked in bands of `band` tile rows of i1.
struct TileCfg {
  int lx, ly, band;
  int waves = 1;  // waves per 64-point tile of the solo kernel: 1 (rhs_fused.hip) or 2 (rhs_pair.hip)
};

// The stencil code reads the periodic direction (phi: i1 on SinhCylindrical
// grids, i2 otherwise) with a wave-uniform wrapped index, so a tile must
// have extent 1 along it.
inline bool tile_fits_periodic(int coord, const TileCfg& c) {
  return coord == BHAH_SINH_CYLINDRICAL ? c.ly == 0 : c.lx + c.ly == 6;
}

// The right-hand-side kernel is built per coordinate family, per phi extent
// and per differencing order: a grid with exactly two interior phi planes
// (axisymmetric runs) gets a variant that reads each phi stencil as its two
// planes and drops the phi derivatives that vanish identically there.
// Variant = 2 coord + that, plus 6 for the 8th-order grids (5 ghost layers).
constexpr int NVAR = 12;
__host__ __device__ inline int rhs_variant(int coord, int N1, int N2, int ng = NG) {
  return 2 * coord + ((coord == BHAH_SINH_CYLINDRICAL ? N1 : N2) == 2 ? 1 : 0) + (ng == 5 ? 6 : 0);
}

struct TileMap {
  int lx, ly;
  int tx, ty, tz;  // tiles along i0, i1, i2
  int band;        // tile rows of i1 per band
  int ntiles;      // tx * ty * tz
};

// One job of an ensemble as the batched kernels see it. Stage s in 0..3 is
// RK4 stage s + 1 (the right-hand side of in[s] combined as in st[s], then
// the ghost fill of gdst[s] from list gh[0] (ghosts with an interior phi
// index, all the stencils read) or gh[1] (all ghosts, after the last stage
// of a batch step)); stage 4 stores the right-hand side of in[4] in
// st[4].rhs and fills nothing (used to time tile shapes).
struct BatchJob {
  GridDev G;
  GhostDev gh[2];  // ghosts with an interior phi index; all ghosts
  RadDev rad;      // outer points evolved by the radiation condition (n = 0 otherwise)
  TileMap T;
  StageArgs st[5];
  const double* in[5];
  double* gdst[5];
};

// Work list header: the (job, tile) list of kernel variant v (rhs_variant)
// starts at tile_off[v] and holds n_tiles[v] entries; the (job, chunk of 256 ghost
// points) list of ghost list w (as BatchJob::gh) starts at chunk_off[w] and
// holds n_chunks[w] entries; chunk list 2 is the (job, chunk of 256
// radiation points) list.
struct BatchHdr {
  int n_tiles[NVAR];
  int tile_off[NVAR];
  int n_chunks[3];
  int chunk_off[3];
};

// Ghost classification of a point from the closed-form index reflections
// that the Cartesian round trip reduces to (Sec. 3): 0 interior, 1 pure
// outer (the round trip returns the point itself), 2 inner, with the source
// point and parity bits (bit d: the direction-d basis vector reverses).
struct Classifier {
  int coord = 0;
  int ng = NG;
  int N[3] = {0, 0, 0};
  int n[3] = {0, 0, 0};
  int flat(int a, int b, int c) const { return (int)(a + n[0] * (b + n[1] * (long long)c)); }
  int wrap(int j, int N) const {
    int m = (j - ng) % N;
    if (m < 0) m += N;
    return ng + m;
  }
  int operator()(int i0, int i1, int i2, int& src, int& par) const {
    src = flat(i0, i1, i2);
    par = 0;
    if (i0 >= ng && i0 < ng + N[0] && i1 >= ng && i1 < ng + N[1] && i2 >= ng && i2 < ng + N[2]) return 0;
    int j0 = i0, j1 = i1, j2 = i2;
    if (coord == BHAH_SINH_CYLINDRICAL) {
      if (j0 < ng) { j0 = 2 * ng - 1 - j0; j1 += N[1] / 2; par ^= 0b011; }
      j1 = wrap(j1, N[1]);
    } else {
      if (j0 < ng) { j0 = 2 * ng - 1 - j0; j1 = N[1] + 2 * ng - 1 - j1; j2 += N[2] / 2; par ^= 0b101; }
      if (j1 < ng) { j1 = 2 * ng - 1 - j1; j2 += N[2] / 2; par ^= 0b110; }
      else if (j1 >= N[1] + ng) { j1 = 2 * (N[1] + ng) - 1 - j1; j2 += N[2] / 2; par ^= 0b110; }
      j2 = wrap(j2, N[2]);
    }
    if (j0 == i0 && j1 == i1 && j2 == i2) { par = 0; return 1; }
    src = flat(j0, j1, j2);
    return 2;
  }
};

}  // namespace bhah

struct bhah_grid {
  bhah_grid_params params;
  bhah_grid_info info;
  int device;
  bhah::GridDev dev;       // device pointers inside
  bhah::GhostDev ghost;    // device pointers inside
  // host copies
  std::vector<double> tab[3];
  bhah::Classifier classify;  // ghost class of any point (closed form)
  std::vector<int> g_dst, g_start, g_par, g_src;
  std::vector<double> g_w;
  // ghosts filled after the first three RK stages: those whose phi index is
  // an interior one (phi ghost planes are never read by the stencils, which
  // wrap phi onto the interior; they are filled after the last stage)
  std::vector<int> r_dst, r_start, r_par, r_src;
  std::vector<double> r_w;
  bhah::GhostDev ghost_stage;  // device view of the r_* list
  int max_terms;
  bhah::TileCfg tile;  // tile shape and walk of the RHS kernel
  // radiation outer boundary: the evolved outer points and the inner ghosts
  // as one-hop parity copies (all of them; those with an interior phi index)
  std::vector<int> rad_q, rad_shift;
  std::vector<double> rad_coef, rad_w;
  bhah::HostGhosts inner_full, inner_stage;
  bhah::RadDev rad{};
  bhah::GhostDev ghost_inner{}, ghost_inner_stage{};
  int* d_rad_i = nullptr;     // q | shift
  double* d_rad_c = nullptr;
  int* d_inner_ints[2] = {nullptr, nullptr};
  double* d_inner_w[2] = {nullptr, nullptr};
  // device allocations
  double* d_tab[3];
  int* d_ints;      // dst | start | parity | src packed
  double* d_w;
  int* d_rints;     // the same for the stage ghost list
  double* d_rw;
  long long n_int_block;
};

namespace bhah {
// kernel launchers (device code in the .hip sources)
void launch_ghosts(const GhostDev& gh, double* y, long long sgf, hipStream_t s);
int launch_brill_lindquist(const GridDev& G, int n, const double* m, const double* pos, int lapse_kind,
                           double* y, hipStream_t s);
void launch_rhs_fused(const GridDev& G, const Gauge& ga, const double* y, double* aux, const StageArgs& st,
                      hipStream_t s, const TileCfg& cfg);
TileMap make_tilemap(const GridDev& G, int lx, int ly, int band);
// the right-hand side with two waves per tile (rhs_pair.hip); same
// arguments and results as the one-wave kernel, to rounding; built for the
// variants have_rhs_pair reports
bool have_rhs_pair(const GridDev& G, bool ko);
void launch_rhs_pair(const GridDev& G, const Gauge& ga, const double* y, double* aux, const StageArgs& st,
                     hipStream_t s, const TileMap& T);
// mix: the stages may combine two states (SSPRK3); RK4 stages never do.
// counts (device, one int per job; NULL: every job) and kk: step kk of a
// graph launch runs only the jobs with kk < counts[job].
void launch_rhs_batch(int variant, const BatchJob* jobs, const BatchHdr* hdr, const int2* work, int stage,
                      const int* counts, int kk, const Gauge& ga, bool mix, int blocks, hipStream_t s);
// last: the last stage of step kk (a job at its last active step then
// fills all its ghosts)
void launch_ghosts_batch(const BatchJob* jobs, const BatchHdr* hdr, const int2* work, int stage, const int* counts,
                         int kk, bool last, int blocks, hipStream_t s);
void launch_hamiltonian(const GridDev& G, const double* y, double* H, hipStream_t s);
// radiation condition at the pure-outer points of one stage: the right-hand
// side of `in` combined as in st (same semantics as the RHS kernel)
void launch_radiation(const GridDev& G, const RadDev& R, const double* in, const StageArgs& st, hipStream_t s);
void launch_radiation_batch(const BatchJob* jobs, const BatchHdr* hdr, const int2* work, int stage,
                            const int* counts, int kk, int blocks, hipStream_t s);
void launch_constraints(const GridDev& G, const double* y, double* H, double* Mo, double* Co, hipStream_t s);

// The four stages of one classical RK4 step on state y with workspace ws
// (three state-sized arrays A, B, Cacc): inputs, stage combinations and the
// array whose ghosts are filled after each stage.
void rk4_stages(double dt, double* y, double* ws, long long n, StageArgs st[4], const double* in[4],
                double* gdst[4]);
// The same for the three stages of one SSPRK3 step (arrays A, B of ws).
void ssprk3_stages(double dt, double* y, double* ws, long long n, StageArgs st[3], const double* in[3],
                   double* gdst[3]);

// device address of this device's bhah_rk4_step_noalloc workspace (3 x NGF x
// BHAH_NOALLOC_MAX_POINTS doubles), looked up on first use per device
int noalloc_workspace(double** ws);

void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int check_hip(hipError_t e, const char* what);
}  // namespace bhah
