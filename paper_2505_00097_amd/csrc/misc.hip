// misc.hip -- ghost fill and Brill-Lindquist initial data; the workspace of
// the allocation-free RK4 entry point.
#include <mutex>

#include "bhah_internal.h"

namespace bhah {

// Workspace of bhah_rk4_step_noalloc (three states of at most
// BHAH_NOALLOC_MAX_POINTS points): a file-scope device array, one copy per
// device. In host code its name is a host-side stand-in, never a device
// address: kernels get the address that hipGetSymbolAddress returns for the
// current device, looked up once per device and kept below.
constexpr long long kScratchDoubles = 3LL * NGF * BHAH_NOALLOC_MAX_POINTS;
static __device__ __align__(256) double scratch[kScratchDoubles];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

int noalloc_workspace(double** ws) {
  int dev = 0;
  if (int rc = check_hip(hipGetDevice(&dev), "hipGetDevice")) return rc;
  if (dev < 0 || dev >= kMaxDevices) return fail(BHAH_EINVAL, "bhah_rk4_step_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (int rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress")) return rc;
    g_scratch_ptr[dev] = (double*)p;
  }
  *ws = g_scratch_ptr[dev];
  return BHAH_OK;
}

// Every ghost point takes sign * sum_t w_t y[src_t]; all sources are interior
// points, so ghosts can be filled in any order and in parallel (Sec. 3
// outer-then-inner boundary order is folded into the weights on the host).
// A thread fills GF_PER gridfunctions of one ghost point; blockIdx.y picks the
// group of gridfunctions, so a fill runs NGF / GF_PER times more threads than
// ghost points and keeps more loads in flight.
constexpr int GF_PER = 4;
static_assert(NGF % GF_PER == 0, "gridfunction groups");
// Terms are fetched GT at a time: the chunk's weights and source indices in
// one round of loads, then its values in the next, so a ghost of up to GT
// terms (every face ghost of an extrapolating boundary has three) costs three
// dependent rounds (record, terms, values) instead of two per term. The sum
// still runs in term order, one fused multiply-add per term.
constexpr int GT = 4;

__device__ __forceinline__ void ghost_point(const GhostDev& gh, double* __restrict__ y, long long sgf, int t,
                                            int g0) {
  const int dst = gh.dst[t], s0 = gh.start[t], s1 = gh.start[t + 1], par = gh.parity[t];
  // all loads before any store: sources are interior points, never ghosts,
  // but the compiler cannot know that and would otherwise keep each load
  // behind the previous store
  double v[GF_PER];
  if (s1 - s0 == 1) {
    const int src = gh.src[s0];
#pragma unroll
    for (int j = 0; j < GF_PER; j++) v[j] = y[(g0 + j) * sgf + src];
  } else {
#pragma unroll
    for (int j = 0; j < GF_PER; j++) v[j] = 0.0;
    for (int k = s0; k < s1; k += GT) {
      // past the last term the chunk rereads that term (in bounds, not summed)
      double w[GT], x[GT][GF_PER];
#pragma unroll
      for (int u = 0; u < GT; u++) {
        const int ku = min(k + u, s1 - 1);
        w[u] = gh.w[ku];
        const int src = gh.src[ku];
#pragma unroll
        for (int j = 0; j < GF_PER; j++) x[u][j] = y[(g0 + j) * sgf + src];
      }
#pragma unroll
      for (int u = 0; u < GT; u++)
        if (k + u < s1) {
#pragma unroll
          for (int j = 0; j < GF_PER; j++) v[j] += w[u] * x[u][j];
        }
    }
  }
#pragma unroll
  for (int j = 0; j < GF_PER; j++) y[(g0 + j) * sgf + dst] = gf_flip(g0 + j, par) ? -v[j] : v[j];
}

__global__ void __launch_bounds__(256) k_ghosts(GhostDev gh, double* __restrict__ y, long long sgf) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < gh.n_ghost) ghost_point(gh, y, sgf, t, (int)blockIdx.y * GF_PER);
}

void launch_ghosts(const GhostDev& gh, double* y, long long sgf, hipStream_t s) {
  if (gh.n_ghost == 0) return;
  hipLaunchKernelGGL(k_ghosts, dim3((gh.n_ghost + 255) / 256, NGF / GF_PER), dim3(256), 0, s, gh, y, sgf);
}

// Ensemble form: a fixed grid of blocks strides over the (job, chunk of 256
// ghost points) work lists (x) for one group of gridfunctions (y) and fills
// the ghosts of the stage's target array, for the jobs active in step kk of
// the launch (kk < counts[job]): list 0 (ghosts with an interior phi index,
// all that the stencils read) after every stage, except after the last
// stage of a job's last active step (last != 0 and kk == counts[job] - 1),
// which fills list 1 (all ghosts).
__global__ void __launch_bounds__(256) k_ghosts_batch(const BatchJob* __restrict__ jobs,
                                                      const BatchHdr* __restrict__ hdr,
                                                      const int2* __restrict__ work, int stage,
                                                      const int* __restrict__ counts, int kk, int last) {
  const int n0 = hdr->n_chunks[0];
  const int n = last ? n0 + hdr->n_chunks[1] : n0;
  const int g0 = (int)blockIdx.y * GF_PER;
  for (int c = (int)blockIdx.x; c < n; c += (int)gridDim.x) {
    const int w = c < n0 ? 0 : 1;
    const int2 wk = work[hdr->chunk_off[w] + (w ? c - n0 : c)];
    const int cnt = counts[wk.x];
    if (kk >= cnt) continue;  // the job takes no more steps in this launch
    if (w != (last && kk == cnt - 1 ? 1 : 0)) continue;
    const BatchJob* J = jobs + wk.x;
    const int t = wk.y * 256 + (int)threadIdx.x;
    if (t < J->gh[w].n_ghost) ghost_point(J->gh[w], J->gdst[stage], J->G.sgf, t, g0);
  }
}

void launch_ghosts_batch(const BatchJob* jobs, const BatchHdr* hdr, const int2* work, int stage, const int* counts,
                         int kk, bool last, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_ghosts_batch, dim3(blocks, NGF / GF_PER), dim3(256), 0, s, jobs, hdr, work, stage, counts,
                     kk, last ? 1 : 0);
}

constexpr int MAX_PUNCT = 16;
struct Punctures {
  int n;
  int lapse_kind;
  double m[MAX_PUNCT];
  double x[MAX_PUNCT][3];
};

// Brill-Lindquist (analytic stand-in for the TwoPunctures data of Sec. 4.1):
// psi = 1 + sum m_n / (2 |x - x_n|); W = psi^-2; alpha =
// psi^-2 (precollapsed) or 1; all other variables zero. Interior points.
__global__ void __launch_bounds__(64) k_brill_lindquist(GridDev G, Punctures P, double* __restrict__ y) {
  const int i0 = G.ng + (int)(blockIdx.x * blockDim.x + threadIdx.x);
  const int i1 = G.ng + (int)blockIdx.y, i2 = G.ng + (int)blockIdx.z;
  if (i0 >= G.ng + G.N0) return;
  const double r = G.tab0[i0 * TAB_W];
  double x[3];
  if (G.coord == BHAH_SINH_CYLINDRICAL) {
    const double sp = G.tab1[i1 * TAB_W], cp = G.tab1[i1 * TAB_W + 1];
    x[0] = r * cp; x[1] = r * sp; x[2] = G.tab2[i2 * TAB_W];
  } else {
    const double st = G.tab1[i1 * TAB_W], ct = G.tab1[i1 * TAB_W + 1];
    const double sp = G.tab2[i2 * TAB_W], cp = G.tab2[i2 * TAB_W + 1];
    x[0] = r * st * cp; x[1] = r * st * sp; x[2] = r * ct;
  }
  double psi = 1.0;
  for (int n = 0; n < P.n; n++) {
    const double dx = x[0] - P.x[n][0], dy = x[1] - P.x[n][1], dz = x[2] - P.x[n][2];
    psi += P.m[n] / (2.0 * sqrt(dx * dx + dy * dy + dz * dz));
  }
  const double ip2 = 1.0 / (psi * psi);
  const long long q = i0 + (long long)G.s1 * i1 + (long long)G.s2 * i2;
#pragma unroll
  for (int g = 0; g < NGF; g++) y[g * G.sgf + q] = 0.0;
  y[10 * G.sgf + q] = ip2;                              // cf
  y[6 * G.sgf + q] = P.lapse_kind == 0 ? ip2 : 1.0;     // alpha
}

// ---- Sommerfeld radiation condition at the pure-outer points --------------
// d_t f = -v (f - f_inf)/r - v (c0 D0 f + c2 D2 f), with D_k the
// (2R+1)-point first derivative of the grid's order (R = N_G - 1) in grid
// units along xx^k starting s_k points from the point (s = -R centred, lower
// at a max face, higher at a min face) and c_k = (rhat . grad xx^k)/dxx^k
// precomputed per point; the weights of every start come from the grid's
// table. One thread per (outer point, group of GF_PER gridfunctions); the
// result is combined into the stage arrays exactly as the right-hand-side
// kernel does it.
template <int RS>
__device__ __forceinline__ void radiation_point(const GridDev& G, const RadDev& R, int t,
                                                const double* __restrict__ in, const StageArgs& st, int g0) {
  constexpr int W = 2 * RS + 1;  // RS: the stencil radius R.R
  const long long q = R.q[t];
  const int sh = R.shift[t];
  const int s0 = (sh & 15) - 2 * RS, s2 = ((sh >> 4) & 15) - 2 * RS;
  double w0[W], w2[W];
#pragma unroll
  for (int m = 0; m < W; m++) {
    w0[m] = R.w[(s0 + 2 * RS) * W + m];
    w2[m] = R.w[(s2 + 2 * RS) * W + m];
  }
  const double ir = R.coef[3 * t], c0 = R.coef[3 * t + 1], c2 = R.coef[3 * t + 2];
  const bool cyl = G.coord == BHAH_SINH_CYLINDRICAL;
  double k[GF_PER];
#pragma unroll
  for (int j = 0; j < GF_PER; j++) {
    const int g = g0 + j;
    const double* f = in + g * G.sgf + q;
    double d0 = 0.0, d2 = 0.0;
#pragma unroll
    for (int m = 0; m < W; m++) d0 += w0[m] * f[s0 + m];
    if (cyl) {
#pragma unroll
      for (int m = 0; m < W; m++) d2 += w2[m] * f[(long long)(s2 + m) * G.s2];
    }
    const double v = g == BHAH_ALPHA ? 1.4142135623730951 : 1.0;  // sqrt(2) for the lapse
    const double finf = (g == BHAH_ALPHA || g == BHAH_CF) ? 1.0 : 0.0;
    k[j] = -v * (f[0] - finf) * ir - v * (c0 * d0 + c2 * d2);
  }
  // the stage combination (semantics of StageArgs)
#pragma unroll
  for (int j = 0; j < GF_PER; j++) {
    const long long e = (g0 + j) * G.sgf + q;
    if (st.rhs) {
      st.rhs[e] = k[j];
    } else if (st.out2 == nullptr && st.base2 != nullptr) {
      st.out1[e] = st.m1 * st.base1[e] + st.m2 * st.base2[e] + st.c1 * k[j];
    } else {
      const double b1 = st.base1[e], b2 = st.out2 ? st.base2[e] : 0.0;
      st.out1[e] = b1 + st.c1 * k[j];
      if (st.out2) st.out2[e] = b2 + st.c2 * k[j];
    }
  }
}

template <int RS>
__global__ void __launch_bounds__(256) k_radiation(GridDev G, RadDev R, const double* __restrict__ in,
                                                   StageArgs st) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < R.n) radiation_point<RS>(G, R, t, in, st, (int)blockIdx.y * GF_PER);
}

void launch_radiation(const GridDev& G, const RadDev& R, const double* in, const StageArgs& st, hipStream_t s) {
  if (R.n == 0) return;
  const dim3 grid((R.n + 255) / 256, NGF / GF_PER);
  if (R.R == 4) hipLaunchKernelGGL(k_radiation<4>, grid, dim3(256), 0, s, G, R, in, st);
  else hipLaunchKernelGGL(k_radiation<2>, grid, dim3(256), 0, s, G, R, in, st);
}

// Ensemble form: blocks stride over the (job, chunk of 256 radiation points)
// list; each job's stage input, combination and stencil radius come from its
// table entry. Jobs with no step kk in this launch (kk >= counts[job]) idle.
__global__ void __launch_bounds__(256) k_radiation_batch(const BatchJob* __restrict__ jobs,
                                                         const BatchHdr* __restrict__ hdr,
                                                         const int2* __restrict__ work, int stage,
                                                         const int* __restrict__ counts, int kk) {
  const int n = hdr->n_chunks[2];
  const int2* wl = work + hdr->chunk_off[2];
  const int g0 = (int)blockIdx.y * GF_PER;
  for (int c = (int)blockIdx.x; c < n; c += (int)gridDim.x) {
    const int2 wk = wl[c];
    if (kk >= counts[wk.x]) continue;
    const BatchJob* J = jobs + wk.x;
    const int t = wk.y * 256 + (int)threadIdx.x;
    if (t < J->rad.n) {
      if (J->rad.R == 4) radiation_point<4>(J->G, J->rad, t, J->in[stage], J->st[stage], g0);
      else radiation_point<2>(J->G, J->rad, t, J->in[stage], J->st[stage], g0);
    }
  }
}

void launch_radiation_batch(const BatchJob* jobs, const BatchHdr* hdr, const int2* work, int stage,
                            const int* counts, int kk, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_radiation_batch, dim3(blocks, NGF / GF_PER), dim3(256), 0, s, jobs, hdr, work, stage, counts,
                     kk);
}

int launch_brill_lindquist(const GridDev& G, int n, const double* m, const double* pos, int lapse_kind,
                           double* y, hipStream_t s) {
  if (n < 0 || n > MAX_PUNCT) return -1;
  Punctures P{};
  P.n = n;
  P.lapse_kind = lapse_kind;
  for (int i = 0; i < n; i++) {
    P.m[i] = m[i];
    for (int d = 0; d < 3; d++) P.x[i][d] = pos[3 * i + d];
  }
  hipLaunchKernelGGL(k_brill_lindquist, dim3((G.N0 + 63) / 64, G.N1, G.N2), dim3(64), 0, s, G, P, y);
  return 0;
}

}  // namespace bhah
