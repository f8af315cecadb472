// hamiltonian.hip -- the Hamiltonian constraint (Eq. 16 of arXiv:2505.00097),
// one thread per interior point, centred 4th-order differences.
#include "rhs_common.h"

namespace bhah {

// Thread -> interior point: blockIdx.y/z walk i1/i2, x covers i0.
struct PointIdx {
  int i0, i1, i2;
  unsigned q;
  bool valid;
};

__device__ __forceinline__ PointIdx point_of(const GridDev& G) {
  PointIdx p;
  p.i0 = NG + (int)(blockIdx.x * blockDim.x + threadIdx.x);
  p.i1 = NG + (int)blockIdx.y;
  p.i2 = NG + (int)blockIdx.z;
  p.valid = p.i0 < NG + G.N0;
  p.q = (unsigned)(p.i0 + G.s1 * p.i1 + G.s2 * p.i2);
  return p;
}

// ---------------------------------------------------------------------------
// Hamiltonian constraint, Eq. 16:
// H = 2/3 K^2 - Abar_ij Abar^ij + W^2 (Rbar - 8 Dbar^i phi Dbar_i phi - 8 Dbar^2 phi)
template <int C>
__global__ void __launch_bounds__(64) k_hamiltonian(GridDev G, const double* __restrict__ y,
                                                   double* __restrict__ H) {
  const PointIdx p = point_of(G);
  if (!p.valid) return;
  const Pt P(y, G, C, p.i0, p.i1, p.i2);
  const Spacing sp = make_spacing(G);
  Ref R;
  load_ref<C>(G, p.i0, p.i1, p.i2, R);
  double Gh[3][3][3];
  ref_christoffel(R, Gh);
  Metric M;
  metric_first(P, R, Gh, sp, M);
  double Rc[6], Q[3];
  ricci_and_Q<C>(P, R, Gh, sp, M, Rc, Q, false);
  const double W = P.at(G_CF, 0, 0, 0), K = P.at(G_TRK, 0, 0, 0);
  const double iW = 1.0 / W;
  double dW[3], phi_d[3];
#pragma unroll
  for (int k = 0; k < 3; k++) { dW[k] = fd1k(P, G_CF, k, sp); phi_d[k] = -0.5 * dW[k] * iW; }
  double Rtr = 0.0, dphi2 = 0.0, lap = 0.0;
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) {
      const int c = sy(i, j);
      const double phi_dd = -0.5 * fd2kl(P, G_CF, i, j, sp) * iW + 0.5 * dW[i] * dW[j] * (iW * iW);
      double Dd = phi_dd;
#pragma unroll
      for (int k = 0; k < 3; k++) Dd -= (Gh[k][i][j] + M.DUDD[k][c]) * phi_d[k];
      Rtr += M.gbU[c] * Rc[c];
      dphi2 += M.gbU[c] * phi_d[i] * phi_d[j];
      lap += M.gbU[c] * Dd;
    }
  double Abar[6], AUD[3][3], AA = 0.0;
#pragma unroll
  for (int c = 0; c < 6; c++) Abar[c] = P.at(G_ADD00 + c, 0, 0, 0) * M.SS[c];
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 3; k++) s += M.gbU[sy(i, k)] * Abar[sy(k, j)];
      AUD[i][j] = s;
    }
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) AA += AUD[i][j] * AUD[j][i];
  H[p.q] = (2.0 / 3.0) * K * K - AA + W * W * (Rtr - 8.0 * dphi2 - 8.0 * lap);
}

// ---- launchers -------------------------------------------------------------
static dim3 grid_of(const GridDev& G, int bx) {
  return dim3((G.N0 + bx - 1) / bx, G.N1, G.N2);
}

void launch_hamiltonian(const GridDev& G, const double* y, double* H, hipStream_t s) {
  const dim3 g = grid_of(G, 64);
  switch (G.coord) {
    case BHAH_SINH_SPHERICAL: hipLaunchKernelGGL(k_hamiltonian<BHAH_SINH_SPHERICAL>, g, dim3(64), 0, s, G, y, H); break;
    case BHAH_SINH_CYLINDRICAL: hipLaunchKernelGGL(k_hamiltonian<BHAH_SINH_CYLINDRICAL>, g, dim3(64), 0, s, G, y, H); break;
    default: hipLaunchKernelGGL(k_hamiltonian<BHAH_SPHERICAL>, g, dim3(64), 0, s, G, y, H); break;
  }
}

}  // namespace bhah
