// hamiltonian.hip -- the constraints: Hamiltonian (Eq. 16 of arXiv:2505.00097),
// momentum (Eq. 17) and C^i, one thread per interior point, centred
// differences of the grid's order (4th with 3 ghost layers, 8th with 5).
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
  p.i0 = G.ng + (int)(blockIdx.x * blockDim.x + threadIdx.x);
  p.i1 = G.ng + (int)blockIdx.y;
  p.i2 = G.ng + (int)blockIdx.z;
  p.valid = p.i0 < G.ng + G.N0;
  p.q = (unsigned)(p.i0 + G.s1 * p.i1 + G.s2 * p.i2);
  return p;
}

// ---------------------------------------------------------------------------
// Constraints at one interior point:
//   H   = 2/3 K^2 - Abar_ij Abar^ij + W^2 (Rbar - 8 Dbar^i phi Dbar_i phi - 8 Dbar^2 phi)   (Eq. 16)
//   M^i = W^2 (Dhat_j Abar^ij + 2 Abar^k(i Delta^j)_jk + 6 Abar^ij d_j phi
//              - 2/3 gammabar^ij d_j K)                                              (Eq. 17)
//   C^i = Lambdabar^i - Delta^i
// with phi = -ln(W)/2 (W^2 = e^{-4 phi}); M^i and C^i are returned rescaled
// like lambda^i (times S_i). Any of H, Mo, Co may be null.
template <int C, int NH>
__device__ __forceinline__ void constraints_point(const GridDev& G, const double* __restrict__ y,
                                                  const PointIdx& p, double* __restrict__ H,
                                                  double* __restrict__ Mo, double* __restrict__ Co) {
  const PtT<NH> P(y, G, C, p.i0, p.i1, p.i2);
  const Spacing sp = make_spacing<NH - 1>(G);
  Ref R;
  load_ref<C>(G, p.i0, p.i1, p.i2, R);
  double Gh[3][3][3];
  ref_christoffel(R, Gh);
  Metric M;
  metric_first(P, R, Gh, sp, M);
  const double W = P.at(G_CF, 0, 0, 0), K = P.at(G_TRK, 0, 0, 0);
  const double iW = 1.0 / W;
  double dW[3], phi_d[3];
#pragma unroll
  for (int k = 0; k < 3; k++) { dW[k] = fd1k(P, G_CF, k, sp); phi_d[k] = -0.5 * dW[k] * iW; }
  double Abar[6], AUD[3][3], AUU[6];
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
    for (int j = i; j < 3; j++) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 3; k++) s += AUD[i][k] * M.gbU[sy(k, j)];
      AUU[sy(i, j)] = s;
    }
  if (H) {
    double Rc[6], Q[3];
    ricci_and_Q<C>(P, R, Gh, sp, M, Rc, Q, false);
    double Rtr = 0.0, dphi2 = 0.0, lap = 0.0, AA = 0.0;
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
        AA += AUD[i][j] * AUD[j][i];
      }
    H[p.q] = (2.0 / 3.0) * K * K - AA + W * W * (Rtr - 8.0 * dphi2 - 8.0 * lap);
  }
  if (Mo) {
    // d_k gammabar_ab = d_k eps_ab + d_k gammahat_ab, gammahat = diag(S^2)
    double dgb[6][3];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
      for (int b = a; b < 3; b++)
#pragma unroll
        for (int k = 0; k < 3; k++)
          dgb[sy(a, b)][k] = M.deps[sy(a, b)][k] + (a == b ? 2.0 * R.S[a] * R.dS[a][k] : 0.0);
    // d_k Abar_ab from the rescaled a_ab
    double dAbar[6][3];
#pragma unroll
    for (int c = 0; c < 6; c++)
#pragma unroll
      for (int k = 0; k < 3; k++)
        dAbar[c][k] = fd1k(P, G_ADD00 + c, k, sp) * M.SS[c] + P.at(G_ADD00 + c, 0, 0, 0) * M.dSS[c][k];
    double dK[3];
#pragma unroll
    for (int k = 0; k < 3; k++) dK[k] = fd1k(P, G_TRK, k, sp);
    // d_k Abar^ij = d_k (gammabar^ia gammabar^jb Abar_ab), with
    // d_k gammabar^ij = -gammabar^ia d_k gammabar_ab gammabar^bj
#pragma unroll
    for (int i = 0; i < 3; i++) {
      double div = 0.0;
#pragma unroll
      for (int j = 0; j < 3; j++) {
        const int k = j;  // the divergence contracts the derivative index with j
        double dAUU = 0.0;
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
          for (int b = 0; b < 3; b++) {
            double dgUia = 0.0, dgUjb = 0.0;
#pragma unroll
            for (int c = 0; c < 3; c++)
#pragma unroll
              for (int d = 0; d < 3; d++) {
                dgUia -= M.gbU[sy(i, c)] * dgb[sy(c, d)][k] * M.gbU[sy(d, a)];
                dgUjb -= M.gbU[sy(j, c)] * dgb[sy(c, d)][k] * M.gbU[sy(d, b)];
              }
            dAUU += dgUia * M.gbU[sy(j, b)] * Abar[sy(a, b)] + M.gbU[sy(i, a)] * dgUjb * Abar[sy(a, b)] +
                    M.gbU[sy(i, a)] * M.gbU[sy(j, b)] * dAbar[sy(a, b)][k];
          }
        div += dAUU;
#pragma unroll
        for (int m = 0; m < 3; m++) div += Gh[i][j][m] * AUU[sy(m, j)] + Gh[j][j][m] * AUU[sy(i, m)];
      }
      double sym = 0.0, t6 = 0.0, tK = 0.0;
#pragma unroll
      for (int j = 0; j < 3; j++) {
#pragma unroll
        for (int k = 0; k < 3; k++) sym += AUU[sy(k, i)] * M.DUDD[j][sy(j, k)] + AUU[sy(k, j)] * M.DUDD[i][sy(j, k)];
        t6 += 6.0 * AUU[sy(i, j)] * phi_d[j];
        tK += -(2.0 / 3.0) * M.gbU[sy(i, j)] * dK[j];
      }
      Mo[i * G.sgf + p.q] = W * W * (div + sym + t6 + tK) * R.S[i];
    }
  }
  if (Co) {
#pragma unroll
    for (int i = 0; i < 3; i++) Co[i * G.sgf + p.q] = P.at(G_LAMU0 + i, 0, 0, 0) - M.DU[i] * R.S[i];
  }
}

template <int C, int NH>
__global__ void __launch_bounds__(64) k_hamiltonian(GridDev G, const double* __restrict__ y,
                                                   double* __restrict__ H) {
  const PointIdx p = point_of(G);
  if (p.valid) constraints_point<C, NH>(G, y, p, H, nullptr, nullptr);
}

template <int C, int NH>
__global__ void __launch_bounds__(64) k_constraints(GridDev G, const double* __restrict__ y, double* __restrict__ H,
                                                   double* __restrict__ Mo, double* __restrict__ Co) {
  const PointIdx p = point_of(G);
  if (p.valid) constraints_point<C, NH>(G, y, p, H, Mo, Co);
}

// ---- launchers -------------------------------------------------------------
static dim3 grid_of(const GridDev& G, int bx) {
  return dim3((G.N0 + bx - 1) / bx, G.N1, G.N2);
}

template <int NH>
static void launch_constraints_t(const GridDev& G, const double* y, double* H, double* Mo, double* Co,
                                 hipStream_t s) {
  const dim3 g = grid_of(G, 64);
  const bool only_H = Mo == nullptr && Co == nullptr;
  switch (G.coord) {
    case BHAH_SINH_SPHERICAL:
      if (only_H) hipLaunchKernelGGL((k_hamiltonian<BHAH_SINH_SPHERICAL, NH>), g, dim3(64), 0, s, G, y, H);
      else hipLaunchKernelGGL((k_constraints<BHAH_SINH_SPHERICAL, NH>), g, dim3(64), 0, s, G, y, H, Mo, Co);
      break;
    case BHAH_SINH_CYLINDRICAL:
      if (only_H) hipLaunchKernelGGL((k_hamiltonian<BHAH_SINH_CYLINDRICAL, NH>), g, dim3(64), 0, s, G, y, H);
      else hipLaunchKernelGGL((k_constraints<BHAH_SINH_CYLINDRICAL, NH>), g, dim3(64), 0, s, G, y, H, Mo, Co);
      break;
    default:
      if (only_H) hipLaunchKernelGGL((k_hamiltonian<BHAH_SPHERICAL, NH>), g, dim3(64), 0, s, G, y, H);
      else hipLaunchKernelGGL((k_constraints<BHAH_SPHERICAL, NH>), g, dim3(64), 0, s, G, y, H, Mo, Co);
      break;
  }
}

void launch_hamiltonian(const GridDev& G, const double* y, double* H, hipStream_t s) {
  if (G.ng == 5) launch_constraints_t<5>(G, y, H, nullptr, nullptr, s);
  else launch_constraints_t<3>(G, y, H, nullptr, nullptr, s);
}

void launch_constraints(const GridDev& G, const double* y, double* H, double* Mo, double* Co, hipStream_t s) {
  if (G.ng == 5) launch_constraints_t<5>(G, y, H, Mo, Co, s);
  else launch_constraints_t<3>(G, y, H, Mo, Co, s);
}

}  // namespace bhah
