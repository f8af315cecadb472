// rhs.hip -- BSSN + gauge right-hand sides (Eqs. 7-15 with Eq. 12 of
// arXiv:2505.00097), the fused RK4 stage update, and the Hamiltonian
// constraint (Eq. 16), one thread per interior point.
//
// The right-hand side is split over two kernels to bound register use:
//   k_ricci : everything that needs second derivatives of h_ij -- the
//             conformal Ricci tensor (Eq. 12, rescaled by 1/(S_i S_j)) and
//             Q_k = (d_k Gammabar^j_jm) beta^m -- written to `aux`;
//   k_main  : the remaining terms of Eqs. 7-15, reading aux at the point.
// k_main optionally ends with an RK4 stage combination instead of storing the
// right-hand side (see StageArgs).
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
template <int C>
__device__ __forceinline__ void ricci_point(const GridDev& G, const double* __restrict__ y,
                                            double* __restrict__ aux, int i0, int i1, int i2,
                                            unsigned q) {
  Pt P{y, G.sgf, G.s1, G.s2, q};
  const Spacing sp = make_spacing(G);
  Ref R;
  load_ref<C>(G, i0, i1, i2, R);
  double Gh[3][3][3];
  ref_christoffel(R, Gh);
  Metric M;
  metric_first(P, R, Gh, sp, M);
  double Rc[6], Q[3];
  ricci_and_Q<C>(P, R, Gh, sp, M, Rc, Q, true);
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = i; j < 3; j++) aux[sy(i, j) * G.sgf + q] = Rc[sy(i, j)] * (R.iS[i] * R.iS[j]);
#pragma unroll
  for (int k = 0; k < 3; k++) aux[(6 + k) * G.sgf + q] = Q[k];
}

template <int C>
__global__ void __launch_bounds__(64) k_ricci(GridDev G, const double* __restrict__ y,
                                              double* __restrict__ aux) {
  const PointIdx p = point_of(G);
  if (!p.valid) return;
  ricci_point<C>(G, y, aux, p.i0, p.i1, p.i2, p.q);
}

// ---------------------------------------------------------------------------
// Upwinded advection beta^k d_k f of a rescaled gridfunction (Sec. 3: shift
// advection terms use the stencil shifted one point upwind). With
// sigma = sign(vet^k) and f(m) = f at offset m*sigma along k:
//   beta^k U_k f = |beta^k|/(12 dxx^k) [3 (f(1) - f(-1)) + 10 (f(1) - f(0))
//                                       - 6 (f(2) - f(1)) + (f(3) - f(1))].
struct Upwind {
  unsigned ip[3], im[3], i2[3], i3[3];  // per-lane point indices q+s, q-s, q+2s, q+3s
  double w[3];                          // |beta^k| / (12 dxx^k)
};

__device__ __forceinline__ double advect(const Pt& P, int g, const Upwind& U) {
  const double* f = P.y + g * P.sgf;
  const double f0 = f[P.q];
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    const double fp = f[U.ip[k]], fm = f[U.im[k]], f2 = f[U.i2[k]], f3 = f[U.i3[k]];
    const double u = 3.0 * (fp - fm) + 10.0 * (fp - f0) - 6.0 * (f2 - fp) + (f3 - fp);
    s += U.w[k] * u;
  }
  return s;
}

template <int C>
__device__ __forceinline__ void main_point(const GridDev& G, double eta,
                                           const double* __restrict__ y,
                                           const double* __restrict__ aux, const StageArgs& st,
                                           int i0, int i1, int i2, unsigned q) {
  Pt P{y, G.sgf, G.s1, G.s2, q};
  const Spacing sp = make_spacing(G);
  Ref R;
  load_ref<C>(G, i0, i1, i2, R);
  double Gh[3][3][3];
  ref_christoffel(R, Gh);
  Metric M;
  metric_first(P, R, Gh, sp, M);

  // ---- shift, its derivatives, upwind stencil offsets --------------------
  double vet[3], beta[3], dbeta[3][3], diS[3][3];  // dbeta[i][j] = d_j beta^i, diS[i][k] = d_k (1/S_i)
#pragma unroll
  for (int i = 0; i < 3; i++) {
    vet[i] = P.at(G_VETU0 + i, 0, 0, 0);
    beta[i] = vet[i] * R.iS[i];
#pragma unroll
    for (int k = 0; k < 3; k++) diS[i][k] = -R.dS[i][k] * (R.iS[i] * R.iS[i]);
#pragma unroll
    for (int j = 0; j < 3; j++) dbeta[i][j] = fd1k(P, G_VETU0 + i, j, sp) * R.iS[i] + vet[i] * diS[i][j];
  }
  Upwind U;
  {
    const int str[3] = {1, G.s1, G.s2};
#pragma unroll
    for (int k = 0; k < 3; k++) {
      const int o = vet[k] > 0.0 ? str[k] : -str[k];
      U.ip[k] = q + o; U.im[k] = q - o; U.i2[k] = q + 2 * o; U.i3[k] = q + 3 * o;
      U.w[k] = fabs(beta[k]) * sp.i12h[k];
    }
  }
  // beta^k d_k of the rescaling factors, divided by the factor:
  //   bS[i] = beta^k d_k S_i / S_i
  double bS[3];
#pragma unroll
  for (int i = 0; i < 3; i++) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 3; k++) s += beta[k] * R.dS[i][k];
    bS[i] = s * R.iS[i];
  }

  // ---- scalars: W, alpha, K ---------------------------------------------
  const double W = P.at(G_CF, 0, 0, 0), alpha = P.at(G_ALPHA, 0, 0, 0), K = P.at(G_TRK, 0, 0, 0);
  const double iW = 1.0 / W;
  double dW[3], dalpha[3], dK[3], phi_d[3];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    dW[k] = fd1k(P, G_CF, k, sp);
    dalpha[k] = fd1k(P, G_ALPHA, k, sp);
    dK[k] = fd1k(P, G_TRK, k, sp);
    phi_d[k] = -0.5 * dW[k] * iW;
  }
  // Gammabar = Gammahat + Delta; D_i D_j alpha, D_i D_j phi (Sec. 2.1)
  double DDalpha[6], DDphi[6];
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = i; j < 3; j++) {
      const int a = sy(i, j);
      const double ddW = fd2kl(P, G_CF, i, j, sp);
      const double dda = fd2kl(P, G_ALPHA, i, j, sp);
      const double phi_dd = -0.5 * ddW * iW + 0.5 * dW[i] * dW[j] * (iW * iW);
      double sa = dda, sp_ = phi_dd;
#pragma unroll
      for (int k = 0; k < 3; k++) {
        const double Gb = Gh[k][i][j] + M.DUDD[k][a];
        sa -= Gb * dalpha[k];
        sp_ -= Gb * phi_d[k];
      }
      DDalpha[a] = sa;
      DDphi[a] = sp_;
    }
  // Dbar_k beta^k = d_k beta^k + Gammabar^k_km beta^m
  double Gbc[3];  // Gammabar^k_km
#pragma unroll
  for (int m = 0; m < 3; m++) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 3; k++) s += Gh[k][k][m] + M.DUDD[k][sy(k, m)];
    Gbc[m] = s;
  }
  double Dbeta = 0.0;
#pragma unroll
  for (int k = 0; k < 3; k++) Dbeta += dbeta[k][k] + Gbc[k] * beta[k];

  // ---- Abar and its contractions -----------------------------------------
  double a[6], Abar[6], AUD[3][3], AUU[6];
#pragma unroll
  for (int c = 0; c < 6; c++) { a[c] = P.at(G_ADD00 + c, 0, 0, 0); Abar[c] = a[c] * M.SS[c]; }
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
  double trA = 0.0, AA = 0.0;
#pragma unroll
  for (int i = 0; i < 3; i++) {
    trA += AUD[i][i];
#pragma unroll
    for (int j = 0; j < 3; j++) AA += Abar[sy(i, j)] * AUU[sy(i, j)];
  }
  const double W2 = W * W;  // exp(-4 phi)

  double out[NGF];

  // ---- Eq. 9 (W) and Eq. 10 (K), Eq. 13 (alpha) --------------------------
  out[G_CF] = -(1.0 / 3.0) * W * (Dbeta - alpha * K) + advect(P, G_CF, U);
  {
    double lap = 0.0, da_dphi = 0.0;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = 0; j < 3; j++) {
        lap += M.gbU[sy(i, j)] * DDalpha[sy(i, j)];
        da_dphi += M.gbU[sy(i, j)] * dalpha[i] * phi_d[j];
      }
    out[G_TRK] = (1.0 / 3.0) * alpha * K * K + alpha * AA - W2 * (lap + 2.0 * da_dphi) + advect(P, G_TRK, U);
  }
  out[G_ALPHA] = -2.0 * alpha * K + advect(P, G_ALPHA, U);

  // ---- Eq. 7: eps ----------------------------------------------------------
  // Dhat_j beta^i and the Lie-derivative pieces
  double Dbeta_hat[3][3];  // [i][j] = Dhat_j beta^i
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) {
      double s = dbeta[i][j];
#pragma unroll
      for (int m = 0; m < 3; m++) s += Gh[i][j][m] * beta[m];
      Dbeta_hat[i][j] = s;
    }
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = i; j < 3; j++) {
      const int c = sy(i, j);
      double r = (2.0 / 3.0) * M.gb[c] * (alpha * trA - Dbeta) +
                 R.S[j] * R.S[j] * Dbeta_hat[j][i] + R.S[i] * R.S[i] * Dbeta_hat[i][j] -
                 2.0 * alpha * Abar[c];
#pragma unroll
      for (int k = 0; k < 3; k++) r += M.eps[sy(k, j)] * dbeta[k][i] + M.eps[sy(i, k)] * dbeta[k][j];
      out[G_HDD00 + c] = r * (R.iS[i] * R.iS[j]) + advect(P, G_HDD00 + c, U) + M.h[c] * (bS[i] + bS[j]);
    }

  // ---- Eq. 8: Abar ---------------------------------------------------------
  {
    double X[6], trX = 0.0;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = i; j < 3; j++) {
        const int c = sy(i, j);
        const double Rc = aux[c * G.sgf + q] * M.SS[c];
        X[c] = -2.0 * alpha * DDphi[c] + 4.0 * alpha * phi_d[i] * phi_d[j] +
               2.0 * (dalpha[i] * phi_d[j] + dalpha[j] * phi_d[i]) - DDalpha[c] + alpha * Rc;
      }
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = 0; j < 3; j++) trX += M.gbU[sy(i, j)] * X[sy(i, j)];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = i; j < 3; j++) {
        const int c = sy(i, j);
        double AikAkj = 0.0;
#pragma unroll
        for (int k = 0; k < 3; k++) AikAkj += Abar[sy(i, k)] * AUD[k][j];
        double r = -(2.0 / 3.0) * Abar[c] * Dbeta - 2.0 * alpha * AikAkj + alpha * Abar[c] * K +
                   W2 * (X[c] - (1.0 / 3.0) * M.gb[c] * trX);
#pragma unroll
        for (int k = 0; k < 3; k++) r += Abar[sy(k, j)] * dbeta[k][i] + Abar[sy(i, k)] * dbeta[k][j];
        out[G_ADD00 + c] = r * (R.iS[i] * R.iS[j]) + advect(P, G_ADD00 + c, U) + a[c] * (bS[i] + bS[j]);
      }
  }

  // ---- Eq. 11: Lambdabar (lapse factors restored in the Abar terms) ------
  {
    double dGh[3][3][3][3];
    ref_christoffel_deriv(R, dGh);
    double Lam[3];
#pragma unroll
    for (int i = 0; i < 3; i++) Lam[i] = P.at(G_LAMU0 + i, 0, 0, 0) * R.iS[i];
    // d_j d_k beta^i
    double ddbeta[3][6];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = 0; j < 3; j++)
#pragma unroll
        for (int k = j; k < 3; k++) {
          const double v = vet[i];
          const double ddiS = -R.ddS[i][j][k] * (R.iS[i] * R.iS[i]) +
                              2.0 * R.dS[i][j] * R.dS[i][k] * (R.iS[i] * R.iS[i] * R.iS[i]);
          ddbeta[i][sy(j, k)] = fd2kl(P, G_VETU0 + i, j, k, sp) * R.iS[i] +
                                fd1k(P, G_VETU0 + i, j, sp) * diS[i][k] +
                                fd1k(P, G_VETU0 + i, k, sp) * diS[i][j] + v * ddiS;
        }
    double dDbeta[3];  // d_k (Dbar_j beta^j) = d_k d_j beta^j + Q_k + Gammabar^j_jm d_k beta^m
#pragma unroll
    for (int k = 0; k < 3; k++) {
      double s = aux[(6 + k) * G.sgf + q];
#pragma unroll
      for (int j = 0; j < 3; j++) s += ddbeta[j][sy(j, k)];
#pragma unroll
      for (int m = 0; m < 3; m++) s += Gbc[m] * dbeta[m][k];
      dDbeta[k] = s;
    }
    double rl[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
      // gammabar^jk Dhat_j Dhat_k beta^i
      double t2 = 0.0;
#pragma unroll
      for (int j = 0; j < 3; j++)
#pragma unroll
        for (int k = 0; k < 3; k++) {
          double s = ddbeta[i][sy(j, k)];
#pragma unroll
          for (int m = 0; m < 3; m++)
            s += dGh[i][k][m][j] * beta[m] + Gh[i][k][m] * dbeta[m][j] + Gh[i][j][m] * Dbeta_hat[m][k] -
                 Gh[m][j][k] * Dbeta_hat[i][m];
          t2 += M.gbU[sy(j, k)] * s;
        }
      double t4 = 0.0, t5 = 0.0, t6 = 0.0, t7 = 0.0, lie = 0.0;
#pragma unroll
      for (int j = 0; j < 3; j++) {
        t4 += M.gbU[sy(i, j)] * dDbeta[j];
        t5 += AUU[sy(i, j)] * (dalpha[j] - 6.0 * alpha * phi_d[j]);
        t7 += M.gbU[sy(i, j)] * dK[j];
        lie -= Lam[j] * dbeta[i][j];
#pragma unroll
        for (int k = 0; k < 3; k++) t6 += AUU[sy(j, k)] * M.DUDD[i][sy(j, k)];
      }
      const double r = t2 + (2.0 / 3.0) * M.DU[i] * Dbeta + (1.0 / 3.0) * t4 - 2.0 * t5 +
                       2.0 * alpha * t6 - (4.0 / 3.0) * alpha * t7 + lie;
      const double lam = P.at(G_LAMU0 + i, 0, 0, 0);
      rl[i] = r * R.S[i] + advect(P, G_LAMU0 + i, U) - lam * bS[i];
      out[G_LAMU0 + i] = rl[i];
    }
    // ---- Eqs. 14-15: shift and B (d_t Lambdabar is the full value above) -
#pragma unroll
    for (int i = 0; i < 3; i++) {
      const double bet = P.at(G_BETU0 + i, 0, 0, 0);
      out[G_VETU0 + i] = bet + advect(P, G_VETU0 + i, U) - vet[i] * bS[i];
      out[G_BETU0 + i] = 0.75 * rl[i] - eta * bet + advect(P, G_BETU0 + i, U) - bet * bS[i];
    }
  }

  // ---- store / RK stage combination ----------------------------------------
  if (st.rhs) {
#pragma unroll
    for (int g = 0; g < NGF; g++) st.rhs[g * G.sgf + q] = out[g];
  } else {
#pragma unroll
    for (int g = 0; g < NGF; g++) {
      const long long e = g * G.sgf + q;
      st.out1[e] = st.base1[e] + st.c1 * out[g];
      if (st.out2) st.out2[e] = st.base2[e] + st.c2 * out[g];
    }
  }
}

template <int C>
__global__ void __launch_bounds__(64) k_main(GridDev G, double eta, const double* __restrict__ y,
                                             const double* __restrict__ aux, StageArgs st) {
  const PointIdx p = point_of(G);
  if (!p.valid) return;
  main_point<C>(G, eta, y, aux, st, p.i0, p.i1, p.i2, p.q);
}

// ---------------------------------------------------------------------------
// Hamiltonian constraint, Eq. 16:
// H = 2/3 K^2 - Abar_ij Abar^ij + W^2 (Rbar - 8 Dbar^i phi Dbar_i phi - 8 Dbar^2 phi)
template <int C>
__global__ void __launch_bounds__(64) k_hamiltonian(GridDev G, const double* __restrict__ y,
                                                   double* __restrict__ H) {
  const PointIdx p = point_of(G);
  if (!p.valid) return;
  Pt P{y, G.sgf, G.s1, G.s2, p.q};
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

template <int C>
static void launch_rhs_t(const GridDev& G, double eta, const double* y, double* aux,
                         const StageArgs& st, hipStream_t s) {
  const dim3 g = grid_of(G, 64);
  hipLaunchKernelGGL(k_ricci<C>, g, dim3(64), 0, s, G, y, aux);
  hipLaunchKernelGGL(k_main<C>, g, dim3(64), 0, s, G, eta, y, aux, st);
}

void launch_rhs(const GridDev& G, double eta, const double* y, double* aux, const StageArgs& st,
                hipStream_t s) {
  switch (G.coord) {
    case BHAH_SINH_SPHERICAL: launch_rhs_t<BHAH_SINH_SPHERICAL>(G, eta, y, aux, st, s); break;
    case BHAH_SINH_CYLINDRICAL: launch_rhs_t<BHAH_SINH_CYLINDRICAL>(G, eta, y, aux, st, s); break;
    default: launch_rhs_t<BHAH_SPHERICAL>(G, eta, y, aux, st, s); break;
  }
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
