// rhs_pair.hip -- the BSSN + gauge right-hand side of one 64-point tile split
// over two cooperating waves of one block (Eqs. 7-15 with the conformal Ricci
// tensor of Eq. 12, arXiv:2505.00097), with the RK stage combination as
// epilogue: the two-waves-per-tile mode of the right-hand side.
//
// Lane l of both waves holds the same point; each wave does about half of
// the point's work and keeps about half of its live values. The kernel is
// built for one wave per SIMD, so the two waves of a tile run on two SIMDs
// side by side and a tile takes about as long as its longer half. Where a
// grid has at most half as many tiles as the device has SIMDs (the tiny and
// the paper's desktop grids), every tile gets its two SIMDs and a step is
// shorter than with one wave per tile; where it has more, two-wave tiles
// wait for SIMDs and the one-wave kernel is as fast or faster. The solo
// tuner picks the mode by timing.
//   metric wave (0): the stencils of h_ij (second derivatives contracted
//     into gammabar^kl d_k d_l h_ij and the beta-weighted trace of Q_k,
//     first derivatives, advection), the reference-metric and Delta terms of
//     the Ricci tensor, Q_k, then (after the first barrier) the
//     Lambdabar terms of the Ricci tensor and Eq. 7; it stores the six
//     h_ij results.
//   gauge wave (1): the stencils of W, alpha and vet^i (the second-
//     derivative contractions of the Abar, K and Lambdabar equations), of
//     lambda^i, the advection of Abar_ij, B^i and K; after the first barrier
//     Eqs. 9, 10, 11, 13, 14, 15, after the second Eq. 8; it stores the
//     other 18 results.
// The exchange runs through per-point LDS slots (slot v of lane l at
// xs[v * 64 + l]):
//   metric -> gauge before barrier 1: Delta^k_ij, Delta^k, Q_k
//   gauge -> metric before barrier 1: d_k vet^i, d_k lambda^i
//   metric -> gauge before barrier 2: the rescaled Ricci tensor
// Values the gauge wave still needs after barrier 2 are copied out of the
// exchange slots before it.
#include "rhs_stencil.h"

namespace bhah {

enum {
  XS_DUDD = 0,   // 18  Delta^k_ij at [3 * ... ] k-major: XS_DUDD + 6 k + sy(i, j)
  XS_DU = 18,    // 3   Delta^k
  XS_Q = 21,     // 3   Q_k
  XS_DVET = 24,  // 9   d_k vet^i at XS_DVET + 3 i + k
  XS_DLAM = 33,  // 9   d_k lambda^i at XS_DLAM + 3 i + k (read by the metric wave before it writes XS_RT)
  XS_RT = 33,    // 6   rescaled Ricci tensor (after barrier 1)
  XS_DH = 42,    // 18  metric wave's park: d_k h_ij at XS_DH + 3 sy(i, j) + k
  XS_GOUT = 60,  // 18  gauge wave's park of its results (gridfunctions 0..10, 17..23)
  XSLOTS = 78    // 78 x 64 lanes x 8 B = 39 KB per block; two blocks (four waves) per CU
};

// the gauge wave's result slot of gridfunction g (not one of h_ij)
__device__ __forceinline__ constexpr int gslot(int g) { return XS_GOUT + (g < G_HDD00 ? g : g - 6); }

__device__ __forceinline__ void pair_barrier() { __syncthreads(); }

// RK stage epilogue for the gridfunctions in [g0, g1) (skipping h_ij when
// skip_h) with results res(g): every base value is read before any store.
template <bool MIX, class RES>
__device__ __forceinline__ void stage_store(const GridDev& G, const StageArgs& st, unsigned q, int g0, int g1,
                                            bool skip_h, const RES& res) {
  auto take = [&](int g) { return !(skip_h && g >= G_HDD00 && g < G_HDD00 + 6); };
  if (st.rhs) {
#pragma unroll
    for (int g = g0; g < g1; g++)
      if (take(g)) st.rhs[g * G.sgf + q] = res(g);
    return;
  }
  const bool two = st.out2 != nullptr, mix = MIX && !two && st.base2 != nullptr, same = st.base2 == st.base1;
  double b1[NGF], b2[NGF];
#pragma unroll
  for (int g = g0; g < g1; g++)
    if (take(g)) b1[g] = gf_ld(st.base1, G.sgf, g, q * 8u, 0);
  if ((two || mix) && !same) {
#pragma unroll
    for (int g = g0; g < g1; g++)
      if (take(g)) b2[g] = gf_ld(st.base2, G.sgf, g, q * 8u, 0);
  } else {
#pragma unroll
    for (int g = g0; g < g1; g++)
      if (take(g)) b2[g] = b1[g];
  }
  BHAH_PHASE_BARRIER();
  if (mix) {
#pragma unroll
    for (int g = g0; g < g1; g++)
      if (take(g)) st.out1[g * G.sgf + q] = st.m1 * b1[g] + st.m2 * b2[g] + st.c1 * res(g);
  } else {
#pragma unroll
    for (int g = g0; g < g1; g++)
      if (take(g)) {
        const long long e = g * G.sgf + q;
        const double k = res(g);
        st.out1[e] = b1[g] + st.c1 * k;
        if (two) st.out2[e] = b2[g] + st.c2 * k;
      }
  }
}

// ---- metric wave -----------------------------------------------------------
template <int C, bool AX, bool KO, bool MIX, int H>
__device__ __forceinline__ void metric_wave(const GridDev& G, const Gauge& ga, const double* __restrict__ y,
                                            const StageArgs& st, int i0, int i1, int i2, unsigned q, bool valid,
                                            double* __restrict__ aux, double* __restrict__ xs) {
  constexpr int PD = C == BHAH_SINH_CYLINDRICAL ? 1 : 2;
  constexpr int RR = H - 1, SW = 2 * RR + 1;
  double kw[3];
#pragma unroll
  for (int k = 0; k < 3; k++) kw[k] = G.inv_dx[k] * (1.0 / FdW<RR>::kden);
  auto put = [&](int v, double x) { xs[v * 64] = x; };
  auto get = [&](int v) { return xs[v * 64]; };
  const PtT<H> P(y, G, C, i0, i1, i2);
  const Spacing sp = make_spacing<RR>(G);
  Ref R;
  load_ref<C>(G, i0, i1, i2, R);

  // ---- point values, the conformal metric and its inverse (Eq. 3) --------
  double h[6], SS[6], gb[6], gbU[6];
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = i; j < 3; j++) {
      const int a = sy(i, j);
      SS[a] = R.S[i] * R.S[j];
      h[a] = P.at(G_HDD00 + a, 0, 0, 0);
      gb[a] = (i == j ? R.S[i] * R.S[i] : 0.0) + h[a] * SS[a];
    }
  sym_inverse(gb, gbU);
  double vet[3], beta[3];
#pragma unroll
  for (int i = 0; i < 3; i++) {
    vet[i] = P.at(G_VETU0 + i, 0, 0, 0);
    beta[i] = vet[i] * R.iS[i];
  }
  UpwindT<H> U;
  U.v0 = q * 8u;
  {
    const int str[3] = {1, G.s1, G.s2};
#pragma unroll
    for (int k = 0; k < 3; k++) {
      const int s = vet[k] > 0.0 ? 1 : -1;
      if (k == P.pd) {
        const bool up = s > 0;
        U.vu[k][0] = up ? P.vper(1) : P.vper(-1);
        U.vd[k][0] = up ? P.vper(-1) : P.vper(1);
#pragma unroll
        for (int m = 2; m <= H; m++) U.vu[k][m - 1] = up ? P.vper(m) : P.vper(-m);
#pragma unroll
        for (int m = 2; m <= H; m++) U.vd[k][m - 1] = up ? P.vper(-m) : P.vper(m);
      } else {
        const int o = s * str[k];
        U.vu[k][0] = (q + o) * 8u;
        U.vd[k][0] = (q - o) * 8u;
#pragma unroll
        for (int m = 2; m <= H; m++) U.vu[k][m - 1] = (q + m * o) * 8u;
#pragma unroll
        for (int m = 2; m <= H; m++) U.vd[k][m - 1] = (q - m * o) * 8u;
      }
      U.w[k] = fabs(beta[k]) * sp.d1s[k];
    }
  }

  // ---- second derivatives of h_ij, pair (k,l) by pair --------------------
  //   Pc_ij = sum_kl gammabar^kl d_k d_l h_ij                (Ricci)
  //   Qs_k  = sum_m beta^m gammabar^ab S_a S_b d_k d_m h_ab    (Q_k)
  // the diagonal gathers also give d_k h_ij and the advection of h_ij
  double Pc[6], Qs[3], adv[6];
#pragma unroll
  for (int a = 0; a < 6; a++) { Pc[a] = 0.0; adv[a] = 0.0; }
#pragma unroll
  for (int i = 0; i < 3; i++) Qs[i] = 0.0;
  {
    double G2[6];  // gammabar^ab S_a S_b, doubled off the diagonal
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
      for (int b = a; b < 3; b++) G2[sy(a, b)] = (a == b ? 1.0 : 2.0) * gbU[sy(a, b)] * SS[sy(a, b)];
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
      for (int l = k; l < 3; l++) {
        double dd[6];
        if (k == l) {
          constexpr int TB = H == 3 ? 6 : 3;
#pragma unroll
          for (int t0 = 0; t0 < 6; t0 += TB) {
            double v[TB][SW], fu[TB], fd[KO ? TB : 1];
#pragma unroll
            for (int t = 0; t < TB; t++) {
              gather_axis_k<PD, AX>(P, G_HDD00 + t0 + t, k, v[t]);
              fu[t] = upwind_far<PD, AX>(P, G_HDD00 + t0 + t, k, U.vu, v[t]);
              if constexpr (KO) fd[t] = upwind_far<PD, AX>(P, G_HDD00 + t0 + t, k, U.vd, v[t]);
            }
            BHAH_PHASE_BARRIER();
            const bool up = vet[k] > 0.0;
#pragma unroll
            for (int t = 0; t < TB; t++) {
              const int a = t0 + t;
              adv[a] += U.w[k] * upwind_sum<RR>(v[t], fu[t], up);
              if constexpr (KO) adv[a] += ga.dm * kw[k] * ko_v<RR>(v[t], fu[t], fd[t]);
              dd[a] = d2_axis<RR>(v[t], sp.d2s[k]);
              put(XS_DH + 3 * a + k, AX && k == PD ? 0.0 : d1_axis<RR>(v[t], sp.d1s[k]));
            }
          }
        } else if (AX && (k == PD || l == PD)) {
#pragma unroll
          for (int a = 0; a < 6; a++) dd[a] = 0.0;
        } else {
          constexpr int TX = H == 3 ? 3 : 1;
#pragma unroll
          for (int t0 = 0; t0 < 6; t0 += TX) {
            double v[TX][4 * RR * RR];
#pragma unroll
            for (int t = 0; t < TX; t++) gather_cross_kl(P, G_HDD00 + t0 + t, k, l, v[t]);
            BHAH_PHASE_BARRIER();
#pragma unroll
            for (int t = 0; t < TX; t++) dd[t0 + t] = d2_cross<RR>(v[t], sp.crs[k][l]);
          }
        }
        const double wg = (k == l ? 1.0 : 2.0) * gbU[sy(k, l)];
        double c = 0.0;
#pragma unroll
        for (int a = 0; a < 6; a++) {
          Pc[a] += wg * dd[a];
          c += G2[a] * dd[a];
        }
        Qs[k] += beta[l] * c;
        if (k != l) Qs[l] += beta[k] * c;
      }
  }
  BHAH_PHASE_BARRIER();

  // ---- first derivatives of h, eps, Dhat eps ------------------------------
  double Gh[3][3][3];
  ref_christoffel(R, Gh);
  double dh[6][3], eps[6], Dh_eps[6][3];
#pragma unroll
  for (int a = 0; a < 6; a++)
#pragma unroll
    for (int k = 0; k < 3; k++) dh[a][k] = get(XS_DH + 3 * a + k);
#pragma unroll
  for (int a = 0; a < 6; a++) eps[a] = h[a] * SS[a];
  auto deps = [&](int i, int j, int k) {
    const int a = sy(i, j);
    return dh[a][k] * SS[a] + h[a] * (R.dS[i][k] * R.S[j] + R.S[i] * R.dS[j][k]);
  };
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = i; j < 3; j++)
#pragma unroll
      for (int k = 0; k < 3; k++) {
        double s = deps(i, j, k);
#pragma unroll
        for (int m = 0; m < 3; m++) s -= Gh[m][k][i] * eps[sy(m, j)] + Gh[m][k][j] * eps[sy(i, m)];
        Dh_eps[sy(i, j)][k] = s;
      }
  BHAH_PHASE_BARRIER();

  // ---- Ricci (Eq. 12): Dhat Dhat eps below second order; Q_k -------------
  double Rl[6];
#pragma unroll
  for (int a = 0; a < 6; a++) Rl[a] = 0.0;
  {
    double dGh[3][3][3][3];
    ref_christoffel_deriv(R, dGh);
    double cq[6];
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
      for (int l = k; l < 3; l++) {
        const double wkl = (k == l ? -0.5 : -1.0) * gbU[sy(k, l)];
        double cqa = 0.0;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
          for (int j = i; j < 3; j++) {
            const int a = sy(i, j);
            const double ddSS = R.ddS[i][k][l] * R.S[j] + R.dS[i][k] * R.dS[j][l] +
                                R.dS[i][l] * R.dS[j][k] + R.S[i] * R.ddS[j][k][l];
            const double dSSk = R.dS[i][k] * R.S[j] + R.S[i] * R.dS[j][k];
            const double dSSl = R.dS[i][l] * R.S[j] + R.S[i] * R.dS[j][l];
            const double low = dh[a][k] * dSSl + dh[a][l] * dSSk + h[a] * ddSS;
            double s = low;
#pragma unroll
            for (int m = 0; m < 3; m++)
              s -= dGh[m][l][i][k] * eps[sy(m, j)] + Gh[m][l][i] * deps(m, j, k) +
                   dGh[m][l][j][k] * eps[sy(i, m)] + Gh[m][l][j] * deps(i, m, k);
#pragma unroll
            for (int m = 0; m < 3; m++)
              s -= Gh[m][k][l] * Dh_eps[a][m] + Gh[m][k][i] * Dh_eps[sy(m, j)][l] +
                   Gh[m][k][j] * Dh_eps[sy(i, m)][l];
            Rl[a] += wkl * s;
            const double ddgh = i == j ? 2.0 * (R.dS[i][k] * R.dS[i][l] + R.S[i] * R.ddS[i][k][l]) : 0.0;
            cqa += (i == j ? 1.0 : 2.0) * gbU[a] * (ddgh + low);
          }
        cq[sy(k, l)] = cqa;
      }
    // A_k = gammabar^-1 d_k gammabar; Q_k = 1/2 beta^m (Qs + cq - tr(A_k A_m))
    double A[3][3][3];
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
      for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) {
          double s = 0.0;
#pragma unroll
          for (int c = 0; c < 3; c++)
            s += gbU[sy(a, c)] * ((c == b ? 2.0 * R.S[c] * R.dS[c][k] : 0.0) + deps(c, b, k));
          A[k][a][b] = s;
        }
#pragma unroll
    for (int k = 0; k < 3; k++) {
      double s = Qs[k];
#pragma unroll
      for (int m = 0; m < 3; m++) {
        double tr = 0.0;
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
          for (int b = 0; b < 3; b++) tr += A[k][a][b] * A[m][b][a];
        s += beta[m] * (cq[sy(k, m)] - tr);
      }
      put(XS_Q + k, 0.5 * s);
    }
  }
  BHAH_PHASE_BARRIER();

  // ---- Delta^k_ij (Eq. 4), Delta^k (Eq. 5), Delta terms of the Ricci tensor
  double DUDD[3][6], DU[3];
#pragma unroll
  for (int k = 0; k < 3; k++)
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = i; j < 3; j++) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < 3; l++)
          s += gbU[sy(k, l)] * (Dh_eps[sy(l, j)][i] + Dh_eps[sy(i, l)][j] - Dh_eps[sy(i, j)][l]);
        DUDD[k][sy(i, j)] = 0.5 * s;
      }
#pragma unroll
  for (int k = 0; k < 3; k++) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = 0; j < 3; j++) s += gbU[sy(i, j)] * DUDD[k][sy(i, j)];
    DU[k] = s;
  }
#pragma unroll
  for (int k = 0; k < 3; k++) {
#pragma unroll
    for (int a = 0; a < 6; a++) put(XS_DUDD + 6 * k + a, DUDD[k][a]);
    put(XS_DU + k, DU[k]);
  }
  {
    auto Dl = [&](int a, int b, int c) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < 3; l++) s += gb[sy(a, l)] * DUDD[l][sy(b, c)];
      return s;
    };
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = i; j < 3; j++) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 3; k++) s += 0.5 * DU[k] * (Dl(i, j, k) + Dl(j, i, k));
#pragma unroll
        for (int k = 0; k < 3; k++)
#pragma unroll
          for (int l = 0; l < 3; l++) {
            double t = 0.0;
#pragma unroll
            for (int m = 0; m < 3; m++)
              t += DUDD[m][sy(k, i)] * Dl(j, m, l) + DUDD[m][sy(k, j)] * Dl(i, m, l) +
                   DUDD[m][sy(i, k)] * Dl(m, j, l);
            s += gbU[sy(k, l)] * t;
          }
        Rl[sy(i, j)] += s;
      }
  }
  pair_barrier();  // 1: Delta, Q to the gauge wave; d vet, d lambda from it

  // ---- Lambdabar terms of the Ricci tensor: gammabar_k(i Dhat_j) Lambdabar^k
  {
    double Lam[3], DLam[3][3];
#pragma unroll
    for (int k = 0; k < 3; k++) Lam[k] = P.at(G_LAMU0 + k, 0, 0, 0) * R.iS[k];
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
      for (int j = 0; j < 3; j++) {
        double d = get(XS_DLAM + 3 * k + j) * R.iS[k] - Lam[k] * R.dS[k][j] * R.iS[k];
#pragma unroll
        for (int m = 0; m < 3; m++) d += Gh[k][j][m] * Lam[m];
        DLam[k][j] = d;
      }
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = i; j < 3; j++) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 3; k++) s += gb[sy(k, i)] * DLam[k][j] + gb[sy(k, j)] * DLam[k][i];
        Rl[sy(i, j)] += 0.5 * s;
      }
  }
  double dvet[3][3];  // read before XS_RT (which aliases the lambda slots) is written
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int k = 0; k < 3; k++) dvet[i][k] = get(XS_DVET + 3 * i + k);
  double RT[6];
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = i; j < 3; j++) {
      const int a = sy(i, j);
      RT[a] = -0.5 * Pc[a] + Rl[a] * (R.iS[i] * R.iS[j]);
      put(XS_RT + a, RT[a]);
    }
  pair_barrier();  // 2: the Ricci tensor to the gauge wave

  // ---- Eq. 7 (eps) ------------------------------------------------------------
  double res[6];
  {
    double dbeta[3][3], bS[3];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = 0; j < 3; j++) {
        const double diS = -R.dS[i][j] * (R.iS[i] * R.iS[i]);  // d_j (1/S_i)
        dbeta[i][j] = dvet[i][j] * R.iS[i] + vet[i] * diS;
      }
#pragma unroll
    for (int i = 0; i < 3; i++) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 3; k++) s += beta[k] * R.dS[i][k];
      bS[i] = s * R.iS[i];
    }
    double Dbeta = 0.0;  // Dbar_k beta^k with Gammabar^k_km = Gammahat^k_km + Delta^k_km
#pragma unroll
    for (int m = 0; m < 3; m++) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 3; k++) s += Gh[k][k][m] + DUDD[k][sy(k, m)];
      Dbeta += dbeta[m][m] + s * beta[m];
    }
    const double alpha = P.at(G_ALPHA, 0, 0, 0);
    double Abar[6];
#pragma unroll
    for (int c = 0; c < 6; c++) Abar[c] = P.at(G_ADD00 + c, 0, 0, 0) * SS[c];
    double trA = 0.0;
#pragma unroll
    for (int i = 0; i < 3; i++) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 3; k++) s += gbU[sy(i, k)] * Abar[sy(k, i)];
      trA += s;
    }
    double Dbh[3][3];  // Dhat_j beta^i
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = 0; j < 3; j++) {
        double s = dbeta[i][j];
#pragma unroll
        for (int m = 0; m < 3; m++) s += Gh[i][j][m] * beta[m];
        Dbh[i][j] = s;
      }
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = i; j < 3; j++) {
        const int c = sy(i, j);
        double r = (2.0 / 3.0) * gb[c] * (alpha * trA - Dbeta) + R.S[j] * R.S[j] * Dbh[j][i] +
                   R.S[i] * R.S[i] * Dbh[i][j] - 2.0 * alpha * Abar[c];
#pragma unroll
        for (int k = 0; k < 3; k++) r += eps[sy(k, j)] * dbeta[k][i] + eps[sy(i, k)] * dbeta[k][j];
        res[c] = adv[c] + (r * (R.iS[i] * R.iS[j]) + h[c] * (bS[i] + bS[j]));
      }
  }
  if (valid) {
    stage_store<MIX>(G, st, q, G_HDD00, G_HDD00 + 6, false, [&](int g) { return res[g - G_HDD00]; });
    if (aux) {
#pragma unroll
      for (int a = 0; a < 6; a++) aux[a * G.sgf + q] = RT[a];
#pragma unroll
      for (int k = 0; k < 3; k++) aux[(6 + k) * G.sgf + q] = get(XS_Q + k);
    }
  }
}

// ---- gauge wave ------------------------------------------------------------
template <int C, bool AX, bool KO, bool MIX, int H>
__device__ __forceinline__ void gauge_wave(const GridDev& G, const Gauge& ga, const double* __restrict__ y,
                                           const StageArgs& st, int i0, int i1, int i2, unsigned q, bool valid,
                                           double* __restrict__ xs) {
  constexpr int PD = C == BHAH_SINH_CYLINDRICAL ? 1 : 2;
  constexpr int RR = H - 1, SW = 2 * RR + 1;
  const double eta = ga.eta;
  double kw[3];
#pragma unroll
  for (int k = 0; k < 3; k++) kw[k] = G.inv_dx[k] * (1.0 / FdW<RR>::kden);
  auto put = [&](int v, double x) { xs[v * 64] = x; };
  auto get = [&](int v) { return xs[v * 64]; };
  // results accumulate in the park: the advection terms first, then each
  // equation adds the rest of its right-hand side
  auto emit = [&](int g, double v) { put(gslot(g), get(gslot(g)) + v); };
  const PtT<H> P(y, G, C, i0, i1, i2);
  const Spacing sp = make_spacing<RR>(G);
  Ref R;
  load_ref<C>(G, i0, i1, i2, R);

  // ---- point values and the conformal metric (Eq. 3) ----------------------
  double SS[6], gb[6], gbU[6];
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = i; j < 3; j++) {
      const int a = sy(i, j);
      SS[a] = R.S[i] * R.S[j];
      gb[a] = (i == j ? R.S[i] * R.S[i] : 0.0) + P.at(G_HDD00 + a, 0, 0, 0) * SS[a];
    }
  sym_inverse(gb, gbU);
  const double W = P.at(G_CF, 0, 0, 0), alpha = P.at(G_ALPHA, 0, 0, 0);
  const double iW = 1.0 / W;
  double vet[3], beta[3];
#pragma unroll
  for (int i = 0; i < 3; i++) {
    vet[i] = P.at(G_VETU0 + i, 0, 0, 0);
    beta[i] = vet[i] * R.iS[i];
  }
  UpwindT<H> U;
  U.v0 = q * 8u;
  {
    const int str[3] = {1, G.s1, G.s2};
#pragma unroll
    for (int k = 0; k < 3; k++) {
      const int s = vet[k] > 0.0 ? 1 : -1;
      if (k == P.pd) {
        const bool up = s > 0;
        U.vu[k][0] = up ? P.vper(1) : P.vper(-1);
        U.vd[k][0] = up ? P.vper(-1) : P.vper(1);
#pragma unroll
        for (int m = 2; m <= H; m++) U.vu[k][m - 1] = up ? P.vper(m) : P.vper(-m);
#pragma unroll
        for (int m = 2; m <= H; m++) U.vd[k][m - 1] = up ? P.vper(-m) : P.vper(m);
      } else {
        const int o = s * str[k];
        U.vu[k][0] = (q + o) * 8u;
        U.vd[k][0] = (q - o) * 8u;
#pragma unroll
        for (int m = 2; m <= H; m++) U.vu[k][m - 1] = (q + m * o) * 8u;
#pragma unroll
        for (int m = 2; m <= H; m++) U.vd[k][m - 1] = (q - m * o) * 8u;
      }
      U.w[k] = fabs(beta[k]) * sp.d1s[k];
    }
  }

  // ---- lambda^i: first derivatives (to the metric wave) and advection ----
  {
    constexpr int LB = H == 3 ? 3 : 1;
#pragma unroll
    for (int c0 = 0; c0 < 3; c0 += LB) {
      double v[LB][3][SW], f3[LB][3], fm3[KO ? LB : 1][3];
#pragma unroll
      for (int ii = 0; ii < LB; ii++)
#pragma unroll
        for (int k = 0; k < 3; k++) {
          gather_axis_k<PD, AX>(P, G_LAMU0 + c0 + ii, k, v[ii][k]);
          f3[ii][k] = upwind_far<PD, AX>(P, G_LAMU0 + c0 + ii, k, U.vu, v[ii][k]);
          if constexpr (KO) fm3[ii][k] = upwind_far<PD, AX>(P, G_LAMU0 + c0 + ii, k, U.vd, v[ii][k]);
        }
      BHAH_PHASE_BARRIER();
#pragma unroll
      for (int ii = 0; ii < LB; ii++) {
        const int i = c0 + ii;
        double a = 0.0, d = 0.0;
#pragma unroll
        for (int k = 0; k < 3; k++) {
          const bool up = vet[k] > 0.0;
          a += U.w[k] * upwind_sum<RR>(v[ii][k], f3[ii][k], up);
          if constexpr (KO) d += kw[k] * ko_v<RR>(v[ii][k], f3[ii][k], fm3[ii][k]);
          put(XS_DLAM + 3 * i + k, AX && k == PD ? 0.0 : d1_axis<RR>(v[ii][k], sp.d1s[k]));
        }
        put(gslot(G_LAMU0 + i), a + ga.dm * d);
        // bet^i's right-hand side takes 3/4 of lambda^i's undissipated one:
        // its result starts at -3/4 of lambda's dissipation, which the 3/4
        // of lambda's full result then cancels
        put(gslot(G_BETU0 + i), KO ? -0.75 * (ga.dm * d) : 0.0);
      }
    }
  }

  // ---- second derivatives of W, alpha and vet^i, pair (k,l) by pair -------
  //   Y_kl = (alpha/W) d_k d_l W - d_k d_l alpha       (Abar equation)
  //   Za   = gammabar^kl d_k d_l alpha                 (K equation)
  //   Bv^i = gammabar^kl d_k d_l vet^i, Bd_k = sum_j d_k d_j vet^j / S_j
  // the diagonal gathers also give the first derivatives and advection
  double Y[6], Za = 0.0, Bv[3], Bd[3], dW[3], dalpha[3], dvet[3][3];
#pragma unroll
  for (int i = 0; i < 3; i++) { Bv[i] = 0.0; Bd[i] = 0.0; }
  {
    const double aW = alpha * iW;
    constexpr int G5[5] = {G_CF, G_ALPHA, G_VETU0, G_VETU0 + 1, G_VETU0 + 2};
    double adv[5];
#pragma unroll
    for (int t = 0; t < 5; t++) adv[t] = 0.0;
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
      for (int l = k; l < 3; l++) {
        double dd[5];
        if (k == l) {
          constexpr int TB = H == 3 ? 5 : 3;
#pragma unroll
          for (int t0 = 0; t0 < 5; t0 += TB) {
            double v[TB][SW], fu[TB], fd[KO ? TB : 1];
#pragma unroll
            for (int t = 0; t < TB; t++)
              if (t0 + t < 5) {
                gather_axis_k<PD, AX>(P, G5[t0 + t], k, v[t]);
                fu[t] = upwind_far<PD, AX>(P, G5[t0 + t], k, U.vu, v[t]);
                if constexpr (KO) fd[t] = upwind_far<PD, AX>(P, G5[t0 + t], k, U.vd, v[t]);
              }
            BHAH_PHASE_BARRIER();
            const bool up = vet[k] > 0.0;
#pragma unroll
            for (int t = 0; t < TB; t++)
              if (t0 + t < 5) {
                const int tt = t0 + t;
                adv[tt] += U.w[k] * upwind_sum<RR>(v[t], fu[t], up);
                // W takes the metric strength, alpha and vet^i the gauge one
                if constexpr (KO) adv[tt] += (tt < 1 ? ga.dm : ga.dg) * kw[k] * ko_v<RR>(v[t], fu[t], fd[t]);
                dd[tt] = d2_axis<RR>(v[t], sp.d2s[k]);
                const double d1 = AX && k == PD ? 0.0 : d1_axis<RR>(v[t], sp.d1s[k]);
                if (tt == 0) dW[k] = d1;
                else if (tt == 1) dalpha[k] = d1;
                else dvet[tt - 2][k] = d1;
              }
          }
        } else if (AX && (k == PD || l == PD)) {
#pragma unroll
          for (int t = 0; t < 5; t++) dd[t] = 0.0;
        } else {
          constexpr int TX = H == 3 ? 3 : 1;
#pragma unroll
          for (int t0 = 0; t0 < 5; t0 += TX) {
            double v[TX][4 * RR * RR];
#pragma unroll
            for (int t = 0; t < TX; t++)
              if (t0 + t < 5) gather_cross_kl(P, G5[t0 + t], k, l, v[t]);
            BHAH_PHASE_BARRIER();
#pragma unroll
            for (int t = 0; t < TX; t++)
              if (t0 + t < 5) dd[t0 + t] = d2_cross<RR>(v[t], sp.crs[k][l]);
          }
        }
        const int kl = sy(k, l);
        const double wg = (k == l ? 1.0 : 2.0) * gbU[kl];
        Y[kl] = aW * dd[0] - dd[1];
        Za += wg * dd[1];
#pragma unroll
        for (int i = 0; i < 3; i++) {
          Bv[i] += wg * dd[2 + i];
          if (i == l) Bd[k] += dd[2 + i] * R.iS[l];
          if (k != l && i == k) Bd[l] += dd[2 + i] * R.iS[k];
        }
      }
    put(gslot(G_CF), adv[0]);
    put(gslot(G_ALPHA), adv[1]);
#pragma unroll
    for (int i = 0; i < 3; i++) put(gslot(G_VETU0 + i), adv[2 + i]);
  }
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int k = 0; k < 3; k++) put(XS_DVET + 3 * i + k, dvet[i][k]);
  BHAH_PHASE_BARRIER();

  // ---- advection of Abar_ij, B^i and K; K's first derivatives --------------
  if constexpr (H == 3) {
    constexpr int GA[3] = {G_ADD00, G_ADD00 + 1, G_ADD00 + 2}, GC[3] = {G_ADD00 + 3, G_ADD00 + 4, G_ADD00 + 5};
    const double e3[3] = {ga.dm, ga.dm, ga.dm};
    double a3[3];
    advect_batch<3, PD, AX, KO>(P, GA, U, a3, e3, kw);
#pragma unroll
    for (int t = 0; t < 3; t++) put(gslot(GA[t]), a3[t]);
    advect_batch<3, PD, AX, KO>(P, GC, U, a3, e3, kw);
#pragma unroll
    for (int t = 0; t < 3; t++) put(gslot(GC[t]), a3[t]);
    constexpr int GB[3] = {G_BETU0, G_BETU0 + 1, G_BETU0 + 2};
    const double eg[3] = {ga.dg, ga.dg, ga.dg};
    advect_batch<3, PD, AX, KO>(P, GB, U, a3, eg, kw);
#pragma unroll
    for (int t = 0; t < 3; t++) emit(GB[t], a3[t]);
  } else {
    constexpr int NB = AX ? 2 : 1;  // wider stencils: smaller batches
#pragma unroll
    for (int t = 0; t < 6; t += NB) {
      int gl[NB];
      double e[NB];
#pragma unroll
      for (int u = 0; u < NB; u++) {
        gl[u] = G_ADD00 + t + u;
        e[u] = ga.dm;
      }
      double a[NB];
      advect_batch<NB, PD, AX, KO>(P, gl, U, a, e, kw);
#pragma unroll
      for (int u = 0; u < NB; u++) put(gslot(gl[u]), a[u]);
    }
#pragma unroll
    for (int t = 0; t < 3; t++) {
      const int gl[1] = {G_BETU0 + t};
      const double e[1] = {ga.dg};
      double a[1];
      advect_batch<1, PD, AX, KO>(P, gl, U, a, e, kw);
      emit(G_BETU0 + t, a[0]);
    }
  }
  double dK[3];
  {
    double v[3][SW], f3[3], fm3[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
      gather_axis_k<PD, AX>(P, G_TRK, k, v[k]);
      f3[k] = upwind_far<PD, AX>(P, G_TRK, k, U.vu, v[k]);
      if constexpr (KO) fm3[k] = upwind_far<PD, AX>(P, G_TRK, k, U.vd, v[k]);
    }
    BHAH_PHASE_BARRIER();
    double advK = 0.0;
#pragma unroll
    for (int k = 0; k < 3; k++) {
      const bool up = vet[k] > 0.0;
      advK += U.w[k] * upwind_sum<RR>(v[k], f3[k], up);
      if constexpr (KO) advK += ga.dm * kw[k] * ko_v<RR>(v[k], f3[k], fm3[k]);
      dK[k] = AX && k == PD ? 0.0 : d1_axis<RR>(v[k], sp.d1s[k]);
    }
    put(gslot(G_TRK), advK);
  }
  pair_barrier();  // 1: Delta, Q from the metric wave; d vet, d lambda to it

  // everything still needed from the exchange slots, before barrier 2 (the
  // metric wave's next tile may overwrite them after it)
  double DUDD[3][6], DU[3], Q[3];
#pragma unroll
  for (int k = 0; k < 3; k++) {
#pragma unroll
    for (int a = 0; a < 6; a++) DUDD[k][a] = get(XS_DUDD + 6 * k + a);
    DU[k] = get(XS_DU + k);
    Q[k] = get(XS_Q + k);
  }
  double Gh[3][3][3];
  ref_christoffel(R, Gh);
  double diS[3][3];  // d_k (1/S_i)
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int k = 0; k < 3; k++) diS[i][k] = -R.dS[i][k] * (R.iS[i] * R.iS[i]);
  double dbeta[3][3], phi_d[3];
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) dbeta[i][j] = dvet[i][j] * R.iS[i] + vet[i] * diS[i][j];
#pragma unroll
  for (int k = 0; k < 3; k++) phi_d[k] = -0.5 * dW[k] * iW;
  double bS[3];  // beta^k d_k S_i / S_i
#pragma unroll
  for (int i = 0; i < 3; i++) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 3; k++) s += beta[k] * R.dS[i][k];
    bS[i] = s * R.iS[i];
  }
  const double K = P.at(G_TRK, 0, 0, 0);
  double Gbc[3];  // Gammabar^k_km
#pragma unroll
  for (int m = 0; m < 3; m++) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 3; k++) s += Gh[k][k][m] + DUDD[k][sy(k, m)];
    Gbc[m] = s;
  }
  double Dbeta = 0.0;  // Dbar_k beta^k
#pragma unroll
  for (int k = 0; k < 3; k++) Dbeta += dbeta[k][k] + Gbc[k] * beta[k];

  double a6[6], Abar[6], AUD[3][3], AUU[6];
#pragma unroll
  for (int c = 0; c < 6; c++) { a6[c] = P.at(G_ADD00 + c, 0, 0, 0); Abar[c] = a6[c] * SS[c]; }
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 3; k++) s += gbU[sy(i, k)] * Abar[sy(k, j)];
      AUD[i][j] = s;
    }
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = i; j < 3; j++) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 3; k++) s += AUD[i][k] * gbU[sy(k, j)];
      AUU[sy(i, j)] = s;
    }
  double AA = 0.0;
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) AA += Abar[sy(i, j)] * AUU[sy(i, j)];
  const double W2 = W * W;

  // Eq. 9 (W), Eq. 13 (alpha), Eq. 10 (K)
  emit(G_CF, -(1.0 / 3.0) * W * (Dbeta - alpha * K));
  emit(G_ALPHA, -2.0 * alpha * K);
  {
    double lap = Za, da_dphi = 0.0;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = 0; j < 3; j++) {
        double Ga = 0.0;
#pragma unroll
        for (int k = 0; k < 3; k++) Ga += (Gh[k][i][j] + DUDD[k][sy(i, j)]) * dalpha[k];
        lap -= gbU[sy(i, j)] * Ga;
        da_dphi += gbU[sy(i, j)] * dalpha[i] * phi_d[j];
      }
    emit(G_TRK, (1.0 / 3.0) * alpha * K * K + alpha * AA - W2 * (lap + 2.0 * da_dphi));
  }
  BHAH_PHASE_BARRIER();

  // Eq. 11 (Lambdabar, lapse factors restored), Eqs. 14-15 (shift, B)
  {
    double dGh[3][3][3][3];
    ref_christoffel_deriv(R, dGh);
    double ddiS[3][6];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = 0; j < 3; j++)
#pragma unroll
        for (int k = j; k < 3; k++)
          ddiS[i][sy(j, k)] = -R.ddS[i][j][k] * (R.iS[i] * R.iS[i]) +
                              2.0 * R.dS[i][j] * R.dS[i][k] * (R.iS[i] * R.iS[i] * R.iS[i]);
    double Dbh[3][3];  // Dhat_j beta^i
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = 0; j < 3; j++) {
        double s = dbeta[i][j];
#pragma unroll
        for (int m = 0; m < 3; m++) s += Gh[i][j][m] * beta[m];
        Dbh[i][j] = s;
      }
    double dDbeta[3];  // d_k (Dbar_j beta^j)
#pragma unroll
    for (int k = 0; k < 3; k++) {
      double s = Bd[k] + Q[k];
#pragma unroll
      for (int j = 0; j < 3; j++) s += dvet[j][k] * diS[j][j] + dvet[j][j] * diS[j][k] + vet[j] * ddiS[j][sy(j, k)];
#pragma unroll
      for (int m = 0; m < 3; m++) s += Gbc[m] * dbeta[m][k];
      dDbeta[k] = s;
    }
#pragma unroll
    for (int i = 0; i < 3; i++) {
      double t2 = Bv[i] * R.iS[i];  // gammabar^jk Dhat_j Dhat_k beta^i
#pragma unroll
      for (int j = 0; j < 3; j++)
#pragma unroll
        for (int k = 0; k < 3; k++) {
          double s = dvet[i][j] * diS[i][k] + dvet[i][k] * diS[i][j] + vet[i] * ddiS[i][sy(j, k)];
#pragma unroll
          for (int m = 0; m < 3; m++)
            s += dGh[i][k][m][j] * beta[m] + Gh[i][k][m] * dbeta[m][j] + Gh[i][j][m] * Dbh[m][k] -
                 Gh[m][j][k] * Dbh[i][m];
          t2 += gbU[sy(j, k)] * s;
        }
      double t4 = 0.0, t5 = 0.0, t6 = 0.0, t7 = 0.0, lie = 0.0;
#pragma unroll
      for (int j = 0; j < 3; j++) {
        const double Lamj = P.at(G_LAMU0 + j, 0, 0, 0) * R.iS[j];
        t4 += gbU[sy(i, j)] * dDbeta[j];
        t5 += AUU[sy(i, j)] * (dalpha[j] - 6.0 * alpha * phi_d[j]);
        t7 += gbU[sy(i, j)] * dK[j];
        lie -= Lamj * dbeta[i][j];
#pragma unroll
        for (int k = 0; k < 3; k++) t6 += AUU[sy(j, k)] * DUDD[i][sy(j, k)];
      }
      const double r = t2 + (2.0 / 3.0) * DU[i] * Dbeta + (1.0 / 3.0) * t4 - 2.0 * t5 + 2.0 * alpha * t6 -
                       (4.0 / 3.0) * alpha * t7 + lie;
      const double lam = P.at(G_LAMU0 + i, 0, 0, 0);
      emit(G_LAMU0 + i, r * R.S[i] - lam * bS[i]);
      const double rl = get(gslot(G_LAMU0 + i));  // full d_t lambda^i, advection included
      const double bet = P.at(G_BETU0 + i, 0, 0, 0);
      emit(G_VETU0 + i, bet - vet[i] * bS[i]);
      emit(G_BETU0 + i, 0.75 * rl - eta * bet - bet * bS[i]);
    }
  }
  pair_barrier();  // 2: the Ricci tensor from the metric wave

  // Eq. 8 (Abar)
  {
    double X[6], trX = 0.0;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = i; j < 3; j++) {
        const int c = sy(i, j);
        double Gphi = 0.0;
#pragma unroll
        for (int k = 0; k < 3; k++)
          Gphi += (Gh[k][i][j] + DUDD[k][c]) * (2.0 * alpha * phi_d[k] + dalpha[k]);
        X[c] = Y[c] - alpha * dW[i] * dW[j] * (iW * iW) + Gphi + 4.0 * alpha * phi_d[i] * phi_d[j] +
               2.0 * (dalpha[i] * phi_d[j] + dalpha[j] * phi_d[i]) + alpha * get(XS_RT + c) * SS[c];
      }
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = 0; j < 3; j++) trX += gbU[sy(i, j)] * X[sy(i, j)];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = i; j < 3; j++) {
        const int c = sy(i, j);
        double AikAkj = 0.0;
#pragma unroll
        for (int k = 0; k < 3; k++) AikAkj += Abar[sy(i, k)] * AUD[k][j];
        double r = -(2.0 / 3.0) * Abar[c] * Dbeta - 2.0 * alpha * AikAkj + alpha * Abar[c] * K +
                   W2 * (X[c] - (1.0 / 3.0) * gb[c] * trX);
#pragma unroll
        for (int k = 0; k < 3; k++) r += Abar[sy(k, j)] * dbeta[k][i] + Abar[sy(i, k)] * dbeta[k][j];
        emit(G_ADD00 + c, r * (R.iS[i] * R.iS[j]) + a6[c] * (bS[i] + bS[j]));
      }
  }
  if (valid) stage_store<MIX>(G, st, q, 0, NGF, true, [&](int g) { return get(gslot(g)); });
}

// tile_point for the two-wave form: a lane past the grid's end takes the
// nearest interior point instead (the phi index, uniform over the tile, is
// never past the end), so both waves reach their barriers; its results are
// not stored.
template <int H>
__device__ __forceinline__ bool tile_point_clamped(const GridDev& G, const TileMap& T, int w, int lane, int& i0,
                                                   int& i1, int& i2) {
  const bool ok = tile_point<H>(G, T, w, lane, i0, i1, i2);
  i0 = min(i0, H + G.N0 - 1);
  i1 = min(i1, H + G.N1 - 1);
  i2 = min(i2, H + G.N2 - 1);
  return ok;
}

// one block of two waves per 64-point tile, each wave on its own SIMD
template <int C, bool AX, bool KO, int H>
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_rhs_pair(GridDev G, TileMap T, Gauge ga, const double* __restrict__ y, StageArgs st, double* __restrict__ aux) {
  const int per = (T.ntiles + BHAH_NXCD - 1) / BHAH_NXCD;
  const int w = xcd_remap((int)blockIdx.x, per);
  if (w >= T.ntiles) return;  // the whole block
  const int lane = (int)threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  int i0, i1, i2;
  const bool valid = tile_point_clamped<H>(G, T, w, lane, i0, i1, i2);
  const unsigned q = (unsigned)(i0 + G.s1 * i1 + G.s2 * i2);
  __shared__ double xs[XSLOTS * 64];
  if (wave == 0)
    metric_wave<C, AX, KO, true, H>(G, ga, y, st, i0, i1, i2, q, valid, aux, xs + lane);
  else
    gauge_wave<C, AX, KO, true, H>(G, ga, y, st, i0, i1, i2, q, valid, xs + lane);
}

template <int C, bool AX, bool KO, int H>
void launch_pair_t(dim3 g, hipStream_t s, const GridDev& G, const TileMap& T, const Gauge& ga, const double* y,
                   const StageArgs& st, double* aux) {
  hipLaunchKernelGGL((k_rhs_pair<C, AX, KO, H>), g, dim3(128), 0, s, G, T, ga, y, st, aux);
}
using PairLaunch = void (*)(dim3, hipStream_t, const GridDev&, const TileMap&, const Gauge&, const double*,
                            const StageArgs&, double*);
// Built where the split fits one wave per SIMD without spilling: 4th order,
// no dissipation, every variant but the general SinhSpherical one (108 bytes
// per lane of spills), and the two-plane SinhCylindrical variant with
// dissipation (the head-on production numerics at 4th order). Elsewhere the
// entry is empty and the one-wave kernel runs. [variant][dissipation]
constexpr int PSS = BHAH_SINH_SPHERICAL, PSC = BHAH_SINH_CYLINDRICAL, PSP = BHAH_SPHERICAL;
static const PairLaunch kPair[NVAR][2] = {
    {nullptr, nullptr},
    {launch_pair_t<PSS, true, false, 3>, nullptr},
    {launch_pair_t<PSC, false, false, 3>, nullptr},
    {launch_pair_t<PSC, true, false, 3>, launch_pair_t<PSC, true, true, 3>},
    {launch_pair_t<PSP, false, false, 3>, nullptr},
    {launch_pair_t<PSP, true, false, 3>, nullptr}};

bool have_rhs_pair(const GridDev& G, bool ko) {
  return G.ng == 3 && kPair[rhs_variant(G.coord, G.N1, G.N2)][ko ? 1 : 0] != nullptr;
}

// callers check have_rhs_pair first
void launch_rhs_pair(const GridDev& G, const Gauge& ga, const double* y, double* aux, const StageArgs& st,
                     hipStream_t s, const TileMap& T) {
  const int per = (T.ntiles + BHAH_NXCD - 1) / BHAH_NXCD;
  kPair[rhs_variant(G.coord, G.N1, G.N2)][ga.ko() ? 1 : 0](dim3(per * BHAH_NXCD), s, G, T, ga, y, st, aux);
}

}  // namespace bhah
