// rhs_common.h -- device building blocks of the BSSN right-hand sides.
//
// Notation follows Sec. 2.1-2.2 of arXiv:2505.00097: eps_ij = gammabar_ij -
// gammahat_ij, Delta^k_ij = Gammabar^k_ij - Gammahat^k_ij, W = exp(-2 phi),
// rescaled variables h_ij = eps_ij/(S_i S_j), lambda^i = S_i Lambdabar^i, ...
// All tensors are in the coordinate basis of the logical coordinates xx^i;
// reference-metric quantities come from 1-D tables and are assembled with
// their structural zeros as literal zeros, which the compiler folds away for
// each coordinate family (this translation unit is built with
// -fno-signed-zeros -ffinite-math-only; no reassociation is enabled).
#pragma once

#include "bhah_internal.h"

namespace bhah {

enum {
  G_ADD00 = 0, G_ALPHA = 6, G_BETU0 = 7, G_CF = 10, G_HDD00 = 11, G_LAMU0 = 17,
  G_TRK = 20, G_VETU0 = 21
};

// symmetric pair (i,j) -> 0..5 in the order 00,01,02,11,12,22
__host__ __device__ constexpr int sy(int i, int j) {
  return i <= j ? (i * (5 - i)) / 2 + j : (j * (5 - j)) / 2 + i;
}

// Stencil loads through buffer descriptors: one descriptor per group of four
// gridfunctions (base = the group's first element, range = its size in
// bytes), the gridfunction's place in its group and the wave-uniform part of
// the stencil offset as scalar offset, the per-lane part as vector offset.
// Few descriptors stay live (scalar registers are scarce in the stencil
// kernels); an access outside the group returns 0 instead of faulting.
// Grids are limited to 2^26 points so every offset fits 31 bits.
typedef unsigned int bhah_u2 __attribute__((ext_vector_type(2)));

typedef unsigned int bhah_u4 __attribute__((ext_vector_type(4)));

// two consecutive doubles (along i0) in one 16-byte load: a wave's vector
// memory pipeline moves twice the data per instruction
__device__ __forceinline__ void gf_ld2(const double* y, long long sgf, int g, unsigned voff, int soff, double& lo,
                                       double& hi) {
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc((void*)(y + (g >> 2) * 4 * sgf), (short)0, (int)(4 * sgf * 8), 0x00020000);
  const bhah_u4 v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff + (g & 3) * (int)(sgf * 8), 0);
  lo = __builtin_bit_cast(double, (unsigned long long)v.x | ((unsigned long long)v.y << 32));
  hi = __builtin_bit_cast(double, (unsigned long long)v.z | ((unsigned long long)v.w << 32));
}

__device__ __forceinline__ double gf_ld(const double* y, long long sgf, int g, unsigned voff, int soff) {
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc((void*)(y + (g >> 2) * 4 * sgf), (short)0, (int)(4 * sgf * 8), 0x00020000);
  const bhah_u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff + (g & 3) * (int)(sgf * 8), 0);
  return __builtin_bit_cast(double, v);
}

// Stencil access around one point. Stencil values are read with raw buffer
// loads: the per-lane part of the byte offset goes in the vector offset, the
// part shared by the wave in the scalar offset. The periodic direction phi
// (i1 on SinhCylindrical grids, i2 on spherical ones) is read with the index
// wrapped onto the interior planes, so phi ghost points are never read: they
// are exact copies of those planes (periodicity, no parity change), and the
// values read are identical. The phi index must be the same for every lane of
// the wave (tile extent 1 along phi).
struct Pt {
  const double* __restrict__ y;
  long long sgf;
  int pd;       // periodic direction (1 or 2)
  int se;       // stride of the other transverse direction
  unsigned vb;  // per-lane byte offset of (i0 - 3, i_e - 3) with the phi index removed
  int sw[7];    // byte offsets of the wrapped phi planes at offsets -3..3 (wave-uniform)

  __device__ __forceinline__ Pt(const double* y_, const GridDev& G, int C, int i0, int i1, int i2)
      : y(y_), sgf(G.sgf) {
    pd = C == BHAH_SINH_CYLINDRICAL ? 1 : 2;
    const int sd = pd == 1 ? G.s1 : G.s2;
    const int nd = pd == 1 ? G.N1 : G.N2;
    se = pd == 1 ? G.s2 : G.s1;
    const int ie = pd == 1 ? i2 : i1;
    const int id = __builtin_amdgcn_readfirstlane((pd == 1 ? i1 : i2) - NG);
    vb = (unsigned)(i0 - 3 + se * (ie - 3)) * 8u;
#pragma unroll
    for (int o = -3; o <= 3; o++) {
      int x = id + o;
      x += x < 0 ? nd : 0;
      x += x < 0 ? nd : 0;
      x -= x >= nd ? nd : 0;
      x -= x >= nd ? nd : 0;
      sw[o + 3] = (NG + x) * sd * 8;
    }
  }

  // value at offsets (a, b, c) along (i0, i1, i2)
  __device__ __forceinline__ double at(int g, int a, int b, int c) const {
    const int od = pd == 1 ? b : c, oe = pd == 1 ? c : b;
    return gf_ld(y, sgf, g, vb + (unsigned)((a + 3) * 8), sw[od + 3] + (oe + 3) * se * 8);
  }
  // values at offsets (a, b, c) and (a + 1, b, c)
  __device__ __forceinline__ void at2(int g, int a, int b, int c, double& lo, double& hi) const {
    const int od = pd == 1 ? b : c, oe = pd == 1 ? c : b;
    gf_ld2(y, sgf, g, vb + (unsigned)((a + 3) * 8), sw[od + 3] + (oe + 3) * se * 8, lo, hi);
  }
  // byte offset of the point shifted by m along the periodic direction
  __device__ __forceinline__ unsigned vper(int m) const { return vb + 24u + (unsigned)(3 * se * 8 + sw[m + 3]); }
  template <int K>
  __device__ __forceinline__ double ax(int g, int m) const {
    return K == 0 ? at(g, m, 0, 0) : (K == 1 ? at(g, 0, m, 0) : at(g, 0, 0, m));
  }
  // value at offsets m along K and n along L (K != L)
  template <int K, int L>
  __device__ __forceinline__ double pl(int g, int m, int n) const {
    const int a = (K == 0 ? m : 0) + (L == 0 ? n : 0);
    const int b = (K == 1 ? m : 0) + (L == 1 ? n : 0);
    const int c = (K == 2 ? m : 0) + (L == 2 ? n : 0);
    return at(g, a, b, c);
  }
};

struct Spacing {
  double i12h[3];       // 1/(12 dxx^k)
  double i12hh[3];      // 1/(12 dxx^k^2)
  double i144[3][3];    // 1/(144 dxx^k dxx^l)
};

__device__ __forceinline__ Spacing make_spacing(const GridDev& G) {
  Spacing s;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    s.i12h[k] = G.inv_dx[k] * (1.0 / 12.0);
    s.i12hh[k] = G.inv_dx[k] * G.inv_dx[k] * (1.0 / 12.0);
  }
#pragma unroll
  for (int k = 0; k < 3; k++)
#pragma unroll
    for (int l = 0; l < 3; l++) s.i144[k][l] = G.inv_dx[k] * G.inv_dx[l] * (1.0 / 144.0);
  return s;
}

// ---- 4th-order finite differences (Sec. 3): centred 5-point stencils,
// their tensor product for mixed derivatives. Sums are grouped into
// differences so constant fields have exactly zero derivatives.
template <int K>
__device__ __forceinline__ double fd1(const Pt& P, int g, const Spacing& s) {
  return (8.0 * (P.ax<K>(g, 1) - P.ax<K>(g, -1)) - (P.ax<K>(g, 2) - P.ax<K>(g, -2))) * s.i12h[K];
}
template <int K>
__device__ __forceinline__ double fd2(const Pt& P, int g, const Spacing& s) {
  return (16.0 * (P.ax<K>(g, 1) + P.ax<K>(g, -1)) - (P.ax<K>(g, 2) + P.ax<K>(g, -2)) -
          30.0 * P.ax<K>(g, 0)) *
         s.i12hh[K];
}
template <int K, int L>
__device__ __forceinline__ double fdm(const Pt& P, int g, const Spacing& s) {
  // D_K D_L f; the inner differences are left unnormalised
  auto e = [&](int m) {
    return 8.0 * (P.pl<K, L>(g, m, 1) - P.pl<K, L>(g, m, -1)) -
           (P.pl<K, L>(g, m, 2) - P.pl<K, L>(g, m, -2));
  };
  return (8.0 * (e(1) - e(-1)) - (e(2) - e(-2))) * s.i144[K][L];
}
// Batched stencil gathers: values land in a local array first so that a
// whole batch of loads is in flight before any is consumed.
//   axis : f(-2), f(-1), f(0), f(1), f(2) along K
//   cross: f(m, n) along (K, L) for m, n in {-2, -1, 1, 2}, m-major
template <int K>
__device__ __forceinline__ void gather_axis(const Pt& P, int g, double v[5]) {
  if constexpr (K == 0) {  // i0 neighbours are adjacent in memory: pairs per load
    P.at2(g, -2, 0, 0, v[0], v[1]);
    v[2] = P.at(g, 0, 0, 0);
    P.at2(g, 1, 0, 0, v[3], v[4]);
  } else {
#pragma unroll
    for (int t = 0; t < 5; t++) v[t] = P.ax<K>(g, t - 2);
  }
}
template <int K, int L>
__device__ __forceinline__ void gather_cross(const Pt& P, int g, double v[16]) {
  constexpr int off[4] = {-2, -1, 1, 2};
  if constexpr (K == 0) {  // rows along i0 in pairs per load
#pragma unroll
    for (int b = 0; b < 4; b++) {
      const int o1 = L == 1 ? off[b] : 0, o2 = L == 2 ? off[b] : 0;
      P.at2(g, -2, o1, o2, v[b], v[4 + b]);
      P.at2(g, 1, o1, o2, v[8 + b], v[12 + b]);
    }
  } else {
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
      for (int b = 0; b < 4; b++) v[4 * a + b] = P.pl<K, L>(g, off[a], off[b]);
  }
}
__device__ __forceinline__ double d1_axis(const double v[5], double s) {
  return (8.0 * (v[3] - v[1]) - (v[4] - v[0])) * s;
}
__device__ __forceinline__ double d2_axis(const double v[5], double s) {
  return (16.0 * (v[3] + v[1]) - (v[4] + v[0]) - 30.0 * v[2]) * s;
}
__device__ __forceinline__ double d2_cross(const double v[16], double s) {
  auto e = [&](int a) { return 8.0 * (v[4 * a + 2] - v[4 * a + 1]) - (v[4 * a + 3] - v[4 * a + 0]); };
  return (8.0 * (e(2) - e(1)) - (e(3) - e(0))) * s;
}

__device__ __forceinline__ double fd1k(const Pt& P, int g, int k, const Spacing& s) {
  return k == 0 ? fd1<0>(P, g, s) : (k == 1 ? fd1<1>(P, g, s) : fd1<2>(P, g, s));
}
// second derivative d_k d_l (any order of k, l)
__device__ __forceinline__ double fd2kl(const Pt& P, int g, int k, int l, const Spacing& s) {
  if (k == l) return k == 0 ? fd2<0>(P, g, s) : (k == 1 ? fd2<1>(P, g, s) : fd2<2>(P, g, s));
  const int a = k < l ? k : l, b = k < l ? l : k;
  return a == 0 ? (b == 1 ? fdm<0, 1>(P, g, s) : fdm<0, 2>(P, g, s)) : fdm<1, 2>(P, g, s);
}

// ---- reference metric at a point -----------------------------------------
// gammahat_ij = diag(S_i^2): (r'^2, r^2, r^2 sin^2 theta) for the spherical
// family, (rho'^2, rho^2, z'^2) for the cylindrical one.
struct Ref {
  double S[3], iS[3];
  double dS[3][3];      // [i][k] = d_k S_i
  double ddS[3][3][3];  // [i][k][l] = d_k d_l S_i
};

template <int C>
__device__ __forceinline__ void load_ref(const GridDev& G, int i0, int i1, int i2, Ref& R) {
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) {
      R.dS[a][b] = 0.0;
#pragma unroll
      for (int c = 0; c < 3; c++) R.ddS[a][b][c] = 0.0;
    }
  const double* t0 = G.tab0 + i0 * TAB_W;
  const double r = t0[0], rp = t0[1];
  const double rpp = C == BHAH_SPHERICAL ? 0.0 : t0[2];
  const double rppp = C == BHAH_SPHERICAL ? 0.0 : t0[3];
  const double ir = t0[4], irp = t0[5];
  if constexpr (C == BHAH_SINH_CYLINDRICAL) {
    const double* t2 = G.tab2 + i2 * TAB_W;
    R.S[0] = rp; R.S[1] = r; R.S[2] = t2[1];
    R.iS[0] = irp; R.iS[1] = ir; R.iS[2] = t2[5];
    R.dS[0][0] = rpp; R.dS[1][0] = rp; R.dS[2][2] = t2[2];
    R.ddS[0][0][0] = rppp; R.ddS[1][0][0] = rpp; R.ddS[2][2][2] = t2[3];
  } else {
    const double* t1 = G.tab1 + i1 * TAB_W;
    const double st = t1[0], ct = t1[1], ist = t1[2];
    R.S[0] = rp; R.S[1] = r; R.S[2] = r * st;
    R.iS[0] = irp; R.iS[1] = ir; R.iS[2] = ir * ist;
    R.dS[0][0] = rpp; R.dS[1][0] = rp; R.dS[2][0] = rp * st; R.dS[2][1] = r * ct;
    R.ddS[0][0][0] = rppp; R.ddS[1][0][0] = rpp; R.ddS[2][0][0] = rpp * st;
    R.ddS[2][0][1] = rp * ct; R.ddS[2][1][0] = rp * ct; R.ddS[2][1][1] = -r * st;
  }
}

// Christoffel symbols of the diagonal reference metric:
// Gh^i_ik = Gh^i_ki = d_k S_i / S_i, Gh^i_jj = -S_j d_i S_j / S_i^2 (j != i).
__device__ __forceinline__ void ref_christoffel(const Ref& R, double Gh[3][3][3]) {
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++)
#pragma unroll
      for (int k = 0; k < 3; k++) {
        double v = 0.0;
        if (i == j) v = R.dS[i][k] * R.iS[i];
        else if (i == k) v = R.dS[i][j] * R.iS[i];
        else if (j == k) v = -R.S[j] * R.dS[j][i] * (R.iS[i] * R.iS[i]);
        Gh[i][j][k] = v;
      }
}

// dGh[i][j][k][l] = d_l Gammahat^i_jk
__device__ __forceinline__ void ref_christoffel_deriv(const Ref& R, double dGh[3][3][3][3]) {
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++)
#pragma unroll
      for (int k = 0; k < 3; k++)
#pragma unroll
        for (int l = 0; l < 3; l++) {
          const double i2 = R.iS[i] * R.iS[i];
          double v = 0.0;
          if (i == j || i == k) {
            const int m = i == j ? k : j;  // Gh^i_im = dS[i][m]/S_i
            v = R.ddS[i][m][l] * R.iS[i] - R.dS[i][m] * R.dS[i][l] * i2;
          } else if (j == k) {  // Gh^i_jj = -S_j dS[j][i] / S_i^2
            v = -(R.dS[j][l] * R.dS[j][i] + R.S[j] * R.ddS[j][i][l]) * i2 +
                2.0 * R.S[j] * R.dS[j][i] * R.dS[i][l] * (i2 * R.iS[i]);
          }
          dGh[i][j][k][l] = v;
        }
}

// ---- metric pieces shared by the kernels ------------------------------------
struct Metric {
  double SS[6];        // S_i S_j
  double dSS[6][3];    // d_k (S_i S_j)
  double h[6];         // rescaled
  double dh[6][3];
  double eps[6], deps[6][3];
  double gb[6], gbU[6];  // gammabar_ij and its inverse
  double Dh_eps[6][3];   // Dhat_k eps_ij at [ij][k]
  double DUDD[3][6];     // Delta^k_ij
  double DU[3];          // Delta^k
};

__device__ __forceinline__ void sym_inverse(const double g[6], double gi[6]) {
  const double c00 = g[3] * g[5] - g[4] * g[4];
  const double c01 = g[2] * g[4] - g[1] * g[5];
  const double c02 = g[1] * g[4] - g[2] * g[3];
  const double det = g[0] * c00 + g[1] * c01 + g[2] * c02;
  const double id = 1.0 / det;
  gi[0] = c00 * id;
  gi[1] = c01 * id;
  gi[2] = c02 * id;
  gi[3] = (g[0] * g[5] - g[2] * g[2]) * id;
  gi[4] = (g[1] * g[2] - g[0] * g[4]) * id;
  gi[5] = (g[0] * g[3] - g[1] * g[1]) * id;
}

// eps, its first derivatives, gammabar, its inverse, Dhat eps and Delta
// (Eq. 3; Eq. 4 in the form Delta^k_ij = 1/2 gammabar^kl (Dhat_i eps_lj +
// Dhat_j eps_il - Dhat_l eps_ij); Eq. 5).
__device__ __forceinline__ void metric_first(const Pt& P, const Ref& R, const double Gh[3][3][3],
                                             const Spacing& sp, Metric& M) {
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = i; j < 3; j++) {
      const int a = sy(i, j);
      M.SS[a] = R.S[i] * R.S[j];
#pragma unroll
      for (int k = 0; k < 3; k++) M.dSS[a][k] = R.dS[i][k] * R.S[j] + R.S[i] * R.dS[j][k];
      M.h[a] = P.at(G_HDD00 + a, 0, 0, 0);
#pragma unroll
      for (int k = 0; k < 3; k++) M.dh[a][k] = fd1k(P, G_HDD00 + a, k, sp);
      M.eps[a] = M.h[a] * M.SS[a];
#pragma unroll
      for (int k = 0; k < 3; k++) M.deps[a][k] = M.dh[a][k] * M.SS[a] + M.h[a] * M.dSS[a][k];
      M.gb[a] = (i == j ? R.S[i] * R.S[i] : 0.0) + M.eps[a];
    }
  sym_inverse(M.gb, M.gbU);
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = i; j < 3; j++)
#pragma unroll
      for (int k = 0; k < 3; k++) {
        double s = M.deps[sy(i, j)][k];
#pragma unroll
        for (int m = 0; m < 3; m++) s -= Gh[m][k][i] * M.eps[sy(m, j)] + Gh[m][k][j] * M.eps[sy(i, m)];
        M.Dh_eps[sy(i, j)][k] = s;
      }
#pragma unroll
  for (int k = 0; k < 3; k++)
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = i; j < 3; j++) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < 3; l++)
          s += M.gbU[sy(k, l)] * (M.Dh_eps[sy(l, j)][i] + M.Dh_eps[sy(i, l)][j] - M.Dh_eps[sy(i, j)][l]);
        M.DUDD[k][sy(i, j)] = 0.5 * s;
      }
#pragma unroll
  for (int k = 0; k < 3; k++) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = 0; j < 3; j++) s += M.gbU[sy(i, j)] * M.DUDD[k][sy(i, j)];
    M.DU[k] = s;
  }
}

// Conformal Ricci tensor, Eq. 12, and Q_k = (d_k Gammabar^j_jm) beta^m with
// d_k Gammabar^j_jm = 1/2 (gammabar^jl d_k d_m gammabar_jl
//                          - gammabar^ja gammabar^lb d_k gammabar_ab d_m gammabar_jl).
// Rc[ij] is the coordinate-basis Rbar_ij.
template <int C>
__device__ __forceinline__ void ricci_and_Q(const Pt& P, const Ref& R, const double Gh[3][3][3],
                                            const Spacing& sp, const Metric& M, double Rc[6],
                                            double Q[3], bool want_Q) {
  double dGh[3][3][3][3];
  ref_christoffel_deriv(R, dGh);
  // Delta_ijk = gammabar_il Delta^l_jk
  double DDDD[3][6];
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int jk = 0; jk < 6; jk++) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < 3; l++) s += M.gb[sy(i, l)] * M.DUDD[l][jk];
      DDDD[i][jk] = s;
    }
  // algebraic Delta terms
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = i; j < 3; j++) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 3; k++) s += 0.5 * M.DU[k] * (DDDD[i][sy(j, k)] + DDDD[j][sy(i, k)]);
#pragma unroll
      for (int k = 0; k < 3; k++)
#pragma unroll
        for (int l = 0; l < 3; l++) {
          double t = 0.0;
#pragma unroll
          for (int m = 0; m < 3; m++)
            t += M.DUDD[m][sy(k, i)] * DDDD[j][sy(m, l)] + M.DUDD[m][sy(k, j)] * DDDD[i][sy(m, l)] +
                 M.DUDD[m][sy(i, k)] * DDDD[m][sy(j, l)];
          s += M.gbU[sy(k, l)] * t;
        }
      Rc[sy(i, j)] = s;
    }
  // Lambdabar terms: gammabar_k(i Dhat_j) Lambdabar^k
  {
    double Lam[3], DLam[3][3];  // DLam[k][j] = Dhat_j Lambdabar^k
#pragma unroll
    for (int k = 0; k < 3; k++) Lam[k] = P.at(G_LAMU0 + k, 0, 0, 0) * R.iS[k];
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
      for (int j = 0; j < 3; j++) {
        const double lam = P.at(G_LAMU0 + k, 0, 0, 0);
        double d = fd1k(P, G_LAMU0 + k, j, sp) * R.iS[k] - lam * R.dS[k][j] * (R.iS[k] * R.iS[k]);
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
        for (int k = 0; k < 3; k++) s += M.gb[sy(k, i)] * DLam[k][j] + M.gb[sy(k, j)] * DLam[k][i];
        Rc[sy(i, j)] += 0.5 * s;
      }
  }
  // second-derivative terms, one (k,l) pair at a time
  double cQ[6];
#pragma unroll
  for (int k = 0; k < 3; k++)
#pragma unroll
    for (int l = k; l < 3; l++) {
      double ddeps[6];
#pragma unroll
      for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = i; j < 3; j++) {
          const int a = sy(i, j);
          const double ddSS = R.ddS[i][k][l] * R.S[j] + R.dS[i][k] * R.dS[j][l] +
                              R.dS[i][l] * R.dS[j][k] + R.S[i] * R.ddS[j][k][l];
          ddeps[a] = fd2kl(P, G_HDD00 + a, k, l, sp) * M.SS[a] + M.dh[a][k] * M.dSS[a][l] +
                     M.dh[a][l] * M.dSS[a][k] + M.h[a] * ddSS;
        }
      const double wkl = (k == l ? -0.5 : -1.0) * M.gbU[sy(k, l)];
#pragma unroll
      for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = i; j < 3; j++) {
          // Dhat_k Dhat_l eps_ij
          double s = ddeps[sy(i, j)];
#pragma unroll
          for (int m = 0; m < 3; m++)
            s -= dGh[m][l][i][k] * M.eps[sy(m, j)] + Gh[m][l][i] * M.deps[sy(m, j)][k] +
                 dGh[m][l][j][k] * M.eps[sy(i, m)] + Gh[m][l][j] * M.deps[sy(i, m)][k];
#pragma unroll
          for (int m = 0; m < 3; m++)
            s -= Gh[m][k][l] * M.Dh_eps[sy(i, j)][m] + Gh[m][k][i] * M.Dh_eps[sy(m, j)][l] +
                 Gh[m][k][j] * M.Dh_eps[sy(i, m)][l];
          Rc[sy(i, j)] += wkl * s;
        }
      if (want_Q) {
        // 1/2 gammabar^ab d_k d_l gammabar_ab
        double c = 0.0;
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
          for (int b = 0; b < 3; b++) {
            const double ddgh = a == b ? 2.0 * (R.dS[a][k] * R.dS[a][l] + R.S[a] * R.ddS[a][k][l]) : 0.0;
            c += M.gbU[sy(a, b)] * (ddgh + ddeps[sy(a, b)]);
          }
        cQ[sy(k, l)] = 0.5 * c;
      }
    }
  if (want_Q) {
    // A_k = gammabar^-1 d_k gammabar
    double A[3][3][3];
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
      for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) {
          double s = 0.0;
#pragma unroll
          for (int c = 0; c < 3; c++) {
            const double dg = (c == b ? 2.0 * R.S[c] * R.dS[c][k] : 0.0) + M.deps[sy(c, b)][k];
            s += M.gbU[sy(a, c)] * dg;
          }
          A[k][a][b] = s;
        }
    double beta[3];
#pragma unroll
    for (int m = 0; m < 3; m++) beta[m] = P.at(G_VETU0 + m, 0, 0, 0) * R.iS[m];
#pragma unroll
    for (int k = 0; k < 3; k++) {
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < 3; m++) {
        double tr = 0.0;
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
          for (int b = 0; b < 3; b++) tr += A[k][a][b] * A[m][b][a];
        s += beta[m] * (cQ[sy(k, m)] - 0.5 * tr);
      }
      Q[k] = s;
    }
  }
}

}  // namespace bhah
