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

// two consecutive doubles stored with one 16-byte store, through the same
// descriptors as the loads
__device__ __forceinline__ void gf_st2(double* y, long long sgf, int g, unsigned voff, double lo, double hi) {
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc((void*)(y + (g >> 2) * 4 * sgf), (short)0, (int)(4 * sgf * 8), 0x00020000);
  const unsigned long long a = __builtin_bit_cast(unsigned long long, lo), b = __builtin_bit_cast(unsigned long long, hi);
  const bhah_u4 v = {(unsigned)a, (unsigned)(a >> 32), (unsigned)b, (unsigned)(b >> 32)};
  __builtin_amdgcn_raw_buffer_store_b128(v, r, voff, (g & 3) * (int)(sgf * 8), 0);
}

__device__ __forceinline__ double gf_ld(const double* y, long long sgf, int g, unsigned voff, int soff) {
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc((void*)(y + (g >> 2) * 4 * sgf), (short)0, (int)(4 * sgf * 8), 0x00020000);
  const bhah_u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff + (g & 3) * (int)(sgf * 8), 0);
  return __builtin_bit_cast(double, v);
}

// Finite-difference weights of order N_FD = 2R (Sec. 3: N_G = R + 1 ghost
// layers, the extra layer for the upwinded advection stencils), as integers
// over a common denominator, unit spacing:
//   D f  = sum_{j=1..R} d1[j] (f_j - f_-j) / den1
//   D2 f = (sum_{j=1..R} d2[j] (f_j + f_-j) + d2[0] f_0) / den2
//   U f  = sum_{m != 1} up[m + R - 1] (f_m - f_1) / den1, m = -(R-1)..R+1,
//          the centred stencil shifted one point upwind (offsets times the
//          sign of the shift component)
//   KO f = (sum_{j=1..R+1} ko[j] (f_j + f_-j) + ko[0] f_0) / kden, the
//          difference of order 2(R+1) scaled to the Fourier symbol
//          -sin^(2R+2)(theta/2) (Kreiss-Oliger dissipation of order 2R+1,
//          Sec. 4.1)
// R = 2: the 4th-order stencils; R = 4: the 8th-order ones of the
// production head-on run (Sec. 4.1).
template <int R>
struct FdW;
template <>
struct FdW<2> {
  static constexpr double d1[3] = {0.0, 8.0, -1.0}, den1 = 12.0;
  static constexpr double d2[3] = {-30.0, 16.0, -1.0}, den2 = 12.0;
  static constexpr double up[5] = {-3.0, -10.0, 18.0, -6.0, 1.0};
  static constexpr double ko[4] = {-20.0, 15.0, -6.0, 1.0}, kden = 64.0;
};
template <>
struct FdW<4> {
  static constexpr double d1[5] = {0.0, 672.0, -168.0, 32.0, -3.0}, den1 = 840.0;
  static constexpr double d2[5] = {-14350.0, 8064.0, -1008.0, 128.0, -9.0}, den2 = 5040.0;
  static constexpr double up[9] = {-5.0, 60.0, -420.0, -378.0, 1050.0, -420.0, 140.0, -30.0, 3.0};
  static constexpr double ko[6] = {-252.0, 210.0, -120.0, 45.0, -10.0, 1.0}, kden = 1024.0;
};

// Stencil access around one point, H = N_G ghost layers (stencil radius up
// to H). Stencil values are read with raw buffer loads: the per-lane part of
// the byte offset goes in the vector offset, the part shared by the wave in
// the scalar offset. The periodic direction phi (i1 on SinhCylindrical
// grids, i2 on spherical ones) is read with the index wrapped onto the
// interior planes, so phi ghost points are never read: they are exact copies
// of those planes (periodicity, no parity change), and the values read are
// identical. The phi index must be the same for every lane of the wave (tile
// extent 1 along phi).
template <int H_>
struct PtT {
  static constexpr int H = H_, R = H_ - 1;
  const double* __restrict__ y;
  long long sgf;
  int pd;            // periodic direction (1 or 2)
  int se;            // stride of the other transverse direction
  unsigned vb;       // per-lane byte offset of (i0 - H, i_e - H) with the phi index removed
  int sw[2 * H + 1];  // byte offsets of the wrapped phi planes at offsets -H..H (wave-uniform)

  __device__ __forceinline__ PtT(const double* y_, const GridDev& G, int C, int i0, int i1, int i2)
      : y(y_), sgf(G.sgf) {
    pd = C == BHAH_SINH_CYLINDRICAL ? 1 : 2;
    const int sd = pd == 1 ? G.s1 : G.s2;
    const int nd = pd == 1 ? G.N1 : G.N2;
    se = pd == 1 ? G.s2 : G.s1;
    const int ie = pd == 1 ? i2 : i1;
    const int id = __builtin_amdgcn_readfirstlane((pd == 1 ? i1 : i2) - H);
    vb = (unsigned)(i0 - H + se * (ie - H)) * 8u;
#pragma unroll
    for (int o = -H; o <= H; o++) {
      int x = id + o;
      if constexpr (H == 3) {  // nd >= 2: two corrections each way suffice
        x += x < 0 ? nd : 0;
        x += x < 0 ? nd : 0;
        x -= x >= nd ? nd : 0;
        x -= x >= nd ? nd : 0;
      } else {
        x %= nd;
        x += x < 0 ? nd : 0;
      }
      sw[o + H] = (H + x) * sd * 8;
    }
  }

  // value at offsets (a, b, c) along (i0, i1, i2)
  __device__ __forceinline__ double at(int g, int a, int b, int c) const {
    const int od = pd == 1 ? b : c, oe = pd == 1 ? c : b;
    return gf_ld(y, sgf, g, vb + (unsigned)((a + H) * 8), sw[od + H] + (oe + H) * se * 8);
  }
  // values at offsets (a, b, c) and (a + 1, b, c)
  __device__ __forceinline__ void at2(int g, int a, int b, int c, double& lo, double& hi) const {
    const int od = pd == 1 ? b : c, oe = pd == 1 ? c : b;
    gf_ld2(y, sgf, g, vb + (unsigned)((a + H) * 8), sw[od + H] + (oe + H) * se * 8, lo, hi);
  }
  // byte offset of the point shifted by m along the periodic direction
  __device__ __forceinline__ unsigned vper(int m) const {
    return vb + (unsigned)(H * 8) + (unsigned)(H * se * 8 + sw[m + H]);
  }
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

// 1/(den1 dxx^k), 1/(den2 dxx^k^2), 1/(den1^2 dxx^k dxx^l) for order 2R
struct Spacing {
  double d1s[3];
  double d2s[3];
  double crs[3][3];
};

template <int R>
__device__ __forceinline__ Spacing make_spacing(const GridDev& G) {
  Spacing s;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    s.d1s[k] = G.inv_dx[k] * (1.0 / FdW<R>::den1);
    s.d2s[k] = G.inv_dx[k] * G.inv_dx[k] * (1.0 / FdW<R>::den2);
  }
#pragma unroll
  for (int k = 0; k < 3; k++)
#pragma unroll
    for (int l = 0; l < 3; l++) s.crs[k][l] = G.inv_dx[k] * G.inv_dx[l] * (1.0 / (FdW<R>::den1 * FdW<R>::den1));
  return s;
}

// ---- centred finite differences (Sec. 3) on gathered values:
//   axis : v[R + m] = f(m) along one direction, m = -R..R
//   cross: v[2R a + b] = f(m_a, n_b) for m, n in {-R..-1, 1..R}, a-major
// Sums are grouped into differences: first differences pair f(j) with
// f(-j), second differences take f(j) - f(0) and f(-j) - f(0) before any
// weight. Constant fields then have exactly zero derivatives, and the
// subtractions of nearby values are exact, so the rounding error stays of
// the size of the differences rather than of |f| / h^2 (an ungrouped
// 16 (f1 + f-1) - (f2 + f-2) - 30 f0 loses about 30 eps |f| / h^2 where f
// is nearly constant, far above 1e-12 of the result on fine sinh cells).
template <int R>
__device__ __forceinline__ double d1_axis(const double (&v)[2 * R + 1], double s) {
  double a = FdW<R>::d1[1] * (v[R + 1] - v[R - 1]);
#pragma unroll
  for (int j = 2; j <= R; j++) a += FdW<R>::d1[j] * (v[R + j] - v[R - j]);
  return a * s;
}
template <int R>
__device__ __forceinline__ double d2_axis(const double (&v)[2 * R + 1], double s) {
  double a = FdW<R>::d2[1] * ((v[R + 1] - v[R]) + (v[R - 1] - v[R]));
#pragma unroll
  for (int j = 2; j <= R; j++) a += FdW<R>::d2[j] * ((v[R + j] - v[R]) + (v[R - j] - v[R]));
  return a * s;
}
// index of offset m (m != 0) in a cross-stencil row
template <int R>
__host__ __device__ constexpr int xo(int m) { return m < 0 ? m + R : m + R - 1; }
template <int R>
__device__ __forceinline__ double d2_cross(const double (&v)[4 * R * R], double s) {
  auto e = [&](int a) {
    double t = FdW<R>::d1[1] * (v[2 * R * a + xo<R>(1)] - v[2 * R * a + xo<R>(-1)]);
#pragma unroll
    for (int j = 2; j <= R; j++) t += FdW<R>::d1[j] * (v[2 * R * a + xo<R>(j)] - v[2 * R * a + xo<R>(-j)]);
    return t;
  };
  double t = FdW<R>::d1[1] * (e(xo<R>(1)) - e(xo<R>(-1)));
#pragma unroll
  for (int j = 2; j <= R; j++) t += FdW<R>::d1[j] * (e(xo<R>(j)) - e(xo<R>(-j)));
  return t * s;
}

// Batched stencil gathers: values land in a local array first so that a
// whole batch of loads is in flight before any is consumed.
template <int K, class PT>
__device__ __forceinline__ void gather_axis(const PT& P, int g, double (&v)[2 * PT::R + 1]) {
  constexpr int R = PT::R;
  if constexpr (K == 0) {  // i0 neighbours are adjacent in memory: pairs per load
#pragma unroll
    for (int m = -R; m < 0; m += 2) P.at2(g, m, 0, 0, v[R + m], v[R + m + 1]);
    v[R] = P.at(g, 0, 0, 0);
#pragma unroll
    for (int m = 1; m <= R; m += 2) P.at2(g, m, 0, 0, v[R + m], v[R + m + 1]);
  } else {
#pragma unroll
    for (int t = 0; t < 2 * R + 1; t++) v[t] = P.template ax<K>(g, t - R);
  }
}
template <int K, int L, class PT>
__device__ __forceinline__ void gather_cross(const PT& P, int g, double (&v)[4 * PT::R * PT::R]) {
  constexpr int R = PT::R, W = 2 * R;
  if constexpr (K == 0) {  // rows along i0 in pairs per load
#pragma unroll
    for (int b = 0; b < W; b++) {
      const int n = b < R ? b - R : b - R + 1;
      const int o1 = L == 1 ? n : 0, o2 = L == 2 ? n : 0;
#pragma unroll
      for (int m = -R; m < 0; m += 2) P.at2(g, m, o1, o2, v[W * xo<R>(m) + b], v[W * xo<R>(m + 1) + b]);
#pragma unroll
      for (int m = 1; m <= R; m += 2) P.at2(g, m, o1, o2, v[W * xo<R>(m) + b], v[W * xo<R>(m + 1) + b]);
    }
  } else {
#pragma unroll
    for (int a = 0; a < W; a++)
#pragma unroll
      for (int b = 0; b < W; b++)
        v[W * a + b] = P.template pl<K, L>(g, a < R ? a - R : a - R + 1, b < R ? b - R : b - R + 1);
  }
}

template <int K, class PT>
__device__ __forceinline__ double fd1(const PT& P, int g, const Spacing& s) {
  double v[2 * PT::R + 1];
#pragma unroll
  for (int t = 0; t < 2 * PT::R + 1; t++) v[t] = P.template ax<K>(g, t - PT::R);
  return d1_axis<PT::R>(v, s.d1s[K]);
}
template <int K, class PT>
__device__ __forceinline__ double fd2(const PT& P, int g, const Spacing& s) {
  double v[2 * PT::R + 1];
#pragma unroll
  for (int t = 0; t < 2 * PT::R + 1; t++) v[t] = P.template ax<K>(g, t - PT::R);
  return d2_axis<PT::R>(v, s.d2s[K]);
}
template <int K, int L, class PT>
__device__ __forceinline__ double fdm(const PT& P, int g, const Spacing& s) {
  // D_K D_L f; the inner differences are left unnormalised
  double v[4 * PT::R * PT::R];
#pragma unroll
  for (int a = 0; a < 2 * PT::R; a++)
#pragma unroll
    for (int b = 0; b < 2 * PT::R; b++)
      v[2 * PT::R * a + b] =
          P.template pl<K, L>(g, a < PT::R ? a - PT::R : a - PT::R + 1, b < PT::R ? b - PT::R : b - PT::R + 1);
  return d2_cross<PT::R>(v, s.crs[K][L]);
}

template <class PT>
__device__ __forceinline__ double fd1k(const PT& P, int g, int k, const Spacing& s) {
  return k == 0 ? fd1<0>(P, g, s) : (k == 1 ? fd1<1>(P, g, s) : fd1<2>(P, g, s));
}
// second derivative d_k d_l (any order of k, l)
template <class PT>
__device__ __forceinline__ double fd2kl(const PT& P, int g, int k, int l, const Spacing& s) {
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
template <class PT>
__device__ __forceinline__ void metric_first(const PT& P, const Ref& R, const double Gh[3][3][3],
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
template <int C, class PT>
__device__ __forceinline__ void ricci_and_Q(const PT& P, const Ref& R, const double Gh[3][3][3],
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
