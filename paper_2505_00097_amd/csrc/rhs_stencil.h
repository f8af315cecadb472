// rhs_stencil.h -- the stencil building blocks shared by the right-hand-side
// kernels (one wave per tile in rhs_fused.hip, two waves per tile in
// rhs_pair.hip): upwinded advection and Kreiss-Oliger sums, the stencil
// gathers, the batched advection of several gridfunctions, and the tile walk.
#pragma once

#include "rhs_common.h"

namespace bhah {

// Upwinded advection beta^k d_k f of a rescaled gridfunction (Sec. 3: shift
// advection terms use the stencil shifted one point upwind). With
// sigma = sign(vet^k) and f(m) = f at offset m*sigma along k:
//   beta^k U_k f = |beta^k|/(den1 dxx^k) sum_{m != 1} up_m (f(m) - f(1)),
// m = -(R-1)..R+1; at 4th order
//   |beta^k|/(12 dxx^k) [3 (f(1) - f(-1)) + 10 (f(1) - f(0))
//                        - 6 (f(2) - f(1)) + (f(3) - f(1))].
template <int H>
struct UpwindT {
  unsigned vu[3][H];  // per-lane byte offsets of q + m s, m = 1..H (upwind side)
  unsigned vd[3][H];  // q - m s (downwind side; beyond R - 1 for dissipation only)
  unsigned v0;
  double w[3];        // |beta^k| / (den1 dxx^k)
};

// the upwinded sum for f(m), m = -(R-1)..R+1 in upwind orientation; at 4th
// order in the grouping written above
template <int R, class F>
__device__ __forceinline__ double upwind_f(const F& f) {
  if constexpr (R == 2) {
    const double fp = f(1), fm = f(-1), f2 = f(2), f0 = f(0), f3 = f(3);
    return 3.0 * (fp - fm) + 10.0 * (fp - f0) - 6.0 * (f2 - fp) + (f3 - fp);
  } else {
    const double f1 = f(1);
    double a = FdW<R>::up[0] * (f(1 - R) - f1);
#pragma unroll
    for (int m = 2 - R; m <= R + 1; m++)
      if (m != 1) a += FdW<R>::up[m + R - 1] * (f(m) - f1);
    return a;
  }
}

// upwinded stencil sum from centred values v[R + m] = f(m) and the value fu
// at (R+1) sigma; up selects the side (sigma = +1)
template <int R>
__device__ __forceinline__ double upwind_sum(const double (&v)[2 * R + 1], double fu, bool up) {
  auto f = [&](int m) { return m == R + 1 ? fu : (up ? v[R + m] : v[R - m]); };
  return upwind_f<R>(f);
}

// Kreiss-Oliger dissipation (Sec. 4.1): the difference of order 2(R+1)
// along each logical direction, weighted by eps/(kden dxx^k); at 4th order
// delta^6 f = f(3) + f(-3) - 6 (f(2) + f(-2)) + 15 (f(1) + f(-1)) - 20 f(0)
// over 64 dxx^k. Symmetric in the two sides, so the upwind-ordered stencil
// values serve as they are. fp[j], fm[j] are f(+-j), j = 1..R+1; the sums
// are taken as differences from f(0) (exact zero on constants, rounding
// of the size of the differences).
template <int R>
__device__ __forceinline__ double ko_sum(const double (&fp)[R + 2], const double (&fm)[R + 2], double f0) {
  double a = FdW<R>::ko[R + 1] * ((fp[R + 1] - f0) + (fm[R + 1] - f0));
#pragma unroll
  for (int j = R; j >= 1; j--) a += FdW<R>::ko[j] * ((fp[j] - f0) + (fm[j] - f0));
  return a;
}
// the same from centred values v (offsets -R..R) and the two outermost
template <int R>
__device__ __forceinline__ double ko_v(const double (&v)[2 * R + 1], double fu, double fd) {
  double fp[R + 2], fm[R + 2];
#pragma unroll
  for (int j = 1; j <= R; j++) { fp[j] = v[R + j]; fm[j] = v[R - j]; }
  fp[R + 1] = fu;
  fm[R + 1] = fd;
  fp[0] = fm[0] = v[R];
  return ko_sum<R>(fp, fm, v[R]);
}

#define BHAH_PHASE_BARRIER() __builtin_amdgcn_sched_barrier(0)

// Two-plane phi (AX): with exactly two interior phi planes the wrapped odd
// offsets land on the other plane and the even ones on the point's own, so
// a phi stencil reads two values, every centred phi first derivative and
// every mixed derivative involving phi vanishes identically (the grouped
// differences of equal values), and the upwinded phi stencil reduces to the
// two planes. The arithmetic on the values read is unchanged.

// axis gather along K; along phi on a two-plane grid only the two planes are
// read
template <int K, int PD, bool AX, class PT>
__device__ __forceinline__ void gather_axis_ax(const PT& P, int g, double (&v)[2 * PT::R + 1]) {
  if constexpr (AX && K == PD) {
    const double c = P.at(g, 0, 0, 0), o = P.template ax<K>(g, 1);
#pragma unroll
    for (int t = 0; t < 2 * PT::R + 1; t++) v[t] = ((t - PT::R) & 1) ? o : c;
  } else {
    gather_axis<K>(P, g, v);
  }
}

// compile-time dispatch of the gathers on a (compile-time after unrolling)
// direction index
template <int PD, bool AX, class PT>
__device__ __forceinline__ void gather_axis_k(const PT& P, int g, int k, double (&v)[2 * PT::R + 1]) {
  if (k == 0) gather_axis_ax<0, PD, AX>(P, g, v);
  else if (k == 1) gather_axis_ax<1, PD, AX>(P, g, v);
  else gather_axis_ax<2, PD, AX>(P, g, v);
}
// value R+1 points upwind along k (the last point of the shifted stencil),
// or, with the offsets of the other side, R+1 points downwind; on a
// two-plane grid R+1 is odd, the other plane
template <int PD, bool AX, class PT>
__device__ __forceinline__ double upwind_far(const PT& P, int g, int k, const unsigned (&vo)[3][PT::H],
                                             const double (&v)[2 * PT::R + 1]) {
  if (AX && k == PD) return v[PT::R - 1];
  return gf_ld(P.y, P.sgf, g, vo[k][PT::H - 1], 0);
}
template <class PT>
__device__ __forceinline__ void gather_cross_kl(const PT& P, int g, int k, int l, double (&v)[4 * PT::R * PT::R]) {
  if (k == 0 && l == 1) gather_cross<0, 1>(P, g, v);
  else if (k == 0) gather_cross<0, 2>(P, g, v);
  else gather_cross<1, 2>(P, g, v);
}

// upwinded advection of N gridfunctions in one batch of loads; with KO also
// their dissipation (strength eps[t], weights kw[k] = 1/(kden dxx^k))
template <int N, int PD, bool AX, bool KO, class PT>
__device__ __forceinline__ void advect_batch(const PT& P, const int (&gl)[N], const UpwindT<PT::H>& U,
                                             double (&out)[N], const double (&eps)[N], const double (&kw)[3]) {
  constexpr int H = PT::H, R = PT::R;
  constexpr int ND = KO ? H : R - 1;  // downwind points read
  double f0[N], fu[N][3][H + 1], fd[N][3][ND + 1];
#pragma unroll
  for (int t = 0; t < N; t++) {
    const int g = gl[t];
    f0[t] = gf_ld(P.y, P.sgf, g, U.v0, 0);
#pragma unroll
    for (int k = 0; k < 3; k++) {
      fu[t][k][1] = gf_ld(P.y, P.sgf, g, U.vu[k][0], 0);
      if (AX && k == PD) {  // two phi planes: odd offsets are the other plane, even ones this one
#pragma unroll
        for (int m = 2; m <= H; m++) fu[t][k][m] = (m & 1) ? fu[t][k][1] : f0[t];
#pragma unroll
        for (int m = 1; m <= ND; m++) fd[t][k][m] = (m & 1) ? fu[t][k][1] : f0[t];
      } else {  // in the order q - s, q + 2s .. q + Hs, then further downwind
        if constexpr (ND >= 1) fd[t][k][1] = gf_ld(P.y, P.sgf, g, U.vd[k][0], 0);
#pragma unroll
        for (int m = 2; m <= H; m++) fu[t][k][m] = gf_ld(P.y, P.sgf, g, U.vu[k][m - 1], 0);
#pragma unroll
        for (int m = 2; m <= ND; m++) fd[t][k][m] = gf_ld(P.y, P.sgf, g, U.vd[k][m - 1], 0);
      }
    }
  }
  BHAH_PHASE_BARRIER();
#pragma unroll
  for (int t = 0; t < N; t++) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 3; k++) {
      // f(m) for m = -(R-1)..R+1 in upwind orientation
      auto f = [&](int m) { return m == 0 ? f0[t] : (m > 0 ? fu[t][k][m] : fd[t][k][-m]); };
      s += U.w[k] * upwind_f<R>(f);
    }
    if constexpr (KO) {
      double d = 0.0;
#pragma unroll
      for (int k = 0; k < 3; k++) {
        double fp[R + 2], fm[R + 2];
#pragma unroll
        for (int j = 0; j <= H; j++) {
          fp[j] = j == 0 ? f0[t] : fu[t][k][j];
          fm[j] = j == 0 ? f0[t] : fd[t][k][j];
        }
        d += kw[k] * ko_sum<R>(fp, fm, f0[t]);
      }
      s += eps[t] * d;
    }
    out[t] = s;
  }
}

// Tiles: 64 points, 2^lx along i0 times 2^ly along i1 times 64 >> (lx + ly)
// along i2; the tile grid is walked in bands of `band` tile rows of i1, and
// within a band by i0 tile column, then i2, then i1 (fastest), so the tiles
// that run at the same time form a compact block of one column whose
// stencils overlap. The hardware hands consecutive workgroup ids to the XCDs
// in turn; block ids are remapped so that every XCD works through one
// contiguous range of the walk (its L2 then holds a compact part of the
// grid). On the 3-D grid the column-first order moves a third (4th order)
// to a quarter (8th order) of the HBM bytes of an i0-fastest order, at the
// same speed.
template <int H>
__device__ __forceinline__ bool tile_point(const GridDev& G, const TileMap& T, int w, int lane, int& i0,
                                           int& i1, int& i2) {
  const int full = T.band * T.tz * T.tx;  // tiles in one full band
  const int nb = (T.ty + T.band - 1) / T.band;
  int bi = w / full;
  if (bi > nb - 1) bi = nb - 1;
  const int start = bi * T.band;
  const int hgt = min(T.band, T.ty - start);
  const int idx = w - start * T.tz * T.tx;
  const int xt = idx / (hgt * T.tz);
  const int r = idx - xt * hgt * T.tz;
  const int j2 = r / hgt;
  const int j1 = start + (r - j2 * hgt);
  const int ex = 1 << T.lx, ey = 1 << T.ly;
  i0 = H + xt * ex + (lane & (ex - 1));
  i1 = H + j1 * ey + ((lane >> T.lx) & (ey - 1));
  i2 = H + (j2 << (6 - T.lx - T.ly)) + (lane >> (T.lx + T.ly));
  return i0 < H + G.N0 && i1 < H + G.N1 && i2 < H + G.N2;
}

// logical position in the walk of the tile a block works on; with G_blocks a
// multiple of the XCD count, block b runs on XCD b % nxcd
__device__ __forceinline__ int xcd_remap(int b, int per) { return (b % BHAH_NXCD) * per + b / BHAH_NXCD; }

}  // namespace bhah
