// rhs_fused.hip -- the full BSSN + gauge right-hand side (Eqs. 7-15 with the
// conformal Ricci tensor of Eq. 12, arXiv:2505.00097) in one kernel, one
// thread per interior point, with the RK4 stage combination as epilogue.
//
// The per-point work is ordered to keep few values live at a time; values
// needed by a later phase wait in a per-lane LDS park.
//   phase 0  point values, the conformal metric and its inverse, the upwind
//            stencil offsets
//   phase 1  stencil loop over the six index pairs (k,l) of h_ij, W, alpha
//            and vet^i: every second derivative is consumed at once into the
//            contractions the equations need (22 accumulators):
//              P_ij  = sum_kl gammabar^kl d_k d_l h_ij            (Ricci)
//              Qs_k  = sum_m beta^m gammabar^ab S_a S_b d_k d_m h_ab
//              Y_kl  = (alpha/W) d_k d_l W - d_k d_l alpha         (Abar eq.)
//              Za    = gammabar^kl d_k d_l alpha                   (K eq.)
//              Bv^i  = gammabar^kl d_k d_l vet^i, Bd_k = sum_j d_k d_j vet^j / S_j
//            the diagonal gathers also give these gridfunctions' first
//            derivatives and upwinded advection terms
//   phase 2  the metric pieces (Eqs. 3-5), the Ricci tensor (Eq. 12), Delta
//            terms; lambda^i's derivatives and advection
//   phase 3  the remaining advection, then Eqs. 7-15 and the rescaling
//   epilogue the right-hand side, or the RK stage combination
// Stencil values are loaded in batches of up to about 64 ahead of the
// arithmetic that uses them. Reference-metric structural zeros fold away per
// coordinate family.
#include "rhs_stencil.h"

namespace bhah {

// LDS slots per thread for values carried from one phase to a later one, and
// for the 24 results: they are written to global memory only at the end, so
// no global store sits between two stencil loads (the compiler would have to
// keep such loads and stores in order, exposing memory latency each time).
constexpr int PARK = 78;
// PK_DH (first derivatives of h_ij, 18 slots) shares the result slots of
// gridfunctions 0-17: it is written in phase 1 and read in phase 2, before
// phase 3 writes results. PK_D1 holds d_k vet^i (9), d_k W (3) and d_k alpha
// (3) from phase 1 to 3; PK_ADV the advection terms of h_ij (6), W and alpha
// formed in phase 1 (those of vet^i go straight to their result slots,
// which PK_DH does not cover). 78 slots x 64 lanes x 8 B = 39 KB per wave:
// four waves still fit one CU's 160 KB.
enum { PK_PC = 0, PK_QS = 6, PK_Y = 9, PK_ZA = 15, PK_BV = 16, PK_BD = 19, PK_RT = 22, PK_Q = 28, PK_OUT = 31,
       PK_DH = PK_OUT, PK_D1 = 55, PK_ADV = 70 };
static_assert(PK_ADV + 8 == PARK && PK_DH + 18 <= PK_OUT + G_VETU0, "park layout");

// Phase 1 through an LDS stage, on grids with two phi planes and tiles of
// 64 points along i0. The CU's vector memory address unit takes about the
// same time for every load instruction of a wave, whatever its width, so the
// per-lane stencil gathers (one or two values per instruction) keep it busy
// while the SIMDs wait. Here the wave brings in, for one gridfunction at a
// time, the values its stencils read on the tile's own phi plane -- rows
// -H..H along the other transverse direction e, columns -H..63+H along i0 --
// with a few 16-byte loads shared by the whole wave, and every stencil value
// then comes from LDS. The stage takes the park slots that phase 1 writes
// only at its end (0..30); gridfunctions go in batches that fit there, the
// next batch's loads in flight while the current one is worked. Every
// accumulation takes the same terms in the same order as the pair-by-pair
// loop, each as an explicit fused multiply-add (left to itself, the compiler
// may fuse either product of a sum of two), so the results are bitwise the
// same.
template <int H>
struct StageGeom {
  static constexpr int RL = 64 + 2 * H;                  // doubles per stage row
  static constexpr int NP = (2 * H + 1) * RL / 2;        // 16-byte pieces per gridfunction
  static constexpr int NR = (NP + 63) / 64;              // pieces per lane
  static constexpr int PER = (31 * 64 * 8) / (NP * 16);  // gridfunctions per batch (at most)
};

// The same on grids with more than two phi planes, for the mixed pairs
// (0, l), l = 1, 2: the 2R rows a gridfunction's stencil reads along l
// (offsets -R..-1, 1..R, in that order), columns -R..63+R along i0.
template <int H>
struct CrossGeom {
  static constexpr int R = H - 1;
  static constexpr int RL = 64 + 2 * R;              // doubles per stage row
  static constexpr int NP = R * RL;                  // 16-byte pieces per gridfunction
  static constexpr int NR = (NP + 63) / 64;          // pieces per lane
  static constexpr int PER = H == 3 ? 6 : 2;         // gridfunctions per batch
  static_assert(PER * NP * 2 <= PK_OUT * 64, "the stage must stay below the slots phase 1 writes");
};

template <int C, bool KO, int H>
__device__ __forceinline__ void phase1_staged(const PtT<H>& P, const Gauge& ga, const Spacing& sp, const Ref& R,
                                              const UpwindT<H>& U, const double (&vet)[3], const double (&beta)[3],
                                              const double (&gbU)[6], const double (&SS)[6], const double (&kw)[3],
                                              double aW, double* __restrict__ stage, double* __restrict__ park,
                                              int lane, double (&Pc)[6], double (&Qs)[3], double (&Y)[6],
                                              double& Za, double (&Bv)[3], double (&Bd)[3], double (&adv)[11]) {
  constexpr int PD = C == BHAH_SINH_CYLINDRICAL ? 1 : 2;  // phi
  constexpr int E = 3 - PD;                               // the other transverse direction
  constexpr int RR = H - 1, SW = 2 * RR + 1, XW = 2 * RR;
  using SG = StageGeom<H>;
  // two gridfunctions per batch at 4th order and one at 8th: faster than
  // the four and two that fit (and two spill at 8th order with dissipation)
  constexpr int RL = SG::RL, NP = SG::NP, NR = SG::NR, PER = H == 3 ? 2 : 1;
  constexpr int NB = (11 + PER - 1) / PER;
  static_assert(PER * NP * 2 <= PK_OUT * 64, "the stage must stay below the slots phase 1 writes");
  constexpr int G11[11] = {G_HDD00, G_HDD00 + 1, G_HDD00 + 2, G_HDD00 + 3, G_HDD00 + 4, G_HDD00 + 5,
                           G_CF, G_ALPHA, G_VETU0, G_VETU0 + 1, G_VETU0 + 2};
  auto put = [&](int v, double x) { park[v * 64] = x; };

  // piece r*64 + lane of a gridfunction's stage (the last ones repeated to
  // fill the last load): its byte offset from the tile's first column
  const unsigned vb0 = __builtin_amdgcn_readfirstlane(P.vb);  // lane 0 is never clamped
  unsigned voff[NR];
  int poff[NR];
#pragma unroll
  for (int r = 0; r < NR; r++) {
    const int p = min(r * 64 + lane, NP - 1);
    const int row = p / (RL / 2), col = 2 * (p - row * (RL / 2));
    voff[r] = vb0 + (unsigned)((col + row * P.se) * 8);
    poff[r] = 2 * p;
  }
  const int soff = P.sw[H];  // the tile's own phi plane

  double G2[6];  // gammabar^ab S_a S_b, doubled off the diagonal
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = a; b < 3; b++) G2[sy(a, b)] = (a == b ? 1.0 : 2.0) * gbU[sy(a, b)] * SS[sy(a, b)];
  double ck[6], ddW[6];
#pragma unroll
  for (int a = 0; a < 6; a++) ck[a] = 0.0;

  const bool up0 = vet[0] > 0.0, upE = vet[E] > 0.0;
  const int fu0 = up0 ? H : -H, fuE = upE ? H * RL : -H * RL;  // upwind far points
  double nlo[PER][NR], nhi[PER][NR], nph[PER];
  auto issue = [&](int b) {
#pragma unroll
    for (int t = 0; t < PER; t++)
      if (b * PER + t < 11) {
        const int g = G11[b * PER + t];
#pragma unroll
        for (int r = 0; r < NR; r++) gf_ld2(P.y, P.sgf, g, voff[r], soff, nlo[t][r], nhi[t][r]);
        nph[t] = P.template ax<PD>(g, 1);  // the other phi plane
      }
  };
  issue(0);
#pragma unroll
  for (int b = 0; b < NB; b++) {
    double oph[PER];
#pragma unroll
    for (int t = 0; t < PER; t++)
      if (b * PER + t < 11) {
#pragma unroll
        for (int r = 0; r < NR; r++) {
          stage[t * 2 * NP + poff[r]] = nlo[t][r];
          stage[t * 2 * NP + poff[r] + 1] = nhi[t][r];
        }
        oph[t] = nph[t];
      }
    if (b + 1 < NB) issue(b + 1);
    BHAH_PHASE_BARRIER();
#pragma unroll
    for (int t = 0; t < PER; t++) {
      const int tt = b * PER + t;
      if (tt >= 11) continue;
      const double* F = stage + t * 2 * NP + H * RL + H + lane;  // this point's value
      auto at = [&](int de, int d0) { return F[de * RL + d0]; };
      double v0[SW], vE[SW], vP[SW], vx[XW * XW];
#pragma unroll
      for (int m = -RR; m <= RR; m++) {
        v0[RR + m] = at(0, m);
        vE[RR + m] = at(m, 0);
      }
#pragma unroll
      for (int m = 0; m < SW; m++) vP[m] = ((m - RR) & 1) ? oph[t] : v0[RR];
#pragma unroll
      for (int a = 0; a < XW; a++)
#pragma unroll
        for (int c = 0; c < XW; c++) vx[XW * a + c] = at(c < RR ? c - RR : c - RR + 1, a < RR ? a - RR : a - RR + 1);
      const double far0 = F[fu0], farE = F[fuE];
      double near0 = 0.0, nearE = 0.0;
      if constexpr (KO) {
        near0 = F[-fu0];
        nearE = F[-fuE];
      }
      // diagonal pairs in the order k = 0, 1, 2: advection, first derivative
#pragma unroll
      for (int k = 0; k < 3; k++) {
        const double(&vk)[SW] = k == 0 ? v0 : (k == PD ? vP : vE);
        const double fu = k == 0 ? far0 : (k == PD ? vP[RR - 1] : farE);
        const bool up = vet[k] > 0.0;
        adv[tt] = fma(U.w[k], upwind_sum<RR>(vk, fu, up), adv[tt]);
        if constexpr (KO) {
          const double fd = k == 0 ? near0 : (k == PD ? vP[RR - 1] : nearE);
          adv[tt] = fma((tt < 7 ? ga.dm : ga.dg) * kw[k], ko_v<RR>(vk, fu, fd), adv[tt]);
        }
        const double d1 = k == PD ? 0.0 : d1_axis<RR>(vk, sp.d1s[k]);
        const int slot =
            tt < 6 ? PK_DH + 3 * tt : (tt == 6 ? PK_D1 + 9 : (tt == 7 ? PK_D1 + 12 : PK_D1 + 3 * (tt - 8)));
        put(slot + k, d1);
      }
      const double dd00 = d2_axis<RR>(v0, sp.d2s[0]), ddPP = d2_axis<RR>(vP, sp.d2s[PD]);
      const double ddEE = d2_axis<RR>(vE, sp.d2s[E]), dd0E = d2_cross<RR>(vx, sp.crs[0][E]);
      // the pairs (k, l) in the loop's order; those with a phi index vanish
#pragma unroll
      for (int k = 0; k < 3; k++)
#pragma unroll
        for (int l = k; l < 3; l++) {
          const int kl = sy(k, l);
          if (k != l && (k == PD || l == PD)) {
            if (tt == 7) Y[kl] = 0.0;
            continue;
          }
          const double dd = k != l ? dd0E : (k == 0 ? dd00 : (k == PD ? ddPP : ddEE));
          const double wg = (k == l ? 1.0 : 2.0) * gbU[kl];
          if (tt < 6) {
            Pc[tt] = fma(wg, dd, Pc[tt]);
            ck[kl] = fma(G2[tt], dd, ck[kl]);
          } else if (tt == 6) {
            ddW[kl] = dd;
          } else if (tt == 7) {
            Y[kl] = fma(aW, ddW[kl], -dd);
            Za = fma(wg, dd, Za);
          } else {
            const int i = tt - 8;
            Bv[i] = fma(wg, dd, Bv[i]);
            if (i == l) Bd[k] = fma(dd, R.iS[l], Bd[k]);
            if (k != l && i == k) Bd[l] = fma(dd, R.iS[k], Bd[l]);
          }
        }
    }
  }
#pragma unroll
  for (int k = 0; k < 3; k++)
#pragma unroll
    for (int l = k; l < 3; l++) {
      if (k != l && (k == PD || l == PD)) continue;
      const double c = ck[sy(k, l)];
      Qs[k] = fma(beta[l], c, Qs[k]);
      if (k != l) Qs[l] = fma(beta[k], c, Qs[l]);
    }
}

// MIX: the epilogue also handles stages that mix two states (SSPRK3); the
// ensemble kernel is built with it only for SSPRK3 batches (keeping the
// two-state path out of RK4 stages saves registers there).
// H: ghost layers N_G; the differences are of order 2(H-1) (3: 4th order,
// 5: 8th order).
// STG: phase 1 through the LDS stage (tiles of 64 points along i0): every
// stencil of phase 1 on two-phi-plane grids, the mixed pairs (0, l)
// otherwise. Every lane of the wave takes part, and a lane whose point lies
// past the grid (live false) computes a clamped point and stores nothing.
template <int C, bool AX, bool KO, bool MIX, int H, bool STG = false>
__device__ __forceinline__ void fused_point(const GridDev& G, const Gauge& ga, const double* __restrict__ y,
                                            const StageArgs& st, int i0, int i1, int i2, unsigned q,
                                            double* __restrict__ aux, double* __restrict__ park, bool live = true) {
  constexpr int PD = C == BHAH_SINH_CYLINDRICAL ? 1 : 2;  // the periodic (phi) direction
  constexpr int RR = H - 1, SW = 2 * RR + 1;               // stencil radius and width
  const double eta = ga.eta;
  double kw[3];  // dissipation weights 1/(kden dxx^k)
#pragma unroll
  for (int k = 0; k < 3; k++) kw[k] = G.inv_dx[k] * (1.0 / FdW<RR>::kden);
  // park[v * 64] is this thread's slot v (lane-consecutive, bank-conflict free)
  auto put = [&](int v, double x) { park[v * 64] = x; };
  auto get = [&](int v) { return park[v * 64]; };
  const PtT<H> P(y, G, C, i0, i1, i2);
  const Spacing sp = make_spacing<RR>(G);
  Ref R;
  load_ref<C>(G, i0, i1, i2, R);
  // staged mixed pairs (general grids): per lane and load, the byte offset
  // of its piece of row xo(n) for l = 1, 2, and the piece's LDS index
  using CG = CrossGeom<H>;
  unsigned cvo[2][CG::NR];
  int cpo[CG::NR];
  if constexpr (STG && !AX) {
    const int lane = (int)(threadIdx.x & 63);
    const unsigned vb0 = __builtin_amdgcn_readfirstlane(P.vb);  // lane 0 is never clamped
    const int sd = PD == 1 ? G.s1 : G.s2, nd = PD == 1 ? G.N1 : G.N2;
    const int id = __builtin_amdgcn_readfirstlane((PD == 1 ? i1 : i2) - H);
#pragma unroll
    for (int r = 0; r < CG::NR; r++) {
      const int p = min(r * 64 + lane, CG::NP - 1);
      const int row = p / (CG::RL / 2), col = 2 * (p - row * (CG::RL / 2));
      const int n = row < RR ? row - RR : row - RR + 1;
      cpo[r] = 2 * p;
      const unsigned base = vb0 + (unsigned)((col - RR + H) * 8);
#pragma unroll
      for (int li = 0; li < 2; li++) {
        int off;
        if (li + 1 == PD) {  // rows on the wrapped phi planes, as the accessor wraps them
          int x = id + n;
          if constexpr (H == 3) {
            x += x < 0 ? nd : 0;
            x += x < 0 ? nd : 0;
            x -= x >= nd ? nd : 0;
            x -= x >= nd ? nd : 0;
          } else {
            x %= nd;
            x += x < 0 ? nd : 0;
          }
          off = (H + x) * sd * 8 + H * P.se * 8;
        } else {
          off = P.sw[H] + (n + H) * P.se * 8;
        }
        cvo[li][r] = base + (unsigned)off;
      }
    }
  }

  // ---- phase 0: point values and the conformal metric (Eq. 3) -----------
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
  const double W = P.at(G_CF, 0, 0, 0), alpha = P.at(G_ALPHA, 0, 0, 0);
  const double iW = 1.0 / W;
  double vet[3], beta[3];
#pragma unroll
  for (int i = 0; i < 3; i++) {
    vet[i] = P.at(G_VETU0 + i, 0, 0, 0);
    beta[i] = vet[i] * R.iS[i];
  }

  // upwind stencil offsets (shift one point towards the side vet^k points to)
  UpwindT<H> U;
  U.v0 = q * 8u;
  {
    const int str[3] = {1, G.s1, G.s2};
#pragma unroll
    for (int k = 0; k < 3; k++) {
      const int s = vet[k] > 0.0 ? 1 : -1;
      // in the order q + s, q - s, q + 2s .. q + Hs, q - 2s .. q - Hs
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

  // ---- phase 1: second-derivative contractions ---------------------------
  double Pc[6], Qs[3], Y[6], Za = 0.0, Bv[3], Bd[3], adv[11];
#pragma unroll
  for (int t = 0; t < 11; t++) adv[t] = 0.0;
#pragma unroll
  for (int a = 0; a < 6; a++) Pc[a] = 0.0;
#pragma unroll
  for (int i = 0; i < 3; i++) { Qs[i] = 0.0; Bv[i] = 0.0; Bd[i] = 0.0; }
  if constexpr (STG && AX) {
    const int lane = (int)(threadIdx.x & 63);
    phase1_staged<C, KO, H>(P, ga, sp, R, U, vet, beta, gbU, SS, kw, alpha * iW, park - lane, park, lane, Pc,
                            Qs, Y, Za, Bv, Bd, adv);
  } else {
    double G2[6];  // gammabar^ab S_a S_b, doubled off the diagonal
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
      for (int b = a; b < 3; b++) G2[sy(a, b)] = (a == b ? 1.0 : 2.0) * gbU[sy(a, b)] * SS[sy(a, b)];
    const double aW = alpha * iW;
    // the 11 gridfunctions whose second derivatives enter: h_ij, W, alpha, vet^i
    constexpr int G11[11] = {G_HDD00, G_HDD00 + 1, G_HDD00 + 2, G_HDD00 + 3, G_HDD00 + 4, G_HDD00 + 5,
                             G_CF, G_ALPHA, G_VETU0, G_VETU0 + 1, G_VETU0 + 2};
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
      for (int l = k; l < 3; l++) {
        double dd[11];
        if (k == l) {
          // f(-R..R) along k, and f((R+1) s) on the upwind side for the
          // advection; at 8th order in batches of four gridfunctions
          constexpr int TB = H == 3 ? 11 : 4;
#pragma unroll
          for (int t0 = 0; t0 < 11; t0 += TB) {
            double v[TB][SW], fu[TB], fd[KO ? TB : 1];
#pragma unroll
            for (int t = 0; t < TB; t++)
              if (t0 + t < 11) {
                gather_axis_k<PD, AX>(P, G11[t0 + t], k, v[t]);
                fu[t] = upwind_far<PD, AX>(P, G11[t0 + t], k, U.vu, v[t]);
                if constexpr (KO) fd[t] = upwind_far<PD, AX>(P, G11[t0 + t], k, U.vd, v[t]);
              }
            BHAH_PHASE_BARRIER();
            const bool up = vet[k] > 0.0;
#pragma unroll
            for (int t = 0; t < TB; t++)
              if (t0 + t < 11) {
                const int tt = t0 + t;
                adv[tt] = fma(U.w[k], upwind_sum<RR>(v[t], fu[t], up), adv[tt]);
                // h_ij and W take the metric strength, alpha and vet^i the gauge one
                if constexpr (KO)
                  adv[tt] = fma((tt < 7 ? ga.dm : ga.dg) * kw[k], ko_v<RR>(v[t], fu[t], fd[t]), adv[tt]);
              }
#pragma unroll
            for (int t = 0; t < TB; t++)
              if (t0 + t < 11) dd[t0 + t] = d2_axis<RR>(v[t], sp.d2s[k]);
            // the same stencil values give the first derivatives along k
#pragma unroll
            for (int t = 0; t < TB; t++)
              if (t0 + t < 11) {
                const int tt = t0 + t;
                const double d1 = AX && k == PD ? 0.0 : d1_axis<RR>(v[t], sp.d1s[k]);
                const int slot =
                    tt < 6 ? PK_DH + 3 * tt : (tt == 6 ? PK_D1 + 9 : (tt == 7 ? PK_D1 + 12 : PK_D1 + 3 * (tt - 8)));
                put(slot + k, d1);
              }
          }
        } else if (AX && (k == PD || l == PD)) {
#pragma unroll
          for (int t = 0; t < 11; t++) dd[t] = 0.0;
        } else if (STG && !AX && k == 0) {
          // rows along l through the LDS stage (park slots 0..30, free in phase 1)
          const int lane = (int)(threadIdx.x & 63), li = l - 1;
          double* stg = park - lane;
#pragma unroll
          for (int t0 = 0; t0 < 11; t0 += CG::PER) {
            double lo[CG::PER][CG::NR], hi[CG::PER][CG::NR];
#pragma unroll
            for (int t = 0; t < CG::PER; t++)
              if (t0 + t < 11) {
#pragma unroll
                for (int r = 0; r < CG::NR; r++) gf_ld2(P.y, P.sgf, G11[t0 + t], cvo[li][r], 0, lo[t][r], hi[t][r]);
              }
#pragma unroll
            for (int t = 0; t < CG::PER; t++)
              if (t0 + t < 11) {
#pragma unroll
                for (int r = 0; r < CG::NR; r++) {
                  stg[t * 2 * CG::NP + cpo[r]] = lo[t][r];
                  stg[t * 2 * CG::NP + cpo[r] + 1] = hi[t][r];
                }
              }
            BHAH_PHASE_BARRIER();
#pragma unroll
            for (int t = 0; t < CG::PER; t++)
              if (t0 + t < 11) {
                const double* F = stg + t * 2 * CG::NP + RR + lane;  // row 0, this point's column
                double v[4 * RR * RR];
#pragma unroll
                for (int a = 0; a < 2 * RR; a++)
#pragma unroll
                  for (int b = 0; b < 2 * RR; b++) v[2 * RR * a + b] = F[b * CG::RL + (a < RR ? a - RR : a - RR + 1)];
                dd[t0 + t] = d2_cross<RR>(v, sp.crs[k][l]);
              }
            BHAH_PHASE_BARRIER();
          }
        } else {
          constexpr int TX = H == 3 ? 4 : 1;  // gridfunctions per batch of cross loads
#pragma unroll
          for (int t0 = 0; t0 < 11; t0 += TX) {
            double v[TX][4 * RR * RR];
#pragma unroll
            for (int t = 0; t < TX; t++)
              if (t0 + t < 11) gather_cross_kl(P, G11[t0 + t], k, l, v[t]);
            BHAH_PHASE_BARRIER();
#pragma unroll
            for (int t = 0; t < TX; t++)
              if (t0 + t < 11) dd[t0 + t] = d2_cross<RR>(v[t], sp.crs[k][l]);
          }
        }
        const int kl = sy(k, l);
        const double wg = (k == l ? 1.0 : 2.0) * gbU[kl];
        double c = 0.0;
#pragma unroll
        for (int a = 0; a < 6; a++) {
          Pc[a] = fma(wg, dd[a], Pc[a]);
          c = fma(G2[a], dd[a], c);
        }
        Qs[k] = fma(beta[l], c, Qs[k]);
        if (k != l) Qs[l] = fma(beta[k], c, Qs[l]);
        Y[kl] = fma(aW, dd[6], -dd[7]);
        Za = fma(wg, dd[7], Za);
#pragma unroll
        for (int i = 0; i < 3; i++) {
          Bv[i] = fma(wg, dd[8 + i], Bv[i]);
          if (i == l) Bd[k] = fma(dd[8 + i], R.iS[l], Bd[k]);
          if (k != l && i == k) Bd[l] = fma(dd[8 + i], R.iS[k], Bd[l]);
        }
      }
  }
#pragma unroll
  for (int a = 0; a < 6; a++) { put(PK_PC + a, Pc[a]); put(PK_Y + a, Y[a]); }
#pragma unroll
  for (int i = 0; i < 3; i++) { put(PK_QS + i, Qs[i]); put(PK_BV + i, Bv[i]); put(PK_BD + i, Bd[i]); }
  put(PK_ZA, Za);
#pragma unroll
  for (int t = 0; t < 8; t++) put(PK_ADV + t, adv[t]);
#pragma unroll
  for (int i = 0; i < 3; i++) put(PK_OUT + G_VETU0 + i, adv[8 + i]);
  BHAH_PHASE_BARRIER();

  // ---- phase 2a: first derivatives of h, eps, Dhat eps -------------------
  double Gh[3][3][3];
  ref_christoffel(R, Gh);
  double dh[6][3], eps[6], Dh_eps[6][3];
#pragma unroll
  for (int a = 0; a < 6; a++)
#pragma unroll
    for (int k = 0; k < 3; k++) dh[a][k] = get(PK_DH + 3 * a + k);
#pragma unroll
  for (int a = 0; a < 6; a++) eps[a] = h[a] * SS[a];
  // d_k eps_ij = S_i S_j d_k h_ij + h_ij d_k (S_i S_j)
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

  // ---- phase 2b: Ricci (Eq. 12) terms from Dhat Dhat eps below second
  // order, and the pieces of Q_k -----------------------------------------
  double Rl[6], Q[3];
#pragma unroll
  for (int a = 0; a < 6; a++) Rl[a] = 0.0;
  {
    double dGh[3][3][3][3];
    ref_christoffel_deriv(R, dGh);
    double cq[6];  // gammabar^ab (d_k d_m gammahat_ab + lower-order part of d_k d_m eps_ab)
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
      double s = get(PK_QS + k);
#pragma unroll
      for (int m = 0; m < 3; m++) {
        double tr = 0.0;
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
          for (int b = 0; b < 3; b++) tr += A[k][a][b] * A[m][b][a];
        s += beta[m] * (cq[sy(k, m)] - tr);
      }
      Q[k] = 0.5 * s;
    }
  }
  BHAH_PHASE_BARRIER();

  // ---- phase 2c: Delta^k_ij (Eq. 4, as 1/2 gammabar^kl (Dhat_i eps_lj +
  // Dhat_j eps_il - Dhat_l eps_ij)), Delta^k (Eq. 5), remaining Ricci terms --
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
  {
    // Delta terms, Delta_abc = gammabar_al Delta^l_bc formed on the fly
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
    // Lambdabar terms: gammabar_k(i Dhat_j) Lambdabar^k
    // lambda^i: first derivatives and advection from one gather (the
    // result slots of lambda are free: phase 2 no longer reads PK_DH)
    double Lam[3], DLam[3][3], dlam[3][3];
    // at 8th order one component per batch of loads
    constexpr int LB = H == 3 ? 3 : 1;
#pragma unroll
    for (int i0 = 0; i0 < 3; i0 += LB) {
      double v[LB][3][SW], f3[LB][3], fm3[KO ? LB : 1][3];
#pragma unroll
      for (int ii = 0; ii < LB; ii++)
#pragma unroll
        for (int k = 0; k < 3; k++) {
          gather_axis_k<PD, AX>(P, G_LAMU0 + i0 + ii, k, v[ii][k]);
          f3[ii][k] = upwind_far<PD, AX>(P, G_LAMU0 + i0 + ii, k, U.vu, v[ii][k]);
          if constexpr (KO) fm3[ii][k] = upwind_far<PD, AX>(P, G_LAMU0 + i0 + ii, k, U.vd, v[ii][k]);
        }
      BHAH_PHASE_BARRIER();
#pragma unroll
      for (int ii = 0; ii < LB; ii++) {
        const int i = i0 + ii;
        double a = 0.0, d = 0.0;
#pragma unroll
        for (int k = 0; k < 3; k++) {
          const bool up = vet[k] > 0.0;
          a += U.w[k] * upwind_sum<RR>(v[ii][k], f3[ii][k], up);
          if constexpr (KO) d += kw[k] * ko_v<RR>(v[ii][k], f3[ii][k], fm3[ii][k]);
          dlam[i][k] = AX && k == PD ? 0.0 : d1_axis<RR>(v[ii][k], sp.d1s[k]);
        }
        put(PK_OUT + G_LAMU0 + i, a + ga.dm * d);
        // bet^i's right-hand side takes 3/4 of lambda^i's undissipated one:
        // its result slot (free until phase 3) starts at -3/4 of lambda's
        // dissipation, which the 3/4 of lambda's full slot then cancels
        if constexpr (KO) put(PK_OUT + G_BETU0 + i, -0.75 * (ga.dm * d));
      }
    }
#pragma unroll
    for (int k = 0; k < 3; k++) Lam[k] = P.at(G_LAMU0 + k, 0, 0, 0) * R.iS[k];
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
      for (int j = 0; j < 3; j++) {
        double d = dlam[k][j] * R.iS[k] - Lam[k] * R.dS[k][j] * R.iS[k];
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
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = i; j < 3; j++) {
        const int a = sy(i, j);
        put(PK_RT + a, -0.5 * get(PK_PC + a) + Rl[a] * (R.iS[i] * R.iS[j]));
      }
#pragma unroll
    for (int k = 0; k < 3; k++) put(PK_Q + k, Q[k]);
  }
  BHAH_PHASE_BARRIER();

  // ---- phase 3: the evolution equations ----------------------------------
  // the result slots start out holding the upwinded advection terms; each
  // equation then adds the rest of its right-hand side
  auto emit = [&](int g, double v) { put(PK_OUT + g, get(PK_OUT + g) + v); };
  double diS[3][3];  // d_k (1/S_i)
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int k = 0; k < 3; k++) diS[i][k] = -R.dS[i][k] * (R.iS[i] * R.iS[i]);
  double dvet[3][3], dbeta[3][3];  // d_j vet^i, d_j beta^i
  double dW[3], dalpha[3], dK[3], phi_d[3];
#pragma unroll
  for (int k = 0; k < 3; k++) {
#pragma unroll
    for (int i = 0; i < 3; i++) dvet[i][k] = get(PK_D1 + 3 * i + k);
    dW[k] = get(PK_D1 + 9 + k);
    dalpha[k] = get(PK_D1 + 12 + k);
    phi_d[k] = -0.5 * dW[k] * iW;
  }
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) dbeta[i][j] = dvet[i][j] * R.iS[i] + vet[i] * diS[i][j];
  // upwinded advection of Abar_ij and B^i (five and four gridfunctions per
  // batch of loads), K's first derivatives and advection from one gather in
  // the second batch; the terms formed earlier move to their result slots
  if constexpr (H == 3) {
    constexpr int GA[5] = {G_ADD00, G_ADD00 + 1, G_ADD00 + 2, G_ADD00 + 3, G_ADD00 + 4};
    double a5[5];
    const double e5[5] = {ga.dm, ga.dm, ga.dm, ga.dm, ga.dm};
    advect_batch<5, PD, AX, KO>(P, GA, U, a5, e5, kw);
#pragma unroll
    for (int t = 0; t < 5; t++) put(PK_OUT + GA[t], a5[t]);
  } else if constexpr (!AX) {  // wider stencils in three directions: one gridfunction per batch
#pragma unroll
    for (int t = 0; t < 5; t++) {
      const int gl[1] = {G_ADD00 + t};
      const double e1[1] = {ga.dm};
      double a1[1];
      advect_batch<1, PD, AX, KO>(P, gl, U, a1, e1, kw);
      put(PK_OUT + G_ADD00 + t, a1[0]);
    }
  } else {  // wider stencils: batches of three and two
    constexpr int GA[3] = {G_ADD00, G_ADD00 + 1, G_ADD00 + 2}, GC[2] = {G_ADD00 + 3, G_ADD00 + 4};
    double a3[3], a2[2];
    const double e3[3] = {ga.dm, ga.dm, ga.dm}, e2[2] = {ga.dm, ga.dm};
    advect_batch<3, PD, AX, KO>(P, GA, U, a3, e3, kw);
#pragma unroll
    for (int t = 0; t < 3; t++) put(PK_OUT + GA[t], a3[t]);
    advect_batch<2, PD, AX, KO>(P, GC, U, a2, e2, kw);
#pragma unroll
    for (int t = 0; t < 2; t++) put(PK_OUT + GC[t], a2[t]);
  }
  {
    constexpr int GB[4] = {G_ADD00 + 5, G_BETU0, G_BETU0 + 1, G_BETU0 + 2};
    double a4[4];
    double v[3][SW], f3[3], fm3[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
      gather_axis_k<PD, AX>(P, G_TRK, k, v[k]);
      f3[k] = upwind_far<PD, AX>(P, G_TRK, k, U.vu, v[k]);
      if constexpr (KO) fm3[k] = upwind_far<PD, AX>(P, G_TRK, k, U.vd, v[k]);
    }
    const double e4[4] = {ga.dm, ga.dg, ga.dg, ga.dg};
    if constexpr (H == 3) {
      advect_batch<4, PD, AX, KO>(P, GB, U, a4, e4, kw);
    } else if constexpr (!AX) {  // wider stencils in three directions: one per batch
#pragma unroll
      for (int t = 0; t < 4; t++) {
        const int gl[1] = {GB[t]};
        const double e1[1] = {e4[t]};
        double a1[1];
        advect_batch<1, PD, AX, KO>(P, gl, U, a1, e1, kw);
        a4[t] = a1[0];
      }
    } else {  // wider stencils: two batches of two
      constexpr int G1[2] = {GB[0], GB[1]}, G2[2] = {GB[2], GB[3]};
      const double d1e[2] = {e4[0], e4[1]}, d2e[2] = {e4[2], e4[3]};
      double b1[2], b2[2];
      advect_batch<2, PD, AX, KO>(P, G1, U, b1, d1e, kw);
      advect_batch<2, PD, AX, KO>(P, G2, U, b2, d2e, kw);
      a4[0] = b1[0]; a4[1] = b1[1]; a4[2] = b2[0]; a4[3] = b2[1];
    }
    put(PK_OUT + GB[0], a4[0]);
#pragma unroll
    for (int t = 1; t < 4; t++) put(PK_OUT + GB[t], KO ? get(PK_OUT + GB[t]) + a4[t] : a4[t]);
    double advK = 0.0;
#pragma unroll
    for (int k = 0; k < 3; k++) {
      const bool up = vet[k] > 0.0;
      advK += U.w[k] * upwind_sum<RR>(v[k], f3[k], up);
      if constexpr (KO) advK += ga.dm * kw[k] * ko_v<RR>(v[k], f3[k], fm3[k]);
      dK[k] = AX && k == PD ? 0.0 : d1_axis<RR>(v[k], sp.d1s[k]);
    }
    put(PK_OUT + G_TRK, advK);
  }
#pragma unroll
  for (int a = 0; a < 6; a++) put(PK_OUT + G_HDD00 + a, get(PK_ADV + a));
  put(PK_OUT + G_CF, get(PK_ADV + 6));
  put(PK_OUT + G_ALPHA, get(PK_ADV + 7));
  BHAH_PHASE_BARRIER();
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
  double trA = 0.0, AA = 0.0;
#pragma unroll
  for (int i = 0; i < 3; i++) {
    trA += AUD[i][i];
#pragma unroll
    for (int j = 0; j < 3; j++) AA += Abar[sy(i, j)] * AUU[sy(i, j)];
  }
  const double W2 = W * W;

  // Eq. 9 (W), Eq. 13 (alpha), Eq. 10 (K)
  emit(G_CF, -(1.0 / 3.0) * W * (Dbeta - alpha * K));
  emit(G_ALPHA, -2.0 * alpha * K);
  {
    double lap = get(PK_ZA), da_dphi = 0.0;
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

  // Eq. 7 (eps)
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
      emit(G_HDD00 + c, r * (R.iS[i] * R.iS[j]) + h[c] * (bS[i] + bS[j]));
    }
  BHAH_PHASE_BARRIER();

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
        X[c] = get(PK_Y + c) - alpha * dW[i] * dW[j] * (iW * iW) + Gphi + 4.0 * alpha * phi_d[i] * phi_d[j] +
               2.0 * (dalpha[i] * phi_d[j] + dalpha[j] * phi_d[i]) + alpha * get(PK_RT + c) * SS[c];
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
    double dDbeta[3];  // d_k (Dbar_j beta^j)
#pragma unroll
    for (int k = 0; k < 3; k++) {
      double s = get(PK_BD + k) + get(PK_Q + k);
#pragma unroll
      for (int j = 0; j < 3; j++) s += dvet[j][k] * diS[j][j] + dvet[j][j] * diS[j][k] + vet[j] * ddiS[j][sy(j, k)];
#pragma unroll
      for (int m = 0; m < 3; m++) s += Gbc[m] * dbeta[m][k];
      dDbeta[k] = s;
    }
#pragma unroll
    for (int i = 0; i < 3; i++) {
      double t2 = get(PK_BV + i) * R.iS[i];  // gammabar^jk Dhat_j Dhat_k beta^i
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
      const double rl = get(PK_OUT + G_LAMU0 + i);  // full d_t lambda^i, advection included
      const double bet = P.at(G_BETU0 + i, 0, 0, 0);
      emit(G_VETU0 + i, bet - vet[i] * bS[i]);
      emit(G_BETU0 + i, 0.75 * rl - eta * bet - bet * bS[i]);
    }
  }
  BHAH_PHASE_BARRIER();

  // ---- results: right-hand side or RK stage combination ------------------
  if (STG && !live) return;
  // Every base value is read before any result is stored. Within a stage
  // the arrays never overlap (RK4: base1 is y or Cacc, out1 is A, B or y;
  // base2 and out2 are Cacc at the same point; SSPRK3 mixes y with A or B
  // into B or y), but the compiler cannot know it and would otherwise put
  // each load behind the stores before it. The combinations are explicit
  // fused multiply-adds, so both forms below round alike.
  const bool two = st.out2 != nullptr, mix = MIX && !two && st.base2 != nullptr, same = st.base2 == st.base1;
  auto out1m = [&](double k, double x1, double x2) { return fma(st.c1, k, fma(st.m2, x2, st.m1 * x1)); };
  // Row pairs: when all 64 lanes are live and lanes 2p, 2p+1 hold adjacent
  // points of one row, lane l stores (and loads the bases of) points 2p and
  // 2p+1, p = l mod 32, of gridfunction g + l / 32, reading the results
  // from the park: one 16-byte access per two gridfunctions and two points,
  // half the vector memory instructions of the per-lane form (each costs
  // the CU's address unit the same time whatever its width).
  const int lane = (int)(threadIdx.x & 63), p2 = 2 * (lane & 31), gs = lane >> 5;
  bool paired = false;
  unsigned qa = 0;
  if (__builtin_amdgcn_read_exec() == ~0ull) {
    qa = (unsigned)__shfl((int)q, p2);
    const unsigned qb = (unsigned)__shfl((int)q, p2 + 1);
    paired = __all(qb == qa + 1u);
  }
  if (paired) {
    const double* pk = park - lane + p2;
    auto kv = [&](int g, int h) { return pk[(PK_OUT + g + gs) * 64 + h]; };
    // gridfunction g + gs, g even: the descriptor and scalar offset of g (the
    // pair never leaves its group of four), the lane's gs in the vector offset
    const unsigned vo = qa * 8u + (unsigned)(gs * G.sgf * 8);
    if (st.rhs) {
#pragma unroll
      for (int g = 0; g < NGF; g += 2) gf_st2(st.rhs, G.sgf, g, vo, kv(g, 0), kv(g, 1));
    } else {
      double b1[NGF / 2][2], b2[NGF / 2][2];
#pragma unroll
      for (int g = 0; g < NGF; g += 2) gf_ld2(st.base1, G.sgf, g, vo, 0, b1[g / 2][0], b1[g / 2][1]);
      if ((two || mix) && !same) {
#pragma unroll
        for (int g = 0; g < NGF; g += 2) gf_ld2(st.base2, G.sgf, g, vo, 0, b2[g / 2][0], b2[g / 2][1]);
      } else {
#pragma unroll
        for (int g = 0; g < NGF / 2; g++) { b2[g][0] = b1[g][0]; b2[g][1] = b1[g][1]; }
      }
      BHAH_PHASE_BARRIER();
      if (mix) {
#pragma unroll
        for (int g = 0; g < NGF; g += 2) {
          const int j = g / 2;
          gf_st2(st.out1, G.sgf, g, vo, out1m(kv(g, 0), b1[j][0], b2[j][0]), out1m(kv(g, 1), b1[j][1], b2[j][1]));
        }
      } else {
#pragma unroll
        for (int g = 0; g < NGF; g += 2) {
          const int j = g / 2;
          const double k0 = kv(g, 0), k1 = kv(g, 1);
          gf_st2(st.out1, G.sgf, g, vo, fma(st.c1, k0, b1[j][0]), fma(st.c1, k1, b1[j][1]));
          if (two) gf_st2(st.out2, G.sgf, g, vo, fma(st.c2, k0, b2[j][0]), fma(st.c2, k1, b2[j][1]));
        }
      }
    }
  } else if (st.rhs) {
#pragma unroll
    for (int g = 0; g < NGF; g++) st.rhs[g * G.sgf + q] = get(PK_OUT + g);
  } else {
    double b1[NGF], b2[NGF];
#pragma unroll
    for (int g = 0; g < NGF; g++) b1[g] = gf_ld(st.base1, G.sgf, g, q * 8u, 0);
    if ((two || mix) && !same) {
#pragma unroll
      for (int g = 0; g < NGF; g++) b2[g] = gf_ld(st.base2, G.sgf, g, q * 8u, 0);
    } else {
#pragma unroll
      for (int g = 0; g < NGF; g++) b2[g] = b1[g];
    }
    BHAH_PHASE_BARRIER();
    if (mix) {
#pragma unroll
      for (int g = 0; g < NGF; g++) st.out1[g * G.sgf + q] = out1m(get(PK_OUT + g), b1[g], b2[g]);
    } else {
#pragma unroll
      for (int g = 0; g < NGF; g++) {
        const long long e = g * G.sgf + q;
        const double k = get(PK_OUT + g);
        st.out1[e] = fma(st.c1, k, b1[g]);
        if (two) st.out2[e] = fma(st.c2, k, b2[g]);
      }
    }
  }
  if (aux) {
#pragma unroll
    for (int a = 0; a < 6; a++) aux[a * G.sgf + q] = get(PK_RT + a);
#pragma unroll
    for (int k = 0; k < 3; k++) aux[(6 + k) * G.sgf + q] = get(PK_Q + k);
  }
}

// The fused kernel runs one wave per SIMD: every value of a point fits the
// wave's vector and accumulation registers plus its LDS park. At two waves
// per SIMD the compiler spills 700-1000 bytes per lane and the kernel is
// slower.

template <int C, bool AX, bool KO, int H, bool STG>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_rhs_fused(GridDev G, TileMap T, Gauge ga, const double* __restrict__ y, StageArgs st,
            double* __restrict__ aux) {
  const int per = (T.ntiles + BHAH_NXCD - 1) / BHAH_NXCD;
  const int w = xcd_remap((int)blockIdx.x, per);
  if (w >= T.ntiles) return;
  int i0, i1, i2;
  const bool live = tile_point<H>(G, T, w, (int)threadIdx.x, i0, i1, i2);
  if (!STG && !live) return;
  // a row tile (64 x 1 x 1) can only run past the grid along i0
  if (STG && !live) i0 = H + G.N0 - 1;
  const unsigned q = (unsigned)(i0 + G.s1 * i1 + G.s2 * i2);
  __shared__ __attribute__((aligned(16))) double park[PARK * 64];
  fused_point<C, AX, KO, true, H, STG>(G, ga, y, st, i0, i1, i2, q, aux, park + threadIdx.x, live);
}

// Persistent form for ensembles: a fixed grid of blocks (a multiple of the
// XCD count) strides over one kernel variant's (job, tile) work list (the
// jobs of one family, phi extent and order, H ghost layers); every point
// runs the same fused_point as above.
template <int C, bool AX, bool KO, bool MIX, int H>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_rhs_batch(const BatchJob* __restrict__ jobs, const BatchHdr* __restrict__ hdr, const int2* __restrict__ work,
            int stage, const int* __restrict__ counts, int kk, Gauge ga) {
  constexpr int V = 2 * C + AX + (H == 5 ? 6 : 0);
  const int n = hdr->n_tiles[V];
  const int2* wl = work + hdr->tile_off[V];
  const int per = (n + BHAH_NXCD - 1) / BHAH_NXCD;
  __shared__ double park[PARK * 64];
  for (int t = (int)blockIdx.x; t < per * BHAH_NXCD; t += (int)gridDim.x) {
    const int w = xcd_remap(t, per);
    if (w >= n) continue;
    const int2 wk = wl[w];
    if (counts && kk >= counts[wk.x]) continue;  // the job takes no step kk in this launch
    const BatchJob* J = jobs + wk.x;
    const GridDev G = J->G;
    int i0, i1, i2;
    if (!tile_point<H>(G, J->T, wk.y, (int)threadIdx.x, i0, i1, i2)) continue;
    const unsigned q = (unsigned)(i0 + G.s1 * i1 + G.s2 * i2);
    const StageArgs st = J->st[stage];
    fused_point<C, AX, KO, MIX, H>(G, ga, J->in[stage], st, i0, i1, i2, q, nullptr, park + threadIdx.x);
  }
}

TileMap make_tilemap(const GridDev& G, int lx, int ly, int band) {
  TileMap T;
  T.lx = lx;
  T.ly = ly;
  const int ex = 1 << lx, ey = 1 << ly, ez = 64 >> (lx + ly);
  T.tx = (G.N0 + ex - 1) / ex;
  T.ty = (G.N1 + ey - 1) / ey;
  T.tz = (G.N2 + ez - 1) / ez;
  T.ntiles = T.tx * T.ty * T.tz;
  T.band = band < 1 ? 1 : (band > T.ty ? T.ty : band);
  return T;
}

// launch tables over (ghost layers 3 or 5, variant = 2 coord + two phi
// planes, dissipation on)
template <int C, bool AX, bool KO, int H, bool STG = false>
void launch_fused_t(dim3 g, hipStream_t s, const GridDev& G, const TileMap& T, const Gauge& ga, const double* y,
                    const StageArgs& st, double* aux) {
  hipLaunchKernelGGL((k_rhs_fused<C, AX, KO, H, STG>), g, dim3(64), 0, s, G, T, ga, y, st, aux);
}
template <int C, bool AX, bool KO, bool MIX, int H>
void launch_batch_t(dim3 g, hipStream_t s, const BatchJob* jobs, const BatchHdr* hdr, const int2* work, int stage,
                    const int* counts, int kk, const Gauge& ga) {
  hipLaunchKernelGGL((k_rhs_batch<C, AX, KO, MIX, H>), g, dim3(64), 0, s, jobs, hdr, work, stage, counts, kk, ga);
}
using FusedLaunch = void (*)(dim3, hipStream_t, const GridDev&, const TileMap&, const Gauge&, const double*,
                             const StageArgs&, double*);
using BatchLaunch = void (*)(dim3, hipStream_t, const BatchJob*, const BatchHdr*, const int2*, int, const int*, int,
                             const Gauge&);
constexpr int SS = BHAH_SINH_SPHERICAL, SC = BHAH_SINH_CYLINDRICAL, SP = BHAH_SPHERICAL;
#define BHAH_FUSED_ROWS(H)                                                                            \
  {                                                                                                   \
    {launch_fused_t<SS, false, false, H>, launch_fused_t<SS, false, true, H>},                        \
        {launch_fused_t<SS, true, false, H>, launch_fused_t<SS, true, true, H>},                      \
        {launch_fused_t<SC, false, false, H>, launch_fused_t<SC, false, true, H>},                    \
        {launch_fused_t<SC, true, false, H>, launch_fused_t<SC, true, true, H>},                      \
        {launch_fused_t<SP, false, false, H>, launch_fused_t<SP, false, true, H>},                    \
    {                                                                                                 \
      launch_fused_t<SP, true, false, H>, launch_fused_t<SP, true, true, H>                           \
    }                                                                                                 \
  }
static const FusedLaunch kFused[2][NVAR][2] = {BHAH_FUSED_ROWS(3), BHAH_FUSED_ROWS(5)};
#undef BHAH_FUSED_ROWS
// the staged forms, [ghost layers 3 or 5][variant][dissipation]. At 8th
// order only the two-plane forms: the general ones spill kilobytes of
// registers.
#define BHAH_STAGED_ROW3(C)                                                                        \
  {launch_fused_t<C, false, false, 3, true>, launch_fused_t<C, false, true, 3, true>},             \
      {launch_fused_t<C, true, false, 3, true>, launch_fused_t<C, true, true, 3, true>}
#define BHAH_STAGED_ROW5(C) {nullptr, nullptr}, {launch_fused_t<C, true, false, 5, true>, launch_fused_t<C, true, true, 5, true>}
static const FusedLaunch kStaged[2][NVAR / 2][2] = {
    {BHAH_STAGED_ROW3(SS), BHAH_STAGED_ROW3(SC), BHAH_STAGED_ROW3(SP)},
    {BHAH_STAGED_ROW5(SS), BHAH_STAGED_ROW5(SC), BHAH_STAGED_ROW5(SP)}};
#undef BHAH_STAGED_ROW3
#undef BHAH_STAGED_ROW5
// [variant][dissipation][two-state stages (SSPRK3)]
#define BHAH_BATCH_ROW(C, AX, H)                                                                 \
  {                                                                                              \
    {launch_batch_t<C, AX, false, false, H>, launch_batch_t<C, AX, false, true, H>},             \
    { launch_batch_t<C, AX, true, false, H>, launch_batch_t<C, AX, true, true, H> }              \
  }
static const BatchLaunch kBatch[NVAR][2][2] = {
    BHAH_BATCH_ROW(SS, false, 3), BHAH_BATCH_ROW(SS, true, 3), BHAH_BATCH_ROW(SC, false, 3),
    BHAH_BATCH_ROW(SC, true, 3),  BHAH_BATCH_ROW(SP, false, 3), BHAH_BATCH_ROW(SP, true, 3),
    BHAH_BATCH_ROW(SS, false, 5), BHAH_BATCH_ROW(SS, true, 5), BHAH_BATCH_ROW(SC, false, 5),
    BHAH_BATCH_ROW(SC, true, 5),  BHAH_BATCH_ROW(SP, false, 5), BHAH_BATCH_ROW(SP, true, 5)};
#undef BHAH_BATCH_ROW

// the staged forms on row tiles (build with BHAH_RHS_STAGE=0 to keep the
// per-lane gathers there too)
#ifndef BHAH_RHS_STAGE
#define BHAH_RHS_STAGE 1
#endif
static constexpr bool rhs_stage_enabled() { return BHAH_RHS_STAGE != 0; }

void launch_rhs_fused(const GridDev& G, const Gauge& ga, const double* y, double* aux, const StageArgs& st,
                      hipStream_t s, const TileCfg& cfg_in) {
  const TileCfg cfg = tile_fits_periodic(G.coord, cfg_in) ? cfg_in : TileCfg{6, 0, cfg_in.band, cfg_in.waves};
  const TileMap T = make_tilemap(G, cfg.lx, cfg.ly, cfg.band);
  if (cfg.waves == 2 && have_rhs_pair(G, ga.ko())) {
    launch_rhs_pair(G, ga, y, aux, st, s, T);
    return;
  }
  const int per = (T.ntiles + BHAH_NXCD - 1) / BHAH_NXCD;
  const int v = rhs_variant(G.coord, G.N1, G.N2);
  const FusedLaunch staged =
      T.lx == 6 && rhs_stage_enabled() ? kStaged[G.ng == 5 ? 1 : 0][v][ga.ko() ? 1 : 0] : nullptr;
  if (staged) {
    staged(dim3(per * BHAH_NXCD), s, G, T, ga, y, st, aux);
    return;
  }
  kFused[G.ng == 5 ? 1 : 0][v][ga.ko() ? 1 : 0](dim3(per * BHAH_NXCD), s, G, T, ga, y, st, aux);
}

void launch_rhs_batch(int variant, const BatchJob* jobs, const BatchHdr* hdr, const int2* work, int stage,
                      const int* counts, int kk, const Gauge& ga, bool mix, int blocks, hipStream_t s) {
  kBatch[variant][ga.ko() ? 1 : 0][mix ? 1 : 0](dim3(blocks), s, jobs, hdr, work, stage, counts, kk, ga);
}

}  // namespace bhah
