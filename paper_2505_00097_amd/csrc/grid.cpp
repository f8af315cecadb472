// grid.cpp -- host-side grid construction: 1-D reference-metric tables, the
// CFL time step, and the ghost-fill lists.
//
// Ghost classes (Sec. 3 of arXiv:2505.00097, Fig. 1): outer-boundary points
// lie beyond the outer edge of a non-periodic logical direction and are
// filled by quadratic extrapolation; inner-boundary points come from the
// coordinate singularities (r < 0, theta outside [0,pi], rho < 0) and from
// phi periodicity, and copy the value of the point they coincide with, with
// the sign flips of the rescaled basis vectors (Sec. 2.2). Here the inner maps
// are the closed-form index reflections of the coordinates:
//   spherical family  r -> -r      : (i0,i1,i2) -> (2NG-1-i0, N1+2NG-1-i1, i2+N2/2), flips e~0, e~2
//                     theta < 0    : i1 -> 2NG-1-i1, i2 -> i2+N2/2,                 flips e~1, e~2
//                     theta > pi   : i1 -> 2(N1+NG)-1-i1, i2 -> i2+N2/2,            flips e~1, e~2
//   cylindrical       rho -> -rho  : (i0,i1) -> (2NG-1-i0, i1+N1/2),                flips e~0, e~1
//   phi (either)      periodic wrap into the interior range.
// Classes compose (indices applied in turn, flips multiplied).
//
// The outer extrapolation is applied, in exact arithmetic, layer by layer in
// the order x0 faces, x1 faces, x2 faces with face ranges growing as layers
// are filled. Because it is linear, every outer ghost is an integer-weighted
// combination of interior values; the host composes these weights exactly and
// the device evaluates each ghost in one pass with no ordering between
// ghosts. Inner ghosts whose source is an outer ghost take that combination.
#include <algorithm>
#include <cmath>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "bhah_internal.h"

namespace bhah {

namespace {

struct Dom {
  double lo[3], hi[3];
};

Dom domain_of(int coord) {
  Dom d;
  if (coord == BHAH_SINH_CYLINDRICAL) {
    d.lo[0] = 0; d.hi[0] = 1;
    d.lo[1] = -M_PI; d.hi[1] = M_PI;
    d.lo[2] = -1; d.hi[2] = 1;
  } else {
    d.lo[0] = 0; d.hi[0] = 1;
    d.lo[1] = 0; d.hi[1] = M_PI;
    d.lo[2] = -M_PI; d.hi[2] = M_PI;
  }
  return d;
}

// sinh map of Eq. 22 (uniform for plain spherical): value and derivatives
void map_row(bool linear, double A, double w, double x, double* out) {
  if (linear) {
    out[0] = A * x; out[1] = A; out[2] = 0.0; out[3] = 0.0;
    return;
  }
  const double s = std::sinh(1.0 / w);
  const double sh = std::sinh(x / w), ch = std::cosh(x / w);
  out[0] = A * sh / s;
  out[1] = A * ch / (w * s);
  out[2] = A * sh / (w * w * s);
  out[3] = A * ch / (w * w * w * s);
}

using Comb = std::map<int, long long>;  // interior flat index -> integer weight

// d/dx at 0 of the polynomial interpolating f at the integer nodes s..s+2R:
// weights w_j = L_j'(0) of the Lagrange basis, summed in exact rational
// arithmetic (numerators and denominators stay below 2^40 for R <= 4) and
// rounded once to double.
struct Frac {
  long long p = 0, q = 1;
  static long long gcd(long long a, long long b) {
    a = a < 0 ? -a : a;
    while (b) { const long long t = a % b; a = b; b = t; }
    return a;
  }
  Frac norm() const {
    const long long g = gcd(p, q < 0 ? -q : q);
    Frac r{p / g, q / g};
    if (r.q < 0) { r.p = -r.p; r.q = -r.q; }
    return r;
  }
  Frac operator*(const Frac& o) const { return Frac{p * o.p, q * o.q}.norm(); }
  Frac operator+(const Frac& o) const { return Frac{p * o.q + o.p * q, q * o.q}.norm(); }
};
std::vector<double> one_sided_weights(int R) {
  const int W = 2 * R + 1;
  std::vector<double> out((size_t)W * W);
  for (int row = 0; row < W; row++) {
    const int s = row - 2 * R;
    for (int j = 0; j < W; j++) {
      Frac sum;
      for (int k = 0; k < W; k++) {
        if (k == j) continue;
        Frac prod{1, j - k};
        for (int i = 0; i < W; i++)
          if (i != j && i != k) prod = prod * Frac{-(s + i), j - i};
        sum = sum + prod.norm();
      }
      out[(size_t)row * W + j] = (double)sum.p / (double)sum.q;
    }
  }
  return out;
}

}  // namespace

int build_grid_host(const bhah_grid_params* p, bhah_grid* g) {
  const int coord = p->coord;
  if (coord < 0 || coord > 2) return fail(BHAH_EINVAL, "coord must be 0, 1 or 2");
  // N_G = 3: 4th-order differences; N_G = 5: 8th order (Sec. 3, N_G = N_FD/2 + 1)
  if (p->nghosts != 3 && p->nghosts != 5) return fail(BHAH_EINVAL, "nghosts must be 3 or 5");
  const int ng = p->nghosts;
  if (p->bc_kind != BHAH_BC_EXTRAP && p->bc_kind != BHAH_BC_RADIATION)
    return fail(BHAH_EINVAL, "bc_kind must be BHAH_BC_EXTRAP or BHAH_BC_RADIATION");
  const int dphi = coord == BHAH_SINH_CYLINDRICAL ? 1 : 2;
  for (int d = 0; d < 3; d++) {
    if (d != dphi && p->N[d] < ng) return fail(BHAH_EINVAL, "N[d] < nghosts in a non-periodic direction");
  }
  if (p->N[dphi] < 2 || p->N[dphi] % 2) return fail(BHAH_EINVAL, "N_phi must be even and >= 2");
  if (!(p->ampl[0] > 0)) return fail(BHAH_EINVAL, "ampl[0] must be > 0");
  if (coord != BHAH_SPHERICAL && !(p->sinhw[0] > 0)) return fail(BHAH_EINVAL, "sinhw[0] must be > 0");
  if (coord == BHAH_SINH_CYLINDRICAL && (!(p->ampl[2] > 0) || !(p->sinhw[2] > 0)))
    return fail(BHAH_EINVAL, "ampl[2] and sinhw[2] must be > 0");
  if (!(p->cfl > 0)) return fail(BHAH_EINVAL, "cfl must be > 0");
  const long long n0 = p->N[0] + 2 * ng, n1 = p->N[1] + 2 * ng, n2 = p->N[2] + 2 * ng;
  if (n0 * n1 * n2 >= (1LL << 26))
    return fail(BHAH_EINVAL, "grid too large: at most 2^26 points including ghosts (31-bit stencil offsets)");

  g->params = *p;
  bhah_grid_info& I = g->info;
  const Dom dom = domain_of(coord);
  int n[3] = {(int)n0, (int)n1, (int)n2};
  for (int d = 0; d < 3; d++) {
    I.n_total[d] = n[d];
    I.xxmin[d] = dom.lo[d];
    I.dxx[d] = (dom.hi[d] - dom.lo[d]) / p->N[d];
  }
  I.n_points = n0 * n1 * n2;
  I.n_interior = (long long)p->N[0] * p->N[1] * p->N[2];
  I.state_doubles = NGF * I.n_points;
  I.aux_doubles = NAUX * I.n_points;
  I.workspace_doubles = 3 * I.state_doubles;

  // ---- 1-D tables --------------------------------------------------------
  auto xx = [&](int d, int j) { return dom.lo[d] + ((double)(j - ng) + 0.5) * I.dxx[d]; };
  for (int d = 0; d < 3; d++) g->tab[d].assign((size_t)n[d] * TAB_W, 0.0);
  auto map_full = [&](bool linear, double A, double w, double x, double* row) {
    map_row(linear, A, w, x, row);
    row[4] = 1.0 / row[0];
    row[5] = 1.0 / row[1];
  };
  auto angle = [&](double a, double* row) {
    row[0] = std::sin(a);
    row[1] = std::cos(a);
    row[2] = 1.0 / row[0];
  };
  for (int j = 0; j < n[0]; j++)
    map_full(coord == BHAH_SPHERICAL, p->ampl[0], p->sinhw[0], xx(0, j), &g->tab[0][(size_t)j * TAB_W]);
  for (int j = 0; j < n[1]; j++) angle(xx(1, j), &g->tab[1][(size_t)j * TAB_W]);
  for (int j = 0; j < n[2]; j++) {
    if (coord == BHAH_SINH_CYLINDRICAL)
      map_full(false, p->ampl[2], p->sinhw[2], xx(2, j), &g->tab[2][(size_t)j * TAB_W]);
    else
      angle(xx(2, j), &g->tab[2][(size_t)j * TAB_W]);
  }

  // ---- CFL time step: cfl * min over interior points of min_i S_i dxx^i ----
  double dsmin = INFINITY;
  for (int i2 = ng; i2 < ng + p->N[2]; i2++)
    for (int i1 = ng; i1 < ng + p->N[1]; i1++)
      for (int i0 = ng; i0 < ng + p->N[0]; i0++) {
        const double* t0 = &g->tab[0][(size_t)i0 * TAB_W];
        double S[3];
        if (coord == BHAH_SINH_CYLINDRICAL) {
          S[0] = t0[1]; S[1] = t0[0]; S[2] = g->tab[2][(size_t)i2 * TAB_W + 1];
        } else {
          S[0] = t0[1]; S[1] = t0[0]; S[2] = t0[0] * g->tab[1][(size_t)i1 * TAB_W + 0];
        }
        for (int d = 0; d < 3; d++) dsmin = std::min(dsmin, std::fabs(S[d]) * I.dxx[d]);
      }
  I.dt = p->cfl * dsmin;

  // ---- ghost classification by index reflection -------------------------
  const long long np = I.n_points;
  auto flat = [&](int a, int b, int c) { return (int)(a + n0 * (b + n1 * (long long)c)); };
  auto coords = [&](int q, int& a, int& b, int& c) {
    a = q % n[0];
    b = (q / n[0]) % n[1];
    c = q / (n[0] * n[1]);
  };
  Classifier& classify = g->classify;
  classify.coord = coord;
  classify.ng = ng;
  for (int d = 0; d < 3; d++) {
    classify.N[d] = p->N[d];
    classify.n[d] = n[d];
  }
  auto kind_of = [&](int q) {
    int a, b, c, s2, p2;
    coords(q, a, b, c);
    return classify(a, b, c, s2, p2);
  };

  // ---- outer extrapolation composed into interior weights ---------------
  // combinations of the outer points only (a few layers of a large grid)
  std::unordered_map<int, Comb> comb;
  const Comb none;
  auto comb_of = [&](int q) -> const Comb& {
    const auto it = comb.find(q);
    return it == comb.end() ? none : it->second;
  };
  int lo[3] = {ng, ng, ng}, hi[3] = {ng + p->N[0], ng + p->N[1], ng + p->N[2]};
  const long long st[3] = {1, n0, n0 * n1};
  for (int layer = 0; layer < ng; layer++) {
    for (int d = 0; d < 3; d++) {
      for (int side = 0; side < 2; side++) {
        const int face = side == 0 ? lo[d] - 1 : hi[d];
        const long long step = (side == 0 ? 1 : -1) * st[d];
        int a[3] = {lo[0], lo[1], lo[2]}, b[3] = {hi[0], hi[1], hi[2]};
        a[d] = face; b[d] = face + 1;
        for (int i2 = a[2]; i2 < b[2]; i2++)
          for (int i1 = a[1]; i1 < b[1]; i1++)
            for (int i0 = a[0]; i0 < b[0]; i0++) {
              int src, par;
              if (classify(i0, i1, i2, src, par) != 1) continue;
              const int q = flat(i0, i1, i2);
              Comb c;
              const long long w3[3] = {3, -3, 1};
              for (int t = 1; t <= 3; t++) {
                const int s = (int)(q + t * step);
                const int ks = kind_of(s);
                if (ks == 0) {
                  c[s] += w3[t - 1];
                } else if (ks == 1 && !comb_of(s).empty()) {
                  for (auto& kv : comb_of(s)) c[kv.first] += w3[t - 1] * kv.second;
                } else {
                  return fail(BHAH_EINVAL, "extrapolation reads a point not yet filled");
                }
              }
              for (auto it = c.begin(); it != c.end();) it = it->second == 0 ? c.erase(it) : std::next(it);
              comb[q] = std::move(c);
            }
      }
      lo[d]--;
      hi[d]++;
    }
  }

  // ---- ghost list --------------------------------------------------------
  const long long n_ghosts = np - I.n_interior;
  g->g_dst.clear(); g->g_start.clear(); g->g_par.clear(); g->g_src.clear(); g->g_w.clear();
  g->g_dst.reserve(n_ghosts); g->g_start.reserve(n_ghosts + 1); g->g_par.reserve(n_ghosts);
  g->g_src.reserve(n_ghosts); g->g_w.reserve(n_ghosts);
  g->max_terms = 0;
  long long n_outer = 0, n_inner = 0;
  std::vector<std::pair<int, long long>> single(1);
  for (int i2 = 0; i2 < n[2]; i2++)
    for (int i1 = 0; i1 < n[1]; i1++)
      for (int i0 = 0; i0 < n[0]; i0++) {
        int src, par;
        const int k = classify(i0, i1, i2, src, par);
        if (k == 0) continue;
        const int q = flat(i0, i1, i2);
        const Comb* c = nullptr;
        bool one = false;
        if (k == 1) {
          c = &comb_of(q);
          n_outer++;
          if (c->empty()) return fail(BHAH_EINVAL, "outer ghost not reached by the shell order");
        } else {
          n_inner++;
          const int ks = kind_of(src);
          // inner ghosts map to interior or outer points (one hop)
          if (ks == 2) return fail(BHAH_EINVAL, "inner ghost maps to another inner ghost");
          if (ks == 0) one = true;
          else c = &comb_of(src);
        }
        g->g_dst.push_back(q);
        g->g_start.push_back((int)g->g_src.size());
        g->g_par.push_back(par);
        if (one) {
          g->g_src.push_back(src);
          g->g_w.push_back(1.0);
          g->max_terms = std::max(g->max_terms, 1);
        } else {
          for (auto& kv : *c) { g->g_src.push_back(kv.first); g->g_w.push_back((double)kv.second); }
          g->max_terms = std::max(g->max_terms, (int)c->size());
        }
      }
  g->g_start.push_back((int)g->g_src.size());

  // ---- ghosts needed by the stencils during the RK stages ---------------
  // (phi ghost planes are skipped: reads wrap phi onto the interior)
  const int pd = coord == BHAH_SINH_CYLINDRICAL ? 1 : 2;
  g->r_dst.clear(); g->r_start.clear(); g->r_par.clear(); g->r_src.clear(); g->r_w.clear();
  g->r_dst.reserve(g->g_dst.size()); g->r_start.reserve(g->g_dst.size() + 1); g->r_par.reserve(g->g_dst.size());
  g->r_src.reserve(g->g_src.size()); g->r_w.reserve(g->g_src.size());
  for (size_t t = 0; t < g->g_dst.size(); t++) {
    const int q = g->g_dst[t];
    const int idx = pd == 1 ? (q / n[0]) % n[1] : q / (n[0] * n[1]);
    if (idx < ng || idx >= ng + p->N[pd]) continue;
    g->r_dst.push_back(q);
    g->r_start.push_back((int)g->r_src.size());
    g->r_par.push_back(g->g_par[t]);
    for (int k = g->g_start[t]; k < g->g_start[t + 1]; k++) {
      g->r_src.push_back(g->g_src[k]);
      g->r_w.push_back(g->g_w[k]);
    }
  }
  g->r_start.push_back((int)g->r_src.size());
  I.n_pure_outer = n_outer;
  I.n_inner = n_inner;

  // ---- radiation outer boundary ------------------------------------------
  g->rad_q.clear(); g->rad_shift.clear(); g->rad_coef.clear();
  g->rad_w = one_sided_weights(ng - 1);
  g->inner_full = HostGhosts{};
  g->inner_stage = HostGhosts{};
  if (p->bc_kind == BHAH_BC_RADIATION) {
    // (2R+1)-point stencil start along a direction of n points at index i
    // (R = N_G - 1, the order of the differencing): centred where it fits,
    // else shifted to stay inside the array
    const int R = ng - 1;
    auto start_of = [R](int i, int nd) { return i - R < 0 ? -i : (i + R > nd - 1 ? nd - 1 - i - 2 * R : -R); };
    for (int i2 = 0; i2 < n[2]; i2++)
      for (int i1 = 0; i1 < n[1]; i1++)
        for (int i0 = 0; i0 < n[0]; i0++) {
          int src, par;
          const int k = classify(i0, i1, i2, src, par);
          if (k == 0) continue;
          const int q = flat(i0, i1, i2);
          if (k == 1) {
            // rhat . grad xx^k from the radial maps: r = r(xx0) on the
            // spherical families; r = sqrt(rho^2 + z^2), rho(xx0), z(xx2) on
            // the cylindrical one
            const double* t0 = &g->tab[0][(size_t)i0 * TAB_W];
            double r, a0, a2 = 0.0;
            if (coord == BHAH_SINH_CYLINDRICAL) {
              const double* t2 = &g->tab[2][(size_t)i2 * TAB_W];
              r = std::sqrt(t0[0] * t0[0] + t2[0] * t2[0]);
              a0 = t0[0] / r / t0[1];
              a2 = t2[0] / r / t2[1];
            } else {
              r = t0[0];
              a0 = 1.0 / t0[1];
            }
            const int s0 = start_of(i0, n[0]);
            const int s2 = coord == BHAH_SINH_CYLINDRICAL ? start_of(i2, n[2]) : -R;
            g->rad_q.push_back(q);
            g->rad_shift.push_back((s0 + 2 * R) | ((s2 + 2 * R) << 4));
            g->rad_coef.push_back(1.0 / r);
            g->rad_coef.push_back(a0 / I.dxx[0]);
            g->rad_coef.push_back(a2 / I.dxx[2]);
          } else {
            const int idx = pd == 1 ? i1 : i2;
            for (HostGhosts* L : {&g->inner_full, &g->inner_stage}) {
              if (L == &g->inner_stage && (idx < ng || idx >= ng + p->N[pd])) continue;
              L->dst.push_back(q);
              L->start.push_back((int)L->src.size());
              L->par.push_back(par);
              L->src.push_back(src);
              L->w.push_back(1.0);
            }
          }
        }
    for (HostGhosts* L : {&g->inner_full, &g->inner_stage}) L->start.push_back((int)L->src.size());
  }
  return BHAH_OK;
}

}  // namespace bhah
