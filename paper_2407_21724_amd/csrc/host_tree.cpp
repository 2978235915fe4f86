// Quadtree, sphere grids, Lagrange stencils, phase and translation tables.
// Sec. IV (grouping, eqs. addition_th / translation_fun, truncation rule);
// Sec. V (L = 10 at the finest level, K = 2 L^2, 4 x 4 Lagrange).
#include "host_tree.hpp"

#include <algorithm>
#include <stdexcept>

namespace mlfma {

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), pp = 0;
    for (int it = 0; it < 100; ++it) {
      double p1 = 1.0, p2 = 0.0;
      for (int j = 1; j <= n; ++j) {
        double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
      }
      pp = n * (z * p1 - p2) / (z * z - 1.0);
      double dz = p1 / pp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    {
      double p1 = 1.0, p2 = 0.0;
      for (int j = 1; j <= n; ++j) {
        double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
      }
      pp = n * (z * p1 - p2) / (z * z - 1.0);
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
}

static void make_grid(LevelGrid& g) {
  g.nt = g.L;
  g.np = 2 * g.nt;
  g.K = g.nt * g.np;
  std::vector<double> x, wx;
  gauss_legendre(g.nt, x, wx);
  // theta ascending <=> cos(theta) descending
  g.theta.resize(g.nt);
  g.wtheta.resize(g.nt);
  for (int i = 0; i < g.nt; ++i) {
    g.theta[i] = std::acos(x[g.nt - 1 - i]);
    g.wtheta[i] = wx[g.nt - 1 - i];
  }
  g.w.resize(g.K);
  g.khat.resize(g.K);
  g.th_hat.resize(g.K);
  g.ph_hat.resize(g.K);
  const double dphi = 2.0 * kPi / g.np;
  for (int it = 0; it < g.nt; ++it)
    for (int ip = 0; ip < g.np; ++ip) {
      const int s = it * g.np + ip;
      const double th = g.theta[it], ph = ip * dphi;
      const double st = std::sin(th), ct = std::cos(th), sp = std::sin(ph), cp = std::cos(ph);
      g.khat[s] = {st * cp, st * sp, ct};
      g.th_hat[s] = {ct * cp, ct * sp, -st};
      g.ph_hat[s] = {-sp, cp, 0.0};
      g.w[s] = g.wtheta[it] * dphi;
    }
}

static void lagrange_weights(const double* xs, int n, double x, double* out) {
  for (int i = 0; i < n; ++i) {
    double v = 1.0;
    for (int j = 0; j < n; ++j)
      if (j != i) v *= (x - xs[j]) / (xs[i] - xs[j]);
    out[i] = v;
  }
}

static void build_interp(const LevelGrid& c, const LevelGrid& p, int order, double k, InterpTables& T) {
  T.order = order;
  const int half = order / 2;
  // extended child theta nodes: `half` reflections below 0 and above pi
  std::vector<double> ext;
  std::vector<int> ext_row;
  std::vector<int> ext_flip;
  for (int m = half; m >= 1; --m) {
    ext.push_back(-c.theta[m - 1]);
    ext_row.push_back(m - 1);
    ext_flip.push_back(1);
  }
  for (int i = 0; i < c.nt; ++i) {
    ext.push_back(c.theta[i]);
    ext_row.push_back(i);
    ext_flip.push_back(0);
  }
  for (int m = 0; m < half; ++m) {
    ext.push_back(2.0 * kPi - c.theta[c.nt - 1 - m]);
    ext_row.push_back(c.nt - 1 - m);
    ext_flip.push_back(1);
  }
  T.vrow = ext_row;
  T.vflip.assign(ext_flip.begin(), ext_flip.end());
  T.th_s0.assign(p.nt, 0);
  T.th_row.assign((size_t)p.nt * order, 0);
  T.th_w.assign((size_t)p.nt * order, 0.0);
  T.th_flip.assign((size_t)p.nt * order, 0);
  for (int it = 0; it < p.nt; ++it) {
    const double th = p.theta[it];
    int j0 = (int)(std::upper_bound(ext.begin(), ext.end(), th) - ext.begin()) - 1;
    int s0 = j0 - half + 1;
    if (s0 < 0 || s0 + order > (int)ext.size()) throw std::runtime_error("interp: theta stencil out of range");
    double wts[8];
    T.th_s0[it] = s0;
    lagrange_weights(&ext[s0], order, th, wts);
    for (int a = 0; a < order; ++a) {
      const int e = s0 + a;
      const double sw = ext_flip[e] ? -wts[a] : wts[a];
      T.th_row[(size_t)it * order + a] = ext_row[e];
      T.th_w[(size_t)it * order + a] = sw;
      T.th_flip[(size_t)it * order + a] = (uint8_t)ext_flip[e];
    }
  }
  const double dpc = 2.0 * kPi / c.np;
  T.ph_col.assign((size_t)p.np * order, 0);
  T.ph_w.assign((size_t)p.np * order, 0.0);
  for (int ip = 0; ip < p.np; ++ip) {
    const double ph = ip * 2.0 * kPi / p.np;
    int i0 = (int)std::floor(ph / dpc + 1e-12);
    double xs[8], wts[8];
    for (int b = 0; b < order; ++b) xs[b] = (i0 - half + 1 + b) * dpc;
    lagrange_weights(xs, order, ph, wts);
    for (int b = 0; b < order; ++b) {
      int col = ((i0 - half + 1 + b) % c.np + c.np) % c.np;
      T.ph_col[(size_t)ip * order + b] = col;
      T.ph_w[(size_t)ip * order + b] = wts[b];
    }
  }
  // phases for the four child quadrants
  T.phase.assign((size_t)4 * p.K, 0.0);
  for (int q = 0; q < 4; ++q) {
    const int bx = q & 1, by = q >> 1;
    const V3 d{(bx - 0.5) * c.a, (by - 0.5) * c.a, 0.0};
    for (int s = 0; s < p.K; ++s) {
      const double ph = k * dot(p.khat[s], d);
      T.phase[(size_t)q * p.K + s] = cd(std::cos(ph), std::sin(ph));
    }
  }
}

std::string build_tree(int nx, int ny, double leaf, int L_leaf, int L_rule, double digits, int order,
                       double k, Tree& tr) {
  if (nx < 1 || ny < 1) return "tree: empty grid";
  if (L_leaf < 2 || L_leaf > 400) return "tree: L_leaf out of range [2, 400]";
  if (order != 4 && order != 6) return "tree: interp_order must be 4 or 6";
  if (!(leaf > 0)) return "tree: leaf_size must be positive";
  tr = Tree();
  int bx = nx, by = ny, l = 0;
  double a = leaf;
  while (true) {
    LevelGrid g;
    g.nx = bx;
    g.ny = by;
    g.a = a;
    if (l == 0) {
      g.L = L_leaf;
    } else if (L_rule == 1) {
      g.L = L_leaf << l;
    } else {
      const double kd = k * std::sqrt(2.0) * a;
      g.L = std::max(L_leaf, (int)std::ceil(kd + 1.8 * std::pow(digits, 2.0 / 3.0) * std::cbrt(kd)));
    }
    if (g.L > 1000) return "tree: truncation above 1000 (array too large for this rule)";
    tr.lv.push_back(g);
    if (std::max(bx, by) < 3) break;
    bx = (bx + 1) / 2;
    by = (by + 1) / 2;
    a *= 2.0;
    ++l;
    if (l > 15) return "tree: more than 16 levels";
  }
  tr.ntl = (int)tr.lv.size() - 1;  // the last level has no far pairs
  for (int i = 0; i < tr.ntl; ++i) make_grid(tr.lv[i]);
  tr.it.resize(std::max(tr.ntl, 1));
  for (int i = 1; i < tr.ntl; ++i) build_interp(tr.lv[i - 1], tr.lv[i], order, k, tr.it[i]);
  return "";
}

void translation_function(const LevelGrid& g, V3 r, double k, std::vector<cd>& out) {
  const double D = norm(r);
  const V3 rh = (1.0 / D) * r;
  const int L = g.L;
  const double x = k * D;
  // spherical Hankel h_l^(2)(x) by upward recurrence (dominated by y_l)
  std::vector<cd> h(L + 1);
  const cd j(0.0, 1.0);
  const cd e = std::exp(-j * x);
  h[0] = j * e / x;
  if (L >= 1) h[1] = e * (j / (x * x) - 1.0 / x);
  for (int l = 1; l < L; ++l) h[l + 1] = (2.0 * l + 1.0) / x * h[l] - h[l - 1];
  // coefficients (-j)^l (2l+1) h_l
  std::vector<cd> c(L + 1);
  const cd mj[4] = {cd(1, 0), cd(0, -1), cd(-1, 0), cd(0, 1)};
  for (int l = 0; l <= L; ++l) c[l] = mj[l & 3] * (2.0 * l + 1.0) * h[l];
  const cd pref = -j * k / (kFourPi * kFourPi);
  out.assign(g.K, 0.0);
  for (int s = 0; s < g.K; ++s) {
    const double mu = dot(g.khat[s], rh);
    double p0 = 1.0, p1 = mu;
    cd acc = c[0];
    if (L >= 1) acc += c[1] * p1;
    for (int l = 1; l < L; ++l) {
      double p2 = ((2.0 * l + 1.0) * mu * p1 - l * p0) / (l + 1.0);
      acc += c[l + 1] * p2;
      p0 = p1;
      p1 = p2;
    }
    out[s] = pref * acc;
  }
}

void build_translations(Tree& tr, double k) {
  tr.TL.assign(tr.ntl, {});
  for (int l = 0; l < tr.ntl; ++l) {
    const LevelGrid& g = tr.lv[l];
    tr.TL[l].assign((size_t)49 * g.K, 0.0);
    parallel_for(49, [&](int64_t o) {
      const int dy = (int)o / 7 - 3, dx = (int)o % 7 - 3;
      if (std::abs(dx) <= 1 && std::abs(dy) <= 1) return;
      // source box displaced by (dx, dy): r_obs - r_src = -(dx, dy) a
      std::vector<cd> t;
      translation_function(g, V3{-dx * g.a, -dy * g.a, 0.0}, k, t);
      std::copy(t.begin(), t.end(), tr.TL[l].begin() + (size_t)o * g.K);
    });
  }
}

}  // namespace mlfma
