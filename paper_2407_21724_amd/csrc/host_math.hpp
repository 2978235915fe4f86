// Host-side FP64 numerics shared by the setup stages of the library:
// small vector algebra, a thread pool helper, the degree-5 triangle rule and
// the closed-form potential integrals over a flat triangle.
#pragma once

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdint>
#include <functional>
#include <thread>
#include <vector>

namespace mlfma {

using cd = std::complex<double>;
constexpr double kPi = 3.14159265358979323846;
constexpr double kFourPi = 4.0 * kPi;

struct V3 {
  double x, y, z;
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }

// Run body(i) for i in [0, n) on up to hardware_concurrency threads.
inline void parallel_for(int64_t n, const std::function<void(int64_t)>& body) {
  unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  int64_t nt = std::min<int64_t>(hw, n);
  if (nt <= 1) {
    for (int64_t i = 0; i < n; ++i) body(i);
    return;
  }
  std::vector<std::thread> pool;
  std::atomic<int64_t> next{0};
  for (int64_t t = 0; t < nt; ++t)
    pool.emplace_back([&] {
      for (int64_t i; (i = next.fetch_add(1)) < n;) body(i);
    });
  for (auto& th : pool) th.join();
}

// Radon's 7-point rule on a triangle (exact to total degree 5): barycentric
// nodes and weights normalised to sum 1.
struct TriRule {
  std::vector<std::array<double, 3>> bary;
  std::vector<double> w;
};

inline TriRule radon7() {
  TriRule r;
  const double s = std::sqrt(15.0);
  r.bary.push_back({1.0 / 3, 1.0 / 3, 1.0 / 3});
  r.w.push_back(9.0 / 40.0);
  const double as[2] = {(6.0 - s) / 21.0, (6.0 + s) / 21.0};
  const double ws[2] = {(155.0 - s) / 1200.0, (155.0 + s) / 1200.0};
  for (int o = 0; o < 2; ++o) {
    double a = as[o], b = 1.0 - 2.0 * a;
    r.bary.push_back({b, a, a});
    r.bary.push_back({a, b, a});
    r.bary.push_back({a, a, b});
    for (int k = 0; k < 3; ++k) r.w.push_back(ws[o]);
  }
  return r;
}

// Radon rule applied on each of the 4^levels pieces of a uniform midpoint
// subdivision of the reference triangle.
inline TriRule radon7_subdivided(int levels) {
  using T3 = std::array<std::array<double, 3>, 3>;
  std::vector<T3> pieces = {T3{{{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}}};
  for (int l = 0; l < levels; ++l) {
    std::vector<T3> nxt;
    for (auto& t : pieces) {
      auto mid = [](const std::array<double, 3>& a, const std::array<double, 3>& b) {
        return std::array<double, 3>{(a[0] + b[0]) / 2, (a[1] + b[1]) / 2, (a[2] + b[2]) / 2};
      };
      auto m01 = mid(t[0], t[1]), m12 = mid(t[1], t[2]), m20 = mid(t[2], t[0]);
      nxt.push_back(T3{t[0], m01, m20});
      nxt.push_back(T3{m01, t[1], m12});
      nxt.push_back(T3{m20, m12, t[2]});
      nxt.push_back(T3{m01, m12, m20});
    }
    pieces.swap(nxt);
  }
  TriRule base = radon7(), out;
  for (auto& t : pieces)
    for (size_t q = 0; q < base.w.size(); ++q) {
      std::array<double, 3> b{0, 0, 0};
      for (int v = 0; v < 3; ++v)
        for (int c = 0; c < 3; ++c) b[c] += base.bary[q][v] * t[v][c];
      out.bary.push_back(b);
      out.w.push_back(base.w[q] / pieces.size());
    }
  return out;
}

// Closed-form static potentials of a flat triangle (vertices a0,a1,a2,
// counter-clockwise about its unit normal) at an observation point r:
//   I0  = int 1/|r-r'| dS',  J = int (r'-r)/|r-r'| dS',
//   gI0 = grad_r int 1/|r-r'| dS'.
// Edge-by-edge line-integral formulas; on the triangle's plane the normal
// part of gI0 is the principal value (zero).
struct Potentials {
  double I0;
  V3 J, gI0;
};

inline Potentials triangle_potentials(V3 r, const V3 a[3]) {
  V3 n = cross(a[1] - a[0], a[2] - a[0]);
  n = (1.0 / norm(n)) * n;
  const double d = dot(r - a[0], n);
  const double ad = std::fabs(d);
  const V3 rho = r - d * n;
  const double scale = norm(a[1] - a[0]);
  const double tiny = 1e-14 * scale;
  double I0 = 0, omega = 0;
  V3 J{0, 0, 0}, gin{0, 0, 0};
  for (int i = 0; i < 3; ++i) {
    const V3 p = a[i], q = a[(i + 1) % 3];
    const double L = norm(q - p);
    const V3 lh = (1.0 / L) * (q - p);
    const V3 uh = cross(lh, n);  // outward in-plane normal of the edge
    const double lp = dot(q - rho, lh), lm = dot(p - rho, lh);
    const double P0 = dot(p - rho, uh);
    const double R0sq = P0 * P0 + d * d;
    const double Rp = std::sqrt(R0sq + lp * lp), Rm = std::sqrt(R0sq + lm * lm);
    double f = 0.0;  // ln((R+ + l+)/(R- + l-)) without cancellation
    if (R0sq > tiny * tiny) {
      if (lm >= 0)
        f = std::log((Rp + lp) / (Rm + lm));
      else if (lp < 0)
        f = std::log((Rm - lm) / (Rp - lp));
      else
        f = std::log((Rp + lp) * (Rm - lm) / R0sq);
    } else if ((lp < 0) == (lm < 0) && std::fabs(lp) > tiny && std::fabs(lm) > tiny) {
      f = std::log(std::fabs(lp) / std::fabs(lm)) * (lp > 0 ? 1.0 : -1.0);
    }
    double beta = 0.0;
    if (std::fabs(P0) > tiny)
      beta = std::atan(P0 * lp / (R0sq + ad * Rp)) - std::atan(P0 * lm / (R0sq + ad * Rm));
    if (std::fabs(P0) > tiny) I0 += P0 * f;
    I0 -= ad * beta;
    const double jc = 0.5 * ((R0sq > tiny * tiny ? R0sq * f : 0.0) + lp * Rp - lm * Rm);
    J = J + jc * uh;
    gin = gin - f * uh;
    omega += beta;
  }
  Potentials out;
  out.I0 = I0;
  out.J = J - (d * I0) * n;
  const double sd = ad > tiny ? (d > 0 ? 1.0 : -1.0) : 0.0;
  out.gI0 = gin - (sd * omega) * n;
  return out;
}

}  // namespace mlfma
