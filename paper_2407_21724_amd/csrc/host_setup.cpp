// Host FP64 setup of a particle class (Sec. II.A Galerkin entries, Sec. III
// static modes, eq. kspace_Rap patterns).  See host_setup.hpp.
#include "host_setup.hpp"

#include <array>
#include <atomic>
#include <map>
#include <mutex>
#include <stdexcept>

#include "host_linalg.hpp"

namespace mlfma {

std::string Mesh::build(int nv, const double* verts, int nt, const int32_t* tris, int ne,
                        const int32_t* edges) {
  if (nv < 4 || nt < 4 || ne < 6 || !verts || !tris || !edges) return "mesh: too small or null";
  if (nv - ne + nt != 2) return "mesh: Euler characteristic is not 2 (closed genus-0 surface required)";
  v.resize(nv);
  for (int i = 0; i < nv; ++i) {
    v[i] = {verts[3 * i], verts[3 * i + 1], verts[3 * i + 2]};
    if (!std::isfinite(v[i].x) || !std::isfinite(v[i].y) || !std::isfinite(v[i].z))
      return "mesh: non-finite vertex";
  }
  t.resize(nt);
  for (int i = 0; i < nt; ++i)
    for (int k = 0; k < 3; ++k) {
      int idx = tris[3 * i + k];
      if (idx < 0 || idx >= nv) return "mesh: triangle vertex index out of range";
      t[i][k] = idx;
    }
  e.resize(ne);
  for (int i = 0; i < ne; ++i)
    for (int k = 0; k < 4; ++k) e[i][k] = edges[4 * i + k];
  area.resize(nt);
  normal.resize(nt);
  loc_a.resize(nt);
  for (int i = 0; i < nt; ++i) {
    V3 a0 = vert(i, 0), a1 = vert(i, 1), a2 = vert(i, 2);
    V3 c = cross(a1 - a0, a2 - a0);
    double A = 0.5 * norm(c);
    if (!(A > 0)) return "mesh: degenerate triangle";
    area[i] = A;
    normal[i] = (1.0 / (2 * A)) * c;
    loc_a[i] = {norm(a2 - a1) / (2 * A), norm(a0 - a2) / (2 * A), norm(a1 - a0) / (2 * A)};
  }
  rwg_loc.resize(ne);
  rwg_len.resize(ne);
  std::vector<int> uses((size_t)nt, 0);
  for (int i = 0; i < ne; ++i) {
    int v0 = e[i][0], v1 = e[i][1], tp = e[i][2], tm = e[i][3];
    if (v0 < 0 || v0 >= nv || v1 < 0 || v1 >= nv || tp < 0 || tp >= nt || tm < 0 || tm >= nt || tp == tm)
      return "mesh: edge table index out of range";
    auto slot = [&](int tri, int a, int b) -> int {  // free-vertex slot if a->b is a CCW edge
      for (int k = 0; k < 3; ++k)
        if (t[tri][k] == a && t[tri][(k + 1) % 3] == b) return 3 * tri + (k + 2) % 3;
      return -1;
    };
    int sp = slot(tp, v0, v1), sm = slot(tm, v1, v0);
    if (sp < 0 || sm < 0) return "mesh: edge table inconsistent with triangle orientation";
    rwg_loc[i] = {sp, sm};
    rwg_len[i] = norm(v[v1] - v[v0]);
    uses[tp]++;
    uses[tm]++;
  }
  for (int i = 0; i < nt; ++i)
    if (uses[i] != 3) return "mesh: every triangle must border exactly three table edges";
  TriRule rr = radon7();
  qp.resize((size_t)nt * 7);
  qw.resize((size_t)nt * 7);
  for (int i = 0; i < nt; ++i)
    for (int q = 0; q < 7; ++q) {
      V3 p = rr.bary[q][0] * vert(i, 0) + rr.bary[q][1] * vert(i, 1) + rr.bary[q][2] * vert(i, 2);
      qp[(size_t)i * 7 + q] = p;
      qw[(size_t)i * 7 + q] = area[i] * rr.w[q];
    }
  return "";
}

void Sampled::build(const Mesh& m, const std::vector<double>& C, int N_) {
  N = N_;
  const int F = m.nF(), E = m.nE();
  Q = F * 7;
  B.assign((size_t)N * 3 * F, 0.0);
  for (int n = 0; n < N; ++n)
    for (int e = 0; e < E; ++e) {
      double c = C[(size_t)n * E + e];
      B[(size_t)n * 3 * F + m.rwg_loc[e][0]] += c;
      B[(size_t)n * 3 * F + m.rwg_loc[e][1]] -= c;
    }
  alpha.assign((size_t)N * F, 0.0);
  beta.assign((size_t)N * F, V3{0, 0, 0});
  for (int n = 0; n < N; ++n)
    for (int t = 0; t < F; ++t) {
      double al = 0;
      V3 be{0, 0, 0};
      for (int i = 0; i < 3; ++i) {
        double c = B[(size_t)n * 3 * F + 3 * t + i] * m.loc_a[t][i];
        al += c;
        be = be - c * m.vert(t, i);
      }
      alpha[(size_t)n * F + t] = al;
      beta[(size_t)n * F + t] = be;
    }
  val.assign((size_t)Q * 7 * N, 0.0);
  for (int q = 0; q < Q; ++q) {
    int t = q / 7;
    V3 r = m.qp[q];
    double* p = &val[(size_t)q * 7 * N];
    for (int n = 0; n < N; ++n) {
      double al = alpha[(size_t)n * F + t];
      V3 ps = al * r + beta[(size_t)n * F + t];
      V3 pxr = cross(ps, r);
      p[0 * N + n] = ps.x;
      p[1 * N + n] = ps.y;
      p[2 * N + n] = ps.z;
      p[3 * N + n] = 2.0 * al;
      p[4 * N + n] = pxr.x;
      p[5 * N + n] = pxr.y;
      p[6 * N + n] = pxr.z;
    }
  }
}

void TouchData::build(const Mesh& m, int outer_levels) {
  const int F = m.nF();
  touch.assign((size_t)F * F, 0);
  std::vector<std::vector<int>> around(m.v.size());
  for (int t = 0; t < F; ++t)
    for (int k = 0; k < 3; ++k) around[m.t[t][k]].push_back(t);
  for (auto& lst : around)
    for (int a : lst)
      for (int b : lst) touch[(size_t)a * F + b] = 1;
  pairs.clear();
  for (int a = 0; a < F; ++a)
    for (int b = 0; b < F; ++b)
      if (touch[(size_t)a * F + b]) pairs.push_back({a, b});
  const size_t np = pairs.size();
  Xvec.assign(np, {});
  Xdiv.assign(np, {});
  XK.assign(np, {});
  TriRule outer = radon7_subdivided(outer_levels);
  parallel_for((int64_t)np, [&](int64_t pi) {
    const int a = pairs[pi][0], b = pairs[pi][1];
    const V3 tb[3] = {m.vert(b, 0), m.vert(b, 1), m.vert(b, 2)};
    std::array<double, 9> xv{}, xd{}, xk{};
    for (size_t q = 0; q < outer.w.size(); ++q) {
      V3 r = outer.bary[q][0] * m.vert(a, 0) + outer.bary[q][1] * m.vert(a, 1) +
             outer.bary[q][2] * m.vert(a, 2);
      double w = outer.w[q] * m.area[a];
      Potentials P = triangle_potentials(r, tb);
      for (int i = 0; i < 3; ++i) {
        V3 hi = m.loc_a[a][i] * (r - m.vert(a, i));
        for (int j = 0; j < 3; ++j) {
          double abj = m.loc_a[b][j];
          V3 ext = abj * (r - m.vert(b, j));                      // affine extension at r
          V3 inner_vec = (1.0 / kFourPi) * (abj * P.J + P.I0 * ext);  // int h_bj g0
          V3 inner_k = (1.0 / kFourPi) * cross(ext, P.gI0);      // int h_bj x grad g0
          xv[3 * i + j] += w * dot(hi, inner_vec);
          xk[3 * i + j] += w * dot(hi, inner_k);
          xd[3 * i + j] += w * (2 * m.loc_a[a][i]) * (2 * abj) * P.I0 / kFourPi;
        }
      }
    }
    Xvec[pi] = xv;
    Xdiv[pi] = xd;
    XK[pi] = xk;
  });
}

// ---------------------------------------------------------------- modes --

namespace {

// Local-basis (3F x 3F) static matrices: vector single layer, scalar
// (divergence) single layer, and the Gram matrix.
void static_local(const Mesh& m, const TouchData& td, std::vector<double>& S, std::vector<double>& D,
                  std::vector<double>& G) {
  const int F = m.nF(), L = 3 * F;
  S.assign((size_t)L * L, 0.0);
  D.assign((size_t)L * L, 0.0);
  G.assign((size_t)L * L, 0.0);
  parallel_for(F, [&](int64_t a) {
    for (int b = 0; b < F; ++b) {
      if (td.touch[(size_t)a * F + b]) continue;
      double s[9] = {0}, d = 0;
      for (int qa = 0; qa < 7; ++qa) {
        V3 ra = m.qp[(size_t)a * 7 + qa];
        double wa = m.qw[(size_t)a * 7 + qa];
        for (int qb = 0; qb < 7; ++qb) {
          V3 rb = m.qp[(size_t)b * 7 + qb];
          double g = wa * m.qw[(size_t)b * 7 + qb] / (kFourPi * norm(ra - rb));
          d += g;
          for (int i = 0; i < 3; ++i) {
            V3 hi = m.loc_a[a][i] * (ra - m.vert(a, i));
            for (int j = 0; j < 3; ++j) s[3 * i + j] += g * dot(hi, m.loc_a[b][j] * (rb - m.vert(b, j)));
          }
        }
      }
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          S[(size_t)(3 * a + i) * L + 3 * b + j] = s[3 * i + j];
          D[(size_t)(3 * a + i) * L + 3 * b + j] = 4 * m.loc_a[a][i] * m.loc_a[b][j] * d;
        }
    }
    // Gram on the triangle itself (7-point rule exact for the quadratic integrand)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double g = 0;
        for (int q = 0; q < 7; ++q) {
          V3 r = m.qp[(size_t)a * 7 + q];
          g += m.qw[(size_t)a * 7 + q] * dot(m.loc_a[a][i] * (r - m.vert(a, i)), m.loc_a[a][j] * (r - m.vert(a, j)));
        }
        G[(size_t)(3 * a + i) * L + 3 * a + j] = g;
      }
  });
  for (size_t p = 0; p < td.pairs.size(); ++p) {
    int a = td.pairs[p][0], b = td.pairs[p][1];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        S[(size_t)(3 * a + i) * L + 3 * b + j] += td.Xvec[p][3 * i + j];
        D[(size_t)(3 * a + i) * L + 3 * b + j] += td.Xdiv[p][3 * i + j];
      }
  }
}

// RWG-basis matrix from a local-basis one: A_rwg[e][f] = sum of the four
// local entries with the +/- signs of the two halves of f_e and f_f.
std::vector<double> to_rwg(const Mesh& m, const std::vector<double>& Aloc) {
  const int E = m.nE(), L = 3 * m.nF();
  std::vector<double> A((size_t)E * E);
  parallel_for(E, [&](int64_t e) {
    for (int f = 0; f < E; ++f) {
      double s = 0;
      for (int u = 0; u < 2; ++u)
        for (int w = 0; w < 2; ++w) {
          double sg = (u == w) ? 1.0 : -1.0;
          s += sg * Aloc[(size_t)m.rwg_loc[e][u] * L + m.rwg_loc[f][w]];
        }
      A[(size_t)e * E + f] = s;
    }
  });
  return A;
}

// Project an E x E matrix onto functions given as sparse RWG combinations:
// out = C^T A C, C columns = functions.
std::vector<double> project(const std::vector<double>& A, int E,
                            const std::vector<std::vector<std::pair<int, double>>>& fn) {
  const int n = (int)fn.size();
  std::vector<double> AC((size_t)E * n, 0.0);
  parallel_for(E, [&](int64_t e) {
    for (int j = 0; j < n; ++j) {
      double s = 0;
      for (auto& [f, c] : fn[j]) s += A[(size_t)e * E + f] * c;
      AC[(size_t)e * n + j] = s;
    }
  });
  std::vector<double> out((size_t)n * n, 0.0);
  parallel_for(n, [&](int64_t i) {
    for (int j = 0; j < n; ++j) {
      double s = 0;
      for (auto& [e, c] : fn[i]) s += c * AC[(size_t)e * n + j];
      out[(size_t)i * n + j] = s;
    }
  });
  return out;
}

}  // namespace

void static_modes(const Mesh& m, const TouchData& td, int n_perp, int n_par, std::vector<double>& M,
                  std::vector<double>& gamma) {
  const int E = m.nE(), F = m.nF(), V = (int)m.v.size();
  if (n_perp < 0 || n_par < 0 || n_perp > V - 1 || n_par > F - 1)
    throw std::invalid_argument("static_modes: requested more modes than loop/star functions");
  std::vector<double> Sloc, Dloc, Gloc;
  static_local(m, td, Sloc, Dloc, Gloc);
  std::vector<double> S0 = to_rwg(m, Sloc), Phi0 = to_rwg(m, Dloc), Gr = to_rwg(m, Gloc);
  // loop functions n x grad(hat_v): +1/l on edges leaving v (as v0), -1/l entering (as v1)
  std::vector<std::vector<std::pair<int, double>>> loops(V - 1), stars(F - 1);
  for (int e = 0; e < E; ++e) {
    int v0 = m.e[e][0], v1 = m.e[e][1], tp = m.e[e][2], tm = m.e[e][3];
    double il = 1.0 / m.rwg_len[e];
    if (v0 < V - 1) loops[v0].push_back({e, il});
    if (v1 < V - 1) loops[v1].push_back({e, -il});
    if (tp < F - 1) stars[tp].push_back({e, 1.0});
    if (tm < F - 1) stars[tm].push_back({e, -1.0});
  }
  auto solve = [&](const std::vector<double>& A, const std::vector<std::vector<std::pair<int, double>>>& fn,
                   int nkeep, bool largest, std::vector<std::vector<double>>& rows, std::vector<double>& g) {
    const int n = (int)fn.size();
    std::vector<double> Ap = project(A, E, fn), Bp = project(Gr, E, fn);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j) {
        double s = 0.5 * (Ap[(size_t)i * n + j] + Ap[(size_t)j * n + i]);
        Ap[(size_t)i * n + j] = Ap[(size_t)j * n + i] = s;
        double b = 0.5 * (Bp[(size_t)i * n + j] + Bp[(size_t)j * n + i]);
        Bp[(size_t)i * n + j] = Bp[(size_t)j * n + i] = b;
      }
    std::vector<double> ev, Vec;
    generalized_eigen(Ap, Bp, n, ev, Vec);
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return largest ? ev[a] > ev[b] : ev[a] < ev[b]; });
    for (int k = 0; k < nkeep; ++k) {
      int c = order[k];
      std::vector<double> row(E, 0.0);
      for (int j = 0; j < n; ++j)
        for (auto& [e, cf] : fn[j]) row[e] += cf * Vec[(size_t)j * n + c];
      rows.push_back(row);
      g.push_back(ev[c]);
    }
  };
  std::vector<std::vector<double>> rows;
  gamma.clear();
  solve(S0, loops, n_perp, true, rows, gamma);
  solve(Phi0, stars, n_par, false, rows, gamma);
  const int N = n_perp + n_par;
  M.assign((size_t)N * E, 0.0);
  for (int i = 0; i < N; ++i) {
    auto& r = rows[i];
    double nn = 0;
    for (int e = 0; e < E; ++e)
      for (int f = 0; f < E; ++f) nn += r[e] * Gr[(size_t)e * E + f] * r[f];
    double inv = 1.0 / std::sqrt(nn);
    int imax = 0;
    for (int e = 1; e < E; ++e)
      if (std::fabs(r[e]) > std::fabs(r[imax])) imax = e;
    if (r[imax] < 0) inv = -inv;
    for (int e = 0; e < E; ++e) M[(size_t)i * E + e] = r[e] * inv;
  }
}

// ------------------------------------------------------------- Galerkin --

void galerkin_TK(const Mesh& mp, const Sampled& sp, const Mesh& mq, const Sampled& sq, V3 offset, cd k,
                 const TouchData* td, std::vector<cd>& T, std::vector<cd>& K) {
  const int Np = sp.N, Nq = sq.N, Qp = sp.Q, Qq = sq.Q;
  const int Fq = mq.nF();
  const bool real_k = k.imag() == 0.0;
  const double kr = k.real();
  const cd jj(0.0, 1.0);
  unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int nthreads = (int)std::min<unsigned>(hw, (unsigned)Qp);
  std::vector<std::vector<cd>> Tp(nthreads, std::vector<cd>((size_t)Np * Nq)),
      Kp(nthreads, std::vector<cd>((size_t)Np * Nq));
  std::atomic<int> next{0};
  std::vector<std::thread> pool;
  for (int th = 0; th < nthreads; ++th)
    pool.emplace_back([&, th] {
      std::vector<double> agr(4 * Nq), agi(4 * Nq), ahr(6 * Nq), ahi(6 * Nq);
      std::vector<cd>& Tl = Tp[th];
      std::vector<cd>& Kl = Kp[th];
      for (int a; (a = next.fetch_add(1)) < Qp;) {
        std::fill(agr.begin(), agr.end(), 0.0);
        std::fill(agi.begin(), agi.end(), 0.0);
        std::fill(ahr.begin(), ahr.end(), 0.0);
        std::fill(ahi.begin(), ahi.end(), 0.0);
        const V3 ra = mp.qp[a];
        const int ta = a / 7;
        for (int b = 0; b < Qq; ++b) {
          const V3 rb = mq.qp[b] + offset;
          const V3 d = ra - rb;
          const double R = norm(d);
          cd g, h;
          const bool tch = td && td->touch[(size_t)ta * Fq + b / 7];
          if (real_k && !tch) {
            const double kR = kr * R, c = std::cos(kR), s = std::sin(kR);
            const double inv = 1.0 / (kFourPi * R), inv3 = inv / (R * R);
            g = cd(c * inv, -s * inv);
            h = cd(-(c + kR * s) * inv3, -(kR * c - s) * inv3);
          } else if (R == 0.0) {
            g = -jj * k / kFourPi;  // limit of (exp(-jkR) - 1)/(4 pi R)
            h = 0.0;
          } else {
            const cd e = std::exp(-jj * k * R);
            g = e / (kFourPi * R);
            h = -(1.0 + jj * k * R) * e / (kFourPi * R * R * R);
            if (tch) {
              g -= 1.0 / (kFourPi * R);
              h += 1.0 / (kFourPi * R * R * R);
            }
          }
          const double wb = mq.qw[b];
          const double gr = g.real() * wb, gi = g.imag() * wb, hr = h.real() * wb, hi = h.imag() * wb;
          const double* v = &sq.val[(size_t)b * 7 * Nq];
          for (int f = 0; f < 4; ++f)
            for (int n = 0; n < Nq; ++n) {
              agr[f * Nq + n] += gr * v[f * Nq + n];
              agi[f * Nq + n] += gi * v[f * Nq + n];
            }
          for (int f = 0; f < 3; ++f)
            for (int n = 0; n < Nq; ++n) {
              ahr[f * Nq + n] += hr * v[f * Nq + n];
              ahi[f * Nq + n] += hi * v[f * Nq + n];
              ahr[(3 + f) * Nq + n] += hr * v[(4 + f) * Nq + n];
              ahi[(3 + f) * Nq + n] += hi * v[(4 + f) * Nq + n];
            }
        }
        // the stored psi x r_b is particle-local: add (sum_b h psi_n(b)) x offset
        if (offset.x != 0.0 || offset.y != 0.0 || offset.z != 0.0) {
          for (int n = 0; n < Nq; ++n) {
            const double ux = ahr[n], uy = ahr[Nq + n], uz = ahr[2 * Nq + n];
            const double vx = ahi[n], vy = ahi[Nq + n], vz = ahi[2 * Nq + n];
            ahr[3 * Nq + n] += uy * offset.z - uz * offset.y;
            ahr[4 * Nq + n] += uz * offset.x - ux * offset.z;
            ahr[5 * Nq + n] += ux * offset.y - uy * offset.x;
            ahi[3 * Nq + n] += vy * offset.z - vz * offset.y;
            ahi[4 * Nq + n] += vz * offset.x - vx * offset.z;
            ahi[5 * Nq + n] += vx * offset.y - vy * offset.x;
          }
        }
        const double wa = mp.qw[a];
        const double* pv = &sp.val[(size_t)a * 7 * Np];
        for (int m = 0; m < Np; ++m) {
          const V3 pm{pv[m], pv[Np + m], pv[2 * Np + m]};
          const double dm = pv[3 * Np + m];
          const V3 rxp = cross(ra, pm);
          for (int n = 0; n < Nq; ++n) {
            cd vecg(pm.x * agr[n] + pm.y * agr[Nq + n] + pm.z * agr[2 * Nq + n],
                    pm.x * agi[n] + pm.y * agi[Nq + n] + pm.z * agi[2 * Nq + n]);
            cd divg(dm * agr[3 * Nq + n], dm * agi[3 * Nq + n]);
            Tl[(size_t)m * Nq + n] += wa * (-jj * k * vecg + (jj / k) * divg);
            cd ku(rxp.x * ahr[n] + rxp.y * ahr[Nq + n] + rxp.z * ahr[2 * Nq + n] -
                      (pm.x * ahr[3 * Nq + n] + pm.y * ahr[4 * Nq + n] + pm.z * ahr[5 * Nq + n]),
                  rxp.x * ahi[n] + rxp.y * ahi[Nq + n] + rxp.z * ahi[2 * Nq + n] -
                      (pm.x * ahi[3 * Nq + n] + pm.y * ahi[4 * Nq + n] + pm.z * ahi[5 * Nq + n]));
            Kl[(size_t)m * Nq + n] += wa * ku;
          }
        }
      }
    });
  for (auto& t : pool) t.join();
  T.assign((size_t)Np * Nq, 0.0);
  K.assign((size_t)Np * Nq, 0.0);
  for (int th = 0; th < nthreads; ++th)
    for (size_t i = 0; i < T.size(); ++i) {
      T[i] += Tp[th][i];
      K[i] += Kp[th][i];
    }
  if (td) {
    // closed-form g0 parts over touching pairs: B X B^T
    const int F = mp.nF();
    std::vector<double> sv((size_t)Np * Nq, 0.0), sd((size_t)Np * Nq, 0.0), sk((size_t)Np * Nq, 0.0);
    for (size_t p = 0; p < td->pairs.size(); ++p) {
      const int a = td->pairs[p][0], b = td->pairs[p][1];
      for (int m = 0; m < Np; ++m)
        for (int i = 0; i < 3; ++i) {
          const double bm = sp.B[(size_t)m * 3 * F + 3 * a + i];
          if (bm == 0.0) continue;
          for (int n = 0; n < Nq; ++n) {
            const double* bn = &sq.B[(size_t)n * 3 * F + 3 * b];
            double xv = 0, xd = 0, xk = 0;
            for (int j = 0; j < 3; ++j) {
              xv += td->Xvec[p][3 * i + j] * bn[j];
              xd += td->Xdiv[p][3 * i + j] * bn[j];
              xk += td->XK[p][3 * i + j] * bn[j];
            }
            sv[(size_t)m * Nq + n] += bm * xv;
            sd[(size_t)m * Nq + n] += bm * xd;
            sk[(size_t)m * Nq + n] += bm * xk;
          }
        }
    }
    for (size_t i = 0; i < T.size(); ++i) {
      T[i] += -jj * k * sv[i] + (jj / k) * sd[i];
      K[i] += sk[i];
    }
  }
}

void kspace_patterns(const Mesh& m, const Sampled& s, double k, const std::vector<V3>& dirs,
                     std::vector<cd>& out) {
  const int N = s.N, Q = s.Q;
  out.assign(dirs.size() * 3 * N, 0.0);
  parallel_for((int64_t)dirs.size(), [&](int64_t d) {
    const V3 kh = dirs[d];
    cd* o = &out[(size_t)d * 3 * N];
    for (int q = 0; q < Q; ++q) {
      const double ph = -k * dot(kh, m.qp[q]);
      const cd e = m.qw[q] * cd(std::cos(ph), std::sin(ph));
      const double* v = &s.val[(size_t)q * 7 * N];
      for (int c = 0; c < 3; ++c)
        for (int n = 0; n < N; ++n) o[c * N + n] += e * v[c * N + n];
    }
  });
}

}  // namespace mlfma
