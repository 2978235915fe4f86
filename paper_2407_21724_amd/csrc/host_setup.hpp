// Host FP64 setup of one particle class: RWG/local functions, static modes,
// the Galerkin self and neighbour blocks, and the k-space patterns.
#pragma once

#include <array>
#include <string>
#include <vector>

#include "host_math.hpp"

namespace mlfma {

// A closed, outward-oriented triangle mesh with its edge table
// (v0, v1, t_plus, t_minus), in particle-local coordinates.
struct Mesh {
  std::vector<V3> v;
  std::vector<std::array<int, 3>> t;
  std::vector<std::array<int, 4>> e;
  // derived
  std::vector<double> area;
  std::vector<V3> normal;
  std::vector<std::array<double, 3>> loc_a;  // h_{t,i}(r) = loc_a[t][i] (r - v_{t,i})
  std::vector<std::array<int, 2>> rwg_loc;   // local slots (3t+i) of f_e on T+ and T-
  std::vector<double> rwg_len;
  // quadrature points (7 per triangle)
  std::vector<V3> qp;
  std::vector<double> qw;

  // Validates the topology; returns an empty string or an error message.
  std::string build(int nv, const double* verts, int nt, const int32_t* tris, int ne,
                    const int32_t* edges);
  int nF() const { return (int)t.size(); }
  int nE() const { return (int)e.size(); }
  V3 vert(int tri, int i) const { return v[t[tri][i]]; }
};

// N functions given by their coefficients over the RWG functions, sampled
// at the quadrature points: values, divergence, and per-triangle affine
// form psi_n(r) = alpha r + beta on each triangle.
struct Sampled {
  int N = 0, Q = 0;
  std::vector<double> B;      // [N][3F] local-basis coefficients
  std::vector<double> val;    // [Q][7][N]: psi x,y,z, div, (psi x r) x,y,z
  std::vector<double> alpha;  // [N][F]
  std::vector<V3> beta;       // [N][F]
  void build(const Mesh& m, const std::vector<double>& C, int N);
  V3 psi(int n, int q, const Mesh& m) const {
    (void)m;
    const double* p = &val[(size_t)q * 7 * N];
    return {p[0 * N + n], p[1 * N + n], p[2 * N + n]};
  }
};

// Closed-form g0 parts on touching triangle pairs (local basis, per pair).
struct TouchData {
  std::vector<std::array<int, 2>> pairs;     // (a, b) triangles sharing a vertex
  std::vector<std::array<double, 9>> Xvec;   // [pair][3i*3j]
  std::vector<std::array<double, 9>> Xdiv;
  std::vector<std::array<double, 9>> XK;
  std::vector<uint8_t> touch;                // F x F flags
  void build(const Mesh& m, int outer_levels);
};

// Static modes (transverse from loops with S0, longitudinal from stars with
// Phi0), ordered {transverse (gamma descending), longitudinal (ascending)},
// unit Gram norm, largest RWG coefficient positive.  M is [(np+nl)][E].
void static_modes(const Mesh& m, const TouchData& td, int n_perp, int n_par,
                  std::vector<double>& M, std::vector<double>& gamma);

// Galerkin T and K (N x N, row-major) between functions sampled on mesh mp
// (observation) and mesh mq translated by `offset` (source), wavenumber k.
// If td != nullptr the pair is the self pair of one mesh: touching pairs use
// the regularised kernels plus the closed-form g0 parts.
void galerkin_TK(const Mesh& mp, const Sampled& sp, const Mesh& mq, const Sampled& sq, V3 offset,
                 cd k, const TouchData* td, std::vector<cd>& T, std::vector<cd>& K);

// Receiving pattern psi_hat_n(khat) = int psi_n exp(-j k khat.r) dS for each
// direction; returns [dir][3][N] complex.
void kspace_patterns(const Mesh& m, const Sampled& s, double k, const std::vector<V3>& dirs,
                     std::vector<cd>& out);

}  // namespace mlfma
