// Quadtree levels, sphere sampling grids, interpolation/anterpolation
// stencils, phase-shift tables and translation tables (host FP64).
#pragma once

#include <string>
#include <vector>

#include "host_math.hpp"

namespace mlfma {

// One level of the quadtree with its sphere sampling: nt Gauss-Legendre
// nodes in cos(theta) (theta ascending) times np = 2 nt uniform phi.
// Sample index = it * np + ip.
struct LevelGrid {
  int nx = 0, ny = 0;  // boxes
  double a = 0;        // box edge (wavelengths)
  int L = 0, nt = 0, np = 0, K = 0;
  std::vector<double> theta, wtheta;  // [nt]
  std::vector<double> w;              // [K] quadrature weights (sum 4 pi)
  std::vector<V3> khat, th_hat, ph_hat;
};

// Separable Lagrange interpolation from child level (l-1) to parent (l) and
// the child-to-parent phase shifts (the kernels' anterpolation, its
// quadrature-weighted transpose, is built from these tables by the engine).
struct InterpTables {
  int order = 4;
  // forward theta: for each parent row, `order` (child row, signed weight,
  // flip) -- flip means the node is a pole reflection: the value is read at
  // phi + pi (column + np_c/2) and the sign is folded into the weight.
  std::vector<int> th_row;
  std::vector<double> th_w;
  std::vector<uint8_t> th_flip;
  // the same stencils on the extended child rows: `order/2` pole
  // reflections, the nt_c rows, `order/2` reflections (virtual row e holds
  // child row vrow[e], read half a turn on in phi where vflip[e]); parent
  // row it uses virtual rows th_s0[it] .. th_s0[it] + order - 1
  std::vector<int> th_s0, vrow;
  std::vector<uint8_t> vflip;
  // forward phi: for each parent column, `order` (child column, weight)
  std::vector<int> ph_col;
  std::vector<double> ph_w;
  // exp(+j k khat . d_q) at the parent samples for child quadrant q =
  // 2*by + bx, d_q = ((bx - 1/2) a_c, (by - 1/2) a_c, 0): [4][K_p]
  std::vector<cd> phase;
};

struct Tree {
  std::vector<LevelGrid> lv;       // lv[0] = leaf; translations on 0..ntl-1
  int ntl = 0;                      // number of translation levels
  std::vector<InterpTables> it;     // it[l], l = 1..ntl-1 (it[0] unused)
  std::vector<std::vector<cd>> TL;  // [l] -> [49][K_l], offset (dy+3)*7+(dx+3)
};

// Builds the levels and interpolation tables.  Returns "" or an error.
std::string build_tree(int nx, int ny, double leaf, int L_leaf, int L_rule, double digits, int order,
                       double k, Tree& tr);

// Translation function of eq. translation_fun at every sample of level l
// for the centre separation r = r_obs - r_src (FP64).
void translation_function(const LevelGrid& g, V3 r, double k, std::vector<cd>& out);

// Fills tr.TL for all translation levels.
void build_translations(Tree& tr, double k);

// Gauss-Legendre nodes and weights on [-1, 1].
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

}  // namespace mlfma
