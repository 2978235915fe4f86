// Interface between the host-side context (api.cpp, plain C++) and the
// device engine (engine.hip: HIP memory, kernels and the GMRES driver).
#pragma once

#include <string>
#include <vector>

#include "host_math.hpp"
#include "host_tree.hpp"

namespace mlfma {

// Everything the device path needs, assembled on the host in FP64.
struct Upload {
  int precision = 0;  // 0 = complex float, 1 = complex double, 2 = complex float with BF16-split products
  double k = 0;       // background wavenumber
  int N = 0, n = 0;   // modes per current, unknowns per particle (2N)
  int P = 0;
  int n_classes = 0;
  int nx0 = 0, ny0 = 0;  // leaf grid
  const Tree* tree = nullptr;
  std::vector<int> box_of;     // [P] leaf box of each particle
  std::vector<int> class_of;   // [P]
  // particle tiles of one class: particles order[tile_start[t] ..
  // tile_start[t] + tile_count[t]) share class tile_class[t]
  std::vector<int> order, tile_start, tile_count, tile_class;
  // per class, radiation matrix Rm [n][2 K0] (column m = comp*K0 + sample)
  // and receiving matrix Qm [2 K0][n] (quadrature weight and -jk folded in)
  std::vector<std::vector<cd>> Rm, Qm;
  // near blocks: slot matrices stored transposed [k][j] (n x n), and per
  // particle the 9 (neighbour particle, slot) pairs (-1 = none), offset
  // index o = (dy+1)*3 + (dx+1)
  std::vector<std::vector<cd>> near_mats;
  std::vector<int> near_nbr, near_slot;
  // per class inverse self block, transposed [k][j]
  std::vector<std::vector<cd>> Zinv;
  std::vector<V3> centers;
};

struct GmresResult {
  int iterations = 0;
  double true_rel_res = 0;
  double time_s = 0;
  int converged = 0;
  int reorth = 0;   // iterations that took the second Gram-Schmidt pass
  int cycles = 0;   // restart cycles
};

struct StageTime {
  std::string name;
  std::string kernel;  // symbol of the kernel the stage launched (template arguments included)
  double total_ms = 0;
  long long launches = 0;
  double bytes = 0, flops = 0;
};

class Engine {
 public:
  virtual void profile(bool enable) = 0;
  virtual int profile_read(std::vector<StageTime>& out, std::string& err) = 0;
  virtual ~Engine() = default;
  virtual int upload(const Upload& u, std::string& err) = 0;
  virtual int matvec(const void* x, void* y, int R, int parts, void* stream, std::string& err) = 0;
  // the product with its scratch in the library's static device array (no allocation)
  virtual int matvec_noalloc(const void* x, void* y, int R, void* stream, std::string& err) = 0;
  virtual int precondition(const void* x, void* y, int R, void* stream, std::string& err) = 0;
  // b[r][p] = -exp(-j k khat_r . r_p) * pat[class_p][r] with pat [C][R][n]
  virtual int rhs(const std::vector<cd>& pat, const std::vector<V3>& khat, int R, void* b, void* stream,
                  std::string& err) = 0;
  virtual int gmres(const void* b, void* x, int R, double rtol, int max_iter, int restart, bool use_x0,
                    bool always_reorth, bool fp32_basis, std::vector<GmresResult>& res, void* stream, std::string& err) = 0;
  // scattered E at n_points observation points (host FP64 [n][3]) from the
  // leaf patterns of x: E[r][i][3] in the context precision (device)
  virtual int fields(const void* x, int R, int n_points, const double* points, void* E, void* stream,
                     std::string& err) = 0;
  virtual long long device_bytes() const = 0;
  // interpolation strip heights per level (0 = default planner); agg_rows
  // indexed by the parent level, dis_rows by the child level
  virtual int set_tuning(const std::vector<int>& agg_rows, const std::vector<int>& dis_rows, std::string& err) = 0;
  virtual void get_tuning(std::vector<int>& agg_rows, std::vector<int>& dis_rows) const = 0;
  // row tiles (of 16) per block of the matrix-core GEMMs: 1, 2 or 4
  virtual int set_gemm_tiles(int rt_near_project, int rt_receive, std::string& err) = 0;
  virtual void get_gemm_tiles(int& rt_near_project, int& rt_receive) const = 0;
};

Engine* make_engine(int precision);

// Quadrature samples of one particle class for the device pair assembler:
// points qp [Q] (particle-local), weights qw [Q], and the values
// val [Q][7][N] (psi x, y, z, div, (psi x r) x, y, z) of the N functions.
struct PairSamples {
  const std::vector<V3>* qp = nullptr;
  const std::vector<double>* qw = nullptr;
  const std::vector<double>* val = nullptr;
  int N = 0;
};
// One block between distinct particles: observation class cp, source class
// cq whose centre sits at `offset` from the observation particle's centre.
struct PairRequest {
  int cp = 0, cq = 0;
  V3 offset{0, 0, 0};
};
// Galerkin T and K (N x N, row-major, exterior wavenumber k) of every
// request on the GPU in FP64: the same point-pair quadrature as
// galerkin_TK for particles that share no triangle.  T[i], K[i] are filled.
int gpu_pair_blocks(const std::vector<PairSamples>& cls, const std::vector<PairRequest>& req, double k,
                    std::vector<std::vector<cd>>& T, std::vector<std::vector<cd>>& K, std::string& err);

}  // namespace mlfma
