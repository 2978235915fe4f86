// C ABI of the MLFMA-SMR library: context, validation, host setup
// orchestration and dispatch to the device engine.  See include/mlfma.h.
#include "mlfma.h"

#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <set>
#include <memory>
#include <new>
#include <stdexcept>
#include <tuple>

#include "engine.hpp"
#include "mlp.hpp"
#include "host_linalg.hpp"
#include "host_setup.hpp"
#include "host_tree.hpp"

using namespace mlfma;

namespace {

constexpr double kK0 = 2.0 * kPi;  // background wavenumber (lengths in wavelengths)

struct ClassData {
  bool set = false;
  Mesh mesh;
  Sampled smp;
  TouchData td;
  int n_perp = 0, n_par = 0;
  cd eps{1.0, 0.0};
  std::vector<cd> Zs, Zinv;  // n x n row-major
  std::vector<cd> leafpat;   // [K0][3][N]
};

using NearKey = std::tuple<int, int, int, int>;

}  // namespace

struct mlfma_ctx {
  std::string err;
  mlfma_tree_params tp{};
  int P = 0, C = 0;
  std::vector<V3> centers;
  std::vector<int> cls;
  double eps_bg = 1.0;  // background permittivity (real, > 0)
  V3 origin{0, 0, 0};
  int nx = 0, ny = 0;
  std::vector<int> box_of, part_of_box;
  Tree tree;
  // per-class setup and the neighbour-block cache; shared between contexts
  // by mlfma_share_setup
  std::shared_ptr<std::vector<ClassData>> classes = std::make_shared<std::vector<ClassData>>();
  int N = -1;
  bool prepared = false;
  bool tl_built = false;
  std::shared_ptr<std::map<NearKey, std::vector<cd>>> near_cache =
      std::make_shared<std::map<NearKey, std::vector<cd>>>();  // n x n row-major blocks
  std::unique_ptr<Engine> eng;
};

namespace {

int fail(mlfma_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// Z^{mu nu} for distinct particles: [[T, K], [-K, T]] (zeta- = 1).
std::vector<cd> assemble_pair(const std::vector<cd>& T, const std::vector<cd>& K, int N) {
  const int n = 2 * N;
  std::vector<cd> Z((size_t)n * n);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      Z[(size_t)i * n + j] = T[(size_t)i * N + j];
      Z[(size_t)i * n + N + j] = K[(size_t)i * N + j];
      Z[(size_t)(N + i) * n + j] = -K[(size_t)i * N + j];
      Z[(size_t)(N + i) * n + N + j] = T[(size_t)i * N + j];
    }
  return Z;
}

const std::vector<cd>& near_block(mlfma_ctx* ctx, int cp, int cq, int dx, int dy) {
  NearKey key{cp, cq, dx, dy};
  auto it = ctx->near_cache->find(key);
  if (it != ctx->near_cache->end()) return it->second;
  const int N = ctx->N, n = 2 * N;
  if (dx == 0 && dy == 0 && cp == cq) {
    return (*ctx->near_cache)[key] = (*ctx->classes)[cp].Zs;
  }
  // reciprocity: Z^{nu mu}(-d) = D (Z^{mu nu}(d))^T D, D = diag(I, -I)
  auto rev = ctx->near_cache->find(NearKey{cq, cp, -dx, -dy});
  if (rev != ctx->near_cache->end()) {
    std::vector<cd> Z((size_t)n * n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double s = ((i < N) == (j < N)) ? 1.0 : -1.0;
        Z[(size_t)i * n + j] = s * rev->second[(size_t)j * n + i];
      }
    return (*ctx->near_cache)[key] = Z;
  }
  const ClassData &A = (*ctx->classes)[cp], &B = (*ctx->classes)[cq];
  std::vector<cd> T, K;
  const double s = ctx->tp.leaf_size;
  galerkin_TK(A.mesh, A.smp, B.mesh, B.smp, V3{dx * s, dy * s, 0.0}, cd(kK0, 0.0), nullptr, T, K);
  return (*ctx->near_cache)[key] = assemble_pair(T, K, N);
}

// Computes on the GPU every block between distinct particles in `keys` that
// neither the cache nor its reciprocal partner already holds.
int device_pair_blocks(mlfma_ctx* ctx, const std::vector<NearKey>& keys) {
  std::vector<NearKey> todo;
  std::set<NearKey> seen;
  for (const NearKey& key : keys) {
    const auto [cp, cq, dx, dy] = key;
    if (dx == 0 && dy == 0) continue;
    const NearKey rev{cq, cp, -dx, -dy};
    if (ctx->near_cache->count(key) || ctx->near_cache->count(rev) || seen.count(key) || seen.count(rev)) continue;
    seen.insert(key);
    todo.push_back(key);
  }
  if (todo.empty()) return MLFMA_OK;
  std::vector<PairSamples> smp(ctx->C);
  for (int c = 0; c < ctx->C; ++c)
    if ((*ctx->classes)[c].set) smp[c] = {&(*ctx->classes)[c].mesh.qp, &(*ctx->classes)[c].mesh.qw, &(*ctx->classes)[c].smp.val,
                                       ctx->N};
  std::vector<PairRequest> req;
  const double s = ctx->tp.leaf_size;
  for (const NearKey& key : todo) {
    const auto [cp, cq, dx, dy] = key;
    req.push_back({cp, cq, V3{dx * s, dy * s, 0.0}});
  }
  std::vector<std::vector<cd>> T, K;
  std::string err;
  if (int rc = gpu_pair_blocks(smp, req, kK0, T, K, err)) return fail(ctx, rc == -1 ? MLFMA_EINVAL : rc, err);
  for (size_t i = 0; i < todo.size(); ++i) (*ctx->near_cache)[todo[i]] = assemble_pair(T[i], K[i], ctx->N);
  return MLFMA_OK;
}

std::vector<cd> transpose(const std::vector<cd>& A, int n) {
  std::vector<cd> B((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) B[(size_t)j * n + i] = A[(size_t)i * n + j];
  return B;
}

int do_prepare(mlfma_ctx* ctx) {
  if (ctx->prepared) return MLFMA_OK;
  for (int p = 0; p < ctx->P; ++p)
    if (!(*ctx->classes)[ctx->cls[p]].set)
      return fail(ctx, MLFMA_ENOTREADY, "class " + std::to_string(ctx->cls[p]) + " has no static modes");
  const int N = ctx->N, n = 2 * N;
  if (!ctx->tl_built) {
    build_translations(ctx->tree, kK0);
    ctx->tl_built = true;
  }
  Upload u;
  u.precision = ctx->tp.precision;
  u.k = kK0;
  u.N = N;
  u.n = n;
  u.P = ctx->P;
  u.n_classes = ctx->C;
  u.nx0 = ctx->nx;
  u.ny0 = ctx->ny;
  u.tree = &ctx->tree;
  u.box_of = ctx->box_of;
  u.class_of = ctx->cls;
  u.centers = ctx->centers;
  // tiles of one class (particle order sorted by class, then index)
  const int TP = ctx->tp.precision == MLFMA_C128 ? 8 : 16;
  for (int c = 0; c < ctx->C; ++c) {
    std::vector<int> mem;
    for (int p = 0; p < ctx->P; ++p)
      if (ctx->cls[p] == c) mem.push_back(p);
    for (size_t s = 0; s < mem.size(); s += TP) {
      u.tile_start.push_back((int)u.order.size() + (int)s);
      u.tile_count.push_back((int)std::min<size_t>(TP, mem.size() - s));
      u.tile_class.push_back(c);
    }
    u.order.insert(u.order.end(), mem.begin(), mem.end());
  }
  // near blocks between distinct particles: assembled on the GPU in one pass
  {
    std::vector<NearKey> keys;
    for (int p = 0; p < ctx->P; ++p) {
      const int ix = ctx->box_of[p] % ctx->nx, iy = ctx->box_of[p] / ctx->nx;
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int jx = ix + dx, jy = iy + dy;
          if ((dx == 0 && dy == 0) || jx < 0 || jy < 0 || jx >= ctx->nx || jy >= ctx->ny) continue;
          const int q = ctx->part_of_box[jy * ctx->nx + jx];
          if (q >= 0) keys.push_back(NearKey{ctx->cls[p], ctx->cls[q], dx, dy});
        }
    }
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    if (int rc = device_pair_blocks(ctx, keys)) return rc;
  }
  // near blocks and slots
  std::map<NearKey, int> slot_of;
  u.near_nbr.assign((size_t)ctx->P * 9, -1);
  u.near_slot.assign((size_t)ctx->P * 9, 0);
  for (int p = 0; p < ctx->P; ++p) {
    const int ix = ctx->box_of[p] % ctx->nx, iy = ctx->box_of[p] / ctx->nx;
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int jx = ix + dx, jy = iy + dy;
        if (jx < 0 || jy < 0 || jx >= ctx->nx || jy >= ctx->ny) continue;
        const int q = ctx->part_of_box[jy * ctx->nx + jx];
        if (q < 0) continue;
        NearKey key{ctx->cls[p], ctx->cls[q], dx, dy};
        auto it = slot_of.find(key);
        int slot;
        if (it == slot_of.end()) {
          slot = (int)u.near_mats.size();
          slot_of[key] = slot;
          u.near_mats.push_back(transpose(near_block(ctx, ctx->cls[p], ctx->cls[q], dx, dy), n));
        } else {
          slot = it->second;
        }
        const int o = (dy + 1) * 3 + (dx + 1);
        u.near_nbr[(size_t)p * 9 + o] = q;
        u.near_slot[(size_t)p * 9 + o] = slot;
      }
  }
  // per-class pattern matrices and preconditioner blocks
  u.Rm.resize(ctx->C);
  u.Qm.resize(ctx->C);
  u.Zinv.resize(ctx->C);
  const bool far = ctx->tree.ntl > 0;
  for (int c = 0; c < ctx->C; ++c) {
    const ClassData& cdt = (*ctx->classes)[c];
    if (!cdt.set) {
      u.Zinv[c].assign((size_t)n * n, 0.0);
      if (far) {
        u.Rm[c].assign((size_t)n * 2 * ctx->tree.lv[0].K, 0.0);
        u.Qm[c].assign((size_t)n * 2 * ctx->tree.lv[0].K, 0.0);
      }
      continue;
    }
    u.Zinv[c] = transpose(cdt.Zinv, n);
    if (!far) continue;
    const LevelGrid& g = ctx->tree.lv[0];
    const int K0 = g.K, M2 = 2 * K0;
    std::vector<cd>& Rm = u.Rm[c];
    std::vector<cd>& Qm = u.Qm[c];
    Rm.assign((size_t)n * M2, 0.0);
    Qm.assign((size_t)M2 * n, 0.0);
    const cd mjk(0.0, -kK0);
    for (int s = 0; s < K0; ++s) {
      for (int m = 0; m < N; ++m) {
        const cd* pv = &cdt.leafpat[(size_t)s * 3 * N];
        const cd pt = pv[m] * g.th_hat[s].x + pv[N + m] * g.th_hat[s].y + pv[2 * N + m] * g.th_hat[s].z;
        const cd pp = pv[m] * g.ph_hat[s].x + pv[N + m] * g.ph_hat[s].y + pv[2 * N + m] * g.ph_hat[s].z;
        // radiation: U_th = a_th + b_ph, U_ph = a_ph - b_th with a, b the
        // conjugate patterns weighted by J_e, J_m (zeta- = 1)
        Rm[(size_t)m * M2 + s] = std::conj(pt);
        Rm[(size_t)(N + m) * M2 + s] = std::conj(pp);
        Rm[(size_t)m * M2 + K0 + s] = std::conj(pp);
        Rm[(size_t)(N + m) * M2 + K0 + s] = -std::conj(pt);
        // receiving: e-rows test G, m-rows test khat x G
        const double w = g.w[s];
        Qm[(size_t)s * n + m] = mjk * w * pt;
        Qm[(size_t)(K0 + s) * n + m] = mjk * w * pp;
        Qm[(size_t)s * n + N + m] = mjk * w * pp;
        Qm[(size_t)(K0 + s) * n + N + m] = -mjk * w * pt;
      }
    }
  }
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return fail(ctx, MLFMA_EHIP, std::string("no HIP device: ") + hipGetErrorString(he));
  std::unique_ptr<Engine> eng(make_engine(ctx->tp.precision));
  std::string err;
  int rc = eng->upload(u, err);
  if (rc) return fail(ctx, rc, err);
  ctx->eng = std::move(eng);
  ctx->prepared = true;
  return MLFMA_OK;
}

template <typename F>
int guarded(mlfma_ctx* ctx, F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(ctx, MLFMA_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(ctx, MLFMA_EINVAL, e.what());
  } catch (...) {
    return fail(ctx, MLFMA_EINVAL, "unknown error");
  }
}

}  // namespace

extern "C" {

void mlfma_default_params(mlfma_tree_params* tp) {
  if (!tp) return;
  tp->leaf_size = 0.5;
  tp->L_leaf = 11;
  tp->L_rule = 0;
  tp->digits = 3.0;
  tp->interp_order = 6;
  tp->precision = MLFMA_C64;
  tp->outer_levels = 2;
  tp->near_rule = 0;
}

int mlfma_build_tree(const mlfma_problem* pb, const mlfma_tree_params* tp, mlfma_ctx** out) {
  if (!out) return MLFMA_EINVAL;
  *out = nullptr;
  std::unique_ptr<mlfma_ctx> ctx;
  try {
    ctx.reset(new mlfma_ctx());
  } catch (...) {
    return MLFMA_ENOMEM;
  }
  if (!pb || !tp || !pb->centers || !pb->class_id || pb->n_particles < 1 || pb->n_classes < 1)
    return MLFMA_EINVAL;
  if (tp->precision != MLFMA_C64 && tp->precision != MLFMA_C128 && tp->precision != MLFMA_C64_BF16)
    return MLFMA_EINVAL;
  if (tp->outer_levels < 0 || tp->outer_levels > 5 || !(tp->digits > 0) || (tp->L_rule != 0 && tp->L_rule != 1) ||
      tp->near_rule != 0)
    return MLFMA_EINVAL;
  ctx->tp = *tp;
  if (!std::isfinite(pb->eps_bg_re) || !std::isfinite(pb->eps_bg_im)) return MLFMA_ENONFINITE;
  if (pb->eps_bg_im != 0.0 || pb->eps_bg_re < 0.0) return MLFMA_EINVAL;
  ctx->eps_bg = pb->eps_bg_re == 0.0 ? 1.0 : pb->eps_bg_re;
  const int P = pb->n_particles;
  if (!finite_all(pb->centers, (size_t)3 * P)) return MLFMA_ENONFINITE;
  ctx->P = P;
  ctx->C = pb->n_classes;
  ctx->centers.resize(P);
  ctx->cls.resize(P);
  double x0 = 1e300, y0 = 1e300;
  for (int p = 0; p < P; ++p) {
    ctx->centers[p] = {pb->centers[3 * p], pb->centers[3 * p + 1], pb->centers[3 * p + 2]};
    ctx->cls[p] = pb->class_id[p];
    if (ctx->cls[p] < 0 || ctx->cls[p] >= ctx->C) return MLFMA_EINVAL;
    x0 = std::min(x0, ctx->centers[p].x);
    y0 = std::min(y0, ctx->centers[p].y);
  }
  const double z0 = ctx->centers[0].z, s = tp->leaf_size;
  if (!(s > 0)) return MLFMA_EINVAL;
  const double tol = 1e-6 * s;
  ctx->origin = {x0, y0, z0};
  std::vector<int> ix(P), iy(P);
  int mx = 0, my = 0;
  for (int p = 0; p < P; ++p) {
    const V3 c = ctx->centers[p];
    if (std::fabs(c.z - z0) > tol) return MLFMA_EINVAL;
    const double fx = (c.x - x0) / s, fy = (c.y - y0) / s;
    ix[p] = (int)std::lround(fx);
    iy[p] = (int)std::lround(fy);
    if (std::fabs(fx - ix[p]) * s > tol || std::fabs(fy - iy[p]) * s > tol) return MLFMA_EINVAL;
    mx = std::max(mx, ix[p]);
    my = std::max(my, iy[p]);
  }
  if ((int64_t)(mx + 1) * (my + 1) > 100000000LL) return MLFMA_EINVAL;
  ctx->nx = mx + 1;
  ctx->ny = my + 1;
  ctx->part_of_box.assign((size_t)ctx->nx * ctx->ny, -1);
  ctx->box_of.resize(P);
  for (int p = 0; p < P; ++p) {
    const int b = iy[p] * ctx->nx + ix[p];
    if (ctx->part_of_box[b] >= 0) return MLFMA_EINVAL;  // two particles on one site
    ctx->part_of_box[b] = p;
    ctx->box_of[p] = b;
  }
  try {
    std::string e = build_tree(ctx->nx, ctx->ny, s, tp->L_leaf, tp->L_rule, tp->digits, tp->interp_order, kK0, ctx->tree);
    if (!e.empty()) return MLFMA_EINVAL;
    ctx->classes->resize(ctx->C);
  } catch (...) {
    return MLFMA_EINVAL;
  }
  *out = ctx.release();
  return MLFMA_OK;
}

int mlfma_static_modes(int32_t nv, const double* verts, int32_t nt, const int32_t* tris, int32_t ne,
                       const int32_t* edges, int32_t n_perp, int32_t n_par, double* M_out, double* gamma_out) {
  try {
    if (!M_out || n_perp < 0 || n_par < 0 || n_perp + n_par < 1) return MLFMA_EINVAL;
    if (!verts || !finite_all(verts, (size_t)3 * std::max(nv, 0))) return MLFMA_ENONFINITE;
    Mesh m;
    if (!m.build(nv, verts, nt, tris, ne, edges).empty()) return MLFMA_EINVAL;
    if (n_perp > nv - 1 || n_par > nt - 1) return MLFMA_EINVAL;
    TouchData td;
    td.build(m, 2);
    std::vector<double> M, g;
    static_modes(m, td, n_perp, n_par, M, g);
    if (!finite_all(M.data(), M.size())) return MLFMA_ENONFINITE;
    std::memcpy(M_out, M.data(), M.size() * sizeof(double));
    if (gamma_out) std::memcpy(gamma_out, g.data(), g.size() * sizeof(double));
    return MLFMA_OK;
  } catch (const std::bad_alloc&) {
    return MLFMA_ENOMEM;
  } catch (...) {
    return MLFMA_EINVAL;
  }
}

int mlfma_set_static_modes(mlfma_ctx* ctx, int32_t class_id, int32_t nv, const double* verts, int32_t nt,
                           const int32_t* tris, int32_t ne, const int32_t* edges, int32_t n_perp, int32_t n_par,
                           const double* M, double eps_re, double eps_im) {
  if (!ctx) return MLFMA_EINVAL;
  return guarded(ctx, [&]() -> int {
    if (class_id < 0 || class_id >= ctx->C) return fail(ctx, MLFMA_EINVAL, "class_id out of range");
    if (n_perp < 0 || n_par < 0 || n_perp + n_par < 1) return fail(ctx, MLFMA_EINVAL, "mode counts");
    const int N = n_perp + n_par;
    if (ctx->N >= 0 && ctx->N != N) return fail(ctx, MLFMA_EINVAL, "all classes must have the same mode count");
    if (2 * N > 128) return fail(ctx, MLFMA_EINVAL, "at most 64 modes per current");
    if (!M || ne < 1) return fail(ctx, MLFMA_EINVAL, "null modes");
    if (!finite_all(M, (size_t)N * ne) || !std::isfinite(eps_re) || !std::isfinite(eps_im))
      return fail(ctx, MLFMA_ENONFINITE, "non-finite modes or permittivity");
    if (!verts || !finite_all(verts, (size_t)3 * std::max(nv, 0))) return fail(ctx, MLFMA_ENONFINITE, "vertices");
    ClassData cdt;
    std::string e = cdt.mesh.build(nv, verts, nt, tris, ne, edges);
    if (!e.empty()) return fail(ctx, MLFMA_EINVAL, e);
    cdt.n_perp = n_perp;
    cdt.n_par = n_par;
    cdt.eps = cd(eps_re, eps_im) / ctx->eps_bg;  // eps+ / eps-
    std::vector<double> Mv(M, M + (size_t)N * ne);
    cdt.smp.build(cdt.mesh, Mv, N);
    cdt.td.build(cdt.mesh, ctx->tp.outer_levels);
    // self block, both media (eq. Zpq_delta with delta = 1)
    const cd sq = std::sqrt(cdt.eps);
    const cd k_in = kK0 * sq, z_in = 1.0 / sq;
    std::vector<cd> To, Ko, Ti, Ki;
    galerkin_TK(cdt.mesh, cdt.smp, cdt.mesh, cdt.smp, V3{0, 0, 0}, cd(kK0, 0.0), &cdt.td, To, Ko);
    galerkin_TK(cdt.mesh, cdt.smp, cdt.mesh, cdt.smp, V3{0, 0, 0}, k_in, &cdt.td, Ti, Ki);
    const int n = 2 * N;
    cdt.Zs.assign((size_t)n * n, 0.0);
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        const cd t_o = To[(size_t)i * N + j], t_i = Ti[(size_t)i * N + j];
        const cd kk = Ko[(size_t)i * N + j] + Ki[(size_t)i * N + j];
        cdt.Zs[(size_t)i * n + j] = t_o + z_in * t_i;
        cdt.Zs[(size_t)i * n + N + j] = kk;
        cdt.Zs[(size_t)(N + i) * n + j] = -kk;
        cdt.Zs[(size_t)(N + i) * n + N + j] = t_o + t_i / z_in;
      }
    for (auto& z : cdt.Zs)
      if (!std::isfinite(z.real()) || !std::isfinite(z.imag())) return fail(ctx, MLFMA_ENONFINITE, "self block");
    cdt.Zinv = cdt.Zs;
    if (!complex_inverse(cdt.Zinv, n)) return fail(ctx, MLFMA_ENONFINITE, "self block is singular");
    if (ctx->tree.ntl > 0) kspace_patterns(cdt.mesh, cdt.smp, kK0, ctx->tree.lv[0].khat, cdt.leafpat);
    cdt.set = true;
    (*ctx->classes)[class_id] = std::move(cdt);
    ctx->N = N;
    ctx->prepared = false;
    ctx->eng.reset();
    // blocks involving this class must be recomputed
    for (auto it = ctx->near_cache->begin(); it != ctx->near_cache->end();) {
      if (std::get<0>(it->first) == class_id || std::get<1>(it->first) == class_id)
        it = ctx->near_cache->erase(it);
      else
        ++it;
    }
    return MLFMA_OK;
  });
}

int mlfma_set_tuning(mlfma_ctx* ctx, const mlfma_tuning* t) {
  if (!ctx || !t) return MLFMA_EINVAL;
  return guarded(ctx, [&]() -> int {
    if (int rc = do_prepare(ctx)) return rc;
    const int L = ctx->tree.ntl;
    if (t->n_levels != L || L > MLFMA_MAX_LEVELS) return fail(ctx, MLFMA_EINVAL, "n_levels does not match the tree");
    std::vector<int> a(L, 0), d(L, 0);
    for (int l = 0; l < L; ++l) {
      if (t->agg_rows[l] < 0 || t->dis_rows[l] < 0) return fail(ctx, MLFMA_EINVAL, "negative strip height");
      a[l] = t->agg_rows[l];
      d[l] = t->dis_rows[l];
    }
    std::string err;
    int rc = ctx->eng->set_gemm_tiles(t->gemm_rows_near, t->gemm_rows_receive, err);
    if (!rc) rc = ctx->eng->set_tuning(a, d, err);
    return rc ? fail(ctx, rc == -1 ? MLFMA_EINVAL : rc, err) : MLFMA_OK;
  });
}

int mlfma_get_tuning(mlfma_ctx* ctx, mlfma_tuning* t) {
  if (!ctx || !t) return MLFMA_EINVAL;
  return guarded(ctx, [&]() -> int {
    if (int rc = do_prepare(ctx)) return rc;
    std::vector<int> a, d;
    ctx->eng->get_tuning(a, d);
    std::memset(t, 0, sizeof(*t));
    t->n_levels = ctx->tree.ntl;
    for (int l = 0; l < ctx->tree.ntl && l < MLFMA_MAX_LEVELS; ++l) {
      t->agg_rows[l] = a[l];
      t->dis_rows[l] = d[l];
    }
    int rn = 0, rr = 0;
    ctx->eng->get_gemm_tiles(rn, rr);
    t->gemm_rows_near = rn;
    t->gemm_rows_receive = rr;
    return MLFMA_OK;
  });
}

int mlfma_share_setup(mlfma_ctx* dst, const mlfma_ctx* src) {
  if (!dst || !src || dst == src) return MLFMA_EINVAL;
  return guarded(dst, [&]() -> int {
    const mlfma_tree_params &a = dst->tp, &b = src->tp;
    if (dst->C != src->C || a.leaf_size != b.leaf_size || a.L_leaf != b.L_leaf || a.L_rule != b.L_rule ||
        a.digits != b.digits || a.outer_levels != b.outer_levels)
      return fail(dst, MLFMA_EINVAL, "contexts differ in class count or tree parameters");
    if (dst->tree.ntl > 0)
      for (const ClassData& c : *src->classes)
        if (c.set && c.leafpat.empty())
          return fail(dst, MLFMA_EINVAL, "source context has no far-field patterns (build it with far levels)");
    dst->classes = src->classes;
    dst->near_cache = src->near_cache;
    dst->N = src->N;
    dst->prepared = false;
    dst->eng.reset();
    return MLFMA_OK;
  });
}

int mlfma_prepare(mlfma_ctx* ctx) {
  if (!ctx) return MLFMA_EINVAL;
  return guarded(ctx, [&] { return do_prepare(ctx); });
}

int mlfma_plane_wave_rhs(mlfma_ctx* ctx, int32_t R, const double* khat, const double* pol, void* b_dev,
                         void* stream) {
  if (!ctx) return MLFMA_EINVAL;
  return guarded(ctx, [&]() -> int {
    if (R < 1 || !khat || !pol || !b_dev) return fail(ctx, MLFMA_EINVAL, "rhs arguments");
    if (!finite_all(khat, (size_t)3 * R) || !finite_all(pol, (size_t)6 * R))
      return fail(ctx, MLFMA_ENONFINITE, "non-finite incidence");
    if (int rc = do_prepare(ctx)) return rc;
    const int N = ctx->N, n = 2 * N;
    std::vector<V3> dirs(R);
    for (int r = 0; r < R; ++r) {
      dirs[r] = {khat[3 * r], khat[3 * r + 1], khat[3 * r + 2]};
      const double nn = norm(dirs[r]);
      if (std::fabs(nn - 1.0) > 1e-6) return fail(ctx, MLFMA_EINVAL, "khat must be unit vectors");
    }
    std::vector<cd> pat((size_t)ctx->C * R * n, 0.0);
    for (int c = 0; c < ctx->C; ++c) {
      if (!(*ctx->classes)[c].set) continue;
      std::vector<cd> ps;
      kspace_patterns((*ctx->classes)[c].mesh, (*ctx->classes)[c].smp, kK0, dirs, ps);
      for (int r = 0; r < R; ++r) {
        const cd e[3] = {cd(pol[6 * r], pol[6 * r + 1]), cd(pol[6 * r + 2], pol[6 * r + 3]),
                         cd(pol[6 * r + 4], pol[6 * r + 5])};
        const V3 kh = dirs[r];
        // h = khat x e (zeta- = 1)
        const cd h[3] = {kh.y * e[2] - kh.z * e[1], kh.z * e[0] - kh.x * e[2], kh.x * e[1] - kh.y * e[0]};
        for (int m = 0; m < N; ++m) {
          cd ve = 0, vh = 0;
          for (int c3 = 0; c3 < 3; ++c3) {
            const cd psi = ps[((size_t)r * 3 + c3) * N + m];
            ve += e[c3] * psi;
            vh += h[c3] * psi;
          }
          pat[((size_t)c * R + r) * n + m] = ve;
          pat[((size_t)c * R + r) * n + N + m] = vh;
        }
      }
    }
    std::string err;
    int rc = ctx->eng->rhs(pat, dirs, R, b_dev, stream, err);
    return rc ? fail(ctx, rc, err) : MLFMA_OK;
  });
}

int mlfma_matvec_parts(mlfma_ctx* ctx, const void* x_dev, void* y_dev, int32_t R, int32_t parts, void* stream) {
  if (!ctx) return MLFMA_EINVAL;
  return guarded(ctx, [&]() -> int {
    if (!x_dev || !y_dev || R < 1 || parts < 1 || parts > 3) return fail(ctx, MLFMA_EINVAL, "matvec arguments");
    if (x_dev == y_dev) return fail(ctx, MLFMA_EINVAL, "x and y must not alias");
    if (((uintptr_t)x_dev | (uintptr_t)y_dev) & 15) return fail(ctx, MLFMA_EINVAL, "x and y must be 16-byte aligned");
    if (int rc = do_prepare(ctx)) return rc;
    const size_t bytes = (size_t)R * ctx->P * 2 * ctx->N * (ctx->tp.precision == MLFMA_C128 ? 16 : 8);
    const char *xa = (const char*)x_dev, *ya = (const char*)y_dev;
    if (xa < ya + bytes && ya < xa + bytes) return fail(ctx, MLFMA_EINVAL, "x and y overlap");
    std::string err;
    int rc = ctx->eng->matvec(x_dev, y_dev, R, parts, stream, err);
    return rc ? fail(ctx, rc, err) : MLFMA_OK;
  });
}

int mlfma_matvec(mlfma_ctx* ctx, const void* x_dev, void* y_dev, int32_t R, void* stream) {
  return mlfma_matvec_parts(ctx, x_dev, y_dev, R, MLFMA_PART_ALL, stream);
}

int mlfma_matvec_noalloc(mlfma_ctx* ctx, const void* x_dev, void* y_dev, int32_t R, void* stream) {
  if (!ctx) return MLFMA_EINVAL;
  return guarded(ctx, [&]() -> int {
    if (!x_dev || !y_dev || R < 1) return fail(ctx, MLFMA_EINVAL, "matvec_noalloc arguments");
    if (((uintptr_t)x_dev | (uintptr_t)y_dev) & 15) return fail(ctx, MLFMA_EINVAL, "x and y must be 16-byte aligned");
    if (!ctx->prepared)
      return fail(ctx, MLFMA_ENOTREADY, "matvec_noalloc: the context is not prepared (call mlfma_prepare first)");
    const size_t bytes = (size_t)R * ctx->P * 2 * ctx->N * (ctx->tp.precision == MLFMA_C128 ? 16 : 8);
    const char *xa = (const char*)x_dev, *ya = (const char*)y_dev;
    if (xa < ya + bytes && ya < xa + bytes) return fail(ctx, MLFMA_EINVAL, "x and y overlap");
    std::string err;
    int rc = ctx->eng->matvec_noalloc(x_dev, y_dev, R, stream, err);
    return rc ? fail(ctx, rc == -1 ? MLFMA_EINVAL : rc, err) : MLFMA_OK;
  });
}

int mlfma_fields(mlfma_ctx* ctx, const void* x_dev, int32_t R, int32_t n_points, const double* points, void* E_dev,
                 void* stream) {
  if (!ctx) return MLFMA_EINVAL;
  return guarded(ctx, [&]() -> int {
    if (!x_dev || !E_dev || R < 1 || n_points < 0 || (n_points > 0 && !points) || x_dev == E_dev)
      return fail(ctx, MLFMA_EINVAL, "fields arguments");
    if ((uintptr_t)x_dev & 15) return fail(ctx, MLFMA_EINVAL, "x must be 16-byte aligned");
    for (int i = 0; i < 3 * n_points; ++i)
      if (!std::isfinite(points[i])) return fail(ctx, MLFMA_EINVAL, "non-finite observation point");
    if (int rc = do_prepare(ctx)) return rc;
    // every point farther from every centre than half a leaf-box diagonal
    // (the expansion of a particle's field about its centre holds outside
    // the sphere that circumscribes it): only the sites next to a point in
    // the array plane can be that close
    const double s = ctx->tp.leaf_size, rmin = 0.5 * std::sqrt(2.0) * s;
    for (int i = 0; i < n_points; ++i) {
      const V3 q{points[3 * i], points[3 * i + 1], points[3 * i + 2]};
      if (std::fabs(q.z - ctx->origin.z) > rmin) continue;
      const long cx = std::lround((q.x - ctx->origin.x) / s), cy = std::lround((q.y - ctx->origin.y) / s);
      for (long jy = cy - 1; jy <= cy + 1; ++jy)
        for (long jx = cx - 1; jx <= cx + 1; ++jx) {
          if (jx < 0 || jy < 0 || jx >= ctx->nx || jy >= ctx->ny) continue;
          const int p = ctx->part_of_box[(size_t)jy * ctx->nx + jx];
          if (p >= 0 && norm(q - ctx->centers[p]) <= rmin)
            return fail(ctx, MLFMA_EINVAL, "observation point within half a leaf-box diagonal of a particle");
        }
    }
    std::string err;
    int rc = ctx->eng->fields(x_dev, R, n_points, points, E_dev, stream, err);
    return rc ? fail(ctx, rc, err) : MLFMA_OK;
  });
}

int mlfma_precondition(mlfma_ctx* ctx, const void* x_dev, void* y_dev, int32_t R, void* stream) {
  if (!ctx) return MLFMA_EINVAL;
  return guarded(ctx, [&]() -> int {
    if (!x_dev || !y_dev || R < 1 || x_dev == y_dev) return fail(ctx, MLFMA_EINVAL, "precondition arguments");
    if (int rc = do_prepare(ctx)) return rc;
    std::string err;
    int rc = ctx->eng->precondition(x_dev, y_dev, R, stream, err);
    return rc ? fail(ctx, rc, err) : MLFMA_OK;
  });
}

int mlfma_gmres_solve(mlfma_ctx* ctx, const void* b_dev, void* x_dev, int32_t R, double rtol, int32_t max_iter,
                      int32_t restart, int32_t flags, mlfma_solve_stats* stats, void* stream) {
  if (!ctx) return MLFMA_EINVAL;
  return guarded(ctx, [&]() -> int {
    if (!b_dev || !x_dev || R < 1 || !(rtol > 0) || max_iter < 1 || restart < 1 || restart > 1000 || b_dev == x_dev)
      return fail(ctx, MLFMA_EINVAL, "gmres arguments");
    if (int rc = do_prepare(ctx)) return rc;
    std::vector<GmresResult> res;
    std::string err;
    int rc = ctx->eng->gmres(b_dev, x_dev, R, rtol, max_iter, restart, (flags & MLFMA_SOLVE_USE_X0) != 0,
                              (flags & MLFMA_SOLVE_ALWAYS_REORTH) != 0, (flags & MLFMA_SOLVE_FP32_BASIS) != 0, res,
                              stream, err);
    if (rc) return fail(ctx, rc, err);
    bool all = true;
    for (int r = 0; r < R; ++r) {
      if (!std::isfinite(res[r].true_rel_res)) return fail(ctx, MLFMA_ENONFINITE, "non-finite residual");
      all &= res[r].converged != 0;
      if (stats) {
        stats[r].iterations = res[r].iterations;
        stats[r].true_rel_res = res[r].true_rel_res;
        stats[r].time_s = res[r].time_s;
        stats[r].converged = res[r].converged;
        stats[r].reorth = res[r].reorth;
        stats[r].cycles = res[r].cycles;
      }
    }
    if (!all) {
      ctx->err = "not converged within max_iter";
      return MLFMA_NOT_CONVERGED;
    }
    return MLFMA_OK;
  });
}

int mlfma_profile(mlfma_ctx* ctx, int32_t enable) {
  if (!ctx) return MLFMA_EINVAL;
  return guarded(ctx, [&]() -> int {
    if (int rc = do_prepare(ctx)) return rc;
    ctx->eng->profile(enable != 0);
    return MLFMA_OK;
  });
}

int mlfma_profile_read(mlfma_ctx* ctx, int32_t max, mlfma_stage_time* out, int32_t* count) {
  if (!ctx || !count || (max > 0 && !out)) return MLFMA_EINVAL;
  return guarded(ctx, [&]() -> int {
    if (!ctx->eng) return fail(ctx, MLFMA_ENOTREADY, "not prepared");
    std::vector<StageTime> t;
    std::string err;
    if (int rc = ctx->eng->profile_read(t, err)) return fail(ctx, rc, err);
    *count = (int32_t)t.size();
    for (int i = 0; i < (int)t.size() && i < max; ++i) {
      std::memset(out[i].name, 0, sizeof(out[i].name));
      std::strncpy(out[i].name, t[i].name.c_str(), sizeof(out[i].name) - 1);
      out[i].total_ms = t[i].total_ms;
      out[i].launches = t[i].launches;
      out[i].bytes_per_launch = t[i].bytes;
      out[i].flops_per_launch = t[i].flops;
      std::memset(out[i].kernel, 0, sizeof(out[i].kernel));
      std::strncpy(out[i].kernel, t[i].kernel.c_str(), sizeof(out[i].kernel) - 1);
    }
    return MLFMA_OK;
  });
}

int mlfma_info(const mlfma_ctx* ctx, mlfma_info_t* info) {
  if (!ctx || !info) return MLFMA_EINVAL;
  std::memset(info, 0, sizeof(*info));
  info->n_levels = ctx->tree.ntl;
  for (int l = 0; l < ctx->tree.ntl && l < 16; ++l) {
    info->L[l] = ctx->tree.lv[l].L;
    info->K[l] = ctx->tree.lv[l].K;
    info->nx[l] = ctx->tree.lv[l].nx;
    info->ny[l] = ctx->tree.lv[l].ny;
  }
  info->n_modes = ctx->N;
  info->n_unknowns = ctx->N > 0 ? (int64_t)2 * ctx->N * ctx->P : 0;
  info->device_bytes = ctx->eng ? ctx->eng->device_bytes() : 0;
  return MLFMA_OK;
}

void mlfma_destroy(mlfma_ctx* ctx) { delete ctx; }

const char* mlfma_last_error(const mlfma_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int mlfma_debug_near_block(mlfma_ctx* ctx, int32_t cp, int32_t cq, int32_t dx, int32_t dy, double* out) {
  if (!ctx || !out) return MLFMA_EINVAL;
  return guarded(ctx, [&]() -> int {
    if (cp < 0 || cq < 0 || cp >= ctx->C || cq >= ctx->C) return fail(ctx, MLFMA_EINVAL, "class out of range");
    if (!(*ctx->classes)[cp].set || !(*ctx->classes)[cq].set) return fail(ctx, MLFMA_ENOTREADY, "class not set");
    if (dx == 0 && dy == 0 && cp != cq) return fail(ctx, MLFMA_EINVAL, "two classes on one site");
    const auto& Z = near_block(ctx, cp, cq, dx, dy);
    std::memcpy(out, Z.data(), Z.size() * sizeof(cd));
    return MLFMA_OK;
  });
}

int mlfma_debug_pair_block_device(mlfma_ctx* ctx, int32_t cp, int32_t cq, int32_t dx, int32_t dy, double* out) {
  if (!ctx || !out) return MLFMA_EINVAL;
  return guarded(ctx, [&]() -> int {
    if (cp < 0 || cq < 0 || cp >= ctx->C || cq >= ctx->C) return fail(ctx, MLFMA_EINVAL, "class out of range");
    if (!(*ctx->classes)[cp].set || !(*ctx->classes)[cq].set) return fail(ctx, MLFMA_ENOTREADY, "class not set");
    if (dx == 0 && dy == 0) return fail(ctx, MLFMA_EINVAL, "not a pair of distinct sites");
    std::vector<PairSamples> smp(ctx->C);
    for (int c : {cp, cq}) smp[c] = {&(*ctx->classes)[c].mesh.qp, &(*ctx->classes)[c].mesh.qw, &(*ctx->classes)[c].smp.val, ctx->N};
    const double s = ctx->tp.leaf_size;
    std::vector<std::vector<cd>> T, K;
    std::string err;
    if (int rc = gpu_pair_blocks(smp, {PairRequest{cp, cq, V3{dx * s, dy * s, 0.0}}}, kK0, T, K, err))
      return fail(ctx, rc == -1 ? MLFMA_EINVAL : rc, err);
    const auto Z = assemble_pair(T[0], K[0], ctx->N);
    std::memcpy(out, Z.data(), Z.size() * sizeof(cd));
    return MLFMA_OK;
  });
}

int mlfma_debug_leaf_pattern(mlfma_ctx* ctx, int32_t c, double* out) {
  if (!ctx || !out) return MLFMA_EINVAL;
  if (c < 0 || c >= ctx->C || !(*ctx->classes)[c].set) return fail(ctx, MLFMA_ENOTREADY, "class not set");
  if (ctx->tree.ntl < 1) return fail(ctx, MLFMA_EINVAL, "no far-field levels");
  const LevelGrid& g = ctx->tree.lv[0];
  const int N = ctx->N;
  const auto& pat = (*ctx->classes)[c].leafpat;
  cd* o = reinterpret_cast<cd*>(out);
  for (int s = 0; s < g.K; ++s)
    for (int m = 0; m < N; ++m) {
      const cd* pv = &pat[(size_t)s * 3 * N];
      o[((size_t)s * 2 + 0) * N + m] = pv[m] * g.th_hat[s].x + pv[N + m] * g.th_hat[s].y + pv[2 * N + m] * g.th_hat[s].z;
      o[((size_t)s * 2 + 1) * N + m] = pv[m] * g.ph_hat[s].x + pv[N + m] * g.ph_hat[s].y + pv[2 * N + m] * g.ph_hat[s].z;
    }
  return MLFMA_OK;
}

int mlfma_debug_level_grid(mlfma_ctx* ctx, int32_t level, double* khat, double* w) {
  if (!ctx || !khat || !w) return MLFMA_EINVAL;
  if (level < 0 || level >= ctx->tree.ntl) return fail(ctx, MLFMA_EINVAL, "level out of range");
  const LevelGrid& g = ctx->tree.lv[level];
  for (int s = 0; s < g.K; ++s) {
    khat[3 * s] = g.khat[s].x;
    khat[3 * s + 1] = g.khat[s].y;
    khat[3 * s + 2] = g.khat[s].z;
    w[s] = g.w[s];
  }
  return MLFMA_OK;
}

int mlfma_debug_interpolate(mlfma_ctx* ctx, int32_t level, const double* in, double* out) {
  if (!ctx || !in || !out) return MLFMA_EINVAL;
  return guarded(ctx, [&]() -> int {
    if (level < 1 || level >= ctx->tree.ntl) return fail(ctx, MLFMA_EINVAL, "level out of range");
    const LevelGrid &c = ctx->tree.lv[level - 1], &p = ctx->tree.lv[level];
    const InterpTables& T = ctx->tree.it[level];
    const int ord = T.order;
    const cd* u = reinterpret_cast<const cd*>(in);
    cd* v = reinterpret_cast<cd*>(out);
    for (int it = 0; it < p.nt; ++it)
      for (int ip = 0; ip < p.np; ++ip)
        for (int comp = 0; comp < 2; ++comp) {
          cd acc = 0;
          for (int a = 0; a < ord; ++a) {
            const size_t ta = (size_t)it * ord + a;
            const int row = T.th_row[ta], shift = T.th_flip[ta] ? c.np / 2 : 0;
            cd rs = 0;
            for (int b = 0; b < ord; ++b) {
              const size_t pb = (size_t)ip * ord + b;
              const int col = (T.ph_col[pb] + shift) % c.np;
              rs += T.ph_w[pb] * u[((size_t)row * c.np + col) * 2 + comp];
            }
            acc += T.th_w[ta] * rs;
          }
          v[((size_t)it * p.np + ip) * 2 + comp] = acc;
        }
    return MLFMA_OK;
  });
}

int mlfma_debug_translation(mlfma_ctx* ctx, int32_t level, int32_t dx, int32_t dy, double* out) {
  if (!ctx || !out) return MLFMA_EINVAL;
  return guarded(ctx, [&]() -> int {
    if (level < 0 || level >= ctx->tree.ntl) return fail(ctx, MLFMA_EINVAL, "level out of range");
    if (dx == 0 && dy == 0) return fail(ctx, MLFMA_EINVAL, "zero separation");
    const LevelGrid& g = ctx->tree.lv[level];
    std::vector<cd> t;
    translation_function(g, V3{-dx * g.a, -dy * g.a, 0.0}, kK0, t);
    std::memcpy(out, t.data(), t.size() * sizeof(cd));
    return MLFMA_OK;
  });
}

}  // extern "C"

struct mlfma_mlp {
  mlfma::Mlp* m = nullptr;
  std::string err;
};

namespace {
int mlp_fail(mlfma_mlp* net, int code, const std::string& msg) {
  if (net) net->err = msg;
  return code;
}
template <typename F>
int mlp_guarded(mlfma_mlp* net, F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return mlp_fail(net, MLFMA_ENOMEM, "out of host memory");
  } catch (const std::exception& e) {
    return mlp_fail(net, MLFMA_EINVAL, e.what());
  }
}
}  // namespace

int mlfma_mlp_create(int32_t n_layers, const int32_t* sizes, uint64_t seed, mlfma_mlp** out) {
  if (!out || !sizes || n_layers < 1 || n_layers > 64) return MLFMA_EINVAL;
  *out = nullptr;
  auto* net = new (std::nothrow) mlfma_mlp();
  if (!net) return MLFMA_ENOMEM;
  std::vector<int> sz(sizes, sizes + n_layers + 1);
  std::string err;
  net->m = mlp_create(sz, seed, err);
  if (!net->m) {
    delete net;
    return err.find("failed") != std::string::npos ? MLFMA_EHIP : MLFMA_EINVAL;
  }
  *out = net;
  return MLFMA_OK;
}

void mlfma_mlp_destroy(mlfma_mlp* net) {
  if (!net) return;
  mlp_destroy(net->m);
  delete net;
}

const char* mlfma_mlp_last_error(const mlfma_mlp* net) { return net ? net->err.c_str() : "null network"; }

int64_t mlfma_mlp_num_params(const mlfma_mlp* net) { return net ? mlp_num_params(net->m) : -1; }

int mlfma_mlp_get_params(const mlfma_mlp* net, float* host) {
  if (!net || !host) return MLFMA_EINVAL;
  std::string err;
  int rc = mlp_get_params(net->m, host, err);
  return rc ? mlp_fail(const_cast<mlfma_mlp*>(net), rc, err) : MLFMA_OK;
}

int mlfma_mlp_set_params(mlfma_mlp* net, const float* host) {
  if (!net || !host) return MLFMA_EINVAL;
  for (int64_t i = 0; i < mlp_num_params(net->m); ++i)
    if (!std::isfinite(host[i])) return mlp_fail(net, MLFMA_ENONFINITE, "non-finite parameter");
  std::string err;
  int rc = mlp_set_params(net->m, host, err);
  return rc ? mlp_fail(net, rc, err) : MLFMA_OK;
}

int mlfma_mlp_forward(mlfma_mlp* net, const float* X_dev, int32_t n, float* Y_dev, void* stream) {
  if (!net || !X_dev || !Y_dev || n < 1) return MLFMA_EINVAL;
  return mlp_guarded(net, [&]() -> int {
    std::string err;
    int rc = mlp_forward(net->m, X_dev, n, Y_dev, stream, err);
    return rc ? mlp_fail(net, rc, err) : MLFMA_OK;
  });
}

int mlfma_mlp_loss_grad(mlfma_mlp* net, const float* X_dev, const float* T_dev, int32_t n, double* loss,
                        float* grads_host, void* stream) {
  if (!net || !X_dev || !T_dev || n < 1) return MLFMA_EINVAL;
  return mlp_guarded(net, [&]() -> int {
    std::string err;
    int rc = mlp_loss_grad(net->m, X_dev, T_dev, n, loss, grads_host, stream, err);
    return rc ? mlp_fail(net, rc, err) : MLFMA_OK;
  });
}

int mlfma_mlp_train_step(mlfma_mlp* net, const float* X_dev, const float* T_dev, int32_t n, float lr,
                         double* loss, void* stream) {
  if (!net || !X_dev || !T_dev || n < 1 || !(lr > 0)) return MLFMA_EINVAL;
  return mlp_guarded(net, [&]() -> int {
    std::string err;
    int rc = mlp_train_step(net->m, X_dev, T_dev, n, lr, loss, stream, err);
    if (rc) return mlp_fail(net, rc, err);
    if (loss && !std::isfinite(*loss)) return mlp_fail(net, MLFMA_ENONFINITE, "non-finite loss");
    return MLFMA_OK;
  });
}

namespace {
// features [R][P][C + 11] and incident phases [R][P] of the learned guess:
// one-hot class of p, class_param / scale of the 8 neighbouring sites (0 if
// empty), khat_x, khat_y, and the distance in sites to the nearest edge of
// the lattice, capped at kEdgeCap and divided by it
constexpr int kEdgeCap = 6;
int guess_nfeat(const mlfma_ctx* ctx) { return ctx->C + 11; }
void guess_features(const mlfma_ctx* ctx, const double* class_param, double scale, int R, const double* khat,
                    std::vector<float>& X, std::vector<cd>& phase) {
  const int P = ctx->P, nf = guess_nfeat(ctx);
  X.assign((size_t)R * P * nf, 0.f);
  phase.assign((size_t)R * P, cd(1.0, 0.0));
  for (int r = 0; r < R; ++r) {
    const V3 kh{khat[3 * r], khat[3 * r + 1], khat[3 * r + 2]};
    for (int p = 0; p < P; ++p) {
      float* f = &X[((size_t)r * P + p) * nf];
      const int ix = ctx->box_of[p] % ctx->nx, iy = ctx->box_of[p] / ctx->nx;
      f[ctx->cls[p]] = 1.f;
      int slot = ctx->C;
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          if (dx == 0 && dy == 0) continue;
          const int jx = ix + dx, jy = iy + dy;
          int q = -1;
          if (jx >= 0 && jy >= 0 && jx < ctx->nx && jy < ctx->ny) q = ctx->part_of_box[jy * ctx->nx + jx];
          f[slot++] = q >= 0 ? (float)(class_param[ctx->cls[q]] / scale) : 0.f;
        }
      f[slot++] = (float)kh.x;
      f[slot++] = (float)kh.y;
      const int edge = std::min(std::min(ix, iy), std::min(ctx->nx - 1 - ix, ctx->ny - 1 - iy));
      f[slot] = (float)std::min(edge, kEdgeCap) / kEdgeCap;
      const double a = -kK0 * dot(kh, ctx->centers[p]);
      phase[(size_t)r * P + p] = cd(std::cos(a), std::sin(a));
    }
  }
}
}  // namespace

int mlfma_guess_features(mlfma_ctx* ctx, const double* class_param, double scale, int32_t R, const double* khat,
                         float* X_host) {
  if (!ctx || !class_param || !khat || !X_host || R < 1 || !(scale > 0)) return MLFMA_EINVAL;
  return guarded(ctx, [&]() -> int {
    std::vector<float> X;
    std::vector<cd> phase;
    guess_features(ctx, class_param, scale, R, khat, X, phase);
    std::memcpy(X_host, X.data(), X.size() * sizeof(float));
    return MLFMA_OK;
  });
}

int mlfma_learned_guess(mlfma_ctx* ctx, mlfma_mlp* net, const double* class_param, double scale, int32_t R,
                        const double* khat, void* x_dev, void* stream) {
  if (!ctx || !net || !class_param || !khat || !x_dev || R < 1 || !(scale > 0)) return MLFMA_EINVAL;
  return guarded(ctx, [&]() -> int {
    if (ctx->N < 0) return fail(ctx, MLFMA_ENOTREADY, "no class has static modes");
    const int N = ctx->N, n = 2 * N, P = ctx->P;
    if (mlp_inputs(net->m) != guess_nfeat(ctx) || mlp_outputs(net->m) != 2 * n)
      return fail(ctx, MLFMA_EINVAL, "network must have n_classes + 11 inputs and 4N outputs");
    std::vector<float> X;
    std::vector<cd> phase;
    guess_features(ctx, class_param, scale, R, khat, X, phase);
    std::string err;
    int rc = mlp_guess(net->m, X, phase, R, P, N * 2, ctx->tp.precision == MLFMA_C128 ? 1 : 0, x_dev, stream,
                       err);
    return rc ? fail(ctx, rc == -1 ? MLFMA_EINVAL : rc, err) : MLFMA_OK;
  });
}
