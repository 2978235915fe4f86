/*
 * mlfma.h -- C ABI of the MI355X (gfx950) MLFMA-SMR library.
 *
 * The library applies and solves the static-mode PMCHWT system of
 * Corsaro et al., "Multilevel Fast Multipole Algorithm for Electromagnetic
 * Scattering by Large Metasurfaces using Static Mode Representation":
 *
 *   Z J = V   (Sec. II, eqs. PMCHWT_finite / Zpq_delta)
 *
 * for p particles, each carrying N = N_perp + N_par static modes (Sec. III)
 * for its electric and for its magnetic equivalent current, i.e. 2N unknowns
 * per particle.  The product Z x is computed by the multilevel fast multipole
 * algorithm of Sec. IV: near blocks (self and adjacent particles) applied
 * directly; far interactions by leaf radiation patterns (eq. kspace_Rap),
 * aggregation with Lagrange interpolation and phase shifts, diagonal
 * translation (eqs. addition_th / translation_fun), disaggregation
 * (anterpolation) and receiving patterns (eqs. Tmn_fmm / Kmn_fmm).
 *
 * Conventions
 *  - Time dependence exp(+j w t).  Lengths are in wavelengths of the
 *    background medium, so k- = 2 pi; the background impedance is the unit
 *    of impedance (zeta- = 1); mu = 1 everywhere.
 *  - Unknown layout: [R][P][2][N] complex, interleaved (re, im), in the
 *    context precision (complex float for MLFMA_C64, complex double for
 *    MLFMA_C128): for right-hand side r and particle p, first the N
 *    electric-current coefficients J_e (transverse modes first), then the N
 *    magnetic ones J_m (Sec. II.A eq. galerkin ordering).
 *  - Galerkin entries: T_mn = <psi_m, L psi_n> with L the field operator of
 *    an electric current over zeta, K_mn = <psi_m, int psi_n x grad g>;
 *    blocks [[z-T- + z+T+, K- + K+], [-(K- + K+), T-/z- + T+/z+]] (eq.
 *    Zpq_delta), exterior only between distinct particles.  Right-hand side
 *    V = -[<psi, E_inc>; <psi, H_inc>].
 *
 * Status codes: 0 success, < 0 error, > 0 warning.  Every call that takes a
 * context records a message readable with mlfma_last_error().  No call
 * throws across the ABI or terminates the process.  A context is not
 * thread-safe: calls on one context must be serialised by the caller.
 */
#ifndef MLFMA_H
#define MLFMA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MLFMA_OK = 0,
  MLFMA_EINVAL = -1,     /* invalid argument, size or layout              */
  MLFMA_ENOMEM = -2,     /* host or device allocation failed              */
  MLFMA_EHIP = -3,       /* a HIP runtime call failed (no GPU, fault)      */
  MLFMA_ENOTREADY = -4,  /* a particle class in use has no static modes    */
  MLFMA_ENONFINITE = -5, /* NaN/Inf in an input or a breakdown             */
  MLFMA_NOT_CONVERGED = 1
};

/* MLFMA_C64: complex FP32 data and arithmetic (FP32 matrix-core products);
 * MLFMA_C128: complex FP64; MLFMA_C64_BF16: complex FP32 data with the dense
 * contractions (near field, projection, receive) as three BF16 matrix-core
 * products per FP32 product (a_hi b_hi + a_hi b_lo + a_lo b_hi, each operand
 * split into a BF16 head and a BF16 remainder), accumulated in FP32. */
enum { MLFMA_C64 = 0, MLFMA_C128 = 1, MLFMA_C64_BF16 = 2 };

/* Parts of the operator applied by mlfma_matvec_parts(). */
enum { MLFMA_PART_NEAR = 1, MLFMA_PART_FAR = 2, MLFMA_PART_ALL = 3 };

typedef struct mlfma_ctx mlfma_ctx;

/* Particle array (Sec. II problem statement; Sec. IV grouping: every
 * particle is a finest-level group).  Centres must lie on one plane z = z0
 * at the sites origin + (i, j) * leaf_size of a square lattice, at most one
 * particle per site (empty sites are allowed).
 * Background medium (Sec. II: particles (eps+, mu+) in a background
 * (eps-, mu-), here mu = 1 everywhere): eps_bg is eps- relative to vacuum,
 * and the permittivities given to mlfma_set_static_modes are relative to
 * vacuum as well.  With lengths in wavelengths of the background and zeta-
 * as the unit of impedance, the operator depends on the media only through
 * eps+ / eps- (k+ / k- = sqrt(eps+ / eps-), zeta+ / zeta- = 1 / that), which
 * is how the library uses eps_bg.  eps_bg must be real and positive (a
 * lossy background would make k- complex); 0 + 0j reads as 1 (vacuum), so
 * a zero-initialised struct keeps the vacuum background.  EINVAL otherwise. */
typedef struct {
  int32_t n_particles;      /* P >= 1                                     */
  const double* centers;    /* [P][3], background wavelengths             */
  const int32_t* class_id;  /* [P], 0 <= class_id < n_classes             */
  int32_t n_classes;        /* number of particle shapes/materials        */
  double eps_bg_re;         /* background permittivity eps- (real part)   */
  double eps_bg_im;         /* imaginary part: must be 0                  */
} mlfma_problem;

/* Tree and accuracy parameters (Sec. IV; Sec. V: L = 10 at the finest
 * level, K = 2 L^2 directions, 4 x 4 Lagrange interpolation). */
typedef struct {
  double leaf_size;      /* finest box edge = lattice pitch (0.5)           */
  int32_t L_leaf;        /* truncation at the finest level (default 11, the
                            excess-bandwidth rule at a 0.5 leaf; the paper
                            uses 10)                                        */
  int32_t L_rule;        /* coarser levels: 0 = excess-bandwidth rule
                            L = kd + 1.8 d0^(2/3) (kd)^(1/3), d = sqrt2 a;
                            1 = doubling per level                          */
  double digits;         /* d0 of the excess-bandwidth rule (3)             */
  int32_t interp_order;  /* points per direction of the Lagrange stencil
                            (default 6; 4 = the paper's 4 x 4)              */
  int32_t precision;     /* MLFMA_C64, MLFMA_C128 or MLFMA_C64_BF16          */
  int32_t outer_levels;  /* subdivision levels of the outer triangle in the
                            singular (touching-pair) quadrature (2)         */
  int32_t near_rule;     /* which pairs take the direct (near) blocks: 0 =
                            the particles in adjacent finest-level boxes,
                            the 3 x 3 block of boxes around a particle's
                            own (Sec. IV); the only rule (EINVAL otherwise) */
} mlfma_tree_params;

typedef struct {
  int32_t n_levels;          /* levels with translations                   */
  int32_t L[16];             /* truncation per level (leaf first)          */
  int32_t K[16];             /* directions per level = 2 L^2               */
  int32_t nx[16], ny[16];    /* boxes per level                            */
  int64_t n_unknowns;        /* 2 N P                                      */
  int32_t n_modes;           /* N                                          */
  int64_t device_bytes;      /* device memory held by the context          */
} mlfma_info_t;

typedef struct {
  int32_t iterations;    /* GMRES iterations (matrix-vector products)      */
  double true_rel_res;   /* ||V - Z x|| / ||V|| recomputed at exit         */
  double time_s;         /* wall time of the solve                         */
  int32_t converged;     /* 1 if true_rel_res <= rtol                      */
  int32_t reorth;        /* iterations that took a second Gram-Schmidt pass */
  int32_t cycles;        /* restart cycles                                  */
} mlfma_solve_stats;

/* Fill *tp with the defaults: leaf 0.5, L_leaf 11, rule 0, digits 3,
 * interp_order 6, MLFMA_C64, outer_levels 2, near_rule 0. */
void mlfma_default_params(mlfma_tree_params* tp);

/* Build the quadtree, interaction lists and sphere grids for a particle
 * array.  Host-only: makes no HIP call.  The library copies every input;
 * the caller keeps ownership of pb's arrays.  On success *out owns a new
 * context, released with mlfma_destroy().
 * Errors: EINVAL (null pointers, P < 1, class ids out of range, centres not
 * on one lattice plane, two particles on one site, bad parameters, a
 * background permittivity that is not real and positive). */
int mlfma_build_tree(const mlfma_problem* pb, const mlfma_tree_params* tp, mlfma_ctx** out);

/* Static modes of one closed particle surface (Sec. III): the N_perp
 * transverse modes of eq. AuxProb_Tt (loop functions, largest eigenvalues)
 * followed by the N_par longitudinal modes of eq. AuxProb_Tl (star
 * functions, smallest eigenvalues).  Host-only, FP64.
 *  verts [nv][3], tris [nt][3] (counter-clockwise seen from outside),
 *  edges [ne][4] = (v0, v1, t_plus, t_minus): t_plus has the directed edge
 *  v0 -> v1, t_minus has v1 -> v0.  RWG f_e is +(l/2A)(r - p) on t_plus and
 *  -(l/2A)(r - p) on t_minus, p the vertex opposite the edge.
 * Output: M_out [(n_perp+n_par)][ne] RWG coefficients (caller-allocated),
 * each mode with unit norm <psi, psi> = 1 and its largest-magnitude
 * coefficient positive; gamma_out [(n_perp+n_par)] eigenvalues (may be
 * NULL).  Errors: EINVAL (inconsistent mesh, too many modes), ENONFINITE. */
int mlfma_static_modes(int32_t nv, const double* verts, int32_t nt, const int32_t* tris, int32_t ne,
                       const int32_t* edges, int32_t n_perp, int32_t n_par, double* M_out,
                       double* gamma_out);

/* Attach the mesh, static modes and permittivity of particle class
 * `class_id` (mesh in particle-local coordinates, centred on the particle
 * centre; eps_re + j eps_im is eps+ relative to vacuum, divided by the
 * problem's eps_bg inside).  M is [(n_perp+n_par)][ne] as produced by mlfma_static_modes.
 * Computes in FP64 on the host: the leaf radiation/receiving patterns of
 * eq. kspace_Rap, the self block Z_s of eq. Zpq_delta (singular quadrature
 * on touching triangle pairs), and its inverse for the block-diagonal
 * preconditioner.  Host-only; copies every input.  All classes must share
 * the same n_perp + n_par.  Errors: EINVAL, ENONFINITE. */
int mlfma_set_static_modes(mlfma_ctx* ctx, int32_t class_id, int32_t nv, const double* verts, int32_t nt,
                           const int32_t* tris, int32_t ne, const int32_t* edges, int32_t n_perp,
                           int32_t n_par, const double* M, double eps_re, double eps_im);

/* Compute the neighbour blocks and translation tables and upload every
 * table to the current HIP device.  Called implicitly by the first
 * mlfma_matvec / mlfma_gmres_solve / mlfma_plane_wave_rhs.
 * Errors: ENOTREADY (a class in use has no modes), EHIP, ENOMEM. */
int mlfma_prepare(mlfma_ctx* ctx);

/* Right-hand side of a plane wave E = pol exp(-j k khat . r) (Sec. II:
 * e0 = -n x n x E_inc tested with the modes), H = khat x E / zeta-:
 * b = -[<psi, E_inc>; <psi, H_inc>] for R incidences.
 *  khat [R][3] unit vectors; pol [R][3] complex interleaved (re, im);
 *  b_dev: device buffer [R][P][2][N] complex in the context precision.
 * Asynchronous on `stream` (hipStream_t, NULL = default stream). */
int mlfma_plane_wave_rhs(mlfma_ctx* ctx, int32_t R, const double* khat, const double* pol, void* b_dev,
                         void* stream);

/* y = Z x for R right-hand sides (the hot path, Sec. IV).  x_dev, y_dev:
 * caller-owned device buffers [R][P][2][N] in the context precision,
 * 16-byte aligned; they must not overlap (EINVAL otherwise).  Asynchronous on `stream`; no host
 * synchronisation.  Scratch pattern buffers are held by the context and
 * grow to the largest R seen. */
int mlfma_matvec(mlfma_ctx* ctx, const void* x_dev, void* y_dev, int32_t R, void* stream);

/* y = Z x as mlfma_matvec, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the product's pattern buffers (and the class-pair near
 * partials) are laid out in a static device array of the library, 64 MiB per
 * GPU, held until the process ends; the call makes no allocation, no graph
 * and no memset (the leaf buffer is cleared by a kernel) and launches the
 * kernels of mlfma_matvec directly on `stream`.  The context must already be
 * prepared (mlfma_prepare or any earlier call that prepares it; ENOTREADY
 * otherwise).  EINVAL if the buffers for R RHS exceed the 64 MiB (about a
 * 40 x 40 array at R = 1; larger arrays use mlfma_matvec).  Every call on a
 * GPU shares that GPU's array and leaves its contents behind: calls that
 * overlap on one GPU (two streams, two threads, two contexts) race and must
 * be serialised by the caller. */
int mlfma_matvec_noalloc(mlfma_ctx* ctx, const void* x_dev, void* y_dev, int32_t R, void* stream);

/* As mlfma_matvec, restricted to the near part (self + adjacent blocks),
 * the far part (multilevel expansion), or both (MLFMA_PART_*). */
int mlfma_matvec_parts(mlfma_ctx* ctx, const void* x_dev, void* y_dev, int32_t R, int32_t parts,
                       void* stream);

/* dst uses src's per-class setup (modes, self blocks, patterns) and its
 * cache of neighbour blocks from now on, so that many arrays of the same
 * particle classes are prepared without repeating the per-class work.  Both
 * contexts must have the same class count and tree parameters.  The shared
 * data stays alive while either context does; mlfma_set_static_modes on
 * either context changes it for both, and the two must not be used from
 * different threads at once. */
int mlfma_share_setup(mlfma_ctx* dst, const mlfma_ctx* src);

/* Block-diagonal preconditioner y_p = Z_s^-1 x_p (Sec. V stage v), same
 * layout and precision as mlfma_matvec. */
int mlfma_precondition(mlfma_ctx* ctx, const void* x_dev, void* y_dev, int32_t R, void* stream);

#define MLFMA_SOLVE_USE_X0 1
#define MLFMA_SOLVE_ALWAYS_REORTH 2
#define MLFMA_SOLVE_FP32_BASIS 4

/* Right-preconditioned restarted GMRES (Sec. V stage v; preconditioner
 * blockdiag(Z_s)) for R right-hand sides solved in lock-step.  Arnoldi is
 * classical Gram-Schmidt with a second pass where the first removed more
 * than half of |w|^2 (Daniel-Gragg-Kaufman-Stewart test), or always with
 * flags & MLFMA_SOLVE_ALWAYS_REORTH.  Arnoldi and Givens rotations are
 * FP64; the Krylov basis is stored in FP64, or in FP32 with flags &
 * MLFMA_SOLVE_FP32_BASIS (half the memory and traffic of the Arnoldi
 * sweeps, basis orthogonal to FP32 rounding); the matrix-vector products run
 * in the context precision.
 *  b_dev, x_dev: device [R][P][2][N] in the context precision.  x_dev holds
 *  the initial guess if flags & MLFMA_SOLVE_USE_X0 (else zero is used) and
 *  the best iterate on return.  A guess x0 is first scaled by the complex
 *  factor a = (Z x0)^H b / |Z x0|^2 that minimises |b - a Z x0|, so it never
 *  starts worse than zero (a = 0 for a guess orthogonal to b).  rtol: relative tolerance on the true
 *  residual; max_iter: total matrix-vector products per RHS; restart: Krylov
 *  dimension m.  stats [R] (may be NULL).  Synchronous: returns after the
 *  solution is in x_dev.  Returns MLFMA_NOT_CONVERGED (1) if some RHS did
 *  not reach rtol within max_iter.
 *  Kernels are launched one by one; with the environment variable
 *  MLFMA_GMRES_GRAPHS set when the context is prepared, each product and
 *  each Arnoldi step is instead one replayed HIP graph (the same results
 *  bit for bit; slower on ROCm 7, where each graph boundary idles the GPU
 *  for a few microseconds). */
int mlfma_gmres_solve(mlfma_ctx* ctx, const void* b_dev, void* x_dev, int32_t R, double rtol,
                      int32_t max_iter, int32_t restart, int32_t flags, mlfma_solve_stats* stats,
                      void* stream);

/* Work division of the interpolation kernels and the matrix-core GEMMs:
 * agg_rows[l] parent theta rows per streaming chunk of the aggregation into
 * level l (l >= 1), dis_rows[l] extended child theta rows per chunk of the
 * disaggregation into level l (l < n_levels - 1); 0 selects the built-in
 * planner (chunks that fill the chip for the launch's batch size).  set
 * re-plans the chunks (the product's arithmetic and its order are
 * unchanged, only which wave forms an output) and fails with EINVAL for a
 * negative value; get returns the values set (0: planner).  Prepares the
 * context if needed.  Used by the autotuner of the binding. */
#define MLFMA_MAX_LEVELS 16
typedef struct {
  int32_t n_levels;
  int32_t agg_rows[MLFMA_MAX_LEVELS];
  int32_t dis_rows[MLFMA_MAX_LEVELS];
  int32_t gemm_rows_near;     /* 16-row MFMA tiles per block of the near +   */
  int32_t gemm_rows_receive;  /* projection and receive GEMMs: 1, 2, 4 (0: 4) */
} mlfma_tuning;
int mlfma_set_tuning(mlfma_ctx* ctx, const mlfma_tuning* t);
int mlfma_get_tuning(mlfma_ctx* ctx, mlfma_tuning* t);

/* Scattered electric field of the currents x at observation points (the
 * near/focal fields of Sec. V): E(r) = sum_p E_p(r) with each particle's
 * field expanded about its centre c_p, from its leaf radiation pattern U_p
 * (eq. kspace_Rap, the product's projection stage) and the translation
 * operator of eq. translation_fun taken to the point itself:
 *   E(r) = -jk sum_p sum_s w_s T_L(khat_s, r - c_p) (U_th,p(s) th_s + U_ph,p(s) ph_s)
 * over the leaf sphere samples s.  Exact to the leaf level's truncation for
 * any point outside the particle's circumscribing sphere.
 *  x_dev: device [R][P][2][N] currents in the context precision;
 *  points: host FP64 [n_points][3]; each must lie farther than half a leaf-
 *  box diagonal from every particle centre (EINVAL otherwise);
 *  E_dev: device [R][n_points][3] complex in the context precision.
 *  Needs at least one far level and a leaf sphere of at most 256 samples
 *  (L_leaf <= 11).  Returns after E_dev is written (synchronises stream). */
int mlfma_fields(mlfma_ctx* ctx, const void* x_dev, int32_t R, int32_t n_points, const double* points, void* E_dev,
                 void* stream);

/* Per-kernel timing: while enabled, every kernel launch of mlfma_matvec is
 * bracketed by HIP events recorded on the launch stream.  Enabling clears
 * the accumulated table. */
typedef struct {
  char name[32];               /* stage and level, e.g. "aggregate_l1"     */
  double total_ms;             /* summed event time over the launches      */
  int64_t launches;
  double bytes_per_launch;     /* algorithmic HBM bytes of one launch      */
  double flops_per_launch;     /* algorithmic real floating-point ops      */
  char kernel[96];             /* symbol of the launched kernel with its
                                  template arguments, e.g.
                                  "k_dis_stream<float, 6, 12, 16>" (the unit
                                  kernel traces report; "" if unknown)     */
} mlfma_stage_time;

int mlfma_profile(mlfma_ctx* ctx, int32_t enable);
/* Synchronises the recorded events and returns up to `max` rows. */
int mlfma_profile_read(mlfma_ctx* ctx, int32_t max, mlfma_stage_time* out, int32_t* count);

int mlfma_info(const mlfma_ctx* ctx, mlfma_info_t* info);
void mlfma_destroy(mlfma_ctx* ctx);
const char* mlfma_last_error(const mlfma_ctx* ctx);

/* Diagnostic accessors of host-side setup tables (FP64, interleaved
 * complex), for tests.  Host-only.
 *  near_block: Z^{mu nu} for a particle of class cp observing one of class
 *    cq displaced by (dx, dy) lattice steps (dx = dy = 0 and cp == cq: the
 *    self block); out [2N][2N] row-major.  Computed on demand by host
 *    quadrature, or after mlfma_prepare the block the product uses.
 *  leaf_pattern: receiving pattern psi_hat of class c at the finest-level
 *    directions, out [K0][2 (theta, phi)][N].
 *  level_grid: directions khat [K][3] and quadrature weights w [K] of level l.
 *  translation: T_L of eq. translation_fun at level l for the source box
 *    displaced by (dx, dy) boxes, out [K]. */
int mlfma_debug_near_block(mlfma_ctx* ctx, int32_t cp, int32_t cq, int32_t dx, int32_t dy, double* out);
/* The same block between distinct sites (dx, dy) != (0, 0) as
 * mlfma_debug_near_block, assembled by the GPU quadrature that prepare uses
 * (FP64; needs a GPU).  out: [2N][2N] complex row-major. */
int mlfma_debug_pair_block_device(mlfma_ctx* ctx, int32_t cp, int32_t cq, int32_t dx, int32_t dy, double* out);
int mlfma_debug_leaf_pattern(mlfma_ctx* ctx, int32_t c, double* out);
int mlfma_debug_level_grid(mlfma_ctx* ctx, int32_t level, double* khat, double* w);
int mlfma_debug_translation(mlfma_ctx* ctx, int32_t level, int32_t dx, int32_t dy, double* out);
/* The separable Lagrange interpolation of aggregation (Sec. IV: a pattern
 * sampled at level l - 1 resampled on the finer grid of level l, before
 * the phase shift to the parent centre), applied on the host in FP64 with
 * the stencil tables the kernels use: in [K_{l-1}][2] and out [K_l][2]
 * (theta, phi components; interleaved complex; sample index row * np + col).
 * A stencil tap across a pole reads the row at phi + pi with both transverse
 * components negated.  1 <= level < n_levels.  Host-only. */
int mlfma_debug_interpolate(mlfma_ctx* ctx, int32_t level, const double* in, double* out);

/* ------------------------------------------------ learned initial guess --
 * A fully connected ReLU network, trained on solutions the method itself
 * produces on small arrays, maps each particle's class, its eight
 * neighbours' geometry parameters and the incidence direction to its
 * static-mode coefficients; the prediction is the GMRES initial guess
 * (mlfma_gmres_solve with MLFMA_SOLVE_USE_X0, which scales it to its least
 * residual; the zero start is the limit of that scaling).
 * The paper has no such network: this is an addition around its solver (the
 * solution vector of Sec. V stage v).  All network arithmetic is FP32 on
 * the GPU.  A network is not tied to a context. */
typedef struct mlfma_mlp mlfma_mlp;

/* sizes[0..n_layers]: inputs, hidden widths, outputs; weights He-normal
 * from `seed` (splitmix64 + Box-Muller), biases zero.  EINVAL on bad sizes. */
int mlfma_mlp_create(int32_t n_layers, const int32_t* sizes, uint64_t seed, mlfma_mlp** out);
void mlfma_mlp_destroy(mlfma_mlp* net);
const char* mlfma_mlp_last_error(const mlfma_mlp* net);
/* Parameters as one FP32 vector: for each layer W [out][in] row-major, then
 * b [out].  set_params also clears the Adam moments. */
int64_t mlfma_mlp_num_params(const mlfma_mlp* net);
int mlfma_mlp_get_params(const mlfma_mlp* net, float* host);
int mlfma_mlp_set_params(mlfma_mlp* net, const float* host);
/* Y [n][out] = net(X [n][in]); device FP32 pointers; asynchronous on stream. */
int mlfma_mlp_forward(mlfma_mlp* net, const float* X_dev, int32_t n, float* Y_dev, void* stream);
/* loss = 0.5/n * sum over samples and outputs of (net(X) - T)^2, T [n][out]
 * on the device; the gradient (parameter layout) is copied to grads_host
 * when not NULL.  Synchronous. */
int mlfma_mlp_loss_grad(mlfma_mlp* net, const float* X_dev, const float* T_dev, int32_t n, double* loss,
                        float* grads_host, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the
 * minibatch; *loss = the loss before the step.  Synchronous. */
int mlfma_mlp_train_step(mlfma_mlp* net, const float* X_dev, const float* T_dev, int32_t n, float lr,
                         double* loss, void* stream);

/* The features described below, [R][P][n_classes + 11] FP32, on the host
 * (the inputs a network for mlfma_learned_guess is trained on).  Host-only. */
int mlfma_guess_features(mlfma_ctx* ctx, const double* class_param, double scale, int32_t R, const double* khat,
                         float* X_host);
/* Writes the network's prediction for R plane-wave incidences (directions
 * khat [R][3]) into x_dev [R][P][2][N] (context precision).  Features of
 * particle p, in this order: one-hot of its class (n_classes entries; the
 * static-mode basis differs between classes), class_param[class] / scale
 * of the 8 neighbouring sites (dy, dx in -1..1 row-major, centre skipped;
 * 0 where a site holds no particle), khat_x, khat_y, and the distance in
 * sites from p to the nearest edge of the lattice, capped at 6, over 6.
 * The network outputs
 * (re, im) of the 2N coefficients with the incident phase removed; the
 * guess multiplies them by exp(-j k khat . r_p).  EINVAL if the network
 * does not have n_classes + 11 inputs and 4N outputs.  Synchronous. */
int mlfma_learned_guess(mlfma_ctx* ctx, mlfma_mlp* net, const double* class_param, double scale, int32_t R,
                        const double* khat, void* x_dev, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MLFMA_H */
