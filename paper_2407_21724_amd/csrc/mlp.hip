// Learned initial guess network on gfx950: FP32 matrix-core GEMMs with LDS
// tiles for the layers and their gradients, plus the elementwise kernels of
// the loss, the ReLU masks, the bias gradients and Adam.  See mlp.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "mlp.hpp"

namespace mlfma {
namespace {

#define MLP_TRY(expr)                                                     \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess) {                                               \
      err = std::string(#expr " failed: ") + hipGetErrorString(e_);       \
      return -3;                                                          \
    }                                                                     \
  } while (0)

constexpr int kT = 256;
typedef float f32x4 __attribute__((ext_vector_type(4)));

// C(m, n) (+)= sum_k A(m, k) B(k, n) with arbitrary element strides:
// A(m, k) = A[m*sa0 + k*sa1], B(k, n) = B[k*sb0 + n*sb1], C at m*sc0 + n*sc1.
// Epilogue: + bias[m] (if set), then ReLU (relu) or a multiply by
// (mask(m, n) > 0) with mask at m*sc0 + n*sc1 (if set).  Block tile 64 x 64,
// K in chunks of 16 through LDS; wave w owns rows [16w, 16w + 16) as four
// 16 x 16 tiles of v_mfma_f32_16x16x4f32 (A[i][k] from lane i + 16k, B[k][j]
// from lane j + 16k, result row 4*(lane/16) + v, column lane % 16).
struct Gemm {
  const float* A;
  const float* B;
  float* C;
  const float* bias;
  const float* mask;
  long sa0, sa1, sb0, sb1, sc0, sc1;
  int M, N, K, accumulate, relu;
};

__global__ __launch_bounds__(kT) void k_gemm(Gemm g) {
  __shared__ float As[64][17];
  __shared__ float Bs[16][65];
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = lane & 15, kq = lane >> 4;
  f32x4 acc[4];
  for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < g.K; k0 += 16) {
    for (int e = threadIdx.x; e < 64 * 16; e += kT) {
      const int r = e / 16, c = e % 16;
      const int m = m0 + r, k = k0 + c;
      As[r][c] = (m < g.M && k < g.K) ? g.A[(long)m * g.sa0 + (long)k * g.sa1] : 0.f;
      const int kb = e / 64, nb = e % 64;
      const int k2 = k0 + kb, n = n0 + nb;
      Bs[kb][nb] = (k2 < g.K && n < g.N) ? g.B[(long)k2 * g.sb0 + (long)n * g.sb1] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const float a = As[wave * 16 + i][kk * 4 + kq];
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, Bs[kk * 4 + kq][t * 16 + i], acc[t], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = m0 + wave * 16 + 4 * kq + v, n = n0 + t * 16 + i;
      if (m >= g.M || n >= g.N) continue;
      const long o = (long)m * g.sc0 + (long)n * g.sc1;
      float c = acc[t][v];
      if (g.accumulate) c += g.C[o];
      if (g.bias) c += g.bias[m];
      if (g.relu) c = fmaxf(c, 0.f);
      if (g.mask && !(g.mask[o] > 0.f)) c = 0.f;
      g.C[o] = c;
    }
}

// G[j][s] = (Y[j][s] - T[s][j]) / n (feature-major G, Y; sample-major T) and
// per-block partial sums of (Y - T)^2 in double.
__global__ __launch_bounds__(kT) void k_mse(int out, int n, int ld, const float* __restrict__ Y,
                                            const float* __restrict__ T, float* __restrict__ G,
                                            double* __restrict__ part) {
  __shared__ double red[kT / 64];
  double s2 = 0;
  const long cnt = (long)out * n;
  for (long e = (long)blockIdx.x * kT + threadIdx.x; e < cnt; e += (long)gridDim.x * kT) {
    const int j = (int)(e / n), s = (int)(e % n);
    const float d = Y[(long)j * ld + s] - T[(long)s * out + j];
    G[(long)j * ld + s] = d / (float)n;
    s2 += (double)d * d;
  }
  for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < kT / 64; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

// db[j] = sum_s G[j][s]  (one block per row, fixed order)
__global__ __launch_bounds__(kT) void k_rowsum(int n, int ld, const float* __restrict__ G, float* __restrict__ db) {
  __shared__ float red[kT / 64];
  const int j = blockIdx.x;
  float s = 0.f;
  for (int e = threadIdx.x; e < n; e += kT) s += G[(long)j * ld + e];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int w = 0; w < kT / 64; ++w) t += red[w];
    db[j] = t;
  }
}

// Adam (beta1, beta2, eps; bias corrections c1 = 1 - beta1^t, c2 = 1 - beta2^t)
__global__ __launch_bounds__(kT) void k_adam(long cnt, float* __restrict__ p, const float* __restrict__ g,
                                             float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                             float b2, float eps, float c1, float c2) {
  for (long e = (long)blockIdx.x * kT + threadIdx.x; e < cnt; e += (long)gridDim.x * kT) {
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  }
}

// x[r][p][j] = (Y[s][2j] + i Y[s][2j+1]) * phase[s], s = r * P + p
template <typename T>
__global__ __launch_bounds__(kT) void k_guess(int S, int n, const float* __restrict__ Y,
                                              const double* __restrict__ phase, T* __restrict__ x) {
  const long cnt = (long)S * n;
  for (long e = (long)blockIdx.x * kT + threadIdx.x; e < cnt; e += (long)gridDim.x * kT) {
    const int s = (int)(e / n), j = (int)(e % n);
    const double re = Y[(long)s * 2 * n + 2 * j], im = Y[(long)s * 2 * n + 2 * j + 1];
    const double pr = phase[2 * s], pi = phase[2 * s + 1];
    x[2 * e] = (T)(re * pr - im * pi);
    x[2 * e + 1] = (T)(re * pi + im * pr);
  }
}

__global__ __launch_bounds__(kT) void k_relu_copy(long cnt, const float* __restrict__ a, float* __restrict__ b,
                                                  int relu) {
  for (long e = (long)blockIdx.x * kT + threadIdx.x; e < cnt; e += (long)gridDim.x * kT)
    b[e] = relu ? fmaxf(a[e], 0.f) : a[e];
}

// Y[s][j] = act[j][s] (feature-major to sample-major)
__global__ __launch_bounds__(kT) void k_to_samples(int out, int n, const float* __restrict__ a, float* __restrict__ Y) {
  const long cnt = (long)out * n;
  for (long e = (long)blockIdx.x * kT + threadIdx.x; e < cnt; e += (long)gridDim.x * kT) {
    const int s = (int)(e / out), j = (int)(e % out);
    Y[e] = a[(long)j * n + s];
  }
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    std::swap(p, o.p);
    std::swap(bytes, o.bytes);
    return *this;
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t ensure(size_t b) {
    if (b <= bytes) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipMalloc(&p, b);
    if (e == hipSuccess) bytes = b;
    return e;
  }
  float* f() const { return static_cast<float*>(p); }
  double* d() const { return static_cast<double*>(p); }
};

int grid(long work) { return (int)std::max<long>(1, std::min<long>((work + kT - 1) / kT, 4096)); }

uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

class Mlp {
 public:
  std::vector<int> sizes;
  std::vector<long> woff, boff;  // offsets of each layer's W [out][in] and b [out] in the parameter vector
  long nparam = 0;
  DevBuf params, grads, m1, m2;
  std::vector<DevBuf> act, pre;  // per layer, feature-major [width][n]
  DevBuf gcur, gprev, part;
  int n_cap = 0;
  long step = 0;

  int layers() const { return (int)sizes.size() - 1; }

  int ensure_batch(int n, std::string& err) {
    if (n <= n_cap) return 0;
    act.resize(layers());
    pre.resize(layers());
    int widest = sizes[0];
    for (int l = 0; l < layers(); ++l) {
      MLP_TRY(act[l].ensure((size_t)sizes[l + 1] * n * sizeof(float)));
      MLP_TRY(pre[l].ensure((size_t)sizes[l + 1] * n * sizeof(float)));
      widest = std::max(widest, sizes[l + 1]);
    }
    MLP_TRY(gcur.ensure((size_t)widest * n * sizeof(float)));
    MLP_TRY(gprev.ensure((size_t)widest * n * sizeof(float)));
    MLP_TRY(part.ensure(4096 * sizeof(double)));
    n_cap = n;
    return 0;
  }

  void gemm(const Gemm& g, hipStream_t st) {
    hipLaunchKernelGGL(k_gemm, dim3((g.M + 63) / 64, (g.N + 63) / 64), dim3(kT), 0, st, g);
  }

  // forward pass on X [n][in] (sample-major); pre-activations and outputs
  // of every layer kept feature-major
  void forward(const float* X, int n, hipStream_t st) {
    for (int l = 0; l < layers(); ++l) {
      Gemm g{};
      g.A = params.f() + woff[l];
      g.sa0 = sizes[l];
      g.sa1 = 1;
      if (l == 0) {
        g.B = X;
        g.sb0 = 1;
        g.sb1 = sizes[0];
      } else {
        g.B = act[l - 1].f();
        g.sb0 = n;
        g.sb1 = 1;
      }
      g.C = pre[l].f();
      g.sc0 = n;
      g.sc1 = 1;
      g.bias = params.f() + boff[l];
      g.M = sizes[l + 1];
      g.N = n;
      g.K = sizes[l];
      gemm(g, st);
      const long cnt = (long)g.M * n;
      hipLaunchKernelGGL(k_relu_copy, dim3(grid(cnt)), dim3(kT), 0, st, cnt, (const float*)pre[l].f(), act[l].f(),
                         l + 1 < layers() ? 1 : 0);
    }
  }

  // gradients of 0.5/n sum |net(X) - T|^2 into `grads`; returns the loss
  int backward(const float* X, const float* T, int n, double* loss, hipStream_t st, std::string& err) {
    const int L = layers(), out = sizes[L];
    const int nb = grid((long)out * n);
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(kT), 0, st, out, n, n, (const float*)act[L - 1].f(), T, gcur.f(),
                       part.d());
    std::vector<double> hp(nb);
    MLP_TRY(hipMemcpyAsync(hp.data(), part.p, nb * sizeof(double), hipMemcpyDeviceToHost, st));
    for (int l = L - 1; l >= 0; --l) {
      // dW = G H_{l-1}^T  (H_{-1} = X)
      Gemm g{};
      g.A = gcur.f();
      g.sa0 = n;
      g.sa1 = 1;
      if (l == 0) {
        g.B = X;
        g.sb0 = sizes[0];
        g.sb1 = 1;
      } else {
        g.B = act[l - 1].f();
        g.sb0 = 1;
        g.sb1 = n;
      }
      g.C = grads.f() + woff[l];
      g.sc0 = sizes[l];
      g.sc1 = 1;
      g.M = sizes[l + 1];
      g.N = sizes[l];
      g.K = n;
      gemm(g, st);
      hipLaunchKernelGGL(k_rowsum, dim3(sizes[l + 1]), dim3(kT), 0, st, n, n, (const float*)gcur.f(),
                         grads.f() + boff[l]);
      if (l == 0) break;
      // G_{l-1} = (W^T G) * (pre_{l-1} > 0)
      Gemm b{};
      b.A = params.f() + woff[l];
      b.sa0 = 1;
      b.sa1 = sizes[l];
      b.B = gcur.f();
      b.sb0 = n;
      b.sb1 = 1;
      b.C = gprev.f();
      b.sc0 = n;
      b.sc1 = 1;
      b.mask = pre[l - 1].f();
      b.M = sizes[l];
      b.N = n;
      b.K = sizes[l + 1];
      gemm(b, st);
      std::swap(gcur, gprev);
    }
    MLP_TRY(hipGetLastError());
    MLP_TRY(hipStreamSynchronize(st));
    double s = 0;
    for (double v : hp) s += v;
    if (loss) *loss = 0.5 * s / n;
    return 0;
  }
};

Mlp* mlp_create(const std::vector<int>& sizes, uint64_t seed, std::string& err) {
  if (sizes.size() < 2) {
    err = "a network needs at least an input and an output size";
    return nullptr;
  }
  for (int v : sizes)
    if (v < 1 || v > 65536) {
      err = "layer sizes must be in [1, 65536]";
      return nullptr;
    }
  auto* m = new Mlp();
  m->sizes = sizes;
  long off = 0;
  for (size_t l = 0; l + 1 < sizes.size(); ++l) {
    m->woff.push_back(off);
    off += (long)sizes[l] * sizes[l + 1];
    m->boff.push_back(off);
    off += sizes[l + 1];
  }
  m->nparam = off;
  // He-normal weights (Box-Muller on a splitmix64 stream), zero biases
  std::vector<float> h(off, 0.f);
  uint64_t st = seed;
  for (size_t l = 0; l + 1 < sizes.size(); ++l) {
    const double sd = std::sqrt(2.0 / sizes[l]);
    for (long e = 0; e < (long)sizes[l] * sizes[l + 1]; ++e) {
      const double u1 = ((splitmix64(st) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
      const double u2 = ((splitmix64(st) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
      h[m->woff[l] + e] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * 3.14159265358979323846 * u2));
    }
  }
  if (mlp_set_params(m, h.data(), err)) {
    delete m;
    return nullptr;
  }
  return m;
}

void mlp_destroy(Mlp* m) { delete m; }
int64_t mlp_num_params(const Mlp* m) { return m->nparam; }
int mlp_inputs(const Mlp* m) { return m->sizes.front(); }
int mlp_outputs(const Mlp* m) { return m->sizes.back(); }

int mlp_get_params(const Mlp* m, float* host, std::string& err) {
  MLP_TRY(hipMemcpy(host, m->params.p, m->nparam * sizeof(float), hipMemcpyDeviceToHost));
  return 0;
}

int mlp_set_params(Mlp* m, const float* host, std::string& err) {
  const size_t b = m->nparam * sizeof(float);
  MLP_TRY(m->params.ensure(b));
  MLP_TRY(m->grads.ensure(b));
  MLP_TRY(m->m1.ensure(b));
  MLP_TRY(m->m2.ensure(b));
  MLP_TRY(hipMemcpy(m->params.p, host, b, hipMemcpyHostToDevice));
  MLP_TRY(hipMemset(m->m1.p, 0, b));
  MLP_TRY(hipMemset(m->m2.p, 0, b));
  m->step = 0;
  return 0;
}

int mlp_forward(Mlp* m, const float* X, int n, float* Y, void* stream, std::string& err) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (int rc = m->ensure_batch(n, err)) return rc;
  m->forward(X, n, st);
  const int out = m->sizes.back();
  hipLaunchKernelGGL(k_to_samples, dim3(grid((long)out * n)), dim3(kT), 0, st, out, n,
                     (const float*)m->act.back().f(), Y);
  MLP_TRY(hipGetLastError());
  return 0;
}

int mlp_loss_grad(Mlp* m, const float* X, const float* T, int n, double* loss, float* grads, void* stream,
                  std::string& err) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (int rc = m->ensure_batch(n, err)) return rc;
  m->forward(X, n, st);
  if (int rc = m->backward(X, T, n, loss, st, err)) return rc;
  if (grads) MLP_TRY(hipMemcpy(grads, m->grads.p, m->nparam * sizeof(float), hipMemcpyDeviceToHost));
  return 0;
}

int mlp_train_step(Mlp* m, const float* X, const float* T, int n, float lr, double* loss, void* stream,
                   std::string& err) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (int rc = m->ensure_batch(n, err)) return rc;
  m->forward(X, n, st);
  if (int rc = m->backward(X, T, n, loss, st, err)) return rc;
  m->step++;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = (float)(1.0 - std::pow(0.9, (double)m->step)), c2 = (float)(1.0 - std::pow(0.999, (double)m->step));
  hipLaunchKernelGGL(k_adam, dim3(grid(m->nparam)), dim3(kT), 0, st, m->nparam, m->params.f(),
                     (const float*)m->grads.f(), m->m1.f(), m->m2.f(), lr, b1, b2, 1e-8f, c1, c2);
  MLP_TRY(hipGetLastError());
  return 0;
}

int mlp_guess(Mlp* m, const std::vector<float>& X, const std::vector<std::complex<double>>& phase, int R, int P,
              int n, int precision, void* x_dev, void* stream, std::string& err) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int S = R * P, in = m->sizes.front();
  if ((long)X.size() != (long)S * in || m->sizes.back() != 2 * n) {
    err = "network inputs/outputs do not match the features / unknowns per particle";
    return -1;
  }
  DevBuf dx, dy, dph;
  MLP_TRY(dx.ensure(X.size() * sizeof(float)));
  MLP_TRY(dy.ensure((size_t)S * 2 * n * sizeof(float)));
  MLP_TRY(dph.ensure((size_t)S * 2 * sizeof(double)));
  MLP_TRY(hipMemcpyAsync(dx.p, X.data(), X.size() * sizeof(float), hipMemcpyHostToDevice, st));
  MLP_TRY(hipMemcpyAsync(dph.p, phase.data(), (size_t)S * 2 * sizeof(double), hipMemcpyHostToDevice, st));
  if (int rc = mlp_forward(m, dx.f(), S, dy.f(), stream, err)) return rc;
  const long cnt = (long)S * n;
  if (precision == 1)
    hipLaunchKernelGGL(k_guess<double>, dim3(grid(cnt)), dim3(kT), 0, st, S, n, (const float*)dy.f(),
                       (const double*)dph.d(), static_cast<double*>(x_dev));
  else
    hipLaunchKernelGGL(k_guess<float>, dim3(grid(cnt)), dim3(kT), 0, st, S, n, (const float*)dy.f(),
                       (const double*)dph.d(), static_cast<float*>(x_dev));
  MLP_TRY(hipGetLastError());
  MLP_TRY(hipStreamSynchronize(st));  // the staging buffers are released on return
  return 0;
}

}  // namespace mlfma
