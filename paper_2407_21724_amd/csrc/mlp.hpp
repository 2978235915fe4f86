// Fully connected ReLU network of the learned initial guess (FP32 on the
// device): forward, mean-squared-error gradients, Adam, and the scatter of
// its outputs into a right-hand-side-shaped solution vector.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

namespace mlfma {

class Mlp;

Mlp* mlp_create(const std::vector<int>& sizes, uint64_t seed, std::string& err);
void mlp_destroy(Mlp* m);
int64_t mlp_num_params(const Mlp* m);
int mlp_get_params(const Mlp* m, float* host, std::string& err);
int mlp_set_params(Mlp* m, const float* host, std::string& err);
int mlp_inputs(const Mlp* m);
int mlp_outputs(const Mlp* m);
// Y [n][out] = net(X [n][in]), device pointers.
int mlp_forward(Mlp* m, const float* X, int n, float* Y, void* stream, std::string& err);
// loss = 0.5 / n * sum |net(X) - T|^2; grads (host, parameter layout) if not null.
int mlp_loss_grad(Mlp* m, const float* X, const float* T, int n, double* loss, float* grads, void* stream,
                  std::string& err);
// one Adam step; *loss = the loss before the step
int mlp_train_step(Mlp* m, const float* X, const float* T, int n, float lr, double* loss, void* stream,
                   std::string& err);
// x[r][p][j] = (Y[r*P+p][2j] + i Y[r*P+p][2j+1]) * phase[r*P+p] in the
// context precision (0: complex float, 1: complex double); X features
// [R*P][in] on the host.
int mlp_guess(Mlp* m, const std::vector<float>& X, const std::vector<std::complex<double>>& phase, int R, int P,
              int n, int precision, void* x_dev, void* stream, std::string& err);

}  // namespace mlfma
