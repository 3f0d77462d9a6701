// Coarse-grid MLP (device state and host driver); see mlp.hip.
#pragma once
#include <vector>

#include "hhg_internal.h"

namespace hhg {

struct Mlp {
  int n_in = 0, hidden = 0, n_out = 0, max_batch = 0;
  int kin = 0, kout = 0, bpad = 0;     // padded to multiples of 16
  int rows[4], cols[4];                // device layer shapes (padded)
  long woff[4], boff[4], nparams_dev = 0;
  float *P = nullptr, *Gr = nullptr, *Mo = nullptr, *Vo = nullptr;  // params, grads, Adam moments (float32)
  unsigned short* Pb = nullptr;        // bf16 copy of the params
  unsigned short* A0 = nullptr;        // bf16 input
  float* Z[4] = {nullptr, nullptr, nullptr, nullptr};             // pre-activations (float32)
  unsigned short* Ab[3] = {nullptr, nullptr, nullptr};            // bf16 hidden activations
  unsigned short* G[4] = {nullptr, nullptr, nullptr, nullptr};    // bf16 gradients wrt pre-activations
  float* dA = nullptr;
  double* partial = nullptr;
  double* loss_acc = nullptr;          // device loss accumulator (2 doubles)
  long step = 0;
  std::vector<void*> allocs;

  ~Mlp();
  void init(int n_in, int hidden, int n_out, int max_batch);
  long host_params() const;                       // unpadded parameter count
  void set_params(const float* host);             // host order W1,b1,...,W4,b4 (row-major W)
  void unpack(const float* dev_vec, float* host) const;
  void forward_dev(hipStream_t s, const float* x, int B);          // output in Z[3]
  void forward(hipStream_t s, const float* x, int B, float* y);
  // grads in Gr; *_dev add the batch's mean loss to loss_acc[0] on the device (no host sync)
  void loss_grad_dev(hipStream_t s, const float* x, const float* y, int B, double* loss_acc);
  double loss_grad(hipStream_t s, const float* x, const float* y, int B);
  void train_step_dev(hipStream_t s, const float* x, const float* y, int B, float lr, double* loss_acc);
};

}  // namespace hhg
