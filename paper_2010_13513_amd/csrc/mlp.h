// Coarse-grid MLP (device state and host driver); see mlp.hip.
#pragma once
#include <vector>

#include "hhg_internal.h"

namespace hhg {

// Offsets and (padded) shapes of the four weight matrices in the parameter vector.
struct WShapes {
  long off[4];
  int rows[4], cols[4];
};

struct Mlp {
  int n_in = 0, hidden = 0, n_out = 0, max_batch = 0;
  int kin = 0, kout = 0, bpad = 0;     // padded to multiples of 16
  int rows[4], cols[4];                // device layer shapes (padded)
  long woff[4], boff[4], nparams_dev = 0;
  float *P = nullptr, *Gr = nullptr, *Mo = nullptr, *Vo = nullptr;  // params, grads, Adam moments (float32)
  unsigned short* Pb = nullptr;        // bf16 copy of the params
  unsigned short* PbT = nullptr;       // bf16 transposed weight matrices (same offsets, cols x rows)
  unsigned short* A0 = nullptr;        // bf16 input
  unsigned short* A0T = nullptr;       // and transposed (kin x bpad), for the weight gradients
  float* Z[4] = {nullptr, nullptr, nullptr, nullptr};             // pre-activations (float32)
  unsigned short* Ab[3] = {nullptr, nullptr, nullptr};            // bf16 hidden activations
  unsigned short* AbT[3] = {nullptr, nullptr, nullptr};           // transposed (rows x bpad)
  unsigned short* G[4] = {nullptr, nullptr, nullptr, nullptr};    // bf16 gradients wrt pre-activations
  unsigned short* GT[4] = {nullptr, nullptr, nullptr, nullptr};   // transposed (rows x bpad)
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
  // output in Z[3]; rows idx[b] of x (idx null: rows 0..B-1); train: also the
  // transposed activations for the backward products
  void forward_dev(hipStream_t s, const float* x, const int* idx, int B, bool train);
  void transpose_weights(hipStream_t s);           // PbT from Pb
  WShapes shapes() const;
  void forward(hipStream_t s, const float* x, int B, float* y);
  // grads in Gr; *_dev add the batch's mean loss to loss_acc[0] on the device (no host sync)
  void loss_grad_dev(hipStream_t s, const float* x, const float* y, const int* idx, int B, double* loss_acc);
  double loss_grad(hipStream_t s, const float* x, const float* y, int B);
  // minibatch = rows idx[0..B) of the data sets x, y
  void train_step_dev(hipStream_t s, const float* x, const float* y, const int* idx, int B, float lr,
                      double* loss_acc);
};

}  // namespace hhg
