// Coarse-grid MLP on MFMA: forward, backward, Adam (not in the paper; the
// learned stand-in for the exact coarse solve of Alg. fmg).
//
// Model: four dense layers n_in -> H -> H -> H -> n_out, ReLU between them.
// Weights and every layer input are stored in bfloat16 (round to nearest
// even); products run on the bf16 matrix cores with float32 accumulation
// (v_mfma_f32_16x16x16_bf16); biases, pre-activations, master weights and
// Adam moments are float32.  Loss: mean squared error over the n_out outputs.
#include <cmath>
#include <cstring>
#include <vector>

#include "kernels.h"
#include "mlp.h"

namespace hhg {
namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (unsigned short)((u >> 16) | 0x40);  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(((unsigned)b) << 16); }

// C[m][n] (+)= sum_p A(m, p) B(p, n), A(m,p) = A[m*sam + p*sap], B(p,n) =
// B[p*sbp + n*sbn], bf16 inputs, float32 output with leading dimension ldc.
// One wavefront per 16 x 16 tile of C; operand lanes: row/column = lane % 16,
// k = 4 (lane / 16) + q; result lanes: row 4 (lane / 16) + q, column lane % 16.
// Epilogue (Ep): bias != null: C = acc + bias[n]; act != null: act[m][n] =
// bf16(relu(C)) (relu != 0) or bf16(C) (ldc-strided, the next layer's input);
// mask != null: no C; gout[m][n] = bf16(acc * (bf16 mask[m][n] > 0)) (the
// ReLU backward of the previous layer).
struct GemmEpilogue {
  const float* bias = nullptr;
  unsigned short* act = nullptr;
  int relu = 0;
  const unsigned short* mask = nullptr;
  unsigned short* gout = nullptr;
};
__global__ void __launch_bounds__(64) k_gemm_bf16(int M, int N, int K, const unsigned short* __restrict__ A,
                                                  long sam, long sap, const unsigned short* __restrict__ B, long sbp,
                                                  long sbn, float* __restrict__ C, long ldc, int accumulate,
                                                  GemmEpilogue ep) {
  const int lane = threadIdx.x;
  const int tm = blockIdx.x * 16, tn = blockIdx.y * 16;
  const int r = lane & 15, kg = lane >> 4;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  const int m = tm + r, n = tn + r;
  for (int p0 = 0; p0 < K; p0 += 16) {
    v4s a, b;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int p = p0 + 4 * kg + q;
      a[q] = (short)((m < M && p < K) ? A[m * sam + p * sap] : 0);
      b[q] = (short)((n < N && p < K) ? B[p * sbp + n * sbn] : 0);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int mm = tm + 4 * kg + q;
    if (mm < M && n < N) {
      const long o = mm * ldc + n;
      if (ep.gout) {
        ep.gout[o] = f2bf(bf2f(ep.mask[o]) > 0.f ? acc[q] : 0.f);
        continue;
      }
      float v = accumulate ? C[o] + acc[q] : acc[q];
      if (ep.bias) v += ep.bias[n];
      C[o] = v;
      if (ep.act) ep.act[o] = f2bf(ep.relu ? fmaxf(v, 0.f) : v);
    }
  }
}

// Input features (float32, B x n_in) -> bf16, padded to Kpad columns.
__global__ void k_pack_input(int B, int n_in, int Kpad, const float* __restrict__ X, unsigned short* __restrict__ A0) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * Kpad) return;
  const int b = t / Kpad, k = t % Kpad;
  A0[t] = k < n_in ? f2bf(X[b * n_in + k]) : (unsigned short)0;
}

// Output (B x Npad float32) -> y (B x n_out float32).
__global__ void k_unpack_output(int B, int n_out, int Npad, const float* __restrict__ Z, float* __restrict__ y) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * n_out) return;
  y[t] = Z[(t / n_out) * Npad + t % n_out];
}

// MSE: g = bf16(2 (Z - Y) / (B n_out)) (0 in padding); per-block partial loss sums.
__global__ void __launch_bounds__(256) k_mse(int B, int n_out, int Npad, const float* __restrict__ Z,
                                             const float* __restrict__ Y, unsigned short* __restrict__ G,
                                             double* __restrict__ partial) {
  __shared__ double s[256];
  const int t = blockIdx.x * 256 + threadIdx.x;
  double l = 0.0;
  if (t < B * Npad) {
    const int b = t / Npad, n = t % Npad;
    float g = 0.f;
    if (n < n_out) {
      const float d = Z[t] - Y[b * n_out + n];
      l = (double)d * d;
      g = 2.f * d / (float)(B * n_out);
    }
    G[t] = f2bf(g);
  }
  s[threadIdx.x] = l;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

// acc[0] += sum of the block partials / (B n_out) (one workgroup, fixed order).
__global__ void __launch_bounds__(256) k_loss_accum(const double* __restrict__ partial, int nblk, double scale,
                                                    double* __restrict__ acc) {
  __shared__ double s[256];
  double a = 0.0;
  for (int q = threadIdx.x; q < nblk; q += 256) a += partial[q];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) acc[0] += s[0] * scale;
}

// db[n] = sum_b G[b][n] for n < N (bf16 inputs, float32 sum)
__global__ void k_colsum(int B, int N, int Npad, const unsigned short* __restrict__ G, float* __restrict__ db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += bf2f(G[b * Npad + n]);
  db[n] = s;
}

// Adam on float32 masters; bf16 copies of weight matrices refreshed.
__global__ void k_adam(long n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, unsigned short* __restrict__ pb, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float gg = g[t];
  const float mm = b1 * m[t] + (1.f - b1) * gg;
  const float vv = b2 * v[t] + (1.f - b2) * gg * gg;
  m[t] = mm;
  v[t] = vv;
  const float w = p[t] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  p[t] = w;
  if (pb) pb[t] = f2bf(w);
}

__global__ void k_fill_f64(double* __restrict__ x, int n) {
  if ((int)threadIdx.x < n) x[threadIdx.x] = 0.0;
}

__global__ void k_to_bf16(long n, const float* __restrict__ p, unsigned short* __restrict__ pb) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) pb[t] = f2bf(p[t]);
}

unsigned nb(long n, int b = 256) { return (unsigned)((n + b - 1) / b); }
int pad16(int n) { return (n + 15) & ~15; }

}  // namespace

// ------------------------------------------------------------------ host
Mlp::~Mlp() {
  for (void* p : allocs) (void)hipFree(p);
}

void Mlp::init(int in, int H, int out, int max_b) {
  n_in = in, hidden = H, n_out = out, max_batch = max_b;
  kin = pad16(in), kout = pad16(out), bpad = pad16(max_b);
  rows[0] = H, cols[0] = kin;
  rows[1] = H, cols[1] = H;
  rows[2] = H, cols[2] = H;
  rows[3] = kout, cols[3] = H;
  nparams_dev = 0;
  for (int l = 0; l < 4; ++l) {
    woff[l] = nparams_dev;
    nparams_dev += (long)rows[l] * cols[l];
    boff[l] = nparams_dev;
    nparams_dev += rows[l];
  }
  auto al = [&](size_t bytes) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes ? bytes : 4);
    if (e != hipSuccess) throw Error{HHG_ERR_OOM, "hipMalloc (mlp)"};
    allocs.push_back(p);
    HHG_CHECK_HIP(hipMemset(p, 0, bytes ? bytes : 4));
    return p;
  };
  P = (float*)al(nparams_dev * 4);
  Gr = (float*)al(nparams_dev * 4);
  Mo = (float*)al(nparams_dev * 4);
  Vo = (float*)al(nparams_dev * 4);
  Pb = (unsigned short*)al(nparams_dev * 2);
  A0 = (unsigned short*)al((size_t)bpad * kin * 2);
  for (int l = 0; l < 4; ++l) {
    Z[l] = (float*)al((size_t)bpad * rows[l] * 4);
    G[l] = (unsigned short*)al((size_t)bpad * rows[l] * 2);
    if (l < 3) Ab[l] = (unsigned short*)al((size_t)bpad * rows[l] * 2);
  }
  dA = (float*)al((size_t)bpad * H * 4);
  partial = (double*)al(sizeof(double) * ((size_t)bpad * kout / 256 + 2));
  loss_acc = (double*)al(sizeof(double) * 2);
  step = 0;
}

long Mlp::host_params() const {
  long n = 0;
  const int r[4] = {hidden, hidden, hidden, n_out}, c[4] = {n_in, hidden, hidden, hidden};
  for (int l = 0; l < 4; ++l) n += (long)r[l] * c[l] + r[l];
  return n;
}

void Mlp::set_params(const float* host) {
  std::vector<float> dev(nparams_dev, 0.f);
  const int r[4] = {hidden, hidden, hidden, n_out}, c[4] = {n_in, hidden, hidden, hidden};
  long q = 0;
  for (int l = 0; l < 4; ++l) {
    for (int i = 0; i < r[l]; ++i)
      for (int j = 0; j < c[l]; ++j) dev[woff[l] + (long)i * cols[l] + j] = host[q++];
    for (int i = 0; i < r[l]; ++i) dev[boff[l] + i] = host[q++];
  }
  HHG_CHECK_HIP(hipMemcpy(P, dev.data(), nparams_dev * 4, hipMemcpyHostToDevice));
  HHG_CHECK_HIP(hipMemset(Mo, 0, nparams_dev * 4));
  HHG_CHECK_HIP(hipMemset(Vo, 0, nparams_dev * 4));
  hipLaunchKernelGGL(k_to_bf16, dim3(nb(nparams_dev)), dim3(256), 0, 0, nparams_dev, P, Pb);
  HHG_CHECK_HIP(hipDeviceSynchronize());
  step = 0;
}

void Mlp::unpack(const float* dev_vec, float* host) const {
  std::vector<float> dev(nparams_dev);
  HHG_CHECK_HIP(hipMemcpy(dev.data(), dev_vec, nparams_dev * 4, hipMemcpyDeviceToHost));
  const int r[4] = {hidden, hidden, hidden, n_out}, c[4] = {n_in, hidden, hidden, hidden};
  long q = 0;
  for (int l = 0; l < 4; ++l) {
    for (int i = 0; i < r[l]; ++i)
      for (int j = 0; j < c[l]; ++j) host[q++] = dev[woff[l] + (long)i * cols[l] + j];
    for (int i = 0; i < r[l]; ++i) host[q++] = dev[boff[l] + i];
  }
}

static void gemm(hipStream_t s, int M, int N, int K, const unsigned short* A, long sam, long sap,
                 const unsigned short* B, long sbp, long sbn, float* C, long ldc, int acc,
                 const GemmEpilogue& ep = GemmEpilogue()) {
  KScope ks(s, KF_MLP, 2.0 * M * N * K);
  // one wavefront per 16 x 16 tile: these products (batch <= 256, widths <= 512)
  // are small, and the finest tiling spreads them over the most CUs (a
  // 64 x 64 LDS-tiled form measured 3x slower here)
  hipLaunchKernelGGL(k_gemm_bf16, dim3((M + 15) / 16, (N + 15) / 16), dim3(64), 0, s, M, N, K, A, sam, sap, B, sbp,
                     sbn, C, ldc, acc, ep);
}

void Mlp::forward_dev(hipStream_t s, const float* x, int B) {
  hipLaunchKernelGGL(k_pack_input, dim3(nb((long)B * kin)), dim3(256), 0, s, B, n_in, kin, x, A0);
  const unsigned short* a = A0;
  int ka = kin;
  for (int l = 0; l < 4; ++l) {
    // Z[b][n] = sum_k a[b][k] W[n][k] + bias[n]; hidden layers: Ab = bf16(relu(Z))
    // (padded output columns: zero weights and bias, so Z = 0 there)
    GemmEpilogue ep;
    ep.bias = P + boff[l];
    ep.act = l < 3 ? Ab[l] : nullptr;
    ep.relu = 1;
    gemm(s, B, rows[l], ka, a, ka, 1, Pb + woff[l], 1, cols[l], Z[l], rows[l], 0, ep);
    if (l < 3) {
      a = Ab[l];
      ka = rows[l];
    }
  }
}

void Mlp::forward(hipStream_t s, const float* x, int B, float* y) {
  forward_dev(s, x, B);
  hipLaunchKernelGGL(k_unpack_output, dim3(nb((long)B * n_out)), dim3(256), 0, s, B, n_out, kout, Z[3], y);
}

void Mlp::loss_grad_dev(hipStream_t s, const float* x, const float* y, int B, double* loss_acc) {
  forward_dev(s, x, B);
  const long nG = (long)B * kout;
  const unsigned nblk = nb(nG);
  hipLaunchKernelGGL(k_mse, dim3(nblk), dim3(256), 0, s, B, n_out, kout, Z[3], y, G[3], partial);
  hipLaunchKernelGGL(k_loss_accum, dim3(1), dim3(256), 0, s, partial, (int)nblk, 1.0 / ((double)B * n_out),
                     loss_acc);
  for (int l = 3; l >= 0; --l) {
    const unsigned short* a = l > 0 ? Ab[l - 1] : A0;
    const int ka = l > 0 ? rows[l - 1] : kin;
    // dW[n][k] = sum_b G[b][n] a[b][k]
    gemm(s, rows[l], ka, B, G[l], 1, rows[l], a, ka, 1, Gr + woff[l], cols[l], 0);
    hipLaunchKernelGGL(k_colsum, dim3(nb(rows[l])), dim3(256), 0, s, B, rows[l], rows[l], G[l], Gr + boff[l]);
    if (l > 0) {
      // dA[b][k] = sum_n G[b][n] W[n][k], then G[l-1] = bf16(dA * (A[l-1] > 0)) in the epilogue
      GemmEpilogue ep;
      ep.mask = Ab[l - 1];
      ep.gout = G[l - 1];
      gemm(s, B, ka, rows[l], G[l], rows[l], 1, Pb + woff[l], cols[l], 1, dA, ka, 0, ep);
    }
  }
}

double Mlp::loss_grad(hipStream_t s, const float* x, const float* y, int B) {
  hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, loss_acc, 2);
  loss_grad_dev(s, x, y, B, loss_acc);
  double l = 0.0;
  HHG_CHECK_HIP(hipMemcpyAsync(&l, loss_acc, sizeof(double), hipMemcpyDeviceToHost, s));
  HHG_CHECK_HIP(hipStreamSynchronize(s));
  return l;
}

void Mlp::train_step_dev(hipStream_t s, const float* x, const float* y, int B, float lr, double* loss_acc) {
  loss_grad_dev(s, x, y, B, loss_acc);
  ++step;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(nb(nparams_dev)), dim3(256), 0, s, nparams_dev, P, Gr, Mo, Vo, Pb, lr, b1, b2,
                     1e-8f, c1, c2);
}

}  // namespace hhg
