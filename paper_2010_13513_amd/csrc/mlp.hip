// Coarse-grid MLP on MFMA: forward, backward, Adam (not in the paper; the
// learned stand-in for the exact coarse solve of Alg. fmg).
//
// Model: four dense layers n_in -> H -> H -> H -> n_out, ReLU between them.
// Weights and every layer input are stored in bfloat16 (round to nearest
// even); products run on the bf16 matrix cores with float32 accumulation
// (v_mfma_f32_16x16x32_bf16); biases, pre-activations, master weights and
// Adam moments are float32.  Loss: mean squared error over the n_out outputs.
#include <algorithm>
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

// C[m][n] = sum_k A[m][k] B[n][k] (both operands row-major with the
// contraction index contiguous: lda, ldb in elements, multiples of 8), bf16
// inputs, float32 output with leading dimension ldc.  One wavefront per
// 16 x 16 tile of C on v_mfma_f32_16x16x32_bf16: lane l holds A row
// l % 16 and B row l % 16 at k = 8 (l / 16) + 0..7 of each 32-wide k step
// (one 16-byte load per operand; the same k slots for both operands, so the
// product is the full sum over k whatever order the unit adds the slots in);
// result lanes: row 4 (l / 16) + q, column l % 16.  A k tail (K not a
// multiple of 32) is loaded element by element and zero-filled.
// rowsum != null: the blocks of the first column of tiles also write the row
// sums of A (the bias gradient of the weight-gradient product).
// Epilogue: bias != null: C = acc + bias[n]; act != null: act[m][n] =
// bf16(relu(C)) (relu != 0) or bf16(C), actT != null: the same into
// actT[n][m] (leading dimension ldt); mask != null: no C, gout[m][n] =
// bf16(acc * (bf16 mask[m][n] > 0)) (the ReLU backward of the previous
// layer), goutT likewise transposed.
struct GemmEpilogue {
  const float* bias = nullptr;
  unsigned short* act = nullptr;
  unsigned short* actT = nullptr;
  int relu = 0;
  const unsigned short* mask = nullptr;
  unsigned short* gout = nullptr;
  unsigned short* goutT = nullptr;
  long ldt = 0;
  float* rowsum = nullptr;  // != null: rowsum[m] = sum_k A[m][k] (from the tiles of the first column block)
};
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned short v8us __attribute__((ext_vector_type(8)));

__device__ __forceinline__ v8bf load8(const unsigned short* __restrict__ row, int k, int K, bool in) {
  v8us v = {0, 0, 0, 0, 0, 0, 0, 0};
  if (in) {
    if (k + 8 <= K) {
      v = *reinterpret_cast<const v8us*>(row + k);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = k + e < K ? row[k + e] : (unsigned short)0;
    }
  }
  return __builtin_bit_cast(v8bf, v);
}

constexpr int kKSteps = 16;  // 32-wide k steps held in registers at once (k chunk 512)

__global__ void __launch_bounds__(64) k_gemm_bf16(int M, int N, int K, const unsigned short* __restrict__ A, long lda,
                                                  const unsigned short* __restrict__ B, long ldb,
                                                  float* __restrict__ C, long ldc, GemmEpilogue ep) {
  const int lane = threadIdx.x;
  const int tm = blockIdx.x * 16, tn = blockIdx.y * 16;
  const int r = lane & 15, kg = lane >> 4;
  const int m = tm + r, n = tn + r;
  const unsigned short* arow = A + (long)min(m, M - 1) * lda;
  const unsigned short* brow = B + (long)min(n, N - 1) * ldb;
  const bool rsum = ep.rowsum && blockIdx.y == 0;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  float asum = 0.f;
  // a whole k chunk of both operands is loaded before the first product, so
  // the wavefront waits for memory once per chunk, not once per step
  for (int c0 = 0; c0 < K; c0 += 32 * kKSteps) {
    v8bf a[kKSteps], b[kKSteps];
#pragma unroll
    for (int st = 0; st < kKSteps; ++st) {
      const int k = c0 + 32 * st + 8 * kg;
      const bool live = c0 + 32 * st < K;
      a[st] = load8(arow, k, K, live && m < M);
      b[st] = load8(brow, k, K, live && n < N);
    }
#pragma unroll
    for (int st = 0; st < kKSteps; ++st)
      if (c0 + 32 * st < K) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[st], b[st], acc, 0, 0, 0);
        if (rsum)
#pragma unroll
          for (int e = 0; e < 8; ++e) asum += (float)a[st][e];
      }
  }
  if (rsum) {  // sum over the four k lane groups of row r
    asum += __shfl_xor(asum, 16);
    asum += __shfl_xor(asum, 32);
    if (kg == 0 && m < M) ep.rowsum[m] = asum;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int mm = tm + 4 * kg + q;
    if (mm < M && n < N) {
      const float a = acc[q];
      const long o = mm * ldc + n;
      if (ep.gout) {
        const unsigned short g = f2bf(bf2f(ep.mask[o]) > 0.f ? a : 0.f);
        ep.gout[o] = g;
        if (ep.goutT) ep.goutT[n * ep.ldt + mm] = g;
        continue;
      }
      float v = a;
      if (ep.bias) v += ep.bias[n];
      C[o] = v;
      if (ep.act) {
        const unsigned short h = f2bf(ep.relu ? fmaxf(v, 0.f) : v);
        ep.act[o] = h;
        if (ep.actT) ep.actT[n * ep.ldt + mm] = h;
      }
    }
  }
}

// out[c][r] = in[r][c] for the four weight matrices (bf16, blockIdx.y =
// layer): the transposed copies feed the input-gradient products.
__global__ void k_transpose_w(WShapes w, const unsigned short* __restrict__ in, unsigned short* __restrict__ out) {
  const int l = blockIdx.y;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long n = (long)w.rows[l] * w.cols[l];
  if (t >= n) return;
  const int r = (int)(t / w.cols[l]), c = (int)(t % w.cols[l]);
  out[w.off[l] + (long)c * w.rows[l] + r] = in[w.off[l] + t];
}

// Input features (float32, B x n_in) -> bf16, padded to Kpad columns, and
// (A0T != null) transposed into A0T[k][b] (leading dimension ldt).
__global__ void k_pack_input(int B, int n_in, int Kpad, const float* __restrict__ X, const int* __restrict__ idx,
                             unsigned short* __restrict__ A0, unsigned short* __restrict__ A0T, long ldt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * Kpad) return;
  const int b = t / Kpad, k = t % Kpad;
  const long row = idx ? idx[b] : b;  // sample row of the data set (minibatch gather)
  const unsigned short v = k < n_in ? f2bf(X[row * n_in + k]) : (unsigned short)0;
  A0[t] = v;
  if (A0T) A0T[k * ldt + b] = v;
}

// Output (B x Npad float32) -> y (B x n_out float32).
__global__ void k_unpack_output(int B, int n_out, int Npad, const float* __restrict__ Z, float* __restrict__ y) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * n_out) return;
  y[t] = Z[(t / n_out) * Npad + t % n_out];
}

// MSE: g = bf16(2 (Z - Y) / (B n_out)) (0 in padding); per-block partial loss sums.
__global__ void __launch_bounds__(256) k_mse(int B, int n_out, int Npad, const float* __restrict__ Z,
                                             const float* __restrict__ Y, const int* __restrict__ idx,
                                             unsigned short* __restrict__ G, unsigned short* __restrict__ GT,
                                             long ldt, double* __restrict__ partial) {
  __shared__ double s[256];
  const int t = blockIdx.x * 256 + threadIdx.x;
  double l = 0.0;
  if (t < B * Npad) {
    const int b = t / Npad, n = t % Npad;
    float g = 0.f;
    if (n < n_out) {
      const float d = Z[t] - Y[(idx ? (long)idx[b] : (long)b) * n_out + n];
      l = (double)d * d;
      g = 2.f * d / (float)(B * n_out);
    }
    G[t] = f2bf(g);
    GT[n * ldt + b] = G[t];
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

// Adam on float32 masters; bf16 copies of weight matrices refreshed.
__global__ void k_adam(long n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, unsigned short* __restrict__ pb, unsigned short* __restrict__ pbt,
                       WShapes w, float lr, float b1, float b2, float eps, float c1, float c2) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float gg = g[t];
  const float mm = b1 * m[t] + (1.f - b1) * gg;
  const float vv = b2 * v[t] + (1.f - b2) * gg * gg;
  m[t] = mm;
  v[t] = vv;
  const float wt = p[t] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  p[t] = wt;
  if (pb) pb[t] = f2bf(wt);
  if (pbt)  // weight entries also into the transposed bf16 copies
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const long o = t - w.off[l];
      if (o >= 0 && o < (long)w.rows[l] * w.cols[l]) {
        const int r = (int)(o / w.cols[l]), c = (int)(o % w.cols[l]);
        pbt[w.off[l] + (long)c * w.rows[l] + r] = f2bf(wt);
      }
    }
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
  PbT = (unsigned short*)al(nparams_dev * 2);
  A0 = (unsigned short*)al((size_t)bpad * kin * 2);
  A0T = (unsigned short*)al((size_t)bpad * kin * 2);
  for (int l = 0; l < 4; ++l) {
    Z[l] = (float*)al((size_t)bpad * rows[l] * 4);
    G[l] = (unsigned short*)al((size_t)bpad * rows[l] * 2);
    GT[l] = (unsigned short*)al((size_t)bpad * rows[l] * 2);
    if (l < 3) {
      Ab[l] = (unsigned short*)al((size_t)bpad * rows[l] * 2);
      AbT[l] = (unsigned short*)al((size_t)bpad * rows[l] * 2);
    }
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
  transpose_weights(0);
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

static void gemm(hipStream_t s, int M, int N, int K, const unsigned short* A, long lda, const unsigned short* B,
                 long ldb, float* C, long ldc, const GemmEpilogue& ep = GemmEpilogue()) {
  KScope ks(s, KF_MLP, 2.0 * M * N * K);
  // one wavefront per 16 x 16 tile: these products (batch <= 256, widths <= 512)
  // are small, and the finest tiling spreads them over the most CUs (a
  // 64 x 64 LDS-tiled form measured 3x slower here)
  hipLaunchKernelGGL(k_gemm_bf16, dim3((M + 15) / 16, (N + 15) / 16), dim3(64), 0, s, M, N, K, A, lda, B, ldb, C, ldc,
                     ep);
}

void Mlp::transpose_weights(hipStream_t s) {
  long mx = 0;
  for (int l = 0; l < 4; ++l) mx = std::max(mx, (long)rows[l] * cols[l]);
  hipLaunchKernelGGL(k_transpose_w, dim3(nb(mx), 4), dim3(256), 0, s, shapes(), Pb, PbT);
}

WShapes Mlp::shapes() const {
  WShapes w;
  for (int l = 0; l < 4; ++l) {
    w.off[l] = woff[l];
    w.rows[l] = rows[l];
    w.cols[l] = cols[l];
  }
  return w;
}

void Mlp::forward_dev(hipStream_t s, const float* x, const int* idx, int B, bool train) {
  hipLaunchKernelGGL(k_pack_input, dim3(nb((long)B * kin)), dim3(256), 0, s, B, n_in, kin, x, idx, A0,
                     train ? A0T : nullptr, (long)bpad);
  const unsigned short* a = A0;
  int ka = kin;
  for (int l = 0; l < 4; ++l) {
    // Z[b][n] = sum_k a[b][k] W[n][k] + bias[n]; hidden layers: Ab = bf16(relu(Z))
    // (padded output columns: zero weights and bias, so Z = 0 there)
    GemmEpilogue ep;
    ep.bias = P + boff[l];
    ep.act = l < 3 ? Ab[l] : nullptr;
    ep.actT = l < 3 && train ? AbT[l] : nullptr;
    ep.ldt = bpad;
    ep.relu = 1;
    gemm(s, B, rows[l], ka, a, ka, Pb + woff[l], cols[l], Z[l], rows[l], ep);
    if (l < 3) {
      a = Ab[l];
      ka = rows[l];
    }
  }
}

void Mlp::forward(hipStream_t s, const float* x, int B, float* y) {
  forward_dev(s, x, nullptr, B, false);
  hipLaunchKernelGGL(k_unpack_output, dim3(nb((long)B * n_out)), dim3(256), 0, s, B, n_out, kout, Z[3], y);
}

void Mlp::loss_grad_dev(hipStream_t s, const float* x, const float* y, const int* idx, int B, double* loss_acc) {
  forward_dev(s, x, idx, B, true);
  const long nG = (long)B * kout;
  const unsigned nblk = nb(nG);
  hipLaunchKernelGGL(k_mse, dim3(nblk), dim3(256), 0, s, B, n_out, kout, Z[3], y, idx, G[3], GT[3], (long)bpad,
                     partial);
  hipLaunchKernelGGL(k_loss_accum, dim3(1), dim3(256), 0, s, partial, (int)nblk, 1.0 / ((double)B * n_out),
                     loss_acc);
  for (int l = 3; l >= 0; --l) {
    const unsigned short* aT = l > 0 ? AbT[l - 1] : A0T;
    const int ka = l > 0 ? rows[l - 1] : kin;
    // dW[n][k] = sum_b G[b][n] a[b][k] = sum_b GT[n][b] aT[k][b]; db[n] = sum_b GT[n][b]
    GemmEpilogue ew;
    ew.rowsum = Gr + boff[l];
    gemm(s, rows[l], ka, B, GT[l], bpad, aT, bpad, Gr + woff[l], cols[l], ew);
    if (l > 0) {
      // dA[b][k] = sum_n G[b][n] W[n][k] = sum_n G[b][n] WT[k][n], then G[l-1] =
      // bf16(dA * (A[l-1] > 0)) (and its transpose) in the epilogue
      GemmEpilogue ep;
      ep.mask = Ab[l - 1];
      ep.gout = G[l - 1];
      ep.goutT = GT[l - 1];
      ep.ldt = bpad;
      gemm(s, B, ka, rows[l], G[l], rows[l], PbT + woff[l], rows[l], dA, ka, ep);
    }
  }
}

double Mlp::loss_grad(hipStream_t s, const float* x, const float* y, int B) {
  hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, loss_acc, 2);
  loss_grad_dev(s, x, y, nullptr, B, loss_acc);
  double l = 0.0;
  HHG_CHECK_HIP(hipMemcpyAsync(&l, loss_acc, sizeof(double), hipMemcpyDeviceToHost, s));
  HHG_CHECK_HIP(hipStreamSynchronize(s));
  return l;
}

void Mlp::train_step_dev(hipStream_t s, const float* x, const float* y, const int* idx, int B, float lr,
                         double* loss_acc) {
  loss_grad_dev(s, x, y, idx, B, loss_acc);
  ++step;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(nb(nparams_dev)), dim3(256), 0, s, nparams_dev, P, Gr, Mo, Vo, Pb, PbT, shapes(),
                     lr, b1, b2, 1e-8f, c1, c2);
}

}  // namespace hhg
