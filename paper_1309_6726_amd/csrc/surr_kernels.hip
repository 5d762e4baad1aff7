// Kernels of the MLP surrogate (5 -> 256 -> 256 -> 256 -> 65, ReLU) that maps
// capillary parameters (width, length, reaction rate, contact angle,
// precipitation threshold) to the front trajectory and the pore-closure time.
//
// Every dense-layer product, forward and backward, has the form
//   C[M x N] = A[M x K] * Bt[N x K]^T
// with both operands BF16 and contiguous along K, computed on the matrix
// cores with v_mfma_f32_32x32x16_bf16 (FP32 accumulation).  One wavefront
// owns one 32 x 32 tile of C; lane l loads the 8 consecutive K elements
// k0 + 8 (l / 32) .. +7 of row m0 + (l mod 32) of A and of row n0 + (l mod 32)
// of Bt with one 16-byte load each.  The 16 accumulators of lane l hold
// C[m0 + 8 (i / 4) + 4 (l / 32) + (i mod 4)][n0 + (l mod 32)], i = 0..15.
// Shapes are padded: M, N multiples of 32, K a multiple of 16, leading
// dimensions multiples of 8 elements.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "surr_dev.h"

namespace surrdev {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

template <int EPI>
__global__ void __launch_bounds__(256) k_gemm_nt(const GemmArgs g) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tile = blockIdx.x * 4 + wave;
  const int tn = g.N >> 5;
  if (tile >= (g.M >> 5) * tn) return;  // whole wavefront leaves; no barriers below
  const int m0 = (tile / tn) << 5, n0 = (tile % tn) << 5;
  const __bf16* a = g.A + (size_t)(m0 + (lane & 31)) * g.lda + 8 * (lane >> 5);
  const __bf16* b = g.Bt + (size_t)(n0 + (lane & 31)) * g.ldb + 8 * (lane >> 5);
  floatx16 acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
  for (int k = 0; k < g.K; k += 16) {
    const bf16x8 av = *(const bf16x8*)(a + k);
    const bf16x8 bv = *(const bf16x8*)(b + k);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
  }
  const int n = n0 + (lane & 31);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int m = m0 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
    const float v = acc[i];
    if (EPI == EPI_HIDDEN) {          // h = relu(v + b): FP32, BF16, BF16 transposed
      const float h = fmaxf(v + g.bias[n], 0.0f);
      g.outf[(size_t)m * g.ldo + n] = h;
      g.outb[(size_t)m * g.ldo + n] = (__bf16)h;
      g.outt[(size_t)n * g.ldt + m] = (__bf16)h;
    } else if (EPI == EPI_OUTPUT) {   // y = v + b
      g.outf[(size_t)m * g.ldo + n] = v + g.bias[n];
    } else if (EPI == EPI_BACKWARD) { // dh = v * relu'(h)
      const float d = g.act[(size_t)m * g.ldo + n] > 0.0f ? v : 0.0f;
      g.outb[(size_t)m * g.ldo + n] = (__bf16)d;
      g.outt[(size_t)n * g.ldt + m] = (__bf16)d;
    } else {                          // EPI_WGRAD: raw FP32 product
      g.outf[(size_t)m * g.ldo + n] = v;
    }
  }
}

// Rows idx[r] (or r when idx is null) of the raw inputs and targets of the
// resident data set: normalised inputs (BF16, row-major and transposed) and
// FP32 targets; padding rows and columns are zero.  Inputs x = (W, L, k_r,
// theta, threshold); x' = 2 (x - lo) / (hi - lo) - 1, with log10 applied to
// k_r and its bounds.  One thread per (row, column) of the KIN input columns
// followed by the NOUTP target columns, rows fastest (so the transposed input
// stores are coalesced); the row weight is written by column 0.
__global__ void k_gather(const float* __restrict__ X, const float* __restrict__ Y,
                         const float* __restrict__ RW, const int32_t* __restrict__ idx, int rows,
                         int Bp, const float* __restrict__ lo, const float* __restrict__ hi,
                         __bf16* __restrict__ x0, __bf16* __restrict__ x0t, float* __restrict__ t,
                         float* __restrict__ rw) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int ncol = KIN + (t ? NOUTP : 0);
  if (e >= Bp * ncol) return;
  const int r = e % Bp, j = e / Bp;
  const bool real = r < rows;
  const int src = real ? (idx ? idx[r] : r) : 0;
  if (j < KIN) {
    float v = 0.0f;
    if (real && j < NIN) {
      float x = X[(size_t)src * NIN + j], a = lo[j], b = hi[j];
      if (j == 2) { x = log10f(x); a = log10f(a); b = log10f(b); }
      v = 2.0f * (x - a) / (b - a) - 1.0f;
    }
    x0[(size_t)r * KIN + j] = (__bf16)v;
    x0t[(size_t)j * Bp + r] = (__bf16)v;
    if (j == 0 && rw) rw[r] = real ? (RW ? RW[src] : 1.0f) : 0.0f;
  } else {
    const int c = j - KIN;
    t[(size_t)r * NOUTP + c] = (real && Y && c < NOUT) ? Y[(size_t)src * NOUT + c] : 0.0f;
  }
}

// Weighted mean-squared error over the real rows and outputs:
// loss = sum_rows c_r sum_j w_j (y - t)^2 / (rows * sum_j w_j) with per-output
// weights w and per-row weights c, its gradient dY (BF16 row-major and
// transposed) and the loss added to *loss_acc.
__global__ void __launch_bounds__(256) k_loss(const float* __restrict__ y, const float* __restrict__ t,
                                              const float* __restrict__ w, const float* __restrict__ rw,
                                              int rows, int Bp,
                                              __bf16* __restrict__ dy, __bf16* __restrict__ dyt,
                                              double* __restrict__ loss_acc) {
  __shared__ double red[256];
  double s = 0.0;
  float wsum = 0.0f;
  for (int j = 0; j < NOUT; ++j) wsum += w[j];
  const float scale = 1.0f / ((float)rows * wsum);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < Bp * NOUTP; e += gridDim.x * blockDim.x) {
    const int r = e / NOUTP, j = e - r * NOUTP;
    float d = 0.0f;
    if (r < rows && j < NOUT) {
      const float diff = y[e] - t[e];
      const float c = w[j] * rw[r] * scale;
      d = 2.0f * c * diff;
      s += (double)(c * diff * diff);
    }
    dy[e] = (__bf16)d;
    dyt[(size_t)j * Bp + r] = (__bf16)d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss_acc, red[0]);
}

// Bias gradients: column sums of dH, read from its transposed copy (one
// wavefront per output unit, fixed summation order).
__global__ void __launch_bounds__(64) k_colsum(const __bf16* __restrict__ dht, int Bp, int n_units,
                                               float* __restrict__ db) {
  const int n = blockIdx.x;
  if (n >= n_units) return;
  float s = 0.0f;
  for (int m = threadIdx.x; m < Bp; m += 64) s += (float)dht[(size_t)n * Bp + m];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o);
  if (threadIdx.x == 0) db[n] = s;
}

// Adam on the padded FP32 master parameters, then the BF16 copies used by the
// GEMMs: W (row-major [N x K]) and W^T ([K x N]).  Entries of a weight matrix
// at index < nw; biases follow.
__global__ void k_adam(float* __restrict__ p, float* __restrict__ m1, float* __restrict__ m2,
                       const float* __restrict__ grad, int count, int nw, int N, int K,
                       float lr, float b1, float b2, float eps, float c1, float c2,
                       __bf16* __restrict__ wb, __bf16* __restrict__ wt) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    const float gi = grad[i];
    const float a = b1 * m1[i] + (1.0f - b1) * gi;
    const float v = b2 * m2[i] + (1.0f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    const float w = p[i] - lr * (a / c1) / (sqrtf(v / c2) + eps);
    p[i] = w;
    if (i < nw) {
      const int r = i / K, c = i - r * K;
      wb[i] = (__bf16)w;
      wt[(size_t)c * N + r] = (__bf16)w;
    }
  }
}

// BF16 copies of one padded weight matrix (after parameters are set).
__global__ void k_weight_copies(const float* __restrict__ w, int N, int K, __bf16* __restrict__ wb,
                                __bf16* __restrict__ wt) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N * K; i += gridDim.x * blockDim.x) {
    const int r = i / K, c = i - r * K;
    wb[i] = (__bf16)w[i];
    wt[(size_t)c * N + r] = (__bf16)w[i];
  }
}

// ---- launchers ------------------------------------------------------------
hipError_t gemm(int epi, const GemmArgs& g, hipStream_t st) {
  const int tiles = (g.M / 32) * (g.N / 32);
  const dim3 grid((tiles + 3) / 4), block(256);
  switch (epi) {
    case EPI_HIDDEN: hipLaunchKernelGGL(k_gemm_nt<EPI_HIDDEN>, grid, block, 0, st, g); break;
    case EPI_OUTPUT: hipLaunchKernelGGL(k_gemm_nt<EPI_OUTPUT>, grid, block, 0, st, g); break;
    case EPI_BACKWARD: hipLaunchKernelGGL(k_gemm_nt<EPI_BACKWARD>, grid, block, 0, st, g); break;
    default: hipLaunchKernelGGL(k_gemm_nt<EPI_WGRAD>, grid, block, 0, st, g); break;
  }
  return hipGetLastError();
}

hipError_t gather(const float* X, const float* Y, const float* RW, const int32_t* idx, int rows,
                  int Bp, const float* lo, const float* hi, __bf16* x0, __bf16* x0t, float* t,
                  float* rw, hipStream_t st) {
  const int n = Bp * (KIN + (t ? NOUTP : 0));
  hipLaunchKernelGGL(k_gather, dim3((n + 255) / 256), dim3(256), 0, st, X, Y, RW, idx, rows, Bp,
                     lo, hi, x0, x0t, t, rw);
  return hipGetLastError();
}

hipError_t loss(const float* y, const float* t, const float* w, const float* rw, int rows, int Bp,
                __bf16* dy, __bf16* dyt, double* acc, hipStream_t st) {
  const int blocks = (Bp * NOUTP + 255) / 256 < 256 ? (Bp * NOUTP + 255) / 256 : 256;
  hipLaunchKernelGGL(k_loss, dim3(blocks), dim3(256), 0, st, y, t, w, rw, rows, Bp, dy, dyt, acc);
  return hipGetLastError();
}

hipError_t colsum(const __bf16* dht, int Bp, int n_units, float* db, hipStream_t st) {
  hipLaunchKernelGGL(k_colsum, dim3(n_units), dim3(64), 0, st, dht, Bp, n_units, db);
  return hipGetLastError();
}

hipError_t adam(float* p, float* m1, float* m2, const float* grad, int count, int nw, int N, int K,
                float lr, float b1, float b2, float eps, float c1, float c2, __bf16* wb,
                __bf16* wt, hipStream_t st) {
  const int blocks = (count + 255) / 256 < 1024 ? (count + 255) / 256 : 1024;
  hipLaunchKernelGGL(k_adam, dim3(blocks), dim3(256), 0, st, p, m1, m2, grad, count, nw, N, K, lr,
                     b1, b2, eps, c1, c2, wb, wt);
  return hipGetLastError();
}

hipError_t weight_copies(const float* w, int N, int K, __bf16* wb, __bf16* wt, hipStream_t st) {
  const int blocks = (N * K + 255) / 256 < 1024 ? (N * K + 255) / 256 : 1024;
  hipLaunchKernelGGL(k_weight_copies, dim3(blocks), dim3(256), 0, st, w, N, K, wb, wt);
  return hipGetLastError();
}

}  // namespace surrdev
