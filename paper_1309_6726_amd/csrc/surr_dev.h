// Private declarations of the surrogate kernels (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace surrdev {

constexpr int NIN = 5;      // width, length, reaction rate, contact angle, threshold
constexpr int KIN = 32;     // padded input width
constexpr int NHID = 256;   // hidden units
constexpr int NOUT = 65;    // 64 front positions + closure time
constexpr int NOUTP = 96;   // padded output width

enum { EPI_HIDDEN = 0, EPI_OUTPUT = 1, EPI_BACKWARD = 2, EPI_WGRAD = 3 };

struct GemmArgs {
  const __bf16* A;   // [M x K], leading dimension lda
  const __bf16* Bt;  // [N x K], leading dimension ldb
  int M, N, K, lda, ldb;
  const float* bias; // [N] (hidden, output)
  const float* act;  // [M x ldo] activations of this layer (backward mask)
  float* outf;       // FP32 output [M x ldo]
  __bf16* outb;      // BF16 output [M x ldo]
  __bf16* outt;      // BF16 transposed output [N x ldt]
  int ldo, ldt;
};

hipError_t gemm(int epi, const GemmArgs& g, hipStream_t st);
hipError_t gather(const float* X, const float* Y, const float* RW, const int32_t* idx, int rows,
                  int Bp, const float* lo, const float* hi, __bf16* x0, __bf16* x0t, float* t,
                  float* rw, hipStream_t st);
hipError_t loss(const float* y, const float* t, const float* w, const float* rw, int rows, int Bp,
                __bf16* dy, __bf16* dyt, double* acc, hipStream_t st);
hipError_t colsum(const __bf16* dht, int Bp, int n_units, float* db, hipStream_t st);
hipError_t adam(float* p, float* m1, float* m2, const float* grad, int count, int nw, int N, int K,
                float lr, float b1, float b2, float eps, float c1, float c2, __bf16* wb,
                __bf16* wt, hipStream_t st);
hipError_t weight_copies(const float* w, int N, int K, __bf16* wb, __bf16* wt, hipStream_t st);

}  // namespace surrdev
