// Host side of the surrogate C ABI (include/lbm.h, surr_*): workspace layout,
// parameter packing, training epochs, gradients and prediction.  All
// arithmetic runs in the kernels of surr_kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "lbm.h"
#include "lbm_dev.h"
#include "surr_dev.h"

using lbmdev::fail;
using namespace surrdev;

namespace {

constexpr int NL = 4;
// padded layer shapes [N x K] and the real ones
constexpr int LN[NL] = {NHID, NHID, NHID, NOUTP};
constexpr int LK[NL] = {KIN, NHID, NHID, NHID};
constexpr int RN[NL] = {NHID, NHID, NHID, NOUT};
constexpr int RK[NL] = {NIN, NHID, NHID, NHID};

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

struct SLayout {
  size_t p[NL], m1[NL], m2[NL], g[NL], wb[NL], wt[NL];
  size_t x0, x0t, hf[3], hb[3], ht[3], y, t, dy, dyt, dhb[3], dht[3];
  size_t X, Y, RW, perm, qx, qy, lo, hi, lw, rw, loss, total;
  int Bp, max_data;
};

SLayout slayout(int max_batch, int max_data) {
  SLayout S;
  S.Bp = (max_batch + 31) / 32 * 32;
  S.max_data = max_data;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = a256(off + bytes); return o; };
  for (int l = 0; l < NL; ++l) {
    const size_t cnt = (size_t)LN[l] * LK[l] + LN[l];
    S.p[l] = take(cnt * 4);
    S.m1[l] = take(cnt * 4);
    S.m2[l] = take(cnt * 4);
    S.g[l] = take(cnt * 4);
    S.wb[l] = take((size_t)LN[l] * LK[l] * 2);
    S.wt[l] = take((size_t)LN[l] * LK[l] * 2);
  }
  const size_t B = S.Bp;
  S.x0 = take(B * KIN * 2);
  S.x0t = take(B * KIN * 2);
  for (int i = 0; i < 3; ++i) {
    S.hf[i] = take(B * NHID * 4);
    S.hb[i] = take(B * NHID * 2);
    S.ht[i] = take(B * NHID * 2);
    S.dhb[i] = take(B * NHID * 2);
    S.dht[i] = take(B * NHID * 2);
  }
  S.y = take(B * NOUTP * 4);
  S.t = take(B * NOUTP * 4);
  S.dy = take(B * NOUTP * 2);
  S.dyt = take(B * NOUTP * 2);
  S.X = take((size_t)max_data * NIN * 4);
  S.Y = take((size_t)max_data * NOUT * 4);
  S.RW = take((size_t)max_data * 4);
  S.rw = take(B * 4);
  S.perm = take((size_t)max_data * 4);
  S.qx = take(B * NIN * 4);
  S.qy = take(B * NOUT * 4);
  S.lo = take(NIN * 4);
  S.hi = take(NIN * 4);
  S.lw = take(NOUT * 4);
  S.loss = take(8);
  S.total = off;
  return S;
}

// ---- scratch of the prediction that allocates nothing ---------------------
// surr_predict_noalloc keeps its activations in this file-scope device array
// instead of the handle's workspace; every GPU the library runs on holds its
// own copy until the process ends.  In host code `scratch` names a host-side
// stand-in, not a device address: host code uses the address that
// scratch_ptr() looked up for the device.
constexpr int SCRATCH_ROWS = 1024;  // most query rows per call
constexpr size_t SC_X0 = 0;                                             // BF16 [R x KIN]
constexpr size_t SC_X0T = SC_X0 + (size_t)SCRATCH_ROWS * KIN * 2;        // BF16 [KIN x R]
constexpr size_t SC_HA = SC_X0T + (size_t)KIN * SCRATCH_ROWS * 2;        // BF16 [R x NHID]
constexpr size_t SC_HB = SC_HA + (size_t)SCRATCH_ROWS * NHID * 2;        // BF16 [R x NHID]
constexpr size_t SC_HF = SC_HB + (size_t)SCRATCH_ROWS * NHID * 2;        // FP32 [R x NHID] (unread)
constexpr size_t SC_HT = SC_HF + (size_t)SCRATCH_ROWS * NHID * 4;        // BF16 [NHID x R] (unread)
constexpr size_t SC_Y = SC_HT + (size_t)NHID * SCRATCH_ROWS * 2;         // FP32 [R x NOUTP]
constexpr size_t SCRATCH_BYTES = SC_Y + (size_t)SCRATCH_ROWS * NOUTP * 4;  // 3.2 MB

static __device__ __align__(256) char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch[MAX_DEVICES] = {};

// Device address of `scratch` on device dev, which must be the current
// device; looked up once per device and kept.
lbm_status scratch_ptr(int dev, char** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(LBM_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(LBM_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch[dev] = (char*)p;
  }
  *out = g_scratch[dev];
  return LBM_OK;
}

}  // namespace

struct surr_net {
  SLayout S;
  char* ws;
  hipStream_t stream;
  int n_data;
  long long adam_t;
  template <typename T> T* at(size_t off) const { return (T*)(ws + off); }
};

namespace {

#define HC(expr)                                                                            \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(LBM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// forward pass for `rows` samples gathered from (X, Y) by idx (or in order)
lbm_status forward(surr_net* s, const float* X, const float* Y, const float* RW,
                   const int32_t* idx, int rows) {
  const SLayout& S = s->S;
  const int B = S.Bp;
  HC(gather(X, Y, RW, idx, rows, B, s->at<float>(S.lo), s->at<float>(S.hi), s->at<__bf16>(S.x0),
            s->at<__bf16>(S.x0t), Y ? s->at<float>(S.t) : nullptr, s->at<float>(S.rw), s->stream));
  const __bf16* in = s->at<__bf16>(S.x0);
  int ldin = KIN;
  for (int l = 0; l < 3; ++l) {
    GemmArgs g{};
    g.A = in; g.lda = ldin; g.Bt = s->at<__bf16>(S.wb[l]); g.ldb = LK[l];
    g.M = B; g.N = LN[l]; g.K = LK[l];
    g.bias = s->at<float>(S.p[l]) + (size_t)LN[l] * LK[l];
    g.outf = s->at<float>(S.hf[l]); g.outb = s->at<__bf16>(S.hb[l]); g.outt = s->at<__bf16>(S.ht[l]);
    g.ldo = NHID; g.ldt = B;
    HC(gemm(EPI_HIDDEN, g, s->stream));
    in = s->at<__bf16>(S.hb[l]);
    ldin = NHID;
  }
  GemmArgs g{};
  g.A = in; g.lda = NHID; g.Bt = s->at<__bf16>(S.wb[3]); g.ldb = NHID;
  g.M = B; g.N = NOUTP; g.K = NHID;
  g.bias = s->at<float>(S.p[3]) + (size_t)NOUTP * NHID;
  g.outf = s->at<float>(S.y); g.ldo = NOUTP;
  HC(gemm(EPI_OUTPUT, g, s->stream));
  return LBM_OK;
}

// loss gradient and the parameter gradients of every layer (into S.g)
lbm_status backward(surr_net* s, int rows) {
  const SLayout& S = s->S;
  const int B = S.Bp;
  HC(loss(s->at<float>(S.y), s->at<float>(S.t), s->at<float>(S.lw), s->at<float>(S.rw), rows, B,
          s->at<__bf16>(S.dy), s->at<__bf16>(S.dyt), s->at<double>(S.loss), s->stream));
  // layer l has input activations in[l] (BF16 transposed) and output gradient dout
  const __bf16* dout_t = s->at<__bf16>(S.dyt);   // [N_l x B]
  const __bf16* dout_b = s->at<__bf16>(S.dy);    // [B x N_l]
  int ld_dout = NOUTP;
  for (int l = NL - 1; l >= 0; --l) {
    const __bf16* in_t = l == 0 ? s->at<__bf16>(S.x0t) : s->at<__bf16>(S.ht[l - 1]);
    float* gw = s->at<float>(S.g[l]);
    GemmArgs w{};
    w.A = dout_t; w.lda = B; w.Bt = in_t; w.ldb = B;
    w.M = LN[l]; w.N = LK[l]; w.K = B;
    w.outf = gw; w.ldo = LK[l];
    HC(gemm(EPI_WGRAD, w, s->stream));
    HC(colsum(dout_t, B, LN[l], gw + (size_t)LN[l] * LK[l], s->stream));
    if (l == 0) break;
    GemmArgs d{};
    d.A = dout_b; d.lda = ld_dout; d.Bt = s->at<__bf16>(S.wt[l]); d.ldb = LN[l];
    d.M = B; d.N = LK[l]; d.K = LN[l];
    d.act = s->at<float>(S.hf[l - 1]);
    d.outb = s->at<__bf16>(S.dhb[l - 1]); d.outt = s->at<__bf16>(S.dht[l - 1]);
    d.ldo = NHID; d.ldt = B;
    HC(gemm(EPI_BACKWARD, d, s->stream));
    dout_b = s->at<__bf16>(S.dhb[l - 1]);
    dout_t = s->at<__bf16>(S.dht[l - 1]);
    ld_dout = NHID;
  }
  return LBM_OK;
}

lbm_status adam_all(surr_net* s, float lr) {
  const SLayout& S = s->S;
  s->adam_t += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = (float)(1.0 - std::pow(0.9, (double)s->adam_t));
  const float c2 = (float)(1.0 - std::pow(0.999, (double)s->adam_t));
  for (int l = 0; l < NL; ++l) {
    const int cnt = LN[l] * LK[l] + LN[l];
    HC(adam(s->at<float>(S.p[l]), s->at<float>(S.m1[l]), s->at<float>(S.m2[l]),
            s->at<float>(S.g[l]), cnt, LN[l] * LK[l], LN[l], LK[l], lr, b1, b2, eps, c1, c2,
            s->at<__bf16>(S.wb[l]), s->at<__bf16>(S.wt[l]), s->stream));
  }
  return LBM_OK;
}

// packed (real) <-> padded layout
void pack_offsets(int l, size_t* w_off, size_t* b_off) {
  size_t o = 0;
  for (int k = 0; k < l; ++k) o += (size_t)RN[k] * RK[k] + RN[k];
  *w_off = o;
  *b_off = o + (size_t)RN[l] * RK[l];
}

}  // namespace

extern "C" {

lbm_status surr_workspace_bytes(int32_t max_batch, int32_t max_data, size_t* bytes) {
  if (!bytes || max_batch < 1 || max_batch > 65536 || max_data < 0 || max_data > (1 << 24))
    return fail(LBM_EINVAL, "bad surrogate sizes");
  *bytes = slayout(max_batch, max_data).total;
  return LBM_OK;
}

lbm_status surr_init(const double* lo, const double* hi, int32_t max_batch, int32_t max_data,
                     void* stream, void* workspace, size_t ws_bytes, surr_net** out) {
  if (!out || !lo || !hi) return fail(LBM_EINVAL, "NULL argument");
  *out = nullptr;
  size_t need = 0;
  lbm_status st = surr_workspace_bytes(max_batch, max_data, &need);
  if (st != LBM_OK) return st;
  if (!workspace || ((uintptr_t)workspace & 255u)) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < need) return fail(LBM_EINVAL, "workspace too small: %zu < %zu", ws_bytes, need);
  for (int j = 0; j < NIN; ++j)
    if (!(hi[j] > lo[j]) || !std::isfinite(lo[j]) || !std::isfinite(hi[j]) || (j == 2 && !(lo[j] > 0)))
      return fail(LBM_EINVAL, "bad normalisation box for input %d", j);
  surr_net* s = new (std::nothrow) surr_net();
  if (!s) return fail(LBM_ENOMEM, "surrogate handle");
  s->S = slayout(max_batch, max_data);
  s->ws = (char*)workspace;
  s->stream = (hipStream_t)stream;
  s->n_data = 0;
  s->adam_t = 0;
  float lof[NIN], hif[NIN], lw[NOUT];
  for (int j = 0; j < NIN; ++j) { lof[j] = (float)lo[j]; hif[j] = (float)hi[j]; }
  for (int j = 0; j < NOUT; ++j) lw[j] = 1.0f;
  hipError_t e = hipMemsetAsync(s->ws, 0, s->S.total, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(s->ws + s->S.lo, lof, sizeof lof, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(s->ws + s->S.hi, hif, sizeof hif, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(s->ws + s->S.lw, lw, sizeof lw, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) { delete s; return fail(LBM_EDEVICE, "surrogate init: %s", hipGetErrorString(e)); }
  // the scratch of surr_predict_noalloc on this (the current) device
  int dev = 0;
  char* sc = nullptr;
  if (hipGetDevice(&dev) != hipSuccess) { delete s; return fail(LBM_EDEVICE, "no current device"); }
  if ((st = scratch_ptr(dev, &sc)) != LBM_OK) { delete s; return st; }
  *out = s;
  return LBM_OK;
}

lbm_status surr_set_params(surr_net* s, const float* packed) {
  if (!s || !packed) return fail(LBM_EINVAL, "NULL argument");
  for (int l = 0; l < NL; ++l) {
    std::vector<float> pad((size_t)LN[l] * LK[l] + LN[l], 0.0f);
    size_t wo, bo;
    pack_offsets(l, &wo, &bo);
    for (int r = 0; r < RN[l]; ++r) {
      for (int c = 0; c < RK[l]; ++c) pad[(size_t)r * LK[l] + c] = packed[wo + (size_t)r * RK[l] + c];
      pad[(size_t)LN[l] * LK[l] + r] = packed[bo + r];
    }
    HC(hipMemcpyAsync(s->ws + s->S.p[l], pad.data(), pad.size() * 4, hipMemcpyHostToDevice, s->stream));
    HC(hipMemsetAsync(s->ws + s->S.m1[l], 0, pad.size() * 4, s->stream));
    HC(hipMemsetAsync(s->ws + s->S.m2[l], 0, pad.size() * 4, s->stream));
    HC(weight_copies(s->at<float>(s->S.p[l]), LN[l], LK[l], s->at<__bf16>(s->S.wb[l]),
                     s->at<__bf16>(s->S.wt[l]), s->stream));
  }
  HC(hipStreamSynchronize(s->stream));
  s->adam_t = 0;
  return LBM_OK;
}

lbm_status surr_get_params(surr_net* s, float* packed) {
  if (!s || !packed) return fail(LBM_EINVAL, "NULL argument");
  for (int l = 0; l < NL; ++l) {
    std::vector<float> pad((size_t)LN[l] * LK[l] + LN[l]);
    HC(hipMemcpyAsync(pad.data(), s->ws + s->S.p[l], pad.size() * 4, hipMemcpyDeviceToHost, s->stream));
    HC(hipStreamSynchronize(s->stream));
    size_t wo, bo;
    pack_offsets(l, &wo, &bo);
    for (int r = 0; r < RN[l]; ++r) {
      for (int c = 0; c < RK[l]; ++c) packed[wo + (size_t)r * RK[l] + c] = pad[(size_t)r * LK[l] + c];
      packed[bo + r] = pad[(size_t)LN[l] * LK[l] + r];
    }
  }
  return LBM_OK;
}

lbm_status surr_set_loss_weights(surr_net* s, const float* w) {
  if (!s || !w) return fail(LBM_EINVAL, "NULL argument");
  for (int j = 0; j < NOUT; ++j)
    if (!(w[j] >= 0.0f) || !std::isfinite(w[j])) return fail(LBM_EINVAL, "bad loss weight %d", j);
  HC(hipMemcpyAsync(s->ws + s->S.lw, w, NOUT * 4, hipMemcpyHostToDevice, s->stream));
  HC(hipStreamSynchronize(s->stream));
  return LBM_OK;
}

lbm_status surr_set_data(surr_net* s, const float* x, const float* y, const float* row_w, int32_t n) {
  if (!s || !x || !y || n < 1 || n > s->S.max_data) return fail(LBM_EINVAL, "bad training data");
  std::vector<float> w(n, 1.0f);
  if (row_w)
    for (int i = 0; i < n; ++i) {
      if (!(row_w[i] >= 0.0f) || !std::isfinite(row_w[i])) return fail(LBM_EINVAL, "bad row weight %d", i);
      w[i] = row_w[i];
    }
  HC(hipMemcpyAsync(s->ws + s->S.X, x, (size_t)n * NIN * 4, hipMemcpyHostToDevice, s->stream));
  HC(hipMemcpyAsync(s->ws + s->S.Y, y, (size_t)n * NOUT * 4, hipMemcpyHostToDevice, s->stream));
  HC(hipMemcpyAsync(s->ws + s->S.RW, w.data(), (size_t)n * 4, hipMemcpyHostToDevice, s->stream));
  HC(hipStreamSynchronize(s->stream));
  s->n_data = n;
  return LBM_OK;
}

lbm_status surr_train_epoch(surr_net* s, const int32_t* perm, int32_t batch, float lr,
                            double* mean_loss) {
  if (!s || !perm) return fail(LBM_EINVAL, "NULL argument");
  if (s->n_data < 1) return fail(LBM_EINVAL, "no training data");
  if (batch < 1 || batch > s->S.Bp) return fail(LBM_EINVAL, "batch must be in [1, %d]", s->S.Bp);
  if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(LBM_EINVAL, "bad learning rate");
  for (int i = 0; i < s->n_data; ++i)
    if (perm[i] < 0 || perm[i] >= s->n_data) return fail(LBM_EINVAL, "perm[%d] out of range", i);
  HC(hipMemcpyAsync(s->ws + s->S.perm, perm, (size_t)s->n_data * 4, hipMemcpyHostToDevice, s->stream));
  HC(hipMemsetAsync(s->ws + s->S.loss, 0, 8, s->stream));
  const float* X = s->at<float>(s->S.X);
  const float* Y = s->at<float>(s->S.Y);
  int nb = 0;
  for (int off = 0; off < s->n_data; off += batch, ++nb) {
    const int rows = std::min(batch, s->n_data - off);
    lbm_status st;
    if ((st = forward(s, X, Y, s->at<float>(s->S.RW), s->at<int32_t>(s->S.perm) + off, rows)) != LBM_OK)
      return st;
    if ((st = backward(s, rows)) != LBM_OK) return st;
    if ((st = adam_all(s, lr)) != LBM_OK) return st;
  }
  double acc = 0.0;
  HC(hipMemcpyAsync(&acc, s->ws + s->S.loss, 8, hipMemcpyDeviceToHost, s->stream));
  HC(hipStreamSynchronize(s->stream));
  if (mean_loss) *mean_loss = acc / nb;
  return LBM_OK;
}

lbm_status surr_gradients(surr_net* s, const float* x, const float* y, int32_t n, float* grad,
                          double* loss_out) {
  if (!s || !x || !y || !grad || n < 1 || n > s->S.Bp) return fail(LBM_EINVAL, "bad arguments");
  HC(hipMemcpyAsync(s->ws + s->S.qx, x, (size_t)n * NIN * 4, hipMemcpyHostToDevice, s->stream));
  HC(hipMemcpyAsync(s->ws + s->S.qy, y, (size_t)n * NOUT * 4, hipMemcpyHostToDevice, s->stream));
  HC(hipMemsetAsync(s->ws + s->S.loss, 0, 8, s->stream));
  lbm_status st;
  if ((st = forward(s, s->at<float>(s->S.qx), s->at<float>(s->S.qy), nullptr, nullptr, n)) != LBM_OK)
    return st;
  if ((st = backward(s, n)) != LBM_OK) return st;
  for (int l = 0; l < NL; ++l) {
    std::vector<float> pad((size_t)LN[l] * LK[l] + LN[l]);
    HC(hipMemcpyAsync(pad.data(), s->ws + s->S.g[l], pad.size() * 4, hipMemcpyDeviceToHost, s->stream));
    HC(hipStreamSynchronize(s->stream));
    size_t wo, bo;
    pack_offsets(l, &wo, &bo);
    for (int r = 0; r < RN[l]; ++r) {
      for (int c = 0; c < RK[l]; ++c) grad[wo + (size_t)r * RK[l] + c] = pad[(size_t)r * LK[l] + c];
      grad[bo + r] = pad[(size_t)LN[l] * LK[l] + r];
    }
  }
  double acc = 0.0;
  HC(hipMemcpyAsync(&acc, s->ws + s->S.loss, 8, hipMemcpyDeviceToHost, s->stream));
  HC(hipStreamSynchronize(s->stream));
  if (loss_out) *loss_out = acc;
  return LBM_OK;
}

lbm_status surr_predict(surr_net* s, const float* x, int32_t n, float* y) {
  if (!s || !x || !y || n < 0) return fail(LBM_EINVAL, "bad arguments");
  for (int off = 0; off < n; off += s->S.Bp) {
    const int rows = std::min(s->S.Bp, n - off);
    HC(hipMemcpyAsync(s->ws + s->S.qx, x + (size_t)off * NIN, (size_t)rows * NIN * 4,
                      hipMemcpyHostToDevice, s->stream));
    lbm_status st = forward(s, s->at<float>(s->S.qx), nullptr, nullptr, nullptr, rows);
    if (st != LBM_OK) return st;
    HC(hipMemcpy2DAsync(y + (size_t)off * NOUT, NOUT * 4, s->ws + s->S.y, NOUTP * 4, NOUT * 4, rows,
                        hipMemcpyDeviceToHost, s->stream));
  }
  HC(hipStreamSynchronize(s->stream));
  return LBM_OK;
}

lbm_status surr_predict_noalloc(const surr_net* s, const float* x, int32_t n, float* y,
                                void* stream) {
  if (!s || !x || !y) return fail(LBM_EINVAL, "NULL argument");
  if (n < 1 || n > SCRATCH_ROWS)
    return fail(LBM_EINVAL, "surr_predict_noalloc takes 1..%d rows per call, got %d", SCRATCH_ROWS, n);
  const hipStream_t st = (hipStream_t)stream;
  int cur = 0, dev = 0;
  HC(hipGetDevice(&cur));
  dev = cur;
  if (st) HC(hipStreamGetDevice(st, &dev));
  if (dev != cur) return fail(LBM_EINVAL, "the stream's device %d is not the current device %d", dev, cur);
  char* sc = nullptr;
  lbm_status r = scratch_ptr(dev, &sc);
  if (r != LBM_OK) return r;
  const SLayout& S = s->S;
  const int B = (n + 31) / 32 * 32;
  HC(gather(x, nullptr, nullptr, nullptr, n, B, s->at<float>(S.lo), s->at<float>(S.hi),
            (__bf16*)(sc + SC_X0), (__bf16*)(sc + SC_X0T), nullptr, nullptr, st));
  const __bf16* in = (const __bf16*)(sc + SC_X0);
  int ldin = KIN;
  for (int l = 0; l < 3; ++l) {
    __bf16* out = (__bf16*)(sc + (l % 2 == 0 ? SC_HA : SC_HB));
    GemmArgs g{};
    g.A = in; g.lda = ldin; g.Bt = s->at<__bf16>(S.wb[l]); g.ldb = LK[l];
    g.M = B; g.N = LN[l]; g.K = LK[l];
    g.bias = s->at<float>(S.p[l]) + (size_t)LN[l] * LK[l];
    g.outf = (float*)(sc + SC_HF); g.outb = out; g.outt = (__bf16*)(sc + SC_HT);
    g.ldo = NHID; g.ldt = B;
    HC(gemm(EPI_HIDDEN, g, st));
    in = out;
    ldin = NHID;
  }
  GemmArgs g{};
  g.A = in; g.lda = NHID; g.Bt = s->at<__bf16>(S.wb[3]); g.ldb = NHID;
  g.M = B; g.N = NOUTP; g.K = NHID;
  g.bias = s->at<float>(S.p[3]) + (size_t)NOUTP * NHID;
  g.outf = (float*)(sc + SC_Y); g.ldo = NOUTP;
  HC(gemm(EPI_OUTPUT, g, st));
  HC(hipMemcpy2DAsync(y, NOUT * 4, sc + SC_Y, NOUTP * 4, NOUT * 4, n, hipMemcpyDeviceToDevice, st));
  return LBM_OK;
}

void surr_destroy(surr_net* s) { delete s; }

}  // extern "C"
