// Host side of the C ABI declared in include/lbm.h: parameter checks,
// workspace layout, launch sequencing on the caller's stream, observe /
// checkpoint transfers and the launch-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_dev.h"

using namespace lbmdev;

namespace lbmdev {
thread_local std::string g_err;

lbm_status fail(lbm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}
}  // namespace lbmdev

namespace {

#define HIPCHECK(expr)                                                                  \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(LBM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr uint64_t kMagic = 0x4C424D5853494D31ull;  // "LBMXSIM1"
constexpr int kVersion = 2;  // 2: three rotating pending bits in the mask

struct Layout {
  long long N = 0, P = 0, ev_cap = 0;
  int nblocks = 0;
  bool solute = false, react = false;
  size_t f[2] = {0, 0}, g[2] = {0, 0}, mask = 0, m = 0, sstep = 0, drop = 0, ev = 0, evc = 0,
         partial = 0, out = 0, total = 0;
};

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

Layout make_layout(const lbm_params& p) {
  Layout L;
  L.N = (long long)p.nx * p.ny;
  L.P = (L.N + 63) / 64 * 64;
  L.solute = p.tau_g > 0.0;
  L.react = p.k_r > 0.0;
  L.ev_cap = L.react ? L.N : 0;
  L.nblocks = (int)std::min<long long>(1024, (L.N + 255) / 256);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = a256(off + bytes);
    return o;
  };
  L.f[0] = take(18 * L.P * sizeof(float));
  L.f[1] = take(18 * L.P * sizeof(float));
  if (L.solute) {
    L.g[0] = take(5 * L.P * sizeof(float));
    L.g[1] = take(5 * L.P * sizeof(float));
  }
  L.mask = take(L.P);
  if (L.react) {
    L.m = take(L.P * sizeof(double));
    L.sstep = take(L.P * sizeof(int32_t));
    L.drop = take(3 * L.P * sizeof(float));
    L.ev = take(L.ev_cap * sizeof(lbm_event));
  }
  L.evc = take(sizeof(unsigned long long));
  L.partial = take((size_t)L.nblocks * OBS_SLOTS * sizeof(double));
  L.out = take(OBS_OUT * sizeof(double));
  L.total = off;
  return L;
}

lbm_status check_params(const lbm_params* p) {
  if (!p) return fail(LBM_EINVAL, "params is NULL");
  if (p->nx < 3 || p->ny < 3) return fail(LBM_EINVAL, "nx, ny must be >= 3");
  // 32-bit element offsets in the kernels: 23 population planes below 2^31
  if (((long long)p->nx * p->ny + 63) / 64 * 64 * 23 > (1ll << 31) - 1)
    return fail(LBM_EINVAL, "lattice too large (at most ~93 million nodes)");
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return fail(LBM_EINVAL, "tau must be > 1/2");
  if (!(p->tau_g == 0.0 || (p->tau_g > 0.5 && std::isfinite(p->tau_g))))
    return fail(LBM_EINVAL, "tau_g must be 0 or > 1/2");
  if (!(p->k_r >= 0.0) || 4.0 * p->k_r > 1.0) return fail(LBM_EINVAL, "need 0 <= 4 k_r <= 1");
  if (p->k_r > 0.0 && p->tau_g == 0.0) return fail(LBM_EINVAL, "reaction needs the solute lattice");
  if (!(p->threshold > 0.0) || !std::isfinite(p->threshold)) return fail(LBM_EINVAL, "threshold must be > 0");
  if (!std::isfinite(p->G) || !std::isfinite(p->G_ads[0]) || !std::isfinite(p->G_ads[1]) ||
      !std::isfinite(p->accel[0]) || !std::isfinite(p->accel[1]))
    return fail(LBM_EINVAL, "non-finite force parameter");
  if (!(p->c_eq >= 0.0) || !std::isfinite(p->c_eq)) return fail(LBM_EINVAL, "c_eq must be finite and >= 0");
  if (!(p->c_hold >= 0.0) || !std::isfinite(p->c_hold))
    return fail(LBM_EINVAL, "c_hold must be finite and >= 0");
  if (p->hold_x < 0 || p->hold_x > p->nx) return fail(LBM_EINVAL, "hold_x must be in [0, nx]");
  if (p->hold_x > 0 && p->tau_g == 0.0) return fail(LBM_EINVAL, "a held source needs the solute lattice");
  if (p->solute_q != 0 && p->solute_q != 4 && p->solute_q != 5)
    return fail(LBM_EINVAL, "solute_q must be 0, 4 or 5");
  if (p->W < 0) return fail(LBM_EINVAL, "W must be >= 0");
  if (p->W > 0) {
    if (p->x_in < 0 || p->x_out > p->nx || p->x_in + 2 > p->x_out)
      return fail(LBM_EINVAL, "capillary section out of range");
    if (p->y0 < 0 || p->y0 + p->W > p->ny) return fail(LBM_EINVAL, "capillary rows out of range");
  }
  return LBM_OK;
}

}  // namespace

struct lbm_sim {
  lbm_params p;
  Layout L;
  hipStream_t stream;
  char* ws;
  int cur;         // buffer holding the current state
  long long step;  // current state index
  int tx, sy;
  int nt;          // 1: the step's loads carry the non-temporal cache hint
  int scheme;      // LBM_SCHEME_*
  bool mom;        // f[cur] holds moments of the last step, not populations
  bool poisoned;
  float* f(int i) const { return (float*)(ws + L.f[i]); }
  float* g(int i) const { return L.solute ? (float*)(ws + L.g[i]) : nullptr; }
  uint8_t* mask() const { return (uint8_t*)(ws + L.mask); }
  double* m() const { return L.react ? (double*)(ws + L.m) : nullptr; }
  int32_t* sstep() const { return L.react ? (int32_t*)(ws + L.sstep) : nullptr; }
  float* drop() const { return L.react ? (float*)(ws + L.drop) : nullptr; }
  lbm_event* ev() const { return L.react ? (lbm_event*)(ws + L.ev) : nullptr; }
  unsigned long long* evc() const { return (unsigned long long*)(ws + L.evc); }
  double* partial() const { return (double*)(ws + L.partial); }
  double* out() const { return (double*)(ws + L.out); }
};

namespace {

lbm_status guard(const lbm_sim* s) {
  if (!s) return fail(LBM_EINVAL, "handle is NULL");
  if (s->poisoned) return fail(LBM_ESTATE, "handle poisoned by an earlier failure; lbm_load a checkpoint");
  return LBM_OK;
}

bool tile_ok(int tx, int sy) { return (tx == 64 || tx == 128 || tx == 256) && sy >= 1 && sy <= 4096; }

void default_tile(const lbm_params& p, int* tx, int* sy) {
  *tx = p.nx >= 1024 ? 256 : (p.nx >= 256 ? 128 : 64);
  *sy = 16;
}

bool use_moments(int scheme, const lbm_params& p) {
  return scheme == LBM_SCHEME_MOMENTS || (scheme == LBM_SCHEME_AUTO && p.tau == 1.0);
}

// Populations of the current state written over the stored moments (the
// idle buffer is the scratch), so the state is held as populations again.
lbm_status materialize(lbm_sim* s) {
  if (!s->mom) return LBM_OK;
  const lbm_params& p = s->p;
  hipError_t e = launch_unpack(s->f(s->cur), s->mask(), p.nx, p.ny, s->L.P,
                               1u | pending_bit(s->step - 2), s->f(s->cur ^ 1), s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->f(s->cur), s->f(s->cur ^ 1), 18 * s->L.P * sizeof(float),
                       hipMemcpyDeviceToDevice, s->stream);
  if (e != hipSuccess) {
    s->poisoned = true;
    return fail(LBM_EDEVICE, "unpack moments: %s", hipGetErrorString(e));
  }
  s->mom = false;
  return LBM_OK;
}

lbm_status queue_steps(lbm_sim* s, long long n) {
  const lbm_params& p = s->p;
  const bool moments = use_moments(s->scheme, p);
  if (n > 0 && !moments && s->mom) {
    lbm_status st = materialize(s);
    if (st != LBM_OK) return st;
  }
  StepArgs a{};
  a.mask = s->mask();
  a.m = s->m();
  a.sstep = s->sstep();
  a.drop = s->drop();
  a.ev = s->ev();
  a.ev_count = s->evc();
  a.ev_cap = s->L.ev_cap;
  a.P = s->L.P;
  a.nx = p.nx;
  a.ny = p.ny;
  a.sy = s->sy;
  a.nsegs = (p.ny + s->sy - 1) / s->sy;
  a.solute = s->L.solute;
  a.react = s->L.react;
  a.omega = 1.0 / p.tau;
  a.tau = p.tau;
  a.G = p.G;
  a.Gads1 = p.G_ads[0];
  a.Gads2 = p.G_ads[1];
  a.ax = p.accel[0];
  a.ay = p.accel[1];
  a.omega_g = s->L.solute ? 1.0 / p.tau_g : 0.0;
  a.k_r = p.k_r;
  a.threshold = p.threshold;
  a.c_eq = p.c_eq;
  a.c_hold = p.c_hold;
  a.hold_x = p.hold_x;
  a.q4 = p.solute_q == 4;
  for (long long t = 0; t < n; ++t) {
    const int kind = !moments ? KIND_POP : (s->mom ? KIND_MM : KIND_PM);
    a.tx_owned = kind == KIND_MM ? 60 : s->tx - 2;  // the moment step: 64-lane tiles
    a.nstrips = (p.nx + a.tx_owned - 1) / a.tx_owned;
    a.remap = (a.nstrips * a.nsegs) >= 8;
    a.fin = s->f(s->cur);
    a.fout = s->f(s->cur ^ 1);
    a.gin = s->g(s->cur);
    a.gout = s->g(s->cur ^ 1);
    a.step = s->step;
    a.bit_p1 = pending_bit(s->step - 1);
    a.bit_p2 = pending_bit(s->step - 2);
    a.bit_cur = pending_bit(s->step);
    hipError_t e = launch_step(a, s->tx, kind, s->nt, s->stream);
    if (e != hipSuccess) {
      s->poisoned = true;
      return fail(LBM_EDEVICE, "step launch: %s", hipGetErrorString(e));
    }
    s->cur ^= 1;
    s->step += 1;
    s->mom = kind != KIND_POP;
  }
  return LBM_OK;
}

size_t blob_size(const lbm_sim* s, long long nev) {
  const long long N = s->L.N;
  size_t n = 8 + 4 * 4 + 8 + 8;  // header
  n += 18 * N * sizeof(float);
  if (s->L.solute) n += 5 * N * sizeof(float);
  n += N;
  if (s->L.react) n += N * (sizeof(double) + sizeof(int32_t) + 3 * sizeof(float)) + nev * sizeof(lbm_event);
  return n;
}

// Capillary observables from the observer's output: front, growth, closure
// and the radii of Fig. 4 (r_min, r_ave = A / L, r_h = A / P with P the
// lower wall's profile length: one unit per column plus its vertical steps).
void capillary_radii(const lbm_params& p, const double* h, lbm_obs* o) {
  if (p.W > 0) {
    const double L = (double)(p.x_out - p.x_in);
    o->front_z = h[OBS_SLOTS];
    o->delta_e = h[OBS_SLOTS + 1];
    o->closure_step = (int64_t)h[OBS_SLOTS + 2];
    o->r_min = h[OBS_SLOTS + 4];
    o->r_ave = h[OBS_SLOTS + 3] / L;
    o->r_h = h[OBS_SLOTS + 3] / (L + h[OBS_SLOTS + 5]);
  } else {
    o->front_z = NAN;
    o->delta_e = 0.0;
    o->closure_step = -1;
    o->r_min = o->r_ave = o->r_h = NAN;
  }
}

lbm_status copy_planes_d2h(char* dst, const char* src_dev, int planes, long long N, long long P,
                           size_t esz, hipStream_t st) {
  for (int q = 0; q < planes; ++q)
    HIPCHECK(hipMemcpyAsync(dst + q * N * esz, src_dev + q * P * esz, N * esz, hipMemcpyDeviceToHost, st));
  return LBM_OK;
}

lbm_status copy_planes_h2d(char* dst_dev, const char* src, int planes, long long N, long long P,
                           size_t esz, hipStream_t st) {
  for (int q = 0; q < planes; ++q)
    HIPCHECK(hipMemcpyAsync(dst_dev + q * P * esz, src + q * N * esz, N * esz, hipMemcpyHostToDevice, st));
  return LBM_OK;
}

}  // namespace

extern "C" {

const char* lbm_last_error(void) { return g_err.c_str(); }

const char* lbm_strerror(lbm_status s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "out of host memory";
    case LBM_EDEVICE: return "device error";
    case LBM_ENONFINITE: return "non-finite density or concentration";
    case LBM_ESTATE: return "handle poisoned by an earlier failure";
  }
  return "unknown status";
}

lbm_status lbm_workspace_bytes(const lbm_params* p, size_t* bytes) {
  lbm_status st = check_params(p);
  if (st != LBM_OK) return st;
  if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
  *bytes = make_layout(*p).total;
  return LBM_OK;
}

lbm_status lbm_init(const lbm_params* p, const uint8_t* solid, const double* rho1,
                    const double* rho2, const double* conc, void* stream, void* workspace,
                    size_t ws_bytes, lbm_sim** out) {
  lbm_status st = check_params(p);
  if (st != LBM_OK) return st;
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!solid || !rho1 || !rho2) return fail(LBM_EINVAL, "solid, rho1, rho2 are required");
  const bool solute = p->tau_g > 0.0;
  if (solute && !conc) return fail(LBM_EINVAL, "conc is required when tau_g > 0");
  Layout L = make_layout(*p);
  if (!workspace) return fail(LBM_EINVAL, "workspace is NULL");
  if (((uintptr_t)workspace & 255u) != 0) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total) return fail(LBM_EINVAL, "workspace too small: %zu < %zu", ws_bytes, L.total);
  const long long N = L.N;
  for (long long i = 0; i < N; ++i) {
    if (solid[i] > 1) return fail(LBM_EINVAL, "mask value %d at node %lld", (int)solid[i], i);
    if (solid[i]) continue;
    if (!(rho1[i] >= 0.0) || !(rho2[i] >= 0.0) || !std::isfinite(rho1[i]) || !std::isfinite(rho2[i]))
      return fail(LBM_EINVAL, "density at node %lld must be finite and >= 0", i);
    if (rho1[i] + rho2[i] <= 0.0) return fail(LBM_EINVAL, "fluid node %lld has zero density", i);
    if (solute && (!(conc[i] >= 0.0) || !std::isfinite(conc[i])))
      return fail(LBM_EINVAL, "concentration at node %lld must be finite and >= 0", i);
  }
  lbm_sim* s = (lbm_sim*)calloc(1, sizeof(lbm_sim));
  if (!s) return fail(LBM_ENOMEM, "handle allocation");
  s->p = *p;
  s->L = L;
  s->stream = (hipStream_t)stream;
  s->ws = (char*)workspace;
  s->cur = 0;
  s->step = 0;
  default_tile(*p, &s->tx, &s->sy);
  s->nt = 0;
  s->scheme = LBM_SCHEME_AUTO;
  s->mom = false;
  // stage the FP64 inputs in the second population buffer (72 B per node)
  char* stage = (char*)s->f(1);
  hipStream_t hs = s->stream;
  auto bail = [&](lbm_status e) { free(s); return e; };
#define CK(expr) do { hipError_t e_ = (expr); if (e_ != hipSuccess) { fail(LBM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); return bail(LBM_EDEVICE); } } while (0)
  CK(hipMemcpyAsync(stage, rho1, N * sizeof(double), hipMemcpyHostToDevice, hs));
  CK(hipMemcpyAsync(stage + N * sizeof(double), rho2, N * sizeof(double), hipMemcpyHostToDevice, hs));
  if (solute) CK(hipMemcpyAsync(stage + 2 * N * sizeof(double), conc, N * sizeof(double), hipMemcpyHostToDevice, hs));
  CK(hipMemcpyAsync(s->mask(), solid, N, hipMemcpyHostToDevice, hs));
  CK(hipMemsetAsync(s->evc(), 0, sizeof(unsigned long long), hs));
  CK(launch_init((const double*)stage, (const double*)(stage + N * sizeof(double)),
                 solute ? (const double*)(stage + 2 * N * sizeof(double)) : nullptr, s->mask(),
                 s->f(0), s->g(0), s->m(), s->sstep(), s->drop(), N, L.P, solute, L.react,
                 p->solute_q == 4, hs));
  CK(hipStreamSynchronize(hs));
#undef CK
  *out = s;
  return LBM_OK;
}

lbm_status lbm_step(lbm_sim* s, int64_t nsteps) {
  lbm_status st = guard(s);
  if (st != LBM_OK) return st;
  if (nsteps < 0) return fail(LBM_EINVAL, "nsteps < 0");
  return queue_steps(s, nsteps);
}

lbm_status lbm_observe(lbm_sim* s, lbm_obs* o) {
  lbm_status st = guard(s);
  if (st != LBM_OK) return st;
  if (!o) return fail(LBM_EINVAL, "out is NULL");
  const lbm_params& p = s->p;
  hipError_t e = launch_observe(s->f(s->cur), s->g(s->cur), s->mask(), s->m(), s->drop(),
                                s->sstep(), p.nx, p.ny, s->L.P, pending_bit(s->step - 1),
                                pending_bit(s->step - 2), s->mom, s->L.solute, s->L.react,
                                s->L.nblocks, s->partial(), s->out(), p.x_in, p.x_out, p.y0, p.W,
                                s->stream);
  if (e != hipSuccess) { s->poisoned = true; return fail(LBM_EDEVICE, "observe launch: %s", hipGetErrorString(e)); }
  double h[OBS_OUT];
  unsigned long long nev = 0;
  e = hipMemcpyAsync(h, s->out(), sizeof h, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&nev, s->evc(), sizeof nev, hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) { s->poisoned = true; return fail(LBM_EDEVICE, "observe: %s", hipGetErrorString(e)); }
  memset(o, 0, sizeof *o);
  o->step = s->step;
  o->mass[0] = h[0];
  o->mass[1] = h[1];
  o->solute = h[2];
  o->precipitate = h[3];
  o->mass_removed[0] = h[4];
  o->mass_removed[1] = h[5];
  o->solute_removed = h[6];
  o->n_solid = (int64_t)h[7];
  o->nonfinite = h[8] > 0.0;
  o->n_events = (int64_t)nev;
  capillary_radii(p, h, o);
  if ((long long)nev > s->L.ev_cap)
    return fail(LBM_EDEVICE, "event log overflow (%llu > %lld)", nev, s->L.ev_cap);
  if (o->nonfinite) {
    s->poisoned = true;
    return fail(LBM_ENONFINITE, "%lld fluid nodes hold a NaN/Inf at step %lld", (long long)h[8], s->step);
  }
  return LBM_OK;
}

lbm_status lbm_fields(lbm_sim* s, uint32_t mask, double* host) {
  lbm_status st = guard(s);
  if (st != LBM_OK) return st;
  if (!host && mask) return fail(LBM_EINVAL, "host_fields is NULL");
  if (mask >> 7) return fail(LBM_EINVAL, "unknown field bits");
  const lbm_params& p = s->p;
  const long long N = s->L.N;
  // staging: the idle population buffer (72 B per node >= 7 doubles per node);
  // the next step overwrites every fluid slot of it before reading it
  double* stage = (double*)s->f(s->cur ^ 1);
  hipError_t e = launch_fields(s->f(s->cur), s->g(s->cur), s->mask(), s->m(), p.nx, p.ny, s->L.P,
                               pending_bit(s->step - 1), pending_bit(s->step - 2), s->mom,
                               s->L.solute, s->L.react, p.G, p.G_ads[0], p.G_ads[1],
                               p.accel[0], p.accel[1], stage, s->stream);
  int k = 0;
  for (int b = 0; b < 7 && e == hipSuccess; ++b) {
    if (!(mask & (1u << b))) continue;
    e = hipMemcpyAsync(host + (size_t)k * N, stage + (size_t)b * N, N * sizeof(double),
                       hipMemcpyDeviceToHost, s->stream);
    ++k;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) { s->poisoned = true; return fail(LBM_EDEVICE, "fields: %s", hipGetErrorString(e)); }
  return LBM_OK;
}

lbm_status lbm_events(lbm_sim* s, int64_t first, lbm_event* buf, int64_t cap, int64_t* n) {
  lbm_status st = guard(s);
  if (st != LBM_OK) return st;
  if (!n || first < 0 || cap < 0 || (cap > 0 && !buf)) return fail(LBM_EINVAL, "bad events arguments");
  unsigned long long nev = 0;
  HIPCHECK(hipMemcpyAsync(&nev, s->evc(), sizeof nev, hipMemcpyDeviceToHost, s->stream));
  HIPCHECK(hipStreamSynchronize(s->stream));
  *n = (int64_t)nev;
  long long avail = std::min<long long>((long long)nev, s->L.ev_cap) - first;
  long long k = std::min<long long>(avail, cap);
  if (k > 0) {
    HIPCHECK(hipMemcpyAsync(buf, s->ev() + first, k * sizeof(lbm_event), hipMemcpyDeviceToHost, s->stream));
    HIPCHECK(hipStreamSynchronize(s->stream));
  }
  return LBM_OK;
}

lbm_status lbm_save(lbm_sim* s, void* blob, size_t cap, size_t* n) {
  if (!s) return fail(LBM_EINVAL, "handle is NULL");
  if (!n) return fail(LBM_EINVAL, "n is NULL");
  unsigned long long nev = 0;
  HIPCHECK(hipMemcpyAsync(&nev, s->evc(), sizeof nev, hipMemcpyDeviceToHost, s->stream));
  HIPCHECK(hipStreamSynchronize(s->stream));
  nev = std::min<unsigned long long>(nev, (unsigned long long)s->L.ev_cap);
  const size_t need = blob_size(s, (long long)nev);
  *n = need;
  if (!blob) return LBM_OK;
  if (cap < need) return fail(LBM_EINVAL, "blob too small: %zu < %zu", cap, need);
  // a checkpoint holds populations: moments are unpacked first, and the run
  // continues from those FP32 populations, so a resumed run is bit-identical
  lbm_status mst = materialize(s);
  if (mst != LBM_OK) return mst;
  char* b = (char*)blob;
  const long long N = s->L.N, P = s->L.P;
  const int32_t hdr32[4] = {s->p.nx, s->p.ny, (s->L.solute ? 1 : 0) | (s->L.react ? 2 : 0), kVersion};
  const int64_t step = s->step, nev64 = (int64_t)nev;
  memcpy(b, &kMagic, 8); b += 8;
  memcpy(b, hdr32, 16); b += 16;
  memcpy(b, &step, 8); b += 8;
  memcpy(b, &nev64, 8); b += 8;
  lbm_status st;
  if ((st = copy_planes_d2h(b, (const char*)s->f(s->cur), 18, N, P, 4, s->stream)) != LBM_OK) return st;
  b += 18 * N * 4;
  if (s->L.solute) {
    if ((st = copy_planes_d2h(b, (const char*)s->g(s->cur), 5, N, P, 4, s->stream)) != LBM_OK) return st;
    b += 5 * N * 4;
  }
  HIPCHECK(hipMemcpyAsync(b, s->mask(), N, hipMemcpyDeviceToHost, s->stream));
  b += N;
  if (s->L.react) {
    HIPCHECK(hipMemcpyAsync(b, s->m(), N * 8, hipMemcpyDeviceToHost, s->stream));
    b += N * 8;
    HIPCHECK(hipMemcpyAsync(b, s->sstep(), N * 4, hipMemcpyDeviceToHost, s->stream));
    b += N * 4;
    if ((st = copy_planes_d2h(b, (const char*)s->drop(), 3, N, P, 4, s->stream)) != LBM_OK) return st;
    b += 3 * N * 4;
    if (nev) HIPCHECK(hipMemcpyAsync(b, s->ev(), nev * sizeof(lbm_event), hipMemcpyDeviceToHost, s->stream));
  }
  HIPCHECK(hipStreamSynchronize(s->stream));
  return LBM_OK;
}

lbm_status lbm_load(lbm_sim* s, const void* blob, size_t n) {
  if (!s) return fail(LBM_EINVAL, "handle is NULL");
  if (!blob || n < 40) return fail(LBM_EINVAL, "blob too small");
  const char* b = (const char*)blob;
  uint64_t magic;
  int32_t hdr32[4];
  int64_t step, nev;
  memcpy(&magic, b, 8);
  memcpy(hdr32, b + 8, 16);
  memcpy(&step, b + 24, 8);
  memcpy(&nev, b + 32, 8);
  const int flags = (s->L.solute ? 1 : 0) | (s->L.react ? 2 : 0);
  if (magic != kMagic || hdr32[3] != kVersion) return fail(LBM_EINVAL, "not a checkpoint of this library");
  if (hdr32[0] != s->p.nx || hdr32[1] != s->p.ny || hdr32[2] != flags)
    return fail(LBM_EINVAL, "checkpoint is for another lattice or feature set");
  if (step < 0 || nev < 0 || nev > s->L.ev_cap) return fail(LBM_EINVAL, "bad checkpoint counters");
  if (n != blob_size(s, nev)) return fail(LBM_EINVAL, "checkpoint size mismatch");
  b += 40;
  const long long N = s->L.N, P = s->L.P;
  // the mask may hold only bit0 and the pending bits of the last two steps
  const char* mb = b + 18 * N * 4 + (s->L.solute ? 5 * N * 4 : 0);
  const unsigned allowed = 1u | pending_bit(step - 1) | pending_bit(step - 2);
  for (long long i = 0; i < N; ++i)
    if ((unsigned)(uint8_t)mb[i] & ~allowed) return fail(LBM_EINVAL, "bad mask byte at node %lld", i);
  if (s->L.solute && s->p.solute_q == 4) {
    // the D2Q4 solute lattice has no rest link: its plane must be empty
    const float* g0 = (const float*)(b + 18 * N * 4);
    for (long long i = 0; i < N; ++i)
      if (g0[i] != 0.0f) return fail(LBM_EINVAL, "D2Q4 checkpoint with a rest solute population at node %lld", i);
  }
  lbm_status st;
  if ((st = copy_planes_h2d((char*)s->f(0), b, 18, N, P, 4, s->stream)) != LBM_OK) return st;
  b += 18 * N * 4;
  if (s->L.solute) {
    if ((st = copy_planes_h2d((char*)s->g(0), b, 5, N, P, 4, s->stream)) != LBM_OK) return st;
    b += 5 * N * 4;
  }
  HIPCHECK(hipMemcpyAsync(s->mask(), b, N, hipMemcpyHostToDevice, s->stream));
  b += N;
  unsigned long long nev_u = (unsigned long long)nev;
  if (s->L.react) {
    HIPCHECK(hipMemcpyAsync(s->m(), b, N * 8, hipMemcpyHostToDevice, s->stream));
    b += N * 8;
    HIPCHECK(hipMemcpyAsync(s->sstep(), b, N * 4, hipMemcpyHostToDevice, s->stream));
    b += N * 4;
    if ((st = copy_planes_h2d((char*)s->drop(), b, 3, N, P, 4, s->stream)) != LBM_OK) return st;
    b += 3 * N * 4;
    if (nev) HIPCHECK(hipMemcpyAsync(s->ev(), b, nev * sizeof(lbm_event), hipMemcpyHostToDevice, s->stream));
  }
  HIPCHECK(hipMemcpyAsync(s->evc(), &nev_u, sizeof nev_u, hipMemcpyHostToDevice, s->stream));
  HIPCHECK(hipStreamSynchronize(s->stream));
  s->cur = 0;
  s->step = step;
  s->mom = false;
  s->poisoned = false;
  return LBM_OK;
}

lbm_status lbm_set_scheme(lbm_sim* s, int32_t scheme) {
  if (!s) return fail(LBM_EINVAL, "handle is NULL");
  if (scheme != LBM_SCHEME_AUTO && scheme != LBM_SCHEME_POPULATIONS && scheme != LBM_SCHEME_MOMENTS)
    return fail(LBM_EINVAL, "unknown scheme %d", scheme);
  if (scheme == LBM_SCHEME_MOMENTS && s->p.tau != 1.0)
    return fail(LBM_EINVAL, "the moment scheme needs tau = 1");
  s->scheme = scheme;
  return LBM_OK;
}

lbm_status lbm_set_tile(lbm_sim* s, int32_t tx, int32_t sy) {
  if (!s) return fail(LBM_EINVAL, "handle is NULL");
  if (!tile_ok(tx, sy)) return fail(LBM_EINVAL, "tile %d x %d not supported", tx, sy);
  s->tx = tx;
  s->sy = sy;
  return LBM_OK;
}

lbm_status lbm_set_load_hint(lbm_sim* s, int32_t nontemporal) {
  if (!s) return fail(LBM_EINVAL, "handle is NULL");
  if (nontemporal != 0 && nontemporal != 1) return fail(LBM_EINVAL, "load hint must be 0 or 1");
  s->nt = nontemporal;
  return LBM_OK;
}

lbm_status lbm_get_load_hint(const lbm_sim* s, int32_t* nontemporal) {
  if (!s || !nontemporal) return fail(LBM_EINVAL, "NULL argument");
  *nontemporal = s->nt;
  return LBM_OK;
}

lbm_status lbm_get_tile(const lbm_sim* s, int32_t* tx, int32_t* sy) {
  if (!s || !tx || !sy) return fail(LBM_EINVAL, "NULL argument");
  *tx = use_moments(s->scheme, s->p) ? 64 : s->tx;  // moment step: 64-lane tiles
  *sy = s->sy;
  return LBM_OK;
}

}  // extern "C"

namespace {

// Autotune cache: a JSON-lines file named by LBM_AUTOTUNE_CACHE, one object
// per line {"key": "<arch>:<nx>x<ny>:<flags>:<scheme>", "tx": .., "sy": .., "ms": ..,
// "nt": ..} (a line without "nt" means the default load policy).
std::string tune_key(const lbm_sim* s) {
  hipDeviceProp_t prop{};
  int dev = 0;
  char arch[64] = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
    for (char* c = arch; *c; ++c)
      if (*c == ':' || *c == '"' || *c == ' ') *c = '_';
  }
  char buf[160];
  snprintf(buf, sizeof buf, "%s:%dx%d:%d:%s", arch, s->p.nx, s->p.ny,
           (s->L.solute ? 1 : 0) | (s->L.react ? 2 : 0), use_moments(s->scheme, s->p) ? "mom" : "pop");
  return buf;
}

bool tune_lookup(const std::string& key, int* tx, int* sy, double* ms, int* nt) {
  const char* path = getenv("LBM_AUTOTUNE_CACHE");
  if (!path || !*path) return false;
  FILE* fh = fopen(path, "r");
  if (!fh) return false;
  char line[512], k[256];
  bool found = false;
  while (fgets(line, sizeof line, fh)) {
    int a = 0, b = 0;
    double m = 0;
    if (sscanf(line, " {\"key\": \"%255[^\"]\", \"tx\": %d, \"sy\": %d, \"ms\": %lf", k, &a, &b, &m) == 4 &&
        key == k && tile_ok(a, b)) {
      int h = 0;
      const char* q = strstr(line, "\"nt\":");
      if (q && (sscanf(q, "\"nt\": %d", &h) != 1 || (h != 0 && h != 1))) continue;
      *tx = a; *sy = b; *ms = m; *nt = h;
      found = true;  // the last entry for a key wins
    }
  }
  fclose(fh);
  return found;
}

void tune_store(const std::string& key, int tx, int sy, double ms, int nt) {
  const char* path = getenv("LBM_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  FILE* fh = fopen(path, "a");
  if (!fh) return;
  fprintf(fh, "{\"key\": \"%s\", \"tx\": %d, \"sy\": %d, \"ms\": %.6f, \"nt\": %d}\n", key.c_str(), tx,
          sy, ms, nt);
  fclose(fh);
}

// A launch shape and its measured time per step.
struct TuneCand {
  int tx, sy, nt;
  float ms;
};

// Second pass of the autotuners: a single short timing per shape cannot
// separate shapes a few percent apart (clock ramps and other work on the GPU
// move it by as much), so the three fastest of the first pass are timed
// again, interleaved, in three rounds of at least 4 x steps steps and min_ms
// each; the lowest median wins and its median is the reported time.
template <typename TimeFn>
TuneCand pick_shape(std::vector<TuneCand> cands, int steps, double min_ms, TimeFn&& time_shape,
                    lbm_status* st) {
  std::stable_sort(cands.begin(), cands.end(),
                   [](const TuneCand& a, const TuneCand& b) { return a.ms < b.ms; });
  const int k = (int)std::min<size_t>(3, cands.size());
  const double fast = std::max(1e-4, (double)cands[0].ms);
  const int steps2 = (int)std::min(20000.0, std::max(4.0 * steps, std::ceil(min_ms / fast)));
  std::vector<float> t(3 * k, 0.0f);
  for (int r = 0; r < 3 && *st == LBM_OK; ++r)
    for (int c = 0; c < k && *st == LBM_OK; ++c) *st = time_shape(cands[c], steps2, &t[3 * c + r]);
  if (*st != LBM_OK) return cands[0];
  TuneCand best = cands[0];
  best.ms = 1e30f;
  for (int c = 0; c < k; ++c) {
    float* v = &t[3 * c];
    std::sort(v, v + 3);
    if (v[1] < best.ms) {
      best = cands[c];
      best.ms = v[1];
    }
  }
  return best;
}

}  // namespace

extern "C" {

lbm_status lbm_autotune(lbm_sim* s, int32_t steps, int32_t* tx_out, int32_t* sy_out, double* best_ms) {
  lbm_status st = guard(s);
  if (st != LBM_OK) return st;
  if (steps < 1) return fail(LBM_EINVAL, "steps_per_candidate must be >= 1");
  {
    int ctx = 0, csy = 0, cnt = 0;
    double cms = 0;
    if (tune_lookup(tune_key(s), &ctx, &csy, &cms, &cnt)) {
      s->tx = ctx;
      s->sy = csy;
      s->nt = cnt;
      if (tx_out) *tx_out = ctx;
      if (sy_out) *sy_out = csy;
      if (best_ms) *best_ms = cms;
      return LBM_OK;
    }
  }
  size_t n = 0;
  if ((st = lbm_save(s, nullptr, 0, &n)) != LBM_OK) return st;
  std::vector<char> blob;
  try { blob.resize(n); } catch (...) { return fail(LBM_ENOMEM, "checkpoint buffer"); }
  if ((st = lbm_save(s, blob.data(), n, &n)) != LBM_OK) return st;
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  // ms per step of `nsteps` steps at shape c, after two untimed ones
  auto time_shape = [&](const TuneCand& c, int nsteps, float* ms_step) -> lbm_status {
    s->tx = c.tx;
    s->sy = c.sy;
    s->nt = c.nt;
    lbm_status r;
    if ((r = queue_steps(s, 2)) != LBM_OK) return r;
    if (hipEventRecord(e0, s->stream) != hipSuccess) return fail(LBM_EDEVICE, "autotune event");
    if ((r = queue_steps(s, nsteps)) != LBM_OK) return r;
    float ms = 0;
    if (hipEventRecord(e1, s->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      return fail(LBM_EDEVICE, "autotune timing");
    *ms_step = ms / nsteps;
    return LBM_OK;
  };
  const int txs[] = {64, 128, 256};
  const int sys[] = {6, 8, 9, 10, 12, 16, 20, 24, 28, 32, 40, 48, 64, 96, 128};
  std::vector<TuneCand> cands;
  for (int nt = 0; nt < 2 && st == LBM_OK; ++nt) {
    for (int tx : txs) {
      if (use_moments(s->scheme, s->p) && tx != 64) continue;  // 64-lane tiles only
      if (tx > 2 * s->p.nx + 2 && tx != 64) continue;
      for (int sy : sys) {
        if (sy > 2 * s->p.ny && sy != 8) continue;
        TuneCand c{tx, sy, nt, 0.0f};
        if ((st = time_shape(c, steps, &c.ms)) != LBM_OK) break;
        cands.push_back(c);
      }
      if (st != LBM_OK) break;
    }
  }
  // a single lattice runs long after tuning: 20 ms per second-pass timing
  TuneCand best{s->tx, s->sy, s->nt, 1e30f};
  if (st == LBM_OK && !cands.empty()) best = pick_shape(cands, steps, 20.0, time_shape, &st);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != LBM_OK) return st;
  if ((st = lbm_load(s, blob.data(), n)) != LBM_OK) return st;
  s->tx = best.tx;
  s->sy = best.sy;
  s->nt = best.nt;
  tune_store(tune_key(s), best.tx, best.sy, best.ms, best.nt);
  if (tx_out) *tx_out = best.tx;
  if (sy_out) *sy_out = best.sy;
  if (best_ms) *best_ms = best.ms;
  return LBM_OK;
}

void lbm_destroy(lbm_sim* s) { free(s); }

}  // extern "C"

// ===========================================================================
// Batched sweep: many independent lattices advanced by one launch per step.
// ===========================================================================

struct lbm_batch {
  int n;
  std::vector<lbm_params> p;
  std::vector<Layout> L;
  std::vector<size_t> base;   // workspace offset of each instance's buffers
  std::vector<size_t> stage;  // workspace offset of each instance's FP64 inputs
  hipStream_t stream;
  char* ws;
  StepArgs* d_insts;          // [n][2]: arguments for state parity 0 and 1
  std::vector<StepArgs> h_insts;
  int4* d_tiles;
  int max_tiles, ntiles;
  int4* d_capi;
  long long* d_step;
  double* d_table;
  int nslots;
  double* d_partial;
  double* d_out;
  int max_blocks;
  long long step;
  int tx, sy;
  int scheme;                 // LBM_SCHEME_*
  bool mom;                   // instance buffers hold moments of the last step
  bool solute, react, poisoned;
  int graph_chunk;
  hipGraphExec_t graph;
  hipStream_t cap_stream;     // library-owned stream used only to capture the graph
};

namespace {

struct BatchLayout {
  size_t insts, tiles, capi, stepc, table, partial, out, common, total;
  std::vector<Layout> L;
  std::vector<size_t> base, stage;
  int max_tiles, max_blocks;
};

// Columns a workgroup owns.  The moment step runs one wavefront (64 lanes)
// per tile and its stencil reaches two columns out; the population step
// reaches one.  A batch in the moment scheme runs its first
// (population-in) step on the same 64-lane tiling.
int owned_cols(int tx, bool moments) { return moments ? 60 : tx - 2; }

int tiles_for(const lbm_params& p, int tx, int sy) {
  const int own = owned_cols(tx, true);
  return ((p.nx + own - 1) / own) * ((p.ny + sy - 1) / sy);
}

bool batch_moments(const lbm_batch* b) { return use_moments(b->scheme, b->p[0]); }
bool batch_variants(const lbm_batch* b) {
  for (const lbm_params& p : b->p)
    if (p.c_eq > 0.0 || p.hold_x > 0 || p.solute_q == 4) return true;
  return false;
}
int batch_tx(const lbm_batch* b) { return batch_moments(b) ? 64 : b->tx; }

lbm_status batch_layout(int n, const lbm_params* p, int nslots, BatchLayout* B) {
  if (n < 1 || !p) return fail(LBM_EINVAL, "batch needs n >= 1 parameter records");
  if (nslots < 0 || nslots > 4096) return fail(LBM_EINVAL, "nslots must be in [0, 4096]");
  const bool solute = p[0].tau_g > 0.0, react = p[0].k_r > 0.0;
  B->max_tiles = 0;
  B->max_blocks = 1;
  for (int i = 0; i < n; ++i) {
    lbm_status st = check_params(&p[i]);
    if (st != LBM_OK) return fail(st, "instance %d: %s", i, g_err.c_str());
    if (p[i].tau != p[0].tau || p[i].G != p[0].G || p[i].accel[0] != p[0].accel[0] ||
        p[i].accel[1] != p[0].accel[1])
      return fail(LBM_EINVAL, "instance %d: tau, G and accel must be shared by the batch", i);
    if ((p[i].tau_g > 0.0) != solute || (p[i].k_r > 0.0) != react)
      return fail(LBM_EINVAL, "instance %d: solute/reaction switches must be shared", i);
    B->max_tiles += tiles_for(p[i], 64, 8);
    B->max_blocks = std::max(B->max_blocks, (int)std::min<long long>(1024, ((long long)p[i].nx * p[i].ny + 255) / 256));
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = a256(off + bytes);
    return o;
  };
  B->insts = take((size_t)2 * n * sizeof(StepArgs));
  B->tiles = take((size_t)B->max_tiles * sizeof(int4));
  B->capi = take((size_t)n * sizeof(int4));
  B->stepc = take(sizeof(long long));
  B->table = take((size_t)n * std::max(nslots, 1) * sizeof(double));
  B->partial = take((size_t)B->max_blocks * OBS_SLOTS * sizeof(double));
  B->out = take(OBS_OUT * sizeof(double));
  B->common = off;
  B->L.clear();
  B->base.clear();
  B->stage.clear();
  for (int i = 0; i < n; ++i) {
    Layout li = make_layout(p[i]);
    B->L.push_back(li);
    B->base.push_back(take(li.total));
    B->stage.push_back(take((size_t)3 * li.N * sizeof(double) + li.N));
  }
  B->total = off;
  return LBM_OK;
}

StepArgs instance_args(const lbm_batch* b, int i, int parity) {
  const lbm_params& p = b->p[i];
  const Layout& L = b->L[i];
  char* w = b->ws + b->base[i];
  StepArgs a{};
  a.fin = (float*)(w + L.f[parity]);
  a.fout = (float*)(w + L.f[parity ^ 1]);
  a.gin = L.solute ? (float*)(w + L.g[parity]) : nullptr;
  a.gout = L.solute ? (float*)(w + L.g[parity ^ 1]) : nullptr;
  a.mask = (uint8_t*)(w + L.mask);
  a.m = L.react ? (double*)(w + L.m) : nullptr;
  a.sstep = L.react ? (int32_t*)(w + L.sstep) : nullptr;
  a.drop = L.react ? (float*)(w + L.drop) : nullptr;
  a.ev = L.react ? (lbm_event*)(w + L.ev) : nullptr;
  a.ev_count = (unsigned long long*)(w + L.evc);
  a.ev_cap = L.ev_cap;
  a.P = L.P;
  a.nx = p.nx;
  a.ny = p.ny;
  a.tx_owned = owned_cols(b->tx, batch_moments(b));
  a.sy = b->sy;
  a.nstrips = (p.nx + a.tx_owned - 1) / a.tx_owned;
  a.nsegs = (p.ny + b->sy - 1) / b->sy;
  a.remap = 0;
  a.solute = L.solute;
  a.react = L.react;
  a.omega = 1.0 / p.tau;
  a.tau = p.tau;
  a.G = p.G;
  a.Gads1 = p.G_ads[0];
  a.Gads2 = p.G_ads[1];
  a.ax = p.accel[0];
  a.ay = p.accel[1];
  a.omega_g = L.solute ? 1.0 / p.tau_g : 0.0;
  a.k_r = p.k_r;
  a.threshold = p.threshold;
  a.c_eq = p.c_eq;
  a.c_hold = p.c_hold;
  a.hold_x = p.hold_x;
  a.q4 = p.solute_q == 4;
  return a;
}

void drop_graph(lbm_batch* b) {
  if (b->graph) {
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
}

// Rebuild the per-instance arguments and the tile list for the launch shape.
lbm_status batch_configure(lbm_batch* b) {
  drop_graph(b);
  b->h_insts.resize(2 * b->n);
  for (int i = 0; i < b->n; ++i) {
    b->h_insts[2 * i] = instance_args(b, i, 0);
    b->h_insts[2 * i + 1] = instance_args(b, i, 1);
  }
  std::vector<int4> order;
  const int own = owned_cols(b->tx, batch_moments(b));
  for (int i = 0; i < b->n; ++i) {
    const int ns = (b->p[i].nx + own - 1) / own, nq = (b->p[i].ny + b->sy - 1) / b->sy;
    // segment-major inside an instance, like the single-lattice step
    for (int q = 0; q < nq; ++q)
      for (int s = 0; s < ns; ++s) order.push_back(make_int4(i, s, q, 0));
  }
  const int T = (int)order.size();
  if (T > b->max_tiles) return fail(LBM_EINVAL, "tile list exceeds its buffer");
  std::vector<int4> tiles(T);
  for (int k = 0; k < T; ++k) tiles[k] = T >= 8 ? order[host_xcd_tile(k, T)] : order[k];
  b->ntiles = T;
  HIPCHECK(hipMemcpyAsync(b->d_insts, b->h_insts.data(), b->h_insts.size() * sizeof(StepArgs),
                          hipMemcpyHostToDevice, b->stream));
  HIPCHECK(hipMemcpyAsync(b->d_tiles, tiles.data(), T * sizeof(int4), hipMemcpyHostToDevice, b->stream));
  HIPCHECK(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

// Initial state of every instance from its staged FP64 inputs.
lbm_status batch_reset(lbm_batch* b) {
  drop_graph(b);
  for (int i = 0; i < b->n; ++i) {
    const Layout& L = b->L[i];
    char* w = b->ws + b->base[i];
    const double* st = (const double*)(b->ws + b->stage[i]);
    // the mask is restored too: growth changes it
    HIPCHECK(hipMemcpyAsync(w + L.mask, st + 3 * L.N, L.N, hipMemcpyDeviceToDevice, b->stream));
    HIPCHECK(hipMemsetAsync(w + L.evc, 0, sizeof(unsigned long long), b->stream));
    HIPCHECK(launch_init(st, st + L.N, L.solute ? st + 2 * L.N : nullptr,
                         (const uint8_t*)(w + L.mask), (float*)(w + L.f[0]),
                         L.solute ? (float*)(w + L.g[0]) : nullptr,
                         L.react ? (double*)(w + L.m) : nullptr,
                         L.react ? (int32_t*)(w + L.sstep) : nullptr,
                         L.react ? (float*)(w + L.drop) : nullptr, L.N, L.P, L.solute, L.react,
                         b->p[i].solute_q == 4, b->stream));
  }
  HIPCHECK(hipMemsetAsync(b->d_step, 0, sizeof(long long), b->stream));
  HIPCHECK(hipStreamSynchronize(b->stream));
  b->step = 0;
  b->mom = false;
  return LBM_OK;
}

int batch_kind(const lbm_batch* b) {
  return !batch_moments(b) ? KIND_POP : (b->mom ? KIND_MM : KIND_PM);
}

// Queues nsteps batched steps on stream st (offsets 0..nsteps-1 from the
// device step counter) and the counter's advance; the host-side step and
// scheme state follow.  Also used to capture the replayed graph.
lbm_status queue_batch(lbm_batch* b, int nsteps, hipStream_t st) {
  for (int t = 0; t < nsteps; ++t) {
    const int kind = batch_kind(b);
    hipError_t e = launch_step_batch(b->d_insts, b->d_tiles, b->ntiles, b->d_step, t, batch_tx(b),
                                     b->solute, b->react, batch_variants(b), kind, st);
    if (e != hipSuccess) return fail(LBM_EDEVICE, "batch step launch: %s", hipGetErrorString(e));
    b->mom = kind != KIND_POP;
  }
  if (nsteps > 0) {
    hipError_t e = launch_tick(b->d_step, nsteps, st);
    if (e != hipSuccess) return fail(LBM_EDEVICE, "step counter launch: %s", hipGetErrorString(e));
  }
  return LBM_OK;
}

lbm_status batch_launch(lbm_batch* b, long long nsteps) {
  while (nsteps > 0) {
    const int n = (int)std::min<long long>(nsteps, 1 << 20);
    lbm_status st = queue_batch(b, n, b->stream);
    if (st != LBM_OK) {
      b->poisoned = true;
      return st;
    }
    b->step += n;
    nsteps -= n;
  }
  return LBM_OK;
}

lbm_status bguard(const lbm_batch* b) {
  if (!b) return fail(LBM_EINVAL, "batch handle is NULL");
  if (b->poisoned) return fail(LBM_ESTATE, "batch poisoned by an earlier failure");
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_batch_workspace_bytes(int32_t n, const lbm_params* p, int32_t nslots, size_t* bytes) {
  if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
  BatchLayout B;
  lbm_status st = batch_layout(n, p, nslots, &B);
  if (st != LBM_OK) return st;
  *bytes = B.total;
  return LBM_OK;
}

lbm_status lbm_batch_init(int32_t n, const lbm_params* p, const uint8_t* const* solid,
                          const double* const* rho1, const double* const* rho2,
                          const double* const* conc, int32_t nslots, void* stream,
                          void* workspace, size_t ws_bytes, lbm_batch** out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  BatchLayout B;
  lbm_status st = batch_layout(n, p, nslots, &B);
  if (st != LBM_OK) return st;
  if (!solid || !rho1 || !rho2) return fail(LBM_EINVAL, "solid, rho1, rho2 arrays are required");
  if (!workspace || ((uintptr_t)workspace & 255u)) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < B.total) return fail(LBM_EINVAL, "workspace too small: %zu < %zu", ws_bytes, B.total);
  const bool solute = p[0].tau_g > 0.0;
  if (solute && !conc) return fail(LBM_EINVAL, "conc arrays are required when tau_g > 0");
  for (int i = 0; i < n; ++i) {
    const long long N = (long long)p[i].nx * p[i].ny;
    if (!solid[i] || !rho1[i] || !rho2[i] || (solute && !conc[i]))
      return fail(LBM_EINVAL, "instance %d: NULL input array", i);
    for (long long k = 0; k < N; ++k) {
      if (solid[i][k] > 1) return fail(LBM_EINVAL, "instance %d: mask value at node %lld", i, k);
      if (solid[i][k]) continue;
      if (!(rho1[i][k] >= 0.0) || !(rho2[i][k] >= 0.0) || !std::isfinite(rho1[i][k]) ||
          !std::isfinite(rho2[i][k]) || rho1[i][k] + rho2[i][k] <= 0.0)
        return fail(LBM_EINVAL, "instance %d: bad density at node %lld", i, k);
      if (solute && (!(conc[i][k] >= 0.0) || !std::isfinite(conc[i][k])))
        return fail(LBM_EINVAL, "instance %d: bad concentration at node %lld", i, k);
    }
  }
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return fail(LBM_ENOMEM, "batch handle");
  b->n = n;
  b->p.assign(p, p + n);
  b->L = B.L;
  b->base = B.base;
  b->stage = B.stage;
  b->stream = (hipStream_t)stream;
  b->ws = (char*)workspace;
  b->d_insts = (StepArgs*)(b->ws + B.insts);
  b->d_tiles = (int4*)(b->ws + B.tiles);
  b->max_tiles = B.max_tiles;
  b->d_capi = (int4*)(b->ws + B.capi);
  b->d_step = (long long*)(b->ws + B.stepc);
  b->d_table = (double*)(b->ws + B.table);
  b->nslots = nslots;
  b->d_partial = (double*)(b->ws + B.partial);
  b->d_out = (double*)(b->ws + B.out);
  b->max_blocks = B.max_blocks;
  b->tx = 128;
  b->sy = 24;
  b->scheme = LBM_SCHEME_AUTO;
  b->mom = false;
  b->solute = solute;
  b->react = p[0].k_r > 0.0;
  b->graph = nullptr;
  b->graph_chunk = 0;
  b->cap_stream = nullptr;
  std::vector<int4> capi(n);
  for (int i = 0; i < n; ++i) {
    const long long N = b->L[i].N;
    char* stg = b->ws + b->stage[i];
    capi[i] = make_int4(p[i].x_in, p[i].x_out, p[i].y0, p[i].W);
#define BCK(expr) do { hipError_t e_ = (expr); if (e_ != hipSuccess) { delete b; return fail(LBM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); } } while (0)
    BCK(hipMemcpyAsync(stg, rho1[i], N * 8, hipMemcpyHostToDevice, b->stream));
    BCK(hipMemcpyAsync(stg + N * 8, rho2[i], N * 8, hipMemcpyHostToDevice, b->stream));
    if (solute) BCK(hipMemcpyAsync(stg + 2 * N * 8, conc[i], N * 8, hipMemcpyHostToDevice, b->stream));
    BCK(hipMemcpyAsync(stg + 3 * N * 8, solid[i], N, hipMemcpyHostToDevice, b->stream));
  }
  BCK(hipMemcpyAsync(b->d_capi, capi.data(), n * sizeof(int4), hipMemcpyHostToDevice, b->stream));
#undef BCK
  if ((st = batch_configure(b)) != LBM_OK || (st = batch_reset(b)) != LBM_OK) {
    delete b;
    return st;
  }
  *out = b;
  return LBM_OK;
}

lbm_status lbm_batch_set_tile(lbm_batch* b, int32_t tx, int32_t sy) {
  lbm_status st = bguard(b);
  if (st != LBM_OK) return st;
  if (!(tx == 64 || tx == 128 || tx == 256) || sy < 8 || sy > 4096)
    return fail(LBM_EINVAL, "batch tile %d x %d not supported (tx 64/128/256, sy >= 8)", tx, sy);
  b->tx = tx;
  b->sy = sy;
  return batch_configure(b);
}

lbm_status lbm_batch_set_graph(lbm_batch* b, int32_t chunk) {
  lbm_status st = bguard(b);
  if (st != LBM_OK) return st;
  if (chunk < 0 || chunk > 100000) return fail(LBM_EINVAL, "chunk must be in [0, 100000]");
  drop_graph(b);
  b->graph_chunk = chunk;
  return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps) {
  lbm_status st = bguard(b);
  if (st != LBM_OK) return st;
  if (nsteps < 0) return fail(LBM_EINVAL, "nsteps < 0");
  long long left = nsteps;
  // the first step of a moment-scheme run reads populations: launch it
  // directly, so that the captured chunk holds moment steps only
  if (left > 0 && batch_kind(b) == KIND_PM) {
    if ((st = batch_launch(b, 1)) != LBM_OK) return st;
    left -= 1;
  }
  if (b->graph_chunk > 0 && left >= b->graph_chunk) {
    if (!b->graph) {
      // capture chunk steps once; the kernels read the step index from the
      // device counter, so every replay continues where the last one ended
      // captured on a library-owned stream (the caller's may be the legacy
      // default stream, which cannot be captured), launched on the caller's
      hipGraph_t g = nullptr;
      if (!b->cap_stream) HIPCHECK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
      HIPCHECK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
      const lbm_status cst = queue_batch(b, b->graph_chunk, b->cap_stream);
      if (cst != LBM_OK) {
        (void)hipStreamEndCapture(b->cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        return cst;
      }
      HIPCHECK(hipStreamEndCapture(b->cap_stream, &g));
      hipError_t e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        b->graph = nullptr;
        return fail(LBM_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
      }
    }
    while (left >= b->graph_chunk) {
      HIPCHECK(hipGraphLaunch(b->graph, b->stream));
      left -= b->graph_chunk;
      b->step += b->graph_chunk;
    }
  }
  return batch_launch(b, left);
}

lbm_status lbm_batch_record_fronts(lbm_batch* b, int32_t slot) {
  lbm_status st = bguard(b);
  if (st != LBM_OK) return st;
  if (slot < 0 || slot >= b->nslots) return fail(LBM_EINVAL, "slot out of range");
  HIPCHECK(launch_front_batch(b->d_insts, b->d_capi, b->d_step, b->n, slot, b->nslots, b->mom,
                              b->d_table, b->stream));
  return LBM_OK;
}

lbm_status lbm_batch_fronts(lbm_batch* b, double* host) {
  lbm_status st = bguard(b);
  if (st != LBM_OK) return st;
  if (!host) return fail(LBM_EINVAL, "host is NULL");
  HIPCHECK(hipMemcpyAsync(host, b->d_table, (size_t)b->n * b->nslots * sizeof(double),
                          hipMemcpyDeviceToHost, b->stream));
  HIPCHECK(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

lbm_status lbm_batch_observe(lbm_batch* b, int32_t i, lbm_obs* o) {
  lbm_status st = bguard(b);
  if (st != LBM_OK) return st;
  if (i < 0 || i >= b->n || !o) return fail(LBM_EINVAL, "bad instance or NULL out");
  const lbm_params& p = b->p[i];
  const StepArgs& a = b->h_insts[2 * i + (int)(b->step & 1)];
  const Layout& L = b->L[i];
  const int nblocks = (int)std::min<long long>(b->max_blocks, (L.N + 255) / 256);
  hipError_t e = launch_observe(a.fin, a.gin, a.mask, a.m, a.drop, a.sstep, p.nx, p.ny, L.P,
                                pending_bit(b->step - 1), pending_bit(b->step - 2), b->mom,
                                L.solute, L.react, nblocks, b->d_partial, b->d_out, p.x_in, p.x_out,
                                p.y0, p.W, b->stream);
  double h[OBS_OUT];
  unsigned long long nev = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(h, b->d_out, sizeof h, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&nev, a.ev_count, sizeof nev, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) { b->poisoned = true; return fail(LBM_EDEVICE, "batch observe: %s", hipGetErrorString(e)); }
  memset(o, 0, sizeof *o);
  o->step = b->step;
  o->mass[0] = h[0];
  o->mass[1] = h[1];
  o->solute = h[2];
  o->precipitate = h[3];
  o->mass_removed[0] = h[4];
  o->mass_removed[1] = h[5];
  o->solute_removed = h[6];
  o->n_solid = (int64_t)h[7];
  o->nonfinite = h[8] > 0.0;
  o->n_events = (int64_t)nev;
  capillary_radii(p, h, o);
  if (o->nonfinite) {
    b->poisoned = true;
    return fail(LBM_ENONFINITE, "instance %d holds a NaN/Inf at step %lld", i, b->step);
  }
  return LBM_OK;
}

lbm_status lbm_batch_fields(lbm_batch* b, int32_t i, uint32_t mask, double* host) {
  lbm_status st = bguard(b);
  if (st != LBM_OK) return st;
  if (i < 0 || i >= b->n || (mask && !host) || (mask >> 7)) return fail(LBM_EINVAL, "bad arguments");
  const lbm_params& p = b->p[i];
  const StepArgs& a = b->h_insts[2 * i + (int)(b->step & 1)];
  const long long N = b->L[i].N;
  double* stage = (double*)a.fout;  // idle buffer: rewritten by the next step before it is read
  hipError_t e = launch_fields(a.fin, a.gin, a.mask, a.m, p.nx, p.ny, b->L[i].P,
                               pending_bit(b->step - 1), pending_bit(b->step - 2), b->mom,
                               b->L[i].solute, b->L[i].react, p.G, p.G_ads[0], p.G_ads[1],
                               p.accel[0], p.accel[1], stage, b->stream);
  int k = 0;
  for (int bit = 0; bit < 7 && e == hipSuccess; ++bit) {
    if (!(mask & (1u << bit))) continue;
    e = hipMemcpyAsync(host + (size_t)k * N, stage + (size_t)bit * N, N * sizeof(double),
                       hipMemcpyDeviceToHost, b->stream);
    ++k;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) { b->poisoned = true; return fail(LBM_EDEVICE, "batch fields: %s", hipGetErrorString(e)); }
  return LBM_OK;
}

lbm_status lbm_batch_events(lbm_batch* b, int32_t i, int64_t first, lbm_event* buf, int64_t cap,
                            int64_t* n) {
  lbm_status st = bguard(b);
  if (st != LBM_OK) return st;
  if (i < 0 || i >= b->n || !n || first < 0 || cap < 0 || (cap > 0 && !buf))
    return fail(LBM_EINVAL, "bad events arguments");
  const StepArgs& a = b->h_insts[2 * i];
  unsigned long long nev = 0;
  HIPCHECK(hipMemcpyAsync(&nev, a.ev_count, sizeof nev, hipMemcpyDeviceToHost, b->stream));
  HIPCHECK(hipStreamSynchronize(b->stream));
  *n = (int64_t)nev;
  long long k = std::min<long long>(std::min<long long>((long long)nev, a.ev_cap) - first, cap);
  if (k > 0) {
    HIPCHECK(hipMemcpyAsync(buf, a.ev + first, k * sizeof(lbm_event), hipMemcpyDeviceToHost, b->stream));
    HIPCHECK(hipStreamSynchronize(b->stream));
  }
  return LBM_OK;
}

lbm_status lbm_batch_autotune(lbm_batch* b, int32_t steps, int32_t* tx_out, int32_t* sy_out,
                              double* best_ms) {
  lbm_status st = bguard(b);
  if (st != LBM_OK) return st;
  if (steps < 1) return fail(LBM_EINVAL, "steps must be >= 1");
  if (b->step != 0) return fail(LBM_EINVAL, "batch autotune runs before the first step");
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  auto time_shape = [&](const TuneCand& c, int nsteps, float* ms_step) -> lbm_status {
    b->tx = c.tx;
    b->sy = c.sy;
    lbm_status r;
    if ((r = batch_configure(b)) != LBM_OK || (r = batch_launch(b, 2)) != LBM_OK) return r;
    if (hipEventRecord(e0, b->stream) != hipSuccess) return fail(LBM_EDEVICE, "autotune event");
    if ((r = batch_launch(b, nsteps)) != LBM_OK) return r;
    float ms = 0;
    if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      return fail(LBM_EDEVICE, "autotune timing");
    *ms_step = ms / nsteps;
    return LBM_OK;
  };
  const int txs[] = {64, 128, 256};
  const int sys[] = {8, 9, 10, 12, 16, 20, 24, 32, 40, 48, 64, 80};
  std::vector<TuneCand> cands;
  for (int tx : txs) {
    if (batch_moments(b) && tx != 64) continue;  // 64-lane tiles only
    for (int sy : sys) {
      TuneCand c{tx, sy, 0, 0.0f};
      if ((st = time_shape(c, steps, &c.ms)) != LBM_OK) break;
      cands.push_back(c);
    }
    if (st != LBM_OK) break;
  }
  // a sweep's tuning is part of its cost: 5 ms per second-pass timing
  TuneCand best{b->tx, b->sy, 0, 1e30f};
  if (st == LBM_OK && !cands.empty()) best = pick_shape(cands, steps, 5.0, time_shape, &st);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != LBM_OK) return st;
  b->tx = best.tx;
  b->sy = best.sy;
  if ((st = batch_configure(b)) != LBM_OK || (st = batch_reset(b)) != LBM_OK) return st;
  if (tx_out) *tx_out = best.tx;
  if (sy_out) *sy_out = best.sy;
  if (best_ms) *best_ms = best.ms;
  return LBM_OK;
}

lbm_status lbm_batch_set_scheme(lbm_batch* b, int32_t scheme) {
  lbm_status st = bguard(b);
  if (st != LBM_OK) return st;
  if (scheme != LBM_SCHEME_AUTO && scheme != LBM_SCHEME_POPULATIONS && scheme != LBM_SCHEME_MOMENTS)
    return fail(LBM_EINVAL, "unknown scheme %d", scheme);
  if (scheme == LBM_SCHEME_MOMENTS && b->p[0].tau != 1.0)
    return fail(LBM_EINVAL, "the moment scheme needs tau = 1");
  if (b->step != 0) return fail(LBM_EINVAL, "the batch scheme is chosen before the first step");
  b->scheme = scheme;
  return batch_configure(b);
}

lbm_status lbm_batch_get_tile(const lbm_batch* b, int32_t* tx, int32_t* sy) {
  if (!b || !tx || !sy) return fail(LBM_EINVAL, "NULL argument");
  *tx = batch_tx(b);
  *sy = b->sy;
  return LBM_OK;
}

void lbm_batch_destroy(lbm_batch* b) {
  if (!b) return;
  drop_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
}

}  // extern "C"
