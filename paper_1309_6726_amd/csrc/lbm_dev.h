// Private declarations shared by the kernels and the host layer of the HIP
// library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm.h"

namespace lbmdev {

constexpr int OBS_SLOTS = 9;   // per-block partial sums of the observe reduction
constexpr int OBS_OUT = OBS_SLOTS + 3;

struct StepArgs {
  const float* fin;
  float* fout;
  const float* gin;
  float* gout;
  uint8_t* mask;
  double* m;
  int32_t* sstep;
  float* drop;
  lbm_event* ev;
  unsigned long long* ev_count;
  long long ev_cap;
  long long P;        // plane stride in elements
  long long step;     // index n of the state being advanced (n -> n+1)
  int nx, ny;
  int tx_owned;       // columns owned per workgroup (blockDim.x - 2)
  int sy;             // rows owned per workgroup
  int nstrips, nsegs;
  int remap;          // XCD-aware tile order (tile count divisible by 8)
  int solute, react;
  unsigned bit_prev;  // pending bit written by the previous step
  unsigned bit_cur;   // pending bit this step writes
  float omega;        // 1/tau
  float tau;
  float G, Gads1, Gads2, ax, ay;
  float omega_g;      // 1/tau_g
  double k_r, threshold;
};

// Records a message for lbm_last_error() and returns s.
lbm_status fail(lbm_status s, const char* fmt, ...);

hipError_t launch_step(const StepArgs& a, int tx, int arith64, hipStream_t st);
hipError_t launch_step_batch(const StepArgs* insts, const int4* tiles, int ntiles,
                             const long long* stepc, int tx, int solute, int react, int arith64,
                             hipStream_t st);
hipError_t launch_front_batch(const StepArgs* insts, const int4* capi, const long long* stepc,
                              int n, int slot, int nslots, double* table, hipStream_t st);
int host_xcd_tile(int b, int T);
hipError_t launch_init(const double* r1, const double* r2, const double* c, const uint8_t* mask,
                       float* f, float* g, double* m, int32_t* sstep, float* drop, long long N,
                       long long P, int solute, int react, hipStream_t st);
hipError_t launch_observe(const float* f, const float* g, const uint8_t* mask, const double* m,
                          const float* drop, const int32_t* sstep, long long N, long long P,
                          int nx, unsigned bit_prev, int solute, int react, int nblocks,
                          double* partial, double* out, int x_in, int x_out, int y0, int W,
                          hipStream_t st);
hipError_t launch_fields(const float* f, const float* g, const uint8_t* mask, const double* m,
                         int nx, int ny, long long P, unsigned bit_prev, int solute, int react,
                         float G, float Gads1, float Gads2, float ax, float ay, double* out,
                         hipStream_t st);

}  // namespace lbmdev
