// Private declarations shared by the kernels and the host layer of the HIP
// library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm.h"

namespace lbmdev {

constexpr int OBS_SLOTS = 9;   // per-block partial sums of the observe reduction
constexpr int OBS_OUT = OBS_SLOTS + 6;  // + capillary: z, delta_e, closure, area, min width, steps

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
  int tx_owned;       // columns owned per workgroup (blockDim.x - 2, or - 4 in
                      // the moment step, whose stencil reaches two columns out)
  int sy;             // rows owned per workgroup
  int nstrips, nsegs;
  int remap;          // XCD-aware tile order (tile count divisible by 8)
  int solute, react;
  unsigned bit_p1;    // pending bit written by step n-1 (solid in state n)
  unsigned bit_p2;    // pending bit written by step n-2 (folded into bit0 now)
  unsigned bit_cur;   // pending bit this step writes
  // model parameters in FP64 (kernel arguments stay in scalar registers)
  double omega;       // 1/tau
  double tau;
  double G, Gads1, Gads2, ax, ay;
  double omega_g;     // 1/tau_g
  double k_r, threshold;
  double c_eq;        // saturation concentration of the reaction (0: plain first order)
  double c_hold;      // held concentration of the source region x < hold_x
  int hold_x;         // 0: no held source
  int q4;             // 1: D2Q4 solute lattice, 0: D2Q5
};

// Growth marks rotate over three pending bits: step n marks a node with
// pending_bit(n); step n+1 books the populations it carried; step n+2 folds
// the mark into bit0.  In state n the solid set of state n-1 is
// bit0 | pending(n-2) and that of state n adds pending(n-1); both stay
// readable while a step runs, whatever order its workgroups take.
__host__ __device__ inline unsigned pending_bit(long long n) {
  return 2u << (unsigned)(((n % 3) + 3) % 3);
}

// Kinds of step kernel.  POP: populations in, populations out.  At tau = 1
// the post-collision populations are the equilibria of (rho_s, v_s) of each
// component, so the state can be kept as six moments per node: PM collides
// populations and stores moments, MM reads moments (rebuilding the incoming
// populations by gathering from the neighbours) and stores moments.
enum StepKind { KIND_POP = 0, KIND_PM = 1, KIND_MM = 2 };

// Records a message for lbm_last_error() and returns s.
lbm_status fail(lbm_status s, const char* fmt, ...);

// nt: non-temporal load hint (moment and population steps)
hipError_t launch_step(const StepArgs& a, int tx, int kind, int nt, hipStream_t st);
// var: some instance uses a reaction or solute-lattice variant
// One batched step at index *stepc + j; a sequence of n such launches
// (j = 0..n-1) is followed by launch_tick(stepc, n).
hipError_t launch_step_batch(const StepArgs* insts, const int4* tiles, int ntiles,
                             const long long* stepc, int j, int tx, int solute, int react,
                             int var, int kind, hipStream_t st);
hipError_t launch_tick(long long* stepc, int n, hipStream_t st);
hipError_t launch_front_batch(const StepArgs* insts, const int4* capi, const long long* stepc,
                              int n, int slot, int nslots, int mom, double* table, hipStream_t st);
// Populations of state n rebuilt from stored moments (zero at nodes solid in
// state n-1) into fout[18][P].
hipError_t launch_unpack(const float* M, const uint8_t* mask, int nx, int ny, long long P,
                         unsigned sprev, float* fout, hipStream_t st);
int host_xcd_tile(int b, int T);
hipError_t launch_init(const double* r1, const double* r2, const double* c, const uint8_t* mask,
                       float* f, float* g, double* m, int32_t* sstep, float* drop, long long N,
                       long long P, int solute, int react, int q4, hipStream_t st);
// Observers of state n.  f holds populations (mom = 0) or the moments of the
// last step (mom = 1); p1, p2 are pending(n-1), pending(n-2).
hipError_t launch_observe(const float* f, const float* g, const uint8_t* mask, const double* m,
                          const float* drop, const int32_t* sstep, int nx, int ny, long long P,
                          unsigned p1, unsigned p2, int mom, int solute, int react, int nblocks,
                          double* partial, double* out, int x_in, int x_out, int y0, int W,
                          hipStream_t st);
hipError_t launch_fields(const float* f, const float* g, const uint8_t* mask, const double* m,
                         int nx, int ny, long long P, unsigned p1, unsigned p2, int mom,
                         int solute, int react, double G, double Gads1, double Gads2, double ax,
                         double ay, double* out, hipStream_t st);

}  // namespace lbmdev
