// Device kernels of the reactive two-component lattice Boltzmann step for
// gfx950 (MI355X).  The step follows the model of Sergi, Grossi, Leidi &
// Ortona (section "LB models"): D2Q9 BGK for both fluid components with
// bounce-back at solids, cohesion and adhesion forces, D2Q5 BGK solute lattice
// advected by the flow, first-order precipitation at wall-adjacent nodes and
// threshold growth of the solid phase.
//
// Memory layout in HBM (structure of arrays, plane stride P >= nx*ny, P a
// multiple of 64 so every plane starts 256-byte aligned):
//   f  float[18][P]  populations, component-major, link order
//                    (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1)
//   g  float[5][P]   solute populations (first five links)
//   mask uint8[P]    bit0 solid; bit1 / bit2 growth pending, set by the step
//                    of even / odd parity
//   m  double[P]     precipitated mass (touched only at wall-adjacent nodes)
//   sstep int32[P]   state index at which the node turned solid (-1 fluid)
//   drop float[3][P] populations a node carried when it turned solid
// f and g are double-buffered (A/B); a step reads one buffer and pushes into
// the other.
//
// Fused step, one kernel per time step.  A workgroup of TX threads owns
// TX-2 consecutive columns (one column per thread, plus one halo column on
// each side) and SY consecutive rows, and marches up its rows.  For every row
// it loads the node populations (coalesced along x), forms the densities,
// puts rho1, rho2 and the solid flag of the row into a 4-row LDS ring, and
// then collides the row below with the cohesion/adhesion stencil read from
// LDS, applies the reaction, and pushes the post-collision populations to the
// neighbours (or back into the node's own opposite link at a solid neighbour).
// Per-node arithmetic does not depend on the launch shape, so every tile shape
// gives bit-identical results.
//
// Growth timing.  In the step n -> n+1 a node whose precipitate exceeds the
// threshold still streams as fluid (the step uses the mask of state n); it is
// marked pending with the bit of parity n.  In the next step every thread
// reads bit0 | pending(n) as the solid flag, and the owner of the node books
// its populations into `drop` and folds the pending bit into bit0.  A node
// being marked in the current step is read as fluid by its neighbours, so
// concurrent workgroups never disagree on the mask.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_dev.h"

namespace lbmdev {

template <typename R>
__device__ __forceinline__ R feq(R w, R rho, R eu, R uu) {
  return w * rho * (R(1) + R(3) * eu + R(4.5) * eu * eu - R(1.5) * uu);
}

template <typename R>
__device__ __forceinline__ R sum9(const float* v) {
  return (((R)v[0] + (R)v[1]) + ((R)v[2] + (R)v[3])) + (((R)v[4] + (R)v[5]) + ((R)v[6] + (R)v[7])) +
         (R)v[8];
}

// s_waitcnt immediate for vmcnt(0) with expcnt and lgkmcnt left open (gfx9
// encoding: vmcnt[3:0] and [15:14], expcnt[6:4], lgkmcnt[11:8]).
#define VMCNT0 0x0F70

// Workgroup-wide LDS barrier that leaves outstanding global memory operations
// in flight (only LDS traffic is ordered); a single-wave workgroup needs no
// s_barrier at all.
__device__ __forceinline__ void lds_barrier(int TX) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  if (TX > 64) __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// R is the arithmetic type (float or double); populations are stored as FP32.
//
// Per workgroup, iteration k handles row r = ys - 1 + k: its populations,
// precipitate (owned rows) and the mask byte of row k+1 are requested
// together (the mask of row k arrived one iteration earlier), so each
// iteration waits on one memory round trip.  The densities of row k go to
// the LDS ring; after an LDS-only barrier row k-1 is collided and pushed.
// Offsets are 32-bit (the host guarantees 23 planes fit below 2^31).  The
// register budget is held to three waves per SIMD: a row iteration costs one
// memory round trip plus ~1 us of VALU work per wave, so resident waves are
// what hides the memory latency.
template <bool SOLUTE, bool REACT, typename R>
__device__ __forceinline__ void step_tile(const StepArgs& a, int strip, int seg, char* lds_raw) {
  const int TX = blockDim.x;
  R* s_r1 = (R*)lds_raw;                 // [4][TX] density of component 1 (0 at solid)
  R* s_r2 = s_r1 + 4 * TX;               // [4][TX] density of component 2
  float* s_s = (float*)(s_r2 + 4 * TX);  // [4][TX] solid flag 0/1

  const int t = threadIdx.x;
  const int nx = a.nx, ny = a.ny;
  const unsigned P = (unsigned)a.P;
  const int x0 = strip * a.tx_owned;
  const int nown = min(a.tx_owned, nx - x0);
  const bool active = t <= nown + 1;
  const bool owner = t >= 1 && t <= nown;
  int xc = x0 - 1 + t;
  if (xc < 0) xc += nx;
  if (xc >= nx) xc -= nx;
  const int xl = xc == 0 ? nx - 1 : xc - 1;
  const int xr = xc == nx - 1 ? 0 : xc + 1;
  const int ys = seg * a.sy;
  const int ye = min(ys + a.sy, ny);
  const int nrows = ye - ys + 2;
  const unsigned solid_bits = 1u | a.bit_prev;
  const int lane = __lane_id();
  const R WA = R(1) / R(9), WD = R(1) / R(36), W5A = R(1) / R(6);
  const float* __restrict__ fin = a.fin;
  const float* __restrict__ gin = a.gin;
  const uint8_t* __restrict__ maskp = a.mask;

  auto row_y = [&](int k) {
    int yr = ys - 1 + k;
    if (yr < 0) yr += ny;
    if (yr >= ny) yr -= ny;
    return yr;
  };

  float f[18], g[5], fn[18], gn[5];
  double m_cur = 0.0, m_nxt = 0.0;
  unsigned b_cur = 1, b_nxt = 1;
  unsigned mask_ahead = active ? (unsigned)maskp[(unsigned)row_y(0) * (unsigned)nx + (unsigned)xc] : 1u;

  for (int k = 0; k < nrows; ++k) {
    // ---- request row k: populations (+ solute, precipitate), next mask ----
    const unsigned idn = (unsigned)row_y(k) * (unsigned)nx + (unsigned)xc;
    const bool owned_row = k >= 1 && k <= nrows - 2;
    b_nxt = mask_ahead;
    if (active) {
      if (!(b_nxt & 1u)) {
#pragma unroll
        for (int q = 0; q < 18; ++q) fn[q] = fin[q * P + idn];
        if (SOLUTE && owner && owned_row) {
#pragma unroll
          for (int q = 0; q < 5; ++q) gn[q] = gin[q * P + idn];
        }
        if (REACT && owner && owned_row) m_nxt = a.m[idn];
      }
      if (k + 1 < nrows) mask_ahead = maskp[(unsigned)row_y(k + 1) * (unsigned)nx + (unsigned)xc];
    }
    // one wait per row, on every path: the row's loads (and the previous
    // row's stores, issued earlier) complete here, so nothing is pending on
    // the loop back edge
    __builtin_amdgcn_s_waitcnt(VMCNT0);
    R r1 = R(0), r2 = R(0);
    float sv = 1.0f;
    if (active && !(b_nxt & solid_bits)) {
      r1 = sum9<R>(fn);
      r2 = sum9<R>(fn + 9);
      sv = 0.0f;
    }
    const int slot = k & 3;
    s_r1[slot * TX + t] = r1;
    s_r2[slot * TX + t] = r2;
    s_s[slot * TX + t] = sv;
    lds_barrier(TX);

    // ---- collide and push row y = r - 1 -----------------------------------
    bool ev = false;
    int evx = 0, evy = 0;
    if (k >= 2 && owner) {
      const int y = ys + k - 2;
      const int yd = y == 0 ? ny - 1 : y - 1;
      const int yu = y == ny - 1 ? 0 : y + 1;
      const unsigned idx = (unsigned)y * (unsigned)nx + (unsigned)xc;
      const int sb = ((k - 2) & 3) * TX, sm = ((k - 1) & 3) * TX, sa = (k & 3) * TX;
      const R* A1 = s_r1;
      const R* A2 = s_r2;
      const float* AS = s_s;
      if (AS[sm + t] != 0.0f) {
        if (REACT && (b_cur & a.bit_prev)) {
          // turned solid at the end of the previous step: book its populations
          a.drop[idx] = (float)sum9<R>(f);
          a.drop[P + idx] = (float)sum9<R>(f + 9);
          a.drop[2 * P + idx] =
              SOLUTE ? (float)((((R)g[0] + (R)g[1]) + ((R)g[2] + (R)g[3])) + (R)g[4]) : 0.0f;
          a.mask[idx] = 1;
        }
      } else {
        const R rho1 = A1[sm + t], rho2 = A2[sm + t];
        const float sE = AS[sm + t + 1], sN = AS[sa + t], sW = AS[sm + t - 1], sS = AS[sb + t];
        const float sNE = AS[sa + t + 1], sNW = AS[sa + t - 1], sSW = AS[sb + t - 1], sSE = AS[sb + t + 1];
        // sum_i w_i v(x+e_i) e_i of the other component and of the solid mask
        const R c2x = WA * (A2[sm + t + 1] - A2[sm + t - 1]) +
                      WD * ((A2[sa + t + 1] - A2[sa + t - 1]) + (A2[sb + t + 1] - A2[sb + t - 1]));
        const R c2y = WA * (A2[sa + t] - A2[sb + t]) +
                      WD * ((A2[sa + t + 1] + A2[sa + t - 1]) - (A2[sb + t + 1] + A2[sb + t - 1]));
        const R c1x = WA * (A1[sm + t + 1] - A1[sm + t - 1]) +
                      WD * ((A1[sa + t + 1] - A1[sa + t - 1]) + (A1[sb + t + 1] - A1[sb + t - 1]));
        const R c1y = WA * (A1[sa + t] - A1[sb + t]) +
                      WD * ((A1[sa + t + 1] + A1[sa + t - 1]) - (A1[sb + t + 1] + A1[sb + t - 1]));
        const R csx = WA * R(sE - sW) + WD * R((sNE - sNW) + (sSE - sSW));
        const R csy = WA * R(sN - sS) + WD * R((sNE + sNW) - (sSE + sSW));

        const R G = (R)a.G, Ga1 = (R)a.Gads1, Ga2 = (R)a.Gads2, ax = (R)a.ax, ay = (R)a.ay;
        const R F1x = -G * rho1 * c2x - Ga1 * rho1 * csx + rho1 * ax;
        const R F1y = -G * rho1 * c2y - Ga1 * rho1 * csy + rho1 * ay;
        const R F2x = -G * rho2 * c1x - Ga2 * rho2 * csx + rho2 * ax;
        const R F2y = -G * rho2 * c1y - Ga2 * rho2 * csy + rho2 * ay;

        const R j1x = ((R)f[1] - (R)f[3]) + ((R)f[5] - (R)f[6]) + ((R)f[8] - (R)f[7]);
        const R j1y = ((R)f[2] - (R)f[4]) + ((R)f[5] + (R)f[6]) - ((R)f[7] + (R)f[8]);
        const R j2x = ((R)f[10] - (R)f[12]) + ((R)f[14] - (R)f[15]) + ((R)f[17] - (R)f[16]);
        const R j2y = ((R)f[11] - (R)f[13]) + ((R)f[14] + (R)f[15]) - ((R)f[16] + (R)f[17]);

        const R rt = rho1 + rho2;
        const R irt = R(1) / rt;
        const R upx = (j1x + j2x) * irt, upy = (j1y + j2y) * irt;
        const R tau = (R)a.tau;
        R v1x = upx, v1y = upy, v2x = upx, v2y = upy;
        if (rho1 > R(0)) { const R s = tau / rho1; v1x += s * F1x; v1y += s * F1y; }
        if (rho2 > R(0)) { const R s = tau / rho2; v2x += s * F2x; v2y += s * F2y; }
        const R ux = (j1x + j2x + R(0.5) * (F1x + F2x)) * irt;
        const R uy = (j1y + j2y + R(0.5) * (F1y + F2y)) * irt;

        // target offsets of the eight neighbours
        const unsigned iE = (unsigned)y * nx + xr, iW = (unsigned)y * nx + xl;
        const unsigned iN = (unsigned)yu * nx + xc, iS = (unsigned)yd * nx + xc;
        const unsigned iNE = (unsigned)yu * nx + xr, iNW = (unsigned)yu * nx + xl;
        const unsigned iSW = (unsigned)yd * nx + xl, iSE = (unsigned)yd * nx + xr;
        float* __restrict__ fo = a.fout;
        const R om = (R)a.omega;
        // collide one component and push each moving population as soon as it
        // is formed (halfway bounce-back into the node's own opposite link at
        // a solid neighbour); the rest population closes the mass balance
        // exactly (the moving-link weights are not exact binary fractions)
        auto collide_push = [&](const float* fc, unsigned base, R rho, R vx, R vy) {
          const R uu = vx * vx + vy * vy;
          R sum = R(0);
#define CP(i, opp, w, eu, bs, tgt)                                          \
  do {                                                                      \
    const R fi = (R)fc[i];                                                  \
    const R v = fi + om * (feq<R>(w, rho, eu, uu) - fi);                    \
    sum += v;                                                               \
    if (bs != 0.0f) fo[(base + (opp)) * P + idx] = (float)v;                \
    else fo[(base + (i)) * P + (tgt)] = (float)v;                           \
  } while (0)
          CP(1, 3, WA, vx, sE, iE);
          CP(2, 4, WA, vy, sN, iN);
          CP(3, 1, WA, -vx, sW, iW);
          CP(4, 2, WA, -vy, sS, iS);
          CP(5, 7, WD, vx + vy, sNE, iNE);
          CP(6, 8, WD, -vx + vy, sNW, iNW);
          CP(7, 5, WD, -vx - vy, sSW, iSW);
          CP(8, 6, WD, vx - vy, sSE, iSE);
#undef CP
          fo[base * P + idx] = (float)(rho - sum);
        };
        collide_push(f, 0u, rho1, v1x, v1y);
        collide_push(f + 9, 9u, rho2, v2x, v2y);

        if (SOLUTE) {
          const R C = (((R)g[0] + (R)g[1]) + ((R)g[2] + (R)g[3])) + (R)g[4];
          const R og = (R)a.omega_g;
          R gs[5];
          gs[1] = (R)g[1] + og * (W5A * C * (R(1) + R(3) * ux) - (R)g[1]);
          gs[2] = (R)g[2] + og * (W5A * C * (R(1) + R(3) * uy) - (R)g[2]);
          gs[3] = (R)g[3] + og * (W5A * C * (R(1) - R(3) * ux) - (R)g[3]);
          gs[4] = (R)g[4] + og * (W5A * C * (R(1) - R(3) * uy) - (R)g[4]);
          gs[0] = C - ((gs[1] + gs[2]) + (gs[3] + gs[4]));
          if (REACT) {
            const int ns = (int)sE + (int)sN + (int)sW + (int)sS;
            if (ns > 0) {
              const double phi = (double)rho1 / ((double)rho1 + (double)rho2);
              const double rr = a.k_r * (double)ns * phi;
              const double mm = m_cur + rr * (double)C;
              a.m[idx] = mm;
              const R keep = (R)(1.0 - rr);
#pragma unroll
              for (int q = 0; q < 5; ++q) gs[q] *= keep;
              if (mm > a.threshold) {
                a.mask[idx] = (uint8_t)a.bit_cur;
                a.sstep[idx] = (int32_t)(a.step + 1);
                ev = true;
                evx = xc;
                evy = y;
              }
            }
          }
          float* __restrict__ go = a.gout;
          go[idx] = (float)gs[0];
          if (sE != 0.0f) go[3 * P + idx] = (float)gs[1]; else go[1 * P + iE] = (float)gs[1];
          if (sN != 0.0f) go[4 * P + idx] = (float)gs[2]; else go[2 * P + iN] = (float)gs[2];
          if (sW != 0.0f) go[1 * P + idx] = (float)gs[3]; else go[3 * P + iW] = (float)gs[3];
          if (sS != 0.0f) go[2 * P + idx] = (float)gs[4]; else go[4 * P + iS] = (float)gs[4];
        }
      }
    }
    if (REACT) {
      // one atomic per wavefront reserves the event-log slots of its lanes
      const unsigned long long bal = __ballot(ev);
      if (bal) {
        const int leader = __ffsll((unsigned long long)bal) - 1;
        unsigned long long base = 0;
        if (lane == leader) base = atomicAdd(a.ev_count, (unsigned long long)__popcll(bal));
        base = __shfl(base, leader);
        if (ev) {
          const unsigned long long e = base + __popcll(bal & ((1ull << lane) - 1ull));
          if ((long long)e < a.ev_cap) {
            a.ev[e].x = evx;
            a.ev[e].y = evy;
            a.ev[e].step = a.step + 1;
          }
        }
      }
    }
    // rotate: row k becomes the row to collide next iteration
#pragma unroll
    for (int q = 0; q < 18; ++q) f[q] = fn[q];
    if (SOLUTE) {
#pragma unroll
      for (int q = 0; q < 5; ++q) g[q] = gn[q];
    }
    m_cur = m_nxt;
    b_cur = b_nxt;
  }
}

// XCD-aware order: the hardware hands block b to XCD b mod 8, so XCD x
// receives q + (x < r) of T blocks (q = T / 8, r = T mod 8).  Give each XCD a
// contiguous run of tiles, so vertically adjacent segments of a strip share
// one L2 and their halo rows are fetched from HBM once.
__host__ __device__ inline int xcd_tile(int b, int T) {
  const int q = T >> 3, r = T & 7, x = b & 7, j = b >> 3;
  return (x < r) ? x * (q + 1) + j : r * (q + 1) + (x - r) * q + j;
}

template <bool SOLUTE, bool REACT, typename R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8)))
k_step(const StepArgs a) {
  extern __shared__ char lds_raw[];
  const int T = a.nstrips * a.nsegs;
  const int tile = a.remap ? xcd_tile(blockIdx.x, T) : (int)blockIdx.x;
  const int strip = tile / a.nsegs;
  step_tile<SOLUTE, REACT, R>(a, strip, tile - strip * a.nsegs, lds_raw);
}

// Batched step: one launch advances every instance of a batch by one step.
// Block b takes tile tiles[b] (instance, strip, segment; the host orders the
// list per XCD); the instance's arguments for the current parity come from
// device memory, and the step index from the device counter, so a sequence of
// launches can be captured once in a graph and replayed.
template <bool SOLUTE, bool REACT, typename R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8)))
k_step_batch(const StepArgs* __restrict__ insts, const int4* __restrict__ tiles,
             const long long* __restrict__ stepc) {
  extern __shared__ char lds_raw[];
  const long long step = *stepc;
  const int4 e = tiles[blockIdx.x];
  StepArgs a = insts[2 * e.x + (int)(step & 1)];
  a.step = step;
  a.bit_prev = ((step - 1) & 1) ? 4u : 2u;
  a.bit_cur = (step & 1) ? 4u : 2u;
  step_tile<SOLUTE, REACT, R>(a, e.y, e.z, lds_raw);
}

// Advances the device step counter (a vector atomic, one lane).
__global__ void k_tick(long long* stepc) {
  if (threadIdx.x == 0) atomicAdd((unsigned long long*)stepc, 1ull);
}

// Rest-state populations from the FP64 densities (rounded once to FP32).
__global__ void k_init(const double* __restrict__ rho1, const double* __restrict__ rho2,
                       const double* __restrict__ conc, const uint8_t* __restrict__ mask,
                       float* __restrict__ f, float* __restrict__ g, double* __restrict__ m,
                       int32_t* __restrict__ sstep, float* __restrict__ drop, long long N,
                       long long P, int solute, int react) {
  const float w9[9] = {4.0f / 9.0f, 1.0f / 9.0f, 1.0f / 9.0f, 1.0f / 9.0f, 1.0f / 9.0f,
                       1.0f / 36.0f, 1.0f / 36.0f, 1.0f / 36.0f, 1.0f / 36.0f};
  const float w5[5] = {1.0f / 3.0f, 1.0f / 6.0f, 1.0f / 6.0f, 1.0f / 6.0f, 1.0f / 6.0f};
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const bool s = mask[i] != 0;
    const float r1 = s ? 0.0f : (float)rho1[i];
    const float r2 = s ? 0.0f : (float)rho2[i];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      f[q * P + i] = w9[q] * r1;
      f[(9 + q) * P + i] = w9[q] * r2;
    }
    if (solute) {
      const float c = s ? 0.0f : (float)conc[i];
#pragma unroll
      for (int q = 0; q < 5; ++q) g[q * P + i] = w5[q] * c;
    }
    if (react) {
      m[i] = 0.0;
      sstep[i] = s ? 0 : -1;
      drop[i] = 0.0f;
      drop[P + i] = 0.0f;
      drop[2 * P + i] = 0.0f;
    }
  }
}

// Observe, pass 1: per-block FP64 partial sums.  Slots:
// 0 mass1, 1 mass2, 2 solute, 3 precipitate, 4 removed1, 5 removed2,
// 6 removed solute, 7 solid count, 8 non-finite count.
__global__ void __launch_bounds__(256) k_obs_partial(const float* __restrict__ f,
                                                     const float* __restrict__ g,
                                                     const uint8_t* __restrict__ mask,
                                                     const double* __restrict__ m,
                                                     const float* __restrict__ drop, long long N,
                                                     long long P, unsigned bit_prev, int solute,
                                                     int react, double* __restrict__ partial) {
  __shared__ double red[OBS_SLOTS][256];
  double acc[OBS_SLOTS];
#pragma unroll
  for (int j = 0; j < OBS_SLOTS; ++j) acc[j] = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const unsigned b = mask[i];
    double s1 = 0, s2 = 0, sc = 0;
    if (!(b & 1u)) {
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        s1 += (double)f[q * P + i];
        s2 += (double)f[(9 + q) * P + i];
      }
      if (solute) {
#pragma unroll
        for (int q = 0; q < 5; ++q) sc += (double)g[q * P + i];
      }
    }
    if (b & (1u | bit_prev)) {
      acc[7] += 1.0;
      if (b & bit_prev) {  // turned solid at the end of the last step, not yet booked
        acc[4] += s1;
        acc[5] += s2;
        acc[6] += sc;
      }
    } else {
      acc[0] += s1;
      acc[1] += s2;
      acc[2] += sc;
      if (!isfinite(s1) || !isfinite(s2) || !isfinite(sc)) acc[8] += 1.0;
    }
    if (react) {
      acc[3] += m[i];
      acc[4] += (double)drop[i];
      acc[5] += (double)drop[P + i];
      acc[6] += (double)drop[2 * P + i];
    }
  }
#pragma unroll
  for (int j = 0; j < OBS_SLOTS; ++j) red[j][threadIdx.x] = acc[j];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int j = 0; j < OBS_SLOTS; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x < OBS_SLOTS) partial[blockIdx.x * OBS_SLOTS + threadIdx.x] = red[threadIdx.x][0];
}

// Observe, pass 2: fixed-order sum of the partials (deterministic).
__global__ void k_obs_final(const double* __restrict__ partial, int nblocks, double* __restrict__ out) {
  const int j = threadIdx.x;
  if (j >= OBS_SLOTS) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += partial[b * OBS_SLOTS + j];
  out[j] = s;
}

__device__ __forceinline__ void node_rho(const float* __restrict__ f, long long P, long long i,
                                         double* r1, double* r2) {
  double a = 0, b = 0;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    a += (double)f[q * P + i];
    b += (double)f[(9 + q) * P + i];
  }
  *r1 = a;
  *r2 = b;
}

// Capillary observables computed by one workgroup of 256 threads: centreline
// front, largest grown width and first closure.  out: [0] z, [1] delta_e,
// [2] closure step (-1 if none).
__device__ void capillary_obs(const float* __restrict__ f, const uint8_t* __restrict__ mask,
                              const int32_t* __restrict__ sstep, int nx, long long P,
                              unsigned bit_prev, int x_in, int x_out, int y0, int W, int react,
                              double* __restrict__ out) {
  __shared__ int s_min[256];
  __shared__ double s_de[256];
  __shared__ long long s_cl[256];
  const unsigned sb = 1u | bit_prev;
  const int nr = (W % 2 == 0) ? 2 : 1;
  const int row0 = (W % 2 == 0) ? (y0 + W / 2 - 1) : (y0 + (W - 1) / 2);
  int best = x_out;  // first x where the scan stops
  double de = 0.0;
  long long cl = -1;
  for (int x = x_in + threadIdx.x; x < x_out; x += blockDim.x) {
    // front predicate at x
    bool blocked = false, nblocked = false;
    double phi = 0, phin = 0;
    for (int r = 0; r < nr; ++r) {
      const long long i = (long long)(row0 + r) * nx + x;
      if (mask[i] & sb) blocked = true;
      else { double a, b; node_rho(f, P, i, &a, &b); phi += a / (a + b); }
    }
    phi /= nr;
    if (x + 1 < x_out) {
      for (int r = 0; r < nr; ++r) {
        const long long i = (long long)(row0 + r) * nx + x + 1;
        if (mask[i] & sb) nblocked = true;
        else { double a, b; node_rho(f, P, i, &a, &b); phin += a / (a + b); }
      }
      phin /= nr;
    }
    const bool stop = blocked || (x == x_in && phi < 0.5) ||
                      (x + 1 < x_out && !nblocked && phi >= 0.5 && phin < 0.5);
    if (stop && x < best) best = x;
    // growth from the two walls in this column
    int db = 0, dt = 0;
    while (db < W && (mask[(long long)(y0 + db) * nx + x] & sb)) ++db;
    while (dt < W && (mask[(long long)(y0 + W - 1 - dt) * nx + x] & sb)) ++dt;
    double col;
    if (db >= W) {
      col = 0.5 * W;
      long long last = 0;
      if (react)
        for (int y = y0; y < y0 + W; ++y) {
          const long long st = sstep[(long long)y * nx + x];
          if (st > last) last = st;
        }
      if (cl < 0 || last < cl) cl = last;
    } else {
      col = (double)(db > dt ? db : dt);
    }
    if (col > de) de = col;
  }
  s_min[threadIdx.x] = best;
  s_de[threadIdx.x] = de;
  s_cl[threadIdx.x] = cl;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      s_min[threadIdx.x] = min(s_min[threadIdx.x], s_min[threadIdx.x + s]);
      s_de[threadIdx.x] = fmax(s_de[threadIdx.x], s_de[threadIdx.x + s]);
      const long long o = s_cl[threadIdx.x + s];
      if (o >= 0 && (s_cl[threadIdx.x] < 0 || o < s_cl[threadIdx.x])) s_cl[threadIdx.x] = o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int x = s_min[0];
    double z = (double)(x_out - x_in);
    if (x < x_out) {
      bool blocked = false;
      double phi = 0, phin = 0;
      for (int r = 0; r < nr; ++r) {
        const long long i = (long long)(row0 + r) * nx + x;
        if (mask[i] & sb) blocked = true;
        else { double a, b; node_rho(f, P, i, &a, &b); phi += a / (a + b); }
      }
      phi /= nr;
      if (blocked) z = (double)(x - x_in);
      else if (x == x_in && phi < 0.5) z = 0.0;
      else {
        for (int r = 0; r < nr; ++r) {
          const long long i = (long long)(row0 + r) * nx + x + 1;
          double a, b; node_rho(f, P, i, &a, &b); phin += a / (a + b);
        }
        phin /= nr;
        z = (double)x + (phi - 0.5) / (phi - phin) - x_in;
      }
    }
    out[0] = z;
    out[1] = s_de[0];
    out[2] = (double)s_cl[0];
  }
}

__global__ void __launch_bounds__(256) k_obs_capillary(const float* __restrict__ f,
                                                       const uint8_t* __restrict__ mask,
                                                       const int32_t* __restrict__ sstep,
                                                       int nx, long long P, unsigned bit_prev,
                                                       int x_in, int x_out, int y0, int W,
                                                       int react, double* __restrict__ out) {
  capillary_obs(f, mask, sstep, nx, P, bit_prev, x_in, x_out, y0, W, react, out);
}

// Front of every instance of a batch (workgroup i -> instance i) into column
// `slot` of the n x nslots table; queued without synchronisation.
__global__ void __launch_bounds__(256) k_front_batch(const StepArgs* __restrict__ insts,
                                                     const int4* __restrict__ capi,
                                                     const long long* __restrict__ stepc,
                                                     int slot, int nslots,
                                                     double* __restrict__ table) {
  __shared__ double res[3];
  const long long step = *stepc;
  const int i = blockIdx.x;
  const StepArgs& a = insts[2 * i + (int)(step & 1)];
  const int4 c = capi[i];  // x_in, x_out, y0, W
  if (c.w <= 0) {
    if (threadIdx.x == 0) table[(long long)i * nslots + slot] = __builtin_nan("");
    return;
  }
  capillary_obs(a.fin, a.mask, a.sstep, a.nx, a.P, ((step - 1) & 1) ? 4u : 2u, c.x, c.y, c.z,
                c.w, a.react, res);
  if (threadIdx.x == 0) table[(long long)i * nslots + slot] = res[0];
}

// Macroscopic fields of the current state as FP64 planes:
// 0 rho1, 1 rho2, 2 ux, 3 uy, 4 conc, 5 precipitate, 6 solid.
__global__ void k_fields(const float* __restrict__ f, const float* __restrict__ g,
                         const uint8_t* __restrict__ mask, const double* __restrict__ m, int nx,
                         int ny, long long P, unsigned bit_prev, int solute, int react, float G,
                         float Gads1, float Gads2, float ax, float ay, double* __restrict__ out) {
  const long long N = (long long)nx * ny;
  const unsigned sb = 1u | bit_prev;
  const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % nx), y = (int)(i / nx);
    const bool s = (mask[i] & sb) != 0;
    double r1 = 0, r2 = 0, ux = 0, uy = 0, c = 0;
    if (!s) {
      double j1x = 0, j1y = 0, j2x = 0, j2y = 0;
      for (int q = 0; q < 9; ++q) {
        const double a = f[q * P + i], b = f[(9 + q) * P + i];
        r1 += a; r2 += b;
        j1x += a * ex[q]; j1y += a * ey[q];
        j2x += b * ex[q]; j2y += b * ey[q];
      }
      double c1x = 0, c1y = 0, c2x = 0, c2y = 0, sx = 0, sy = 0;
      for (int q = 1; q < 9; ++q) {
        int xn = x + ex[q], yn = y + ey[q];
        xn = xn < 0 ? xn + nx : (xn >= nx ? xn - nx : xn);
        yn = yn < 0 ? yn + ny : (yn >= ny ? yn - ny : yn);
        const long long k = (long long)yn * nx + xn;
        if (mask[k] & sb) { sx += w[q] * ex[q]; sy += w[q] * ey[q]; continue; }
        double a, b;
        node_rho(f, P, k, &a, &b);
        c1x += w[q] * a * ex[q]; c1y += w[q] * a * ey[q];
        c2x += w[q] * b * ex[q]; c2y += w[q] * b * ey[q];
      }
      const double F1x = -G * r1 * c2x - Gads1 * r1 * sx + r1 * ax;
      const double F1y = -G * r1 * c2y - Gads1 * r1 * sy + r1 * ay;
      const double F2x = -G * r2 * c1x - Gads2 * r2 * sx + r2 * ax;
      const double F2y = -G * r2 * c1y - Gads2 * r2 * sy + r2 * ay;
      ux = (j1x + j2x + 0.5 * (F1x + F2x)) / (r1 + r2);
      uy = (j1y + j2y + 0.5 * (F1y + F2y)) / (r1 + r2);
      if (solute)
        for (int q = 0; q < 5; ++q) c += g[q * P + i];
    }
    out[i] = r1;
    out[N + i] = r2;
    out[2 * N + i] = ux;
    out[3 * N + i] = uy;
    out[4 * N + i] = c;
    out[5 * N + i] = react ? m[i] : 0.0;
    out[6 * N + i] = s ? 1.0 : 0.0;
  }
}

// ---- launchers ------------------------------------------------------------
hipError_t launch_step(const StepArgs& a, int tx, int arith64, hipStream_t st) {
  const int T = a.nstrips * a.nsegs;
  const size_t lds = (size_t)4 * tx * (2 * (arith64 ? sizeof(double) : sizeof(float)) + sizeof(float));
  if (arith64) {
    if (a.solute && a.react)
      hipLaunchKernelGGL((k_step<true, true, double>), dim3(T), dim3(tx), lds, st, a);
    else if (a.solute)
      hipLaunchKernelGGL((k_step<true, false, double>), dim3(T), dim3(tx), lds, st, a);
    else
      hipLaunchKernelGGL((k_step<false, false, double>), dim3(T), dim3(tx), lds, st, a);
  } else {
    if (a.solute && a.react)
      hipLaunchKernelGGL((k_step<true, true, float>), dim3(T), dim3(tx), lds, st, a);
    else if (a.solute)
      hipLaunchKernelGGL((k_step<true, false, float>), dim3(T), dim3(tx), lds, st, a);
    else
      hipLaunchKernelGGL((k_step<false, false, float>), dim3(T), dim3(tx), lds, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_step_batch(const StepArgs* insts, const int4* tiles, int ntiles,
                             const long long* stepc, int tx, int solute, int react, int arith64,
                             hipStream_t st) {
  const size_t lds = (size_t)4 * tx * (2 * (arith64 ? sizeof(double) : sizeof(float)) + sizeof(float));
  if (arith64) {
    if (solute && react)
      hipLaunchKernelGGL((k_step_batch<true, true, double>), dim3(ntiles), dim3(tx), lds, st, insts, tiles, stepc);
    else if (solute)
      hipLaunchKernelGGL((k_step_batch<true, false, double>), dim3(ntiles), dim3(tx), lds, st, insts, tiles, stepc);
    else
      hipLaunchKernelGGL((k_step_batch<false, false, double>), dim3(ntiles), dim3(tx), lds, st, insts, tiles, stepc);
  } else {
    if (solute && react)
      hipLaunchKernelGGL((k_step_batch<true, true, float>), dim3(ntiles), dim3(tx), lds, st, insts, tiles, stepc);
    else if (solute)
      hipLaunchKernelGGL((k_step_batch<true, false, float>), dim3(ntiles), dim3(tx), lds, st, insts, tiles, stepc);
    else
      hipLaunchKernelGGL((k_step_batch<false, false, float>), dim3(ntiles), dim3(tx), lds, st, insts, tiles, stepc);
  }
  hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, st, (long long*)stepc);
  return hipGetLastError();
}

hipError_t launch_front_batch(const StepArgs* insts, const int4* capi, const long long* stepc,
                              int n, int slot, int nslots, double* table, hipStream_t st) {
  hipLaunchKernelGGL(k_front_batch, dim3(n), dim3(256), 0, st, insts, capi, stepc, slot, nslots, table);
  return hipGetLastError();
}

int host_xcd_tile(int b, int T) { return xcd_tile(b, T); }

hipError_t launch_init(const double* r1, const double* r2, const double* c, const uint8_t* mask,
                       float* f, float* g, double* m, int32_t* sstep, float* drop, long long N,
                       long long P, int solute, int react, hipStream_t st) {
  const int blocks = (int)((N + 255) / 256 < 8192 ? (N + 255) / 256 : 8192);
  hipLaunchKernelGGL(k_init, dim3(blocks), dim3(256), 0, st, r1, r2, c, mask, f, g, m, sstep,
                     drop, N, P, solute, react);
  return hipGetLastError();
}

hipError_t launch_observe(const float* f, const float* g, const uint8_t* mask, const double* m,
                          const float* drop, const int32_t* sstep, long long N, long long P,
                          int nx, unsigned bit_prev, int solute, int react, int nblocks,
                          double* partial, double* out, int x_in, int x_out, int y0, int W,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_obs_partial, dim3(nblocks), dim3(256), 0, st, f, g, mask, m, drop, N, P,
                     bit_prev, solute, react, partial);
  hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(64), 0, st, partial, nblocks, out);
  if (W > 0)
    hipLaunchKernelGGL(k_obs_capillary, dim3(1), dim3(256), 0, st, f, mask, sstep, nx, P,
                       bit_prev, x_in, x_out, y0, W, react, out + OBS_SLOTS);
  return hipGetLastError();
}

hipError_t launch_fields(const float* f, const float* g, const uint8_t* mask, const double* m,
                         int nx, int ny, long long P, unsigned bit_prev, int solute, int react,
                         float G, float Gads1, float Gads2, float ax, float ay, double* out,
                         hipStream_t st) {
  const long long N = (long long)nx * ny;
  const int blocks = (int)((N + 255) / 256 < 8192 ? (N + 255) / 256 : 8192);
  hipLaunchKernelGGL(k_fields, dim3(blocks), dim3(256), 0, st, f, g, mask, m, nx, ny, P, bit_prev,
                     solute, react, G, Gads1, Gads2, ax, ay, out);
  return hipGetLastError();
}

}  // namespace lbmdev
