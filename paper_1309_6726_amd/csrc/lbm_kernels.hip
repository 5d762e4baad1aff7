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
//                    (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1);
//                    in the moment scheme planes 0..5 hold instead the
//                    post-collision moments rho1, v1x, v1y, rho2, v2x, v2y
//   g  float[5][P]   solute populations (first five links)
//   mask uint8[P]    bit0 solid; bits 1..3 growth pending (see pending_bit)
//   m  double[P]     precipitated mass (touched only at wall-adjacent nodes)
//   sstep int32[P]   state index at which the node turned solid (-1 fluid)
//   drop float[3][P] populations a node carried when it turned solid
// f and g are double-buffered (A/B); a step reads one buffer and writes the
// other.
//
// Population step (any tau), one kernel per time step.  A workgroup of TX
// threads owns TX-2 consecutive columns (one column per thread, plus one halo
// column on each side) and SY consecutive rows, and marches up its rows.  For
// every row it loads the node populations (coalesced along x), forms the
// densities, puts rho1, rho2 and the solid flag of the row into a 4-row LDS
// ring, and then collides the row below with the cohesion/adhesion stencil
// read from LDS, applies the reaction, and pushes the post-collision
// populations to the neighbours (or back into the node's own opposite link at
// a solid neighbour).
//
// Moment step (tau = 1).  With full relaxation the post-collision populations
// of a component are its equilibria at (rho_s, v_s), so a node stores those
// three numbers per component (24 bytes instead of 72) and the next step
// rebuilds the populations that arrive at x by evaluating the equilibrium of
// each upstream neighbour (halfway bounce-back: the node's own moments with
// the velocity reversed when the upstream node is solid).  A workgroup then
// owns TX-4 columns: the gathered densities feed the force stencil, which
// reaches two columns and two rows out.  Per-node arithmetic is independent
// of the launch shape in both steps, so every tile shape gives bit-identical
// results.
//
// Growth timing.  In the step n -> n+1 a node whose precipitate exceeds the
// threshold still streams as fluid (the step uses the solid set of state n);
// it is marked with pending_bit(n).  Step n+1 reads it as solid and books the
// populations it carried into `drop`; step n+2 folds the mark into bit0.  A
// node being marked in the current step is read as fluid by its neighbours,
// so concurrent workgroups never disagree on the solid sets of states n-1
// and n, which the moment step needs both of.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lbm_dev.h"

// Multiply-adds are fused only where one source expression states them: the
// compiler may peel or duplicate loop iterations, and fusion chosen per copy
// would make the rounding of a node depend on which copy computes it (and so
// on the launch shape).
#pragma clang fp contract(on)

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

typedef unsigned v2u __attribute__((ext_vector_type(2)));

// Cache-policy operand of the buffer builtins: the non-temporal bit (nt).
#define CPOL_NT 2

// Raw buffer descriptor (stride 0, no format conversion) over bytes [0, extent)
// of base.  Word 3 is the value the gfx9-family buffer instructions take for
// untyped dword access.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, unsigned extent) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)extent, 0x00020000);
}

// Workgroup-wide LDS barrier that leaves outstanding global memory operations
// in flight (only LDS traffic is ordered); a single-wave workgroup needs no
// s_barrier at all.
__device__ __forceinline__ void lds_barrier(int TX) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  if (TX > 64) __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Shan-Chen interaction forces plus the body force at a fluid node (section
// "LB models": cohesion between the two components and adhesion to the solid,
// each a weight-normalised sum over the eight neighbours).  n1, n2: the
// neighbours' densities (zero at solid nodes); sf: their solid flags (0/1);
// index = link, 1..8 = E, N, W, S, NE, NW, SW, SE (index 0 unused).
template <typename R>
__device__ __forceinline__ void sc_forces(const StepArgs& a, const R* n1, const R* n2,
                                          const float* sf, R rho1, R rho2, R& F1x, R& F1y,
                                          R& F2x, R& F2y) {
  const R WA = R(1) / R(9), WD = R(1) / R(36);
  const R c2x = WA * (n2[1] - n2[3]) + WD * ((n2[5] - n2[6]) + (n2[8] - n2[7]));
  const R c2y = WA * (n2[2] - n2[4]) + WD * ((n2[5] + n2[6]) - (n2[8] + n2[7]));
  const R c1x = WA * (n1[1] - n1[3]) + WD * ((n1[5] - n1[6]) + (n1[8] - n1[7]));
  const R c1y = WA * (n1[2] - n1[4]) + WD * ((n1[5] + n1[6]) - (n1[8] + n1[7]));
  const R csx = WA * R(sf[1] - sf[3]) + WD * R((sf[5] - sf[6]) + (sf[8] - sf[7]));
  const R csy = WA * R(sf[2] - sf[4]) + WD * R((sf[5] + sf[6]) - (sf[8] + sf[7]));
  const R G = (R)a.G, Ga1 = (R)a.Gads1, Ga2 = (R)a.Gads2, ax = (R)a.ax, ay = (R)a.ay;
  F1x = -G * rho1 * c2x - Ga1 * rho1 * csx + rho1 * ax;
  F1y = -G * rho1 * c2y - Ga1 * rho1 * csy + rho1 * ay;
  F2x = -G * rho2 * c1x - Ga2 * rho2 * csx + rho2 * ax;
  F2y = -G * rho2 * c1y - Ga2 * rho2 * csy + rho2 * ay;
}

// 1/x from the hardware estimate refined by two Newton steps (a few ulp; the
// correctly rounded division sequence costs twice the instructions).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ float recip(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
}

// Equilibrium velocities of the two components (common velocity shifted by
// tau F_s / rho_s) and the physical velocity (j + F/2) / rho that advects the
// solute.
template <typename R>
__device__ __forceinline__ void sc_velocities(R tau, R rho1, R rho2, R j1x, R j1y, R j2x, R j2y,
                                              R F1x, R F1y, R F2x, R F2y, R& v1x, R& v1y,
                                              R& v2x, R& v2y, R& ux, R& uy) {
  const R rt = rho1 + rho2;
  const R irt = recip(rt);
  const R upx = (j1x + j2x) * irt, upy = (j1y + j2y) * irt;
  v1x = upx; v1y = upy; v2x = upx; v2y = upy;
  if (rho1 > R(0)) { const R s = tau * recip(rho1); v1x += s * F1x; v1y += s * F1y; }
  if (rho2 > R(0)) { const R s = tau * recip(rho2); v2x += s * F2x; v2y += s * F2y; }
  ux = (j1x + j2x + R(0.5) * (F1x + F2x)) * irt;
  uy = (j1y + j2y + R(0.5) * (F1y + F2y)) * irt;
}

// Solute collision (BGK on D2Q5, or on D2Q4 with weights 1/4 and no rest
// link, advected by u), first-order precipitation at a node with ns > 0 solid
// axis neighbours (rate k_r ns phi, phi the wetting fraction; with a
// saturation concentration c_eq > 0 only the excess C - c_eq precipitates),
// the held source (post-collision solute of a node with x < hold_x set to the
// equilibrium at c_hold), threshold test, and push of the solute populations
// (bounce-back at solid axis neighbours).  sf: solid flags of the axis
// neighbours 1..4.
// What solute_step leaves for memory every step: the five pushed populations
// with their element offsets in gout, and the new precipitate of the node
// (wm: the node is next to a wall, so m changed).
struct SoluteOut {
  float g[5];
  unsigned off[5];
  double m;
  bool wm;
};

template <bool REACT>
__device__ __forceinline__ void store_solute(const StepArgs& a, const SoluteOut& o, unsigned idx) {
  float* __restrict__ go = a.gout;
#pragma unroll
  for (int q = 0; q < 5; ++q) go[o.off[q]] = o.g[q];
  if (REACT && o.wm) a.m[idx] = o.m;
}

template <bool REACT, bool VAR, typename R>
__device__ __forceinline__ void solute_step(const StepArgs& a, const float* g, R ux, R uy,
                                            R rho1, R rho2, const float* sf, double m_cur,
                                            unsigned P, unsigned idx, unsigned iE, unsigned iN,
                                            unsigned iW, unsigned iS, int xc, int y, bool& ev,
                                            int& evx, int& evy, SoluteOut& so) {
  so.wm = false;
  so.m = 0.0;
  // VAR = false: the plain model (D2Q5, c_eq = 0, no held source)
  const bool q4 = VAR && a.q4 != 0;
  const R WQ = q4 ? R(0.25) : R(1) / R(6), CQ = q4 ? R(2) : R(3);
  const R C = (((R)g[0] + (R)g[1]) + ((R)g[2] + (R)g[3])) + (R)g[4];
  const R og = (R)a.omega_g;
  R gs[5];
  gs[1] = (R)g[1] + og * (WQ * C * (R(1) + CQ * ux) - (R)g[1]);
  gs[2] = (R)g[2] + og * (WQ * C * (R(1) + CQ * uy) - (R)g[2]);
  gs[3] = (R)g[3] + og * (WQ * C * (R(1) - CQ * ux) - (R)g[3]);
  gs[4] = (R)g[4] + og * (WQ * C * (R(1) - CQ * uy) - (R)g[4]);
  gs[0] = q4 ? R(0) : C - ((gs[1] + gs[2]) + (gs[3] + gs[4]));
  if (REACT) {
    const int ns = (int)sf[1] + (int)sf[2] + (int)sf[3] + (int)sf[4];
    if (ns > 0) {
      const double phi = (double)rho1 / ((double)rho1 + (double)rho2);
      const double rr = a.k_r * (double)ns * phi;
      double dm, keep;
      if (VAR && a.c_eq > 0.0) {
        const double excess = (double)C > a.c_eq ? (double)C - a.c_eq : 0.0;
        dm = rr * excess;
        keep = dm > 0.0 ? 1.0 - dm / (double)C : 1.0;
      } else {
        dm = rr * (double)C;
        keep = 1.0 - rr;
      }
      const double mm = m_cur + dm;
      so.m = mm;
      so.wm = true;
#pragma unroll
      for (int q = 0; q < 5; ++q) gs[q] *= (R)keep;
      if (mm > a.threshold) {
        a.mask[idx] = (uint8_t)a.bit_cur;
        a.sstep[idx] = (int32_t)(a.step + 1);
        ev = true;
        evx = xc;
        evy = y;
      }
    }
  }
  if (VAR && xc < a.hold_x) {
    const R Ch = (R)a.c_hold;
    gs[1] = WQ * Ch * (R(1) + CQ * ux);
    gs[2] = WQ * Ch * (R(1) + CQ * uy);
    gs[3] = WQ * Ch * (R(1) - CQ * ux);
    gs[4] = WQ * Ch * (R(1) - CQ * uy);
    gs[0] = q4 ? R(0) : (R(1) - R(4) * WQ) * Ch;
  }
  // push; at a solid axis neighbour the value bounces into the opposite link
#pragma unroll
  for (int q = 0; q < 5; ++q) so.g[q] = (float)gs[q];
  so.off[0] = idx;
  so.off[1] = sf[1] != 0.0f ? 3 * P + idx : 1 * P + iE;
  so.off[2] = sf[2] != 0.0f ? 4 * P + idx : 2 * P + iN;
  so.off[3] = sf[3] != 0.0f ? 1 * P + idx : 3 * P + iW;
  so.off[4] = sf[4] != 0.0f ? 2 * P + idx : 4 * P + iS;
}

// One lane per wavefront reserves event-log slots for every lane that marked
// a node in this row, with a single atomic.
__device__ __forceinline__ void log_events(const StepArgs& a, bool ev, int evx, int evy) {
  const int lane = __lane_id();
  const unsigned long long bal = __ballot(ev);
  if (bal) {
    const int leader = __ffsll((unsigned long long)bal) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(a.ev_count, (unsigned long long)__popcll(bal));
    base = __shfl(base, leader);
    if (ev) {
      // events of lower lanes in this row come first
      const unsigned below = __builtin_amdgcn_mbcnt_hi(
          (unsigned)(bal >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
      const unsigned long long e = base + below;
      if ((long long)e < a.ev_cap) {
        a.ev[e].x = evx;
        a.ev[e].y = evy;
        a.ev[e].step = a.step + 1;
      }
    }
  }
}

// Incoming populations of a node in state n rebuilt from stored moments
// (moment scheme, tau = 1).  r, vx, vy: the node's own post-collision moments
// (index 0) and those of the upstream node x - e_i of link i (index i); up[i]:
// that upstream node was fluid in state n-1.  A link whose upstream node was
// solid carries the node's own equilibrium on the opposite link (halfway
// bounce-back), i.e. the same expression with the node's velocity reversed.
// f[0] is the node's own rest equilibrium.
template <typename R>
__device__ __forceinline__ void gather_links(const float* r, const float* vx, const float* vy,
                                             const bool* up, R* f) {
  const R WA = R(1) / R(9), WD = R(1) / R(36), W0 = R(4) / R(9);
  const R r0 = (R)r[0], x0 = (R)vx[0], y0 = (R)vy[0];
  const R uu0 = x0 * x0 + y0 * y0;
  f[0] = feq<R>(W0, r0, R(0), uu0);
#define GL(i, w, EU)                                                  \
  do {                                                                \
    const R rr = up[i] ? (R)r[i] : r0;                                \
    const R ux = up[i] ? (R)vx[i] : -x0;                              \
    const R uy = up[i] ? (R)vy[i] : -y0;                              \
    const R uu = up[i] ? ux * ux + uy * uy : uu0;                     \
    f[i] = feq<R>(w, rr, EU, uu);                                     \
  } while (0)
  GL(1, WA, ux);
  GL(2, WA, uy);
  GL(3, WA, -ux);
  GL(4, WA, -uy);
  GL(5, WD, ux + uy);
  GL(6, WD, -ux + uy);
  GL(7, WD, -ux - uy);
  GL(8, WD, ux - uy);
#undef GL
}

// Density and momentum of nine populations (the summation order of the
// population step).
template <typename R>
__device__ __forceinline__ void moments9(const R* f, R& rho, R& jx, R& jy) {
  rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
}

// R is the arithmetic type (float or double); populations are stored as FP32.
//
// Population step.  Per workgroup, iteration k handles row r = ys - 1 + k: its
// populations, precipitate (owned rows) and the mask byte of row k+1 are
// requested together (the mask of row k arrived one iteration earlier), so
// each iteration waits on one memory round trip.  The densities of row k go
// to the LDS ring; after an LDS-only barrier row k-1 is collided and pushed.
// Offsets are 32-bit (the host guarantees 23 planes fit below 2^31).  The
// register budget is held to three waves per SIMD: a row iteration costs one
// memory round trip plus ~1 us of VALU work per wave, so resident waves are
// what hides the memory latency.  OUTM (tau = 1 only): store the moments
// (rho_s, v_s) of the collided node instead of pushing populations.
template <bool SOLUTE, bool REACT, bool VAR, typename R, bool OUTM, bool NT>
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
  const unsigned SPREV = 1u | a.bit_p2;    // solid in state n-1
  const unsigned SCUR = SPREV | a.bit_p1;  // solid in state n
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
      if (!(b_nxt & SPREV)) {
        // read once per step (NT: with the non-temporal hint)
#pragma unroll
        for (int q = 0; q < 18; ++q)
          fn[q] = NT ? __builtin_nontemporal_load(&fin[q * P + idn]) : fin[q * P + idn];
        if (SOLUTE && owner && owned_row) {
#pragma unroll
          for (int q = 0; q < 5; ++q)
            gn[q] = NT ? __builtin_nontemporal_load(&gin[q * P + idn]) : gin[q * P + idn];
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
    if (active && !(b_nxt & SCUR)) {
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
      if (s_s[sm + t] != 0.0f) {
        if (REACT) {
          if (b_cur & a.bit_p1) {
            // turned solid at the end of the previous step: book its populations
            a.drop[idx] = (float)sum9<R>(f);
            a.drop[P + idx] = (float)sum9<R>(f + 9);
            a.drop[2 * P + idx] =
                SOLUTE ? (float)((((R)g[0] + (R)g[1]) + ((R)g[2] + (R)g[3])) + (R)g[4]) : 0.0f;
          } else if (b_cur & a.bit_p2) {
            a.mask[idx] = 1;  // booked one step ago: fold the mark into bit0
          }
        }
      } else {
        const R rho1 = s_r1[sm + t], rho2 = s_r2[sm + t];
        // neighbours in link order 1..8 = E, N, W, S, NE, NW, SW, SE
        const int no[9] = {sm + t, sm + t + 1, sa + t, sm + t - 1, sb + t,
                           sa + t + 1, sa + t - 1, sb + t - 1, sb + t + 1};
        R n1[9], n2[9];
        float sf[9];
#pragma unroll
        for (int i = 1; i < 9; ++i) {
          n1[i] = s_r1[no[i]];
          n2[i] = s_r2[no[i]];
          sf[i] = s_s[no[i]];
        }
        R F1x, F1y, F2x, F2y;
        sc_forces<R>(a, n1, n2, sf, rho1, rho2, F1x, F1y, F2x, F2y);
        const R j1x = ((R)f[1] - (R)f[3]) + ((R)f[5] - (R)f[6]) + ((R)f[8] - (R)f[7]);
        const R j1y = ((R)f[2] - (R)f[4]) + ((R)f[5] + (R)f[6]) - ((R)f[7] + (R)f[8]);
        const R j2x = ((R)f[10] - (R)f[12]) + ((R)f[14] - (R)f[15]) + ((R)f[17] - (R)f[16]);
        const R j2y = ((R)f[11] - (R)f[13]) + ((R)f[14] + (R)f[15]) - ((R)f[16] + (R)f[17]);
        R v1x, v1y, v2x, v2y, ux, uy;
        sc_velocities<R>((R)a.tau, rho1, rho2, j1x, j1y, j2x, j2y, F1x, F1y, F2x, F2y, v1x, v1y,
                         v2x, v2y, ux, uy);

        // target offsets of the four axis neighbours (and the diagonals)
        const unsigned iE = (unsigned)y * nx + xr, iW = (unsigned)y * nx + xl;
        const unsigned iN = (unsigned)yu * nx + xc, iS = (unsigned)yd * nx + xc;
        float* __restrict__ fo = a.fout;
        if (OUTM) {
          fo[idx] = (float)rho1;
          fo[P + idx] = (float)v1x;
          fo[2 * P + idx] = (float)v1y;
          fo[3 * P + idx] = (float)rho2;
          fo[4 * P + idx] = (float)v2x;
          fo[5 * P + idx] = (float)v2y;
        } else {
          const unsigned iNE = (unsigned)yu * nx + xr, iNW = (unsigned)yu * nx + xl;
          const unsigned iSW = (unsigned)yd * nx + xl, iSE = (unsigned)yd * nx + xr;
          const R om = (R)a.omega;
          // collide one component and push each moving population as soon as
          // it is formed (halfway bounce-back into the node's own opposite
          // link at a solid neighbour); the rest population closes the mass
          // balance exactly (the moving-link weights are not exact binary
          // fractions)
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
            const R WA = R(1) / R(9), WD = R(1) / R(36);
            CP(1, 3, WA, vx, sf[1], iE);
            CP(2, 4, WA, vy, sf[2], iN);
            CP(3, 1, WA, -vx, sf[3], iW);
            CP(4, 2, WA, -vy, sf[4], iS);
            CP(5, 7, WD, vx + vy, sf[5], iNE);
            CP(6, 8, WD, -vx + vy, sf[6], iNW);
            CP(7, 5, WD, -vx - vy, sf[7], iSW);
            CP(8, 6, WD, vx - vy, sf[8], iSE);
#undef CP
            fo[base * P + idx] = (float)(rho - sum);
          };
          collide_push(f, 0u, rho1, v1x, v1y);
          collide_push(f + 9, 9u, rho2, v2x, v2y);
        }
        if (SOLUTE) {
          SoluteOut so;
          solute_step<REACT, VAR, R>(a, g, ux, uy, rho1, rho2, sf, m_cur, P, idx, iE, iN, iW, iS, xc, y,
                                ev, evx, evy, so);
          store_solute<REACT>(a, so, idx);
        }
      }
    }
    if (REACT) log_events(a, ev, evx, evy);
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

// Cross-lane moves within one wavefront (DPP wave shifts): from_left(v) in
// lane t is v of lane t-1, from_right(v) is v of lane t+1; the end lane
// without a source reads 0.  Called with every lane active.
__device__ __forceinline__ int from_left_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x138, 0xF, 0xF, true);  // wave_shr:1
}
__device__ __forceinline__ int from_right_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true);  // wave_shl:1
}
__device__ __forceinline__ float from_left(float v) {
  return __int_as_float(from_left_i(__float_as_int(v)));
}
__device__ __forceinline__ float from_right(float v) {
  return __int_as_float(from_right_i(__float_as_int(v)));
}
__device__ __forceinline__ double from_left(double v) {
  return __hiloint2double(from_left_i(__double2hiint(v)), from_left_i(__double2loint(v)));
}
__device__ __forceinline__ double from_right(double v) {
  return __hiloint2double(from_right_i(__double2hiint(v)), from_right_i(__double2loint(v)));
}

// Mask bytes of a lane and of its two neighbours packed as own | left << 8 |
// right << 16.
__device__ __forceinline__ unsigned pack_row_mask(unsigned m) {
  return m | ((unsigned)from_left_i((int)m) << 8) | ((unsigned)from_right_i((int)m) << 16);
}

// Equilibrium of a link from the stored moments of its node: wr = w rho,
// c = 1 - 3/2 |v|^2, eu = e . v  ->  w rho (1 + 3 eu + 9/2 eu^2 - 3/2 |v|^2).
template <typename R>
__device__ __forceinline__ R feq_m(R wr, R c, R eu) {
  return wr * (c + eu * (R(3) + R(4.5) * eu));
}

// Moment step (tau = 1), one wavefront per workgroup: lane t holds column
// x0 - 2 + t and the workgroup owns the 60 columns of lanes 2..61.  At
// iteration k the lanes take the stored moments of row k (ys - 2 + k) and
// evaluate the eight outgoing equilibria of their node (zero at nodes solid
// in state n-1).  Each value is added to the accumulator (rho_s, j_s) of the
// node it streams to: same lane for vertical links, the neighbouring lane
// (DPP wave shift) for the others; a value streaming into a solid node is
// bounced back into the sender's own accumulator on the opposite link.  Row
// k-1 is then complete; its densities (zero at solids in state n) join a
// three-row window held in registers, from which row k-2 is collided: forces,
// new moments, solute, reaction and growth.
//
// Memory: the moments of row k+1 and the solute populations and precipitate
// of row k-1 are copied from HBM straight into an LDS double buffer (no
// registers held while in flight) before row k is computed, and the mask two
// rows ahead into a register, so one iteration's arithmetic covers the next
// iteration's memory latency.  The summation order of every node is fixed,
// so results do not depend on the tile shape.
//
// NT: the copies of data that only this wavefront reads in the step carry
// the non-temporal cache hint: the moments of the tile's own rows and the
// solute populations.  The two halo rows at each end (rows of the
// neighbouring segments, which read them too) and the precipitate (read here
// and rewritten by the same wavefront an iteration later) keep the normal
// policy.  Whether the hint pays depends on how the step's footprint meets
// the caches, so the single-lattice step takes it as an autotuned choice.
template <bool SOLUTE, bool REACT, bool VAR, typename R, bool NT>
__device__ __forceinline__ void mom_wave(const StepArgs& a, int strip, int seg) {
  // prefetch slots per buffer: 0..5 moments, 6..10 solute, 11..12 precipitate
  __shared__ float pf[2][13][64];
  const int t = threadIdx.x;
  const int nx = a.nx, ny = a.ny;
  const unsigned P = (unsigned)a.P;
  const int x0 = strip * a.tx_owned;
  const int nown = min(a.tx_owned, nx - x0);
  const bool active = t <= nown + 3;
  const bool owner = t >= 2 && t <= nown + 1;
  int xc = x0 - 2 + t;
  if (xc < 0) xc += nx;
  if (xc >= nx) xc -= nx;
  const int xl = xc == 0 ? nx - 1 : xc - 1;
  const int xr = xc == nx - 1 ? 0 : xc + 1;
  const int ys = seg * a.sy;
  const int ye = min(ys + a.sy, ny);
  const int nrows = ye - ys + 4;
  const unsigned SPREV = 1u | a.bit_p2;    // solid in state n-1
  const unsigned SCUR = SPREV | a.bit_p1;  // solid in state n
  const R WA = R(1) / R(9), WD = R(1) / R(36), WR = R(4) / R(9);
  // Buffer descriptors: one per array, plane q at scalar offset q * P * 4
  // bytes, so an access costs one 32-bit lane offset per row instead of a
  // 64-bit address per plane.  The extent covers every plane the kernel
  // touches: the hardware checks lane offset plus scalar offset against it,
  // and a lane beyond it reads 0 and drops its store.
  const unsigned PB = P * 4u;
  const auto rMin = make_rsrc(a.fin, 6u * PB);
  const auto rMout = make_rsrc(a.fout, 6u * PB);
  const auto rGin = make_rsrc(a.gin, SOLUTE ? 5u * PB : 0u);
  const auto rGout = make_rsrc(a.gout, SOLUTE ? 5u * PB : 0u);
  const auto rMask = make_rsrc(a.mask, P);
  const auto rPrec = make_rsrc(a.m, REACT ? 2u * PB : 0u);

  auto row_y = [&](int k) {
    int yr = ys - 2 + k;
    if (yr < 0) yr += ny;
    if (yr >= ny) yr -= ny;
    return yr;
  };
  auto sol = [](unsigned pk, int sh, unsigned bits) { return ((pk >> sh) & bits) != 0u; };
  auto mask_at = [&](int k) -> unsigned {
    return (active && k < nrows)
               ? (unsigned)__builtin_amdgcn_raw_buffer_load_b8(
                     rMask, (int)((unsigned)row_y(k) * (unsigned)nx + (unsigned)xc), 0, 0)
               : 1u;
  };
  using lds_ptr = __attribute__((address_space(3))) void*;
  // One dword per lane at byte offset voff + soff into prefetch slot
  // (buf, slot), with the normal cache policy (to_lds) or the non-temporal
  // one (to_lds_nt).
  auto to_lds = [&](__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, int buf, int slot) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr)&pf[buf][slot][0], 4, (int)voff, (int)soff,
                                             0, 0);
  };
  auto to_lds_nt = [&](__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, int buf, int slot) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr)&pf[buf][slot][0], 4, (int)voff, (int)soff,
                                             0, CPOL_NT);
  };
  // Copy row k's moments (fluid nodes of state n-1) and row k-2's solute
  // and precipitate (fluid owned nodes, precipitate only next to a wall of
  // state n) into buffer buf.  Every lane issues every load; a lane with
  // nothing to copy gives a lane offset past every extent (such an offset
  // stays out of range whatever scalar offset is added), so the hardware
  // writes 0 to its slot without touching memory, and the reader needs no
  // select.
  constexpr unsigned NONE = 0xFFFFFFF0u;
  auto prefetch = [&](int buf, int k, unsigned own_k, unsigned pkm3, unsigned pkm2,
                      unsigned pkm1) {
    if (k >= nrows) return;
    const bool got_m = active && !(own_k & SPREV);
    const unsigned vm = got_m ? 4u * ((unsigned)row_y(k) * (unsigned)nx + (unsigned)xc) : NONE;
    if (NT && k >= 2 && k < nrows - 2) {
#pragma unroll
      for (int q = 0; q < 6; ++q) to_lds_nt(rMin, vm, (unsigned)q * PB, buf, q);
    } else {
#pragma unroll
      for (int q = 0; q < 6; ++q) to_lds(rMin, vm, (unsigned)q * PB, buf, q);
    }
    if (SOLUTE && k >= 4) {
      const unsigned ownC = pkm2 & 0xFFu;
      const unsigned i = (unsigned)(ys + k - 4) * (unsigned)nx + (unsigned)xc;
      const bool got_g = owner && !(ownC & SPREV);
      const unsigned vg = got_g ? 4u * i : NONE;
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        if (NT) to_lds_nt(rGin, vg, (unsigned)q * PB, buf, 6 + q);
        else to_lds(rGin, vg, (unsigned)q * PB, buf, 6 + q);
      }
      if (REACT) {
        const bool got_p =
            owner && !(ownC & SCUR) &&
            (sol(pkm2, 16, SCUR) || sol(pkm1, 0, SCUR) || sol(pkm2, 8, SCUR) || sol(pkm3, 0, SCUR));
        const unsigned vp = got_p ? 8u * i : NONE;
        to_lds(rPrec, vp, 0u, buf, 11);
        to_lds(rPrec, vp, 4u, buf, 12);
      }
    }
  };

  // packed masks of rows k-3 .. k+1 (rows outside the tile read as solid)
  const unsigned SOLID3 = 0x010101u;
  unsigned pk_m3 = SOLID3, pk_m2 = SOLID3, pk_m1 = SOLID3;
  unsigned pk_0 = pack_row_mask(mask_at(0));
  unsigned m_ahead = mask_at(1);  // raw mask of row k+1 (then k+2)
  prefetch(0, 0, pk_0 & 0xFFu, pk_m3, pk_m2, pk_m1);

  R acc0[6], acc1[6];  // (rho1, j1x, j1y, rho2, j2x, j2y) of rows k and k-1
#pragma unroll
  for (int q = 0; q < 6; ++q) { acc0[q] = R(0); acc1[q] = R(0); }
  R rC[6];  // complete (rho, j) of row k-2
#pragma unroll
  for (int q = 0; q < 6; ++q) rC[q] = R(0);
  // density window (zero at solids of state n): centre, from left, from right
  R W1[6], W2[6];  // rows k-2, k-3: (c1, c2, l1, l2, r1, r2)
#pragma unroll
  for (int q = 0; q < 6; ++q) { W1[q] = R(0); W2[q] = R(0); }

  for (int k = 0; k < nrows; ++k) {
    const int buf = k & 1;
    // everything requested during the previous iteration has arrived
    __builtin_amdgcn_s_waitcnt(VMCNT0);
    const unsigned pk_p1 = pack_row_mask(m_ahead);
    // buffer buf holds row k's moments and row k-2's solute and precipitate
    // (0 where nothing was copied)
    auto take = [&](int slot) { return pf[buf][slot][t]; };
    const unsigned own0 = pk_0 & 0xFFu;
    // requests for the next iteration: row k+1's moments, row k-1's solute,
    // the mask of row k+2
    prefetch(buf ^ 1, k + 1, pk_p1 & 0xFFu, pk_m2, pk_m1, pk_0);
    m_ahead = mask_at(k + 2);

    const bool crow = k >= 4 && owner;
    const int yC = ys + k - 4;
    const unsigned idxC = (unsigned)(crow ? yC : 0) * (unsigned)nx + (unsigned)xc;
    const unsigned ownC = pk_m2 & 0xFFu;

    // links of this node whose target is solid in state n-1 (bit i = link i)
    const unsigned bb =
        (sol(pk_0, 16, SPREV) ? 0x02u : 0u) | (sol(pk_p1, 0, SPREV) ? 0x04u : 0u) |
        (sol(pk_0, 8, SPREV) ? 0x08u : 0u) | (sol(pk_m1, 0, SPREV) ? 0x10u : 0u) |
        (sol(pk_p1, 16, SPREV) ? 0x20u : 0u) | (sol(pk_p1, 8, SPREV) ? 0x40u : 0u) |
        (sol(pk_m1, 8, SPREV) ? 0x80u : 0u) | (sol(pk_m1, 16, SPREV) ? 0x100u : 0u);
    const bool bounce = bb != 0u && !(own0 & SPREV);

    // ---- sources of row k: outgoing equilibria, streamed -----------------
    R accN[6];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      // with u3 = 3 v: w rho (1 + 3 e.v + 9/2 (e.v)^2 - 3/2 v^2)
      //              = w rho (cc + e3 (1 + e3 / 2)), e3 = e . u3, cc = 1 - u3^2 / 6
      const R rho = (R)take(3 * c);
      const R ux = R(3) * (R)take(3 * c + 1), uy = R(3) * (R)take(3 * c + 2);
      const R cc = fmar(ux * ux + uy * uy, R(-1) / R(6), R(1));
      const R ra = WA * rho, rd = WD * rho;
      auto out = [&](R r, R e3) { return r * fmar(e3, fmar(e3, R(0.5), R(1)), cc); };
      const R o0 = WR * rho * cc;
      const R o1 = out(ra, ux), o2 = out(ra, uy), o3 = out(ra, -ux), o4 = out(ra, -uy);
      const R o5 = out(rd, ux + uy), o6 = out(rd, uy - ux), o7 = out(rd, -ux - uy),
              o8 = out(rd, ux - uy);
      // up links (2, 5, 6) start the accumulator of row k+1
      const R a5 = from_left(o5), a6 = from_right(o6);
      const R up = (o2 + a5) + a6;
      accN[3 * c] = up;
      accN[3 * c + 1] = a5 - a6;
      accN[3 * c + 2] = up;
      // rest and horizontal links (1, 3) into row k
      const R a1 = from_left(o1), a3 = from_right(o3);
      acc0[3 * c] += (o0 + a1) + a3;
      acc0[3 * c + 1] += a1 - a3;
      // down links (4, 7, 8) complete row k-1
      const R a7 = from_right(o7), a8 = from_left(o8);
      const R dn = (o4 + a7) + a8;
      acc1[3 * c] += dn;
      acc1[3 * c + 1] += a8 - a7;
      acc1[3 * c + 2] -= dn;
      // values streaming into a node solid in state n-1 bounce back into the
      // sender's opposite link: rho += o_i, j -= e_i o_i
      if (bounce) {
        const R s1 = (R)((bb >> 1) & 1u), s2 = (R)((bb >> 2) & 1u), s3 = (R)((bb >> 3) & 1u),
                s4 = (R)((bb >> 4) & 1u), s5 = (R)((bb >> 5) & 1u), s6 = (R)((bb >> 6) & 1u),
                s7 = (R)((bb >> 7) & 1u), s8 = (R)((bb >> 8) & 1u);
        R br = s1 * o1, bx = s3 * o3, by = s4 * o4;
        br = fmar(s2, o2, br); br = fmar(s3, o3, br);
        br = fmar(s4, o4, br); br = fmar(s5, o5, br);
        br = fmar(s6, o6, br); br = fmar(s7, o7, br);
        br = fmar(s8, o8, br);
        bx = fmar(-s1, o1, bx); bx = fmar(-s5, o5, bx);
        bx = fmar(s6, o6, bx); bx = fmar(s7, o7, bx);
        bx = fmar(-s8, o8, bx);
        by = fmar(-s2, o2, by); by = fmar(-s5, o5, by);
        by = fmar(-s6, o6, by); by = fmar(s7, o7, by);
        by = fmar(s8, o8, by);
        acc0[3 * c] += br;
        acc0[3 * c + 1] += bx;
        acc0[3 * c + 2] += by;
      }
    }

    // ---- row k-1 complete: density window --------------------------------
    R W0[6];
    {
      const bool s1 = sol(pk_m1, 0, SCUR);
      const R d1 = s1 ? R(0) : acc1[0], d2 = s1 ? R(0) : acc1[3];
      W0[0] = d1; W0[1] = d2;
      W0[2] = from_left(d1); W0[3] = from_left(d2);
      W0[4] = from_right(d1); W0[5] = from_right(d2);
    }

    // ---- collide row k-2 ---------------------------------------------------
    bool ev = false;
    int evx = 0, evy = 0;
    if (crow) {
      const int y = yC;
      const unsigned idx = idxC;
      float gv[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) gv[q] = take(6 + q);
      // outgoing moments; zero at a node solid in state n, which no reader of
      // the next state takes as fluid.  Every owned lane stores, so each plane
      // is written as whole rows rather than lines with holes at solids.
      float mo[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
      if (ownC & SCUR) {
        if (REACT) {
          if (ownC & a.bit_p1) {
            // turned solid at the end of the previous step: book what it carried
            a.drop[idx] = (float)rC[0];
            a.drop[P + idx] = (float)rC[3];
            a.drop[2 * P + idx] =
                SOLUTE ? (float)((((R)gv[0] + (R)gv[1]) + ((R)gv[2] + (R)gv[3])) + (R)gv[4]) : 0.0f;
          } else if (ownC & a.bit_p2) {
            a.mask[idx] = 1;  // booked one step ago: fold the mark into bit0
          }
        }
      } else {
        // neighbours x + e_i, link order 1..8 = E, N, W, S, NE, NW, SW, SE
        R n1[9], n2[9];
        float sf[9];
        n1[1] = W1[4]; n2[1] = W1[5]; sf[1] = sol(pk_m2, 16, SCUR) ? 1.0f : 0.0f;
        n1[2] = W0[0]; n2[2] = W0[1]; sf[2] = sol(pk_m1, 0, SCUR) ? 1.0f : 0.0f;
        n1[3] = W1[2]; n2[3] = W1[3]; sf[3] = sol(pk_m2, 8, SCUR) ? 1.0f : 0.0f;
        n1[4] = W2[0]; n2[4] = W2[1]; sf[4] = sol(pk_m3, 0, SCUR) ? 1.0f : 0.0f;
        n1[5] = W0[4]; n2[5] = W0[5]; sf[5] = sol(pk_m1, 16, SCUR) ? 1.0f : 0.0f;
        n1[6] = W0[2]; n2[6] = W0[3]; sf[6] = sol(pk_m1, 8, SCUR) ? 1.0f : 0.0f;
        n1[7] = W2[2]; n2[7] = W2[3]; sf[7] = sol(pk_m3, 8, SCUR) ? 1.0f : 0.0f;
        n1[8] = W2[4]; n2[8] = W2[5]; sf[8] = sol(pk_m3, 16, SCUR) ? 1.0f : 0.0f;
        R F1x, F1y, F2x, F2y;
        sc_forces<R>(a, n1, n2, sf, rC[0], rC[3], F1x, F1y, F2x, F2y);
        R v1x, v1y, v2x, v2y, ux, uy;
        sc_velocities<R>((R)a.tau, rC[0], rC[3], rC[1], rC[2], rC[4], rC[5], F1x, F1y, F2x, F2y,
                         v1x, v1y, v2x, v2y, ux, uy);
        mo[0] = (float)rC[0];
        mo[1] = (float)v1x;
        mo[2] = (float)v1y;
        mo[3] = (float)rC[3];
        mo[4] = (float)v2x;
        mo[5] = (float)v2y;
        if (SOLUTE) {
          const int yd = y == 0 ? ny - 1 : y - 1;
          const int yu = y == ny - 1 ? 0 : y + 1;
          const unsigned iE = (unsigned)y * nx + xr, iW = (unsigned)y * nx + xl;
          const unsigned iN = (unsigned)yu * nx + xc, iS = (unsigned)yd * nx + xc;
          const double mC =
              REACT ? __hiloint2double(__float_as_int(pf[buf][12][t]), __float_as_int(pf[buf][11][t]))
                    : 0.0;
          SoluteOut so;
          solute_step<REACT, VAR, R>(a, gv, ux, uy, rC[0], rC[3], sf, mC, P, idx, iE, iN, iW, iS, xc,
                                y, ev, evx, evy, so);
#pragma unroll
          for (int q = 0; q < 5; ++q)
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(so.g[q]), rGout,
                                                  (int)(4u * so.off[q]), 0, 0);
          if (REACT && so.wm) {
            const v2u mb = {(unsigned)__double2loint(so.m), (unsigned)__double2hiint(so.m)};
            __builtin_amdgcn_raw_buffer_store_b64(mb, rPrec, (int)(8u * idx), 0, 0);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 6; ++q)
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(mo[q]), rMout, (int)(4u * idx),
                                              (int)((unsigned)q * PB), 0);
    }
    if (REACT) log_events(a, ev, evx, evy);

    // ---- rotate ------------------------------------------------------------
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      rC[q] = acc1[q];
      acc1[q] = acc0[q];
      acc0[q] = accN[q];
      W2[q] = W1[q];
      W1[q] = W0[q];
    }
    pk_m3 = pk_m2;
    pk_m2 = pk_m1;
    pk_m1 = pk_0;
    pk_0 = pk_p1;
  }
  // drain: no request may still be writing this wavefront's LDS at exit
  __builtin_amdgcn_s_waitcnt(VMCNT0);
}

// XCD-aware order: the hardware hands block b to XCD b mod 8, so XCD x
// receives q + (x < r) of T blocks (q = T / 8, r = T mod 8).  Give each XCD a
// contiguous run of tiles.  Tiles are numbered segment-major, so a run is a
// horizontal band of full rows: the waves resident on one XCD read whole
// rows together (DRAM pages stay open), and both halo directions are shared
// in one L2 except at the band's edges.
__host__ __device__ inline int xcd_tile(int b, int T) {
  const int q = T >> 3, r = T & 7, x = b & 7, j = b >> 3;
  return (x < r) ? x * (q + 1) + j : r * (q + 1) + (x - r) * q + j;
}

template <bool SOLUTE, bool REACT, bool VAR, typename R, int KIND, bool NT>
__device__ __forceinline__ void run_tile(const StepArgs& a, int strip, int seg, char* lds_raw) {
  if (KIND == KIND_MM)
    mom_wave<SOLUTE, REACT, VAR, R, NT>(a, strip, seg);
  else
    step_tile<SOLUTE, REACT, VAR, R, KIND == KIND_PM, NT>(a, strip, seg, lds_raw);
}

template <bool SOLUTE, bool REACT, bool VAR, typename R, int KIND, bool NT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8)))
k_step(const StepArgs a) {
  extern __shared__ char lds_raw[];
  const int T = a.nstrips * a.nsegs;
  const int tile = a.remap ? xcd_tile(blockIdx.x, T) : (int)blockIdx.x;
  const int seg = tile / a.nstrips;
  run_tile<SOLUTE, REACT, VAR, R, KIND, NT>(a, tile - seg * a.nstrips, seg, lds_raw);
}

// Batched step: one launch advances every instance of a batch by one step.
// Block b takes tile tiles[b] (instance, strip, segment; the host orders the
// list per XCD); the instance's arguments for the current parity come from
// device memory, and the step index is the device counter *stepc plus the
// launch's offset j within its sequence.  A sequence of n launches (offsets
// 0..n-1) is followed by k_tick(stepc, n), so a captured sequence replays
// from where the last one ended.
template <bool SOLUTE, bool REACT, bool VAR, typename R, int KIND>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8)))
k_step_batch(const StepArgs* __restrict__ insts, const int4* __restrict__ tiles,
             const long long* __restrict__ stepc, int j) {
  extern __shared__ char lds_raw[];
  const long long step = *stepc + j;
  const int4 e = tiles[blockIdx.x];
  StepArgs a = insts[2 * e.x + (int)(step & 1)];
  a.step = step;
  a.bit_p1 = pending_bit(step - 1);
  a.bit_p2 = pending_bit(step - 2);
  a.bit_cur = pending_bit(step);
  run_tile<SOLUTE, REACT, VAR, R, KIND, false>(a, e.y, e.z, lds_raw);
}

// Advances the device step counter by n (one lane).
__global__ void k_tick(long long* stepc, int n) {
  if (threadIdx.x == 0) *stepc += n;
}

// Rest-state populations from the FP64 densities (rounded once to FP32).
__global__ void k_init(const double* __restrict__ rho1, const double* __restrict__ rho2,
                       const double* __restrict__ conc, const uint8_t* __restrict__ mask,
                       float* __restrict__ f, float* __restrict__ g, double* __restrict__ m,
                       int32_t* __restrict__ sstep, float* __restrict__ drop, long long N,
                       long long P, int solute, int react, int q4) {
  const float w9[9] = {4.0f / 9.0f, 1.0f / 9.0f, 1.0f / 9.0f, 1.0f / 9.0f, 1.0f / 9.0f,
                       1.0f / 36.0f, 1.0f / 36.0f, 1.0f / 36.0f, 1.0f / 36.0f};
  const float w5[5] = {q4 ? 0.0f : 1.0f / 3.0f, q4 ? 0.25f : 1.0f / 6.0f, q4 ? 0.25f : 1.0f / 6.0f,
                       q4 ? 0.25f : 1.0f / 6.0f, q4 ? 0.25f : 1.0f / 6.0f};
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

// ---- observers -------------------------------------------------------------
// Node densities and momenta of state n, from stored populations or, in the
// moment scheme, gathered from the stored moments of the node and its
// upstream neighbours (the same arithmetic as the moment step, in FP64).
struct PopSrc {
  const float* __restrict__ f;
  long long P;
  __device__ void rho(long long i, int, int, double& r1, double& r2) const {
    double a = 0, b = 0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      a += (double)f[q * P + i];
      b += (double)f[(9 + q) * P + i];
    }
    r1 = a;
    r2 = b;
  }
  __device__ void full(long long i, int, int, double* o) const {
    const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    double r1 = 0, r2 = 0, j1x = 0, j1y = 0, j2x = 0, j2y = 0;
    for (int q = 0; q < 9; ++q) {
      const double a = f[q * P + i], b = f[(9 + q) * P + i];
      r1 += a; r2 += b;
      j1x += a * ex[q]; j1y += a * ey[q];
      j2x += b * ex[q]; j2y += b * ey[q];
    }
    o[0] = r1; o[1] = r2; o[2] = j1x; o[3] = j1y; o[4] = j2x; o[5] = j2y;
  }
};

struct MomSrc {
  const float* __restrict__ M;
  const uint8_t* __restrict__ mask;
  long long P;
  int nx, ny;
  unsigned sprev;  // solid bits of state n-1
  __device__ void links(int x, int y, int comp, double* fl) const {
    const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    float r[9], vx[9], vy[9];
    bool up[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      int xs = x - ex[q], ysrc = y - ey[q];
      xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
      ysrc = ysrc < 0 ? ysrc + ny : (ysrc >= ny ? ysrc - ny : ysrc);
      const long long k = (long long)ysrc * nx + xs;
      up[q] = !(mask[k] & sprev);
      r[q] = M[(3 * comp) * P + k];
      vx[q] = M[(3 * comp + 1) * P + k];
      vy[q] = M[(3 * comp + 2) * P + k];
    }
    gather_links<double>(r, vx, vy, up, fl);
  }
  __device__ void full(long long, int x, int y, double* o) const {
    double fl[9];
    links(x, y, 0, fl);
    moments9<double>(fl, o[0], o[2], o[3]);
    links(x, y, 1, fl);
    moments9<double>(fl, o[1], o[4], o[5]);
  }
  __device__ void rho(long long i, int x, int y, double& r1, double& r2) const {
    double o[6];
    full(i, x, y, o);
    r1 = o[0];
    r2 = o[1];
  }
};

// Observe, pass 1: per-block FP64 partial sums.  Slots:
// 0 mass1, 1 mass2, 2 solute, 3 precipitate, 4 removed1, 5 removed2,
// 6 removed solute, 7 solid count, 8 non-finite count.
template <typename Src>
__global__ void __launch_bounds__(256) k_obs_partial(Src src, const float* __restrict__ g,
                                                     const uint8_t* __restrict__ mask,
                                                     const double* __restrict__ m,
                                                     const float* __restrict__ drop, int nx,
                                                     long long N, long long P, unsigned p1,
                                                     unsigned p2, int solute, int react,
                                                     double* __restrict__ partial) {
  __shared__ double red[OBS_SLOTS][256];
  const unsigned sprev = 1u | p2, scur = sprev | p1;
  double acc[OBS_SLOTS];
#pragma unroll
  for (int j = 0; j < OBS_SLOTS; ++j) acc[j] = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const unsigned b = mask[i];
    double s1 = 0, s2 = 0, sc = 0;
    if (!(b & sprev)) {
      src.rho(i, (int)(i % nx), (int)(i / nx), s1, s2);
      if (solute) {
#pragma unroll
        for (int q = 0; q < 5; ++q) sc += (double)g[q * P + i];
      }
    }
    if (b & scur) {
      acc[7] += 1.0;
      if (b & p1) {  // turned solid at the end of the last step, not yet booked
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

// Capillary observables computed by one workgroup of 256 threads: centreline
// front, largest grown width, first closure, and the sums behind the radii of
// Fig. 4.  out: [0] z, [1] delta_e, [2] closure step (-1 if none), [3] open
// area A (fluid nodes between the walls), [4] narrowest open column, [5] sum
// over neighbouring columns of |h(x+1) - h(x)|, h the growth on the lower
// wall.  sb: solid bits of state n.
template <typename Src>
__device__ void capillary_obs(const Src& src, const uint8_t* __restrict__ mask,
                              const int32_t* __restrict__ sstep, int nx, unsigned sb, int x_in,
                              int x_out, int y0, int W, int react, double* __restrict__ out) {
  __shared__ int s_min[256];
  __shared__ double s_de[256];
  __shared__ long long s_cl[256];
  __shared__ int s_area[256], s_wmin[256], s_steps[256];
  const int nr = (W % 2 == 0) ? 2 : 1;
  const int row0 = (W % 2 == 0) ? (y0 + W / 2 - 1) : (y0 + (W - 1) / 2);
  int best = x_out;  // first x where the scan stops
  double de = 0.0;
  long long cl = -1;
  int area = 0, wmin = W, steps = 0;
  for (int x = x_in + threadIdx.x; x < x_out; x += blockDim.x) {
    // front predicate at x
    bool blocked = false, nblocked = false;
    double phi = 0, phin = 0;
    for (int r = 0; r < nr; ++r) {
      const long long i = (long long)(row0 + r) * nx + x;
      if (mask[i] & sb) blocked = true;
      else { double a, b; src.rho(i, x, row0 + r, a, b); phi += a / (a + b); }
    }
    phi /= nr;
    if (x + 1 < x_out) {
      for (int r = 0; r < nr; ++r) {
        const long long i = (long long)(row0 + r) * nx + x + 1;
        if (mask[i] & sb) nblocked = true;
        else { double a, b; src.rho(i, x + 1, row0 + r, a, b); phin += a / (a + b); }
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
    int w = 0;
    for (int y = y0; y < y0 + W; ++y) w += (mask[(long long)y * nx + x] & sb) ? 0 : 1;
    area += w;
    wmin = min(wmin, w);
    if (x + 1 < x_out) {
      int dn = 0;
      while (dn < W && (mask[(long long)(y0 + dn) * nx + x + 1] & sb)) ++dn;
      steps += abs(dn - db);
    }
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
  s_area[threadIdx.x] = area;
  s_wmin[threadIdx.x] = wmin;
  s_steps[threadIdx.x] = steps;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      s_area[threadIdx.x] += s_area[threadIdx.x + s];
      s_wmin[threadIdx.x] = min(s_wmin[threadIdx.x], s_wmin[threadIdx.x + s]);
      s_steps[threadIdx.x] += s_steps[threadIdx.x + s];
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
        else { double a, b; src.rho(i, x, row0 + r, a, b); phi += a / (a + b); }
      }
      phi /= nr;
      if (blocked) z = (double)(x - x_in);
      else if (x == x_in && phi < 0.5) z = 0.0;
      else {
        for (int r = 0; r < nr; ++r) {
          const long long i = (long long)(row0 + r) * nx + x + 1;
          double a, b; src.rho(i, x + 1, row0 + r, a, b); phin += a / (a + b);
        }
        phin /= nr;
        z = (double)x + (phi - 0.5) / (phi - phin) - x_in;
      }
    }
    out[0] = z;
    out[1] = s_de[0];
    out[2] = (double)s_cl[0];
    out[3] = (double)s_area[0];
    out[4] = (double)s_wmin[0];
    out[5] = (double)s_steps[0];
  }
}

template <typename Src>
__global__ void __launch_bounds__(256) k_obs_capillary(Src src, const uint8_t* __restrict__ mask,
                                                       const int32_t* __restrict__ sstep,
                                                       int nx, unsigned sb, int x_in, int x_out,
                                                       int y0, int W, int react,
                                                       double* __restrict__ out) {
  capillary_obs(src, mask, sstep, nx, sb, x_in, x_out, y0, W, react, out);
}

// Front of every instance of a batch (workgroup i -> instance i) into column
// `slot` of the n x nslots table; queued without synchronisation.
__global__ void __launch_bounds__(256) k_front_batch(const StepArgs* __restrict__ insts,
                                                     const int4* __restrict__ capi,
                                                     const long long* __restrict__ stepc,
                                                     int slot, int nslots, int mom,
                                                     double* __restrict__ table) {
  __shared__ double res[6];
  const long long step = *stepc;
  const int i = blockIdx.x;
  const StepArgs& a = insts[2 * i + (int)(step & 1)];
  const int4 c = capi[i];  // x_in, x_out, y0, W
  if (c.w <= 0) {
    if (threadIdx.x == 0) table[(long long)i * nslots + slot] = __builtin_nan("");
    return;
  }
  const unsigned p1 = pending_bit(step - 1), p2 = pending_bit(step - 2);
  const unsigned sb = 1u | p1 | p2;
  if (mom) {
    const MomSrc src{a.fin, a.mask, a.P, a.nx, a.ny, 1u | p2};
    capillary_obs(src, a.mask, a.sstep, a.nx, sb, c.x, c.y, c.z, c.w, a.react, res);
  } else {
    const PopSrc src{a.fin, a.P};
    capillary_obs(src, a.mask, a.sstep, a.nx, sb, c.x, c.y, c.z, c.w, a.react, res);
  }
  if (threadIdx.x == 0) table[(long long)i * nslots + slot] = res[0];
}

// Macroscopic fields of the current state as FP64 planes:
// 0 rho1, 1 rho2, 2 ux, 3 uy, 4 conc, 5 precipitate, 6 solid.
template <typename Src>
__global__ void k_fields(Src src, const float* __restrict__ g, const uint8_t* __restrict__ mask,
                         const double* __restrict__ m, int nx, int ny, long long P, unsigned sb,
                         int solute, int react, double G, double Gads1, double Gads2, double ax,
                         double ay, double* __restrict__ out) {
  const long long N = (long long)nx * ny;
  const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % nx), y = (int)(i / nx);
    const bool s = (mask[i] & sb) != 0;
    double r1 = 0, r2 = 0, ux = 0, uy = 0, c = 0;
    if (!s) {
      double o[6];
      src.full(i, x, y, o);
      r1 = o[0];
      r2 = o[1];
      double c1x = 0, c1y = 0, c2x = 0, c2y = 0, sx = 0, sy = 0;
      for (int q = 1; q < 9; ++q) {
        int xn = x + ex[q], yn = y + ey[q];
        xn = xn < 0 ? xn + nx : (xn >= nx ? xn - nx : xn);
        yn = yn < 0 ? yn + ny : (yn >= ny ? yn - ny : yn);
        const long long k = (long long)yn * nx + xn;
        if (mask[k] & sb) { sx += w[q] * ex[q]; sy += w[q] * ey[q]; continue; }
        double a, b;
        src.rho(k, xn, yn, a, b);
        c1x += w[q] * a * ex[q]; c1y += w[q] * a * ey[q];
        c2x += w[q] * b * ex[q]; c2y += w[q] * b * ey[q];
      }
      const double F1x = -G * r1 * c2x - Gads1 * r1 * sx + r1 * ax;
      const double F1y = -G * r1 * c2y - Gads1 * r1 * sy + r1 * ay;
      const double F2x = -G * r2 * c1x - Gads2 * r2 * sx + r2 * ax;
      const double F2y = -G * r2 * c1y - Gads2 * r2 * sy + r2 * ay;
      ux = (o[2] + o[4] + 0.5 * (F1x + F2x)) / (r1 + r2);
      uy = (o[3] + o[5] + 0.5 * (F1y + F2y)) / (r1 + r2);
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

// Populations of state n rebuilt from the stored moments (zero at nodes that
// were solid in state n-1, which carry none).
__global__ void k_unpack(MomSrc src, float* __restrict__ fout) {
  const long long N = (long long)src.nx * src.ny;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % src.nx), y = (int)(i / src.nx);
    const bool fluid = !(src.mask[i] & src.sprev);
    for (int comp = 0; comp < 2; ++comp) {
      double fl[9];
      if (fluid) src.links(x, y, comp, fl);
#pragma unroll
      for (int q = 0; q < 9; ++q) fout[(9 * comp + q) * src.P + i] = fluid ? (float)fl[q] : 0.0f;
    }
  }
}

// ---- launchers ------------------------------------------------------------
size_t step_lds_bytes(int kind, int tx) {
  if (kind == KIND_MM) return 0;  // registers and cross-lane moves only
  return (size_t)4 * tx * (2 * sizeof(double) + sizeof(float));
}

// Runs that use a reaction or solute-lattice variant (saturation, held
// source, D2Q4) take their own instantiation, so the plain model keeps its
// instruction stream.
inline bool uses_variants(const StepArgs& a) { return a.c_eq > 0.0 || a.hold_x > 0 || a.q4; }

template <typename R, int KIND, bool NT>
void launch_step_t(const StepArgs& a, int T, int tx, size_t lds, hipStream_t st) {
  if (a.solute && a.react && uses_variants(a))
    hipLaunchKernelGGL((k_step<true, true, true, R, KIND, NT>), dim3(T), dim3(tx), lds, st, a);
  else if (a.solute && a.react)
    hipLaunchKernelGGL((k_step<true, true, false, R, KIND, NT>), dim3(T), dim3(tx), lds, st, a);
  else if (a.solute && uses_variants(a))
    hipLaunchKernelGGL((k_step<true, false, true, R, KIND, NT>), dim3(T), dim3(tx), lds, st, a);
  else if (a.solute)
    hipLaunchKernelGGL((k_step<true, false, false, R, KIND, NT>), dim3(T), dim3(tx), lds, st, a);
  else
    hipLaunchKernelGGL((k_step<false, false, false, R, KIND, NT>), dim3(T), dim3(tx), lds, st, a);
}

// nt: the non-temporal load hint, compiled for the moment and population
// steps (the one-off PM step ignores it).  The arithmetic is FP64 throughout.
hipError_t launch_step(const StepArgs& a, int tx, int kind, int nt, hipStream_t st) {
  const int T = a.nstrips * a.nsegs;
  if (kind == KIND_MM) tx = 64;  // the moment step runs one wavefront per tile
  const size_t lds = step_lds_bytes(kind, tx);
  if (kind == KIND_MM) {
    if (nt) launch_step_t<double, KIND_MM, true>(a, T, tx, lds, st);
    else launch_step_t<double, KIND_MM, false>(a, T, tx, lds, st);
  } else if (kind == KIND_PM) {
    launch_step_t<double, KIND_PM, false>(a, T, tx, lds, st);
  } else {
    if (nt) launch_step_t<double, KIND_POP, true>(a, T, tx, lds, st);
    else launch_step_t<double, KIND_POP, false>(a, T, tx, lds, st);
  }
  return hipGetLastError();
}

template <typename R, int KIND>
void launch_batch_t(const StepArgs* insts, const int4* tiles, int ntiles, const long long* stepc,
                    int j, int tx, int solute, int react, int var, size_t lds, hipStream_t st) {
  if (solute && react && var)
    hipLaunchKernelGGL((k_step_batch<true, true, true, R, KIND>), dim3(ntiles), dim3(tx), lds, st, insts, tiles, stepc, j);
  else if (solute && react)
    hipLaunchKernelGGL((k_step_batch<true, true, false, R, KIND>), dim3(ntiles), dim3(tx), lds, st, insts, tiles, stepc, j);
  else if (solute && var)
    hipLaunchKernelGGL((k_step_batch<true, false, true, R, KIND>), dim3(ntiles), dim3(tx), lds, st, insts, tiles, stepc, j);
  else if (solute)
    hipLaunchKernelGGL((k_step_batch<true, false, false, R, KIND>), dim3(ntiles), dim3(tx), lds, st, insts, tiles, stepc, j);
  else
    hipLaunchKernelGGL((k_step_batch<false, false, false, R, KIND>), dim3(ntiles), dim3(tx), lds, st, insts, tiles, stepc, j);
}

hipError_t launch_step_batch(const StepArgs* insts, const int4* tiles, int ntiles,
                             const long long* stepc, int j, int tx, int solute, int react,
                             int var, int kind, hipStream_t st) {
  if (kind == KIND_MM) tx = 64;
  const size_t lds = step_lds_bytes(kind, tx);
  if (kind == KIND_MM) launch_batch_t<double, KIND_MM>(insts, tiles, ntiles, stepc, j, tx, solute, react, var, lds, st);
  else if (kind == KIND_PM) launch_batch_t<double, KIND_PM>(insts, tiles, ntiles, stepc, j, tx, solute, react, var, lds, st);
  else launch_batch_t<double, KIND_POP>(insts, tiles, ntiles, stepc, j, tx, solute, react, var, lds, st);
  return hipGetLastError();
}

hipError_t launch_tick(long long* stepc, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, st, stepc, n);
  return hipGetLastError();
}

hipError_t launch_front_batch(const StepArgs* insts, const int4* capi, const long long* stepc,
                              int n, int slot, int nslots, int mom, double* table, hipStream_t st) {
  hipLaunchKernelGGL(k_front_batch, dim3(n), dim3(256), 0, st, insts, capi, stepc, slot, nslots,
                     mom, table);
  return hipGetLastError();
}

int host_xcd_tile(int b, int T) { return xcd_tile(b, T); }

static int grid_for(long long N) { return (int)((N + 255) / 256 < 8192 ? (N + 255) / 256 : 8192); }

hipError_t launch_init(const double* r1, const double* r2, const double* c, const uint8_t* mask,
                       float* f, float* g, double* m, int32_t* sstep, float* drop, long long N,
                       long long P, int solute, int react, int q4, hipStream_t st) {
  hipLaunchKernelGGL(k_init, dim3(grid_for(N)), dim3(256), 0, st, r1, r2, c, mask, f, g, m, sstep,
                     drop, N, P, solute, react, q4);
  return hipGetLastError();
}

hipError_t launch_unpack(const float* M, const uint8_t* mask, int nx, int ny, long long P,
                         unsigned sprev, float* fout, hipStream_t st) {
  const MomSrc src{M, mask, P, nx, ny, sprev};
  hipLaunchKernelGGL(k_unpack, dim3(grid_for((long long)nx * ny)), dim3(256), 0, st, src, fout);
  return hipGetLastError();
}

template <typename Src>
void observe_t(const Src& src, const float* g, const uint8_t* mask, const double* m,
               const float* drop, const int32_t* sstep, int nx, int ny, long long P, unsigned p1,
               unsigned p2, int solute, int react, int nblocks, double* partial, double* out,
               int x_in, int x_out, int y0, int W, hipStream_t st) {
  const long long N = (long long)nx * ny;
  hipLaunchKernelGGL(k_obs_partial<Src>, dim3(nblocks), dim3(256), 0, st, src, g, mask, m, drop,
                     nx, N, P, p1, p2, solute, react, partial);
  hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(64), 0, st, partial, nblocks, out);
  if (W > 0)
    hipLaunchKernelGGL(k_obs_capillary<Src>, dim3(1), dim3(256), 0, st, src, mask, sstep, nx,
                       1u | p1 | p2, x_in, x_out, y0, W, react, out + OBS_SLOTS);
}

hipError_t launch_observe(const float* f, const float* g, const uint8_t* mask, const double* m,
                          const float* drop, const int32_t* sstep, int nx, int ny, long long P,
                          unsigned p1, unsigned p2, int mom, int solute, int react, int nblocks,
                          double* partial, double* out, int x_in, int x_out, int y0, int W,
                          hipStream_t st) {
  if (mom)
    observe_t(MomSrc{f, mask, P, nx, ny, 1u | p2}, g, mask, m, drop, sstep, nx, ny, P, p1, p2,
              solute, react, nblocks, partial, out, x_in, x_out, y0, W, st);
  else
    observe_t(PopSrc{f, P}, g, mask, m, drop, sstep, nx, ny, P, p1, p2, solute, react, nblocks,
              partial, out, x_in, x_out, y0, W, st);
  return hipGetLastError();
}

hipError_t launch_fields(const float* f, const float* g, const uint8_t* mask, const double* m,
                         int nx, int ny, long long P, unsigned p1, unsigned p2, int mom,
                         int solute, int react, double G, double Gads1, double Gads2, double ax,
                         double ay, double* out, hipStream_t st) {
  const int blocks = grid_for((long long)nx * ny);
  const unsigned sb = 1u | p1 | p2;
  if (mom)
    hipLaunchKernelGGL(k_fields<MomSrc>, dim3(blocks), dim3(256), 0, st,
                       MomSrc{f, mask, P, nx, ny, 1u | p2}, g, mask, m, nx, ny, P, sb, solute,
                       react, G, Gads1, Gads2, ax, ay, out);
  else
    hipLaunchKernelGGL(k_fields<PopSrc>, dim3(blocks), dim3(256), 0, st, PopSrc{f, P}, g, mask, m,
                       nx, ny, P, sb, solute, react, G, Gads1, Gads2, ax, ay, out);
  return hipGetLastError();
}

}  // namespace lbmdev
