/*
 * lbm.h - C ABI of the MI355X (gfx950) reactive capillary-infiltration
 * lattice Boltzmann library.
 *
 * The library advances the 2D lattice Boltzmann model of Sergi, Grossi,
 * Leidi & Ortona, "Lattice Boltzmann simulation of the surface growth effects
 * for the infiltration of molten Si in carbon preforms" (section "LB models"):
 * two fluid components (wetting Si and the other substance) on a D2Q9 BGK
 * lattice with bounce-back at the solid phase, fluid-fluid cohesion and
 * solid-fluid adhesion forces, a D2Q5 BGK lattice for the dissolved species
 * weakly coupled to the flow, and surface reaction by mass precipitation
 * with rate constant k_r: the precipitated mass accumulates at wall-adjacent
 * nodes and a node whose mass exceeds a threshold turns solid.  The
 * observables are the centreline position of the invading front z(t)
 * (Results, Eq. (1) and Fig. 2), the largest grown solid width Delta e and
 * pore closure (Fig. 3).
 *
 * Conventions for every call:
 *   - Every call returns lbm_status; nothing throws across the ABI.  On an
 *     error lbm_last_error() returns a message for the calling thread.
 *   - Lattice nx*ny nodes, node index y*nx + x, periodic in x and y; walls
 *     exist only through the solid mask.  Host arrays are row-major (ny, nx).
 *   - Host inputs are copied before the call returns.
 *   - `stream` (a hipStream_t) and `workspace` (device memory) are borrowed:
 *     the caller keeps both alive until lbm_destroy.  All device work of a
 *     handle is queued on that stream.
 *   - lbm_step only queues work.  Faults of queued kernels surface at the
 *     next synchronising call (lbm_observe, lbm_fields, lbm_events,
 *     lbm_save), which returns LBM_EDEVICE.
 *   - A handle is used by one host thread at a time.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* bad argument, parameter, mask value or buffer size */
  LBM_ENOMEM = -2,     /* host allocation failed */
  LBM_EDEVICE = -3,    /* a HIP call or a queued kernel failed */
  LBM_ENONFINITE = -4, /* a density or concentration is NaN/Inf: handle poisoned */
  LBM_ESTATE = -5      /* handle poisoned by an earlier LBM_ENONFINITE/LBM_EDEVICE */
} lbm_status;

typedef struct lbm_sim lbm_sim; /* opaque; owned by the library until lbm_destroy */

/* Model and run parameters.  Readings of the paper that fix these forms are
 * stated per field. */
typedef struct {
  int32_t nx, ny;    /* lattice size, both >= 3 */
  double tau;        /* flow BGK relaxation time of both components, > 1/2 */
  double G;          /* cohesion between unlike components (Shan-Chen/Martys-Chen
                        type: F_s = -G rho_s sum_i w_i rho_other(x+e_i) e_i) */
  double G_ads[2];   /* adhesion of component 1 (wetting, negative = attracted
                        to the wall) and 2: F_s -= G_ads[s] rho_s sum_i w_i s(x+e_i) e_i */
  double tau_g;      /* D2Q5 solute relaxation time, D = (tau_g - 1/2)/3;
                        0 switches the solute lattice off, else > 1/2 */
  double k_r;        /* reaction-rate constant [lu/ts]: a fluid node with n_s solid
                        axis neighbours loses r = k_r n_s phi of its solute per step
                        (phi = rho1/(rho1+rho2)) to the precipitate; 0 = off.
                        Requires 0 <= 4 k_r <= 1 and tau_g > 0 when non-zero. */
  double threshold;  /* precipitated mass above which (strictly) a node turns solid, > 0 */
  double accel[2];   /* uniform body acceleration on both components (tests) */
  int32_t x_in, x_out, y0, W; /* capillary for the observables: section
                        x_in <= x < x_out, channel rows y0..y0+W-1; W = 0: none */
  /* Variants of the reaction and the solute lattice (section "LB models":
     precipitation at the surface, an advection-diffusion BGK lattice); all
     zero gives the plain model above. */
  double c_eq;       /* saturation concentration: a reacting node precipitates
                        k_r n_s phi (C - c_eq) when C > c_eq, nothing otherwise;
                        >= 0 */
  double c_hold;     /* held source: every fluid node with x < hold_x has its
                        solute reset each step to the equilibrium at c_hold */
  int32_t hold_x;    /* 0 = no held source; else 1..nx, needs tau_g > 0 */
  int32_t solute_q;  /* solute lattice: 0 or 5 = D2Q5 (w0 = 1/3, D = (tau_g-1/2)/3),
                        4 = D2Q4 (w = 1/4, no rest link, D = (tau_g-1/2)/2) */
} lbm_params;

/* Observables of the current state (lbm_observe).  Sums are FP64. */
typedef struct {
  int64_t step;              /* number of steps taken since lbm_init */
  double mass[2];            /* sum of rho_1, rho_2 over fluid nodes */
  double mass_removed[2];    /* fluid mass taken out by nodes that turned solid */
  double solute;             /* sum of the solute concentration over fluid nodes */
  double precipitate;        /* sum of precipitated mass over all nodes */
  double solute_removed;     /* solute taken out by nodes that turned solid */
  double front_z;            /* centreline front measured from x_in [lu]; NaN if W == 0;
                                x_out - x_in if no crossing (breakthrough) */
  double delta_e;            /* largest solid width grown from one channel wall;
                                W/2 for a closed column */
  int64_t closure_step;      /* first step with a closed capillary column, -1 if none */
  int64_t n_solid;           /* number of solid nodes */
  int64_t n_events;          /* number of growth events so far */
  int32_t nonfinite;         /* 1 if any fluid density/concentration is NaN/Inf */
  int32_t pad;
  /* Radii of the capillary section (section "Results and discussion", Fig. 4),
     each equal to W for the unreacted slit; NaN if W == 0.  With w(x) the
     fluid nodes of column x between the walls and A = sum w the open area:
     r_min = min w, r_ave = A / L (L = x_out - x_in), and the hydraulic radius
     r_h = A / P, P the length of the lower wall's profile (one unit per column
     plus the vertical steps between neighbouring columns).  The effective
     radius of Eq. (1) needs a front time series and a run without reaction:
     see paper_1309_6726_amd/radii.py. */
  double r_min, r_ave, r_h;
} lbm_obs;

/* A growth event: node (x, y) is solid from state `step` on. */
typedef struct {
  int32_t x, y;
  int64_t step;
} lbm_event;

/* Field selection for lbm_fields; host_fields receives one nx*ny double array
 * per selected field, in this bit order. */
enum {
  LBM_FIELD_RHO1 = 1u << 0,
  LBM_FIELD_RHO2 = 1u << 1,
  LBM_FIELD_UX = 1u << 2,   /* barycentric velocity (sum_s j_s + F_s/2)/(rho1+rho2) */
  LBM_FIELD_UY = 1u << 3,
  LBM_FIELD_CONC = 1u << 4,
  LBM_FIELD_PRECIP = 1u << 5,
  LBM_FIELD_SOLID = 1u << 6 /* 0/1 */
};

/* Device memory needed by lbm_init for these parameters (bytes). */
lbm_status lbm_workspace_bytes(const lbm_params* p, size_t* bytes);

/* Create a simulation.  solid: host nx*ny bytes, values 0/1.  rho1, rho2: host
 * nx*ny FP64 densities (>= 0, finite; ignored at solid nodes), rounded once to
 * FP32.  conc: host nx*ny FP64 solute concentration, or NULL when tau_g == 0.
 * The initial populations are the rest equilibria f_i = w_i rho, g_k = w_k C.
 * workspace: device buffer of at least lbm_workspace_bytes, 256-byte aligned.
 * LBM_EINVAL on any bad argument (see the lbm_params fields). */
lbm_status lbm_init(const lbm_params* p, const uint8_t* solid, const double* rho1,
                    const double* rho2, const double* conc, void* stream, void* workspace,
                    size_t ws_bytes, lbm_sim** out);

/* Queue nsteps time steps (nsteps >= 0).  One step: moments, cohesion and
 * adhesion forces, BGK collision of both components, solute BGK, surface
 * reaction, streaming with halfway bounce-back, and growth of every node
 * whose precipitate exceeds the threshold (synchronous, end of step). */
lbm_status lbm_step(lbm_sim* sim, int64_t nsteps);

/* Observables of the current state.  Synchronises the stream.
 * LBM_ENONFINITE (and a poisoned handle) if a NaN/Inf is found. */
lbm_status lbm_observe(lbm_sim* sim, lbm_obs* out);

/* Copy selected macroscopic fields of the current state to the host as FP64
 * (host_fields: popcount(field_mask) * nx*ny doubles).  Synchronises. */
lbm_status lbm_fields(lbm_sim* sim, uint32_t field_mask, double* host_fields);

/* Copy growth events [first, first+cap) to buf; *n receives the total count.
 * Events are unordered within a step.  Synchronises. */
lbm_status lbm_events(lbm_sim* sim, int64_t first, lbm_event* buf, int64_t cap, int64_t* n);

/* Checkpoint: serialise the whole state (populations, mask, precipitate,
 * ledgers, events, step) into blob.  With blob == NULL only *n is set to the
 * size needed.  lbm_load restores a blob written by lbm_save for a handle with
 * the same parameters; it also clears a poisoned state.  Blob layout (native
 * endianness, no padding): header {uint64 magic 0x4C424D5853494D31, int32 nx,
 * ny, int32 flags (1 solute, 2 reaction), int32 version 2, int64 step,
 * int64 n_events}, then f float[18][N] (component-major, link order e0..e8 =
 * (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1)), g float[5][N]
 * if solute, mask uint8[N] (bit0 solid; bit 1 + (s mod 3) marks a node that
 * turned solid at the end of step s, kept for the two steps after it, so a
 * state at step n may also hold the marks of steps n-1 and n-2), then if
 * reaction: m double[N], solid step int32[N] (-1 fluid), removed float[3][N],
 * events lbm_event[n_events].  In a state at step n, the population slots of
 * nodes already solid before (bit0, or the mark of step n-2) carry no
 * information: no step reads them, and a step may leave them or write zeros
 * there.  A node marked at the end of step n-1 still holds the populations it
 * carried, which step n books.  Populations are always saved: in the moment
 * scheme (lbm_set_scheme) the moments are first unpacked into populations
 * and the run goes on from those, so a loaded checkpoint continues bit for
 * bit like the run that saved it. */
lbm_status lbm_save(lbm_sim* sim, void* blob, size_t cap, size_t* n);
lbm_status lbm_load(lbm_sim* sim, const void* blob, size_t n);

/* Launch shape of the fused step: tx threads per workgroup (64, 128 or 256)
 * covering tx-2 owned columns (tx-4 in the moment scheme), sy owned rows per
 * workgroup (1..4096).  The shape changes no result bit. */
lbm_status lbm_set_tile(lbm_sim* sim, int32_t tx, int32_t sy);
lbm_status lbm_get_tile(const lbm_sim* sim, int32_t* tx, int32_t* sy);

/* Cache hint on the step's loads: 0 (default) the normal policy, 1 the
 * non-temporal hint on the streamed state (population step: the populations;
 * moment step: the moments of a workgroup's own rows and the solute
 * populations, while the halo rows, which the neighbouring workgroup reads
 * too, and the precipitate keep the normal policy).  Which is faster
 * depends on how the lattice's footprint meets the GPU's caches, so
 * lbm_autotune chooses it along with the launch shape.  It applies to the
 * single-lattice steps (not the batched step) and changes no result bit. */
lbm_status lbm_set_load_hint(lbm_sim* sim, int32_t nontemporal);
lbm_status lbm_get_load_hint(const lbm_sim* sim, int32_t* nontemporal);

/* State representation between steps (section "LB models": BGK relaxation
 * with relaxation time tau).  At tau = 1 a collision relaxes every
 * population fully onto the equilibrium of its component, so the
 * post-collision state of a node is fixed by (rho_s, v_s) of each component:
 * LBM_SCHEME_MOMENTS stores those six numbers per node instead of eighteen
 * populations and rebuilds the populations arriving at a node from the
 * equilibria of its upstream neighbours (bounce-back: the node's own
 * equilibrium on the opposite link).  This moves 48 instead of 144 bytes of
 * flow state per fluid node and step; the results agree with the population
 * scheme to FP32 rounding.  LBM_SCHEME_AUTO (default) takes moments when
 * tau == 1 and populations otherwise; LBM_SCHEME_MOMENTS with tau != 1 is
 * LBM_EINVAL.  The first step after init or load reads populations.
 * Observers and checkpoints work in both schemes. */
enum { LBM_SCHEME_AUTO = 0, LBM_SCHEME_POPULATIONS = 1, LBM_SCHEME_MOMENTS = 2 };
lbm_status lbm_set_scheme(lbm_sim* sim, int32_t scheme);

/* Time the launch shapes and both load hints (steps_per_candidate steps
 * each, on a saved copy of the state, which is restored), time the three
 * fastest again, interleaved, three times over at least 20 ms each, keep the
 * one with the lowest median and report its shape and median time per step
 * (the hint is read with lbm_get_load_hint).  When the environment variable
 * LBM_AUTOTUNE_CACHE names a file, a cached choice for the same (GPU
 * architecture, nx x ny, solute/reaction switches, scheme) is used without
 * timing, and new choices are appended to it as JSON lines
 * {"key": ..., "tx": ..., "sy": ..., "ms": ..., "nt": ...}. */
lbm_status lbm_autotune(lbm_sim* sim, int32_t steps_per_candidate, int32_t* tx, int32_t* sy,
                        double* best_ms_per_step);

/* ------------------------------------------------------------------------
 * Batched sweeps: many independent lattices of different sizes and
 * parameters advanced together, one launch per step for the whole batch (a
 * flat list of (instance, strip, segment) tiles), optionally replayed from a
 * captured HIP graph of `chunk` steps.  Every instance computes exactly what
 * lbm_step computes for it alone (bit for bit).  All instances share tau, G,
 * accel and the solute/reaction switches; the rest of lbm_params is per
 * instance.  Front positions can be recorded into a device table at chosen
 * steps without synchronising (used to sample z(t) for parameter sweeps).
 * ------------------------------------------------------------------------ */
typedef struct lbm_batch lbm_batch;

/* Device memory for n instances (p: n records) and an n x nslots front table. */
lbm_status lbm_batch_workspace_bytes(int32_t n, const lbm_params* p, int32_t nslots, size_t* bytes);

/* As lbm_init for each instance i (solid[i], rho1[i], rho2[i], conc[i] host
 * arrays of its own size; conc may be NULL when tau_g == 0).  The inputs stay
 * staged in the workspace so the batch can be reset to its initial state. */
lbm_status lbm_batch_init(int32_t n, const lbm_params* p, const uint8_t* const* solid,
                          const double* const* rho1, const double* const* rho2,
                          const double* const* conc, int32_t nslots, void* stream,
                          void* workspace, size_t ws_bytes, lbm_batch** out);

/* Launch shape (tx 64/128/256, sy >= 8); changes no result bit. */
lbm_status lbm_batch_set_tile(lbm_batch* b, int32_t tx, int32_t sy);
lbm_status lbm_batch_get_tile(const lbm_batch* b, int32_t* tx, int32_t* sy);

/* As lbm_set_scheme, for every instance; only before the first step (the
 * tau of the batch decides LBM_SCHEME_AUTO). */
lbm_status lbm_batch_set_scheme(lbm_batch* b, int32_t scheme);

/* chunk > 0: lbm_batch_step replays a HIP graph of `chunk` captured steps
 * (captured at first use) and launches the remainder directly; 0: direct. */
lbm_status lbm_batch_set_graph(lbm_batch* b, int32_t chunk);

/* Queue nsteps steps of every instance (asynchronous). */
lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps);

/* Queue: front position of every instance into column `slot` of the table
 * (NaN for instances with W == 0).  lbm_batch_fronts copies the n x nslots
 * table (row-major) to the host and synchronises. */
lbm_status lbm_batch_record_fronts(lbm_batch* b, int32_t slot);
lbm_status lbm_batch_fronts(lbm_batch* b, double* host);

/* Per-instance observables, fields and growth events (as the single-lattice
 * calls; synchronise). */
lbm_status lbm_batch_observe(lbm_batch* b, int32_t i, lbm_obs* out);
lbm_status lbm_batch_fields(lbm_batch* b, int32_t i, uint32_t field_mask, double* host_fields);
lbm_status lbm_batch_events(lbm_batch* b, int32_t i, int64_t first, lbm_event* buf, int64_t cap,
                            int64_t* n);

/* Before the first step only: time the launch shapes, time the three
 * fastest again (interleaved, three times over at least 5 ms each), keep the
 * lowest median and reset every instance to its initial state. */
lbm_status lbm_batch_autotune(lbm_batch* b, int32_t steps, int32_t* tx, int32_t* sy,
                              double* best_ms_per_step);

void lbm_batch_destroy(lbm_batch* b);

/* ------------------------------------------------------------------------
 * Learned surrogate of the sweep: an MLP 5 -> 256 -> 256 -> 256 -> 65 (ReLU)
 * mapping capillary width W, length L, reaction rate k_r, contact angle
 * (degrees) and precipitation threshold to 65 outputs, which the sweep
 * pipeline trains as the centreline front z(t_j) at the 64 sample times
 * t_j = ceil(j T / 64), divided by a Washburn travel scale, and the
 * pore-closure time / T (1 if no closure within T).  Inputs are normalised inside the library to [-1, 1]
 * over the box [lo, hi] (log10 for k_r).  Dense layers run on the matrix cores
 * (BF16 operands, FP32 accumulation) in forward and backward; training keeps
 * FP32 master weights and uses Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the
 * weighted mean-squared error.  Parameters are exchanged packed in FP32:
 * W1 [256 x 5] row-major, b1 [256], W2 [256 x 256], b2, W3 [256 x 256], b3,
 * W4 [65 x 256], b4 [65] (149,825 values).  The outputs are only meaningful
 * inside the training box; callers check their queries against it and run
 * the lattice Boltzmann model (lbm_batch_*) for the rest.
 * ------------------------------------------------------------------------ */
typedef struct surr_net surr_net;

/* Workspace for minibatches / prediction chunks of up to max_batch rows and a
 * resident training set of up to max_data samples. */
lbm_status surr_workspace_bytes(int32_t max_batch, int32_t max_data, size_t* bytes);
lbm_status surr_init(const double* lo, const double* hi, int32_t max_batch, int32_t max_data,
                     void* stream, void* workspace, size_t ws_bytes, surr_net** out);
/* Parameters (packed layout above); setting them clears the Adam state. */
lbm_status surr_set_params(surr_net* s, const float* packed);
lbm_status surr_get_params(surr_net* s, float* packed);
/* Per-output weights of the loss (65 values, >= 0; default 1). */
lbm_status surr_set_loss_weights(surr_net* s, const float* w);
/* Training set x [n x 5] (raw inputs), y [n x 65] (targets) and optional
 * per-sample loss weights row_w [n] (NULL: all 1), copied to HBM.  The loss of
 * a minibatch is sum_rows row_w sum_j w_j (y - t)^2 / (rows * sum_j w_j). */
lbm_status surr_set_data(surr_net* s, const float* x, const float* y, const float* row_w, int32_t n);
/* One epoch over the resident set in the order perm (host, n indices):
 * minibatches of `batch` rows, one Adam step each.  *mean_loss: mean of the
 * minibatch losses (the only device-to-host transfer). */
lbm_status surr_train_epoch(surr_net* s, const int32_t* perm, int32_t batch, float lr,
                            double* mean_loss);
/* Loss and packed parameter gradients for one batch (n <= max_batch), no update. */
lbm_status surr_gradients(surr_net* s, const float* x, const float* y, int32_t n, float* grad,
                          double* loss);
/* y [n x 65] for x [n x 5] (host arrays). */
lbm_status surr_predict(surr_net* s, const float* x, int32_t n, float* y);
/* For callers that cannot allocate device memory or synchronise (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same prediction as surr_predict, with x [n x 5] and y [n x 65] FP32 arrays
 * in device memory, queued on `stream` (whose device must be current) without
 * waiting for it.  The activations live in a static array of the library
 * (3.2 MB per GPU, held until the process ends), so n is 1..1024 per call
 * (more is LBM_EINVAL) and no memory is allocated.  Every call on one GPU
 * uses the same array: calls that overlap on a GPU (concurrent streams or
 * threads) race and must be ordered by the caller.  The handle is only read;
 * it must not be trained concurrently. */
lbm_status surr_predict_noalloc(const surr_net* s, const float* x, int32_t n, float* y,
                                void* stream);
void surr_destroy(surr_net* s);

void lbm_destroy(lbm_sim* sim);
const char* lbm_strerror(lbm_status s);
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
