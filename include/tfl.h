/*
 * tfl.h -- C ABI of the two-fluid (Maxwell + London) FDTD library for AMD
 * MI355X (gfx950).
 *
 * The method (arXiv 2305.13419, Sec. 2 and Sec. 3, Algorithm 1): Maxwell's
 * equations on a Yee grid (Sec. 3) with the total current J = sigma E + Js
 * (Sec. 2), where the supercurrent obeys the first London equation
 * dJs/dt = E / (lambda_L^2 mu0) (Eq. London1a), advanced by the explicit
 * leap-frog of Algorithm 1 with the theta-weighted Ohmic term (Algorithm 1,
 * step 3).  The library keeps the staggered state (E^n, H^{n-1/2}, Js^{n-1/2})
 * and applies Algorithm 1's split half steps of B and Js only where
 * integer-time values are set or read (tfl_set_initial_integer_time,
 * tfl_sync_integer_time); one tfl_step is analytically the same as the five
 * sub-steps of Algorithm 1.
 *
 * Conventions shared by every entry point
 *  - Every call returns an int: TFL_OK (0) or a negative TFL_E_* code.  The
 *    message of the last failure on a handle is returned by tfl_last_error()
 *    and stays valid until the next call on that handle; failures of
 *    tfl_create are reported by tfl_last_error(NULL).  Handles are not thread
 *    safe: one host thread per handle at a time.
 *  - Units are SI.  Fields: E in V/m, H in A/m, Js in A/m^2.  Maps: eps_r
 *    (dimensionless, > 0), sigma_n in S/m (>= 0), inv_lambda2 = 1/lambda_L^2
 *    in m^-2 (>= 0; 0 marks a non-superconducting cell, Sec. 3).
 *  - Layout: every grid array is one component, nz x ny x nx, x fastest,
 *    contiguous, element index (k*ny + j)*nx + i, in the precision chosen by
 *    tfl_config.dtype (double for TFL_F64, float for TFL_F32).  Component c of
 *    E and Js at index (i,j,k) lives on the edge along axis c through node
 *    (i,j,k) (Ex at (i+1/2, j, k), Ey at (i, j+1/2, k), Ez at (i, j, k+1/2));
 *    component c of H lives on the face normal to axis c (Hx at
 *    (i, j+1/2, k+1/2), Hy at (i+1/2, j, k+1/2), Hz at (i+1/2, j+1/2, k)).
 *    Material maps are per cell (i,j,k), the cell [i,i+1]x[j,j+1]x[k,k+1].
 *    Indices wrap on every axis.
 *  - Ownership: the library never allocates device memory.  All device
 *    buffers (fields, maps, workspace, probe outputs, checkpoints, gradients)
 *    belong to the caller, are passed as raw device pointers, must be
 *    256-byte aligned, and must stay alive until tfl_destroy or a re-bind.
 *    Host structs and arrays passed in are copied during the call.
 *  - Streams: every call that touches the device takes a hipStream_t passed
 *    as void* (NULL = the null stream).  Calls are asynchronous on that
 *    stream except those documented to return host values, which
 *    synchronise it.
 *  - No exception crosses the ABI.
 */
#ifndef TFL_H
#define TFL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tfl_sim tfl_sim;

enum {
    TFL_OK = 0,
    TFL_E_INVAL = -1,     /* bad argument (size, pointer, value)              */
    TFL_E_STATE = -2,     /* wrong call order or buffers not bound            */
    TFL_E_UNSTABLE = -3,  /* dt above the stability bound of the scheme       */
    TFL_E_NONFINITE = -4, /* NaN or Inf found in the state                     */
    TFL_E_DEVICE = -5,    /* a HIP runtime error; the message names it        */
    TFL_E_NOMEM = -6,     /* a caller buffer is smaller than required          */
    TFL_E_RANGE = -7      /* more distinct values than a compact table holds   */
};

enum { TFL_F64 = 0, TFL_F32 = 1 };
enum { TFL_PERIODIC = 0, TFL_CPML = 1 };
enum { TFL_WAVE_SIN = 0, TFL_WAVE_GAUSS = 1, TFL_WAVE_MOD_GAUSS = 2 };

#define TFL_MAX_SOURCES 32
#define TFL_MAX_PROBES 32
#define TFL_MAX_FREQS 16

/* Problem statement (Sec. 3): grid, spacing, time step, theta of Algorithm 1
 * step 3, storage precision and boundaries.
 *  bc[a]       TFL_PERIODIC or TFL_CPML for axis a (x, y, z).  A CPML axis
 *              has a PEC wall on node plane 0 (tangential E held at 0), which
 *              both of its absorbing slabs back onto through the index wrap;
 *              with zero slab cells it is a bare PEC wall (Sec. 3 lists
 *              periodic, PEC and PML boundaries).
 *  pml_lo[a], pml_hi[a]  absorbing cells at the low and high end of a CPML axis.
 *  pml_order, pml_scale, kappa_max, alpha_max  grading of the convolutional
 *              PML (Roden and Gedney 2000): sigma(d) = pml_scale *
 *              0.8 (m+1)/(eta0 dx) * d^m, kappa(d) = 1 + (kappa_max-1) d^m,
 *              alpha(d) = alpha_max (1-d), d in [0,1] the normalised depth. */
typedef struct {
    int64_t nx, ny, nz;
    double dx, dy, dz;
    double dt;
    double theta;        /* in [0.5, 1]; 1 = backward Euler, 0.5 = centred     */
    int32_t dtype;       /* TFL_F64 or TFL_F32                                */
    int32_t bc[3];
    int32_t pml_lo[3], pml_hi[3];
    double pml_order, pml_scale, kappa_max, alpha_max;
} tfl_config;

/* Additive ("soft") E source (Sec. 4.1, 4.2, 5): after the E update of step
 * n -> n+1, E_comp += amplitude * g(t_{n+1}) on every edge of the half-open
 * index box [i0,i1) x [j0,j1) x [k0,k1), t_{n+1} = (n+1) dt, with
 * g = sin(2 pi freq t), exp(-(t-t0)^2/(2 tw^2)), or their product. */
typedef struct {
    int32_t comp;        /* 0,1,2 = Ex, Ey, Ez                                */
    int64_t box[6];      /* i0, i1, j0, j1, k0, k1                            */
    double amplitude;
    int32_t waveform;    /* TFL_WAVE_*                                        */
    double freq, t0, tw;
} tfl_source;

/* Field probe (Sec. 4.2, Sec. 5): s_n = sum of E_comp over the index box at
 * time level n, accumulated in FP64.  series[n] = s_n for n < capacity (the
 * sample at the step index where tfl_step first runs, normally n = 0, is
 * taken then).  For each frequency f_q the running DFT
 * F_q += s_n * dt * exp(-i 2 pi f_q n dt) is kept in dft[2q], dft[2q+1]
 * (real, imaginary).  series and dft are caller-owned device FP64 buffers;
 * either may be NULL when capacity or nfreq is 0.  Calls never read them
 * back: the caller clears them before a run. */
typedef struct {
    int32_t comp;
    int64_t box[6];
    double *series;      /* device, FP64 [capacity]                           */
    int64_t capacity;
    int32_t nfreq;       /* <= TFL_MAX_FREQS                                  */
    const double *freqs; /* host, [nfreq], copied                             */
    double *dft;         /* device, FP64 [2*nfreq]                            */
} tfl_probe;

/* Create a handle; validates sizes (>= 1, nx * ny <= 2^29 so that one x-y
 * plane is addressed with 32-bit byte offsets), spacings and dt (> 0), theta
 * in [0.5, 1], dtype, bc and PML cell counts (lo + hi <= n on a CPML axis).
 * TFL_E_INVAL on bad values. */
int tfl_create(const tfl_config *cfg, tfl_sim **out);
int tfl_destroy(tfl_sim *sim);
const char *tfl_last_error(const tfl_sim *sim);

/* Byte sizes of the caller-owned buffers: the workspace (CPML coefficient
 * tables and auxiliary variables; 0 when no axis is CPML), a scratch buffer
 * (1 MiB: reductions, probe descriptors, and the copies of the probe boxes
 * that the sweeps hand to the next sweep), and one saved state (E, H, Js and
 * the workspace). */
int tfl_buffer_sizes(const tfl_sim *sim, size_t *workspace_bytes, size_t *scratch_bytes, size_t *state_bytes);

/* Bind the nine state arrays (device, dtype, N elements each). */
int tfl_bind_state(tfl_sim *sim, void *const E[3], void *const H[3], void *const J[3]);

/* Bind the workspace and scratch buffers (sizes from tfl_buffer_sizes).
 * Uploads the CPML tables and clears the auxiliary variables on `stream`.
 * workspace may be NULL when its size is 0. */
int tfl_bind_workspace(tfl_sim *sim, void *workspace, void *scratch, void *stream);

/* Optional second set of E, H and Js fields for the fused sweeps.
 * tfl_fused_buffer_bytes reports its size: 9 fields (E, H, Js), each padded
 * to 256 bytes, then on each CPML axis a second set of its four auxiliary
 * variables (two H-side, two E-side; 4 x the slab cells of the axis, padded
 * to 256 bytes).  With a buffer bound, tfl_step runs H and E updates of a step
 * in one sweep (Algorithm 1, steps 1-5 of a time step fused): it reads E^n,
 * H^{n-1/2} (and the H-side CPML variables) from one set and writes E^{n+1},
 * H^{n+1/2} (and the new variables) to the other, recomputing the few H values
 * a cell needs from its x-1 and y-1 neighbours, so each cell's fields cross
 * HBM once per step instead of twice; results equal those of the two passes
 * bit for bit.  Steps run in pairs (bound fields -> buffer -> bound fields),
 * an odd last step with the two passes, so the state is in the bound fields
 * and the workspace after every call.  With edge classes bound, stretches of
 * at least four steps with no non-finite checks and no probe launches (soft
 * sources are added inside the sweep to both steps' E, and folded probes copy
 * both steps' E) can run two time steps per sweep (temporal blocking): each
 * sweep reads E^n, H^{n-1/2}, Js^{n-1/2} (and all CPML variables) from one set
 * and writes E^{n+2}, H^{n+3/2}, Js^{n+3/2} (and the variables) to the other,
 * so per step each cell's fields cross HBM half as often; the results again
 * equal those of the two passes bit for bit.  The buffer is caller-owned
 * device memory, 256-byte aligned, holding nothing between calls; bind NULL
 * to go back to the two passes.  TFL_E_INVAL on a misaligned buffer. */
int tfl_fused_buffer_bytes(const tfl_sim *sim, size_t *bytes);
int tfl_bind_fused_buffer(tfl_sim *sim, void *buffer);

/* Which sweeps a step may take (the results are the same bits on every path).
 *  TFL_SWEEP_AUTO      (default) the two-step sweep where it applies and pays
 *                      (grids of at least 3 * 2^20 cells, past the GPU's
 *                      infinity cache, nx >= 64, ny >= 32, nz >= 16; on
 *                      CPML grids in FP64, and in FP32 where rows of 64
 *                      cells leave a fifth of their lanes idle), else the
 *                      fused sweep where a buffer is bound, else the two
 *                      passes;
 *  TFL_SWEEP_TWO_PASS  always the H and E passes;
 *  TFL_SWEEP_FUSED     the fused sweep wherever a buffer is bound, no
 *                      two-step sweep;
 *  TFL_SWEEP_TWO_STEP  the two-step sweep wherever it applies (edge
 *                      classes bound, buffer bound, no checks, probes
 *                      folded with two steps' copies in a half of the copy
 *                      space, stretches of four steps), whatever the size;
 *                      the fused sweep elsewhere.
 * tfl_sweep_counts: steps the last tfl_step call ran on the two passes, the
 * fused sweep and the two-step sweep (counts[0..2]).  TFL_E_INVAL on a bad
 * value. */
enum { TFL_SWEEP_AUTO = 0, TFL_SWEEP_TWO_PASS = 1, TFL_SWEEP_FUSED = 2, TFL_SWEEP_TWO_STEP = 3 };
int tfl_set_sweep(tfl_sim *sim, int32_t sweep);
int tfl_sweep_counts(const tfl_sim *sim, int64_t counts[3]);

/* Bind the per-cell maps (device, dtype, N elements each).  Validates them
 * on the device (eps_r > 0, sigma >= 0, inv_lambda2 >= 0, all finite) and
 * checks dt against the stability bound of the scheme with the London term,
 * dt_max = 2 / (c0 sqrt(4/dx^2 + 4/dy^2 + 4/dz^2 + max inv_lambda2))
 * (from the single-mode amplification matrix of Algorithm 1 with eps_r = 1).
 * Synchronises `stream`.  TFL_E_INVAL on bad values, TFL_E_UNSTABLE when
 * dt > dt_max.  The per-edge material is formed inside the kernels: an edge
 * is superconducting when any of the four cells sharing it is (Sec. 3) and
 * then takes the mean of (eps_r, sigma, inv_lambda2) over those cells;
 * otherwise it takes the mean of (eps_r, sigma) over all four. */
int tfl_bind_materials(tfl_sim *sim, const void *eps_r, const void *sigma_n, const void *inv_lambda2, void *stream);

/* Edge-coefficient classes (optional; forward and adjoint sweeps).  The E update of
 * an edge uses three coefficients fixed by the four cells sharing it (Sec. 3
 * edge rule, Algorithm 1 step 3): E^{n+1} = ca E^n + cb (curl H - Js^{n+1/2}),
 * Js^{n+1/2} = Js^{n-1/2} + cj E^n.  When the grid holds few distinct
 * materials, tfl_bind_edge_classes replaces the three per-cell maps read by
 * the E update with one 16-bit class per edge and a table of (ca, cb, cj):
 * 6 bytes per cell instead of 3 x sizeof(dtype) plus neighbour reads.  The
 * table entries are computed on the device by the same code as the per-edge
 * coefficients of the map path, so results are bit-identical.
 *
 * buffer: caller-owned device memory of tfl_edge_class_bytes bytes, 256-byte
 * aligned; holds, in this order, the classes of the x, y and z edges (N
 * uint16 each, each array padded to 256 bytes), the table
 * (TFL_MAX_EDGE_CLASSES entries of 4 dtype values: ca, cb, cj, 0) and the
 * staging area the table is built from.  The classes are a snapshot of the
 * maps bound when the call is made: tfl_bind_materials unbinds them, so after
 * binding (or changing) the maps, bind the classes again.  Builds on the host
 * (the maps are copied to host memory) and synchronises `stream`.
 * *nclasses (may be NULL) receives the number of classes.  TFL_E_RANGE, with
 * the simulation left on the map path, when the grid has more than 65536
 * distinct cell materials or more than TFL_MAX_EDGE_CLASSES distinct edge
 * materials; TFL_E_STATE without bound maps.  A NULL buffer unbinds.  With
 * classes bound, the adjoint's edge sweep reads them as well (the same
 * coefficients); the adjoint's gather of per-edge gradients onto cells and the
 * integer-time half kicks read the maps. */
#define TFL_MAX_EDGE_CLASSES 65535
int tfl_edge_class_bytes(const tfl_sim *sim, size_t *bytes);
int tfl_bind_edge_classes(tfl_sim *sim, void *buffer, int *nclasses, void *stream);

/* The bound H and Js hold integer-time values H^0, Js^0 (E holds E^0):
 * replace them with H^{-1/2} and Js^{-1/2} by running the first half
 * updates of Algorithm 1 (steps 1 and 2) backwards, and reset the step
 * index to 0 and the CPML auxiliary variables to 0. */
int tfl_set_initial_integer_time(tfl_sim *sim, void *stream);

/* Register a source or a probe; *id receives its index.  Boxes must lie in
 * the grid; at most TFL_MAX_SOURCES / TFL_MAX_PROBES per handle. */
int tfl_add_source(tfl_sim *sim, const tfl_source *src, int *id);
int tfl_add_probe(tfl_sim *sim, const tfl_probe *probe, int *id);
int tfl_clear_sources_probes(tfl_sim *sim);

/* Advance nsteps >= 0 time steps (Algorithm 1), with sources and probes.
 * The sources are added inside the sweep that updates E.  With at most four
 * probes whose boxes fit the scratch copy space (448 KiB per copy: e.g. 57344
 * FP64 values over all boxes), each sweep also copies the new E on the boxes to
 * scratch and the next sweep sums the copies of the previous one (one probe
 * launch after the call's last step sums the last copies), so a step is one
 * launch; otherwise a probe launch follows every step.  A two-step sweep
 * copies both of its steps' E, each to a quarter of the space (224 KiB), and
 * the next sweep records both samples in order; probes whose copies exceed a
 * quarter keep the one-step sweeps.  The sums are formed in the same order
 * every way. */
int tfl_step(tfl_sim *sim, int64_t nsteps, void *stream);

/* Optional non-finite check (a guard for long runs; off by default).  With
 * every > 0, each step of tfl_step and tfl_forward_checkpointed whose new step
 * index is a multiple of `every` is followed by a device count of the NaN and
 * Inf values in E, H and Js.  A call during which a check ran reads the counts
 * back at its end, synchronising `stream`, and returns TFL_E_NONFINITE (the
 * message gives the count and the first step index where one was seen) if any
 * was found; all nsteps steps are still taken, and a checkpointed run that
 * fails the check leaves no run for tfl_adjoint.  every = 0 turns the check
 * off.  TFL_E_INVAL when every < 0.  The counters live in the scratch buffer.
 * (Stability is otherwise guarded by the dt bound of tfl_bind_materials.) */
int tfl_set_nonfinite_check(tfl_sim *sim, int64_t every);

/* tfl_step with HIP events recorded on `stream` at the start of every step and
 * after its first launch; returns the summed device time of the first launches
 * (the H pass of the two passes, the whole fused sweep) and of the rest of the
 * steps (the E pass, probe launches) in milliseconds.  Synchronises `stream`.
 * For measurement only. */
int tfl_profile_step(tfl_sim *sim, int64_t nsteps, void *stream, double *h_ms, double *e_ms);

/* Integer-time values at the current step n (Algorithm 1 steps 1 and 2 of
 * the next step read as the end of this one): H^n = H^{n-1/2} - dt/(2 mu0)
 * curl E^n and Js^n = Js^{n-1/2} + dt/2 inv_lambda2 E^n / mu0 on
 * superconducting edges (0 elsewhere), written to caller buffers (device,
 * dtype, N elements each; Hn or Jn may be NULL to skip).  The state is not
 * modified. */
int tfl_sync_integer_time(tfl_sim *sim, void *const Hn[3], void *const Jn[3], void *stream);

/* Discrete energy W^n = dV [sum_e eps_e E_e^2/2 + sum_f mu0 H^{n-1/2}_f H^{n+1/2}_f/2
 * + sum_{SC e} mu0 Js^{n-1/2}_e Js^{n+1/2}_e/(2 inv_lambda2_e)] in FP64 (the
 * quantity the lossless leap-frog conserves exactly on periodic grids;
 * H^{n+1/2}, Js^{n+1/2} formed on the fly without PML stretching), and the
 * number of non-finite values in E, H and Js.  Synchronises `stream`. */
int tfl_energy(tfl_sim *sim, double *energy, int64_t *nonfinite, void *stream);

/* Allocation-free variant of tfl_energy, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same two results, written to the caller's device buffer
 * out (FP64 [2]: out[0] = W^n, out[1] = the non-finite count as a double),
 * asynchronously on `stream` (no host copy, no synchronisation).  The block
 * partials of the reduction live in a fixed device array of the library
 * (2 x 1024 doubles, 16 KiB, one copy per GPU, held until the process ends)
 * instead of the bound scratch buffer; the call allocates nothing.  Every
 * block writes its partial before the final fold reads it, so nothing of a
 * previous call is read.  All calls on one GPU share that array: calls that
 * overlap in time on one GPU (two streams, or two host threads) race and may
 * return wrong values.  Results are bitwise those of tfl_energy.  Needs bound
 * state and materials (no bound workspace is read).  TFL_E_INVAL on a null or
 * misaligned out, TFL_E_NOMEM if a reduction would need more partials than
 * the array holds (no grid does: the count is fixed). */
int tfl_energy_noalloc(tfl_sim *sim, double *out, void *stream);

/* Step index n (the state is at E^n) and its override (for restarts). */
int tfl_get_step(const tfl_sim *sim, int64_t *step);
int tfl_set_step(tfl_sim *sim, int64_t step);

/* Copy the state (E, H, Js, workspace) to / from a caller device buffer of
 * state_bytes (tfl_buffer_sizes).  The step index is not part of the copy. */
int tfl_save_state(tfl_sim *sim, void *dst, void *stream);
int tfl_load_state(tfl_sim *sim, const void *src, void *stream);

/* ----------------------------------------------------------------------
 * Gradients by the adjoint (reverse-time) method
 *
 * Objective: J = |F|^2 with F = sum_{n=n0}^{n0+N} dt exp(-i 2 pi f0 n dt) s_n,
 * s_n the sum of E_comp over the index box at time level n (the probe of
 * Sec. 4.2 and Sec. 5 with a single DFT frequency), n0 the step index where
 * the run starts and N its number of steps.  Gradients are taken with respect
 * to the per-cell maps inv_lambda2 and sigma_n, holding fixed which edges are
 * superconducting: an edge's value is the mean over its superconducting
 * cells (weight 1/|S| each) or over all four cells (sigma of a normal edge,
 * weight 1/4); cells with inv_lambda2 = 0 receive no inv_lambda2 gradient.
 * The forward run is checkpointed every `seg` steps (sqrt(N) memory); the
 * reverse sweep recomputes one segment at a time, storing E after every
 * step, and runs the transposed leap-frog with FP64 gradient accumulation.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t comp;
    int64_t box[6];
    double f0;
} tfl_objective;

/* Byte sizes of the caller-owned buffers for a run of nsteps with segments
 * of seg steps: checkpoints (ceil(nsteps/seg) saved states), E snapshots
 * (two sets of seg + 1: one segment is recomputed into one set while the
 * adjoint sweeps of the next read the other) and the adjoint workspace
 * (adjoint fields, eight steps of mu, PML adjoint variables, FP64 per-edge
 * gradient accumulators). */
int tfl_adjoint_sizes(const tfl_sim *sim, int64_t nsteps, int64_t seg, size_t *ckpt_bytes, size_t *snap_bytes,
                      size_t *adj_bytes);

/* nsteps >= 1 forward steps from the current state, as tfl_step (sources and
 * probes included), saving the state at the start of every segment into
 * ckpt (segment g at byte offset g * state_bytes) and accumulating F in
 * FP64.  F[0], F[1] receive Re F, Im F on the host; synchronises `stream`. */
int tfl_forward_checkpointed(tfl_sim *sim, const tfl_objective *obj, int64_t nsteps, int64_t seg, void *ckpt,
                             double F[2], void *stream);

/* Reverse sweep of the last tfl_forward_checkpointed run (same obj, nsteps,
 * seg and ckpt; F as returned by it).  Writes dJ/d inv_lambda2 and
 * dJ/d sigma_n per cell to grad_ell and grad_sigma (device FP64, N each).
 * snap and adj are device buffers of snap_bytes and adj_bytes.  Probes are
 * not sampled during the recomputation, which runs the fused sweep when a
 * fused buffer is bound (as tfl_step; same results), on a second stream the
 * call creates and destroys (each segment's recomputation overlaps the adjoint
 * sweeps of the segment after it); all work is ordered before the end of the
 * call's work on `stream`.  On return the state
 * arrays (and the fused buffer) hold intermediate values of the
 * recomputation: load a saved state (and set the step index) before stepping
 * again.  TFL_E_STATE if no matching forward run exists: none was made, it had
 * another nsteps, seg or objective, or the maps (tfl_bind_materials) or the
 * sources (tfl_add_source, tfl_clear_sources_probes) changed after it, since the
 * recomputation would then not reproduce the run whose checkpoints are stored. */
int tfl_adjoint(tfl_sim *sim, const tfl_objective *obj, int64_t nsteps, int64_t seg, const void *ckpt,
                const double F[2], void *snap, void *adj, double *grad_ell, double *grad_sigma, void *stream);

/* ----------------------------------------------------------------------
 * Resonance frequency and quality factor from a ringdown (Sec. 5, Table 7)
 *
 * The paper extracts f and Q from probe time series with ESPRIT, which
 * tfl_esprit_fit below implements.  tfl_ringdown_fit is a second, independent
 * estimator, a linear predictor (Prony's method): the series
 * x_m = series[start + m*decim], m = 0 .. count-1, is modelled as
 * x_m = sum_{k=1}^{P} a_k x_{m-k}; the GPU forms the FP64 normal equations
 * (Gram matrix of the lagged samples) and the host solves the P x P system
 * (refined twice with the residual correction formed on the device) and finds
 * the roots z of z^P - a_1 z^{P-1} - ... - a_P.  Each root gives a mode
 * z = exp((-alpha + i 2 pi f) decim dt); the modes' complex amplitudes follow
 * from a least-squares fit of the window; Q = pi f / alpha.
 * ---------------------------------------------------------------------- */
#define TFL_FIT_MAX_ORDER 16

typedef struct {
    int64_t start, count, decim;  /* window of the probe series and decimation  */
    int32_t order;                /* P <= TFL_FIT_MAX_ORDER; 0: the numerical rank of
                                     the order-16 normal matrix (eigenvalues above
                                     1e-8 of the largest), at least 2             */
    double f_hint;                /* report the largest-amplitude mode with f in
                                     [0.5, 1.5] f_hint (Hz); <= 0 or none there:
                                     the largest-amplitude mode with f > 0        */
} tfl_fit_req;

typedef struct {
    double f0, alpha, Q;          /* Hz, 1/s, pi f0 / alpha                         */
    double residual;              /* prediction residual energy / signal energy     */
    int32_t order;                /* order used                                      */
    int32_t nmodes;               /* roots found                                     */
    double modes[2 * TFL_FIT_MAX_ORDER]; /* (f_m, alpha_m) of every root              */
} tfl_fit_result;

/* Fit the series of probe `probe_id` (its FP64 device buffer).  Requires
 * count > order and start + (count-1)*decim < capacity.  Synchronises
 * `stream`.  TFL_E_INVAL on bad windows, TFL_E_NONFINITE if the normal
 * equations are singular or the root iteration does not converge. */
int tfl_ringdown_fit(tfl_sim *sim, int probe_id, const tfl_fit_req *req, tfl_fit_result *out, void *stream);

/* ESPRIT, the paper's own f / Q extraction (Sec. 5, Table 7; Roy and Kailath's
 * estimation of signal parameters via rotational invariance, least-squares
 * form).  The window x_m of req (start, count, decim) is taken as a sum of
 * damped complex exponentials c_q z_q^m.  With the Hankel matrix H[r][a] =
 * x_{r+a} of `pencil` columns, the GPU forms the FP64 Gram matrix H^T H; the
 * host takes its eigenvectors of the req->order largest eigenvalues as the
 * signal subspace V_s (pencil x P), solves V_s[1:] = V_s[:-1] Phi by least
 * squares, and the eigenvalues of Phi (Hessenberg QR) are the modes
 * z = exp((-alpha + i 2 pi f) decim dt).  Amplitudes and the reported mode
 * (f_hint rule) as for tfl_ringdown_fit; a real damped cosine gives a
 * conjugate pair, so P = 2 per mode.
 *   req->order: P <= min(TFL_FIT_MAX_ORDER, pencil - 1); 0: the numerical rank
 *               of H^T H (eigenvalues above 1e-8 of the largest), at least 2.
 *   pencil:     3 .. TFL_ESPRIT_MAX_PENCIL, at most count / 2; 0: min(64, count / 3).
 *   out->residual: fraction of the trace of H^T H outside the signal subspace.
 * Synchronises `stream`.  TFL_E_INVAL on bad windows or sizes, TFL_E_NONFINITE
 * if the Gram matrix is zero or an iteration does not converge. */
#define TFL_ESPRIT_MAX_PENCIL 64
int tfl_esprit_fit(tfl_sim *sim, int probe_id, const tfl_fit_req *req, int32_t pencil, tfl_fit_result *out,
                   void *stream);

/* Three-level variant for runs whose two-level schedule does not fit in
 * memory: after the same tfl_forward_checkpointed run (checkpoints every seg
 * steps), each outer segment is recomputed saving inner checkpoints every
 * seg2 steps (1 <= seg2 <= seg) into ckpt2, and each inner segment is
 * recomputed into the snapshots and swept backwards.  Sizes from
 * tfl_adjoint_nested_sizes (ckpt2 holds ceil(seg/seg2) states, snap seg2 + 1
 * E fields).  Same results, outputs and errors as tfl_adjoint. */
int tfl_adjoint_nested_sizes(const tfl_sim *sim, int64_t nsteps, int64_t seg, int64_t seg2, size_t *ckpt_bytes,
                             size_t *ckpt2_bytes, size_t *snap_bytes, size_t *adj_bytes);
int tfl_adjoint_nested(tfl_sim *sim, const tfl_objective *obj, int64_t nsteps, int64_t seg, const void *ckpt,
                       const double F[2], int64_t seg2, void *ckpt2, void *snap, void *adj, double *grad_ell,
                       double *grad_sigma, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TFL_H */
