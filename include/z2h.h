/*
 * z2h -- Trotterized adiabatic state-vector evolution of the toric code in two
 * transverse fields (the Z2 gauge-Higgs model in its mapped form) on one
 * MI355X (gfx950) GPU.
 *
 * Model (Sec. II, Eq. (effi), with the star and plaquette couplings made
 * parameters):
 *     H(c) = -JA sum_v A_v - JB sum_p B_p - hx sum_l X_l - hz sum_l Z_l
 * on the n = 2*Lx*Ly link qubits of a periodic Lx x Ly lattice.  The paper's
 * point (g, lambda) with J = h = 1/2 is c = (1/2, 1/2, g, lambda).
 *
 * Method (Sec. III): an adiabatic ramp c(s) = (1-s) c_start + s c_end in M
 * steps of equal duration dt, each a second-order Trotter-Suzuki step
 * exp(-iH1 dt/2) exp(-iH2 dt/2) exp(-iH3 dt) exp(-iH2 dt/2) exp(-iH1 dt/2).
 * Because every summand inside each factor commutes (Eq. (decom)), the step
 * equals exp(-iHX dt/2) exp(-iHZ dt) exp(-iHX dt/2) with HX = star + x-field
 * terms and HZ = plaquette + z-field terms; the library applies HZ as one
 * diagonal phase in the computational basis and HX as one diagonal phase in
 * the Hadamard basis reached by an in-place Walsh-Hadamard transform.
 *
 * Conventions
 *   - Link numbering (library): h(x,y) = link from vertex (x,y) to (x+1,y),
 *     bit y*Lx + x; v(x,y) = link from (x,y) to (x,y+1), bit Lx*Ly + y*Lx + x.
 *     Star A(x,y) = X on {h(x,y), h(x-1,y), v(x,y), v(x,y-1)}; plaquette
 *     B(x,y) = Z on {h(x,y), h(x,y+1), v(x,y), v(x+1,y)}.  z2h_link_bit()
 *     gives the map; observables do not depend on it.
 *   - Bit l of a basis index = 0 means sigma^z_l = +1.
 *   - A state is 2^n interleaved complex numbers (re, im), complex64
 *     (2 x float) or complex128 (2 x double), in device memory.
 *
 * Ownership: the caller owns every device buffer (state, workspace, outputs)
 * and the stream; the library only borrows them for the call.  A plan or a
 * batch owns its small device tables and frees them in *_destroy.  After
 * creation no call allocates device memory.
 *
 * Errors: every function returns a z2h_status and never aborts.  Arguments
 * are validated before anything is enqueued; on error nothing is enqueued
 * and z2h_last_error() describes the problem.  Device work is asynchronous
 * on the given stream; functions with host outputs synchronize that stream
 * and report earlier device failures as Z2H_ERR_HIP.
 */
#ifndef Z2H_H
#define Z2H_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t z2h_status;
#define Z2H_OK 0
#define Z2H_ERR_INVALID (-1)     /* bad argument (null pointer, size, range) */
#define Z2H_ERR_UNSUPPORTED (-2) /* valid but not supported (n > 32, ...) */
#define Z2H_ERR_OOM (-3)         /* host or device allocation failed at creation */
#define Z2H_ERR_HIP (-4)         /* HIP runtime error, or no usable device */
#define Z2H_ERR_NUMERIC (-5)     /* non-finite norm or energy */
#define Z2H_ERR_WORKSPACE (-6)   /* workspace smaller than required */

typedef int32_t z2h_dtype;
#define Z2H_C64 0  /* complex64: FP32 butterflies, FP64 angles and reductions */
#define Z2H_C128 1 /* complex128 */

typedef int32_t z2h_init;
#define Z2H_INIT_PSI1 0  /* Eq. (ini1): all plaquettes even, equal weights */
#define Z2H_INIT_PSI1P 1 /* Eq. (ini2): all stars +1 (projected |0...0>) */
#define Z2H_INIT_ZERO 2  /* |0...0> */
#define Z2H_INIT_PLUS 3  /* |+...+> */

typedef struct {
    double JA, JB, hx, hz; /* H = -JA sum A - JB sum B - hx sum X - hz sum Z */
} z2h_couplings;

/*
 * Schedule of an adiabatic ramp (Sec. III): M = steps steps of duration dt.
 * Step k uses c(s) = (1-s) start + s end with s = s_k:
 *   sampling 0: s_k = (k + 1/2)/M (midpoint), 1: s_k = (k + 1)/M (the
 *   paper's g = k*dg, Appendix Eq. (target)).
 * If sZ / sX are non-NULL (host arrays of length steps) they replace s_k for
 * the z-type couplings (JB, hz) and the x-type couplings (JA, hx) of each
 * step; these are the "schedule angles" the adjoint differentiates.
 * Only steps k_begin <= k < k_end are applied (0, steps: the whole ramp), so
 * a ramp can be split across calls and resumed from a saved state.
 * order 0: x-z-x step (the paper's); 1: z-x-z (used by duality checks).
 * renorm 1: rescale the state to unit norm once per step (from the norm
 * measured during the previous diagonal pass); 0: unitary passes only.
 */
typedef struct {
    z2h_couplings start, end;
    int64_t steps;
    double dt;
    int64_t k_begin, k_end;
    int32_t sampling;
    int32_t order;
    int32_t renorm;
    int32_t reserved;
    const double *sZ;
    const double *sX;
} z2h_schedule;

#define Z2H_MAX_LOOPS 8
#define Z2H_DOS_BINS 33
/*
 * Observables of a state psi (Sec. IV, V).  All expectations are divided by
 * the norm <psi|psi>.  energy = <H(c)> for the couplings passed to observe.
 * sumA = sum_v <A_v>, sumB = sum_p <B_p>; mx, mz = mean over links of <X_l>
 * and <Z_l>.  zloop[j] = <prod over zmask_j of Z>, xloop[j] = <prod over
 * xmask_j of X> (Wilson and 't Hooft loops).  dos[w] = weight of psi on the
 * eigenvalue Ztilde = 2w - n of Ztilde = -sum_l Z_l (Sec. V), w = 0..n.
 * The same 56 doubles are the device output layout (index order below).
 */
typedef struct {
    double norm, energy, sumA, sumB, mx, mz; /* 0..5 */
    double zloop[Z2H_MAX_LOOPS];             /* 6..13 */
    double xloop[Z2H_MAX_LOOPS];             /* 14..21 */
    double dos[Z2H_DOS_BINS];                /* 22..54 */
    double xnorm;                            /* 55: norm measured in the X basis */
} z2h_obs;
#define Z2H_OBS_DOUBLES 56

typedef struct z2h_plan z2h_plan;
typedef struct z2h_batch z2h_batch;

/* ------------------------------------------------------------------ lattice */

/* Library bit of link h(x,y) (dir 0) or v(x,y) (dir 1); x, y taken modulo
 * the lattice.  Host only. */
z2h_status z2h_link_bit(int32_t Lx, int32_t Ly, int32_t x, int32_t y, int32_t dir,
                        int32_t *bit);

/* Star and plaquette masks (Sec. II) in library numbering, one uint64 per
 * vertex (index y*Lx + x); caller arrays of Lx*Ly entries.  Host only. */
z2h_status z2h_masks(int32_t Lx, int32_t Ly, uint64_t *stars, uint64_t *plaqs);

/* Loop masks reported by batches (library numbering): zl = {Wilson loop
 * around the 1 x min(3, Lx) strip of plaquettes in row 0, around the
 * L-shaped plaquettes (0,0), (1,0), (0,1), noncontractible W1 along x, W2
 * along y}; xl = {'t Hooft loops V1 (crossing the vertical links of row 0),
 * V2 (crossing the horizontal links of column 0)} (Sec. IV).  Caller arrays
 * of Z2H_MAX_LOOPS entries.  Host only. */
z2h_status z2h_loop_masks(int32_t Lx, int32_t Ly, uint64_t *zl, int32_t *nz, uint64_t *xl,
                          int32_t *nx);

/* ------------------------------------------------------------------ plans */

/*
 * Plan for one lattice and precision on the current HIP device: masks,
 * syndrome data, pass schedule (tile geometry of every Walsh-Hadamard pass).
 * Lx, Ly >= 2, n = 2 Lx Ly <= 32.  max_tile_bits 0 = automatic; a smaller
 * value forces more passes per step (used to test the multi-group schedule
 * at small n).
 */
z2h_status z2h_plan_create(int32_t Lx, int32_t Ly, z2h_dtype dtype, int32_t max_tile_bits,
                           z2h_plan **out);
void z2h_plan_destroy(z2h_plan *plan); /* NULL-safe */

/* state_bytes = 2^n * sizeof(complex); ws_evolve_bytes = workspace needed by
 * z2h_evolve (the z passes' norm partials and, for multi-group plans whose
 * phase groups are whole windows, room for the phase tables of 1024
 * levels, which one launch computes ahead of the pass launches that read
 * them; ",tables=0" in a schedule string leaves them out);
 * ws_observe_bytes = workspace needed by z2h_observe (includes a
 * state-sized scratch copy); ws_adjoint_bytes = workspace for z2h_adjoint
 * without its per-step part: add 64 bytes per Trotter step plus 1024. */
z2h_status z2h_plan_sizes(const z2h_plan *plan, size_t *state_bytes, size_t *ws_evolve_bytes,
                          size_t *ws_observe_bytes, size_t *ws_adjoint_bytes);

/* Passes (HBM sweeps of the state) per Trotter step, and the number of
 * qubit groups the Walsh-Hadamard transform is split into. */
z2h_status z2h_plan_info(const z2h_plan *plan, int32_t *n, int32_t *groups,
                         int32_t *passes_per_step, int32_t *tile_bits);

/* JSON description of the pass schedule (host only, for diagnostics and
 * tests): R (log2 amplitudes per thread) and, per group, the tile bits m,
 * carried low bits c, first transformed global bit b0, transformed local
 * range [x0, x1), register layouts p[] and their butterfly ranges. */
z2h_status z2h_plan_describe(const z2h_plan *plan, char *buf, size_t len);

/* Fill d_state (256-byte aligned, state_bytes) with an initial state
 * (Sec. IV, Eqs. (ini1), (ini2)). */
z2h_status z2h_state_init(const z2h_plan *plan, void *d_state, z2h_init kind, void *stream);

/*
 * Apply steps [k_begin, k_end) of the schedule to d_state in place.
 * d_ws: workspace of at least ws_evolve_bytes (device).  If d_norms is not
 * NULL it receives, per applied step, the norm measured in that step's
 * diagonal z pass (device doubles, k_end - k_begin entries).
 */
z2h_status z2h_evolve(const z2h_plan *plan, void *d_state, void *d_ws, size_t ws_bytes,
                      const z2h_schedule *sched, double *d_norms, void *stream);

/*
 * z2h_evolve for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): no
 * workspace argument, and no allocation of any kind.  The scratch z2h_evolve
 * takes from its workspace (the z passes' per-tile norm partials; device
 * copies of sZ/sX when the schedule has them) lives in a fixed device array
 * of Z2H_NOALLOC_SCRATCH_BYTES that the library holds on every device it
 * runs on until the process ends; its address is looked up on the first
 * call on each device.  A call needs ws_evolve_bytes of it (z2h_plan_sizes)
 * less the phase-table room (here every workgroup builds its own table),
 * plus 16 bytes per step and 512 when sZ or sX is given; beyond the array's
 * size it returns Z2H_ERR_UNSUPPORTED before touching the device (the 4x4
 * torus needs 8 MiB).  Arguments, schedule semantics, d_norms and the
 * result are those of z2h_evolve, with the same kernels.  Every call on a
 * device shares that device's array: calls that overlap in time on one
 * device (other streams, other threads) race and corrupt each other's norm
 * partials; serialize them.  Nothing in the array needs clearing between
 * calls: each call writes what it reads.  With sZ/sX the host arrays are
 * copied in and the stream synchronized, as in z2h_evolve.
 */
#define Z2H_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
z2h_status z2h_evolve_noalloc(const z2h_plan *plan, void *d_state, const z2h_schedule *sched,
                              double *d_norms, void *stream);

/*
 * Observables of d_state (not modified) for the couplings H (Sec. IV-V).
 * zmasks/xmasks: up to Z2H_MAX_LOOPS loop masks each (library numbering,
 * bits < n), may be NULL when the count is 0.  h_out (host) is filled after
 * a stream synchronization if not NULL; d_out (device, Z2H_OBS_DOUBLES
 * doubles, same order as z2h_obs) is filled asynchronously if not NULL.
 * Returns Z2H_ERR_NUMERIC when h_out is requested and the norm or energy is
 * not finite.
 */
z2h_status z2h_observe(const z2h_plan *plan, const void *d_state, void *d_ws, size_t ws_bytes,
                       const z2h_couplings *H, const uint64_t *zmasks, int32_t nz,
                       const uint64_t *xmasks, int32_t nx, z2h_obs *h_out, double *d_out,
                       void *stream);

/*
 * Gradient of L = <psi_M| H(lossH) |psi_M> / <psi_M|psi_M> with respect to
 * the per-step schedule values sZ[k] and sX[k] (see z2h_schedule), by
 * reverse evolution with the inverse passes (every pass is unitary, so no
 * intermediate state is stored):
 *   dL/dsZ[k] = 2 dt Im <lambda|dH_Z/ds|psi> at the z pass of step k,
 *   dL/dsX[k] = dt Im <lambda|dH_X/ds|psi> summed over its two x halves,
 * with lambda = H psi_M carried backwards beside psi.  d_psi_final: the state
 * after the full forward ramp of sched from its initial state (k_begin = 0,
 * k_end = steps, order 0, renorm 0); it is not modified.  d_gradZ, d_gradX:
 * device arrays of steps doubles.  d_ws: see z2h_plan_sizes.  h_loss (host,
 * may be NULL): L.  The call synchronizes the stream once (to read L and the
 * norm).  Plans whose transform groups have no straight-line kernel return
 * Z2H_ERR_UNSUPPORTED.
 */
z2h_status z2h_adjoint(const z2h_plan *plan, const void *d_psi_final, void *d_ws,
                       size_t ws_bytes, const z2h_schedule *sched, const z2h_couplings *lossH,
                       double *d_gradZ, double *d_gradX, double *h_loss, void *stream);

/* ------------------------------------------------------------------ paths */

/*
 * A piecewise-linear path through coupling space (Sec. III, Fig. evo: the
 * red path P(p,0) -> R(p,r) -> R'(0,r), the blue path P(p,0) -> P'(0,p);
 * Sec. V: the path (0,0.5) -> (0.5,0.5) -> O along the dual line).  Leg i
 * ramps linearly from vert[i] to vert[i+1] in steps[i] Trotter steps of
 * duration dt (sampling, order, renorm as in z2h_schedule; the paper's
 * protocol is sampling 1 with dg = 1e-5 per step, dt = 0.02).  Consecutive
 * legs join with unmerged x halves, so a path is the exact product of its
 * legs' Trotter steps.  trace_every > 0 observes the state every trace_every
 * steps of each leg and at each leg's end; 0 observes at leg ends only.
 */
typedef struct {
    int32_t nvert;              /* >= 2 */
    int32_t reserved;           /* 0 */
    const z2h_couplings *vert;  /* host, nvert entries */
    const int64_t *steps;       /* host, nvert - 1 entries, >= 0 */
    double dt;
    int32_t sampling, order, renorm, trace_every;
} z2h_path;

/*
 * Evolve d_state along the path and record observables (z2h_obs layout,
 * Z2H_OBS_DOUBLES doubles per sample, device) into d_trace: sample 0 is the
 * initial state observed at vert[0]; then, for each leg with steps > 0, one
 * sample after every trace_every steps and one at the leg's end, each
 * observed with the couplings of the point reached, vert[i] + (k/M)
 * (vert[i+1] - vert[i]) after k of the leg's M steps.  Loop masks as in
 * z2h_observe.  n_samples (host, may be NULL) receives the number of
 * samples; with d_trace NULL nothing is enqueued (size query).  trace_cap:
 * samples d_trace can hold (Z2H_ERR_WORKSPACE if fewer are needed).
 * d_ws: at least the larger of ws_evolve_bytes and ws_observe_bytes.
 */
z2h_status z2h_path_evolve(const z2h_plan *plan, void *d_state, void *d_ws, size_t ws_bytes,
                           const z2h_path *path, const uint64_t *zmasks, int32_t nz,
                           const uint64_t *xmasks, int32_t nx, double *d_trace, int64_t trace_cap,
                           int64_t *n_samples, void *stream);

/*
 * Many paths on one lattice at once (the paper's protocols batched over the
 * paths' parameters, e.g. the red paths for several r, Secs. IV-V).  The
 * npaths states lie contiguously at d_states (state j at element offset
 * j * 2^n; initialise them with z2h_state_init), and all paths must have the
 * same number of vertices, trace_every and step order; vertices, step
 * counts, dt, sampling and renorm may differ per path.  Leg i runs for all
 * paths together in segments of trace_every steps of the longest leg i (one
 * segment if trace_every is 0); after each segment every path is observed
 * with the couplings of the point it reached (a path whose leg is shorter
 * repeats its end state; a leg of zero steps is observed at its end
 * vertex).  Segment boundaries are those of z2h_path_evolve, so a path whose
 * legs all have the longest length gets exactly z2h_path_evolve's samples.
 * One pass launch serves every path.
 *
 * z2h_paths_sizes: samples (1 + the segments of every leg) and the workspace
 * (norm partials, one transformed copy per path, observable records, segment
 * records).  z2h_paths_evolve: d_trace (device) receives samples * npaths
 * records of Z2H_OBS_DOUBLES doubles, sample-major (record of path j in
 * sample s at (s * npaths + j) * Z2H_OBS_DOUBLES).  Loop masks as in
 * z2h_observe.  Synchronizes the stream once per leg.  Errors:
 * Z2H_ERR_INVALID (paths, masks, buffers), Z2H_ERR_WORKSPACE.
 */
z2h_status z2h_paths_sizes(const z2h_plan *plan, int32_t npaths, const z2h_path *paths, int64_t *n_samples,
                           size_t *ws_bytes);
z2h_status z2h_paths_evolve(const z2h_plan *plan, int32_t npaths, void *d_states, void *d_ws, size_t ws_bytes,
                            const z2h_path *paths, const uint64_t *zmasks, int32_t nz, const uint64_t *xmasks,
                            int32_t nx, double *d_trace, void *stream);

/* ------------------------------------------------------------------ batches */

/*
 * A batch of independent ramps (phase-diagram points, lattices of uneven
 * size) evolved together: lattice (Lx[j], Ly[j]), schedule sched[j] (sZ, sX
 * must be NULL; k range must be the whole ramp), initial state init[j], and
 * the couplings obsH[j] whose energy is reported.  All states live in one
 * device buffer; state_offsets[j] (host output, bytes) is where state j
 * starts.  The launch sequence of the whole batch (initialization, every
 * pass of every job, observables) is recorded once in a HIP graph.  Jobs
 * of one lattice run level by level (one launch per pass level for every
 * job that has one); where their step counts differ the host may pack them
 * into slots, jobs of a slot running back to back, so that launches keep
 * one size (chosen by a launch-cost model; the environment variable
 * Z2H_TUNE may force "slots=N", 0 = never pack).  Packing changes only the
 * grouping of launches, never a job's arithmetic: results are identical.
 */
z2h_status z2h_batch_create(int32_t njobs, const int32_t *Lx, const int32_t *Ly,
                            const z2h_schedule *sched, const z2h_init *init,
                            const z2h_couplings *obsH, z2h_dtype dtype, z2h_batch **out,
                            size_t *states_bytes, size_t *ws_bytes, uint64_t *state_offsets);

/* Run the batch: every state is initialized, evolved and observed.
 * d_obs: device, njobs * Z2H_OBS_DOUBLES doubles.  zloop[0] of each job is
 * the Wilson loop around the 1 x 3 (or 1 x Lx) strip of plaquettes in row 0,
 * zloop[1] the L-shaped three-plaquette loop, zloop[2] and [3] the
 * noncontractible Wilson loops, xloop[0..1] the 't Hooft loops.
 * The workspace (ws_bytes at least z2h_batch_create's figure) holds only
 * scratch that each run writes before reading it: the caller may use it for
 * anything else between runs.  Job records and norm partials are the
 * batch's own.  Runs of one batch must not overlap in time (they share the
 * batch's norm partials and graph). */
z2h_status z2h_batch_run(z2h_batch *batch, void *d_states, void *d_ws, size_t ws_bytes,
                         double *d_obs, void *stream);
void z2h_batch_destroy(z2h_batch *batch); /* NULL-safe */

/*
 * Traced batch runs (Sec. V diagnostics over a whole scan): every job's ramp
 * is split into segments of `every` Trotter steps (steps [s*every,
 * (s+1)*every) clipped to the job's M steps, joined with unmerged x halves,
 * so each sample is the state of the uninterrupted ramp) and all jobs are
 * observed after each segment with the couplings of the point reached,
 * c_start + (k/M) (c_end - c_start) after k steps.  A job that has finished
 * is observed again in later samples.  Lattices whose jobs mix the two step
 * orders are rejected.
 *
 * z2h_batch_trace_sizes: samples per job (ceil(max M / every)) and the
 * workspace a traced run needs (the same as z2h_batch_run's).
 *
 * z2h_batch_run_trace: like z2h_batch_run (d_obs receives the final
 * observables), plus d_trace (device, samples * njobs * Z2H_OBS_DOUBLES
 * doubles, sample-major: the record of job j in sample s starts at
 * (s * njobs + j) * Z2H_OBS_DOUBLES).  The launch sequence is recorded in a
 * HIP graph of its own (or issued directly with timing enabled).  The
 * per-segment job records are the batch's own: the first traced run with a
 * given interval synchronizes the stream, allocates device memory for them
 * if the batch's table is too small (freed by z2h_batch_destroy) and uploads
 * them; later runs with the same interval reuse them.  The workspace, as for
 * z2h_batch_run, holds only per-run scratch.  Errors: Z2H_ERR_OOM if that
 * allocation fails; Z2H_ERR_INVALID for a NULL or
 * misaligned buffer, every < 1, mixed step orders within a lattice or a
 * batch created on another device; Z2H_ERR_WORKSPACE if ws_bytes is below
 * z2h_batch_trace_sizes' figure.
 */
z2h_status z2h_batch_trace_sizes(const z2h_batch *batch, int32_t every, int64_t *samples_per_job,
                                 size_t *ws_bytes);
z2h_status z2h_batch_run_trace(z2h_batch *batch, void *d_states, void *d_ws, size_t ws_bytes, double *d_obs,
                               int32_t every, double *d_trace, void *stream);

/* Per-kind pass-kernel times (see z2h_timing_read) of the most recent
 * z2h_batch_run made while timing was enabled.  With timing enabled a batch
 * run issues its launch sequence directly on the stream, with an event pair
 * around every pass kernel, instead of replaying its HIP graph (the kernels
 * and their order are the same).  Synchronizes. */
z2h_status z2h_batch_timing(z2h_batch *batch, int64_t counts[4], double ms[4]);

/* ------------------------------------------------------------------ exact solvers */

/*
 * Exact references for the Trotterized evolution (Sec. VII compares against
 * exact diagonalisation; these extend it to every lattice the plans cover).
 * They act on states of the plan's lattice and precision (device buffers,
 * 256-byte aligned, library bit order) and share its pass geometry.
 *
 * z2h_hamiltonian_apply: d_y = H d_x with H the Hamiltonian of Eq. (effi),
 * H = -JA sum_v A_v - JB sum_p B_p - hx sum_l X_l - hz sum_l Z_l.  d_x and
 * d_y must not overlap; d_x is not modified.  Needs no workspace.  Computed
 * as D_Z x + 2^-n W D_X W x (W: Walsh-Hadamard transform over all links,
 * D_Z / D_X: the diagonal terms in the computational / Hadamard basis).
 * Errors: Z2H_ERR_INVALID for NULL, misaligned or overlapping buffers or
 * non-finite couplings.
 */
z2h_status z2h_hamiltonian_apply(const z2h_plan *plan, const void *d_x, void *d_y, const z2h_couplings *H,
                                 void *stream);

/*
 * Ground energy of H by the Lanczos recurrence.  d_v holds the start vector
 * on entry (any nonzero vector; the library's Z2H_INIT_PLUS state overlaps
 * the ground state whenever all couplings are >= 0, as H is then stoquastic)
 * and is overwritten by Lanczos vectors.  d_ws: z2h_lanczos_sizes bytes (two
 * state-sized vectors plus coefficients); must not overlap d_v.  The
 * recurrence runs without reorthogonalisation; every 8 iterations the
 * lowest eigenvalue of the tridiagonal matrix T is found by Sturm bisection,
 * and the run stops when it changes by at most tol * max(1, |e0|) between
 * checks, when an invariant subspace is reached (beta ~ 0), or after
 * max_iter iterations.  Outputs (host): *e0 the lowest eigenvalue of T,
 * *iters its dimension, h_alpha / h_beta (may be NULL; max_iter entries):
 * T's diagonal and the beta_1 .. beta_iters of the recurrence (h_beta[i]
 * couples Lanczos vectors i and i + 1).  Synchronizes the stream.  Errors:
 * Z2H_ERR_INVALID (arguments, max_iter outside [1, 100000], tol < 0),
 * Z2H_ERR_WORKSPACE, Z2H_ERR_NUMERIC (zero start vector, non-finite
 * coefficients).
 */
z2h_status z2h_lanczos_sizes(const z2h_plan *plan, int32_t max_iter, size_t *ws_bytes);
z2h_status z2h_lanczos_ground(const z2h_plan *plan, void *d_v, void *d_ws, size_t ws_bytes, const z2h_couplings *H,
                              int32_t max_iter, double tol, double *h_alpha, double *h_beta, int32_t *iters,
                              double *e0, void *stream);

/*
 * Exact stepwise evolution: for every step k_begin <= k < k_end of the
 * schedule, d_state <- exp(-i dt H_k) d_state, where H_k has the couplings
 * the Trotter step k uses (z-type JB, hz at sZ[k] or s_k; x-type JA, hx at
 * sX[k] or s_k), i.e. the product of exact exponentials that the Trotter
 * product of Eq. (decom) approximates.  Each exponential is taken in the
 * Krylov space of dimension krylov_dim (1..32) spanned by the state and
 * its images under H (Lanczos basis; exp(-i dt T) e_1 from a Jacobi
 * eigendecomposition of the small tridiagonal T).  order and renorm of the
 * schedule are ignored.  *err_est (may be NULL): the sum over steps of the
 * a posteriori estimate |psi| beta_m |(exp(-i dt T) e_1)_m| of the Krylov
 * truncation error.  d_ws: z2h_exact_sizes bytes (krylov_dim + 1 state-sized
 * vectors plus coefficients); must not overlap d_state.  Synchronizes the
 * stream once per step.  Errors as z2h_lanczos_ground, plus the schedule
 * checks of z2h_evolve.
 */
z2h_status z2h_exact_sizes(const z2h_plan *plan, int32_t krylov_dim, size_t *ws_bytes);
z2h_status z2h_exact_evolve(const z2h_plan *plan, void *d_state, void *d_ws, size_t ws_bytes,
                            const z2h_schedule *sched, int32_t krylov_dim, double *err_est, void *stream);

/*
 * Ground-state vector from a finished z2h_lanczos_ground run: d_v must hold
 * the same start vector that run began from (the recurrence is repeated with
 * the same kernels, so it reproduces the same Lanczos vectors), and receives
 * the unit-norm Ritz vector of the lowest eigenvalue of T, i.e.
 * sum_k s_k v_k with s the eigenvector of T (inverse iteration on the host).
 * h_alpha, h_beta, iters: that run's outputs.  energy (may be NULL) gets the
 * Rayleigh quotient <v|H|v>, residual (may be NULL) the norm |H v - E v|;
 * either costs one more application of H.  d_ws: z2h_lanczos_vector_sizes
 * bytes (three state-sized vectors plus coefficients).  Synchronizes.
 * Errors as z2h_lanczos_ground.
 */
z2h_status z2h_lanczos_vector_sizes(const z2h_plan *plan, int32_t iters, size_t *ws_bytes);
z2h_status z2h_lanczos_vector(const z2h_plan *plan, void *d_v, void *d_ws, size_t ws_bytes, const z2h_couplings *H,
                              const double *h_alpha, const double *h_beta, int32_t iters, double *energy,
                              double *residual, void *stream);

/* <a|b> of two states of the plan (FP64 reduction); d_ws: at least 32768
 * bytes of device scratch.  Synchronizes. */
z2h_status z2h_overlap(const z2h_plan *plan, const void *d_a, const void *d_b, void *d_ws, size_t ws_bytes,
                       double *re, double *im, void *stream);

/* Host-only helpers of the two solvers above, for a symmetric tridiagonal
 * matrix with diagonal alpha[0..m) and off-diagonal beta[0..m-1):
 * z2h_tridiag_lowest: its lowest eigenvalue (Sturm bisection);
 * z2h_tridiag_expv: exp(-i tau T) e_1 (m <= 32; Jacobi eigendecomposition). */
z2h_status z2h_tridiag_lowest(int32_t m, const double *alpha, const double *beta, double *out);
z2h_status z2h_tridiag_expv(int32_t m, const double *alpha, const double *beta, double tau, double *out_re,
                            double *out_im);

/* ------------------------------------------------------------------ gate-level circuits */

/*
 * Gate-level emulation of the paper's circuits (Sec. III; state preparation
 * Eqs. (ini1), (ini2)) on n + 1 qubits: the n links in library bit order and
 * one ancilla at bit n.  These run the circuit as written, gate by gate, as
 * a check of the circuit itself: the Trotter path above applies the same
 * operator through fused diagonal phases and needs no ancilla.
 *
 * Gate kinds (rotation convention R_a(theta) = exp(-i theta sigma^a / 2)):
 *   Z2H_GATE_H      Hadamard on q0
 *   Z2H_GATE_RX     R_x(theta) on q0
 *   Z2H_GATE_RZ     R_z(theta) on q0
 *   Z2H_GATE_CNOT   control q0, target q1
 *   Z2H_GATE_PROJ0  projection of q0 on |0> (not renormalised)
 *   Z2H_GATE_NORM   rescale the state to unit norm (q0 unused)
 */
#define Z2H_GATE_H 0
#define Z2H_GATE_RX 1
#define Z2H_GATE_RZ 2
#define Z2H_GATE_CNOT 3
#define Z2H_GATE_PROJ0 4
#define Z2H_GATE_NORM 5
typedef struct {
    int32_t kind;
    int32_t q0, q1;
    int32_t reserved; /* 0 */
    double theta;
} z2h_gate;

/*
 * The gates of one Trotter step of Sec. III for the couplings cx (used by
 * the x-type terms: JA, hx) and cz (z-type: JB, hz), duration dt, in time
 * order (the first gate acts first).  order 0 (x-z-x):
 *   R_x(-hx dt) on every link; the half stabilizer layer; R_z(-2 hz dt) on
 *   every link; the half stabilizer layer; R_x(-hx dt) on every link.
 * The half stabilizer layer realises exp(i JB B_p dt/2) per plaquette as
 * CNOTs from its links to the ancilla, R_z(-JB dt) on the ancilla, the same
 * CNOTs; then exp(i JA A_v dt/2) per star as Hadamards on its links, the
 * same CNOT / R_z(-JA dt) / CNOT gadget, Hadamards.  The ancilla starts and
 * ends in |0>.  order 1 (z-x-z) swaps the field layers (R_z(-hz dt) halves,
 * R_x(-2 hx dt) in the middle).  At 3x3: 522 gates.
 * out: host array of cap gates; *count receives the number written (and is
 * set even when cap is too small, which returns Z2H_ERR_WORKSPACE).  Host only.
 */
z2h_status z2h_circuit_step(int32_t Lx, int32_t Ly, const z2h_couplings *cx, const z2h_couplings *cz, double dt,
                            int32_t order, z2h_gate *out, int32_t cap, int32_t *count);

/* The preparation circuit of Eq. (ini1) (which = Z2H_INIT_PSI1: Hadamards
 * on every link, then per plaquette CNOTs to the ancilla, projection of the
 * ancilla on |0>, CNOTs) or Eq. (ini2) (Z2H_INIT_PSI1P: per star Hadamards
 * on its links, CNOTs, projection, CNOTs, Hadamards), from |0...0>, followed
 * by one NORM gate.  Host only; out / cap / count as above. */
z2h_status z2h_circuit_prep(int32_t Lx, int32_t Ly, int32_t which, z2h_gate *out, int32_t cap, int32_t *count);

/*
 * Apply gates[0..ngates) (host array, time order) to the state of nq qubits
 * (2^nq complex elements of dtype at d_state, 256-byte aligned; nq in
 * [2, 34]).  fuse 0: one kernel launch per gate (each a pass over the
 * state).  fuse 1 and 2 group the gates, and may move a gate ahead of gates
 * on other qubits (with which it commutes); groups never cross a NORM gate.
 * fuse 1: gates whose qubits fit one tile are applied
 * together, one pass per group; a tile always holds the four lowest qubits
 * (coalesced rows) and up to 8 (complex128) or 9 (complex64) others, each
 * thread holds 32 of its amplitudes in registers and the gates run there in
 * phases of at most five qubits, with layout changes through LDS; states of
 * fewer than 6 qubits use fuse 0.  fuse 2: gates on at most five qubits are
 * applied together in registers (each thread holds the 32
 * amplitudes that differ in those qubits), one pass per group (a group
 * holding qubits 0, 1 and 2 runs as a tile group, with coalesced rows);
 * states of fewer than 11 qubits use fuse 1.
 * NORM gates end a group; NORM leaves a zero state zero.  Results agree
 * with fuse 0 to rounding.  d_ws: z2h_gates_ws_bytes bytes (norm partials).
 * Errors: Z2H_ERR_INVALID (qubit out of range, q0 == q1 for CNOT, unknown
 * kind, nq out of range, bad buffers), Z2H_ERR_WORKSPACE.
 */
size_t z2h_gates_ws_bytes(int32_t nq);
z2h_status z2h_gates_run(int32_t nq, z2h_dtype dtype, void *d_state, void *d_ws, size_t ws_bytes,
                         const z2h_gate *gates, int32_t ngates, int32_t fuse, void *stream);

/*
 * The passes z2h_gates_run would make for this gate list (host only, no
 * device work): pass_of[i] (host array of ngates) receives the index of the
 * pass that applies gates[i], counting each NORM gate as a pass of its own;
 * *npasses the number of passes.  With fuse 0, or below the fused
 * executors' minimum state sizes, every gate is its own pass.  Passes run
 * in index order; gates within one pass keep their relative order.
 * Errors: as z2h_gates_run's argument checks.
 */
z2h_status z2h_gates_schedule(int32_t nq, z2h_dtype dtype, const z2h_gate *gates, int32_t ngates, int32_t fuse,
                              int32_t *pass_of, int32_t *npasses);

/* The adiabatic ramp of the schedule at gate level: for each step
 * k_begin <= k < k_end, the circuit of z2h_circuit_step with the step's
 * couplings (x-type at sX[k] or s_k, z-type at sZ[k] or s_k), applied by
 * z2h_gates_run on the n + 1 qubit state d_state.  renorm is ignored. */
z2h_status z2h_circuit_evolve(int32_t Lx, int32_t Ly, z2h_dtype dtype, void *d_state, void *d_ws, size_t ws_bytes,
                              const z2h_schedule *sched, int32_t fuse, void *stream);

/* ------------------------------------------------------------------ tuning */

/*
 * Autotuner: times candidate pass schedules (transform-group split, register
 * windows, tile size, carried contiguous bits, streaming loads) for Trotter
 * steps of `batch` states of the lattice on the current device, and keeps
 * the fastest for plans (batch 1) and batches of similar size (classes 1,
 * 2..63, >= 64) of this lattice and precision created afterwards in this
 * process.  If cache_path is not NULL the choice is appended to it (text,
 * one "n c128 batch-class schedule" line per entry; z2h_tune_load or the
 * environment variable Z2H_TUNE_CACHE read it back).  Allocates and frees
 * device memory for the trial states (batch * state_bytes) and synchronizes
 * the device.  best (may be NULL): the winning schedule string;
 * best_ms_per_step (may be NULL): its time per Trotter step.
 */
z2h_status z2h_autotune(int32_t Lx, int32_t Ly, z2h_dtype dtype, int32_t batch, const char *cache_path,
                        char *best, size_t best_len, double *best_ms_per_step);

/* Plan with an explicit schedule string (as returned by z2h_autotune):
 * "split=G:R:m:c/..." lists each transform group's width G, register window
 * 2^R, tile bits m and carried low bits c (group 0: qubits 0..G-1, c = 0).
 * A group may add ":2" (two neighbouring tiles per workgroup, in two
 * register windows per thread) or ":1c" (one tile per workgroup whose
 * layout changes move the real and then the imaginary parts through half
 * the LDS), then ":at<Q>" (its qubits start at Q) and ":h<N>[@<Q>]" (its
 * top N qubits are a second run at qubits Q..Q+N-1, or the highest free
 * ones).  A group without positions takes the lowest free qubits, in two
 * runs if they are not contiguous.  Groups in two runs need ":1c" when
 * their width is a whole number of windows.  "uniform,m=..,c=..,R=..,g0=.."
 * is the general planner with fixed tile parameters.  Either may end in
 * ",nt=1" (streaming loads and stores), ",xcd=<mask>" (bit j set: the
 * workgroups of the passes over group j are renumbered so that each of the
 * eight XCDs walks a contiguous range of tiles; launches whose block count
 * is not a multiple of 8 keep the hardware order; default 1, group 0 only)
 * and ",tables=0" (z2h_evolve lets every workgroup build its phase table
 * instead of computing the tables ahead).  Z2H_ERR_INVALID for an
 * unreadable string or qubits taken twice or left out;
 * Z2H_ERR_UNSUPPORTED for a group whose workgroup or LDS would not fit. */
z2h_status z2h_plan_create_config(int32_t Lx, int32_t Ly, z2h_dtype dtype, const char *schedule,
                                  z2h_plan **out);

/* The autotuner's candidate schedules for a lattice, one per line (host). */
z2h_status z2h_tune_candidates(int32_t Lx, int32_t Ly, z2h_dtype dtype, char *buf, size_t len);

/* Load schedules written by z2h_autotune. */
z2h_status z2h_tune_load(const char *cache_path);

/* ------------------------------------------------------------------ misc */

/* Enable (1) or disable (0) per-kernel event timing of the pass kernels
 * launched by this thread; z2h_timing_read returns the number of timed
 * launches and the summed milliseconds per pass kind (0: z pass, 1: x pass,
 * 2: plain transform pass, 3: other) and resets the counters.  Timing
 * synchronizes each launch's end event when read. */
z2h_status z2h_timing_enable(int32_t on);
z2h_status z2h_timing_read(int64_t counts[4], double ms[4]);

/* Library version string and the last error message of this thread. */
const char *z2h_version(void);
const char *z2h_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* Z2H_H */
