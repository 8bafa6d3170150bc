/*
 * af.h -- C ABI of the MI355X (gfx950) fully discrete Active Flux library:
 * the RB-TAI time step of Duraisamy, "Fully Discrete Active Flux Method based on
 * Transported Acoustic Increments for the Compressible Euler Equations".
 *
 * Problem (Sec. 2): 2-D compressible Euler, ideal gas, periodic Cartesian grid of
 * nx x ny square cells of side h.  Cell C_ij = [x_i, x_{i+1}] x [y_j, y_{j+1}].
 *
 * State (Sec. 2, list of degrees of freedom; Fig. 1): 16 planes of nx*ny scalars,
 * row-major with i (x) fastest, element (i, j) at offset j*nx + i:
 *   avg[0..3] = conservative cell averages (rho, rho u, rho v, E) of C_ij,
 *   V[0..3]   = primitive (rho, u, v, p) at the vertex (x_i, y_j),
 *   EV[0..3]  = primitive at the vertical-edge midpoint (x_i, y_{j+1/2}),
 *   EH[0..3]  = primitive at the horizontal-edge midpoint (x_{i+1/2}, y_j).
 * Element type: double for AF_F64 contexts; for AF_F32 contexts float
 * perturbations about the context's background state (see af_config.bg).
 * All state pointers are DEVICE pointers owned by the caller.
 *
 * Every function returns an af_status; none aborts or prints.  Work is enqueued on
 * the HIP stream given to af_init (borrowed, not owned) and is asynchronous unless
 * stated otherwise.  A context is not thread-safe: its calls must not overlap (they
 * share its scratch, status flag and events); distinct contexts are independent.
 * The caller keeps the state buffers alive and unmodified until the enqueued work
 * that uses them has completed on the stream.
 */
#ifndef AF_H_
#define AF_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t af_status;

enum {
    AF_OK = 0,
    AF_ERR_ARG = 1,          /* null pointer, nx < 4 or ny < 4, nx ny > 2^31 cells, h <= 0,
                                gamma <= 1, bad dt */
    AF_ERR_HIP = 2,          /* HIP runtime error; af_last_hip_error() returns its code */
    AF_ERR_ACOUSTIC_CFL = 3, /* some node has c_K dt / h > 1/2 (node-centred wedges invalid) */
    AF_ERR_FOOT = 4,         /* some convective foot moved one cell or more */
    AF_ERR_NONPHYSICAL = 5,  /* rho <= 0 or p <= 0 at a node or recovered centre, or NaN */
    AF_ERR_UNSUPPORTED = 6,  /* operation not available for this context's precision */
    AF_ERR_SCRATCH = 7,      /* grid larger than the fixed scratch of af_step_adjoint_noalloc */
    AF_ERR_FOOTPRINT = 8     /* AF_SCHEME_FC: a disk of radius c* tau / h about a foot leaves the
                                half-cell footprint |F - P| + R < h/2 (App. C, eq. fc-half-footprint) */
};

enum { AF_F64 = 0, AF_F32 = 1 };

enum {
    AF_CHECK = 1,       /* af_step reads back the device status flag after each call
                           (one host synchronisation per call) and returns the error */
    AF_SCHEME_RB = 2,   /* additive RB point update (eq. barsukow-additive) instead of
                           the transported-increment update (eq. transported-update) */
    AF_SCHEME_FC = 4    /* foot-centred exact frozen-acoustic point update (App. C; Sec. 4,
                           the paragraph on an exact frozen acoustic update): the frozen
                           state taken at the convective foot and the exact solution of the
                           frozen acoustic system evaluated there by quadrature of spherical
                           means; density from the linear closure.  An analytical reference
                           several hundred times the transported update's cost.  AF_F64
                           single-grid contexts only, not with AF_SCHEME_RB; no adjoint.
                           Fails with AF_ERR_FOOTPRINT when |F - P| + c* tau / h >= 1/2 */
};

typedef struct af_config {
    int32_t nx, ny;      /* cells in x and y (>= 4; nx ny <= 2^31) */
    double x0, y0;       /* lower-left corner (informational) */
    double h;            /* cell size, dx = dy = h (Sec. 2) */
    double gamma;        /* ratio of specific heats (> 1) */
    int32_t precision;   /* AF_F64 or AF_F32 */
    double bg[4];        /* AF_F32: background primitive state (rho, u, v, p) about which
                            the float planes hold perturbations; ignored for AF_F64 */
    int32_t flags;       /* AF_CHECK | AF_SCHEME_RB or AF_SCHEME_FC */
} af_config;

typedef struct af_state {
    void* avg[4];
    void* V[4];
    void* EV[4];
    void* EH[4];
} af_state;

typedef struct af_diag {
    double mass, momx, momy, energy; /* h^2 * sum over cells of the averages */
    double entropy;                  /* -int rho log(p / rho^gamma) dA, tensor Simpson
                                        over the nine Q2 nodes of every cell */
    double min_rho, min_p;           /* over V, EV, EH nodes and recovered centres */
    double max_speed;                /* max(|u| + c) over the same nodes */
    double max_acoustic_r;           /* max c dt / h over the same nodes, for dt given */
    double vorticity;                /* int omega dA, omega = dv/dx - du/dy of the continuous
                                        piecewise-Q2 velocity reconstruction (Sec. 6, low-Mach
                                        shear); zero up to round-off on a periodic grid */
    double enstrophy;                /* int omega^2 dA of the same field (both by 3x3
                                        Gauss-Legendre per cell, exact) */
} af_diag;

typedef struct af_ctx af_ctx;

/* Create a context for one grid.  cfg is copied.  hip_stream: a hipStream_t (may be
 * NULL for the null stream), borrowed for the life of the context.  Allocates the
 * context's device scratch (a second state for ping-ponging, reduction buffers, the
 * status flag) on the current device.  *out receives the context. */
af_status af_init(const af_config* cfg, void* hip_stream, af_ctx** out);

/* Advance nsteps >= 1 steps of size dt (fixed) in place.  Each step is the algorithm
 * of Sec. 6.1: centre recovery (eq. center-node), node-centred exact acoustic
 * increments at V, EV, EH and recovered centres for tau = dt/2 and dt (App. D,
 * eq. compact-monomial-block), cellwise Q2 interpolants of the increments, the
 * two-Picard convective foot (eq. adv-footpoint), the transported point update
 * (eq. transported-update; density from the frozen invariant), space-time Simpson
 * fluxes and the conservative average update (eq. af-average-update).
 * inout: caller-owned device planes, overwritten with the state after nsteps.
 * Errors: AF_ERR_ARG for a bad dt (<= 0 or not finite); with AF_CHECK set, the
 * acoustic-CFL, foot and non-physical checks are read back after every step and, if
 * one fired, the call returns its status with *inout (and, for AF_F32, the context's
 * compensation planes) restored to the input of the call, whichever of the nsteps
 * steps failed.  The rollback copy is taken on the device before the first step
 * (allocated by the first such call).  Without AF_CHECK the flag is only accumulated
 * on the device (read it with af_read_status) and no copy is taken.
 * AF_F32: the Kahan compensation planes of the average update carry over from one
 * call to the next only when the call's input is the buffer that holds the previous
 * call's output (here *inout itself); any other input starts a new trajectory with
 * zeroed compensation (see also af_reset_trajectory). */
af_status af_step(af_ctx* ctx, af_state* inout, double dt, int32_t nsteps);

/* One step from `in` to `out` (distinct buffers, both caller-owned); same operation
 * and errors as af_step with nsteps = 1, except that `in` is never modified (on an
 * error `out` holds the failed step and, with AF_CHECK, an AF_F32 context's
 * compensation is restored).  AF_F32: the compensation continues when `in` is the
 * previous call's output buffer (stepping out of a state twice restarts it).
 * AF_ERR_ARG if the two states share a plane pointer. */
af_status af_step_out(af_ctx* ctx, const af_state* in, af_state* out, double dt);

/* AF_F32 contexts: forget the trajectory, so that the next step starts with zeroed
 * compensation even if its input buffer is the previous output's (for a caller that
 * reuses a buffer for unrelated data).  Batch contexts: the same for every grid.
 * No effect on AF_F64 contexts.  Host-only; AF_ERR_ARG for a null context. */
af_status af_reset_trajectory(af_ctx* ctx);

/* Read and clear the device status flag accumulated since the last read
 * (synchronises the stream).  *status receives AF_OK or the first error class. */
af_status af_read_status(af_ctx* ctx, af_status* status);

/* Reverse-mode derivative of one step (AF_F64 only; either point update, TAI or
 * AF_SCHEME_RB): cot_n = (d step / d state_n)^T cot_np1 at fixed dt, where step is the
 * map of af_step_out.  primal_n: the state the step was taken from; cot_np1:
 * cotangent of the step's output; cot_n: overwritten (not accumulated), distinct from
 * the other two.  All three are caller-owned device states of doubles.  Asynchronous
 * on the context stream; the first call allocates the context's adjoint scratch (56
 * planes).  Errors: AF_ERR_ARG for a bad pointer or dt (<= 0 or not finite) or for
 * cot_n sharing a plane pointer with cot_np1 or primal_n,
 * AF_ERR_UNSUPPORTED on an AF_F32 or batch context.  The derivative of the foot's cell
 * (a floor) is taken as zero. */
af_status af_step_adjoint(af_ctx* ctx, const af_state* primal_n, const af_state* cot_np1,
                          af_state* cot_n, double dt);

/* Allocation-free form of af_step_adjoint, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc).  Same operation, arguments and errors as af_step_adjoint, without a
 * context: cfg (read only; precision must be AF_F64, flags may hold AF_SCHEME_RB and
 * AF_CHECK) and hip_stream (borrowed; NULL for the null stream) stand in for it.
 * The call allocates nothing: the 56 scratch planes and the status word live in a
 * static device array that every GPU loading the library holds for the life of the
 * process, sized for grids of at most 65536 cells (nx ny <= 2^16, e.g. 256 x 256;
 * 29.4 MB).  Larger grids return AF_ERR_SCRATCH before any work is enqueued.  All
 * calls on one GPU share that array and the array keeps the last call's contents: the
 * kernels zero what must start at zero, but calls that overlap on one GPU (different
 * streams or threads without ordering) race and give wrong results.  Asynchronous on
 * hip_stream; with AF_CHECK the call synchronises the stream and returns the step's
 * acoustic-CFL, foot and non-physical status. */
af_status af_step_adjoint_noalloc(const af_config* cfg, void* hip_stream, const af_state* primal_n,
                                  const af_state* cot_np1, af_state* cot_n, double dt);

/* Diagnostics of a state (Sec. 6, opening paragraph: CFL and entropy; Sec. 3:
 * conservation), reduced in FP64 on the device.  Synchronous: returns when *out is
 * filled.  dt only enters max_acoustic_r. */
af_status af_diagnostics(af_ctx* ctx, const af_state* s, double dt, af_diag* out);

/* Time the step kernel(s): runs nsteps steps on a scratch copy of `s` bracketed by
 * HIP events recorded on the context stream and returns the elapsed milliseconds of
 * the whole sequence and of the dominant kernel's launches (sum).  `s` is unchanged. */
af_status af_time_steps(af_ctx* ctx, const af_state* s, double dt, int32_t nsteps,
                        double* total_ms, double* kernel_ms);

/* Batching form.  n grids (each described by its own af_config; all AF_F32, all with
 * the same point update: TAI, or AF_SCHEME_RB for every grid) stepped together: every step is ONE kernel launch over the list of
 * (grid, tile) work items of the whole batch, and af_step_batch replays nsteps such
 * launches captured in a hipGraph (built on first use for each nsteps and kept; at
 * most 16 distinct nsteps are kept at a time).  The tile shape is chosen by an
 * autotuner on the first af_step_batch call: every compiled candidate is timed on a
 * copy of the batch's states and the fastest is kept (af_batch_info reports the
 * timings); the environment variable AF_BATCH_TILE=k (0 <= k < 15), read by
 * af_init_batch, fixes candidate k instead.  With AF_BATCH_TUNE_CACHE=path (also read
 * by af_init_batch) the tuner first looks the batch up in that text file, keyed by
 * device architecture and compute units, candidate table, point update and the grids'
 * sizes in order, and takes the recorded choice without timing; otherwise it tunes and
 * appends a line (an unreadable file is ignored; af_batch_info reports
 * "tuned_from_cache").  Candidates (cells x cells / threads per
 * workgroup): 32x8/512, 32x8/256, 32x16/512, 32x16/256, 64x8/512, 16x16/256, first
 * in the persistent grid mode (k < 6: CUs x resident workgroups looping over the
 * work list), then in the direct mode (6 <= k < 12: one workgroup per work item),
 * and k = 12, 13: 32x8/512 and 24x13/512 direct with registers capped for two
 * workgroups per CU, and k = 14: 31x10/512 direct, capped, with the point-update
 * targets in rows of 32 lanes (the single-grid FP32 kernel's configuration).  Each
 * grid keeps its own Kahan compensation planes, tied to the trajectory as for AF_F32
 * contexts.  The library allocates one partner state and four compensation planes
 * per grid.  hip_stream is borrowed; replays run on an internal stream ordered after
 * it. */
af_status af_init_batch(const af_config* cfgs, int32_t n, void* hip_stream, af_ctx** out);
/* (af_init_batch errors: AF_ERR_ARG for n outside 1..4096, a config af_init would
 * reject, or more than 2^31 cells in all; AF_ERR_UNSUPPORTED for a config that is not AF_F32, or whose AF_SCHEME_RB
 * flag differs from the first config's.  Configs are checked before any HIP call.) */

/* Advance every grid q of a batch context by nsteps (1..65536) steps of size dts[q]
 * in place; states[q] are caller-owned float perturbation planes (layout as above).
 * The result for grid q is the one af_step gives on an AF_F32 context of cfgs[q].
 * The library's descriptor copy is re-uploaded (one host synchronisation) only when
 * a state pointer or dt changed since the previous call.  With AF_CHECK in
 * cfgs[0].flags the status of the whole batch is read back after the call and, if a
 * check fired in any grid at any of the nsteps steps, every grid's state and
 * compensation are restored to the input of the call (copies taken on the device
 * before the replay; the first such call allocates one copy per grid).  Errors:
 * AF_ERR_ARG for bad pointers or dts, AF_ERR_UNSUPPORTED on a single-grid context
 * (and the single-grid calls return it on a batch context). */
af_status af_step_batch(af_ctx* ctx, af_state* states, const double* dts, int32_t nsteps);

/* JSON text describing a batch context's work list and tuning (chosen tile shape and
 * the measured ms per step of every candidate) into buf (NUL-terminated, truncated
 * to buflen); returns the full length, or -1 for a non-batch context. */
int32_t af_batch_info(af_ctx* ctx, char* buf, int32_t buflen);

void af_destroy(af_ctx* ctx);
const char* af_status_string(af_status s);
int32_t af_last_hip_error(void);
/* Name of the kernel af_time_steps reports as dominant. */
const char* af_dominant_kernel(af_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* AF_H_ */
