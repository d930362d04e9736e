/*
 * mrtfd.h -- C ABI of the MI355X (gfx950) implementation of the per-time-step
 * update of the two-dimensional MRT finite-difference lattice-Boltzmann model
 * of Chen, Xu, Zhang and Wang, "Two dimensional MRT LB model for
 * compressible and incompressible flows" (arXiv:1305.4736).
 *
 * The method (what one step computes, Sec. III update equation):
 *   f_i^{n+1} = f_i^n - nu_ix [F_{i,J+1/2} - F_{i,J-1/2}]_x
 *                     - nu_iy [F_{i,J+1/2} - F_{i,J-1/2}]_y
 *                     - dt M^-1 [ S (fhat - fhat^eq) + C ]
 * on the 16-velocity Kataoka-Tsutahara set (Sec. II, Fig. 1), with fhat = M f
 * (Appendix, m_1..m_16), equilibria of the non-conserved moments from the
 * seven moment relations (Appendix), the energy-flux correction C_8, C_9 of
 * moments 8 and 9 (Sec. II), face fluxes limited by psi(theta) (Sec. III,
 * flux, limiter and smoothness equations) and every term taken at level n.
 *
 * Conventions shared by every entry point
 *  - Velocity order: four groups of four, |v| = 1, 6, 2, 3; inside a group
 *    counter-clockwise, axis groups starting at +x, diagonal groups at (+,+).
 *  - Fields are row-major (ny, nx) arrays, x fastest; f and the
 *    non-equilibrium planes are (16, ny, nx).  All exchanged values are
 *    double precision, whatever the storage precision.
 *  - R = 1 (P = rho T); gamma = (b + 2) / b; eta0 is the extra-DOF
 *    parameter of the |v| = 1 group (5/2 in the paper, Appendix).
 *  - on_device = 1: pointers are device pointers (e.g. torch tensors' data
 *    pointers) valid on the handle's stream; on_device = 0: host pointers,
 *    the call then synchronises the stream before returning.
 *  - Every call returns MRTFD_OK or a negative status; no exception crosses
 *    the ABI.  mrtfd_last_error() gives the message of the last failure on
 *    the calling thread.
 *  - A handle is not thread-safe; separate handles are independent.  The
 *    caller owns every buffer it passes; the library owns all device state of
 *    a handle and frees it in mrtfd_destroy().
 */
#ifndef MRTFD_H
#define MRTFD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MRTFD_OK 0
#define MRTFD_EINVAL (-1)     /* invalid argument or unsupported combination */
#define MRTFD_ENOMEM (-2)     /* device allocation failed */
#define MRTFD_EDEVICE (-3)    /* HIP runtime error (message has the HIP error) */
#define MRTFD_ENONFINITE (-4) /* a node had rho <= 0, T <= 0 or NaN since the last check */
#define MRTFD_ESTATE (-5)     /* call out of order (e.g. step before init) */

/* Boundary kinds (Sec. IV-A: f = M^-1 fhat^eq of a fixed state; Sec. IV-C:
 * periodic and non-equilibrium-extrapolation walls; Sec. V: inflow, outflow). */
enum {
    MRTFD_BC_PERIODIC = 0,    /* must be used on both sides of an axis */
    MRTFD_BC_EQUILIBRIUM = 1, /* two ghost layers fixed at f^eq(rho, u, T); also inflow */
    MRTFD_BC_OUTFLOW = 2,     /* ghosts copy the last interior node (zero gradient) */
    MRTFD_BC_WALL_NEE = 3     /* wall on the first/last grid line: f_w = f^eq(rho_w, u_w, T_w)
                                 + (f_1 - f^eq_1), rho_w T_w = rho_1 T_1, ghosts continue the
                                 line through f_1 and f_w; walls on one axis only */
};

/* Flux limiter psi(theta) (Sec. III): the paper's piecewise form (MC),
 * minmod, Lax-Wendroff (psi = 1) and first-order upwind (psi = 0). */
enum { MRTFD_LIM_MC = 0, MRTFD_LIM_MINMOD = 1, MRTFD_LIM_LW = 2, MRTFD_LIM_UPWIND = 3 };

/* Storage precision: FP64 everywhere, or f stored and convected in FP32 with
 * the conserved-moment sums, temperature, equilibria, collision and the
 * M / M^-1 constants in FP64.  FP32 storage also stores, per node, the FP64
 * conserved moments (rho, j_x, j_y, e) of the populations each step
 * computes before rounding them, and every step first puts the rounded
 * populations back onto those moments: rounding to FP32 then never moves
 * mass, momentum or energy (96 bytes per node and buffer, against 128 in
 * FP64 storage). */
enum { MRTFD_FP64 = 0, MRTFD_FP32_STORAGE = 1 };

typedef struct {
    int kind;                /* MRTFD_BC_* */
    double rho, ux, uy, T;   /* state used by EQUILIBRIUM; ux, uy, T by WALL_NEE */
} mrtfd_bc;

typedef struct {
    int nx, ny;              /* grid nodes, wall nodes included; >= 1 */
    double dx, dy, dt;       /* spacing and time step (> 0) */
    double eta0;             /* 2.5 in the paper */
    double s[16];            /* relaxation rates s_1..s_16 (s_1..s_4 have no effect) */
    double b;                /* gamma = (b + 2) / b, > 0 */
    int limiter;             /* MRTFD_LIM_* */
    int precision;           /* MRTFD_FP64 or MRTFD_FP32_STORAGE */
    int energy_flux_correction; /* 1: C_8, C_9 on (needs s_5 != 0); 0: off */
    mrtfd_bc bc[4];          /* sides x-lo, x-hi, y-lo, y-hi */
} mrtfd_params;

typedef struct mrtfd_s* mrtfd_t;

/* Validate the parameters, allocate the two ping-pong state buffers (16
 * planes each, two ghost layers, rows padded to 128-byte lines) and bind the
 * handle to `hip_stream` (a hipStream_t; NULL = the null stream).  Rejects:
 * non-positive sizes or steps, unpaired periodic sides, walls on both axes,
 * grids too small for their walls, a velocity whose unsplit Courant sum
 * |v_x| dt / dx + |v_y| dt / dy exceeds 1 (for the axis groups this is
 * |v| dt / min(dx, dy) <= 1, i.e. 6 dt / min(dx, dy) <= 1 for |v| = 6),
 * negative rates, dt * max(s_5..s_16) >= 2, and the energy-flux correction
 * with s_5 = 0. */
int mrtfd_create(const mrtfd_params* p, void* hip_stream, mrtfd_t* out);

/* Device bytes a handle with these parameters will hold (state buffers and
 * scratch), for admission control.  Host-only. */
int mrtfd_footprint(const mrtfd_params* p, size_t* bytes);

/* f = M^-1 fhat^eq(rho, u, T) at every node (Sec. IV-A), then the boundary
 * fill (ghosts, wall nodes).  Each input is an (ny, nx) array. */
int mrtfd_init(mrtfd_t h, const double* rho, const double* ux, const double* uy,
               const double* T, int on_device);

/* Advance by nsteps explicit stages (Sec. III update eq., every term at
 * level n): a fused kernel computes moments, equilibria, correction,
 * collision, limited fluxes and the update.  On grids large enough to
 * fill the device (FP64 from about 1024 x 256 nodes, FP32 storage from
 * about 1024 x 512), where supported (no NEE wall along x, state below
 * 2 GiB), one launch takes two steps, the second reading
 * the first's rows (wall rows along y refilled among them) from on-chip
 * memory, so the state crosses HBM once per two steps; an odd remainder,
 * and handles set to one step per launch, take one launch per step (the
 * row-marching form for state buffers below 2 GiB, else the LDS-tile
 * form).  NEE walls along y are refilled by the row-marching kernels
 * themselves; other walls (along x, or in the LDS-tile form) by a small
 * launch after each step.  Every form gives the same bits.
 * Asynchronous on the handle's stream; non-finite or unphysical nodes are
 * flagged on the device and reported by mrtfd_sync. */
int mrtfd_step(mrtfd_t h, long nsteps);

/* Steps taken per kernel launch by mrtfd_step: k = 2 (the default on large
 * grids, where supported) fuses pairs of steps, k = 1 (the default
 * otherwise) launches once per step.  Results are bitwise the same either
 * way.  MRTFD_EINVAL for k other than 1 or 2,
 * or k = 2 on a handle with a wall along x or a state of 2 GiB or more
 * (the setting is then unchanged). */
int mrtfd_set_steps_per_launch(mrtfd_t h, int k);
int mrtfd_get_steps_per_launch(mrtfd_t h, int* k);

/* As mrtfd_step, and report the elapsed device time of those launches in
 * milliseconds, measured with HIP events on the handle's stream
 * (synchronises). */
int mrtfd_step_timed(mrtfd_t h, long nsteps, double* elapsed_ms);

/* rho, u_x, u_y, T (Sec. II: P = rho T, e = b rho T + rho u^2) at every node;
 * any output may be NULL. */
int mrtfd_macros(mrtfd_t h, double* rho, double* ux, double* uy, double* T, int on_device);

/* Non-equilibrium moments (Sec. V): star = 0 gives Delta = M (f - f^eq),
 * star = 1 gives Delta* = M*(u) (f - f^eq), M* being M with v replaced by
 * v - u (Appendix).  Output: (16, ny, nx). */
int mrtfd_noneq(mrtfd_t h, int star, double* delta, int on_device);

/* The interior distribution as FP64 populations, out / in, (16, ny, nx)
 * doubles.  FP32 storage keeps each node as its populations rounded to FP32
 * plus the FP64 conserved moments (rho, j_x, j_y, e) of the populations
 * they were rounded from; mrtfd_get_f gives the rounded populations with
 * their conserved moments put back onto the stored ones, mrtfd_set_f rounds
 * the populations and stores their conserved moments.  mrtfd_set_f refills
 * ghosts and wall nodes. */
int mrtfd_get_f(mrtfd_t h, double* f, int on_device);
int mrtfd_set_f(mrtfd_t h, const double* f, int on_device);

/* Checkpoint of the stored state, bit for bit: (nplanes, ny, nx) doubles,
 * the 16 stored populations (exact in FP64) followed, in FP32 storage, by
 * the 4 stored conserved moments.  mrtfd_state_planes gives nplanes (16 in
 * FP64 storage, 20 in FP32 storage).  mrtfd_set_state refills ghosts and
 * wall nodes; stepping on from it gives the same bits as stepping on from
 * the state it was taken from. */
int mrtfd_state_planes(mrtfd_t h, int* nplanes);
int mrtfd_get_state(mrtfd_t h, double* state, int on_device);
int mrtfd_set_state(mrtfd_t h, const double* state, int on_device);

/* Wait for the handle's stream; returns MRTFD_ENONFINITE (and clears the
 * flag) if any updated node saw rho <= 0, T <= 0 or NaN since the last
 * check. */
int mrtfd_sync(mrtfd_t h);

/* Steps taken since mrtfd_init / mrtfd_set_f. */
long mrtfd_steps_done(mrtfd_t h);

int mrtfd_destroy(mrtfd_t h);

/* Message of the last failure on this thread ("" if none).  The string is
 * owned by the library and valid until the next call on this thread. */
const char* mrtfd_last_error(void);

/* Free and total device memory of the current device in bytes (for
 * admission by free HBM). */
int mrtfd_device_memory(size_t* free_bytes, size_t* total_bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid allocation): one whole
 * solve -- as mrtfd_create, mrtfd_init, mrtfd_step(nsteps) and mrtfd_macros
 * with device pointers, same kernels, same bits -- whose state lives in a
 * file-scope device array of 64 MiB that each GPU holds until the process
 * ends, instead of in library allocations.  No hipMalloc, hipFree or other
 * allocating call is made; the array, the constants and the arguments are
 * set up by kernels on hip_stream.  rho, ux, uy, T: (ny, nx) device inputs;
 * rho_out .. T_out: (ny, nx) device outputs (any may be NULL).  Limits and
 * errors: MRTFD_EINVAL when the two state buffers (mrtfd_footprint) and a
 * 4 KiB set-up area exceed 64 MiB (square grids up to 492 x 492 nodes fit
 * in FP64 storage, 568 x 568 in FP32 storage), and for what mrtfd_create
 * rejects.
 * Asynchronous on hip_stream; non-finite nodes are not reported (check the
 * outputs).  Every call on a GPU uses that GPU's one array: calls that
 * overlap on one GPU (other streams or threads) race and must be ordered
 * by the caller; a call starts from a cleared array and leaves its last
 * state there. */
int mrtfd_solve_noalloc(const mrtfd_params* p, void* hip_stream, const double* rho, const double* ux,
                        const double* uy, const double* T, long nsteps, double* rho_out, double* ux_out,
                        double* uy_out, double* T_out);

/* Diagnostics: enqueue on hip_stream (a hipStream_t) a kernel of one block
 * per XCD that writes, to the device array out[16], each XCD's shader-clock
 * counter (s_memtime; out[2 x]) and real-time counter (s_memrealtime, taken
 * as 100 MHz; out[2 x + 1]), x the XCD number.  Two stamps around a
 * stretch of launches estimate the clock each XCD ran at as
 * counts / (ticks / 1e8) (the counters of different XCDs are not aligned;
 * pairs a stamp did not write keep their old contents).  The estimate
 * follows the clock's changes within a run but has read above the 2.4 GHz
 * maximum on some machines: it is not an exact core clock.  Asynchronous;
 * read out after the stream has finished. */
int mrtfd_clock_stamp(void* hip_stream, unsigned long long* out);

/* Host-only: the dense 16x16 M and M^-1 (row-major) the kernels use in their
 * factored form (per-group angular sums times small blocks), for checks. */
int mrtfd_constants(double eta0, double* M, double* Minv);

/* ------------------------------------------------------------------------
 * Batched form: many independent instances (different grids, states,
 * rates, b and boundaries; one precision and one limiter per batch) advance
 * together, one persistent launch per tile-shape class per step (or per
 * two steps, for the instances that take two steps per launch).  The
 * per-instance arithmetic is the one above, so a slot's result does not
 * depend on the other slots.  Slots own their device state (allocated from
 * the stream-ordered pool on the batch's stream) and a step budget; slots
 * that have used their budget stop stepping and stay readable until
 * removed.  Slot numbers are reused after mrtfd_batch_remove.
 * ------------------------------------------------------------------------ */
typedef struct mrtfd_batch_s* mrtfd_batch_t;

/* capacity slots (1 .. 65536); precision MRTFD_FP64 / MRTFD_FP32_STORAGE;
 * limiter MRTFD_LIM_*; hip_stream a hipStream_t (NULL = null stream).  All
 * work is ordered on hip_stream; the batch also owns one internal stream
 * (default priority), forked from and joined back to hip_stream inside
 * each step call. */
int mrtfd_batch_create(int capacity, int precision, int limiter, void* hip_stream, mrtfd_batch_t* out);
int mrtfd_batch_destroy(mrtfd_batch_t b);

/* Validate p (its precision and limiter must be the batch's), allocate the
 * slot's state, initialise it to f^eq(rho, u, T) (Sec. IV-A) and give it a
 * budget of nsteps steps (nsteps < 0: unlimited).  Fails with MRTFD_ENOMEM
 * when no slot is free or the device allocation fails.  *slot receives the
 * slot number. */
int mrtfd_batch_add(mrtfd_batch_t b, const mrtfd_params* p, const double* rho, const double* ux,
                    const double* uy, const double* T, int on_device, long nsteps, int* slot);
int mrtfd_batch_remove(mrtfd_batch_t b, int slot);

/* New budget for a slot, counted from now (nsteps < 0: unlimited). */
int mrtfd_batch_set_steps(mrtfd_batch_t b, int slot, long nsteps);

/* Advance every slot that still has budget by nsteps steps (each slot stops
 * when its budget is spent), in rounds of one step, or of two steps where
 * mrtfd_batch_set_steps_per_launch allows.  Asynchronous on the batch's
 * stream.  The timed form synchronises and reports the device time of
 * those launches (HIP events). */
int mrtfd_batch_step(mrtfd_batch_t b, long nsteps);

/* Steps per launch of the batch's two-step rounds: with k = 2 (default),
 * slots in the strip class without walls along x and with at least 4 rows
 * take two steps per launch (the second step reading the first's rows from
 * on-chip memory) in rounds where their work fills the device (a smaller
 * batch is faster one step at a time); other slots, and such slots with one
 * step left, take one-step launches in those rounds.  k = 1: one step per
 * launch for every slot.  Results are bitwise the same either way;
 * MRTFD_EINVAL for k other than 1 or 2. */
int mrtfd_batch_set_steps_per_launch(mrtfd_batch_t b, int k);
int mrtfd_batch_get_steps_per_launch(mrtfd_batch_t b, int* k);
int mrtfd_batch_step_timed(mrtfd_batch_t b, long nsteps, double* elapsed_ms);

/* Steps a slot has taken since it was added or its state set, and the steps
 * left in its budget (-1: unlimited). */
long mrtfd_batch_steps_done(mrtfd_batch_t b, int slot);
int mrtfd_batch_remaining(mrtfd_batch_t b, int slot, long* remaining);

/* Diagnostics: rounds the batch has run since it was created, of one step
 * and of two steps (see mrtfd_batch_set_steps_per_launch).  MRTFD_EINVAL
 * for NULL arguments. */
int mrtfd_batch_rounds(mrtfd_batch_t b, long* one_step, long* two_step);

/* Diagnostics: the band height (rows) of the batch's two-step launches as
 * last fitted to the load: the tallest of 160, 128, 96, 80, 64, 48 and 32
 * rows that gives every resident pair of the two-step kernel eight work
 * items (1.25 times that to grow), refitted whenever the work lists change.
 * The height changes no result, only the launch shape.  MRTFD_EINVAL for
 * NULL arguments. */
int mrtfd_batch_pair_rows(mrtfd_batch_t b, int* rows);

/* Per-slot outputs and checkpoint, as the single-instance calls. */
int mrtfd_batch_macros(mrtfd_batch_t b, int slot, double* rho, double* ux, double* uy, double* T,
                       int on_device);
int mrtfd_batch_get_f(mrtfd_batch_t b, int slot, double* f, int on_device);
int mrtfd_batch_set_f(mrtfd_batch_t b, int slot, const double* f, int on_device);

/* Synchronise; flags[capacity] (may be NULL) receives 1 for every slot with
 * a node at rho <= 0, T <= 0 or NaN since the last check, and the call
 * returns MRTFD_ENONFINITE if any (flags are then cleared). */
int mrtfd_batch_status(mrtfd_batch_t b, int* flags);
int mrtfd_batch_sync(mrtfd_batch_t b);

/* Work decomposition of a slot: its shape class (see below) as the output
 * nodes per work item along x and y (txw x byr); for the row-marching
 * strips, 60 columns by the rows of one band. */
int mrtfd_batch_shape(mrtfd_batch_t b, int slot, int* txw, int* byr);

/* Shape classes of a slot: 0..3 are LDS tiles of 256 nodes (32 x 8, 64 x 4,
 * 128 x 2, and 256 x 1 for one-row instances whose y sides are periodic or
 * outflow); 4 is the row-marching form (one wavefront per strip of 60
 * columns and band of up to 12 rows; instances whose state buffer is below
 * 2 GiB).  All classes give bitwise identical results.  Force a slot into
 * class `shape` (for tuning and comparison); the slot's state is kept.
 * MRTFD_EINVAL for an unknown class or one that does not fit the slot. */
int mrtfd_batch_set_shape(mrtfd_batch_t b, int slot, int shape);

/* Autotuner: measure the device time per work unit of each shape class (a
 * tile; a strip row including its bands' halo rows) and of one small launch
 * of it on calibration instances, write the former to cost_per_unit_us[5]
 * (may be NULL), and give every slot the class with the smallest units x
 * cost, except that a class whose slots together would save less than its
 * launch costs leaves them in the strip class.  Slot states are untouched;
 * later additions use the measured costs (a class not yet in use is charged
 * its launch). */
int mrtfd_batch_autotune(mrtfd_batch_t b, double* cost_per_unit_us);

#ifdef __cplusplus
}
#endif

#endif /* MRTFD_H */
