/*
 * grpic.h -- C ABI of the MI355X GRPIC hot path.
 *
 * One handle holds one general-relativistic electromagnetic particle-in-cell
 * run in Kerr space-time, Cartesian Kerr-Schild coordinates (Watson &
 * Nishikawa, arXiv:0904.0232).  The problem statement follows Sec. 2.2 of the
 * paper: particles carry (q, m, x, u) with u the four-velocity, and the
 * Maxwell field tensor lives on a Yee-staggered grid (Sec. 3).  Units: the
 * cell edge is 1 and x^4 = c t; m (hole mass) and a (spin parameter, the
 * hole carries angular momentum m a) are lengths in cells.
 *
 * All device memory belongs to the handle (allocated through the optional
 * allocator callbacks, else hipMalloc).  Host pointers passed in are only
 * read during the call; the caller keeps ownership.  Every call returns 0 or
 * a negative GRPIC_E* code and never throws.  A handle is not thread-safe.
 * Work is enqueued on the HIP stream given at creation; grpic_step is
 * asynchronous, the dump and diagnostics calls synchronise that stream.
 */
#ifndef GRPIC_H
#define GRPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GRPIC_MAX_SPECIES 8
#define GRPIC_DEAD 0xFF

enum {
    GRPIC_OK = 0,
    GRPIC_EINVAL = -1,    /* invalid argument or configuration              */
    GRPIC_ENOMEM = -2,    /* allocation failed or capacity exceeded         */
    GRPIC_EDEVICE = -3,   /* a HIP call failed                              */
    GRPIC_EOVERFLOW = -4, /* fixed-point current accumulator out of range   */
    GRPIC_ESTATE = -5,    /* call not valid in the handle's current state   */
    GRPIC_EAGAIN = -6     /* batch: no slot or memory free right now         */
};

enum { GRPIC_FP64 = 0, GRPIC_FP32_MIXED = 1 };
/* Stage time-dilation factor of the RK4 pusher (Sec. 3.3, the gamma_i
 * estimate): PAPER = the printed estimate from u^4 and a^4; U4 = u^4/c. */
enum { GRPIC_GAMMA_PAPER = 0, GRPIC_GAMMA_U4 = 1 };
/* Transverse current weights (Sec. 4): CURVED = face-area fractions with the
 * metric area density; FLAT = bilinear (exactly charge conserving). */
enum { GRPIC_DEPOSIT_CURVED = 0, GRPIC_DEPOSIT_FLAT = 1 };
/* RK4 structure of the pusher (Sec. 3.3).  CLASSIC = the default reading of
 * the printed steps: stages at dt/2, dt/2, dt of the slopes
 * (u_k, a_k)/gamma_k in coordinate time, combined 1:2:2:1 over 6 (fourth
 * order).  PRINTED = the four steps exactly as printed (averaged stage
 * velocities, dtau = dt/2gamma, dt/gamma, dt/gamma, dt/2gamma, final sums
 * added to x_n and u_n; their weights sum to 5/6), an ablation that
 * quantifies the printed form.  FP64 only. */
enum { GRPIC_RK_CLASSIC = 0, GRPIC_RK_PRINTED = 1 };
/* Where the pusher gathers the field tensor (Sec. 3.3): STAGE = at every RK
 * stage position (default); STEP = once at x_n for all four stages (an
 * ablation; the Christoffel symbols stay at the stage positions).  FP64 only. */
enum { GRPIC_GATHER_STAGE = 0, GRPIC_GATHER_STEP = 1 };
/* Cloud-in-cell weights of the gather (Sec. 3.3).  TRILINEAR = sub-volumes
 * with the 4-metric density sqrt(-det g), which is exactly 1 here (the
 * default reading); SPATIAL = sub-volumes weighted by the spatial density
 * sqrt(det g_ij) = sqrt(1 + f) at their centres, normalised (reading B, an
 * ablation).  FP64 only. */
enum { GRPIC_WEIGHTS_TRILINEAR = 0, GRPIC_WEIGHTS_SPATIAL = 1 };

typedef void *(*grpic_alloc_fn)(size_t bytes, void *ctx);
typedef void (*grpic_free_fn)(void *ptr, void *ctx);

typedef struct {
    int32_t nx, ny, nz;     /* cells per axis, each >= 4                          */
    int32_t precision;      /* GRPIC_FP64 or GRPIC_FP32_MIXED                      */
    int32_t gamma_mode;     /* GRPIC_GAMMA_*                                        */
    int32_t deposit_mode;   /* GRPIC_DEPOSIT_*                                      */
    int32_t field_iters;    /* constitutive passes per half-cycle, >= 1 (3)         */
    int32_t sort_every;     /* steps between cell sorts; 0 = never                 */
    int32_t tile;           /* sort tile edge in cells (4)                         */
    int32_t fp_bits;        /* fraction bits of the int64 current accumulator, 16..50 (44) */
    int32_t nspecies;       /* 1..GRPIC_MAX_SPECIES                                 */
    int32_t init_covariant; /* 0: uniform contravariant B0 (paper); 1: covariant    */
    int32_t rk_mode;        /* GRPIC_RK_* (FP64 only; CLASSIC otherwise)            */
    int32_t gather_mode;    /* GRPIC_GATHER_* (FP64 only; STAGE otherwise)          */
    int32_t gather_weights; /* GRPIC_WEIGHTS_* (FP64 only; TRILINEAR otherwise)     */
    double c, dt;           /* speed of light and time step                        */
    double m, a;            /* hole mass and spin parameter, |a| <= m               */
    double center[3];       /* hole position in node coordinates                   */
    double r_rm;            /* particles with r < r_rm are removed                 */
    double r_exc;           /* field points with r < r_exc are frozen (flat)        */
    double r_damp;          /* fields relax to their initial values below r_damp   */
    double damp_max;        /* relaxation fraction per step at r = r_exc            */
    double outer_layer;     /* width in cells of the outer absorbing layer (0: off, the
                               outer faces are frozen); single runs only             */
    double outer_damp;      /* its relaxation fraction per step at the faces, 0..1 */
    double B0[3];           /* initial (F^23, F^31, F^12), or covariant if flagged  */
    double charge[GRPIC_MAX_SPECIES]; /* macro-particle charge per species          */
    double mass[GRPIC_MAX_SPECIES];   /* macro-particle mass per species (> 0)      */
    double density[GRPIC_MAX_SPECIES];/* nominal macro-particles per unit cell volume
                                         per species, for the plasma-frequency check
                                         (Sec. 5.1); 0: not checked                */
    int64_t capacity;       /* particle slots to allocate                          */
    grpic_alloc_fn alloc;   /* optional device allocator (NULL: hipMalloc)          */
    grpic_free_fn free;
    void *alloc_ctx;
} grpic_config;

typedef struct {
    int64_t n_alive[GRPIC_MAX_SPECIES];
    int64_t n_removed_horizon; /* cumulative removals inside r_rm          */
    int64_t n_removed_outer;   /* cumulative removals at the outer boundary */
    int64_t gamma_clamps;      /* negative gamma discriminants clamped       */
    int64_t flags;             /* bit 0: a move > 1 cell (not deposited);
                                  bit 1: an int64 fixed-point sum (current or
                                  absorbed charge) left the int64 range     */
    double charge_total;
    double energy_particles;   /* sum M c (-u_4)                              */
    double lz_particles;       /* sum M (x u_y - y u_x), covariant u          */
    double energy_field;       /* (1/8pi)[sum -E_cov D + sum B_cov H]         */
    double gauss_residual_max; /* max |-div D - 4 pi rho| at checked nodes    */
    double mass_shell_residual_max; /* max |g(u,u) + c^2|                    */
    int64_t deposit_blocks_lds;    /* cumulative deposit blocks whose current was
                                      summed in an LDS box, then flushed       */
    int64_t deposit_blocks_global; /* ... added with global atomics instead     */
    int64_t push_blocks_lds;       /* cumulative push blocks with live particles
                                      that gathered from an LDS node box       */
    int64_t push_blocks_global;    /* ... that found no box within the LDS
                                      budget and gathered from global memory   */
} grpic_diag;

typedef struct grpic_s grpic_t;

/* Fill *cfg with the defaults for an nx x ny x nz grid: c = 1, dt = 0.5,
 * m = a = 0, centre at the grid centre, r_rm = 1.1 r_+, r_exc = 0.5 r_+,
 * r_damp = r_+, damp_max = 0.1, field_iters = 3, sort_every = 10, tile = 4,
 * fp_bits = 44, FP64, PAPER gamma, CURVED deposit, CLASSIC RK, STAGE gather,
 * TRILINEAR weights, one species (-1, 1). */
void grpic_config_default(grpic_config *cfg, int32_t nx, int32_t ny, int32_t nz);

/* sizeof(grpic_config) as this library was built, so bindings can check
 * their copy of the layout. */
size_t grpic_config_size(void);

/* The validation of grpic_create without creating a run (host only, no
 * device call): GRPIC_OK or GRPIC_EINVAL.  Besides the limits listed at
 * grpic_create it applies the plasma-frequency criterion of Sec. 5.1,
 * omega_p dt < 2 with omega_p^2 = 4 pi n q^2 / m for every species whose
 * nominal density n = cfg->density[s] is set (> 0), with the macro-particle
 * charge and mass.  The general-relativistic form of the criterion,
 * gamma^(-1/2) omega_p dt < 2, holds wherever the flat one does, since the
 * time-dilation factor gamma is at least 1. */
int grpic_config_check(const grpic_config *cfg);

/* Create a run.  Validates the configuration (grid >= 4 cells per axis,
 * 0 <= |a| <= m, c > 0, dt > 0, the Courant condition c dt < 1/sqrt(3) of
 * Sec. 5.2, the plasma-frequency criterion of Sec. 5.1 where densities are
 * given (grpic_config_check), r_exc < r_rm, masses > 0, rk_mode, gather_mode
 * and gather_weights at their defaults unless FP64, outer_layer >= 0,
 * 0 <= outer_damp <= 1) and initialises the fields (Sec. 6: uniform
 * contravariant field).  stream is a hipStream_t on which every call of the
 * run enqueues its work; NULL: the run creates a stream of its own (blocking,
 * so it stays ordered with the null stream both ways; default priority) and
 * destroys it in grpic_destroy.
 * Returns GRPIC_EINVAL, GRPIC_ENOMEM or GRPIC_EDEVICE on failure. */
int grpic_create(const grpic_config *cfg, void *stream, grpic_t **out);

/* Load n particles of one species.  x: host SoA [3][n] node coordinates;
 * ucov: host SoA [3][n] covariant spatial four-velocity u_1..u_3.  u_4 is
 * the future root of the mass shell g(u,u) = -c^2 (Sec. 2.1) and the stored
 * state is the contravariant u^a.  Particles with non-finite input, outside
 * [0, n)^3 or inside r_rm are dropped; *kept (may be NULL) receives the
 * number kept.  Synchronous.  GRPIC_ENOMEM if the capacity is exceeded. */
int grpic_load_particles(grpic_t *h, int32_t species, int64_t n, const double *x,
                         const double *ucov, int64_t *kept);

/* grpic_load_particles for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid
 * allocation): the same load, with the same arguments and results, but the
 * host arrays are staged in a fixed device array of the library instead of
 * a buffer allocated for the call, and no allocation happens.  At most
 * 1,048,576 particles per call (48 MiB of staging, 6 doubles a particle);
 * a larger n gives GRPIC_EINVAL with a message on stderr, and nothing is
 * loaded.  Load more with several calls.  Every device the library runs on
 * holds one copy of the staging array until the process ends, shared by all
 * runs on that device: calls on one device must not overlap (from several
 * threads, or with another run's call of this function), since they would
 * race on the staging.  Synchronous, like grpic_load_particles. */
int grpic_load_particles_noalloc(grpic_t *h, int32_t species, int64_t n, const double *x,
                                 const double *ucov, int64_t *kept);

/* Enqueue nsteps full cycles (Sec. 2.2 and Sec. 3): magnetic half-step,
 * RK4 push, magnetic half-step, current deposition, electric step, removal,
 * and a cell sort every sort_every steps.  Asynchronous.
 * Errors are sticky: once a call has failed, every later call returns the
 * same code.  GRPIC_EOVERFLOW: an int64 fixed-point sum of an earlier step
 * (the current of Sec. 4, or the charge absorbed at removal) left the int64
 * range, so the run's fields can no longer be trusted.  The device raises
 * the flag during the step; its value is copied to the host at the end of
 * each call, so the next call after that copy has completed (at the latest
 * once the stream has synchronised), or grpic_diagnostics, reports it. */
int grpic_step(grpic_t *h, int32_t nsteps);

/* Synchronise and compute the diagnostics (FP64, deterministic order).
 * *out is filled in every case; the return value is the run's sticky error,
 * GRPIC_EOVERFLOW when flags bit 1 is set. */
int grpic_diagnostics(grpic_t *h, grpic_diag *out);

/* Number of particle slots in use (alive or dead) and capacity. */
int grpic_particle_count(grpic_t *h, int64_t *n_slots, int64_t *capacity);

/* Copy the particle state to host: x [3][n] node coordinates, u [4][n]
 * contravariant four-velocity, sp [n] species (GRPIC_DEAD when removed);
 * n = the slot count of grpic_particle_count.  x and u of a GRPIC_DEAD slot
 * are unspecified (the pusher no longer writes them).  Synchronous. */
int grpic_dump_particles(grpic_t *h, double *x, double *u, uint8_t *sp);

/* Replace the particle state verbatim (the inverse of the dump).  n <= capacity. */
int grpic_restore_particles(grpic_t *h, int64_t n, const double *x, const double *u,
                            const uint8_t *sp);

/* Number of entries of one ghosted field component: (nx+3)(ny+3)(nz+3);
 * entry (i,j,k), i in [-1, nx+1], is at ((k+1)(ny+3) + j+1)(nx+3) + i+1, and a
 * component staggered by +1/2 along an axis stores i+1/2 at index i. */
int64_t grpic_field_size(const grpic_t *h);

/* Copy fields to host, each [3][field_size] doubles.  which: 0 D = F^{j4},
 * 1 B_cov = (F_23, F_31, F_12), 2 E_cov = F_{j4}, 3 H = (F^23, F^31, F^12),
 * 4 J (current of the last step).  Synchronous. */
int grpic_dump_fields(grpic_t *h, int32_t which, double *out);

/* Replace the evolved fields D and B_cov (each [3][field_size]). */
int grpic_restore_fields(grpic_t *h, const double *D, const double *B);

/* Checkpoint and resume.  A state holds everything a run carries from one
 * cycle to the next: the evolved fields D and B_cov, the particle slots
 * (order, species, x, u), the absorbed charge of the removal, the device
 * counters and the cycle count (which schedules the cell sort), plus a
 * header with the configuration it was saved under.  A run created with the
 * same configuration (capacity may differ, allocator ignored) that loads the
 * state continues bit-identically to the run that saved it.
 *
 * The particles are kept as the run stores them (FP64: positions and
 * four-velocities as doubles; FP32-mixed: the packed cell, FP32 offsets and
 * FP32 four-velocity), so a resumed run holds the same bits.
 *
 * grpic_state_bytes: the size of the run's current state in bytes (< 0: an
 * error code).
 * grpic_save_state: write it into buf (host memory, 8-byte aligned, bytes >=
 * the state size; the caller owns buf).  Synchronous.
 * grpic_load_state: replace the run's state by one saved earlier.  Returns
 * GRPIC_EINVAL for a misaligned or short buffer, a buffer that is not a state
 * of this format, a different configuration, or more slots than the capacity;
 * the run is unchanged then.  Synchronous. */
int64_t grpic_state_bytes(grpic_t *h);
int grpic_save_state(grpic_t *h, void *buf, int64_t bytes);
int grpic_load_state(grpic_t *h, const void *buf, int64_t bytes);

/* Copy the node tensor F^a_b of the last step, [(nx+1)(ny+1)(nz+1)][4][4]. */
int grpic_dump_nodes(grpic_t *h, double *out);

/* Push the particles nsteps times with the node tensor frozen and without
 * deposition, removal or field update (test-particle mode).  Recomputes the
 * node tensor from the current fields first. */
int grpic_push_only(grpic_t *h, int32_t nsteps);

/* Stable cell sort now, by key then particle order.  The key of a live
 * particle in cell (i,j,k) is rank * T^3 + local with T = cfg->tile, rank
 * the tile's place on a path through all tiles on which consecutive tiles
 * share a face (the planes of tiles in z order; rows of tiles in y order in
 * even planes and reversed in odd ones; tiles in x order in even rows and
 * reversed in odd ones, counting rows across the planes), and local =
 * (layer T + slow) T + fast the cell's place inside its tile: layer counts
 * the tile's T cell layers across the axis along which the path leaves the
 * tile (along its row; from a row's last tile along y; from a plane's last
 * tile along +z), the exit side last; slow and fast are the cell's other two
 * tile coordinates, the larger axis slow.  The paper has no sort; this one
 * keeps the particles of a block of threads in a few neighbouring cells, also
 * where the block straddles two tiles.
 * If keys_out is not NULL it receives the sorted keys of all slots
 * (dead particles: 0xFFFFFFFF), and perm_out the original slot index of each
 * sorted position; with both NULL nothing is copied to the host.  Dead
 * particles are compacted away afterwards. */
int grpic_sort(grpic_t *h, uint32_t *keys_out, int64_t *perm_out);

/* Kernel timing with HIP events recorded on the run's stream around each
 * kernel group: PUSH (gather + RK4 pusher), DEPOSIT (current + removal),
 * FIELDS (every field kernel of a step), SORT.  Off by default. */
enum { GRPIC_TIMER_PUSH = 0, GRPIC_TIMER_DEPOSIT = 1, GRPIC_TIMER_FIELDS = 2, GRPIC_TIMER_SORT = 3,
       GRPIC_NTIMERS = 4 };
int grpic_set_timing(grpic_t *h, int32_t enable);

/* Launch each cycle's kernels (all but the cell sort) as one captured HIP
 * graph (enable != 0, the default) or one by one.  A run captures the cycle
 * once per buffer parity and slot count and replays it, which removes the
 * host's launch work from the steps; while timing is on the kernels are
 * launched one by one, so every group can be bracketed with events.  The
 * results are bit-identical either way.  Capture needs a stream other than
 * the null stream, which every run has (grpic_create).
 * Disabling synchronises the run's stream and frees the graphs. */
int grpic_set_graphs(grpic_t *h, int32_t enable);

/* Synchronise; ms[t] receives the summed event time of timer t and
 * launches[t] the number of timed groups since the previous read (both
 * arrays of GRPIC_NTIMERS entries, either may be NULL).  Resets the sums. */
int grpic_read_timing(grpic_t *h, double *ms, int64_t *launches);

/* Synchronise; *out = particle pushes performed since creation (the sum
 * over steps of the live particles pushed). */
int grpic_particle_steps(grpic_t *h, int64_t *out);

void grpic_destroy(grpic_t *h);
const char *grpic_strerror(int code);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of independent FP32-mixed runs.  A batch
 * owns up to max_slots (at most 64) runs whose device memory together stays
 * within budget_bytes.  Each admitted run keeps its state on the device
 * until it finishes or is preempted (grpic_batch_preempt).
 * One batch iteration advances every active run by one cycle with a single
 * set of batched launches (one per stage of the cycle, each covering the
 * particles or grid points of all runs), captured once as a HIP graph and
 * replayed; a run table in device memory, rewritten before each replay,
 * tells the launches which runs are active and where their state is.  The
 * cell sort, when due, runs per run after the replay.  Runs that reach
 * their step count are finished: their diagnostics are taken and their
 * memory is freed at once, which admits queued work.  All work of a batch
 * runs on its own HIP stream.  One batch is not thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct grpic_batch_s grpic_batch_t;

enum { GRPIC_RUN_UNKNOWN = 0, GRPIC_RUN_ACTIVE = 1, GRPIC_RUN_DONE = 2, GRPIC_RUN_PREEMPTED = 3 };

/* Device bytes a run with this configuration allocates (admission estimate). */
int64_t grpic_run_bytes(const grpic_config *cfg);

/* GRPIC_EINVAL unless 1 <= max_slots <= 64 and budget_bytes > 0. */
int grpic_batch_create(int64_t budget_bytes, int32_t max_slots, grpic_batch_t **out);

/* Admit a run if a slot and budget_bytes allow it (else GRPIC_EAGAIN and no
 * state changes).  Particles of species s (s < cfg->nspecies): n[s] entries,
 * x[s] and ucov[s] as for grpic_load_particles; cfg->precision must be
 * GRPIC_FP32_MIXED, cfg->alloc NULL (the batch allocates) and the outer
 * absorbing layer off, else GRPIC_EINVAL.  Waits for the batch's queued work.  The run advances one cycle per grpic_batch_step until
 * nsteps are done.  keep_state != 0 keeps a host copy of the final particle
 * state for grpic_batch_dump. */
int grpic_batch_submit(grpic_batch_t *b, const grpic_config *cfg, int32_t nsteps, int32_t keep_state,
                       const int64_t *n, const double *const *x, const double *const *ucov, int64_t *run_id);

/* One cycle of every active run.  *finished receives how many runs
 * completed in this iteration. */
int grpic_batch_step(grpic_batch_t *b, int32_t *finished);

/* State of a run (GRPIC_RUN_*), cycles done, and for a finished run its
 * diagnostics, the slot count of its kept final state (0 if not kept) and
 * the particle pushes it performed.
 * Unknown or released ids give GRPIC_RUN_UNKNOWN.  Pointers may be NULL. */
int grpic_batch_poll(grpic_batch_t *b, int64_t run_id, int32_t *state, int32_t *steps_done, grpic_diag *diag,
                     int64_t *n_slots, int64_t *particle_steps);

/* Copy a finished run's kept final particle state (layout of grpic_dump_particles). */
int grpic_batch_dump(grpic_batch_t *b, int64_t run_id, double *x, double *u, uint8_t *sp);

/* Forget a finished or preempted run (its device memory was already
 * returned at completion or preemption).  GRPIC_ESTATE for an active run. */
int grpic_batch_release(grpic_batch_t *b, int64_t run_id);

/* Preemption, built on the checkpoint format of grpic_save_state.
 *
 * grpic_batch_state_bytes: the size of an active run's state (< 0: an error
 * code; GRPIC_ESTATE unless the run is active).
 * grpic_batch_preempt: wait for the batch's queued work, save the active
 * run's state into buf (host memory, 8-byte aligned, bytes >= the state
 * size; the caller owns it), then free the run's device memory and slot.
 * The run keeps its id and cycle count in state GRPIC_RUN_PREEMPTED and no
 * longer advances.  On an error (a short or misaligned buffer: GRPIC_EINVAL)
 * the run stays active and unchanged.
 * grpic_batch_resume: re-admit a preempted run from the state its preemption
 * saved, when a slot and the budget allow it (else GRPIC_EAGAIN, nothing
 * changes).  A state saved under another configuration or after a different
 * number of cycles than the run has done gives GRPIC_EINVAL, and the run
 * stays preempted.  Resumed from the state its preemption saved, the run
 * continues bit-identically to a run that was never preempted, and finishes
 * after the nsteps it was submitted with.
 * Unknown ids give GRPIC_EINVAL. */
int64_t grpic_batch_state_bytes(grpic_batch_t *b, int64_t run_id);
int grpic_batch_preempt(grpic_batch_t *b, int64_t run_id, void *buf, int64_t bytes);
int grpic_batch_resume(grpic_batch_t *b, int64_t run_id, const void *buf, int64_t bytes);

/* Active runs and device bytes they hold. */
int grpic_batch_stats(grpic_batch_t *b, int32_t *active, int64_t *bytes_in_use);

void grpic_batch_destroy(grpic_batch_t *b);

#ifdef __cplusplus
}
#endif
#endif /* GRPIC_H */
