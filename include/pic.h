/*
 * pic.h - C ABI of the MI355X (gfx950) 1D3V particle-in-cell hot path with
 * radiation reaction, after Tamburini et al., "Radiation Reaction Effects on
 * Radiation Pressure Acceleration".
 *
 * What one step computes (pic_step):
 *   1. gather E^n, B^n at every particle by linear weighting on a 1D Yee grid;
 *   2. Boris push for the Lorentz force, u^{n-1/2} -> u_L^{n+1/2} (Section 3);
 *   3. for electrons, the radiation-reaction force of Eq. (f_r), evaluated at
 *      the mid-step estimate of Eqs. (estim1), (estimgamma), added by the
 *      leapfrog superposition of Eq. (pertfull): u^{n+1/2} = u_L + dt f_R;
 *   4. leapfrog move x^{n+1} = x^n + dt u^{n+1/2} / gamma^{n+1/2};
 *   5. charge-conserving current deposition in 64-bit fixed point;
 *   6. Yee field advance with laser injection at x = 0 and absorbing ends;
 *   7. every sort_interval steps, a counting sort of particles by cell.
 * The grid, shape, deposition, solver and boundaries are not specified by
 * the paper ("a standard PIC code", Section 3); the choices are documented
 * with each entry point and in the library's design notes.
 *
 * Units (Section 2): t in 1/omega, x in c/omega, momentum in m c, fields in
 * m omega c/|e|, densities in n_c.  One laser wavelength = one period = 2 pi.
 *
 * Conventions for every entry point:
 *   - Return value: PIC_OK (0) or a negative pic_status; no C++ exception
 *     crosses the ABI.  On error pic_last_error() returns a thread-local
 *     message describing the first failure.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Entry points marked "async" only enqueue work on it; "blocking" ones
 *     synchronise it before returning.  Errors of asynchronous work surface
 *     at the next blocking call.
 *   - The library never allocates device memory: the caller owns one
 *     device workspace per run (size from pic_workspace_bytes), keeps it
 *     alive until pic_free, and owns the stream.  A pic_run handle owns only
 *     host metadata.
 *   - A run is not thread-safe; different runs may be used from different
 *     threads.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_ABI_VERSION 2

typedef enum pic_status {
  PIC_OK = 0,
  PIC_EINVAL = -1,     /* invalid argument or configuration */
  PIC_ENOMEM = -2,     /* workspace too small / capacity exceeded */
  PIC_EHIP = -3,       /* HIP runtime error */
  PIC_ENONFINITE = -4, /* a particle momentum or position became NaN/Inf */
  PIC_EBUSY = -5       /* no free slot in a batch */
} pic_status;

enum pic_precision { PIC_FP32 = 0, PIC_FP64 = 1 };
enum pic_polarisation { PIC_LP = 0, PIC_CP = 1 };

/* Run configuration (caller-owned, copied by pic_init).
 * Geometry: box of box_lambda wavelengths, cells_per_lambda cells per
 * wavelength (n_cells = round(box_lambda * cells_per_lambda)), dt = cfl*dx
 * with 0 < cfl <= 0.5 so that no particle crosses more than one cell edge.
 * Laser (Section 4): enters at x = 0 from t = 0; LP: E_y = a0 f(t) sin t;
 * CP: E_y = (a0/sqrt2) f sin t, E_z = (a0/sqrt2) f cos t (same intensity for
 * the same a0); f = sin^2 rise over t_rise periods, 1 for t_flat periods,
 * sin^2 fall over t_fall periods.
 * Foil (Section 4): electrons and protons (mass_ratio electron masses),
 * density n0 n_c, front at x_foil wavelengths, thickness wavelengths; ppc
 * particles per cell per species on a quiet start (offsets ((k + 1/2) +
 * jitter (U - 1/2)) / ppc, U the SplitMix64 output number i of the stream
 * seeded with `seed`, i the particle index; both species share positions),
 * cold, weight n0 dx / ppc.
 * Radiation reaction (Section 3): on electrons when rr != 0, with strength
 * (4 pi / 3) r_e / lambda for the wavelength lambda_um in micrometres.
 * rr_compensated (fp32 only): the RR increment is added with a
 * compensated (TwoSum) sum whose rounding residual is carried per particle. */
typedef struct pic_config {
  uint32_t struct_size;      /* sizeof(pic_config) of the caller */
  int32_t precision;         /* PIC_FP32 or PIC_FP64 storage and arithmetic */
  double lambda_um;          /* laser wavelength in micrometres (> 0) */
  int32_t cells_per_lambda;  /* >= 4 */
  int32_t ppc;               /* particles per cell per species (>= 1) */
  double box_lambda;         /* box length in wavelengths */
  double cfl;                /* dt / dx, in (0, 0.5] */
  int32_t pol;               /* PIC_LP or PIC_CP */
  int32_t rr;                /* radiation reaction on electrons (0/1) */
  double a0;                 /* normalised laser amplitude */
  double t_rise, t_flat, t_fall; /* envelope, in periods */
  double n0;                 /* foil density in n_c */
  double x_foil;             /* foil front, wavelengths */
  double thickness;          /* foil thickness, wavelengths */
  double mass_ratio;         /* ion / electron mass (ion charge +1) */
  int32_t rr_compensated;    /* 0/1, fp32 only */
  int32_t sort_interval;     /* steps between sorts (>= 1) */
  uint64_t seed;             /* quiet-start jitter seed */
  double jitter;             /* jitter amplitude in units of the spacing, [0, 1] */
  int64_t capacity;          /* particles per species to reserve; 0 = foil count */
} pic_config;

/* Run constants derived by pic_init (read-only). */
typedef struct pic_info {
  int32_t n_cells;
  int32_t precision;
  double dx, dt, eps_rr, w_ref;
  int64_t capacity;          /* per species */
  int64_t n_init[2];         /* particles per species after pic_init */
  int64_t step;              /* steps enqueued so far */
  int32_t tile;              /* particles per push work-group of a single run: 5120, or 1024 when
                                the foil gives fewer than two 5120-particle tiles per compute unit
                                (chosen at pic_init; batched steps use 1024) */
  int32_t lds_slots;         /* 64-bit LDS current accumulators per push work-group */
} pic_info;

/* Diagnostics at the current step n (particles at x^n with u^{n-1/2},
 * fields E^n, B^n): the energy balance of Section 2, in which the field and
 * kinetic energies plus the energy radiated by the RR force (a loss, counted
 * as it is emitted) and the energy that left the box account for the laser
 * energy that entered it.  Energies are in units of
 * m^2 omega^2 c^2 / (4 pi e^2) per unit transverse area (field: sum of
 * field^2/2 dx; particle: sum of w M (gamma - 1)); all reductions in FP64. */
typedef struct pic_diag_out {
  int64_t step;
  double t;
  int64_t n_alive[2];        /* electrons, ions */
  double U_Ex, U_Et, U_B;    /* longitudinal E, transverse E, B field energy */
  double K_e, K_i;           /* kinetic energy from u^{n-1/2} */
  double E_rad;              /* cumulative RR loss, sum w (gamma_L - gamma^{n+1/2}) */
  double E_in;               /* cumulative incident laser energy at x = 0 */
  double E_out_left, E_out_right; /* cumulative outgoing field energy */
  double E_esc;              /* cumulative kinetic energy of removed particles */
  double gauss;              /* max |dEx/dx - rho| over nodes 1..n-1 (field units) */
  int64_t gauss_int;         /* the same residual in the integer units (expect 0) */
  int64_t n_stiff;           /* RR pushes with dt|f_R| > 0.1 |u_L| (cumulative) */
  int32_t nonfinite;         /* 1 if a NaN/Inf particle was seen */
  int32_t reserved;
  double U_field;            /* U_Ex + U_Et + U_B */
  double balance;            /* U_field + K_e + K_i + E_rad + E_out_left + E_out_right
                                + E_esc - E_in (0 for exact conservation) */
} pic_diag_out;

/* Host-side particle and field state for pic_get_state / pic_set_state.
 * Arrays of type `real` are float for PIC_FP32 runs and double for PIC_FP64.
 * Any pointer may be NULL to skip that array (get) or leave it unchanged
 * (set; particle arrays must then all be given or all be NULL).
 * Grid layout: node i (x = i dx, i = 0..n) for Ey, Ez; half-node h
 * (x = (h - 1/2) dx, h = 0..n+1, h = 0 and n+1 are boundary guards) for
 * Ex, By, Bz.  Integer currents: Jx_int on half-nodes (n + 2 entries),
 * Jy_int, Jz_int on nodes -1..n+1 stored at index node + 1 (n + 3 entries);
 * Ex_int on half-nodes (n + 2).  Fixed-point scale: Ex = Ex_int w_ref 2^-32,
 * Jx = Jx_int w_ref 2^-32 / dt, Jy = Jy_int w_ref 2^-32 / dx. */
typedef struct pic_species_state {
  int64_t count;             /* get: alive count after compaction; set: count */
  int32_t* cell;             /* [count] cell index, 0..n-1 */
  void* off;                 /* [count] real offset in [0, 1) */
  void* ux; void* uy; void* uz; /* [count] real momentum u^{n-1/2} (p / M c) */
  void* w;                   /* [count] real weight (density x length) */
  float* rx; float* ry; float* rz; /* [count] fp32 RR residuals (electrons) */
} pic_species_state;

/* Cumulative budget terms of a run (the time integrals of the energy
 * balance above), carried by a checkpoint so that a resumed run continues
 * its balance instead of restarting it from zero. */
typedef struct pic_budget_state {
  int32_t valid;             /* get: set to 1; set: 1 = replace the run's totals, 0 = keep them */
  int32_t nonfinite;         /* the run's non-finite flag */
  double E_in, E_out_left, E_out_right; /* energy through the boundaries */
  double E_rad;              /* RR loss */
  double E_esc[2];           /* kinetic energy of removed electrons, ions */
  double n_stiff;            /* stiff RR pushes */
} pic_budget_state;

typedef struct pic_state {
  pic_species_state sp[2];
  void* Ex; void* Ey; void* Ez; void* By; void* Bz; /* real arrays, see above */
  int64_t* Ex_int;           /* [n + 2] */
  int64_t* Jx_int;           /* [n + 2] current deposited at the current step */
  int64_t* Jy_int;           /* [n + 3] */
  int64_t* Jz_int;           /* [n + 3] */
  int64_t step;              /* step counter n (set: also sets the laser clock) */
  pic_budget_state budget;   /* cumulative budget terms and the non-finite flag */
} pic_state;

/* The run handle: opaque, owned by the library (pic_init creates it,
 * pic_free destroys it).  Declared here at file scope so that the
 * prototypes below refer to one type in C as in C++. */
struct pic_run;

/* Workspace bytes a run with `cfg` needs (host-only; no GPU access). */
pic_status pic_workspace_bytes(const pic_config* cfg, size_t* bytes);

/* Validate cfg, carve the caller's device workspace d_ws (ws_bytes bytes,
 * 256-byte aligned) and initialise the quiet-start foil, zero fields and
 * budgets.  Async on `stream`.  On success *out is a new handle. */
pic_status pic_init(const pic_config* cfg, void* d_ws, size_t ws_bytes,
                    void* stream, struct pic_run** out);

/* Enqueue n_steps full steps (push-deposit, field advance, periodic sort).
 * Async.  Particles leaving [0, n dx) are removed. */
pic_status pic_step(struct pic_run* run, int64_t n_steps, void* stream);

/* Compute diagnostics on the device (FP64), copy them to *out.  Blocking.
 * Returns PIC_ENONFINITE (with *out filled) if a non-finite particle was
 * seen since pic_init. */
pic_status pic_diag(struct pic_run* run, pic_diag_out* out, void* stream);

/* Copy run constants. Host-only. */
pic_status pic_get_info(const struct pic_run* run, pic_info* out);

/* Release host metadata; the workspace stays owned by the caller. */
void pic_free(struct pic_run* run);

/* Message of the last failed call on this thread ("" if none). */
const char* pic_last_error(void);

/* Bound the work-groups of one launch of the push and of the sort passes
 * (0, the default: one launch per pass).  A run of 2e8 particles pushes in
 * about 39,000 work-groups per step; split into launches of a few thousand,
 * kernels that other streams enqueue meanwhile (small runs served beside
 * it) are dispatched between the pieces instead of after the whole pass.
 * Results do not change.  Host-only. */
pic_status pic_set_max_grid(struct pic_run* run, int32_t max_workgroups);

/* Stage entry points (one kernel each), for tests and profiling.  Async.
 *   pic_push_deposit: steps 1-5 for every particle; leaves J_int of this
 *     push in the run (readable with pic_get_state) and does not advance
 *     the fields or the step counter.
 *   pic_field_advance: step 6 with the J_int left by the last push; advances
 *     the step counter.
 *   pic_sort: step 7 now (compacts removed particles). */
pic_status pic_push_deposit(struct pic_run* run, void* stream);
pic_status pic_field_advance(struct pic_run* run, void* stream);
pic_status pic_sort(struct pic_run* run, void* stream);

/* Checkpoint / test I/O of the full state (host buffers).  Blocking.
 * Particle arrays given to pic_get_state must hold `capacity` entries
 * (pic_get_info); removed particles are skipped, so counts are alive counts
 * (all particle arrays NULL: fields and currents only, count set to 0).
 * pic_get_state always fills `budget` (valid = 1).
 * pic_set_state validates cells and offsets, replaces the particle arrays
 * (count <= capacity; the current buffers of both parities are cleared when
 * particles are replaced) and/or fields, Ex_int and the current buffers of
 * the current step; step >= 0 also resets the step counter; budget.valid = 1
 * replaces the cumulative budget terms and the non-finite flag.
 * A state taken at step n and set into a fresh run of the same
 * configuration continues as the original run would: particles, fields and
 * integer currents, the boundary energies and every integer diagnostic
 * repeat bit for bit; FP64 sums over particles (kinetic, radiated, escaped
 * energy) agree to rounding, since their order follows the particle order
 * within a cell, which the sort leaves open. */
pic_status pic_get_state(struct pic_run* run, pic_state* st, void* stream);

/* Raw read of particles first .. first + count - 1 of one species (0
 * electrons, 1 protons) from the current buffers, without compaction:
 * removed particles keep their slot, with cell = INT32_MIN, until the next
 * sort.  Indices do not change between sorts, so reads before and after
 * pic_push_deposit see the same particles.  Copies min(count, n - first)
 * entries (n: the species' current slot count) into the host arrays of
 * *out (any may be NULL; residuals exist for FP32 electrons with
 * compensation only) and sets out->count to that number.  Blocking. */
pic_status pic_get_particles(struct pic_run* run, int32_t species, int64_t first, int64_t count,
                             pic_species_state* out, void* stream);
pic_status pic_set_state(struct pic_run* run, const pic_state* st, void* stream);

/* Ion energy spectrum (Section 4 spectra): weighted histogram of proton
 * kinetic energy (gamma - 1) mass_ratio 0.51099895 MeV in `bins` bins on
 * [0, e_max_mev), weights summed exactly in fixed point; host_hist gets
 * protons per MeV (weight / bin width).  Blocking. */
pic_status pic_spectrum(struct pic_run* run, int32_t bins, double e_max_mev,
                        double* host_hist, void* stream);

/* pic_spectrum for callers that cannot allocate device memory: the same
 * histogram, with its counters in a fixed device array inside the library
 * (512 KiB per device, held until the process ends) instead of the run's
 * workspace.  At most 65536 bins (more: PIC_EINVAL).  host_hist (bins
 * doubles) also serves as the staging buffer of the counts, so the call
 * allocates nothing.  Every call on one device shares that array: calls
 * that overlap on one device (several threads, or streams running at once)
 * race and must be serialised by the caller; each call clears the bins it
 * uses.  Blocking. */
pic_status pic_spectrum_static(struct pic_run* run, int32_t bins, double e_max_mev,
                               double* host_hist, void* stream);

/* Friction coefficient of Eq. (damping), the strength of the RR force in
 * units of m omega c (Section 2): d = eps gamma^2 [f_L^2 - (v.f_L)^2] with
 * f_L = -(E + v x B), for every electron at the current step (E^n, B^n
 * gathered at x^n as the push gathers them, v from the stored momentum),
 * in FP64.  host_hist[bins]: electron weight (density x length) with
 * log10 d in bin floor((log10 d - log10_lo) / (log10_hi - log10_lo) bins);
 * host_stats[4]: the maximum of d, the weight-averaged d, the weight with
 * d <= 0 or log10 d < log10_lo, and the weight with log10 d >= log10_hi.
 * bins <= 65531.  Blocking. */
pic_status pic_friction(struct pic_run* run, int32_t bins, double log10_lo, double log10_hi,
                        double* host_hist, double* host_stats, void* stream);

/* ------------------------------------------------------------------------
 * Test electrons in a given plane wave (the single-particle tests of
 * Section 3): independent of any run.  The wave travels along +x with
 * A_y = a_y sin(phi + psi), A_z = a_z cos(phi + psi), phi = t - x,
 * E = (0, -dA_y/dphi, -dA_z/dphi), B = (0, -E_z, E_y) (a_z = 0: linear
 * polarisation); units as in the runs.
 * scheme PIC_TRACK_LEAPFROG: the pusher of the runs (Boris plus the RR
 *   step of Eqs. (estim1)-(pertfull)); on entry x = x^0 at time t0 and
 *   u = u^{-1/2}, on return x^{steps} and u^{steps - 1/2}.  FP32 adds the
 *   RR increment by TwoSum as the runs do; the returned u includes the
 *   carried residual.
 * scheme PIC_TRACK_RK4: classical fourth-order Runge-Kutta of Eq. (3dLL),
 *   x and u both at t0 on entry and at t0 + steps dt on return.
 * rr: PIC_RR_OFF (Lorentz force), PIC_RR_REDUCED (plus the non-derivative
 *   terms of Eq. (3dLL), i.e. Eq. (f_r): the force of the runs), PIC_RR_FULL
 *   (plus the derivative term, with the wave's exact field derivatives).
 * precision: arithmetic of the momentum step (positions and phases FP64).
 * d_x, d_ux, d_uy, d_uz: device arrays of n doubles (x: position along the
 * propagation direction), updated in place.  Asynchronous on stream; invalid
 * arguments return PIC_EINVAL before any launch. */
typedef struct pic_wave {
  double a_y, a_z, psi;
} pic_wave;

enum { PIC_TRACK_LEAPFROG = 0, PIC_TRACK_RK4 = 1 };
enum { PIC_RR_OFF = 0, PIC_RR_REDUCED = 1, PIC_RR_FULL = 2 };

pic_status pic_track(const pic_wave* wave, int32_t scheme, int32_t rr, int32_t precision,
                     double lambda_um, double dt, double t0, int64_t steps, int64_t n, double* d_x,
                     double* d_ux, double* d_uy, double* d_uz, void* stream);

/* Self-check of the move arithmetic (the correctly rounded square root and
 * reciprocal of the deposition contract are computed from hardware estimates
 * plus FMA corrections): for every float whose bit pattern lies in
 * [first, first + count) and that is finite and >= 1, compare with the
 * compiler's correctly rounded sqrtf and 1.0f / x (the reciprocal below 2^126
 * only) and add the number of differing results to *d_mismatches, a device
 * counter the caller zeroes and reads.  Asynchronous on stream; first + count
 * above 2^32 is PIC_EINVAL. */
pic_status pic_check_rounding(uint32_t first, uint32_t count, unsigned long long* d_mismatches,
                              void* stream);

/* Per-kernel timing for profiling: with period p > 0, every p-th launch of
 * each kernel kind records a HIP event pair at its own start and end
 * (hipExtLaunchKernel), so the time is the kernel's execution (for the sort,
 * from the start of its first pass to the end of its last); p = 1 times
 * every launch, p = 0 turns timing off and p < 0 is PIC_EINVAL.  pic_timing_read synchronises the stream and returns
 * the accumulated milliseconds and the number of timed launches for kernel
 * k = 0 push-deposit, 1 field advance, 2 sort (all passes). */
pic_status pic_timing_enable(struct pic_run* run, int32_t period);
pic_status pic_timing_read(struct pic_run* run, double ms[3], int64_t launches[3],
                           void* stream);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of independent runs (laser-foil requests of
 * uneven size).  A batch keeps a device table of up to max_slots resident
 * runs and advances all of them with the same launches: per quantum
 * (= the runs' sort_interval steps) one sort stage (hist, scan, scatter) and
 * then, per step, one push-deposit and one field launch whose work-groups
 * are spread over the runs' tiles (the field launch also advances each
 * run's step counter), or, in the persistent form (pic_batch_set_persistent),
 * one launch that runs all the quantum's steps with grid-wide barriers
 * between the passes.  Each run derives its buffer
 * parities, sort schedule and laser clock from its own device step counter,
 * so the quantum is captured once into a HIP graph and replayed while runs
 * join and leave; every run executes exactly the kernels it would execute
 * alone, so its fields and integer currents are bit-identical to a run
 * stepped alone (particle order within a cell may differ).
 * The caller owns the batch workspace (pic_batch_workspace_bytes) and every
 * run's workspace; admission by device-memory budget is the caller's policy
 * (the Python server implements one).  The stream must not be the null
 * stream (graph capture).  A run inside a batch rejects the single-run
 * entry points (PIC_EBUSY) until it is released.
 * ------------------------------------------------------------------------ */
typedef struct pic_batch pic_batch;

/* Bytes of the batch workspace (host-only). */
pic_status pic_batch_workspace_bytes(int32_t precision, int32_t max_slots, size_t* bytes);

/* Create a batch.  max_particles / max_cells bound the total particles
 * (both species) and cells of all resident runs; they size the captured
 * launches.  Blocking (initialises the slot table on `stream`). */
pic_status pic_batch_create(int32_t precision, int32_t max_slots, int32_t quantum,
                            int64_t max_particles, int64_t max_cells, void* d_ws,
                            size_t ws_bytes, void* stream, pic_batch** out);

/* Admit a run at step 0 (fresh from pic_init) to be advanced to step
 * n_steps.  Its sort_interval must equal the quantum and its precision the
 * batch's.  PIC_EBUSY if no slot or work capacity is free now; PIC_EINVAL
 * if the run exceeds the capacity of an empty batch.  Blocking. */
pic_status pic_batch_admit(pic_batch* b, struct pic_run* run, int64_t n_steps, void* stream,
                           int32_t* slot);

/* Whether a run of configuration cfg would be admitted, before any device
 * memory is set aside for it: *now = 1 if a slot and the work capacity are
 * free at this moment, *ever = 1 if it fits an empty batch (0: it can never
 * be admitted).  PIC_EINVAL for an invalid config or one whose precision or
 * sort_interval the batch cannot take.  Host-only. */
pic_status pic_batch_fits(const pic_batch* b, const pic_config* cfg, int32_t* now, int32_t* ever);

/* Enqueue n_quanta graph replays (quantum steps each) for every resident
 * run; runs stop at their n_steps.  Async.  The first call captures the graph. */
pic_status pic_batch_step(pic_batch* b, int32_t n_quanta, void* stream);

/* Copy every slot's current step to steps[max_slots] (-1 for free slots).
 * PIC_EHIP if a persistent launch timed out in a grid barrier (its steps
 * are not valid; the batch stays in error).  Blocking. */
pic_status pic_batch_poll(pic_batch* b, int64_t* steps, void* stream);

/* Queue a poll of every slot's step behind the replays already queued on
 * `stream`, without waiting: the counters land in pinned host memory the
 * batch owns.  One poll may be queued at a time (PIC_EINVAL otherwise).
 * With pic_batch_poll_wait this keeps the device busy while the host reads
 * the previous round's steps.  Async. */
pic_status pic_batch_poll_async(pic_batch* b, void* stream);

/* Wait for the queued poll and copy its steps to steps[max_slots]: -1 for
 * slots free now or whose run was admitted or released after the poll was
 * queued (their counters belong to another run).  PIC_EINVAL if no poll is
 * queued; PIC_EHIP as pic_batch_poll.  Blocking (on the poll only). */
pic_status pic_batch_poll_wait(pic_batch* b, int64_t* steps);

/* Advance every resident run to its n_steps: poll, enqueue the graph
 * replays the longest remainder needs, poll again.  *quanta (may be null)
 * receives the number of replays enqueued.  Runs stay resident (release
 * them to read their state).  Blocking. */
pic_status pic_batch_drain(pic_batch* b, int64_t* quanta, void* stream);

/* Choose how a quantum's steps are launched: on = 0 (default), one
 * push-deposit and one field launch per step, 2 x quantum launches after the
 * sort; on = 1, one persistent launch per quantum whose work-groups (as many
 * as the work needs, no more than fit the device at once) loop over the
 * push tiles and then the field chunks of every run, with a grid-wide
 * barrier after each pass, and advance the step counters once at the end.
 * Both forms execute the same per-particle and per-node arithmetic, so a
 * run's fields, integer currents and particles are bit-identical either way
 * (Section 2 leapfrog cycle: gather-push-deposit, then the field advance).
 * on = 2 is the persistent form with every grid-barrier wait cut to zero:
 * the launch still finishes but its barrier waits time out, its steps are
 * not valid and the next poll returns PIC_EHIP (a test of that error path;
 * the batch stays in error).
 * The persistent launch's work-groups wait for each other at the barriers,
 * so they must all be resident at once: keep other launches (another
 * batch's included) off the device while its replays run.  A barrier wait
 * longer than about a second ends the launch and the next poll returns
 * PIC_EHIP, as above.
 * The persistent form needs max_slots <= 128 (PIC_EINVAL otherwise).  Takes
 * effect at the next pic_batch_step (the graph is captured again).  Call it
 * while no replay of the batch is in flight (before the first
 * pic_batch_step, or after pic_batch_poll / pic_batch_drain): the old graph
 * is destroyed here.  Host-only. */
pic_status pic_batch_set_persistent(pic_batch* b, int32_t on);

/* Detach the run of `slot` (its state stays in its workspace; pic_diag and
 * the other single-run calls work again).  Blocking. */
pic_status pic_batch_release(pic_batch* b, int32_t slot, void* stream);

/* Destroy the batch (detaches resident runs; the workspace stays the caller's). */
void pic_batch_free(pic_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* PIC_H */
