/*
 * pic2d.h - C ABI of the 2D3V form of the hot path: the same step as
 * pic.h (gather, Boris push, radiation reaction of Eq. (f_r) on electrons
 * by the leapfrog splitting of Section 3, leapfrog move, charge-conserving
 * fixed-point deposition, Yee field advance, periodic cell sort) on a 2D
 * grid, x by y, periodic in y.  Section 4 points out that the momentum
 * space of the 1D code is already three dimensional, so a multi-dimensional
 * code uses the same particle pusher; this library runs the pusher of the
 * 1D kernels unchanged except that B_x is no longer zero.
 *
 * Conventions (status codes, streams, workspace ownership, thread safety,
 * pic_last_error) are those of pic.h.  Units as in pic.h; dy = dx.
 *
 * Readings the paper leaves open (it gives no multi-dimensional scheme):
 *   - Grid: 2D Yee.  With node i at x = i dx (i = 0..nx), half-node h at
 *     x = (h - 1/2) dx (h = 0..nx+1, the ends are boundary guards), row j at
 *     y = j dy and half-row g at y = (g + 1/2) dy (j, g = 0..ny-1):
 *       E_z (node, row); E_y, B_x (node, half-row); E_x, B_y (half-node, row);
 *       B_z (half-node, half-row).
 *     Maxwell with d/dz = 0; B in two half steps around the E step.
 *   - Boundaries: per row, the first-order Silver-Mueller guards of pic.h at
 *     both x ends, the laser entering at x = 0; periodic in y for fields and
 *     particles; particles leaving [0, nx dx) are removed.
 *   - Laser: the incident field of pic.h times exp(-((y - L_y/2)/W)^2),
 *     W = waist wavelengths (waist = 0: plane wave), at each row's y.
 *   - Shape: linear in x and y; gather by bilinear weights at each
 *     component's position.
 *   - Deposition contract (exact integers, independent of summation order):
 *     the position update is the 1D one in x and in y (float32 offsets
 *     ox, oy in [0, 1); g = sqrt(((1 + ux^2) + uy^2) + uz^2), v = u / g,
 *     s = o + v cfl, floor, a result of exactly 1 moves on); weights are
 *     q = floor(o 2^12) per direction on the 4 nodes (old cell - 1) ..
 *     (old cell + 2); with dS = S_new - S_old, Sig = S_old + S_new and
 *     C[a] = -(dS[0] + .. + dS[a]) (Esirkepov's decomposition):
 *       Jx_int[face a + 1/2, row b]      += qw C_x[a] Sig_y[b]
 *       Jy_int[node a, half-row b + 1/2] += qw Sig_x[a] C_y[b]
 *       Jz_int[node a, row b] += qw rint(v_z 2^12)
 *                                ((S_old_x S_old_y + S_new_x S_new_y)[a, b] >> 12)
 *     (qw = Z rint(w 256 / w_ref)).  The charge of a particle on node
 *     (a, b) is 2 qw S_x[a] S_y[b], and charge' - charge + div J = 0 holds
 *     exactly node by node.  dt Jx = Jx_int w_ref 2^-33 / dx (also Jy),
 *     dt Jz = Jz_int w_ref 2^-33 dt / dx^2, charge density
 *     rho = charge_int w_ref 2^-33 / dx^2.
 *   - Quiet start: ppc_x ppc_y particles per cell per species on a lattice
 *     with jitter; particle i of the foil (cells column by column, rows
 *     fastest; k = i mod ppc, kx = k / ppc_y, ky = k mod ppc_y) at offsets
 *     ((kx + 1/2) + jitter (U_2i - 1/2)) / ppc_x and
 *     ((ky + 1/2) + jitter (U_2i+1 - 1/2)) / ppc_y, U_m the SplitMix64
 *     draw m of the stream seeded with `seed`; electrons and protons
 *     co-located; weight n0 dx dy / (ppc_x ppc_y).
 *
 * Cell index of a particle (state I/O): cell = ix * 2^y_shift + iy with
 * y_shift = ceil(log2 ny) (pic2d_info).  The cell sort (pic2d_sort, and
 * every sort_interval steps) orders particles by blocks of 8 x min(8,
 * 2^y_shift) cells (pic2d_info's sort block shifts): blocks column by
 * column (bx = ix >> sx, by = iy >> sy; by fastest), the cells of a block
 * column by column, so that the particles of a push tile lie in a compact
 * patch of the grid.  The order of particles within a cell is unspecified.  Grid arrays (state I/O) are
 * y-fastest: element (column, row) at column * ny + row, with nx + 1
 * columns for node components, nx + 2 for half-node components, nx + 2
 * for Jx_int, nx + 3 for Jy_int and Jz_int (column = node + 1), nx + 1 for
 * charge_int.
 */
#ifndef PIC2D_H
#define PIC2D_H

#include "pic.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Field advance kernels.  TILES: work-groups of 8 columns x 32 rows, each
 * loading its tile with halos into LDS; any period.  STRIPS: a work-group
 * owns a strip of columns and the whole period (one thread per row, at most
 * 1024 rows in FP32, 512 in FP64) and marches along x, reading every value
 * once; automatic where it fits. */
#define PIC2D_FIELD_TILES 1
#define PIC2D_FIELD_STRIPS 2

typedef struct pic2d_config {
  uint32_t struct_size;      /* sizeof(pic2d_config) of the caller */
  int32_t precision;         /* PIC_FP32 or PIC_FP64 */
  double lambda_um;          /* laser wavelength in micrometres (> 0) */
  int32_t cells_per_lambda;  /* >= 4, in x and y */
  int32_t ppc_x, ppc_y;      /* lattice of particles per cell per species */
  int32_t pol;               /* PIC_LP or PIC_CP */
  double box_x, box_y;       /* box in wavelengths: 8 .. 2^20 columns, 2 .. 65536 rows */
  double cfl;                /* dt / dx, in (0, 0.5] */
  int32_t rr;                /* radiation reaction on electrons (0/1) */
  int32_t rr_compensated;    /* TwoSum accumulation of the RR increment (fp32 only) */
  double a0;                 /* normalised laser amplitude */
  double waist;              /* transverse 1/e half width in wavelengths, 0 = plane wave */
  double t_rise, t_flat, t_fall; /* envelope, in periods */
  double n0;                 /* foil density in n_c (> 0) */
  double x_foil;             /* foil front, wavelengths */
  double thickness;          /* foil thickness, wavelengths (the foil fills y) */
  double mass_ratio;         /* ion / electron mass */
  int32_t sort_interval;     /* steps between sorts (>= 1) */
  int32_t field_kernel;      /* field advance: 0 automatic, PIC2D_FIELD_TILES or
                                PIC2D_FIELD_STRIPS (both compute the same step) */
  uint64_t seed;             /* quiet-start jitter seed */
  double jitter;             /* in [0, 1] */
  int64_t capacity;          /* particles per species to reserve; 0 = foil count */
} pic2d_config;

typedef struct pic2d_info {
  int32_t nx, ny;            /* cells in x and y */
  int32_t y_shift;           /* cell index = ix << y_shift | iy */
  int32_t precision;
  double dx, dt, eps_rr, w_ref;
  int64_t capacity;          /* per species */
  int64_t n_init[2];
  int64_t step;
  int32_t tile;              /* particles per push work-group */
  int32_t lds_slots;         /* 64-bit LDS current accumulators per push work-group */
  int32_t field_kernel;      /* the field advance in use: PIC2D_FIELD_TILES or _STRIPS */
  int32_t field_blocks;      /* its work-groups per launch */
  int32_t sort_block_x_shift, sort_block_y_shift; /* sort order: blocks of 2^sx x 2^sy cells */
  int32_t reserved_info;
} pic2d_info;

/* Particle arrays for state I/O: as pic_species_state, with two offsets. */
typedef struct pic2d_species_state {
  int64_t count;
  int32_t* cell;             /* ix << y_shift | iy */
  void* ox; void* oy;        /* real offsets in [0, 1) */
  void* ux; void* uy; void* uz;
  void* w;
  float* rx; float* ry; float* rz;
} pic2d_species_state;

typedef struct pic2d_state {
  pic2d_species_state sp[2];
  void* Ex; void* Ey; void* Ez; void* Bx; void* By; void* Bz; /* real, layout above */
  int64_t* Jx_int; int64_t* Jy_int; int64_t* Jz_int; /* current of the current step */
  int64_t* charge_int;       /* [(nx + 1) ny] running charge: initial charge minus the
                                integrated divergence of the current */
  int64_t step;
  pic_budget_state budget;   /* cumulative budget terms and the non-finite flag, as in pic.h */
} pic2d_state;

/* The 2D run handle: opaque, owned by the library (file-scope declaration,
 * as for struct pic_run). */
struct pic2d_run;

/* Workspace bytes (host-only). */
pic_status pic2d_workspace_bytes(const pic2d_config* cfg, size_t* bytes);

/* Validate, carve the caller's workspace (256-byte aligned), quiet start,
 * zero fields.  Async. */
pic_status pic2d_init(const pic2d_config* cfg, void* d_ws, size_t ws_bytes, void* stream,
                      struct pic2d_run** out);

/* Enqueue n_steps full steps.  Async. */
pic_status pic2d_step(struct pic2d_run* run, int64_t n_steps, void* stream);

/* Stages, as in pic.h: push-deposit (leaves J_int of this push), field
 * advance (advances the step counter), sort.  Async. */
pic_status pic2d_push_deposit(struct pic2d_run* run, void* stream);
pic_status pic2d_field_advance(struct pic2d_run* run, void* stream);
pic_status pic2d_sort(struct pic2d_run* run, void* stream);

/* Diagnostics (FP64), as pic_diag_out; energies per unit length in z.
 * gauss: max |div E - rho| over nodes 1..nx-1 (field units, rho from the
 * particles' fixed-point charge); gauss_int: max |charge_int - charge of the
 * particles| over nodes 1..nx-1, exact integers (expect 0; the end nodes
 * keep the share of removed particles' last shapes that lay inside).
 * Blocking. */
pic_status pic2d_diag(struct pic2d_run* run, pic_diag_out* out, void* stream);

pic_status pic2d_get_info(const struct pic2d_run* run, pic2d_info* out);
void pic2d_free(struct pic2d_run* run);

/* State I/O (host buffers), blocking.  get: particle arrays hold `capacity`
 * entries, removed particles are skipped; any pointer may be NULL.  set:
 * validates cells and offsets; replacing particles clears both current
 * buffers and restarts charge_int from the new particles' charge; fields,
 * currents and charge_int are written when given; step >= 0 resets the
 * step counter (and the laser clock); budget as in pic_get_state and
 * pic_set_state (get always fills it; set with budget.valid = 1 replaces the
 * run's cumulative terms).  A checkpoint set into a fresh run continues the
 * run: state and integer diagnostics repeat bit for bit, FP64 sums to
 * rounding. */
pic_status pic2d_get_state(struct pic2d_run* run, pic2d_state* st, void* stream);
pic_status pic2d_set_state(struct pic2d_run* run, const pic2d_state* st, void* stream);

/* Per-kernel timing as pic_timing_enable / pic_timing_read (kinds 0 push,
 * 1 field advance, 2 sort: its four launches). */
pic_status pic2d_timing_enable(struct pic2d_run* run, int32_t period);
pic_status pic2d_timing_read(struct pic2d_run* run, double ms[3], int64_t launches[3], void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PIC2D_H */
