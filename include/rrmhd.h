/*
 * rrmhd.h -- C-ABI of the MI355X (gfx950) library for the recursive
 * regularised lattice Boltzmann method for 2D incompressible MHD
 * (De Rosis, arXiv 2602.14667).
 *
 * The library advances a D2Q9 fluid population set (fourth-order Hermite
 * equilibrium carrying the Maxwell stress, recursive regularisation of the
 * non-equilibrium part) and a D2Q5 vector magnetic population set (BGK) by
 * one fused stream-and-collide kernel per time step, following the six
 * per-node tasks of the paper's "Algorithm of computation" (Sec. II.B).
 *
 * Conventions shared by every call
 *  - Units are lattice units (dx = dt = 1).
 *  - Field arrays are C-contiguous FP64 in DEVICE memory: a scalar field is
 *    [ny][nx] (x fastest), a vector field is [2][ny][nx] (component, y, x).
 *  - The library owns the population buffers.  The caller owns every I/O
 *    array and keeps it alive until the handle's stream has reached the call.
 *  - Calls are stream-ordered on the handle's HIP stream and return before
 *    the GPU work ends, except where a call says it synchronises.
 *  - Every call returns RRMHD_OK (0) or a negative code; no exception or
 *    abort crosses the ABI.  On failure an output handle is set to NULL;
 *    other failures leave the handle valid.  rrmhd_strerror gives the text,
 *    rrmhd_last_error_detail the HIP message of the last device error.
 *  - A handle is not thread-safe; distinct handles are independent.
 *  - Environment (read at rrmhd_create or rrmhd_*autotune): RRMHD_TILE =
 *    "BXxBY" or "BXxBYxRY" replaces the default launch shape of the step
 *    kernel (one node per thread; ignored unless BX*BY <= 256);
 *    RRMHD_DEBUG_POISON = 1 turns on the debug poison mode of two-buffer
 *    handles; RRMHD_AUTOTUNE_CACHE names the autotuner's cache file when the
 *    call passes none; RRMHD_PLANE_PAD_BYTES (a multiple of 256) sets the
 *    gap between population planes of [ny][nx]; RRMHD_LAYOUT = "planar"
 *    keeps planes of [ny][nx] for every handle; RRMHD_ROW_PAD_BYTES (a
 *    multiple of 256) sets the gap between row groups of the row-interleaved
 *    layout.
 */
#ifndef RRMHD_H
#define RRMHD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  RRMHD_OK = 0,
  RRMHD_EINVAL = -1,     /* bad argument: tau <= 1/2, size < 1, bad enum... */
  RRMHD_ENOMEM = -2,     /* device allocation failed */
  RRMHD_EDEVICE = -3,    /* a HIP call failed */
  RRMHD_ENONFINITE = -4, /* a diagnostic came out NaN or infinite */
  RRMHD_ESTATE = -5,     /* e.g. rrmhd_step before rrmhd_init */
  RRMHD_EIO = -6         /* a checkpoint file could not be opened, read or written */
};

/* Population storage.  Both store f_i - w_i for the fluid populations and
 * g_j for the magnetic ones, times the codec scale; arithmetic is FP32.
 * RRMHD_STORE_INPLACE may be OR-ed into rrmhd_grid.storage: the handle then
 * holds one population buffer instead of two (half the device memory).  Its
 * steps alternate between two forms that each write only the locations they
 * have just read: a pull of the upstream populations whose results go into
 * the slots just read for the opposite directions, then a read of the node's
 * own (swapped) slots with a local store, which restores the usual layout.
 * The per-node arithmetic is unchanged, so a single-buffer handle evolves
 * bit for bit as a two-buffer one; moments, diagnostics, fields and
 * rrmhd_save_state read either layout (save returns the usual one).  Not
 * with the learned closure or the equilibrium ablation (EINVAL); of the
 * launch shape's nt bits, bit 1 (non-temporal loads) does not apply, and
 * bits 2 and 3 (two or four nodes per thread) apply, on periodic grids, only
 * together with bit 0. */
enum { RRMHD_STORE_F32 = 0, RRMHD_STORE_F16 = 1, RRMHD_STORE_INPLACE = 0x100 };
/* RRMHD_STORE_F16_SR: FP16 storage whose step stores round stochastically
 * (each value goes to one of its two FP16 neighbours, away from zero with
 * probability equal to its distance from the neighbour toward zero in units
 * of the gap -- exactly in FP16's normal range, to 2^-13 of the gap for
 * subnormal results, magnitudes below 2^-37 storing zero -- results beyond
 * the FP16 range store infinity and NaN a quiet NaN; the rule is written
 * out at rrmhd_sr_encode),
 * with random bits from a counter-based hash of the step count, the node
 * and the plane, so runs are reproducible and independent of the launch
 * shape.  An optional variant of the prescribed round-to-nearest-even
 * codec, reported separately; initialisation still rounds to nearest.  It
 * combines with RRMHD_STORE_INPLACE (each value draws the bits of the node
 * that computes it and of its own plane, whichever slot receives it, so the
 * single-buffer handle stays bitwise equal to the two-buffer one, and the
 * two- and four-node updates equal one node per thread); not with graph
 * replay, the learned closure or the equilibrium ablation (EINVAL). */
enum { RRMHD_STORE_F16_SR = 2 };
/* Layout of the populations in device memory (not visible through the API:
 * moments, diagnostics, rrmhd_save_state and checkpoint files are the same
 * for either).  Periodic handles (one or two buffers) keep the 19 planes
 * row-interleaved: each grid row holds its 19 plane rows side by side, each
 * starting on a 256-byte boundary, and the FP32 step then updates two nodes
 * per thread with 64-bit words.  Handles with walls, or with
 * RRMHD_STORE_PLANAR OR-ed into rrmhd_grid.storage, keep 19 planes of
 * [ny][nx].  Results are bitwise the same in both layouts. */
enum { RRMHD_STORE_PLANAR = 0x200 };

/* Boundary kinds.  PERIODIC: doubly periodic.  WALLS_Y: periodic in x,
 * walls half-way at y = -1/2 and y = ny - 1/2 (half-way bounce-back for f,
 * anti-bounce-back imposing b_wall for g). */
enum { RRMHD_BC_PERIODIC = 0, RRMHD_BC_WALLS_Y = 1 };

typedef struct {
  int32_t nx, ny;    /* nodes in x and y, >= 1 (ny >= 2 with walls) */
  int32_t storage;   /* RRMHD_STORE_F32 or _F16, optionally | _INPLACE */
  float codec_scale; /* power-of-two storage scale S; 0 selects 1 */
} rrmhd_grid;

typedef struct {
  int32_t kind;     /* RRMHD_BC_* */
  double force[2];  /* body force per unit mass G (F = rho G), Guo-type */
  double b_wall[2]; /* wall field imposed by the magnetic anti-bounce-back */
} rrmhd_bc;

typedef struct rrmhd rrmhd;

/* Create a solver on the current HIP device.  tau_f and tau_m are the fluid
 * and magnetic relaxation times (omega = 1/tau_f, omega_m = 1/tau_m in the
 * collision of algorithm task 5), both > 1/2 and finite.  bc may be NULL
 * (periodic, no force).  hip_stream may be NULL (the null stream) or a
 * hipStream_t such as torch's current stream.  Allocates the two population
 * buffers (19 planes each) and a diagnostics workspace.  A plane of
 * nx * ny stored values must stay below 4 GiB (in-plane offsets are 32-bit
 * byte offsets): nx * ny < 2^30 for FP32 storage, < 2^31 for FP16 (EINVAL
 * otherwise). */
int rrmhd_create(const rrmhd_grid *grid, double tau_f, double tau_m,
                 const rrmhd_bc *bc, void *hip_stream, rrmhd **out);

/* Initial state from the macroscopic fields of Sec. III: rho = 1 and the
 * populations at their equilibria f_eq(1, u, b), g_eq(u, b) (algorithm task
 * 2), so rrmhd_moments right after init returns (1, u, b).  u and b are
 * device [2][ny][nx] FP64.  Resets the step counter. */
int rrmhd_init(rrmhd *h, const double *u, const double *b);

/* Advance n >= 0 time steps.  One step is tasks 1-6 of the algorithm at every
 * node: moments, equilibria, non-equilibrium Hermite coefficients with the
 * recursive third/fourth orders, regularised reconstruction, collision and
 * streaming (done as a pull, fused into one kernel).  Asynchronous. */
int rrmhd_step(rrmhd *h, int64_t n);

/* Pre-collision macroscopic fields of the current state (task 1): rho
 * [ny][nx], u and b [2][ny][nx], FP64 device arrays; any may be NULL.  With a
 * body force u includes half the force impulse.  Asynchronous. */
int rrmhd_moments(rrmhd *h, double *rho, double *u, double *b);

/* Host scalars: E_kin = sum |u|^2 / (2 nx ny), E_mag = sum |b|^2 / (2 nx ny)
 * (the averaged energies of Sec. III.B with the integral as a node sum) and
 * max |div b| with the isotropic lattice gradient of Sec. III (interior rows
 * only with walls).  Accumulated in FP64 on the GPU with a fixed reduction
 * order.  Synchronises the stream.  Returns RRMHD_ENONFINITE, with the
 * outputs set to NaN, if any result is not finite.  Any pointer may be NULL. */
int rrmhd_diagnostics(rrmhd *h, double *E_kin, double *E_mag,
                      double *max_div_b);

/* For callers that cannot allocate device memory (code that runs where
 * hipMalloc is forbidden or too slow: tight serving loops, harnesses that
 * forbid it): rrmhd_diagnostics with the same arguments, results, kernels
 * and reduction order (the results are bit for bit those of
 * rrmhd_diagnostics), but no allocation.  Its workspace (the pass's
 * per-workgroup partial sums and its eight results) is a static device array
 * of 72 KiB that each GPU the library runs on holds until the process ends;
 * its device address is looked up once per device at rrmhd_create.  The
 * workspace the pass needs does not grow with the grid (768 persistent
 * workgroups at most); a build whose pass would need more than the array
 * holds returns RRMHD_EINVAL (rrmhd_last_error_detail gives the sizes)
 * before anything is launched.  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (two host threads, or two handles
 * whose streams run concurrently) race on it and must be serialised by the
 * caller.  Nothing in the array needs clearing between calls: each pass
 * writes every partial sum before its final reduction reads it.  Call with
 * the handle's device current, as for every call.  Synchronises the
 * stream. */
int rrmhd_diagnostics_noalloc(rrmhd *h, double *E_kin, double *E_mag,
                              double *max_div_b);

/* Derived fields of a periodic grid, FP64 device arrays [ny][nx] (either
 * may be NULL): the local current density j_z of Eq. current, computed from
 * the magnetic populations' departure from equilibrium (no finite
 * differences), and the vorticity w_z = d_x u_y - d_y u_x with the isotropic
 * lattice gradient of Sec. III.  EINVAL with walls.  Asynchronous. */
int rrmhd_current_vorticity(rrmhd *h, double *jz, double *wz);

/* Host out[5] = mass sum rho, momentum sum_i c_i f_i (x, y), total field
 * sum b (x, y), FP64, over the current state.  Synchronises the stream. */
int rrmhd_invariants(rrmhd *h, double out[5]);

/* Steps taken since rrmhd_init (host value, no synchronisation). */
int rrmhd_step_count(const rrmhd *h, int64_t *out);

/* Raw stored state for checkpoint/resume: 19 planes of nx*ny elements of
 * the storage type (4 bytes for F32, 2 for F16) in the order f_0..f_8,
 * g_0x, g_0y, ..., g_4x, g_4y, each plane [ny][nx].  These are the
 * post-collision values of the last step at their source nodes (the pull
 * layout), not the pre-collision populations.  `bytes` must be at least
 * rrmhd_state_bytes().  dst/src are device pointers.  Asynchronous. */
int64_t rrmhd_state_bytes(const rrmhd *h);
int rrmhd_save_state(rrmhd *h, void *dst, int64_t bytes);
int rrmhd_load_state(rrmhd *h, const void *src, int64_t bytes,
                     int64_t step_count);

/* Checkpoint files.  rrmhd_save writes a 104-byte header, then the state of
 * rrmhd_save_state (19 planes in the pull layout).  The header is the magic
 * "RRMHDCK1", then int32 version (1), nx, ny, storage kind (RRMHD_STORE_F32,
 * _F16 or _F16_SR; the single-buffer flag is not recorded, the layout
 * being the same), float codec scale, int32 boundary kind, int32
 * equilibrium kind, int32 zero, then double tau_f, tau_m, force[2],
 * b_wall[2], then int64 step count and payload bytes, little-endian.  It
 * synchronises the handle's stream and copies one plane at a time through
 * host memory.  A single-buffer handle between its two step forms also
 * needs a device buffer of the state's size for the gather.
 * rrmhd_load reads such a file into a handle with the same nx, ny, element
 * size, codec scale, relaxation times, boundary conditions and equilibrium
 * kind; the stochastic-rounding flag may differ, since the rounding applies
 * only to later steps.  It then continues exactly as the saved run would
 * have (bitwise).  A mismatch or a malformed file gives EINVAL (the handle
 * is unchanged; rrmhd_last_error_detail names the field); I/O failures give
 * RRMHD_EIO (a read that fails part-way leaves the handle uninitialised:
 * ESTATE until rrmhd_init or a load succeeds).  Synchronous. */
int rrmhd_save(rrmhd *h, const char *path);
int rrmhd_load(rrmhd *h, const char *path);

/* Launch shape of the step kernel (the tuning knob of the autotuner; the
 * default is picked from the grid).  bx x by threads per workgroup
 * (bx * by <= 256, bx >= 1, by >= 1), ry consecutive rows per thread (>= 1),
 * xcd = 1 renumbers workgroups so each XCD gets one contiguous run of tiles,
 * xcd = 2 so each XCD gets 8 neighbouring tiles out of every 64; nt bit 0
 * writes populations with non-temporal stores, bit 1 reads them with
 * non-temporal loads (periodic grids), bit 2 lets each thread update two
 * neighbouring nodes with one word per plane (FP16 storage: 32-bit words;
 * FP32 storage on row-interleaved planes: 64-bit words; periodic grids with
 * even nx), bit 3 four neighbouring nodes with 64-bit words (FP16 storage,
 * nx a multiple of 4); a workgroup then covers 2 bx or 4 bx nodes in x.  On
 * row-interleaved planes the multi-node forms need bx a multiple of 64 or
 * by = 1; where a form does not apply the bit is ignored.  Results do not
 * depend on the shape (bitwise).  Host-side only. */
int rrmhd_set_launch(rrmhd *h, int bx, int by, int ry, int xcd, int nt);
/* The handle's current launch shape (any pointer may be NULL). */
int rrmhd_get_launch(const rrmhd *h, int *bx, int *by, int *ry, int *xcd, int *nt);

/* Stream used by the handle; NULL is the null stream. */
int rrmhd_set_stream(rrmhd *h, void *hip_stream);

/* Graph replay for launch-bound grids: with chunk > 0, rrmhd_step(n) runs
 * whole runs of `chunk` steps as one captured hipGraph each (captured on
 * first use, one graph per starting buffer or in-place phase, replayed on
 * an internal stream that is ordered after the handle's stream with events)
 * and launches the remaining n mod chunk steps directly.  Results are
 * bitwise those of plain launches.  Changing the launch shape, the
 * equilibrium or the closure's on/off state drops the graphs; new closure
 * parameters do not (the graph reads them at run time).  chunk = 0 (the
 * default) launches every step directly.  EINVAL for chunk < 0. */
int rrmhd_set_graph_chunk(rrmhd *h, int chunk);

/* Debug aid: with on != 0, every later step first fills the buffer it
 * writes with a NaN pattern (all planes, padding included), so a stored
 * value that a step fails to write shows up as NaN in the moments and as
 * RRMHD_ENONFINITE from the diagnostics.  Results are otherwise unchanged
 * (a step reads only the other buffer); each step costs one more write of
 * the whole buffer.  For the callers that check kernel coverage (tests);
 * EINVAL for a single-buffer handle, whose steps read what they write. */
int rrmhd_set_debug_poison(rrmhd *h, int on);

/* Equilibrium of the fluid populations.  RRMHD_FEQ_ALGORITHM (the default)
 * is the fourth-order Hermite equilibrium the algorithm uses (Eq. feq_4th,
 * task 2 of the algorithm in Sec. II.B), with the Maxwell stress in the
 * second-order coefficient only.  RRMHD_FEQ_FULL_MAXWELL adds the u.M cross
 * terms of the third- and fourth-order equilibrium coefficients (Eq.
 * eq:a0_4) on the D2Q9-supported components xxy, xyy and xxyy: an ablation
 * of the reading that the two equilibria differ, for comparing them on the
 * same kernels.  It applies to every following rrmhd_init and rrmhd_step of
 * the handle (single-node update with non-temporal stores; the launch
 * shape's nt bits are ignored).  EINVAL for another kind, or for
 * FULL_MAXWELL while the learned closure is enabled (the closure was
 * trained on the algorithm's equilibrium).  Host-side only. */
enum { RRMHD_FEQ_ALGORITHM = 0, RRMHD_FEQ_FULL_MAXWELL = 1 };
int rrmhd_set_equilibrium(rrmhd *h, int kind);

int rrmhd_destroy(rrmhd *h);

/* ---- Three-dimensional extension ----------------------------------------
 * The paper is two-dimensional and names three-dimensional lattices as the
 * next step (Conclusions).  This handle advances the direct generalisation
 * of the algorithm of Sec. II.B on a periodic nx x ny x nz box:
 *  - fluid D3Q27, c_s^2 = 1/3: equilibrium = the D3Q27 Hermite series up to
 *    sixth order (the product of three D1Q3 factors) with the Maxwell stress
 *    M = |b|^2/2 I - b b at second order only; a1^(2) by projection; every
 *    D3Q27-supported coefficient of orders 3 to 6 from the recursion of task
 *    3 in general form (a sum over index pairs of a1^(2) times the other
 *    velocities); collision f* = f_eq + (1 - 1/tau_f) f_neq,reg;
 *  - magnetic D3Q7 vector BGK, weights 1/4 (rest) and 1/8, so
 *    eta = (tau_m - 1/2)/4; g_eq,j = psi_j [b + 4 e_j.(u b - b u)].
 * nu = (tau_f - 1/2)/3.  Storage RRMHD_STORE_F32 or _F16 (f - w and g, S = 1),
 * FP32 arithmetic, two buffers of 48 planes, or one with RRMHD_STORE_INPLACE
 * OR-ed into storage (the alternating single-buffer steps of the
 * two-dimensional handle; bitwise the same results; moments and
 * diagnostics read either layout).  Fields are [3][nz][ny][nx]
 * (component, z, y, x) FP64 device arrays, rho [nz][ny][nx].  Errors as for
 * the two-dimensional handle (EINVAL also for ny or nz above 65535 or
 * nx ny nz * element size >= 2^32).  Diagnostics: E = sum |u|^2 / (2N),
 * sum |b|^2 / (2N), max |div b| with the isotropic D3Q27 gradient;
 * invariants: mass, sum rho u (3), sum b (3). */
typedef struct rrmhd3d rrmhd3d;
int rrmhd3d_create(int32_t nx, int32_t ny, int32_t nz, int32_t storage, double tau_f,
                   double tau_m, void *hip_stream, rrmhd3d **out);
int rrmhd3d_init(rrmhd3d *h, const double *u, const double *b);
int rrmhd3d_step(rrmhd3d *h, int64_t n);
int rrmhd3d_step_count(const rrmhd3d *h, int64_t *out);
int rrmhd3d_moments(rrmhd3d *h, double *rho, double *u, double *b);
int rrmhd3d_diagnostics(rrmhd3d *h, double *E_kin, double *E_mag, double *max_div_b);
int rrmhd3d_invariants(rrmhd3d *h, double out[7]);
/* bx x by threads per workgroup over x and y (bx * by <= 256); xcd = 1
 * hands each XCD 8 neighbouring row tiles out of every 64 workgroups, 0 keeps
 * the plain order, -1 leaves the current setting (default: 1 for FP16
 * storage or one buffer, 0 for FP32 with two).  Results do not depend on
 * the shape or the order.  Host-side only. */
int rrmhd3d_set_launch(rrmhd3d *h, int bx, int by, int xcd);
int rrmhd3d_destroy(rrmhd3d *h);
/* Checkpoint files of the 3D handle, as rrmhd_save / rrmhd_load: a 64-byte
 * header (magic "RRMHD3C1", int32 version 1, nx, ny, nz, storage kind,
 * zero, double tau_f, tau_m, int64 step count, payload bytes) and the 48
 * planes of nx*ny*nz stored values in the pull layout (a single-buffer
 * handle between its two step forms gathers them through a temporary
 * device buffer of the state's size).  Load requires the same box,
 * storage kind and relaxation times (EINVAL otherwise, handle unchanged),
 * accepts files of one- and two-buffer handles alike, and continues
 * bitwise; RRMHD_EIO for I/O failures.  Synchronous. */
/* As rrmhd_set_debug_poison, for the 3D two-buffer handle (EINVAL for a
 * single-buffer one).  For the callers that check kernel coverage (tests). */
int rrmhd3d_set_debug_poison(rrmhd3d *h, int on);
int rrmhd3d_save(rrmhd3d *h, const char *path);
int rrmhd3d_load(rrmhd3d *h, const char *path);

/* ---- Batched ensemble --------------------------------------------------
 * Many independent doubly periodic domains of uneven sizes and relaxation
 * times, all advanced together: one persistent kernel launch per time step
 * strides over a flat list of 256-thread tiles covering every domain (the
 * same per-node update as rrmhd_step, so each domain evolves bitwise as a
 * standalone handle would).  With a graph chunk set, runs of that many steps
 * are captured once into a hipGraph and replayed.  One storage type for the
 * whole ensemble.  Domain indices run 0..n-1; field arrays follow the
 * single-domain conventions for the domain's own nx, ny. */
typedef struct rrmhd_batch rrmhd_batch;

/* grids[d] gives nx, ny of domain d (storage/codec_scale fields ignored; the
 * storage argument applies to all); tau_f[d], tau_m[d] > 1/2 (host arrays).
 * Allocates both population buffers for all domains. */
int rrmhd_batch_create(int n, const rrmhd_grid *grids, const double *tau_f,
                       const double *tau_m, int storage, void *hip_stream,
                       rrmhd_batch **out);
/* Equilibrium initial state of domain d (as rrmhd_init). */
int rrmhd_batch_init(rrmhd_batch *b, int d, const double *u, const double *bf);
/* Advance every domain n steps (all domains must have been initialised). */
int rrmhd_batch_step(rrmhd_batch *b, int64_t n);
/* Steps per captured hipGraph (0: plain launches, the default). */
int rrmhd_batch_set_graph_chunk(rrmhd_batch *b, int chunk);
/* Tile width bx (a divisor of 256, tile = bx x 256/bx) for domain d, or for
 * all domains when d = -1 (0 keeps it); workgroups per launch grid (0 keeps
 * it, -1 = one workgroup per tile); nt = 1/0 non-temporal stores (-1 keeps
 * it).  Results do not depend on these (bitwise). */
int rrmhd_batch_set_shape(rrmhd_batch *b, int d, int bx, int grid, int nt);
/* Work distribution inside a launch: 0 (default) = static, workgroup w
 * takes tiles w, w + grid, ...; k in 1..64 = dynamic: the tile list is cut
 * into 8 contiguous segments, one per XCD, and each workgroup takes its next
 * k consecutive tiles of its segment from that segment's device counter
 * (persistent workgroups; the counters return to zero at the end of every
 * launch).  Results do not depend on it (bitwise).  EINVAL outside 0..64. */
int rrmhd_batch_set_fetch(rrmhd_batch *b, int tiles_per_fetch);
int rrmhd_batch_moments(rrmhd_batch *b, int d, double *rho, double *u,
                        double *bf);
/* As rrmhd_diagnostics for domain d (synchronises). */
int rrmhd_batch_diagnostics(rrmhd_batch *b, int d, double *E_kin,
                            double *E_mag, double *max_div_b);
/* Total nodes, steps taken, tiles in the work list, workgroups per launch. */
int rrmhd_batch_info(const rrmhd_batch *b, int64_t *nodes, int64_t *steps,
                     int *ntiles, int *grid);
int rrmhd_batch_destroy(rrmhd_batch *b);
const char *rrmhd_batch_last_error_detail(void);

/* ---- Learned closure (a project addition; the paper has none) -------------
 * A per-node MLP maps the node's pre-collision features x = (rho, u_x, u_y,
 * b_x, b_y, a_xx, a_xy, a_yy) -- a_1^(2) from the projection of algorithm
 * task 3 -- to a correction of a_1^(2) applied before the recursion:
 *   x_hat = (x - mu) / sigma,  h1 = GELU(W1 x_hat + b1)  (64 units),
 *   h2 = GELU(W2 h1 + b2)  (64),  y = W3 h2 + b3  (3),
 *   (a_xx, a_xy, a_yy) += sigma_out * y,
 * GELU(z) = z/2 (1 + tanh(sqrt(2/pi)(z + 0.044715 z^3))).  On the GPU the
 * layers run as BF16 MFMA (x_hat, weights, h1, h2 rounded to BF16, FP32
 * accumulation and biases) fused into the step kernel; GELU is applied to
 * the BF16-rounded pre-activation through a table holding, for each of the
 * 65,536 BF16 bit patterns, the tanh-form GELU evaluated in FP64 and
 * correctly rounded to BF16.
 * params: 4931 FP32 = W1[64][8], b1[64], W2[64][64], b2[64], W3[3][64],
 * b3[3]; norm: 19 FP32 = mu[8], sigma[8], sigma_out[3]; both DEVICE
 * pointers, read at the call (stream-ordered).  Zero weights and biases give
 * a correction of exactly zero. */
/* Install parameters on a handle (params == NULL disables the closure). */
int rrmhd_closure_set(rrmhd *h, const float *params, const float *norm);
/* Turn the installed closure on or off for subsequent rrmhd_step calls
 * (periodic, unforced grids only; EINVAL otherwise or if none is set). */
int rrmhd_closure_enable(rrmhd *h, int on);
/* Network outputs y[n][3] (before the sigma_out scaling) for raw features
 * x[n][8], all device FP32, with the same BF16 MFMA arithmetic as the fused
 * step.  Synchronises hip_stream. */
int rrmhd_closure_eval(const float *params, const float *norm, const float *x,
                       int64_t n, float *y, void *hip_stream);
/* The GELU table the inference uses: out[v] (65,536 uint16, DEVICE) is the
 * BF16 bit pattern of GELU(bf16 value with bit pattern v).  Stream-ordered on
 * hip_stream, asynchronous. */
int rrmhd_closure_gelu_table(uint16_t *out, void *hip_stream);

/* Training of the closure (FP32 kernels).  Data (a-priori regression): fine
 * moments rho[nf][nf], u, b [2][nf][nf] (device FP64, e.g. from
 * rrmhd_moments) are box-filtered over factor x factor blocks; each coarse
 * node gives features x = (rho_bar, u_bar, b_bar, a_CE) with u_bar =
 * (rho u)_bar / rho_bar and a_CE = -rho_bar c_s^2 tau_c (grad u_bar +
 * grad u_bar^T) (isotropic gradient on the coarse grid), and a target
 * tau_sgs / (tau_c - 1) with tau_sgs = (rho u u)_bar - rho_bar u_bar u_bar
 * + M(b)_bar - M(b_bar).  work: 10 (nf/factor)^2 doubles; x [Nc][8] and
 * target [Nc][3] FP32, Nc = (nf/factor)^2.  Asynchronous. */
int rrmhd_train_samples(const double *rho, const double *u, const double *b,
                        int nf, int factor, double tau_c, double *work,
                        float *x, float *target, void *hip_stream);
/* The box filter of the training data alone: out [10][Nc] FP64 (device),
 * Nc = (nf/factor)^2, holds the factor x factor block means of rho, rho u_x,
 * rho u_y, b_x, b_y, rho u_x u_x, rho u_x u_y, rho u_y u_y, M(b)_xx, M(b)_xy
 * of the fine moments (layout of rrmhd_moments).  Asynchronous on
 * hip_stream; EINVAL for null pointers or nf not a multiple of factor. */
int rrmhd_train_box_filter(const double *rho, const double *u, const double *b,
                           int nf, int factor, double *out, void *hip_stream);
/* Replace the fluid populations of a periodic two-buffer handle so that, at
 * every node, its current state holds the equilibrium of Eq. feq_4th (the
 * Maxwell stress at second order) for the given density rho [ny][nx],
 * momentum j [2][ny][nx] and magnetic field b [2][ny][nx] (device FP64, u =
 * j / rho), with no non-equilibrium part; the magnetic populations are kept.
 * For the closure protocol's best-velocity bound (a project addition): the
 * coarse run's velocity is replaced every step by the filtered fine one, b
 * being the run's own current field.  Asynchronous on the handle's stream;
 * EINVAL for null pointers, walls or a single-buffer handle, ESTATE before
 * rrmhd_init. */
int rrmhd_train_impose_fluid(rrmhd *h, const double *rho, const double *j,
                             const double *b);
typedef struct rrmhd_trainer rrmhd_trainer;
/* Workspace for minibatches of up to max_batch samples. */
int rrmhd_train_create(int64_t max_batch, void *hip_stream,
                       rrmhd_trainer **out);
/* grad[4931] and *loss (device FP32; loss may be NULL) of the mean squared
 * error (1/n) sum_s sum_o (y_o(x_s) - target_so / sigma_out_o)^2 of the
 * FP32 network over samples x[n][8], target[n][3] (device).  Reductions run
 * in a fixed order (deterministic).  Asynchronous. */
int rrmhd_train_loss_grad(rrmhd_trainer *t, const float *params,
                          const float *norm, const float *x,
                          const float *target, int64_t n, float *grad,
                          float *loss);
/* One-step solver-in-the-loop data (training objective of the closure).
 * Fine moments at t (rho0, u0, b0) and at t + factor (rho1, u1, b1), device
 * FP64 in the layout of rrmhd_moments, nf x nf periodic; the coarse grid has
 * nc = nf/factor nodes per side and relaxation time tau_c (coarse step =
 * factor fine steps).  The coarse grid is restarted from the filtered fields
 * at t with f = f_eq(rho_bar, u_bar, b_bar) + f_neq,reg(u_bar, a_CE) and g =
 * g_eq(u_bar, b_bar) (features x as in rrmhd_train_samples).  Outputs
 * (device): x[Nc][8] FP32; r0[Nc][2] FP32 = momentum j_c(X) after one coarse
 * step without correction minus j_bar(X, t + factor) (computed in FP64);
 * *den FP64 = sum_X |j_bar(t + factor) - j_bar(t)|^2.  work: 29 Nc doubles.
 * Asynchronous; EINVAL for null pointers, nf not a multiple of factor or
 * tau_c <= 1/2. */
int rrmhd_train_onestep_samples(const double *rho0, const double *u0,
                                const double *b0, const double *rho1,
                                const double *u1, const double *b1, int nf,
                                int factor, double tau_c, double *work,
                                float *x, float *r0, double *den,
                                void *hip_stream);
/* grad[4931] and *loss (device FP32; loss may be NULL) of the one-step
 * objective L = sum_X |r(X)|^2 / den over nsnap snapshots stored back to back
 * (x [nsnap][Nc][8], r0 [nsnap][Nc][2] from rrmhd_train_onestep_samples, den
 * their summed denominators, host value > 0), where r = r0 plus the effect of
 * the correction D = sigma_out * y(x) added to a_1^(2) at every coarse node
 * before the recursion: one collision of the restart state and the pull of
 * one step.  feedback = 1: the restart also carries the closure's own steady
 * response q = (tau_c - 1) D0, D0 = sigma_out * y(x) (a correction added every
 * step settles at a non-equilibrium (tau - 1) D), and the step's correction
 * is D = sigma_out * y(x1) on the features x1 of that restart (a_1^(2)
 * entries shifted by q), so the collision relaxes q + D; feedback = 0: the
 * plain form.  The gradient is exact: the transpose of the stencil, then
 * reverse mode through the FP32 network (through both evaluations in the
 * feedback form).  nsnap nc^2 <= max_batch.  Asynchronous; EINVAL for
 * feedback outside {0, 1}. */
int rrmhd_train_onestep_loss_grad(rrmhd_trainer *t, const float *params,
                                  const float *norm, const float *x,
                                  const float *r0, int nsnap, int nc,
                                  double tau_c, double den, int feedback,
                                  float *grad, float *loss);
/* One Adam step (Kingma & Ba 2015) on params[4931] with moments m, v
 * (device FP32) at step number step >= 1.  Asynchronous. */
int rrmhd_train_adam(rrmhd_trainer *t, float *params, float *m, float *v,
                     const float *grad, float lr, float beta1, float beta2,
                     float eps, int step);
int rrmhd_train_destroy(rrmhd_trainer *t);
const char *rrmhd_train_last_error_detail(void);

/* ---- Autotuner -----------------------------------------------------------
 * Times candidate launch shapes of the step kernel on the handle's own grid
 * (trials steps each, best of three repetitions, HIP events) and installs
 * the fastest.  The handle's state and step count are preserved (a handle
 * that was never initialised is timed on the rest state and stays
 * uninitialised).  cache_path (may be NULL) names a JSON file of earlier
 * results keyed by device architecture, grid size and storage; a cached
 * entry is installed without timing, and new results are added to it.
 * Outputs (may be NULL): the chosen bx, by, xcd and its time per step. */
int rrmhd_autotune(rrmhd *h, const char *cache_path, int trials, int *out_bx,
                   int *out_by, int *out_xcd, double *out_ms);
/* Ensemble version: a tile width for every distinct domain size (timed on a
 * standalone grid of that size) and then the work distribution (workgroup
 * count and static or dynamic schedule, timed on the ensemble, state
 * preserved); same cache file. */
int rrmhd_batch_autotune(rrmhd_batch *b, const char *cache_path, int trials);

/* Measurement helper, not part of the method: copies `bytes` (a multiple of
 * 16, both pointers 16-byte aligned, device memory) with a plain streaming
 * kernel on hip_stream.  Used as the measured device-bandwidth reference
 * and to calibrate memory-traffic counters against a known byte count. */
int rrmhd_bandwidth_probe(void *dst, const void *src, int64_t bytes,
                          void *hip_stream);

/* The encode of RRMHD_STORE_F16_SR on arrays (device memory, codec scale 1):
 * out[i] = the FP16 bit pattern of x[i] rounded stochastically with the 32
 * random bits r[i] -- with e the biased FP32 exponent of x and m its 24-bit
 * significand, d = max(126 - e, 13) dropped bits, the dropped fraction kept
 * to 13 bits, t = floor(m 2^(13-d)), and the kept integer k = floor((t + r_13)
 * 2^-13) with r_13 the top 13 bits of r; past the largest finite value
 * infinity, NaN a quiet NaN of its sign and the top ten payload bits.  For callers that check the codec (tests).  n >= 0;
 * asynchronous on hip_stream. */
int rrmhd_sr_encode(const float *x, const uint32_t *r, uint16_t *out, int64_t n,
                    void *hip_stream);

const char *rrmhd_strerror(int code);
const char *rrmhd_last_error_detail(void);

#ifdef __cplusplus
}
#endif

#endif /* RRMHD_H */
