/*
 * lb.h -- C ABI of liblb.so: the two-component colour-gradient lattice
 * Boltzmann update on a D3Q19 lattice, for AMD Instinct MI355X (gfx950).
 *
 * What one step computes (arXiv 2005.12764, "Towards Exascale Design of Soft
 * Mesoscale Materials"):
 *   - two fluid components r and b, each with its own 19 populations
 *     (Sec. 2.1, eq:twobgk), relaxed by BGK toward the second-order equilibrium
 *     (Sec. 2, eq:equil) with one mixture rate w_eff taken from the
 *     density-weighted harmonic mean of the component viscosities
 *     nu_k = (tau_k - 1/2)/3 (Sec. 2.1, eq:twobgk with Sec. 2, eq:eq3);
 *   - a force density F acting through the exact-difference source
 *     S_i = f^eq(rho_k, u + F/rho) - f^eq(rho_k, u) (Sec. 2.1, eq:edm):
 *     a uniform body force plus the near-contact repulsion
 *     F_rep = -A_h[h] n delta_I of Sec. 4 (F_rep equation);
 *   - the colour-gradient surface-tension perturbation and recolouring of
 *     colour-gradient models (the paper uses them without writing them out);
 *   - streaming, an exact memory shift (Sec. 2), with periodic axes or halfway
 *     bounce-back walls.
 * Beside the step, lb_korteweg projects the Korteweg tensor of the phase field
 * onto blocks, the data step of the coarse-graining proposal (Sec. 4.1).
 * The readings of the paper that the library takes where the text is silent
 * or garbled (sign of w_eff, force split, the discrete near-contact probe,
 * gradient at walls) are documented with the design notes of the repository.
 *
 * Conventions
 *   - Fields are C-order [z][y][x], x fastest.  Vector fields are SoA
 *     [3][z][y][x].  Populations exchanged through lb_get_state/lb_set_state
 *     are [2][19][z][y][x]: component (0 red, 1 blue), direction, site, in the
 *     post-streaming (pre-collision) state f_i(x, t).
 *   - Direction order: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 = (1,1,0),
 *     (-1,-1,0), (1,-1,0), (-1,1,0), (1,0,1), (-1,0,-1), (1,0,-1), (-1,0,1),
 *     (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1).  Weights 1/3, 1/18, 1/36.
 *   - "on_device" = 1: the pointer is device memory of the handle's device
 *     (e.g. a torch tensor's data_ptr()); 0: host memory.
 *   - Return value: LB_OK (0) or a negative LB_E* code; lb_last_error() gives
 *     a message for the calling thread.  A failed call leaves the state as it
 *     was.  No C++ exception crosses this interface.
 *   - Stream semantics: every call is ordered on the handle's HIP stream.
 *     lb_step and device-pointer transfers do not block the host; calls that
 *     read into host memory (or fill `totals`) synchronise the stream.
 *   - Thread safety: one handle must not be used from two threads at once.
 */
#ifndef LB_H
#define LB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LB_OK 0
#define LB_EINVAL (-1)  /* bad argument or parameter */
#define LB_ENOMEM (-2)  /* device allocation failed */
#define LB_EDEVICE (-3) /* HIP runtime error (launch, copy, no device) */
#define LB_ESTATE (-4)  /* call out of order, e.g. stepping before init */

/* Population storage. */
#define LB_STORE_F64 0  /* raw FP64 populations, 2 x 19 x 8 B per site */
#define LB_STORE_F32 1  /* raw FP32 populations, 2 x 19 x 4 B per site */
#define LB_STORE_F16 2  /* 16-bit moment-split: per site FP32 density, momentum term of
                           the equilibrium, phase and recolouring vector (32 B) + per
                           direction the deviation of the total population from the
                           equilibrium's first-order part in fp16, scaled by
                           2^scale_log2 (38 B); computes in FP32 */
#define LB_STORE_BF16 3 /* as LB_STORE_F16 with bf16 deviations (no scale) */

/* Kernel selection for lb_step. */
#define LB_KERNEL_AUTO 0    /* the one-read step, except (two-pass) for the Shan-Chen model
                               and lattices too large for its 32-bit buffer offsets */
#define LB_KERNEL_TWOPASS 1 /* phase-field pass, then collide-and-stream pass */
#define LB_KERNEL_FUSED 2   /* one-read step: the collide-and-stream tiles also gather the
                               next phase field's sums, a light pass adds the terms
                               that cross tiles; every population is read once per
                               step.  The first step of a 16-bit lattice with moving
                               walls takes two passes. */

/* Tile kinds of lb_set_tiles. */
#define LB_TILES_PHASE 0    /* phase-field pass of two-pass steps (16-bit storage) */
#define LB_TILES_COLLIDE 1  /* collide-and-stream pass of two-pass steps */
#define LB_TILES_ONE_READ 2 /* one-read step (rows 4, 8 or 16) */
#define LB_TILES_BATCH 3    /* tiles of the batched step (rows 4 or 8; other values: 8 at
                               or above 8, else 4) */

/* Interface model (lb_params.model). */
#define LB_MODEL_COLOUR_GRADIENT 0 /* colour gradient: perturbation, recolouring, near contact */
#define LB_MODEL_SHAN_CHEN 1       /* Shan-Chen inter-component force with exact-difference
                                      sources (Sec. 2.1, eq. shanchen_force with eq:edm) */

/* Element type of caller fields. */
#define LB_DTYPE_F64 0
#define LB_DTYPE_F32 1

/* Largest near-contact probe range K the kernels support. */
#define LB_MAX_NC_RANGE 4

typedef struct lb_t lb_t; /* opaque, owned by the library */

typedef struct {
    int32_t nx, ny, nz;     /* lattice size, >= 1 each; every site is fluid */
    int32_t bc[3];          /* per axis x,y,z: 0 periodic, 1 halfway bounce-back walls at both
                               faces (walls at -1/2 and n-1/2) */
    int32_t storage;        /* LB_STORE_* */
    int32_t kernel;         /* LB_KERNEL_* */
    double tau_r, tau_b;    /* relaxation times of the components, > 1/2 (eq:eq3) */
    double A;               /* surface-tension perturbation amplitude, >= 0 */
    double beta;            /* recolouring segregation parameter, in [0, 1] */
    double nc_strength;     /* near-contact strength A of Sec. 4 (0 = off) */
    int32_t nc_range;       /* probe range K in sites, 0..LB_MAX_NC_RANGE */
    int32_t scale_log2;     /* LB_STORE_F16 scale exponent; 0 = default (16) */
    double nc_hmin;         /* h_min: full strength for h <= h_min, h^-3 decay beyond */
    double body_force[3];   /* uniform force density */
    double eps_g;           /* |G| at or below which the interface normal is zero;
                               <= 0 selects 1e-12 (F64) or 1e-6 (other storage) */
    double g_iface;         /* |G| threshold of interface sites for the near-contact
                               probe; <= 0 selects 0.05 */
    double wall_velocity[6][3]; /* velocity of each wall face, faces -x,+x,-y,+y,-z,+z
                               (used on wall axes only; zero = resting walls).  A
                               population reflected by a moving face gains
                               2 w_i (c_i . U)/c_s^2 (reference density 1), shared
                               between the components by the reflecting site's
                               rho_k/rho; edges get the sum of both faces' terms.
                               The sheared channel of Sec. 5 slides two walls at +-U. */
    int32_t model;          /* LB_MODEL_*.  LB_MODEL_SHAN_CHEN replaces the perturbation,
                               recolouring and near-contact force (A, beta, nc_* unused) by
                               the force F^k(x) = -g_sc rho_k(x) sum_i w_i rho_k'(x + c_i) c_i
                               on each component k (k' the other one; a neighbour beyond a
                               wall is its mirror image), entering each component's
                               exact-difference source with its share (rho_k/rho) of the
                               body force.  Raw storage (F64, F32) and two-pass steps only. */
    double g_sc;            /* Shan-Chen coupling G_C (> 0 repels the components) */
} lb_params;

/* Create a lattice on the current HIP device: the problem statement of
 * Sec. 2 (D3Q19 populations on a cubic lattice, eq:eq1 to eq:equil) for the
 * two components of Sec. 2.1 (eq:twobgk), with the relaxation times, forces
 * and boundaries of lb_params.  Allocates the two population buffers
 * (ping-pong) and the phase-field scratch; the library owns them.
 * hip_stream: a hipStream_t to order all work on, or NULL for the default
 * stream.  On success *out is a new handle; nothing is allocated on failure.
 * LB_EINVAL: size < 1, tau <= 1/2, nc_range outside 0..LB_MAX_NC_RANGE,
 * unknown storage or kernel, lattice too large for 32-bit site indices. */
int lb_create(const lb_params* params, void* hip_stream, lb_t** out);

/* Set the initial state f^k_i = f^eq_i(rho_k, u) (Sec. 2, eq:equil).
 * rho_r, rho_b: N = nx*ny*nz component densities; u: 3N velocity (SoA) or
 * NULL for zero.  dtype: LB_DTYPE_*.  The densities must be >= 0 with
 * rho_r + rho_b > 0 (not checked on device pointers).  Resets the step count. */
int lb_init_fields(lb_t* h, const void* rho_r, const void* rho_b, const void* u, int32_t dtype,
                   int32_t on_device);

/* Initial state from a droplet list instead of fields: phase field
 * phi0(x) = max(background, max_j tanh((R_j - d_j(x))/width)) over droplets
 * with d_j <= R_j + 6 width (d_j the distance to centre j, minimum image on
 * periodic axes), rho_r = rho0 (1 + phi0)/2, rho_b = rho0 (1 - phi0)/2, u = 0;
 * then as lb_init_fields.  centres: n x 3 (x, y, z) and radii: n, host memory. */
int lb_init_droplets(lb_t* h, const double* centres, const double* radii, int32_t n, double width,
                     double background, double rho0);

/* Enqueue n >= 0 full steps of the update: collision with the mixture BGK
 * rate (Sec. 2.1, eq:twobgk; Sec. 2, eq:eq3), the exact-difference force
 * source (Sec. 2.1, eq:edm) of the body force plus the near-contact force
 * (Sec. 4, F_rep equation), the colour-gradient perturbation and recolouring
 * (or the Shan-Chen force of Sec. 2.1, eq. shanchen_force, per lb_params.model),
 * then streaming (Sec. 2, after eq:eq3) with periodic or bounce-back axes.
 * LB_ESTATE before lb_init_fields; LB_EDEVICE when a launch fails. */
int lb_step(lb_t* h, int32_t n);

/* As lb_step, timing every pass with HIP events on the handle's stream;
 * blocks until the n steps are done.  kernel_ms (host, 3 values) receives the
 * mean milliseconds per step of: [0] the phase-field pass (two-pass) or the
 * phase-field assembly (one-read), [1] the collide-and-stream pass, [2] the
 * whole step. */
int lb_step_timed(lb_t* h, int32_t n, double kernel_ms[3]);

/* Moments of the current state (Sec. 2, eq:eq2): rho_r, rho_b (N each) and the
 * bare momentum mom = sum_i (f^r_i + f^b_i) c_i (3N, SoA).  Any of the three may
 * be NULL.  The physical velocity is (mom + F/2)/rho with F the force density
 * of the last step.  totals (host, may be NULL) receives 7 compensated FP64
 * (sum, correction) pairs, in order: total red mass, total blue mass, momentum
 * x, y, z, kinetic energy sum |mom|^2/(2 rho), and the number of sites with a
 * non-finite or non-positive density; each total is sum + correction. */
int lb_moments(lb_t* h, void* rho_r, void* rho_b, void* mom, int32_t dtype, int32_t on_device,
               double totals[14]);

/* Korteweg-tensor diagnostic of the coarse-graining pipeline (Sec. 4.1: the
 * Korteweg tensor from the Laplacian and gradient products of the field, and
 * the projection of fine data by block averages).  The field is the phase
 * field phi = (rho_r - rho_b)/(rho_r + rho_b) of the current state, as the
 * next collision sees it; at every site
 *   K_ab = lambda [phi Lap(phi) + |grad phi|^2 / 2] delta_ab - lambda d_a phi d_b phi
 * with grad phi = 3 sum_i w_i c_i phi(x + c_i) and
 * Lap(phi) = 6 sum_i w_i (phi(x + c_i) - phi(x)), sites beyond a wall replaced
 * by their mirror images.  K and phi are averaged over blocks of b x b x b
 * sites (b = 1, 2, 4 or 8, dividing every extent).
 * k_blocks: 6 x Nc values (xx, yy, zz, xy, xz, yz, each [nz/b][ny/b][nx/b]);
 * phi_blocks: Nc values; either may be NULL, not both; dtype LB_DTYPE_F64 or
 * LB_DTYPE_F32; on_device selects device (caller's stream order) or host
 * buffers.  accumulate != 0 adds to the outputs instead of overwriting them
 * (device outputs only), so that b calls over b consecutive steps give the
 * space-time block of B = b^4 values once divided by b.  Uses the handle's
 * phase-field scratch; allocates only when staging host outputs.
 * Errors: LB_EINVAL (arguments), LB_ESTATE (before lb_init_fields). */
int lb_korteweg(lb_t* h, double lambda, int32_t b, void* k_blocks, void* phi_blocks, int32_t dtype,
                int32_t on_device, int32_t accumulate);

/* Export the populations f_i(x, t) (post-streaming state) as [2][19][N]
 * values of the given dtype.  For 16-bit storage these are the decoded values. */
int lb_get_state(lb_t* h, void* f, int32_t dtype, int32_t on_device);

/* Import populations in the layout of lb_get_state (16-bit storage re-encodes
 * them).  Keeps the step count. */
int lb_set_state(lb_t* h, const void* f, int32_t dtype, int32_t on_device);

/* Raw storage of the current state (checkpoint): lb_state_bytes gives the
 * size; lb_save_raw/lb_load_raw copy it out/in unchanged (bitwise resume). */
int64_t lb_state_bytes(const lb_t* h);
int lb_save_raw(lb_t* h, void* dst, int32_t on_device);
int lb_load_raw(lb_t* h, const void* src, int32_t on_device);

/* Steps taken since lb_init_fields. */
int64_t lb_step_count(const lb_t* h);

/* Kernel lb_step actually uses (LB_KERNEL_TWOPASS or LB_KERNEL_FUSED). */
int lb_kernel_in_use(const lb_t* h);

/* Release every buffer of the handle (after finishing its queued work); the
 * handle is invalid afterwards. */
int lb_destroy(lb_t* h);

/* Message of the calling thread's last failure ("" if none). */
const char* lb_last_error(void);

/* Tile shape of one kind of tile kernel for one storage type, for this
 * process: rows ty of a 64-wide tile and planes tz of the z chunk a workgroup
 * marches; 0 leaves the library's choice (measured defaults, or the
 * LB_*_TY / LB_*_TZ environment variables).  Lattices take the setting at
 * each step (a one-read lattice whose tile shape changed re-sums its phase
 * field before its next step); a batch takes it at lb_batch_create.  Rows
 * that do not fit the LDS budget are halved until they do.  For tools that
 * time tile shapes (the package's autotuner) and for callers applying their
 * results.  Results of two-pass steps do not depend on the tile shape; the
 * one-read and batched steps' phase sums follow their tile boxes, so their
 * results move by rounding (a batched job equals, bitwise, the same lattice
 * stepped alone by the one-read step on the batch's tile boxes).  Not
 * thread-safe against concurrent steps.
 * Errors: LB_EINVAL (unknown kind or storage, ty or tz out of range). */
int lb_set_tiles(int32_t kind, int32_t storage, int32_t ty, int32_t tz);

/* Bytes of device memory a lattice with these parameters holds. */
int64_t lb_footprint_bytes(const lb_params* params);

/* Measurement aid for the roofline of the one-read step (not part of the
 * method): the memory access pattern of the FP32 one-read step on a periodic
 * lattice of params' sizes, with no arithmetic -- per site the 19 (t_i, d_i)
 * pair loads at the pull's upstream sites and the 19 pair stores, on that
 * step's tiles, z chunks, workgroup-to-XCD mapping, two barriers per plane and
 * LDS allocation (params->storage is ignored; tile settings apply as for an
 * FP32 lattice).  Allocates two population buffers, runs 2 untimed and `reps`
 * timed launches on its own stream, frees them, and stores the average launch
 * duration in milliseconds in *ms.  The rate it gives bounds what the
 * collide-and-stream kernel can reach with this access pattern on the device.
 * Errors: LB_EINVAL (params, reps < 1, walls, a lattice the one-read step does
 * not take, ms NULL), LB_EDEVICE (allocation, launch). */
int lb_pattern_ms(const lb_params* params, int32_t reps, double* ms);

/* ------------------------------------------------------------------------
 * Batched form: many independent lattices (jobs) of uneven sizes and
 * parameters advanced together: each step is the one-read step of every
 * active job in two persistent kernel launches (the face-site assembly of the
 * phase field, then the collide-and-stream tiles), replayed as a captured HIP
 * graph of steps.
 * All jobs of a batch share one storage type.  Job populations live in one
 * arena owned by the batch; admission fails with LB_ENOMEM when the arena has
 * no room, so the arena size is the HBM budget.
 * ------------------------------------------------------------------------ */
typedef struct lb_batch_t lb_batch_t;

/* max_jobs: slots; arena_bytes: device memory for job populations;
 * storage: LB_STORE_*; graph_steps: steps per captured graph (even, >= 2).
 * hip_stream NULL: the batch creates its own stream (graph capture cannot use
 * the legacy default stream). */
int lb_batch_create(int32_t max_jobs, int64_t arena_bytes, int32_t storage, int32_t graph_steps,
                    void* hip_stream, lb_batch_t** out);

/* Admit one job that will run `steps` steps: validates params (storage must
 * equal the batch's; colour-gradient model; near-contact range at most 2; no
 * moving walls), places it in the arena (two population buffers and two
 * phase-sum buffers), writes its initial state f^eq(rho_k, u) and, when
 * steps >= 1, takes its first step here with the single lattice's one-read
 * step on the batch's tile boxes (a 16-bit job from its raw FP32 initial
 * state, so 16-bit jobs need steps >= 1; each keeps its own deviation scale
 * 2^scale_log2).  *slot gets its slot index.  LB_EINVAL for invalid
 * parameters, a 16-bit job with steps = 0 or a job too large for the step's
 * 32-bit buffer offsets; LB_ENOMEM when no slot or arena space is free.
 * Synchronises the stream. */
int lb_batch_add(lb_batch_t* b, const lb_params* params, const void* rho_r, const void* rho_b,
                 const void* u, int32_t dtype, int32_t on_device, int64_t steps, int32_t* slot);

/* As lb_batch_add with the initial state of lb_init_droplets. */
int lb_batch_add_droplets(lb_batch_t* b, const lb_params* params, const double* centres,
                          const double* radii, int32_t n, double width, double background,
                          double rho0, int64_t steps, int32_t* slot);

/* Arena bytes one job with these parameters takes (-1 if invalid). */
int64_t lb_batch_job_bytes(const lb_params* params);

/* Remove a job and free its arena space (after its queued work). */
int lb_batch_remove(lb_batch_t* b, int32_t slot);

/* Advance the batch by n global steps: every job inside its step window
 * takes a step each time (full multiples of graph_steps replay the captured
 * graph; a remainder runs eagerly).  A job stops after its `steps` steps and
 * keeps its final state until removed. */
int lb_batch_step(lb_batch_t* b, int32_t n);

/* Per-job moments and state export, as lb_moments / lb_get_state. */
int lb_batch_moments(lb_batch_t* b, int32_t slot, void* rho_r, void* rho_b, void* mom,
                     int32_t dtype, int32_t on_device, double totals[14]);
int lb_batch_get_state(lb_batch_t* b, int32_t slot, void* f, int32_t dtype, int32_t on_device);

/* Steps the job in `slot` has taken; -1 for an empty slot. */
int64_t lb_batch_job_steps(const lb_batch_t* b, int32_t slot);

/* Arena bytes still free (largest contiguous block). */
int64_t lb_batch_free_bytes(const lb_batch_t* b);

int lb_batch_destroy(lb_batch_t* b);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the seven
 * compensated totals of lb_moments (same order and meaning: red mass, blue
 * mass, momentum x, y, z, kinetic energy, non-finite or non-positive sites;
 * (sum, correction) pairs) of a population state the caller holds in device
 * memory, in the layout of lb_get_state ([2][19][N], f^r then f^b; dtype
 * LB_DTYPE_F64 or LB_DTYPE_F32).  params: only nx, ny, nz are read.
 * totals: device memory, 14 doubles.  Enqueued on hip_stream (NULL = the
 * default stream); does not synchronise.  Allocates nothing: the per-block
 * partial sums live in a static array of the library (512 x 7 (sum,
 * correction) pairs = 57,344 bytes on each device it runs on, held until the
 * process ends), shared by every call on that device, so calls that overlap
 * on one device race; every call rewrites all of it before reading it.
 * Errors: LB_EINVAL (NULL pointer, bad dtype, size < 1 or >= 2^31 sites),
 * LB_EDEVICE (no device, launch failure).
 * ------------------------------------------------------------------------ */
int lb_state_totals_noalloc(const lb_params* params, const void* f, int32_t dtype, double* totals,
                            void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LB_H */
