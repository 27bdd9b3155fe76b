/*
 * lbpf.h -- C ABI of the MI355X (gfx950) lattice-Boltzmann phase-field library.
 *
 * The library advances the three-field phase-field model of dilute binary-alloy
 * solidification of Cartalade, Younsi & Plapp, "Lattice Boltzmann simulations
 * of 3D crystal growth: numerical schemes for a phase-field model with
 * anti-trapping current" (arXiv:1602.07483):
 *   phase field phi       -- Sec. 3.2, non-local BGK scheme, eq. (LBE_Eq_Phase),
 *                            equilibrium eq. (Feq_Phase), source eq. (LBE_SourceTerm),
 *                            relaxation time eq. (LBE_RelaxationTime);
 *   supersaturation U     -- Sec. 3.3, reformulated equation (Supersaturation_Bis),
 *                            BGK scheme eq. (LBE_Eq_Transport), equilibrium
 *                            eq. (Feq_Transport), relaxation eq. (RelaxationTime_Concentration);
 *   temperature theta     -- Sec. 3.1, BGK scheme eq. (LBE_Eq_Temp) with
 *                            eqs. (EqFunction_Tempr), (Source_Tempr), (ThermalDiffusivity);
 * on the D3Q7, D3Q15 or D3Q19 lattice (Sec. 3.4, Tables 1 and 2) -- U and theta
 * optionally on another one than phi (lbpf_grid.lattice_ut) -- in the order of
 * Sec. 3.4 "Algorithm implementation": phi first, then U and theta with the
 * new phi; split collision (eq. Collision_Stage) and streaming
 * (eq. Deplacement_STD); bounce-back walls.
 *
 * Conventions
 *  - Every call returns an lbpf_status (0 = success, < 0 = error).  After an
 *    error, lbpf_last_error(ctx) describes it.
 *  - Host field arrays are double, shape [nz][ny][nx] with x fastest
 *    ("canonical layout"), owned by the caller; the library copies them.
 *  - The context owns all device memory.  It is created on the current HIP
 *    device and runs on the borrowed HIP stream given at creation; with NULL
 *    the context creates and owns a non-blocking stream of default priority.
 *    A borrowed stream must belong to the HIP runtime this library is
 *    linked against (the system ROCm); a package that bundles its own HIP
 *    runtime has streams of its own that are not interchangeable, so pass
 *    NULL (or that package's default stream, which is NULL) there.
 *    A context is not thread-safe; one context per stream.
 *  - Work is asynchronous on that stream except where a call says it
 *    synchronises.
 *  - Units: the model parameters are in the paper's (physical) units, the
 *    node spacing is dx and the time step dt.  Positions returned by the
 *    reductions are in node-index units.
 */
#ifndef LBPF_H
#define LBPF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbpf_ctx lbpf_ctx;
typedef struct lbpf_batch lbpf_batch;

typedef enum {
    LBPF_OK = 0,
    LBPF_EINVAL = -1,     /* invalid argument or parameter set */
    LBPF_ENOMEM = -2,     /* device or host allocation failed */
    LBPF_EDEVICE = -3,    /* a HIP runtime call failed */
    LBPF_EUNSTABLE = -4,  /* health check failed: non-finite value or |phi| > 1 + 1e-3 */
    LBPF_ESTATE = -5,     /* call out of order (e.g. step before set_fields) */
    LBPF_EIO = -6         /* a file could not be read or written */
} lbpf_status;

/* D3Q7 (e^2 = 1/4), D3Q15 and D3Q19 (e^2 = 1/3): Sec. 3.4, Tables 1 and 2. */
typedef enum { LBPF_D3Q7 = 7, LBPF_D3Q15 = 15, LBPF_D3Q19 = 19 } lbpf_lattice;

/* Walls lie half a link outside the first/last node of each axis. */
typedef enum {
    LBPF_WALL_NOFLUX = 0,    /* half-way bounce-back (zero flux, Sec. 4) */
    LBPF_WALL_SYMMETRY = 1   /* mirror plane: specular reflection */
} lbpf_wall;

/* How the populations are stored in HBM.  Every type stores the deviation of
 * each population from its rest equilibrium (w_i phi, (A_i + B_i q/zeta) U,
 * w_i theta) and updates it in increment form.  Arithmetic is FP32 except F64. */
typedef enum {
    LBPF_F32 = 0,       /* FP32 deviations, FP32 fields and collision */
    LBPF_F16_DEV = 1,   /* FP16 deviations, FP32 fields and collision */
    LBPF_BF16_DEV = 2,  /* BF16 deviations, FP32 fields and collision */
    LBPF_F64 = 3        /* FP64 everywhere (verification build) */
} lbpf_storage;

typedef enum {
    LBPF_ANISO_CUBIC = 0,   /* eq. (Anisotropic-Function_As): 1 - 3 eps + 4 eps sum n^4 */
    LBPF_ANISO_K41K61 = 1   /* eq. (As_K41-K61): cubic harmonics K41 (eps) + K61 (delta) */
} lbpf_aniso;

typedef struct {
    int32_t nx, ny, nz;     /* nodes per axis, each >= 1 */
    int32_t lattice;        /* lbpf_lattice */
    int32_t wall[6];        /* lbpf_wall for faces -x,+x,-y,+y,-z,+z */
    int32_t storage;        /* lbpf_storage */
    int32_t lattice_ut;     /* lattice of U and theta: 0 = that of phi, else an
                               lbpf_lattice.  Each scheme then takes the e^2 of
                               its own lattice (Sec. 4.1 runs phi on D2Q9 and
                               theta on D2Q5).  Batches take it per domain. */
} lbpf_grid;

typedef struct {
    double dx, dt;          /* node spacing, time step */
    double W0, tau0;        /* interface width, phase-field time scale */
    double lambda;          /* coupling constant of eq. (PhaseField_KarmaRappel) */
    double Mcinf;           /* M c_inf, scaled liquidus slope */
    double k;               /* partition coefficient, 0 < k < 1 */
    double D, kappa;        /* solute and thermal diffusivities */
    int32_t aniso;          /* lbpf_aniso */
    double eps, delta;      /* anisotropy strengths (delta used by K41K61 only) */
    int32_t reduce_every;   /* >0: record the reductions every that many steps */
    double centre[3];       /* reference point of the tip positions (node units) */
    double vel[3];          /* uniform imposed velocity of the thermal (or
                               solute) carrier, physical units: the theta
                               equilibrium gains the advective term of the
                               advection-diffusion equilibrium of Sec. 3.1,
                               w_i theta (1 + e_i.v dt / (e^2 dx)). All zero
                               (the paper's runs) is the pure-diffusion scheme.
                               Nonzero runs k_ut on its advection tile, 32x8
                               (FP64 32x4): lbpf_set_launch refuses other k_ut
                               tiles, lbpf_autotune does not try them. Refused by
                               lbpf_batch_create; non-finite -> LBPF_EINVAL. */
    int32_t skip_U;         /* 1: pure substance (Mcinf must be 0, as in the
                               thermal dendrites of Sec. 4.1 and 4.3, where U
                               does not act on phi): U is not advanced, its
                               field keeps the value lbpf_set_fields gave it and
                               the h populations are left untouched; k_ut then
                               moves only the theta populations.  Runs k_ut on
                               its advection tile (32x8; FP64 32x4).  0: solve U.
                               Other values, or 1 with Mcinf != 0, are
                               LBPF_EINVAL; batches refuse 1. */
    int32_t skip_theta;     /* 1: isothermal (the alloy benchmark of Sec. 4.2
                               has theta = 0): the heat equation is not solved,
                               theta keeps the value lbpf_set_fields gave it
                               and the f populations are left untouched; k_ut
                               then moves only the U populations.  Runs k_ut on
                               its advection tile.  0: solve theta.  Other
                               values, 1 together with skip_U = 1 or with an
                               advective velocity, are LBPF_EINVAL; batches
                               refuse 1. */
} lbpf_params;

/* Diagnostics of one state, accumulated in FP64 on the device.  The paper
 * defines only the tip velocity (Sec. 4.1); the others are conservation and
 * health checks: solute content from the definition of U in Sec. 2,
 * c/c_inf = zeta(phi)(1 + (1-k)U). */
typedef struct {
    int64_t step;             /* time steps taken when the record was made */
    double solid_fraction;    /* mean of (1 + phi)/2 */
    double solute_mass;       /* sum of zeta(phi)(1 + (1-k)U) dx^3 */
    double enthalpy;          /* sum of (theta - phi/2) dx^3, conserved exactly */
    double tip[3];            /* furthest phi=0 crossing along +x,+y,+z minus centre
                                 (linear interpolation between nodes; NaN if none) */
    double phi_min, phi_max;
    double nonfinite;         /* count of non-finite phi, U, theta values */
    double sum_U, sum_phi;    /* sums of U and phi, times dx^3 */
    double tip_vel[3];        /* tip velocity along +x,+y,+z since the previous
                                 record of the history: (tip - tip_prev) dx /
                                 ((step - step_prev) dt), physical units (times
                                 tau0/W0 it is the dimensionless V_p of Sec.
                                 4.1).  NaN without an earlier record. */
} lbpf_reductions;

/* Create a context for one domain of the model of Sec. 2 (phase field
 * eq. PhaseField_KarmaRappel, supersaturation eq. Concentration_Echebarria
 * with the anti-trapping current eq. AntiTrapping_Current, temperature
 * eq. Temp_Ramirez), discretised by the schemes of Sec. 3.1-3.3 on the
 * lattice of Sec. 3.4 (Tables 1 and 2) with the bounce-back walls of
 * Sec. 3.4: validates the parameters, allocates the populations
 * (two lattices per field), the fields and the reduction buffers on the
 * current device.  Device arrays have their rows padded to a multiple of 32
 * values; that layout stays inside the library (every copy in or out uses
 * the packed [nz][ny][nx] layout).  Errors: EINVAL (n < 1, unsupported
 * lattice, storage, wall or anisotropy, k not in (0,1), dx, dt, W0,
 * tau0 <= 0, D or kappa < 0, eps outside [0, 0.25], reduce_every < 0,
 * non-finite vel, skip_U or skip_theta not 0/1 or in a refused combination),
 * ENOMEM, EDEVICE.  *out is NULL on error. */
lbpf_status lbpf_create(const lbpf_grid* grid, const lbpf_params* params,
                        void* hip_stream, lbpf_ctx** out);

/* Release every device buffer owned by the context.  NULL is accepted. */
lbpf_status lbpf_destroy(lbpf_ctx* ctx);

/* Load the initial fields (host, canonical layout, nx*ny*nz doubles each) and
 * set every population to its equilibrium (phi: eq. Feq_Phase with N from
 * grad phi; U: eq. Feq_Transport with the anti-trapping current zero; theta:
 * eq. EqFunction_Tempr).  Resets the step counter and the history.
 * Synchronises the stream.  Errors: EINVAL (NULL array), EDEVICE. */
lbpf_status lbpf_set_fields(lbpf_ctx* ctx, const double* phi, const double* U,
                            const double* theta);

/* Advance nsteps >= 0 time steps, asynchronously on the context stream.  One
 * step is the algorithm of Sec. 3.4: the phase-field node terms (a_s(n) of
 * eq. Anisotropic-Function_As or As_K41-K61, N of eq. TermesAnisotropes,
 * eta_phi of eq. LBE_RelaxationTime, Q_phi of eq. LBE_SourceTerm), the
 * non-local collision eq. Collision_Stage and streaming eq. Deplacement_STD
 * with bounce-back; then, with the new phi, U by eqs. LBE_Eq_Transport and
 * Feq_Transport (J_tot eq. Def_Jtot, S eq. Def_S, Q_U eq. Def_Qu) and theta
 * by eqs. LBE_Eq_Temp and EqFunction_Tempr (source eq. Source_Tempr).  When
 * reduce_every > 0 a reduction record is appended to the history after every
 * step whose count is a multiple of reduce_every.  Errors: ESTATE (no fields
 * yet), EINVAL (nsteps < 0), EDEVICE. */
lbpf_status lbpf_step(lbpf_ctx* ctx, int64_t nsteps);

/* Replay the step loop from a captured HIP graph of steps_per_graph time
 * steps (0 = plain launches; otherwise even, so that the two lattices are in
 * the same roles after each replay).  lbpf_step uses the graph for every
 * whole chunk that ends before the next reduction point and while kernel
 * timing is off; the graph is captured on first use and again after the
 * launch shape or the lattice parity changed.  Results are identical to
 * plain launches.  Errors: EINVAL (odd or negative). */
lbpf_status lbpf_set_graph(lbpf_ctx* ctx, int32_t steps_per_graph);

/* Wait for the stream, then check the most recent history record, if any:
 * returns EUNSTABLE when it holds a non-finite value or |phi| > 1 + 1e-3. */
lbpf_status lbpf_sync(lbpf_ctx* ctx);

/* Copy the current fields to host arrays (each may be NULL to skip it) and,
 * when red != NULL, compute a fresh reduction record of the current state:
 * the fields are the zeroth moments of the populations (phi = sum g_i,
 * U = sum h_i, theta = sum f_i, Sec. 3.1-3.3); the record holds the solid
 * fraction, the solute content zeta(phi)(1 + (1-k)U) summed over the nodes
 * (the definition of U in Sec. 2 solved for c/c_inf), the enthalpy, and the
 * tip position and velocity (V_p of Sec. 4.1).
 * Synchronises the stream.  Returns EUNSTABLE (after copying) when that
 * record fails the health check. */
lbpf_status lbpf_read(lbpf_ctx* ctx, double* phi, double* U, double* theta,
                      lbpf_reductions* red);

/* Copy up to max_records history records, oldest first, into out; *count
 * receives the number copied.  The history keeps the latest 8192 records.
 * Synchronises the stream. */
lbpf_status lbpf_history(lbpf_ctx* ctx, lbpf_reductions* out, int32_t max_records,
                         int32_t* count);

/* Element types of device-resident field arrays. */
typedef enum { LBPF_FIELD_F32 = 0, LBPF_FIELD_F64 = 1 } lbpf_field_type;

/* As lbpf_set_fields, with phi, U and theta in device memory of the
 * context's device ([nz][ny][nx], x fastest, element type dtype).  They are
 * read on the context's stream (the caller orders their production before
 * the call) and converted there to the context's field type (FP64 for the
 * F64 storage, FP32 otherwise, round to nearest); the equilibrium
 * populations follow as in lbpf_set_fields (Sec. 4 initial seed, equilibria
 * of eqs. (Feq_Phase), (Feq_Transport), (EqFunction_Tempr)).  The caller keeps
 * ownership.  Synchronises the stream before returning.  Errors: EINVAL
 * (NULL array, dtype not 0/1), EDEVICE. */
lbpf_status lbpf_set_fields_device(lbpf_ctx* ctx, const void* phi, const void* U, const void* theta,
                                   int32_t dtype);
/* Copy the current fields into device arrays of element type dtype (any of
 * the three may be NULL).  Asynchronous on the context's stream: the arrays
 * hold the values once the stream has reached this point (lbpf_sync).  No
 * reductions and no health check.  Errors: EINVAL, ESTATE (no fields set),
 * EDEVICE. */
lbpf_status lbpf_read_fields_device(lbpf_ctx* ctx, void* phi, void* U, void* theta, int32_t dtype);

/* Raw stored population bits of one field (0 = g/phi, 1 = h/U, 2 = f/theta),
 * layout [Q][nz][ny][nx], in the storage type.  Every storage type holds the
 * deviation of each population from its rest equilibrium (w_i phi,
 * (A_i + B_i q(phi)/zeta(phi)) U, w_i theta), so the stored state is the pair
 * (fields, deviations): a checkpoint is lbpf_read of the fields plus these
 * three arrays; a restore is lbpf_set_fields of the saved fields followed by
 * the three writes.  Q is the field's lattice (lbpf_grid.lattice for phi,
 * lattice_ut, when set, for U and theta); the size of dst/src is
 * Q*nx*ny*nz*lbpf_storage_bytes.
 * The device layout is the library's own (h and f share one array when
 * both fields are solved); a write of one field leaves the others' stored
 * bits unchanged.
 * Both synchronise; the fields are not changed by a write.
 * Errors: EINVAL (bad field, NULL), ESTATE (write before set_fields). */
lbpf_status lbpf_read_populations(lbpf_ctx* ctx, int32_t field, void* dst);
lbpf_status lbpf_write_populations(lbpf_ctx* ctx, int32_t field, const void* src);

/* Full populations (deviation + rest equilibrium) of one field in FP64,
 * layout [Q][nz][ny][nx] (Q as above), for inspection.  Allocates a
 * temporary device buffer of Q*nx*ny*nz doubles; synchronises.  Errors as above, ENOMEM. */
lbpf_status lbpf_read_populations_f64(lbpf_ctx* ctx, int32_t field, double* dst);

/* Streaming only (collision = identity) of all three population sets, raw
 * bits, with the wall rules, each set on its own lattice: checks the index
 * mapping.  Asynchronous. */
lbpf_status lbpf_debug_stream_only(lbpf_ctx* ctx, int64_t nsteps);

/* Per-node advective velocity of the heat equation (Sec. 3.1: the theta
 * equilibrium w_i theta (1 + e_i.v dt / (e^2 dx)) with v = v(x)), the step
 * toward a coupled flow solver that Sec. 5 outlines.  vx, vy, vz: host
 * arrays of n doubles each, same layout as the fields, physical units;
 * copied to the device in the compute type (FP32, FP64 for FP64 storage).
 * The field replaces lbpf_params.vel; all three NULL removes it.  It acts
 * from the next step and in the next lbpf_set_fields (whose theta
 * populations start from the advective equilibrium: set the field first to
 * start there).  Puts k_ut on its advection tile (32x8; FP64 32x4), the
 * only one with the advective variant, and drops a captured step graph.
 * Removing the field leaves k_ut's launch as it is.  Synchronises.
 * Errors: EINVAL (one or two NULL, non-finite value, skip_theta set),
 * ESTATE (a batch member), ENOMEM. */
lbpf_status lbpf_set_velocity_field(lbpf_ctx* ctx, const double* vx, const double* vy, const double* vz);

/* Per-kernel timing with HIP events recorded on the context stream around
 * each launch.  Enabling resets the accumulators.  lbpf_kernel_times
 * synchronises and returns the summed milliseconds and launch counts of the
 * phase-field kernel (index 0), the supersaturation/heat kernel (1) and the
 * reduction kernels (2). */
lbpf_status lbpf_set_timing(lbpf_ctx* ctx, int32_t enable);
lbpf_status lbpf_kernel_times(lbpf_ctx* ctx, double ms[3], int64_t launches[3]);

/* Launch shape of the step kernels: a tile of tile_x x tile_y nodes per
 * block (one thread per node), marching through zslab planes; xcd_remap = 1
 * deals each of the 8 XCDs one contiguous run of tiles (neighbouring tiles
 * then share that XCD's L2), 0 keeps the hardware's round-robin order.
 * Supported tiles: 64x2, 64x4, 32x4, 32x8, 32x16 (FP64 storage: 64x2 and
 * 32x4); zslab >= 1.  The shape changes speed only, never results.
 *
 * The two kernels of a step (kernel 0: k_phi, the phase-field update;
 * kernel 1: k_ut, the U and theta update) are separate launches, each with a
 * launch of its own.  lbpf_set_launch sets both (all or nothing);
 * lbpf_set_kernel_launch one.  lbpf_get_launch reports k_ut's, the kernel
 * that moves the most bytes; lbpf_get_kernel_launch either.
 * Defaults: k_phi 32x8 zslab 6, remap 1; k_ut 64x4 zslab 6 remap 0 (FP32)
 * or 32x8 zslab 6 remap 1 (16-bit); FP64 32x4 zslab 4 remap 1 for both.
 * With an advective velocity (lbpf_params.vel or a velocity field) k_ut
 * runs on its advection tile, 32x8 (FP64 32x4), the only one with the
 * advective variant.
 * Errors: EINVAL (unsupported shape, flag or kernel index; another k_ut
 * tile while advecting). */
lbpf_status lbpf_set_launch(lbpf_ctx* ctx, int32_t tile_x, int32_t tile_y, int32_t zslab,
                            int32_t xcd_remap);
lbpf_status lbpf_get_launch(lbpf_ctx* ctx, int32_t* tile_x, int32_t* tile_y, int32_t* zslab,
                            int32_t* xcd_remap);
lbpf_status lbpf_set_kernel_launch(lbpf_ctx* ctx, int32_t kernel, int32_t tile_x, int32_t tile_y,
                                   int32_t zslab, int32_t xcd_remap);
lbpf_status lbpf_get_kernel_launch(lbpf_ctx* ctx, int32_t kernel, int32_t* tile_x, int32_t* tile_y,
                                   int32_t* zslab, int32_t* xcd_remap);

/* Autotuner: times every supported tile shape with zslab in
 * {2,4,6,8,12,16} and both XCD orders (steps_per_candidate steps each, after
 * two untimed steps, with events around each kernel), keeps for each of the
 * two kernels its fastest launch, and restores the state it started from (a
 * temporary device snapshot of the populations and fields is allocated).
 * *best_ms_per_step (may be NULL) receives the sum of the two kernels' best
 * times.  Launches timed before the call are added to the lbpf_kernel_times
 * accumulators; the tuner's own are not.  Synchronises.
 * Errors: ESTATE (no fields yet), EINVAL, ENOMEM, EDEVICE. */
lbpf_status lbpf_autotune(lbpf_ctx* ctx, int32_t steps_per_candidate, double* best_ms_per_step);

/* The autotuner with a persisted result, so that a configuration is timed
 * once per machine type.  cache_path names a text file with one line per
 * tuned configuration:
 *   lbpf-autotune-2 k<kernel build> <gcnArchName> cu<CUs> q<lattice>
 *     qut<lattice_ut> s<storage> <nx>x<ny>x<nz> pin<0|1>
 *     <k_phi: tx ty zslab remap> <k_ut: tx ty zslab remap> <ms per step>
 * where the kernel build is a digest of the kernel sources the library was
 * compiled from (so launches tuned for other kernels are not reused) and
 * pin = 1 when k_ut runs one of its variants (advection, skip_U or
 * skip_theta).  If a line's key matches this context (kernel build, device
 * architecture and CU count, lattices, storage, domain size, pin), its
 * launches are set
 * without any timing and *hit = 1; *best_ms_per_step receives the stored
 * time.  Otherwise lbpf_autotune runs, its result is appended to the file
 * (created if missing) and *hit = 0.  Lines that do not parse or name a
 * launch this context refuses are skipped.  hit and best_ms_per_step may
 * be NULL.  Concurrent writers append whole lines; the first matching line
 * wins.
 * Errors: those of lbpf_autotune; EINVAL (NULL cache_path); EIO (the file
 * exists but cannot be read, or cannot be appended to: the tuned launches
 * are then set all the same). */
lbpf_status lbpf_autotune_cached(lbpf_ctx* ctx, int32_t steps_per_candidate, const char* cache_path,
                                 int32_t* hit, double* best_ms_per_step);

/* Bytes of one stored population for a storage type (0 if invalid). */
int32_t lbpf_storage_bytes(int32_t storage);

/* Plain device-to-device copy kernel of nbytes (multiple of 16, 16-byte
 * aligned pointers) on hip_stream, used as the bandwidth reference of the
 * benchmark.  Asynchronous.  Errors: EINVAL, EDEVICE. */
lbpf_status lbpf_bench_copy(void* dst, const void* src, int64_t nbytes, void* hip_stream);

/* Bandwidth reference kernels (measurement only, no part of the method):
 * mode 0 reads nbytes from src, mode 1 writes nbytes to dst, mode 2 copies
 * src to dst; width = bytes per lane and access (2, 4, 8 or 16); nontemporal =
 * 1 adds streaming cache hints; blocks = grid size in 256-thread blocks
 * (0: one thread per four elements, at most 4096 blocks), each thread
 * striding over the array with four accesses in flight.  Device pointers,
 * 16-byte aligned, nbytes a multiple of width; mode 0 may write one word at
 * dst.  Asynchronous on hip_stream.  Errors: EINVAL, EDEVICE. */
lbpf_status lbpf_bench_bandwidth(int32_t mode, int32_t width, int32_t nontemporal, int32_t blocks, void* dst,
                                 const void* src, int64_t nbytes, void* hip_stream);

/* Reductions of caller-held device fields, allocating nothing -- for callers
 * that cannot allocate device memory: code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc.  A variant of the reduction record
 * of lbpf_read (same kernels, same grid, so the same values bit for bit) that
 * needs no context: phi, U, theta are device arrays of the current device,
 * [nz][ny][nx] with x fastest and no padding, element type dtype
 * (LBPF_FIELD_F32 or _F64); k and dx as in lbpf_params; centre is a host
 * array of 3 doubles (node units).  rec receives, in device memory, 12
 * doubles: step (always 0), solid fraction, solute mass, enthalpy, tip x, y,
 * z (minus centre; NaN when no crossing), phi min, phi max, non-finite
 * count, sum U, sum phi -- the fields of lbpf_reductions in that order.
 * Asynchronous on hip_stream.  The per-block partial sums live in a fixed
 * scratch array of 1024 x 16 doubles (128 KiB) in the library's device
 * image, one per device, kept until the process ends: calls that overlap on
 * one device race on it and must be serialised (one stream, or events).
 * Every call rewrites the whole part of the scratch it reads, so nothing
 * must be cleared between calls.  At most 2^31 nodes.  No hipMalloc, no
 * hipFree, no memset.  Errors (lbpf_last_error(NULL)): EINVAL (NULL
 * pointer, bad dtype, n < 1 or > 2^31, k outside (0,1), dx <= 0), EDEVICE. */
lbpf_status lbpf_reduce_fields_noalloc(const void* phi, const void* U, const void* theta, int32_t dtype,
                                       int32_t nx, int32_t ny, int32_t nz, double k, double dx,
                                       const double* centre, double* rec, void* hip_stream);

/* Description of the last error on ctx (or of the last failed creation when
 * ctx is NULL); valid until the next call on the same context. */
const char* lbpf_last_error(const lbpf_ctx* ctx);

/* ---- Ensembles of independent domains ------------------------------------
 * A batch holds n domains (own grid, lattices D3Q7, D3Q15 or D3Q19 for phi
 * and for U, theta (lattice_ut), parameters;
 * one storage type for all) on one stream.  Each domain is an lbpf_ctx
 * reached with lbpf_batch_domain, through which its fields are set and read
 * with the calls above (lbpf_step on it is refused: ESTATE).  lbpf_batch_step
 * advances every domain with one launch per lattice type and kernel (k_phi
 * grouped by the phi lattice, k_ut by the U/theta lattice): a work
 * table maps each block to a (domain, tile) pair, ordered so that each XCD
 * receives a contiguous run of tiles; with lbpf_batch_set_graph the loop is
 * replayed from a captured graph.  A domain follows the same arithmetic as
 * when it is stepped alone; the batch kernels are compiled separately and
 * may contract floating-point operations differently, so FP32 results agree
 * with the single-domain ones to a few units in the last place, not bit for
 * bit.  Step chunking and graph replay do not change the batch's results;
 * another tile shape (lbpf_batch_set_launch) is another instantiation of the
 * batch kernels and may round a few ulp differently. */
lbpf_status lbpf_batch_create(int32_t n, const lbpf_grid* grids, const lbpf_params* params,
                              void* hip_stream, lbpf_batch** out);
/* Domain i (borrowed pointer, valid until lbpf_batch_destroy); NULL if out of range. */
lbpf_ctx* lbpf_batch_domain(lbpf_batch* b, int32_t i);
/* As lbpf_set_graph, for the whole batch. */
lbpf_status lbpf_batch_set_graph(lbpf_batch* b, int32_t steps_per_graph);
/* Launch of the batch kernel k_phi (kernel 0) or k_ut (1) over all domains:
 * tile shape (as lbpf_set_kernel_launch: 64x2, 64x4, 32x4, 32x8, 32x16;
 * FP64 64x2 and 32x4) and z slab.  Takes effect at the next step (the work
 * tables are rebuilt and a captured graph is recaptured).  The default is
 * 32x8 (FP64 32x4) with slab 8 (16-bit storage) or 4.  Errors: EINVAL. */
lbpf_status lbpf_batch_set_launch(lbpf_batch* b, int32_t kernel, int32_t tile_x, int32_t tile_y, int32_t zslab);
lbpf_status lbpf_batch_get_launch(lbpf_batch* b, int32_t kernel, int32_t* tile_x, int32_t* tile_y,
                                  int32_t* zslab);
/* Autotuner of the batch launches: times every tile shape of the storage
 * type with z slabs {2, 4, 6, 8, 12} (both kernels alike, two untimed steps
 * and steps_per_candidate timed steps each, events around the k_phi and the
 * k_ut launches), keeps for each kernel its fastest launch, and restores
 * every domain's state (a temporary device snapshot of all populations and
 * fields is allocated).  *best_ms_per_step (may be NULL) receives the sum of
 * the two kernels' best times per batch step.  Synchronises.  Errors:
 * EINVAL, ESTATE (a domain without fields, parities differ), EDEVICE. */
lbpf_status lbpf_batch_autotune(lbpf_batch* b, int32_t steps_per_candidate, double* best_ms_per_step);
/* Advance every domain nsteps; all must have fields and equal step parity.
 * Asynchronous.  Errors: ESTATE, EINVAL, EDEVICE. */
lbpf_status lbpf_batch_step(lbpf_batch* b, int64_t nsteps);
lbpf_status lbpf_batch_sync(lbpf_batch* b);
lbpf_status lbpf_batch_destroy(lbpf_batch* b);
const char* lbpf_batch_last_error(const lbpf_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* LBPF_H */
