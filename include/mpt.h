/*
 * mpt.h -- C ABI of libmpt: the per-particle time step of a Lagrangian
 * transport model on one AMD Instinct MI355X (gfx950).
 *
 * The operation is the model's "chemistry-physics processing" loop
 * (Sec. 3.2, module list; Sec. 3.4: every air parcel is advanced
 * independently): for each parcel and time step,
 *   - module_timesteps  (Sec. 4.3): skip parcels that are not active;
 *   - module_advection  (Sec. 3.2): kinematic trajectory from the winds,
 *     here explicit midpoint with 4D (lon, lat, p, t) interpolation;
 *   - module_position   (Sec. 3.2): keep the parcel inside the domain;
 *   - module_diffusion_turb / module_diffusion_meso (Sec. 3.2): stochastic
 *     perturbations, with the random numbers of Sec. 4.3 (Listing 6: three
 *     normals per parcel and step for each) drawn from a counter-based
 *     Philox4x32-10 keyed by (parcel id, step, purpose);
 *   - particle sorting by grid box (Sec. 6 lists the sorting modules).
 * The meteorological time levels (met0/met1 of Sec. 4.1's data regions)
 * live on the device for the whole run; the parcel state (atm_t, Sec. 4.4)
 * is SoA in caller-owned device memory.
 *
 * Conventions
 *   - Units: lon/lat in degrees, p in hPa, u/v in m/s, w (omega) in hPa/s,
 *     time in seconds, diffusivities in m^2/s.
 *   - Ownership: the caller owns every device buffer (particles, both
 *     ping-pong sets, the workspace).  The library never allocates device
 *     memory; it carves met storage and sort scratch out of the workspace.
 *     Host arrays passed in (plev, release table) are copied at the call.
 *   - Streams: every call that enqueues work takes a hipStream_t as void*
 *     (NULL = the null stream).  Device pointers must stay valid until the
 *     work enqueued on that stream has completed.  The library never
 *     synchronizes; device faults surface at the caller's next sync.
 *   - Errors: every call validates its arguments synchronously and returns
 *     a negative mpt_status with nothing enqueued on error.  No exceptions
 *     cross the ABI.  One context per stream; contexts are independent.
 *   - Determinism: results are a pure function of (inputs, seed, step
 *     indices); they do not depend on the number of parcels, their order in
 *     memory or whether they were sorted.
 */
#ifndef MPT_H
#define MPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpt_ctx mpt_ctx; /* opaque */

typedef enum {
    MPT_OK = 0,
    MPT_ERR_ARG = -1,          /* null/misaligned pointer, bad size or value */
    MPT_ERR_STATE = -2,        /* met level not initialized, no release table */
    MPT_ERR_TIME = -3,         /* a step falls outside the resident met levels */
    MPT_ERR_WORKSPACE = -4,    /* workspace too small or n > n_max */
    MPT_ERR_HIP = -5,          /* a HIP runtime call failed (or no GPU) */
    MPT_ERR_UNSUPPORTED = -6   /* combination of options not provided */
} mpt_status;

/* Arithmetic of the step.  F64: FP64 throughout.  F32: FP32 interpolation,
 * tendencies and random numbers; FP64 position accumulation and longitude
 * wrap.  The mesoscale state (up, vp, wp) is double for F64, float for F32. */
typedef enum { MPT_MATH_F64 = 0, MPT_MATH_F32 = 1 } mpt_math;

/* Storage of the wind fields.  BF16 / F16 store q = RNE(f / s) with one FP32
 * scale s = max|f| per (variable, level, time level) and decode q * s in
 * FP32.  BF16 and F16 require MPT_MATH_F32 and dt <= 1.998 dt_met (else
 * MPT_ERR_UNSUPPORTED); their kernel launches advance at most
 * floor(0.999 dt_met / dt + 1/2) steps whatever fuse says, so that the
 * times one launch reads span less than one met interval. */
typedef enum { MPT_DT_F32 = 0, MPT_DT_BF16 = 1, MPT_DT_F16 = 2 } mpt_dtype;

/* Module flags (mpt_params.flags).  MPT_CONV and MPT_SEDI (module_convection
 * and module_sedi, Sec. 3.2) act in mpt_step and mpt_step_graph only, after
 * the diffusion, and need the fields of mpt_set_met_phys on every resident
 * level. */
enum { MPT_ADVECT = 1u, MPT_TURB = 2u, MPT_MESO = 4u, MPT_CONV = 8u, MPT_SEDI = 16u };

/* Regular lon-lat grid with fixed pressure levels and nt resident time
 * levels (read_met / read_met_periodic, Sec. 3.1).
 *   nx * dlon == 360 (periodic longitude starting at lon0);
 *   lat0 == -90, lat0 + (ny-1)*dlat == 90;
 *   plev: host array of nz pressures [hPa], strictly decreasing (copied);
 *   time level l sits at t_met0 + l*dt_met, l = 0 .. nt-1.
 * Requires nx >= 2, ny >= 3, nz >= 2, nt >= 2, nx*ny*nz < 2^31. */
typedef struct {
    int32_t nx, ny, nz, nt;
    double lon0, dlon, lat0, dlat;
    const double *plev;
    double t_met0, dt_met;
    int32_t dtype;       /* mpt_dtype */
    int32_t reserved;    /* must be 0 */
} mpt_grid;

/* Control parameters (read_ctl, Sec. 3.1).  Step n starts at
 * t_start + n*dt.  Every step n used must satisfy
 * t_met0 <= t_n and t_n + dt <= t_met0 + (nt-1)*dt_met. */
typedef struct {
    double dt, t_start;        /* s, dt > 0 */
    double turb_dx, turb_dz;   /* turbulent diffusivities [m^2/s], >= 0 */
    double meso_fh, meso_fv;   /* mesoscale factors, >= 0 */
    uint64_t seed;             /* Philox key */
    int32_t sort_interval;     /* mpt_step sorts before every step n with
                                  n % sort_interval == 0; 0 = never */
    int32_t math;              /* mpt_math */
    uint32_t flags;            /* MPT_ADVECT | MPT_TURB | MPT_MESO */
    int32_t fuse;              /* max steps one kernel launch may advance
                                  with the state kept in registers (>= 1) */
    double conv_cape;          /* MPT_CONV: CAPE threshold [J/kg], finite */
    double sedi_radius;        /* MPT_SEDI: particle radius [m], > 0 */
    double sedi_density;       /* MPT_SEDI: particle density [kg/m^3], > 0 */
    int32_t presort;           /* 0 or 1, see below */
    int32_t reserved;          /* must be 0 */
} mpt_params;
/* Sort keys inside the step.  Without scenarios, a kernel launch of mpt_step
 * or mpt_step_graph that ends where a sort follows also computes the sort
 * keys of its final positions, and that sort skips its own key pass.  With
 * presort = 1 the last launch of each mpt_step call does the same, and the
 * keys are kept for the next sort of the same particles (same primary lon
 * array and count): mpt_sort_particles, or the sort an mpt_step call
 * starting on a multiple of sort_interval begins with; any other call that
 * moves or sorts parcels drops them.  A caller that changes positions
 * itself in between gets a sort by the previous cells: still a permutation
 * of the whole state, so results do not change (they never depend on the
 * order). */

/* Parcel state (atm_t, Sec. 4.4, plus the mesoscale state of `cache`).
 * All pointers are device pointers to arrays of n elements.
 *   lon, lat, p: double; id: uint32 (the Philox counter uses it);
 *   up, vp, wp: double (MPT_MATH_F64) or float (MPT_MATH_F32);
 *   scen: uint16 scenario index per parcel, or NULL (all active from step 0).
 * The *2 set has the same types and is the target of mpt_sort_particles; it
 * may be NULL when no sort is requested.  The two sets must not overlap. */
typedef struct {
    int64_t n;
    double *lon, *lat, *p;
    uint32_t *id;
    void *up, *vp, *wp;
    uint16_t *scen;
    double *lon2, *lat2, *p2;
    uint32_t *id2;
    void *up2, *vp2, *wp2;
    uint16_t *scen2;
} mpt_particles;

/* Bytes of device workspace needed for this grid and up to n_max parcels
 * (met storage for nt levels, level table, sort scratch).  Returns 0 on
 * invalid arguments.  n_max < 2^32 - 1 (the sort's positions are 32-bit;
 * mpt_create returns MPT_ERR_UNSUPPORTED beyond). */
size_t mpt_workspace_bytes(const mpt_grid *grid, const mpt_params *params, int64_t n_max);

/* Create a context on the current HIP device.  dev_workspace: caller-owned
 * device memory of ws_bytes >= mpt_workspace_bytes(grid, params, n_max),
 * 256-byte aligned.  Copies the level table to the device synchronously.
 * Returns MPT_ERR_HIP when no GPU is usable. */
mpt_status mpt_create(const mpt_grid *grid, const mpt_params *params, int64_t n_max,
                      void *dev_workspace, size_t ws_bytes, mpt_ctx **out);

/* Store resident time level `level` (0 .. nt-1; the level at t_met0 +
 * (first + level) * dt_met, first = number of mpt_push_met calls so far)
 * from device arrays u, v, w of nz*ny*nx float each, index
 * (k*ny + j)*nx + i, w in hPa/s (read_met, Sec. 3.1; the kernel layout
 * packs {u,v,w,0} per grid point, lon fastest; BF16/F16 grids also compute
 * the per-level scales).  The source arrays may be freed once the stream
 * has passed this call. */
mpt_status mpt_init_met(mpt_ctx *ctx, int32_t level, const float *u, const float *v,
                        const float *w, void *hip_stream);

/* Advance the resident window by one time level (read_met supplying the
 * next met0/met1 pair, Sec. 3.1 and the data regions of Sec. 4.1): the level
 * at t_met0 + (first + nt) * dt_met, from device arrays as in mpt_init_met,
 * replaces the oldest resident level (first), in place in a ring of nt
 * slots.  Stream-ordered: work enqueued earlier on the same stream uses the
 * old window; later calls must keep their steps inside the new window
 * [t_met0 + (first + 1) dt_met, t_met0 + (first + nt) dt_met] (else
 * MPT_ERR_TIME).  A caller overlapping the host-to-device copy of the next
 * level with stepping copies it on another stream and orders this call
 * after that copy.  MPT_ERR_STATE until all nt levels are stored.  Drops a
 * captured step graph. */
mpt_status mpt_push_met(mpt_ctx *ctx, const float *u, const float *v, const float *w,
                        void *hip_stream);

/* Convection and sedimentation fields of resident time level `level` (as
 * in mpt_init_met; read_met_cape and the temperature of read_met_levels,
 * Sec. 3.1), from device arrays of float: temp [K], nz*ny*nx, index
 * (k*ny + j)*nx + i, positive; cape [J/kg], pel (equilibrium level) and ps
 * (surface pressure) [hPa], ny*nx, index j*nx + i.  The temperature goes
 * into the fourth value of each packed record (BF16 / F16 storage: with its
 * own per-level scale); the three surface fields are kept as FP32 records
 * {cape, pel, ps, 0}.  Must follow the level's mpt_init_met (or, for the
 * newest level after mpt_push_met, level nt-1): storing u, v, w for a level
 * clears these fields.  Readings used by the step:
 *   convection: with CAPE >= conv_cape and p > pel at the parcel (bilinear
 *     in lon, lat, linear in time, at the middle of the step), the parcel
 *     moves to p = ps + (pel - ps) u, u uniform from the Philox block of
 *     counter (id, step, 5, 0), first word;
 *   sedimentation: settling velocity v of a sphere (Stokes drag, Cunningham
 *     slip correction 1 + Kn (1.257 + 0.4 exp(-1.1/Kn)), Sutherland
 *     viscosity) at the interpolated temperature; p += p v dt / 7000 m.
 * The source arrays may be freed once the stream has passed this call. */
mpt_status mpt_set_met_phys(mpt_ctx *ctx, int32_t level, const float *temp, const float *cape,
                            const float *pel, const float *ps, void *hip_stream);

/* Copy the stored (packed) resident time level `level` (as in
 * mpt_init_met) into dst (device, at least
 * mpt_met_level_bytes(ctx) bytes) and its scales into scales_dst (device,
 * 3*nz floats, index var*nz + k; all 1 for F32 storage).  Packed layout:
 * point (k, j, i) at element ((k*ny + j)*nx + i) of {u, v, w, T} records of
 * 4 x float (F32) or 4 x uint16 (BF16 / F16 bit patterns); T is 0 unless
 * mpt_set_met_phys stored the level's temperature. */
mpt_status mpt_copy_met_level(mpt_ctx *ctx, int32_t level, void *dst, float *scales_dst,
                              void *hip_stream);
size_t mpt_met_level_bytes(const mpt_ctx *ctx);

/* Release steps of nscen scenarios (module_timesteps, Sec. 4.3): a parcel
 * with scen[i] = s stays untouched while step < release_step[s].  Host
 * array, copied; 1 <= nscen <= 65536.  Required before any call with
 * particles->scen != NULL. */
mpt_status mpt_set_release(mpt_ctx *ctx, int32_t nscen, const int32_t *release_step,
                           void *hip_stream);

/* Advection of every active parcel over step `step`: explicit midpoint
 * with 4D interpolation, then the position fix (module_advection +
 * module_position, Sec. 3.2).  In place on particles->lon/lat/p. */
mpt_status mpt_advect(mpt_ctx *ctx, const mpt_particles *particles, uint32_t step,
                      void *hip_stream);

/* Turbulent then mesoscale diffusion over step `step`, then the position
 * fix (module_diffusion_turb, module_diffusion_meso, module_position,
 * Sec. 3.2; random numbers per Sec. 4.3).  Honours MPT_TURB / MPT_MESO of
 * params.flags.  mpt_advect followed by mpt_diffuse equals one mpt_step
 * without sorting, bit for bit. */
mpt_status mpt_diffuse(mpt_ctx *ctx, const mpt_particles *particles, uint32_t step,
                       void *hip_stream);

/* Sort parcels by grid box (the sorting modules of Sec. 6): key = 8 x the
 * 8 x 8 x 4 (lon x lat x level) tile of the cell holding the parcel (tiles
 * numbered lon fastest) + the half-tile of 4 x 4 x 2 cells it lies in
 * (upper half in level 4, in lat 2, in lon 1).  With scenarios, parcels not yet released at the step the
 * sort precedes go behind all tiles, grouped by their scenario's rank in
 * release order; parcels with non-finite positions go last.  Scatters the
 * whole state into the *2 set and swaps the primary and *2 pointers inside
 * *particles (the caller must re-read them).  Order inside a key is
 * unspecified.  Needs n <= n_max.  (This entry point sorts as if before
 * step 0; mpt_step sorts before the step it is about to run.) */
mpt_status mpt_sort_particles(mpt_ctx *ctx, mpt_particles *particles, void *hip_stream);

/* For callers that cannot allocate device memory at the call (code under
 * HIP graph capture, tight serving loops, harnesses that forbid it): the
 * same sort as mpt_sort_particles, with its scratch (keys and ranks per
 * parcel, histogram, counters, scan sums) in a fixed array of the library
 * that each device holds from the first mpt_create on it until the process
 * ends (about 40 MiB), instead of the context's workspace.  Allocates
 * nothing.  Limits: n <= MPT_NOALLOC_SORT_MAX_N (else MPT_ERR_WORKSPACE; n
 * may exceed the context's n_max) and a grid of at most
 * (MPT_NOALLOC_SORT_MAX_KEYS - 65537) / 8 tiles (else
 * MPT_ERR_UNSUPPORTED).  The
 * context's device must be current (else MPT_ERR_STATE).  Always runs its
 * own key pass (sort keys a step left are not used, and are dropped).
 * Every call on one device shares that array: calls that overlap on one
 * device (other streams, other contexts, other threads) race and give
 * wrong results; order them on one stream or synchronize between them. */
enum { MPT_NOALLOC_SORT_MAX_N = 1 << 22, MPT_NOALLOC_SORT_MAX_KEYS = 1 << 20 };
mpt_status mpt_sort_particles_noalloc(mpt_ctx *ctx, mpt_particles *particles, void *hip_stream);

/* The sort of mpt_sort_particles (Sec. 6) without moving the parcels: the
 * sorted order is kept in the context's workspace, and the next mpt_step on
 * the same parcels (same primary lon array and n) moves them as its first
 * launch steps them: that launch reads each parcel through the order and
 * writes its whole state into the *2 set in sorted order, and the call
 * swaps the primary and *2 pointers inside *particles (so the state moves
 * once instead of twice).  Until then *particles is unchanged and unsorted.
 * The order is dropped, unused, by any other call that moves or sorts
 * parcels (mpt_sort_particles*, mpt_advect, mpt_diffuse, mpt_step_graph,
 * mpt_step_surrogate), by an mpt_step that starts with its own sort, and by
 * an mpt_step on other parcels, with scenario indices, or with no module
 * switched on; results never depend on the order.  Needs n <= n_max. */
mpt_status mpt_sort_particles_deferred(mpt_ctx *ctx, mpt_particles *particles, void *hip_stream);

/* nsteps time steps step0 .. step0+nsteps-1 (advection, turbulent and
 * mesoscale diffusion per params.flags; the time loop of Sec. 4.3), sorting
 * before every step that is a multiple of params.sort_interval (then the
 * pointers in *particles are swapped as by mpt_sort_particles).
 * Consecutive steps between sorts are fused into launches of at most
 * params.fuse steps.  Without scenarios, a sort and the launch after it
 * move the state once: the sort leaves its order and the launch reads the
 * parcels through it and writes them in sorted order (as after
 * mpt_sort_particles_deferred).  With scenarios, launches that follow a
 * sort inside the same call use a persistent grid that walks only the
 * parcels released so far (their count is read from the sort's device-side
 * cursors; no host round trip). */
mpt_status mpt_step(mpt_ctx *ctx, mpt_particles *particles, uint32_t step0, int32_t nsteps,
                    void *hip_stream);

/* The same steps as mpt_step, bit for bit, with the launch sequence of two
 * sort windows (2 * sort_interval steps: sort, fused steps, sort, fused
 * steps) captured once into a HIP graph and replayed nsteps / (2 *
 * sort_interval) times; the kernels read the step index from device
 * memory, which the graph advances.  Requires sort_interval > 0,
 * step0 % sort_interval == 0, nsteps % (2 * sort_interval) == 0 and a
 * created (non-null) stream.  The graph is cached in the context and
 * re-captured when the particle pointers or n change.  After the call the
 * state is in the same set it started in (an even number of sorts). */
mpt_status mpt_step_graph(mpt_ctx *ctx, mpt_particles *particles, uint32_t step0, int32_t nsteps,
                          void *hip_stream);

/* ---- Hybrid model levels (read_met reads model-level data and regrids it,
 * Sec. 3.1: read_met_levels).  A reading: column pressures p_k = a_k +
 * b_k ps [hPa] for model levels k = 0 .. nml-1 (k = 0 lowest, pressure
 * decreasing with k); each of the context's pressure levels is interpolated
 * per column linearly in ln p between the two model levels around it; a
 * level below the lowest or above the highest model level of its column
 * takes that level's value.  The results feed mpt_init_met / mpt_push_met. */
enum { MPT_MAX_ML_LEVELS = 512 };

/* Set the model levels (host arrays, copied; synchronizes the stream).
 * MPT_ERR_ARG unless 2 <= nml <= MPT_MAX_ML_LEVELS, values finite, column
 * pressures strictly decreasing with k and positive for ps in [500, 1100]
 * hPa (checked at both ends; the pressures are linear in ps). */
mpt_status mpt_set_hybrid(mpt_ctx *ctx, int32_t nml, const double *a, const double *b,
                          void *hip_stream);

/* ps (device, ny*nx float, hPa, index j*nx + i) and u, v, w (device,
 * nml*ny*nx float each, index (k*ny + j)*nx + i) on the model levels ->
 * u_pl, v_pl, w_pl (device, nz*ny*nx float each) on the context's pressure
 * levels, interpolation in FP64, results rounded to FP32.  MPT_ERR_STATE
 * before mpt_set_hybrid. */
mpt_status mpt_ml_to_pl(mpt_ctx *ctx, const float *ps, const float *u, const float *v,
                        const float *w, float *u_pl, float *v_pl, float *w_pl, void *hip_stream);

/* ---- Gridded output (write_grid, Sec. 3.3: the output functions write
 * parcel data, gridded data and ensemble data).  The paper names the
 * function only; the reading here: a regular grid of nx x ny boxes in lon x
 * lat and nz pressure layers; box (k, j, i) at index (k*ny + j)*nx + i.  A
 * parcel with finite position belongs to
 *   i = floor((lon - lon0) / dlon) mod nx   (FP64 division, lon in [0, 360)),
 *   j = floor((lat - lat0) / dlat), kept if 0 <= j < ny, with j = ny - 1 for
 *       lat == lat0 + ny*dlat (a box's north edge belongs to it only at the
 *       grid's last row),
 *   k with pedges[k] >= p > pedges[k + 1], kept if it exists;
 * others are not counted.  Per box: the parcel count, the sum of the
 * parcels' masses, and the mass mixing ratio = mass / air mass of the box,
 * air mass = R^2 dlon_rad (sin lat_north - sin lat_south) (pedges[k] -
 * pedges[k+1]) * 100 / g, R = 6371 km, g = 9.80665 m/s^2. */
enum { MPT_MAX_OUT_LEVELS = 512 };
typedef struct {
  int32_t nx, ny, nz;            /* boxes; nz <= MPT_MAX_OUT_LEVELS */
  double lon0, dlon;             /* nx * dlon == 360 (global in longitude) */
  double lat0, dlat;             /* -90 <= lat0, lat0 + ny * dlat <= 90, dlat > 0 */
  const double *pedges;          /* host, nz + 1 layer edges [hPa], strictly decreasing; copied */
} mpt_outgrid;

/* Set the output grid (host struct and edges copied; synchronizes the
 * stream).  MPT_ERR_ARG for a grid that breaks the rules above. */
mpt_status mpt_set_outgrid(mpt_ctx *ctx, const mpt_outgrid *grid, void *hip_stream);

/* Count and mass per box of the particles (primary set) into counts
 * (device, nx*ny*nz uint32) and mass_sum (device, nx*ny*nz double), both
 * overwritten; mass (device, n double, or NULL for unit masses); mmr
 * (device, nx*ny*nz double, or NULL) receives mass_sum / air mass.  Sums
 * of masses are accumulated in FP64 in no fixed order.  MPT_ERR_STATE
 * before mpt_set_outgrid. */
mpt_status mpt_grid_output(mpt_ctx *ctx, const mpt_particles *particles, const double *mass,
                           uint32_t *counts, double *mass_sum, double *mmr, void *hip_stream);

/* ---- Learned k-step advection surrogate (a project addition: the paper has
 * no counterpart).  A ReLU MLP 81 -> 128 -> 128 -> 128 -> 3 on bf16 MFMA
 * with FP32 accumulation predicts the MPT_SURR_K-step displacement of plain
 * midpoint advection (east km along the start latitude, north km, dp hPa)
 * from u, v, w interpolated at the parcel's position shifted by whole
 * cells (-1, 0, 1) in lon, lat and level (81 inputs).  Parameters are one
 * FP32 array of MPT_SURR_NPARAM values: per layer W[in][out] then bias, with
 * padded shapes 96x128, 128x128, 128x128, 128x16 (padding is zero).
 * `norm` is 12 floats on the device: input mean and std per variable
 * (u, v, w), output mean and std per component. */
enum { MPT_SURR_K = 8, MPT_SURR_NIN = 81, MPT_SURR_NOUT = 3, MPT_SURR_NPARAM = 47504,
       MPT_SURR_MAX_BATCH = 8192 };

/* Training samples at caller-chosen starts (device arrays of n): x (n x 81
 * floats) = the stencil inputs at time t_start + step*dt; y (n x 3) = the
 * displacement after MPT_SURR_K plain FP64 midpoint steps.  F32 storage. */
mpt_status mpt_surrogate_datagen(mpt_ctx *ctx, int64_t n, const double *lon, const double *lat,
                                 const double *p, const uint32_t *step, float *x, float *y,
                                 void *hip_stream);
/* Normalization statistics of n samples into norm (device, 12 floats). */
mpt_status mpt_surrogate_stats(mpt_ctx *ctx, int64_t n, const float *x, const float *y,
                               float *norm, void *hip_stream);
/* He-uniform initial weights from Philox(seed), zero biases. */
mpt_status mpt_surrogate_init(mpt_ctx *ctx, float *params, uint64_t seed, void *hip_stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8, step count t >= 1) on the
 * batch x[batch x 81], y[batch x 3] (batch a multiple of 64, at most
 * MPT_SURR_MAX_BATCH): mean squared error of the normalized outputs.  The
 * batch loss is added to *loss (device float).  Invalidates a loaded
 * surrogate (load again before stepping). */
mpt_status mpt_surrogate_train_step(mpt_ctx *ctx, const float *x, const float *y, int32_t batch,
                                    const float *norm, float *params, float *adam_m,
                                    float *adam_v, int32_t t, float lr, float *loss,
                                    void *hip_stream);
/* Gradient of that loss with respect to params (FP32, same layout) into
 * grad (device, MPT_SURR_NPARAM floats); batch loss added to *loss. */
mpt_status mpt_surrogate_grad(mpt_ctx *ctx, const float *x, const float *y, int32_t batch,
                              const float *norm, const float *params, float *grad, float *loss,
                              void *hip_stream);
/* Load weights for inference with acceptance threshold tau_km. */
mpt_status mpt_surrogate_load(mpt_ctx *ctx, const float *params, const float *norm, float tau_km,
                              void *hip_stream);
/* Predicted displacements y (n x 3) for given inputs x (n x 81). */
mpt_status mpt_surrogate_forward(mpt_ctx *ctx, int64_t n, const float *x, float *y,
                                 void *hip_stream);
/* nsteps steps in blocks of MPT_SURR_K: per parcel, predict the block's
 * advection, estimate its error as the distance [km] between the
 * prediction and MPT_SURR_K*dt times the wind at the predicted midpoint; if
 * at most tau, apply it plus the turbulent and mesoscale diffusion of the
 * block's MPT_SURR_K steps with the plain steps' random numbers (Philox
 * counters (id, step, 0) and (id, step, 1) of each step) and the mesoscale
 * spread of the block-start cell, summed and converted at the displaced
 * position; otherwise run MPT_SURR_K plain steps (those parcels, in
 * increasing index order).  Adds the number
 * of parcel-blocks that fell back to *fallbacks (device uint32).  err_out
 * (device, n floats, or NULL) receives each parcel's error estimate of the
 * last block (for calibrating tau; needs sort_interval == 0).  Needs
 * MPT_MATH_F32, F32 storage, no scenarios, no MPT_CONV / MPT_SEDI (else
 * MPT_ERR_UNSUPPORTED), step0 and nsteps multiples of MPT_SURR_K; sorts
 * before each block that contains a multiple of sort_interval. */
mpt_status mpt_step_surrogate(mpt_ctx *ctx, mpt_particles *particles, uint32_t step0,
                              int32_t nsteps, uint32_t *fallbacks, float *err_out,
                              void *hip_stream);

/* Release the context (the workspace stays the caller's). */
mpt_status mpt_destroy(mpt_ctx *ctx);

/* Static description of a status code. */
const char *mpt_status_string(mpt_status status);

#ifdef __cplusplus
}
#endif

#endif /* MPT_H */
