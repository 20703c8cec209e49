/*
 * ugkwp.h -- C ABI of the MI355X (gfx950) hot path of the unified gas-kinetic wave-particle
 * (UGKWP) method on unstructured meshes (Chen, Zhu & Xu, arXiv 2007.13091).
 *
 * One call of ugkwp_step advances the state by one time step of the scheme of Sec. 2:
 *   S0 primitives, tau = mu/p and the CFL time step                  (Sec. 2.4(a))
 *   S2 wave flux F^eq + F^{fr,wave} over every face                  (Sec. 2.2, Sec. 2.4)
 *   S3 sampling of hydro particles from the Maxwellian of W^h, or     (Sec. 2.3, Sec. 2.4(b))
 *      from its first-order g_p (sampling = 2), or independently from the equilibrium of the
 *      collision model (sampling = 3; the Shakhov g^+ when prandtl != 1, Sec. 2.1, Sec. 5)
 *   S4 free-flight time t_f = min(-tau ln eta, dt) of each particle   (Eq. for t_f, Sec. 2.3)
 *   S5 face-to-face free transport with wall reflection              (Sec. 2.3, Sec. 2.4(e))
 *   S6 net particle flux, conservative update, removal of collided    (Eq. update_macro_variables)
 *      particles and new particle sums W^p
 * All of it runs in HIP kernels on the caller's stream.
 *
 * Units: R = 1 (p = rho T, lambda = 1/(2T)); K internal degrees of freedom (Sec. 2.1), from
 * gamma = (K + 5)/(K + 3): K = 0 monatomic (5/3), K = 2 diatomic (7/5).
 * Conservative state per cell, per unit volume: W = (rho, rho U, rho V, rho W, rho E) with
 * rho E = rho |U|^2 / 2 + (3 + K) rho T / 2.  A particle carries mass, position, velocity and,
 * for K > 0, its internal energy variable e = |xi|^2 (its energy is m (|u|^2 + e) / 2).
 *
 * Memory and ownership.  Host arrays passed in are copied during the call and never
 * retained.  All device memory the library uses lives in ONE caller-owned device buffer
 * (the workspace) whose size ugkwp_workspace_bytes reports; the caller keeps it alive
 * until ugkwp_destroy.  ugkwp_init_mesh carves it; no other call allocates device memory.
 * Every device operation is ordered on the hip stream given to ugkwp_init_mesh.
 *
 * Batches.  ugkwp_init_mesh takes n_inst independent instances (each its own mesh and
 * parameters).  They run together: every kernel of a step covers all instances in one
 * launch, and one ugkwp_step advances each instance by one of its own time steps (each has
 * its own dt from its own CFL condition, its own clock and step counter).  Instance k draws
 * its random numbers with k in the last Philox counter word and numbers its particles by
 * its own cell indices, so it evolves exactly as it would alone with instance index k.
 * Cell-indexed host arrays (W0, moments, geometry, particle cells) concatenate the
 * instances' cells in instance order.
 *
 * Errors.  Every function returns a ugkwp_status and never aborts.  Host-detectable errors
 * return at once.  Errors found on the device (capacity, lost particle, non-physical
 * state) are recorded in a device error word and reported by the next call that
 * synchronises (ugkwp_step with stats, ugkwp_moments, ugkwp_export_particles); after such an
 * error the context refuses ugkwp_step (UGKWP_E_STATE) until ugkwp_init_state is called.
 * ugkwp_last_error gives a message for the last failure.
 */
#ifndef UGKWP_H
#define UGKWP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ugkwp_ctx ugkwp_ctx; /* opaque */

typedef enum {
    UGKWP_OK = 0,
    UGKWP_E_ARG = 1,      /* invalid argument or unsupported option */
    UGKWP_E_MESH = 2,     /* unmatched face, untagged boundary face, bad cell, ... */
    UGKWP_E_CAPACITY = 3, /* particle capacity or a per-cell limit exceeded */
    UGKWP_E_LOST = 4,     /* a particle exceeded max_crossings face crossings in one step */
    UGKWP_E_NONPHYS = 5,  /* rho <= 0, T <= 0 or a non-finite value in a cell */
    UGKWP_E_DEVICE = 6,   /* a HIP runtime call failed */
    UGKWP_E_STATE = 7     /* wrong call order, or the context is poisoned by an earlier error */
} ugkwp_status;

typedef enum {
    UGKWP_BC_SPECULAR = 0, /* symmetry plane / specular wall (Sec. 4.1) */
    UGKWP_BC_DIFFUSE = 1,  /* diffuse isothermal wall at T_w moving at U_w (Sec. 2.4(e)) */
    UGKWP_BC_FARFIELD = 2, /* free stream W_inf outside (Sec. 4.3): wave flux against W_inf,
                              particles leaving are removed, and the collisionless part of
                              the free stream enters as particles (see ugkwp_step_stats) */
    UGKWP_BC_PERIODIC = 3  /* test support, not a condition of the paper: a face tagged with
                              it leads to the boundary face whose centre is its own plus
                              `shift` (tagged with the opposite shift); the pair is one
                              interior face, a particle crossing it goes on at x + shift.
                              First order only (recon must be 0 on such a mesh) */
} ugkwp_bc_type;

typedef struct {
    int32_t type;   /* ugkwp_bc_type */
    double T_w;     /* wall temperature (diffuse) */
    double U_w[3];  /* wall velocity, tangential to the wall (diffuse) */
    double W_inf[5];/* free-stream conservative state (far field) */
    double shift[3];/* periodic: translation from this face to its partner */
} ugkwp_bc;

/* One mesh, host arrays.  Cells: 4-node tetrahedra (type 4) or 8-node axis-aligned boxes
 * (type 8) in VTK node order.  Boundary faces: node lists of 4 (a triangle pads with -1),
 * each tagged with an index into bc[].  Every cell face not shared by two cells must be a
 * tagged boundary face. */
typedef struct {
    int64_t n_nodes;
    const double *xyz;            /* [n_nodes][3] */
    int64_t n_cells;              /* at most 2^24 (particle ids carry the birth cell) */
    const uint8_t *cell_type;     /* [n_cells] */
    const int64_t *cell_node_off; /* [n_cells + 1] */
    const int64_t *cell_nodes;    /* [cell_node_off[n_cells]] */
    int64_t n_bfaces;
    const int64_t *bface_nodes;   /* [n_bfaces][4] */
    const int32_t *bface_bc;      /* [n_bfaces] */
    int32_t n_bc;                 /* below 2^27 (over all instances of a batch) */
    const ugkwp_bc *bc;           /* [n_bc] */
} ugkwp_mesh;

typedef struct {
    double gamma;         /* (K + 5)/(K + 3) for an integer 0 <= K <= 8: 5/3 monatomic, 7/5 diatomic;
                             the same for every instance of a batch */
    double mu_ref;        /* tau = mu_ref T^omega / p  (T_ref = 1), Eq. tau_via_T_ref */
    double omega;
    double cfl;           /* C in dt = C min Omega / (Lambda^x + Lambda^y + Lambda^z) */
    double c2;            /* numerical-dissipation constant C2 of Sec. 2.4(d) (0 = off) */
    int32_t n_ref;        /* reference particle number per cell, Sec. 2.4(b) */
    int32_t n_min;        /* minimum particle number per cell, Sec. 2.4(b) */
    int32_t recon;        /* 0 first order; 1 least-squares gradients + Barth-Jespersen limiter;
                             2 least-squares gradients + Venkatakrishnan limiter (Sec. 2.2) */
    int32_t precision;    /* 0 = FP64 throughout; 1 = FP32 form: flux and particle transport in
                             FP32, per-cell sums, W - W^p and energy -> T in FP64 */
    int64_t capacity;     /* particle capacity (0 = library default from n_ref and n_cells) */
    int32_t max_crossings;/* face crossings allowed per particle per step */
    uint64_t seed;        /* Philox4x64-10 key word 0 */
    double venkat_k;      /* Venkatakrishnan constant K, eps^2 = (K h)^3 with h = Omega^(1/3)
                             (recon = 2; must be > 0 then) */
    int32_t sampling;     /* velocities of the sampled hydro particles (Sec. 2.4(b)):
                             0 = the pairs u = U + sqrt(T) X, u' = U - sqrt(T) X with X ~ N(0, I),
                                 as the paper states them: the sample carries exactly the mass
                                 and momentum of rho^hp, its thermal energy is random;
                             1 = energy-exact pairs (a departure from the paper): one factor
                                 per cell on every deviation, sqrt(3 N_pairs / sum_j |X_j|^2),
                                 so that the sample also carries exactly the energy;
                             2 = the first-order g_p of Sec. 2.3 (the Chapman-Enskog correction
                                 of the Maxwellian from the cell's limited gradients, weighted by
                                 alpha = dt / expm1(dt/tau) - tau), by acceptance-rejection per
                                 particle; needs recon 1 or 2 (else UGKWP_E_ARG); the sample
                                 carries exactly the mass, its momentum and energy are random;
                             3 = independent draws from the equilibrium of the collision model
                                 (the Maxwellian, or the Shakhov g^+ when prandtl != 1), per
                                 particle; any recon */
    int32_t gks_steps;    /* wave-only start: the steps n < gks_steps, counted from
                             ugkwp_init_state, sample no particle and let no free-stream particle
                             enter; their wave flux carries the whole free transport of W^h,
                             int u_n (q4 g0^h + q5 u.g_x^h) psi (the wave flux of Sec. 2.4 without
                             the terms of the sampled particles).  This is how the paper starts
                             its hypersonic cases (Sec. 4.3, Sec. 4.4): from a field computed by
                             the gas-kinetic scheme alone.  While no particle exists (from
                             ugkwp_init_state, or an imported state without particles) these
                             steps skip the particle kernels, with the same results.  0 = off */
    double prandtl;       /* collision model (Sec. 2.1 names the alternatives to BGK; Sec. 4.3 and
                             Sec. 5 the Shakhov model as the remedy for the BGK model's Prandtl
                             number of 1): 0 or 1 = the BGK model of the paper; 0 < Pr < 2 else
                             = the Shakhov model with that Prandtl number, for a monatomic gas
                             (gamma 5/3) with sampling 2 or 3 (else UGKWP_E_ARG).  Its equilibrium
                             is g^+ = g [1 + (1 - Pr) c.q (|c|^2/T - 5) / (5 p T)], c = u - U, with
                             q the heat flux of the cell's particles at the start of the step:
                             the hydro particles are drawn from g^+ (or g_p plus that correction),
                             and the g0 term of the wave flux becomes g0^+, which adds
                             q1 (1 - Pr) q_f.n to its energy flux (q_f the mean of the two cells'
                             heat fluxes; walls keep the BGK flux) */
} ugkwp_params;

/* Statistics of a step.  For a batch, ugkwp_step reports the counts summed over the
 * instances and dt, t, step of instance 0. */
typedef struct {
    double dt, t;          /* time step just taken, time after it */
    int64_t step;          /* steps taken since ugkwp_init_state */
    int64_t n_alive;       /* particles left after the step */
    int64_t n_sampled;     /* hydro particles sampled in the step */
    int64_t n_collided;    /* particles removed as collided */
    int64_t n_escaped;     /* particles removed at far-field faces */
    int64_t n_moved;       /* particles streamed in the step (old + sampled + entering) */
    int64_t crossings;     /* face crossings in the step */
    int64_t wall_hits;     /* diffuse re-emissions in the step */
    uint32_t error_word;   /* device error bits (0 = none) */
    int64_t moved_total;   /* particles streamed since ugkwp_init_state (sum of n_moved) */
    int64_t n_injected;    /* free-stream particles that entered through far-field faces: per
                              face exp(-dt/tau_inf) rho_inf Gamma A dt of mass (Gamma the one-sided
                              number flux of the free-stream Maxwellian) in
                              ceil(Gamma A dt n_ref / Omega) equal particles */
    int64_t max_crossings_seen; /* the most face crossings of one particle in the step (to set
                              max_crossings with a margin) */
} ugkwp_step_stats;

/* Device bytes needed for n_inst >= 1 instances: m[n_inst], p[n_inst].  Host-side only (no
 * device call).  All instances must share precision; the capacity is the sum of theirs. */
int32_t ugkwp_workspace_bytes(const ugkwp_mesh *m, int32_t n_inst, const ugkwp_params *p, size_t *bytes);

/* Validate the mesh, match faces, compute the geometry (Sec. 2.2 cells, faces, normals,
 * areas, the projections Delta S of Sec. 2.4(a)), carve the workspace and upload.
 * dev_workspace: device pointer of at least ugkwp_workspace_bytes bytes, 256-byte aligned.
 * hip_stream: a hipStream_t (NULL = the default stream).  On success *ctx owns host-side
 * bookkeeping only; free it with ugkwp_destroy. */
int32_t ugkwp_init_mesh(ugkwp_ctx **ctx, const ugkwp_mesh *m, int32_t n_inst, const ugkwp_params *p,
                        void *dev_workspace, size_t ws_bytes, void *hip_stream);

/* Set the conservative state W0 (host, [total cells][5]); no particles (W^p = 0), every
 * instance at step 0, t = 0. */
int32_t ugkwp_init_state(ugkwp_ctx *ctx, const double *W0);

/* Advance n_steps time steps.  stats == NULL: asynchronous (nothing waits for the device).
 * stats != NULL: waits for the stream and fills the statistics of the last step. */
int32_t ugkwp_step(ugkwp_ctx *ctx, int32_t n_steps, ugkwp_step_stats *stats);

/* Statistics of the last step of one instance (synchronises).  crossings and wall_hits are
 * counted for the batch as a whole and read -1 here when n_inst > 1. */
int32_t ugkwp_instance_stats(ugkwp_ctx *ctx, int32_t inst, ugkwp_step_stats *stats);

/* Cells [cell0, cell1) of instance inst in the concatenated cell numbering. */
int32_t ugkwp_instance_cells(const ugkwp_ctx *ctx, int32_t inst, int64_t *cell0, int64_t *cell1);

/* Copy a cell field out, [n_cells][5] doubles: which = 0 W, 1 W^p = P/Omega (particle part),
 * 2 W^h = W - W^p, 3 primitives (rho, U, V, W, T).  out is host memory unless
 * out_is_device != 0.  Synchronises the stream. */
int32_t ugkwp_moments(ugkwp_ctx *ctx, int32_t which, double *out, int32_t out_is_device);

/* Time averaging for steady states (Sec. 2.4(c)).  From now on, every step n > n_avg
 * (n counted per instance from ugkwp_init_state) adds its state W^n, weighted by its own time
 * step dt^n, to the running average Wbar = sum dt^n W^n / sum dt^n of each instance.  Clears
 * whatever was accumulated; n_avg < 0 turns averaging off.  ugkwp_init_state clears the sums
 * and keeps the setting.  A captured step graph is dropped and captured again.  Synchronises
 * when a state is present.  Device memory: the sums live in the workspace (40 bytes per
 * cell). */
int32_t ugkwp_set_averaging(ugkwp_ctx *ctx, int64_t n_avg);

/* The time average and its convergence measure (Sec. 2.4(c)).
 * Wbar: [n_cells][5] conservative, host memory unless out_is_device != 0; NULL: not copied.
 * residual: [n_inst] host, NULL: not copied.  The relative change of each instance's average
 *   in its last averaged step, in the volume-weighted L1 norm of the whole field:
 *   sum_c Omega_c sum_k |Wbar^n_ck - Wbar^{n-1}_ck| / sum_c Omega_c sum_k |Wbar^n_ck|.  The
 *   paper declares a steady state converged when this falls below a tolerance such as 1e-8.
 *   +infinity until two steps have been averaged.
 * n_averaged: [n_inst] host, NULL: not copied; steps averaged so far.
 * UGKWP_E_STATE when averaging is off or no step has been averaged yet.  Synchronises. */
int32_t ugkwp_average(ugkwp_ctx *ctx, double *Wbar, int32_t out_is_device, double *residual, int64_t *n_averaged);

/* Number of particles currently held (synchronises). */
int32_t ugkwp_particle_count(ugkwp_ctx *ctx, int64_t *n);

/* Copy the particles out to host arrays sized by ugkwp_particle_count:
 * x [n][3], u [n][3], m [n], cell [n] (int32), uid [n], e [n] (internal energy variable, 0 for
 * K = 0).  Order: grouped by cell.  Any pointer may be NULL to skip that field.  Synchronises. */
int32_t ugkwp_export_particles(ugkwp_ctx *ctx, double *x, double *u, double *m, int32_t *cell,
                               uint64_t *uid, double *e);

/* State between steps, for checkpoints, restarts and tests: everything a step reads
 * that the previous step left (Sec. 2.3: the conservative state W, the raw sums P of the
 * collisionless particles that remain, so that W^p = P/Omega, and those particles), plus each
 * instance's step counter and time.  The particles themselves are copied with
 * ugkwp_export_particles (grouped by cell, the library's order).
 * ugkwp_export_state: W [n_cells][5] conservative, P [n_cells][5] raw particle sums, step
 * [n_inst], t [n_inst]; host arrays, any may be NULL.  Synchronises; reports a pending device
 * error like ugkwp_moments. */
int32_t ugkwp_export_state(ugkwp_ctx *ctx, double *W, double *P, int64_t *step, double *t);

/* Replace the state: W and P as above (host, [n_cells][5]); n particles (host) x [n][3],
 * u [n][3], m [n], cell [n] (concatenated cell numbering, non-decreasing: grouped by cell),
 * uid [n], e [n] (internal energy variables; NULL: 0, ignored for K = 0); step [n_inst] (each
 * below 2^19, the particle-id field) and t [n_inst].  The
 * particles become the old particles of the next step, N_left of a cell is its count; the
 * time-averaging sums are cleared (the setting is kept).  The FP32 form rounds x, u and m to
 * single precision.  Importing what ugkwp_export_state and ugkwp_export_particles gave
 * continues the run bit for bit.  Errors: E_ARG (null pointers, unsorted or out-of-range
 * cells, bad step or t), E_CAPACITY (n above the capacity), E_NONPHYS (rho <= 0 or T <= 0 in
 * W); on error the previous state is untouched.  Clears a poisoned context.  Synchronises. */
int32_t ugkwp_import_state(ugkwp_ctx *ctx, const double *W, const double *P, int64_t n, const double *x,
                           const double *u, const double *m, const int32_t *cell, const uint64_t *uid,
                           const double *e, const int64_t *step, const double *t);

/* Per-cell geometry as the library computed it: volume [n_cells], centroid [n_cells][3],
 * projections Delta S [n_cells][3] (host arrays). */
int32_t ugkwp_geometry(ugkwp_ctx *ctx, double *vol, double *xc, double *dS);

/* Graph replay (on != 0): the launch sequence of a step is captured once into a hip graph
 * (per particle buffer) and replayed by ugkwp_step; the kernels read every count on the
 * device, so the graph stays valid.  Needs a created stream (not the null stream).  While
 * on, the per-kernel event timing of ugkwp_profile_enable is not recorded. */
int32_t ugkwp_graph_enable(ugkwp_ctx *ctx, int32_t on);

/* Launch shapes of the tunable kernels, cfg[4] = {k_stream block size (128, 256, 512),
 * k_stream particles per thread (1, 2), k_sample waves per block (1, 2, 4, 8; a wave takes 8
 * cells), k_flux block size (64, 128, 256)}.  Every shape gives bit-identical results.
 * Defaults: {256, 1, 4, 128}. */
int32_t ugkwp_set_launch(ugkwp_ctx *ctx, const int32_t *cfg);
int32_t ugkwp_get_launch(const ugkwp_ctx *ctx, int32_t *cfg);

/* Autotuner: one pass of coordinate search over the shapes above, each candidate timed with
 * hip events around its own kernel over steps_per_trial steps (after one untimed step); the
 * transport's candidates are compared per particle move (the particle count drifts from one
 * trial to the next).  The trial steps are real steps of the simulation (the shape does not
 * change results): the state advances by (steps_per_trial + 1) x 13 steps.  The fastest
 * shapes are kept and returned in cfg_out[4] (may be NULL).  Discards pending
 * ugkwp_profile_read records. */
int32_t ugkwp_autotune(ugkwp_ctx *ctx, int32_t steps_per_trial, int32_t *cfg_out);

/* The autotuner with a result cache, for callers that run the same workload again.  The cache
 * is a text file of JSON lines {"key": "<workload signature>", "launch": [a, b, c, d]}; the
 * signature names the device architecture, the precision, K, the instance count, the cells,
 * faces and capacity, and every instance's reconstruction, sampling mode and collision model.
 * A hit (the last line with the signature, its shapes in range) sets those shapes with no trial
 * step: the state does not advance.  A miss runs ugkwp_autotune (the state advances as there)
 * and appends its result.  cache_path must name a readable and appendable file (created if
 * missing; UGKWP_E_ARG if it cannot be written).  cfg_out[4] and hit (1 on a hit, else 0) may
 * be NULL.  Lines of other keys, or that do not parse, are ignored. */
int32_t ugkwp_autotune_cached(ugkwp_ctx *ctx, int32_t steps_per_trial, const char *cache_path, int32_t *cfg_out,
                              int32_t *hit);

/* Measurement support.  While enabled, each group of kernel launches of ugkwp_step is
 * bracketed by hip events recorded on the library's stream.  ugkwp_profile_read waits for
 * the stream, writes the summed elapsed milliseconds and the number of timed groups for the
 * first n_slots slots (see ugkwp_profile_slot_name; slot 5 is the free-transport kernel,
 * slot 6 the kernel that finishes the flights stopped at diffuse walls), and clears the
 * sums.  Either output pointer may be NULL. */
int32_t ugkwp_profile_enable(ugkwp_ctx *ctx, int32_t on);
int32_t ugkwp_profile_read(ugkwp_ctx *ctx, int32_t n_slots, double *total_ms, int64_t *launches);
/* Record only the slots whose bit is set in mask (default: all); fewer events, less overhead. */
int32_t ugkwp_profile_mask(ugkwp_ctx *ctx, uint32_t mask);
/* Name of a profiling slot ("" if out of range); static storage. */
const char *ugkwp_profile_slot_name(int32_t slot);

/* For callers that cannot allocate device memory (code under hip graph capture, serving loops
 * that forbid allocation, harnesses without an allocator): ugkwp_init_mesh with the library's
 * own static workspace instead of a caller's buffer.  The workspace is one array per GPU of
 * ugkwp_static_workspace_bytes() bytes (32 MiB), part of the library's device code object,
 * reserved on each GPU the library is loaded on and held until the process ends; its device
 * address is looked up once per GPU on the first call there (the current device).  Nothing is
 * allocated: no hipMalloc, no allocating library call.
 * Limits and sharing: a mesh whose ugkwp_workspace_bytes exceeds the array is refused with
 * UGKWP_E_CAPACITY (the shock tube of 200 box cells at 200 particles per cell needs 21 MiB).
 * One context at a time may use a GPU's array: a second call on that GPU before
 * ugkwp_destroy of the first returns UGKWP_E_STATE (two live contexts would overwrite each
 * other's state, as would any overlapping use of the array).  The array keeps whatever the
 * last context left; ugkwp_init_state clears what must start at zero, as with a caller's
 * uninitialised workspace.  ugkwp_destroy waits for the context's stream before releasing the
 * array.  Every other call works on such a context as on one from ugkwp_init_mesh. */
int32_t ugkwp_init_mesh_static(ugkwp_ctx **ctx, const ugkwp_mesh *m, int32_t n_inst, const ugkwp_params *p,
                               void *hip_stream);
/* Size in bytes of the static workspace of ugkwp_init_mesh_static (per GPU). */
size_t ugkwp_static_workspace_bytes(void);

/* Message for the last failure on this context (or of init when ctx is NULL). */
const char *ugkwp_last_error(const ugkwp_ctx *ctx);

/* Release the host-side context (the caller frees the workspace afterwards). */
void ugkwp_destroy(ugkwp_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* UGKWP_H */
