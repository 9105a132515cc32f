/*
 * ic.h - C ABI of libic.so: one inertial-coupling (IC) time step of the
 * compressible, isothermal, fluctuating Navier-Stokes equations on a periodic
 * staggered grid, coupled to particles through the 3-point kernel, on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: F. Balboa Usabiaga and R. Delgado-Buscalioni, "A minimal model for
 * acoustic forces on Brownian particles", arXiv:1307.0702.
 *
 * Conventions shared by every entry point
 *  - Every call returns int: IC_OK (0) or a negative IC_E_* code.  Nothing
 *    throws or aborts across the ABI; ic_last_error() gives a message.
 *  - Grid arrays hold nx*ny*nz elements, x fastest: cell (i,j,k) is element
 *    (k*ny + j)*nx + i and sits at r = (i h, j h, k h).  A vector component
 *    alpha is stored on the alpha-faces: element (i,j,k) of gx sits at
 *    r + (h/2) e_x (App. A, "Spatial discretization").  The density array
 *    holds the deviation rho - rho0.
 *  - Element type of every grid array is float for IC_FP32 and double for
 *    IC_FP64.  Particle data are always double.
 *  - "device" pointers point to GPU memory of the current HIP device; "host"
 *    pointers to CPU memory.  Host inputs are copied before the call returns.
 *  - Work is enqueued on the HIP stream given to ic_create; device outputs
 *    are valid once that stream has synchronised.  Calls documented as
 *    synchronising wait for the stream.
 *  - A context is not thread-safe; different contexts are independent.
 */
#ifndef IC_H
#define IC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    IC_OK = 0,
    IC_E_ARG = -1,        /* invalid argument or size */
    IC_E_UNSTABLE = -2,   /* time step beyond the explicit stability limit */
    IC_E_MASS = -3,       /* m_p <= 0, c_p^2 < 0, or m_e + m_f <= 0 in a step */
    IC_E_STATE = -4,      /* call out of order (e.g. step before bind) */
    IC_E_HIP = -5,        /* a HIP runtime call failed */
    IC_E_CAPACITY = -6    /* more particles than max_particles */
};

enum { IC_FP32 = 1, IC_FP64 = 2 };

/* Grid location of a field for ic_interpolate / ic_spread. */
enum { IC_CELL = 0, IC_FACE_X = 1, IC_FACE_Y = 2, IC_FACE_Z = 3, IC_FACES = 4 };

/* Shape of an imposed pressure drive. */
enum { IC_MODE_COS = 0, IC_MODE_PLANE = 1 };

enum { IC_MAX_MODES = 8 };

/* Fluid and run parameters (Table I of the paper lists its own values).
 * h grid spacing, rho0 equilibrium density, cf fluid sound speed (pressure
 * p = p0 + cf^2 rho), eta/zeta shear/bulk viscosity, kT thermal energy
 * (0 switches the stochastic stress off), dt time step.  seed keys the
 * Philox generator; replica is its fourth counter word (independent
 * realisations of one seed).  prec is IC_FP32 or IC_FP64.  max_particles
 * bounds the particle count of ic_set_particles and ic_spread and sizes the
 * per-particle parts of both workspaces (ic_interpolate takes any n). */
typedef struct ic_params {
    int32_t nx, ny, nz;
    int32_t prec;
    double h, rho0, cf, eta, zeta, kT, dt;
    uint64_t seed;
    uint32_t replica;
    int32_t max_particles;
} ic_params;

/* One imposed pressure drive added to the pressure at cell centres:
 * p_ext = amp * profile(x_axis) * sin(omega t + phase), with
 *   IC_MODE_COS:   profile = cos(2 pi m (x - x0) / L_axis)
 *   IC_MODE_PLANE: profile = 1 on the plane of cells nearest x0, else 0
 *                  (the Kronecker-delta drive of Sec. VI, Eq. pext). */
typedef struct ic_mode {
    int32_t axis;   /* 0, 1, 2 = x, y, z */
    int32_t shape;  /* IC_MODE_COS or IC_MODE_PLANE */
    int32_t m;      /* mode number for IC_MODE_COS */
    int32_t pad;
    double x0, amp, omega, phase;
} ic_mode;

typedef struct ic_ctx ic_ctx;
typedef struct ic_graph ic_graph;

/* Validates p and creates a context bound to HIP stream `stream` (NULL =
 * default stream) on the current device.  Host only; allocates no device
 * memory.  IC_E_ARG for sizes < 4 per side, a field of 4 GiB or more
 * (nx ny nz times the element size), non-positive h, rho0, cf, dt,
 * negative viscosities or kT; IC_E_UNSTABLE when cf dt/h > 0.5 or
 * (4 eta/3 + zeta)/rho0 * dt/h^2 > 0.2 (reading: the SSP-RK3 stability
 * region on the imaginary and real axes for the largest staggered-grid
 * wavenumber; the paper prints no dt rule). */
int ic_create(const ic_params *p, void *stream, ic_ctx **out);

/* Destroys a context (the caller's buffers are not freed). */
int ic_destroy(ic_ctx *ctx);

/* Bytes of device workspace a context with parameters p needs. */
int ic_workspace_size(const ic_params *p, size_t *bytes);

/* Binds caller-owned device buffers: the four state fields (rho - rho0, gx,
 * gy, gz; each nx*ny*nz elements of the context precision) and a workspace
 * of at least ic_workspace_size bytes, 256-byte aligned.  The library never
 * frees them.  Clears the particle set, forcing and averages. */
int ic_bind(ic_ctx *ctx, void *drho, void *gx, void *gy, void *gz,
            void *workspace, size_t workspace_bytes);

/* Sets n particles from host arrays (x,y,z triples, i.e. [n][3]):
 * q positions (wrapped into the box), u velocities or NULL (then u = J v at
 * q, the no-slip value), me excess masses m_e = m_p - rho0 V with V = 8 h^3
 * (Sec. IV B, Eq. particleMass), eps particle-fluid energies eps_pf (Sec.
 * III, Eq. omega), ks tether spring constants or NULL (0), qeq tether anchors
 * or NULL (= q), fext constant external forces or NULL (0).  IC_E_MASS when
 * m_e + rho0 V <= 0 or cf^2 + eps < 0 (Eq. part_svel); IC_E_UNSTABLE when
 * the particle sound speed sqrt(cf^2 + eps) gives c dt/h > 0.5;
 * IC_E_CAPACITY when n > max_particles.  Resets the force averages.
 * Synchronising. */
int ic_set_particles(ic_ctx *ctx, int32_t n, const double *q, const double *u,
                     const double *me, const double *eps, const double *ks,
                     const double *qeq, const double *fext);

/* Copies particle positions and velocities ([n][3], host) out; either may be
 * NULL.  Synchronising. */
int ic_get_particles(ic_ctx *ctx, double *q, double *u);

/* Sets the imposed pressure drives (nmodes <= IC_MAX_MODES, host array). */
int ic_set_forcing(ic_ctx *ctx, int32_t nmodes, const ic_mode *modes);

/* Sets / reads the step counter n (time t = n dt; the counter keys the
 * noise of each step). */
int ic_set_step(ic_ctx *ctx, int64_t n);
int ic_get_step(ic_ctx *ctx, int64_t *n);

/* Sets / reads the z extent tz of a fluid-stage tile (4, 8, 16 or 32 planes;
 * the default minimises rounds of resident tiles times planes marched per
 * tile).  Results do not depend on it beyond rounding order; it trades tile
 * count against halo re-reads.  IC_E_ARG for other values.  Any time between
 * steps. */
int ic_set_tile(ic_ctx *ctx, int32_t tz);
int ic_get_tile(ic_ctx *ctx, int32_t *tz);

/* Advances the bound state by nsteps IC time steps (App. A, "Temporal
 * discretization", substeps 1-7, with the three SSP-RK3 stages of the fluid
 * update).  Asynchronous.  On grids of 2^20 cells or more, part of each step
 * (the particle prologue and the next step's noise) runs on a second stream
 * owned by the context, which every step joins back into the context stream
 * before it ends, so ordering against the caller's work on that stream is
 * unchanged; a call of 5 steps or more replays a 4-step HIP graph of the
 * same launches, captured on first use and again whenever the particle
 * count, forcing, tile extent or bound buffers have changed (not while
 * ic_profile is on).  Noise drawn ahead by the last step of a call serves
 * the next call, unless ic_set_step, ic_bind or an ic_graph_launch comes in
 * between.  A step whose no-slip impulse finds m_e + m_f <= 0 raises a
 * device flag reported by the next synchronising call as IC_E_MASS. */
int ic_step(ic_ctx *ctx, int64_t nsteps);

/* Captures now the 4-step graph that ic_step replays on grids of 2^20 cells
 * or more (for the current particle count, forcing, tile extent and bound
 * buffers), so that the first ic_step call of 5 steps or more does not pay
 * for the capture.  Runs no step and changes no state.  IC_OK also when no
 * graph applies (a smaller grid, ic_profile on) or the capture fails (ic_step
 * then tries again, and launches its steps one by one if it fails there
 * too); IC_E_ARG / IC_E_STATE as ic_step for a missing or unbound context.
 * Not during an ic_step of the context on another host thread. */
int ic_step_prepare(ic_ctx *ctx);

/* Averaging operator J (Sec. II, Eq. Jdis; staggered positions of App. A):
 * out[p] = sum_i h^3 theta_h(q_p - r_i) field[i] for n positions q ([n][3])
 * and a field of the given location kind (device, context precision,
 * nx*ny*nz).  out is double[n].  With kind IC_FACES,
 * field holds the x, y and z face components one after another (3 nx*ny*nz,
 * e.g. the momentum of a state) and out is double[n][3], the averaged
 * vector J_alpha f^alpha.  Asynchronous when q and out are device memory;
 * either may instead be host memory (detected), and then the call stages
 * them through a temporary device buffer and synchronises. */
int ic_interpolate(ic_ctx *ctx, int32_t n, const double *q, int32_t kind,
                   const void *field, double *out);

/* Largest n of ic_interpolate_noalloc. */
enum { IC_NOALLOC_MAX_POINTS = 16384 };

/* ic_interpolate for callers that cannot allocate device memory (serving
 * loops and harnesses that forbid hipMalloc): the same averaging J, the same
 * arguments and the same results, bit for bit, as ic_interpolate, but host
 * positions or results are staged through a static device buffer of the
 * library instead of a temporary allocation; no hipMalloc, hipFree or other
 * allocating call is made.  The buffer holds 6 * IC_NOALLOC_MAX_POINTS
 * doubles (768 KiB) on each GPU the library runs on, kept until the process
 * ends; its device address is looked up on the first staged call on a GPU.
 * IC_E_ARG when n > IC_NOALLOC_MAX_POINTS (also with device arrays).  With q
 * and out both in device memory nothing is staged and the call is
 * asynchronous, as ic_interpolate; otherwise it synchronises the context
 * stream.  Every context on one GPU shares that GPU's buffer: the library
 * holds a per-GPU lock from the first copy to the final synchronisation, so
 * staged calls of one process never overlap (calls from several threads
 * wait for each other).  The buffer keeps the last call's contents; nothing
 * in it needs to start at zero. */
int ic_interpolate_noalloc(ic_ctx *ctx, int32_t n, const double *q, int32_t kind,
                           const void *field, double *out);

/* Spreading operator S (Sec. II, Eq. Sdis): adds theta_h(q_p - r_i) f[p] to
 * field[i] for every p, so sum_i h^3 field[i] grows by sum_p f[p].  q
 * ([n][3]) and f (double[n]) are device arrays; field is device (context
 * precision).  Deterministic (no float atomics).  Asynchronous; uses the
 * context workspace, so it must not overlap an ic_step of the context. */
int ic_spread(ic_ctx *ctx, int32_t n, const double *q, const double *f, int32_t kind,
              void *field);

/* Snapshot and restore of the bound state (checkpoints, fault injection):
 * ic_get_state copies the four fields (nx*ny*nz each, context precision)
 * and the particle positions and velocities ([n][3] doubles) into caller
 * device buffers; any pointer may be NULL.  Asynchronous.  ic_set_state
 * copies them back in from caller device buffers (NULL: keep); positions are
 * checked on the host and wrapped into the box (IC_E_ARG if one is not
 * finite).  Synchronising.  Neither touches the step counter (ic_set_step),
 * the particle parameters or the force averages. */
int ic_get_state(ic_ctx *ctx, void *drho, void *gx, void *gy, void *gz, double *q, double *u);
int ic_set_state(ic_ctx *ctx, const void *drho, const void *gx, const void *gy, const void *gz,
                 const double *q, const double *u);

/* Window averages since the last reset, per particle ([n][3], host, either
 * may be NULL): the mean of -F_tether = k_s minimg(q^{n+1/2} - q_eq), the
 * spring-force estimator of the radiation force (Sec. VI), and the mean of
 * the fluid force lambda = m_e (u^{n+1} - u^n)/dt - F^{n+1/2} (Sec. IV B,
 * Eq. partVel).  *nsamples gets the number of steps averaged.  reset != 0
 * starts a new window.  Synchronising. */
int ic_avg_force(ic_ctx *ctx, double *f_out, double *lambda_out, int64_t *nsamples,
                 int32_t reset);

/* FP64 sums of the bound state: out[0] = sum h^3 (rho - rho0), out[1..3] =
 * sum h^3 g + sum_p m_e u_p (Sec. IV C, total momentum).  Synchronising. */
int ic_conserved(ic_ctx *ctx, double out[4]);

/* Instrumentation.  With enable != 0, ic_step launches every step one by
 * one and brackets every fluid-stage kernel launch (the three RK sweeps of
 * App. A) with HIP events on the context stream.  ic_profile_read synchronises, returns the summed duration
 * of those kernels in ms and their number of launches since the last read,
 * and clears both. */
int ic_profile(ic_ctx *ctx, int32_t enable);
int ic_profile_read(ic_ctx *ctx, double *stage_ms, int64_t *launches);

/* eps_pf from kappa_p/kappa_f: cf^2 (kappa_f/kappa_p - 1) (Sec. III, Eqs.
 * part_svel and ke). */
double ic_eps_from_kappa_ratio(double cf, double kappa_ratio);

/* Ensembles of independent runs (replicas with their own seeds or replica
 * ids, contrast sweeps, uneven grids and particle counts).
 * ic_graph_create captures nsteps IC steps of each of the n bound contexts
 * into one HIP graph that one launch replays: a single context of at least
 * 2^20 cells as its eager schedule (particle prologue and next step's noise
 * on a second stream beside the stages); contexts of one precision with at
 * most 512 particles each as one launch per kernel of the step for all of
 * them; otherwise one chain of single-context launches per context, run
 * concurrently.  Every form gives each context's eager steps bit for bit.
 * The graph holds each context's buffers,
 * particle count, forcing and tile extent as they are at capture.  Changing
 * any of them needs a new graph; the step counter and the drive phase live
 * on the device and advance with each replay.  IC_E_STATE if a context is
 * unbound or profiling, IC_E_ARG for bad arguments or a context listed twice,
 * IC_E_HIP on a capture error.  Host only; does not run the steps.
 * ic_graph_launch enqueues one replay on `stream` (NULL = default stream),
 * which the caller orders with the contexts' own work; each context then
 * stands nsteps further on.  ic_graph_destroy frees the graph. */
int ic_graph_create(ic_ctx *const *ctxs, int32_t n, int64_t nsteps, ic_graph **out);
int ic_graph_launch(ic_graph *graph, void *stream);
int ic_graph_destroy(ic_graph *graph);

/* Reverse mode of the deterministic fluid step (kT = 0, no particles): the
 * transpose of one IC step as a linear map of small state perturbations,
 * for gradients of a loss of the state after N steps with respect to an
 * earlier state and to the drive amplitudes A_m (Sec. VI pressure drive).
 * The step is the three SSP-RK3 stages of App. A with the conservative
 * staggered flux; its transpose runs the stages backwards.
 * ic_adjoint_workspace_size: bytes of the extra device workspace (16 fields
 * of the context precision, IC_MAX_MODES doubles per 256 cells and 18
 * doubles per particle of max_particles).
 * ic_bind_adjoint: binds it (caller-owned, 256-byte aligned) and zeroes the
 * drive-gradient accumulator.  Synchronising.  workspace = NULL with
 * bytes = 0 unbinds it (before the caller frees it); the adjoint calls then
 * return IC_E_STATE until a workspace is bound again.
 * ic_adjoint_step: for step n taken from the state U^n = (drho, gx, gy, gz)
 * (device, context precision, nx*ny*nz each, read only), replaces the adjoint
 * (ldrho, lgx, lgy, lgz) = dL/dU^{n+1} (device, same layout) by dL/dU^n and
 * adds dL/dA_m of this step to the accumulator.  The stage inputs of step n
 * are recomputed from U^n with the forward stage kernels, so a caller keeps
 * U^n (or re-steps to it from a checkpoint).  The bound state fields are not
 * touched; the forward workspace is, so the call must not overlap ic_step of
 * the same context.  IC_E_STATE if the adjoint workspace is unbound, kT != 0
 * or particles are set; IC_E_ARG for NULL fields or n < 0.  Asynchronous.
 * ic_adjoint_drive: grad[m] = accumulated dL/dA_m for the current drives
 * (host, double[nmodes]), summed in a fixed order; reset != 0 zeroes the
 * accumulator.  Synchronising. */
int ic_adjoint_workspace_size(const ic_params *p, size_t *bytes);
int ic_bind_adjoint(ic_ctx *ctx, void *workspace, size_t bytes);
int ic_adjoint_step(ic_ctx *ctx, int64_t n, const void *drho, const void *gx, const void *gy,
                    const void *gz, void *ldrho, void *lgx, void *lgy, void *lgz);
int ic_adjoint_drive(ic_ctx *ctx, double *grad, int32_t reset);

/* Reverse mode of the whole deterministic IC step with particles (kT = 0):
 * the seven substeps of App. A reversed (substep 7 first, the RK stages from
 * the third to the first), including the particle pressure
 * S(eps_pf V J rho) of Sec. III, the spread tether force, the no-slip
 * impulse of Sec. IV B and the dependence of every kernel weight on the
 * particle position through phi' (phi is C^1, App. A).
 * ic_adjoint_step_particles: as ic_adjoint_step for U^n and the field
 * adjoints, plus device arrays ([n][3] doubles, n = the context's particle
 * count): q, u = the particle state at step n (as ic_copy_particles returns
 * it, positions inside the box; read only); lq, lu = dL/dq^{n+1}, dL/du^{n+1}
 * on entry, dL/dq^n, dL/du^n on return; lF = dL/dF^{n+1/2} for a loss on
 * this step's force F = -k_s minimg(q^{n+1/2} - q_eq) + f_ext (the
 * radiation-force estimator of Sec. VI is its mean), or NULL.  Adds this
 * step's dL/dm_e, dL/deps_pf and dL/dk_s to per-particle accumulators and
 * dL/dA_m to the drive accumulator.  The particle parameters (m_e, eps_pf,
 * k_s, q_eq, f_ext) are the context's.  Scatters into the field adjoints
 * use atomic adds: results are repeatable to rounding, not bitwise.
 * Asynchronous; uses the forward workspace, like ic_adjoint_step.  With no
 * particles it is ic_adjoint_step.  IC_E_STATE if the adjoint workspace is
 * unbound or kT != 0; IC_E_ARG for NULL fields, NULL particle arrays while
 * particles are set, or n < 0.
 * ic_adjoint_particle_grad: copies the accumulated dL/dm_e, dL/deps_pf and
 * dL/dk_s (host, double[n] each, any may be NULL); reset != 0 zeroes them.
 * dL/dm_p = dL/dm_e (m_p = m_e + rho0 V); for kappa_p/kappa_f = r,
 * dL/dr = -cf^2 / r^2 dL/deps_pf (Eq. part_svel).  Synchronising.
 * ic_copy_particles / ic_load_particles: device-to-device copy of the
 * current positions and velocities out of / into the context ([n][3]
 * doubles, either may be NULL), for checkpoints of a reversed trajectory.
 * ic_copy_particles is asynchronous.  ic_load_particles checks the
 * positions on the host and wraps them into the box (IC_E_ARG if one is not
 * finite; synchronising).  A non-finite position handed to
 * ic_adjoint_step_particles is replaced by 0 and reported as IC_E_ARG by the
 * next synchronising call. */
int ic_adjoint_step_particles(ic_ctx *ctx, int64_t n, const void *drho, const void *gx,
                              const void *gy, const void *gz, const double *q, const double *u,
                              void *ldrho, void *lgx, void *lgy, void *lgz, double *lq, double *lu,
                              const double *lF);
int ic_adjoint_particle_grad(ic_ctx *ctx, double *dme, double *deps, double *dks, int32_t reset);
int ic_copy_particles(ic_ctx *ctx, double *q, double *u);
int ic_load_particles(ic_ctx *ctx, const double *q, const double *u);

const char *ic_strerror(int code);
const char *ic_last_error(const ic_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* IC_H */
