/*
 * lbmgls.h -- C ABI of the MI355X (gfx950) library for the coupled D2Q9
 * phase-field / flow lattice Boltzmann method of Zhan, Liu, Chai & Shi,
 * "A thermodynamically consistent and conservative diffuse-interface model
 * for gas-liquid-solid multiphase flows" (arXiv 2311.05097).
 *
 * The library advances, on one GPU, the two sets of D2Q9 distributions of
 * Sec. 3: g_i for the Cahn-Hilliard phase field (Sec. 3.1; chemical potential
 * of Eq. (potential) with the solid penalty and wetting terms) and f_i for the
 * consistent Navier-Stokes flow (Sec. 3.2; viscosity mu/(1-phi0) in the
 * solid), with the Hermite-moment MRT collision of Sec. 4 and the procedure
 * of Sec. 3.3 (steps 1-6, stationary solids u_s = 0).  Domains are periodic in
 * x unless bounce_x is set and in y unless bounce_y is set; other walls are
 * diffuse solids given through phi0.
 *
 * Conventions for every function:
 *   - return value: LBM_OK (0) or a negative LBM_E* code; nothing throws
 *     across the ABI; lbm_last_error() gives a message (thread-local).
 *   - host arrays are row-major [ny][nx] doubles, x fastest, caller-owned;
 *     they are copied (create) or filled (read) before the call returns.
 *   - device memory is never allocated by the library: the caller passes a
 *     device workspace of at least lbm_workspace_bytes() bytes (for example a
 *     torch uint8 tensor) and keeps it alive until lbm_destroy().  The opaque
 *     handles themselves are small host allocations.
 *   - work is enqueued on the HIP stream given at creation (NULL = the null
 *     stream).  Calls that return host data synchronise that stream.
 *   - a handle is used by one host thread at a time.
 */
#ifndef LBMGLS_H
#define LBMGLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,       /* bad argument (sizes, parameters, null pointers)    */
    LBM_ENOMEM = -2,       /* workspace too small                                 */
    LBM_EDEVICE = -3,      /* a HIP call failed                                   */
    LBM_ENONFINITE = -4,   /* a NaN/Inf appeared in phi, u or P                   */
    LBM_EUNSUPPORTED = -5, /* storage / tile option not built                     */
    LBM_ESTATE = -6        /* handle unusable (after ENONFINITE, or misuse)       */
};

/* Storage of the distributions.  Arithmetic is FP64 for LBM_STORE_FP64 and
 * FP32 otherwise.  The *DEV modes keep the eight moving phase-field
 * populations and all nine flow populations as scaled 16-bit values (their
 * deviation from the rest-state equilibrium, which is 0 for every moving g_i
 * and every f_i) and the rest population g_0 as a 64-bit fixed-point number
 * chosen so that sum_i g_i -- the order parameter -- is conserved exactly. */
enum {
    LBM_STORE_FP64 = 0,
    LBM_STORE_FP32 = 1,
    LBM_STORE_FP16DEV = 2,
    LBM_STORE_BF16DEV = 3
};

/* Tile shapes of the fused step kernel: 64 columns x TY rows (256 threads for
 * TY = 4, 512 otherwise; 64x32 is not built for FP64). */
enum { LBM_TILE_AUTO = 0, LBM_TILE_64x4 = 4, LBM_TILE_64x8 = 8, LBM_TILE_64x16 = 16, LBM_TILE_64x32 = 32 };

typedef struct {
    int32_t nx, ny;        /* lattice size (periodic unless walled); nx, ny >= 8;
                              nx * ny < 2^31, and <= 2^30 for FP32 and 16-bit
                              storage (planes addressed by 32-bit byte offsets) */
    int32_t storage;       /* LBM_STORE_*                                          */
    int32_t tile;          /* LBM_TILE_*                                           */
    double d0;             /* c_s^2 / c^2 in (0, 1); D2Q9 weights (Sec. 4)         */
    double sigma;          /* sigma_12 > 0 (Eq. 2energyDensity)                    */
    double D;              /* interface width > 0                                  */
    double M;              /* mobility > 0 (Eq. CHE)                               */
    double rho1, rho2;     /* densities of phase 1 (phi = +1) and 2, > 0 (Eq. rho) */
    double mu1, mu2;       /* dynamic viscosities, > 0                             */
    double tau_phi;        /* 1/s_{1phi} > 1/2; M = (tau_phi - 1/2) eta c_s^2      */
    double s0, s1, s2, s3, s4; /* other rates of S_H^1 = diag(s0,s1phi,s1phi,s2,s2,
                                  s2,s3,s3,s4) and S_H^2 = diag(s0,s1,s1,s2a,s2a,
                                  s2b,s3,s3,s4), each in (0, 2)                     */
    double gx, gy, rho_ref;/* body force (rho - rho_ref) g                         */
    double fbx, fby;       /* body force (1 - phi0) f_b                            */
    double solid_eps;      /* floor of 1 - phi0 in mu/(rho(1 - phi0)), in (0, 1)   */
    /* free rigid particles (Sec. 2.4; lbm_create_particles) */
    double rep_xi, rep_eps;/* Sec. 4.5 repulsion threshold xi and stiffness eps,
                              lattice units; eps <= 0: no repulsion             */
    double wall_x0, wall_x1, wall_y0, wall_y1; /* wall planes for the particle-
                              wall repulsion (mirror image of the particle)    */
    int32_t np;            /* number of free particles, 0..1024                  */
    int32_t walls;         /* bit 0: wall_y0, 1: wall_y1, 2: wall_x0, 3: wall_x1 */
    /* 1: no-flux walls half a node below row 0 and above row ny - 1 (the
       no-flux condition of the channel cases of Sec. 4.2 and 4.5): halfway
       bounce-back of g_i and f_i (no slip), ghost rows of the finite
       differences mirrored (phi, mu, rho, phi0, psi even: a neutral 90-degree
       wall; the mass flux S as their gradient; the velocity in F_c odd),
       particle distances in y without the periodic image.  0: periodic. */
    int32_t bounce_y;
    /* the same left of column 0 and right of column nx - 1 (the side walls of
       the sedimentation channel of Sec. 4.3); at a corner a population that would leave
       through either wall returns to its node. */
    int32_t bounce_x;
    /* H of the pressure recovery (Sec. 3.2, after Eq. u).  0: the factor that
       the first-order non-equilibrium moments of this model give,
       H = -K (1 - 3 d0) (1/s2a - 1/2) (default; with it a planar interface
       translating at a uniform speed keeps that speed to the interface's
       discretisation error).  1: the factor as printed,
       K [(1 - d0)/s0 - (2 - 4 d0)/s2a + (1 - 3 d0)/2]; the two differ by
       K^2 (1/s0 - 1/s2a) and agree when s0 = s2a. */
    int32_t h_form;
} lbm_params;

typedef struct lbm_domain lbm_domain;

/* Fill *p with the paper's defaults (Sec. 4.1: d0 = 0.4, sigma = 1e-3, D = 4,
 * M = 0.1, rho = mu-ratio 1, s_i = 1, tau_phi = 1, solid_eps = 0.01) for an
 * nx x ny grid. */
void lbm_default_params(lbm_params *p, int32_t nx, int32_t ny);

/* Device bytes a domain with these parameters needs (0 if p is invalid). */
size_t lbm_workspace_bytes(const lbm_params *p);

/* Procedure step 1 (Sec. 3.3): build the static solid fields from phi0 (the
 * smooth solid indicator, clamped to [0,1]) and cos_theta (the contact angle
 * of phase 1 per node; NULL = 90 degrees), compute the chemical potential and
 * mass flux of the initial phi, and set g = g^eq, f = f^eq with the given
 * velocity (ux, uy; NULL = 0) and P = 0.  Copies every host array.
 * dev_workspace: caller-owned device memory of >= lbm_workspace_bytes(p)
 * bytes, 256-byte aligned.  hip_stream: a hipStream_t or NULL.
 * Errors: LBM_EINVAL (parameters out of range, non-finite input, null
 * phi/phi0/out), LBM_ENOMEM (bytes too small), LBM_EDEVICE. */
int lbm_create(const lbm_params *p, void *dev_workspace, size_t bytes, void *hip_stream,
               const double *phi, const double *phi0, const double *cos_theta,
               const double *ux, const double *uy, lbm_domain **out);

/* Free rigid disks (Sec. 2.4, procedure steps 7-10): as lbm_create, plus
 * particles: p->np rows of 8 doubles (x, y, ux, uy, omega, R, rho_p,
 * cos_theta): centre in lattice units (x along nx), translational and angular
 * velocity, radius > 0, density, cos of the contact angle of phase 1 on the
 * particle.  A density <= 0 marks a solid of prescribed motion (e.g. a
 * rotating cylinder): its velocity and angular velocity are held, its centre
 * advances with its velocity, and its force and torque are still reported.  phi0 and cos_theta describe the stationary solid only; each
 * particle adds its tanh indicator (Sec. 4.5; every node, as the plain
 * formula) and every
 * node takes the angle and solid velocity u_p + omega_p x (x - x_p) of the
 * largest indicator component.  After every step except the first, the
 * hydrodynamic force and torque (Eq. Ff) are summed in FP64 over each
 * particle's nodes, the particles advance by explicit Euler (Eq. particle,
 * internal-fluid corrections of Eq. Ffin, gravity (gx, gy), Sec. 4.5
 * repulsion) and the indicator is regenerated.  Copies `particles`.
 * Errors: those of lbm_create; LBM_EINVAL for np outside 0..1024, a NULL
 * particles array with np > 0 or a non-finite particle, R <= 0, |cos| > 1;
 * domains with particles cannot join a batch (LBM_EUNSUPPORTED). */
int lbm_create_particles(const lbm_params *p, void *dev_workspace, size_t bytes, void *hip_stream,
                         const double *phi, const double *phi0, const double *cos_theta,
                         const double *ux, const double *uy, const double *particles,
                         lbm_domain **out);

/* The particles after the steps taken (np x 8, the columns of
 * lbm_create_particles) and the outputs of the last particle update (np x 7:
 * F_f x, y and T_f of Eq. Ff, the internal-fluid corrections F^in x, y and
 * T^in carried to the next update, and the internal fluid density); either
 * pointer may be NULL.  A step launch computes the macroscopic fields of its
 * level before colliding, so the update that belongs to the current level is
 * done by the next step; this call computes it on demand (one macroscopic
 * pass, like lbm_read) without changing the domain.  Blocks.
 * Errors: LBM_EINVAL (NULL domain), LBM_ESTATE (failed finiteness check). */
int lbm_particles(lbm_domain *d, double *state, double *outputs);

/* Voxel solids.  Sec. 4.1 smooths its binary micro-CT solid by a few
 * iterations of a standard Cahn-Hilliard equation before using it as the
 * indicator phi0.  This runs `iters` explicit steps of
 *     d chi/dt = lap mu,  mu = chi^3 - chi - (D^2/8) lap chi
 * on chi = 2 solid - 1 (the planar equilibrium tanh(2 z / D) is the
 * indicator profile of Sec. 2.1), with the isotropic Laplacian, periodic or
 * mirrored at the walls of p->bounce_x / p->bounce_y, and writes
 * phi0 = clamp((1 + chi)/2, 0, 1), ready for lbm_create.  dtau <= 0 takes
 * half the stability limit of the step linearised about chi = +-1,
 * 1 / (2 (kappa L^2 + 2 L)), L = 16/3.  Uses p->nx, ny, D, bounce_x,
 * bounce_y (the rest of p must be valid).  solid, phi0: host [ny][nx]
 * doubles (solid in [0, 1], 1 = solid); the device workspace holds three
 * FP64 planes (lbm_smooth_workspace_bytes; 0 for invalid sizes), 256-byte
 * aligned, free for reuse once the call returns.  Blocks.
 * Errors: LBM_EINVAL (params, NULL pointers, iters outside 0..2^20,
 * non-finite dtau, unaligned workspace), LBM_ENOMEM (workspace too small),
 * LBM_EDEVICE. */
size_t lbm_smooth_workspace_bytes(int32_t nx, int32_t ny);
int lbm_smooth_solid(const lbm_params *p, int32_t iters, double dtau, void *dev_workspace, size_t bytes,
                     void *hip_stream, const double *solid, double *phi0);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, hosts that forbid allocation): lbm_smooth_solid without
 * a workspace.  Its three FP64 planes live in a device array of the library
 * (3 * LBM_NOALLOC_MAX_NODES doubles, 6 MiB), one per device, held until the
 * process ends; the call makes no device allocation.  Same arguments, result
 * and errors as lbm_smooth_solid, plus LBM_EINVAL for grids of more than
 * LBM_NOALLOC_MAX_NODES nodes.  Every call on a device uses that device's one
 * array: calls that overlap on one device (other host threads, other streams)
 * race and must be serialised by the caller.  Blocks. */
#define LBM_NOALLOC_MAX_NODES (1 << 18)
int lbm_smooth_solid_noalloc(const lbm_params *p, int32_t iters, double dtau, void *hip_stream,
                             const double *solid, double *phi0);

/* Procedure steps 2-6, nsteps >= 0 times: one fused kernel per step (stencils
 * for mu, grad phi, S and F_c from a halo tile, velocity and pressure
 * recovery, both MRT collisions, streaming).  Enqueued on the stream; returns
 * without waiting unless a finiteness check is due (lbm_set_check). */
int lbm_step(lbm_domain *d, int64_t nsteps);

/* Check for NaN/Inf every `every` steps inside lbm_step (0 = never, the
 * default).  A failed check returns LBM_ENONFINITE and the domain enters
 * LBM_ESTATE until lbm_import_state(). */
int lbm_set_check(lbm_domain *d, int64_t every);

/* Finiteness check of phi, u and P at the current level (one fused pass over
 * the domain).  Returns LBM_OK, or LBM_ENONFINITE and the domain enters
 * LBM_ESTATE.  Blocks. */
int lbm_check(lbm_domain *d);

/* phi, u = (ux, uy) and P at the current time level (Sec. 3.2, Eqs. phi, u),
 * each nx*ny doubles; any pointer may be NULL.  Blocks. */
int lbm_read(lbm_domain *d, double *phi, double *ux, double *uy, double *p);

/* Total order parameter sum phi (FP64 reduction in a fixed order; for the
 * *DEV storage modes the exact fixed-point sum, in units of 2^-40, carried
 * without overflow for every domain size and rounded once to a double).
 * Blocks. */
int lbm_mass(lbm_domain *d, double *sum_phi);

/* Discrete free energy E_F of Eq. (2energy) (wetting terms through
 * psi = cos(theta) phi0) and kinetic energy E_K = sum rho |u|^2 / 2 (Sec. 2.3),
 * FP64 reductions in a fixed order.  Blocks. */
int lbm_energy(lbm_domain *d, double *e_free, double *e_kin);

/* Steps taken since lbm_create (or the imported state's count). */
int64_t lbm_steps_done(const lbm_domain *d);

/* Exact checkpoint: the distributions, the history of the previous level,
 * the particles (state and carried corrections) and the step count.
 * lbm_state_bytes gives the host buffer size. Blocks. */
size_t lbm_state_bytes(const lbm_domain *d);
int lbm_export_state(lbm_domain *d, void *host_buf, size_t bytes);
int lbm_import_state(lbm_domain *d, const void *host_buf, size_t bytes);

/* Average duration in milliseconds of one step (the fused step kernel, plus
 * the particle kernels when there are particles) over the last lbm_step
 * call, timed with HIP events on the domain's stream (0 if none). */
double lbm_last_step_ms(const lbm_domain *d);

/* Release the handle (not the caller's workspace). */
int lbm_destroy(lbm_domain *d);

/* ---- batching: several domains advanced by one fused launch per step ----
 * All members share one storage mode.  The batch keeps a device tile table
 * (one entry per 64 x TY tile of every member) and a member table in a
 * caller-owned device workspace; each step is ONE kernel launch over all
 * tiles of all members, and lbm_batch_step captures the steps of a call in a
 * HIP graph that is replayed while the member set is unchanged. */
typedef struct lbm_batch lbm_batch;

size_t lbm_batch_workspace_bytes(int32_t max_members, int64_t max_tiles);
/* hip_stream must be a created (non-null) stream: the steps are captured into
 * a HIP graph on it, and members must have been created on the same stream. */
int lbm_batch_create(int32_t storage, int32_t tile, int32_t max_members, int64_t max_tiles,
                     void *dev_workspace, size_t bytes, void *hip_stream, lbm_batch **out);
/* Add / remove a domain (created with the same storage mode).  A member may
 * belong to one batch at a time; removing does not destroy it. */
int lbm_batch_add(lbm_batch *b, lbm_domain *d);
int lbm_batch_remove(lbm_batch *b, lbm_domain *d);
/* Advance every member by min(nsteps, budget) where budget[k] is the number
 * of steps member k may still take (NULL = nsteps for all).  Enqueued. */
int lbm_batch_step(lbm_batch *b, int64_t nsteps, const int64_t *budget);
int lbm_batch_size(const lbm_batch *b);
int lbm_batch_destroy(lbm_batch *b);

/* Thread-local message describing the last error. */
const char *lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBMGLS_H */
