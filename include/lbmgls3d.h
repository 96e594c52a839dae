/*
 * lbmgls3d.h -- C ABI of the three-dimensional path of the MI355X (gfx950)
 * library for the coupled phase-field / flow lattice Boltzmann method of
 * Zhan, Liu, Chai & Shi, "A thermodynamically consistent and conservative
 * diffuse-interface model for gas-liquid-solid multiphase flows"
 * (arXiv 2311.05097).
 *
 * The library advances, on one GPU, the two sets of 15-velocity distributions
 * of the three-dimensional form of Sec. 3: g_i for the Cahn-Hilliard phase
 * field (Sec. 3.1; chemical potential of Eq. (potential) with the solid
 * penalty and wetting terms) and f_i for the consistent Navier-Stokes flow
 * (Sec. 3.2; viscosity mu/(1-phi0) in the solid; the 3-D K = 1 - 2 d0 and H of
 * Sec. 3.2), with a Hermite-moment collision, on a stationary smooth solid
 * phi0 (procedure steps 1-6 and 11 of Sec. 3.3), periodic in x, y and z.
 * The paper prints the lattice and the collision matrices for two dimensions
 * only; this path uses the 15-velocity set whose weights give the printed 3-D
 * K, w_0 = (1 - d0)(1 - 2 d0), w_face = (d0 - d0^2)/2, w_corner = d0^2/8, the
 * Hermite rows 1, c_a, c_a^2 - c_s^2, c_a c_b, c_x (c_y^2 - c_s^2) (and its
 * cyclic images), c_x c_y c_z, c_x^2 c_y^2 - c_s^2 |c|^2 + 2 c_s^4, and relaxes
 * the flow's zeroth and fourth moments with the per-node s_2a of the second
 * moments (with other rates the scheme has a growing mode at the wave vector
 * (pi, pi, pi)); with that choice the printed 3-D H is
 * -2 K (1 - 3 d0)(1/s_2a - 1/2).
 *
 * Conventions: those of lbmgls.h (return codes LBM_OK / LBM_E*, no throw;
 * lbm3_last_error() for a message; host arrays are [nz][ny][nx] doubles, x
 * fastest, caller-owned and copied or filled before the call returns; the
 * caller provides the device workspace, at least lbm3_workspace_bytes(),
 * 256-byte aligned, alive until lbm3_destroy; work goes on the HIP stream
 * given at creation; calls that return host data synchronise that stream; a
 * handle is used by one host thread at a time).
 */
#ifndef LBMGLS3D_H
#define LBMGLS3D_H

#include "lbmgls.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Storage of the distributions and the history: LBM_STORE_FP64 or
 * LBM_STORE_FP32 (the other modes of lbmgls.h are not built in 3-D).
 * Arithmetic is FP64 in both; the order parameter, chemical potential and
 * mass flux planes between the kernels of a step are FP64. */
typedef struct lbm3_params {
    int32_t nx, ny, nz;   /* grid, each >= 3                                    */
    int32_t storage;      /* LBM_STORE_FP64 or LBM_STORE_FP32                   */
    double d0;            /* c_s^2 / c^2, in (0, 1/2)                           */
    double sigma, D, M;   /* surface tension, interface width, mobility         */
    double rho1, rho2, mu1, mu2; /* densities and dynamic viscosities, > 0       */
    double tau_phi;       /* 1 / s_1phi of the phase field, > 1/2               */
    double s0, s1, s2, s3, s4; /* phase-field rates s0, s2, s3, s4 (s_1phi from
                             tau_phi); flow rates s1 (first moments) and s3
                             (third moments); the flow's other rates follow
                             from the viscosity per node                      */
    double gx, gy, gz, rho_ref; /* body force (rho - rho_ref) g                  */
    double fbx, fby, fbz;  /* body force (1 - phi0) f_b                          */
    double solid_eps;     /* floor of 1 - phi0 in mu / (rho (1 - phi0)), > 0    */
} lbm3_params;

typedef struct lbm3_domain lbm3_domain;

/* Message of the last failed call on this thread ("" if none). */
const char *lbm3_last_error(void);

/* Sec. 4.1 values: d0 = 0.4, sigma = 1e-3, D = 4, M = 0.1, rho1 = rho2 = 1,
 * mu1 = mu2 = 0.1, tau_phi = 1, all rates 1, no body force, solid_eps 0.01,
 * FP64 storage. */
void lbm3_default_params(lbm3_params *p, int32_t nx, int32_t ny, int32_t nz);

/* Device workspace bytes for these parameters (0 if they are invalid). */
size_t lbm3_workspace_bytes(const lbm3_params *p);

/* Procedure step 1: phi, u = (ux, uy, uz) given (NULL velocity components =
 * 0), phi0 the solid indicator in [0, 1] (clamped), cos_theta the contact
 * angle per node (NULL = 90 degrees); P = 0, history = the initial values,
 * distributions at equilibrium.  Errors: LBM_EINVAL (parameters, NULL
 * phi / phi0 / out, non-finite input, |cos_theta| > 1, unaligned workspace),
 * LBM_ENOMEM (workspace too small), LBM_EDEVICE. */
int lbm3_create(const lbm3_params *p, void *dev_workspace, size_t bytes, void *hip_stream, const double *phi,
                const double *phi0, const double *cos_theta, const double *ux, const double *uy,
                const double *uz, lbm3_domain **out);

/* Procedure steps 2-6, nsteps >= 0 times; three kernels per step (order
 * parameter, chemical potential, then the node update: mass flux, gradients,
 * F_c, forces, velocity and pressure recovery, both collisions, streaming).
 * Enqueued; returns without waiting. */
int lbm3_step(lbm3_domain *d, int64_t nsteps);

/* phi, u and P at the current level (nx*ny*nz doubles each, any pointer may
 * be NULL).  Returns LBM_ENONFINITE if any of them is NaN/Inf.  Blocks. */
int lbm3_read(lbm3_domain *d, double *phi, double *ux, double *uy, double *uz, double *p);

/* Total order parameter, FP64 in a fixed order.  Blocks. */
int lbm3_mass(lbm3_domain *d, double *sum_phi);

/* Discrete E_F of Eq. (2energy) (wetting terms through psi = cos(theta) phi0)
 * and E_K = sum rho |u|^2 / 2, FP64 in a fixed order.  Blocks. */
int lbm3_energy(lbm3_domain *d, double *e_free, double *e_kin);

/* HIP-event time of the last lbm3_step call's kernels, ms. */
double lbm3_last_step_ms(const lbm3_domain *d);

/* Release the handle (not the workspace).  Waits for the stream. */
int lbm3_destroy(lbm3_domain *d);

#ifdef __cplusplus
}
#endif
#endif
