/*
 * lbm_oracle.c -- plain FP64 CPU oracle for the coupled D2Q9 lattice
 * Boltzmann method of Zhan, Liu, Chai & Shi, "A thermodynamically consistent
 * and conservative diffuse-interface model for gas-liquid-solid multiphase
 * flows" (arXiv 2311.05097).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header, table or generator
 * with the HIP library.
 *
 * Everything is FP64, scalar, unfused, and follows the paper in its own
 * order and notation:
 *   - collision in literal matrix form  f* = f - Lam (f - f^eq) + (I - Lam/2) F,
 *     Lam = M_H^{-1} S_H M_H, M_H = N_H C_d M_0 built from the printed
 *     matrices and inverted numerically (Sec. 3, Eq. LBE; Sec. 4, matrices);
 *   - equilibria and sources written term by term as printed (Sec. 3.1, 3.2);
 *   - finite differences: second-order isotropic central schemes (Sec. 3.2,
 *     last paragraph);
 *   - macroscopic recovery u*, f, u, P (Sec. 3.2, Eqs. uStar and u);
 *   - procedure steps 1-6 and 11 of Sec. 3.3, and with free rigid particles
 *     steps 7-10: hydrodynamic force and torque (Eq. Ff), the particle
 *     equations of Sec. 2.4 by explicit Euler, the tanh indicator of every
 *     particle regenerated at its new position, the internal-fluid
 *     corrections (Eq. Ffin), the force mu_phi0 grad phi0 (Eq. muPhi0) and the
 *     short-range repulsion of Sec. 4.5.
 *
 * Readings where the paper is silent or ambiguous (each one is listed in the
 * design notes of the repository):
 *   R-CH     the phase equation is the Cahn-Hilliard equation of Sec. 2.1.
 *   R-FD     gradient / Laplacian use the isotropic D2Q9 weights
 *            (4/9, 1/9, 1/36) with c_s^2 = 1/3, independent of d0.
 *   R-FC     F_c = div(Su - uS)/2 is evaluated with the current S and the
 *            velocity of the previous time level (u would otherwise depend
 *            on itself through u*).
 *   R-DT     d/dt terms are backward Euler differences over one step; the
 *            history values of the previous level are kept per node.
 *            d/dt(rho u u) is u F + F u with F of Sec. 3.2 (no rho f).
 *   R-H      H in the pressure of Eq. (u) is -K (1 - 3 d0)(1/s_2a - 1/2),
 *            the factor the first-order non-equilibrium moments of this
 *            model give for sum_{i!=0} f_i: the zeroth moment carries
 *            -u.grad(rho)/2 and the trace of the second Hermite moments
 *            [(1 - 3 d0)/s_2a - (1 - 2 d0)] u.grad(rho) - d_t(q)/2, so that
 *            (1/2 + H) u.grad(rho) + (K/2) d_t q removes exactly the
 *            non-equilibrium part.  The printed factor
 *            K [(1 - d0)/s_0 - (2 - 4 d0)/s_2a + (1 - 3 d0)/2] differs from
 *            it by K^2 (1/s_0 - 1/s_2a); with it a planar interface
 *            translating at a uniform speed U gains velocity errors of order
 *            U that do not shrink with the interface width.  h_form = 1
 *            selects the printed factor.
 *   R-NU     mu/(rho (1-phi0)) uses max(1-phi0, solid_eps) so that s_2a,
 *            s_2b and H stay finite where the indicator saturates at 1.
 *   R-PSI    with a per-node contact angle, cos(theta) phi0 is one field psi;
 *            the wetting terms of Eqs. (2energy) and (potential) use psi.
 *   R-INIT   t = 0: the given phi, u; P = 0; u* = u; f_s = phi0 (u_s - u);
 *            history = current values so every d/dt term is 0 at the first
 *            collision; distributions = equilibria (procedure step 1).
 *   R-FB     F_b = (rho - rho_ref) g + (1 - phi0) f_b.
 *   R-CLAMP  the density and viscosity laws (Eq. rho) are evaluated on phi
 *            clamped to [-1, 1] (overshoots past -1 would make rho <= 0 at
 *            density ratios >= 100); grad rho is the gradient of that field.
 *   R-STAT   stationary solids: u_s = 0 and no mu_phi0 grad phi0 force (the
 *            paper adds it only for freely moving solids).
 *   R-PART   free particles (Sec. 2.4, procedure steps 7-10):
 *            - phi0 = clamp(phi0_static + sum_k phi0_k, 0, 1), phi0_k the
 *              tanh indicator of Sec. 4.5 with the periodic nearest image,
 *              evaluated at every node;
 *            - each node has one owner: the largest of phi0_static and the
 *              phi0_k (ties to the static solid, then the lower k); cos(theta)
 *              and u_s = u_p + omega_p x (x - x_p) are the owner's (u_s = 0
 *              for the static solid), and mu_phi0 grad phi0 is added where
 *              the owner is a particle;
 *            - F_f, T_f sum -rho f over the nodes the particle owns; rho in
 *              (1 - rho/rho_p), F^in = rho V_p du_p/dt and I_f = I_p rho/rho_p
 *              is the indicator-weighted mean density of those nodes;
 *            - M_p = rho_p pi R^2, I_p = M_p R^2 / 2, V_p = pi R^2 (disks);
 *            - explicit Euler over one step, all right-hand sides at the old
 *              level; F^in, T^in are the explicit differences of that update
 *              and enter the next one;
 *            - the particles move after each macroscopic update of the loop,
 *              not after the initial one (procedure: step 1, then steps 2-10
 *              repeated); the next update of the fields sees the new phi0.
 *            - a particle with rho_p <= 0 has prescribed motion (e.g. the
 *              rotating inner cylinder of Sec. 4.5): u_p and omega_p are
 *              held, the centre advances with u_p, F_f and T_f are still
 *              summed (reported), F^in = T^in = 0;
 *            - repulsion (Sec. 4.5) as printed, particle-particle with the
 *              nearest periodic image, particle-wall against optional
 *              axis-aligned wall planes (mirror image of the particle);
 *              none when the stiffness parameter is <= 0.
 *   R-WALL   with bounce_y (bounce_x) set, no-flux walls half a node
 *            outside the first and last rows (columns): populations that
 *            would cross a wall return to their node in the opposite
 *            direction (halfway bounce-back, no slip); the finite-difference
 *            stencils read ghost nodes mirrored about the wall (-1 -> 0,
 *            -2 -> 1, ...): scalars unchanged (a neutral 90-degree wall), the
 *            mass flux S as the gradient of such a scalar (its normal
 *            component changes sign) and the lagged velocity in T of F_c odd
 *            in both components (no slip), each mirror applied in turn at a
 *            corner; free particles measure distances across a walled
 *            direction without the periodic image.
 *   R-VOX    a voxel (binary) solid s is smoothed before use as phi0 by
 *            a few explicit steps of the standard Cahn-Hilliard equation
 *            d chi/dt = lap(mu), mu = chi^3 - chi - kappa lap(chi), on
 *            chi = 2 s - 1, with kappa = D^2/8 (its planar equilibrium
 *            tanh(2 z / D) is the indicator profile of Sec. 2.1), the
 *            isotropic stencils (periodic or mirrored at walls), and a
 *            time step of half the explicit stability limit about chi = +-1
 *            unless one is given; phi0 = clamp((1 + chi)/2, 0, 1).
 *   Periodic in every direction without walls.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- parameters (layout mirrored by the ctypes wrapper in oracle.py) ---- */
typedef struct {
    int32_t nx, ny;
    double d0;        /* c_s^2 / c^2 (Sec. 4, weights)                      */
    double sigma;     /* sigma_12 (Eq. 2energyDensity)                      */
    double D;         /* interface width                                    */
    double M;         /* mobility (Eq. CHE)                                 */
    double rho1, rho2, mu1, mu2; /* Eq. (rho) and the viscosity law         */
    double tau_phi;   /* 1 / s_{1phi}                                       */
    double s0, s1, s2, s3, s4;   /* the remaining entries of S_H^1, S_H^2   */
    double gx, gy, rho_ref;      /* R-FB                                    */
    double fbx, fby;             /* R-FB                                    */
    double solid_eps;            /* R-NU                                    */
    double rep_xi, rep_eps;      /* repulsion threshold and stiffness (Sec. 4.5) */
    double wall_x0, wall_x1, wall_y0, wall_y1; /* wall planes for the repulsion  */
    int32_t walls;               /* bit 0: y0, 1: y1, 2: x0, 3: x1 present  */
    int32_t bounce_y;            /* R-WALL: no-flux walls below and above   */
    int32_t bounce_x;            /* R-WALL: no-flux walls left and right    */
    int32_t h_form;              /* R-H: 0 from the first-order moments, 1 as printed */
} orc_params;

/* Planted mistakes, for the tests that show a pin would catch them: each
 * factor multiplies one term of the method where the stepper uses it.  All
 * are 1 (the method as the paper states it) unless a test sets one through
 * orc_plant and restores it with orc_plant_reset.  Terms:
 *   PL_H      H in (1/2 + H) u.grad rho of the pressure (Sec. 3.2, Eq. u)
 *   PL_KDT    the (K/c^2)(dt/2) d_t(rho u.u - S.u) term of the pressure
 *   PL_G      d_t(phi u) in the phase-field source G_i (Sec. 3.1)
 *   PL_FC     F_c = div(Su - uS)/2 in the total force (Sec. 3.2)
 *   PL_FEQS   the mass flux S in the flow equilibrium's momentum flux
 *   PL_M2FDT  -d_t((Su + uS)/2) in M_2F
 *   PL_M2FUF  d_t(rho u u) = uF + Fu in M_2F
 *   PL_M2FD0  c_s^2 (u grad rho + grad rho u) in M_2F
 *   PL_M2FISO (c^2 - 3 c_s^2)(u.grad rho) I in M_2F
 *   PL_UDR    u.grad rho, the zeroth moment of F_{i,2}
 * Parity unpinned: the -d_t((Su + uS)/2) part of M_2F.  Its effect stays
 * below the discretisation error of every closed-form case built for it
 * (scaling it by 0 or 2 moves no measured error by more than a few parts in
 * a thousand), so no test can show that it is right; it is written as
 * printed and only the GPU path is checked against it. */
enum { PL_H, PL_KDT, PL_G, PL_FC, PL_FEQS, PL_M2FDT, PL_M2FUF, PL_M2FD0, PL_M2FISO, PL_UDR, PL_N };
static double plant[PL_N] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1};

int orc_plant(int which, double factor)
{
    if (which < 0 || which >= PL_N) return -1;
    plant[which] = factor;
    return 0;
}

void orc_plant_reset(void)
{
    for (int k = 0; k < PL_N; ++k) plant[k] = 1.0;
}

/* One free rigid disk (Sec. 2.4): centre, translational and angular velocity,
 * radius, density, cos of the contact angle of phase 1 on its surface. */
enum { P_X, P_Y, P_UX, P_UY, P_OM, P_R, P_RHO, P_COS, NPIN };
/* Per-particle outputs: hydrodynamic force and torque of the last update,
 * internal-fluid corrections carried to the next one, internal density. */
enum { Q_FX, Q_FY, Q_T, Q_FINX, Q_FINY, Q_TIN, Q_RHOIN, NPOUT };

/* ---- D2Q9 lattice: velocity order as in rows 2-3 of M_0 (Sec. 4) ---- */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

void orc_lattice(double d0, double w[9], int cx[9], int cy[9])
{
    /* Sec. 4: w0 = 1 - 2 d0 + d0^2, w1-4 = (d0 - d0^2)/2, w5-8 = d0^2/4 */
    for (int i = 0; i < 9; ++i) {
        if (i == 0)
            w[i] = 1.0 - 2.0 * d0 + d0 * d0;
        else if (i <= 4)
            w[i] = (d0 - d0 * d0) / 2.0;
        else
            w[i] = d0 * d0 / 4.0;
        if (cx) cx[i] = CX[i];
        if (cy) cy[i] = CY[i];
    }
}

/* ---- dense 9x9 helpers ---- */
static void matmul9(const double *A, const double *B, double *C)
{
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 9; ++j) {
            double s = 0.0;
            for (int k = 0; k < 9; ++k) s += A[i * 9 + k] * B[k * 9 + j];
            C[i * 9 + j] = s;
        }
}

/* Gauss-Jordan elimination with partial pivoting; returns 0 on success. */
static int invert9(const double *A, double *Ainv)
{
    double a[9][18];
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 18; ++j)
            a[i][j] = j < 9 ? A[i * 9 + j] : (j - 9 == i ? 1.0 : 0.0);
    for (int col = 0; col < 9; ++col) {
        int piv = col;
        for (int r = col + 1; r < 9; ++r)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (a[piv][col] == 0.0) return -1;
        if (piv != col)
            for (int j = 0; j < 18; ++j) {
                double t = a[col][j]; a[col][j] = a[piv][j]; a[piv][j] = t;
            }
        double d = a[col][col];
        for (int j = 0; j < 18; ++j) a[col][j] /= d;
        for (int r = 0; r < 9; ++r) {
            if (r == col) continue;
            double m = a[r][col];
            if (m != 0.0)
                for (int j = 0; j < 18; ++j) a[r][j] -= m * a[col][j];
        }
    }
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 9; ++j) Ainv[i * 9 + j] = a[i][j + 9];
    return 0;
}

/*
 * Sec. 4 matrices.  M_0 rows: 1, cx, cy, cx^2, cy^2, cx cy, cx cy^2,
 * cx^2 cy, cx^2 cy^2 (the printed matrix), C_d = diag(1,c,c,c^2,c^2,c^2,
 * c^3,c^3,c^4) with c = dx/dt = 1, N_H the printed lower-triangular matrix,
 * M_H = N_H C_d M_0.
 */
void orc_matrices(double d0, double M0[81], double NH[81], double MH[81], double MHinv[81])
{
    const double c = 1.0, cs2 = d0 * c * c;
    double m0[81], nh[81], cd[81], tmp[81], mh[81], mhi[81];
    for (int i = 0; i < 9; ++i) {
        double x = CX[i], y = CY[i];
        double row[9] = {1.0, x, y, x * x, y * y, x * y, x * y * y, x * x * y, x * x * y * y};
        for (int k = 0; k < 9; ++k) m0[k * 9 + i] = row[k];
    }
    memset(cd, 0, sizeof cd);
    const double cpow[9] = {1, c, c, c * c, c * c, c * c, c * c * c, c * c * c, c * c * c * c};
    for (int k = 0; k < 9; ++k) cd[k * 9 + k] = cpow[k];
    memset(nh, 0, sizeof nh);
    for (int k = 0; k < 9; ++k) nh[k * 9 + k] = 1.0;
    nh[3 * 9 + 0] = -cs2;
    nh[4 * 9 + 0] = -cs2;
    nh[6 * 9 + 1] = -cs2;
    nh[7 * 9 + 2] = -cs2;
    nh[8 * 9 + 0] = cs2 * cs2;
    nh[8 * 9 + 3] = -cs2;
    nh[8 * 9 + 4] = -cs2;
    matmul9(cd, m0, tmp);
    matmul9(nh, tmp, mh);
    invert9(mh, mhi);
    if (M0) memcpy(M0, m0, sizeof m0);
    if (NH) memcpy(NH, nh, sizeof nh);
    if (MH) memcpy(MH, mh, sizeof mh);
    if (MHinv) memcpy(MHinv, mhi, sizeof mhi);
}

/* Lam = M_H^{-1} diag(s) M_H (Sec. 4). */
static void lam_from(const double *MH, const double *MHinv, const double s[9], double *Lam)
{
    double sm[81];
    for (int k = 0; k < 9; ++k)
        for (int j = 0; j < 9; ++j) sm[k * 9 + j] = s[k] * MH[k * 9 + j];
    matmul9(MHinv, sm, Lam);
}

void orc_collision_matrix(double d0, const double s[9], double Lam[81])
{
    double MH[81], MHinv[81];
    orc_matrices(d0, NULL, NULL, MH, MHinv);
    lam_from(MH, MHinv, s, Lam);
}

/* Eq. (LBE) at one node, dt = 1: out = f - Lam (f - feq) + (I - Lam/2) F. */
static void collide(const double *Lam, const double *fi, const double *feq,
                    const double *Fi, double *out)
{
    for (int i = 0; i < 9; ++i) {
        double acc = fi[i];
        for (int j = 0; j < 9; ++j) acc -= Lam[i * 9 + j] * (fi[j] - feq[j]);
        for (int j = 0; j < 9; ++j)
            acc += ((i == j ? 1.0 : 0.0) - 0.5 * Lam[i * 9 + j]) * Fi[j];
        out[i] = acc;
    }
}

/* ---- Sec. 3.1: phase-field equilibrium and source ---- */
void orc_geq(double d0, double eta, double phi, double mu, double ux, double uy, double out[9])
{
    double w[9];
    const double cs2 = d0;
    orc_lattice(d0, w, NULL, NULL);
    for (int i = 0; i < 9; ++i) {
        if (i == 0)
            out[i] = phi + (w[i] - 1.0) * eta * mu;
        else
            out[i] = w[i] * eta * mu + w[i] * (CX[i] * phi * ux + CY[i] * phi * uy) / cs2;
    }
}

/* G_i = w_i c_i . d_t(phi u) / c_s^2 */
void orc_gsrc(double d0, double dtphiux, double dtphiuy, double out[9])
{
    double w[9];
    orc_lattice(d0, w, NULL, NULL);
    for (int i = 0; i < 9; ++i) out[i] = w[i] * (CX[i] * dtphiux + CY[i] * dtphiuy) / d0;
}

/* ---- Sec. 3.2: flow equilibrium (diagonal part summed over alpha) ---- */
void orc_feq(double d0, double P, double rho, double ux, double uy, double Sx, double Sy, double out[9])
{
    double w[9];
    const double c2 = 1.0, cs2 = d0, cs4 = d0 * d0;
    orc_lattice(d0, w, NULL, NULL);
    const double u[2] = {ux, uy}, S[2] = {Sx, Sy};
    for (int i = 0; i < 9; ++i) {
        const double ci[2] = {CX[i], CY[i]};
        double lam = (i == 0) ? (w[i] - 1.0) * P / cs2 : w[i] * P / cs2;
        double lin = w[i] * (ci[0] * rho * u[0] + ci[1] * rho * u[1]) / cs2;
        double diag = 0.0;
        for (int a = 0; a < 2; ++a)
            diag += (ci[a] * ci[a] - cs2) * (rho * u[a] * u[a] - S[a] * u[a]) / (c2 * cs2 - cs4);
        double off = ci[0] * ci[1] / cs4 * (rho * u[0] * u[1] - (S[0] * u[1] + u[0] * S[1]) / 2.0);
        out[i] = lam + lin + w[i] * (diag + off);
    }
}

/* F_{i,2} = w_i [u.grad rho + c_i.(F + rho f)/cs2 + diag(M2F) + offdiag(M2F)] */
void orc_fsrc(double d0, double ux, double uy, double drx, double dry, double Fx, double Fy,
              double rfx, double rfy, double M2xx, double M2xy, double M2yy, double out[9])
{
    double w[9];
    const double c2 = 1.0, cs2 = d0, cs4 = d0 * d0;
    orc_lattice(d0, w, NULL, NULL);
    const double M2d[2] = {M2xx, M2yy};
    for (int i = 0; i < 9; ++i) {
        const double ci[2] = {CX[i], CY[i]};
        double t0 = ux * drx + uy * dry;
        double t1 = (ci[0] * (Fx + rfx) + ci[1] * (Fy + rfy)) / cs2;
        double diag = 0.0;
        for (int a = 0; a < 2; ++a) diag += (ci[a] * ci[a] - cs2) * M2d[a] / (c2 * cs2 - cs4);
        double off = ci[0] * ci[1] * M2xy / cs4;
        out[i] = w[i] * (t0 + t1 + diag + off);
    }
}

/* ---- Sec. 3.2 (last paragraph): isotropic central differences ---- */
static const double WT[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

static inline long nb(int nx, int ny, int x, int y, int i)
{
    int xx = ((x + CX[i]) % nx + nx) % nx;
    int yy = ((y + CY[i]) % ny + ny) % ny;
    return (long)yy * nx + xx;
}

/* Index along one direction of a node that v (at most one node outside
 * 0..n-1) stands for: the periodic image, or with walls (R-WALL) the mirror
 * image; *ghost tells which. */
static inline int img(int v, int n, int walls, int *ghost)
{
    *ghost = walls && (v < 0 || v >= n);
    if (*ghost) return v < 0 ? -1 - v : 2 * n - 1 - v;
    return (v % n + n) % n;
}

/* Neighbour value of a scalar in direction i (even under every mirror). */
static inline double nbv(const double *chi, int nx, int ny, int wx, int wy, int x, int y, int i)
{
    int gx, gy;
    const int xx = img(x + CX[i], nx, wx, &gx), yy = img(y + CY[i], ny, wy, &gy);
    return chi[(long)yy * nx + xx];
}

static void grad_b(int nx, int ny, int wx, int wy, const double *chi, double *gx, double *gy)
{
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double sx = 0.0, sy = 0.0;
            for (int i = 0; i < 9; ++i) {
                double v = nbv(chi, nx, ny, wx, wy, x, y, i);
                sx += WT[i] * CX[i] * v;
                sy += WT[i] * CY[i] * v;
            }
            gx[(long)y * nx + x] = 3.0 * sx; /* 1 / c_s^2 with c_s^2 = 1/3 */
            gy[(long)y * nx + x] = 3.0 * sy;
        }
}

static void lap_b(int nx, int ny, int wx, int wy, const double *chi, double *lap)
{
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long o = (long)y * nx + x;
            double s = 0.0;
            for (int i = 0; i < 9; ++i) s += WT[i] * (nbv(chi, nx, ny, wx, wy, x, y, i) - chi[o]);
            lap[o] = 6.0 * s; /* 2 / c_s^2 with c_s^2 = 1/3 */
        }
}

void orc_grad(int nx, int ny, const double *chi, double *gx, double *gy)
{
    grad_b(nx, ny, 0, 0, chi, gx, gy);
}

void orc_lap(int nx, int ny, const double *chi, double *lap)
{
    lap_b(nx, ny, 0, 0, chi, lap);
}

/* ---- Eq. (potential): chemical potential, wetting terms through psi ---- */
void orc_mu(const orc_params *p, const double *phi, const double *phi0, const double *psi,
            double *mu)
{
    const int nx = p->nx, ny = p->ny;
    const long N = (long)nx * ny;
    double *lphi = malloc(N * sizeof(double)), *lpsi = malloc(N * sizeof(double));
    lap_b(nx, ny, p->bounce_x, p->bounce_y, phi, lphi);
    lap_b(nx, ny, p->bounce_x, p->bounce_y, psi, lpsi);
    const double s = p->sigma, D = p->D;
    for (long o = 0; o < N; ++o) {
        double f = phi[o], z = phi0[o], q = psi[o];
        mu[o] = 3.0 * s / D * f * (f - 1.0) * (f + 1.0) - 3.0 * D * s / 8.0 * lphi[o]
              + 9.0 * s / D * z * z * f + 3.0 * s / D * q * (3.0 * f * f + z * z - 1.0)
              - 3.0 * D * s / 8.0 * lpsi[o];
    }
    free(lphi);
    free(lpsi);
}

/* ---- state ---- */
enum {
    F_PHI, F_RHO, F_MUV, F_MU, F_DPHIX, F_DPHIY, F_DRHOX, F_DRHOY, F_SX, F_SY,
    F_FCX, F_FCY, F_FX, F_FY, F_USX, F_USY, F_AX, F_AY, F_UX, F_UY, F_P,
    F_S2A, F_S2B, F_H,
    /* history of the previous time level */
    F_PHIUXP, F_PHIUYP, F_TXXP, F_TXYP, F_TYYP, F_QP, F_ULX, F_ULY,
    /* static (regenerated from the particles every step) */
    F_PHI0, F_PSI,
    /* stationary solid as given, node owner (-1 static, k particle), solid
     * velocity, mu_phi0 (Eq. muPhi0) */
    F_ZB, F_CB, F_OWN, F_USOLX, F_USOLY, F_MUZ,
    NFIELDS
};
static const char *FIELD_NAMES[NFIELDS] = {
    "phi", "rho", "muv", "mu", "dphix", "dphiy", "drhox", "drhoy", "Sx", "Sy",
    "Fcx", "Fcy", "Fx", "Fy", "ustarx", "ustary", "asx", "asy", "ux", "uy", "P",
    "s2a", "s2b", "H",
    "phiux_p", "phiuy_p", "Txx_p", "Txy_p", "Tyy_p", "q_p", "ulagx", "ulagy",
    "phi0", "psi",
    "phi0_static", "cos_static", "owner", "usolx", "usoly", "mu_phi0"};

typedef struct orc_state {
    orc_params p;
    long N;
    double w[9], MH[81], MHinv[81], LamG[81];
    double eta;
    double *g, *f, *gpost, *fpost; /* [9][N] each */
    double *fld[NFIELDS];
    long steps;
    int np;          /* number of free particles               */
    double *pin;     /* [np][NPIN]  particle state             */
    double *pout;    /* [np][NPOUT] forces and corrections     */
} orc_state;

static double clamp01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

/* Relaxation of the flow second moments from mu/(rho(1-phi0)) (Sec. 3.2),
 * and H of the 2-D pressure (Sec. 3.2, after Eq. u). */
static void viscous_rates(const orc_params *p, double rho, double muv, double phi0,
                          double *s2a, double *s2b, double *H)
{
    const double d0 = p->d0, c2 = 1.0, cs2 = d0;
    double one_m = 1.0 - phi0;
    if (one_m < p->solid_eps) one_m = p->solid_eps; /* R-NU */
    double nu = muv / (rho * one_m);
    double tau_a = nu / ((c2 - cs2) / 2.0) + 0.5; /* nu = (1/s2a - 1/2)(c^2-c_s^2)/2 */
    double tau_b = nu / cs2 + 0.5;                /* nu = (1/s2b - 1/2) c_s^2      */
    *s2a = 1.0 / tau_a;
    *s2b = 1.0 / tau_b;
    double K = 1.0 - d0;
    if (p->h_form == 1) /* as printed after Eq. (u) */
        *H = K * ((1.0 - d0) / p->s0 - (2.0 - 4.0 * d0) * tau_a + (1.0 - 3.0 * d0) / 2.0);
    else                /* R-H */
        *H = -K * (1.0 - 3.0 * d0) * (tau_a - 0.5);
}

/* Steps 5-6 at one node (Sec. 3.2, Eqs. uStar and u).  f: the 9 flow
 * distributions; F: total force; S: mass flux; drho: grad rho; q_p: the
 * history value of rho u.u - S.u; (u0x, u0y): the given velocity, used only
 * when init != 0 (R-INIT); (usolx, usoly): the solid velocity u_s at the node.
 * out = u*x, u*y, f_x dt, f_y dt, ux, uy, s2a, s2b, H, P. */
void orc_macro_node(const orc_params *p, int init, const double f[9], double rho, double muv,
                    double phi0, double Fx, double Fy, double Sx, double Sy, double drx,
                    double dry, double q_p, double u0x, double u0y, double usolx, double usoly,
                    double out[10])
{
    const double d0 = p->d0, c2 = 1.0, cs2 = d0, K = 1.0 - d0;
    double w[9];
    orc_lattice(d0, w, NULL, NULL);
    double usx, usy;
    if (init) {
        usx = u0x;
        usy = u0y;
    } else {
        double jx = 0.0, jy = 0.0;
        for (int i = 0; i < 9; ++i) {
            jx += CX[i] * f[i];
            jy += CY[i] * f[i];
        }
        usx = jx / rho + Fx / (2.0 * rho); /* Eq. uStar, dt = 1 */
        usy = jy / rho + Fy / (2.0 * rho);
    }
    /* f = phi0 (u_s - u*) / dt; u_s = 0 for a stationary solid */
    double ax = phi0 * (usolx - usx), ay = phi0 * (usoly - usy);
    double ux = init ? usx : usx + ax / 2.0; /* Eq. u */
    double uy = init ? usy : usy + ay / 2.0;
    double s2a, s2b, H;
    viscous_rates(p, rho, muv, phi0, &s2a, &s2b, &H);
    double P = 0.0;
    if (!init) {
        double sum = 0.0;
        for (int i = 1; i < 9; ++i) sum += f[i];
        double udr = ux * drx + uy * dry;
        double q = rho * (ux * ux + uy * uy) - (Sx * ux + Sy * uy);
        P = cs2 / (1.0 - w[0]) *
            (sum + (0.5 + plant[PL_H] * H) * udr - w[0] * ((rho * ux - Sx) * ux + (rho * uy - Sy) * uy) / (c2 - cs2)
             + plant[PL_KDT] * K / c2 * 0.5 * (q - q_p));
    }
    out[0] = usx; out[1] = usy; out[2] = ax; out[3] = ay; out[4] = ux; out[5] = uy;
    out[6] = s2a; out[7] = s2b; out[8] = H; out[9] = P;
}

/* Procedure steps 3-6 at the current time from phi (already in the state),
 * the flow distributions and the lagged velocity.  If init != 0, u* is the
 * given velocity and P = 0 (R-INIT). */
/* T_alpha,beta = (S_alpha u_beta - u_alpha S_beta)/2 of R-FC at node (x, y).
 * Nodes outside the domain are periodic images, or with walls (R-WALL) ghost
 * nodes built from the mirrored node: S is the gradient of a scalar mirrored
 * evenly (its component normal to the wall changes sign) and the no-slip
 * velocity is odd in both components; at a corner both mirrors apply. */
static double t_ab(const orc_state *st, int a, int b, int x, int y)
{
    double sS[2] = {1.0, 1.0}, sU[2] = {1.0, 1.0};
    int gx, gy;
    x = img(x, st->p.nx, st->p.bounce_x, &gx);
    y = img(y, st->p.ny, st->p.bounce_y, &gy);
    if (gx) { sS[0] = -sS[0]; sU[0] = -sU[0]; sU[1] = -sU[1]; }
    if (gy) { sS[1] = -sS[1]; sU[0] = -sU[0]; sU[1] = -sU[1]; }
    const long o = (long)y * st->p.nx + x;
    double *const *F = st->fld;
    const double S[2] = {sS[0] * F[F_SX][o], sS[1] * F[F_SY][o]};
    const double u[2] = {sU[0] * F[F_ULX][o], sU[1] * F[F_ULY][o]};
    return (S[a] * u[b] - u[a] * S[b]) / 2.0;
}

static void macro(orc_state *st, int init)
{
    const orc_params *p = &st->p;
    const int nx = p->nx, ny = p->ny;
    const long N = st->N;
    double **F = st->fld;
    /* step 3: density and viscosity laws (Eq. rho) */
    for (long o = 0; o < N; ++o) {
        double ph = F[F_PHI][o];
        ph = ph < -1.0 ? -1.0 : (ph > 1.0 ? 1.0 : ph); /* R-CLAMP */
        F[F_RHO][o] = (p->rho1 - p->rho2) / 2.0 * ph + (p->rho1 + p->rho2) / 2.0;
        F[F_MUV][o] = (p->mu1 - p->mu2) / 2.0 * ph + (p->mu1 + p->mu2) / 2.0;
    }
    /* chemical potential, gradients, consistent mass flux S = M grad(mu)(rho1-rho2)/2 */
    orc_mu(p, F[F_PHI], F[F_PHI0], F[F_PSI], F[F_MU]);
    const int WX = p->bounce_x, WY = p->bounce_y;
    grad_b(nx, ny, WX, WY, F[F_PHI], F[F_DPHIX], F[F_DPHIY]);
    grad_b(nx, ny, WX, WY, F[F_RHO], F[F_DRHOX], F[F_DRHOY]);
    double *gmx = malloc(N * sizeof(double)), *gmy = malloc(N * sizeof(double));
    grad_b(nx, ny, WX, WY, F[F_MU], gmx, gmy);
    for (long o = 0; o < N; ++o) {
        F[F_SX][o] = p->M * gmx[o] * (p->rho1 - p->rho2) / 2.0;
        F[F_SY][o] = p->M * gmy[o] * (p->rho1 - p->rho2) / 2.0;
    }
    /* step 4: F_c = div(S u - u S)/2 with the lagged velocity (R-FC):
     * F_c,beta = d_alpha T_alpha,beta,  T_alpha,beta = (S_alpha u_beta - u_alpha S_beta)/2 */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            for (int b = 0; b < 2; ++b) {
                double sx = 0.0, sy = 0.0;
                for (int i = 0; i < 9; ++i) sx += WT[i] * CX[i] * t_ab(st, 0, b, x + CX[i], y + CY[i]);
                for (int i = 0; i < 9; ++i) sy += WT[i] * CY[i] * t_ab(st, 1, b, x + CX[i], y + CY[i]);
                /* d_x T_x,beta + d_y T_y,beta, 1 / c_s^2 = 3 */
                F[b == 0 ? F_FCX : F_FCY][(long)y * nx + x] = plant[PL_FC] * (3.0 * sx + 3.0 * sy);
            }
        }
    /* mu_phi0 (Eq. muPhi0) where a free particle owns the node (R-PART) */
    double *gzx = malloc(N * sizeof(double)), *gzy = malloc(N * sizeof(double));
    double *lphi = malloc(N * sizeof(double));
    grad_b(nx, ny, WX, WY, F[F_PHI0], gzx, gzy);
    lap_b(nx, ny, WX, WY, F[F_PHI], lphi);
    for (long o = 0; o < N; ++o) {
        F[F_MUZ][o] = 0.0;
        int k = (int)F[F_OWN][o];
        if (k < 0) continue;
        double f = F[F_PHI][o], z = F[F_PHI0][o], c = st->pin[k * NPIN + P_COS];
        const double sg = p->sigma, D = p->D;
        F[F_MUZ][o] = 9.0 * sg / D * z * f * f + 3.0 * sg * c / D * f * (3.0 * z * z + f * f - 1.0)
                    - 3.0 * D * sg * c / 8.0 * lphi[o];
    }
    /* total force F = mu grad(phi) + mu_phi0 grad(phi0) + F_b + F_c */
    for (long o = 0; o < N; ++o) {
        double mu = F[F_MU][o], rho = F[F_RHO][o], z = F[F_PHI0][o];
        double fbx = (rho - p->rho_ref) * p->gx + (1.0 - z) * p->fbx;
        double fby = (rho - p->rho_ref) * p->gy + (1.0 - z) * p->fby;
        F[F_FX][o] = mu * F[F_DPHIX][o] + F[F_MUZ][o] * gzx[o] + fbx + F[F_FCX][o];
        F[F_FY][o] = mu * F[F_DPHIY][o] + F[F_MUZ][o] * gzy[o] + fby + F[F_FCY][o];
    }
    free(gzx); free(gzy); free(lphi);
    /* steps 5-6 */
    for (long o = 0; o < N; ++o) {
        double fi[9], out[10];
        for (int i = 0; i < 9; ++i) fi[i] = st->f[i * N + o];
        orc_macro_node(p, init, fi, F[F_RHO][o], F[F_MUV][o], F[F_PHI0][o], F[F_FX][o], F[F_FY][o],
                       F[F_SX][o], F[F_SY][o], F[F_DRHOX][o], F[F_DRHOY][o], F[F_QP][o],
                       F[F_ULX][o], F[F_ULY][o], F[F_USOLX][o], F[F_USOLY][o], out);
        F[F_USX][o] = out[0]; F[F_USY][o] = out[1];
        F[F_AX][o] = out[2];  F[F_AY][o] = out[3];
        F[F_UX][o] = out[4];  F[F_UY][o] = out[5];
        F[F_S2A][o] = out[6]; F[F_S2B][o] = out[7]; F[F_H][o] = out[8];
        F[F_P][o] = out[9];
    }
    free(gmx); free(gmy);
}

/* Save the values of the current level as the history of the next one. */
static void save_history(orc_state *st)
{
    double **F = st->fld;
    for (long o = 0; o < st->N; ++o) {
        double ph = F[F_PHI][o], rho = F[F_RHO][o];
        double ux = F[F_UX][o], uy = F[F_UY][o], Sx = F[F_SX][o], Sy = F[F_SY][o];
        F[F_PHIUXP][o] = ph * ux;
        F[F_PHIUYP][o] = ph * uy;
        F[F_TXXP][o] = (Sx * ux + ux * Sx) / 2.0;
        F[F_TXYP][o] = (Sx * uy + ux * Sy) / 2.0;
        F[F_TYYP][o] = (Sy * uy + uy * Sy) / 2.0;
        F[F_QP][o] = rho * (ux * ux + uy * uy) - (Sx * ux + Sy * uy);
        F[F_ULX][o] = ux;
        F[F_ULY][o] = uy;
    }
}

static const double PI = 3.14159265358979323846;

/* Nearest periodic image of a coordinate difference. */
static double per(double d, int n)
{
    return d - n * floor(d / n + 0.5);
}

/* The same along x and y, where a walled direction has no image (R-WALL). */
static double perx(const orc_params *p, double d)
{
    return p->bounce_x ? d : per(d, p->nx);
}
static double pery(const orc_params *p, double d)
{
    return p->bounce_y ? d : per(d, p->ny);
}

/* Procedure step 9 (and step 1): the indicator field from the stationary
 * solid and the particles at their current positions, the node owners, the
 * owner's contact angle (psi = cos(theta) phi0) and solid velocity (R-PART). */
static void particle_statics(orc_state *st)
{
    const orc_params *p = &st->p;
    const int nx = p->nx, ny = p->ny;
    double **F = st->fld;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long o = (long)y * nx + x;
            double best = F[F_ZB][o], sum = F[F_ZB][o], c = F[F_CB][o];
            int own = -1;
            for (int k = 0; k < st->np; ++k) {
                const double *q = st->pin + k * NPIN;
                double r = hypot(perx(p, x - q[P_X]), pery(p, y - q[P_Y]));
                double zk = 0.5 + 0.5 * tanh((q[P_R] - r) / (p->D / 2.0));
                sum += zk;
                if (zk > best) { best = zk; own = k; c = q[P_COS]; }
            }
            double z = clamp01(sum);
            F[F_PHI0][o] = z;
            F[F_PSI][o] = c * z;
            F[F_OWN][o] = own;
            F[F_USOLX][o] = 0.0;
            F[F_USOLY][o] = 0.0;
            if (own >= 0) { /* u_s = u_p + omega_p x (x - x_p) */
                const double *q = st->pin + own * NPIN;
                double rx = perx(p, x - q[P_X]), ry = pery(p, y - q[P_Y]);
                F[F_USOLX][o] = q[P_UX] - q[P_OM] * ry;
                F[F_USOLY][o] = q[P_UY] + q[P_OM] * rx;
            }
        }
}

/* Sec. 4.5: the repulsion on particle k from particle j (pp) or from the
 * mirror image x' of k across a wall (pw: stiffness eps/2, radii 2R). */
static void repulsion(double dx, double dy, double Rsum, double xi, double eps, double out[2])
{
    double d = hypot(dx, dy), m;
    if (d > Rsum + xi) m = 0.0;
    else if (d >= Rsum) m = (Rsum + xi - d) * (Rsum + xi - d) / eps;
    else m = (Rsum - d) / eps;
    out[0] = m * dx;
    out[1] = m * dy;
}

void orc_repulsion(double dx, double dy, double Rsum, double xi, double eps, double out[2])
{
    repulsion(dx, dy, Rsum, xi, eps, out);
}

/* Procedure steps 7, 8 and 10 after a macroscopic update (R-PART). */
static void particles_update(orc_state *st)
{
    const orc_params *p = &st->p;
    const int nx = p->nx, ny = p->ny, np = st->np;
    const long N = st->N;
    double **F = st->fld;
    double *acc = calloc((size_t)np * 5, sizeof(double)); /* Fx, Fy, T, sum phi0 rho, sum phi0 */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long o = (long)y * nx + x;
            int k = (int)F[F_OWN][o];
            if (k < 0) continue;
            const double *q = st->pin + k * NPIN;
            double rho = F[F_RHO][o];
            double fx = rho * F[F_AX][o], fy = rho * F[F_AY][o]; /* rho f dt, Eq. Ff */
            double rx = perx(p, x - q[P_X]), ry = pery(p, y - q[P_Y]);
            acc[k * 5 + 0] -= fx;
            acc[k * 5 + 1] -= fy;
            acc[k * 5 + 2] -= rx * fy - ry * fx;
            acc[k * 5 + 3] += F[F_PHI0][o] * rho;
            acc[k * 5 + 4] += F[F_PHI0][o];
        }
    (void)N;
    double *nw = malloc((size_t)np * NPIN * sizeof(double));
    for (int k = 0; k < np; ++k) {
        const double *q = st->pin + k * NPIN;
        double *o = st->pout + k * NPOUT;
        const double R = q[P_R], rp = q[P_RHO];
        const double V = PI * R * R, Mp = rp * V, Ip = Mp * R * R / 2.0;
        double rin = acc[k * 5 + 4] > 0.0 ? acc[k * 5 + 3] / acc[k * 5 + 4] : 0.0;
        o[Q_FX] = acc[k * 5 + 0];
        o[Q_FY] = acc[k * 5 + 1];
        o[Q_T] = acc[k * 5 + 2];
        o[Q_RHOIN] = rin;
        double fr[2] = {0.0, 0.0}, t[2];
        for (int j = 0; j < np && p->rep_eps > 0.0; ++j) {
            if (j == k) continue;
            const double *qj = st->pin + j * NPIN;
            repulsion(perx(p, q[P_X] - qj[P_X]), pery(p, q[P_Y] - qj[P_Y]), R + qj[P_R], p->rep_xi, p->rep_eps, t);
            fr[0] += t[0]; fr[1] += t[1];
        }
        const double wall[4] = {p->wall_y0, p->wall_y1, p->wall_x0, p->wall_x1};
        for (int w = 0; w < 4 && p->rep_eps > 0.0; ++w) {
            if (!(p->walls >> w & 1)) continue;
            double dx = 0.0, dy = 0.0; /* x_p - x', x' the mirror image of x_p */
            if (w < 2) dy = 2.0 * (q[P_Y] - wall[w]);
            else dx = 2.0 * (q[P_X] - wall[w]);
            repulsion(dx, dy, 2.0 * R, p->rep_xi, p->rep_eps / 2.0, t);
            fr[0] += t[0]; fr[1] += t[1];
        }
        double *n = nw + k * NPIN;
        for (int i = 0; i < NPIN; ++i) n[i] = q[i];
        if (rp > 0.0) { /* Eq. (particle), explicit Euler with dt = 1 */
            double Fx = o[Q_FX] + o[Q_FINX] + (1.0 - rin / rp) * Mp * p->gx + fr[0];
            double Fy = o[Q_FY] + o[Q_FINY] + (1.0 - rin / rp) * Mp * p->gy + fr[1];
            double Tz = o[Q_T] + o[Q_TIN];
            n[P_UX] = q[P_UX] + Fx / Mp;
            n[P_UY] = q[P_UY] + Fy / Mp;
            n[P_OM] = q[P_OM] + Tz / Ip;
        }
        n[P_X] = q[P_X] + q[P_UX];
        n[P_Y] = q[P_Y] + q[P_UY];
        if (!p->bounce_x) n[P_X] -= nx * floor(n[P_X] / nx);
        if (!p->bounce_y) n[P_Y] -= ny * floor(n[P_Y] / ny);
        /* Eq. (Ffin), explicit: carried to the next update */
        o[Q_FINX] = rp > 0.0 ? rin * V * (n[P_UX] - q[P_UX]) : 0.0;
        o[Q_FINY] = rp > 0.0 ? rin * V * (n[P_UY] - q[P_UY]) : 0.0;
        o[Q_TIN] = rp > 0.0 ? Ip * rin / rp * (n[P_OM] - q[P_OM]) : 0.0;
    }
    memcpy(st->pin, nw, (size_t)np * NPIN * sizeof(double));
    free(nw);
    free(acc);
    particle_statics(st); /* step 9 */
}

/* R-VOX (Sec. 4.1: the binary micro-CT solid is smoothed by a finite number
 * of iterations of a standard CH equation): iters explicit steps on chi =
 * 2 s - 1; dtau <= 0 takes half the stability limit of the step linearised
 * about chi = +-1, 1 / (kappa L^2 + 2 L) with L = 16/3 the largest magnitude
 * of the discrete Laplacian's symbol. */
double orc_vox_dtau(double D)
{
    const double kappa = D * D / 8.0, L = 16.0 / 3.0;
    return 0.5 / (kappa * L * L + 2.0 * L);
}

/* iters explicit CH steps from chi0 (R-VOX), chi unclamped. */
void orc_smooth_chi(int nx, int ny, int wx, int wy, double D, int iters, double dtau, const double *chi0,
                    double *chi)
{
    const long N = (long)nx * ny;
    const double kappa = D * D / 8.0;
    if (dtau <= 0.0) dtau = orc_vox_dtau(D);
    double *mu = malloc(N * sizeof(double)), *lap = malloc(N * sizeof(double));
    for (long o = 0; o < N; ++o) chi[o] = chi0[o];
    for (int it = 0; it < iters; ++it) {
        lap_b(nx, ny, wx, wy, chi, lap);
        for (long o = 0; o < N; ++o) mu[o] = chi[o] * chi[o] * chi[o] - chi[o] - kappa * lap[o];
        lap_b(nx, ny, wx, wy, mu, lap);
        for (long o = 0; o < N; ++o) chi[o] += dtau * lap[o];
    }
    free(mu); free(lap);
}

/* phi0 = clamp((1 + chi)/2, 0, 1) after smoothing chi = 2 s - 1. */
void orc_smooth_solid(int nx, int ny, int wx, int wy, double D, int iters, double dtau, const double *s,
                      double *phi0)
{
    const long N = (long)nx * ny;
    double *chi0 = calloc(N, sizeof(double)), *chi = calloc(N, sizeof(double));
    for (long o = 0; o < N; ++o) chi0[o] = 2.0 * s[o] - 1.0;
    orc_smooth_chi(nx, ny, wx, wy, D, iters, dtau, chi0, chi);
    for (long o = 0; o < N; ++o) {
        double z = (1.0 + chi[o]) / 2.0;
        phi0[o] = z < 0.0 ? 0.0 : (z > 1.0 ? 1.0 : z);
    }
    free(chi0); free(chi);
}

void orc_destroy(orc_state *st)
{
    if (!st) return;
    free(st->pin); free(st->pout);
    free(st->g); free(st->f); free(st->gpost); free(st->fpost);
    for (int k = 0; k < NFIELDS; ++k) free(st->fld[k]);
    free(st);
}

/* Procedure step 1.  Arrays are [ny][nx], x fastest; cos_theta may be NULL
 * (90 degrees everywhere).  phi0 and cos_theta describe the stationary solid;
 * parts holds np free particles, NPIN values each (P_X ... P_COS). */
int orc_create_particles(const orc_params *p, const double *phi, const double *phi0,
                         const double *cos_theta, const double *ux, const double *uy, int np,
                         const double *parts, orc_state **out)
{
    if (p->nx < 3 || p->ny < 3) return -1;
    orc_state *st = calloc(1, sizeof(orc_state));
    st->p = *p;
    st->N = (long)p->nx * p->ny;
    const long N = st->N;
    orc_lattice(p->d0, st->w, NULL, NULL);
    orc_matrices(p->d0, NULL, NULL, st->MH, st->MHinv);
    st->eta = p->M / ((p->tau_phi - 0.5) * p->d0); /* M = (1/s1phi - 1/2) eta c_s^2 dt */
    double sg[9] = {p->s0, 1.0 / p->tau_phi, 1.0 / p->tau_phi, p->s2, p->s2, p->s2, p->s3, p->s3, p->s4};
    lam_from(st->MH, st->MHinv, sg, st->LamG);
    st->g = malloc(9 * N * sizeof(double));
    st->f = malloc(9 * N * sizeof(double));
    st->gpost = malloc(9 * N * sizeof(double));
    st->fpost = malloc(9 * N * sizeof(double));
    for (int k = 0; k < NFIELDS; ++k) st->fld[k] = calloc(N, sizeof(double));
    double **F = st->fld;
    st->np = np > 0 ? np : 0;
    st->pin = calloc((size_t)(st->np ? st->np : 1) * NPIN, sizeof(double));
    st->pout = calloc((size_t)(st->np ? st->np : 1) * NPOUT, sizeof(double));
    if (st->np) memcpy(st->pin, parts, (size_t)st->np * NPIN * sizeof(double));
    for (long o = 0; o < N; ++o) {
        F[F_ZB][o] = clamp01(phi0[o]);
        F[F_CB][o] = cos_theta ? cos_theta[o] : 0.0;
        F[F_PHI][o] = phi[o];
        F[F_ULX][o] = ux ? ux[o] : 0.0;
        F[F_ULY][o] = uy ? uy[o] : 0.0;
    }
    particle_statics(st);
    macro(st, 1);
    save_history(st); /* every d/dt term is zero at the first collision */
    for (long o = 0; o < N; ++o) {
        double ge[9], fe[9];
        orc_geq(p->d0, st->eta, F[F_PHI][o], F[F_MU][o], F[F_UX][o], F[F_UY][o], ge);
        orc_feq(p->d0, F[F_P][o], F[F_RHO][o], F[F_UX][o], F[F_UY][o], F[F_SX][o], F[F_SY][o], fe);
        for (int i = 0; i < 9; ++i) {
            st->g[i * N + o] = ge[i];
            st->f[i * N + o] = fe[i];
        }
    }
    st->steps = 0;
    *out = st;
    return 0;
}

int orc_create(const orc_params *p, const double *phi, const double *phi0,
               const double *cos_theta, const double *ux, const double *uy, orc_state **out)
{
    return orc_create_particles(p, phi, phi0, cos_theta, ux, uy, 0, NULL, out);
}

int orc_nparticles(const orc_state *st) { return st->np; }

/* Current particle state (np x NPIN) and outputs of the last update
 * (np x NPOUT); either may be NULL. */
void orc_get_particles(const orc_state *st, double *state, double *outputs)
{
    if (state && st->np) memcpy(state, st->pin, (size_t)st->np * NPIN * sizeof(double));
    if (outputs && st->np) memcpy(outputs, st->pout, (size_t)st->np * NPOUT * sizeof(double));
}

/* Procedure step 2 (collision part) at every node. */
static void collide_all(orc_state *st)
{
    const orc_params *p = &st->p;
    const long N = st->N;
    double **F = st->fld;
    const double d0 = p->d0;
#pragma omp parallel for schedule(static) if (st->N >= 2048) /* threads only where they pay */
    for (long o = 0; o < N; ++o) {
        double gi[9], fi[9], ge[9], fe[9], G[9], F2[9], out[9], Lam[81];
        for (int i = 0; i < 9; ++i) { gi[i] = st->g[i * N + o]; fi[i] = st->f[i * N + o]; }
        double ph = F[F_PHI][o], rho = F[F_RHO][o], ux = F[F_UX][o], uy = F[F_UY][o];
        double Sx = F[F_SX][o], Sy = F[F_SY][o];
        /* phase field */
        orc_geq(d0, st->eta, ph, F[F_MU][o], ux, uy, ge);
        orc_gsrc(d0, plant[PL_G] * (ph * ux - F[F_PHIUXP][o]), plant[PL_G] * (ph * uy - F[F_PHIUYP][o]), G);
        collide(st->LamG, gi, ge, G, out);
        for (int i = 0; i < 9; ++i) st->gpost[i * N + o] = out[i];
        /* flow field */
        orc_feq(d0, F[F_P][o], rho, ux, uy, plant[PL_FEQS] * Sx, plant[PL_FEQS] * Sy, fe);
        double Fx = F[F_FX][o], Fy = F[F_FY][o], drx = F[F_DRHOX][o], dry = F[F_DRHOY][o];
        double Txx = (Sx * ux + ux * Sx) / 2.0, Txy = (Sx * uy + ux * Sy) / 2.0, Tyy = (Sy * uy + uy * Sy) / 2.0;
        double udr = ux * drx + uy * dry;
        /* M_2F = d_t(rho u u - (Su+uS)/2) + cs2 (u grad rho + grad rho u) + (c^2 - 3 cs2)(u.grad rho) I */
        const double kuf = plant[PL_M2FUF], kdt = plant[PL_M2FDT], kd0 = plant[PL_M2FD0], kiso = plant[PL_M2FISO];
        double M2xx = kuf * (ux * Fx + Fx * ux) - kdt * (Txx - F[F_TXXP][o]) + kd0 * d0 * (ux * drx + drx * ux)
                    + kiso * (1.0 - 3.0 * d0) * udr;
        double M2xy = kuf * (ux * Fy + Fx * uy) - kdt * (Txy - F[F_TXYP][o]) + kd0 * d0 * (ux * dry + drx * uy);
        double M2yy = kuf * (uy * Fy + Fy * uy) - kdt * (Tyy - F[F_TYYP][o]) + kd0 * d0 * (uy * dry + dry * uy)
                    + kiso * (1.0 - 3.0 * d0) * udr;
        /* the zeroth moment u.grad rho of F_{i,2} enters through grad rho's
         * projection on u; scaling grad rho's share there scales that moment
         * alone (orc_fsrc uses drx, dry only in it) */
        orc_fsrc(d0, ux, uy, plant[PL_UDR] * drx, plant[PL_UDR] * dry, Fx, Fy, rho * F[F_AX][o], rho * F[F_AY][o],
                 M2xx, M2xy, M2yy, F2);
        double sf[9] = {p->s0, p->s1, p->s1, F[F_S2A][o], F[F_S2A][o], F[F_S2B][o], p->s3, p->s3, p->s4};
        lam_from(st->MH, st->MHinv, sf, Lam);
        collide(Lam, fi, fe, F2, out);
        for (int i = 0; i < 9; ++i) st->fpost[i * N + o] = out[i];
    }
}

/* Streaming: f_i(x + c_i, t + 1) = f_i*(x, t), periodic; with walls a
 * population that would cross one returns to its node in the opposite
 * direction (R-WALL). */
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static void stream_all(orc_state *st)
{
    const int nx = st->p.nx, ny = st->p.ny;
    const long N = st->N;
    for (int i = 0; i < 9; ++i)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long o = (long)y * nx + x, d = nb(nx, ny, x, y, i);
                int j = i;
                const int xx = x + CX[i], yy = y + CY[i];
                if ((st->p.bounce_y && (yy < 0 || yy >= ny)) || (st->p.bounce_x && (xx < 0 || xx >= nx))) {
                    d = o;
                    j = OPP[i];
                }
                st->g[j * N + d] = st->gpost[i * N + o];
                st->f[j * N + d] = st->fpost[i * N + o];
            }
}

void orc_step(orc_state *st, long nsteps)
{
    for (long n = 0; n < nsteps; ++n) {
        collide_all(st);      /* step 2 */
        stream_all(st);
        save_history(st);     /* values at t^n become the history of t^{n+1} */
        double **F = st->fld;
        for (long o = 0; o < st->N; ++o) { /* Eq. (phi): phi = sum_i g_i */
            double s = 0.0;
            for (int i = 0; i < 9; ++i) s += st->g[i * st->N + o];
            F[F_PHI][o] = s;
        }
        macro(st, 0);         /* steps 3-6 */
        if (st->np) particles_update(st); /* steps 7-10 */
        st->steps++;
    }
}

long orc_steps_done(const orc_state *st) { return st->steps; }
int orc_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int orc_nfields(void) { return NFIELDS; }
const char *orc_field_name(int k) { return (k >= 0 && k < NFIELDS) ? FIELD_NAMES[k] : NULL; }

int orc_get_field(const orc_state *st, int k, double *out)
{
    if (k < 0 || k >= NFIELDS) return -1;
    memcpy(out, st->fld[k], st->N * sizeof(double));
    return 0;
}

/* Post-stream distributions [9][N] of the current level. */
void orc_get_pops(const orc_state *st, double *g, double *f)
{
    if (g) memcpy(g, st->g, 9 * st->N * sizeof(double));
    if (f) memcpy(f, st->f, 9 * st->N * sizeof(double));
}

/* Total order parameter, summed in node order. */
double orc_mass(const orc_state *st)
{
    double s = 0.0;
    for (long o = 0; o < st->N; ++o) s += st->fld[F_PHI][o];
    return s;
}

/* Discrete E_F of Eq. (2energy) (with psi, R-PSI) and E_K = sum rho |u|^2 / 2
 * over the whole domain including the solid. */
void orc_energy(const orc_state *st, double *EF, double *EK)
{
    const orc_params *p = &st->p;
    const int nx = p->nx, ny = p->ny;
    const long N = st->N;
    double *const *F = st->fld;
    double *gx = malloc(N * sizeof(double)), *gy = malloc(N * sizeof(double));
    double *qx = malloc(N * sizeof(double)), *qy = malloc(N * sizeof(double));
    grad_b(nx, ny, p->bounce_x, p->bounce_y, F[F_PHI], gx, gy);
    grad_b(nx, ny, p->bounce_x, p->bounce_y, F[F_PSI], qx, qy);
    const double s = p->sigma, D = p->D;
    double ef = 0.0, ek = 0.0;
    for (long o = 0; o < N; ++o) {
        double f = F[F_PHI][o], z = F[F_PHI0][o], q = F[F_PSI][o];
        ef += 3.0 * s / (4.0 * D) * (1.0 - f) * (1.0 - f) * (1.0 + f) * (1.0 + f)
            + 3.0 * D * s / 16.0 * (gx[o] * gx[o] + gy[o] * gy[o])
            + 9.0 * s / (2.0 * D) * z * z * f * f
            + 3.0 * s / D * q * f * (f * f + z * z - 1.0)
            + 3.0 * D * s / 8.0 * (qx[o] * gx[o] + qy[o] * gy[o]);
        double ux = F[F_UX][o], uy = F[F_UY][o];
        ek += F[F_RHO][o] * (ux * ux + uy * uy) / 2.0;
    }
    *EF = ef;
    *EK = ek;
    free(gx); free(gy); free(qx); free(qy);
}
