/*
 * lbm3d_oracle.c -- plain FP64 CPU oracle for the three-dimensional form of
 * the coupled lattice Boltzmann method of Zhan, Liu, Chai & Shi, "A
 * thermodynamically consistent and conservative diffuse-interface model for
 * gas-liquid-solid multiphase flows" (arXiv 2311.05097): the phase-field and
 * flow models of Sec. 3.1-3.2 with the three-dimensional K and H the paper
 * gives after Eq. (u), on a stationary smooth solid (procedure steps 1-6 and
 * 11 of Sec. 3.3).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library's three-dimensional path is checked
 * against.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the product path never does.  It shares no
 * code, header, table or generator with the HIP library (nor with the
 * two-dimensional oracle).
 *
 * Everything is FP64, scalar and unfused:
 *   - collision in literal matrix form  f* = f - Lam (f - f^eq) + (I - Lam/2) F,
 *     Lam = M_H^{-1} S_H M_H, M_H = N_H C_d M_0, inverted numerically
 *     (Sec. 4, the collision matrix);
 *   - equilibria and sources term by term as in Sec. 3.1 and 3.2 (every
 *     expression there is written for any dimension d);
 *   - macroscopic recovery u*, f, u, P of Eqs. (uStar) and (u), with the
 *     three-dimensional K;
 *   - second-order isotropic central differences (Sec. 3.2, last paragraph).
 *
 * Readings where the paper is silent (the paper prints the lattice and the
 * matrices for two dimensions only):
 *   R3-LAT   D3Q15: the rest velocity, the 6 face neighbours and the 8 corner
 *            neighbours, with w_0 = (1 - d0)(1 - 2 d0), w_face = (d0 - d0^2)/2,
 *            w_corner = d0^2 / 8.  These are the weights for which
 *            sum w c_a c_b = c_s^2 delta_ab and sum w c_x^2 c_y^2 = c_s^4 (the
 *            conditions the D2Q9 weights of Sec. 4 meet) and for which the
 *            coefficient of the second-moment trace in sum_{i != 0} f_i,
 *            w_0 c_s^2 / (c^2 c_s^2 - c_s^4), is the printed 3-D K = 1 - 2 d0
 *            (the 19- and 27-velocity sets give other values).  Summed along
 *            one axis they are the D2Q9 weights of Sec. 4.
 *   R3-MH    Hermite moments: 1; c_a; c_a^2 - c_s^2; c_a c_b (a < b);
 *            c_x (c_y^2 - c_s^2), c_y (c_z^2 - c_s^2), c_z (c_x^2 - c_s^2);
 *            c_x c_y c_z; c_x^2 c_y^2 - c_s^2 |c|^2 + 2 c_s^4 (on these 15
 *            velocities c_x c_y^2 = c_x c_z^2 and the three mixed fourth
 *            powers coincide; the last row is the one orthogonal to the
 *            lower ones under the weights).  M_0 holds the raw monomials,
 *            N_H the lower-triangular map to these rows, C_d = I (c = 1).
 *            Phase field: S_H^1 = diag(s0, s_1phi x3, s2 x6, s3 x4, s4); flow:
 *            S_H^2 of R3-RATES.
 *   R3-FD    gradient and Laplacian use the isotropic D3Q15 weights at
 *            c_s^2 = 1/3 (2/9, 1/9, 1/72).
 *   R3-NU    the viscosity relations of Sec. 3.2 as printed:
 *            nu = (1/s_2a - 1/2)(c^2 - c_s^2)/2 = (1/s_2b - 1/2) c_s^2 (on this
 *            lattice the diagonal and off-diagonal second moments carry the
 *            same third-moment fluxes as on D2Q9).
 *   R3-RATES the flow distributions relax their zeroth moment and their
 *            fourth-order moment with the per-node s_2a, like the trace of the
 *            second moments: S_H^2 = diag(s_2a, s1 x3, s_2a x3, s_2b x3, s3 x4,
 *            s_2a).  These three scalar moments make up the rest population;
 *            relaxed at different rates (s_0 = s_4 = 1 as in two dimensions)
 *            the linearised scheme has a growing mode at the wave vector
 *            (pi, pi, pi) for every s_2a > 1 (a growth factor up to 1.3 per
 *            step), relaxed at one rate it has none for any s_2a in (0, 2).
 *   R3-H     H = K [(1 - d0)/s_0 - (3 - 7 d0)/s_2a + (1 - 3 d0)] as printed,
 *            which with s_0 = s_2a (R3-RATES) is -2 K (1 - 3 d0)(1/s_2a - 1/2):
 *            the factor that cancels the first-order non-equilibrium part of
 *            sum_{i != 0} f_i on this lattice (the zeroth moment carries
 *            -u.grad(rho)/2, the trace of the second Hermite moments
 *            [2 (1 - 3 d0)/s_2a - (3 - 7 d0)/2] u.grad(rho) - d_t(q)/2).  So
 *            the printed factor and the derived one agree here.
 *   and, as in two dimensions: the Cahn-Hilliard phase equation; F_c from the
 *   current S and the lagged velocity; backward differences for d/dt with
 *   d_t(rho u u) = u F + F u; (1 - phi0) floored at solid_eps in the
 *   viscosity; rho(phi), mu(phi) on phi clamped to [-1, 1]; psi = cos(theta)
 *   phi0 in the wetting terms; the initial state of procedure step 1 with
 *   P = 0, u* = u and the history equal to the current values;
 *   F_b = (rho - rho_ref) g + (1 - phi0) f_b; a stationary solid (u_s = 0).
 *   Periodic in every direction.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 15

/* ---- parameters (layout mirrored by the ctypes wrapper in oracle3d.py) ---- */
typedef struct {
    int32_t nx, ny, nz;
    int32_t pad;                 /* unused (keeps the doubles aligned)      */
    double d0;                   /* c_s^2 / c^2                             */
    double sigma, D, M;          /* Eq. (2energyDensity), mobility          */
    double rho1, rho2, mu1, mu2; /* Eq. (rho) and the viscosity law         */
    double tau_phi;              /* 1 / s_1phi                              */
    double s0, s1, s2, s3, s4;   /* the remaining relaxation rates (s0, s2,
                                    s4: phase field only, R3-RATES)         */
    double gx, gy, gz, rho_ref;  /* gravity part of F_b                     */
    double fbx, fby, fbz;        /* driving part of F_b                     */
    double solid_eps;            /* floor of 1 - phi0 in the viscosity      */
} orc3_params;

/* Planted mistakes for the tests that show a pin would catch them (each
 * factor multiplies one term; 1 = the method as stated):
 *   P3_H      H in (1/2 + H) u.grad rho of the pressure
 *   P3_KDT    the (K/c^2)(dt/2) d_t(rho u.u - S.u) term of the pressure
 *   P3_G      d_t(phi u) in the phase-field source
 *   P3_FC     F_c in the total force
 *   P3_ISO    (c^2 - 3 c_s^2)(u.grad rho) I in M_2F
 *   P3_UDR    u.grad rho, the zeroth moment of F_{i,2} */
enum { P3_H, P3_KDT, P3_G, P3_FC, P3_ISO, P3_UDR, P3_N };
static double plant3[P3_N] = {1, 1, 1, 1, 1, 1};

int orc3_plant(int which, double factor)
{
    if (which < 0 || which >= P3_N) return -1;
    plant3[which] = factor;
    return 0;
}

void orc3_plant_reset(void)
{
    for (int k = 0; k < P3_N; ++k) plant3[k] = 1.0;
}

/* ---- R3-LAT: velocities (opposite pairs adjacent) and weights ---- */
static const int EX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
static const int EY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1};
static const int EZ[Q] = {0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1, 1, -1};

static void weights(double d0, double w[Q])
{
    for (int i = 0; i < Q; ++i) {
        const int n = abs(EX[i]) + abs(EY[i]) + abs(EZ[i]);
        w[i] = n == 0 ? (1.0 - d0) * (1.0 - 2.0 * d0) : (n == 1 ? (d0 - d0 * d0) / 2.0 : d0 * d0 / 8.0);
    }
}

void orc3_lattice(double d0, double w[Q], int cx[Q], int cy[Q], int cz[Q])
{
    weights(d0, w);
    for (int i = 0; i < Q; ++i) {
        if (cx) cx[i] = EX[i];
        if (cy) cy[i] = EY[i];
        if (cz) cz[i] = EZ[i];
    }
}

/* ---- dense 15 x 15 helpers ---- */
static void matmul(const double *A, const double *B, double *C)
{
    for (int i = 0; i < Q; ++i)
        for (int j = 0; j < Q; ++j) {
            double s = 0.0;
            for (int k = 0; k < Q; ++k) s += A[i * Q + k] * B[k * Q + j];
            C[i * Q + j] = s;
        }
}

static int invert(const double *A, double *Ainv)
{
    double a[Q][2 * Q];
    for (int i = 0; i < Q; ++i)
        for (int j = 0; j < 2 * Q; ++j) a[i][j] = j < Q ? A[i * Q + j] : (j - Q == i ? 1.0 : 0.0);
    for (int col = 0; col < Q; ++col) {
        int piv = col;
        for (int r = col + 1; r < Q; ++r)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (a[piv][col] == 0.0) return -1;
        if (piv != col)
            for (int j = 0; j < 2 * Q; ++j) {
                double t = a[col][j]; a[col][j] = a[piv][j]; a[piv][j] = t;
            }
        const double d = a[col][col];
        for (int j = 0; j < 2 * Q; ++j) a[col][j] /= d;
        for (int r = 0; r < Q; ++r) {
            if (r == col) continue;
            const double m = a[r][col];
            if (m != 0.0)
                for (int j = 0; j < 2 * Q; ++j) a[r][j] -= m * a[col][j];
        }
    }
    for (int i = 0; i < Q; ++i)
        for (int j = 0; j < Q; ++j) Ainv[i * Q + j] = a[i][j + Q];
    return 0;
}

/* R3-MH: M_0 (raw monomials, one row per moment, one column per velocity),
 * N_H, and M_H = N_H M_0 with its inverse. */
int orc3_matrices(double d0, double M0[Q * Q], double NH[Q * Q], double MH[Q * Q], double MHinv[Q * Q])
{
    const double cs2 = d0;
    double m0[Q * Q], nh[Q * Q], mh[Q * Q], mhi[Q * Q];
    for (int i = 0; i < Q; ++i) {
        const double x = EX[i], y = EY[i], z = EZ[i];
        const double row[Q] = {1.0, x, y, z, x * x, y * y, z * z, x * y, x * z, y * z,
                               x * y * y, y * z * z, z * x * x, x * y * z, x * x * y * y};
        for (int k = 0; k < Q; ++k) m0[k * Q + i] = row[k];
    }
    memset(nh, 0, sizeof nh);
    for (int k = 0; k < Q; ++k) nh[k * Q + k] = 1.0;
    for (int a = 0; a < 3; ++a) {
        nh[(4 + a) * Q + 0] = -cs2;       /* c_a^2 - c_s^2              */
        nh[(10 + a) * Q + (1 + a)] = -cs2; /* c_a (c_b^2 - c_s^2)        */
        nh[14 * Q + (4 + a)] = -cs2;      /* ... - c_s^2 |c|^2          */
    }
    nh[14 * Q + 0] = 2.0 * cs2 * cs2;     /* ... + 2 c_s^4              */
    matmul(nh, m0, mh);
    if (invert(mh, mhi)) return -1;
    if (M0) memcpy(M0, m0, sizeof m0);
    if (NH) memcpy(NH, nh, sizeof nh);
    if (MH) memcpy(MH, mh, sizeof mh);
    if (MHinv) memcpy(MHinv, mhi, sizeof mhi);
    return 0;
}

static void lam_from(const double *MH, const double *MHinv, const double s[Q], double *Lam)
{
    double sm[Q * Q];
    for (int k = 0; k < Q; ++k)
        for (int j = 0; j < Q; ++j) sm[k * Q + j] = s[k] * MH[k * Q + j];
    matmul(MHinv, sm, Lam);
}

void orc3_collision_matrix(double d0, const double s[Q], double Lam[Q * Q])
{
    double MH[Q * Q], MHinv[Q * Q];
    orc3_matrices(d0, NULL, NULL, MH, MHinv);
    lam_from(MH, MHinv, s, Lam);
}

/* out = f - Lam (f - feq) + (I - Lam/2) F */
static void collide(const double *Lam, const double *fi, const double *feq, const double *Fi, double *out)
{
    for (int i = 0; i < Q; ++i) {
        double acc = fi[i];
        for (int j = 0; j < Q; ++j) acc -= Lam[i * Q + j] * (fi[j] - feq[j]);
        for (int j = 0; j < Q; ++j) acc += ((i == j ? 1.0 : 0.0) - 0.5 * Lam[i * Q + j]) * Fi[j];
        out[i] = acc;
    }
}

/* ---- Sec. 3.1: phase-field equilibrium and source ---- */
void orc3_geq(double d0, double eta, double phi, double mu, const double u[3], double out[Q])
{
    double w[Q];
    weights(d0, w);
    for (int i = 0; i < Q; ++i) {
        if (i == 0)
            out[i] = phi + (w[i] - 1.0) * eta * mu;
        else
            out[i] = w[i] * eta * mu + w[i] * (EX[i] * phi * u[0] + EY[i] * phi * u[1] + EZ[i] * phi * u[2]) / d0;
    }
}

void orc3_gsrc(double d0, const double dtphiu[3], double out[Q])
{
    double w[Q];
    weights(d0, w);
    for (int i = 0; i < Q; ++i)
        out[i] = w[i] * (EX[i] * dtphiu[0] + EY[i] * dtphiu[1] + EZ[i] * dtphiu[2]) / d0;
}

/* ---- Sec. 3.2: flow equilibrium and source ---- */
void orc3_feq(double d0, double P, double rho, const double u[3], const double S[3], double out[Q])
{
    double w[Q];
    weights(d0, w);
    const double c2 = 1.0, cs2 = d0, cs4 = d0 * d0;
    for (int i = 0; i < Q; ++i) {
        const double ci[3] = {EX[i], EY[i], EZ[i]};
        const double lam = (i == 0) ? (w[i] - 1.0) * P / cs2 : w[i] * P / cs2;
        const double lin = w[i] * (ci[0] * rho * u[0] + ci[1] * rho * u[1] + ci[2] * rho * u[2]) / cs2;
        double diag = 0.0, off = 0.0;
        for (int a = 0; a < 3; ++a) {
            diag += (ci[a] * ci[a] - cs2) * (rho * u[a] * u[a] - S[a] * u[a]) / (c2 * cs2 - cs4);
            for (int b = a + 1; b < 3; ++b)
                off += ci[a] * ci[b] / cs4 * (rho * u[a] * u[b] - (S[a] * u[b] + u[a] * S[b]) / 2.0);
        }
        out[i] = lam + lin + w[i] * (diag + off);
    }
}

/* F_{i,2} = w_i [u.grad rho + c_i.(F + rho f)/c_s^2 + diagonal and
 * off-diagonal parts of M_2F]; M2 = {xx, yy, zz, xy, xz, yz}. */
void orc3_fsrc(double d0, const double u[3], const double drho[3], const double F[3], const double rf[3],
               const double M2[6], double out[Q])
{
    double w[Q];
    weights(d0, w);
    const double c2 = 1.0, cs2 = d0, cs4 = d0 * d0;
    const double udr = plant3[P3_UDR] * (u[0] * drho[0] + u[1] * drho[1] + u[2] * drho[2]);
    const int OA[3] = {0, 0, 1}, OB[3] = {1, 2, 2};
    for (int i = 0; i < Q; ++i) {
        const double ci[3] = {EX[i], EY[i], EZ[i]};
        const double t1 = (ci[0] * (F[0] + rf[0]) + ci[1] * (F[1] + rf[1]) + ci[2] * (F[2] + rf[2])) / cs2;
        double diag = 0.0, off = 0.0;
        for (int a = 0; a < 3; ++a) diag += (ci[a] * ci[a] - cs2) * M2[a] / (c2 * cs2 - cs4);
        for (int k = 0; k < 3; ++k) off += ci[OA[k]] * ci[OB[k]] * M2[3 + k] / cs4;
        out[i] = w[i] * (udr + t1 + diag + off);
    }
}

/* ---- R3-FD: isotropic central differences, periodic ---- */
typedef struct { int nx, ny, nz; } dims3;

static inline long nbr(dims3 d, int x, int y, int z, int i)
{
    const int xx = ((x + EX[i]) % d.nx + d.nx) % d.nx;
    const int yy = ((y + EY[i]) % d.ny + d.ny) % d.ny;
    const int zz = ((z + EZ[i]) % d.nz + d.nz) % d.nz;
    return ((long)zz * d.ny + yy) * d.nx + xx;
}

static double WFD[Q];

static void fd_weights(void)
{
    weights(1.0 / 3.0, WFD);
}

static void grad(dims3 d, const double *chi, double *g[3])
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < d.nz; ++z)
        for (int y = 0; y < d.ny; ++y)
            for (int x = 0; x < d.nx; ++x) {
                double s[3] = {0.0, 0.0, 0.0};
                for (int i = 0; i < Q; ++i) {
                    const double v = chi[nbr(d, x, y, z, i)];
                    s[0] += WFD[i] * EX[i] * v;
                    s[1] += WFD[i] * EY[i] * v;
                    s[2] += WFD[i] * EZ[i] * v;
                }
                const long o = ((long)z * d.ny + y) * d.nx + x;
                for (int a = 0; a < 3; ++a) g[a][o] = 3.0 * s[a]; /* 1 / c_s^2 */
            }
}

static void lap(dims3 d, const double *chi, double *out)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < d.nz; ++z)
        for (int y = 0; y < d.ny; ++y)
            for (int x = 0; x < d.nx; ++x) {
                const long o = ((long)z * d.ny + y) * d.nx + x;
                double s = 0.0;
                for (int i = 0; i < Q; ++i) s += WFD[i] * (chi[nbr(d, x, y, z, i)] - chi[o]);
                out[o] = 6.0 * s; /* 2 / c_s^2 */
            }
}

void orc3_grad(int nx, int ny, int nz, const double *chi, double *gx, double *gy, double *gz)
{
    fd_weights();
    double *g[3] = {gx, gy, gz};
    grad((dims3){nx, ny, nz}, chi, g);
}

void orc3_lap(int nx, int ny, int nz, const double *chi, double *out)
{
    fd_weights();
    lap((dims3){nx, ny, nz}, chi, out);
}

/* ---- state ---- */
enum {
    F_PHI, F_RHO, F_MUV, F_MU, F_DPX, F_DPY, F_DPZ, F_DRX, F_DRY, F_DRZ, F_SX, F_SY, F_SZ,
    F_FCX, F_FCY, F_FCZ, F_FX, F_FY, F_FZ, F_USX, F_USY, F_USZ, F_AX, F_AY, F_AZ,
    F_UX, F_UY, F_UZ, F_P, F_S2A, F_S2B, F_H,
    /* history of the previous time level */
    F_PUXP, F_PUYP, F_PUZP, F_TXXP, F_TYYP, F_TZZP, F_TXYP, F_TXZP, F_TYZP, F_QP,
    F_ULX, F_ULY, F_ULZ,
    /* static */
    F_PHI0, F_PSI,
    NF
};
static const char *NAMES[NF] = {
    "phi", "rho", "muv", "mu", "dphix", "dphiy", "dphiz", "drhox", "drhoy", "drhoz", "Sx", "Sy", "Sz",
    "Fcx", "Fcy", "Fcz", "Fx", "Fy", "Fz", "ustarx", "ustary", "ustarz", "asx", "asy", "asz",
    "ux", "uy", "uz", "P", "s2a", "s2b", "H",
    "phiux_p", "phiuy_p", "phiuz_p", "Txx_p", "Tyy_p", "Tzz_p", "Txy_p", "Txz_p", "Tyz_p", "q_p",
    "ulagx", "ulagy", "ulagz", "phi0", "psi"};

typedef struct orc3_state {
    orc3_params p;
    dims3 d;
    long N;
    double w[Q], MH[Q * Q], MHinv[Q * Q], LamG[Q * Q];
    double eta;
    double *g, *f, *gpost, *fpost; /* [Q][N] */
    double *fld[NF];
    long steps;
} orc3_state;

/* Sec. 3.2: relaxation of the flow second moments from mu/(rho (1 - phi0))
 * (R3-NU) and the 3-D H of the pressure (R3-H). */
static void viscous_rates(const orc3_params *p, double rho, double muv, double phi0,
                          double *s2a, double *s2b, double *H)
{
    const double d0 = p->d0, c2 = 1.0, cs2 = d0, K = 1.0 - 2.0 * d0;
    double one_m = 1.0 - phi0;
    if (one_m < p->solid_eps) one_m = p->solid_eps;
    const double nu = muv / (rho * one_m);
    const double tau_a = nu / ((c2 - cs2) / 2.0) + 0.5;
    const double tau_b = nu / cs2 + 0.5;
    *s2a = 1.0 / tau_a;
    *s2b = 1.0 / tau_b;
    /* the printed factor with s_0 = s_2a (R3-RATES) */
    *H = K * ((1.0 - d0) * tau_a - (3.0 - 7.0 * d0) * tau_a + (1.0 - 3.0 * d0));
}

/* Eqs. (uStar) and (u) at one node.  out = u* (3), f dt (3), u (3), s2a,
 * s2b, H, P. */
void orc3_macro_node(const orc3_params *p, int init, const double f[Q], double rho, double muv, double phi0,
                     const double F[3], const double S[3], const double drho[3], double q_p,
                     const double u0[3], double out[13])
{
    const double d0 = p->d0, c2 = 1.0, cs2 = d0, K = 1.0 - 2.0 * d0;
    double w[Q];
    weights(d0, w);
    double us[3], a[3], u[3];
    for (int k = 0; k < 3; ++k) {
        if (init) {
            us[k] = u0[k];
        } else {
            double j = 0.0;
            for (int i = 0; i < Q; ++i) j += (k == 0 ? EX[i] : (k == 1 ? EY[i] : EZ[i])) * f[i];
            us[k] = j / rho + F[k] / (2.0 * rho);
        }
        a[k] = phi0 * (0.0 - us[k]); /* f = phi0 (u_s - u*)/dt, u_s = 0 */
        u[k] = init ? us[k] : us[k] + a[k] / 2.0;
    }
    double s2a, s2b, H;
    viscous_rates(p, rho, muv, phi0, &s2a, &s2b, &H);
    double P = 0.0;
    if (!init) {
        double sum = 0.0;
        for (int i = 1; i < Q; ++i) sum += f[i];
        const double udr = u[0] * drho[0] + u[1] * drho[1] + u[2] * drho[2];
        const double q = rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) - (S[0] * u[0] + S[1] * u[1] + S[2] * u[2]);
        const double rus = (rho * u[0] - S[0]) * u[0] + (rho * u[1] - S[1]) * u[1] + (rho * u[2] - S[2]) * u[2];
        P = cs2 / (1.0 - w[0]) * (sum + (0.5 + plant3[P3_H] * H) * udr - w[0] * rus / (c2 - cs2)
                                  + plant3[P3_KDT] * K / c2 * 0.5 * (q - q_p));
    }
    for (int k = 0; k < 3; ++k) {
        out[k] = us[k];
        out[3 + k] = a[k];
        out[6 + k] = u[k];
    }
    out[9] = s2a; out[10] = s2b; out[11] = H; out[12] = P;
}

/* T_ab = (S_a u_b - u_a S_b)/2 with the current S and the lagged u */
static double t_ab(const orc3_state *st, int a, int b, long o)
{
    double *const *F = st->fld;
    const double S[3] = {F[F_SX][o], F[F_SY][o], F[F_SZ][o]};
    const double u[3] = {F[F_ULX][o], F[F_ULY][o], F[F_ULZ][o]};
    return (S[a] * u[b] - u[a] * S[b]) / 2.0;
}

/* Procedure steps 3-6 (init: u* = the given velocity, P = 0). */
static void macro(orc3_state *st, int init)
{
    const orc3_params *p = &st->p;
    const dims3 d = st->d;
    const long N = st->N;
    double **F = st->fld;
    for (long o = 0; o < N; ++o) {
        double ph = F[F_PHI][o];
        ph = ph < -1.0 ? -1.0 : (ph > 1.0 ? 1.0 : ph);
        F[F_RHO][o] = (p->rho1 - p->rho2) / 2.0 * ph + (p->rho1 + p->rho2) / 2.0;
        F[F_MUV][o] = (p->mu1 - p->mu2) / 2.0 * ph + (p->mu1 + p->mu2) / 2.0;
    }
    /* Eq. (potential) with psi */
    double *lphi = malloc(N * sizeof(double)), *lpsi = malloc(N * sizeof(double));
    lap(d, F[F_PHI], lphi);
    lap(d, F[F_PSI], lpsi);
    const double sg = p->sigma, D = p->D;
    for (long o = 0; o < N; ++o) {
        const double f = F[F_PHI][o], z = F[F_PHI0][o], q = F[F_PSI][o];
        F[F_MU][o] = 3.0 * sg / D * f * (f - 1.0) * (f + 1.0) - 3.0 * D * sg / 8.0 * lphi[o]
                   + 9.0 * sg / D * z * z * f + 3.0 * sg / D * q * (3.0 * f * f + z * z - 1.0)
                   - 3.0 * D * sg / 8.0 * lpsi[o];
    }
    free(lphi);
    free(lpsi);
    double *gp[3] = {F[F_DPX], F[F_DPY], F[F_DPZ]}, *gr[3] = {F[F_DRX], F[F_DRY], F[F_DRZ]};
    grad(d, F[F_PHI], gp);
    grad(d, F[F_RHO], gr);
    double *gm[3] = {malloc(N * sizeof(double)), malloc(N * sizeof(double)), malloc(N * sizeof(double))};
    grad(d, F[F_MU], gm);
    /* consistent mass flux S = M grad(mu) (rho1 - rho2)/2 */
    for (long o = 0; o < N; ++o) {
        F[F_SX][o] = p->M * gm[0][o] * (p->rho1 - p->rho2) / 2.0;
        F[F_SY][o] = p->M * gm[1][o] * (p->rho1 - p->rho2) / 2.0;
        F[F_SZ][o] = p->M * gm[2][o] * (p->rho1 - p->rho2) / 2.0;
    }
    for (int k = 0; k < 3; ++k) free(gm[k]);
    /* F_c,b = d_a T_ab */
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < d.nz; ++z)
        for (int y = 0; y < d.ny; ++y)
            for (int x = 0; x < d.nx; ++x) {
                const long o = ((long)z * d.ny + y) * d.nx + x;
                for (int b = 0; b < 3; ++b) {
                    double s = 0.0;
                    for (int i = 0; i < Q; ++i) {
                        const long n = nbr(d, x, y, z, i);
                        s += WFD[i] * (EX[i] * t_ab(st, 0, b, n) + EY[i] * t_ab(st, 1, b, n)
                                       + EZ[i] * t_ab(st, 2, b, n));
                    }
                    F[F_FCX + b][o] = plant3[P3_FC] * 3.0 * s;
                }
            }
    /* total force F = mu grad(phi) + F_b + F_c */
    for (long o = 0; o < N; ++o) {
        const double mu = F[F_MU][o], rho = F[F_RHO][o], z = F[F_PHI0][o];
        F[F_FX][o] = mu * F[F_DPX][o] + (rho - p->rho_ref) * p->gx + (1.0 - z) * p->fbx + F[F_FCX][o];
        F[F_FY][o] = mu * F[F_DPY][o] + (rho - p->rho_ref) * p->gy + (1.0 - z) * p->fby + F[F_FCY][o];
        F[F_FZ][o] = mu * F[F_DPZ][o] + (rho - p->rho_ref) * p->gz + (1.0 - z) * p->fbz + F[F_FCZ][o];
    }
    /* steps 5-6 */
#pragma omp parallel for schedule(static)
    for (long o = 0; o < N; ++o) {
        double fi[Q], out[13];
        for (int i = 0; i < Q; ++i) fi[i] = st->f[i * N + o];
        const double Fv[3] = {F[F_FX][o], F[F_FY][o], F[F_FZ][o]};
        const double S[3] = {F[F_SX][o], F[F_SY][o], F[F_SZ][o]};
        const double dr[3] = {F[F_DRX][o], F[F_DRY][o], F[F_DRZ][o]};
        const double u0[3] = {F[F_ULX][o], F[F_ULY][o], F[F_ULZ][o]};
        orc3_macro_node(p, init, fi, F[F_RHO][o], F[F_MUV][o], F[F_PHI0][o], Fv, S, dr, F[F_QP][o], u0, out);
        for (int k = 0; k < 3; ++k) {
            F[F_USX + k][o] = out[k];
            F[F_AX + k][o] = out[3 + k];
            F[F_UX + k][o] = out[6 + k];
        }
        F[F_S2A][o] = out[9]; F[F_S2B][o] = out[10]; F[F_H][o] = out[11]; F[F_P][o] = out[12];
    }
}

static void save_history(orc3_state *st)
{
    double **F = st->fld;
    for (long o = 0; o < st->N; ++o) {
        const double ph = F[F_PHI][o], rho = F[F_RHO][o];
        const double u[3] = {F[F_UX][o], F[F_UY][o], F[F_UZ][o]};
        const double S[3] = {F[F_SX][o], F[F_SY][o], F[F_SZ][o]};
        for (int k = 0; k < 3; ++k) F[F_PUXP + k][o] = ph * u[k];
        F[F_TXXP][o] = (S[0] * u[0] + u[0] * S[0]) / 2.0;
        F[F_TYYP][o] = (S[1] * u[1] + u[1] * S[1]) / 2.0;
        F[F_TZZP][o] = (S[2] * u[2] + u[2] * S[2]) / 2.0;
        F[F_TXYP][o] = (S[0] * u[1] + u[0] * S[1]) / 2.0;
        F[F_TXZP][o] = (S[0] * u[2] + u[0] * S[2]) / 2.0;
        F[F_TYZP][o] = (S[1] * u[2] + u[1] * S[2]) / 2.0;
        F[F_QP][o] = rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) - (S[0] * u[0] + S[1] * u[1] + S[2] * u[2]);
        for (int k = 0; k < 3; ++k) F[F_ULX + k][o] = u[k];
    }
}

/* Procedure step 2 (collision) at every node. */
static void collide_all(orc3_state *st)
{
    const orc3_params *p = &st->p;
    const long N = st->N;
    double **F = st->fld;
    const double d0 = p->d0;
#pragma omp parallel for schedule(static)
    for (long o = 0; o < N; ++o) {
        double gi[Q], fi[Q], ge[Q], fe[Q], G[Q], F2[Q], out[Q], Lam[Q * Q];
        for (int i = 0; i < Q; ++i) { gi[i] = st->g[i * N + o]; fi[i] = st->f[i * N + o]; }
        const double ph = F[F_PHI][o], rho = F[F_RHO][o];
        const double u[3] = {F[F_UX][o], F[F_UY][o], F[F_UZ][o]};
        const double S[3] = {F[F_SX][o], F[F_SY][o], F[F_SZ][o]};
        /* phase field (Sec. 3.1) */
        orc3_geq(d0, st->eta, ph, F[F_MU][o], u, ge);
        const double dtpu[3] = {plant3[P3_G] * (ph * u[0] - F[F_PUXP][o]),
                                plant3[P3_G] * (ph * u[1] - F[F_PUYP][o]),
                                plant3[P3_G] * (ph * u[2] - F[F_PUZP][o])};
        orc3_gsrc(d0, dtpu, G);
        collide(st->LamG, gi, ge, G, out);
        for (int i = 0; i < Q; ++i) st->gpost[i * N + o] = out[i];
        /* flow field (Sec. 3.2) */
        orc3_feq(d0, F[F_P][o], rho, u, S, fe);
        const double Fv[3] = {F[F_FX][o], F[F_FY][o], F[F_FZ][o]};
        const double dr[3] = {F[F_DRX][o], F[F_DRY][o], F[F_DRZ][o]};
        const double udr = u[0] * dr[0] + u[1] * dr[1] + u[2] * dr[2];
        /* T = (Su + uS)/2 now and at the previous level */
        const double T[6] = {S[0] * u[0], S[1] * u[1], S[2] * u[2], (S[0] * u[1] + u[0] * S[1]) / 2.0,
                             (S[0] * u[2] + u[0] * S[2]) / 2.0, (S[1] * u[2] + u[1] * S[2]) / 2.0};
        const double Tp[6] = {F[F_TXXP][o], F[F_TYYP][o], F[F_TZZP][o], F[F_TXYP][o], F[F_TXZP][o], F[F_TYZP][o]};
        const int A[6] = {0, 1, 2, 0, 0, 1}, B[6] = {0, 1, 2, 1, 2, 2};
        double M2[6];
        for (int k = 0; k < 6; ++k) {
            const int a = A[k], b = B[k];
            /* d_t(rho u u) = uF + Fu; d_t T by a backward difference;
             * c_s^2 (u grad rho + grad rho u); (c^2 - 3 c_s^2)(u.grad rho) I */
            M2[k] = (u[a] * Fv[b] + Fv[a] * u[b]) - (T[k] - Tp[k]) + d0 * (u[a] * dr[b] + dr[a] * u[b])
                  + (a == b ? plant3[P3_ISO] * (1.0 - 3.0 * d0) * udr : 0.0);
        }
        const double rf[3] = {rho * F[F_AX][o], rho * F[F_AY][o], rho * F[F_AZ][o]};
        orc3_fsrc(d0, u, dr, Fv, rf, M2, F2);
        const double s2a = F[F_S2A][o], s2b = F[F_S2B][o];
        const double sf[Q] = {s2a, p->s1, p->s1, p->s1, s2a, s2a, s2a, s2b, s2b, s2b,
                              p->s3, p->s3, p->s3, p->s3, s2a}; /* R3-RATES */
        lam_from(st->MH, st->MHinv, sf, Lam);
        collide(Lam, fi, fe, F2, out);
        for (int i = 0; i < Q; ++i) st->fpost[i * N + o] = out[i];
    }
}

/* Streaming: f_i(x + c_i, t + 1) = f_i*(x, t), periodic. */
static void stream_all(orc3_state *st)
{
    const dims3 d = st->d;
    const long N = st->N;
    for (int i = 0; i < Q; ++i)
        for (int z = 0; z < d.nz; ++z)
            for (int y = 0; y < d.ny; ++y)
                for (int x = 0; x < d.nx; ++x) {
                    const long o = ((long)z * d.ny + y) * d.nx + x, n = nbr(d, x, y, z, i);
                    st->g[i * N + n] = st->gpost[i * N + o];
                    st->f[i * N + n] = st->fpost[i * N + o];
                }
}

void orc3_step(orc3_state *st, long nsteps)
{
    for (long n = 0; n < nsteps; ++n) {
        collide_all(st);
        stream_all(st);
        save_history(st);
        double **F = st->fld;
        for (long o = 0; o < st->N; ++o) { /* Eq. (phi) */
            double s = 0.0;
            for (int i = 0; i < Q; ++i) s += st->g[i * st->N + o];
            F[F_PHI][o] = s;
        }
        macro(st, 0);
        st->steps++;
    }
}

void orc3_destroy(orc3_state *st)
{
    if (!st) return;
    free(st->g); free(st->f); free(st->gpost); free(st->fpost);
    for (int k = 0; k < NF; ++k) free(st->fld[k]);
    free(st);
}

/* Procedure step 1.  Arrays are [nz][ny][nx], x fastest; cos_theta, ux, uy,
 * uz may be NULL (90 degrees, rest). */
int orc3_create(const orc3_params *p, const double *phi, const double *phi0, const double *cos_theta,
                const double *ux, const double *uy, const double *uz, orc3_state **out)
{
    if (p->nx < 3 || p->ny < 3 || p->nz < 3) return -1;
    fd_weights();
    orc3_state *st = calloc(1, sizeof(orc3_state));
    st->p = *p;
    st->d = (dims3){p->nx, p->ny, p->nz};
    st->N = (long)p->nx * p->ny * p->nz;
    const long N = st->N;
    weights(p->d0, st->w);
    if (orc3_matrices(p->d0, NULL, NULL, st->MH, st->MHinv)) {
        free(st);
        return -1;
    }
    st->eta = p->M / ((p->tau_phi - 0.5) * p->d0); /* M = (1/s_1phi - 1/2) eta c_s^2 dt */
    const double sg[Q] = {p->s0, 1.0 / p->tau_phi, 1.0 / p->tau_phi, 1.0 / p->tau_phi, p->s2, p->s2, p->s2,
                          p->s2, p->s2, p->s2, p->s3, p->s3, p->s3, p->s3, p->s4};
    lam_from(st->MH, st->MHinv, sg, st->LamG);
    st->g = malloc(Q * N * sizeof(double));
    st->f = malloc(Q * N * sizeof(double));
    st->gpost = malloc(Q * N * sizeof(double));
    st->fpost = malloc(Q * N * sizeof(double));
    for (int k = 0; k < NF; ++k) st->fld[k] = calloc(N, sizeof(double));
    double **F = st->fld;
    for (long o = 0; o < N; ++o) {
        double z = phi0[o];
        z = z < 0.0 ? 0.0 : (z > 1.0 ? 1.0 : z);
        F[F_PHI0][o] = z;
        F[F_PSI][o] = (cos_theta ? cos_theta[o] : 0.0) * z;
        F[F_PHI][o] = phi[o];
        F[F_ULX][o] = ux ? ux[o] : 0.0;
        F[F_ULY][o] = uy ? uy[o] : 0.0;
        F[F_ULZ][o] = uz ? uz[o] : 0.0;
    }
    macro(st, 1);
    save_history(st);
    for (long o = 0; o < N; ++o) {
        double ge[Q], fe[Q];
        const double u[3] = {F[F_UX][o], F[F_UY][o], F[F_UZ][o]};
        const double S[3] = {F[F_SX][o], F[F_SY][o], F[F_SZ][o]};
        orc3_geq(p->d0, st->eta, F[F_PHI][o], F[F_MU][o], u, ge);
        orc3_feq(p->d0, F[F_P][o], F[F_RHO][o], u, S, fe);
        for (int i = 0; i < Q; ++i) {
            st->g[i * N + o] = ge[i];
            st->f[i * N + o] = fe[i];
        }
    }
    st->steps = 0;
    *out = st;
    return 0;
}

long orc3_steps_done(const orc3_state *st) { return st->steps; }
int orc3_nfields(void) { return NF; }
const char *orc3_field_name(int k) { return (k >= 0 && k < NF) ? NAMES[k] : NULL; }
void orc3_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }

int orc3_get_field(const orc3_state *st, int k, double *out)
{
    if (k < 0 || k >= NF) return -1;
    memcpy(out, st->fld[k], st->N * sizeof(double));
    return 0;
}

void orc3_get_pops(const orc3_state *st, double *g, double *f)
{
    if (g) memcpy(g, st->g, Q * st->N * sizeof(double));
    if (f) memcpy(f, st->f, Q * st->N * sizeof(double));
}

/* Replace the current post-stream distributions and recompute the
 * macroscopic fields from them (for moment tests). */
void orc3_set_pops(orc3_state *st, const double *g, const double *f)
{
    if (g) memcpy(st->g, g, Q * st->N * sizeof(double));
    if (f) memcpy(st->f, f, Q * st->N * sizeof(double));
    double **F = st->fld;
    for (long o = 0; o < st->N; ++o) {
        double s = 0.0;
        for (int i = 0; i < Q; ++i) s += st->g[i * st->N + o];
        F[F_PHI][o] = s;
    }
    macro(st, 0);
}

double orc3_mass(const orc3_state *st)
{
    double s = 0.0;
    for (long o = 0; o < st->N; ++o) s += st->fld[F_PHI][o];
    return s;
}

/* Discrete E_F of Eq. (2energy) with psi and E_K = sum rho |u|^2 / 2. */
void orc3_energy(const orc3_state *st, double *EF, double *EK)
{
    const orc3_params *p = &st->p;
    const long N = st->N;
    double *const *F = st->fld;
    double *gp[3], *gq[3];
    for (int k = 0; k < 3; ++k) {
        gp[k] = malloc(N * sizeof(double));
        gq[k] = malloc(N * sizeof(double));
    }
    grad(st->d, F[F_PHI], gp);
    grad(st->d, F[F_PSI], gq);
    const double s = p->sigma, D = p->D;
    double ef = 0.0, ek = 0.0;
    for (long o = 0; o < N; ++o) {
        const double f = F[F_PHI][o], z = F[F_PHI0][o], q = F[F_PSI][o];
        const double g2 = gp[0][o] * gp[0][o] + gp[1][o] * gp[1][o] + gp[2][o] * gp[2][o];
        const double gpq = gq[0][o] * gp[0][o] + gq[1][o] * gp[1][o] + gq[2][o] * gp[2][o];
        ef += 3.0 * s / (4.0 * D) * (1.0 - f) * (1.0 - f) * (1.0 + f) * (1.0 + f) + 3.0 * D * s / 16.0 * g2
            + 9.0 * s / (2.0 * D) * z * z * f * f + 3.0 * s / D * q * f * (f * f + z * z - 1.0)
            + 3.0 * D * s / 8.0 * gpq;
        const double ux = F[F_UX][o], uy = F[F_UY][o], uz = F[F_UZ][o];
        ek += F[F_RHO][o] * (ux * ux + uy * uy + uz * uz) / 2.0;
    }
    *EF = ef;
    *EK = ek;
    for (int k = 0; k < 3; ++k) {
        free(gp[k]);
        free(gq[k]);
    }
}
