// lbm3d.hip -- three-dimensional path of the library (C ABI in lbmgls3d.h):
// the phase-field and flow lattice Boltzmann models of Sec. 3.1-3.2 on a
// 15-velocity lattice, three kernels per time step.
//
// Why three kernels and not one fused tile kernel as in two dimensions: the
// node update needs the order parameter on a 3-node ring (mu needs its
// Laplacian, the mass flux S the gradient of mu, F_c the divergence of a
// tensor built from S).  In 3-D a 64 x 4 x 4 block would have to rebuild the
// order parameter from 15 populations at ~7x as many ring nodes as it owns.
// Instead the order parameter and mu are written once per step as FP64
// planes (8 + 8 bytes per node).  The mu kernel and the node update
// (k3_march) march along z over 64 x 4 columns, holding slices of what they
// read on rings in LDS (mu: phi on the one-node ring; the node update: phi
// and the lagged velocity on the one-node ring and mu on the two-node ring,
// forming S on the ring there), so that each of those values is loaded under
// twice per step instead of once per neighbour that needs it.
//
// Arithmetic is FP64 for either storage; FP32 storage rounds what is stored.
//
// Layout (one domain, N = nx ny nz nodes, x fastest, planes of `pitch`
// entries, pitch = N rounded up to 64):
//   pop[2]  : 15 g planes then 15 f planes, storage type T (double or float);
//             g_0 holds g_0 - phi_hist (the history order parameter stored
//             at the same node) so that FP32 rounds only small numbers;
//   hist[2] : phi, ux, uy, uz, Sx, Sy, Sz of the previous level, type T;
//   stat    : phi0, psi = cos(theta) phi0, lap psi (FP64, built at creation);
//   phi, mu, S (3): FP64 planes of the current level;
//   out     : phi, ux, uy, uz, P (FP64) for reads;  part: per-block sums.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "lbmgls3d.h"

namespace lbm3 {

constexpr int Q = 15;
constexpr int NT = 256;  // threads per block, one node each
constexpr int NPART3 = 4;  // per-block sums: mass, E_F, E_K, non-finite count

// Velocities: rest, the six faces, the eight corners.  This ordering is the
// library's own: +x, +y, +z, -x, -y, -z, then the corners by sign pattern.
__host__ __device__ constexpr int cxv(int i) {
    return i == 0 ? 0 : (i <= 6 ? (i == 1 ? 1 : (i == 4 ? -1 : 0)) : (((i - 7) & 1) ? -1 : 1));
}
__host__ __device__ constexpr int cyv(int i) {
    return i == 0 ? 0 : (i <= 6 ? (i == 2 ? 1 : (i == 5 ? -1 : 0)) : (((i - 7) & 2) ? -1 : 1));
}
__host__ __device__ constexpr int czv(int i) {
    return i == 0 ? 0 : (i <= 6 ? (i == 3 ? 1 : (i == 6 ? -1 : 0)) : (((i - 7) & 4) ? -1 : 1));
}

// Hermite row k at velocity (x, y, z), cs2 = c_s^2 (c = 1).
__host__ __device__ inline double hrow(int k, int x, int y, int z, double cs2) {
    switch (k) {
        case 0: return 1.0;
        case 1: return x;
        case 2: return y;
        case 3: return z;
        case 4: return x * x - cs2;
        case 5: return y * y - cs2;
        case 6: return z * z - cs2;
        case 7: return x * y;
        case 8: return x * z;
        case 9: return y * z;
        case 10: return x * (y * y - cs2);
        case 11: return y * (z * z - cs2);
        case 12: return z * (x * x - cs2);
        case 13: return x * y * z;
        default: return x * x * y * y - cs2 * (x * x + y * y + z * z) + 2.0 * cs2 * cs2;
    }
}

// Hermite moments m_k = sum_i H_k(c_i) f_i of 15 populations in the order
// rest, +x +y +z -x -y -z, corners (bits of i - 7: x, y, z sign), through
// the face sums and differences and a three-stage butterfly over the eight
// corners (about 50 additions instead of the dense 15 x 15 product).
template <class R>
__host__ __device__ inline void moments15(const R f[Q], R cs2, R m[Q]) {
    const R sx = f[1] + f[4], dx = f[1] - f[4];
    const R sy = f[2] + f[5], dy = f[2] - f[5];
    const R sz = f[3] + f[6], dz = f[3] - f[6];
    const R px0 = f[7] + f[8], mx0 = f[7] - f[8];      // y+, z+
    const R px1 = f[9] + f[10], mx1 = f[9] - f[10];    // y-, z+
    const R px2 = f[11] + f[12], mx2 = f[11] - f[12];  // y+, z-
    const R px3 = f[13] + f[14], mx3 = f[13] - f[14];  // y-, z-
    const R e0 = px0 + px1, ey0 = px0 - px1, e1 = px2 + px3, ey1 = px2 - px3;
    const R o0 = mx0 + mx1, oy0 = mx0 - mx1, o1 = mx2 + mx3, oy1 = mx2 - mx3;
    const R K = e0 + e1, Kz = e0 - e1, Ky = ey0 + ey1, Kyz = ey0 - ey1;
    const R Kx = o0 + o1, Kxz = o0 - o1, Kxy = oy0 + oy1, Kxyz = oy0 - oy1;
    const R m0 = f[0] + sx + sy + sz + K;
    m[0] = m0;
    m[1] = dx + Kx;
    m[2] = dy + Ky;
    m[3] = dz + Kz;
    m[4] = sx + K - cs2 * m0;
    m[5] = sy + K - cs2 * m0;
    m[6] = sz + K - cs2 * m0;
    m[7] = Kxy;
    m[8] = Kxz;
    m[9] = Kyz;
    m[10] = Kx - cs2 * m[1];  // sum c_x c_y^2 f = the corners' x-odd sum
    m[11] = Ky - cs2 * m[2];
    m[12] = Kz - cs2 * m[3];
    m[13] = Kxyz;
    m[14] = K - cs2 * (sx + sy + sz + R(3) * K) + R(2) * cs2 * cs2 * m0;
}

// d_i = sum_k H_k(c_i) a_k (the inverse transform without the weights), by
// the same structure run backwards.
template <class R>
__host__ __device__ inline void inverse15(const R a[Q], R cs2, R d[Q]) {
    const R tr = a[4] + a[5] + a[6];
    d[0] = a[0] - cs2 * tr + R(2) * cs2 * cs2 * a[14];
    const R base = a[0] - cs2 * tr + (R(2) * cs2 * cs2 - cs2) * a[14];
    const R Ax = base + a[4], Bx = a[1] - cs2 * a[10];
    const R Ay = base + a[5], By = a[2] - cs2 * a[11];
    const R Az = base + a[6], Bz = a[3] - cs2 * a[12];
    d[1] = Ax + Bx;
    d[4] = Ax - Bx;
    d[2] = Ay + By;
    d[5] = Ay - By;
    d[3] = Az + Bz;
    d[6] = Az - Bz;
    const R oc = R(1) - cs2;
    const R E = a[0] + oc * tr + (R(1) - R(3) * cs2 + R(2) * cs2 * cs2) * a[14];
    const R X = a[1] + oc * a[10], Y = a[2] + oc * a[11], Z = a[3] + oc * a[12];
    const R Ezp = E + Z, Ezm = E - Z, Yzp = Y + a[9], Yzm = Y - a[9];
    const R Xzp = X + a[8], Xzm = X - a[8], XYzp = a[7] + a[13], XYzm = a[7] - a[13];
    const R pe0 = Ezp + Yzp, pe1 = Ezp - Yzp, pe2 = Ezm + Yzm, pe3 = Ezm - Yzm;
    const R po0 = Xzp + XYzp, po1 = Xzp - XYzp, po2 = Xzm + XYzm, po3 = Xzm - XYzm;
    d[7] = pe0 + po0;
    d[8] = pe0 - po0;
    d[9] = pe1 + po1;
    d[10] = pe1 - po1;
    d[11] = pe2 + po2;
    d[12] = pe2 - po2;
    d[13] = pe3 + po3;
    d[14] = pe3 - po3;
}

struct Coef3 {
    int32_t nx, ny, nz, first;  // first: the step at level 0 (u* = the given u, P = 0)
    int64_t pitch, n;
    double cs2, w[3], K, eta;   // weights: rest, face, corner
    double sigma, Dw, Mob, rho1, rho2, mu1, mu2;
    double gx, gy, gz, rho_ref, fbx, fby, fbz, solid_eps;
    double s1, s3;              // flow rates of the first and third moments
    double inv_norm[7];         // 1 / sum_i w_i H_k(c_i)^2 by row class (hcls)
    double gA[7];               // phase field: -s_k / |H_k|^2 by row class
    double gB1;                 // phase field: (1 - s_k/2) / |H_k|^2 of the first moments
};

// The Hermite rows fall into seven classes of equal norm and equal
// phase-field rate: 0 | 1-3 | 4-6 | 7-9 | 10-12 | 13 | 14.
__host__ __device__ constexpr int hcls(int k) {
    return k == 0 ? 0 : (k <= 3 ? 1 : (k <= 6 ? 2 : (k <= 9 ? 3 : (k <= 12 ? 4 : (k == 13 ? 5 : 6)))));
}

template <class T>
struct Planes3 {
    T* pop[2];
    T* hist[2];
    double* stat;
    double* phi;
    double* mu;
    double* S;
    double* out;
    double* part;
};

__device__ __forceinline__ double wgt(const Coef3& c, int i) { return i == 0 ? c.w[0] : (i <= 6 ? c.w[1] : c.w[2]); }

// D3Q15 central-difference weights at c_s^2 = 1/3 (2/9, 1/9, 1/72).
__device__ __forceinline__ double wfd(int i) { return i == 0 ? 2.0 / 9.0 : (i <= 6 ? 1.0 / 9.0 : 1.0 / 72.0); }

struct Nb {
    int32_t o[Q];  // node index of x + c_i, periodic (domains hold < 2^31 nodes)
};

__device__ __forceinline__ void neighbours_xyz(const Coef3& c, int x, int y, int z, Nb& nb) {
    const int xs[3] = {x == 0 ? c.nx - 1 : x - 1, x, x == c.nx - 1 ? 0 : x + 1};
    const int ys[3] = {y == 0 ? c.ny - 1 : y - 1, y, y == c.ny - 1 ? 0 : y + 1};
    const int zs[3] = {z == 0 ? c.nz - 1 : z - 1, z, z == c.nz - 1 ? 0 : z + 1};
#pragma unroll
    for (int i = 0; i < Q; ++i)
        nb.o[i] = (zs[czv(i) + 1] * c.ny + ys[cyv(i) + 1]) * c.nx + xs[cxv(i) + 1];
}

__device__ __forceinline__ void neighbours(const Coef3& c, int64_t o, Nb& nb) {
    const int32_t oo = (int32_t)o, nxy = c.nx * c.ny;
    const int z = oo / nxy;
    const int r = oo - z * nxy;
    const int y = r / c.nx, x = r - y * c.nx;
    neighbours_xyz(c, x, y, z, nb);
}

// finite: v - v is 0 for every finite v, NaN for NaN and +-Inf
__device__ __forceinline__ bool fin(double v) { return v - v == 0.0; }

__device__ __forceinline__ double rho_of(const Coef3& c, double ph) {
    ph = ph < -1.0 ? -1.0 : (ph > 1.0 ? 1.0 : ph);
    return c.rho2 + (c.rho1 - c.rho2) * (1.0 + ph) * 0.5;
}

__device__ __forceinline__ double muv_of(const Coef3& c, double ph) {
    ph = ph < -1.0 ? -1.0 : (ph > 1.0 ? 1.0 : ph);
    return c.mu2 + (c.mu1 - c.mu2) * (1.0 + ph) * 0.5;
}

// ---------------------------------------------------------------- statics
// in: [0] phi0, [1] cos theta (staged FP64 inputs)
__global__ __launch_bounds__(NT) void k3_static(Coef3 c, const double* __restrict__ in, double* __restrict__ stat) {
    const int64_t o = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (o >= c.n) return;
    double z = in[o];
    z = z < 0.0 ? 0.0 : (z > 1.0 ? 1.0 : z);
    stat[o] = z;
    stat[c.pitch + o] = in[c.pitch + o] * z;
}

// lap psi from psi (FP64)
__global__ __launch_bounds__(NT) void k3_lap_psi(Coef3 c, double* __restrict__ stat) {
    const int64_t o = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (o >= c.n) return;
    Nb nb;
    neighbours(c, o, nb);
    const double* psi = stat + c.pitch;
    double s = 0.0;
#pragma unroll
    for (int i = 1; i < Q; ++i) s += wfd(i) * (psi[nb.o[i]] - psi[o]);
    stat[2 * c.pitch + o] = 6.0 * s;
}

// ------------------------------------------------------ per-step kernels
// Order parameter of the current level: phi = phi_hist + (g_0 - phi_hist)
// + sum of the moving g_i.
template <class T>
__global__ __launch_bounds__(NT) void k3_phi(Coef3 c, Planes3<T> P, int cur) {
    const int64_t o = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (o >= c.n) return;
    const T* g = P.pop[cur];
    double s = (double)P.hist[cur][o] + (double)g[o];
#pragma unroll
    for (int i = 1; i < Q; ++i) s += (double)g[(int64_t)i * c.pitch + o];
    P.phi[o] = s;
}

// Eq. (potential): mu = (3 sigma/D) phi (phi^2 - 1) - (3 D sigma/8) lap phi
// + (9 sigma/D) phi0^2 phi + (3 sigma/D) psi (3 phi^2 + phi0^2 - 1)
// - (3 D sigma/8) lap psi, at one node from phi at x + c_i (phi_at(i); i = 0:
// the node) and the node's statics phi0, psi, lap psi.
template <class F>
__device__ __forceinline__ double mu_of(const Coef3& c, F phi_at, double z, double q, double lq) {
    const double f = phi_at(0);
    double lap = 0.0;
#pragma unroll
    for (int i = 1; i < Q; ++i) lap += wfd(i) * (phi_at(i) - f);
    lap *= 6.0;
    const double a = 3.0 * c.sigma / c.Dw, b = 3.0 * c.Dw * c.sigma / 8.0;
    return a * f * (f - 1.0) * (f + 1.0) - b * lap + 3.0 * a * z * z * f + a * q * (3.0 * f * f + z * z - 1.0) - b * lq;
}

// Consistent mass flux S = M grad(mu) (rho1 - rho2)/2 at one node from mu at
// its neighbours (mu_at(i): mu at x + c_i); every kernel that forms S uses
// this, so the sums and their order are the same wherever S is formed.
template <class F>
__device__ __forceinline__ void flux_of(const Coef3& c, F mu_at, double S[3]) {
    double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const double v = wfd(i) * mu_at(i);
        gx += cxv(i) * v;
        gy += cyv(i) * v;
        gz += czv(i) * v;
    }
    const double k = 3.0 * c.Mob * (c.rho1 - c.rho2) * 0.5;
    S[0] = k * gx;
    S[1] = k * gy;
    S[2] = k * gz;
}

// S planes of the current level (for creation and the output pass; the
// marching node update forms S itself)
template <class T>
__global__ __launch_bounds__(NT) void k3_flux(Coef3 c, Planes3<T> P) {
    const int64_t o = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (o >= c.n) return;
    Nb nb;
    neighbours(c, o, nb);
    double S[3];
    flux_of(c, [&](int i) { return P.mu[nb.o[i]]; }, S);
    P.S[o] = S[0];
    P.S[c.pitch + o] = S[1];
    P.S[2 * c.pitch + o] = S[2];
}

enum { M3_STEP = 0, M3_OUT = 1 };

// Block sum of NPART3 values in a fixed order (deterministic), thread 0 of
// the block writes them.
__device__ void block_sums(double v[NPART3], double* out) {
    __shared__ double red[NPART3][NT];
#pragma unroll
    for (int k = 0; k < NPART3; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int k = 0; k < NPART3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NPART3; ++k) out[(int64_t)blockIdx.x * NPART3 + k] = red[k][0];
}

// sum_i c_i v_i over the nonzero components of a lattice velocity (the
// unrolled loops fold it to additions and negations: -0 + v is v exactly)
template <class R>
__device__ __forceinline__ R cdot(int cx, int cy, int cz, const R v[3]) {
    R s = R(-0.0);
    if (cx) s = cx > 0 ? s + v[0] : s - v[0];
    if (cy) s = cy > 0 ? s + v[1] : s - v[1];
    if (cz) s = cz > 0 ? s + v[2] : s - v[2];
    return s;
}


// Neighbour values of the current level at x + c_i (i = 0: the node
// itself): the order parameter, the mass flux S and the lagged velocity,
// from the planes (NbPlanes) or from the slices a marching block holds in LDS
// (NbLds).
template <class T>
struct NbPlanes {
    const double* phi;
    const double* S;
    const T* u;  // history plane of u_x; u_y and u_z follow at pitch strides
    int64_t pt;
    __device__ __forceinline__ double ph(int i, const Nb& nb) const { return phi[nb.o[i]]; }
    __device__ __forceinline__ double s(int i, int k, const Nb& nb) const { return (double)S[k * pt + nb.o[i]]; }
    __device__ __forceinline__ T v(int i, int k, const Nb& nb) const { return u[k * pt + nb.o[i]]; }
};

constexpr int MX = 64, MY = NT / MX, MZ = 16;  // marching column and slices per block
constexpr int MW = MX + 2, MP = MW * (MY + 2);  // LDS slice with the one-node ring
constexpr int MW2 = MX + 4, MP2 = MW2 * (MY + 4);  // with the two-node ring

template <class T>
struct NbLds {
    const double* phi[3];  // slices z - 1, z, z + 1
    const double* S[3];     // [3][MP] each
    const T* u[3];
    int q;                 // the node's index in its slice
    __device__ __forceinline__ int at(int i) const { return q + cyv(i) * MW + cxv(i); }
    __device__ __forceinline__ double ph(int i, const Nb&) const { return phi[czv(i) + 1][at(i)]; }
    __device__ __forceinline__ double s(int i, int k, const Nb&) const { return S[czv(i) + 1][k * MP + at(i)]; }
    __device__ __forceinline__ T v(int i, int k, const Nb&) const { return u[czv(i) + 1][k * MP + at(i)]; }
};

// Node update of the current level (steps 4-6 and 2 of the procedure):
// grad phi, grad rho, F_c, F, u*, the solid force, u, P, then in M3_STEP
// both collisions, the push into the other copy and the history of this
// level; in M3_OUT phi, u, P and the reductions.
// The phase-field collision acts on g with g_0 taken relative to the
// history order parameter (g_0 - phi_hist, as it is stored): the moments of
// g then differ from those of the full g by phi_hist times the Hermite rows
// at the rest velocity, which the equilibria below subtract as well.
template <class T, int MODE, class NbA>
__device__ __forceinline__ void node_body(const Coef3& c, const Planes3<T>& P, int cur, int64_t o,
                                          const Nb& nb, const NbA& A, double red[NPART3]) {
    using R = double;  // FP64 arithmetic for either storage
    const int64_t pt = c.pitch;
    const T* H = P.hist[cur];
    const R cs2 = c.cs2;
    // ---- gradients of phi and rho (FP64), F_c = div(S u_lag - u_lag S)/2
    const double phd = A.ph(0, nb);
    double dpd[3] = {0.0, 0.0, 0.0}, drd[3] = {0.0, 0.0, 0.0};
    R fc[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const double wi = wfd(i);
        const double pn = A.ph(i, nb), rn = rho_of(c, pn);
        const int ci[3] = {cxv(i), cyv(i), czv(i)};
        const R Sn[3] = {A.s(i, 0, nb), A.s(i, 1, nb), A.s(i, 2, nb)};
        const R un[3] = {A.v(i, 0, nb), A.v(i, 1, nb), A.v(i, 2, nb)};
        const R cS = cdot(ci[0], ci[1], ci[2], Sn);
        const R cu = cdot(ci[0], ci[1], ci[2], un);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if (ci[b]) {
                dpd[b] += (ci[b] > 0 ? wi : -wi) * pn;
                drd[b] += (ci[b] > 0 ? wi : -wi) * rn;
            }
            fc[b] += R(wi) * (cS * un[b] - cu * Sn[b]);
        }
    }
    R dp[3], dr[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        dpd[b] *= 3.0;
        dp[b] = (R)dpd[b];
        dr[b] = (R)(3.0 * drd[b]);
        fc[b] *= R(1.5);  // 3 (1/c_s^2) x 1/2
    }
    const R ph = (R)phd;
    const R rho = rho_of(c, ph);
    const R mu = (R)P.mu[o];
    const R S[3] = {A.s(0, 0, nb), A.s(0, 1, nb), A.s(0, 2, nb)};
    const R z = (R)P.stat[o];
    const R F[3] = {mu * dp[0] + (rho - c.rho_ref) * c.gx + (R(1) - z) * c.fbx + fc[0],
                    mu * dp[1] + (rho - c.rho_ref) * c.gy + (R(1) - z) * c.fby + fc[1],
                    mu * dp[2] + (rho - c.rho_ref) * c.gz + (R(1) - z) * c.fbz + fc[2]};
    // ---- history of the previous level
    const T php = H[o];
    const R up[3] = {A.v(0, 0, nb), A.v(0, 1, nb), A.v(0, 2, nb)};
    const R Sp[3] = {H[4 * pt + o], H[5 * pt + o], H[6 * pt + o]};
    // ---- flow populations and their Hermite moments
    const T* gp = P.pop[cur];
    const T* fp = gp + (int64_t)Q * pt;
    R f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = fp[(int64_t)i * pt + o];
    // ---- viscosity: nu = (1/s2a - 1/2)(1 - c_s^2)/2 = (1/s2b - 1/2) c_s^2
    R om = R(1) - z;
    om = om < c.solid_eps ? c.solid_eps : om;
    const R nu = muv_of(c, ph) / (rho * om);
    const R ta = nu / ((R(1) - cs2) * R(0.5)) + R(0.5), tb = nu / cs2 + R(0.5);
    const R s2a = R(1) / ta, s2b = R(1) / tb;
    // ---- u*, solid force, u, P (Eqs. uStar, u)
    R us[3], af[3], u[3];
    if (c.first) {
#pragma unroll
        for (int b = 0; b < 3; ++b) us[b] = up[b];
    } else {
        const R j[3] = {(f[1] - f[4]) + (((f[7] - f[8]) + (f[9] - f[10])) + ((f[11] - f[12]) + (f[13] - f[14]))),
            (f[2] - f[5]) + (((f[7] + f[8]) - (f[9] + f[10])) + ((f[11] + f[12]) - (f[13] + f[14]))),
            (f[3] - f[6]) + (((f[7] + f[8]) + (f[9] + f[10])) - ((f[11] + f[12]) + (f[13] + f[14])))};
#pragma unroll
        for (int b = 0; b < 3; ++b) us[b] = (j[b] + R(0.5) * F[b]) / rho;
    }
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        af[b] = -z * us[b];  // phi0 (u_s - u*) with u_s = 0
        u[b] = c.first ? us[b] : us[b] + R(0.5) * af[b];
    }
    const R udr = u[0] * dr[0] + u[1] * dr[1] + u[2] * dr[2];
    const R Su = S[0] * u[0] + S[1] * u[1] + S[2] * u[2];
    const R q = rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) - Su;
    const R rhop = rho_of(c, (R)php);
    const R qp = rhop * (up[0] * up[0] + up[1] * up[1] + up[2] * up[2]) -
                 (Sp[0] * up[0] + Sp[1] * up[1] + Sp[2] * up[2]);
    R Pr = R(0);
    if (!c.first) {
        R sum = f[1];
#pragma unroll
        for (int i = 2; i < Q; ++i) sum += f[i];
        // H = -2 K (1 - 3 d0)(1/s2a - 1/2) (the printed 3-D factor with s0 = s2a)
        const R Hf = R(-2) * c.K * (R(1) - R(3) * cs2) * (ta - R(0.5));
        Pr = cs2 / (R(1) - c.w[0]) * (sum + (R(0.5) + Hf) * udr - c.w[0] * q / (R(1) - cs2) + R(0.5) * c.K * (q - qp));
    }
    if (MODE == M3_OUT) {
        double* out = P.out;
        const double ud[3] = {(double)u[0], (double)u[1], (double)u[2]};
        out[o] = phd;
        out[pt + o] = ud[0];
        out[2 * pt + o] = ud[1];
        out[3 * pt + o] = ud[2];
        out[4 * pt + o] = (double)Pr;
        // Eq. (2energy) with psi; grad psi from the static plane
        const double* psi = P.stat + pt;
        double gq[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const double v = wfd(i) * psi[nb.o[i]];
            gq[0] += cxv(i) * v;
            gq[1] += cyv(i) * v;
            gq[2] += czv(i) * v;
        }
        const double zd = P.stat[o], qq = psi[o], s = c.sigma, D = c.Dw;
        const double g2 = dpd[0] * dpd[0] + dpd[1] * dpd[1] + dpd[2] * dpd[2];
        const double gpq = 3.0 * (gq[0] * dpd[0] + gq[1] * dpd[1] + gq[2] * dpd[2]);
        red[0] = phd;
        red[1] = 3.0 * s / (4.0 * D) * (1.0 - phd) * (1.0 - phd) * (1.0 + phd) * (1.0 + phd) + 3.0 * D * s / 16.0 * g2 +
                 9.0 * s / (2.0 * D) * zd * zd * phd * phd + 3.0 * s / D * qq * phd * (phd * phd + zd * zd - 1.0) +
                 3.0 * D * s / 8.0 * gpq;
        red[2] = 0.5 * (double)rho * (ud[0] * ud[0] + ud[1] * ud[1] + ud[2] * ud[2]);
        red[3] = (fin(phd) && fin(ud[0]) && fin(ud[1]) && fin(ud[2]) && fin((double)Pr)) ? 0.0 : 1.0;
    } else {
        const int nxt = cur ^ 1;
        T* gn = P.pop[nxt];
        T* fn = gn + (int64_t)Q * pt;
        // ---- flow collision in Hermite moments: dm_k = -s_k (m_k - m_k^eq) + (1 - s_k/2) F_k,
        // f* = f + w_i sum_k H_k(c_i) dm_k / |H_k|^2
        const int A6[6] = {0, 1, 2, 0, 0, 1}, B6[6] = {0, 1, 2, 1, 2, 2};
        R M2[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int ka = A6[k], kb = B6[k];
            const R T_now = R(0.5) * (S[ka] * u[kb] + u[ka] * S[kb]);
            const R T_old = R(0.5) * (Sp[ka] * up[kb] + up[ka] * Sp[kb]);
            M2[k] = (u[ka] * F[kb] + F[ka] * u[kb]) - (T_now - T_old) + cs2 * (u[ka] * dr[kb] + dr[ka] * u[kb]) +
                    (ka == kb ? (R(1) - R(3) * cs2) * udr : R(0));
        }
        R m[Q];
        moments15(f, cs2, m);
        R meq[Q], src[Q], rate[Q];
        meq[0] = R(0);
        src[0] = udr;
        rate[0] = s2a;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            meq[1 + b] = rho * u[b];
            src[1 + b] = F[b] + rho * af[b];
            rate[1 + b] = c.s1;
            meq[4 + b] = Pr + rho * u[b] * u[b] - S[b] * u[b];
            src[4 + b] = M2[b];
            rate[4 + b] = s2a;
        }
        meq[7] = rho * u[0] * u[1] - R(0.5) * (S[0] * u[1] + u[0] * S[1]);
        meq[8] = rho * u[0] * u[2] - R(0.5) * (S[0] * u[2] + u[0] * S[2]);
        meq[9] = rho * u[1] * u[2] - R(0.5) * (S[1] * u[2] + u[1] * S[2]);
        src[7] = M2[3];
        src[8] = M2[4];
        src[9] = M2[5];
        rate[7] = rate[8] = rate[9] = s2b;
#pragma unroll
        for (int k = 10; k < 14; ++k) {
            meq[k] = R(0);
            src[k] = R(0);
            rate[k] = c.s3;
        }
        meq[14] = R(-2) * cs2 * Pr;
        src[14] = R(0);
        rate[14] = s2a;
        R dm[Q];
#pragma unroll
        for (int k = 0; k < Q; ++k)
            dm[k] = (-rate[k] * (m[k] - meq[k]) + (R(1) - R(0.5) * rate[k]) * src[k]) * c.inv_norm[hcls(k)];
        R df[Q];
        inverse15(dm, cs2, df);
#pragma unroll
        for (int i = 0; i < Q; ++i) fn[(int64_t)i * pt + nb.o[i]] = f[i] + wgt(c, i) * df[i];
        // ---- phase-field collision (Sec. 3.1), g_0 relative to phi_hist
        R g[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) g[i] = gp[(int64_t)i * pt + o];
        R mg[Q];
        moments15(g, cs2, mg);
        const R em = c.eta * mu;
        const R dph = (R)(phd - (double)php);  // phi - phi_hist
        R geq[Q], gsrc[Q];
        geq[0] = dph;
        gsrc[0] = R(0);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            geq[1 + b] = ph * u[b];
            gsrc[1 + b] = ph * u[b] - php * up[b];  // d_t(phi u), backward difference
            geq[4 + b] = -cs2 * (dph - em);
            gsrc[4 + b] = R(0);
        }
#pragma unroll
        for (int k = 7; k < 14; ++k) {
            geq[k] = R(0);
            gsrc[k] = R(0);
        }
        geq[14] = R(2) * cs2 * cs2 * (dph - em);
        gsrc[14] = R(0);
#pragma unroll
        for (int k = 0; k < Q; ++k)
            dm[k] = c.gA[hcls(k)] * (mg[k] - geq[k]) + (hcls(k) == 1 ? c.gB1 * gsrc[k] : R(0));
        const T phs = (T)phd;  // the history value g_0 is stored against
        R dg[Q];
        inverse15(dm, cs2, dg);
        gn[o] = g[0] + wgt(c, 0) * dg[0] + (R)((double)php - (double)phs);
#pragma unroll
        for (int i = 1; i < Q; ++i) gn[(int64_t)i * pt + nb.o[i]] = g[i] + wgt(c, i) * dg[i];
        // ---- history of this level
        T* Hn = P.hist[nxt];
        Hn[o] = phs;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            Hn[(1 + b) * pt + o] = u[b];
            Hn[(4 + b) * pt + o] = S[b];
        }
    }
}

template <class T, int MODE>
__global__ __launch_bounds__(NT) void k3_node(Coef3 c, Planes3<T> P, int cur) {
    const int64_t o = (int64_t)blockIdx.x * NT + threadIdx.x;
    double red[NPART3] = {0.0, 0.0, 0.0, 0.0};
    if (o < c.n) {
        Nb nb;
        neighbours(c, o, nb);
        const NbPlanes<T> A{P.phi, P.S, P.hist[cur] + c.pitch, c.pitch};
        node_body<T, MODE>(c, P, cur, o, nb, A, red);
    }
    if (MODE == M3_OUT) block_sums(red, P.part);
}

// The node update marching along z: a block owns an MX x MY column of nodes
// over MZ slices and keeps three slices (z - 1, z, z + 1) of the order
// parameter, S and the lagged velocity on the column and its one-node ring in
// LDS, loading one new slice per step along z.  S is formed here, on the ring
// of each new slice, from three slices of mu on the two-node ring (also in
// LDS), with the sums k3_flux makes.  Every value the node update reads is
// the one k3_node would read; only where it comes from differs.
// Blocks are dealt to the 8 XCDs in turn; this renumbering gives each XCD a
// contiguous range of the columns, so that the columns sharing ring rows run
// on one XCD and meet in its L2.
__device__ __forceinline__ int xcd_slab(int b, int G) {
    const int q = G >> 3, r = G & 7;
    const int k = b & 7, j = b >> 3;
    return k * q + (k < r ? k : r) + j;
}

// In-slice offset of point p of a w-wide LDS slice holding a column at
// (x0, y0) with its h-node ring, periodic; columns and rows past the ring a
// ragged or narrow column needs are clamped into the grid and never read.
__device__ __forceinline__ int ring_offset(const Coef3& c, int x0, int y0, int p, int w, int h) {
    int gx = x0 + p % w - h, gy = y0 + p / w - h;
    gx = gx < 0 ? gx + c.nx : (gx >= c.nx ? gx - c.nx : gx);
    gy = gy < 0 ? gy + c.ny : (gy >= c.ny ? gy - c.ny : gy);
    gx = gx < c.nx ? gx : c.nx - 1;
    gy = gy < c.ny ? gy : c.ny - 1;
    return gy * c.nx + gx;
}

// mu planes of the current level, marching along z over the columns of
// k3_march with three slices of phi and their one-node ring in LDS.
template <class T>
__global__ __launch_bounds__(NT) void k3_mu(Coef3 c, Planes3<T> P, int ntx, int nty) {
    __shared__ double s_phi[3][MP];
    int b = xcd_slab((int)blockIdx.x, (int)gridDim.x);
    const int tx = b % ntx;
    b /= ntx;
    const int ty = b % nty;
    const int z0 = (b / nty) * MZ;
    const int z1 = z0 + MZ < c.nz ? z0 + MZ : c.nz;
    const int x0 = tx * MX, y0 = ty * MY;
    const int t = threadIdx.x;
    const int x = x0 + (t % MX), y = y0 + t / MX;
    const bool in = x < c.nx && y < c.ny;
    int off[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) off[r] = ring_offset(c, x0, y0, t + r * NT < MP ? t + r * NT : MP - 1, MW, 1);
    auto load = [&](int s) {  // phi of slice s into slot (s - z0 + 1) % 3
        const int slot = (s - z0 + 1) % 3;
        const int zz = s < 0 ? s + c.nz : (s >= c.nz ? s - c.nz : s);
        const int64_t base = (int64_t)zz * c.nx * c.ny;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int p = t + r * NT;
            if (p < MP) s_phi[slot][p] = P.phi[base + off[r]];
        }
    };
    load(z0 - 1);
    load(z0);
    const int q = (t / MX + 1) * MW + (t % MX) + 1;
    for (int k = 0; z0 + k < z1; ++k) {
        const int z = z0 + k;
        __syncthreads();  // the slot written next is no longer read
        load(z + 1);
        __syncthreads();
        if (in) {
            const int64_t o = ((int64_t)z * c.ny + y) * c.nx + x, pt = c.pitch;
            const double* sl[3] = {s_phi[k % 3], s_phi[(k + 1) % 3], s_phi[(k + 2) % 3]};
            P.mu[o] = mu_of(c, [&](int i) { return sl[czv(i) + 1][q + cyv(i) * MW + cxv(i)]; }, P.stat[o],
                            P.stat[pt + o], P.stat[2 * pt + o]);
        }
    }
}

template <class T>
__global__ __launch_bounds__(NT) void k3_march(Coef3 c, Planes3<T> P, int cur, int ntx, int nty) {
    __shared__ double s_phi[3][MP];
    __shared__ double s_S[3][3 * MP];
    __shared__ T s_u[3][3 * MP];
    __shared__ double s_mu[3][MP2];
    int b = xcd_slab((int)blockIdx.x, (int)gridDim.x);
    const int tx = b % ntx;
    b /= ntx;
    const int ty = b % nty;
    const int z0 = (b / nty) * MZ;
    const int z1 = z0 + MZ < c.nz ? z0 + MZ : c.nz;
    const int x0 = tx * MX, y0 = ty * MY;
    const int t = threadIdx.x;
    const int x = x0 + (t % MX), y = y0 + t / MX;
    const bool in = x < c.nx && y < c.ny;
    const int64_t pt = c.pitch;
    const T* U = P.hist[cur] + pt;
    // in-slice offsets of the ring points this thread loads: the one-node
    // ring (two rounds) and the two-node ring (three rounds); columns and rows
    // past the ring a ragged or narrow tile needs are clamped into the grid
    // and never read
    auto ring_off = [&](int p, int w, int h) { return ring_offset(c, x0, y0, p, w, h); };
    int off[2], off2[3];
#pragma unroll
    for (int r = 0; r < 2; ++r) off[r] = ring_off(t + r * NT < MP ? t + r * NT : MP - 1, MW, 1);
#pragma unroll
    for (int r = 0; r < 3; ++r) off2[r] = ring_off(t + r * NT < MP2 ? t + r * NT : MP2 - 1, MW2, 2);
    auto wrapz = [&](int zz) { return zz < 0 ? zz + c.nz : (zz >= c.nz ? zz - c.nz : zz); };
    // slots: phi, S and u of slice s in (s - z0 + 1) % 3, mu of slice s in (s - z0 + 3) % 3
    auto load = [&](int s) {
        const int slot = (s - z0 + 1) % 3;
        const int64_t base = (int64_t)wrapz(s) * c.nx * c.ny;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int p = t + r * NT;
            if (p < MP) {
                const int64_t n = base + off[r];
                s_phi[slot][p] = P.phi[n];
#pragma unroll
                for (int k = 0; k < 3; ++k) s_u[slot][k * MP + p] = U[k * pt + n];
            }
        }
    };
    auto load_mu = [&](int s) {
        const int slot = (s - z0 + 3) % 3;
        const int64_t base = (int64_t)wrapz(s) * c.nx * c.ny;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const int p = t + r * NT;
            if (p < MP2) s_mu[slot][p] = P.mu[base + off2[r]];
        }
    };
    auto flux = [&](int s) {  // S of slice s on the ring, from mu of slices s - 1, s, s + 1
        const double* m3[3] = {s_mu[(s - z0 + 2) % 3], s_mu[(s - z0 + 3) % 3], s_mu[(s - z0 + 4) % 3]};
        double* S = s_S[(s - z0 + 1) % 3];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int p = t + r * NT;
            if (p < MP) {
                const int q2 = (p / MW + 1) * MW2 + (p % MW) + 1;
                double v[3];
                flux_of(c, [&](int i) { return m3[czv(i) + 1][q2 + cyv(i) * MW2 + cxv(i)]; }, v);
#pragma unroll
                for (int k = 0; k < 3; ++k) S[k * MP + p] = v[k];
            }
        }
    };
    load(z0 - 1);
    load(z0);
    load_mu(z0 - 2);
    load_mu(z0 - 1);
    load_mu(z0);
    __syncthreads();
    flux(z0 - 1);
    __syncthreads();
    load_mu(z0 + 1);  // into the slot of z0 - 2
    __syncthreads();
    flux(z0);
    double red[NPART3];
    for (int k = 0; z0 + k < z1; ++k) {
        const int z = z0 + k;
        __syncthreads();  // the slots written next are no longer read
        load(z + 1);
        load_mu(z + 2);
        __syncthreads();
        flux(z + 1);
        __syncthreads();
        if (in) {
            Nb nb;
            neighbours_xyz(c, x, y, z, nb);
            const int q = (t / MX + 1) * MW + (t % MX) + 1;
            const int sm = k % 3, s0 = (k + 1) % 3, sp = (k + 2) % 3;
            const NbLds<T> A{{s_phi[sm], s_phi[s0], s_phi[sp]}, {s_S[sm], s_S[s0], s_S[sp]}, {s_u[sm], s_u[s0], s_u[sp]}, q};
            node_body<T, M3_STEP>(c, P, cur, ((int64_t)z * c.ny + y) * c.nx + x, nb, A, red);
        }
    }
}

// Equilibria of the initial state (procedure step 1): g = g^eq(phi, mu, u),
// f = f^eq(P = 0, rho, u, S), history = (phi, u, S); u from the staged input.
template <class T>
__global__ __launch_bounds__(NT) void k3_equilibrium(Coef3 c, Planes3<T> P, const double* __restrict__ uin) {
    const int64_t o = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (o >= c.n) return;
    const int64_t pt = c.pitch;
    const double cs2 = c.cs2;
    const double ph = P.phi[o], rho = rho_of(c, ph), em = c.eta * P.mu[o];
    const double u[3] = {uin[o], uin[pt + o], uin[2 * pt + o]};
    const double S[3] = {P.S[o], P.S[pt + o], P.S[2 * pt + o]};
    T* g = P.pop[0];
    T* f = g + (int64_t)Q * pt;
    const T phs = (T)ph;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double ci[3] = {(double)cxv(i), (double)cyv(i), (double)czv(i)};
        const double w = wgt(c, i);
        const double cu = ci[0] * u[0] + ci[1] * u[1] + ci[2] * u[2];
        // Sec. 3.1
        const double gi = (i == 0 ? ph + (w - 1.0) * em : w * em) + w * ph * cu / cs2;
        // Sec. 3.2 with P = 0
        double diag = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) diag += (ci[a] * ci[a] - cs2) * (rho * u[a] * u[a] - S[a] * u[a]);
        diag /= cs2 - cs2 * cs2;
        const double off = (ci[0] * ci[1] * (rho * u[0] * u[1] - 0.5 * (S[0] * u[1] + u[0] * S[1])) +
                            ci[0] * ci[2] * (rho * u[0] * u[2] - 0.5 * (S[0] * u[2] + u[0] * S[2])) +
                            ci[1] * ci[2] * (rho * u[1] * u[2] - 0.5 * (S[1] * u[2] + u[1] * S[2]))) /
                           (cs2 * cs2);
        const double fi = w * rho * cu / cs2 + w * (diag + off);
        g[(int64_t)i * pt + o] = (T)(i == 0 ? gi - (double)phs : gi);
        f[(int64_t)i * pt + o] = (T)fi;
    }
    T* H = P.hist[0];
    H[o] = phs;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        H[(1 + a) * pt + o] = (T)u[a];
        H[(4 + a) * pt + o] = (T)S[a];
    }
}

}  // namespace lbm3

using namespace lbm3;

struct lbm3_domain {
    lbm3_params p{};
    Coef3 c{};
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    int cur = 0;
    int64_t steps = 0;
    int64_t blocks = 0;
    int64_t timed_steps = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    size_t off_pop[2]{}, off_hist[2]{}, off_stat = 0, off_phi = 0, off_mu = 0, off_S = 0, off_out = 0, off_part = 0;
};

namespace {

thread_local std::string g_err3;

int fail3(int code, const std::string& msg) {
    g_err3 = msg;
    return code;
}

#define HIPCHK3(x)                                                                         \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            return fail3(LBM_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));      \
    } while (0)

size_t up256(size_t v) { return (v + 255) / 256 * 256; }

int validate3(const lbm3_params* p) {
    if (!p) return fail3(LBM_EINVAL, "params is NULL");
    if (p->nx < 3 || p->ny < 3 || p->nz < 3) return fail3(LBM_EINVAL, "nx, ny, nz must be >= 3");
    if ((int64_t)p->nx * p->ny * p->nz > (int64_t)1 << 31) return fail3(LBM_EINVAL, "more than 2^31 nodes");
    if (p->storage != LBM_STORE_FP64 && p->storage != LBM_STORE_FP32)
        return fail3(LBM_EUNSUPPORTED, "3-D storage must be LBM_STORE_FP64 or LBM_STORE_FP32");
    const double v[] = {p->d0, p->sigma, p->D, p->M, p->rho1, p->rho2, p->mu1, p->mu2, p->tau_phi, p->s0, p->s1,
                        p->s2, p->s3, p->s4, p->gx, p->gy, p->gz, p->rho_ref, p->fbx, p->fby, p->fbz, p->solid_eps};
    for (double x : v)
        if (!std::isfinite(x)) return fail3(LBM_EINVAL, "non-finite parameter");
    if (!(p->d0 > 0.0 && p->d0 < 0.5)) return fail3(LBM_EINVAL, "d0 must be in (0, 1/2)");
    if (!(p->D > 0.0) || !(p->M > 0.0) || !(p->sigma >= 0.0)) return fail3(LBM_EINVAL, "D, M must be > 0, sigma >= 0");
    if (!(p->rho1 > 0.0 && p->rho2 > 0.0 && p->mu1 > 0.0 && p->mu2 > 0.0))
        return fail3(LBM_EINVAL, "densities and viscosities must be > 0");
    if (!(p->tau_phi > 0.5)) return fail3(LBM_EINVAL, "tau_phi must be > 1/2");
    const double s[] = {p->s0, p->s1, p->s2, p->s3, p->s4};
    for (double x : s)
        if (!(x > 0.0 && x < 2.0)) return fail3(LBM_EINVAL, "relaxation rates must be in (0, 2)");
    if (!(p->solid_eps > 0.0 && p->solid_eps <= 1.0)) return fail3(LBM_EINVAL, "solid_eps must be in (0, 1]");
    return LBM_OK;
}

struct Sizes3 {
    int64_t n, pitch, blocks;
    size_t pop, hist, total;
    size_t off_pop[2], off_hist[2], off_stat, off_phi, off_mu, off_S, off_out, off_part;
};

Sizes3 sizes3(const lbm3_params& p) {
    Sizes3 s{};
    s.n = (int64_t)p.nx * p.ny * p.nz;
    s.pitch = (s.n + 63) / 64 * 64;
    s.blocks = (s.n + NT - 1) / NT;
    const size_t r = p.storage == LBM_STORE_FP64 ? 8 : 4;
    s.pop = up256((size_t)2 * Q * s.pitch * r);
    s.hist = up256((size_t)7 * s.pitch * r);
    size_t o = 0;
    for (int k = 0; k < 2; ++k) { s.off_pop[k] = o; o += s.pop; }
    for (int k = 0; k < 2; ++k) { s.off_hist[k] = o; o += s.hist; }
    s.off_stat = o; o += up256((size_t)3 * s.pitch * 8);
    s.off_phi = o; o += up256((size_t)s.pitch * 8);
    s.off_mu = o; o += up256((size_t)s.pitch * 8);
    s.off_S = o; o += up256((size_t)3 * s.pitch * 8);
    s.off_out = o; o += up256((size_t)5 * s.pitch * 8);
    s.off_part = o; o += up256((size_t)s.blocks * NPART3 * 8);
    s.total = o;
    return s;
}

void fill_coef3(const lbm3_params& p, const Sizes3& z, Coef3& c) {
    const double d0 = p.d0, cs2 = d0;
    c.nx = p.nx; c.ny = p.ny; c.nz = p.nz; c.first = 1;
    c.pitch = z.pitch; c.n = z.n;
    c.cs2 = cs2;
    c.w[0] = (1.0 - d0) * (1.0 - 2.0 * d0);
    c.w[1] = (d0 - d0 * d0) / 2.0;
    c.w[2] = d0 * d0 / 8.0;
    c.K = 1.0 - 2.0 * d0;
    c.eta = p.M / ((p.tau_phi - 0.5) * cs2);  // M = (1/s_1phi - 1/2) eta c_s^2
    c.sigma = p.sigma; c.Dw = p.D; c.Mob = p.M;
    c.rho1 = p.rho1; c.rho2 = p.rho2; c.mu1 = p.mu1; c.mu2 = p.mu2;
    c.gx = p.gx; c.gy = p.gy; c.gz = p.gz; c.rho_ref = p.rho_ref;
    c.fbx = p.fbx; c.fby = p.fby; c.fbz = p.fbz; c.solid_eps = p.solid_eps;
    const double s1p = 1.0 / p.tau_phi;
    const double sg[Q] = {p.s0, s1p, s1p, s1p, p.s2, p.s2, p.s2, p.s2, p.s2, p.s2, p.s3, p.s3, p.s3, p.s3, p.s4};
    c.s1 = p.s1; c.s3 = p.s3;
    // norms of the Hermite rows under the weights, one row per class (the
    // others of a class are its images under the lattice's symmetries)
    const int first_of_class[7] = {0, 1, 4, 7, 10, 13, 14};
    for (int j = 0; j < 7; ++j) {
        const int k = first_of_class[j];
        double s = 0.0;
        for (int i = 0; i < Q; ++i) {
            const double w = i == 0 ? c.w[0] : (i <= 6 ? c.w[1] : c.w[2]);
            const double h = hrow(k, cxv(i), cyv(i), czv(i), cs2);
            s += w * h * h;
        }
        c.inv_norm[j] = 1.0 / s;
        c.gA[j] = -sg[k] * c.inv_norm[j];
    }
    c.gB1 = (1.0 - 0.5 * sg[1]) * c.inv_norm[1];
}

template <class T>
Planes3<T> planes(lbm3_domain* d) {
    Planes3<T> P{};
    for (int k = 0; k < 2; ++k) {
        P.pop[k] = (T*)(d->ws + d->off_pop[k]);
        P.hist[k] = (T*)(d->ws + d->off_hist[k]);
    }
    P.stat = (double*)(d->ws + d->off_stat);
    P.phi = (double*)(d->ws + d->off_phi);
    P.mu = (double*)(d->ws + d->off_mu);
    P.S = (double*)(d->ws + d->off_S);
    P.out = (double*)(d->ws + d->off_out);
    P.part = (double*)(d->ws + d->off_part);
    return P;
}

// the marching kernels' grid: MX x MY columns of MZ slices
struct March {
    int ntx, nty, nzc;
    dim3 grid() const { return dim3((unsigned)((int64_t)ntx * nty * nzc)); }
};
March march(const Coef3& c) { return March{(c.nx + MX - 1) / MX, (c.ny + MY - 1) / MY, (c.nz + MZ - 1) / MZ}; }

// phi of the current level from the populations, then mu, and S unless the
// marching node update forms it
template <class T>
int fields3(lbm3_domain* d, bool with_S) {
    Planes3<T> P = planes<T>(d);
    const dim3 g((unsigned)d->blocks), b(NT);
    const March m = march(d->c);
    hipLaunchKernelGGL(k3_phi<T>, g, b, 0, d->stream, d->c, P, d->cur);
    hipLaunchKernelGGL(k3_mu<T>, m.grid(), b, 0, d->stream, d->c, P, m.ntx, m.nty);
    if (with_S) hipLaunchKernelGGL(k3_flux<T>, g, b, 0, d->stream, d->c, P);
    HIPCHK3(hipGetLastError());
    return LBM_OK;
}

template <class T>
int step3(lbm3_domain* d, int64_t nsteps) {
    HIPCHK3(hipEventRecord(d->ev0, d->stream));
    for (int64_t s = 0; s < nsteps; ++s) {
        int rc = fields3<T>(d, false);
        if (rc) return rc;
        Planes3<T> P = planes<T>(d);
        const March m = march(d->c);
        hipLaunchKernelGGL(k3_march<T>, m.grid(), dim3(NT), 0, d->stream, d->c, P, d->cur, m.ntx, m.nty);
        HIPCHK3(hipGetLastError());
        d->cur ^= 1;
        d->c.first = 0;
        d->steps++;
    }
    HIPCHK3(hipEventRecord(d->ev1, d->stream));
    d->timed_steps = nsteps;
    return LBM_OK;
}

// macroscopic pass of the current level into `out` and the block sums
template <class T>
int out3(lbm3_domain* d, double res[NPART3]) {
    int rc = fields3<T>(d, true);
    if (rc) return rc;
    Planes3<T> P = planes<T>(d);
    hipLaunchKernelGGL((k3_node<T, M3_OUT>), dim3((unsigned)d->blocks), dim3(NT), 0, d->stream, d->c, P, d->cur);
    HIPCHK3(hipGetLastError());
    std::vector<double> part((size_t)d->blocks * NPART3);
    HIPCHK3(hipMemcpyAsync(part.data(), P.part, part.size() * 8, hipMemcpyDeviceToHost, d->stream));
    HIPCHK3(hipStreamSynchronize(d->stream));
    for (int k = 0; k < NPART3; ++k) res[k] = 0.0;
    for (int64_t b = 0; b < d->blocks; ++b)
        for (int k = 0; k < NPART3; ++k) res[k] += part[(size_t)b * NPART3 + k];
    return LBM_OK;
}

template <class T>
int create3(lbm3_domain* d, const double* phi, const double* phi0, const double* cth, const double* ux,
            const double* uy, const double* uz) {
    Planes3<T> P = planes<T>(d);
    const int64_t n = d->c.n, pt = d->c.pitch;
    const dim3 g((unsigned)d->blocks), b(NT);
    // stage: out[0] phi0, out[1] cos theta, out[2..4] u (FP64)
    double* st = P.out;
    std::vector<double> tmp((size_t)n, 0.0);
    HIPCHK3(hipMemcpyAsync(st, phi0, n * 8, hipMemcpyHostToDevice, d->stream));
    HIPCHK3(hipMemcpyAsync(st + pt, cth ? cth : tmp.data(), n * 8, hipMemcpyHostToDevice, d->stream));
    const double* us[3] = {ux, uy, uz};
    for (int a = 0; a < 3; ++a)
        HIPCHK3(hipMemcpyAsync(st + (2 + a) * pt, us[a] ? us[a] : tmp.data(), n * 8, hipMemcpyHostToDevice, d->stream));
    HIPCHK3(hipMemcpyAsync(P.phi, phi, n * 8, hipMemcpyHostToDevice, d->stream));
    hipLaunchKernelGGL(k3_static, g, b, 0, d->stream, d->c, (const double*)st, P.stat);
    hipLaunchKernelGGL(k3_lap_psi, g, b, 0, d->stream, d->c, P.stat);
    const March m = march(d->c);
    hipLaunchKernelGGL(k3_mu<T>, m.grid(), b, 0, d->stream, d->c, P, m.ntx, m.nty);
    hipLaunchKernelGGL(k3_flux<T>, g, b, 0, d->stream, d->c, P);
    hipLaunchKernelGGL(k3_equilibrium<T>, g, b, 0, d->stream, d->c, P, (const double*)(st + 2 * pt));
    HIPCHK3(hipGetLastError());
    HIPCHK3(hipStreamSynchronize(d->stream));  // tmp must outlive the copies
    d->cur = 0;
    d->c.first = 1;
    return LBM_OK;
}

template <class F>
int dispatch3(int storage, F&& f) {
    if (storage == LBM_STORE_FP64) return f(double{});
    return f(float{});
}

}  // namespace

extern "C" {

const char* lbm3_last_error(void) { return g_err3.c_str(); }

void lbm3_default_params(lbm3_params* p, int32_t nx, int32_t ny, int32_t nz) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->nx = nx; p->ny = ny; p->nz = nz;
    p->storage = LBM_STORE_FP64;
    p->d0 = 0.4; p->sigma = 1e-3; p->D = 4.0; p->M = 0.1;
    p->rho1 = p->rho2 = 1.0; p->mu1 = p->mu2 = 0.1;
    p->tau_phi = 1.0;
    p->s0 = p->s1 = p->s2 = p->s3 = p->s4 = 1.0;
    p->solid_eps = 0.01;
}

size_t lbm3_workspace_bytes(const lbm3_params* p) {
    if (validate3(p)) return 0;
    return sizes3(*p).total;
}

int lbm3_create(const lbm3_params* p, void* dev_workspace, size_t bytes, void* hip_stream, const double* phi,
                const double* phi0, const double* cos_theta, const double* ux, const double* uy, const double* uz,
                lbm3_domain** out) {
    if (!out) return fail3(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate3(p);
    if (rc) return rc;
    if (!phi || !phi0) return fail3(LBM_EINVAL, "phi and phi0 are required");
    if (!dev_workspace || ((uintptr_t)dev_workspace & 255)) return fail3(LBM_EINVAL, "workspace NULL or not 256-byte aligned");
    const Sizes3 z = sizes3(*p);
    if (bytes < z.total) return fail3(LBM_ENOMEM, "workspace too small: need " + std::to_string(z.total) + " bytes");
    for (int64_t o = 0; o < z.n; ++o) {
        if (!std::isfinite(phi[o]) || !std::isfinite(phi0[o]) || (cos_theta && !(std::fabs(cos_theta[o]) <= 1.0)) ||
            (ux && !std::isfinite(ux[o])) || (uy && !std::isfinite(uy[o])) || (uz && !std::isfinite(uz[o])))
            return fail3(LBM_EINVAL, "non-finite or out-of-range input at node " + std::to_string(o));
    }
    lbm3_domain* d = new lbm3_domain();
    d->p = *p;
    d->stream = (hipStream_t)hip_stream;
    d->ws = (char*)dev_workspace;
    d->blocks = z.blocks;
    for (int k = 0; k < 2; ++k) {
        d->off_pop[k] = z.off_pop[k];
        d->off_hist[k] = z.off_hist[k];
    }
    d->off_stat = z.off_stat; d->off_phi = z.off_phi; d->off_mu = z.off_mu; d->off_S = z.off_S;
    d->off_out = z.off_out; d->off_part = z.off_part;
    fill_coef3(*p, z, d->c);
    if (hipEventCreate(&d->ev0) != hipSuccess || hipEventCreate(&d->ev1) != hipSuccess) {
        lbm3_destroy(d);
        return fail3(LBM_EDEVICE, "hipEventCreate failed");
    }
    rc = dispatch3(p->storage, [&](auto s) { return create3<decltype(s)>(d, phi, phi0, cos_theta, ux, uy, uz); });
    if (rc) {
        lbm3_destroy(d);
        return rc;
    }
    *out = d;
    return LBM_OK;
}

int lbm3_step(lbm3_domain* d, int64_t nsteps) {
    if (!d) return fail3(LBM_EINVAL, "domain is NULL");
    if (nsteps < 0) return fail3(LBM_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return LBM_OK;
    return dispatch3(d->p.storage, [&](auto s) { return step3<decltype(s)>(d, nsteps); });
}

int lbm3_read(lbm3_domain* d, double* phi, double* ux, double* uy, double* uz, double* p) {
    if (!d) return fail3(LBM_EINVAL, "domain is NULL");
    return dispatch3(d->p.storage, [&](auto s) -> int {
        double res[NPART3];
        int rc = out3<decltype(s)>(d, res);
        if (rc) return rc;
        const double* o = (const double*)(d->ws + d->off_out);
        double* dst[5] = {phi, ux, uy, uz, p};
        for (int k = 0; k < 5; ++k)
            if (dst[k]) HIPCHK3(hipMemcpyAsync(dst[k], o + k * d->c.pitch, d->c.n * 8, hipMemcpyDeviceToHost, d->stream));
        HIPCHK3(hipStreamSynchronize(d->stream));
        if (res[3] > 0.0) return fail3(LBM_ENONFINITE, "non-finite phi, u or P at step " + std::to_string(d->steps));
        return LBM_OK;
    });
}

int lbm3_mass(lbm3_domain* d, double* sum_phi) {
    if (!d || !sum_phi) return fail3(LBM_EINVAL, "domain or sum_phi is NULL");
    return dispatch3(d->p.storage, [&](auto s) -> int {
        double res[NPART3];
        int rc = out3<decltype(s)>(d, res);
        if (rc) return rc;
        *sum_phi = res[0];
        return LBM_OK;
    });
}

int lbm3_energy(lbm3_domain* d, double* e_free, double* e_kin) {
    if (!d) return fail3(LBM_EINVAL, "domain is NULL");
    return dispatch3(d->p.storage, [&](auto s) -> int {
        double res[NPART3];
        int rc = out3<decltype(s)>(d, res);
        if (rc) return rc;
        if (e_free) *e_free = res[1];
        if (e_kin) *e_kin = res[2];
        return LBM_OK;
    });
}

double lbm3_last_step_ms(const lbm3_domain* d) {
    if (!d || d->timed_steps <= 0) return 0.0;
    if (hipEventSynchronize(d->ev1) != hipSuccess) return 0.0;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, d->ev0, d->ev1) != hipSuccess) return 0.0;
    return (double)ms / (double)d->timed_steps;
}

int lbm3_destroy(lbm3_domain* d) {
    if (!d) return LBM_OK;
    if (d->stream || d->ev1) (void)hipStreamSynchronize(d->stream);
    if (d->ev0) (void)hipEventDestroy(d->ev0);
    if (d->ev1) (void)hipEventDestroy(d->ev1);
    delete d;
    return LBM_OK;
}

}  // extern "C"
