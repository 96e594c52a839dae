// lbm_device.h -- device code for gfx950: the fused per-step kernel of the
// coupled D2Q9 phase-field / flow lattice Boltzmann method (Zhan, Liu, Chai &
// Shi, arXiv 2311.05097), its initialisation, read-out and reductions.
//
// Data layout in HBM (per domain, N = nx*ny nodes, row pitch nx, x fastest;
// every array padded to a multiple of 64 nodes, `pitch`):
//   pop[2]   two copies of the 18 distributions (ping-pong; step n reads
//            pop[n&1] and writes pop[(n+1)&1]).  Population i of a node is
//            stored at that node after streaming ("push": a node collides its
//            own post-stream populations and writes population i to the node
//            x + c_i of the other copy).
//   hist[2]  the previous time level phi, ux, uy, Sx, Sy (5 planes), also
//            ping-pong: step n reads hist[n&1] (level n-1), writes hist[(n+1)&1].
//   stat     phi0, psi = cos(theta) phi0 and its Laplacian (3 planes, static).
// Two copies are needed because the step kernel reads, besides each node's own
// populations, a 3-node halo of the order parameter that neighbouring tiles
// are updating in the same launch; an in-place (single-copy) update would race.
//
// Per step, one launch over 64 x TY tiles (64 x 4 tiles: 256 threads = 4
// wavefronts; taller tiles: 512 threads = 8 wavefronts, TileCfg):
//   A  phi = sum_i g_i on the tile plus a 3-node halo -> LDS
//   B  mu (Eq. potential) on tile + 2                 -> LDS
//   C  S = M (rho1-rho2)/2 grad mu and w = (S x u^{n-1})_z / 2 on tile + 1 -> LDS
//   D  per node: grad phi, F_c = (-d_y w, d_x w), F, u*, solid force, u, P
//      (Sec. 3.2), both Hermite-MRT collisions in moment space (Sec. 4), push
//      of the 18 post-collision values, history write.
// The same tile code in mode INIT builds the equilibria of procedure step 1,
// and in mode OUT recovers phi, u, P at the current level and accumulates
// per-tile FP64 partial sums for mass and energy.
#pragma once
#include <stdint.h>
#include <type_traits>

namespace lbm {

constexpr int TX = 64;        // tile width: one wavefront per row
constexpr int NT = 256;       // threads per block
constexpr int NWAVE = NT / 64;
constexpr int NPART = 4;      // partial sums per tile: mass, E_F, E_K, non-finite count
constexpr int FIX_BITS = 40;  // fixed point of the rest population g_0 (16-bit modes)

enum { MODE_STEP = 0, MODE_OUT = 1, MODE_INIT = 2 };

// Per-domain constants, in the arithmetic type R.
template <class R>
struct Coef {
    R a;                 // c_s^2 = d0 (c = 1)
    R one_a;             // 1 - d0
    R w0, w1, w2;        // weights of rest, axis and diagonal directions
    R inv_n1, inv_n2, inv_n11, inv_n12, inv_n22;  // 1 / Hermite norms
    R eta;               // M / ((tau_phi - 1/2) d0)
    R s0, s1, s1phi, s2, s3, s4;
    R k3s_D;             // 3 sigma / D
    R k3Ds_8;            // 3 D sigma / 8
    R k9s_D;             // 9 sigma / D
    R k3s_4D;            // 3 sigma / (4 D)     (energy)
    R k3Ds_16;           // 3 D sigma / 16      (energy)
    R k9s_2D;            // 9 sigma / (2 D)     (energy)
    R kS;                // M (rho1 - rho2) / 2
    R drho, rho2;        // (rho1 - rho2)/2, rho2: rho = rho2 + (rho1 - rho2)(1 + phi)/2
    R dmu, mu2;          // (mu1 - mu2)/2, mu2: the same law for the viscosity
    R gx, gy, rho_ref, fbx, fby;
    R solid_eps;
    R ka;                // (c^2 - c_s^2)/2 = (1 - d0)/2
    R Pfac;              // c_s^2 / (1 - w0)
    R Pw0;               // w0 / (c^2 - c_s^2)
    R K2;                // K / 2 = (1 - d0) / 2
    R Hc0, Hc1;          // H = Hc0 - Hc1 / s2a
    float sg, isg;       // 16-bit modes: scale of the moving g_i and its inverse
    float sf, isf;       // 16-bit modes: scale of the f_i
    float gfix;          // 2^(FIX_BITS) / sg: decoded g code -> fixed point
};

struct TileEntry {
    int32_t job, x0, y0, pad;
};

// ------------------------------------------------------------- storage modes
struct StF64 {
    using R = double;
    struct Pop { double* p; };  // [18][pitch]: g_0..g_8, f_0..f_8
    static constexpr bool kFix = false;
    static constexpr bool kRel = false;
    static constexpr int kMode = 0;
};
struct StF32 {
    using R = float;
    struct Pop { float* p; };
    static constexpr bool kFix = false;
    // g_0 is stored relative to the order parameter that the same step writes
    // to history plane 0 at the same node: the stored value is g_0 - phi^n, of
    // the size of the moving populations.  An O(1) rest population rounded to
    // FP32 every step carries a rounding bias that is the same at every bulk
    // node (same state, same rounding direction), so the total order parameter
    // drifts linearly in time; the relative form rounds only the small part.
    static constexpr bool kRel = true;
    static constexpr int kMode = 1;
};
struct StHalfBase {
    using R = float;
    // g_0 as 64-bit fixed point, g_1..g_8 and f_0..f_8 as 16-bit codes
    struct Pop { int64_t* g0; uint16_t* gm; uint16_t* fm; };
    static constexpr bool kFix = true;
    static constexpr bool kRel = false;
};

__device__ __forceinline__ uint16_t f16_enc(float v) {
    _Float16 h = (_Float16)v;  // round to nearest even
    return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_dec(uint16_t u) {
    return (float)__builtin_bit_cast(_Float16, u);
}
__device__ __forceinline__ uint16_t bf16_enc(float v) {
    uint32_t b = __builtin_bit_cast(uint32_t, v);
    if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu))
        return (uint16_t)((b >> 16) | 0x40u);  // keep NaN a NaN
    b += 0x7fffu + ((b >> 16) & 1u);           // round to nearest even
    return (uint16_t)(b >> 16);
}
__device__ __forceinline__ float bf16_dec(uint16_t u) {
    return __builtin_bit_cast(float, (uint32_t)u << 16);
}

struct StF16 : StHalfBase {
    static constexpr int kMode = 2;
    static __device__ __forceinline__ uint16_t enc(float v) { return f16_enc(v); }
    static __device__ __forceinline__ float dec(uint16_t u) { return f16_dec(u); }
};
struct StBF16 : StHalfBase {
    static constexpr int kMode = 3;
    static __device__ __forceinline__ uint16_t enc(float v) { return bf16_enc(v); }
    static __device__ __forceinline__ float dec(uint16_t u) { return bf16_dec(u); }
};

template <class S>
struct Job {
    typename S::Pop pop[2];
    typename S::R* hist[2];   // [5][pitch]: phi, ux, uy, Sx, Sy of the previous level
    typename S::R* stat;      // [3][pitch]: phi0, psi, lap psi
    const double* in;         // INIT: [5][pitch] phi, phi0 (unused), cos (unused), ux, uy
    double* out;              // OUT: [4][pitch] phi, ux, uy, P (NULL: reductions only)
    double* part;             // OUT: [ntiles][NPART] partial sums
    int64_t* ipart;           // OUT, 16-bit modes: [ntiles] exact fixed-point mass
    int64_t pitch;
    int64_t step0;            // steps taken before the launch sequence
    int32_t nx, ny;
    int32_t n_active;         // launches with t >= n_active leave this job alone
    int32_t tile_base;        // first tile of this job in the tile table
    int32_t np;               // free particles (0: none)
    int32_t walls;            // no-flux bounce-back walls: bit 0 below row 0 and above row
                              // ny - 1, bit 1 left of column 0 and right of column nx - 1
    const double* parts;      // [np][PSTRIDE] particle state (Sec. 2.4)
    const int32_t* owner;     // [pitch] owning particle of each node, -1 if none
    typename S::R* pf;        // [3][pitch] rho f dt (x, y) and rho at owned nodes
    Coef<typename S::R> c;
};

// Particle state columns: centre, translational and angular velocity, radius,
// density, cos of the contact angle of phase 1; per-particle outputs of an
// update: hydrodynamic force and torque (Eq. Ff), internal-fluid corrections
// carried to the next update (Eq. Ffin), internal fluid density.
enum { PX, PY, PUX, PUY, POM, PRAD, PRHO, PCOS, PSTRIDE };
enum { QFX, QFY, QT, QFINX, QFINY, QTIN, QRHOIN, QSTRIDE };
// A particle's indicator [1 + tanh(2 (R - r) / D)] / 2 is exactly 0 in FP64
// from r = R + 9.53 D on (tanh rounds to -1 below -19.06) and in FP32 from
// R + 4.6 D on, so skipping nodes beyond R + PCUT D changes no value: the
// indicator equals the plain tanh profile at every node.
constexpr double PCUT = 10.0;

// ------------------------------------------------------------------ helpers
// nearest periodic image of a coordinate difference (the division only when
// the difference is not already within half the period, where the formula
// returns it unchanged)
__device__ __forceinline__ double perd(double d, int n) {
    if (fabs(d) < 0.5 * n) return d;
    return d - n * floor(d / n + 0.5);
}

__device__ __forceinline__ int wrapi(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Row (column) of the node that row v, possibly outside 0..n-1, stands for:
// the periodic image, or with walls at -1/2 and n - 1/2 the mirrored one
// (-1 -> 0, -2 -> 1, n -> n - 1; rows further out, which only ragged tiles
// larger than the domain visit, fold again and stay inside).
__device__ __forceinline__ int imgof(int v, int n, int walled) {
    if (!walled) return wrapi(v, n);
    const int m = wrapi(v, 2 * n);
    return m < n ? m : 2 * n - 1 - m;
}

// Coordinate difference along a direction: the nearest periodic image, or the
// plain difference between walls.
__device__ __forceinline__ double perdw(double d, int n, int walled) {
    return walled ? d : perd(d, n);
}

// Map the hardware block index so that each of the 8 XCDs (blocks are dealt
// round-robin) gets one contiguous range of tiles: neighbouring tiles, whose
// halos overlap, then share an L2.
__device__ __forceinline__ int xcd_remap(int b, int G) {
    const int q = G >> 3, r = G & 7;
    const int k = b & 7, j = b >> 3;
    return k * q + (k < r ? k : r) + j;
}

// Isotropic central differences (weights 4/9, 1/9, 1/36, c_s^2 = 1/3) on an
// LDS tile of width W around index q.
template <class R>
__device__ __forceinline__ void grad9(const R* s, int q, int W, R& gx, R& gy) {
    const R e = s[q + 1], w = s[q - 1], n = s[q + W], so = s[q - W];
    const R ne = s[q + W + 1], nw = s[q + W - 1], se = s[q - W + 1], sw = s[q - W - 1];
    gx = (e - w) * R(1.0 / 3.0) + ((ne + se) - (nw + sw)) * R(1.0 / 12.0);
    gy = (n - so) * R(1.0 / 3.0) + ((ne + nw) - (se + sw)) * R(1.0 / 12.0);
}
template <class R>
__device__ __forceinline__ R lap9(const R* s, int q, int W) {
    const R c4 = R(4) * s[q];
    const R ax = (s[q + 1] + s[q - 1]) + (s[q + W] + s[q - W]);
    const R dg = (s[q + W + 1] + s[q + W - 1]) + (s[q - W + 1] + s[q - W - 1]);
    return (ax - c4) * R(2.0 / 3.0) + (dg - c4) * R(1.0 / 6.0);
}

// a / b in the node update: IEEE division, except with 16-bit storage, whose
// FP32 arithmetic is instruction-bound and whose storage rounding dwarfs an
// ulp: there the hardware reciprocal (1 ulp) times a, one instruction
// instead of a division sequence (4% of the 1024^2 step).
template <class S, class R>
__device__ __forceinline__ R sdiv(R a, R b) {
    if constexpr (S::kFix)
        return a * __builtin_amdgcn_rcpf(b);
    else
        return a / b;
}

template <class R>
__device__ __forceinline__ R clamp1(R v) {
    return v < R(-1) ? R(-1) : (v > R(1) ? R(1) : v);
}
// Gradient of the order parameter clamped to [-1, 1] (the field the density
// law is evaluated on).
template <class R>
__device__ __forceinline__ void grad9c(const R* s, int q, int W, R& gx, R& gy) {
    const R e = clamp1(s[q + 1]), w = clamp1(s[q - 1]), n = clamp1(s[q + W]), so = clamp1(s[q - W]);
    const R ne = clamp1(s[q + W + 1]), nw = clamp1(s[q + W - 1]);
    const R se = clamp1(s[q - W + 1]), sw = clamp1(s[q - W - 1]);
    gx = (e - w) * R(1.0 / 3.0) + ((ne + se) - (nw + sw)) * R(1.0 / 12.0);
    gy = (n - so) * R(1.0 / 3.0) + ((ne + nw) - (se + sw)) * R(1.0 / 12.0);
}

// Chemical potential, Eq. (potential), wetting terms through psi.
// T: the arithmetic of the evaluation (FP64 for the FP32 storage mode, whose
// order parameter is carried in FP64 in LDS), C: the coefficient set.
template <class T, class C>
__device__ __forceinline__ T chem_pot(const C& c, T ph, T lap, T z, T psi, T lpsi) {
    const T ph2 = ph * ph;
    return T(c.k3s_D) * (ph * (ph2 - T(1)) + psi * (T(3) * ph2 + z * z - T(1)))
         + T(c.k9s_D) * z * z * ph - T(c.k3Ds_8) * (lap + lpsi);
}

// Hermite moments m_k = sum_i h_k(c_i) f_i of the D2Q9 basis
// (1, cx, cy, cx^2-a, cy^2-a, cx cy, cx(cy^2-a), cy(cx^2-a), (cx^2-a)(cy^2-a)),
// computed as a 3x3 tensor transform (x then y).  Velocity order
// 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1).
template <class R>
__device__ __forceinline__ void hermite_fwd(const R* f, R a, R one_a, R* m) {
    const R A00 = (f[3] + f[1]) + f[0], A10 = f[1] - f[3], A20 = one_a * (f[1] + f[3]) - a * f[0];
    const R A0p = (f[6] + f[5]) + f[2], A1p = f[5] - f[6], A2p = one_a * (f[5] + f[6]) - a * f[2];
    const R A0m = (f[7] + f[8]) + f[4], A1m = f[8] - f[7], A2m = one_a * (f[8] + f[7]) - a * f[4];
    m[0] = A00 + (A0p + A0m);
    m[1] = A10 + (A1p + A1m);
    m[2] = A0p - A0m;
    m[3] = A20 + (A2p + A2m);
    m[4] = one_a * (A0p + A0m) - a * A00;
    m[5] = A1p - A1m;
    m[6] = one_a * (A1p + A1m) - a * A10;
    m[7] = A2p - A2m;
    m[8] = one_a * (A2p + A2m) - a * A20;
}

// Inverse transform f_i = w_i sum_k h_k(c_i) m_k / N_k (discrete
// orthogonality of the Hermite basis under the D2Q9 weights).
template <class R>
__device__ __forceinline__ void hermite_inv(const Coef<R>& c, const R* m, R* f) {
    const R a = c.a, one_a = c.one_a;
    const R M00 = m[0], M10 = m[1] * c.inv_n1, M01 = m[2] * c.inv_n1;
    const R M20 = m[3] * c.inv_n2, M02 = m[4] * c.inv_n2, M11 = m[5] * c.inv_n11;
    const R M12 = m[6] * c.inv_n12, M21 = m[7] * c.inv_n12, M22 = m[8] * c.inv_n22;
    // y transform: B_j(cy) = sum_k p_k(cy) M_jk, p = (1, c, c^2 - a)
    const R B00 = M00 - a * M02, B0p = (M00 + M01) + one_a * M02, B0m = (M00 - M01) + one_a * M02;
    const R B10 = M10 - a * M12, B1p = (M10 + M11) + one_a * M12, B1m = (M10 - M11) + one_a * M12;
    const R B20 = M20 - a * M22, B2p = (M20 + M21) + one_a * M22, B2m = (M20 - M21) + one_a * M22;
    f[0] = c.w0 * (B00 - a * B20);
    f[1] = c.w1 * ((B00 + B10) + one_a * B20);
    f[3] = c.w1 * ((B00 - B10) + one_a * B20);
    f[2] = c.w1 * (B0p - a * B2p);
    f[4] = c.w1 * (B0m - a * B2m);
    f[5] = c.w2 * ((B0p + B1p) + one_a * B2p);
    f[6] = c.w2 * ((B0p - B1p) + one_a * B2p);
    f[7] = c.w2 * ((B0m - B1m) + one_a * B2m);
    f[8] = c.w2 * ((B0m + B1m) + one_a * B2m);
}

// ------------------------------------------------------ population access
// Halfway bounce-back at a node next to walls (bb: bit 0 wall below, 1 above,
// 2 left, 3 right): a direction that would cross one of them is stored into
// the opposite direction's plane at the node itself.
__device__ __forceinline__ constexpr bool crosses(int i, int bb) {
    constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1}, cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    return (cy[i] < 0 && (bb & 1)) || (cy[i] > 0 && (bb & 2)) || (cx[i] < 0 && (bb & 4)) ||
           (cx[i] > 0 && (bb & 8));
}
__device__ __forceinline__ constexpr int opposite(int i) {
    constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    return opp[i];
}

// Node offsets are 32-bit (domains hold fewer than 2^31 nodes); each plane
// base is a uniform pointer, so loads use a scalar base plus a 32-bit vector
// offset.
// Global-address-space view of a device pointer.  The planes reach the
// kernels through the job table, so the compiler cannot tell that they are
// device memory and would access them with flat instructions, which also
// count against the LDS wait counter: every wait for an LDS read would then
// wait for the population loads in flight as well.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* G(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}

template <class S> struct Access;

// Element o of a plane.  A plane of 2- or 4-byte elements is addressed by a
// 32-bit byte offset from its base, which is the same for the whole block:
// each load or store then takes the base in scalar registers and one 32-bit
// vector offset, with no 64-bit address arithmetic per access (such planes
// hold at most 4 GiB: FP32 and 16-bit storage take at most 2^30 nodes, more
// than fit in the device's memory).  FP64 planes keep 64-bit indexing
// (offsets measured no faster there).
template <class T>
__device__ __forceinline__ T* boff(T* base, uint32_t off) {
    using B = __attribute__((address_space(1))) char;
    return (T*)((B*)base + off);
}
template <class R>
__device__ __forceinline__ __attribute__((address_space(1))) R& pel(R* plane, uint32_t o) {
    if constexpr (sizeof(R) == 8)
        return G(plane)[o];
    else
        return *boff(G(plane), o * (uint32_t)sizeof(R));
}
template <class R>
__device__ __forceinline__ const __attribute__((address_space(1))) R& pel(
    const __attribute__((address_space(1))) R* plane, uint32_t o) {
    if constexpr (sizeof(R) == 8)
        return plane[o];
    else
        return *boff(plane, o * (uint32_t)sizeof(R));
}

template <class Sf>
struct AccessFull {  // FP64 / FP32: plain values
    using R = typename Sf::R;
    using Pop = typename Sf::Pop;
    static __device__ __forceinline__ R phi(const Pop& P, int64_t pitch, uint32_t o, const Coef<R>&) {
        R* p = P.p;
        return ((pel(p, o) + (pel(p + pitch, o) + pel(p + 3 * pitch, o))) + (pel(p + 2 * pitch, o) + pel(p + 4 * pitch, o)))
             + ((pel(p + 5 * pitch, o) + pel(p + 7 * pitch, o)) + (pel(p + 6 * pitch, o) + pel(p + 8 * pitch, o)));
    }
    static __device__ __forceinline__ void load_g(const Pop& P, int64_t pitch, uint32_t o, const Coef<R>&,
                                                  R* g, int64_t& mfix) {
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] = pel(P.p + i * pitch, o);
        mfix = 0;
    }
    static __device__ __forceinline__ R phi_of(const R* g, int64_t, const Coef<R>&) {
        return ((g[0] + (g[1] + g[3])) + (g[2] + g[4])) + ((g[5] + g[7]) + (g[6] + g[8]));
    }
    static __device__ __forceinline__ void load_f(const Pop& P, int64_t pitch, uint32_t o, const Coef<R>&,
                                                  R* f) {
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = pel(P.p + (9 + i) * pitch, o);
    }
    static __device__ __forceinline__ void store(const Pop& P, int64_t pitch, const uint32_t* dst,
                                                 const Coef<R>&, const R* g, const R* f, int64_t) {
#pragma unroll
        for (int i = 0; i < 9; ++i) pel(P.p + i * pitch, dst[i]) = g[i];
#pragma unroll
        for (int i = 0; i < 9; ++i) pel(P.p + (9 + i) * pitch, dst[i]) = f[i];
    }
    // next to walls: the crossing directions go to the opposite planes at o
    static __device__ __forceinline__ void store_bb(const Pop& P, int64_t pitch, const uint32_t* dst,
                                                    uint32_t o, int bb, const Coef<R>&, const R* g, const R* f,
                                                    int64_t) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const bool cr = crosses(i, bb);
            const int64_t pl = cr ? opposite(i) : i;
            const uint32_t d = cr ? o : dst[i];
            pel(P.p + pl * pitch, d) = g[i];
            pel(P.p + (9 + pl) * pitch, d) = f[i];
        }
    }
};
template <> struct Access<StF64> : AccessFull<StF64> {};
template <> struct Access<StF32> : AccessFull<StF32> {};

template <class Sh>
struct AccessHalf {  // 16-bit codes + fixed-point rest population
    using Pop = typename Sh::Pop;
    // Fixed-point value (units of 2^-40) of a moving-population code, as an
    // integer-valued double.  FP16 codes give multiples of 2^(16-kg) below
    // 2^(56-kg), i.e. at most 40 significant bits; BF16 codes are rounded to
    // integers (far below 2^53 for any finite state).  Sums of eight of them
    // are therefore exact in double precision.
    static __device__ __forceinline__ double gfix(const Coef<float>& c, uint16_t code) {
        // FP16: every finite code times 2^(40 - kg), kg <= 16, is an integer
        // below 2^57, i.e. an exact FP32 product of its 11-bit significand:
        // the same value with one FP32 multiply instead of FP64 arithmetic
        if constexpr (Sh::kMode == 2) return (double)(Sh::dec(code) * c.gfix);
        return rint((double)Sh::dec(code) * (double)c.gfix);
    }
    static __device__ __forceinline__ float fix2f(int64_t m) {
        return (float)m * 0x1p-40f;
    }
    static __device__ __forceinline__ float phi(const Pop& P, int64_t pitch, uint32_t o, const Coef<float>& c) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i) s += gfix(c, pel(P.gm + i * pitch, o));
        return fix2f(G(P.g0)[o] + (int64_t)s);
    }
    static __device__ __forceinline__ void load_g(const Pop& P, int64_t pitch, uint32_t o, const Coef<float>& c,
                                                  float* g, int64_t& mfix) {
        const int64_t rest = G(P.g0)[o];
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const uint16_t code = pel(P.gm + i * pitch, o);
            g[i + 1] = Sh::dec(code) * c.isg;
            s += gfix(c, code);
        }
        g[0] = fix2f(rest);
        mfix = rest + (int64_t)s;
    }
    static __device__ __forceinline__ float phi_of(const float*, int64_t mfix, const Coef<float>&) {
        return fix2f(mfix);
    }
    static __device__ __forceinline__ void load_f(const Pop& P, int64_t pitch, uint32_t o, const Coef<float>& c,
                                                  float* f) {
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = Sh::dec(pel(P.fm + i * pitch, o)) * c.isf;
    }
    // mfix: the node's conserved sum_i g_i in fixed point; g_0 is written so
    // that the stored values sum to it exactly.
    static __device__ __forceinline__ void store(const Pop& P, int64_t pitch, const uint32_t* dst,
                                                 const Coef<float>& c, const float* g, const float* f,
                                                 int64_t mfix) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const uint16_t code = Sh::enc(g[i + 1] * c.sg);
            pel(P.gm + i * pitch, dst[i + 1]) = code;
            s += gfix(c, code);
        }
        G(P.g0)[dst[0]] = mfix - (int64_t)s;
#pragma unroll
        for (int i = 0; i < 9; ++i) pel(P.fm + i * pitch, dst[i]) = Sh::enc(f[i] * c.sf);
    }
    // next to walls: the crossing directions go to the opposite planes at o
    // (dst[0] == o); the stored values still sum to mfix at this node's share
    static __device__ __forceinline__ void store_bb(const Pop& P, int64_t pitch, const uint32_t* dst,
                                                    uint32_t o, int bb, const Coef<float>& c, const float* g,
                                                    const float* f, int64_t mfix) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const bool cr = crosses(i + 1, bb);
            const int64_t pl = cr ? opposite(i + 1) : i + 1;
            const uint16_t code = Sh::enc(g[i + 1] * c.sg);
            pel(P.gm + (pl - 1) * pitch, cr ? o : dst[i + 1]) = code;
            s += gfix(c, code);
        }
        G(P.g0)[dst[0]] = mfix - (int64_t)s;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const bool cr = crosses(i, bb);
            const int64_t pl = cr ? opposite(i) : i;
            pel(P.fm + pl * pitch, cr ? o : dst[i]) = Sh::enc(f[i] * c.sf);
        }
    }
};
template <> struct Access<StF16> : AccessHalf<StF16> {};
template <> struct Access<StBF16> : AccessHalf<StBF16> {};

// ------------------------------------------------ block reduction (FP64)
template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ------------------------------------------------------------ tile kernel
// Block size per tile height: 256 threads (4 wavefronts) for 64 x 4 tiles,
// 512 (8 wavefronts) for 64 x 8, 64 x 16 and 64 x 32, i.e. one, one, two and
// four owned nodes per thread.  (64 x 8 with 256 threads, two nodes each,
// was slower in every storage mode and grid measured.)
template <int TY>
struct TileCfg {
    static constexpr int NT = TY == 4 ? 256 : 512;
};

// Thread (lane, wave) owns the nodes (x0 + lane, y0 + wave + NW k), k < NOWN.
// All global reads a block needs beyond its own nodes -- the order parameter
// on the 3-node halo ring, the static fields on the 2-node halo, the previous
// velocity on the 1-node halo -- are issued in one phase (A) before the first
// barrier, so their latencies overlap.
// PART: the domain has free particles (their branch and its LDS are compiled
// only into this variant, so the plain kernel keeps its register budget).
// WALL: some job may have bounce-back walls (Job::walls); the plain kernel
// carries none of their instructions.
template <class S, int TY, int MODE, bool PART = false, bool WALL = false>
__global__ __launch_bounds__(TileCfg<TY>::NT) void k_tile(const Job<S>* __restrict__ jobs,
                                                         const TileEntry* __restrict__ tiles, int ntiles,
                                                         int t) {
    using R = typename S::R;
    // the order parameter in LDS: FP64 for FP32 storage, where it is the sum
    // of the FP32 history value and the small FP32 remainder of the
    // populations (exact in FP64), so that the stencils of mu (Laplacian) and
    // grad phi see phi to the precision the populations carry it, not rounded
    // to FP32 (near phi = +-1 that rounding, 3e-8, put 1e-10 into mu and, divided
    // by a light phase's density, into the velocity)
    using RX = typename std::conditional<S::kRel, double, R>::type;
    using A = Access<S>;
    constexpr int NTH = TileCfg<TY>::NT;
    constexpr int NW = NTH / 64;
    constexpr int W3 = TX + 6, H3 = TY + 6;
    constexpr int W2 = TX + 4, H2 = TY + 4;
    constexpr int W1 = TX + 2, H1 = TY + 2;
    constexpr int NOWN = TY / NW;                 // owned nodes per thread
    constexpr bool KEEP = NOWN <= 2;              // keep owned data in registers from phase A
    constexpr int NRING = 6 * W3 + 6 * TY;        // halo ring of the order parameter
    constexpr int NB = (H2 * W2 + NTH - 1) / NTH; // stage-B points per thread
    constexpr int NC = (H1 * W1 + NTH - 1) / NTH; // stage-C points per thread
    __shared__ RX sphi[H3 * W3];
    __shared__ R smu[H2 * W2];
    __shared__ R sz[PART ? H2 * W2 : 1];          // phi0 on the stage-B points (particles)
    __shared__ R sSx[H1 * W1];
    __shared__ R sSy[H1 * W1];
    __shared__ R sw[H1 * W1];
    __shared__ int s_col[W3];                     // x of LDS column lx (x0 + lx - 3), periodic or mirrored
    __shared__ int s_row[H3];                     // y * nx of LDS row ly (y0 + ly - 3), periodic or mirrored
    __shared__ double sred[NW][NPART];
    __shared__ long long sired[NW];

    const int e = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    if (e >= ntiles) return;
    const TileEntry te = tiles[e];
    const Job<S>& J = jobs[te.job];
    if (MODE == MODE_STEP && t >= J.n_active) return;
    const int nx = J.nx, ny = J.ny;
    const int64_t pitch = J.pitch;
    const int64_t step = J.step0 + (MODE == MODE_STEP ? t : 0);
    const int par = (int)(step & 1);
    const bool first = (step == 0);
    const Coef<R>& c = J.c;
    const typename S::Pop cur = J.pop[par];
    const __attribute__((address_space(1))) R* __restrict__ hprev = G(J.hist[par]);
    const __attribute__((address_space(1))) R* __restrict__ st = G(J.stat);
    const int x0 = te.x0, y0 = te.y0;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // walls this tile can see: only tiles whose 3-node halo reaches past the
    // domain edge read ghost nodes or hold wall nodes
    int walls = WALL ? J.walls : 0;
    if (WALL && y0 >= 3 && y0 + TY + 3 <= ny) walls &= ~1;
    if (WALL && x0 >= 3 && x0 + TX + 3 <= nx) walls &= ~2;

    // index tables (the only integer divisions of the kernel); with walls a
    // row or column outside the domain reads its mirror image (ghost nodes)
    for (int i = tid; i < W3 + H3; i += NTH) {
        if (i < W3)
            s_col[i] = imgof(x0 + i - 3, nx, walls & 2);
        else
            s_row[i - W3] = imgof(y0 + (i - W3) - 3, ny, walls & 1) * nx;
    }
    __syncthreads();

    // ---- phase A: every global read ----
    R g[KEEP ? NOWN : 1][9], f[KEEP ? NOWN : 1][9], hp[KEEP ? NOWN : 1][5];
    int64_t mfix[KEEP ? NOWN : 1];
    R zz[NOWN];
    uint32_t own[NOWN];
#pragma unroll
    for (int k = 0; k < NOWN; ++k) {
        const int ly = wv + NW * k;
        const uint32_t o = (uint32_t)(s_row[ly + 3] + s_col[lane + 3]);
        own[k] = o;
        RX* sp = &sphi[(ly + 3) * W3 + lane + 3];
        if (MODE == MODE_INIT) {
            *sp = (RX)G(J.in)[o];
        } else if (KEEP) {
            const int kk = KEEP ? k : 0;
            A::load_g(cur, pitch, o, c, g[kk], mfix[kk]);
            A::load_f(cur, pitch, o, c, f[kk]);
#pragma unroll
            for (int v = 0; v < 5; ++v) hp[kk][v] = pel(hprev + v * pitch, o);
            *sp = S::kRel ? (RX)hp[kk][0] + (RX)A::phi_of(g[kk], mfix[kk], c) : (RX)A::phi_of(g[kk], mfix[kk], c);
        } else {
            *sp = S::kRel ? (RX)pel(hprev, o) + (RX)A::phi(cur, pitch, o, c) : (RX)A::phi(cur, pitch, o, c);
        }
        zz[k] = pel(st, o);
    }
    for (int p = tid; p < NRING; p += NTH) {
        int ly, lx;
        if (p < 3 * W3) {
            ly = p / W3; lx = p - ly * W3;
        } else if (p < 6 * W3) {
            const int q = p - 3 * W3;
            ly = TY + 3 + q / W3; lx = q - (q / W3) * W3;
        } else {
            const int q = p - 6 * W3;
            const int r = q / 6, cc = q - r * 6;
            ly = 3 + r; lx = cc < 3 ? cc : TX + cc;
        }
        const uint32_t o = (uint32_t)(s_row[ly] + s_col[lx]);
        if (MODE == MODE_INIT)
            sphi[ly * W3 + lx] = (RX)G(J.in)[o];
        else if (S::kRel)
            sphi[ly * W3 + lx] = (RX)pel(hprev, o) + (RX)A::phi(cur, pitch, o, c);
        else
            sphi[ly * W3 + lx] = A::phi(cur, pitch, o, c);
    }
    // static fields on the stage-B points and previous velocity on the
    // stage-C points, held in registers until those stages
    R bz[NB], bpsi[NB], blp[NB], cux[NC], cuy[NC];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const int p = tid + k * NTH;
        if (p < H2 * W2) {
            const int ly = p / W2, lx = p - ly * W2;
            const uint32_t o = (uint32_t)(s_row[ly + 1] + s_col[lx + 1]);
            bz[k] = pel(st, o);
            bpsi[k] = pel(st + pitch, o);
            blp[k] = pel(st + 2 * pitch, o);
        }
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const int p = tid + k * NTH;
        cux[k] = R(0);
        cuy[k] = R(0);
        if (MODE != MODE_INIT && p < H1 * W1) {
            const int ly = p / W1, lx = p - ly * W1;
            const uint32_t o = (uint32_t)(s_row[ly + 2] + s_col[lx + 2]);
            // ghost nodes hold the mirrored no-slip velocity: both components
            // odd under each mirror (even at a corner)
            const int yy = y0 + ly - 1, xx = x0 + lx - 1;
            const bool gy = (walls & 1) && (yy < 0 || yy >= ny), gx = (walls & 2) && (xx < 0 || xx >= nx);
            const R sg = gx != gy ? R(-1) : R(1);
            cux[k] = sg * pel(hprev + pitch, o);
            cuy[k] = sg * pel(hprev + 2 * pitch, o);
        }
    }
    __syncthreads();

    // ---- B: chemical potential on the tile and a 2-node halo ----
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const int p = tid + k * NTH;
        if (p < H2 * W2) {
            const int ly = p / W2, lx = p - ly * W2;
            const int q = (ly + 1) * W3 + (lx + 1);
            smu[p] = (R)chem_pot<RX>(c, sphi[q], lap9(sphi, q, W3), (RX)bz[k], (RX)bpsi[k], (RX)blp[k]);
            if (PART) sz[p] = bz[k];
        }
    }
    __syncthreads();

    // ---- C: mass flux S and w = (S_x u_y - S_y u_x)/2 with the previous velocity ----
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const int p = tid + k * NTH;
        if (p < H1 * W1) {
            const int ly = p / W1, lx = p - ly * W1;
            R gmx, gmy;
            grad9(smu, (ly + 1) * W2 + (lx + 1), W2, gmx, gmy);
            const R Sx = c.kS * gmx, Sy = c.kS * gmy;
            sSx[p] = Sx;
            sSy[p] = Sy;
            if (MODE != MODE_INIT) sw[p] = (Sx * cuy[k] - Sy * cux[k]) * R(0.5);
        }
    }
    __syncthreads();

    // ---- D: node update ----
    double acc_m = 0.0, acc_ef = 0.0, acc_ek = 0.0, acc_nf = 0.0;
    long long acc_im = 0;
    // owned data for the node being updated (prefetched one node ahead when
    // it is not kept from phase A)
    R gn[9], fn[9], hn[5];
    int64_t mn = 0;
    if (!KEEP && MODE != MODE_INIT) {
        A::load_g(cur, pitch, own[0], c, gn, mn);
        A::load_f(cur, pitch, own[0], c, fn);
#pragma unroll
        for (int v = 0; v < 5; ++v) hn[v] = pel(hprev + v * pitch, own[0]);
    }
#pragma unroll
    for (int k = 0; k < NOWN; ++k) {
        R gk[9], fk[9], hk[5];
        int64_t mk = 0;
        if (MODE != MODE_INIT) {
            if (KEEP) {
                const int kk = KEEP ? k : 0;
#pragma unroll
                for (int i = 0; i < 9; ++i) { gk[i] = g[kk][i]; fk[i] = f[kk][i]; }
#pragma unroll
                for (int v = 0; v < 5; ++v) hk[v] = hp[kk][v];
                mk = mfix[kk];
            } else {
#pragma unroll
                for (int i = 0; i < 9; ++i) { gk[i] = gn[i]; fk[i] = fn[i]; }
#pragma unroll
                for (int v = 0; v < 5; ++v) hk[v] = hn[v];
                mk = mn;
                if (k + 1 < NOWN) {
                    const uint32_t o1 = own[k + 1 < NOWN ? k + 1 : k];
                    A::load_g(cur, pitch, o1, c, gn, mn);
                    A::load_f(cur, pitch, o1, c, fn);
#pragma unroll
                    for (int v = 0; v < 5; ++v) hn[v] = pel(hprev + v * pitch, o1);
                }
            }
        }
        const int ly = wv + NW * k;
        const int x = x0 + lane, y = y0 + ly;
        if (x >= nx || y >= ny) continue;
        const uint32_t o = own[k];
        const int q3 = (ly + 3) * W3 + (lane + 3);
        const int q2 = (ly + 2) * W2 + (lane + 2);
        const int q1 = (ly + 1) * W1 + (lane + 1);
        const RX phx = sphi[q3];
        const R ph = (R)phx;
        R dpx, dpy;
        {
            RX gx, gy;
            grad9(sphi, q3, W3, gx, gy);
            dpx = (R)gx;
            dpy = (R)gy;
        }
        const R mu = smu[q2];
        const R Sx = sSx[q1], Sy = sSy[q1];
        const R z = zz[k];
        // density and viscosity laws (Eq. rho) on phi clamped to [-1, 1],
        // written as rho2 + (rho1 - rho2)(1 + phi)/2: the light phase's density
        // is then not the difference of two O(1) numbers (at density ratio
        // 1000 that difference lost 4 of FP32's 7 digits, and the velocity
        // j / rho with them); 1 + phi comes from the FP64 phi of FP32 storage
        const R op = (R)(RX(1) + clamp1(phx));
        const R rho = c.rho2 + c.drho * op;
        const R muv = c.mu2 + c.dmu * op;
        // neighbours for the push (periodic); bb: the walls next to this node
        // (bit 0 below, 1 above, 2 left, 3 right), whose crossing populations
        // are reflected at the store, and across which neighbours mirror
        const int bb = !WALL ? 0
                             : ((walls & 1) && y == 0 ? 1 : 0) | ((walls & 1) && y == ny - 1 ? 2 : 0) |
                                   ((walls & 2) && x == 0 ? 4 : 0) | ((walls & 2) && x == nx - 1 ? 8 : 0);
        const int xe = x + 1 == nx ? ((bb & 8) ? x : 0) : x + 1, xw = x == 0 ? ((bb & 4) ? 0 : nx - 1) : x - 1;
        const uint32_t rc = (uint32_t)y * (uint32_t)nx;
        const uint32_t rn = (uint32_t)(y + 1 == ny ? ((bb & 2) ? y : 0) : y + 1) * (uint32_t)nx;
        const uint32_t rs = (uint32_t)(y == 0 ? ((bb & 1) ? 0 : ny - 1) : y - 1) * (uint32_t)nx;

        if (MODE == MODE_INIT) {
            // Procedure step 1: g = g^eq, f = f^eq at P = 0 with the given u.
            const R ux = (R)G(J.in)[3 * pitch + o], uy = (R)G(J.in)[4 * pitch + o];
            // g^eq of Sec. 3.1, term by term (keeps the small moving values exact)
            const R emu = c.eta * mu, ia = R(1) / c.a;
            const R jxa = ph * ux * ia, jya = ph * uy * ia;
            R m[9], gg[9], ff[9];
            // relative rest population: g_0^eq - phi_h with phi_h = FP32(phi),
            // the history value below; phi - phi_h keeps phi's lower bits
            gg[0] = S::kRel ? (c.w0 - R(1)) * emu + (R)(phx - (RX)ph) : ph + (c.w0 - R(1)) * emu;
            gg[1] = c.w1 * (emu + jxa);
            gg[3] = c.w1 * (emu - jxa);
            gg[2] = c.w1 * (emu + jya);
            gg[4] = c.w1 * (emu - jya);
            gg[5] = c.w2 * (emu + (jxa + jya));
            gg[6] = c.w2 * (emu + (jya - jxa));
            gg[7] = c.w2 * (emu - (jxa + jya));
            gg[8] = c.w2 * (emu + (jxa - jya));
            m[0] = R(0); m[1] = rho * ux; m[2] = rho * uy;
            m[3] = rho * ux * ux - Sx * ux; m[4] = rho * uy * uy - Sy * uy;
            m[5] = rho * ux * uy - (Sx * uy + ux * Sy) * R(0.5);
            m[6] = R(0); m[7] = R(0); m[8] = R(0);
            hermite_inv(c, m, ff);
            uint32_t dst[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) dst[i] = o;
            int64_t mf = 0;
            if (S::kFix) mf = llrint(G(J.in)[o] * 0x1p40);
            A::store(J.pop[0], pitch, dst, c, gg, ff, mf);
            __attribute__((address_space(1))) R* h0 = G(J.hist[0]);
            h0[o] = ph; h0[pitch + o] = ux; h0[2 * pitch + o] = uy;
            h0[3 * pitch + o] = Sx; h0[4 * pitch + o] = Sy;
            continue;
        }

        R wx, wy;
        grad9(sw, q1, W1, wx, wy);
        R dcx, dcy;
        {
            RX gx, gy;
            grad9c(sphi, q3, W3, gx, gy);
            dcx = (R)gx;
            dcy = (R)gy;
        }
        const R drx = c.drho * dcx, dry = c.drho * dcy;
        // free particles (Sec. 2.4): the owning particle's solid velocity
        // u_s = u_p + omega_p x (x - x_p) and the force mu_phi0 grad phi0 of
        // Eq. (muPhi0) on the nodes a particle owns
        R usolx = R(0), usoly = R(0), Fpx = R(0), Fpy = R(0);
        int own = -1;
        if (PART) {
            own = G(J.owner)[o];
            if (own >= 0) {
                const __attribute__((address_space(1))) double* q = G(J.parts) + own * PSTRIDE;
                // the domain's walls, not the tile's: a particle's support
                // reaches tiles whose halo stays inside the domain
                const int dw = WALL ? J.walls : 0;
                const double rx = perdw((double)x - q[PX], nx, dw & 2);
                const double ry = perdw((double)y - q[PY], ny, dw & 1);
                usolx = (R)(q[PUX] - q[POM] * ry);
                usoly = (R)(q[PUY] + q[POM] * rx);
                const R cth = (R)q[PCOS];
                R gzx, gzy;
                grad9(sz, q2, W2, gzx, gzy);
                const R muz = c.k9s_D * z * ph * ph + c.k3s_D * cth * ph * (R(3) * z * z + ph * ph - R(1))
                            - c.k3Ds_8 * cth * (R)lap9(sphi, q3, W3);
                Fpx = muz * gzx;
                Fpy = muz * gzy;
            }
        }
        // total force F = mu grad phi + mu_phi0 grad phi0 + F_b + F_c, F_c = (-d_y w, d_x w)
        const R Fx = (mu * dpx + ((rho - c.rho_ref) * c.gx + (R(1) - z) * c.fbx) - wy) + Fpx;
        const R Fy = (mu * dpy + ((rho - c.rho_ref) * c.gy + (R(1) - z) * c.fby) + wx) + Fpy;
        const R php = hk[0], uxp = hk[1], uyp = hk[2], Sxp = hk[3], Syp = hk[4];

        // Eq. uStar, solid forcing f = phi0 (u_s - u*), Eq. u (u_s = 0 unless a
        // particle owns the node)
        R usx, usy;
        if (first) {
            usx = uxp;
            usy = uyp;
        } else {
            const R jx = ((fk[1] - fk[3]) + (fk[5] - fk[6])) + (fk[8] - fk[7]);
            const R jy = ((fk[2] - fk[4]) + (fk[5] + fk[6])) - (fk[7] + fk[8]);
            const R irho = sdiv<S>(R(1), rho);
            usx = (jx + R(0.5) * Fx) * irho;
            usy = (jy + R(0.5) * Fy) * irho;
        }
        const R ax = z * (usolx - usx), ay = z * (usoly - usy);
        if (PART && own >= 0) {  // rho f dt and rho for the particle sums
            G(J.pf)[o] = rho * ax;
            G(J.pf)[pitch + o] = rho * ay;
            G(J.pf)[2 * pitch + o] = rho;
        }
        const R ux = first ? usx : usx + R(0.5) * ax;
        const R uy = first ? usy : usy + R(0.5) * ay;
        // flow relaxation from mu/(rho (1 - phi0)), kept finite in the solid
        R one_m = R(1) - z;
        one_m = one_m < c.solid_eps ? c.solid_eps : one_m;
        const R nu = sdiv<S>(muv, rho * one_m);
        const R tau_a = sdiv<S>(nu, c.ka) + R(0.5);
        const R tau_b = sdiv<S>(nu, c.a) + R(0.5);
        const R s2a = sdiv<S>(R(1), tau_a), s2b = sdiv<S>(R(1), tau_b);
        const R udr = ux * drx + uy * dry;
        const R q = rho * (ux * ux + uy * uy) - (Sx * ux + Sy * uy);
        const R rhop = c.rho2 + c.drho * (R(1) + clamp1(php));
        const R qp = rhop * (uxp * uxp + uyp * uyp) - (Sxp * uxp + Syp * uyp);
        R P = R(0);
        if (!first) {
            const R H = c.Hc0 - c.Hc1 * tau_a;
            const R sum = ((fk[1] + fk[3]) + (fk[2] + fk[4])) + ((fk[5] + fk[7]) + (fk[6] + fk[8]));
            P = c.Pfac * (sum + (R(0.5) + H) * udr
                          - c.Pw0 * ((rho * ux - Sx) * ux + (rho * uy - Sy) * uy) + c.K2 * (q - qp));
        }

        if (MODE == MODE_OUT) {
            if (J.out) {
                G(J.out)[o] = (double)phx;
                G(J.out)[pitch + o] = (double)ux;
                G(J.out)[2 * pitch + o] = (double)uy;
                G(J.out)[3 * pitch + o] = (double)P;
            }
            // energy densities (Eq. 2energy with psi; e_K = rho |u|^2 / 2)
            R qx, qy;
            {
                const auto* psi = st + pitch;
                const R e_ = psi[rc + xe], w_ = psi[rc + xw], n_ = psi[rn + x], s_ = psi[rs + x];
                const R ne = psi[rn + xe], nw = psi[rn + xw], se = psi[rs + xe], sw_ = psi[rs + xw];
                qx = (e_ - w_) * R(1.0 / 3.0) + ((ne + se) - (nw + sw_)) * R(1.0 / 12.0);
                qy = (n_ - s_) * R(1.0 / 3.0) + ((ne + nw) - (se + sw_)) * R(1.0 / 12.0);
            }
            const R psi0 = st[pitch + o];
            const R om = R(1) - ph * ph;
            const R ef = c.k3s_4D * om * om + c.k3Ds_16 * (dpx * dpx + dpy * dpy)
                       + c.k9s_2D * z * z * ph * ph + c.k3s_D * psi0 * ph * (ph * ph + z * z - R(1))
                       + R(2) * c.k3Ds_16 * (qx * dpx + qy * dpy);
            const R ek = R(0.5) * rho * (ux * ux + uy * uy);
            // relative rest population: sum the history value and the small
            // remainder separately, so the readout adds no FP32 rounding
            acc_m += S::kRel ? (double)php + (double)A::phi_of(gk, mk, c) : (double)ph;
            acc_ef += (double)ef;
            acc_ek += (double)ek;
            if (S::kFix) acc_im += (long long)mk;
            const bool bad = !(ph == ph && ux == ux && uy == uy && P == P) ||
                             !(ph - ph == R(0) && ux - ux == R(0) && uy - uy == R(0) && P - P == R(0));
            acc_nf += bad ? 1.0 : 0.0;
            continue;
        }

        // ---- phase field collision (Sec. 3.1, Hermite MRT) ----
        // Done as g* = g + M_H^{-1} dm with dm = -S (m - m^eq) + (I - S/2) m^G.
        // The non-equilibrium moments m - m^eq are formed from raw moments of
        // the eight moving populations only (the O(1) order parameter carried
        // by g_0 cancels analytically), so the small moving populations keep
        // their relative precision in FP32.
        const R a = c.a, one_a = c.one_a;
        R m[9];
        {
            const R jx = (gk[1] - gk[3]) + ((gk[5] - gk[6]) + (gk[8] - gk[7]));
            const R jy = (gk[2] - gk[4]) + ((gk[5] + gk[6]) - (gk[7] + gk[8]));
            const R dsum = (gk[5] + gk[6]) + (gk[7] + gk[8]);
            const R Pxx = (gk[1] + gk[3]) + dsum, Pyy = (gk[2] + gk[4]) + dsum;
            const R Pxy = (gk[5] + gk[7]) - (gk[6] + gk[8]);
            const R Qxyy = (gk[5] + gk[8]) - (gk[6] + gk[7]);
            const R Qxxy = (gk[5] + gk[6]) - (gk[7] + gk[8]);
            const R aem = a * c.eta * mu;
            const R Vx = ph * ux - php * uxp, Vy = ph * uy - php * uyp;  // d_t(phi u)
            const R kG = R(1) - R(0.5) * c.s1phi;
            m[0] = R(0);
            m[1] = kG * Vx - c.s1phi * (jx - ph * ux);
            m[2] = kG * Vy - c.s1phi * (jy - ph * uy);
            m[3] = -c.s2 * (Pxx - aem);
            m[4] = -c.s2 * (Pyy - aem);
            m[5] = -c.s2 * Pxy;
            m[6] = -c.s3 * (Qxyy - a * jx);
            m[7] = -c.s3 * (Qxxy - a * jy);
            m[8] = -c.s4 * ((dsum - a * (Pxx + Pyy)) + a * aem);
            R corr[9];
            hermite_inv(c, m, corr);
#pragma unroll
            for (int i = 0; i < 9; ++i) gk[i] += corr[i];
        }

        // ---- flow collision (Sec. 3.2, Hermite MRT, per-node s2a, s2b) ----
        hermite_fwd(fk, a, one_a, m);
        {
            const R Txx = Sx * ux, Tyy = Sy * uy, Txy = R(0.5) * (Sx * uy + ux * Sy);
            const R Txxp = Sxp * uxp, Tyyp = Syp * uyp, Txyp = R(0.5) * (Sxp * uyp + uxp * Syp);
            const R c3 = R(1) - R(3) * a;
            const R M2xx = R(2) * ux * Fx - (Txx - Txxp) + R(2) * a * ux * drx + c3 * udr;
            const R M2yy = R(2) * uy * Fy - (Tyy - Tyyp) + R(2) * a * uy * dry + c3 * udr;
            const R M2xy = (ux * Fy + Fx * uy) - (Txy - Txyp) + a * (ux * dry + drx * uy);
            const R Fpx = Fx + rho * ax, Fpy = Fy + rho * ay;
            const R rux = rho * ux, ruy = rho * uy;
            m[0] = m[0] - c.s0 * m[0] + (R(1) - R(0.5) * c.s0) * udr;
            m[1] = m[1] - c.s1 * (m[1] - rux) + (R(1) - R(0.5) * c.s1) * Fpx;
            m[2] = m[2] - c.s1 * (m[2] - ruy) + (R(1) - R(0.5) * c.s1) * Fpy;
            m[3] = m[3] - s2a * (m[3] - (P + rux * ux - Sx * ux)) + (R(1) - R(0.5) * s2a) * M2xx;
            m[4] = m[4] - s2a * (m[4] - (P + ruy * uy - Sy * uy)) + (R(1) - R(0.5) * s2a) * M2yy;
            m[5] = m[5] - s2b * (m[5] - (rux * uy - R(0.5) * (Sx * uy + ux * Sy)))
                 + (R(1) - R(0.5) * s2b) * M2xy;
            m[6] = m[6] - c.s3 * m[6];
            m[7] = m[7] - c.s3 * m[7];
            m[8] = m[8] - c.s4 * (m[8] + a * P);
        }
        hermite_inv(c, m, fk);

        // ---- push to the other copy, periodic ----
        // Next to a wall (halfway bounce-back) the populations that would
        // cross it return to this node in the opposite directions.
        uint32_t dst[9];
        dst[0] = o;
        dst[1] = rc + xe;
        dst[2] = rn + x;
        dst[3] = rc + xw;
        dst[4] = rs + x;
        dst[5] = rn + xe;
        dst[6] = rn + xw;
        dst[7] = rs + xw;
        dst[8] = rs + xe;
        // relative rest population: g_0 - phi^n with phi^n the value written
        // to history below; (php - ph) is exact for nearby values
        if (S::kRel) gk[0] += php - ph;
        if (WALL && bb)
            A::store_bb(J.pop[par ^ 1], pitch, dst, o, bb, c, gk, fk, mk);
        else
            A::store(J.pop[par ^ 1], pitch, dst, c, gk, fk, mk);
        R* hw = J.hist[par ^ 1];
        pel(hw, o) = ph;
        pel(hw + pitch, o) = ux;
        pel(hw + 2 * pitch, o) = uy;
        pel(hw + 3 * pitch, o) = Sx;
        pel(hw + 4 * pitch, o) = Sy;
    }

    if (MODE == MODE_OUT) {
        acc_m = wave_sum(acc_m);
        acc_ef = wave_sum(acc_ef);
        acc_ek = wave_sum(acc_ek);
        acc_nf = wave_sum(acc_nf);
        acc_im = wave_sum(acc_im);
        if (lane == 0) {
            sred[wv][0] = acc_m;
            sred[wv][1] = acc_ef;
            sred[wv][2] = acc_ek;
            sred[wv][3] = acc_nf;
            sired[wv] = acc_im;
        }
        __syncthreads();
        if (tid < NPART) {
            double s = 0.0;
            for (int w = 0; w < NW; ++w) s += sred[w][tid];
            G(J.part)[(int64_t)(e - J.tile_base) * NPART + tid] = s;
        }
        if (S::kFix && tid == NPART) {
            long long s = 0;
            for (int w = 0; w < NW; ++w) s += sired[w];
            G(J.ipart)[e - J.tile_base] = s;
        }
    }
}

// ---------------------------------------------------------- static fields
// phi0 clamped to [0, 1], psi = cos(theta) phi0 (input staging planes 1, 2).
template <class R>
__global__ __launch_bounds__(NT) void k_static(const double* __restrict__ in, R* __restrict__ st,
                                               int64_t pitch, int64_t n) {
    const int64_t o = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (o >= n) return;
    double z = in[pitch + o];
    z = z < 0.0 ? 0.0 : (z > 1.0 ? 1.0 : z);
    st[o] = (R)z;
    st[pitch + o] = (R)(in[2 * pitch + o] * z);
}

// Stationary solid when there are free particles: phi0 clamped to [0, 1] and
// cos(theta) as given (input staging planes 1, 2); the particles are added to
// them every step.
template <class R>
__global__ __launch_bounds__(NT) void k_part_base(const double* __restrict__ in, R* __restrict__ base,
                                                  int64_t pitch, int64_t n) {
    const int64_t o = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (o >= n) return;
    double z = in[pitch + o];
    z = z < 0.0 ? 0.0 : (z > 1.0 ? 1.0 : z);
    base[o] = (R)z;
    base[pitch + o] = (R)in[2 * pitch + o];
}

// Laplacian of psi (static wetting field), periodic, or mirrored at walls,
// evaluated in FP64 on psi = cos(theta) clamp(phi0) from the FP64 input planes
// (staging planes 1 and 2) and rounded once: a Laplacian of psi values already
// rounded to the storage type would carry their rounding (about 1e-7 in FP32)
// into the chemical potential next to every solid.
__device__ __forceinline__ double psi_in(const double* in, int64_t pitch, int64_t o) {
    double z = in[pitch + o];
    z = z < 0.0 ? 0.0 : (z > 1.0 ? 1.0 : z);
    return in[2 * pitch + o] * z;
}
template <class R>
__global__ __launch_bounds__(NT) void k_lap_psi(const double* __restrict__ in, R* __restrict__ st, int64_t pitch,
                                                int nx, int ny, int walls) {
    const int64_t o = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (o >= (int64_t)nx * ny) return;
    const int y = (int)(o / nx), x = (int)(o - (int64_t)y * nx);
    const int xe = imgof(x + 1, nx, walls & 2), xw = imgof(x - 1, nx, walls & 2);
    const int64_t rc = (int64_t)y * nx, rn = (int64_t)imgof(y + 1, ny, walls & 1) * nx;
    const int64_t rs = (int64_t)imgof(y - 1, ny, walls & 1) * nx;
    const double c4 = 4.0 * psi_in(in, pitch, o);
    const double ax = (psi_in(in, pitch, rc + xe) + psi_in(in, pitch, rc + xw)) +
                      (psi_in(in, pitch, rn + x) + psi_in(in, pitch, rs + x));
    const double dg = (psi_in(in, pitch, rn + xe) + psi_in(in, pitch, rn + xw)) +
                      (psi_in(in, pitch, rs + xe) + psi_in(in, pitch, rs + xw));
    st[2 * pitch + o] = (R)((ax - c4) * (2.0 / 3.0) + (dg - c4) * (1.0 / 6.0));
}

// ---------------------------------------------------------- free particles
// Procedure step 9: the indicator field phi0 = clamp(phi0_static + sum_k
// phi0_k, 0, 1) with phi0_k the tanh indicator of particle k (nearest periodic
// image, zero from R + PCUT D on), the owner of every node (the largest
// component; ties to the static solid, then the lower k), psi = cos(theta)
// phi0 with the owner's angle, and the Laplacian of psi.  One block per 64 x 8
// nodes, computing psi on a 1-node halo for the Laplacian; the particles whose
// support reaches the block are listed first, in index order, so every node
// sums the same terms in the same order.  A block that no particle reaches now
// and none reached at its previous call keeps its fields (touched[] remembers).
constexpr int PT_X = 64, PT_Y = 8, PT_NT = PT_X * PT_Y, PT_MAXLIST = 256;
template <class R>
__global__ __launch_bounds__(PT_NT) void k_part_static(const double* __restrict__ parts, int np,
                                                           const R* __restrict__ base, R* __restrict__ st,
                                                           int32_t* __restrict__ owner,
                                                           unsigned char* __restrict__ touched, int64_t pitch,
                                                           int nx, int ny, double D, int walls) {
    constexpr int HW = PT_X + 2, HH = PT_Y + 2;
    constexpr int NWV = PT_NT / 64;
    __shared__ int list[PT_MAXLIST];
    __shared__ int cnt;
    __shared__ double spsi[HH * HW];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int ntx = (nx + PT_X - 1) / PT_X;
    const int x0 = (int)(blockIdx.x % ntx) * PT_X, y0 = (int)(blockIdx.x / ntx) * PT_Y;
    const double cx = x0 + 0.5 * (PT_X - 1), cy = y0 + 0.5 * (PT_Y - 1);
    // candidate list in index order, built by the first wave alone (ballot
    // over 64 particles at a time), then one barrier
    if (wv == 0) {
        int c = 0;
        for (int k0 = 0; k0 < np; k0 += 64) {
            const int k = k0 + lane;
            bool h = false;
            if (k < np) {
                const double* q = parts + k * PSTRIDE;
                const double reach = q[PRAD] + PCUT * D + 1.0;  // + the halo of the Laplacian
                const double dx = fabs(perdw(cx - q[PX], nx, walls & 2)), dy = fabs(perdw(cy - q[PY], ny, walls & 1));
                h = dx <= 0.5 * PT_X + reach && dy <= 0.5 * PT_Y + reach;
            }
            const unsigned long long m = __ballot(h);
            const int pos = c + __popcll(m & ((1ull << lane) - 1ull));
            if (h && pos < PT_MAXLIST) list[pos] = k;
            c += __popcll(m);
        }
        if (lane == 0) cnt = c < PT_MAXLIST ? c : PT_MAXLIST;
    }
    __syncthreads();
    const unsigned char was = touched[blockIdx.x];
    if (cnt == 0 && !was) return;  // uniform: nothing here changed
    for (int i = tid; i < HH * HW; i += PT_NT) {
        const int ly = i / HW, lx = i - ly * HW;
        const int x = imgof(x0 + lx - 1, nx, walls & 2), y = imgof(y0 + ly - 1, ny, walls & 1);
        const int64_t o = (int64_t)y * nx + x;
        // the indicator in the storage's arithmetic (FP64 for FP64 storage)
        R sum = base[o], best = sum, cth = base[pitch + o];
        int own = -1;
        for (int j = 0; j < cnt; ++j) {
            const int k = list[j];
            const double* q = parts + k * PSTRIDE;
            const R dx = (R)perdw(x - q[PX], nx, walls & 2), dy = (R)perdw(y - q[PY], ny, walls & 1);
            const R rad = (R)q[PRAD], cut = rad + (R)(PCUT * D);
            // clearly outside the support: skip the square root and tanh
            if (dx * dx + dy * dy > cut * cut * R(1.000001)) continue;
            const R r = hypot(dx, dy);
            const R zk = r < cut ? R(0.5) + R(0.5) * tanh((rad - r) / (R)(D / 2.0)) : R(0);
            sum += zk;
            if (zk > best) {
                best = zk;
                own = k;
                cth = (R)q[PCOS];
            }
        }
        const R z = sum < R(0) ? R(0) : (sum > R(1) ? R(1) : sum);
        spsi[i] = (double)(cth * z);  // the stored value, as k_lap_psi would read it
        const bool inner = lx >= 1 && lx <= PT_X && ly >= 1 && ly <= PT_Y && x0 + lx - 1 < nx && y0 + ly - 1 < ny;
        if (inner) {
            st[o] = z;
            st[pitch + o] = cth * z;
            owner[o] = own;
        }
    }
    __syncthreads();
    const int x = x0 + (tid & (PT_X - 1)), y = y0 + tid / PT_X;
    if (tid == 0) touched[blockIdx.x] = cnt > 0;
    if (x >= nx || y >= ny) return;
    // the same stencil and rounding as k_lap_psi, on the stored psi values
    const int q = (tid / PT_X + 1) * HW + (tid & (PT_X - 1)) + 1;
    const R c4 = R(4) * (R)spsi[q];
    const R ax = ((R)spsi[q + 1] + (R)spsi[q - 1]) + ((R)spsi[q + HW] + (R)spsi[q - HW]);
    const R dg = ((R)spsi[q + HW + 1] + (R)spsi[q + HW - 1]) + ((R)spsi[q - HW + 1] + (R)spsi[q - HW - 1]);
    st[2 * pitch + (int64_t)y * nx + x] = (ax - c4) * R(2.0 / 3.0) + (dg - c4) * R(1.0 / 6.0);
}

// Procedure step 7 (Eq. Ff): per particle, over the nodes it owns,
// F_f = -sum rho f dt, T_f = -sum (x - x_p) x rho f dt, and the sums of
// phi0 rho and phi0 for the internal fluid density.  Each particle's support
// box is cut into PR_CH row bands, one block each; every block writes its own
// FP64 partials (fixed-order tree reduction), summed in band order by the
// update.
constexpr int PR_NT = 256, PR_CH = 8;
template <class R>
__global__ __launch_bounds__(PR_NT) void k_part_reduce(const double* __restrict__ parts,
                                                      const int32_t* __restrict__ owner,
                                                      const R* __restrict__ pf, const R* __restrict__ st,
                                                      int64_t pitch, int nx, int ny, double D, int walls,
                                                      double* __restrict__ acc) {
    __shared__ double sh[PR_NT][5];
    const int k = blockIdx.x / PR_CH, band = blockIdx.x % PR_CH, tid = threadIdx.x;
    const double* q = parts + k * PSTRIDE;
    const double reach = q[PRAD] + PCUT * D;
    int xl = (int)ceil(q[PX] - reach), yl = (int)ceil(q[PY] - reach);
    int w = (int)floor(q[PX] + reach) - xl + 1, h = (int)floor(q[PY] + reach) - yl + 1;
    if (walls & 2) {  // no image in x: the box is cut at the walls
        const int xh = xl + w - 1 < nx - 1 ? xl + w - 1 : nx - 1;
        xl = xl > 0 ? xl : 0;
        w = xh >= xl ? xh - xl + 1 : 0;
    }
    if (walls & 1) {  // likewise in y
        const int yh = yl + h - 1 < ny - 1 ? yl + h - 1 : ny - 1;
        yl = yl > 0 ? yl : 0;
        h = yh >= yl ? yh - yl + 1 : 0;
    }
    // a box narrower than the domain holds each node once, and there the plain
    // difference is the nearest periodic image
    const bool wrap_x = !(walls & 2) && w >= nx, wrap_y = !(walls & 1) && h >= ny;
    w = wrap_x ? nx : w;
    h = wrap_y ? ny : h;
    const int r0 = band * h / PR_CH, r1 = (band + 1) * h / PR_CH;
    double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = tid; i < (r1 - r0) * w; i += PR_NT) {
        const int iy = r0 + i / w, ix = i - (i / w) * w;
        const int xu = xl + ix, yu = yl + iy;
        const int x = wrapi(xu, nx), y = wrapi(yu, ny);
        const int64_t o = (int64_t)y * nx + x;
        if (owner[o] != k) continue;
        const double fx = (double)pf[o], fy = (double)pf[pitch + o], rho = (double)pf[2 * pitch + o];
        const double rx = wrap_x ? perd(x - q[PX], nx) : xu - q[PX];
        const double ry = wrap_y ? perd(y - q[PY], ny) : yu - q[PY];
        const double z = (double)st[o];
        a[0] -= fx;
        a[1] -= fy;
        a[2] -= rx * fy - ry * fx;
        a[3] += z * rho;
        a[4] += z;
    }
#pragma unroll
    for (int j = 0; j < 5; ++j) sh[tid][j] = a[j];
    __syncthreads();
    for (int s = PR_NT / 2; s > 0; s >>= 1) {
        if (tid < s) {
#pragma unroll
            for (int j = 0; j < 5; ++j) sh[tid][j] += sh[tid + s][j];
        }
        __syncthreads();
    }
    if (tid < 5) acc[(int64_t)blockIdx.x * 5 + tid] = sh[0][tid];
}

// Sec. 4.5 repulsion on a particle at (dx, dy) from the other centre (or from
// its mirror image across a wall); m scales the separation vector.
__device__ __forceinline__ double rep_scale(double d, double rsum, double xi, double eps) {
    if (d > rsum + xi) return 0.0;
    if (d >= rsum) return (rsum + xi - d) * (rsum + xi - d) / eps;
    return (rsum - d) / eps;
}

struct PartParams {
    double gx, gy;                       // gravity acting on the particles
    double xi, eps;                      // repulsion threshold and stiffness (eps <= 0: none)
    double wall[4];                      // wall planes y0, y1, x0, x1
    int walls;                           // bit w: wall[w] present
    int nx, ny;
    int bounce_x, bounce_y;              // bounce-back walls: no periodic image in x, y
};

// Procedure steps 8 and 10: Eq. (particle) by explicit Euler (dt = 1, every
// right-hand side at the old level), M_p = rho_p pi R^2, I_p = M_p R^2 / 2,
// V_p = pi R^2; rho of the internal fluid = sum phi0 rho / sum phi0 over the
// owned nodes; F^in = rho V_p du_p, T^in = I_p rho / rho_p dw_p carried to the
// next update.  A particle with rho_p <= 0 has prescribed motion: u_p and
// omega_p are held, the centre advances, F_f and T_f are still reported.
// One block of 1024 threads (np <= 1024): the particle-particle
// repulsion of particle k is split over PU_SPLIT(np) threads (partner j in
// steps of the split), whose partial sums thread k adds in a fixed order.  The
// old state of all particles is read before any thread writes, so the new
// state may replace it (nparts == parts, nout == out) or go elsewhere.
constexpr int PU_NT = 1024;
__host__ __device__ constexpr int pu_split(int np) {
    int s = 1;
    while (s * 2 * np <= PU_NT) s *= 2;
    return s;
}
__global__ __launch_bounds__(PU_NT) void k_part_update(const double* parts, const double* out,
                                                     const double* __restrict__ acc, int np, PartParams pp,
                                                     double* nparts, double* nout) {
    __shared__ double rx[PU_NT], ry[PU_NT];
    const int t = threadIdx.x, split = pu_split(np);
    {
        const int k = t / split, part = t % split;
        double sx = 0.0, sy = 0.0;
        if (k < np && pp.eps > 0.0) {
            const double* q = parts + k * PSTRIDE;
            const double R = q[PRAD];
            for (int j = part; j < np; j += split) {
                if (j == k) continue;
                const double* qj = parts + j * PSTRIDE;
                // far pairs (no image within the threshold) contribute nothing
                const double lim = R + qj[PRAD] + pp.xi;
                const double ax = fabs(q[PX] - qj[PX]), ay = fabs(q[PY] - qj[PY]);
                if ((ax > lim && (pp.bounce_x || pp.nx - ax > lim)) || (ay > lim && (pp.bounce_y || pp.ny - ay > lim)))
                    continue;
                const double dx = perdw(q[PX] - qj[PX], pp.nx, pp.bounce_x);
                const double dy = perdw(q[PY] - qj[PY], pp.ny, pp.bounce_y);
                const double m = rep_scale(hypot(dx, dy), R + qj[PRAD], pp.xi, pp.eps);
                sx += m * dx;
                sy += m * dy;
            }
        }
        rx[t] = sx;
        ry[t] = sy;
    }
    __syncthreads();
    const int k = t;
    const double PI = 3.14159265358979323846;
    double n[PSTRIDE], o7[QSTRIDE];
    if (k < np) {
        const double* q = parts + k * PSTRIDE;
        const double R = q[PRAD], rp = q[PRHO];
        const double V = PI * R * R, Mp = rp * V, Ip = Mp * R * R / 2.0;
        double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int c = 0; c < PR_CH; ++c)
            for (int j = 0; j < 5; ++j) a[j] += acc[((int64_t)k * PR_CH + c) * 5 + j];
        const double rin = a[4] > 0.0 ? a[3] / a[4] : 0.0;
        double frx = 0.0, fry = 0.0;
        if (pp.eps > 0.0) {
            for (int p = 0; p < split; ++p) {
                frx += rx[k * split + p];
                fry += ry[k * split + p];
            }
            for (int w = 0; w < 4; ++w) {
                if (!(pp.walls >> w & 1)) continue;
                const double dx = w < 2 ? 0.0 : 2.0 * (q[PX] - pp.wall[w]);
                const double dy = w < 2 ? 2.0 * (q[PY] - pp.wall[w]) : 0.0;
                const double m = rep_scale(hypot(dx, dy), 2.0 * R, pp.xi, pp.eps / 2.0);
                frx += m * dx;
                fry += m * dy;
            }
        }
        const double* po = out + k * QSTRIDE;
        for (int i = 0; i < PSTRIDE; ++i) n[i] = q[i];
        if (rp > 0.0) {  // free; rho_p <= 0: prescribed motion, u_p and omega_p held
            const double Fx = a[0] + po[QFINX] + (1.0 - rin / rp) * Mp * pp.gx + frx;
            const double Fy = a[1] + po[QFINY] + (1.0 - rin / rp) * Mp * pp.gy + fry;
            const double Tz = a[2] + po[QTIN];
            n[PUX] = q[PUX] + Fx / Mp;
            n[PUY] = q[PUY] + Fy / Mp;
            n[POM] = q[POM] + Tz / Ip;
        }
        n[PX] = q[PX] + q[PUX];
        n[PY] = q[PY] + q[PUY];
        if (!pp.bounce_x) n[PX] -= pp.nx * floor(n[PX] / pp.nx);
        if (!pp.bounce_y) n[PY] -= pp.ny * floor(n[PY] / pp.ny);
        o7[QFX] = a[0];
        o7[QFY] = a[1];
        o7[QT] = a[2];
        o7[QFINX] = rp > 0.0 ? rin * V * (n[PUX] - q[PUX]) : 0.0;
        o7[QFINY] = rp > 0.0 ? rin * V * (n[PUY] - q[PUY]) : 0.0;
        o7[QTIN] = rp > 0.0 ? Ip * rin / rp * (n[POM] - q[POM]) : 0.0;
        o7[QRHOIN] = rin;
    }
    __syncthreads();
    if (k < np) {
        for (int i = 0; i < PSTRIDE; ++i) nparts[k * PSTRIDE + i] = n[i];
        for (int i = 0; i < QSTRIDE; ++i) nout[k * QSTRIDE + i] = o7[i];
    }
}

// ------------------------------------------------------------ voxel solids
// A binary (voxel) solid is smoothed before it serves as phi0 by a few
// explicit steps of the standard Cahn-Hilliard equation on chi = 2 s - 1
// (Sec. 4.1 smooths its micro-CT solid this way): d chi/dt = lap mu,
// mu = chi^3 - chi - kappa lap chi, kappa = D^2/8 (planar equilibrium
// tanh(2 z / D), the indicator profile), isotropic Laplacian, periodic or
// mirrored at walls (bit 0: walls in y, 1: in x).  FP64: a one-off pass.
__device__ __forceinline__ double vox_lap(const double* c, int x, int y, int nx, int ny, int walls) {
    const int xe = imgof(x + 1, nx, walls & 2), xw = imgof(x - 1, nx, walls & 2);
    const int64_t rc = (int64_t)y * nx, rn = (int64_t)imgof(y + 1, ny, walls & 1) * nx;
    const int64_t rs = (int64_t)imgof(y - 1, ny, walls & 1) * nx;
    const double c4 = 4.0 * c[rc + x];
    const double ax = (c[rc + xe] + c[rc + xw]) + (c[rn + x] + c[rs + x]);
    const double dg = (c[rn + xe] + c[rn + xw]) + (c[rs + xe] + c[rs + xw]);
    return (ax - c4) * (2.0 / 3.0) + (dg - c4) * (1.0 / 6.0);
}
// mode 0: chi = 2 s - 1; 1: mu from chi; 2: chi += dtau lap mu (into out);
// 3: phi0 = clamp((1 + chi)/2, 0, 1)
__global__ __launch_bounds__(NT) void k_vox(const double* __restrict__ a, const double* __restrict__ b,
                                            double* __restrict__ out, int nx, int ny, int walls, double kappa,
                                            double dtau, int mode) {
    const int64_t o = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (o >= (int64_t)nx * ny) return;
    const int y = (int)(o / nx), x = (int)(o - (int64_t)y * nx);
    if (mode == 0) {
        out[o] = 2.0 * a[o] - 1.0;
    } else if (mode == 1) {
        const double c = a[o];
        out[o] = c * c * c - c - kappa * vox_lap(a, x, y, nx, ny, walls);
    } else if (mode == 2) {
        out[o] = a[o] + dtau * vox_lap(b, x, y, nx, ny, walls);
    } else {
        const double z = (1.0 + a[o]) * 0.5;
        out[o] = z < 0.0 ? 0.0 : (z > 1.0 ? 1.0 : z);
    }
}

// Fixed-order sum of the per-tile partials: res[k] = sum_i part[i][k], and
// (16-bit modes) the exact fixed-point mass as two 64-bit integers, ires[0]
// the sum of the tiles' upper halves (v >> 32) and ires[1] the sum of their
// lower 32 bits, so that mass = ires[0] 2^32 + ires[1] in units of 2^-40.
// A tile's partial is below 2^51 in magnitude; a single 64-bit total would
// wrap once |sum phi| passes 2^23, while the halves stay below 2^44 and 2^57
// for every domain of fewer than 2^31 nodes.
__global__ __launch_bounds__(NT) void k_final_sum(const double* __restrict__ part,
                                                  const int64_t* __restrict__ ipart, int ntiles,
                                                  double* __restrict__ res, int64_t* __restrict__ ires) {
    __shared__ double s[NT][NPART];
    __shared__ long long si[NT][2];
    double acc[NPART] = {0.0, 0.0, 0.0, 0.0};
    long long ah = 0, al = 0;
    for (int i = threadIdx.x; i < ntiles; i += NT) {
#pragma unroll
        for (int k = 0; k < NPART; ++k) acc[k] += part[(int64_t)i * NPART + k];
        if (ipart) {
            const long long v = ipart[i];
            ah += v >> 32;
            al += v & 0xffffffffLL;
        }
    }
#pragma unroll
    for (int k = 0; k < NPART; ++k) s[threadIdx.x][k] = acc[k];
    si[threadIdx.x][0] = ah;
    si[threadIdx.x][1] = al;
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
#pragma unroll
            for (int k = 0; k < NPART; ++k) s[threadIdx.x][k] += s[threadIdx.x + h][k];
            si[threadIdx.x][0] += si[threadIdx.x + h][0];
            si[threadIdx.x][1] += si[threadIdx.x + h][1];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int k = 0; k < NPART; ++k) res[k] = s[0][k];
        ires[0] = si[0][0];
        ires[1] = si[0][1];
    }
}

}  // namespace lbm
