// lbm_abi.hip -- host side of the C ABI declared in include/lbmgls.h.
//
// The library never allocates device memory: every domain lives in a caller
// workspace laid out as (256-byte aligned blocks)
//   pop[0], pop[1]        distributions, two copies (layout: lbm_device.h)
//   hist[0], hist[1]      previous-level phi, u, S (5 planes each)
//   stat                  phi0, psi, lap psi
//   stage                 5 FP64 planes: create() input, read() output
//   part / ipart / res    reduction partials and results
//   job                   the Job<S> descriptor read by the kernels
//   tiles                 the 64 x TY tile table
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lbm_device.h"
#include "lbmgls.h"

using namespace lbm;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            return fail(LBM_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));       \
    } while (0)

constexpr size_t ALIGN = 256;
size_t up(size_t v, size_t a = ALIGN) { return (v + a - 1) / a * a; }

struct Layout {
    int64_t pitch = 0;
    int ty = 8;
    int tiles_x = 0, tiles_y = 0, ntiles = 0;
    size_t pop_bytes = 0, hist_bytes = 0;
    size_t off_pop[2] = {0, 0}, off_hist[2] = {0, 0};
    size_t off_stat = 0, off_stage = 0, off_part = 0, off_ipart = 0, off_res = 0, off_ires = 0;
    size_t off_job = 0, off_tiles = 0, total = 0;
    // free particles (np > 0): static solid, owners, rho f planes, FP64 state
    size_t off_base = 0, off_owner = 0, off_pf = 0, off_parts = 0, off_pout = 0, off_pacc = 0, off_pscr = 0;
    size_t off_touch = 0;
    int pt_blocks = 0;  // 64 x 4 blocks of the particle indicator kernel
};

size_t real_size(int storage) { return storage == LBM_STORE_FP64 ? 8 : 4; }

size_t job_size(int storage) {
    switch (storage) {
        case LBM_STORE_FP64: return sizeof(Job<StF64>);
        case LBM_STORE_FP32: return sizeof(Job<StF32>);
        case LBM_STORE_FP16DEV: return sizeof(Job<StF16>);
        default: return sizeof(Job<StBF16>);
    }
}

int pick_ty(const lbm_params& p) {
    if (p.tile == LBM_TILE_64x4 || p.tile == LBM_TILE_64x8 || p.tile == LBM_TILE_64x16) return p.tile;
    if (p.tile == LBM_TILE_64x32 && p.storage != LBM_STORE_FP64) return p.tile;
    // default: 64 x 8 (the autotuner in the Python layer overrides per shape)
    return 8;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Job::walls of a domain: bit 0 walls in y, bit 1 walls in x.
int wall_bits(const lbm_params& p) { return (p.bounce_y ? 1 : 0) | (p.bounce_x ? 2 : 0); }

int validate(const lbm_params* p) {
    if (!p) return fail(LBM_EINVAL, "params is NULL");
    if (p->nx < 8 || p->ny < 8) return fail(LBM_EINVAL, "nx and ny must be >= 8");
    if ((int64_t)p->nx * p->ny >= (int64_t)1 << 31) return fail(LBM_EINVAL, "domain too large (2^31 nodes)");
    if (p->storage < LBM_STORE_FP64 || p->storage > LBM_STORE_BF16DEV)
        return fail(LBM_EUNSUPPORTED, "unknown storage mode");
    // FP32 and 16-bit planes are addressed by 32-bit byte offsets (4 GiB a
    // plane): at most 2^30 nodes, about the most their state fits on one
    // device anyway
    if (p->storage != LBM_STORE_FP64 && ((int64_t)p->nx * p->ny + 63) / 64 * 64 > (int64_t)1 << 30)
        return fail(LBM_EINVAL, "domain too large for FP32 or 16-bit storage (2^30 nodes)");
    if (!(p->tile == LBM_TILE_AUTO || p->tile == LBM_TILE_64x4 || p->tile == LBM_TILE_64x8 ||
          p->tile == LBM_TILE_64x16 || p->tile == LBM_TILE_64x32))
        return fail(LBM_EUNSUPPORTED, "unknown tile shape");
    if (p->tile == LBM_TILE_64x32 && p->storage == LBM_STORE_FP64)
        return fail(LBM_EUNSUPPORTED, "64x32 tiles are not built for FP64 (LDS)");
    if (!(p->d0 > 0.0 && p->d0 < 1.0)) return fail(LBM_EINVAL, "d0 must lie in (0, 1)");
    if (!finite_pos(p->sigma) || !finite_pos(p->D) || !finite_pos(p->M))
        return fail(LBM_EINVAL, "sigma, D and M must be positive");
    if (!finite_pos(p->rho1) || !finite_pos(p->rho2) || !finite_pos(p->mu1) || !finite_pos(p->mu2))
        return fail(LBM_EINVAL, "densities and viscosities must be positive");
    if (!(p->tau_phi > 0.5) || !std::isfinite(p->tau_phi)) return fail(LBM_EINVAL, "tau_phi must exceed 1/2");
    const double s[5] = {p->s0, p->s1, p->s2, p->s3, p->s4};
    for (double v : s)
        if (!(v > 0.0 && v < 2.0)) return fail(LBM_EINVAL, "relaxation rates must lie in (0, 2)");
    const double b[5] = {p->gx, p->gy, p->rho_ref, p->fbx, p->fby};
    for (double v : b)
        if (!std::isfinite(v)) return fail(LBM_EINVAL, "body-force parameters must be finite");
    if (!(p->solid_eps > 0.0 && p->solid_eps < 1.0)) return fail(LBM_EINVAL, "solid_eps must lie in (0, 1)");
    if (p->np < 0 || p->np > 1024) return fail(LBM_EINVAL, "np must lie in 0..1024");
    const double r[6] = {p->rep_xi, p->rep_eps, p->wall_x0, p->wall_x1, p->wall_y0, p->wall_y1};
    for (double v : r)
        if (!std::isfinite(v)) return fail(LBM_EINVAL, "repulsion and wall parameters must be finite");
    if (p->walls < 0 || p->walls > 15) return fail(LBM_EINVAL, "walls must lie in 0..15");
    if (p->bounce_y != 0 && p->bounce_y != 1) return fail(LBM_EINVAL, "bounce_y must be 0 or 1");
    if (p->bounce_x != 0 && p->bounce_x != 1) return fail(LBM_EINVAL, "bounce_x must be 0 or 1");
    if (p->h_form != 0 && p->h_form != 1) return fail(LBM_EINVAL, "h_form must be 0 or 1");
    return LBM_OK;
}

Layout layout(const lbm_params& p) {
    Layout L;
    L.ty = pick_ty(p);
    const int64_t N = (int64_t)p.nx * p.ny;
    L.pitch = (N + 63) / 64 * 64;
    L.tiles_x = (p.nx + TX - 1) / TX;
    L.tiles_y = (p.ny + L.ty - 1) / L.ty;
    L.ntiles = L.tiles_x * L.tiles_y;
    const size_t R = real_size(p.storage);
    if (p.storage == LBM_STORE_FP16DEV || p.storage == LBM_STORE_BF16DEV)
        L.pop_bytes = up(L.pitch * 8) + up(8 * L.pitch * 2) + up(9 * L.pitch * 2);
    else
        L.pop_bytes = up(18 * L.pitch * R);
    L.hist_bytes = up(5 * L.pitch * R);
    size_t o = 0;
    for (int k = 0; k < 2; ++k) { L.off_pop[k] = o; o += L.pop_bytes; }
    for (int k = 0; k < 2; ++k) { L.off_hist[k] = o; o += L.hist_bytes; }
    L.off_stat = o;  o += up(3 * L.pitch * R);
    L.off_stage = o; o += up(5 * L.pitch * 8);
    L.off_part = o;  o += up((size_t)L.ntiles * NPART * 8);
    L.off_ipart = o; o += up((size_t)L.ntiles * 8);
    L.off_res = o;   o += up(8 * 8);
    L.off_ires = o;  o += up(8 * 8);
    L.off_job = o;   o += up(job_size(p.storage));
    L.off_tiles = o; o += up((size_t)L.ntiles * sizeof(TileEntry));
    if (p.np > 0) {
        L.off_base = o;  o += up(2 * L.pitch * R);
        L.off_owner = o; o += up(L.pitch * 4);
        L.off_pf = o;    o += up(3 * L.pitch * R);
        L.off_parts = o; o += up((size_t)p.np * PSTRIDE * 8);
        L.off_pout = o;  o += up((size_t)p.np * QSTRIDE * 8);
        L.off_pacc = o;  o += up((size_t)p.np * PR_CH * 5 * 8);
        L.off_pscr = o;  o += up((size_t)p.np * (PSTRIDE + QSTRIDE) * 8);
        L.pt_blocks = ((p.nx + PT_X - 1) / PT_X) * ((p.ny + PT_Y - 1) / PT_Y);
        L.off_touch = o; o += up((size_t)L.pt_blocks);
    }
    L.total = o;
    return L;
}

template <class R>
void fill_coef(const lbm_params& p, Coef<R>& c) {
    const double a = p.d0, one_a = 1.0 - a;
    const double w0 = one_a * one_a, w1 = a * one_a / 2.0, w2 = a * a / 4.0;
    const double n1 = a, n2 = a * one_a;
    const double eta = p.M / ((p.tau_phi - 0.5) * a);
    c.a = (R)a; c.one_a = (R)one_a;
    c.w0 = (R)w0; c.w1 = (R)w1; c.w2 = (R)w2;
    c.inv_n1 = (R)(1.0 / n1); c.inv_n2 = (R)(1.0 / n2); c.inv_n11 = (R)(1.0 / (n1 * n1));
    c.inv_n12 = (R)(1.0 / (n1 * n2)); c.inv_n22 = (R)(1.0 / (n2 * n2));
    c.eta = (R)eta;
    c.s0 = (R)p.s0; c.s1 = (R)p.s1; c.s1phi = (R)(1.0 / p.tau_phi); c.s2 = (R)p.s2;
    c.s3 = (R)p.s3; c.s4 = (R)p.s4;
    const double s = p.sigma, D = p.D;
    c.k3s_D = (R)(3.0 * s / D); c.k3Ds_8 = (R)(3.0 * D * s / 8.0); c.k9s_D = (R)(9.0 * s / D);
    c.k3s_4D = (R)(3.0 * s / (4.0 * D)); c.k3Ds_16 = (R)(3.0 * D * s / 16.0);
    c.k9s_2D = (R)(9.0 * s / (2.0 * D));
    c.kS = (R)(p.M * (p.rho1 - p.rho2) / 2.0);
    c.drho = (R)((p.rho1 - p.rho2) / 2.0); c.rho2 = (R)p.rho2;
    c.dmu = (R)((p.mu1 - p.mu2) / 2.0); c.mu2 = (R)p.mu2;
    c.gx = (R)p.gx; c.gy = (R)p.gy; c.rho_ref = (R)p.rho_ref; c.fbx = (R)p.fbx; c.fby = (R)p.fby;
    c.solid_eps = (R)p.solid_eps;
    c.ka = (R)(one_a / 2.0);
    c.Pfac = (R)(a / (1.0 - w0));
    c.Pw0 = (R)(w0 / one_a);
    const double K = 1.0 - a;
    c.K2 = (R)(K / 2.0);
    if (p.h_form == 1) {  // as printed: K [(1 - d0)/s0 - (2 - 4 d0) tau_a + (1 - 3 d0)/2]
        c.Hc0 = (R)(K * (one_a / p.s0 + (1.0 - 3.0 * a) / 2.0));
        c.Hc1 = (R)(K * (2.0 - 4.0 * a));
    } else {              // first-order moments: -K (1 - 3 d0)(tau_a - 1/2)
        c.Hc0 = (R)(K * (1.0 - 3.0 * a) / 2.0);
        c.Hc1 = (R)(K * (1.0 - 3.0 * a));
    }
    // 16-bit modes: power-of-two scales that bring the typical magnitude of
    // the moving phase-field populations (w1 eta 3 sigma / D) and of the flow
    // populations (pressure scale) to about one.
    const double gmag = w1 * eta * 3.0 * s / D;
    double pmag = 3.0 * s / D;
    pmag = std::fmax(pmag, p.rho1 * std::fabs(p.gx) * p.nx + p.rho1 * std::fabs(p.gy) * p.ny);
    pmag = std::fmax(pmag, std::fabs(p.fbx) * p.nx + std::fabs(p.fby) * p.ny);
    pmag *= one_a / 2.0;
    int kg = (int)std::lround(std::log2(1.0 / gmag));
    kg = kg < 0 ? 0 : (kg > 16 ? 16 : kg);  // 40 - kg >= 24 keeps FP16 codes exact in fixed point
    int kf = (int)std::lround(std::log2(1.0 / pmag));
    kf = kf < 0 ? 0 : (kf > 24 ? 24 : kf);
    c.sg = std::ldexp(1.0f, kg); c.isg = std::ldexp(1.0f, -kg);
    c.sf = std::ldexp(1.0f, kf); c.isf = std::ldexp(1.0f, -kf);
    c.gfix = std::ldexp(1.0f, FIX_BITS - kg);
}

}  // namespace

// ----------------------------------------------------------------- domain
struct lbm_domain {
    lbm_params p;
    Layout L;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    int64_t steps = 0;
    int64_t check_every = 0;
    bool failed = false;
    double last_ms = 0.0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    lbm_batch* batch = nullptr;
    std::vector<unsigned char> job;  // host image of the Job<S> descriptor
    std::vector<TileEntry> tiles;
};

namespace {

template <class S>
void make_job(lbm_domain* d, int32_t n_active, int64_t step0, bool with_out, int32_t tile_base,
              Job<S>& J) {
    using R = typename S::R;
    std::memset(&J, 0, sizeof J);
    const Layout& L = d->L;
    char* ws = d->ws;
    for (int k = 0; k < 2; ++k) {
        char* base = ws + L.off_pop[k];
        if constexpr (S::kFix) {
            J.pop[k].g0 = (int64_t*)base;
            J.pop[k].gm = (uint16_t*)(base + up(L.pitch * 8));
            J.pop[k].fm = (uint16_t*)(base + up(L.pitch * 8) + up(8 * L.pitch * 2));
        } else {
            J.pop[k].p = (R*)base;
        }
        J.hist[k] = (R*)(ws + L.off_hist[k]);
    }
    J.stat = (R*)(ws + L.off_stat);
    J.in = (const double*)(ws + L.off_stage);
    J.out = with_out ? (double*)(ws + L.off_stage) : nullptr;
    J.part = (double*)(ws + L.off_part);
    J.ipart = (int64_t*)(ws + L.off_ipart);
    J.pitch = L.pitch;
    J.step0 = step0;
    J.nx = d->p.nx;
    J.ny = d->p.ny;
    J.n_active = n_active;
    J.tile_base = tile_base;
    J.np = d->p.np;
    J.walls = wall_bits(d->p);
    if (d->p.np > 0) {
        J.parts = (const double*)(ws + L.off_parts);
        J.owner = (const int32_t*)(ws + L.off_owner);
        J.pf = (R*)(ws + L.off_pf);
    }
    fill_coef<R>(d->p, J.c);
}

template <class S>
int upload_job(lbm_domain* d, int32_t n_active, bool with_out) {
    Job<S> J;
    make_job<S>(d, n_active, d->steps, with_out, 0, J);
    std::memcpy(d->job.data(), &J, sizeof J);
    HIPCHK(hipMemcpyAsync(d->ws + d->L.off_job, d->job.data(), sizeof J, hipMemcpyHostToDevice, d->stream));
    return LBM_OK;
}

template <class S, int TY, int MODE>
int launch_tiles(lbm_domain* d, int t) {
    const Job<S>* J = (const Job<S>*)(d->ws + d->L.off_job);
    const TileEntry* T = (const TileEntry*)(d->ws + d->L.off_tiles);
    const dim3 grid(d->L.ntiles), block(TileCfg<TY>::NT);
    const bool part = MODE != MODE_INIT && d->p.np > 0, wall = wall_bits(d->p) != 0;
    if (part && wall)
        hipLaunchKernelGGL((k_tile<S, TY, MODE, true, true>), grid, block, 0, d->stream, J, T, d->L.ntiles, t);
    else if (part)
        hipLaunchKernelGGL((k_tile<S, TY, MODE, true>), grid, block, 0, d->stream, J, T, d->L.ntiles, t);
    else if (wall)
        hipLaunchKernelGGL((k_tile<S, TY, MODE, false, true>), grid, block, 0, d->stream, J, T, d->L.ntiles, t);
    else
        hipLaunchKernelGGL((k_tile<S, TY, MODE>), grid, block, 0, d->stream, J, T, d->L.ntiles, t);
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

template <class S, int MODE>
int launch_tiles_ty(lbm_domain* d, int t) {
    switch (d->L.ty) {
        case 4: return launch_tiles<S, 4, MODE>(d, t);
        case 16: return launch_tiles<S, 16, MODE>(d, t);
        case 32:
            if constexpr (sizeof(typename S::R) == 4) return launch_tiles<S, 32, MODE>(d, t);
            return fail(LBM_EUNSUPPORTED, "64x32 tiles are not built for FP64");
        default: return launch_tiles<S, 8, MODE>(d, t);
    }
}

// Reductions at the current level; res[0..3] = mass, E_F, E_K, #non-finite.
template <class S>
int reduce(lbm_domain* d, bool with_out, double res[NPART], int64_t* imass = nullptr) {
    int rc = upload_job<S>(d, 0, with_out);
    if (rc) return rc;
    if ((rc = launch_tiles_ty<S, MODE_OUT>(d, 0))) return rc;
    double* r = (double*)(d->ws + d->L.off_res);
    int64_t* ir = (int64_t*)(d->ws + d->L.off_ires);
    hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(NT), 0, d->stream,
                       (const double*)(d->ws + d->L.off_part),
                       S::kFix ? (const int64_t*)(d->ws + d->L.off_ipart) : nullptr, d->L.ntiles, r, ir);
    HIPCHK(hipGetLastError());
    double hr[NPART];
    int64_t hi[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(hr, r, sizeof hr, hipMemcpyDeviceToHost, d->stream));
    HIPCHK(hipMemcpyAsync(hi, ir, sizeof hi, hipMemcpyDeviceToHost, d->stream));
    HIPCHK(hipStreamSynchronize(d->stream));
    for (int k = 0; k < NPART; ++k) res[k] = hr[k];
    if (imass) {  // normalised: imass[0] 2^32 + imass[1], 0 <= imass[1] < 2^32
        imass[0] = hi[0] + (hi[1] >> 32);
        imass[1] = hi[1] & 0xffffffffLL;
    }
    return LBM_OK;
}

// Procedure step 9: phi0, psi, the node owners and the Laplacian of psi from
// the stationary solid and the particles at their current positions.  With
// all = true every block recomputes (after create or import); otherwise
// blocks no particle reaches now or reached last time keep their fields.
template <class R>
int particle_statics(lbm_domain* d, bool all = false) {
    const Layout& L = d->L;
    if (all) HIPCHK(hipMemsetAsync(d->ws + L.off_touch, 1, (size_t)L.pt_blocks, d->stream));
    hipLaunchKernelGGL((k_part_static<R>), dim3((unsigned)L.pt_blocks), dim3(PT_X * PT_Y), 0, d->stream,
                       (const double*)(d->ws + L.off_parts), d->p.np, (const R*)(d->ws + L.off_base),
                       (R*)(d->ws + L.off_stat), (int32_t*)(d->ws + L.off_owner),
                       (unsigned char*)(d->ws + L.off_touch), L.pitch, d->p.nx, d->p.ny, d->p.D,
                       wall_bits(d->p));
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

// Procedure steps 7, 8 and 10 from the rho f planes of the last macroscopic
// update: force and torque sums, then the particle update into (nparts, nout)
// (the particle buffers themselves, or scratch for a preview).
template <class R>
int particle_update(lbm_domain* d, double* nparts, double* nout) {
    const Layout& L = d->L;
    const lbm_params& p = d->p;
    hipLaunchKernelGGL((k_part_reduce<R>), dim3((unsigned)(p.np * PR_CH)), dim3(PR_NT), 0, d->stream,
                       (const double*)(d->ws + L.off_parts), (const int32_t*)(d->ws + L.off_owner),
                       (const R*)(d->ws + L.off_pf), (const R*)(d->ws + L.off_stat), L.pitch, p.nx, p.ny, p.D,
                       wall_bits(p), (double*)(d->ws + L.off_pacc));
    HIPCHK(hipGetLastError());
    PartParams pp;
    pp.gx = p.gx;
    pp.gy = p.gy;
    pp.xi = p.rep_xi;
    pp.eps = p.rep_eps;
    pp.wall[0] = p.wall_y0;
    pp.wall[1] = p.wall_y1;
    pp.wall[2] = p.wall_x0;
    pp.wall[3] = p.wall_x1;
    pp.walls = p.walls;
    pp.nx = p.nx;
    pp.ny = p.ny;
    pp.bounce_x = p.bounce_x;
    pp.bounce_y = p.bounce_y;
    hipLaunchKernelGGL(k_part_update, dim3(1), dim3(PU_NT), 0, d->stream, (const double*)(d->ws + L.off_parts),
                       (const double*)(d->ws + L.off_pout), (const double*)(d->ws + L.off_pacc), p.np, pp, nparts,
                       nout);
    HIPCHK(hipGetLastError());
    return LBM_OK;
}

// Procedure steps 7-10 after a step: the update in place, then the
// regenerated indicator for the next step.
template <class R>
int particle_step(lbm_domain* d) {
    int rc = particle_update<R>(d, (double*)(d->ws + d->L.off_parts), (double*)(d->ws + d->L.off_pout));
    if (rc) return rc;
    return particle_statics<R>(d);
}

template <class S>
int create_impl(lbm_domain* d, const double* phi, const double* phi0, const double* cth,
                const double* ux, const double* uy, const double* parts) {
    using R = typename S::R;
    const Layout& L = d->L;
    const int64_t N = (int64_t)d->p.nx * d->p.ny;
    std::vector<double> stage((size_t)5 * L.pitch, 0.0);
    for (int64_t o = 0; o < N; ++o) {
        stage[o] = phi[o];
        stage[L.pitch + o] = phi0[o];
        stage[2 * L.pitch + o] = cth ? cth[o] : 0.0;
        stage[3 * L.pitch + o] = ux ? ux[o] : 0.0;
        stage[4 * L.pitch + o] = uy ? uy[o] : 0.0;
    }
    HIPCHK(hipMemcpyAsync(d->ws + L.off_stage, stage.data(), stage.size() * 8, hipMemcpyHostToDevice,
                          d->stream));
    HIPCHK(hipMemcpyAsync(d->ws + L.off_tiles, d->tiles.data(), d->tiles.size() * sizeof(TileEntry),
                          hipMemcpyHostToDevice, d->stream));
    R* st = (R*)(d->ws + L.off_stat);
    const unsigned nb = (unsigned)((N + NT - 1) / NT);
    std::vector<double> pstate;
    if (d->p.np > 0) {
        // the stationary solid goes to the base planes; phi0, psi and the
        // owners come from it and the particles
        hipLaunchKernelGGL((k_part_base<R>), dim3(nb), dim3(NT), 0, d->stream,
                           (const double*)(d->ws + L.off_stage), (R*)(d->ws + L.off_base), L.pitch, N);
        HIPCHK(hipGetLastError());
        pstate.assign(parts, parts + (size_t)d->p.np * PSTRIDE);
        HIPCHK(hipMemcpyAsync(d->ws + L.off_parts, pstate.data(), pstate.size() * 8, hipMemcpyHostToDevice,
                              d->stream));
        HIPCHK(hipMemsetAsync(d->ws + L.off_pout, 0, (size_t)d->p.np * QSTRIDE * 8, d->stream));
        int rc = particle_statics<R>(d, true);
        if (rc) return rc;
    } else {
        hipLaunchKernelGGL((k_static<R>), dim3(nb), dim3(NT), 0, d->stream,
                           (const double*)(d->ws + L.off_stage), st, L.pitch, N);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL((k_lap_psi<R>), dim3(nb), dim3(NT), 0, d->stream,
                           (const double*)(d->ws + L.off_stage), st, L.pitch, d->p.nx, d->p.ny, wall_bits(d->p));
        HIPCHK(hipGetLastError());
    }
    int rc = upload_job<S>(d, 0, false);
    if (rc) return rc;
    if ((rc = launch_tiles_ty<S, MODE_INIT>(d, 0))) return rc;
    HIPCHK(hipStreamSynchronize(d->stream));
    return LBM_OK;
}

template <class S>
int step_impl(lbm_domain* d, int64_t nsteps) {
    int64_t done = 0;
    double total_ms = 0.0;
    int64_t timed = 0;
    while (done < nsteps) {
        int64_t chunk = nsteps - done;
        if (d->check_every > 0) {
            const int64_t to_check = d->check_every - (d->steps % d->check_every);
            if (chunk > to_check) chunk = to_check;
        }
        if (chunk > (int64_t)1 << 30) chunk = (int64_t)1 << 30;
        int rc = upload_job<S>(d, (int32_t)chunk, false);
        if (rc) return rc;
        HIPCHK(hipEventRecord(d->ev0, d->stream));
        for (int64_t t = 0; t < chunk; ++t) {
            if ((rc = launch_tiles_ty<S, MODE_STEP>(d, (int)t))) return rc;
            // the particles move after every macroscopic update except the
            // initial one (the step-0 launch recomputes it)
            if (d->p.np > 0 && d->steps + t >= 1 && (rc = particle_step<typename S::R>(d))) return rc;
        }
        HIPCHK(hipEventRecord(d->ev1, d->stream));
        d->steps += chunk;
        done += chunk;
        if (d->check_every > 0 && d->steps % d->check_every == 0) {
            double res[NPART];
            if ((rc = reduce<S>(d, false, res, nullptr))) return rc;
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, d->ev0, d->ev1));
            total_ms += ms;
            timed += chunk;
            if (res[3] > 0.0) {
                d->failed = true;
                return fail(LBM_ENONFINITE, "non-finite phi, u or P at step " + std::to_string(d->steps));
            }
        } else if (done == nsteps) {
            HIPCHK(hipEventSynchronize(d->ev1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, d->ev0, d->ev1));
            total_ms += ms;
            timed += chunk;
        }
    }
    d->last_ms = timed ? total_ms / (double)timed : 0.0;
    return LBM_OK;
}

template <class S>
int read_impl(lbm_domain* d, double* phi, double* ux, double* uy, double* P) {
    double res[NPART];
    int rc = reduce<S>(d, true, res, nullptr);
    if (rc) return rc;
    const int64_t N = (int64_t)d->p.nx * d->p.ny;
    double* outs[4] = {phi, ux, uy, P};
    for (int k = 0; k < 4; ++k)
        if (outs[k])
            HIPCHK(hipMemcpyAsync(outs[k], d->ws + d->L.off_stage + (size_t)k * d->L.pitch * 8, N * 8,
                                  hipMemcpyDeviceToHost, d->stream));
    HIPCHK(hipStreamSynchronize(d->stream));
    return LBM_OK;
}

template <class F>
int dispatch(int storage, F&& f) {
    switch (storage) {
        case LBM_STORE_FP64: return f(StF64{});
        case LBM_STORE_FP32: return f(StF32{});
        case LBM_STORE_FP16DEV: return f(StF16{});
        case LBM_STORE_BF16DEV: return f(StBF16{});
    }
    return fail(LBM_EUNSUPPORTED, "unknown storage mode");
}

int usable(const lbm_domain* d) {
    if (!d) return fail(LBM_EINVAL, "domain is NULL");
    if (d->failed) return fail(LBM_ESTATE, "domain failed a finiteness check; import a state first");
    return LBM_OK;
}

}  // namespace

extern "C" {

const char* lbm_last_error(void) { return g_err.c_str(); }

void lbm_default_params(lbm_params* p, int32_t nx, int32_t ny) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->nx = nx; p->ny = ny;
    p->storage = LBM_STORE_FP32;
    p->tile = LBM_TILE_AUTO;
    p->d0 = 0.4; p->sigma = 1e-3; p->D = 4.0; p->M = 0.1;
    p->rho1 = 1.0; p->rho2 = 1.0; p->mu1 = 0.1; p->mu2 = 0.1;
    p->tau_phi = 1.0;
    p->s0 = p->s1 = p->s2 = p->s3 = p->s4 = 1.0;
    p->solid_eps = 1e-2;
}

size_t lbm_workspace_bytes(const lbm_params* p) {
    if (validate(p) != LBM_OK) return 0;
    return layout(*p).total;
}

namespace {
int create_common(const lbm_params* p, void* dev_workspace, size_t bytes, void* hip_stream,
                  const double* phi, const double* phi0, const double* cos_theta, const double* ux,
                  const double* uy, const double* parts, lbm_domain** out) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(p);
    if (rc) return rc;
    if (!phi || !phi0) return fail(LBM_EINVAL, "phi and phi0 are required");
    if (!dev_workspace) return fail(LBM_EINVAL, "workspace is NULL");
    if ((uintptr_t)dev_workspace % ALIGN) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
    const Layout L = layout(*p);
    if (bytes < L.total)
        return fail(LBM_ENOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
    const int64_t N = (int64_t)p->nx * p->ny;
    for (int64_t o = 0; o < N; ++o) {
        if (!std::isfinite(phi[o]) || !std::isfinite(phi0[o]) ||
            (cos_theta && !(std::fabs(cos_theta[o]) <= 1.0)) || (ux && !std::isfinite(ux[o])) ||
            (uy && !std::isfinite(uy[o])))
            return fail(LBM_EINVAL, "non-finite or out-of-range input at node " + std::to_string(o));
    }
    lbm_domain* d = new lbm_domain();
    d->p = *p;
    d->L = L;
    d->stream = (hipStream_t)hip_stream;
    d->ws = (char*)dev_workspace;
    d->job.resize(job_size(p->storage));
    // Band-major tile order: bands of BAND tiles (512 columns) are walked top
    // to bottom, row by row inside a band.  Each XCD gets a contiguous run of
    // the table (xcd_remap), so the tile above a tile ran only BAND tiles
    // earlier on the same XCD and the halo rows they share are still in its
    // L2, while every row segment read is 2 KB contiguous per plane.
    // (Measured: a plain row-major order re-reads the halo from memory on
    // wide grids; a column-major order strides through memory at the row
    // pitch and is slower still.)  Rows of up to 32 tiles (2048 columns) stay
    // row-major: the tile rows an XCD runs then hold each other's halos in its
    // L2 (on 2048 x 1024, row-major measured 7-8% faster than bands of 8 in
    // FP32 and FP64, and the same in 16-bit storage).
    const int BAND = L.tiles_x <= 32 ? L.tiles_x : 8;
    for (int b0 = 0; b0 < L.tiles_x; b0 += BAND)
        for (int ty = 0; ty < L.tiles_y; ++ty)
            for (int tx = b0; tx < L.tiles_x && tx < b0 + BAND; ++tx)
                d->tiles.push_back(TileEntry{0, tx * TX, ty * L.ty, 0});
    if (hipEventCreate(&d->ev0) != hipSuccess || hipEventCreate(&d->ev1) != hipSuccess) {
        delete d;
        return fail(LBM_EDEVICE, "hipEventCreate failed");
    }
    rc = dispatch(p->storage,
                  [&](auto s) { return create_impl<decltype(s)>(d, phi, phi0, cos_theta, ux, uy, parts); });
    if (rc) {
        lbm_destroy(d);
        return rc;
    }
    *out = d;
    return LBM_OK;
}
}  // namespace

int lbm_create(const lbm_params* p, void* dev_workspace, size_t bytes, void* hip_stream,
               const double* phi, const double* phi0, const double* cos_theta, const double* ux,
               const double* uy, lbm_domain** out) {
    if (p && p->np != 0) {
        if (out) *out = nullptr;
        return fail(LBM_EINVAL, "np > 0: use lbm_create_particles");
    }
    return create_common(p, dev_workspace, bytes, hip_stream, phi, phi0, cos_theta, ux, uy, nullptr, out);
}

int lbm_create_particles(const lbm_params* p, void* dev_workspace, size_t bytes, void* hip_stream,
                         const double* phi, const double* phi0, const double* cos_theta, const double* ux,
                         const double* uy, const double* particles, lbm_domain** out) {
    if (out) *out = nullptr;
    if (p && p->np > 0) {
        if (!particles) return fail(LBM_EINVAL, "particles is NULL");
        for (int k = 0; k < p->np && k <= 1024; ++k) {
            const double* q = particles + (size_t)k * PSTRIDE;
            for (int i = 0; i < PSTRIDE; ++i)
                if (!std::isfinite(q[i])) return fail(LBM_EINVAL, "non-finite particle " + std::to_string(k));
            if (!(q[PRAD] > 0.0) || !(std::fabs(q[PCOS]) <= 1.0))
                return fail(LBM_EINVAL, "particle " + std::to_string(k) + ": R must be positive, |cos theta| <= 1");
        }
    }
    return create_common(p, dev_workspace, bytes, hip_stream, phi, phi0, cos_theta, ux, uy, particles, out);
}

size_t lbm_smooth_workspace_bytes(int32_t nx, int32_t ny) {
    if (nx < 8 || ny < 8 || (int64_t)nx * ny >= (int64_t)1 << 31) return 0;
    return 3 * up((size_t)nx * ny * 8);
}

namespace {
// The arguments of a smoothing call, checked; dtau resolved.
int smooth_args(const lbm_params* p, int32_t iters, double& dtau, const double* solid, const double* phi0) {
    int rc = validate(p);
    if (rc) return rc;
    if (!solid || !phi0) return fail(LBM_EINVAL, "NULL argument");
    if (iters < 0 || iters > (1 << 20)) return fail(LBM_EINVAL, "iters out of range");
    if (!std::isfinite(dtau)) return fail(LBM_EINVAL, "dtau must be finite");
    const double kappa = p->D * p->D / 8.0, L = 16.0 / 3.0;
    // default: half the stability limit of the step linearised about chi = +-1
    if (dtau <= 0.0) dtau = 0.5 / (kappa * L * L + 2.0 * L);
    return LBM_OK;
}

// The smoothing itself on three FP64 device planes of N nodes each: the host
// solid is copied into the third, `iters` explicit steps alternate the first
// and third, and phi0 is copied back.  Blocks on the stream.
int smooth_run(const lbm_params* p, int32_t iters, double dtau, hipStream_t st, double* chi, double* mu,
               double* nxt, const double* solid, double* phi0) {
    const int64_t N = (int64_t)p->nx * p->ny;
    const double kappa = p->D * p->D / 8.0;
    const unsigned nb = (unsigned)((N + NT - 1) / NT);
    const int w = wall_bits(*p);
    HIPCHK(hipMemcpyAsync(nxt, solid, (size_t)N * 8, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_vox, dim3(nb), dim3(NT), 0, st, nxt, nullptr, chi, p->nx, p->ny, w, kappa, dtau, 0);
    for (int32_t it = 0; it < iters; ++it) {
        hipLaunchKernelGGL(k_vox, dim3(nb), dim3(NT), 0, st, chi, nullptr, mu, p->nx, p->ny, w, kappa, dtau, 1);
        hipLaunchKernelGGL(k_vox, dim3(nb), dim3(NT), 0, st, chi, mu, nxt, p->nx, p->ny, w, kappa, dtau, 2);
        std::swap(chi, nxt);
    }
    hipLaunchKernelGGL(k_vox, dim3(nb), dim3(NT), 0, st, chi, nullptr, nxt, p->nx, p->ny, w, kappa, dtau, 3);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(phi0, nxt, (size_t)N * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return LBM_OK;
}

// Scratch of the allocation-free smoothing: three FP64 planes of at most
// LBM_NOALLOC_MAX_NODES nodes, one copy per device for the life of the
// process.  In host code `scratch` is only a stand-in for the symbol: its
// device address, per device, comes from hipGetSymbolAddress at the first
// call on that device and is the only form in which it is passed on.
__device__ __align__(256) double scratch[3 * (size_t)LBM_NOALLOC_MAX_NODES];
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_ptr[MAX_DEVICES] = {};

int scratch_for_current_device(double** out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(LBM_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(LBM_EDEVICE, "no device address for the scratch array");
        scratch_ptr[dev] = (double*)ptr;
    }
    *out = scratch_ptr[dev];
    return LBM_OK;
}
}  // namespace

int lbm_smooth_solid(const lbm_params* p, int32_t iters, double dtau, void* dev_workspace, size_t bytes,
                     void* hip_stream, const double* solid, double* phi0) {
    int rc = smooth_args(p, iters, dtau, solid, phi0);
    if (rc) return rc;
    if (!dev_workspace) return fail(LBM_EINVAL, "NULL argument");
    if ((uintptr_t)dev_workspace % ALIGN) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = lbm_smooth_workspace_bytes(p->nx, p->ny);
    if (bytes < need) return fail(LBM_ENOMEM, "workspace too small");
    const size_t plane = up((size_t)p->nx * p->ny * 8);
    char* ws = (char*)dev_workspace;
    return smooth_run(p, iters, dtau, (hipStream_t)hip_stream, (double*)ws, (double*)(ws + plane),
                      (double*)(ws + 2 * plane), solid, phi0);
}

int lbm_smooth_solid_noalloc(const lbm_params* p, int32_t iters, double dtau, void* hip_stream,
                             const double* solid, double* phi0) {
    int rc = smooth_args(p, iters, dtau, solid, phi0);
    if (rc) return rc;
    const int64_t N = (int64_t)p->nx * p->ny;
    if (N > (int64_t)LBM_NOALLOC_MAX_NODES)
        return fail(LBM_EINVAL, "grid of " + std::to_string(N) + " nodes exceeds the " +
                                    std::to_string((long long)LBM_NOALLOC_MAX_NODES) +
                                    "-node limit of the allocation-free smoothing");
    double* base = nullptr;
    if ((rc = scratch_for_current_device(&base))) return rc;
    const size_t plane = (size_t)LBM_NOALLOC_MAX_NODES;
    return smooth_run(p, iters, dtau, (hipStream_t)hip_stream, base, base + plane, base + 2 * plane, solid,
                      phi0);
}

int lbm_particles(lbm_domain* d, double* state, double* outputs) {
    int rc = usable(d);
    if (rc) return rc;
    if (d->p.np == 0) return LBM_OK;
    // A step launch computes the macroscopic fields of its level first; the
    // particle update that belongs to the current level (procedure steps
    // 7-10 after steps 3-6) therefore runs after the next launch.  Here it is
    // computed now from a macroscopic pass at the current level, into scratch,
    // without changing the domain.
    const size_t ps = (size_t)d->p.np * PSTRIDE * 8, qs = (size_t)d->p.np * QSTRIDE * 8;
    const char* src_p = d->ws + d->L.off_parts;
    const char* src_q = d->ws + d->L.off_pout;
    if (d->steps >= 1) {
        rc = dispatch(d->p.storage, [&](auto s) -> int {
            using S = decltype(s);
            double res[NPART];
            int r = reduce<S>(d, false, res, nullptr);
            if (r) return r;
            double* scr = (double*)(d->ws + d->L.off_pscr);
            return particle_update<typename S::R>(d, scr, scr + (size_t)d->p.np * PSTRIDE);
        });
        if (rc) return rc;
        src_p = d->ws + d->L.off_pscr;
        src_q = src_p + ps;
    }
    if (state) HIPCHK(hipMemcpyAsync(state, src_p, ps, hipMemcpyDeviceToHost, d->stream));
    if (outputs) HIPCHK(hipMemcpyAsync(outputs, src_q, qs, hipMemcpyDeviceToHost, d->stream));
    HIPCHK(hipStreamSynchronize(d->stream));
    return LBM_OK;
}

int lbm_step(lbm_domain* d, int64_t nsteps) {
    int rc = usable(d);
    if (rc) return rc;
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    if (d->batch) return fail(LBM_ESTATE, "domain is a batch member; step the batch");
    if (nsteps == 0) return LBM_OK;
    return dispatch(d->p.storage, [&](auto s) { return step_impl<decltype(s)>(d, nsteps); });
}

int lbm_set_check(lbm_domain* d, int64_t every) {
    if (!d) return fail(LBM_EINVAL, "domain is NULL");
    if (every < 0) return fail(LBM_EINVAL, "every must be >= 0");
    d->check_every = every;
    return LBM_OK;
}

int lbm_check(lbm_domain* d) {
    int rc = usable(d);
    if (rc) return rc;
    return dispatch(d->p.storage, [&](auto s) -> int {
        double res[NPART];
        int r = reduce<decltype(s)>(d, false, res, nullptr);
        if (r) return r;
        if (res[3] > 0.0) {
            d->failed = true;
            return fail(LBM_ENONFINITE, "non-finite phi, u or P at step " + std::to_string(d->steps));
        }
        return LBM_OK;
    });
}

int lbm_read(lbm_domain* d, double* phi, double* ux, double* uy, double* P) {
    int rc = usable(d);
    if (rc) return rc;
    return dispatch(d->p.storage, [&](auto s) { return read_impl<decltype(s)>(d, phi, ux, uy, P); });
}

int lbm_mass(lbm_domain* d, double* sum_phi) {
    int rc = usable(d);
    if (rc) return rc;
    if (!sum_phi) return fail(LBM_EINVAL, "sum_phi is NULL");
    return dispatch(d->p.storage, [&](auto s) -> int {
        using S = decltype(s);
        double res[NPART];
        int64_t im[2] = {0, 0};
        int r = reduce<S>(d, false, res, im);
        if (r) return r;
        // im[0] 2^32 and im[1] are exact doubles (|im[0]| < 2^44, im[1] < 2^32):
        // their sum is the exact fixed-point mass rounded once
        *sum_phi = S::kFix ? std::ldexp((double)im[0] * 4294967296.0 + (double)im[1], -FIX_BITS) : res[0];
        return LBM_OK;
    });
}

int lbm_energy(lbm_domain* d, double* e_free, double* e_kin) {
    int rc = usable(d);
    if (rc) return rc;
    return dispatch(d->p.storage, [&](auto s) -> int {
        double res[NPART];
        int r = reduce<decltype(s)>(d, false, res, nullptr);
        if (r) return r;
        if (e_free) *e_free = res[1];
        if (e_kin) *e_kin = res[2];
        return LBM_OK;
    });
}

int64_t lbm_steps_done(const lbm_domain* d) { return d ? d->steps : -1; }

double lbm_last_step_ms(const lbm_domain* d) { return d ? d->last_ms : 0.0; }

size_t lbm_state_bytes(const lbm_domain* d) {
    if (!d) return 0;
    return 16 + d->L.pop_bytes + d->L.hist_bytes + (size_t)d->p.np * (PSTRIDE + QSTRIDE) * 8;
}

int lbm_export_state(lbm_domain* d, void* host_buf, size_t bytes) {
    if (!d || !host_buf) return fail(LBM_EINVAL, "NULL argument");
    if (bytes < lbm_state_bytes(d)) return fail(LBM_ENOMEM, "buffer too small");
    const int par = (int)(d->steps & 1);
    char* h = (char*)host_buf;
    int64_t hdr[2] = {d->steps, (int64_t)d->p.storage};
    std::memcpy(h, hdr, 16);
    HIPCHK(hipMemcpyAsync(h + 16, d->ws + d->L.off_pop[par], d->L.pop_bytes, hipMemcpyDeviceToHost, d->stream));
    HIPCHK(hipMemcpyAsync(h + 16 + d->L.pop_bytes, d->ws + d->L.off_hist[par], d->L.hist_bytes,
                          hipMemcpyDeviceToHost, d->stream));
    if (d->p.np > 0) {
        char* hp = h + 16 + d->L.pop_bytes + d->L.hist_bytes;
        HIPCHK(hipMemcpyAsync(hp, d->ws + d->L.off_parts, (size_t)d->p.np * PSTRIDE * 8, hipMemcpyDeviceToHost,
                              d->stream));
        HIPCHK(hipMemcpyAsync(hp + (size_t)d->p.np * PSTRIDE * 8, d->ws + d->L.off_pout,
                              (size_t)d->p.np * QSTRIDE * 8, hipMemcpyDeviceToHost, d->stream));
    }
    HIPCHK(hipStreamSynchronize(d->stream));
    return LBM_OK;
}

int lbm_import_state(lbm_domain* d, const void* host_buf, size_t bytes) {
    if (!d || !host_buf) return fail(LBM_EINVAL, "NULL argument");
    if (bytes < lbm_state_bytes(d)) return fail(LBM_EINVAL, "buffer too small");
    const char* h = (const char*)host_buf;
    int64_t hdr[2];
    std::memcpy(hdr, h, 16);
    if (hdr[1] != d->p.storage || hdr[0] < 0) return fail(LBM_EINVAL, "state is from another storage mode");
    const int par = (int)(hdr[0] & 1);
    HIPCHK(hipMemcpyAsync(d->ws + d->L.off_pop[par], h + 16, d->L.pop_bytes, hipMemcpyHostToDevice, d->stream));
    HIPCHK(hipMemcpyAsync(d->ws + d->L.off_hist[par], h + 16 + d->L.pop_bytes, d->L.hist_bytes,
                          hipMemcpyHostToDevice, d->stream));
    if (d->p.np > 0) {
        const char* hp = h + 16 + d->L.pop_bytes + d->L.hist_bytes;
        HIPCHK(hipMemcpyAsync(d->ws + d->L.off_parts, hp, (size_t)d->p.np * PSTRIDE * 8, hipMemcpyHostToDevice,
                              d->stream));
        HIPCHK(hipMemcpyAsync(d->ws + d->L.off_pout, hp + (size_t)d->p.np * PSTRIDE * 8,
                              (size_t)d->p.np * QSTRIDE * 8, hipMemcpyHostToDevice, d->stream));
        const int rc =
            dispatch(d->p.storage, [&](auto s) { return particle_statics<typename decltype(s)::R>(d, true); });
        if (rc) return rc;
    }
    HIPCHK(hipStreamSynchronize(d->stream));
    d->steps = hdr[0];
    d->failed = false;
    return LBM_OK;
}

int lbm_destroy(lbm_domain* d) {
    if (!d) return LBM_OK;
    if (d->batch) lbm_batch_remove(d->batch, d);
    if (d->ev0) (void)hipEventDestroy(d->ev0);
    if (d->ev1) (void)hipEventDestroy(d->ev1);
    delete d;
    return LBM_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batch
struct lbm_batch {
    int storage = 0;
    int ty = 8;
    int max_members = 0;
    int64_t max_tiles = 0;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    size_t off_jobs = 0, off_tiles = 0;
    std::vector<lbm_domain*> members;
    std::vector<unsigned char> jobs;  // host image of the job table
    std::vector<TileEntry> tiles;
    bool tiles_dirty = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t graph_steps = -1;
    int graph_ntiles = -1;
};

namespace {

constexpr int64_t BATCH_CHUNK = 50;  // launches per captured batch graph

void drop_graph(lbm_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_steps = -1;
}

template <class S, int TY>
int batch_capture(lbm_batch* b, int64_t nsteps) {
    drop_graph(b);
    const Job<S>* J = (const Job<S>*)(b->ws + b->off_jobs);
    const TileEntry* T = (const TileEntry*)(b->ws + b->off_tiles);
    const int nt = (int)b->tiles.size();
    bool wall = false;  // the wall variant when any member has bounce-back walls
    for (const lbm_domain* d : b->members) wall = wall || wall_bits(d->p) != 0;
    HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t le = hipSuccess;
    for (int64_t t = 0; t < nsteps && le == hipSuccess; ++t) {
        if (wall)
            hipLaunchKernelGGL((k_tile<S, TY, MODE_STEP, false, true>), dim3(nt), dim3(TileCfg<TY>::NT), 0,
                               b->stream, J, T, nt, (int)t);
        else
            hipLaunchKernelGGL((k_tile<S, TY, MODE_STEP>), dim3(nt), dim3(TileCfg<TY>::NT), 0, b->stream, J, T,
                               nt, (int)t);
        le = hipGetLastError();
    }
    hipError_t ce = hipStreamEndCapture(b->stream, &b->graph);  // always leave capture mode
    if (le != hipSuccess) return fail(LBM_EDEVICE, std::string("launch in capture: ") + hipGetErrorString(le));
    if (ce != hipSuccess) return fail(LBM_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
    HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_steps = nsteps;
    b->graph_ntiles = nt;
    return LBM_OK;
}

template <class S>
int batch_step_impl(lbm_batch* b, int64_t nsteps, const int64_t* budget) {
    const size_t js = sizeof(Job<S>);
    if (b->tiles_dirty) {
        b->tiles.clear();
        for (size_t k = 0; k < b->members.size(); ++k)
            for (const TileEntry& t : b->members[k]->tiles) b->tiles.push_back(TileEntry{(int32_t)k, t.x0, t.y0, 0});
        if ((int64_t)b->tiles.size() > b->max_tiles) return fail(LBM_ENOMEM, "batch tile table full");
        if (!b->tiles.empty())
            HIPCHK(hipMemcpyAsync(b->ws + b->off_tiles, b->tiles.data(), b->tiles.size() * sizeof(TileEntry),
                                  hipMemcpyHostToDevice, b->stream));
        b->tiles_dirty = false;
        drop_graph(b);
    }
    if (b->members.empty() || nsteps == 0) return LBM_OK;
    // The graph holds a fixed chunk of BATCH_CHUNK launches and is replayed;
    // before each replay the job table gets the chunk's first step and the
    // number of its launches each member takes part in (the rest of its tiles
    // return at once).  Membership changes recapture only one chunk.
    const int64_t nchunks = (nsteps + BATCH_CHUNK - 1) / BATCH_CHUNK;
    const size_t nm = b->members.size();
    b->jobs.assign(js * nm * (size_t)nchunks, 0);
    std::vector<int64_t> adv(nm);
    for (size_t k = 0; k < nm; ++k) {
        int64_t n = nsteps;
        if (budget) n = budget[k] < n ? budget[k] : n;
        if (n < 0) n = 0;
        if (b->members[k]->failed) n = 0;
        adv[k] = n;
    }
    for (int64_t c = 0; c < nchunks; ++c) {
        int32_t base = 0;
        for (size_t k = 0; k < nm; ++k) {
            lbm_domain* d = b->members[k];
            const int64_t done = std::min(c * BATCH_CHUNK, adv[k]);
            const int64_t n = std::min(adv[k] - done, BATCH_CHUNK);
            Job<S> J;
            make_job<S>(d, (int32_t)n, d->steps + done, false, base, J);
            std::memcpy(b->jobs.data() + ((size_t)c * nm + k) * js, &J, js);
            base += (int32_t)d->tiles.size();
        }
    }
    if (!b->exec || b->graph_steps != BATCH_CHUNK || b->graph_ntiles != (int)b->tiles.size()) {
        int rc;
        switch (b->ty) {
            case 4: rc = batch_capture<S, 4>(b, BATCH_CHUNK); break;
            case 16: rc = batch_capture<S, 16>(b, BATCH_CHUNK); break;
            case 32:
                if constexpr (sizeof(typename S::R) == 4) {
                    rc = batch_capture<S, 32>(b, BATCH_CHUNK);
                    break;
                }
                return fail(LBM_EUNSUPPORTED, "64x32 tiles are not built for FP64");
            default: rc = batch_capture<S, 8>(b, BATCH_CHUNK); break;
        }
        if (rc) return rc;
    }
    for (int64_t c = 0; c < nchunks; ++c) {
        HIPCHK(hipMemcpyAsync(b->ws + b->off_jobs, b->jobs.data() + (size_t)c * nm * js, nm * js,
                              hipMemcpyHostToDevice, b->stream));
        HIPCHK(hipGraphLaunch(b->exec, b->stream));
    }
    for (size_t k = 0; k < nm; ++k) b->members[k]->steps += adv[k];
    return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_batch_workspace_bytes(int32_t max_members, int64_t max_tiles) {
    if (max_members <= 0 || max_tiles <= 0) return 0;
    size_t js = 0;
    for (int s = 0; s < 4; ++s) js = js > job_size(s) ? js : job_size(s);
    return up((size_t)max_members * js) + up((size_t)max_tiles * sizeof(TileEntry));
}

int lbm_batch_create(int32_t storage, int32_t tile, int32_t max_members, int64_t max_tiles,
                     void* dev_workspace, size_t bytes, void* hip_stream, lbm_batch** out) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (storage < LBM_STORE_FP64 || storage > LBM_STORE_BF16DEV) return fail(LBM_EUNSUPPORTED, "unknown storage");
    if (!(tile == LBM_TILE_AUTO || tile == 4 || tile == 8 || tile == 16 || tile == 32))
        return fail(LBM_EUNSUPPORTED, "unknown tile");
    if (tile == 32 && storage == LBM_STORE_FP64) return fail(LBM_EUNSUPPORTED, "64x32 tiles are not built for FP64");
    if (max_members <= 0 || max_tiles <= 0) return fail(LBM_EINVAL, "sizes must be positive");
    if (!dev_workspace || (uintptr_t)dev_workspace % ALIGN) return fail(LBM_EINVAL, "workspace NULL or unaligned");
    if (bytes < lbm_batch_workspace_bytes(max_members, max_tiles)) return fail(LBM_ENOMEM, "workspace too small");
    if (!hip_stream) return fail(LBM_EINVAL, "a batch needs its own stream (the null stream cannot be captured)");
    lbm_batch* b = new lbm_batch();
    b->storage = storage;
    b->ty = tile == LBM_TILE_AUTO ? 8 : tile;
    b->max_members = max_members;
    b->max_tiles = max_tiles;
    b->stream = (hipStream_t)hip_stream;
    b->ws = (char*)dev_workspace;
    size_t js = 0;
    for (int s = 0; s < 4; ++s) js = js > job_size(s) ? js : job_size(s);
    b->off_jobs = 0;
    b->off_tiles = up((size_t)max_members * js);
    *out = b;
    return LBM_OK;
}

int lbm_batch_add(lbm_batch* b, lbm_domain* d) {
    if (!b || !d) return fail(LBM_EINVAL, "NULL argument");
    if (d->batch) return fail(LBM_ESTATE, "domain already in a batch");
    if (d->p.storage != b->storage) return fail(LBM_EINVAL, "storage mode differs from the batch's");
    if (d->L.ty != b->ty) return fail(LBM_EINVAL, "tile shape differs from the batch's");
    if (d->p.np > 0) return fail(LBM_EUNSUPPORTED, "domains with free particles cannot join a batch");
    if (d->stream != b->stream) return fail(LBM_EINVAL, "domain must use the batch's stream");
    if ((int)b->members.size() >= b->max_members) return fail(LBM_ENOMEM, "batch is full");
    b->members.push_back(d);
    d->batch = b;
    b->tiles_dirty = true;
    return LBM_OK;
}

int lbm_batch_remove(lbm_batch* b, lbm_domain* d) {
    if (!b || !d) return fail(LBM_EINVAL, "NULL argument");
    for (size_t k = 0; k < b->members.size(); ++k)
        if (b->members[k] == d) {
            b->members.erase(b->members.begin() + k);
            d->batch = nullptr;
            b->tiles_dirty = true;
            return LBM_OK;
        }
    return fail(LBM_EINVAL, "domain is not a member");
}

int lbm_batch_step(lbm_batch* b, int64_t nsteps, const int64_t* budget) {
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (nsteps < 0 || nsteps > (1 << 20)) return fail(LBM_EINVAL, "nsteps out of range");
    return dispatch(b->storage, [&](auto s) { return batch_step_impl<decltype(s)>(b, nsteps, budget); });
}

int lbm_batch_size(const lbm_batch* b) { return b ? (int)b->members.size() : -1; }

int lbm_batch_destroy(lbm_batch* b) {
    if (!b) return LBM_OK;
    for (lbm_domain* d : b->members) d->batch = nullptr;
    drop_graph(b);
    delete b;
    return LBM_OK;
}

}  // extern "C"
