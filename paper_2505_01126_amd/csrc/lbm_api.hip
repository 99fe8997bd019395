// C ABI of liblbm (declared in include/lbm.h): handle lifetime, workspace
// layout, argument checks and kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>
#include <algorithm>

#include "lbm.h"
#include "lbm_internal.h"

namespace {

constexpr size_t ALIGN = 256;
constexpr int DEFAULT_ZCHUNK = 32;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

size_t elem_bytes(int storage) { return storage == LBM_STORE_F32 ? 4 : 2; }

// Byte offsets of every array inside the caller's workspace.
struct Layout {
    size_t f[2], phi[2], u[2], frow, fx, partials, red, mlp, sph, hcount, total;
};

Layout layout_of(const lbm_config &c)
{
    Layout L{};
    const size_t N = (size_t)c.nx * c.ny * c.nz;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    L.f[0] = take(27 * N * elem_bytes(c.storage));
    L.f[1] = take(27 * N * elem_bytes(c.storage));
    if (c.two_phase) {
        L.phi[0] = take(8 * N);
        L.phi[1] = take(8 * N);
        L.u[0] = take(12 * N);
        L.u[1] = take(12 * N);
    } else {
        L.phi[0] = L.phi[1] = L.u[0] = L.u[1] = (size_t)-1;
    }
    if (c.n_modes > 0) {
        L.frow = take(sizeof(float) * lbm::FROW * (size_t)c.ny * c.nz);
        L.fx = take(sizeof(float) * 4 * (size_t)c.nx);
    } else {
        L.frow = L.fx = (size_t)-1;
    }
    L.partials = take(sizeof(double) * lbm::RED_BLOCKS * lbm::NRED);
    L.red = take(sizeof(double) * lbm::NRED);
    L.mlp = take(sizeof(uint16_t) * LBM_MLP_NPARAM);
    L.sph = take(sizeof(double) * 4 * lbm::MAX_SPHERES);
    L.hcount = take(sizeof(long long) * 2 * lbm::HARVEST_BLOCKS);
    L.total = off;
    return L;
}

const char *validate(const lbm_config *c)
{
    if (!c) return "config is NULL";
    if (c->nx < 8 || c->ny < 8 || c->nz < 8) return "nx, ny, nz must be >= 8";
    const double N = (double)c->nx * c->ny * c->nz;
    if (N > 1073741824.0) return "nx*ny*nz must be <= 2^30";
    if ((double)c->nx * c->ny > 16777216.0) return "nx*ny must be <= 2^24";
    if (c->storage < LBM_STORE_F32 || c->storage > LBM_STORE_BF16) return "storage must be F32, F16 or BF16";
    if (c->two_phase != 0 && c->two_phase != 1) return "two_phase must be 0 or 1";
    if (c->curv_mode != LBM_CURV_FD && c->curv_mode != LBM_CURV_MLP) return "curv_mode must be FD or MLP";
    if (c->curv_mode == LBM_CURV_MLP && !c->two_phase) return "MLP curvature needs two_phase";
    if (!(c->tau > 0.5) || !std::isfinite(c->tau)) return "tau must be > 1/2";
    if (!(c->rho_l > 0.0) || !std::isfinite(c->rho_l)) return "rho_l must be > 0";
    if (c->two_phase) {
        if (!(c->rho_g > 0.0) || !std::isfinite(c->rho_g)) return "rho_g must be > 0";
        if (!(c->width > 0.0) || !std::isfinite(c->width)) return "width must be > 0";
        if (!(c->mobility >= 0.0) || !std::isfinite(c->mobility)) return "mobility must be >= 0";
        if (!std::isfinite(c->sigma)) return "sigma must be finite";
    }
    if (!std::isfinite(c->p0)) return "p0 must be finite";
    if (c->n_modes < 0 || c->n_modes > LBM_MAX_MODES) return "n_modes out of range";
    if (c->n_modes > 0 && !c->modes) return "modes is NULL";
    for (int m = 0; m < c->n_modes; m++) {
        const double *r = c->modes + 9 * m;
        for (int k = 0; k < 3; k++)
            if (r[k] != std::floor(r[k]) || std::fabs(r[k]) > 1024.0) return "mode wave numbers must be integers";
        if (std::fabs(r[0]) > 2.0) return "mode kx must satisfy |kx| <= 2";
        for (int k = 3; k < 9; k++)
            if (!std::isfinite(r[k])) return "mode amplitudes must be finite";
    }
    if (c->zchunk < 0) return "zchunk must be >= 0";
    if (c->curv_mode == LBM_CURV_MLP) {
        double lo = c->mlp_k_lo, hi = c->mlp_k_hi;
        if (lo == 0.0 && hi == 0.0) {
            lo = 0.4;
            hi = 0.6;
        }
        if (!(hi > lo) || !(lo >= 0.0)) return "mlp_k_hi must exceed mlp_k_lo >= 0";
    }
    return nullptr;
}

}  // namespace

struct lbm_handle {
    lbm_config cfg{};
    lbm::Params P{};
    Layout L{};
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    int cur = 0;
    int64_t steps = 0;
    bool mlp_set = false;
    std::vector<float> frow_host, fx_host;
    std::string err;

    void *f(int k) { return ws + L.f[k]; }
    double *phi(int k) { return cfg.two_phase ? (double *)(ws + L.phi[k]) : nullptr; }
    float *u(int k) { return cfg.two_phase ? (float *)(ws + L.u[k]) : nullptr; }

    int fail(int code, const std::string &msg)
    {
        err = msg;
        return code;
    }
    int hip(hipError_t e, const char *what)
    {
        if (e == hipSuccess) return LBM_OK;
        err = std::string(what) + ": " + hipGetErrorString(e);
        return LBM_EHIP;
    }
};

extern "C" {

int lbm_abi_version(void) { return LBM_ABI_VERSION; }

size_t lbm_workspace_bytes(const lbm_config *cfg)
{
    if (validate(cfg)) return 0;
    return layout_of(*cfg).total;
}

static thread_local std::string g_init_err;

int lbm_init(lbm_handle **out, const lbm_config *cfg, void *d_ws, size_t ws_bytes, const double *d_phi0,
             const double *d_u0, const double *d_pstar0, void *stream)
{
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    if (const char *why = validate(cfg)) {
        g_init_err = why;
        return LBM_EINVAL;
    }
    if (cfg->two_phase && !d_phi0) {
        g_init_err = "two_phase needs d_phi0";
        return LBM_EINVAL;
    }
    if (!d_ws || ((uintptr_t)d_ws % ALIGN) != 0) {
        g_init_err = "workspace must be a 256-byte aligned device pointer";
        return LBM_EINVAL;
    }
    const Layout L = layout_of(*cfg);
    if (ws_bytes < L.total) {
        g_init_err = "workspace too small";
        return LBM_ENOSPACE;
    }
    lbm_handle *h = new (std::nothrow) lbm_handle();
    if (!h) return LBM_EINVAL;
    h->cfg = *cfg;
    h->cfg.modes = nullptr;  // the host table is read only here
    h->L = L;
    h->ws = (char *)d_ws;
    h->stream = (hipStream_t)stream;

    lbm::Params &P = h->P;
    P.nx = cfg->nx;
    P.ny = cfg->ny;
    P.nz = cfg->nz;
    int zc = cfg->zchunk > 0 ? cfg->zchunk : DEFAULT_ZCHUNK;
    P.zchunk = zc > cfg->nz ? cfg->nz : zc;
    P.two_phase = cfg->two_phase;
    P.curv_mode = cfg->curv_mode;
    P.n_modes = cfg->n_modes;
    P.omega = (float)(1.0 / cfg->tau);
    P.p0 = (float)cfg->p0;
    P.rho_l = (float)cfg->rho_l;
    P.rho_g = cfg->two_phase ? (float)cfg->rho_g : (float)cfg->rho_l;
    const double nu = (cfg->tau - 0.5) / 3.0;
    P.fs_coef = (float)(1.5 * cfg->width * cfg->sigma);
    P.fnu_coef = (float)(nu / (cfg->tau / 3.0));
    P.d6 = (float)(6.0 * cfg->mobility);
    P.k3 = cfg->width > 0.0 ? (float)(3.0 * 4.0 * cfg->mobility / cfg->width) : 0.f;
    double lo = cfg->mlp_k_lo, hi = cfg->mlp_k_hi;
    if (lo == 0.0 && hi == 0.0) {
        lo = 0.4;
        hi = 0.6;
    }
    P.k_lo = (float)lo;
    P.k_hi = (float)hi;
    P.mlp = h->ws + L.mlp;
    P.frow = nullptr;
    P.fx = nullptr;
    P.gx = (cfg->nx + lbm::TX - 1) / lbm::TX;
    P.gy = (cfg->ny + lbm::TY - 1) / lbm::TY;
    P.gz = (cfg->nz + P.zchunk - 1) / P.zchunk;
    P.nblocks = P.gx * P.gy * P.gz;

    if (cfg->n_modes > 0) {
        // body-force tables in FP64 on the host, stored as FP32: per mode,
        // B = A e^{i (ky ty + kz tz)} is folded into the row coefficients of
        // cos(|kx| t) (Re B) and sin(|kx| t) (-sign(kx) Im B), t = 2 pi x / nx
        const int nx = cfg->nx, ny = cfg->ny, nz = cfg->nz, nm = cfg->n_modes;
        h->frow_host.assign((size_t)lbm::FROW * ny * nz, 0.0f);
        h->fx_host.assign((size_t)4 * nx, 0.0f);
        const double two_pi = 6.283185307179586476925286766559;
        auto twiddle = [&](long k, long v, long n, double &c, double &s) {
            const long f = ((k * v) % n + n) % n;  // exact phase index
            c = std::cos(two_pi * (double)f / n);
            s = std::sin(two_pi * (double)f / n);
        };
        std::vector<double> ey(2 * (size_t)nm * ny), ez(2 * (size_t)nm * nz);
        for (int m = 0; m < nm; m++) {
            const double *r = cfg->modes + 9 * m;
            for (int y = 0; y < ny; y++) twiddle((long)r[1], y, ny, ey[2 * ((size_t)m * ny + y)], ey[2 * ((size_t)m * ny + y) + 1]);
            for (int z = 0; z < nz; z++) twiddle((long)r[2], z, nz, ez[2 * ((size_t)m * nz + z)], ez[2 * ((size_t)m * nz + z) + 1]);
        }
        double acc[lbm::FROW];
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < ny; y++) {
                std::fill(acc, acc + lbm::FROW, 0.0);
                for (int m = 0; m < nm; m++) {
                    const double *r = cfg->modes + 9 * m;
                    const long kx = (long)r[0];
                    const double *cy = &ey[2 * ((size_t)m * ny + y)], *cz = &ez[2 * ((size_t)m * nz + z)];
                    const double pc = cy[0] * cz[0] - cy[1] * cz[1], ps = cy[0] * cz[1] + cy[1] * cz[0];
                    const int kk = (int)(kx < 0 ? -kx : kx);
                    const double sg = kx < 0 ? -1.0 : 1.0;
                    for (int a = 0; a < 3; a++) {
                        const double ar = r[3 + 2 * a], ai = r[4 + 2 * a];
                        const double br = ar * pc - ai * ps, bi = ar * ps + ai * pc;
                        if (kk == 0) {
                            acc[a] += br;
                        } else {
                            acc[3 + 6 * (kk - 1) + a] += br;
                            acc[6 + 6 * (kk - 1) + a] -= sg * bi;
                        }
                    }
                }
                float *dst = &h->frow_host[((size_t)z * ny + y) * lbm::FROW];
                for (int k = 0; k < lbm::FROW; k++) dst[k] = (float)acc[k];
            }
        for (int x = 0; x < nx; x++) {
            double c, s;
            twiddle(1, x, nx, c, s);
            h->fx_host[4 * x + 0] = (float)c;
            h->fx_host[4 * x + 1] = (float)s;
            twiddle(2, x, nx, c, s);
            h->fx_host[4 * x + 2] = (float)c;
            h->fx_host[4 * x + 3] = (float)s;
        }
        float *drow = (float *)(h->ws + L.frow);
        float4 *dx = (float4 *)(h->ws + L.fx);
        hipError_t e = hipMemcpyAsync(drow, h->frow_host.data(), sizeof(float) * h->frow_host.size(),
                                      hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dx, h->fx_host.data(), sizeof(float) * h->fx_host.size(), hipMemcpyHostToDevice,
                               h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);  // host staging is released below
        h->frow_host.clear();
        h->frow_host.shrink_to_fit();
        h->fx_host.clear();
        h->fx_host.shrink_to_fit();
        if (e != hipSuccess) {
            g_init_err = std::string("forcing table upload: ") + hipGetErrorString(e);
            delete h;
            return LBM_EHIP;
        }
        P.frow = drow;
        P.fx = dx;
    }
    hipError_t e = lbm::launch_init(P, cfg->storage, h->f(0), h->phi(0), h->u(0), d_phi0, d_u0, d_pstar0, h->stream);
    if (e != hipSuccess) {
        g_init_err = std::string("init kernel: ") + hipGetErrorString(e);
        delete h;
        return LBM_EHIP;
    }
    *out = h;
    return LBM_OK;
}

int lbm_step(lbm_handle *h, int64_t nsteps)
{
    if (!h) return LBM_EINVAL;
    if (nsteps < 0) return h->fail(LBM_EINVAL, "nsteps must be >= 0");
    if (h->cfg.curv_mode == LBM_CURV_MLP && !h->mlp_set) return h->fail(LBM_ESTATE, "MLP weights not set");
    for (int64_t n = 0; n < nsteps; n++) {
        const int c = h->cur, o = 1 - c;
        lbm::Buffers b{h->f(c), h->f(o), h->phi(c), h->phi(o), h->u(c), h->u(o)};
        hipError_t e = lbm::launch_step(h->P, h->cfg.storage, b, h->stream);
        if (e != hipSuccess) return h->hip(e, "step kernel");
        h->cur = o;
        h->steps++;
    }
    return LBM_OK;
}

int lbm_moments(lbm_handle *h, float *d_rho, float *d_p, float *d_u, double *d_phi)
{
    if (!h) return LBM_EINVAL;
    if (h->cfg.curv_mode == LBM_CURV_MLP && !h->mlp_set) return h->fail(LBM_ESTATE, "MLP weights not set");
    const int c = h->cur;
    hipError_t e = lbm::launch_moments(h->P, h->cfg.storage, h->f(c), h->phi(c), d_rho, d_p, d_u, d_phi, h->stream);
    return h->hip(e, "moments kernel");
}

int lbm_reduce(lbm_handle *h, double *out, int out_is_host)
{
    if (!h || !out) return LBM_EINVAL;
    if (h->cfg.curv_mode == LBM_CURV_MLP && !h->mlp_set) return h->fail(LBM_ESTATE, "MLP weights not set");
    const int c = h->cur;
    double *red = (double *)(h->ws + h->L.red);
    hipError_t e = lbm::launch_reduce(h->P, h->cfg.storage, h->f(c), h->phi(c), (double *)(h->ws + h->L.partials),
                                      red, h->stream);
    if (e != hipSuccess) return h->hip(e, "reduce kernel");
    if (out_is_host) {
        e = hipMemcpyAsync(out, red, sizeof(double) * LBM_NRED, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    } else {
        e = hipMemcpyAsync(out, red, sizeof(double) * LBM_NRED, hipMemcpyDeviceToDevice, h->stream);
    }
    return h->hip(e, "reduce copy");
}

int64_t lbm_steps_done(const lbm_handle *h) { return h ? h->steps : -1; }

size_t lbm_mlp_work_bytes(int64_t batch)
{
    if (batch < 0) return 0;
    return sizeof(float) * (size_t)lbm::mlp_backward_blocks(batch) * (LBM_MLP_NPARAM + 1);
}

int lbm_mlp_forward(const uint16_t *d_w, const uint16_t *d_x, int64_t batch, float *d_y, void *stream)
{
    if (!d_w || batch < 0 || (batch > 0 && (!d_x || !d_y))) return LBM_EINVAL;
    return lbm::launch_mlp_forward(d_w, d_x, batch, d_y, (hipStream_t)stream) == hipSuccess ? LBM_OK : LBM_EHIP;
}

int lbm_mlp_backward(const uint16_t *d_w, const uint16_t *d_x, const float *d_t, int64_t batch, float *d_grad,
                     float *d_loss, void *d_work, size_t work_bytes, void *stream)
{
    if (!d_w || batch < 0 || !d_grad || !d_loss || !d_work || (batch > 0 && (!d_x || !d_t))) return LBM_EINVAL;
    if (work_bytes < lbm_mlp_work_bytes(batch)) return LBM_ENOSPACE;
    return lbm::launch_mlp_backward(d_w, d_x, d_t, batch, d_grad, d_loss, (float *)d_work, (hipStream_t)stream) ==
                   hipSuccess
               ? LBM_OK
               : LBM_EHIP;
}

int lbm_mlp_adam(float *d_master, float *d_m, float *d_v, const float *d_grad, uint16_t *d_w16, int64_t step,
                 float lr, float beta1, float beta2, float eps, void *stream)
{
    if (!d_master || !d_m || !d_v || !d_grad || !d_w16 || step < 1) return LBM_EINVAL;
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f)) return LBM_EINVAL;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)step)));
    return lbm::launch_mlp_adam(d_master, d_m, d_v, d_grad, d_w16, lr, beta1, beta2, eps, c1, c2,
                                (hipStream_t)stream) == hipSuccess
               ? LBM_OK
               : LBM_EHIP;
}

int lbm_set_mlp(lbm_handle *h, const uint16_t *d_w)
{
    if (!h || !d_w) return LBM_EINVAL;
    hipError_t e = hipMemcpyAsync(h->ws + h->L.mlp, d_w, sizeof(uint16_t) * LBM_MLP_NPARAM, hipMemcpyDeviceToDevice,
                                  h->stream);
    if (e != hipSuccess) return h->hip(e, "set_mlp copy");
    h->mlp_set = true;
    return LBM_OK;
}

int lbm_harvest(lbm_handle *h, const double *centers, const double *radii, int nb, uint16_t *d_x, float *d_y,
                int64_t cap, int64_t *n_out)
{
    if (!h || !n_out || cap < 0 || nb < 0 || nb > LBM_MLP_MAX_SPHERES || (nb > 0 && (!centers || !radii)) ||
        (cap > 0 && (!d_x || !d_y)))
        return LBM_EINVAL;
    if (!h->cfg.two_phase) return h->fail(LBM_ESTATE, "harvest needs a two-phase handle");
    const uint32_t N = (uint32_t)h->cfg.nx * h->cfg.ny * h->cfg.nz;
    const int blocks = (int)std::min<uint32_t>((N + 255) / 256, lbm::HARVEST_BLOCKS);
    const uint32_t chunk = ((N + blocks - 1) / blocks + 255) / 256 * 256;
    std::vector<double> sph(4 * (size_t)std::max(nb, 1), 0.0);
    for (int k = 0; k < nb; k++) {
        sph[4 * k + 0] = centers[3 * k + 0];
        sph[4 * k + 1] = centers[3 * k + 1];
        sph[4 * k + 2] = centers[3 * k + 2];
        sph[4 * k + 3] = radii[k];
    }
    long long *counts = (long long *)(h->ws + h->L.hcount);
    long long *offsets = counts + lbm::HARVEST_BLOCKS;
    std::vector<long long> hc(blocks), ho(blocks);
    const double *phi = h->phi(h->cur);
    hipError_t e = hipMemcpyAsync(h->ws + h->L.sph, sph.data(), sizeof(double) * 4 * nb, hipMemcpyHostToDevice,
                                  h->stream);
    if (e == hipSuccess) e = lbm::launch_harvest_count(phi, N, chunk, blocks, counts, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hc.data(), counts, sizeof(long long) * blocks, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return h->hip(e, "harvest count");
    long long total = 0;
    for (int b = 0; b < blocks; b++) {
        ho[b] = total;
        total += hc[b];
    }
    e = hipMemcpyAsync(offsets, ho.data(), sizeof(long long) * blocks, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess && cap > 0)
        e = lbm::launch_harvest_write(h->P, phi, chunk, blocks, offsets, h->ws + h->L.sph, nb, d_x, d_y, cap,
                                      h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return h->hip(e, "harvest write");
    *n_out = total;
    return LBM_OK;
}

int lbm_set_stream(lbm_handle *h, void *stream)
{
    if (!h) return LBM_EINVAL;
    h->stream = (hipStream_t)stream;
    return LBM_OK;
}

int lbm_destroy(lbm_handle *h)
{
    delete h;
    return LBM_OK;
}

const char *lbm_strerror(int code)
{
    switch (code) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOSPACE: return "workspace too small";
    case LBM_EHIP: return "HIP runtime error";
    case LBM_ESTATE: return "invalid state";
    default: return "unknown error";
    }
}

const char *lbm_last_error(const lbm_handle *h)
{
    if (!h) return g_init_err.c_str();
    return h->err.c_str();
}

}  // extern "C"
