// C ABI of liblbm (declared in include/lbm.h): handle lifetime, workspace
// layout, argument checks and kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "lbm.h"
#include "lbm_internal.h"

namespace {

constexpr size_t ALIGN = 256;
constexpr int DEFAULT_ZCHUNK = 32;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

size_t elem_bytes(int storage) { return storage == LBM_STORE_F32 ? 4 : 2; }

// Byte offsets of every array inside the caller's workspace.
struct Layout {
    size_t f[2], phi[2], u[2], modes, partials, red, mlp, total;
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
    L.modes = take(sizeof(lbm::ModeTable));
    L.partials = take(sizeof(double) * lbm::RED_BLOCKS * lbm::NRED);
    L.red = take(sizeof(double) * lbm::NRED);
    L.mlp = take(sizeof(uint16_t) * LBM_MLP_NPARAM);
    L.total = off;
    return L;
}

const char *validate(const lbm_config *c)
{
    if (!c) return "config is NULL";
    if (c->nx < 8 || c->ny < 8 || c->nz < 8) return "nx, ny, nz must be >= 8";
    const double N = (double)c->nx * c->ny * c->nz;
    if (N > 1073741824.0) return "nx*ny*nz must be <= 2^30";
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
        if (std::fabs(r[2]) > 2.0) return "mode kz must satisfy |kz| <= 2";
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
    lbm::ModeTable modes_host{};
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
    P.modes = nullptr;

    if (cfg->n_modes > 0) {
        lbm::ModeTable &mt = h->modes_host;
        mt.n = cfg->n_modes;
        for (int m = 0; m < cfg->n_modes; m++) {
            const double *r = cfg->modes + 9 * m;
            // Re(A e^{i k.x}) = Re(conj(A) e^{-i k.x}): store every row with kz >= 0
            const double sg = r[2] < 0 ? -1.0 : 1.0;
            mt.kx[m] = (int)(sg * r[0]);
            mt.ky[m] = (int)(sg * r[1]);
            mt.kz[m] = (int)(sg * r[2]);
            for (int a = 0; a < 3; a++) {
                mt.re[m][a] = (float)r[3 + 2 * a];
                mt.im[m][a] = (float)(sg * r[4 + 2 * a]);
            }
        }
        lbm::ModeTable *dm = (lbm::ModeTable *)(h->ws + L.modes);
        hipError_t e = hipMemcpyAsync(dm, &mt, sizeof(mt), hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);  // host staging must outlive the copy
        if (e != hipSuccess) {
            g_init_err = std::string("mode table upload: ") + hipGetErrorString(e);
            delete h;
            return LBM_EHIP;
        }
        P.modes = dm;
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
    const int c = h->cur;
    hipError_t e = lbm::launch_moments(h->P, h->cfg.storage, h->f(c), h->phi(c), d_rho, d_p, d_u, d_phi, h->stream);
    return h->hip(e, "moments kernel");
}

int lbm_reduce(lbm_handle *h, double *out, int out_is_host)
{
    if (!h || !out) return LBM_EINVAL;
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
