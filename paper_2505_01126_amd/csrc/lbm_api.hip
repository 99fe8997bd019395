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
#include <map>
#include <mutex>

#include "lbm.h"
#include "lbm_internal.h"

namespace {

constexpr size_t ALIGN = 256;
// default z planes per work item: 32 for FP32 populations, 64 for 16-bit ones
// (measured on 512^3: FP16 5.54 ms at 64 vs 5.67 at 32; FP32 equal at both)
int default_zchunk(int storage) { return storage == LBM_STORE_F32 ? 32 : 64; }

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

size_t elem_bytes(int storage) { return storage == LBM_STORE_F32 ? 4 : 2; }

// Byte offsets of every array inside the caller's workspace.
struct Layout {
    size_t f[2], phi[2], u[2], stage[2], mlpy, iflag, frow, fx, self_batch, partials, red, mlp, sph, hcount, total;
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
        const size_t pb = c.phi_storage == LBM_PHI_FIX32 ? 4 : 8;
        L.phi[0] = take(pb * N);
        L.phi[1] = take(pb * N);
        L.u[0] = take(12 * N);
        L.u[1] = take(12 * N);
    } else {
        L.phi[0] = L.phi[1] = L.u[0] = L.u[1] = (size_t)-1;
    }
    if (c.two_phase && c.curv_mode == LBM_CURV_MLP) {  // network outputs and interface flags
        L.mlpy = take(16 * N);
        L.iflag = take((size_t)lbm::flag_segments(c.nx) * c.ny * c.nz);
    } else {
        L.mlpy = L.iflag = (size_t)-1;
    }
    if (c.two_phase && c.ac_rk3) {  // the two intermediate Runge-Kutta stages of phi
        L.stage[0] = take(8 * N);
        L.stage[1] = take(8 * N);
    } else {
        L.stage[0] = L.stage[1] = (size_t)-1;
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
    L.self_batch = take(lbm_batch_bytes(1));  // tables of the box's own one-member batch
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
    if (c->phi_storage != LBM_PHI_F64 && c->phi_storage != LBM_PHI_FIX32) return "phi_storage must be F64 or FIX32";
    if (c->ac_rk3 != 0 && c->ac_rk3 != 1) return "ac_rk3 must be 0 or 1";
    if (c->ac_rk3 && c->two_phase && c->phi_storage == LBM_PHI_FIX32)
        return "the Runge-Kutta phase-field update needs phi_storage F64";
    if (!(c->tau > 0.5) || !std::isfinite(c->tau)) return "tau must be > 1/2";
    if (!(c->rho_l > 0.0) || !std::isfinite(c->rho_l)) return "rho_l must be > 0";
    if (c->two_phase) {
        if (!(c->rho_g > 0.0) || !std::isfinite(c->rho_g)) return "rho_g must be > 0";
        if (!(c->width > 0.0) || !std::isfinite(c->width)) return "width must be > 0";
        if (!(c->mobility >= 0.0) || !std::isfinite(c->mobility)) return "mobility must be >= 0";
        if (!std::isfinite(c->sigma)) return "sigma must be finite";
    }
    if (!std::isfinite(c->p0)) return "p0 must be finite";
    for (int a = 0; a < 3; a++)
        if (!std::isfinite(c->gravity[a])) return "gravity must be finite";
    if (c->tau_g != 0.0 && !(c->tau_g > 0.5 && std::isfinite(c->tau_g))) return "tau_g must be 0 or > 1/2";
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

struct lbm_batch {
    std::vector<lbm_handle *> m;
    std::vector<int> cur0;        // members' buffer parity when the tables were built
    std::vector<lbm::Params> P;   // per-member parameters (the batch's own z-chunk)
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;  // private stream the step-pair graph is recorded on
    char *table = nullptr;
    size_t off_tab = 0, off_buf = 0, off_first = 0, off_counter = 0;
    int storage = 0, grid = 0, parity = 0, zchunk = 32, tile = 64;
    bool tp = false, frc = false, ml = false, fix = false, rk3 = false, phys = false, dirty = true;
    int grid_ac = 0;  // persistent grid of the Runge-Kutta stage kernel
    int grid_ml = 0;  // persistent grid of the learned-curvature pass
    hipGraphExec_t exec = nullptr;
    std::string err;

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
    lbm::Params *d_tab() { return (lbm::Params *)(table + off_tab); }
    // buffer tables [kind][parity][member]: kind 0 the step, 1 and 2 the
    // second and third Runge-Kutta stages of phi, 3 the learned-curvature pass
    lbm::Buffers *d_buf(int kind = 0, int parity = 0)
    {
        return (lbm::Buffers *)(table + off_buf) + (size_t)(2 * kind + parity) * m.size();
    }
    uint32_t *d_first() { return (uint32_t *)(table + off_first); }
    uint32_t *d_counter() { return (uint32_t *)(table + off_counter); }
    void drop_graph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
    }
};

struct lbm_handle {
    lbm_config cfg{};
    lbm::Params P{};
    Layout L{};
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    int cur = 0;
    int64_t steps = 0;
    bool mlp_set = false;
    lbm_batch *self = nullptr;  // lbm_step runs the box as a one-member batch
    std::vector<float> frow_host, fx_host;
    std::string err;

    void *f(int k) { return ws + L.f[k]; }
    void *phi(int k) { return cfg.two_phase ? (void *)(ws + L.phi[k]) : nullptr; }
    void *stage(int k) { return cfg.two_phase && cfg.ac_rk3 ? (void *)(ws + L.stage[k]) : nullptr; }
    void *mlpy() { return cfg.two_phase && cfg.curv_mode == LBM_CURV_MLP ? (void *)(ws + L.mlpy) : nullptr; }
    uint8_t *iflag() { return cfg.two_phase && cfg.curv_mode == LBM_CURV_MLP ? (uint8_t *)(ws + L.iflag) : nullptr; }
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
    int zc = cfg->zchunk > 0 ? cfg->zchunk : default_zchunk(cfg->storage);
    P.zchunk = zc > cfg->nz ? cfg->nz : zc;
    P.two_phase = cfg->two_phase;
    P.curv_mode = cfg->curv_mode;
    P.n_modes = cfg->n_modes;
    P.phi_fix = cfg->two_phase && cfg->phi_storage == LBM_PHI_FIX32;
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
    P.gravity_on = cfg->two_phase && (cfg->gravity[0] != 0.0 || cfg->gravity[1] != 0.0 || cfg->gravity[2] != 0.0);
    for (int a = 0; a < 3; a++) P.grav[a] = P.gravity_on ? (float)cfg->gravity[a] : 0.0f;
    P.rho_mean = P.rho_l;
    P.tau_l = (float)cfg->tau;
    P.tau_g = cfg->two_phase && cfg->tau_g > 0.0 ? (float)cfg->tau_g : 0.0f;
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
    if (e == hipSuccess && h->iflag())  // every item holds interface cells until a step has flagged them
        e = hipMemsetAsync(h->iflag(), 1, (size_t)lbm::flag_segments(cfg->nx) * cfg->ny * cfg->nz, h->stream);
    if (e == hipSuccess && P.gravity_on) {
        // box-mean density from sum phi of the initial state (finite-difference
        // curvature for this reduction: the network weights are not set yet)
        lbm::Params Pr = P;
        Pr.curv_mode = LBM_CURV_FD;
        double red[LBM_NRED];
        double *dred = (double *)(h->ws + L.red);
        e = lbm::launch_reduce(Pr, cfg->storage, h->f(0), h->phi(0), (double *)(h->ws + L.partials), dred,
                               h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(red, dred, sizeof(double) * LBM_NRED, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e == hipSuccess) {
            const double N = (double)cfg->nx * cfg->ny * cfg->nz;
            P.rho_mean = (float)(cfg->rho_g + (cfg->rho_l - cfg->rho_g) * (red[0] / N));
        }
    }
    if (e != hipSuccess) {
        g_init_err = std::string("init kernel: ") + hipGetErrorString(e);
        delete h;
        return LBM_EHIP;
    }
    if (lbm_batch_create(&h->self, &h, 1, h->ws + L.self_batch, lbm_batch_bytes(1)) != LBM_OK) {
        g_init_err = std::string("step tables: ") + lbm_batch_last_error(nullptr);
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
    h->self->stream = h->stream;
    const int rc = lbm_batch_step(h->self, nsteps);
    if (rc != LBM_OK) h->err = h->self->err;
    return rc;
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
    const void *phi = h->phi(h->cur);
    hipError_t e = hipMemcpyAsync(h->ws + h->L.sph, sph.data(), sizeof(double) * 4 * nb, hipMemcpyHostToDevice,
                                  h->stream);
    if (e == hipSuccess) e = lbm::launch_harvest_count(phi, h->P.phi_fix, N, chunk, blocks, counts, h->stream);
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
    if (h) lbm_batch_destroy(h->self);
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
    case LBM_ERANGE: return "size above the fixed maximum of an entry point without a workspace";
    default: return "unknown error";
    }
}

const char *lbm_last_error(const lbm_handle *h)
{
    if (!h) return g_init_err.c_str();
    return h->err.c_str();
}

}  // extern "C"

// ------------------------------------------------------------------ batches

namespace {

struct BatchOffsets {
    size_t tab, buf, first, counter, total;
};

BatchOffsets batch_offsets(int n)
{
    BatchOffsets o{};
    size_t off = 0;
    o.tab = off;
    off = align_up(off + sizeof(lbm::Params) * (size_t)n);
    o.buf = off;
    off = align_up(off + sizeof(lbm::Buffers) * 4 * 2 * (size_t)n);
    o.first = off;
    off = align_up(off + sizeof(uint32_t) * ((size_t)n + 1));
    o.counter = off;
    off = align_up(off + sizeof(uint32_t) * 4 * lbm::QCOUNTERS);  // queue counters of the four kernel kinds
    o.total = off;
    return o;
}

// work decomposition of one box: tile width (64 or 32 sites in x, 256 sites
// per tile) and z-chunk length
void set_tiling(lbm::Params &P, int tile, int zc)
{
    const int ty = lbm::NTHREADS / tile;
    P.gx = (P.nx + tile - 1) / tile;
    P.gy = (P.ny + ty - 1) / ty;
    P.zchunk = zc > P.nz ? P.nz : zc;
    P.gz = (P.nz + P.zchunk - 1) / P.zchunk;
    P.nblocks = P.gx * P.gy * P.gz;
}

// Upload the parameter table, both parities of the buffer table and the
// work-item prefix sums for the members' current state.
int batch_upload(lbm_batch *b)
{
    const int n = (int)b->m.size();
    std::vector<lbm::Buffers> buf(4 * 2 * (size_t)n, lbm::Buffers{});
    std::vector<uint32_t> first((size_t)n + 1, 0u);
    for (int i = 0; i < n; i++) {
        lbm_handle *h = b->m[i];
        b->cur0[i] = h->cur;
        for (int p = 0; p < 2; p++) {
            const int c = h->cur ^ p, o = c ^ 1;
            // with the Runge-Kutta update the step's own Euler update of phi
            // is the first stage (into stage 0); stages 2 and 3 follow
            // the kernel that writes a step's final phi also writes the interface
            // flags that the next network pass reads (with Runge-Kutta, the last stage)
            buf[(size_t)p * n + i] = lbm::Buffers{h->f(c), h->f(o), h->phi(c), b->rk3 ? h->stage(0) : h->phi(o),
                                                  h->u(c), h->u(o), nullptr, h->mlpy(),
                                                  b->rk3 ? nullptr : h->iflag()};
            if (b->ml)
                buf[(size_t)(6 + p) * n + i] = lbm::Buffers{nullptr, nullptr, h->phi(c), nullptr, nullptr,
                                                            nullptr, nullptr, h->mlpy(), h->iflag()};
            if (b->rk3) {
                buf[(size_t)(2 + p) * n + i] =
                    lbm::Buffers{nullptr, nullptr, h->stage(0), h->stage(1), h->u(c), nullptr, h->phi(c)};
                buf[(size_t)(4 + p) * n + i] = lbm::Buffers{nullptr, nullptr, h->stage(1), h->phi(o), h->u(c),
                                                            nullptr, h->phi(c), nullptr, h->iflag()};
            }
        }
        first[i + 1] = first[i] + (uint32_t)b->P[i].nblocks;
    }
    // all queue counters start at zero (each launch clears the other parity's counters)
    hipError_t e = hipMemsetAsync(b->d_counter(), 0, 4 * lbm::QCOUNTERS * sizeof(uint32_t), b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_tab(), b->P.data(), sizeof(lbm::Params) * n, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_buf(), buf.data(), sizeof(lbm::Buffers) * 4 * 2 * n, hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_first(), first.data(), sizeof(uint32_t) * (n + 1), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);  // host staging is released below
    if (e != hipSuccess) return b->hip(e, "batch table upload");
    b->parity = 0;
    b->dirty = false;
    b->drop_graph();
    return LBM_OK;
}

// one time step of the batch with the given parity of the buffer tables: with
// the learned curvature its network pass, then the step kernel, then, with the
// Runge-Kutta phase-field update, its second and third stages (Shu-Osher
// coefficients 3/4, 1/4 and 1/3, 2/3)
hipError_t batch_launch(lbm_batch *b, int parity, hipStream_t s)
{
    const int n = (int)b->m.size();
    if (b->ml) {
        hipError_t e = lbm::launch_mlp_pass_batch(b->d_tab(), b->d_buf(3, parity), b->d_first(), n,
                                                  b->d_counter() + 3 * lbm::QCOUNTERS, parity, b->fix, b->tile,
                                                  b->grid_ml, s);
        if (e != hipSuccess) return e;
    }
    hipError_t e = lbm::launch_step_batch(b->d_tab(), b->d_buf(0, parity), b->d_first(), n, b->d_counter(), parity,
                                          b->storage, b->tp, b->frc, b->ml, b->fix, b->phys, b->tile, b->grid, s);
    if (e == hipSuccess && b->rk3)
        e = lbm::launch_ac_stage_batch(b->d_tab(), b->d_buf(1, parity), b->d_first(), n,
                                       b->d_counter() + 1 * lbm::QCOUNTERS, parity, 0.75, 0.25, b->tile, b->grid_ac, s);
    if (e == hipSuccess && b->rk3)
        e = lbm::launch_ac_stage_batch(b->d_tab(), b->d_buf(2, parity), b->d_first(), n,
                                       b->d_counter() + 2 * lbm::QCOUNTERS, parity, 1.0 / 3.0, 2.0 / 3.0, b->tile,
                                       b->grid_ac, s);
    return e;
}

void batch_advance(lbm_batch *b, int64_t k)
{
    for (lbm_handle *h : b->m) {
        h->cur ^= (int)(k & 1);
        h->steps += k;
    }
    b->parity ^= (int)(k & 1);
}

std::mutex g_tune_mu;
std::map<std::string, std::pair<int, int>> g_tune_cache;  // member shapes and kernel flags -> (tile, z-chunk)
thread_local std::string g_batch_err;

}  // namespace

extern "C" {

size_t lbm_batch_bytes(int n)
{
    if (n < 1 || n > LBM_BATCH_MAX) return 0;
    return batch_offsets(n).total;
}

int lbm_batch_create(lbm_batch **out, lbm_handle *const *members, int n, void *d_table, size_t table_bytes)
{
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    auto bad = [](int code, const char *why) {
        g_batch_err = why;
        return code;
    };
    if (n < 1 || n > LBM_BATCH_MAX || !members) return bad(LBM_EINVAL, "n must be in 1 .. LBM_BATCH_MAX");
    if (!d_table || ((uintptr_t)d_table % ALIGN) != 0)
        return bad(LBM_EINVAL, "table must be a 256-byte aligned device pointer");
    const BatchOffsets o = batch_offsets(n);
    if (table_bytes < o.total) return bad(LBM_ENOSPACE, "table smaller than lbm_batch_bytes(n)");
    const lbm_handle *h0 = members[0];
    if (!h0) return bad(LBM_EINVAL, "NULL member");
    std::vector<lbm_handle *> m(members, members + n);
    std::vector<lbm_handle *> sorted(m);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) return bad(LBM_EINVAL, "repeated member");
    for (lbm_handle *h : m) {
        if (!h) return bad(LBM_EINVAL, "NULL member");
        if (h->cfg.storage != h0->cfg.storage || h->cfg.two_phase != h0->cfg.two_phase ||
            h->cfg.curv_mode != h0->cfg.curv_mode || (h->cfg.n_modes > 0) != (h0->cfg.n_modes > 0) ||
            h->P.phi_fix != h0->P.phi_fix || (h->cfg.two_phase && h->cfg.ac_rk3) != (h0->cfg.two_phase && h0->cfg.ac_rk3) ||
            (h->P.gravity_on || h->P.tau_g > 0.0f) != (h0->P.gravity_on || h0->P.tau_g > 0.0f))
            return bad(LBM_EINVAL, "members differ in storage, phi storage or integrator, two_phase, curv_mode, "
                                   "forcing, or in having buoyancy or a viscosity contrast");
        if (h->stream != h0->stream) return bad(LBM_EINVAL, "members are on different streams");
    }
    lbm_batch *b = new (std::nothrow) lbm_batch();
    if (!b) return bad(LBM_EINVAL, "out of host memory");
    b->m = m;
    b->cur0.assign(n, 0);
    b->stream = h0->stream;
    b->table = (char *)d_table;
    b->off_tab = o.tab;
    b->off_buf = o.buf;
    b->off_first = o.first;
    b->off_counter = o.counter;
    b->storage = h0->cfg.storage;
    b->tp = h0->cfg.two_phase != 0;
    b->frc = h0->cfg.n_modes > 0;
    b->ml = h0->cfg.curv_mode == LBM_CURV_MLP;
    b->fix = h0->P.phi_fix != 0;
    b->rk3 = h0->cfg.two_phase && h0->cfg.ac_rk3;
    b->phys = h0->P.gravity_on || h0->P.tau_g > 0.0f;
    for (lbm_handle *h : m) b->P.push_back(h->P);
    b->grid = lbm::batch_grid(b->storage, b->tp, b->frc, b->ml, b->fix, b->phys, b->tile);
    b->grid_ac = b->rk3 ? lbm::ac_stage_grid(b->tile) : 1;
    b->grid_ml = b->ml ? lbm::mlp_pass_grid(b->fix, b->tile) : 1;
    if (b->grid <= 0 || b->grid_ac <= 0 || b->grid_ml <= 0) {
        delete b;
        return bad(LBM_EHIP, "occupancy query failed");
    }
    if (hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess) {
        delete b;
        return bad(LBM_EHIP, "capture stream creation failed");
    }
    if (int rc = batch_upload(b)) {
        g_batch_err = b->err;
        (void)hipStreamDestroy(b->capture);
        delete b;
        return rc;
    }
    *out = b;
    return LBM_OK;
}

int lbm_batch_step(lbm_batch *b, int64_t nsteps)
{
    if (!b) return LBM_EINVAL;
    if (nsteps < 0) return b->fail(LBM_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return LBM_OK;
    const int n = (int)b->m.size();
    for (int i = 0; i < n; i++) {
        lbm_handle *h = b->m[i];
        if (b->ml && !h->mlp_set) return b->fail(LBM_ESTATE, "MLP weights not set on a member");
        if (h->cur != (b->cur0[i] ^ b->parity)) b->dirty = true;  // stepped on its own meanwhile
    }
    if (b->dirty)
        if (int rc = batch_upload(b)) return rc;
    int64_t left = nsteps;
    if (b->parity == 1) {  // realign so that graph replays start at parity 0
        if (int rc = b->hip(batch_launch(b, 1, b->stream), "batch kernel")) return rc;
        batch_advance(b, 1);
        left--;
    }
    if (left >= 2 && !b->exec) {
        hipGraph_t g = nullptr;
        // recorded on the private stream (the members' stream may be the
        // legacy default stream, which cannot be captured), replayed on theirs
        hipError_t e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t e0 = batch_launch(b, 0, b->capture);
            hipError_t e1 = batch_launch(b, 1, b->capture);
            e = hipStreamEndCapture(b->capture, &g);
            if (e == hipSuccess) e = e0 != hipSuccess ? e0 : e1;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            b->exec = nullptr;
            return b->hip(e, "batch graph capture");
        }
    }
    for (; left >= 2; left -= 2) {
        if (int rc = b->hip(hipGraphLaunch(b->exec, b->stream), "batch graph launch")) return rc;
        batch_advance(b, 2);
    }
    if (left == 1) {
        if (int rc = b->hip(batch_launch(b, 0, b->stream), "batch kernel")) return rc;
        batch_advance(b, 1);
    }
    return LBM_OK;
}

int lbm_batch_tune(lbm_batch *b, int steps_per_candidate, int *tile_out, int *zchunk_out)
{
    if (!b) return LBM_EINVAL;
    if (steps_per_candidate < 1) return b->fail(LBM_EINVAL, "steps_per_candidate must be >= 1");
    std::vector<std::string> shapes;
    for (lbm_handle *h : b->m)
        shapes.push_back(std::to_string(h->cfg.nx) + "x" + std::to_string(h->cfg.ny) + "x" + std::to_string(h->cfg.nz));
    std::sort(shapes.begin(), shapes.end());
    std::string key = std::to_string(b->storage) + (b->tp ? "t" : "s") + (b->frc ? "f" : "-") + (b->ml ? "m" : "d") + (b->fix ? "q" : "") + (b->rk3 ? "r" : "") + (b->phys ? "g" : "");
    for (const std::string &sh : shapes) key += "," + sh;
    auto apply = [&](int tile, int zc) -> int { return lbm_batch_set_tiling(b, tile, zc); };
    int best_tile = -1, best_zc = -1;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            best_tile = it->second.first;
            best_zc = it->second.second;
        }
    }
    if (best_tile < 0) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (int rc = b->hip(hipEventCreate(&e0), "event")) return rc;
        if (int rc = b->hip(hipEventCreate(&e1), "event")) {
            (void)hipEventDestroy(e0);
            return rc;
        }
        float best_ms = 0.f;
        int rc = LBM_OK;
        for (int tile : {64, 32}) {
            for (int zc : {8, 16, 32, 64}) {
                if ((rc = apply(tile, zc))) break;
                if ((rc = lbm_batch_step(b, 1))) break;
                if ((rc = b->hip(hipEventRecord(e0, b->stream), "event"))) break;
                if ((rc = lbm_batch_step(b, steps_per_candidate))) break;
                if ((rc = b->hip(hipEventRecord(e1, b->stream), "event"))) break;
                if ((rc = b->hip(hipEventSynchronize(e1), "event"))) break;
                float ms = 0.f;
                if ((rc = b->hip(hipEventElapsedTime(&ms, e0, e1), "event"))) break;
                if (best_tile < 0 || ms < best_ms) {
                    best_tile = tile;
                    best_zc = zc;
                    best_ms = ms;
                }
            }
            if (rc) break;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc) return rc;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = {best_tile, best_zc};
    }
    if (int rc = apply(best_tile, best_zc)) return rc;
    if (tile_out) *tile_out = best_tile;
    if (zchunk_out) *zchunk_out = best_zc;
    return LBM_OK;
}

int lbm_batch_set_tiling(lbm_batch *b, int tile, int zchunk)
{
    if (!b) return LBM_EINVAL;
    if (tile != 64 && tile != 32) return b->fail(LBM_EINVAL, "tile must be 64 or 32");
    if (zchunk < 1) return b->fail(LBM_EINVAL, "zchunk must be >= 1");
    const int grid = lbm::batch_grid(b->storage, b->tp, b->frc, b->ml, b->fix, b->phys, tile);
    const int grid_ac = b->rk3 ? lbm::ac_stage_grid(tile) : 1;
    const int grid_ml = b->ml ? lbm::mlp_pass_grid(b->fix, tile) : 1;
    if (grid <= 0 || grid_ac <= 0 || grid_ml <= 0) return b->fail(LBM_EHIP, "occupancy query failed");
    for (lbm::Params &P : b->P) set_tiling(P, tile, zchunk);
    b->tile = tile;
    b->zchunk = zchunk;
    b->grid = grid;
    b->grid_ac = grid_ac;
    b->grid_ml = grid_ml;
    b->dirty = true;
    return LBM_OK;
}

int lbm_batch_destroy(lbm_batch *b)
{
    if (b) {
        b->drop_graph();
        if (b->capture) (void)hipStreamDestroy(b->capture);
    }
    delete b;
    return LBM_OK;
}

const char *lbm_batch_last_error(const lbm_batch *b)
{
    if (!b) return g_batch_err.c_str();
    return b->err.c_str();
}

}  // extern "C"
