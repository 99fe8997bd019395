// Internal declarations shared by the kernel and host translation units of liblbm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lbm {

// workgroup tile: one wave per x-row of 64 sites, 4 rows, marching in z
constexpr int TX = 64;
constexpr int TY = 4;
constexpr int NTHREADS = TX * TY;
constexpr int MAX_MODES = 64;
constexpr int NRED = 10;
constexpr int RED_BLOCKS = 1024;  // fixed grid of the reduction (deterministic order)

// Body-force tables, built on the host from the mode table (kz in 0..2 after
// mapping kz < 0 rows to (-k, conj A)):
//   fcol [15][ny * nx] floats, per column (x, y): Re C0 (3), Re C1 (3), Im C1 (3),
//        Re C2 (3), Im C2 (3) with C_k = sum_{rows with kz = k} A e^{2 pi i (kx x/nx + ky y/ny)};
//   fz   [nz] float4: cos, sin of 2 pi z/nz and of 4 pi z/nz.
// a(x, y, z) = Re C0 + Re(C1 t) + Re(C2 t^2), t = e^{2 pi i z/nz}.
constexpr int FCOL = 15;

// Scalar parameters of one configuration, passed by value to every kernel.
struct Params {
    int nx, ny, nz, zchunk;
    int two_phase, curv_mode, n_modes, pad;
    int gx, gy, gz, nblocks;  // step-kernel tile grid (x tiles, y tiles, z chunks)
    float omega;    // 1 / tau
    float p0;       // pressure gauge / storage shift
    float rho_l, rho_g;
    float fs_coef;  // (3/2) delta sigma  (surface-tension normalisation)
    float fnu_coef; // nu / (tau c_s^2)
    float d6;       // 6 D     (diffusion link coefficient, times w_i)
    float k3;       // 3 kappa (sharpening link coefficient, times w_i)
    float k_lo, k_hi;
    const float *fcol;       // device forcing column table, or nullptr
    const float4 *fz;        // device forcing plane twiddles, or nullptr
    const void *mlp;         // device fp16 weights, or nullptr
};

struct Buffers {
    const void *fin;
    void *fout;
    const double *phin;
    double *phout;
    const float *uin;
    float *uout;
};

hipError_t launch_init(const Params &p, int storage, void *fout, double *phi_out, float *u_out, const double *phi0,
                       const double *u0, const double *ps0, hipStream_t s);
hipError_t launch_step(const Params &p, int storage, const Buffers &b, hipStream_t s);
hipError_t launch_moments(const Params &p, int storage, const void *fin, const double *phi, float *rho, float *pr,
                          float *u, double *phi_out, hipStream_t s);
constexpr int HARVEST_BLOCKS = 1024;
constexpr int MAX_SPHERES = 1024;
int mlp_backward_blocks(int64_t B);
hipError_t launch_mlp_forward(const uint16_t *w, const uint16_t *x, int64_t B, float *y, hipStream_t s);
hipError_t launch_mlp_backward(const uint16_t *w, const uint16_t *x, const float *t, int64_t B, float *grad,
                               float *loss, float *partial, hipStream_t s);
hipError_t launch_mlp_adam(float *w, float *m, float *v, const float *g, uint16_t *w16, float lr, float b1, float b2,
                           float eps, float c1, float c2, hipStream_t s);
hipError_t launch_harvest_count(const double *phi, uint32_t N, uint32_t chunk, int blocks, long long *counts,
                                hipStream_t s);
hipError_t launch_harvest_write(const Params &p, const double *phi, uint32_t chunk, int blocks,
                                const long long *offsets, const void *sph, int nb, uint16_t *X, float *Y, int64_t cap,
                                hipStream_t s);
hipError_t launch_reduce(const Params &p, int storage, const void *fin, const double *phi, double *partials,
                         double *out, hipStream_t s);

}  // namespace lbm
