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

// Forcing table in device memory.  Rows with equal kz share one column sum.
struct ModeTable {
    int n;
    int kx[MAX_MODES], ky[MAX_MODES], kz[MAX_MODES];
    float re[MAX_MODES][3], im[MAX_MODES][3];
};

// Scalar parameters of one configuration, passed by value to every kernel.
struct Params {
    int nx, ny, nz, zchunk;
    int two_phase, curv_mode, n_modes, pad;
    float omega;    // 1 / tau
    float p0;       // pressure gauge / storage shift
    float rho_l, rho_g;
    float fs_coef;  // (3/2) delta sigma  (surface-tension normalisation)
    float fnu_coef; // nu / (tau c_s^2)
    float d6;       // 6 D     (diffusion link coefficient, times w_i)
    float k3;       // 3 kappa (sharpening link coefficient, times w_i)
    float k_lo, k_hi;
    const ModeTable *modes;  // device, or nullptr
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
hipError_t launch_reduce(const Params &p, int storage, const void *fin, const double *phi, double *partials,
                         double *out, hipStream_t s);

}  // namespace lbm
