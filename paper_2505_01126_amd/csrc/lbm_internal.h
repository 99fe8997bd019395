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
constexpr int QCOUNTERS = 2;  // work-queue counters of one kernel kind (one per launch parity)

// Body-force tables, built on the host in FP64 from the mode table (|kx| <= 2)
// and stored as FP32:
//   frow [nz * ny][16] per x-row (y, z): P0 (3), P1 (3), Q1 (3), P2 (3), Q2 (3), pad,
//        the coefficients of a(x) = P0 + P1 cos t + Q1 sin t + P2 cos 2t + Q2 sin 2t
//        with t = 2 pi x / nx (modes grouped by |kx|, the y and z phases folded in);
//   fx   [nx] float4: cos t, sin t, cos 2t, sin 2t.
// A workgroup row is one wave, so the row coefficients are wave-uniform.
constexpr int FROW = 16;

// Fixed-point phase field: phi = q * 2^-30 with q an int32, so phi in [-2, 2)
// with a quantum of 9.3e-10.  Sums of q are exact, so the phase volume of a
// run with this storage is conserved bit for bit.
constexpr int PHI_FIX_BITS = 30;

// phi of site s as FP64 (exact in both storages)
__device__ __forceinline__ double phi_load(const void *phi, uint32_t s, int fix)
{
    return fix ? (double)((const int32_t *)phi)[s] * 0x1p-30 : ((const double *)phi)[s];
}

// Scalar parameters of one configuration, passed by value to every kernel.
struct Params {
    int nx, ny, nz, zchunk;
    int two_phase, curv_mode, n_modes;
    int phi_fix;    // 1: phi held as int32 fixed point q = phi * 2^PHI_FIX_BITS, 0: FP64
    int gx, gy, gz, nblocks;  // step-kernel tile grid (x tiles, y tiles, z chunks)
    float omega;    // 1 / tau
    float p0;       // pressure gauge / storage shift
    float rho_l, rho_g;
    float fs_coef;  // (3/2) delta sigma  (surface-tension normalisation)
    float fnu_coef; // nu / (tau c_s^2)
    float d6;       // 6 D     (diffusion link coefficient, times w_i)
    float k3;       // 3 kappa (sharpening link coefficient, times w_i)
    float k_lo, k_hi;
    // buoyancy (rho - rho_mean) g when gravity_on; phase-dependent relaxation
    // time tau(phi) = phi tau_l + (1 - phi) tau_g (phi clamped to [0, 1]) when tau_g > 0
    int gravity_on;
    float rho_mean;
    float grav[3];
    float tau_l, tau_g;
    const float *frow;       // device forcing row table, or nullptr
    const float4 *fx;        // device forcing x twiddles, or nullptr
    const void *mlp;         // device fp16 weights, or nullptr
};

struct Buffers {
    const void *fin;
    void *fout;
    const void *phin;  // FP64 or int32 fixed point (Params::phi_fix)
    void *phout;
    const float *uin;
    float *uout;
    const void *phin0;  // phi^n for the Runge-Kutta stages of the phase field
    void *mlpy;         // learned curvature: network outputs (float4 per site; NaN at the
                        // interface cells the criterion does not select), from the pass before the step
    uint8_t *iflag;     // learned curvature: interface flags, one byte per 32-site x-segment of a row,
                        // iflag[(z * ny + y) * nseg + x / 32] (nseg = ceil(nx / 32)), 1 when a site of the
                        // segment has 0.02 < phi < 0.98; written by the kernel that writes the final
                        // phi of a step, read by the network pass of the next; nullptr elsewhere
};

// x-segments of 32 sites per row of the interface flags
__host__ __device__ inline int flag_segments(int nx) { return (nx + 31) / 32; }

hipError_t launch_init(const Params &p, int storage, void *fout, void *phi_out, float *u_out, const double *phi0,
                       const double *u0, const double *ps0, hipStream_t s);
// the time step of one or many boxes in one persistent launch (see k_step_batch)
// tile: workgroup tile width in x, 64 (64 x 4 sites) or 32 (32 x 8)
// fix: phi held as int32 fixed point (two-phase only)
// phys: buoyancy / phase-dependent relaxation time compiled in (two-phase only)
int batch_grid(int storage, bool tp, bool frc, bool ml, bool fix, bool phys, int tile);
hipError_t launch_step_batch(const Params *tab, const Buffers *buf, const uint32_t *first, int nbox,
                             uint32_t *counter, int parity, int storage, bool tp, bool frc, bool ml, bool fix,
                             bool phys, int tile, int grid, hipStream_t s);
// the learned-curvature pass ahead of the step (fix: fixed-point phi)
int mlp_pass_grid(bool fix, int tile);
hipError_t launch_mlp_pass_batch(const Params *tab, const Buffers *buf, const uint32_t *first, int nbox,
                                 uint32_t *counter, int parity, bool fix, int tile, int grid, hipStream_t s);
// one Runge-Kutta stage of the phase field: phout = rk_a phin0 + rk_b (phin + L(phin))
int ac_stage_grid(int tile);
hipError_t launch_ac_stage_batch(const Params *tab, const Buffers *buf, const uint32_t *first, int nbox,
                                 uint32_t *counter, int parity, double rk_a, double rk_b, int tile, int grid,
                                 hipStream_t s);
hipError_t launch_moments(const Params &p, int storage, const void *fin, const void *phi, float *rho, float *pr,
                          float *u, double *phi_out, hipStream_t s);
constexpr int HARVEST_BLOCKS = 1024;
constexpr int MAX_SPHERES = 1024;
int mlp_backward_blocks(int64_t B);
hipError_t launch_mlp_forward(const uint16_t *w, const uint16_t *x, int64_t B, float *y, hipStream_t s);
hipError_t launch_mlp_backward(const uint16_t *w, const uint16_t *x, const float *t, int64_t B, float *grad,
                               float *loss, float *partial, hipStream_t s);
hipError_t launch_mlp_adam(float *w, float *m, float *v, const float *g, uint16_t *w16, float lr, float b1, float b2,
                           float eps, float c1, float c2, hipStream_t s);
hipError_t launch_harvest_count(const void *phi, int fix, uint32_t N, uint32_t chunk, int blocks, long long *counts,
                                hipStream_t s);
hipError_t launch_harvest_write(const Params &p, const void *phi, uint32_t chunk, int blocks,
                                const long long *offsets, const void *sph, int nb, uint16_t *X, float *Y, int64_t cap,
                                hipStream_t s);
hipError_t launch_reduce(const Params &p, int storage, const void *fin, const void *phi, double *partials,
                         double *out, hipStream_t s);

}  // namespace lbm
