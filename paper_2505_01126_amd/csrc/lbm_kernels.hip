// Hand-written gfx950 kernels of one accLB time step (arXiv 2505.01126, Secs. 2-3)
// other than the step itself (whose device code is in lbm_step.h): the initial
// state, field read-out, reductions, the Runge-Kutta phase-field stage, and the
// host launchers.
#include "lbm_step.h"

namespace lbm {

extern template int step_grid<0>(bool, bool, bool, bool, bool, int);
extern template int step_grid<1>(bool, bool, bool, bool, bool, int);
extern template int step_grid<2>(bool, bool, bool, bool, bool, int);
extern template hipError_t step_launch<0>(const Params *, const Buffers *, const uint32_t *, int, uint32_t *, int, bool,
                                          bool, bool, bool, bool, int, int, hipStream_t);
extern template hipError_t step_launch<1>(const Params *, const Buffers *, const uint32_t *, int, uint32_t *, int, bool,
                                          bool, bool, bool, bool, int, int, hipStream_t);
extern template hipError_t step_launch<2>(const Params *, const Buffers *, const uint32_t *, int, uint32_t *, int, bool,
                                          bool, bool, bool, bool, int, int, hipStream_t);

// ----------------------------------------------------------- initial state
// f^0 = f^eq(p*0, u0) + w H : A0 / (2 c_s^4), A0 = -c_s^2 tau (grad u0 + grad u0^T),
// written pre-shifted (slot of x - c_i) so that the first pull yields f^0 at x.
template <int S>
__global__ void __launch_bounds__(NTHREADS) k_init(Params P, void *fout_, void *phi_out, float *u_out,
                                                   const double *phi0, const double *u0, const double *ps0)
{
    using T = typename Pop<S>::T;
    T *fout = (T *)fout_;
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const uint32_t plane = (uint32_t)nx * ny, N = plane * (uint32_t)nz;
    const uint32_t s = blockIdx.x * NTHREADS + threadIdx.x;
    if (s >= N) return;
    const int x = s % nx, y = (s / nx) % ny, z = s / plane;
    auto nb = [&](int dx, int dy, int dz) {
        return (uint32_t)wrapi(z + dz, nz) * plane + (uint32_t)wrapi(y + dy, ny) * nx + (uint32_t)wrapi(x + dx, nx);
    };
    double u[3] = {0, 0, 0}, G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    if (u0) {
        for (int a = 0; a < 3; a++) u[a] = u0[(size_t)a * N + s];
#pragma unroll
        for (int i = 0; i < 27; i++) {
            const uint32_t t = nb(CX(i), CY(i), CZ(i));
            for (int a = 0; a < 3; a++) {
                const double v = 3.0 * WTD(i) * u0[(size_t)a * N + t];  // G[a][b] = d_b u_a
                G[a][0] += v * CX(i);
                G[a][1] += v * CY(i);
                G[a][2] += v * CZ(i);
            }
        }
    }
    double tau = 1.0 / (double)P.omega;
    if (P.two_phase && P.tau_g > 0.0f) {  // relaxation time of the initial phase field
        const double c = fmin(fmax(phi0[s], 0.0), 1.0);
        tau = c * (double)P.tau_l + (1.0 - c) * (double)P.tau_g;
    }
    double A[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) A[a][b] = -(tau / 3.0) * (G[a][b] + G[b][a]);
    const double dp = (ps0 ? ps0[s] : (double)P.p0) - (double)P.p0;
    const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
    for (int i = 0; i < 27; i++) {
        const double c[3] = {(double)CX(i), (double)CY(i), (double)CZ(i)};
        const double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
        double hA = 0.0;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) hA += (c[a] * c[b] - (a == b ? 1.0 / 3.0 : 0.0)) * A[a][b];
        const double h = dp + 3.0 * cu + 4.5 * cu * cu - 1.5 * u2 + 4.5 * hA;
        // slot of x - c_i in the plane-major layout
        const size_t slot = ((size_t)wrapi(z - CZ(i), nz) * 27 + i) * plane +
                            (uint32_t)wrapi(y - CY(i), ny) * nx + (uint32_t)wrapi(x - CX(i), nx);
        fout[slot] = Pop<S>::enc((float)h);
    }
    if (phi_out) {
        const double ph = P.two_phase ? phi0[s] : 0.0;
        if (P.phi_fix)  // nearest point of the fixed-point grid, clamped to its range [-2, 2)
            ((int32_t *)phi_out)[s] = (int32_t)__builtin_rint(fmin(fmax(ph * 0x1p30, -0x1p31), 0x1p31 - 1.0));
        else
            ((double *)phi_out)[s] = ph;
    }
    if (u_out)
        for (int a = 0; a < 3; a++) u_out[(size_t)a * N + s] = (float)u[a];
}

// -------------------------------------------------- fields and reductions
// Per-site macroscopic state at time n (pull + stencils from global memory).
// Every lane of the wave calls this together (the network stage is a
// wave-wide MFMA); lanes with valid == false only take part in that stage.
template <int S, bool TP, bool FRC, bool ML>
__device__ __forceinline__ void site_state(const Params &P, const void *fin_, const void *phi, uint32_t s,
                                           bool valid, Macro &m, const MlpW &W, MlpWave &wv, int lane)
{
    using T = typename Pop<S>::T;
    const T *fin = (const T *)fin_;
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const uint32_t plane = (uint32_t)nx * ny, N = plane * (uint32_t)nz;
    const int x = s % nx, y = (s / nx) % ny, z = s / plane;
    // the periodic neighbours' coordinates, once per site: index k = 1 + offset
    const uint32_t xk[3] = {(uint32_t)wrapi(x - 1, nx), (uint32_t)x, (uint32_t)wrapi(x + 1, nx)};
    const uint32_t yk[3] = {(uint32_t)wrapi(y - 1, ny) * nx, (uint32_t)y * nx, (uint32_t)wrapi(y + 1, ny) * nx};
    const uint32_t zk[3] = {(uint32_t)wrapi(z - 1, nz), (uint32_t)z, (uint32_t)wrapi(z + 1, nz)};
    // population i of site s + d (plane-major layout) and the phase field there
    auto pop_at = [&](int i, int dx, int dy, int dz) {
        return ((size_t)zk[1 + dz] * 27 + i) * plane + yk[1 + dy] + xk[1 + dx];
    };
    auto site_at = [&](int dx, int dy, int dz) { return zk[1 + dz] * plane + yk[1 + dy] + xk[1 + dx]; };
    M10 M;
    PhiGrad G;
    float ph[27];
    float kfd = 0.f, gn = 0.f;
    bool sel = false;
    if (valid) {
        float hv[27];
#pragma unroll
        for (int i = 0; i < 27; i++) hv[i] = Pop<S>::dec(fin[pop_at(i, -CX(i), -CY(i), -CZ(i))]);
        moments10(hv, M);
        if constexpr (TP) {
#pragma unroll
            for (int i = 0; i < 27; i++) ph[i] = (float)phi_load(phi, site_at(CX(i), CY(i), CZ(i)), P.phi_fix);
            phi_stencil(ph, G);
            if constexpr (ML) sel = mlp_select(G, P, kfd, gn);
        }
    }
    float fs[3] = {0.f, 0.f, 0.f};
    if constexpr (ML) {
        float yv[4] = {0.f, 0.f, 0.f, 0.f};
        mlp_wave(W, wv, sel, ph, yv, lane);
        if (valid) {
            if (sel) surface_blend(G, P, kfd, gn, yv, fs);
            else surface_fd(G, P, fs);
        }
    } else if constexpr (TP) {
        if (valid) surface_fd(G, P, fs);
    }
    if (valid) {
        float aext[3] = {0.f, 0.f, 0.f};
        if constexpr (FRC) {
            forcing_at<false>(P, P.fx[x], (uint32_t)z * ny + y, aext);
        }
        site_macro<TP>(M, G, fs, aext, P, m);
    }
}

template <int S, bool TP, bool FRC, bool ML>
__global__ void __launch_bounds__(NTHREADS) k_moments(Params P, const void *fin, const void *phi, float *rho,
                                                      float *pr, float *u, double *phi_out)
{
    __shared__ char mlp_raw[ML ? sizeof(MlpW) + (NTHREADS / 64) * sizeof(MlpWave) : 1];
    MlpW &W = *(MlpW *)mlp_raw;
    MlpWave *wv = (MlpWave *)(mlp_raw + (ML ? sizeof(MlpW) : 0));
    if constexpr (ML) {
        load_weights((const uint16_t *)P.mlp, W, threadIdx.x, NTHREADS);
        __syncthreads();
    }
    const uint32_t N = (uint32_t)P.nx * P.ny * P.nz;
    const uint32_t s = blockIdx.x * NTHREADS + threadIdx.x;
    const bool valid = s < N;
    Macro m;
    site_state<S, TP, FRC, ML>(P, fin, phi, valid ? s : 0u, valid, m, W, wv[threadIdx.x >> 6], threadIdx.x & 63);
    if (!valid) return;
    if (rho) rho[s] = m.rho;
    if (pr) pr[s] = (P.p0 + m.dp) * m.rho * (1.0f / 3.0f);
    if (u) {
        u[s] = m.u[0];
        u[(size_t)N + s] = m.u[1];
        u[2 * (size_t)N + s] = m.u[2];
    }
    if (phi_out) phi_out[s] = TP ? phi_load(phi, s, P.phi_fix) : 0.0;
}

// Wavefront reductions in FP64: a butterfly over the 64 lanes (xor
// partners 32, 16, .., 1).  Each lane combines the same two operands in the same
// order as its partner, so all lanes end with the same bits, and the pattern is
// fixed, so the result does not depend on scheduling.
constexpr bool red_is_max(int k) { return k == 7 || k == 8; }
template <int K> __device__ __forceinline__ double wave_reduce(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double w = __shfl_xor(v, o, 64);
        v = red_is_max(K) ? fmax(v, w) : v + w;
    }
    return v;
}
__device__ __forceinline__ long long wave_sum_i64(long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// the NRED statistics of this workgroup: one wavefront reduction per
// statistic, then lane 0 of every wave writes its value and thread k < NRED
// combines the NTHREADS / 64 wave values of statistic k in a fixed order
__device__ __forceinline__ void block_reduce(const double (&acc)[NRED], double (&wred)[NTHREADS / 64][NRED],
                                            double &res)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double v[NRED];
    v[0] = wave_reduce<0>(acc[0]);
    v[1] = wave_reduce<1>(acc[1]);
    v[2] = wave_reduce<2>(acc[2]);
    v[3] = wave_reduce<3>(acc[3]);
    v[4] = wave_reduce<4>(acc[4]);
    v[5] = wave_reduce<5>(acc[5]);
    v[6] = wave_reduce<6>(acc[6]);
    v[7] = wave_reduce<7>(acc[7]);
    v[8] = wave_reduce<8>(acc[8]);
    v[9] = wave_reduce<9>(acc[9]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NRED; k++) wred[wave][k] = v[k];
    }
    __syncthreads();
    const int k = threadIdx.x;
    if (k < NRED) {
        res = wred[0][k];
#pragma unroll
        for (int w = 1; w < NTHREADS / 64; w++) res = red_is_max(k) ? fmax(res, wred[w][k]) : res + wred[w][k];
    }
}

// FP64 partial sums per block over a fixed grid-stride partition, combined in
// a fixed order: the result does not depend on scheduling.  With the
// fixed-point phi, sum phi is accumulated as the integer sum of q (exact in
// the FP64 block partials, which stay below 2^53, and in the final int64 sum),
// so it is a function of that integer alone.
template <int S, bool TP, bool FRC, bool ML>
__global__ void __launch_bounds__(NTHREADS) k_reduce(Params P, const void *fin, const void *phi, double *partials)
{
    __shared__ char mlp_raw[ML ? sizeof(MlpW) + (NTHREADS / 64) * sizeof(MlpWave) : 1];
    MlpW &W = *(MlpW *)mlp_raw;
    MlpWave *wv = (MlpWave *)(mlp_raw + (ML ? sizeof(MlpW) : 0));
    if constexpr (ML) {
        load_weights((const uint16_t *)P.mlp, W, threadIdx.x, NTHREADS);
        __syncthreads();
    }
    const uint32_t N = (uint32_t)P.nx * P.ny * P.nz;
    double acc[NRED];
#pragma unroll
    for (int k = 0; k < NRED; k++) acc[k] = 0.0;
    // uniform trip count across the block (the network stage is wave-wide)
    for (uint32_t base = blockIdx.x * NTHREADS; base < N; base += gridDim.x * NTHREADS) {
        const uint32_t s = base + threadIdx.x;
        const bool valid = s < N;
        Macro m;
        site_state<S, TP, FRC, ML>(P, fin, phi, valid ? s : 0u, valid, m, W, wv[threadIdx.x >> 6],
                                   threadIdx.x & 63);
        if (!valid) continue;
        const double ph = TP ? phi_load(phi, s, P.phi_fix) : 0.0;
        const double r = m.rho, pstar = (double)P.p0 + (double)m.dp;
        const double ux = m.u[0], uy = m.u[1], uz = m.u[2];
        const bool bad = !isfinite(pstar) || !isfinite(ux) || !isfinite(uy) || !isfinite(uz) || !isfinite(ph);
        if (bad) {
            acc[9] += 1.0;
            continue;
        }
        const double u2 = ux * ux + uy * uy + uz * uz;
        acc[0] += P.phi_fix ? ph * 0x1p30 : ph;
        acc[1] += r;
        acc[2] += pstar;
        acc[3] += r * ux;
        acc[4] += r * uy;
        acc[5] += r * uz;
        acc[6] += 0.5 * r * u2;
        acc[7] = fmax(acc[7], sqrt(u2));
        acc[8] = TP ? fmax(acc[8], fmax(ph - 1.0, fmax(-ph, 0.0))) : 0.0;
    }
    __shared__ double wred[NTHREADS / 64][NRED];
    double res = 0.0;
    block_reduce(acc, wred, res);
    if (threadIdx.x < NRED) partials[(size_t)blockIdx.x * NRED + threadIdx.x] = res;
}

__global__ void __launch_bounds__(NTHREADS) k_reduce_final(const double *partials, int nblocks, int fix, double *out)
{
    __shared__ double wred[NTHREADS / 64][NRED];
    __shared__ long long wq[NTHREADS / 64];
    double acc[NRED];
    long long q = 0;  // fixed-point phi: integer sum of q
#pragma unroll
    for (int k = 0; k < NRED; k++) acc[k] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += NTHREADS) {
#pragma unroll
        for (int k = 0; k < NRED; k++) {
            const double v = partials[(size_t)b * NRED + k];
            acc[k] = red_is_max(k) ? fmax(acc[k], v) : acc[k] + v;
        }
        if (fix) q += (long long)partials[(size_t)b * NRED];
    }
    q = wave_sum_i64(q);
    if ((threadIdx.x & 63) == 0) wq[threadIdx.x >> 6] = q;
    double res = 0.0;
    block_reduce(acc, wred, res);  // its barrier also publishes wq
    if (threadIdx.x < NRED) {
        long long qs = 0;
#pragma unroll
        for (int w = 0; w < NTHREADS / 64; w++) qs += wq[w];
        out[threadIdx.x] = (fix && threadIdx.x == 0) ? (double)qs * 0x1p-30 : res;
    }
}

// --------------------------------------------------------------- launchers
int batch_grid(int storage, bool tp, bool frc, bool ml, bool fix, bool phys, int tile)
{
    if (storage == 0) return step_grid<0>(tp, frc, ml, fix, phys, tile);
    if (storage == 1) return step_grid<1>(tp, frc, ml, fix, phys, tile);
    return step_grid<2>(tp, frc, ml, fix, phys, tile);
}

hipError_t launch_step_batch(const Params *tab, const Buffers *buf, const uint32_t *first, int nbox,
                             uint32_t *counter, int parity, int storage, bool tp, bool frc, bool ml, bool fix,
                             bool phys, int tile, int grid, hipStream_t s)
{
    if (storage == 0)
        return step_launch<0>(tab, buf, first, nbox, counter, parity, tp, frc, ml, fix, phys, tile, grid, s);
    if (storage == 1)
        return step_launch<1>(tab, buf, first, nbox, counter, parity, tp, frc, ml, fix, phys, tile, grid, s);
    return step_launch<2>(tab, buf, first, nbox, counter, parity, tp, frc, ml, fix, phys, tile, grid, s);
}

int mlp_pass_grid(bool fix, int tile)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (tile == 32) {
        if (fix) (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_mlp_pass_batch<32, true>, NTHREADS, 0);
        else (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_mlp_pass_batch<32, false>, NTHREADS, 0);
    } else {
        if (fix) (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_mlp_pass_batch<64, true>, NTHREADS, 0);
        else (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_mlp_pass_batch<64, false>, NTHREADS, 0);
    }
    return per_cu * cus;
}

hipError_t launch_mlp_pass_batch(const Params *tab, const Buffers *buf, const uint32_t *first, int nbox,
                                 uint32_t *counter, int parity, bool fix, int tile, int grid, hipStream_t s)
{
    dim3 g(grid), block(tile, NTHREADS / tile, 1);
#define PASS(TW_, X_) hipLaunchKernelGGL((k_mlp_pass_batch<TW_, X_>), g, block, 0, s, tab, buf, first, nbox, counter, parity)
    if (tile == 32) {
        if (fix) PASS(32, true);
        else PASS(32, false);
    } else {
        if (fix) PASS(64, true);
        else PASS(64, false);
    }
#undef PASS
    return hipGetLastError();
}

int ac_stage_grid(int tile)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (tile == 32)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_ac_stage_batch<32>, NTHREADS, 0);
    else
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_ac_stage_batch<64>, NTHREADS, 0);
    return per_cu * cus;
}

hipError_t launch_ac_stage_batch(const Params *tab, const Buffers *buf, const uint32_t *first, int nbox,
                                 uint32_t *counter, int parity, double rk_a, double rk_b, int tile, int grid,
                                 hipStream_t s)
{
    dim3 g(grid), block(tile, NTHREADS / tile, 1);
    if (tile == 32)
        hipLaunchKernelGGL(k_ac_stage_batch<32>, g, block, 0, s, tab, buf, first, nbox, counter, parity, rk_a, rk_b);
    else
        hipLaunchKernelGGL(k_ac_stage_batch<64>, g, block, 0, s, tab, buf, first, nbox, counter, parity, rk_a, rk_b);
    return hipGetLastError();
}

hipError_t launch_init(const Params &p, int storage, void *fout, void *phi_out, float *u_out, const double *phi0,
                       const double *u0, const double *ps0, hipStream_t s)
{
    const uint32_t N = (uint32_t)p.nx * p.ny * p.nz;
    dim3 grid((N + NTHREADS - 1) / NTHREADS), block(NTHREADS);
    if (storage == 0) hipLaunchKernelGGL(k_init<0>, grid, block, 0, s, p, fout, phi_out, u_out, phi0, u0, ps0);
    else if (storage == 1) hipLaunchKernelGGL(k_init<1>, grid, block, 0, s, p, fout, phi_out, u_out, phi0, u0, ps0);
    else hipLaunchKernelGGL(k_init<2>, grid, block, 0, s, p, fout, phi_out, u_out, phi0, u0, ps0);
    return hipGetLastError();
}

hipError_t launch_moments(const Params &p, int storage, const void *fin, const void *phi, float *rho, float *pr,
                          float *u, double *phi_out, hipStream_t s)
{
    const uint32_t N = (uint32_t)p.nx * p.ny * p.nz;
    dim3 grid((N + NTHREADS - 1) / NTHREADS), block(NTHREADS);
    const bool tp = p.two_phase != 0, frc = p.n_modes > 0, ml = p.curv_mode == 1;
#define CALL(S_, TP_, F_, M_) \
    hipLaunchKernelGGL((k_moments<S_, TP_, F_, M_>), grid, block, 0, s, p, fin, phi, rho, pr, u, phi_out);
    LBM_DISPATCH(storage, tp, frc, ml, CALL);
#undef CALL
    return hipGetLastError();
}

hipError_t launch_reduce(const Params &p, int storage, const void *fin, const void *phi, double *partials,
                         double *out, hipStream_t s)
{
    dim3 grid(RED_BLOCKS), block(NTHREADS);
    const bool tp = p.two_phase != 0, frc = p.n_modes > 0, ml = p.curv_mode == 1;
#define CALL(S_, TP_, F_, M_) \
    hipLaunchKernelGGL((k_reduce<S_, TP_, F_, M_>), grid, block, 0, s, p, fin, phi, partials);
    LBM_DISPATCH(storage, tp, frc, ml, CALL);
#undef CALL
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_final, dim3(1), block, 0, s, partials, (int)RED_BLOCKS, p.phi_fix, out);
    return hipGetLastError();
}

}  // namespace lbm
