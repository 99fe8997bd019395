// Learned curvature network on gfx950 FP16 MFMA: forward, backward (MSE),
// Adam, and the harvest of training samples from a phase field.
//
// Network 27 -> 64 -> 64 -> 4 with tanh hidden layers; fp16 weights and
// activations, FP32 accumulation (v_mfma_f32_16x16x32_f16).  One wave handles
// a tile of 16 samples.  Operand layouts of the 16x16x32 MFMA (lane l):
//   A: row l % 16, k = 8 (l / 16) + j, j = 0..7
//   B: column l % 16, k = 8 (l / 16) + j
//   C: column l % 16, rows 4 (l / 16) + i, i = 0..3
#include <hip/hip_runtime.h>

#include <mutex>

#include "lbm.h"
#include "lbm_internal.h"
#include "lbm_mlp_device.h"

namespace lbm {

constexpr int CHUNK = 64;  // samples per workgroup pass of the backward (4 waves x 16)

__device__ __forceinline__ half8 load_x(const uint16_t *__restrict__ x, int64_t row, int64_t B, int kq)
{
    half8 v;
    if (row < B) {
        const uint4 raw = *(const uint4 *)(x + row * KIN + 8 * kq);
        v = __builtin_bit_cast(half8, raw);
    } else {
#pragma unroll
        for (int j = 0; j < 8; j++) v[j] = (_Float16)0.0f;
    }
    return v;
}

__global__ void __launch_bounds__(256) k_mlp_forward(const uint16_t *__restrict__ w, const uint16_t *__restrict__ x,
                                                     int64_t B, float *__restrict__ y)
{
    __shared__ WLds L;
    __shared__ _Float16 hbuf[4][2][16][NH];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    load_weights(w, L, tid, 256);
    __syncthreads();
    const int64_t ntiles = (B + 15) / 16;
    for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t < ntiles; t += (int64_t)gridDim.x * 4) {
        const int64_t s0 = t * 16;
        const half8 xa = load_x(x, s0 + (lane & 15), B, lane >> 4);
        const f32x4 o = forward_tile(L, xa, hbuf[wave][0], hbuf[wave][1], lane);
        const int col = lane & 15, kq = lane >> 4;
        if (col < NOUT)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int64_t s = s0 + 4 * kq + i;
                if (s < B) y[s * NOUT + col] = o[i];
            }
    }
}

// ------------------------------------------------------------- backward
// Per workgroup: a fixed set of 64-sample chunks (chunk c -> block c % grid);
// forward with saved activations, then
//   d3 = 2 (y - t)               (the 1/B is applied at the end)
//   d2 = (d3 W3) * (1 - h2^2),   d1 = (d2 W2) * (1 - h1^2)
//   gW3 = d3^T h2, gW2 = d2^T h1, gW1 = d1^T x, gb = column sums,
// accumulated over the block's chunks; block partials are summed in block
// order by k_mlp_reduce.
struct BLds {
    WLds W;
    _Float16 x[CHUNK][KIN];
    _Float16 h1[CHUNK][NH];
    _Float16 h2[CHUNK][NH];
    _Float16 d2[CHUNK][NH];
    _Float16 d1[CHUNK][NH];
    float d3[CHUNK][NOUT];
};

__device__ __forceinline__ half8 gather8(const _Float16 (*m)[NH], int s0, int col)
{
    half8 v;
#pragma unroll
    for (int j = 0; j < 8; j++) v[j] = m[s0 + j][col];
    return v;
}
__device__ __forceinline__ half8 gather8x(const _Float16 (*m)[KIN], int s0, int col)
{
    half8 v;
#pragma unroll
    for (int j = 0; j < 8; j++) v[j] = m[s0 + j][col];
    return v;
}

__global__ void __launch_bounds__(256) k_mlp_backward(const uint16_t *__restrict__ w, const uint16_t *__restrict__ x,
                                                      const float *__restrict__ tgt, int64_t B,
                                                      float *__restrict__ partial)
{
    extern __shared__ char lds_raw[];
    BLds &S = *(BLds *)lds_raw;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r = lane & 15, kq = lane >> 4;
    load_weights(w, S.W, tid, 256);
    // accumulators: wave owns neuron tile n = 16 wave .. +15 of gW2 (4 column
    // tiles) and of gW1 (2 column tiles); gW3 / biases by thread
    f32x4 acc2[4], acc1[2];
#pragma unroll
    for (int t = 0; t < 4; t++) acc2[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 2; t++) acc1[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    float gw3 = 0.f, gb = 0.f, loss = 0.f;  // gw3: (o = tid/64, k = tid%64); gb: tid < 64 b1, < 128 b2, < 132 b3
    __syncthreads();
    const int64_t nchunks = (B + CHUNK - 1) / CHUNK;
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int64_t s0 = c * CHUNK + 16 * wave;
        // forward, saving x, h1, h2 of this wave's 16 samples
        const half8 xa = load_x(x, s0 + r, B, kq);
#pragma unroll
        for (int j = 0; j < 8; j++) S.x[16 * wave + r][8 * kq + j] = xa[j];
        const f32x4 y = forward_tile(S.W, xa, &S.h1[16 * wave], &S.h2[16 * wave], lane);
        if (r < NOUT)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int64_t s = s0 + 4 * kq + i;
                float d = 0.f;
                if (s < B) {
                    const float e = y[i] - tgt[s * NOUT + r];
                    loss += e * e;
                    d = 2.0f * e;
                }
                S.d3[16 * wave + 4 * kq + i][r] = d;
            }
        __syncthreads();
        // d2 = (d3 W3) (1 - h2^2): thread -> sample tid / 4, 16 neurons
        {
            const int s = tid >> 2, k0 = (tid & 3) * 16;
#pragma unroll
            for (int k = k0; k < k0 + 16; k++) {
                float v = 0.f;
#pragma unroll
                for (int o = 0; o < NOUT; o++) v += S.d3[s][o] * (float)S.W.w3[o][k];
                const float h = (float)S.h2[s][k];
                S.d2[s][k] = (_Float16)(v * (1.0f - h * h));
            }
        }
        __syncthreads();
        // d1 = (d2 W2) (1 - h1^2) on MFMA: wave's 16 samples, 4 column tiles
        {
            const int sw = 16 * wave;
            const half8 a0 = ld8(&S.d2[sw + r][8 * kq]), a1 = ld8(&S.d2[sw + r][32 + 8 * kq]);
#pragma unroll
            for (int nt = 0; nt < 4; nt++) {
                f32x4 cc = {0.f, 0.f, 0.f, 0.f};
                cc = mfma(a0, ld8(&S.W.w2t[16 * nt + r][8 * kq]), cc);
                cc = mfma(a1, ld8(&S.W.w2t[16 * nt + r][32 + 8 * kq]), cc);
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    const int s = sw + 4 * kq + i, k = 16 * nt + r;
                    const float h = (float)S.h1[s][k];
                    S.d1[s][k] = (_Float16)(cc[i] * (1.0f - h * h));
                }
            }
        }
        __syncthreads();
        // weight gradients over the 64 samples of the chunk (K = 2 x 32)
        {
            const int n = 16 * wave + r;  // A row (neuron) of this lane
#pragma unroll
            for (int ks = 0; ks < 2; ks++) {
                const int sb = 32 * ks + 8 * kq;
                const half8 a2 = gather8(S.d2, sb, n);
                const half8 a1 = gather8(S.d1, sb, n);
#pragma unroll
                for (int nt = 0; nt < 4; nt++) acc2[nt] = mfma(a2, gather8(S.h1, sb, 16 * nt + r), acc2[nt]);
#pragma unroll
                for (int nt = 0; nt < 2; nt++) acc1[nt] = mfma(a1, gather8x(S.x, sb, 16 * nt + r), acc1[nt]);
            }
            const int o = tid >> 6, k = tid & 63;
            for (int s = 0; s < CHUNK; s++) gw3 += S.d3[s][o] * (float)S.h2[s][k];
            if (tid < 64) {
                for (int s = 0; s < CHUNK; s++) gb += (float)S.d1[s][tid];
            } else if (tid < 128) {
                for (int s = 0; s < CHUNK; s++) gb += (float)S.d2[s][tid - 64];
            } else if (tid < 128 + NOUT) {
                for (int s = 0; s < CHUNK; s++) gb += S.d3[s][tid - 128];
            }
        }
        __syncthreads();
    }
    // block partial: [NPARAM + 1] floats (gradient, then the loss)
    float *P = partial + (size_t)blockIdx.x * (NPARAM + 1);
    {
        const int n0 = 16 * wave;
#pragma unroll
        for (int nt = 0; nt < 4; nt++)
#pragma unroll
            for (int i = 0; i < 4; i++) P[OW2 + (n0 + 4 * kq + i) * NH + 16 * nt + r] = acc2[nt][i];
#pragma unroll
        for (int nt = 0; nt < 2; nt++)
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int k = 16 * nt + r;
                if (k < NIN) P[OW1 + (n0 + 4 * kq + i) * NIN + k] = acc1[nt][i];
            }
        P[OW3 + (tid >> 6) * NH + (tid & 63)] = gw3;
        if (tid < 64) P[OB1 + tid] = gb;
        else if (tid < 128) P[OB2 + tid - 64] = gb;
        else if (tid < 128 + NOUT) P[OB3 + tid - 128] = gb;
    }
    // loss: fixed-order sum over the lanes that hold outputs
    __shared__ float lsum[256];
    lsum[tid] = loss;
    __syncthreads();
    if (tid == 0) {
        float s = 0.f;
        for (int t = 0; t < 256; t++) s += lsum[t];
        P[NPARAM] = s;
    }
}

__global__ void __launch_bounds__(256) k_mlp_reduce(const float *__restrict__ partial, int nblocks, float inv_b,
                                                    float *__restrict__ grad, float *__restrict__ loss)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p > NPARAM) return;
    float s = 0.f;
    for (int b = 0; b < nblocks; b++) s += partial[(size_t)b * (NPARAM + 1) + p];
    if (p < NPARAM) grad[p] = s * inv_b;
    else loss[0] = s * inv_b;
}

// ----------------------------------------------------------------- Adam
__global__ void __launch_bounds__(256) k_mlp_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                                                  const float *__restrict__ g, uint16_t *__restrict__ w16, float lr,
                                                  float b1, float b2, float eps, float c1, float c2)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= NPARAM) return;
    const float gi = g[p];
    const float mi = b1 * m[p] + (1.0f - b1) * gi;
    const float vi = b2 * v[p] + (1.0f - b2) * gi * gi;
    m[p] = mi;
    v[p] = vi;
    const float wi = w[p] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    w[p] = wi;
    w16[p] = __builtin_bit_cast(uint16_t, (_Float16)wi);
}

// -------------------------------------------------------------- harvest
// Interface cells (0.02 < phi < 0.98) in site order: pass 1 counts them per
// workgroup range, the host scans the counts, pass 2 writes rows at
// offset + rank within the range (workgroup prefix over waves).
__device__ __forceinline__ bool is_interface(double p) { return p > 0.02 && p < 0.98; }

__global__ void __launch_bounds__(256) k_harvest_count(const void *__restrict__ phi, int fix, uint32_t N,
                                                       uint32_t chunk, long long *__restrict__ counts)
{
    __shared__ int wsum[4];
    const uint32_t b0 = blockIdx.x * chunk, b1 = min(b0 + chunk, N);
    int cnt = 0;
    for (uint32_t s = b0 + threadIdx.x; s < b1; s += 256) cnt += is_interface(phi_load(phi, s, fix)) ? 1 : 0;
    // wave sums then fixed-order block sum
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = (long long)wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

struct Sphere {
    double x, y, z, r;
};

__global__ void __launch_bounds__(256) k_harvest_write(Params P, const void *__restrict__ phi, uint32_t chunk,
                                                       const long long *__restrict__ offsets,
                                                       const Sphere *__restrict__ sph, int nb,
                                                       uint16_t *__restrict__ X, float *__restrict__ Y, int64_t cap)
{
    __shared__ int wcnt[4];
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const uint32_t plane = (uint32_t)nx * ny, N = plane * (uint32_t)nz;
    const uint32_t b0 = blockIdx.x * chunk, b1 = min(b0 + chunk, N);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    long long base = offsets[blockIdx.x];
    for (uint32_t s0 = b0; s0 < b1; s0 += 256) {
        const uint32_t s = s0 + threadIdx.x;
        const bool sel = s < b1 && is_interface(phi_load(phi, s, P.phi_fix));
        const unsigned long long ballot = __ballot(sel);
        const int rank = __popcll(ballot & ((1ull << lane) - 1ull));
        if (lane == 0) wcnt[wave] = __popcll(ballot);
        __syncthreads();
        int before = 0;
        for (int w = 0; w < wave; w++) before += wcnt[w];
        const int total = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
        if (sel) {
            const long long row = base + before + rank;
            if (row < cap) {
                const int x = s % nx, y = (s / nx) % ny, z = s / plane;
                uint16_t *xr = X + row * KIN;
#pragma unroll
                for (int i = 0; i < 27; i++) {
                    const int dx = i % 3 - 1, dy = (i / 3) % 3 - 1, dz = i / 9 - 1;
                    const int xx = (x + dx + nx) % nx, yy = (y + dy + ny) % ny, zz = (z + dz + nz) % nz;
                    const double p = phi_load(phi, (uint32_t)zz * plane + (uint32_t)yy * nx + xx, P.phi_fix);
                    xr[i] = __builtin_bit_cast(uint16_t, (_Float16)(2.0 * p - 1.0));  // one rounding
                }
                for (int i = 27; i < KIN; i++) xr[i] = 0;
                // nearest sphere surface (periodic minimum image)
                int best = -1;
                double bestd = 1e300, bd[3] = {0, 0, 0}, br = 0;
                for (int k = 0; k < nb; k++) {
                    double d[3] = {x - sph[k].x, y - sph[k].y, z - sph[k].z};
                    const double L[3] = {(double)nx, (double)ny, (double)nz};
                    for (int a = 0; a < 3; a++) d[a] -= L[a] * rint(d[a] / L[a]);
                    const double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                    const double gap = fabs(rr - fabs(sph[k].r));
                    if (gap < bestd) {
                        bestd = gap;
                        best = k;
                        br = rr;
                        bd[0] = d[0];
                        bd[1] = d[1];
                        bd[2] = d[2];
                    }
                }
                float *yr = Y + row * 4;
                if (best >= 0 && br > 1e-12) {
                    const double R = sph[best].r;
                    const double sg = R > 0 ? -1.0 : 1.0;  // toward phi = 1
                    yr[0] = (float)(R > 0 ? -2.0 / R : 2.0 / (-R));
                    for (int a = 0; a < 3; a++) yr[1 + a] = (float)(sg * bd[a] / br);
                } else {
                    yr[0] = yr[1] = yr[2] = yr[3] = 0.f;
                }
            }
        }
        base += total;
        __syncthreads();
    }
}

// --------------------------------------------------------------- launchers
int mlp_backward_blocks(int64_t B)
{
    const int64_t nchunks = (B + CHUNK - 1) / CHUNK;
    return (int)(nchunks < 512 ? (nchunks > 0 ? nchunks : 1) : 512);
}

hipError_t launch_mlp_forward(const uint16_t *w, const uint16_t *x, int64_t B, float *y, hipStream_t s)
{
    if (B <= 0) return hipSuccess;
    const int64_t ntiles = (B + 15) / 16;
    const int grid = (int)((ntiles + 3) / 4 < 4096 ? (ntiles + 3) / 4 : 4096);
    hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(256), 0, s, w, x, B, y);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const uint16_t *w, const uint16_t *x, const float *t, int64_t B, float *grad,
                               float *loss, float *partial, hipStream_t s)
{
    const int blocks = mlp_backward_blocks(B);
    const size_t lds = sizeof(BLds);
    hipError_t e = hipFuncSetAttribute((const void *)k_mlp_backward, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_backward, dim3(blocks), dim3(256), lds, s, w, x, t, B, partial);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const float inv_b = B > 0 ? 1.0f / (float)B : 0.0f;
    hipLaunchKernelGGL(k_mlp_reduce, dim3((NPARAM + 1 + 255) / 256), dim3(256), 0, s, partial, blocks, inv_b, grad,
                       loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *w, float *m, float *v, const float *g, uint16_t *w16, float lr, float b1, float b2,
                           float eps, float c1, float c2, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, s, w, m, v, g, w16, lr, b1, b2, eps, c1,
                       c2);
    return hipGetLastError();
}

hipError_t launch_harvest_count(const void *phi, int fix, uint32_t N, uint32_t chunk, int blocks, long long *counts,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_harvest_count, dim3(blocks), dim3(256), 0, s, phi, fix, N, chunk, counts);
    return hipGetLastError();
}

hipError_t launch_harvest_write(const Params &p, const void *phi, uint32_t chunk, int blocks,
                                const long long *offsets, const void *sph, int nb, uint16_t *X, float *Y, int64_t cap,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_harvest_write, dim3(blocks), dim3(256), 0, s, p, phi, chunk, offsets, (const Sphere *)sph,
                       nb, X, Y, cap);
    return hipGetLastError();
}

// ------------------------------------------- backward without a workspace
// The block partials of lbm_mlp_backward_static live in a file-scope device
// array sized for LBM_MLP_STATIC_MAX_BATCH samples, one instance per GPU for
// the life of the process.  On the host the array's name is only a stand-in
// for the symbol: kernels get the device address that hipGetSymbolAddress
// returns, looked up once per device (the first call on that device).
constexpr int STATIC_BLOCKS = (LBM_MLP_STATIC_MAX_BATCH + CHUNK - 1) / CHUNK;
static_assert(STATIC_BLOCKS <= 512, "the backward grid is capped at 512 blocks");
static __device__ __align__(256) float scratch[(size_t)STATIC_BLOCKS * (NPARAM + 1)];
constexpr int MAX_DEVICES = 64;

hipError_t mlp_static_scratch(float **out)
{
    static std::mutex mu;
    static float *addr[MAX_DEVICES] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = (float *)p;
    }
    *out = addr[dev];
    return hipSuccess;
}

}  // namespace lbm

int lbm_mlp_backward_static(const uint16_t *d_w, const uint16_t *d_x, const float *d_t, int64_t batch, float *d_grad,
                            float *d_loss, void *stream)
{
    if (!d_w || batch < 0 || !d_grad || !d_loss || (batch > 0 && (!d_x || !d_t))) return LBM_EINVAL;
    if (batch > LBM_MLP_STATIC_MAX_BATCH) return LBM_ERANGE;
    float *partial = nullptr;
    if (lbm::mlp_static_scratch(&partial) != hipSuccess) return LBM_EHIP;
    return lbm::launch_mlp_backward(d_w, d_x, d_t, batch, d_grad, d_loss, partial, (hipStream_t)stream) ==
                   hipSuccess
               ? LBM_OK
               : LBM_EHIP;
}
