// Device code of the learned-curvature network shared by the training kernels
// and the fused step: FP16 MFMA (v_mfma_f32_16x16x32_f16) tiles of 16 samples.
//
// Operand layouts of the 16x16x32 MFMA (lane l):
//   A: row l % 16, k = 8 (l / 16) + j, j = 0..7
//   B: column l % 16, k = 8 (l / 16) + j
//   C: column l % 16, rows 4 (l / 16) + i, i = 0..3
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbm {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// 27 -> 64 -> 64 -> 4, tanh hidden layers; parameter order
// W1[64][27], b1[64], W2[64][64], b2[64], W3[4][64], b3[4]
constexpr int NIN = 27, KIN = 32, NH = 64, NOUT = 4;
constexpr int OW1 = 0, OB1 = OW1 + NH * NIN, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NOUT * NH, NPARAM = OB3 + NOUT;
static_assert(NPARAM == 6212, "parameter count");

__device__ __forceinline__ f32x4 mfma(half8 a, half8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ _Float16 h16(uint16_t bits) { return __builtin_bit_cast(_Float16, bits); }

// LDS written by lanes of this wave becomes visible to its other lanes: LDS
// operations of one wave complete in order; wait for them and keep the
// compiler from moving LDS accesses across.
__device__ __forceinline__ void wave_lds_sync()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
}

// Weights staged in LDS in the layouts the B operands read contiguously.
struct MlpW {
    _Float16 w1[NH][KIN];   // [n][k], k padded 27 -> 32 with zeros
    _Float16 w2[NH][NH];    // [n][k]
    _Float16 w3[16][NH];    // [o][k], rows 4..15 zero
    float b1[NH], b2[NH], b3[16];
};

// training also needs W2 transposed ([k][n]) for the backward product
struct WLds : MlpW {
    _Float16 w2t[NH][NH];
};

// WPtr: pointer to the fp16 weight bits (generic, or global address space)
template <bool TRANSPOSE, class WPtr>
__device__ void load_weights_t(WPtr w, MlpW &L, _Float16 (*w2t)[NH], int tid, int nthr)
{
    for (int e = tid; e < NH * KIN; e += nthr) {
        const int n = e / KIN, k = e % KIN;
        L.w1[n][k] = k < NIN ? h16(w[OW1 + n * NIN + k]) : (_Float16)0.0f;
    }
    for (int e = tid; e < NH * NH; e += nthr) {
        const int n = e / NH, k = e % NH;
        const _Float16 v = h16(w[OW2 + n * NH + k]);
        L.w2[n][k] = v;
        if constexpr (TRANSPOSE) w2t[k][n] = v;
    }
    for (int e = tid; e < 16 * NH; e += nthr) {
        const int o = e / NH, k = e % NH;
        L.w3[o][k] = o < NOUT ? h16(w[OW3 + o * NH + k]) : (_Float16)0.0f;
    }
    for (int e = tid; e < NH; e += nthr) {
        L.b1[e] = (float)h16(w[OB1 + e]);
        L.b2[e] = (float)h16(w[OB2 + e]);
    }
    for (int e = tid; e < 16; e += nthr) L.b3[e] = e < NOUT ? (float)h16(w[OB3 + e]) : 0.0f;
}

template <class WPtr> __device__ inline void load_weights(WPtr w, WLds &L, int tid, int nthr)
{
    load_weights_t<true>(w, L, L.w2t, tid, nthr);
}

template <class WPtr> __device__ inline void load_weights(WPtr w, MlpW &L, int tid, int nthr)
{
    load_weights_t<false>(w, L, nullptr, tid, nthr);
}

__device__ __forceinline__ half8 ld8(const _Float16 *p)
{
    half8 v;
#pragma unroll
    for (int j = 0; j < 8; j++) v[j] = p[j];
    return v;
}

// Forward pass of one 16-sample tile held by a wave.  xa: this lane's A
// fragment of the inputs (row l%16, k = 8(l/16)..+7).  h1, h2: wave-private
// LDS tiles [16][64] receiving the fp16 activations (they may be one tile: the
// MFMAs consume every lane's reads of h1 before the first write of h2);
// returns the FP32 outputs in C layout (column o = l%16 < 4, rows 4(l/16)+i).
__device__ __forceinline__ f32x4 forward_tile(const MlpW &L, half8 xa, _Float16 (*h1)[NH], _Float16 (*h2)[NH],
                                              int lane)
{
    const int r = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
        f32x4 c = {0.f, 0.f, 0.f, 0.f};
        c = mfma(xa, ld8(&L.w1[16 * nt + r][8 * kq]), c);
        const float b = L.b1[16 * nt + r];
#pragma unroll
        for (int i = 0; i < 4; i++) h1[4 * kq + i][16 * nt + r] = (_Float16)tanhf(c[i] + b);
    }
    wave_lds_sync();
    const half8 a0 = ld8(&h1[r][8 * kq]), a1 = ld8(&h1[r][32 + 8 * kq]);
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
        f32x4 c = {0.f, 0.f, 0.f, 0.f};
        c = mfma(a0, ld8(&L.w2[16 * nt + r][8 * kq]), c);
        c = mfma(a1, ld8(&L.w2[16 * nt + r][32 + 8 * kq]), c);
        const float b = L.b2[16 * nt + r];
#pragma unroll
        for (int i = 0; i < 4; i++) h2[4 * kq + i][16 * nt + r] = (_Float16)tanhf(c[i] + b);
    }
    wave_lds_sync();
    const half8 g0 = ld8(&h2[r][8 * kq]), g1 = ld8(&h2[r][32 + 8 * kq]);
    f32x4 y = {0.f, 0.f, 0.f, 0.f};
    y = mfma(g0, ld8(&L.w3[r][8 * kq]), y);
    y = mfma(g1, ld8(&L.w3[r][32 + 8 * kq]), y);
    const float b = L.b3[r];
#pragma unroll
    for (int i = 0; i < 4; i++) y[i] += b;
    return y;
}

// Wave-private LDS scratch for the network evaluation of selected cells: the
// staged inputs [16][KIN] and the activations of both hidden layers share one
// tile (each is read into registers, and consumed by the MFMAs, before the
// next is written).
struct MlpWave {
    _Float16 h[16][NH];
    float y[16][NOUT];
    __device__ _Float16 (*stage())[KIN] { return (_Float16 (*)[KIN]) & h[0][0]; }
};

// Network outputs for the lanes of this wave with sel set (every lane of the
// wave must call this together): the selected lanes are ranked, their stencil
// rows 2 phi - 1 staged 16 at a time and run through one MFMA tile each.
__device__ __forceinline__ void mlp_wave(const MlpW &W, MlpWave &S, bool sel, const float (&ph)[27], float (&y)[4],
                                         int lane)
{
    _Float16 (*stage)[KIN] = S.stage();
    const unsigned long long bal = __ballot(sel);
    const int nsel = __popcll(bal);
    const int rank = __popcll(bal & ((1ull << lane) - 1ull));
    const int row = lane & 15, kq = lane >> 4;
    for (int t = 0; t < nsel; t += 16) {
        const bool mine = sel && rank >= t && rank < t + 16;
        if (mine) {
#pragma unroll
            for (int i = 0; i < NIN; i++) stage[rank - t][i] = (_Float16)(2.0f * ph[i] - 1.0f);
#pragma unroll
            for (int i = NIN; i < KIN; i++) stage[rank - t][i] = (_Float16)0.0f;
        }
        wave_lds_sync();
        half8 xa;
        if (t + row < nsel) {
            xa = ld8(&stage[row][8 * kq]);
        } else {
#pragma unroll
            for (int j = 0; j < 8; j++) xa[j] = (_Float16)0.0f;
        }
        const f32x4 o = forward_tile(W, xa, S.h, S.h, lane);
        if (row < NOUT)
#pragma unroll
            for (int i = 0; i < 4; i++) S.y[4 * kq + i][row] = o[i];
        wave_lds_sync();
        if (mine)
#pragma unroll
            for (int k = 0; k < NOUT; k++) y[k] = S.y[rank - t][k];
        wave_lds_sync();
    }
}

}  // namespace lbm
