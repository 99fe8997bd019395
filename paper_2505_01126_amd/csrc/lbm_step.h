#pragma once

// Device code of one accLB time step (arXiv 2505.01126, Secs. 2-3): the fused
// step kernel and everything it is built from.
//
// k_step fuses, per lattice site and time step:
//   pull-streaming of the 27 D3Q27 populations (structure of arrays, one
//   coalesced row per direction), their moments, the phase-field stencils (LDS-staged phi tile),
//   the forces of Eq. (8), the regularised collision of Eqs. (6)-(7) rebuilt
//   from p*, u and a^(2) (each site writes only its own slots, Sec. 3), and the
//   conservative Allen-Cahn update of Eq. (3).
//
// Populations are stored as h_i = f_i / w_i - P0 in FP32, FP16 or BF16, plane
// by plane: population i of site (x, y, z) at ((z * 27 + i) * ny + y) * nx + x,
// so the 27 rows a site reads or writes lie within 3 x 27 planes and are
// addressed from one per-plane base pointer with 32-bit offsets; all
// arithmetic is FP32.  Each phase-field flux through a face or lattice link is
// evaluated by contraction-free code from identical operands on both sides of
// the link (or once, shared through LDS), so the two sites see bit-identical
// values; the fluxes are accumulated in FP64 into the FP64 phi, so sum phi is
// conserved to FP64 round-off, or, with the int32 fixed-point phi, rounded
// once each to the fixed-point grid and summed exactly, so sum phi is
// conserved bit for bit.
//
// Instruction economy: the D3Q27 weights are a tensor product,
// w(c) = w1(cx) w1(cy) w1(cz) with w1(0) = 2/3, w1(+-1) = 1/6, so the moments
// up to second order (of the populations and of the phi stencil) are computed
// axis by axis, and the post-collision populations, a quadratic polynomial in
// c, are generated the same way.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lbm_internal.h"
#include "lbm_mlp_device.h"

namespace lbm {

// ------------------------------------------------------------------ lattice
// D3Q27 velocity i: c = (i % 3 - 1, (i / 3) % 3 - 1, i / 9 - 1); rest = 13; -c_i = c_{26-i}
__host__ __device__ constexpr int CX(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int CY(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int CZ(int i) { return i / 9 - 1; }
__host__ __device__ constexpr int C2(int i) { return CX(i) * CX(i) + CY(i) * CY(i) + CZ(i) * CZ(i); }
__host__ __device__ constexpr float WT(int i)
{
    return C2(i) == 0 ? 8.0f / 27.0f : C2(i) == 1 ? 2.0f / 27.0f : C2(i) == 2 ? 1.0f / 54.0f : 1.0f / 216.0f;
}
__host__ __device__ constexpr double WTD(int i)
{
    return C2(i) == 0 ? 8.0 / 27.0 : C2(i) == 1 ? 2.0 / 27.0 : C2(i) == 2 ? 1.0 / 54.0 : 1.0 / 216.0;
}

// ----------------------------------------------------------------- storage
template <int S> struct Pop;
// enc: round to nearest even (the initial state); enc_step: the encode of the
// step's post-collision values, given the bits of another population of the
// same site as a source of dither (used by BF16 only).
template <> struct Pop<0> {
    using T = float;
    __device__ static float dec(T v) { return v; }
    __device__ static T enc(float v) { return v; }
    __device__ static T enc_step(float v, uint32_t) { return v; }
};
template <> struct Pop<1> {
    using T = _Float16;
    __device__ static float dec(T v) { return (float)v; }
    __device__ static T enc(float v)  // round to nearest even
    {
        // the conversion is an instruction of its own: the compiler could
        // otherwise fuse the multiply-add that produced v into it (one
        // rounding instead of two) in some template variants and not in
        // others, and the variants would no longer agree bit for bit
        uint32_t r;
        asm("v_cvt_f16_f32 %0, %1" : "=v"(r) : "v"(v));
        return __builtin_bit_cast(T, (uint16_t)r);
    }
    __device__ static T enc_step(float v, uint32_t) { return enc(v); }
};
template <> struct Pop<2> {
    using T = __bf16;
    __device__ static float dec(T v) { return (float)v; }
    __device__ static T enc(float v)  // round to nearest even
    {
        // an instruction of its own, as for FP16 (the low half of the packed
        // conversion of (v, 0))
        uint32_t r;
        asm("v_cvt_pk_bf16_f32 %0, %1, 0" : "=v"(r) : "v"(v));
        return __builtin_bit_cast(T, (uint16_t)r);
    }
    // Stochastic rounding: a BF16 ulp of a shifted population (|h| ~ 0.03) is
    // about 1e-4, far above the change that a weak body force makes in one
    // step, so rounding to nearest drops that change at every step and the
    // flow drifts.  Adding 16 dither bits below the kept mantissa before
    // cutting them off rounds up with probability equal to the cut fraction,
    // so the change survives in expectation.  The dither is the low 16 bits
    // of another population of the site (their low mantissa bits are close to
    // uniform): deterministic, with no state, the same bits in every kernel
    // variant.  A NaN stays a NaN; a value within a dither of the largest
    // finite one may round to infinity.
    __device__ static T enc_step(float v, uint32_t dither)
    {
        const uint32_t b = __builtin_bit_cast(uint32_t, v) + (dither & 0xffffu);
        return __builtin_bit_cast(T, (uint16_t)(b >> 16));
    }
};

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
__device__ __forceinline__ int modi(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// Pointers into global memory.  Kernel arguments are known to be global; a
// pointer read from a descriptor table (the batch kernel) is generic, and
// generic (flat) accesses also count against the LDS wait counter, so every
// LDS wait would then wait for the prefetches too.  These casts restore global
// addressing.
#define LBM_GLOBAL __attribute__((address_space(1)))
template <class T> __device__ __forceinline__ const LBM_GLOBAL T *gconst(const T *p)
{
    return (const LBM_GLOBAL T *)p;
}
template <class T> __device__ __forceinline__ LBM_GLOBAL T *gmut(T *p) { return (LBM_GLOBAL T *)p; }
// Element at a 32-bit byte offset from a wave-uniform base (a plane of a
// field): the scalar-base + 32-bit vector-offset form of a global load, with
// no 64-bit address arithmetic per lane.
template <class T> __device__ __forceinline__ T ldg(const LBM_GLOBAL T *base, uint32_t byte_off)
{
    return *(const LBM_GLOBAL T *)((const LBM_GLOBAL char *)base + byte_off);
}

// Phase-field storage of the step: FP64 (fluxes summed in FP64), or int32
// fixed point q = phi 2^30 (each flux rounded to nearest on that grid, summed
// in wrapping 32-bit integers, so the two sites of a link add and subtract
// exactly the same integer).
template <bool FX> struct PhiStore;
template <> struct PhiStore<false> {
    using T = double;    // stored value
    using Acc = double;  // flux accumulator
    __device__ static float f32(T v) { return (float)v; }
    __device__ static Acc flux(float f) { return (double)f; }
    __device__ static T add(T phi, Acc d) { return phi + d; }
};
template <> struct PhiStore<true> {
    using T = int32_t;
    using Acc = uint32_t;
    __device__ static float f32(T q) { return (float)q * 0x1p-30f; }
    __device__ static Acc flux(float f) { return (uint32_t)(int32_t)__builtin_rintf(f * 0x1p30f); }
    __device__ static T add(T q, Acc d) { return (int32_t)((uint32_t)q + d); }
};

// Raw buffer access to one z plane of populations (27 rows of nx * ny): the
// row offset i * plane goes in the scalar offset, the in-plane offset in the
// vector offset, so no per-row vector address arithmetic is needed.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
template <class T> __device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
}
// Stores of the step's outputs may be non-temporal (cache policy nt): nothing
// reads them before the next launch, by which time a 512^3 state has long left
// L2 and the Infinity Cache, so caching them only evicts input lines that
// neighbouring work items still fetch (measured 2-4 % faster per step on
// 512^3).  The step uses them only where every tile row covers whole 128-byte
// lines: a partial line written past the caches measured slower (a batch of
// boxes with edges 32-96, 8 % slower).  Loads keep the default policy:
// non-temporal loads measured slower.
constexpr int STORE_NT = 2;
template <class T, int AUX = 0>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, T v)
{
    if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, AUX);
    else
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, voff, soff, AUX);
}
template <class T> __device__ __forceinline__ void gstore(LBM_GLOBAL T *p, T v, bool nt)
{
    if (nt)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}
// gstore at a 32-bit byte offset from a wave-uniform base (see ldg)
template <class T> __device__ __forceinline__ void gstb(LBM_GLOBAL T *base, uint32_t byte_off, T v, bool nt)
{
    gstore((LBM_GLOBAL T *)((LBM_GLOBAL char *)base + byte_off), v, nt);
}

// ------------------------------------------------------ separable moments
// Ten sums M_abc = 216 sum_c w(c) v(c) cx^a cy^b cz^c (a + b + c <= 2) of 27
// lattice-ordered values, taken axis by axis (x, then y, then z); along each
// axis the weights are (1, 4, 1) = 6 w1.
struct M10 {
    float m000, m100, m010, m001, m200, m020, m002, m110, m101, m011;
};

__device__ __forceinline__ void moments10(const float (&v)[27], M10 &M)
{
    float r0[9], r1[9], r2[9];
#pragma unroll
    for (int row = 0; row < 9; row++) {
        const float vm = v[3 * row], v0 = v[3 * row + 1], vp = v[3 * row + 2];
        r2[row] = vp + vm;
        r1[row] = vp - vm;
        r0[row] = fmaf(4.0f, v0, r2[row]);
    }
    float p00[3], p01[3], p02[3], p10[3], p11[3], p20[3];
#pragma unroll
    for (int z = 0; z < 3; z++) {
        const int a = 3 * z, b = 3 * z + 1, c = 3 * z + 2;
        float s = r0[c] + r0[a];
        p00[z] = fmaf(4.0f, r0[b], s);
        p01[z] = r0[c] - r0[a];
        p02[z] = s;
        s = r1[c] + r1[a];
        p10[z] = fmaf(4.0f, r1[b], s);
        p11[z] = r1[c] - r1[a];
        p20[z] = fmaf(4.0f, r2[b], r2[c] + r2[a]);
    }
    float s = p00[2] + p00[0];
    M.m000 = fmaf(4.0f, p00[1], s);
    M.m001 = p00[2] - p00[0];
    M.m002 = s;
    s = p01[2] + p01[0];
    M.m010 = fmaf(4.0f, p01[1], s);
    M.m011 = p01[2] - p01[0];
    M.m020 = fmaf(4.0f, p02[1], p02[2] + p02[0]);
    s = p10[2] + p10[0];
    M.m100 = fmaf(4.0f, p10[1], s);
    M.m101 = p10[2] - p10[0];
    M.m110 = fmaf(4.0f, p11[1], p11[2] + p11[0]);
    M.m200 = fmaf(4.0f, p20[1], p20[2] + p20[0]);
}

// ------------------------------------------------------- per-site physics
struct Macro {
    float dp;     // p* - P0
    float rho;
    float u[3];   // u = j + a/2
    float a[3];   // F / rho
    float S[6];   // Pi - p* c_s^2 I  (xx yy zz xy xz yz)
    float omega;  // 1 / tau at this site
};

// Phase-field stencil quantities at a site: g = grad phi, H = Hessian (lattice
// stencils of Sec. 2.3): g = M1 / 72, H_aa = (M_aa - M000/3) / 24, H_ab = M_ab / 24.
struct PhiGrad {
    float phi, g[3], H[6];
};

__device__ __forceinline__ void phi_stencil(const float (&ph)[27], PhiGrad &G)
{
    M10 M;
    moments10(ph, M);
    const float k1 = 1.0f / 72.0f, k2 = 1.0f / 24.0f, t = M.m000 * (1.0f / 3.0f);
    G.phi = ph[13];
    G.g[0] = M.m100 * k1;
    G.g[1] = M.m010 * k1;
    G.g[2] = M.m001 * k1;
    G.H[0] = (M.m200 - t) * k2;
    G.H[1] = (M.m020 - t) * k2;
    G.H[2] = (M.m002 - t) * k2;
    G.H[3] = M.m110 * k2;
    G.H[4] = M.m101 * k2;
    G.H[5] = M.m011 * k2;
}

// Surface-tension force with the finite-difference curvature (Sec. 2.3 CSF
// form): F^s = -(3 delta/2) sigma K |g| g, with K |g| = tr H - g.H.g / |g|^2
// (K = div n, n = g/|g| toward phi = 1); zero where |g| <= 1e-12.
__device__ __forceinline__ void surface_fd(const PhiGrad &G, const Params &P, float (&fs)[3])
{
    const float *g = G.g, *H = G.H;
    const float g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    float cs = 0.f;
    if (g2 > 1e-24f) {
        const float trH = H[0] + H[1] + H[2];
        const float gHg = g[0] * (H[0] * g[0] + H[3] * g[1] + H[4] * g[2]) +
                          g[1] * (H[3] * g[0] + H[1] * g[1] + H[5] * g[2]) +
                          g[2] * (H[4] * g[0] + H[5] * g[1] + H[2] * g[2]);
        cs = -P.fs_coef * (trH - gHg * __builtin_amdgcn_rcpf(g2));
    }
#pragma unroll
    for (int a = 0; a < 3; a++) fs[a] = cs * g[a];
}

// Learned curvature: K_FD and |g| at the site, and whether the network is
// consulted (interface cell 0.02 < phi < 0.98 with |K_FD| > k_lo).
// (The learned-curvature helpers are contraction-free, so that every inlined
// copy -- single-box and batch kernels -- rounds identically.)
__device__ __forceinline__ bool mlp_select(const PhiGrad &G, const Params &P, float &kfd, float &gn)
{
#pragma clang fp contract(off)
    const float *g = G.g, *H = G.H;
    const float g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    kfd = 0.f;
    gn = 0.f;
    if (!(g2 > 1e-24f)) return false;
    const float trH = H[0] + H[1] + H[2];
    const float gHg = g[0] * (H[0] * g[0] + H[3] * g[1] + H[4] * g[2]) +
                      g[1] * (H[3] * g[0] + H[1] * g[1] + H[5] * g[2]) +
                      g[2] * (H[4] * g[0] + H[5] * g[1] + H[2] * g[2]);
    gn = sqrtf(g2);
    kfd = (trH - gHg / g2) / gn;
    return G.phi > 0.02f && G.phi < 0.98f && fabsf(kfd) > P.k_lo;
}

// Blend of the network output y = (K, n) with the finite-difference K and n:
// s = smoothstep((|K_FD| - k_lo) / (k_hi - k_lo)), K = s K_net + (1 - s) K_FD,
// n_s = normalise(s n_net/|n_net| + (1 - s) g/|g|), F^s = -(3 delta/2) sigma K |g|^2 n_s;
// the finite-difference force is kept when the output is non-finite or
// |n_net| is outside [0.5, 1.5].
__device__ __forceinline__ void surface_blend(const PhiGrad &G, const Params &P, float kfd, float gn,
                                              const float (&y)[4], float (&fs)[3])
{
#pragma clang fp contract(off)
    const float nn = sqrtf(y[1] * y[1] + y[2] * y[2] + y[3] * y[3]);
    if (!(isfinite(y[0]) && isfinite(nn) && nn >= 0.5f && nn <= 1.5f)) {
        surface_fd(G, P, fs);
        return;
    }
    const float t = fminf((fabsf(kfd) - P.k_lo) / (P.k_hi - P.k_lo), 1.0f);
    const float sw = t * t * (3.0f - 2.0f * t);
    const float K = sw * y[0] + (1.0f - sw) * kfd;
    float b[3], bn2 = 0.f;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        b[a] = sw * y[1 + a] / nn + (1.0f - sw) * G.g[a] / gn;
        bn2 += b[a] * b[a];
    }
    const float bn = sqrtf(bn2);
    const float c = -P.fs_coef * K * gn * gn;
#pragma unroll
    for (int a = 0; a < 3; a++) fs[a] = c * (bn > 1e-12f ? b[a] / bn : G.g[a] / gn);
}

// Forces of Eq. (8) and the velocity u = j + a/2 from the moments M of the
// pulled populations h_i = f_i / w_i - P0 (Sec. 2.2); fs is the surface-tension force.
//   F^p = -p* c_s^2 grad rho,  grad rho = (rho_l - rho_g) g
//   F^b = rho a_ext
//   F^nu = -(nu / (tau c_s^2)) (Pi - p* c_s^2 I - u0 u0) grad rho, u0 = j + (F^s + F^p + F^b)/(2 rho)
// PH: buoyancy and the phase-dependent relaxation time are compiled in (each
// still switched by its parameter); without them the step keeps one tau.
template <bool TP, bool PH = true>
__device__ __forceinline__ void site_macro(const M10 &M, const PhiGrad &G, const float (&fs)[3],
                                           const float (&aext)[3], const Params &P, Macro &m)
{
    const float r = 1.0f / 216.0f;
    m.dp = M.m000 * r;
    float j[3] = {M.m100 * r, M.m010 * r, M.m001 * r};
    const float pc = m.dp * (1.0f / 3.0f);
    m.S[0] = fmaf(M.m200, r, -pc);
    m.S[1] = fmaf(M.m020, r, -pc);
    m.S[2] = fmaf(M.m002, r, -pc);
    m.S[3] = M.m110 * r;
    m.S[4] = M.m101 * r;
    m.S[5] = M.m011 * r;
    if constexpr (TP) {
        const float rho = P.rho_g + (P.rho_l - P.rho_g) * G.phi;
        const float *g = G.g;
        const float drho = P.rho_l - P.rho_g;
        const float cp = -(P.p0 + m.dp) * (1.0f / 3.0f) * drho;  // F^p = cp * g
        const float inv_rho = __builtin_amdgcn_rcpf(rho);
        float F[3], u0[3];
#pragma unroll
        for (int a = 0; a < 3; a++) F[a] = fs[a] + cp * g[a] + rho * aext[a];
        if (PH && P.gravity_on) {  // buoyancy against the box-mean hydrostatic balance
            const float dr = rho - P.rho_mean;
#pragma unroll
            for (int a = 0; a < 3; a++) F[a] += dr * P.grav[a];
        }
#pragma unroll
        for (int a = 0; a < 3; a++) u0[a] = j[a] + 0.5f * F[a] * inv_rho;
        // relaxation rate and viscous-correction coefficient nu / (tau c_s^2) = 1 - omega / 2
        float omega = P.omega, fnu = P.fnu_coef;
        if (PH && P.tau_g > 0.0f) {
            const float c = fminf(fmaxf(G.phi, 0.0f), 1.0f);
            omega = 1.0f / fmaf(c, P.tau_l - P.tau_g, P.tau_g);
            fnu = 1.0f - 0.5f * omega;
        }
        m.omega = omega;
        const float n0 = m.S[0] - u0[0] * u0[0], n1 = m.S[1] - u0[1] * u0[1], n2 = m.S[2] - u0[2] * u0[2];
        const float n3 = m.S[3] - u0[0] * u0[1], n4 = m.S[4] - u0[0] * u0[2], n5 = m.S[5] - u0[1] * u0[2];
        const float cnu = -fnu * drho;
        F[0] += cnu * (n0 * g[0] + n3 * g[1] + n4 * g[2]);
        F[1] += cnu * (n3 * g[0] + n1 * g[1] + n5 * g[2]);
        F[2] += cnu * (n4 * g[0] + n5 * g[1] + n2 * g[2]);
#pragma unroll
        for (int a = 0; a < 3; a++) {
            m.a[a] = F[a] * inv_rho;
            m.u[a] = j[a] + 0.5f * m.a[a];
        }
        m.rho = rho;
    } else {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            m.a[a] = aext[a];
            m.u[a] = j[a] + 0.5f * aext[a];
        }
        m.rho = P.rho_l;
        m.omega = P.omega;
    }
}

// Regularised post-collision h_i = f^post_i / w_i - P0,
//   f^post = f^eq(p*, u) + (1 - omega) w H : a2 / (2 c_s^4) + S/2,
//   a2 = Pi - p* c_s^2 I - u u + (u a + a u)/2  (closed form of Eq. (7)),
// which is the quadratic polynomial h(c) = base + b.c + c.B.c with
//   b = 3 (u + a/2), B = (9/4)(u w + w u) + (9/2)(1 - omega) a2, w = u + a,
//   base = p* - P0 - (3/2)(u.u + u.a) - (3/2)(1 - omega) tr a2,
// evaluated on the 27 velocities axis by axis.
__device__ __forceinline__ void collide(const Macro &m, float omega, float (&h)[27])
{
    const float ux = m.u[0], uy = m.u[1], uz = m.u[2];
    const float ax = m.a[0], ay = m.a[1], az = m.a[2];
    const float wx = ux + ax, wy = uy + ay, wz = uz + az;
    const float k = 4.5f * (1.0f - omega);
    const float Axx = m.S[0] - ux * ux + ux * ax;
    const float Ayy = m.S[1] - uy * uy + uy * ay;
    const float Azz = m.S[2] - uz * uz + uz * az;
    const float Axy = m.S[3] - ux * uy + 0.5f * (ux * ay + ax * uy);
    const float Axz = m.S[4] - ux * uz + 0.5f * (ux * az + ax * uz);
    const float Ayz = m.S[5] - uy * uz + 0.5f * (uy * az + ay * uz);
    const float Bxx = fmaf(k, Axx, 4.5f * ux * wx);
    const float Byy = fmaf(k, Ayy, 4.5f * uy * wy);
    const float Bzz = fmaf(k, Azz, 4.5f * uz * wz);
    const float Bxy2 = 2.0f * fmaf(k, Axy, 2.25f * (ux * wy + wx * uy));
    const float Bxz2 = 2.0f * fmaf(k, Axz, 2.25f * (ux * wz + wx * uz));
    const float Byz2 = 2.0f * fmaf(k, Ayz, 2.25f * (uy * wz + wy * uz));
    const float bx = 3.0f * ux + 1.5f * ax, by = 3.0f * uy + 1.5f * ay, bz = 3.0f * uz + 1.5f * az;
    const float u2 = ux * ux + uy * uy + uz * uz, ua = ux * ax + uy * ay + uz * az;
    const float base = m.dp - 1.5f * (u2 + ua) - (k * (1.0f / 3.0f)) * (Axx + Ayy + Azz);
    const float gz = base + Bzz;
    const float G[3] = {gz - bz, base, gz + bz};
    const float Y[3] = {by - Byz2, by, by + Byz2};
    const float X[3] = {bx - Bxz2, bx, bx + Bxz2};
#pragma unroll
    for (int z = 0; z < 3; z++) {
        const float ty = G[z] + Byy;
        const float T[3] = {ty - Y[z], G[z], ty + Y[z]};
        const float Xc[3] = {X[z] - Bxy2, X[z], X[z] + Bxy2};
#pragma unroll
        for (int y = 0; y < 3; y++) {
            const int row = 3 * z + y;
            const float tx = T[y] + Bxx;
            h[3 * row] = tx - Xc[y];
            h[3 * row + 1] = T[y];
            h[3 * row + 2] = tx + Xc[y];
        }
    }
}

// ----------------------------------------------------- phase-field fluxes
// WENO-5 (Jiang & Shu) value at the face right of cell c from the upwind-biased
// cells (a, b, c, d, e) = (c-2 .. c+2): candidates q_k, smoothness beta_k with
// the 13/12 and 1/4 factors, linear weights (1/10, 6/10, 3/10), eps = 1e-6,
// p = 2; the nonlinear weights d_k / (eps + beta_k)^2 are taken with one
// reciprocal after scaling by the product of the three denominators.
// Contraction-free (explicit fma only) so both cells of a face get the same bits.
__device__ __forceinline__ float weno5(float a, float b, float c, float d, float e)
{
#pragma clang fp contract(off)
    const float q0 = fmaf(11.0f / 6.0f, c, fmaf(-7.0f / 6.0f, b, (1.0f / 3.0f) * a));
    const float q1 = fmaf(1.0f / 3.0f, d, fmaf(5.0f / 6.0f, c, (-1.0f / 6.0f) * b));
    const float q2 = fmaf(-1.0f / 6.0f, e, fmaf(5.0f / 6.0f, d, (1.0f / 3.0f) * c));
    const float t0 = fmaf(-2.0f, b, a + c), r0 = fmaf(-4.0f, b, fmaf(3.0f, c, a));
    const float t1 = fmaf(-2.0f, c, b + d), r1 = b - d;
    const float t2 = fmaf(-2.0f, d, c + e), r2 = fmaf(3.0f, c, fmaf(-4.0f, d, e));
    float s0 = fmaf((13.0f / 12.0f) * t0, t0, fmaf(0.25f * r0, r0, 1e-6f));
    float s1 = fmaf((13.0f / 12.0f) * t1, t1, fmaf(0.25f * r1, r1, 1e-6f));
    float s2 = fmaf((13.0f / 12.0f) * t2, t2, fmaf(0.25f * r2, r2, 1e-6f));
    s0 = s0 * s0;
    s1 = s1 * s1;
    s2 = s2 * s2;
    const float w0 = 0.1f * (s1 * s2), w1 = 0.6f * (s0 * s2), w2 = 0.3f * (s0 * s1);
    const float num = fmaf(w2, q2, fmaf(w1, q1, w0 * q0));
    return num * __builtin_amdgcn_rcpf((w0 + w1) + w2);
}

// Advective flux ubar * phi_face through the face between cells l and l+1:
// v0..v5 = phi at l-2 .. l+3, ul / ur = velocity component at l / l+1;
// upwinded by the sign of ubar, zero when ubar == 0.
__device__ __forceinline__ float face_flux(float v0, float v1, float v2, float v3, float v4, float v5, float ul,
                                           float ur)
{
#pragma clang fp contract(off)
    const float ub = 0.5f * (ul + ur);
    const bool pos = ub > 0.0f;
    const float a = pos ? v0 : v5, b = pos ? v1 : v4, c = pos ? v2 : v3, d = pos ? v3 : v2, e = pos ? v4 : v1;
    const float h = weno5(a, b, c, d, e);
    return ub == 0.0f ? 0.0f : ub * h;
}

// Diffusion + sharpening flux leaving a toward b = a + c_I (canonical I > 13):
// w_I [6 D (phi_a - phi_b) + 3 kappa (Q_a + Q_b) . c_I]; the projection on c_I
// takes the nonzero components in x, y, z order.
template <int I>
__device__ __forceinline__ float link_flux(float pa, float pb, const float4 &qa, const float4 &qb, float d6w,
                                           float k3w)
{
#pragma clang fp contract(off)
    constexpr int cx = CX(I), cy = CY(I), cz = CZ(I);
    const float tx = qa.x + qb.x, ty = qa.y + qb.y, tz = qa.z + qb.z;
    float s;
    if constexpr (cx != 0) {
        s = cx > 0 ? tx : -tx;
        if constexpr (cy != 0) s = cy > 0 ? s + ty : s - ty;
        if constexpr (cz != 0) s = cz > 0 ? s + tz : s - tz;
    } else if constexpr (cy != 0) {
        s = cy > 0 ? ty : -ty;
        if constexpr (cz != 0) s = cz > 0 ? s + tz : s - tz;
    } else {
        s = cz > 0 ? tz : -tz;
    }
    return fmaf(k3w, s, d6w * (pa - pb));
}

// Q = phi (1 - phi) n, n = g / |g| (zero where |g| <= 1e-12), g from the
// separable first moments (g = M1 / 72; n needs only M1).  Neighbouring
// workgroups, and the prologue and body of one workgroup, evaluate Q at the
// same point from different inlined copies: contraction-free, so every copy
// rounds identically.
__device__ __forceinline__ void q_of(const float (&v)[27], float (&q)[3])
{
#pragma clang fp contract(off)
    float d[9], m[9];
#pragma unroll
    for (int row = 0; row < 9; row++) {
        d[row] = v[3 * row + 2] - v[3 * row];
        m[row] = fmaf(4.0f, v[3 * row + 1], v[3 * row + 2] + v[3 * row]);
    }
    float dx[3], ey[3], sy[3];
#pragma unroll
    for (int z = 0; z < 3; z++) {
        dx[z] = fmaf(4.0f, d[3 * z + 1], d[3 * z + 2] + d[3 * z]);
        ey[z] = m[3 * z + 2] - m[3 * z];
        sy[z] = fmaf(4.0f, m[3 * z + 1], m[3 * z + 2] + m[3 * z]);
    }
    const float Mx = fmaf(4.0f, dx[1], dx[2] + dx[0]);
    const float My = fmaf(4.0f, ey[1], ey[2] + ey[0]);
    const float Mz = sy[2] - sy[0];
    const float m2 = fmaf(Mx, Mx, fmaf(My, My, Mz * Mz));
    const float c = v[13] * (1.0f - v[13]);
    const float s = m2 > 5.184e-21f ? c * __frsqrt_rn(m2) : 0.0f;  // |g| > 1e-12 <=> |M1| > 7.2e-11
    q[0] = s * Mx;
    q[1] = s * My;
    q[2] = s * Mz;
}

// ----------------------------------------------------------------- forcing
// Time-independent body acceleration (Sec. 5.1 uses a fixed large-scale
// field).  The host groups the modes by |kx| and folds the y and z phases into
// per-row coefficients (see lbm_internal.h); a site combines its row's 15
// coefficients with the x twiddles ex = (cos t, sin t, cos 2t, sin 2t).
// UNIFORM: the row is the same in every lane of the wave (one x-row per wave);
// its coefficients are then read with scalar loads through the constant
// address space (the table is read-only while a step runs), which the scalar
// data cache serves and which leave the vector-memory counter to the
// population loads.
#define LBM_CONST __attribute__((address_space(4)))
template <bool UNIFORM>
__device__ __forceinline__ void forcing_at(const Params &P, float4 ex, uint32_t row, float (&a)[3])
{
    float c[15];
    if constexpr (UNIFORM) {
        const LBM_CONST float *r = (const LBM_CONST float *)P.frow + (size_t)row * FROW;
#pragma unroll
        for (int k = 0; k < 15; k++) c[k] = r[k];
    } else {
        const LBM_GLOBAL float *r = gconst(P.frow) + (size_t)row * FROW;
#pragma unroll
        for (int k = 0; k < 15; k++) c[k] = r[k];
    }
#pragma unroll
    for (int d = 0; d < 3; d++)
        a[d] = c[d] + (c[3 + d] * ex.x + c[6 + d] * ex.y) + (c[9 + d] * ex.z + c[12 + d] * ex.w);
}

// ------------------------------------------------------------ fused step
constexpr int HX = 3, HY = 3;                  // phi tile halo (WENO-5 needs 3)
constexpr int NRING = 7;                       // phi planes z-3 .. z+3

// Workgroup tile of TW x (256 / TW) sites: TW = 64 is one wave per x-row (the
// single-box kernel); TW = 32 puts two rows in a wave (boxes of 32 or 96 sites
// in x waste no lanes).  LDS tiles and per-thread work rounds derive from it.
template <int TW> struct Tile {
    static constexpr int X = TW, Y = NTHREADS / TW;
    static constexpr int PX = X + 2 * HX, PY = Y + 2 * HY;
    static constexpr int PLANE = PX * PY;         // phi values per staged plane
    static constexpr int QX = X + 2, QY = Y + 2;  // Q tile (halo 1)
    static constexpr int QPLANE = QX * QY;
    static constexpr int LOADS = (PLANE + NTHREADS - 1) / NTHREADS;
    static constexpr int QPTS = (QPLANE + NTHREADS - 1) / NTHREADS;
    static constexpr int NXF = Y * (X + 1);       // x faces of a plane tile (left of each site + 1)
    static constexpr int NYF = (Y + 1) * X;       // y faces
};

__device__ __forceinline__ int ring(int z) { return (z + 4 * NRING) % NRING; }

// Workgroup barrier for LDS traffic only: waits for this wave's LDS operations,
// not for its outstanding global loads, so prefetches stay in flight across it.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0), vmcnt / expcnt untouched
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Software pipeline over the z planes of a chunk: while plane z is processed,
// the phi plane z+4, the face velocities of plane z+1, the 27 populations of
// plane z+1 and the site's own phi and u_z ahead are already being fetched.
// One work item: the xy tile and z chunk with linear index L (x tile fastest,
// then y tile, then z chunk) of one box.  Every thread of the workgroup calls
// it; it leaves no LDS state that the next call relies on.
//
// ACO (Allen-Cahn only): one Runge-Kutta stage of the phase field and nothing
// else: phi_out = rk_a phi^n + rk_b (phi_in + L(phi_in)) with phi_in staged in
// the LDS ring (B.phin), phi^n read at the site (B.phin0), FP64 phi.
template <int S, bool TP, bool FRC, bool ML, int TW = TX, bool LATE_PF = (S == 0), bool FX = false,
          bool ACO = false, bool PH = false>
__device__ __forceinline__ void step_tile(const Params &P, const Buffers &B, const uint32_t L, double rk_a = 0.0,
                                          double rk_b = 1.0)
{
    static_assert(!ACO || (TP && !FX && !ML), "a Runge-Kutta stage needs the FP64 phase field");
    // ML: the learned curvature.  The network pass (pass_tile) that runs
    // before the step leaves in B.mlpy the network output at every interface
    // cell that the curvature criterion selects (NaN at the other interface
    // cells); the step reads it where its own criterion selects the cell (the
    // same test on the same stencil, so the pass has written there) and falls
    // back to finite differences on NaN, so the network's registers and LDS
    // are not part of the step kernel.
    constexpr bool LBM = !ACO;  // the populations are streamed and collided
    using T = typename Pop<S>::T;
    using PS = PhiStore<FX>;
    using PT = typename PS::T;
    using AT = typename PS::Acc;
    using TL = Tile<TW>;
    constexpr int TXW = TL::X, TYW = TL::Y, PX = TL::PX, PLANE = TL::PLANE, QX = TL::QX, QPLANE = TL::QPLANE,
                  LOADS = TL::LOADS, QPTS = TL::QPTS, NXF = TL::NXF, NYF = TL::NYF;
    // Where the next plane's populations are fetched: 16-bit values pack two
    // to a register, so FP16/BF16 fetch right after the moments (longest
    // prefetch distance) and still fit three waves per SIMD; FP32 fetches after
    // the phase-field work, the shorter live range that fits three waves.  The
    // batch kernel, which holds a few more registers for its work queue, fetches
    // late in every storage mode (a spilled prefetch register would stall).
    constexpr bool kLatePrefetch = TP && LATE_PF;
    constexpr uint32_t ES = sizeof(T);
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t N = plane * (uint32_t)nz;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TXW + tx;
    const int bx = (int)(L % (uint32_t)P.gx), by = (int)((L / (uint32_t)P.gx) % (uint32_t)P.gy);
    const int bz = (int)(L / ((uint32_t)P.gx * (uint32_t)P.gy));
    const int x0 = bx * TXW, y0 = by * TYW, z0 = bz * P.zchunk;
    const int zend = min(z0 + P.zchunk, nz);
    // Lanes past the box's edge (a ragged last tile) step the periodic image of
    // their site: the same inputs give the same bits, so their writes repeat
    // the owner's.  Keeping every lane busy keeps every memory operation
    // unconditional, so the compiler counts the loads in flight exactly instead
    // of draining all of them (stores included) before the next plane.
    const int xg = (x0 + tx) % nx, yg = (y0 + ty) % ny;
    // every tile row of populations, u and phi fills whole 128-byte lines
    const bool nt_rows = (TW * ES) % 128 == 0 && nx % 64 == 0;
    const T *__restrict__ fin = (const T *)B.fin;
    T *__restrict__ fout = (T *)B.fout;
    const LBM_GLOBAL float *__restrict__ ux_in = gconst(B.uin);
    const LBM_GLOBAL float *__restrict__ uy_in = ux_in + N;
    const LBM_GLOBAL float *__restrict__ uz_in = ux_in + 2 * (size_t)N;
    const LBM_GLOBAL PT *__restrict__ phin = gconst((const PT *)B.phin);
    LBM_GLOBAL PT *__restrict__ phout = gmut((PT *)B.phout);
    LBM_GLOBAL float *__restrict__ uout = gmut(B.uout);

    // with one x-row per wave the row is wave-uniform (scalar forcing loads)
    const int yw = TW == 64 ? __builtin_amdgcn_readfirstlane(yg) : yg;
    uint32_t src_xy[9];
#pragma unroll
    for (int dy = -1; dy <= 1; dy++)
#pragma unroll
        for (int dx = -1; dx <= 1; dx++)
            src_xy[(dy + 1) * 3 + dx + 1] = (uint32_t)wrapi(yg - dy, ny) * nx + (uint32_t)wrapi(xg - dx, nx);
    const uint32_t own_xy = (uint32_t)yg * nx + xg;

    float4 ex = {0.f, 0.f, 0.f, 0.f};
    if constexpr (FRC) {
        const LBM_GLOBAL float *fx = gconst((const float *)P.fx) + 4 * xg;
        ex = make_float4(fx[0], fx[1], fx[2], fx[3]);
    }
    const uint32_t yrow = (uint32_t)yw;

    // pull-stream of plane z into hv: h_i(x) = h^post_i(x - c_i)
    // raw storage values: decoded only where they are consumed, so the loads of
    // the next plane stay in flight (a decode right after the load would wait for it)
    // 16-bit values are held zero-extended in full registers: packed two to a
    // register, each pair would wait for its loads on arrival (a 16-bit load
    // into half a register depends on the other half), which would make the
    // prefetch synchronous
    using HT = std::conditional_t<sizeof(T) == 2, uint32_t, T>;
    HT hv[27];
    const size_t pstride = (size_t)27 * plane;  // elements per z plane of populations
    const uint32_t pbytes = 27u * plane * ES;   // bytes per z plane of populations
    auto fetch_pops = [&](int z) {
        const __amdgpu_buffer_rsrc_t zsrc[3] = {plane_rsrc(fin + (size_t)wrapi(z + 1, nz) * pstride, pbytes),
                                                plane_rsrc(fin + (size_t)z * pstride, pbytes),
                                                plane_rsrc(fin + (size_t)wrapi(z - 1, nz) * pstride, pbytes)};
        // running row offset, kept opaque so that the 27 offsets are not all
        // precomputed into scalar registers
        uint32_t soff = 0;
#pragma unroll
        for (int i = 0; i < 27; i++) {
            if constexpr (std::is_same_v<HT, T>)
                hv[i] = bload<T>(zsrc[CZ(i) + 1], src_xy[(CY(i) + 1) * 3 + CX(i) + 1] * ES, soff);
            else
                hv[i] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(zsrc[CZ(i) + 1],
                                                                       src_xy[(CY(i) + 1) * 3 + CX(i) + 1] * ES, soff, 0);
            soff += plane * ES;
            asm volatile("" : "+s"(soff));
        }
    };

    // LDS: phi ring (FP32), Q planes z-1..z+1, x/y face fluxes of plane z, and
    // the global xy offset of every position of the phi tile
    __shared__ float sphi[TP ? NRING : 1][TP ? PLANE : 1];
    constexpr bool AC = TP;  // the Allen-Cahn update runs here
    __shared__ float4 sq[AC ? 3 : 1][AC ? QPLANE : 1];  // Q (x, y, z, unused) per point
    __shared__ float sjx[AC ? NXF : 1];
    __shared__ float sjy[AC ? NYF : 1];
    __shared__ uint32_t sxy[TP ? PLANE : 1];
    const int lc = (ty + HY) * PX + (tx + HX);  // own phi tile index
    const int qc = (ty + 1) * QX + (tx + 1);    // own Q tile index
    int q_lds[QPTS];
    PT phn[LOADS];          // prefetched phi plane
    // The x and y faces of a plane tile are evaluated in three rounds, each
    // wave taking one direction in each: (A) the x face left of every site,
    // (B) the y face below every site, (C) the y faces above the top row
    // (threads 0 .. TXW-1, the first wave) and the x faces right of the last
    // column (threads 64 .. 64+TYW-1, the second wave).  c_lc: the phi tile
    // index of the left (lower) cell of a round-C face.
    const bool c_top = tid < TXW, c_right = tid >= 64 && tid < 64 + TYW;
    const int c_lc = c_top ? (TYW - 1 + HY) * PX + tid + HX : (tid - 64 + HY) * PX + (TXW - 1 + HX);
    float fa_l, fa_r, fb_l, fb_r, fc_l = 0.f, fc_r = 0.f;  // prefetched face velocities
    float jz_left = 0.f, uz_c = 0.f, uz_n = 0.f;
    PT po = 0;              // prefetched own phi

    auto fetch_plane = [&](int z) {
        const LBM_GLOBAL PT *src = phin + (size_t)modi(z, nz) * plane;
#pragma unroll
        for (int k = 0; k < LOADS; k++) {
            const int e = tid + k * NTHREADS;
            if (e < PLANE) phn[k] = src[sxy[e]];
        }
    };
    auto store_plane = [&](int z) {
        float *dst = sphi[ring(z)];
#pragma unroll
        for (int k = 0; k < LOADS; k++) {
            const int e = tid + k * NTHREADS;
            if (e < PLANE) dst[e] = PS::f32(phn[k]);
        }
    };
    // (64-bit per-lane addresses: the scalar-base form of ldg made these loads
    // cost the FP32 step 0.8 %)
    auto fetch_face_u = [&](int z) {
        const uint32_t zo = (uint32_t)z * plane;
        fa_l = ux_in[zo + src_xy[5]];
        fa_r = ux_in[zo + own_xy];
        fb_l = uy_in[zo + src_xy[7]];
        fb_r = uy_in[zo + own_xy];
        if (c_top) {
            fc_l = uy_in[zo + sxy[c_lc]];
            fc_r = uy_in[zo + sxy[c_lc + PX]];
        } else if (c_right) {
            fc_l = ux_in[zo + sxy[c_lc]];
            fc_r = ux_in[zo + sxy[c_lc + 1]];
        }
    };
    auto compute_q = [&](int z) {
        const float *p0 = sphi[ring(z - 1)];
        const float *p1 = sphi[ring(z)];
        const float *p2 = sphi[ring(z + 1)];
        const int slot = (z + 3) % 3;
#pragma unroll
        for (int k = 0; k < QPTS; k++) {
            const int p = tid + k * NTHREADS;
            if (p < QPLANE) {
                const int c = q_lds[k];
                float st[27];
#pragma unroll
                for (int i = 0; i < 27; i++) {
                    const float *pl = CZ(i) < 0 ? p0 : (CZ(i) > 0 ? p2 : p1);
                    st[i] = pl[c + CY(i) * PX + CX(i)];
                }
                float q[3];
                q_of(st, q);
                sq[slot][p] = make_float4(q[0], q[1], q[2], 0.0f);
            }
        }
    };
    // advective x and y fluxes of plane z through the faces of the tile, each
    // face once: x face f of row r lies between tile columns f-1 and f
    // (f = 0..TXW), y face r of column x between tile rows r-1 and r (r = 0..TYW)
    auto compute_faces = [&](int z) {
        const float *pl = sphi[ring(z)];
        {
            const float *p = pl + lc - 3;  // cells x-3 .. x+2 of the row
            sjx[ty * (TXW + 1) + tx] = face_flux(p[0], p[1], p[2], p[3], p[4], p[5], fa_l, fa_r);
        }
        {
            const float *p = pl + lc - 3 * PX;  // cells y-3 .. y+2 of the column
            sjy[ty * TXW + tx] = face_flux(p[0], p[PX], p[2 * PX], p[3 * PX], p[4 * PX], p[5 * PX], fb_l, fb_r);
        }
        if (c_top) {
            const float *p = pl + c_lc - 2 * PX;
            sjy[TYW * TXW + tid] = face_flux(p[0], p[PX], p[2 * PX], p[3 * PX], p[4 * PX], p[5 * PX], fc_l, fc_r);
        } else if (c_right) {
            const float *p = pl + c_lc - 2;
            sjx[(tid - 64) * (TXW + 1) + TXW] = face_flux(p[0], p[1], p[2], p[3], p[4], p[5], fc_l, fc_r);
        }
    };


    if constexpr (TP) {
#pragma unroll
        for (int k = 0; k < LOADS; k++) {
            const int e = tid + k * NTHREADS;
            const int ly = e / PX, lx = e - ly * PX;
            if (e < PLANE) sxy[e] = (uint32_t)modi(y0 + ly - HY, ny) * nx + (uint32_t)modi(x0 + lx - HX, nx);
        }
#pragma unroll
        for (int k = 0; k < QPTS; k++) {
            const int p = tid + k * NTHREADS;
            const int qy = p / QX, qx = p - qy * QX;
            q_lds[k] = (qy + 2) * PX + (qx + 2);  // phi tile centre of Q point (qx, qy)
        }
        for (int z = z0 - 3; z <= z0 + 2; z++) {
            fetch_plane(z);
            store_plane(z);
        }
        fetch_plane(z0 + 3);
        lds_barrier();
        {
            fetch_face_u(z0);
            compute_q(z0 - 1);
            compute_q(z0);
            // z face below the first plane: cells z0-3 .. z0+2, velocities at z0-1, z0
            const float um = uz_in[(uint32_t)modi(z0 - 1, nz) * plane + own_xy];
            uz_c = uz_in[(uint32_t)z0 * plane + own_xy];
            uz_n = ldg(uz_in + (size_t)wrapi(z0 + 1, nz) * plane, own_xy * 4u);
            po = phin[(size_t)z0 * plane + own_xy];
            float v[6];
#pragma unroll
            for (int k = 0; k < 6; k++) v[k] = sphi[ring(z0 - 3 + k)][lc];
            jz_left = face_flux(v[0], v[1], v[2], v[3], v[4], v[5], um, uz_c);
        }
    }
    if (LBM) fetch_pops(z0);

    for (int z = z0; z < zend; z++) {
        const bool more = z + 1 < zend;
        // The prefetches for the next plane run in the last plane of the chunk
        // too, re-reading the current plane's data (in L2, valid addresses): an
        // unconditional load keeps the prefetched values in the same registers
        // on every path, where a skipped one made the compiler copy all 27
        // populations and the other prefetched values on both sides of the branch.
        const int zn = more ? z + 1 : z;
        if constexpr (TP) {
            store_plane(z + 3);
            fetch_plane(zn + 3);
            lds_barrier();
            compute_q(z + 1);
            compute_faces(z);
            fetch_face_u(zn);
            lds_barrier();
        }
        const uint32_t own = (uint32_t)z * plane + own_xy;
        M10 M;
        PhiGrad G;
        float ph[27];
        float kfd = 0.f, gn = 0.f;
        bool sel = false;
        float aext[3] = {0.f, 0.f, 0.f};
        float y[4] = {0.f, 0.f, 0.f, 0.f};  // learned curvature: network output at a selected cell
        {
            if constexpr (LBM) {
                float hf[27];
#pragma unroll
                for (int i = 0; i < 27; i++) {
                    if constexpr (std::is_same_v<HT, T>) hf[i] = Pop<S>::dec(hv[i]);
                    else hf[i] = Pop<S>::dec(__builtin_bit_cast(T, (uint16_t)hv[i]));
                }
                moments10(hf, M);
            }
            if (LBM && !kLatePrefetch) fetch_pops(zn);

            if constexpr (TP) {
                // Allen-Cahn: phi^{n+1} = phi^n - sum (outgoing - incoming) face and link fluxes
                // four independent partial sums keep the dependent add chains short
                AT acc[4];
                acc[0] = PS::flux(sjx[ty * (TXW + 1) + tx]) - PS::flux(sjx[ty * (TXW + 1) + tx + 1]);
                acc[0] += PS::flux(sjy[ty * TXW + tx]) - PS::flux(sjy[(ty + 1) * TXW + tx]);
                {
                    float v[6];
#pragma unroll
                    for (int k = 0; k < 6; k++) v[k] = sphi[ring(z - 2 + k)][lc];
                    const float jr = face_flux(v[0], v[1], v[2], v[3], v[4], v[5], uz_c, uz_n);
                    acc[1] = PS::flux(jz_left) - PS::flux(jr);
                    jz_left = jr;
                    uz_c = uz_n;
                    uz_n = ldg(uz_in + (size_t)wrapi(zn + 1, nz) * plane, own_xy * 4u);
                }
                {
                    // phase-field stencil of this site (LDS)
                    const float *pm = sphi[ring(z - 1)];
                    const float *pc = sphi[ring(z)];
                    const float *pp = sphi[ring(z + 1)];
#pragma unroll
                    for (int i = 0; i < 27; i++) {
                        const float *pl = CZ(i) < 0 ? pm : (CZ(i) > 0 ? pp : pc);
                        ph[i] = pl[lc + CY(i) * PX + CX(i)];
                    }
                    if constexpr (!ACO) phi_stencil(ph, G);
                    if constexpr (ML) sel = mlp_select(G, P, kfd, gn);
                    const float4 *q0 = sq[(z - 1 + 3) % 3];
                    const float4 *q1 = sq[(z + 3) % 3];
                    const float4 *q2 = sq[(z + 1 + 3) % 3];
                    const float4 qo = q1[qc];
                    const float d6w[4] = {0.f, P.d6 * WT(14), P.d6 * WT(15), P.d6 * WT(26)};
                    const float k3w[4] = {0.f, P.k3 * WT(14), P.k3 * WT(15), P.k3 * WT(26)};
                    // links 14 and 15 open the partial sums 2 and 3
#define LB_LINK(I)                                                                                    \
    {                                                                                                 \
        const float4 qn = (CZ(I) > 0 ? q2 : q1)[qc + CY(I) * QX + CX(I)];                             \
        const float4 qs = (CZ(I) > 0 ? q0 : q1)[qc - CY(I) * QX - CX(I)];                             \
        const float fo = link_flux<I>(ph[13], ph[I], qo, qn, d6w[C2(I)], k3w[C2(I)]);                 \
        const float fi = link_flux<I>(ph[26 - I], ph[13], qs, qo, d6w[C2(I)], k3w[C2(I)]);            \
        const AT d = PS::flux(fi) - PS::flux(fo);                                                     \
        if constexpr (I == 14 || I == 15) acc[I & 3] = d;                                             \
        else acc[I & 3] += d;                                                                         \
    }
                    LB_LINK(14) LB_LINK(15) LB_LINK(16) LB_LINK(17) LB_LINK(18) LB_LINK(19) LB_LINK(20)
                    LB_LINK(21) LB_LINK(22) LB_LINK(23) LB_LINK(24) LB_LINK(25) LB_LINK(26)
#undef LB_LINK
                }
                PT pnew;
                if constexpr (ACO)
                    pnew = rk_a * gconst((const double *)B.phin0)[own] +
                           rk_b * (po + ((acc[0] + acc[1]) + (acc[2] + acc[3])));
                else
                    pnew = PS::add(po, (acc[0] + acc[1]) + (acc[2] + acc[3]));
                gstb(phout + (size_t)z * plane, own_xy * (uint32_t)sizeof(PT), pnew, nt_rows && !ACO);
                if constexpr (ML || ACO) {
                    // interface flags of the new phi, as the next network pass
                    // will see it (its FP32 value): one byte per 32-lane half
                    // of the wave, each half one 32-site segment of one row
                    if (B.iflag) {
                        const float pf = PS::f32(pnew);
                        const uint64_t m = __ballot(pf > 0.02f && pf < 0.98f);
                        const int lane = tid & 63;
                        if ((lane & 31) == 0 && x0 + tx < nx && y0 + ty < ny)
                            B.iflag[((size_t)z * ny + yg) * flag_segments(nx) + xg / 32] =
                                (uint8_t)(((lane < 32 ? m : m >> 32) & 0xffffffffull) != 0);
                    }
                }
                po = ldg(phin + (size_t)zn * plane, own_xy * (uint32_t)sizeof(PT));
            }
            // Every other load of this plane is issued before the populations of
            // the next one: loads complete in order, so waiting for a load
            // issued after the 27 prefetches would wait for them as well.
            if constexpr (FRC && LBM) forcing_at<TW == 64>(P, ex, (uint32_t)z * ny + yrow, aext);
            if constexpr (ML) {
                if (sel) {  // the network output that the learned-curvature pass left here
                    const LBM_GLOBAL float *yi = gconst((const float *)B.mlpy) + 4 * (size_t)own;
                    y[0] = yi[0];
                    y[1] = yi[1];
                    y[2] = yi[2];
                    y[3] = yi[3];
                }
            }
            if (LBM && kLatePrefetch) fetch_pops(zn);
        }
        if constexpr (ACO) continue;
        // surface tension: finite differences, or blended with the network
        // output that the learned-curvature pass left for the selected cells
        float fs[3] = {0.f, 0.f, 0.f};
        if constexpr (ML) {
            if (sel)
                surface_blend(G, P, kfd, gn, y, fs);
            else
                surface_fd(G, P, fs);
        } else if constexpr (TP) {
            surface_fd(G, P, fs);
        }
        {
            // moments -> forces, velocity
            Macro m;
            site_macro<TP, PH>(M, G, fs, aext, P, m);

            // regularised collision, written to this site's own slots
            float h[27];
            collide(m, m.omega, h);
            const __amdgpu_buffer_rsrc_t dst = plane_rsrc(fout + (size_t)z * pstride, pbytes);
            auto store_pops = [&](auto aux) {
                uint32_t soff = 0;
#pragma unroll
                for (int i = 0; i < 27; i++) {
                    bstore<T, decltype(aux)::value>(dst, own_xy * ES, soff,
                                                    Pop<S>::enc_step(h[i], __builtin_bit_cast(uint32_t, h[(i + 1) % 27])));
                    soff += plane * ES;
                    asm volatile("" : "+s"(soff));
                }
            };
            if (nt_rows)
                store_pops(std::integral_constant<int, STORE_NT>{});
            else
                store_pops(std::integral_constant<int, 0>{});

            if constexpr (TP) {  // velocity of this step, advects phi in the next one
                gstb(uout + (size_t)z * plane, own_xy * 4u, m.u[0], nt_rows);
                gstb(uout + (size_t)N + (size_t)z * plane, own_xy * 4u, m.u[1], nt_rows);
                gstb(uout + 2 * (size_t)N + (size_t)z * plane, own_xy * 4u, m.u[2], nt_rows);
            }
        }
    }
}

// The learned-curvature pass over one work item, ahead of the step: at every
// interface cell (0.02 < phi < 0.98) it leaves in B.mlpy (float4 per site) the
// network output where the curvature criterion selects the cell and NaN
// elsewhere.  The 3^3 stencil needs phi at halo 1 only, so the pass stages a
// (TW + 2) x (256/TW + 2) tile in a four-plane ring (the step stages halo 3 and
// seven planes for WENO-5): half the phi bytes per item.  The staged values,
// the stencil and the criterion are the step's, so the step selects exactly
// the cells written here.  A work item none of whose sites is an interface
// cell is skipped: its flags are the x-segments of its rows in its planes.
// W: the weights in LDS; *loaded: the weights W holds (reloaded when a box of
// the batch brings others).
template <int TW, bool FX>
__device__ __forceinline__ void pass_tile(const Params &P, const Buffers &B, const uint32_t L, MlpW &W,
                                          MlpWave *wave_lds, const void *&loaded)
{
    using PS = PhiStore<FX>;
    using PT = typename PS::T;
    constexpr int TXW = TW, TYW = NTHREADS / TW;
    constexpr int PX = TXW + 2, PY = TYW + 2, PLANE = PX * PY;
    constexpr int LOADS = (PLANE + NTHREADS - 1) / NTHREADS;
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TXW + tx;
    const int bx = (int)(L % (uint32_t)P.gx), by = (int)((L / (uint32_t)P.gx) % (uint32_t)P.gy);
    const int bz = (int)(L / ((uint32_t)P.gx * (uint32_t)P.gy));
    const int x0 = bx * TXW, y0 = by * TYW, z0 = bz * P.zchunk;
    const int zend = min(z0 + P.zchunk, nz);
    // lanes past a ragged box edge evaluate the periodic image of their site
    // and write the owner's bits again
    const int xg = (x0 + tx) % nx, yg = (y0 + ty) % ny;
    // planes zs .. ze-1 of the chunk hold every interface cell of the item:
    // the first and last planes with a flag set (a candidate cell of plane z
    // sets its segment's flag of plane z)
    int zs = z0, ze = zend;
    if (B.iflag) {
        __shared__ int s_kmin, s_kmax;
        const int nseg = flag_segments(nx);
        const int s0 = x0 / 32, ns = min((x0 + TXW + 31) / 32, nseg) - s0;
        const int nr = min(TYW, ny - y0), np = zend - z0;
        if (tid == 0) {
            s_kmin = np;
            s_kmax = -1;
        }
        __syncthreads();
        int kmin = np, kmax = -1;
        for (int e = tid; e < ns * nr * np; e += NTHREADS) {
            const int si = e % ns, r = (e / ns) % nr, k = e / (ns * nr);
            if (B.iflag[((size_t)(z0 + k) * ny + (y0 + r)) * nseg + s0 + si] != 0) {
                kmin = min(kmin, k);
                kmax = max(kmax, k);
            }
        }
        if (kmax >= 0) {
            atomicMin(&s_kmin, kmin);
            atomicMax(&s_kmax, kmax);
        }
        __syncthreads();
        if (s_kmax < 0) return;  // uniform: no interface cell in the item
        zs = z0 + s_kmin;
        ze = z0 + s_kmax + 1;
    }
    if (P.mlp != loaded) {  // uniform: one box per work item
        load_weights(gconst((const uint16_t *)P.mlp), W, tid, NTHREADS);
        loaded = P.mlp;
    }
    const LBM_GLOBAL PT *__restrict__ phin = gconst((const PT *)B.phin);
    LBM_GLOBAL float *__restrict__ yout = gmut((float *)B.mlpy);
    __shared__ float sphi[4][PLANE];
    __shared__ uint32_t sxy[PLANE];
#pragma unroll
    for (int k = 0; k < LOADS; k++) {
        const int e = tid + k * NTHREADS;
        const int ly = e / PX, lx = e - ly * PX;
        if (e < PLANE) sxy[e] = (uint32_t)modi(y0 + ly - 1, ny) * nx + (uint32_t)modi(x0 + lx - 1, nx);
    }
    __syncthreads();
    // phi planes in flight: three register sets, each fetched three planes
    // ahead of its store into the ring (one plane of work is too short to
    // hide a load from memory); every fetch and store is unconditional (a
    // plane past the chunk re-reads a valid plane) so that the compiler waits
    // for exactly the set it stores
    PT ra[LOADS], rb[LOADS], rc[LOADS];
    auto fetch_plane = [&](PT(&r)[LOADS], int z) {
        const LBM_GLOBAL PT *src = phin + (size_t)modi(z, nz) * plane;
#pragma unroll
        for (int k = 0; k < LOADS; k++) {
            const int e = tid + k * NTHREADS;
            r[k] = src[sxy[e < PLANE ? e : PLANE - 1]];  // spare lanes re-read the last point
        }
    };
    auto store_plane = [&](const PT(&r)[LOADS], int z) {
        float *dst = sphi[(z + 4) & 3];
#pragma unroll
        for (int k = 0; k < LOADS; k++) {
            const int e = tid + k * NTHREADS;
            if (e < PLANE) dst[e] = PS::f32(r[k]);
        }
    };
    const int lc = (ty + 1) * PX + (tx + 1);  // own phi tile index
    const uint32_t own_xy = (uint32_t)yg * nx + xg;
    // stencil, criterion and network of plane z (planes z-1 .. z+1 in the ring)
    auto compute = [&](int z) {
        const float *pm = sphi[(z + 3) & 3];
        const float *pc = sphi[z & 3];
        const float *pp = sphi[(z + 1) & 3];
        const float c0 = pc[lc];
        const bool cand = c0 > 0.02f && c0 < 0.98f;
        if (__ballot(cand) == 0ull) return;  // most waves hold no interface cell
        float ph[27];
        float y[4] = {0.f, 0.f, 0.f, 0.f};
        bool sel = false;
        if (cand) {
#pragma unroll
            for (int i = 0; i < 27; i++) {
                const float *pl = CZ(i) < 0 ? pm : (CZ(i) > 0 ? pp : pc);
                ph[i] = pl[lc + CY(i) * PX + CX(i)];
            }
            PhiGrad G;
            float kfd, gn;
            phi_stencil(ph, G);
            sel = mlp_select(G, P, kfd, gn);
        }
        mlp_wave(W, wave_lds[tid >> 6], sel, ph, y, tid & 63);
        if (cand) {
            const float nan = __builtin_nanf("");
            LBM_GLOBAL float *yo = yout + 4 * (size_t)((uint32_t)z * plane + own_xy);
            yo[0] = sel ? y[0] : nan;
            yo[1] = sel ? y[1] : nan;
            yo[2] = sel ? y[2] : nan;
            yo[3] = sel ? y[3] : nan;
        }
    };
    // plane z: plane z+1 into the ring (its slot held z-3, last read two
    // planes ago), plane z+4 into the freed register set, one barrier
    auto plane_step = [&](int z, PT(&r)[LOADS]) {
        store_plane(r, z + 1);
        fetch_plane(r, z + 4);
        lds_barrier();
        if (z < ze) compute(z);
    };
    fetch_plane(ra, zs - 1);
    store_plane(ra, zs - 1);
    fetch_plane(ra, zs);
    store_plane(ra, zs);
    // issued in this order (the compiler would otherwise reorder the three
    // sets, and the first wait of every pass through the loop would then
    // cover all of them)
    fetch_plane(ra, zs + 1);
    asm volatile("" ::: "memory");
    fetch_plane(rb, zs + 2);
    asm volatile("" ::: "memory");
    fetch_plane(rc, zs + 3);
    for (int z = zs; z < ze; z += 3) {
        plane_step(z, ra);
        plane_step(z + 1, rb);
        plane_step(z + 2, rc);
    }
}

// ------------------------------------------------------------ work queue
// The persistent loop of a batched launch over the boxes of a batch: a
// workgroup takes the next work item from one queue counter per launch, so the
// load stays balanced to the last item; item k belongs to the box b with
// first[b] <= k < first[b + 1].  The counter of this launch is counter[parity];
// the launch clears the other one for the next launch on the stream.
// body(b, item within the box) runs with every thread of the workgroup.
// (Per-die queues, each die draining a contiguous range of items first so that
// neighbouring tiles share its L2, cut the L2-miss reads by a fifth (FP32) to a
// third (FP16) but made the FP32 step 2.5 % slower and left FP16 unchanged: the
// step is not bound by the L2-miss traffic, and one queue keeps all dies on the
// same z range.)
template <int TW, class Body>
__device__ __forceinline__ void batch_loop(const uint32_t *__restrict__ first, int nbox, uint32_t *counter,
                                           int parity, Body body)
{
    __shared__ uint32_t s_item;
    const int tid = threadIdx.y * TW + threadIdx.x;
    const uint32_t total = first[nbox];
    if (blockIdx.x == 0 && tid == 0) counter[parity ^ 1] = 0u;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(&counter[parity], 1u);
        __syncthreads();
        const uint32_t item = (uint32_t)__builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();  // s_item read by all; the previous item's LDS traffic is over
        if (item >= total) break;
        int lo = 0, hi = nbox - 1;  // last box with first[b] <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (first[mid] <= item) lo = mid;
            else hi = mid - 1;
        }
        const int b = __builtin_amdgcn_readfirstlane(lo);
        body(b, item - first[b]);
    }
}

// One Runge-Kutta stage of the phase field of one or many boxes, on the same
// work items as the step (buf[b].phin: the stage input, buf[b].phin0: phi^n,
// buf[b].phout: the stage output).
template <int TW>
__global__ void __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(3)))
k_ac_stage_batch(const Params *__restrict__ tab, const Buffers *__restrict__ buf, const uint32_t *__restrict__ first,
                 int nbox, uint32_t *counter, int parity, double rk_a, double rk_b)
{
    batch_loop<TW>(first, nbox, counter, parity, [&](int b, uint32_t L) {
        step_tile<0, true, false, false, TW, true, false, true>(tab[b], buf[b], L, rk_a, rk_b);
    });
}

// The learned-curvature pass of one or many boxes ahead of their step, on the
// same work items (buf[b].phin: phi^n; buf[b].mlpy: the network outputs the
// step reads).
template <int TW, bool FX>
__global__ void __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(3)))
k_mlp_pass_batch(const Params *__restrict__ tab, const Buffers *__restrict__ buf, const uint32_t *__restrict__ first,
                 int nbox, uint32_t *counter, int parity)
{
    __shared__ MlpW w_lds;
    __shared__ MlpWave wave_lds[NTHREADS / 64];
    const void *loaded = nullptr;
    batch_loop<TW>(first, nbox, counter, parity, [&](int b, uint32_t L) {
        pass_tile<TW, FX>(tab[b], buf[b], L, w_lds, wave_lds, loaded);
    });
}

// The time step of one or many independent boxes in one launch (a single box
// is a batch of one); tab[b] and buf[b] are the box's parameters and this
// step's buffers.
template <int S, bool TP, bool FRC, bool ML, int TW, bool FX, bool PH>
__global__ void __launch_bounds__(NTHREADS) __attribute__((amdgpu_waves_per_eu(3)))
k_step_batch(const Params *__restrict__ tab, const Buffers *__restrict__ buf, const uint32_t *__restrict__ first,
             int nbox, uint32_t *counter, int parity)
{
    batch_loop<TW>(first, nbox, counter, parity, [&](int b, uint32_t L) {
        step_tile<S, TP, FRC, ML, TW, true, FX, false, PH>(tab[b], buf[b], L);
    });
}

// ------------------------------------------------------- step dispatch
// template dispatch: storage x two-phase x forcing x learned curvature
// (the learned curvature exists only with the phase field)
#define LBM_DISPATCH_S(S_, tp, frc, ml, CALL)                                  \
    do {                                                                       \
        if (tp) {                                                              \
            if (ml) { if (frc) CALL(S_, true, true, true) else CALL(S_, true, false, true) } \
            else { if (frc) CALL(S_, true, true, false) else CALL(S_, true, false, false) }  \
        } else {                                                               \
            if (frc) CALL(S_, false, true, false) else CALL(S_, false, false, false)        \
        }                                                                      \
    } while (0)
#define LBM_DISPATCH(storage, tp, frc, ml, CALL)                               \
    do {                                                                       \
        if (storage == 0) LBM_DISPATCH_S(0, tp, frc, ml, CALL);                \
        else if (storage == 1) LBM_DISPATCH_S(1, tp, frc, ml, CALL);           \
        else LBM_DISPATCH_S(2, tp, frc, ml, CALL);                             \
    } while (0)

// the step kernel also takes the phi storage and whether buoyancy or a
// viscosity contrast is compiled in (both exist only with the phase field)
#define LBM_STEP_CALL(S_, TP_, F_, M_)                                                               \
    {                                                                                                \
        if constexpr (TP_) {                                                                         \
            if (fix) {                                                                               \
                if (phys) STEP_CALL(S_, TP_, F_, M_, true, true) else STEP_CALL(S_, TP_, F_, M_, true, false) \
            } else {                                                                                 \
                if (phys) STEP_CALL(S_, TP_, F_, M_, false, true) else STEP_CALL(S_, TP_, F_, M_, false, false) \
            }                                                                                        \
        } else                                                                                       \
            STEP_CALL(S_, TP_, F_, M_, false, false)                                                 \
    }

// Occupancy-sized persistent grid and launch of the step kernel for one
// population storage S; each storage is instantiated in a translation unit
// of its own (lbm_step_s0/s1/s2.hip) so that the build compiles them in parallel.
template <int S>
int step_grid(bool tp, bool frc, bool ml, bool fix, bool phys, int tile)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
#define STEP_CALL(S_, TP_, F_, M_, X_, H_)                                                                         \
    {                                                                                                          \
        if (tile == 32)                                                                                        \
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step_batch<S_, TP_, F_, M_, 32, X_, H_>,  \
                                                               NTHREADS, 0);                                   \
        else                                                                                                   \
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step_batch<S_, TP_, F_, M_, 64, X_, H_>,  \
                                                               NTHREADS, 0);                                   \
    }
    LBM_DISPATCH_S(S, tp, frc, ml, LBM_STEP_CALL);
#undef STEP_CALL
    return per_cu * cus;
}

template <int S>
hipError_t step_launch(const Params *tab, const Buffers *buf, const uint32_t *first, int nbox, uint32_t *counter,
                       int parity, bool tp, bool frc, bool ml, bool fix, bool phys, int tile, int grid, hipStream_t s)
{
    dim3 g(grid), block(tile, NTHREADS / tile, 1);
#define STEP_CALL(S_, TP_, F_, M_, X_, H_)                                                                         \
    {                                                                                                          \
        if (tile == 32)                                                                                        \
            hipLaunchKernelGGL((k_step_batch<S_, TP_, F_, M_, 32, X_, H_>), g, block, 0, s, tab, buf, first, nbox,  \
                               counter, parity);                                                               \
        else                                                                                                   \
            hipLaunchKernelGGL((k_step_batch<S_, TP_, F_, M_, 64, X_, H_>), g, block, 0, s, tab, buf, first, nbox,  \
                               counter, parity);                                                               \
    }
    LBM_DISPATCH_S(S, tp, frc, ml, LBM_STEP_CALL);
#undef STEP_CALL
    return hipGetLastError();
}

}  // namespace lbm
