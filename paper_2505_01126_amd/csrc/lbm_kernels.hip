// Hand-written gfx950 kernels of one accLB time step (arXiv 2505.01126, Secs. 2-3).
//
// k_step fuses, per lattice site and time step:
//   pull-streaming of the 27 D3Q27 populations (SoA, one coalesced row per
//   direction), their moments, the phase-field stencils (LDS-staged phi tile),
//   the forces of Eq. (8), the regularised collision of Eqs. (6)-(7) rebuilt
//   from p*, u and a^(2) (each site writes only its own slots, Sec. 3), and the
//   conservative Allen-Cahn update of Eq. (3).
//
// Populations are stored as h_i = f_i / w_i - P0 in FP32, FP16 or BF16; all
// arithmetic is FP32.  Each phase-field flux through a face or lattice link is
// evaluated by the same contraction-free code from identical operands on both
// sides of the link, so the two sites see bit-identical values, and the fluxes
// are accumulated in FP64 into the FP64 phi: sum phi is conserved to FP64
// round-off.
#include <hip/hip_runtime.h>

#include "lbm_internal.h"

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
template <> struct Pop<0> {
    using T = float;
    __device__ static float dec(T v) { return v; }
    __device__ static T enc(float v) { return v; }
};
template <> struct Pop<1> {
    using T = _Float16;
    __device__ static float dec(T v) { return (float)v; }
    __device__ static T enc(float v) { return (T)v; }  // round to nearest even
};
template <> struct Pop<2> {
    using T = __bf16;
    __device__ static float dec(T v) { return (float)v; }
    __device__ static T enc(float v) { return (T)v; }  // round to nearest even
};

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// -------------------------------------------------------- per-site physics
struct Macro {
    float dp;     // p* - P0
    float rho;
    float u[3];   // u = j + a/2
    float a[3];   // F / rho
    float S[6];   // Pi - p* c_s^2 I  (xx yy zz xy xz yz)
};

// Moments of the deviation populations hw_i = f_i - w_i P0 (Sec. 2.2).
__device__ __forceinline__ void moments(const float (&hw)[27], float &dp, float (&j)[3], float (&S)[6])
{
    float p = 0.f, jx = 0.f, jy = 0.f, jz = 0.f, xx = 0.f, yy = 0.f, zz = 0.f, xy = 0.f, xz = 0.f, yz = 0.f;
#pragma unroll
    for (int i = 0; i < 27; i++) {
        const float v = hw[i];
        p += v;
        if (CX(i) > 0) jx += v; else if (CX(i) < 0) jx -= v;
        if (CY(i) > 0) jy += v; else if (CY(i) < 0) jy -= v;
        if (CZ(i) > 0) jz += v; else if (CZ(i) < 0) jz -= v;
        if (CX(i) != 0) xx += v;
        if (CY(i) != 0) yy += v;
        if (CZ(i) != 0) zz += v;
        if (CX(i) * CY(i) > 0) xy += v; else if (CX(i) * CY(i) < 0) xy -= v;
        if (CX(i) * CZ(i) > 0) xz += v; else if (CX(i) * CZ(i) < 0) xz -= v;
        if (CY(i) * CZ(i) > 0) yz += v; else if (CY(i) * CZ(i) < 0) yz -= v;
    }
    dp = p;
    j[0] = jx; j[1] = jy; j[2] = jz;
    const float pc = p * (1.0f / 3.0f);
    S[0] = xx - pc; S[1] = yy - pc; S[2] = zz - pc;
    S[3] = xy; S[4] = xz; S[5] = yz;
}

// Lattice gradient (1/c_s^2) sum w_i psi(x+c_i) c_i and Hessian
// (1/c_s^4) sum w_i psi(x+c_i) (c_i c_i - c_s^2 I) of a 27-point stencil (Sec. 2.3).
__device__ __forceinline__ void grad27(const float (&ph)[27], float (&g)[3])
{
    float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
    for (int i = 0; i < 27; i++) {
        const float v = 3.0f * WT(i) * ph[i];
        if (CX(i) > 0) gx += v; else if (CX(i) < 0) gx -= v;
        if (CY(i) > 0) gy += v; else if (CY(i) < 0) gy -= v;
        if (CZ(i) > 0) gz += v; else if (CZ(i) < 0) gz -= v;
    }
    g[0] = gx; g[1] = gy; g[2] = gz;
}

__device__ __forceinline__ void hess27(const float (&ph)[27], float (&H)[6])
{
    // H_aa = 9 sum_{c_a != 0} w psi - 3 sum w psi ; H_ab = 9 sum w psi c_a c_b
    float s0 = 0.f, sx = 0.f, sy = 0.f, sz = 0.f, xy = 0.f, xz = 0.f, yz = 0.f;
#pragma unroll
    for (int i = 0; i < 27; i++) {
        const float v = WT(i) * ph[i];
        s0 += v;
        if (CX(i) != 0) sx += v;
        if (CY(i) != 0) sy += v;
        if (CZ(i) != 0) sz += v;
        if (CX(i) * CY(i) > 0) xy += v; else if (CX(i) * CY(i) < 0) xy -= v;
        if (CX(i) * CZ(i) > 0) xz += v; else if (CX(i) * CZ(i) < 0) xz -= v;
        if (CY(i) * CZ(i) > 0) yz += v; else if (CY(i) * CZ(i) < 0) yz -= v;
    }
    H[0] = 9.0f * sx - 3.0f * s0;
    H[1] = 9.0f * sy - 3.0f * s0;
    H[2] = 9.0f * sz - 3.0f * s0;
    H[3] = 9.0f * xy; H[4] = 9.0f * xz; H[5] = 9.0f * yz;
}

// Forces of Eq. (8) and the velocity u = j + a/2 at one site.
//   F^s = -(3 delta/2) sigma K |g| g  with K |g| = tr H - g.H.g / |g|^2
//   F^p = -p* c_s^2 grad rho,  grad rho = (rho_l - rho_g) g
//   F^b = rho a_ext
//   F^nu = -(nu / (tau c_s^2)) (Pi - p* c_s^2 I - u0 u0) grad rho, u0 = j + (F^s + F^p + F^b)/(2 rho)
template <bool TP>
__device__ __forceinline__ void site_macro(const float (&hw)[27], const float (&ph)[27], const float (&aext)[3],
                                           const Params &P, Macro &m)
{
    float j[3];
    moments(hw, m.dp, j, m.S);
    if constexpr (TP) {
        const float phic = ph[13];
        const float rho = P.rho_g + (P.rho_l - P.rho_g) * phic;
        float g[3], H[6];
        grad27(ph, g);
        hess27(ph, H);
        const float g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
        float cs = 0.f;
        if (g2 > 1e-24f) {
            const float trH = H[0] + H[1] + H[2];
            const float gHg = g[0] * (H[0] * g[0] + H[3] * g[1] + H[4] * g[2]) +
                              g[1] * (H[3] * g[0] + H[1] * g[1] + H[5] * g[2]) +
                              g[2] * (H[4] * g[0] + H[5] * g[1] + H[2] * g[2]);
            cs = -P.fs_coef * (trH - gHg / g2);
        }
        const float drho = P.rho_l - P.rho_g;
        const float pstar = P.p0 + m.dp;
        const float cp = -pstar * (1.0f / 3.0f) * drho;  // F^p = cp * g
        const float inv_rho = 1.0f / rho;
        float F[3], u0[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            F[a] = (cs + cp) * g[a] + rho * aext[a];
            u0[a] = j[a] + 0.5f * F[a] * inv_rho;
        }
        // non-equilibrium stress at u0 contracted with grad rho
        const float n0 = m.S[0] - u0[0] * u0[0], n1 = m.S[1] - u0[1] * u0[1], n2 = m.S[2] - u0[2] * u0[2];
        const float n3 = m.S[3] - u0[0] * u0[1], n4 = m.S[4] - u0[0] * u0[2], n5 = m.S[5] - u0[1] * u0[2];
        const float cnu = -P.fnu_coef * drho;
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
    }
}

// Regularised post-collision h_i = f^post_i / w_i - P0 for all 27 directions,
// f^post = f^eq(p*, u) + (1 - omega) w H : a2 / (2 c_s^4) + S/2 with the
// closed form a2 = Pi - p* c_s^2 I - u u + (u a + a u)/2.  Each +-c pair shares
// its even part E and flips its odd part O.
__device__ __forceinline__ void collide(const Macro &m, float omega, float (&hout)[27])
{
    const float ux = m.u[0], uy = m.u[1], uz = m.u[2];
    const float ax = m.a[0], ay = m.a[1], az = m.a[2];
    const float k = 4.5f * (1.0f - omega);
    const float Axx = k * (m.S[0] - ux * ux + ux * ax);
    const float Ayy = k * (m.S[1] - uy * uy + uy * ay);
    const float Azz = k * (m.S[2] - uz * uz + uz * az);
    const float Axy = k * (m.S[3] - ux * uy + 0.5f * (ux * ay + ax * uy));
    const float Axz = k * (m.S[4] - ux * uz + 0.5f * (ux * az + ax * uz));
    const float Ayz = k * (m.S[5] - uy * uz + 0.5f * (uy * az + ay * uz));
    const float u2 = ux * ux + uy * uy + uz * uz;
    const float ua = ux * ax + uy * ay + uz * az;
    const float base = m.dp - 1.5f * (u2 + ua) - (Axx + Ayy + Azz) * (1.0f / 3.0f);
    hout[13] = base;
#pragma unroll
    for (int i = 14; i < 27; i++) {
        const int X = CX(i), Y = CY(i), Z = CZ(i);
        float cu = 0.f, ca = 0.f, ccA = 0.f;
        if (X) { cu += X * ux; ca += X * ax; ccA += Axx; }
        if (Y) { cu += Y * uy; ca += Y * ay; ccA += Ayy; }
        if (Z) { cu += Z * uz; ca += Z * az; ccA += Azz; }
        if (X * Y) ccA += 2.0f * X * Y * Axy;
        if (X * Z) ccA += 2.0f * X * Z * Axz;
        if (Y * Z) ccA += 2.0f * Y * Z * Ayz;
        const float E = base + 4.5f * cu * (cu + ca) + ccA;
        const float O = 3.0f * cu + 1.5f * ca;
        hout[i] = E + O;
        hout[26 - i] = E - O;
    }
}

// ----------------------------------------------------- phase-field fluxes
// WENO-5 (Jiang & Shu) value at the face right of cell c from the upwind-biased
// cells (a, b, c, d, e) = (c-2 .. c+2), linear weights (1/10, 6/10, 3/10),
// eps = 1e-6; written with one division.  Contraction-free so that both cells
// of a face compute the same bits.
__device__ __forceinline__ float weno5(float a, float b, float c, float d, float e)
{
#pragma clang fp contract(off)
    const float q0 = (2.0f * a - 7.0f * b + 11.0f * c) * (1.0f / 6.0f);
    const float q1 = (-b + 5.0f * c + 2.0f * d) * (1.0f / 6.0f);
    const float q2 = (2.0f * c + 5.0f * d - e) * (1.0f / 6.0f);
    const float t0 = a - 2.0f * b + c, r0 = a - 4.0f * b + 3.0f * c;
    const float t1 = b - 2.0f * c + d, r1 = b - d;
    const float t2 = c - 2.0f * d + e, r2 = 3.0f * c - 4.0f * d + e;
    float s0 = 1e-6f + ((13.0f / 12.0f) * (t0 * t0) + 0.25f * (r0 * r0));
    float s1 = 1e-6f + ((13.0f / 12.0f) * (t1 * t1) + 0.25f * (r1 * r1));
    float s2 = 1e-6f + ((13.0f / 12.0f) * (t2 * t2) + 0.25f * (r2 * r2));
    s0 = s0 * s0;
    s1 = s1 * s1;
    s2 = s2 * s2;
    // alpha_k = d_k / s_k, scaled by s0 s1 s2
    const float w0 = 0.1f * (s1 * s2), w1 = 0.6f * (s0 * s2), w2 = 0.3f * (s0 * s1);
    return (w0 * q0 + w1 * q1 + w2 * q2) / (w0 + w1 + w2);
}

// Advective flux through the face between cells l and l+1 along one axis:
// v[k] = phi at l-2+k (k = 0..5), ul / ur = velocity component at l / l+1.
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
// w_I [6 D (phi_a - phi_b) + 3 kappa (Q_a + Q_b) . c_I]
template <int I>
__device__ __forceinline__ float link_flux(float pa, float pb, const float *qa, const float *qb, float d6w, float k3w)
{
#pragma clang fp contract(off)
    float s = 0.0f;
    if constexpr (CX(I) > 0) s = s + (qa[0] + qb[0]);
    if constexpr (CX(I) < 0) s = s - (qa[0] + qb[0]);
    if constexpr (CY(I) > 0) s = s + (qa[1] + qb[1]);
    if constexpr (CY(I) < 0) s = s - (qa[1] + qb[1]);
    if constexpr (CZ(I) > 0) s = s + (qa[2] + qb[2]);
    if constexpr (CZ(I) < 0) s = s - (qa[2] + qb[2]);
    return d6w * (pa - pb) + k3w * s;
}

// Q = phi (1 - phi) n, n = g / |g| (zero where |g| <= 1e-12), from a 27-point
// stencil.  Neighbouring workgroups (and the prologue and body of one
// workgroup) evaluate Q at the same point from different inlined copies of
// this code, so it is contraction-free: every copy rounds identically.
__device__ __forceinline__ void q_of(const float (&ph)[27], float (&q)[3])
{
#pragma clang fp contract(off)
    float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
    for (int i = 0; i < 27; i++) {
        const float v = (3.0f * WT(i)) * ph[i];
        if (CX(i) > 0) gx = gx + v; else if (CX(i) < 0) gx = gx - v;
        if (CY(i) > 0) gy = gy + v; else if (CY(i) < 0) gy = gy - v;
        if (CZ(i) > 0) gz = gz + v; else if (CZ(i) < 0) gz = gz - v;
    }
    const float g2 = gx * gx + gy * gy + gz * gz;
    const float c = ph[13] * (1.0f - ph[13]);
    const float s = g2 > 1e-24f ? c * __frsqrt_rn(g2) : 0.0f;
    q[0] = s * gx;
    q[1] = s * gy;
    q[2] = s * gz;
}

// ----------------------------------------------------------------- forcing
// Column sums C_k(x, y) = sum_{rows with kz = k} A e^{2 pi i (kx x/nx + ky y/ny)}
// for k = -2..2; per plane a(x) = sum_k Re(C_k e^{2 pi i k z / nz}).
struct Forcing {
    float cr[5][3], ci[5][3];
};

__device__ __forceinline__ void forcing_column(const ModeTable *mt, int n, int x, int y, int nx, int ny, Forcing &F)
{
#pragma unroll
    for (int k = 0; k < 5; k++)
#pragma unroll
        for (int a = 0; a < 3; a++) F.cr[k][a] = F.ci[k][a] = 0.f;
    for (int m = 0; m < n; m++) {
        const int kx = mt->kx[m], ky = mt->ky[m], kz = mt->kz[m];
        int fx = (kx * x) % nx;
        if (fx < 0) fx += nx;
        int fy = (ky * y) % ny;
        if (fy < 0) fy += ny;
        const float t = 2.0f * ((float)fx / (float)nx + (float)fy / (float)ny);
        float sn, cs;
        sincospif(t, &sn, &cs);
#pragma unroll
        for (int k = 0; k < 5; k++) {
            if (kz == k - 2) {
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    const float ar = mt->re[m][a], ai = mt->im[m][a];
                    F.cr[k][a] += ar * cs - ai * sn;
                    F.ci[k][a] += ar * sn + ai * cs;
                }
            }
        }
    }
}

__device__ __forceinline__ void forcing_at(const Forcing &F, int z, int nz, float (&a)[3])
{
    float s1, c1;
    sincospif(2.0f * (float)z / (float)nz, &s1, &c1);
    const float c2 = c1 * c1 - s1 * s1, s2 = 2.0f * s1 * c1;
    const float tr[5] = {c2, c1, 1.0f, c1, c2};
    const float ti[5] = {-s2, -s1, 0.0f, s1, s2};
#pragma unroll
    for (int d = 0; d < 3; d++) {
        float v = 0.f;
#pragma unroll
        for (int k = 0; k < 5; k++) v += F.cr[k][d] * tr[k] - F.ci[k][d] * ti[k];
        a[d] = v;
    }
}

// ------------------------------------------------------------ fused step
constexpr int HX = 3, HY = 3;                 // phi tile halo (WENO-5 needs 3)
constexpr int PX = TX + 2 * HX, PY = TY + 2 * HY;
constexpr int PLANE = PX * PY;                 // phi values per staged plane
constexpr int QX = TX + 2, QY = TY + 2;        // Q tile (halo 1)
constexpr int QPLANE = QX * QY;
constexpr int NRING = 8;                       // phi planes z-3 .. z+4 (power of two)
constexpr int LOADS = (PLANE + NTHREADS - 1) / NTHREADS;
constexpr int QPTS = (QPLANE + NTHREADS - 1) / NTHREADS;

template <int S, bool TP, bool FRC>
__global__ void __launch_bounds__(NTHREADS) k_step(Params P, Buffers B)
{
    using T = typename Pop<S>::T;
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t N = plane * (uint32_t)nz;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * P.zchunk;
    const int zend = min(z0 + P.zchunk, nz);
    const int xg = (x0 + tx) % nx, yg = (y0 + ty) % ny;
    const bool active = (x0 + tx < nx) && (y0 + ty < ny);
    const T *__restrict__ fin = (const T *)B.fin;
    T *__restrict__ fout = (T *)B.fout;

    // pull sources in the xy plane: index (cy+1)*3 + (cx+1) -> (x - cx, y - cy)
    uint32_t src_xy[9];
#pragma unroll
    for (int dy = -1; dy <= 1; dy++)
#pragma unroll
        for (int dx = -1; dx <= 1; dx++)
            src_xy[(dy + 1) * 3 + dx + 1] = (uint32_t)wrapi(yg - dy, ny) * nx + (uint32_t)wrapi(xg - dx, nx);
    const uint32_t own_xy = (uint32_t)yg * nx + xg;

    Forcing frc;
    if constexpr (FRC) forcing_column(P.modes, P.n_modes, xg, yg, nx, ny, frc);

    // LDS: phi ring (FP32) and Q planes z-1, z, z+1
    __shared__ float sphi[TP ? NRING : 1][TP ? PLANE : 1];
    __shared__ float sq[TP ? 3 : 1][3][TP ? QPLANE : 1];
    uint32_t ld_xy[LOADS];
    int q_lds[QPTS];

    if constexpr (TP) {
#pragma unroll
        for (int k = 0; k < LOADS; k++) {
            const int e = tid + k * NTHREADS;
            const int ly = e / PX, lx = e - ly * PX;
            ld_xy[k] = (uint32_t)(((y0 + ly - HY) % ny + ny) % ny) * nx + (uint32_t)(((x0 + lx - HX) % nx + nx) % nx);
        }
#pragma unroll
        for (int k = 0; k < QPTS; k++) {
            const int p = tid + k * NTHREADS;
            const int qy = p / QX, qx = p - qy * QX;
            q_lds[k] = (qy + 2) * PX + (qx + 2);  // phi tile centre of Q point (qx, qy)
        }
    }

    auto load_plane = [&](int z) {
        const int zw = ((z % nz) + nz) % nz;
        const double *src = B.phin + (size_t)zw * plane;
        float *dst = sphi[(z + NRING) & (NRING - 1)];
#pragma unroll
        for (int k = 0; k < LOADS; k++) {
            const int e = tid + k * NTHREADS;
            if (e < PLANE) dst[e] = (float)src[ld_xy[k]];
        }
    };
    auto compute_q = [&](int z) {
        const float *p0 = sphi[(z - 1 + NRING) & (NRING - 1)];
        const float *p1 = sphi[(z + NRING) & (NRING - 1)];
        const float *p2 = sphi[(z + 1 + NRING) & (NRING - 1)];
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
                sq[slot][0][p] = q[0];
                sq[slot][1][p] = q[1];
                sq[slot][2][p] = q[2];
            }
        }
    };

    float uz_m = 0.f, uz_c = 0.f;  // u_z at (x, y, z-1) and (x, y, z) for the z faces
    if constexpr (TP) {
        for (int z = z0 - 3; z <= z0 + 2; z++) load_plane(z);
        __syncthreads();
        compute_q(z0 - 1);
        compute_q(z0);
        const uint32_t zm = (uint32_t)wrapi(z0 - 1, nz);
        uz_m = B.uin[2 * (size_t)N + zm * plane + own_xy];
        uz_c = B.uin[2 * (size_t)N + (uint32_t)z0 * plane + own_xy];
    }

    const int lc = (ty + HY) * PX + (tx + HX);     // own phi tile index
    const int qc = (ty + 1) * QX + (tx + 1);       // own Q tile index

    for (int z = z0; z < zend; z++) {
        if constexpr (TP) {
            load_plane(z + 3);
            __syncthreads();
            compute_q(z + 1);
            __syncthreads();
        }
        if (!active) continue;

        const uint32_t zc = (uint32_t)z * plane;
        const uint32_t zsrc[3] = {(uint32_t)wrapi(z + 1, nz) * plane, zc, (uint32_t)wrapi(z - 1, nz) * plane};
        const uint32_t own = zc + own_xy;

        // 1. pull-stream: f_i(x) = f^post_i(x - c_i)
        float hw[27];
#pragma unroll
        for (int i = 0; i < 27; i++) {
            const uint32_t s = zsrc[CZ(i) + 1] + src_xy[(CY(i) + 1) * 3 + CX(i) + 1];
            hw[i] = WT(i) * Pop<S>::dec(fin[(size_t)i * N + s]);
        }

        // 2. phase-field stencil of this site
        float ph[27];
        if constexpr (TP) {
            const float *pm = sphi[(z - 1 + NRING) & (NRING - 1)];
            const float *pc = sphi[(z + NRING) & (NRING - 1)];
            const float *pp = sphi[(z + 1 + NRING) & (NRING - 1)];
#pragma unroll
            for (int i = 0; i < 27; i++) {
                const float *pl = CZ(i) < 0 ? pm : (CZ(i) > 0 ? pp : pc);
                ph[i] = pl[lc + CY(i) * PX + CX(i)];
            }
        } else {
#pragma unroll
            for (int i = 0; i < 27; i++) ph[i] = 0.f;
        }

        float aext[3] = {0.f, 0.f, 0.f};
        if constexpr (FRC) forcing_at(frc, z, nz, aext);

        // 3. moments, forces, velocity
        Macro m;
        site_macro<TP>(hw, ph, aext, P, m);

        // 4. regularised collision, written to this site's own slots
        float h[27];
        collide(m, P.omega, h);
#pragma unroll
        for (int i = 0; i < 27; i++) fout[(size_t)i * N + own] = Pop<S>::enc(h[i]);

        if constexpr (TP) {
            // 5. Allen-Cahn: phi^{n+1} = phi^n - sum (outgoing - incoming) face and link fluxes
            const float *pc = sphi[(z + NRING) & (NRING - 1)];
            double acc = 0.0;
            // convective faces; x
            {
                const float *r = pc + lc;
                const float ul = B.uin[zc + (uint32_t)yg * nx + wrapi(xg - 1, nx)];
                const float uc = B.uin[own];
                const float ur = B.uin[zc + (uint32_t)yg * nx + wrapi(xg + 1, nx)];
                const float jr = face_flux(r[-2], r[-1], r[0], r[1], r[2], r[3], uc, ur);
                const float jl = face_flux(r[-3], r[-2], r[-1], r[0], r[1], r[2], ul, uc);
                acc += (double)jl - (double)jr;
            }
            {  // y
                const float *r = pc + lc;
                const float *uy = B.uin + N;
                const float ul = uy[zc + (uint32_t)wrapi(yg - 1, ny) * nx + xg];
                const float uc = uy[own];
                const float ur = uy[zc + (uint32_t)wrapi(yg + 1, ny) * nx + xg];
                const float jr = face_flux(r[-2 * PX], r[-PX], r[0], r[PX], r[2 * PX], r[3 * PX], uc, ur);
                const float jl = face_flux(r[-3 * PX], r[-2 * PX], r[-PX], r[0], r[PX], r[2 * PX], ul, uc);
                acc += (double)jl - (double)jr;
            }
            {  // z
                float v[7];
#pragma unroll
                for (int k = 0; k < 7; k++) v[k] = sphi[(z - 3 + k + NRING) & (NRING - 1)][lc];
                const uint32_t zp = (uint32_t)wrapi(z + 1, nz) * plane;
                const float up = B.uin[2 * (size_t)N + zp + own_xy];
                const float jr = face_flux(v[1], v[2], v[3], v[4], v[5], v[6], uz_c, up);
                const float jl = face_flux(v[0], v[1], v[2], v[3], v[4], v[5], uz_m, uz_c);
                acc += (double)jl - (double)jr;
                uz_m = uz_c;
                uz_c = up;
            }
            // diffusion + sharpening through the 13 canonical links, both directions
            {
                const float *q0 = sq[(z - 1 + 3) % 3][0];
                const float *q1 = sq[(z + 3) % 3][0];
                const float *q2 = sq[(z + 1 + 3) % 3][0];
                float qs[27][3];
#pragma unroll
                for (int i = 0; i < 27; i++) {
                    const float *ql = CZ(i) < 0 ? q0 : (CZ(i) > 0 ? q2 : q1);
                    const int o = qc + CY(i) * QX + CX(i);
                    qs[i][0] = ql[o];
                    qs[i][1] = ql[o + QPLANE];
                    qs[i][2] = ql[o + 2 * QPLANE];
                }
                const float d6w[4] = {0.f, P.d6 * WT(14), P.d6 * WT(15), P.d6 * WT(26)};
                const float k3w[4] = {0.f, P.k3 * WT(14), P.k3 * WT(15), P.k3 * WT(26)};
#define LB_LINK(I)                                                                                     \
    {                                                                                                  \
        const float fo = link_flux<I>(ph[13], ph[I], qs[13], qs[I], d6w[C2(I)], k3w[C2(I)]);          \
        const float fi = link_flux<I>(ph[26 - I], ph[13], qs[26 - I], qs[13], d6w[C2(I)], k3w[C2(I)]); \
        acc += (double)fi - (double)fo;                                                                \
    }
                LB_LINK(14) LB_LINK(15) LB_LINK(16) LB_LINK(17) LB_LINK(18) LB_LINK(19) LB_LINK(20)
                LB_LINK(21) LB_LINK(22) LB_LINK(23) LB_LINK(24) LB_LINK(25) LB_LINK(26)
#undef LB_LINK
            }
            B.phout[own] = B.phin[own] + acc;
        }
        if constexpr (TP) {  // velocity of this step, advects phi in the next one
            B.uout[own] = m.u[0];
            B.uout[(size_t)N + own] = m.u[1];
            B.uout[2 * (size_t)N + own] = m.u[2];
        }
    }
}

// ----------------------------------------------------------- initial state
// f^0 = f^eq(p*0, u0) + w H : A0 / (2 c_s^4), A0 = -c_s^2 tau (grad u0 + grad u0^T),
// written pre-shifted (slot of x - c_i) so that the first pull yields f^0 at x.
template <int S>
__global__ void __launch_bounds__(NTHREADS) k_init(Params P, void *fout_, double *phi_out, float *u_out,
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
    const double tau = 1.0 / (double)P.omega;
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
        fout[(size_t)i * N + nb(-CX(i), -CY(i), -CZ(i))] = Pop<S>::enc((float)h);
    }
    if (phi_out) phi_out[s] = P.two_phase ? phi0[s] : 0.0;
    if (u_out)
        for (int a = 0; a < 3; a++) u_out[(size_t)a * N + s] = (float)u[a];
}

// -------------------------------------------------- fields and reductions
// Per-site macroscopic state at time n (pull + stencils from global memory).
template <int S, bool TP, bool FRC>
__device__ __forceinline__ void site_state(const Params &P, const void *fin_, const double *phi, uint32_t s,
                                           Macro &m, float &phic)
{
    using T = typename Pop<S>::T;
    const T *fin = (const T *)fin_;
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const uint32_t plane = (uint32_t)nx * ny, N = plane * (uint32_t)nz;
    const int x = s % nx, y = (s / nx) % ny, z = s / plane;
    auto nb = [&](int dx, int dy, int dz) {
        return (uint32_t)wrapi(z + dz, nz) * plane + (uint32_t)wrapi(y + dy, ny) * nx + (uint32_t)wrapi(x + dx, nx);
    };
    float hw[27], ph[27];
#pragma unroll
    for (int i = 0; i < 27; i++) hw[i] = WT(i) * Pop<S>::dec(fin[(size_t)i * N + nb(-CX(i), -CY(i), -CZ(i))]);
    if constexpr (TP) {
#pragma unroll
        for (int i = 0; i < 27; i++) ph[i] = (float)phi[nb(CX(i), CY(i), CZ(i))];
    } else {
#pragma unroll
        for (int i = 0; i < 27; i++) ph[i] = 0.f;
    }
    float aext[3] = {0.f, 0.f, 0.f};
    if constexpr (FRC) {
        Forcing F;
        forcing_column(P.modes, P.n_modes, x, y, nx, ny, F);
        forcing_at(F, z, nz, aext);
    }
    site_macro<TP>(hw, ph, aext, P, m);
    phic = TP ? (float)phi[s] : 0.f;
}

template <int S, bool TP, bool FRC>
__global__ void __launch_bounds__(NTHREADS) k_moments(Params P, const void *fin, const double *phi, float *rho,
                                                      float *pr, float *u, double *phi_out)
{
    const uint32_t N = (uint32_t)P.nx * P.ny * P.nz;
    const uint32_t s = blockIdx.x * NTHREADS + threadIdx.x;
    if (s >= N) return;
    Macro m;
    float phic;
    site_state<S, TP, FRC>(P, fin, phi, s, m, phic);
    if (rho) rho[s] = m.rho;
    if (pr) pr[s] = (P.p0 + m.dp) * m.rho * (1.0f / 3.0f);
    if (u) {
        u[s] = m.u[0];
        u[(size_t)N + s] = m.u[1];
        u[2 * (size_t)N + s] = m.u[2];
    }
    if (phi_out) phi_out[s] = TP ? phi[s] : 0.0;
}

// FP64 partial sums per block over a fixed grid-stride partition, combined in
// a fixed order: the result does not depend on scheduling.
template <int S, bool TP, bool FRC>
__global__ void __launch_bounds__(NTHREADS) k_reduce(Params P, const void *fin, const double *phi, double *partials)
{
    const uint32_t N = (uint32_t)P.nx * P.ny * P.nz;
    double acc[NRED];
#pragma unroll
    for (int k = 0; k < NRED; k++) acc[k] = 0.0;
    for (uint32_t s = blockIdx.x * NTHREADS + threadIdx.x; s < N; s += gridDim.x * NTHREADS) {
        Macro m;
        float phic_f;
        site_state<S, TP, FRC>(P, fin, phi, s, m, phic_f);
        const double ph = TP ? phi[s] : 0.0;
        const double r = m.rho, pstar = (double)P.p0 + (double)m.dp;
        const double ux = m.u[0], uy = m.u[1], uz = m.u[2];
        const bool bad = !isfinite(pstar) || !isfinite(ux) || !isfinite(uy) || !isfinite(uz) || !isfinite(ph);
        if (bad) {
            acc[9] += 1.0;
            continue;
        }
        const double u2 = ux * ux + uy * uy + uz * uz;
        acc[0] += ph;
        acc[1] += r;
        acc[2] += pstar;
        acc[3] += r * ux;
        acc[4] += r * uy;
        acc[5] += r * uz;
        acc[6] += 0.5 * r * u2;
        acc[7] = fmax(acc[7], sqrt(u2));
        acc[8] = TP ? fmax(acc[8], fmax(ph - 1.0, fmax(-ph, 0.0))) : 0.0;
    }
    __shared__ double red[NRED][NTHREADS];
#pragma unroll
    for (int k = 0; k < NRED; k++) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = NTHREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int k = 0; k < NRED; k++) {
                const double o = red[k][threadIdx.x + w];
                red[k][threadIdx.x] = (k == 7 || k == 8) ? fmax(red[k][threadIdx.x], o) : red[k][threadIdx.x] + o;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < NRED) partials[(size_t)blockIdx.x * NRED + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(NTHREADS) k_reduce_final(const double *partials, int nblocks, double *out)
{
    __shared__ double red[NRED][NTHREADS];
    double acc[NRED];
#pragma unroll
    for (int k = 0; k < NRED; k++) acc[k] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += NTHREADS)
#pragma unroll
        for (int k = 0; k < NRED; k++) {
            const double v = partials[(size_t)b * NRED + k];
            acc[k] = (k == 7 || k == 8) ? fmax(acc[k], v) : acc[k] + v;
        }
#pragma unroll
    for (int k = 0; k < NRED; k++) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = NTHREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int k = 0; k < NRED; k++) {
                const double o = red[k][threadIdx.x + w];
                red[k][threadIdx.x] = (k == 7 || k == 8) ? fmax(red[k][threadIdx.x], o) : red[k][threadIdx.x] + o;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < NRED) out[threadIdx.x] = red[threadIdx.x][0];
}

// --------------------------------------------------------------- launchers
#define LBM_DISPATCH(storage, tp, frc, CALL)                      \
    do {                                                          \
        if (storage == 0) {                                       \
            if (tp) { if (frc) CALL(0, true, true) else CALL(0, true, false) }   \
            else { if (frc) CALL(0, false, true) else CALL(0, false, false) }    \
        } else if (storage == 1) {                                \
            if (tp) { if (frc) CALL(1, true, true) else CALL(1, true, false) }   \
            else { if (frc) CALL(1, false, true) else CALL(1, false, false) }    \
        } else {                                                  \
            if (tp) { if (frc) CALL(2, true, true) else CALL(2, true, false) }   \
            else { if (frc) CALL(2, false, true) else CALL(2, false, false) }    \
        }                                                         \
    } while (0)

hipError_t launch_step(const Params &p, int storage, const Buffers &b, hipStream_t s)
{
    dim3 grid((p.nx + TX - 1) / TX, (p.ny + TY - 1) / TY, (p.nz + p.zchunk - 1) / p.zchunk);
    dim3 block(TX, TY, 1);
    const bool tp = p.two_phase != 0, frc = p.n_modes > 0;
#define CALL(S_, TP_, F_) hipLaunchKernelGGL((k_step<S_, TP_, F_>), grid, block, 0, s, p, b);
    LBM_DISPATCH(storage, tp, frc, CALL);
#undef CALL
    return hipGetLastError();
}

hipError_t launch_init(const Params &p, int storage, void *fout, double *phi_out, float *u_out, const double *phi0,
                       const double *u0, const double *ps0, hipStream_t s)
{
    const uint32_t N = (uint32_t)p.nx * p.ny * p.nz;
    dim3 grid((N + NTHREADS - 1) / NTHREADS), block(NTHREADS);
    if (storage == 0) hipLaunchKernelGGL(k_init<0>, grid, block, 0, s, p, fout, phi_out, u_out, phi0, u0, ps0);
    else if (storage == 1) hipLaunchKernelGGL(k_init<1>, grid, block, 0, s, p, fout, phi_out, u_out, phi0, u0, ps0);
    else hipLaunchKernelGGL(k_init<2>, grid, block, 0, s, p, fout, phi_out, u_out, phi0, u0, ps0);
    return hipGetLastError();
}

hipError_t launch_moments(const Params &p, int storage, const void *fin, const double *phi, float *rho, float *pr,
                          float *u, double *phi_out, hipStream_t s)
{
    const uint32_t N = (uint32_t)p.nx * p.ny * p.nz;
    dim3 grid((N + NTHREADS - 1) / NTHREADS), block(NTHREADS);
    const bool tp = p.two_phase != 0, frc = p.n_modes > 0;
#define CALL(S_, TP_, F_) \
    hipLaunchKernelGGL((k_moments<S_, TP_, F_>), grid, block, 0, s, p, fin, phi, rho, pr, u, phi_out);
    LBM_DISPATCH(storage, tp, frc, CALL);
#undef CALL
    return hipGetLastError();
}

hipError_t launch_reduce(const Params &p, int storage, const void *fin, const double *phi, double *partials,
                         double *out, hipStream_t s)
{
    dim3 grid(RED_BLOCKS), block(NTHREADS);
    const bool tp = p.two_phase != 0, frc = p.n_modes > 0;
#define CALL(S_, TP_, F_) hipLaunchKernelGGL((k_reduce<S_, TP_, F_>), grid, block, 0, s, p, fin, phi, partials);
    LBM_DISPATCH(storage, tp, frc, CALL);
#undef CALL
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_final, dim3(1), block, 0, s, partials, (int)RED_BLOCKS, out);
    return hipGetLastError();
}

}  // namespace lbm
