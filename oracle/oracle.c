/*
 * FP64 CPU oracle of the accLB lattice update (arXiv 2505.01126, Sec. 2).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the GPU product path.  It is a plain,
 * slow transcription of the method in the paper's own order and notation:
 *
 *   per site, from the populations f_i and the phase field phi at time n
 *     moments         p* = sum f_i, j = sum f_i c_i                      (Sec. 2.2)
 *     forces          F = F^s + F^p + F^nu (+ body force)                (Sec. 2.3, Eq. 8)
 *     velocity        u = j + a/2, a = F / rho                           (Sec. 2.2)
 *     non-equilibrium f^neq = f - f^eq + S/2, a^(2) = sum f^neq H^(2)    (Eqs. 6-7)
 *     regularised     f^post = f^eq + (1 - omega) w H:a^(2)/(2 c_s^4) + S/2
 *     streaming       f_i(x + c_i, n + 1) = f^post_i(x, n)               (Eq. 4)
 *   and the Allen-Cahn update of phi (Eq. 3) with WENO-5 convection and the
 *   lattice stencils of Sec. 2.3 for diffusion and sharpening.
 *
 * Readings where the printed text is ambiguous (each one is listed in the
 * design notes of the repository):
 *   - equilibrium tanh profile: 1/2 (1 + tanh(2 d / delta)) with Euclidean d;
 *   - regularised f^neq carries the weight and the Hermite tensor, w_i H_i : a2 / (2 c_s^4);
 *   - velocity u = sum f c + (1/2) sum S c, i.e. j + a/2;
 *   - Guo term driven by the acceleration F / rho (pressure-based scheme);
 *   - F^s = -(3 delta / 2) sigma K |grad phi| grad phi, K = div(n), n toward phi = 1;
 *   - F^nu contracts the non-equilibrium stress with d_beta rho, evaluated with
 *     f^eq at the velocity u0 that holds every force except F^nu;
 *   - Laplacian (2/c_s^2) sum w_i (psi(x+c_i) - psi(x)), Hessian (1/c_s^4) sum w_i psi(x+c_i) H_i;
 *   - Allen-Cahn convection in flux form div(u phi), explicit Euler with the
 *     velocity of the previous step, one update per LB step.
 *
 * Pins (tests/test_oracle_*.py): lattice identities, equilibrium and Guo
 * moments, collision invariants and the closed-form a^(2), stencil exactness
 * on polynomials, WENO-5 order, the steady tanh profile and its translation,
 * Taylor-Green and ABC decay, conservation, Laplace's law, fp16 rounding, the
 * network's identity reduction and its gradient against finite differences;
 * the initial non-equilibrium part against the shear-wave closed form; every
 * branch of the learned-curvature blend against a constant-output network;
 * the viscous correction F^nu and the phase-dependent relaxation time through
 * the steady layered flow of a variable-property momentum equation.  Several
 * of these tests compile a copy of this file with a planted mistake and show
 * that the pin catches it.  The one-step lag of the Allen-Cahn velocity (a
 * reading of the time integration) is pinned by a slab pushed from rest: the
 * push reaches phi one step after the velocity that carries it.
 */
#include "oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q ORC_Q
static const double CS2 = 1.0 / 3.0;

/* ---------------------------------------------------------------- lattice */

static int CI[Q][3];
static double WI[Q];
static double HT[Q][3][3];
static int lattice_ready = 0;

static void lattice_init(void)
{
    if (lattice_ready)
        return;
    for (int i = 0; i < Q; i++) {
        CI[i][0] = i % 3 - 1;
        CI[i][1] = (i / 3) % 3 - 1;
        CI[i][2] = i / 9 - 1;
        int n2 = CI[i][0] * CI[i][0] + CI[i][1] * CI[i][1] + CI[i][2] * CI[i][2];
        WI[i] = n2 == 0 ? 8.0 / 27.0 : n2 == 1 ? 2.0 / 27.0 : n2 == 2 ? 1.0 / 54.0 : 1.0 / 216.0;
    }
    for (int i = 0; i < Q; i++)
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++)
                HT[i][a][b] = CI[i][a] * CI[i][b] - (a == b ? CS2 : 0.0);
    lattice_ready = 1;
}

void orc_lattice(int *c, double *w)
{
    lattice_init();
    for (int i = 0; i < Q; i++) {
        for (int a = 0; a < 3; a++)
            c[3 * i + a] = CI[i][a];
        w[i] = WI[i];
    }
}

static inline long wrap(long v, long n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

static inline long site(int nx, int ny, long x, long y, long z)
{
    return (z * ny + y) * nx + x;
}

/* index of the site at x + (dx, dy, dz), periodic */
static inline long nbr(int nx, int ny, int nz, long x, long y, long z, int dx, int dy, int dz)
{
    return site(nx, ny, wrap(x + dx, nx), wrap(y + dy, ny), wrap(z + dz, nz));
}

/* Hermite tensor H_i,ab = c_ia c_ib - c_s^2 delta_ab (tabulated by lattice_init) */
static inline double herm(int i, int a, int b)
{
    return HT[i][a][b];
}

/* --------------------------------------------------- single-site pieces */

/* pressure-based equilibrium (Sec. 2.2):
 * f^eq_i = w_i ( p* + c.u / c_s^2 + (c c - c_s^2 I) : u u / (2 c_s^4) ) */
void orc_feq(double pstar, const double u[3], double out[Q])
{
    lattice_init();
    for (int i = 0; i < Q; i++) {
        double cu = 0.0, quad = 0.0;
        for (int a = 0; a < 3; a++)
            cu += CI[i][a] * u[a];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++)
                quad += herm(i, a, b) * u[a] * u[b];
        out[i] = WI[i] * (pstar + cu / CS2 + quad / (2.0 * CS2 * CS2));
    }
}

/* Guo forcing (Eq. 5) driven by the acceleration acc = F / rho:
 * S_i = w_i ( (c_i - u)/c_s^2 + (c_i . u) c_i / c_s^4 ) . acc */
void orc_guo(const double u[3], const double acc[3], double out[Q])
{
    lattice_init();
    for (int i = 0; i < Q; i++) {
        double cu = 0.0;
        for (int a = 0; a < 3; a++)
            cu += CI[i][a] * u[a];
        double s = 0.0;
        for (int a = 0; a < 3; a++)
            s += ((CI[i][a] - u[a]) / CS2 + cu * CI[i][a] / (CS2 * CS2)) * acc[a];
        out[i] = WI[i] * s;
    }
}

static const int PAIR[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};

/* Regularised collision in the form of Eq. (6) with the Hermite projection of Eq. (7). */
void orc_collide(const double f[Q], const double u[3], const double acc[3], double tau,
                 double fpost[Q], double a2[6])
{
    lattice_init();
    double pstar = 0.0;
    for (int i = 0; i < Q; i++)
        pstar += f[i];
    double feq[Q], S[Q], fneq[Q];
    orc_feq(pstar, u, feq);
    orc_guo(u, acc, S);
    for (int i = 0; i < Q; i++)
        fneq[i] = f[i] - feq[i] + 0.5 * S[i];
    /* a^(2)_ab = sum_i f^neq_i H_i,ab  (Eq. 7) */
    double A[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double s = 0.0;
            for (int i = 0; i < Q; i++)
                s += fneq[i] * herm(i, a, b);
            A[a][b] = s;
        }
    double omega = 1.0 / tau;
    for (int i = 0; i < Q; i++) {
        double hA = 0.0;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++)
                hA += herm(i, a, b) * A[a][b];
        double freg = WI[i] * hA / (2.0 * CS2 * CS2);
        fpost[i] = feq[i] + (1.0 - omega) * freg + 0.5 * S[i];
    }
    if (a2)
        for (int k = 0; k < 6; k++)
            a2[k] = A[PAIR[k][0]][PAIR[k][1]];
}

/* ------------------------------------------------------------- stencils */

/* nb[i] = index of x + c_i (periodic) for the 27 lattice directions */
static void neighbours(int nx, int ny, int nz, long x, long y, long z, long nb[Q])
{
    for (int i = 0; i < Q; i++)
        nb[i] = nbr(nx, ny, nz, x, y, z, CI[i][0], CI[i][1], CI[i][2]);
}

static void grad_nb(const double *psi, const long nb[Q], double g[3])
{
    g[0] = g[1] = g[2] = 0.0;
    for (int i = 0; i < Q; i++) {
        double v = psi[nb[i]];
        for (int a = 0; a < 3; a++)
            g[a] += WI[i] * v * CI[i][a];
    }
    for (int a = 0; a < 3; a++)
        g[a] /= CS2;
}

static void hess_nb(const double *psi, const long nb[Q], double H[3][3])
{
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
            H[a][b] = 0.0;
    for (int i = 0; i < Q; i++) {
        double v = psi[nb[i]];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++)
                H[a][b] += WI[i] * v * herm(i, a, b);
    }
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
            H[a][b] /= CS2 * CS2;
}

/* d_a psi = (1/c_s^2) sum_i w_i psi(x + c_i) c_ia   (Sec. 2.3) */
static void grad_at(int nx, int ny, int nz, const double *psi, long x, long y, long z, double g[3])
{
    long nb[Q];
    neighbours(nx, ny, nz, x, y, z, nb);
    grad_nb(psi, nb, g);
}

/* d_a d_b psi = (1/c_s^4) sum_i w_i psi(x + c_i) H_i,ab  (Hessian; exact on cubics) */
static void hess_at(int nx, int ny, int nz, const double *psi, long x, long y, long z, double H[3][3])
{
    long nb[Q];
    neighbours(nx, ny, nz, x, y, z, nb);
    hess_nb(psi, nb, H);
}

/* laplacian (2/c_s^2) sum_{i != 0} w_i (psi(x + c_i) - psi(x)) */
static double lap_at(int nx, int ny, int nz, const double *psi, long x, long y, long z)
{
    double c = psi[site(nx, ny, x, y, z)];
    double s = 0.0;
    for (int i = 0; i < Q; i++) {
        if (i == 13)
            continue;
        s += WI[i] * (psi[nbr(nx, ny, nz, x, y, z, CI[i][0], CI[i][1], CI[i][2])] - c);
    }
    return 2.0 * s / CS2;
}

/* Loops over the sites of boxes below this size run on one thread: the
   thread start-up of each parallel loop would cost more than the loop. */
#define ORC_PAR_MIN 32768L
static int orc_par(long n) { return n >= ORC_PAR_MIN; }

void orc_gradient(int nx, int ny, int nz, const double *psi, double *grad)
{
    lattice_init();
    long N = (long)nx * ny * nz;
#pragma omp parallel for if (orc_par((long)nx * ny * nz))
    for (long z = 0; z < nz; z++)
        for (long y = 0; y < ny; y++)
            for (long x = 0; x < nx; x++) {
                double g[3];
                grad_at(nx, ny, nz, psi, x, y, z, g);
                long s = site(nx, ny, x, y, z);
                for (int a = 0; a < 3; a++)
                    grad[a * N + s] = g[a];
            }
}

void orc_hessian(int nx, int ny, int nz, const double *psi, double *hess)
{
    lattice_init();
    long N = (long)nx * ny * nz;
#pragma omp parallel for if (orc_par((long)nx * ny * nz))
    for (long z = 0; z < nz; z++)
        for (long y = 0; y < ny; y++)
            for (long x = 0; x < nx; x++) {
                double H[3][3];
                hess_at(nx, ny, nz, psi, x, y, z, H);
                long s = site(nx, ny, x, y, z);
                for (int k = 0; k < 6; k++)
                    hess[k * N + s] = H[PAIR[k][0]][PAIR[k][1]];
            }
}

void orc_laplacian(int nx, int ny, int nz, const double *psi, double *lap)
{
    lattice_init();
#pragma omp parallel for if (orc_par((long)nx * ny * nz))
    for (long z = 0; z < nz; z++)
        for (long y = 0; y < ny; y++)
            for (long x = 0; x < nx; x++)
                lap[site(nx, ny, x, y, z)] = lap_at(nx, ny, nz, psi, x, y, z);
}

/* unit normal n = grad phi / |grad phi| (toward phi = 1) and curvature
 * K = div n = (|g|^2 tr H - g.H.g) / |g|^3; both zero where |g| <= 1e-12 */
static void normal_curv(const double g[3], const double H[3][3], double nhat[3], double *K)
{
    double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    double gn = sqrt(g2);
    if (gn > 1e-12) {
        double trH = H[0][0] + H[1][1] + H[2][2];
        double gHg = 0.0;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++)
                gHg += g[a] * H[a][b] * g[b];
        for (int a = 0; a < 3; a++)
            nhat[a] = g[a] / gn;
        *K = (g2 * trH - gHg) / (g2 * gn);
    } else {
        nhat[0] = nhat[1] = nhat[2] = 0.0;
        *K = 0.0;
    }
}

void orc_curvature(int nx, int ny, int nz, const double *phi, double *K, double *nhat)
{
    lattice_init();
    long N = (long)nx * ny * nz;
#pragma omp parallel for if (orc_par((long)nx * ny * nz))
    for (long z = 0; z < nz; z++)
        for (long y = 0; y < ny; y++)
            for (long x = 0; x < nx; x++) {
                double g[3], H[3][3], n[3], k;
                grad_at(nx, ny, nz, phi, x, y, z, g);
                hess_at(nx, ny, nz, phi, x, y, z, H);
                normal_curv(g, H, n, &k);
                long s = site(nx, ny, x, y, z);
                K[s] = k;
                if (nhat)
                    for (int a = 0; a < 3; a++)
                        nhat[a * N + s] = n[a];
            }
}

/* ------------------------------------------------------------- WENO-5 */

/* Jiang & Shu (1996) fifth-order WENO value at i+1/2 from the upwind-biased
 * cells i-2..i+2: three third-order candidates, smoothness indicators with
 * the 13/12 and 1/4 factors, linear weights (1/10, 6/10, 3/10), eps = 1e-6, p = 2. */
double orc_weno5(double vm2, double vm1, double v0, double vp1, double vp2)
{
    const double eps = 1e-6;
    double q0 = (2.0 * vm2 - 7.0 * vm1 + 11.0 * v0) / 6.0;
    double q1 = (-vm1 + 5.0 * v0 + 2.0 * vp1) / 6.0;
    double q2 = (2.0 * v0 + 5.0 * vp1 - vp2) / 6.0;
    double b0 = 13.0 / 12.0 * pow(vm2 - 2.0 * vm1 + v0, 2) + 0.25 * pow(vm2 - 4.0 * vm1 + 3.0 * v0, 2);
    double b1 = 13.0 / 12.0 * pow(vm1 - 2.0 * v0 + vp1, 2) + 0.25 * pow(vm1 - vp1, 2);
    double b2 = 13.0 / 12.0 * pow(v0 - 2.0 * vp1 + vp2, 2) + 0.25 * pow(3.0 * v0 - 4.0 * vp1 + vp2, 2);
    double a0 = 0.1 / pow(eps + b0, 2);
    double a1 = 0.6 / pow(eps + b1, 2);
    double a2 = 0.3 / pow(eps + b2, 2);
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

/* ------------------------------------------------------- Allen-Cahn step */

/* advective flux through the face between cell y and y + e_axis:
 * ubar * WENO-5 value upwinded by the sign of ubar (zero flux when ubar == 0) */
static double face_flux(int nx, int ny, int nz, const double *phi, const double *u, long x, long y, long z,
                        int axis)
{
    long N = (long)nx * ny * nz;
    int e[3] = {0, 0, 0};
    e[axis] = 1;
    long s0 = site(nx, ny, x, y, z);
    long s1 = nbr(nx, ny, nz, x, y, z, e[0], e[1], e[2]);
    double ubar = 0.5 * (u[axis * N + s0] + u[axis * N + s1]);
    if (ubar == 0.0)
        return 0.0;
    double v[6]; /* phi at y-2 .. y+3 along the axis */
    for (int k = -2; k <= 3; k++)
        v[k + 2] = phi[nbr(nx, ny, nz, x, y, z, k * e[0], k * e[1], k * e[2])];
    double face = ubar > 0.0 ? orc_weno5(v[0], v[1], v[2], v[3], v[4]) : orc_weno5(v[5], v[4], v[3], v[2], v[1]);
    return ubar * face;
}

/* phi^{n+1} = phi^n - div(u phi) + D lap(phi) - kappa div(phi (1 - phi) n), kappa = 4 D / delta */
void orc_ac_update(int nx, int ny, int nz, const double *phi, const double *u, double D, double width,
                   double *phi_new)
{
    lattice_init();
    long N = (long)nx * ny * nz;
    double kappa = 4.0 * D / width;
    double *Qv = (double *)malloc(sizeof(double) * 3 * N); /* phi (1 - phi) n at every site */
    double *J = (double *)malloc(sizeof(double) * 3 * N);  /* flux through the face x + e_a / 2 */
#pragma omp parallel for if (orc_par((long)nx * ny * nz))
    for (long z = 0; z < nz; z++)
        for (long y = 0; y < ny; y++)
            for (long x = 0; x < nx; x++) {
                double g[3], H[3][3], n[3], k;
                grad_at(nx, ny, nz, phi, x, y, z, g);
                memset(H, 0, sizeof H); /* the normal needs only g */
                normal_curv(g, H, n, &k);
                long s = site(nx, ny, x, y, z);
                double p = phi[s];
                for (int a = 0; a < 3; a++) {
                    Qv[a * N + s] = p * (1.0 - p) * n[a];
                    J[a * N + s] = face_flux(nx, ny, nz, phi, u, x, y, z, a);
                }
            }
#pragma omp parallel for if (orc_par((long)nx * ny * nz))
    for (long z = 0; z < nz; z++)
        for (long y = 0; y < ny; y++)
            for (long x = 0; x < nx; x++) {
                long s = site(nx, ny, x, y, z);
                long nb[Q];
                neighbours(nx, ny, nz, x, y, z, nb);
                /* convection: outgoing minus incoming face flux on each axis
                 * (nb[12] = x - e_x, nb[10] = x - e_y, nb[4] = x - e_z) */
                double adv = (J[s] - J[nb[12]]) + (J[N + s] - J[N + nb[10]]) + (J[2 * N + s] - J[2 * N + nb[4]]);
                /* diffusion (2/c_s^2) sum w_i (phi(x+c_i) - phi(x)) and sharpening (1/c_s^2) sum w_i Q(x+c_i).c_i */
                double lap = 0.0, divQ = 0.0;
                for (int i = 0; i < Q; i++) {
                    if (i != 13)
                        lap += WI[i] * (phi[nb[i]] - phi[s]);
                    for (int a = 0; a < 3; a++)
                        divQ += WI[i] * Qv[a * N + nb[i]] * CI[i][a];
                }
                lap *= 2.0 / CS2;
                divQ /= CS2;
                phi_new[s] = phi[s] - adv + D * lap - kappa * divQ;
            }
    free(Qv);
    free(J);
}

/* ------------------------------------------------------------- state */

struct orc_state {
    orc_params p;
    long N;
    long steps;
    double *f;      /* [27][N] pre-collision populations at time n */
    double *fpost;  /* [27][N] scratch */
    double *phi;    /* [N] */
    double *phinew; /* [N] */
    double *stage;  /* [N] Runge-Kutta stage (ac_rk3) */
    double *uprev;  /* [3][N] velocity of the previous step (Allen-Cahn advection) */
    double *unew;   /* [3][N] */
    double *aext;   /* [3][N] body acceleration */
    double *modes;  /* private copy */
    double *mlp;    /* private copy */
    double rho_mean; /* box-mean density (constant: sum phi is conserved) */
};

/* Relaxation time at phase field phi: the kinematic viscosity, affine in tau,
 * interpolates linearly between the phases, so tau does too; phi is clamped to
 * [0, 1] so that overshoots of the interface profile stay within the two
 * phases' values.  Uniform tau when tau_g <= 0 or in single phase. */
static double tau_at(const orc_params *p, double phi)
{
    if (!p->two_phase || p->tau_g <= 0.0)
        return p->tau;
    double c = phi < 0.0 ? 0.0 : (phi > 1.0 ? 1.0 : phi);
    return c * p->tau + (1.0 - c) * p->tau_g;
}

/* body acceleration a(x) = sum_m Re(A_m exp(i 2 pi (kx x/nx + ky y/ny + kz z/nz))) of an
 * nx x ny x nz periodic box, evaluated on the window of wx x wy x wz sites whose first
 * site is (ox, oy, oz) (global coordinates taken modulo the box); out [3][wz][wy][wx] */
void orc_forcing_window(const double *modes, int n_modes, int nx, int ny, int nz, int ox, int oy, int oz, int wx,
                        int wy, int wz, double *out)
{
    const long W = (long)wx * wy * wz;
    memset(out, 0, sizeof(double) * 3 * W);
#pragma omp parallel for if (orc_par((long)wx * wy * wz))
    for (long k = 0; k < wz; k++)
        for (long j = 0; j < wy; j++)
            for (long i = 0; i < wx; i++) {
                const long x = ((ox + i) % nx + nx) % nx, y = ((oy + j) % ny + ny) % ny, z = ((oz + k) % nz + nz) % nz;
                const long st = (k * wy + j) * wx + i;
                for (int m = 0; m < n_modes; m++) {
                    const double *r = modes + 9 * m;
                    double th = 2.0 * M_PI * (r[0] * x / nx + r[1] * y / ny + r[2] * z / nz);
                    double c = cos(th), sn = sin(th);
                    for (int a = 0; a < 3; a++)
                        out[a * W + st] += r[3 + 2 * a] * c - r[4 + 2 * a] * sn;
                }
            }
}

static void eval_forcing(orc_state *s)
{
    const orc_params *p = &s->p;
    if (p->n_modes <= 0) {
        memset(s->aext, 0, sizeof(double) * 3 * s->N);
        return;
    }
    orc_forcing_window(s->modes, p->n_modes, p->nx, p->ny, p->nz, 0, 0, 0, p->nx, p->ny, p->nz, s->aext);
}

/* fp16 round-to-nearest-even of a double (IEEE binary16: 10 fraction bits,
 * minimum normal 2^-14, subnormal quantum 2^-24, largest finite 65504) */
static int mlp_fp16 = 1;
void orc_mlp_set_fp16(int on) { mlp_fp16 = on; }

double orc_to_half(double v)
{
    if (!isfinite(v) || v == 0.0)
        return v;
    double a = fabs(v);
    int e;
    frexp(a, &e); /* a = m 2^e, m in [0.5, 1) */
    int ulp_exp = e - 11; /* 11 significant bits */
    if (ulp_exp < -24)
        ulp_exp = -24;
    double q = ldexp(nearbyint(ldexp(a, -ulp_exp)), ulp_exp);
    if (q > 65504.0)
        q = INFINITY;
    return v < 0 ? -q : q;
}

static double to_half(double v) { return mlp_fp16 ? orc_to_half(v) : v; }

/* MLP layout: W1[64][27], b1[64], W2[64][64], b2[64], W3[4][64], b3[4] */
#define H1 64
#define H2 64
#define NIN 27
#define NOUT 4
static void mlp_one(const double *w, const double *xin, double h1[H1], double h2[H2], double y[NOUT])
{
    const double *W1 = w, *b1 = W1 + H1 * NIN, *W2 = b1 + H1, *b2 = W2 + H2 * H1, *W3 = b2 + H2, *b3 = W3 + NOUT * H2;
    double x[NIN];
    for (int k = 0; k < NIN; k++)
        x[k] = to_half(xin[k]);
    for (int j = 0; j < H1; j++) {
        double s = b1[j];
        for (int k = 0; k < NIN; k++)
            s += W1[j * NIN + k] * x[k];
        h1[j] = to_half(tanh(s));
    }
    for (int j = 0; j < H2; j++) {
        double s = b2[j];
        for (int k = 0; k < H1; k++)
            s += W2[j * H1 + k] * h1[k];
        h2[j] = to_half(tanh(s));
    }
    for (int j = 0; j < NOUT; j++) {
        double s = b3[j];
        for (int k = 0; k < H2; k++)
            s += W3[j * H2 + k] * h2[k];
        y[j] = s;
    }
}

void orc_mlp_forward(const double *w, const double *x, long B, double *y)
{
#pragma omp parallel for if (orc_par(B * 64))
    for (long b = 0; b < B; b++) {
        double h1[H1], h2[H2];
        mlp_one(w, x + NIN * b, h1, h2, y + NOUT * b);
    }
}

/* loss = (1/B) sum_b sum_k (y_bk - t_bk)^2; gradient by the chain rule through
 * the two tanh layers (fp16 rounding of activations treated as identity) */
double orc_mlp_loss_grad(const double *w, const double *x, const double *yt, long B, double *grad)
{
    const double *W2 = w + H1 * NIN + H1, *W3 = W2 + H2 * H1 + H2;
    memset(grad, 0, sizeof(double) * ORC_MLP_NPARAM);
    double *gW1 = grad, *gb1 = gW1 + H1 * NIN, *gW2 = gb1 + H1, *gb2 = gW2 + H2 * H1, *gW3 = gb2 + H2,
           *gb3 = gW3 + NOUT * H2;
    double loss = 0.0;
    for (long b = 0; b < B; b++) {
        double h1[H1], h2[H2], y[NOUT], xin[NIN];
        mlp_one(w, x + NIN * b, h1, h2, y);
        for (int k = 0; k < NIN; k++)
            xin[k] = to_half(x[NIN * b + k]);
        double dy[NOUT], d2[H2], d1[H1];
        for (int j = 0; j < NOUT; j++) {
            double r = y[j] - yt[NOUT * b + j];
            loss += r * r;
            dy[j] = 2.0 * r / (double)B;
        }
        for (int j = 0; j < NOUT; j++) {
            gb3[j] += dy[j];
            for (int k = 0; k < H2; k++)
                gW3[j * H2 + k] += dy[j] * h2[k];
        }
        for (int k = 0; k < H2; k++) {
            double s = 0.0;
            for (int j = 0; j < NOUT; j++)
                s += W3[j * H2 + k] * dy[j];
            d2[k] = s * (1.0 - h2[k] * h2[k]);
        }
        for (int j = 0; j < H2; j++) {
            gb2[j] += d2[j];
            for (int k = 0; k < H1; k++)
                gW2[j * H1 + k] += d2[j] * h1[k];
        }
        for (int k = 0; k < H1; k++) {
            double s = 0.0;
            for (int j = 0; j < H2; j++)
                s += W2[j * H1 + k] * d2[j];
            d1[k] = s * (1.0 - h1[k] * h1[k]);
        }
        for (int j = 0; j < H1; j++) {
            gb1[j] += d1[j];
            for (int k = 0; k < NIN; k++)
                gW1[j * NIN + k] += d1[j] * xin[k];
        }
    }
    return loss / (double)B;
}

/* Adam (Kingma & Ba 2015) on FP64 master weights with bias correction at
 * step t >= 1; w16 receives the fp16 rounding of the updated weights. */
void orc_adam(double *w, double *m, double *v, const double *g, long n, long t, double lr, double b1, double b2,
              double eps, double *w16)
{
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (long p = 0; p < n; p++) {
        m[p] = b1 * m[p] + (1.0 - b1) * g[p];
        v[p] = b2 * v[p] + (1.0 - b2) * g[p] * g[p];
        double mhat = m[p] / c1, vhat = v[p] / c2;
        w[p] -= lr * mhat / (sqrt(vhat) + eps);
        if (w16)
            w16[p] = orc_to_half(w[p]);
    }
}

/* curvature and normal used by the surface-tension force: finite differences,
 * or the smooth blend with the network output where |K_FD| exceeds k_lo */
static void site_curvature(const orc_state *s, long st, const long nb[Q], const double g[3], double *K,
                           double nhat[3])
{
    const orc_params *p = &s->p;
    double H[3][3];
    hess_nb(s->phi, nb, H);
    normal_curv(g, H, nhat, K);
    if (p->curv_mode != 1 || !s->mlp)
        return;
    double phic = s->phi[st];
    if (!(phic > 0.02 && phic < 0.98))
        return;
    double kfd = fabs(*K);
    if (!(kfd > p->k_lo))
        return;
    double t = (kfd - p->k_lo) / (p->k_hi - p->k_lo);
    if (t > 1.0)
        t = 1.0;
    double sw = t * t * (3.0 - 2.0 * t); /* smoothstep */
    double xin[NIN], h1[H1], h2[H2], out[NOUT];
    for (int i = 0; i < Q; i++)
        xin[i] = 2.0 * s->phi[nb[i]] - 1.0;
    mlp_one(s->mlp, xin, h1, h2, out);
    double nn = sqrt(out[1] * out[1] + out[2] * out[2] + out[3] * out[3]);
    if (!isfinite(out[0]) || !isfinite(nn) || nn < 0.5 || nn > 1.5)
        return;
    *K = sw * out[0] + (1.0 - sw) * (*K);
    double b[3], bn = 0.0;
    for (int a = 0; a < 3; a++) {
        b[a] = sw * out[1 + a] / nn + (1.0 - sw) * nhat[a];
        bn += b[a] * b[a];
    }
    bn = sqrt(bn);
    if (bn > 1e-12)
        for (int a = 0; a < 3; a++)
            nhat[a] = b[a] / bn;
}

typedef struct {
    double pstar, rho, j[3], u[3], acc[3], tau;
} macro_t;

/* moments, forces and velocity at one site (Sec. 2.2-2.3, Eq. 8) */
static void site_macro(const orc_state *s, long x, long y, long z, const double f[Q], macro_t *m)
{
    const orc_params *p = &s->p;
    long N = s->N;
    long st = site(p->nx, p->ny, x, y, z);
    double pstar = 0.0, j[3] = {0, 0, 0};
    for (int i = 0; i < Q; i++) {
        pstar += f[i];
        for (int a = 0; a < 3; a++)
            j[a] += f[i] * CI[i][a];
    }
    double rho, g[3] = {0, 0, 0}, K = 0.0, ns[3] = {0, 0, 0}, phic = 1.0;
    if (p->two_phase) {
        phic = s->phi[st];
        rho = phic * p->rho_l + (1.0 - phic) * p->rho_g;
        long nb[Q];
        neighbours(p->nx, p->ny, p->nz, x, y, z, nb);
        grad_nb(s->phi, nb, g);
        site_curvature(s, st, nb, g, &K, ns);
    } else {
        rho = p->rho_l;
    }
    double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    double Fs[3], Fp[3], Fb[3], grho[3], u0[3];
    for (int a = 0; a < 3; a++) {
        Fs[a] = -1.5 * p->width * p->sigma * K * g2 * ns[a]; /* -(3 delta/2) sigma K |g|^2 n_s */
        grho[a] = (p->rho_l - p->rho_g) * g[a];
        Fp[a] = -pstar * CS2 * grho[a];
        /* body force, plus buoyancy against the box-mean hydrostatic balance
           (absent, not multiplied by zero, without gravity: a non-finite site
           would otherwise reach every site through the box mean) */
        Fb[a] = rho * s->aext[a * N + st];
        if (p->gravity[a] != 0.0)
            Fb[a] += (rho - s->rho_mean) * p->gravity[a];
        u0[a] = j[a] + (Fs[a] + Fp[a] + Fb[a]) / (2.0 * rho);
    }
    /* viscous correction with the non-equilibrium stress at u0 */
    double feq0[Q], P[3][3];
    orc_feq(pstar, u0, feq0);
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double sum = 0.0;
            for (int i = 0; i < Q; i++)
                sum += (f[i] - feq0[i]) * CI[i][a] * CI[i][b];
            P[a][b] = sum;
        }
    double tau = tau_at(p, phic);
    double nu = CS2 * (tau - 0.5);
    for (int a = 0; a < 3; a++) {
        double Fnu = 0.0;
        for (int b = 0; b < 3; b++)
            Fnu += P[a][b] * grho[b];
        Fnu *= -(nu / (tau * CS2));
        double F = Fs[a] + Fp[a] + Fb[a] + Fnu;
        m->acc[a] = F / rho;
        m->j[a] = j[a];
        m->u[a] = j[a] + 0.5 * m->acc[a];
    }
    m->pstar = pstar;
    m->rho = rho;
    m->tau = tau;
}

orc_state *orc_create(const orc_params *p, const double *phi0, const double *u0, const double *pstar0)
{
    lattice_init();
    if (p->nx < 1 || p->ny < 1 || p->nz < 1 || p->tau <= 0.5 || (p->tau_g > 0.0 && p->tau_g <= 0.5))
        return NULL;
    orc_state *s = (orc_state *)calloc(1, sizeof(orc_state));
    s->p = *p;
    long N = (long)p->nx * p->ny * p->nz;
    s->N = N;
    s->f = (double *)malloc(sizeof(double) * Q * N);
    s->fpost = (double *)malloc(sizeof(double) * Q * N);
    s->phi = (double *)calloc(N, sizeof(double));
    s->phinew = (double *)calloc(N, sizeof(double));
    s->stage = (double *)calloc(N, sizeof(double));
    s->uprev = (double *)calloc(3 * N, sizeof(double));
    s->unew = (double *)calloc(3 * N, sizeof(double));
    s->aext = (double *)calloc(3 * N, sizeof(double));
    if (p->n_modes > 0) {
        s->modes = (double *)malloc(sizeof(double) * 9 * p->n_modes);
        memcpy(s->modes, p->modes, sizeof(double) * 9 * p->n_modes);
    }
    if (p->mlp) {
        s->mlp = (double *)malloc(sizeof(double) * ORC_MLP_NPARAM);
        memcpy(s->mlp, p->mlp, sizeof(double) * ORC_MLP_NPARAM);
    }
    s->p.modes = s->modes;
    s->p.mlp = s->mlp;
    if (phi0 && p->two_phase)
        memcpy(s->phi, phi0, sizeof(double) * N);
    if (p->two_phase) {
        double sum = 0.0;
        for (long i = 0; i < N; i++)
            sum += s->phi[i];
        s->rho_mean = p->rho_g + (p->rho_l - p->rho_g) * (sum / (double)N);
    } else {
        s->rho_mean = p->rho_l;
    }
    if (u0)
        memcpy(s->uprev, u0, sizeof(double) * 3 * N);
    eval_forcing(s);
    /* f^0 = f^eq(p*0, u0) + w H : A0 / (2 c_s^4), A0 = -c_s^2 tau (grad u0 + grad u0^T),
     * the second-order coefficient of Sec. 2.2 with the lattice gradient */
    int nx = p->nx, ny = p->ny, nz = p->nz;
#pragma omp parallel for if (orc_par((long)nx * ny * nz))
    for (long z = 0; z < nz; z++)
        for (long y = 0; y < ny; y++)
            for (long x = 0; x < nx; x++) {
                long st = site(nx, ny, x, y, z);
                double u[3], G[3][3], feq[Q];
                for (int a = 0; a < 3; a++) {
                    u[a] = s->uprev[a * N + st];
                    grad_at(nx, ny, nz, s->uprev + a * N, x, y, z, G[a]); /* G[a][b] = d_b u_a */
                }
                double A[3][3];
                for (int a = 0; a < 3; a++)
                    for (int b = 0; b < 3; b++)
                        A[a][b] = -CS2 * tau_at(p, s->phi[st]) * (G[a][b] + G[b][a]);
                double ps = pstar0 ? pstar0[st] : p->p0;
                orc_feq(ps, u, feq);
                for (int i = 0; i < Q; i++) {
                    double hA = 0.0;
                    for (int a = 0; a < 3; a++)
                        for (int b = 0; b < 3; b++)
                            hA += herm(i, a, b) * A[a][b];
                    s->f[i * N + st] = feq[i] + WI[i] * hA / (2.0 * CS2 * CS2);
                }
            }
    return s;
}

void orc_destroy(orc_state *s)
{
    if (!s)
        return;
    free(s->f);
    free(s->fpost);
    free(s->phi);
    free(s->phinew);
    free(s->stage);
    free(s->uprev);
    free(s->unew);
    free(s->aext);
    free(s->modes);
    free(s->mlp);
    free(s);
}

void orc_step(orc_state *s, long nsteps)
{
    const orc_params *p = &s->p;
    int nx = p->nx, ny = p->ny, nz = p->nz;
    long N = s->N;
    for (long it = 0; it < nsteps; it++) {
        /* 1. collide every site with the fields of time n */
#pragma omp parallel for if (orc_par((long)nx * ny * nz))
        for (long z = 0; z < nz; z++)
            for (long y = 0; y < ny; y++)
                for (long x = 0; x < nx; x++) {
                    long st = site(nx, ny, x, y, z);
                    double f[Q], fp[Q];
                    macro_t m;
                    for (int i = 0; i < Q; i++)
                        f[i] = s->f[i * N + st];
                    site_macro(s, x, y, z, f, &m);
                    orc_collide(f, m.u, m.acc, m.tau, fp, NULL);
                    for (int i = 0; i < Q; i++)
                        s->fpost[i * N + st] = fp[i];
                    for (int a = 0; a < 3; a++)
                        s->unew[a * N + st] = m.u[a];
                }
        /* 2. Allen-Cahn update with the velocity of the previous step */
        if (p->two_phase)
        {
            if (p->ac_rk3) {
                /* three-stage strong-stability-preserving Runge-Kutta (Shu & Osher),
                 * each stage an Euler step of the same right-hand side with the
                 * velocity held at u^(n-1):
                 *   phi1 = phi + L(phi),  phi2 = 3/4 phi + 1/4 (phi1 + L(phi1)),
                 *   phi^{n+1} = 1/3 phi + 2/3 (phi2 + L(phi2)) */
                orc_ac_update(nx, ny, nz, s->phi, s->uprev, p->mobility, p->width, s->phinew);
                orc_ac_update(nx, ny, nz, s->phinew, s->uprev, p->mobility, p->width, s->stage);
                for (long i = 0; i < N; i++)
                    s->stage[i] = 0.75 * s->phi[i] + 0.25 * s->stage[i];
                orc_ac_update(nx, ny, nz, s->stage, s->uprev, p->mobility, p->width, s->phinew);
                for (long i = 0; i < N; i++)
                    s->phinew[i] = s->phi[i] / 3.0 + (2.0 / 3.0) * s->phinew[i];
            } else {
                orc_ac_update(nx, ny, nz, s->phi, s->uprev, p->mobility, p->width, s->phinew);
            }
        }
        /* 3. streaming: f_i(x, n+1) = f^post_i(x - c_i, n) */
#pragma omp parallel for if (orc_par((long)nx * ny * nz))
        for (long z = 0; z < nz; z++)
            for (long y = 0; y < ny; y++)
                for (long x = 0; x < nx; x++) {
                    long st = site(nx, ny, x, y, z);
                    for (int i = 0; i < Q; i++)
                        s->f[i * N + st] = s->fpost[i * N + nbr(nx, ny, nz, x, y, z, -CI[i][0], -CI[i][1], -CI[i][2])];
                }
        double *t;
        if (p->two_phase) {
            t = s->phi;
            s->phi = s->phinew;
            s->phinew = t;
        }
        t = s->uprev;
        s->uprev = s->unew;
        s->unew = t;
        s->steps++;
    }
}

void orc_moments(const orc_state *s, double *rho, double *pr, double *u, double *phi)
{
    const orc_params *p = &s->p;
    int nx = p->nx, ny = p->ny, nz = p->nz;
    long N = s->N;
#pragma omp parallel for if (orc_par((long)nx * ny * nz))
    for (long z = 0; z < nz; z++)
        for (long y = 0; y < ny; y++)
            for (long x = 0; x < nx; x++) {
                long st = site(nx, ny, x, y, z);
                double f[Q];
                macro_t m;
                for (int i = 0; i < Q; i++)
                    f[i] = s->f[i * N + st];
                site_macro(s, x, y, z, f, &m);
                if (rho)
                    rho[st] = m.rho;
                if (pr)
                    pr[st] = m.pstar * m.rho * CS2; /* p = p* rho c_s^2 */
                if (u)
                    for (int a = 0; a < 3; a++)
                        u[a * N + st] = m.u[a];
                if (phi)
                    phi[st] = p->two_phase ? s->phi[st] : 0.0;
            }
}

/* out: 0 sum phi, 1 sum rho, 2 sum p*, 3-5 sum rho u, 6 (1/2) sum rho |u|^2,
 *      7 max |u|, 8 max overshoot of phi outside [0, 1], 9 count of sites with
 *      a non-finite p*, u or phi */
void orc_reduce(const orc_state *s, double out[ORC_NRED])
{
    long N = s->N;
    double *rho = (double *)malloc(sizeof(double) * N), *ps = (double *)malloc(sizeof(double) * N);
    double *u = (double *)malloc(sizeof(double) * 3 * N), *phi = (double *)malloc(sizeof(double) * N);
    orc_moments(s, rho, ps, u, phi);
    for (int k = 0; k < ORC_NRED; k++)
        out[k] = 0.0;
    for (long st = 0; st < N; st++) {
        double r = rho[st];
        double pstar = ps[st] / (r * CS2);
        double ux = u[st], uy = u[N + st], uz = u[2 * N + st];
        double ph = phi[st];
        int bad = !isfinite(pstar) || !isfinite(ux) || !isfinite(uy) || !isfinite(uz) || !isfinite(ph);
        if (bad) {
            out[9] += 1.0;
            continue;
        }
        out[0] += ph;
        out[1] += r;
        out[2] += pstar;
        out[3] += r * ux;
        out[4] += r * uy;
        out[5] += r * uz;
        double u2 = ux * ux + uy * uy + uz * uz;
        out[6] += 0.5 * r * u2;
        if (sqrt(u2) > out[7])
            out[7] = sqrt(u2);
        double ov = ph > 1.0 ? ph - 1.0 : (ph < 0.0 ? -ph : 0.0);
        if (s->p.two_phase && ov > out[8])
            out[8] = ov;
    }
    free(rho);
    free(ps);
    free(u);
    free(phi);
}

void orc_get_f(const orc_state *s, double *f) { memcpy(f, s->f, sizeof(double) * Q * s->N); }
void orc_set_f(orc_state *s, const double *f) { memcpy(s->f, f, sizeof(double) * Q * s->N); }
void orc_get_uprev(const orc_state *s, double *u) { memcpy(u, s->uprev, sizeof(double) * 3 * s->N); }
void orc_set_aext(orc_state *s, const double *a) { memcpy(s->aext, a, sizeof(double) * 3 * s->N); }
long orc_steps_done(const orc_state *s) { return s->steps; }

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Training samples: every interface cell (0.02 < phi < 0.98) is labelled with
 * the nearest sphere's curvature (-2/R for a phi = 1 sphere, +2/R for a phi = 0
 * sphere; radii < 0 mark phi = 0 spheres) and the radial unit normal pointing
 * toward phi = 1; the input is 2 phi - 1 on the 3^3 stencil in lattice order. */
void orc_harvest(int nx, int ny, int nz, const double *phi, const double *centers, const double *radii, int nb,
                 double *X, double *Y, long cap, long *n_out)
{
    lattice_init();
    long n = 0;
    for (long z = 0; z < nz; z++)
        for (long y = 0; y < ny; y++)
            for (long x = 0; x < nx; x++) {
                double ph = phi[site(nx, ny, x, y, z)];
                if (!(ph > 0.02 && ph < 0.98))
                    continue;
                int best = -1;
                double bestd = INFINITY, d[3] = {0, 0, 0}, r = 0.0;
                for (int b = 0; b < nb; b++) {
                    double dd[3] = {x - centers[3 * b], y - centers[3 * b + 1], z - centers[3 * b + 2]};
                    double L[3] = {nx, ny, nz};
                    for (int a = 0; a < 3; a++)
                        dd[a] -= L[a] * nearbyint(dd[a] / L[a]);
                    double rr = sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
                    double gap = fabs(rr - fabs(radii[b]));
                    if (gap < bestd) {
                        bestd = gap;
                        best = b;
                        r = rr;
                        memcpy(d, dd, sizeof d);
                    }
                }
                if (best < 0 || r < 1e-12)
                    continue;
                if (n < cap) {
                    for (int i = 0; i < Q; i++)
                        X[27 * n + i] = 2.0 * phi[nbr(nx, ny, nz, x, y, z, CI[i][0], CI[i][1], CI[i][2])] - 1.0;
                    double R = radii[best];
                    double sgn = R > 0 ? -1.0 : 1.0; /* toward phi = 1 */
                    Y[4 * n + 0] = R > 0 ? -2.0 / R : 2.0 / (-R);
                    for (int a = 0; a < 3; a++)
                        Y[4 * n + 1 + a] = sgn * d[a] / r;
                }
                n++;
            }
    *n_out = n;
}
