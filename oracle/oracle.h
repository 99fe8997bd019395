/*
 * FP64 CPU oracle of the accLB lattice update (arXiv 2505.01126, Sec. 2).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header or
 * table with the GPU library; the two meet only through the seeded input arrays.
 *
 * Layout: every field is C order with x fastest, site index
 *   s = (z * ny + y) * nx + x,   N = nx * ny * nz.
 * Vector fields are component major (SoA): v[c * N + s].
 * Populations are f[i * N + s] with the D3Q27 velocity
 *   c_i = (i % 3 - 1, (i / 3) % 3 - 1, i / 9 - 1),  i = 0..26 (rest = 13).
 */
#ifndef ACCLB_ORACLE_H
#define ACCLB_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_Q 27
#define ORC_NRED 10
#define ORC_MLP_NPARAM 6212 /* 27*64+64 + 64*64+64 + 64*4+4 */

typedef struct {
    int nx, ny, nz;
    int two_phase;          /* 0: single phase (rho = rho_l, no phase field) */
    double tau;             /* BGK relaxation time, nu = c_s^2 (tau - 1/2) */
    double rho_l, rho_g;    /* densities of the phi = 1 and phi = 0 phases */
    double sigma;           /* surface tension (gamma in the paper) */
    double mobility;        /* interface diffusivity D */
    double width;           /* interface width delta; kappa_AC = 4 D / delta */
    double p0;              /* p* used where no initial pressure is given */
    int n_modes;            /* forcing table rows (0 = no body force) */
    const double *modes;    /* [n_modes][9]: kx ky kz ReAx ImAx ReAy ImAy ReAz ImAz */
    int curv_mode;          /* 0 = finite-difference curvature, 1 = MLP blend */
    double k_lo, k_hi;      /* blend ramp on |K_FD| for curv_mode = 1 */
    const double *mlp;      /* ORC_MLP_NPARAM weights (values already fp16-exact) */
    double gravity[3];      /* buoyancy acceleration g: force (rho - rho_mean) g, rho_mean the box mean */
    double tau_g;           /* relaxation time of the phi = 0 phase (<= 0: tau); tau(phi) interpolates */
    int ac_rk3;             /* Allen-Cahn time integration: 0 explicit Euler, 1 three-stage SSP Runge-Kutta */
} orc_params;

typedef struct orc_state orc_state;

/* lattice tables */
void orc_lattice(int *c /* 27*3 */, double *w /* 27 */);

/* single-site building blocks (Sec. 2.2) */
void orc_feq(double pstar, const double u[3], double out[ORC_Q]);
void orc_guo(const double u[3], const double acc[3], double out[ORC_Q]);
/* regularised post-collision populations, Eqs. (6)-(7); returns a^(2) in a2[6] (xx yy zz xy xz yz) */
void orc_collide(const double f[ORC_Q], const double u[3], const double acc[3], double tau,
                 double fpost[ORC_Q], double a2[6]);

/* lattice stencils (Sec. 2.3), periodic */
void orc_gradient(int nx, int ny, int nz, const double *psi, double *grad /* 3N */);
void orc_hessian(int nx, int ny, int nz, const double *psi, double *hess /* 6N */);
void orc_laplacian(int nx, int ny, int nz, const double *psi, double *lap);
void orc_curvature(int nx, int ny, int nz, const double *phi, double *K, double *nhat /* 3N or NULL */);

/* WENO-5 (Jiang-Shu) reconstruction at i+1/2 from v[i-2..i+2] */
double orc_weno5(double vm2, double vm1, double v0, double vp1, double vp2);

/* One explicit Allen-Cahn update, Eq. (3) in flux form, with cell velocity u (3N). */
void orc_ac_update(int nx, int ny, int nz, const double *phi, const double *u, double D, double width,
                   double *phi_new);

/* whole-solver state */
orc_state *orc_create(const orc_params *p, const double *phi0, const double *u0, const double *pstar0);
void orc_destroy(orc_state *s);
void orc_step(orc_state *s, long nsteps);
void orc_moments(const orc_state *s, double *rho, double *p, double *u, double *phi);
void orc_reduce(const orc_state *s, double out[ORC_NRED]);
void orc_get_f(const orc_state *s, double *f);
void orc_set_f(orc_state *s, const double *f);
void orc_get_uprev(const orc_state *s, double *u);
/* replace the body acceleration field [3][N] (e.g. a window of a larger box's forcing) */
void orc_set_aext(orc_state *s, const double *a);
/* the mode-table body acceleration of an nx x ny x nz box on a window of it (see oracle.c) */
void orc_forcing_window(const double *modes, int n_modes, int nx, int ny, int nz, int ox, int oy, int oz, int wx,
                        int wy, int wz, double *out);
long orc_steps_done(const orc_state *s);
int orc_threads(void);

/* learned curvature network 27 -> 64 -> 64 -> 4 (tanh hidden), fp16 rounding of
 * inputs and hidden activations emulated; weights layout in orc_mlp_forward. */
double orc_to_half(double v);          /* IEEE binary16 round-to-nearest-even, as a double */
void orc_mlp_set_fp16(int on);         /* 0 disables the fp16 emulation (gradient checks) */
void orc_mlp_forward(const double *w, const double *x /* B*27 */, long B, double *y /* B*4 */);
double orc_mlp_loss_grad(const double *w, const double *x, const double *yt, long B, double *grad /* NPARAM */);
void orc_adam(double *w, double *m, double *v, const double *g, long n, long t, double lr, double b1, double b2,
              double eps, double *w16);
void orc_harvest(int nx, int ny, int nz, const double *phi, const double *centers, const double *radii, int nb,
                 double *X /* cap*27 */, double *Y /* cap*4 */, long cap, long *n_out);

#ifdef __cplusplus
}
#endif
#endif
