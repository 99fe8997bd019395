/*
 * lbm.h -- C ABI of the MI355X lattice update library (liblbm.so).
 *
 * One time step of the method of accLB (arXiv 2505.01126, Sec. 2):
 *   - D3Q27 populations, pull-streamed and rebuilt by the regularised collision
 *     of Eqs. (6)-(7) from p*, u and the Hermite coefficient a^(2), so every
 *     site writes only its own slots (Sec. 3, thread-safe formulation);
 *   - Guo forcing, Eq. (5), with the total force of Eq. (8): surface tension
 *     F^s, pressure correction F^p, viscous correction F^nu, plus an optional
 *     time-independent body force (Sec. 5.1);
 *   - the conservative Allen-Cahn phase field, Eq. (3), advected with WENO-5
 *     and diffused/sharpened with the lattice stencils of Sec. 2.3, on its own
 *     array, coupled to the same kernel.
 *
 * Conventions
 *   Grid: periodic nx * ny * nz, site s = (z * ny + y) * nx + x, N = nx*ny*nz.
 *   Vector fields are component major (SoA): v[c * N + s], c = x, y, z.
 *   Lattice units: dx = dt = 1, c_s^2 = 1/3, nu = c_s^2 (tau - 1/2).
 *   All device pointers belong to the caller; the library never allocates or
 *   frees device memory (it owns one fixed device array, the scratch of
 *   lbm_mlp_backward_static).  Every call is asynchronous on the stream given to
 *   lbm_init / lbm_set_stream unless stated otherwise.
 *   One handle per stream; a handle is not thread safe.
 *
 * Errors: every int-returning call gives LBM_OK (0) or a negative code;
 * lbm_last_error() holds the text of the latest failure on a handle.  Nothing
 * throws across the ABI.  Non-finite fields are reported by lbm_reduce
 * (out[9]), not as an error code.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 5
#define LBM_NRED 10          /* number of lbm_reduce outputs */
#define LBM_MAX_MODES 64     /* forcing table rows */
#define LBM_MLP_NPARAM 6212  /* 27*64+64 + 64*64+64 + 64*4+4 */

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,   /* bad dimensions or parameters */
    LBM_ENOSPACE = -2, /* workspace smaller than lbm_workspace_bytes() */
    LBM_EHIP = -3,     /* a HIP runtime error (text in lbm_last_error) */
    LBM_ESTATE = -4,   /* call not valid in the handle's state */
    LBM_ERANGE = -5    /* a size above the fixed maximum of an entry point without a workspace */
};

/* population storage: FP32, or FP16 / BF16 holding h_i = f_i / w_i - P0
 * (arithmetic is FP32 in every mode; FP32 storage holds the same shifted h_i).
 * FP16 rounds to nearest even.  BF16 rounds the step's stores stochastically
 * (dither: the low 16 bits of another population of the same site, so the
 * result is deterministic), which keeps a weak body force's per-step change
 * that rounding to nearest would drop; lbm_init rounds to nearest. */
enum { LBM_STORE_F32 = 0, LBM_STORE_F16 = 1, LBM_STORE_BF16 = 2 };

/* phase-field storage (two-phase runs; the arithmetic is FP32 in both):
 *   F64:   FP64 phi; each face and link flux of Eq. (3) is added in FP64, so
 *          sum phi is conserved to FP64 round-off;
 *   FIX32: int32 fixed point q = phi * 2^30 (phi in [-2, 2), quantum 2^-30);
 *          each flux is rounded to nearest on that grid and the two sites of a
 *          face or link add and subtract the same integer, so sum phi is
 *          conserved bit for bit; 4 bytes less read and written per site and
 *          step.  Initial values outside [-2, 2) are clamped. */
enum { LBM_PHI_F64 = 0, LBM_PHI_FIX32 = 1 };

/* curvature used by the surface-tension force */
enum { LBM_CURV_FD = 0, LBM_CURV_MLP = 1 };

typedef struct lbm_handle lbm_handle;

typedef struct {
    int32_t nx, ny, nz;  /* each >= 8, nx*ny <= 2^24, nx*ny*nz <= 2^30 */
    int32_t storage;     /* LBM_STORE_* */
    int32_t two_phase;   /* 0: single phase (rho = rho_l, no phase field), 1: coupled Allen-Cahn */
    int32_t curv_mode;   /* LBM_CURV_*; LBM_CURV_MLP needs lbm_set_mlp before stepping */
    double tau;          /* relaxation time > 1/2 (omega = 1/tau, Sec. 2.2) */
    double rho_l, rho_g; /* densities of the phi = 1 and phi = 0 phases, > 0 */
    double sigma;        /* surface tension (gamma of Sec. 2.3) */
    double mobility;     /* interface diffusivity D of Eq. (3) */
    double width;        /* interface width delta; kappa = 4 D / delta */
    double p0;           /* pressure gauge P0: storage shift and the p* used when no initial p* is given */
    int32_t n_modes;     /* forcing rows, 0 .. LBM_MAX_MODES */
    int32_t zchunk;      /* z planes per work item (0 = library default: 32 for FP32 storage, 64 for FP16/BF16) */
    const double *modes; /* HOST table [n_modes][9]: kx ky kz Re(Ax) Im(Ax) Re(Ay) Im(Ay) Re(Az) Im(Az);
                            integer wave numbers with |kx| <= 2; body acceleration
                            a(x) = sum_m Re(A_m exp(2 pi i (kx x/nx + ky y/ny + kz z/nz)));
                            read during lbm_init only */
    double mlp_k_lo;     /* MLP blend ramp on |K_FD| (defaults 0.4 .. 0.6 when both are 0) */
    double mlp_k_hi;
    int32_t phi_storage; /* LBM_PHI_* (ignored in single phase) */
    int32_t reserved;    /* 0 */
    /* Two-phase only (ignored in single phase).  Buoyancy: body force
     * (rho - rho_mean) g, rho_mean the box-mean density (constant, since
     * sum phi is conserved), so a periodic box with gravity does not accelerate
     * as a whole; with g != 0, lbm_init measures rho_mean on the device and
     * waits for the stream.  Viscosity contrast: tau_g > 1/2 is the relaxation
     * time of the phi = 0 phase and tau(phi) = phi tau + (1 - phi) tau_g with
     * phi clamped to [0, 1] (the kinematic viscosity interpolates linearly);
     * tau_g = 0 keeps one tau. */
    double gravity[3];   /* g (x, y, z), lattice units */
    double tau_g;
    /* Time integration of the phase field (two-phase only): 0 explicit Euler,
     * one update per step inside the step kernel; 1 three-stage strong-
     * stability-preserving Runge-Kutta (Shu-Osher) with the velocity held at
     * the previous step's: the step kernel's Euler update is the first stage
     * and two more launches per step add the others (needs phi_storage F64;
     * 2 x 8 bytes per site more workspace). */
    int32_t ac_rk3;
    int32_t reserved2;   /* 0 */
} lbm_config;

/* LBM_ABI_VERSION of the loaded library. */
int lbm_abi_version(void);

/* Device bytes the caller must provide to lbm_init for this configuration;
 * 0 when the configuration is invalid. */
size_t lbm_workspace_bytes(const lbm_config *cfg);

/* Create a handle and write the initial state into the workspace.
 *   d_ws     device buffer of ws_bytes >= lbm_workspace_bytes(cfg), 256-byte
 *            aligned, owned by the caller and kept alive for the handle's life;
 *            it holds the whole solver state (populations, phi, u).
 *   d_phi0   device FP64 [N], phi at t = 0 (required when two_phase, else ignored)
 *   d_u0     device FP64 [3N] SoA velocity at t = 0, or NULL for rest
 *   d_pstar0 device FP64 [N] p* at t = 0, or NULL for p* = P0 everywhere
 *   stream   hipStream_t (NULL = default stream); the inputs may be released
 *            once the stream has passed this call.
 * Populations start at f^eq(p*, u) plus the regularised non-equilibrium part
 * with a^(2) = -c_s^2 tau (grad u + grad u^T) (Sec. 2.2).
 * Returns LBM_EINVAL (bad config or NULL d_phi0 with two_phase),
 * LBM_ENOSPACE, LBM_EHIP. */
int lbm_init(lbm_handle **out, const lbm_config *cfg, void *d_ws, size_t ws_bytes, const double *d_phi0,
             const double *d_u0, const double *d_pstar0, void *stream);

/* Advance nsteps >= 0 time steps of the coupled scheme: per step, the pull
 * streaming of the populations (Sec. 2.2, Eq. 4), their moments, the
 * surface-tension, pressure and viscous forces (Sec. 2.3, Eq. 8) with the
 * velocity u = j + a/2, the regularised collision (Sec. 2.2, Eqs. 6-7) and the
 * conservative Allen-Cahn update of phi (Sec. 2.1, Eq. 3; WENO-5 convection).
 * One fused kernel launch per step, plus the learned-curvature network pass
 * ahead of it (LBM_CURV_MLP) and two more phase-field stages after it
 * (ac_rk3); pairs of steps replay a captured graph.  Asynchronous on the
 * handle's stream; the state stays in the caller's workspace.  Returns
 * LBM_EINVAL (NULL handle or nsteps < 0), LBM_ESTATE (LBM_CURV_MLP before
 * lbm_set_mlp), LBM_EHIP (launch failure, text in lbm_last_error). */
int lbm_step(lbm_handle *h, int64_t nsteps);

/* Fields at the current time n, written to caller device buffers; any pointer
 * may be NULL.  rho and p = p* rho c_s^2 are FP32 [N], u FP32 [3N] SoA with
 * u = j + a/2 (Sec. 2.2), phi FP64 [N] (converted exactly from the fixed-point
 * storage). */
int lbm_moments(lbm_handle *h, float *d_rho, float *d_p, float *d_u, double *d_phi);

/* Global FP64 statistics at time n: the conserved phase volume sum phi that
 * the conservative Allen-Cahn form keeps constant (Sec. 2.1, Eq. 3), and the
 * mass, momentum and kinetic-energy sums of the flow (the energy budget of the
 * forced turbulence of Sec. 5.1), in a deterministic order of summation:
 *   out[0] sum phi, [1] sum rho, [2] sum p*, [3..5] sum rho u, [6] 1/2 sum rho |u|^2,
 *   [7] max |u|, [8] max overshoot of phi outside [0, 1], [9] sites with a non-finite
 *   p*, u or phi.
 * out_is_host = 1: out is host memory and the call waits for the stream;
 * out_is_host = 0: out is device memory, written asynchronously. */
int lbm_reduce(lbm_handle *h, double *out, int out_is_host);

/* Steps taken since lbm_init. */
int64_t lbm_steps_done(const lbm_handle *h);

/* Change the stream later calls run on. */
int lbm_set_stream(lbm_handle *h, void *stream);

/* Release the handle (host memory only; the workspace stays the caller's). */
int lbm_destroy(lbm_handle *h);

/* ------------------------------------------------------------------ learned curvature
 * A small network maps the 3^3 phi stencil of an interface cell to its
 * curvature and normal (an extension of the finite-difference curvature of
 * Sec. 2.3, used where bubbles are under-resolved): inputs x = 2 phi - 1 on
 * the 27 lattice directions (fp16, rows padded to LBM_MLP_IN = 32 with zeros),
 * two tanh hidden layers of 64, outputs (K, n_x, n_y, n_z).  Parameters are
 * LBM_MLP_NPARAM IEEE binary16 values (uint16_t bits) in the order
 * W1[64][27], b1[64], W2[64][64], b2[64], W3[4][64], b3[4].  Matrix products run
 * on FP16 MFMA with FP32 accumulation; hidden activations are rounded to fp16. */
#define LBM_MLP_IN 32
#define LBM_MLP_MAX_SPHERES 1024

/* Device bytes of scratch lbm_mlp_backward needs for a batch of B samples. */
size_t lbm_mlp_work_bytes(int64_t batch);

/* y[B][4] (FP32) = network(x[B][32]) for B >= 0 samples; asynchronous on stream. */
int lbm_mlp_forward(const uint16_t *d_w, const uint16_t *d_x, int64_t batch, float *d_y, void *stream);

/* Gradient of the loss (1/B) sum_b sum_k (y_bk - t_bk)^2 with respect to the
 * parameters, written as FP32 [LBM_MLP_NPARAM] to d_grad (same order as the
 * weights), and the loss to d_loss[0] (FP32).  d_work: lbm_mlp_work_bytes(B)
 * bytes of device scratch.  Deterministic (fixed reduction order). */
int lbm_mlp_backward(const uint16_t *d_w, const uint16_t *d_x, const float *d_t, int64_t batch, float *d_grad,
                     float *d_loss, void *d_work, size_t work_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * gradient and loss as lbm_mlp_backward, bit for bit, with the block partials
 * in a device array that the library owns instead of a caller workspace.  The
 * array holds the partials of up to LBM_MLP_STATIC_MAX_BATCH samples (256
 * blocks x 6213 floats = 6.4 MB), one copy on each GPU the library runs on,
 * kept until the process ends.  batch > LBM_MLP_STATIC_MAX_BATCH returns
 * LBM_ERANGE; NULL pointers or batch < 0 return LBM_EINVAL.  No device memory
 * is allocated or freed.  Each call overwrites every partial it reads, so
 * nothing has to be cleared between calls, but all calls on one GPU share the
 * array: calls that overlap on one GPU (other streams, other threads) race
 * and give wrong results.  Asynchronous on stream. */
#define LBM_MLP_STATIC_MAX_BATCH 16384
int lbm_mlp_backward_static(const uint16_t *d_w, const uint16_t *d_x, const float *d_t, int64_t batch,
                            float *d_grad, float *d_loss, void *stream);

/* One Adam step on FP32 master weights (Kingma & Ba): m = b1 m + (1-b1) g,
 * v = b2 v + (1-b2) g^2, w -= lr mhat / (sqrt(vhat) + eps) with bias correction
 * at step >= 1; the fp16 copy d_w16 is refreshed (round to nearest even). */
int lbm_mlp_adam(float *d_master, float *d_m, float *d_v, const float *d_grad, uint16_t *d_w16, int64_t step,
                 float lr, float beta1, float beta2, float eps, void *stream);

/* Install network weights (device fp16 array) into the handle; required before
 * lbm_step when curv_mode is LBM_CURV_MLP.  Asynchronous on the handle's stream. */
int lbm_set_mlp(lbm_handle *h, const uint16_t *d_w);

/* Training samples from the handle's current phi: every interface cell
 * (0.02 < phi < 0.98), in site order, gives the input row 2 phi - 1 on its 3^3
 * stencil and the label of the nearest sphere (by | |x - c| - |R| |, periodic):
 * K = -2/R for a phi = 1 sphere (R > 0), +2/R for a phi = 0 sphere (R < 0),
 * normal = radial unit vector toward phi = 1.  centers [nb][3] (x, y, z) and
 * radii [nb] are HOST arrays, nb <= LBM_MLP_MAX_SPHERES.  At most cap rows are
 * written to d_x [cap][32] (fp16) and d_y [cap][4] (FP32); *n_out (host) gets
 * the total count.  Waits for the stream. */
int lbm_harvest(lbm_handle *h, const double *centers, const double *radii, int nb, uint16_t *d_x, float *d_y,
                int64_t cap, int64_t *n_out);

/* ------------------------------------------------------------------ batches
 * Many independent boxes advanced together: one persistent kernel launch per
 * time step takes work items (box, xy tile, z chunk) from a queue, so boxes of
 * uneven size share the GPU without one launch each; steps are replayed from
 * a captured HIP graph.  Not in the paper (its runs are one box per job); it
 * is the ensemble mode of this library.  A box advanced in a batch gives
 * bit-identical fields to the same box advanced alone with lbm_step.
 *
 * Members are lbm_handle's created with lbm_init; they must share storage,
 * phi_storage, ac_rk3, two_phase, curv_mode, the presence of a body force and
 * whether buoyancy or a viscosity contrast is on, and be on the same
 * stream (the first member's).  They must outlive the batch.  A member may
 * still be stepped, read or reduced on its own; the batch picks up its state
 * at the next lbm_batch_step. */
#define LBM_BATCH_MAX 4096
typedef struct lbm_batch lbm_batch;

/* Device bytes of the batch tables for n members (0 if n is out of range). */
size_t lbm_batch_bytes(int n);

/* Create a batch of n members (1 <= n <= LBM_BATCH_MAX).  d_table: caller's
 * device buffer of table_bytes >= lbm_batch_bytes(n), 256-byte aligned, owned
 * by the caller and used by the batch until lbm_batch_destroy.  Errors:
 * LBM_EINVAL (n, NULL or repeated member, mixed storage / phi storage /
 * integrator / two_phase / curv_mode / forcing / buoyancy or viscosity
 * contrast / stream), LBM_ENOSPACE, LBM_EHIP. */
int lbm_batch_create(lbm_batch **out, lbm_handle *const *members, int n, void *d_table, size_t table_bytes);

/* Advance every member by nsteps (>= 0), asynchronously on the members' stream.
 * Pairs of steps replay a captured graph of two launches.  LBM_ESTATE if an
 * MLP member has no weights. */
int lbm_batch_step(lbm_batch *b, int64_t nsteps);

/* Autotuner of the work decomposition: time steps_per_candidate (>= 1) steps,
 * after one warm-up step, for each workgroup tile (64 x 4 or 32 x 8 sites:
 * one or two x-rows per wave) and z-chunk length in {8, 16, 32, 64}, and keep
 * the fastest, cached per set of member shapes for the life of the process (a
 * cached set is not timed again).  The timed steps advance the members like
 * lbm_batch_step; results do not depend on the decomposition.  Waits for the
 * stream.  *tile_out and *zchunk_out (host, may be NULL) get the choice. */
int lbm_batch_tune(lbm_batch *b, int steps_per_candidate, int *tile_out, int *zchunk_out);

/* Set the work decomposition by hand: tile 64 (64 x 4 sites) or 32 (32 x 8),
 * z-chunk length >= 1 (clamped to each member's nz).  Takes effect at the next
 * lbm_batch_step.  LBM_EINVAL for other values. */
int lbm_batch_set_tiling(lbm_batch *b, int tile, int zchunk);

/* Free the host-side batch (not the members, not d_table). */
int lbm_batch_destroy(lbm_batch *b);

/* Text of the latest failure on b, or of the latest failed lbm_batch_create
 * when b is NULL. */
const char *lbm_batch_last_error(const lbm_batch *b);

/* Static text for an error code. */
const char *lbm_strerror(int code);

/* Text of the latest failure on h (empty string when none). */
const char *lbm_last_error(const lbm_handle *h);

#ifdef __cplusplus
}
#endif
#endif
