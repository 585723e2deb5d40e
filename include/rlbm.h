/*
 * rlbm.h -- C ABI of the MI355X (gfx950) library for the fully dissipative
 * two-dimensional ultra-relativistic lattice Boltzmann method on the d2v72
 * lattice (Coelho, Mendoza, Doria, Herrmann, arXiv:1709.09073).
 *
 * Problem statement (Sec. 2 and Sec. 3 of the paper): given initial macroscopic
 * fields per cell -- particle density n or fugacity z, temperature theta and
 * velocity u -- a statistic (Maxwell-Juttner, Fermi-Dirac or Bose-Einstein), a
 * relaxation time (constant, or tau = tau_a/theta + tau_b as in Sec. 3.2 and
 * Sec. 3.5) and boundary rules, evolve the populations by the discrete
 * Anderson-Witting equation (Sec. 2.1) with bilinear pull streaming (Sec. 2.4)
 * and report n, eps (P = eps/2), theta, z, u and the heat flux q (Eqs.
 * density-eq, theta-eq, n-eps-eq, heat-eq2).
 *
 * Conventions
 *  - Populations f_q, q = 6*n + k with direction n = 0..11 (angle n*pi/6; the
 *    paper's label i = n + 1) and radial shell k = 0..5; cell c = y*nx + x at
 *    integer coordinates (x, y).  A buffer holds 12 direction blocks of P = nx*ny
 *    cells; inside block n the six shells of a cell form 16-byte records: FP32
 *    (float) shells 0..3 at byte 16*c, shells 4..5 at 16*P + 8*c; FP64 (double)
 *    shells 2j, 2j+1 at 16*j*P + 16*c (j = 0, 1, 2).  72*nx*ny elements per buffer.
 *    RLBM_DEV16 buffers hold 192*nx*ny bytes (layout at enum rlbm_precision).
 *  - The stored state is the post-collision population.  One step is: pull
 *    streaming, moments N^mu and T^{mu nu}, Landau frame (Eq. eigen-eq), density
 *    (Eq. density-eq), inversion to (theta, z), relaxation time, fifth-order
 *    equilibrium (Eq. expansion-eq), relaxation; fixed-temperature wall cells
 *    are then set to f^eq(n_nb, theta_wall, u_nb) with n and u taken from the
 *    first fluid cell (Sec. 3.3).
 *  - Field arrays are double, nx*ny elements, row-major [y][x].
 *  - Ownership: the caller allocates every population and field buffer in
 *    device memory and keeps it alive until rlbm_free.  The library allocates
 *    only small per-context device memory (status word, two counters, and for a
 *    batch its descriptor tables) plus the captured graphs; the network calls use
 *    a workspace the caller provides.  No pointer passed in is freed by the
 *    library.
 *  - Errors: every int-returning call returns RLBM_OK (0) or a negative code;
 *    rlbm_strerror gives its text.  No C++ exception crosses this interface.
 *    Domain failures found inside kernels (non-positive n or eps, |u| >= 1,
 *    a Bose-Einstein state beyond the condensation bound, an inversion outside
 *    its table range, a solve that did not converge) set bits of a device
 *    status word, reported as RLBM_EDOMAIN by the next rlbm_sync or
 *    rlbm_moments (which then clear it); rlbm_status returns the bits.
 *  - Streams: all work is enqueued on the stream given in rlbm_params
 *    (a hipStream_t, NULL for the default stream) and is asynchronous except
 *    rlbm_sync, rlbm_status and rlbm_moments (which synchronises).
 */
#ifndef RLBM_H
#define RLBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum rlbm_status_code {
    RLBM_OK = 0,
    RLBM_EINVAL = -1,     /* bad argument: shape, order, statistic, precision, tau, boundary */
    RLBM_EDOMAIN = -2,    /* a kernel flagged a state outside the method's domain */
    RLBM_EHIP = -3,       /* a HIP runtime call failed */
    RLBM_ENONFINITE = -4, /* a kernel produced a non-finite field */
    RLBM_ENOTIMPL = -5    /* valid request the library does not implement */
};

enum rlbm_stats { RLBM_MJ = 0, RLBM_FD = 1, RLBM_BE = 2 };         /* Eqs. mj-w-eq, fd-w-eq, be-w-eq */
/* Population storage.  RLBM_DEV16 (project extension): per cell the deviations
 * e_i = (f_i / w_k - R_i) / s_k as SNORM16 (q = round(32767 e), |e| <= 1), with
 * R_{k,n} = rho_k + p_k (alpha cos phi_n + beta sin phi_n) (direction average of f/w per
 * shell plus a least-squares p-weighted dipole) and one scale per shell,
 * s_k >= max_n |f_{k,n} / w_k - R_{k,n}| (an IEEE half, rounded up).  A buffer holds 12
 * direction blocks, each nx*ny cells (y-major, x fastest) of 6 SNORM16 (shells k = 0..5,
 * 12 bytes), then nx*ny cells of 48 bytes: floats rho_0..rho_5, alpha, beta, halves
 * s_0..s_5, 4 bytes of padding: 192 bytes per cell.  Decoding is f_i = w_k (R_i +
 * s_k q_i / 32767).  The codes are taken against the least-squares rho, alpha, beta; the
 * stored rho_k, alpha, beta are then corrected so that the decoded populations keep
 * the cell's shell sums and momentum density T^{0x}, T^{0y} (Sec. 2.4 moments) to
 * rounding.  Arithmetic as RLBM_FP32. */
enum rlbm_precision { RLBM_FP64 = 0, RLBM_FP32 = 1, RLBM_DEV16 = 2 };
enum rlbm_tau_mode { RLBM_TAU_CONST = 0, RLBM_TAU_INV_THETA = 1 };  /* tau, or tau_a/theta + tau_b */
enum rlbm_bc {
    RLBM_BC_PERIODIC = 0, /* wrap (both sides of an axis must be periodic) */
    RLBM_BC_OPEN = 1,     /* zero gradient: a pull from outside takes the nearest edge cell */
    RLBM_BC_WALL_T = 2,   /* fixed-temperature wall cell on the edge column (x sides only) */
    RLBM_BC_WALL_NEQ = 3  /* wall node on the edge row (y sides only, Sec. 3.4): equilibrium of
                             (wall_n, wall_theta, u = 0) plus the post-collision non-equilibrium
                             part f* - f^eq of the nearest fluid row */
};
enum rlbm_guess { RLBM_GUESS_FIXED = 0, RLBM_GUESS_MLP = 1 };       /* FD/BE inversion start */

/* status-word bits (rlbm_status) */
#define RLBM_FLAG_NONPOSITIVE  0x1u  /* n <= 0 or eps <= 0 */
#define RLBM_FLAG_SUPERLUMINAL 0x2u  /* |u| >= 1 */
#define RLBM_FLAG_CONDENSED    0x4u  /* BE: 2n^3/(pi eps^2) >= h(z_c); z clamped to z_c */
#define RLBM_FLAG_RANGE        0x8u  /* FD: ln z above the table range (12.125) */
#define RLBM_FLAG_NOCONV       0x10u /* Landau or inversion iteration hit its limit */
#define RLBM_FLAG_NONFINITE    0x20u /* a non-finite moment (NaN or infinite population) */
#define RLBM_FLAG_UNSTABLE     0x40u /* init: tau <= gamma (1 + |u|) / 2 in some cell, where the largest
                                        Anderson-Witting weight gamma (1 - v.u) / tau reaches 2 */

typedef struct rlbm_params {
    int32_t nx, ny;          /* grid size, both >= 2 (walls need nx >= 4) */
    int32_t stats;           /* rlbm_stats */
    int32_t order;           /* expansion order N of Eq. expansion-eq: 5 for every statistic; 2, 3, 4
                                for Maxwell-Juttner with FP64/FP32 populations on single grids */
    int32_t precision;       /* rlbm_precision: element type of f_a, f_b */
    int32_t tau_mode;        /* rlbm_tau_mode */
    double tau;              /* constant relaxation time, > 0.5 (see rlbm_init for the per-cell bound) */
    double tau_a, tau_b;     /* tau = tau_a / theta + tau_b (Sec. 3.2: 4 eta/s, 0.2546) */
    int32_t bc[4];           /* sides x-low, x-high, y-low, y-high: rlbm_bc */
    double theta_wall[2];    /* wall temperature of the x-low and x-high sides */
    int32_t guess;           /* rlbm_guess */
    const float *mlp;        /* device pointer to the MLP weights (RLBM_GUESS_MLP), else NULL */
    void *f_a, *f_b;         /* device population buffers (ping-pong), 72*nx*ny elements each
                                (DEV16: 192*nx*ny bytes each, 16-byte aligned) */
    void *stream;            /* hipStream_t, NULL = default stream */
    int32_t tile_x, tile_y;  /* cells per workgroup tile, tile_x * tile_y = 256 with tile_x a power
                                of two >= 16; 0, 0 = automatic (32 x 8; 128 x 2 when nx >= 4096;
                                64 x 4 or 128 x 2 for ny < 8, 4) */
    int32_t collect_stats;   /* 1: count Newton iterations of the FD/BE inversion (rlbm_inversion_stats) */
    double force[2];         /* constant acceleration (a_x, a_y) applied by momentum update: the
                                collision uses u + a tau (Sec. 3.4); 0, 0 = none */
    double wall_n, wall_theta; /* imposed density and temperature of RLBM_BC_WALL_NEQ sides */
    int32_t check;           /* 1: check mode, every rlbm_step call waits for its steps and returns
                                the status word's verdict (RLBM_ENONFINITE, RLBM_EDOMAIN); 0: asynchronous */
} rlbm_params;

typedef struct rlbm_init_fields {
    /* device pointers, nx*ny doubles each.  Either n (given_z = 0) or z (given_z = 1). */
    const double *n, *z, *theta, *ux, *uy;
    int32_t given_z;
} rlbm_init_fields;

typedef struct rlbm_out_fields {
    /* device pointers, nx*ny doubles each; a NULL entry is not written */
    double *n, *eps, *theta, *z, *ux, *uy, *qx, *qy;
    /* optional raw moments of the same populations (Sec. 2.4, Eq. density-eq): the particle
       current N^mu = sum_i f_i p_i^mu and the energy-momentum tensor T^{mu nu} =
       sum_i f_i p_i^mu p_i^nu (symmetric, traceless: T^00 = T^xx + T^yy) */
    double *N0, *Nx, *Ny, *T00, *T0x, *T0y, *Txx, *Txy, *Tyy;
} rlbm_out_fields;

typedef struct rlbm_ctx rlbm_ctx;

/* Validate p, build a context and write the initial state f* = f^eq(fields)
 * into f_a: the equilibrium of Eq. expansion-eq on the quadrature of Sec. 2.4; for
 * FD/BE with n given, z solves n = 2 pi theta^2 g_2(z) (Eq. n-eps-eq).  Synchronises
 * the stream.  On success *ctx owns a status word; on failure *ctx is NULL.
 * Errors: RLBM_EINVAL (bad parameters, or a cell where tau <= gamma (1 + |u|)/2: the
 * Anderson-Witting weight gamma (1 - v.u)/tau of Sec. 2.1 would reach 2 there, an
 * over-relaxation the update does not survive), RLBM_EHIP.  Domain flags raised while
 * building the state (e.g. a BE density above condensation) stay in the status word. */
int rlbm_init(rlbm_ctx **ctx, const rlbm_params *p, const rlbm_init_fields *init);

/* Several independent grids of uneven sizes in one context (project extension for
 * the transport sweeps of Sec. 3.2 and Sec. 3.3): p[g] and init[g] for
 * g < ngrids, each with its own shape, relaxation time, boundaries and buffers;
 * stats, precision, order, guess, mlp, stream, tile and collect_stats must agree.
 * Every step advances all grids with one launch over all their tiles (one
 * workgroup per tile, or a persistent sweep: rlbm_configure, rlbm_autotune).
 * Intended for transport-coefficient sweeps.  Errors as rlbm_init. */
int rlbm_init_batch(rlbm_ctx **ctx, int32_t ngrids, const rlbm_params *p, const rlbm_init_fields *init);

/* Enqueue nsteps >= 0 time steps (ping-pong between f_a and f_b of every grid).  A
 * step is the discrete Anderson-Witting update of Sec. 2.1 with the pull streaming of
 * Sec. 2.4: moments, Landau frame (Eq. eigen-eq), density (Eq. density-eq), inversion
 * (Eqs. theta-eq, n-eps-eq, gz-eq), relaxation time (Sec. 3.2), equilibrium (Eq.
 * expansion-eq), relaxation; the order is spelled out at the top of this file.
 * Runs of 64 or more steps replay captured graphs of 32 steps (one graph launch
 * per 32 steps).  Asynchronous, except in check mode (rlbm_params.check = 1), where
 * the call waits for its steps and returns as rlbm_sync.  Errors: RLBM_EINVAL (nsteps
 * < 0 or ctx NULL), RLBM_EHIP; in check mode also RLBM_ENONFINITE, RLBM_EDOMAIN. */
int rlbm_step(rlbm_ctx *ctx, int64_t nsteps);

/* Capture the 32-step graphs that rlbm_step replays (for both parities) now, so
 * that a later timed run does not include capture and instantiation.  Runs no step.
 * (Project extension: scheduling of the update of Sec. 2.1, not part of the method.) */
int rlbm_capture(rlbm_ctx *ctx);

/* (Project extension; scheduling only, results do not depend on it: every shape and
 * mode gives the same bits.)
 * Set the workgroup tile (tile_x * tile_y = 256, tile_x a power of two >= 16) and,
 * for a batch, the launch mode: persistent > 0 launches that many workgroups per
 * XCD, each sweeping tiles of its XCD's range; 0 launches one workgroup per tile.
 * The tile also selects the pull of FP32 and 16-bit populations at order 5 without
 * forcing: tiles whose (tile_x + 2)(tile_y + 2) halo has at most 512 cells (32x8, 64x4,
 * 16x16) read each direction's halo once into LDS, the others (128x2, 256x1) read the
 * taps directly.  Drops captured graphs.  Errors: RLBM_EINVAL, RLBM_EHIP. */
int rlbm_configure(rlbm_ctx *ctx, int32_t tile_x, int32_t tile_y, int32_t persistent);

/* (Project extension; scheduling only.)
 * Time trial_steps steps with each workgroup tile shape in {32x8, 64x4, 16x16,
 * 128x2, 256x1} (one workgroup per tile) and, for a batch, also 32x8 and 64x4 with
 * 96 persistent workgroups per XCD, in three rounds (one warm-up step before each
 * timing); keep the shape with the fastest round and return it.  The trial steps
 * (3 x candidates x (trial_steps + 1)) are real steps of the simulation (they
 * advance the state and the step count); the inversion counters restart from zero
 * after the trials.  Synchronises the stream. */
int rlbm_autotune(rlbm_ctx *ctx, int32_t trial_steps, int32_t *tile_x, int32_t *tile_y);

/* rlbm_moments for grid g of a batch (g = 0 for a single grid). */
int rlbm_moments_grid(rlbm_ctx *ctx, int32_t g, const rlbm_out_fields *out);

/* Fields of the current state (moments of the pre-collision populations the next
 * step would see), written to the non-NULL device arrays of out: n (Eq. density-eq),
 * eps and u (Eq. eigen-eq), theta and z (Eqs. theta-eq, n-eps-eq), q (Eq. heat-eq2),
 * and the raw moments N^mu, T^{mu nu} (Sec. 2.4).  Synchronises the stream.  Returns
 * as rlbm_sync (the status word includes what this call's own kernel raised). */
int rlbm_moments(rlbm_ctx *ctx, const rlbm_out_fields *out);

/* Diagonal x components of the non-equilibrium tensors of ranks 2 to 5 (Eq.
 * tensors-eq, Sec. 3.1), pi^{x..x} = sum_i (f_i - f^eq_i) (p_i^x)^r, of grid g's current state:
 * f are the pre-collision populations the next step would see and f^eq the
 * equilibrium of the expansion order in use at the cell's own (theta, z, u).
 * Outputs are device arrays of nx*ny doubles (y-major); a NULL one is skipped.
 * Synchronises the stream; errors as rlbm_moments. */
int rlbm_noneq_tensors(rlbm_ctx *ctx, int32_t g, double *pi_xx, double *pi_xxx, double *pi_xxxx,
                       double *pi_xxxxx);

/* 0 if f_a holds the current state, 1 if f_b does (the stored state is the
 * post-collision population of Sec. 2.1's update). */
int rlbm_state_index(const rlbm_ctx *ctx);

/* Number of steps taken since rlbm_init. */
int64_t rlbm_steps_done(const rlbm_ctx *ctx);

/* Wait for the stream and report the status word, then clear it: RLBM_ENONFINITE if
 * RLBM_FLAG_NONFINITE is set, else RLBM_EDOMAIN if any bit is set, else RLBM_OK. */
int rlbm_sync(rlbm_ctx *ctx);

/* Wait for the stream and return the status-word bits without clearing them. */
uint32_t rlbm_status(rlbm_ctx *ctx);

/* Newton iterations and solves of the FD/BE (n, eps) -> (theta, z) inversion (Eqs.
 * n-eps-eq, gz-eq) summed over all step launches since rlbm_init or since the last
 * rlbm_autotune (collect_stats = 1; otherwise zeros).  Synchronises the stream.
 * Errors: RLBM_EINVAL, RLBM_EHIP. */
int rlbm_inversion_stats(rlbm_ctx *ctx, uint64_t *iterations, uint64_t *solves);

/* Training pairs from the current state, one per cell (FP32 device arrays of
 * nx*ny): x = ln r with r = 2 n^3 / (pi eps^2), t = ln z (the one-dimensional form of
 * Eq. n-eps-eq, theta cancelling), from the same moments, Landau frame and inversion
 * as rlbm_moments.  Synchronises the stream; returns as rlbm_sync. */
int rlbm_inversion_samples(rlbm_ctx *ctx, float *x, float *t);

/* ---- the inversion-guess network (project extension, not in the paper) -------
 * One hidden layer of RLBM_MLP_HIDDEN ReLU units maps L = ln r to mu = ln z; it
 * supplies the starting point of the safeguarded Newton solve, which still
 * decides the result.  Weight buffer: RLBM_MLP_FLOATS floats in device memory,
 * layout [a, b, m, s, W1[H], b1[H], W2[H], b2] with x = (L - a) b and
 * mu = m + s (b2 + sum_h W2_h max(W1_h x + b1_h, 0)).  The loss is the mean over
 * samples of (y - (t - m)/s)^2.  All arrays are caller-owned device memory;
 * calls are asynchronous on `stream` (hipStream_t, NULL = default). */
#define RLBM_MLP_HIDDEN 32
#define RLBM_MLP_FLOATS (4 + 3 * RLBM_MLP_HIDDEN + 1)
#define RLBM_MLP_NTRAIN (3 * RLBM_MLP_HIDDEN + 1)

/* Bytes of device workspace the training calls need for n samples. */
uint64_t rlbm_mlp_workspace_bytes(int64_t n);

/* Initialise w from the data (n >= 2): a, b map [min x, max x] to [-1, 1]; m, s are
 * the mean and standard deviation of t; hidden unit h gets W1 = 1 and its kink at
 * x = -1 + 2(h + 1/2)/H; W2 and b2 are noise[0..H] * 0.1 (noise: H + 1 caller-drawn
 * standard normals, device floats).  Errors: RLBM_EINVAL, RLBM_EHIP. */
int rlbm_mlp_init(float *w, const float *x, const float *t, int64_t n, const float *noise, void *workspace,
                  void *stream);

/* Full-batch loss and its gradient with respect to the RLBM_MLP_NTRAIN trainable
 * parameters (order W1, b1, W2, b2), summed in a fixed order (deterministic).
 * grad and loss are device floats. */
int rlbm_mlp_loss_grad(const float *w, const float *x, const float *t, int64_t n, float *grad, float *loss,
                       void *workspace, void *stream);

/* iters steps of Adam (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the
 * full batch, updating the trainable part of w in place.  loss_out (device, may be
 * NULL) receives the loss before each step (iters floats). */
int rlbm_mlp_train(float *w, const float *x, const float *t, int64_t n, int32_t iters, float lr,
                   float *loss_out, void *workspace, void *stream);

/* Allocation-free rlbm_mlp_train for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * kernels and arithmetic (bit-identical results), with the workspace taken from a
 * library-owned device array of rlbm_mlp_workspace_bytes(RLBM_MLP_NOALLOC_MAX) bytes
 * (about 13 MB), one per GPU, held until the process ends.  n must be in
 * 1 .. RLBM_MLP_NOALLOC_MAX, else RLBM_EINVAL; RLBM_EHIP if the array's address
 * cannot be obtained.  Allocates nothing.  Every call on one GPU uses that GPU's array:
 * calls that overlap on one GPU (other streams or threads) race and must be ordered
 * by the caller.  Enqueued on `stream`; the moments of Adam are cleared by a kernel,
 * not a memset, so the launches may be captured into a graph. */
#define RLBM_MLP_NOALLOC_MAX 32768
int rlbm_mlp_train_noalloc(float *w, const float *x, const float *t, int64_t n, int32_t iters, float lr,
                           float *loss_out, void *stream);

/* y[i] = network(x[i]) for n inputs (device floats). */
int rlbm_mlp_predict(const float *w, const float *x, float *y, int64_t n, void *stream);

/* Release the context (not the caller's buffers).  NULL is a no-op. */
void rlbm_free(rlbm_ctx *ctx);

/* Text of a status code. */
const char *rlbm_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* RLBM_H */
