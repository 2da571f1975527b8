/*
 * evlbm.h -- C ABI of the MI355X (gfx950) Enskog-Vlasov lattice Boltzmann
 * library.  It implements the explicit lattice Boltzmann model of
 * Karlin & Hosseini, "Practical Kinetic Models for Dense Fluids"
 * (arXiv 2508.00577): the update eq. pre_LBM with the half-step fields of
 * eq. u_shift / T_shift, the Enskog-gauge force of eq. EVforce1 under
 * eq. P0E, the product equilibria eq. feq / f_star / geq / gstar with the
 * corrections eq. correction_u / correction_gamma / correction_q, on the
 * D3Q27 velocity set (text before eq. phi) and its z-summed D2Q9 form.
 *
 * Conventions
 *   - Every call returns an int: EVLBM_OK (0) or a negative error code;
 *     evlbm_last_error() gives a message for the calling thread.
 *   - Lattice units: dt = dx = 1, particle mass 1 (rho = n).
 *   - Fields are SoA with x fastest: scalar[nz][ny][nx], vector[D][nz][ny][nx],
 *     populations [Q][nz][ny][nx] (f) followed by the same for g.
 *     Velocity index i = (cx+1) + 3 (cy+1) + 9 (cz+1) on D3Q27 and
 *     i = (cx+1) + 3 (cy+1) on D2Q9, c in {-1,0,1}.
 *   - `where` selects host FP64 arrays or device arrays (FP32/FP64) on the
 *     handle's device; the caller owns every buffer it passes and keeps it
 *     alive for the duration of the call.  Host reads block until the data
 *     is on the host; everything else is enqueued on the handle's stream.
 *   - A handle is not thread-safe; separate handles are independent.
 *   - The lattice is periodic; evlbm_set_walls puts diffuse walls normal to x.
 */
#ifndef EVLBM_H
#define EVLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    EVLBM_OK = 0,
    EVLBM_EINVAL = -1,      /* invalid argument */
    EVLBM_ENOMEM = -2,      /* device or host allocation failed */
    EVLBM_EHIP = -3,        /* a HIP runtime call failed */
    EVLBM_ESTATE = -4,      /* call not valid in the handle's state */
    EVLBM_ENONFINITE = -5,  /* a non-finite density was found */
    EVLBM_EIO = -6,         /* file I/O failed */
    EVLBM_ENONPHYS = -7     /* rho <= 0, b rho >= 1 or T <= 0 in an input */
};

enum { EVLBM_D2Q9 = 2, EVLBM_D3Q27 = 3 };

/* Population storage.  F16DEV/BF16DEV store the scaled deviation
 * h_i(x) = (f_i(x) - f^ref_i(x))/s_i(x) in 16 bits (round to nearest even) and
 * decode to FP32 for the arithmetic: f^ref, g^ref are the equilibria at rest
 * (eq. feq, eq. geq with u = 0) of a per-cell reference state (rho_ref,
 * theta_ref), s = f^ref for f and theta_ref/(1 - theta_ref) f^ref for g.
 * The reference state is set from the initial fields and, on a lattice,
 * refreshed from the stored state of every cell every EVLBM_OPT_REREF_EVERY
 * steps (default 100).
 * F16DEV keeps the density within 1e-3 of FP32 storage and of the FP64 oracle.
 * BF16DEV (8-bit significand) is experimental: it misses that bar in 3D
 * (about 1.3e-3 after 1e4 steps at 128^3, 3e-3 against the oracle after 1000
 * steps on a small droplet). */
enum { EVLBM_F64 = 0, EVLBM_F32 = 1, EVLBM_F16DEV = 2, EVLBM_BF16DEV = 3 };

enum { EVLBM_HOST_F64 = 0, EVLBM_DEVICE_F32 = 1, EVLBM_DEVICE_F64 = 2 };

enum {
    EVLBM_OPT_SPHI = 1,        /* sign in front of the first term of eq. correction_u (default -1) */
    EVLBM_OPT_CHECK_EVERY = 4, /* scan for non-finite densities every K steps (0 = never) */
    EVLBM_OPT_USE_GRAPH = 5,   /* 1: replay step chunks from a captured hipGraph (default 1) */
    EVLBM_OPT_REREF_EVERY = 6, /* 16-bit storage: re-reference every K steps (0 = never; default 100) */
    EVLBM_OPT_EOS = 8,         /* contact factor of Enskog's pressure: EVLBM_EOS_VDW (default) or EVLBM_EOS_CS */
    EVLBM_OPT_PRANDTL = 9,     /* Prandtl number Pr > 0 (default 1, the paper's scheme; the concluding paragraph
                                  names a quasi-equilibrium relaxation of g for other values, the scheme is this
                                  library's): g relaxes with tau_g = tau/Pr in both terms of eq. pre_LBM and keeps
                                  f's relaxation for its viscous-heating flux u . Pi^neq (Pi^neq = sum c c
                                  (fh - f^eq)) through a zero-mass, zero-energy term on the axis directions; then
                                  k = (5/2) R mu/Pr. */
    EVLBM_OPT_PUSH_MOMENTS = 7 /* 1 = one-pass step (default), 0 = two-pass step, where the moments are pulled
                                  again before each collision.  D3Q27 with FP32 or FP64 storage: the collision
                                  pushes the next moments (16-bit D3Q27 storage is always two-pass).  D2Q9:
                                  the collision sums its tile's halo moments from the pulled populations;
                                  the result is bit for bit the two-pass step's */
};

/* Enskog's pressure P_E = rho R T (1 + b rho chi) with the contact value chi
 * of the pair distribution (the text after eq. Ework): VDW chi = 1/(1 - b rho),
 * i.e. P_E = rho R T/(1 - b rho), the paper's form; CS the Carnahan-Starling
 * hard-sphere value chi = (1 - eta/2)/(1 - eta)^3 with eta = b rho/4.  Under
 * the gauge P0 = P_E (eq. P0E) the closure enters theta = P0/rho and gamma_0
 * of eq. gamma. */
enum { EVLBM_EOS_VDW = 0, EVLBM_EOS_CS = 1 };

enum { EVLBM_MEASURE_SLAB = 1, EVLBM_MEASURE_DROPLET = 2 };

typedef struct evlbm_lattice *evlbm_t;

/* Message of the last failed call on this thread (never NULL). */
const char *evlbm_last_error(void);

/* Create a periodic lattice of N = nx*ny*nz cells (D2Q9 needs nz == 1) with
 * the given storage, bound to `stream` (a hipStream_t; NULL = default stream)
 * on the current device.  Allocates two population buffers of 2Q direction
 * arrays each (N values, consecutive arrays 1280 bytes apart beyond their
 * size), a moment field and, for 16-bit storage, the per-cell reference
 * state.  Parameters start at R = 1, a = b = kappa = 0, tau = lambda = 1.
 * Errors: EINVAL (unknown lattice or storage, sizes <= 0, nz != 1 for D2Q9,
 * N*8 + 1280 >= 2^32 for FP64 storage or N*4 + 1280 >= 2^32 otherwise: the
 * kernels address each per-direction array with 32-bit byte offsets),
 * ENOMEM, EHIP. */
int evlbm_create(int lattice, int nx, int ny, int nz, int storage, void *stream, evlbm_t *out);

/* Release every resource of the handle; NULL is accepted. */
int evlbm_destroy(evlbm_t h);

/* Equation of state: Enskog pressure P_E = rho R T/(1 - b rho) (or the
 * Carnahan-Starling form, EVLBM_OPT_EOS), mean-field pressure P_V = -a rho^2
 * and capillarity kappa (eq. EVforce1 and the text after it).
 * a = b = kappa = 0 is the ideal gas.
 * Errors: EINVAL if R <= 0 or a, b, kappa < 0. */
int evlbm_set_eos(evlbm_t h, double R, double a, double b, double kappa);

/* Relaxation: bare time tau (beta = dt/(2 tau + dt), eq. beta) and the shifted-
 * equilibrium time lambda.  Errors: EINVAL if tau <= 0, lambda <= 0 or
 * tau > lambda (negative effective relaxation time, eq. final_kinetic_model2). */
int evlbm_set_relaxation(evlbm_t h, double tau, double lambda);

/* Set an EVLBM_OPT_* option.  Errors: EINVAL (unknown key or bad value). */
int evlbm_set_option(evlbm_t h, int key, double value);

/* Initialise f = f^eq(rho, u, P0/rho) and g = g^eq(u, RT) cell by cell from
 * rho[N], u[D*N] (may be NULL: at rest) and T[N]; resets the step count.
 * With 16-bit storage the per-cell reference state is taken from rho and T.
 * Errors: EINVAL (bad where), ENONPHYS (rho <= 0, b rho >= 1 or T <= 0),
 * ENONFINITE, EHIP. */
int evlbm_init_fields(evlbm_t h, const void *rho, const void *u, const void *T, int where);

/* Advance nsteps time steps on the handle's stream (asynchronous unless the
 * non-finite scan is enabled).  Errors: ESTATE (not initialised), ENONFINITE
 * (scan), EHIP. */
int evlbm_step(evlbm_t h, int64_t nsteps);

/* Steps taken since the last initialisation. */
int evlbm_step_count(evlbm_t h, int64_t *out);

/* Moments of the current state (pull, raw moments, force and half-step
 * fields, eq. u_shift and eq. T_shift): rho[N], u[D*N], T[N] (any may be
 * NULL).  Errors: ESTATE, EINVAL, EHIP. */
int evlbm_read_moments(evlbm_t h, void *rho, void *u, void *T, int where);

/* FP64 global sums of the current state: out[0] = sum rho (every cell's
 * decoded pulled populations summed in FP64: the stored mass), out[1..3] =
 * sum rho u, out[4] = sum rho E, out[5] = sum [rho E - a rho^2 +
 * (kappa/2)|grad rho|^2], out[6] = max |u|, out[7] = min of the streamed f.
 * Blocks.  Errors: ESTATE, EHIP. */
int evlbm_global_sums(evlbm_t h, double out[8]);

/* The global sums of evlbm_global_sums written to device memory without any
 * allocation, for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): out_dev[8]
 * (device FP64, caller owned) receives the same values as evlbm_global_sums,
 * enqueued on the handle's stream (no synchronisation).  The reduction's
 * partials live in a fixed device array of the library (4 MiB per GPU, held
 * until the process ends), so lattices of at most 2^24 cells are accepted.
 * Calls that overlap on one GPU share that array and race: order them (one
 * stream, or events).  Call with the lattice's device current.
 * Errors: EINVAL (null argument, more than 2^24 cells, another device
 * current), ESTATE, EHIP. */
int evlbm_global_sums_noalloc(evlbm_t h, double *out_dev);

/* FP64 region means for the coexistence (Fig. 1) and Laplace checks.
 * SLAB: geom = {xl0, xl1, xv0, xv1, xv2, xv3}: liquid x in [xl0, xl1),
 *   vapour x in [xv0, xv1) U [xv2, xv3) (all y, z).
 * DROPLET: geom = {cx, cy, cz, r_in, r_out}: inside r < r_in, outside r > r_out.
 * out = {rho_in, rho_out, T_in, T_out, P_in, P_out, R_e, cells_in}
 * with P_in, P_out the region means of the cell pressures
 * P = rho R T Z(rho) - a rho^2 of the lattice's pressure closure (van der
 * Waals Z = 1/(1 - b rho), or Carnahan-Starling; EVLBM_OPT_EOS) and, for
 * droplets, the equimolar radius R_e from sum (rho - rho_out)/(rho_in -
 * rho_out) (2D: area, 3D: volume).  Blocks.  Errors: EINVAL, ESTATE, EHIP. */
int evlbm_measure(evlbm_t h, int kind, const double *geom, double out[8]);

/* Copy the stored populations out (decoded) or in (encoded): f[Q*N], g[Q*N]
 * dense, [Q][nz][ny][nx] each, FP64 on the host (HOST_F64) or the device
 * (DEVICE_F64).  With 16-bit storage, set_populations also takes the per-cell
 * reference state from the values it is given.  Blocks.  Errors: EINVAL (null
 * pointer, other `where`), ENOMEM, EHIP. */
int evlbm_get_populations(evlbm_t h, void *f, void *g, int where);
int evlbm_set_populations(evlbm_t h, const void *f, const void *g, int where);

/* Bit-exact dump of the stored populations, dense [2Q][N], after a one-line
 * JSON header (format evlbm-5: lattice, storage, sizes, parameters incl. the pressure closure, Prandtl number and walls, step,
 * byte counts), followed for 16-bit storage by the per-cell reference state
 * as four FP32 values per cell, and for the one-pass D3Q27 step by the
 * moment field rho, j, e ([D+2][N] in the arithmetic precision), which that
 * step carries from one step to the next.  Load restores all of it into a
 * handle of the same lattice, sizes and storage, so the run resumes bit for
 * bit.  Errors: EIO (open, read, write, bad header, wrong byte count),
 * EINVAL (null argument, different lattice). */
int evlbm_checkpoint_save(evlbm_t h, const char *path);
int evlbm_checkpoint_load(evlbm_t h, const char *path);

/* Time the two kernels of a step with HIP events on the handle's stream:
 * runs nsteps real steps (launched one by one, no graph) and returns the
 * average durations in milliseconds: out[1] = stencil + collision kernel,
 * out[0] = the other kernel of the step: the pulled-moment kernel of the
 * two-pass step, or the fix-up of the pushed moments of the one-pass D3Q27
 * step (EVLBM_OPT_PUSH_MOMENTS); 0 for the one-pass D2Q9 step.  Blocks.
 * Errors: EINVAL (nsteps outside 1..4096), ESTATE, EHIP. */
int evlbm_profile_step(evlbm_t h, int nsteps, double out[2]);

/* Wait for all work enqueued on the handle's stream. */
int evlbm_synchronize(evlbm_t h);

/* Size of one population buffer (A or B) in bytes, and its direction stride
 * in elements: a buffer holds 2Q direction arrays (f then g, velocity index i
 * = (cx+1) + 3(cy+1) + 9(cz+1)) of N cells each, x fastest, consecutive
 * arrays `stride` elements apart (N plus a pad that keeps the arrays off
 * each other's HBM channels), elements of the storage's type (8, 4 or 2
 * bytes; 16-bit storage holds scaled deviations from the per-cell reference
 * state).  stride is nullable.  Errors: EINVAL (null handle or bytes). */
int evlbm_population_bytes(evlbm_t h, size_t *bytes, long *stride);

/* Let the lattice keep its populations in caller-owned device memory (e.g.
 * two torch tensors): a and b (distinct, non-overlapping, 256-byte aligned,
 * at least evlbm_population_bytes bytes each, on the lattice's device)
 * replace the library's two buffers.  The current state is copied into them
 * (the call blocks on the handle's stream), the library's own buffers are
 * freed, and captured step graphs are rebuilt.  The caller keeps a and b
 * alive until evlbm_destroy, which does not free them.  Errors: EINVAL
 * (null, too small, misaligned, overlapping or non-device buffers), EHIP. */
int evlbm_attach_buffers(evlbm_t h, void *a, void *b, size_t bytes);

/* Diffuse walls normal to x for the thermal Couette flow (the paragraph after
 * eq. P0E, Fig. 2): a wall at rest half a cell before the first cell
 * (x = -1/2) and one moving with U_wall along y half a cell after the last
 * (x = nx - 1/2), both at temperature T_wall; y and z stay periodic.  The
 * paper gives the wall values only; the scheme: a population entering a cell
 * from a wall is the wall's equilibrium (eq. feq, eq. geq at the wall's
 * velocity, R T_wall and theta = R T_wall Z(rho) at the cell's stored
 * density) times the density that makes it carry the mass the cell's
 * populations send into the wall in the same step (diffuse reflection:
 * mass conserving); the finite-difference stencils take a field beyond a wall
 * as the linear extrapolation through the two cells next to it.  enable = 0
 * restores the periodic lattice.  FP64 and FP32 storage.  With walls the step
 * takes four plain launches (pull with the walls, Laplacian, fields,
 * collision); evlbm_read_moments, evlbm_global_sums and the checkpoints follow
 * the walls; evlbm_measure and evlbm_profile_step return EINVAL.
 * Errors: EINVAL (16-bit storage, nx < 2, T_wall <= 0, U_wall not finite),
 * ENOMEM (work buffers: 2Q + 3D + 2 values per cell). */
int evlbm_set_walls(evlbm_t h, int enable, double T_wall, double U_wall);

/* Liquid-vapour coexistence of the bulk pressure P = P_E - a rho^2 of closure
 * `eos` (EVLBM_EOS_*) at temperature T: out = {rho_l, rho_v, P_coex} (equal
 * pressure and chemical potential, Newton iteration).  Used for the initial
 * profiles.  Errors: EINVAL if eos is unknown, a or b <= 0, or T is not below
 * T_c (evlbm_eos_critical). */
int evlbm_eos_coexistence(int eos, double R, double a, double b, double T, double out[3]);

/* Critical point of the bulk pressure P = P_E - a rho^2 of closure `eos`:
 * out = {rho_c, T_c, P_c}.  van der Waals: 1/(3b), 8a/(27 b R), a/(27 b^2);
 * Carnahan-Starling: eta_c = b rho_c/4 solves s'(eta) = eta s''(eta) for
 * s = 4 eta Z(eta) (bisection), R T_c = 32 a/(b s''(eta_c)).
 * Errors: EINVAL if eos is unknown or a, b <= 0. */
int evlbm_eos_critical(int eos, double R, double a, double b, double out[3]);

/* Attainable HBM bandwidth: a plain device-to-device streaming copy of
 * `bytes` total traffic (half read, half written), timed over `reps` launches
 * with HIP events on the default stream.  Context for the roofline figures
 * and the reference for byte-counter calibration.  Blocks.
 * Errors: EINVAL, ENOMEM, EHIP. */
int evlbm_copy_probe(double bytes, int reps, double *gbps_out);

/* ------------------------------------------------------------------------
 * Batched D2Q9 domains (a sweep over many uneven periodic domains sharing the
 * EOS and relaxation parameters, e.g. a T/Tc sweep).  All domains advance
 * together: each step is one persistent launch of the one-pass stencil +
 * collision kernel over the tiles of every domain (the collision sums its
 * tile's halo moments from the pulled populations; a moment kernel runs for
 * readouts only), replayed from captured hipGraphs.  A domain of the batch
 * evolves bit for bit as the same domain stepped alone as a lattice of the
 * same storage.
 * ------------------------------------------------------------------------ */
typedef struct evlbm_batch *evlbm_batch_t;
typedef struct {
    int nx, ny;
} evlbm_domain_desc;

/* Create a batch of n domains (sizes d[k]) with the given storage on
 * `stream` (a hipStream_t).  Errors: EINVAL, ENOMEM. */
int evlbm_batch_create(int n, const evlbm_domain_desc *d, int storage, void *stream, evlbm_batch_t *out);
int evlbm_batch_destroy(evlbm_batch_t b);

/* Shared parameters (as evlbm_set_eos, evlbm_set_relaxation, EVLBM_OPT_SPHI). */
int evlbm_batch_set_params(evlbm_batch_t b, double R, double a, double bexcl, double kappa, double tau,
                           double lambda, double sphi);

/* Batch options: EVLBM_OPT_SPHI, EVLBM_OPT_REREF_EVERY, EVLBM_OPT_EOS and
 * EVLBM_OPT_PRANDTL, as on a lattice, shared by every domain.  Errors: EINVAL
 * (other keys, bad values). */
int evlbm_batch_set_option(evlbm_batch_t b, int key, double value);

/* Initialise domain k from host FP64 fields rho[N_k], u[2 N_k] (nullable), T[N_k].
 * With 16-bit storage the domain's per-cell reference state is taken from
 * these fields and refreshed every 100 steps of the batch, as on a lattice.
 * Errors: EINVAL, ENONPHYS, ENONFINITE. */
int evlbm_batch_init_domain(evlbm_batch_t b, int k, const double *rho, const double *u, const double *T);

/* Advance every domain nsteps.  Errors: ESTATE (a domain not initialised). */
int evlbm_batch_step(evlbm_batch_t b, int64_t nsteps);

/* Moments (rho, u[2 N_k], T) of domain k into host FP64 arrays; blocks. */
int evlbm_batch_read(evlbm_batch_t b, int k, double *rho, double *u, double *T);

/* Decoded populations f[9 N_k], g[9 N_k] of domain k (host FP64); blocks. */
int evlbm_batch_get_populations(evlbm_batch_t b, int k, double *f, double *g);

/* Tile shape of the persistent kernels: 0 = 64x4, 1 = 64x16 (a single lattice's D2Q9 tile), 2 = 128x2, 3 = 64x8. */
int evlbm_batch_set_tile(evlbm_batch_t b, int variant);

/* Time `steps` steps with each tile shape on the current state (restored
 * afterwards), select the fastest; best and ms_per_step[4] (nullable) out. */
int evlbm_batch_autotune(evlbm_batch_t b, int steps, int *best, double *ms_per_step);

/* Total cells, tiles of the current shape, the shape index and its size. */
int evlbm_batch_info(evlbm_batch_t b, int64_t *cells, int *ntiles, int *variant, int *tile_x, int *tile_y);

/* ------------------------------------------------------------------------
 * Warm-start network: (T/Tc, R, r/R) -> 3 x 64 tanh hidden layers -> rho/rho_c,
 * FP32 parameters in the flat layout W1[64][3], b1[64], W2[64][64], b2[64],
 * W3[64][64], b3[64], W4[64], b4 (8641 values); inputs normalised as
 * x1 = (T/Tc - 0.8)/0.15, x2 = (R - 47.5)/32.5, x3 = r/R - 1.  Trained on
 * the GPU (mean squared error, Adam with beta1 0.9, beta2 0.999, eps 1e-8) on
 * droplet profiles the solver itself produces; used to seed new droplets.
 * Host arrays: X[n][3], Y[n].
 * ------------------------------------------------------------------------ */
typedef struct evlbm_mlp *evlbm_mlp_t;

enum { EVLBM_PROFILE_TANH = 0, EVLBM_PROFILE_MLP = 1 };

int evlbm_mlp_create(void *stream, evlbm_mlp_t *out);
int evlbm_mlp_destroy(evlbm_mlp_t m);
int evlbm_mlp_num_params(void);
/* Set or read the parameters (n must be 8641); set resets the Adam state. */
int evlbm_mlp_set_params(evlbm_mlp_t m, const float *params, int n);
int evlbm_mlp_get_params(evlbm_mlp_t m, float *params, int n);
/* Outputs Y[n] for inputs X[n][3]; blocks. */
int evlbm_mlp_forward(evlbm_mlp_t m, const float *X, float *Y, int n);
/* Gradient of the mean squared error (grad[8641], nullable) and the loss
 * (nullable) at the current parameters; blocks. */
int evlbm_mlp_grad(evlbm_mlp_t m, const float *X, const float *Y, int n, float *grad, float *loss);
/* iters full-batch Adam steps with learning rate lr; loss_hist[iters]
 * (nullable) receives the loss before each step; blocks.  The network's
 * trusted (T/Tc, R) box grows to cover the training inputs. */
int evlbm_mlp_train(evlbm_mlp_t m, const float *X, const float *Y, int n, int iters, float lr, float *loss_hist);
/* The (T/Tc, R) box the network is trusted on, [tr_lo, tr_hi] x [r_lo, r_hi]:
 * empty for a new network, the training inputs' box after evlbm_mlp_train;
 * set it for parameters trained elsewhere.  get: out = {tr_lo, tr_hi, r_lo,
 * r_hi}.  Errors: EINVAL (null handle, lo > hi). */
int evlbm_mlp_set_hull(evlbm_mlp_t m, double tr_lo, double tr_hi, double r_lo, double r_hi);
int evlbm_mlp_get_hull(evlbm_mlp_t m, double out[4]);
/* Device FP64 density field rho_c * y(T/Tc, R, min(|x - c|/R, 3)) of a
 * lattice of nx*ny*nz cells (nz = 1: 2D distance), enqueued on the network's
 * stream.  Beyond r/R = 3, the radial range of the training profiles (r/R in
 * [0, 3]) and of evlbm_init_droplet's checks, the field keeps its value at 3. */
int evlbm_mlp_density_field(evlbm_mlp_t m, int nx, int ny, int nz, double cx, double cy, double cz, double R,
                            double Tr, double rho_c, double *rho_dev);

/* ------------------------------------------------------------------------
 * Initialisers of the workloads' synthetic states.  Each builds FP64 density
 * and temperature fields on the device and calls evlbm_init_fields (f = f^eq,
 * g = g^eq at rest, eq. feq and eq. geq).  Densities come from the handle's
 * pressure closure: the coexistence densities rho_l, rho_v at T = Tr T_c
 * (evlbm_eos_coexistence, evlbm_eos_critical), so a > 0 and b > 0 are needed.
 * Seeded noise is multiplicative on the density, rho <- rho (1 + noise
 * (2 u_c - 1)), with u_c the splitmix64 output (Steele, Lea & Flood, OOPSLA
 * 2014) number c + 1 of the stream `seed`, c the cell's linear index
 * x + nx (y + ny z), taken as a double in [0, 1) from its top 53 bits; noise 0
 * adds none.  Synchronous.  Errors: EINVAL (bad geometry, Tr outside (0, 1),
 * noise outside [0, 1), no two phases), ENOMEM, ENONPHYS, EHIP.
 * ------------------------------------------------------------------------ */

/* Flat liquid slab between x0 and x1 along x, uniform in y and z:
 * rho = rho_v + (rho_l - rho_v)/2 [tanh((x - x0)/width) - tanh((x - x1)/width)],
 * T = Tr T_c, at rest (the flat-interface workload of Fig. 1). */
int evlbm_init_slab(evlbm_t h, double x0, double x1, double Tr, double width, uint64_t seed, double noise);

/* Droplet of radius R centred at (cx, cy, cz) at T/Tc = Tr, at rest:
 * TANH = (rho_l + rho_v)/2 - (rho_l - rho_v)/2 tanh((r - R)/width); MLP = the
 * network's profile, falling back to TANH when (Tr, R) lies outside the
 * network's trusted box (evlbm_mlp_set_hull; compared in FP32, the network's
 * input precision) or the radial profile on r/R in [0, 3] is non-finite,
 * increasing in r or outside [0.5 rho_v, 1.2 rho_l].
 * *used_mlp (nullable) tells which was used. */
int evlbm_init_droplet(evlbm_t h, double cx, double cy, double cz, double R, double Tr, int profile, evlbm_mlp_t mlp,
                       double width, uint64_t seed, double noise, int *used_mlp);

/* The droplet of evlbm_init_droplet carrying a given total mass and total
 * energy (global sums 0 and 5 of another state, e.g. the plain run it is to
 * meet: a periodic lattice conserves both, so two runs can only reach the
 * same state from equal values).  The density profile is scaled to `mass`,
 * and the uniform temperature T is found by Newton steps from Tr T_c with the
 * slope d(sum 5)/dT = (3/2) R mass of a state at rest, until the energy agrees
 * to 1e-13 relative (at most 8 steps); *T_used (nullable) receives it.
 * Errors as above, ENONPHYS if the temperature comes out <= 0. */
int evlbm_init_droplet_matched(evlbm_t h, double cx, double cy, double cz, double R, double Tr, int profile,
                               evlbm_mlp_t mlp, double width, uint64_t seed, double noise, double mass,
                               double energy, int *used_mlp, double *T_used);

/* Build information: the library, its target, lattices and storages,
 * "evlbm gfx950 D2Q9/D3Q27 F64/F32/F16DEV/BF16DEV" (static string). */
const char *evlbm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EVLBM_H */
