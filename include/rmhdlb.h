/*
 * rmhdlb.h -- C ABI of the MI355X (gfx950) lattice Boltzmann solver for
 * resistive relativistic magnetohydrodynamics (Mohseni, Mendoza, Succi,
 * Herrmann, arXiv:1508.03452, Sec. III).
 *
 * One time step per cell: transport of the post-collision fluid
 * distributions f (D3Q19, energy-momentum) and g (D3Q19, number) with
 * minmod-limited fluxes and the bulk-viscosity term (Eq. rlb), streaming of
 * the D3Q13 Maxwell distributions h (Eq. LB_Maxwell), the moments (Eqs.
 * Cal_E, Cal_B, Cal_rhoc), the Landau-frame recovery of eps, u, n, p
 * (Sec. III, "Coupling between fluid and electromagnetic fields"), the
 * force-corrected E with the Ohm current (Eqs. Ex_force, Ohm), and the
 * collisions towards f_eq (Eq. Dis_fun_EM), g_eq (Eq. Hupp) and h_eq
 * (Eq. Maxwell-eq).  All of it runs in one fused kernel per step.
 *
 * Conventions for every entry point:
 *  - Return value: RMHDLB_OK (0) or a negative error code; no exception
 *    crosses the ABI.  rmhdlb_strerror() names a code.
 *  - Arrays: contiguous FP64, nx*ny*nz values, x fastest, then y, then z.
 *    Field pointers are DEVICE pointers on the context's device unless an
 *    entry point says otherwise.  Inputs are borrowed for the call only.
 *  - Units: the paper's numerical units with mu0 = 1 by default; dt is fixed
 *    by dx/dt = sqrt(2) c (Sec. III, end of the coupling subsection).
 *  - Streams: all work is queued on the HIP stream given to rmhdlb_create
 *    (NULL = the default stream).  Only rmhdlb_moments and the state copy
 *    calls synchronise (that stream).
 *  - A context is used by one host thread at a time; contexts are
 *    independent.
 */
#ifndef RMHDLB_H
#define RMHDLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RMHDLB_OK = 0,
    RMHDLB_EINVAL = -1,      /* invalid argument or parameter */
    RMHDLB_ENOMEM = -2,      /* device allocation failed */
    RMHDLB_EDEVICE = -3,     /* HIP runtime or launch error */
    RMHDLB_ERECOVERY = -4,   /* primitive recovery failed in some cell (state holds NaN there) */
    RMHDLB_EUNSUPPORTED = -5, /* parameter value outside what the method supports */
    RMHDLB_ESTATE = -6,       /* call out of order: no state yet (rmhdlb_init_fields or rmhdlb_set_state
                                 not called), or instances of a batch at different time levels */
    RMHDLB_ELIMIT = -7        /* size beyond the fixed device memory of a no-allocation entry point */
};

/* Face types.  Periodic pairs both faces of an axis.  Open: the ghosts are
 * copies of the first interior cell along the face normal (Sec. IV, Alfven
 * test), and with divb_fix the normal B of a face cell is adjusted so that
 * div B vanishes there (Sec. IV, KH set-up).  Driven (low face of z only,
 * the high z face then open): two ghost planes below z = 0 hold the fixed
 * post-collision state of prescribed face fields (rmhdlb_set_driven_face),
 * an equilibrium boundary of this library's own (not in the paper). */
enum { RMHDLB_BC_PERIODIC = 0, RMHDLB_BC_OPEN = 1, RMHDLB_BC_DRIVEN = 2 };

/* Storage of the state between steps.  F64 is the plain path.  F32 and F16
 * store f and g as deviations from w_i E_ref and w'_i N_ref (references: the
 * means of eps and n over the initial fields), h in the same type and E_prev
 * in FP32; the step then runs in FP32 arithmetic with the recovery and the
 * Ohm solve in FP64.  rmhdlb_get_state / set_state always use the FP64,
 * unshifted layout. */
enum { RMHDLB_STORE_F64 = 0, RMHDLB_STORE_F32 = 1, RMHDLB_STORE_F16 = 2 };

typedef struct {
    int32_t nx, ny, nz;          /* cells per axis, each >= 1 */
    int32_t bc_lo[3], bc_hi[3];  /* face types per axis (periodic on both faces or open on both) */
    double dx;                   /* cell size (> 0) */
    double c;                    /* light speed (> 0); dt = dx / (sqrt(2) c) */
    double mu0;                  /* permeability (> 0); eps0 = 1 / (mu0 c^2) */
    double tau;                  /* fluid relaxation time in units of dt (> 0; the paper uses 1) */
    double tau_h;                /* Maxwell relaxation time; only 1/2 is supported (Eq. Ex_force) */
    double alpha;                /* bulk-viscosity constant, lambda_i = alpha dx (>= 0; the paper uses 0.1) */
    double Gamma;                /* adiabatic index of p = (Gamma - 1)(eps - n c^2), Eq. EOS (> 1) */
    double sigma;                /* conductivity of Eq. Ohm (>= 0) */
    double nu;                   /* lattice nu = c / c_s (> 0); sqrt(27) makes every g weight positive */
    int32_t storage;             /* RMHDLB_STORE_* */
    int32_t divb_fix;            /* 1: adjust the normal B on open faces so div B = 0 there; 0: off
                                    (recommended: in runs of ~10^3 steps at sigma = 1e3 the adjustment
                                    grew B at face edges until cells failed: a 256 x 512 KH slab at
                                    step 1200, the flare box by step 900) */
    int32_t null_band;           /* reconnection-rate null search: rows with |y| <= null_band cells
                                    (cell centres y_j = j + 1/2 - ny/2); < 1 selects 64 */
    int32_t collision;           /* RMHDLB_COLL_*: the f collision (see below) */
    int32_t flux;                /* RMHDLB_FLUX_*: the face values of the transport (see below) */
    int32_t b_prev;              /* RMHDLB_BPREV_*: the B of the recovery and of f_eq (see below) */
    int32_t reserved[2];         /* must be zero */
    void *workspace;             /* optional caller-owned DEVICE buffer that holds every buffer the context
                                    needs (state, scratch, partial sums): at least rmhdlb_workspace_bytes
                                    bytes, 256-byte aligned, on the current device, untouched by the caller
                                    until rmhdlb_destroy.  NULL: rmhdlb_create allocates it (hipMalloc). */
    size_t workspace_bytes;      /* size of *workspace (ignored when workspace is NULL) */
} rmhdlb_params;

/* Which magnetic field enters the recovery's fluid tensor T_fl = T - T_EM(E, B)
 * and the T_EM part of f_eq (Sec. III, coupling subsection, which names the
 * fields of the previous time step).  E is always the previous step's (the
 * current one needs the velocity, through Eq. Ohm).  CURRENT (default): B of
 * this step, a moment of the streamed h (Eq. Cal_B) known before the
 * recovery; with it the Alfven speed is exact for every tau.  PREVIOUS: the
 * previous step's B as the paper words it; the state then also carries B_prev
 * (69 instead of 66 arrays).  PREVIOUS lags the field inertia by a step,
 * which grows a mode in strongly magnetised states (B^2 of the order of
 * eps + p); it is built for 64-wide tiles with the default collision and
 * faces, without the learned guess, a force or batches
 * (RMHDLB_EUNSUPPORTED). */
enum { RMHDLB_BPREV_CURRENT = 0, RMHDLB_BPREV_PREVIOUS = 1 };

/* The face value h_i^a of the transport in Eq. rlb, which the paper takes
 * from a reference it cites: the upwind value along the link of population i
 * plus a minmod-limited slope term.  MUSCL (default): slope weight 1/2.
 * LAX_WENDROFF: weight (1 - C)/2 with C the Courant number along a link,
 * the limited Lax-Wendroff form, which translates quadratic profiles exactly
 * where the limiter keeps the upwind-side slope.  Like the printed collision
 * it is built for 64-wide tiles without the learned guess or batches. */
enum { RMHDLB_FLUX_MUSCL = 0, RMHDLB_FLUX_LAX_WENDROFF = 1 };

/* The f collision of Eq. rlb.  EXPLICIT (default): f' = f - omega (f - f_eq)
 * on the transported f, which conserves T^{0 nu} exactly in every cell.
 * PRINTED: the form the paper prints, with f(t + dt) in the collision term,
 * in closed form f' = (f + omega f_eq) / (1 + omega); it is not exactly
 * conservative (the rate depends on the direction) but stays stable in
 * supersonic shear flows where the explicit form fails (the paper's KH runs
 * at U0 = 0.4c and 0.6c).  PRINTED is built for 64-wide tiles without the
 * learned guess: rmhdlb_set_guess(.., RMHDLB_GUESS_MLP) and batches with it
 * return RMHDLB_EUNSUPPORTED, rmhdlb_set_tuning with px != 64 RMHDLB_EINVAL. */
enum { RMHDLB_COLL_EXPLICIT = 0, RMHDLB_COLL_PRINTED = 1 };

/* Initial primitive fields (Sec. IV): number density n, pressure p,
 * velocity u, electric field E, magnetic field B, charge density rho_c
 * (rho_c may be NULL: then eps0 div E by central differences, Eq. Gauss_E). */
typedef struct {
    const double *n, *p;
    const double *u[3], *E[3], *B[3];
    const double *rho_c;
} rmhdlb_fields_in;

/* Primitive fields of the current state; any pointer may be NULL. */
typedef struct {
    double *n, *p, *eps;
    double *u[3], *E[3], *B[3], *J[3];
    double *rho_c;
} rmhdlb_fields_out;

/* Global diagnostics of the current state (sums over cells, FP64, in a
 * fixed order: per-block trees, then the blocks in order). */
typedef struct {
    double energy;       /* sum of T^00 (fluid + field, the moment of f) */
    double mass;         /* sum of N^0 */
    double momentum[3];  /* sum of T^0a */
    double em_energy;    /* sum of eps0 (E^2 + c^2 B^2) / 2 */
    double max_divB;     /* max over cells of |div B|: central differences, one-sided on the faces of
                            non-periodic axes */
    double charge;       /* sum of rho_c (Eq. Cal_rhoc) */
    double mean_iters;   /* mean Newton iterations of the recovery */
    double recon_rate;   /* R = (E^z - E^z_0) / B0 at the null point (Sec. IV, KH reconnection): the
                            null is the cell of least B_x^2 + B_y^2 in the null_band rows (first cell in
                            x-fastest order on ties), E^z_0 its initial E^z, B0 = max |B| of the
                            initial fields; NaN when B0 = 0 */
    double B0;           /* max |B| of the initial fields */
    int64_t null_index;  /* linear cell index of the null point (-1: none) */
    int64_t newton_hist[16]; /* cells by Newton iterations of the recovery (last bin: 15 or more) */
    int64_t n_failed;    /* cells whose recovery failed */
    int64_t n_fallback;  /* cells whose learned guess was rejected (Newton started from T_fl^00) */
    int64_t step;        /* steps taken since rmhdlb_init_fields */
    int64_t guess_steps; /* of those, steps that ran the learned guess's network (see rmhdlb_set_guess) */
} rmhdlb_diag;

/* Prescribed fields of a driven face: nx*ny DEVICE values each, x fastest. */
typedef struct {
    const double *n, *p;
    const double *u[3], *B[3];
} rmhdlb_face_in;

typedef struct rmhdlb_ctx rmhdlb_ctx; /* opaque, owned by the library */

/* Bytes of device memory a context with these parameters needs for its two
 * state buffers, scratch and partial sums: the size of params->workspace
 * (256-byte alignment included).  The learned guess's tables and an external
 * force, when set later, take memory of their own.  0 for invalid params. */
size_t rmhdlb_workspace_bytes(const rmhdlb_params *params);

/* Create a solver.  Validates *params (RMHDLB_EINVAL, also for a workspace
 * smaller than rmhdlb_workspace_bytes or not 256-byte aligned, and for a grid
 * of 2^30 cells or more, since cell indices are 32-bit; tau_h != 1/2
 * gives RMHDLB_EUNSUPPORTED), takes its device memory from params->workspace
 * or allocates it on the current HIP device (RMHDLB_ENOMEM), clears it on
 * `hip_stream` (a hipStream_t, may be NULL) and keeps that stream.  On
 * success *out uses the memory until rmhdlb_destroy (and frees it there if it
 * allocated it); on failure *out is NULL and nothing stays allocated. */
int rmhdlb_create(const rmhdlb_params *params, void *hip_stream, rmhdlb_ctx **out);

/* Set the state from primitive fields (device pointers, see rmhdlb_fields_in).
 * The stored state is post-collision: f and g are the equilibria of the given
 * fields (f_eq of Eq. Dis_fun_EM, g_eq of Eq. Hupp), the Maxwell
 * populations are laid out so that the first streaming delivers h_eq of
 * (J0, E0 + (dt/2) mu0 c^2 J0, B0) with J0 from Eq. Ohm, and the rest
 * population holds rho_c.  Returns RMHDLB_EINVAL for NULL pointers; physically
 * invalid inputs (|u| >= c, n <= 0, p < 0) surface as failed cells at the
 * next rmhdlb_moments.  Resets the step counter. */
int rmhdlb_init_fields(rmhdlb_ctx *ctx, const rmhdlb_fields_in *in);

/* Queue nsteps >= 0 fused time steps on the context's stream and return
 * without waiting.  Only launch errors are reported here (RMHDLB_EDEVICE);
 * recovery failures are deferred to rmhdlb_moments.  RMHDLB_ESTATE before the
 * first rmhdlb_init_fields or rmhdlb_set_state (also from rmhdlb_moments,
 * rmhdlb_get_state, rmhdlb_autotune and the guess training calls). */
int rmhdlb_step(rmhdlb_ctx *ctx, int64_t nsteps);

/* Primitive fields of the current state (what the next step computes first:
 * transport, moments, recovery, E and J), written to the non-NULL device
 * pointers of *out, and the global diagnostics written to *diag (host
 * memory).  Either may be NULL.  Synchronises the stream.  Returns
 * RMHDLB_ERECOVERY when some cell failed its recovery (its primitives are
 * NaN; diag->n_failed counts them). */
int rmhdlb_moments(rmhdlb_ctx *ctx, rmhdlb_fields_out *out, rmhdlb_diag *diag);

/* Driven low-z face (bc_lo[2] = RMHDLB_BC_DRIVEN): set the fields whose
 * relaxed state fills the two ghost planes below z = 0.  Each ghost cell
 * holds f_eq and g_eq of (n, p, u, E = -u x B, B) and h* = h_eq of (J, E +
 * (dt/2) mu0 c^2 J, B) with J of Eq. Ohm at zero charge, and E_prev = E;
 * the step never writes them.  rmhdlb_init_fields fills them from the
 * z = 0 plane of its fields; call this afterwards to prescribe others (the
 * state and the step counter are kept).  Returns RMHDLB_EINVAL, with the
 * ghost planes unchanged, for a context without a driven face, NULL
 * pointers, or any face cell with |u| >= c, n <= 0 or p < 0 (checked on the
 * device; this call synchronises the stream). */
int rmhdlb_set_driven_face(rmhdlb_ctx *ctx, const rmhdlb_face_in *face);

/* External force density (the flare driver of Sec. IV, stellar flare; the
 * paper gives no lattice form, this library's reading): F[a] are device
 * arrays of N = nx ny nz FP64 values in cell order (x fastest), copied on the
 * context's stream; NULL switches the force off.  Each step adds, after the
 * collision, c dt F^a to the momentum T^{0a} of a cell through its moving f
 * populations, (19/9) w_i (e_i . c dt F) / kappa each (no change of T^00 or
 * T^ab from these), and the work c dt F . beta to T^00 through the rest
 * population, with beta of that step's recovery.  The force acts while the
 * largest |beta| of the previous step's recovery over the box is below gate
 * (gate <= 0: always); the gate opens again at rmhdlb_init_fields.  Built for
 * 64-wide tiles with MUSCL faces and either collision: RMHDLB_EUNSUPPORTED
 * with the Lax-Wendroff faces or the learned guess on, and batches with a
 * forced instance refuse to step.  RMHDLB_EINVAL for NULL
 * entries or a non-finite gate, RMHDLB_ENOMEM if the buffers cannot be
 * allocated. */
int rmhdlb_set_force(rmhdlb_ctx *ctx, const double *const F[3], double gate);

/* ---- learned recovery guess (not in the paper) ----------------------------
 * The recovery (Sec. III, coupling subsection) finds the timelike eigenpair
 * of the fluid tensor; this library solves it by Newton on the secular
 * equation from lambda = T_fl^00.  A 6 -> 32 -> 32 -> 2 perceptron (tanh
 * hidden layers) can seed that Newton iteration instead: from six rotation
 * and scale invariants of the cell's fluid tensor (|S|/E_f, S^.Pi S^/E_f,
 * tr Pi/E_f, |Pi S^ - (S^.Pi S^) S^|/E_f, |Pi|_F/E_f, N^0/E_f with E_f =
 * T_fl^00, S = T_fl^0a, Pi = T_fl^ab, S^ = S/|S|), normalised, it predicts
 * (lambda/E_f, |beta|) normalised.  Cells with |S|/E_f <= 0.02 take no
 * guess (Newton from E_f needs one or two steps there), and a wavefront of
 * only such cells skips the network.  The guess is used when it lies below
 * E_f with Pi + lambda I positive definite and phi' > 0 there (and predicted
 * |beta| < 0.999); otherwise Newton starts from E_f (a fallback).  Newton
 * then converges to the same root, so the guess changes iteration counts,
 * not results.  Inference runs inside the step on MFMA (FP16 weights and
 * inputs, FP32 accumulation), 32 cells per wavefront. */
enum { RMHDLB_GUESS_PLAIN = 0, RMHDLB_GUESS_MLP = 1 };
#define RMHDLB_GUESS_PARAMS 1346 /* W1 (32 x 6), b1, W2 (32 x 32), b2, W3 (2 x 32), b3, row-major */

typedef struct {
    float w[RMHDLB_GUESS_PARAMS];
    float mu_x[6], sd_x[6]; /* input normalisation x = (f - mu_x) / sd_x */
    float mu_t[2], sd_t[2]; /* outputs: t = mu_t + sd_t y */
} rmhdlb_guess_weights;

typedef struct {
    int32_t n_samples; /* cells sampled from the current state: cell floor(i N / n_samples), 128 <= n_samples <= N */
    int32_t iters;     /* Adam iterations (>= 0) */
    int32_t batch;     /* minibatch size: a multiple of 128, <= n_samples */
    int32_t stride;    /* minibatch b takes samples (b batch + i) stride mod n_samples (>= 1) */
    float lr;          /* Adam learning rate (> 0; beta1 0.9, beta2 0.999, eps 1e-8) */
    int32_t reserved[3]; /* must be zero */
} rmhdlb_train_opts;

/* Train the guess on the GPU from cells of the current state: their features
 * and, as targets, (lambda / E_f, |beta|) of the plain recovery; normalise
 * with the sample mean and standard deviation (floor 1e-6); minibatch Adam
 * from init_w (host, RMHDLB_GUESS_PARAMS values: the library draws no random
 * numbers) on the mean squared error / 2 of the normalised outputs.  Installs
 * the result (see rmhdlb_set_guess) and returns it in *out and the loss of
 * every iteration in losses (host, iters values); both may be NULL.  Returns
 * RMHDLB_ERECOVERY if a sampled cell fails its recovery.  Synchronises. */
int rmhdlb_train_guess(rmhdlb_ctx *ctx, const rmhdlb_train_opts *opts, const float *init_w,
                       rmhdlb_guess_weights *out, float *losses);

/* Install guess weights (host struct) for the context's steps and moments. */
int rmhdlb_set_guess_weights(rmhdlb_ctx *ctx, const rmhdlb_guess_weights *w);

/* RMHDLB_GUESS_PLAIN (default) or RMHDLB_GUESS_MLP (needs installed
 * weights, else RMHDLB_EINVAL).  Applies to later steps and moments.  With
 * the guess a cell whose flow ratio |S| / T_fl^00 is at most 0.1 still starts
 * Newton from T_fl^00, and a step runs the network only while the step before
 * it met a cell above that ratio (enabling the guess, rmhdlb_init_fields and
 * rmhdlb_set_state open this gate for the next step); the other steps run the
 * plain recovery in a kernel that carries none of the network's registers.
 * rmhdlb_diag.guess_steps counts the steps that ran the network. */
int rmhdlb_set_guess(rmhdlb_ctx *ctx, int32_t mode);

/* The training samples of rmhdlb_train_guess without training: features
 * F (DEVICE, n_samples x 6) and targets T (DEVICE, n_samples x 2) of cells
 * floor(i N / n_samples) of the current state.  Synchronises. */
int rmhdlb_guess_samples(rmhdlb_ctx *ctx, int32_t n_samples, double *F, double *T);

/* The same samples with no device allocation, for callers that cannot allocate
 * (code in tight training or serving loops, harnesses that forbid hipMalloc):
 * the per-block partial sums of the sampling pass live in a fixed array of the
 * library, one per device, of 17 * RMHDLB_NOALLOC_MAX_SAMPLES / 256 doubles
 * (544 KiB), which every device the library is loaded on holds until the process ends.  The
 * caller still passes F and T.  Every call on a device shares that device's
 * array: calls that overlap on one device (from other host threads or on
 * other streams) race and must be serialised by the caller; each call writes
 * every partial sum it reads, so nothing carries over from an earlier call.
 * Results are those of rmhdlb_guess_samples, bit for bit.  RMHDLB_ELIMIT for
 * n_samples > RMHDLB_NOALLOC_MAX_SAMPLES, other errors as rmhdlb_guess_samples.
 * Synchronises. */
#define RMHDLB_NOALLOC_MAX_SAMPLES (1 << 20)
int rmhdlb_guess_samples_noalloc(rmhdlb_ctx *ctx, int32_t n_samples, double *F, double *T);

/* One forward and backward pass of the network on a batch: w (host,
 * RMHDLB_GUESS_PARAMS), normalised inputs X (DEVICE, n x 6) and targets Yt
 * (DEVICE, n x 2), n a multiple of 128 (<= 65536).  Writes the outputs Y
 * (DEVICE, n x 2, may be NULL), the gradient of sum (Y - Yt)^2 / (2 n) with
 * respect to w (DEVICE, RMHDLB_GUESS_PARAMS) and that loss (DEVICE, 1 value),
 * using the training kernel's MFMA arithmetic.  Queued on hip_stream and
 * synchronised. */
int rmhdlb_mlp_eval(const float *w, const float *X, const float *Yt, int32_t n, float *Y, float *grad, float *loss,
                    void *hip_stream);

/* ---- launch tuning and batched sweeps --------------------------------------
 * The fused step runs blocks of 256 threads over row groups of px x (R / px)
 * cells, px in {64, 32, 16} (128 too in batches): R = 128 with FP64
 * storage (two lanes per cell), R = 256 with FP32 and FP16 (one lane per
 * cell);
 * a block takes yw such groups stacked along y (a tile of px x (R / px) yw
 * cells) and walks zb z-planes.  With zg > 1 the planes are taken in chunks
 * of zg * zb per column, and the zg blocks of a chunk walk them interleaved
 * (block r: planes r, r + zg, ...), so that they run at neighbouring planes
 * together and share the z-neighbour planes in the L2 cache.  The shape
 * changes the order of work only: results are bitwise the same for every
 * shape. */

/* Time the launch shapes on the context's current state with HIP events and
 * keep the fastest for its later steps: every (px, zb) with zb in
 * {1, 2, 4, 8, 16} up to nz and zg = yw = 1, plus px = 64 with zb in
 * {16, 32, 64} and zg in {2, 4} where zg * zb <= nz; on a slab (nz = 1) every
 * px with yw in {1, 2, 4}.  The state is not advanced (each timed step reads
 * the current buffer and writes the other).  Results are cached per process
 * by grid size, storage, boundary kinds, guess mode, collision, flux, force
 * and previous-B reading; a cached shape is reused without timing.  With the
 * learned guess, the printed collision, the Lax-Wendroff flux, a force or the
 * previous-B reading only px = 64 is timed, and with a force only zg = yw = 1.
 * The chosen shape is returned in *px, *zb, *zg, *yw (any may be NULL).
 * Synchronises.  RMHDLB_ESTATE before the state is set. */
int rmhdlb_autotune(rmhdlb_ctx *ctx, int32_t *px, int32_t *zb, int32_t *zg, int32_t *yw);

/* Set the shape directly: px in {64, 32, 16}, zb >= 1, 1 <= zg <= 64,
 * 1 <= yw <= 8; px = 64 with the learned guess, the printed collision, the
 * Lax-Wendroff flux or the previous-B reading, and zg = yw = 1 with a force
 * (RMHDLB_EINVAL otherwise).  zb above nz acts as nz, and zg above
 * ceil(nz / zb) is reduced to it.  A force set later runs with zg = yw = 1
 * whatever the tuning. */
int rmhdlb_set_tuning(rmhdlb_ctx *ctx, int32_t px, int32_t zb, int32_t zg, int32_t yw);

/* A batch of independent instances (for example a parameter sweep) stepped
 * together: every step is one launch over the blocks of all instances (plus
 * one face-pass launch when some instance has open faces with the div B
 * adjustment), instead of one launch per instance.  On a non-NULL stream
 * two consecutive steps are captured once into a hipGraph and replayed.
 * Every instance is a full context (rmhdlb_batch_instance) for
 * init_fields, set_driven_face, moments, get/set_state; all share the
 * storage type and the stream; the learned guess is not used in batched
 * steps (RMHDLB_EUNSUPPORTED if an instance has it on).  Results are
 * bitwise those of stepping each instance alone with the same tile shape. */
typedef struct rmhdlb_batch rmhdlb_batch;

/* params: n parameter sets (n >= 1); on failure *out is NULL. */
int rmhdlb_batch_create(const rmhdlb_params *params, int32_t n, void *hip_stream, rmhdlb_batch **out);

/* Instance i (0 <= i < n) as a context owned by the batch (NULL if out of range). */
rmhdlb_ctx *rmhdlb_batch_instance(rmhdlb_batch *batch, int32_t i);

/* Queue nsteps batched steps.  Every instance must hold a state and be at
 * the same buffer parity (stepped only through the batch since init_fields),
 * else RMHDLB_ESTATE.  Steps are replayed from hipGraphs captured on the
 * batch's stream (64 steps per graph, then 2, then one eager launch); a graph
 * is captured again whenever the launch geometry changed (an instance's
 * tuning, the batch's tile shape).  In persistent mode
 * (rmhdlb_batch_set_persistent) the call is one cooperative launch instead. */
int rmhdlb_batch_step(rmhdlb_batch *batch, int64_t nsteps);

/* Time the tiles of the batched step (state not advanced) and keep the
 * fastest: px x (R / px) yw cells, R = 128 cells per row group with FP64
 * storage (two lanes per cell) and 256 with FP32 and FP16 (one lane per
 * cell), so that the shapes 64 x 4, 32 x 8, 128 x 2, 16 x 16 and 64 x 8 are
 * among them for every storage type (eight shapes in all), each with the
 * kernel compiled for 2 and (FP32 storage) 3 waves per SIMD.  Cached per process by storage and the grids
 * of the instances.  *px, *yw, *waves receive the choice (any may be NULL).
 * Synchronises.  RMHDLB_ESTATE as for rmhdlb_batch_step. */
int rmhdlb_batch_autotune(rmhdlb_batch *batch, int32_t *px, int32_t *yw, int32_t *waves);

/* Set the batch's tile directly: px in {128, 64, 32, 16}, 1 <= yw <= 8,
 * waves 2, or 3 with FP32 storage (RMHDLB_EINVAL otherwise). */
int rmhdlb_batch_set_tuning(rmhdlb_batch *batch, int32_t px, int32_t yw, int32_t waves);

/* Launch mode of rmhdlb_batch_step (Sec. III step, run over many instances).
 * on = 0 (the default): one launch per step, replayed from hipGraphs.  on = 1:
 * each call runs its nsteps steps in one cooperative launch of a persistent
 * kernel whose blocks (as many as are resident at once, a multiple of 8) take
 * the tiles of a step in turn and meet at a grid barrier before the next step;
 * the batch's tile shape and waves apply, and the states are bitwise those of
 * mode 0.  A batch with an instance that adjusts its open faces (divb_fix)
 * has no face pass in this mode: rmhdlb_batch_step returns
 * RMHDLB_EUNSUPPORTED for it (mode 0 steps it).  The launch needs all of
 * its blocks resident together, so a caller starts it with no other kernels
 * in flight on the device (synchronise first) and runs one at a time per
 * device.  RMHDLB_EINVAL for on outside {0, 1}, RMHDLB_EUNSUPPORTED when the
 * device cannot launch cooperatively; a failed launch makes
 * rmhdlb_batch_step return RMHDLB_EDEVICE. */
int rmhdlb_batch_set_persistent(rmhdlb_batch *batch, int32_t on);

/* Release the batch and its instances.  NULL is accepted. */
int rmhdlb_batch_destroy(rmhdlb_batch *batch);

/* A plain device copy of `bytes` bytes from src to dst (both DEVICE pointers
 * on the current device, 16-byte aligned, not overlapping; bytes a multiple
 * of 16, else RMHDLB_EINVAL), queued on hip_stream: one 16-byte load and
 * store per lane with non-temporal hints, the access pattern of the step's
 * streams.  Not part of the method: the achievable HBM rate the step's
 * roofline fraction is read against, and the reference that calibrates
 * traffic counters (its bytes read and written are known exactly). */
int rmhdlb_device_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

/* Release the context and its device memory.  NULL is accepted. */
int rmhdlb_destroy(rmhdlb_ctx *ctx);

/* Static text for an error code. */
const char *rmhdlb_strerror(int code);

/* Number of FP64 values of the raw state: 66 * nx*ny*nz (F[19], G[19],
 * h*[24 moving + 1 rest], E_prev[3], each nx*ny*nz values, post-collision),
 * 69 * nx*ny*nz with RMHDLB_BPREV_PREVIOUS (B_prev[3] after E_prev). */
int64_t rmhdlb_state_len(const rmhdlb_ctx *ctx);

/* Copy the raw state to / from a DEVICE buffer of rmhdlb_state_len FP64
 * values in the layout above (checkpoint and restart; FP32 storage is
 * widened or rounded).  Synchronise the stream. */
/* The ghost planes of a driven face are configuration, not state: they
 * come from rmhdlb_init_fields / rmhdlb_set_driven_face and are not copied. */
int rmhdlb_get_state(rmhdlb_ctx *ctx, double *dst);
int rmhdlb_set_state(rmhdlb_ctx *ctx, const double *src);

/* The lattice tables the library uses (host memory, no device work):
 * e19[19*3] D3Q19 unit vectors and w19[19] weights in state order; for the
 * 24 moving Maxwell populations in state order the lattice offsets
 * s24[24*3] (v_k dt / dx), ehat24[24*3] (e_k = c ehat_k / sqrt 2) and
 * bhat24[24*3] (b_k = bhat_k).  Sec. III, Eq. cellconfigs1 and the D3Q13
 * definitions. */
int rmhdlb_lattice_tables(int32_t *e19, double *w19, int32_t *s24, int32_t *ehat24, int32_t *bhat24);

#ifdef __cplusplus
}
#endif
#endif
