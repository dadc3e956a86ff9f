/*
 * ldrop.h -- C ABI of libldrop, an MI355X (gfx950) engine for the Langevin
 * nanoparticle-aggregation model of Derkachov et al., "A numerical toy model
 * of Langevin dynamics provides real-time visualization of colloidal
 * microdroplet evaporation" (arXiv:2501.04456).
 *
 * One context holds one droplet: N nanoparticles (NPs) of up to LD_MAX_TYPES
 * types in a spherical droplet whose radius R(t) follows a schedule.  Per
 * step (section 2.2, steps (ii)-(vi)) the library evaluates
 *   - pair forces over all NP pairs: Lennard-Jones truncated (not shifted) at
 *     lj_cut * sigma_ij plus Coulomb over all pairs;
 *   - external forces: the surface spring at R(t), gravity, the centrifugal
 *     force, with viscous drag as the mobility 1/gamma;
 *   - an overdamped Langevin (Euler-Maruyama) update with Gaussian Brownian
 *     noise from a counter-based Philox4x32-10 stream.
 *
 * Units are reduced: lengths in units of the type-0 diameter, energies in
 * units where kT is a parameter, charges in elementary charges.  Forces:
 *   f_LJ(i<-j) = 24 eps_ij [2 (s/r)^12 - (s/r)^6] r_ij / r^2  if r < lj_cut*s
 *   f_C (i<-j) = kT l_B q_i q_j r_ij / r^3
 * with r_ij = x_i - x_j, s = sigma_ij = (sigma_i + sigma_j)/2 and
 * eps_ij = sqrt(eps_i eps_j) (Lorentz-Berthelot) or an explicit matrix.
 *
 * Conventions shared by every call:
 *   - Every call returns an ld_status; on failure ld_last_error() describes
 *     it.  No C++ exception crosses the ABI.
 *   - Array arguments may be host or device pointers; the library asks the
 *     HIP runtime which one it got.  The caller owns every array; inputs are
 *     copied during the call and never retained.
 *   - Outputs are in the caller's original particle order.
 *   - Work is enqueued on the HIP stream given to ld_init.  ld_step returns
 *     without waiting; calls that return values to host memory wait for the
 *     stream.  A step whose move is non-finite or larger than jump_max sets a
 *     device-side flag; ld_sync reports the first such step once as
 *     LD_ENONFINITE and clears the flag (the state stays readable).
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - Pair math runs in FP32; per-particle force totals, the external forces,
 *     the update and all diagnostics in FP64.  Positions are kept as an FP32
 *     pair (hi, lo) whose sum carries about 48 significant bits.
 */
#ifndef LDROP_H
#define LDROP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LD_MAX_TYPES 8

typedef struct ld_ctx ld_ctx;
typedef int32_t ld_status;

enum {
    LD_OK = 0,
    LD_EINVAL = -1,        /* an argument is out of range (message says which) */
    LD_ENOMEM = -2,        /* device allocation failed */
    LD_EHIP = -3,          /* a HIP runtime call failed */
    LD_ENONFINITE = -4,    /* a step produced a non-finite or too large move */
    LD_ESTATE = -5,        /* call not valid in the context's current state */
    LD_EUNSUPPORTED = -6   /* feature not built for this configuration */
};

/* Physical parameters (section 2.1: per-type radius, mass, charge, freely set
 * interactions within and between types, per-type surface spring, gravity,
 * centrifugal force, Stokes viscosity, controllable Brownian motion). */
typedef struct {
    int32_t n_types;                      /* 1 .. LD_MAX_TYPES */
    int32_t use_eps_matrix;               /* 0: eps_ij = sqrt(eps_i eps_j) */
    double sigma[LD_MAX_TYPES];           /* LJ size = contact diameter (> 0) */
    double eps[LD_MAX_TYPES];             /* LJ well depth (>= 0) */
    double mass[LD_MAX_TYPES];            /* buoyancy-corrected mass */
    double gamma[LD_MAX_TYPES];           /* Stokes drag (> 0); mobility 1/gamma */
    double k_wall[LD_MAX_TYPES];          /* surface spring constant (>= 0) */
    double wall_offset[LD_MAX_TYPES];     /* spring equilibrium this far inside R */
    double eps_matrix[LD_MAX_TYPES * LD_MAX_TYPES]; /* row-major [ti*LD_MAX_TYPES+tj] */
    double lj_cut;                        /* LJ range in units of sigma_ij (> 0) */
    double coul_cut;                      /* must be <= 0: Coulomb over all pairs */
    double bjerrum;                       /* Bjerrum length l_B (>= 0) */
    double kT;                            /* thermal energy (>= 0) */
    double gravity[3];                    /* acceleration; force = mass * gravity */
    double omega;                         /* effective rotation rate */
    int32_t rotation;                     /* 0: isotropic m w^2 x; 1: about z */
    int32_t wall_band;                    /* 1: spring only within sigma/2 of R */
    int32_t noise;                        /* 0 off, 1 Gaussian, 2 fixed magnitude */
    int32_t reserved;                     /* must be 0 */
    double jump_max;                      /* |move| per component flagged (<=0: off) */
} ld_params;

/* Droplet radius schedule (section 2.1: radius-square law with a freely
 * defined rate, or no movement; section 2.2 step (iii)).  Step n uses the
 * radius at the end of the step, R(t_n + dt).  LD_R_TABLE: a freely defined
 * history, piecewise linear between n_knots knots (tab_t strictly
 * increasing), R(t) = tab_R[0] before the first knot and tab_R[n_knots - 1]
 * after the last. */
enum { LD_R_CONST = 0, LD_R_LINEAR = 1, LD_R_SQUARE_LAW = 2, LD_R_TABLE = 3 };
#define LD_R_TABLE_MAX 16
typedef struct {
    int32_t kind;
    int32_t n_knots;       /* table: knots used, 2..LD_R_TABLE_MAX (else ignored) */
    double R0, R1, T;      /* linear: R0 -> R1 over time T, then constant */
    double a;              /* square law: R^2 = R0^2 - 2 a t  (dR/dt = -a/R) */
    double R_min;          /* square law: R is clamped at R_min */
    double tab_t[LD_R_TABLE_MAX];  /* table: knot times */
    double tab_R[LD_R_TABLE_MAX];  /* table: radii at the knots (>= 0) */
} ld_radius;

/* Launch configuration of the pair kernel (filled in by ld_autotune or set
 * by hand).  Zero fields mean "library default". */
typedef struct {
    int32_t block;          /* work-items per workgroup: 64, 128, 256 or 512 */
    int32_t j_split;        /* number of j ranges per i tile (1 .. 64) */
    int32_t comp;           /* 0: FP32 blocks flushed to FP64; 1: blocked Kahan */
    int32_t sort_every;     /* steps between spatial re-sorts (<0: never) */
    int32_t cull;           /* 1: skip the LJ test for tile pairs beyond range */
    int32_t graph_steps;    /* > 0: replay steps from a captured HIP graph; a
                               chunk is sort_every steps starting with the
                               re-sort (graph_steps steps when sorting is off) */
    int32_t reserved[2];
} ld_tuning;

/* ---------------------------------------------------------------------- */
/* Life cycle                                                              */
/* ---------------------------------------------------------------------- */

/* Create a context for n >= 2 NPs.
 *   type   [n] int32 in [0, p->n_types)
 *   charge [n] FP64 charges in elementary charges
 *   pos    [n*3] FP32 positions (x0 y0 z0 x1 ...), all finite; or NULL:
 *          sampled here, uniform in the ball of radius R(0) with no pair
 *          closer than sigma_ij (section 2.1: NPs placed at random in the
 *          droplet).  Particle i in index order takes its k-th candidate
 *          (k = 0, 1, ...) from Philox4x32-10 with counter (i, k, 0, 1) and
 *          the noise key: v_c = 2 ((u_c >> 9) + 1/2) 2^-23 - 1 from the
 *          first three words; |v|^2 > 1 is dropped, else x = FP32(R(0) v) is
 *          kept when |x - x_j|^2 >= sigma_ij^2 (FP64) for every kept j < i.
 *          LD_EINVAL if a particle finds no place in 100000 candidates.
 *   p, R   parameters and radius schedule (copied)
 *   seed   Philox key of the Brownian noise stream
 *   stream hipStream_t to enqueue on (NULL: the null stream)
 * The noise for NP i at step k is Philox4x32-10 with counter (i, k mod 2^32,
 * k div 2^32, 0) and key (seed mod 2^32, seed div 2^32); the four words become
 * uniforms ((u >> 9) + 0.5) 2^-23 (exact in FP32) and then three normals by
 * Box-Muller in FP64: (sqrt(-2 ln U0) cos 2 pi U1, sqrt(-2 ln U0) sin 2 pi U1,
 * sqrt(-2 ln U2) cos 2 pi U3).
 * Errors: LD_EINVAL (n, types, parameters), LD_ENOMEM, LD_EHIP. */
ld_status ld_init(ld_ctx** out, int64_t n, const int32_t* type, const double* charge,
                  const float* pos, const ld_params* p, const ld_radius* R, uint64_t seed,
                  void* stream);

/* Release all device memory of the context (NULL is ignored). */
void ld_destroy(ld_ctx* ctx);

/* Text of the last error on this thread ("" if none). */
const char* ld_last_error(void);

/* ---------------------------------------------------------------------- */
/* The hot path                                                            */
/* ---------------------------------------------------------------------- */

/* Forces at the current state (section 2.2 steps (ii), (iv), (v)).
 *   F_pair [n*3] FP64 pair forces (LJ + Coulomb), or NULL
 *   F_ext  [n*3] FP64 external forces at R(t) of the current time t, or NULL
 *   S      [n]   FP64 sum_j |f_LJ,ij| + |f_C,ij| (error scale), or NULL
 *   U      [2]   FP64 total LJ and Coulomb pair energies, or NULL
 * Waits for the stream.  Errors: LD_EINVAL, LD_EHIP. */
ld_status ld_forces(ld_ctx* ctx, double* F_pair, double* F_ext, double* S, double* U);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the pair forces of
 * ld_forces for one set of particles, with no context and no allocation.
 * The pair kernels' scratch (packed positions and charges, low words,
 * types, group boxes, the FP64 partial sums of 4 j splits) lives in a static
 * device array of 8.3 MiB per GPU, held from the first call on that GPU
 * until the process ends.  Same arithmetic as ld_forces (FP32 Coulomb
 * terms, FP64 Lennard-Jones terms and totals, no spatial re-sort).
 *   n       2 .. 65536 particles (larger n: LD_EINVAL)
 *   type    [n] int32, device; values outside [0, p->n_types) are clamped
 *   charge  [n] FP64 charges (units of e), device
 *   pos     [n*3] FP32 positions, device
 *   p       parameters (host; LJ, l_B and kT are used)
 *   F_pair  [n*3] FP64 pair forces, device, same order as the inputs
 *   stream  hipStream_t to enqueue on (NULL: the null stream)
 * Asynchronous: nothing waits for the stream.  Every call on one GPU uses
 * that GPU's one scratch array: calls that overlap on a GPU (other streams,
 * other threads) race, so order them on one stream.  Errors: LD_EINVAL
 * (n, a pointer that is not device memory, parameters), LD_EHIP. */
ld_status ld_forces_noalloc(int64_t n, const int32_t* type, const double* charge,
                            const float* pos, const ld_params* p, double* F_pair, void* stream);

/* State and FP64 diagnostics after a call of ld_step (section 2.2; the
 * energies and momentum balance of the overdamped model). */
typedef struct {
    int64_t step;          /* global step counter */
    double t;              /* time */
    double R;              /* droplet radius R(t) */
    double U[5];           /* U_LJ, U_C, U_wall, U_grav, U_centrifugal at R(t) */
    double net_force[3];   /* sum_i F_pair,i (zero up to rounding: Newton's third law) */
    double max_force;      /* max_i |F_pair,i| */
    double max_radius;     /* max_i |x_i| */
    double msd;            /* mean_i |x_i - x_i,ref|^2 (reference: see ld_msd) */
    int64_t bad_step;      /* first step with a non-finite or too large move
                              since the previous report, or -1 */
} ld_diag;

/* Advance n_steps >= 0 steps of size dt > 0 (section 2.2 steps (ii)-(vi)):
 *   x <- x + mu dt (F_pair + F_ext(R(t+dt))) + sqrt(2 kT mu dt) xi,  mu = 1/gamma.
 *   R     radius schedule to use from the first of these steps on (section
 *         2.1: a freely defined evaporation or condensation rate; section
 *         2.2: a run can be restarted with new parameters); NULL keeps the
 *         current one.  Same effect as ld_set_params(ctx, NULL, R).
 *   seed  new Philox key for the noise from the first of these steps on
 *         (the counter keeps running on the global step count); NULL keeps
 *         the current one.  A checkpoint saves the key in use.
 *   diag  NULL: asynchronous, returns once the work is enqueued (errors of
 *         the steps themselves surface at the next synchronising call).
 *         Non-NULL: waits for the steps and fills *diag at the state after
 *         them (periodic diagnostics = chunks of ld_step with a diag); a
 *         step that blew up is reported as LD_ENONFINITE with diag->bad_step
 *         set and the rest of *diag filled.
 * A new R or seed is applied on the stream before the steps; a captured
 * step graph is re-captured with it.  Errors: LD_EINVAL (dt, n_steps, R),
 * LD_EHIP, LD_ENONFINITE (diag only). */
ld_status ld_step(ld_ctx* ctx, double dt, int64_t n_steps, const ld_radius* R,
                  const uint64_t* seed, ld_diag* diag);

/* Mean square displacement mean_i |x_i - x_i,ref|^2 (FP64, from the hi + lo
 * positions) against the reference positions: the positions at ld_init,
 * ld_checkpoint_load or the last ld_msd_reset.  Free diffusion gives
 * 6 (kT / gamma) t.  Waits for the stream.  Errors: LD_EINVAL, LD_EHIP. */
ld_status ld_msd(ld_ctx* ctx, double* msd);

/* Take the current positions as the MSD reference.  Errors: LD_EINVAL,
 * LD_EHIP. */
ld_status ld_msd_reset(ld_ctx* ctx);

/* Wait for the stream; report a pending device-side blow-up once and clear
 * it.  Errors: LD_EHIP, LD_ENONFINITE (ld_last_error names the first bad
 * step since the previous report). */
ld_status ld_sync(ld_ctx* ctx);

/* ---------------------------------------------------------------------- */
/* State access                                                            */
/* ---------------------------------------------------------------------- */

/* Positions [n*3] FP32 in original order: pos = hi part, pos_lo = lo part
 * (either may be NULL).  Waits for the stream. */
ld_status ld_get_positions(ld_ctx* ctx, float* pos, float* pos_lo);

/* Replace the positions: pos [n*3] FP32 in original order (host or device),
 * pos_lo [n*3] the low parts of the FP32 pairs or NULL for zeros.  Types,
 * charges, parameters, the step clock and the noise stream are kept (section
 * 2.2: a run restarts from a given configuration).  The slots are re-sorted
 * at the next step; group boxes are rebuilt at once.  Errors: LD_EINVAL
 * (NULL pos, non-finite coordinate), LD_EHIP. */
ld_status ld_set_positions(ld_ctx* ctx, const float* pos, const float* pos_lo);

/* Global step counter, time t and current radius R(t) (any may be NULL). */
ld_status ld_get_state(ld_ctx* ctx, int64_t* step, double* t, double* R);

/* Replace parameters and/or schedule mid-run (section 2.2: a run can be
 * stopped and restarted with different parameters).  NULL keeps the old. */
ld_status ld_set_params(ld_ctx* ctx, const ld_params* p, const ld_radius* R);

/* Save the complete state (parameters, schedule, seed, tuning, step counter,
 * time, and the slot-ordered positions hi/lo, types and original indices) to
 * a little-endian binary file (section 2.2: a run can be stopped and
 * restarted from the saved configuration).  A context loaded from it
 * continues bit for bit as the saved one would have.  The learned far field
 * is not saved.  Errors: LD_EINVAL, LD_EHIP, LD_ESTATE (file I/O). */
ld_status ld_checkpoint_save(ld_ctx* ctx, const char* path);

/* Create a context from a checkpoint on the given stream.  Errors:
 * LD_EINVAL (not a checkpoint / wrong version), LD_ENOMEM, LD_EHIP,
 * LD_ESTATE (file I/O). */
ld_status ld_checkpoint_load(ld_ctx** out, const char* path, void* stream);

/* FP64 diagnostics at the current state with R = R(t):
 * out[0] U_LJ, out[1] U_C, out[2] U_wall, out[3] U_grav, out[4] U_centrifugal,
 * out[5..7] net pair force, out[8] max |F_pair_i|, out[9] max |x_i|. */
ld_status ld_diagnostics(ld_ctx* ctx, double out[10]);

/* ---------------------------------------------------------------------- */
/* Post-processing (section 3)                                             */
/* ---------------------------------------------------------------------- */

/* Radial distribution function, Eq. (6), and radial concentration, Eq. (8),
 * over bins [b dr, (b+1) dr), dr = r_max / n_bins.  V is the sample volume
 * (<= 0: the droplet volume 4/3 pi R(t)^3).  centre: 0 droplet centre,
 * 1 centre of mass.  Outputs (host or device, any may be NULL):
 *   counts [n_bins] uint64 unordered pair counts, g [n_bins] FP64,
 *   ccounts [n_bins] uint64 particle counts from the centre, cbar [n_bins].
 * Distances use the full (hi + lo) positions in FP64. */
ld_status ld_rdf(ld_ctx* ctx, double r_max, int32_t n_bins, double V, int32_t centre,
                 uint64_t* counts, double* g, uint64_t* ccounts, double* cbar);

/* Eq. (8) for the NPs of one type (C-bar of a single type): ccounts
 * [n_bins] uint64 counts of type-`type` NPs at distance [b dr, (b+1) dr)
 * from the centre (0 droplet centre, 1 centre of mass of all NPs), cbar
 * [n_bins] = (count / N_type) / (dV_b / V), V <= 0: the droplet volume.
 * Outputs host or device, either may be NULL.  Errors: LD_EINVAL, LD_EHIP. */
ld_status ld_cbar_type(ld_ctx* ctx, int32_t type, double r_max, int32_t n_bins, double V,
                       int32_t centre, uint64_t* ccounts, double* cbar);

/* Fractal dimension, section 3.1: out[0] R_g (Eq. 3, about the centre of
 * mass, Eq. 4), out[1] D_f solving Eq. (2) with prefactor k_f and mean NP
 * diameter d (d <= 0: number-mean sigma), out[2] box-counting dimension over
 * box sides eps0 * 2^k <= R_g (eps0 <= 0: smallest sigma), fitted by least
 * squares over k >= 1, out[3] the number of box sizes.  box_counts[k]
 * (k < max_scales, may be NULL) receives the occupied-box counts. */
ld_status ld_fractal(ld_ctx* ctx, double k_f, double d, double eps0, int32_t max_scales,
                     double out[4], int64_t* box_counts);

/* ---------------------------------------------------------------------- */
/* Performance controls                                                    */
/* ---------------------------------------------------------------------- */

ld_status ld_get_tuning(ld_ctx* ctx, ld_tuning* t);
ld_status ld_set_tuning(ld_ctx* ctx, const ld_tuning* t);

/* Search the pair kernel's launch shape (workgroup size 128/256/512 x j
 x j split 1..32) by timing launches on the current state with HIP events, keep
 * the fastest, and return the resulting tuning in *out (may be NULL).
 * compensation, culling, sorting and graph settings are kept.  cache_path
 * (may be NULL) is a text file of "key block j_split ms" lines, keyed by GPU
 * architecture, size bucket (quarter octaves of n), type count and mode; a
 * hit is applied without timing unless force != 0.  Leaves positions and
 * the step state unchanged.  Errors: LD_EINVAL, LD_EHIP. */
ld_status ld_autotune(ld_ctx* ctx, const char* cache_path, int32_t force, ld_tuning* out);

/* Time every launch of the all-pairs Coulomb kernel with HIP events on the
 * context's stream (the short-ranged Lennard-Jones kernel that follows it is
 * not included).  enable = 1 starts (and clears) the record, 0 stops it.
 * ld_kernel_time waits for the stream and returns the number of timed
 * launches and their total duration in milliseconds. */
ld_status ld_kernel_timing(ld_ctx* ctx, int32_t enable);
ld_status ld_kernel_time(ld_ctx* ctx, int64_t* launches, double* total_ms);
/* With the learned far field on (ld_ff_enable), the same record also times
 * the near-field pair kernels of every step that builds the near part (from
 * the first near kernel's start to the last one's end); this returns their
 * count and total duration in milliseconds, as ld_kernel_time does for the
 * Coulomb kernel.  Errors: LD_EINVAL, LD_EHIP. */
ld_status ld_near_kernel_time(ld_ctx* ctx, int64_t* launches, double* total_ms);

/* ---------------------------------------------------------------------- */
/* Learned far field                                                        */
/* ---------------------------------------------------------------------- */

/* The pair sum split into an exact near part and a far Coulomb part,
 * F_i = F_near + q_hat_i (E_coarse + E_mlp), on a grid^3 grid over the cube
 * [-L, L]^3, L = max_i max(|x_i|, |y_i|, |z_i|) (1 + 2^-10) in FP32; a
 * particle's cell is floor((x + L) / h), h = 2L / grid, clamped to the grid.
 * Cell moments: Q = sum q_hat and dipole P = sum q_hat (x - centre).
 *
 * near_mode 0 (radial): pairs with r < r_c are summed exactly (LJ +
 *   Coulomb) over a cell list of side >= r_c; E_coarse is the field at the
 *   centre of i's cell from the monopole + dipole of every cell outside the
 *   block^3 neighbourhood of that cell; the network predicts the rest of the
 *   Coulomb field of the pairs with r >= r_c.
 * near_mode 1 (block): the Coulomb pairs with j in i's block^3 neighbourhood
 *   (and every LJ pair) are summed exactly; E_coarse is the second-order
 *   Taylor expansion about i's cell centre of the monopole + dipole field of
 *   every cell outside the neighbourhood (the cells of 2x2x2 parents beyond
 *   parent_reach taken together through the parent's moments), evaluated at
 *   x_i; the network predicts the rest of the field of the particles outside
 *   the block.  near_cut is unused.
 *
 * The MLP (K = 4 block^3 + 3 inputs -> hidden -> hidden -> 3, SiLU, BF16
 * operands, FP32 accumulation) reads the neighbourhood's (Q / sq,
 * P / (sq h)) (cells ordered z-major, then y, then x; zero outside the grid)
 * and the offset (x - centre) / h, and predicts the remaining far field
 * divided by out_scale.  q_hat = q sqrt(kT l_B). */
typedef struct {
    double near_cut;        /* r_c (>= the largest LJ range), near_mode 0 */
    int32_t grid;           /* G, 4..64 */
    int32_t block;          /* B, odd, 1..7 */
    int32_t hidden;         /* H, multiple of 16, 16..256 */
    int32_t judge_every;    /* steps between judge evaluations (mode 2) */
    double judge_tol;       /* median relative force error allowed */
    int32_t near_mode;      /* 0 radial cutoff r_c, 1 the block^3 cells */
    int32_t parent_reach;   /* block mode, even grid: > 0 groups far cells by 2x2x2
                               parent cells beyond this Chebyshev distance (in parent
                               cells) from the target's parent; 0 = one level, every
                               far cell on its own (a grid convolution evaluated by
                               FFT for grid <= 32, direct sums above) */
} ld_ff_config;

typedef struct {
    int32_t epochs;
    int32_t batch;          /* 16..65536 */
    double lr;              /* Adam learning rate */
    uint64_t seed;          /* shuffle stream (Philox, tag 3) */
    double val_fraction;    /* last fraction of the samples held out */
    int32_t reset_scale;    /* 1: set out_scale to the RMS of the targets */
    int32_t calibrate;      /* 1: after training, scale the output by the least-squares
                               gain on the held-out samples, clipped to [0, 1] */
} ld_ff_train_cfg;

typedef struct {
    int64_t samples, iterations;
    double final_loss;      /* MSE of the scaled residual, last batch */
    double val_rel_rms;     /* relative RMS error of the residual, held out (after
                               the gain) */
    double out_scale;       /* final output scale (gain included) */
    double gain;            /* the fitted gain (1 without calibration) */
    double val_rel_rms_raw; /* held-out relative RMS error before the gain */
} ld_ff_train_report;

/* Allocate the learned far field for this context (weights get small
 * deterministic initial values; sq = largest |q_hat|).  Errors: LD_EINVAL,
 * LD_ENOMEM. */
ld_status ld_ff_enable(ld_ctx* ctx, const ld_ff_config* cfg);

/* 0: direct summation; 1: learned far field every step; 2: learned with a
 * judge every judge_every steps that falls back to direct summation for the
 * next window when the median relative error of the pair forces exceeds
 * judge_tol. */
ld_status ld_ff_mode(ld_ctx* ctx, int32_t mode);

/* Number of packed FP32 weights: W1 [Kp x H] (Kp = K rounded up to 32; rows
 * >= K unused), b1 [H], W2 [H x H], b2 [H], W3 [H x 16] (columns >= 3
 * unused), b3 [16]; all row-major [in][out]. */
int64_t ld_ff_weights_size(ld_ctx* ctx);
ld_status ld_ff_set_weights(ld_ctx* ctx, const float* w, int64_t count, double sq,
                            double out_scale);
ld_status ld_ff_get_weights(ld_ctx* ctx, float* w, int64_t count, double* sq, double* out_scale);

/* Save the trained model (the configuration that fixes its inputs: grid,
 * block, hidden, near mode, parent reach, near cut; sq, out_scale and the
 * packed weights) to a binary file, and load it into a context whose
 * ld_ff_enable configuration matches (else LD_EINVAL naming both).  File:
 * "LDFFW001", int32 grid, block, hidden, near_mode, parent_reach, 0; FP64
 * near_cut, sq, out_scale; int64 count; FP32 weights[count].  Errors:
 * LD_ESTATE (no learned field), LD_EINVAL (path, I/O, format, mismatch). */
ld_status ld_ff_save(ld_ctx* ctx, const char* path);
ld_status ld_ff_load(ld_ctx* ctx, const char* path);

/* The cube half width L and near cells per axis for the current positions. */
ld_status ld_ff_grid(ld_ctx* ctx, double* L, int32_t* near_cells);

/* Parts of the learned pair force at the current state, [n*3] FP64 in
 * original order: 0 near (exact), 1 q E_coarse, 2 q E_mlp, 3 their sum (the
 * learned pair force), 4 the exact far force (the Coulomb force of the pairs
 * not in the near part). */
ld_status ld_ff_forces(ld_ctx* ctx, int32_t part, double* out);

/* MLP output [m*3] for m feature rows X [m*K] (FP32, host or device). */
ld_status ld_ff_mlp(ld_ctx* ctx, const float* X, int64_t m, float* Y);

/* Mean-squared loss of the MLP on (X [m*K], T [m*3]) and its gradients in
 * the packed weight layout. */
ld_status ld_ff_grads(ld_ctx* ctx, const float* X, const float* T, int64_t m, float* grads,
                      double* loss);

/* Append one training snapshot of the current state: for every particle
 * its cell, offset and target (exact far field minus the coarse field).
 * reset = 1 starts a new store with room for max_snapshots snapshots. */
ld_status ld_ff_collect(ld_ctx* ctx, int32_t reset, int32_t max_snapshots);

/* Train the MLP on the stored samples with Adam (forward and backward on the
 * matrix cores). */
ld_status ld_ff_train(ld_ctx* ctx, const ld_ff_train_cfg* cfg, ld_ff_train_report* report);

/* Median relative error of the learned pair forces against direct
 * summation at the current state. */
ld_status ld_ff_judge(ld_ctx* ctx, double* median_rel_err);

/* out = {judges, fallbacks, learned steps, direct steps}; last judge error. */
ld_status ld_ff_stats(ld_ctx* ctx, int64_t out[4], double* last_err);

/* ---------------------------------------------------------------------- */
/* Ensembles of independent droplets                                       */
/* ---------------------------------------------------------------------- */

typedef struct ld_ens ld_ens;

/* Create n_drop >= 1 independent droplets that step together.  Droplet d
 * owns particles [offsets[d], offsets[d+1]) (offsets: host int64
 * [n_drop+1], offsets[0] = 0, at least 2 particles per droplet) of the
 * concatenated arrays type [total] int32, charge [total] FP64 and pos
 * [total*3] FP32 (host or device).  p, R and seeds are host arrays of
 * n_drop entries: each droplet has its own parameters, radius schedule and
 * noise seed.  Particle i of droplet d draws the noise it would draw alone,
 * i.e. Philox counter (i - offsets[d], step, 0) with key seeds[d].  All
 * droplets share the step counter and time.  Pair forces couple particles of
 * the same droplet only.  Errors: LD_EINVAL, LD_ENOMEM, LD_EHIP. */
ld_status ld_ens_init(ld_ens** out, int32_t n_drop, const int64_t* offsets, const int32_t* type,
                      const double* charge, const float* pos, const ld_params* p,
                      const ld_radius* R, const uint64_t* seeds, void* stream);
void ld_ens_destroy(ld_ens* e);

/* Launch shape of the persistent pair kernel (workgroups of 256 work-items;
 * 0 keeps the current count), compensation mode (0 FP64 flush, 1 blocked
 * Kahan), and the number of steps captured in one HIP graph (0: no graph).
 * Captured steps replay with the dt they were captured with. */
ld_status ld_ens_set_tuning(ld_ens* e, int32_t workgroups, int32_t comp, int32_t graph_steps);

/* out = {workgroups, comp, graph_steps, unroll, rows}. */
ld_status ld_ens_get_tuning(ld_ens* e, int32_t out[5]);

/* Coulomb pairs in flight per lane in the persistent pair kernel: 8, 16
 * (default) or 32.  Errors: LD_EINVAL. */
ld_status ld_ens_set_unroll(ld_ens* e, int32_t unroll);

/* Slots per work item of the persistent pair kernel: 64 (default; a
 * wavefront per 64-slot tile, each staging its own j tiles) or 256 (a
 * workgroup per block of four tiles, sharing staged j tiles of 256).  The
 * forces are bit for bit the same either way.  Errors: LD_EINVAL. */
ld_status ld_ens_set_rows(ld_ens* e, int32_t rows);

/* Choose the persistent pair kernel's workgroup count (2..8 per compute
 * unit), unroll (8, 16, 32) and work-item rows (64, 256) by timing the pair
 * step (forces only; the droplets do not move) with HIP events, keeping the
 * compensation mode and graph length; none of the searched settings changes
 * the forces.  A spatial re-sort that is due (a new ensemble's first, or
 * one the sort interval calls for) is done first, as the next step would
 * have done it, so the timings see the slot order the steps use and the
 * trajectory is unchanged; forces read right after this call come in that
 * order's summation.  The four fastest settings of one pass are timed again
 * as bursts of launches.  cache_path (or NULL): a text file of lines
 * "key workgroups unroll rows ms"; the key holds the GPU architecture, the
 * droplet count, quarter-octave buckets of sum_d N_d^2 and of the largest
 * N_d, the culling and compensation modes.  A cached key is used without
 * timing unless force != 0; new results are appended.  out (or NULL) as in
 * ld_ens_get_tuning.  Errors: LD_EINVAL, LD_EHIP. */
ld_status ld_ens_autotune(ld_ens* e, const char* cache_path, int32_t force, int32_t out[5]);

/* Advance all droplets n_steps >= 0 steps of size dt > 0 (asynchronous). */
ld_status ld_ens_step(ld_ens* e, double dt, int64_t n_steps);

/* Pair forces [total*3] FP64 of every particle at the current state. */
ld_status ld_ens_forces(ld_ens* e, double* F_pair);

/* Positions [total*3] FP32 hi and lo parts (either may be NULL). */
ld_status ld_ens_get_positions(ld_ens* e, float* pos, float* pos_lo);

/* Shared step counter and time. */
ld_status ld_ens_get_state(ld_ens* e, int64_t* step, double* t);

/* Wait; report a pending blow-up once (LD_ENONFINITE) and clear it. */
ld_status ld_ens_sync(ld_ens* e);

/* HIP-event timing of every persistent pair launch (see ld_kernel_timing);
 * timing disables graph replay while it is on. */
ld_status ld_ens_kernel_timing(ld_ens* e, int32_t enable);
ld_status ld_ens_kernel_time(ld_ens* e, int64_t* launches, double* total_ms);

/* Trajectory recording (section 2.2: results recorded in a binary file for
 * viewing and post-processing, every j-th frame).  After every `every`-th
 * step of ld_step (global step count a multiple of every) the positions --
 * FP32 of hi + lo, original order -- are copied asynchronously and appended
 * to `path` by a writer thread, so stepping continues meanwhile (graph
 * replay is off while recording).  File: "LDTRAJ01", int64 n, int32
 * n_types, int32 every, int32 type[n]; then per frame int64 step, FP64 t,
 * FP64 R(t), float32 x[n][3].  Errors: LD_EINVAL (path, every), LD_ESTATE
 * (already recording), LD_ENOMEM, LD_EHIP. */
ld_status ld_record_open(ld_ctx* ctx, const char* path, int32_t every);

/* Finish writing (waits for frames in flight) and close; *frames (may be
 * NULL) receives the number written.  Errors: LD_ESTATE, LD_EHIP. */
ld_status ld_record_close(ld_ctx* ctx, int64_t* frames);

/* Sub-aggregates (section 2.1 lists their number and aggregate statistics
 * among the model's post-processing outputs): the connected components of
 * the contact graph at the current positions, two NPs in contact when
 * r < contact_factor sigma_ij (FP64 distances).  stats (host) receives
 * [components, aggregates = components of >= 2 NPs, size of the largest];
 * labels (optional, [n] int32, host or device, original order) the smallest
 * original index of each NP's component, so the result is unique.  The
 * slot order is not changed.  Errors: LD_EINVAL, LD_ENOMEM, LD_EHIP. */
ld_status ld_aggregates(ld_ctx* ctx, double contact_factor, int64_t stats[3], int32_t* labels);

/* N_surf (section 1: the number of NPs at the droplet surface): per type,
 * the NPs with | |x| - R | < sigma_t / 2, into counts[n_types] (host).  R < 0
 * means the droplet's radius at the current time.  Errors: LD_EINVAL,
 * LD_ENOMEM, LD_EHIP. */
ld_status ld_surface_count(ld_ctx* ctx, double R, int64_t* counts);

/* Surface fractal dimension (section 3.1: the fractal equation, Eqs. (2)-(4),
 * holds at dimension two for the NP structure on the droplet surface, with
 * the sphere's geometry taken into account).  Surface NPs as
 * ld_surface_count (R < 0: the current radius); surface aggregates = the
 * components of the contact graph among them (r < contact_factor sigma_ij,
 * FP64).  For the largest (equal sizes: the smallest label): u_i = x_i/|x_i|,
 * u_0 = the normalised sum of the u_i, R_g^2 = mean over its NPs of
 * (R angle(u_i, u_0))^2 (geodesic distances on the sphere of radius R),
 * D_f = ln(N / k_f) / ln(2 R_g / d), d <= 0: the aggregate's number-mean
 * sigma.  k_f = pi / sqrt(3) makes a compact hexagonal disk two-dimensional
 * (the planar counterpart of the compact prefactor 1.593 the paper takes in
 * three dimensions).  stats (host) = [surface aggregates, size of the
 * largest, its label] ([0, 0, -1] without surface NPs); out (host) = [R_g,
 * d, D_f]: D_f NaN below two NPs, all NaN without surface NPs.  labels
 * (optional, [n] int32, host or device, original order): the smallest
 * original index of a surface NP's aggregate, -1 for NPs off the surface.
 * The slot order is not changed.  Errors: LD_EINVAL, LD_ENOMEM, LD_EHIP. */
ld_status ld_surface_fractal(ld_ctx* ctx, double R, double contact_factor, double k_f, double d,
                             int64_t stats[3], double out[3], int32_t* labels);

/* ---------------------------------------------------------------------- */
/* The paper's own scheme (section 2.2 steps (i)-(vi) read literally)      */
/* ---------------------------------------------------------------------- */

/* Pairs interact when closer than range_factor (r_i + r_j), r = sigma / 2
 * (step (i): the paper uses 4); LJ and Coulomb are both truncated there
 * without shift (step (ii)).  Each ld_step of the context then does: slots
 * sorted by cells of side >= the largest range (step (i)); the truncated pair
 * forces over the 27 neighbouring cells, FP64 (step (ii)); R(t + dt) (step
 * (iii)); surface spring, gravity and centrifugal force of ld_params
 * (steps (iv)-(v); wall_band = 1 with wall_offset = sigma/2 is the paper's
 * spring acting within one radius of the surface); then Newton's equation
 * with Stokes drag and the random velocity vector (step (vi)):
 *   v <- v + dt (F_pair + F_ext - gamma v) / inertial_mass,
 *   v <- v + kick u,   u = the normalised Box-Muller triple of the ld_init
 *                      noise stream (uniform on the unit sphere),
 *   x <- x + dt v.
 * ld_params.noise is not used (kT still scales Coulomb through l_B).
 * Velocities are FP64, kept in slot order on the device. */
typedef struct {
    double range_factor;                 /* > 0 (the paper: 4) */
    double kick;                         /* >= 0: magnitude of the random velocity */
    double inertial_mass[LD_MAX_TYPES];  /* > 0 for every type in use */
} ld_paper_config;

/* Switch ld_step to the paper's scheme, velocities zero.  Graph replay is off
 * meanwhile and checkpoints are refused (they hold no velocities).
 * Errors: LD_EINVAL (cfg), LD_ESTATE (learned far field on), LD_ENOMEM. */
ld_status ld_paper_enable(ld_ctx* ctx, const ld_paper_config* cfg);

/* Back to the overdamped scheme (velocities dropped).  NULL-safe context. */
ld_status ld_paper_disable(ld_ctx* ctx);

/* Truncated pair forces F [n*3] FP64 (original order) at the current
 * positions (re-sorts the slots by cell).  Errors: LD_EINVAL, LD_ESTATE. */
ld_status ld_paper_forces(ld_ctx* ctx, double* F);

/* Velocities v [n*3] FP64 in original order (host or device pointers).
 * set: every value must be finite.  Errors: LD_EINVAL, LD_ESTATE. */
ld_status ld_paper_get_velocities(ld_ctx* ctx, double* v);
ld_status ld_paper_set_velocities(ld_ctx* ctx, const double* v);

#ifdef __cplusplus
}
#endif

#endif /* LDROP_H */
