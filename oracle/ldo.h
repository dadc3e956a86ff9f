/*
 * ldo.h -- CPU FP64 oracle for the Langevin droplet-aggregation model of
 * Derkachov et al., "A numerical toy model of Langevin dynamics provides
 * real-time visualization of colloidal microdroplet evaporation"
 * (arXiv:2501.04456).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously-correct reference
 * that the GPU library is checked against.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or helper with the GPU library; neither side includes
 * or links the other.
 *
 * Everything is plain scalar C in double precision.  Sums over particles run
 * in ascending index order with Neumaier compensation, so results do not
 * depend on the number of OpenMP threads.
 *
 * Units are reduced: lengths in units of the type-0 diameter, energies in kT
 * units where kT is a parameter, charges in elementary charges.
 *
 * Parity status per function is stated next to each declaration.  Every
 * function below is pinned by CPU tests against closed forms, invariants,
 * brute force or an independent implementation, unless it says
 * "parity unpinned".
 */
#ifndef LDO_H
#define LDO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LDO_MAX_TYPES 8

/* Physical parameters of one droplet (section 2.1 lists the interactions:
 * LJ and Coulomb between NPs; viscosity, centrifugal force, gravity and the
 * surface spring as external forces; Brownian motion). */
typedef struct {
    int32_t n_types;
    int32_t use_eps_matrix;          /* 0: Lorentz-Berthelot eps_ij = sqrt(eps_i eps_j) */
    double sigma[LDO_MAX_TYPES];     /* LJ size = contact diameter; NP radius = sigma/2 */
    double eps[LDO_MAX_TYPES];       /* LJ well depth per type */
    double mass[LDO_MAX_TYPES];      /* buoyancy-corrected mass (gravity, centrifugal) */
    double gamma[LDO_MAX_TYPES];     /* Stokes drag coefficient; mobility = 1/gamma */
    double k_wall[LDO_MAX_TYPES];    /* surface spring constant per type */
    double wall_offset[LDO_MAX_TYPES]; /* spring equilibrium distance inside the surface */
    double eps_matrix[LDO_MAX_TYPES * LDO_MAX_TYPES];
    double lj_cut;                   /* LJ range in units of sigma_ij (truncated, not shifted) */
    double coul_cut;                 /* <= 0: Coulomb over all pairs; > 0: truncated at this r */
    double bjerrum;                  /* Bjerrum length l_B */
    double kT;                       /* thermal energy; sets the Coulomb scale and noise */
    double gravity[3];               /* acceleration vector; force = mass * gravity */
    double omega;                    /* effective rotation rate */
    int32_t rotation;                /* 0: isotropic centrifugal m w^2 x; 1: about z axis */
    int32_t wall_band;               /* 1: spring acts only for | |x| - R | < sigma/2 */
    int32_t noise;                   /* 0: off, 1: Gaussian, 2: fixed magnitude, random direction */
    int32_t reserved;
    double jump_max;                 /* per-step displacement component flagged as a blow-up */
} ldo_params;

/* Droplet radius schedule (section 2.1: radius-square law with a freely set
 * rate; section 2.2 step (iii)). */
enum { LDO_R_CONST = 0, LDO_R_LINEAR = 1, LDO_R_SQUARE_LAW = 2, LDO_R_TABLE = 3 };
#define LDO_R_TABLE_MAX 16
typedef struct {
    int32_t kind;
    int32_t n_knots;    /* table: knots used */
    double R0, R1, T;   /* linear: R0 -> R1 over time T, then constant */
    double a;           /* square law: R^2 = R0^2 - 2 a t (a < 0: condensation) */
    double R_min;       /* square law: clamp R >= R_min (dry aggregate) */
    double tab_t[LDO_R_TABLE_MAX];  /* table: increasing knot times */
    double tab_R[LDO_R_TABLE_MAX];  /* table: radii; linear in between, end values outside */
} ldo_radius;

/* --- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Pinned against
 *     rocRAND's independent host implementation and by statistics. */
void ldo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Three standard normal variates for particle `id` at step `step` with the
 * given seed and stream tag (Box-Muller on Philox output).  Pinned by
 * moments and by the uniform mapping's exactness. */
void ldo_gauss3(int64_t id, int64_t step, uint64_t seed, uint32_t tag, double xi[3]);

/* Initial positions uniform in the ball of radius R0 with every pair at
 * least sigma_ij = (sigma_a + sigma_b) / 2 apart (section 2.1: NPs placed at
 * random in the droplet; no two may overlap).  Particle i (in index order)
 * takes its k-th candidate (k = 0, 1, ...) from Philox4x32-10 with counter
 * (i, k, 0, 1) and key (seed mod 2^32, seed div 2^32): the first three
 * words give v_c = 2 ((u_c >> 9) + 1/2) 2^-23 - 1; a candidate with
 * |v|^2 > 1 is outside the ball and is dropped; otherwise x = FP32(R0 v_c)
 * per component, accepted when |x - x_j|^2 >= sigma_ij^2 (FP64 on the FP32
 * values) for every accepted j < i.  x [n*3] receives the FP32 values as
 * FP64.  Returns 0, or the first index that found no place in max_tries
 * candidates (then x holds the particles before it).  Plain O(n^2). */
int64_t ldo_sample_ball(int64_t n, const int32_t* type, const double* sigma, double R0,
                        uint64_t seed, int64_t max_tries, double* x);

/* R(t).  Pinned by closed forms. */
double ldo_radius_at(const ldo_radius* R, double t);

/* Pair forces (section 2.2 step (ii)) on the particles listed in rows
 * (rows == NULL: all n, in order).  pos is [n*3] FP64.  Outputs per listed
 * row: F[r*3..] (FP64), S[r] = sum_j |f_LJ,ij| + |f_C,ij| (conditioning
 * scale), and U[0..1] += per-row half-sums of LJ and Coulomb energies (so
 * that with rows == NULL they are the total pair energies).  Any output may
 * be NULL.  Pinned by closed forms, Newton's third law, F = -grad U and brute
 * force. */
void ldo_pair_forces(int64_t n, const double* pos, const int32_t* type, const double* q,
                     const ldo_params* p, const int64_t* rows, int64_t n_rows,
                     double* F, double* S, double* U);

/* External force on one particle at position x, type t, droplet radius R
 * (section 2.2 steps (iv)-(v)): surface spring, gravity, centrifugal.  Drag
 * enters the update through the mobility.  Pinned by closed forms. */
void ldo_external_force(const double x[3], int32_t t, const ldo_params* p, double R,
                        double F[3]);

/* Overdamped Langevin (Euler-Maruyama) steps (section 2.2 step (vi), read in
 * the overdamped limit):
 *   x <- x + mu dt (F_pair + F_ext(R(t + dt))) + sqrt(2 kT mu dt) xi
 * x is [n*3] FP64, updated in place.  ids[i] is the Philox stream id of
 * particle i (NULL: i).  *step and *t are the global step counter and time,
 * advanced in place.  Returns the first step index whose update was
 * non-finite or exceeded jump_max, or -1.  Pinned by settling, relaxation,
 * centrifugal growth, free diffusion and equipartition. */
int64_t ldo_run(int64_t n, double* x, const int32_t* type, const double* q,
                const int64_t* ids, const ldo_params* p, const ldo_radius* R,
                double dt, int64_t n_steps, uint64_t seed, int64_t* step, double* t);

/* The paper's own scheme (section 2.2 steps (i)-(vi) read literally):
 * pairs interact when closer than range_factor (r_i + r_j), r = sigma / 2,
 * LJ and Coulomb both truncated there without shift; Newton's equation with
 * Stokes drag and a random velocity vector of fixed magnitude `kick` in a
 * uniformly random direction. */
typedef struct {
    double range_factor;                 /* 4 in the paper */
    double kick;                         /* |random velocity| added per step */
    double inertial_mass[LDO_MAX_TYPES]; /* mass in Newton's equation per type */
} ldo_paper;

/* Truncated pair forces F [m*3] and S [m] = sum_j |f_LJ| + |f_C| of the pairs
 * in range (either may be NULL) for the rows listed (rows NULL: all n, m = n;
 * else m = n_rows, each row against all n particles).  Pinned against
 * ldo_pair_forces where the two definitions coincide, by Newton's third law
 * and by truncation invariance. */
void ldo_paper_forces(int64_t n, const double* pos, const int32_t* type, const double* q,
                      const ldo_params* p, const ldo_paper* m, const int64_t* rows,
                      int64_t n_rows, double* F, double* S);

/* Steps of the paper's scheme; x and v [n*3] FP64 updated in place:
 *   v <- v + dt (F_pair + F_ext(R(t + dt)) - gamma v) / m;  v <- v + kick u;
 *   x <- x + dt v,
 * u = the normalised ldo_gauss3 triple (tag 0) of particle ids[i] (NULL: i).
 * Returns the first step whose move was non-finite or beyond jump_max, or
 * -1.  Pinned by the drag decay and terminal velocity (closed forms), the
 * damped harmonic trap (the scheme's 2x2 linear map raised to the n-th power)
 * and the kick's magnitude and isotropy. */
int64_t ldo_paper_run(int64_t n, double* x, double* v, const int32_t* type, const double* q,
                      const int64_t* ids, const ldo_params* p, const ldo_paper* m,
                      const ldo_radius* R, double dt, int64_t n_steps, uint64_t seed,
                      int64_t* step, double* t);

/* Sub-aggregates (section 2.1 names their number among the post-processing
 * outputs): connected components of the contact graph, a pair in contact
 * when r < contact_factor sigma_ij.  labels[i] (may be NULL) = the smallest
 * index in i's component.  Returns the number of components.  Pinned
 * against scipy's kd-tree pairs + connected components and hand-built
 * chains. */
int64_t ldo_components(int64_t n, const double* x, const int32_t* type, const ldo_params* p,
                       double contact_factor, int64_t* labels);

/* N_surf (section 1): NPs with | |x| - R | < sigma_t / 2, per type into
 * counts[n_types].  Pinned by constructed shells. */
void ldo_surface_count(int64_t n, const double* x, const int32_t* type, const ldo_params* p,
                       double R, int64_t* counts);

/* Surface fractal dimension (section 3.1's fractal equation at dimension two
 * on the sphere).  Surface NPs as ldo_surface_count; their contact-graph
 * components (r < contact_factor sigma_ij); stats = [components, size of the
 * largest, its label] (label = smallest original index; ties between sizes:
 * the smaller label; no surface NP: [0, 0, -1]).  For the largest: u_i =
 * x_i / |x_i|, u_0 = the normalised sum of the u_i, out[0] = R_g =
 * sqrt(mean (R angle(u_i, u_0))^2), out[1] = d (d <= 0: the component's
 * number-mean sigma), out[2] = D_f = ln(N / k_f) / ln(2 R_g / d) (NaN below
 * two NPs; all NaN without surface NPs or when the u_i sum to zero).
 * labels[n] (may be NULL): the component label of surface NPs, -1 elsewhere.
 * Pinned by two-NP and ring closed forms, the flat-plane limit, rotation
 * invariance, and the components against scipy. */
void ldo_surface_fractal(int64_t n, const double* x, const int32_t* type, const ldo_params* p,
                         double R, double contact_factor, double k_f, double d, int64_t stats[3],
                         double out[3], int64_t* labels);

/* One step for the listed rows only (pair forces from all n particles at the
 * current positions); writes the rows' new positions, leaves x unchanged.
 * Returns step if a listed row blew up, else -1.  Pinned against whole
 * ldo_run steps (bit for bit, with and without noise, band wall, a moving
 * radius and a step counter other than zero) and against the noise stream
 * for a free particle. */
int64_t ldo_step_rows(int64_t n, const double* x, const int32_t* type, const double* q,
                      const int64_t* ids, const ldo_params* p, const ldo_radius* R,
                      double dt, uint64_t seed, int64_t step, double t,
                      const int64_t* rows, int64_t n_rows, double* x_rows_out);

/* Diagnostics (FP64): out[0] U_LJ, out[1] U_C, out[2] U_wall, out[3] U_grav,
 * out[4] U_centrifugal, out[5..7] net pair force, out[8] max |F_pair_i|,
 * out[9] max |x_i|.  R is the radius used for the wall.  Pinned by the
 * single-NP closed forms of the three external energies, by their negative
 * gradient against ldo_external_force (central differences), by Newton's
 * third law for the net force and by hand-built maxima. */
void ldo_diagnostics(int64_t n, const double* x, const int32_t* type, const double* q,
                     const ldo_params* p, double R, double out[10]);

/* Mean square displacement: the mean over particles of |x_i - x0_i|^2.
 * Pinned by a hand-built case and by free diffusion (6 D t). */
double ldo_msd(int64_t n, const double* x, const double* x0);

/* Radial distribution function, Eq. (6), and radial concentration, Eq. (8).
 * Bins are [b*dr, (b+1)*dr) with dr = r_max / n_bins.  counts[b] is the
 * number of unordered pairs in bin b; ccounts[b] the number of particles at
 * distance from `centre` in bin b.  V is the sample volume.  g and cbar may
 * be NULL.  Pinned by brute force, lattice shells and the uniform ball. */
void ldo_rdf(int64_t n, const double* x, double r_max, int32_t n_bins, double V,
             const double centre[3], uint64_t* counts, uint64_t* ccounts,
             double* g, double* cbar);

/* Fractal dimension from the radius of gyration, Eqs. (2)-(4), with
 * prefactor k_f and mean NP diameter d: out[0] = R_g, out[1] = D_f.
 * Box counting: out[2] = D_box, out[3] = number of scales used; occupied-box
 * counts at eps_k = eps0 * 2^k go to box_counts[k] (k < max_scales).
 * Pinned by Eq. (2) round trip and lattice / Sierpinski fractals. */
void ldo_fractal(int64_t n, const double* x, double k_f, double d, double eps0,
                 int32_t max_scales, double out[4], int64_t* box_counts);

/* ---- learned far field (ldo_ff.c) ------------------------------------- */

/* BF16 round-to-nearest-even of v (through its FP32 value).  Pinned against
 * torch's bfloat16 conversion. */
double ldo_bf16(double v);

/* Cell moments of the G^3 grid over [-L, L]^3: out[4*cell] = (Q, Px, Py, Pz)
 * with Q = sum q_hat and P = sum q_hat (x - cell centre); cell index
 * (iz*G + iy)*G + ix; positions outside the cube clamp to the edge cells.
 * Pinned by charge conservation and single-particle dipoles. */
void ldo_ff_moments(int64_t n, const double* x, const double* qhat, int G, double L,
                    double* out);

/* Field at each cell centre from the monopole + dipole of every cell outside
 * the B^3 block around it.  Pinned against exact point-charge sums. */
void ldo_ff_coarse(int G, double L, int B, const double* mom, double* E);

/* Pair forces of pairs closer than rc (LJ + Coulomb) and the Coulomb field
 * sum_{j: r >= rc} q_hat_j r_ij / r^3 for the listed rows.  Pinned by
 * F_near + q_hat E_far = the full pair force. */
void ldo_ff_split(int64_t n, const double* x, const int32_t* type, const double* q,
                  const ldo_params* p, double rc, const int64_t* rows, int64_t n_rows,
                  double* F_near, double* E_far);

/* Block split: pairs whose cells lie within the B^3 block (Chebyshev cell
 * distance <= B/2) are summed exactly (LJ + Coulomb); LJ of pairs outside the
 * block but within LJ range is added to F_near too; E_far is the Coulomb
 * field sum over j outside the block (without q_hat_i).  Pinned by
 * F_near + q_hat E_far = the full pair force and brute-force block
 * membership. */
void ldo_ff_split_block(int64_t n, const double* x, const int32_t* type, const double* q,
                        const ldo_params* p, int G, double L, int B, const int64_t* rows,
                        int64_t n_rows, double* F_near, double* E_far);

/* Second-order local expansion at every cell centre of the monopole + dipole
 * field of every cell outside the B^3 block: out[19*cell] = E (x, y, z),
 * J = dE_c/dx_d (xx, xy, xz, yy, yz, zz), H = d2E_c/dx_d dx_e (xxx, xxy,
 * xxz, xyy, xyz, xzz, yyy, yyz, yzz, zzz).  Pinned by finite differences of
 * point-charge and point-dipole fields and by Laplace's equation. */
void ldo_ff_local(int G, double L, int B, const double* mom, double* out);

/* The same expansion with far cells grouped by 2x2x2 parent cells (G even):
 * parents farther than D (Chebyshev, in parent cells) from the target's
 * parent enter through their own monopole + dipole.  Pinned by D >= G/2
 * reproducing ldo_ff_local, parent moments against ldo_ff_moments on the
 * G/2 grid, and the method's accuracy on a droplet. */
void ldo_ff_local2(int G, double L, int B, int D, const double* mom, double* out);

/* E(x) = E + J d + (1/2) H d d, d = x - centre of x's cell, for n points. */
void ldo_ff_local_eval(int64_t n, const double* x, int G, double L, const double* loc,
                       double* E);

/* MLP features [n * (4 B^3 + 3)]: normalised moments of the B^3 block
 * around each particle's cell (dz-major), then its offset / h. */
void ldo_ff_features(int64_t n, const double* x, int G, double L, int B, const double* mom,
                     double sq, double* X);

/* Three-layer SiLU MLP forward (optionally with BF16 operands) and its FP64
 * backpropagation for the mean-squared loss.  Pinned against torch (CPU,
 * FP64) and finite differences. */
void ldo_mlp_forward(int64_t m, int K, int H, int O, const double* X, const double* W1,
                     const double* b1, const double* W2, const double* b2, const double* W3,
                     const double* b3, int bf16, double* Y, double* Z1, double* A1, double* Z2,
                     double* A2);
double ldo_mlp_backward(int64_t m, int K, int H, int O, const double* X, const double* T,
                        const double* W1, const double* b1, const double* W2, const double* b2,
                        const double* W3, const double* b3, int bf16, double* dW1, double* db1,
                        double* dW2, double* db2, double* dW3, double* db3);

#ifdef __cplusplus
}
#endif
#endif
