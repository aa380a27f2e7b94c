/*
 * mlb: multicomponent Enskog lattice-Boltzmann step on MI355X (gfx950).
 *
 * C ABI of the GPU library libmlb.so.  Plain pointers and sizes only.
 *
 * The method (Marini Bettolo Marconi & Melchionna, "Multicomponent diffusion
 * in nanosystems"): M species of hard spheres with diameters sigma_aa,
 * masses m_alpha, uniform temperature T and optional attractive tails evolve
 * by the kinetic equation of Sec. 2, eq. (evolution): relaxation at rate
 * omega towards the orthogonalised local equilibrium psi_perp of
 * eqs. (psia)-(prefactor), plus the molecular-field term
 * Phi_a . (v - u) psi_a / kT, where Phi_a is the self-consistent field of
 * Sec. 3, eq. (splitforce):
 *   - hard-core mean field, a shell integral of g_ab n_b at radius sigma_ab,
 *     eq. (potmeanforce);
 *   - RPA attractive field, a convolution of n_b with grad U_ab, below
 *     eq. (potmeanforce);
 *   - drag and viscous forces, eqs. (gammaab), (tensorgamma), (viscousforce),
 *     evaluated as one pair form with a Crank-Nicolson treatment of the
 *     velocity dependence (one local Jacobi predictor sweep);
 *   - an external body force F^a (eq. evolution).
 * Space and velocity are discretised on a D3Q19 lattice (spacing and time
 * step 1, kT = 1/3 = c_s^2).  Populations count particles (sum_i f_ai = n_a,
 * sum_i c_i f_ai = j_a, the number flux); species a's equilibrium is the
 * second-order Hermite form of eq. (psia) with thermal speed^2
 * theta_a = kT/m_a, i.e. the c_s^2 form plus (9/2)(theta_a - 1/3)(c.c - 1);
 * the orthogonalising factor of eq. (prefactor) is m_a/kT, and a force
 * density N_a changes j_a at the rate N_a/m_a.  Unit masses give the plain
 * D3Q19 equilibrium.
 *
 * Conventions for every entry point:
 *   - Device pointers are HIP device addresses; "host" pointers are CPU
 *     memory.  Field arrays are species-major, x fastest:
 *       scalar field  [M][nz][ny][nx]
 *       vector field  [M][3][nz][ny][nx]
 *       populations   [M][19][nz][ny][nx]   (velocity order below)
 *     in the mixture's precision (float for 32, double for 64) unless a
 *     function says float64.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *     asynchronous on that stream unless documented as synchronising.
 *   - The caller owns every buffer, including the workspace; the library
 *     allocates no device memory.  Workspace contents belong to the library
 *     between mlb_init_mixture and mlb_destroy.
 *   - Status codes, never exceptions; mlb_last_error() gives a message for
 *     the last failing call of the calling thread.
 *   - Calls on one handle must not overlap on different streams.
 *
 * D3Q19 velocity order: rest; +x, -x, +y, -y, +z, -z; then
 * (1,1,0), (-1,-1,0), (1,-1,0), (-1,1,0), (1,0,1), (-1,0,-1), (1,0,-1),
 * (-1,0,1), (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1).
 */
#ifndef MLB_H
#define MLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MLB_MAX_SPECIES 4
#define MLB_Q 19

typedef enum {
    MLB_OK = 0,
    MLB_EINVAL = -1,       /* invalid argument or parameter set                   */
    MLB_ENOMEM = -2,       /* workspace smaller than mlb_workspace_bytes()         */
    MLB_EHIP = -3,         /* a HIP runtime call failed                            */
    MLB_EUNSTABLE = -4,    /* the scheme is linearly unstable at the given state    */
    MLB_ENONFINITE = -5,   /* a conserved sum is not finite                        */
    MLB_ESTATE = -6,       /* call not valid in the handle's current state        */
    MLB_EUNSUPPORTED = -7  /* option not available for this precision or geometry */
} mlb_status;

enum { MLB_SCHEME_CN_J1 = 0, MLB_SCHEME_FE = 1 };
enum { MLB_TAIL_AUTO = 0, MLB_TAIL_DIRECT = 1, MLB_TAIL_SPECTRAL = 2 };
enum { MLB_OPT_TUNE = 1u,       /* time every float32 tiling (tile shape, block order, thread groups
                                   of the first gather), then the two fastest again, longer, with
                                   the plain and the sign-grouped shell loop and with the first
                                   gather on the tiling's shape and on its own 4x8x8 tiles, at
                                   init; keep the fastest */
       MLB_OPT_NO_GRAPH = 2u,   /* launch the passes eagerly instead of replaying a graph */
       MLB_OPT_NO_STABILITY_CHECK = 512u }; /* skip the linear-stability guard at init (studies of
                                           unstable schemes) */
/* Fixed float32 tiling instead of the default or tuned one (overrides
 * MLB_OPT_TUNE): tile shape 0 = 16x4x4, 1 = 8x8x4, 2 = 32x4x2 sites; block
 * order 0 = linear, 1 = XCD-chunked.  Reproducible profiles use it.  With
 * MLB_OPT_TILING, MLB_OPT_GATHER1_SPLIT(s) also fixes the thread groups per
 * site of the first gather (2 or 3; 3 when not given), and
 * MLB_OPT_GATHER1_SIGN_GROUPS(g) its shell loop: 0 = plain (also when not
 * given), 1 = sign-grouped (the points of a half-shell that differ only in
 * the signs of their y and z components summed together: the same sums of
 * eqs. potmeanforce, tensorgamma and viscousforce in another association,
 * equal to the plain loop to float32 rounding), and MLB_OPT_GATHER1_OWN_TILES(t)
 * the first gather's tiles: 0 = the tiling's shape (also when not given),
 * 1 = 4x8x8 sites (its 16-byte LDS reads free of bank conflicts at the
 * LDS size of 8x8x4; the sums are those of every other shape, bit for bit). */
#define MLB_OPT_TILING(shape, order) ((((uint32_t)(shape) + 1u) & 15u) << 4 | ((uint32_t)(order) & 1u) << 8)
#define MLB_OPT_GATHER1_SPLIT(s) (((uint32_t)(s) & 3u) << 10)
#define MLB_OPT_GATHER1_SIGN_GROUPS(g) (((uint32_t)(g) ? 2u : 1u) << 12)
#define MLB_OPT_GATHER1_OWN_TILES(t) (((uint32_t)(t) ? 2u : 1u) << 14)
enum { MLB_PART_MF = 1u, MLB_PART_TAIL = 2u, MLB_PART_DISS = 4u, MLB_PART_EXT = 8u,
       MLB_PART_ALL = 15u };

/* Problem statement (Sec. 2 and Sec. 3).  Lattice units. */
typedef struct {
    int32_t nx, ny, nz;            /* lattice size; x and z periodic                  */
    int32_t nspecies;              /* M, 1..4                                         */
    int32_t precision;             /* 32 (float) or 64 (double)                       */
    int32_t scheme;                /* MLB_SCHEME_CN_J1 (default) or MLB_SCHEME_FE     */
    int32_t tail_mode;             /* MLB_TAIL_*: AUTO = spectral in 32, direct in 64 */
    int32_t walls_y;               /* 0: y periodic; 1: solid layers y=0 and y=ny-1   */
    double tau;                    /* relaxation time, omega = 1/tau (one for all)    */
    double kT;                     /* must be 1/3 (the D3Q19 lattice's c_s^2)         */
    double mass[MLB_MAX_SPECIES];  /* m_a in [0.625, 2.5]: species a's equilibrium has
                                      thermal speed^2 kT/m_a in [2/15, 8/15] (see
                                      below); the barycentric velocity is mass-weighted */
    double sigma[MLB_MAX_SPECIES]; /* hard-core diameters sigma_aa; sigma_ab = mean   */
    double eps[MLB_MAX_SPECIES * MLB_MAX_SPECIES]; /* U_ab = -eps_ab (sigma_ab/r)^6 for
                                      sigma_ab < r <= rc_factor sigma_ab; 0 = off; row
                                      stride MLB_MAX_SPECIES, must be symmetric        */
    double rc_factor;              /* tail cutoff in units of sigma_ab                */
    double ext_force[MLB_MAX_SPECIES * 3]; /* uniform body force F^a per species      */
    double wall_ux[2];             /* x velocity of the wall at y=0 and at y=ny-1     */
} mlb_params;

typedef struct mlb_mixture_s *mlb_mixture;

/* Bytes of device workspace a mixture with these parameters needs (256-byte
 * aligned pointer required).  Returns 0 if the parameters are invalid (the
 * reason is in mlb_last_error()).  Conditions: 1 <= M <= 4, masses in [0.625, 2.5],
 * kT = 1/3, sigma > 0, every stencil offset smaller than the box edge in
 * each periodic direction. */
size_t mlb_workspace_bytes(const mlb_params *p);

/* Create a mixture: builds the stencil tables on the host, lays out the
 * workspace and sets the populations to psi_perp(n0, n0 u0, u) (eq.
 * prefactor with u the barycentric velocity), i.e. the local equilibrium of
 * the given fields.  n0 [M][N], u0 [M][3][N]: DEVICE float64 arrays
 * (species densities and velocities); values on solid layers are ignored.
 * Synchronises `stream`.  On success *out receives a handle that must be
 * released with mlb_destroy. */
mlb_status mlb_init_mixture(const mlb_params *p, void *workspace, size_t workspace_bytes,
                            const double *n0, const double *u0, void *stream, mlb_mixture *out);

/* As mlb_init_mixture, with options (MLB_OPT_TUNE, MLB_OPT_NO_GRAPH; see the
 * batched ensemble below).  With MLB_OPT_TUNE the float32 tile shape and
 * block order are chosen by timing full steps of every candidate, after
 * which the populations are reset to the initial state. */
mlb_status mlb_init_mixture_ex(const mlb_params *p, void *workspace, size_t workspace_bytes,
                               const double *n0, const double *u0, uint32_t options, void *stream,
                               mlb_mixture *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * mlb_init_mixture, but the workspace is a static device array of the
 * library, MLB_STATIC_WORKSPACE_BYTES bytes per GPU, held by every GPU the
 * library runs on until the process ends.  The caller still owns n0 and u0
 * (DEVICE float64, as mlb_init_mixture) and every output buffer of later
 * calls.  The array of the calling thread's current device is used.
 *   - MLB_ENOMEM if mlb_workspace_bytes(p) exceeds the maximum (no device
 *     work is done then); MLB_EINVAL for invalid parameters.
 *   - One such mixture per GPU at a time: while one is alive (until its
 *     mlb_destroy) a second call on the same GPU returns MLB_ESTATE.  The
 *     array keeps the contents of the last mixture that used it; the
 *     library initialises everything a mixture reads before reading it.
 *     Calls on one GPU that overlap (e.g. from two threads) race.
 *   - Neither this call nor mlb_step on the handle allocates device memory:
 *     the handle replays no graph (graph capture and instantiation
 *     allocate; mlb_set_graph(h, 1) turns them back on) and runs every pass
 *     on the caller's stream (no second stream).  Options of
 *     mlb_init_mixture_ex are not available (no autotuning). */
#define MLB_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
mlb_status mlb_init_mixture_static(const mlb_params *p, const double *n0, const double *u0, void *stream,
                                   mlb_mixture *out);

/* Linear stability of the step at uniform species densities n_bulk (HOST
 * float64 [M]) with velocities zero: the spectral radius of the step
 * linearised around that state (contact values, mean field, attractive
 * field, the dissipative pair form of eqs. gammaab, tensorgamma and
 * viscousforce under the chosen time scheme, collision and streaming) over
 * the wavevectors k = pi (i, j, l) / 4, i, j, l = 0..4, k = 0 excluded
 * (power iteration on the 19 M populations).  radius (HOST, may be NULL)
 * receives it.  MLB_EUNSTABLE if it exceeds 1 + 1e-6: the forward-Euler
 * friction grows once the friction rate per step is of order one.  Host
 * only; lattice size and walls do not enter.  mlb_init_mixture, _ex,
 * _static and mlb_init_batch run this guard on every system at its
 * box-mean densities (fluid sites) unless MLB_OPT_NO_STABILITY_CHECK is
 * given; states denser than the mean (e.g. a composition step) can still
 * be unstable where the mean is not. */
mlb_status mlb_check_stability(const mlb_params *p, const double *n_bulk, double *radius);

/* Tile shape and block order in use (see mlb_batch_tuning). */
mlb_status mlb_tuning(mlb_mixture h, int32_t *shape, int32_t *order, double *trial_ms);
/* As mlb_tuning, with the first gather's thread groups per site and the
 * time of every candidate (see mlb_batch_tuning_ex). */
mlb_status mlb_tuning_ex(mlb_mixture h, int32_t *shape, int32_t *order, int32_t *gather1_split, double *trial_ms);
/* The first gather's shell loop in use (see mlb_batch_tuning_groups). */
mlb_status mlb_tuning_groups(mlb_mixture h, int32_t *sign_groups, double *groups_ms);
/* The first gather's tile shape in use (see mlb_batch_tuning_gather1_shape). */
mlb_status mlb_tuning_gather1_shape(mlb_mixture h, int32_t *shape);

/* Advance the populations by nsteps >= 0 time steps of the kinetic equation
 * (Sec. 2, eq. evolution, with the field of Sec. 3). */
mlb_status mlb_step(mlb_mixture h, int32_t nsteps, void *stream);

/* Species densities n_a [M][N] and momentum densities n_a u_a [M][3][N]
 * (eq. colonna) of the current populations, into caller device buffers. */
mlb_status mlb_moments(mlb_mixture h, void *n_out, void *j_out, void *stream);

/* Force density n_a Phi_a [M][3][N] acting in the next step (eq. splitforce,
 * times n_a), restricted to the parts in `parts` (MLB_PART_* mask):
 * MF = hard-core mean field, TAIL = attractive field, EXT = n_a F^a,
 * DISS = drag + viscous force as applied by the time integrator. */
mlb_status mlb_forces(mlb_mixture h, void *nphi_out, uint32_t parts, void *stream);

/* Every intermediate field of one step evaluated on the current
 * populations (for per-kernel checks); NULL skips an output.
 * n [M][N], j [M][3][N], u [3][N] barycentric velocity, g [P][N] contact
 * values for the pairs (0,0),(0,1)..(0,M-1),(1,1).. (P = M(M+1)/2),
 * vhat [M][3][N] predicted velocities, H [M][3][N] predictor-time force,
 * nphi [M][3][N] total force density. */
mlb_status mlb_fields(mlb_mixture h, void *n, void *j, void *u, void *g, void *vhat, void *H,
                      void *nphi, void *stream);

/* Copy the populations [M][19][N] out of / into the mixture (device).
 * Checkpoint and resume: the populations and the step count are the whole
 * state of a run (every other field is derived from the populations at the
 * start of each step), so a mixture created with the same parameters, given
 * a saved f by mlb_set_populations and the saved count by
 * mlb_set_step_count, continues bit for bit as the run it was saved from. */
mlb_status mlb_get_populations(mlb_mixture h, void *f_out, void *stream);
mlb_status mlb_set_populations(mlb_mixture h, const void *f_in, void *stream);
/* Set the step count (the time stamp of recorded samples and the phase of
 * closure checks) for a resumed run; MLB_EINVAL if negative. */
mlb_status mlb_set_step_count(mlb_mixture h, int64_t steps);

/* Body force varying across the lattice rows (the external force F^a of
 * Sec. 2, eq. evolution, as a function of y; a y-periodic profile drives the
 * periodically modulated shear flow of Sec. 5.2, eq. ushape).  profile: HOST
 * float64 [M][3][ny]; from the next step on, species a at a site of row y
 * feels F^a(y) = ext_force[a] + profile[a][.][y] (the sum formed in float64,
 * then rounded to the mixture's precision).  NULL removes the profile
 * (back to the uniform ext_force).  Solid wall layers feel no force.
 * Synchronises `stream`.  MLB_EINVAL for non-finite values. */
mlb_status mlb_set_force_profile(mlb_mixture h, const double *profile, void *stream);

/* Global FP64 sums of the current state, accumulated on the GPU in float64:
 * mass[a] = sum_r n_a (particles of species a), mom[3a+d] = sum_r j_a,d
 * (number flux; the conserved momentum of eqs. continuity and
 * momentcomponent is sum_a m_a mom[3a+d]).  HOST outputs; synchronises the
 * stream.  Returns MLB_ENONFINITE if any sum is not finite. */
mlb_status mlb_conserved(mlb_mixture h, double *mass, double *mom, void *stream);

/* Composition-mode projection (Sec. 5.1): appends one float64 sample
 * (t, |sum_r (n_a - n_b) exp(-i 2 pi x / nx)|) for species pair (a, b) to the
 * handle's on-device time series (capacity mlb_series_capacity()).  With
 * b = -1 the sample is the mode of species a alone, |sum_r n_a exp(-i 2 pi x
 * / nx)|: the section-averaged mode of a tracer band, which decays at
 * D_eff q^2 (Sec. 5.2, eqs. c99 and taylordiff) and, unlike its variance,
 * does not depend on where the band sits in the periodic box. */
mlb_status mlb_record_mode(mlb_mixture h, int32_t a, int32_t b, void *stream);
/* Second-moment record for a tracer band (Sec. 5.2): appends (t, Var_x) of
 * the y,z-summed density of species a along x, in float64. */
mlb_status mlb_record_spread(mlb_mixture h, int32_t a, void *stream);
int32_t mlb_series_capacity(void);
/* Clear the time series (length 0). */
mlb_status mlb_series_reset(mlb_mixture h, void *stream);
/* Least-squares fit over the recorded samples with t >= t_min, in float64 on
 * the GPU.  kind 0 (mode): D = -slope(ln A, t) / (2 pi / nx)^2, the decay
 * 1/tau = D q^2 of Sec. 5.1, over the samples with t >= min(t_min, first t
 * at which A <= 0.1 A_first) and A >= 1e-6 A_first (A_first = the first
 * recorded amplitude): a fast mode is fitted before it reaches the rounding
 * floor of the densities.  kind 1 (spread): D = slope(Var, t) / 2.  Fewer
 * than two samples give NaN.  HOST output; synchronises the stream. */
mlb_status mlb_fit_series(mlb_mixture h, int32_t kind, double t_min, double *D_out, void *stream);
/* As mlb_fit_series, with the fit's quality: out5 (HOST, 5 doubles) =
 * D, the slope, the number of samples fitted, the coefficient of
 * determination R^2 of the line, and a well-conditioned flag (1.0 when the
 * samples lie on a straight line, R^2 >= 0.98, at least five of them, and a
 * mode fit's window stays above 1e-4 of the first amplitude; 0.0
 * otherwise: oscillating decay, or a mode lost in the rounding floor of the
 * densities).  Synchronises. */
mlb_status mlb_fit_series_ex(mlb_mixture h, int32_t kind, double t_min, double *out5, void *stream);
/* Copy the recorded series to HOST memory: t[count], v[count]; returns the
 * count through *count.  Synchronises. */
mlb_status mlb_get_series(mlb_mixture h, double *t, double *v, int32_t capacity, int32_t *count,
                          void *stream);

/* Per-pass GPU timing.  While profiling is on, mlb_step records a HIP event
 * pair around every kernel pass on the step's stream.  mlb_profile_end
 * synchronises that stream and returns, per pass k < MLB_NPASS, the summed
 * milliseconds ms[k] and the number of launches launches[k] (HOST arrays),
 * then turns profiling off.  Pass order: moments, contact values, spectral
 * tail, first gather, second gather + collision + streaming, closure
 * network (with a closure attached; its steps time their collision and
 * streaming under pass 4).  While profiling, the passes run one after the
 * other on `stream` (outside profiling the spectral tail overlaps the
 * contact values and the first gather on a second stream), and steps
 * launch eagerly. */
#define MLB_NPASS 6
mlb_status mlb_profile_begin(mlb_mixture h);
mlb_status mlb_profile_end(mlb_mixture h, double *ms, int32_t *launches, void *stream);
const char *mlb_pass_name(int32_t k);

/* Step loop as a graph: when enabled (the default), mlb_step captures two
 * consecutive steps once into a hipGraph (on a private capture stream) and
 * replays it on `stream`; odd remainders and profiled runs launch eagerly.
 * Results are identical either way. */
mlb_status mlb_set_graph(mlb_mixture h, int32_t enable);

/* Number of steps taken since init. */
int64_t mlb_step_count(mlb_mixture h);

/* Release the handle (host memory only; the caller frees the workspace). */
mlb_status mlb_destroy(mlb_mixture h);

/* Message of the calling thread's last failure ("" if none). */
const char *mlb_last_error(void);


/* ------------------------------------------------------------------------
 * Batched ensemble: many independent mixtures of uneven size, composition
 * and packing advanced together.  Every pass of a step is one launch over
 * the blocks of all systems (a block->system map in the workspace), and the
 * step loop is replayed as one captured hipGraph.  All systems share the
 * precision; attractive tails are summed directly (no spectral path) and
 * float32 batches without tails use the LDS-tile gathers.
 * ---------------------------------------------------------------------- */
typedef struct mlb_batch_s *mlb_batch;

/* Workspace bytes for `count` systems described by systems[0..count-1]; 0 if
 * any is invalid. */
size_t mlb_batch_workspace_bytes(const mlb_params *systems, int32_t count);
/* Create the ensemble.  n0[k], u0[k]: DEVICE float64 fields of system k
 * ([M_k][N_k], [M_k][3][N_k]); the arrays n0 and u0 themselves are HOST
 * arrays of `count` pointers.  Synchronises `stream`.  With MLB_OPT_TUNE the
 * autotuner runs full trial steps of every candidate and then restores the
 * initial populations. */
mlb_status mlb_init_batch(const mlb_params *systems, int32_t count, void *workspace, size_t workspace_bytes,
                          const double *const *n0, const double *const *u0, uint32_t options, void *stream,
                          mlb_batch *out);
mlb_status mlb_batch_step(mlb_batch h, int32_t nsteps, void *stream);
/* Per-system views: densities / momenta, populations of system k (device). */
mlb_status mlb_batch_moments(mlb_batch h, int32_t system, void *n_out, void *j_out, void *stream);
mlb_status mlb_batch_get_populations(mlb_batch h, int32_t system, void *f_out, void *stream);
/* Checkpoint and resume of an ensemble, as for one mixture: the populations
 * of system k (device, [M_k][19][N_k]) and the batch's step count. */
mlb_status mlb_batch_set_populations(mlb_batch h, int32_t system, const void *f_in, void *stream);
mlb_status mlb_batch_set_step_count(mlb_batch h, int64_t steps);
/* Append the (species 0 - species 1) mode amplitude of every system to its
 * own float64 time series (systems with one species are skipped). */
mlb_status mlb_batch_record_modes(mlb_batch h, void *stream);
/* Mode-decay fit of every system (kind 0 of mlb_fit_series): D_out is a
 * HOST array of `count` values.  Synchronises. */
mlb_status mlb_batch_fit(mlb_batch h, double t_min, double *D_out, void *stream);
/* As mlb_batch_fit with the quality of every fit: out5 is a HOST array of
 * count x 5 doubles laid out as mlb_fit_series_ex's. */
mlb_status mlb_batch_fit_ex(mlb_batch h, double t_min, double *out5, void *stream);
/* Recorded series of one system, as mlb_get_series (HOST outputs;
 * synchronises; an out-of-range system is MLB_EINVAL). */
mlb_status mlb_batch_get_series(mlb_batch h, int32_t system, double *t, double *v, int32_t capacity,
                                int32_t *count, void *stream);
/* The tile shape (0: 16x4x4, 1: 8x8x4, 2: 32x4x2) and block order (0:
 * linear, 1: XCD-chunked) in use; trial_ms (HOST, 6 values, may be NULL)
 * receives the measured milliseconds per step of each tile shape and order
 * (index 2 * shape + order; the faster of the first gather's two splits;
 * 0 when not measured).  -1 outputs for untiled handles. */
mlb_status mlb_batch_tuning(mlb_batch h, int32_t *shape, int32_t *order, double *trial_ms);
/* As mlb_batch_tuning, with the first gather's thread groups per tile site
 * (2 or 3) in use and trial_ms (HOST, 12 values, may be NULL) for every
 * candidate: index (split - 2) 6 + 2 shape + order. */
mlb_status mlb_batch_tuning_ex(mlb_batch h, int32_t *shape, int32_t *order, int32_t *gather1_split,
                               double *trial_ms);
/* The first gather's shell loop in use: *sign_groups = 1 for the
 * sign-grouped loop, 0 for the plain one, -1 for untiled handles; groups_ms
 * (HOST, may be NULL) receives the autotuner's milliseconds per step of the
 * chosen tiling with the sign-grouped loop (0 when not measured; the plain
 * loop's time is that tiling's trial_ms entry). */
mlb_status mlb_batch_tuning_groups(mlb_batch h, int32_t *sign_groups, double *groups_ms);
/* shape (HOST, may be NULL): the first gather's tile shape, 0..2 as in
 * MLB_OPT_TILING or 3 = its own 4x8x8 tiles; -1 when the float32 tiles are
 * not in use. */
mlb_status mlb_batch_tuning_gather1_shape(mlb_batch h, int32_t *shape);
mlb_status mlb_batch_profile_begin(mlb_batch h);
mlb_status mlb_batch_profile_end(mlb_batch h, double *ms, int32_t *launches, void *stream);
int64_t mlb_batch_step_count(mlb_batch h);
mlb_status mlb_batch_destroy(mlb_batch h);


/* ------------------------------------------------------------------------
 * Learned force closure.  A 3D convolutional network stands in for the
 * evaluation of the force densities N_a = n_a Phi_a of a binary mixture
 * (the field of Sec. 3, eq. (splitforce), with its Crank-Nicolson friction
 * as used by the collision of eq. (evolution)): from the local densities
 * and momentum densities it predicts both species' force fields, and a
 * step with a closure attached needs only the moments, the network and
 * the collision with streaming.
 *
 * Network: four 3x3x3 convolutions on the periodic lattice, channels
 * 14 -> 32 -> 32 -> 32 -> 6, SiLU s(z) = z / (1 + exp(-z)) after the first
 * three.  Input channels: 0..1 n_a / n_ref - 1; 2..7 j_a,d / j_ref at
 * 2 + 3a + d; 8..13 the lattice pressure gradients c_s^2 (n_a(r + e_d) -
 * n_a(r - e_d)) / 2 / f_ref at 8 + 3a + d (c_s^2 = 1/3, periodic wrap).
 * Output channels N_a,d / f_ref at index 3a + d.  Weights and activations
 * are bfloat16 with float32 accumulation on the matrix cores; Adam keeps
 * float32 master weights.
 *
 * Parameters (mlb_net_param_count() floats) travel as HOST float32 arrays,
 * layer by layer: W[co][ci][kz][ky][kx] (kz, ky, kx = offset + 1; the
 * layer computes y[co](r) = b[co] + sum W[co][ci][d + 1] x[ci](r + d) with
 * periodic wrap), then b[co].
 *
 * A network object is bound to one grid (nx, ny, nz); its workspace
 * (device memory, owned by the caller) holds parameters, Adam moments and
 * activation buffers, plus gradient buffers if `training` is 1.
 * ---------------------------------------------------------------------- */
typedef struct mlb_net_s *mlb_net;

size_t mlb_net_param_count(void);
/* Workspace bytes for a network on an nx x ny x nz grid (fewer than 2^29
 * sites, as for a mixture); 0 if invalid. */
size_t mlb_net_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t training);
/* Create with all parameters zero (asynchronous on `stream`). */
mlb_status mlb_net_create(int32_t nx, int32_t ny, int32_t nz, int32_t training, void *workspace,
                          size_t workspace_bytes, void *stream, mlb_net *out);
/* Load / read all parameters (HOST arrays, layout above).  Loading resets
 * the Adam moments and step count.  Both synchronise `stream`. */
mlb_status mlb_net_set_params(mlb_net net, const float *params, void *stream);
mlb_status mlb_net_get_params(mlb_net net, float *params, void *stream);
/* Input and output scales n_ref, j_ref, f_ref (all > 0; default 1). */
mlb_status mlb_net_set_scales(mlb_net net, double n_ref, double j_ref, double f_ref);
/* y [6][N] = network(x [14][N]); DEVICE float32, channel-first, x fastest. */
mlb_status mlb_net_forward(mlb_net net, const float *x, float *y, void *stream);
/* One training step on loss_weight times the mean squared error over all
 * N x 6 outputs: forward, backward, and (update != 0) one Adam step with
 * rate lr, b1 = 0.9, b2 = 0.999, eps = 1e-8.  x [14][N] and target [6][N]
 * are DEVICE float32; loss_weight > 0 (e.g. the reciprocal mean square of
 * the target, for a relative error).  loss (HOST, may be NULL) receives the
 * weighted loss before the update; grads (HOST, may be NULL,
 * mlb_net_param_count() floats, parameter layout) the gradients.  Asking
 * for either synchronises.  Needs training buffers (MLB_ESTATE
 * otherwise). */
mlb_status mlb_net_train_step(mlb_net net, const float *x, const float *target, float lr, float loss_weight,
                              int32_t update, double *loss, float *grads, void *stream);
/* Statistics of a training pool of `count` samples, x [count][14][N] and
 * targets t [count][6][N] (DEVICE float32, channel-first): out (HOST,
 * count + 1 doubles) receives out[0] = the mean square of the momentum
 * channels 2..7 of x over the pool and out[1 + s] = the mean square of
 * target s (float64 sums).  Synchronises. */
mlb_status mlb_net_pool_stats(mlb_net net, const float *x, const float *t, int32_t count, double *out, void *stream);
/* In place on the same pool: x's momentum channels 2..7 divided by j_div,
 * its gradient channels 8..13 and the targets by f_div (both > 0). */
mlb_status mlb_net_pool_rescale(mlb_net net, float *x, float *t, int32_t count, double j_div, double f_div,
                                void *stream);
/* err (HOST) = ||y - t||_2 / ||t||_2 over [6][N] DEVICE float32 arrays of the
 * net's grid, float64 sums (the closure check's measure).  Synchronises. */
mlb_status mlb_net_rel_error(mlb_net net, const float *y, const float *t, double *err, void *stream);
/* Adam steps taken since the last mlb_net_set_params. */
int32_t mlb_net_adam_steps(mlb_net net);
mlb_status mlb_net_destroy(mlb_net net);

/* Attach a closure network to a float32 binary periodic mixture (the net's
 * grid must equal the mixture's; net = NULL detaches).  Steps whose index
 * (the mlb_step_count before the step) is a multiple of check_every are
 * checks: they evaluate the exact force, use it, and compare it with the
 * network's, err = ||N_net - N_exact||_2 / ||N_exact||_2 over all sites,
 * species and components (float64 sums; synchronises the stream).  The
 * steps up to the next check take the network's force if err <= tol, and
 * the exact force otherwise (err > tol, or not finite: NaN in either
 * force); the next check decides again.  Steps before the first check
 * (attaching at an index that is not a multiple) take the network's force.
 * The handle keeps the network; the caller keeps it alive while attached. */
mlb_status mlb_set_closure(mlb_mixture h, mlb_net net, int32_t check_every, double tol);
/* checks made, step index of the first failed check (-1 if none), error of
 * the last check (-1 before the first), whether the last check passed (the
 * network's force is in use until the next check). */
mlb_status mlb_closure_stats(mlb_mixture h, int64_t *checks, int64_t *fallback_step, double *last_err,
                             int32_t *active);
/* steps taken with the network's force since mlb_set_closure, and failed
 * checks; HOST outputs (either may be NULL). */
mlb_status mlb_closure_usage(mlb_mixture h, int64_t *net_steps, int64_t *failed_checks);
/* A training pair from the current state (populations are not changed):
 * x_out [14][N] the network input with `net`'s scales and target_out [6][N]
 * the exact force divided by f_ref; DEVICE float32.  Needs a float32
 * binary mixture on `net`'s grid. */
mlb_status mlb_closure_sample(mlb_mixture h, mlb_net net, float *x_out, float *target_out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MLB_H */
