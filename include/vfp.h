/*
 * vfp.h -- C ABI of libvfp.so, an MI355X (gfx950) implementation of one time
 * step of the discretised Vlasov-Fokker-Planck split map of Schoenfeldt et
 * al., "A Parallelized Vlasov-Fokker-Planck-Solver for Desktop PCs"
 * (arXiv:1611.05293).
 *
 * The state is the longitudinal phase-space density psi(q, p) on an n x n
 * node grid (Sec. III.A, Eq. "coordinate trafo"): q_i = q_min + i*dq,
 * p_j = p_min + j*dp, dq = (q_max - q_min)/(n - 1), dp likewise.  Every
 * psi array crossing this ABI is row-major psi[i*n + j] with the p index j
 * fastest (Sec. III.B: z = N_y*x + y), FP64, in host memory.
 *
 * One step (Sec. III.B, f = f_rot + f_kick + f_damp,diff) with
 * dtheta = 2*pi/steps_per_period radians:
 *   1. profile   rho_i = dp * sum_j psi_ij                      (Sec. II.B)
 *   2. wake      V_i = S * sum_j w[(i - j) mod M] rho_j,
 *                w[l] = (1/M) sum_k Z_k e^{+2 pi i k l/M}     (Eq. "wakepotential")
 *   3. rotation  pull from (q c - p s, q s + p c), c = cos dtheta, s = sin dtheta,
 *                K x K Lagrange interpolation (standard), or the Manhattan
 *                drift + RF kick pair of 1-D interpolations      (Sec. III.A-B)
 *   4. kick      pull along p from p + V_i * dtheta              (Sec. III.B)
 *   5. damping/diffusion  psi += beta*dtheta * [D1(p psi) + D2 psi], D1 the
 *                derivative of the cubic interpolant (Eq. "cubic diff"),
 *                D2 the 3-point second difference; zero outside the grid
 *   6. renormalisation of the charge dq*dp*sum(psi) to its initial value Q0
 *                (optional; FP64 on the device).
 * rho and V are taken from psi at the start of the step (the collective
 * force is constant over a small step, Sec. II.A).
 *
 * Threading and ownership: a handle is used from one host thread at a time.
 * Every array passed in is deep-copied before the call returns; output
 * arrays are caller-owned host memory of the stated size.  A workspace, if
 * given, is device memory of at least vfp_workspace_size() bytes that must
 * outlive the handle; with ws == NULL the library allocates and frees its
 * own.  The stream is the caller's hipStream_t; with NULL the handle creates
 * a non-blocking stream of its own (graphs cannot be captured on the null
 * stream).
 * Stepping calls (vfp_step, vfp_batch_step) only enqueue work on that
 * stream: they never allocate, never synchronise and never capture or
 * instantiate a graph.  The work layout of every retirement phase and the
 * graphs are prepared by create and by the calls that change the set of
 * simulations, their state or the tuning (set_psi, seed, haissinski, record,
 * set_tuning, kernel_timing, autotune), which may allocate and synchronise.
 * The query calls (profile, csr_power, moments, get_psi, read_record)
 * synchronise the stream.
 *
 * Errors: every int-returning call returns one of the VFP_* codes and never
 * aborts; vfp_last_error() returns a thread-local description of the last
 * failure.  Invalid parameters are rejected at create time.
 */
#ifndef VFP_H
#define VFP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    VFP_OK = 0,
    VFP_EINVAL = -1,     /* invalid argument                                  */
    VFP_ENOMEM = -2,     /* device allocation failed or workspace too small   */
    VFP_EDEVICE = -3,    /* HIP runtime error, or non-finite state detected    */
    VFP_ESTATE = -4,     /* call not valid in the handle's current state       */
    VFP_EUNSTABLE = -5   /* explicit damping step unstable for these settings  */
};

/* Arithmetic of psi and of the wake (Sec. IV.A compares binary32/binary64
 * and fixed point with a chosen number of fractional bits). */
enum {
    VFP_FP64 = 0,        /* psi, rotation, kick, damping and wake in FP64          */
    VFP_FP32 = 1,        /* psi and the step in FP32, wake FP32 on the vector ALU  */
    VFP_MIXED_BF16 = 2,  /* psi FP32; wake on BF16 matrix cores, hi/lo split       */
    VFP_MIXED_FP16 = 3,  /* psi FP32; wake on FP16 matrix cores, hi/lo split       */
    VFP_FIXED = 4        /* psi as 64-bit fixed point with fix_bits fractional bits
                            (Sec. III.A, last paragraph): FP64 coefficients
                            rounded to fix_bits, weighted sums exact in 128-bit
                            integers rounded once, exact integer charge; wake
                            FP64 */
};
/* Charge renormalisation, moments and CSR power are FP64 in every mode. */

enum {
    VFP_ROT_STANDARD = 0,   /* 2-D K x K tensor interpolation (Sec. III.B)        */
    VFP_ROT_MANHATTAN = 1   /* drift then RF kick, two 1-D interpolations         */
};

typedef struct vfp_params {
    int32_t n;                /* grid points per axis, 16..4096                    */
    double  q_min, q_max;     /* node range in q (bunch length units)              */
    double  p_min, p_max;     /* node range in p (energy spread units)             */
    int32_t steps_per_period; /* >= 1; dtheta = 2*pi/steps_per_period               */
    double  beta;             /* damping/diffusion coefficient per radian, >= 0    */
    int32_t interp;           /* K = 3 (quadratic) or 4 (cubic), Sec. III.A        */
    int32_t clamp;            /* 1: clip interpolants to the bracketing nodes'
                                 range (Eq. "clamping"); 0: plain interpolation  */
    int32_t renormalize;      /* 1: keep the charge at Q0 each step                */
    int32_t precision;        /* VFP_FP64 / VFP_FP32 / VFP_MIXED_*                  */
    int32_t padding;          /* M = padding*n wake samples, >= 2                   */
    int32_t rotation;         /* VFP_ROT_*                                          */
    const double *z_re;       /* floor(M/2)+1 impedance samples Z_k, k = 0..M/2 at  */
    const double *z_im;       /* kappa_k = 2*pi*k/(M*dq); both NULL: zero current.  */
                              /* Im Z_0 and Im Z_{M/2} are ignored (Hermitian).     */
    double  z_scale;          /* S in V = S * (w conv rho) (normalised current)    */
    const double *psi0;       /* n*n initial density, index i*n+j (p fastest);
                                 NULL: unit Gaussian.  Finite, within the binary32
                                 range unless VFP_FP64, and with a positive,
                                 finite sum (Q0 > 0), else VFP_EINVAL.            */
    int64_t max_steps;        /* batch only: the simulation stops advancing after
                                 this many steps (0: never)                        */
    int32_t z_model;          /* VFP_Z_*: where Z_k comes from.  VFP_Z_SAMPLES:
                                 the z_re/z_im arrays above; otherwise Z_k is
                                 computed on the device at the same kappa_k and
                                 z_re/z_im must be NULL (Sec. II.B models).      */
    double  z_shield;         /* VFP_Z_PARALLEL_PLATES: shielding parameter
                                 Pi > 0 (P = Pi^(2/3)); ignored otherwise         */
    int32_t fix_bits;         /* VFP_FIXED: fractional bits F, 16..59 (psi0 then
                                 bounded by |psi| < 2^(61-F)); ignored otherwise  */
} vfp_params;

/* Impedance models of Sec. II.B in normalised form (kappa = k sigma_z0, all
 * physical prefactors in z_scale):
 *   free space:       Z = Gamma(2/3) 3^(-1/3) kappa^(1/3) (sqrt(3)/2 + i/2)
 *   parallel plates:  Z = 4 pi^2 2^(1/3) P kappa^(-1/3)
 *                         sum_{p>=0} [Ai'(u_p) Ci'(u_p) + u_p Ai(u_p) Ci(u_p)],
 *                     Ci = Ai - i Bi, u_p = pi^2 (2p+1)^2 2^(-2/3) P^2 kappa^(-4/3)
 * Z_0 = 0 in both (the mean of the wake is not a force). */
enum {
    VFP_Z_SAMPLES = 0,          /* caller-supplied samples z_re/z_im (or none)      */
    VFP_Z_PARALLEL_PLATES = 1,  /* shielded CSR, Pi = z_shield                       */
    VFP_Z_FREE_SPACE = 2        /* unshielded CSR                                    */
};

typedef struct vfp_batch vfp_batch;   /* a set of independent simulations      */
typedef struct vfp_batch vfp_sim;     /* a single simulation: a set of one     */

/* Defaults: n = 256, [-8, 8]^2, 1000 steps per period, beta = 1e-3, K = 4,
 * no clamp, renormalize = 1, VFP_FP32, padding = 2, standard rotation,
 * zero current, Gaussian start, max_steps = 0, VFP_Z_SAMPLES, z_shield = 1,
 * fix_bits = 44. */
void vfp_params_init(vfp_params *p);

/* The impedance samples a simulation with z_model = `model` uses: Z_k at
 * kappa_k = 2*pi*k/(M*dq), k = 0..M/2, M = padding*n, dq = (q_max-q_min)/(n-1)
 * (Sec. II.B; the sampling of the wake's discrete convolution, Sec. III.C),
 * computed in FP64 on the current device with the same code the create calls
 * use.  z_re/z_im are HOST arrays of M/2+1 doubles owned by the caller.
 * model: VFP_Z_PARALLEL_PLATES (Pi > 0) or VFP_Z_FREE_SPACE.  Synchronous.
 * Returns VFP_EINVAL for bad arguments, VFP_EDEVICE on a HIP failure. */
int vfp_impedance_samples(int32_t model, int32_t n, int32_t padding, double q_min, double q_max,
                          double Pi, double *z_re, double *z_im);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * samples as vfp_impedance_samples, bit for bit, with the device buffer taken
 * from a static array of the library instead of hipMalloc.  Each GPU the
 * library runs on holds its own copy of that array (2 * VFP_NOALLOC_MAX_SAMPLES
 * doubles, 256 KiB) until the process ends; its device address is looked up
 * on the first call on each device.  Arguments, layout and ownership as
 * vfp_impedance_samples; additionally returns VFP_EINVAL when
 * padding*n/2 + 1 > VFP_NOALLOC_MAX_SAMPLES.  Calls no hipMalloc/hipFree.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (from several host threads) race and must be serialised by the caller. */
#define VFP_NOALLOC_MAX_SAMPLES 16385
int vfp_impedance_samples_noalloc(int32_t model, int32_t n, int32_t padding, double q_min,
                                  double q_max, double Pi, double *z_re, double *z_im);

/* sizeof(vfp_params) as compiled into the library (binding layout check). */
size_t vfp_params_sizeof(void);

/* Device bytes a workspace must hold for `count` simulations described by
 * p[0..count-1].  Returns VFP_EINVAL for invalid parameters. */
int vfp_workspace_size(const vfp_params *p, int32_t count, size_t *bytes);

/* ---------------------------------------------------------------------- */
/* Plain per-simulation form: one simulation, launched on its own.          */
/* ---------------------------------------------------------------------- */

/* Validates p (see vfp_params; also the explicit-Euler bound
 * beta*dtheta/dp^2 <= 0.25, else VFP_EUNSTABLE), builds the wake table
 * from Z on the device and uploads psi0.  Q0 = dq*dp*sum(psi0). */
int vfp_create(const vfp_params *p, void *hip_stream, void *workspace, size_t ws_bytes,
               vfp_sim **out);

/* Enqueue nsteps >= 0 steps on the stream; no host synchronisation. */
int vfp_step(vfp_sim *sim, int64_t nsteps);

/* rho[0..n-1] = dp * sum_j psi_ij of the current (renormalised) state. */
int vfp_profile(vfp_sim *sim, double *rho);

/* CSR power of the current state (Sec. IV.C): *power = sum_i rho_i V_i,
 * equal by Parseval to (S/M) sum_k Re Z_k |rho~_k|^2 over all M bins.  The
 * FP64 wake is used for this diagnostic in every precision mode. */
int vfp_csr_power(vfp_sim *sim, double *power);

/* out = {Q, <q>, sigma_q, <p>, sigma_p} of the current state (FP64). */
int vfp_moments(vfp_sim *sim, double out[5]);

/* Copy the current state out (n*n FP64) / replace it (resets Q0 to the
 * charge of the new psi and the step counter to 0; psi is checked as psi0
 * is, VFP_EINVAL otherwise). */
int vfp_get_psi(vfp_sim *sim, double *psi);
int vfp_set_psi(vfp_sim *sim, const double *psi);

/* Time series (the paper's `outstep` output): after every `every`-th step a
 * row {step, Q, <q>, sigma_q, <p>, sigma_p, P} of the state after that
 * step is written on the device, up to `cap` rows (every = 0 stops).
 * vfp_read_record copies rows*7 doubles into out (out may be NULL to only
 * query *rows). */
int vfp_record(vfp_sim *sim, int32_t every, int64_t cap);
int vfp_read_record(vfp_sim *sim, double *out, int64_t *rows);

/* Steps taken since create / the last set_psi. */
int vfp_steps_done(vfp_sim *sim, int64_t *steps);

void vfp_destroy(vfp_sim *sim);
const char *vfp_last_error(void);

/* ---------------------------------------------------------------------- */
/* Batched form: `count` independent simulations (a current or shielding   */
/* scan; grid sizes and steps per period may differ) advanced together.    */
/* One tick advances every active simulation by one of its own steps.  The */
/* FP32-storage forms (VFP_FP32 and the mixed forms) run one of two tick   */
/* forms (vfp_batch_set_tuning): split, a wake launch then the fused step  */
/* launch; or fused, ONE launch per tick whose wake tiles (first in the    */
/* launch) compute each simulation's wake while its work units stage and   */
/* rotate their strips; a unit waits for its simulation's tiles only      */
/* before it kicks.                                                        */
/* VFP_FP64 and VFP_FIXED compute the wake slice of each strip inside      */
/* their one step launch.  The simulations are split in stream groups     */
/* (vfp_batch_set_streams) whose launches overlap.  Ticks are replayed     */
/* from hipGraphs prepared outside the step call.  A simulation with       */
/* max_steps > 0 retires after that many steps; retirements switch between */
/* work layouts prepared in advance.  All simulations of a batch share     */
/* interp, clamp, precision and rotation.                                  */
/* ---------------------------------------------------------------------- */
int vfp_batch_create(const vfp_params *p, int32_t count, void *hip_stream, void *workspace,
                     size_t ws_bytes, vfp_batch **out);
int vfp_batch_step(vfp_batch *b, int64_t nticks);
int vfp_batch_profile(vfp_batch *b, int32_t i, double *rho);
int vfp_batch_csr_power(vfp_batch *b, double *power /* count */);
int vfp_batch_moments(vfp_batch *b, double *out /* 5*count */);
int vfp_batch_get_psi(vfp_batch *b, int32_t i, double *psi);
int vfp_batch_set_psi(vfp_batch *b, int32_t i, const double *psi);
int vfp_batch_record(vfp_batch *b, int32_t every, int64_t cap);
int vfp_batch_read_record(vfp_batch *b, int32_t i, double *out, int64_t *rows);
int vfp_batch_steps_done(vfp_batch *b, int32_t i, int64_t *steps);
void vfp_batch_destroy(vfp_batch *b);

/* The stored density of simulation i exactly as held on the device, for
 * bit-exact checks and checkpoints: n*n values of the storage type (double
 * for VFP_FP64, int64_t raw values with fix_bits fractional bits for
 * VFP_FIXED, float otherwise; index i*n+j) copied to the host buffer out,
 * which must hold n*n*8 bytes (n*n*4 for the FP32 storage).  The physical
 * density is *s times the stored one; s is Q0 / Q of the stored density
 * (1 with renormalize = 0), computed from the exact integer charge in the
 * fixed-point form.  Synchronises the batch's stream. */
int vfp_batch_get_raw(vfp_batch *b, int32_t i, void *out, double *s);

/* Launch tuning: columns per work unit are chosen per grid size.  cells is
 * the number of phase-space cells one workgroup owns (0 restores the
 * built-in choice); use_graph = 0 launches every tick directly; staged
 * selects the FP32-storage step kernel and tick form: 0 the generic kernel
 * (taps through the caches; the wake in a launch of its own), 1 the
 * LDS-staged kernel with a separate wake launch per tick (split), 2 the
 * LDS-staged kernel with the one-launch tick (fused).  The three give the
 * same arithmetic definition with different evaluation orders; 1 and 2 give
 * bit-identical results.  Other values return VFP_EINVAL.  Grids the staged
 * kernel does not take (n % 4 != 0, rotation source more than 2 cells away)
 * use the generic kernel either way.  A new batch uses cells_per_unit 8192
 * (1024 for VFP_FP64 and 2048 for VFP_FIXED, whose strips take 16 bytes per
 * cell of LDS; for the FP32-storage forms narrowed while the batch would
 * have fewer than 2560 work units, down to strips of two columns on its
 * largest grid), graph replay, and staged = 2 for batches of at most 2 Mi
 * cells per tick (a separate wake launch would sit on the tick's critical
 * path) or staged = 1 above; 0 restores the default cells.
 * Synchronises the stream and prepares the work layout. */
int vfp_batch_set_tuning(vfp_batch *b, int32_t cells_per_unit, int32_t use_graph, int32_t staged);

/* Stream groups: with groups = 2, 3 (the default) or 4 the active
 * simulations are split in that many parts of about equal cell count (never
 * more parts than simulations), each advanced on its own stream (the others
 * are created by the library, default priority), so that the launches of one
 * part overlap the others' and the tail of each launch is filled; the
 * streams are joined before every record and at the end of every step call.
 * groups = 1 advances all simulations on the batch's stream.  Results are
 * identical either way.  Per-kernel timing (vfp_batch_kernel_timing) uses
 * one group.  Returns VFP_EINVAL for groups outside [1, 4]; synchronises the
 * stream and prepares the work layout. */
int vfp_batch_set_streams(vfp_batch *b, int32_t groups);

/* The tuning in force: cells per unit, graph replay on/off, kernel layout
 * (any output pointer may be NULL). */
int vfp_batch_get_tuning(vfp_batch *b, int32_t *cells_per_unit, int32_t *use_graph, int32_t *staged);

/* CSR spectrum of simulation i's current state (Sec. IV.C, P(t,k) ~ Re Z_k
 * |rho~(k,t)|^2): out[k], k = 0..M/2 (floor(M/2)+1 values, FP64), with
 * rho~ the DFT of the zero-padded profile and the bins 0 < k < M/2 counting
 * both k and M-k, so that sum_k out[k] = the CSR power.  Synchronises.
 * VFP_ESTATE when the simulation has no impedance. */
int vfp_batch_csr_spectrum(vfp_batch *b, int32_t i, double *out);
int vfp_csr_spectrum(vfp_sim *sim, double *out);

/* Haissinski start (Appendix A, the equilibrium below threshold): replace
 * simulation i's state by rho(q) g(p) with rho ~ exp(-q^2/2 - U(q)),
 * U' = V[rho] its own wake potential, dq*sum(rho) = Q0 (unchanged), and g
 * the unit Gaussian in p normalised on the grid.  Solved on the device in
 * FP64 by `iters` damped fixed-point iterations rho <- (1-alpha) rho +
 * alpha F(rho) from the Gaussian (0 < alpha <= 1).  Step counter restarts. */
int vfp_batch_haissinski(vfp_batch *b, int32_t i, int32_t iters, double alpha);
int vfp_haissinski(vfp_sim *sim, int32_t iters, double alpha);

/* Adiabatic chaining (Appendix A: the final distribution of one run starts
 * the next): simulation dst takes simulation src's current state on the
 * device, including its charge Q0; dst's step counter restarts at 0 and a
 * retired dst rejoins the batch.  Both must have the same grid. */
int vfp_batch_seed(vfp_batch *b, int32_t dst, int32_t src);

/* The wake V[0..n-1] that the latest step of simulation i used (taken from
 * the state at the start of that step), as computed by that step's own
 * arithmetic (FP64/FP32 Toeplitz row slice or the matrix-core product),
 * returned as FP64.  For comparing each precision form's wake with the FP64
 * definition.  VFP_ESTATE when the simulation has no impedance; the values
 * are undefined before the first step.  FP64 mode keeps it in FP32. */
int vfp_batch_last_wake(vfp_batch *b, int32_t i, double *V);

/* Per-kernel timing with HIP events on the handle's stream: while enabled,
 * ticks are launched directly (not from a graph) and every step launch (the
 * fused tick) and every separate wake launch is bracketed by a pair of
 * events, from a pool of 3072 events made when timing is enabled (launches
 * beyond the pool run untimed).  Enabling (or disabling) clears the
 * accumulated events.
 * vfp_batch_kernel_times synchronises and returns
 * out = {step kernel total ms, step launches, wake kernel total ms, wake launches}. */
int vfp_batch_kernel_timing(vfp_batch *b, int32_t enable);
int vfp_batch_kernel_times(vfp_batch *b, double out[4]);

/* Autotuner: times `ticks` ticks for every candidate (cells per unit in
 * {2048, 4096, 8192, 16384} and, for FP32 storage, the split and fused tick
 * forms; {1024, 2048, 4096, 8192} with the generic kernel for the 8-byte
 * forms) with HIP events on the batch's stream in the batch's stream groups,
 * keeps the fastest and returns it.  The state is saved and restored around
 * the trials. */
int vfp_batch_autotune(vfp_batch *b, int32_t ticks, int32_t *chosen_cells, int32_t *chosen_staged);

/* Architecture name of the current device (e.g. "gfx950:sramecc+:xnack-"),
 * the key of autotuning caches. */
int vfp_device_arch(char *name, int32_t len);

#ifdef __cplusplus
}
#endif
#endif /* VFP_H */
