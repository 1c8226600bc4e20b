/*
 * vfp_oracle.c -- plain FP64 CPU reference for one time step of the
 * discretised Vlasov-Fokker-Planck (VFP) split map of
 * Schoenfeldt et al., "A Parallelized Vlasov-Fokker-Planck-Solver for
 * Desktop PCs" (arXiv:1611.05293).
 *
 * TEST INFRASTRUCTURE.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the HIP library; the two are written separately
 * from the paper.
 *
 * Every routine is a direct transcription of a definition: plain loops,
 * FP64 throughout, no blocking, no fusion, no reordering beyond what the
 * definition states.  Compile with -O2 -ffp-contract=off so that no FMA
 * contraction changes the rounding of the written expressions.
 * OpenMP is used only across independent columns or simulations.
 *
 * Conventions (the paper leaves these open; the same readings are listed
 * in the design notes of the repository):
 *   grid   q_i = q_min + i*dq, p_j = p_min + j*dp, dq = (q_max-q_min)/(n-1)
 *          (Sec. III.A, Eq. "coordinate trafo": nodes at integer grid
 *          coordinates, both range ends are nodes);
 *   layout psi[i*n + j], p (index j) fastest (Sec. III.B: z = N_y*x + y);
 *   time   one step turns the phase space by dtheta = 2*pi/steps_per_period
 *          radians; the kick moves p by -V*dtheta and the Fokker-Planck
 *          coefficient per step is beta*dtheta (Eq. VFP with theta read
 *          as synchrotron phase in radians);
 *   boundary psi is zero outside the grid for every sub-step.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* number of OpenMP threads a parallel loop of the oracle uses */
int vfo_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* set the thread count of the parallel loops (timing on 1 core vs all) */
void vfo_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

typedef struct {
    int    n;                 /* grid points per axis                          */
    double q_min, q_max;      /* node range in q                               */
    double p_min, p_max;      /* node range in p                               */
    int    steps_per_period;  /* dtheta = 2*pi / steps_per_period             */
    double beta;              /* Fokker-Planck coefficient per radian          */
    int    interp;            /* K = 3 (quadratic) or 4 (cubic)                */
    int    clamp;             /* 1: clamp interpolants to bracketing nodes     */
    int    renormalize;       /* 1: rescale psi to the initial charge Q0       */
    int    padding;           /* M = padding * n wake samples                  */
    double z_scale;           /* S: V = S * (w conv rho)                       */
    int    rotation;          /* 0: standard 2-D rotation, 1: Manhattan        */
} vfo_params;

static double grid_dq(const vfo_params *p) { return (p->q_max - p->q_min) / (p->n - 1); }
static double grid_dp(const vfo_params *p) { return (p->p_max - p->p_min) / (p->n - 1); }
static double step_angle(const vfo_params *p) { return 2.0 * M_PI / (double)p->steps_per_period; }

/* ------------------------------------------------------------------ */
/* Lagrange interpolation (Sec. III.A, Eqs. "interpolation" and        */
/* "lagrange-basis-polynomials").  Stencil nodes m + o_k with          */
/* o_k = k - floor((K-1)/2), k = 0..K-1; basis                          */
/* l_k(t) = prod_{k' != k} (t - o_k') / (o_k - o_k').                   */
/* ------------------------------------------------------------------ */
static int stencil_offset(int K, int k) { return k - (K - 1) / 2; }

void vfo_lagrange_weights(int K, double t, double *l)
{
    for (int k = 0; k < K; ++k) {
        double v = 1.0;
        for (int kk = 0; kk < K; ++kk) {
            if (kk == k) continue;
            v *= (t - stencil_offset(K, kk)) /
                 (double)(stencil_offset(K, k) - stencil_offset(K, kk));
        }
        l[k] = v;
    }
}

/* value of the grid function at integer node (i, j); zero outside the grid */
static double node(const double *psi, int n, int i, int j)
{
    if (i < 0 || i >= n || j < 0 || j >= n) return 0.0;
    return psi[(size_t)i * n + j];
}

/* 1-D interpolation of column i at fractional p-coordinate r (Eq.
 * "interpolation"): m = floor(r), t = r - m, sum_k l_k(t) f(m + o_k).
 * With clamping (Eq. "clamping", read as a clip to the range spanned by
 * the two bracketing nodes f(m), f(m+1)). */
static double interp_column(const double *psi, int n, int K, int clamp, int i, double r)
{
    double m = floor(r);
    double t = r - m;
    int mi = (int)m;
    double l[4];
    vfo_lagrange_weights(K, t, l);
    double v = 0.0;
    for (int k = 0; k < K; ++k) v += l[k] * node(psi, n, i, mi + stencil_offset(K, k));
    if (clamp) {
        double a = node(psi, n, i, mi), b = node(psi, n, i, mi + 1);
        double lo = a < b ? a : b, hi = a < b ? b : a;
        if (v < lo) v = lo;
        if (v > hi) v = hi;
    }
    return v;
}

/* same along q: row j, fractional q-coordinate r */
static double interp_row(const double *psi, int n, int K, int clamp, int j, double r)
{
    double m = floor(r);
    double t = r - m;
    int mi = (int)m;
    double l[4];
    vfo_lagrange_weights(K, t, l);
    double v = 0.0;
    for (int k = 0; k < K; ++k) v += l[k] * node(psi, n, mi + stencil_offset(K, k), j);
    if (clamp) {
        double a = node(psi, n, mi, j), b = node(psi, n, mi + 1, j);
        double lo = a < b ? a : b, hi = a < b ? b : a;
        if (v < lo) v = lo;
        if (v > hi) v = hi;
    }
    return v;
}

/* ------------------------------------------------------------------ */
/* Projection (Sec. II.B): bunch profile rho(q_i) = dp * sum_j psi_ij  */
/* ------------------------------------------------------------------ */
void vfo_profile(const vfo_params *p, const double *psi, double *rho)
{
    const int n = p->n;
    const double dp = grid_dp(p);
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += psi[(size_t)i * n + j];
        rho[i] = dp * s;
    }
}

/* total charge Q = dq * dp * sum_ij psi_ij */
double vfo_charge(const vfo_params *p, const double *psi)
{
    const size_t nn = (size_t)p->n * p->n;
    double s = 0.0;
    for (size_t z = 0; z < nn; ++z) s += psi[z];
    return grid_dq(p) * grid_dp(p) * s;
}

/* ------------------------------------------------------------------ */
/* Wake kernel (Sec. II.B, Eq. "wakepotential"; Sec. III.B on the       */
/* Hermitian transform): w[l] = (1/M) sum_{k=0}^{M-1} Z_k e^{+2 pi i k l/M}*/
/* with Z_{M-k} = conj(Z_k); Z_0 and Z_{M/2} taken as their real parts. */
/* Input: the floor(M/2)+1 samples k = 0..floor(M/2).  Output: w[0..M-1].*/
/* ------------------------------------------------------------------ */
void vfo_wake_kernel(int M, const double *z_re, const double *z_im, double *w)
{
    for (int l = 0; l < M; ++l) {
        double acc = 0.0;
        for (int k = 0; k < M; ++k) {
            double zr, zi;
            if (k == 0 || 2 * k == M) { zr = z_re[k]; zi = 0.0; }
            else if (2 * k < M)      { zr = z_re[k]; zi = z_im[k]; }
            else                     { zr = z_re[M - k]; zi = -z_im[M - k]; }
            /* angle 2*pi*k*l/M reduced exactly modulo M */
            long long kl = ((long long)k * l) % M;
            double phi = 2.0 * M_PI * (double)kl / (double)M;
            acc += zr * cos(phi) - zi * sin(phi);   /* Re(Z_k e^{i phi}) */
        }
        w[l] = acc / (double)M;
    }
}

/* Wake potential (Sec. II.B, convolution of the wake function with the
 * profile): V[i] = S * sum_{j=0}^{n-1} w[(i - j) mod M] rho[j]. */
void vfo_wake(const vfo_params *p, const double *w, const double *rho, double *V)
{
    const int n = p->n;
    const int M = p->padding * n;
    for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int j = 0; j < n; ++j) {
            int l = ((i - j) % M + M) % M;
            acc += w[l] * rho[j];
        }
        V[i] = p->z_scale * acc;
    }
}

/* ------------------------------------------------------------------ */
/* Standard rotation (Sec. III.B, "standard rotation"; interpolation    */
/* Sec. III.A).  The unperturbed Hamiltonian H = (q^2+p^2)/2 turns the  */
/* phase space clockwise: dq/dtheta = p, dp/dtheta = -q.  The new value */
/* at node (q_i, p_j) is pulled from the point that arrives there,      */
/* (q0, p0) = (q c - p s, q s + p c), c = cos dtheta, s = sin dtheta,   */
/* by the K x K tensor product of the 1-D Lagrange weights.             */
/* ------------------------------------------------------------------ */
void vfo_rotate(const vfo_params *p, const double *src, double *dst)
{
    const int n = p->n, K = p->interp;
    const double dq = grid_dq(p), dp = grid_dp(p);
    const double th = step_angle(p);
    const double c = cos(th), s = sin(th);
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        const double q = p->q_min + i * dq;
        for (int j = 0; j < n; ++j) {
            const double pp = p->p_min + j * dp;
            const double q0 = q * c - pp * s;
            const double p0 = q * s + pp * c;
            const double rx = (q0 - p->q_min) / dq;   /* Eq. coordinate trafo */
            const double ry = (p0 - p->p_min) / dp;
            const double mx = floor(rx), my = floor(ry);
            const int ix = (int)mx, iy = (int)my;
            double lx[4], ly[4];
            vfo_lagrange_weights(K, rx - mx, lx);
            vfo_lagrange_weights(K, ry - my, ly);
            double v = 0.0;
            for (int a = 0; a < K; ++a)
                for (int b = 0; b < K; ++b)
                    v += lx[a] * ly[b] * node(src, n, ix + stencil_offset(K, a), iy + stencil_offset(K, b));
            if (p->clamp) {
                /* clip to the range of the four bracketing nodes */
                double lo = node(src, n, ix, iy), hi = lo;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        double f = node(src, n, ix + a, iy + b);
                        if (f < lo) lo = f;
                        if (f > hi) hi = f;
                    }
                if (v < lo) v = lo;
                if (v > hi) v = hi;
            }
            dst[(size_t)i * n + j] = v;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Manhattan (symplectic) rotation (Sec. III.B): an energy-dependent    */
/* drift followed by a position-dependent RF kick, each a 1-D           */
/* interpolation.  Forward map: q1 = q + dtheta*p, p1 = p - dtheta*q1.  */
/* Pulled in two 1-D passes: the drift pulls along q from               */
/* q - dtheta*p_j, the RF kick pulls along p from p + dtheta*q_i.       */
/* ------------------------------------------------------------------ */
void vfo_rotate_manhattan(const vfo_params *p, const double *src, double *dst, double *tmp)
{
    const int n = p->n, K = p->interp;
    const double dq = grid_dq(p), dp = grid_dp(p);
    const double th = step_angle(p);
    /* drift: tmp(q, p) = src(q - th*p, p) */
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        const double q = p->q_min + i * dq;
        for (int j = 0; j < n; ++j) {
            const double pp = p->p_min + j * dp;
            const double rx = (q - th * pp - p->q_min) / dq;
            tmp[(size_t)i * n + j] = interp_row(src, n, K, p->clamp, j, rx);
        }
    }
    /* RF kick: dst(q, p) = tmp(q, p + th*q) */
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        const double q = p->q_min + i * dq;
        for (int j = 0; j < n; ++j) {
            const double pp = p->p_min + j * dp;
            const double ry = (pp + th * q - p->p_min) / dp;
            dst[(size_t)i * n + j] = interp_column(tmp, n, K, p->clamp, i, ry);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Kick (Sec. III.B, last paragraph; perturbation Hamiltonian of        */
/* Eq. "perturbation"): the collective potential moves every particle   */
/* in column i by -V_i*dtheta in p.  Pulled: new(q_i, p_j) =            */
/* old(q_i, p_j + V_i*dtheta), i.e. grid coordinate r = j + V_i*th/dp.  */
/* ------------------------------------------------------------------ */
void vfo_kick(const vfo_params *p, const double *V, const double *src, double *dst)
{
    const int n = p->n, K = p->interp;
    const double dp = grid_dp(p);
    const double th = step_angle(p);
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        const double shift = V[i] * th / dp;
        for (int j = 0; j < n; ++j)
            dst[(size_t)i * n + j] = interp_column(src, n, K, p->clamp, i, (double)j + shift);
    }
}

/* ------------------------------------------------------------------ */
/* Damping and diffusion (right-hand side of Eq. VFP):                  */
/*   d psi = beta*dtheta * [ d/dp (p psi) + d^2 psi / dp^2 ],           */
/* one explicit Euler step.  d/dp uses the derivative of the cubic      */
/* interpolation polynomial (Eq. "cubic diff"),                          */
/*   f'(x0) ~ (-2 f(x0-1) - 3 f(x0) + 6 f(x0+1) - f(x0+2)) / (6 dp),    */
/* applied to g = p*psi; d^2/dp^2 is the 3-point central stencil        */
/* (f(x0-1) - 2 f(x0) + f(x0+1)) / dp^2.  Zero outside the grid.        */
/* ------------------------------------------------------------------ */
void vfo_fokker_planck(const vfo_params *p, const double *src, double *dst)
{
    const int n = p->n;
    const double dp = grid_dp(p);
    const double bt = p->beta * step_angle(p);
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) {
            double g[4];   /* g at j-1, j, j+1, j+2 */
            for (int o = -1; o <= 2; ++o) {
                const double pj = p->p_min + (j + o) * dp;
                g[o + 1] = pj * node(src, n, i, j + o);
            }
            const double d1 = (-2.0 * g[0] - 3.0 * g[1] + 6.0 * g[2] - g[3]) / (6.0 * dp);
            const double d2 = (node(src, n, i, j - 1) - 2.0 * node(src, n, i, j) + node(src, n, i, j + 1)) / (dp * dp);
            dst[(size_t)i * n + j] = node(src, n, i, j) + bt * (d1 + d2);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Moments of the density: out = {Q, <q>, sigma_q, <p>, sigma_p}        */
/* (the bunch length and energy spread observed throughout Sec. IV.A).  */
/* ------------------------------------------------------------------ */
void vfo_moments(const vfo_params *p, const double *psi, double *out)
{
    const int n = p->n;
    const double dq = grid_dq(p), dp = grid_dp(p);
    double s0 = 0.0, sq = 0.0, sp = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const double f = psi[(size_t)i * n + j];
            s0 += f;
            sq += (p->q_min + i * dq) * f;
            sp += (p->p_min + j * dp) * f;
        }
    const double mq = sq / s0, mp = sp / s0;
    double vq = 0.0, vp = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const double f = psi[(size_t)i * n + j];
            const double dqq = p->q_min + i * dq - mq;
            const double dpp = p->p_min + j * dp - mp;
            vq += dqq * dqq * f;
            vp += dpp * dpp * f;
        }
    out[0] = dq * dp * s0;
    out[1] = mq;
    out[2] = sqrt(vq / s0);
    out[3] = mp;
    out[4] = sqrt(vp / s0);
}

/* CSR power of the current state (Sec. IV.C):                          */
/* P = sum_i rho_i V_i, the discrete form of integral Re Z |rho~|^2 dk. */
double vfo_csr_power(const vfo_params *p, const double *w, const double *psi, double *rho, double *V)
{
    vfo_profile(p, psi, rho);
    vfo_wake(p, w, rho, V);
    double s = 0.0;
    for (int i = 0; i < p->n; ++i) s += rho[i] * V[i];
    return s;
}

/* CSR spectrum of the current state (Sec. IV.C): P(k) ~ Re Z_k |rho~_k|^2 */
/* with rho~_k = sum_j rho_j e^{-2 pi i k j/M} the DFT of the zero-padded */
/* profile.  Bins k = 0..M/2; the bins 0 < k < M/2 stand for k and M-k, */
/* so out[k] = (S/M) * m_k * Re Z_k * |rho~_k|^2 with m_k = 2 there and */
/* 1 at k = 0 and k = M/2 (M even); sum_k out[k] = sum_i rho_i V_i.      */
void vfo_csr_spectrum(const vfo_params *p, const double *z_re, const double *psi, double *rho, double *out)
{
    const int n = p->n, M = p->padding * n;
    vfo_profile(p, psi, rho);
    for (int k = 0; k <= M / 2; ++k) {
        double re = 0.0, im = 0.0;
        for (int j = 0; j < n; ++j) {
            const long long kj = ((long long)k * j) % M;
            const double phi = 2.0 * M_PI * (double)kj / (double)M;
            re += rho[j] * cos(phi);
            im -= rho[j] * sin(phi);
        }
        const double mult = (k == 0 || 2 * k == M) ? 1.0 : 2.0;
        out[k] = p->z_scale / (double)M * mult * z_re[k] * (re * re + im * im);
    }
}

/* ------------------------------------------------------------------ */
/* Haissinski starting distribution (Appendix A: the equilibrium profile */
/* below threshold).  The profile solves rho(q) ~ exp(-q^2/2 - U(q)),     */
/* U' = V[rho] the wake potential of rho itself, with dq*sum(rho) = Q0;   */
/* the energy distribution is the unit Gaussian.  Solved by the damped    */
/* fixed-point iteration rho <- (1-alpha) rho + alpha F(rho), starting    */
/* from the Gaussian; U by the cumulative trapezoid rule from q_min (its  */
/* constant drops out in the normalisation).  psi_ij = rho_i g_j with    */
/* g_j = exp(-p_j^2/2) / (dp sum_j exp(-p_j^2/2)).                        */
/* ------------------------------------------------------------------ */
void vfo_haissinski(const vfo_params *p, const double *w, int iters, double alpha, double Q0, double *psi)
{
    const int n = p->n;
    const double dq = grid_dq(p), dp = grid_dp(p);
    double *rho = (double *)malloc(sizeof(double) * 4 * n);
    double *V = rho + n, *U = V + n, *F = U + n;
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        const double q = p->q_min + i * dq;
        rho[i] = exp(-0.5 * q * q);
        s += rho[i];
    }
    for (int i = 0; i < n; ++i) rho[i] *= Q0 / (dq * s);
    for (int it = 0; it < iters; ++it) {
        vfo_wake(p, w, rho, V);
        U[0] = 0.0;
        for (int i = 1; i < n; ++i) U[i] = U[i - 1] + 0.5 * (V[i - 1] + V[i]) * dq;
        s = 0.0;
        for (int i = 0; i < n; ++i) {
            const double q = p->q_min + i * dq;
            F[i] = exp(-0.5 * q * q - U[i]);
            s += F[i];
        }
        for (int i = 0; i < n; ++i) rho[i] = (1.0 - alpha) * rho[i] + alpha * F[i] * (Q0 / (dq * s));
    }
    double g = 0.0;
    for (int j = 0; j < n; ++j) {
        const double pp = p->p_min + j * dp;
        g += exp(-0.5 * pp * pp);
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const double pp = p->p_min + j * dp;
            psi[(size_t)i * n + j] = rho[i] * exp(-0.5 * pp * pp) / (dp * g);
        }
    free(rho);
}

/* ------------------------------------------------------------------ */
/* One time step (Sec. III.B, f = f_rot + f_kick + f_damp,diff, applied */
/* in that order).  The collective force is held constant over the step */
/* (Sec. II.A), so rho and V are taken from psi at the start.  After    */
/* the step the charge is rescaled to Q0 when renormalize is set.       */
/* work must hold 2*n*n + 2*n doubles.  w may be NULL (zero current).   */
/* ------------------------------------------------------------------ */
void vfo_step(const vfo_params *p, const double *w, double *psi, double Q0, double *work)
{
    const int n = p->n;
    const size_t nn = (size_t)n * n;
    double *a = work, *b = work + nn, *rho = work + 2 * nn, *V = rho + n;
    if (w) {
        vfo_profile(p, psi, rho);
        vfo_wake(p, w, rho, V);
    } else {
        for (int i = 0; i < n; ++i) V[i] = 0.0;
    }
    if (p->rotation == 1) vfo_rotate_manhattan(p, psi, a, b);
    else                  vfo_rotate(p, psi, a);
    vfo_kick(p, V, a, b);
    vfo_fokker_planck(p, b, psi);
    if (p->renormalize) {
        const double Q = vfo_charge(p, psi);
        const double f = Q0 / Q;
        for (size_t z = 0; z < nn; ++z) psi[z] *= f;
    }
}

/* Run nsteps steps.  If every > 0 and rec != NULL, after each step t   */
/* (t counted from 1) with t % every == 0 a row of 7 doubles            */
/* {t, Q, <q>, sigma_q, <p>, sigma_p, P} describing the state after the */
/* step is appended, up to cap rows.  Returns the number of rows.       */
long vfo_run(const vfo_params *p, const double *w, double *psi, long nsteps, double Q0,
             int every, double *rec, long cap)
{
    const int n = p->n;
    const size_t nn = (size_t)n * n;
    double *work = (double *)malloc(sizeof(double) * (2 * nn + 4 * (size_t)n));
    if (!work) return -1;
    long rows = 0;
    for (long t = 1; t <= nsteps; ++t) {
        vfo_step(p, w, psi, Q0, work);
        if (every > 0 && rec && t % every == 0 && rows < cap) {
            double *r = rec + 7 * rows;
            double m[5];
            vfo_moments(p, psi, m);
            r[0] = (double)t;
            for (int k = 0; k < 5; ++k) r[1 + k] = m[k];
            r[6] = w ? vfo_csr_power(p, w, psi, work + 2 * nn, work + 2 * nn + n) : 0.0;
            ++rows;
        }
    }
    free(work);
    return rows;
}

/* Independent simulations, OpenMP across simulations (the inner loops  */
/* then run on one thread each).  psis[s] is updated in place.          */
void vfo_run_many(int count, const vfo_params *ps, const double *const *ws, double *const *psis,
                  const long *nsteps, const double *Q0s)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < count; ++s)
        vfo_run(&ps[s], ws[s], psis[s], nsteps[s], Q0s[s], 0, NULL, 0);
}

/* ================================================================== */
/* Fixed-point density (Sec. III.A, last paragraph: psi held in memory */
/* as a fixed-point number whose count F of fractional bits is chosen   */
/* freely; Sec. IV.A and the table of converged bunch lengths compare   */
/* F = 34 .. 59 with binary32 and binary64).  A stored value is a       */
/* two's-complement integer raw with value raw * 2^-F.                  */
/*                                                                      */
/* The paper does not say how the arithmetic around the stored values   */
/* is done; the reading taken here:                                     */
/*  - every coefficient (interpolation weights, Fokker-Planck stencil   */
/*    coefficients, renormalisation factor) is evaluated in FP64 exactly */
/*    as in the FP64 form above, then rounded to the nearest F-bit       */
/*    fixed-point value (ties to even);                                  */
/*  - each weighted sum is accumulated exactly in 128-bit integers and   */
/*    rounded once to F bits, half up: (acc + 2^(F-1)) >> F;             */
/*  - the 2-D rotation sums each stencil row along p, rounds, then sums  */
/*    the rows along q and rounds (the tensor product taken row first);  */
/*  - the charge is an exact integer sum, converted as                   */
/*    (double)H * 2^32 + (double)L, where H and L sum the arithmetic     */
/*    high halves (raw >> 32) and the low halves (raw & (2^32-1));       */
/*  - the stored density is not rescaled in place: the factor            */
/*    s_t = Q0 / Q(psi_t) multiplies the rotated values of step t, so    */
/*    the state after a step is s_{t+1} * psi_{t+1};                     */
/*  - the wake stays FP64 (the paper computes it for floating-point      */
/*    types only), from rho_i = s_t * dp * colsum_i;                     */
/*  - the kick shift V_i*dtheta/dp is split once per column into its     */
/*    floor and fraction, so every row of a column uses the same weights.*/
/* F must lie in [16, 59] and |psi| stay below 2^(61-F).                */
/* ================================================================== */
typedef long long fx_t;
typedef __int128 fx2_t;

/* round a FP64 coefficient to F fractional bits */
static fx_t fx_coef(double x, int F) { return llrint(ldexp(x, F)); }

/* round an exact sum of F+F fractional bits to F bits, half up */
static fx_t fx_round(fx2_t acc, int F) { return (fx_t)((acc + ((fx2_t)1 << (F - 1))) >> F); }

static fx_t fx_node(const fx_t *psi, int n, int i, int j)
{
    if (i < 0 || i >= n || j < 0 || j >= n) return 0;
    return psi[(size_t)i * n + j];
}

/* high/low half sums of one column, exact */
static void fx_column_parts(const fx_t *col, int n, long long *h, long long *l)
{
    long long a = 0, b = 0;
    for (int j = 0; j < n; ++j) {
        a += col[j] >> 32;
        b += col[j] & 0xffffffffLL;
    }
    *h = a;
    *l = b;
}

static double fx_parts_value(long long h, long long l) { return (double)h * 4294967296.0 + (double)l; }

void vfo_fix_quantize(int F, const double *x, fx_t *raw, long count)
{
    for (long z = 0; z < count; ++z) raw[z] = fx_coef(x[z], F);
}

/* charge dq*dp*sum(psi) of a fixed-point density, from the exact sum */
double vfo_fix_charge(const vfo_params *p, int F, const fx_t *psi)
{
    const int n = p->n;
    long long H = 0, L = 0;
    for (int i = 0; i < n; ++i) {
        long long h, l;
        fx_column_parts(psi + (size_t)i * n, n, &h, &l);
        H += h;
        L += l;
    }
    return ldexp(fx_parts_value(H, L), -F) * grid_dq(p) * grid_dp(p);
}

/* 1-D fixed-point interpolation with weights W at integer base m, along
 * p (column i) or along q (row j); clamp to the two bracketing nodes */
static fx2_t fx_interp(const fx_t *psi, int n, int K, int along_p, int fixed, int m, const fx_t *W)
{
    fx2_t acc = 0;
    for (int k = 0; k < K; ++k) {
        const int x = m + stencil_offset(K, k);
        const fx_t f = along_p ? fx_node(psi, n, fixed, x) : fx_node(psi, n, x, fixed);
        acc += (fx2_t)W[k] * f;
    }
    return acc;   /* exact, 2F fractional bits; rounded by the caller */
}

static fx_t fx_clip(fx_t v, fx_t a, fx_t b)
{
    const fx_t lo = a < b ? a : b, hi = a < b ? b : a;
    return v < lo ? lo : (v > hi ? hi : v);
}

static void fx_weights(int K, double t, int F, fx_t *W)
{
    double l[4];
    vfo_lagrange_weights(K, t, l);
    for (int k = 0; k < K; ++k) W[k] = fx_coef(l[k], F);
}

/* One time step of the fixed-point density (same sub-steps and order as
 * vfo_step).  psi holds the stored density psi_t and is replaced by
 * psi_{t+1}; *s_used receives s_t.  work: 2*n*n fixed values and 4*n
 * doubles.  w may be NULL (zero current). */
void vfo_fix_step(const vfo_params *p, int F, const double *w, fx_t *psi, double Q0, double *s_used,
                  fx_t *work, double *dwork)
{
    const int n = p->n, K = p->interp;
    const size_t nn = (size_t)n * n;
    const double dq = grid_dq(p), dp = grid_dp(p), th = step_angle(p);
    fx_t *a = work, *b = work + nn;
    double *cd = dwork, *rho = dwork + n, *V = dwork + 2 * n;
    /* renormalisation factor from the exact charge */
    long long H = 0, L = 0;
    for (int i = 0; i < n; ++i) {
        long long h, l;
        fx_column_parts(psi + (size_t)i * n, n, &h, &l);
        H += h;
        L += l;
        cd[i] = fx_parts_value(h, l);
    }
    const double Qh = ldexp(fx_parts_value(H, L), -F) * dq * dp;
    const double s = p->renormalize ? Q0 / Qh : 1.0;
    const fx_t sfix = p->renormalize ? fx_coef(s, F) : ((fx_t)1 << F);
    *s_used = s;
    /* FP64 wake of the renormalised profile */
    for (int i = 0; i < n; ++i) V[i] = 0.0;
    if (w) {
        for (int i = 0; i < n; ++i) rho[i] = s * dp * ldexp(cd[i], -F);
        vfo_wake(p, w, rho, V);
    }
    /* rotation, then the renormalisation factor */
    if (p->rotation == 1) {
        /* drift along q from q - dtheta*p_j into b */
        for (int i = 0; i < n; ++i) {
            const double q = p->q_min + i * dq;
            for (int j = 0; j < n; ++j) {
                const double pp = p->p_min + j * dp;
                const double rx = (q - th * pp - p->q_min) / dq;
                const double m = floor(rx);
                fx_t W[4];
                fx_weights(K, rx - m, F, W);
                fx_t v = fx_round(fx_interp(psi, n, K, 0, j, (int)m, W), F);
                if (p->clamp) v = fx_clip(v, fx_node(psi, n, (int)m, j), fx_node(psi, n, (int)m + 1, j));
                b[(size_t)i * n + j] = v;
            }
        }
        /* RF kick along p from p + dtheta*q_i into a */
        for (int i = 0; i < n; ++i) {
            const double q = p->q_min + i * dq;
            for (int j = 0; j < n; ++j) {
                const double pp = p->p_min + j * dp;
                const double ry = (pp + th * q - p->p_min) / dp;
                const double m = floor(ry);
                fx_t W[4];
                fx_weights(K, ry - m, F, W);
                fx_t v = fx_round(fx_interp(b, n, K, 1, i, (int)m, W), F);
                if (p->clamp) v = fx_clip(v, fx_node(b, n, i, (int)m), fx_node(b, n, i, (int)m + 1));
                a[(size_t)i * n + j] = fx_round((fx2_t)v * sfix, F);
            }
        }
    } else {
        const double c = cos(th), sn = sin(th);
        for (int i = 0; i < n; ++i) {
            const double q = p->q_min + i * dq;
            for (int j = 0; j < n; ++j) {
                const double pp = p->p_min + j * dp;
                const double q0 = q * c - pp * sn;
                const double p0 = q * sn + pp * c;
                const double rx = (q0 - p->q_min) / dq;
                const double ry = (p0 - p->p_min) / dp;
                const double mx = floor(rx), my = floor(ry);
                const int ix = (int)mx, iy = (int)my;
                fx_t Wx[4], Wy[4], r[4];
                fx_weights(K, rx - mx, F, Wx);
                fx_weights(K, ry - my, F, Wy);
                for (int ka = 0; ka < K; ++ka)   /* stencil row ix + o_a, summed along p */
                    r[ka] = fx_round(fx_interp(psi, n, K, 1, ix + stencil_offset(K, ka), iy, Wy), F);
                fx2_t acc = 0;
                for (int ka = 0; ka < K; ++ka) acc += (fx2_t)Wx[ka] * r[ka];
                fx_t v = fx_round(acc, F);
                if (p->clamp) {
                    fx_t lo = fx_node(psi, n, ix, iy), hi = lo;
                    for (int da = 0; da < 2; ++da)
                        for (int db = 0; db < 2; ++db) {
                            const fx_t f = fx_node(psi, n, ix + da, iy + db);
                            if (f < lo) lo = f;
                            if (f > hi) hi = f;
                        }
                    v = v < lo ? lo : (v > hi ? hi : v);
                }
                a[(size_t)i * n + j] = fx_round((fx2_t)v * sfix, F);
            }
        }
    }
    /* kick along p: shift V_i*dtheta/dp split once per column */
    for (int i = 0; i < n; ++i) {
        const double shift = V[i] * th / dp;
        double fl = floor(shift);
        fx_t W[4];
        fx_weights(K, shift - fl, F, W);
        if (fl > 2.0 * n) fl = 2.0 * n;          /* every tap is outside the grid */
        if (fl < -2.0 * n) fl = -2.0 * n;
        const int m0 = (int)fl;
        for (int j = 0; j < n; ++j) {
            fx_t v = fx_round(fx_interp(a, n, K, 1, i, j + m0, W), F);
            if (p->clamp) v = fx_clip(v, fx_node(a, n, i, j + m0), fx_node(a, n, i, j + m0 + 1));
            b[(size_t)i * n + j] = v;
        }
    }
    /* damping/diffusion: out = g_j + sum_o E_o(j) g_{j+o}, o = -1..2, with
     * the coefficients of vfo_fokker_planck collected per row:
     * E_-1 = k2 - 2 k1 u_-1, E_0 = -3 k1 u_0 - 2 k2, E_1 = 6 k1 u_1 + k2,
     * E_2 = -k1 u_2; k1 = beta*dtheta/6, k2 = beta*dtheta/dp^2,
     * u_o = p_min/dp + (j + o) */
    const double bt = p->beta * th;
    const double k1 = bt / 6.0, k2 = bt / (dp * dp), pm = p->p_min / dp;
    for (int j = 0; j < n; ++j) {
        const double um = pm + (double)(j - 1), u0 = pm + (double)j, u1 = pm + (double)(j + 1),
                     u2 = pm + (double)(j + 2);
        const fx_t E[4] = {fx_coef(k2 - 2.0 * k1 * um, F), fx_coef(-3.0 * k1 * u0 - 2.0 * k2, F),
                           fx_coef(6.0 * k1 * u1 + k2, F), fx_coef(-k1 * u2, F)};
        for (int i = 0; i < n; ++i) {
            fx2_t acc = 0;
            for (int o = -1; o <= 2; ++o) acc += (fx2_t)E[o + 1] * fx_node(b, n, i, j + o);
            psi[(size_t)i * n + j] = b[(size_t)i * n + j] + fx_round(acc, F);
        }
    }
}

/* Run nsteps fixed-point steps; *s_final receives the renormalisation
 * factor of the final state (its physical density is s_final*psi*2^-F).
 * Returns 0, or -1 when out of memory. */
int vfo_fix_run(const vfo_params *p, int F, const double *w, fx_t *psi, long nsteps, double Q0, double *s_final)
{
    const int n = p->n;
    const size_t nn = (size_t)n * n;
    fx_t *work = (fx_t *)malloc(sizeof(fx_t) * 2 * nn);
    double *dwork = (double *)malloc(sizeof(double) * 4 * (size_t)n);
    if (!work || !dwork) {
        free(work);
        free(dwork);
        return -1;
    }
    double s = 1.0;
    for (long t = 0; t < nsteps; ++t) vfo_fix_step(p, F, w, psi, Q0, &s, work, dwork);
    /* factor of the final state */
    const double Qh = vfo_fix_charge(p, F, psi);
    *s_final = p->renormalize ? Q0 / Qh : 1.0;
    free(work);
    free(dwork);
    return 0;
}
