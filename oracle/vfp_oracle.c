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
