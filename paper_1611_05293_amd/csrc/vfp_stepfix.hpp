// vfp_stepfix.hpp -- the split step on a fixed-point density (included by
// vfp.hip after vfp_kernels.hpp).
//
// The density is stored as two's-complement 64-bit integers with F
// fractional bits (value = raw * 2^-F), the representation whose number of
// fractional bits the paper varies in its data-type study (Sec. III.A last
// paragraph, Sec. IV.A).  The arithmetic around the stored values:
//   * coefficients (interpolation weights, damping/diffusion coefficients,
//     the renormalisation factor) are evaluated in FP64 and rounded to the
//     nearest F-bit value (ties to even); the FP64 expressions are written
//     out operation by operation with contraction off, so they round the
//     same way on every IEEE-754 machine;
//   * a weighted sum is accumulated exactly in 128-bit integers and rounded
//     once to F bits, half up;
//   * the 2-D rotation sums each stencil row along p first, rounds, then
//     sums the rows along q and rounds;
//   * the charge is an exact integer sum, kept as the sums of the high
//     (raw >> 32) and low (raw & 0xffffffff) halves of the raw values and
//     converted as (double)H * 2^32 + (double)L;
//   * psi is not rescaled in place: s_t = Q0 / Q(psi_t) multiplies the
//     rotated values of step t;
//   * the wake is FP64, and the kick shift V_i*dtheta/dp is split once per
//     column into floor and fraction.
// One workgroup owns a strip of whole columns; phases as in step_kernel:
// rotation -> LDS A, kick A -> B, damping/diffusion B -> HBM, then the exact
// column sums.  Dynamic LDS: 2*w*n int64.
#pragma once

namespace vfp {

typedef __int128 fx2;

__device__ __forceinline__ int64_t fx_coef(double x, int F) { return llrint(ldexp(x, F)); }
__device__ __forceinline__ int64_t fx_round(fx2 acc, int F)
{
    return (int64_t)((acc + ((fx2)1 << (F - 1))) >> F);
}
__device__ __forceinline__ double fx_parts(int64_t h, int64_t l) { return (double)h * 4294967296.0 + (double)l; }

// Lagrange basis at t over the stencil offsets o_k = k - (K-1)/2, as the
// plain product over the other nodes, each factor (t - o_k') / (o_k - o_k')
template <int K>
__device__ __forceinline__ void fx_weights(double t, int F, int64_t *W)
{
#pragma clang fp contract(off)
    constexpr int o0 = (K - 1) / 2;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double v = 1.0;
#pragma unroll
        for (int kk = 0; kk < K; ++kk) {
            if (kk == k) continue;
            v *= (t - (double)(kk - o0)) / (double)(k - kk);
        }
        W[k] = fx_coef(v, F);
    }
}

__device__ __forceinline__ int64_t fx_node(const int64_t *__restrict__ psi, int n, int i, int j)
{
    return (i < 0 || i >= n || j < 0 || j >= n) ? 0 : psi[(size_t)i * n + j];
}

__device__ __forceinline__ int64_t fx_clip(int64_t v, int64_t a, int64_t b)
{
    const int64_t lo = a < b ? a : b, hi = a < b ? b : a;
    return v < lo ? lo : (v > hi ? hi : v);
}

template <int K, int WAKE, bool CLAMP, int ROT>
__global__ __launch_bounds__(kThreads) void stepfix_kernel(const SimDev *__restrict__ sims,
                                                           const Unit *__restrict__ units, int nunits,
                                                           int parity)
{
#pragma clang fp contract(off)
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[kThreads];
    __shared__ int64_t redi[kWaves];
    __shared__ int64_t sh_kw[kMaxStrip][4];
    __shared__ int sh_km[kMaxStrip];
    constexpr int o0 = (K - 1) / 2;

    const Unit u = units[blockIdx.x];
    if (u.w == 0) return;                     // padding slot
    const SimDev &sd = sims[u.sim];
    const int n = sd.n, w = u.w, i0 = u.i0, tid = threadIdx.x, F = sd.fixb;
    const int64_t *__restrict__ src = (const int64_t *)sd.psi[parity];
    int64_t *__restrict__ dst = (int64_t *)sd.psi[parity ^ 1];
    const int64_t *__restrict__ cs = (const int64_t *)sd.colsum[parity];     // {high, low} per column
    int64_t *__restrict__ cs_next = (int64_t *)sd.colsum[parity ^ 1];
    int64_t *A = (int64_t *)smem_raw;
    int64_t *B = A + (size_t)w * n;

    // ---- prologue: exact charge -> s, its F-bit value, the wake, kick weights
    int64_t ph = 0, pl = 0;
    for (int k = tid; k < n; k += kThreads) {
        ph += cs[2 * k];
        pl += cs[2 * k + 1];
    }
    const int64_t H = block_sum_i64(ph, redi);
    const int64_t L = block_sum_i64(pl, redi);
    const double Qh = ldexp(fx_parts(H, L), -F) * sd.dq * sd.dp;
    const double s = sd.renorm ? sd.Q0 / Qh : 1.0;
    const int64_t sfix = sd.renorm ? fx_coef(s, F) : ((int64_t)1 << F);
    double shift = 0.0;                               // kick of column tid (tid < w), in rows
    if constexpr (WAKE == WAKE_FUSED) {
        // V_i = S * sum_j w[i-j] rho_j, rho_j = s * dp * colsum_j
        const int parts = kThreads / w;
        const int c = tid / parts, pt = tid - c * parts;
        double acc = 0.0;
        if (c < w) {
            const int i = i0 + c;
            for (int j = pt; j < n; j += parts) {
                const double rho = s * sd.dp * ldexp(fx_parts(cs[2 * j], cs[2 * j + 1]), -F);
                acc += sd.wl64[i - j + n - 1] * rho;
            }
        }
        __syncthreads();
        red[tid] = acc;
        __syncthreads();
        if (tid < w) {
            double v = 0.0;
            for (int k = 0; k < parts; ++k) v += red[tid * parts + k];
            const double V = sd.S * v;
            shift = V * sd.th / sd.dp;
            sd.vext[parity * n + i0 + tid] = (float)V;             // the wake this step used
        }
    }
    if (tid < w) {
        double fl = floor(shift);
        int64_t W[K];
        fx_weights<K>(shift - fl, F, W);
        for (int k = 0; k < K; ++k) sh_kw[tid][k] = W[k];
        fl = fl > 2.0 * n ? 2.0 * n : (fl < -2.0 * n ? -2.0 * n : fl);   // all taps outside the grid
        sh_km[tid] = (int)fl;
    }
    __syncthreads();

    // ---- rotation -> A (times the renormalisation factor)
    if constexpr (ROT == 0) {
        const double c = sd.c, sn = sd.s;
        for_strip(w, n, [&](int cc, int j) {
            const int i = i0 + cc;
            const double q = sd.q_min + i * sd.dq;
            const double pp = sd.p_min + j * sd.dp;
            const double q0 = q * c - pp * sn;
            const double p0 = q * sn + pp * c;
            const double rx = (q0 - sd.q_min) / sd.dq;
            const double ry = (p0 - sd.p_min) / sd.dp;
            const double mx = floor(rx), my = floor(ry);
            const int ix = (int)mx, iy = (int)my;
            int64_t Wx[K], Wy[K];
            fx_weights<K>(rx - mx, F, Wx);
            fx_weights<K>(ry - my, F, Wy);
            fx2 acc = 0;
#pragma unroll
            for (int a = 0; a < K; ++a) {
                fx2 r = 0;
#pragma unroll
                for (int b = 0; b < K; ++b) r += (fx2)Wy[b] * fx_node(src, n, ix + a - o0, iy + b - o0);
                acc += (fx2)Wx[a] * fx_round(r, F);
            }
            int64_t v = fx_round(acc, F);
            if constexpr (CLAMP) {
                int64_t lo = fx_node(src, n, ix, iy), hi = lo;
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        const int64_t f = fx_node(src, n, ix + a, iy + b);
                        lo = f < lo ? f : lo;
                        hi = f > hi ? f : hi;
                    }
                v = v < lo ? lo : (v > hi ? hi : v);
            }
            A[(size_t)cc * n + j] = fx_round((fx2)v * sfix, F);
        });
        __syncthreads();
    } else {
        // Manhattan: drift along q from q - dtheta*p_j (taps from HBM) -> B
        for_strip(w, n, [&](int cc, int j) {
            const int i = i0 + cc;
            const double q = sd.q_min + i * sd.dq;
            const double pp = sd.p_min + j * sd.dp;
            const double rx = (q - sd.th * pp - sd.q_min) / sd.dq;
            const double m = floor(rx);
            const int mi = (int)m;
            int64_t W[K];
            fx_weights<K>(rx - m, F, W);
            fx2 acc = 0;
#pragma unroll
            for (int k = 0; k < K; ++k) acc += (fx2)W[k] * fx_node(src, n, mi + k - o0, j);
            int64_t v = fx_round(acc, F);
            if constexpr (CLAMP) v = fx_clip(v, fx_node(src, n, mi, j), fx_node(src, n, mi + 1, j));
            B[(size_t)cc * n + j] = v;
        });
        __syncthreads();
        // RF kick along p from p + dtheta*q_i (taps from the LDS column) -> A
        for_strip(w, n, [&](int cc, int j) {
            const int i = i0 + cc;
            const double q = sd.q_min + i * sd.dq;
            const double pp = sd.p_min + j * sd.dp;
            const double ry = (pp + sd.th * q - sd.p_min) / sd.dp;
            const double m = floor(ry);
            const int mi = (int)m;
            int64_t W[K];
            fx_weights<K>(ry - m, F, W);
            const int64_t *col = B + (size_t)cc * n;
            fx2 acc = 0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int jj = mi + k - o0;
                acc += (fx2)W[k] * ((jj >= 0 && jj < n) ? col[jj] : 0);
            }
            int64_t v = fx_round(acc, F);
            if constexpr (CLAMP) {
                const int64_t a = (mi >= 0 && mi < n) ? col[mi] : 0, b = (mi + 1 >= 0 && mi + 1 < n) ? col[mi + 1] : 0;
                v = fx_clip(v, a, b);
            }
            A[(size_t)cc * n + j] = fx_round((fx2)v * sfix, F);
        });
        __syncthreads();
    }

    // ---- kick along p: A -> B, per-column weights
    for_strip(w, n, [&](int cc, int j) {
        const int64_t *col = A + (size_t)cc * n;
        const int m = j + sh_km[cc];
        fx2 acc = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int jj = m + k - o0;
            acc += (fx2)sh_kw[cc][k] * ((jj >= 0 && jj < n) ? col[jj] : 0);
        }
        int64_t v = fx_round(acc, F);
        if constexpr (CLAMP) {
            const int64_t a = (m >= 0 && m < n) ? col[m] : 0, b = (m + 1 >= 0 && m + 1 < n) ? col[m + 1] : 0;
            v = fx_clip(v, a, b);
        }
        B[(size_t)cc * n + j] = v;
    });
    __syncthreads();

    // ---- damping/diffusion: out = g_j + sum_o E_o(j) g_{j+o}, o = -1..2,
    // E_-1 = k2 - 2 k1 u_-1, E_0 = -3 k1 u_0 - 2 k2, E_1 = 6 k1 u_1 + k2,
    // E_2 = -k1 u_2 with k1 = beta*dtheta/6, k2 = beta*dtheta/dp^2,
    // u_o = p_min/dp + (j + o); B -> HBM and A
    const double k1 = sd.bt / 6.0, k2 = sd.bt / (sd.dp * sd.dp), pm = sd.p_min / sd.dp;
    for_strip(w, n, [&](int cc, int j) {
        const double um = pm + (double)(j - 1), u0 = pm + (double)j, u1 = pm + (double)(j + 1),
                     u2 = pm + (double)(j + 2);
        const int64_t E0 = fx_coef(k2 - 2.0 * k1 * um, F), E1 = fx_coef(-3.0 * k1 * u0 - 2.0 * k2, F),
                      E2 = fx_coef(6.0 * k1 * u1 + k2, F), E3 = fx_coef(-k1 * u2, F);
        const int64_t *col = B + (size_t)cc * n;
        const int64_t gm = j > 0 ? col[j - 1] : 0, g0 = col[j];
        const int64_t g1 = j + 1 < n ? col[j + 1] : 0, g2 = j + 2 < n ? col[j + 2] : 0;
        const fx2 acc = (fx2)E0 * gm + (fx2)E1 * g0 + (fx2)E2 * g1 + (fx2)E3 * g2;
        const int64_t out = g0 + fx_round(acc, F);
        dst[(size_t)(i0 + cc) * n + j] = out;
        A[(size_t)cc * n + j] = out;
    });
    __syncthreads();

    // ---- exact column sums {high halves, low halves}: one wave per column
    {
        const int lane = tid & 63, wv = tid >> 6;
        for (int cc = wv; cc < w; cc += kWaves) {
            int64_t h = 0, l = 0;
            for (int j = lane; j < n; j += 64) {
                const int64_t v = A[(size_t)cc * n + j];
                h += v >> 32;
                l += v & 0xffffffffLL;
            }
            h = wave_sum_i64(h);
            l = wave_sum_i64(l);
            if (lane == 0) {
                cs_next[2 * (i0 + cc)] = h;
                cs_next[2 * (i0 + cc) + 1] = l;
            }
        }
    }
}

// Exact column sums {high, low} of a stored fixed-point density (after an
// upload): grid.x column blocks of kWaves (one wave per column), grid.y sims.
__global__ __launch_bounds__(kThreads) void projectfix_kernel(const SimDev *__restrict__ sims,
                                                              const int *__restrict__ which, int parity)
{
    const SimDev &sd = sims[which[blockIdx.y]];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = blockIdx.x * kWaves + wv;
    if (i >= sd.n) return;
    const int64_t *f = (const int64_t *)sd.psi[parity] + (size_t)i * sd.n;
    int64_t h = 0, l = 0;
    for (int j = lane; j < sd.n; j += 64) {
        h += f[j] >> 32;
        l += f[j] & 0xffffffffLL;
    }
    h = wave_sum_i64(h);
    l = wave_sum_i64(l);
    if (lane == 0) {
        int64_t *cs = (int64_t *)sd.colsum[parity];
        cs[2 * i] = h;
        cs[2 * i + 1] = l;
    }
}

}  // namespace vfp
