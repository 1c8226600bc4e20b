// vfp_kernels.hpp -- gfx950 device code for the VFP split step
// (arXiv:1611.05293, Sec. III).  Included once, by vfp.hip.
//
// Data layout in HBM (per simulation): psi[2][n][n] (double buffer, p index
// fastest), colsum[2][n] FP64 column sums of the stored density, the wake
// table wl[2n-1] indexed by lag + n - 1, and the FP64 diagnostics.
//
// The stored density psi^ is not renormalised: the physical state is
// s * psi^ with s = Q0 / (dq dp sum psi^).  Because rotation, kick and
// damping are linear in psi for a fixed wake, a step multiplies the rotated
// values by s and uses the wake of s * rho^; the stored result is then the
// un-renormalised image of the renormalised state, exactly as if the
// renormalisation had been applied at the end of the previous step
// (Sec. III.B step composition; the rescaling itself is not in the paper).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace vfp {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxStrip = 128;      // columns per work unit

enum WakeMode { WAKE_NONE = 0, WAKE_FUSED = 1, WAKE_EXTERNAL = 2 };

struct SimDev {
    int32_t n, K, rotation, clamp;
    int32_t renorm, has_wake, M, fixb;   // fixb: fractional bits of the fixed-point storage
    int64_t step0;                   // global tick at which this simulation was at step 0
    double q_min, p_min, dq, dp;
    double c, s, th, bt;             // cos, sin of dtheta; dtheta; beta*dtheta
    double kick;                     // dtheta / dp
    double S, Q0;
    // displacement of the rotation source in cells: dx = ax0 + i*axi + j*bx,
    // dy = cy0 + i*cyi + j*by (exact rewriting of the pull map)
    double ax0, axi, bx, cy0, cyi, by;
    double pm;                       // p_min / dp
    double tw;                       // Manhattan drift per p cell: dtheta*dp/dq
    double tk;                       // Manhattan RF kick: dtheta*dq/dp
    void *psi[2];
    double *colsum[2];
    const double *wl64;              // 2n-1 lags, FP64
    const float *wl32;               // 2n-1 lags, FP32
    const uint16_t *wsplit;          // matrix-core wake: reversed hi/lo lag tables (wake_split_kernel)
    float *vext;                     // [2][n]: vext[p] is the wake of the state held in buffer p (FP32)
    double *sext;                    // {s of buffer 0, s of buffer 1, inverse lag scale of the hi/lo wake}
    double *rho_out, *v_out;         // FP64 diagnostics (n each)
    const double *zr64;              // Re Z_k, k = 0..M/2 (CSR spectrum)
    double *stat;                    // {Q, <q>, sq, <p>, sp, P, s, bad}
    double *mom;                     // per column: sum psi, sum p psi, sum p^2 psi (3n, FP64)
    double *ring;                    // record rows (7 doubles each) or NULL
    int64_t ring_cap;
    int64_t *ring_rows;
    // FP32 constants of the chunked staged kernel, rounded once on the host:
    // bx, by (displacement per p row), k1 = beta*dtheta/6, the four
    // p-independent damping/diffusion coefficients {2k1+k2, 1-2k2, 6k1+k2,
    // -2k1} (k2 = beta*dtheta/dp^2), and the Manhattan drift shift
    // -tw*(pm + row) as fd0 + row*fd1
    float fbx, fby, fk1, fe[4], fd0, fd1, fpad;
    // staged kernel: source columns staged to the left and right of a strip
    // (every stencil column the rotation or drift reads, at most kH each side)
    int32_t hl, hr;
};

// A work unit: simulation, first column i0 and width w of its strip.  In the
// item list of the fused tick, w == 0 is an empty slot and w < 0 a wake tile
// (tile index in i0); nu is the number of units of the simulation.
struct Unit {
    int32_t sim, i0, w;
    int32_t nu;
    // copies of the simulation's grid size, halo widths and density buffers,
    // so that a staged unit can issue its first loads before its SimDev arrives
    int32_t n, hl, hr, pad;
    const void *psi[2];
};

// ---------------------------------------------------------------- helpers
// value of a stored density element (raw * 2^-F for the fixed-point storage)
template <typename T>
__device__ __forceinline__ double stored_value(T v, int fixb)
{
    if constexpr (std::is_same_v<T, int64_t>) return ldexp((double)v, -fixb);
    else return (double)v;
}
// a density value rounded to the storage type (ties to even in fixed point)
template <typename T>
__device__ __forceinline__ T to_stored(double x, int fixb)
{
    if constexpr (std::is_same_v<T, int64_t>) return llrint(ldexp(x, fixb));
    else return (T)x;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// exact workgroup sum of 64-bit integers (red: at least kWaves entries)
__device__ __forceinline__ int64_t block_sum_i64(int64_t v, int64_t *red)
{
    v = wave_sum_i64(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    int64_t t = 0;
    for (int k = 0; k < kWaves; ++k) t += red[k];
    __syncthreads();
    return t;
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// deterministic block sum (fixed tree); all threads get the result
__device__ __forceinline__ double block_sum(double v, double *red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < kWaves; ++k) t += red[k];
    __syncthreads();
    return t;
}

// Column sums shared between the workgroups of one launch (the fused tick's
// last unit of a simulation reads every unit's sums): written and read as
// agent-scope relaxed atomics, which on this GPU are stores written through
// to, and loads served from, the level coherent across the XCDs.  The writer
// waits for its stores to complete (vmcnt 0) before it counts itself done.
template <bool COH>
__device__ __forceinline__ double load_cs(const double *p)
{
    typedef const __attribute__((address_space(1))) double gd;
    if constexpr (COH) return __hip_atomic_load((gd *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *(gd *)p;
}
// values p[k], k = k0 + q*kThreads (q < kCsBatch), 0 beyond k1: the loads are
// issued together, so a batch costs one memory round trip
constexpr int kCsBatch = 8;
template <bool COH>
__device__ __forceinline__ void load_cs_batch(const double *p, int k0, int k1, double (&v)[kCsBatch])
{
#pragma unroll
    for (int q = 0; q < kCsBatch; ++q) {
        const int k = k0 + q * kThreads;
        v[q] = k < k1 ? load_cs<COH>(p + k) : 0.0;
    }
}
template <bool COH>
__device__ __forceinline__ void store_cs(double *p, double v)
{
    if constexpr (COH) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}
__device__ __forceinline__ void wait_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }   // s_waitcnt vmcnt(0)

// stores of the wake (V, s) that workgroups of the same launch read: written
// through to the level coherent across the XCDs when OUTCOH
template <bool OUTCOH>
__device__ __forceinline__ void store_wake_f(float *p, float v)
{
    if constexpr (OUTCOH) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}
template <bool OUTCOH>
__device__ __forceinline__ void store_wake_d(double *p, double v)
{
    if constexpr (OUTCOH) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = v;
}

// Work units of a step launch: the host lays them out in dispatch order
// (block k*8 + x runs on XCD x), so block b takes units[b]; slots with
// w == 0 are padding and their blocks return at once, before any barrier.

// ----------------------------------------------- Lagrange weights (Sec. III.A)
// FP64 closed forms of the basis over the offsets -1, 0, 1[, 2], with a
// shared factor a = t(t-1): l_-1 = -a(t-2)/6, l_0 = (t+1)(t-1)(t-2)/2,
// l_1 = -(t+1)t(t-2)/2, l_2 = a(t+1)/6 for K = 4; t(t-1)/2, 1-t^2,
// t(t+1)/2 for K = 3.
template <int K>
__device__ __forceinline__ void lagrange64(double t, double *l)
{
    if constexpr (K == 4) {
        const double a = fma(t, t, -t);               // t(t-1)
        const double a6 = a * (1.0 / 6.0);
        const double b2 = fma(a, 0.5, -1.0);          // (t+1)(t-2)/2
        l[0] = fma(-a6, t, a * (1.0 / 3.0));
        l[1] = fma(b2, t, -b2);
        l[2] = -b2 * t;
        l[3] = fma(a6, t, a6);
    } else {
        const double a = fma(t, t, -t);
        l[0] = 0.5 * a;
        l[1] = fma(-t, t, 1.0);
        l[2] = fma(0.5, a, t);
    }
}

// FP32 closed forms of the same polynomials (offsets -1,0,1[,2])
template <int K>
__device__ __forceinline__ void lagrange32(float t, float *l)
{
    if constexpr (K == 4) {
        const float tp = t + 1.0f, tm = t - 1.0f, t2 = t - 2.0f;
        const float a = t * tm;                 // t(t-1)
        const float b = tp * t2;                // (t+1)(t-2)
        l[0] = a * t2 * (-1.0f / 6.0f);
        l[1] = b * tm * 0.5f;
        l[2] = b * t * (-0.5f);
        l[3] = a * tp * (1.0f / 6.0f);
    } else {
        l[0] = 0.5f * t * (t - 1.0f);
        l[1] = (1.0f - t) * (1.0f + t);
        l[2] = 0.5f * t * (t + 1.0f);
    }
}

template <typename T>
__device__ __forceinline__ T ld_node(const T *__restrict__ f, int n, int i, int j)
{
    return (i >= 0 && i < n && j >= 0 && j < n) ? f[(size_t)i * n + j] : T(0);
}

// ------------------------------------------------- standard rotation, FP64
// The source point in cells is (i + dx, j + dy) with the displacement in the
// exact linear form dx = ax0 + i*axi + j*bx, dy = cy0 + i*cyi + j*by; the
// K x K sum is taken along p first, then along q.
template <int K, bool CLAMP>
__device__ double rotate_at64(const double *__restrict__ src, const SimDev &sd, int i, int j)
{
    const int n = sd.n;
    constexpr int o0 = (K - 1) / 2;
    const double dx = fma((double)j, sd.bx, fma((double)i, sd.axi, sd.ax0));
    const double dy = fma((double)j, sd.by, fma((double)i, sd.cyi, sd.cy0));
    const double fx = floor(dx), fy = floor(dy);
    const int ix = i + (int)fx, iy = j + (int)fy;
    double lx[K], ly[K];
    lagrange64<K>(dx - fx, lx);
    lagrange64<K>(dy - fy, ly);
    double f[K][K];
    if (ix - o0 >= 0 && ix + K - 1 - o0 < n && iy - o0 >= 0 && iy + K - 1 - o0 < n) {
        const double *base = src + (size_t)(ix - o0) * n + (iy - o0);
#pragma unroll
        for (int a = 0; a < K; ++a)
#pragma unroll
            for (int b = 0; b < K; ++b) f[a][b] = base[(size_t)a * n + b];
    } else {
#pragma unroll
        for (int a = 0; a < K; ++a)
#pragma unroll
            for (int b = 0; b < K; ++b) f[a][b] = ld_node(src, n, ix - o0 + a, iy - o0 + b);
    }
    double v = 0.0;
#pragma unroll
    for (int a = 0; a < K; ++a) {
        double r = ly[0] * f[a][0];
#pragma unroll
        for (int b = 1; b < K; ++b) r = fma(ly[b], f[a][b], r);
        v = a == 0 ? lx[0] * r : fma(lx[a], r, v);
    }
    if constexpr (CLAMP) {
        const double lo = fmin(fmin(f[o0][o0], f[o0][o0 + 1]), fmin(f[o0 + 1][o0], f[o0 + 1][o0 + 1]));
        const double hi = fmax(fmax(f[o0][o0], f[o0][o0 + 1]), fmax(f[o0 + 1][o0], f[o0 + 1][o0 + 1]));
        v = v < lo ? lo : (v > hi ? hi : v);
    }
    return v;
}

// ------------------------------------------------- standard rotation, FP32
// Source displacement computed in FP64 from the exact linear form, then the
// fraction and the K x K weighted sum in FP32.
template <int K, bool CLAMP>
__device__ float rotate_at32(const float *__restrict__ src, const SimDev &sd, int i, int j,
                             double Ai, double Ci)
{
    const int n = sd.n;
    const double dx = fma((double)j, sd.bx, Ai);
    const double dy = fma((double)j, sd.by, Ci);
    const double fx = floor(dx), fy = floor(dy);
    const float tx = (float)(dx - fx), ty = (float)(dy - fy);
    const int mx = i + (int)fx, my = j + (int)fy;
    float lx[K], ly[K];
    lagrange32<K>(tx, lx);
    lagrange32<K>(ty, ly);
    constexpr int o0 = (K - 1) / 2;
    float f[K][K];
    if (mx - o0 >= 0 && mx + K - 1 - o0 < n && my - o0 >= 0 && my + K - 1 - o0 < n) {
        const float *base = src + (size_t)(mx - o0) * n + (my - o0);
#pragma unroll
        for (int a = 0; a < K; ++a)
#pragma unroll
            for (int b = 0; b < K; ++b) f[a][b] = base[(size_t)a * n + b];
    } else {
#pragma unroll
        for (int a = 0; a < K; ++a)
#pragma unroll
            for (int b = 0; b < K; ++b) f[a][b] = ld_node(src, n, mx - o0 + a, my - o0 + b);
    }
    float v = 0.0f;
#pragma unroll
    for (int a = 0; a < K; ++a) {
        float r = 0.0f;
#pragma unroll
        for (int b = 0; b < K; ++b) r = fmaf(ly[b], f[a][b], r);
        v = fmaf(lx[a], r, v);
    }
    if constexpr (CLAMP) {
        const float lo = fminf(fminf(f[o0][o0], f[o0][o0 + 1]), fminf(f[o0 + 1][o0], f[o0 + 1][o0 + 1]));
        const float hi = fmaxf(fmaxf(f[o0][o0], f[o0][o0 + 1]), fmaxf(f[o0 + 1][o0], f[o0 + 1][o0 + 1]));
        v = fminf(fmaxf(v, lo), hi);
    }
    return v;
}

// 1-D interpolation of an LDS column (length n) at integer base m and
// fraction weights l (stencil offsets -(K-1)/2 ..), zero outside [0, n)
template <typename T, int K, bool CLAMP>
__device__ __forceinline__ T interp_lds(const T *col, int n, int m, const T *l)
{
    constexpr int o0 = (K - 1) / 2;
    T v = T(0);
    T f[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int jj = m - o0 + k;
        f[k] = (jj >= 0 && jj < n) ? col[jj] : T(0);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) v += l[k] * f[k];
    if constexpr (CLAMP) {
        const T a = f[o0], b = f[o0 + 1];
        const T lo = a < b ? a : b, hi = a < b ? b : a;
        v = v < lo ? lo : (v > hi ? hi : v);
    }
    return v;
}

// Visit every (column c < w, row j < n) of a strip with 256 threads, lanes
// along j (contiguous in memory).
template <typename F>
__device__ __forceinline__ void for_strip(int w, int n, F &&body)
{
    const int tid = threadIdx.x;
    if (n >= kThreads) {
        for (int c = 0; c < w; ++c)
            for (int j = tid; j < n; j += kThreads) body(c, j);
    } else {
        const int G = kThreads / n;
        const int g = tid / n, j = tid - g * n;
        if (g < G)
            for (int c = g; c < w; c += G) body(c, j);
    }
}

// =====================================================================
// The fused step.  One workgroup owns a strip of whole columns
// (i0 .. i0+w-1, all j) of one simulation:
//   prologue  s = Q0/Q^ from the FP64 column sums; wake V for the strip's
//             columns (FP64 / FP32 Toeplitz row slice) or read V from the
//             matrix-core wake;
//   phase R   rotated, renormalised values of the strip -> LDS A
//             (taps read from the previous density in global memory);
//   phase K   kick along p -> LDS B;
//   phase F   damping/diffusion, store psi^_{t+1}, and its FP64 column sums.
// =====================================================================
template <typename T, int K, int WAKE, bool CLAMP, int ROT>
__global__ __launch_bounds__(kThreads) void step_kernel(const SimDev *__restrict__ sims,
                                                        const Unit *__restrict__ units,
                                                        int nunits, int parity)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[kThreads];
    __shared__ double sh_shift[kMaxStrip];
    __shared__ T sh_kw[kMaxStrip][4];
    __shared__ int sh_km[kMaxStrip];
    __shared__ double sh_s;

    const Unit u = units[blockIdx.x];
    if (u.w == 0) return;                     // padding slot
    const SimDev &sd = sims[u.sim];
    const int n = sd.n, w = u.w, i0 = u.i0, tid = threadIdx.x;
    const T *__restrict__ src = (const T *)sd.psi[parity];
    T *__restrict__ dst = (T *)sd.psi[parity ^ 1];
    const double *__restrict__ cs = sd.colsum[parity];
    double *__restrict__ cs_next = sd.colsum[parity ^ 1];
    T *A = (T *)smem_raw;
    T *B = A + (size_t)w * n;

    // ---- prologue: renormalisation factor and the wake slice
    double s;
    if constexpr (WAKE == WAKE_EXTERNAL) {
        s = sd.sext[parity];
    } else {
        double part = 0.0;
        for (int k = tid; k < n; k += kThreads) part += cs[k];
        const double Qh = block_sum(part, red) * sd.dq * sd.dp;
        s = sd.renorm ? sd.Q0 / Qh : 1.0;
    }
    if constexpr (WAKE == WAKE_FUSED) {
        // V_i = S * s * sum_j w[i-j] * dp * colsum_j for the strip's columns
        const int parts = w <= kThreads ? kThreads / w : 1;
        const int c = tid / parts, pt = tid - c * parts;
        double acc = 0.0;
        if (c < w) {
            const int i = i0 + c;
            if constexpr (sizeof(T) == 8) {
                for (int j = pt; j < n; j += parts) acc += sd.wl64[i - j + n - 1] * (sd.dp * cs[j]);
            } else {
                float a32 = 0.0f;
                int cnt = 0;
                for (int j = pt; j < n; j += parts) {
                    a32 = fmaf(sd.wl32[i - j + n - 1], (float)(sd.dp * cs[j]), a32);
                    if (++cnt == 32) { acc += a32; a32 = 0.0f; cnt = 0; }
                }
                acc += a32;
            }
        }
        __syncthreads();
        red[tid] = acc;
        __syncthreads();
        if (tid < w) {
            double v = 0.0;
            for (int k = 0; k < parts; ++k) v += red[tid * parts + k];
            sh_shift[tid] = sd.S * s * v * sd.kick;      // kick shift in cells
            sd.vext[parity * n + i0 + tid] = (float)(sd.S * s * v);   // the wake this step used
        }
    } else if constexpr (WAKE == WAKE_EXTERNAL) {
        if (tid < w) sh_shift[tid] = (double)sd.vext[parity * n + i0 + tid] * sd.kick;
    } else {
        if (tid < w) sh_shift[tid] = 0.0;
    }
    if (tid == 0) sh_s = s;
    __syncthreads();
    // per-column kick weights: integer base and fraction of the shift
    if (tid < w) {
        const double sh = sh_shift[tid];
        const double fl = floor(sh);
        T l[K];
        if constexpr (sizeof(T) == 8) lagrange64<K>(sh - fl, (double *)l);
        else lagrange32<K>((float)(sh - fl), (float *)l);
        for (int k = 0; k < K; ++k) sh_kw[tid][k] = l[k];
        sh_km[tid] = (int)fmax(fmin(fl, 1.0e6), -1.0e6);
    }
    __syncthreads();
    const T sT = (T)sh_s;

    // ---- phase R: rotation -> A
    if constexpr (ROT == 0) {
        for_strip(w, n, [&](int c, int j) {
            const int i = i0 + c;
            T v;
            if constexpr (sizeof(T) == 8) {
                v = rotate_at64<K, CLAMP>((const double *)src, sd, i, j);
            } else {
                const double Ai = fma((double)i, sd.axi, sd.ax0);
                const double Ci = fma((double)i, sd.cyi, sd.cy0);
                v = rotate_at32<K, CLAMP>((const float *)src, sd, i, j, Ai, Ci);
            }
            A[(size_t)c * n + j] = v * sT;
        });
        __syncthreads();
    } else {
        // Manhattan: drift along q (pull from q - dtheta*p) from global -> B
        for_strip(w, n, [&](int c, int j) {
            const int i = i0 + c;
            T l[K];
            int m;
            if constexpr (sizeof(T) == 8) {
                const double rx = (double)i - sd.tw * (sd.pm + (double)j);
                const double mf = floor(rx);
                lagrange64<K>(rx - mf, (double *)l);
                m = (int)mf;
            } else {
                const double rx = (double)i - sd.tw * (sd.pm + (double)j);
                const double mf = floor(rx);
                lagrange32<K>((float)(rx - mf), (float *)l);
                m = (int)mf;
            }
            constexpr int o0 = (K - 1) / 2;
            T f[K];
            T v = T(0);
            for (int k = 0; k < K; ++k) f[k] = ld_node(src, n, m - o0 + k, j);
            for (int k = 0; k < K; ++k) v += l[k] * f[k];
            if (CLAMP) {
                const T a = f[o0], b = f[o0 + 1];
                const T lo = a < b ? a : b, hi = a < b ? b : a;
                v = v < lo ? lo : (v > hi ? hi : v);
            }
            B[(size_t)c * n + j] = v;
        });
        __syncthreads();
        // RF kick along p (pull from p + dtheta*q) B -> A
        for_strip(w, n, [&](int c, int j) {
            const int i = i0 + c;
            T l[K];
            int m;
            if constexpr (sizeof(T) == 8) {
                const double ry = (double)j + sd.tk * (sd.q_min / sd.dq + (double)i);
                const double mf = floor(ry);
                lagrange64<K>(ry - mf, (double *)l);
                m = (int)mf;
            } else {
                const double ry = (double)j + sd.tk * (sd.q_min / sd.dq + (double)i);
                const double mf = floor(ry);
                lagrange32<K>((float)(ry - mf), (float *)l);
                m = (int)mf;
            }
            A[(size_t)c * n + j] = interp_lds<T, K, CLAMP>(B + (size_t)c * n, n, m, l) * sT;
        });
        __syncthreads();
    }

    // ---- phase K: kick along p, A -> B
    for_strip(w, n, [&](int c, int j) {
        const T *col = A + (size_t)c * n;
        B[(size_t)c * n + j] = interp_lds<T, K, CLAMP>(col, n, j + sh_km[c], sh_kw[c]);
    });
    __syncthreads();

    // ---- phase F: damping/diffusion B -> global and A (for the column sums)
    for_strip(w, n, [&](int c, int j) {
        const T *col = B + (size_t)c * n;
        const T fm = j > 0 ? col[j - 1] : T(0);
        const T f0 = col[j];
        const T f1 = j + 1 < n ? col[j + 1] : T(0);
        const T f2 = j + 2 < n ? col[j + 2] : T(0);
        T out;
        if constexpr (sizeof(T) == 8) {
            // the same per-row coefficients as the FP32 branch below, in FP64
            const double u = sd.pm + (double)j;
            const double k1 = sd.bt / 6.0, k2 = sd.bt / (sd.dp * sd.dp);
            const double em = fma(-2.0 * k1, u - 1.0, k2);
            const double e0 = fma(-3.0 * k1, u, -2.0 * k2);
            const double e1 = fma(6.0 * k1, u + 1.0, k2);
            const double e2 = -k1 * (u + 2.0);
            out = f0 + fma(em, fm, fma(e0, f0, fma(e1, f1, e2 * f2)));
        } else {
            // psi + bt*[(-2 g_{j-1} - 3 g_j + 6 g_{j+1} - g_{j+2})/(6dp) + (f_{j-1} - 2 f_j + f_{j+1})/dp^2]
            // with g = p*psi, p_{j+o}/dp = u + o, u = p_min/dp + j
            const float u = (float)(sd.pm + (double)j);
            const float k1 = (float)(sd.bt / 6.0), k2 = (float)(sd.bt / (sd.dp * sd.dp));
            const float em = fmaf(-2.0f * k1, u - 1.0f, k2);
            const float e0 = fmaf(-3.0f * k1, u, -2.0f * k2);
            const float e1 = fmaf(6.0f * k1, u + 1.0f, k2);
            const float e2 = -k1 * (u + 2.0f);
            out = f0 + fmaf(em, fm, fmaf(e0, f0, fmaf(e1, f1, e2 * f2)));
        }
        dst[(size_t)(i0 + c) * n + j] = out;
        A[(size_t)c * n + j] = out;
    });
    __syncthreads();

    // ---- FP64 column sums of the stored density: one wave per column
    {
        const int lane = tid & 63, wv = tid >> 6;
        for (int c = wv; c < w; c += kWaves) {
            double acc = 0.0;
            for (int j = lane; j < n; j += 64) acc += (double)A[(size_t)c * n + j];
            acc = wave_sum(acc);
            if (lane == 0) cs_next[i0 + c] = acc;
        }
    }
}

// =====================================================================
// Column sums of a stored density (initial projection after an upload).
// grid.x: column blocks of 4 (one wave per column), grid.y: simulation.
// =====================================================================
template <typename T>
__global__ __launch_bounds__(kThreads) void project_kernel(const SimDev *__restrict__ sims,
                                                           const int *__restrict__ which, int parity)
{
    const SimDev &sd = sims[which[blockIdx.y]];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = blockIdx.x * kWaves + wv;
    if (i >= sd.n) return;
    const T *f = (const T *)sd.psi[parity] + (size_t)i * sd.n;
    double acc = 0.0;
    for (int j = lane; j < sd.n; j += 64) acc += (double)f[j];
    acc = wave_sum(acc);
    if (lane == 0) sd.colsum[parity][i] = acc;
}

// =====================================================================
// FP64 diagnostics of the current state, in four launches:
//   moments_kernel (16 columns per workgroup): per column sum psi,
//     sum p psi, sum p^2 psi;
//   stats_kernel (one workgroup per simulation): s, rho = s*dp*colsum and
//     the moments from the column sums; dynamic LDS: 2n doubles;
//   wakev_kernel (64 rows per workgroup): V = S*T(w)*rho (FP64 Toeplitz);
//   power_kernel (one workgroup per simulation): P = sum rho V, the
//     non-finite flag and, optionally, a record row.
// =====================================================================
template <typename T>
__global__ __launch_bounds__(kThreads) void moments_kernel(const SimDev *__restrict__ sims,
                                                           const int *__restrict__ which,
                                                           const int *__restrict__ bufidx)
{
    const SimDev &sd = sims[which[blockIdx.y]];
    const int n = sd.n, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const T *f = (const T *)sd.psi[bufidx[blockIdx.y]];
    for (int c = 0; c < 4; ++c) {
        const int i = blockIdx.x * 16 + c * kWaves + wv;
        if (i >= n) break;
        // blocks of 256 rows, four consecutive rows per lane, a wave sum per
        // block, the blocks added in order: the order in which the staged step
        // kernel forms the same sums when a record row follows it
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int j0 = 0; j0 < n; j0 += 256) {
            double m0 = 0.0, m1 = 0.0, m2 = 0.0;
            const int j = j0 + 4 * lane;
            for (int r = 0; r < 4 && j + r < n; ++r) {
                const double v = stored_value(f[(size_t)i * n + j + r], sd.fixb);
                const double pj = fma((double)(j + r), sd.dp, sd.p_min);
                m0 += v;
                m1 = fma(pj, v, m1);
                m2 = fma(pj * pj, v, m2);
            }
            a0 += wave_sum(m0);
            a1 += wave_sum(m1);
            a2 += wave_sum(m2);
        }
        if (lane == 0) {
            sd.mom[3 * i] = a0;
            sd.mom[3 * i + 1] = a1;
            sd.mom[3 * i + 2] = a2;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void stats_kernel(const SimDev *__restrict__ sims,
                                                         const int *__restrict__ which,
                                                         const int *__restrict__ bufidx)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[kThreads];
    const SimDev &sd = sims[which[blockIdx.x]];
    const int n = sd.n, tid = threadIdx.x;
    double *c0 = (double *)smem_raw;       // column sums
    double *rho = c0 + n;
    double spc = 0.0, sppc = 0.0;          // per-thread partials of sum p psi, p^2 psi
    for (int i = tid; i < n; i += kThreads) {
        c0[i] = sd.mom[3 * i];
        spc += sd.mom[3 * i + 1];
        sppc += sd.mom[3 * i + 2];
    }
    __syncthreads();
    double s0 = 0.0, sq = 0.0, sqq = 0.0;
    for (int i = tid; i < n; i += kThreads) {
        const double q = sd.q_min + i * sd.dq;
        s0 += c0[i];
        sq += q * c0[i];
        sqq += q * q * c0[i];
    }
    s0 = block_sum(s0, red);
    sq = block_sum(sq, red);
    sqq = block_sum(sqq, red);
    const double sp = block_sum(spc, red);
    const double spp = block_sum(sppc, red);
    double Qh = sd.dq * sd.dp * s0;
    if constexpr (std::is_same_v<T, int64_t>) {
        // the fixed-point step's factor: exact integer charge from the column sums
        const int64_t *cs = (const int64_t *)sd.colsum[bufidx[blockIdx.x]];
        int64_t ph = 0, pl = 0;
        for (int k = tid; k < n; k += kThreads) {
            ph += cs[2 * k];
            pl += cs[2 * k + 1];
        }
        const int64_t H = block_sum_i64(ph, (int64_t *)red);
        const int64_t L = block_sum_i64(pl, (int64_t *)red);
        Qh = ldexp((double)H * 4294967296.0 + (double)L, -sd.fixb) * sd.dq * sd.dp;
    }
    const double s = sd.renorm ? sd.Q0 / Qh : 1.0;
    for (int i = tid; i < n; i += kThreads) {
        rho[i] = s * sd.dp * c0[i];
        sd.rho_out[i] = rho[i];
    }
    if (tid == 0) {
        const double mq = sq / s0, mp = sp / s0;
        const double st[7] = {s * Qh, mq, sqrt(fmax(sqq / s0 - mq * mq, 0.0)), mp,
                              sqrt(fmax(spp / s0 - mp * mp, 0.0)), 0.0, s};
        for (int k = 0; k < 7; ++k) sd.stat[k] = st[k];
    }
}

// V_i = S sum_j w[i-j] rho_j for 64 rows i per workgroup (grid.x: row tiles
// of the largest grid, grid.y: simulations); the four waves take every
// fourth j and their sums are added in a fixed order
__global__ __launch_bounds__(kThreads) void wakev_kernel(const SimDev *__restrict__ sims,
                                                         const int *__restrict__ which)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double part[kWaves][64];
    const SimDev &sd = sims[which[blockIdx.y]];
    const int n = sd.n, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int i0 = blockIdx.x * 64;
    if (i0 >= n) return;
    // rho and the tile's lag window in LDS: lw[k] = w[i0 - (n - 1) + k], so that
    // w[i - j] = lw[i - i0 + n - 1 - j] (dynamic LDS: (2 n + 63) doubles at most)
    double *rho = (double *)smem_raw;
    double *lw = rho + n;
    if (sd.has_wake) {
        const int nl = min(n + 63, 2 * n - 1 - i0);
        for (int k = tid; k < n; k += kThreads) rho[k] = sd.rho_out[k];
        for (int k = tid; k < nl; k += kThreads) lw[k] = sd.wl64[i0 + k];
    }
    __syncthreads();
    const int i = i0 + lane;
    double v = 0.0;
    if (sd.has_wake && i < n) {
        const double *wi = lw + lane + n - 1;            // wi[-j] = w[i - j]
        double v0 = 0.0, v1 = 0.0;
        int j = wv;
        for (; j + kWaves < n; j += 2 * kWaves) {
            v0 = fma(wi[-j], rho[j], v0);
            v1 = fma(wi[-j - kWaves], rho[j + kWaves], v1);
        }
        if (j < n) v0 = fma(wi[-j], rho[j], v0);
        v = v0 + v1;
    }
    part[wv][lane] = v;
    __syncthreads();
    if (wv == 0 && i < n) sd.v_out[i] = sd.has_wake ? sd.S * ((part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane])) : 0.0;
}

// dynamic LDS of wakev_kernel for grids of at most n points
__host__ __device__ inline size_t wakev_lds(int n) { return (size_t)(2 * n + 63) * sizeof(double); }

// P = sum_i rho_i V_i, the non-finite flag, and the record row
__global__ __launch_bounds__(kThreads) void power_kernel(const SimDev *__restrict__ sims,
                                                         const int *__restrict__ which, int64_t rec_base,
                                                         int every, int record)
{
    __shared__ double red[kThreads];
    const SimDev &sd = sims[which[blockIdx.x]];
    const int n = sd.n, tid = threadIdx.x;
    double pw = 0.0;
    for (int i = tid; i < n; i += kThreads) pw += sd.rho_out[i] * sd.v_out[i];
    pw = block_sum(pw, red);
    if (tid == 0) {
        double st[7];
        for (int k = 0; k < 7; ++k) st[k] = sd.stat[k];
        st[5] = pw;
        sd.stat[5] = pw;
        sd.stat[7] = (isfinite(st[0]) && isfinite(pw)) ? 0.0 : 1.0;
        if (record && sd.ring) {
            const int64_t row = *sd.ring_rows;
            if (row < sd.ring_cap) {
                double *r = sd.ring + 7 * row;
                r[0] = (double)(rec_base + (row + 1) * every - sd.step0);
                for (int k = 0; k < 5; ++k) r[1 + k] = st[k];
                r[6] = pw;
            }
            *sd.ring_rows = row + 1;
        }
    }
}

// =====================================================================
// Wake table (Sec. II.B, Eq. "wakepotential"): for every lag
// m in [-(n-1), n-1], wl[m+n-1] = (1/M) sum_{k<M} Re(Z_k e^{2 pi i k m'/M}),
// m' = m mod M, Z Hermitian-extended (Im Z_0, Im Z_{M/2} ignored).
// =====================================================================
__global__ __launch_bounds__(kThreads) void wake_table_kernel(int n, int M, const double *__restrict__ zr,
                                                              const double *__restrict__ zi,
                                                              double *__restrict__ wl64,
                                                              float *__restrict__ wl32)
{
    const int idx = blockIdx.x * kThreads + threadIdx.x;
    if (idx >= 2 * n - 1) return;
    const int m = idx - (n - 1);
    const int mm = ((m % M) + M) % M;
    double acc = 0.0;
    for (int k = 0; k < M; ++k) {
        double a, b;
        if (k == 0 || 2 * k == M) { a = zr[k]; b = 0.0; }
        else if (2 * k < M)       { a = zr[k]; b = zi[k]; }
        else                      { a = zr[M - k]; b = -zi[M - k]; }
        const long long kl = ((long long)k * mm) % M;
        double sn, cn;
        sincospi(2.0 * (double)kl / (double)M, &sn, &cn);
        acc += a * cn - b * sn;
    }
    const double v = acc / (double)M;
    wl64[idx] = v;
    wl32[idx] = (float)v;
}

// =====================================================================
// Matrix-core wake (mixed precision).  The Toeplitz product V = S T rho is
// rewritten in 16 x 16 blocks: with V and rho viewed as 16 x nb matrices
// (column J holds entries 16J .. 16J+15), V[:, I] = sum_d T_d rho[:, I-d]
// where T_d[a][c] = w[16d + a - c] depends only on the block diagonal d.
// For a tile of 16 output columns every d is one 16x16x16 product, so the
// N^2 multiply-adds run on the matrix cores.  Operands are split into a
// high and a low 16-bit part (x = hi + lo) and three products
// hi*hi + hi*lo + lo*hi are accumulated in FP32.  For FP16 both operands
// are pre-scaled by powers of two so that the low parts stay normal.
// Operand layout of the 16x16x16 instructions: lane l holds A[l%16][4(l/16)+q],
// B[4(l/16)+q][l%16] and D[4(l/16)+q][l%16], q = 0..3.
// =====================================================================
typedef short  v4s __attribute__((ext_vector_type(4)));
typedef _Float16 v4h __attribute__((ext_vector_type(4)));
typedef float  v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <bool FP16>
__device__ __forceinline__ void split16(float x, uint16_t &hi, uint16_t &lo)
{
    if constexpr (FP16) {
        const _Float16 h = (_Float16)x;
        const _Float16 l = (_Float16)(x - (float)h);
        hi = __builtin_bit_cast(uint16_t, h);
        lo = __builtin_bit_cast(uint16_t, l);
    } else {
        hi = f32_to_bf16_rne(x);
        lo = f32_to_bf16_rne(x - bf16_to_f32(hi));
    }
}

// ---------------------------------------------------------------------
// Matrix-core wake, one workgroup of kWaves waves per (simulation, tile of
// 16 block columns).  The high and low 16-bit parts of the (power-of-two
// scaled) lag table are made once at set-up (wake_split_kernel).  The
// workgroup stages rho's hi/lo parts for the block columns the tile touches
// and two copies of its lag range, reversed and offset by one element, so
// that every lane reads its four consecutive Toeplitz entries as two aligned
// 32-bit words.  The block diagonals d are dealt out to the waves in turn;
// the per-wave partial products are added in FP64 in wave order.
// ---------------------------------------------------------------------
struct WakeTile {
    int32_t sim, tile, pad0, pad1;
};

// Lag tables of the matrix-core wake, made once at set-up: four arrays of
// wake_rev_len(n) 16-bit values, the hi and lo parts of w[lag] * wscale in
// reversed lag order (entry P + k holds lag n - 1 - k, k = 0 .. 2n-2; zero
// elsewhere), and the same two arrays shifted by one entry.  A tile's lag
// window is then one contiguous, 16-byte aligned run of each array.
__host__ __device__ inline int wake_rev_pad(int n) { return 16 + ((8 - (n & 7)) & 7); }
__host__ __device__ inline int wake_rev_len(int n) { return (wake_rev_pad(n) + 2 * n + 24 + 7) & ~7; }

template <bool FP16>
__global__ void wake_split_kernel(int n, const double *__restrict__ wl64, double wscale, uint16_t *__restrict__ split)
{
    const int LW = wake_rev_len(n), P = wake_rev_pad(n);
    const int idx = blockIdx.x * kThreads + threadIdx.x;
    if (idx >= LW) return;
    uint16_t h[2] = {0, 0}, l[2] = {0, 0};
    for (int sft = 0; sft < 2; ++sft) {
        const int k = idx + sft - P;                    // reversed position: lag n - 1 - k
        if (k >= 0 && k <= 2 * n - 2) split16<FP16>((float)(wl64[2 * n - 2 - k] * wscale), h[sft], l[sft]);
    }
    split[idx] = h[0];
    split[LW + idx] = l[0];
    split[2 * LW + idx] = h[1];
    split[3 * LW + idx] = l[1];
}


// LDS bytes of tile `tile` of an n-point wake: the staged rho and lag runs,
// then (8-byte aligned) the FP64 wave partials and the block reductions.
__host__ __device__ inline size_t wake_mfma_tile_lds(int n, int tile)
{
    const int nb = (n + 15) / 16, I0 = 16 * tile;
    const int dmin = max(-(nb - 1), I0 - (nb - 1)), dmax = min(nb - 1, I0 + 15);
    const size_t NR = 16 * (16 + dmax - dmin), NL = 16 * (dmax - dmin) + 31;
    const size_t NLp = (NL + 1 + 7) & ~(size_t)7;
    const size_t head = ((2 * NR + 4 * NLp) * sizeof(uint16_t) + 15) & ~(size_t)15;
    return head + ((size_t)(kWaves - 1) * 64 * 4 + 2 * kWaves) * sizeof(double);
}
__host__ __device__ inline size_t wake_mfma_lds(int n)
{
    size_t m = 0;
    const int nb = (n + 15) / 16;
    for (int t = 0; t < (nb + 15) / 16; ++t) m = m > wake_mfma_tile_lds(n, t) ? m : wake_mfma_tile_lds(n, t);
    return m;
}

// One tile of the matrix-core wake of simulation sd from the column sums in
// buffer `parity`; writes V (vext[parity]) for the tile's rows and, for tile
// 0, the factor s the wake was made with (sext[parity]).  All LDS is the
// dynamic buffer.
template <bool FP16, bool COH = false, bool OUTCOH = false>
__device__ void wake_mfma_tile(const SimDev &sd, int tile, int parity)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int n = sd.n, tid = threadIdx.x, lane = tid & 63, nb = (n + 15) / 16;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int I0 = 16 * tile;
    const int dmin = max(-(nb - 1), I0 - (nb - 1)), dmax = min(nb - 1, I0 + 15);
    const int Jlo = I0 - dmax;
    const int NR = 16 * (16 + dmax - dmin);            // rho entries of block columns Jlo..Jhi
    const int Lhi = 16 * dmax + 15;                     // highest lag used
    const int NL = 16 * (dmax - dmin) + 31;             // lags Lhi-NL+1 .. Lhi
    const int NLp = (NL + 1 + 7) & ~7;                  // staged entries per copy (16-byte runs)
    uint16_t *rhi = (uint16_t *)smem_raw;
    uint16_t *rlo = rhi + NR;
    uint16_t *c0h = rlo + NR, *c0l = c0h + NLp, *c1h = c0l + NLp, *c1l = c1h + NLp;
    double *wsum = (double *)(smem_raw + (((2 * NR + 4 * NLp) * sizeof(uint16_t) + 15) & ~(size_t)15));
    double *red = wsum + (kWaves - 1) * 64 * 4;        // 2 * kWaves entries
    typedef const __attribute__((address_space(1))) double gdouble;
    typedef const __attribute__((address_space(1))) uint16_t gu16;
    const double *cs = sd.colsum[parity];

    // charge and largest column sum (each thread adds its columns in order,
    // then a fixed tree); read again below for the split, so that no
    // per-thread array of column sums stays live in registers
    double part = 0.0, mx = 0.0;
    for (int k0 = tid; k0 < n; k0 += kCsBatch * kThreads) {
        double v[kCsBatch];
        load_cs_batch<COH>(cs, k0, n, v);
#pragma unroll
        for (int q = 0; q < kCsBatch; ++q) {
            part += v[q];
            mx = fmax(mx, fabs(v[q]));
        }
    }
    // lag window: copy 0 (entry y = lag Lhi - y) and copy 1 (shifted by one),
    // hi and lo, each one aligned run of the reversed tables
    {
        const int LW = wake_rev_len(n), st0 = wake_rev_pad(n) + n - 1 - Lhi;   // st0 % 8 == 0
        typedef unsigned int v4u __attribute__((ext_vector_type(4)));
        typedef const __attribute__((address_space(1))) v4u gv4u;
        const int q8 = NLp / 8;
        for (int k = tid; k < 4 * q8; k += kThreads) {
            const int arr = k / q8, q = k - arr * q8;
            const v4u v = *(gv4u *)(sd.wsplit + (size_t)arr * LW + st0 + 8 * q);
            *(v4u *)(c0h + (size_t)arr * NLp + 8 * q) = v;
        }
    }
    // rho entries outside the grid are zero
    for (int k = tid; k < NR; k += kThreads) {
        const int g = 16 * Jlo + k;
        if (g < 0 || g >= n) { rhi[k] = 0; rlo[k] = 0; }
    }
    part = wave_sum(part);
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if (lane == 0) { red[wv] = part; red[kWaves + wv] = mx; }
    __syncthreads();
    part = red[0];
    mx = red[kWaves];
    for (int k = 1; k < kWaves; ++k) { part += red[k]; mx = fmax(mx, red[kWaves + k]); }
    const double Qh = part * sd.dq * sd.dp;
    const double s = sd.renorm ? sd.Q0 / Qh : 1.0;
    const double rmax = mx * s * sd.dp;
    int e = 0;
    if (FP16 && rmax > 0.0) { frexp(rmax, &e); e = 14 - e; }
    const double rscale = ldexp(s * sd.dp, e);
    {
        const int g0 = max(0, 16 * Jlo), g1 = min(n, 16 * Jlo + NR);
        for (int k0 = g0 + tid; k0 < g1; k0 += kCsBatch * kThreads) {
            double v[kCsBatch];
            load_cs_batch<COH>(cs, k0, g1, v);
#pragma unroll
            for (int q = 0; q < kCsBatch; ++q) {
                const int g = k0 + q * kThreads;
                if (g < g1) {
                    uint16_t h, l;
                    split16<FP16>((float)(v[q] * rscale), h, l);
                    rhi[g - 16 * Jlo] = h;
                    rlo[g - 16 * Jlo] = l;
                }
            }
        }
    }
    __syncthreads();

    const int a = lane & 15, kq = 4 * (lane >> 4);
    // y0 = Lhi - (16d + a - kq) for d = dmax is 15 - a + kq; even y0 read copy 0 at y0,
    // odd y0 read copy 1 (shifted by one) at y0 - 1
    const int y00 = 15 - a + kq;
    const bool odd = y00 & 1;
    const uint16_t *ah = odd ? c1h + (y00 - 1) : c0h + y00;
    const uint16_t *al = odd ? c1l + (y00 - 1) : c0l + y00;
    v4f acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = acc0, acc2 = acc0;
    // fragments of block diagonal d, loaded one iteration ahead of their use
    auto frag = [&](int d, uint2 &A_h, uint2 &A_l, uint2 &B_h, uint2 &B_l) {
        const int yo = 16 * (dmax - d);
        A_h = make_uint2(*(const uint32_t *)(ah + yo), *(const uint32_t *)(ah + yo + 2));
        A_l = make_uint2(*(const uint32_t *)(al + yo), *(const uint32_t *)(al + yo + 2));
        const int bidx = 16 * (I0 + a - d - Jlo) + kq;
        B_h = *(const uint2 *)(rhi + bidx);
        B_l = *(const uint2 *)(rlo + bidx);
    };
    int d = dmax - wv;
    uint2 A_h, A_l, B_h, B_l;
    if (d >= dmin) frag(d, A_h, A_l, B_h, B_l);
    for (; d >= dmin; d -= kWaves) {
        uint2 nA_h = A_h, nA_l = A_l, nB_h = B_h, nB_l = B_l;
        if (d - kWaves >= dmin) frag(d - kWaves, nA_h, nA_l, nB_h, nB_l);
        if constexpr (FP16) {
            acc0 = __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(v4h, A_h), __builtin_bit_cast(v4h, B_h), acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(v4h, A_h), __builtin_bit_cast(v4h, B_l), acc1, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(v4h, A_l), __builtin_bit_cast(v4h, B_h), acc2, 0, 0, 0);
        } else {
            acc0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(v4s, A_h), __builtin_bit_cast(v4s, B_h), acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(v4s, A_h), __builtin_bit_cast(v4s, B_l), acc1, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(v4s, A_l), __builtin_bit_cast(v4s, B_h), acc2, 0, 0, 0);
        }
        A_h = nA_h; A_l = nA_l; B_h = nB_h; B_l = nB_l;
    }
    double t[4];
    for (int q = 0; q < 4; ++q) t[q] = (double)acc0[q] + ((double)acc1[q] + (double)acc2[q]);
    if (wv > 0)
        for (int q = 0; q < 4; ++q) wsum[((wv - 1) * 64 + lane) * 4 + q] = t[q];
    __syncthreads();
    if (wv == 0) {
        const double outscale = ldexp(sd.S, -e) * sd.sext[2];
        for (int q = 0; q < 4; ++q) {
            double v = t[q];
            for (int k = 0; k < kWaves - 1; ++k) v += wsum[(k * 64 + lane) * 4 + q];
            const int i = 16 * (I0 + a) + kq + q;
            if (i < n) store_wake_f<OUTCOH>(sd.vext + parity * n + i, (float)(v * outscale));
        }
        if (tile == 0 && lane == 0) store_wake_d<OUTCOH>(sd.sext + parity, s);
    }
}

template <bool FP16>
__global__ __launch_bounds__(kThreads) void wake_mfma2_kernel(const SimDev *__restrict__ sims,
                                                              const WakeTile *__restrict__ tiles, int parity)
{
    const WakeTile wt = tiles[blockIdx.x];
    wake_mfma_tile<FP16>(sims[wt.sim], wt.tile, parity);
}


// Vector-ALU wake of the FP32 form, one workgroup per (simulation, tile of
// kWakeVecRows rows, one per lane): V_i = S s sum_j w[i-j] rho_j with FP32
// products and partial sums over blocks of 32 consecutive j, added in FP64;
// each wave takes a quarter of the j range and the four quarters are added
// in order (Sec. II.B; the same term definition as the fused wake of the
// FP64/generic kernel).  LDS: rho (n floats) and the tile's lag window
// (n + kWakeVecRows - 1 floats), then (16-byte aligned) the charge's wave
// sums and the quarters' partial wakes.  Small tiles keep the wake short on
// the one-launch tick of a single simulation, whose units wait for it.
constexpr int kWakeVecRows = 64;
__host__ __device__ inline size_t wake_vec_head(int n)
{
    return ((size_t)(2 * n + kWakeVecRows - 1) * sizeof(float) + 15) & ~(size_t)15;
}
__host__ __device__ inline size_t wake_vec_lds(int n)
{
    return wake_vec_head(n) + (size_t)kWaves * (1 + kWakeVecRows) * sizeof(double);
}

template <bool COH = false, bool OUTCOH = false>
__device__ void wake_vec_tile(const SimDev &sd, int tile, int parity)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int n = sd.n, tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int i0 = kWakeVecRows * tile;
    float *rho = (float *)smem_raw;
    float *lag = rho + n;                              // lag[k] = w[i0 + k - (n - 1)]
    double *red = (double *)(smem_raw + wake_vec_head(n));
    double *wpart = red + kWaves;                      // [kWaves][kWakeVecRows] partial wakes
    typedef const __attribute__((address_space(1))) double gdouble;
    typedef const __attribute__((address_space(1))) float gfloat;
    const double *cs = sd.colsum[parity];
    gfloat *wl = (gfloat *)sd.wl32;
    double part = 0.0;
    for (int k0 = tid; k0 < n; k0 += kCsBatch * kThreads) {
        double v[kCsBatch];
        load_cs_batch<COH>(cs, k0, n, v);
#pragma unroll
        for (int q = 0; q < kCsBatch; ++q) {
            const int k = k0 + q * kThreads;
            part += v[q];
            if (k < n) rho[k] = (float)(sd.dp * v[q]);
        }
    }
    for (int k = tid; k < n + kWakeVecRows - 1; k += kThreads) {
        const int ix = i0 + k;                         // wl32 index = lag + n - 1
        lag[k] = ix <= 2 * n - 2 ? wl[ix] : 0.0f;
    }
    part = wave_sum(part);
    if (lane == 0) red[wv] = part;
    __syncthreads();
    part = red[0];
    for (int k = 1; k < kWaves; ++k) part += red[k];
    const double s = sd.renorm ? sd.Q0 / (part * sd.dq * sd.dp) : 1.0;
    // row i = i0 + lane; wave wv sums j over its quarter [ja, jz) in FP32 blocks of 32
    const int i = i0 + lane;
    double acc = 0.0;
    if (i < n) {
        const float *lw = lag + lane + n - 1;          // lw[-j] = w[i - j]
        const int qn = (n + kWaves - 1) / kWaves, ja = wv * qn, jz = min(n, ja + qn);
        for (int jb = ja; jb < jz; jb += 32) {
            float a32 = 0.0f;
            const int je = jb + 32 < jz ? jb + 32 : jz;
#pragma unroll 8
            for (int j = jb; j < je; ++j) a32 = fmaf(lw[-j], rho[j], a32);
            acc += a32;
        }
    }
    wpart[wv * kWakeVecRows + lane] = acc;
    __syncthreads();
    if (wv == 0 && i < n) {
        const double v = (wpart[lane] + wpart[kWakeVecRows + lane]) +
                         (wpart[2 * kWakeVecRows + lane] + wpart[3 * kWakeVecRows + lane]);
        store_wake_f<OUTCOH>(sd.vext + parity * n + i, (float)(sd.S * s * v));
    }
    if (tile == 0 && tid == 0) store_wake_d<OUTCOH>(sd.sext + parity, s);
}

__global__ __launch_bounds__(kThreads) void wake_vec_kernel(const SimDev *__restrict__ sims,
                                                            const WakeTile *__restrict__ tiles, int parity)
{
    const WakeTile wt = tiles[blockIdx.x];
    wake_vec_tile(sims[wt.sim], wt.tile, parity);
}

// CSR spectrum of the state whose profile the diagnostics kernel left in
// rho_out (Sec. IV.C): out[k] = (S/M) m_k Re Z_k |rho~_k|^2, k = 0..M/2,
// rho~_k the DFT of the zero-padded profile, m_k = 2 for the bins that stand
// for k and M-k.  One thread per bin, over as many workgroups as needed.
__global__ __launch_bounds__(kThreads) void spectrum_kernel(const SimDev *__restrict__ sims, int which,
                                                            double *__restrict__ out)
{
    const SimDev &sd = sims[which];
    const int n = sd.n, M = sd.M;
    for (int k = blockIdx.x * kThreads + threadIdx.x; k <= M / 2; k += gridDim.x * kThreads) {
        double re = 0.0, im = 0.0;
        for (int j = 0; j < n; ++j) {
            const long long kj = ((long long)k * j) % M;
            double sn, cn;
            sincospi(2.0 * (double)kj / (double)M, &sn, &cn);
            re += sd.rho_out[j] * cn;
            im -= sd.rho_out[j] * sn;
        }
        const double mult = (k == 0 || 2 * k == M) ? 1.0 : 2.0;
        out[k] = sd.S / (double)M * mult * sd.zr64[k] * (re * re + im * im);
    }
}

// Haissinski starting distribution (Appendix A): rho ~ exp(-q^2/2 - U),
// U' = V[rho], dq*sum(rho) = Q0, solved by the damped fixed-point iteration
// rho <- (1-alpha) rho + alpha F(rho) from the Gaussian, U by the cumulative
// trapezoid rule from q_min; psi_ij = rho_i g_j with the unit Gaussian g in p
// normalised on the grid.  The iterate lives in rho_out, its wake in v_out
// (computed between the phases by wakev_kernel); one workgroup per phase:
//   phase 0: the Gaussian start;
//   phase 1: one damped update from V (cumulative trapezoid in order);
//   phase 2: psi from the final profile, in the storage type.
// dynamic LDS (phase 1): n doubles.
template <typename T>
__global__ __launch_bounds__(kThreads) void haissinski_kernel(const SimDev *__restrict__ sims, int which, int buf,
                                                              int phase, double alpha)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[kThreads];
    const SimDev &sd = sims[which];
    const int n = sd.n, tid = threadIdx.x;
    double *rho = sd.rho_out;
    if (phase == 0) {
        double part = 0.0;
        for (int i = tid; i < n; i += kThreads) {
            const double q = sd.q_min + i * sd.dq;
            part += exp(-0.5 * q * q);
        }
        const double tot = block_sum(part, red);
        for (int i = tid; i < n; i += kThreads) {
            const double q = sd.q_min + i * sd.dq;
            rho[i] = exp(-0.5 * q * q) * (sd.Q0 / (sd.dq * tot));
        }
    } else if (phase == 1) {
        double *F = (double *)smem_raw;
        const double *V = sd.v_out;
        if (tid == 0) {                      // cumulative trapezoid, in order
            double u = 0.0;
            F[0] = 0.0;
            for (int i = 1; i < n; ++i) {
                u += 0.5 * (V[i - 1] + V[i]) * sd.dq;
                F[i] = u;
            }
        }
        __syncthreads();
        double part = 0.0;
        for (int i = tid; i < n; i += kThreads) {
            const double q = sd.q_min + i * sd.dq;
            F[i] = exp(-0.5 * q * q - F[i]);
            part += F[i];
        }
        const double tot = block_sum(part, red);
        for (int i = tid; i < n; i += kThreads) rho[i] = (1.0 - alpha) * rho[i] + alpha * F[i] * (sd.Q0 / (sd.dq * tot));
    } else {
        double part = 0.0;
        for (int j = tid; j < n; j += kThreads) {
            const double p = sd.p_min + j * sd.dp;
            part += exp(-0.5 * p * p);
        }
        const double G = block_sum(part, red);
        T *out = (T *)sd.psi[buf];
        for (int i = blockIdx.x; i < n; i += gridDim.x)
            for (int j = tid; j < n; j += kThreads) {
                const double p = sd.p_min + j * sd.dp;
                out[(size_t)i * n + j] = to_stored<T>(rho[i] * exp(-0.5 * p * p) / (sd.dp * G), sd.fixb);
            }
    }
}

// Q0 = dq * dp * sum psi0 of the FP64 input, before any conversion to the
// storage type (one workgroup, fixed summation order)
__global__ __launch_bounds__(kThreads) void charge64_kernel(const double *__restrict__ psi, size_t nn, double dqdp,
                                                            double *__restrict__ out)
{
    __shared__ double red[kThreads];
    double part = 0.0;
    for (size_t z = threadIdx.x; z < nn; z += kThreads) part += psi[z];
    const double t = block_sum(part, red);
    if (threadIdx.x == 0) out[0] = t * dqdp;
}

// psi^ <- psi64 in the storage type; used by create and set_psi
template <typename T>
__global__ void import_kernel(const double *__restrict__ in, T *__restrict__ out, size_t nn, int fixb)
{
    const size_t z = (size_t)blockIdx.x * kThreads + threadIdx.x;
    if (z < nn) out[z] = to_stored<T>(in[z], fixb);
}

// psi64 <- s * psi^ (s from the latest diagnostics)
template <typename T>
__global__ void export_kernel(const T *__restrict__ in, const double *__restrict__ stat,
                              double *__restrict__ out, size_t nn, int fixb)
{
    const size_t z = (size_t)blockIdx.x * kThreads + threadIdx.x;
    if (z < nn) out[z] = stat[6] * stored_value(in[z], fixb);
}

}  // namespace vfp
