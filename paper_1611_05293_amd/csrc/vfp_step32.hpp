// vfp_step32.hpp -- the FP32 fused step for the standard rotation, staged
// through LDS (included by vfp.hip after vfp_kernels.hpp).
//
// One workgroup owns W whole q-columns (i0 .. i0+W-1, every p row j) of one
// simulation.  LDS holds
//   A[W][n + 2*kPad]   rotated, renormalised values (zero pads of kPad rows)
//   B[W][n + 2*kPad]   after the kick
//   S[W + 2*kH][kSY]   the previous density around the current 64-row chunk
//   Dm[W][kSY]         Manhattan rotation: the drifted chunk
// Phases:
//   R  per 64-row chunk: stage S with raw buffer loads (out-of-grid reads
//      return zero), then every wave interpolates one column of 64 rows
//      (lanes along p) from 16 LDS taps -> A;
//   K  kick along p with per-column weights (whole column in LDS) -> B;
//   F  damping/diffusion on 4 rows per lane, float4 stores of psi^_{t+1},
//      FP64 column sums by wave reduction.
// Phase R is either the standard 2-D rotation or the Manhattan pair (drift
// along q with one shift per row, then RF kick along p with one shift per
// column, both 1-D).  The source displacement must stay below 2 cells in
// each direction (floor in [-2, 1]); the host routes other grids to the
// generic kernel.
#pragma once

namespace vfp {

constexpr int kPad = 8;            // zero rows above and below each LDS column
constexpr int kH = 3;              // rotation halo in cells
constexpr int kJ = 64;             // rows per rotation chunk: one per lane
constexpr int kSY = kJ + 2 * kH;   // staged rows per chunk
constexpr int kPF = 10;            // staged columns per wave prefetched into registers

// Raw buffer over one column of n floats: reads outside [0, n) return 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t column_rsrc(const float *col, int n)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)col, (short)0, n * 4, 0x00020000);
}

// Cubic (K=4, offsets -1..2) and quadratic (K=3, offsets -1..1) Lagrange
// weights, rearranged for fused multiply-adds.
template <int K>
__device__ __forceinline__ void lagrange_fma(float t, float *l)
{
    if constexpr (K == 4) {
        const float a = fmaf(t, t, -t);              // t(t-1)
        const float a6 = a * (1.0f / 6.0f);
        const float a3 = a * (1.0f / 3.0f);
        const float b2 = fmaf(a, 0.5f, -1.0f);       // (t+1)(t-2)/2
        l[0] = fmaf(-a6, t, a3);                     // -t(t-1)(t-2)/6
        l[1] = fmaf(b2, t, -b2);                     // (t+1)(t-1)(t-2)/2
        l[2] = -b2 * t;                              // -(t+1)t(t-2)/2
        l[3] = fmaf(a6, t, a6);                      // (t+1)t(t-1)/6
    } else {
        const float a = fmaf(t, t, -t);              // t(t-1)
        l[0] = 0.5f * a;                             // t(t-1)/2
        l[1] = fmaf(-t, t, 1.0f);                    // 1 - t^2
        l[2] = fmaf(0.5f, a, t);                     // t(t+1)/2
    }
}

template <int K, int WAKE, bool CLAMP, int ROT>
__global__ __launch_bounds__(kThreads) void step32_kernel(const SimDev *__restrict__ sims,
                                                          const Unit *__restrict__ units, int nunits,
                                                          int parity)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[kThreads];
    __shared__ float sh_kw[kMaxStrip][4];
    __shared__ int sh_km[kMaxStrip];
    __shared__ double sh_shift[kMaxStrip];
    __shared__ float sh_rw[kMaxStrip][4];     // Manhattan RF kick: per-column weights
    __shared__ int sh_rm[kMaxStrip];          //                   and integer shift
    __shared__ float sh_s;
    constexpr int o0 = (K - 1) / 2;

    const Unit u = units[blockIdx.x];
    if (u.w == 0) return;                     // padding slot
    const SimDev &sd = sims[u.sim];
    const int n = sd.n, W = u.w, i0 = u.i0, tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);     // wave index, uniform
    const int LA = n + 2 * kPad;
    float *A = (float *)smem_raw;
    float *B = A + (size_t)W * LA;
    float *S = B + (size_t)W * LA;
    float *Dm = S + (size_t)(W + 2 * kH) * kSY;     // Manhattan: drifted chunk [W][kSY]
    const float *__restrict__ src = (const float *)sd.psi[parity];
    float *__restrict__ dst = (float *)sd.psi[parity ^ 1];
    const double *__restrict__ cs = sd.colsum[parity];
    double *__restrict__ cs_next = sd.colsum[parity ^ 1];

    // ---- prologue: renormalisation factor, wake slice, kick weights, pads
    double s;
    if constexpr (WAKE == WAKE_EXTERNAL) {
        s = sd.sext[0];
    } else {
        double part = 0.0;
        for (int k = tid; k < n; k += kThreads) part += cs[k];
        const double Qh = block_sum(part, red) * sd.dq * sd.dp;
        s = sd.renorm ? sd.Q0 / Qh : 1.0;
    }
    if constexpr (WAKE == WAKE_FUSED) {
        const int parts = kThreads / W;
        const int c = tid / parts, pt = tid - c * parts;
        double acc = 0.0;
        if (c < W) {
            const int i = i0 + c;
            float a32 = 0.0f;
            int cnt = 0;
            for (int j = pt; j < n; j += parts) {
                a32 = fmaf(sd.wl32[i - j + n - 1], (float)(sd.dp * cs[j]), a32);
                if (++cnt == 32) { acc += a32; a32 = 0.0f; cnt = 0; }
            }
            acc += a32;
        }
        __syncthreads();
        red[tid] = acc;
        __syncthreads();
        if (tid < W) {
            double v = 0.0;
            for (int k = 0; k < parts; ++k) v += red[tid * parts + k];
            sh_shift[tid] = sd.S * s * v * sd.kick;
            sd.vext[i0 + tid] = (float)(sd.S * s * v);      // the wake this step used
        }
    } else if constexpr (WAKE == WAKE_EXTERNAL) {
        if (tid < W) sh_shift[tid] = (double)sd.vext[i0 + tid] * sd.kick;
    } else {
        if (tid < W) sh_shift[tid] = 0.0;
    }
    if (tid == 0) sh_s = (float)s;
    __syncthreads();
    if (tid < W) {
        const double sh = sh_shift[tid];
        const double fl = floor(sh);
        float l[K];
        lagrange_fma<K>((float)(sh - fl), l);
        for (int k = 0; k < K; ++k) sh_kw[tid][k] = l[k];
        for (int k = K; k < 4; ++k) sh_kw[tid][k] = 0.0f;
        sh_km[tid] = (int)fmax(fmin(fl, 1.0e6), -1.0e6);
    }
    if constexpr (ROT == 1) {
        // RF kick of column i pulls along p from p + dtheta*q_i: shift tk*(q_min/dq + i) rows
        if (tid < W) {
            const double sh = sd.tk * (sd.q_min / sd.dq + (double)(i0 + tid));
            const double fl = floor(sh);
            float l[K];
            lagrange_fma<K>((float)(sh - fl), l);
            for (int k = 0; k < K; ++k) sh_rw[tid][k] = l[k];
            for (int k = K; k < 4; ++k) sh_rw[tid][k] = 0.0f;
            sh_rm[tid] = (int)fl;
        }
    }
    for (int k = tid; k < W * 2 * kPad; k += kThreads) {
        const int c = k / (2 * kPad), r = k - c * (2 * kPad);
        const int off = c * LA + (r < kPad ? r : n + r);
        A[off] = 0.0f;
        B[off] = 0.0f;
    }
    const float sT = sh_s;       // read after the barrier below

    // ---- phase R: rotation, chunk by chunk.  The staged rows of chunk k+1 are
    // loaded into registers (up to kPF columns per wave) while chunk k is
    // computed; barriers wait on LDS only, so the loads stay in flight.
    const int SX = W + 2 * kH;
    float pv[kPF][2];
    auto load_chunk = [&](int j0) {
#pragma unroll
        for (int k = 0; k < kPF; ++k) {
            const int x = wv + kWaves * k;
            const int gi = i0 - kH + x;
            pv[k][0] = 0.0f;
            pv[k][1] = 0.0f;
            if (x < SX && gi >= 0 && gi < n) {
                const __amdgpu_buffer_rsrc_t r = column_rsrc(src + (size_t)gi * n, n);
                // the builtin returns the raw 32 bits: reinterpret, do not convert
                pv[k][0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (j0 - kH + lane) * 4, 0, 0));
                if (lane < kSY - 64)
                    pv[k][1] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (j0 - kH + 64 + lane) * 4, 0, 0));
            }
        }
    };
    load_chunk(0);
    for (int j0 = 0; j0 < n; j0 += kJ) {
        __syncthreads();
        // S[x][y] = psi(i0 - kH + x, j0 - kH + y), zero outside the grid
#pragma unroll
        for (int k = 0; k < kPF; ++k) {
            const int x = wv + kWaves * k;
            if (x < SX) {
                S[x * kSY + lane] = pv[k][0];
                if (lane < kSY - 64) S[x * kSY + 64 + lane] = pv[k][1];
            }
        }
        for (int x = wv + kWaves * kPF; x < SX; x += kWaves) {      // wide strips: the rest
            const int gi = i0 - kH + x;
            float v0 = 0.0f, v1 = 0.0f;
            if (gi >= 0 && gi < n) {
                const __amdgpu_buffer_rsrc_t r = column_rsrc(src + (size_t)gi * n, n);
                v0 = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (j0 - kH + lane) * 4, 0, 0));
                if (lane < kSY - 64)
                    v1 = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (j0 - kH + 64 + lane) * 4, 0, 0));
            }
            S[x * kSY + lane] = v0;
            if (lane < kSY - 64) S[x * kSY + 64 + lane] = v1;
        }
        __syncthreads();
        if (j0 + kJ < n) load_chunk(j0 + kJ);
        if constexpr (ROT == 0) {
            const int j = j0 + lane;
            if (j < n) {
                // source displacement (dx, dy) of column i0+wv, then +kWaves columns per step
                double dx = fma((double)(i0 + wv), sd.axi, sd.ax0) + (double)j * sd.bx;
                double dy = fma((double)(i0 + wv), sd.cyi, sd.cy0) + (double)j * sd.by;
                const double ddx = kWaves * sd.axi, ddy = kWaves * sd.cyi;
                // LDS index of the first tap: (c + kH + fx - o0) * kSY + lane + kH + fy - o0
                // u.pad holds (kH - o0) * (kSY + 1) from the host: a run-time value keeps the
                // tap offsets within the 8-bit dword offsets of ds_read2
                int cbase = wv * kSY + lane + u.pad;
                for (int c = wv; c < W; c += kWaves, dx += ddx, dy += ddy, cbase += kWaves * kSY) {
                    const double fx = floor(dx), fy = floor(dy);
                    float lx[K], ly[K];
                    lagrange_fma<K>((float)(dx - fx), lx);
                    lagrange_fma<K>((float)(dy - fy), ly);
                    const float *base = S + (cbase + (int)fma(fx, (double)kSY, fy));
                    float f[K][K];
#pragma unroll
                    for (int a = 0; a < K; ++a)
#pragma unroll
                        for (int b = 0; b < K; ++b) f[a][b] = base[a * kSY + b];
                    float v = 0.0f;
#pragma unroll
                    for (int a = 0; a < K; ++a) {
                        float r = ly[0] * f[a][0];
#pragma unroll
                        for (int b = 1; b < K; ++b) r = fmaf(ly[b], f[a][b], r);
                        v = fmaf(lx[a], r, v);
                    }
                    if constexpr (CLAMP) {
                        const float lo = fminf(fminf(f[o0][o0], f[o0][o0 + 1]), fminf(f[o0 + 1][o0], f[o0 + 1][o0 + 1]));
                        const float hi = fmaxf(fmaxf(f[o0][o0], f[o0][o0 + 1]), fmaxf(f[o0 + 1][o0], f[o0 + 1][o0 + 1]));
                        v = fminf(fmaxf(v, lo), hi);
                    }
                    A[c * LA + kPad + j] = v * sT;
                }
            }
        } else {
            // Manhattan drift: row y of the chunk (global j0 - kH + y) pulls along q from
            // q - dtheta*p_j, i.e. a shift of -tw*(p_min/dp + j) columns, the same for
            // every column; rows outside the grid stay zero (their staged rows are zero)
            for (int y = lane; y < kSY; y += 64) {
                const double sh = -sd.tw * (sd.pm + (double)(j0 - kH + y));
                const double fl = floor(sh);
                float l[K];
                lagrange_fma<K>((float)(sh - fl), l);
                const int xo = kH + (int)fl - o0;
                for (int c = wv; c < W; c += kWaves) {
                    const float *col = S + (c + xo) * kSY + y;
                    float f[K];
#pragma unroll
                    for (int k = 0; k < K; ++k) f[k] = col[k * kSY];
                    float v = l[0] * f[0];
#pragma unroll
                    for (int k = 1; k < K; ++k) v = fmaf(l[k], f[k], v);
                    if constexpr (CLAMP) v = fminf(fmaxf(v, fminf(f[o0], f[o0 + 1])), fmaxf(f[o0], f[o0 + 1]));
                    Dm[c * kSY + y] = v;
                }
            }
            __syncthreads();
            // RF kick: column c pulls along p by its own shift sh_rm + fraction
            const int j = j0 + lane;
            if (j < n) {
                for (int c = wv; c < W; c += kWaves) {
                    const float *col = Dm + c * kSY + lane + kH + sh_rm[c] - o0;
                    float f[K];
#pragma unroll
                    for (int k = 0; k < K; ++k) f[k] = col[k];
                    float v = sh_rw[c][0] * f[0];
#pragma unroll
                    for (int k = 1; k < K; ++k) v = fmaf(sh_rw[c][k], f[k], v);
                    if constexpr (CLAMP) v = fminf(fmaxf(v, fminf(f[o0], f[o0 + 1])), fmaxf(f[o0], f[o0 + 1]));
                    A[c * LA + kPad + j] = v * sT;
                }
            }
        }
    }
    __syncthreads();

    // ---- phase K: kick along p, A -> B, 4 rows per lane.  The zero pads cover
    // every stencil read when km - o0 in [-kPad, kPad - K - 2]; larger shifts
    // take the bounds-checked path.
    for (int c = wv; c < W; c += kWaves) {
        const int km = sh_km[c];
        float w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = sh_kw[c][k];
        const float *acol = A + c * LA + kPad;
        float *bcol = B + c * LA + kPad;
        const bool fast = km - o0 >= -kPad && km - o0 + K + 2 <= kPad;
        for (int j = 4 * lane; j < n; j += 256) {
            float f[K + 3];
            if (fast) {
                const float *a = acol + j + km - o0;
#pragma unroll
                for (int k = 0; k < K + 3; ++k) f[k] = a[k];
            } else {
#pragma unroll
                for (int k = 0; k < K + 3; ++k) {
                    const int jj = j + km - o0 + k;
                    f[k] = (jj >= 0 && jj < n) ? acol[jj] : 0.0f;
                }
            }
            float o[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float v = w[0] * f[r];
#pragma unroll
                for (int k = 1; k < K; ++k) v = fmaf(w[k], f[r + k], v);
                if constexpr (CLAMP) {
                    const float p0 = f[r + o0], p1 = f[r + o0 + 1];
                    v = fminf(fmaxf(v, fminf(p0, p1)), fmaxf(p0, p1));
                }
                o[r] = v;
            }
            *(float4 *)(bcol + j) = make_float4(o[0], o[1], o[2], o[3]);
        }
    }
    __syncthreads();

    // ---- phase F: damping/diffusion, 4 rows per lane, FP64 column sums.
    // With g = p*psi, p_{j+o} = dp (u + o), u = p_min/dp + j:
    //   psi + bt[(-2g_{-1} - 3g_0 + 6g_1 - g_2)/(6dp) + (f_{-1} - 2f_0 + f_1)/dp^2]
    //   = f_0 + E + (k1 u) D,  D = -2f_{-1} - 3f_0 + 6f_1 - f_2,
    //   E = (2k1 + k2) f_{-1} - 2k2 f_0 + (6k1 + k2) f_1 - 2k1 f_2,
    // k1 = bt/6, k2 = bt/dp^2.
    const float k1 = (float)(sd.bt / 6.0), k2 = (float)(sd.bt / (sd.dp * sd.dp));
    const float cm = 2.0f * k1 + k2, c0 = -2.0f * k2, c1 = 6.0f * k1 + k2, c2 = -2.0f * k1;
    for (int c = wv; c < W; c += kWaves) {
        const float *bcol = B + c * LA + kPad;
        float *orow = dst + (size_t)(i0 + c) * n;
        double csum = 0.0;
        for (int j = 4 * lane; j < n; j += 256) {
            const float4 mid = *(const float4 *)(bcol + j);
            const float2 up = *(const float2 *)(bcol + j + 4);
            const float f[7] = {bcol[j - 1], mid.x, mid.y, mid.z, mid.w, up.x, up.y};
            float ku = k1 * (float)(sd.pm + (double)j);
            float o[4];
#pragma unroll
            for (int r = 0; r < 4; ++r, ku += k1) {
                const float D = fmaf(-2.0f, f[r], fmaf(-3.0f, f[r + 1], fmaf(6.0f, f[r + 2], -f[r + 3])));
                const float E = fmaf(cm, f[r], fmaf(c0, f[r + 1], fmaf(c1, f[r + 2], c2 * f[r + 3])));
                o[r] = fmaf(ku, D, f[r + 1] + E);
            }
            *(float4 *)(orow + j) = make_float4(o[0], o[1], o[2], o[3]);
            csum += (double)((o[0] + o[1]) + (o[2] + o[3]));
        }
        csum = wave_sum(csum);
        if (lane == 0) cs_next[i0 + c] = csum;
    }
}

}  // namespace vfp
