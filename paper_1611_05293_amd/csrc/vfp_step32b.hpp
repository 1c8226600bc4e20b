// vfp_step32b.hpp -- second layout of the FP32 staged step (included by
// vfp.hip after vfp_step32.hpp; chosen with the tuning switch).
//
// Differences from step32_kernel: the rotation works on chunks of CH = 256
// rows (or the grid rounded up to 64) split into 64-row blocks per column,
// so every wave has several cells per chunk; the previous density of the
// next chunk is prefetched into at most kPFB registers per lane; and the
// kick and the damping stencil are merged (each lane interpolates the seven
// kicked values its four output rows need), which removes the second LDS
// column buffer.  LDS: A[W][n + 2*kPad], S[W + 2*kH][CH + 2*kH] and, for the
// Manhattan rotation, Dm[W][CH + 2*kH].
#pragma once

namespace vfp {

constexpr int kPFB = 32;           // prefetch registers per lane

__device__ __forceinline__ int chunk_rows(int n) { return n >= 256 ? 256 : ((n + 63) / 64) * 64; }

template <int K, int WAKE, bool CLAMP, int ROT>
__global__ __launch_bounds__(kThreads) void step32b_kernel(const SimDev *__restrict__ sims,
                                                           const Unit *__restrict__ units, int nunits,
                                                           int parity)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[kThreads];
    __shared__ float sh_kw[kMaxStrip][4];
    __shared__ int sh_km[kMaxStrip];
    __shared__ double sh_shift[kMaxStrip];
    __shared__ float sh_rw[kMaxStrip][4];
    __shared__ int sh_rm[kMaxStrip];
    __shared__ float sh_s;
    constexpr int o0 = (K - 1) / 2;

    const Unit u = units[blockIdx.x];
    if (u.w == 0) return;                     // padding slot
    const SimDev &sd = sims[u.sim];
    const int n = sd.n, W = u.w, i0 = u.i0, tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int LA = n + 2 * kPad;
    const int CH = chunk_rows(n), SY = CH + 2 * kH, SX = W + 2 * kH;
    float *A = (float *)smem_raw;
    float *S = A + (size_t)W * LA;
    float *Dm = S + (size_t)SX * SY;
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
        A[c * LA + (r < kPad ? r : n + r)] = 0.0f;
    }
    const float sT = sh_s;

    // ---- phase R: chunks of CH rows; staged rows of the next chunk prefetched
    const int nseg = (SY + 63) / 64;            // 64-row segments of a staged column
    const int ncolw = (SX - wv + kWaves - 1) / kWaves;  // staged columns of this wave
    float pv[kPFB];
    auto load_chunk = [&](int j0) {
#pragma unroll
        for (int k = 0; k < kPFB; ++k) {
            const int cw = k / 5, sg = k - 5 * cw;          // at most 5 segments per column
            const int x = wv + kWaves * cw, y = 64 * sg + lane;
            const int gi = i0 - kH + x;
            pv[k] = 0.0f;
            if (cw < ncolw && sg < nseg && y < SY && gi >= 0 && gi < n) {
                const __amdgpu_buffer_rsrc_t r = column_rsrc(src + (size_t)gi * n, n);
                pv[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (j0 - kH + y) * 4, 0, 0));
            }
        }
    };
    load_chunk(0);
    for (int j0 = 0; j0 < n; j0 += CH) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPFB; ++k) {
            const int cw = k / 5, sg = k - 5 * cw;
            const int x = wv + kWaves * cw, y = 64 * sg + lane;
            if (cw < ncolw && sg < nseg && y < SY) S[x * SY + y] = pv[k];
        }
        for (int cw = kPFB / 5; cw < ncolw; ++cw) {          // columns beyond the prefetch
            const int x = wv + kWaves * cw, gi = i0 - kH + x;
            for (int y = lane; y < SY; y += 64) {
                float v = 0.0f;
                if (gi >= 0 && gi < n) {
                    const __amdgpu_buffer_rsrc_t r = column_rsrc(src + (size_t)gi * n, n);
                    v = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (j0 - kH + y) * 4, 0, 0));
                }
                S[x * SY + y] = v;
            }
        }
        __syncthreads();
        if (j0 + CH < n) load_chunk(j0 + CH);
        if constexpr (ROT == 0) {
            for (int rb = 0; rb < CH; rb += 64) {
                const int j = j0 + rb + lane;
                if (j0 + rb >= n) break;
                if (j < n) {
                    double dx = fma((double)(i0 + wv), sd.axi, sd.ax0) + (double)j * sd.bx;
                    double dy = fma((double)(i0 + wv), sd.cyi, sd.cy0) + (double)j * sd.by;
                    const double ddx = kWaves * sd.axi, ddy = kWaves * sd.cyi;
                    // u.pad = (kH - o0) * (SY + 1) for this unit's grid (set by the host)
                    int cbase = wv * SY + rb + lane + u.pad;
                    for (int c = wv; c < W; c += kWaves, dx += ddx, dy += ddy, cbase += kWaves * SY) {
                        const double fx = floor(dx), fy = floor(dy);
                        float lx[K], ly[K];
                        lagrange_fma<K>((float)(dx - fx), lx);
                        lagrange_fma<K>((float)(dy - fy), ly);
                        const float *base = S + (cbase + (int)fma(fx, (double)SY, fy));
                        float f[K][K];
#pragma unroll
                        for (int a = 0; a < K; ++a)
#pragma unroll
                            for (int b = 0; b < K; ++b) f[a][b] = base[a * SY + b];
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
            }
        } else {
            // drift along q, one shift per row, for every staged row
            for (int y = lane; y < SY; y += 64) {
                const double sh = -sd.tw * (sd.pm + (double)(j0 - kH + y));
                const double fl = floor(sh);
                float l[K];
                lagrange_fma<K>((float)(sh - fl), l);
                const int xo = kH + (int)fl - o0;
                for (int c = wv; c < W; c += kWaves) {
                    const float *col = S + (c + xo) * SY + y;
                    float f[K];
#pragma unroll
                    for (int k = 0; k < K; ++k) f[k] = col[k * SY];
                    float v = l[0] * f[0];
#pragma unroll
                    for (int k = 1; k < K; ++k) v = fmaf(l[k], f[k], v);
                    if constexpr (CLAMP) v = fminf(fmaxf(v, fminf(f[o0], f[o0 + 1])), fmaxf(f[o0], f[o0 + 1]));
                    Dm[c * SY + y] = v;
                }
            }
            __syncthreads();
            // RF kick along p, one shift per column
            for (int rb = 0; rb < CH; rb += 64) {
                const int j = j0 + rb + lane;
                if (j0 + rb >= n) break;
                if (j < n) {
                    for (int c = wv; c < W; c += kWaves) {
                        const float *col = Dm + c * SY + rb + lane + kH + sh_rm[c] - o0;
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
    }
    __syncthreads();

    // ---- kick and damping merged: 4 output rows per lane need the kicked
    // values of rows j-1 .. j+5, i.e. A rows j-1+km-o0 .. j+5+km-o0+K-1
    const float k1 = (float)(sd.bt / 6.0), k2 = (float)(sd.bt / (sd.dp * sd.dp));
    const float cm = 2.0f * k1 + k2, c0 = -2.0f * k2, c1 = 6.0f * k1 + k2, c2 = -2.0f * k1;
    for (int c = wv; c < W; c += kWaves) {
        const int km = sh_km[c];
        float w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = sh_kw[c][k];
        const float *acol = A + c * LA + kPad;
        float *orow = dst + (size_t)(i0 + c) * n;
        // reads A rows j+km-o0-1 .. j+km-o0+K+4 for j in [0, n-4]: inside the zero pads when
        const bool fast = km - o0 - 1 >= -kPad && km - o0 + K <= kPad - 1;
        double csum = 0.0;
        for (int j = 4 * lane; j < n; j += 256) {
            float f[K + 6];
            if (fast) {
                const float *a = acol + j + km - o0 - 1;
#pragma unroll
                for (int k = 0; k < K + 6; ++k) f[k] = a[k];
            } else {
#pragma unroll
                for (int k = 0; k < K + 6; ++k) {
                    const int jj = j + km - o0 - 1 + k;
                    f[k] = (jj >= 0 && jj < n) ? acol[jj] : 0.0f;
                }
            }
            float g[7];                       // kicked values of rows j-1 .. j+5
#pragma unroll
            for (int r = 0; r < 7; ++r) {
                float v = w[0] * f[r];
#pragma unroll
                for (int k = 1; k < K; ++k) v = fmaf(w[k], f[r + k], v);
                if constexpr (CLAMP) {
                    const float p0 = f[r + o0], p1 = f[r + o0 + 1];
                    v = fminf(fmaxf(v, fminf(p0, p1)), fmaxf(p0, p1));
                }
                g[r] = v;
            }
            if (j == 0) g[0] = 0.0f;                 // rows outside the grid are zero
            if (j + 4 >= n) { g[5] = 0.0f; g[6] = 0.0f; }
            float ku = k1 * (float)(sd.pm + (double)j);
            float o[4];
#pragma unroll
            for (int r = 0; r < 4; ++r, ku += k1) {
                const float D = fmaf(-2.0f, g[r], fmaf(-3.0f, g[r + 1], fmaf(6.0f, g[r + 2], -g[r + 3])));
                const float E = fmaf(cm, g[r], fmaf(c0, g[r + 1], fmaf(c1, g[r + 2], c2 * g[r + 3])));
                o[r] = fmaf(ku, D, g[r + 1] + E);
            }
            *(float4 *)(orow + j) = make_float4(o[0], o[1], o[2], o[3]);
            csum += (double)((o[0] + o[1]) + (o[2] + o[3]));
        }
        csum = wave_sum(csum);
        if (lane == 0) cs_next[i0 + c] = csum;
    }
}

}  // namespace vfp
