// vfp_step32c.hpp -- the FP32 fused step, staged through LDS (included by
// vfp.hip after vfp_kernels.hpp), and the fused tick of the FP32-storage
// forms.
//
// One workgroup owns a strip of W whole q-columns of one simulation and
// computes the whole split step for them (rotation, kick, damping/diffusion,
// FP64 column sums), arranged so that every cell costs as few vector ALU
// instructions as possible:
//   * staging: each wave owns whole staged columns; a lane moves four rows
//     with one 16-byte buffer load and one 16-byte LDS store.  The loads of
//     the next chunk are issued before the rotation of the current one and
//     consumed after it (register prefetch, kPF4 columns per wave).
//   * rotation: the source displacement is evaluated in FP32 from per-column
//     constants, dx = j*bx + (ax0 + i*axi); floor and fraction take one
//     instruction each.  A wave owns a 64-row block of the chunk and walks
//     the strip's columns; the K*K taps stay in registers as a window that
//     slides one stencil column per output column, so a cell reads K taps
//     from LDS unless its stencil base moved.  The rotated values are stored
//     unscaled.
//   * kick + damping/diffusion: a wave owns a block of 256 rows (four per
//     lane) and walks over the columns, so the four stencil coefficients of
//     each row (with the renormalisation factor s and the zero rows outside
//     the grid folded in) are formed once per block instead of per cell.
// Chunks are CH = 256 rows for every grid size (whole chunks on the
// power-of-two grids; 192 with the Manhattan rotation); a staged column holds
// rows j0-4 .. j0+CH+3, so every 16-byte load is aligned (n % 4 == 0), and
// its fixed length keeps all tap offsets compile-time immediates.  Its 66
// quads (CH = 256) are one per lane plus eight rows that travel one per lane
// in a shared prefetch register.
// LDS: A[W][n + 2*kPad], S[W + hl + hr][CH + 8] and, for the Manhattan
// rotation, Dm[W][CH + 8].
#pragma once

namespace vfp {

constexpr int kPad = 8;            // zero rows above and below each rotated column in LDS
constexpr int kH = 3;              // largest rotation halo in cells (per side)

// Raw buffer over one column of n floats: reads outside [0, n) return 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t column_rsrc(const float *col, int n)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)col, (short)0, n * 4, 0x00020000);
}

// Cubic (K=4, offsets -1..2) and quadratic (K=3, offsets -1..1) Lagrange
// weights (Sec. III.A), rearranged for fused multiply-adds.
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

// rows per chunk (a multiple of 64): 256 for the standard rotation, 192 for
// the Manhattan rotation, whose drifted rows take a third buffer of the
// chunk's length; a staged column holds rows j0-4 .. j0+CH+3
__host__ __device__ constexpr int chunk_rows_c(int rot) { return rot == 1 ? 192 : 256; }
__host__ __device__ constexpr int staged_rows_c(int rot) { return chunk_rows_c(rot) + 8; }
constexpr int kPF4 = 4;           // staged columns per wave held in registers across a chunk
// polls of a bounded wait for other workgroups of the same launch (about a second)
constexpr unsigned kWakeSpinLimit = 1u << 20;
constexpr int kMaxStripC = 64;    // columns per work unit in this layout

__device__ __forceinline__ int cvt_floor(float x)
{
    int m;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(m) : "v"(x));
    return m;
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// a * b + c for a, b within 24-bit signed range (one full-rate instruction)
__device__ __forceinline__ int mad_i24(int a, int b, int c)
{
    int r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
    return r;
}

// The value of v in the lane that DPP control CTRL selects (every lane
// active; FP64 moved as two 32-bit halves)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// LDS byte address of a pointer into the workgroup's shared memory
__device__ __forceinline__ unsigned lds_addr(const void *p)
{
    return (unsigned)(uintptr_t)(const __attribute__((address_space(3))) void *)p;
}

// An LDS byte address as a pointer into the workgroup's shared memory
typedef __attribute__((address_space(3))) const float lds_f32;
__device__ __forceinline__ lds_f32 *lds_ptr(unsigned addr)
{
    return (lds_f32 *)(uintptr_t)addr;
}

// Tensor Lagrange value of one cell from its K x K taps (clamped to the four
// nearest nodes when CLAMP).
template <int K, bool CLAMP>
__device__ __forceinline__ float interp_taps(const float (&f)[K][K], const float (&lx)[K], const float (&ly)[K])
{
    constexpr int o0 = (K - 1) / 2;
    float v;
#pragma unroll
    for (int a = 0; a < K; ++a) {
        float r = ly[0] * f[a][0];
#pragma unroll
        for (int b = 1; b < K; ++b) r = fmaf(ly[b], f[a][b], r);
        v = a == 0 ? lx[0] * r : fmaf(lx[a], r, v);
    }
    if constexpr (CLAMP) {
        const float lo = fminf(fminf(f[o0][o0], f[o0][o0 + 1]), fminf(f[o0 + 1][o0], f[o0 + 1][o0 + 1]));
        const float hi = fmaxf(fmaxf(f[o0][o0], f[o0][o0 + 1]), fmaxf(f[o0 + 1][o0], f[o0 + 1][o0 + 1]));
        v = fminf(fmaxf(v, lo), hi);
    }
    return v;
}

// Kick and damping/diffusion of four consecutive rows j .. j+3 of one column.
// a points at A row j + st - SH (16-byte aligned), where st = km - o0 - 1 is
// the first row the kick reads and SH = st mod 4, so the K+6 values needed
// are read as aligned 16-byte words (conflict-free for lanes four rows apart).
template <int K, bool CLAMP, int SH>
__device__ __forceinline__ void kick_damp4(const float *a, const float (&w)[4], const float (&C)[4][4], float (&o)[4])
{
    constexpr int o0 = (K - 1) / 2;
    constexpr int NQ = (SH + K + 6 + 3) / 4;
    float buf[4 * NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const float4 v = *(const float4 *)(a + 4 * q);
        buf[4 * q] = v.x; buf[4 * q + 1] = v.y; buf[4 * q + 2] = v.z; buf[4 * q + 3] = v.w;
    }
    float g[7];                                     // kicked rows j-1 .. j+5
#pragma unroll
    for (int r = 0; r < 7; ++r) {
        float v = w[0] * buf[SH + r];
#pragma unroll
        for (int k = 1; k < K; ++k) v = fmaf(w[k], buf[SH + r + k], v);
        if constexpr (CLAMP) {
            const float p0 = buf[SH + r + o0], p1 = buf[SH + r + o0 + 1];
            v = fminf(fmaxf(v, fminf(p0, p1)), fmaxf(p0, p1));
        }
        g[r] = v;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        o[r] = fmaf(C[r][3], g[r + 3], fmaf(C[r][2], g[r + 2], fmaf(C[r][1], g[r + 1], C[r][0] * g[r])));
}

// One work unit (a strip of whole columns of one simulation): reads buffer
// `parity`, writes the next state and its FP64 column sums to parity ^ 1.
// With MOM it also writes the per-column moments sum psi, sum p psi and
// sum p^2 psi of the new state (FP64, sd.mom), which a record row would
// otherwise read the whole state again for.
// With WAITW (the one-launch tick) the wake of the state is made in the same
// launch: the unit rotates first, then waits until the simulation's nt wake
// tiles have counted themselves in *rdy (a bounded wait; *flag reports one
// that ran out), and only then reads V and s and forms its kick weights.
template <int K, int WAKE, bool CLAMP, int ROT, bool COH = false, bool MOM = false, bool WAITW = false>
__device__ __forceinline__ void step32c_unit(const SimDev &sd, const Unit &u, int parity,
                                             const unsigned *rdy = nullptr, int nt = 0, int *flag = nullptr)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double red[kThreads];
    __shared__ __align__(16) float sh_kw[kMaxStripC][4];
    __shared__ int sh_km[kMaxStripC];
    __shared__ float sh_rw[kMaxStripC][4];
    __shared__ int sh_rm[kMaxStripC];
    __shared__ float2 sh_xy[kMaxStripC + 3];   // per column: ax0 + i*axi, cy0 + i*cyi (read in groups of K)
    constexpr int o0 = (K - 1) / 2;

    const int n = u.n, W = u.w, i0 = u.i0, tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int LA = n + 2 * kPad;
    constexpr int CH = chunk_rows_c(ROT), SY = staged_rows_c(ROT), Q4 = SY / 4;
    const int hl = u.hl, SX = W + hl + u.hr;
    float *A = (float *)smem_raw;
    float *S = A + (size_t)W * LA;
    float *Dm = S + (size_t)SX * SY;
    const float *__restrict__ src = (const float *)(parity ? u.psi[1] : u.psi[0]);
    // global address space for the stores, so they are global (not flat) stores
    typedef __attribute__((address_space(1))) float gfloat;
    gfloat *__restrict__ dst = (gfloat *)(parity ? u.psi[0] : u.psi[1]);
    const double *__restrict__ cs = sd.colsum[parity];
    double *__restrict__ cs_next = sd.colsum[parity ^ 1];

    // ---- staging of CH-row chunks
    // staged column x is source column i0 - hl + x; its LDS row y is row j0 - 4 + y;
    // lane l moves rows j0 - 4 + 4l .. +3 (lanes l < Q4).  A staged column of
    // more than 64 quads (CH > 248) has DX = 4 (Q4 - 64) rows beyond the
    // lanes' quads (rows j0 + 252 ..); those of prefetched column k are one
    // row per lane in lanes DX k .. DX k + DX-1 of a single register.
    constexpr int DX = Q4 > 64 ? 4 * (Q4 - 64) : 0;
    static_assert(DX * kPF4 <= 64, "the extra rows of every prefetched column fit one register");
    const int ncolw = (SX - wv + kWaves - 1) / kWaves;
    const bool lane_ld = lane < Q4;
    u32x4 pf[kPF4];
    unsigned pfx = 0;
    auto load_cols = [&](int j0, int cw0) {
        // rows above the grid (first chunk, lane 0) get an offset far past the
        // column instead of a negative one, so the 16-byte range check cannot wrap
        const int row = j0 - 4 + 4 * lane;
        const int voff = row >= 0 ? row * 4 : 0x40000000;
#pragma unroll
        for (int k = 0; k < kPF4; ++k) {
            const int x = wv + kWaves * (cw0 + k), gi = i0 - hl + x;
            if (cw0 + k < ncolw && lane_ld) {
                const bool ok = gi >= 0 && gi < n;
                const __amdgpu_buffer_rsrc_t r = column_rsrc(src + (size_t)(ok ? gi : 0) * n, ok ? n : 0);
                pf[k] = __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 0);
            }
            if constexpr (DX > 0) {
                if (cw0 + k < ncolw && lane / DX == k) {
                    const bool ok = gi >= 0 && gi < n;
                    const __amdgpu_buffer_rsrc_t r = column_rsrc(src + (size_t)(ok ? gi : 0) * n, ok ? n : 0);
                    pfx = __builtin_amdgcn_raw_buffer_load_b32(r, (j0 + 252 + lane % DX) * 4, 0, 0);
                }
            }
        }
    };
    auto store_cols = [&](int cw0) {
#pragma unroll
        for (int k = 0; k < kPF4; ++k) {
            const int x = wv + kWaves * (cw0 + k);
            if (cw0 + k < ncolw && lane_ld) *(u32x4 *)(S + x * SY + 4 * lane) = pf[k];
        }
        if constexpr (DX > 0) {
            const int k = lane / DX;
            if (k < kPF4 && cw0 + k < ncolw)
                *(unsigned *)(S + (wv + kWaves * (cw0 + k)) * SY + 256 + lane % DX) = pfx;
        }
    };
    // the first chunk's loads go out before the prologue, so that their
    // latency overlaps the prologue's loads and arithmetic
    load_cols(0, 0);

    // ---- prologue: renormalisation factor, wake slice, kick weights, pads
    double s = 1.0;
    if constexpr (WAITW) {
        static_assert(WAKE == WAKE_EXTERNAL, "the one-launch tick reads the wake of its own launch");
    } else if constexpr (WAKE == WAKE_EXTERNAL) {
        s = ((const __attribute__((address_space(1))) double *)sd.sext)[parity];   // a global (not flat) load
    } else {
        double part = 0.0;
        for (int k = tid; k < n; k += kThreads) part += cs[k];
        const double Qh = block_sum(part, red) * sd.dq * sd.dp;
        s = sd.renorm ? sd.Q0 / Qh : 1.0;
    }
    double shift = 0.0;                       // kick of column tid (tid < W), in rows
    if constexpr (WAKE == WAKE_FUSED) {
        const int parts = kThreads / W;
        const int c = tid / parts, pt = tid - c * parts;
        double acc = 0.0;
        if (c < W) {
            // FP32 partial sums over blocks of 32 of this thread's terms, added in FP64;
            // the unrolled block lets the loads of several terms be in flight together
            typedef const __attribute__((address_space(1))) float gfloat;
            typedef const __attribute__((address_space(1))) double gdouble;
            gfloat *wl = (gfloat *)sd.wl32 + (i0 + c) + n - 1;
            gdouble *gcs = (gdouble *)cs;
            const double dp = sd.dp;
            for (int jb = pt; jb < n; jb += 32 * parts) {
                float a32 = 0.0f;
                for (int q0 = 0; q0 < 32 && jb + q0 * parts < n; q0 += 8) {
#pragma unroll
                    for (int q = q0; q < q0 + 8; ++q) {
                        const int j = jb + q * parts, jj = j < n ? j : n - 1;   // loads stay in bounds
                        const float t = fmaf(wl[-jj], (float)(dp * gcs[jj]), a32);
                        a32 = j < n ? t : a32;
                    }
                }
                acc += a32;
            }
        }
        __syncthreads();
        red[tid] = acc;
        __syncthreads();
        if (tid < W) {
            double v = 0.0;
            for (int k = 0; k < parts; ++k) v += red[tid * parts + k];
            shift = sd.S * s * v * sd.kick;
            sd.vext[parity * n + i0 + tid] = (float)(sd.S * s * v);      // the wake this step used
        }
    }
    // the wake of an external-wake step: loaded here by every thread (no branch
    // around the load), used only once the strip is rotated, so that its
    // latency stays off the prologue
    float vcol = 0.0f;
    if constexpr (WAKE == WAKE_EXTERNAL && !WAITW)
        vcol = ((const __attribute__((address_space(1))) float *)sd.vext)[parity * n + i0 + min(tid, W - 1)];
    // kick weights of column tid from its shift in rows
    auto kick_weights = [&](double sh) {
        const double fl = floor(sh);
        float l[K];
        lagrange_fma<K>((float)(sh - fl), l);
        for (int k = 0; k < K; ++k) sh_kw[tid][k] = l[k];
        for (int k = K; k < 4; ++k) sh_kw[tid][k] = 0.0f;
        sh_km[tid] = (int)fmax(fmin(fl, 1.0e6), -1.0e6);
    };
    if (tid < W) {
        const double ic = (double)(i0 + tid);
        sh_xy[tid] = make_float2((float)fma(ic, sd.axi, sd.ax0), (float)fma(ic, sd.cyi, sd.cy0));
        if constexpr (WAKE != WAKE_EXTERNAL) kick_weights(shift);
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

    // ---- phase R: chunks of CH rows
    for (int j0 = 0; j0 < n; j0 += CH) {
        __syncthreads();
        store_cols(0);
        for (int cw0 = kPF4; cw0 < ncolw; cw0 += kPF4) {       // columns beyond the prefetch
            load_cols(j0, cw0);
            store_cols(cw0);
        }
        __syncthreads();
        if (j0 + CH < n) load_cols(j0 + CH, 0);
        if constexpr (ROT == 0) {
            const float bxf = sd.fbx, byf = sd.fby;
            static_assert(CH == 64 * kWaves, "one 64-row block of the chunk per wave");
            // wave wv owns rows rb = 64 wv .. rb + 63 of the chunk and walks the
            // strip's columns in order.  The K x K taps stay in registers as a
            // window that slides by one stencil column per output column (slot
            // (c + a) % K holds stencil column a of output column c), so a column
            // step reads only the K taps of the new stencil column unless the
            // lane's stencil base (mx, my) moved.
            const int rb = 64 * wv;
            const int j = j0 + rb + lane;
            if (j < n) {
                const float jf = (float)j;
                // LDS byte address of staged row rb + lane + 4 - o0 in staged column
                // hl - o0 + K - 1: the last stencil column of output column 0 when the
                // lane's stencil base is (0, 0)
                int rbase = (int)lds_addr(S + (hl - o0 + K - 1) * SY + rb + lane + 4 - o0);
                asm volatile("" : "+v"(rbase));      // kept whole, so the taps sit at offsets 0 .. K-1 of base
                float *acol = A + kPad + j;
                float fs[K][K];
                // window key: the lane's last-stencil-column address without the column
                // term; it changes exactly when the stencil base (mx, my) moves
                int pkey = INT_MIN;
                for (int c0 = 0; c0 < W; c0 += K) {
                    float2 xy[K];
#pragma unroll
                    for (int u = 0; u < K; ++u) xy[u] = sh_xy[c0 + u];
#pragma unroll
                    for (int u = 0; u < K; ++u) {
                        const int c = c0 + u;
                        if (c < W) {
                            const float dx = fmaf(jf, bxf, xy[u].x), dy = fmaf(jf, byf, xy[u].y);
                            const int mx = cvt_floor(dx), my = cvt_floor(dy);
                            // stencil column a of output column c is staged column c + mx + a + hl - o0
                            const int key = mad_i24(mx, 4 * SY, (my << 2) + rbase);
                            int cterm = c * (4 * SY);
                            asm volatile("" : "+s"(cterm));  // one scalar column term per column
                            const unsigned base = (unsigned)(key + cterm);
                            if (key != pkey) {
#pragma unroll
                                for (int a = 0; a < K - 1; ++a) {
                                    const lds_f32 *t = lds_ptr(base - 4 * (K - 1 - a) * SY);
#pragma unroll
                                    for (int b = 0; b < K; ++b) fs[(u + a) % K][b] = t[b];
                                }
                            }
                            {
                                const lds_f32 *t = lds_ptr(base);
#pragma unroll
                                for (int b = 0; b < K; ++b) fs[(u + K - 1) % K][b] = t[b];
                            }
                            pkey = key;
                            float lx[K], ly[K];
                            lagrange_fma<K>(__builtin_amdgcn_fractf(dx), lx);
                            lagrange_fma<K>(__builtin_amdgcn_fractf(dy), ly);
                            float f[K][K];
#pragma unroll
                            for (int a = 0; a < K; ++a)
#pragma unroll
                                for (int b = 0; b < K; ++b) f[a][b] = fs[(u + a) % K][b];
                            acol[c * LA] = interp_taps<K, CLAMP>(f, lx, ly);
                        }
                    }
                }
            }
        } else {
            // drift along q, one shift per staged row (row j0 - 4 + y), rows split over the waves
            for (int y = tid; y < SY; y += kThreads) {
                const float sh = fmaf((float)(j0 - 4 + y), sd.fd1, sd.fd0);
                const int fl = cvt_floor(sh);
                float l[K];
                lagrange_fma<K>(__builtin_amdgcn_fractf(sh), l);
                // the shift is the row's, so the K taps slide by one staged column per
                // output column: slot (c + k) % K holds tap k of output column c
                const float *col = S + (hl + fl - o0) * SY + y;
                float fw[K];
#pragma unroll
                for (int k = 0; k < K - 1; ++k) fw[k] = col[k * SY];
                for (int c0 = 0; c0 < W; c0 += K) {
#pragma unroll
                    for (int u = 0; u < K; ++u) {
                        const int c = c0 + u;
                        if (c < W) {
                            fw[(u + K - 1) % K] = col[(c + K - 1) * SY];
                            float f[K];
#pragma unroll
                            for (int k = 0; k < K; ++k) f[k] = fw[(u + k) % K];
                            float v = l[0] * f[0];
#pragma unroll
                            for (int k = 1; k < K; ++k) v = fmaf(l[k], f[k], v);
                            if constexpr (CLAMP) v = fminf(fmaxf(v, fminf(f[o0], f[o0 + 1])), fmaxf(f[o0], f[o0 + 1]));
                            Dm[c * SY + y] = v;
                        }
                    }
                }
            }
            __syncthreads();
            // RF kick along p, one shift per column
            for (int c = wv; c < W; c += kWaves) {
                float rw[K];
#pragma unroll
                for (int k = 0; k < K; ++k) rw[k] = sh_rw[c][k];
                const float *col = Dm + c * SY + lane + 4 + sh_rm[c] - o0;
                float *acol = A + c * LA + kPad + j0 + lane;
#pragma unroll
                for (int rb = 0; rb < CH; rb += 64) {
                    if (j0 + rb >= n) break;
                    if (j0 + rb + lane < n) {
                        float f[K];
#pragma unroll
                        for (int k = 0; k < K; ++k) f[k] = col[rb + k];
                        float v = rw[0] * f[0];
#pragma unroll
                        for (int k = 1; k < K; ++k) v = fmaf(rw[k], f[k], v);
                        if constexpr (CLAMP) v = fminf(fmaxf(v, fminf(f[o0], f[o0 + 1])), fmaxf(f[o0], f[o0 + 1]));
                        acol[rb] = v;
                    }
                }
            }
        }
    }
    if constexpr (WAKE == WAKE_EXTERNAL && !WAITW) {
        if (tid < W) kick_weights((double)vcol * sd.kick);
    }
    __syncthreads();
    if constexpr (WAITW) {
        if (tid == 0 && __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
            unsigned spins = 0;
            while (__hip_atomic_load(rdy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)nt) {
                if (++spins == kWakeSpinLimit) {
                    __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __syncthreads();
        s = __hip_atomic_load(sd.sext + parity, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (tid < W)
            kick_weights((double)__hip_atomic_load(sd.vext + parity * n + i0 + tid, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT) * sd.kick);
        __syncthreads();
    }

    // ---- kick and damping/diffusion.  Output row j uses the kicked values of
    // rows j-1 .. j+2 with coefficients s*(e_k + ku_j*d_k), ku_j = k1*p_j/dp,
    // d = (-2, -3, 6, -1); a lane's four rows need the kicked rows j-1 .. j+5,
    // which read A rows j-1+km-o0 .. j+5+km-o0+K-1.
    const int nb = (n + 255) >> 8;                 // 256-row blocks
    int b0 = nb, bst = kWaves, c0 = 0, cst = 1;
    if (nb >= kWaves) {
        b0 = wv;
    } else {
        const int g = kWaves / nb;
        if (wv < nb * g) { b0 = wv % nb; bst = nb; c0 = wv / nb; cst = g; }
    }
    const float sf = (float)s;
    const float sk1 = sf * sd.fk1;
    const float se0 = sf * sd.fe[0], se1 = sf * sd.fe[1], se2 = sf * sd.fe[2], se3 = sf * sd.fe[3];
    float *Sp = S;     // per-lane partial sums of the outputs, [W][nb][64] (fits: host bound)
    double *Mp = (double *)(Sp + (size_t)W * nb * 64);   // MOM: per (column, block) moments, [W][nb][3]
    for (int b = b0; b < nb; b += bst) {
        const int j = 256 * b + 4 * lane;
        const bool act = j < n;
        float C[4][4];
        {
            const float ku0 = sk1 * (float)(sd.pm + (double)j);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float ku = fmaf(sk1, (float)r, ku0);
                C[r][0] = fmaf(-2.0f, ku, se0);
                C[r][1] = fmaf(-3.0f, ku, se1);
                C[r][2] = fmaf(6.0f, ku, se2);
                C[r][3] = se3 - ku;
            }
            if (j == 0) C[0][0] = 0.0f;                          // row -1 is outside the grid
            if (j + 4 == n) { C[2][3] = 0.0f; C[3][2] = 0.0f; C[3][3] = 0.0f; }   // rows n, n+1
        }
        for (int c = c0; c < W; c += cst) {
            float part = 0.0f;
            double m0 = 0.0, m1 = 0.0, m2 = 0.0;
            if (act) {
                const int km = sh_km[c];
                const float4 w4 = *(const float4 *)sh_kw[c];
                const float w[4] = {w4.x, w4.y, w4.z, w4.w};
                const float *acol = A + c * LA + kPad;
                const int st = km - o0 - 1;                     // first A row read, relative to j
                const int sh = st & 3, q0 = st - sh;            // aligned start (q0 % 4 == 0)
                const int nq = (sh + K + 6 + 3) / 4;
                float o[4];
                if (q0 >= -kPad && q0 + 4 * nq <= kPad + 4) {
                    const float *a = acol + j + q0;
                    switch (sh) {
                    case 0: kick_damp4<K, CLAMP, 0>(a, w, C, o); break;
                    case 1: kick_damp4<K, CLAMP, 1>(a, w, C, o); break;
                    case 2: kick_damp4<K, CLAMP, 2>(a, w, C, o); break;
                    default: kick_damp4<K, CLAMP, 3>(a, w, C, o); break;
                    }
                } else {                                        // kick beyond the zero pads
                    float f[K + 6];
#pragma unroll
                    for (int k = 0; k < K + 6; ++k) {
                        const int jj = j + st + k;
                        f[k] = (jj >= 0 && jj < n) ? acol[jj] : 0.0f;
                    }
                    float g[7];
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
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        o[r] = fmaf(C[r][3], g[r + 3], fmaf(C[r][2], g[r + 2], fmaf(C[r][1], g[r + 1], C[r][0] * g[r])));
                }
                typedef float f32x4 __attribute__((ext_vector_type(4)));
                *(__attribute__((address_space(1))) f32x4 *)(dst + (size_t)(i0 + c) * n + j) =
                    f32x4{o[0], o[1], o[2], o[3]};
                part = (o[0] + o[1]) + (o[2] + o[3]);
                if constexpr (MOM) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const double v = (double)o[r], pj = fma((double)(j + r), sd.dp, sd.p_min);
                        m0 += v;
                        m1 = fma(pj, v, m1);
                        m2 = fma(pj * pj, v, m2);
                    }
                }
            }
            Sp[(c * nb + b) * 64 + lane] = part;              // the staging buffer is free now
            if constexpr (MOM) {
                m0 = wave_sum(m0);
                m1 = wave_sum(m1);
                m2 = wave_sum(m2);
                if (lane == 0) {
                    Mp[(c * nb + b) * 3] = m0;
                    Mp[(c * nb + b) * 3 + 1] = m1;
                    Mp[(c * nb + b) * 3 + 2] = m2;
                }
            }
        }
    }
    __syncthreads();
    // FP64 column sums: g = 2^lg threads per column, each adding every g-th
    // partial of its column in order (loads issued four at a time), then a
    // reduction over the g lanes in a fixed order: lanes 1 and 2 apart, the
    // other quad of the half-row and the other half of the row by DPP moves,
    // the other rows by lane permutes
    {
        const int lg = W <= 4 ? 6 : W <= 8 ? 5 : W <= 16 ? 4 : W <= 32 ? 3 : 2;
        const int g = 1 << lg, c = tid >> lg, sub = tid & (g - 1), cnt = nb * 64;
        double t = 0.0;
        if (c < W) {
            const float *pp = Sp + c * cnt;
            for (int k = sub; k < cnt; k += 4 * g) {
                float a[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) a[q] = pp[min(k + q * g, cnt - 1)];   // in bounds, no branch
#pragma unroll
                for (int q = 0; q < 4; ++q) t += k + q * g < cnt ? (double)a[q] : 0.0;
            }
        }
        t += dpp_f64<0xB1>(t);                      // quad_perm 1,0,3,2
        t += dpp_f64<0x4E>(t);                      // quad_perm 2,3,0,1
        if (g >= 8) t += dpp_f64<0x141>(t);         // row_half_mirror
        if (g >= 16) t += dpp_f64<0x140>(t);        // row_mirror
        if (g >= 32) t += __shfl_xor(t, 16, 64);
        if (g >= 64) t += __shfl_xor(t, 32, 64);
        if (c < W && sub == 0) store_cs<COH>(cs_next + i0 + c, t);
    }
    if constexpr (MOM) {
        // the column's blocks added in block order
        if (tid < 3 * W) {
            const int c = tid / 3, k = tid - 3 * c;
            double t = 0.0;
            for (int b = 0; b < nb; ++b) t += Mp[(c * nb + b) * 3 + k];
            sd.mom[3 * (i0 + c) + k] = t;
        }
    }
}

template <int K, int WAKE, bool CLAMP, int ROT, bool MOM = false>
__global__ __launch_bounds__(kThreads) void step32c_kernel(const SimDev *__restrict__ sims,
                                                           const Unit *__restrict__ units, int nunits,
                                                           int parity)
{
    const Unit u = units[blockIdx.x];
    // every field of the unit in one round trip, ahead of the padding test
    asm volatile("" ::"s"(u.sim), "s"(u.n), "s"(u.hl), "s"(u.hr), "s"(u.psi[0]), "s"(u.psi[1]), "s"(parity));
    if (u.w == 0) return;                     // padding slot
    step32c_unit<K, WAKE, CLAMP, ROT, false, MOM>(sims[u.sim], u, parity);
}

// Wake kinds of the fused tick: FP32 vector ALU, FP16 or BF16 hi/lo matrix cores.
enum TickWake { TW_VEC = 0, TW_FP16 = 1, TW_BF16 = 2 };

// One tick of a batch in one launch.  The grid walks one list of items: the
// wake tiles of every simulation first (w < 0, tile index in i0), then the
// work units (w > 0, nu = the simulation's wake tile count), with empty
// slots (w == 0) between the two parts (with MOM, on a tick followed by a
// record row, the units also leave the new state's per-column moments, as
// the split tick's step does).  A wake tile computes its part of
// the wake V_t and the factor s_t of the current state from its column sums
// (made by the previous launch; Sec. II.B, Eq. "wakepotential"), stores them
// through to the coherent level, waits for the stores and counts itself in
// ready[parity][sim]; tile 0 also clears the previous launch's counter
// ready[parity^1][sim] for the launch after this one.  A unit stages and
// rotates its strip, which needs no wake, and only then waits for its
// simulation's tiles and kicks.  Tiles wait for nothing and come first in
// the list, so every wait ends once they have run; a wait longer than
// kWakeSpinLimit polls (about a second, far beyond any tick) sets *flag
// instead, reported by the host as a device error, and once it is set no unit
// waits any more, so every launch finishes.
template <int K, bool CLAMP, int ROT, int WK, bool MOM = false>
__global__ __launch_bounds__(kThreads) void tick32_kernel(const SimDev *__restrict__ sims,
                                                          const Unit *__restrict__ items, int nitems, int parity,
                                                          unsigned *__restrict__ ready, int count,
                                                          int *__restrict__ flag)
{
    const Unit u = items[blockIdx.x];
    // every field of the item in one round trip, ahead of the tests
    asm volatile("" ::"s"(u.sim), "s"(u.n), "s"(u.hl), "s"(u.hr), "s"(u.psi[0]), "s"(u.psi[1]), "s"(parity));
    if (u.w == 0) return;                     // empty slot
    const SimDev &sd = sims[u.sim];
    if (u.w > 0) {
        step32c_unit<K, WAKE_EXTERNAL, CLAMP, ROT, false, MOM, true>(sd, u, parity, ready + parity * count + u.sim,
                                                                    u.nu, flag);
        return;
    }
    if (u.i0 == 0 && threadIdx.x == 0)
        __hip_atomic_store(ready + (parity ^ 1) * count + u.sim, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if constexpr (WK == TW_VEC) wake_vec_tile<false, true>(sd, u.i0, parity);
    else wake_mfma_tile<WK == TW_FP16, false, true>(sd, u.i0, parity);
    wait_stores();                            // this wave's V and s have reached the coherent level
    __syncthreads();
    if (threadIdx.x == 0)
        (void)__hip_atomic_fetch_add(ready + parity * count + u.sim, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace vfp
