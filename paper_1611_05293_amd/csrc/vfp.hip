// vfp.hip -- host engine and C ABI of libvfp.so (see include/vfp.h).
//
// A handle owns a set of simulations (one for the plain form).  Device
// memory is one arena (caller workspace or hipMalloc) carved per
// simulation; work is described by "units" (a simulation and a strip of
// whole q-columns) and one tick is one launch of the fused step kernel over
// all units of the active simulations (preceded, in the mixed modes, by the
// matrix-core wake).  Ticks are replayed from a captured hipGraph in the
// batched form.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "vfp.h"
#include "vfp_kernels.hpp"
#include "vfp_step32c.hpp"
#include "vfp_impedance.hpp"
#include "vfp_stepfix.hpp"

using namespace vfp;

// Device scratch of vfp_impedance_samples_noalloc: Re and Im of at most
// VFP_NOALLOC_MAX_SAMPLES impedance samples (256 KiB).
static __device__ __align__(256) double scratch[2 * VFP_NOALLOC_MAX_SAMPLES];

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(VFP_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

constexpr size_t kAlign = 256;

// Raise a kernel's dynamic-LDS limit when a launch needs more than before.
template <typename K>
void lds_limit(K kernel, size_t bytes, int &cur)
{
    if ((int)bytes > cur) {
        if (hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) ==
            hipSuccess)
            cur = (int)bytes;
    }
}
// one limit per kernel for every caller (the limit only ever grows)
void wakev_limit(size_t bytes)
{
    static int cur = 0;
    lds_limit(wakev_kernel, bytes, cur);
}
constexpr int kMaxGraphPhases = 8;   // retirement phases that get graphs
constexpr int kMaxGroups = 4;        // stream groups of a batch
constexpr int kXcds = 8;             // XCDs of the GPU: the dispatcher deals blocks to them round-robin
// tuning values of `staged`: the generic kernel, the LDS-staged kernel with a
// separate wake launch per tick, the LDS-staged kernel with the one-launch tick
constexpr int kStagedGeneric = 0, kStagedSplit = 1, kStagedFused = 2;
constexpr size_t kFusedTickCells = (size_t)2 << 20;   // largest batch (cells per tick) that defaults to the fused tick
constexpr int kTimingEvents = 3 * 1024;   // event pool of the kernel timing mode

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct HostSim {
    vfp_params p{};
    std::vector<double> zr, zi;
    int64_t steps = 0;       // steps since create / set_psi
    bool active = true;
    int frozen_buf = 0;      // buffer holding the state once retired
    // arena offsets
    size_t off_psi[2], off_cs[2], off_wl64, off_wl32, off_frag, off_vext, off_sext, off_rho,
        off_v, off_stat, off_zr, off_mom;
    int nb = 0;
    bool fast = false;       // eligible for the LDS-staged FP32 step kernel
    int halo = 2 * kH;       // staged columns beside a strip (left + right) in that kernel
};

int choose_strip(int n, int cells)
{
    int w = cells / n;
    w = std::max(1, std::min(w, std::min(n, kMaxStrip)));
    return w;
}

// Strip width of the chunked staged layout: at most kMaxStripC columns, the
// per-(column, 256-row block, lane) partial sums and the per-(column, block)
// FP64 moments of a record tick fit the staging buffer
// (W * nb * (64 + 6) <= (W + halo) * staged_rows_c floats), and every staged column
// of a wave travels in the prefetch registers (a fifth column per wave would be
// loaded and stored with its latency exposed: 128-row grids measured 8 % faster
// with 12-column strips than with 13).
// The dynamic LDS of a unit stays under kLdsBudgetC so that five workgroups
// fit on a compute unit.
#ifndef VFP_LDS_BUDGET
#define VFP_LDS_BUDGET (28 * 1024)
#endif
constexpr size_t kLdsBudgetC = VFP_LDS_BUDGET;
size_t lds_bytes_c(int n, int w, int rotation, int halo)
{
    const size_t sy = staged_rows_c(rotation);
    return ((size_t)w * (n + 2 * kPad) + (size_t)(w + halo) * sy + (rotation ? (size_t)w * sy : 0)) * 4;
}
int choose_strip_c(int n, int cells, int rotation, int halo)
{
    int w = std::max(1, std::min(cells / n, std::min(n, kMaxStripC)));
    const int nb = (n + 255) / 256;
    while (w > 1 && (size_t)w * nb * (64 + 6) > (size_t)(w + halo) * staged_rows_c(rotation)) --w;
    w = std::min(w, kWaves * kPF4 - halo);
    while (w > 1 && lds_bytes_c(n, w, rotation, halo) > kLdsBudgetC) --w;
    return std::max(w, 1);
}


// a density must be finite and, in the FP32-storage forms, representable in
// binary32, with a positive, finite charge (the moments are charge-weighted)
const char *density_error(const double *psi, size_t nn, int precision, int fix_bits)
{
    const double lim = precision == VFP_FP64    ? DBL_MAX
                       : precision == VFP_FIXED ? std::ldexp(1.0, 61 - fix_bits)
                                                : (double)FLT_MAX;
    double sum = 0.0;
    for (size_t z = 0; z < nn; ++z) {
        if (precision == VFP_FIXED && !(std::fabs(psi[z]) < lim)) return "psi must be finite with |psi| < 2^(61-fix_bits)";
        if (!(std::fabs(psi[z]) <= lim))
            return precision == VFP_FP64 ? "psi must be finite" : "psi must be finite and within the binary32 range";
        sum += psi[z];
    }
    if (!(sum > 0.0) || !std::isfinite(sum)) return "psi must have a positive, finite charge";
    return nullptr;
}

int validate(const vfp_params &p, std::string &why)
{
    if (p.n < 16 || p.n > 4096) { why = "n must be in [16, 4096]"; return VFP_EINVAL; }
    if (!(p.q_max > p.q_min) || !(p.p_max > p.p_min) || !std::isfinite(p.q_min) ||
        !std::isfinite(p.q_max) || !std::isfinite(p.p_min) || !std::isfinite(p.p_max)) {
        why = "need finite q_min < q_max and p_min < p_max";
        return VFP_EINVAL;
    }
    if (p.steps_per_period < 1) { why = "steps_per_period must be >= 1"; return VFP_EINVAL; }
    if (!(p.beta >= 0.0) || !std::isfinite(p.beta)) { why = "beta must be finite and >= 0"; return VFP_EINVAL; }
    if (p.interp != 3 && p.interp != 4) { why = "interp must be 3 or 4"; return VFP_EINVAL; }
    if (p.clamp != 0 && p.clamp != 1) { why = "clamp must be 0 or 1"; return VFP_EINVAL; }
    if (p.renormalize != 0 && p.renormalize != 1) { why = "renormalize must be 0 or 1"; return VFP_EINVAL; }
    if (p.precision < VFP_FP64 || p.precision > VFP_FIXED) { why = "unknown precision"; return VFP_EINVAL; }
    if (p.precision == VFP_FIXED && (p.fix_bits < 16 || p.fix_bits > 59)) { why = "fix_bits must be in [16, 59]"; return VFP_EINVAL; }
    if (p.padding < 2 || (int64_t)p.padding * p.n > (1 << 24)) { why = "padding must be >= 2"; return VFP_EINVAL; }
    if (p.rotation != VFP_ROT_STANDARD && p.rotation != VFP_ROT_MANHATTAN) { why = "unknown rotation"; return VFP_EINVAL; }
    if ((p.z_re == nullptr) != (p.z_im == nullptr)) { why = "z_re and z_im must both be set or both NULL"; return VFP_EINVAL; }
    if (p.z_model < VFP_Z_SAMPLES || p.z_model > VFP_Z_FREE_SPACE) { why = "unknown z_model"; return VFP_EINVAL; }
    if (p.z_model != VFP_Z_SAMPLES && p.z_re) { why = "z_re/z_im must be NULL when z_model computes Z"; return VFP_EINVAL; }
    if (p.z_model == VFP_Z_PARALLEL_PLATES && !(p.z_shield > 0.0 && std::isfinite(p.z_shield))) {
        why = "z_shield must be finite and > 0";
        return VFP_EINVAL;
    }
    if (!std::isfinite(p.z_scale)) { why = "z_scale must be finite"; return VFP_EINVAL; }
    if (p.max_steps < 0) { why = "max_steps must be >= 0"; return VFP_EINVAL; }
    const double dp = (p.p_max - p.p_min) / (p.n - 1);
    const double th = 2.0 * M_PI / p.steps_per_period;
    if (p.beta * th / (dp * dp) > 0.25) {
        why = "explicit damping/diffusion step unstable: beta*dtheta/dp^2 > 0.25";
        return VFP_EUNSTABLE;
    }
    if (p.z_re) {
        const int M = p.padding * p.n;
        for (int k = 0; k <= M / 2; ++k)
            if (!std::isfinite(p.z_re[k]) || !std::isfinite(p.z_im[k])) {
                why = "impedance samples must be finite";
                return VFP_EINVAL;
            }
    }
    if (p.psi0) {
        if (const char *e = density_error(p.psi0, (size_t)p.n * p.n, p.precision, p.fix_bits)) {
            why = std::string("psi0: ") + e;
            return VFP_EINVAL;
        }
    }
    return VFP_OK;
}

size_t elem_size(int precision) { return precision == VFP_FP64 || precision == VFP_FIXED ? 8 : 4; }
bool is_mixed(int precision) { return precision == VFP_MIXED_BF16 || precision == VFP_MIXED_FP16; }
// FP32 storage: the staged kernels and a separate wake kernel apply
bool is_fp32_storage(int precision) { return precision == VFP_FP32 || is_mixed(precision); }
// bytes of the per-column sums: FP64 sums, or {high, low} integer sums in fixed point
size_t cs_bytes(int precision, int n) { return (precision == VFP_FIXED ? 2 : 1) * (size_t)n * 8; }
// default cells per work unit: the 8-byte forms hold two copies of their strip
// in LDS (16 bytes per cell), so small strips leave room for several
// workgroups per CU (measured on the 200-simulation scan)
int default_cells(int precision)
{
    return precision == VFP_FP64 ? 1024 : precision == VFP_FIXED ? 2048 : 8192;
}

// arena layout for count simulations; fills offsets when hs != nullptr
size_t layout(const vfp_params *p, int count, std::vector<HostSim> *hs)
{
    size_t off = 0;
    for (int s = 0; s < count; ++s) {
        const vfp_params &q = p[s];
        const size_t n = q.n, es = elem_size(q.precision);
        const int nb = (q.n + 15) / 16;
        HostSim tmp;
        HostSim &h = hs ? (*hs)[s] : tmp;
        h.nb = nb;
        for (int b = 0; b < 2; ++b) { h.off_psi[b] = off; off = align_up(off + n * n * es); }
        for (int b = 0; b < 2; ++b) { h.off_cs[b] = off; off = align_up(off + cs_bytes(q.precision, q.n)); }
        h.off_wl64 = off; off = align_up(off + (2 * n - 1) * 8);
        h.off_wl32 = off; off = align_up(off + (2 * n - 1) * 4);
        h.off_frag = off;
        if (is_mixed(q.precision)) off = align_up(off + (size_t)4 * wake_rev_len(q.n) * sizeof(uint16_t));
        h.off_vext = off; off = align_up(off + 2 * n * 4);
        h.off_sext = off; off = align_up(off + 3 * 8);
        h.off_rho = off; off = align_up(off + n * 8);
        h.off_v = off; off = align_up(off + n * 8);
        h.off_stat = off; off = align_up(off + 8 * 8);
        h.off_mom = off; off = align_up(off + 3 * n * 8);
        h.off_zr = off; off = align_up(off + (size_t)(q.padding * q.n / 2 + 1) * 8);
    }
    return off;
}

}  // namespace

// One stream's share of a phase: its units (and wake tiles, and for the fused
// tick the interleaved item list) in the shared device arrays.
struct Group {
    size_t unit_off = 0, unit_cnt = 0, tile_off = 0, tile_cnt = 0, item_off = 0, item_cnt = 0;
    size_t act_off = 0, act_cnt = 0;                 // the group's simulations, into d_active
    hipGraph_t graph[2] = {nullptr, nullptr};        // G ticks of this group starting at parity 0 / 1
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
};

// Work of one retirement phase: the simulations active between two
// retirements (absolute ticks [start, end)), split in stream groups, each
// with graphs of G ticks starting at either parity (one stream per graph: a
// graph holds no dependency on another stream).  Built outside the step call
// (create and every call that changes the set, the state or the tuning), so
// that stepping only selects among them.
struct Phase {
    int64_t start = 0, end = INT64_MAX;
    std::vector<int> active;        // active simulations
    std::vector<int> retire;        // simulations whose budget ends at `end`
    int ngroups = 1;
    Group grp[kMaxGroups];
    bool fast = false;              // every active simulation takes the staged FP32 kernel
    bool wake = false;              // some active simulation has an impedance
    size_t lds_step = 0;            // dynamic LDS of the step launch (fused tick: with the wake)
    size_t lds_wake = 0;            // dynamic LDS of a separate wake launch
    bool graphs = false;            // every group has its graphs
};

struct vfp_batch {
    int count = 0;
    int precision = VFP_FP32, K = 4, clamp = 0, rotation = 0;
    bool plain = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<HostSim> hs;
    std::vector<SimDev> sd;
    SimDev *d_sd = nullptr;
    unsigned char *arena = nullptr;
    size_t arena_bytes = 0;
    bool own_arena = false;
    int cells = 0;                 // tuning: cells per work unit
    int staged = kStagedSplit;     // tuning: kernel and tick form (kStaged*)
    bool use_graph = true;         // tuning: replay ticks from hipGraphs
    int lanes = 3;                 // tuning: stream groups requested (1 .. kMaxGroups)
    // retirement phases; all phases' units, items, active lists and wake tiles on the device
    std::vector<Phase> phases;
    int cur = 0;                   // current phase
    int G = 16;                    // ticks per graph replay
    std::vector<Unit> units, items;
    std::vector<int> actv;
    std::vector<WakeTile> wtiles;
    Unit *d_units = nullptr, *d_items = nullptr;
    int *d_active = nullptr;
    WakeTile *d_wtiles = nullptr;
    size_t units_cap = 0, items_cap = 0, actv_cap = 0, wtiles_cap = 0;
    unsigned *d_done = nullptr;    // fused tick: [2][count] finished wake tiles per simulation and tick parity
    int *d_flag = nullptr;         // fused tick: set when a unit's wait for its wake exceeded its bound
    int *d_idx = nullptr;          // scratch index arrays for per-call kernels (2*count)
    int *d_buf01 = nullptr;        // count zeros then count ones: buffer tables for records
    int64_t tick = 0;              // ticks since create
    int parity = 0;                // buffer holding the state of active simulations
    // stream groups: group 0 runs on the batch's stream, groups 1.. on streams of
    // the library (default priority), forked from and joined into the batch's stream
    hipStream_t xstream[kMaxGroups - 1] = {};
    hipEvent_t ev_fork = nullptr, ev_join[kMaxGroups - 1] = {};
    bool forked = false;
    int forked_groups = 0;
    // record
    int every = 0;
    int64_t rec_cap = 0, rec_base = 0;
    double *d_ring = nullptr;
    int64_t *d_ring_rows = nullptr;
    // staging for psi transfers and impedance uploads
    double *d_stage = nullptr;
    size_t stage_elems = 0;
    size_t lds_stats = 0;
    // per-kernel event timing (direct launches in one group while enabled); the
    // events are made when timing is switched on, never inside a step call
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, int>> ev_step, ev_wake;   // (start, stop) indices into ev_pool
};

namespace {

int ensure_stage(vfp_batch *b, size_t elems)
{
    if (b->stage_elems >= elems) return VFP_OK;
    if (b->d_stage) HIPCHK(hipFree(b->d_stage));
    b->d_stage = nullptr;
    b->stage_elems = 0;
    HIPCHK(hipMalloc(&b->d_stage, elems * sizeof(double)));
    b->stage_elems = elems;
    return VFP_OK;
}

// host -> device copy that has completed when it returns (sources are often
// short-lived host vectors)
int upload(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return VFP_OK;
}

int upload_sims(vfp_batch *b) { return upload(b->d_sd, b->sd.data(), sizeof(SimDev) * b->count, b->stream); }

template <typename T>
int upload_vec(vfp_batch *b, T *&dev, size_t &cap, const std::vector<T> &v)
{
    if (v.size() > cap) {
        if (dev) HIPCHK(hipFree(dev));
        dev = nullptr;
        cap = 0;
        HIPCHK(hipMalloc(&dev, sizeof(T) * v.size()));
        cap = v.size();
    }
    return v.empty() ? VFP_OK : upload(dev, v.data(), sizeof(T) * v.size(), b->stream);
}

// the FP32-storage forms on the staged kernel: split tick (wake launch, then
// step launch) or fused tick (one launch)
bool staged_wake(const vfp_batch *b, const Phase &ph) { return is_fp32_storage(b->precision) && ph.fast && ph.wake; }
bool fused_tick(const vfp_batch *b, const Phase &ph) { return staged_wake(b, ph) && b->staged == kStagedFused; }

// Cells per work unit of a batch left at its default: the precision's
// default, narrowed for the FP32-storage forms while the batch would have
// fewer work units than about two rounds of resident workgroups
// (kTargetUnits), down to strips of two columns on its largest grid.  A small
// batch runs latency-bound, and more, narrower strips spread it over more
// compute units (single 256^2 and 512^2 simulations and the 64-simulation
// 256^2 scan each about 6 % faster per tick); the 200-simulation scan has
// 10,400 units at the default and keeps it.
constexpr size_t kTargetUnits = 2560;
int auto_cells(const vfp_batch *b)
{
    const int def = default_cells(b->precision);
    if (!is_fp32_storage(b->precision)) return def;
    int nmax = 0;
    for (const HostSim &h : b->hs) nmax = std::max(nmax, h.p.n);
    int cells = def;
    for (const int c : {8192, 6144, 4096, 3072, 2048, 1536, 1024, 768, 512, 384, 256, 192, 128, 96, 64, 48, 32, 16}) {
        if (c > def) continue;
        if (c < 2 * nmax) break;                  // strips of at least two columns
        cells = c;
        size_t units = 0;
        for (const HostSim &h : b->hs) {
            const int n = h.p.n, w = choose_strip_c(n, c, b->rotation, h.halo);
            units += (size_t)((n + w - 1) / w);
        }
        if (units >= kTargetUnits) break;
    }
    return cells;
}

// Units of the simulations in `sims`, appended in dispatch order: block
// k*kXcds + x of a launch runs on XCD x (the dispatcher deals blocks
// round-robin).  Every XCD gets an equal share of each grid size's strips
// (contiguous runs of strips, so neighbouring strips of a simulation share
// their halo columns in that XCD's L2), larger grids first; the slot list is
// padded with empty units (w = 0) where an XCD's share is shorter.
void lay_out_units(vfp_batch *b, std::vector<int> sims, std::vector<Unit> &out)
{
    std::stable_sort(sims.begin(), sims.end(), [&](int x, int y) { return b->hs[x].p.n > b->hs[y].p.n; });
    std::vector<std::vector<Unit>> xcd(kXcds);
    int x0 = 0;                              // next XCD to take a remainder strip
    for (size_t a = 0; a < sims.size();) {
        const int n = b->hs[sims[a]].p.n;
        std::vector<Unit> cls;               // strips of every simulation of this grid size
        for (; a < sims.size() && b->hs[sims[a]].p.n == n; ++a) {
            const int s = sims[a];
            const int w = b->staged ? choose_strip_c(n, b->cells, b->rotation, b->hs[s].halo) : choose_strip(n, b->cells);
            const int nu = (n + w - 1) / w;
            for (int i0 = 0; i0 < n; i0 += w) cls.push_back(Unit{s, i0, std::min(w, n - i0), nu});
        }
        // q strips to every XCD and one more to r of them, taken in turn
        // across the grid sizes so that the remainders do not pile up
        const size_t q = cls.size() / kXcds, r = cls.size() % kXcds;
        size_t at = 0;
        for (int x = 0; x < kXcds; ++x) {
            const size_t len = q + ((size_t)((x - x0 + kXcds) % kXcds) < r ? 1 : 0);
            xcd[x].insert(xcd[x].end(), cls.begin() + at, cls.begin() + at + len);
            at += len;
        }
        x0 = (int)((x0 + r) % kXcds);
    }
    size_t rounds = 0;
    for (int x = 0; x < kXcds; ++x) rounds = std::max(rounds, xcd[x].size());
    for (size_t k = 0; k < rounds; ++k)
        for (int x = 0; x < kXcds; ++x) out.push_back(k < xcd[x].size() ? xcd[x][k] : Unit{0, 0, 0, 0});
}

// Item list of the fused tick for one group: each simulation's wake tiles
// (w = -1, tile index in i0) first, padded to whole rounds of kXcds slots so
// that the units keep their XCD placement, then the group's units in
// dispatch order with nu = their simulation's wake tile count.  A unit waits
// only for its simulation's tiles, which all come before it and wait for
// nothing.
void lay_out_items(vfp_batch *b, const Group &g)
{
    std::vector<int> nt(b->count, 0);
    for (size_t t = g.tile_off; t < g.tile_off + g.tile_cnt; ++t) {
        const WakeTile &w = b->wtiles[t];
        b->items.push_back(Unit{w.sim, w.tile, -1, 0});
        ++nt[w.sim];
    }
    while (b->items.size() % kXcds) b->items.push_back(Unit{0, 0, 0, 0});
    for (size_t k = g.unit_off; k < g.unit_off + g.unit_cnt; ++k) {
        Unit u = b->units[k];
        if (u.w > 0) u.nu = nt[u.sim];
        b->items.push_back(u);
    }
}

void destroy_graphs(vfp_batch *b)
{
    for (Phase &ph : b->phases) {
        for (Group &gr : ph.grp)
            for (int p = 0; p < 2; ++p) {
                if (gr.gexec[p]) (void)hipGraphExecDestroy(gr.gexec[p]);
                if (gr.graph[p]) (void)hipGraphDestroy(gr.graph[p]);
                gr.gexec[p] = nullptr;
                gr.graph[p] = nullptr;
            }
        ph.graphs = false;
    }
}

int capture_graph(vfp_batch *b, Phase &ph, int g, int par);

// Retirement phases from the current state, their device arrays and graphs.
// Called by create and by every call that changes the set of simulations,
// their state or the tuning; never by a step call.  Drains the stream first
// (queued launches may still read the arrays it replaces).
int rebuild(vfp_batch *b)
{
    HIPCHK(hipStreamSynchronize(b->stream));
    for (int g = 0; g < kMaxGroups - 1; ++g)
        if (b->xstream[g]) HIPCHK(hipStreamSynchronize(b->xstream[g]));
    b->forked = false;
    destroy_graphs(b);
    b->phases.clear();
    b->cur = 0;
    b->units.clear();
    b->items.clear();
    b->actv.clear();
    b->wtiles.clear();
    // simulations whose step budget is used up retire now
    std::vector<int64_t> ends;
    for (int s = 0; s < b->count; ++s) {
        HostSim &h = b->hs[s];
        if (!h.active || h.p.max_steps <= 0) continue;
        if (h.steps >= h.p.max_steps) {
            h.active = false;
            h.frozen_buf = b->parity;
        } else {
            ends.push_back(b->tick + (h.p.max_steps - h.steps));
        }
    }
    std::sort(ends.begin(), ends.end());
    ends.erase(std::unique(ends.begin(), ends.end()), ends.end());
    ends.push_back(INT64_MAX);
    int64_t start = b->tick;
    for (int64_t e : ends) {
        Phase ph;
        ph.start = start;
        ph.end = e;
        for (int s = 0; s < b->count; ++s) {
            const HostSim &h = b->hs[s];
            if (!h.active) continue;
            const int64_t rt = h.p.max_steps > 0 ? b->tick + (h.p.max_steps - h.steps) : INT64_MAX;
            if (rt <= start) continue;
            ph.active.push_back(s);
            if (rt == e) ph.retire.push_back(s);
        }
        start = e;
        b->phases.push_back(std::move(ph));
        if (b->phases.back().active.empty()) break;
    }
    if (b->phases.back().end != INT64_MAX || !b->phases.back().active.empty()) {
        Phase tail;                         // every simulation has retired
        tail.start = b->phases.back().end;
        b->phases.push_back(tail);
    }
    for (Phase &ph : b->phases) {
        ph.fast = b->staged > 0 && is_fp32_storage(b->precision) && !ph.active.empty();
        ph.wake = false;
        for (int s : ph.active) {
            ph.fast = ph.fast && b->hs[s].fast;
            ph.wake = ph.wake || b->sd[s].has_wake;
        }
        // groups: balance the cells over the streams (largest grids first, each to
        // the group with the fewest cells so far); one group while timing
        ph.ngroups = b->timing ? 1 : std::max(1, std::min(b->lanes, (int)ph.active.size()));
        std::vector<std::vector<int>> gs(ph.ngroups);
        {
            std::vector<int> order(ph.active);
            std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->hs[x].p.n > b->hs[y].p.n; });
            double load[kMaxGroups] = {};
            for (int s : order) {
                int g = 0;
                for (int h = 1; h < ph.ngroups; ++h)
                    if (load[h] < load[g]) g = h;
                gs[g].push_back(s);
                load[g] += (double)b->hs[s].p.n * b->hs[s].p.n;
            }
        }
        size_t mx = 0;
        ph.lds_wake = 0;
        for (int g = 0; g < ph.ngroups; ++g) {
            Group &gr = ph.grp[g];
            gr.act_off = b->actv.size();
            gr.act_cnt = gs[g].size();
            b->actv.insert(b->actv.end(), gs[g].begin(), gs[g].end());
            gr.unit_off = b->units.size();
            lay_out_units(b, gs[g], b->units);
            gr.unit_cnt = b->units.size() - gr.unit_off;
            for (size_t k = gr.unit_off; k < gr.unit_off + gr.unit_cnt; ++k) {
                const Unit &u = b->units[k];
                if (u.w == 0) continue;
                const size_t n = b->hs[u.sim].p.n;
                mx = std::max(mx, ph.fast ? lds_bytes_c((int)n, u.w, b->rotation, b->hs[u.sim].halo)
                                          : 2 * (size_t)u.w * n * elem_size(b->precision));
            }
            gr.tile_off = b->wtiles.size();
            if (is_fp32_storage(b->precision)) {
                for (int s : gs[g]) {
                    const int n = b->hs[s].p.n;
                    const int nt = b->precision == VFP_FP32 ? (n + kWakeVecRows - 1) / kWakeVecRows
                                                            : ((n + 15) / 16 + 15) / 16;
                    for (int t = 0; t < nt; ++t) b->wtiles.push_back(WakeTile{s, t, 0, 0});
                    ph.lds_wake = std::max(ph.lds_wake, b->precision == VFP_FP32 ? wake_vec_lds(n) : wake_mfma_lds(n));
                }
            }
            gr.tile_cnt = b->wtiles.size() - gr.tile_off;
            gr.item_off = b->items.size();
            if (fused_tick(b, ph)) lay_out_items(b, gr);
            gr.item_cnt = b->items.size() - gr.item_off;
        }
        ph.lds_step = fused_tick(b, ph) ? std::max(mx, ph.lds_wake) : mx;
        if (ph.lds_step > 150 * 1024 || ph.lds_wake > 150 * 1024)
            return fail(VFP_EINVAL, "strip does not fit the workgroup's LDS; lower cells_per_unit");
    }
    // counters of the fused tick start from zero in every new layout (a revived
    // simulation may have left its last tick's count behind)
    HIPCHK(hipMemsetAsync(b->d_done, 0, sizeof(unsigned) * 2 * b->count, b->stream));
    for (std::vector<Unit> *v : {&b->units, &b->items})
        for (Unit &u : *v)
            if (u.w > 0) {
                const SimDev &d = b->sd[u.sim];
                u.n = d.n;
                u.hl = d.hl;
                u.hr = d.hr;
                u.psi[0] = d.psi[0];
                u.psi[1] = d.psi[1];
            }
    int rc = upload_vec(b, b->d_units, b->units_cap, b->units);
    if (rc == VFP_OK) rc = upload_vec(b, b->d_items, b->items_cap, b->items);
    if (rc == VFP_OK) rc = upload_vec(b, b->d_active, b->actv_cap, b->actv);
    if (rc == VFP_OK) rc = upload_vec(b, b->d_wtiles, b->wtiles_cap, b->wtiles);
    if (rc) return rc;
    // graph length: even (keeps the parity) and a multiple of the record cadence
    b->G = b->every > 0 ? (b->every % 2 ? 2 * b->every : b->every) : 16;
    while (b->G < 16) b->G *= 2;
    if (b->use_graph && !b->timing) {
        int made = 0;
        for (Phase &ph : b->phases) {
            if (ph.active.empty() || ph.end - ph.start < b->G) continue;
            if (made++ == kMaxGraphPhases) break;
            for (int g = 0; g < ph.ngroups; ++g)
                for (int par = 0; par < 2; ++par) {
                    rc = capture_graph(b, ph, g, par);
                    if (rc) return rc;
                }
            ph.graphs = true;
        }
    }
    return VFP_OK;
}

// ------------------------------------------------------------- launches
// launch target: one group of a phase on its stream
struct Target {
    const Unit *units;
    int nunits;
    const Unit *items;
    int nitems;
    const WakeTile *tiles;
    int ntiles;
    size_t lds_step, lds_wake;
    hipStream_t st;
};

Target target(vfp_batch *b, const Phase &ph, int g)
{
    const Group &gr = ph.grp[g];
    return Target{b->d_units + gr.unit_off, (int)gr.unit_cnt, b->d_items ? b->d_items + gr.item_off : nullptr,
                  (int)gr.item_cnt, b->d_wtiles ? b->d_wtiles + gr.tile_off : nullptr, (int)gr.tile_cnt,
                  ph.lds_step, ph.lds_wake, g == 0 ? b->stream : b->xstream[g - 1]};
}

template <typename T, int K, int WAKE, bool CL, int ROT>
void launch_step_t(vfp_batch *b, const Target &t, int parity)
{
    auto k = [] {
        if constexpr (std::is_same_v<T, int64_t>) return stepfix_kernel<K, WAKE, CL, ROT>;
        else return step_kernel<T, K, WAKE, CL, ROT>;
    }();
    static int cur = 0;
    lds_limit(k, t.lds_step, cur);
    hipLaunchKernelGGL(k, dim3((unsigned)t.nunits), dim3(kThreads), t.lds_step, t.st, b->d_sd, t.units, t.nunits,
                       parity);
}

template <int K, int WAKE, bool CL, int ROT, bool MOM = false>
void launch_step32c_t(vfp_batch *b, const Target &t, int parity)
{
    static int cur = 0;
    lds_limit(step32c_kernel<K, WAKE, CL, ROT, MOM>, t.lds_step, cur);
    hipLaunchKernelGGL((step32c_kernel<K, WAKE, CL, ROT, MOM>), dim3((unsigned)t.nunits), dim3(kThreads), t.lds_step,
                       t.st, b->d_sd, t.units, t.nunits, parity);
}

// the staged step of the split tick, with the per-column moments of the new
// state when a record row follows (`mom`)
template <int K, int WAKE, bool CL, int ROT>
void launch_step32c_m(vfp_batch *b, const Target &t, int parity, bool mom)
{
    if constexpr (WAKE == WAKE_EXTERNAL) {
        if (mom) {
            launch_step32c_t<K, WAKE, CL, ROT, true>(b, t, parity);
            return;
        }
    }
    launch_step32c_t<K, WAKE, CL, ROT>(b, t, parity);
}

template <int K, bool CL, int ROT, int WK, bool MOM>
void launch_tick32_t(vfp_batch *b, const Target &t, int parity)
{
    static int cur = 0;
    lds_limit(tick32_kernel<K, CL, ROT, WK, MOM>, t.lds_step, cur);
    hipLaunchKernelGGL((tick32_kernel<K, CL, ROT, WK, MOM>), dim3((unsigned)t.nitems), dim3(kThreads), t.lds_step,
                       t.st, b->d_sd, t.items, t.nitems, parity, b->d_done, b->count, b->d_flag);
}

template <int K, bool CL, int ROT, int WK>
void launch_tick32_m(vfp_batch *b, const Target &t, int parity, bool mom)
{
    if (mom) launch_tick32_t<K, CL, ROT, WK, true>(b, t, parity);
    else launch_tick32_t<K, CL, ROT, WK, false>(b, t, parity);
}

template <int K, bool CL, int ROT>
void launch_tick32_w(vfp_batch *b, const Target &t, int parity, bool mom)
{
    if (b->precision == VFP_MIXED_FP16) launch_tick32_m<K, CL, ROT, TW_FP16>(b, t, parity, mom);
    else if (b->precision == VFP_MIXED_BF16) launch_tick32_m<K, CL, ROT, TW_BF16>(b, t, parity, mom);
    else launch_tick32_m<K, CL, ROT, TW_VEC>(b, t, parity, mom);
}

// the step launch of a tick: kernel by storage type, wake mode, layout and tick form
// (mom: the staged step of either tick form also leaves the new state's
// per-column moments; the caller reads *mom_done to know whether it did)
template <typename T, int K, int WAKE>
void launch_step_w(vfp_batch *b, const Phase &ph, const Target &t, int parity, bool mom, bool *mom_done)
{
    if constexpr (sizeof(T) == 4) {
        if (ph.fast) {
            if (WAKE == WAKE_EXTERNAL && b->staged == kStagedFused) {
                if (b->rotation) {
                    if (b->clamp) launch_tick32_w<K, true, 1>(b, t, parity, mom);
                    else launch_tick32_w<K, false, 1>(b, t, parity, mom);
                } else {
                    if (b->clamp) launch_tick32_w<K, true, 0>(b, t, parity, mom);
                    else launch_tick32_w<K, false, 0>(b, t, parity, mom);
                }
                if (mom_done) *mom_done = mom;
            } else {
                if (b->rotation) {
                    if (b->clamp) launch_step32c_m<K, WAKE, true, 1>(b, t, parity, mom);
                    else launch_step32c_m<K, WAKE, false, 1>(b, t, parity, mom);
                } else {
                    if (b->clamp) launch_step32c_m<K, WAKE, true, 0>(b, t, parity, mom);
                    else launch_step32c_m<K, WAKE, false, 0>(b, t, parity, mom);
                }
                if (mom_done) *mom_done = mom && WAKE == WAKE_EXTERNAL;
            }
            return;
        }
    }
    if (b->clamp) {
        if (b->rotation) launch_step_t<T, K, WAKE, true, 1>(b, t, parity);
        else launch_step_t<T, K, WAKE, true, 0>(b, t, parity);
    } else {
        if (b->rotation) launch_step_t<T, K, WAKE, false, 1>(b, t, parity);
        else launch_step_t<T, K, WAKE, false, 0>(b, t, parity);
    }
}

template <typename T, int WAKE>
void launch_step_k(vfp_batch *b, const Phase &ph, const Target &t, int parity, bool mom = false,
                   bool *mom_done = nullptr)
{
    if (b->K == 3) launch_step_w<T, 3, WAKE>(b, ph, t, parity, mom, mom_done);
    else launch_step_w<T, 4, WAKE>(b, ph, t, parity, mom, mom_done);
}

// the wake of every simulation of the target from the column sums in buffer
// `parity` (a launch of its own: every tick of the split form and of the
// generic FP32 kernel, and the first tick of the fused form)
void launch_wake(vfp_batch *b, const Target &t, int parity)
{
    if (t.ntiles == 0) return;
    if (b->precision == VFP_FP32) {
        static int cur = 0;
        lds_limit(wake_vec_kernel, t.lds_wake, cur);
        hipLaunchKernelGGL(wake_vec_kernel, dim3((unsigned)t.ntiles), dim3(kThreads), t.lds_wake, t.st, b->d_sd,
                           t.tiles, parity);
    } else {
        const bool fp16 = b->precision == VFP_MIXED_FP16;
        auto wk = fp16 ? wake_mfma2_kernel<true> : wake_mfma2_kernel<false>;
        static int cur16 = 0, cur8 = 0;
        lds_limit(wk, t.lds_wake, fp16 ? cur16 : cur8);
        hipLaunchKernelGGL(wk, dim3((unsigned)t.ntiles), dim3(kThreads), t.lds_wake, t.st, b->d_sd, t.tiles, parity);
    }
}

// the other groups' streams start after the work already queued on the batch's stream
int fork_streams(vfp_batch *b, const Phase &ph)
{
    if (ph.ngroups < 2 || b->forked) return VFP_OK;
    HIPCHK(hipEventRecord(b->ev_fork, b->stream));
    for (int g = 1; g < ph.ngroups; ++g) HIPCHK(hipStreamWaitEvent(b->xstream[g - 1], b->ev_fork, 0));
    b->forked = true;
    b->forked_groups = ph.ngroups;
    return VFP_OK;
}

// the batch's stream continues after the other groups' work
int join_streams(vfp_batch *b)
{
    if (!b->forked) return VFP_OK;
    for (int g = 1; g < b->forked_groups; ++g) {
        HIPCHK(hipEventRecord(b->ev_join[g - 1], b->xstream[g - 1]));
        HIPCHK(hipStreamWaitEvent(b->stream, b->ev_join[g - 1], 0));
    }
    b->forked = false;
    return VFP_OK;
}

// next event of the timing pool (recorded on the batch's stream), or -1 once
// the pool is used up
int timing_event(vfp_batch *b)
{
    if (b->ev_used >= b->ev_pool.size()) return -1;
    const int idx = (int)b->ev_used++;
    return hipEventRecord(b->ev_pool[idx], b->stream) == hipSuccess ? idx : -1;
}

// the launches of one tick of group g that reads buffer `parity`, on the
// group's stream: the FP32-storage forms on the staged kernel run a wake
// launch then a step launch (split) or one launch (fused); FP64 and fixed
// point one step launch with the wake slice inside; the generic FP32 kernel a
// wake launch then its step launch
int launch_group_tick(vfp_batch *b, const Phase &ph, int g, int parity, bool rec = false, bool *mom_done = nullptr)
{
    const bool sep_wake = is_fp32_storage(b->precision) && ph.wake && !fused_tick(b, ph);
    const Target t = target(b, ph, g);
    if (t.nunits == 0) return VFP_OK;
    const bool timed = b->timing;             // timing runs in one group, on the batch's stream
    const int t0 = timed ? timing_event(b) : -1;
    int t1 = -1;
    if (b->precision == VFP_FP64) {
        if (ph.wake) launch_step_k<double, WAKE_FUSED>(b, ph, t, parity);
        else launch_step_k<double, WAKE_NONE>(b, ph, t, parity);
    } else if (b->precision == VFP_FIXED) {
        if (ph.wake) launch_step_k<int64_t, WAKE_FUSED>(b, ph, t, parity);
        else launch_step_k<int64_t, WAKE_NONE>(b, ph, t, parity);
    } else if (!ph.wake) {
        launch_step_k<float, WAKE_NONE>(b, ph, t, parity);
    } else {
        if (sep_wake) {
            launch_wake(b, t, parity);
            if (timed) t1 = timing_event(b);
        }
        launch_step_k<float, WAKE_EXTERNAL>(b, ph, t, parity, rec, mom_done);
    }
    HIPCHK(hipGetLastError());
    if (timed) {
        const int t2 = timing_event(b);
        if (t0 >= 0 && t2 >= 0) {
            if (sep_wake && t1 >= 0) {
                b->ev_wake.push_back({t0, t1});
                b->ev_step.push_back({t1, t2});
            } else if (!sep_wake) {
                b->ev_step.push_back({t0, t2});
            }
        }
    }
    return VFP_OK;
}

// stats over an explicit list of (simulation, buffer) pairs
int launch_stats(vfp_batch *b, const int *d_which, const int *d_buf, int cnt, int record, hipStream_t st,
                 bool have_moments = false)
{
    if (cnt == 0) return VFP_OK;
    // per-column sums over 16-column tiles of the largest grid (unless the
    // step that made the state left them)
    const int maxn = (int)(b->lds_stats / (2 * sizeof(double)));
    const dim3 mgrid((unsigned)((maxn + 15) / 16), (unsigned)cnt);
    if (have_moments)
        ;
    else if (b->precision == VFP_FP64)
        hipLaunchKernelGGL(moments_kernel<double>, mgrid, dim3(kThreads), 0, st, b->d_sd, d_which, d_buf);
    else if (b->precision == VFP_FIXED)
        hipLaunchKernelGGL(moments_kernel<int64_t>, mgrid, dim3(kThreads), 0, st, b->d_sd, d_which, d_buf);
    else
        hipLaunchKernelGGL(moments_kernel<float>, mgrid, dim3(kThreads), 0, st, b->d_sd, d_which, d_buf);
    if (b->precision == VFP_FP64) {
        static int cur = 0;
        lds_limit(stats_kernel<double>, b->lds_stats, cur);
        hipLaunchKernelGGL(stats_kernel<double>, dim3(cnt), dim3(kThreads), b->lds_stats, st, b->d_sd,
                           d_which, d_buf);
    } else if (b->precision == VFP_FIXED) {
        static int cur = 0;
        lds_limit(stats_kernel<int64_t>, b->lds_stats, cur);
        hipLaunchKernelGGL(stats_kernel<int64_t>, dim3(cnt), dim3(kThreads), b->lds_stats, st, b->d_sd,
                           d_which, d_buf);
    } else {
        static int cur = 0;
        lds_limit(stats_kernel<float>, b->lds_stats, cur);
        hipLaunchKernelGGL(stats_kernel<float>, dim3(cnt), dim3(kThreads), b->lds_stats, st, b->d_sd,
                           d_which, d_buf);
    }
    // the wake of every listed simulation over row tiles of the largest grid, then P
    const unsigned tiles = (unsigned)((maxn + 63) / 64);
    wakev_limit(wakev_lds(maxn));
    hipLaunchKernelGGL(wakev_kernel, dim3(tiles, (unsigned)cnt), dim3(kThreads), wakev_lds(maxn), st, b->d_sd,
                       d_which);
    hipLaunchKernelGGL(power_kernel, dim3(cnt), dim3(kThreads), 0, st, b->d_sd, d_which, b->rec_base,
                       b->every, record);
    HIPCHK(hipGetLastError());
    return VFP_OK;
}

// record launch of group g after a tick that read buffer `par`: the group's
// simulations' fresh states are in buffer par ^ 1
int launch_record(vfp_batch *b, const Phase &ph, int g, int par, bool have_moments)
{
    const Group &gr = ph.grp[g];
    return launch_stats(b, b->d_active + gr.act_off, b->d_buf01 + (par ^ 1) * b->count, (int)gr.act_cnt, 1,
                        g == 0 ? b->stream : b->xstream[g - 1], have_moments);
}

// d_idx[0..count) = all simulations, d_idx[count..2count) = their buffers
int stage_all_indices(vfp_batch *b)
{
    std::vector<int> v(2 * b->count);
    for (int s = 0; s < b->count; ++s) {
        v[s] = s;
        v[b->count + s] = b->hs[s].active ? b->parity : b->hs[s].frozen_buf;
    }
    return upload(b->d_idx, v.data(), sizeof(int) * v.size(), b->stream);
}

int refresh_stats(vfp_batch *b)
{
    int rc = stage_all_indices(b);
    if (rc) return rc;
    rc = launch_stats(b, b->d_idx, b->d_idx + b->count, b->count, 0, b->stream);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(b->stream));
    return VFP_OK;
}

int check_finite(vfp_batch *b, int s)
{
    double bad = 0.0;
    int late = 0;
    HIPCHK(hipMemcpy(&bad, (double *)(b->arena + b->hs[s].off_stat) + 7, sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&late, b->d_flag, sizeof(int), hipMemcpyDeviceToHost));
    if (late != 0) return fail(VFP_EDEVICE, "a unit's wait for its simulation's wake tiles exceeded its bound");
    if (bad != 0.0) return fail(VFP_EDEVICE, "non-finite density or wake detected");
    return VFP_OK;
}

// the launches of one tick of group g at tick position `tk` reading buffer
// `par`, plus the group's record launch when due
int enqueue_group_tick(vfp_batch *b, const Phase &ph, int g, int par, int64_t tk)
{
    const bool rec = b->every > 0 && ((tk + 1 - b->rec_base) % b->every) == 0;
    bool mom = false;
    int rc = launch_group_tick(b, ph, g, par, rec, &mom);
    if (rc == VFP_OK && rec) rc = launch_record(b, ph, g, par, mom);
    return rc;
}

// one tick of every group (the groups forked from the batch's stream first)
int enqueue_tick(vfp_batch *b, const Phase &ph, int par, int64_t tk)
{
    int rc = fork_streams(b, ph);
    for (int g = 0; g < ph.ngroups && rc == VFP_OK; ++g) rc = enqueue_group_tick(b, ph, g, par, tk);
    return rc;
}

// capture G ticks of group g of phase ph starting at parity par, on the
// group's stream alone; the graph is replayed only at ticks aligned with the
// record cadence, so record positions are those of a start at rec_base
int capture_graph(vfp_batch *b, Phase &ph, int g, int par)
{
    const int p0 = par;
    hipStream_t st = g == 0 ? b->stream : b->xstream[g - 1];
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    int rc = VFP_OK;
    for (int t = 0; t < b->G && rc == VFP_OK; ++t) {
        rc = enqueue_group_tick(b, ph, g, par, b->rec_base + t);
        par ^= 1;
    }
    hipGraph_t gr = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &gr);
    if (rc) { if (gr) (void)hipGraphDestroy(gr); return rc; }
    if (e != hipSuccess) return fail(VFP_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    ph.grp[g].graph[p0] = gr;
    HIPCHK(hipGraphInstantiate(&ph.grp[g].gexec[p0], gr, nullptr, nullptr, 0));
    HIPCHK(hipGraphUpload(ph.grp[g].gexec[p0], st));      // its first replay starts at once
    return VFP_OK;
}


// Enqueue nticks ticks: graph replays where a whole graph fits before the
// next retirement (and starts on the record cadence), single ticks otherwise;
// retirements switch to the next prepared phase.  The groups run forked on
// their streams and are joined into the batch's stream at the end of the
// call.  Host bookkeeping and enqueued work only: no allocation, no
// synchronisation.
int advance(vfp_batch *b, int64_t nticks)
{
    if (nticks < 0) return fail(VFP_EINVAL, "negative step count");
    int rc = VFP_OK;
    while (nticks > 0 && rc == VFP_OK) {
        Phase &ph = b->phases[b->cur];
        if (ph.active.empty()) break;                  // every simulation has retired
        const int64_t until = std::min(nticks, ph.end - b->tick);
        int64_t done = 0;
        while (done < until) {
            const int64_t left = until - done;
            const bool aligned = b->every == 0 || ((b->tick - b->rec_base) % b->every) == 0;
            if (ph.graphs && !b->timing && left >= b->G && aligned) {
                rc = fork_streams(b, ph);
                for (int g = 0; g < ph.ngroups && rc == VFP_OK; ++g)
                    if (hipGraphLaunch(ph.grp[g].gexec[b->parity], g == 0 ? b->stream : b->xstream[g - 1]) !=
                        hipSuccess)
                        rc = fail(VFP_EDEVICE, "graph launch failed");
                if (rc) break;
                b->tick += b->G;
                done += b->G;
            } else {
                rc = enqueue_tick(b, ph, b->parity, b->tick);
                if (rc) break;
                b->parity ^= 1;
                ++b->tick;
                ++done;
            }
        }
        for (int s : ph.active) b->hs[s].steps += done;
        nticks -= done;
        if (b->tick == ph.end) {
            for (int s : ph.retire) {
                b->hs[s].active = false;
                b->hs[s].frozen_buf = b->parity;
            }
            ++b->cur;
            if (rc == VFP_OK) rc = join_streams(b);    // the next phase forks its own groups
        }
    }
    const int jrc = join_streams(b);                   // the call ends with everything on the batch's stream
    return rc ? rc : jrc;
}

void free_batch(vfp_batch *b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    destroy_graphs(b);
    if (b->own_arena && b->arena) (void)hipFree(b->arena);
    if (b->d_sd) (void)hipFree(b->d_sd);
    if (b->d_units) (void)hipFree(b->d_units);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_active) (void)hipFree(b->d_active);
    if (b->d_wtiles) (void)hipFree(b->d_wtiles);
    if (b->d_done) (void)hipFree(b->d_done);
    if (b->d_flag) (void)hipFree(b->d_flag);
    if (b->d_idx) (void)hipFree(b->d_idx);
    if (b->d_buf01) (void)hipFree(b->d_buf01);
    if (b->d_ring) (void)hipFree(b->d_ring);
    if (b->d_ring_rows) (void)hipFree(b->d_ring_rows);
    if (b->d_stage) (void)hipFree(b->d_stage);
    for (hipEvent_t e : b->ev_pool) (void)hipEventDestroy(e);
    for (int g = 0; g < kMaxGroups - 1; ++g) {
        if (b->xstream[g]) {
            (void)hipStreamSynchronize(b->xstream[g]);
            (void)hipStreamDestroy(b->xstream[g]);
        }
        if (b->ev_join[g]) (void)hipEventDestroy(b->ev_join[g]);
    }
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

// Haissinski iteration of simulation i (named in d_idx[0]): Gaussian start,
// then per iteration the wake of the profile over 64-row tiles and one damped
// update, then psi into buffer buf
template <typename T>
int launch_haissinski(vfp_batch *b, int i, int buf, int iters, double alpha)
{
    const int n = b->hs[i].p.n;
    const size_t lds = (size_t)n * sizeof(double);
    static int cur = 0;
    lds_limit(haissinski_kernel<T>, lds, cur);
    hipLaunchKernelGGL(haissinski_kernel<T>, dim3(1), dim3(kThreads), 0, b->stream, b->d_sd, i, buf, 0, alpha);
    wakev_limit(wakev_lds(n));
    for (int it = 0; it < iters; ++it) {
        hipLaunchKernelGGL(wakev_kernel, dim3((unsigned)((n + 63) / 64), 1), dim3(kThreads), wakev_lds(n), b->stream,
                           b->d_sd, b->d_idx);
        hipLaunchKernelGGL(haissinski_kernel<T>, dim3(1), dim3(kThreads), lds, b->stream, b->d_sd, i, buf, 1, alpha);
    }
    hipLaunchKernelGGL(haissinski_kernel<T>, dim3((unsigned)std::min(n, 1024)), dim3(kThreads), 0, b->stream, b->d_sd,
                       i, buf, 2, alpha);
    HIPCHK(hipGetLastError());
    return VFP_OK;
}

// column sums of the stored density of the simulation named in d_idx[0], buffer buf
int launch_project(vfp_batch *b, int n, int buf)
{
    const unsigned cb = (unsigned)((n + kWaves - 1) / kWaves);
    if (b->precision == VFP_FP64)
        hipLaunchKernelGGL(project_kernel<double>, dim3(cb, 1), dim3(kThreads), 0, b->stream, b->d_sd, b->d_idx, buf);
    else if (b->precision == VFP_FIXED)
        hipLaunchKernelGGL(projectfix_kernel, dim3(cb, 1), dim3(kThreads), 0, b->stream, b->d_sd, b->d_idx, buf);
    else
        hipLaunchKernelGGL(project_kernel<float>, dim3(cb, 1), dim3(kThreads), 0, b->stream, b->d_sd, b->d_idx, buf);
    HIPCHK(hipGetLastError());
    return VFP_OK;
}

int upload_psi(vfp_batch *b, int s, const double *psi, bool gaussian)
{
    const HostSim &h = b->hs[s];
    const int n = h.p.n;
    const size_t nn = (size_t)n * n;
    std::vector<double> g;
    if (gaussian) {
        // unit Gaussian on the node grid, normalised to unit charge (input data)
        g.resize(nn);
        const double dq = (h.p.q_max - h.p.q_min) / (n - 1), dp = (h.p.p_max - h.p.p_min) / (n - 1);
        double sum = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double q = h.p.q_min + i * dq, p = h.p.p_min + j * dp;
                g[(size_t)i * n + j] = std::exp(-0.5 * (q * q + p * p));
                sum += g[(size_t)i * n + j];
            }
        for (double &v : g) v /= sum * dq * dp;
        psi = g.data();
    }
    int rc = ensure_stage(b, nn);
    if (rc) return rc;
    rc = upload(b->d_stage, psi, nn * sizeof(double), b->stream);
    if (rc) return rc;
    const int buf = h.active ? b->parity : h.frozen_buf;
    void *dst = b->arena + h.off_psi[buf];
    const unsigned blocks = (unsigned)((nn + kThreads - 1) / kThreads);
    const int fixb = b->sd[s].fixb;
    if (b->precision == VFP_FP64)
        hipLaunchKernelGGL(import_kernel<double>, dim3(blocks), dim3(kThreads), 0, b->stream, b->d_stage,
                           (double *)dst, nn, fixb);
    else if (b->precision == VFP_FIXED)
        hipLaunchKernelGGL(import_kernel<int64_t>, dim3(blocks), dim3(kThreads), 0, b->stream, b->d_stage,
                           (int64_t *)dst, nn, fixb);
    else
        hipLaunchKernelGGL(import_kernel<float>, dim3(blocks), dim3(kThreads), 0, b->stream, b->d_stage,
                           (float *)dst, nn, fixb);
    HIPCHK(hipGetLastError());
    // column sums of the new state, then Q0 = dq*dp*sum from the device
    const int v[2] = {s, buf};
    rc = upload(b->d_idx, v, sizeof(v), b->stream);
    if (rc) return rc;
    rc = launch_project(b, n, buf);
    if (rc) return rc;
    if (b->precision == VFP_FIXED) {
        // Q0 of the stored (rounded) density from its exact integer sum, as every step takes it
        std::vector<int64_t> parts(2 * (size_t)n);
        HIPCHK(hipMemcpyAsync(parts.data(), b->arena + h.off_cs[buf], cs_bytes(VFP_FIXED, n), hipMemcpyDeviceToHost,
                              b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
        int64_t H = 0, L = 0;
        for (int i = 0; i < n; ++i) {
            H += parts[2 * i];
            L += parts[2 * i + 1];
        }
        const double Q0 = std::ldexp((double)H * 4294967296.0 + (double)L, -fixb) * b->sd[s].dq * b->sd[s].dp;
        if (!(Q0 > 0.0) || !std::isfinite(Q0))
            return fail(VFP_EINVAL, "initial density must have a positive, finite charge");
        b->sd[s].Q0 = Q0;
        b->sd[s].step0 = b->tick;
        return upload_sims(b);
    }
    // Q0 = dq*dp*sum(psi0) of the FP64 input (stat[0] is scratch here)
    double *q0dev = (double *)(b->arena + h.off_stat);
    hipLaunchKernelGGL(charge64_kernel, dim3(1), dim3(kThreads), 0, b->stream, b->d_stage, nn,
                       b->sd[s].dq * b->sd[s].dp, q0dev);
    HIPCHK(hipGetLastError());
    double Q0 = 0.0;
    HIPCHK(hipMemcpyAsync(&Q0, q0dev, sizeof(double), hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    if (!(Q0 > 0.0) || !std::isfinite(Q0)) return fail(VFP_EINVAL, "initial density must have a positive, finite charge");
    b->sd[s].Q0 = Q0;
    b->sd[s].step0 = b->tick;
    return upload_sims(b);
}

int create_impl(const vfp_params *p, int32_t count, void *stream, void *ws, size_t ws_bytes, bool plain,
                vfp_batch **out)
{
    if (!out) return fail(VFP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p || count < 1) return fail(VFP_EINVAL, "need at least one parameter set");
    std::string why;
    for (int s = 0; s < count; ++s) {
        const int rc = validate(p[s], why);
        if (rc) return fail(rc, "simulation " + std::to_string(s) + ": " + why);
        if (p[s].interp != p[0].interp || p[s].clamp != p[0].clamp || p[s].precision != p[0].precision ||
            p[s].rotation != p[0].rotation)
            return fail(VFP_EINVAL, "interp, clamp, precision and rotation must agree across a batch");
    }
    vfp_batch *b = new vfp_batch();
    b->count = count;
    b->plain = plain;
    b->use_graph = !plain;
    b->precision = p[0].precision;
    b->K = p[0].interp;
    b->clamp = p[0].clamp;
    b->rotation = p[0].rotation;
    b->cells = default_cells(p[0].precision);
    {
        // the tick form: one launch per tick for a small batch, whose separate
        // wake launch would sit on the tick's critical path, split for a large
        // one, where the other stream groups' step launches hide each wake
        // launch (one 256^2 simulation 9.7 against 12.6 us per tick, one 512^2
        // simulation 13.6 against 17.2 us; the 64-simulation 256^2 scan 17.4
        // against 16.9 us and the 200-simulation scan 94.5 against 85.2 us with
        // three stream groups)
        size_t cells = 0;
        for (int s = 0; s < count; ++s) cells += (size_t)p[s].n * (size_t)p[s].n;
        b->staged = cells <= kFusedTickCells ? kStagedFused : kStagedSplit;
    }
    b->stream = (hipStream_t)stream;
    if (!b->stream) {
        // graphs cannot be captured on the null stream: use a stream of our own
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            delete b;
            return fail(VFP_EDEVICE, "stream creation failed");
        }
        b->own_stream = true;
    }
    bool made = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) == hipSuccess;
    for (int g = 0; g < kMaxGroups - 1 && made; ++g)
        made = hipStreamCreateWithFlags(&b->xstream[g], hipStreamNonBlocking) == hipSuccess &&
               hipEventCreateWithFlags(&b->ev_join[g], hipEventDisableTiming) == hipSuccess;
    if (!made) {
        free_batch(b);
        return fail(VFP_EDEVICE, "stream creation failed");
    }
    b->hs.resize(count);
    for (int s = 0; s < count; ++s) {
        HostSim &h = b->hs[s];
        h.p = p[s];
        if (p[s].z_re) {
            const int M = p[s].padding * p[s].n;
            h.zr.assign(p[s].z_re, p[s].z_re + M / 2 + 1);
            h.zi.assign(p[s].z_im, p[s].z_im + M / 2 + 1);
        }
        h.p.z_re = h.p.z_im = nullptr;
        h.p.psi0 = nullptr;
    }
    const size_t need = layout(p, count, &b->hs);
    if (ws) {
        if (ws_bytes < need) {
            free_batch(b);
            return fail(VFP_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
        }
        b->arena = (unsigned char *)ws;
    } else {
        if (hipMalloc(&b->arena, need) != hipSuccess) {
            free_batch(b);
            return fail(VFP_ENOMEM, "device allocation of " + std::to_string(need) + " bytes failed");
        }
        b->own_arena = true;
    }
    b->arena_bytes = need;
    int rc = VFP_OK;
    auto bail = [&](int code) { free_batch(b); return code; };
    if (hipMalloc(&b->d_sd, sizeof(SimDev) * count) != hipSuccess ||
        hipMalloc(&b->d_done, sizeof(unsigned) * 2 * count) != hipSuccess ||
        hipMalloc(&b->d_flag, sizeof(int)) != hipSuccess ||
        hipMalloc(&b->d_idx, sizeof(int) * 2 * count) != hipSuccess ||
        hipMalloc(&b->d_buf01, sizeof(int) * 2 * count) != hipSuccess)
        return bail(fail(VFP_ENOMEM, "device allocation failed"));
    if (hipMemsetAsync(b->d_flag, 0, sizeof(int), b->stream) != hipSuccess)
        return bail(fail(VFP_EDEVICE, "setup failed"));
    {
        std::vector<int> t01(2 * count, 0);
        for (int s = 0; s < count; ++s) t01[count + s] = 1;
        if (hipMemcpy(b->d_buf01, t01.data(), sizeof(int) * t01.size(), hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(VFP_EDEVICE, "upload failed"));
    }
    // descriptors
    b->sd.resize(count);
    int maxn = 0;
    for (int s = 0; s < count; ++s) {
        const HostSim &h = b->hs[s];
        const vfp_params &q = h.p;
        SimDev &d = b->sd[s];
        std::memset(&d, 0, sizeof(d));
        maxn = std::max(maxn, q.n);
        d.n = q.n;
        d.K = q.interp;
        d.rotation = q.rotation;
        d.clamp = q.clamp;
        d.renorm = q.renormalize;
        d.has_wake = (p[s].z_re != nullptr || p[s].z_model != VFP_Z_SAMPLES) ? 1 : 0;
        d.M = q.padding * q.n;
        d.fixb = q.precision == VFP_FIXED ? q.fix_bits : 0;
        d.q_min = q.q_min;
        d.p_min = q.p_min;
        d.dq = (q.q_max - q.q_min) / (q.n - 1);
        d.dp = (q.p_max - q.p_min) / (q.n - 1);
        d.th = 2.0 * M_PI / q.steps_per_period;
        d.c = std::cos(d.th);
        d.s = std::sin(d.th);
        d.bt = q.beta * d.th;
        d.kick = d.th / d.dp;
        d.S = q.z_scale;
        d.Q0 = 1.0;
        const double cm1 = -2.0 * std::sin(0.5 * d.th) * std::sin(0.5 * d.th);   // cos - 1
        d.ax0 = (q.q_min * cm1 - q.p_min * d.s) / d.dq;
        d.axi = cm1;
        d.bx = -d.s * d.dp / d.dq;
        d.cy0 = (q.q_min * d.s + q.p_min * cm1) / d.dp;
        d.cyi = d.s * d.dq / d.dp;
        d.by = cm1;
        d.pm = q.p_min / d.dp;
        d.tw = d.th * d.dp / d.dq;
        d.tk = d.th * d.dq / d.dp;
        {
            const double k1 = d.bt / 6.0, k2 = d.bt / (d.dp * d.dp);
            d.fbx = (float)d.bx;
            d.fby = (float)d.by;
            d.fk1 = (float)k1;
            d.fe[0] = (float)(2.0 * k1 + k2);
            d.fe[1] = (float)(1.0 - 2.0 * k2);
            d.fe[2] = (float)(6.0 * k1 + k2);
            d.fe[3] = (float)(-2.0 * k1);
            d.fd0 = (float)(-d.tw * d.pm);
            d.fd1 = (float)(-d.tw);
        }
        unsigned char *A = b->arena;
        d.psi[0] = A + h.off_psi[0];
        d.psi[1] = A + h.off_psi[1];
        d.colsum[0] = (double *)(A + h.off_cs[0]);
        d.colsum[1] = (double *)(A + h.off_cs[1]);
        d.wl64 = (const double *)(A + h.off_wl64);
        d.wl32 = (const float *)(A + h.off_wl32);
        d.wsplit = (const uint16_t *)(A + h.off_frag);
        d.vext = (float *)(A + h.off_vext);
        d.sext = (double *)(A + h.off_sext);
        d.rho_out = (double *)(A + h.off_rho);
        d.v_out = (double *)(A + h.off_v);
        d.stat = (double *)(A + h.off_stat);
        d.mom = (double *)(A + h.off_mom);
        d.zr64 = (const double *)(A + h.off_zr);
        // the staged kernel needs n % 4 == 0 and a rotation source within 2 cells of every
        // node; dx, dy are linear in (i, j), so the corners bound them
        double lo = 1e300, hi = -1e300, lox = 1e300, hix = -1e300;
        for (int ci = 0; ci < 2; ++ci)
            for (int cj = 0; cj < 2; ++cj) {
                const double i = ci ? q.n - 1 : 0, j = cj ? q.n - 1 : 0;
                const double dx = d.ax0 + i * d.axi + j * d.bx, dy = d.cy0 + i * d.cyi + j * d.by;
                lo = std::min(lo, std::min(dx, dy));
                hi = std::max(hi, std::max(dx, dy));
                lox = std::min(lox, dx);
                hix = std::max(hix, dx);
            }
        if (q.rotation == VFP_ROT_MANHATTAN) {
            // drift shifts -tw*(p_min/dp + j), RF kick shifts tk*(q_min/dq + i)
            lo = lox = 1e300;
            hi = hix = -1e300;
            // (the drift runs over every staged row, four beyond each end of the grid)
            for (int e = 0; e < 2; ++e) {
                const double k = e ? q.n - 1 : 0, ky = e ? q.n + 3 : -4;
                const double a = -d.tw * (d.pm + ky), c = d.tk * (q.q_min / d.dq + k);
                lo = std::min(lo, std::min(a, c));
                hi = std::max(hi, std::max(a, c));
                lox = std::min(lox, a);
                hix = std::max(hix, a);
            }
        }
        // (the margin covers FP32 evaluation of the displacement in the staged kernels)
        b->hs[s].fast = q.n % 4 == 0 && lo > -2.0 + 1e-5 && hi < 2.0 - 1e-5;
        // staged columns beside a strip: output column c reads source columns
        // c + floor(dx) - o0 .. c + floor(dx) + K - 1 - o0 (dx: the column
        // displacement, or the drift shift of the Manhattan rotation)
        {
            const int o0 = (q.interp - 1) / 2;
            const int mlo = (int)std::floor(std::max(lox - 1e-5, -2.0)), mhi = (int)std::floor(std::min(hix + 1e-5, 1.9));
            d.hl = std::min(kH, std::max(0, o0 - mlo));
            d.hr = std::min(kH, std::max(0, q.interp - 1 - o0 + mhi));
            b->hs[s].halo = d.hl + d.hr;
        }
    }
    b->lds_stats = 2 * (size_t)maxn * sizeof(double);
    HIPCHK(hipMemsetAsync(b->arena, 0, need, b->stream));
    rc = upload_sims(b);
    if (rc) return bail(rc);
    // wake tables from the impedance samples
    for (int s = 0; s < count; ++s) {
        const HostSim &h = b->hs[s];
        if (!b->sd[s].has_wake) continue;
        const int n = h.p.n, M = b->sd[s].M, nz = M / 2 + 1;
        rc = ensure_stage(b, 2 * (size_t)nz);
        if (rc) return bail(rc);
        if (h.p.z_model != VFP_Z_SAMPLES) {
            // Z_k computed on the device at kappa_k = 2 pi k / (M dq)
            const double dq = (h.p.q_max - h.p.q_min) / (n - 1);
            hipLaunchKernelGGL(impedance_kernel, dim3((nz + kThreads - 1) / kThreads), dim3(kThreads), 0, b->stream,
                               nz, 2.0 * M_PI / (M * dq), h.p.z_model, std::pow(h.p.z_shield, 2.0 / 3.0),
                               b->d_stage, b->d_stage + nz);
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(b->arena + h.off_zr, b->d_stage, nz * sizeof(double), hipMemcpyDeviceToDevice,
                               b->stream) != hipSuccess)
                return bail(fail(VFP_EDEVICE, "impedance evaluation failed"));
        } else {
            if (upload(b->d_stage, h.zr.data(), nz * sizeof(double), b->stream) ||
                upload(b->d_stage + nz, h.zi.data(), nz * sizeof(double), b->stream))
                return bail(fail(VFP_EDEVICE, "impedance upload failed"));
            if (upload(b->arena + h.off_zr, h.zr.data(), nz * sizeof(double), b->stream))
                return bail(fail(VFP_EDEVICE, "impedance upload failed"));
        }
        hipLaunchKernelGGL(wake_table_kernel, dim3((2 * n - 1 + kThreads - 1) / kThreads), dim3(kThreads), 0,
                           b->stream, n, M, b->d_stage, b->d_stage + nz, (double *)(b->arena + h.off_wl64),
                           (float *)(b->arena + h.off_wl32));
        if (b->precision >= VFP_MIXED_BF16) {
            // power-of-two scale of the wake fragments from max |w| (device table read back)
            std::vector<double> wl(2 * n - 1);
            if (hipMemcpyAsync(wl.data(), b->arena + h.off_wl64, wl.size() * sizeof(double), hipMemcpyDeviceToHost,
                               b->stream) ||
                hipStreamSynchronize(b->stream))
                return bail(fail(VFP_EDEVICE, "wake table readback failed"));
            double mw = 0.0;
            for (double v : wl) mw = std::max(mw, std::fabs(v));
            int e = 0;
            if (b->precision == VFP_MIXED_FP16 && mw > 0.0) {
                std::frexp(mw, &e);
                e = 14 - e;
            }
            const double wscale = std::ldexp(1.0, e), wback = std::ldexp(1.0, -e);
            const unsigned fb = (unsigned)((wake_rev_len(n) + kThreads - 1) / kThreads);
            if (b->precision == VFP_MIXED_FP16)
                hipLaunchKernelGGL(wake_split_kernel<true>, dim3(fb), dim3(kThreads), 0, b->stream, n,
                                   (const double *)(b->arena + h.off_wl64), wscale, (uint16_t *)(b->arena + h.off_frag));
            else
                hipLaunchKernelGGL(wake_split_kernel<false>, dim3(fb), dim3(kThreads), 0, b->stream, n,
                                   (const double *)(b->arena + h.off_wl64), wscale, (uint16_t *)(b->arena + h.off_frag));
            const double sx[3] = {1.0, 1.0, wback};
            if (upload(b->arena + h.off_sext, sx, sizeof(sx), b->stream))
                return bail(fail(VFP_EDEVICE, "fragment setup failed"));
        }
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(b->stream) != hipSuccess)
            return bail(fail(VFP_EDEVICE, "wake table setup failed"));
    }
    for (int s = 0; s < count; ++s) {
        rc = upload_psi(b, s, p[s].psi0, p[s].psi0 == nullptr);
        if (rc) return bail(rc);
    }
    b->cells = auto_cells(b);
    rc = rebuild(b);
    if (rc) return bail(rc);
    if (hipStreamSynchronize(b->stream) != hipSuccess) return bail(fail(VFP_EDEVICE, "setup failed"));
    *out = b;
    return VFP_OK;
}

const double *stat_ptr(vfp_batch *b, int s) { return (const double *)(b->arena + b->hs[s].off_stat); }

int get_psi_impl(vfp_batch *b, int s, double *psi)
{
    if (!psi) return fail(VFP_EINVAL, "psi is NULL");
    int rc = refresh_stats(b);
    if (rc) return rc;
    const HostSim &h = b->hs[s];
    const size_t nn = (size_t)h.p.n * h.p.n;
    rc = ensure_stage(b, nn);
    if (rc) return rc;
    const int buf = h.active ? b->parity : h.frozen_buf;
    const unsigned blocks = (unsigned)((nn + kThreads - 1) / kThreads);
    const int fixb = b->sd[s].fixb;
    if (b->precision == VFP_FP64)
        hipLaunchKernelGGL(export_kernel<double>, dim3(blocks), dim3(kThreads), 0, b->stream,
                           (const double *)(b->arena + h.off_psi[buf]), stat_ptr(b, s), b->d_stage, nn, fixb);
    else if (b->precision == VFP_FIXED)
        hipLaunchKernelGGL(export_kernel<int64_t>, dim3(blocks), dim3(kThreads), 0, b->stream,
                           (const int64_t *)(b->arena + h.off_psi[buf]), stat_ptr(b, s), b->d_stage, nn, fixb);
    else
        hipLaunchKernelGGL(export_kernel<float>, dim3(blocks), dim3(kThreads), 0, b->stream,
                           (const float *)(b->arena + h.off_psi[buf]), stat_ptr(b, s), b->d_stage, nn, fixb);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(psi, b->d_stage, nn * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return check_finite(b, s);
}

int record_impl(vfp_batch *b, int32_t every, int64_t cap)
{
    if (every < 0 || cap < 0) return fail(VFP_EINVAL, "every and cap must be >= 0");
    HIPCHK(hipStreamSynchronize(b->stream));
    if (b->d_ring) { HIPCHK(hipFree(b->d_ring)); b->d_ring = nullptr; }
    if (b->d_ring_rows) { HIPCHK(hipFree(b->d_ring_rows)); b->d_ring_rows = nullptr; }
    b->every = 0;
    b->rec_cap = 0;
    for (int s = 0; s < b->count; ++s) {
        b->sd[s].ring = nullptr;
        b->sd[s].ring_rows = nullptr;
        b->sd[s].ring_cap = 0;
    }
    if (every > 0 && cap > 0) {
        HIPCHK(hipMalloc(&b->d_ring, sizeof(double) * 7 * (size_t)cap * b->count));
        HIPCHK(hipMalloc(&b->d_ring_rows, sizeof(int64_t) * b->count));
        HIPCHK(hipMemsetAsync(b->d_ring_rows, 0, sizeof(int64_t) * b->count, b->stream));
        for (int s = 0; s < b->count; ++s) {
            b->sd[s].ring = b->d_ring + 7 * (size_t)cap * s;
            b->sd[s].ring_rows = b->d_ring_rows + s;
            b->sd[s].ring_cap = cap;
        }
        b->every = every;
        b->rec_cap = cap;
        b->rec_base = b->tick;
    }
    const int rc = upload_sims(b);
    return rc ? rc : rebuild(b);        // graphs follow the record cadence
}

int read_record_impl(vfp_batch *b, int s, double *out, int64_t *rows)
{
    if (!rows) return fail(VFP_EINVAL, "rows is NULL");
    *rows = 0;
    if (!b->d_ring) return VFP_OK;
    HIPCHK(hipStreamSynchronize(b->stream));
    int64_t r = 0;
    HIPCHK(hipMemcpy(&r, b->d_ring_rows + s, sizeof(int64_t), hipMemcpyDeviceToHost));
    r = std::min(r, b->rec_cap);
    *rows = r;
    if (out && r > 0)
        HIPCHK(hipMemcpy(out, b->d_ring + 7 * (size_t)b->rec_cap * s, sizeof(double) * 7 * r, hipMemcpyDeviceToHost));
    return VFP_OK;
}

// ----------------------------------------------------- impedance sampling
int impedance_args(int32_t model, int32_t n, int32_t padding, double q_min, double q_max, double Pi,
                   const double *z_re, const double *z_im)
{
    if (model != VFP_Z_PARALLEL_PLATES && model != VFP_Z_FREE_SPACE) return fail(VFP_EINVAL, "unknown impedance model");
    if (n < 16 || n > 4096 || padding < 2 || (int64_t)padding * n > (1 << 24))
        return fail(VFP_EINVAL, "need n in [16, 4096] and padding >= 2");
    if (!(q_max > q_min) || !std::isfinite(q_min) || !std::isfinite(q_max))
        return fail(VFP_EINVAL, "need finite q_min < q_max");
    if (model == VFP_Z_PARALLEL_PLATES && !(Pi > 0.0 && std::isfinite(Pi)))
        return fail(VFP_EINVAL, "Pi must be finite and > 0");
    if (!z_re || !z_im) return fail(VFP_EINVAL, "z_re and z_im are required");
    return VFP_OK;
}

// Samples into the device buffer d (2*(M/2+1) doubles: Re then Im) on the
// null stream, then copied to the host arrays; true on success.
bool impedance_on_device(int32_t model, int32_t n, int32_t padding, double q_min, double q_max, double Pi, double *d,
                         double *z_re, double *z_im)
{
    const int M = padding * n, nz = M / 2 + 1;
    const double dq = (q_max - q_min) / (n - 1);
    hipLaunchKernelGGL(impedance_kernel, dim3((nz + kThreads - 1) / kThreads), dim3(kThreads), 0, nullptr, nz,
                       2.0 * M_PI / (M * dq), model, std::pow(Pi, 2.0 / 3.0), d, d + nz);
    return hipGetLastError() == hipSuccess &&
           hipMemcpy(z_re, d, nz * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess &&
           hipMemcpy(z_im, d + nz, nz * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess;
}

// Static scratch of the allocation-free sampler: every device the library
// runs on holds one copy until the process ends.  Host code never passes the
// symbol itself to a kernel or copy (on the host it only names the variable);
// it uses the device address that hipGetSymbolAddress returns for the
// current device, looked up once per device.
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kScratchDevices] = {};

int scratch_on_current_device(double **out)
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchDevices) return fail(VFP_EDEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(VFP_EDEVICE, "no device address for the static scratch");
        g_scratch_ptr[dev] = (double *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return VFP_OK;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

void vfp_params_init(vfp_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->n = 256;
    p->q_min = p->p_min = -8.0;
    p->q_max = p->p_max = 8.0;
    p->steps_per_period = 1000;
    p->beta = 1e-3;
    p->interp = 4;
    p->clamp = 0;
    p->renormalize = 1;
    p->precision = VFP_FP32;
    p->padding = 2;
    p->rotation = VFP_ROT_STANDARD;
    p->z_scale = 0.0;
    p->max_steps = 0;
    p->z_model = VFP_Z_SAMPLES;
    p->z_shield = 1.0;
    p->fix_bits = 44;
}

size_t vfp_params_sizeof(void) { return sizeof(vfp_params); }

int vfp_impedance_samples(int32_t model, int32_t n, int32_t padding, double q_min, double q_max, double Pi,
                          double *z_re, double *z_im)
{
    const int rc = impedance_args(model, n, padding, q_min, q_max, Pi, z_re, z_im);
    if (rc) return rc;
    const int nz = padding * n / 2 + 1;
    double *d = nullptr;
    HIPCHK(hipMalloc(&d, 2 * (size_t)nz * sizeof(double)));
    const bool ok = impedance_on_device(model, n, padding, q_min, q_max, Pi, d, z_re, z_im);
    (void)hipFree(d);
    return ok ? VFP_OK : fail(VFP_EDEVICE, "impedance evaluation failed");
}

int vfp_impedance_samples_noalloc(int32_t model, int32_t n, int32_t padding, double q_min, double q_max, double Pi,
                                  double *z_re, double *z_im)
{
    const int rc = impedance_args(model, n, padding, q_min, q_max, Pi, z_re, z_im);
    if (rc) return rc;
    const int nz = padding * n / 2 + 1;
    if (nz > VFP_NOALLOC_MAX_SAMPLES)
        return fail(VFP_EINVAL, "padding*n/2 + 1 = " + std::to_string(nz) + " samples exceed the static scratch of " +
                                    std::to_string(VFP_NOALLOC_MAX_SAMPLES) + " (use vfp_impedance_samples)");
    double *d = nullptr;
    const int rs = scratch_on_current_device(&d);
    if (rs) return rs;
    return impedance_on_device(model, n, padding, q_min, q_max, Pi, d, z_re, z_im)
               ? VFP_OK
               : fail(VFP_EDEVICE, "impedance evaluation failed");
}

const char *vfp_last_error(void) { return g_err.c_str(); }

int vfp_workspace_size(const vfp_params *p, int32_t count, size_t *bytes)
{
    if (!p || !bytes || count < 1) return fail(VFP_EINVAL, "invalid arguments");
    std::string why;
    for (int s = 0; s < count; ++s) {
        const int rc = validate(p[s], why);
        if (rc) return fail(rc, why);
    }
    *bytes = layout(p, count, nullptr);
    return VFP_OK;
}

int vfp_create(const vfp_params *p, void *hip_stream, void *workspace, size_t ws_bytes, vfp_sim **out)
{
    return create_impl(p, 1, hip_stream, workspace, ws_bytes, true, out);
}

int vfp_batch_create(const vfp_params *p, int32_t count, void *hip_stream, void *workspace, size_t ws_bytes,
                     vfp_batch **out)
{
    return create_impl(p, count, hip_stream, workspace, ws_bytes, false, out);
}

int vfp_step(vfp_sim *sim, int64_t nsteps)
{
    if (!sim) return fail(VFP_EINVAL, "NULL handle");
    return advance(sim, nsteps);
}

int vfp_batch_step(vfp_batch *b, int64_t nticks)
{
    if (!b) return fail(VFP_EINVAL, "NULL handle");
    return advance(b, nticks);
}

int vfp_batch_profile(vfp_batch *b, int32_t i, double *rho)
{
    if (!b || !rho || i < 0 || i >= b->count) return fail(VFP_EINVAL, "invalid arguments");
    int rc = refresh_stats(b);
    if (rc) return rc;
    HIPCHK(hipMemcpy(rho, b->arena + b->hs[i].off_rho, sizeof(double) * b->hs[i].p.n, hipMemcpyDeviceToHost));
    return check_finite(b, i);
}

int vfp_profile(vfp_sim *sim, double *rho) { return vfp_batch_profile(sim, 0, rho); }

int vfp_batch_csr_power(vfp_batch *b, double *power)
{
    if (!b || !power) return fail(VFP_EINVAL, "invalid arguments");
    int rc = refresh_stats(b);
    if (rc) return rc;
    for (int s = 0; s < b->count; ++s) {
        HIPCHK(hipMemcpy(power + s, stat_ptr(b, s) + 5, sizeof(double), hipMemcpyDeviceToHost));
        rc = check_finite(b, s);
        if (rc) return rc;
    }
    return VFP_OK;
}

int vfp_csr_power(vfp_sim *sim, double *power) { return vfp_batch_csr_power(sim, power); }

int vfp_batch_moments(vfp_batch *b, double *out)
{
    if (!b || !out) return fail(VFP_EINVAL, "invalid arguments");
    int rc = refresh_stats(b);
    if (rc) return rc;
    for (int s = 0; s < b->count; ++s) {
        HIPCHK(hipMemcpy(out + 5 * s, stat_ptr(b, s), 5 * sizeof(double), hipMemcpyDeviceToHost));
        rc = check_finite(b, s);
        if (rc) return rc;
    }
    return VFP_OK;
}

int vfp_moments(vfp_sim *sim, double out[5]) { return vfp_batch_moments(sim, out); }

int vfp_batch_get_psi(vfp_batch *b, int32_t i, double *psi)
{
    if (!b || i < 0 || i >= b->count) return fail(VFP_EINVAL, "invalid arguments");
    return get_psi_impl(b, i, psi);
}

int vfp_batch_get_raw(vfp_batch *b, int32_t i, void *out, double *sfac)
{
    if (!b || !out || !sfac || i < 0 || i >= b->count) return fail(VFP_EINVAL, "invalid arguments");
    int rc = refresh_stats(b);
    if (rc) return rc;
    const HostSim &h = b->hs[i];
    const size_t nn = (size_t)h.p.n * h.p.n;
    const int buf = h.active ? b->parity : h.frozen_buf;
    HIPCHK(hipMemcpy(out, b->arena + h.off_psi[buf], nn * elem_size(b->precision), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(sfac, stat_ptr(b, i) + 6, sizeof(double), hipMemcpyDeviceToHost));
    return check_finite(b, i);
}

int vfp_get_psi(vfp_sim *sim, double *psi) { return vfp_batch_get_psi(sim, 0, psi); }

int vfp_batch_set_psi(vfp_batch *b, int32_t i, const double *psi)
{
    if (!b || !psi || i < 0 || i >= b->count) return fail(VFP_EINVAL, "invalid arguments");
    const size_t nn = (size_t)b->hs[i].p.n * b->hs[i].p.n;
    if (const char *e = density_error(psi, nn, b->precision, b->sd[i].fixb)) return fail(VFP_EINVAL, e);
    HIPCHK(hipStreamSynchronize(b->stream));
    const int rc = upload_psi(b, i, psi, false);
    if (rc) return rc;
    b->hs[i].steps = 0;
    if (b->hs[i].p.max_steps > 0 && !b->hs[i].active) {
        b->hs[i].active = true;
        // a revived simulation rejoins at the batch parity
        if (b->hs[i].frozen_buf != b->parity) {
            const size_t es = elem_size(b->precision);
            HIPCHK(hipMemcpyAsync(b->arena + b->hs[i].off_psi[b->parity], b->arena + b->hs[i].off_psi[b->hs[i].frozen_buf],
                                  nn * es, hipMemcpyDeviceToDevice, b->stream));
            HIPCHK(hipMemcpyAsync(b->arena + b->hs[i].off_cs[b->parity], b->arena + b->hs[i].off_cs[b->hs[i].frozen_buf],
                                  cs_bytes(b->precision, b->hs[i].p.n), hipMemcpyDeviceToDevice, b->stream));
            HIPCHK(hipStreamSynchronize(b->stream));
        }
    }
    return rebuild(b);                  // its retirement tick has moved
}

int vfp_set_psi(vfp_sim *sim, const double *psi) { return vfp_batch_set_psi(sim, 0, psi); }

int vfp_batch_record(vfp_batch *b, int32_t every, int64_t cap)
{
    if (!b) return fail(VFP_EINVAL, "NULL handle");
    return record_impl(b, every, cap);
}

int vfp_record(vfp_sim *sim, int32_t every, int64_t cap) { return vfp_batch_record(sim, every, cap); }

int vfp_batch_read_record(vfp_batch *b, int32_t i, double *out, int64_t *rows)
{
    if (!b || i < 0 || i >= b->count) return fail(VFP_EINVAL, "invalid arguments");
    return read_record_impl(b, i, out, rows);
}

int vfp_read_record(vfp_sim *sim, double *out, int64_t *rows) { return vfp_batch_read_record(sim, 0, out, rows); }

int vfp_batch_steps_done(vfp_batch *b, int32_t i, int64_t *steps)
{
    if (!b || !steps || i < 0 || i >= b->count) return fail(VFP_EINVAL, "invalid arguments");
    *steps = b->hs[i].steps;
    return VFP_OK;
}

int vfp_steps_done(vfp_sim *sim, int64_t *steps) { return vfp_batch_steps_done(sim, 0, steps); }

void vfp_batch_destroy(vfp_batch *b) { free_batch(b); }
void vfp_destroy(vfp_sim *sim) { free_batch(sim); }

int vfp_batch_set_tuning(vfp_batch *b, int32_t cells_per_unit, int32_t use_graph, int32_t staged)
{
    if (!b || cells_per_unit < 0) return fail(VFP_EINVAL, "invalid arguments");
    const int cells = cells_per_unit ? cells_per_unit : auto_cells(b);
    if (cells * elem_size(b->precision) * 2 > 128 * 1024)
        return fail(VFP_EINVAL, "cells_per_unit too large for the workgroup's LDS");
    if (cells < 16) return fail(VFP_EINVAL, "cells_per_unit too small");
    if (staged < kStagedGeneric || staged > kStagedFused)
        return fail(VFP_EINVAL, "staged must be 0 (generic kernel), 1 (staged, split tick) or 2 (staged, fused tick)");
    const int cells0 = b->cells, staged0 = b->staged;
    const bool graph0 = b->use_graph;
    b->cells = cells;
    b->use_graph = use_graph != 0;
    b->staged = staged;
    const int rc = rebuild(b);
    if (rc == VFP_OK) return VFP_OK;
    const std::string why = g_err;          // keep the previous tuning
    b->cells = cells0;
    b->use_graph = graph0;
    b->staged = staged0;
    const int rc2 = rebuild(b);
    return rc2 ? rc2 : fail(rc, why);
}

int vfp_batch_set_streams(vfp_batch *b, int32_t groups)
{
    if (!b || groups < 1 || groups > kMaxGroups) return fail(VFP_EINVAL, "groups must be in [1, 4]");
    const int lanes0 = b->lanes;
    b->lanes = groups;
    const int rc = rebuild(b);
    if (rc) b->lanes = lanes0;
    return rc;
}

int vfp_batch_get_tuning(vfp_batch *b, int32_t *cells_per_unit, int32_t *use_graph, int32_t *staged)
{
    if (!b) return fail(VFP_EINVAL, "invalid arguments");
    if (cells_per_unit) *cells_per_unit = b->cells;
    if (use_graph) *use_graph = b->use_graph ? 1 : 0;
    if (staged) *staged = b->staged;
    return VFP_OK;
}

int vfp_batch_csr_spectrum(vfp_batch *b, int32_t i, double *out)
{
    if (!b || !out || i < 0 || i >= b->count) return fail(VFP_EINVAL, "invalid arguments");
    if (!b->sd[i].has_wake) return fail(VFP_ESTATE, "simulation has no impedance");
    int rc = refresh_stats(b);
    if (rc) return rc;
    const int nk = b->sd[i].M / 2 + 1;
    rc = ensure_stage(b, nk);
    if (rc) return rc;
    hipLaunchKernelGGL(spectrum_kernel, dim3((unsigned)((b->sd[i].M / 2 + kThreads) / kThreads)), dim3(kThreads), 0,
                       b->stream, b->d_sd, i, b->d_stage);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(out, b->d_stage, nk * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return check_finite(b, i);
}

int vfp_csr_spectrum(vfp_sim *sim, double *out) { return vfp_batch_csr_spectrum(sim, 0, out); }

int vfp_batch_haissinski(vfp_batch *b, int32_t i, int32_t iters, double alpha)
{
    if (!b || i < 0 || i >= b->count || iters < 0 || !(alpha > 0.0 && alpha <= 1.0))
        return fail(VFP_EINVAL, "invalid arguments");
    HIPCHK(hipStreamSynchronize(b->stream));
    HostSim &h = b->hs[i];
    h.active = true;                    // a retired simulation rejoins at the batch parity
    const int buf = b->parity, n = h.p.n;
    const int v[2] = {i, buf};
    int rc = upload(b->d_idx, v, sizeof(v), b->stream);
    if (rc) return rc;
    if (b->precision == VFP_FP64) rc = launch_haissinski<double>(b, i, buf, iters, alpha);
    else if (b->precision == VFP_FIXED) rc = launch_haissinski<int64_t>(b, i, buf, iters, alpha);
    else rc = launch_haissinski<float>(b, i, buf, iters, alpha);
    if (rc) return rc;
    rc = launch_project(b, n, buf);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(b->stream));
    b->sd[i].step0 = b->tick;
    h.steps = 0;
    rc = upload_sims(b);
    return rc ? rc : rebuild(b);
}

int vfp_haissinski(vfp_sim *sim, int32_t iters, double alpha) { return vfp_batch_haissinski(sim, 0, iters, alpha); }

int vfp_batch_seed(vfp_batch *b, int32_t dst, int32_t src)
{
    if (!b || dst < 0 || src < 0 || dst >= b->count || src >= b->count || dst == src)
        return fail(VFP_EINVAL, "invalid arguments");
    const vfp_params &a = b->hs[dst].p, &c = b->hs[src].p;
    if (a.n != c.n || a.q_min != c.q_min || a.q_max != c.q_max || a.p_min != c.p_min || a.p_max != c.p_max)
        return fail(VFP_EINVAL, "seeding needs the same grid");
    if (b->sd[dst].fixb != b->sd[src].fixb) return fail(VFP_EINVAL, "seeding needs the same fix_bits");
    HIPCHK(hipStreamSynchronize(b->stream));
    HostSim &hd = b->hs[dst];
    const HostSim &hsrc = b->hs[src];
    hd.active = true;                         // a retired simulation rejoins at the batch parity
    const int bs = hsrc.active ? b->parity : hsrc.frozen_buf;
    const int bd = b->parity;
    const size_t nn = (size_t)a.n * a.n, es = elem_size(b->precision);
    HIPCHK(hipMemcpyAsync(b->arena + hd.off_psi[bd], b->arena + hsrc.off_psi[bs], nn * es, hipMemcpyDeviceToDevice,
                          b->stream));
    HIPCHK(hipMemcpyAsync(b->arena + hd.off_cs[bd], b->arena + hsrc.off_cs[bs], cs_bytes(b->precision, a.n),
                          hipMemcpyDeviceToDevice, b->stream));
    // the copied density is the source's stored one: its physical state is s*psi^ with the
    // source's Q0, which the destination takes over
    b->sd[dst].Q0 = b->sd[src].Q0;
    b->sd[dst].step0 = b->tick;
    hd.steps = 0;
    const int rc = upload_sims(b);
    return rc ? rc : rebuild(b);
}

int vfp_batch_last_wake(vfp_batch *b, int32_t i, double *V)
{
    if (!b || !V || i < 0 || i >= b->count) return fail(VFP_EINVAL, "invalid arguments");
    if (!b->sd[i].has_wake) return fail(VFP_ESTATE, "simulation has no impedance");
    HIPCHK(hipStreamSynchronize(b->stream));
    // the latest step read the buffer opposite to the one now holding the state
    const HostSim &h = b->hs[i];
    const int prev = (h.active ? b->parity : h.frozen_buf) ^ 1;
    std::vector<float> v(h.p.n);
    HIPCHK(hipMemcpy(v.data(), b->arena + h.off_vext + (size_t)prev * h.p.n * sizeof(float), v.size() * sizeof(float),
                     hipMemcpyDeviceToHost));
    for (size_t k = 0; k < v.size(); ++k) V[k] = v[k];
    return VFP_OK;
}

int vfp_batch_kernel_timing(vfp_batch *b, int32_t enable)
{
    if (!b) return fail(VFP_EINVAL, "NULL handle");
    HIPCHK(hipStreamSynchronize(b->stream));
    for (hipEvent_t e : b->ev_pool) HIPCHK(hipEventDestroy(e));
    b->ev_pool.clear();
    b->ev_used = 0;
    b->ev_step.clear();
    b->ev_wake.clear();
    b->timing = enable != 0;
    if (b->timing) {
        b->ev_pool.resize(kTimingEvents);
        for (hipEvent_t &e : b->ev_pool) HIPCHK(hipEventCreate(&e));
    }
    return rebuild(b);                  // no graphs while timing
}

int vfp_batch_kernel_times(vfp_batch *b, double out[4])
{
    if (!b || !out) return fail(VFP_EINVAL, "invalid arguments");
    HIPCHK(hipStreamSynchronize(b->stream));
    double st = 0.0, wk = 0.0;
    for (const auto &pr : b->ev_step) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, b->ev_pool[pr.first], b->ev_pool[pr.second]));
        st += ms;
    }
    for (const auto &pr : b->ev_wake) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, b->ev_pool[pr.first], b->ev_pool[pr.second]));
        wk += ms;
    }
    out[0] = st;
    out[1] = (double)b->ev_step.size();
    out[2] = wk;
    out[3] = (double)b->ev_wake.size();
    return VFP_OK;
}

int vfp_batch_autotune(vfp_batch *b, int32_t ticks, int32_t *chosen_cells, int32_t *chosen_staged)
{
    if (!b || ticks < 1) return fail(VFP_EINVAL, "invalid arguments");
    HIPCHK(hipStreamSynchronize(b->stream));
    // save the state of every simulation (both buffers and column sums)
    std::vector<std::vector<unsigned char>> save(b->count);
    const size_t es = elem_size(b->precision);
    for (int s = 0; s < b->count; ++s) {
        const HostSim &h = b->hs[s];
        const size_t nn = (size_t)h.p.n * h.p.n;
        const size_t cb = cs_bytes(b->precision, h.p.n);
        save[s].resize(2 * nn * es + 2 * cb);
        HIPCHK(hipMemcpy(save[s].data(), b->arena + h.off_psi[0], nn * es, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(save[s].data() + nn * es, b->arena + h.off_psi[1], nn * es, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(save[s].data() + 2 * nn * es, b->arena + h.off_cs[0], cb, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(save[s].data() + 2 * nn * es + cb, b->arena + h.off_cs[1], cb, hipMemcpyDeviceToHost));
    }
    const int64_t tick0 = b->tick;
    const int parity0 = b->parity, every0 = b->every, staged0 = b->staged, cells0 = b->cells;
    const bool timing0 = b->timing, graph0 = b->use_graph;
    b->every = 0;                   // no records, graphs or event timing during the trials
    b->timing = false;
    b->use_graph = false;
    const std::vector<int> layouts = is_fp32_storage(b->precision) ? std::vector<int>{kStagedSplit, kStagedFused}
                                                                    : std::vector<int>{kStagedGeneric};
    const std::vector<int> cand = es == 8 ? std::vector<int>{1024, 2048, 4096, 8192}
                                          : std::vector<int>{2048, 4096, 8192, 16384};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    float best = 1e30f;
    int best_c = cells0, best_l = staged0;
    int rc = VFP_OK;
    for (int layout : layouts) {
        for (int c : cand) {
            b->cells = c;
            b->staged = layout;
            rc = rebuild(b);                // drains the previous candidate's ticks first
            if (rc == VFP_EINVAL) { rc = VFP_OK; continue; }   // does not fit the LDS
            if (rc) break;
            // trial ticks of the first phase (the whole batch), warm-up then timed;
            // a phase shorter than the trial is stepped past its end: only the time counts
            const Phase &ph = b->phases[0];
            if (ph.active.empty()) break;
            for (int t = 0; t < 2 + ticks && rc == VFP_OK; ++t) {
                if (t == 2) {
                    rc = join_streams(b);
                    if (rc == VFP_OK && hipEventRecord(e0, b->stream) != hipSuccess)
                        rc = fail(VFP_EDEVICE, "autotune event failed");
                }
                if (rc == VFP_OK) rc = enqueue_tick(b, ph, b->parity, b->tick);
                b->parity ^= 1;
            }
            if (rc == VFP_OK) rc = join_streams(b);
            if (rc) break;
            HIPCHK(hipEventRecord(e1, b->stream));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) { best = ms; best_c = c; best_l = layout; }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    {
        const int jrc = join_streams(b);
        if (rc == VFP_OK) rc = jrc;
    }
    HIPCHK(hipStreamSynchronize(b->stream));
    for (int g = 0; g < kMaxGroups - 1; ++g)
        if (b->xstream[g]) HIPCHK(hipStreamSynchronize(b->xstream[g]));
    for (int s = 0; s < b->count; ++s) {
        const HostSim &h = b->hs[s];
        const size_t nn = (size_t)h.p.n * h.p.n;
        const size_t cb = cs_bytes(b->precision, h.p.n);
        HIPCHK(hipMemcpyAsync(b->arena + h.off_psi[0], save[s].data(), nn * es, hipMemcpyHostToDevice, b->stream));
        HIPCHK(hipMemcpyAsync(b->arena + h.off_psi[1], save[s].data() + nn * es, nn * es, hipMemcpyHostToDevice,
                              b->stream));
        HIPCHK(hipMemcpyAsync(b->arena + h.off_cs[0], save[s].data() + 2 * nn * es, cb, hipMemcpyHostToDevice,
                              b->stream));
        HIPCHK(hipMemcpyAsync(b->arena + h.off_cs[1], save[s].data() + 2 * nn * es + cb, cb, hipMemcpyHostToDevice,
                              b->stream));
    }
    HIPCHK(hipStreamSynchronize(b->stream));
    b->tick = tick0;
    b->parity = parity0;
    b->every = every0;
    b->timing = timing0;
    b->use_graph = graph0;
    b->cells = rc ? cells0 : best_c;
    b->staged = rc ? staged0 : best_l;
    const int rc2 = rebuild(b);         // the chosen tuning; the wake is recomputed from the restored state
    if (rc) return rc;
    if (rc2) return rc2;
    if (chosen_cells) *chosen_cells = best_c;
    if (chosen_staged) *chosen_staged = best_l;
    return VFP_OK;
}

int vfp_device_arch(char *name, int32_t len)
{
    if (!name || len < 1) return fail(VFP_EINVAL, "invalid arguments");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    std::snprintf(name, (size_t)len, "%s", prop.gcnArchName);
    return VFP_OK;
}

}  // extern "C"
