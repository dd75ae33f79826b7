// qnsch_lib.hip -- host driver of the FP64 multigrid time step behind the C
// ABI of include/qnsch.h: per-simulation contexts, the operation programme of
// a time step, and a continuous-batching server that runs many simulations
// through the same work-list kernels.
//
// One step (sec. 6.1 solved as in sec. 7.1): fix the time-n data on every
// level, then run FAS V-cycles (red-black CH point Newton + Vanka box
// smoothing, residual restriction, coarse-grid correction) until every
// per-equation residual norm is below tol.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "qnsch.h"
#include "qnsch_mxk.hpp"

using namespace qn;

// ===========================================================================
// operations of a time step

enum OpKind { OP_BEGIN, OP_RN, OP_NORM0, OP_NORM, OP_HS, OP_RESTRICT, OP_COARSE, OP_PROLONG, OP_STEPEND,
              OP_RESTORE,
              // mixed precision: FP32 correction cycle, FP64 update
              OP_MXRN, OP_MXHS, OP_MXRESTRICT, OP_MXCOARSE, OP_MXPROLONG, OP_MXUPDATE,
              // diagnostics of the current state
              OP_DISSIP, OP_DIAG, OP_PJFINAL,
              // colour field = number of sweeps: all sweeps of a small level
              // in one workgroup with the level resident in LDS
              OP_SMOOTH, OP_MXSMOOTH,
              // acceleration of the cycle iteration: residual norms that also
              // record the result, and the combination before the next cycle
              OP_NORMACC, OP_ACCEL,
              // one red + black sweep of a level in one launch (temporal
              // blocking); colour field = direction of the cell sets
              OP_FUSED, OP_MXFUSED, NOPS };
struct Op {
    int kind, level, colour;
};
// timing tags: operation * PROF_LEVELS + level
#define PROF_LEVELS 16
static bool is_smoother_op(int kind) { return kind == OP_HS || kind == OP_MXHS || kind == OP_FUSED || kind == OP_MXFUSED; }
// operations that launch one kernel (timed by the kernel's own timestamps);
// the reductions launch two or three
static bool single_kernel_op(int kind)
{
    return !(kind == OP_NORM0 || kind == OP_NORM || kind == OP_NORMACC || kind == OP_STEPEND || kind == OP_DISSIP
             || kind == OP_DIAG);
}

// nu sweeps of level l: one launch per colour half-sweep, or, on a coarse
// level that fits in LDS (l >= small), all of them in one workgroup, or, on a
// level marked in fuse, one launch per sweep (an even number of them, so that
// the cell unknowns end in the set they started in; an odd last sweep takes
// two half-sweeps), all with the same arithmetic in the same order
static void smooth_ops(int l, int nu, int small, int hs_kind, int lds_kind, unsigned fuse, std::vector<Op> &out)
{
    const int fused_kind = hs_kind == OP_MXHS ? OP_MXFUSED : OP_FUSED;
    if (nu <= 0) return;
    if (l > 0 && l >= small) {
        out.push_back({ lds_kind, l, nu });
        return;
    }
    int s = 0;
    if ((fuse >> l) & 1)
        for (; s + 1 < nu; s += 2) {
            out.push_back({ fused_kind, l, 0 });
            out.push_back({ fused_kind, l, 1 });
        }
    for (; s < nu; s++) {
        out.push_back({ hs_kind, l, 0 });
        out.push_back({ hs_kind, l, 1 });
    }
}
// prolongation onto level l, then its post-smoothing; a level-resident
// smoothing takes the correction as it loads the level (colour field
// nu + PROLONG_FIRST), and so does the first fused sweep of an FP64 level
// (colour field 2 + direction 0), which saves the prolongation launch
#define PROLONG_FIRST 16
#define FUSED_PROLONG 2
static void prolong_smooth_ops(int l, int nu, int small, int pr_kind, int hs_kind, int lds_kind, unsigned fuse,
                               std::vector<Op> &out)
{
    if (nu > 0 && nu < PROLONG_FIRST && l > 0 && l >= small) {
        out.push_back({ lds_kind, l, nu + PROLONG_FIRST });
        return;
    }
    if (pr_kind == OP_PROLONG && nu >= 2 && !(l > 0 && l >= small) && ((fuse >> l) & 1)) {
        const size_t first = out.size();
        smooth_ops(l, nu, small, hs_kind, lds_kind, fuse, out);
        out[first].colour |= FUSED_PROLONG;
        return;
    }
    out.push_back({ pr_kind, l, 0 });
    smooth_ops(l, nu, small, hs_kind, lds_kind, fuse, out);
}

// one V-cycle of a hierarchy of L levels, ending with the residual norms and
// the pbar mean removal
static void vcycle_program(int L, int nu1, int nu2, int small, unsigned fuse, bool acc, std::vector<Op> &out)
{
    for (int l = 0; l + 1 < L; l++) {
        smooth_ops(l, nu1, small, OP_HS, OP_SMOOTH, fuse, out);
        out.push_back({ OP_RESTRICT, l, 0 }); // with the coarse FAS right-hand side
    }
    out.push_back({ OP_COARSE, L - 1, 0 });
    for (int l = L - 2; l >= 0; l--) prolong_smooth_ops(l, nu2, small, OP_PROLONG, OP_HS, OP_SMOOTH, fuse, out);
    out.push_back({ acc ? OP_NORMACC : OP_NORM, 0, 0 });
}
// one outer iteration of the mixed-precision step: an FP32 correction
// V-cycle on J(w^) delta = r, w += delta in FP64, then the FP64 residual
// (which also prepares the next cycle) and the pbar mean removal
static void mixed_program(int L, int nu1, int nu2, int small, unsigned fuse, bool acc, std::vector<Op> &out)
{
    for (int l = 0; l + 1 < L; l++) {
        smooth_ops(l, nu1, small, OP_MXHS, OP_MXSMOOTH, fuse, out);
        out.push_back({ OP_MXRESTRICT, l, 0 });
    }
    out.push_back({ OP_MXCOARSE, L - 1, 0 });
    for (int l = L - 2; l >= 0; l--)
        prolong_smooth_ops(l, nu2, small, OP_MXPROLONG, OP_MXHS, OP_MXSMOOTH, fuse, out);
    out.push_back({ OP_MXUPDATE, 0, 0 });
    out.push_back({ acc ? OP_NORMACC : OP_NORM, 0, 0 });
}
// time-n data of every level, then the residual of the initial iterate
static void begin_program(int L, bool mixed, std::vector<Op> &out)
{
    out.push_back({ OP_BEGIN, 0, 0 });
    for (int l = 0; l + 1 < L; l++) out.push_back({ mixed ? OP_MXRN : OP_RN, l, 0 });
    out.push_back({ OP_NORM0, 0, 0 });
}

// ===========================================================================
// contexts

namespace {
// device memory of contexts: hipMalloc / hipFree, or the functions set by
// qnsch_set_allocator (taken by a context when it is created; it frees with
// the functions it allocated with)
struct Allocator {
    qnsch_alloc_fn alloc = nullptr;
    qnsch_free_fn free = nullptr;
    void *user = nullptr;
};
std::mutex g_alloc_mu;
Allocator g_alloc;

struct DLev {
    int m1 = 0, m2 = 0, pitch = 0;
    double h = 0;
    int cur = 0; // current u/v buffer
    size_t n() const { return (size_t)pitch * m2; }
};
} // namespace

struct qnsch_ctx {
    qnsch_grid g;
    qnsch_params prm;
    qnsch_opts opt;
    int nlev = 0;
    DLev L[16];
    Desc *hd = nullptr;   // pinned host copy of the level descriptors
    Desc *dd = nullptr;   // device descriptors
    hipStream_t s = nullptr;
    Allocator al;                                    // device memory functions of this context
    std::vector<std::pair<void *, size_t>> allocs;   // device blocks and their sizes
    double *red_host = nullptr; // pinned
    double *stage = nullptr;    // pinned staging for state transfers (server contexts)
    void *arena = nullptr;      // the device arrays (one allocation)
    size_t arena_bytes = 0;
    hipEvent_t ev = nullptr;    // completion of the last host-read reduction
    size_t footprint = 0;
    std::string err;
    // launch timing with HIP events on the context's stream (qnsch_profile,
    // qnsch_profile_ops): mode 1 the launches of the operations in prof_mask
    // (on the finest level only if prof_fine_only), carrying the events
    // themselves (the kernel's own start and end; event records around the
    // operations that launch several kernels), mode 2 every launch between
    // event records; accumulated per (operation, level)
    int prof = 0, prof_used = 0;
    uint64_t prof_mask = 0;
    bool prof_fine_only = false;
    std::vector<hipEvent_t> pev;
    std::vector<int> ptag;
    double prof_ms = 0.0;
    long prof_n = 0;
    double tag_ms[NOPS * PROF_LEVELS] = {};
    long tag_n[NOPS * PROF_LEVELS] = {};
    int in_step = 0;
    double dt = 0;
    qnsch_step_stats st;
    // dissipation of the last step in st: 0 no completed step since the
    // state was set, 1 a completed step whose dissipation was not asked for
    // yet, 2 in st (qnsch_dissipation keeps it there)
    int diss_state = 0;
    size_t lds_max = 65536; // LDS a level-resident workgroup may use on this device
    int ncu = 256;          // compute units of the device
    // acceleration of the cycle iteration (opt.accel = m > 0): ring of m + 1
    // recorded results on the device
    int acc_pos = 0;      // slot of the latest recorded result
    int acc_cnt = 0;      // results in the current history, the latest included
    int acc_dots = 0;     // earlier results the latest one's reduction paired it with
    int acc_use = 0;      // earlier results the pending combination uses (0: none pending)
    bool acc_wait = false;  // a recording reduction is in flight
    bool acc_first = true;  // the next cycle is the first of its step (not recorded)
    double acc_g[3] = { 0.0, 0.0, 0.0 };
    double acc_last = 0.0;  // largest residual norm of the latest result
    // replay of a cycle's operations before its residual reduction as one
    // executable graph (qnsch_graphs; off by default).  One graph per pattern
    // of the levels' current face buffers (bit l = L[l].cur) the cycle
    // starts from; every cycle toggles each level's buffer an even number of
    // times, so the pattern after the cycle is the one it started from.
    // Captured on a stream of the context's own (the caller's stream may be
    // the null stream, which cannot capture) and launched on the caller's.
    bool graphs = false;
    hipStream_t cap = nullptr;
    std::vector<std::pair<unsigned, hipGraphExec_t>> cyc_graphs;
};

static bool is_mixed(const qnsch_ctx *x) { return x->opt.precision == QNSCH_MIXED; }
static void step_begin_program(const qnsch_ctx *x, std::vector<Op> &out) { begin_program(x->nlev, is_mixed(x), out); }
// first level from which every coarser level fits in LDS for the
// level-resident smoothing (nlev if none); lds_max is set at context creation
static int small_level(const qnsch_ctx *x)
{
    int small = x->nlev;
    for (int l = x->nlev - 1; l >= 1; l--) {
        const int m1 = x->L[l].m1, m2 = x->L[l].m2;
        const size_t b = is_mixed(x) ? mx_coarse_lds_floats(m1, m2) * sizeof(float)
                                     : coarse_lds_doubles(m1, m2) * sizeof(double);
        if (b > x->lds_max) break;
        small = l;
    }
    return small;
}
// whether the opts give the levels a second set of cell unknowns (FP64) or
// cell corrections (mixed precision)
static bool two_sets(const qnsch_opts &o) { return o.blocking > 0; }
// levels whose sweeps run fused (bit l): those smoothed by half-sweep
// launches (below small) with a periodic axis at least TX + 3 (TY + 3) cells
// long (the widened tile wraps once) and few enough tiles: coarse levels with
// at most two tiles per compute unit; the finest level with at most one
// (blocking 1), or two (blocking 2).  A fused sweep pays for its redundant red
// work (200 red cells per tile instead of 128, with the workgroup's LDS tile
// widened) with a launch less, which is worth it only where a launch's fixed
// cost is as large as its relaxation.  Measured on one MI355X (alternating
// settings on one box): fusing the finest level too, 32 x 64 capillary (8
// tiles) 0.326-0.329 against 0.340-0.341 ms per step, 64 x 128 droplet (32
// tiles) 1.354-1.357 against 1.389-1.392, 128 x 256 (128 tiles) 1.901
// against 1.965-1.966, but 256 x 512 (512 tiles, two per CU) 2.716-2.722
// against 2.652-2.656 ms and 512 x 2048 (4096 tiles) 17 % slower.
static unsigned fused_levels(const qnsch_ctx *x)
{
    if (!two_sets(x->opt)) return 0u;
    unsigned m = 0;
    const int small = small_level(x);
    for (int l = 0; l < small && l < x->nlev; l++) {
        const DLev &D = x->L[l];
        if ((x->g.bc_x == QNSCH_BC_PERIODIC && D.m1 < TX + 3) || (x->g.bc_y == QNSCH_BC_PERIODIC && D.m2 < TY + 3))
            continue;
        const int tiles = ((D.m1 + TX - 1) / TX) * ((D.m2 + TY - 1) / TY);
        if (tiles > (l > 0 || x->opt.blocking >= 2 ? 2 : 1) * x->ncu) continue;
        m |= 1u << l;
    }
    return m;
}
// one cycle; with acceleration its residual reduction records the result,
// from the second cycle of a step on (acc_record_launch skips the first: its
// residual direction is dominated by the change of the time-n data; leaving
// it out costs no cycle on the droplet, Rayleigh-Taylor and drop-box
// workloads and saves its recording).  Every cycle has the same operations,
// so served requests at different cycles of their steps share launches.
static void cycle_program(const qnsch_ctx *x, std::vector<Op> &out)
{
    const bool rec = x->opt.accel > 0;
    if (is_mixed(x)) mixed_program(x->nlev, x->opt.nu1, x->opt.nu2, small_level(x), fused_levels(x), rec, out);
    else vcycle_program(x->nlev, x->opt.nu1, x->opt.nu2, small_level(x), fused_levels(x), rec, out);
}

#define HIPCHK(ctx, x)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) {                                                               \
            (ctx)->err = std::string(#x) + ": " + hipGetErrorString(e_);                      \
            return QNSCH_EDEVICE;                                                             \
        }                                                                                     \
    } while (0)

static unsigned nblocks(size_t n) { return (unsigned)((n + BLK - 1) / BLK); }
static int tiles_x(int m1) { return (m1 + TX - 1) / TX; }
static int tiles_y(int m2) { return (m2 + TY - 1) / TY; }

// ---------------------------------------------------------------------------
// work lists

struct ItemList {
    Items it;
    int blocks = 0;
    size_t lds = 0;
    bool all_fine = true;
    ItemList() { memset(&it, 0, sizeof(it)); }
};

// workgroups of an operation on (context, level)
static int op_blocks(const qnsch_ctx *x, int kind, int l)
{
    const DLev &D = x->L[l];
    switch (kind) {
    case OP_HS: case OP_RESTRICT: case OP_NORM: case OP_NORM0: case OP_NORMACC: case OP_MXHS:
    case OP_MXRESTRICT: case OP_FUSED: case OP_MXFUSED:
        return tiles_x(D.m1) * tiles_y(D.m2);
    case OP_COARSE: case OP_MXCOARSE: case OP_SMOOTH: case OP_MXSMOOTH: return 1;
    case OP_RN: case OP_MXRN: return (int)nblocks((size_t)x->L[l + 1].m1 * x->L[l + 1].m2);
    default: return (int)nblocks((size_t)D.m1 * D.m2);
    }
}

static void add_item(ItemList &W, const qnsch_ctx *x, int kind, int l)
{
    Items &it = W.it;
    const int start = ((W.blocks + NXCD - 1) / NXCD) * NXCD;
    const int k = it.n;
    it.start[k] = start;
    it.d[k] = x->dd + l;
    it.par[k] = x->L[l].cur;
    it.cpar[k] = l + 1 < x->nlev ? x->L[l + 1].cur : 0;
    it.tx[k] = tiles_x(x->L[l].m1);
    it.acc[k] = -1;
    W.blocks = start + op_blocks(x, kind, l);
    it.n = k + 1;
    it.start[k + 1] = W.blocks;
    if (l != 0) W.all_fine = false;
    if (kind == OP_COARSE || kind == OP_SMOOTH)
        W.lds = std::max(W.lds, coarse_lds_doubles(x->L[l].m1, x->L[l].m2) * sizeof(double));
    if (kind == OP_MXCOARSE || kind == OP_MXSMOOTH)
        W.lds = std::max(W.lds, mx_coarse_lds_floats(x->L[l].m1, x->L[l].m2) * sizeof(float));
}

// finalize list: one workgroup per simulation, tx = number of partials
static ItemList finalize_list(const std::vector<std::pair<qnsch_ctx *, int>> &v, int partial_kind)
{
    ItemList F;
    for (auto &e : v) {
        qnsch_ctx *x = e.first;
        const int k = F.it.n;
        F.it.d[k] = x->dd;
        F.it.par[k] = x->L[0].cur;
        F.it.tx[k] = op_blocks(x, partial_kind, 0);
        F.it.acc[k] = -1;
        F.it.start[k] = k;
        F.it.n = k + 1;
        F.it.start[k + 1] = k + 1;
    }
    F.blocks = F.it.n;
    return F;
}

static int prof_collect(qnsch_ctx *x)
{
    for (int q = 0; q < x->prof_used; q++) {
        float ms = 0.f;
        HIPCHK(x, hipEventElapsedTime(&ms, x->pev[2 * q], x->pev[2 * q + 1]));
        const int tag = x->ptag[q];
        if (is_smoother_op(tag / PROF_LEVELS) && tag % PROF_LEVELS == 0) {
            x->prof_ms += ms;
            x->prof_n++;
        }
        x->tag_ms[tag] += ms;
        x->tag_n[tag]++;
    }
    x->prof_used = 0;
    return QNSCH_OK;
}

// timing tag of a launch (-1: not timed)
static int prof_tag(int kind, const std::vector<std::pair<qnsch_ctx *, int>> &part)
{
    const qnsch_ctx *x = part[0].first;
    const int l = part[0].second;
    if (part.size() != 1 || !x->prof || l >= PROF_LEVELS) return -1;
    if (x->prof == 1 && (!((x->prof_mask >> kind) & 1u) || (x->prof_fine_only && l != 0))) return -1;
    return kind * PROF_LEVELS + l;
}

// timed launches whose events are kept before they are read back
#define PROF_POOL 4096
static int prof_grow(qnsch_ctx *x, int launches)
{
    for (int q = 0; q < 2 * launches; q++) {
        hipEvent_t ev;
        HIPCHK(x, hipEventCreateWithFlags(&ev, hipEventDisableSystemFence));
        x->pev.push_back(ev);
    }
    return QNSCH_OK;
}

static int prof_mark(qnsch_ctx *x, hipStream_t s, int tag, bool end, bool stamped = false)
{
    if (!end) {
        // the pool is read back only when it is full (or the counters are
        // read): a full pool waits for its last launch once
        if ((size_t)(2 * x->prof_used + 2) > x->pev.size()) {
            if (x->pev.size() >= 2 * PROF_POOL) {
                HIPCHK(x, hipStreamSynchronize(s));
                int rc;
                if ((rc = prof_collect(x))) return rc;
            } else {
                int rc;
                if ((rc = prof_grow(x, 64))) return rc;
            }
        }
        if ((size_t)x->prof_used + 1 > x->ptag.size()) x->ptag.resize(x->prof_used + 64);
        x->ptag[x->prof_used] = tag;
        // a launch that carries the events itself records nothing here
        if (!stamped) HIPCHK(x, hipEventRecord(x->pev[2 * x->prof_used], s));
    } else {
        if (!stamped) HIPCHK(x, hipEventRecord(x->pev[2 * x->prof_used + 1], s));
        x->prof_used++;
    }
    return QNSCH_OK;
}

// ---------------------------------------------------------------------------
// acceleration of the cycle iteration (host side)

// a recording residual reduction is being launched: the result goes to the
// next ring slot, paired with up to m earlier results of the history
static void acc_record_launch(qnsch_ctx *x, int &acc)
{
    if (x->acc_first) {
        x->acc_first = false;
        acc = -1;
        x->acc_use = 0;
        return;
    }
    const int m = x->opt.accel, R = m + 1;
    x->acc_pos = (x->acc_pos + 1) % R;
    x->acc_dots = std::min(x->acc_cnt, m);
    acc = x->acc_pos | (x->acc_dots << 4);
    x->acc_wait = true;
    x->acc_use = 0;
}

// Normal equations H g = -b of the combination (H packed by columns in
// v[0..5], b in v[6..8]) over the n earlier results the newest one was paired
// with (the most recent first), solved by Cholesky; the leading block whose
// pivots exceed 1e-12 times their diagonal entry is used.  Returns the number
// of coefficients (the rest are 0).
static int acc_solve(const double *v, int n, double g[3])
{
    auto H = [&](int i, int j) { return i <= j ? v[j * (j + 1) / 2 + i] : v[i * (i + 1) / 2 + j]; };
    double Lf[3][3] = {};
    int use = 0;
    for (int c = 0; c < n; c++) {
        double dg = H(c, c);
        for (int k = 0; k < c; k++) dg -= Lf[c][k] * Lf[c][k];
        if (!(dg > 1e-12 * H(c, c)) || !std::isfinite(dg)) break;
        Lf[c][c] = sqrt(dg);
        for (int r = c + 1; r < n; r++) {
            double a = H(c, r);
            for (int k = 0; k < c; k++) a -= Lf[r][k] * Lf[c][k];
            Lf[r][c] = a / Lf[c][c];
        }
        use = c + 1;
    }
    double y[3] = { 0.0, 0.0, 0.0 };
    for (int i = 0; i < use; i++) {
        double a = -v[6 + i];
        for (int k = 0; k < i; k++) a -= Lf[i][k] * y[k];
        y[i] = a / Lf[i][i];
    }
    for (int b = 0; b < 3; b++) g[b] = 0.0;
    for (int i = use - 1; i >= 0; i--) {
        double a = y[i];
        for (int k = i + 1; k < use; k++) a -= Lf[k][i] * g[k];
        g[i] = a / Lf[i][i];
    }
    return use;
}

// after a recording reduction (norms and normal equations in red_host): the
// coefficients of the next combination.  A result whose largest norm does
// not improve on the previous one starts a new history.
static void acc_after(qnsch_ctx *x)
{
    x->acc_wait = false;
    double mx = 0.0;
    for (int q = 0; q < 5; q++) mx = std::max(mx, x->red_host[q]);
    int n = x->acc_dots;
    if (n > 0 && !(mx < x->acc_last)) n = 0;
    x->acc_use = n > 0 ? acc_solve(x->red_host + 7, n, x->acc_g) : 0;
    if (x->acc_use == 0)
        for (int b = 0; b < 3; b++) x->acc_g[b] = 0.0;
    x->acc_cnt = n + 1;
    x->acc_last = mx;
}

static void acc_reset(qnsch_ctx *x)
{
    x->acc_cnt = 0;
    x->acc_dots = 0;
    x->acc_use = 0;
    x->acc_wait = false;
    x->acc_last = 0.0;
    x->acc_first = true;
}

// a work list of one item in its compact form
static Item1 one_of(const Items &a)
{
    Item1 b;
    memset(&b, 0, sizeof(b));
    b.n = 1;
    b.start[0] = a.start[0];
    b.start[1] = a.start[1];
    b.d[0] = a.d[0];
    b.par[0] = a.par[0];
    b.cpar[0] = a.cpar[0];
    b.tx[0] = a.tx[0];
    b.acc[0] = a.acc[0];
    return b;
}
// launch kernel template K on list L (ItemList): the one-item instantiation
// when the list has a single item; a timed launch (e0 set in the calling
// scope) carries the events that take the kernel's own start and end
#define KLAUNCH(K, L, GRID, BLOCK, LDS, ST, ...)                                                     \
    do {                                                                                           \
        if (e0) {                                                                                  \
            if ((L).it.n == 1)                                                                     \
                hipExtLaunchKernelGGL(K<Item1>, GRID, BLOCK, LDS, ST, e0, e1, 0, one_of((L).it), ##__VA_ARGS__); \
            else hipExtLaunchKernelGGL(K<Items>, GRID, BLOCK, LDS, ST, e0, e1, 0, (L).it, ##__VA_ARGS__); \
        } else if ((L).it.n == 1)                                                                  \
            hipLaunchKernelGGL(K<Item1>, GRID, BLOCK, LDS, ST, one_of((L).it), ##__VA_ARGS__);     \
        else hipLaunchKernelGGL(K<Items>, GRID, BLOCK, LDS, ST, (L).it, ##__VA_ARGS__);            \
    } while (0)

// Launch one operation for a set of (context, level) entries, in lists of at
// most MAXITEMS; all entries share the kind and colour.  Errors are reported
// on the first context.
static int launch_op(int kind, int colour, const std::vector<std::pair<qnsch_ctx *, int>> &v, hipStream_t s)
{
    if (v.empty()) return QNSCH_OK;
    qnsch_ctx *x0 = v[0].first;
    for (size_t b = 0; b < v.size(); b += MAXITEMS) {
        const size_t e = std::min(v.size(), b + MAXITEMS);
        std::vector<std::pair<qnsch_ctx *, int>> part(v.begin() + b, v.begin() + e);
        ItemList W;
        for (auto &pe : part) add_item(W, pe.first, kind, pe.second);
        const double omega = x0->opt.vanka_omega;
        const int tag = prof_tag(kind, part);
        // launches timed in mode 1 take the kernel's own start and end
        // timestamps; other timed launches are bracketed by event records
        const bool stamp = tag >= 0 && single_kernel_op(kind) && part[0].first->prof == 1;
        int rc;
        if (tag >= 0 && (rc = prof_mark(part[0].first, s, tag, false, stamp))) return rc;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (stamp) {
            qnsch_ctx *x = part[0].first;
            e0 = x->pev[2 * x->prof_used];
            e1 = x->pev[2 * x->prof_used + 1];
        }
        switch (kind) {
        case OP_HS:
        case OP_MXHS: {
            const dim3 gr(W.blocks), bl(TBLK);
            if (kind == OP_MXHS) {
                if (W.all_fine)
                    KLAUNCH(k_mx_halfsweep_fine, W, gr, bl, 0, s, colour, (float)omega);
                else KLAUNCH(k_mx_halfsweep, W, gr, bl, 0, s, colour, (float)omega);
            } else if (W.all_fine) {
                KLAUNCH(k_halfsweep_fine, W, gr, bl, 0, s, colour, omega);
            } else {
                KLAUNCH(k_halfsweep, W, gr, bl, 0, s, colour, omega);
            }
            for (auto &pe : part) pe.first->L[pe.second].cur ^= 1;
            break;
        }
        case OP_FUSED: {
            KLAUNCH(k_hs_fused, W, dim3(W.blocks), dim3(FBLK), 0, s, colour & 1, omega, colour >> 1);
            for (auto &pe : part) pe.first->L[pe.second].cur ^= 1;
            break;
        }
        case OP_MXFUSED: {
            KLAUNCH(k_mx_fused, W, dim3(W.blocks), dim3(FBLK), 0, s, colour, (float)omega);
            for (auto &pe : part) pe.first->L[pe.second].cur ^= 1;
            break;
        }
        case OP_RESTRICT: KLAUNCH(k_restrict, W, dim3(W.blocks), dim3(RBLK), 0, s); break;
        case OP_COARSE:
        case OP_SMOOTH: {
            int nmax = 0;
            for (auto &pe : part) nmax = std::max(nmax, pe.first->L[pe.second].m1 * pe.first->L[pe.second].m2 / 2);
            const unsigned th = (unsigned)(2 * nmax < 512 ? ((2 * nmax + 63) / 64) * 64 : 512);
            // the coarsest level over-relaxes the velocity and pressure
            // updates (the primitive box, the projection pressure step)
            const bool coarsest = kind == OP_COARSE, pj = x0->opt.scheme == QNSCH_PROJECTION;
            const int sweeps = coarsest ? x0->opt.nu_coarse : colour % PROLONG_FIRST;
            const int prolong = coarsest ? 0 : colour / PROLONG_FIRST;
            const double om = coarsest && !pj ? x0->opt.coarse_omega : omega;
            const double pom = coarsest && pj ? x0->opt.coarse_omega : 1.0;
            KLAUNCH(k_coarse_solve, W, dim3(W.blocks), dim3(th), W.lds, s, sweeps, om, pom, prolong);
            break;
        }
        case OP_PROLONG: KLAUNCH(k_prolong, W, dim3(W.blocks), dim3(BLK), 0, s); break;
        case OP_MXRESTRICT: KLAUNCH(k_mx_restrict, W, dim3(W.blocks), dim3(TBLK), 0, s); break;
        case OP_MXCOARSE:
        case OP_MXSMOOTH: {
            int nmax = 0;
            for (auto &pe : part) nmax = std::max(nmax, pe.first->L[pe.second].m1 * pe.first->L[pe.second].m2 / 2);
            const unsigned th = (unsigned)(2 * nmax < 512 ? ((2 * nmax + 63) / 64) * 64 : 512);
            const bool coarsest = kind == OP_MXCOARSE;
            const int sweeps = coarsest ? x0->opt.nu_coarse : colour % PROLONG_FIRST;
            const int prolong = coarsest ? 0 : colour / PROLONG_FIRST;
            const double om = coarsest ? x0->opt.coarse_omega : omega;
            KLAUNCH(k_mx_coarse_solve, W, dim3(W.blocks), dim3(th), W.lds, s, sweeps, (float)om, prolong);
            break;
        }
        case OP_MXPROLONG: KLAUNCH(k_mx_prolong, W, dim3(W.blocks), dim3(BLK), 0, s); break;
        case OP_MXUPDATE: KLAUNCH(k_mx_update, W, dim3(W.blocks), dim3(BLK), 0, s); break;
        case OP_MXRN: KLAUNCH(k_mx_restrict_n, W, dim3(W.blocks), dim3(BLK), 0, s); break;
        case OP_BEGIN: KLAUNCH(k_begin, W, dim3(W.blocks), dim3(BLK), 0, s); break;
        case OP_RN: KLAUNCH(k_restrict_n, W, dim3(W.blocks), dim3(BLK), 0, s); break;
        case OP_RESTORE: KLAUNCH(k_restore, W, dim3(W.blocks), dim3(BLK), 0, s); break;
        case OP_NORM0:
        case OP_NORM:
        case OP_NORMACC: {
            if (kind == OP_NORMACC)
                for (size_t q = 0; q < part.size(); q++) acc_record_launch(part[q].first, W.it.acc[q]);
            KLAUNCH(k_resid_norm, W, dim3(W.blocks), dim3(TBLK), 0, s);
            ItemList F = finalize_list(part, OP_NORM);
            for (size_t q = 0; q < part.size(); q++) F.it.acc[q] = W.it.acc[q];
            KLAUNCH(k_finalize, F, dim3(F.blocks), dim3(BLK), 0, s, 0);
            if (kind != OP_NORM0) {
                ItemList S;
                for (auto &pe : part) add_item(S, pe.first, OP_BEGIN, 0);
                KLAUNCH(k_shift_p, S, dim3(S.blocks), dim3(BLK), 0, s);
            }
            break;
        }
        case OP_STEPEND: {
            KLAUNCH(k_mass_energy, W, dim3(W.blocks), dim3(BLK), 0, s);
            ItemList F = finalize_list(part, OP_STEPEND);
            KLAUNCH(k_finalize, F, dim3(F.blocks), dim3(BLK), 0, s, 1);
            break;
        }
        case OP_DISSIP: {
            KLAUNCH(k_dissipation, W, dim3(W.blocks), dim3(BLK), 0, s);
            ItemList F = finalize_list(part, OP_DISSIP);
            KLAUNCH(k_finalize, F, dim3(F.blocks), dim3(BLK), 0, s, 1);
            break;
        }
        case OP_ACCEL: {
            AccCoef<MAXITEMS> G;
            memset(&G, 0, sizeof(G));
            for (size_t q = 0; q < part.size(); q++) {
                qnsch_ctx *x = part[q].first;
                W.it.acc[q] = x->acc_pos | (x->acc_use << 4);
                for (int b = 0; b < 3; b++) G.g[q][b] = x->acc_g[b];
                x->acc_use = 0;
            }
            if (W.it.n == 1) {
                AccCoef<1> G1;
                for (int b = 0; b < 3; b++) G1.g[0][b] = G.g[0][b];
                if (e0) hipExtLaunchKernelGGL((k_accel<Item1, 1>), dim3(W.blocks), dim3(BLK), 0, s, e0, e1, 0, one_of(W.it), G1);
                else hipLaunchKernelGGL((k_accel<Item1, 1>), dim3(W.blocks), dim3(BLK), 0, s, one_of(W.it), G1);
            } else if (e0) {
                hipExtLaunchKernelGGL((k_accel<Items, MAXITEMS>), dim3(W.blocks), dim3(BLK), 0, s, e0, e1, 0, W.it, G);
            } else {
                hipLaunchKernelGGL((k_accel<Items, MAXITEMS>), dim3(W.blocks), dim3(BLK), 0, s, W.it, G);
            }
            break;
        }
        case OP_PJFINAL: {
            KLAUNCH(k_pj_final, W, dim3(W.blocks), dim3(BLK), 0, s);
            for (auto &pe : part) pe.first->L[0].cur ^= 1;
            break;
        }
        case OP_DIAG: {
            KLAUNCH(k_diagnostics, W, dim3(W.blocks), dim3(BLK), 0, s);
            ItemList F = finalize_list(part, OP_DIAG);
            KLAUNCH(k_finalize, F, dim3(F.blocks), dim3(BLK), 0, s, 2);
            break;
        }
        default: break;
        }
        if (tag >= 0 && (rc = prof_mark(part[0].first, s, tag, true, stamp))) return rc;
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) {
            x0->err = std::string("kernel launch: ") + hipGetErrorString(err);
            return QNSCH_EDEVICE;
        }
    }
    return QNSCH_OK;
}

// run a sequence of operations on one context
static int run_ops(qnsch_ctx *x, const std::vector<Op> &prog)
{
    std::vector<std::pair<qnsch_ctx *, int>> v(1);
    for (const Op &o : prog) {
        v[0] = { x, o.level };
        int rc = launch_op(o.kind, o.colour, v, x->s);
        if (rc) return rc;
    }
    return QNSCH_OK;
}

// pattern of the levels' current face buffers
static unsigned cur_key(const qnsch_ctx *x)
{
    unsigned k = 0;
    for (int l = 0; l < x->nlev; l++) k |= (unsigned)(x->L[l].cur & 1) << l;
    return k;
}

// the operations of a cycle before its residual reduction: launched one by
// one while launches are timed or graphs are off, else as the replay of the
// graph captured for the current buffer pattern (captured on first use)
static int run_body(qnsch_ctx *x, const std::vector<Op> &body)
{
    if (!x->graphs || x->prof) return run_ops(x, body);
    const unsigned key = cur_key(x);
    hipGraphExec_t ge = nullptr;
    for (auto &c : x->cyc_graphs)
        if (c.first == key) ge = c.second;
    if (!ge) {
        if (!x->cap) HIPCHK(x, hipStreamCreateWithFlags(&x->cap, hipStreamNonBlocking));
        HIPCHK(x, hipStreamBeginCapture(x->cap, hipStreamCaptureModeThreadLocal));
        const hipStream_t s = x->s;
        x->s = x->cap;
        const int rc = run_ops(x, body);
        x->s = s;
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(x->cap, &g);
        if (rc || e != hipSuccess || !g || cur_key(x) != key) {
            if (g) (void)hipGraphDestroy(g);
            for (int l = 0; l < x->nlev; l++) x->L[l].cur = (int)((key >> l) & 1);
            if (rc) return rc;
            x->err = e != hipSuccess ? std::string("hipStreamEndCapture: ") + hipGetErrorString(e)
                                     : std::string("cycle capture: the levels' buffer pattern changed");
            return QNSCH_EDEVICE;
        }
        const hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(x, ei);
        x->cyc_graphs.push_back({ key, ge });
    }
    HIPCHK(x, hipGraphLaunch(ge, x->s));
    return QNSCH_OK;
}

// one cycle: the pending combination of the acceleration, the operations of
// the cycle programme cyc before its residual reduction, the reduction
static int run_cycle(qnsch_ctx *x, const std::vector<Op> &cyc, const std::vector<Op> &body)
{
    int rc;
    if (x->acc_use > 0 && (rc = run_ops(x, { { OP_ACCEL, 0, 0 } }))) return rc;
    if ((rc = run_body(x, body))) return rc;
    return run_ops(x, { cyc.back() });
}

// wait for the context's stream (the reduced values are then in red_host).
// The host polls the completion of an event for a while before blocking: a
// step waits here once per V-cycle, and a blocking wait wakes up tens of
// microseconds late, during which the device has nothing queued.
static int read_red(qnsch_ctx *x)
{
    HIPCHK(x, hipEventRecord(x->ev, x->s));
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const hipError_t q = hipEventQuery(x->ev);
        if (q == hipSuccess) break;
        if (q != hipErrorNotReady) HIPCHK(x, q);
        if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(50)) {
            HIPCHK(x, hipEventSynchronize(x->ev));
            break;
        }
    }
    return QNSCH_OK;
}

// a device block of the context (256-byte aligned), or nullptr with the
// message in x->err
static void *dev_alloc(qnsch_ctx *x, size_t bytes)
{
    void *p = nullptr;
    if (x->al.alloc) {
        p = x->al.alloc(bytes, x->al.user);
        if (p && ((uintptr_t)p & 255)) {
            x->al.free(p, bytes, x->al.user);
            x->err = "allocator returned memory not aligned to 256 bytes";
            return nullptr;
        }
        if (!p) x->err = "allocator returned NULL";
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        x->err = "hipMalloc failed";
        p = nullptr;
    }
    if (p) x->allocs.push_back({ p, bytes });
    return p;
}

static double *dalloc(qnsch_ctx *x, size_t n, int *rc)
{
    void *p = dev_alloc(x, n * sizeof(double));
    if (!p) {
        *rc = QNSCH_ENOMEM;
        return nullptr;
    }
    x->footprint += n * sizeof(double);
    if (hipMemsetAsync(p, 0, n * sizeof(double), x->s) != hipSuccess) *rc = QNSCH_EDEVICE;
    return (double *)p;
}

// level count of a grid (0 = automatic) or -1 if invalid
static int level_count(const qnsch_grid *g)
{
    int nl = g->levels;
    if (nl <= 0) {
        // coarsen while the coarsest level has more than 32 cells and the next
        // one keeps even dimensions: the coarsest solve is a fixed number of
        // sweeps, which converge on a few dozen cells but not on an elongated
        // grid of 64 or more
        nl = 1;
        while (nl < 16 && g->m1 % (1 << (nl + 1)) == 0 && g->m2 % (1 << (nl + 1)) == 0
               && (g->m1 >> (nl - 1)) * (g->m2 >> (nl - 1)) > 32)
            nl++;
    }
    if (nl > 16 || g->m1 % (1 << nl) != 0 || g->m2 % (1 << nl) != 0) return -1;
    if (coarse_lds_doubles(g->m1 >> (nl - 1), g->m2 >> (nl - 1)) * sizeof(double) > 65536) return -1;
    return nl;
}

// The device arrays of a context live in one allocation, carved here: with
// base == nullptr only the size is computed (the footprint), otherwise the
// level descriptors get their pointers.  FP64 mode: the FP64 state, time-n
// data and FAS arrays on every level.  Mixed mode: the FP64 state and time-n
// data on the finest level only (one u/v buffer, both slots aliased) and the
// FP32 correction hierarchy on every level.
static size_t carve(const qnsch_grid *g, int nl, bool mixed, int accel, bool two, char *base, Desc *hd)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> void * {
        void *p = base ? (void *)(base + off) : nullptr;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    auto dbl = [&](size_t n) { return (double *)take(n * sizeof(double)); };
    auto flt = [&](size_t n) { return (float *)take(n * sizeof(float)); };
    Desc scratch;
    for (int l = 0; l < nl; l++) {
        const size_t n = (size_t)(g->m1 >> l) * (g->m2 >> l);
        Desc &d = hd ? hd[l] : scratch;
        if (!mixed || l == 0) {
            d.c = dbl(n); d.mu = dbl(n); d.p = dbl(n);
            d.ub[0] = dbl(n); d.vb[0] = dbl(n);
            if (mixed) { d.ub[1] = d.ub[0]; d.vb[1] = d.vb[0]; }
            else { d.ub[1] = dbl(n); d.vb[1] = dbl(n); }
            d.cn = dbl(n); d.un = dbl(n); d.vn = dbl(n);
        }
        if (two && !mixed) { d.c2 = dbl(n); d.mu2 = dbl(n); d.p2 = dbl(n); }
        if (two && mixed) { d.dc2 = flt(n); d.dmu2 = flt(n); d.dp2 = flt(n); }
        if (!mixed && l > 0) {
            d.fc = dbl(n); d.fmu = dbl(n); d.fp = dbl(n); d.fu = dbl(n); d.fv = dbl(n);
            d.c0 = dbl(n); d.mu0 = dbl(n); d.p0 = dbl(n); d.u0 = dbl(n); d.v0 = dbl(n);
        }
        if (mixed) {
            d.xc = flt(n); d.xmu = flt(n); d.xu = flt(n); d.xv = flt(n);
            d.dc = flt(n); d.dmu = flt(n); d.dp = flt(n);
            d.dub[0] = flt(n); d.dub[1] = flt(n); d.dvb[0] = flt(n); d.dvb[1] = flt(n);
            d.rc = flt(n); d.rmu = flt(n); d.rp = flt(n); d.ru = flt(n); d.rv = flt(n);
            d.cnf = flt(n); d.unf = flt(n); d.vnf = flt(n);
        }
    }
    const size_t n0 = (size_t)g->m1 * g->m2;
    Desc &d0 = hd ? hd[0] : scratch;
    d0.mus = dbl(n0);
    d0.ps = dbl(n0);
    d0.partials = dbl((size_t)std::max(tiles_x(g->m1) * tiles_y(g->m2), (int)nblocks(n0)) * NRED);
    d0.red = dbl(NRED);
    if (accel > 0) {
        d0.am = accel + 1;
        d0.aw = dbl((size_t)5 * d0.am * n0);
        d0.ar = dbl((size_t)5 * d0.am * n0);
        d0.amean = dbl((size_t)d0.am);
    }
    return off;
}

// device bytes of a context (the allocations of qnsch_create)
static size_t footprint_of(const qnsch_grid *g, const qnsch_opts &o)
{
    const int nl = level_count(g);
    if (nl < 0) return 0;
    return carve(g, nl, o.precision == QNSCH_MIXED, o.accel, two_sets(o), nullptr, nullptr) + (size_t)nl * sizeof(Desc);
}

static void phys_of(const qnsch_params *p, Phys &P)
{
    P.rho1 = p->rho1; P.rho2 = p->rho2; P.rho12 = p->rho1 * p->rho2; P.drho = p->rho2 - p->rho1;
    P.visc1 = p->visc1; P.visc2 = p->visc2; P.visc12 = p->visc1 * p->visc2; P.dvisc = p->visc2 - p->visc1;
    P.alpha = (p->rho2 - p->rho1) / (p->rho1 * p->rho2);
    P.inv_Re = 1.0 / p->Re; P.inv_M = 1.0 / p->M; P.inv_Pe = 1.0 / p->Pe;
    P.K1 = p->M * p->eta / (p->eps * p->We);
    P.K2 = p->eps * p->eta * p->M / (2.0 * p->We);
    P.K3 = p->eps * p->eta * p->M / p->We;
    P.inv_Fr = p->inv_Fr; P.rho_ref = p->rho_ref; P.mob_reg = p->mob_reg;
    P.inv_dt = 0.0;
    P.dt = 0.0;
    P.coupled = 1;
    P.scheme = 0;
}

static PhysF physf_of(const Phys &P)
{
    PhysF F;
    F.rho1 = (float)P.rho1; F.rho12 = (float)P.rho12; F.drho = (float)P.drho;
    F.visc1 = (float)P.visc1; F.visc12 = (float)P.visc12; F.dvisc = (float)P.dvisc;
    F.alpha = (float)P.alpha; F.inv_Re = (float)P.inv_Re; F.inv_M = (float)P.inv_M; F.inv_Pe = (float)P.inv_Pe;
    F.K1 = (float)P.K1; F.K2 = (float)P.K2; F.K3 = (float)P.K3; F.mob_reg = (float)P.mob_reg;
    F.inv_dt = 0.0f;
    F.coupled = P.coupled;
    return F;
}

static int upload_desc(qnsch_ctx *x)
{
    HIPCHK(x, hipMemcpyAsync(x->dd, x->hd, x->nlev * sizeof(Desc), hipMemcpyHostToDevice, x->s));
    return QNSCH_OK;
}

// ===========================================================================
// C ABI

extern "C" {

void qnsch_default_opts(qnsch_opts *o)
{
    o->precision = QNSCH_FP64;
    o->tol = 1e-10;
    o->max_vcycles = 50;
    o->nu1 = 2;
    o->nu2 = 2;
    o->nu_coarse = 0;
    o->vanka_omega = 1.0;
    o->smoother = QNSCH_SMOOTH_COUPLED;
    o->scheme = QNSCH_PRIMITIVE;
    o->coarse_omega = 0.0;
    o->accel = 2;
    o->blocking = 1;
}

const char *qnsch_last_error(const qnsch_ctx *x) { return x ? x->err.c_str() : "null context"; }
int qnsch_levels(const qnsch_ctx *x) { return x ? x->nlev : 0; }

void qnsch_destroy(qnsch_ctx *x)
{
    if (!x) return;
    (void)hipStreamSynchronize(x->s);
    for (auto &a : x->allocs) {
        if (x->al.free) x->al.free(a.first, a.second, x->al.user);
        else (void)hipFree(a.first);
    }
    for (hipEvent_t e : x->pev) (void)hipEventDestroy(e);
    if (x->ev) (void)hipEventDestroy(x->ev);
    for (auto &c : x->cyc_graphs) (void)hipGraphExecDestroy(c.second);
    if (x->cap) (void)hipStreamDestroy(x->cap);
    if (x->red_host) (void)hipHostFree(x->red_host);
    if (x->stage) (void)hipHostFree(x->stage);
    if (x->hd) (void)hipHostFree(x->hd);
    delete x;
}

// the finest grid alone (even dimensions of at least 4, square cells,
// boundary kinds) and the physical parameters
static int validate_grid_params(const qnsch_grid *g, const qnsch_params *p)
{
    if (!g || !p) return QNSCH_EINVAL;
    if (g->m1 < 4 || g->m2 < 4 || (g->m1 & 1) || (g->m2 & 1)) return QNSCH_EINVAL;
    if (!(g->Lx > 0) || !(g->Ly > 0)) return QNSCH_EINVAL;
    const double hx = g->Lx / g->m1, hy = g->Ly / g->m2;
    if (fabs(hx - hy) > 1e-12 * hx) return QNSCH_EINVAL;
    if ((g->bc_x != 0 && g->bc_x != 1) || (g->bc_y != 0 && g->bc_y != 1)) return QNSCH_EINVAL;
    if (!(p->rho1 > 0) || !(p->rho2 > 0) || !(p->visc1 > 0) || !(p->visc2 > 0) || !(p->Re > 0) || !(p->We > 0)
        || !(p->Pe > 0) || !(p->M > 0) || !(p->eps > 0) || std::isnan(p->eta) || std::isnan(p->mob_reg))
        return QNSCH_EINVAL;
    return QNSCH_OK;
}

// the parameters with their defaults filled in: eta <= 0 takes the interface
// ratio of sec. 8.1 for the density pair, mob_reg < 0 takes eps (the constant
// under the square root of the mobility in sec. 6.1)
static qnsch_params resolve_params(const qnsch_params &p)
{
    qnsch_params q = p;
    if (!(q.eta > 0)) q.eta = qnsch_default_eta(q.rho1, q.rho2);
    if (q.mob_reg < 0) q.mob_reg = q.eps;
    return q;
}

static int validate(const qnsch_grid *g, const qnsch_params *p, const qnsch_opts *o)
{
    if (validate_grid_params(g, p)) return QNSCH_EINVAL;
    if (o && (o->nu1 < 0 || o->nu2 < 0 || o->nu1 >= PROLONG_FIRST || o->nu2 >= PROLONG_FIRST || o->nu_coarse < 0
              || o->max_vcycles < 0
              || (o->precision != QNSCH_FP64 && o->precision != QNSCH_MIXED)
              || (o->smoother != QNSCH_SMOOTH_SEGREGATED && o->smoother != QNSCH_SMOOTH_COUPLED)
              || (o->scheme != QNSCH_PRIMITIVE && o->scheme != QNSCH_PROJECTION)
              || (o->scheme == QNSCH_PROJECTION && o->precision != QNSCH_FP64)
              || !(o->coarse_omega == 0.0 || (o->coarse_omega > 0.0 && o->coarse_omega < 2.0)) || !(o->vanka_omega > 0.0 && o->vanka_omega < 2.0)
              || o->accel < 0 || o->accel > 3 || o->blocking < 0 || o->blocking > 2))
        return QNSCH_EINVAL;
    if (level_count(g) < 0) return QNSCH_EINVAL;
    return QNSCH_OK;
}

// the coarsest solve's automatic settings (0 in the options) for a
// hierarchy of nlev levels: 4 sweeps over-relaxed by 1.75 for the primitive
// scheme on hierarchies of 6 levels or more, else 6 sweeps by 1.6.
// Measured on one MI355X (V-cycles per step and step time over the droplet,
// Rayleigh-Taylor, capillary, Cauchy-study and drop-box workloads, tol 1e-8
// and 1e-10): on deep hierarchies 4 x 1.75 takes as many or fewer cycles
// and shorter steps; on 4- and 5-level ones (a coarsest level that is a
// larger share of the grid) it costs cycles, and the projection scheme
// needs the 6 sweeps everywhere.
static void resolve_opts(qnsch_opts &o, int nlev)
{
    const bool deep = o.scheme == QNSCH_PRIMITIVE && nlev >= 6;
    if (o.nu_coarse == 0) o.nu_coarse = deep ? 4 : 6;
    if (o.coarse_omega == 0.0) o.coarse_omega = deep ? 1.75 : 1.6;
}

// physical parameters of every level descriptor (host copy)
static void set_params(qnsch_ctx *x, const qnsch_params *p)
{
    x->prm = resolve_params(*p);
    Phys P;
    phys_of(&x->prm, P);
    P.coupled = x->opt.smoother == QNSCH_SMOOTH_COUPLED;
    P.scheme = x->opt.scheme == QNSCH_PROJECTION;
    const PhysF Pf = physf_of(P);
    for (int l = 0; l < x->nlev; l++) {
        x->hd[l].P = P;
        x->hd[l].Pf = Pf;
    }
}

// Allocate and lay out a context (validated arguments); the device arrays
// are cleared on the stream; the descriptors are not uploaded yet.
// LDS one workgroup may allocate on the current device (160 KiB on gfx950),
// with the level-resident kernels allowed to use it; 64 KiB if the device
// does not report more or the attribute cannot be set.  Once per device.
static size_t device_lds_max()
{
    static size_t cache[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536;
    if (cache[dev]) return cache[dev];
    int v = 0;
    size_t r = 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 65536
        && hipFuncSetAttribute((const void *)k_coarse_solve<Items>, hipFuncAttributeMaxDynamicSharedMemorySize, v) == hipSuccess
        && hipFuncSetAttribute((const void *)k_coarse_solve<Item1>, hipFuncAttributeMaxDynamicSharedMemorySize, v) == hipSuccess
        && hipFuncSetAttribute((const void *)k_mx_coarse_solve<Items>, hipFuncAttributeMaxDynamicSharedMemorySize, v)
               == hipSuccess
        && hipFuncSetAttribute((const void *)k_mx_coarse_solve<Item1>, hipFuncAttributeMaxDynamicSharedMemorySize, v)
               == hipSuccess)
        r = (size_t)v;
    (void)hipGetLastError();
    cache[dev] = r;
    return r;
}

// the workgroup size as block_threads() reads it, written by the first thread
// of a one-workgroup launch of BLK threads, for group_size_check below
static __device__ int g_group_size;
__global__ __launch_bounds__(BLK) void k_group_size_check()
{
    if (threadIdx.x == 0) g_group_size = block_threads();
}

// The kernels read their workgroup size from a fixed place of the dispatch's
// implicit kernel arguments (block_threads: code object versions 5 and 6); a
// build for another layout must not run.  One check per device, before the
// first kernel there: QNSCH_OK, or QNSCH_EDEVICE with the reason in err.
static int group_size_check(std::string &err)
{
    static std::mutex mu;
    static int state[64] = {}; // 0 unchecked, 1 passed, -1 failed
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        err = "no current HIP device";
        return QNSCH_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (state[dev] == 0) {
        hipLaunchKernelGGL(k_group_size_check, dim3(1), dim3(BLK), 0, nullptr);
        int h = 0;
        const hipError_t e = hipMemcpyFromSymbol(&h, HIP_SYMBOL(g_group_size), sizeof(h));
        state[dev] = (e == hipSuccess && h == BLK) ? 1 : -1;
        if (state[dev] < 0) {
            char b[160];
            snprintf(b, sizeof(b), "workgroup size check: %d read from the dispatch for %d threads (%s)", h, BLK,
                     hipGetErrorString(e));
            err = b;
        }
    }
    if (state[dev] < 0 && err.empty()) err = "workgroup size check failed on this device";
    return state[dev] > 0 ? QNSCH_OK : QNSCH_EDEVICE;
}

static int ctx_init(qnsch_ctx *x, const qnsch_grid *g, const qnsch_params *p, const qnsch_opts *o, void *stream)
{
    int rc = QNSCH_OK;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        x->al = g_alloc;
    }
    x->g = *g;
    x->nlev = level_count(g);
    x->g.levels = x->nlev;
    x->prm = resolve_params(*p);
    qnsch_default_opts(&x->opt);
    if (o) x->opt = *o;
    resolve_opts(x->opt, x->nlev);
    x->lds_max = device_lds_max();
    if ((rc = group_size_check(x->err))) {
        fprintf(stderr, "qnsch: %s\n", x->err.c_str());
        return rc;
    }
    {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess
            && v > 0)
            x->ncu = v;
    }
    x->s = (hipStream_t)stream;
    memset(&x->st, 0, sizeof(x->st));
    const double hx = g->Lx / g->m1;
    if (hipHostMalloc((void **)&x->hd, x->nlev * sizeof(Desc), hipHostMallocDefault) != hipSuccess
        || hipHostMalloc((void **)&x->red_host, 16 * sizeof(double), hipHostMallocDefault) != hipSuccess)
        return QNSCH_ENOMEM;
    memset((void *)x->hd, 0, x->nlev * sizeof(Desc));
    memset(x->red_host, 0, 16 * sizeof(double));
    void *ddp = dev_alloc(x, x->nlev * sizeof(Desc));
    if (!ddp) return QNSCH_ENOMEM;
    x->dd = (Desc *)ddp;
    const bool mixed = is_mixed(x);
    const size_t bytes = carve(g, x->nlev, mixed, x->opt.accel, two_sets(x->opt), nullptr, nullptr);
    void *arena = dev_alloc(x, bytes);
    if (!arena) return QNSCH_ENOMEM;
    x->arena = arena;
    x->arena_bytes = bytes;
    x->footprint = bytes + (size_t)x->nlev * sizeof(Desc);
    if (hipMemsetAsync(arena, 0, bytes, x->s) != hipSuccess) rc = QNSCH_EDEVICE;
    carve(g, x->nlev, mixed, x->opt.accel, two_sets(x->opt), (char *)arena, x->hd);
    for (int l = 0; l < x->nlev; l++) {
        DLev &D = x->L[l];
        D.m1 = g->m1 >> l;
        D.m2 = g->m2 >> l;
        D.pitch = D.m1;
        D.h = hx * (double)(1 << l);
        Desc &d = x->hd[l];
        d.m1 = D.m1; d.m2 = D.m2; d.pitch = D.pitch; d.bcx = g->bc_x; d.bcy = g->bc_y;
        d.h = D.h; d.inv_h = 1.0 / D.h; d.finv_h = (float)d.inv_h;
        d.coarse = l + 1 < x->nlev ? x->dd + l + 1 : nullptr;
    }
    set_params(x, p);
    x->hd[0].red_host = x->red_host;
    x->hd[0].rout = nullptr;
    if (!rc && hipEventCreateWithFlags(&x->ev, hipEventDisableTiming) != hipSuccess) rc = QNSCH_EDEVICE;
    return rc;
}

int qnsch_create(const qnsch_grid *g, const qnsch_params *p, const qnsch_opts *o, void *stream, qnsch_ctx **out)
{
    if (!out) return QNSCH_EINVAL;
    *out = nullptr;
    int rc = validate(g, p, o);
    if (rc) return rc;
    qnsch_ctx *x = new qnsch_ctx();
    rc = ctx_init(x, g, p, o, stream);
    if (!rc) rc = upload_desc(x);
    if (!rc && hipStreamSynchronize(x->s) != hipSuccess) rc = QNSCH_EDEVICE;
    if (rc) {
        qnsch_destroy(x);
        return rc;
    }
    *out = x;
    return QNSCH_OK;
}

// host (m1*m2, packed) <-> device (pitch) copies
static int put(qnsch_ctx *x, double *dst, const double *src)
{
    DLev &D = x->L[0];
    HIPCHK(x, hipMemcpy2DAsync(dst, D.pitch * sizeof(double), src, D.m1 * sizeof(double), D.m1 * sizeof(double), D.m2,
                               hipMemcpyHostToDevice, x->s));
    return QNSCH_OK;
}
static int get(qnsch_ctx *x, double *dst, const double *src)
{
    DLev &D = x->L[0];
    HIPCHK(x, hipMemcpy2DAsync(dst, D.m1 * sizeof(double), src, D.pitch * sizeof(double), D.m1 * sizeof(double), D.m2,
                               hipMemcpyDeviceToHost, x->s));
    return QNSCH_OK;
}

static int upload(qnsch_ctx *x, const double *c, const double *mu, const double *p, const double *u, const double *v)
{
    DLev &D = x->L[0];
    Desc &d = x->hd[0];
    const size_t n = (size_t)D.m1 * D.m2;
    std::vector<double> z(n, 0.0), uu(n, 0.0), vv(n, 0.0);
    if (u) memcpy(uu.data(), u, n * sizeof(double));
    if (v) memcpy(vv.data(), v, n * sizeof(double));
    if (x->g.bc_x == QNSCH_BC_WALL)
        for (int j = 0; j < D.m2; j++) uu[(size_t)j * D.m1] = 0.0;
    if (x->g.bc_y == QNSCH_BC_WALL)
        for (int i = 0; i < D.m1; i++) vv[i] = 0.0;
    int rc;
    if ((rc = put(x, d.c, c))) return rc;
    if ((rc = put(x, d.mu, mu ? mu : z.data()))) return rc;
    if ((rc = put(x, d.p, p ? p : z.data()))) return rc;
    if ((rc = put(x, d.ub[D.cur], uu.data()))) return rc;
    if ((rc = put(x, d.vb[D.cur], vv.data()))) return rc;
    HIPCHK(x, hipStreamSynchronize(x->s));
    return QNSCH_OK;
}

int qnsch_set_state(qnsch_ctx *x, const double *c, const double *mu, const double *p, const double *u, const double *v)
{
    if (!x || !c) return QNSCH_EINVAL;
    int rc = upload(x, c, mu, p, u, v);
    x->in_step = 0;
    x->diss_state = 0;
    return rc;
}

int qnsch_set_iterate(qnsch_ctx *x, const double *c, const double *mu, const double *p, const double *u,
                      const double *v)
{
    if (!x || !c) return QNSCH_EINVAL;
    if (!x->in_step) { x->err = "set_iterate outside a step"; return QNSCH_EBUSY; }
    x->diss_state = 0;
    return upload(x, c, mu, p, u, v);
}

int qnsch_get_state(qnsch_ctx *x, double *c, double *mu, double *p, double *u, double *v)
{
    if (!x) return QNSCH_EINVAL;
    DLev &D = x->L[0];
    Desc &d = x->hd[0];
    int rc;
    if (c && (rc = get(x, c, d.c))) return rc;
    if (mu && (rc = get(x, mu, d.mu))) return rc;
    if (p && (rc = get(x, p, d.p))) return rc;
    if (u && (rc = get(x, u, d.ub[D.cur]))) return rc;
    if (v && (rc = get(x, v, d.vb[D.cur]))) return rc;
    HIPCHK(x, hipStreamSynchronize(x->s));
    return QNSCH_OK;
}

static int set_dt(qnsch_ctx *x, double dt)
{
    x->dt = dt;
    for (int l = 0; l < x->nlev; l++) {
        x->hd[l].P.inv_dt = 1.0 / dt;
        x->hd[l].P.dt = dt;
        x->hd[l].Pf.inv_dt = (float)(1.0 / dt);
    }
    return upload_desc(x);
}

int qnsch_begin_step(qnsch_ctx *x, double dt)
{
    if (!x || !(dt > 0)) return QNSCH_EINVAL;
    int rc;
    if ((rc = set_dt(x, dt))) return rc;
    std::vector<Op> prog;
    step_begin_program(x, prog);
    prog.pop_back(); // no residual here
    acc_reset(x);
    x->diss_state = 0;
    if ((rc = run_ops(x, prog))) return rc;
    x->in_step = 1;
    x->st.vcycles = 0;
    return QNSCH_OK;
}

int qnsch_vcycle(qnsch_ctx *x)
{
    if (!x) return QNSCH_EINVAL;
    if (!x->in_step) { x->err = "vcycle outside a step"; return QNSCH_EBUSY; }
    std::vector<Op> prog;
    x->acc_use = 0; // a combination not applied by qnsch_accelerate is dropped
    cycle_program(x, prog);
    const std::vector<Op> body(prog.begin(), prog.end() - 1);
    int rc;
    if ((rc = run_cycle(x, prog, body))) return rc;
    if ((rc = read_red(x))) return rc;
    if (x->acc_wait) acc_after(x);
    x->st.vcycles++;
    return QNSCH_OK;
}

int qnsch_accelerate(qnsch_ctx *x)
{
    if (!x) return QNSCH_EINVAL;
    if (!x->in_step) { x->err = "accelerate outside a step"; return QNSCH_EBUSY; }
    if (x->acc_use == 0) return QNSCH_OK;
    int rc;
    if ((rc = run_ops(x, { { OP_ACCEL, 0, 0 } }))) return rc;
    HIPCHK(x, hipStreamSynchronize(x->s));
    return QNSCH_OK;
}

int qnsch_residual(qnsch_ctx *x, double *r_out, double nrm[5])
{
    if (!x) return QNSCH_EINVAL;
    if (!x->in_step) { x->err = "residual outside a step"; return QNSCH_EBUSY; }
    DLev &D = x->L[0];
    const size_t n = (size_t)D.m1 * D.m2;
    int rc = QNSCH_OK;
    if (r_out && !x->hd[0].rout) {
        x->hd[0].rout = dalloc(x, 5 * n, &rc);
        if (rc) return rc;
        if ((rc = upload_desc(x))) return rc;
    }
    if ((rc = run_ops(x, { { OP_NORM0, 0, 0 } }))) return rc;
    if ((rc = read_red(x))) return rc;
    if (nrm) memcpy(nrm, x->red_host, 5 * sizeof(double));
    if (r_out) HIPCHK(x, hipMemcpy(r_out, x->hd[0].rout, 5 * n * sizeof(double), hipMemcpyDeviceToHost));
    return QNSCH_OK;
}

int qnsch_halfsweep(qnsch_ctx *x, int colour)
{
    if (!x) return QNSCH_EINVAL;
    if (!x->in_step) { x->err = "halfsweep outside a step"; return QNSCH_EBUSY; }
    if (is_mixed(x)) { x->err = "halfsweep: the nonlinear FP64 smoother needs an FP64 context"; return QNSCH_EINVAL; }
    int rc;
    if ((rc = run_ops(x, { { OP_HS, 0, colour & 1 } }))) return rc;
    HIPCHK(x, hipStreamSynchronize(x->s));
    return QNSCH_OK;
}

int qnsch_lin_apply(qnsch_ctx *x, const double *dw, double *out)
{
    if (!x || !dw || !out) return QNSCH_EINVAL;
    if (!is_mixed(x)) { x->err = "lin_apply needs a mixed-precision context"; return QNSCH_EINVAL; }
    if (!x->in_step) { x->err = "lin_apply outside a step"; return QNSCH_EBUSY; }
    DLev &D = x->L[0];
    Desc &d = x->hd[0];
    const size_t n = (size_t)D.m1 * D.m2;
    int rc = QNSCH_OK;
    if (!d.rout) {
        d.rout = dalloc(x, 5 * n, &rc);
        if (rc) return rc;
        if ((rc = upload_desc(x))) return rc;
    }
    // linearisation point = the current iterate; then a zero right-hand side
    // and the given correction
    if ((rc = run_ops(x, { { OP_NORM0, 0, 0 } }))) return rc;
    float *rhs[5] = { d.rc, d.rmu, d.rp, d.ru, d.rv };
    for (int q = 0; q < 5; q++) HIPCHK(x, hipMemsetAsync(rhs[q], 0, D.n() * sizeof(float), x->s));
    std::vector<float> f(n);
    float *dst[5] = { d.dc, d.dmu, d.dp, d.dub[D.cur], d.dvb[D.cur] };
    for (int q = 0; q < 5; q++) {
        for (size_t k = 0; k < n; k++) f[k] = (float)dw[q * n + k];
        HIPCHK(x, hipMemcpy2DAsync(dst[q], D.pitch * sizeof(float), f.data(), D.m1 * sizeof(float),
                                   D.m1 * sizeof(float), D.m2, hipMemcpyHostToDevice, x->s));
        HIPCHK(x, hipStreamSynchronize(x->s)); // f is reused
    }
    ItemList W;
    add_item(W, x, OP_MXHS, 0);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    KLAUNCH(k_mx_linresid, W, dim3(W.blocks), dim3(TBLK), 0, x->s);
    HIPCHK(x, hipGetLastError());
    HIPCHK(x, hipMemcpyAsync(out, d.rout, 5 * n * sizeof(double), hipMemcpyDeviceToHost, x->s));
    HIPCHK(x, hipStreamSynchronize(x->s));
    for (size_t k = 0; k < 5 * n; k++) out[k] = -out[k];
    return QNSCH_OK;
}

// projection scheme: the velocity of time n+1 replaces the intermediate one
// in the current face buffer (the latter kept for the dissipation)
static int pj_final(qnsch_ctx *x)
{
    if (x->opt.scheme != QNSCH_PROJECTION) return QNSCH_OK;
    return run_ops(x, { { OP_PJFINAL, 0, 0 } });
}

int qnsch_end_step(qnsch_ctx *x)
{
    if (!x) return QNSCH_EINVAL;
    int rc = QNSCH_OK;
    if (x->in_step) {
        rc = pj_final(x);
        if (!rc) x->diss_state = 1;
    }
    x->in_step = 0;
    return rc;
}

// decision after a residual reduction: 1 converged, 0 continue, <0 error
static int stop_test(qnsch_ctx *x, int vcycles)
{
    double mx = 0.0;
    bool finite = true;
    for (int q = 0; q < 5; q++) {
        if (!std::isfinite(x->red_host[q])) finite = false;
        mx = x->red_host[q] > mx ? x->red_host[q] : mx;
    }
    if (!finite || x->red_host[6] != 0.0) {
        x->err = "diverged: non-finite residual or c past the density pole";
        return QNSCH_EDIVERGED;
    }
    if (mx <= x->opt.tol) return 1;
    if (vcycles >= x->opt.max_vcycles) {
        x->err = "no convergence within max_vcycles";
        return QNSCH_ENOCONV;
    }
    return 0;
}

// a step that fails after its time-n data were fixed: the state goes back to
// time n (cell unknowns, faces, mubar and pbar), the step ends, and the error
// of the failure (code and message) is returned even if the restore fails too
static int fail_step(qnsch_ctx *x, int code)
{
    const std::string msg = x->err;
    (void)run_ops(x, { { OP_RESTORE, 0, 0 } });
    (void)hipStreamSynchronize(x->s);
    x->err = msg;
    x->in_step = 0;
    return code;
}

int qnsch_step(qnsch_ctx *x, double dt)
{
    if (!x || !(dt > 0)) return QNSCH_EINVAL;
    auto t0 = std::chrono::steady_clock::now();
    int rc;
    x->diss_state = 0;
    if ((rc = set_dt(x, dt))) return rc;
    std::vector<Op> begin, cyc;
    step_begin_program(x, begin);
    cycle_program(x, cyc);
    const std::vector<Op> body(cyc.begin(), cyc.end() - 1);
    acc_reset(x);
    // the begin programme only copies the state into the time-n data
    if ((rc = run_ops(x, begin))) { x->in_step = 0; return rc; }
    x->in_step = 1;
    if ((rc = read_red(x))) return fail_step(x, rc);
    memcpy(x->st.res0, x->red_host, 5 * sizeof(double));
    memcpy(x->st.hist[0], x->red_host, 5 * sizeof(double));
    x->st.hist_len = 1;
    int it = 0;
    x->st.vcycles = 0;
    for (;;) {
        const int j = stop_test(x, it);
        if (j < 0) return fail_step(x, j);
        if (j == 1) break;
        if ((rc = run_cycle(x, cyc, body))) return fail_step(x, rc);
        if ((rc = read_red(x))) return fail_step(x, rc);
        if (x->acc_wait) acc_after(x);
        it++;
        x->st.vcycles = it;
        if (it < QNSCH_HIST) {
            memcpy(x->st.hist[it], x->red_host, 5 * sizeof(double));
            x->st.hist_len = it + 1;
        }
    }
    memcpy(x->st.res, x->red_host, 5 * sizeof(double));
    if ((rc = pj_final(x))) return fail_step(x, rc);
    x->in_step = 0;
    x->diss_state = 1;
    x->st.step_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return QNSCH_OK;
}

static int reduce_me(qnsch_ctx *x)
{
    int rc;
    if ((rc = run_ops(x, { { OP_STEPEND, 0, 0 } }))) return rc;
    return read_red(x);
}

// mass and energy from the sums of k_mass_energy
static void me_from_sums(const qnsch_ctx *x, const double *s, double mass[2], double en[5])
{
    const double h2 = x->L[0].h * x->L[0].h;
    const qnsch_params &p = x->prm;
    if (mass) {
        mass[0] = h2 * s[0];
        mass[1] = h2 * s[1];
    }
    if (en) {
        en[1] = h2 * s[2];
        en[2] = p.eps * p.eta / (2.0 * p.We) * h2 * s[3];
        en[3] = p.eta / (p.eps * p.We) * h2 * s[4];
        en[4] = p.inv_Fr * h2 * s[5];
        en[0] = en[1] + en[2] + en[3] + en[4];
    }
}

int qnsch_mass(qnsch_ctx *x, double out[2])
{
    if (!x || !out) return QNSCH_EINVAL;
    int rc;
    if ((rc = reduce_me(x))) return rc;
    me_from_sums(x, x->red_host, out, nullptr);
    return QNSCH_OK;
}

int qnsch_energy(qnsch_ctx *x, double out[5])
{
    if (!x || !out) return QNSCH_EINVAL;
    int rc;
    if ((rc = reduce_me(x))) return rc;
    me_from_sums(x, x->red_host, nullptr, out);
    return QNSCH_OK;
}

int qnsch_dissipation(qnsch_ctx *x, double out[5])
{
    if (!x || !out) return QNSCH_EINVAL;
    if (!(x->dt > 0)) { x->err = "dissipation before any step"; return QNSCH_EBUSY; }
    int rc;
    if ((rc = run_ops(x, { { OP_DISSIP, 0, 0 } }))) return rc;
    if ((rc = read_red(x))) return rc;
    const double h2 = x->L[0].h * x->L[0].h;
    const qnsch_params &p = x->prm;
    out[0] = x->dt / p.Re * h2 * x->red_host[0];
    out[1] = x->dt / (3.0 * p.Re) * h2 * x->red_host[1];
    out[2] = x->dt / (p.M * p.Pe) * h2 * x->red_host[2];
    out[3] = 0.5 * h2 * x->red_host[3];
    out[4] = 0.5 * h2 * x->red_host[4];
    if (x->diss_state == 1) {
        memcpy(x->st.dissipation, out, 5 * sizeof(double));
        x->diss_state = 2;
    }
    return QNSCH_OK;
}

int qnsch_diagnostics(qnsch_ctx *x, double out[8])
{
    if (!x || !out) return QNSCH_EINVAL;
    int rc;
    if ((rc = run_ops(x, { { OP_DIAG, 0, 0 } }))) return rc;
    if ((rc = read_red(x))) return rc;
    const double h = x->L[0].h, *r = x->red_host;
    const double nan = std::nan("");
    out[0] = r[1] != 0.0 ? r[0] / r[1] : nan;
    out[1] = h * h * r[1];
    out[2] = r[2];
    out[3] = sqrt(h * h * r[3]);
    out[4] = r[5] > -1e299 ? r[5] : nan;
    out[5] = r[6] < 1e299 ? r[6] : nan;
    out[6] = r[7] > -1e299 ? r[7] : nan;
    out[7] = h * h * r[4];
    return QNSCH_OK;
}

int qnsch_stats(qnsch_ctx *x, qnsch_step_stats *out)
{
    if (!x || !out) return QNSCH_EINVAL;
    *out = x->st;
    if (x->diss_state != 2)
        for (int q = 0; q < 5; q++) out->dissipation[q] = std::nan("");
    return QNSCH_OK;
}

int qnsch_synchronize(qnsch_ctx *x)
{
    if (!x) return QNSCH_EINVAL;
    HIPCHK(x, hipStreamSynchronize(x->s));
    return QNSCH_OK;
}

static int profile_reset(qnsch_ctx *x, int mode, uint64_t mask, bool fine_only)
{
    HIPCHK(x, hipStreamSynchronize(x->s));
    int rc;
    if ((rc = prof_collect(x))) return rc;
    x->prof = mode;
    x->prof_mask = mask;
    x->prof_fine_only = fine_only;
    if (mode && x->pev.size() < 2 * PROF_POOL && (rc = prof_grow(x, PROF_POOL - (int)x->pev.size() / 2))) return rc;
    x->prof_ms = 0.0;
    x->prof_n = 0;
    for (int q = 0; q < NOPS * PROF_LEVELS; q++) {
        x->tag_ms[q] = 0.0;
        x->tag_n[q] = 0;
    }
    return QNSCH_OK;
}

int qnsch_profile(qnsch_ctx *x, int enable)
{
    if (!x) return QNSCH_EINVAL;
    const int mode = enable < 0 || enable > 2 ? 1 : enable;
    const uint64_t smoothers = (1ull << OP_HS) | (1ull << OP_MXHS) | (1ull << OP_FUSED) | (1ull << OP_MXFUSED);
    return profile_reset(x, mode, mode == 1 ? smoothers : 0, mode == 1);
}

int qnsch_profile_ops(qnsch_ctx *x, uint64_t op_mask)
{
    if (!x) return QNSCH_EINVAL;
    return profile_reset(x, op_mask ? 1 : 0, op_mask, false);
}

int qnsch_set_allocator(qnsch_alloc_fn alloc, qnsch_free_fn free_fn, void *user)
{
    if ((alloc == nullptr) != (free_fn == nullptr)) return QNSCH_EINVAL;
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc.alloc = alloc;
    g_alloc.free = free_fn;
    g_alloc.user = alloc ? user : nullptr;
    return QNSCH_OK;
}

int qnsch_graphs(qnsch_ctx *x, int enable)
{
    if (!x) return QNSCH_EINVAL;
    x->graphs = enable != 0;
    return QNSCH_OK;
}

int qnsch_profile_read(qnsch_ctx *x, double out[2])
{
    if (!x || !out) return QNSCH_EINVAL;
    HIPCHK(x, hipStreamSynchronize(x->s));
    int rc;
    if ((rc = prof_collect(x))) return rc;
    out[0] = (double)x->prof_n;
    out[1] = x->prof_ms;
    return QNSCH_OK;
}

int qnsch_profile_breakdown(qnsch_ctx *x, int32_t *kinds, double *out, int32_t cap)
{
    if (!x || (cap > 0 && (!kinds || !out))) return QNSCH_EINVAL;
    HIPCHK(x, hipStreamSynchronize(x->s));
    int rc;
    if ((rc = prof_collect(x))) return rc;
    int k = 0;
    for (int t = 0; t < NOPS * PROF_LEVELS; t++) {
        if (!x->tag_n[t]) continue;
        if (k < cap) {
            kinds[k] = t;
            out[2 * k] = (double)x->tag_n[t];
            out[2 * k + 1] = x->tag_ms[t];
        }
        k++;
    }
    return k;
}

double qnsch_default_eta(double rho1, double rho2)
{
    if (!(rho1 > 0) || !(rho2 > 0)) return NAN;
    const double x = rho2 / rho1 - 1.0;
    if (fabs(x) < 0.05) {
        // f(x) = (1+x)^2 - 1 - 2(1+x) ln(1+x) = sum_{k>=3} (-1)^(k+1) 2 x^k / (k(k-1));
        // eta = x^3 / (2 sqrt2 rho1 (1+x) f(x)), f(x)/x^3 summed to x^14
        double s = 0.0, xp = 1.0;
        for (int k = 3; k <= 17; k++) {
            s += ((k & 1) ? 2.0 : -2.0) * xp / (k * (k - 1.0));
            xp *= x;
        }
        return 1.0 / (2.0 * sqrt(2.0) * rho1 * (1.0 + x) * s);
    }
    const double d = rho2 - rho1;
    return d * d * d / (2.0 * sqrt(2.0) * rho1 * rho2 * (rho2 * rho2 - rho1 * rho1 - 2.0 * rho1 * rho2 * log(rho2 / rho1)));
}

int qnsch_copy_probe(size_t n, int reps, double out[2])
{
    if (n == 0 || reps < 1 || !out) return QNSCH_EINVAL;
    double *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, n * sizeof(double)) != hipSuccess) return QNSCH_ENOMEM;
    if (hipMalloc(&b, n * sizeof(double)) != hipSuccess) { (void)hipFree(a); return QNSCH_ENOMEM; }
    int rc = QNSCH_OK;
    hipEvent_t e0, e1;
    if (hipMemset(a, 0, n * sizeof(double)) != hipSuccess || hipEventCreate(&e0) != hipSuccess
        || hipEventCreate(&e1) != hipSuccess) {
        rc = QNSCH_EDEVICE;
    } else {
        const unsigned grid = 256u * 8u;
        hipLaunchKernelGGL(k_copy_probe, dim3(grid), dim3(BLK), 0, nullptr, a, b, n); // warm-up
        (void)hipEventRecord(e0, nullptr);
        for (int r = 0; r < reps; r++) hipLaunchKernelGGL(k_copy_probe, dim3(grid), dim3(BLK), 0, nullptr, a, b, n);
        (void)hipEventRecord(e1, nullptr);
        float ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = QNSCH_EDEVICE;
        out[1] = ms / reps;
        out[0] = 2.0 * n * sizeof(double) / (out[1] * 1e-3) / 1e9;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    (void)hipFree(a);
    (void)hipFree(b);
    return rc;
}

// ---------------------------------------------------------------------------
// residual norms without allocation.  The level descriptor, the reduction's
// partial sums and the reduced values live in `scratch`, a static device
// array of every device the library runs on (held until the process ends);
// host code reaches it only through the device address hipGetSymbolAddress
// gives for the current device.

} // extern "C"

#define NOALLOC_MAX_CELLS (1 << 22)
#define NOALLOC_DESC_BYTES ((sizeof(Desc) + 255) & ~(size_t)255)
#define NOALLOC_TILES 20480
#define NOALLOC_BYTES (NOALLOC_DESC_BYTES + (size_t)(NOALLOC_TILES + 2) * NRED * sizeof(double))
static __device__ __align__(256) char scratch[NOALLOC_BYTES];

// device address of `scratch` on the current device (nullptr on error)
static char *noalloc_scratch(std::string &err)
{
    static std::mutex mu;
    static char *ptr[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        err = "no current HIP device";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        ptr[dev] = (char *)p;
    }
    return ptr[dev];
}

static std::string noalloc_err;

extern "C" {

const char *qnsch_residual_noalloc_error(void) { return noalloc_err.c_str(); }

int qnsch_residual_noalloc(const qnsch_grid *g, const qnsch_params *prm, double dt, const double *c,
                           const double *mu, const double *p, const double *u, const double *v, const double *cn,
                           const double *un, const double *vn, void *stream, double norms[5])
{
    if (!g || !prm || !c || !mu || !p || !u || !v || !cn || !un || !vn || !norms || !(dt > 0)) {
        noalloc_err = "residual_noalloc: NULL argument or dt <= 0";
        return QNSCH_EINVAL;
    }
    if (validate_grid_params(g, prm)) {
        noalloc_err = "residual_noalloc: invalid grid or parameters";
        return QNSCH_EINVAL;
    }
    if ((size_t)g->m1 * g->m2 > NOALLOC_MAX_CELLS || (size_t)tiles_x(g->m1) * tiles_y(g->m2) > NOALLOC_TILES) {
        noalloc_err = "residual_noalloc: more than 4194304 cells or 20480 tiles of 16 x 16";
        return QNSCH_EINVAL;
    }
    char *base = noalloc_scratch(noalloc_err);
    if (!base) return QNSCH_EDEVICE;
    {
        // the workgroup-size check (a launch and a synchronous copy), unless
        // the stream is being captured: then it waits for a call outside a
        // capture or a context creation on this device
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing((hipStream_t)stream, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone
            && group_size_check(noalloc_err))
            return QNSCH_EDEVICE;
    }
    hipStream_t s = (hipStream_t)stream;
    const int tx = tiles_x(g->m1), ty = tiles_y(g->m2);
    Desc d;
    memset((void *)&d, 0, sizeof(d));
    Phys P;
    const qnsch_params pr = resolve_params(*prm);
    phys_of(&pr, P);
    P.inv_dt = 1.0 / dt;
    P.dt = dt;
    d.P = P;
    d.Pf = physf_of(P);
    d.c = (double *)c; d.mu = (double *)mu; d.p = (double *)p;
    d.ub[0] = d.ub[1] = (double *)u;
    d.vb[0] = d.vb[1] = (double *)v;
    d.cn = (double *)cn; d.un = (double *)un; d.vn = (double *)vn;
    d.m1 = g->m1; d.m2 = g->m2; d.pitch = g->m1; d.bcx = g->bc_x; d.bcy = g->bc_y;
    d.h = g->Lx / g->m1;
    d.inv_h = 1.0 / d.h;
    d.finv_h = (float)d.inv_h;
    d.partials = (double *)(base + NOALLOC_DESC_BYTES);
    d.red = d.partials + (size_t)NOALLOC_TILES * NRED;
    d.red_host = d.red + NRED;  // the reduced values stay on the device
    hipError_t e = hipMemcpyAsync(base, &d, sizeof(d), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        Item1 it;
        memset(&it, 0, sizeof(it));
        it.n = 1;
        it.start[0] = 0;
        it.start[1] = tx * ty;
        it.d[0] = (const Desc *)base;
        it.tx[0] = tx;
        it.acc[0] = -1;
        hipLaunchKernelGGL(k_resid_norm<Item1>, dim3(tx * ty), dim3(TBLK), 0, s, it);
        Item1 f = it;
        f.start[1] = 1;
        f.tx[0] = tx * ty;
        hipLaunchKernelGGL(k_finalize<Item1>, dim3(1), dim3(BLK), 0, s, f, 0);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(norms, d.red, 5 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        noalloc_err = std::string("residual_noalloc: ") + hipGetErrorString(e);
        return QNSCH_EDEVICE;
    }
    return QNSCH_OK;
}

} // extern "C"

// ===========================================================================
// continuous-batching server
//
// Requests (independent simulations) are admitted first come, first served
// while a slot is free and their device footprint fits the budget, each into
// one of several lanes (HIP streams; the least loaded).  Every running request
// holds a programme of operations (the phases of its current step, then of
// its next V-cycle once its residual is known).  Each tick the scheduler takes,
// in every lane, the largest set of ready requests whose next operations are
// of the same kind (any level) and runs them as ONE work-list launch on that
// lane's stream; the requests left waiting catch up with the next largest
// set, which keeps a lane's population in step and its launches full, while
// the lanes overlap on the device (one lane's single-workgroup coarsest
// solves leave most CUs to the others).  Host round trips happen only at
// residual and step-end reductions (events, no stream drain).  Contexts are
// recycled by shape: a finished request's final state is downloaded through
// pinned staging and its device arrays serve the next request of that shape,
// so steady-state admission allocates nothing.

namespace {
enum { RQ_QUEUED = 0, RQ_RUNNING = 1, RQ_DONE = 2 };
enum { W_NONE = 0, W_NORM = 1, W_STEPEND = 2, W_DOWNLOAD = 3 };

struct Req {
    uint64_t id = 0;
    qnsch_grid g;
    qnsch_params p;
    qnsch_opts o;
    std::vector<double> c0;
    int nsteps = 0;
    double dt = 0;
    qnsch_ctx *x = nullptr;
    int state = RQ_QUEUED, status = QNSCH_OK;
    size_t foot = 0;
    int lane = 0;
    int step = 0, vcycles = 0;
    std::vector<Op> prog; // operations still to issue, from pc on
    size_t pc = 0;
    int wait = W_NONE;    // what the request waits for
    hipEvent_t gate = nullptr; // W_NORM / W_STEPEND: the event of its group's reduction
    std::chrono::steady_clock::time_point t_submit, t_admit, t_step0, t_done;
    std::vector<double> step_ms, mass, energy;
    std::vector<int> vc;
    std::vector<double> out[5]; // final state
};

// what fixes the device layout of a context
typedef std::tuple<int, int, double, double, int, int, int, int> Shape;
Shape shape_of(const qnsch_grid &g, const qnsch_opts &o)
{
    return Shape(g.m1, g.m2, g.Lx, g.Ly, g.bc_x, g.bc_y, level_count(&g),
                 o.precision * 16 + o.accel + 64 * (int)two_sets(o));
}

typedef std::chrono::steady_clock Clock;
} // namespace

struct qnsch_server {
    std::vector<hipStream_t> lanes; // streams the requests run on
    std::vector<int> lane_load;     // running requests per lane
    std::vector<bool> own;          // streams created by the server
    size_t budget = 0, used = 0, pooled = 0; // bytes of running / idle contexts
    int max_slots = 0;
    uint64_t next_id = 1;
    std::deque<Req *> queue;
    std::vector<Req *> active;
    std::map<uint64_t, Req *> all;
    std::multimap<Shape, qnsch_ctx *> pool; // idle contexts for reuse
    std::vector<double> lat_ms;             // every completed step
    double cell_steps = 0.0;
    bool started = false;
    Clock::time_point t_first, t_last;
    long launches = 0, ticks = 0, created = 0;
    double host_admit_ms = 0, host_finish_ms = 0, host_wait_ms = 0;
    std::string err;
    // one event per launched reduction, shared by the requests of its group
    std::vector<hipEvent_t> gate_pool;
    std::map<hipEvent_t, int> gate_users;
};

// an event for the reduction of a group of requests (from the pool)
static hipEvent_t gate_take(qnsch_server *S)
{
    if (!S->gate_pool.empty()) {
        hipEvent_t e = S->gate_pool.back();
        S->gate_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}
static void gate_release(qnsch_server *S, Req *r)
{
    if (!r->gate) return;
    auto it = S->gate_users.find(r->gate);
    if (it != S->gate_users.end() && --it->second == 0) {
        S->gate_pool.push_back(r->gate);
        S->gate_users.erase(it);
    }
    r->gate = nullptr;
}

static double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

static void start_step(Req *r)
{
    r->prog.clear();
    r->pc = 0;
    step_begin_program(r->x, r->prog);
    acc_reset(r->x);
    r->vcycles = 0;
    r->t_step0 = Clock::now();
}

// a context for request r: an idle one of the same shape, else a new one
// (idle contexts of other shapes are released first if the budget needs it);
// parameters, options, dt and the initial state are set, all asynchronously
static int admit(qnsch_server *S, Req *r)
{
    const auto t0 = Clock::now();
    const Shape key = shape_of(r->g, r->o);
    qnsch_ctx *x = nullptr;
    int rc = QNSCH_OK;
    r->lane = (int)(std::min_element(S->lane_load.begin(), S->lane_load.end()) - S->lane_load.begin());
    hipStream_t st = S->lanes[r->lane];
    auto it = S->pool.find(key);
    if (it != S->pool.end()) {
        x = it->second;
        S->pool.erase(it);
        S->pooled -= x->footprint;
        x->s = st; // its earlier work has completed (its download was observed)
        x->opt = r->o;
        set_params(x, &r->p);
        for (int l = 0; l < x->nlev; l++) x->L[l].cur = 0;
        x->in_step = 0;
        memset(&x->st, 0, sizeof(x->st));
        if (hipMemsetAsync(x->arena, 0, x->arena_bytes, st) != hipSuccess) rc = QNSCH_EDEVICE;
    } else {
        while (!S->pool.empty() && S->used + S->pooled + r->foot > S->budget) {
            auto v = S->pool.begin();
            S->pooled -= v->second->footprint;
            qnsch_destroy(v->second);
            S->pool.erase(v);
        }
        x = new qnsch_ctx();
        S->created++;
        rc = ctx_init(x, &r->g, &r->p, &r->o, st);
        const size_t n = (size_t)r->g.m1 * r->g.m2;
        if (!rc && hipHostMalloc((void **)&x->stage, 5 * n * sizeof(double), hipHostMallocDefault) != hipSuccess)
            rc = QNSCH_ENOMEM;
    }
    if (!rc) {
        x->dt = r->dt;
        for (int l = 0; l < x->nlev; l++) {
            x->hd[l].P.inv_dt = 1.0 / r->dt;
            x->hd[l].P.dt = r->dt;
            x->hd[l].Pf.inv_dt = (float)(1.0 / r->dt);
        }
        // hd and stage are pinned and not touched again before this
        // context's next admission, long after these copies have run
        rc = upload_desc(x);
    }
    if (!rc) {
        const DLev &D = x->L[0];
        memcpy(x->stage, r->c0.data(), (size_t)D.m1 * D.m2 * sizeof(double));
        if (hipMemcpy2DAsync(x->hd[0].c, D.pitch * sizeof(double), x->stage, D.m1 * sizeof(double),
                             D.m1 * sizeof(double), D.m2, hipMemcpyHostToDevice, st) != hipSuccess)
            rc = QNSCH_EDEVICE;
    }
    r->x = x;
    S->host_admit_ms += ms_between(t0, Clock::now());
    return rc;
}

// queue the download of the final state; the request completes when the
// copies have run
static void begin_finish(qnsch_server *S, Req *r, int status)
{
    const auto t0 = Clock::now();
    r->status = status;
    r->prog.clear();
    r->pc = 0;
    qnsch_ctx *x = r->x;
    const DLev &D = x->L[0];
    const Desc &d = x->hd[0];
    const size_t n = (size_t)D.m1 * D.m2;
    const double *src[5] = { d.c, d.mu, d.p, d.ub[D.cur], d.vb[D.cur] };
    bool ok = true;
    for (int q = 0; q < 5; q++)
        ok = ok && hipMemcpy2DAsync(x->stage + q * n, D.m1 * sizeof(double), src[q], D.pitch * sizeof(double),
                                    D.m1 * sizeof(double), D.m2, hipMemcpyDeviceToHost, x->s) == hipSuccess;
    ok = ok && hipEventRecord(x->ev, x->s) == hipSuccess;
    if (!ok && r->status == QNSCH_OK) r->status = QNSCH_EDEVICE;
    r->wait = W_DOWNLOAD;
    S->host_finish_ms += ms_between(t0, Clock::now());
}

static void complete_finish(qnsch_server *S, Req *r)
{
    const auto t0 = Clock::now();
    qnsch_ctx *x = r->x;
    const size_t n = (size_t)r->g.m1 * r->g.m2;
    for (int q = 0; q < 5; q++) r->out[q].assign(x->stage + q * n, x->stage + (q + 1) * n);
    r->state = RQ_DONE;
    r->wait = W_NONE;
    r->t_done = Clock::now();
    S->t_last = r->t_done;
    S->used -= r->foot;
    S->lane_load[r->lane]--;
    S->pool.insert({ shape_of(r->g, r->o), x });
    S->pooled += x->footprint;
    r->x = nullptr;
    S->host_finish_ms += ms_between(t0, Clock::now());
}

// act on a completed reduction of request r
static void after_reduction(qnsch_server *S, Req *r)
{
    qnsch_ctx *x = r->x;
    gate_release(S, r);
    if (r->wait == W_STEPEND) { // step-end sums: record mass and energy, next step
        double m[2], e[5];
        me_from_sums(x, x->red_host, m, e);
        r->mass.insert(r->mass.end(), m, m + 2);
        r->energy.insert(r->energy.end(), e, e + 5);
        const double ms = ms_between(r->t_step0, Clock::now());
        r->step_ms.push_back(ms);
        r->vc.push_back(r->vcycles);
        S->lat_ms.push_back(ms);
        S->cell_steps += (double)r->g.m1 * r->g.m2;
        r->step++;
        r->wait = W_NONE;
        if (r->step >= r->nsteps) begin_finish(S, r, QNSCH_OK);
        else start_step(r);
        return;
    }
    r->wait = W_NONE;
    if (x->acc_wait) acc_after(x);
    const int j = stop_test(x, r->vcycles);
    r->prog.clear();
    r->pc = 0;
    if (j < 0) {
        r->prog.push_back({ OP_RESTORE, 0, 0 });
        r->status = j;
    } else if (j == 1) {
        r->prog.push_back({ OP_STEPEND, 0, 0 });
    } else {
        if (x->acc_use > 0) r->prog.push_back({ OP_ACCEL, 0, 0 });
        cycle_program(x, r->prog);
        r->vcycles++;
    }
}

extern "C" {

size_t qnsch_footprint(const qnsch_grid *g, const qnsch_opts *o)
{
    qnsch_opts d;
    qnsch_default_opts(&d);
    return g ? footprint_of(g, o ? *o : d) : 0;
}

int qnsch_server_create(size_t hbm_budget, int32_t max_slots, int32_t lanes, void *stream, qnsch_server **out)
{
    if (!out || max_slots < 1 || hbm_budget == 0 || lanes < 1 || lanes > 16) return QNSCH_EINVAL;
    *out = nullptr;
    qnsch_server *S = new qnsch_server();
    S->budget = hbm_budget;
    S->max_slots = max_slots;
    for (int l = 0; l < lanes; l++) {
        hipStream_t st = nullptr;
        bool own = true;
        if (l == 0 && stream) {
            st = (hipStream_t)stream;
            own = false;
        } else if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            qnsch_server_destroy(S);
            return QNSCH_EDEVICE;
        }
        S->lanes.push_back(st);
        S->own.push_back(own);
        S->lane_load.push_back(0);
    }
    *out = S;
    return QNSCH_OK;
}

void qnsch_server_destroy(qnsch_server *S)
{
    if (!S) return;
    for (hipStream_t st : S->lanes) (void)hipStreamSynchronize(st);
    for (auto &kv : S->all) {
        if (kv.second->x) qnsch_destroy(kv.second->x);
        delete kv.second;
    }
    for (auto &kv : S->pool) qnsch_destroy(kv.second);
    for (hipEvent_t e : S->gate_pool) (void)hipEventDestroy(e);
    for (auto &kv : S->gate_users) (void)hipEventDestroy(kv.first);
    for (size_t l = 0; l < S->lanes.size(); l++)
        if (S->own[l]) (void)hipStreamDestroy(S->lanes[l]);
    delete S;
}

int qnsch_server_submit(qnsch_server *S, const qnsch_grid *g, const qnsch_params *p, const qnsch_opts *o,
                        const double *c0, int32_t nsteps, double dt, uint64_t *id)
{
    if (!S || !g || !p || !c0 || nsteps < 1 || !(dt > 0) || !id) return QNSCH_EINVAL;
    int rc = validate(g, p, o);
    if (rc) return rc;
    if (o && o->scheme != QNSCH_PRIMITIVE) {
        S->err = "the server runs the primitive scheme only";
        return QNSCH_EINVAL;
    }
    Req *r = new Req();
    r->id = S->next_id++;
    r->g = *g;
    r->p = resolve_params(*p);
    qnsch_default_opts(&r->o);
    if (o) r->o = *o;
    resolve_opts(r->o, level_count(g));
    // no temporal blocking in a server: its launches merge the same sweep of
    // many requests and so fill the device, where a fused sweep's redundant
    // red work costs more than the launch it saves (measured on one MI355X,
    // the served droplet stream: 5 % lower throughput with it)
    r->o.blocking = 0;
    r->c0.assign(c0, c0 + (size_t)g->m1 * g->m2);
    r->nsteps = nsteps;
    r->dt = dt;
    r->foot = footprint_of(g, r->o);
    if (r->foot > S->budget) {
        delete r;
        return QNSCH_ENOMEM;
    }
    r->t_submit = Clock::now();
    S->queue.push_back(r);
    S->all[r->id] = r;
    *id = r->id;
    return QNSCH_OK;
}

int qnsch_server_progress(qnsch_server *S, int32_t max_ticks)
{
    if (!S) return QNSCH_EINVAL;
    auto done = [](Req *r) { return r->state == RQ_DONE; };
    for (int tick = 0; tick < max_ticks; tick++) {
        while (!S->queue.empty() && (int)S->active.size() < S->max_slots
               && S->used + S->queue.front()->foot <= S->budget) {
            Req *r = S->queue.front();
            S->queue.pop_front();
            r->t_admit = Clock::now();
            if (!S->started) { S->started = true; S->t_first = r->t_admit; }
            const int rc = admit(S, r);
            if (rc) {
                if (r->x) qnsch_destroy(r->x);
                r->x = nullptr;
                r->status = rc;
                r->state = RQ_DONE;
                r->t_done = Clock::now();
                continue;
            }
            S->used += r->foot;
            S->lane_load[r->lane]++;
            r->state = RQ_RUNNING;
            start_step(r);
            S->active.push_back(r);
        }
        // completed events: reductions (one event per group, queried once
        // per tick) and downloads
        std::map<hipEvent_t, bool> ready;
        for (Req *r : S->active) {
            if (r->wait == W_NONE) continue;
            hipEvent_t e = r->wait == W_DOWNLOAD ? r->x->ev : r->gate;
            auto q = ready.find(e);
            const bool ok = q != ready.end() ? q->second : (ready[e] = hipEventQuery(e) == hipSuccess);
            if (!ok) continue;
            if (r->wait == W_DOWNLOAD) complete_finish(S, r);
            else after_reduction(S, r);
        }
        S->active.erase(std::remove_if(S->active.begin(), S->active.end(), done), S->active.end());
        // per lane, the largest set of ready requests with the same next
        // operation (kind, colour, coarse sweeps, relaxation factors); the
        // requests left out catch up while the others wait for a reduction,
        // which keeps a lane's requests in step and its launches full
        // (launching the largest set again and again within a tick lets it
        // run ahead: 0.84 instead of 0.78 of the launches the requests need
        // alone in the serving test, with the same throughput)
        typedef std::tuple<int, int, int, double, double> Key;
        bool launched = false;
        for (size_t lane = 0; lane < S->lanes.size(); lane++) {
            for (int burst = 0; burst < 1; burst++) {
                std::map<Key, std::vector<Req *>> groups;
                for (Req *r : S->active) {
                    if (r->lane != (int)lane || r->wait != W_NONE || r->pc >= r->prog.size()) continue;
                    const Op &o = r->prog[r->pc];
                    groups[Key(o.kind, o.colour, r->x->opt.nu_coarse, r->x->opt.vanka_omega, r->x->opt.coarse_omega)]
                        .push_back(r);
                }
                if (groups.empty()) break;
                auto best = groups.begin();
                for (auto g = groups.begin(); g != groups.end(); ++g)
                    if (g->second.size() > best->second.size()) best = g;
                std::vector<std::pair<qnsch_ctx *, int>> items;
                for (Req *r : best->second) items.push_back({ r->x, r->prog[r->pc].level });
                const int kind = std::get<0>(best->first);
                hipStream_t st = S->lanes[lane];
                int rc = launch_op(kind, std::get<1>(best->first), items, st);
                if (rc) {
                    S->err = items[0].first->err;
                    return rc;
                }
                launched = true;
                S->launches += (long)((items.size() + MAXITEMS - 1) / MAXITEMS);
                hipEvent_t gate = nullptr;
                if (kind == OP_NORM0 || kind == OP_NORM || kind == OP_NORMACC || kind == OP_STEPEND) {
                    gate = gate_take(S);
                    if (!gate || hipEventRecord(gate, st) != hipSuccess) {
                        S->err = "event for a reduction";
                        return QNSCH_EDEVICE;
                    }
                    S->gate_users[gate] = (int)best->second.size();
                }
                for (Req *r : best->second) {
                    r->pc++;
                    if (gate) {
                        r->wait = kind == OP_STEPEND ? W_STEPEND : W_NORM;
                        r->gate = gate;
                    } else if (kind == OP_RESTORE) {
                        begin_finish(S, r, r->status);
                    }
                }
            }
        }
        S->ticks++;
        if (!launched) {
            if (S->active.empty()) break; // nothing running (queue empty or waiting for budget)
            // everyone waits for an event: block on the oldest one
            const auto t0 = Clock::now();
            for (Req *r : S->active)
                if (r->wait != W_NONE) {
                    (void)hipEventSynchronize(r->wait == W_DOWNLOAD ? r->x->ev : r->gate);
                    break;
                }
            S->host_wait_ms += ms_between(t0, Clock::now());
        }
    }
    return (int)(S->queue.size() + S->active.size());
}

int qnsch_server_poll(qnsch_server *S, uint64_t id, int32_t *state, int32_t *status)
{
    if (!S) return QNSCH_EINVAL;
    auto it = S->all.find(id);
    if (it == S->all.end()) return QNSCH_EINVAL;
    if (state) *state = it->second->state;
    if (status) *status = it->second->status;
    return QNSCH_OK;
}

int qnsch_server_result(qnsch_server *S, uint64_t id, double *c, double *mu, double *p, double *u, double *v,
                        double *mass_hist, double *energy_hist, double *step_ms, int32_t *vcycles, double *times)
{
    if (!S) return QNSCH_EINVAL;
    auto it = S->all.find(id);
    if (it == S->all.end()) return QNSCH_EINVAL;
    Req *r = it->second;
    if (r->state != RQ_DONE) return QNSCH_EBUSY;
    double *dst[5] = { c, mu, p, u, v };
    for (int q = 0; q < 5; q++)
        if (dst[q] && !r->out[q].empty()) memcpy(dst[q], r->out[q].data(), r->out[q].size() * sizeof(double));
    if (mass_hist && !r->mass.empty()) memcpy(mass_hist, r->mass.data(), r->mass.size() * sizeof(double));
    if (energy_hist && !r->energy.empty()) memcpy(energy_hist, r->energy.data(), r->energy.size() * sizeof(double));
    if (step_ms && !r->step_ms.empty()) memcpy(step_ms, r->step_ms.data(), r->step_ms.size() * sizeof(double));
    if (vcycles && !r->vc.empty()) memcpy(vcycles, r->vc.data(), r->vc.size() * sizeof(int32_t));
    if (times) {
        times[0] = ms_between(r->t_submit, r->t_admit);
        times[1] = ms_between(r->t_submit, r->t_done);
    }
    return r->status;
}

int qnsch_server_latency(qnsch_server *S, double *p50, double *p99, double *cell_steps_per_s)
{
    double st[12];
    const int rc = qnsch_server_stats(S, st);
    if (rc) return rc;
    if (p50) *p50 = st[0];
    if (p99) *p99 = st[1];
    if (cell_steps_per_s) *cell_steps_per_s = st[4];
    return QNSCH_OK;
}

int qnsch_server_stats(qnsch_server *S, double out[12])
{
    if (!S || !out) return QNSCH_EINVAL;
    std::vector<double> l = S->lat_ms;
    std::sort(l.begin(), l.end());
    auto pct = [&](double q) {
        if (l.empty()) return 0.0;
        const double pos = q * (l.size() - 1);
        const size_t a = (size_t)pos;
        const size_t b = std::min(a + 1, l.size() - 1);
        return l[a] + (pos - a) * (l[b] - l[a]);
    };
    const double wall = S->started ? ms_between(S->t_first, S->t_last) * 1e-3 : 0.0;
    out[0] = pct(0.5);
    out[1] = pct(0.99);
    out[2] = S->cell_steps;
    out[3] = wall;
    out[4] = wall > 0 ? S->cell_steps / wall : 0.0;
    out[5] = (double)l.size();
    out[6] = (double)S->launches;
    out[7] = (double)S->ticks;
    out[8] = S->host_admit_ms;
    out[9] = S->host_finish_ms;
    out[10] = S->host_wait_ms;
    out[11] = (double)S->created;
    return QNSCH_OK;
}

const char *qnsch_server_last_error(const qnsch_server *S) { return S ? S->err.c_str() : "null server"; }

} // extern "C"
