// qnsch_kern.hpp -- work-list kernels of the FP64 multigrid step.
//
// Every kernel takes a work list: up to MAXITEMS items, each naming one level
// of one simulation (a device descriptor) and the range of workgroups that
// work on it.  A launch therefore applies the same operation (a colour
// half-sweep, a restriction, ...) to many simulations at once, at whatever
// level each of them is; a single simulation is a list of one item.  The
// work of a workgroup depends only on its item, so a simulation's results do
// not depend on what else shares the launch.
#pragma once
#include "qnsch_dev.hpp"
#include "qnsch_lin.hpp"

namespace qn {

#define BLK 256
#define NRED 16 // reduction slots
// Tile of cells per workgroup (one lane pair per cell of a colour).  16 x 16
// cells and 256 lanes: small levels spread over more CUs, and two or three
// workgroups share a CU on large ones (measured against 32 x 16 and 32 x 8).
#ifndef QN_TX
#define QN_TX 16
#endif
#ifndef QN_TY
#define QN_TY 16
#endif
#define TX QN_TX
#define TY QN_TY
#define TBLK (TX * TY)
// The FP64 finest-level half-sweep is register-limited to 2 waves per SIMD.
// With the segregated smoother alone, asking for 3 cost a few spilled
// registers and bought a third resident workgroup per CU (18 % faster on
// 512 x 2048); the coupled box needs some 25 more registers, whose spills at 3
// waves cost more than the third workgroup gains, so the finest level keeps 2.
// The attribute stays separate so that the trade can be re-measured.
#ifndef QN_FINE_WAVES
#define QN_FINE_WAVES 2
#endif
#define HS_ATTR __launch_bounds__(TBLK)
#define FINE_ATTR __launch_bounds__(TBLK) __attribute__((amdgpu_waves_per_eu(QN_FINE_WAVES)))
#define TILE_DOUBLES (T_NF * (TX + 3) * (TY + 3))
#define NXCD 8
#define MAXITEMS 64
static_assert(TILE_DOUBLES * 8 + 16 * NRED * 8 <= 65536, "tile exceeds 64 KiB of LDS");

// one level of one simulation, in device memory
struct Desc {
    Phys P;
    double *c, *mu, *p, *ub[2], *vb[2], *cn, *un, *vn; // level arrays (u/v ping-pong)
    double *fc, *fmu, *fp, *fu, *fv;                    // FAS right-hand side (NULL on the finest level)
    double *c0, *mu0, *p0, *u0, *v0;                    // restricted iterate (coarse levels)
    int m1, m2, pitch, bcx, bcy;
    double h, inv_h;
    const Desc *coarse;                                 // next coarser level (NULL on the coarsest)
    double *partials;                                   // per-simulation reduction partials (finest level)
    double *red;                                        // reduced values (device)
    double *red_host;                                   // reduced values (pinned host)
    double *mus, *ps;                                   // mubar, pbar of time n (finest level)
    double *c2, *mu2, *p2;                              // second set of cell unknowns (fused sweeps; else NULL)
    double *rout;                                       // residual fields (finest level, optional)
    // acceleration history (finest level): a ring of am slots, each holding
    // a cycle result (aw, pbar before its mean removal) and its residual (ar)
    // as 5 fields of pitch*m2, and the pbar mean removed from it (amean)
    double *aw, *ar, *amean;
    int am;
    // mixed precision: the FP32 correction hierarchy (NULL in FP64 mode; on
    // coarse levels the FP64 arrays above are NULL instead)
    PhysF Pf;
    float *xc, *xmu, *xu, *xv;                          // linearisation point
    float *dc, *dmu, *dp, *dub[2], *dvb[2];             // correction (u/v ping-pong)
    float *rc, *rmu, *rp, *ru, *rv;                     // right-hand side
    float *dc2, *dmu2, *dp2;                            // second set of cell corrections (fused sweeps)
    float *cnf, *unf, *vnf;                             // time-n data
    float finv_h;
};

// (The small entries are 32-bit: a kernel reads them with scalar loads,
// which have no 16-bit form; a 16-bit entry cost a vector load and its
// memory latency at the start of every kernel.)
struct Items {
    int n;
    int start[MAXITEMS + 1];  // first workgroup of each item; start[n] = total
    const Desc *d[MAXITEMS];  // the level worked on
    int par[MAXITEMS];        // current u/v buffer of that level
    int cpar[MAXITEMS];       // current u/v buffer of the next coarser level
    int tx[MAXITEMS];         // tiles per row (tile kernels); partial count (k_finalize)
    int acc[MAXITEMS];        // acceleration ring slot s | (earlier results used) << 4; -1 none
};
// The same for a list of one item (a simulation run on its own): 40 bytes
// of kernel arguments instead of 1.8 KB, which a dependent launch pays for
// (about 1.5 us measured per launch with 1.4 KB).  Kernels are instantiated
// for both.
struct Item1 {
    int n;
    int start[2];
    const Desc *d[1];
    int par[1];
    int cpar[1];
    int tx[1];
    int acc[1];
};

template <typename IT> __device__ __forceinline__ int find_item(const IT &it)
{
    int k = 0;
    while (k + 1 < it.n && (int)blockIdx.x >= it.start[k + 1]) k++;
    return k;
}

__device__ __forceinline__ View view_of(const Desc &d, int par)
{
    View V;
    V.c = d.c; V.mu = d.mu; V.p = d.p;
    V.u = d.ub[par]; V.v = d.vb[par];
    V.cn = d.cn; V.un = d.un; V.vn = d.vn;
    V.m1 = d.m1; V.m2 = d.m2; V.pitch = d.pitch;
    V.bcx = d.bcx; V.bcy = d.bcy;
    V.inv_h = d.inv_h;
    return V;
}
__device__ __forceinline__ Rhs rhs_of(const Desc &d)
{
    const Rhs F = { d.fc, d.fmu, d.fp, d.fu, d.fv };
    return F;
}

// Workgroups are dispatched round-robin over the XCDs, each with its own L2.
// Items start at multiples of NXCD and their tiles are renumbered so that an
// XCD gets a contiguous band of tiles: neighbouring tiles, which read each
// other's halos, share one L2.
template <typename R, typename IT>
__device__ __forceinline__ TileT<R> item_tile(R *sm, const IT &it, int k, const Desc &d)
{
    const int tx = it.tx[k];
    const int ty = (d.m2 + TY - 1) / TY;
    const int n = tx * ty, lin = (int)blockIdx.x - it.start[k];
    const int t = (n % NXCD == 0) ? (lin % NXCD) * (n / NXCD) + lin / NXCD : lin;
    TileT<R> T;
    T.s = sm;
    T.i0 = (t % tx) * TX;
    T.j0 = (t / tx) * TY;
    T.W = TX + 3;
    T.H = TY + 3;
    return T;
}
template <typename IT> __device__ __forceinline__ bool tile_valid(const IT &it, int k, const Desc &d)
{
    return (int)blockIdx.x - it.start[k] < it.tx[k] * ((d.m2 + TY - 1) / TY);
}

// --------------------------------------------------------------------------
// one colour half-sweep (sec. 7.1) on a tile: a lane pair per cell of the
// colour.  The u/v snapshot is buffer par, the new faces go to buffer par^1.
template <typename IT> __device__ __forceinline__ void halfsweep_body(const IT &it, int colour, double omega)
{
    __shared__ double sm[TILE_DOUBLES];
    const int k = find_item(it);
    const Desc &d = *it.d[k];
    if (!tile_valid(it, k, d)) return;
    // generic accesses and the constants by reference, as in k_hs_fused: the
    // two kernels then compile the relaxation alike and give bitwise the
    // same results
    const Phys &P = d.P;
    const int par = it.par[k];
    const View L = view_of(d, par);
    const Tile T = item_tile(sm, it, k, d);
    tile_load(P, L, T);
    __syncthreads();
    const int pr = threadIdx.x >> 1, hlf = threadIdx.x & 1;
    const int lj = pr / (TX / 2), kk = pr - lj * (TX / 2);
    const int j = T.j0 + lj;
    const int i = T.i0 + 2 * kk + ((j + colour) & 1);
    if (i < L.m1 && j < L.m2) relax_pair<0>(P, L, T, rhs_of(d), d.ub[par ^ 1], d.vb[par ^ 1], i, j, hlf, omega, 1.0);
}
template <typename IT> __global__ HS_ATTR void k_halfsweep(IT it, int colour, double omega)
{
    halfsweep_body(it, colour, omega);
}
// the same kernel under its own name for launches whose items are all finest
// levels, so that profiles tell the finest level apart
template <typename IT> __global__ FINE_ATTR void k_halfsweep_fine(IT it, int colour, double omega)
{
    halfsweep_body(it, colour, omega);
}

// --------------------------------------------------------------------------
// temporal blocking: one sweep (red, then black half-sweep of sec. 7.1, the
// same arithmetic as two k_halfsweep launches) in one launch.  A workgroup
// relaxes the red cells of its tile widened by two cells on every side (the
// red results its black cells read; neighbouring workgroups compute the
// overlap again), keeps them in LDS, then relaxes the black cells of its
// tile.  Workgroups still read their neighbours' cells as halo while others
// write, so the cell unknowns go from one set to the other (dir 0: c, mu, p
// to c2, mu2, p2; dir 1 back) and the faces from buffer par to par ^ 1.
#define FUSED_W (TX + 7)
#define FUSED_H (TY + 7)
#define FBLK (2 * TBLK)
#define FUSED_DOUBLES ((T_NF + 2) * FUSED_W * FUSED_H)
static_assert(FUSED_DOUBLES * 8 <= 65536, "fused tile exceeds 64 KiB of LDS");
static_assert((TX + 4) * (TY + 4) <= FBLK, "widened red region exceeds the workgroup");

// the coarse level's arrays that the coarse-grid correction reads, and the
// fine level's boundary kinds, taken from the level descriptors once per
// workgroup (read inside the tile loader, the descriptors would be reloaded
// per element behind the tile stores)
struct PSrc {
    const double *c, *c0, *mu, *mu0, *p, *p0, *u, *u0, *v, *v0;
    int pitch, m1, m2, bcx, bcy;
};
__device__ __forceinline__ PSrc psrc_of(const Desc &d, const Desc *cp, int cpar)
{
    // the descriptor is in global memory: read through a global pointer, its
    // fields are scalar loads issued at once (a generic pointer would make
    // them vector loads)
    const __attribute__((address_space(1))) Desc &C = *(const __attribute__((address_space(1))) Desc *)cp;
    PSrc s;
    s.c = C.c; s.c0 = C.c0; s.mu = C.mu; s.mu0 = C.mu0; s.p = C.p; s.p0 = C.p0;
    s.u = C.ub[cpar]; s.u0 = C.u0; s.v = C.vb[cpar]; s.v0 = C.v0;
    s.pitch = C.pitch; s.m1 = C.m1; s.m2 = C.m2; s.bcx = d.bcx; s.bcy = d.bcy;
    return s;
}
// The coarse-grid correction P(w_H - R w_h) of the fine unknowns: a cell takes
// its coarse cell's value (piecewise constant); a face copies the coincident
// coarse face, or, between two coarse faces, averages them; a face on a wall
// is no unknown.  For one tile element it comes in two parts so that every
// load is in flight before any value is used.  prolong_load reads the coarse
// cell of the cell source (ic, jc) with its restricted iterate, and for each
// face source the coarse face it lies on and the next one along its axis (the
// periodic image, or, where there is none, the same face again: loaded, not
// used).
struct PRaw {
    double c, c0, mu, mu0, p, p0, u[4], v[4];
};
__device__ __forceinline__ PRaw prolong_load(const PSrc &C, int ic, int jc, int iu, int ju, int iv, int jv)
{
    PRaw r;
    const size_t kc = (size_t)(jc >> 1) * C.pitch + (ic >> 1);
    r.c = lda<1>(C.c, kc); r.c0 = lda<1>(C.c0, kc); r.mu = lda<1>(C.mu, kc); r.mu0 = lda<1>(C.mu0, kc);
    r.p = lda<1>(C.p, kc); r.p0 = lda<1>(C.p0, kc);
    {
        const int I = iu >> 1, J = ju >> 1;
        const size_t k0 = (size_t)J * C.pitch + I;
        const size_t k1 = I + 1 < C.m1 ? k0 + 1 : (C.bcx ? (size_t)J * C.pitch : k0);
        r.u[0] = lda<1>(C.u, k0); r.u[1] = lda<1>(C.u0, k0); r.u[2] = lda<1>(C.u, k1); r.u[3] = lda<1>(C.u0, k1);
    }
    {
        const int I = iv >> 1, J = jv >> 1;
        const size_t k0 = (size_t)J * C.pitch + I;
        const size_t k1 = J + 1 < C.m2 ? k0 + C.pitch : (C.bcy ? (size_t)I : k0);
        r.v[0] = lda<1>(C.v, k0); r.v[1] = lda<1>(C.v0, k0); r.v[2] = lda<1>(C.v, k1); r.v[3] = lda<1>(C.v0, k1);
    }
    return r;
}
// ... and the corrections: the cell unknowns, the u face (iu, ju) and the v
// face (iv, jv) (zero for a face on a wall)
__device__ __forceinline__ void prolong_apply(const PSrc &C, const PRaw &r, int iu, int iv, int jv, double &c,
                                              double &mu, double &p, double &du, double &dv)
{
    c = r.c - r.c0;
    mu = r.mu - r.mu0;
    p = r.p - r.p0;
    du = r.u[0] - r.u[1];
    if (iu & 1) {
        const double e = ((iu >> 1) + 1 < C.m1 || C.bcx) ? r.u[2] - r.u[3] : 0.0;
        du = 0.5 * (du + e);
    }
    if (!(C.bcx || iu >= 1)) du = 0.0;
    dv = r.v[0] - r.v[1];
    if (jv & 1) {
        const double e = ((jv >> 1) + 1 < C.m2 || C.bcy) ? r.v[2] - r.v[3] : 0.0;
        dv = 0.5 * (dv + e);
    }
    if (!(C.bcy || jv >= 1)) dv = 0.0;
}

// the widened tile: every field at tile positions i0-1 .. i0+W-2 (level
// coordinates; periodic images at their unwrapped positions), plus copies of
// u and v in the fields T_NF, T_NF + 1 that the red pass overwrites.  A
// periodic axis needs m >= TX + 3 so that a single wrap reaches every position.
// With pc set (the first sweep of a post-smoothing), each unknown first takes
// the coarse-grid correction P(w_H - R w_h) of its source (k_prolong's
// arithmetic); the sweep writes every unknown of the level, so the corrected
// values need no store of their own.
__device__ __forceinline__ void fused_load(const Phys &P, const View &L, const Tile &T, const PSrc *pc = nullptr)
{
    const int n = T.W * T.H;
    for (int e = threadIdx.x; e < n; e += block_threads()) {
        const int b = e / T.W, a = e - b * T.W;
        int i = T.i0 - 1 + a, j = T.j0 - 1 + b;
        if (L.bcx) i = wrapi(i, L.m1);
        if (L.bcy) j = wrapi(j, L.m2);
        const TileSrc q = tile_src(L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j);
        double *s = T.s + e;
        if (q.sc == 0) {
            for (int f = 0; f < T_NF + 2; f++) s[f * n] = 0.0;
            continue;
        }
        double v[8] = { lda<1>(L.c, q.c), lda<1>(L.mu, q.c), lda<1>(L.p, q.c), lda<1>(L.u, q.u),
                        lda<1>(L.v, q.v), lda<1>(L.cn, q.c), lda<1>(L.un, q.u), lda<1>(L.vn, q.v) };
        PRaw raw = {};
        int iu = 0, iv = 0, jv = 0;
        if (pc) {
            iu = q.u % L.pitch;
            iv = q.v % L.pitch;
            jv = q.v / L.pitch;
            raw = prolong_load(*pc, q.c % L.pitch, q.c / L.pitch, iu, q.u / L.pitch, iv, jv);
        }
        // every load above is issued before anything uses a loaded value (the
        // scheduler otherwise interleaves uses with the loads, one memory
        // latency each)
        __builtin_amdgcn_sched_barrier(0);
        if (pc) {
            double rc, rm, rp, du, dv;
            prolong_apply(*pc, raw, iu, iv, jv, rc, rm, rp, du, dv);
            v[0] += rc;
            v[1] += rm;
            v[2] += rp;
            if (q.su) v[3] += du;
            if (q.sv) v[4] += dv;
        }
        s[T_C * n] = v[0];
        s[T_MU * n] = v[1];
        s[T_P * n] = v[2];
        s[T_U * n] = s[T_NF * n] = signed_val(q.su, v[3]);
        s[T_V * n] = s[(T_NF + 1) * n] = signed_val(q.sv, v[4]);
        s[T_CN * n] = v[5];
        s[T_UN * n] = signed_val(q.su, v[6]);
        s[T_VN * n] = signed_val(q.sv, v[7]);
        s[T_RN * n] = rho_of(P, v[5]);
        s[T_MV * n] = visc_of(P, v[5]);
        s[T_MOB * n] = mob_of(P, v[5]);
        s[T_RS * n] = rho_of(P, v[0]);
    }
}
// after the red pass: the new faces become the snapshot of the black pass,
// and the images across walls follow their sources (ldc clamps a cell to the
// wall row; ldu, ldv zero a face on or beyond a wall and reflect a
// tangential ghost).  Periodic images were relaxed in place.
__device__ __forceinline__ void fused_refresh(const View &L, const Tile &T)
{
    const int n = T.W * T.H;
    const double *un = T.s + T_NF * n, *vn = T.s + (T_NF + 1) * n;
    for (int e = threadIdx.x; e < n; e += block_threads()) {
        const int b = e / T.W, a = e - b * T.W;
        const int i = T.i0 - 1 + a, j = T.j0 - 1 + b;
        const bool gx = !L.bcx && (i < 0 || i >= L.m1), gy = !L.bcy && (j < 0 || j >= L.m2);
        const int si = gx ? (i < 0 ? 0 : L.m1 - 1) : i, sj = gy ? (j < 0 ? 0 : L.m2 - 1) : j;
        const int su = (!L.bcx && (i <= 0 || i >= L.m1)) ? 0 : (gy ? -1 : 1);
        const int sv = (!L.bcy && (j <= 0 || j >= L.m2)) ? 0 : (gx ? -1 : 1);
        // every value the element may take, before any store (an image's
        // source q is never an image, so no element read here is written)
        const int q = T.idx(si, sj);
        const double u = un[T.idx(i, sj)], v = vn[T.idx(si, j)], c = T.s[T_C * n + q], mu = T.s[T_MU * n + q],
                     p = T.s[T_P * n + q], rs = T.s[T_RS * n + q];
        __builtin_amdgcn_sched_barrier(0);
        T.s[T_U * n + e] = signed_val(su, u);
        T.s[T_V * n + e] = signed_val(sv, v);
        if (gx || gy) {
            T.s[T_C * n + e] = c;
            T.s[T_MU * n + e] = mu;
            T.s[T_P * n + e] = p;
            T.s[T_RS * n + e] = rs;
        }
    }
}
template <typename IT> __global__ __launch_bounds__(FBLK) void k_hs_fused(IT it, int dir, double omega, int prolong)
{
    __shared__ double sm[FUSED_DOUBLES];
    const int k = find_item(it);
    const Desc &d = *it.d[k];
    if (!tile_valid(it, k, d)) return;
    // generic accesses and the constants by reference: global-typed accesses
    // with the constants held by value measured 3 % slower for this kernel
    const Phys &P = d.P;
    const int par = it.par[k];
    View L = view_of(d, par);
    View O = L; // where the sweep's cell results go
    if (dir) {
        L.c = d.c2; L.mu = d.mu2; L.p = d.p2;
    } else {
        O.c = d.c2; O.mu = d.mu2; O.p = d.p2;
    }
    const Tile T0 = item_tile(sm, it, k, d);
    Tile T;
    T.s = sm; T.i0 = T0.i0 - 2; T.j0 = T0.j0 - 2; T.W = FUSED_W; T.H = FUSED_H;
    {
        // the loader's constants by value (no tile store can change them)
        const Phys Pv = d.P;
        if (prolong) {
            const PSrc ps = psrc_of(d, d.coarse, it.cpar[k]);
            fused_load(Pv, L, T, &ps);
        } else {
            fused_load(Pv, L, T);
        }
    }
    __syncthreads();
    const Rhs F = rhs_of(d);
    const int pr = threadIdx.x >> 1, hlf = threadIdx.x & 1;
    {
        // red: cells with i + j even of i0-2 .. i0+TX+1, j0-2 .. j0+TY+1
        const int lj = pr / ((TX + 4) / 2), kk = pr - lj * ((TX + 4) / 2);
        const int tj = T0.j0 - 2 + lj;
        const int ti = T0.i0 - 2 + 2 * kk + (tj & 1);
        const bool in = lj < TY + 4 && (L.bcx || (ti >= 0 && ti < L.m1)) && (L.bcy || (tj >= 0 && tj < L.m2));
        if (in) {
            const int i = L.bcx ? wrapi(ti, L.m1) : ti, j = L.bcy ? wrapi(tj, L.m2) : tj;
            relax_cell<true, 0>(P, L, T, F, nullptr, nullptr, i, j, ti, tj, hlf, omega, 1.0);
        }
    }
    __syncthreads();
    fused_refresh(L, T);
    __syncthreads();
    if (threadIdx.x < TBLK) {
        // black cells of the tile: the box faces go to buffer par ^ 1
        const int lj = pr / (TX / 2), kk = pr - lj * (TX / 2);
        const int j = T0.j0 + lj;
        const int i = T0.i0 + 2 * kk + ((j + 1) & 1);
        if (i < L.m1 && j < L.m2) relax_cell<false, 0>(P, O, T, F, d.ub[par ^ 1], d.vb[par ^ 1], i, j, i, j, hlf, omega, 1.0);
    } else {
        // red cells of the tile: their final values
        const int q = pr - TBLK / 2;
        const int lj = q / (TX / 2), kk = q - lj * (TX / 2);
        const int j = T0.j0 + lj;
        const int i = T0.i0 + 2 * kk + (j & 1);
        if (i < L.m1 && j < L.m2) {
            const int e = T.idx(i, j), n = T.W * T.H;
            const size_t g = (size_t)j * L.pitch + i;
            if (hlf == 0) { O.c[g] = T.s[T_C * n + e]; O.mu[g] = T.s[T_MU * n + e]; }
            else O.p[g] = T.s[T_P * n + e];
        }
    }
}

// plain copy, used to measure the copy bandwidth and to calibrate counters
__global__ __launch_bounds__(BLK) void k_copy_probe(const double *__restrict__ a, double *__restrict__ b, size_t n)
{
    for (size_t q = (size_t)blockIdx.x * BLK + threadIdx.x; q < n; q += (size_t)gridDim.x * BLK) b[q] = a[q];
}

// LDS doubles of the level-resident solve: 15 per cell (the level arrays and
// right-hand sides take 12) + one tile + the tile's source map (4 ints per
// element)
__host__ __device__ inline size_t coarse_lds_doubles(int m1, int m2)
{
    return (size_t)15 * m1 * m2 + (size_t)(T_NF + 2) * (m1 + 3) * (m2 + 3);
}

// all sweeps of a level in one workgroup per item, with the whole level
// resident in LDS: the solve of the coarsest level, and the pre- and
// post-smoothing of coarse levels small enough (the same arithmetic as the
// half-sweep launches); the u/v buffers alternate, the number of half-sweeps
// is even, so the result stays in buffer par.  With prolong set the level
// first takes the coarse-grid correction (k_prolong's arithmetic) as it is
// loaded.
template <typename IT>
__global__ __launch_bounds__(512) void k_coarse_solve(IT it, int sweeps, double omega, double pomega, int prolong)
{
    extern __shared__ double sm[];
    const int k = find_item(it);
    const Desc &d = *it.d[k];
    // the constants by value (no store can change them, so they are not
    // reloaded after one); the relaxation works on LDS arrays (address space 3)
    const Phys P = d.P;
    const int par = it.par[k];
    const View L = view_of(d, par);
    double *ua = d.ub[par], *va = d.vb[par];
    const int m1 = L.m1, m2 = L.m2, n = m1 * m2;
    double *hc = sm, *hmu = sm + n, *hp = sm + 2 * n, *uA = sm + 3 * n, *vA = sm + 4 * n, *uB = sm + 5 * n,
           *vB = sm + 6 * n, *hf = sm + 7 * n;
    Tile T;
    T.s = sm + 15 * n; T.i0 = 0; T.j0 = 0; T.W = m1 + 3; T.H = m2 + 3;
    const int nt = T.W * T.H;
    int *map = (int *)(T.s + (size_t)T_NF * nt);
    // one pass over the tile's elements: each loads its sources from the level
    // arrays (the boundary images of tile_load), adds the coarse-grid
    // correction of each source, and fills the tile (with the cell functions),
    // the refresh map (level indices in LDS, as tile_map_build) and, for an
    // element that is a cell of the level, the level arrays in LDS and the
    // right-hand sides
    PSrc ps = {};
    if (prolong) ps = psrc_of(d, d.coarse, it.cpar[k]);
    // the right-hand sides' arrays read before the first store (read after
    // one, every element would reload them from the descriptor)
    const double *const rfc = d.fc, *const rfmu = d.fmu, *const rfp = d.fp, *const rfu = d.fu, *const rfv = d.fv;
    for (int e = threadIdx.x; e < nt; e += block_threads()) {
        const int b = e / T.W, a = e - b * T.W;
        const int i = a - 1, j = b - 1;
        const TileSrcIJ q = tile_src_ij(m1, m2, L.bcx, L.bcy, i, j);
        const size_t kc = (size_t)q.jc * L.pitch + q.ic, ku = (size_t)q.ju * L.pitch + q.iu,
                     kv = (size_t)q.jv * L.pitch + q.iv;
        const bool cell = i >= 0 && i < m1 && j >= 0 && j < m2;
        const size_t ql = cell ? (size_t)j * L.pitch + i : 0;
        // every load of the element before any use: its sources, the
        // right-hand sides (a cell of the level; index 0 otherwise, not used)
        // and the coarse values of the correction at each source
        double c = lda<1>(L.c, kc), mu = lda<1>(L.mu, kc), p = lda<1>(L.p, kc), u = lda<1>(ua, ku),
               v = lda<1>(va, kv);
        const double cn = lda<1>(L.cn, kc), un = lda<1>(L.un, ku), vn = lda<1>(L.vn, kv);
        const double f0 = rfc ? lda<1>(rfc, ql) : 0.0, f1 = rfmu ? lda<1>(rfmu, ql) : 0.0,
                     f2 = rfp ? lda<1>(rfp, ql) : 0.0, f3 = rfu ? lda<1>(rfu, ql) : 0.0,
                     f4 = rfv ? lda<1>(rfv, ql) : 0.0;
        PRaw raw = {};
        if (prolong) raw = prolong_load(ps, q.ic, q.jc, q.iu, q.ju, q.iv, q.jv);
        __builtin_amdgcn_sched_barrier(0);
        if (prolong) {
            double rc, rm, rp, du, dv;
            prolong_apply(ps, raw, q.iu, q.iv, q.jv, rc, rm, rp, du, dv);
            c += rc; mu += rm; p += rp;
            if (ps.bcx || q.iu >= 1) u += du;
            if (ps.bcy || q.jv >= 1) v += dv;
        }
        const bool out = i > m1 + 1 || j > m2 + 1;
        map[4 * e] = q.jc * m1 + q.ic;
        map[4 * e + 1] = q.ju * m1 + q.iu;
        map[4 * e + 2] = q.jv * m1 + q.iv;
        map[4 * e + 3] = (q.su + 1) | ((q.sv + 1) << 2) | (((q.ic + q.jc) & 1) << 5) | (out ? 16 : 0);
        double *t = T.s + e;
        if (q.sc == 0) {
            for (int f = 0; f < T_NF; f++) t[f * nt] = 0.0;
        } else {
            t[T_C * nt] = c;
            t[T_MU * nt] = mu;
            t[T_P * nt] = p;
            t[T_U * nt] = signed_val(q.su, u);
            t[T_V * nt] = signed_val(q.sv, v);
            t[T_CN * nt] = cn;
            t[T_UN * nt] = signed_val(q.su, un);
            t[T_VN * nt] = signed_val(q.sv, vn);
            t[T_RN * nt] = rho_of(P, cn);
            t[T_MV * nt] = visc_of(P, cn);
            t[T_MOB * nt] = mob_of(P, cn);
            t[T_RS * nt] = rho_of(P, c);
        }
        if (cell) {
            // a cell of the level: its own source for every field
            const int el = j * m1 + i;
            hc[el] = c; hmu[el] = mu; hp[el] = p; uA[el] = u; vA[el] = v;
            hf[el] = f0;
            hf[n + el] = f1;
            hf[2 * n + el] = f2;
            hf[3 * n + el] = f3;
            hf[4 * n + el] = f4;
        }
    }
    __syncthreads();
    View H = L;
    H.c = hc; H.mu = hmu; H.p = hp; H.pitch = m1;
    const Rhs FH = { hf, hf + n, hf + 2 * n, hf + 3 * n, hf + 4 * n };
    const int half = m1 >> 1;
    for (int s = 0; s < 2 * sweeps; s++) {
        const int colour = s & 1;
        double *uw, *vw;
        if (s & 1) { H.u = uB; H.v = vB; uw = uA; vw = vA; }
        else { H.u = uA; H.v = vA; uw = uB; vw = vB; }
        if (s > 0) {
            tile_refresh_map(P, H, T, map, colour ^ 1);
            __syncthreads();
        }
        for (int t = threadIdx.x; t < 2 * half * m2; t += block_threads()) {
            const int pr = t >> 1;
            const int j = pr / half;
            const int i = 2 * (pr - j * half) + ((j + colour) & 1);
            relax_pair<3>(P, H, T, FH, uw, vw, i, j, t & 1, omega, pomega);
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < n; e += block_threads()) {
        const int j = e / m1, i = e - j * m1;
        const size_t q = (size_t)j * L.pitch + i;
        L.c[q] = hc[e]; L.mu[q] = hmu[e]; L.p[q] = hp[e]; ua[q] = uA[e]; va[q] = vA[e];
    }
}

// R w of a coarse cell from the values of its four children (a, b: the
// children (0, 0), (1, 0); c, d: (0, 1), (1, 1)): the mean, summed in the order
// k_restrict sums the children's residuals
__device__ __forceinline__ double rw_mean(double a, double b, double c, double d)
{
    return 0.25 * ((a + b) + (c + d));
}

// fine residual r = f - N(w) restricted to the coarse grid together with the
// iterate (cells: mean of the four children; faces: mean of the two coincident
// fine faces), and the FAS right-hand side f_H = N_H(R w) + R r of the coarse
// cells.  A tile of fine cells covers (TX/2) x (TY/2) coarse cells, one lane
// pair each; N_H is evaluated on a coarse tile whose halo takes R w from the
// fine arrays directly (the neighbouring workgroups write the coarse iterate
// meanwhile).
#define RBLK (2 * TBLK)
template <typename IT> __global__ __launch_bounds__(RBLK) void k_restrict(IT it)
{
    __shared__ double sm[TILE_DOUBLES];
    __shared__ double smc[T_NF * (TX / 2 + 3) * (TY / 2 + 3)];
    // sums of the three fine cells of a coarse cell other than its (0, 0)
    // child: the x lane's residuals and iterate (rc, rm, rp, rf, c, mu, p,
    // u face), the y lane's face residual and v face
    __shared__ double part[3][(TX / 2) * (TY / 2)][10];
    const int k = find_item(it);
    const Desc &d = *it.d[k];
    if (!tile_valid(it, k, d)) return;
    const Desc &C = *d.coarse;
    // the coarse constants stay by reference: held by value they raised the
    // kernel from 120 to 143 VGPRs (one workgroup less per compute unit)
    const Phys P = d.P;
    const Phys &PC = C.P;
    const int cp = it.cpar[k];
    const View Lf = view_of(d, it.par[k]);
    const View Lc = view_of(C, cp);
    const Tile T = item_tile(sm, it, k, d);
    tile_load(P, Lf, T);
    // the coarse tile of R w, from the fine arrays directly (its halo lies
    // in the neighbouring workgroups' tiles), loaded together with the fine
    // tile: cells the mean of the four children, faces the mean of the two
    // coincident fine faces
    Tile Tc;
    Tc.s = smc; Tc.i0 = T.i0 / 2; Tc.j0 = T.j0 / 2; Tc.W = TX / 2 + 3; Tc.H = TY / 2 + 3;
    {
        const int n = Tc.W * Tc.H;
        for (int e = threadIdx.x; e < n; e += block_threads()) {
            const int bb = e / Tc.W, aa = e - bb * Tc.W;
            const TileSrc s = tile_src(C.m1, C.m2, C.pitch, C.bcx, C.bcy, Tc.i0 - 1 + aa, Tc.j0 - 1 + bb);
            double *t = Tc.s + e;
            if (s.sc == 0) {
                for (int f = 0; f < T_NF; f++) t[f * n] = 0.0;
                continue;
            }
            const int Ic = s.c % C.pitch, Jc = s.c / C.pitch;
            const int Iu = s.u % C.pitch, Ju = s.u / C.pitch, Iv = s.v % C.pitch, Jv = s.v / C.pitch;
            const size_t fu = (size_t)(2 * Ju) * Lf.pitch + 2 * Iu, fv = (size_t)(2 * Jv) * Lf.pitch + 2 * Iv;
            // every load before any use (the faces of a wall: loaded in any
            // case, the indices are valid)
            const size_t fa = (size_t)(2 * Jc) * Lf.pitch + 2 * Ic, fb = fa + Lf.pitch;
            const double c4[4] = { lda<1>(Lf.c, fa), lda<1>(Lf.c, fa + 1), lda<1>(Lf.c, fb), lda<1>(Lf.c, fb + 1) };
            const double m4[4] = { lda<1>(Lf.mu, fa), lda<1>(Lf.mu, fa + 1), lda<1>(Lf.mu, fb), lda<1>(Lf.mu, fb + 1) };
            const double p4[4] = { lda<1>(Lf.p, fa), lda<1>(Lf.p, fa + 1), lda<1>(Lf.p, fb), lda<1>(Lf.p, fb + 1) };
            const double u0 = lda<1>(Lf.u, fu), u1 = lda<1>(Lf.u, fu + Lf.pitch);
            const double w0 = lda<1>(Lf.v, fv), w1 = lda<1>(Lf.v, fv + 1);
            const double cn = lda<1>(C.cn, s.c), un = lda<1>(C.un, s.u), vn = lda<1>(C.vn, s.v);
            __builtin_amdgcn_sched_barrier(0);
            const double c = rw_mean(c4[0], c4[1], c4[2], c4[3]);
            const double u = s.su ? 0.5 * (u0 + u1) : 0.0;
            const double w = s.sv ? 0.5 * (w0 + w1) : 0.0;
            t[T_C * n] = c;
            t[T_MU * n] = rw_mean(m4[0], m4[1], m4[2], m4[3]);
            t[T_P * n] = rw_mean(p4[0], p4[1], p4[2], p4[3]);
            t[T_U * n] = signed_val(s.su, u);
            t[T_V * n] = signed_val(s.sv, w);
            t[T_CN * n] = cn;
            t[T_UN * n] = signed_val(s.su, un);
            t[T_VN * n] = signed_val(s.sv, vn);
            t[T_RN * n] = rho_of(PC, cn);
            t[T_MV * n] = visc_of(PC, cn);
            t[T_MOB * n] = mob_of(PC, cn);
            t[T_RS * n] = rho_of(PC, c);
        }
    }
    __syncthreads();
    // lane pair pr: coarse cell cc of the tile, fine child (a, b) = (ch & 1,
    // ch >> 1) of it; children other than (0, 0) hand their values to the
    // (0, 0) pair through LDS
    const int pr = threadIdx.x >> 1, hlf = threadIdx.x & 1;
    const int NC = (TX / 2) * (TY / 2);
    const int cc = pr % NC, ch = pr / NC, a = ch & 1, b = ch >> 1;
    const int I = T.i0 / 2 + cc % (TX / 2), J = T.j0 / 2 + cc / (TX / 2);
    const bool on = I < C.m1 && J < C.m2;
    double v[8] = { 0, 0, 0, 0, 0, 0, 0, 0 }; // rc, rm, rp, rf, c, mu, p, face
    if (on) {
        const int i = 2 * I + a, j = 2 * J + b;
        double xc, xm, xp, xf;
        resid_pair(P, Lf, T, rhs_of(d), i, j, hlf, xc, xm, xp, xf);
        v[0] = xc; v[1] = xm; v[2] = xp;
        // the lane's faces of the coarse cell: west faces (a = 0) on the x
        // lane, south faces (b = 0) on the y lane
        if ((hlf ? b : a) == 0) { v[3] = xf; v[7] = T.q(hlf ? T_V : T_U, i, j); }
        v[4] = T.q(T_C, i, j); v[5] = T.q(T_MU, i, j); v[6] = T.q(T_P, i, j);
        if (ch > 0) {
            double *o = part[ch - 1][cc];
            if (hlf == 0) {
#pragma unroll
                for (int q = 0; q < 8; q++) o[q] = v[q];
            } else {
                o[8] = v[3];
                o[9] = v[7];
            }
        }
    }
    __syncthreads();
    if (!on || ch != 0) return;
    // sums over the four children as (0,0) + (1,0) plus (0,1) + (1,1), the
    // order in which the coarse tile's R w was summed (rw_mean)
    if (hlf == 0) {
#pragma unroll
        for (int q = 0; q < 8; q++) v[q] = (v[q] + part[0][cc][q]) + (part[1][cc][q] + part[2][cc][q]);
    } else {
#pragma unroll
        for (int g = 0; g < 3; g++) {
            v[3] += part[g][cc][8];
            v[7] += part[g][cc][9];
        }
    }
    const size_t q = (size_t)J * C.pitch + I;
    if (hlf == 0) {
        C.c[q] = C.c0[q] = 0.25 * v[4];
        C.mu[q] = C.mu0[q] = 0.25 * v[5];
        C.p[q] = C.p0[q] = 0.25 * v[6];
        C.ub[cp][q] = C.u0[q] = 0.5 * v[7];
    } else {
        C.vb[cp][q] = C.v0[q] = 0.5 * v[7];
    }
    // f_H = N_H(R w) + R r on the coarse cell
    const Rhs Z = { nullptr, nullptr, nullptr, nullptr, nullptr };
    double rc, rm, rp, rf;
    resid_pair(PC, Lc, Tc, Z, I, J, hlf, rc, rm, rp, rf); // r = -N_H(R w)
    if (hlf == 0) {
        C.fc[q] = 0.25 * v[0] - rc;
        C.fmu[q] = 0.25 * v[1] - rm;
        C.fp[q] = 0.25 * v[2] - rp;
        C.fu[q] = u_unk(Lc, I) ? 0.5 * v[3] - rf : 0.0;
    } else {
        C.fv[q] = v_unk(Lc, J) ? 0.5 * v[3] - rf : 0.0;
    }
}

// the two cells of a tile handled by lane pair pr: (2k, lj) and (2k+1, lj)
template <typename TT> __device__ __forceinline__ void pair_cells(const TT &T, int &i, int &j)
{
    const int pr = threadIdx.x >> 1;
    const int lj = pr / (TX / 2), kk = pr - lj * (TX / 2);
    i = T.i0 + 2 * kk;
    j = T.j0 + lj;
}

// w_h += P(w_H - R w_h) on the level the item names, one thread per fine cell
template <typename IT> __global__ __launch_bounds__(BLK) void k_prolong(IT it)
{
    const int k = find_item(it);
    const Desc &d = *it.d[k];
    const Desc &C = *d.coarse;
    const int t = ((int)blockIdx.x - it.start[k]) * BLK + threadIdx.x;
    if (t >= d.m1 * d.m2) return;
    const int j = t / d.m1, i = t - j * d.m1;
    const size_t kf = (size_t)j * d.pitch + i;
    // the correction of the cell and its west and south faces, every load
    // issued before any use
    const PSrc ps = psrc_of(d, &C, it.cpar[k]);
    double *ub = d.ub[it.par[k]], *vb = d.vb[it.par[k]];
    const PRaw raw = prolong_load(ps, i, j, i, j, i, j);
    const double c = lda<1>(d.c, kf), mu = lda<1>(d.mu, kf), p = lda<1>(d.p, kf), u = lda<1>(ub, kf),
                 v = lda<1>(vb, kf);
    __builtin_amdgcn_sched_barrier(0);
    double rc, rm, rp, du, dv;
    prolong_apply(ps, raw, i, i, j, rc, rm, rp, du, dv);
    sta<1>(d.c, kf, c + rc);
    sta<1>(d.mu, kf, mu + rm);
    sta<1>(d.p, kf, p + rp);
    if (ps.bcx || i >= 1) sta<1>(ub, kf, u + du);
    if (ps.bcy || j >= 1) sta<1>(vb, kf, v + dv);
}

// wave64 + LDS block sum of NRED values (blocks of up to 16 waves)
__device__ __forceinline__ void block_sum_store(double (&v)[NRED], double *out)
{
    __shared__ double sh[16][NRED];
#pragma unroll
    for (int q = 0; q < NRED; q++)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0)
#pragma unroll
        for (int q = 0; q < NRED; q++) sh[w][q] = v[q];
    __syncthreads();
    if (threadIdx.x < NRED) {
        double s = 0.0;
        for (int ww = 0; ww < (int)(block_threads() >> 6); ww++) s += sh[ww][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// Acceleration of the cycle iteration, recording of a cycle result in ring
// slot s: the residual and the iterate of the cell at index w (lane 0: c,
// mubar, pbar and the west face; lane 1: the south face).
template <typename TT>
__device__ __forceinline__ void acc_put(const Desc &d, int s, size_t w, int hlf, double rc, double rm, double rp,
                                        double rf, const TT &T, int i, int j)
{
    const size_t st = (size_t)d.pitch * d.m2;
    double *ar = d.ar + (size_t)s * 5 * st + w, *aw = d.aw + (size_t)s * 5 * st + w;
    if (hlf == 0) {
        ar[0] = rc; ar[st] = rm; ar[2 * st] = rp; ar[3 * st] = rf;
        aw[0] = T.q(T_C, i, j); aw[st] = T.q(T_MU, i, j); aw[2 * st] = T.q(T_P, i, j); aw[3 * st] = T.q(T_U, i, j);
    } else {
        ar[4 * st] = rf;
        aw[4 * st] = T.q(T_V, i, j);
    }
}
// ... and the lane's share of the normal equations of
// min || r + sum_a g_a (r - r_a) ||, r_a the residual a + 1 slots back
// (a < np): v[7 + b(b+1)/2 + a] += e_a e_b (a <= b), v[13 + a] += e_a r,
// e_a = r - r_a.  Reads back what acc_put of the same lane wrote (the
// residuals' registers are free by then), all slots of all the lane's fields
// (lane 0: four, lane 1: one) before the first product.
__device__ __forceinline__ void acc_dots(const Desc &d, int ac, size_t w, int hlf, double (&v)[NRED])
{
    const int s = ac & 15, np = ac >> 4, R = d.am;
    const size_t st = (size_t)d.pitch * d.m2;
    const int nf = hlf ? 1 : 4;
    double x[4], old[4][3];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int f = hlf ? 4 : q;
        x[q] = q < nf ? d.ar[(size_t)(s * 5 + f) * st + w] : 0.0;
#pragma unroll
        for (int a = 0; a < 3; a++)
            old[q][a] = (q < nf && a < np) ? d.ar[(size_t)(((s - 1 - a + R) % R) * 5 + f) * st + w] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
        if (q >= nf) continue;
        double e[3] = { 0.0, 0.0, 0.0 };
#pragma unroll
        for (int a = 0; a < 3; a++)
            if (a < np) e[a] = x[q] - old[q][a];
#pragma unroll
        for (int b = 0; b < 3; b++)
#pragma unroll
            for (int a = 0; a <= b; a++) v[7 + b * (b + 1) / 2 + a] += e[a] * e[b];
#pragma unroll
        for (int a = 0; a < 3; a++) v[13 + a] += e[a] * x[q];
    }
}

// residual norms of a finest level: per tile sums of r^2 for the five
// equations, the sum of pbar, and the count of cells that are non-finite or
// past the density pole (partials indexed by the tile's place in the band
// order); optionally the residual fields themselves
template <typename IT> __global__ __launch_bounds__(TBLK) void k_resid_norm(IT it)
{
    __shared__ double sm[TILE_DOUBLES];
    const int k = find_item(it);
    const Desc &d = *it.d[k];
    if (!tile_valid(it, k, d)) return;
    const Phys P = d.P;
    const View L = view_of(d, it.par[k]);
    const Tile T = item_tile(sm, it, k, d);
    tile_load(P, L, T);
    __syncthreads();
    double v[NRED] = {};
    const size_t n = (size_t)L.m1 * L.m2;
    const int hlf = threadIdx.x & 1;
    const Rhs F = rhs_of(d);
    int i, j;
    pair_cells(T, i, j);
    for (int a = 0; a < 2; a++, i++) {
        if (i >= L.m1 || j >= L.m2) continue;
        double rc, rm, rp, rf;
        resid_pair(P, L, T, F, i, j, hlf, rc, rm, rp, rf);
        const size_t q = (size_t)j * L.m1 + i;
        v[3 + hlf] += rf * rf;
        if (d.rout) d.rout[(3 + hlf) * n + q] = rf;
        if (d.rc) {
            // mixed precision: the right-hand side and linearisation point of
            // the next correction cycle, whose correction starts at zero
            const size_t w = (size_t)j * L.pitch + i;
            const int par = it.par[k];
            if (hlf == 0) {
                d.rc[w] = (float)rc; d.rmu[w] = (float)rm; d.rp[w] = (float)rp; d.ru[w] = (float)rf;
                d.xc[w] = (float)T.q(T_C, i, j); d.xmu[w] = (float)T.q(T_MU, i, j);
                d.xu[w] = (float)T.q(T_U, i, j);
                d.dc[w] = 0.0f; d.dmu[w] = 0.0f; d.dp[w] = 0.0f; d.dub[par][w] = 0.0f;
            } else {
                d.rv[w] = (float)rf;
                d.xv[w] = (float)T.q(T_V, i, j);
                d.dvb[par][w] = 0.0f;
            }
        }
        if (hlf == 0) {
            v[0] += rc * rc; v[1] += rm * rm; v[2] += rp * rp;
            const double c = T.q(T_C, i, j), pp = T.q(T_P, i, j);
            v[5] += pp;
            const bool ok = isfinite(c) && isfinite(T.q(T_MU, i, j)) && isfinite(pp) && isfinite(T.q(T_U, i, j))
                          && isfinite(T.q(T_V, i, j)) && (P.drho * c + P.rho1 > 0.0);
            v[6] += ok ? 0.0 : 1.0;
            if (d.rout) { d.rout[q] = rc; d.rout[n + q] = rm; d.rout[2 * n + q] = rp; }
        }
        if (it.acc[k] >= 0 && d.ar) acc_put(d, it.acc[k] & 15, (size_t)j * L.pitch + i, hlf, rc, rm, rp, rf, T, i, j);
    }
    // the normal equations after the residuals, whose registers are free by now
    if (it.acc[k] >= 0 && d.ar && (it.acc[k] >> 4) > 0) {
        pair_cells(T, i, j);
#pragma unroll 1
        for (int a = 0; a < 2; a++, i++)
            if (i < L.m1 && j < L.m2) acc_dots(d, it.acc[k], (size_t)j * L.pitch + i, hlf, v);
    }
    const int tl = (T.j0 / TY) * it.tx[k] + T.i0 / TX;
    block_sum_store(v, d.partials + (size_t)tl * NRED);
}

// mass and energy partial sums of the current state, one thread per cell
template <typename IT> __global__ __launch_bounds__(BLK) void k_mass_energy(IT it)
{
    const int k = find_item(it);
    const Desc &d = *it.d[k];
    const View L = view_of(d, it.par[k]);
    const Phys &P = d.P;
    const int b = (int)blockIdx.x - it.start[k];
    const int t = b * BLK + threadIdx.x;
    double v[NRED] = {};
    if (t < L.m1 * L.m2) {
        const int j = t / L.m1, i = t - j * L.m1;
        const size_t q = (size_t)j * L.pitch + i;
        const double c = L.c[q], r = rho_of(P, c);
        v[0] = r * c;
        v[1] = r * (1.0 - c);
        const double cw = ldc(L.c, L.m1, L.m2, L.pitch, L.bcx, L.bcy, i - 1, j);
        const double cs = ldc(L.c, L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j - 1);
        const double rw = rho_of(P, cw), rs = rho_of(P, cs);
        // kinetic energy on the west and south faces of the cell (App. A.7)
        if (u_unk(L, i)) { const double u = L.u[q]; v[2] += 0.25 * (r + rw) * u * u; }
        if (v_unk(L, j)) { const double w = L.v[q]; v[2] += 0.25 * (r + rs) * w * w; }
        // gradient energy [rho D c, D c] on the same faces (walls carry none)
        if (L.bcx || i > 0) { const double g = (c - cw) * L.inv_h; v[3] += 0.5 * (r + rw) * g * g; }
        if (L.bcy || j > 0) { const double g = (c - cs) * L.inv_h; v[3] += 0.5 * (r + rs) * g * g; }
        v[4] = r * dwell(c);
        v[5] = (r - P.rho_ref) * (j + 0.5) * d.h;
    }
    block_sum_store(v, d.partials + (size_t)b * NRED);
}

// Dissipation of the step just taken (Theorem of sec. 6.1 with the norms of
// App. A.7), from the new iterate and the time-n data still held by the
// level: partial sums, per cell, of
//   0: mu(c^n) (|d_x u|^2 + |d_y v|^2 + 1/4 sum over the 4 corners of
//      |calD_y u|^2 + |calD_x v|^2)        (viscous gradient norm)
//   1: mu(c^n) (d_x u + d_y v)^2           (viscous divergence norm)
//   2: A m(c^n) |D mu_c|^2 on the west and south faces, mu_c = mubar + alpha pbar
//   3: A rho^n |u - u^n|^2 on the west and south faces (unknown faces only)
// One thread per cell.
template <typename IT> __global__ __launch_bounds__(BLK) void k_dissipation(IT it)
{
    const int k = find_item(it);
    const Desc &d = *it.d[k];
    // projection scheme: the viscous parts and the time-difference part are
    // taken on the intermediate velocity (the other face buffer), and slot 4
    // sums A rho(c) (u^{n+1} - u~)^2 over the faces
    const bool pj = d.P.scheme != 0;
    const View L = view_of(d, pj ? it.par[k] ^ 1 : it.par[k]);
    const double *uf = d.ub[it.par[k]], *vf = d.vb[it.par[k]];
    const Phys &P = d.P;
    const int b = (int)blockIdx.x - it.start[k];
    const int t = b * BLK + threadIdx.x;
    double v[NRED] = {};
    if (t < L.m1 * L.m2) {
        const int j = t / L.m1, i = t - j * L.m1;
        const int m1 = L.m1, m2 = L.m2, pt = L.pitch, bx = L.bcx, by = L.bcy;
        const double ih = L.inv_h;
        auto U = [&](int a, int c) { return ldu(L.u, m1, m2, pt, bx, by, a, c); };
        auto V = [&](int a, int c) { return ldv(L.v, m1, m2, pt, bx, by, a, c); };
        auto CN = [&](int a, int c) { return ldc(L.cn, m1, m2, pt, bx, by, a, c); };
        const double mv = visc_of(P, CN(i, j));
        const double dxu = (U(i + 1, j) - U(i, j)) * ih, dyv = (V(i, j + 1) - V(i, j)) * ih;
        double sv = 0.0;
#pragma unroll
        for (int a = 0; a <= 1; a++)
#pragma unroll
            for (int c = 0; c <= 1; c++) {
                const double dyu = (U(i + a, j + c) - U(i + a, j + c - 1)) * ih;
                const double dxv = (V(i + a, j + c) - V(i + a - 1, j + c)) * ih;
                sv += dyu * dyu + dxv * dxv;
            }
        v[0] = mv * (dxu * dxu + dyv * dyv + 0.25 * sv);
        v[1] = mv * (dxu + dyv) * (dxu + dyv);
        const double c0 = CN(i, j), mob0 = mob_of(P, c0), r0 = rho_of(P, c0);
        const double mu0 = ldc(L.mu, m1, m2, pt, bx, by, i, j), p0 = ldc(L.p, m1, m2, pt, bx, by, i, j);
        const size_t q = (size_t)j * pt + i;
        if (bx || i > 0) {
            const double cw = CN(i - 1, j);
            const double g = (mu0 - ldc(L.mu, m1, m2, pt, bx, by, i - 1, j)) * ih
                           + P.alpha * (p0 - ldc(L.p, m1, m2, pt, bx, by, i - 1, j)) * ih;
            v[2] += 0.5 * (mob0 + mob_of(P, cw)) * g * g;
            const double du = L.u[q] - L.un[q];
            v[3] += 0.5 * (r0 + rho_of(P, cw)) * du * du;
            if (pj) {
                const double dp = uf[q] - L.u[q];
                v[4] += 0.5 * (rho_of(P, L.c[q]) + rho_of(P, ldc(L.c, m1, m2, pt, bx, by, i - 1, j))) * dp * dp;
            }
        }
        if (by || j > 0) {
            const double cs = CN(i, j - 1);
            const double g = (mu0 - ldc(L.mu, m1, m2, pt, bx, by, i, j - 1)) * ih
                           + P.alpha * (p0 - ldc(L.p, m1, m2, pt, bx, by, i, j - 1)) * ih;
            v[2] += 0.5 * (mob0 + mob_of(P, cs)) * g * g;
            const double dv = L.v[q] - L.vn[q];
            v[3] += 0.5 * (r0 + rho_of(P, cs)) * dv * dv;
            if (pj) {
                const double dp = vf[q] - L.v[q];
                v[4] += 0.5 * (rho_of(P, L.c[q]) + rho_of(P, ldc(L.c, m1, m2, pt, bx, by, i, j - 1))) * dp * dp;
            }
        }
    }
    block_sum_store(v, d.partials + (size_t)b * NRED);
}

// Projection scheme, end of a converged step: the velocity of time n+1 from
// the projection equation (pj-num-pjx) (as face_final) on every west and
// south face, written to the other face buffer, which becomes the current
// one; the intermediate velocity stays in buffer par for the dissipation.
template <typename IT> __global__ __launch_bounds__(BLK) void k_pj_final(IT it)
{
    const int k = find_item(it);
    const Desc &d = *it.d[k];
    const int par = it.par[k];
    const View L = view_of(d, par);
    const Phys &P = d.P;
    const int t = ((int)blockIdx.x - it.start[k]) * BLK + threadIdx.x;
    if (t >= L.m1 * L.m2) return;
    const int j = t / L.m1, i = t - j * L.m1;
    const int m1 = L.m1, m2 = L.m2, pt = L.pitch, bx = L.bcx, by = L.bcy;
    const double ih = L.inv_h;
    const size_t q = (size_t)j * pt + i;
    const double c0 = L.c[q], mu0 = L.mu[q], p0 = L.p[q], r0 = rho_of(P, c0);
    double uf = 0.0, vf = 0.0;
    if (bx || i > 0) {
        const double cw = ldc(L.c, m1, m2, pt, bx, by, i - 1, j), rw = rho_of(P, cw), Ar = 0.5 * (rw + r0);
        const double st = 0.5 * (r0 * ldc(L.mu, m1, m2, pt, bx, by, i - 1, j) + rw * mu0) * (c0 - cw) * ih;
        uf = L.u[q] + P.dt * frcp(Ar) * (P.inv_M * (st - (p0 - ldc(L.p, m1, m2, pt, bx, by, i - 1, j)) * ih));
    }
    if (by || j > 0) {
        const double cs = ldc(L.c, m1, m2, pt, bx, by, i, j - 1), rs = rho_of(P, cs), Ar = 0.5 * (rs + r0);
        const double st = 0.5 * (r0 * ldc(L.mu, m1, m2, pt, bx, by, i, j - 1) + rs * mu0) * (c0 - cs) * ih;
        vf = L.v[q] + P.dt * frcp(Ar)
                        * (P.inv_M * (st - (p0 - ldc(L.p, m1, m2, pt, bx, by, i, j - 1)) * ih) - P.inv_Fr * (Ar - P.rho_ref));
    }
    d.ub[par ^ 1][q] = uf;
    d.vb[par ^ 1][q] = vf;
}

// Physical diagnostics of the current state (sec. 8), per-block partials:
//   0: sum c v_cell (v_cell = mean of the cell's south and north faces)
//   1: sum c
//   2: max |div_d u|            3: sum (div_d u)^2          4: sum div_d u
//   5: max height of a c = 1/2 crossing between vertically adjacent cells
//      (linear interpolation; walls in y: interior pairs only)
//   6: min height of such a crossing
//   7: max height of a crossing in the first column (x = h/2)
// (5-7 hold -inf / +inf where there is none.)
#define DIAG_NONE 1e300
template <typename IT> __global__ __launch_bounds__(BLK) void k_diagnostics(IT it)
{
    __shared__ double sh[BLK / 64][NRED];
    const int k = find_item(it);
    const Desc &d = *it.d[k];
    const View L = view_of(d, it.par[k]);
    const int b = (int)blockIdx.x - it.start[k];
    const int t = b * BLK + threadIdx.x;
    double v[NRED] = { 0, 0, 0, 0, 0, -DIAG_NONE, DIAG_NONE, -DIAG_NONE };
    if (t < L.m1 * L.m2) {
        const int j = t / L.m1, i = t - j * L.m1;
        const int m1 = L.m1, m2 = L.m2, pt = L.pitch, bx = L.bcx, by = L.bcy;
        const size_t q = (size_t)j * pt + i;
        const double c = L.c[q];
        const double vs = ldv(L.v, m1, m2, pt, bx, by, i, j), vn = ldv(L.v, m1, m2, pt, bx, by, i, j + 1);
        const double us = ldu(L.u, m1, m2, pt, bx, by, i, j), ue = ldu(L.u, m1, m2, pt, bx, by, i + 1, j);
        v[0] = c * 0.5 * (vs + vn);
        v[1] = c;
        const double dv = (ue - us + vn - vs) * L.inv_h;
        v[2] = fabs(dv);
        v[3] = dv * dv;
        v[4] = dv;
        if (by || j + 1 < m2) {
            const double cn = L.c[(size_t)(j + 1 < m2 ? j + 1 : 0) * pt + i];
            if ((c - 0.5) * (cn - 0.5) < 0.0) {
                const double y = (j + 0.5 + (0.5 - c) / (cn - c)) * d.h;
                v[5] = y;
                v[6] = y;
                if (i == 0) v[7] = y;
            }
        }
    }
    // wave and block reductions: sums for 0, 1, 3, 4; max for 2, 5, 7; min for 6
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int r = 0; r < NRED; r++) {
            const double w = __shfl_xor(v[r], o, 64);
            v[r] = (r == 2 || r == 5 || r == 7) ? fmax(v[r], w) : (r == 6 ? fmin(v[r], w) : v[r] + w);
        }
    }
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0)
#pragma unroll
        for (int r = 0; r < NRED; r++) sh[wv][r] = v[r];
    __syncthreads();
    if (threadIdx.x < NRED) {
        const int r = threadIdx.x;
        double acc = sh[0][r];
        for (int ww = 1; ww < BLK / 64; ww++) {
            const double w = sh[ww][r];
            acc = (r == 2 || r == 5 || r == 7) ? fmax(acc, w) : (r == 6 ? fmin(acc, w) : acc + w);
        }
        d.partials[(size_t)b * NRED + r] = acc;
    }
}

// fixed-order sum of a simulation's partials (one workgroup per item); the
// norms become sqrt(h^2 sum r^2); written to device and pinned host memory.
// mode 0: residual reduction (5 norms, sum p, bad count); 1: plain sums;
// 2: the diagnostics slots (sum, max or min per slot as in k_diagnostics).
template <typename IT> __global__ __launch_bounds__(BLK) void k_finalize(IT it, int mode)
{
    __shared__ double sh[BLK][NRED];
    const int k = blockIdx.x;
    if (k >= it.n) return;
    const Desc &d = *it.d[k];
    const int nblk = it.tx[k];
    // slot q combines by sum, or (diagnostics) by max (op 1) or min (op 2)
    auto op = [&](int q) { return mode != 2 ? 0 : (q == 2 || q == 5 || q == 7) ? 1 : (q == 6 ? 2 : 0); };
    auto comb = [&](int q, double a, double b) { const int o = op(q); return o == 0 ? a + b : (o == 1 ? fmax(a, b) : fmin(a, b)); };
    double s[NRED];
#pragma unroll
    for (int q = 0; q < NRED; q++) s[q] = op(q) == 0 ? 0.0 : (op(q) == 1 ? -DIAG_NONE : DIAG_NONE);
    for (int b = threadIdx.x; b < nblk; b += BLK)
#pragma unroll
        for (int q = 0; q < NRED; q++) s[q] = comb(q, s[q], d.partials[(size_t)b * NRED + q]);
#pragma unroll
    for (int q = 0; q < NRED; q++) sh[threadIdx.x][q] = s[q];
    __syncthreads();
    for (int o = BLK / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
#pragma unroll
            for (int q = 0; q < NRED; q++) sh[threadIdx.x][q] = comb(q, sh[threadIdx.x][q], sh[threadIdx.x + o][q]);
        __syncthreads();
    }
    if (threadIdx.x < NRED) {
        double x = sh[0][threadIdx.x];
        if (mode == 0 && threadIdx.x < 5) x = sqrt(d.h * d.h * x);
        d.red[threadIdx.x] = x;
        d.red_host[threadIdx.x] = x;
        // a recorded cycle result: the pbar mean k_shift_p removes from it
        if (mode == 0 && threadIdx.x == 5 && it.acc[k] >= 0 && d.amean)
            d.amean[it.acc[k] & 15] = x / (double)(d.m1 * d.m2);
    }
}

// pbar -= mean(pbar), the mean from the reduced sums
template <typename IT> __global__ __launch_bounds__(BLK) void k_shift_p(IT it)
{
    const int k = find_item(it);
    const Desc &d = *it.d[k];
    const int t = ((int)blockIdx.x - it.start[k]) * BLK + threadIdx.x;
    if (t >= d.m1 * d.m2) return;
    const int j = t / d.m1, i = t - j * d.m1;
    d.p[(size_t)j * d.pitch + i] -= d.red[5] / (double)(d.m1 * d.m2);
}

// coefficients of the accelerated combination, per item
template <int N> struct AccCoef {
    double g[N][3];
};

// Acceleration step of the cycle iteration: the current iterate w (the last
// cycle result, recorded in ring slot s) becomes w + sum_a g_a (w - w_a), w_a
// the result a + 1 slots back (a < np; its pbar less the mean removed from it,
// which makes it the iterate that result was).  Mixed precision: the next
// correction cycle's right-hand side becomes the same combination of the
// recorded residuals, its linearisation point the combined iterate.
template <typename IT, int N> __global__ __launch_bounds__(BLK) void k_accel(IT it, AccCoef<N> G)
{
    const int k = find_item(it);
    const Desc &d = *it.d[k];
    const int t = ((int)blockIdx.x - it.start[k]) * BLK + threadIdx.x;
    if (t >= d.m1 * d.m2 || !d.aw || it.acc[k] < 0) return;
    const int j = t / d.m1, i = t - j * d.m1;
    const size_t q = (size_t)j * d.pitch + i, st = (size_t)d.pitch * d.m2;
    const int ac = it.acc[k], s = ac & 15, np = ac >> 4, R = d.am, par = it.par[k];
    int sl[3];
#pragma unroll
    for (int b = 0; b < 3; b++) sl[b] = (s - 1 - b + R) % R;
    double *const live[5] = { d.c, d.mu, d.p, d.ub[par], d.vb[par] };
    const bool mixed = d.rc != nullptr;
    // every value the cell's combination needs, loaded before any use or
    // store (the stores into the live arrays would otherwise hold back the
    // next field's loads)
    // (global-typed, so that a wait for a scalar load does not also wait for
    // them)
    const double *const aw = d.aw, *const ar = d.ar, *const amean = d.amean;
    double x[5], w[5][3], am[3], xr[5], wr[5][3];
#pragma unroll
    for (int b = 0; b < 3; b++) am[b] = b < np ? lda<1>(amean, sl[b]) : 0.0;
#pragma unroll
    for (int f = 0; f < 5; f++) {
        x[f] = lda<1>(live[f], q);
        xr[f] = mixed ? lda<1>(ar, (size_t)(s * 5 + f) * st + q) : 0.0;
#pragma unroll
        for (int b = 0; b < 3; b++) {
            w[f][b] = b < np ? lda<1>(aw, (size_t)(sl[b] * 5 + f) * st + q) : 0.0;
            wr[f][b] = (mixed && b < np) ? lda<1>(ar, (size_t)(sl[b] * 5 + f) * st + q) : 0.0;
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    double y[5];
#pragma unroll
    for (int f = 0; f < 5; f++) {
        double a = x[f];
#pragma unroll
        for (int b = 0; b < 3; b++)
            if (b < np) {
                const double wb = w[f][b] - (f == 2 ? am[b] : 0.0);
                a += G.g[k][b] * (x[f] - wb);
            }
        y[f] = a;
        live[f][q] = a;
    }
    if (mixed) {
        float r[5];
#pragma unroll
        for (int f = 0; f < 5; f++) {
            double a = xr[f];
#pragma unroll
            for (int b = 0; b < 3; b++)
                if (b < np) a += G.g[k][b] * (xr[f] - wr[f][b]);
            r[f] = (float)a;
        }
        d.rc[q] = r[0]; d.rmu[q] = r[1]; d.rp[q] = r[2]; d.ru[q] = r[3]; d.rv[q] = r[4];
        d.xc[q] = (float)y[0]; d.xmu[q] = (float)y[1]; d.xu[q] = (float)y[3]; d.xv[q] = (float)y[4];
    }
}

// time-n data of the finest level = current iterate; keep mubar, pbar of time n
template <typename IT> __global__ __launch_bounds__(BLK) void k_begin(IT it)
{
    const int k = find_item(it);
    const Desc &d = *it.d[k];
    const int t = ((int)blockIdx.x - it.start[k]) * BLK + threadIdx.x;
    if (t >= d.m1 * d.m2) return;
    const int j = t / d.m1, i = t - j * d.m1;
    const size_t q = (size_t)j * d.pitch + i;
    const int par = it.par[k];
    d.cn[q] = d.c[q];
    d.un[q] = d.ub[par][q];
    d.vn[q] = d.vb[par][q];
    d.mus[q] = d.mu[q];
    d.ps[q] = d.p[q];
    if (d.cnf) {
        d.cnf[q] = (float)d.c[q];
        d.unf[q] = (float)d.ub[par][q];
        d.vnf[q] = (float)d.vb[par][q];
    }
}

// time-n data of the coarser level of the item's level
template <typename IT> __global__ __launch_bounds__(BLK) void k_restrict_n(IT it)
{
    const int k = find_item(it);
    const Desc &F = *it.d[k];
    const Desc &C = *F.coarse;
    const int t = ((int)blockIdx.x - it.start[k]) * BLK + threadIdx.x;
    if (t >= C.m1 * C.m2) return;
    const int J = t / C.m1, I = t - J * C.m1;
    const size_t f = (size_t)(2 * J) * F.pitch + 2 * I, q = (size_t)J * C.pitch + I;
    C.cn[q] = 0.25 * (F.cn[f] + F.cn[f + 1] + F.cn[f + F.pitch] + F.cn[f + F.pitch + 1]);
    C.un[q] = 0.5 * (F.un[f] + F.un[f + F.pitch]);
    C.vn[q] = 0.5 * (F.vn[f] + F.vn[f + 1]);
}

// restore the state of time n on the finest level (failed step)
template <typename IT> __global__ __launch_bounds__(BLK) void k_restore(IT it)
{
    const int k = find_item(it);
    const Desc &d = *it.d[k];
    const int t = ((int)blockIdx.x - it.start[k]) * BLK + threadIdx.x;
    if (t >= d.m1 * d.m2) return;
    const int j = t / d.m1, i = t - j * d.m1;
    const size_t q = (size_t)j * d.pitch + i;
    const int par = it.par[k];
    d.c[q] = d.cn[q];
    d.ub[par][q] = d.un[q];
    d.vb[par][q] = d.vn[q];
    d.mu[q] = d.mus[q];
    d.p[q] = d.ps[q];
}

} // namespace qn
