// qnsch_lib.hip -- kernels and host driver of the FP64 multigrid time step,
// behind the C ABI of include/qnsch.h.
//
// One step (sec. 6.1 solved as in sec. 7.1): fix the time-n data on every
// level, then run FAS V-cycles (red-black CH point Newton + Vanka box
// smoothing, residual restriction, coarse-grid correction) until every
// per-equation residual norm is below tol.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <algorithm>
#include <vector>

#include "qnsch.h"
#include "qnsch_dev.hpp"

using namespace qn;

#define BLK 256
#define NRED 8 // reduction slots per block

// ===========================================================================
// kernels

// Tiles of TX x TY cells; TX even so that the colour of a cell is fixed by its
// parity inside the tile.  Static LDS: T_NF * (TX+3) * (TY+3) doubles.  Tile
// kernels run TX*TY threads: a lane pair per cell of one colour (half-sweeps)
// or a lane pair per two cells (residual kernels).
#define TX 32
#define TY 16
#define TBLK (TX * TY)
#define TILE_DOUBLES (T_NF * (TX + 3) * (TY + 3))
static_assert(TILE_DOUBLES * 8 + 16 * NRED * 8 <= 65536, "tile exceeds 64 KiB of LDS");

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// Renumber the tiles so that XCD x gets a contiguous band of tiles (rows of
// the tile grid): neighbouring tiles, which read each other's halos, then
// share one L2.
#define NXCD 8
__device__ __forceinline__ int tile_id()
{
    const int n = gridDim.x * gridDim.y, lin = blockIdx.x + blockIdx.y * gridDim.x;
    return (n % NXCD == 0) ? (lin % NXCD) * (n / NXCD) + lin / NXCD : lin;
}
__device__ __forceinline__ Tile block_tile(double *sm)
{
    const int t = tile_id();
    Tile T;
    T.s = sm;
    T.i0 = (t % gridDim.x) * TX;
    T.j0 = (t / gridDim.x) * TY;
    T.W = TX + 3;
    T.H = TY + 3;
    return T;
}

// one colour half-sweep on a tile.  The finest level (no FAS right-hand side)
// and the coarse levels are separate kernels so that profiles tell them apart.
__device__ __forceinline__ void halfsweep_body(const Phys &P, const View &L, const Rhs &F, double *unew,
                                               double *vnew, int colour, double omega)
{
    __shared__ double sm[TILE_DOUBLES];
    const Tile T = block_tile(sm);
    tile_load(P, L, T);
    __syncthreads();
    const int pr = threadIdx.x >> 1, hlf = threadIdx.x & 1;
    const int lj = pr / (TX / 2), k = pr - lj * (TX / 2);
    const int j = T.j0 + lj;
    const int i = T.i0 + 2 * k + ((j + colour) & 1);
    if (i < L.m1 && j < L.m2) relax_pair(P, L, T, F, unew, vnew, i, j, hlf, omega);
}
__global__ __launch_bounds__(TBLK) void k_halfsweep_fine(Phys P, View L, double *unew, double *vnew, int colour,
                                                         double omega)
{
    const Rhs F = { nullptr, nullptr, nullptr, nullptr, nullptr };
    halfsweep_body(P, L, F, unew, vnew, colour, omega);
}
__global__ __launch_bounds__(TBLK) void k_halfsweep_coarse(Phys P, View L, Rhs F, double *unew, double *vnew,
                                                           int colour, double omega)
{
    halfsweep_body(P, L, F, unew, vnew, colour, omega);
}

// plain copy, used to measure the copy bandwidth and to calibrate counters
__global__ __launch_bounds__(BLK) void k_copy_probe(const double *__restrict__ a, double *__restrict__ b, size_t n)
{
    for (size_t k = (size_t)blockIdx.x * BLK + threadIdx.x; k < n; k += (size_t)gridDim.x * BLK) b[k] = a[k];
}

// LDS bytes of the coarsest-level solve: 15 level arrays + one tile
__host__ __device__ inline size_t coarse_lds_doubles(int m1, int m2)
{
    return (size_t)15 * m1 * m2 + (size_t)T_NF * (m1 + 3) * (m2 + 3);
}

// all sweeps of the coarsest level in one workgroup with the whole level
// resident in LDS; the u/v buffers alternate (a -> b -> a ...), the number of
// half-sweeps is even, so the result is in a
__global__ __launch_bounds__(512) void k_coarse_solve(Phys P, View L, Rhs F, double *ua, double *va, int sweeps,
                                                      double omega)
{
    extern __shared__ double sm[];
    const int m1 = L.m1, m2 = L.m2, n = m1 * m2;
    double *hc = sm, *hmu = sm + n, *hp = sm + 2 * n, *uA = sm + 3 * n, *vA = sm + 4 * n, *uB = sm + 5 * n,
           *vB = sm + 6 * n, *hcn = sm + 7 * n, *hun = sm + 8 * n, *hvn = sm + 9 * n, *hf = sm + 10 * n;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int j = e / m1, i = e - j * m1;
        const size_t k = (size_t)j * L.pitch + i;
        hc[e] = L.c[k]; hmu[e] = L.mu[k]; hp[e] = L.p[k]; uA[e] = ua[k]; vA[e] = va[k];
        hcn[e] = L.cn[k]; hun[e] = L.un[k]; hvn[e] = L.vn[k];
        hf[e] = F.fc ? F.fc[k] : 0.0;
        hf[n + e] = F.fmu ? F.fmu[k] : 0.0;
        hf[2 * n + e] = F.fp ? F.fp[k] : 0.0;
        hf[3 * n + e] = F.fu ? F.fu[k] : 0.0;
        hf[4 * n + e] = F.fv ? F.fv[k] : 0.0;
    }
    __syncthreads();
    View H = L;
    H.c = hc; H.mu = hmu; H.p = hp; H.cn = hcn; H.un = hun; H.vn = hvn; H.pitch = m1;
    const Rhs FH = { hf, hf + n, hf + 2 * n, hf + 3 * n, hf + 4 * n };
    Tile T;
    T.s = sm + 15 * n; T.i0 = 0; T.j0 = 0; T.W = m1 + 3; T.H = m2 + 3;
    const int half = m1 >> 1;
    for (int s = 0; s < 2 * sweeps; s++) {
        const int colour = s & 1;
        double *uw, *vw;
        if (s & 1) { H.u = uB; H.v = vB; uw = uA; vw = vA; }
        else { H.u = uA; H.v = vA; uw = uB; vw = vB; }
        tile_load(P, H, T);
        __syncthreads();
        for (int t = threadIdx.x; t < 2 * half * m2; t += blockDim.x) {
            const int pr = t >> 1;
            const int j = pr / half;
            const int i = 2 * (pr - j * half) + ((j + colour) & 1);
            relax_pair(P, H, T, FH, uw, vw, i, j, t & 1, omega);
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        const int j = e / m1, i = e - j * m1;
        const size_t k = (size_t)j * L.pitch + i;
        L.c[k] = hc[e]; L.mu[k] = hmu[e]; L.p[k] = hp[e]; ua[k] = uA[e]; va[k] = vA[e];
    }
}

struct Coarse {
    double *c, *mu, *p, *u, *v;
    double *c0, *mu0, *p0, *u0, *v0;
    double *fc, *fmu, *fp, *fu, *fv;
    int m1, m2, pitch;
};

// fine residual r = f - N(w) restricted to the coarse grid together with the
// iterate (cells: mean of the four children; faces: mean of the two coincident
// fine faces); the coarse rhs holds R r until k_coarse_rhs adds N_H(R w).
// A tile of fine cells covers (TX/2) x (TY/2) coarse cells, one lane pair each.
__global__ __launch_bounds__(TBLK) void k_restrict(Phys P, View Lf, Rhs F, Coarse C)
{
    __shared__ double sm[TILE_DOUBLES];
    const Tile T = block_tile(sm);
    tile_load(P, Lf, T);
    __syncthreads();
    const int pr = threadIdx.x >> 1, hlf = threadIdx.x & 1;
    if (pr >= (TX / 2) * (TY / 2)) return;
    const int I = T.i0 / 2 + pr % (TX / 2), J = T.j0 / 2 + pr / (TX / 2);
    if (I >= C.m1 || J >= C.m2) return;
    double rc = 0, rm = 0, rp = 0, rf = 0, sc = 0, smu = 0, sp = 0, sf = 0;
    const int fN = hlf ? T_V : T_U;
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
        for (int a = 0; a < 2; a++) {
            const int i = 2 * I + a, j = 2 * J + b;
            double xc, xm, xp, xf;
            resid_pair(P, Lf, T, F, i, j, hlf, xc, xm, xp, xf);
            rc += xc; rm += xm; rp += xp;
            // the lane's face of the coarse cell: west faces (a = 0) on the x
            // lane, south faces (b = 0) on the y lane
            if ((hlf ? b : a) == 0) { rf += xf; sf += T.q(fN, i, j); }
            sc += T.q(T_C, i, j); smu += T.q(T_MU, i, j); sp += T.q(T_P, i, j);
        }
    const size_t k = (size_t)J * C.pitch + I;
    if (hlf == 0) {
        C.c[k] = C.c0[k] = 0.25 * sc;
        C.mu[k] = C.mu0[k] = 0.25 * smu;
        C.p[k] = C.p0[k] = 0.25 * sp;
        C.fc[k] = 0.25 * rc;
        C.fmu[k] = 0.25 * rm;
        C.fp[k] = 0.25 * rp;
        C.u[k] = C.u0[k] = 0.5 * sf;
        C.fu[k] = 0.5 * rf;
    } else {
        C.v[k] = C.v0[k] = 0.5 * sf;
        C.fv[k] = 0.5 * rf;
    }
}

// the two cells of a tile handled by lane pair pr: (2k, lj) and (2k+1, lj)
__device__ __forceinline__ void pair_cells(const Tile &T, int &i, int &j)
{
    const int pr = threadIdx.x >> 1;
    const int lj = pr / (TX / 2), k = pr - lj * (TX / 2);
    i = T.i0 + 2 * k;
    j = T.j0 + lj;
}

// f_H = N_H(R w) + R r (FAS coarse right-hand side); walls carry no equation
__global__ __launch_bounds__(TBLK) void k_coarse_rhs(Phys P, View Lc, Coarse C)
{
    __shared__ double sm[TILE_DOUBLES];
    const Tile T = block_tile(sm);
    tile_load(P, Lc, T);
    __syncthreads();
    const int hlf = threadIdx.x & 1;
    int i, j;
    pair_cells(T, i, j);
    const Rhs Z = { nullptr, nullptr, nullptr, nullptr, nullptr };
    for (int a = 0; a < 2; a++, i++) {
        if (i >= C.m1 || j >= C.m2) continue;
        double rc, rm, rp, rf;
        resid_pair(P, Lc, T, Z, i, j, hlf, rc, rm, rp, rf); // r = -N_H(R w)
        const size_t k = (size_t)j * C.pitch + i;
        if (hlf == 0) {
            C.fc[k] -= rc;
            C.fmu[k] -= rm;
            C.fp[k] -= rp;
            C.fu[k] = u_unk(Lc, i) ? C.fu[k] - rf : 0.0;
        } else {
            C.fv[k] = v_unk(Lc, j) ? C.fv[k] - rf : 0.0;
        }
    }
}

// w_h += P(w_H - R w_h): cells piecewise constant; faces copy the coincident
// coarse face and average the two coarse faces across the coarse cell
__global__ __launch_bounds__(BLK) void k_prolong(View Lf, double *uf, double *vf, Coarse C, int bcx, int bcy)
{
    const int t = blockIdx.x * BLK + threadIdx.x;
    if (t >= Lf.m1 * Lf.m2) return;
    const int j = t / Lf.m1, i = t - j * Lf.m1;
    const int I = i >> 1, J = j >> 1;
    const size_t kc = (size_t)J * C.pitch + I, kf = (size_t)j * Lf.pitch + i;
    Lf.c[kf] += C.c[kc] - C.c0[kc];
    Lf.mu[kf] += C.mu[kc] - C.mu0[kc];
    Lf.p[kf] += C.p[kc] - C.p0[kc];
    if (u_unk(Lf, i)) {
        double d = C.u[kc] - C.u0[kc];
        if (i & 1) {
            double e = 0.0;
            if (I + 1 < C.m1) e = C.u[kc + 1] - C.u0[kc + 1];
            else if (bcx) e = C.u[(size_t)J * C.pitch] - C.u0[(size_t)J * C.pitch];
            d = 0.5 * (d + e);
        }
        uf[kf] += d;
    }
    if (v_unk(Lf, j)) {
        double d = C.v[kc] - C.v0[kc];
        if (j & 1) {
            double e = 0.0;
            if (J + 1 < C.m2) e = C.v[kc + C.pitch] - C.v0[kc + C.pitch];
            else if (bcy) e = C.v[I] - C.v0[I];
            d = 0.5 * (d + e);
        }
        vf[kf] += d;
    }
}

// wave64 + LDS block sum of NRED values (blocks of up to 16 waves); one
// partial row per block
__device__ __forceinline__ void block_sum_store(double (&v)[NRED], double *out, int block)
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
        for (int ww = 0; ww < (int)(blockDim.x >> 6); ww++) s += sh[ww][threadIdx.x];
        out[(size_t)block * NRED + threadIdx.x] = s;
    }
}

// residual norms of the finest level: per block sums of r^2 for the five
// equations, the sum of pbar, and the count of cells that are non-finite or
// past the density pole; optionally the residual fields themselves
__global__ __launch_bounds__(TBLK) void k_resid_norm(Phys P, View L, Rhs F, double *partials, double *rout)
{
    __shared__ double sm[TILE_DOUBLES];
    const Tile T = block_tile(sm);
    tile_load(P, L, T);
    __syncthreads();
    double v[NRED] = { 0, 0, 0, 0, 0, 0, 0, 0 };
    const size_t n = (size_t)L.m1 * L.m2;
    const int hlf = threadIdx.x & 1;
    int i, j;
    pair_cells(T, i, j);
    for (int a = 0; a < 2; a++, i++) {
        if (i >= L.m1 || j >= L.m2) continue;
        double rc, rm, rp, rf;
        resid_pair(P, L, T, F, i, j, hlf, rc, rm, rp, rf);
        const size_t q = (size_t)j * L.m1 + i;
        v[3 + hlf] += rf * rf;
        if (rout) rout[(3 + hlf) * n + q] = rf;
        if (hlf == 0) {
            v[0] += rc * rc; v[1] += rm * rm; v[2] += rp * rp;
            const double c = T.q(T_C, i, j), pp = T.q(T_P, i, j);
            v[5] += pp;
            const bool ok = isfinite(c) && isfinite(T.q(T_MU, i, j)) && isfinite(pp) && isfinite(T.q(T_U, i, j))
                          && isfinite(T.q(T_V, i, j)) && (P.drho * c + P.rho1 > 0.0);
            v[6] += ok ? 0.0 : 1.0;
            if (rout) { rout[q] = rc; rout[n + q] = rm; rout[2 * n + q] = rp; }
        }
    }
    block_sum_store(v, partials, tile_id());
}

// mass and energy partial sums of the current state
__global__ __launch_bounds__(BLK) void k_mass_energy(Phys P, View L, double h, double *partials)
{
    const int t = blockIdx.x * BLK + threadIdx.x;
    double v[NRED] = { 0, 0, 0, 0, 0, 0, 0, 0 };
    if (t < L.m1 * L.m2) {
        const int j = t / L.m1, i = t - j * L.m1;
        const size_t k = (size_t)j * L.pitch + i;
        const double c = L.c[k], r = rho_of(P, c);
        v[0] = r * c;
        v[1] = r * (1.0 - c);
        // kinetic energy on the west and south faces of the cell (App. A.7)
        const double cw = ldc(L.c, L.m1, L.m2, L.pitch, L.bcx, L.bcy, i - 1, j);
        const double cs = ldc(L.c, L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j - 1);
        const double rw = rho_of(P, cw), rs = rho_of(P, cs);
        if (u_unk(L, i)) { const double u = L.u[k]; v[2] += 0.25 * (r + rw) * u * u; }
        if (v_unk(L, j)) { const double w = L.v[k]; v[2] += 0.25 * (r + rs) * w * w; }
        // gradient energy [rho D c, D c] on the same faces (walls carry none)
        if (L.bcx || i > 0) { const double d = (c - cw) * L.inv_h; v[3] += 0.5 * (r + rw) * d * d; }
        if (L.bcy || j > 0) { const double d = (c - cs) * L.inv_h; v[3] += 0.5 * (r + rs) * d * d; }
        v[4] = r * dwell(c);
        v[5] = (r - P.rho_ref) * (j + 0.5) * h;
    }
    block_sum_store(v, partials, blockIdx.x);
}

// single-block fixed-order sum of the per-block partials
__global__ __launch_bounds__(BLK) void k_finalize(const double *partials, int nblk, double *out)
{
    __shared__ double sh[BLK][NRED];
    double s[NRED] = { 0, 0, 0, 0, 0, 0, 0, 0 };
    for (int b = threadIdx.x; b < nblk; b += BLK)
#pragma unroll
        for (int q = 0; q < NRED; q++) s[q] += partials[(size_t)b * NRED + q];
#pragma unroll
    for (int q = 0; q < NRED; q++) sh[threadIdx.x][q] = s[q];
    __syncthreads();
    for (int o = BLK / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o)
#pragma unroll
            for (int q = 0; q < NRED; q++) sh[threadIdx.x][q] += sh[threadIdx.x + o][q];
        __syncthreads();
    }
    if (threadIdx.x < NRED) out[threadIdx.x] = sh[0][threadIdx.x];
}

// pbar -= mean(pbar), the mean taken from the reduced sums
__global__ __launch_bounds__(BLK) void k_shift_p(double *p, int m1, int m2, int pitch, const double *red)
{
    const int t = blockIdx.x * BLK + threadIdx.x;
    if (t >= m1 * m2) return;
    const int j = t / m1, i = t - j * m1;
    p[(size_t)j * pitch + i] -= red[5] / (double)(m1 * m2);
}

// time-n data of the finest level = current iterate; keep mubar, pbar of time n
__global__ __launch_bounds__(BLK) void k_begin(View L, double *cn, double *un, double *vn, double *mus, double *ps)
{
    const int t = blockIdx.x * BLK + threadIdx.x;
    if (t >= L.m1 * L.m2) return;
    const int j = t / L.m1, i = t - j * L.m1;
    const size_t k = (size_t)j * L.pitch + i;
    cn[k] = L.c[k];
    un[k] = L.u[k];
    vn[k] = L.v[k];
    mus[k] = L.mu[k];
    ps[k] = L.p[k];
}

// time-n data of a coarse level from the next finer one
__global__ __launch_bounds__(BLK) void k_restrict_n(const double *fcn, const double *fun, const double *fvn, int fpitch,
                                                    double *ccn, double *cun, double *cvn, int m1, int m2, int pitch)
{
    const int t = blockIdx.x * BLK + threadIdx.x;
    if (t >= m1 * m2) return;
    const int J = t / m1, I = t - J * m1;
    const size_t f = (size_t)(2 * J) * fpitch + 2 * I, k = (size_t)J * pitch + I;
    ccn[k] = 0.25 * (fcn[f] + fcn[f + 1] + fcn[f + fpitch] + fcn[f + fpitch + 1]);
    cun[k] = 0.5 * (fun[f] + fun[f + fpitch]);
    cvn[k] = 0.5 * (fvn[f] + fvn[f + 1]);
}

// ===========================================================================
// host side

namespace {

struct DLev {
    int m1 = 0, m2 = 0, pitch = 0;
    double h = 0;
    double *c = nullptr, *mu = nullptr, *p = nullptr, *ub[2] = { nullptr, nullptr }, *vb[2] = { nullptr, nullptr };
    int cur = 0;
    double *cn = nullptr, *un = nullptr, *vn = nullptr;
    double *fc = nullptr, *fmu = nullptr, *fp = nullptr, *fu = nullptr, *fv = nullptr;
    double *c0 = nullptr, *mu0 = nullptr, *p0 = nullptr, *u0 = nullptr, *v0 = nullptr;
    size_t n() const { return (size_t)pitch * m2; }
};

} // namespace

struct qnsch_ctx {
    qnsch_grid g;
    qnsch_params prm;
    qnsch_opts opt;
    Phys P;
    int nlev = 0;
    DLev L[16];
    hipStream_t s = nullptr;
    std::vector<void *> allocs;
    double *mu_save = nullptr, *p_save = nullptr;
    double *partials = nullptr, *red = nullptr, *rout = nullptr;
    double *hred = nullptr; // pinned
    std::string err;
    // timing of the finest-level half-sweep launches (HIP events on the
    // context's stream), enabled by qnsch_profile
    int prof = 0, prof_used = 0;
    std::vector<hipEvent_t> ev;
    double prof_ms = 0.0;
    long prof_n = 0;
    int in_step = 0;
    double dt = 0;
    qnsch_step_stats st;
};

#define HIPCHK(ctx, x)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (x);                                                                  \
        if (e_ != hipSuccess) {                                                               \
            (ctx)->err = std::string(#x) + ": " + hipGetErrorString(e_);                      \
            return QNSCH_EDEVICE;                                                             \
        }                                                                                     \
    } while (0)

static int launch_check(qnsch_ctx *x, const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        x->err = std::string(what) + ": " + hipGetErrorString(e);
        return QNSCH_EDEVICE;
    }
    return QNSCH_OK;
}

static View view_of(qnsch_ctx *x, int l)
{
    DLev &D = x->L[l];
    View V;
    V.c = D.c; V.mu = D.mu; V.p = D.p;
    V.u = D.ub[D.cur]; V.v = D.vb[D.cur];
    V.cn = D.cn; V.un = D.un; V.vn = D.vn;
    V.m1 = D.m1; V.m2 = D.m2; V.pitch = D.pitch;
    V.bcx = x->g.bc_x; V.bcy = x->g.bc_y;
    V.inv_h = 1.0 / D.h;
    return V;
}
static Rhs rhs_of(qnsch_ctx *x, int l)
{
    DLev &D = x->L[l];
    Rhs F;
    F.fc = D.fc; F.fmu = D.fmu; F.fp = D.fp; F.fu = D.fu; F.fv = D.fv;
    return F;
}
static Coarse coarse_of(qnsch_ctx *x, int l)
{
    DLev &D = x->L[l];
    Coarse C;
    C.c = D.c; C.mu = D.mu; C.p = D.p; C.u = D.ub[D.cur]; C.v = D.vb[D.cur];
    C.c0 = D.c0; C.mu0 = D.mu0; C.p0 = D.p0; C.u0 = D.u0; C.v0 = D.v0;
    C.fc = D.fc; C.fmu = D.fmu; C.fp = D.fp; C.fu = D.fu; C.fv = D.fv;
    C.m1 = D.m1; C.m2 = D.m2; C.pitch = D.pitch;
    return C;
}
static unsigned nblocks(size_t n) { return (unsigned)((n + BLK - 1) / BLK); }
static dim3 tiles(int m1, int m2) { return dim3((unsigned)((m1 + TX - 1) / TX), (unsigned)((m2 + TY - 1) / TY)); }

static int prof_collect(qnsch_ctx *x)
{
    for (int q = 0; q < x->prof_used; q++) {
        float ms = 0.f;
        HIPCHK(x, hipEventElapsedTime(&ms, x->ev[2 * q], x->ev[2 * q + 1]));
        x->prof_ms += ms;
        x->prof_n++;
    }
    x->prof_used = 0;
    return QNSCH_OK;
}

static int halfsweep(qnsch_ctx *x, int l, int colour)
{
    DLev &D = x->L[l];
    View V = view_of(x, l);
    if (l == 0) {
        const bool tm = x->prof != 0;
        if (tm) {
            if ((size_t)(2 * x->prof_used + 2) > x->ev.size()) {
                for (int q = 0; q < 64; q++) {
                    hipEvent_t e;
                    HIPCHK(x, hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
                    x->ev.push_back(e);
                }
            }
            HIPCHK(x, hipEventRecord(x->ev[2 * x->prof_used], x->s));
        }
        hipLaunchKernelGGL(k_halfsweep_fine, tiles(D.m1, D.m2), dim3(TBLK), 0, x->s, x->P, V, D.ub[D.cur ^ 1],
                           D.vb[D.cur ^ 1], colour, x->opt.vanka_omega);
        if (tm) {
            HIPCHK(x, hipEventRecord(x->ev[2 * x->prof_used + 1], x->s));
            x->prof_used++;
        }
    } else {
        hipLaunchKernelGGL(k_halfsweep_coarse, tiles(D.m1, D.m2), dim3(TBLK), 0, x->s, x->P, V, rhs_of(x, l),
                           D.ub[D.cur ^ 1], D.vb[D.cur ^ 1], colour, x->opt.vanka_omega);
    }
    D.cur ^= 1;
    return launch_check(x, "k_halfsweep");
}

static int vcycle_rec(qnsch_ctx *x, int l)
{
    DLev &D = x->L[l];
    int rc;
    if (l == x->nlev - 1) {
        size_t n = (size_t)(D.m1 / 2) * D.m2;
        unsigned th = (unsigned)(2 * n < 512 ? ((2 * n + 63) / 64) * 64 : 512);
        size_t lds = coarse_lds_doubles(D.m1, D.m2) * sizeof(double);
        Rhs F = l > 0 ? rhs_of(x, l) : Rhs{ nullptr, nullptr, nullptr, nullptr, nullptr };
        hipLaunchKernelGGL(k_coarse_solve, dim3(1), dim3(th), lds, x->s, x->P, view_of(x, l), F, D.ub[D.cur],
                           D.vb[D.cur], x->opt.nu_coarse, x->opt.vanka_omega);
        return launch_check(x, "k_coarse_solve");
    }
    for (int s = 0; s < x->opt.nu1; s++) {
        if ((rc = halfsweep(x, l, 0))) return rc;
        if ((rc = halfsweep(x, l, 1))) return rc;
    }
    DLev &C = x->L[l + 1];
    size_t nc = (size_t)C.m1 * C.m2;
    hipLaunchKernelGGL(k_restrict, tiles(D.m1, D.m2), dim3(TBLK), 0, x->s, x->P, view_of(x, l), rhs_of(x, l),
                       coarse_of(x, l + 1));
    if ((rc = launch_check(x, "k_restrict"))) return rc;
    hipLaunchKernelGGL(k_coarse_rhs, tiles(C.m1, C.m2), dim3(TBLK), 0, x->s, x->P, view_of(x, l + 1),
                       coarse_of(x, l + 1));
    if ((rc = launch_check(x, "k_coarse_rhs"))) return rc;
    if ((rc = vcycle_rec(x, l + 1))) return rc;
    size_t nf = (size_t)D.m1 * D.m2;
    hipLaunchKernelGGL(k_prolong, dim3(nblocks(nf)), dim3(BLK), 0, x->s, view_of(x, l), D.ub[D.cur], D.vb[D.cur],
                       coarse_of(x, l + 1), x->g.bc_x, x->g.bc_y);
    if ((rc = launch_check(x, "k_prolong"))) return rc;
    for (int s = 0; s < x->opt.nu2; s++) {
        if ((rc = halfsweep(x, l, 0))) return rc;
        if ((rc = halfsweep(x, l, 1))) return rc;
    }
    return QNSCH_OK;
}

// residual norms of the finest level into hred[0..7]: 5 norms, sum p, bad count
static int norms(qnsch_ctx *x, double *rout, bool shift)
{
    DLev &D = x->L[0];
    size_t n = (size_t)D.m1 * D.m2;
    const dim3 tg = tiles(D.m1, D.m2);
    unsigned nbt = tg.x * tg.y, nb = nblocks(n);
    Rhs F = {};
    hipLaunchKernelGGL(k_resid_norm, tg, dim3(TBLK), 0, x->s, x->P, view_of(x, 0), F, x->partials, rout);
    int rc;
    if ((rc = launch_check(x, "k_resid_norm"))) return rc;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(BLK), 0, x->s, x->partials, (int)nbt, x->red);
    if ((rc = launch_check(x, "k_finalize"))) return rc;
    if (shift) {
        hipLaunchKernelGGL(k_shift_p, dim3(nb), dim3(BLK), 0, x->s, D.p, D.m1, D.m2, D.pitch, x->red);
        if ((rc = launch_check(x, "k_shift_p"))) return rc;
    }
    HIPCHK(x, hipMemcpyAsync(x->hred, x->red, NRED * sizeof(double), hipMemcpyDeviceToHost, x->s));
    HIPCHK(x, hipStreamSynchronize(x->s));
    for (int q = 0; q < 5; q++) x->hred[q] = sqrt(D.h * D.h * x->hred[q]);
    return prof_collect(x);
}

static int restore(qnsch_ctx *x)
{
    DLev &D = x->L[0];
    size_t bytes = D.n() * sizeof(double);
    HIPCHK(x, hipMemcpyAsync(D.c, D.cn, bytes, hipMemcpyDeviceToDevice, x->s));
    HIPCHK(x, hipMemcpyAsync(D.ub[D.cur], D.un, bytes, hipMemcpyDeviceToDevice, x->s));
    HIPCHK(x, hipMemcpyAsync(D.vb[D.cur], D.vn, bytes, hipMemcpyDeviceToDevice, x->s));
    HIPCHK(x, hipMemcpyAsync(D.mu, x->mu_save, bytes, hipMemcpyDeviceToDevice, x->s));
    HIPCHK(x, hipMemcpyAsync(D.p, x->p_save, bytes, hipMemcpyDeviceToDevice, x->s));
    HIPCHK(x, hipStreamSynchronize(x->s));
    x->in_step = 0;
    return QNSCH_OK;
}

static double *dalloc(qnsch_ctx *x, size_t n, int *rc)
{
    void *p = nullptr;
    if (hipMalloc(&p, n * sizeof(double)) != hipSuccess) {
        *rc = QNSCH_ENOMEM;
        return nullptr;
    }
    x->allocs.push_back(p);
    if (hipMemsetAsync(p, 0, n * sizeof(double), x->s) != hipSuccess) *rc = QNSCH_EDEVICE;
    return (double *)p;
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
    o->nu_coarse = 30;
    o->vanka_omega = 1.0;
}

const char *qnsch_last_error(const qnsch_ctx *x) { return x ? x->err.c_str() : "null context"; }
int qnsch_levels(const qnsch_ctx *x) { return x ? x->nlev : 0; }

void qnsch_destroy(qnsch_ctx *x)
{
    if (!x) return;
    if (x->s) (void)hipStreamSynchronize(x->s);
    for (void *p : x->allocs) (void)hipFree(p);
    for (hipEvent_t e : x->ev) (void)hipEventDestroy(e);
    if (x->hred) (void)hipHostFree(x->hred);
    delete x;
}

int qnsch_create(const qnsch_grid *g, const qnsch_params *p, const qnsch_opts *o, void *stream, qnsch_ctx **out)
{
    if (!g || !p || !out) return QNSCH_EINVAL;
    *out = nullptr;
    if (g->m1 < 4 || g->m2 < 4 || (g->m1 & 1) || (g->m2 & 1)) return QNSCH_EINVAL;
    if (!(g->Lx > 0) || !(g->Ly > 0)) return QNSCH_EINVAL;
    const double hx = g->Lx / g->m1, hy = g->Ly / g->m2;
    if (fabs(hx - hy) > 1e-12 * hx) return QNSCH_EINVAL;
    if ((g->bc_x != 0 && g->bc_x != 1) || (g->bc_y != 0 && g->bc_y != 1)) return QNSCH_EINVAL;
    if (!(p->rho1 > 0) || !(p->rho2 > 0) || !(p->visc1 > 0) || !(p->visc2 > 0) || !(p->Re > 0) || !(p->We > 0)
        || !(p->Pe > 0) || !(p->M > 0) || !(p->eps > 0) || !(p->eta > 0) || !(p->mob_reg >= 0))
        return QNSCH_EINVAL;
    qnsch_opts opt;
    qnsch_default_opts(&opt);
    if (o) opt = *o;
    if (opt.nu1 < 0 || opt.nu2 < 0 || opt.nu_coarse < 1 || opt.max_vcycles < 0 || opt.precision != QNSCH_FP64)
        return QNSCH_EINVAL;
    int nl = g->levels;
    if (nl <= 0) {
        nl = 1;
        while (nl < 16 && g->m1 % (1 << (nl + 1)) == 0 && g->m2 % (1 << (nl + 1)) == 0 && (g->m1 >> nl) >= 4
               && (g->m2 >> nl) >= 4)
            nl++;
    }
    if (nl > 16 || g->m1 % (1 << nl) != 0 || g->m2 % (1 << nl) != 0) return QNSCH_EINVAL;
    // the coarsest level is relaxed by one workgroup with the level in LDS
    if (coarse_lds_doubles(g->m1 >> (nl - 1), g->m2 >> (nl - 1)) * sizeof(double) > 65536) return QNSCH_EINVAL;

    qnsch_ctx *x = new qnsch_ctx();
    x->g = *g;
    x->g.levels = nl;
    x->prm = *p;
    x->opt = opt;
    x->nlev = nl;
    x->s = (hipStream_t)stream;
    Phys &P = x->P;
    P.rho1 = p->rho1; P.rho2 = p->rho2; P.rho12 = p->rho1 * p->rho2; P.drho = p->rho2 - p->rho1;
    P.visc1 = p->visc1; P.visc2 = p->visc2; P.visc12 = p->visc1 * p->visc2; P.dvisc = p->visc2 - p->visc1;
    P.alpha = (p->rho2 - p->rho1) / (p->rho1 * p->rho2);
    P.inv_Re = 1.0 / p->Re; P.inv_M = 1.0 / p->M; P.inv_Pe = 1.0 / p->Pe;
    P.K1 = p->M * p->eta / (p->eps * p->We);
    P.K2 = p->eps * p->eta * p->M / (2.0 * p->We);
    P.K3 = p->eps * p->eta * p->M / p->We;
    P.inv_Fr = p->inv_Fr; P.rho_ref = p->rho_ref; P.mob_reg = p->mob_reg;
    P.inv_dt = 0.0;
    int rc = QNSCH_OK;
    for (int l = 0; l < nl; l++) {
        DLev &D = x->L[l];
        D.m1 = g->m1 >> l;
        D.m2 = g->m2 >> l;
        D.pitch = D.m1;
        D.h = hx * (double)(1 << l);
        size_t n = D.n();
        D.c = dalloc(x, n, &rc); D.mu = dalloc(x, n, &rc); D.p = dalloc(x, n, &rc);
        D.ub[0] = dalloc(x, n, &rc); D.ub[1] = dalloc(x, n, &rc);
        D.vb[0] = dalloc(x, n, &rc); D.vb[1] = dalloc(x, n, &rc);
        D.cn = dalloc(x, n, &rc); D.un = dalloc(x, n, &rc); D.vn = dalloc(x, n, &rc);
        if (l > 0) {
            D.fc = dalloc(x, n, &rc); D.fmu = dalloc(x, n, &rc); D.fp = dalloc(x, n, &rc);
            D.fu = dalloc(x, n, &rc); D.fv = dalloc(x, n, &rc);
            D.c0 = dalloc(x, n, &rc); D.mu0 = dalloc(x, n, &rc); D.p0 = dalloc(x, n, &rc);
            D.u0 = dalloc(x, n, &rc); D.v0 = dalloc(x, n, &rc);
        }
        if (rc) break;
    }
    size_t n0 = x->L[0].n();
    if (!rc) {
        x->mu_save = dalloc(x, n0, &rc);
        x->p_save = dalloc(x, n0, &rc);
        const dim3 tg = tiles(g->m1, g->m2);
        const size_t nbmax = std::max((size_t)nblocks((size_t)g->m1 * g->m2), (size_t)tg.x * tg.y);
        x->partials = dalloc(x, nbmax * NRED, &rc);
        x->red = dalloc(x, NRED, &rc);
        x->rout = nullptr;
    }
    if (!rc && hipHostMalloc((void **)&x->hred, 16 * sizeof(double), hipHostMallocDefault) != hipSuccess)
        rc = QNSCH_ENOMEM;
    if (!rc && hipStreamSynchronize(x->s) != hipSuccess) rc = QNSCH_EDEVICE;
    if (rc) {
        qnsch_destroy(x);
        return rc;
    }
    memset(&x->st, 0, sizeof(x->st));
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
    const size_t n = (size_t)D.m1 * D.m2;
    std::vector<double> z(n, 0.0), uu(n), vv(n);
    if (u) memcpy(uu.data(), u, n * sizeof(double)); else std::fill(uu.begin(), uu.end(), 0.0);
    if (v) memcpy(vv.data(), v, n * sizeof(double)); else std::fill(vv.begin(), vv.end(), 0.0);
    if (x->g.bc_x == QNSCH_BC_WALL)
        for (int j = 0; j < D.m2; j++) uu[(size_t)j * D.m1] = 0.0;
    if (x->g.bc_y == QNSCH_BC_WALL)
        for (int i = 0; i < D.m1; i++) vv[i] = 0.0;
    int rc;
    if ((rc = put(x, D.c, c))) return rc;
    if ((rc = put(x, D.mu, mu ? mu : z.data()))) return rc;
    if ((rc = put(x, D.p, p ? p : z.data()))) return rc;
    if ((rc = put(x, D.ub[D.cur], uu.data()))) return rc;
    if ((rc = put(x, D.vb[D.cur], vv.data()))) return rc;
    HIPCHK(x, hipStreamSynchronize(x->s));
    return QNSCH_OK;
}

int qnsch_set_state(qnsch_ctx *x, const double *c, const double *mu, const double *p, const double *u, const double *v)
{
    if (!x || !c) return QNSCH_EINVAL;
    int rc = upload(x, c, mu, p, u, v);
    x->in_step = 0;
    return rc;
}

int qnsch_set_iterate(qnsch_ctx *x, const double *c, const double *mu, const double *p, const double *u,
                      const double *v)
{
    if (!x || !c) return QNSCH_EINVAL;
    if (!x->in_step) { x->err = "set_iterate outside a step"; return QNSCH_EBUSY; }
    return upload(x, c, mu, p, u, v);
}

int qnsch_get_state(qnsch_ctx *x, double *c, double *mu, double *p, double *u, double *v)
{
    if (!x) return QNSCH_EINVAL;
    DLev &D = x->L[0];
    int rc;
    if (c && (rc = get(x, c, D.c))) return rc;
    if (mu && (rc = get(x, mu, D.mu))) return rc;
    if (p && (rc = get(x, p, D.p))) return rc;
    if (u && (rc = get(x, u, D.ub[D.cur]))) return rc;
    if (v && (rc = get(x, v, D.vb[D.cur]))) return rc;
    HIPCHK(x, hipStreamSynchronize(x->s));
    return QNSCH_OK;
}

int qnsch_begin_step(qnsch_ctx *x, double dt)
{
    if (!x || !(dt > 0)) return QNSCH_EINVAL;
    x->dt = dt;
    x->P.inv_dt = 1.0 / dt;
    DLev &D = x->L[0];
    hipLaunchKernelGGL(k_begin, dim3(nblocks((size_t)D.m1 * D.m2)), dim3(BLK), 0, x->s, view_of(x, 0), D.cn, D.un,
                       D.vn, x->mu_save, x->p_save);
    int rc;
    if ((rc = launch_check(x, "k_begin"))) return rc;
    for (int l = 1; l < x->nlev; l++) {
        DLev &F = x->L[l - 1], &C = x->L[l];
        hipLaunchKernelGGL(k_restrict_n, dim3(nblocks((size_t)C.m1 * C.m2)), dim3(BLK), 0, x->s, F.cn, F.un, F.vn,
                           F.pitch, C.cn, C.un, C.vn, C.m1, C.m2, C.pitch);
        if ((rc = launch_check(x, "k_restrict_n"))) return rc;
    }
    x->in_step = 1;
    x->st.vcycles = 0;
    return QNSCH_OK;
}

int qnsch_vcycle(qnsch_ctx *x)
{
    if (!x) return QNSCH_EINVAL;
    if (!x->in_step) { x->err = "vcycle outside a step"; return QNSCH_EBUSY; }
    int rc;
    if ((rc = vcycle_rec(x, 0))) return rc;
    // pbar mean to zero (the reduction also gives the residual norms)
    return norms(x, nullptr, true);
}

int qnsch_residual(qnsch_ctx *x, double *r_out, double nrm[5])
{
    if (!x) return QNSCH_EINVAL;
    if (!x->in_step) { x->err = "residual outside a step"; return QNSCH_EBUSY; }
    DLev &D = x->L[0];
    const size_t n = (size_t)D.m1 * D.m2;
    int rc = QNSCH_OK;
    if (r_out && !x->rout) {
        x->rout = dalloc(x, 5 * n, &rc);
        if (rc) return rc;
    }
    if ((rc = norms(x, r_out ? x->rout : nullptr, false))) return rc;
    if (nrm) memcpy(nrm, x->hred, 5 * sizeof(double));
    if (r_out) {
        HIPCHK(x, hipMemcpy(r_out, x->rout, 5 * n * sizeof(double), hipMemcpyDeviceToHost));
    }
    return QNSCH_OK;
}

int qnsch_halfsweep(qnsch_ctx *x, int colour)
{
    if (!x) return QNSCH_EINVAL;
    if (!x->in_step) { x->err = "halfsweep outside a step"; return QNSCH_EBUSY; }
    int rc;
    if ((rc = halfsweep(x, 0, colour & 1))) return rc;
    HIPCHK(x, hipStreamSynchronize(x->s));
    return QNSCH_OK;
}

int qnsch_end_step(qnsch_ctx *x)
{
    if (!x) return QNSCH_EINVAL;
    x->in_step = 0;
    return QNSCH_OK;
}

int qnsch_step(qnsch_ctx *x, double dt)
{
    auto t0 = std::chrono::steady_clock::now();
    int rc;
    if ((rc = qnsch_begin_step(x, dt))) return rc;
    if ((rc = norms(x, nullptr, false))) return rc;
    memcpy(x->st.res0, x->hred, 5 * sizeof(double));
    int it = 0;
    for (;;) {
        double mx = 0.0;
        bool finite = true;
        for (int q = 0; q < 5; q++) {
            if (!std::isfinite(x->hred[q])) finite = false;
            mx = x->hred[q] > mx ? x->hred[q] : mx;
        }
        if (!finite || x->hred[6] != 0.0) {
            restore(x);
            x->err = "diverged: non-finite residual or c past the density pole";
            return QNSCH_EDIVERGED;
        }
        if (mx <= x->opt.tol) break;
        if (it >= x->opt.max_vcycles) {
            restore(x);
            x->err = "no convergence within max_vcycles";
            return QNSCH_ENOCONV;
        }
        if ((rc = vcycle_rec(x, 0))) return rc;
        if ((rc = norms(x, nullptr, true))) return rc;
        it++;
        x->st.vcycles = it;
    }
    memcpy(x->st.res, x->hred, 5 * sizeof(double));
    x->in_step = 0;
    x->st.step_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return QNSCH_OK;
}

static int reduce_me(qnsch_ctx *x)
{
    DLev &D = x->L[0];
    size_t n = (size_t)D.m1 * D.m2;
    unsigned nb = nblocks(n);
    hipLaunchKernelGGL(k_mass_energy, dim3(nb), dim3(BLK), 0, x->s, x->P, view_of(x, 0), D.h, x->partials);
    int rc;
    if ((rc = launch_check(x, "k_mass_energy"))) return rc;
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(BLK), 0, x->s, x->partials, (int)nb, x->red);
    if ((rc = launch_check(x, "k_finalize"))) return rc;
    HIPCHK(x, hipMemcpyAsync(x->hred, x->red, NRED * sizeof(double), hipMemcpyDeviceToHost, x->s));
    HIPCHK(x, hipStreamSynchronize(x->s));
    return QNSCH_OK;
}

int qnsch_mass(qnsch_ctx *x, double out[2])
{
    if (!x || !out) return QNSCH_EINVAL;
    int rc;
    if ((rc = reduce_me(x))) return rc;
    const double h2 = x->L[0].h * x->L[0].h;
    out[0] = h2 * x->hred[0];
    out[1] = h2 * x->hred[1];
    return QNSCH_OK;
}

int qnsch_energy(qnsch_ctx *x, double out[5])
{
    if (!x || !out) return QNSCH_EINVAL;
    int rc;
    if ((rc = reduce_me(x))) return rc;
    const double h2 = x->L[0].h * x->L[0].h;
    const qnsch_params &p = x->prm;
    out[1] = h2 * x->hred[2];
    out[2] = p.eps * p.eta / (2.0 * p.We) * h2 * x->hred[3];
    out[3] = p.eta / (p.eps * p.We) * h2 * x->hred[4];
    out[4] = p.inv_Fr * h2 * x->hred[5];
    out[0] = out[1] + out[2] + out[3] + out[4];
    return QNSCH_OK;
}

int qnsch_profile(qnsch_ctx *x, int enable)
{
    if (!x) return QNSCH_EINVAL;
    HIPCHK(x, hipStreamSynchronize(x->s));
    int rc;
    if ((rc = prof_collect(x))) return rc;
    x->prof = enable ? 1 : 0;
    x->prof_ms = 0.0;
    x->prof_n = 0;
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

int qnsch_synchronize(qnsch_ctx *x)
{
    if (!x) return QNSCH_EINVAL;
    HIPCHK(x, hipStreamSynchronize(x->s));
    return QNSCH_OK;
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

int qnsch_stats(const qnsch_ctx *x, qnsch_step_stats *out)
{
    if (!x || !out) return QNSCH_EINVAL;
    *out = x->st;
    return QNSCH_OK;
}

} // extern "C"
