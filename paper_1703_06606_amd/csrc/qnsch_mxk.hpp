// qnsch_mxk.hpp -- work-list kernels of the mixed-precision step: one FP32
// multigrid V-cycle on the correction equation J(w^) delta = r (see
// qnsch_lin.hpp), with the FP64 residual, update and reductions done by the
// kernels of qnsch_kern.hpp.
//
// Correction cycle on a hierarchy of levels (the coarse-grid correction
// scheme for a linear problem; sec. 7.1 gives the smoother and transfers):
//   smooth (nu1 red-black sweeps), restrict r - J delta and the linearisation
//   point to the next level with delta_H = 0, recurse, solve the coarsest
//   level in LDS, prolongate delta_H and add it, smooth (nu2 sweeps);
// then w += delta in FP64.  The coarse operators are the rediscretised
// Jacobians J_H(R w^).
#pragma once
#include "qnsch_kern.hpp"

namespace qn {

#define LTILE_FLOATS (L_NF * (TX + 3) * (TY + 3))
static_assert(LTILE_FLOATS * 4 <= 65536, "FP32 tile exceeds 64 KiB of LDS");

__device__ __forceinline__ LView lview_of(const Desc &d, int par)
{
    LView V;
    V.c = d.xc; V.mu = d.xmu; V.u = d.xu; V.v = d.xv;
    V.dc = d.dc; V.dmu = d.dmu; V.dp = d.dp;
    V.du = d.dub[par]; V.dv = d.dvb[par];
    V.cn = d.cnf; V.un = d.unf; V.vn = d.vnf;
    V.rc = d.rc; V.rmu = d.rmu; V.rp = d.rp; V.ru = d.ru; V.rv = d.rv;
    V.m1 = d.m1; V.m2 = d.m2; V.pitch = d.pitch;
    V.bcx = d.bcx; V.bcy = d.bcy;
    V.inv_h = d.finv_h;
    return V;
}

// one colour half-sweep of the correction smoother; the correction faces are
// read from buffer par and written to par^1
template <typename IT> __device__ __forceinline__ void mx_halfsweep_body(const IT &it, int colour, float omega)
{
    __shared__ float sm[LTILE_FLOATS];
    const int k = find_item(it);
    const Desc &d = *it.d[k];
    if (!tile_valid(it, k, d)) return;
    const int par = it.par[k];
    const LView L = lview_of(d, par);
    const TileF T = item_tile(sm, it, k, d);
    ltile_load(d.Pf, L, T);
    __syncthreads();
    const int pr = threadIdx.x >> 1, hlf = threadIdx.x & 1;
    const int lj = pr / (TX / 2), kk = pr - lj * (TX / 2);
    const int j = T.j0 + lj;
    const int i = T.i0 + 2 * kk + ((j + colour) & 1);
    if (i < L.m1 && j < L.m2) lrelax_pair<1>(d.Pf, L, T, d.dub[par ^ 1], d.dvb[par ^ 1], i, j, hlf, omega);
}
template <typename IT> __global__ HS_ATTR void k_mx_halfsweep(IT it, int colour, float omega)
{
    mx_halfsweep_body(it, colour, omega);
}
// finest-level launches under their own name (profiles)
template <typename IT> __global__ HS_ATTR void k_mx_halfsweep_fine(IT it, int colour, float omega)
{
    mx_halfsweep_body(it, colour, omega);
}

// temporal blocking of the correction smoother: one red + black sweep per
// launch, as k_hs_fused (the widened tile in LDS, the cell corrections from
// one set to the other, the face corrections from buffer par to par ^ 1)
#define MX_FUSED_FLOATS ((L_NF + 2) * FUSED_W * FUSED_H)
static_assert(MX_FUSED_FLOATS * 4 <= 65536, "fused FP32 tile exceeds 64 KiB of LDS");

__device__ __forceinline__ void mx_fused_load(const PhysF &P, const LView &L, const TileF &T)
{
    const int n = T.W * T.H;
    for (int e = threadIdx.x; e < n; e += block_threads()) {
        const int b = e / T.W, a = e - b * T.W;
        int i = T.i0 - 1 + a, j = T.j0 - 1 + b;
        if (L.bcx) i = wrapi(i, L.m1);
        if (L.bcy) j = wrapi(j, L.m2);
        const TileSrc q = tile_src(L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j);
        float *s = T.s + e;
        if (q.sc == 0) {
            for (int f = 0; f < L_NF + 2; f++) s[f * n] = 0.0f;
            continue;
        }
        // the level is in global memory; every load before any use
        const float v[9] = { lda<1>(L.c, q.c), lda<1>(L.dc, q.c), lda<1>(L.dmu, q.c), lda<1>(L.dp, q.c),
                             lda<1>(L.du, q.u), lda<1>(L.dv, q.v), lda<1>(L.cn, q.c), lda<1>(L.un, q.u),
                             lda<1>(L.vn, q.v) };
        __builtin_amdgcn_sched_barrier(0);
        s[L_C * n] = v[0];
        s[L_DC * n] = v[1];
        s[L_MU * n] = v[2];
        s[L_P * n] = v[3];
        s[L_U * n] = s[L_NF * n] = signed_val(q.su, v[4]);
        s[L_V * n] = s[(L_NF + 1) * n] = signed_val(q.sv, v[5]);
        s[L_CN * n] = v[6];
        s[L_UN * n] = signed_val(q.su, v[7]);
        s[L_VN * n] = signed_val(q.sv, v[8]);
        s[L_RN * n] = rhof(P, v[6]);
        s[L_MV * n] = viscf(P, v[6]);
        s[L_MOB * n] = mobf(P, v[6]);
        const float rs = rhof(P, v[0]);
        s[L_RS * n] = rs;
        s[L_DRS * n] = -P.alpha * rs * rs * v[1];
    }
}
// after the red pass (as fused_refresh): the new face corrections become the
// black pass's snapshot, and the wall images follow their sources
__device__ __forceinline__ void mx_fused_refresh(const LView &L, const TileF &T)
{
    const int n = T.W * T.H;
    const float *un = T.s + L_NF * n, *vn = T.s + (L_NF + 1) * n;
    for (int e = threadIdx.x; e < n; e += block_threads()) {
        const int b = e / T.W, a = e - b * T.W;
        const int i = T.i0 - 1 + a, j = T.j0 - 1 + b;
        const bool gx = !L.bcx && (i < 0 || i >= L.m1), gy = !L.bcy && (j < 0 || j >= L.m2);
        const int si = gx ? (i < 0 ? 0 : L.m1 - 1) : i, sj = gy ? (j < 0 ? 0 : L.m2 - 1) : j;
        const int su = (!L.bcx && (i <= 0 || i >= L.m1)) ? 0 : (gy ? -1 : 1);
        const int sv = (!L.bcy && (j <= 0 || j >= L.m2)) ? 0 : (gx ? -1 : 1);
        // every value the element may take, before any store (as
        // fused_refresh)
        const int q = T.idx(si, sj);
        const float u = un[T.idx(i, sj)], v = vn[T.idx(si, j)], dc = T.s[L_DC * n + q], mu = T.s[L_MU * n + q],
                    p = T.s[L_P * n + q], drs = T.s[L_DRS * n + q];
        __builtin_amdgcn_sched_barrier(0);
        T.s[L_U * n + e] = signed_val(su, u);
        T.s[L_V * n + e] = signed_val(sv, v);
        if (gx || gy) {
            T.s[L_DC * n + e] = dc;
            T.s[L_MU * n + e] = mu;
            T.s[L_P * n + e] = p;
            T.s[L_DRS * n + e] = drs;
        }
    }
}
template <typename IT> __global__ __launch_bounds__(FBLK) void k_mx_fused(IT it, int dir, float omega)
{
    __shared__ float sm[MX_FUSED_FLOATS];
    const int k = find_item(it);
    const Desc &d = *it.d[k];
    if (!tile_valid(it, k, d)) return;
    const int par = it.par[k];
    LView L = lview_of(d, par);
    LView O = L;
    if (dir) {
        L.dc = d.dc2; L.dmu = d.dmu2; L.dp = d.dp2;
    } else {
        O.dc = d.dc2; O.dmu = d.dmu2; O.dp = d.dp2;
    }
    const TileF T0 = item_tile(sm, it, k, d);
    TileF T;
    T.s = sm; T.i0 = T0.i0 - 2; T.j0 = T0.j0 - 2; T.W = FUSED_W; T.H = FUSED_H;
    mx_fused_load(d.Pf, L, T);
    __syncthreads();
    const int pr = threadIdx.x >> 1, hlf = threadIdx.x & 1;
    {
        const int lj = pr / ((TX + 4) / 2), kk = pr - lj * ((TX + 4) / 2);
        const int tj = T0.j0 - 2 + lj;
        const int ti = T0.i0 - 2 + 2 * kk + (tj & 1);
        const bool in = lj < TY + 4 && (L.bcx || (ti >= 0 && ti < L.m1)) && (L.bcy || (tj >= 0 && tj < L.m2));
        if (in) {
            const int i = L.bcx ? wrapi(ti, L.m1) : ti, j = L.bcy ? wrapi(tj, L.m2) : tj;
            lrelax_cell<true, 1>(d.Pf, L, T, nullptr, nullptr, i, j, ti, tj, hlf, omega);
        }
    }
    __syncthreads();
    mx_fused_refresh(L, T);
    __syncthreads();
    if (threadIdx.x < TBLK) {
        const int lj = pr / (TX / 2), kk = pr - lj * (TX / 2);
        const int j = T0.j0 + lj;
        const int i = T0.i0 + 2 * kk + ((j + 1) & 1);
        if (i < L.m1 && j < L.m2) lrelax_cell<false, 1>(d.Pf, O, T, d.dub[par ^ 1], d.dvb[par ^ 1], i, j, i, j, hlf, omega);
    } else {
        const int q = pr - TBLK / 2;
        const int lj = q / (TX / 2), kk = q - lj * (TX / 2);
        const int j = T0.j0 + lj;
        const int i = T0.i0 + 2 * kk + (j & 1);
        if (i < L.m1 && j < L.m2) {
            const int e = T.idx(i, j), n = T.W * T.H;
            const size_t g = (size_t)j * L.pitch + i;
            if (hlf == 0) { O.dc[g] = T.s[L_DC * n + e]; O.dmu[g] = T.s[L_MU * n + e]; }
            else O.dp[g] = T.s[L_P * n + e];
        }
    }
}

// r - J delta on the item's level, restricted to the next coarser level
// (cells: mean of four; faces: mean of the two coincident fine faces),
// together with the linearisation point; the coarse correction starts at 0
template <typename IT> __global__ __launch_bounds__(TBLK) void k_mx_restrict(IT it)
{
    __shared__ float sm[LTILE_FLOATS];
    const int k = find_item(it);
    const Desc &d = *it.d[k];
    if (!tile_valid(it, k, d)) return;
    const Desc &C = *d.coarse;
    const LView Lf = lview_of(d, it.par[k]);
    const TileF T = item_tile(sm, it, k, d);
    ltile_load(d.Pf, Lf, T);
    __syncthreads();
    const int pr = threadIdx.x >> 1, hlf = threadIdx.x & 1;
    if (pr >= (TX / 2) * (TY / 2)) return;
    const int I = T.i0 / 2 + pr % (TX / 2), J = T.j0 / 2 + pr / (TX / 2);
    if (I >= C.m1 || J >= C.m2) return;
    float rc = 0, rm = 0, rp = 0, rf = 0, sc = 0, smu = 0, sf = 0;
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
        for (int a = 0; a < 2; a++) {
            const int i = 2 * I + a, j = 2 * J + b;
            const size_t q = (size_t)j * Lf.pitch + i;
            float xc, xm, xp, xf;
            lresid_pair(d.Pf, Lf, T, i, j, hlf, xc, xm, xp, xf);
            rc += xc; rm += xm; rp += xp;
            if ((hlf ? b : a) == 0) { rf += xf; sf += lda<1>(hlf ? Lf.v : Lf.u, q); }
            sc += T.q(L_C, i, j); smu += lda<1>(Lf.mu, q);
        }
    const size_t q = (size_t)J * C.pitch + I;
    const int cp = it.cpar[k];
    if (hlf == 0) {
        C.xc[q] = 0.25f * sc;
        C.xmu[q] = 0.25f * smu;
        C.xu[q] = 0.5f * sf;
        C.rc[q] = 0.25f * rc;
        C.rmu[q] = 0.25f * rm;
        C.rp[q] = 0.25f * rp;
        C.ru[q] = 0.5f * rf;
        C.dc[q] = 0.0f; C.dmu[q] = 0.0f; C.dp[q] = 0.0f;
        C.dub[cp][q] = 0.0f;
    } else {
        C.xv[q] = 0.5f * sf;
        C.rv[q] = 0.5f * rf;
        C.dvb[cp][q] = 0.0f;
    }
}

// P delta_H of the FP32 correction at fine cell (i, j): cells piecewise
// constant, faces as in prolong_load / prolong_apply (a face on a wall is no
// unknown), in two parts so that every load is in flight before any value is
// used.  The coarse arrays are read from the descriptor once per workgroup,
// through a global pointer (scalar loads).
struct PSrcF {
    const float *dc, *dmu, *dp, *du, *dv;
    int pitch, m1, m2, bcx, bcy;
};
__device__ __forceinline__ PSrcF psrcf_of(const Desc &d, const Desc *cp, int cpar)
{
    const __attribute__((address_space(1))) Desc &C = *(const __attribute__((address_space(1))) Desc *)cp;
    PSrcF s;
    s.dc = C.dc; s.dmu = C.dmu; s.dp = C.dp; s.du = C.dub[cpar]; s.dv = C.dvb[cpar];
    s.pitch = C.pitch; s.m1 = C.m1; s.m2 = C.m2; s.bcx = d.bcx; s.bcy = d.bcy;
    return s;
}
// the coarse cell of fine cell (i, j), and for its west (south) face the
// coarse face it lies on and the next one east (north): the periodic image,
// or, where there is none, the same face again (loaded, not used)
struct PRawF {
    float c, mu, p, u[2], v[2];
};
__device__ __forceinline__ PRawF mx_prolong_load(const PSrcF &C, int i, int j)
{
    PRawF r;
    const int I = i >> 1, J = j >> 1;
    const size_t kc = (size_t)J * C.pitch + I;
    r.c = lda<1>(C.dc, kc); r.mu = lda<1>(C.dmu, kc); r.p = lda<1>(C.dp, kc);
    const size_t ke = I + 1 < C.m1 ? kc + 1 : (C.bcx ? (size_t)J * C.pitch : kc);
    const size_t kn = J + 1 < C.m2 ? kc + C.pitch : (C.bcy ? (size_t)I : kc);
    r.u[0] = lda<1>(C.du, kc); r.u[1] = lda<1>(C.du, ke);
    r.v[0] = lda<1>(C.dv, kc); r.v[1] = lda<1>(C.dv, kn);
    return r;
}
// ... the corrections; hu / hv: the face is an unknown
__device__ __forceinline__ void mx_prolong_apply(const PSrcF &C, const PRawF &r, int i, int j, float &c, float &mu,
                                                 float &p, float &du, float &dv, bool &hu, bool &hv)
{
    c = r.c; mu = r.mu; p = r.p;
    hu = C.bcx || i >= 1;
    hv = C.bcy || j >= 1;
    du = r.u[0];
    if (i & 1) {
        const float e = ((i >> 1) + 1 < C.m1 || C.bcx) ? r.u[1] : 0.0f;
        du = 0.5f * (du + e);
    }
    dv = r.v[0];
    if (j & 1) {
        const float e = ((j >> 1) + 1 < C.m2 || C.bcy) ? r.v[1] : 0.0f;
        dv = 0.5f * (dv + e);
    }
}

// delta_h += P delta_H, one thread per fine cell
template <typename IT> __global__ __launch_bounds__(BLK) void k_mx_prolong(IT it)
{
    const int k = find_item(it);
    const Desc &d = *it.d[k];
    const int t = ((int)blockIdx.x - it.start[k]) * BLK + threadIdx.x;
    if (t >= d.m1 * d.m2) return;
    const int j = t / d.m1, i = t - j * d.m1;
    const size_t kf = (size_t)j * d.pitch + i;
    const PSrcF ps = psrcf_of(d, d.coarse, it.cpar[k]);
    float *ub = d.dub[it.par[k]], *vb = d.dvb[it.par[k]];
    const PRawF raw = mx_prolong_load(ps, i, j);
    const float c0 = lda<1>(d.dc, kf), m0 = lda<1>(d.dmu, kf), p0 = lda<1>(d.dp, kf), u0 = lda<1>(ub, kf),
                v0 = lda<1>(vb, kf);
    __builtin_amdgcn_sched_barrier(0);
    float c, mu, p, du, dv;
    bool hu, hv;
    mx_prolong_apply(ps, raw, i, j, c, mu, p, du, dv, hu, hv);
    sta<1>(d.dc, kf, c0 + c);
    sta<1>(d.dmu, kf, m0 + mu);
    sta<1>(d.dp, kf, p0 + p);
    if (hu) sta<1>(ub, kf, u0 + du);
    if (hv) sta<1>(vb, kf, v0 + dv);
}

// LDS floats of the coarsest-level correction solve: 19 level arrays + a tile
// + the tile's source map (4 ints per element)
__host__ __device__ inline size_t mx_coarse_lds_floats(int m1, int m2)
{
    return (size_t)19 * m1 * m2 + (size_t)(L_NF + 4) * (m1 + 3) * (m2 + 3);
}

// all correction sweeps of a level in one workgroup per item, the level
// resident in LDS (the coarsest level, and the smoothing of small coarse
// levels); an even number of half-sweeps keeps the result in buffer par
template <typename IT>
__global__ __launch_bounds__(512) void k_mx_coarse_solve(IT it, int sweeps, float omega, int prolong)
{
    extern __shared__ float smf[];
    const int k = find_item(it);
    const Desc &d = *it.d[k];
    const int par = it.par[k];
    const LView L = lview_of(d, par);
    float *ua = d.dub[par], *va = d.dvb[par];
    const int m1 = L.m1, m2 = L.m2, n = m1 * m2;
    float *hxc = smf, *hxmu = smf + n, *hxu = smf + 2 * n, *hxv = smf + 3 * n, *hdc = smf + 4 * n,
          *hdmu = smf + 5 * n, *hdp = smf + 6 * n, *uA = smf + 7 * n, *vA = smf + 8 * n, *uB = smf + 9 * n,
          *vB = smf + 10 * n, *hcn = smf + 11 * n, *hun = smf + 12 * n, *hvn = smf + 13 * n, *hr = smf + 14 * n;
    PSrcF ps = {};
    if (prolong) ps = psrcf_of(d, d.coarse, it.cpar[k]);
    for (int e = threadIdx.x; e < n; e += block_threads()) {
        const int j = e / m1, i = e - j * m1;
        const size_t q = (size_t)j * L.pitch + i;
        // every load of the element before any use
        const float xc = lda<1>(L.c, q), xmu = lda<1>(L.mu, q), xu = lda<1>(L.u, q), xv = lda<1>(L.v, q);
        float dc = lda<1>(L.dc, q), dmu = lda<1>(L.dmu, q), dp = lda<1>(L.dp, q), du = lda<1>(ua, q),
              dv = lda<1>(va, q);
        const float cn = lda<1>(L.cn, q), un = lda<1>(L.un, q), vn = lda<1>(L.vn, q);
        const float r0 = lda<1>(L.rc, q), r1 = lda<1>(L.rmu, q), r2 = lda<1>(L.rp, q), r3 = lda<1>(L.ru, q),
                    r4 = lda<1>(L.rv, q);
        PRawF raw = {};
        if (prolong) raw = mx_prolong_load(ps, i, j);
        __builtin_amdgcn_sched_barrier(0);
        if (prolong) {
            float c, mu, p, pu, pv;
            bool hu, hv;
            mx_prolong_apply(ps, raw, i, j, c, mu, p, pu, pv, hu, hv);
            dc += c; dmu += mu; dp += p;
            if (hu) du += pu;
            if (hv) dv += pv;
        }
        hxc[e] = xc; hxmu[e] = xmu; hxu[e] = xu; hxv[e] = xv;
        hdc[e] = dc; hdmu[e] = dmu; hdp[e] = dp; uA[e] = du; vA[e] = dv;
        hcn[e] = cn; hun[e] = un; hvn[e] = vn;
        hr[e] = r0; hr[n + e] = r1; hr[2 * n + e] = r2; hr[3 * n + e] = r3;
        hr[4 * n + e] = r4;
    }
    __syncthreads();
    LView H = L;
    H.c = hxc; H.mu = hxmu; H.u = hxu; H.v = hxv; H.dc = hdc; H.dmu = hdmu; H.dp = hdp;
    H.cn = hcn; H.un = hun; H.vn = hvn;
    H.rc = hr; H.rmu = hr + n; H.rp = hr + 2 * n; H.ru = hr + 3 * n; H.rv = hr + 4 * n;
    H.pitch = m1;
    TileF T;
    T.s = smf + 19 * n; T.i0 = 0; T.j0 = 0; T.W = m1 + 3; T.H = m2 + 3;
    int *map = (int *)(T.s + (size_t)L_NF * T.W * T.H);
    tile_map_build(H, T, map);
    const int half = m1 >> 1;
    for (int s = 0; s < 2 * sweeps; s++) {
        const int colour = s & 1;
        float *uw, *vw;
        if (s & 1) { H.du = uB; H.dv = vB; uw = uA; vw = vA; }
        else { H.du = uA; H.dv = vA; uw = uB; vw = vB; }
        if (s == 0) ltile_load(d.Pf, H, T);
        else ltile_refresh_map(d.Pf, H, T, map, colour ^ 1);
        __syncthreads();
        for (int t = threadIdx.x; t < 2 * half * m2; t += block_threads()) {
            const int pr = t >> 1;
            const int j = pr / half;
            const int i = 2 * (pr - j * half) + ((j + colour) & 1);
            lrelax_pair<3>(d.Pf, H, T, uw, vw, i, j, t & 1, omega);
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < n; e += block_threads()) {
        const int j = e / m1, i = e - j * m1;
        const size_t q = (size_t)j * L.pitch + i;
        L.dc[q] = hdc[e]; L.dmu[q] = hdmu[e]; L.dp[q] = hdp[e]; ua[q] = uA[e]; va[q] = vA[e];
    }
}

// w += delta on the finest level (FP64 state, single u/v buffer in mixed
// mode); faces on walls are not unknowns
template <typename IT> __global__ __launch_bounds__(BLK) void k_mx_update(IT it)
{
    const int k = find_item(it);
    const Desc &d = *it.d[k];
    const int t = ((int)blockIdx.x - it.start[k]) * BLK + threadIdx.x;
    if (t >= d.m1 * d.m2) return;
    const int j = t / d.m1, i = t - j * d.m1;
    const size_t q = (size_t)j * d.pitch + i;
    const int par = it.par[k];
    d.c[q] += (double)d.dc[q];
    d.mu[q] += (double)d.dmu[q];
    d.p[q] += (double)d.dp[q];
    if (d.bcx || i >= 1) d.ub[0][q] += (double)d.dub[par][q];
    if (d.bcy || j >= 1) d.vb[0][q] += (double)d.dvb[par][q];
}

// FP32 time-n data of the next coarser level
template <typename IT> __global__ __launch_bounds__(BLK) void k_mx_restrict_n(IT it)
{
    const int k = find_item(it);
    const Desc &F = *it.d[k];
    const Desc &C = *F.coarse;
    const int t = ((int)blockIdx.x - it.start[k]) * BLK + threadIdx.x;
    if (t >= C.m1 * C.m2) return;
    const int J = t / C.m1, I = t - J * C.m1;
    const size_t f = (size_t)(2 * J) * F.pitch + 2 * I, q = (size_t)J * C.pitch + I;
    C.cnf[q] = 0.25f * (F.cnf[f] + F.cnf[f + 1] + F.cnf[f + F.pitch] + F.cnf[f + F.pitch + 1]);
    C.unf[q] = 0.5f * (F.unf[f] + F.unf[f + F.pitch]);
    C.vnf[q] = 0.5f * (F.vnf[f] + F.vnf[f + 1]);
}

// r - J delta on a level into the FP64 residual-field buffer (m1 x m2 per
// field, packed), for checking the linearisation
template <typename IT> __global__ __launch_bounds__(TBLK) void k_mx_linresid(IT it)
{
    __shared__ float sm[LTILE_FLOATS];
    const int k = find_item(it);
    const Desc &d = *it.d[k];
    if (!tile_valid(it, k, d)) return;
    const LView L = lview_of(d, it.par[k]);
    const TileF T = item_tile(sm, it, k, d);
    ltile_load(d.Pf, L, T);
    __syncthreads();
    const size_t n = (size_t)L.m1 * L.m2;
    const int hlf = threadIdx.x & 1;
    int i, j;
    pair_cells(T, i, j);
    for (int a = 0; a < 2; a++, i++) {
        if (i >= L.m1 || j >= L.m2) continue;
        float rc, rm, rp, rf;
        lresid_pair(d.Pf, L, T, i, j, hlf, rc, rm, rp, rf);
        const size_t q = (size_t)j * L.m1 + i;
        d.rout[(3 + hlf) * n + q] = rf;
        if (hlf == 0) { d.rout[q] = rc; d.rout[n + q] = rm; d.rout[2 * n + q] = rp; }
    }
}

} // namespace qn
