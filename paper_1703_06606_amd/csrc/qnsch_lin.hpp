// qnsch_lin.hpp -- FP32 linearised smoother of the mixed-precision step.
//
// Mixed precision solves the nonlinear system N(w) = 0 of sec. 6.1 by defect
// correction: the residual r = -N(w) and the update w += delta are FP64, and
// delta comes from one multigrid V-cycle on the linearisation
//     J(w^) delta = r,   w^ = w rounded to FP32,
// run entirely in FP32.  J is the exact Jacobian of the discrete equations
// (the same equations as the FP64 smoother, differentiated by hand), so the
// outer iteration is an inexact Newton method whose inner solve has the
// colour ordering, box smoother and transfers of the FP64 V-cycle (sec. 7.1).
//
// Nonlinear terms of N and their linearisations (rho* = rho(c), rho' =
// -alpha rho^2; every other coefficient is time-n data and constant):
//   phase    rho*(c)(c - c^n)/dt                     -> Jcc dc (pointwise)
//   chem.    rho* mubar, the bulk terms in c          -> pointwise in dc, dmu
//            |grad c|^2 r(c)                          -> 5-point in dc
//            div(A rho* grad c) (App. A.6)            -> 5-point in dc
//   momentum (A rho* - A rho^n) u/(2 dt)              -> faces: du, and dc of
//                                                        the two adjacent cells
// The rest (advection with time-n velocity, viscous, pressure, surface-tension
// and mass-equation terms) is linear in the unknowns and is applied to delta
// with the FP64 formulas; gravity and time-n sources drop out.
//
// Tile layout: the field indices of the FP64 tile are kept for the fields that
// play the same role (so the axis descriptor Ax is shared), with the
// unknowns replaced by their corrections.
#pragma once
#include "qnsch_dev.hpp"

namespace qn {

struct PhysF {
    float rho1, rho12, drho, visc1, visc12, dvisc;
    float alpha, inv_Re, inv_M, inv_Pe, K1, K2, K3, mob_reg, inv_dt;
    int coupled; // smoother as in Phys
};

// one level of the correction problem
struct LView {
    const float *c, *mu, *u, *v;          // linearisation point (cells; faces)
    float *dc, *dmu, *dp;                 // correction of the cell unknowns
    const float *du, *dv;                 // correction of the faces (buffer being read)
    const float *cn, *un, *vn;            // time-n data
    const float *rc, *rmu, *rp, *ru, *rv; // right-hand side
    int m1, m2, pitch, bcx, bcy;
    float inv_h;
};

// tile fields: L_C holds c^ (the linearisation point), L_MU, L_P, L_U, L_V
// the corrections dmu, dp, du, dv; L_DC the correction dc and L_DRS the
// induced change of density rho'(c^) dc
enum { L_C = T_C, L_MU = T_MU, L_P = T_P, L_U = T_U, L_V = T_V, L_CN = T_CN, L_UN = T_UN, L_VN = T_VN, L_RN = T_RN,
       L_MV = T_MV, L_MOB = T_MOB, L_RS = T_RS, L_DC = T_NF, L_DRS, L_NF };
typedef TileT<float> TileF;

__device__ __forceinline__ float frcpf(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rhof(const PhysF &P, float c) { return P.rho12 * frcpf(P.drho * c + P.rho1); }
__device__ __forceinline__ float viscf(const PhysF &P, float c) { return P.visc12 * frcpf(P.dvisc * c + P.visc1); }
__device__ __forceinline__ float mobf(const PhysF &P, float c)
{
    const float q = c * (1.0f - c);
    return __builtin_sqrtf(q * q + P.mob_reg);
}

__device__ __forceinline__ void ltile_load(const PhysF &P, const LView &L, const TileF &T)
{
    const int n = T.W * T.H;
    if (tile_inner(L.m1, L.m2, T.i0, T.j0, T.W, T.H) && n <= 2 * (int)block_threads()) {
        // no boundary images: plain strided loads, a thread's two elements
        // loaded together (see tile_load)
        const int e0 = threadIdx.x, e1r = threadIdx.x + block_threads(), e1 = e1r < n ? e1r : n - 1;
        auto at = [&](int e) {
            const int b = e / T.W, a = e - b * T.W;
            return (size_t)(T.j0 - 1 + b) * L.pitch + (T.i0 - 1 + a);
        };
        const size_t q0 = at(e0 < n ? e0 : n - 1), q1 = at(e1);
        float v0[9], v1[9];
        const float *src[9] = { L.c, L.dc, L.dmu, L.dp, L.du, L.dv, L.cn, L.un, L.vn };
#pragma unroll
        for (int f = 0; f < 9; f++) {
            v0[f] = src[f][q0];
            v1[f] = src[f][q1];
        }
        auto put = [&](int e, const float *v) {
            float *s = T.s + e;
            s[L_C * n] = v[0];
            s[L_DC * n] = v[1];
            s[L_MU * n] = v[2];
            s[L_P * n] = v[3];
            s[L_U * n] = v[4];
            s[L_V * n] = v[5];
            s[L_CN * n] = v[6];
            s[L_UN * n] = v[7];
            s[L_VN * n] = v[8];
            s[L_RN * n] = rhof(P, v[6]);
            s[L_MV * n] = viscf(P, v[6]);
            s[L_MOB * n] = mobf(P, v[6]);
            const float rs = rhof(P, v[0]);
            s[L_RS * n] = rs;
            s[L_DRS * n] = -P.alpha * rs * rs * v[1];
        };
        if (e0 < n) put(e0, v0);
        if (e1r < n) put(e1r, v1);
        return;
    }
    if (n <= 2 * (int)block_threads()) {
        // boundary images: sources first, then all loads together (see tile_load)
        const int e0 = threadIdx.x, e1 = threadIdx.x + block_threads();
        auto src = [&](int e) {
            const int b = e / T.W, a = e - b * T.W;
            TileSrc q = tile_src(L.m1, L.m2, L.pitch, L.bcx, L.bcy, T.i0 - 1 + a, T.j0 - 1 + b);
            if (e >= n) q.sc = q.su = q.sv = 0;
            return q;
        };
        const TileSrc s0 = src(e0 < n ? e0 : 0), s1 = src(e1 < n ? e1 : 0);
        const float v0[9] = { L.c[s0.c], L.dc[s0.c], L.dmu[s0.c], L.dp[s0.c], L.du[s0.u], L.dv[s0.v],
                              L.cn[s0.c], L.un[s0.u], L.vn[s0.v] };
        const float v1[9] = { L.c[s1.c], L.dc[s1.c], L.dmu[s1.c], L.dp[s1.c], L.du[s1.u], L.dv[s1.v],
                              L.cn[s1.c], L.un[s1.u], L.vn[s1.v] };
        auto put = [&](int e, const TileSrc &q, const float *v) {
            float *s = T.s + e;
            if (q.sc == 0) {
                for (int f = 0; f < L_NF; f++) s[f * n] = 0.0f;
                return;
            }
            s[L_C * n] = v[0];
            s[L_DC * n] = v[1];
            s[L_MU * n] = v[2];
            s[L_P * n] = v[3];
            s[L_U * n] = signed_val(q.su, v[4]);
            s[L_V * n] = signed_val(q.sv, v[5]);
            s[L_CN * n] = v[6];
            s[L_UN * n] = signed_val(q.su, v[7]);
            s[L_VN * n] = signed_val(q.sv, v[8]);
            s[L_RN * n] = rhof(P, v[6]);
            s[L_MV * n] = viscf(P, v[6]);
            s[L_MOB * n] = mobf(P, v[6]);
            const float rs = rhof(P, v[0]);
            s[L_RS * n] = rs;
            s[L_DRS * n] = -P.alpha * rs * rs * v[1];
        };
        if (e0 < n) put(e0, s0, v0);
        if (e1 < n) put(e1, s1, v1);
        return;
    }
    for (int e = threadIdx.x; e < n; e += block_threads()) {
        const int b = e / T.W, a = e - b * T.W;
        const int i = T.i0 - 1 + a, j = T.j0 - 1 + b;
        float *s = T.s + e;
        if (i > L.m1 + 1 || j > L.m2 + 1) {
            for (int f = 0; f < L_NF; f++) s[f * n] = 0.0f;
            continue;
        }
        const float c = ldc(L.c, L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j);
        const float cn = ldc(L.cn, L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j);
        const float dc = ldc(L.dc, L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j);
        s[L_C * n] = c;
        s[L_DC * n] = dc;
        s[L_MU * n] = ldc(L.dmu, L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j);
        s[L_P * n] = ldc(L.dp, L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j);
        s[L_U * n] = ldu(L.du, L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j);
        s[L_V * n] = ldv(L.dv, L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j);
        s[L_CN * n] = cn;
        s[L_UN * n] = ldu(L.un, L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j);
        s[L_VN * n] = ldv(L.vn, L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j);
        s[L_RN * n] = rhof(P, cn);
        s[L_MV * n] = viscf(P, cn);
        s[L_MOB * n] = mobf(P, cn);
        const float rs = rhof(P, c);
        s[L_RS * n] = rs;
        s[L_DRS * n] = -P.alpha * rs * rs * dc;
    }
}

// reload of the corrections into a tile that ltile_load filled before, after
// a half-sweep of the given colour, with the sources computed once
// (tile_map_build): all face corrections, and the cell corrections and the
// density change of the elements whose source cell has that colour (the
// linearisation point and time-n fields stay)
__device__ __forceinline__ void ltile_refresh_map(const PhysF &P, const LView &L, const TileF &T, const int *map,
                                                  int colour)
{
    const int n = T.W * T.H;
    for (int e = threadIdx.x; e < n; e += block_threads()) {
        // the map entry, then every value the element may take, before any
        // use (as tile_refresh_map)
        const int q = map[4 * e], qu = map[4 * e + 1], qv = map[4 * e + 2], fl = map[4 * e + 3];
        float *s = T.s + e;
        const float du = L.du[qu], dv = L.dv[qv], dc = L.dc[q], dmu = L.dmu[q], dp = L.dp[q], rs = s[L_RS * n];
        __builtin_amdgcn_sched_barrier(0);
        if (fl & 16) continue;
        s[L_U * n] = signed_val((fl & 3) - 1, du);
        s[L_V * n] = signed_val(((fl >> 2) & 3) - 1, dv);
        if (((fl >> 5) & 1) != colour) continue;
        s[L_DC * n] = dc;
        s[L_MU * n] = dmu;
        s[L_P * n] = dp;
        s[L_DRS * n] = -P.alpha * rs * rs * dc;
    }
}

// one axis of the linearised cell equations at element e: the linear terms
// applied to the corrections, the linearised gradient-energy and
// capillary-divergence terms (dG, dL), and the values at c^ that the local
// Jacobian needs
struct LCellAx {
    float adv, div, Lmu, Lp, Sm, Gc, Gn, dG, dL, dGc, dLra, dLrb;
};

__device__ __forceinline__ LCellAx lcell_axis(const TileF &T, const Ax &a, int e, float ih)
{
    const float ih2 = ih * ih;
    const float wP = (a.per || a.ia < a.ma - 1) ? 1.0f : 0.0f, wM = (a.per || a.ia > 0) ? 1.0f : 0.0f;
    const int eP = e + a.dn, eM = e - a.dn;
    const float c = tq(T, L_C, e), cP = tq(T, L_C, eP), cM = tq(T, L_C, eM);
    const float n = tq(T, L_CN, e), nP = tq(T, L_CN, eP), nM = tq(T, L_CN, eM);
    const float dc = tq(T, L_DC, e), dcP = tq(T, L_DC, eP), dcM = tq(T, L_DC, eM);
    const float mu = tq(T, L_MU, e), p = tq(T, L_P, e);
    const float rnP = tq(T, L_RN, eP), rnM = tq(T, L_RN, eM), rn = tq(T, L_RN, e);
    const float rs = tq(T, L_RS, e);
    const float m0 = tq(T, L_MOB, e);
    const float mP = 0.5f * (tq(T, L_MOB, eP) + m0) * wP, mM = 0.5f * (tq(T, L_MOB, eM) + m0) * wM;
    const float uP = tq(T, a.FN, eP), u0 = tq(T, a.FN, e);
    LCellAx x;
    x.adv = 0.5f * ih * (rnP * (nP - n) * uP + rnM * (n - nM) * u0);
    x.div = ih * (uP - u0);
    x.Lmu = ih2 * (mP * (tq(T, L_MU, eP) - mu) - mM * (mu - tq(T, L_MU, eM)));
    x.Lp = ih2 * (mP * (tq(T, L_P, eP) - p) - mM * (p - tq(T, L_P, eM)));
    x.Sm = ih2 * (mP + mM);
    const float dP = cP - c, dM = c - cM, gP = nP - n, gM = n - nM;
    x.Gc = 0.5f * ih2 * (dP * dP + dM * dM);
    x.Gn = 0.5f * ih2 * (gP * gP + gM * gM);
    // d(Gc) = ih2 (dP d(dP) + dM d(dM)); across a wall the mirrored ghost
    // makes both dP and d(dP) vanish
    x.dG = ih2 * (dP * (dcP - dc) + dM * (dc - dcM));
    const float rh = 0.5f * (rs + rn);
    const float kP = 0.5f * (0.5f * (tq(T, L_RS, eP) + rnP) + rh) * wP;
    const float kM = 0.5f * (0.5f * (tq(T, L_RS, eM) + rnM) + rh) * wM;
    const float hP = 0.5f * (dP + gP), hM = 0.5f * (dM + gM);
    const float drs = tq(T, L_DRS, e);
    const float dkP = 0.25f * (tq(T, L_DRS, eP) + drs) * wP, dkM = 0.25f * (tq(T, L_DRS, eM) + drs) * wM;
    x.dL = ih2 * (dkP * hP + kP * 0.5f * (dcP - dc) - dkM * hM - kM * 0.5f * (dc - dcM));
    x.dGc = ih2 * (wP * (-dP) + wM * dM);
    x.dLra = ih2 * (wP * hP - wM * hM);
    x.dLrb = ih2 * (kP + kM);
    return x;
}

__device__ __forceinline__ LCellAx lcell_sum(const LCellAx &x)
{
    LCellAx s;
    s.adv = x.adv + other(x.adv);
    s.div = x.div + other(x.div);
    s.Lmu = x.Lmu + other(x.Lmu);
    s.Lp = x.Lp + other(x.Lp);
    s.Sm = x.Sm + other(x.Sm);
    s.Gc = x.Gc + other(x.Gc);
    s.Gn = x.Gn + other(x.Gn);
    s.dG = x.dG + other(x.dG);
    s.dL = x.dL + other(x.dL);
    s.dGc = x.dGc + other(x.dGc);
    s.dLra = x.dLra + other(x.dLra);
    s.dLrb = x.dLrb + other(x.dLrb);
    return s;
}

// J delta for the three cell equations and the local 2x2 Jacobian in
// (c_ij, mubar_ij) at c^ (the matrix of the FP64 point smoother)
struct LCellEq {
    float Nc, Nmu, Np;
    float Jcc, Jcm, Jmc, Jmm, Jpp;
};

__device__ __forceinline__ LCellEq lcell_eq(const PhysF &P, const TileF &T, int e, const LCellAx &s, float muh)
{
    const float c = tq(T, L_C, e), n = tq(T, L_CN, e);
    const float rs = tq(T, L_RS, e), rn = tq(T, L_RN, e);
    const float dc = tq(T, L_DC, e), dmu = tq(T, L_MU, e);
    const float drs = -P.alpha * rs * rs;
    LCellEq q;
    q.Jcc = (drs * (c - n) + rs) * P.inv_dt;
    q.Nc = q.Jcc * dc + s.adv - P.inv_Pe * s.Lmu - P.alpha * P.inv_Pe * s.Lp;
    q.Np = s.div - P.alpha * P.inv_Pe * s.Lmu - P.alpha * P.alpha * P.inv_Pe * s.Lp;
    const float rh = 0.5f * (rs + rn);
    const float q1 = c * (c - 1.0f), q0 = n * (n - 1.0f);
    const float g = 0.25f * (q1 + q0) * (c + n - 1.0f);
    const float Fh = 0.5f * (0.25f * q1 * q1 + 0.25f * q0 * q0);
    const float r = -P.alpha * rs * rn;
    const float Gh = 0.5f * (s.Gc + s.Gn);
    const float dg = 0.25f * ((2.0f * c - 1.0f) * (c + n - 1.0f) + q1 + q0);
    const float f1 = q1 * (c - 0.5f);
    const float dr = P.alpha * P.alpha * rs * rs * rn;
    // derivative in the cell's own c of every term that is pointwise in it
    const float Jpw = drs * muh - P.K1 * (0.5f * drs * g + rh * dg + 0.5f * f1 * r + Fh * dr) - P.K2 * Gh * dr;
    q.Nmu = rs * dmu + Jpw * dc - P.K2 * 0.5f * s.dG * r + P.K3 * s.dL;
    q.Jcm = P.inv_Pe * s.Sm;
    q.Jmm = rs;
    const float dLr = 0.25f * drs * s.dLra - 0.5f * s.dLrb;
    q.Jmc = Jpw - P.K2 * 0.5f * s.dGc * r + P.K3 * dLr;
    q.Jpp = P.alpha * P.alpha * P.inv_Pe * s.Sm;
    return q;
}

struct FaceEqF {
    float N, diag;
};

// J delta for the momentum equation on the face at element ef, and the
// derivative in the face's own velocity at w^ (uh = that face's velocity at
// w^, which multiplies the change of the density average)
__device__ __forceinline__ FaceEqF lface_eq(const PhysF &P, const TileF &T, const Ax &a, int ef, int it, float ih,
                                            float uh)
{
    const float ih2 = ih * ih;
    const int eL = ef - a.dn, eR = ef, dt = a.dt;
    const float rL = tq(T, L_RN, eL), rR = tq(T, L_RN, eR);
    const float Rt = 0.25f * (rL + rR + tq(T, L_RN, eL + dt) + tq(T, L_RN, eR + dt));
    const float Rb = 0.25f * (rL + rR + tq(T, L_RN, eL - dt) + tq(T, L_RN, eR - dt));
    const float mvL = tq(T, L_MV, eL), mvR = tq(T, L_MV, eR);
    const float nut = 0.25f * (mvL + mvR + tq(T, L_MV, eL + dt) + tq(T, L_MV, eR + dt));
    const float nub = 0.25f * (mvL + mvR + tq(T, L_MV, eL - dt) + tq(T, L_MV, eR - dt));
    const float Arn = 0.5f * (rL + rR);
    const float Ars = 0.5f * (tq(T, L_RS, eL) + tq(T, L_RS, eR));
    const float dArs = 0.5f * (tq(T, L_DRS, eL) + tq(T, L_DRS, eR));
    const float un0 = tq(T, a.FNN, ef);
    const float wL = rL * 0.5f * (tq(T, a.FNN, ef - a.dn) + un0);
    const float wR = rR * 0.5f * (un0 + tq(T, a.FNN, ef + a.dn));
    const float Vt = 0.5f * (tq(T, a.FTN, eL + dt) + tq(T, a.FTN, eR + dt));
    const float Vb = 0.5f * (tq(T, a.FTN, eL) + tq(T, a.FTN, eR));
    const float u0 = tq(T, a.FN, ef), uE = tq(T, a.FN, ef + a.dn), uW = tq(T, a.FN, ef - a.dn);
    const float uN = tq(T, a.FN, ef + dt), uS = tq(T, a.FN, ef - dt);
    const float thR = ih * (uE - u0 + tq(T, a.FT, eR + dt) - tq(T, a.FT, eR));
    const float thL = ih * (u0 - uW + tq(T, a.FT, eL + dt) - tq(T, a.FT, eL));
    const float nL = tq(T, L_CN, eL), nR = tq(T, L_CN, eR);
    FaceEqF q;
    q.N = Arn * u0 * P.inv_dt
        + 0.5f * ih * (wR * uE - wL * uW + Rt * Vt * uN - Rb * Vb * uS)
        + 0.5f * (Ars - Arn) * P.inv_dt * u0 + 0.5f * dArs * P.inv_dt * uh
        + P.inv_M * ih * (tq(T, L_P, eR) - tq(T, L_P, eL))
        - P.inv_M * ih * 0.5f * (rR * tq(T, L_MU, eL) + rL * tq(T, L_MU, eR)) * (nR - nL)
        - P.inv_Re * ih2 * (mvR * (uE - u0) - mvL * (u0 - uW) + nut * (uN - u0) - nub * (u0 - uS))
        - (P.inv_Re / 3.0f) * ih * (mvR * thR - mvL * thL);
    const float gt = (!a.pert && it == a.mt - 1) ? 1.0f : 0.0f, gb = (!a.pert && it == 0) ? 1.0f : 0.0f;
    q.diag = 0.5f * (Arn + Ars) * P.inv_dt + (4.0f / 3.0f) * P.inv_Re * ih2 * (mvL + mvR)
           + P.inv_Re * ih2 * (nut * (1.0f + gt) + nub * (1.0f + gb)) + 0.5f * ih * (gb * Rb * Vb - gt * Rt * Vt);
    return q;
}


// one cell of the current colour: the FP64 smoother applied to the
// correction equation J(w^) delta = r.  Segregated: step 1 is a 2x2 solve for
// (dc, dmu) of the cell, step 2 the 5x5 Vanka box for its four faces and dp.
// Coupled: the seven-unknown box of the FP64 smoother with the entries of J at
// w^ (the face rows' dc entry multiplies the face velocity at w^), eliminated
// the same way.
// With TO set, as relax_cell: the cell at tile position (ti, tj), results
// kept in the tile (dc, dmu, dp and the density change in place, the face
// corrections in the fields L_NF (u) and L_NF + 1 (v)).
template <bool TO, int AS = 0>
__device__ __forceinline__ void lrelax_cell(const PhysF &P, const LView &L, const TileF &T, float *dunew,
                                            float *dvnew, int i, int j, int ti, int tj, int hlf, float omega)
{
    const size_t k = (size_t)j * L.pitch + i;
    const float ih = L.inv_h, ih2 = ih * ih;
    const int e = T.idx(ti, tj);
    const Ax a = make_ax(L, T, i, j, hlf);
    const bool cpl = P.coupled;
    const LCellAx s = lcell_sum(lcell_axis(T, a, e, ih));
    const LCellEq q = lcell_eq(P, T, e, s, lda<AS>(L.mu, k));
    const float r1 = lda<AS>(L.rc, k) - q.Nc, r2 = lda<AS>(L.rmu, k) - q.Nmu;
    const float c0 = tq(T, L_DC, e), m0 = tq(T, L_MU, e);
    const int st = T.W * T.H;
    const float rs = tq(T, L_RS, e);
    float mnew = m0;
    if (!cpl) {
        // ---- step 1
        const float idet = frcpf(q.Jcc * q.Jmm - q.Jcm * q.Jmc);
        const float cnew = c0 + (q.Jmm * r1 - q.Jcm * r2) * idet;
        mnew = m0 + (q.Jcc * r2 - q.Jmc * r1) * idet;
        if (!TO && hlf == 0) {
            sta<AS>(L.dc, k, cnew);
            sta<AS>(L.dmu, k, mnew);
        }
        T.s[L_DC * st + e] = cnew;
        T.s[L_MU * st + e] = mnew;
        T.s[L_DRS * st + e] = -P.alpha * rs * rs * cnew;
    }
    // ---- the box
    const bool hlo = a.per || a.ia >= 1, hhi = a.per || a.ia + 1 < a.ma;
    const int ihi = hlf ? i : (i + 1 < L.m1 ? i + 1 : 0), jhi = hlf ? (j + 1 < L.m2 ? j + 1 : 0) : j;
    const size_t khi = (size_t)jhi * L.pitch + ihi;
    // the velocity at w^ on the lane's two faces (west and east, or south and
    // north, of the cell)
    const float uhlo = lda<AS>(hlf ? L.v : L.u, k), uhhi = lda<AS>(hlf ? L.v : L.u, khi);
    const FaceEqF flo = lface_eq(P, T, a, e, a.it, ih, uhlo);
    const FaceEqF fhi = lface_eq(P, T, a, e + a.dn, a.it, ih, uhhi);
    const float *rN = hlf ? L.rv : L.ru;
    const float blo = hlo ? lda<AS>(rN, k) - flo.N : 0.0f, dlo = hlo ? flo.diag : 1.0f;
    const float bhi = hhi ? lda<AS>(rN, khi) - fhi.N : 0.0f, dhi = hhi ? fhi.diag : 1.0f;
    const float Lmu_new = s.Lmu - s.Sm * (mnew - m0);
    const float bp = lda<AS>(L.rp, k) - (s.div - P.alpha * P.inv_Pe * Lmu_new - P.alpha * P.alpha * P.inv_Pe * s.Lp);
    const float w_ax = tq(T, L_RN, e) * 0.5f * (tq(T, a.FNN, e) + tq(T, a.FNN, e + a.dn));
    const float mv0 = tq(T, L_MV, e);
    const float vis = (4.0f / 3.0f) * P.inv_Re * ih2 * mv0, gd = P.inv_Re * ih2 * mv0 / 3.0f;
    const float gp = P.inv_M * ih;
    // periodic axis of two cells: the box faces meet twice (as in relax_pair)
    float xlo = 0.0f, xhi = 0.0f;
    if (a.per && a.ma == 2) {
        const float w_o = tq(T, L_RN, e - a.dn) * 0.5f * (tq(T, a.FNN, e) + tq(T, a.FNN, e + a.dn));
        const float v_o = (4.0f / 3.0f) * P.inv_Re * ih2 * tq(T, L_MV, e - a.dn);
        xlo = -0.5f * ih * w_o - v_o;
        xhi = 0.5f * ih * w_o - v_o;
    }
    // the box's unknowns in the lane's order, its own axis first (as in the
    // FP64 box)
    const float o_blo = other(blo), o_dlo = other(dlo), o_bhi = other(bhi), o_dhi = other(dhi), o_w = other(w_ax);
    const float o_xlo = other(xlo), o_xhi = other(xhi);
    const int o_hlo = other((int)hlo), o_hhi = other((int)hhi);
    float A[5][5], b[5];
    b[0] = blo; b[1] = bhi; b[2] = o_blo; b[3] = o_bhi; b[4] = bp;
    const float m0l = hlo ? 1.0f : 0.0f, m0h = hhi ? 1.0f : 0.0f, m1l = o_hlo ? 1.0f : 0.0f, m1h = o_hhi ? 1.0f : 0.0f;
    A[0][0] = dlo; A[0][1] = m0l * (0.5f * ih * w_ax - vis) + xlo; A[0][2] = m0l * gd; A[0][3] = -m0l * gd; A[0][4] = m0l * gp;
    A[1][1] = dhi; A[1][0] = m0h * (-0.5f * ih * w_ax - vis) + xhi; A[1][2] = -m0h * gd; A[1][3] = m0h * gd; A[1][4] = -m0h * gp;
    A[2][2] = o_dlo; A[2][3] = m1l * (0.5f * ih * o_w - vis) + o_xlo; A[2][0] = m1l * gd; A[2][1] = -m1l * gd; A[2][4] = m1l * gp;
    A[3][3] = o_dhi; A[3][2] = m1h * (-0.5f * ih * o_w - vis) + o_xhi; A[3][0] = -m1h * gd; A[3][1] = m1h * gd; A[3][4] = -m1h * gp;
    A[4][0] = -m0l * ih; A[4][1] = m0h * ih; A[4][2] = -m1l * ih; A[4][3] = m1h * ih; A[4][4] = q.Jpp;
    float ac[5] = { 0.0f, 0.0f, 0.0f, 0.0f, 0.0f }, icc = 0.0f, bc = 0.0f, imm = 0.0f;
    if (cpl) {
        const int e1 = e + a.dn;
        const float alo = hlo ? 0.5f * ih * tq(T, L_RN, e - a.dn) * (tq(T, L_CN, e) - tq(T, L_CN, e - a.dn)) : 0.0f;
        const float ahi = hhi ? 0.5f * ih * tq(T, L_RN, e1) * (tq(T, L_CN, e1) - tq(T, L_CN, e)) : 0.0f;
        const float ulo = hlo ? uhlo : 0.0f, uhi = hhi ? uhhi : 0.0f;
        ac[0] = alo; ac[1] = ahi; ac[2] = other(alo); ac[3] = other(ahi);
        const float uf[4] = { ulo, uhi, other(ulo), other(uhi) };
        const float gc = 0.25f * (-P.alpha * rs * rs) * P.inv_dt;
        const float Jcp = P.alpha * P.inv_Pe * s.Sm;
        ac[4] = Jcp;
        imm = frcpf(q.Jmm);
        const float kmc = q.Jmc * imm, kbm = r2 * imm;
        icc = frcpf(q.Jcc - q.Jcm * kmc);
        bc = r1 - q.Jcm * kbm;
        float gam[5];
#pragma unroll
        for (int f = 0; f < 4; f++) {
            const float lam = -P.inv_M * ac[f];
            gam[f] = gc * uf[f] - lam * kmc;
            b[f] -= lam * kbm;
        }
        gam[4] = -Jcp * kmc;
        b[4] -= Jcp * kbm;
#pragma unroll
        for (int r = 0; r < 5; r++) {
            const float t = gam[r] * icc;
#pragma unroll
            for (int cc = 0; cc < 5; cc++) A[r][cc] -= t * ac[cc];
            b[r] -= t * bc;
        }
    }
    float inv[5];
#pragma unroll
    for (int cc = 0; cc < 4; cc++) {
        inv[cc] = frcpf(A[cc][cc]);
#pragma unroll
        for (int r = cc + 1; r < 5; r++) {
            const float l = A[r][cc] * inv[cc];
#pragma unroll
            for (int t = cc + 1; t < 5; t++) A[r][t] -= l * A[cc][t];
            b[r] -= l * b[cc];
        }
    }
    inv[4] = frcpf(A[4][4]);
#pragma unroll
    for (int cc = 4; cc >= 0; cc--) {
        float acc = b[cc];
#pragma unroll
        for (int t = cc + 1; t < 5; t++) acc -= A[cc][t] * b[t];
        b[cc] = acc * inv[cc];
    }
    if (cpl && hlf == 0) {
        float acc = bc;
#pragma unroll
        for (int t = 0; t < 5; t++) acc -= ac[t] * b[t];
        const float dc = acc * icc;
        if (TO) {
            T.s[L_DC * st + e] = c0 + dc;
            T.s[L_MU * st + e] = m0 + (r2 - q.Jmc * dc) * imm;
            T.s[L_DRS * st + e] = -P.alpha * rs * rs * (c0 + dc);
        } else {
            sta<AS>(L.dc, k, c0 + dc);
            sta<AS>(L.dmu, k, m0 + (r2 - q.Jmc * dc) * imm);
        }
    }
    const float dl = b[0], dh = b[1];
    if (TO) {
        float *fo = T.s + (L_NF + hlf) * st;
        if (hlo) fo[e] = tq(T, a.FN, e) + omega * dl;
        if (hhi) fo[e + a.dn] = tq(T, a.FN, e + a.dn) + omega * dh;
        if (hlf == 0) T.s[L_P * st + e] = tq(T, L_P, e) + omega * b[4];
        return;
    }
    float *dst = hlf ? dvnew : dunew;
    if (hlo) sta<AS>(dst, k, tq(T, a.FN, e) + omega * dl);
    if (hhi) sta<AS>(dst, khi, tq(T, a.FN, e + a.dn) + omega * dh);
    if (hlf == 0) sta<AS>(L.dp, k, tq(T, L_P, e) + omega * b[4]);
}
template <int AS = 0>
__device__ __forceinline__ void lrelax_pair(const PhysF &P, const LView &L, const TileF &T, float *dunew,
                                            float *dvnew, int i, int j, int hlf, float omega)
{
    lrelax_cell<false, AS>(P, L, T, dunew, dvnew, i, j, i, j, hlf, omega);
}

// residual of the correction equation r - J(w^) delta for the five equations
// attached to cell (i, j) (cell equations; west face on lane 0, south face on
// lane 1, zero for a face on a wall); the level is in global memory
__device__ __forceinline__ void lresid_pair(const PhysF &P, const LView &L, const TileF &T, int i, int j, int hlf,
                                            float &rc, float &rm, float &rp, float &rf)
{
    const size_t k = (size_t)j * L.pitch + i;
    const int e = T.idx(i, j);
    const Ax a = make_ax(L, T, i, j, hlf);
    const LCellAx s = lcell_sum(lcell_axis(T, a, e, L.inv_h));
    const LCellEq q = lcell_eq(P, T, e, s, lda<1>(L.mu, k));
    rc = lda<1>(L.rc, k) - q.Nc;
    rm = lda<1>(L.rmu, k) - q.Nmu;
    rp = lda<1>(L.rp, k) - q.Np;
    const bool hlo = a.per || a.ia >= 1;
    // (the velocity at w^ on the lane's face)
    const FaceEqF f = lface_eq(P, T, a, e, a.it, L.inv_h, lda<1>(hlf ? L.v : L.u, k));
    rf = hlo ? lda<1>(hlf ? L.rv : L.ru, k) - f.N : 0.0f;
}

} // namespace qn
