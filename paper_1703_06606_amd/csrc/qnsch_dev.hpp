// qnsch_dev.hpp -- device side of the FP64 multigrid step (gfx950).
//
// The discrete system is the fully discrete primitive scheme of sec. 6.1
// ((pm-num-mx)-(pm-num-chem), App. A.4-A.6); every equation is written as
// "left side minus right side", N(w) = 0 at time n+1.  The smoother is the
// one of sec. 7.1: per cell a Newton step on the Cahn-Hilliard pair
// (c, mubar), then a Vanka box solve for the four faces and the pressure of
// the cell, in red-black order.
//
// Layout: every field of a level is an m2 x pitch array of doubles, row j,
// column i.  Cell fields at cell (i,j); u(i,j) on the west face of cell (i,j)
// (x = i h); v(i,j) on the south face (y = j h).  Ghosts are not stored: the
// loaders below apply the boundary conditions of App. A.4.
#pragma once
#include <hip/hip_runtime.h>

namespace qn {

struct Phys {
    double rho1, rho2, rho12, drho;  // rho(c) = rho12 / (drho c + rho1)
    double visc1, visc2, visc12, dvisc;
    double alpha, inv_Re, inv_M, inv_Pe, K1, K2, K3, inv_Fr, rho_ref, mob_reg;
    double inv_dt;
};

struct View {
    double *c, *mu, *p;         // cell unknowns
    const double *u, *v;        // face unknowns (the buffer being read)
    const double *cn, *un, *vn; // time-n data
    int m1, m2, pitch;
    int bcx, bcy;               // 0 wall, 1 periodic
    double inv_h;
};

// --------------------------------------------------------------------------
// loaders with boundary conditions

__device__ __forceinline__ int wrapi(int k, int n) { return k < 0 ? k + n : (k >= n ? k - n : k); }

// cell field: Neumann mirror or periodic image (x first, then y)
__device__ __forceinline__ double ldc(const double *f, const View &L, int i, int j)
{
    if (i < 0 || i >= L.m1) i = L.bcx ? wrapi(i, L.m1) : (i < 0 ? 0 : L.m1 - 1);
    if (j < 0 || j >= L.m2) j = L.bcy ? wrapi(j, L.m2) : (j < 0 ? 0 : L.m2 - 1);
    return f[(size_t)j * L.pitch + i];
}
// east-west face field at x = i h, row j: zero on x-walls, reflected
// (ghost = -interior) across y-walls
__device__ __forceinline__ double ldu(const double *f, const View &L, int i, int j)
{
    if (L.bcx) i = wrapi(i, L.m1);
    else if (i <= 0 || i >= L.m1) return 0.0;
    if (j < 0 || j >= L.m2) {
        if (L.bcy) j = wrapi(j, L.m2);
        else return -f[(size_t)(j < 0 ? 0 : L.m2 - 1) * L.pitch + i];
    }
    return f[(size_t)j * L.pitch + i];
}
__device__ __forceinline__ double ldv(const double *f, const View &L, int i, int j)
{
    if (L.bcy) j = wrapi(j, L.m2);
    else if (j <= 0 || j >= L.m2) return 0.0;
    if (i < 0 || i >= L.m1) {
        if (L.bcx) i = wrapi(i, L.m1);
        else return -f[(size_t)j * L.pitch + (i < 0 ? 0 : L.m1 - 1)];
    }
    return f[(size_t)j * L.pitch + i];
}
__device__ __forceinline__ bool u_unk(const View &L, int i) { return L.bcx || (i >= 1 && i <= L.m1 - 1); }
__device__ __forceinline__ bool v_unk(const View &L, int j) { return L.bcy || (j >= 1 && j <= L.m2 - 1); }

// --------------------------------------------------------------------------
// material laws (sec. 2.1, sec. 6.1)

__device__ __forceinline__ double rho_of(const Phys &P, double c) { return P.rho12 / (P.drho * c + P.rho1); }
__device__ __forceinline__ double visc_of(const Phys &P, double c) { return P.visc12 / (P.dvisc * c + P.visc1); }
__device__ __forceinline__ double mob_of(const Phys &P, double c)
{
    double q = c * (1.0 - c);
    return sqrt(q * q + P.mob_reg);
}
__device__ __forceinline__ double dwell(double c)
{
    double q = c * (c - 1.0);
    return 0.25 * q * q;
}

// --------------------------------------------------------------------------
// cell equations: phase (pm-num-phase), chemical potential (pm-num-chem) and
// mass (pm-num-mass), with the entries of their Jacobian the smoother needs

struct CellEq {
    double Nc, Nmu, Np;
    double Jcc, Jcm, Jmc, Jmm; // d(Nc,Nmu)/d(c,mu) at the cell
    double Jpp;                // dNp/dp at the cell
};

__device__ __forceinline__ CellEq eq_cell(const Phys &P, const View &L, int i, int j)
{
    const double ih = L.inv_h, ih2 = ih * ih;
    // 5-point gathers (E, W, N, S) with boundary images
    const double c = ldc(L.c, L, i, j), cE = ldc(L.c, L, i + 1, j), cW = ldc(L.c, L, i - 1, j),
                 cN = ldc(L.c, L, i, j + 1), cS = ldc(L.c, L, i, j - 1);
    const double n = ldc(L.cn, L, i, j), nE = ldc(L.cn, L, i + 1, j), nW = ldc(L.cn, L, i - 1, j),
                 nN = ldc(L.cn, L, i, j + 1), nS = ldc(L.cn, L, i, j - 1);
    const double mu = ldc(L.mu, L, i, j), muE = ldc(L.mu, L, i + 1, j), muW = ldc(L.mu, L, i - 1, j),
                 muN = ldc(L.mu, L, i, j + 1), muS = ldc(L.mu, L, i, j - 1);
    const double p = ldc(L.p, L, i, j), pE = ldc(L.p, L, i + 1, j), pW = ldc(L.p, L, i - 1, j),
                 pN = ldc(L.p, L, i, j + 1), pS = ldc(L.p, L, i, j - 1);
    const double uE = ldu(L.u, L, i + 1, j), uW = ldu(L.u, L, i, j);
    const double vN = ldv(L.v, L, i, j + 1), vS = ldv(L.v, L, i, j);
    // faces that lie on a wall carry no flux (the mirrored ghost equals the cell)
    const double wE = (L.bcx || i < L.m1 - 1) ? 1.0 : 0.0, wW = (L.bcx || i > 0) ? 1.0 : 0.0;
    const double wN = (L.bcy || j < L.m2 - 1) ? 1.0 : 0.0, wS = (L.bcy || j > 0) ? 1.0 : 0.0;

    const double rn = rho_of(P, n), rnE = rho_of(P, nE), rnW = rho_of(P, nW), rnN = rho_of(P, nN), rnS = rho_of(P, nS);
    const double rs = rho_of(P, c);
    // mobility m(c^n) averaged to the faces (A m)
    const double m0 = mob_of(P, n);
    const double mE = 0.5 * (mob_of(P, nE) + m0) * wE, mW = 0.5 * (mob_of(P, nW) + m0) * wW;
    const double mN = 0.5 * (mob_of(P, nN) + m0) * wN, mS = 0.5 * (mob_of(P, nS) + m0) * wS;
    const double Lmu = ih2 * (mE * (muE - mu) - mW * (mu - muW) + mN * (muN - mu) - mS * (mu - muS));
    const double Lp = ih2 * (mE * (pE - p) - mW * (p - pW) + mN * (pN - p) - mS * (p - pS));
    const double Sm = ih2 * (mE + mW + mN + mS);

    CellEq e;
    // advection rho^n u . grad c^n in the special form of App. A.5
    const double adv = 0.5 * ih * (rnE * (nE - n) * uE + rnW * (n - nW) * uW + rnN * (nN - n) * vN + rnS * (n - nS) * vS);
    e.Nc = rs * (c - n) * P.inv_dt + adv - P.inv_Pe * Lmu - P.alpha * P.inv_Pe * Lp;
    e.Np = ih * (uE - uW + vN - vS) - P.alpha * P.inv_Pe * Lmu - P.alpha * P.alpha * P.inv_Pe * Lp;

    // chemical potential: time averages of sec. 4.1, pointwise |grad_D c|^2
    const double rh = 0.5 * (rs + rn);
    const double q1 = c * (c - 1.0), q0 = n * (n - 1.0);
    const double g = 0.25 * (q1 + q0) * (c + n - 1.0);
    const double Fh = 0.5 * (dwell(c) + dwell(n));
    const double r = -P.alpha * rs * rn;
    const double dE = cE - c, dW = c - cW, dN = cN - c, dS = c - cS;
    const double Gc = 0.5 * ih2 * (dE * dE + dW * dW + dN * dN + dS * dS);
    const double eE = nE - n, eW = n - nW, eN = nN - n, eS = n - nS;
    const double Gn = 0.5 * ih2 * (eE * eE + eW * eW + eN * eN + eS * eS);
    const double Gh = 0.5 * (Gc + Gn);
    // div_d(A rho^{n+1/2} grad_D c^{n+1/2}); rho^{n+1/2} of a neighbour from its c and c^n
    const double rhE = 0.5 * (rho_of(P, cE) + rnE), rhW = 0.5 * (rho_of(P, cW) + rnW);
    const double rhN = 0.5 * (rho_of(P, cN) + rnN), rhS = 0.5 * (rho_of(P, cS) + rnS);
    const double kE = 0.5 * (rhE + rh) * wE, kW = 0.5 * (rhW + rh) * wW, kN = 0.5 * (rhN + rh) * wN, kS = 0.5 * (rhS + rh) * wS;
    const double hE = 0.5 * (dE + eE), hW = 0.5 * (dW + eW), hN = 0.5 * (dN + eN), hS = 0.5 * (dS + eS);
    const double Lr = ih2 * (kE * hE - kW * hW + kN * hN - kS * hS);
    e.Nmu = rs * mu - P.K1 * (rh * g + Fh * r) - P.K2 * Gh * r + P.K3 * Lr;

    // Jacobian in (c_ij, mubar_ij); rho' = -alpha rho^2
    const double drs = -P.alpha * rs * rs;
    e.Jcc = (drs * (c - n) + rs) * P.inv_dt;
    e.Jcm = P.inv_Pe * Sm;
    e.Jmm = rs;
    const double dg = 0.25 * ((2.0 * c - 1.0) * (c + n - 1.0) + q1 + q0);
    const double f1 = q1 * (c - 0.5);                  // F'(c)
    const double dr = P.alpha * P.alpha * rs * rs * rn; // dr/dc
    const double dGc = ih2 * (wE * (-dE) + wW * dW + wN * (-dN) + wS * dS);
    // d Lr / dc: the cell's own rho^{n+1/2} and c^{n+1/2} both move
    const double dLr = ih2 * (0.25 * drs * (wE * hE - wW * hW + wN * hN - wS * hS) - 0.5 * (kE + kW + kN + kS));
    e.Jmc = drs * mu - P.K1 * (0.5 * drs * g + rh * dg + 0.5 * f1 * r + Fh * dr) - P.K2 * (0.5 * dGc * r + Gh * dr) + P.K3 * dLr;
    e.Jpp = P.alpha * P.alpha * P.inv_Pe * Sm;
    return e;
}

// --------------------------------------------------------------------------
// momentum equations (pm-num-mx) at a face, with the derivative with respect
// to the face's own velocity.  The advection (e1e1-1) plus the half-divergence
// term (e1e1-2) are combined into their skew form
//   1/(2h) [w_R u_{i+1} - w_L u_{i-1} + Z_t u_{j+1} - Z_b u_{j-1}],
// which is the same sum with the terms on the face's own value cancelled.

struct FaceEq {
    double N, diag;
};

__device__ __forceinline__ FaceEq eq_u(const Phys &P, const View &L, int i, int j)
{
    const double ih = L.inv_h, ih2 = ih * ih;
    // cells L = (i-1, j), R = (i, j) and the rows above and below
    const double nL = ldc(L.cn, L, i - 1, j), nR = ldc(L.cn, L, i, j);
    const double nLt = ldc(L.cn, L, i - 1, j + 1), nRt = ldc(L.cn, L, i, j + 1);
    const double nLb = ldc(L.cn, L, i - 1, j - 1), nRb = ldc(L.cn, L, i, j - 1);
    const double rL = rho_of(P, nL), rR = rho_of(P, nR);
    const double Rt = 0.25 * (rL + rR + rho_of(P, nLt) + rho_of(P, nRt));
    const double Rb = 0.25 * (rL + rR + rho_of(P, nLb) + rho_of(P, nRb));
    const double mvL = visc_of(P, nL), mvR = visc_of(P, nR);
    const double nut = 0.25 * (mvL + mvR + visc_of(P, nLt) + visc_of(P, nRt));
    const double nub = 0.25 * (mvL + mvR + visc_of(P, nLb) + visc_of(P, nRb));
    const double Arn = 0.5 * (rL + rR);
    const double Ars = 0.5 * (rho_of(P, ldc(L.c, L, i - 1, j)) + rho_of(P, ldc(L.c, L, i, j)));
    const double un0 = ldu(L.un, L, i, j);
    const double wL = rL * 0.5 * (ldu(L.un, L, i - 1, j) + un0);
    const double wR = rR * 0.5 * (un0 + ldu(L.un, L, i + 1, j));
    const double Vt = 0.5 * (ldv(L.vn, L, i - 1, j + 1) + ldv(L.vn, L, i, j + 1));
    const double Vb = 0.5 * (ldv(L.vn, L, i - 1, j) + ldv(L.vn, L, i, j));
    const double u0 = ldu(L.u, L, i, j), uE = ldu(L.u, L, i + 1, j), uW = ldu(L.u, L, i - 1, j);
    const double uN = ldu(L.u, L, i, j + 1), uS = ldu(L.u, L, i, j - 1);
    const double thR = ih * (uE - u0 + ldv(L.v, L, i, j + 1) - ldv(L.v, L, i, j));
    const double thL = ih * (u0 - uW + ldv(L.v, L, i - 1, j + 1) - ldv(L.v, L, i - 1, j));
    const double pL = ldc(L.p, L, i - 1, j), pR = ldc(L.p, L, i, j);
    const double muL = ldc(L.mu, L, i - 1, j), muR = ldc(L.mu, L, i, j);

    FaceEq e;
    e.N = Arn * (u0 - un0) * P.inv_dt
        + 0.5 * ih * (wR * uE - wL * uW + Rt * Vt * uN - Rb * Vb * uS)
        + 0.5 * (Ars - Arn) * P.inv_dt * u0
        + P.inv_M * ih * (pR - pL)
        - P.inv_M * ih * 0.5 * (rR * muL + rL * muR) * (nR - nL)
        - P.inv_Re * ih2 * (mvR * (uE - u0) - mvL * (u0 - uW) + nut * (uN - u0) - nub * (u0 - uS))
        - (P.inv_Re / 3.0) * ih * (mvR * thR - mvL * thL);
    // own-face derivative; across a y-wall the reflected ghost doubles the
    // viscous coupling and the advection coefficient enters with a sign flip
    const bool gt = !L.bcy && j == L.m2 - 1, gb = !L.bcy && j == 0;
    e.diag = 0.5 * (Arn + Ars) * P.inv_dt + (4.0 / 3.0) * P.inv_Re * ih2 * (mvL + mvR)
           + P.inv_Re * ih2 * (nut * (gt ? 2.0 : 1.0) + nub * (gb ? 2.0 : 1.0))
           + 0.5 * ih * ((gb ? Rb * Vb : 0.0) - (gt ? Rt * Vt : 0.0));
    return e;
}

__device__ __forceinline__ FaceEq eq_v(const Phys &P, const View &L, int i, int j)
{
    const double ih = L.inv_h, ih2 = ih * ih;
    // cells B = (i, j-1), T = (i, j) and the columns left and right
    const double nB = ldc(L.cn, L, i, j - 1), nT = ldc(L.cn, L, i, j);
    const double nBr = ldc(L.cn, L, i + 1, j - 1), nTr = ldc(L.cn, L, i + 1, j);
    const double nBl = ldc(L.cn, L, i - 1, j - 1), nTl = ldc(L.cn, L, i - 1, j);
    const double rB = rho_of(P, nB), rT = rho_of(P, nT);
    const double Rr = 0.25 * (rB + rT + rho_of(P, nBr) + rho_of(P, nTr));
    const double Rl = 0.25 * (rB + rT + rho_of(P, nBl) + rho_of(P, nTl));
    const double mvB = visc_of(P, nB), mvT = visc_of(P, nT);
    const double nur = 0.25 * (mvB + mvT + visc_of(P, nBr) + visc_of(P, nTr));
    const double nul = 0.25 * (mvB + mvT + visc_of(P, nBl) + visc_of(P, nTl));
    const double Arn = 0.5 * (rB + rT);
    const double Ars = 0.5 * (rho_of(P, ldc(L.c, L, i, j - 1)) + rho_of(P, ldc(L.c, L, i, j)));
    const double vn0 = ldv(L.vn, L, i, j);
    const double wB = rB * 0.5 * (ldv(L.vn, L, i, j - 1) + vn0);
    const double wT = rT * 0.5 * (vn0 + ldv(L.vn, L, i, j + 1));
    const double Ur = 0.5 * (ldu(L.un, L, i + 1, j - 1) + ldu(L.un, L, i + 1, j));
    const double Ul = 0.5 * (ldu(L.un, L, i, j - 1) + ldu(L.un, L, i, j));
    const double v0 = ldv(L.v, L, i, j), vN = ldv(L.v, L, i, j + 1), vS = ldv(L.v, L, i, j - 1);
    const double vE = ldv(L.v, L, i + 1, j), vW = ldv(L.v, L, i - 1, j);
    const double thT = ih * (ldu(L.u, L, i + 1, j) - ldu(L.u, L, i, j) + vN - v0);
    const double thB = ih * (ldu(L.u, L, i + 1, j - 1) - ldu(L.u, L, i, j - 1) + v0 - vS);
    const double pB = ldc(L.p, L, i, j - 1), pT = ldc(L.p, L, i, j);
    const double muB = ldc(L.mu, L, i, j - 1), muT = ldc(L.mu, L, i, j);

    FaceEq e;
    e.N = Arn * (v0 - vn0) * P.inv_dt
        + 0.5 * ih * (Rr * Ur * vE - Rl * Ul * vW + wT * vN - wB * vS)
        + 0.5 * (Ars - Arn) * P.inv_dt * v0
        + P.inv_M * ih * (pT - pB)
        - P.inv_M * ih * 0.5 * (rT * muB + rB * muT) * (nT - nB)
        - P.inv_Re * ih2 * (nur * (vE - v0) - nul * (v0 - vW) + mvT * (vN - v0) - mvB * (v0 - vS))
        - (P.inv_Re / 3.0) * ih * (mvT * thT - mvB * thB)
        + P.inv_Fr * (Arn - P.rho_ref);
    const bool gr = !L.bcx && i == L.m1 - 1, gl = !L.bcx && i == 0;
    e.diag = 0.5 * (Arn + Ars) * P.inv_dt + (4.0 / 3.0) * P.inv_Re * ih2 * (mvB + mvT)
           + P.inv_Re * ih2 * (nur * (gr ? 2.0 : 1.0) + nul * (gl ? 2.0 : 1.0))
           + 0.5 * ih * ((gl ? Rl * Ul : 0.0) - (gr ? Rr * Ur : 0.0));
    return e;
}

// --------------------------------------------------------------------------
// smoother for one cell of the current colour (sec. 7.1)

struct Rhs {
    const double *fc, *fmu, *fp, *fu, *fv; // FAS right-hand side; NULL = 0
};
__device__ __forceinline__ double ldf(const double *f, const View &L, int i, int j)
{
    return f ? f[(size_t)j * L.pitch + i] : 0.0;
}

// Step 1 (CH point Newton) and step 2 (Vanka box) at cell (i,j).  Velocities
// are read from L.u/L.v (the snapshot of this colour) and the box faces are
// written to unew/vnew; c, mubar, pbar are updated in place.
__device__ __forceinline__ void relax_cell(const Phys &P, const View &L, const Rhs &F, double *unew, double *vnew,
                                           int i, int j, double omega)
{
    const size_t k = (size_t)j * L.pitch + i;
    // ---- step 1: Newton on (N_c, N_mu) in (c_ij, mubar_ij)
    {
        CellEq e = eq_cell(P, L, i, j);
        const double r1 = ldf(F.fc, L, i, j) - e.Nc, r2 = ldf(F.fmu, L, i, j) - e.Nmu;
        const double det = e.Jcc * e.Jmm - e.Jcm * e.Jmc;
        const double dc = (e.Jmm * r1 - e.Jcm * r2) / det;
        const double dm = (e.Jcc * r2 - e.Jmc * r1) / det;
        L.c[k] += dc;
        L.mu[k] += dm;
    }
    // ---- step 2: Vanka box, unknowns (uW, uE, vS, vN, p)
    const int ie = i + 1 < L.m1 ? i + 1 : 0; // storage column of the east face (periodic)
    const int jn = j + 1 < L.m2 ? j + 1 : 0;
    const bool hW = u_unk(L, i), hE = L.bcx || i + 1 < L.m1;
    const bool hS = v_unk(L, j), hN = L.bcy || j + 1 < L.m2;
    const double ih = L.inv_h, ih2 = ih * ih;
    double A[5][5], b[5];
    for (int r = 0; r < 5; r++)
        for (int s = 0; s < 5; s++) A[r][s] = 0.0;
    // box-cell coefficients of the off-diagonal couplings
    const double n0 = ldc(L.cn, L, i, j);
    const double r0 = rho_of(P, n0), mv0 = visc_of(P, n0);
    const double wx = r0 * 0.5 * (ldu(L.un, L, i, j) + ldu(L.un, L, i + 1, j)); // rho^n a_x u^n at the cell
    const double wy = r0 * 0.5 * (ldv(L.vn, L, i, j) + ldv(L.vn, L, i, j + 1));
    const double vis = (4.0 / 3.0) * P.inv_Re * ih2 * mv0, gd = P.inv_Re * ih2 * mv0 / 3.0;
    const double gp = P.inv_M * ih;
    if (hW) {
        FaceEq e = eq_u(P, L, i, j);
        A[0][0] = e.diag; A[0][1] = 0.5 * ih * wx - vis; A[0][2] = gd; A[0][3] = -gd; A[0][4] = gp;
        b[0] = ldf(F.fu, L, i, j) - e.N;
    } else { A[0][0] = 1.0; b[0] = 0.0; }
    if (hE) {
        FaceEq e = eq_u(P, L, i + 1, j);
        A[1][1] = e.diag; A[1][0] = -0.5 * ih * wx - vis; A[1][2] = -gd; A[1][3] = gd; A[1][4] = -gp;
        b[1] = ldf(F.fu, L, ie, j) - e.N;
    } else { A[1][1] = 1.0; b[1] = 0.0; }
    if (hS) {
        FaceEq e = eq_v(P, L, i, j);
        A[2][2] = e.diag; A[2][3] = 0.5 * ih * wy - vis; A[2][0] = gd; A[2][1] = -gd; A[2][4] = gp;
        b[2] = ldf(F.fv, L, i, j) - e.N;
    } else { A[2][2] = 1.0; b[2] = 0.0; }
    if (hN) {
        FaceEq e = eq_v(P, L, i, j + 1);
        A[3][3] = e.diag; A[3][2] = -0.5 * ih * wy - vis; A[3][0] = -gd; A[3][1] = gd; A[3][4] = -gp;
        b[3] = ldf(F.fv, L, i, jn) - e.N;
    } else { A[3][3] = 1.0; b[3] = 0.0; }
    {
        CellEq e = eq_cell(P, L, i, j);
        A[4][0] = hW ? -ih : 0.0; A[4][1] = hE ? ih : 0.0; A[4][2] = hS ? -ih : 0.0; A[4][3] = hN ? ih : 0.0;
        A[4][4] = e.Jpp;
        b[4] = ldf(F.fp, L, i, j) - e.Np;
    }
    // Gaussian elimination in the order u, u, v, v, p: the velocity block has a
    // positive definite symmetric part (mass + viscous; advection is skew) and
    // the last pivot is the positive pressure Schur complement
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const double inv = 1.0 / A[q][q];
#pragma unroll
        for (int r = q + 1; r < 5; r++) {
            const double l = A[r][q] * inv;
#pragma unroll
            for (int s = q + 1; s < 5; s++) A[r][s] -= l * A[q][s];
            b[r] -= l * b[q];
        }
    }
#pragma unroll
    for (int q = 4; q >= 0; q--) {
        double s = b[q];
#pragma unroll
        for (int t = q + 1; t < 5; t++) s -= A[q][t] * b[t];
        b[q] = s / A[q][q];
    }
    if (hW) unew[k] = L.u[k] + omega * b[0];
    if (hE) unew[(size_t)j * L.pitch + ie] = L.u[(size_t)j * L.pitch + ie] + omega * b[1];
    if (hS) vnew[k] = L.v[k] + omega * b[2];
    if (hN) vnew[(size_t)jn * L.pitch + i] = L.v[(size_t)jn * L.pitch + i] + omega * b[3];
    L.p[k] += omega * b[4];
}

} // namespace qn
