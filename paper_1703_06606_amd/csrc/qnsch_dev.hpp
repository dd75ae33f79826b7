// qnsch_dev.hpp -- device side of the FP64 multigrid step (gfx950).
//
// The discrete system is the fully discrete primitive scheme of sec. 6.1
// ((pm-num-mx)-(pm-num-chem), App. A.4-A.6); every equation is written as
// "left side minus right side", N(w) = 0 at time n+1.  The smoother is the
// one of sec. 7.1: per cell a Newton step on the Cahn-Hilliard pair
// (c, mubar), then a Vanka box solve for the four faces and the pressure of
// the cell (or one Newton step on all seven), in red-black order.  The
// projection scheme of sec. 6.2 is the second option (P.scheme, end of file).
//
// Layout: every field of a level is an m2 x pitch array of doubles, row j,
// column i.  Cell fields at cell (i,j); u(i,j) on the west face of cell (i,j)
// (x = i h); v(i,j) on the south face (y = j h).  Ghosts are not stored.
//
// Work is organised in LDS tiles: a workgroup loads a TX x TY block of cells
// with a halo of one cell below and two above in each direction (the reach of
// a Vanka box), applying the boundary conditions of App. A.4 while loading,
// and computes the cell functions of the time-n data (rho^n, mu(c^n), m(c^n))
// and rho(c) once per tile element.  The equations below then read the tile
// without any boundary logic.
#pragma once
#include <hip/hip_runtime.h>

namespace qn {

// threads of the workgroup.  Every launch of this library has whole
// workgroups, so this is the dispatch's group size: the 16-bit field at byte
// 12 of the implicit kernel arguments (code object v5), read with a scalar
// load of its 32-bit word.  blockDim.x also allows for a partial last
// workgroup and reads the field with a vector load, one memory latency at the
// start of every kernel that uses it.
__device__ __forceinline__ int block_threads()
{
    const __attribute__((address_space(4))) unsigned int *p =
        (const __attribute__((address_space(4))) unsigned int *)__builtin_amdgcn_implicitarg_ptr();
    return (int)(p[3] & 0xffffu);
}

struct Phys {
    double rho1, rho2, rho12, drho;  // rho(c) = rho12 / (drho c + rho1)
    double visc1, visc2, visc12, dvisc;
    double alpha, inv_Re, inv_M, inv_Pe, K1, K2, K3, inv_Fr, rho_ref, mob_reg;
    double inv_dt, dt;
    int coupled; // smoother: 1 = one Newton step on the seven-unknown box, 0 = the two steps
    int scheme;  // 0 = primitive scheme (sec. 6.1), 1 = projection scheme (sec. 6.2)
};

struct View {
    double *c, *mu, *p;         // cell unknowns
    const double *u, *v;        // face unknowns (the buffer being read)
    const double *cn, *un, *vn; // time-n data
    int m1, m2, pitch;
    int bcx, bcy;               // 0 wall, 1 periodic
    double inv_h;
};

struct Rhs {
    const double *fc, *fmu, *fp, *fu, *fv; // FAS right-hand side; NULL = 0
};

// --------------------------------------------------------------------------
// loaders with boundary conditions (used only by the tile loader)

__device__ __forceinline__ int wrapi(int k, int n) { return k < 0 ? k + n : (k >= n ? k - n : k); }

// cell field: Neumann mirror or periodic image (x first, then y)
template <typename R>
__device__ __forceinline__ R ldc(const R *f, int m1, int m2, int pitch, int bcx, int bcy, int i, int j)
{
    if (i < 0 || i >= m1) i = bcx ? wrapi(i, m1) : (i < 0 ? 0 : m1 - 1);
    if (j < 0 || j >= m2) j = bcy ? wrapi(j, m2) : (j < 0 ? 0 : m2 - 1);
    return f[(size_t)j * pitch + i];
}
// east-west face field at x = i h, row j: zero on (and beyond) x-walls,
// reflected (ghost = -interior) across y-walls
template <typename R>
__device__ __forceinline__ R ldu(const R *f, int m1, int m2, int pitch, int bcx, int bcy, int i, int j)
{
    if (bcx) i = wrapi(i, m1);
    else if (i <= 0 || i >= m1) return R(0);
    if (j < 0 || j >= m2) {
        if (bcy) j = wrapi(j, m2);
        else return -f[(size_t)(j < 0 ? 0 : m2 - 1) * pitch + i];
    }
    return f[(size_t)j * pitch + i];
}
template <typename R>
__device__ __forceinline__ R ldv(const R *f, int m1, int m2, int pitch, int bcx, int bcy, int i, int j)
{
    if (bcy) j = wrapi(j, m2);
    else if (j <= 0 || j >= m2) return R(0);
    if (i < 0 || i >= m1) {
        if (bcx) i = wrapi(i, m1);
        else return -f[(size_t)j * pitch + (i < 0 ? 0 : m1 - 1)];
    }
    return f[(size_t)j * pitch + i];
}
// Where a tile element (i, j) comes from, for each kind of field: the array
// index and a sign (1; -1 for a reflected tangential ghost of a face field;
// 0 for a wall face, which is zero) as ldc, ldu, ldv resolve them; beyond the
// reach of any cell of the level (a tile larger than the level) every sign
// is 0 and the element is all zero.  Computing all sources first lets a
// thread issue all its loads at once.
struct TileSrc {
    int c, u, v;    // array indices (always valid)
    int sc, su, sv; // signs
};
__device__ __forceinline__ TileSrc tile_src(int m1, int m2, int pitch, int bcx, int bcy, int i, int j)
{
    TileSrc s;
    if (i > m1 + 1 || j > m2 + 1) {
        s.c = s.u = s.v = 0;
        s.sc = s.su = s.sv = 0;
        return s;
    }
    int ic = i, jc = j;
    if (ic < 0 || ic >= m1) ic = bcx ? wrapi(ic, m1) : (ic < 0 ? 0 : m1 - 1);
    if (jc < 0 || jc >= m2) jc = bcy ? wrapi(jc, m2) : (jc < 0 ? 0 : m2 - 1);
    s.c = jc * pitch + ic;
    s.sc = 1;
    int iu = i, ju = j;
    s.su = 1;
    if (bcx) iu = wrapi(iu, m1);
    else if (iu <= 0 || iu >= m1) { s.su = 0; iu = 0; }
    if (ju < 0 || ju >= m2) {
        if (bcy) ju = wrapi(ju, m2);
        else { s.su = -s.su; ju = ju < 0 ? 0 : m2 - 1; }
    }
    s.u = ju * pitch + iu;
    int iv = i, jv = j;
    s.sv = 1;
    if (bcy) jv = wrapi(jv, m2);
    else if (jv <= 0 || jv >= m2) { s.sv = 0; jv = 0; }
    if (iv < 0 || iv >= m1) {
        if (bcx) iv = wrapi(iv, m1);
        else { s.sv = -s.sv; iv = iv < 0 ? 0 : m1 - 1; }
    }
    s.v = jv * pitch + iv;
    return s;
}
// the sources of tile_src as level coordinates: cell (ic, jc), u face
// (iu, ju), v face (iv, jv), resolved by the same rules (tile_src keeps its own
// copy: composing it from this one measured slower in the tile loads)
struct TileSrcIJ {
    int ic, jc, iu, ju, iv, jv;
    int sc, su, sv;
};
__device__ __forceinline__ TileSrcIJ tile_src_ij(int m1, int m2, int bcx, int bcy, int i, int j)
{
    TileSrcIJ s;
    if (i > m1 + 1 || j > m2 + 1) {
        s.ic = s.jc = s.iu = s.ju = s.iv = s.jv = 0;
        s.sc = s.su = s.sv = 0;
        return s;
    }
    int ic = i, jc = j;
    if (ic < 0 || ic >= m1) ic = bcx ? wrapi(ic, m1) : (ic < 0 ? 0 : m1 - 1);
    if (jc < 0 || jc >= m2) jc = bcy ? wrapi(jc, m2) : (jc < 0 ? 0 : m2 - 1);
    s.ic = ic; s.jc = jc;
    s.sc = 1;
    int iu = i, ju = j;
    s.su = 1;
    if (bcx) iu = wrapi(iu, m1);
    else if (iu <= 0 || iu >= m1) { s.su = 0; iu = 0; }
    if (ju < 0 || ju >= m2) {
        if (bcy) ju = wrapi(ju, m2);
        else { s.su = -s.su; ju = ju < 0 ? 0 : m2 - 1; }
    }
    s.iu = iu; s.ju = ju;
    int iv = i, jv = j;
    s.sv = 1;
    if (bcy) jv = wrapi(jv, m2);
    else if (jv <= 0 || jv >= m2) { s.sv = 0; jv = 0; }
    if (iv < 0 || iv >= m1) {
        if (bcx) iv = wrapi(iv, m1);
        else { s.sv = -s.sv; iv = iv < 0 ? 0 : m1 - 1; }
    }
    s.iv = iv; s.jv = jv;
    return s;
}
template <typename R> __device__ __forceinline__ R signed_val(int sg, R x) { return sg > 0 ? x : (sg < 0 ? -x : R(0)); }

__device__ __forceinline__ bool u_unk(const View &L, int i) { return L.bcx || (i >= 1 && i <= L.m1 - 1); }
__device__ __forceinline__ bool v_unk(const View &L, int j) { return L.bcy || (j >= 1 && j <= L.m2 - 1); }

// --------------------------------------------------------------------------
// material laws (sec. 2.1, sec. 6.1)

// reciprocal: hardware estimate refined by two Newton steps (relative error a
// few ulp, far below the solver tolerances)
__device__ __forceinline__ double frcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ double rho_of(const Phys &P, double c) { return P.rho12 * frcp(P.drho * c + P.rho1); }
__device__ __forceinline__ double visc_of(const Phys &P, double c) { return P.visc12 * frcp(P.dvisc * c + P.visc1); }
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
// LDS tile

enum { T_C = 0, T_MU, T_P, T_U, T_V, T_CN, T_UN, T_VN, T_RN, T_MV, T_MOB, T_RS, T_NF };

// A tile covers level cells i0-1 .. i0+TX+1, j0-1 .. j0+TY+1 (W = TX+3
// columns); q(f, i, j) takes level coordinates.
template <typename R> struct TileT {
    R *s; // field arrays of W*H elements in LDS
    int i0, j0, W, H;
    __device__ __forceinline__ int idx(int i, int j) const { return (j - j0 + 1) * W + (i - i0 + 1); }
    __device__ __forceinline__ R q(int f, int i, int j) const { return s[f * W * H + idx(i, j)]; }
    __device__ __forceinline__ void set(int f, int i, int j, R v) const { s[f * W * H + idx(i, j)] = v; }
};
typedef TileT<double> Tile;

// cooperative load of a tile (all threads of the block take part; the caller
// synchronises afterwards).  The level may be in global memory or in LDS.
// true if every element of the tile (halo included) is an interior element
// of the level for every field, so that no boundary image is involved: cells
// and faces 1 .. m-1 in each direction
__device__ __forceinline__ bool tile_inner(int m1, int m2, int i0, int j0, int W, int H)
{
    return i0 >= 2 && j0 >= 2 && i0 + W - 2 <= m1 - 1 && j0 + H - 2 <= m2 - 1;
}

__device__ __forceinline__ void tile_load(const Phys &P, const View &L, const Tile &T)
{
    const int n = T.W * T.H;
    if (tile_inner(L.m1, L.m2, T.i0, T.j0, T.W, T.H) && n <= 2 * (int)block_threads()) {
        // no boundary images: plain strided loads, the two elements of a
        // thread loaded together (the second one clamped to a valid element
        // and stored only if it exists) so that all loads are in flight at once
        const int e0 = threadIdx.x, e1r = threadIdx.x + block_threads(), e1 = e1r < n ? e1r : n - 1;
        auto at = [&](int e) {
            const int b = e / T.W, a = e - b * T.W;
            return (size_t)(T.j0 - 1 + b) * L.pitch + (T.i0 - 1 + a);
        };
        const size_t q0 = at(e0 < n ? e0 : n - 1), q1 = at(e1);
        double v0[8], v1[8];
        const double *src[8] = { L.c, L.mu, L.p, L.u, L.v, L.cn, L.un, L.vn };
#pragma unroll
        for (int f = 0; f < 8; f++) {
            v0[f] = src[f][q0];
            v1[f] = src[f][q1];
        }
        auto put = [&](int e, const double *v) {
            double *s = T.s + e;
            s[T_C * n] = v[0];
            s[T_MU * n] = v[1];
            s[T_P * n] = v[2];
            s[T_U * n] = v[3];
            s[T_V * n] = v[4];
            s[T_CN * n] = v[5];
            s[T_UN * n] = v[6];
            s[T_VN * n] = v[7];
            s[T_RN * n] = rho_of(P, v[5]);
            s[T_MV * n] = visc_of(P, v[5]);
            s[T_MOB * n] = mob_of(P, v[5]);
            s[T_RS * n] = rho_of(P, v[0]);
        };
        if (e0 < n) put(e0, v0);
        if (e1r < n) put(e1r, v1);
        return;
    }
    if (n <= 2 * (int)block_threads()) {
        // boundary images: the sources of both elements of the thread first,
        // then all sixteen loads together, then the signs and cell functions
        const int e0 = threadIdx.x, e1 = threadIdx.x + block_threads();
        auto src = [&](int e) {
            const int b = e / T.W, a = e - b * T.W;
            TileSrc q = tile_src(L.m1, L.m2, L.pitch, L.bcx, L.bcy, T.i0 - 1 + a, T.j0 - 1 + b);
            if (e >= n) q.sc = q.su = q.sv = 0;
            return q;
        };
        const TileSrc s0 = src(e0 < n ? e0 : 0), s1 = src(e1 < n ? e1 : 0);
        const double v0[8] = { L.c[s0.c], L.mu[s0.c], L.p[s0.c], L.u[s0.u], L.v[s0.v], L.cn[s0.c], L.un[s0.u], L.vn[s0.v] };
        const double v1[8] = { L.c[s1.c], L.mu[s1.c], L.p[s1.c], L.u[s1.u], L.v[s1.v], L.cn[s1.c], L.un[s1.u], L.vn[s1.v] };
        auto put = [&](int e, const TileSrc &q, const double *v) {
            double *s = T.s + e;
            if (q.sc == 0) {
                for (int f = 0; f < T_NF; f++) s[f * n] = 0.0;
                return;
            }
            s[T_C * n] = v[0];
            s[T_MU * n] = v[1];
            s[T_P * n] = v[2];
            s[T_U * n] = signed_val(q.su, v[3]);
            s[T_V * n] = signed_val(q.sv, v[4]);
            s[T_CN * n] = v[5];
            s[T_UN * n] = signed_val(q.su, v[6]);
            s[T_VN * n] = signed_val(q.sv, v[7]);
            s[T_RN * n] = rho_of(P, v[5]);
            s[T_MV * n] = visc_of(P, v[5]);
            s[T_MOB * n] = mob_of(P, v[5]);
            s[T_RS * n] = rho_of(P, v[0]);
        };
        if (e0 < n) put(e0, s0, v0);
        if (e1 < n) put(e1, s1, v1);
        return;
    }
    for (int e = threadIdx.x; e < n; e += block_threads()) {
        const int b = e / T.W, a = e - b * T.W;
        const int i = T.i0 - 1 + a, j = T.j0 - 1 + b;
        double *s = T.s + e;
        const int st = n;
        if (i > L.m1 + 1 || j > L.m2 + 1) {
            // beyond the reach of any cell of the level (tile larger than the level)
            for (int f = 0; f < T_NF; f++) s[f * st] = 0.0;
            continue;
        }
        const double c = ldc(L.c, L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j);
        const double cn = ldc(L.cn, L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j);
        s[T_C * st] = c;
        s[T_MU * st] = ldc(L.mu, L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j);
        s[T_P * st] = ldc(L.p, L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j);
        s[T_U * st] = ldu(L.u, L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j);
        s[T_V * st] = ldv(L.v, L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j);
        s[T_CN * st] = cn;
        s[T_UN * st] = ldu(L.un, L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j);
        s[T_VN * st] = ldv(L.vn, L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j);
        s[T_RN * st] = rho_of(P, cn);
        s[T_MV * st] = visc_of(P, cn);
        s[T_MOB * st] = mob_of(P, cn);
        s[T_RS * st] = rho_of(P, c);
    }
}

// A level resident in LDS is refreshed into its tile after every half-sweep.
// Where each element comes from is fixed, so it is computed once (4 ints per
// element: the cell, u and v source indices as tile_src gives them, and a
// word with the u and v signs, a beyond-reach flag (such elements keep their
// loaded values) and the colour of the source cell).
template <typename V, typename TT> __device__ __forceinline__ void tile_map_build(const V &L, const TT &T, int *map)
{
    const int n = T.W * T.H;
    for (int e = threadIdx.x; e < n; e += block_threads()) {
        const int b = e / T.W, a = e - b * T.W;
        const int i = T.i0 - 1 + a, j = T.j0 - 1 + b;
        const TileSrc q = tile_src(L.m1, L.m2, L.pitch, L.bcx, L.bcy, i, j);
        const int ic = q.c % L.pitch, jc = q.c / L.pitch;
        int fl = (q.su + 1) | ((q.sv + 1) << 2) | (((ic + jc) & 1) << 5);
        if (i > L.m1 + 1 || j > L.m2 + 1) fl |= 16;
        map[4 * e] = q.c;
        map[4 * e + 1] = q.u;
        map[4 * e + 2] = q.v;
        map[4 * e + 3] = fl;
    }
}
// the refresh after a half-sweep of the given colour: all face velocities
// (the new buffer), and c, mubar, pbar, rho(c) of the elements whose source
// cell has that colour (the others did not change), with the boundary images
// of ldc, ldu, ldv
__device__ __forceinline__ void tile_refresh_map(const Phys &P, const View &L, const Tile &T, const int *map,
                                                 int colour)
{
    const int n = T.W * T.H;
    for (int e = threadIdx.x; e < n; e += block_threads()) {
        // the map entry, then every value the element may take (the indices
        // are valid in any case), before any use: two round trips to LDS
        // instead of one per dependent step
        const int q = map[4 * e], qu = map[4 * e + 1], qv = map[4 * e + 2], fl = map[4 * e + 3];
        const double u = L.u[qu], v = L.v[qv], c = L.c[q], mu = L.mu[q], p = L.p[q];
        __builtin_amdgcn_sched_barrier(0);
        if (fl & 16) continue;
        double *s = T.s + e;
        s[T_U * n] = signed_val((fl & 3) - 1, u);
        s[T_V * n] = signed_val(((fl >> 2) & 3) - 1, v);
        if (((fl >> 5) & 1) != colour) continue;
        s[T_C * n] = c;
        s[T_MU * n] = mu;
        s[T_P * n] = p;
        s[T_RS * n] = rho_of(P, c);
    }
}

// --------------------------------------------------------------------------
// Lane pairs.  Each cell (or box) is handled by two adjacent lanes: lane 0
// takes every x-direction contribution, lane 1 the same code on transposed
// strides (y-direction), so the pair runs one instruction stream without
// divergence.  Partial sums are exchanged with a one-lane shuffle.

struct Ax {
    int dn, dt;            // element strides of the tile along the normal / tangential axis
    int FN, FT, FNN, FTN;  // own velocity, other velocity and their time-n fields
    int per, ia, ma;       // periodic along the axis; cell index and count along it
    int pert, it, mt;      // the same for the tangential axis
    double grav;           // 1 on the y lane: gravity acts on the north-south faces
    int hlf;
};

template <typename V, typename TT>
__device__ __forceinline__ Ax make_ax(const V &L, const TT &T, int i, int j, int hlf)
{
    Ax a;
    a.hlf = hlf;
    a.dn = hlf ? T.W : 1;
    a.dt = hlf ? 1 : T.W;
    a.FN = hlf ? T_V : T_U;
    a.FT = hlf ? T_U : T_V;
    a.FNN = hlf ? T_VN : T_UN;
    a.FTN = hlf ? T_UN : T_VN;
    a.per = hlf ? L.bcy : L.bcx;
    a.ia = hlf ? j : i;
    a.ma = hlf ? L.m2 : L.m1;
    a.pert = hlf ? L.bcx : L.bcy;
    a.it = hlf ? i : j;
    a.mt = hlf ? L.m1 : L.m2;
    a.grav = hlf ? 1.0 : 0.0;
    return a;
}

// value of the partner lane (lane ^ 1): a DPP quad permutation [1,0,3,2]
// within the wave's registers, no LDS round trip
__device__ __forceinline__ int other(int x) { return __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false); }
__device__ __forceinline__ float other(float x) { return __int_as_float(other(__float_as_int(x))); }
__device__ __forceinline__ double other(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = other((int)(b & 0xffffffffll)), hi = other((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// element-indexed tile read
template <typename R> __device__ __forceinline__ R tq(const TileT<R> &T, int f, int e) { return T.s[f * T.W * T.H + e]; }

// contributions of one axis to the cell equations at cell element e
struct CellAx {
    double adv, div, Lmu, Lp, Sm, Gc, Gn, Lr, dGc, dLra, dLrb;
};

__device__ __forceinline__ CellAx cell_axis(const Tile &T, const Ax &a, int e, double ih)
{
    const double ih2 = ih * ih;
    // faces of the cell on a wall carry no flux (the mirrored ghost equals the
    // cell); the masks matter for derivatives only
    const double wP = (a.per || a.ia < a.ma - 1) ? 1.0 : 0.0, wM = (a.per || a.ia > 0) ? 1.0 : 0.0;
    const int eP = e + a.dn, eM = e - a.dn;
    const double c = tq(T, T_C, e), cP = tq(T, T_C, eP), cM = tq(T, T_C, eM);
    const double n = tq(T, T_CN, e), nP = tq(T, T_CN, eP), nM = tq(T, T_CN, eM);
    const double mu = tq(T, T_MU, e), p = tq(T, T_P, e);
    const double rnP = tq(T, T_RN, eP), rnM = tq(T, T_RN, eM), rn = tq(T, T_RN, e);
    const double rs = tq(T, T_RS, e);
    const double m0 = tq(T, T_MOB, e);
    const double mP = 0.5 * (tq(T, T_MOB, eP) + m0) * wP, mM = 0.5 * (tq(T, T_MOB, eM) + m0) * wM;
    const double uP = tq(T, a.FN, eP), u0 = tq(T, a.FN, e);
    CellAx x;
    // rho^n u . grad c^n in the special form of App. A.5
    x.adv = 0.5 * ih * (rnP * (nP - n) * uP + rnM * (n - nM) * u0);
    x.div = ih * (uP - u0);
    x.Lmu = ih2 * (mP * (tq(T, T_MU, eP) - mu) - mM * (mu - tq(T, T_MU, eM)));
    x.Lp = ih2 * (mP * (tq(T, T_P, eP) - p) - mM * (p - tq(T, T_P, eM)));
    x.Sm = ih2 * (mP + mM);
    const double dP = cP - c, dM = c - cM, gP = nP - n, gM = n - nM;
    x.Gc = 0.5 * ih2 * (dP * dP + dM * dM);
    x.Gn = 0.5 * ih2 * (gP * gP + gM * gM);
    const double rh = 0.5 * (rs + rn);
    const double kP = 0.5 * (0.5 * (tq(T, T_RS, eP) + rnP) + rh) * wP;
    const double kM = 0.5 * (0.5 * (tq(T, T_RS, eM) + rnM) + rh) * wM;
    const double hP = 0.5 * (dP + gP), hM = 0.5 * (dM + gM);
    x.Lr = ih2 * (kP * hP - kM * hM);
    x.dGc = ih2 * (wP * (-dP) + wM * dM);
    x.dLra = ih2 * (wP * hP - wM * hM);
    x.dLrb = ih2 * (kP + kM);
    return x;
}

__device__ __forceinline__ CellAx cell_sum(const CellAx &x)
{
    CellAx s;
    s.adv = x.adv + other(x.adv);
    s.div = x.div + other(x.div);
    s.Lmu = x.Lmu + other(x.Lmu);
    s.Lp = x.Lp + other(x.Lp);
    s.Sm = x.Sm + other(x.Sm);
    s.Gc = x.Gc + other(x.Gc);
    s.Gn = x.Gn + other(x.Gn);
    s.Lr = x.Lr + other(x.Lr);
    s.dGc = x.dGc + other(x.dGc);
    s.dLra = x.dLra + other(x.dLra);
    s.dLrb = x.dLrb + other(x.dLrb);
    return s;
}

// cell equations: phase (pm-num-phase), chemical potential (pm-num-chem) and
// mass (pm-num-mass), with the Jacobian entries the smoother needs, from the
// two axis sums
struct CellEq {
    double Nc, Nmu, Np;
    double Jcc, Jcm, Jmc, Jmm; // d(Nc,Nmu)/d(c,mu) at the cell
    double Jpp;                // dNp/dp at the cell
};

__device__ __forceinline__ CellEq cell_eq(const Phys &P, const Tile &T, int e, const CellAx &s)
{
    const double c = tq(T, T_C, e), n = tq(T, T_CN, e), mu = tq(T, T_MU, e);
    const double rs = tq(T, T_RS, e), rn = tq(T, T_RN, e);
    CellEq q;
    q.Nc = rs * (c - n) * P.inv_dt + s.adv - P.inv_Pe * s.Lmu - P.alpha * P.inv_Pe * s.Lp;
    q.Np = s.div - P.alpha * P.inv_Pe * s.Lmu - P.alpha * P.alpha * P.inv_Pe * s.Lp;
    // time averages of sec. 4.1; pointwise |grad_D c|^2 = a_x((D_x c)^2) + a_y((D_y c)^2)
    const double rh = 0.5 * (rs + rn);
    const double q1 = c * (c - 1.0), q0 = n * (n - 1.0);
    const double g = 0.25 * (q1 + q0) * (c + n - 1.0);
    const double Fh = 0.5 * (dwell(c) + dwell(n));
    const double r = -P.alpha * rs * rn;
    const double Gh = 0.5 * (s.Gc + s.Gn);
    q.Nmu = rs * mu - P.K1 * (rh * g + Fh * r) - P.K2 * Gh * r + P.K3 * s.Lr;
    // Jacobian in (c_ij, mubar_ij); rho' = -alpha rho^2
    const double drs = -P.alpha * rs * rs;
    q.Jcc = (drs * (c - n) + rs) * P.inv_dt;
    q.Jcm = P.inv_Pe * s.Sm;
    q.Jmm = rs;
    const double dg = 0.25 * ((2.0 * c - 1.0) * (c + n - 1.0) + q1 + q0);
    const double f1 = q1 * (c - 0.5);                   // F'(c)
    const double dr = P.alpha * P.alpha * rs * rs * rn; // dr/dc
    const double dLr = 0.25 * drs * s.dLra - 0.5 * s.dLrb;
    q.Jmc = drs * mu - P.K1 * (0.5 * drs * g + rh * dg + 0.5 * f1 * r + Fh * dr) - P.K2 * (0.5 * s.dGc * r + Gh * dr)
          + P.K3 * dLr;
    q.Jpp = P.alpha * P.alpha * P.inv_Pe * s.Sm;
    return q;
}

// --------------------------------------------------------------------------
// momentum equation (pm-num-mx) on the face stored at element ef (the west
// face of its cell on the x lane, the south face on the y lane), with the
// derivative with respect to the face's own velocity.  Advection (e1e1-1) plus
// the half-divergence term (e1e1-2) are used in their skew form
//   1/(2h) [w_R u_{+1} - w_L u_{-1} + Z_t u_{t+1} - Z_b u_{t-1}],
// which is the same sum with the terms on the face's own value cancelled.
// (it = tangential index of the face's row.)
struct FaceEq {
    double N, diag;
};

__device__ __forceinline__ FaceEq face_eq(const Phys &P, const Tile &T, const Ax &a, int ef, int it, double ih,
                                          bool proj = false)
{
    const double ih2 = ih * ih;
    const int eL = ef - a.dn, eR = ef, dt = a.dt;
    const double rL = tq(T, T_RN, eL), rR = tq(T, T_RN, eR);
    const double Rt = 0.25 * (rL + rR + tq(T, T_RN, eL + dt) + tq(T, T_RN, eR + dt));
    const double Rb = 0.25 * (rL + rR + tq(T, T_RN, eL - dt) + tq(T, T_RN, eR - dt));
    const double mvL = tq(T, T_MV, eL), mvR = tq(T, T_MV, eR);
    const double nut = 0.25 * (mvL + mvR + tq(T, T_MV, eL + dt) + tq(T, T_MV, eR + dt));
    const double nub = 0.25 * (mvL + mvR + tq(T, T_MV, eL - dt) + tq(T, T_MV, eR - dt));
    const double Arn = 0.5 * (rL + rR);
    const double Ars = 0.5 * (tq(T, T_RS, eL) + tq(T, T_RS, eR));
    const double un0 = tq(T, a.FNN, ef);
    const double wL = rL * 0.5 * (tq(T, a.FNN, ef - a.dn) + un0);
    const double wR = rR * 0.5 * (un0 + tq(T, a.FNN, ef + a.dn));
    const double Vt = 0.5 * (tq(T, a.FTN, eL + dt) + tq(T, a.FTN, eR + dt));
    const double Vb = 0.5 * (tq(T, a.FTN, eL) + tq(T, a.FTN, eR));
    const double u0 = tq(T, a.FN, ef), uE = tq(T, a.FN, ef + a.dn), uW = tq(T, a.FN, ef - a.dn);
    const double uN = tq(T, a.FN, ef + dt), uS = tq(T, a.FN, ef - dt);
    const double thR = ih * (uE - u0 + tq(T, a.FT, eR + dt) - tq(T, a.FT, eR));
    const double thL = ih * (u0 - uW + tq(T, a.FT, eL + dt) - tq(T, a.FT, eL));
    const double nL = tq(T, T_CN, eL), nR = tq(T, T_CN, eR);
    FaceEq q;
    q.N = Arn * (u0 - un0) * P.inv_dt
        + 0.5 * ih * (wR * uE - wL * uW + Rt * Vt * uN - Rb * Vb * uS)
        + 0.5 * (Ars - Arn) * P.inv_dt * u0
        - P.inv_Re * ih2 * (mvR * (uE - u0) - mvL * (u0 - uW) + nut * (uN - u0) - nub * (u0 - uS))
        - (P.inv_Re / 3.0) * ih * (mvR * thR - mvL * thL);
    // the projection scheme's intermediate velocity (pj-num-mx) has neither
    // pressure, surface tension nor gravity: they act in (pj-num-pjx)
    if (!proj)
        q.N += P.inv_M * ih * (tq(T, T_P, eR) - tq(T, T_P, eL))
             - P.inv_M * ih * 0.5 * (rR * tq(T, T_MU, eL) + rL * tq(T, T_MU, eR)) * (nR - nL)
             + a.grav * P.inv_Fr * (Arn - P.rho_ref);
    // own-face derivative; across a tangential wall the reflected ghost doubles
    // the viscous coupling and the advection coefficient enters with a sign flip
    const double gt = (!a.pert && it == a.mt - 1) ? 1.0 : 0.0, gb = (!a.pert && it == 0) ? 1.0 : 0.0;
    q.diag = 0.5 * (Arn + Ars) * P.inv_dt + (4.0 / 3.0) * P.inv_Re * ih2 * (mvL + mvR)
           + P.inv_Re * ih2 * (nut * (1.0 + gt) + nub * (1.0 + gb)) + 0.5 * ih * (gb * Rb * Vb - gt * Rt * Vt);
    return q;
}

// loads and stores through a pointer of address space AS (1: global memory,
// 3: LDS, 0: either).  A level's arrays reach the kernels inside structures,
// so without it the compiler issues generic accesses, which count as LDS
// accesses too: every wait for an LDS read would then also wait for the
// outstanding global loads.
template <int AS, typename R> __device__ __forceinline__ R lda(const R *p, size_t k)
{
    if constexpr (AS == 1)
        return ((const __attribute__((address_space(1))) R *)p)[k];
    else if constexpr (AS == 3)
        return ((const __attribute__((address_space(3))) R *)p)[k];
    else
        return p[k];
}
template <int AS, typename R> __device__ __forceinline__ void sta(R *p, size_t k, R v)
{
    if constexpr (AS == 1)
        ((__attribute__((address_space(1))) R *)p)[k] = v;
    else if constexpr (AS == 3)
        ((__attribute__((address_space(3))) R *)p)[k] = v;
    else
        p[k] = v;
}

template <int AS = 0> __device__ __forceinline__ double ldf(const double *f, const View &L, int i, int j)
{
    return f ? lda<AS>(f, (size_t)j * L.pitch + i) : 0.0;
}

// face right-hand side of the lane's axis: the select is taken on the pointer
// values (a select between the two struct members made the compiler stage
// them in scratch memory)
__device__ __forceinline__ const double *face_rhs(const Rhs &F, int hlf)
{
    const uintptr_t a = (uintptr_t)F.fu, b = (uintptr_t)F.fv;
    return (const double *)(hlf ? b : a);
}

// --------------------------------------------------------------------------
// smoother for one cell of the current colour (sec. 7.1), run by a lane pair.
// Segregated (P.coupled = 0): step 1 is Newton on (N_c, N_mu) in (c_ij,
// mubar_ij); step 2 the Vanka box on (uW, uE, vS, vN, p).  Coupled: one Newton
// step on all seven unknowns of the cell with the box equations plus N_c and
// N_mu of the cell.  Its matrix is the 5x5 box matrix bordered by
//   face rows:  dN_f/dc = rho'(c) u_f / (4 dt),  dN_f/dmubar = -a_f / M,
//   mass row:   dN_p/dmubar = alpha Sm / Pe,
//   phase row:  dN_c/du_f = a_f (the advection weights of App. A.5),
//               dN_c/dp = alpha Sm / Pe, Jcc, Jcm,
//   chem. row:  Jmc, Jmm,
// with a_f = rho^n (c^n jump across the face) / (2h), signed along the axis.
// mubar and c are eliminated first (N_mu, then N_c; the pivots are Jmm = rho
// and Jcc - Jcm Jmc / Jmm, which exceeds Jcc where the gradient-energy term
// makes Jmc negative, as on any grid that resolves the interface), which
// leaves a rank-one update of the 5x5 box matrix; after its solve, c and mubar
// follow by back substitution.
// Velocities come from the tile (the snapshot of this colour); the box faces
// go to unew/vnew, c, mubar, pbar to the level arrays.  In the segregated
// form c, mubar and rho(c) of the cell are also written to the tile between
// the steps (identical values from both lanes), which no other pair of this
// colour reads.
template <bool TO, int AS>
__device__ __forceinline__ void relax_pair_pj(const Phys &P, const View &L, const Tile &T, const Rhs &F, double *unew, double *vnew,
                              int i, int j, int ti, int tj, int hlf, double omega, double pomega);
__device__ __forceinline__ void resid_pair_pj(const Phys &P, const View &L, const Tile &T, const Rhs &F, int i, int j, int hlf,
                              double &rc, double &rm, double &rp, double &rf);

// omega relaxes the box's velocity and pressure updates; pomega the
// projection scheme's separate pressure step
// With TO set (primitive scheme only), the cell sits at tile position (ti,
// tj), which differs from its level position (i, j) at a periodic image, and
// the results stay in the tile: c, mubar, pbar and rho(c) in place (no other
// cell of the colour reads them), the box faces in the fields T_NF (u) and
// T_NF + 1 (v), whose elements only this cell's box writes.  AS is the
// address space of the level arrays and right-hand sides (1: global memory,
// 3: LDS, where the level resides in the workgroup's LDS).
template <bool TO, int AS>
__device__ __forceinline__ void relax_cell(const Phys &P, const View &L, const Tile &T, const Rhs &F, double *unew,
                                           double *vnew, int i, int j, int ti, int tj, int hlf, double omega,
                                           double pomega)
{
    if (P.scheme) {
        relax_pair_pj<TO, AS>(P, L, T, F, unew, vnew, i, j, ti, tj, hlf, omega, pomega);
        return;
    }
    const size_t k = (size_t)j * L.pitch + i;
    const double ih = L.inv_h, ih2 = ih * ih;
    const int e = T.idx(ti, tj);
    const Ax a = make_ax(L, T, i, j, hlf);
    const bool cpl = P.coupled;
    // the right-hand sides first: their loads are then in flight during the
    // cell equations
    const bool hlo = a.per || a.ia >= 1, hhi = a.per || a.ia + 1 < a.ma;
    const double *fN = face_rhs(F, hlf);
    const int ihi = hlf ? i : (i + 1 < L.m1 ? i + 1 : 0), jhi = hlf ? (j + 1 < L.m2 ? j + 1 : 0) : j;
    const size_t khi = (size_t)jhi * L.pitch + ihi;
    const double f_c = ldf<AS>(F.fc, L, i, j), f_mu = ldf<AS>(F.fmu, L, i, j), f_p = ldf<AS>(F.fp, L, i, j);
    const double f_lo = hlo ? ldf<AS>(fN, L, i, j) : 0.0, f_hi = hhi ? ldf<AS>(fN, L, ihi, jhi) : 0.0;
    CellAx x = cell_axis(T, a, e, ih);
    CellAx s = cell_sum(x);
    CellEq q = cell_eq(P, T, e, s);
    const double r1 = f_c - q.Nc, r2 = f_mu - q.Nmu;
    const double c0 = tq(T, T_C, e), m0 = tq(T, T_MU, e);
    double cnew = c0, mnew = m0;
    // coupled box: mubar eliminated by N_mu (pivot Jmm), then c by N_c (pivot
    // 1/icc); what the box needs of the cell rows afterwards
    double imm = 0.0, kmc = 0.0, kbm = 0.0, icc = 0.0, bc = 0.0, Jcp = 0.0, gc = 0.0;
    if (cpl) {
        imm = frcp(q.Jmm);
        kmc = q.Jmc * imm;
        kbm = r2 * imm;
        icc = frcp(q.Jcc - q.Jcm * kmc);
        bc = r1 - q.Jcm * kbm;
        Jcp = P.alpha * P.inv_Pe * s.Sm; // dN_c/dpbar = dN_p/dmubar
        const double rs = tq(T, T_RS, e);
        gc = 0.25 * (-P.alpha * rs * rs) * P.inv_dt; // dN_f/dc per unit u_f
    }
    if (!cpl) {
        // ---- step 1
        const double idet = frcp(q.Jcc * q.Jmm - q.Jcm * q.Jmc);
        cnew = c0 + (q.Jmm * r1 - q.Jcm * r2) * idet;
        mnew = m0 + (q.Jcc * r2 - q.Jmc * r1) * idet;
        if (!TO && hlf == 0) {
            sta<AS>(L.c, k, cnew);
            sta<AS>(L.mu, k, mnew);
        }
        T.s[T_C * T.W * T.H + e] = cnew;
        T.s[T_MU * T.W * T.H + e] = mnew;
        T.s[T_RS * T.W * T.H + e] = rho_of(P, cnew);
    }
    // ---- the box: this lane's two faces along its axis
    const FaceEq flo = face_eq(P, T, a, e, a.it, ih);
    const FaceEq fhi = face_eq(P, T, a, e + a.dn, a.it, ih);
    const double blo = hlo ? f_lo - flo.N : 0.0, dlo = hlo ? flo.diag : 1.0;
    const double bhi = hhi ? f_hi - fhi.N : 0.0, dhi = hhi ? fhi.diag : 1.0;
    // mass equation with the new mubar of the cell (linear in it: -Sm per axis)
    const double Lmu_new = s.Lmu - s.Sm * (mnew - m0);
    const double bp = f_p - (s.div - P.alpha * P.inv_Pe * Lmu_new - P.alpha * P.alpha * P.inv_Pe * s.Lp);
    // box-cell coefficients of the off-diagonal couplings
    const double w_ax = tq(T, T_RN, e) * 0.5 * (tq(T, a.FNN, e) + tq(T, a.FNN, e + a.dn)); // rho^n a u^n
    const double mv0 = tq(T, T_MV, e);
    const double vis = (4.0 / 3.0) * P.inv_Re * ih2 * mv0, gd = P.inv_Re * ih2 * mv0 / 3.0;
    const double gp = P.inv_M * ih;
    // periodic axis of two cells: the next face beyond each box face is the
    // box's other face, which so enters each face row a second time (through
    // the other cell's advection weight and viscosity)
    double xlo = 0.0, xhi = 0.0;
    if (a.per && a.ma == 2) {
        const double w_o = tq(T, T_RN, e - a.dn) * 0.5 * (tq(T, a.FNN, e) + tq(T, a.FNN, e + a.dn));
        const double v_o = (4.0 / 3.0) * P.inv_Re * ih2 * tq(T, T_MV, e - a.dn);
        xlo = -0.5 * ih * w_o - v_o;
        xhi = 0.5 * ih * w_o - v_o;
    }
    // exchange: each lane of the pair now holds the rows of both axes.  A
    // lane orders the box's unknowns with its own axis first: lane 0 as uW,
    // uE, vS, vN, p, lane 1 as vS, vN, uW, uE, p; the rows of the two axes
    // have the same form, so the matrix is assembled without selecting by
    // lane, and each lane eliminates its own faces first (lane 0 in the
    // order of the oracle, lane 1 with the axes swapped, a symmetric
    // permutation that keeps the pivots positive)
    const double o_blo = other(blo), o_dlo = other(dlo), o_bhi = other(bhi), o_dhi = other(dhi), o_w = other(w_ax);
    const double o_xlo = other(xlo), o_xhi = other(xhi);
    const int o_hlo = other((int)hlo), o_hhi = other((int)hhi);
    double A[5][5], b[5];
    b[0] = blo; b[1] = bhi; b[2] = o_blo; b[3] = o_bhi; b[4] = bp;
    // rows: momentum at the own axis' low and high faces, the other axis' low
    // and high faces, then mass; columns in the same order; a face on a wall
    // is not an unknown (identity row, no coupling)
    const double m0l = hlo ? 1.0 : 0.0, m0h = hhi ? 1.0 : 0.0, m1l = o_hlo ? 1.0 : 0.0, m1h = o_hhi ? 1.0 : 0.0;
    A[0][0] = dlo; A[0][1] = m0l * (0.5 * ih * w_ax - vis) + xlo; A[0][2] = m0l * gd; A[0][3] = -m0l * gd; A[0][4] = m0l * gp;
    A[1][1] = dhi; A[1][0] = m0h * (-0.5 * ih * w_ax - vis) + xhi; A[1][2] = -m0h * gd; A[1][3] = m0h * gd; A[1][4] = -m0h * gp;
    A[2][2] = o_dlo; A[2][3] = m1l * (0.5 * ih * o_w - vis) + o_xlo; A[2][0] = m1l * gd; A[2][1] = -m1l * gd; A[2][4] = m1l * gp;
    A[3][3] = o_dhi; A[3][2] = m1h * (-0.5 * ih * o_w - vis) + o_xhi; A[3][0] = -m1h * gd; A[3][1] = m1h * gd; A[3][4] = -m1h * gp;
    A[4][0] = -m0l * ih; A[4][1] = m0h * ih; A[4][2] = -m1l * ih; A[4][3] = m1h * ih; A[4][4] = q.Jpp;
    // coupled box: border of the c and mubar rows and columns, eliminated
    // into the 5x5 system (see above)
    double ac[5] = { 0.0, 0.0, 0.0, 0.0, 0.0 };
    if (cpl) {
        const int e1 = e + a.dn;
        const double alo = hlo ? 0.5 * ih * tq(T, T_RN, e - a.dn) * (tq(T, T_CN, e) - tq(T, T_CN, e - a.dn)) : 0.0;
        const double ahi = hhi ? 0.5 * ih * tq(T, T_RN, e1) * (tq(T, T_CN, e1) - tq(T, T_CN, e)) : 0.0;
        const double ulo = hlo ? tq(T, a.FN, e) : 0.0, uhi = hhi ? tq(T, a.FN, e1) : 0.0;
        ac[0] = alo; ac[1] = ahi; ac[2] = other(alo); ac[3] = other(ahi);
        const double uf[4] = { ulo, uhi, other(ulo), other(uhi) };
        ac[4] = Jcp;
        double gam[5];
#pragma unroll
        for (int f = 0; f < 4; f++) {
            const double lam = -P.inv_M * ac[f];
            gam[f] = gc * uf[f] - lam * kmc;
            b[f] -= lam * kbm;
        }
        gam[4] = -Jcp * kmc;
        b[4] -= Jcp * kbm;
#pragma unroll
        for (int r = 0; r < 5; r++) {
            const double t = gam[r] * icc;
#pragma unroll
            for (int cc = 0; cc < 5; cc++) A[r][cc] -= t * ac[cc];
            b[r] -= t * bc;
        }
    }
    // Gaussian elimination in the lane's order (own faces, other faces, p):
    // the velocity block has a positive definite symmetric part (mass +
    // viscous; advection is skew) and the last pivot is the positive pressure
    // Schur complement
    double inv[5];
#pragma unroll
    for (int c = 0; c < 4; c++) {
        inv[c] = frcp(A[c][c]);
#pragma unroll
        for (int r = c + 1; r < 5; r++) {
            const double l = A[r][c] * inv[c];
#pragma unroll
            for (int t = c + 1; t < 5; t++) A[r][t] -= l * A[c][t];
            b[r] -= l * b[c];
        }
    }
    inv[4] = frcp(A[4][4]);
#pragma unroll
    for (int c = 4; c >= 0; c--) {
        double acc = b[c];
#pragma unroll
        for (int t = c + 1; t < 5; t++) acc -= A[c][t] * b[t];
        b[c] = acc * inv[c];
    }
    if (cpl && hlf == 0) {
        double acc = bc;
#pragma unroll
        for (int t = 0; t < 5; t++) acc -= ac[t] * b[t];
        const double dc = acc * icc;
        if (TO) {
            const int n = T.W * T.H;
            T.s[T_C * n + e] = c0 + dc;
            T.s[T_MU * n + e] = m0 + kbm - kmc * dc;
            T.s[T_RS * n + e] = rho_of(P, c0 + dc);
        } else {
            sta<AS>(L.c, k, c0 + dc);
            sta<AS>(L.mu, k, m0 + kbm - kmc * dc);
        }
    }
    const double nlo = tq(T, a.FN, e) + omega * b[0], nhi = tq(T, a.FN, e + a.dn) + omega * b[1];
    if (TO) {
        const int n = T.W * T.H;
        double *fo = T.s + (T_NF + hlf) * n;
        if (hlo) fo[e] = nlo;
        if (hhi) fo[e + a.dn] = nhi;
        if (hlf == 0) T.s[T_P * n + e] = tq(T, T_P, e) + omega * b[4];
        return;
    }
    if (hlf) {
        if (hlo) sta<AS>(vnew, k, nlo);
        if (hhi) sta<AS>(vnew, khi, nhi);
    } else {
        if (hlo) sta<AS>(unew, k, nlo);
        if (hhi) sta<AS>(unew, khi, nhi);
    }
    if (hlf == 0) sta<AS>(L.p, k, tq(T, T_P, e) + omega * b[4]);
}
template <int AS>
__device__ __forceinline__ void relax_pair(const Phys &P, const View &L, const Tile &T, const Rhs &F, double *unew,
                                           double *vnew, int i, int j, int hlf, double omega, double pomega)
{
    relax_cell<false, AS>(P, L, T, F, unew, vnew, i, j, i, j, hlf, omega, pomega);
}

// residuals r = f - N(w) of the five equations attached to cell (i,j): the
// cell equations and the momentum equation of its west face (lane 0) or south
// face (lane 1); zero for a face on a wall.  Both lanes return rc, rm, rp;
// rf is this lane's face residual.  The level and its right-hand sides are
// in global memory.
__device__ __forceinline__ void resid_pair(const Phys &P, const View &L, const Tile &T, const Rhs &F, int i, int j,
                                           int hlf, double &rc, double &rm, double &rp, double &rf)
{
    if (P.scheme) {
        resid_pair_pj(P, L, T, F, i, j, hlf, rc, rm, rp, rf);
        return;
    }
    const int e = T.idx(i, j);
    const Ax a = make_ax(L, T, i, j, hlf);
    const CellAx s = cell_sum(cell_axis(T, a, e, L.inv_h));
    const CellEq q = cell_eq(P, T, e, s);
    rc = ldf<1>(F.fc, L, i, j) - q.Nc;
    rm = ldf<1>(F.fmu, L, i, j) - q.Nmu;
    rp = ldf<1>(F.fp, L, i, j) - q.Np;
    const bool hlo = a.per || a.ia >= 1;
    const FaceEq f = face_eq(P, T, a, e, a.it, L.inv_h);
    rf = hlo ? ldf<1>(face_rhs(F, hlf), L, i, j) - f.N : 0.0;
}

// --------------------------------------------------------------------------
// Projection scheme (sec. 6.2).  The unknowns are c, mubar, pbar and the
// intermediate velocity u~, which the face fields (T_U, T_V) hold during a
// step.  The velocity of time n+1 is eliminated through the projection
// equation (pj-num-pjx): on the face at element ef of the lane's axis,
//   u = u~ + dt / A rho (A(rho_ew mubar) D c / M - D pbar / M - grav),
// rho = rho(c) and c, mubar of the iterate, grav = (1/Fr)(A_y rho - rho_ref)
// on north-south faces (gravity acts in the projection equation, as in the
// time-discrete scheme (pj-pj)); zero on a wall face.  ut is u~ on the face.
__device__ __forceinline__ double face_final(const Phys &P, const Tile &T, const Ax &a, int ef, double ih, bool unk,
                                             double ut)
{
    const int eL = ef - a.dn;
    const double rL = tq(T, T_RS, eL), rR = tq(T, T_RS, ef), Ar = 0.5 * (rL + rR);
    const double st = 0.5 * (rR * tq(T, T_MU, eL) + rL * tq(T, T_MU, ef)) * (tq(T, T_C, ef) - tq(T, T_C, eL)) * ih;
    const double f = P.inv_M * (st - (tq(T, T_P, ef) - tq(T, T_P, eL)) * ih) - a.grav * P.inv_Fr * (Ar - P.rho_ref);
    return unk ? ut + P.dt * frcp(Ar) * f : 0.0;
}

// axis parts of the projection cell equations from the velocity of time n+1
// on the lane's two faces (ulo, uhi): the advection of (pj-num-phase) in the
// form (e1e2) of App. A.5 at time n+1, its derivative in the cell's own c (the
// velocities held fixed), and the divergence of (pj-num-mass)
struct PjAx {
    double adv, dadv, div;
};
__device__ __forceinline__ PjAx pj_axis(const Tile &T, const Ax &a, int e, double ih, double ulo, double uhi)
{
    const int eP = e + a.dn, eM = e - a.dn;
    const double c = tq(T, T_C, e), rP = tq(T, T_RS, eP), rM = tq(T, T_RS, eM);
    PjAx x;
    x.adv = 0.5 * ih * (rP * (tq(T, T_C, eP) - c) * uhi + rM * (c - tq(T, T_C, eM)) * ulo);
    x.dadv = 0.5 * ih * (rM * ulo - rP * uhi);
    x.div = ih * (uhi - ulo);
    return x;
}

// Smoother of sec. 7.2 for one cell of the current colour, by a lane pair:
//  1. one Newton step on (N_c, N_mu) in (c, mubar) of the cell, the velocity
//     of time n+1 on its faces held at its value before the update; with the
//     coupled smoother (P.coupled, the default) pbar and the mass equation
//     join this step, the velocity of time n+1 following pbar in its column
//     only;
//  2. the Vanka box of the four intermediate-velocity faces on (pj-num-mx),
//     exact (linear in u~), Jacobi within the colour;
//  3. one Newton step in pbar on the mass equation (pj-num-mass) with the
//     velocity of time n+1 from the new u~, c, mubar (exact: linear in pbar);
//  4. the velocity of time n+1 is never stored, so nothing is left to update.
// (pj-num-phase) and (pj-num-chem) differ from the primitive equations in
// rho^n (c - c^n)/dt, the advection at time n+1 and rho^n mubar.  The tile
// entries of the cell (c, mubar, rho(c)) are updated after step 1; no other
// pair of this colour reads them.
template <bool TO, int AS>
__device__ __forceinline__ void relax_pair_pj(const Phys &P, const View &L, const Tile &T, const Rhs &F, double *unew, double *vnew,
                              int i, int j, int ti, int tj, int hlf, double omega, double pomega)
{
    const size_t k = (size_t)j * L.pitch + i;
    const double ih = L.inv_h, ih2 = ih * ih;
    const int e = T.idx(ti, tj);
    const Ax a = make_ax(L, T, i, j, hlf);
    const bool hlo = a.per || a.ia >= 1, hhi = a.per || a.ia + 1 < a.ma;
    const int st = T.W * T.H;
    // ---- step 1
    const double ulo0 = face_final(P, T, a, e, ih, hlo, tq(T, a.FN, e));
    const double uhi0 = face_final(P, T, a, e + a.dn, ih, hhi, tq(T, a.FN, e + a.dn));
    const PjAx x0 = pj_axis(T, a, e, ih, ulo0, uhi0);
    const CellAx s = cell_sum(cell_axis(T, a, e, ih));
    const CellEq q = cell_eq(P, T, e, s);
    const double adv = x0.adv + other(x0.adv), dadv = x0.dadv + other(x0.dadv);
    const double c0 = tq(T, T_C, e), m0 = tq(T, T_MU, e), n0 = tq(T, T_CN, e);
    const double rs = tq(T, T_RS, e), rn = tq(T, T_RN, e), drs = -P.alpha * rs * rs;
    const double Nc = rn * (c0 - n0) * P.inv_dt + adv - P.inv_Pe * s.Lmu - P.alpha * P.inv_Pe * s.Lp;
    const double Nmu = q.Nmu - (rs - rn) * m0;
    const double Jcc = rn * P.inv_dt + dadv, Jcm = q.Jcm, Jmm = rn, Jmc = q.Jmc - drs * m0;
    const double r1 = ldf<AS>(F.fc, L, i, j) - Nc, r2 = ldf<AS>(F.fmu, L, i, j) - Nmu;
    const double p0 = tq(T, T_P, e);
    double cnew, mnew, pnew = p0;
    if (P.coupled) {
        // pbar joins the step with the mass equation: its column lets the
        // velocity of time n+1 follow pbar through (pj-num-pjx) (on the lo
        // face D pbar falls by pbar/h, on the hi face it rises), the c and
        // mubar columns hold it
        const double dlo = hlo ? -P.dt * P.inv_M * ih * frcp(0.5 * (tq(T, T_RS, e - a.dn) + rs)) : 0.0;
        const double dhi = hhi ? P.dt * P.inv_M * ih * frcp(0.5 * (rs + tq(T, T_RS, e + a.dn))) : 0.0;
        const double cl = 0.5 * ih * (tq(T, T_RS, e - a.dn) * (c0 - tq(T, T_C, e - a.dn)) * dlo
                                      + tq(T, T_RS, e + a.dn) * (tq(T, T_C, e + a.dn) - c0) * dhi);
        const double jx = ih * (dhi - dlo), dv = x0.div;
        const double Jcp = cl + other(cl) + P.alpha * P.inv_Pe * s.Sm, Jpm = P.alpha * P.inv_Pe * s.Sm;
        const double Jpp = jx + other(jx) + q.Jpp;
        const double Np = dv + other(dv) - P.alpha * P.inv_Pe * s.Lmu - P.alpha * P.alpha * P.inv_Pe * s.Lp;
        const double r3 = ldf<AS>(F.fp, L, i, j) - Np;
        // eliminate pbar by the mass row (pivot Jpp), then mubar by the
        // chemical row (pivot Jmm): a 2x2 system in c and mubar remains
        const double ipp = frcp(Jpp);
        const double kcm = Jcm - Jcp * Jpm * ipp, rc1 = r1 - Jcp * r3 * ipp;
        const double idet = frcp(Jcc * Jmm - kcm * Jmc);
        const double dc = (Jmm * rc1 - kcm * r2) * idet;
        const double dm = (Jcc * r2 - Jmc * rc1) * idet;
        cnew = c0 + dc;
        mnew = m0 + dm;
        pnew = p0 + (r3 - Jpm * dm) * ipp;
        T.s[T_P * st + e] = pnew;
    } else {
        const double idet = frcp(Jcc * Jmm - Jcm * Jmc);
        cnew = c0 + (Jmm * r1 - Jcm * r2) * idet;
        mnew = m0 + (Jcc * r2 - Jmc * r1) * idet;
    }
    if (!TO && hlf == 0) {
        sta<AS>(L.c, k, cnew);
        sta<AS>(L.mu, k, mnew);
    }
    T.s[T_C * st + e] = cnew;
    T.s[T_MU * st + e] = mnew;
    T.s[T_RS * st + e] = rho_of(P, cnew);
    // ---- step 2: the intermediate-velocity box
    const FaceEq flo = face_eq(P, T, a, e, a.it, ih, true);
    const FaceEq fhi = face_eq(P, T, a, e + a.dn, a.it, ih, true);
    const double *fN = face_rhs(F, hlf);
    const int ihi = hlf ? i : (i + 1 < L.m1 ? i + 1 : 0), jhi = hlf ? (j + 1 < L.m2 ? j + 1 : 0) : j;
    const size_t khi = (size_t)jhi * L.pitch + ihi;
    const double blo = hlo ? ldf<AS>(fN, L, i, j) - flo.N : 0.0, dlo = hlo ? flo.diag : 1.0;
    const double bhi = hhi ? ldf<AS>(fN, L, ihi, jhi) - fhi.N : 0.0, dhi = hhi ? fhi.diag : 1.0;
    const double w_ax = tq(T, T_RN, e) * 0.5 * (tq(T, a.FNN, e) + tq(T, a.FNN, e + a.dn));
    const double mv0 = tq(T, T_MV, e);
    const double vis = (4.0 / 3.0) * P.inv_Re * ih2 * mv0, gd = P.inv_Re * ih2 * mv0 / 3.0;
    double xlo = 0.0, xhi = 0.0;
    if (a.per && a.ma == 2) {
        const double w_o = tq(T, T_RN, e - a.dn) * 0.5 * (tq(T, a.FNN, e) + tq(T, a.FNN, e + a.dn));
        const double v_o = (4.0 / 3.0) * P.inv_Re * ih2 * tq(T, T_MV, e - a.dn);
        xlo = -0.5 * ih * w_o - v_o;
        xhi = 0.5 * ih * w_o - v_o;
    }
    // the four faces in the lane's order, its own axis first (as in the box
    // of the primitive scheme)
    const double o_blo = other(blo), o_dlo = other(dlo), o_bhi = other(bhi), o_dhi = other(dhi), o_w = other(w_ax);
    const double o_xlo = other(xlo), o_xhi = other(xhi);
    const int o_hlo = other((int)hlo), o_hhi = other((int)hhi);
    double A[4][4], b[4];
    b[0] = blo; b[1] = bhi; b[2] = o_blo; b[3] = o_bhi;
    const double m0l = hlo ? 1.0 : 0.0, m0h = hhi ? 1.0 : 0.0, m1l = o_hlo ? 1.0 : 0.0, m1h = o_hhi ? 1.0 : 0.0;
    A[0][0] = dlo; A[0][1] = m0l * (0.5 * ih * w_ax - vis) + xlo; A[0][2] = m0l * gd; A[0][3] = -m0l * gd;
    A[1][1] = dhi; A[1][0] = m0h * (-0.5 * ih * w_ax - vis) + xhi; A[1][2] = -m0h * gd; A[1][3] = m0h * gd;
    A[2][2] = o_dlo; A[2][3] = m1l * (0.5 * ih * o_w - vis) + o_xlo; A[2][0] = m1l * gd; A[2][1] = -m1l * gd;
    A[3][3] = o_dhi; A[3][2] = m1h * (-0.5 * ih * o_w - vis) + o_xhi; A[3][0] = -m1h * gd; A[3][1] = m1h * gd;
    double inv[4];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        inv[c] = frcp(A[c][c]);
#pragma unroll
        for (int r = c + 1; r < 4; r++) {
            const double l = A[r][c] * inv[c];
#pragma unroll
            for (int t = c + 1; t < 4; t++) A[r][t] -= l * A[c][t];
            b[r] -= l * b[c];
        }
    }
    inv[3] = frcp(A[3][3]);
#pragma unroll
    for (int c = 3; c >= 0; c--) {
        double acc = b[c];
#pragma unroll
        for (int t = c + 1; t < 4; t++) acc -= A[c][t] * b[t];
        b[c] = acc * inv[c];
    }
    const double ulo = tq(T, a.FN, e) + omega * b[0];
    const double uhi = tq(T, a.FN, e + a.dn) + omega * b[1];
    if (TO) {
        double *fo = T.s + (T_NF + hlf) * st;
        if (hlo) fo[e] = ulo;
        if (hhi) fo[e + a.dn] = uhi;
    } else if (hlf) {
        if (hlo) sta<AS>(vnew, k, ulo);
        if (hhi) sta<AS>(vnew, khi, uhi);
    } else {
        if (hlo) sta<AS>(unew, k, ulo);
        if (hhi) sta<AS>(unew, khi, uhi);
    }
    // ---- step 3: pbar from the mass equation with the new u~ (passed by
    // value: the tile keeps the snapshot that other boxes of this colour read)
    const double ulo1 = face_final(P, T, a, e, ih, hlo, ulo), uhi1 = face_final(P, T, a, e + a.dn, ih, hhi, uhi);
    const double Alo = 0.5 * (tq(T, T_RS, e - a.dn) + tq(T, T_RS, e)), Ahi = 0.5 * (tq(T, T_RS, e) + tq(T, T_RS, e + a.dn));
    const double jax = P.dt * P.inv_M * ih2 * ((hlo ? frcp(Alo) : 0.0) + (hhi ? frcp(Ahi) : 0.0));
    const double dv = ih * (uhi1 - ulo1);
    const double div = dv + other(dv), jp = jax + other(jax);
    const double Lmu_new = s.Lmu - s.Sm * (mnew - m0), Lp_new = s.Lp - s.Sm * (pnew - p0);
    const double Np = div - P.alpha * P.inv_Pe * Lmu_new - P.alpha * P.alpha * P.inv_Pe * Lp_new;
    const double Jp = jp + q.Jpp;
    if (hlf == 0) {
        const double pf = pnew + pomega * (ldf<AS>(F.fp, L, i, j) - Np) * frcp(Jp);
        if (TO) T.s[T_P * st + e] = pf;
        else sta<AS>(L.p, k, pf);
    }
}

// residuals of the projection scheme's five equations attached to cell (i,j)
// (as resid_pair: rf is the intermediate-velocity momentum residual of this
// lane's west or south face)
__device__ __forceinline__ void resid_pair_pj(const Phys &P, const View &L, const Tile &T, const Rhs &F, int i, int j, int hlf,
                              double &rc, double &rm, double &rp, double &rf)
{
    const double ih = L.inv_h;
    const int e = T.idx(i, j);
    const Ax a = make_ax(L, T, i, j, hlf);
    const bool hlo = a.per || a.ia >= 1, hhi = a.per || a.ia + 1 < a.ma;
    const double ulo = face_final(P, T, a, e, ih, hlo, tq(T, a.FN, e));
    const double uhi = face_final(P, T, a, e + a.dn, ih, hhi, tq(T, a.FN, e + a.dn));
    const PjAx x = pj_axis(T, a, e, ih, ulo, uhi);
    const CellAx s = cell_sum(cell_axis(T, a, e, ih));
    const CellEq q = cell_eq(P, T, e, s);
    const double adv = x.adv + other(x.adv), div = x.div + other(x.div);
    const double c0 = tq(T, T_C, e), m0 = tq(T, T_MU, e), n0 = tq(T, T_CN, e);
    const double rs = tq(T, T_RS, e), rn = tq(T, T_RN, e);
    rc = ldf<1>(F.fc, L, i, j) - (rn * (c0 - n0) * P.inv_dt + adv - P.inv_Pe * s.Lmu - P.alpha * P.inv_Pe * s.Lp);
    rm = ldf<1>(F.fmu, L, i, j) - (q.Nmu - (rs - rn) * m0);
    rp = ldf<1>(F.fp, L, i, j) - (div - P.alpha * P.inv_Pe * s.Lmu - P.alpha * P.alpha * P.inv_Pe * s.Lp);
    const FaceEq f = face_eq(P, T, a, e, a.it, ih, true);
    rf = hlo ? ldf<1>(face_rhs(F, hlf), L, i, j) - f.N : 0.0;
}

} // namespace qn
