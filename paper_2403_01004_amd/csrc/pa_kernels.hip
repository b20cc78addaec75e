// pa_kernels.hip -- stencil kernels of the parabolic operator F(u) on the
// spherical shell (gfx950), fused with what consumes F on the hot path:
//   kApply  F = F(u)                                   (operator apply)
//   kFirst  y0 = F(u0) + per-tile argmax |F|           (PTL pass, Eq. ptl3)
//   kStage  u_k = mu u_{k-1} + nu u_{k-2} + (1-mu-nu) u0
//                 + mu~ dt F(u_{k-1}) + gamma~ dt y0     (STS stage, App. A)
//   kMatvec q = V p + dt L p, per-tile <p, q>          (BE system matvec)
//
// Work decomposition: one thread per (theta, phi) cell of a radial level,
// 256 consecutive plane cells per workgroup (phi fastest, so loads are
// coalesced along phi and the ragged tail of a plane is a partial last
// block), each workgroup marching over a chunk of radial levels.  Radial
// neighbours live in registers (each level is loaded once per chunk); the
// in-plane neighbours come through L1/L2 (the rows j-1 and j+1 are loaded by
// neighbouring waves of the same or the adjacent workgroup).  The logical
// tile order is remapped so that each of the 8 XCDs gets a contiguous range
// of tiles (workgroups are dispatched round-robin over XCDs), keeping a
// tile's theta-neighbour rows in the same XCD's L2.
//
// Field-aligned operator: L = sum_c v_c v_c^T over cell corners c, v_c the
// corner's (ghost-folded) scatter weights; with per-corner coefficients
// e = sqrt(W kappa) bhat / h (three per corner, computed once per
// coefficient update), a corner's flux is t = e . D where D holds the four
// averaged differences per direction, and a cell gathers sum_c w_c t_c over
// its eight corners.  The march computes each corner plane once per thread
// (the four corners around the thread's cell) and carries the upper-cell
// part of the scatter to the next level, so no corner flux goes to memory.
#include "pa_internal.h"

namespace pa {

__device__ __forceinline__ int xcd_tile()
{
    const int per = gridDim.x >> 3;  // grid is a multiple of 8
    return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

static inline int grid_for_tiles(int ntiles) { return ((ntiles + 7) / 8) * 8; }

int stencil_tiles(int P, int nlev, int rch, int nc)
{
    const int nbx = (P + kBlock - 1) / kBlock;
    const int nrc = (nlev + rch - 1) / rch;
    return nbx * nrc * nc;
}

// ------------------------------------------------------------ reductions

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// deterministic block sum; result valid in thread 0
__device__ double block_sum(double v, double* lds)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += lds[i];
    return s;
}

__device__ __forceinline__ bool better(double v, long long i, double bv, long long bi)
{
    return v > bv || (v == bv && i < bi);
}

// block argmax (largest value, lowest index on ties); result in thread 0
__device__ void block_argmax(double& v, long long& idx, double* ldsv, long long* ldsi)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const long long oi = __shfl_xor(idx, off, 64);
        if (better(ov, oi, v, idx)) { v = ov; idx = oi; }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) { ldsv[w] = v; ldsi[w] = idx; }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i)
            if (better(ldsv[i], ldsi[i], v, idx)) { v = ldsv[i]; idx = ldsi[i]; }
}

// ------------------------------------------------------------ epilogue

template <class T, int MODE>
struct Acc {
    double best = -1.0;
    long long bidx = 0x7fffffffffffffffLL;
    double dot = 0.0;
    int bad = 0;
};

// pointwise streams an STS stage combines with F (prefetched one level ahead)
template <class T>
struct Streams {
    T u0 = 0, y0 = 0, km2 = 0;
};

template <class T, int MODE>
__device__ __forceinline__ void load_streams(const KArgs<T>& a, size_t m, Streams<T>& s)
{
    if constexpr (MODE == kStage) {
        s.u0 = __builtin_nontemporal_load(a.u0 + m);
        s.y0 = __builtin_nontemporal_load(a.y0 + m);
        if (a.km2 == kKm2Array) s.km2 = __builtin_nontemporal_load(a.ukm2 + m);
    }
}

template <class T, int MODE>
__device__ __forceinline__ void epilogue(const KArgs<T>& a, size_t m, T Lu, T V, T uc,
                                         const Streams<T>& st, Acc<T, MODE>& acc)
{
    if constexpr (MODE == kApply || MODE == kFirst) {
        const T F = -Lu / V;
        __builtin_nontemporal_store(F, a.out + m);
        if constexpr (MODE == kFirst) {
            const double af = fabs((double)F);
            if (af > acc.best) { acc.best = af; acc.bidx = (long long)m; }
            if (!isfinite((double)F)) acc.bad = 1;
        }
    } else if constexpr (MODE == kStage) {
        const double F = (double)(-Lu / V);
        const double u0v = (double)st.u0;
        const double y0v = (double)st.y0;
        double km2;
        if (a.km2 == kKm2Array) km2 = (double)st.km2;
        else if (a.km2 == kKm2U0) km2 = u0v;
        else km2 = (double)(T)(u0v + a.a1 * y0v);
        const double r = a.mu * (double)uc + a.nu * km2 + a.c0 * u0v + a.mudt * F + a.gdt * y0v;
        __builtin_nontemporal_store((T)r, a.out + m);
    } else {  // kMatvec
        const T q = V * uc + (T)a.dt * Lu;
        __builtin_nontemporal_store(q, a.out + m);
        acc.dot += (double)uc * (double)q;
    }
}

template <class T, int MODE>
__device__ void finish(const KArgs<T>& a, int L, Acc<T, MODE>& acc)
{
    __shared__ double ldsv[kBlock / 64];
    __shared__ long long ldsi[kBlock / 64];
    if constexpr (MODE == kFirst) {
        double v = acc.best;
        long long i = acc.bidx;
        block_argmax(v, i, ldsv, ldsi);
        if (threadIdx.x == 0) { a.part[L] = v; a.part_idx[L] = i; }
        if (acc.bad) atomicOr(a.flag, 1);
    } else if constexpr (MODE == kMatvec) {
        const double s = block_sum(acc.dot, ldsv);
        if (threadIdx.x == 0) a.part[L] = s;
    }
}

template <class T, bool VIRT>
__device__ __forceinline__ T ldu(const KArgs<T>& a, const T* u, const T* y, size_t q)
{
    if constexpr (VIRT) return (T)((double)u[q] + a.a1 * (double)y[q]);
    else return u[q];
}

// ------------------------------------------------------------ 7-point
//
// Registers per thread: the centre column at levels i-1, i, i+1 and the
// four in-plane neighbours at level i; the loads for level i+1 (centre i+2,
// neighbours, coefficients, stage streams) are issued before level i is
// computed, so every wave keeps two levels of loads in flight.

template <class T>
struct Ring7 {
    T up, w, e, s, n, cp, cw, ce, cs, cn;
};

template <class T, int MODE, bool VIRT>
__global__ __launch_bounds__(kBlock) void k_iso7(Geo<T> g, KArgs<T> a)
{
    const int L = xcd_tile();
    if (L >= a.nbx * a.nrc * a.nc) return;
    if (a.done && *a.done) return;
    const int bx = L % a.nbx, rest = L / a.nbx, rc = rest % a.nrc, c = rest / a.nrc;
    const int np = g.np, nt = g.nt, nr = g.nr, P = g.P;
    const int p = bx * kBlock + threadIdx.x;
    const bool valid = p < P;
    const int pp = valid ? p : P - 1;
    const int j = pp / np, k = pp - j * np;
    const int km = (k == 0) ? np - 1 : k - 1, kp = (k == np - 1) ? 0 : k + 1;
    const bool hs = j > 0, hn = j < nt - 1;
    const size_t cb = (size_t)c * nr * P;
    const T* u = a.u + cb;
    const T* y = VIRT ? a.y0 + cb : nullptr;
    const bool varc = a.coef != nullptr;
    const T* cf = a.coef;
    const int i0 = a.r_lo + rc * a.rch;
    const int i1 = min(a.r_hi, i0 + a.rch);
    const T vtj = g.vt[j], vpk = g.vp[k];
    const T gts = g.gtt[j], gtn = g.gtt[j + 1], gpj = g.gpt[j], gpw = g.gpp[k], gpe = g.gpp[kp];
    const size_t ob = (size_t)c * P + pp;  // boundary data offset
    const int rowo = j * np;
    Acc<T, MODE> acc;

    // loads of level lv+1's centre and level lv's in-plane data.  Every load
    // is unconditional at an in-bounds address: across a pole the row is
    // clamped to the cell's own row (the colatitude coupling there is exactly
    // zero), above the outer level the centre is clamped to the last level
    // (the boundary closure replaces it).
    const int rs = hs ? rowo - np : rowo, rn = hn ? rowo + np : rowo;
    auto fetch = [&](int lv, Ring7<T>& R) {
        const size_t lvb = (size_t)lv * P;
        const size_t lup = (lv + 1 < nr) ? lvb + P : lvb;
        R.up = ldu<T, VIRT>(a, u, y, lup + pp);
        R.w = ldu<T, VIRT>(a, u, y, lvb + rowo + km);
        R.e = ldu<T, VIRT>(a, u, y, lvb + rowo + kp);
        R.s = ldu<T, VIRT>(a, u, y, lvb + rs + k);
        R.n = ldu<T, VIRT>(a, u, y, lvb + rn + k);
        if (varc) {
            R.cp = cf[lup + pp];
            R.cw = cf[lvb + rowo + km];
            R.ce = cf[lvb + rowo + kp];
            R.cs = cf[lvb + rs + k];
            R.cn = cf[lvb + rn + k];
        } else {
            R.cp = R.cw = R.ce = R.cs = R.cn = a.cs;
        }
    };

    T um = 0, uc = 0, cm = a.cs, cc = a.cs;
    Ring7<T> cur = {};
    Streams<T> scur;
    if (i0 < i1) {
        uc = ldu<T, VIRT>(a, u, y, (size_t)i0 * P + pp);
        if (varc) cc = cf[(size_t)i0 * P + pp];
        if (i0 > 0) {
            um = ldu<T, VIRT>(a, u, y, (size_t)(i0 - 1) * P + pp);
            if (varc) cm = cf[(size_t)(i0 - 1) * P + pp];
        }
        fetch(i0, cur);
        load_streams<T, MODE>(a, cb + (size_t)i0 * P + pp, scur);
    }
    for (int i = i0; i < i1; ++i) {
        Ring7<T> nxt = {};
        Streams<T> snxt;
        const bool more = i + 1 < i1;
        if (more) {
            fetch(i + 1, nxt);
            load_streams<T, MODE>(a, cb + (size_t)(i + 1) * P + pp, snxt);
        }
        const T half = T(0.5);
        const T gtri = g.gtr[i];
        // radial faces (i is uniform across the workgroup)
        T Cl, ul, Cu, uu;
        if (i > 0) {
            Cl = half * (cc + cm) * (g.gr[i] * vtj * vpk);
            ul = um;
        } else {
            Cl = (a.bc_in == 0) ? cc * (g.gr[0] * vtj * vpk) : T(0);
            ul = a.affine ? a.ub_in[ob] : T(0);
        }
        if (i < nr - 1) {
            Cu = half * (cc + cur.cp) * (g.gr[i + 1] * vtj * vpk);
            uu = cur.up;
        } else {
            Cu = (a.bc_out == 0) ? cc * (g.gr[nr] * vtj * vpk) : T(0);
            uu = a.affine ? a.ub_out[ob] : T(0);
        }
        T Lu = Cl * (uc - ul);
        Lu += Cu * (uc - uu);
        Lu += half * (cc + cur.cs) * (gtri * gts * vpk) * (uc - cur.s);
        Lu += half * (cc + cur.cn) * (gtri * gtn * vpk) * (uc - cur.n);
        Lu += half * (cc + cur.cw) * (gtri * gpj * gpw) * (uc - cur.w);
        Lu += half * (cc + cur.ce) * (gtri * gpj * gpe) * (uc - cur.e);
        const T V = g.vr[i] * vtj * vpk;
        if (valid) epilogue<T, MODE>(a, cb + (size_t)i * P + pp, Lu, V, uc, scur, acc);
        um = uc; uc = cur.up; cm = cc; cc = cur.cp;
        cur = nxt;
        scur = snxt;
    }
    finish<T, MODE>(a, L, acc);
}

// ------------------------------------------------------------ field-aligned
//
// Per thread and level: the 3x3 (theta, phi) neighbourhood of the thread's
// cell (rows j-1, j+1 only when the corners that use them exist) and the
// three coefficients of the four corners A(j,k) B(j,k+1) C(j+1,k) D(j+1,k+1)
// of the corner plane above.  Level i+2 and corner plane i+2 are fetched
// while level i is computed.

template <class T>
struct Nb9 {
    T x00, x01, x02, x10, x11, x12, x20, x21, x22;
};
template <class T>
struct E12 {
    T ar, at, ap, br, bt, bp, cr, ct, cp, dr, dt, dp;
};

// rows r0/r2 are clamped to the cell's own row at the poles, where the
// corners that use them have zero coefficients
template <class T, bool VIRT>
__device__ __forceinline__ void load9(const KArgs<T>& a, const T* u, const T* y, size_t lv, int r0,
                                      int r1, int r2, int c0, int c1, int c2, Nb9<T>& x)
{
    x.x00 = ldu<T, VIRT>(a, u, y, lv + r0 + c0);
    x.x01 = ldu<T, VIRT>(a, u, y, lv + r0 + c1);
    x.x02 = ldu<T, VIRT>(a, u, y, lv + r0 + c2);
    x.x10 = ldu<T, VIRT>(a, u, y, lv + r1 + c0);
    x.x11 = ldu<T, VIRT>(a, u, y, lv + r1 + c1);
    x.x12 = ldu<T, VIRT>(a, u, y, lv + r1 + c2);
    x.x20 = ldu<T, VIRT>(a, u, y, lv + r2 + c0);
    x.x21 = ldu<T, VIRT>(a, u, y, lv + r2 + c1);
    x.x22 = ldu<T, VIRT>(a, u, y, lv + r2 + c2);
}

template <class T>
__device__ __forceinline__ void load_e(const T* e, size_t nco, size_t q0, size_t q1, int k, int kp,
                                       E12<T>& E)
{
    E.ar = e[q0 + k]; E.at = e[nco + q0 + k]; E.ap = e[2 * nco + q0 + k];
    E.br = e[q0 + kp]; E.bt = e[nco + q0 + kp]; E.bp = e[2 * nco + q0 + kp];
    E.cr = e[q1 + k]; E.ct = e[nco + q1 + k]; E.cp = e[2 * nco + q1 + k];
    E.dr = e[q1 + kp]; E.dt = e[nco + q1 + kp]; E.dp = e[2 * nco + q1 + kp];
}

// mirror ghost level across a radial boundary: Dirichlet 2 u_b - u (u_b = 0
// in linear mode), no-flux u
template <class T>
__device__ __forceinline__ T ghost1(T x, const T* ub, size_t o, int bc, int affine)
{
    if (bc != 0) return x;
    const T b = affine ? ub[o] : T(0);
    return T(2) * b - x;
}

template <class T>
__device__ __forceinline__ void ghost9(const Nb9<T>& x, const T* ub, int bc, int affine,
                                       size_t ob, int r0, int r1, int r2, int c0, int c1, int c2,
                                       Nb9<T>& gx)
{
    gx.x00 = ghost1(x.x00, ub, ob + r0 + c0, bc, affine);
    gx.x01 = ghost1(x.x01, ub, ob + r0 + c1, bc, affine);
    gx.x02 = ghost1(x.x02, ub, ob + r0 + c2, bc, affine);
    gx.x10 = ghost1(x.x10, ub, ob + r1 + c0, bc, affine);
    gx.x11 = ghost1(x.x11, ub, ob + r1 + c1, bc, affine);
    gx.x12 = ghost1(x.x12, ub, ob + r1 + c2, bc, affine);
    gx.x20 = ghost1(x.x20, ub, ob + r2 + c0, bc, affine);
    gx.x21 = ghost1(x.x21, ub, ob + r2 + c1, bc, affine);
    gx.x22 = ghost1(x.x22, ub, ob + r2 + c2, bc, affine);
}

// Scatter weights of the thread's cell for one corner plane: as the upper
// cell (wu) and the lower cell (wd) of a corner with coefficients (er, et, ep)
// where st, sp = +1 when the cell is the corner's upper row / column.
// kind 0: interior plane; 1: inner radial boundary (real cells above);
// 2: outer radial boundary (real cells below).
template <class T>
struct PlaneW {
    T ru, rd, tu, td;  // wu = ru*er + tu*tang, wd = rd*er + td*tang
};

template <class T>
__device__ __forceinline__ PlaneW<T> plane_weights(int kind, int bc)
{
    PlaneW<T> w;
    if (kind == 0) {
        w.ru = T(0.25); w.rd = T(-0.25); w.tu = T(0.25); w.td = T(0.25);
    } else if (kind == 1) {
        w.ru = bc == 0 ? T(0.5) : T(0); w.tu = bc == 0 ? T(0) : T(0.5); w.rd = T(0); w.td = T(0);
    } else {
        w.rd = bc == 0 ? T(-0.5) : T(0); w.td = bc == 0 ? T(0) : T(0.5); w.ru = T(0); w.tu = T(0);
    }
    return w;
}

// one corner: flux t = e . D, D the averaged differences over its 2x2x2
// cells (lower level l*, upper level h*: 00 = (row0,col0), 01 = (row0,col1),
// 10 = (row1,col0), 11 = (row1,col1)); accumulates the cell's weight times t
template <class T>
__device__ __forceinline__ void corner1(T l00, T l01, T l10, T l11, T h00, T h01, T h10, T h11,
                                        T er, T et, T ep, T st, T sp, const PlaneW<T>& w, T& up,
                                        T& dn)
{
    const T qt = T(0.25);
    const T s00 = l00 + h00, s01 = l01 + h01, s10 = l10 + h10, s11 = l11 + h11;
    const T Dr = qt * ((h00 - l00) + (h01 - l01) + (h10 - l10) + (h11 - l11));
    const T Dt = qt * (s10 + s11 - s00 - s01);
    const T Dp = qt * (s01 + s11 - s00 - s10);
    const T t = er * Dr + et * Dt + ep * Dp;
    const T tang = st * et + sp * ep;
    up += (w.ru * er + w.tu * tang) * t;
    dn += (w.rd * er + w.td * tang) * t;
}

template <class T>
__device__ __forceinline__ void corner_plane(const Nb9<T>& lo, const Nb9<T>& hi, const E12<T>& E,
                                             const PlaneW<T>& w, T& up, T& dn)
{
    up = 0;
    dn = 0;
    // A: rows (j-1, j), columns (k-1, k): the cell is row 1, column 1
    corner1<T>(lo.x00, lo.x01, lo.x10, lo.x11, hi.x00, hi.x01, hi.x10, hi.x11, E.ar, E.at, E.ap,
               T(1), T(1), w, up, dn);
    // B: rows (j-1, j), columns (k, k+1)
    corner1<T>(lo.x01, lo.x02, lo.x11, lo.x12, hi.x01, hi.x02, hi.x11, hi.x12, E.br, E.bt, E.bp,
               T(1), T(-1), w, up, dn);
    // C: rows (j, j+1), columns (k-1, k)
    corner1<T>(lo.x10, lo.x11, lo.x20, lo.x21, hi.x10, hi.x11, hi.x20, hi.x21, E.cr, E.ct, E.cp,
               T(-1), T(1), w, up, dn);
    // D: rows (j, j+1), columns (k, k+1)
    corner1<T>(lo.x11, lo.x12, lo.x21, lo.x22, hi.x11, hi.x12, hi.x21, hi.x22, E.dr, E.dt, E.dp,
               T(-1), T(-1), w, up, dn);
}

template <class T, int MODE, bool VIRT>
__global__ __launch_bounds__(kBlock) void k_aligned(Geo<T> g, KArgs<T> a)
{
    const int L = xcd_tile();
    if (L >= a.nbx * a.nrc * a.nc) return;
    if (a.done && *a.done) return;
    const int bx = L % a.nbx, rest = L / a.nbx, rc = rest % a.nrc, c = rest / a.nrc;
    const int np = g.np, nt = g.nt, nr = g.nr, P = g.P;
    const int p = bx * kBlock + threadIdx.x;
    const bool valid = p < P;
    const int pp = valid ? p : P - 1;
    const int j = pp / np, k = pp - j * np;
    const int km = (k == 0) ? np - 1 : k - 1, kp = (k == np - 1) ? 0 : k + 1;
    const int r1 = j * np;
    const int r0 = (j >= 1) ? r1 - np : r1, r2 = (j + 1 <= nt - 1) ? r1 + np : r1;
    const size_t cb = (size_t)c * nr * P;
    const T* u = a.u + cb;
    const T* y = VIRT ? a.y0 + cb : nullptr;
    const size_t ob = (size_t)c * P;
    const size_t nco = (size_t)(nr + 1) * (nt + 1) * np;
    const size_t cplane = (size_t)(nt + 1) * np;
    const size_t qa = (size_t)j * np, qc = (size_t)(j + 1) * np;  // corner rows j, j+1 (<= nt)
    const int i0 = a.r_lo + rc * a.rch;
    const int i1 = min(a.r_hi, i0 + a.rch);
    const T vtj = g.vt[j], vpk = g.vp[k];
    Acc<T, MODE> acc;
    Nb9<T> lo = {}, hi = {}, nx = {};
    E12<T> E = {}, En = {};
    Streams<T> scur, snxt;
    T carry = 0;
    if (i0 < i1) {
        load9<T, VIRT>(a, u, y, (size_t)i0 * P, r0, r1, r2, km, k, kp, hi);
        if (i0 == 0)
            ghost9<T>(hi, a.ub_in, a.bc_in, a.affine, ob, r0, r1, r2, km, k, kp, lo);
        else
            load9<T, VIRT>(a, u, y, (size_t)(i0 - 1) * P, r0, r1, r2, km, k, kp, lo);
        load_e<T>(a.e, nco, (size_t)i0 * cplane + qa, (size_t)i0 * cplane + qc, k, kp, E);
        T up, dn;
        corner_plane<T>(lo, hi, E, plane_weights<T>(i0 == 0 ? 1 : 0, a.bc_in), up, dn);
        carry = up;
        // level i0+1 and corner plane i0+1 for the first iteration
        load9<T, VIRT>(a, u, y, (size_t)min(i0 + 1, nr - 1) * P, r0, r1, r2, km, k, kp, nx);
        load_e<T>(a.e, nco, (size_t)(i0 + 1) * cplane + qa, (size_t)(i0 + 1) * cplane + qc, k, kp,
                  E);
        load_streams<T, MODE>(a, cb + (size_t)i0 * P + pp, scur);
    }
    for (int i = i0; i < i1; ++i) {
        const int ic = i + 1;
        lo = hi;
        int kind = 0, bc = 0;
        if (ic < nr) {
            hi = nx;
        } else {
            ghost9<T>(lo, a.ub_out, a.bc_out, a.affine, ob, r0, r1, r2, km, k, kp, hi);
            kind = 2;
            bc = a.bc_out;
        }
        // prefetch level i+2 and corner plane i+2 for the next iteration
        const bool more = i + 1 < i1;
        if (more) {
            load9<T, VIRT>(a, u, y, (size_t)min(ic + 1, nr - 1) * P, r0, r1, r2, km, k, kp, nx);
            load_e<T>(a.e, nco, (size_t)(ic + 1) * cplane + qa, (size_t)(ic + 1) * cplane + qc, k,
                      kp, En);
            load_streams<T, MODE>(a, cb + (size_t)(i + 1) * P + pp, snxt);
        }
        T up, dn;
        corner_plane<T>(lo, hi, E, plane_weights<T>(kind, bc), up, dn);
        const T Lu = carry + dn;
        carry = up;
        const T V = g.vr[i] * vtj * vpk;
        if (valid) epilogue<T, MODE>(a, cb + (size_t)i * P + pp, Lu, V, lo.x11, scur, acc);
        E = En;
        scur = snxt;
    }
    finish<T, MODE>(a, L, acc);
}

// ------------------------------------------------------------ launchers

template <class T, int MODE, bool VIRT>
static void go_iso7(const Geo<T>& g, const KArgs<T>& a, hipStream_t s)
{
    const int nt = a.nbx * a.nrc * a.nc;
    hipLaunchKernelGGL((k_iso7<T, MODE, VIRT>), dim3(grid_for_tiles(nt)), dim3(kBlock), 0, s, g, a);
}
template <class T, int MODE, bool VIRT>
static void go_aligned(const Geo<T>& g, const KArgs<T>& a, hipStream_t s)
{
    const int nt = a.nbx * a.nrc * a.nc;
    hipLaunchKernelGGL((k_aligned<T, MODE, VIRT>), dim3(grid_for_tiles(nt)), dim3(kBlock), 0, s,
                       g, a);
}

#define PA_DISPATCH(FN)                                                 \
    switch (mode) {                                                     \
    case kApply:                                                        \
        if (virt) FN<T, kApply, true>(g, a, s);                         \
        else FN<T, kApply, false>(g, a, s);                             \
        break;                                                          \
    case kFirst: FN<T, kFirst, false>(g, a, s); break;                  \
    case kMatvec: FN<T, kMatvec, false>(g, a, s); break;                \
    default:                                                            \
        if (virt) FN<T, kStage, true>(g, a, s);                         \
        else FN<T, kStage, false>(g, a, s);                             \
    }

template <class T>
void launch_iso7(int mode, bool virt, const Geo<T>& g, const KArgs<T>& a, hipStream_t s)
{
    PA_DISPATCH(go_iso7)
}
template <class T>
void launch_aligned(int mode, bool virt, const Geo<T>& g, const KArgs<T>& a, hipStream_t s)
{
    PA_DISPATCH(go_aligned)
}
template void launch_iso7<double>(int, bool, const Geo<double>&, const KArgs<double>&, hipStream_t);
template void launch_iso7<float>(int, bool, const Geo<float>&, const KArgs<float>&, hipStream_t);
template void launch_aligned<double>(int, bool, const Geo<double>&, const KArgs<double>&, hipStream_t);
template void launch_aligned<float>(int, bool, const Geo<float>&, const KArgs<float>&, hipStream_t);

// ------------------------------------------------------------ setup kernels

__global__ void k_coef(const double* T0, double scale, double expo, int n, double* c64,
                       float* c32, int* flag)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const double c = T0 ? scale * pow(T0[m], expo) : scale;
    if (!isfinite(c) || c < 0.0) atomicOr(flag, 1);
    c64[m] = c;
    if (c32) c32[m] = (float)c;
}

void launch_coef(const double* T0, double scale, double expo, int n, double* c64, float* c32,
                 int* flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_coef, dim3((n + 255) / 256), dim3(256), 0, s, T0, scale, expo, n, c64,
                       c32, flag);
}

// per-corner coefficients e_d = sqrt(W kappa_c) bhat_d / h_d
__global__ void k_corner_e(int nr, int nt, int np, CornerGeo cg, const double* coef,
                           const double* B, double* e64, float* e32, int* flag)
{
    const size_t nco = (size_t)(nr + 1) * (nt + 1) * np;
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nco) return;
    const int kc = (int)(q % np);
    const int jc = (int)((q / np) % (nt + 1));
    const int ic = (int)(q / ((size_t)np * (nt + 1)));
    double er = 0.0, et = 0.0, ep = 0.0;
    if (jc > 0 && jc < nt) {
        const int kl = (kc == 0) ? np - 1 : kc - 1;
        const size_t P = (size_t)nt * np;
        double ks = 0.0;
        int nk = 0;
        for (int a = 0; a < 2; ++a) {
            const int i = ic - 1 + a;
            if (i < 0 || i >= nr) continue;
            for (int b = 0; b < 2; ++b) {
                const size_t rowo = (size_t)i * P + (size_t)(jc - 1 + b) * np;
                ks += coef[rowo + kl] + coef[rowo + kc];
                nk += 2;
            }
        }
        const double kap = ks / nk;
        const double bx = B[q], by = B[nco + q], bz = B[2 * nco + q];
        const double mag = sqrt(bx * bx + by * by + bz * bz);
        if (!isfinite(mag)) atomicOr(flag, 1);
        if (mag > 0.0) {
            const double Rc = cg.R[ic];
            const double hr = cg.hr[ic];
            const double ht = Rc * cg.htt[jc];
            const double hp = Rc * cg.sT[jc] * cg.dpc[kc];
            const double W = cg.wr[ic] * ht * hp;
            const double sw = sqrt(W * kap) / mag;
            er = sw * bx / hr;
            et = sw * by / ht;
            ep = sw * bz / hp;
        }
    }
    e64[q] = er;
    e64[nco + q] = et;
    e64[2 * nco + q] = ep;
    if (e32) {
        e32[q] = (float)er;
        e32[nco + q] = (float)et;
        e32[2 * nco + q] = (float)ep;
    }
}

void launch_corner_e(int nr, int nt, int np, const CornerGeo& cg, const double* coef,
                     const double* B, double* e64, float* e32, int* flag, hipStream_t s)
{
    const size_t nco = (size_t)(nr + 1) * (nt + 1) * np;
    hipLaunchKernelGGL(k_corner_e, dim3((unsigned)((nco + 255) / 256)), dim3(256), 0, s, nr, nt,
                       np, cg, coef, B, e64, e32, flag);
}

// diag(L) and the Gershgorin row bound sum_n |L_mn| / V_m (per-block maxima)
__global__ __launch_bounds__(kBlock) void k_diag_iso7(Geo<double> g, const double* coef,
                                                      double cs, int bc_in, int bc_out,
                                                      double* diag, double* part)
{
    __shared__ double lds[kBlock / 64];
    const int nr = g.nr, nt = g.nt, np = g.np, P = g.P;
    const size_t N = (size_t)nr * P;
    const size_t m = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    double rho = 0.0;
    if (m < N) {
        const int i = (int)(m / P), pp = (int)(m % P), j = pp / np, k = pp % np;
        const int km = (k == 0) ? np - 1 : k - 1, kp = (k == np - 1) ? 0 : k + 1;
        auto cf = [&](size_t q) { return coef ? coef[q] : cs; };
        const double cc = cf(m);
        const double vt = g.vt[j], vp = g.vp[k];
        double d = 0.0, off = 0.0, C;
        if (i > 0) { C = 0.5 * (cc + cf(m - P)) * (g.gr[i] * vt * vp); d += C; off += C; }
        else if (bc_in == 0) d += cc * (g.gr[0] * vt * vp);
        if (i < nr - 1) { C = 0.5 * (cc + cf(m + P)) * (g.gr[i + 1] * vt * vp); d += C; off += C; }
        else if (bc_out == 0) d += cc * (g.gr[nr] * vt * vp);
        if (j > 0) { C = 0.5 * (cc + cf(m - np)) * (g.gtr[i] * g.gtt[j] * vp); d += C; off += C; }
        if (j < nt - 1) { C = 0.5 * (cc + cf(m + np)) * (g.gtr[i] * g.gtt[j + 1] * vp); d += C; off += C; }
        const size_t rb = m - k;
        C = 0.5 * (cc + cf(rb + km)) * (g.gtr[i] * g.gpt[j] * g.gpp[k]); d += C; off += C;
        C = 0.5 * (cc + cf(rb + kp)) * (g.gtr[i] * g.gpt[j] * g.gpp[kp]); d += C; off += C;
        diag[m] = d;
        rho = (d + off) / (g.vr[i] * vt * vp);
    }
    // block maximum (values are >= 0)
    double v = rho;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = lds[0];
        for (int w = 1; w < kBlock / 64; ++w) b = fmax(b, lds[w]);
        part[blockIdx.x] = b;
    }
}

__global__ __launch_bounds__(kBlock) void k_diag_aligned(Geo<double> g, const double* e,
                                                         int bc_in, int bc_out, double* diag,
                                                         double* part)
{
    __shared__ double lds[kBlock / 64];
    const int nr = g.nr, nt = g.nt, np = g.np, P = g.P;
    const size_t N = (size_t)nr * P;
    const size_t nco = (size_t)(nr + 1) * (nt + 1) * np;
    const size_t m = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    double rho = 0.0;
    if (m < N) {
        const int i = (int)(m / P), pp = (int)(m % P), j = pp / np, k = pp % np;
        const int kp = (k == np - 1) ? 0 : k + 1;
        double d = 0.0, s = 0.0;
        for (int a = 0; a < 2; ++a) {        // corner plane ic = i + 1 - a
            const int ic = i + 1 - a;
            const double sr = a ? 1.0 : -1.0;  // a = 1: cell is above the plane
            for (int b = 0; b < 2; ++b) {    // corner row jc = j + 1 - b
                const int jc = j + 1 - b;
                if (jc == 0 || jc == nt) continue;
                const double st = b ? 1.0 : -1.0;
                for (int c = 0; c < 2; ++c) {
                    const int kc = c ? k : kp;
                    const double sp = c ? 1.0 : -1.0;
                    const size_t q = ((size_t)ic * (nt + 1) + jc) * np + kc;
                    const double er = e[q], et = e[nco + q], ep = e[2 * nco + q];
                    double w, wsum = 0.0;
                    const bool bnd = (ic == 0) || (ic == nr);
                    const int bc = (ic == 0) ? bc_in : bc_out;
                    if (!bnd) {
                        w = 0.25 * (sr * er + st * et + sp * ep);
                        for (int x = 0; x < 8; ++x)
                            wsum += fabs(0.25 * ((x & 4 ? 1.0 : -1.0) * er + (x & 2 ? 1.0 : -1.0) * et +
                                                 (x & 1 ? 1.0 : -1.0) * ep));
                    } else if (bc == 0) {
                        w = 0.5 * sr * er;
                        wsum = 4.0 * fabs(0.5 * er);
                    } else {
                        w = 0.5 * (st * et + sp * ep);
                        for (int x = 0; x < 4; ++x)
                            wsum += fabs(0.5 * ((x & 2 ? 1.0 : -1.0) * et + (x & 1 ? 1.0 : -1.0) * ep));
                    }
                    d += w * w;
                    s += fabs(w) * wsum;
                }
            }
        }
        diag[m] = d;
        rho = s / (g.vr[i] * g.vt[j] * g.vp[k]);
    }
    double v = rho;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = lds[0];
        for (int w = 1; w < kBlock / 64; ++w) b = fmax(b, lds[w]);
        part[blockIdx.x] = b;
    }
}

void launch_diag_iso7(const Geo<double>& g, const double* coef, double cs, int bc_in, int bc_out,
                      double* diag, double* part, hipStream_t s, int* nparts)
{
    const size_t N = (size_t)g.nr * g.P;
    const int nb = (int)((N + kBlock - 1) / kBlock);
    *nparts = nb;
    hipLaunchKernelGGL(k_diag_iso7, dim3(nb), dim3(kBlock), 0, s, g, coef, cs, bc_in, bc_out, diag,
                       part);
}

void launch_diag_aligned(const Geo<double>& g, const double* e, int bc_in, int bc_out,
                         double* diag, double* part, hipStream_t s, int* nparts)
{
    const size_t N = (size_t)g.nr * g.P;
    const int nb = (int)((N + kBlock - 1) / kBlock);
    *nparts = nb;
    hipLaunchKernelGGL(k_diag_aligned, dim3(nb), dim3(kBlock), 0, s, g, e, bc_in, bc_out, diag,
                       part);
}

}  // namespace pa
