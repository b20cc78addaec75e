// pa_kernels.hip -- stencil kernels of the parabolic operator F(u) on the
// spherical shell (gfx950), fused with what consumes F on the hot path:
//   kApply  F = F(u)                                   (operator apply)
//   kFirst  y0 = F(u0) + per-tile argmax |F|           (PTL pass, Eq. ptl3)
//   kStage  u_k = mu u_{k-1} + nu u_{k-2} + (1-mu-nu) u0
//                 + mu~ dt F(u_{k-1}) + gamma~ dt y0     (STS stage, App. A)
//   kMatvec q = V p + dt L p, per-tile <p, q>          (BE system matvec)
//
// Work decomposition.  A workgroup of 256 threads owns a 32 (phi) x 8
// (theta) tile of cells and marches over a chunk of radial levels.  Each
// thread owns one tile cell and (threads 0..83) one cell of the one-cell
// halo ring; per level it loads just those values -- plus, for the
// field-aligned operator, the three coefficients of at most two corners, and
// for a stage the pointwise streams u_{k-2}, u0, y0 -- and it issues them two
// levels ahead of their use, so every wave keeps several levels of
// independent HBM loads in flight at the cost of a few registers.  The
// tile's planes are staged in LDS, where the in-plane neighbours are read.
// The logical tile order puts phi tiles fastest and gives each of the 8 XCDs
// a contiguous range (workgroups are dispatched round-robin over XCDs), so
// the halo rows shared by neighbouring tiles are found in that XCD's L2.
//
// Field-aligned operator: L = sum_c v_c v_c^T over cell corners, v_c the
// corner's (ghost-folded) scatter weights; with per-corner coefficients
// e = sqrt(W kappa) bhat / h (three per corner), a corner's flux is
// t = e . D, D the averaged differences over its 2x2x2 cells, and a cell
// gathers sum_c w_c t_c over its eight corners.  Each corner of a plane is
// computed once per tile (9 x 33 corners for 256 cells) into LDS; the upper
// cell's share of a corner plane is carried in a register to the next level.
#include "pa_internal.h"

namespace pa {

constexpr int TX = 32, TY = 8;          // tile (phi x theta)
constexpr int HX = TX + 2, HY = TY + 2;  // tile plus halo ring
constexpr int HN = HX * HY;              // 340 plane slots
constexpr int NHALO = HN - TX * TY;      // 84 halo slots
constexpr int CX = TX + 1, CY = TY + 1;  // corners of a tile plane
constexpr int NCOR = CX * CY;            // 297

__device__ __forceinline__ int xcd_tile()
{
    const int per = gridDim.x >> 3;  // grid is a multiple of 8
    return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

static inline int grid_for_tiles(int ntiles) { return ((ntiles + 7) / 8) * 8; }

int tiles_per_plane(int nt, int np) { return ((np + TX - 1) / TX) * ((nt + TY - 1) / TY); }

int stencil_tiles(int nt, int np, int nlev, int rch, int nc)
{
    const int nrc = (nlev + rch - 1) / rch;
    return tiles_per_plane(nt, np) * nrc * nc;
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

// ------------------------------------------------------------ tile geometry

// Where a thread's two plane slots live: its own cell (slot (ty+1, tx+1))
// and, for threads below NHALO, one halo slot.  Global rows are clamped at
// the poles (those neighbours carry zero coupling) and columns wrap.
struct TileMap {
    int k0, j0;     // tile origin
    int tx, ty;     // thread's cell in the tile
    int j, k;       // thread's global cell (may lie outside the mesh)
    bool valid;     // the thread's cell exists
    int own_off;    // in-plane offset of the own cell (clamped / wrapped)
    int own_slot;   // LDS slot of the own cell
    bool has_h;     // the thread owns a halo slot
    int h_off, h_slot;
};

__device__ __forceinline__ int wrapk(int k, int np)
{
    k %= np;
    return k < 0 ? k + np : k;
}

__device__ __forceinline__ int slot_offset(int hy, int hx, int j0, int k0, int nt, int np)
{
    const int j = min(max(j0 - 1 + hy, 0), nt - 1);
    return j * np + wrapk(k0 - 1 + hx, np);
}

__device__ __forceinline__ TileMap tile_map(int bxk, int bxj, int nt, int np)
{
    TileMap m;
    const int t = threadIdx.x;
    m.k0 = bxk * TX;
    m.j0 = bxj * TY;
    m.tx = t % TX;
    m.ty = t / TX;
    m.j = m.j0 + m.ty;
    m.k = m.k0 + m.tx;
    m.valid = m.j < nt && m.k < np;
    m.own_slot = (m.ty + 1) * HX + (m.tx + 1);
    m.own_off = slot_offset(m.ty + 1, m.tx + 1, m.j0, m.k0, nt, np);
    m.has_h = t < NHALO;
    int hy, hx;
    if (t < HX) { hy = 0; hx = t; }
    else if (t < 2 * HX) { hy = HY - 1; hx = t - HX; }
    else if (t < 2 * HX + TY) { hy = 1 + (t - 2 * HX); hx = 0; }
    else { hy = 1 + (t - 2 * HX - TY); hx = HX - 1; }
    if (!m.has_h) { hy = 1; hx = 1; }
    m.h_slot = hy * HX + hx;
    m.h_off = slot_offset(hy, hx, m.j0, m.k0, nt, np);
    return m;
}

// ------------------------------------------------------------ epilogue

template <class T, int MODE>
struct Acc {
    double best = -1.0;
    long long bidx = 0x7fffffffffffffffLL;
    double dot = 0.0;
    int bad = 0;
};

// pointwise streams an STS stage combines with F
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

// stencil input value: u, or the virtual first stage u0 + a1 y0
template <class T, bool VIRT>
__device__ __forceinline__ T ldu(const KArgs<T>& a, const T* u, const T* y, size_t q)
{
    if constexpr (VIRT) return (T)((double)u[q] + a.a1 * (double)y[q]);
    else return u[q];
}

// ------------------------------------------------------------ 7-point

// one radial level's loads of a thread (own cell, halo slot, coefficients,
// stage streams of the own cell)
template <class T>
struct Lev7 {
    T u, h, c, ch;
    Streams<T> s;
};

template <class T, int MODE, bool VIRT>
__device__ __forceinline__ void fetch7(const KArgs<T>& a, const T* u, const T* y, const T* cf,
                                       const TileMap& tm, size_t cb, int P, int lv, bool plane,
                                       Lev7<T>& R)
{
    const size_t lb = (size_t)lv * P;
    R.u = ldu<T, VIRT>(a, u, y, lb + tm.own_off);
    if (cf) R.c = cf[lb + tm.own_off];
    if (plane) {
        if (tm.has_h) {
            R.h = ldu<T, VIRT>(a, u, y, lb + tm.h_off);
            if (cf) R.ch = cf[lb + tm.h_off];
        }
        load_streams<T, MODE>(a, cb + lb + tm.own_off, R.s);
    }
}

template <class T, int MODE, bool VIRT>
__global__ __launch_bounds__(kBlock) void k_iso7(Geo<T> g, KArgs<T> a)
{
    __shared__ T su[2][HN];
    __shared__ T sc[2][HN];
    const int L = xcd_tile();
    if (L >= a.nbx * a.nrc * a.nc) return;
    if (a.done && *a.done) return;
    const int np = g.np, nt = g.nt, nr = g.nr, P = g.P;
    const int ntk = (np + TX - 1) / TX;
    const int bx = L % a.nbx, rest = L / a.nbx, rc = rest % a.nrc, c = rest / a.nrc;
    const TileMap tm = tile_map(bx % ntk, bx / ntk, nt, np);
    const size_t cb = (size_t)c * nr * P;
    const T* u = a.u + cb;
    const T* y = VIRT ? a.y0 + cb : nullptr;
    const T* cf = a.coef;  // null: constant coefficient a.cs
    const int i0 = a.r_lo + rc * a.rch;
    const int i1 = min(a.r_hi, i0 + a.rch);
    const int j = min(tm.j, nt - 1), k = tm.valid ? tm.k : 0;
    const int kp = (k == np - 1) ? 0 : k + 1;
    const T vtj = g.vt[j], vpk = g.vp[k];
    const T gts = g.gtt[j], gtn = g.gtt[j + 1], gpj = g.gpt[j], gpw = g.gpp[k], gpe = g.gpp[kp];
    const size_t ob = (size_t)c * P + tm.own_off;  // boundary data of the own cell
    const int so = tm.own_slot;
    Acc<T, MODE> acc;

    // ring R[q] = loads of level i + q; level i + DEPTH is issued while
    // level i is computed (DEPTH levels of loads in flight per thread)
    constexpr int DEPTH = 2;
    Lev7<T> R[DEPTH + 1] = {};
    T um = 0, cm = a.cs;
    if (i0 < i1) {
        if (i0 > 0) {
            um = ldu<T, VIRT>(a, u, y, (size_t)(i0 - 1) * P + tm.own_off);
            if (cf) cm = cf[(size_t)(i0 - 1) * P + tm.own_off];
        }
#pragma unroll
        for (int q = 0; q < DEPTH; ++q)
            if (i0 + q < nr && i0 + q <= i1)
                fetch7<T, MODE, VIRT>(a, u, y, cf, tm, cb, P, i0 + q, i0 + q < i1, R[q]);
    }
    for (int i = i0; i < i1; ++i) {
        const int b = i & 1;
        const Lev7<T>& R0 = R[0];
        const Lev7<T>& R1 = R[1];
        su[b][so] = R0.u;
        if (tm.has_h) su[b][tm.h_slot] = R0.h;
        if (cf) {
            sc[b][so] = R0.c;
            if (tm.has_h) sc[b][tm.h_slot] = R0.ch;
        }
        // loads for level i+DEPTH (its own value is a radial neighbour later)
        if (i + DEPTH < nr && i + DEPTH <= i1)
            fetch7<T, MODE, VIRT>(a, u, y, cf, tm, cb, P, i + DEPTH, i + DEPTH < i1, R[DEPTH]);
        __syncthreads();
        const T uc = R0.u;
        const T cc = cf ? R0.c : a.cs;
        const T us = su[b][so - HX], un = su[b][so + HX], uw = su[b][so - 1], ue = su[b][so + 1];
        T cs_ = a.cs, cn = a.cs, cw = a.cs, ce = a.cs;
        if (cf) {
            cs_ = sc[b][so - HX];
            cn = sc[b][so + HX];
            cw = sc[b][so - 1];
            ce = sc[b][so + 1];
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
            Cu = half * (cc + (cf ? R1.c : a.cs)) * (g.gr[i + 1] * vtj * vpk);
            uu = R1.u;
        } else {
            Cu = (a.bc_out == 0) ? cc * (g.gr[nr] * vtj * vpk) : T(0);
            uu = a.affine ? a.ub_out[ob] : T(0);
        }
        T Lu = Cl * (uc - ul);
        Lu += Cu * (uc - uu);
        Lu += half * (cc + cs_) * (gtri * gts * vpk) * (uc - us);
        Lu += half * (cc + cn) * (gtri * gtn * vpk) * (uc - un);
        Lu += half * (cc + cw) * (gtri * gpj * gpw) * (uc - uw);
        Lu += half * (cc + ce) * (gtri * gpj * gpe) * (uc - ue);
        const T V = g.vr[i] * vtj * vpk;
        if (tm.valid) epilogue<T, MODE>(a, cb + (size_t)i * P + tm.own_off, Lu, V, uc, R0.s, acc);
        um = uc;
        cm = cc;
#pragma unroll
        for (int q = 0; q < DEPTH; ++q) R[q] = R[q + 1];
    }
    finish<T, MODE>(a, L, acc);
}

// ------------------------------------------------------------ field-aligned

// one corner plane ic's loads of a thread: its own / halo cell of level ic,
// the coefficients of corners t and t + 256, and the stage streams of the
// own cell at level ic - 1 (the level that plane completes)
template <class T>
struct LevA {
    T u, h;
    T e0r, e0t, e0p, e1r, e1t, e1p;
    Streams<T> s;
};

template <class T, int MODE, bool VIRT>
__device__ __forceinline__ void fetchA(const KArgs<T>& a, const T* u, const T* y, const TileMap& tm,
                                       size_t cb, int P, int nr, int nt, int np, size_t nco,
                                       int ic, int i0, int i1, int cq0, int cq1, bool has_c1,
                                       LevA<T>& R)
{
    if (ic < nr) {
        const size_t lb = (size_t)ic * P;
        R.u = ldu<T, VIRT>(a, u, y, lb + tm.own_off);
        if (tm.has_h) R.h = ldu<T, VIRT>(a, u, y, lb + tm.h_off);
    }
    const size_t qb = (size_t)ic * (nt + 1) * np;
    R.e0r = a.e[qb + cq0];
    R.e0t = a.e[nco + qb + cq0];
    R.e0p = a.e[2 * nco + qb + cq0];
    if (has_c1) {
        R.e1r = a.e[qb + cq1];
        R.e1t = a.e[nco + qb + cq1];
        R.e1p = a.e[2 * nco + qb + cq1];
    }
    if (ic - 1 >= i0 && ic - 1 < i1)
        load_streams<T, MODE>(a, cb + (size_t)(ic - 1) * P + tm.own_off, R.s);
}

// Scatter weights for one corner plane: the cell's weight as the upper cell
// is ru*er + tu*(st*et + sp*ep), as the lower cell rd*er + td*(...), with
// st, sp = +1 when the cell is the corner's upper row / column.
// kind 0: interior plane; 1: inner radial boundary (real cells above);
// 2: outer radial boundary (real cells below).
template <class T>
struct PlaneW {
    T ru, rd, tu, td;
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

// mirror ghost across a radial boundary: Dirichlet 2 u_b - u (u_b = 0 in
// linear mode), no-flux u
template <class T>
__device__ __forceinline__ T ghost(T x, const T* ub, size_t o, int bc, int affine)
{
    if (bc != 0) return x;
    const T b = affine ? ub[o] : T(0);
    return T(2) * b - x;
}

// flux t = e . D of tile corner (cy, cx) between the LDS planes lo and hi;
// gside 1: lo is the mirror ghost of hi, 2: hi is the ghost of lo
template <class T>
__device__ __forceinline__ T corner_flux(const T* lo, const T* hi, int cy, int cx, T er, T et,
                                         T ep, int gside, const T* ub, int bc, int affine,
                                         size_t ubo, int j0, int k0, int nt, int np)
{
    const int s00 = cy * HX + cx, s01 = s00 + 1, s10 = s00 + HX, s11 = s10 + 1;
    T l00, l01, l10, l11, h00, h01, h10, h11;
    if (gside == 1) {
        h00 = hi[s00]; h01 = hi[s01]; h10 = hi[s10]; h11 = hi[s11];
        l00 = ghost(h00, ub, ubo + slot_offset(cy, cx, j0, k0, nt, np), bc, affine);
        l01 = ghost(h01, ub, ubo + slot_offset(cy, cx + 1, j0, k0, nt, np), bc, affine);
        l10 = ghost(h10, ub, ubo + slot_offset(cy + 1, cx, j0, k0, nt, np), bc, affine);
        l11 = ghost(h11, ub, ubo + slot_offset(cy + 1, cx + 1, j0, k0, nt, np), bc, affine);
    } else if (gside == 2) {
        l00 = lo[s00]; l01 = lo[s01]; l10 = lo[s10]; l11 = lo[s11];
        h00 = ghost(l00, ub, ubo + slot_offset(cy, cx, j0, k0, nt, np), bc, affine);
        h01 = ghost(l01, ub, ubo + slot_offset(cy, cx + 1, j0, k0, nt, np), bc, affine);
        h10 = ghost(l10, ub, ubo + slot_offset(cy + 1, cx, j0, k0, nt, np), bc, affine);
        h11 = ghost(l11, ub, ubo + slot_offset(cy + 1, cx + 1, j0, k0, nt, np), bc, affine);
    } else {
        l00 = lo[s00]; l01 = lo[s01]; l10 = lo[s10]; l11 = lo[s11];
        h00 = hi[s00]; h01 = hi[s01]; h10 = hi[s10]; h11 = hi[s11];
    }
    const T qt = T(0.25);
    const T a00 = l00 + h00, a01 = l01 + h01, a10 = l10 + h10, a11 = l11 + h11;
    const T Dr = qt * ((h00 - l00) + (h01 - l01) + (h10 - l10) + (h11 - l11));
    const T Dt = qt * (a10 + a11 - a00 - a01);
    const T Dp = qt * (a01 + a11 - a00 - a10);
    return er * Dr + et * Dt + ep * Dp;
}

template <class T, int MODE, bool VIRT>
__global__ __launch_bounds__(kBlock) void k_aligned(Geo<T> g, KArgs<T> a)
{
    __shared__ T su[3][HN];                        // cell planes (ring of three levels)
    __shared__ T sr[NCOR], sth[NCOR], sph[NCOR];   // t e_r, t e_t, t e_p per tile corner
    const int L = xcd_tile();
    if (L >= a.nbx * a.nrc * a.nc) return;
    if (a.done && *a.done) return;
    const int np = g.np, nt = g.nt, nr = g.nr, P = g.P;
    const int ntk = (np + TX - 1) / TX;
    const int bx = L % a.nbx, rest = L / a.nbx, rc = rest % a.nrc, c = rest / a.nrc;
    const TileMap tm = tile_map(bx % ntk, bx / ntk, nt, np);
    const size_t cb = (size_t)c * nr * P;
    const T* u = a.u + cb;
    const T* y = VIRT ? a.y0 + cb : nullptr;
    const size_t ubo = (size_t)c * P;
    const size_t nco = (size_t)(nr + 1) * (nt + 1) * np;
    const int i0 = a.r_lo + rc * a.rch;
    const int i1 = min(a.r_hi, i0 + a.rch);
    const int j = min(tm.j, nt - 1), k = tm.valid ? tm.k : 0;
    const T vtj = g.vt[j], vpk = g.vp[k];
    const int t = threadIdx.x;
    // the thread's corners of a tile plane: t and t + 256 (< NCOR); corner
    // rows beyond the last pole row read the (zero) pole row
    const bool has_c1 = t + kBlock < NCOR;
    const int ci1 = has_c1 ? t + kBlock : t;
    const int cy0 = t / CX, cx0 = t % CX, cy1 = ci1 / CX, cx1 = ci1 % CX;
    const int cq0 = min(tm.j0 + cy0, nt) * np + wrapk(tm.k0 + cx0, np);
    const int cq1 = min(tm.j0 + cy1, nt) * np + wrapk(tm.k0 + cx1, np);
    // the own cell's corners A (ty, tx), B (ty, tx+1), C (ty+1, tx), D (ty+1, tx+1)
    const int cA = tm.ty * CX + tm.tx;
    Acc<T, MODE> acc;
    // ring R[q] = loads of corner plane ic + q; plane ic + DEPTH is issued
    // while plane ic is computed
    constexpr int DEPTH = 2;
    LevA<T> R[DEPTH + 1] = {};
    T carry = 0;
    if (i0 < i1) {
        if (i0 > 0) {
            const size_t lb = (size_t)(i0 - 1) * P;
            su[(i0 - 1) % 3][tm.own_slot] = ldu<T, VIRT>(a, u, y, lb + tm.own_off);
            if (tm.has_h) su[(i0 - 1) % 3][tm.h_slot] = ldu<T, VIRT>(a, u, y, lb + tm.h_off);
        }
#pragma unroll
        for (int q = 0; q < DEPTH; ++q)
            if (i0 + q <= i1)
                fetchA<T, MODE, VIRT>(a, u, y, tm, cb, P, nr, nt, np, nco, i0 + q, i0, i1, cq0, cq1,
                                      has_c1, R[q]);
    }
    // corner plane ic completes cell level ic-1 and starts level ic
    for (int ic = i0; ic <= i1 && i0 < i1; ++ic) {
        const int bh = ic % 3, bl = (ic + 2) % 3;
        const LevA<T>& R0 = R[0];
        if (ic < nr) {
            su[bh][tm.own_slot] = R0.u;
            if (tm.has_h) su[bh][tm.h_slot] = R0.h;
        }
        if (ic + DEPTH <= i1)
            fetchA<T, MODE, VIRT>(a, u, y, tm, cb, P, nr, nt, np, nco, ic + DEPTH, i0, i1, cq0, cq1,
                                  has_c1, R[DEPTH]);
        __syncthreads();
        int kind = 0, gside = 0, bc = 0;
        const T* ub = nullptr;
        if (ic == 0) { kind = 1; gside = 1; bc = a.bc_in; ub = a.ub_in; }
        else if (ic == nr) { kind = 2; gside = 2; bc = a.bc_out; ub = a.ub_out; }
        const T* lo = su[bl];
        const T* hi = su[bh];
        {
            const T f0 = corner_flux<T>(lo, hi, cy0, cx0, R0.e0r, R0.e0t, R0.e0p, gside, ub, bc,
                                        a.affine, ubo, tm.j0, tm.k0, nt, np);
            sr[t] = f0 * R0.e0r;
            sth[t] = f0 * R0.e0t;
            sph[t] = f0 * R0.e0p;
            if (has_c1) {
                const T f1 = corner_flux<T>(lo, hi, cy1, cx1, R0.e1r, R0.e1t, R0.e1p, gside, ub,
                                            bc, a.affine, ubo, tm.j0, tm.k0, nt, np);
                sr[ci1] = f1 * R0.e1r;
                sth[ci1] = f1 * R0.e1t;
                sph[ci1] = f1 * R0.e1p;
            }
        }
        __syncthreads();
        const PlaneW<T> w = plane_weights<T>(kind, bc);
        T up = 0, dn = 0;
        {
            // A: st=+1 sp=+1; B: st=+1 sp=-1; C: st=-1 sp=+1; D: st=-1 sp=-1
            const T tA = sth[cA] + sph[cA];
            const T tB = sth[cA + 1] - sph[cA + 1];
            const T tC = -sth[cA + CX] + sph[cA + CX];
            const T tD = -sth[cA + CX + 1] - sph[cA + CX + 1];
            const T rA = sr[cA], rB = sr[cA + 1], rC = sr[cA + CX], rD = sr[cA + CX + 1];
            up = w.ru * rA + w.tu * tA;
            up += w.ru * rB + w.tu * tB;
            up += w.ru * rC + w.tu * tC;
            up += w.ru * rD + w.tu * tD;
            dn = w.rd * rA + w.td * tA;
            dn += w.rd * rB + w.td * tB;
            dn += w.rd * rC + w.td * tC;
            dn += w.rd * rD + w.td * tD;
        }
        if (ic - 1 >= i0) {
            const int i = ic - 1;
            const T Lu = carry + dn;
            const T V = g.vr[i] * vtj * vpk;
            const T uc = lo[tm.own_slot];
            if (tm.valid) epilogue<T, MODE>(a, cb + (size_t)i * P + tm.own_off, Lu, V, uc, R0.s, acc);
        }
        carry = up;
#pragma unroll
        for (int q = 0; q < DEPTH; ++q) R[q] = R[q + 1];
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

}  // namespace pa
