// pa_kernels.hip -- stencil kernels of the parabolic operator F(u) on the
// spherical shell (gfx950), fused with what consumes F on the hot path:
//   kApply  F = F(u)                                   (operator apply)
//   kFirst  y0 = F(u0) + per-tile argmax |F|           (PTL pass, Eq. ptl3)
//   kStage  u_k = mu u_{k-1} + nu u_{k-2} + (1-mu-nu) u0
//                 + mu~ dt F(u_{k-1}) + gamma~ dt y0     (STS stage, App. A)
//   kMatvec q = V p + dt L p, per-tile <p, q>          (BE system matvec)
//
// Work decomposition (field-aligned operator, and the 7-point operator in
// FP64; the FP32 7-point form marches wave rows, described at its kernel).
// A workgroup of 256 threads owns a 32 (phi) x 8 (theta) tile of cells and
// marches over a chunk of radial levels.  Each
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
static_assert(TX * TY == kBlock, "a tile is one workgroup's cells");

__device__ __forceinline__ int xcd_tile()
{
    const int per = gridDim.x >> 3;  // grid is a multiple of 8
    return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

static inline int grid_for_tiles(int ntiles) { return ((ntiles + 7) / 8) * 8; }

int tiles_per_plane(int nt, int np) { return ((np + TX - 1) / TX) * ((nt + TY - 1) / TY); }

int iso7_blocks_per_plane(int nt, int np, bool fp32);

int blocks_per_plane(int op, int nt, int np, bool fp32)
{
    return op == kOpIso7 ? iso7_blocks_per_plane(nt, np, fp32) : tiles_per_plane(nt, np);
}

// the vector viscosity kernel treats the three components in one workgroup
int stencil_tiles(int op, int nt, int np, int nlev, int rch, int nc, bool fp32)
{
    const int nrc = (nlev + rch - 1) / rch;
    return blocks_per_plane(op, nt, np, fp32) * nrc * (op == kOpViscVec ? 1 : nc);
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

__device__ __forceinline__ TileMap tile_map(int bxk, int bxj, int nt, int np, int t)
{
    TileMap m;
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
        // kFirst with out == null: the argmax partials only
        if (MODE == kApply || a.out) __builtin_nontemporal_store(F, a.out + m);
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

template <class T, int MODE, int NTHREADS = kBlock>
__device__ void finish(const KArgs<T>& a, int L, Acc<T, MODE>& acc)
{
    __shared__ double ldsv[NTHREADS / 64];
    __shared__ long long ldsi[NTHREADS / 64];
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
//
// Wave rows (the FP32 form): each wave owns 64 consecutive cells of a radial level (phi
// fastest, rows of theta following) and marches them over a chunk of
// levels; the four in-plane neighbours are read straight from the caches
// (neighbouring waves load them as their own cells), the radial neighbours
// come from a register ring filled two levels ahead.  No LDS and no
// barriers in the march, so every wave streams independently.  With a
// variable coefficient (CV) the ring also carries the coefficient at the
// five in-plane points.

constexpr int W7 = 4;        // waves per workgroup
constexpr int RCH_MAX = 32;  // radial levels per workgroup (at most)

// 7-point march form: 32 x 8 tiles staging each level in LDS for FP64
// (measured on the 151x301x400 viscosity operator: matvec 213 against 296 us,
// stage 406 against 474 us), wave rows reading the in-plane neighbours
// through the caches for FP32 (10% faster there than the tiles)
template <class T>
constexpr bool iso7_tiled() { return sizeof(T) == 8; }

int iso7_blocks_per_plane(int nt, int np, bool fp32)
{
    if (fp32 ? iso7_tiled<float>() : iso7_tiled<double>()) return tiles_per_plane(nt, np);
    const int nseg = (nt * np + 63) / 64;
    return (nseg + W7 - 1) / W7;
}

template <class T, bool CV, int MODE>
struct Lev7 {
    T x, w, e, s, n;                  // u at own, phi-, phi+, theta-, theta+
    T cx, cw, ce, cs, cn;             // coefficient at the same points (CV)
    T wt;                             // cell weight of the own cell (WT)
    Streams<T> st;                    // stage streams of the own cell
};

template <class T, bool CV, int MODE, bool VIRT, bool WT>
__device__ __forceinline__ void fetch7(const KArgs<T>& a, const T* u, const T* y, size_t lb,
                                       unsigned pp, unsigned ow, unsigned oe, unsigned os,
                                       unsigned on, size_t sb, Lev7<T, CV, MODE>& R)
{
    R.x = ldu<T, VIRT>(a, u, y, lb + pp);
    if constexpr (WT) R.wt = a.wgt[lb + pp];
    R.w = ldu<T, VIRT>(a, u, y, lb + ow);
    R.e = ldu<T, VIRT>(a, u, y, lb + oe);
    R.s = ldu<T, VIRT>(a, u, y, lb + os);
    R.n = ldu<T, VIRT>(a, u, y, lb + on);
    if constexpr (CV) {
        R.cx = a.coef[lb + pp];
        R.cw = a.coef[lb + ow];
        R.ce = a.coef[lb + oe];
        R.cs = a.coef[lb + os];
        R.cn = a.coef[lb + on];
    }
    load_streams<T, MODE>(a, sb, R.st);
}

// per-thread constants of the 7-point march
template <class T>
struct Pt7 {
    unsigned pp, ow, oe, os, on;
    bool valid;
    T Ar, As, An, Aw, Ae;   // vt vp, gtt vp (theta- / theta+), gpt gpp (phi- / phi+)
    T ubl, ubu;             // mirror data below level 0 / above level nr-1
    T fin, fout;            // 1 for a Dirichlet face at r_in / r_out, else 0
};

// One level i of the march: issue the loads of level i + 2 into Rp
// (clamped to the mesh and the chunk; values of levels past the chunk are
// never used), then combine level i from Rc (own and in-plane values) and
// Rn (the level above).  Levels at or past i1 are computed but not stored:
// the body has no data-dependent branches, and with the ring's roles
// rotating between calls no register copy waits on a load in flight.
template <class T, int MODE, bool VIRT, bool CV, bool WT>
__device__ __forceinline__ void step7(const Geo<T>& g, const KArgs<T>& a, const T* u, const T* y,
                                      size_t cb, const Pt7<T>& t, int i, int i0, int i1,
                                      const T* lgr, const T* lgtr, const T* lvr,
                                      const Lev7<T, CV, MODE>& Rc, const Lev7<T, CV, MODE>& Rn,
                                      Lev7<T, CV, MODE>& Rp, T& um, T& cm, Acc<T, MODE>& acc)
{
    const int nr = g.nr;
    const size_t P = (size_t)g.P;
    {
        const int lv = min(i + 2, nr - 1), ls = min(i + 2, i1 - 1);
        fetch7<T, CV, MODE, VIRT, WT>(a, u, y, (size_t)lv * P, t.pp, t.ow, t.oe, t.os, t.on,
                                      cb + (size_t)ls * P + t.pp, Rp);
    }
    const int ic = min(i, nr - 1);
    const T half = T(0.5);
    const T uc = Rc.x;
    const T cc = CV ? Rc.cx : a.cs;
    const T cs_ = CV ? Rc.cs : a.cs, cn = CV ? Rc.cn : a.cs;
    const T cw = CV ? Rc.cw : a.cs, ce = CV ? Rc.ce : a.cs;
    const T cu = CV ? Rn.cx : a.cs;
    const int il = ic - i0;
    const T gtri = lgtr[il];
    const bool lo = ic > 0, hi = ic < nr - 1;
    const T Cl = lo ? half * (cc + cm) * (lgr[il] * t.Ar) : t.fin * cc * (lgr[il] * t.Ar);
    const T ul = lo ? um : t.ubl;
    const T Cu = hi ? half * (cc + cu) * (lgr[il + 1] * t.Ar) : t.fout * cc * (lgr[il + 1] * t.Ar);
    const T uu = hi ? Rn.x : t.ubu;
    T Lu = Cl * (uc - ul);
    Lu += Cu * (uc - uu);
    Lu += half * (cc + cs_) * (gtri * t.As) * (uc - Rc.s);
    Lu += half * (cc + cn) * (gtri * t.An) * (uc - Rc.n);
    Lu += half * (cc + cw) * (gtri * t.Aw) * (uc - Rc.w);
    Lu += half * (cc + ce) * (gtri * t.Ae) * (uc - Rc.e);
    const T V = WT ? lvr[il] * t.Ar * Rc.wt : lvr[il] * t.Ar;  // (w) V
    if (t.valid && i < i1) epilogue<T, MODE>(a, cb + (size_t)ic * P + t.pp, Lu, V, uc, Rc.st, acc);
    um = uc;
    cm = cc;
}

template <class T, int MODE, bool VIRT, bool CV, bool WT>
__global__ __launch_bounds__(64 * W7) void k_iso7(Geo<T> g, KArgs<T> a)
{
    const int L = xcd_tile();
    if (L >= a.nbx * a.nrc * a.nc) return;
    if (a.done && *a.done) return;
    const int nt = g.nt, np = g.np, nr = g.nr;
    const unsigned P = (unsigned)g.P;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int bx = L % a.nbx, rest = L / a.nbx, rc = rest % a.nrc, c = rest / a.nrc;
    Pt7<T> t;
    unsigned pp = (unsigned)(bx * W7 + wv) * 64u + (unsigned)lane;
    t.valid = pp < P;
    if (!t.valid) pp = P - 1;
    const unsigned j = pp / (unsigned)np, k = pp - j * (unsigned)np;
    const unsigned kp = (k == (unsigned)np - 1) ? 0u : k + 1;
    // in-plane neighbour offsets: phi wraps; at the poles the missing row is
    // replaced by the cell itself (its coupling is zero)
    t.pp = pp;
    t.ow = (k == 0) ? pp + np - 1 : pp - 1;
    t.oe = pp - k + kp;
    t.os = (j > 0) ? pp - np : pp;
    t.on = (j + 1 < (unsigned)nt) ? pp + np : pp;
    // per-cell metric products; the level factors gr, gtr, vr are uniform
    t.Ar = g.vt[j] * g.vp[k];
    t.As = g.gtt[j] * g.vp[k];
    t.An = g.gtt[j + 1] * g.vp[k];
    t.Aw = g.gpt[j] * g.gpp[k];
    t.Ae = g.gpt[j] * g.gpp[kp];
    const size_t cb = (size_t)c * nr * P;
    const T* u = a.u + cb;
    const T* y = VIRT ? a.y0 + cb : nullptr;
    const int i0 = a.r_lo + rc * a.rch;
    const int i1 = min(a.r_hi, i0 + a.rch);
    const size_t ob = (size_t)c * P + pp;  // boundary data of the own cell
    // mirror data across the radial boundaries (zero in linear mode); a
    // Dirichlet face couples to it at half distance (gr[0], gr[nr]), a
    // no-flux face is dropped
    t.ubl = (a.affine && i0 == 0) ? a.ub_in[ob] : T(0);
    t.ubu = (a.affine && i1 == nr) ? a.ub_out[ob] : T(0);
    t.fin = (a.bc_in == 0) ? T(1) : T(0);
    t.fout = (a.bc_out == 0) ? T(1) : T(0);
    // the chunk's level factors gr (faces i0..), gtr, vr, staged in LDS: read
    // there, they do not share the vector-memory counter with the prefetch
    __shared__ T lgr[RCH_MAX + 3], lgtr[RCH_MAX + 3], lvr[RCH_MAX + 3];
    for (int q = threadIdx.x; q < RCH_MAX + 3; q += blockDim.x) {
        const int lv = min(i0 + q, nr - 1);
        lgr[q] = g.gr[min(i0 + q, nr)];
        lgtr[q] = g.gtr[lv];
        lvr[q] = g.vr[lv];
    }
    __syncthreads();
    Acc<T, MODE> acc;
    if (i0 < i1) {
        Lev7<T, CV, MODE> R0, R1, R2;
        T um = 0, cm = a.cs;
        if (i0 > 0) {
            um = ldu<T, VIRT>(a, u, y, (size_t)(i0 - 1) * P + pp);
            if constexpr (CV) cm = a.coef[(size_t)(i0 - 1) * P + pp];
        }
        fetch7<T, CV, MODE, VIRT, WT>(a, u, y, (size_t)i0 * P, t.pp, t.ow, t.oe, t.os, t.on,
                                      cb + (size_t)i0 * P + pp, R0);
        {
            const int lv = min(i0 + 1, nr - 1), ls = min(i0 + 1, i1 - 1);
            fetch7<T, CV, MODE, VIRT, WT>(a, u, y, (size_t)lv * P, t.pp, t.ow, t.oe, t.os, t.on,
                                          cb + (size_t)ls * P + pp, R1);
        }
        // three levels per trip with the ring's roles rotating
        for (int i = i0; i < i1; i += 3) {
            step7<T, MODE, VIRT, CV, WT>(g, a, u, y, cb, t, i, i0, i1, lgr, lgtr, lvr, R0, R1, R2,
                                         um, cm, acc);
            step7<T, MODE, VIRT, CV, WT>(g, a, u, y, cb, t, i + 1, i0, i1, lgr, lgtr, lvr, R1, R2,
                                         R0, um, cm, acc);
            step7<T, MODE, VIRT, CV, WT>(g, a, u, y, cb, t, i + 2, i0, i1, lgr, lgtr, lvr, R2, R0,
                                         R1, um, cm, acc);
        }
    }
    finish<T, MODE>(a, L, acc);
}

// ------------------------------------------------------------ 7-point, tiled
//
// Tiles of 32 (phi) x 8 (theta) cells march a radial chunk.  Each level's
// tile plane with its one-cell halo ring is staged in LDS (double
// buffered, one barrier per level); the four in-plane neighbours are read
// there, the radial ones come from the register ring (the own column,
// loaded three levels ahead) and the previous level's carried value.  A
// thread loads its own cell and, for 84 threads, one halo cell (the others
// load a duplicate), so a level costs two loads per thread.

template <class T, bool CV, int MODE, bool WT>
struct LevT {
    T x, h;           // own and halo cell
    T cx, ch;         // coefficient at the same cells (CV)
    T wt;             // cell weight of the own cell (WT)
    Streams<T> st;    // stage streams of the own cell
};

template <class T, bool CV, int MODE, bool VIRT, bool WT>
__device__ __forceinline__ void fetchT(const KArgs<T>& a, const T* u, const T* y, const TileMap& tm,
                                       size_t lb, size_t sb, LevT<T, CV, MODE, WT>& R)
{
    R.x = ldu<T, VIRT>(a, u, y, lb + tm.own_off);
    R.h = ldu<T, VIRT>(a, u, y, lb + tm.h_off);
    if constexpr (CV) {
        R.cx = a.coef[lb + tm.own_off];
        R.ch = a.coef[lb + tm.h_off];
    }
    if constexpr (WT) R.wt = a.wgt[lb + tm.own_off];
    load_streams<T, MODE>(a, sb, R.st);
}

template <class T>
struct ShT {
    T su[2][HN];
    T sc[2][HN];
    T gr[RCH_MAX + 3], gtr[RCH_MAX + 3], vr[RCH_MAX + 3];
};

template <class T, int MODE, bool VIRT, bool CV, bool WT, int DEPTH>
__device__ __forceinline__ void stepT(const Geo<T>& g, const KArgs<T>& a, const T* u, const T* y,
                                      size_t cb, const TileMap& tm, const Pt7<T>& t, ShT<T>& sh,
                                      int i, int i0, int i1,
                                      const LevT<T, CV, MODE, WT>& Rc,
                                      const LevT<T, CV, MODE, WT>& Rn,
                                      LevT<T, CV, MODE, WT>& Rp, T& um, T& cm, Acc<T, MODE>& acc)
{
    const int nr = g.nr;
    const size_t P = (size_t)g.P;
    const int b = i & 1;
    sh.su[b][tm.own_slot] = Rc.x;
    if (tm.has_h) sh.su[b][tm.h_slot] = Rc.h;
    if constexpr (CV) {
        sh.sc[b][tm.own_slot] = Rc.cx;
        if (tm.has_h) sh.sc[b][tm.h_slot] = Rc.ch;
    }
    {
        const int lv = min(i + DEPTH, nr - 1), ls = min(i + DEPTH, i1 - 1);
        fetchT<T, CV, MODE, VIRT, WT>(a, u, y, tm, (size_t)lv * P, cb + (size_t)ls * P + tm.own_off,
                                      Rp);
    }
    __syncthreads();
    const int o = tm.own_slot;
    const T* su = sh.su[b];
    const T uc = Rc.x;
    const T uw = su[o - 1], ue = su[o + 1], us = su[o - HX], un = su[o + HX];
    const T cc = CV ? Rc.cx : a.cs;
    T cw = a.cs, ce = a.cs, cs_ = a.cs, cn = a.cs;
    if constexpr (CV) {
        const T* sc = sh.sc[b];
        cw = sc[o - 1];
        ce = sc[o + 1];
        cs_ = sc[o - HX];
        cn = sc[o + HX];
    }
    const T cu = CV ? Rn.cx : a.cs;
    const int ic = min(i, nr - 1);
    const T half = T(0.5);
    const int il = ic - i0;
    const T gtri = sh.gtr[il];
    const bool lo = ic > 0, hi = ic < nr - 1;
    const T Cl = lo ? half * (cc + cm) * (sh.gr[il] * t.Ar) : t.fin * cc * (sh.gr[il] * t.Ar);
    const T ul = lo ? um : t.ubl;
    const T Cu = hi ? half * (cc + cu) * (sh.gr[il + 1] * t.Ar) : t.fout * cc * (sh.gr[il + 1] * t.Ar);
    const T uu = hi ? Rn.x : t.ubu;
    T Lu = Cl * (uc - ul);
    Lu += Cu * (uc - uu);
    if constexpr (CV) {
        Lu += half * (cc + cs_) * (gtri * t.As) * (uc - us);
        Lu += half * (cc + cn) * (gtri * t.An) * (uc - un);
        Lu += half * (cc + cw) * (gtri * t.Aw) * (uc - uw);
        Lu += half * (cc + ce) * (gtri * t.Ae) * (uc - ue);
    } else {
        // one coefficient for the four in-plane faces: factored out
        T inp = t.As * (uc - us);
        inp += t.An * (uc - un);
        inp += t.Aw * (uc - uw);
        inp += t.Ae * (uc - ue);
        Lu += (a.cs * gtri) * inp;
    }
    const T V = WT ? sh.vr[il] * t.Ar * Rc.wt : sh.vr[il] * t.Ar;  // (w) V
    if (t.valid && i < i1) epilogue<T, MODE>(a, cb + (size_t)ic * P + tm.own_off, Lu, V, uc, Rc.st, acc);
    um = uc;
    cm = cc;
}

template <class T, int MODE, bool VIRT, bool CV, bool WT>
__global__ __launch_bounds__(kBlock) void k_iso7t(Geo<T> g, KArgs<T> a)
{
    __shared__ ShT<T> sh;
    const int L = xcd_tile();
    if (L >= a.nbx * a.nrc * a.nc) return;
    if (a.done && *a.done) return;
    const int nt = g.nt, np = g.np, nr = g.nr;
    const size_t P = (size_t)g.P;
    const int ntk = (np + TX - 1) / TX;
    const int bx = L % a.nbx, rest = L / a.nbx, rc = rest % a.nrc, c = rest / a.nrc;
    const TileMap tm = tile_map(bx % ntk, bx / ntk, nt, np, threadIdx.x);
    Pt7<T> t;
    t.valid = tm.valid;
    const int j = min(tm.j, nt - 1), k = tm.valid ? tm.k : 0;
    const int kp = (k == np - 1) ? 0 : k + 1;
    // per-cell metric products (the missing row at a pole has zero coupling)
    t.Ar = g.vt[j] * g.vp[k];
    t.As = g.gtt[j] * g.vp[k];
    t.An = g.gtt[j + 1] * g.vp[k];
    t.Aw = g.gpt[j] * g.gpp[k];
    t.Ae = g.gpt[j] * g.gpp[kp];
    const size_t cb = (size_t)c * nr * P;
    const T* u = a.u + cb;
    const T* y = VIRT ? a.y0 + cb : nullptr;
    const int i0 = a.r_lo + rc * a.rch;
    const int i1 = min(a.r_hi, i0 + a.rch);
    const size_t ob = (size_t)c * P + tm.own_off;
    t.ubl = (a.affine && i0 == 0) ? a.ub_in[ob] : T(0);
    t.ubu = (a.affine && i1 == nr) ? a.ub_out[ob] : T(0);
    t.fin = (a.bc_in == 0) ? T(1) : T(0);
    t.fout = (a.bc_out == 0) ? T(1) : T(0);
    for (int q = threadIdx.x; q < RCH_MAX + 3; q += blockDim.x) {
        const int lv = min(i0 + q, nr - 1);
        sh.gr[q] = g.gr[min(i0 + q, nr)];
        sh.gtr[q] = g.gtr[lv];
        sh.vr[q] = g.vr[lv];
    }
    Acc<T, MODE> acc;
    if (i0 < i1) {
        LevT<T, CV, MODE, WT> R0, R1, R2;
        T um = 0, cm = a.cs;
        if (i0 > 0) {
            um = ldu<T, VIRT>(a, u, y, (size_t)(i0 - 1) * P + tm.own_off);
            if constexpr (CV) cm = a.coef[(size_t)(i0 - 1) * P + tm.own_off];
        }
        fetchT<T, CV, MODE, VIRT, WT>(a, u, y, tm, (size_t)i0 * P, cb + (size_t)i0 * P + tm.own_off,
                                      R0);
        {
            const int lv = min(i0 + 1, nr - 1), ls = min(i0 + 1, i1 - 1);
            fetchT<T, CV, MODE, VIRT, WT>(a, u, y, tm, (size_t)lv * P,
                                          cb + (size_t)ls * P + tm.own_off, R1);
        }
        // loads three levels ahead (a level costs two values per thread):
        // four levels per trip with the ring's roles rotating
        LevT<T, CV, MODE, WT> R3;
        {
            const int lv = min(i0 + 2, nr - 1), ls = min(i0 + 2, i1 - 1);
            fetchT<T, CV, MODE, VIRT, WT>(a, u, y, tm, (size_t)lv * P,
                                          cb + (size_t)ls * P + tm.own_off, R2);
        }
        for (int i = i0; i < i1; i += 4) {
            stepT<T, MODE, VIRT, CV, WT, 3>(g, a, u, y, cb, tm, t, sh, i, i0, i1, R0, R1, R3,
                                            um, cm, acc);
            stepT<T, MODE, VIRT, CV, WT, 3>(g, a, u, y, cb, tm, t, sh, i + 1, i0, i1, R1, R2,
                                            R0, um, cm, acc);
            stepT<T, MODE, VIRT, CV, WT, 3>(g, a, u, y, cb, tm, t, sh, i + 2, i0, i1, R2, R3,
                                            R1, um, cm, acc);
            stepT<T, MODE, VIRT, CV, WT, 3>(g, a, u, y, cb, tm, t, sh, i + 3, i0, i1, R3, R0,
                                            R2, um, cm, acc);
        }
    }
    finish<T, MODE>(a, L, acc);
}

// ------------------------------------------------------------ field-aligned

// one corner plane ic's loads of a thread: its own / halo cell of level ic,
// the coefficients of corners t and t + 256, and the stage streams of the
// own cell at level ic - 1 (the level that plane completes).  Indices are
// clamped to the mesh and the chunk, so the loads are unconditional (a
// thread without a halo cell or a second corner loads a duplicate); values
// loaded for planes past the chunk are never used.
template <class T>
struct LevA {
    T u, h;
    T e0r, e0t, e0p, e1r, e1t, e1p;
    T wt;  // cell weight of the own cell at level ic - 1 (WT)
    Streams<T> s;
};

template <class T, int MODE, bool VIRT, bool WT>
__device__ __forceinline__ void fetchA(const KArgs<T>& a, const T* u, const T* y, const TileMap& tm,
                                       size_t cb, int P, int nr, int nt, int np, size_t nco,
                                       int ic, int i0, int i1, int cq0, int cq1, LevA<T>& R)
{
    const size_t lb = (size_t)min(ic, nr - 1) * P;
    R.u = ldu<T, VIRT>(a, u, y, lb + tm.own_off);
    R.h = ldu<T, VIRT>(a, u, y, lb + tm.h_off);
    const size_t qb = (size_t)min(ic, nr) * (nt + 1) * np;
    R.e0r = a.e[qb + cq0];
    R.e0t = a.e[nco + qb + cq0];
    R.e0p = a.e[2 * nco + qb + cq0];
    R.e1r = a.e[qb + cq1];
    R.e1t = a.e[nco + qb + cq1];
    R.e1p = a.e[2 * nco + qb + cq1];
    const int ls = min(max(ic - 1, i0), i1 - 1);
    load_streams<T, MODE>(a, cb + (size_t)ls * P + tm.own_off, R.s);
    if constexpr (WT) R.wt = a.wgt[(size_t)ls * P + tm.own_off];
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

// mirror ghost across a radial boundary: Dirichlet 2 u_b - u (u_b is the
// staged boundary value, 0 in linear mode), no-flux u
template <class T>
__device__ __forceinline__ T ghost(T x, T b, int bc)
{
    return bc != 0 ? x : T(2) * b - x;
}

// flux t = e . D of tile corner (cy, cx) between the LDS planes lo and hi;
// gside 1: lo is the mirror ghost of hi, 2: hi is the ghost of lo, with the
// boundary values of the tile plane in ubp (LDS)
template <class T>
__device__ __forceinline__ T corner_flux(const T* lo, const T* hi, int cy, int cx, T er, T et,
                                         T ep, int gside, const T* ubp, int bc)
{
    const int s00 = cy * HX + cx, s01 = s00 + 1, s10 = s00 + HX, s11 = s10 + 1;
    T l00, l01, l10, l11, h00, h01, h10, h11;
    if (gside == 1) {
        h00 = hi[s00]; h01 = hi[s01]; h10 = hi[s10]; h11 = hi[s11];
        l00 = ghost(h00, ubp[s00], bc);
        l01 = ghost(h01, ubp[s01], bc);
        l10 = ghost(h10, ubp[s10], bc);
        l11 = ghost(h11, ubp[s11], bc);
    } else if (gside == 2) {
        l00 = lo[s00]; l01 = lo[s01]; l10 = lo[s10]; l11 = lo[s11];
        h00 = ghost(l00, ubp[s00], bc);
        h01 = ghost(l01, ubp[s01], bc);
        h10 = ghost(l10, ubp[s10], bc);
        h11 = ghost(l11, ubp[s11], bc);
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

// LDS of the field-aligned march
template <class T>
struct ShA {
    T su[3][HN];                       // cell planes (ring of three levels)
    T sr[NCOR], sth[NCOR], sph[NCOR];  // t e_r, t e_t, t e_p per tile corner
    T ubi[HN], ubo[HN];                // boundary data of the tile plane (r_in, r_out)
    T vr[RCH_MAX + 3];                 // chunk level factors
};

// per-thread constants of the field-aligned march
struct PtA {
    int t, ci1, cy0, cx0, cy1, cx1, cq0, cq1, cA;
    bool has_c1;
};

// Corner plane ic: store its cell level into the LDS ring, issue the loads
// of plane ic + 2 into Rp, compute the plane's corner fluxes, gather the
// upper share into carry and complete level ic - 1.  Planes past i1 are
// computed but complete nothing.
template <class T, int MODE, bool VIRT, bool WT>
__device__ __forceinline__ void stepA(const Geo<T>& g, const KArgs<T>& a, const T* u, const T* y,
                                      const TileMap& tm, const PtA& pt, ShA<T>& sh, size_t cb,
                                      size_t nco, T Ar, int ic, int i0, int i1,
                                      const LevA<T>& Rc, LevA<T>& Rp, T& carry, Acc<T, MODE>& acc)
{
    const int np = g.np, nt = g.nt, nr = g.nr, P = g.P;
    const int bh = ic % 3, bl = (ic + 2) % 3;
    if (ic < nr) {
        sh.su[bh][tm.own_slot] = Rc.u;
        if (tm.has_h) sh.su[bh][tm.h_slot] = Rc.h;
    }
    fetchA<T, MODE, VIRT, WT>(a, u, y, tm, cb, P, nr, nt, np, nco, ic + 2, i0, i1, pt.cq0, pt.cq1, Rp);
    __syncthreads();
    int kind = 0, gside = 0, bc = 0;
    const T* ubp = sh.ubi;
    if (ic == 0) { kind = 1; gside = 1; bc = a.bc_in; }
    else if (ic == nr) { kind = 2; gside = 2; bc = a.bc_out; ubp = sh.ubo; }
    const T* lo = sh.su[bl];
    const T* hi = sh.su[bh];
    {
        const T f0 = corner_flux<T>(lo, hi, pt.cy0, pt.cx0, Rc.e0r, Rc.e0t, Rc.e0p, gside, ubp, bc);
        sh.sr[pt.t] = f0 * Rc.e0r;
        sh.sth[pt.t] = f0 * Rc.e0t;
        sh.sph[pt.t] = f0 * Rc.e0p;
        if (pt.has_c1) {
            const T f1 = corner_flux<T>(lo, hi, pt.cy1, pt.cx1, Rc.e1r, Rc.e1t, Rc.e1p, gside, ubp, bc);
            sh.sr[pt.ci1] = f1 * Rc.e1r;
            sh.sth[pt.ci1] = f1 * Rc.e1t;
            sh.sph[pt.ci1] = f1 * Rc.e1p;
        }
    }
    __syncthreads();
    const PlaneW<T> w = plane_weights<T>(kind, bc);
    const int cA = pt.cA;
    // A: st=+1 sp=+1; B: st=+1 sp=-1; C: st=-1 sp=+1; D: st=-1 sp=-1
    const T tA = sh.sth[cA] + sh.sph[cA];
    const T tB = sh.sth[cA + 1] - sh.sph[cA + 1];
    const T tC = -sh.sth[cA + CX] + sh.sph[cA + CX];
    const T tD = -sh.sth[cA + CX + 1] - sh.sph[cA + CX + 1];
    const T rA = sh.sr[cA], rB = sh.sr[cA + 1], rC = sh.sr[cA + CX], rD = sh.sr[cA + CX + 1];
    T up = w.ru * rA + w.tu * tA;
    up += w.ru * rB + w.tu * tB;
    up += w.ru * rC + w.tu * tC;
    up += w.ru * rD + w.tu * tD;
    T dn = w.rd * rA + w.td * tA;
    dn += w.rd * rB + w.td * tB;
    dn += w.rd * rC + w.td * tC;
    dn += w.rd * rD + w.td * tD;
    const int i = ic - 1;
    if (i >= i0 && i < i1) {
        const T Lu = carry + dn;
        const T V = WT ? sh.vr[i - i0] * Ar * Rc.wt : sh.vr[i - i0] * Ar;  // (w) V
        const T uc = lo[tm.own_slot];
        if (tm.valid) epilogue<T, MODE>(a, cb + (size_t)i * P + tm.own_off, Lu, V, uc, Rc.s, acc);
    }
    carry = up;
}

template <class T, int MODE, bool VIRT, bool WT>
__global__ __launch_bounds__(kBlock) void k_aligned(Geo<T> g, KArgs<T> a)
{
    __shared__ ShA<T> sh;
    const int L = xcd_tile();
    if (L >= a.nbx * a.nrc * a.nc) return;
    if (a.done && *a.done) return;
    const int np = g.np, nt = g.nt, nr = g.nr, P = g.P;
    const int ntk = (np + TX - 1) / TX;
    const int bx = L % a.nbx, rest = L / a.nbx, rc = rest % a.nrc, c = rest / a.nrc;
    const TileMap tm = tile_map(bx % ntk, bx / ntk, nt, np, threadIdx.x);
    const size_t cb = (size_t)c * nr * P;
    const T* u = a.u + cb;
    const T* y = VIRT ? a.y0 + cb : nullptr;
    const size_t nco = (size_t)(nr + 1) * (nt + 1) * np;
    const int i0 = a.r_lo + rc * a.rch;
    const int i1 = min(a.r_hi, i0 + a.rch);
    const int j = min(tm.j, nt - 1), k = tm.valid ? tm.k : 0;
    const T Ar = g.vt[j] * g.vp[k];
    PtA pt;
    pt.t = threadIdx.x;
    // the thread's corners of a tile plane: t and t + 256 (< NCOR); corner
    // rows beyond the last pole row read the (zero) pole row
    pt.has_c1 = pt.t + kBlock < NCOR;
    pt.ci1 = pt.has_c1 ? pt.t + kBlock : pt.t;
    pt.cy0 = pt.t / CX;
    pt.cx0 = pt.t % CX;
    pt.cy1 = pt.ci1 / CX;
    pt.cx1 = pt.ci1 % CX;
    pt.cq0 = min(tm.j0 + pt.cy0, nt) * np + wrapk(tm.k0 + pt.cx0, np);
    pt.cq1 = min(tm.j0 + pt.cy1, nt) * np + wrapk(tm.k0 + pt.cx1, np);
    // the own cell's corners A (ty, tx), B (ty, tx+1), C (ty+1, tx), D (ty+1, tx+1)
    pt.cA = tm.ty * CX + tm.tx;
    // LDS staging: level factors of the chunk, the boundary data of the tile
    // plane (zero in linear mode), and the cell level below the chunk
    for (int q = threadIdx.x; q < RCH_MAX + 3; q += blockDim.x) sh.vr[q] = g.vr[min(i0 + q, nr - 1)];
    {
        const size_t ob = (size_t)c * P;
        const bool lin = !a.affine;
        sh.ubi[tm.own_slot] = (lin || i0 != 0) ? T(0) : a.ub_in[ob + tm.own_off];
        sh.ubo[tm.own_slot] = (lin || i1 != nr) ? T(0) : a.ub_out[ob + tm.own_off];
        if (tm.has_h) {
            sh.ubi[tm.h_slot] = (lin || i0 != 0) ? T(0) : a.ub_in[ob + tm.h_off];
            sh.ubo[tm.h_slot] = (lin || i1 != nr) ? T(0) : a.ub_out[ob + tm.h_off];
        }
    }
    Acc<T, MODE> acc;
    if (i0 < i1) {
        if (i0 > 0) {
            const size_t lb = (size_t)(i0 - 1) * P;
            sh.su[(i0 - 1) % 3][tm.own_slot] = ldu<T, VIRT>(a, u, y, lb + tm.own_off);
            if (tm.has_h) sh.su[(i0 - 1) % 3][tm.h_slot] = ldu<T, VIRT>(a, u, y, lb + tm.h_off);
        }
        LevA<T> R0, R1, R2;
        fetchA<T, MODE, VIRT, WT>(a, u, y, tm, cb, P, nr, nt, np, nco, i0, i0, i1, pt.cq0, pt.cq1, R0);
        fetchA<T, MODE, VIRT, WT>(a, u, y, tm, cb, P, nr, nt, np, nco, i0 + 1, i0, i1, pt.cq0, pt.cq1,
                                  R1);
        T carry = 0;
        // corner plane ic completes cell level ic-1 and starts level ic;
        // three planes per trip with the ring's roles rotating
        for (int ic = i0; ic <= i1; ic += 3) {
            stepA<T, MODE, VIRT, WT>(g, a, u, y, tm, pt, sh, cb, nco, Ar, ic, i0, i1, R0, R2, carry,
                                     acc);
            stepA<T, MODE, VIRT, WT>(g, a, u, y, tm, pt, sh, cb, nco, Ar, ic + 1, i0, i1, R1, R0,
                                     carry, acc);
            stepA<T, MODE, VIRT, WT>(g, a, u, y, tm, pt, sh, cb, nco, Ar, ic + 2, i0, i1, R2, R1,
                                     carry, acc);
        }
    }
    finish<T, MODE>(a, L, acc);
}


// ------------------------------------------------------------ vector viscosity
//
// Eq. (visc) for a velocity in spherical components (v_r, v_theta, v_phi):
// the 7-point operator on the Cartesian components, written in each cell's
// own spherical basis.  A colatitude or longitude face couples component a
// of the cell to w_a = sum_b T_ab v_b(nb), T_ab = e_a(cell) . e_b(nb) (the
// neighbour's vector in the cell's basis); radial faces and the radial
// boundary data share the cell's basis.  Colatitude neighbours differ by a
// rotation about phi-hat by the angle D between the centres,
//   rows (cos D, -sin D, 0), (sin D, cos D, 0), (0, 0, 1);
// longitude neighbours by a rotation about the polar axis by d, with
// s, c = sin, cos of the colatitude and q = 1 - cos d,
//   rows (1 - s^2 q, -s c q, -s sin d), (-s c q, 1 - c^2 q, -c sin d),
//        (s sin d, c sin d, 1 - q).
// Workgroups of 3 x 256 threads own a 32 x 8 tile for all three components
// (threads 256 a .. 256 a + 255 own component a, so the component is
// uniform per wave); each level's three tile planes with their halo rings
// are staged in LDS, where a thread reads its neighbours' three components.
// A thread's loads are those of the scalar 7-point tile march above.

constexpr int kVBlock = 3 * kBlock;

template <class T>
struct ShV {
    T su[2][3][HN];
    T sc[2][HN];
    T gr[RCH_MAX + 3], gtr[RCH_MAX + 3], vr[RCH_MAX + 3];
};

// row a of the change of basis for the faces theta-, theta+, phi-, phi+.
// A colatitude rotation (about phi-hat) leaves the phi component alone and
// mixes only r and theta, so its row has two entries, on components ta and
// tb (0 and 1 for a = 0, 1; 2 and 2 with weights 1, 0 for a = 2)
template <class T>
struct RowsV {
    T t[2][2];
    T q[2][3];
    int ta, tb;
};

template <class T>
__device__ __forceinline__ RowsV<T> rows_viscv(const Geo<T>& g, int a, int j, int k, int kp)
{
    RowsV<T> R;
    const int nt = g.nt, np = g.np;
    // colatitude faces j (neighbour j-1, angle -D_j) and j+1 (angle D_{j+1})
    const T ct[2] = {g.rtf[j], g.rtf[j + 1]};
    const T st[2] = {-g.rtf[nt + 1 + j], g.rtf[nt + 1 + j + 1]};
    R.ta = a == 2 ? 2 : 0;
    R.tb = a == 2 ? 2 : 1;
    for (int f = 0; f < 2; ++f) {
        R.t[f][0] = a == 0 ? ct[f] : a == 1 ? st[f] : T(1);
        R.t[f][1] = a == 0 ? -st[f] : a == 1 ? ct[f] : T(0);
    }
    // longitude faces k (neighbour k-1, angle -d_k) and kp (angle d_kp)
    const T s = g.rtc[j], c = g.rtc[nt + j];
    const T qd[2] = {g.rpf[k], g.rpf[kp]};
    const T sd[2] = {-g.rpf[np + k], g.rpf[np + kp]};
    for (int f = 0; f < 2; ++f) {
        const T q = qd[f], d = sd[f];
        R.q[f][0] = a == 0 ? T(1) - s * s * q : a == 1 ? -s * c * q : s * d;
        R.q[f][1] = a == 0 ? -s * c * q : a == 1 ? T(1) - c * c * q : c * d;
        R.q[f][2] = a == 0 ? -s * d : a == 1 ? -c * d : T(1) - q;
    }
    return R;
}

template <class T, int MODE, bool VIRT, bool CV, bool WT, int DEPTH>
__device__ __forceinline__ void stepV(const Geo<T>& g, const KArgs<T>& a, const T* u, const T* y,
                                      size_t cb, int comp, const TileMap& tm, const Pt7<T>& t,
                                      const RowsV<T>& Q, ShV<T>& sh, int i, int i0, int i1,
                                      const LevT<T, CV, MODE, WT>& Rc,
                                      const LevT<T, CV, MODE, WT>& Rn,
                                      LevT<T, CV, MODE, WT>& Rp, T& um, T& cm, Acc<T, MODE>& acc)
{
    const int nr = g.nr;
    const size_t P = (size_t)g.P;
    const int b = i & 1;
    sh.su[b][comp][tm.own_slot] = Rc.x;
    if (tm.has_h) sh.su[b][comp][tm.h_slot] = Rc.h;
    if constexpr (CV) {
        if (comp == 0) {
            sh.sc[b][tm.own_slot] = Rc.cx;
            if (tm.has_h) sh.sc[b][tm.h_slot] = Rc.ch;
        }
    }
    {
        const int lv = min(i + DEPTH, nr - 1), ls = min(i + DEPTH, i1 - 1);
        fetchT<T, CV, MODE, VIRT, WT>(a, u, y, tm, (size_t)lv * P, cb + (size_t)ls * P + tm.own_off,
                                      Rp);
    }
    __syncthreads();
    const int o = tm.own_slot;
    const T* s0 = sh.su[b][0];
    const T* s1 = sh.su[b][1];
    const T* s2 = sh.su[b][2];
    const T* sa = sh.su[b][Q.ta];
    const T* sb = sh.su[b][Q.tb];
    // the in-plane neighbours' vectors in this cell's basis, component comp
    const T us = Q.t[0][0] * sa[o - HX] + Q.t[0][1] * sb[o - HX];
    const T un = Q.t[1][0] * sa[o + HX] + Q.t[1][1] * sb[o + HX];
    const T uw = Q.q[0][0] * s0[o - 1] + Q.q[0][1] * s1[o - 1] + Q.q[0][2] * s2[o - 1];
    const T ue = Q.q[1][0] * s0[o + 1] + Q.q[1][1] * s1[o + 1] + Q.q[1][2] * s2[o + 1];
    const T uc = Rc.x;
    const T cc = CV ? Rc.cx : a.cs;
    T cw = a.cs, ce = a.cs, cs_ = a.cs, cn = a.cs;
    if constexpr (CV) {
        const T* sc = sh.sc[b];
        cw = sc[o - 1];
        ce = sc[o + 1];
        cs_ = sc[o - HX];
        cn = sc[o + HX];
    }
    const T cu = CV ? Rn.cx : a.cs;
    const int ic = min(i, nr - 1);
    const T half = T(0.5);
    const int il = ic - i0;
    const T gtri = sh.gtr[il];
    const bool lo = ic > 0, hi = ic < nr - 1;
    const T Cl = lo ? half * (cc + cm) * (sh.gr[il] * t.Ar) : t.fin * cc * (sh.gr[il] * t.Ar);
    const T ul = lo ? um : t.ubl;
    const T Cu = hi ? half * (cc + cu) * (sh.gr[il + 1] * t.Ar) : t.fout * cc * (sh.gr[il + 1] * t.Ar);
    const T uu = hi ? Rn.x : t.ubu;
    T Lu = Cl * (uc - ul);
    Lu += Cu * (uc - uu);
    if constexpr (CV) {
        Lu += half * (cc + cs_) * (gtri * t.As) * (uc - us);
        Lu += half * (cc + cn) * (gtri * t.An) * (uc - un);
        Lu += half * (cc + cw) * (gtri * t.Aw) * (uc - uw);
        Lu += half * (cc + ce) * (gtri * t.Ae) * (uc - ue);
    } else {
        // one coefficient for the four in-plane faces: factored out
        T inp = t.As * (uc - us);
        inp += t.An * (uc - un);
        inp += t.Aw * (uc - uw);
        inp += t.Ae * (uc - ue);
        Lu += (a.cs * gtri) * inp;
    }
    const T V = WT ? sh.vr[il] * t.Ar * Rc.wt : sh.vr[il] * t.Ar;  // (w) V
    if (t.valid && i < i1 && (a.only_c < 0 || a.only_c == comp))
        epilogue<T, MODE>(a, cb + (size_t)ic * P + tm.own_off, Lu, V, uc, Rc.st, acc);
    um = uc;
    cm = cc;
    // the next level overwrites the other LDS buffer; this one is reused two
    // levels on, after the next level's barrier
}

template <class T, int MODE, bool VIRT, bool CV, bool WT>
__global__ __launch_bounds__(kVBlock) void k_viscv(Geo<T> g, KArgs<T> a)
{
    __shared__ ShV<T> sh;
    const int L = xcd_tile();
    if (L >= a.nbx * a.nrc) return;
    if (a.done && *a.done) return;
    const int nt = g.nt, np = g.np, nr = g.nr;
    const size_t P = (size_t)g.P;
    const int ntk = (np + TX - 1) / TX;
    const int bx = L % a.nbx, rc = L / a.nbx;
    const int comp = threadIdx.x / kBlock;  // uniform per wave
    const TileMap tm = tile_map(bx % ntk, bx / ntk, nt, np, threadIdx.x % kBlock);
    Pt7<T> t;
    t.valid = tm.valid;
    const int j = min(tm.j, nt - 1), k = tm.valid ? tm.k : 0;
    const int kp = (k == np - 1) ? 0 : k + 1;
    t.Ar = g.vt[j] * g.vp[k];
    t.As = g.gtt[j] * g.vp[k];
    t.An = g.gtt[j + 1] * g.vp[k];
    t.Aw = g.gpt[j] * g.gpp[k];
    t.Ae = g.gpt[j] * g.gpp[kp];
    const RowsV<T> Q = rows_viscv<T>(g, comp, j, k, kp);
    const size_t cb = (size_t)comp * nr * P;
    const T* u = a.u + cb;
    const T* y = VIRT ? a.y0 + cb : nullptr;
    const int i0 = a.r_lo + rc * a.rch;
    const int i1 = min(a.r_hi, i0 + a.rch);
    const size_t ob = (size_t)comp * P + tm.own_off;
    t.ubl = (a.affine && i0 == 0) ? a.ub_in[ob] : T(0);
    t.ubu = (a.affine && i1 == nr) ? a.ub_out[ob] : T(0);
    t.fin = (a.bc_in == 0) ? T(1) : T(0);
    t.fout = (a.bc_out == 0) ? T(1) : T(0);
    for (int q = threadIdx.x; q < RCH_MAX + 3; q += blockDim.x) {
        const int lv = min(i0 + q, nr - 1);
        sh.gr[q] = g.gr[min(i0 + q, nr)];
        sh.gtr[q] = g.gtr[lv];
        sh.vr[q] = g.vr[lv];
    }
    Acc<T, MODE> acc;
    if (i0 < i1) {
        LevT<T, CV, MODE, WT> R0, R1, R2, R3;
        T um = 0, cm = a.cs;
        if (i0 > 0) {
            um = ldu<T, VIRT>(a, u, y, (size_t)(i0 - 1) * P + tm.own_off);
            if constexpr (CV) cm = a.coef[(size_t)(i0 - 1) * P + tm.own_off];
        }
        fetchT<T, CV, MODE, VIRT, WT>(a, u, y, tm, (size_t)i0 * P, cb + (size_t)i0 * P + tm.own_off,
                                      R0);
        {
            const int lv = min(i0 + 1, nr - 1), ls = min(i0 + 1, i1 - 1);
            fetchT<T, CV, MODE, VIRT, WT>(a, u, y, tm, (size_t)lv * P,
                                          cb + (size_t)ls * P + tm.own_off, R1);
        }
        {
            const int lv = min(i0 + 2, nr - 1), ls = min(i0 + 2, i1 - 1);
            fetchT<T, CV, MODE, VIRT, WT>(a, u, y, tm, (size_t)lv * P,
                                          cb + (size_t)ls * P + tm.own_off, R2);
        }
        // loads three levels ahead, four levels per trip with the ring's roles rotating
        for (int i = i0; i < i1; i += 4) {
            stepV<T, MODE, VIRT, CV, WT, 3>(g, a, u, y, cb, comp, tm, t, Q, sh, i, i0, i1, R0, R1,
                                            R3, um, cm, acc);
            stepV<T, MODE, VIRT, CV, WT, 3>(g, a, u, y, cb, comp, tm, t, Q, sh, i + 1, i0, i1, R1,
                                            R2, R0, um, cm, acc);
            stepV<T, MODE, VIRT, CV, WT, 3>(g, a, u, y, cb, comp, tm, t, Q, sh, i + 2, i0, i1, R2,
                                            R3, R1, um, cm, acc);
            stepV<T, MODE, VIRT, CV, WT, 3>(g, a, u, y, cb, comp, tm, t, Q, sh, i + 3, i0, i1, R3,
                                            R0, R2, um, cm, acc);
        }
    }
    finish<T, MODE, kVBlock>(a, L, acc);
}

// ------------------------------------------------------------ launchers

template <class T, int MODE, bool VIRT>
static void go_iso7(const Geo<T>& g, const KArgs<T>& a, hipStream_t s)
{
    const int nt = a.nbx * a.nrc * a.nc;
    if (a.rch > RCH_MAX) return;  // the host never asks for longer chunks
    const dim3 gr(grid_for_tiles(nt));
    if constexpr (iso7_tiled<T>()) {
        const dim3 bl(kBlock);  // one workgroup per tile
        if (a.coef) {
            if (a.wgt) hipLaunchKernelGGL((k_iso7t<T, MODE, VIRT, true, true>), gr, bl, 0, s, g, a);
            else hipLaunchKernelGGL((k_iso7t<T, MODE, VIRT, true, false>), gr, bl, 0, s, g, a);
        } else {
            if (a.wgt) hipLaunchKernelGGL((k_iso7t<T, MODE, VIRT, false, true>), gr, bl, 0, s, g, a);
            else hipLaunchKernelGGL((k_iso7t<T, MODE, VIRT, false, false>), gr, bl, 0, s, g, a);
        }
        return;
    }
    const dim3 bl(64 * W7);
    if (a.coef) {
        if (a.wgt) hipLaunchKernelGGL((k_iso7<T, MODE, VIRT, true, true>), gr, bl, 0, s, g, a);
        else hipLaunchKernelGGL((k_iso7<T, MODE, VIRT, true, false>), gr, bl, 0, s, g, a);
    } else {
        if (a.wgt) hipLaunchKernelGGL((k_iso7<T, MODE, VIRT, false, true>), gr, bl, 0, s, g, a);
        else hipLaunchKernelGGL((k_iso7<T, MODE, VIRT, false, false>), gr, bl, 0, s, g, a);
    }
}
template <class T, int MODE, bool VIRT>
static void go_aligned(const Geo<T>& g, const KArgs<T>& a, hipStream_t s)
{
    const int nt = a.nbx * a.nrc * a.nc;
    if (a.rch > RCH_MAX) return;  // the host never asks for longer chunks
    if (a.wgt)
        hipLaunchKernelGGL((k_aligned<T, MODE, VIRT, true>), dim3(grid_for_tiles(nt)), dim3(kBlock),
                           0, s, g, a);
    else
        hipLaunchKernelGGL((k_aligned<T, MODE, VIRT, false>), dim3(grid_for_tiles(nt)), dim3(kBlock),
                           0, s, g, a);
}

template <class T, int MODE, bool VIRT>
static void go_viscv(const Geo<T>& g, const KArgs<T>& a, hipStream_t s)
{
    const int nt = a.nbx * a.nrc;
    if (a.rch > RCH_MAX) return;  // the host never asks for longer chunks
    const dim3 gr(grid_for_tiles(nt)), bl(kVBlock);
    if (a.coef) {
        if (a.wgt) hipLaunchKernelGGL((k_viscv<T, MODE, VIRT, true, true>), gr, bl, 0, s, g, a);
        else hipLaunchKernelGGL((k_viscv<T, MODE, VIRT, true, false>), gr, bl, 0, s, g, a);
    } else {
        if (a.wgt) hipLaunchKernelGGL((k_viscv<T, MODE, VIRT, false, true>), gr, bl, 0, s, g, a);
        else hipLaunchKernelGGL((k_viscv<T, MODE, VIRT, false, false>), gr, bl, 0, s, g, a);
    }
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
template <class T>
void launch_viscv(int mode, bool virt, const Geo<T>& g, const KArgs<T>& a, hipStream_t s)
{
    PA_DISPATCH(go_viscv)
}
template void launch_viscv<double>(int, bool, const Geo<double>&, const KArgs<double>&, hipStream_t);
template void launch_viscv<float>(int, bool, const Geo<float>&, const KArgs<float>&, hipStream_t);
template void launch_iso7<double>(int, bool, const Geo<double>&, const KArgs<double>&, hipStream_t);
template void launch_iso7<float>(int, bool, const Geo<float>&, const KArgs<float>&, hipStream_t);
template void launch_aligned<double>(int, bool, const Geo<double>&, const KArgs<double>&, hipStream_t);
template void launch_aligned<float>(int, bool, const Geo<float>&, const KArgs<float>&, hipStream_t);

}  // namespace pa
