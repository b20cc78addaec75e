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

template <class T, int MODE, bool VIRT>
__device__ __forceinline__ void epilogue(const KArgs<T>& a, size_t m, T Lu, T V, T uc,
                                         Acc<T, MODE>& acc)
{
    if constexpr (MODE == kApply || MODE == kFirst) {
        const T F = -Lu / V;
        a.out[m] = F;
        if constexpr (MODE == kFirst) {
            const double af = fabs((double)F);
            if (af > acc.best) { acc.best = af; acc.bidx = (long long)m; }
            if (!isfinite((double)F)) acc.bad = 1;
        }
    } else if constexpr (MODE == kStage) {
        const double F = (double)(-Lu / V);
        const double u0v = (double)a.u0[m];
        const double y0v = (double)a.y0[m];
        double km2;
        if (a.km2 == kKm2Array) km2 = (double)a.ukm2[m];
        else if (a.km2 == kKm2U0) km2 = u0v;
        else km2 = (double)(T)(u0v + a.a1 * y0v);
        const double r = a.mu * (double)uc + a.nu * km2 + a.c0 * u0v + a.mudt * F + a.gdt * y0v;
        a.out[m] = (T)r;
    } else {  // kMatvec
        const T q = V * uc + (T)a.dt * Lu;
        a.out[m] = q;
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

// ------------------------------------------------------------ 7-point

template <class T, bool VIRT>
__device__ __forceinline__ T ldu(const KArgs<T>& a, const T* u, const T* y, size_t q)
{
    if constexpr (VIRT) return (T)((double)u[q] + a.a1 * (double)y[q]);
    else return u[q];
}

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
    Acc<T, MODE> acc;
    T um = 0, uc = 0, cm = a.cs, cc = a.cs;
    if (i0 < i1) {
        uc = ldu<T, VIRT>(a, u, y, (size_t)i0 * P + pp);
        if (varc) cc = cf[(size_t)i0 * P + pp];
        if (i0 > 0) {
            um = ldu<T, VIRT>(a, u, y, (size_t)(i0 - 1) * P + pp);
            if (varc) cm = cf[(size_t)(i0 - 1) * P + pp];
        }
    }
    for (int i = i0; i < i1; ++i) {
        const size_t lv = (size_t)i * P;
        T up = 0, cp = a.cs;
        if (i + 1 < nr) {
            up = ldu<T, VIRT>(a, u, y, lv + P + pp);
            if (varc) cp = cf[lv + P + pp];
        }
        const size_t rowb = lv + (size_t)j * np;
        const T uw = ldu<T, VIRT>(a, u, y, rowb + km);
        const T ue = ldu<T, VIRT>(a, u, y, rowb + kp);
        const T us = hs ? ldu<T, VIRT>(a, u, y, rowb - np + k) : T(0);
        const T un = hn ? ldu<T, VIRT>(a, u, y, rowb + np + k) : T(0);
        T cw = a.cs, ce = a.cs, csb = a.cs, cn = a.cs;
        if (varc) {
            cw = cf[rowb + km];
            ce = cf[rowb + kp];
            if (hs) csb = cf[rowb - np + k];
            if (hn) cn = cf[rowb + np + k];
        }
        const T half = T(0.5);
        const T gtri = g.gtr[i];
        T Lu = 0;
        if (i > 0) Lu += half * (cc + cm) * (g.gr[i] * vtj * vpk) * (uc - um);
        else if (a.bc_in == 0) {
            const T ub = a.affine ? a.ub_in[ob] : T(0);
            Lu += cc * (g.gr[0] * vtj * vpk) * (uc - ub);
        }
        if (i < nr - 1) Lu += half * (cc + cp) * (g.gr[i + 1] * vtj * vpk) * (uc - up);
        else if (a.bc_out == 0) {
            const T ub = a.affine ? a.ub_out[ob] : T(0);
            Lu += cc * (g.gr[nr] * vtj * vpk) * (uc - ub);
        }
        if (hs) Lu += half * (cc + csb) * (gtri * gts * vpk) * (uc - us);
        if (hn) Lu += half * (cc + cn) * (gtri * gtn * vpk) * (uc - un);
        Lu += half * (cc + cw) * (gtri * gpj * gpw) * (uc - uw);
        Lu += half * (cc + ce) * (gtri * gpj * gpe) * (uc - ue);
        const T V = g.vr[i] * vtj * vpk;
        if (valid) epilogue<T, MODE, VIRT>(a, cb + lv + pp, Lu, V, uc, acc);
        um = uc; uc = up; cm = cc; cc = cp;
    }
    finish<T, MODE>(a, L, acc);
}

// ------------------------------------------------------------ field-aligned

// values of one radial level on the 3x3 (theta, phi) neighbourhood of the
// thread's cell; rows j-1 / j+1 only when the corners using them exist
template <class T, bool VIRT>
__device__ __forceinline__ void load3x3(const KArgs<T>& a, const T* u, const T* y, size_t lv,
                                        const int (&off)[3][3], bool hasA, bool hasC, T (&x)[3][3])
{
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const bool use = (r == 0) ? hasA : (r == 2) ? hasC : true;
#pragma unroll
        for (int q = 0; q < 3; ++q) x[r][q] = use ? ldu<T, VIRT>(a, u, y, lv + off[r][q]) : T(0);
    }
}

// mirror ghost level across a radial boundary: Dirichlet 2 u_b - u (u_b = 0
// in linear mode), no-flux u
template <class T>
__device__ __forceinline__ void ghost3x3(const T (&x)[3][3], const T* ub, int bc, int affine,
                                         size_t ob, const int (&off)[3][3], bool hasA, bool hasC,
                                         T (&gx)[3][3])
{
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const bool use = (r == 0) ? hasA : (r == 2) ? hasC : true;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (bc == 0) {
                const T b = (affine && use) ? ub[ob + off[r][q]] : T(0);
                gx[r][q] = T(2) * b - x[r][q];
            } else {
                gx[r][q] = x[r][q];
            }
        }
    }
}

// Fluxes t of the four corners A(j,k) B(j,k+1) C(j+1,k) D(j+1,k+1) of corner
// plane ic, between levels lo and hi, and the scatter weights of the
// thread's cell as the upper (wt) and lower (wb) cell of that plane.
template <class T>
__device__ __forceinline__ void corner_plane(const T (&lo)[3][3], const T (&hi)[3][3], const T* e,
                                             size_t nco, size_t qrow0, size_t qrow1, int k, int kp,
                                             bool hasA, bool hasC, int kind, int bc, T& up_sum,
                                             T& dn_sum)
{
    // kind: 0 interior plane, 1 inner boundary (real cells above), 2 outer boundary
    T s[3][3], d[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) { s[r][q] = lo[r][q] + hi[r][q]; d[r][q] = hi[r][q] - lo[r][q]; }
    up_sum = 0;
    dn_sum = 0;
    const T qt = T(0.25), hf = T(0.5);
#pragma unroll
    for (int cr = 0; cr < 4; ++cr) {
        const int r0 = cr >> 1, c0 = cr & 1;
        if ((r0 == 0 && !hasA) || (r0 == 1 && !hasC)) continue;
        const size_t q = (r0 ? qrow1 : qrow0) + (c0 ? kp : k);
        const T er = e[q], et = e[nco + q], ep = e[2 * nco + q];
        const T Dr = qt * (d[r0][c0] + d[r0][c0 + 1] + d[r0 + 1][c0] + d[r0 + 1][c0 + 1]);
        const T Dt = qt * (s[r0 + 1][c0] + s[r0 + 1][c0 + 1] - s[r0][c0] - s[r0][c0 + 1]);
        const T Dp = qt * (s[r0][c0 + 1] + s[r0 + 1][c0 + 1] - s[r0][c0] - s[r0 + 1][c0]);
        const T t = er * Dr + et * Dt + ep * Dp;
        // the thread's cell sits at row 1, column 1 of the neighbourhood
        const T st = r0 ? T(-1) : T(1);
        const T sp = c0 ? T(-1) : T(1);
        const T tang = st * et + sp * ep;
        if (kind == 0) {
            up_sum += qt * (er + tang) * t;
            dn_sum += qt * (-er + tang) * t;
        } else if (kind == 1) {
            up_sum += (bc == 0 ? hf * er : hf * tang) * t;
        } else {
            dn_sum += (bc == 0 ? -hf * er : hf * tang) * t;
        }
    }
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
    const bool hasA = j >= 1, hasC = j + 1 <= nt - 1;
    int off[3][3];
    const int cols[3] = {km, k, kp};
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) off[r][q] = (j + r - 1) * np + cols[q];
    const size_t cb = (size_t)c * nr * P;
    const T* u = a.u + cb;
    const T* y = VIRT ? a.y0 + cb : nullptr;
    const size_t ob = (size_t)c * P;
    const size_t nco = (size_t)(nr + 1) * (nt + 1) * np;
    const size_t cplane = (size_t)(nt + 1) * np;
    const int i0 = a.r_lo + rc * a.rch;
    const int i1 = min(a.r_hi, i0 + a.rch);
    const T vtj = g.vt[j], vpk = g.vp[k];
    Acc<T, MODE> acc;
    T lo[3][3], hi[3][3];
    T carry = 0;
    if (i0 < i1) {
        load3x3<T, VIRT>(a, u, y, (size_t)i0 * P, off, hasA, hasC, hi);
        if (i0 == 0) ghost3x3<T>(hi, a.ub_in, a.bc_in, a.affine, ob, off, hasA, hasC, lo);
        else load3x3<T, VIRT>(a, u, y, (size_t)(i0 - 1) * P, off, hasA, hasC, lo);
        T up, dn;
        const size_t qb = (size_t)i0 * cplane;
        corner_plane<T>(lo, hi, a.e, nco, qb + (size_t)j * np, qb + (size_t)(j + 1) * np, k, kp,
                        hasA, hasC, i0 == 0 ? 1 : 0, a.bc_in, up, dn);
        carry = up;
    }
    for (int i = i0; i < i1; ++i) {
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int q = 0; q < 3; ++q) lo[r][q] = hi[r][q];
        const int ic = i + 1;
        int kind = 0, bc = 0;
        if (ic < nr) {
            load3x3<T, VIRT>(a, u, y, (size_t)ic * P, off, hasA, hasC, hi);
        } else {
            ghost3x3<T>(lo, a.ub_out, a.bc_out, a.affine, ob, off, hasA, hasC, hi);
            kind = 2;
            bc = a.bc_out;
        }
        T up, dn;
        const size_t qb = (size_t)ic * cplane;
        corner_plane<T>(lo, hi, a.e, nco, qb + (size_t)j * np, qb + (size_t)(j + 1) * np, k, kp,
                        hasA, hasC, kind, bc, up, dn);
        const T Lu = carry + dn;
        carry = up;
        const T V = g.vr[i] * vtj * vpk;
        if (valid) epilogue<T, MODE, VIRT>(a, cb + (size_t)i * P + pp, Lu, V, lo[1][1], acc);
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
