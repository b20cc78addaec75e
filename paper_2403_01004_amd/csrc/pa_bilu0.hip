// pa_bilu0.hip -- block ILU(0) preconditioner (PC2 of Sec. 3.1: non-overlapping
// ILU(0)) for the 7-point operator, gfx950.
//
// M = wV + dt L restricted to boxes of kBI x kBJ x kBK cells (r, theta, phi;
// the last box in a direction may be short, the periodic phi coupling is
// never inside a box).  With the 7-point sparsity ILU(0) produces no fill
// that it keeps, so only the pivots differ from M:
//   d_m = M_mm - sum_{n lower neighbour of m in the box} M_mn^2 / d_n,
// with the lower neighbours (i-1,j,k), (i,j-1,k), (i,j,k-1).  P^{-1} r is a
// forward and a backward triangular solve inside each box.
//
// GPU mapping: one wave per box.  Lane l owns the column (j, k) = (l / kBK,
// l % kBK) of the box and walks its kBI levels along the wavefronts
// f = i + j + k: at step f the lane treats level f - j - k, whose three lower
// (upper) neighbours were finished at step f - 1 (f + 1) by itself and by
// lanes l - kBK and l - 1 (l + kBK, l + 1).  Those values pass between lanes
// by a DPP row shift and a lane permute, so the dependent chain stays in
// registers.  The couplings M_mn = -dt c_f G_f are rebuilt at each step from
// per-lane column factors and per-box level factors (separable metric), so
// LDS holds only the lane's own values, the inverse pivots and, for a
// variable coefficient, the coefficients: 8 KB (12 KB) per wave, which keeps
// enough waves resident to stream the PCG update fused in front of the solve
// (x += alpha p, r -= alpha q; r is read once per iteration).
#include "pa_internal.h"

namespace pa {

namespace {

constexpr int kBI = 8, kBJ = 4, kBK = 16;
constexpr int kBL = kBJ * kBK;                 // lanes = columns of a box
constexpr int kBC = kBI * kBL;                 // cells of a box
constexpr int kSteps = kBI + kBJ + kBK - 2;    // wavefronts i + j + k
static_assert(kBL == 64, "one wave per box");

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

struct BoxPos {
    int i0, nib;        // first level, levels present in the grid
    int j, k;           // the lane's column in the grid
    bool col;           // the column lies in the grid
    int jj, kk;         // the lane's column in the box
};

__device__ __forceinline__ BoxPos box_pos(const Geo<double>& g, unsigned b, int lane)
{
    const unsigned nbj = (unsigned)(g.nt + kBJ - 1) / kBJ, nbk = (unsigned)(g.np + kBK - 1) / kBK;
    const unsigned bk = b % nbk, t = b / nbk, bj = t % nbj, bi = t / nbj;
    BoxPos p;
    p.jj = lane / kBK;
    p.kk = lane % kBK;
    p.i0 = (int)bi * kBI;
    p.nib = min(kBI, g.nr - p.i0);
    p.j = (int)bj * kBJ + p.jj;
    p.k = (int)bk * kBK + p.kk;
    p.col = p.j < g.nt && p.k < g.np;
    return p;
}

// The value v of lane l - 1 (row_prev) or l + 1 (row_next) in the same row
// of 16 lanes, 0 past the row's end (DPP row shifts on the two halves).
__device__ __forceinline__ double row_prev(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffll), 0x111, 0xf,
                                               0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x111, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double row_next(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffll), 0x101, 0xf,
                                               0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x101, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Face coupling -dt c_f G_f with c_f the mean of the two cells' coefficients
// and the separable face metric G_f = (level factor) (column factor).  The
// lower coupling of a cell and the upper coupling of its neighbour are
// evaluated from the same operands in the same order, so they are equal bit
// for bit and P stays symmetric.
__device__ __forceinline__ double cpl(double mdt, double ca, double cb, double lev, double colf)
{
    return (mdt * (0.5 * (ca + cb))) * (lev * colf);
}

// The box's geometry: per-lane column factors of the six faces (0 where the
// neighbour is outside the box or the grid) and per-level factors in LDS.
struct BoxGeo {
    double fr;             // vt[j] vp[k]: radial faces
    double ft_lo, ft_hi;   // gtt[j] vp[k], gtt[j+1] vp[k]: colatitude faces
    double fk_lo, fk_hi;   // gpt[j] gpp[k], gpt[j] gpp[k+1]: longitude faces
};

// s_gr[ii] = gr[i0+ii] for the radial face below level ii (0 at ii = 0 and
// at and beyond nib), s_gtr[ii] = gtr[i0+ii] (0 beyond nib); s_c the cell
// coefficients of the box (0 outside the grid) when VC.
template <bool VC>
__device__ __forceinline__ BoxGeo box_geo(const Geo<double>& g, const BoxPos& p, int lane,
                                          const double* __restrict__ coef, double* s_gr,
                                          double* s_gtr, double* s_c)
{
    if (lane <= kBI) {
        const int i = p.i0 + lane;
        s_gr[lane] = (lane > 0 && lane < p.nib) ? g.gr[i] : 0.0;
        if (lane < kBI) s_gtr[lane] = lane < p.nib ? g.gtr[i] : 0.0;
    }
    if constexpr (VC) {
        const size_t base = (size_t)p.j * g.np + p.k;
#pragma unroll
        for (int ii = 0; ii < kBI; ++ii)
            s_c[ii * kBL + lane] =
                (p.col && ii < p.nib) ? coef[(size_t)(p.i0 + ii) * g.P + base] : 0.0;
    }
    BoxGeo q{0.0, 0.0, 0.0, 0.0, 0.0};
    if (p.col) {
        const double vt = g.vt[p.j], vp = g.vp[p.k];
        q.fr = vt * vp;
        if (p.jj > 0) q.ft_lo = g.gtt[p.j] * vp;
        if (p.jj + 1 < kBJ && p.j + 1 < g.nt) q.ft_hi = g.gtt[p.j + 1] * vp;
        if (p.kk > 0) q.fk_lo = g.gpt[p.j] * g.gpp[p.k];
        if (p.kk + 1 < kBK && p.k + 1 < g.np) q.fk_hi = g.gpt[p.j] * g.gpp[p.k + 1];
    }
    return q;
}

// lower couplings M(m, r-), M(m, t-), M(m, p-) of the lane's cell at level
// ii (q = ii * kBL + lane)
template <bool VC>
__device__ __forceinline__ void lower_cpl(const BoxGeo& b, int ii, int q, double mdt, double cs,
                                          const double* s_gr, const double* s_gtr,
                                          const double* s_c, double& ar, double& at, double& ak)
{
    const double gtr = s_gtr[ii];
    if constexpr (VC) {
        const double cm = s_c[q];
        ar = cpl(mdt, cm, s_c[ii > 0 ? q - kBL : q], s_gr[ii], b.fr);
        at = cpl(mdt, cm, s_c[q >= kBK ? q - kBK : q], gtr, b.ft_lo);
        ak = cpl(mdt, cm, s_c[q > 0 ? q - 1 : q], gtr, b.fk_lo);
    } else {
        ar = cpl(mdt, cs, cs, s_gr[ii], b.fr);
        at = cpl(mdt, cs, cs, gtr, b.ft_lo);
        ak = cpl(mdt, cs, cs, gtr, b.fk_lo);
    }
}

// upper couplings M(m, r+), M(m, t+), M(m, p+): the lower couplings of the
// neighbours, same operands in the same order
template <bool VC>
__device__ __forceinline__ void upper_cpl(const BoxGeo& b, int ii, int q, double mdt, double cs,
                                          const double* s_gr, const double* s_gtr,
                                          const double* s_c, double& arp, double& atp,
                                          double& akp)
{
    const double gtr = s_gtr[ii];
    if constexpr (VC) {
        const double cm = s_c[q];
        arp = cpl(mdt, s_c[ii + 1 < kBI ? q + kBL : q], cm, s_gr[ii + 1], b.fr);
        atp = cpl(mdt, s_c[q + kBK < kBC ? q + kBK : q], cm, gtr, b.ft_hi);
        akp = cpl(mdt, s_c[q + 1 < kBC ? q + 1 : q], cm, gtr, b.fk_hi);
    } else {
        arp = cpl(mdt, cs, cs, s_gr[ii + 1], b.fr);
        atp = cpl(mdt, cs, cs, gtr, b.ft_hi);
        akp = cpl(mdt, cs, cs, gtr, b.fk_hi);
    }
}

// Inverse pivots of the box into ip[] (HBM); D = wV + dt diag L.  The chain
// of pivots passes between lanes like the forward solve.
template <bool VC>
__global__ __launch_bounds__(kBL) void k_bilu0_factor(Geo<double> g, const double* __restrict__ coef,
                                                      double cs, double dt,
                                                      const double* __restrict__ D,
                                                      double* __restrict__ ip, int* flag)
{
    __shared__ double s_d[kBC], s_c[VC ? kBC : 1], s_gr[kBI + 1], s_gtr[kBI];
    const int lane = threadIdx.x;
    const BoxPos p = box_pos(g, blockIdx.x, lane);
    const BoxGeo bg = box_geo<VC>(g, p, lane, coef, s_gr, s_gtr, s_c);
    const size_t base = (size_t)p.j * g.np + p.k;
#pragma unroll
    for (int ii = 0; ii < kBI; ++ii)
        s_d[ii * kBL + lane] = (p.col && ii < p.nib) ? D[(size_t)(p.i0 + ii) * g.P + base] : 1.0;
    __syncthreads();
    const double mdt = -dt;
    double cur = 0.0;   // the lane's latest inverse pivot
    bool bad = false;
#pragma unroll 2
    for (int f = 0; f < kSteps; ++f) {
        const double ipk = row_prev(cur);
        const double ipj = __shfl_up(cur, kBK, 64);
        const int ii = f - p.jj - p.kk;
        if (p.col && ii >= 0 && ii < p.nib) {
            const int q = ii * kBL + lane;
            double ar, at, ak;
            lower_cpl<VC>(bg, ii, q, mdt, cs, s_gr, s_gtr, s_c, ar, at, ak);
            double d = s_d[q] - ar * ar * cur - at * at * ipj - ak * ak * ipk;
            if (!(d > 0.0) || !isfinite(d)) {
                bad = true;
                d = 1.0;
            }
            cur = 1.0 / d;
            ip[(size_t)(p.i0 + ii) * g.P + base] = cur;
        }
    }
    if (bad) *flag = 1;
}

__device__ __forceinline__ void load_ip(const Geo<double>& g, const BoxPos& p, int lane,
                                        const double* __restrict__ ip, double* s_ip)
{
    const size_t base = (size_t)p.j * g.np + p.k;
#pragma unroll
    for (int ii = 0; ii < kBI; ++ii)
        s_ip[ii * kBL + lane] =
            (p.col && ii < p.nib) ? ip[(size_t)(p.i0 + ii) * g.P + base] : 0.0;
}

// Forward and backward solve of NV components in place: s_w[v * kBC + q]
// holds r on entry (0 outside the grid) and z = U^{-1} L^{-1} r on exit.  At
// step f a lane needs the values its lower (upper) neighbours produced at
// step f - 1: its own previous output and the outputs of lanes l - 1 and
// l - kBK (l + 1, l + kBK), read across lanes.  Couplings are 0 where a
// neighbour is absent (and the values they multiply are finite), so the
// steps need no tests.  LDS fills of other lanes must be visible (barrier
// before).
template <int NV, bool VC>
__device__ __forceinline__ void box_solve(const BoxPos& p, const BoxGeo& bg, int lane, double mdt,
                                          double cs, double* s_w, const double* s_ip,
                                          const double* s_gr, const double* s_gtr,
                                          const double* s_c)
{
    double cur[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) cur[v] = 0.0;
    // forward: y_m = r_m - sum_lower M_mn y_n / d_n; s_w keeps w_m = y_m / d_m
#pragma unroll 2
    for (int f = 0; f < kSteps; ++f) {
        double wk[NV], wj[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            wk[v] = row_prev(cur[v]);               // (i, j, k-1)
            wj[v] = __shfl_up(cur[v], kBK, 64);     // (i, j-1, k)
        }
        const int ii = f - p.jj - p.kk;
        if (p.col && ii >= 0 && ii < p.nib) {
            const int q = ii * kBL + lane;
            double ar, at, ak;
            lower_cpl<VC>(bg, ii, q, mdt, cs, s_gr, s_gtr, s_c, ar, at, ak);
            const double ipv = s_ip[q];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double y = s_w[v * kBC + q] - ar * cur[v] - at * wj[v] - ak * wk[v];
                cur[v] = y * ipv;
                s_w[v * kBC + q] = cur[v];
            }
        }
    }
    // backward: z_m = w_m - (sum_upper M_mn z_n) / d_m
#pragma unroll
    for (int v = 0; v < NV; ++v) cur[v] = 0.0;
#pragma unroll 2
    for (int f = kSteps - 1; f >= 0; --f) {
        double zk[NV], zj[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            zk[v] = row_next(cur[v]);               // (i, j, k+1)
            zj[v] = __shfl_down(cur[v], kBK, 64);   // (i, j+1, k)
        }
        const int ii = f - p.jj - p.kk;
        if (p.col && ii >= 0 && ii < p.nib) {
            const int q = ii * kBL + lane;
            double arp, atp, akp;
            upper_cpl<VC>(bg, ii, q, mdt, cs, s_gr, s_gtr, s_c, arp, atp, akp);
            const double ipv = s_ip[q];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double sum = arp * cur[v] + atp * zj[v] + akp * zk[v];
                cur[v] = s_w[v * kBC + q] - ipv * sum;
                s_w[v * kBC + q] = cur[v];
            }
        }
    }
}

// z = P^{-1} r for every component (out in PT), NV components per sweep;
// partial <r, z> per box
template <class PT, int NV, bool VC>
__global__ __launch_bounds__(kBL) void k_bilu0_solve(Geo<double> g, int nc,
                                                     const double* __restrict__ coef, double cs,
                                                     double dt, const double* __restrict__ ip,
                                                     const double* __restrict__ r,
                                                     PT* __restrict__ out, double* part)
{
    __shared__ double s_w[NV * kBC], s_ip[kBC], s_c[VC ? kBC : 1], s_gr[kBI + 1], s_gtr[kBI];
    const int lane = threadIdx.x;
    const BoxPos p = box_pos(g, blockIdx.x, lane);
    const BoxGeo bg = box_geo<VC>(g, p, lane, coef, s_gr, s_gtr, s_c);
    load_ip(g, p, lane, ip, s_ip);
    const size_t N = (size_t)g.nr * g.P, base = (size_t)p.j * g.np + p.k;
    double rz = 0.0;
#pragma unroll 1
    for (int c0 = 0; c0 < nc; c0 += NV) {
        double rv[NV][kBI];
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int ii = 0; ii < kBI; ++ii) {
                const bool on = p.col && ii < p.nib;
                rv[v][ii] = on ? r[(c0 + v) * N + (size_t)(p.i0 + ii) * g.P + base] : 0.0;
                s_w[v * kBC + ii * kBL + lane] = rv[v][ii];
            }
        __syncthreads();
        box_solve<NV, VC>(p, bg, lane, -dt, cs, s_w, s_ip, s_gr, s_gtr, s_c);
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int ii = 0; ii < kBI; ++ii)
                if (p.col && ii < p.nib) {
                    const double z = s_w[v * kBC + ii * kBL + lane];
                    out[(c0 + v) * N + (size_t)(p.i0 + ii) * g.P + base] = (PT)z;
                    rz += rv[v][ii] * z;
                }
    }
    rz = wave_sum(rz);
    if (lane == 0) part[blockIdx.x] = rz;
}

// x += alpha p, r -= alpha q, z = P^{-1} r, NV components per sweep;
// partials <r, z>, <r, r>
template <class PT, int NV, bool VC>
__global__ __launch_bounds__(kBL) void k_pcg_update_bilu0(Geo<double> g, int nc,
                                                          const double* __restrict__ coef,
                                                          double cs, double dt,
                                                          const double* __restrict__ ip,
                                                          double* __restrict__ x,
                                                          double* __restrict__ r,
                                                          const PT* __restrict__ pv,
                                                          const PT* __restrict__ qv,
                                                          double* __restrict__ z,
                                                          const DevState* st, double* part)
{
    if (st->done) return;
    __shared__ double s_w[NV * kBC], s_ip[kBC], s_c[VC ? kBC : 1], s_gr[kBI + 1], s_gtr[kBI];
    const double alpha = st->alpha;
    const int lane = threadIdx.x;
    const BoxPos p = box_pos(g, blockIdx.x, lane);
    const BoxGeo bg = box_geo<VC>(g, p, lane, coef, s_gr, s_gtr, s_c);
    load_ip(g, p, lane, ip, s_ip);
    const size_t N = (size_t)g.nr * g.P, base = (size_t)p.j * g.np + p.k;
    double rz = 0.0, rr = 0.0;
#pragma unroll 1
    for (int c0 = 0; c0 < nc; c0 += NV) {
        double rv[NV][kBI];
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int ii = 0; ii < kBI; ++ii) {
                const bool on = p.col && ii < p.nib;
                const size_t m =
                    (c0 + v) * N + (size_t)(p.i0 + (on ? ii : 0)) * g.P + (on ? base : 0);
                // x, r, p, q and z are streamed once: non-temporal accesses
                const double xv = on ? __builtin_nontemporal_load(x + m) : 0.0;
                const double ro = on ? __builtin_nontemporal_load(r + m) : 0.0;
                const double pp = on ? (double)__builtin_nontemporal_load(pv + m) : 0.0;
                const double qq = on ? (double)__builtin_nontemporal_load(qv + m) : 0.0;
                const double rn = ro - alpha * qq;
                rv[v][ii] = rn;
                s_w[v * kBC + ii * kBL + lane] = rn;
                if (on) {
                    __builtin_nontemporal_store(xv + alpha * pp, x + m);
                    __builtin_nontemporal_store(rn, r + m);
                    rr += rn * rn;
                }
            }
        __syncthreads();
        box_solve<NV, VC>(p, bg, lane, -dt, cs, s_w, s_ip, s_gr, s_gtr, s_c);
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int ii = 0; ii < kBI; ++ii)
                if (p.col && ii < p.nib) {
                    const double zv = s_w[v * kBC + ii * kBL + lane];
                    __builtin_nontemporal_store(zv, z + (c0 + v) * N + (size_t)(p.i0 + ii) * g.P + base);
                    rz += rv[v][ii] * zv;
                }
    }
    rz = wave_sum(rz);
    rr = wave_sum(rr);
    if (lane == 0) {
        part[blockIdx.x] = rz;
        part[gridDim.x + blockIdx.x] = rr;
    }
}

// Components that share a sweep's steps.  One: sharing the steps of three
// components takes 8 KB more LDS per wave, and the lower occupancy costs
// more than the shared step latency saves (measured 1.3x slower on the
// three-component viscosity solve).
constexpr int kNV = 1;
static_assert(kNV == 1, "the launchers pass any number of components");

}  // namespace

int bilu0_boxes(int nr, int nt, int np)
{
    return ((nr + kBI - 1) / kBI) * ((nt + kBJ - 1) / kBJ) * ((np + kBK - 1) / kBK);
}

void launch_bilu0_factor(const Geo<double>& g, const double* coef, double cs, double dt,
                         const double* D, double* ip, int* flag, hipStream_t s)
{
    const int nb = bilu0_boxes(g.nr, g.nt, g.np);
    if (coef)
        hipLaunchKernelGGL((k_bilu0_factor<true>), dim3(nb), dim3(kBL), 0, s, g, coef, cs, dt, D,
                           ip, flag);
    else
        hipLaunchKernelGGL((k_bilu0_factor<false>), dim3(nb), dim3(kBL), 0, s, g, coef, cs, dt, D,
                           ip, flag);
}

#define PA_BILU0_SOLVE(NV, VC)                                                                   \
    hipLaunchKernelGGL((k_bilu0_solve<PT, NV, VC>), dim3(nb), dim3(kBL), 0, s, g, nc, coef, cs, \
                       dt, ip, r, out, part)

template <class PT>
void launch_bilu0_solve(const Geo<double>& g, int nc, const double* coef, double cs, double dt,
                        const double* ip, const double* r, PT* out, double* part, int* nparts,
                        hipStream_t s)
{
    const int nb = bilu0_boxes(g.nr, g.nt, g.np);
    *nparts = nb;
    if (coef) PA_BILU0_SOLVE(kNV, true);
    else PA_BILU0_SOLVE(kNV, false);
}
template void launch_bilu0_solve<double>(const Geo<double>&, int, const double*, double, double,
                                         const double*, const double*, double*, double*, int*,
                                         hipStream_t);
template void launch_bilu0_solve<float>(const Geo<double>&, int, const double*, double, double,
                                        const double*, const double*, float*, double*, int*,
                                        hipStream_t);

#define PA_BILU0_UPDATE(NV, VC)                                                               \
    hipLaunchKernelGGL((k_pcg_update_bilu0<PT, NV, VC>), dim3(nb), dim3(kBL), 0, s, g, nc,  \
                       coef, cs, dt, ip, x, r, p, q, z, st, part)

template <class PT>
void launch_pcg_update_bilu0(const Geo<double>& g, int nc, const double* coef, double cs,
                             double dt, const double* ip, double* x, double* r, const PT* p,
                             const PT* q, double* z, const DevState* st, double* part,
                             int* nparts, hipStream_t s)
{
    const int nb = bilu0_boxes(g.nr, g.nt, g.np);
    *nparts = nb;
    if (coef) PA_BILU0_UPDATE(kNV, true);
    else PA_BILU0_UPDATE(kNV, false);
}
template void launch_pcg_update_bilu0<double>(const Geo<double>&, int, const double*, double,
                                              double, const double*, double*, double*,
                                              const double*, const double*, double*,
                                              const DevState*, double*, int*, hipStream_t);
template void launch_pcg_update_bilu0<float>(const Geo<double>&, int, const double*, double,
                                             double, const double*, double*, double*,
                                             const float*, const float*, double*,
                                             const DevState*, double*, int*, hipStream_t);

}  // namespace pa
