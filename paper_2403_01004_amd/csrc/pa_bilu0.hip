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
// lanes l - kBK and l - 1 (l + kBK, l + 1).  In the solves those values pass
// between lanes by DPP row shifts and a lane permute, so the dependent chain
// stays in registers; the box's values, couplings and inverse pivots sit in
// LDS (20 KB per wave).
// The PCG update x += alpha p, r -= alpha q is fused in front of the solve,
// so r is read once per iteration; all components of the box share the
// couplings and pivots.
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

// Lower couplings M(m, r-), M(m, t-), M(m, p-) = -dt c_f G_f of every cell
// of the lane's column into LDS (0 where the neighbour is outside the box or
// the grid, and for cells outside the grid).  c_f is the mean of the two cell
// coefficients (coef == null: the constant cs).
__device__ __forceinline__ void box_couplings(const Geo<double>& g, const BoxPos& p,
                                              const double* __restrict__ coef, double cs,
                                              double dt, int lane, double* s_ar, double* s_at,
                                              double* s_ak)
{
    const size_t P = (size_t)g.P, np = (size_t)g.np;
    double vt = 0.0, vp = 0.0, gtt = 0.0, gpt = 0.0, gpp = 0.0;
    if (p.col) {
        vt = g.vt[p.j]; vp = g.vp[p.k]; gtt = g.gtt[p.j]; gpt = g.gpt[p.j]; gpp = g.gpp[p.k];
    }
#pragma unroll
    for (int ii = 0; ii < kBI; ++ii) {
        double ar = 0.0, at = 0.0, ak = 0.0;
        if (p.col && ii < p.nib) {
            const int i = p.i0 + ii;
            const size_t m = (size_t)i * P + (size_t)p.j * np + (size_t)p.k;
            const double cm = coef ? coef[m] : cs;
            const double gtr = g.gtr[i];
            if (ii > 0) ar = -dt * (0.5 * (cm + (coef ? coef[m - P] : cs))) * (g.gr[i] * vt * vp);
            if (p.jj > 0) at = -dt * (0.5 * (cm + (coef ? coef[m - np] : cs))) * (gtr * gtt * vp);
            if (p.kk > 0) ak = -dt * (0.5 * (cm + (coef ? coef[m - 1] : cs))) * (gtr * gpt * gpp);
        }
        s_ar[ii * kBL + lane] = ar;
        s_at[ii * kBL + lane] = at;
        s_ak[ii * kBL + lane] = ak;
    }
}

// The value v of lane l - 1 (row_prev) or l + 1 (row_next) in the same row
// of 16 lanes, 0 past the row's end (DPP row shifts, two 32-bit halves).
__device__ __forceinline__ double dpp_shift(double v, int ctrl)
{
    const long long b = __double_as_longlong(v);
    int lo = (int)(unsigned)(b & 0xffffffffll), hi = (int)(b >> 32);
    switch (ctrl) {
    case 0:   // row_shr:1
        lo = __builtin_amdgcn_update_dpp(0, lo, 0x111, 0xf, 0xf, true);
        hi = __builtin_amdgcn_update_dpp(0, hi, 0x111, 0xf, 0xf, true);
        break;
    default:  // row_shl:1
        lo = __builtin_amdgcn_update_dpp(0, lo, 0x101, 0xf, 0xf, true);
        hi = __builtin_amdgcn_update_dpp(0, hi, 0x101, 0xf, 0xf, true);
        break;
    }
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double row_prev(double v) { return dpp_shift(v, 0); }
__device__ __forceinline__ double row_next(double v) { return dpp_shift(v, 1); }

// Forward and backward solve of one component in place: s_w holds r on
// entry (0 outside the grid) and z = U^{-1} L^{-1} r on exit.  At step f a
// lane needs the values its lower (upper) neighbours produced at step f - 1:
// its own previous output and the outputs of lanes l - 1 and l - kBK
// (l + 1, l + kBK), read across lanes, so the chain of steps runs through
// registers; s_w only keeps each lane's own values between the sweeps.
// The couplings of the other lanes must be visible in LDS (barrier before).
__device__ __forceinline__ void box_solve(const BoxPos& p, int lane, double* s_w,
                                          const double* s_ar, const double* s_at,
                                          const double* s_ak, const double* s_ip)
{
    // forward: y_m = r_m - sum_lower M_mn y_n / d_n; s_w keeps w_m = y_m / d_m
    double cur = 0.0;
#pragma unroll 2
    for (int f = 0; f < kSteps; ++f) {
        const double wk = row_prev(cur);          // (i, j, k-1)
        const double wj = __shfl_up(cur, kBK, 64);  // (i, j-1, k)
        const int ii = f - p.jj - p.kk;
        if (p.col && ii >= 0 && ii < p.nib) {
            const int q = ii * kBL + lane;
            double y = s_w[q];
            if (ii > 0) y -= s_ar[q] * cur;
            if (p.jj > 0) y -= s_at[q] * wj;
            if (p.kk > 0) y -= s_ak[q] * wk;
            cur = y * s_ip[q];
            s_w[q] = cur;
        }
    }
    // backward: z_m = w_m - (sum_upper M_mn z_n) / d_m
    cur = 0.0;
#pragma unroll 2
    for (int f = kSteps - 1; f >= 0; --f) {
        const double zk = row_next(cur);            // (i, j, k+1)
        const double zj = __shfl_down(cur, kBK, 64);  // (i, j+1, k)
        const int ii = f - p.jj - p.kk;
        if (p.col && ii >= 0 && ii < p.nib) {
            const int q = ii * kBL + lane;
            double s = 0.0;
            if (ii + 1 < p.nib) s += s_ar[q + kBL] * cur;
            if (p.jj + 1 < kBJ) s += s_at[q + kBK] * zj;
            if (p.kk + 1 < kBK) s += s_ak[q + 1] * zk;
            cur = s_w[q] - s_ip[q] * s;
            s_w[q] = cur;
        }
    }
}

// inverse pivots of the box into s_ip (and ip[] in HBM); D = wV + dt diag L
__device__ __forceinline__ void box_factor(const Geo<double>& g, const BoxPos& p, int lane,
                                           const double* __restrict__ D, double* s_w,
                                           const double* s_ar, const double* s_at,
                                           const double* s_ak, double* s_ip, double* ip,
                                           int* flag)
{
    const size_t P = (size_t)g.P;
    const size_t base = (size_t)p.j * g.np + p.k;
#pragma unroll
    for (int ii = 0; ii < kBI; ++ii)
        s_w[ii * kBL + lane] = (p.col && ii < p.nib) ? D[(size_t)(p.i0 + ii) * P + base] : 1.0;
    __syncthreads();
#pragma unroll 1
    for (int f = 0; f < kSteps; ++f) {
        const int ii = f - p.jj - p.kk;
        if (p.col && ii >= 0 && ii < p.nib) {
            const int q = ii * kBL + lane;
            double d = s_w[q];
            if (ii > 0) d -= s_ar[q] * s_ar[q] * s_ip[q - kBL];
            if (p.jj > 0) d -= s_at[q] * s_at[q] * s_ip[q - kBK];
            if (p.kk > 0) d -= s_ak[q] * s_ak[q] * s_ip[q - 1];
            if (!(d > 0.0) || !isfinite(d)) {
                *flag = 1;
                d = 1.0;
            }
            const double v = 1.0 / d;
            s_ip[q] = v;
            if (ip) ip[(size_t)(p.i0 + ii) * P + base] = v;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBL) void k_bilu0_factor(Geo<double> g, const double* __restrict__ coef,
                                                      double cs, double dt,
                                                      const double* __restrict__ D,
                                                      double* __restrict__ ip, int* flag)
{
    __shared__ double s_w[kBC], s_ar[kBC], s_at[kBC], s_ak[kBC], s_ip[kBC];
    const int lane = threadIdx.x;
    const BoxPos p = box_pos(g, blockIdx.x, lane);
    box_couplings(g, p, coef, cs, dt, lane, s_ar, s_at, s_ak);
#pragma unroll
    for (int ii = 0; ii < kBI; ++ii) s_ip[ii * kBL + lane] = 0.0;
    box_factor(g, p, lane, D, s_w, s_ar, s_at, s_ak, s_ip, ip, flag);
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

// z = P^{-1} r for every component (out in PT); partial <r, z> per box
template <class PT>
__global__ __launch_bounds__(kBL) void k_bilu0_solve(Geo<double> g, int nc,
                                                     const double* __restrict__ coef, double cs,
                                                     double dt, const double* __restrict__ ip,
                                                     const double* __restrict__ r,
                                                     PT* __restrict__ out, double* part)
{
    __shared__ double s_w[kBC], s_ar[kBC], s_at[kBC], s_ak[kBC], s_ip[kBC];
    const int lane = threadIdx.x;
    const BoxPos p = box_pos(g, blockIdx.x, lane);
    box_couplings(g, p, coef, cs, dt, lane, s_ar, s_at, s_ak);
    load_ip(g, p, lane, ip, s_ip);
    const size_t N = (size_t)g.nr * g.P, base = (size_t)p.j * g.np + p.k;
    double rz = 0.0;
#pragma unroll 1
    for (int c = 0; c < nc; ++c) {
        double rv[kBI];
#pragma unroll
        for (int ii = 0; ii < kBI; ++ii) {
            rv[ii] = (p.col && ii < p.nib) ? r[c * N + (size_t)(p.i0 + ii) * g.P + base] : 0.0;
            s_w[ii * kBL + lane] = rv[ii];
        }
        __syncthreads();
        box_solve(p, lane, s_w, s_ar, s_at, s_ak, s_ip);
#pragma unroll
        for (int ii = 0; ii < kBI; ++ii)
            if (p.col && ii < p.nib) {
                const double z = s_w[ii * kBL + lane];
                out[c * N + (size_t)(p.i0 + ii) * g.P + base] = (PT)z;
                rz += rv[ii] * z;
            }
        __syncthreads();
    }
    rz = wave_sum(rz);
    if (lane == 0) part[blockIdx.x] = rz;
}

// x += alpha p, r -= alpha q, z = P^{-1} r; partials <r, z>, <r, r>
template <class PT>
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
    __shared__ double s_w[kBC], s_ar[kBC], s_at[kBC], s_ak[kBC], s_ip[kBC];
    const double alpha = st->alpha;
    const int lane = threadIdx.x;
    const BoxPos p = box_pos(g, blockIdx.x, lane);
    box_couplings(g, p, coef, cs, dt, lane, s_ar, s_at, s_ak);
    load_ip(g, p, lane, ip, s_ip);
    const size_t N = (size_t)g.nr * g.P, base = (size_t)p.j * g.np + p.k;
    double rz = 0.0, rr = 0.0;
#pragma unroll 1
    for (int c = 0; c < nc; ++c) {
        double xv[kBI], rv[kBI], pp[kBI], qq[kBI];
#pragma unroll
        for (int ii = 0; ii < kBI; ++ii) {
            const bool on = p.col && ii < p.nib;
            const size_t m = c * N + (size_t)(p.i0 + (on ? ii : 0)) * g.P + (on ? base : 0);
            xv[ii] = on ? x[m] : 0.0;
            rv[ii] = on ? r[m] : 0.0;
            pp[ii] = on ? (double)pv[m] : 0.0;
            qq[ii] = on ? (double)qv[m] : 0.0;
        }
#pragma unroll
        for (int ii = 0; ii < kBI; ++ii) {
            const double rn = rv[ii] - alpha * qq[ii];
            rv[ii] = rn;
            s_w[ii * kBL + lane] = rn;
            if (p.col && ii < p.nib) {
                const size_t m = c * N + (size_t)(p.i0 + ii) * g.P + base;
                x[m] = xv[ii] + alpha * pp[ii];
                r[m] = rn;
                rr += rn * rn;
            }
        }
        __syncthreads();
        box_solve(p, lane, s_w, s_ar, s_at, s_ak, s_ip);
#pragma unroll
        for (int ii = 0; ii < kBI; ++ii)
            if (p.col && ii < p.nib) {
                const double zv = s_w[ii * kBL + lane];
                z[c * N + (size_t)(p.i0 + ii) * g.P + base] = zv;
                rz += rv[ii] * zv;
            }
        __syncthreads();
    }
    rz = wave_sum(rz);
    rr = wave_sum(rr);
    if (lane == 0) {
        part[blockIdx.x] = rz;
        part[gridDim.x + blockIdx.x] = rr;
    }
}

}  // namespace

int bilu0_boxes(int nr, int nt, int np)
{
    return ((nr + kBI - 1) / kBI) * ((nt + kBJ - 1) / kBJ) * ((np + kBK - 1) / kBK);
}

void launch_bilu0_factor(const Geo<double>& g, const double* coef, double cs, double dt,
                         const double* D, double* ip, int* flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_bilu0_factor, dim3(bilu0_boxes(g.nr, g.nt, g.np)), dim3(kBL), 0, s, g,
                       coef, cs, dt, D, ip, flag);
}

template <class PT>
void launch_bilu0_solve(const Geo<double>& g, int nc, const double* coef, double cs, double dt,
                        const double* ip, const double* r, PT* out, double* part, int* nparts,
                        hipStream_t s)
{
    const int nb = bilu0_boxes(g.nr, g.nt, g.np);
    *nparts = nb;
    hipLaunchKernelGGL((k_bilu0_solve<PT>), dim3(nb), dim3(kBL), 0, s, g, nc, coef, cs, dt, ip, r,
                       out, part);
}
template void launch_bilu0_solve<double>(const Geo<double>&, int, const double*, double, double,
                                         const double*, const double*, double*, double*, int*,
                                         hipStream_t);
template void launch_bilu0_solve<float>(const Geo<double>&, int, const double*, double, double,
                                        const double*, const double*, float*, double*, int*,
                                        hipStream_t);

template <class PT>
void launch_pcg_update_bilu0(const Geo<double>& g, int nc, const double* coef, double cs,
                             double dt, const double* ip, double* x, double* r, const PT* p,
                             const PT* q, double* z, const DevState* st, double* part,
                             int* nparts, hipStream_t s)
{
    const int nb = bilu0_boxes(g.nr, g.nt, g.np);
    *nparts = nb;
    hipLaunchKernelGGL((k_pcg_update_bilu0<PT>), dim3(nb), dim3(kBL), 0, s, g, nc, coef, cs, dt,
                       ip, x, r, p, q, z, st, part);
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
