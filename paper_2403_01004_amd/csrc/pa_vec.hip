// pa_vec.hip -- reductions, the PTL finalisation and the PCG vector kernels
// (gfx950).  All reductions are deterministic: per-tile partials written by
// the producing kernel, then one workgroup sums them in a fixed order
// (strided per thread, then a fixed shuffle/LDS tree), so repeated runs are
// bitwise identical.  The PCG scalars (alpha, beta, rho, the stopping test)
// live on the device; a `done` flag turns the remaining kernels of a queued
// batch of iterations into no-ops once the solve has stopped.
#include "pa_internal.h"

namespace pa {

__device__ __forceinline__ double wsum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Streams read or written once per kernel bypass the caches' retention
// (non-temporal): measured on MI355X, 4 reads + 2 writes over 55 M doubles
// stream at 6.8 TB/s this way against 5.9 TB/s with ordinary accesses.
template <class T>
__device__ __forceinline__ T ldnt(const T* a) { return __builtin_nontemporal_load(a); }
template <class T>
__device__ __forceinline__ void stnt(T v, T* a) { __builtin_nontemporal_store(v, a); }

// Jacobi diagonal of a cell: from the rows (JacD) or the per-cell array.  The
// row form is one expression, so every kernel forms the same value.
__device__ __forceinline__ double jac_d(const JacD& jd, const double* Db, unsigned cell)
{
    if (!jd.ab) return Db[cell];
    const unsigned ij = cell / jd.np, k = cell - ij * jd.np;
    return fma(jd.vp[k], jd.ab[2 * ij], jd.ab[2 * ij + 1] * jd.G[k]);
}

// K sums of part[q*n .. q*n + n) by one workgroup of kRedBlock threads,
// results in thread 0.  The K arrays are read in the same loop, so their
// loads overlap (the stopping test needs two sums, the start of a solve
// three); each sum's order is fixed and independent of K.
template <int K>
__device__ void red_sums(const double* part, int n, double (&out)[K])
{
    __shared__ double lds[K][kRedBlock / 64];
    // eight independent accumulators per sum keep eight loads per sum in
    // flight per thread (the partials of a cell-sized grid number N / 512)
    const int bd = blockDim.x;
    double a[K][8];
#pragma unroll
    for (int q = 0; q < K; ++q)
#pragma unroll
        for (int t = 0; t < 8; ++t) a[q][t] = 0.0;
    int i = threadIdx.x;
    for (; i + 7 * bd < n; i += 8 * bd) {
#pragma unroll
        for (int q = 0; q < K; ++q)
#pragma unroll
            for (int t = 0; t < 8; ++t) a[q][t] += part[(size_t)q * n + i + t * bd];
    }
    for (; i < n; i += bd)
#pragma unroll
        for (int q = 0; q < K; ++q) a[q][0] += part[(size_t)q * n + i];
    double v[K];
#pragma unroll
    for (int q = 0; q < K; ++q)
        v[q] = wsum(((a[q][0] + a[q][1]) + (a[q][2] + a[q][3])) +
                    ((a[q][4] + a[q][5]) + (a[q][6] + a[q][7])));
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int q = 0; q < K; ++q) lds[q][threadIdx.x >> 6] = v[q];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < K; ++q) {
            double s = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += lds[q][w];
            out[q] = s;
        }
}

// sum of part[0..n) by one workgroup of kRedBlock threads; result in thread 0
__device__ double red_sum(const double* part, int n)
{
    double s[1] = {0.0};
    red_sums<1>(part, n, s);
    return s[0];
}

__global__ __launch_bounds__(kRedBlock) void k_reduce_max(const double* part, int n, double* outp)
{
    __shared__ double lds[kRedBlock / 64];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v = fmax(v, part[i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = lds[0];
        for (int w = 1; w < kRedBlock / 64; ++w) b = fmax(b, lds[w]);
        *outp = b;
    }
}

void launch_reduce_max(const double* part, int n, double* outp, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_max, dim3(1), dim3(kRedBlock), 0, s, part, n, outp);
}

// ---------------------------------------------------------------- PTL

__device__ __forceinline__ bool better(double v, long long i, double bv, long long bi)
{
    return v > bv || (v == bv && i < bi);
}

// argmax |F| over the per-tile partials (largest value, lowest index on
// ties), one workgroup of kRedBlock threads; the result is valid in thread 0
__device__ long long argmax_partials(const double* pval, const long long* pidx, int n)
{
    __shared__ double lv[kRedBlock / 64];
    __shared__ long long li[kRedBlock / 64];
    double v = -1.0;
    long long ix = 0x7fffffffffffffffLL;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        if (better(pval[i], pidx[i], v, ix)) { v = pval[i]; ix = pidx[i]; }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(v, o, 64);
        const long long oi = __shfl_xor(ix, o, 64);
        if (better(ov, oi, v, ix)) { v = ov; ix = oi; }
    }
    if ((threadIdx.x & 63) == 0) { lv[threadIdx.x >> 6] = v; li[threadIdx.x >> 6] = ix; }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int w = 1; w < kRedBlock / 64; ++w)
            if (better(lv[w], li[w], v, ix)) { v = lv[w]; ix = li[w]; }
    return ix;
}

// Eq. (ptl3): argmax |F| over the per-tile partials, then the minimum over
// the six face neighbours of -(u_k - u_nb)/(F_k - F_nb) where du, dF != 0 and
// du*dF < 0 (Eq. ptl2); +inf if none.  Neighbours: phi periodic, none across
// a pole or a radial boundary.  F is read at the cell and its neighbours only.
template <class T>
__global__ __launch_bounds__(kRedBlock) void k_ptl_finalize(const double* pval,
                                                            const long long* pidx, int n,
                                                            const T* u, const T* F, int nc,
                                                            int nr, int nt, int np, DevState* st)
{
    const long long ix = argmax_partials(pval, pidx, n);
    if (threadIdx.x != 0) return;
    const long long N = (long long)nc * nr * nt * np;
    if (ix < 0 || ix >= N) {  // every |F| was NaN
        st->kmax = -1;
        st->dt_ptl = __builtin_nan("");
        return;
    }
    const long long best = ix;
    const int k = (int)(best % np);
    const int j = (int)((best / np) % nt);
    const int i = (int)((best / ((long long)np * nt)) % nr);
    const long long P = (long long)nt * np;
    long long nb[6];
    int nn = 0;
    if (i > 0) nb[nn++] = best - P;
    if (i < nr - 1) nb[nn++] = best + P;
    if (j > 0) nb[nn++] = best - np;
    if (j < nt - 1) nb[nn++] = best + np;
    nb[nn++] = best - k + (k == 0 ? np - 1 : k - 1);
    nb[nn++] = best - k + (k == np - 1 ? 0 : k + 1);
    double dt = __builtin_inf();
    const double uk = (double)u[best], Fk = (double)F[best];
    for (int q = 0; q < nn; ++q) {
        const double du = uk - (double)u[nb[q]];
        const double dF = Fk - (double)F[nb[q]];
        if (du != 0.0 && dF != 0.0 && du * dF < 0.0) {
            const double c = -du / dF;
            if (c < dt) dt = c;
        }
    }
    st->kmax = best;
    st->dt_ptl = dt;
}

// the argmax step of Eq. (ptl3) alone: st->kmax (-1 when every |F| is NaN)
__global__ __launch_bounds__(kRedBlock) void k_argmax(const double* pval, const long long* pidx,
                                                      int n, long long N, DevState* st)
{
    const long long ix = argmax_partials(pval, pidx, n);
    if (threadIdx.x == 0) st->kmax = (ix < 0 || ix >= N) ? -1 : ix;
}

void launch_argmax(const double* pval, const long long* pidx, int n, long long N, DevState* st,
                   hipStream_t s)
{
    hipLaunchKernelGGL(k_argmax, dim3(1), dim3(kRedBlock), 0, s, pval, pidx, n, N, st);
}

template <class T>
void launch_ptl_finalize(const double* pval, const long long* pidx, int n, const T* u, const T* F,
                         int nc, int nr, int nt, int np, DevState* st, hipStream_t s)
{
    hipLaunchKernelGGL((k_ptl_finalize<T>), dim3(1), dim3(kRedBlock), 0, s, pval, pidx, n, u, F,
                       nc, nr, nt, np, st);
}
template void launch_ptl_finalize<double>(const double*, const long long*, int, const double*,
                                          const double*, int, int, int, int, DevState*, hipStream_t);
template void launch_ptl_finalize<float>(const double*, const long long*, int, const float*,
                                         const float*, int, int, int, int, DevState*, hipStream_t);

// Full-grid limit: the minimum of Eq. (ptl2) over every cell and each of
// its face neighbours (same pairs as Eq. ptl3, at all cells instead of the
// argmax of |F|).  Per-block partials (value, lowest cell index attaining it)
// then a one-workgroup finish into st->dt_full / st->kfull.
template <class T>
__global__ __launch_bounds__(kBlock) void k_ptl_full(const T* u, const T* F, int nc, int nr, int nt,
                                                     int np, double* pval, long long* pidx)
{
    __shared__ double lv[kBlock / 64];
    __shared__ long long li[kBlock / 64];
    const long long P = (long long)nt * np, N = (long long)nr * P, NT = N * nc;
    double best = __builtin_inf();
    long long bi = 0x7fffffffffffffffLL;
    for (long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x; m < NT;
         m += (long long)gridDim.x * blockDim.x) {
        const long long cell = m % N;
        const int i = (int)(cell / P);
        const int pp = (int)(cell - (long long)i * P);
        const int j = pp / np, k = pp - j * np;
        long long nb[6];
        int nn = 0;
        if (i > 0) nb[nn++] = m - P;
        if (i < nr - 1) nb[nn++] = m + P;
        if (j > 0) nb[nn++] = m - np;
        if (j < nt - 1) nb[nn++] = m + np;
        nb[nn++] = m - k + (k == 0 ? np - 1 : k - 1);
        nb[nn++] = m - k + (k == np - 1 ? 0 : k + 1);
        const double um = (double)u[m], Fm = (double)F[m];
        for (int q = 0; q < nn; ++q) {
            const double du = um - (double)u[nb[q]];
            const double dF = Fm - (double)F[nb[q]];
            if (du != 0.0 && dF != 0.0 && du * dF < 0.0) {
                const double c = -du / dF;
                if (c < best || (c == best && m < bi)) { best = c; bi = m; }
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(best, o, 64);
        const long long oi = __shfl_xor(bi, o, 64);
        if (ov < best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if ((threadIdx.x & 63) == 0) { lv[threadIdx.x >> 6] = best; li[threadIdx.x >> 6] = bi; }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int w = 1; w < kBlock / 64; ++w)
        if (lv[w] < best || (lv[w] == best && li[w] < bi)) { best = lv[w]; bi = li[w]; }
    pval[blockIdx.x] = best;
    pidx[blockIdx.x] = bi;
}

__global__ __launch_bounds__(kRedBlock) void k_ptl_full_finish(const double* pval,
                                                               const long long* pidx, int n,
                                                               DevState* st)
{
    __shared__ double lv[kRedBlock / 64];
    __shared__ long long li[kRedBlock / 64];
    double best = __builtin_inf();
    long long bi = 0x7fffffffffffffffLL;
    for (int q = threadIdx.x; q < n; q += blockDim.x)
        if (pval[q] < best || (pval[q] == best && pidx[q] < bi)) { best = pval[q]; bi = pidx[q]; }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(best, o, 64);
        const long long oi = __shfl_xor(bi, o, 64);
        if (ov < best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if ((threadIdx.x & 63) == 0) { lv[threadIdx.x >> 6] = best; li[threadIdx.x >> 6] = bi; }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int w = 1; w < kRedBlock / 64; ++w)
        if (lv[w] < best || (lv[w] == best && li[w] < bi)) { best = lv[w]; bi = li[w]; }
    st->dt_full = best;
    st->kfull = best < __builtin_inf() ? bi : -1;
}

template <class T>
void launch_ptl_full(const T* u, const T* F, int nc, int nr, int nt, int np, double* pval,
                     long long* pidx, DevState* st, hipStream_t s)
{
    const size_t NT = (size_t)nc * nr * nt * np;
    size_t nb = (NT + kBlock - 1) / kBlock;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL((k_ptl_full<T>), dim3((unsigned)nb), dim3(kBlock), 0, s, u, F, nc, nr, nt, np,
                       pval, pidx);
    hipLaunchKernelGGL(k_ptl_full_finish, dim3(1), dim3(kRedBlock), 0, s, pval, pidx, (int)nb, st);
}
template void launch_ptl_full<double>(const double*, const double*, int, int, int, int, double*,
                                      long long*, DevState*, hipStream_t);

// ---------------------------------------------------------------- PCG

// two cells per thread: a grid of many short-lived workgroups keeps more
// loads in flight than a grid-stride loop over a few thousand (measured on
// MI355X: 4 reads + 2 writes stream at 5.3 TB/s with 65536 workgroups of
// 256 threads, 4.6 TB/s with 4096), and two cells per thread halve the
// partials the one-workgroup reductions sum, at the same bandwidth.
static int vec_blocks(size_t n)
{
    return (int)((n + 2 * kBlock - 1) / (2 * kBlock));
}

// deterministic per-block sums of up to 3 accumulators into part[q*nb + b]:
// every wave's sums go to LDS together, one barrier, then thread 0 adds
// the waves' values in order (called once per kernel: nothing waits for
// thread 0 to finish reading the LDS)
template <int NV>
__device__ __forceinline__ void block_partials(const double (&v)[NV], double* part)
{
    __shared__ double lds[NV][kBlock / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double x[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) x[q] = wsum(v[q]);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) lds[q][w] = x[q];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double sacc = 0.0;
            for (int t = 0; t < kBlock / 64; ++t) sacc += lds[q][t];
            part[(size_t)q * gridDim.x + blockIdx.x] = sacc;
        }
}

// Start of a Backward Euler solve, per cell (all components):
// D = V + dt diag(L) (stored), b = V (u + dt hF) with hF = F(0) the
// boundary-data part of F (read on the two radial boundary levels only; may
// be null when both sides are no-flux), r0 = b - M u = dt V F(u) (y0 from
// the PTL pass), p = r0/D.  Writes D, r, p (and b when bout != null);
// partials <r,z>, <r,r>, <b,b>.
template <class PT>
__global__ __launch_bounds__(kBlock) void k_pcg_init(Geo<double> g, int nc, double dt,
                                                     const double* w, const double* u,
                                                     const double* y0,
                                                     const double* hF, const double* dL,
                                                     double* Dout, double* r, PT* p, double* bout,
                                                     double* part, JacD jd)
{
    const int nr = g.nr, np = g.np;
    const unsigned P = (unsigned)g.P, N = (unsigned)nr * P;
    double acc[3] = {0.0, 0.0, 0.0};
    for (unsigned cell = blockIdx.x * blockDim.x + threadIdx.x; cell < N;
         cell += gridDim.x * blockDim.x) {
        const unsigned i = cell / P, pp = cell - i * P, j = pp / (unsigned)np, k = pp - j * np;
        const double V = g.vr[i] * g.vt[j] * g.vp[k] * (w ? w[cell] : 1.0);  // w V
        const double D = jd.ab ? jac_d(jd, nullptr, cell) : V + dt * dL[cell];
        Dout[cell] = D;
        const bool bnd = hF && (i == 0 || i == (unsigned)nr - 1);
        for (int c = 0; c < nc; ++c) {
            const size_t m = (size_t)c * N + cell;
            const double h = bnd ? hF[m] : 0.0;
            const double b = V * ldnt(u + m) + dt * V * h;
            const double rv = dt * V * ldnt(y0 + m);
            const double z = rv / D;
            stnt(rv, r + m);
            stnt((PT)z, p + m);
            if (bout) stnt(b, bout + m);
            acc[0] += rv * z;
            acc[1] += rv * rv;
            acc[2] += b * b;
        }
    }
    block_partials<3>(acc, part);
}

template <class PT>
void launch_pcg_init(const Geo<double>& g, int nc, double dt, const double* w, const double* u,
                     const double* y0, const double* hF, const double* diagL, double* D, double* r,
                     PT* p, double* b, double* part, int* nparts, hipStream_t s, const JacD& jd)
{
    const int nb = vec_blocks((size_t)g.nr * g.P);
    *nparts = nb;
    hipLaunchKernelGGL((k_pcg_init<PT>), dim3(nb), dim3(kBlock), 0, s, g, nc, dt, w, u, y0, hF,
                       diagL, D, r, p, b, part, jd);
}
template void launch_pcg_init<double>(const Geo<double>&, int, double, const double*, const double*,
                                      const double*, const double*, const double*, double*,
                                      double*, double*, double*, double*, int*, hipStream_t,
                                      const JacD&);
template void launch_pcg_init<float>(const Geo<double>&, int, double, const double*, const double*,
                                     const double*, const double*, const double*, double*,
                                     double*, float*, double*, double*, int*, hipStream_t,
                                     const JacD&);

// Defect correction: r = b - q (q = M x from an FP64 matvec), p = r/D;
// partials <r,z>, <r,r>, <b,b>.
template <class PT>
__global__ __launch_bounds__(kBlock) void k_pcg_resid(unsigned N, int nc, const double* b,
                                                      const double* q, const double* D, double* r,
                                                      PT* p, double* part)
{
    double acc[3] = {0.0, 0.0, 0.0};
    for (unsigned cell = blockIdx.x * blockDim.x + threadIdx.x; cell < N;
         cell += gridDim.x * blockDim.x) {
        const double d = D[cell];
        for (int c = 0; c < nc; ++c) {
            const size_t m = (size_t)c * N + cell;
            const double bv = ldnt(b + m);
            const double rv = bv - ldnt(q + m);
            const double z = rv / d;
            stnt(rv, r + m);
            stnt((PT)z, p + m);
            acc[0] += rv * z;
            acc[1] += rv * rv;
            acc[2] += bv * bv;
        }
    }
    block_partials<3>(acc, part);
}

template <class PT>
void launch_pcg_resid(size_t N, int nc, const double* b, const double* q, const double* D,
                      double* r, PT* p, double* part, int* nparts, hipStream_t s)
{
    const int nb = vec_blocks(N);
    *nparts = nb;
    hipLaunchKernelGGL((k_pcg_resid<PT>), dim3(nb), dim3(kBlock), 0, s, (unsigned)N, nc, b, q, D, r,
                       p, part);
}
template void launch_pcg_resid<float>(size_t, int, const double*, const double*, const double*,
                                      double*, float*, double*, int*, hipStream_t);
template void launch_pcg_resid<double>(size_t, int, const double*, const double*, const double*,
                                       double*, double*, double*, int*, hipStream_t);

// mode 0: stop when ||r|| <= tol ||b||.  mode 1 (inner solve of a defect
// correction): stop when ||r|| <= eta ||r0|| or ||r|| <= tol ||b||.
__global__ __launch_bounds__(kRedBlock) void k_pcg_start(const double* part, int n, DevState* st,
                                                          double tol, int max_iter, int force_iters,
                                                          int mode, double eta)
{
    double sums[3] = {0.0, 0.0, 0.0};
    red_sums<3>(part, n, sums);
    const double rz = sums[0], rr = sums[1], bb = sums[2];
    if (threadIdx.x != 0) return;
    st->tol = tol;
    st->max_iter = max_iter;
    st->force_iters = force_iters;
    st->rho = rz;
    st->rr = rr;
    st->bb = bb;
    st->iters = 0;
    st->status = 0;
    st->done = 0;
    st->xpend = 0;
    st->mode = mode;
    st->rr0 = rr;
    st->eta = eta;
    if (!isfinite(rr) || !isfinite(bb)) { st->status = 6; st->done = 1; return; }
    if (st->force_iters <= 0 && sqrt(rr) <= st->tol * sqrt(bb)) st->done = 1;
}

void launch_pcg_start(const double* part, int n, DevState* st, double tol, int max_iter,
                      int force_iters, int mode, double eta, hipStream_t s)
{
    hipLaunchKernelGGL(k_pcg_start, dim3(1), dim3(kRedBlock), 0, s, part, n, st, tol, max_iter,
                       force_iters, mode, eta);
}

__global__ __launch_bounds__(kRedBlock) void k_pcg_alpha(const double* part, int n, DevState* st,
                                                          double* aslot)
{
    // first kernel of an iteration to see the state: the previous
    // iteration's x update has been applied by now (or recorded)
    if (aslot && threadIdx.x == 0) *aslot = 0.0;
    if (st->done) {
        if (threadIdx.x == 0) st->xpend = 0;
        return;
    }
    const double pq = red_sum(part, n);
    if (threadIdx.x != 0) return;
    st->xpend = 0;
    st->pq = pq;
    if (!(pq > 0.0) || !isfinite(pq)) { st->status = 5; st->done = 1; return; }
    st->alpha = st->rho / pq;
}

void launch_pcg_alpha(const double* part, int n, DevState* st, hipStream_t s, double* aslot)
{
    hipLaunchKernelGGL(k_pcg_alpha, dim3(1), dim3(kRedBlock), 0, s, part, n, st, aslot);
}

// r -= alpha q, z = r/D, and x += alpha p when XU (otherwise k_pcg_dir
// applies it: p is then read once per iteration instead of twice);
// partials <r,z>, <r,r>
template <class PT, bool XU>
__global__ __launch_bounds__(kBlock) void k_pcg_update(unsigned N, int nc,
                                                       const double* __restrict__ Db,
                                                       double* __restrict__ x,
                                                       double* __restrict__ r,
                                                       const PT* __restrict__ p,
                                                       const PT* __restrict__ q,
                                                       const DevState* st, double* part, JacD jd)
{
    if (st->done) return;
    const double alpha = st->alpha;
    double acc[2] = {0.0, 0.0};
    for (unsigned cell = blockIdx.x * blockDim.x + threadIdx.x; cell < N;
         cell += gridDim.x * blockDim.x) {
        const double D = jac_d(jd, Db, cell);
        for (int c = 0; c < nc; ++c) {
            const size_t m = (size_t)c * N + cell;
            if (XU) stnt(ldnt(x + m) + alpha * (double)ldnt(p + m), x + m);
            const double rv = ldnt(r + m) - alpha * (double)ldnt(q + m);
            stnt(rv, r + m);
            const double z = rv / D;
            acc[0] += rv * z;
            acc[1] += rv * rv;
        }
    }
    block_partials<2>(acc, part);
}

template <class PT>
void launch_pcg_update(size_t N, int nc, const double* D, double* x, double* r, const PT* p,
                       const PT* q, const DevState* st, double* part, int* nparts, hipStream_t s,
                       const JacD& jd)
{
    const int nb = vec_blocks(N);
    *nparts = nb;
    if (x)
        hipLaunchKernelGGL((k_pcg_update<PT, true>), dim3(nb), dim3(kBlock), 0, s, (unsigned)N, nc,
                           D, x, r, p, q, st, part, jd);
    else
        hipLaunchKernelGGL((k_pcg_update<PT, false>), dim3(nb), dim3(kBlock), 0, s, (unsigned)N, nc,
                           D, x, r, p, q, st, part, jd);
}
template void launch_pcg_update<double>(size_t, int, const double*, double*, double*, const double*,
                                        const double*, const DevState*, double*, int*, hipStream_t,
                                        const JacD&);
template void launch_pcg_update<float>(size_t, int, const double*, double*, double*, const float*,
                                       const float*, const DevState*, double*, int*, hipStream_t,
                                       const JacD&);

// stopping test and beta (PCG with rho = <r, z>)
__global__ __launch_bounds__(kRedBlock) void k_pcg_beta(const double* part, int n, DevState* st,
                                                         double* aslot)
{
    if (st->done) return;
    double sums[2] = {0.0, 0.0};
    red_sums<2>(part, n, sums);
    const double rz = sums[0], rr = sums[1];
    if (threadIdx.x != 0) return;
    st->iters += 1;
    st->xpend = 1;   // this iteration's update ran: its x update is due
    if (aslot) *aslot = st->alpha;
    st->rr = rr;
    if (!isfinite(rr)) { st->status = 6; st->done = 1; return; }
    if (st->force_iters > 0) {
        if (st->iters >= st->force_iters) { st->done = 1; return; }
    } else {
        if (sqrt(rr) <= st->tol * sqrt(st->bb)) { st->done = 1; return; }
        if (st->mode == 1 && sqrt(rr) <= st->eta * sqrt(st->rr0)) { st->done = 1; return; }
        if (st->iters >= st->max_iter) { st->status = 4; st->done = 1; return; }
    }
    st->beta = rz / st->rho;
    st->rho = rz;
}

void launch_pcg_beta(const double* part, int n, DevState* st, hipStream_t s, double* aslot)
{
    hipLaunchKernelGGL(k_pcg_beta, dim3(1), dim3(kRedBlock), 0, s, part, n, st, aslot);
}

// x += alpha p for the iteration whose update just ran (xpend: set by
// k_pcg_beta, cleared by the next k_pcg_alpha), then p = r/D + beta p while
// the solve goes on.  The iteration that stops the solve still applies its
// x update here.
template <class PT>
__global__ __launch_bounds__(kBlock) void k_pcg_dir(unsigned N, int nc,
                                                    const double* __restrict__ Db,
                                                    const double* __restrict__ r,
                                                    double* __restrict__ x,
                                                    PT* __restrict__ p, const DevState* st)
{
    if (!st->xpend) return;
    const double alpha = st->alpha, beta = st->beta;
    const bool more = !st->done;
    for (unsigned cell = blockIdx.x * blockDim.x + threadIdx.x; cell < N;
         cell += gridDim.x * blockDim.x) {
        const double D = more ? Db[cell] : 1.0;   // the last launch reads x and p only
        for (int c = 0; c < nc; ++c) {
            const size_t m = (size_t)c * N + cell;
            const double pv = (double)ldnt(p + m);
            stnt(ldnt(x + m) + alpha * pv, x + m);
            if (more) stnt((PT)(ldnt(r + m) / D + beta * pv), p + m);
        }
    }
}

template <class PT>
void launch_pcg_dir(size_t N, int nc, const double* D, const double* r, double* x, PT* p,
                    const DevState* st, hipStream_t s)
{
    const int nb = vec_blocks(N);
    hipLaunchKernelGGL((k_pcg_dir<PT>), dim3(nb), dim3(kBlock), 0, s, (unsigned)N, nc, D, r, x, p,
                       st);
}
template void launch_pcg_dir<double>(size_t, int, const double*, const double*, double*, double*,
                                     const DevState*, hipStream_t);
template void launch_pcg_dir<float>(size_t, int, const double*, const double*, double*, float*,
                                    const DevState*, hipStream_t);

// the direction of the next iteration into its own buffer, pn = r/D + beta p,
// while the solve goes on (the arithmetic of k_pcg_dir); the x update is
// deferred to k_pcg_xflush (the iteration's alpha recorded by k_pcg_beta)
template <class PT>
__global__ __launch_bounds__(kBlock) void k_pcg_dir_next(unsigned N, int nc,
                                                         const double* __restrict__ Db,
                                                         const double* __restrict__ r,
                                                         const PT* __restrict__ p,
                                                         PT* __restrict__ pn,
                                                         const DevState* st, JacD jd)
{
    if (!st->xpend || st->done) return;
    const double beta = st->beta;
    for (unsigned cell = blockIdx.x * blockDim.x + threadIdx.x; cell < N;
         cell += gridDim.x * blockDim.x) {
        const double D = jac_d(jd, Db, cell);
        for (int c = 0; c < nc; ++c) {
            const size_t m = (size_t)c * N + cell;
            stnt((PT)(ldnt(r + m) / D + beta * (double)ldnt(p + m)), pn + m);
        }
    }
}

template <class PT>
void launch_pcg_dir_next(size_t N, int nc, const double* D, const double* r, const PT* p, PT* pn,
                         const DevState* st, hipStream_t s, const JacD& jd)
{
    hipLaunchKernelGGL((k_pcg_dir_next<PT>), dim3(vec_blocks(N)), dim3(kBlock), 0, s, (unsigned)N,
                       nc, D, r, p, pn, st, jd);
}
template void launch_pcg_dir_next<double>(size_t, int, const double*, const double*,
                                          const double*, double*, const DevState*, hipStream_t,
                                          const JacD&);
template void launch_pcg_dir_next<float>(size_t, int, const double*, const double*, const float*,
                                         float*, const DevState*, hipStream_t, const JacD&);

// x += alpha_t p_t for t = 0 .. count - 1 in that order, the per-iteration
// update of k_pcg_dir applied for a group of iterations; a zero alpha (an
// iteration queued after the solve stopped, or one whose r update did not
// run) leaves x as it is, so its term is skipped
template <class PT>
__global__ __launch_bounds__(kBlock) void k_pcg_xflush(size_t n, double* __restrict__ x,
                                                       XSlots<PT> sl, const double* ahist,
                                                       int count)
{
    double a[kXGroup];
    bool any = false;
#pragma unroll
    for (int t = 0; t < kXGroup; ++t) {
        a[t] = t < count ? ahist[t] : 0.0;
        any = any || a[t] != 0.0;
    }
    if (!any) return;
    for (size_t m = (size_t)blockIdx.x * blockDim.x + threadIdx.x; m < n;
         m += (size_t)gridDim.x * blockDim.x) {
        double xv = ldnt(x + m);
#pragma unroll
        for (int t = 0; t < kXGroup; ++t)
            if (a[t] != 0.0) xv = xv + a[t] * (double)ldnt(sl.p[t] + m);
        stnt(xv, x + m);
    }
}

template <class PT>
void launch_pcg_xflush(size_t n, double* x, const XSlots<PT>& sl, const double* ahist, int count,
                       hipStream_t s)
{
    hipLaunchKernelGGL((k_pcg_xflush<PT>), dim3(vec_blocks(n)), dim3(kBlock), 0, s, n, x, sl, ahist,
                       count);
}
template void launch_pcg_xflush<double>(size_t, double*, const XSlots<double>&, const double*, int,
                                        hipStream_t);
template void launch_pcg_xflush<float>(size_t, double*, const XSlots<float>&, const double*, int,
                                       hipStream_t);

// p = z + beta p while the solve goes on, with z the preconditioned
// residual stored by a block preconditioner (all components, n = nc * N
// values); with XU, x += alpha p first, run condition as k_pcg_dir
template <class PT, bool XU>
__global__ __launch_bounds__(kBlock) void k_pcg_dir_z(size_t n, const double* __restrict__ z,
                                                      double* __restrict__ x,
                                                      PT* __restrict__ p, const DevState* st)
{
    if (XU ? !st->xpend : st->done) return;
    const double alpha = st->alpha, beta = st->beta;
    const bool more = !st->done;
    for (size_t m = (size_t)blockIdx.x * blockDim.x + threadIdx.x; m < n;
         m += (size_t)gridDim.x * blockDim.x) {
        const double pv = (double)ldnt(p + m);
        if (XU) stnt(ldnt(x + m) + alpha * pv, x + m);
        if (more) stnt((PT)(ldnt(z + m) + beta * pv), p + m);
    }
}

template <class PT>
void launch_pcg_dir_z(size_t n, const double* z, double* x, PT* p, const DevState* st,
                      hipStream_t s)
{
    if (x)
        hipLaunchKernelGGL((k_pcg_dir_z<PT, true>), dim3(vec_blocks(n)), dim3(kBlock), 0, s, n, z,
                           x, p, st);
    else
        hipLaunchKernelGGL((k_pcg_dir_z<PT, false>), dim3(vec_blocks(n)), dim3(kBlock), 0, s, n, z,
                           x, p, st);
}
template void launch_pcg_dir_z<double>(size_t, const double*, double*, double*, const DevState*,
                                       hipStream_t);
template void launch_pcg_dir_z<float>(size_t, const double*, double*, float*, const DevState*,
                                      hipStream_t);

// rho = <r, z> from the partials of a preconditioner applied after
// launch_pcg_start (which set rho for point Jacobi)
__global__ __launch_bounds__(kRedBlock) void k_pcg_set_rho(const double* part, int n, DevState* st)
{
    const double rz = red_sum(part, n);
    if (threadIdx.x == 0) st->rho = rz;
}

void launch_pcg_set_rho(const double* part, int n, DevState* st, hipStream_t s)
{
    hipLaunchKernelGGL(k_pcg_set_rho, dim3(1), dim3(kRedBlock), 0, s, part, n, st);
}

// ---------------------------------------------------------------- misc

__global__ void k_f64_to_f32(const double* a, float* b, size_t n)
{
    for (size_t m = (size_t)blockIdx.x * blockDim.x + threadIdx.x; m < n;
         m += (size_t)gridDim.x * blockDim.x)
        b[m] = (float)a[m];
}
__global__ void k_f32_to_f64(const float* a, double* b, size_t n)
{
    for (size_t m = (size_t)blockIdx.x * blockDim.x + threadIdx.x; m < n;
         m += (size_t)gridDim.x * blockDim.x)
        b[m] = (double)a[m];
}
__global__ void k_copy16(const uint4* a, uint4* b, size_t n)
{
    for (size_t m = (size_t)blockIdx.x * blockDim.x + threadIdx.x; m < n;
         m += (size_t)gridDim.x * blockDim.x)
        b[m] = a[m];
}
__global__ void k_copy1(const unsigned char* a, unsigned char* b, size_t n)
{
    for (size_t m = (size_t)blockIdx.x * blockDim.x + threadIdx.x; m < n;
         m += (size_t)gridDim.x * blockDim.x)
        b[m] = a[m];
}
__global__ void k_zero1(unsigned char* a, size_t n)
{
    for (size_t m = (size_t)blockIdx.x * blockDim.x + threadIdx.x; m < n;
         m += (size_t)gridDim.x * blockDim.x)
        a[m] = 0;
}
__global__ void k_nonfinite(const double* a, size_t n, int* flag)
{
    int bad = 0;
    for (size_t m = (size_t)blockIdx.x * blockDim.x + threadIdx.x; m < n;
         m += (size_t)gridDim.x * blockDim.x)
        if (!isfinite(a[m])) bad = 1;
    if (bad) atomicOr(flag, 1);
}

void launch_f64_to_f32(const double* a, float* b, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_f64_to_f32, dim3(vec_blocks(n)), dim3(kBlock), 0, s, a, b, n);
}
void launch_f32_to_f64(const float* a, double* b, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_f32_to_f64, dim3(vec_blocks(n)), dim3(kBlock), 0, s, a, b, n);
}
void launch_copy(const void* a, void* b, size_t bytes, hipStream_t s)
{
    if (((uintptr_t)a % 16 == 0) && ((uintptr_t)b % 16 == 0) && bytes % 16 == 0)
        hipLaunchKernelGGL(k_copy16, dim3(vec_blocks(bytes / 16)), dim3(kBlock), 0, s,
                           (const uint4*)a, (uint4*)b, bytes / 16);
    else
        hipLaunchKernelGGL(k_copy1, dim3(vec_blocks(bytes)), dim3(kBlock), 0, s,
                           (const unsigned char*)a, (unsigned char*)b, bytes);
}
void launch_fill_zero(void* a, size_t bytes, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero1, dim3(vec_blocks(bytes)), dim3(kBlock), 0, s, (unsigned char*)a,
                       bytes);
}
__global__ void k_nonpositive(const double* a, size_t n, int* flag)
{
    for (size_t m = (size_t)blockIdx.x * blockDim.x + threadIdx.x; m < n;
         m += (size_t)gridDim.x * blockDim.x)
        if (!(a[m] > 0.0) || !isfinite(a[m])) atomicOr(flag, 1);
}

void launch_nonpositive(const double* a, size_t n, int* flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_nonpositive, dim3(vec_blocks(n)), dim3(kBlock), 0, s, a, n, flag);
}

void launch_nonfinite(const double* a, size_t n, int* flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_nonfinite, dim3(vec_blocks(n)), dim3(kBlock), 0, s, a, n, flag);
}

}  // namespace pa
