// pa_setup.hip -- per-advance set-up kernels (gfx950): lagged cell coefficients,
// field-aligned corner coefficients, the diagonal of L and the Gershgorin
// bound that gives the explicit Euler limit.
#include "pa_internal.h"

namespace pa {


// c = scale f_c(r_i) f_m(T0) T0^expo (f_m: the conductivity held at its Tc
// value below Tc, Tc <= 0 for none), or scale f_c(r_i) without T0; f_c may
// be null (1)
__global__ void k_coef(const double* T0, double scale, double expo, const double* fc, double Tc,
                       int P, int n, double* c64, float* c32, int* flag)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const double prof = fc ? fc[m / P] : 1.0;
    double c = scale * prof;
    if (T0) {
        const double Te = (Tc > 0.0 && T0[m] < Tc) ? Tc : T0[m];
        c = scale * prof * pow(Te, expo);
    }
    if (!isfinite(c) || c < 0.0) atomicOr(flag, 1);
    c64[m] = c;
    if (c32) c32[m] = (float)c;
}

void launch_coef(const double* T0, double scale, double expo, const double* fc, double Tc, int P,
                 int n, double* c64, float* c32, int* flag, hipStream_t s)
{
    hipLaunchKernelGGL(k_coef, dim3((n + 255) / 256), dim3(256), 0, s, T0, scale, expo, fc, Tc, P, n,
                       c64, c32, flag);
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

// diag(L) and the Gershgorin row bound sum_n |L_mn| / (w_m V_m) (per-block
// maxima; w the cell weight, null for 1)
__global__ __launch_bounds__(kBlock) void k_diag_iso7(Geo<double> g, const double* coef,
                                                      double cs, const double* w, int bc_in,
                                                      int bc_out, double* diag, double* part)
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
        rho = (d + off) / (g.vr[i] * vt * vp * (w ? w[m] : 1.0));
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
                                                         const double* wc, int bc_in, int bc_out,
                                                         double* diag, double* part)
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
        rho = s / (g.vr[i] * g.vt[j] * g.vp[k] * (wc ? wc[m] : 1.0));
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

void launch_diag_iso7(const Geo<double>& g, const double* coef, double cs, const double* w,
                      int bc_in, int bc_out, double* diag, double* part, hipStream_t s, int* nparts)
{
    const size_t N = (size_t)g.nr * g.P;
    const int nb = (int)((N + kBlock - 1) / kBlock);
    *nparts = nb;
    hipLaunchKernelGGL(k_diag_iso7, dim3(nb), dim3(kBlock), 0, s, g, coef, cs, w, bc_in, bc_out, diag,
                       part);
}

// Row form of the BE Jacobi diagonal D = V + dt diag(L) for the 7-point
// operator with the constant coefficient cs and no weight (the terms of
// k_diag_iso7 with every face coefficient equal to cs): every term carries
// either vp_k (cell volume, radial and colatitude faces) or gpp_k, gpp_{k+1}
// (the two longitude faces), so D = vp_k A_ij + B_ij G_k with
// A_ij = vr_i vt_j + dt cs (vt_j (gr_lo + gr_hi) + gtr_i (gtt_lo + gtt_hi)),
// B_ij = dt cs gtr_i gpt_j, G_k = gpp_k + gpp_{k+1}.
__global__ __launch_bounds__(kBlock) void k_jacobi_rows(Geo<double> g, double cs, int bc_in,
                                                        int bc_out, double dt, double* ab,
                                                        double* G)
{
    const int nr = g.nr, nt = g.nt, np = g.np;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < np) G[t] = g.gpp[t] + g.gpp[t == np - 1 ? 0 : t + 1];
    if (t >= nr * nt) return;
    const int i = t / nt, j = t - i * nt;
    const double grl = (i > 0 || bc_in == 0) ? g.gr[i] : 0.0;
    const double grh = (i < nr - 1 || bc_out == 0) ? g.gr[i + 1] : 0.0;
    const double gtl = j > 0 ? g.gtt[j] : 0.0;
    const double gth = j < nt - 1 ? g.gtt[j + 1] : 0.0;
    const double q = cs * (g.vt[j] * (grl + grh) + g.gtr[i] * (gtl + gth));
    ab[2 * t] = g.vr[i] * g.vt[j] + dt * q;
    ab[2 * t + 1] = dt * cs * g.gtr[i] * g.gpt[j];
}

void launch_jacobi_rows(const Geo<double>& g, double cs, int bc_in, int bc_out, double dt,
                        double* ab, double* G, hipStream_t s)
{
    const int n = g.nr * g.nt > g.np ? g.nr * g.nt : g.np;
    hipLaunchKernelGGL(k_jacobi_rows, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, g, cs,
                       bc_in, bc_out, dt, ab, G);
}

void launch_diag_aligned(const Geo<double>& g, const double* e, const double* w, int bc_in,
                         int bc_out, double* diag, double* part, hipStream_t s, int* nparts)
{
    const size_t N = (size_t)g.nr * g.P;
    const int nb = (int)((N + kBlock - 1) / kBlock);
    *nparts = nb;
    hipLaunchKernelGGL(k_diag_aligned, dim3(nb), dim3(kBlock), 0, s, g, e, w, bc_in, bc_out, diag,
                       part);
}

// scatter weight of a cell with signs (sr, st, sp) relative to a corner of
// plane ic: interior 1/4 (sr er + st et + sp ep); at a Dirichlet radial
// boundary 1/2 sr er; at a no-flux one 1/2 (st et + sp ep)
__device__ __forceinline__ double corner_w(const double* e, size_t nco, size_t q, int ic, int nr,
                                           int bc_in, int bc_out, double sr, double st, double sp)
{
    const double er = e[q], et = e[nco + q], ep = e[2 * nco + q];
    if (ic > 0 && ic < nr) return 0.25 * (sr * er + st * et + sp * ep);
    const int bc = ic == 0 ? bc_in : bc_out;
    return bc == 0 ? 0.5 * sr * er : 0.5 * (st * et + sp * ep);
}

// Face couplings L_{m,nb} (nb = r-, r+, t-, t+, p-, p+).  7-point:
// -c_f A_f / d_f.  Corner operator: sum over the four corners the two cells
// share of w_{c,m} w_{c,nb} (L = sum_c v_c v_c^T).
__global__ void k_couplings(Geo<double> g, int op, const double* coef, double cs, const double* e,
                            int bc_in, int bc_out, double* out)
{
    const int nr = g.nr, nt = g.nt, np = g.np, P = g.P;
    const size_t N = (size_t)nr * P;
    const size_t m = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= N) return;
    const int i = (int)(m / P), pp = (int)(m % P), j = pp / np, k = pp % np;
    const int km = (k == 0) ? np - 1 : k - 1, kp = (k == np - 1) ? 0 : k + 1;
    double L[6] = {0, 0, 0, 0, 0, 0};
    if (op == 0) {
        auto cf = [&](size_t q) { return coef ? coef[q] : cs; };
        const double cc = cf(m), vt = g.vt[j], vp = g.vp[k];
        if (i > 0) L[0] = -0.5 * (cc + cf(m - P)) * (g.gr[i] * vt * vp);
        if (i < nr - 1) L[1] = -0.5 * (cc + cf(m + P)) * (g.gr[i + 1] * vt * vp);
        if (j > 0) L[2] = -0.5 * (cc + cf(m - np)) * (g.gtr[i] * g.gtt[j] * vp);
        if (j < nt - 1) L[3] = -0.5 * (cc + cf(m + np)) * (g.gtr[i] * g.gtt[j + 1] * vp);
        L[4] = -0.5 * (cc + cf(m - k + km)) * (g.gtr[i] * g.gpt[j] * g.gpp[k]);
        L[5] = -0.5 * (cc + cf(m - k + kp)) * (g.gtr[i] * g.gpt[j] * g.gpp[kp]);
    } else {
        const size_t nco = (size_t)(nr + 1) * (nt + 1) * np;
        auto cq = [&](int ic, int jc, int kc) { return ((size_t)ic * (nt + 1) + jc) * np + kc; };
        // corners of the shared face: two choices in each of the two
        // transverse directions; the cell's sign in a transverse direction is
        // +1 when it is the corner's upper cell there
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                // radial faces: corners jc = j + 1 - a, kc = (a? k : kp) pattern
                const int jc = j + 1 - a, kc = b ? k : kp;
                const double st = a ? 1.0 : -1.0, sp = b ? 1.0 : -1.0;
                if (jc > 0 && jc < nt) {
                    if (i > 0) {     // r-: plane ic = i, m upper (sr +1), nb lower
                        const size_t q = cq(i, jc, kc);
                        L[0] += corner_w(e, nco, q, i, nr, bc_in, bc_out, 1.0, st, sp) *
                                corner_w(e, nco, q, i, nr, bc_in, bc_out, -1.0, st, sp);
                    }
                    if (i < nr - 1) {  // r+: plane ic = i + 1, m lower
                        const size_t q = cq(i + 1, jc, kc);
                        L[1] += corner_w(e, nco, q, i + 1, nr, bc_in, bc_out, -1.0, st, sp) *
                                corner_w(e, nco, q, i + 1, nr, bc_in, bc_out, 1.0, st, sp);
                    }
                }
                // colatitude faces: corners ic = i + 1 - a, kc as above
                const int ic = i + 1 - a;
                const double sr = a ? 1.0 : -1.0;
                if (j > 0) {         // t-: corner row jc = j, m upper
                    const size_t q = cq(ic, j, kc);
                    L[2] += corner_w(e, nco, q, ic, nr, bc_in, bc_out, sr, 1.0, sp) *
                            corner_w(e, nco, q, ic, nr, bc_in, bc_out, sr, -1.0, sp);
                }
                if (j < nt - 1) {    // t+: corner row jc = j + 1, m lower
                    const size_t q = cq(ic, j + 1, kc);
                    L[3] += corner_w(e, nco, q, ic, nr, bc_in, bc_out, sr, -1.0, sp) *
                            corner_w(e, nco, q, ic, nr, bc_in, bc_out, sr, 1.0, sp);
                }
                // longitude faces: corners ic = i + 1 - a, jc = j + 1 - b
                const int jc2 = j + 1 - b;
                const double st2 = b ? 1.0 : -1.0;
                if (jc2 > 0 && jc2 < nt) {
                    size_t q = cq(ic, jc2, k);     // p-: corner column kc = k, m upper
                    L[4] += corner_w(e, nco, q, ic, nr, bc_in, bc_out, sr, st2, 1.0) *
                            corner_w(e, nco, q, ic, nr, bc_in, bc_out, sr, st2, -1.0);
                    q = cq(ic, jc2, kp);           // p+: corner column kc = k + 1, m lower
                    L[5] += corner_w(e, nco, q, ic, nr, bc_in, bc_out, sr, st2, -1.0) *
                            corner_w(e, nco, q, ic, nr, bc_in, bc_out, sr, st2, 1.0);
                }
            }
    }
    for (int q = 0; q < 6; ++q) out[(size_t)q * N + m] = L[q];
}

void launch_couplings(const Geo<double>& g, int op, const double* coef, double cs, const double* e,
                      int bc_in, int bc_out, double* out, hipStream_t s)
{
    const size_t N = (size_t)g.nr * g.P;
    hipLaunchKernelGGL(k_couplings, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, g, op, coef,
                       cs, e, bc_in, bc_out, out);
}

}  // namespace pa
