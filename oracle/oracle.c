/*
 * oracle.c -- plain, slow, FP64 CPU reference for the parabolic-operator
 * advance of Caplan et al., "Advancing parabolic operators in thermodynamic
 * MHD models II" (arXiv 2403.01004).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's GPU path includes,
 * links or calls this file; only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load it.  It shares no code, header or table
 * with the GPU path.
 *
 * What it computes, step by step in the paper's order:
 *   - the split parabolic operator F(u) of Eq. (par), in the two forms of
 *     Eq. (visc)/(tc): an isotropic 7-point finite-volume Laplacian with a
 *     cell coefficient c = scale * T0^expo (artificial viscosity; constant
 *     coefficient when T0 is absent) and a field-aligned conduction operator
 *     div(kappa bhat bhat . grad T) with lagged kappa = kappa0 T0^{5/2}.
 *     The paper gives only the continuous operators; the discretisation is
 *     this project's reading (finite volume on the spherical mesh; the
 *     field-aligned term as L = G^T W K G over cell corners, with G the
 *     corner gradient averaged over four cell-centre differences per
 *     direction, K = kappa bhat bhat^T and W the corner dual volume),
 *     which is symmetric positive semi-definite by construction; and the
 *     vector form of Eq. (visc) for a velocity in spherical components, the
 *     7-point operator on its Cartesian components written in each cell's
 *     spherical basis (faces couple a cell to its neighbour's vector
 *     rotated into that basis: the curvature coupling of the components);
 *   - the explicit Euler limit dt_E = 2 / rho, rho a Gershgorin bound on
 *     V^{-1} L (App. A uses dt_Euler without defining it);
 *   - the practical time step limit of Eqs. (ptl)-(ptl3): the one-sided
 *     ratio -(u_k - u_nb)/(F_k - F_nb) over the six face neighbours of the
 *     cell k where |F| is largest (Sec. 2);
 *   - dynamic cycling: the PTL re-evaluated after every cycle (Sec. 2, last
 *     paragraph), reading "number of cycles" as n = ceil(t_rem / dt_PTL)
 *     with the remaining time split equally, dt_c = t_rem / n;
 *   - RKG2 (alpha = 3/2) super time stepping with the coefficients of
 *     App. A, and RKL2 with the coefficients of Meyer, Balsara & Aslam
 *     (2014), the paper's reference for RKL2 (Sec. 3.1); stage counts from
 *     the App. A formula (RKG2) and its RKL2 analogue, with the odd-stage
 *     rule of Sec. 3.1 / App. A;
 *   - Backward Euler (Sec. 3.1) solved by textbook preconditioned conjugate
 *     gradients on the symmetric system (V + dt L) x = V u^n + dt h, with
 *     point Jacobi (PC1 of Sec. 3.1) or non-overlapping block ILU(0) (PC2 of
 *     Sec. 3.1): M restricted to boxes of cells, each box factored by
 *     incomplete LU with the sparsity of M (Saad's IKJ elimination, natural
 *     cell order).
 *
 * Index conventions: cell (c,i,j,k) -> ((c*nr+i)*nt+j)*np+k, k fastest;
 * corner (ic,jc,kc) with ic in [0,nr], jc in [0,nt], kc in [0,np) sits at
 * (r_faces[ic], t_faces[jc], p_faces[kc]) and touches cells
 * {ic-1,ic} x {jc-1,jc} x {kc-1,kc} (kc-1 taken periodically).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_api.h"

#define OR_ISO7 0
#define OR_ALIGNED 1
#define OR_VISCV 2   /* vector form of Eq. (visc), components (v_r, v_theta, v_phi) */
#define OR_DIRICHLET 0
#define OR_NOFLUX 1

struct or_ctx {
    int nr, nt, np, nc, op, bc_in, bc_out;
    double *R, *TH, *PH;     /* faces */
    double *rc, *tc, *pc;    /* centres */
    double *cth, *sth, *stc; /* cos, sin of the theta faces; sin of the theta centres */
    double *ctc, *cpc, *spc; /* cos of the theta centres; cos, sin of the phi centres */
    double period;
    double *coef;            /* cell coefficient c, [nr*nt*np] */
    double *bhat;            /* corner unit field [3][(nr+1)(nt+1)np] */
    double *ub_in, *ub_out;  /* [nc][nt][np] */
    double *fbuf;            /* corner flux scratch [3][(nr+1)(nt+1)np] */
    double *wgt;             /* cell weight w of F = (1/w) div(...), NULL: 1 */
    double *fc;              /* radial profile f_c [nr], NULL: 1 */
    double Tc;               /* f_m threshold, <= 0: f_m = 1 */
    int pcond;               /* BE preconditioner: 0 point Jacobi, 2 block ILU(0) */
    int pbi, pbj, pbk;       /* block ILU(0) box in cells (r, theta, phi) */
};

static size_t cell_ix(const or_ctx* o, int c, int i, int j, int k)
{
    return (((size_t)c * o->nr + i) * o->nt + j) * o->np + k;
}
static size_t corner_ix(const or_ctx* o, int ic, int jc, int kc)
{
    return ((size_t)ic * (o->nt + 1) + jc) * o->np + kc;
}
static size_t ncell(const or_ctx* o) { return (size_t)o->nr * o->nt * o->np; }
static size_t ncorner(const or_ctx* o) { return (size_t)(o->nr + 1) * (o->nt + 1) * o->np; }

/* ---------------------------------------------------------------- geometry */

/* finite-volume cell volume: integral of r^2 sin(theta) dr dtheta dphi */
double or_volume(const or_ctx* o, int i, int j, int k)
{
    const double* R = o->R;
    return (R[i + 1] * R[i + 1] * R[i + 1] - R[i] * R[i] * R[i]) / 3.0 *
           (o->cth[j] - o->cth[j + 1]) * (o->PH[k + 1] - o->PH[k]);
}

/* distance in phi between the centres of cells k-1 and k (periodic) */
static double dphi_centres(const or_ctx* o, int k)
{
    if (k == 0) return o->pc[0] + o->period - o->pc[o->np - 1];
    return o->pc[k] - o->pc[k - 1];
}

/* Face transmissibilities A_f / d_f (coefficient not included).
 * r-face "ir" lies at r_faces[ir], ir in [0,nr]. */
static double trans_r(const or_ctx* o, int ir, int j, int k)
{
    const double area = o->R[ir] * o->R[ir] * (o->cth[j] - o->cth[j + 1]) *
                        (o->PH[k + 1] - o->PH[k]);
    double d;
    if (ir == 0) d = o->rc[0] - o->R[0];
    else if (ir == o->nr) d = o->R[o->nr] - o->rc[o->nr - 1];
    else d = o->rc[ir] - o->rc[ir - 1];
    return area / d;
}
/* theta-face jt in [1,nt-1] between cells jt-1 and jt, at radius cell i */
static double trans_t(const or_ctx* o, int i, int jt, int k)
{
    const double area = o->sth[jt] * 0.5 * (o->R[i + 1] * o->R[i + 1] - o->R[i] * o->R[i]) *
                        (o->PH[k + 1] - o->PH[k]);
    const double d = o->rc[i] * (o->tc[jt] - o->tc[jt - 1]);
    return area / d;
}
/* phi-face between cells k-1 and k (periodic), at (i,j) */
static double trans_p(const or_ctx* o, int i, int j, int k)
{
    const double area = 0.5 * (o->R[i + 1] * o->R[i + 1] - o->R[i] * o->R[i]) *
                        (o->TH[j + 1] - o->TH[j]);
    const double d = o->rc[i] * o->stc[j] * dphi_centres(o, k);
    return area / d;
}

/* corner metric: centre-to-centre distances used by the corner gradient and
 * the corner dual volume W (half the radial extent at the two radial
 * boundaries, where one side of the corner is a mirror ghost cell). */
static void corner_metric(const or_ctx* o, int ic, int jc, int kc, double* hr, double* ht,
                          double* hp, double* W)
{
    double wr;
    if (ic == 0) {
        *hr = 2.0 * (o->rc[0] - o->R[0]);
        wr = 0.5 * *hr;
    } else if (ic == o->nr) {
        *hr = 2.0 * (o->R[o->nr] - o->rc[o->nr - 1]);
        wr = 0.5 * *hr;
    } else {
        *hr = o->rc[ic] - o->rc[ic - 1];
        wr = *hr;
    }
    *ht = o->R[ic] * (o->tc[jc] - o->tc[jc - 1]);
    *hp = o->R[ic] * o->sth[jc] * dphi_centres(o, kc);
    *W = wr * *ht * *hp;
}

/* ------------------------------------------------------------- lifecycle */

or_ctx* or_create(int nr, int nt, int np, int nc, const double* r_faces, const double* t_faces,
                  const double* p_faces, int op, int bc_in, int bc_out)
{
    if (nr < 1 || nt < 2 || np < 3 || nc < 1) return NULL;
    if (op == OR_VISCV && nc != 3) return NULL;
    or_ctx* o = (or_ctx*)calloc(1, sizeof(or_ctx));
    o->nr = nr; o->nt = nt; o->np = np; o->nc = nc; o->op = op;
    o->bc_in = bc_in; o->bc_out = bc_out;
    o->R = (double*)malloc(sizeof(double) * (nr + 1));
    o->TH = (double*)malloc(sizeof(double) * (nt + 1));
    o->PH = (double*)malloc(sizeof(double) * (np + 1));
    memcpy(o->R, r_faces, sizeof(double) * (nr + 1));
    memcpy(o->TH, t_faces, sizeof(double) * (nt + 1));
    memcpy(o->PH, p_faces, sizeof(double) * (np + 1));
    o->rc = (double*)malloc(sizeof(double) * nr);
    o->tc = (double*)malloc(sizeof(double) * nt);
    o->pc = (double*)malloc(sizeof(double) * np);
    for (int i = 0; i < nr; ++i) o->rc[i] = 0.5 * (o->R[i] + o->R[i + 1]);
    for (int j = 0; j < nt; ++j) o->tc[j] = 0.5 * (o->TH[j] + o->TH[j + 1]);
    for (int k = 0; k < np; ++k) o->pc[k] = 0.5 * (o->PH[k] + o->PH[k + 1]);
    /* the trigonometric factors of the metric, evaluated once */
    o->cth = (double*)malloc(sizeof(double) * (nt + 1));
    o->sth = (double*)malloc(sizeof(double) * (nt + 1));
    o->stc = (double*)malloc(sizeof(double) * nt);
    for (int j = 0; j <= nt; ++j) { o->cth[j] = cos(o->TH[j]); o->sth[j] = sin(o->TH[j]); }
    for (int j = 0; j < nt; ++j) o->stc[j] = sin(o->tc[j]);
    o->ctc = (double*)malloc(sizeof(double) * nt);
    o->cpc = (double*)malloc(sizeof(double) * np);
    o->spc = (double*)malloc(sizeof(double) * np);
    for (int j = 0; j < nt; ++j) o->ctc[j] = cos(o->tc[j]);
    for (int k = 0; k < np; ++k) { o->cpc[k] = cos(o->pc[k]); o->spc[k] = sin(o->pc[k]); }
    o->period = o->PH[np] - o->PH[0];
    o->coef = (double*)malloc(sizeof(double) * ncell(o));
    for (size_t m = 0; m < ncell(o); ++m) o->coef[m] = 1.0;
    o->ub_in = (double*)calloc((size_t)nc * nt * np, sizeof(double));
    o->ub_out = (double*)calloc((size_t)nc * nt * np, sizeof(double));
    if (op == OR_ALIGNED) {
        o->bhat = (double*)calloc(3 * ncorner(o), sizeof(double));
        o->fbuf = (double*)calloc(3 * ncorner(o), sizeof(double));
    }
    return o;
}

void or_destroy(or_ctx* o)
{
    if (!o) return;
    free(o->R); free(o->TH); free(o->PH); free(o->rc); free(o->tc); free(o->pc);
    free(o->cth); free(o->sth); free(o->stc); free(o->ctc); free(o->cpc); free(o->spc);
    free(o->coef); free(o->bhat); free(o->ub_in); free(o->ub_out); free(o->fbuf);
    free(o->wgt); free(o->fc);
    free(o);
}

/* Full forms of Eqs. (visc) and (tc): the weight w of F = (1/w) div(...)
 * (Eq. visc: rho; Eq. tc: 2 k rho / ((gamma - 1) m_p)), the radial profile
 * f_c(r) and the threshold Tc of f_m (the conductivity is held at its Tc
 * value below Tc: f_m(T0) T0^expo = Tc^expo there).  NULL / Tc <= 0: 1.
 * Copied; used from the next or_set_coefficients on.  Returns -1 on a
 * non-positive weight or a negative / non-finite profile value. */
int or_set_profile(or_ctx* o, const double* w, const double* fc, double Tc)
{
    const size_t n = ncell(o);
    free(o->wgt);
    free(o->fc);
    o->wgt = NULL;
    o->fc = NULL;
    o->Tc = Tc > 0.0 ? Tc : 0.0;
    if (w) {
        for (size_t m = 0; m < n; ++m)
            if (!(w[m] > 0.0) || !isfinite(w[m])) return -1;
        o->wgt = (double*)malloc(n * sizeof(double));
        memcpy(o->wgt, w, n * sizeof(double));
    }
    if (fc) {
        for (int i = 0; i < o->nr; ++i)
            if (!(fc[i] >= 0.0) || !isfinite(fc[i])) return -1;
        o->fc = (double*)malloc(o->nr * sizeof(double));
        memcpy(o->fc, fc, o->nr * sizeof(double));
    }
    return 0;
}

/* weighted cell volume w V: the factor of dF in the time derivative */
static double wvol(const or_ctx* o, int i, int j, int k)
{
    const double V = or_volume(o, i, j, k);
    return o->wgt ? V * o->wgt[cell_ix(o, 0, i, j, k)] : V;
}

double or_wvolume(const or_ctx* o, int i, int j, int k) { return wvol(o, i, j, k); }

/* all cell volumes V (weighted: w V) into out[nr][nt][np] */
void or_volumes(const or_ctx* o, int weighted, double* out)
{
    for (int i = 0; i < o->nr; ++i)
        for (int j = 0; j < o->nt; ++j)
            for (int k = 0; k < o->np; ++k)
                out[cell_ix(o, 0, i, j, k)] = weighted ? wvol(o, i, j, k) : or_volume(o, i, j, k);
}

/* Lagged diffusivity (Eq. tc, T0 = previous temperature):
 * c = scale * f_c(r_i) * f_m(T0) * T0^expo, or scale * f_c(r_i) when T0 is
 * NULL.  B: corner field, normalised here to bhat = B/|B| (zero where
 * |B| = 0).  Returns 0, or -1 on a non-finite or negative coefficient. */
int or_set_coefficients(or_ctx* o, const double* T0, double scale, double expo, const double* B)
{
    const size_t n = ncell(o);
    const size_t P = (size_t)o->nt * o->np;
    for (size_t m = 0; m < n; ++m) {
        const double prof = o->fc ? o->fc[m / P] : 1.0;
        double c = scale * prof;
        if (T0) {
            const double Te = (o->Tc > 0.0 && T0[m] < o->Tc) ? o->Tc : T0[m];
            c = scale * prof * pow(Te, expo);
        }
        if (!isfinite(c) || c < 0.0) return -1;
        o->coef[m] = c;
    }
    if (o->op == OR_ALIGNED) {
        if (!B) return -1;
        const size_t nn = ncorner(o);
        for (size_t q = 0; q < nn; ++q) {
            const double bx = B[q], by = B[nn + q], bz = B[2 * nn + q];
            const double mag = sqrt(bx * bx + by * by + bz * bz);
            if (!isfinite(mag)) return -1;
            if (mag > 0.0) {
                o->bhat[q] = bx / mag; o->bhat[nn + q] = by / mag; o->bhat[2 * nn + q] = bz / mag;
            } else {
                o->bhat[q] = o->bhat[nn + q] = o->bhat[2 * nn + q] = 0.0;
            }
        }
    }
    return 0;
}

void or_set_bc(or_ctx* o, const double* ub_in, const double* ub_out)
{
    const size_t n = (size_t)o->nc * o->nt * o->np;
    if (ub_in) memcpy(o->ub_in, ub_in, n * sizeof(double));
    if (ub_out) memcpy(o->ub_out, ub_out, n * sizeof(double));
}

/* --------------------------------------------------------------- operator */

/* Isotropic operator, one component:  (L u)_m = sum_f c_f (A_f/d_f)(u_m - u_nb)
 * with c_f the mean of the two cell coefficients; a Dirichlet radial face
 * couples to the boundary value with the cell's own coefficient over the half
 * cell distance; a no-flux face and the pole faces carry nothing.
 * F = -(L u - h)/V, h the boundary-data part (absent when affine == 0). */
static void apply_iso7(const or_ctx* o, int c, const double* u, double* F, int affine)
{
    const int nr = o->nr, nt = o->nt, np = o->np;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nt; ++j)
            for (int k = 0; k < np; ++k) {
                const size_t m = cell_ix(o, c, i, j, k);
                const size_t mc = cell_ix(o, 0, i, j, k);
                const double um = u[m], cm = o->coef[mc];
                double Lu = 0.0;
                /* radial faces */
                if (i > 0) {
                    const size_t nb = cell_ix(o, c, i - 1, j, k);
                    Lu += 0.5 * (cm + o->coef[cell_ix(o, 0, i - 1, j, k)]) * trans_r(o, i, j, k) * (um - u[nb]);
                } else if (o->bc_in == OR_DIRICHLET) {
                    const double ub = affine ? o->ub_in[((size_t)c * nt + j) * np + k] : 0.0;
                    Lu += cm * trans_r(o, 0, j, k) * (um - ub);
                }
                if (i < nr - 1) {
                    const size_t nb = cell_ix(o, c, i + 1, j, k);
                    Lu += 0.5 * (cm + o->coef[cell_ix(o, 0, i + 1, j, k)]) * trans_r(o, i + 1, j, k) * (um - u[nb]);
                } else if (o->bc_out == OR_DIRICHLET) {
                    const double ub = affine ? o->ub_out[((size_t)c * nt + j) * np + k] : 0.0;
                    Lu += cm * trans_r(o, nr, j, k) * (um - ub);
                }
                /* colatitude faces (none across a pole) */
                if (j > 0) {
                    const size_t nb = cell_ix(o, c, i, j - 1, k);
                    Lu += 0.5 * (cm + o->coef[cell_ix(o, 0, i, j - 1, k)]) * trans_t(o, i, j, k) * (um - u[nb]);
                }
                if (j < nt - 1) {
                    const size_t nb = cell_ix(o, c, i, j + 1, k);
                    Lu += 0.5 * (cm + o->coef[cell_ix(o, 0, i, j + 1, k)]) * trans_t(o, i, j + 1, k) * (um - u[nb]);
                }
                /* longitude faces (periodic) */
                {
                    const int km = (k + np - 1) % np, kp = (k + 1) % np;
                    Lu += 0.5 * (cm + o->coef[cell_ix(o, 0, i, j, km)]) * trans_p(o, i, j, k) * (um - u[cell_ix(o, c, i, j, km)]);
                    Lu += 0.5 * (cm + o->coef[cell_ix(o, 0, i, j, kp)]) * trans_p(o, i, j, kp) * (um - u[cell_ix(o, c, i, j, kp)]);
                }
                F[m] = -Lu / wvol(o, i, j, k);
            }
}

/* Spherical unit vectors at the centre of cell column (j,k), in Cartesian
 * components: e[0] = r-hat, e[1] = theta-hat, e[2] = phi-hat. */
static void centre_basis(const or_ctx* o, int j, int k, double e[3][3])
{
    const double st = o->stc[j], ct = o->ctc[j], cp = o->cpc[k], sp = o->spc[k];
    e[0][0] = st * cp; e[0][1] = st * sp; e[0][2] = ct;
    e[1][0] = ct * cp; e[1][1] = ct * sp; e[1][2] = -st;
    e[2][0] = -sp;     e[2][1] = cp;      e[2][2] = 0.0;
}

/* Change of basis between two cell columns: T[a][b] = e_a(j,k) . e_b(j2,k2),
 * so that sum_b T[a][b] v_b is component a, in the basis of (j,k), of the
 * vector whose components in the basis of (j2,k2) are v_b. */
static void change_of_basis(const or_ctx* o, int j, int k, int j2, int k2, double T[3][3])
{
    double e[3][3], f[3][3];
    centre_basis(o, j, k, e);
    centre_basis(o, j2, k2, f);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) T[a][b] = e[a][0] * f[b][0] + e[a][1] * f[b][1] + e[a][2] * f[b][2];
}

/* Vector form of Eq. (visc): v in spherical components (v_r, v_theta,
 * v_phi) at the cell centres.  div(c grad v) of a vector is the 7-point
 * operator of apply_iso7 acting on its Cartesian components; written in
 * each cell's own spherical basis, a face adds C_f (v_m - T v_nb), with T
 * the change of basis from the neighbour's unit vectors to the cell's (the
 * curvature coupling between the components).  Radial neighbours and the
 * radial boundary points share the cell's (theta, phi): there T = I, and
 * the Dirichlet data are spherical components at the boundary point. */
static void apply_viscv(const or_ctx* o, const double* u, double* F, int affine)
{
    const int nr = o->nr, nt = o->nt, np = o->np;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nt; ++j)
            for (int k = 0; k < np; ++k) {
                const size_t mc = cell_ix(o, 0, i, j, k);
                const double cm = o->coef[mc];
                double Lu[3] = {0.0, 0.0, 0.0};
                double um[3];
                for (int a = 0; a < 3; ++a) um[a] = u[cell_ix(o, a, i, j, k)];
                /* radial faces: same basis on both sides */
                if (i > 0) {
                    const double C = 0.5 * (cm + o->coef[cell_ix(o, 0, i - 1, j, k)]) * trans_r(o, i, j, k);
                    for (int a = 0; a < 3; ++a) Lu[a] += C * (um[a] - u[cell_ix(o, a, i - 1, j, k)]);
                } else if (o->bc_in == OR_DIRICHLET) {
                    const double C = cm * trans_r(o, 0, j, k);
                    for (int a = 0; a < 3; ++a) {
                        const double ub = affine ? o->ub_in[((size_t)a * nt + j) * np + k] : 0.0;
                        Lu[a] += C * (um[a] - ub);
                    }
                }
                if (i < nr - 1) {
                    const double C = 0.5 * (cm + o->coef[cell_ix(o, 0, i + 1, j, k)]) * trans_r(o, i + 1, j, k);
                    for (int a = 0; a < 3; ++a) Lu[a] += C * (um[a] - u[cell_ix(o, a, i + 1, j, k)]);
                } else if (o->bc_out == OR_DIRICHLET) {
                    const double C = cm * trans_r(o, nr, j, k);
                    for (int a = 0; a < 3; ++a) {
                        const double ub = affine ? o->ub_out[((size_t)a * nt + j) * np + k] : 0.0;
                        Lu[a] += C * (um[a] - ub);
                    }
                }
                /* colatitude and longitude faces: neighbour rotated into this cell's basis */
                const int km = (k + np - 1) % np, kp = (k + 1) % np;
                const int nbj[4] = {j - 1, j + 1, j, j}, nbk[4] = {k, k, km, kp};
                for (int f = 0; f < 4; ++f) {
                    const int j2 = nbj[f], k2 = nbk[f];
                    if (j2 < 0 || j2 >= nt) continue;   /* no face across a pole */
                    double C;
                    if (f == 0) C = trans_t(o, i, j, k);
                    else if (f == 1) C = trans_t(o, i, j + 1, k);
                    else if (f == 2) C = trans_p(o, i, j, k);
                    else C = trans_p(o, i, j, kp);
                    C *= 0.5 * (cm + o->coef[cell_ix(o, 0, i, j2, k2)]);
                    double T[3][3];
                    change_of_basis(o, j, k, j2, k2, T);
                    double vn[3];
                    for (int b = 0; b < 3; ++b) vn[b] = u[cell_ix(o, b, i, j2, k2)];
                    for (int a = 0; a < 3; ++a)
                        Lu[a] += C * (um[a] - (T[a][0] * vn[0] + T[a][1] * vn[1] + T[a][2] * vn[2]));
                }
                const double V = wvol(o, i, j, k);
                for (int a = 0; a < 3; ++a) F[cell_ix(o, a, i, j, k)] = -Lu[a] / V;
            }
}

/* For corner (ic,jc,kc): the value seen at slot (a,b,e) in {0,1}^3 (a radial:
 * 0 lower / 1 upper, b colatitude, e longitude).  Real cells give their
 * value; the mirror ghost across a radial boundary gives 2 u_b - u
 * (Dirichlet) or u (no flux), with u_b = 0 in linear mode. */
static void corner_values(const or_ctx* o, int c, const double* u, int ic, int jc, int kc,
                          int affine, double x[2][2][2])
{
    const int np = o->np, nt = o->nt;
    const int ks[2] = {(kc + np - 1) % np, kc};
    const int js[2] = {jc - 1, jc};
    for (int b = 0; b < 2; ++b)
        for (int e = 0; e < 2; ++e) {
            for (int a = 0; a < 2; ++a) {
                const int i = ic - 1 + a;
                if (i >= 0 && i < o->nr) x[a][b][e] = u[cell_ix(o, c, i, js[b], ks[e])];
            }
            if (ic == 0) {
                const double ur = x[1][b][e];
                const double ub = affine ? o->ub_in[((size_t)c * nt + js[b]) * np + ks[e]] : 0.0;
                x[0][b][e] = (o->bc_in == OR_DIRICHLET) ? 2.0 * ub - ur : ur;
            } else if (ic == o->nr) {
                const double ur = x[0][b][e];
                const double ub = affine ? o->ub_out[((size_t)c * nt + js[b]) * np + ks[e]] : 0.0;
                x[1][b][e] = (o->bc_out == OR_DIRICHLET) ? 2.0 * ub - ur : ur;
            }
        }
}

/* corner diffusivity: mean over the real cells touching the corner */
static double corner_kappa(const or_ctx* o, int ic, int jc, int kc)
{
    const int np = o->np;
    const int ks[2] = {(kc + np - 1) % np, kc};
    double s = 0.0;
    int n = 0;
    for (int a = 0; a < 2; ++a) {
        const int i = ic - 1 + a;
        if (i < 0 || i >= o->nr) continue;
        for (int b = 0; b < 2; ++b)
            for (int e = 0; e < 2; ++e) { s += o->coef[cell_ix(o, 0, i, jc - 1 + b, ks[e])]; ++n; }
    }
    return s / n;
}

/* d g_d / d u for the real cell in slot (a,b,e) of corner (ic,...), including
 * the chain rule through its mirror ghost at a radial boundary corner. */
static void corner_dgdu(const or_ctx* o, int ic, int a, int b, int e, double hr, double ht,
                        double hp, double dg[3])
{
    const double sr = a ? 1.0 : -1.0, st = b ? 1.0 : -1.0, sp = e ? 1.0 : -1.0;
    dg[0] = 0.25 * sr / hr; dg[1] = 0.25 * st / ht; dg[2] = 0.25 * sp / hp;
    int ghost = 0, bc = OR_NOFLUX;
    if (ic == 0) { ghost = 1; bc = o->bc_in; }
    if (ic == o->nr) { ghost = 1; bc = o->bc_out; }
    if (ghost) {
        const double s = (bc == OR_DIRICHLET) ? -1.0 : 1.0;   /* d u_ghost / d u */
        dg[0] += s * 0.25 * (-sr) / hr;
        dg[1] += s * 0.25 * st / ht;
        dg[2] += s * 0.25 * sp / hp;
    }
}

/* Field-aligned operator, one component.  Pass 1, per corner: the gradient
 * g (average of four centre differences per direction), flux
 * f = W kappa_c bhat (bhat . g).  Pass 2, per cell: (L u)_m = sum over the
 * corners touching m of f . dg/du_m  (that is L = G^T W K G), and
 * F = -(L u)/V.  Pole corners (jc = 0, nt) carry no flux. */
static void apply_aligned(or_ctx* o, int c, const double* u, double* F, int affine)
{
    const int nr = o->nr, nt = o->nt, np = o->np;
    const size_t nn = ncorner(o);
    double* f = o->fbuf;
#pragma omp parallel for schedule(static)
    for (int ic = 0; ic <= nr; ++ic)
        for (int jc = 0; jc <= nt; ++jc)
            for (int kc = 0; kc < np; ++kc) {
                const size_t q = corner_ix(o, ic, jc, kc);
                if (jc == 0 || jc == nt) { f[q] = f[nn + q] = f[2 * nn + q] = 0.0; continue; }
                double x[2][2][2], hr, ht, hp, W;
                corner_values(o, c, u, ic, jc, kc, affine, x);
                corner_metric(o, ic, jc, kc, &hr, &ht, &hp, &W);
                double g[3] = {0.0, 0.0, 0.0};
                for (int b = 0; b < 2; ++b)
                    for (int e = 0; e < 2; ++e) g[0] += x[1][b][e] - x[0][b][e];
                for (int a = 0; a < 2; ++a)
                    for (int e = 0; e < 2; ++e) g[1] += x[a][1][e] - x[a][0][e];
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) g[2] += x[a][b][1] - x[a][b][0];
                g[0] *= 0.25 / hr; g[1] *= 0.25 / ht; g[2] *= 0.25 / hp;
                const double* bh = o->bhat;
                const double b0 = bh[q], b1 = bh[nn + q], b2 = bh[2 * nn + q];
                const double bg = b0 * g[0] + b1 * g[1] + b2 * g[2];
                const double K = W * corner_kappa(o, ic, jc, kc);
                f[q] = K * b0 * bg; f[nn + q] = K * b1 * bg; f[2 * nn + q] = K * b2 * bg;
            }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nt; ++j)
            for (int k = 0; k < np; ++k) {
                double Lu = 0.0;
                for (int a = 0; a < 2; ++a)          /* corner radial index ic = i + 1 - a */
                    for (int b = 0; b < 2; ++b)
                        for (int e = 0; e < 2; ++e) {
                            const int ic = i + 1 - a, jc = j + 1 - b, kc = (k + 1 - e) % np;
                            if (jc == 0 || jc == nt) continue;
                            double hr, ht, hp, W, dg[3];
                            corner_metric(o, ic, jc, kc, &hr, &ht, &hp, &W);
                            /* the cell sits in slot (a,b,e) of that corner */
                            corner_dgdu(o, ic, a, b, e, hr, ht, hp, dg);
                            const size_t q = corner_ix(o, ic, jc, kc);
                            Lu += f[q] * dg[0] + f[nn + q] * dg[1] + f[2 * nn + q] * dg[2];
                        }
                F[cell_ix(o, c, i, j, k)] = -Lu / wvol(o, i, j, k);
            }
}

void or_apply(or_ctx* o, const double* u, double* F, int affine)
{
    if (o->op == OR_VISCV) {
        apply_viscv(o, u, F, affine);
        return;
    }
    for (int c = 0; c < o->nc; ++c) {
        if (o->op == OR_ISO7) apply_iso7(o, c, u, F, affine);
        else apply_aligned(o, c, u, F, affine);
    }
}

/* ------------------------------------------- diagonal and Euler limit */

/* Row data of L for cell (i,j,k): diag = L_mm and abs_row = a Gershgorin
 * bound on sum_n |L_mn| (exact for the 7-point operator; for the corner
 * operator the sum over corners of the row sums of each corner's rank-one
 * block, which bounds the exact row sum from above).  The vector form of
 * Eq. (visc) is the 7-point operator on the Cartesian components in a
 * rotated basis (an orthogonal similarity), so it has the 7-point
 * operator's diagonal and spectrum: its bound is the 7-point one. */
static void row_bounds(const or_ctx* o, int i, int j, int k, double* diag, double* absrow)
{
    const int nr = o->nr, nt = o->nt, np = o->np;
    double d = 0.0, s = 0.0;
    if (o->op == OR_ISO7 || o->op == OR_VISCV) {
        const double cm = o->coef[cell_ix(o, 0, i, j, k)];
        double off = 0.0, C;
        if (i > 0) { C = 0.5 * (cm + o->coef[cell_ix(o, 0, i - 1, j, k)]) * trans_r(o, i, j, k); d += C; off += C; }
        else if (o->bc_in == OR_DIRICHLET) d += cm * trans_r(o, 0, j, k);
        if (i < nr - 1) { C = 0.5 * (cm + o->coef[cell_ix(o, 0, i + 1, j, k)]) * trans_r(o, i + 1, j, k); d += C; off += C; }
        else if (o->bc_out == OR_DIRICHLET) d += cm * trans_r(o, nr, j, k);
        if (j > 0) { C = 0.5 * (cm + o->coef[cell_ix(o, 0, i, j - 1, k)]) * trans_t(o, i, j, k); d += C; off += C; }
        if (j < nt - 1) { C = 0.5 * (cm + o->coef[cell_ix(o, 0, i, j + 1, k)]) * trans_t(o, i, j + 1, k); d += C; off += C; }
        const int km = (k + np - 1) % np, kp = (k + 1) % np;
        C = 0.5 * (cm + o->coef[cell_ix(o, 0, i, j, km)]) * trans_p(o, i, j, k); d += C; off += C;
        C = 0.5 * (cm + o->coef[cell_ix(o, 0, i, j, kp)]) * trans_p(o, i, j, kp); d += C; off += C;
        s = d + off;
    } else {
        const size_t nn = ncorner(o);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int e = 0; e < 2; ++e) {
                    const int ic = i + 1 - a, jc = j + 1 - b, kc = (k + 1 - e) % np;
                    if (jc == 0 || jc == nt) continue;
                    double hr, ht, hp, W, dg[3];
                    corner_metric(o, ic, jc, kc, &hr, &ht, &hp, &W);
                    const size_t q = corner_ix(o, ic, jc, kc);
                    const double b0 = o->bhat[q], b1 = o->bhat[nn + q], b2 = o->bhat[2 * nn + q];
                    const double K = W * corner_kappa(o, ic, jc, kc);
                    corner_dgdu(o, ic, a, b, e, hr, ht, hp, dg);
                    const double vm = b0 * dg[0] + b1 * dg[1] + b2 * dg[2];
                    /* sum over the real cells n of this corner of |bhat . dg_n| */
                    double vsum = 0.0;
                    const int alo = (ic == 0) ? 1 : 0, ahi = (ic == nr) ? 0 : 1;
                    for (int a2 = alo; a2 <= ahi; ++a2)
                        for (int b2i = 0; b2i < 2; ++b2i)
                            for (int e2 = 0; e2 < 2; ++e2) {
                                double dn[3];
                                corner_dgdu(o, ic, a2, b2i, e2, hr, ht, hp, dn);
                                vsum += fabs(b0 * dn[0] + b1 * dn[1] + b2 * dn[2]);
                            }
                    d += K * vm * vm;
                    s += K * fabs(vm) * vsum;
                }
    }
    *diag = d;
    *absrow = s;
}

/* diag(L) into out[nr*nt*np] (same for every component) */
void or_diag(const or_ctx* o, double* out)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < o->nr; ++i)
        for (int j = 0; j < o->nt; ++j)
            for (int k = 0; k < o->np; ++k) {
                double d, s;
                row_bounds(o, i, j, k, &d, &s);
                out[cell_ix(o, 0, i, j, k)] = d;
            }
}

/* Explicit Euler limit dt_E = 2 / max_m (sum_n |L_mn|) / V_m. */
double or_dt_explicit(const or_ctx* o)
{
    double rho = 0.0;
    for (int i = 0; i < o->nr; ++i) {
        double rp = 0.0;
#pragma omp parallel for reduction(max : rp) schedule(static)
        for (int j = 0; j < o->nt; ++j)
            for (int k = 0; k < o->np; ++k) {
                double d, s;
                row_bounds(o, i, j, k, &d, &s);
                const double v = s / wvol(o, i, j, k);
                if (v > rp) rp = v;
            }
        if (rp > rho) rho = rp;
    }
    return rho > 0.0 ? 2.0 / rho : INFINITY;
}

/* ------------------------------------------------------ time step limit */

/* Eq. (ptl3): at the cell k of largest |F| (over components and cells, ties
 * to the lowest linear index), the minimum over the six face neighbours nb of
 * -(u_k - u_nb)/(F_k - F_nb), taken only where du != 0, dF != 0 and
 * du*dF < 0 (Eq. ptl2).  Neighbours: periodic in phi, none across a pole or
 * a radial boundary.  +inf when no neighbour constrains. */
double or_ptl_from(int nc, int nr, int nt, int np, const double* u, const double* F,
                   int64_t* kmax)
{
    const size_t n = (size_t)nc * nr * nt * np;
    size_t best = 0;
    double fbest = -1.0;
    for (size_t m = 0; m < n; ++m) {
        const double a = fabs(F[m]);
        if (a > fbest) { fbest = a; best = m; }
    }
    if (kmax) *kmax = (int64_t)best;
    const int k = (int)(best % np);
    const int j = (int)((best / np) % nt);
    const int i = (int)((best / ((size_t)np * nt)) % nr);
    const size_t base = best - ((size_t)i * nt + j) * np - k;   /* start of this component */
    size_t nb[6];
    int nnb = 0;
    if (i > 0) nb[nnb++] = base + ((size_t)(i - 1) * nt + j) * np + k;
    if (i < nr - 1) nb[nnb++] = base + ((size_t)(i + 1) * nt + j) * np + k;
    if (j > 0) nb[nnb++] = base + ((size_t)i * nt + j - 1) * np + k;
    if (j < nt - 1) nb[nnb++] = base + ((size_t)i * nt + j + 1) * np + k;
    nb[nnb++] = base + ((size_t)i * nt + j) * np + (k + np - 1) % np;
    nb[nnb++] = base + ((size_t)i * nt + j) * np + (k + 1) % np;
    double dt = INFINITY;
    for (int q = 0; q < nnb; ++q) {
        const double du = u[best] - u[nb[q]];
        const double dF = F[best] - F[nb[q]];
        if (du != 0.0 && dF != 0.0 && du * dF < 0.0) {
            const double cand = -du / dF;
            if (cand < dt) dt = cand;
        }
    }
    return dt;
}

/* Eq. (ptl2) minimised over every cell and every face direction (the
 * full-grid form the paper mentions before adopting the F_max shortcut). */
double or_ptl_fullgrid(int nc, int nr, int nt, int np, const double* u, const double* F)
{
    double dt = INFINITY;
    for (int c = 0; c < nc; ++c)
        for (int i = 0; i < nr; ++i)
            for (int j = 0; j < nt; ++j)
                for (int k = 0; k < np; ++k) {
                    const size_t m = (((size_t)c * nr + i) * nt + j) * np + k;
                    size_t nb[6];
                    int nnb = 0;
                    if (i > 0) nb[nnb++] = m - (size_t)nt * np;
                    if (i < nr - 1) nb[nnb++] = m + (size_t)nt * np;
                    if (j > 0) nb[nnb++] = m - np;
                    if (j < nt - 1) nb[nnb++] = m + np;
                    nb[nnb++] = m - k + (k + np - 1) % np;
                    nb[nnb++] = m - k + (k + 1) % np;
                    for (int q = 0; q < nnb; ++q) {
                        const double du = u[m] - u[nb[q]], dF = F[m] - F[nb[q]];
                        if (du != 0.0 && dF != 0.0 && du * dF < 0.0 && -du / dF < dt) dt = -du / dF;
                    }
                }
    return dt;
}

double or_ptl(or_ctx* o, const double* u, int64_t* kmax)
{
    const size_t n = (size_t)o->nc * ncell(o);
    double* F = (double*)malloc(n * sizeof(double));
    or_apply(o, u, F, 1);
    const double dt = or_ptl_from(o->nc, o->nr, o->nt, o->np, u, F, kmax);
    free(F);
    return dt;
}

/* ---------------------------------------------------------- STS tables */

/* Fills mu[k], nu[k], mut[k], gam[k] for k = 1..s (index 0 unused; at k=1
 * only mut[1] is used).  kind 0: RKL2 (Meyer, Balsara & Aslam 2014);
 * kind 1: RKG2 with alpha = 3/2 (App. A).  Returns -1 for s < 2. */
int or_sts_coeffs(int kind, int s, double* mu, double* nu, double* mut, double* gam)
{
    if (s < 2) return -1;
    double* b = (double*)malloc(sizeof(double) * (s + 1));
    for (int k = 0; k <= s; ++k) mu[k] = nu[k] = mut[k] = gam[k] = 0.0;
    if (kind == 0) {
        const double w1 = 4.0 / ((double)s * s + s - 2.0);
        for (int j = 0; j <= s; ++j)
            b[j] = (j <= 2) ? 1.0 / 3.0 : ((double)j * j + j - 2.0) / (2.0 * j * (j + 1.0));
        mut[1] = b[1] * w1;
        for (int j = 2; j <= s; ++j) {
            mu[j] = (2.0 * j - 1.0) / j * b[j] / b[j - 1];
            nu[j] = -(j - 1.0) / j * b[j] / b[j - 2];
            mut[j] = mu[j] * w1;
            gam[j] = -(1.0 - b[j - 1]) * mut[j];
        }
    } else {
        const double w = 6.0 / ((s + 4.0) * (s - 1.0));
        b[0] = 1.0;
        b[1] = 1.0 / 3.0;
        b[2] = 1.0 / 15.0;
        for (int k = 3; k <= s; ++k)
            b[k] = 4.0 * (k - 1.0) * (k + 4.0) / (3.0 * k * (k + 1.0) * (k + 2.0) * (k + 3.0));
        mu[1] = 1.0;
        mut[1] = w;
        mu[2] = 0.5;
        nu[2] = -0.1;
        mut[2] = mu[2] * w;
        gam[2] = 0.0;
        for (int k = 3; k <= s; ++k) {
            mu[k] = (2.0 + 1.0 / k) * b[k] / b[k - 1];
            nu[k] = -(1.0 / k + 1.0) * b[k] / b[k - 2];
            mut[k] = mu[k] * w;
            gam[k] = (k * (k + 1.0) / 2.0 * b[k - 1] - 1.0) * mut[k];
        }
    }
    free(b);
    return 0;
}

/* Stage count for ratio = dt / dt_E: RKG2 from App. A,
 * s = ceil(sqrt(25 + 24 ratio)/2 - 3/2); RKL2 from its stability bound
 * dt <= dt_E (s^2 + s - 2)/4, s = ceil((sqrt(9 + 16 ratio) - 1)/2).
 * At least 2; one more when even and force_odd (Sec. 3.1 / App. A). */
int or_sts_stages(int kind, double ratio, int force_odd)
{
    double x = (kind == 0) ? 0.5 * (sqrt(9.0 + 16.0 * ratio) - 1.0)
                           : 0.5 * sqrt(25.0 + 24.0 * ratio) - 1.5;
    int s = (int)ceil(x);
    if (s < 2) s = 2;
    if (force_odd && (s % 2 == 0)) s += 1;
    return s;
}

/* One STS cycle (App. A recurrence) of length dt with s stages, in place. */
static void sts_cycle(or_ctx* o, double* u, double dt, int kind, int s)
{
    const size_t n = (size_t)o->nc * ncell(o);
    double *mu = (double*)malloc(sizeof(double) * (s + 1)), *nu = (double*)malloc(sizeof(double) * (s + 1));
    double *mut = (double*)malloc(sizeof(double) * (s + 1)), *gam = (double*)malloc(sizeof(double) * (s + 1));
    or_sts_coeffs(kind, s, mu, nu, mut, gam);
    double* u0 = (double*)malloc(n * sizeof(double));
    double* y0 = (double*)malloc(n * sizeof(double));
    double* ukm2 = (double*)malloc(n * sizeof(double));
    double* ukm1 = (double*)malloc(n * sizeof(double));
    double* uk = (double*)malloc(n * sizeof(double));
    double* Fk = (double*)malloc(n * sizeof(double));
    memcpy(u0, u, n * sizeof(double));
    or_apply(o, u0, y0, 1);                                   /* y0 = F(u0) */
#pragma omp parallel for schedule(static)
    for (size_t m = 0; m < n; ++m) ukm1[m] = u0[m] + mut[1] * dt * y0[m];   /* u1 */
    memcpy(ukm2, u0, n * sizeof(double));
    for (int k = 2; k <= s; ++k) {
        or_apply(o, ukm1, Fk, 1);
#pragma omp parallel for schedule(static)
        for (size_t m = 0; m < n; ++m)
            uk[m] = mu[k] * ukm1[m] + nu[k] * ukm2[m] + (1.0 - mu[k] - nu[k]) * u0[m] +
                    mut[k] * dt * Fk[m] + gam[k] * dt * y0[m];
        double* t = ukm2; ukm2 = ukm1; ukm1 = uk; uk = t;
    }
    memcpy(u, ukm1, n * sizeof(double));
    free(mu); free(nu); free(mut); free(gam);
    free(u0); free(y0); free(ukm2); free(ukm1); free(uk); free(Fk);
}

/* ------------------------------------------------- block ILU(0) (PC2) */

/* PC2 of Sec. 3.1: non-overlapping ILU(0).  The paper names the method only
 * (its implementation is in the first paper of the series); the reading
 * here: the cells are split into boxes of pbi x pbj x pbk cells starting at
 * cell 0 in each direction (the last box in a direction may be short); the
 * preconditioner is P = L U with L U the incomplete LU factorisation, with
 * the sparsity of M and cells in their natural (i, j, k) order, of the
 * block-diagonal part of M = wV + dt L (every coupling between cells of
 * different boxes dropped).  The periodic phi coupling between k = np-1 and
 * k = 0 is always dropped, also when both cells lie in one box, so that each
 * box is a plain sub-grid.  Implemented for the 7-point operator and for the
 * field-aligned operator (whose sparsity is each cell's 3 x 3 x 3
 * neighbourhood: the cells sharing a corner with it); "the sparsity of M"
 * is its nonzero entries. */

#define OR_PC_JACOBI 0
#define OR_PC_BILU0 2

typedef struct {
    int n;
    int* rowp;      /* CSR, columns ascending, every row holds its diagonal */
    int* col;
    double* m0;     /* entries of the block-diagonal part of M */
    double* lu;     /* after factoring: strict lower part L (unit diagonal
                       implied), diagonal and upper part U */
    int* dpos;      /* position of the diagonal in each row */
} or_csr;

static void csr_free(or_csr* A)
{
    free(A->rowp); free(A->col); free(A->m0); free(A->lu); free(A->dpos);
    memset(A, 0, sizeof(*A));
}

static int same_box(const or_ctx* o, int i, int j, int k, int i2, int j2, int k2)
{
    return i / o->pbi == i2 / o->pbi && j / o->pbj == j2 / o->pbj && k / o->pbk == k2 / o->pbk;
}

/* the block-diagonal part of M = wV + dt L for the 7-point operator: the
 * off-diagonal entry of a face is -dt c_f A_f/d_f (the coupling of
 * apply_iso7), the diagonal wV + dt diag(L) */
static int bilu0_assemble(const or_ctx* o, double dt, or_csr* A)
{
    if (o->op != OR_ISO7) return 3;
    const int nr = o->nr, nt = o->nt, np = o->np;
    const int n = (int)ncell(o);
    A->n = n;
    A->rowp = (int*)malloc((size_t)(n + 1) * sizeof(int));
    A->col = (int*)malloc((size_t)7 * n * sizeof(int));
    A->m0 = (double*)malloc((size_t)7 * n * sizeof(double));
    A->lu = (double*)malloc((size_t)7 * n * sizeof(double));
    A->dpos = (int*)malloc((size_t)n * sizeof(int));
    double* Ld = (double*)malloc((size_t)n * sizeof(double));
    or_diag(o, Ld);
    int q = 0;
    for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nt; ++j)
            for (int k = 0; k < np; ++k) {
                const int m = (int)cell_ix(o, 0, i, j, k);
                const double cm = o->coef[m];
                A->rowp[m] = q;
                /* neighbours in ascending cell order: r-, theta-, phi-, self,
                 * phi+, theta+, r+ (phi without the periodic wrap) */
                const int di[7] = {-1, 0, 0, 0, 0, 0, 1};
                const int dj[7] = {0, -1, 0, 0, 0, 1, 0};
                const int dk[7] = {0, 0, -1, 0, 1, 0, 0};
                for (int t = 0; t < 7; ++t) {
                    const int i2 = i + di[t], j2 = j + dj[t], k2 = k + dk[t];
                    if (i2 < 0 || i2 >= nr || j2 < 0 || j2 >= nt || k2 < 0 || k2 >= np) continue;
                    if (!same_box(o, i, j, k, i2, j2, k2)) continue;
                    const int nb = (int)cell_ix(o, 0, i2, j2, k2);
                    double v;
                    if (t == 3) {
                        v = wvol(o, i, j, k) + dt * Ld[m];
                        A->dpos[m] = q;
                    } else {
                        const double cf = 0.5 * (cm + o->coef[nb]);
                        double tr;
                        if (di[t]) tr = trans_r(o, di[t] < 0 ? i : i + 1, j, k);
                        else if (dj[t]) tr = trans_t(o, i, dj[t] < 0 ? j : j + 1, k);
                        else tr = trans_p(o, i, j, dk[t] < 0 ? k : k + 1);
                        v = -dt * cf * tr;
                    }
                    A->col[q] = nb;
                    A->m0[q] = v;
                    A->lu[q] = v;
                    ++q;
                }
            }
    A->rowp[n] = q;
    free(Ld);
    return 0;
}

/* Colours of the longitude index for reading the field-aligned operator by
 * probes: any three cyclically consecutive k get distinct colours. */
static int kcolours(int np) { return np % 3 == 0 ? 3 : np % 4 == 0 ? 4 : np % 5 == 0 ? 5 : np; }

/* The block-diagonal part of M = wV + dt L for the field-aligned operator,
 * read from the operator itself: with the cells coloured by (i mod 3,
 * j mod 3, k mod kcolours(np)), a cell has at most one cell of each colour
 * in its neighbourhood (phi wrap included), so (L x)_m for x the indicator
 * of one colour (linear mode, L x = -wV F) is L_mn for the neighbour n of m
 * of that colour (the diagonal is taken from or_diag, as the Jacobi
 * preconditioner has it).  Entries are stored in ascending column order;
 * exact zeros off the diagonal are not part of the sparsity. */
static int bilu0_assemble_aligned(const or_ctx* oc, double dt, or_csr* A)
{
    or_ctx* o = (or_ctx*)oc;   /* the apply uses the context's corner buffer */
    const int nr = o->nr, nt = o->nt, np = o->np, nk = kcolours(np);
    const int n = (int)ncell(o);
    double* Lc = (double*)calloc((size_t)27 * n, sizeof(double));
    double* x = (double*)malloc((size_t)n * sizeof(double));
    double* F = (double*)malloc((size_t)n * sizeof(double));
    for (int ci = 0; ci < 3; ++ci)
        for (int cj = 0; cj < 3; ++cj)
            for (int ck = 0; ck < nk; ++ck) {
#pragma omp parallel for schedule(static)
                for (int i = 0; i < nr; ++i)
                    for (int j = 0; j < nt; ++j)
                        for (int k = 0; k < np; ++k)
                            x[cell_ix(o, 0, i, j, k)] =
                                (i % 3 == ci && j % 3 == cj && k % nk == ck) ? 1.0 : 0.0;
                apply_aligned(o, 0, x, F, 0);
#pragma omp parallel for schedule(static)
                for (int i = 0; i < nr; ++i)
                    for (int j = 0; j < nt; ++j)
                        for (int k = 0; k < np; ++k) {
                            const size_t m = cell_ix(o, 0, i, j, k);
                            const double Lm = -F[m] * wvol(o, i, j, k);
                            for (int t = 0; t < 27; ++t) {
                                const int i2 = i + t / 9 - 1, j2 = j + (t / 3) % 3 - 1;
                                const int k2 = (k + t % 3 - 1 + np) % np;
                                if (i2 < 0 || i2 >= nr || j2 < 0 || j2 >= nt) continue;
                                if (i2 % 3 == ci && j2 % 3 == cj && k2 % nk == ck)
                                    Lc[27 * m + t] = Lm;
                            }
                        }
            }
    free(x);
    free(F);
    double* Ld = (double*)malloc((size_t)n * sizeof(double));
    or_diag(o, Ld);   /* the diagonal as the Jacobi preconditioner has it */
    A->n = n;
    A->rowp = (int*)malloc((size_t)(n + 1) * sizeof(int));
    A->col = (int*)malloc((size_t)27 * n * sizeof(int));
    A->m0 = (double*)malloc((size_t)27 * n * sizeof(double));
    A->lu = (double*)malloc((size_t)27 * n * sizeof(double));
    A->dpos = (int*)malloc((size_t)n * sizeof(int));
    int q = 0;
    for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nt; ++j)
            for (int k = 0; k < np; ++k) {
                const int m = (int)cell_ix(o, 0, i, j, k);
                A->rowp[m] = q;
                /* offsets in (di, dj, dk) order are columns in ascending order */
                for (int t = 0; t < 27; ++t) {
                    const int i2 = i + t / 9 - 1, j2 = j + (t / 3) % 3 - 1, k2 = k + t % 3 - 1;
                    if (i2 < 0 || i2 >= nr || j2 < 0 || j2 >= nt || k2 < 0 || k2 >= np) continue;
                    if (!same_box(o, i, j, k, i2, j2, k2)) continue;
                    const double v = (t == 13) ? wvol(o, i, j, k) + dt * Ld[m]
                                               : dt * Lc[27 * (size_t)m + t];
                    if (t != 13 && v == 0.0) continue;
                    if (t == 13) A->dpos[m] = q;
                    A->col[q] = (int)cell_ix(o, 0, i2, j2, k2);
                    A->m0[q] = v;
                    A->lu[q] = v;
                    ++q;
                }
            }
    A->rowp[n] = q;
    free(Lc);
    free(Ld);
    return 0;
}

/* ILU(0) in place on A->lu, IKJ order: for each row i and each k < i in the
 * row, l_ik = a_ik / u_kk, then a_ij -= l_ik u_kj for the j > k of row k
 * that are in the pattern of row i.  7 (not factorable) on a pivot that is
 * not positive and finite. */
static int bilu0_factor(or_csr* A)
{
    const int n = A->n;
    int* pos = (int*)malloc((size_t)n * sizeof(int));
    for (int t = 0; t < n; ++t) pos[t] = -1;
    int status = 0;
    for (int i = 0; i < n && !status; ++i) {
        for (int p = A->rowp[i]; p < A->rowp[i + 1]; ++p) pos[A->col[p]] = p;
        for (int p = A->rowp[i]; p < A->dpos[i]; ++p) {
            const int k = A->col[p];
            A->lu[p] /= A->lu[A->dpos[k]];
            const double lik = A->lu[p];
            for (int qq = A->dpos[k] + 1; qq < A->rowp[k + 1]; ++qq) {
                const int jj = pos[A->col[qq]];
                if (jj >= 0) A->lu[jj] -= lik * A->lu[qq];
            }
        }
        const double piv = A->lu[A->dpos[i]];
        if (!(piv > 0.0) || !isfinite(piv)) status = 7;
        for (int p = A->rowp[i]; p < A->rowp[i + 1]; ++p) pos[A->col[p]] = -1;
    }
    free(pos);
    return status;
}

static int bilu0_make(const or_ctx* o, double dt, or_csr* A)
{
    int e = o->op == OR_ALIGNED ? bilu0_assemble_aligned(o, dt, A) : bilu0_assemble(o, dt, A);
    if (!e) e = bilu0_factor(A);
    return e;
}

/* z = U^{-1} L^{-1} r on one component */
static void bilu0_solve(const or_csr* A, const double* r, double* z)
{
    const int n = A->n;
    for (int i = 0; i < n; ++i) {
        double s = r[i];
        for (int p = A->rowp[i]; p < A->dpos[i]; ++p) s -= A->lu[p] * z[A->col[p]];
        z[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = z[i];
        for (int p = A->dpos[i] + 1; p < A->rowp[i + 1]; ++p) s -= A->lu[p] * z[A->col[p]];
        z[i] = s / A->lu[A->dpos[i]];
    }
}

/* z = P^{-1} r for every component: r / D (Jacobi) or the block ILU(0) solve */
static void precondition(const or_ctx* o, const or_csr* F, const double* D, const double* r,
                         double* z)
{
    const size_t N = ncell(o);
    for (int c = 0; c < o->nc; ++c) {
        if (o->pcond == OR_PC_BILU0) bilu0_solve(F, r + c * N, z + c * N);
        else
#pragma omp parallel for schedule(static)
            for (size_t m = 0; m < N; ++m) z[c * N + m] = r[c * N + m] / D[m];
    }
}

int or_set_pc(or_ctx* o, int pc, int bi, int bj, int bk)
{
    if (pc == OR_PC_JACOBI) { o->pcond = pc; return 0; }
    if (pc != OR_PC_BILU0 || o->op == OR_VISCV || bi < 1 || bj < 1 || bk < 1) return 1;
    o->pcond = pc;
    o->pbi = bi; o->pbj = bj; o->pbk = bk;
    return 0;
}

/* The block ILU(0) factors at dt in CSR form (for the tests): rowp [n+1],
 * col / m0 / lu [cap].  Returns the number of stored entries, or -(status)
 * (-1 no block ILU(0) set, -2 cap too small, -3 operator, -7 pivot). */
int or_bilu0_export(const or_ctx* o, double dt, int* rowp, int* col, double* m0, double* lu,
                    int cap)
{
    if (o->pcond != OR_PC_BILU0) return -1;
    or_csr A;
    memset(&A, 0, sizeof(A));
    int e = bilu0_make(o, dt, &A);
    if (e) { csr_free(&A); return -e; }
    const int nnz = A.rowp[A.n];
    if (nnz > cap) { csr_free(&A); return -2; }
    memcpy(rowp, A.rowp, (size_t)(A.n + 1) * sizeof(int));
    memcpy(col, A.col, (size_t)nnz * sizeof(int));
    memcpy(m0, A.m0, (size_t)nnz * sizeof(double));
    memcpy(lu, A.lu, (size_t)nnz * sizeof(double));
    csr_free(&A);
    return nnz;
}

/* z = P^{-1} r (all components) with the preconditioner set by or_set_pc */
int or_precondition(const or_ctx* o, double dt, const double* r, double* z)
{
    const size_t N = ncell(o);
    or_csr A;
    memset(&A, 0, sizeof(A));
    double* D = NULL;
    if (o->pcond == OR_PC_BILU0) {
        const int e = bilu0_make(o, dt, &A);
        if (e) { csr_free(&A); return e; }
    } else {
        D = (double*)malloc(N * sizeof(double));
        or_diag(o, D);
        for (int i = 0; i < o->nr; ++i)
            for (int j = 0; j < o->nt; ++j)
                for (int k = 0; k < o->np; ++k) {
                    const size_t m = cell_ix(o, 0, i, j, k);
                    D[m] = wvol(o, i, j, k) + dt * D[m];
                }
    }
    precondition(o, &A, D, r, z);
    free(D);
    csr_free(&A);
    return 0;
}

/* ------------------------------------------------------------ BE + PCG */

/* Inner product in a fixed order, independent of the thread count (the
 * paper fixes none): consecutive blocks of DOT_BLOCK terms are summed in
 * index order, then the block sums in block order. */
#define DOT_BLOCK 16384
static double dot(const double* a, const double* b, size_t n)
{
    const size_t nb = (n + DOT_BLOCK - 1) / DOT_BLOCK;
    double* part = (double*)malloc((nb ? nb : 1) * sizeof(double));
#pragma omp parallel for schedule(static)
    for (size_t q = 0; q < nb; ++q) {
        const size_t m1 = (q + 1) * DOT_BLOCK < n ? (q + 1) * DOT_BLOCK : n;
        double s = 0.0;
        for (size_t m = q * DOT_BLOCK; m < m1; ++m) s += a[m] * b[m];
        part[q] = s;
    }
    double s = 0.0;
    for (size_t q = 0; q < nb; ++q) s += part[q];
    free(part);
    return s;
}

/* y = M x = V x + dt L x, with L x = -V F_lin(x) */
static void be_matvec(or_ctx* o, const double* x, double* y, double dt, double* tmp)
{
    or_apply(o, x, tmp, 0);
    const size_t N = ncell(o);
    for (int c = 0; c < o->nc; ++c)
#pragma omp parallel for schedule(static)
        for (int i = 0; i < o->nr; ++i)
            for (int j = 0; j < o->nt; ++j)
                for (int k = 0; k < o->np; ++k) {
                    const size_t m = c * N + cell_ix(o, 0, i, j, k);
                    const double V = wvol(o, i, j, k);
                    y[m] = V * x[m] + dt * (-V * tmp[m]);
                }
}

/* Backward Euler step (I - dt V^{-1}(h - L.))u^{n+1} = u^n written as the
 * SPD system (V + dt L) x = V u^n + dt h, solved by preconditioned CG (point
 * Jacobi, or block ILU(0) when set by or_set_pc) from x0 = u^n, stopping
 * when ||r||_2 <= tol ||b||_2 (or after exactly force_iters iterations when
 * > 0).  Returns 0, 4 (no convergence), 5 (breakdown: <p,Mp> <= 0 or not
 * finite), 3 / 7 (block ILU(0): operator not supported / pivot not positive). */
static int be_solve(or_ctx* o, double* u, double dt, double tol, int max_iter, int force_iters,
                    int* iters, double* relres)
{
    const size_t N = ncell(o), n = (size_t)o->nc * N;
    int status = 0;
    double* b = (double*)malloc(n * sizeof(double));
    double* x = (double*)malloc(n * sizeof(double));
    double* r = (double*)malloc(n * sizeof(double));
    double* z = (double*)malloc(n * sizeof(double));
    double* p = (double*)malloc(n * sizeof(double));
    double* q = (double*)malloc(n * sizeof(double));
    double* tmp = (double*)malloc(n * sizeof(double));
    double* zero = (double*)calloc(n, sizeof(double));
    double* Ld = (double*)malloc(N * sizeof(double));
    double* D = (double*)malloc(N * sizeof(double));
    or_diag(o, Ld);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < o->nr; ++i)
        for (int j = 0; j < o->nt; ++j)
            for (int k = 0; k < o->np; ++k) {
                const size_t m = cell_ix(o, 0, i, j, k);
                D[m] = wvol(o, i, j, k) + dt * Ld[m];
            }
    /* b = V u^n + dt h, with h = V F(0) the boundary-data part of F */
    or_apply(o, zero, tmp, 1);
    for (int c = 0; c < o->nc; ++c)
#pragma omp parallel for schedule(static)
        for (int i = 0; i < o->nr; ++i)
            for (int j = 0; j < o->nt; ++j)
                for (int k = 0; k < o->np; ++k) {
                    const size_t m = c * N + cell_ix(o, 0, i, j, k);
                    const double V = wvol(o, i, j, k);
                    b[m] = V * u[m] + dt * V * tmp[m];
                }
    memcpy(x, u, n * sizeof(double));
    be_matvec(o, x, q, dt, tmp);
#pragma omp parallel for schedule(static)
    for (size_t m = 0; m < n; ++m) r[m] = b[m] - q[m];
    or_csr F;
    memset(&F, 0, sizeof(F));
    if (o->pcond == OR_PC_BILU0) {
        const int e = bilu0_make(o, dt, &F);
        if (e) { status = e; free(b); free(x); free(r); free(z); free(p); free(q); free(tmp);
                 free(zero); free(Ld); free(D); csr_free(&F); *iters = 0; *relres = 0.0; return e; }
    }
    precondition(o, &F, D, r, z);
    memcpy(p, z, n * sizeof(double));
    double rho = dot(r, z, n);
    const double bnorm = sqrt(dot(b, b, n));
    double rnorm = sqrt(dot(r, r, n));
    int it = 0;
    const int limit = force_iters > 0 ? force_iters : max_iter;
    if (!(force_iters > 0) && rnorm <= tol * bnorm) goto done;
    for (it = 1; it <= limit; ++it) {
        be_matvec(o, p, q, dt, tmp);
        const double pq = dot(p, q, n);
        if (!(pq > 0.0) || !isfinite(pq)) { status = 5; break; }
        const double alpha = rho / pq;
#pragma omp parallel for schedule(static)
        for (size_t m = 0; m < n; ++m) x[m] += alpha * p[m];
#pragma omp parallel for schedule(static)
        for (size_t m = 0; m < n; ++m) r[m] -= alpha * q[m];
        rnorm = sqrt(dot(r, r, n));
        if (force_iters > 0) { if (it == force_iters) break; }
        else if (rnorm <= tol * bnorm) break;
        precondition(o, &F, D, r, z);
        const double rho1 = dot(r, z, n);
        const double beta = rho1 / rho;
#pragma omp parallel for schedule(static)
        for (size_t m = 0; m < n; ++m) p[m] = z[m] + beta * p[m];
        rho = rho1;
    }
    if (it > limit) { it = limit; status = 4; }
done:
    memcpy(u, x, n * sizeof(double));
    *iters = it;
    *relres = bnorm > 0.0 ? rnorm / bnorm : rnorm;
    free(b); free(x); free(r); free(z); free(p); free(q); free(tmp); free(zero); free(Ld); free(D);
    csr_free(&F);
    return status;
}

/* ------------------------------------------------------- cycle control */

/* Advance u over dt.  scheme 0: STS (sts_kind 0 RKL2 / 1 RKG2); scheme 1:
 * BE + PCG.  cycles > 0: that many equal cycles, no PTL.  cycles == 0:
 * dynamic PTL cycling -- at each cycle the PTL of the current u gives
 * n = ceil(t_rem / dt_PTL) and the cycle length t_rem / n (Sec. 2).
 * replay_n > 0: use the given cycle lengths instead (parity replays).
 * ptl_floor: the limit used is max(dt_PTL, ptl_floor * dt_E).  The paper sets
 * no lower bound; without one the limit can collapse towards zero once a
 * cycle has flattened the limiting pair (the difference in Eq. ptl2 is then
 * ~0 while dF is not), and a Backward Euler cycle that is then too short to
 * move the iterate leaves it there for good.  0 disables the floor.
 * Returns 0 or an error code (4 no convergence, 5 breakdown, 6 non-finite
 * PTL, 8 more than max_cycles cycles). */
int or_advance(or_ctx* o, double* u, double dt, int cycles, int scheme, int sts_kind,
               int force_odd, int s_override, double tol, int max_iter, int force_iters,
               int max_cycles, double ptl_floor, const double* replay_dt, int replay_n,
               or_stats* st)
{
    memset(st, 0, sizeof(*st));
    st->dt_ptl_first = st->dt_ptl_min = INFINITY;
    const double dtE = or_dt_explicit(o);
    st->dt_explicit = dtE;
    double t_rem = dt;
    int ncyc = 0, status = 0;
    while (1) {
        double dtc;
        int last = 0;
        if (replay_n > 0) {
            dtc = replay_dt[ncyc];
            last = (ncyc + 1 == replay_n);
        } else if (cycles > 0) {
            dtc = dt / cycles;
            last = (ncyc + 1 == cycles);
        } else {
            int64_t km;
            const double ptl = or_ptl(o, u, &km);
            if (isnan(ptl) || ptl <= 0.0) { status = 6; break; }
            if (ncyc == 0) { st->dt_ptl_first = ptl; st->k_first = km; }
            if (ptl < st->dt_ptl_min) st->dt_ptl_min = ptl;
            double lim = ptl;
            if (lim < ptl_floor * dtE) { lim = ptl_floor * dtE; st->floored += 1; }
            const double nreq = ceil(t_rem / lim);
            if (!(nreq > 1.0)) { dtc = t_rem; last = 1; }
            else dtc = t_rem / nreq;
        }
        if (ncyc >= max_cycles) { status = 8; break; }
        if (ncyc < OR_MAX_LOG) st->dt_cycle[ncyc] = dtc;
        if (scheme == 0) {
            const int s = s_override > 0 ? s_override : or_sts_stages(sts_kind, dtc / dtE, force_odd);
            if (ncyc < OR_MAX_LOG) st->s_cycle[ncyc] = s;
            st->s_total += s;
            if (s > st->s_max) st->s_max = s;
            sts_cycle(o, u, dtc, sts_kind, s);
        } else {
            int its;
            double rr;
            status = be_solve(o, u, dtc, tol, max_iter, force_iters, &its, &rr);
            if (ncyc < OR_MAX_LOG) st->s_cycle[ncyc] = its;
            st->iters_total += its;
            if (its > st->iters_max) st->iters_max = its;
            st->rel_residual = rr;
        }
        ++ncyc;
        if (status) break;
        if (last) break;
        t_rem -= dtc;
    }
    st->cycles = ncyc;
    return status;
}

/* number of OpenMP threads the oracle's parallel loops use */
#ifdef _OPENMP
#include <omp.h>
#endif
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads for the following parallel loops (n < 1: one per processor) */
void or_set_num_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
    (void)n;
#endif
}

/* Host memory bandwidth for the CPU timings (not part of the method): the
 * STREAM triad a = b + 3 c over n doubles per array, first touch in
 * parallel, best of reps; 24 bytes per element.  Returns GB/s, or -1 when
 * the arrays cannot be allocated. */
double or_stream_triad(long n, int reps)
{
    double* a = (double*)malloc(sizeof(double) * (size_t)n);
    double* b = (double*)malloc(sizeof(double) * (size_t)n);
    double* c = (double*)malloc(sizeof(double) * (size_t)n);
    double best = -1.0;
    if (a && b && c) {
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) {
            a[i] = 0.0;
            b[i] = 1.0;
            c[i] = 2.0;
        }
        for (int r = 0; r < reps; ++r) {
#ifdef _OPENMP
            const double t0 = omp_get_wtime();
#endif
#pragma omp parallel for schedule(static)
            for (long i = 0; i < n; ++i) a[i] = b[i] + 3.0 * c[i];
#ifdef _OPENMP
            const double t = omp_get_wtime() - t0;
            const double gbs = 24.0 * (double)n / t / 1e9;
            if (t > 0.0 && gbs > best) best = gbs;
#endif
        }
    }
    free(a);
    free(b);
    free(c);
    return best;
}
