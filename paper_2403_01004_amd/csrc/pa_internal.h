// pa_internal.h -- declarations shared by the GPU library's kernel and host
// translation units (gfx950).  Not part of the public ABI (include/paradv.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pa {

constexpr int kBlock = 256;   // threads per workgroup (4 waves of 64)
constexpr int kOpIso7 = 0, kOpAligned = 1, kOpViscVec = 2;  // pa_op
constexpr int kRedBlock = 1024;

// Separable 1-D metric factors of the finite-volume mesh (device arrays).
//  V(i,j,k)           = vr[i] * vt[j] * vp[k]
//  G_r(face ir, j, k) = gr[ir] * vt[j] * vp[k]        ir in [0, nr]
//  G_t(i, face jt, k) = gtr[i] * gtt[jt] * vp[k]      jt in [0, nt], 0 at the poles
//  G_p(i, j, face kf) = gtr[i] * gpt[j] * gpp[kf]     kf in [0, np), face between kf-1, kf
// Change of basis between neighbouring cell centres (vector viscosity):
//  rtf[jt], rtf[nt+1+jt] = cos, sin of tc[jt] - tc[jt-1]  (theta face jt; 1, 0 at the poles)
//  rtc[j],  rtc[nt+j]    = sin, cos of the colatitude tc[j]
//  rpf[kf], rpf[np+kf]   = 1 - cos, sin of pc[kf] - pc[kf-1]  (phi face kf, periodic)
template <class T>
struct Geo {
    int nr, nt, np, P;  // P = nt*np cells per radial level
    const T* vr;
    const T* vt;
    const T* vp;
    const T* gr;
    const T* gtr;
    const T* gtt;
    const T* gpt;
    const T* gpp;
    const T* rtf;
    const T* rtc;
    const T* rpf;
};

enum Mode : int {
    kApply = 0,   // out = F(u)
    kFirst = 1,   // out = F(u); per-block argmax |F|; non-finite flag
    kStage = 2,   // out = mu u + nu ukm2 + c0 u0 + mudt F(u) + gdt y0
    kMatvec = 3,  // out = V u + dt L u (linear part); per-block <u, out>
};

// Source of the u_{k-2} term of an STS stage.
enum Km2 : int { kKm2Array = 0, kKm2U0 = 1, kKm2Virtual = 2 };

template <class T>
struct KArgs {
    const T* u;       // stencil input (or u0 when the input is virtual)
    const T* y0;      // F(u0)
    double a1;        // virtual input u1 = u0 + a1*y0 (a1 = mu~_1 dt)
    const T* coef;    // 7-point: cell coefficient array, or null for constant `cs`
    T cs;
    const T* e;       // field-aligned: corner coefficients [3][nr+1][nt+1][np]
    const T* ub_in;   // [nc][nt][np]
    const T* ub_out;
    int bc_in, bc_out, affine;
    int r_lo, r_hi;   // radial levels processed [r_lo, r_hi)
    int rch;          // radial levels per workgroup
    int nbx, nrc, nc; // logical tiles: x-blocks, radial chunks, components
    T* out;
    const T* ukm2;
    int km2;
    const T* u0;
    double mu, nu, c0, mudt, gdt, dt;
    double* part;     // per-tile partial sums / maxima
    long long* part_idx;
    int* flag;        // non-finite flag (kFirst)
    const int* done;  // skip the launch when *done != 0 (PCG), may be null
    const T* wgt;     // cell weight w of F = (1/w) div(...), [nr][nt][np], null for 1
    int only_c;       // vector viscosity: store only component only_c (-1: all)
};

// stencil launchers (pa_kernels.hip)
template <class T>
void launch_iso7(int mode, bool virt, const Geo<T>& g, const KArgs<T>& a, hipStream_t s);
template <class T>
void launch_aligned(int mode, bool virt, const Geo<T>& g, const KArgs<T>& a, hipStream_t s);
template <class T>
void launch_viscv(int mode, bool virt, const Geo<T>& g, const KArgs<T>& a, hipStream_t s);

// workgroups covering one radial level (op: 0 7-point, 1 field-aligned),
// and logical workgroups of a stencil launch over nlev levels (== entries
// of a.part); the 7-point form depends on the precision (fp32)
int blocks_per_plane(int op, int nt, int np, bool fp32 = false);
int stencil_tiles(int op, int nt, int np, int nlev, int rch, int nc, bool fp32 = false);

// setup kernels
void launch_coef(const double* T0, double scale, double expo, const double* fc, double Tc, int P,
                 int n, double* c64, float* c32, int* flag, hipStream_t s);
struct CornerGeo {
    const double* hr;   // [nr+1] radial centre distance at corner plane ic
    const double* wr;   // [nr+1] radial dual extent
    const double* R;    // [nr+1] face radii
    const double* htt;  // [nt+1] tc[jc]-tc[jc-1] (0 at poles)
    const double* sT;   // [nt+1] sin(t_faces[jc])
    const double* dpc;  // [np] phi centre distance between kc-1 and kc
};
void launch_corner_e(int nr, int nt, int np, const CornerGeo& cg, const double* coef,
                     const double* B, double* e64, float* e32, int* flag, hipStream_t s);
void launch_diag_iso7(const Geo<double>& g, const double* coef, double cs, const double* w,
                      int bc_in, int bc_out, double* diag, double* part, hipStream_t s, int* nparts);
void launch_diag_aligned(const Geo<double>& g, const double* e, const double* w, int bc_in,
                         int bc_out, double* diag, double* part, hipStream_t s, int* nparts);

// reductions and vector kernels (pa_vec.hip)
struct DevState {
    double dt_ptl;
    long long kmax;
    double gmax;       // Gershgorin maximum
    double rho, pq, rz, rr, bb, alpha, beta, rr0, eta;
    int done, iters, status, nonfinite;
    int xpend;         // this iteration's x += alpha p is left to the direction kernel
    int max_iter, force_iters, mode;
    double tol;
    double dt_full;    // full-grid limit (diagnostic)
    long long kfull;
};
void launch_reduce_max(const double* part, int n, double* outp, hipStream_t s);
// minimum of Eq. (ptl2) over every cell and face neighbour -> st->dt_full,
// st->kfull (lowest cell index attaining it, -1 if none); pval / pidx hold
// up to 4096 partials
template <class T>
void launch_ptl_full(const T* u, const T* F, int nc, int nr, int nt, int np, double* pval,
                     long long* pidx, DevState* st, hipStream_t s);
// argmax of |F| over per-tile partials into st->kmax (-1 when every |F| is
// NaN); N = cells of all components
void launch_argmax(const double* pval, const long long* pidx, int n, long long N, DevState* st,
                   hipStream_t s);
template <class T>
void launch_ptl_finalize(const double* pval, const long long* pidx, int n, const T* u, const T* F,
                         int nc, int nr, int nt, int np, DevState* st, hipStream_t s);
// Point-Jacobi diagonal in row form, D = V + dt diag(L) = vp_k A_ij + B_ij G_k,
// for the 7-point operator with a constant coefficient and no weight: the
// metric is separable, so D is two values per (r, theta) row and two per phi
// index instead of one value per cell.  ab interleaves A, B per row
// (nr * nt pairs), G_k = gpp_k + gpp_{k+1}; ab null: D is read from the
// per-cell array.
struct JacD {
    const double* ab = nullptr;
    const double* G = nullptr;
    const double* vp = nullptr;
    unsigned np = 0;
};
// ab and G at step dt (pa_setup.hip)
void launch_jacobi_rows(const Geo<double>& g, double cs, int bc_in, int bc_out, double dt,
                        double* ab, double* G, hipStream_t s);
// with jd.ab set, D is formed from the rows (and still written to D)
template <class PT>
void launch_pcg_init(const Geo<double>& g, int nc, double dt, const double* w, const double* u,
                     const double* y0, const double* hF, const double* diagL, double* D, double* r,
                     PT* p, double* b, double* part, int* nparts, hipStream_t s,
                     const JacD& jd = JacD{});
template <class PT>
void launch_pcg_resid(size_t N, int nc, const double* b, const double* q, const double* D,
                      double* r, PT* p, double* part, int* nparts, hipStream_t s);
void launch_pcg_start(const double* part, int n, DevState* st, double tol, int max_iter,
                      int force_iters, int mode, double eta, hipStream_t s);
// alpha = rho / <p, q>; with aslot, *aslot = 0 first (the iteration's entry
// in the deferred x update; launch_pcg_beta fills it when the r update ran)
void launch_pcg_alpha(const double* part, int n, DevState* st, hipStream_t s,
                      double* aslot = nullptr);
// r -= alpha q, partials <r, r/D>, <r, r>; also x += alpha p when x is not
// null (otherwise launch_pcg_dir applies it, reading p once for both)
template <class PT>
void launch_pcg_update(size_t N, int nc, const double* D, double* x, double* r, const PT* p,
                       const PT* q, const DevState* st, double* part, int* nparts, hipStream_t s,
                       const JacD& jd = JacD{});
void launch_pcg_beta(const double* part, int n, DevState* st, hipStream_t s,
                     double* aslot = nullptr);
// x += alpha p (the update left by launch_pcg_update with x null), then
// p = r/D + beta p unless the solve has stopped
template <class PT>
void launch_pcg_dir(size_t N, int nc, const double* D, const double* r, double* x, PT* p,
                    const DevState* st, hipStream_t s);
// Deferred x update (point-Jacobi solves): the directions of kXGroup
// consecutive iterations live in kXGroup buffers; pn = r/D + beta p while the
// solve goes on, and x += alpha_t p_t for the group's iterations in order
// (the arithmetic of launch_pcg_dir, applied per group: x is read and
// written once per group instead of once per iteration)
constexpr int kXGroup = 8;   // PA_PCG_XGROUP
template <class PT>
struct XSlots {
    const PT* p[kXGroup];
};
template <class PT>
void launch_pcg_dir_next(size_t N, int nc, const double* D, const double* r, const PT* p, PT* pn,
                         const DevState* st, hipStream_t s, const JacD& jd = JacD{});
template <class PT>
void launch_pcg_xflush(size_t n, double* x, const XSlots<PT>& sl, const double* ahist, int count,
                       hipStream_t s);
// face couplings L_{m,nb} for nb = r-, r+, t-, t+, p-, p+ into out[6][N]
// (zero where the neighbour does not exist) (pa_setup.hip)
void launch_couplings(const Geo<double>& g, int op, const double* coef, double cs, const double* e,
                      int bc_in, int bc_out, double* out, hipStream_t s);

// learned preconditioner network (pa_nn.hip).  Flat FP32 parameter vector:
// W1[16][8][27], b1[16], W2[16][16][27], b2[16], W3[1][16][27]
constexpr int NN_OFF_W1 = 0, NN_OFF_B1 = 3456, NN_OFF_W2 = 3472, NN_OFF_B2 = 10384,
              NN_OFF_W3 = 10400, NN_NPARAM = 10832;
struct NNWeights {
    __bf16 *f1, *f2, *f3, *d3, *d2;  // BF16 MFMA operand tables
};
void launch_nn_prep_weights(const float* theta, NNWeights& w, hipStream_t s);
// Network launches run on nb elements of nr x nt x np cells stacked along r
// (zero padding in r and theta per element; phi periodic when per != 0).
// dir 0: forward of `layer` (1: 8->16, 2: 16->16, 3: 16->1 FP32 out);
// dir 1: input gradient of `layer` (3 or 2), masked by mask[p][16] > 0.
// Skipped when *done != 0 (done may be null).
void launch_nn_conv(int layer, int dir, int nb, int nr, int nt, int np, int per, const int* done,
                    const __bf16* x, const NNWeights& w, const float* theta, const __bf16* mask,
                    void* out, hipStream_t s);
// grad[layer's weights and bias] += sum_p G[p][co] X[p + tap][ci];
// part holds nn_wgrad_partials(nb, nr, nt, np) * 16 * 433 floats
int nn_wgrad_partials(int nb, int nr, int nt, int np);
void launch_nn_wgrad(int layer, int nb, int nr, int nt, int np, int per, const __bf16* X,
                     const __bf16* G, float* part, float* grad, hipStream_t s);
void launch_nn_static(const Geo<double>& g, double dt, const double* w, const double* D,
                      const double* cpl, __bf16* x, hipStream_t s);
void launch_nn_c0(size_t N, const double* r, const double* D, const double* sigma, const int* done,
                  __bf16* x, hipStream_t s);
// energy-norm training loss |P(r) - e|_M^2 / |e|_M^2 pieces
void launch_pair_build(size_t N, const __bf16* xs, const double* r, const double* D,
                       const double* sig, __bf16* x, double* zj, hipStream_t s);
void launch_nn_resid(size_t N, const double* zj, const float* out, const double* sig,
                     const double* e, double* d, hipStream_t s);
void launch_energy_gout(size_t N, const double* Md, const double* sig, const double* den,
                        double scale, __bf16* gout, hipStream_t s);
void launch_scal_reduce(const double* part, int n, const double* den, double scale, double* out,
                        hipStream_t s);
void launch_sub(size_t N, const double* a, const double* b, double* out, hipStream_t s);
void launch_jacobi_D(const Geo<double>& g, double dt, const double* w, const double* dL, double* D,
                     hipStream_t s);
void launch_nn_unpack(size_t N, const __bf16* x, float* f, hipStream_t s);
void launch_nn_apply(size_t N, const double* r, const double* D, const float* out,
                     const double* sigma, double* z, hipStream_t s);
void launch_nn_adam(float* th, const float* grad, float* m, float* v, float lr, int t, hipStream_t s);
int launch_fcg_combine(size_t N, int nc, const double* r, const double* q, const double* D,
                       const float* out, const double* sigma, const int* done, double* z,
                       double* part, hipStream_t s);
void launch_nn_sigma(size_t N, const double* r, const double* D, const int* done, double* part,
                     double* sigma, hipStream_t s);
void launch_sum_finish(const double* part, int n, double* out, hipStream_t s);
void launch_fcg_first(const double* part, int n, DevState* st, int* use_jacobi, hipStream_t s);
void launch_fcg_alpha(const double* part, int n, DevState* st, hipStream_t s);
void launch_fcg_check(const double* part, int n, DevState* st, hipStream_t s);
void launch_fcg_beta(const double* part, int n, DevState* st, int* use_jacobi, hipStream_t s);
int launch_fcg_dir(size_t N, int nc, const double* z, const double* r, const double* D,
                   const int* use_jacobi, const DevState* st, double* p, double* part,
                   hipStream_t s);
void launch_fcg_pr(const double* part, int n, DevState* st, hipStream_t s);

void launch_f64_to_f32(const double* a, float* b, size_t n, hipStream_t s);
void launch_f32_to_f64(const float* a, double* b, size_t n, hipStream_t s);
void launch_copy(const void* a, void* b, size_t bytes, hipStream_t s);
void launch_fill_zero(void* a, size_t bytes, hipStream_t s);
void launch_nonfinite(const double* a, size_t n, int* flag, hipStream_t s);
void launch_nonpositive(const double* a, size_t n, int* flag, hipStream_t s);
// block ILU(0) (7-point operator): boxes of 8 x 4 x 16 cells, one wave each
int bilu0_boxes(int nr, int nt, int np);
void launch_bilu0_factor(const Geo<double>& g, const double* coef, double cs, double dt,
                         const double* D, double* ip, int* flag, hipStream_t s);
template <class PT>
void launch_bilu0_solve(const Geo<double>& g, int nc, const double* coef, double cs, double dt,
                        const double* ip, const double* r, PT* out, double* part, int* nparts,
                        hipStream_t s);
template <class PT>
void launch_pcg_update_bilu0(const Geo<double>& g, int nc, const double* coef, double cs,
                             double dt, const double* ip, double* x, double* r, const PT* p,
                             const PT* q, double* z, const DevState* st, double* part,
                             int* nparts, hipStream_t s);
// p = z + beta p unless the solve has stopped; before it x += alpha p when
// x is not null (the update kernel then left x alone)
template <class PT>
void launch_pcg_dir_z(size_t n, const double* z, double* x, PT* p, const DevState* st,
                      hipStream_t s);
void launch_pcg_set_rho(const double* part, int n, DevState* st, hipStream_t s);  // !(a > 0) or NaN

}  // namespace pa
