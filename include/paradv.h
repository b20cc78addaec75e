/*
 * paradv.h -- C ABI of the MI355X (gfx950) parabolic-operator advance library.
 *
 * The library advances one operator-split parabolic term du/dt = F(u)
 * (Caplan et al., arXiv 2403.01004, Sec. 2, Eq. par) on a spherical
 * (r, theta, phi) shell over a time step dt, with
 *   - F the artificial-viscosity operator div(c grad u) per component or the
 *     field-aligned Spitzer conduction operator div(kappa bhat bhat . grad T)
 *     with lagged diffusivity kappa = kappa0 T0^{5/2} (Eqs. visc, tc);
 *   - RKL2 or RKG2 super time stepping (Sec. 3.1, App. A), or Backward Euler
 *     solved by point-Jacobi preconditioned CG (Sec. 3.1, PC1);
 *   - cycling at the practical time step limit of Eqs. (ptl)-(ptl3),
 *     re-evaluated after every cycle (Sec. 2).
 *
 * Discretisation (the paper gives only the continuous operators): finite
 * volume on a mesh given by its cell faces; the isotropic operator is a
 * 7-point stencil with face coefficients the mean of the two cell values;
 * the field-aligned operator is a symmetric corner scheme L = G^T W K G
 * (corner gradients averaged over four cell-centre differences, K = kappa
 * bhat bhat^T at cell corners, W the corner dual volume).  Radial
 * boundaries are Dirichlet (ghost 2 u_b - u) or no-flux; colatitude
 * boundaries (the poles) carry no flux; phi is periodic.
 *
 * Memory layout: a field is [ncomp][nr][nt][np] contiguous, np (phi)
 * fastest; boundary data [ncomp][nt][np]; corner arrays [3][nr+1][nt+1][np]
 * with components (r, theta, phi) at (r_faces[ic], t_faces[jc], p_faces[kc]).
 *
 * Ownership: every pointer argument is borrowed for the duration of the call
 * (the bound field: until it is re-bound or the context destroyed).  Device
 * pointers are HIP device memory on the context's device.  The context owns
 * only its scratch memory.
 *
 * Streams: all device work is queued on the stream given to pa_init; calls
 * that return host values synchronise that stream.  One context per host
 * thread at a time.
 *
 * Errors: every call returns a pa_status; pa_last_error gives a message.
 * Argument and state errors (PA_ERR_ARG, PA_ERR_STATE) leave the bound field
 * untouched; numerical errors (PA_ERR_NOCONV, PA_ERR_BREAKDOWN,
 * PA_ERR_NONFINITE, PA_ERR_MAXCYCLES) leave the last iterate in the field.
 */
#ifndef PARADV_H
#define PARADV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pa_ctx pa_ctx;

typedef enum {
    PA_OK = 0,
    PA_ERR_ARG = 1,        /* invalid argument (null, size, range) */
    PA_ERR_ALLOC = 2,      /* device allocation failed */
    PA_ERR_HIP = 3,        /* a HIP runtime call failed */
    PA_ERR_NOCONV = 4,     /* PCG reached max_iter without meeting tol */
    PA_ERR_BREAKDOWN = 5,  /* PCG: <p, M p> <= 0 or not finite */
    PA_ERR_NONFINITE = 6,  /* NaN/Inf in the field, coefficients or time-step limit */
    PA_ERR_STATE = 7,      /* call out of order (e.g. no field or coefficients) */
    PA_ERR_MAXCYCLES = 8   /* the time-step limit needs more than max_cycles cycles */
} pa_status;

/* PA_OP_ISO7: div(c grad u) of each component as a scalar (7-point);
 * PA_OP_FIELD_ALIGNED: div(c bhat bhat . grad u) (corner scheme);
 * PA_OP_VISC_VECTOR: Eq. (visc) for a velocity given by its spherical
 * components (ncomp = 3: v_r, v_theta, v_phi) -- the 7-point operator on
 * the Cartesian components, written in each cell's spherical basis, so a
 * colatitude or longitude face couples the cell to the neighbour's vector
 * rotated into that basis (the curvature coupling of the components).  It
 * has the 7-point operator's diagonal and spectrum (an orthogonal change of
 * basis), hence its explicit limit. */
typedef enum { PA_OP_ISO7 = 0, PA_OP_FIELD_ALIGNED = 1, PA_OP_VISC_VECTOR = 2 } pa_op;
typedef enum { PA_BC_DIRICHLET = 0, PA_BC_NOFLUX = 1 } pa_bc;
typedef enum { PA_FP64 = 0, PA_FP32_STAGES = 1 } pa_prec;
typedef enum { PA_STS_RKL2 = 0, PA_STS_RKG2 = 1 } pa_sts;
typedef enum { PA_PC_JACOBI = 0, PA_PC_LEARNED = 1, PA_PC_BILU0 = 2 } pa_pc;

/* Boxes of the block ILU(0) preconditioner (PA_PC_BILU0), in cells along
 * r, theta, phi, starting at cell 0 in each direction. */
#define PA_BILU0_BI 8
#define PA_BILU0_BJ 4
#define PA_BILU0_BK 16

/* Backward Euler solves with point Jacobi (FP64, or FP32 matvecs and
 * directions) apply the x update of
 * PA_PCG_XGROUP consecutive PCG iterations together: the group's search
 * directions stay in their own buffers (PA_PCG_XGROUP - 1 fields of device
 * memory besides the solve's own, in the direction type, allocated on first use; without them the
 * solve updates x every iteration), and x is read and written once per
 * group.  The result is that of one x update per iteration, bit for bit;
 * the timing class PA_K_DIR counts both kernels (direction, group update). */
#define PA_PCG_XGROUP 8

#define PA_MAX_LOG 4096

/* Grid and operator description (pa_init).  The face arrays are host
 * memory, copied during pa_init: r_faces[nr+1] and t_faces[nt+1] strictly
 * increasing with 0 <= t_faces < = pi, p_faces[np+1] strictly increasing
 * (one period = p_faces[np] - p_faces[0]).  nr >= 1, nt >= 2, np >= 3,
 * ncomp >= 1 (ncomp = 3 for PA_OP_VISC_VECTOR).  prec selects FP64 throughout or FP32 storage and stencil
 * arithmetic for the STS stages (FP64 recurrence coefficients, FP64
 * combination and FP64 reductions). */
typedef struct {
    int32_t nr, nt, np, ncomp;
    const double* r_faces;
    const double* t_faces;
    const double* p_faces;
    int32_t op;      /* pa_op */
    int32_t bc_in;   /* pa_bc at r_faces[0] */
    int32_t bc_out;  /* pa_bc at r_faces[nr] */
    int32_t prec;    /* pa_prec */
    /* optional device allocator (e.g. a framework's caching allocator);
     * both NULL: hipMalloc / hipFree */
    void* (*alloc)(size_t bytes, void* user);
    void (*free)(void* ptr, void* user);
    void* alloc_user;
} pa_desc;

/* Solver options (pa_set_options; pa_default_options fills defaults). */
typedef struct {
    int32_t force_odd;    /* 1: add a stage when s is even (Sec. 3.1, App. A). default 1 */
    int32_t s_override;   /* >0: use exactly this many stages. default 0 */
    int32_t pc;           /* pa_pc. default PA_PC_JACOBI; PA_PC_LEARNED needs weights
                             (pa_lpc_set_weights), ncomp == 1 and PA_FP64;
                             PA_PC_BILU0 needs PA_OP_ISO7 */
    int32_t max_iter;     /* PCG iteration limit per solve. default 10000 */
    int32_t max_cycles;   /* cycle limit per advance. default 100000 */
    int32_t force_iters;  /* >0: run exactly this many PCG iterations per solve. default 0 */
    int32_t pcg_batch;    /* most PCG iterations queued between host checks (the first
                             batch of a solve follows the previous solve's count, later
                             ones the iterations the residual decrease so far predicts;
                             a quarter of this under force_iters); results do not
                             depend on it. default 16 */
    int32_t replay_n;     /* >0: cycle lengths taken from replay_dt (parity replays) */
    const double* replay_dt; /* host, replay_n entries; copied by pa_set_options */
    double ptl_floor;     /* limit used = max(dt_PTL, ptl_floor * dt_E). default 1.0 */
    int32_t timing;       /* 1: time every kernel launch by class (pa_stats.kernel_*). default 0 */
} pa_opts;

/* kernel classes of pa_stats.kernel_ms / kernel_calls */
enum {
    PA_K_FIRST = 0,   /* y0 = F(u) + argmax |F| (PTL pass) */
    PA_K_STAGE = 1,   /* fused STS stage */
    PA_K_MATVEC = 2,  /* PCG matvec q = M p + <p,q> */
    PA_K_UPDATE = 3,  /* PCG r update + <r,z>, <r,r> (point Jacobi; block ILU(0): x and r
                         update fused with the block solve) */
    PA_K_DIR = 4,     /* PCG direction p = z + beta p (point Jacobi: with x += alpha p) */
    PA_K_INIT = 5,    /* PCG start (residual, boundary data) */
    PA_K_REDUCE = 6,  /* one-workgroup reductions and scalar updates */
    PA_K_OTHER = 7,   /* conversions and copies */
    PA_K_NN = 8,      /* learned preconditioner: features, network, FCG vector steps */
    PA_NKCLASS = 9
};

/* Per-advance statistics. */
typedef struct {
    int32_t cycles, s_total, s_max, iters_total, iters_max;
    int32_t fallbacks;        /* learned PC: Jacobi steps taken plus hand-overs to Jacobi PCG */
    int32_t floored, status;
    int64_t k_first;          /* linear index of max |F| at the first limit evaluation */
    double dt_explicit;       /* explicit Euler limit used */
    double dt_ptl_first, dt_ptl_min;
    double rel_residual;      /* PCG: ||r||/||b|| of the last solve */
    double ms_total;          /* wall time of the call on the stream, ms */
    double kernel_ms[PA_NKCLASS];     /* with opts.timing: summed launch durations per class */
    int32_t kernel_calls[PA_NKCLASS]; /* with opts.timing: launches per class */
    double dt_cycle[PA_MAX_LOG];   /* length of each cycle */
    int32_t per_cycle[PA_MAX_LOG]; /* stages (STS) or PCG iterations (BE) per cycle */
    int32_t jacobi_rows;  /* BE with point-Jacobi PCG: 1 when the diagonal
                             D = V + dt diag(L) was formed from per-(r, theta) row
                             terms (7-point operator, constant coefficient, no
                             weight), so no per-cell D is read in the iterations */
} pa_stats;

/* Create a context on the current HIP device; all work goes to hip_stream
 * (NULL: the null stream).  Copies the mesh, allocates scratch. */
pa_status pa_init(const pa_desc* desc, void* hip_stream, pa_ctx** out);

/* Release everything the context owns.  NULL is ignored. */
void pa_destroy(pa_ctx* ctx);

/* Last error message of this context ("" if none); valid until the next call. */
const char* pa_last_error(const pa_ctx* ctx);

void pa_default_options(pa_opts* opts);
pa_status pa_set_options(pa_ctx* ctx, const pa_opts* opts);

/* Bind the field advanced in place: device double[ncomp][nr][nt][np]. */
pa_status pa_bind_field(pa_ctx* ctx, double* u_dev);

/* Lagged coefficients (Eq. tc: kappa from the previous temperature T0).
 * T0_dev: device double[nr][nt][np] or NULL for the constant coefficient
 * `scale` (viscosity nu); otherwise c = scale * T0^expo (Spitzer: 2.5).
 * B_dev: field-aligned operator only, device double[3][nr+1][nt+1][np],
 * normalised here to bhat = B/|B| (zero where |B| = 0).  Also computes the
 * Jacobi diagonal and the explicit Euler limit.  PA_ERR_NONFINITE if a
 * coefficient is NaN/Inf or negative. */
pa_status pa_set_coefficients(pa_ctx* ctx, const double* T0_dev, double scale, double expo,
                              const double* B_dev);

/* Full forms of Eqs. (visc) and (tc): F = (1/w) div(c grad u) and
 * (1/w) div(c bhat bhat . grad T), with
 *   w_dev: device double[nr][nt][np], the weight of the time derivative
 *          (Eq. visc: rho; Eq. tc: 2 k rho / ((gamma - 1) m_p)), > 0;
 *          NULL for w = 1.  Copied.
 *   fc:    host double[nr], the radial profile f_c(r) of the coefficient,
 *          >= 0; NULL for 1.  Copied.
 *   Tc:    threshold of f_m (Eq. tc cites it without a formula; here the
 *          conductivity is held at its Tc value below Tc: f_m(T0) T0^expo =
 *          Tc^expo for T0 < Tc); <= 0 for f_m = 1.
 * The coefficient becomes c = scale f_c(r_i) f_m(T0) T0^expo (scale f_c(r_i)
 * without T0); for Eq. (visc) pass T0 = nu(x) rho with expo 1.  w V replaces
 * V in F, the explicit limit and the BE system (w V + dt L) x = w V u + dt h.
 * Takes effect with the next pa_set_coefficients, which must follow.
 * PA_ERR_ARG for a non-positive weight or a negative profile value. */
pa_status pa_set_profile(pa_ctx* ctx, const double* w_dev, const double* fc, double Tc);

/* Dirichlet boundary values at r_in and r_out, device double[ncomp][nt][np]
 * (copied; NULL leaves that side unchanged).  Ignored on no-flux sides. */
pa_status pa_set_bc(pa_ctx* ctx, const double* ub_in_dev, const double* ub_out_dev);

/* Explicit Euler stability limit dt_E = 2 / max_m sum_n |(V^-1 L)_mn|
 * (Gershgorin bound; App. A uses dt_Euler without a definition). */
pa_status pa_dt_explicit(pa_ctx* ctx, double* dt_e);

/* F = F(u) (affine != 0: including boundary data) or its linear part, for
 * device arrays of the field's shape.  u_dev and F_dev must not overlap. */
pa_status pa_apply(pa_ctx* ctx, const double* u_dev, double* F_dev, int32_t affine);

/* Diagonal of L = -V dF_lin/du on one component: device double[nr][nt][np]. */
pa_status pa_diag(pa_ctx* ctx, double* diag_dev);

/* Practical time step limit of the bound field, Eq. (ptl3): at the cell k of
 * largest |F| (ties: lowest linear index) the minimum over its six face
 * neighbours of -(u_k - u_nb)/(F_k - F_nb) where that pair has
 * du*dF < 0 (Eq. ptl2); +inf when none constrains.  k_lin may be NULL. */
pa_status pa_compute_ptl(pa_ctx* ctx, double* dt_ptl, int64_t* k_lin);

/* Full-grid form of the limit (Sec. 2 takes Eq. ptl2 at the largest |F|
 * only, assuming the most restrictive pair is found there): the minimum of
 * Eq. (ptl2) over every cell and each of its face neighbours, for the bound
 * field.  k_lin (may be NULL) receives the lowest linear cell index attaining
 * it, -1 when no pair constrains (dt_full = +inf).  A diagnostic of that
 * assumption; the advances use pa_compute_ptl's form. */
pa_status pa_compute_ptl_full(pa_ctx* ctx, double* dt_full, int64_t* k_lin);

/* pa_compute_ptl for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same limit and index, bit for bit, with no allocation in the call.
 * Its scratch -- the per-tile argmax partials and F on the three radial
 * levels around the cell of largest |F| -- is a 16 MiB array of device
 * memory that the library holds on every device it runs on until the
 * process ends.  FP64 contexts only (PA_ERR_ARG otherwise).  PA_ERR_ARG when
 * the problem needs more scratch than that: about 24 bytes per cell of one
 * radial level plus 16 bytes per stencil workgroup (256 x 512 x 1024 with
 * three components needs 12.8 MiB).  PA_ERR_HIP if the array's device
 * address could not be resolved at pa_init.  Every call on one device uses
 * the same array, which keeps the last call's contents: calls that overlap
 * in time on one device (other streams, other host threads) race. */
pa_status pa_compute_ptl_noalloc(pa_ctx* ctx, double* dt_ptl, int64_t* k_lin);

/* Block ILU(0) preconditioner, PC2 of Sec. 3.1 (non-overlapping ILU(0)):
 * z = P^{-1} r for device arrays of the field's shape (all components), P the
 * incomplete LU factorisation, with the sparsity of M and cells in natural
 * (i, j, k) order, of the block-diagonal part of M = wV + dt L on boxes of
 * PA_BILU0_BI x PA_BILU0_BJ x PA_BILU0_BK cells (every coupling between cells
 * of different boxes dropped; the periodic phi coupling is never inside a
 * box).  With the 7-point sparsity only the pivots differ from M.  The same
 * preconditioner serves the BE solves with pc = PA_PC_BILU0.  PA_OP_ISO7
 * only (PA_ERR_ARG otherwise); PA_ERR_BREAKDOWN if a pivot is not positive;
 * coefficients must be set.  r_dev and z_dev must not overlap. */
pa_status pa_bilu0_apply(pa_ctx* ctx, double dt, const double* r_dev, double* z_dev);

/* Advance the bound field over dt with RKL2 (Meyer, Balsara & Aslam 2014,
 * the paper's RKL2 reference) or RKG2 (App. A).  cycles > 0: that many equal
 * cycles; cycles == 0: dynamic PTL cycling (Sec. 2): each cycle takes
 * n = ceil(t_rem / max(dt_PTL, ptl_floor dt_E)) and length t_rem / n.
 * Stages per cycle: App. A formula (RKG2), s = ceil((sqrt(9+16 r)-1)/2)
 * (RKL2), r = dt_cycle/dt_E, odd rule per options.  stats may be NULL. */
pa_status pa_advance_rkl2(pa_ctx* ctx, double dt, int32_t cycles, pa_stats* stats);
pa_status pa_advance_rkg2(pa_ctx* ctx, double dt, int32_t cycles, pa_stats* stats);

/* Advance the bound field over dt with Backward Euler (Sec. 3.1): each
 * cycle solves (V + dt_c L) x = V u + dt_c h by point-Jacobi PCG from
 * x0 = u until ||r||_2 <= tol ||b||_2.  Cycling as pa_advance_rkl2. */
pa_status pa_advance_be_pcg(pa_ctx* ctx, double dt, double tol, int32_t cycles, pa_stats* stats);

/* ------------------------------------------------------------------------
 * Learned preconditioner for the Backward Euler solve.
 *
 * Not part of the paper: it replaces the point-Jacobi step of Sec. 3.1's
 * PCG (the paper keeps Jacobi because its ILU0 alternative does not
 * vectorise) with P(r) = r/D + sigma N(c), where D = V + dt diag(L),
 * sigma = RMS(r/D) over the grid and N is a three-layer 3x3x3 convolutional
 * network 8 -> 16 (+bias, ReLU) -> 16 (+bias, ReLU) -> 1 on the cell grid
 * (zero padding in r and theta, periodic in phi).  Input channels per cell
 * m: c0 = (r/D)/sigma, c1 = V/D, c2..c7 = -dt L(m, nb)/D(m) for the face
 * neighbours nb = r-, r+, theta-, theta+, phi-, phi+ (0 where none).  The
 * network runs in BF16 (round to nearest even) with FP32 accumulation, bias
 * and ReLU, on the matrix cores.  Because P is nonlinear the solve uses
 * flexible CG truncated to one previous direction (Notay, SIAM J. Sci.
 * Comput. 22 (2000)): beta = -<z, q_prev>/<p_prev, q_prev>, alpha =
 * <p, r>/<p, q>.  A step with <z, r> <= 0 takes z = r/D instead.  The
 * network's steps pay off while the error is dominated by local
 * components; once ||r|| falls by less than 10x over 10 iterations the
 * solve continues as Jacobi PCG from the current iterate.  Stopping rule
 * and tolerance as pa_advance_be_pcg.  Single-component FP64 contexts
 * only.
 *
 * Parameters: flat FP32 vector of PA_LPC_NPARAM values, in this order:
 * W1[16][8][3][3][3], b1[16], W2[16][16][3][3][3], b2[16], W3[1][16][3][3][3]
 * (W[co][ci][dr][dtheta][dphi], tap offsets -1, 0, +1).
 * ---------------------------------------------------------------------- */
#define PA_LPC_NPARAM 10832

/* Training options (pa_lpc_default_train_opts fills defaults). */
typedef struct {
    int32_t nsnap;       /* plain-PCG iterates kept as (residual, error) pairs. default 16 */
    int32_t batch;       /* pairs per Adam step. default 2 */
    int32_t epochs;      /* passes over the pairs. default 30 */
    int32_t seed;        /* batch order. default 4300 */
    double lr;           /* Adam step (beta1 0.9, beta2 0.999, eps 1e-8). default 1e-3 */
    double tol_star;     /* tolerance of the reference solve x*. default 1e-12 */
} pa_lpc_train_opts;

typedef struct {
    int32_t pairs, snapshots, steps, ref_iters; /* ref_iters: Jacobi-PCG iterations of x* */
    double loss_first, loss_last;  /* mean loss over the first and last epoch */
    double ms_pairs, ms_train;     /* wall time: pair generation, optimisation */
} pa_lpc_report;

void pa_lpc_default_train_opts(pa_lpc_train_opts* opts);

/* Set / read the network parameters (host float[PA_LPC_NPARAM]).  Setting
 * resets the Adam moments.  PA_ERR_NONFINITE for NaN/Inf values. */
pa_status pa_lpc_set_weights(pa_ctx* ctx, const float* theta);
pa_status pa_lpc_get_weights(pa_ctx* ctx, float* theta);

/* The eight input channels for residual r_dev (device double[nr][nt][np])
 * of the system at step dt, as FP32 values of the BF16 inputs: device
 * float[8][nr][nt][np]. */
pa_status pa_lpc_features(pa_ctx* ctx, double dt, const double* r_dev, float* feat_dev);

/* z = P(r) for the system at step dt (device arrays double[nr][nt][np]). */
pa_status pa_lpc_apply(pa_ctx* ctx, double dt, const double* r_dev, double* z_dev);

/* Training loss over npairs (r, e) pairs on the whole grid (device
 * double[npairs][nr][nt][np] each): the mean over pairs of the energy-norm
 * error of the preconditioned residual, |P(r) - e|_M^2 / |e|_M^2 with
 * M = V + dt L and |v|_M^2 = <v, M v> (the norm CG minimises), and its
 * gradient in the parameters (host double *loss, host float
 * grad[PA_LPC_NPARAM]).  npairs <= 64. */
pa_status pa_lpc_loss_grad(pa_ctx* ctx, double dt, int32_t npairs, const double* r_dev,
                           const double* e_dev, double* loss, float* grad);

/* Train the network on the system (V + dt L) x = V u + dt h of the bound
 * field: a Jacobi-PCG solve from x0 = u to tol_star gives x*; its iterates
 * x_k at up to nsnap iteration counts (0, 1, 2, 3, 4, 6, 9, 13, ...) give
 * the pairs (r_k = b - M x_k, e_k = x* - x_k); Adam minimises the loss of
 * pa_lpc_loss_grad over batches of pairs.  The bound field is left
 * unchanged; on divergence the previous weights are restored
 * (PA_ERR_NONFINITE).  report may be NULL. */
pa_status pa_lpc_train(pa_ctx* ctx, double dt, const pa_lpc_train_opts* opts,
                       pa_lpc_report* report);

#ifdef __cplusplus
}
#endif
#endif
