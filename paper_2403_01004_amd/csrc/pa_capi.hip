// pa_capi.hip -- host side of the C ABI (include/paradv.h): context, mesh
// metrics, coefficient set-up, the practical-time-step-limit controller and
// the RKL2 / RKG2 / Backward-Euler+PCG drivers.  Every arithmetic step on
// field data runs in the kernels of pa_kernels.hip and pa_vec.hip; the host
// computes only 1-D metric factors, recurrence coefficients and the cycle
// schedule.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/paradv.h"
#include "pa_internal.h"

// A host-side range in rocprofv3's marker trace (--marker-trace): the
// entry points and each PTL cycle, so a trace shows where the advance's
// launches were enqueued
namespace {
struct Range {
    explicit Range(const char* name) { roctxRangePush(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};
}  // namespace

using namespace pa;

// Scratch of pa_compute_ptl_noalloc: one copy per device, held from module
// load to process exit, shared by every call on that device.  In host code
// `scratch` names a host-side stand-in: the device copy's address comes from
// hipGetSymbolAddress (pa_init, once per device) and only that address is
// ever passed to kernels.
constexpr size_t kScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
bool g_scratch_done[kMaxDevices] = {};
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// Device address of `scratch` on device dev, which must be current; the
// lookup runs once per device.  Null (with *err set) if it failed.
void* scratch_address(int dev, hipError_t* err)
{
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_done[dev]) {
        void* ptr = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? ptr : nullptr;
        g_scratch_done[dev] = true;
    }
    *err = g_scratch_err[dev];
    return g_scratch_ptr[dev];
}
}  // namespace

namespace {

template <class T>
struct MetricDev {
    T *vr = nullptr, *vt = nullptr, *vp = nullptr, *gr = nullptr, *gtr = nullptr, *gtt = nullptr,
      *gpt = nullptr, *gpp = nullptr, *rtf = nullptr, *rtc = nullptr, *rpf = nullptr;
};

}  // namespace

struct pa_ctx {
    pa_desc d{};
    hipStream_t stream = nullptr;
    int dev = 0;
    std::string err;
    pa_opts opt{};
    std::vector<double> replay;
    size_t N = 0, NT = 0, P = 0, NCO = 0;  // cells per comp, all comps, per level, corners
    bool fp32 = false;
    // mesh metrics
    MetricDev<double> m64;
    MetricDev<float> m32;
    double *c_hr = nullptr, *c_wr = nullptr, *c_R = nullptr, *c_htt = nullptr, *c_sT = nullptr,
           *c_dpc = nullptr;
    // coefficients
    double* coef64 = nullptr;
    float* coef32 = nullptr;
    bool coef_var = false;
    double cscale = 1.0;
    double* e64 = nullptr;
    float* e32 = nullptr;
    double* diagL = nullptr;
    double* Dbuf = nullptr;  // Jacobi diagonal w V + dt diag(L) of the current BE solve
    // full operator forms: cell weight w of F = (1/w) div(...), radial
    // profile f_c and f_m threshold of the coefficient
    bool use_w = false;
    double* w64 = nullptr;
    float* w32 = nullptr;
    bool use_fc = false;
    double* fc_dev = nullptr;  // [nr]
    double Tc = 0.0;
    bool have_coef = false;
    double dtE = 0.0;
    // boundary data
    double *ub_in = nullptr, *ub_out = nullptr;
    float *ub_in32 = nullptr, *ub_out32 = nullptr;
    // field and work buffers
    double* u = nullptr;
    double* w[4] = {nullptr, nullptr, nullptr, nullptr};
    float* f[4] = {nullptr, nullptr, nullptr, nullptr};
    // reductions
    double* part = nullptr;
    long long* part_idx = nullptr;
    size_t part_cap = 0;
    DevState* st = nullptr;
    DevState* hst = nullptr;  // pinned host mirror
    int* flag = nullptr;
    int* hflag = nullptr;
    int rch = 16;
    std::vector<void*> allocs;
    // per-class launch timing (opts.timing): event pairs queued on the
    // stream, read back at the next synchronisation point
    struct Pending {
        int cls;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> ev_free;
    std::vector<Pending> ev_pending;
    pa_stats* tstats = nullptr;
    // learned preconditioner (single-component FP64 contexts)
    bool nn_ready = false;         // weights loaded
    bool nn_cpl_ok = false;        // face couplings match the coefficients
    int nn_adam_t = 0;
    float *nn_th = nullptr, *nn_m = nullptr, *nn_v = nullptr, *nn_grad = nullptr;
    NNWeights nn_w{};
    double* nn_scal = nullptr;     // [0] sigma, [1] loss, [2..2+kMaxPairs) per-pair sigma
    int* nn_flag = nullptr;        // FCG step takes the Jacobi direction
    double* nn_cpl = nullptr;      // [6][N] face couplings L(m, nb)
    __bf16* nn_xs = nullptr;       // [N][8] input channels on the whole grid
    double* nn_z = nullptr;        // [N] preconditioned residual
    double* nn_b = nullptr;        // [N] right-hand side of the current solve
    size_t nn_fcap = 0, nn_bcap = 0;  // points of the forward / backward work buffers
    __bf16 *nn_a1 = nullptr, *nn_a2 = nullptr;   // [cap][16] activations
    float* nn_out = nullptr;                     // [cap] network output
    __bf16 *nn_ga = nullptr, *nn_gb = nullptr;   // [cap][16] activation gradients
    __bf16* nn_g1 = nullptr;                     // [cap] output gradient
    float* nn_wpart = nullptr;                   // weight-gradient partials
    double* bilu0_ip = nullptr;  // [N] inverse block ILU(0) pivots of the current solve
    int pcg_hint = 0;            // iterations of the last PCG solve (first batch of the next)
    // deferred x update of the point-Jacobi solves: the directions of
    // kXGroup consecutive iterations, x updated once per group
    bool xg_on = false;          // the current solve defers its x updates
    double* xg_p = nullptr;      // [kXGroup - 1][NT] directions besides the solve's own
    float* xg_p32 = nullptr;     // the same for the FP32-matvec solves
    double* xg_alpha = nullptr;  // [kXGroup] the group's alphas
    bool jd_on = false;          // the current solve forms D from rows (JacD)
    double* jd_ab = nullptr;     // [nr * nt][2] row terms A, B of D at the solve's step
    double* jd_G = nullptr;      // [np] gpp_k + gpp_{k+1}
    void* xg_p0 = nullptr;       // the solve's own direction buffer (group slot 0)
    long long xg_q = 0;          // iterations queued in the current solve
    void* scratch = nullptr;     // this device's `scratch` (pa_compute_ptl_noalloc)
    hipError_t scratch_err = hipSuccess;
};

namespace {

pa_status fail(pa_ctx* c, pa_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return s;
}

#define HIPCHK(c, call)                                                                   \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail((c), PA_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));  \
    } while (0)

void* dev_alloc(pa_ctx* c, size_t bytes)
{
    void* p = nullptr;
    if (bytes == 0) bytes = 16;
    if (c->d.alloc) {
        p = c->d.alloc(bytes, c->d.alloc_user);
    } else {
        const hipError_t before = hipPeekAtLastError();
        if (hipMalloc(&p, bytes) != hipSuccess) {
            p = nullptr;
            // the caller reports the failure (or falls back, for the lazy
            // buffers of a solve): drop the allocation's own error so that
            // the launch checks do not see it, but keep an earlier one
            if (before == hipSuccess) (void)hipGetLastError();
        }
    }
    if (p) c->allocs.push_back(p);
    return p;
}

template <class T>
bool dev_upload(pa_ctx* c, T** dst, const std::vector<double>& src)
{
    std::vector<T> tmp(src.begin(), src.end());
    *dst = (T*)dev_alloc(c, sizeof(T) * tmp.size());
    if (!*dst) return false;
    return hipMemcpy(*dst, tmp.data(), sizeof(T) * tmp.size(), hipMemcpyHostToDevice) == hipSuccess;
}

template <class T>
Geo<T> geo(const pa_ctx* c, const MetricDev<T>& m)
{
    Geo<T> g;
    g.nr = c->d.nr; g.nt = c->d.nt; g.np = c->d.np; g.P = (int)c->P;
    g.vr = m.vr; g.vt = m.vt; g.vp = m.vp; g.gr = m.gr; g.gtr = m.gtr; g.gtt = m.gtt;
    g.gpt = m.gpt; g.gpp = m.gpp; g.rtf = m.rtf; g.rtc = m.rtc; g.rpf = m.rpf;
    return g;
}

bool ensure_parts(pa_ctx* c, size_t n)
{
    if (n <= c->part_cap) return true;
    c->part = (double*)dev_alloc(c, sizeof(double) * 3 * n);
    c->part_idx = (long long*)dev_alloc(c, sizeof(long long) * n);
    if (!c->part || !c->part_idx) return false;
    c->part_cap = n;
    return true;
}

// radial levels per workgroup: enough workgroups to fill 256 CUs several
// times over, without making each chunk so short that the two halo levels
// dominate
int pick_rch(int op, int nr, int nt, int np)
{
    const int nbx = blocks_per_plane(op, nt, np);
    int rch = 32;
    while (rch > 4 && (long long)nbx * ((nr + rch - 1) / rch) < 2048) rch /= 2;
    return rch;
}

template <class T>
KArgs<T> base_args(pa_ctx* c, int r_lo, int r_hi)
{
    KArgs<T> a;
    memset(&a, 0, sizeof a);
    a.bc_in = c->d.bc_in;
    a.bc_out = c->d.bc_out;
    a.affine = 1;
    a.r_lo = r_lo;
    a.r_hi = r_hi;
    a.rch = c->rch;
    a.nbx = blocks_per_plane(c->d.op, c->d.nt, c->d.np, sizeof(T) == 4);
    a.nrc = (r_hi - r_lo + c->rch - 1) / c->rch;
    a.nc = c->d.ncomp;
    a.only_c = -1;
    a.km2 = kKm2Array;
    a.part = c->part;
    a.part_idx = c->part_idx;
    a.flag = c->flag;
    if constexpr (sizeof(T) == 8) {
        a.coef = c->coef_var ? (const T*)c->coef64 : nullptr;
        a.e = (const T*)c->e64;
        a.ub_in = (const T*)c->ub_in;
        a.ub_out = (const T*)c->ub_out;
    } else {
        a.coef = c->coef_var ? (const T*)c->coef32 : nullptr;
        a.e = (const T*)c->e32;
        a.ub_in = (const T*)c->ub_in32;
        a.ub_out = (const T*)c->ub_out32;
    }
    a.cs = (T)c->cscale;
    if constexpr (sizeof(T) == 8) a.wgt = c->use_w ? (const T*)c->w64 : nullptr;
    else a.wgt = c->use_w ? (const T*)c->w32 : nullptr;
    return a;
}

template <class T>
void stencil(pa_ctx* c, int mode, bool virt, const KArgs<T>& a)
{
    if constexpr (sizeof(T) == 8) {
        const Geo<double> g = geo(c, c->m64);
        if (c->d.op == PA_OP_ISO7) launch_iso7<double>(mode, virt, g, a, c->stream);
        else if (c->d.op == PA_OP_VISC_VECTOR) launch_viscv<double>(mode, virt, g, a, c->stream);
        else launch_aligned<double>(mode, virt, g, a, c->stream);
    } else {
        const Geo<float> g = geo(c, c->m32);
        if (c->d.op == PA_OP_ISO7) launch_iso7<float>(mode, virt, g, a, c->stream);
        else if (c->d.op == PA_OP_VISC_VECTOR) launch_viscv<float>(mode, virt, g, a, c->stream);
        else launch_aligned<float>(mode, virt, g, a, c->stream);
    }
}

int ntiles(pa_ctx* c, int nlev, bool fp32 = false)
{
    return stencil_tiles(c->d.op, c->d.nt, c->d.np, nlev, c->rch, c->d.ncomp, fp32);
}

hipEvent_t get_event(pa_ctx* c)
{
    if (!c->ev_free.empty()) {
        hipEvent_t e = c->ev_free.back();
        c->ev_free.pop_back();
        return e;
    }
    // timing-only events: no system-scope fence at record time (the host
    // reads them after a stream synchronisation).  With the default fence
    // every record writes back and invalidates the caches, which opened a
    // ~10 us gap before and after each timed launch.
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

// times the launches queued during its lifetime under one kernel class
struct KScope {
    pa_ctx* c;
    int cls;
    hipEvent_t a = nullptr;
    KScope(pa_ctx* c_, int cls_) : c(c_), cls(cls_)
    {
        if (c->opt.timing && c->tstats) {
            a = get_event(c);
            if (a) (void)hipEventRecord(a, c->stream);
        }
    }
    ~KScope()
    {
        if (!a) return;
        hipEvent_t b = get_event(c);
        if (!b) { c->ev_free.push_back(a); return; }
        (void)hipEventRecord(b, c->stream);
        c->ev_pending.push_back({cls, a, b});
    }
};

// after a stream synchronisation: accumulate the finished event pairs
void flush_timing(pa_ctx* c)
{
    for (auto& p : c->ev_pending) {
        float ms = 0.f;
        if (c->tstats && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->tstats->kernel_ms[p.cls] += ms;
            c->tstats->kernel_calls[p.cls] += 1;
        }
        c->ev_free.push_back(p.a);
        c->ev_free.push_back(p.b);
    }
    c->ev_pending.clear();
}

pa_status sync_state(pa_ctx* c)
{
    HIPCHK(c, hipMemcpyAsync(c->hst, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->hflag, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    flush_timing(c);
    return PA_OK;
}

// ------------------------------------------------------------ STS tables

// RKL2 (Meyer, Balsara & Aslam 2014) and RKG2 with alpha = 3/2 (App. A):
// mu[k], nu[k], mut[k], gam[k] for k = 1..s.
void sts_table(int kind, int s, std::vector<double>& mu, std::vector<double>& nu,
               std::vector<double>& mut, std::vector<double>& gam)
{
    mu.assign(s + 1, 0.0); nu.assign(s + 1, 0.0); mut.assign(s + 1, 0.0); gam.assign(s + 1, 0.0);
    std::vector<double> b(s + 1);
    if (kind == PA_STS_RKL2) {
        const double w1 = 4.0 / ((double)s * s + s - 2.0);
        for (int j = 0; j <= s; ++j)
            b[j] = j < 2 ? 1.0 / 3.0 : ((double)j * j + j - 2.0) / (2.0 * j * (j + 1.0));
        mut[1] = w1 / 3.0;
        for (int j = 2; j <= s; ++j) {
            mu[j] = (2.0 * j - 1.0) / j * b[j] / b[j - 1];
            nu[j] = -(j - 1.0) / j * b[j] / b[j - 2];
            mut[j] = mu[j] * w1;
            gam[j] = (b[j - 1] - 1.0) * mut[j];
        }
    } else {
        const double w = 6.0 / ((s + 4.0) * (s - 1.0));
        for (int k = 0; k <= s; ++k)
            b[k] = k == 0 ? 1.0 : k == 1 ? 1.0 / 3.0 : k == 2 ? 1.0 / 15.0
                 : 4.0 * (k - 1.0) * (k + 4.0) / (3.0 * k * (k + 1.0) * (k + 2.0) * (k + 3.0));
        mut[1] = w;
        mu[2] = 0.5; nu[2] = -0.1; mut[2] = 0.5 * w; gam[2] = 0.0;
        for (int k = 3; k <= s; ++k) {
            mu[k] = (2.0 + 1.0 / k) * b[k] / b[k - 1];
            nu[k] = -(1.0 + 1.0 / k) * b[k] / b[k - 2];
            mut[k] = mu[k] * w;
            gam[k] = (0.5 * k * (k + 1.0) * b[k - 1] - 1.0) * mut[k];
        }
    }
}

int stage_count(int kind, double ratio, int force_odd)
{
    const double x = kind == PA_STS_RKL2 ? 0.5 * (sqrt(9.0 + 16.0 * ratio) - 1.0)
                                          : 0.5 * sqrt(25.0 + 24.0 * ratio) - 1.5;
    int s = (int)ceil(x);
    if (s < 2) s = 2;
    if (force_odd && s % 2 == 0) ++s;
    return s;
}

// ------------------------------------------------------------ passes

// y0 = F(u0) plus per-tile argmax partials; u0, y0 of storage type T
template <class T>
void first_pass(pa_ctx* c, const T* u0, T* y0)
{
    KArgs<T> a = base_args<T>(c, 0, c->d.nr);
    a.u = u0;
    a.out = y0;
    {
        KScope t(c, PA_K_FIRST);
        stencil<T>(c, kFirst, false, a);
    }
    KScope t(c, PA_K_REDUCE);
    launch_ptl_finalize<T>(c->part, c->part_idx, ntiles(c, c->d.nr, sizeof(T) == 4), u0, y0,
                           c->d.ncomp, c->d.nr,
                           c->d.nt, c->d.np, c->st, c->stream);
}

// one STS cycle of length dt with s stages, in place on u0 (y0 = F(u0) given)
template <class T>
void sts_cycle(pa_ctx* c, int kind, int s, double dt, T* u0, T* y0, T* A, T* B)
{
    std::vector<double> mu, nu, mut, gam;
    sts_table(kind, s, mu, nu, mut, gam);
    const double a1 = mut[1] * dt;
    T* prev = A;   // u_{k-1}
    T* prev2 = B;  // u_{k-2}
    for (int k = 2; k <= s; ++k) {
        KArgs<T> a = base_args<T>(c, 0, c->d.nr);
        a.u0 = u0;
        a.y0 = y0;
        a.a1 = a1;
        a.mu = mu[k];
        a.nu = nu[k];
        a.c0 = 1.0 - mu[k] - nu[k];
        a.mudt = mut[k] * dt;
        a.gdt = gam[k] * dt;
        bool virt = false;
        T* out;
        if (k == 2) {            // input u1 = u0 + a1 y0 (virtual), u_{k-2} = u0
            virt = true;
            a.u = u0;
            a.km2 = kKm2U0;
            out = A;
        } else if (k == 3) {     // input u2 (A), u_{k-2} = u1 (virtual)
            a.u = A;
            a.km2 = kKm2Virtual;
            out = (k == s) ? u0 : B;
        } else {
            a.u = prev;
            a.ukm2 = prev2;
            a.km2 = kKm2Array;
            out = (k == s) ? u0 : prev2;
        }
        a.out = out;
        {
            KScope t(c, PA_K_STAGE);
            stencil<T>(c, kStage, virt, a);
        }
        if (k == 2) { prev = A; prev2 = B; }
        else { T* t = prev2; prev2 = prev; prev = out == u0 ? prev : t; }
    }
    if (s == 2) {
        KScope t(c, PA_K_OTHER);
        launch_copy(A, u0, sizeof(T) * c->NT, c->stream);
    }
}

}  // namespace

// ================================================================ ABI

extern "C" {

void pa_default_options(pa_opts* o)
{
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->force_odd = 1;
    o->pc = PA_PC_JACOBI;
    o->max_iter = 10000;
    o->max_cycles = 100000;
    o->pcg_batch = 16;
    o->ptl_floor = 1.0;
}

const char* pa_last_error(const pa_ctx* c) { return c ? c->err.c_str() : "null context"; }

void pa_destroy(pa_ctx* c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    for (void* p : c->allocs) {
        if (c->d.free) c->d.free(p, c->d.alloc_user);
        else (void)hipFree(p);
    }
    for (auto& p : c->ev_pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (hipEvent_t e : c->ev_free) (void)hipEventDestroy(e);
    if (c->hst) (void)hipHostFree(c->hst);
    if (c->hflag) (void)hipHostFree(c->hflag);
    delete c;
}

pa_status pa_init(const pa_desc* d, void* stream, pa_ctx** out)
{
    if (!out) return PA_ERR_ARG;
    *out = nullptr;
    if (!d) return PA_ERR_ARG;
    if (d->nr < 1 || d->nt < 2 || d->np < 3 || d->ncomp < 1 || !d->r_faces || !d->t_faces ||
        !d->p_faces)
        return PA_ERR_ARG;
    if (d->op != PA_OP_ISO7 && d->op != PA_OP_FIELD_ALIGNED && d->op != PA_OP_VISC_VECTOR)
        return PA_ERR_ARG;
    if (d->op == PA_OP_VISC_VECTOR && d->ncomp != 3) return PA_ERR_ARG;
    if ((d->bc_in != PA_BC_DIRICHLET && d->bc_in != PA_BC_NOFLUX) ||
        (d->bc_out != PA_BC_DIRICHLET && d->bc_out != PA_BC_NOFLUX))
        return PA_ERR_ARG;
    if (d->prec != PA_FP64 && d->prec != PA_FP32_STAGES) return PA_ERR_ARG;
    if ((d->alloc == nullptr) != (d->free == nullptr)) return PA_ERR_ARG;
    const int nr = d->nr, nt = d->nt, np = d->np;
    const double *R = d->r_faces, *TH = d->t_faces, *PH = d->p_faces;
    for (int i = 0; i < nr; ++i)
        if (!(R[i + 1] > R[i]) || !(R[i] > 0.0)) return PA_ERR_ARG;
    for (int j = 0; j < nt; ++j)
        if (!(TH[j + 1] > TH[j])) return PA_ERR_ARG;
    if (TH[0] < 0.0 || TH[nt] > M_PI + 1e-12) return PA_ERR_ARG;
    for (int k = 0; k < np; ++k)
        if (!(PH[k + 1] > PH[k])) return PA_ERR_ARG;
    if ((double)nr * nt * np * d->ncomp > 4.0e9) return PA_ERR_ARG;

    pa_ctx* c = new pa_ctx();
    c->d = *d;
    c->d.r_faces = c->d.t_faces = c->d.p_faces = nullptr;
    c->stream = (hipStream_t)stream;
    pa_default_options(&c->opt);
    (void)hipGetDevice(&c->dev);
    c->scratch = scratch_address(c->dev, &c->scratch_err);
    c->P = (size_t)nt * np;
    c->N = c->P * nr;
    c->NT = c->N * d->ncomp;
    c->NCO = (size_t)(nr + 1) * (nt + 1) * np;
    c->fp32 = d->prec == PA_FP32_STAGES;
    c->rch = pick_rch(d->op, nr, nt, np);

    // 1-D metric factors (finite volume on the face mesh)
    std::vector<double> rc(nr), tc(nt), pc(np);
    for (int i = 0; i < nr; ++i) rc[i] = 0.5 * (R[i] + R[i + 1]);
    for (int j = 0; j < nt; ++j) tc[j] = 0.5 * (TH[j] + TH[j + 1]);
    for (int k = 0; k < np; ++k) pc[k] = 0.5 * (PH[k] + PH[k + 1]);
    const double period = PH[np] - PH[0];
    std::vector<double> dpc(np);  // centre distance between cells k-1 and k
    for (int k = 0; k < np; ++k) dpc[k] = k == 0 ? pc[0] + period - pc[np - 1] : pc[k] - pc[k - 1];
    std::vector<double> vr(nr), vt(nt), vp(np), gr(nr + 1), gtr(nr), gtt(nt + 1, 0.0), gpt(nt),
        gpp(np);
    for (int i = 0; i < nr; ++i) {
        vr[i] = (R[i + 1] * R[i + 1] * R[i + 1] - R[i] * R[i] * R[i]) / 3.0;
        gtr[i] = 0.5 * (R[i + 1] * R[i + 1] - R[i] * R[i]) / rc[i];
    }
    for (int ir = 0; ir <= nr; ++ir) {
        const double dist = ir == 0 ? rc[0] - R[0] : ir == nr ? R[nr] - rc[nr - 1] : rc[ir] - rc[ir - 1];
        gr[ir] = R[ir] * R[ir] / dist;
    }
    for (int j = 0; j < nt; ++j) {
        vt[j] = cos(TH[j]) - cos(TH[j + 1]);
        gpt[j] = (TH[j + 1] - TH[j]) / sin(tc[j]);
    }
    for (int jt = 1; jt < nt; ++jt) gtt[jt] = sin(TH[jt]) / (tc[jt] - tc[jt - 1]);
    for (int k = 0; k < np; ++k) {
        vp[k] = PH[k + 1] - PH[k];
        gpp[k] = 1.0 / dpc[k];
    }
    // corner metric factors
    std::vector<double> hr(nr + 1), wr(nr + 1), Rf(R, R + nr + 1), htt(nt + 1, 0.0), sT(nt + 1);
    for (int ic = 0; ic <= nr; ++ic) {
        if (ic == 0) { hr[ic] = 2.0 * (rc[0] - R[0]); wr[ic] = 0.5 * hr[ic]; }
        else if (ic == nr) { hr[ic] = 2.0 * (R[nr] - rc[nr - 1]); wr[ic] = 0.5 * hr[ic]; }
        else { hr[ic] = rc[ic] - rc[ic - 1]; wr[ic] = hr[ic]; }
    }
    for (int jc = 1; jc < nt; ++jc) htt[jc] = tc[jc] - tc[jc - 1];
    for (int jc = 0; jc <= nt; ++jc) sT[jc] = sin(TH[jc]);
    // change of basis between neighbouring cell centres (vector viscosity)
    std::vector<double> rtf(2 * (nt + 1)), rtc(2 * nt), rpf(2 * np);
    for (int jt = 0; jt <= nt; ++jt) {
        const double d = (jt > 0 && jt < nt) ? tc[jt] - tc[jt - 1] : 0.0;
        rtf[jt] = cos(d);
        rtf[nt + 1 + jt] = sin(d);
    }
    for (int j = 0; j < nt; ++j) { rtc[j] = sin(tc[j]); rtc[nt + j] = cos(tc[j]); }
    for (int k = 0; k < np; ++k) {
        const double h = sin(0.5 * dpc[k]);
        rpf[k] = 2.0 * h * h;  // 1 - cos, without cancellation
        rpf[np + k] = sin(dpc[k]);
    }

    bool ok = dev_upload(c, &c->m64.vr, vr) && dev_upload(c, &c->m64.vt, vt) &&
              dev_upload(c, &c->m64.vp, vp) && dev_upload(c, &c->m64.gr, gr) &&
              dev_upload(c, &c->m64.gtr, gtr) && dev_upload(c, &c->m64.gtt, gtt) &&
              dev_upload(c, &c->m64.gpt, gpt) && dev_upload(c, &c->m64.gpp, gpp) &&
              dev_upload(c, &c->m32.vr, vr) && dev_upload(c, &c->m32.vt, vt) &&
              dev_upload(c, &c->m32.vp, vp) && dev_upload(c, &c->m32.gr, gr) &&
              dev_upload(c, &c->m32.gtr, gtr) && dev_upload(c, &c->m32.gtt, gtt) &&
              dev_upload(c, &c->m32.gpt, gpt) && dev_upload(c, &c->m32.gpp, gpp) &&
              dev_upload(c, &c->m64.rtf, rtf) && dev_upload(c, &c->m64.rtc, rtc) &&
              dev_upload(c, &c->m64.rpf, rpf) && dev_upload(c, &c->m32.rtf, rtf) &&
              dev_upload(c, &c->m32.rtc, rtc) && dev_upload(c, &c->m32.rpf, rpf) &&
              dev_upload(c, &c->c_hr, hr) && dev_upload(c, &c->c_wr, wr) &&
              dev_upload(c, &c->c_R, Rf) && dev_upload(c, &c->c_htt, htt) &&
              dev_upload(c, &c->c_sT, sT) && dev_upload(c, &c->c_dpc, dpc);
    const size_t NT = c->NT, N = c->N, bcn = c->P * d->ncomp;
    c->coef64 = (double*)dev_alloc(c, sizeof(double) * N);
    c->diagL = (double*)dev_alloc(c, sizeof(double) * N);
    c->Dbuf = (double*)dev_alloc(c, sizeof(double) * N);
    c->ub_in = (double*)dev_alloc(c, sizeof(double) * bcn);
    c->ub_out = (double*)dev_alloc(c, sizeof(double) * bcn);
    ok = ok && c->coef64 && c->diagL && c->Dbuf && c->ub_in && c->ub_out;
    if (d->op == PA_OP_FIELD_ALIGNED) {
        c->e64 = (double*)dev_alloc(c, sizeof(double) * 3 * c->NCO);
        ok = ok && c->e64;
    }
    for (int q = 0; q < 4; ++q) {
        c->w[q] = (double*)dev_alloc(c, sizeof(double) * NT);
        ok = ok && c->w[q];
    }
    if (c->fp32) {
        c->coef32 = (float*)dev_alloc(c, sizeof(float) * N);
        c->ub_in32 = (float*)dev_alloc(c, sizeof(float) * bcn);
        c->ub_out32 = (float*)dev_alloc(c, sizeof(float) * bcn);
        ok = ok && c->coef32 && c->ub_in32 && c->ub_out32;
        if (d->op == PA_OP_FIELD_ALIGNED) {
            c->e32 = (float*)dev_alloc(c, sizeof(float) * 3 * c->NCO);
            ok = ok && c->e32;
        }
        for (int q = 0; q < 4; ++q) {
            c->f[q] = (float*)dev_alloc(c, sizeof(float) * NT);
            ok = ok && c->f[q];
        }
    }
    const size_t tiles = (size_t)std::max(stencil_tiles(d->op, nt, np, nr, c->rch, d->ncomp, false),
                                          stencil_tiles(d->op, nt, np, nr, c->rch, d->ncomp, true));
    const size_t nblk = (N + kBlock - 1) / kBlock;
    ok = ok && ensure_parts(c, tiles > nblk ? (tiles > 4096 ? tiles : 4096) : (nblk > 4096 ? nblk : 4096));
    c->st = (DevState*)dev_alloc(c, sizeof(DevState));
    c->flag = (int*)dev_alloc(c, sizeof(int));
    ok = ok && c->st && c->flag;
    if (ok && hipHostMalloc((void**)&c->hst, sizeof(DevState), hipHostMallocDefault) != hipSuccess)
        ok = false;
    if (ok && hipHostMalloc((void**)&c->hflag, sizeof(int), hipHostMallocDefault) != hipSuccess)
        ok = false;
    if (!ok) {
        pa_destroy(c);
        return PA_ERR_ALLOC;
    }
    launch_fill_zero(c->ub_in, sizeof(double) * bcn, c->stream);
    launch_fill_zero(c->ub_out, sizeof(double) * bcn, c->stream);
    launch_fill_zero(c->st, sizeof(DevState), c->stream);
    launch_fill_zero(c->flag, sizeof(int), c->stream);
    if (c->fp32) {
        launch_fill_zero(c->ub_in32, sizeof(float) * bcn, c->stream);
        launch_fill_zero(c->ub_out32, sizeof(float) * bcn, c->stream);
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
        pa_destroy(c);
        return PA_ERR_HIP;
    }
    *out = c;
    return PA_OK;
}

pa_status pa_set_options(pa_ctx* c, const pa_opts* o)
{
    if (!c) return PA_ERR_ARG;
    if (!o) return fail(c, PA_ERR_ARG, "null options");
    if (o->s_override < 0 || o->s_override == 1 || o->max_iter < 1 || o->max_cycles < 1 ||
        o->force_iters < 0 || o->pcg_batch < 1 || o->replay_n < 0 || !(o->ptl_floor >= 0.0) ||
        (o->replay_n > 0 && !o->replay_dt) ||
        (o->pc != PA_PC_JACOBI && o->pc != PA_PC_LEARNED && o->pc != PA_PC_BILU0))
        return fail(c, PA_ERR_ARG, "invalid option value");
    if (o->pc == PA_PC_BILU0 && c->d.op != PA_OP_ISO7)
        return fail(c, PA_ERR_ARG, "block ILU(0): 7-point operator only");
    if (o->pc == PA_PC_LEARNED) {
        if (c->d.ncomp != 1 || c->fp32)
            return fail(c, PA_ERR_ARG, "learned preconditioner: single-component FP64 contexts only");
        if (!c->nn_ready) return fail(c, PA_ERR_STATE, "learned preconditioner: no weights set");
    }
    c->opt = *o;
    c->replay.assign(o->replay_dt, o->replay_dt + (o->replay_n > 0 ? o->replay_n : 0));
    for (double x : c->replay)
        if (!(x > 0.0) || !isfinite(x)) return fail(c, PA_ERR_ARG, "replay lengths must be > 0");
    c->opt.replay_dt = nullptr;
    c->err.clear();
    return PA_OK;
}

pa_status pa_bind_field(pa_ctx* c, double* u)
{
    if (!c) return PA_ERR_ARG;
    if (!u) return fail(c, PA_ERR_ARG, "null field");
    c->u = u;
    return PA_OK;
}

pa_status pa_set_bc(pa_ctx* c, const double* ui, const double* uo)
{
    if (!c) return PA_ERR_ARG;
    const size_t n = c->P * c->d.ncomp;
    if (ui) launch_copy(ui, c->ub_in, sizeof(double) * n, c->stream);
    if (uo) launch_copy(uo, c->ub_out, sizeof(double) * n, c->stream);
    if (c->fp32) {
        launch_f64_to_f32(c->ub_in, c->ub_in32, n, c->stream);
        launch_f64_to_f32(c->ub_out, c->ub_out32, n, c->stream);
    }
    HIPCHK(c, hipGetLastError());
    return PA_OK;
}

pa_status pa_set_profile(pa_ctx* c, const double* w, const double* fc, double Tc)
{
    if (!c) return PA_ERR_ARG;
    if (!isfinite(Tc)) return fail(c, PA_ERR_ARG, "Tc must be finite");
    if (fc)
        for (int i = 0; i < c->d.nr; ++i)
            if (!(fc[i] >= 0.0) || !isfinite(fc[i]))
                return fail(c, PA_ERR_ARG, "f_c must be finite and >= 0");
    c->have_coef = false;
    c->nn_cpl_ok = false;
    c->Tc = Tc > 0.0 ? Tc : 0.0;
    c->use_fc = fc != nullptr;
    if (fc) {
        if (!c->fc_dev) c->fc_dev = (double*)dev_alloc(c, sizeof(double) * c->d.nr);
        if (!c->fc_dev) return fail(c, PA_ERR_ALLOC, "out of device memory");
        HIPCHK(c, hipMemcpy(c->fc_dev, fc, sizeof(double) * c->d.nr, hipMemcpyHostToDevice));
    }
    c->use_w = w != nullptr;
    if (w) {
        if (!c->w64) c->w64 = (double*)dev_alloc(c, sizeof(double) * c->N);
        if (c->fp32 && !c->w32) c->w32 = (float*)dev_alloc(c, sizeof(float) * c->N);
        if (!c->w64 || (c->fp32 && !c->w32)) return fail(c, PA_ERR_ALLOC, "out of device memory");
        launch_copy(w, c->w64, sizeof(double) * c->N, c->stream);
        if (c->fp32) launch_f64_to_f32(c->w64, c->w32, c->N, c->stream);
        launch_fill_zero(c->flag, sizeof(int), c->stream);
        launch_nonpositive(c->w64, c->N, c->flag, c->stream);
        HIPCHK(c, hipGetLastError());
        pa_status s = sync_state(c);
        if (s) return s;
        if (*c->hflag) {
            c->use_w = false;
            return fail(c, PA_ERR_ARG, "weights must be finite and > 0");
        }
    }
    HIPCHK(c, hipGetLastError());
    c->err.clear();
    return PA_OK;
}

pa_status pa_set_coefficients(pa_ctx* c, const double* T0, double scale, double expo,
                              const double* B)
{
    if (!c) return PA_ERR_ARG;
    if (!isfinite(scale) || scale < 0.0 || !isfinite(expo))
        return fail(c, PA_ERR_ARG, "scale must be finite and >= 0, expo finite");
    if (c->d.op == PA_OP_FIELD_ALIGNED && !B) return fail(c, PA_ERR_ARG, "field-aligned operator needs B");
    c->have_coef = false;
    c->nn_cpl_ok = false;
    launch_fill_zero(c->flag, sizeof(int), c->stream);
    const int N = (int)c->N;
    launch_coef(T0, scale, expo, c->use_fc ? c->fc_dev : nullptr, c->Tc, (int)c->P, N, c->coef64,
                c->coef32, c->flag, c->stream);
    c->coef_var = T0 != nullptr || c->use_fc;
    const double* wv = c->use_w ? c->w64 : nullptr;
    c->cscale = scale;
    const Geo<double> g = geo(c, c->m64);
    int np_ = 0;
    if (c->d.op == PA_OP_FIELD_ALIGNED) {
        CornerGeo cg{c->c_hr, c->c_wr, c->c_R, c->c_htt, c->c_sT, c->c_dpc};
        launch_corner_e(c->d.nr, c->d.nt, c->d.np, cg, c->coef64, B, c->e64, c->e32, c->flag,
                        c->stream);
        launch_diag_aligned(g, c->e64, wv, c->d.bc_in, c->d.bc_out, c->diagL, c->part, c->stream,
                            &np_);
    } else {
        launch_diag_iso7(g, c->coef_var ? c->coef64 : nullptr, scale, wv, c->d.bc_in, c->d.bc_out,
                         c->diagL, c->part, c->stream, &np_);
    }
    launch_reduce_max(c->part, np_, &c->st->gmax, c->stream);
    HIPCHK(c, hipGetLastError());
    pa_status s = sync_state(c);
    if (s) return s;
    if (*c->hflag) return fail(c, PA_ERR_NONFINITE, "non-finite or negative coefficient or field B");
    const double gm = c->hst->gmax;
    c->dtE = gm > 0.0 ? 2.0 / gm : INFINITY;
    c->have_coef = true;
    c->err.clear();
    return PA_OK;
}

pa_status pa_dt_explicit(pa_ctx* c, double* dt)
{
    if (!c) return PA_ERR_ARG;
    if (!dt) return fail(c, PA_ERR_ARG, "null output");
    if (!c->have_coef) return fail(c, PA_ERR_STATE, "coefficients not set");
    *dt = c->dtE;
    return PA_OK;
}

pa_status pa_diag(pa_ctx* c, double* out)
{
    if (!c) return PA_ERR_ARG;
    if (!out) return fail(c, PA_ERR_ARG, "null output");
    if (!c->have_coef) return fail(c, PA_ERR_STATE, "coefficients not set");
    launch_copy(c->diagL, out, sizeof(double) * c->N, c->stream);
    HIPCHK(c, hipGetLastError());
    return PA_OK;
}

pa_status pa_apply(pa_ctx* c, const double* u, double* F, int32_t affine)
{
    if (!c) return PA_ERR_ARG;
    if (!u || !F) return fail(c, PA_ERR_ARG, "null array");
    if (!c->have_coef) return fail(c, PA_ERR_STATE, "coefficients not set");
    const size_t bytes = sizeof(double) * c->NT;
    if ((const char*)u < (const char*)F + bytes && (const char*)F < (const char*)u + bytes)
        return fail(c, PA_ERR_ARG, "u and F overlap");
    KArgs<double> a = base_args<double>(c, 0, c->d.nr);
    a.u = u;
    a.out = F;
    a.affine = affine ? 1 : 0;
    stencil<double>(c, kApply, false, a);
    HIPCHK(c, hipGetLastError());
    return PA_OK;
}

pa_status pa_compute_ptl(pa_ctx* c, double* dt, int64_t* k)
{
    Range range("pa_compute_ptl");
    if (!c) return PA_ERR_ARG;
    if (!dt) return fail(c, PA_ERR_ARG, "null output");
    if (!c->have_coef) return fail(c, PA_ERR_STATE, "coefficients not set");
    if (!c->u) return fail(c, PA_ERR_STATE, "no field bound");
    launch_fill_zero(c->flag, sizeof(int), c->stream);
    if (c->fp32) {
        launch_f64_to_f32(c->u, c->f[0], c->NT, c->stream);
        first_pass<float>(c, c->f[0], c->f[1]);
    } else {
        first_pass<double>(c, c->u, c->w[0]);
    }
    HIPCHK(c, hipGetLastError());
    pa_status s = sync_state(c);
    if (s) return s;
    *dt = c->hst->dt_ptl;
    if (k) *k = c->hst->kmax;
    if (*c->hflag || isnan(*dt)) return fail(c, PA_ERR_NONFINITE, "non-finite F");
    return PA_OK;
}

pa_status pa_compute_ptl_full(pa_ctx* c, double* dt, int64_t* k)
{
    Range range("pa_compute_ptl_full");
    if (!c) return PA_ERR_ARG;
    if (!dt) return fail(c, PA_ERR_ARG, "null output");
    if (!c->have_coef) return fail(c, PA_ERR_STATE, "coefficients not set");
    if (!c->u) return fail(c, PA_ERR_STATE, "no field bound");
    launch_fill_zero(c->flag, sizeof(int), c->stream);
    first_pass<double>(c, c->u, c->w[0]);
    launch_ptl_full<double>(c->u, c->w[0], c->d.ncomp, c->d.nr, c->d.nt, c->d.np, c->part,
                            c->part_idx, c->st, c->stream);
    HIPCHK(c, hipGetLastError());
    pa_status s = sync_state(c);
    if (s) return s;
    if (*c->hflag) return fail(c, PA_ERR_NONFINITE, "non-finite F");
    *dt = c->hst->dt_full;
    if (k) *k = c->hst->kfull;
    return PA_OK;
}

pa_status pa_compute_ptl_noalloc(pa_ctx* c, double* dt, int64_t* k)
{
    if (!c) return PA_ERR_ARG;
    if (!dt) return fail(c, PA_ERR_ARG, "null output");
    if (!c->have_coef) return fail(c, PA_ERR_STATE, "coefficients not set");
    if (!c->u) return fail(c, PA_ERR_STATE, "no field bound");
    if (c->fp32) return fail(c, PA_ERR_ARG, "pa_compute_ptl_noalloc: FP64 contexts only");
    if (!c->scratch)
        return fail(c, PA_ERR_HIP, "scratch array of device %d not resolved: %s", c->dev,
                    hipGetErrorString(c->scratch_err));
    const int nr = c->d.nr;
    const size_t P = c->P, N = c->N;
    const int n = ntiles(c, nr);
    // scratch layout: device state | flag | argmax partials (value, index) |
    // F on the three radial levels around the argmax cell (one component)
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t o_flag = up(sizeof(DevState)), o_part = o_flag + 256;
    const size_t o_idx = o_part + up(sizeof(double) * n);
    const size_t o_F = o_idx + up(sizeof(long long) * n);
    const size_t need = o_F + sizeof(double) * 3 * P;
    if (need > kScratchBytes)
        return fail(c, PA_ERR_ARG,
                    "pa_compute_ptl_noalloc: needs %zu bytes of scratch (%d tiles, %zu cells "
                    "per radial level), the maximum is %zu",
                    need, n, P, kScratchBytes);
    unsigned char* sb = (unsigned char*)c->scratch;
    DevState* st = (DevState*)sb;
    int* flag = (int*)(sb + o_flag);
    double* part = (double*)(sb + o_part);
    long long* pidx = (long long*)(sb + o_idx);
    double* F3 = (double*)(sb + o_F);
    // the scratch keeps the previous call's contents: the NaN flag must start at zero
    launch_fill_zero(flag, sizeof(int), c->stream);
    {
        // pass 1: argmax partials of |F| without storing F
        KArgs<double> a = base_args<double>(c, 0, nr);
        a.u = c->u;
        a.out = nullptr;
        a.part = part;
        a.part_idx = pidx;
        a.flag = flag;
        KScope t(c, PA_K_FIRST);
        stencil<double>(c, kFirst, false, a);
    }
    launch_argmax(part, pidx, n, (long long)c->NT, st, c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(&c->hst->kmax, &st->kmax, sizeof(long long), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(c->hflag, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    flush_timing(c);
    const long long km = c->hst->kmax;
    if (*c->hflag || km < 0) return fail(c, PA_ERR_NONFINITE, "non-finite F");
    // pass 2: F of the argmax cell's component on radial levels [lo, hi);
    // the same kernel as pass 1 over fewer levels gives bit-identical values
    const size_t cc = (size_t)km / N;
    const int ik = (int)(((size_t)km % N) / P);
    const int lo = std::max(ik - 1, 0), hi = std::min(ik + 2, nr);
    // F3 holds levels lo..hi-1 of component cc.  The scalar operators treat
    // component cc as a one-component field, written at out + i P; the
    // vector viscosity couples the components, so it reads all three and
    // stores component cc only, at out + m for cell m of the whole field.
    // The finish reads cell m at F + m.  The bases are shifted back so that
    // every access lands in F3.
    const uintptr_t F3a = (uintptr_t)F3;
    {
        KArgs<double> a = base_args<double>(c, lo, hi);
        if (c->d.op == PA_OP_VISC_VECTOR) {
            a.u = c->u;
            a.only_c = (int)cc;
            a.out = (double*)(F3a - sizeof(double) * (cc * N + (size_t)lo * P));
        } else {
            a.nc = 1;
            a.u = c->u + cc * N;
            a.ub_in = c->ub_in + cc * P;
            a.ub_out = c->ub_out + cc * P;
            a.out = (double*)(F3a - sizeof(double) * (size_t)lo * P);
        }
        KScope t(c, PA_K_FIRST);
        stencil<double>(c, kApply, false, a);
    }
    {
        const double* Fw = (const double*)(F3a - sizeof(double) * (cc * N + (size_t)lo * P));
        KScope t(c, PA_K_REDUCE);
        launch_ptl_finalize<double>(part, pidx, n, c->u, Fw, c->d.ncomp, nr, c->d.nt, c->d.np,
                                    st, c->stream);
    }
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(c->hst, st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    flush_timing(c);
    *dt = c->hst->dt_ptl;
    if (k) *k = c->hst->kmax;
    if (isnan(*dt)) return fail(c, PA_ERR_NONFINITE, "non-finite F");
    c->err.clear();
    return PA_OK;
}

}  // extern "C""

// ---------------------------------------------------------------- drivers

namespace {

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    explicit Timer(hipStream_t st) : s(st)
    {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        (void)hipEventRecord(a, s);
    }
    double stop()
    {
        float ms = 0.f;
        (void)hipEventRecord(b, s);
        (void)hipEventSynchronize(b);
        (void)hipEventElapsedTime(&ms, a, b);
        return ms;
    }
    ~Timer()
    {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
};

// Cycle schedule shared by both schemes.  Returns PA_OK with *dtc and *last
// set, or an error.  Requires the PTL pass of the current iterate to have
// been queued when the schedule is dynamic.
pa_status next_cycle(pa_ctx* c, double dt, int cycles, int ncyc, double t_rem, pa_stats* st,
                     double* dtc, int* last)
{
    if (c->opt.replay_n > 0) {
        if (ncyc >= (int)c->replay.size()) return fail(c, PA_ERR_ARG, "replay schedule too short");
        *dtc = c->replay[ncyc];
        *last = ncyc + 1 == (int)c->replay.size();
    } else if (cycles > 0) {
        *dtc = dt / cycles;
        *last = ncyc + 1 == cycles;
    } else {
        pa_status s = sync_state(c);
        if (s) return s;
        const double ptl = c->hst->dt_ptl;
        if (*c->hflag || isnan(ptl) || !(ptl > 0.0))
            return fail(c, PA_ERR_NONFINITE, "non-finite field or time-step limit");
        if (ncyc == 0) { st->dt_ptl_first = ptl; st->k_first = c->hst->kmax; }
        if (ptl < st->dt_ptl_min) st->dt_ptl_min = ptl;
        double lim = ptl;
        if (lim < c->opt.ptl_floor * c->dtE) { lim = c->opt.ptl_floor * c->dtE; st->floored += 1; }
        const double nreq = ceil(t_rem / lim);
        if (!(nreq > 1.0)) { *dtc = t_rem; *last = 1; }
        else { *dtc = t_rem / nreq; *last = 0; }
    }
    if (ncyc >= c->opt.max_cycles) return fail(c, PA_ERR_MAXCYCLES, "more than %d cycles", c->opt.max_cycles);
    return PA_OK;
}

pa_status check_ready(pa_ctx* c, double dt)
{
    if (!c->have_coef) return fail(c, PA_ERR_STATE, "coefficients not set");
    if (!c->u) return fail(c, PA_ERR_STATE, "no field bound");
    if (!(dt > 0.0) || !isfinite(dt)) return fail(c, PA_ERR_ARG, "dt must be finite and > 0");
    return PA_OK;
}

void init_stats(pa_stats* st)
{
    memset(st, 0, sizeof *st);
    st->dt_ptl_first = st->dt_ptl_min = INFINITY;
    st->k_first = -1;
}

template <class T>
pa_status sts_advance(pa_ctx* c, int kind, double dt, int cycles, pa_stats* st, T* u0, T* y0, T* A,
                      T* B)
{
    double t_rem = dt;
    int ncyc = 0;
    pa_status s = PA_OK;
    while (true) {
        Range cyc("pa sts cycle");
        first_pass<T>(c, u0, y0);
        double dtc;
        int last;
        s = next_cycle(c, dt, cycles, ncyc, t_rem, st, &dtc, &last);
        if (s) break;
        const int sv = c->opt.s_override > 0 ? c->opt.s_override
                                             : stage_count(kind, dtc / c->dtE, c->opt.force_odd);
        if (ncyc < PA_MAX_LOG) { st->dt_cycle[ncyc] = dtc; st->per_cycle[ncyc] = sv; }
        st->s_total += sv;
        if (sv > st->s_max) st->s_max = sv;
        sts_cycle<T>(c, kind, sv, dtc, u0, y0, A, B);
        ++ncyc;
        if (last) break;
        t_rem -= dtc;
    }
    st->cycles = ncyc;
    return s;
}

pa_status advance_sts(pa_ctx* c, int kind, double dt, int32_t cycles, pa_stats* user)
{
    Range range(kind == PA_STS_RKL2 ? "pa_advance_rkl2" : "pa_advance_rkg2");
    if (!c) return PA_ERR_ARG;
    pa_status s = check_ready(c, dt);
    if (s) return s;
    if (cycles < 0) return fail(c, PA_ERR_ARG, "cycles must be >= 0");
    pa_stats local;
    pa_stats* st = user ? user : &local;
    init_stats(st);
    st->dt_explicit = c->dtE;
    Timer tm(c->stream);
    c->tstats = st;
    launch_fill_zero(c->flag, sizeof(int), c->stream);
    if (c->fp32) {
        {
            KScope t(c, PA_K_OTHER);
            launch_f64_to_f32(c->u, c->f[0], c->NT, c->stream);
        }
        s = sts_advance<float>(c, kind, dt, cycles, st, c->f[0], c->f[1], c->f[2], c->f[3]);
        KScope t(c, PA_K_OTHER);
        launch_f32_to_f64(c->f[0], c->u, c->NT, c->stream);
    } else {
        s = sts_advance<double>(c, kind, dt, cycles, st, c->u, c->w[0], c->w[1], c->w[2]);
    }
    if (hipGetLastError() != hipSuccess && !s) s = fail(c, PA_ERR_HIP, "kernel launch failed");
    st->ms_total = tm.stop();
    pa_status s2 = sync_state(c);
    if (!s) {
        if (s2) s = s2;
        else if (*c->hflag) s = fail(c, PA_ERR_NONFINITE, "non-finite values in the advance");
    }
    c->tstats = nullptr;
    st->status = s;
    if (!s) c->err.clear();
    return s;
}

}  // namespace

extern "C" {

pa_status pa_advance_rkl2(pa_ctx* c, double dt, int32_t cycles, pa_stats* st)
{
    return advance_sts(c, PA_STS_RKL2, dt, cycles, st);
}

pa_status pa_advance_rkg2(pa_ctx* c, double dt, int32_t cycles, pa_stats* st)
{
    return advance_sts(c, PA_STS_RKG2, dt, cycles, st);
}

}  // extern "C"

namespace {

static_assert(kXGroup == PA_PCG_XGROUP, "x-update group of the header");

// Direction buffers of the deferred x update (PT: the solve's direction
// type), allocated on first use; false when device memory is short (the
// solve then updates x in place)
template <class PT>
PT*& xg_bufs(pa_ctx* c)
{
    if constexpr (sizeof(PT) == 8) return c->xg_p;
    else return c->xg_p32;
}

template <class PT>
bool xg_ready(pa_ctx* c)
{
    PT*& b = xg_bufs<PT>(c);
    if (!b) b = (PT*)dev_alloc(c, sizeof(PT) * c->NT * (kXGroup - 1));
    if (!c->xg_alpha) c->xg_alpha = (double*)dev_alloc(c, sizeof(double) * kXGroup);
    return b && c->xg_alpha;
}

// Row form of the Jacobi diagonal (7-point operator, constant coefficient,
// no weight), arrays allocated on first use; false when not applicable or
// device memory is short (D is then read per cell)
bool jd_ready(pa_ctx* c)
{
    if (c->d.op == PA_OP_FIELD_ALIGNED || c->coef_var || c->use_w) return false;
    if (!c->jd_ab) c->jd_ab = (double*)dev_alloc(c, sizeof(double) * 2 * c->d.nr * c->d.nt);
    if (!c->jd_G) c->jd_G = (double*)dev_alloc(c, sizeof(double) * c->d.np);
    return c->jd_ab && c->jd_G;
}

JacD jd_of(pa_ctx* c)
{
    JacD j;
    if (c->jd_on) {
        j.ab = c->jd_ab;
        j.G = c->jd_G;
        j.vp = c->m64.vp;
        j.np = (unsigned)c->d.np;
    }
    return j;
}

template <class PT>
PT* xg_slot(pa_ctx* c, int t)
{
    return t == 0 ? (PT*)c->xg_p0 : xg_bufs<PT>(c) + (size_t)(t - 1) * c->NT;
}

// x += alpha_t p_t over the first `count` slots of the group
template <class PT>
void xg_flush(pa_ctx* c, int count)
{
    XSlots<PT> sl;
    for (int t = 0; t < kXGroup; ++t) sl.p[t] = xg_slot<PT>(c, t);
    KScope t(c, PA_K_DIR);
    launch_pcg_xflush<PT>(c->NT, c->u, sl, c->xg_alpha, count, c->stream);
}

// Queue n PCG iterations (each skipped on the device once the solve is
// done), point Jacobi or block ILU(0) preconditioned.  PT is the storage
// type of the search direction and the matvec (double, or float for the
// FP32-matvec inner solves); x, r and all scalars are FP64.  Point Jacobi:
// matvec, alpha, r update, stopping test, then the new direction; x +=
// alpha p either in the same kernel (p is read once for both; the iteration
// that stops the solve still applies its x update there) or, when the
// group buffers could be allocated, deferred: once per kXGroup iterations,
// from the group's directions kept in their own buffers.
template <class PT>
void pcg_queue(pa_ctx* c, double dtc, double* r, PT* p, PT* q, int n)
{
    const int nr = c->d.nr, nc = c->d.ncomp;
    const int mt = ntiles(c, nr, sizeof(PT) == 4);
    int nparts = 0;
    // block ILU(0): the preconditioned residual goes to the y0 buffer, free
    // once the solve has started
    const bool bilu0 = c->opt.pc == PA_PC_BILU0;
    const Geo<double> g = geo(c, c->m64);
    const KArgs<double> a64 = base_args<double>(c, 0, nr);
    double* zb = c->w[0];
    for (int b = 0; b < n; ++b) {
        KArgs<PT> a = base_args<PT>(c, 0, nr);
        if (c->xg_on && !bilu0) {
            // deferred x update: iteration k reads its direction from
            // group slot k % kXGroup and writes the next one to the
            // following slot; the group's x update runs after the last
            // iteration's alpha is known and before its slot is reused
            const int sl = (int)(c->xg_q % kXGroup);
            PT* pc = xg_slot<PT>(c, sl);
            PT* pn = xg_slot<PT>(c, (sl + 1) % kXGroup);
            double* as = c->xg_alpha + sl;
            a.u = pc;
            a.out = q;
            a.affine = 0;
            a.dt = dtc;
            a.done = &c->st->done;
            {
                KScope t(c, PA_K_MATVEC);
                stencil<PT>(c, kMatvec, false, a);
            }
            {
                KScope t(c, PA_K_REDUCE);
                launch_pcg_alpha(c->part, mt, c->st, c->stream, as);
            }
            {
                KScope t(c, PA_K_UPDATE);
                launch_pcg_update<PT>(c->N, nc, c->Dbuf, nullptr, r, pc, q, c->st, c->part,
                                      &nparts, c->stream, jd_of(c));
            }
            {
                KScope t(c, PA_K_REDUCE);
                launch_pcg_beta(c->part, nparts, c->st, c->stream, as);
            }
            if (sl == kXGroup - 1) xg_flush<PT>(c, kXGroup);
            {
                KScope t(c, PA_K_DIR);
                launch_pcg_dir_next<PT>(c->N, nc, c->Dbuf, r, pc, pn, c->st, c->stream,
                                        jd_of(c));
            }
            ++c->xg_q;
            continue;
        }
        a.u = p;
        a.out = q;
        a.affine = 0;
        a.dt = dtc;
        a.done = &c->st->done;
        {
            KScope t(c, PA_K_MATVEC);
            stencil<PT>(c, kMatvec, false, a);
        }
        {
            KScope t(c, PA_K_REDUCE);
            launch_pcg_alpha(c->part, mt, c->st, c->stream);
        }
        if (bilu0) {
            {
                KScope t(c, PA_K_UPDATE);
                // the block solve is bound by its wavefront steps, not by
                // HBM: it takes the x update too (measured: cheaper than
                // one more stream in the direction kernel)
                launch_pcg_update_bilu0<PT>(g, nc, a64.coef, a64.cs, dtc, c->bilu0_ip, c->u, r, p,
                                            q, zb, c->st, c->part, &nparts, c->stream);
            }
            {
                KScope t(c, PA_K_REDUCE);
                launch_pcg_beta(c->part, nparts, c->st, c->stream);
            }
            KScope t(c, PA_K_DIR);
            launch_pcg_dir_z<PT>(c->NT, zb, nullptr, p, c->st, c->stream);
            continue;
        }
        {
            KScope t(c, PA_K_UPDATE);
            launch_pcg_update<PT>(c->N, nc, c->Dbuf, nullptr, r, p, q, c->st, c->part, &nparts,
                                  c->stream);
        }
        {
            KScope t(c, PA_K_REDUCE);
            launch_pcg_beta(c->part, nparts, c->st, c->stream);
        }
        KScope t(c, PA_K_DIR);
        launch_pcg_dir<PT>(c->N, nc, c->Dbuf, r, c->u, p, c->st, c->stream);
    }
}

// Iterations still needed, estimated from the residual decrease so far
// (the mean contraction of ||r||^2 per iteration carried on to the stopping
// level); `fallback` when there is nothing to go on
int pcg_remaining(const DevState* h, int fallback)
{
    double target = h->tol * h->tol * h->bb;
    if (h->mode == 1) target = std::max(target, h->eta * h->eta * h->rr0);
    if (h->iters <= 0 || !(target > 0.0) || !(h->rr > target) || !(h->rr < h->rr0))
        return fallback;
    const double per_iter = std::log(h->rr / h->rr0) / h->iters;   // < 0
    const double n = std::ceil(std::log(target / h->rr) / per_iter);
    return n < 1.0 ? 1 : n > 1e6 ? 1000000 : (int)n;
}

// One PCG solve of M d = r0 from the state queued by launch_pcg_init /
// launch_pcg_resid + launch_pcg_start: iterations are queued in batches and
// the host reads the device state after each batch.  The first batch is the
// iteration count of the previous solve on the context (the solves of a
// PTL-cycled advance take similar counts), capped at pcg_batch; a later
// batch is the estimate of pcg_remaining, capped at pcg_batch.  Iterations
// queued after the solve stopped exit at once but still cost their
// launches, and each batch costs a host check; the batching never changes
// the result.
template <class PT>
pa_status pcg_loop(pa_ctx* c, double dtc, double* r, PT* p, PT* q)
{
    int batch = c->opt.pcg_batch;
    if (c->opt.force_iters <= 0 && c->pcg_hint > 0) batch = std::min(batch, c->pcg_hint);
    const int later = std::max(1, c->opt.pcg_batch / 4);
    // the deferred x updates of a last, incomplete group
    auto finish_x = [&] {
        if (c->xg_on && c->xg_q % kXGroup) xg_flush<PT>(c, (int)(c->xg_q % kXGroup));
    };
    while (true) {
        pcg_queue<PT>(c, dtc, r, p, q, batch);
        pa_status s = sync_state(c);
        if (s) {
            finish_x();
            return s;
        }
        if (c->hst->done) {
            finish_x();
            c->pcg_hint = c->hst->iters;
            return PA_OK;
        }
        batch = c->opt.force_iters > 0 ? later
                                        : std::min(c->opt.pcg_batch, pcg_remaining(c->hst, later));
    }
}

// Block ILU(0) of M = wV + dt L at dt (D = wV + dt diag L already in Dbuf):
// inverse pivots into bilu0_ip.  PA_ERR_BREAKDOWN if a pivot is not positive.
pa_status bilu0_factor(pa_ctx* c, double dtc)
{
    const size_t nb = (size_t)bilu0_boxes(c->d.nr, c->d.nt, c->d.np);
    if (!c->bilu0_ip) c->bilu0_ip = (double*)dev_alloc(c, sizeof(double) * c->N);
    if (!c->bilu0_ip || !ensure_parts(c, nb))
        return fail(c, PA_ERR_ALLOC, "block ILU(0): out of device memory");
    const Geo<double> g = geo(c, c->m64);
    const KArgs<double> a = base_args<double>(c, 0, c->d.nr);
    launch_fill_zero(c->flag, sizeof(int), c->stream);
    {
        KScope t(c, PA_K_INIT);
        launch_bilu0_factor(g, a.coef, a.cs, dtc, c->Dbuf, c->bilu0_ip, c->flag, c->stream);
    }
    HIPCHK(c, hipGetLastError());
    pa_status s = sync_state(c);
    if (s) return s;
    if (*c->hflag) return fail(c, PA_ERR_BREAKDOWN, "block ILU(0): pivot not positive");
    return PA_OK;
}

// Start of a block ILU(0) solve after launch_pcg_start: p = z0 = P^{-1} r0
// and rho = <r0, z0>
template <class PT>
void bilu0_start(pa_ctx* c, double dtc, const double* r, PT* p)
{
    const Geo<double> g = geo(c, c->m64);
    const KArgs<double> a = base_args<double>(c, 0, c->d.nr);
    int nb = 0;
    KScope t(c, PA_K_INIT);
    launch_bilu0_solve<PT>(g, c->d.ncomp, a.coef, a.cs, dtc, c->bilu0_ip, r, p, c->part, &nb,
                           c->stream);
    launch_pcg_set_rho(c->part, nb, c->st, c->stream);
}

// F(0) on the two radial boundary levels into q (the boundary-data part of
// F, used to form b = V u + dt V F(0))
void boundary_data(pa_ctx* c, double* q)
{
    const int nr = c->d.nr;
    for (int side = 0; side < 2; ++side) {
        const int lv = side == 0 ? 0 : nr - 1;
        if (side == 1 && nr == 1) break;
        KArgs<double> a = base_args<double>(c, lv, lv + 1);
        a.rch = 1;
        a.nrc = 1;
        a.u = c->u;
        a.y0 = c->u;
        a.a1 = -1.0;  // virtual input u - u = 0
        a.out = q;
        stencil<double>(c, kApply, true, a);
    }
}


// ---------------------------------------------------------------- learned PC

constexpr int kMaxPairs = 64;

void dev_free(pa_ctx* c, void* p)
{
    if (!p) return;
    (void)hipStreamSynchronize(c->stream);
    for (size_t i = 0; i < c->allocs.size(); ++i)
        if (c->allocs[i] == p) {
            c->allocs.erase(c->allocs.begin() + (long)i);
            break;
        }
    if (c->d.free) c->d.free(p, c->d.alloc_user);
    else (void)hipFree(p);
}

template <class T>
bool need(pa_ctx* c, T*& p, size_t bytes)
{
    if (!p) p = (T*)dev_alloc(c, bytes);
    return p != nullptr;
}

// parameters, Adam moments, BF16 operand tables, scalars
bool nn_alloc_base(pa_ctx* c)
{
    const size_t np = sizeof(float) * NN_NPARAM;
    return need(c, c->nn_th, np) && need(c, c->nn_m, np) && need(c, c->nn_v, np) &&
           need(c, c->nn_grad, np) && need(c, c->nn_w.f1, 2 * 16 * 224) &&
           need(c, c->nn_w.f2, 2 * 16 * 448) && need(c, c->nn_w.f3, 2 * 16 * 448) &&
           need(c, c->nn_w.d2, 2 * 16 * 448) && need(c, c->nn_w.d3, 2 * 16 * 32) &&
           need(c, c->nn_scal, sizeof(double) * (2 + kMaxPairs)) &&
           need(c, c->nn_flag, sizeof(int));
}

// whole-grid buffers: couplings, input channels, z, b
bool nn_alloc_grid(pa_ctx* c)
{
    const size_t N = c->N;
    return need(c, c->nn_cpl, sizeof(double) * 6 * N) && need(c, c->nn_xs, 2 * 8 * N) &&
           need(c, c->nn_z, sizeof(double) * N) && need(c, c->nn_b, sizeof(double) * N);
}

bool nn_fwd_work(pa_ctx* c, size_t pts)
{
    if (pts <= c->nn_fcap) return true;
    dev_free(c, c->nn_a1);
    dev_free(c, c->nn_a2);
    dev_free(c, c->nn_out);
    c->nn_a1 = c->nn_a2 = nullptr;
    c->nn_out = nullptr;
    c->nn_fcap = 0;
    if (!need(c, c->nn_a1, 2 * 16 * pts) || !need(c, c->nn_a2, 2 * 16 * pts) ||
        !need(c, c->nn_out, sizeof(float) * pts))
        return false;
    c->nn_fcap = pts;
    return true;
}

bool nn_bwd_work(pa_ctx* c, size_t pts)
{
    if (pts <= c->nn_bcap) return true;
    dev_free(c, c->nn_ga);
    dev_free(c, c->nn_gb);
    dev_free(c, c->nn_g1);
    dev_free(c, c->nn_wpart);
    c->nn_ga = c->nn_gb = c->nn_g1 = nullptr;
    c->nn_wpart = nullptr;
    c->nn_bcap = 0;
    const int nb = (int)((pts + c->N - 1) / c->N);
    const size_t wp = (size_t)nn_wgrad_partials(nb, c->d.nr, c->d.nt, c->d.np) * 16 * 433;
    if (!need(c, c->nn_ga, 2 * 16 * pts) || !need(c, c->nn_gb, 2 * 16 * pts) ||
        !need(c, c->nn_g1, 2 * pts) || !need(c, c->nn_wpart, sizeof(float) * wp))
        return false;
    c->nn_bcap = pts;
    return true;
}

// Static input channels c1..c7 of the system at step dt into nn_xs; also
// D = V + dt diag(L) into Dbuf when make_D
void nn_static(pa_ctx* c, double dt, bool make_D)
{
    const Geo<double> g = geo(c, c->m64);
    if (!c->nn_cpl_ok) {
        launch_couplings(g, c->d.op, c->coef_var ? c->coef64 : nullptr, c->cscale, c->e64,
                         c->d.bc_in, c->d.bc_out, c->nn_cpl, c->stream);
        c->nn_cpl_ok = true;
    }
    const double* wv = c->use_w ? c->w64 : nullptr;
    if (make_D) launch_jacobi_D(g, dt, wv, c->diagL, c->Dbuf, c->stream);
    launch_nn_static(g, dt, wv, c->Dbuf, c->nn_cpl, c->nn_xs, c->stream);
}

// out = N(x) on nb elements of nr x nt x np cells (activations kept in a1, a2)
void nn_forward(pa_ctx* c, int nb, int nr, int nt, int np, int per, const int* done,
                const __bf16* x)
{
    launch_nn_conv(1, 0, nb, nr, nt, np, per, done, x, c->nn_w, c->nn_th, nullptr, c->nn_a1,
                   c->stream);
    launch_nn_conv(2, 0, nb, nr, nt, np, per, done, c->nn_a1, c->nn_w, c->nn_th, nullptr, c->nn_a2,
                   c->stream);
    launch_nn_conv(3, 0, nb, nr, nt, np, per, done, c->nn_a2, c->nn_w, c->nn_th, nullptr, c->nn_out,
                   c->stream);
}

// grad += d(sum g1 * out)/dtheta for the last forward pass on input x
void nn_backward(pa_ctx* c, int nb, int nr, int nt, int np, int per, const __bf16* x)
{
    launch_nn_wgrad(3, nb, nr, nt, np, per, c->nn_a2, c->nn_g1, c->nn_wpart, c->nn_grad, c->stream);
    launch_nn_conv(3, 1, nb, nr, nt, np, per, nullptr, c->nn_g1, c->nn_w, c->nn_th, c->nn_a2,
                   c->nn_ga, c->stream);
    launch_nn_wgrad(2, nb, nr, nt, np, per, c->nn_a1, c->nn_ga, c->nn_wpart, c->nn_grad, c->stream);
    launch_nn_conv(2, 1, nb, nr, nt, np, per, nullptr, c->nn_ga, c->nn_w, c->nn_th, c->nn_a1,
                   c->nn_gb, c->stream);
    launch_nn_wgrad(1, nb, nr, nt, np, per, x, c->nn_gb, c->nn_wpart, c->nn_grad, c->stream);
}

// sigma = RMS(r/D) into nn_scal[0], c0 into nn_xs, network output into nn_out
void nn_precond(pa_ctx* c, const double* r, const int* done)
{
    launch_nn_sigma(c->N, r, c->Dbuf, done, c->part, c->nn_scal, c->stream);
    launch_nn_c0(c->N, r, c->Dbuf, c->nn_scal, done, c->nn_xs, c->stream);
    nn_forward(c, 1, c->d.nr, c->d.nt, c->d.np, 1, done, c->nn_xs);
}

// M v for device v, Mv [N] (one component); per-tile partials of <v, M v>
// into c->part; returns their count
int nn_matvec(pa_ctx* c, double dt, const double* v, double* Mv)
{
    KArgs<double> a = base_args<double>(c, 0, c->d.nr);
    a.u = v;
    a.out = Mv;
    a.affine = 0;
    a.dt = dt;
    stencil<double>(c, kMatvec, false, a);
    return ntiles(c, c->d.nr);
}

// Energy-norm loss |P(r) - e|_M^2 / |e|_M^2 averaged over nb whole-grid
// pairs and its gradient: inputs x [nb][N][8] and zj = r/D [nb][N] built,
// e[b], sig[b] = RMS(r/D), den[b] = |e|_M^2 per pair.  The loss is added to
// *lossacc (device) and the gradient to nn_grad; d, Md are [N] work arrays.
void nn_energy_step(pa_ctx* c, double dt, int nb, const __bf16* x, const double* zj,
                    const double* const* e, const double* const* sig, const double* const* den,
                    double* d, double* Md, double* lossacc)
{
    const int nr = c->d.nr, nt = c->d.nt, np = c->d.np;
    const size_t N = c->N;
    hipStream_t S = c->stream;
    nn_forward(c, nb, nr, nt, np, 1, nullptr, x);
    for (int b = 0; b < nb; ++b) {
        launch_nn_resid(N, zj + (size_t)b * N, c->nn_out + (size_t)b * N, sig[b], e[b], d, S);
        const int mt = nn_matvec(c, dt, d, Md);
        launch_scal_reduce(c->part, mt, den[b], 1.0 / nb, lossacc, S);
        launch_energy_gout(N, Md, sig[b], den[b], 1.0 / nb, c->nn_g1 + (size_t)b * N, S);
    }
    nn_backward(c, nb, nr, nt, np, 1, x);
}

// FCG(1) with the learned preconditioner from the state queued by
// launch_pcg_init (Dbuf, r0, b in nn_b) and launch_pcg_start; less than a
// 10x reduction of ||r|| over 10 iterations hands the solve over to Jacobi
// PCG from the current iterate.  *its: iterations; *fallbacks += Jacobi
// steps + hand-overs.
pa_status fcg_solve(pa_ctx* c, double dtc, double tol, double* r, double* p, double* q, int* its,
                    int* fallbacks)
{
    const int nr = c->d.nr;
    const size_t N = c->N;
    const int mt = ntiles(c, nr);
    const int* done = &c->st->done;
    hipStream_t S = c->stream;
    int nparts = 0;
    launch_fill_zero(&c->st->nonfinite, sizeof(int), S);
    {
        KScope t(c, PA_K_NN);
        nn_static(c, dtc, false);
        nn_precond(c, r, done);
        const int nb = launch_fcg_combine(N, 1, r, r, c->Dbuf, c->nn_out, c->nn_scal, done, c->nn_z,
                                          c->part, S);
        launch_fcg_first(c->part, nb, c->st, c->nn_flag, S);
        const int nd = launch_fcg_dir(N, 1, c->nn_z, r, c->Dbuf, c->nn_flag, c->st, p, c->part, S);
        launch_fcg_pr(c->part, nd, c->st, S);
    }
    pa_status s = sync_state(c);
    if (s) return s;
    // hand-over rule: the network's steps pay off while they cut ||r|| by at
    // least kGain over kWindow iterations (faster than Jacobi PCG's typical
    // rate on stiff systems); after a slower window the solve continues as
    // Jacobi PCG from the current iterate
    constexpr int batch = 10, kWindow = 10;
    constexpr double kGain = 10.0;
    int ref_it = 0;
    double ref_rr = c->hst->rr;
    bool restart = false;
    while (!c->hst->done) {
        for (int b = 0; b < batch; ++b) {
            KArgs<double> a = base_args<double>(c, 0, nr);
            a.u = p;
            a.out = q;
            a.affine = 0;
            a.dt = dtc;
            a.done = done;
            {
                KScope t(c, PA_K_MATVEC);
                stencil<double>(c, kMatvec, false, a);
            }
            {
                KScope t(c, PA_K_REDUCE);
                launch_fcg_alpha(c->part, mt, c->st, S);
            }
            {
                KScope t(c, PA_K_UPDATE);
                launch_pcg_update<double>(N, 1, c->Dbuf, c->u, r, p, q, c->st, c->part, &nparts, S);
            }
            {
                KScope t(c, PA_K_REDUCE);
                launch_fcg_check(c->part, nparts, c->st, S);
            }
            KScope t(c, PA_K_NN);
            nn_precond(c, r, done);
            const int nb = launch_fcg_combine(N, 1, r, q, c->Dbuf, c->nn_out, c->nn_scal, done,
                                              c->nn_z, c->part, S);
            launch_fcg_beta(c->part, nb, c->st, c->nn_flag, S);
            const int nd = launch_fcg_dir(N, 1, c->nn_z, r, c->Dbuf, c->nn_flag, c->st, p, c->part, S);
            launch_fcg_pr(c->part, nd, c->st, S);
        }
        s = sync_state(c);
        if (s) return s;
        if (c->hst->done) break;
        if (c->hst->iters - ref_it >= kWindow) {
            if (kGain * sqrt(c->hst->rr) > sqrt(ref_rr)) {
                restart = true;
                break;
            }
            ref_it = c->hst->iters;
            ref_rr = c->hst->rr;
        }
    }
    *fallbacks += c->hst->nonfinite;
    *its = c->hst->iters;
    if (!restart) return PA_OK;
    ++*fallbacks;
    const int used = c->hst->iters;
    KArgs<double> a = base_args<double>(c, 0, nr);
    a.u = c->u;
    a.out = q;
    a.affine = 0;
    a.dt = dtc;
    {
        KScope t(c, PA_K_INIT);
        stencil<double>(c, kMatvec, false, a);
        launch_pcg_resid<double>(N, 1, c->nn_b, q, c->Dbuf, r, p, c->part, &nparts, S);
    }
    {
        KScope t(c, PA_K_REDUCE);
        const int left = c->opt.max_iter - used;
        const int fleft = c->opt.force_iters > 0 ? std::max(1, c->opt.force_iters - used) : 0;
        launch_pcg_start(c->part, nparts, c->st, tol, std::max(1, left), fleft, 0, 0.0, S);
    }
    s = pcg_loop<double>(c, dtc, r, p, q);
    if (s) return s;
    *its = used + c->hst->iters;
    return PA_OK;
}

}  // namespace

extern "C" {

pa_status pa_advance_be_pcg(pa_ctx* c, double dt, double tol, int32_t cycles, pa_stats* user)
{
    Range range("pa_advance_be_pcg");
    if (!c) return PA_ERR_ARG;
    pa_status s = check_ready(c, dt);
    if (s) return s;
    if (cycles < 0) return fail(c, PA_ERR_ARG, "cycles must be >= 0");
    if (!(tol >= 0.0) || !isfinite(tol)) return fail(c, PA_ERR_ARG, "tol must be finite and >= 0");
    const bool learned = c->opt.pc == PA_PC_LEARNED;
    const bool bilu0 = c->opt.pc == PA_PC_BILU0;
    if (learned) {
        if (!c->nn_ready || c->d.ncomp != 1 || c->fp32)
            return fail(c, PA_ERR_STATE, "learned preconditioner not available on this context");
        if (!nn_alloc_grid(c) || !nn_fwd_work(c, c->N))
            return fail(c, PA_ERR_ALLOC, "learned preconditioner: out of device memory");
    }
    pa_stats local;
    pa_stats* st = user ? user : &local;
    init_stats(st);
    st->dt_explicit = c->dtE;
    Timer tm(c->stream);
    c->tstats = st;
    launch_fill_zero(c->flag, sizeof(int), c->stream);
    double* y0 = c->w[0];
    double* r = c->w[1];
    double* p = c->w[2];
    double* q = c->w[3];
    const Geo<double> g = geo(c, c->m64);
    const int nc = c->d.ncomp, nr = c->d.nr;
    const bool any_dir = c->d.bc_in == PA_BC_DIRICHLET || c->d.bc_out == PA_BC_DIRICHLET;
    // inner solves of the FP32-matvec variant stop at this fraction of the
    // true residual they start from
    const double eta = 1e-5;
    double t_rem = dt;
    int ncyc = 0;
    while (true) {
        Range cyc("pa be cycle");
        first_pass<double>(c, c->u, y0);
        double dtc;
        int last;
        s = next_cycle(c, dt, cycles, ncyc, t_rem, st, &dtc, &last);
        if (s) break;
        int nparts = 0, its = 0;
        if (learned) {
            {
                KScope t(c, PA_K_INIT);
                if (any_dir) boundary_data(c, q);
                launch_pcg_init<double>(g, nc, dtc, c->use_w ? c->w64 : nullptr, c->u, y0,
                                        any_dir ? q : nullptr, c->diagL,
                                        c->Dbuf, r, p, c->nn_b, c->part, &nparts, c->stream);
            }
            {
                KScope t(c, PA_K_REDUCE);
                launch_pcg_start(c->part, nparts, c->st, tol, c->opt.max_iter,
                                 c->opt.force_iters, 0, 0.0, c->stream);
            }
            int fb = 0;
            s = fcg_solve(c, dtc, tol, r, p, q, &its, &fb);
            if (s) break;
            st->fallbacks += fb;
        } else if (!c->fp32) {
            c->jd_on = !bilu0 && jd_ready(c);
            if (c->jd_on) st->jacobi_rows = 1;
            {
                KScope t(c, PA_K_INIT);
                if (any_dir) boundary_data(c, q);
                if (c->jd_on)
                    launch_jacobi_rows(g, c->cscale, c->d.bc_in, c->d.bc_out, dtc, c->jd_ab,
                                       c->jd_G, c->stream);
                launch_pcg_init<double>(g, nc, dtc, c->use_w ? c->w64 : nullptr, c->u, y0,
                                        any_dir ? q : nullptr, c->diagL,
                                        c->Dbuf, r, p, nullptr, c->part, &nparts, c->stream,
                                        jd_of(c));
            }
            {
                KScope t(c, PA_K_REDUCE);
                launch_pcg_start(c->part, nparts, c->st, tol, c->opt.max_iter,
                                 c->opt.force_iters, 0, 0.0, c->stream);
            }
            if (bilu0) {
                s = bilu0_factor(c, dtc);
                if (s) break;
                bilu0_start<double>(c, dtc, r, p);
            }
            c->xg_on = !bilu0 && xg_ready<double>(c);
            c->xg_q = 0;
            c->xg_p0 = p;
            s = pcg_loop<double>(c, dtc, r, p, q);
            c->xg_on = false;
            c->jd_on = false;
            if (s) break;
            its = c->hst->iters;
        } else {
            // defect correction: FP32-matvec PCG on M d = b - M x, x += d,
            // repeated until the FP64 true residual meets tol
            double* bvec = p;  // b lives in the FP64 direction buffer
            float* p32 = c->f[0];
            float* q32 = c->f[1];
            c->jd_on = !bilu0 && jd_ready(c);
            if (c->jd_on) st->jacobi_rows = 1;
            {
                KScope t(c, PA_K_INIT);
                if (any_dir) boundary_data(c, q);
                if (c->jd_on)
                    launch_jacobi_rows(g, c->cscale, c->d.bc_in, c->d.bc_out, dtc, c->jd_ab,
                                       c->jd_G, c->stream);
                launch_pcg_init<float>(g, nc, dtc, c->use_w ? c->w64 : nullptr, c->u, y0,
                                       any_dir ? q : nullptr, c->diagL,
                                       c->Dbuf, r, p32, bvec, c->part, &nparts, c->stream,
                                       jd_of(c));
            }
            if (bilu0) {
                s = bilu0_factor(c, dtc);
                if (s) break;
            }
            int outer = 0;
            while (true) {
                {
                    KScope t(c, PA_K_REDUCE);
                    launch_pcg_start(c->part, nparts, c->st, tol, c->opt.max_iter - its,
                                     c->opt.force_iters, 1, eta, c->stream);
                }
                if (bilu0) bilu0_start<float>(c, dtc, r, p32);
                s = sync_state(c);
                if (s || c->hst->done) break;
                c->xg_on = !bilu0 && xg_ready<float>(c);
                c->xg_q = 0;
                c->xg_p0 = p32;
                s = pcg_loop<float>(c, dtc, r, p32, q32);
                c->xg_on = false;
                if (s) break;
                its += c->hst->iters;
                ++outer;
                if (c->hst->status != 0 || c->opt.force_iters > 0) break;
                if (its >= c->opt.max_iter) { c->hst->status = 4; break; }
                // FP64 true residual r = b - M x and a fresh start
                KArgs<double> a = base_args<double>(c, 0, nr);
                a.u = c->u;
                a.out = q;
                a.affine = 0;
                a.dt = dtc;
                {
                    KScope t(c, PA_K_INIT);
                    stencil<double>(c, kMatvec, false, a);
                    launch_pcg_resid<float>(c->N, nc, bvec, q, c->Dbuf, r, p32, c->part, &nparts,
                                            c->stream);
                }
            }
            c->jd_on = false;
            if (s) break;
        }
        if (ncyc < PA_MAX_LOG) { st->dt_cycle[ncyc] = dtc; st->per_cycle[ncyc] = its; }
        st->iters_total += its;
        if (its > st->iters_max) st->iters_max = its;
        st->rel_residual = c->hst->bb > 0.0 ? sqrt(c->hst->rr / c->hst->bb) : sqrt(c->hst->rr);
        ++ncyc;
        const int pst = c->hst->status;
        if (pst == 4) { s = fail(c, PA_ERR_NOCONV, "PCG did not reach tol in %d iterations", its); break; }
        if (pst == 5) { s = fail(c, PA_ERR_BREAKDOWN, "PCG breakdown (<p,Mp> <= 0)"); break; }
        if (pst == 6) { s = fail(c, PA_ERR_NONFINITE, "non-finite residual"); break; }
        if (last) break;
        t_rem -= dtc;
    }
    st->cycles = ncyc;
    if (hipGetLastError() != hipSuccess && !s) s = fail(c, PA_ERR_HIP, "kernel launch failed");
    st->ms_total = tm.stop();
    (void)sync_state(c);
    c->tstats = nullptr;
    st->status = s;
    if (!s) c->err.clear();
    return s;
}

}  // extern "C"

extern "C" {

pa_status pa_bilu0_apply(pa_ctx* c, double dt, const double* r, double* z)
{
    if (!c) return PA_ERR_ARG;
    if (!r || !z) return fail(c, PA_ERR_ARG, "null vector");
    if (c->d.op != PA_OP_ISO7) return fail(c, PA_ERR_ARG, "block ILU(0): 7-point operator only");
    if (!(dt > 0.0) || !isfinite(dt)) return fail(c, PA_ERR_ARG, "dt must be finite and > 0");
    if (!c->have_coef) return fail(c, PA_ERR_STATE, "coefficients not set");
    const Geo<double> g = geo(c, c->m64);
    launch_jacobi_D(g, dt, c->use_w ? c->w64 : nullptr, c->diagL, c->Dbuf, c->stream);
    pa_status s = bilu0_factor(c, dt);
    if (s) return s;
    const KArgs<double> a = base_args<double>(c, 0, c->d.nr);
    int nb = 0;
    launch_bilu0_solve<double>(g, c->d.ncomp, a.coef, a.cs, dt, c->bilu0_ip, r, z, c->part, &nb,
                               c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->err.clear();
    return PA_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- learned PC ABI

namespace {

// splitmix64 (Steele, Lea & Flood, OOPSLA 2014): the training batch order
struct SplitMix {
    uint64_t x;
    uint64_t next()
    {
        uint64_t z = (x += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    int below(int n) { return n <= 1 ? 0 : (int)(next() % (uint64_t)n); }
};

pa_status lpc_ready(pa_ctx* c, double dt, bool weights)
{
    if (!c->have_coef) return fail(c, PA_ERR_STATE, "coefficients not set");
    if (c->d.ncomp != 1 || c->fp32)
        return fail(c, PA_ERR_ARG, "learned preconditioner: single-component FP64 contexts only");
    if (weights && !c->nn_ready) return fail(c, PA_ERR_STATE, "learned preconditioner: no weights set");
    if (!(dt > 0.0) || !isfinite(dt)) return fail(c, PA_ERR_ARG, "dt must be finite and > 0");
    if (!nn_alloc_base(c) || !nn_alloc_grid(c))
        return fail(c, PA_ERR_ALLOC, "learned preconditioner: out of device memory");
    return PA_OK;
}

// temporary device buffers released on scope exit
struct Temps {
    pa_ctx* c;
    std::vector<void*> v;
    explicit Temps(pa_ctx* c_) : c(c_) {}
    template <class T>
    T* get(size_t n)
    {
        T* p = (T*)dev_alloc(c, sizeof(T) * (n ? n : 1));
        if (p) v.push_back(p);
        return p;
    }
    ~Temps()
    {
        for (void* p : v) dev_free(c, p);
    }
};

}  // namespace

extern "C" {

void pa_lpc_default_train_opts(pa_lpc_train_opts* o)
{
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->nsnap = 16;
    o->batch = 2;
    o->epochs = 30;
    o->seed = 4300;
    o->lr = 1e-3;
    o->tol_star = 1e-12;
}

pa_status pa_lpc_set_weights(pa_ctx* c, const float* theta)
{
    if (!c) return PA_ERR_ARG;
    if (!theta) return fail(c, PA_ERR_ARG, "null weights");
    for (int i = 0; i < NN_NPARAM; ++i)
        if (!isfinite(theta[i])) return fail(c, PA_ERR_NONFINITE, "weight %d is not finite", i);
    if (!nn_alloc_base(c)) return fail(c, PA_ERR_ALLOC, "learned preconditioner: out of device memory");
    HIPCHK(c, hipMemcpyAsync(c->nn_th, theta, sizeof(float) * NN_NPARAM, hipMemcpyHostToDevice,
                             c->stream));
    launch_fill_zero(c->nn_m, sizeof(float) * NN_NPARAM, c->stream);
    launch_fill_zero(c->nn_v, sizeof(float) * NN_NPARAM, c->stream);
    launch_nn_prep_weights(c->nn_th, c->nn_w, c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->nn_adam_t = 0;
    c->nn_ready = true;
    c->err.clear();
    return PA_OK;
}

pa_status pa_lpc_get_weights(pa_ctx* c, float* theta)
{
    if (!c) return PA_ERR_ARG;
    if (!theta) return fail(c, PA_ERR_ARG, "null output");
    if (!c->nn_ready) return fail(c, PA_ERR_STATE, "learned preconditioner: no weights set");
    HIPCHK(c, hipMemcpyAsync(theta, c->nn_th, sizeof(float) * NN_NPARAM, hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PA_OK;
}

pa_status pa_lpc_features(pa_ctx* c, double dt, const double* r, float* feat)
{
    if (!c) return PA_ERR_ARG;
    if (!r || !feat) return fail(c, PA_ERR_ARG, "null array");
    pa_status s = lpc_ready(c, dt, false);
    if (s) return s;
    nn_static(c, dt, true);
    launch_nn_sigma(c->N, r, c->Dbuf, nullptr, c->part, c->nn_scal, c->stream);
    launch_nn_c0(c->N, r, c->Dbuf, c->nn_scal, nullptr, c->nn_xs, c->stream);
    launch_nn_unpack(c->N, c->nn_xs, feat, c->stream);
    HIPCHK(c, hipGetLastError());
    return PA_OK;
}

pa_status pa_lpc_apply(pa_ctx* c, double dt, const double* r, double* z)
{
    if (!c) return PA_ERR_ARG;
    if (!r || !z) return fail(c, PA_ERR_ARG, "null array");
    pa_status s = lpc_ready(c, dt, true);
    if (s) return s;
    if (!nn_fwd_work(c, c->N)) return fail(c, PA_ERR_ALLOC, "learned preconditioner: out of device memory");
    nn_static(c, dt, true);
    nn_precond(c, r, nullptr);
    launch_nn_apply(c->N, r, c->Dbuf, c->nn_out, c->nn_scal, z, c->stream);
    HIPCHK(c, hipGetLastError());
    return PA_OK;
}

pa_status pa_lpc_loss_grad(pa_ctx* c, double dt, int32_t npairs, const double* r, const double* e,
                           double* loss, float* grad)
{
    if (!c) return PA_ERR_ARG;
    if (!r || !e || !loss || !grad) return fail(c, PA_ERR_ARG, "null array");
    if (npairs < 1 || npairs > kMaxPairs) return fail(c, PA_ERR_ARG, "npairs must be in [1, %d]", kMaxPairs);
    pa_status s = lpc_ready(c, dt, true);
    if (s) return s;
    const size_t N = c->N, tot = N * (size_t)npairs;
    hipStream_t S = c->stream;
    Temps tmp(c);
    __bf16* xb = tmp.get<__bf16>(8 * tot);
    double* zj = tmp.get<double>(tot);
    double* d = tmp.get<double>(N);
    double* Md = tmp.get<double>(N);
    double* sd = tmp.get<double>(2 * (size_t)npairs + 1);
    if (!xb || !zj || !d || !Md || !sd || !nn_fwd_work(c, tot) || !nn_bwd_work(c, tot))
        return fail(c, PA_ERR_ALLOC, "learned preconditioner: out of device memory");
    double* lossacc = sd + 2 * npairs;
    std::vector<const double*> ep(npairs), sp(npairs), dp(npairs);
    nn_static(c, dt, true);
    for (int b = 0; b < npairs; ++b) {
        const double* rb = r + (size_t)b * N;
        ep[b] = e + (size_t)b * N;
        sp[b] = sd + b;
        dp[b] = sd + npairs + b;
        launch_nn_sigma(N, rb, c->Dbuf, nullptr, c->part, sd + b, S);
        launch_pair_build(N, c->nn_xs, rb, c->Dbuf, sd + b, xb + 8 * (size_t)b * N, zj + (size_t)b * N, S);
        const int mt = nn_matvec(c, dt, ep[b], Md);
        launch_scal_reduce(c->part, mt, nullptr, 0.0, sd + npairs + b, S);
    }
    launch_fill_zero(lossacc, sizeof(double), S);
    launch_fill_zero(c->nn_grad, sizeof(float) * NN_NPARAM, S);
    nn_energy_step(c, dt, npairs, xb, zj, ep.data(), sp.data(), dp.data(), d, Md, lossacc);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(grad, c->nn_grad, sizeof(float) * NN_NPARAM, hipMemcpyDeviceToHost, S));
    HIPCHK(c, hipMemcpyAsync(loss, lossacc, sizeof(double), hipMemcpyDeviceToHost, S));
    HIPCHK(c, hipStreamSynchronize(S));
    c->err.clear();
    return PA_OK;
}

pa_status pa_lpc_train(pa_ctx* c, double dt, const pa_lpc_train_opts* oin, pa_lpc_report* rep)
{
    Range range("pa_lpc_train");
    if (!c) return PA_ERR_ARG;
    pa_lpc_train_opts o;
    if (oin) o = *oin;
    else pa_lpc_default_train_opts(&o);
    if (!c->u) return fail(c, PA_ERR_STATE, "no field bound");
    pa_status s = lpc_ready(c, dt, true);
    if (s) return s;
    if (o.nsnap < 1 || o.batch < 1 || o.epochs < 1 || !(o.lr > 0.0) || !isfinite(o.lr) ||
        !(o.tol_star >= 0.0) || !isfinite(o.tol_star))
        return fail(c, PA_ERR_ARG, "invalid training option");
    const int nr = c->d.nr;
    const size_t N = c->N;
    hipStream_t S = c->stream;
    pa_lpc_report R;
    memset(&R, 0, sizeof R);
    std::vector<float> th0(NN_NPARAM);
    HIPCHK(c, hipMemcpy(th0.data(), c->nn_th, sizeof(float) * NN_NPARAM, hipMemcpyDeviceToHost));

    Temps tmp(c);
    double* bak = tmp.get<double>(N);
    double* xst = tmp.get<double>(N);
    double* snap = tmp.get<double>(N * (size_t)o.nsnap);   // iterates, then errors
    double* res = tmp.get<double>(N * (size_t)o.nsnap);    // residuals
    double* sd = tmp.get<double>(2 * (size_t)o.nsnap);     // sigma, |e|_M^2 per pair
    if (!bak || !xst || !snap || !res || !sd)
        return fail(c, PA_ERR_ALLOC, "training: out of device memory");
    double* y0 = c->w[0];
    double* r = c->w[1];
    double* p = c->w[2];
    double* q = c->w[3];
    const Geo<double> g = geo(c, c->m64);
    const bool any_dir = c->d.bc_in == PA_BC_DIRICHLET || c->d.bc_out == PA_BC_DIRICHLET;

    // reference solve x* by Jacobi PCG from x0 = u, keeping iterates x_k at
    // k = 0, 1, 2, 3, 4, 6, 9, 13, 19, ... (k <- max(k + 1, 3k/2))
    Timer t_pairs(S);
    launch_copy(c->u, bak, sizeof(double) * N, S);
    launch_fill_zero(c->flag, sizeof(int), S);
    first_pass<double>(c, c->u, y0);
    int nparts = 0;
    if (any_dir) boundary_data(c, q);
    launch_pcg_init<double>(g, 1, dt, c->use_w ? c->w64 : nullptr, c->u, y0, any_dir ? q : nullptr,
                            c->diagL, c->Dbuf, r, p,
                            c->nn_b, c->part, &nparts, S);
    launch_pcg_start(c->part, nparts, c->st, o.tol_star, c->opt.max_iter, 0, 0, 0.0, S);
    s = sync_state(c);
    int taken = 0;
    for (int j = 0, k = 0; !s && j < o.nsnap; ++j) {
        if (c->hst->done) break;
        const int todo = k - c->hst->iters;
        if (todo > 0) {
            pcg_queue<double>(c, dt, r, p, q, todo);
            s = sync_state(c);
            if (s || c->hst->done) break;
        }
        launch_copy(c->u, snap + (size_t)taken * N, sizeof(double) * N, S);
        ++taken;
        k = std::max(k + 1, k * 3 / 2);
    }
    if (!s) s = pcg_loop<double>(c, dt, r, p, q);
    const int pst = c->hst->status;
    R.ref_iters = c->hst->iters;
    launch_copy(c->u, xst, sizeof(double) * N, S);
    launch_copy(bak, c->u, sizeof(double) * N, S);
    if (s) return s;
    if (pst == 4) return fail(c, PA_ERR_NOCONV, "training: reference solve did not reach tol_star");
    if (pst == 5) return fail(c, PA_ERR_BREAKDOWN, "training: reference solve broke down");
    if (pst == 6) return fail(c, PA_ERR_NONFINITE, "training: non-finite residual");
    if (taken == 0) return fail(c, PA_ERR_ARG, "training: the bound field already solves the system");

    // pairs: r_k = b - M x_k, e_k = x* - x_k, sigma_k, |e_k|_M^2
    std::vector<const double*> ep(taken), sp(taken), dp(taken);
    for (int k = 0; k < taken; ++k) {
        double* xk = snap + (size_t)k * N;
        double* rk = res + (size_t)k * N;
        nn_matvec(c, dt, xk, q);
        launch_pcg_resid<double>(N, 1, c->nn_b, q, c->Dbuf, rk, p, c->part, &nparts, S);
        launch_sub(N, xst, xk, xk, S);
        launch_nn_sigma(N, rk, c->Dbuf, nullptr, c->part, sd + k, S);
        const int mt = nn_matvec(c, dt, xk, q);
        launch_scal_reduce(c->part, mt, nullptr, 0.0, sd + taken + k, S);
        ep[k] = xk;
        sp[k] = sd + k;
        dp[k] = sd + taken + k;
    }
    nn_static(c, dt, false);
    HIPCHK(c, hipGetLastError());
    R.ms_pairs = t_pairs.stop();
    R.pairs = R.snapshots = taken;

    // Adam over batches of pairs, order shuffled every epoch
    const int B = std::min(o.batch, taken);
    const int nbatch = taken / B;
    const int steps = nbatch * o.epochs;
    __bf16* xb = tmp.get<__bf16>(8 * N * (size_t)B);
    double* zjb = tmp.get<double>(N * (size_t)B);
    double* lossv = tmp.get<double>(steps);
    if (!xb || !zjb || !lossv || !nn_fwd_work(c, N * B) || !nn_bwd_work(c, N * B))
        return fail(c, PA_ERR_ALLOC, "training: out of device memory");
    launch_fill_zero(lossv, sizeof(double) * steps, S);
    Timer t_train(S);
    SplitMix rng{(uint64_t)(uint32_t)o.seed};
    std::vector<int> perm(taken);
    for (int i = 0; i < taken; ++i) perm[i] = i;
    std::vector<const double*> be(B), bs(B), bd(B);
    int step = 0;
    for (int ep_i = 0; ep_i < o.epochs; ++ep_i) {
        for (int i = taken - 1; i > 0; --i) std::swap(perm[i], perm[rng.below(i + 1)]);
        for (int bi = 0; bi < nbatch; ++bi) {
            for (int b = 0; b < B; ++b) {
                const int k = perm[bi * B + b];
                launch_pair_build(N, c->nn_xs, res + (size_t)k * N, c->Dbuf, sp[k],
                                  xb + 8 * (size_t)b * N, zjb + (size_t)b * N, S);
                be[b] = ep[k];
                bs[b] = sp[k];
                bd[b] = dp[k];
            }
            launch_fill_zero(c->nn_grad, sizeof(float) * NN_NPARAM, S);
            nn_energy_step(c, dt, B, xb, zjb, be.data(), bs.data(), bd.data(), p, q, lossv + step);
            launch_nn_adam(c->nn_th, c->nn_grad, c->nn_m, c->nn_v, (float)o.lr, ++c->nn_adam_t, S);
            launch_nn_prep_weights(c->nn_th, c->nn_w, S);
            ++step;
        }
        HIPCHK(c, hipGetLastError());
    }
    std::vector<double> lh(steps);
    HIPCHK(c, hipMemcpyAsync(lh.data(), lossv, sizeof(double) * steps, hipMemcpyDeviceToHost, S));
    R.ms_train = t_train.stop();
    R.steps = steps;
    for (int i = 0; i < nbatch; ++i) {
        R.loss_first += lh[i] / nbatch;
        R.loss_last += lh[steps - nbatch + i] / nbatch;
    }
    std::vector<float> th(NN_NPARAM);
    HIPCHK(c, hipMemcpy(th.data(), c->nn_th, sizeof(float) * NN_NPARAM, hipMemcpyDeviceToHost));
    bool finite = true;
    for (float v : th) finite = finite && isfinite(v);
    if (rep) *rep = R;
    if (!finite) {
        (void)pa_lpc_set_weights(c, th0.data());
        return fail(c, PA_ERR_NONFINITE, "training diverged; previous weights restored");
    }
    c->err.clear();
    return PA_OK;
}

}  // extern "C"
