/* oracle_api.h -- entry points of the CPU oracle (test infrastructure only;
 * see oracle.c).  Not used by the GPU library. */
#ifndef ORACLE_API_H
#define ORACLE_API_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAX_LOG 4096

typedef struct or_ctx or_ctx;

typedef struct {
    int32_t cycles, s_total, s_max, iters_total, iters_max, floored;
    int64_t k_first;
    double dt_explicit, dt_ptl_first, dt_ptl_min, rel_residual;
    double dt_cycle[OR_MAX_LOG];   /* length of each cycle */
    int32_t s_cycle[OR_MAX_LOG];   /* stages (STS) or PCG iterations (BE) per cycle */
} or_stats;

or_ctx* or_create(int nr, int nt, int np, int nc, const double* r_faces, const double* t_faces,
                  const double* p_faces, int op, int bc_in, int bc_out);
void or_destroy(or_ctx* o);
int or_set_profile(or_ctx* o, const double* w, const double* fc, double Tc);
int or_set_coefficients(or_ctx* o, const double* T0, double scale, double expo, const double* B);
double or_wvolume(const or_ctx* o, int i, int j, int k);
void or_volumes(const or_ctx* o, int weighted, double* out);
void or_set_bc(or_ctx* o, const double* ub_in, const double* ub_out);
double or_volume(const or_ctx* o, int i, int j, int k);
void or_apply(or_ctx* o, const double* u, double* F, int affine);
void or_diag(const or_ctx* o, double* out);
double or_dt_explicit(const or_ctx* o);
double or_ptl_from(int nc, int nr, int nt, int np, const double* u, const double* F, int64_t* kmax);
double or_ptl_fullgrid(int nc, int nr, int nt, int np, const double* u, const double* F);
double or_ptl(or_ctx* o, const double* u, int64_t* kmax);
int or_sts_coeffs(int kind, int s, double* mu, double* nu, double* mut, double* gam);
int or_sts_stages(int kind, double ratio, int force_odd);
int or_num_threads(void);
void or_set_num_threads(int n);
double or_stream_triad(long n, int reps);
int or_set_pc(or_ctx* o, int pc, int bi, int bj, int bk);
int or_bilu0_export(const or_ctx* o, double dt, int* rowp, int* col, double* m0, double* lu,
                    int cap);
int or_precondition(const or_ctx* o, double dt, const double* r, double* z);
int or_advance(or_ctx* o, double* u, double dt, int cycles, int scheme, int sts_kind,
               int force_odd, int s_override, double tol, int max_iter, int force_iters,
               int max_cycles, double ptl_floor, const double* replay_dt, int replay_n,
               or_stats* st);

#ifdef __cplusplus
}
#endif
#endif
