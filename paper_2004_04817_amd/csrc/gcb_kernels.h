// Launch wrappers of the HIP kernels (internal).
#pragma once
#include "gcb_internal.h"

namespace gcb {

struct SupportView {
    const double *sx, *sy, *sz, *wx, *wy, *wz;
};
struct SupportMut {
    double *sx, *sy, *sz, *wx, *wy, *wz;
    int32_t* orig;
    double* M;
};
inline SupportView view(const Support& s) { return SupportView{s.sx, s.sy, s.sz, s.wx, s.wy, s.wz}; }
inline SupportMut mut(Support& s) { return SupportMut{s.sx, s.sy, s.sz, s.wx, s.wy, s.wz, s.orig, s.M}; }

void launch_stage(hipStream_t s, int64_t nb, const double* xyz, const double* disp, const int32_t* perm,
                  double inv_r, Boundary& bd);
void launch_check_finite(hipStream_t s, int64_t count, const double* a, const double* b, int32_t* flag);
void launch_init_nodes(hipStream_t s, const Boundary& bd, int32_t* init, ArgRec* rec);
void launch_init_stage(hipStream_t s, GState* st, const int32_t* init, int t, const int32_t* pos_of);
void launch_append(hipStream_t s, GState* st, const Boundary& bd, Support& sp, int n_ub);
void launch_iteration(hipStream_t s, GState* st, const Boundary& bd, Support& sp, double* P, int32_t Tmax,
                      ArgRec* rec, double tol_abs, int64_t nc_max, int64_t log_cap, int32_t* lg, int32_t* ln,
                      double* le, int8_t* la, int n_ub);
void launch_certify(hipStream_t s, const Boundary& bd, const Support& sp, int n, double* red, double* out);
void launch_volume(hipStream_t s, int64_t nv, const void* xyz, int in_f64, double inv_r, const Support& sp, int n,
                   void* out, int out_f64);

}  // namespace gcb
