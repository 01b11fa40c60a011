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
// Everything one greedy iteration's kernels touch.
struct IterCtx {
    GState* st;
    IterRec* irec;
    ArgRec* srec;          // per-block records of the group sweep
    const int32_t* init;   // the three starting nodes
    const Boundary* bd;
    Support* sp;
    double* Pb;
    double tol_abs;
    int64_t nc_max;
    int64_t log_cap;
    int32_t* log_group;
    int32_t* log_node;
    double* log_err;
    int8_t* log_app;
};

int sweep_blocks(int gmax);
void launch_init_append(hipStream_t s, const IterCtx& ic, int t);
void launch_iteration(hipStream_t s, const IterCtx& ic, int g, int n_ub);
int multi_padded_r(int rc);
bool launch_deform_multi(hipStream_t s, const Support& sp, int n, int rc, const double* modes_dev, double* Dbuf,
                         double* Ybuf, double* Wbuf, int64_t nv, const void* xyz, int in_f64, double inv_r, void* out,
                         int out_f64);
void launch_transpose_factor(hipStream_t s, const double* Mr, double* Mc, int n, int64_t cap);
void launch_certify(hipStream_t s, const Boundary& bd, const Support& sp, int n, double* red, double* out);
void launch_volume(hipStream_t s, int64_t nv, const void* xyz, int in_f64, double inv_r, const Support& sp, int n,
                   void* out, int out_f64);

}  // namespace gcb
