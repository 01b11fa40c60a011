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
// Volume-sweep table: supports scaled by 1/(2R), centred at the first support, and their squared norms.
struct VolTable {
    double *qx, *qy, *qz, *qq;
};
inline VolTable vtable(const Support& s) { return VolTable{s.qx, s.qy, s.qz, s.qq}; }
inline SupportMut mut(Support& s) { return SupportMut{s.sx, s.sy, s.sz, s.wx, s.wy, s.wz, s.orig, s.M}; }

void launch_stage(hipStream_t s, int64_t nb, const double* xyz, const double* disp, const int32_t* perm,
                  double inv_r, Boundary& bd);
void launch_check_finite(hipStream_t s, int64_t count, const double* a, const double* b, int32_t* flag);
void launch_init_nodes(hipStream_t s, const Boundary& bd, int32_t* init, ArgRec* rec);
// Arguments of the three iteration kernels (by value for one surface, from a
// table for a batch of surfaces).
struct SweepArgs {
    const GState* st;
    int t0, T, lpt, tpl;
    const double *px, *py, *pz, *pdx, *pdy, *pdz;
    const uint8_t* inS;
    const int32_t* perm;
    SupportView sv;
    int64_t nub;      // upper bound of |S| at this iteration (<= capacity): extent of the first staged window
    ArgRec* rec;
    int ptop;         // block variant: records per block (its best candidates, in rank order); 0 otherwise
};

// The block variant's two append kernels (the first also ranks the sweep's records and decides).
struct FactorBlkArgs {
    GState* st;
    BlockRec* brec;
    SupportMut sm;
    double* Mc;
    int64_t cap;
    double* lam;       // Lambda = M B, column-major: entry (i, t) at t * cap + i
    double* Pb;
    uint8_t* inS;
    const ArgRec* srec;
    int nrec;
    int ptop;          // nodes the rule may append (per_iter)
    int32_t m;
    int g;
    double tol_abs;
    int64_t nc_max;
    int32_t* log_group;
    int32_t* log_node;
    double* log_err;
    int8_t* log_app;
    int64_t log_cap;
};

struct FactorLArgs {
    GState* st;
    IterRec* irec;
    const ArgRec* srec;
    int nrec;
    int32_t m;
    int g;
    int init_t;
    const int32_t* init;
    const int32_t* pos_of;
    const double *px, *py, *pz, *pdx, *pdy, *pdz;
    SupportView sv;
    const double* Mr;
    double* l;
    double* Pb;
    double tol_abs;
    int64_t nc_max, cap;
    int32_t* log_group;
    int32_t* log_node;
    double* log_err;
    int8_t* log_app;
    int64_t log_cap;
    int32_t active;
};

struct FactorUArgs {
    GState* st;
    const IterRec* irec;
    uint8_t* inS;
    SupportMut sm;
    double* Mc;
    int64_t cap;
    const double* l;
    const double* Pb;
    int32_t active;
};

constexpr int kMaxBatch = 64;
// Blocks of a batched launch: surface s owns blocks [off[s], off[s+1]).
struct BlockMap {
    int count;
    int off[kMaxBatch + 1];
};

// One surface of a batched volume sweep.
struct VolDesc {
    const void* xyz;
    void* out;
    int64_t nv;
    SupportView sv;
    VolTable vt;   // filled by the batched launch itself
    int n;
    double inv_r;
};

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
    double* lam;           // block variant
    BlockRec* brec;
};

int sweep_blocks(int gmax);
// Block records a sweep with these arguments writes (0 for an empty group).
int sweep_records(const SweepArgs& A);
int factor_blocks(int64_t n_ub, int rpw = 1);
void sweep_layout_batch(int T, int& lpt, int& tpl);
SweepArgs make_sweep_args(const IterCtx& ic, int g);
FactorLArgs make_factor_l_args(const IterCtx& ic, int g, int nrec, int init_t);
FactorUArgs make_factor_u_args(const IterCtx& ic);
// table_map: blocks of kBlock supports per surface for the volume tables; map: blocks of kBlock targets.
void launch_volume_batch(hipStream_t s, const VolDesc* tab, const BlockMap& map, const BlockMap& table_map,
                         int in_f64, int out_f64);
// One greedy iteration of every context of a batch: three launches.  rpw
// (1 or kMaxRowsPerWave) is the rows of M per factor wave; it must match the
// block maps, and does not change any result.
void launch_iteration_batch(hipStream_t s, const SweepArgs* sweep_tab, const FactorLArgs* fl_tab,
                            const FactorUArgs* fu_tab, const BlockMap& sweep_map, const BlockMap& factor_map, int rpw);
void launch_init_append(hipStream_t s, const IterCtx& ic, int t);
// One greedy iteration (group sweep, k_factor_l, k_factor_u).  With marks (four events), events are recorded
// before the sweep, before each factor kernel and after the last.  Returns 1 if the sweep was launched.
int launch_iteration(hipStream_t s, const IterCtx& ic, int g, int n_ub, const hipEvent_t* marks = nullptr);
// One iteration of the several-nodes-per-iteration variant (up to p nodes appended): top-p group sweep, then
// the two block-append kernels (the first also ranks and decides).
void launch_iteration_block(hipStream_t s, const IterCtx& ic, int g, int n_ub, int p);
int multi_padded_r(int rc);
// Weights of the kept support set for the displacements disp (nb, 3):
// W = M^T (M Delta_S) into sp.wx/wy/wz.  Dbuf and Ybuf hold 3 n doubles each.
bool launch_support_weights(hipStream_t s, Support& sp, int n, const double* disp, double* Dbuf, double* Ybuf);
void launch_mark_support(hipStream_t s, const Boundary& bd, const Support& sp, int n);

// Dense FP64 refactorisation (matrix cores): A, Md, Tb hold dense_padded(n)^2
// doubles each; on return the lower triangle of Md holds L^-1 and that of Tb
// holds L (their 64 x 64 blocks above the diagonal are not written), A is
// scratch, and *bad = 1 (set, never cleared) if a pivot was not above
// kSingularTol.
int dense_padded(int n);
int dense_pack_blocks();
// The launch sequence of the refactorisation for one padded size (host steps, device work-item table, tile
// counters and partial buffers); rebuilt when the padded size of n changes.
struct DensePlan;
hipError_t dense_plan_for(DensePlan*& plan, int n, hipStream_t s);
void free_dense_plan(DensePlan* plan);
size_t dense_plan_bytes(const DensePlan* plan);
// The whole sequence is captured once per buffer set into a graph and replayed on s.
hipError_t launch_inverse_factor(hipStream_t s, const Support& sp, int n, double* A, double* Md, double* Tb,
                                 int32_t* bad, DensePlan* plan);
// Packed rows of Md into Mp (may equal old); with old, red[2b], red[2b+1]
// get per-block max |new - old| and max |old| (dense_pack_blocks() blocks).
void launch_pack_factor(hipStream_t s, int n, const double* Md, double* Mp, const double* old, double* red);
void launch_gather_support(hipStream_t s, Support& sp, int n, const double* xyz0, double inv_r);
bool launch_deform_multi(hipStream_t s, const Support& sp, int n, int rc, const double* modes_dev, double* Dbuf,
                         double* Ybuf, double* Wbuf, int64_t nv, const void* xyz, int in_f64, double inv_r, void* out,
                         int out_f64);
void launch_transpose_factor(hipStream_t s, const double* Mr, double* Mc, int n, int64_t cap);
// Monitor sample: out[0] = max e^2, out[1] = sum e^2 over all nodes with the current W,
// written only if st->log_len >= need when the kernels run (red: 2 * certify_blocks(nb) doubles).
void launch_monitor(hipStream_t s, const Boundary& bd, const Support& sp, const GState* st, int64_t need,
                    double* red, double* out);
void launch_certify(hipStream_t s, const Boundary& bd, const Support& sp, int n, double* red, double* out);
// Convergence probe: per group, the largest squared error over the nodes not in S with the current W (ties to
// the lowest original index) and their count; perr holds one double per boundary node.
struct GroupMax {
    double e2;       // -1: no node outside S
    int32_t orig;
    int32_t count;
    double all_max;  // largest squared error over all the group's nodes (S included)
    double all_sum;  // their sum, in thread order then waves in order
};
void launch_probe(hipStream_t s, const Boundary& bd, const Support& sp, int n, double* perr, GroupMax* out);
// Blocks of the all-node sweeps (certificate, monitor): red needs 2 doubles per block.
int64_t certify_blocks(int64_t nb);
// FP32 evaluation of Eq. (6) (FP32 copies of the supports and weights are
// refreshed first; sp.fsx..fwz must hold sp.cap floats).
void launch_volume32(hipStream_t s, int64_t nv, const void* xyz, int in_f64, double inv_r, const Support& sp, int n,
                     void* out, int out_f64);
// FP64 Eq. (6); the volume table is refreshed first (sp.qx..qq must hold sp.cap doubles).
void launch_volume(hipStream_t s, int64_t nv, const void* xyz, int in_f64, double inv_r, const Support& sp, int n,
                   void* out, int out_f64);
// Compact-support culling of Eq. (6): the frame of the points' Morton keys (in the volume table's units) and the
// supports sorted in Morton order with the bounding box of every tile of 32.
struct CullFrame {
    double lox, loy, loz, sc;
};
struct CullSupports {
    const double *qx, *qy, *qz, *qq, *wx, *wy, *wz;
    const double* box;   // 6 per tile: min x, y, z, max x, y, z
};
constexpr int kCullTileHost = 32;
void launch_cull_keys(hipStream_t s, int64_t nv, const void* xyz, int in_f64, double inv_r, const double c0[3],
                      const CullFrame& f, uint32_t* keys, int32_t* idx);
void launch_volume_cull(hipStream_t s, int64_t nv, const void* xyz, int in_f64, const int32_t* order, double inv_r,
                        const double c0[3], const CullSupports& cs, int n, void* out, int out_f64,
                        uint64_t* evaluated);
int cull_blocks(int64_t nv);
// The FP64 volume table of the first n supports (scaled by 1/(2R), centred at the first support).
void launch_volume_table(hipStream_t s, const Support& sp, int n);
hipError_t sort_pairs_u32(void* temp, size_t* temp_bytes, const uint32_t* keys_in, uint32_t* keys_out,
                          const int32_t* vals_in, int32_t* vals_out, int64_t n, int bits, hipStream_t s);

// Allocation-free Eq. (6): the refreshed support table (FP64) or support copies (FP32 evaluation) go
// into the module's static scratch array at scratch_ptr (n <= GCB_NOALLOC_MAX_SUPPORTS).
void launch_volume_noalloc(hipStream_t s, int64_t nv, const void* xyz, int in_f64, double inv_r, const Support& sp,
                           int n, void* out, int out_f64, int fp32_eval, void* scratch_ptr);
// Look up, once per device and with that device current, the device address of the static scratch
// array; noalloc_scratch returns it (nullptr before the set-up).
hipError_t noalloc_setup(int device);
void* noalloc_scratch(int device);

}  // namespace gcb
