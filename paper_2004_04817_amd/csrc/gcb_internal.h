// Internal declarations of the MI355X GCB greedy RBF library (not installed).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/gcb.h"

namespace gcb {

constexpr int kBlock = 256;          // threads per workgroup of the sweep kernels (4 wave64)
constexpr int kLdsTile = 256;        // supports staged in LDS per pass
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kBigBlock = 1024;      // threads per workgroup of the factor kernels (16 wave64)
constexpr int kRowsL = kBigBlock / 64;   // rows (columns) of M per factor block and per wave round
constexpr int kMaxRowsPerWave = 4;       // rounds of kRowsL rows a factor block may hold
constexpr int kBWindow = 4096;       // phi-vector entries staged in LDS at a time
constexpr double kSingularTol = 64.0 * 2.220446049250313e-16;  // phi0 - l.l below this: not SPD
constexpr int kMaxPerIter = GCB_MAX_PER_ITER;   // nodes one iteration of the block variant may append
// block partials per 16-row chunk of the block append: b_t.W (3 per node) and lambda_t.lambda_u (a full square)
constexpr int kBlkPart = 3 * kMaxPerIter + kMaxPerIter * kMaxPerIter;

// Greedy state, resident in device memory.  Only the kernel that commits an
// iteration writes k and n, so every block of the other kernels sees the
// values the iteration started with.
struct GState {
    int64_t k;            // iteration counter (Algorithm 1 starts at k = 3)
    int32_t n;            // |S|
    int32_t quiet;        // consecutive iterations without an append
    int32_t done;         // 0 running, 1 converged, 2 cap reached, 3 singular, 4 factor capacity reached
    int32_t init_left;    // forced appends of the starting nodes still to do
    int64_t log_len;      // iterations written to the log
    uint64_t pairs_group;
    uint64_t pairs_append;
    int32_t singular_node;
    int32_t pad;
};

// What one iteration decided, written by the sweep kernel's last block and
// read by the append kernels.
struct IterRec {
    int64_t k;            // the iteration's k
    int32_t n;            // |S| before the append
    int32_t app;          // 1: append node_pos
    int32_t init;         // 1: a starting-node append (k does not advance)
    int32_t ran;          // 1: the iteration ran (advance k)
    int32_t node_pos;     // permuted position of the node to append
    int32_t node_orig;    // its original index
    int32_t singular;     // set by the factor kernel: phi0 - l.l <= tolerance
    int32_t pad;
    double E;             // group maximum error
    double x, y, z;       // the node's scaled coordinates
    double dx, dy, dz;    // its prescribed displacement
};

// What one iteration of the several-nodes-per-iteration variant decided: the q nodes to append, in rank
// order (written by the selection kernel, read by the two append kernels).
struct BlockRec {
    int32_t n;            // |S| before the append
    int32_t q;            // nodes to append (0: none)
    int32_t pad0, pad1;
    int32_t pos[kMaxPerIter], orig[kMaxPerIter];
    double x[kMaxPerIter], y[kMaxPerIter], z[kMaxPerIter];
    double dx[kMaxPerIter], dy[kMaxPerIter], dz[kMaxPerIter];
};

// Per-block argmax record.
struct ArgRec {
    double e2;            // squared error (-1: none)
    int32_t orig;         // original index
    int32_t pos;          // permuted position
    int32_t count;        // candidates (not in S) seen
    int32_t pad;
    double x, y, z;       // the candidate's scaled coordinates
    double dx, dy, dz;    // and its prescribed displacement
};

struct Boundary {
    int64_t nb = 0;
    int32_t m = 0;
    double radius = 0, inv_r = 0;
    // permuted, group-contiguous (within a group ascending original index), coordinates scaled by 1/R
    double *px = nullptr, *py = nullptr, *pz = nullptr;
    double *pdx = nullptr, *pdy = nullptr, *pdz = nullptr;
    float *fx = nullptr, *fy = nullptr, *fz = nullptr;   // FP32 copies (screening mode)
    int32_t *perm = nullptr;     // pos -> original index
    int32_t *pos_of = nullptr;   // original index -> pos
    int32_t *goff = nullptr;     // m+1 group offsets
    uint8_t *inS = nullptr;      // by pos
    // original order (unscaled) for the starting-node rule
    double *xyz0 = nullptr, *disp0 = nullptr;
    int32_t gmax = 0;            // largest group size
    int64_t alloc_nb = 0;        // size the permuted arrays were allocated for
    int32_t alloc_m = 0;         // groups goff was allocated for
    std::vector<int32_t> goff_h;
};

struct Support {
    int64_t cap = 0;             // capacity of the support arrays and of M
    double *sx = nullptr, *sy = nullptr, *sz = nullptr;   // scaled coordinates, selection order
    double *wx = nullptr, *wy = nullptr, *wz = nullptr;   // weights (FP64 master)
    float *fsx = nullptr, *fsy = nullptr, *fsz = nullptr, *fwx = nullptr, *fwy = nullptr, *fwz = nullptr;
    // volume-sweep table (allocated by the first FP64 deformation): coordinates scaled by 1/(2R) and
    // centred at the first support, and their squared norms
    double *qx = nullptr, *qy = nullptr, *qz = nullptr, *qq = nullptr;
    int32_t *orig = nullptr;     // original index of support s
    double *M = nullptr;         // packed lower-triangular inverse factor, row i at i(i+1)/2
    double *Mc = nullptr;        // the same factor by columns: column j (rows j..cap-1) at j*cap - j(j-1)/2
    double *l = nullptr;         // append scratch: l = M b (cap)
};

// Launch-shape choices (process-wide; read from GCB_SWEEP_LPT and GCB_GRAPH
// when the first context is created).
struct Tuning {
    int sweep_lpt_max = 256;   // 64, 128 or 256 lanes sharing one target in the group sweep
    bool use_graph = true;     // replay chunks of iterations as captured hipGraphs
    bool probe = true;         // convergence probe at chunk boundaries (GCB_PROBE=0 turns it off)
    int probe_div = 16;        // ... after max(8, m / probe_div) quiet iterations (GCB_PROBE_DIV)
};
extern Tuning g_tuning;

struct DensePlan;   // dense refactorisation launches (gcb_dense.hip)

}  // namespace gcb

struct gcb_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;
    std::string err;
    gcb_params params{};
    bool have_params = false;
    bool have_groups = false;
    std::vector<int32_t> groups_h;   // explicit partition
    gcb::Boundary bd;
    gcb::Support sp;
    gcb::GState *state = nullptr;    // device
    gcb::GState state_h{};
    gcb::IterRec *irec = nullptr;    // device, the current iteration's record
    double *Pb = nullptr;            // block partials of the factor kernels
    int64_t Pb_cap = 0;
    double *lam = nullptr;           // block variant: Lambda = M B, (cap, kMaxPerIter) by rows
    int64_t lam_cap = 0;
    gcb::BlockRec *brec = nullptr;   // block variant: the iteration's decision
    gcb::ArgRec *argrec = nullptr;   // device, per-block records of the sweeps
    int64_t argrec_cap = 0;
    // per-iteration log (device)
    int32_t *log_group = nullptr;
    int32_t *log_node = nullptr;
    double *log_err = nullptr;
    int8_t *log_app = nullptr;
    int64_t log_cap = 0;
    double *mon = nullptr;             // monitor samples (max e^2, sum e^2), log_cap pairs
    bool selected = false;
    gcb_select_info info{};
    // captured chunk of greedy iterations (replayed while its key is unchanged)
    hipStream_t cap_stream = nullptr;
    std::vector<std::pair<int64_t, hipGraphExec_t>> chunk_execs;   // one per phase k mod m of a chunk start
    std::vector<int64_t> chunk_key;
    // kernel timing (measurement aid): events between the launches of every iteration of a chunk
    bool ktime_on = false;
    std::vector<hipEvent_t> ktime_ev;
    double ktime_ms[4] = {0, 0, 0, 0};   // group sweep, k_factor_l, k_factor_u, certificate
    int64_t ktime_n[4] = {0, 0, 0, 0};
    bool ktime_valid = false;
    uint64_t alloc_gen = 0;            // bumped by every device allocation
    gcb::GState *state_pin = nullptr;   // pinned host copy of the state
    hipEvent_t ev0 = nullptr, ev1 = nullptr;   // selection start / end
    hipEvent_t ev2 = nullptr, ev3 = nullptr;   // kernels of the last deformation: start / end
    bool deform_timed = false;
    int64_t k_host = 3;                // the next iteration's k
    bool in_progress = false;          // a selection started by a batch and not yet finished
    // kept support set for a warm start (valid after a finished selection on this boundary)
    bool warm_ok = false;
    double warm_radius = 0.0;
    int32_t warm_m = 0;
    uint64_t warm_seed = 0;
    int64_t warm_n = 0;
    // compact-support culling of Eq. (6): Morton keys and point order, sorted supports and tile boxes
    uint32_t *ck_in = nullptr, *ck_out = nullptr;
    int32_t *ci_in = nullptr, *ci_out = nullptr;
    int64_t cull_cap = 0;
    double *cs = nullptr;              // 7 x cs_n sorted support entries, then 6 per tile
    int64_t cs_cap = 0;
    uint64_t *cull_ev = nullptr;       // evaluated pairs per block of the last culled sweep
    int64_t cull_ev_cap = 0;
    int64_t cull_nblk = 0;
    uint64_t cull_dense = 0;
    bool cull_valid = false;
    void *sort_tmp = nullptr;
    size_t sort_tmp_cap = 0;
    // convergence probe: per-node errors and per-group maxima
    double *perr = nullptr;
    int64_t perr_cap = 0;
    void *gmax = nullptr;
    int64_t gmax_cap = 0;
    int64_t probes = 0, probe_skipped = 0;   // of the last selection: probes run, iterations they completed
    int64_t probed_n = -1;                   // |S| at the last probe (one probe per run of quiet iterations)
    bool probe_cert = false;                 // the successful probe left the certificate (max, sum of e^2)
    double probe_cert_max = 0.0, probe_cert_sum = 0.0;
    // scratch for certificate / volume
    double *red = nullptr;
    int64_t red_cap = 0;
    void *tmp = nullptr;
    size_t tmp_cap = 0;
    gcb::DensePlan* dplan = nullptr;   // launches of the dense refactorisation for the last padded size
};

namespace gcb {
// Device bytes a context holds now (boundary, support set and factor, records, log, scratch).
size_t ctx_device_bytes(const gcb_ctx* ctx);
}  // namespace gcb
