// Host runtime and C ABI of the MI355X GCB greedy RBF library.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <limits>
#include <new>

#include "gcb_internal.h"
#include "gcb_kernels.h"

using namespace gcb;

namespace {

thread_local std::string g_create_err;

struct Fail {
    int code;
};

#define HIPCHK(ctx, expr)                                                                         \
    do {                                                                                          \
        hipError_t _e = (expr);                                                                   \
        if (_e != hipSuccess) {                                                                   \
            (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(_e);                       \
            throw Fail{_e == hipErrorOutOfMemory ? GCB_E_NOMEM : GCB_E_DEVICE};                   \
        }                                                                                         \
    } while (0)

[[noreturn]] void fail(gcb_ctx* ctx, int code, const std::string& msg) {
    ctx->err = msg;
    throw Fail{code};
}

template <typename T>
void dalloc(gcb_ctx* ctx, T*& p, size_t count) {
    if (p) {
        (void)hipFree(p);
        p = nullptr;
    }
    if (count == 0) count = 1;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, count * sizeof(T));
    if (e != hipSuccess) {
        ctx->err = "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes: " + hipGetErrorString(e);
        throw Fail{GCB_E_NOMEM};
    }
    p = static_cast<T*>(q);
    ctx->alloc_gen++;   // captured graphs bake in buffer addresses
}

// Grow p to at least `need` elements; the recorded capacity changes only once the allocation succeeded.
template <typename T, typename C>
void dalloc_cap(gcb_ctx* ctx, T*& p, C& cap, C need) {
    if (cap >= need && p) return;
    cap = 0;
    dalloc(ctx, p, (size_t)need);
    cap = need;
}

template <typename T>
void dfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

// splitmix64 (Steele, Lea, Flood 2014; 64-bit finaliser of the xoshiro reference)
inline uint64_t splitmix64(uint64_t& state) {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void seeded_partition(int64_t nb, int32_t m, uint64_t seed, int32_t* group_of) {
    std::vector<int64_t> order(static_cast<size_t>(nb));
    for (int64_t i = 0; i < nb; ++i) order[i] = i;
    uint64_t st = seed;
    for (int64_t i = nb - 1; i > 0; --i) {
        const uint64_t j = splitmix64(st) % static_cast<uint64_t>(i + 1);
        std::swap(order[i], order[j]);
    }
    for (int64_t t = 0; t < nb; ++t) group_of[order[t]] = static_cast<int32_t>(t % m);
}

bool all_finite(const double* a, int64_t count) {
    for (int64_t i = 0; i < count; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

void sync(gcb_ctx* ctx) { HIPCHK(ctx, hipStreamSynchronize(ctx->stream)); }

void copy_in(gcb_ctx* ctx, void* dst, const void* src, size_t bytes, int mem) {
    HIPCHK(ctx, hipMemcpyAsync(dst, src, bytes, mem == GCB_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                               ctx->stream));
}

void copy_out(gcb_ctx* ctx, void* dst, const void* src, size_t bytes, int mem) {
    HIPCHK(ctx, hipMemcpyAsync(dst, src, bytes, mem == GCB_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                               ctx->stream));
}

void free_support(Support& sp) {
    dfree(sp.sx); dfree(sp.sy); dfree(sp.sz); dfree(sp.wx); dfree(sp.wy); dfree(sp.wz);
    dfree(sp.fsx); dfree(sp.fsy); dfree(sp.fsz); dfree(sp.fwx); dfree(sp.fwy); dfree(sp.fwz);
    dfree(sp.qx); dfree(sp.qy); dfree(sp.qz); dfree(sp.qq);
    dfree(sp.orig); dfree(sp.M); dfree(sp.Mc); dfree(sp.l);
    sp.cap = 0;
}

void free_boundary(Boundary& bd) {
    dfree(bd.px); dfree(bd.py); dfree(bd.pz); dfree(bd.pdx); dfree(bd.pdy); dfree(bd.pdz);
    dfree(bd.fx); dfree(bd.fy); dfree(bd.fz); dfree(bd.perm); dfree(bd.pos_of); dfree(bd.goff); dfree(bd.inS);
    dfree(bd.xyz0); dfree(bd.disp0);
    bd.nb = 0;
    bd.m = 0;
    bd.alloc_nb = 0;
    bd.alloc_m = 0;
}

// The FP64 volume sweep's table, allocated on first use (sp.cap doubles each).
// (A failed allocation leaves some of the arrays unset: all are allocated again on the next call.)
void ensure_volume_table(gcb_ctx* ctx) {
    Support& sp = ctx->sp;
    if (sp.qx && sp.qy && sp.qz && sp.qq) return;
    dalloc(ctx, sp.qx, sp.cap); dalloc(ctx, sp.qy, sp.cap); dalloc(ctx, sp.qz, sp.cap); dalloc(ctx, sp.qq, sp.cap);
}

// The FP32 evaluation copies, allocated on first use (sp.cap floats each).
void ensure_fp32_copies(gcb_ctx* ctx) {
    Support& sp = ctx->sp;
    if (sp.fsx && sp.fsy && sp.fsz && sp.fwx && sp.fwy && sp.fwz) return;
    dalloc(ctx, sp.fsx, sp.cap); dalloc(ctx, sp.fsy, sp.cap); dalloc(ctx, sp.fsz, sp.cap);
    dalloc(ctx, sp.fwx, sp.cap); dalloc(ctx, sp.fwy, sp.cap); dalloc(ctx, sp.fwz, sp.cap);
}

int per_iter(const gcb_ctx* ctx) { return std::max(1, ctx->params.per_iter); }

// Partials of the append kernels for the current capacity (4 per 16-row chunk; kBlkPart with several nodes per
// iteration), and the block variant's Lambda (cap x kMaxPerIter) and decision record.
void ensure_append_buffers(gcb_ctx* ctx) {
    const int64_t cap = ctx->sp.cap;
    const int64_t nbl = (cap + kRowsL - 1) / kRowsL + 1;
    const bool blk = per_iter(ctx) > 1;
    dalloc_cap(ctx, ctx->Pb, ctx->Pb_cap, (decltype(ctx->Pb_cap))((blk ? kBlkPart : 4) * nbl));
    if (blk) {
        dalloc_cap(ctx, ctx->lam, ctx->lam_cap, (decltype(ctx->lam_cap))(cap * kMaxPerIter));
        if (!ctx->brec) dalloc(ctx, ctx->brec, 1);
    }
}

// (Re)allocate the support arrays for capacity `cap`, keeping the first n
// supports and the first n rows of the factor (both copies).
void grow_support(gcb_ctx* ctx, int64_t cap, int64_t n) {
    Support& sp = ctx->sp;
    Support nw;
    nw.cap = cap;
    const size_t tri = (size_t)cap * (size_t)(cap + 1) / 2;
    try {
        dalloc(ctx, nw.sx, cap); dalloc(ctx, nw.sy, cap); dalloc(ctx, nw.sz, cap);
        dalloc(ctx, nw.wx, cap); dalloc(ctx, nw.wy, cap); dalloc(ctx, nw.wz, cap);
        dalloc(ctx, nw.orig, cap);
        dalloc(ctx, nw.M, tri);
        dalloc(ctx, nw.Mc, tri);
        dalloc(ctx, nw.l, cap);
    } catch (...) {
        free_support(nw);   // the current arrays stay as they were
        throw;
    }
    if (n > 0 && sp.cap > 0) {
        const size_t b8 = sizeof(double) * (size_t)n;
        HIPCHK(ctx, hipMemcpyAsync(nw.sx, sp.sx, b8, hipMemcpyDeviceToDevice, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(nw.sy, sp.sy, b8, hipMemcpyDeviceToDevice, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(nw.sz, sp.sz, b8, hipMemcpyDeviceToDevice, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(nw.wx, sp.wx, b8, hipMemcpyDeviceToDevice, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(nw.wy, sp.wy, b8, hipMemcpyDeviceToDevice, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(nw.wz, sp.wz, b8, hipMemcpyDeviceToDevice, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(nw.orig, sp.orig, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(nw.M, sp.M, sizeof(double) * (size_t)n * (size_t)(n + 1) / 2, hipMemcpyDeviceToDevice,
                                   ctx->stream));
        launch_transpose_factor(ctx->stream, nw.M, nw.Mc, (int)n, cap);
        HIPCHK(ctx, hipGetLastError());
        sync(ctx);
    }
    free_support(sp);
    sp = nw;
    ensure_append_buffers(ctx);
}

template <typename T>
void grow_log_array(gcb_ctx* ctx, T*& p, int64_t old_len, int64_t cap) {
    T* q = nullptr;
    dalloc(ctx, q, cap);
    if (p && old_len > 0) HIPCHK(ctx, hipMemcpyAsync(q, p, sizeof(T) * old_len, hipMemcpyDeviceToDevice, ctx->stream));
    sync(ctx);
    dfree(p);
    p = q;
}

void grow_log(gcb_ctx* ctx, int64_t used, int64_t cap) {
    grow_log_array(ctx, ctx->log_group, used, cap);
    grow_log_array(ctx, ctx->log_node, used, cap);
    grow_log_array(ctx, ctx->log_err, used, cap);
    grow_log_array(ctx, ctx->log_app, used, cap);
    grow_log_array(ctx, ctx->mon, 2 * used, 2 * cap);   // at most one monitor sample per iteration
    ctx->log_cap = cap;
}

void check_params(gcb_ctx* ctx) {
    const gcb_params& p = ctx->params;
    const int64_t nb = ctx->bd.nb;
    if (!ctx->have_params) fail(ctx, GCB_E_STATE, "gcb_set_params has not been called");
    if (nb < 3) fail(ctx, GCB_E_STATE, "gcb_set_boundary has not been called");
    if (!(p.radius > 0.0) || !std::isfinite(p.radius)) fail(ctx, GCB_E_INVALID, "radius must be finite and > 0");
    if (p.m < 1 || p.m > nb) fail(ctx, GCB_E_INVALID, "m must satisfy 1 <= m <= nb");
    if (!(p.tol_abs >= 0.0) || !std::isfinite(p.tol_abs)) fail(ctx, GCB_E_INVALID, "tol_abs must be finite and >= 0");
    if (p.nc_max < 3 || p.nc_max > nb) fail(ctx, GCB_E_INVALID, "nc_max must satisfy 3 <= nc_max <= nb");
    if (p.nc_max > (int64_t)1 << 30) fail(ctx, GCB_E_INVALID, "nc_max too large");
    if (p.precision != GCB_PREC_FP64 && p.precision != GCB_PREC_FP32_EVAL)
        fail(ctx, GCB_E_INVALID, "unknown precision");
    if (p.monitor_every < 0) fail(ctx, GCB_E_INVALID, "monitor_every must be >= 0");
    if (p.per_iter < 0 || p.per_iter > GCB_MAX_PER_ITER) fail(ctx, GCB_E_INVALID, "per_iter must be in [0, 16]");
    if (p.use_init) {
        for (int t = 0; t < 3; ++t)
            if (p.init_idx[t] < 0 || p.init_idx[t] >= nb) fail(ctx, GCB_E_INVALID, "init_idx out of range");
        if (p.init_idx[0] == p.init_idx[1] || p.init_idx[0] == p.init_idx[2] || p.init_idx[1] == p.init_idx[2])
            fail(ctx, GCB_E_INVALID, "init_idx must be distinct");
    }
    if (ctx->have_groups)
        for (int64_t j = 0; j < nb; ++j)
            if (ctx->groups_h[j] < 0 || ctx->groups_h[j] >= p.m) fail(ctx, GCB_E_INVALID, "group id out of [0, m)");
}

// Partition, permutation and staging of the boundary (a1).
void stage_boundary(gcb_ctx* ctx) {
    Boundary& bd = ctx->bd;
    const gcb_params& p = ctx->params;
    const int64_t nb = bd.nb;
    std::vector<int32_t> grp(static_cast<size_t>(nb));
    if (ctx->have_groups) grp = ctx->groups_h;
    else seeded_partition(nb, p.m, p.seed, grp.data());
    std::vector<int32_t> goff(static_cast<size_t>(p.m) + 1, 0);
    for (int64_t j = 0; j < nb; ++j) goff[grp[j] + 1]++;
    int32_t gmax = 0;
    for (int32_t g = 0; g < p.m; ++g) {
        gmax = std::max(gmax, goff[g + 1]);
        goff[g + 1] += goff[g];
    }
    std::vector<int32_t> fill(goff.begin(), goff.end() - 1), perm(static_cast<size_t>(nb));
    for (int64_t j = 0; j < nb; ++j) perm[fill[grp[j]]++] = static_cast<int32_t>(j);
    bd.m = p.m;
    bd.radius = p.radius;
    bd.inv_r = 1.0 / p.radius;
    bd.gmax = gmax;
    bd.goff_h = goff;
    if (bd.alloc_nb != nb) {   // keep the buffers (and any captured graph) when the size is unchanged
        dalloc(ctx, bd.px, nb); dalloc(ctx, bd.py, nb); dalloc(ctx, bd.pz, nb);
        dalloc(ctx, bd.pdx, nb); dalloc(ctx, bd.pdy, nb); dalloc(ctx, bd.pdz, nb);
        dalloc(ctx, bd.perm, nb); dalloc(ctx, bd.pos_of, nb); dalloc(ctx, bd.inS, nb);
        bd.alloc_nb = nb;
    }
    if (bd.alloc_m < p.m) {
        dalloc(ctx, bd.goff, (size_t)p.m + 1);
        bd.alloc_m = p.m;
    }
    HIPCHK(ctx, hipMemcpyAsync(bd.perm, perm.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(bd.goff, goff.data(), sizeof(int32_t) * (p.m + 1), hipMemcpyHostToDevice, ctx->stream));
    launch_stage(ctx->stream, nb, bd.xyz0, bd.disp0, bd.perm, bd.inv_r, bd);
    HIPCHK(ctx, hipGetLastError());
    sync(ctx);   // host vectors above go out of scope
}

int64_t n_upper(const gcb_ctx* ctx, int64_t n, int64_t iters) {
    return std::min<int64_t>(ctx->params.nc_max, n + iters * per_iter(ctx));
}

IterCtx make_ic(gcb_ctx* ctx) {
    IterCtx ic;
    ic.st = ctx->state;
    ic.irec = ctx->irec;
    ic.srec = ctx->argrec;
    ic.init = reinterpret_cast<int32_t*>(ctx->argrec + ctx->argrec_cap - 1);
    ic.bd = &ctx->bd;
    ic.sp = &ctx->sp;
    ic.Pb = ctx->Pb;
    ic.tol_abs = ctx->params.tol_abs;
    ic.nc_max = ctx->params.nc_max;
    ic.log_cap = ctx->log_cap;
    ic.log_group = ctx->log_group;
    ic.log_node = ctx->log_node;
    ic.log_err = ctx->log_err;
    ic.log_app = ctx->log_app;
    ic.lam = ctx->lam;
    ic.brec = ctx->brec;
    return ic;
}

void ensure_red(gcb_ctx* ctx) {
    const int64_t need = 2 * (certify_blocks(ctx->bd.nb) + 2) + 2;
    dalloc_cap(ctx, ctx->red, ctx->red_cap, (decltype(ctx->red_cap))need);
}

void ensure_tmp(gcb_ctx* ctx, size_t need) {
    if (ctx->tmp_cap < need) {
        if (ctx->tmp) (void)hipFree(ctx->tmp);
        ctx->tmp = nullptr;
        ctx->tmp_cap = 0;
        HIPCHK(ctx, hipMalloc(&ctx->tmp, need));
        ctx->tmp_cap = need;
    }
}

// Warm start: keep S0 and its factor, re-stage the boundary with the current
// displacements, W = M^T (M Delta_S0), and end at once if the FP64 all-node
// error already meets E*; else the loop continues from k = |S0|.
void warm_begin(gcb_ctx* ctx) {
    check_params(ctx);
    const gcb_params& p = ctx->params;
    if (!ctx->warm_ok) fail(ctx, GCB_E_STATE, "a warm start needs a finished selection on this boundary");
    if (p.m != ctx->warm_m || p.seed != ctx->warm_seed || p.radius != ctx->warm_radius)
        fail(ctx, GCB_E_STATE, "a warm start needs the radius, m and seed of the kept selection");
    const int64_t n = ctx->warm_n;
    if (p.nc_max < n) fail(ctx, GCB_E_INVALID, "nc_max is below the kept support count");
    ctx->selected = false;
    ctx->warm_ok = false;   // until this selection finishes
    stage_boundary(ctx);    // the same partition; the new displacements; S cleared
    Boundary& bd = ctx->bd;
    launch_mark_support(ctx->stream, bd, ctx->sp, (int)n);
    HIPCHK(ctx, hipMemsetAsync(ctx->irec, 0, sizeof(IterRec), ctx->stream));
    HIPCHK(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    ensure_tmp(ctx, sizeof(double) * 6 * (size_t)n + 256);
    double* D = static_cast<double*>(ctx->tmp);
    if (!launch_support_weights(ctx->stream, ctx->sp, (int)n, bd.disp0, D, D + 3 * (size_t)n))
        fail(ctx, GCB_E_DEVICE, "internal error: weight recomputation rejected");
    ensure_red(ctx);
    launch_certify(ctx->stream, bd, ctx->sp, (int)n, ctx->red, ctx->red + ctx->red_cap - 2);
    HIPCHK(ctx, hipGetLastError());
    double mr[2];
    HIPCHK(ctx, hipMemcpyAsync(mr, ctx->red + ctx->red_cap - 2, sizeof(mr), hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
    GState st{};
    st.k = n;
    st.n = (int32_t)n;
    st.singular_node = -1;
    st.done = std::sqrt(mr[0]) <= p.tol_abs ? 1 : 0;
    *ctx->state_pin = st;
    ctx->state_h = st;
    HIPCHK(ctx, hipMemcpyAsync(ctx->state, ctx->state_pin, sizeof(st), hipMemcpyHostToDevice, ctx->stream));
    sync(ctx);   // the pinned state is read back later
    ctx->k_host = n;
    ctx->in_progress = true;
}

// Stage the boundary, allocate, pick and append the three starting nodes.
void select_begin(gcb_ctx* ctx) {
    for (int q = 0; q < 4; ++q) {
        ctx->ktime_ms[q] = 0.0;
        ctx->ktime_n[q] = 0;
    }
    ctx->ktime_valid = false;
    ctx->probes = 0;
    ctx->probe_skipped = 0;
    ctx->probe_cert = false;
    ctx->probed_n = -1;
    if (ctx->params.warm_start) {
        warm_begin(ctx);
        return;
    }
    check_params(ctx);
    ctx->selected = false;
    ctx->warm_ok = false;   // the support set is rebuilt from three nodes
    stage_boundary(ctx);
    const gcb_params& p = ctx->params;
    Boundary& bd = ctx->bd;
    const int64_t cap0 = std::min<int64_t>(p.nc_max, 1024);
    if (ctx->sp.cap < cap0 || ctx->sp.cap > p.nc_max) {
        free_support(ctx->sp);
        grow_support(ctx, cap0, 0);
    }
    ensure_append_buffers(ctx);
    const int64_t nrec = std::max<int64_t>(512, sweep_blocks(bd.gmax)) * per_iter(ctx);
    // the last record holds the three starting nodes
    dalloc_cap(ctx, ctx->argrec, ctx->argrec_cap, (decltype(ctx->argrec_cap))(nrec + 1));
    if (!ctx->state) dalloc(ctx, ctx->state, 1);
    if (!ctx->irec) dalloc(ctx, ctx->irec, 1);
    if (!ctx->state_pin) HIPCHK(ctx, hipHostMalloc(reinterpret_cast<void**>(&ctx->state_pin), sizeof(GState)));
    if (!ctx->ev0) HIPCHK(ctx, hipEventCreate(&ctx->ev0));
    if (!ctx->ev1) HIPCHK(ctx, hipEventCreate(&ctx->ev1));
    HIPCHK(ctx, hipMemsetAsync(ctx->irec, 0, sizeof(IterRec), ctx->stream));
    if (ctx->log_cap == 0) grow_log(ctx, 0, 65536);
    int32_t* init = reinterpret_cast<int32_t*>(ctx->argrec + ctx->argrec_cap - 1);
    static_assert(sizeof(ArgRec) >= 3 * sizeof(int32_t), "record too small");
    HIPCHK(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    GState st{};
    st.k = 3;
    st.init_left = 3;
    st.singular_node = -1;
    *ctx->state_pin = st;
    ctx->state_h = st;
    HIPCHK(ctx, hipMemcpyAsync(ctx->state, ctx->state_pin, sizeof(st), hipMemcpyHostToDevice, ctx->stream));
    if (p.use_init) {
        int32_t h[3] = {(int32_t)p.init_idx[0], (int32_t)p.init_idx[1], (int32_t)p.init_idx[2]};
        HIPCHK(ctx, hipMemcpyAsync(init, h, sizeof(h), hipMemcpyHostToDevice, ctx->stream));
        sync(ctx);
    } else {
        launch_init_nodes(ctx->stream, bd, init, ctx->argrec);
    }
    const IterCtx ic = make_ic(ctx);
    for (int t = 0; t < 3; ++t) launch_init_append(ctx->stream, ic, t);
    HIPCHK(ctx, hipGetLastError());
    ctx->k_host = 3;
    ctx->in_progress = true;
}

// After the state has been copied to state_pin and the stream synchronised:
// true while the selection runs; grows the factor and the log so the next
// `chunk` iterations fit.
bool select_poll(gcb_ctx* ctx, int chunk) {
    ctx->state_h = *ctx->state_pin;
    const GState& h = ctx->state_h;
    if (h.done == 4) fail(ctx, GCB_E_DEVICE, "internal error: factor capacity exhausted inside a chunk");
    if (h.done != 0) return false;
    const gcb_params& p = ctx->params;
    const int64_t need = h.n + (int64_t)chunk * per_iter(ctx);
    if (need > ctx->sp.cap && ctx->sp.cap < p.nc_max) {
        const int64_t cap = std::min<int64_t>(p.nc_max, std::max<int64_t>(2 * ctx->sp.cap, need + 1));
        grow_support(ctx, cap, h.n);
    }
    if (h.log_len + chunk > ctx->log_cap) grow_log(ctx, h.log_len, std::max<int64_t>(2 * ctx->log_cap, h.log_len + chunk));
    return true;
}

// Certificate and result of a finished selection.
void select_end(gcb_ctx* ctx, gcb_select_info* info) {
    const gcb_params& p = ctx->params;
    Boundary& bd = ctx->bd;
    ctx->in_progress = false;
    HIPCHK(ctx, hipEventRecord(ctx->ev1, ctx->stream));
    const GState& h = ctx->state_h;
    if (h.done == 3) {
        ctx->err = "support matrix not numerically SPD when appending node " + std::to_string(h.singular_node);
        throw Fail{GCB_E_SINGULAR};
    }
    gcb_select_info inf{};
    inf.nc = h.n;
    inf.iterations = h.log_len;
    inf.status = h.done == 2 ? GCB_NOT_CONVERGED : GCB_OK;
    inf.pairs_group = h.pairs_group;
    inf.pairs_append = h.pairs_append;
    // FP64 certificate over all boundary nodes
    ensure_red(ctx);
    const bool ktime = ctx->ktime_on && per_iter(ctx) == 1 && ctx->ktime_ev.size() >= 2;
    double mr[2];
    if (ctx->probe_cert) {
        // the convergence probe already swept every node with the final W
        sync(ctx);   // (the selection's end event)
        mr[0] = ctx->probe_cert_max;
        mr[1] = ctx->probe_cert_sum;
    } else {
        if (ktime) HIPCHK(ctx, hipEventRecord(ctx->ktime_ev[ctx->ktime_ev.size() - 2], ctx->stream));
        launch_certify(ctx->stream, bd, ctx->sp, h.n, ctx->red, ctx->red + ctx->red_cap - 2);
        HIPCHK(ctx, hipGetLastError());
        if (ktime) HIPCHK(ctx, hipEventRecord(ctx->ktime_ev.back(), ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(mr, ctx->red + ctx->red_cap - 2, sizeof(mr), hipMemcpyDeviceToHost, ctx->stream));
        sync(ctx);
    }
    if (ktime) {
        float t = 0.f;
        HIPCHK(ctx, hipEventElapsedTime(&t, ctx->ktime_ev[ctx->ktime_ev.size() - 2], ctx->ktime_ev.back()));
        ctx->ktime_ms[3] += t;
        ctx->ktime_n[3] += 1;
        ctx->ktime_valid = true;
    }
    float ms = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    inf.ms_select = ms;
    inf.final_max_err = std::sqrt(mr[0]);
    inf.final_rms_err = std::sqrt(mr[1] / (double)bd.nb);
    inf.converged = inf.final_max_err <= p.tol_abs;
    inf.pairs_cert = (uint64_t)bd.nb * (uint64_t)h.n;
    inf.probed_iterations = ctx->probe_skipped;
    ctx->info = inf;
    ctx->selected = true;
    ctx->warm_ok = true;
    ctx->warm_radius = p.radius;
    ctx->warm_m = p.m;
    ctx->warm_seed = p.seed;
    ctx->warm_n = h.n;
    if (info) *info = inf;
}

// Iterations per captured chunk, 0 when chunks are not captured.  A chunk
// bakes in the group of every iteration, so its length c divides into the
// schedule: for m <= 256 a multiple of m of about 64 (every chunk starts at
// the same phase of k mod m: one graph); above, a divisor of m in [32, 128]
// (m / c phases, one graph each); none when m has no such divisor.
int graph_chunk(const gcb_ctx* ctx) {
    const int m = ctx->params.m;
    if (!g_tuning.use_graph) return 0;
    if (m <= 256) return m * ((64 + m - 1) / m);
    int best = 0;
    for (int c = 32; c <= 128; ++c)
        if (m % c == 0 && (best == 0 || std::abs(c - 64) < std::abs(best - 64))) best = c;
    return best;
}

void clear_chunk_graphs(gcb_ctx* ctx) {
    for (auto& pe : ctx->chunk_execs) (void)hipGraphExecDestroy(pe.second);
    ctx->chunk_execs.clear();
}

// Enqueue `chunk` iterations from ctx->k_host as one captured graph, kept per
// phase k mod m of its first iteration (all are captured again when anything
// else they baked in has changed).
void launch_chunk(gcb_ctx* ctx, int chunk) {
    const gcb_params& p = ctx->params;
    const int m = p.m;
    const int64_t k = ctx->k_host;
    const IterCtx ic = make_ic(ctx);
    int64_t tol_bits;
    std::memcpy(&tol_bits, &p.tol_abs, sizeof(tol_bits));
    // everything else the captured launches baked in: capacities, buffers, parameters
    const std::vector<int64_t> key = {m, chunk, ctx->sp.cap, ctx->log_cap, p.nc_max, tol_bits,
                                      (int64_t)ctx->alloc_gen, (int64_t)(intptr_t)ctx->stream, per_iter(ctx)};
    if (ctx->chunk_key != key) {
        clear_chunk_graphs(ctx);
        ctx->chunk_key = key;
    }
    const int64_t phase = k % m;
    hipGraphExec_t exec = nullptr;
    for (auto& pe : ctx->chunk_execs)
        if (pe.first == phase) exec = pe.second;
    if (!exec) {
        if (!ctx->cap_stream) HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        hipGraph_t graph;
        HIPCHK(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
        const int n_ub = (int)std::min<int64_t>(p.nc_max, ctx->sp.cap);
        const int pi = per_iter(ctx);
        for (int it = 0; it < chunk; ++it) {
            if (pi > 1) launch_iteration_block(ctx->cap_stream, ic, (int)((k + it) % m), n_ub, pi);
            else launch_iteration(ctx->cap_stream, ic, (int)((k + it) % m), n_ub);
        }
        HIPCHK(ctx, hipStreamEndCapture(ctx->cap_stream, &graph));
        hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(ctx, e);
        ctx->chunk_execs.emplace_back(phase, exec);
    }
    HIPCHK(ctx, hipGraphLaunch(exec, ctx->stream));
    HIPCHK(ctx, hipGetLastError());
    ctx->k_host = k + chunk;
}

// Kernel timing: events between the launches of `chunk` iterations (4 per iteration, reused every chunk).
void ktime_events(gcb_ctx* ctx, int chunk) {
    while ((int)ctx->ktime_ev.size() < 4 * chunk + 2) {
        hipEvent_t e;
        HIPCHK(ctx, hipEventCreate(&e));
        ctx->ktime_ev.push_back(e);
    }
}

// Adds the device times of the chunk just launched (waits for it).
void ktime_collect(gcb_ctx* ctx, int chunk, const std::vector<int>& swept) {
    sync(ctx);
    for (int it = 0; it < chunk; ++it) {
        const hipEvent_t* e = &ctx->ktime_ev[4 * it];
        for (int q = 0; q < 3; ++q) {
            if (q == 0 && !swept[it]) continue;
            float t = 0.f;
            HIPCHK(ctx, hipEventElapsedTime(&t, e[q], e[q + 1]));
            ctx->ktime_ms[q] += t;
            ctx->ktime_n[q] += 1;
        }
    }
}

// Convergence probe (at a chunk boundary, after `quiet` iterations without an append): W has not changed during
// them, so Algorithm 1's next m - quiet iterations are all quiet exactly when every group they visit has no node
// outside S with an error above E*.  One FP64 sweep of all nodes gives every group's maximum; if none exceeds
// E*, the remaining iterations are completed here with the log entries they would write (group, its argmax node
// or -1, its error, nothing appended) and the counters they would add, and the selection ends as converged.
// Returns true if it ended the selection.
bool probe_converged(gcb_ctx* ctx) {
    const gcb_params& p = ctx->params;
    Boundary& bd = ctx->bd;
    const GState h = ctx->state_h;
    const int m = p.m;
    const int rem = m - h.quiet;
    // (no captured graph reads these buffers, so growing them does not invalidate one)
    if (ctx->perr_cap < bd.nb) {
        ctx->perr_cap = 0;
        if (ctx->perr) (void)hipFree(ctx->perr);
        ctx->perr = nullptr;
        HIPCHK(ctx, hipMalloc(reinterpret_cast<void**>(&ctx->perr), sizeof(double) * (size_t)bd.nb));
        ctx->perr_cap = bd.nb;
    }
    if (ctx->gmax_cap < m) {
        ctx->gmax_cap = 0;
        if (ctx->gmax) (void)hipFree(ctx->gmax);
        ctx->gmax = nullptr;
        HIPCHK(ctx, hipMalloc(&ctx->gmax, sizeof(GroupMax) * (size_t)m));
        ctx->gmax_cap = m;
    }
    launch_probe(ctx->stream, bd, ctx->sp, h.n, ctx->perr, static_cast<GroupMax*>(ctx->gmax));
    HIPCHK(ctx, hipGetLastError());
    std::vector<GroupMax> g((size_t)m);
    HIPCHK(ctx, hipMemcpyAsync(g.data(), ctx->gmax, sizeof(GroupMax) * (size_t)m, hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
    ctx->probes += 1;
    const int64_t k = ctx->k_host;
    for (int i = 0; i < rem; ++i) {
        const GroupMax& r = g[(size_t)((k + i) % m)];
        if (r.count > 0 && std::sqrt(r.e2) > p.tol_abs) return false;
    }
    if (h.log_len + rem > ctx->log_cap) grow_log(ctx, h.log_len, std::max<int64_t>(2 * ctx->log_cap, h.log_len + rem));
    std::vector<int32_t> lg((size_t)rem), ln((size_t)rem);
    std::vector<double> le((size_t)rem);
    std::vector<int8_t> la((size_t)rem, 0);
    uint64_t pairs = 0;
    for (int i = 0; i < rem; ++i) {
        const int gi = (int)((k + i) % m);
        const GroupMax& r = g[(size_t)gi];
        lg[(size_t)i] = gi;
        ln[(size_t)i] = r.count > 0 ? r.orig : -1;
        le[(size_t)i] = r.count > 0 ? std::sqrt(r.e2) : 0.0;
        pairs += (uint64_t)r.count * (uint64_t)h.n;
    }
    GState st = h;
    st.k = h.k + rem;
    st.quiet = m;
    st.done = 1;
    st.log_len = h.log_len + rem;
    st.pairs_group = h.pairs_group + pairs;
    const int64_t o = h.log_len;
    HIPCHK(ctx, hipMemcpyAsync(ctx->log_group + o, lg.data(), sizeof(int32_t) * rem, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(ctx->log_node + o, ln.data(), sizeof(int32_t) * rem, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(ctx->log_err + o, le.data(), sizeof(double) * rem, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(ctx->log_app + o, la.data(), sizeof(int8_t) * rem, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(ctx->state, &st, sizeof(GState), hipMemcpyHostToDevice, ctx->stream));
    sync(ctx);   // the host vectors go out of scope
    ctx->state_h = st;
    ctx->k_host = k + rem;
    ctx->probe_skipped = rem;
    // W stays as the probe saw it, so its errors are the certificate's (the same per-node arithmetic): the
    // largest, and the sum in group order
    double mx = 0.0, sum = 0.0;
    for (int gi = 0; gi < m; ++gi) {
        mx = std::max(mx, g[(size_t)gi].all_max);
        sum += g[(size_t)gi].all_sum;
    }
    ctx->probe_cert = true;
    ctx->probe_cert_max = mx;
    ctx->probe_cert_sum = sum;
    return true;
}

// At a chunk or batch-step boundary, with the state just polled: run the probe once per run of quiet
// iterations (W changes with every append), after max(8, m / 16) of them and while at least 8 remain.
// True if it ended the selection.
bool maybe_probe(gcb_ctx* ctx) {
    const int m = ctx->params.m;
    const GState& hs = ctx->state_h;
    if (!g_tuning.probe || ctx->params.monitor_every > 0) return false;
    if (hs.quiet < std::max(8, m / g_tuning.probe_div) || m - hs.quiet < 8 || hs.n == ctx->probed_n) return false;
    ctx->probed_n = hs.n;
    return probe_converged(ctx);
}

void run_select(gcb_ctx* ctx, gcb_select_info* info) {
    select_begin(ctx);
    const gcb_params& p = ctx->params;
    // Every iteration advances k by one, so the host knows the group of each
    // launch.  A chunk of C iterations with C a multiple of m starts at the
    // same phase of k mod m every time and is captured once into a graph.
    const int m = p.m;
    const int every = p.monitor_every;
    const int pi = per_iter(ctx);
    const bool ktime = ctx->ktime_on && pi == 1;   // kernel timing covers Algorithm 1's three kernels
    const int gchunk = (every > 0 || ktime) ? 0 : graph_chunk(ctx);
    const int chunk = gchunk > 0 ? gchunk : 64;
    const int64_t k0 = ctx->k_host;   // loop start (3, or |S0| for a warm start)
    if (every > 0) ensure_red(ctx);
    std::vector<int> swept(ktime ? chunk : 0, 0);
    if (ktime) ktime_events(ctx, chunk);
    for (;;) {
        HIPCHK(ctx, hipMemcpyAsync(ctx->state_pin, ctx->state, sizeof(GState), hipMemcpyDeviceToHost, ctx->stream));
        sync(ctx);
        if (!select_poll(ctx, chunk)) break;
        if (!ktime && maybe_probe(ctx)) break;
        if (gchunk > 0) {
            launch_chunk(ctx, chunk);
        } else {
            const int64_t k = ctx->k_host;
            const IterCtx ic = make_ic(ctx);
            for (int it = 0; it < chunk; ++it) {
                const int n_ub = (int)n_upper(ctx, ctx->state_h.n, it + 1);
                if (pi > 1) {
                    launch_iteration_block(ctx->stream, ic, (int)((k + it) % m), (int)n_ub, pi);
                } else {
                    const int sw = launch_iteration(ctx->stream, ic, (int)((k + it) % m), n_ub,
                                                    ktime ? &ctx->ktime_ev[4 * it] : nullptr);
                    if (ktime) swept[it] = sw;
                }
                const int64_t done_iters = k + it + 1 - k0;   // loop iterations launched so far
                if (every > 0 && done_iters % every == 0) {
                    const int64_t s = done_iters / every - 1;
                    launch_monitor(ctx->stream, ctx->bd, ctx->sp, ctx->state, done_iters, ctx->red,
                                   ctx->mon + 2 * s);
                }
            }
            HIPCHK(ctx, hipGetLastError());
            ctx->k_host = k + chunk;
            if (ktime) ktime_collect(ctx, chunk, swept);
        }
    }
    select_end(ctx, info);
}

template <typename F>
int guard(gcb_ctx* ctx, F&& f) {
    if (!ctx) return GCB_E_INVALID;
    try {
        ctx->err.clear();
        return f();
    } catch (const Fail& e) {
        return e.code;
    } catch (const std::bad_alloc&) {
        ctx->err = "host allocation failed";
        return GCB_E_NOMEM;
    } catch (...) {
        ctx->err = "unexpected internal error";
        return GCB_E_DEVICE;
    }
}

}  // namespace

namespace gcb {
size_t ctx_device_bytes(const gcb_ctx* ctx) {
    if (!ctx) return 0;
    const Boundary& bd = ctx->bd;
    const Support& sp = ctx->sp;
    size_t b = 0;
    if (bd.xyz0) b += 48 * (size_t)bd.nb;                                    // xyz0, disp0
    b += (size_t)bd.alloc_nb * (6 * sizeof(double) + 2 * sizeof(int32_t) + 1);  // staged SoA, perm, pos_of, inS
    b += sizeof(int32_t) * ((size_t)bd.alloc_m + 1);
    const size_t tri = (size_t)sp.cap * (size_t)(sp.cap + 1) / 2;
    b += (size_t)sp.cap * (7 * sizeof(double) + sizeof(int32_t)) + 2 * sizeof(double) * tri;
    if (sp.fsx) b += 6 * sizeof(float) * (size_t)sp.cap;   // FP32 evaluation copies
    if (sp.qx) b += 4 * sizeof(double) * (size_t)sp.cap;   // volume table
    b += sizeof(double) * (size_t)ctx->Pb_cap + sizeof(ArgRec) * (size_t)ctx->argrec_cap;
    b += sizeof(double) * (size_t)ctx->lam_cap + (ctx->brec ? sizeof(BlockRec) : 0);
    b += (size_t)ctx->log_cap * (2 * sizeof(int32_t) + 3 * sizeof(double) + 1);   // log and monitor samples
    b += sizeof(double) * (size_t)ctx->red_cap + ctx->tmp_cap + sizeof(GState) + sizeof(IterRec);
    b += dense_plan_bytes(ctx->dplan);
    return b;
}
}  // namespace gcb

struct gcb_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    bool lone_graph = true;   // a step with one running context replays its captured chunk
    int sweep_tpl = 0;        // 0: automatic
    int factor_rpw = 0;       // 0: automatic
    // per-iteration argument tables (device) and their pinned staging
    void* dtab = nullptr;
    size_t dtab_cap = 0;
    void* htab = nullptr;
    size_t htab_cap = 0;
};

namespace {

struct BFail {
    int code;
};

[[noreturn]] void bfail(gcb_batch* b, int code, const std::string& msg) {
    b->err = msg;
    throw BFail{code};
}

#define BHIPCHK(b, expr)                                                                          \
    do {                                                                                          \
        hipError_t _e = (expr);                                                                   \
        if (_e != hipSuccess) bfail((b), GCB_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

template <typename F>
int bguard(gcb_batch* b, F&& f) {
    if (!b) return GCB_E_INVALID;
    try {
        b->err.clear();
        return f();
    } catch (const BFail& e) {
        return e.code;
    } catch (const Fail& e) {
        return e.code;   // message in the context
    } catch (const std::bad_alloc&) {
        b->err = "host allocation failed";
        return GCB_E_NOMEM;
    } catch (...) {
        b->err = "unexpected internal error";
        return GCB_E_DEVICE;
    }
}

void ensure_tables(gcb_batch* b, size_t bytes) {
    if (b->dtab_cap < bytes) {
        if (b->dtab) (void)hipFree(b->dtab);
        b->dtab = nullptr;
        b->dtab_cap = 0;
        BHIPCHK(b, hipMalloc(&b->dtab, bytes));
        b->dtab_cap = bytes;
    }
    if (b->htab_cap < bytes) {
        if (b->htab) (void)hipHostFree(b->htab);
        b->htab = nullptr;
        b->htab_cap = 0;
        BHIPCHK(b, hipHostMalloc(&b->htab, bytes));
        b->htab_cap = bytes;
    }
}

void attach(gcb_batch* b, gcb_ctx* ctx) {
    if (!ctx) bfail(b, GCB_E_INVALID, "NULL context");
    if (ctx->device != b->device) bfail(b, GCB_E_INVALID, "context on another device");
    if (ctx->stream != b->stream) {
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        ctx->stream = b->stream;
    }
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int32_t batch_step(gcb_batch* b, gcb_ctx* const* ctxs, int32_t count, int32_t iterations, int32_t* running) {
    if (count < 0 || (count > 0 && !ctxs)) bfail(b, GCB_E_INVALID, "bad context list");
    if (iterations < 1 || iterations > 4096) bfail(b, GCB_E_INVALID, "iterations must be in [1, 4096]");
    BHIPCHK(b, hipSetDevice(b->device));
    for (int32_t i = 0; i < count; ++i) {
        attach(b, ctxs[i]);
        if (ctxs[i]->params.per_iter > 1) bfail(b, GCB_E_INVALID, "per_iter > 1 is not available in batches");
        if (ctxs[i]->in_progress)
            HIPCHK(ctxs[i], hipMemcpyAsync(ctxs[i]->state_pin, ctxs[i]->state, sizeof(GState), hipMemcpyDeviceToHost,
                                           b->stream));
    }
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    std::vector<gcb_ctx*> run;
    for (int32_t i = 0; i < count; ++i) {
        gcb_ctx* c = ctxs[i];
        bool r = false;
        if (c->in_progress) r = select_poll(c, iterations);
        if (r && maybe_probe(c)) r = false;   // the probe completed the selection's quiet tail
        if (running) running[i] = r ? 1 : 0;
        if (r) run.push_back(c);
    }
    const int L = (int)run.size();
    if (L == 0) return 0;
    if (L == 1 && b->lone_graph) {
        // a lone running selection replays its own captured chunk (a multiple of m iterations)
        gcb_ctx* c = run[0];
        const int chunk = graph_chunk(c);
        if (chunk > 0) {
            if (chunk > iterations) (void)select_poll(c, chunk);   // capacity for the longer chunk
            launch_chunk(c, chunk);
            return 1;
        }
    }
    if (L > kMaxBatch) bfail(b, GCB_E_INVALID, "at most 64 running contexts per step");
    const size_t s_b = align_up(sizeof(SweepArgs) * (size_t)L);
    const size_t l_b = align_up(sizeof(FactorLArgs) * (size_t)L);
    const size_t u_b = align_up(sizeof(FactorUArgs) * (size_t)L);
    const size_t per_it = s_b + l_b + u_b;
    ensure_tables(b, per_it * (size_t)iterations);
    // With several running contexts the batch supplies the parallelism: blocks take more
    // targets (sweep) and more rows of M (factor), so one launch needs fewer block rounds.
    // automatic layout (measured on 32 uneven surfaces): wide sweeps from four running contexts on,
    // one 16-row chunk per factor wave
    const bool wide = b->sweep_tpl > 0 || L >= 4;
    const int rpw = b->factor_rpw > 0 ? b->factor_rpw : 1;
    std::vector<BlockMap> smaps((size_t)iterations), fmaps((size_t)iterations);
    char* h = static_cast<char*>(b->htab);
    std::vector<IterCtx> ics;
    ics.reserve(L);
    for (int j = 0; j < L; ++j) ics.push_back(make_ic(run[j]));
    for (int it = 0; it < iterations; ++it) {
        SweepArgs* sa = reinterpret_cast<SweepArgs*>(h + per_it * it);
        FactorLArgs* la = reinterpret_cast<FactorLArgs*>(h + per_it * it + s_b);
        FactorUArgs* ua = reinterpret_cast<FactorUArgs*>(h + per_it * it + s_b + l_b);
        BlockMap& sm = smaps[it];
        BlockMap& fm = fmaps[it];
        sm.count = fm.count = L;
        sm.off[0] = fm.off[0] = 0;
        for (int j = 0; j < L; ++j) {
            gcb_ctx* c = run[j];
            const int g = (int)((c->k_host + it) % c->params.m);
            // at most one append per iteration: |S| <= n_poll + it here
            const int64_t n_ub = std::min<int64_t>(c->sp.cap, c->state_h.n + it + 1);
            sa[j] = make_sweep_args(ics[j], g);
            if (wide) {
                sweep_layout_batch(sa[j].T, sa[j].lpt, sa[j].tpl);
                if (b->sweep_tpl > 0) sa[j].tpl = b->sweep_tpl;
            }
            sa[j].nub = n_ub;
            la[j] = make_factor_l_args(ics[j], g, sweep_records(sa[j]), -1);
            ua[j] = make_factor_u_args(ics[j]);
            sm.off[j + 1] = sm.off[j] + sweep_records(sa[j]);
            fm.off[j + 1] = fm.off[j] + factor_blocks(std::min<int64_t>(c->params.nc_max, n_ub), rpw);
        }
    }
    BHIPCHK(b, hipMemcpyAsync(b->dtab, b->htab, per_it * (size_t)iterations, hipMemcpyHostToDevice, b->stream));
    char* d = static_cast<char*>(b->dtab);
    for (int it = 0; it < iterations; ++it) {
        launch_iteration_batch(b->stream, reinterpret_cast<SweepArgs*>(d + per_it * it),
                               reinterpret_cast<FactorLArgs*>(d + per_it * it + s_b),
                               reinterpret_cast<FactorUArgs*>(d + per_it * it + s_b + l_b), smaps[it], fmaps[it],
                               rpw);
    }
    BHIPCHK(b, hipGetLastError());
    for (int j = 0; j < L; ++j) run[j]->k_host += iterations;
    return L;
}

}  // namespace

namespace {

// Events around the kernels of a deformation (not recorded while the stream is being captured).
// Morton interleave of three 10-bit cell indices (supports' order for the culled sweep).
uint32_t morton10(uint32_t x, uint32_t y, uint32_t z) {
    auto spread = [](uint32_t v) {
        v &= 0x3ffu;
        v = (v | (v << 16)) & 0x030000FFu;
        v = (v | (v << 8)) & 0x0300F00Fu;
        v = (v | (v << 4)) & 0x030C30C3u;
        v = (v | (v << 2)) & 0x09249249u;
        return v;
    };
    return spread(x) | (spread(y) << 1) | (spread(z) << 2);
}

// Eq. (6) with compact-support culling (params.cull_volume, FP64): the volume table is formed on the device and
// read back with the weights (7 doubles per support); the host orders the supports in Morton order, forms the
// bounding box of every tile of kCullTileHost and uploads them; the points' Morton keys are sorted on the device
// (radix sort of (key, index) pairs), and the culled sweep evaluates the points in that order.
void deform_culled(gcb_ctx* ctx, int64_t nv, const void* din, bool in_f64, void* dout, bool out_f64) {
    Support& sp = ctx->sp;
    const int n = (int)ctx->info.nc;
    ensure_volume_table(ctx);
    launch_volume_table(ctx->stream, sp, n);
    HIPCHK(ctx, hipGetLastError());
    std::vector<double> h(7 * (size_t)n + 3);
    const double* src[7] = {sp.qx, sp.qy, sp.qz, sp.qq, sp.wx, sp.wy, sp.wz};
    for (int a = 0; a < 7; ++a)
        HIPCHK(ctx, hipMemcpyAsync(h.data() + (size_t)a * n, src[a], sizeof(double) * n, hipMemcpyDeviceToHost,
                                   ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(h.data() + 7 * (size_t)n, sp.sx, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(h.data() + 7 * (size_t)n + 1, sp.sy, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(h.data() + 7 * (size_t)n + 2, sp.sz, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
    const double* q[3] = {h.data(), h.data() + n, h.data() + 2 * (size_t)n};
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = *std::min_element(q[a], q[a] + n);
        hi[a] = *std::max_element(q[a], q[a] + n);
    }
    // frame: the supports' box grown by R (0.5 in these units) on every side, cubic cells
    const double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]}) + 1.0;
    CullFrame f{lo[0] - 0.5, lo[1] - 0.5, lo[2] - 0.5, 1023.0 / ext};
    std::vector<std::pair<uint32_t, int>> key((size_t)n);
    for (int j = 0; j < n; ++j) {
        uint32_t c[3];
        const double fl[3] = {f.lox, f.loy, f.loz};
        for (int a = 0; a < 3; ++a)
            c[a] = (uint32_t)std::min(1023.0, std::max(0.0, (q[a][j] - fl[a]) * f.sc));
        key[(size_t)j] = {morton10(c[0], c[1], c[2]), j};
    }
    std::stable_sort(key.begin(), key.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    const int ntiles = (n + kCullTileHost - 1) / kCullTileHost;
    std::vector<double> hs(7 * (size_t)n + 6 * (size_t)ntiles);
    for (int j = 0; j < n; ++j)
        for (int a = 0; a < 7; ++a) hs[(size_t)a * n + j] = h[(size_t)a * n + key[(size_t)j].second];
    for (int k = 0; k < ntiles; ++k) {
        double* b = hs.data() + 7 * (size_t)n + 6 * (size_t)k;
        for (int a = 0; a < 3; ++a) {
            b[a] = std::numeric_limits<double>::infinity();
            b[3 + a] = -std::numeric_limits<double>::infinity();
        }
        for (int j = k * kCullTileHost; j < std::min(n, (k + 1) * kCullTileHost); ++j)
            for (int a = 0; a < 3; ++a) {
                b[a] = std::min(b[a], hs[(size_t)a * n + j]);
                b[3 + a] = std::max(b[3 + a], hs[(size_t)a * n + j]);
            }
    }
    dalloc_cap(ctx, ctx->cs, ctx->cs_cap, (decltype(ctx->cs_cap))hs.size());
    HIPCHK(ctx, hipMemcpyAsync(ctx->cs, hs.data(), sizeof(double) * hs.size(), hipMemcpyHostToDevice, ctx->stream));
    CullSupports cs{ctx->cs, ctx->cs + n, ctx->cs + 2 * (size_t)n, ctx->cs + 3 * (size_t)n, ctx->cs + 4 * (size_t)n,
                    ctx->cs + 5 * (size_t)n, ctx->cs + 6 * (size_t)n, ctx->cs + 7 * (size_t)n};
    // the points' Morton order
    if (ctx->cull_cap < nv) {
        ctx->cull_cap = 0;
        dalloc(ctx, ctx->ck_in, (size_t)nv); dalloc(ctx, ctx->ck_out, (size_t)nv);
        dalloc(ctx, ctx->ci_in, (size_t)nv); dalloc(ctx, ctx->ci_out, (size_t)nv);
        ctx->cull_cap = nv;
    }
    const double c0[3] = {0.5 * h[7 * (size_t)n], 0.5 * h[7 * (size_t)n + 1], 0.5 * h[7 * (size_t)n + 2]};
    launch_cull_keys(ctx->stream, nv, din, in_f64, ctx->bd.inv_r, c0, f, ctx->ck_in, ctx->ci_in);
    HIPCHK(ctx, hipGetLastError());
    size_t tb = 0;
    HIPCHK(ctx, sort_pairs_u32(nullptr, &tb, ctx->ck_in, ctx->ck_out, ctx->ci_in, ctx->ci_out, nv, 31, ctx->stream));
    if (ctx->sort_tmp_cap < tb) {
        if (ctx->sort_tmp) (void)hipFree(ctx->sort_tmp);
        ctx->sort_tmp = nullptr;
        ctx->sort_tmp_cap = 0;
        HIPCHK(ctx, hipMalloc(&ctx->sort_tmp, tb));
        ctx->sort_tmp_cap = tb;
    }
    HIPCHK(ctx, sort_pairs_u32(ctx->sort_tmp, &tb, ctx->ck_in, ctx->ck_out, ctx->ci_in, ctx->ci_out, nv, 31,
                               ctx->stream));
    const int64_t nblk = cull_blocks(nv);
    dalloc_cap(ctx, ctx->cull_ev, ctx->cull_ev_cap, (decltype(ctx->cull_ev_cap))nblk);
    launch_volume_cull(ctx->stream, nv, din, in_f64, ctx->ci_out, ctx->bd.inv_r, c0, cs, n, dout, out_f64,
                       ctx->cull_ev);
    HIPCHK(ctx, hipGetLastError());
    ctx->cull_nblk = nblk;
    ctx->cull_dense = (uint64_t)nv * (uint64_t)n;
    ctx->cull_valid = true;
    sync(ctx);   // the host copies of the sorted supports go out of scope
}

bool deform_timing_begin(gcb_ctx* ctx) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIPCHK(ctx, hipStreamIsCapturing(ctx->stream, &cs));
    ctx->deform_timed = false;
    if (cs != hipStreamCaptureStatusNone) return false;
    if (!ctx->ev2) HIPCHK(ctx, hipEventCreate(&ctx->ev2));
    if (!ctx->ev3) HIPCHK(ctx, hipEventCreate(&ctx->ev3));
    HIPCHK(ctx, hipEventRecord(ctx->ev2, ctx->stream));
    return true;
}

void deform_timing_end(gcb_ctx* ctx, bool on) {
    if (!on) return;
    HIPCHK(ctx, hipEventRecord(ctx->ev3, ctx->stream));
    ctx->deform_timed = true;
}

}  // namespace

extern "C" {

int gcb_batch_create(gcb_batch** out, int device, void* hip_stream) {
    if (!out) return GCB_E_INVALID;
    *out = nullptr;
    gcb_batch* b = new (std::nothrow) gcb_batch();
    if (!b) return GCB_E_NOMEM;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || device < 0 || device >= n) {
        g_create_err = e != hipSuccess ? std::string("hipGetDeviceCount: ") + hipGetErrorString(e)
                                       : "device index out of range";
        delete b;
        return e != hipSuccess ? GCB_E_DEVICE : GCB_E_INVALID;
    }
    b->device = device;
    e = hipSetDevice(device);
    if (e != hipSuccess) {
        g_create_err = std::string("hipSetDevice: ") + hipGetErrorString(e);
        delete b;
        return GCB_E_DEVICE;
    }
    b->stream = static_cast<hipStream_t>(hip_stream);   // verbatim: NULL is the null stream
    *out = b;
    return GCB_OK;
}

void gcb_batch_destroy(gcb_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->dtab) (void)hipFree(b->dtab);
    if (b->htab) (void)hipHostFree(b->htab);
    delete b;
}

const char* gcb_batch_last_error(const gcb_batch* b) { return b ? b->err.c_str() : g_create_err.c_str(); }

int gcb_batch_set_layout(gcb_batch* b, int32_t sweep_tpl, int32_t factor_rpw, int32_t lone_graph) {
    return bguard(b, [&] {
        if (!(sweep_tpl == 0 || sweep_tpl == 1 || sweep_tpl == 2 || sweep_tpl == 4))
            bfail(b, GCB_E_INVALID, "sweep_tpl must be 0, 1, 2 or 4");
        if (!(factor_rpw == 0 || factor_rpw == 1 || factor_rpw == kMaxRowsPerWave))
            bfail(b, GCB_E_INVALID, "factor_rpw must be 0, 1 or 4");
        b->sweep_tpl = sweep_tpl;
        b->factor_rpw = factor_rpw;
        b->lone_graph = lone_graph != 0;
        return GCB_OK;
    });
}

int gcb_batch_begin(gcb_batch* b, gcb_ctx* ctx) {
    return bguard(b, [&] {
        BHIPCHK(b, hipSetDevice(b->device));
        if (ctx && ctx->params.monitor_every > 0) bfail(b, GCB_E_INVALID, "monitor samples are not taken in batches");
        if (ctx && ctx->params.per_iter > 1) bfail(b, GCB_E_INVALID, "per_iter > 1 is not available in batches");
        attach(b, ctx);
        return guard(ctx, [&] {
            select_begin(ctx);
            return GCB_OK;
        });
    });
}

int32_t gcb_batch_step(gcb_batch* b, gcb_ctx* const* ctxs, int32_t count, int32_t iterations, int32_t* running) {
    int32_t nrun = 0;
    const int rc = bguard(b, [&] {
        nrun = batch_step(b, ctxs, count, iterations, running);
        return GCB_OK;
    });
    return rc < 0 ? rc : nrun;
}

int gcb_batch_end(gcb_batch* b, gcb_ctx* ctx, gcb_select_info* info) {
    return bguard(b, [&] {
        BHIPCHK(b, hipSetDevice(b->device));
        attach(b, ctx);
        return guard(ctx, [&] {
            if (!ctx->in_progress) fail(ctx, GCB_E_STATE, "no selection in progress");
            if (ctx->state_h.done == 0) fail(ctx, GCB_E_STATE, "selection still running");
            select_end(ctx, info);
            return ctx->info.status;
        });
    });
}

int gcb_select_batch(gcb_batch* b, gcb_ctx* const* ctxs, int32_t count, gcb_select_info* infos) {
    return bguard(b, [&] {
        if (count < 1 || !ctxs) bfail(b, GCB_E_INVALID, "need at least one context");
        int status = GCB_OK;
        for (int32_t s0 = 0; s0 < count; s0 += kMaxBatch) {   // slices of at most 64 contexts
            const int32_t sc = std::min<int32_t>(kMaxBatch, count - s0);
            for (int32_t i = s0; i < s0 + sc; ++i) {
                const int rc = gcb_batch_begin(b, ctxs[i]);
                if (rc < 0) return rc;
            }
            for (;;) {
                const int32_t n = gcb_batch_step(b, ctxs + s0, sc, 64, nullptr);
                if (n < 0) return (int)n;
                if (n == 0) break;
            }
            for (int32_t i = s0; i < s0 + sc; ++i) {
                const int rc = gcb_batch_end(b, ctxs[i], infos ? &infos[i] : nullptr);
                if (rc < 0) return rc;
                if (rc == GCB_NOT_CONVERGED) status = GCB_NOT_CONVERGED;
            }
        }
        return status;
    });
}

int gcb_deform_batch(gcb_batch* b, gcb_ctx* const* ctxs, int32_t count, const int64_t* nv, const void* const* xyz,
                     int in_dtype, void* const* out, int out_dtype) {
    return bguard(b, [&] {
        if (count < 1 || count > kMaxBatch || !ctxs || !nv || !xyz || !out)
            bfail(b, GCB_E_INVALID, "bad arguments (1 <= count <= 64, non-NULL arrays)");
        if ((in_dtype != GCB_F32 && in_dtype != GCB_F64) || (out_dtype != GCB_F32 && out_dtype != GCB_F64))
            bfail(b, GCB_E_INVALID, "dtype must be GCB_F32 or GCB_F64");
        BHIPCHK(b, hipSetDevice(b->device));
        const size_t bytes = align_up(sizeof(VolDesc) * (size_t)count);
        ensure_tables(b, bytes);
        BHIPCHK(b, hipStreamSynchronize(b->stream));   // the tables may still be read by earlier launches
        VolDesc* t = static_cast<VolDesc*>(b->htab);
        BlockMap map{}, tmap{};
        map.count = count;
        tmap.count = count;
        for (int32_t i = 0; i < count; ++i) {
            gcb_ctx* c = ctxs[i];
            attach(b, c);
            if (!c->selected) bfail(b, GCB_E_STATE, "context without a finished selection");
            if (nv[i] < 0 || (nv[i] > 0 && (!xyz[i] || !out[i]))) bfail(b, GCB_E_INVALID, "bad volume arguments");
            const int n = nv[i] > 0 ? (int)c->info.nc : 0;   // a surface without targets needs no table
            if (n > 0) ensure_volume_table(c);
            t[i] = VolDesc{xyz[i], out[i], nv[i], view(c->sp), vtable(c->sp), n, c->bd.inv_r};
            map.off[i + 1] = map.off[i] + (int)((nv[i] + kBlock - 1) / kBlock);
            tmap.off[i + 1] = tmap.off[i] + (n + kBlock - 1) / kBlock;
        }
        if (map.off[count] == 0) return GCB_OK;
        BHIPCHK(b, hipMemcpyAsync(b->dtab, b->htab, bytes, hipMemcpyHostToDevice, b->stream));
        launch_volume_batch(b->stream, static_cast<VolDesc*>(b->dtab), map, tmap, in_dtype == GCB_F64,
                            out_dtype == GCB_F64);
        BHIPCHK(b, hipGetLastError());
        return GCB_OK;
    });
}


const char* gcb_version(void) { return "gcb-mi355x 0.1 (gfx950, FP64 sweeps, inverse-factor append)"; }

int gcb_partition(int64_t nb, int32_t m, uint64_t seed, int32_t* group_of) {
    if (nb < 1 || m < 1 || m > nb || !group_of) return GCB_E_INVALID;
    try {
        seeded_partition(nb, m, seed, group_of);
    } catch (...) {
        return GCB_E_NOMEM;
    }
    return GCB_OK;
}

int gcb_create(gcb_ctx** out, int device, void* hip_stream) {
    if (!out) return GCB_E_INVALID;
    if (const char* e = std::getenv("GCB_SWEEP_LPT")) {
        const int v = std::atoi(e);
        if (v == 64 || v == 128 || v == 256) g_tuning.sweep_lpt_max = v;
    }
    if (const char* e = std::getenv("GCB_GRAPH")) g_tuning.use_graph = std::atoi(e) != 0;
    if (const char* e = std::getenv("GCB_PROBE")) g_tuning.probe = std::atoi(e) != 0;
    if (const char* e = std::getenv("GCB_PROBE_DIV")) {
        const int v = std::atoi(e);
        if (v >= 1 && v <= 1024) g_tuning.probe_div = v;
    }
    *out = nullptr;
    gcb_ctx* ctx = new (std::nothrow) gcb_ctx();
    if (!ctx) return GCB_E_NOMEM;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || device < 0 || device >= n) {
        g_create_err = e != hipSuccess ? std::string("hipGetDeviceCount: ") + hipGetErrorString(e)
                                       : "device index out of range";
        delete ctx;
        return e != hipSuccess ? GCB_E_DEVICE : GCB_E_INVALID;
    }
    ctx->device = device;
    e = hipSetDevice(device);
    if (e == hipSuccess && !hip_stream) e = hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        g_create_err = std::string("hip setup: ") + hipGetErrorString(e);
        delete ctx;
        return GCB_E_DEVICE;
    }
    if (e == hipSuccess) e = noalloc_setup(device);   // the scratch address for gcb_deform_noalloc
    if (e != hipSuccess) {
        g_create_err = std::string("hip setup: ") + hipGetErrorString(e);
        if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
        delete ctx;
        return GCB_E_DEVICE;
    }
    ctx->stream = hip_stream ? static_cast<hipStream_t>(hip_stream) : ctx->own_stream;
    *out = ctx;
    return GCB_OK;
}

void gcb_destroy(gcb_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    free_boundary(ctx->bd);
    free_support(ctx->sp);
    dfree(ctx->state); dfree(ctx->argrec); dfree(ctx->red); dfree(ctx->irec); dfree(ctx->Pb);
    dfree(ctx->lam); dfree(ctx->brec);
    if (ctx->perr) (void)hipFree(ctx->perr);
    if (ctx->gmax) (void)hipFree(ctx->gmax);
    dfree(ctx->ck_in); dfree(ctx->ck_out); dfree(ctx->ci_in); dfree(ctx->ci_out); dfree(ctx->cs); dfree(ctx->cull_ev);
    if (ctx->sort_tmp) (void)hipFree(ctx->sort_tmp);
    dfree(ctx->log_group); dfree(ctx->log_node); dfree(ctx->log_err); dfree(ctx->log_app); dfree(ctx->mon);
    if (ctx->tmp) (void)hipFree(ctx->tmp);
    free_dense_plan(ctx->dplan);
    clear_chunk_graphs(ctx);
    for (hipEvent_t e : ctx->ktime_ev) (void)hipEventDestroy(e);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    if (ctx->ev2) (void)hipEventDestroy(ctx->ev2);
    if (ctx->ev3) (void)hipEventDestroy(ctx->ev3);
    if (ctx->state_pin) (void)hipHostFree(ctx->state_pin);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
    delete ctx;
}

const char* gcb_last_error(const gcb_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

int gcb_set_stream(gcb_ctx* ctx, void* hip_stream) {
    return guard(ctx, [&] {
        HIPCHK(ctx, hipSetDevice(ctx->device));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));   // work already enqueued finishes first
        ctx->stream = static_cast<hipStream_t>(hip_stream);
        return GCB_OK;
    });
}

int gcb_set_boundary(gcb_ctx* ctx, int64_t nb, const double* xyz, const double* disp, int mem) {
    return guard(ctx, [&] {
        if (nb < 3 || !xyz || !disp) fail(ctx, GCB_E_INVALID, "need nb >= 3 and non-NULL xyz, disp");
        if (nb > ((int64_t)1 << 30)) fail(ctx, GCB_E_INVALID, "nb too large");
        if (mem != GCB_MEM_HOST && mem != GCB_MEM_DEVICE) fail(ctx, GCB_E_INVALID, "bad mem kind");
        if (mem == GCB_MEM_HOST && (!all_finite(xyz, 3 * nb) || !all_finite(disp, 3 * nb)))
            fail(ctx, GCB_E_INVALID, "non-finite boundary coordinate or displacement");
        HIPCHK(ctx, hipSetDevice(ctx->device));
        ctx->selected = false;
        ctx->warm_ok = false;
        free_boundary(ctx->bd);   // nb = 0 until both copies exist
        dalloc(ctx, ctx->bd.xyz0, 3 * (size_t)nb);
        dalloc(ctx, ctx->bd.disp0, 3 * (size_t)nb);
        ctx->bd.nb = nb;
        copy_in(ctx, ctx->bd.xyz0, xyz, sizeof(double) * 3 * nb, mem);
        copy_in(ctx, ctx->bd.disp0, disp, sizeof(double) * 3 * nb, mem);
        if (mem == GCB_MEM_DEVICE) {
            int32_t* flag = nullptr;
            dalloc(ctx, flag, 1);
            HIPCHK(ctx, hipMemsetAsync(flag, 0, sizeof(int32_t), ctx->stream));
            launch_check_finite(ctx->stream, 3 * nb, ctx->bd.xyz0, ctx->bd.disp0, flag);
            int32_t h = 0;
            HIPCHK(ctx, hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
            sync(ctx);
            dfree(flag);
            if (h) {
                free_boundary(ctx->bd);
                fail(ctx, GCB_E_INVALID, "non-finite boundary coordinate or displacement");
            }
        }
        sync(ctx);
        if (ctx->have_groups && (int64_t)ctx->groups_h.size() != nb) ctx->have_groups = false;
        return GCB_OK;
    });
}

int gcb_set_displacement(gcb_ctx* ctx, const double* disp, int mem) {
    return guard(ctx, [&] {
        if (ctx->bd.nb < 3) fail(ctx, GCB_E_STATE, "gcb_set_boundary has not been called");
        if (!disp) fail(ctx, GCB_E_INVALID, "disp is NULL");
        const int64_t nb = ctx->bd.nb;
        if (mem == GCB_MEM_HOST && !all_finite(disp, 3 * nb)) fail(ctx, GCB_E_INVALID, "non-finite displacement");
        HIPCHK(ctx, hipSetDevice(ctx->device));
        copy_in(ctx, ctx->bd.disp0, disp, sizeof(double) * 3 * nb, mem);
        if (mem == GCB_MEM_DEVICE) {
            int32_t* flag = nullptr;
            dalloc(ctx, flag, 1);
            HIPCHK(ctx, hipMemsetAsync(flag, 0, sizeof(int32_t), ctx->stream));
            launch_check_finite(ctx->stream, 3 * nb, ctx->bd.disp0, nullptr, flag);
            int32_t h = 0;
            HIPCHK(ctx, hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
            sync(ctx);
            dfree(flag);
            if (h) fail(ctx, GCB_E_INVALID, "non-finite displacement");
        }
        sync(ctx);
        ctx->selected = false;
        return GCB_OK;
    });
}

int gcb_set_params(gcb_ctx* ctx, const gcb_params* p) {
    return guard(ctx, [&] {
        if (!p) fail(ctx, GCB_E_INVALID, "params is NULL");
        if (p->per_iter < 0 || p->per_iter > GCB_MAX_PER_ITER) fail(ctx, GCB_E_INVALID, "per_iter must be in [0, 16]");
        if (p->per_iter > 1 && p->warm_start) fail(ctx, GCB_E_INVALID, "per_iter > 1 is not available with warm starts");
        ctx->params = *p;
        ctx->have_params = true;
        ctx->selected = false;
        return GCB_OK;
    });
}

int gcb_set_groups(gcb_ctx* ctx, const int32_t* group_of, int mem) {
    return guard(ctx, [&] {
        if (!group_of) {
            if (ctx->have_groups) ctx->warm_ok = false;
            ctx->have_groups = false;
            ctx->groups_h.clear();
            return GCB_OK;
        }
        if (ctx->bd.nb < 3) fail(ctx, GCB_E_STATE, "gcb_set_boundary has not been called");
        ctx->groups_h.resize(static_cast<size_t>(ctx->bd.nb));
        if (mem == GCB_MEM_DEVICE) {
            HIPCHK(ctx, hipMemcpyAsync(ctx->groups_h.data(), group_of, sizeof(int32_t) * ctx->bd.nb, hipMemcpyDeviceToHost,
                                       ctx->stream));
            sync(ctx);
        } else {
            std::memcpy(ctx->groups_h.data(), group_of, sizeof(int32_t) * ctx->bd.nb);
        }
        ctx->have_groups = true;
        ctx->selected = false;
        ctx->warm_ok = false;
        return GCB_OK;
    });
}

int gcb_select(gcb_ctx* ctx, gcb_select_info* info) {
    return guard(ctx, [&] {
        HIPCHK(ctx, hipSetDevice(ctx->device));
        run_select(ctx, info);
        return ctx->info.status;
    });
}

int gcb_get_support(gcb_ctx* ctx, int64_t* idx, double* w, int mem) {
    return guard(ctx, [&] {
        if (!ctx->selected) fail(ctx, GCB_E_STATE, "no finished selection");
        HIPCHK(ctx, hipSetDevice(ctx->device));
        const int64_t n = ctx->info.nc;
        std::vector<int32_t> o(static_cast<size_t>(n));
        std::vector<double> wx(n), wy(n), wz(n);
        HIPCHK(ctx, hipMemcpyAsync(o.data(), ctx->sp.orig, sizeof(int32_t) * n, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(wx.data(), ctx->sp.wx, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(wy.data(), ctx->sp.wy, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(wz.data(), ctx->sp.wz, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
        sync(ctx);
        std::vector<int64_t> oi(o.begin(), o.end());
        std::vector<double> wa(3 * (size_t)n);
        for (int64_t s = 0; s < n; ++s) {
            wa[3 * s] = wx[s];
            wa[3 * s + 1] = wy[s];
            wa[3 * s + 2] = wz[s];
        }
        if (mem == GCB_MEM_DEVICE) {
            if (idx) HIPCHK(ctx, hipMemcpyAsync(idx, oi.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, ctx->stream));
            if (w) HIPCHK(ctx, hipMemcpyAsync(w, wa.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, ctx->stream));
            sync(ctx);
        } else {
            if (idx) std::memcpy(idx, oi.data(), sizeof(int64_t) * n);
            if (w) std::memcpy(w, wa.data(), sizeof(double) * 3 * n);
        }
        return GCB_OK;
    });
}

int64_t gcb_get_log(gcb_ctx* ctx, int32_t* group, int64_t* node, double* err, int8_t* appended, int64_t cap) {
    if (!ctx) return GCB_E_INVALID;
    int64_t total = 0;
    int rc = guard(ctx, [&] {
        if (!ctx->selected) fail(ctx, GCB_E_STATE, "no finished selection");
        if (cap < 0) fail(ctx, GCB_E_INVALID, "cap < 0");
        HIPCHK(ctx, hipSetDevice(ctx->device));
        total = ctx->state_h.log_len;
        const int64_t n = std::min(cap, std::min(total, ctx->log_cap));
        if (n > 0) {
            std::vector<int32_t> nd(static_cast<size_t>(n));
            if (group) HIPCHK(ctx, hipMemcpyAsync(group, ctx->log_group, sizeof(int32_t) * n, hipMemcpyDeviceToHost, ctx->stream));
            if (node) HIPCHK(ctx, hipMemcpyAsync(nd.data(), ctx->log_node, sizeof(int32_t) * n, hipMemcpyDeviceToHost, ctx->stream));
            if (err) HIPCHK(ctx, hipMemcpyAsync(err, ctx->log_err, sizeof(double) * n, hipMemcpyDeviceToHost, ctx->stream));
            if (appended) HIPCHK(ctx, hipMemcpyAsync(appended, ctx->log_app, n, hipMemcpyDeviceToHost, ctx->stream));
            sync(ctx);
            if (node)
                for (int64_t i = 0; i < n; ++i) node[i] = nd[i];
        }
        return GCB_OK;
    });
    return rc < 0 ? rc : total;
}

int64_t gcb_get_monitor(gcb_ctx* ctx, int64_t* iteration, double* max_err, double* rms_err, int64_t cap) {
    if (!ctx) return GCB_E_INVALID;
    int64_t total = 0;
    int rc = guard(ctx, [&] {
        if (!ctx->selected) fail(ctx, GCB_E_STATE, "no finished selection");
        if (cap < 0) fail(ctx, GCB_E_INVALID, "cap < 0");
        const int every = ctx->params.monitor_every;
        total = every > 0 ? std::min<int64_t>(ctx->state_h.log_len, ctx->log_cap) / every : 0;
        const int64_t n = std::min(cap, total);
        if (n > 0) {
            HIPCHK(ctx, hipSetDevice(ctx->device));
            std::vector<double> h(2 * (size_t)n);
            HIPCHK(ctx, hipMemcpyAsync(h.data(), ctx->mon, sizeof(double) * h.size(), hipMemcpyDeviceToHost, ctx->stream));
            sync(ctx);
            for (int64_t s = 0; s < n; ++s) {
                if (iteration) iteration[s] = (s + 1) * (int64_t)every;
                if (max_err) max_err[s] = std::sqrt(h[2 * s]);
                if (rms_err) rms_err[s] = std::sqrt(h[2 * s + 1] / (double)ctx->bd.nb);
            }
        }
        return GCB_OK;
    });
    return rc < 0 ? rc : total;
}

int gcb_deform(gcb_ctx* ctx, int64_t nv, const void* xyz, int in_dtype, void* out, int out_dtype, int mem) {
    return guard(ctx, [&] {
        if (!ctx->selected) fail(ctx, GCB_E_STATE, "no finished selection");
        if (nv < 0) fail(ctx, GCB_E_INVALID, "nv < 0");
        if (nv == 0) return GCB_OK;
        if (!xyz || !out) fail(ctx, GCB_E_INVALID, "NULL xyz or out");
        if ((in_dtype != GCB_F32 && in_dtype != GCB_F64) || (out_dtype != GCB_F32 && out_dtype != GCB_F64))
            fail(ctx, GCB_E_INVALID, "dtype must be GCB_F32 or GCB_F64");
        if (mem != GCB_MEM_HOST && mem != GCB_MEM_DEVICE) fail(ctx, GCB_E_INVALID, "bad mem kind");
        HIPCHK(ctx, hipSetDevice(ctx->device));
        const size_t in_b = (size_t)nv * 3 * (in_dtype == GCB_F64 ? 8 : 4);
        const size_t out_b = (size_t)nv * 3 * (out_dtype == GCB_F64 ? 8 : 4);
        const size_t in_pad = align_up(in_b);   // the output starts aligned whatever nv and the input type
        const void* din = xyz;
        void* dout = out;
        if (mem == GCB_MEM_HOST) {
            ensure_tmp(ctx, in_pad + out_b);
            HIPCHK(ctx, hipMemcpyAsync(ctx->tmp, xyz, in_b, hipMemcpyHostToDevice, ctx->stream));
            din = ctx->tmp;
            dout = static_cast<char*>(ctx->tmp) + in_pad;
        }
        const bool timed = deform_timing_begin(ctx);
        if (ctx->params.precision == GCB_PREC_FP32_EVAL) {
            Support& sp = ctx->sp;
            ensure_fp32_copies(ctx);
            launch_volume32(ctx->stream, nv, din, in_dtype == GCB_F64, ctx->bd.inv_r, sp, (int)ctx->info.nc, dout,
                            out_dtype == GCB_F64);
        } else if (ctx->params.cull_volume) {
            deform_culled(ctx, nv, din, in_dtype == GCB_F64, dout, out_dtype == GCB_F64);
        } else {
            ensure_volume_table(ctx);
            launch_volume(ctx->stream, nv, din, in_dtype == GCB_F64, ctx->bd.inv_r, ctx->sp, (int)ctx->info.nc, dout,
                          out_dtype == GCB_F64);
        }
        deform_timing_end(ctx, timed);
        HIPCHK(ctx, hipGetLastError());
        if (mem == GCB_MEM_HOST) {
            HIPCHK(ctx, hipMemcpyAsync(out, dout, out_b, hipMemcpyDeviceToHost, ctx->stream));
            sync(ctx);
        }
        return GCB_OK;
    });
}

int gcb_deform_noalloc(gcb_ctx* ctx, int64_t nv, const void* xyz, int in_dtype, void* out, int out_dtype) {
    return guard(ctx, [&] {
        if (!ctx->selected) fail(ctx, GCB_E_STATE, "no finished selection");
        if (nv < 0) fail(ctx, GCB_E_INVALID, "nv < 0");
        if (nv == 0) return GCB_OK;
        if (!xyz || !out) fail(ctx, GCB_E_INVALID, "NULL xyz or out");
        if ((in_dtype != GCB_F32 && in_dtype != GCB_F64) || (out_dtype != GCB_F32 && out_dtype != GCB_F64))
            fail(ctx, GCB_E_INVALID, "dtype must be GCB_F32 or GCB_F64");
        const int64_t n = ctx->info.nc;
        if (n > GCB_NOALLOC_MAX_SUPPORTS)
            fail(ctx, GCB_E_INVALID,
                 "the selection has " + std::to_string(n) + " supports, more than the allocation-free maximum of " +
                     std::to_string(GCB_NOALLOC_MAX_SUPPORTS) + " (gcb_deform has no such limit)");
        void* scr = noalloc_scratch(ctx->device);
        if (!scr) fail(ctx, GCB_E_DEVICE, "no scratch address for this device");
        HIPCHK(ctx, hipSetDevice(ctx->device));
        ctx->deform_timed = false;   // no events are recorded here
        launch_volume_noalloc(ctx->stream, nv, xyz, in_dtype == GCB_F64, ctx->bd.inv_r, ctx->sp, (int)n, out,
                              out_dtype == GCB_F64, ctx->params.precision == GCB_PREC_FP32_EVAL, scr);
        HIPCHK(ctx, hipGetLastError());
        return GCB_OK;
    });
}

int gcb_get_deform_pairs(gcb_ctx* ctx, uint64_t* evaluated, uint64_t* dense) {
    return guard(ctx, [&] {
        if (!ctx->cull_valid) fail(ctx, GCB_E_STATE, "no culled deformation has run");
        HIPCHK(ctx, hipSetDevice(ctx->device));
        std::vector<uint64_t> ev((size_t)ctx->cull_nblk);
        HIPCHK(ctx, hipMemcpyAsync(ev.data(), ctx->cull_ev, sizeof(uint64_t) * ev.size(), hipMemcpyDeviceToHost,
                                   ctx->stream));
        sync(ctx);
        uint64_t sum = 0;
        for (uint64_t v : ev) sum += v;
        if (evaluated) *evaluated = sum;
        if (dense) *dense = ctx->cull_dense;
        return GCB_OK;
    });
}

int gcb_set_kernel_timing(gcb_ctx* ctx, int32_t on) {
    return guard(ctx, [&] {
        if (on != 0 && on != 1) fail(ctx, GCB_E_INVALID, "on must be 0 or 1");
        ctx->ktime_on = on != 0;
        return GCB_OK;
    });
}

int gcb_get_kernel_times(gcb_ctx* ctx, double* ms, int64_t* launches) {
    return guard(ctx, [&] {
        if (!ctx->ktime_valid) fail(ctx, GCB_E_STATE, "no selection ran with kernel timing on");
        for (int q = 0; q < 4; ++q) {
            if (ms) ms[q] = ctx->ktime_ms[q];
            if (launches) launches[q] = ctx->ktime_n[q];
        }
        return GCB_OK;
    });
}

int gcb_deform_time(gcb_ctx* ctx, double* ms) {
    return guard(ctx, [&] {
        if (!ms) fail(ctx, GCB_E_INVALID, "ms is NULL");
        if (!ctx->deform_timed) fail(ctx, GCB_E_STATE, "no timed deformation");
        HIPCHK(ctx, hipSetDevice(ctx->device));
        HIPCHK(ctx, hipEventSynchronize(ctx->ev3));
        float t = 0.f;
        HIPCHK(ctx, hipEventElapsedTime(&t, ctx->ev2, ctx->ev3));
        *ms = t;
        return GCB_OK;
    });
}

int gcb_deform_multi(gcb_ctx* ctx, int32_t k_modes, const double* disp_modes, int64_t nv, const void* xyz,
                     int in_dtype, void* out, int out_dtype, int mem) {
    return guard(ctx, [&] {
        if (!ctx->selected) fail(ctx, GCB_E_STATE, "no finished selection");
        if (k_modes < 1 || 3 * (int64_t)k_modes > 192) fail(ctx, GCB_E_INVALID, "need 1 <= k_modes <= 64");
        if (nv < 0) fail(ctx, GCB_E_INVALID, "nv < 0");
        if (!disp_modes || (nv > 0 && (!xyz || !out))) fail(ctx, GCB_E_INVALID, "NULL pointer");
        if ((in_dtype != GCB_F32 && in_dtype != GCB_F64) || (out_dtype != GCB_F32 && out_dtype != GCB_F64))
            fail(ctx, GCB_E_INVALID, "dtype must be GCB_F32 or GCB_F64");
        if (mem != GCB_MEM_HOST && mem != GCB_MEM_DEVICE) fail(ctx, GCB_E_INVALID, "bad mem kind");
        HIPCHK(ctx, hipSetDevice(ctx->device));
        const int rc = 3 * k_modes;
        const int R = multi_padded_r(rc);
        const int n = (int)ctx->info.nc;
        const int64_t nb = ctx->bd.nb;
        const size_t modes_b = sizeof(double) * (size_t)nb * rc;
        const size_t in_b = (size_t)nv * 3 * (in_dtype == GCB_F64 ? 8 : 4);
        const size_t out_b = (size_t)nv * rc * (out_dtype == GCB_F64 ? 8 : 4);
        const size_t work_b = sizeof(double) * 3 * (size_t)n * R;
        const size_t in_pad = align_up(in_b);   // the output starts aligned whatever nv and the input type
        const size_t need = work_b + modes_b + (mem == GCB_MEM_HOST ? in_pad + out_b : 0) + 1024;
        ensure_tmp(ctx, need);
        char* base = static_cast<char*>(ctx->tmp);
        double* D = reinterpret_cast<double*>(base);
        double* Y = D + (size_t)n * R;
        double* Wm = Y + (size_t)n * R;
        char* p = base + work_b;
        double* modes_d = const_cast<double*>(disp_modes);
        if (mem == GCB_MEM_HOST) {
            modes_d = reinterpret_cast<double*>(p);
            HIPCHK(ctx, hipMemcpyAsync(modes_d, disp_modes, modes_b, hipMemcpyHostToDevice, ctx->stream));
        }
        p += modes_b;
        const void* din = xyz;
        void* dout = out;
        if (mem == GCB_MEM_HOST && nv > 0) {
            HIPCHK(ctx, hipMemcpyAsync(p, xyz, in_b, hipMemcpyHostToDevice, ctx->stream));
            din = p;
            dout = p + in_pad;
        }
        if (!launch_deform_multi(ctx->stream, ctx->sp, n, rc, modes_d, D, Y, Wm, nv, din, in_dtype == GCB_F64,
                                 ctx->bd.inv_r, dout, out_dtype == GCB_F64))
            fail(ctx, GCB_E_INVALID, "unsupported multi-RHS shape");
        HIPCHK(ctx, hipGetLastError());
        if (mem == GCB_MEM_HOST && nv > 0) HIPCHK(ctx, hipMemcpyAsync(out, dout, out_b, hipMemcpyDeviceToHost, ctx->stream));
        if (mem == GCB_MEM_HOST) sync(ctx);
        return GCB_OK;
    });
}

// Inverse factor of the first n supports rebuilt from scratch (dense FP64 on
// the matrix cores) into sp.M / sp.Mc, then W for the current displacements
// and the certificate into ctx->info.  *drift when old factor is compared.
void rebuild_factor(gcb_ctx* ctx, int n, bool compare, double* drift) {
    Support& sp = ctx->sp;
    Boundary& bd = ctx->bd;
    const int np = dense_padded(n);
    const size_t dense_b = sizeof(double) * (size_t)np * np;
    const size_t w_b = sizeof(double) * 6 * (size_t)n;   // Delta_S and M Delta_S, three columns each
    ensure_tmp(ctx, 3 * dense_b + w_b + 1024);
    char* base = static_cast<char*>(ctx->tmp);
    double* A = reinterpret_cast<double*>(base);
    double* Md = reinterpret_cast<double*>(base + dense_b);
    double* Tb = reinterpret_cast<double*>(base + 2 * dense_b);
    double* Wb = reinterpret_cast<double*>(base + 3 * dense_b);
    int32_t* bad = reinterpret_cast<int32_t*>(base + 3 * dense_b + w_b);
    const int nred = dense_pack_blocks();
    dalloc_cap(ctx, ctx->red, ctx->red_cap, (decltype(ctx->red_cap))(2 * nred + 2));
    ensure_red(ctx);
    HIPCHK(ctx, hipMemsetAsync(bad, 0, sizeof(int32_t), ctx->stream));
    HIPCHK(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    HIPCHK(ctx, dense_plan_for(ctx->dplan, n, ctx->stream));
    HIPCHK(ctx, launch_inverse_factor(ctx->stream, sp, n, A, Md, Tb, bad, ctx->dplan));
    HIPCHK(ctx, hipGetLastError());
    int32_t hbad = 0;
    HIPCHK(ctx, hipMemcpyAsync(&hbad, bad, sizeof(hbad), hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
    if (hbad) {
        ctx->err = "support matrix not numerically SPD (a Cholesky pivot <= 64 DBL_EPSILON)";
        throw Fail{GCB_E_SINGULAR};
    }
    launch_pack_factor(ctx->stream, n, Md, sp.M, compare ? sp.M : nullptr, ctx->red);
    launch_transpose_factor(ctx->stream, sp.M, sp.Mc, n, sp.cap);
    if (!launch_support_weights(ctx->stream, sp, n, bd.disp0, Wb, Wb + 3 * (size_t)n))
        fail(ctx, GCB_E_DEVICE, "internal error: weight recomputation rejected");
    HIPCHK(ctx, hipGetLastError());
    if (compare) {
        std::vector<double> red(2 * (size_t)nred);
        HIPCHK(ctx, hipMemcpyAsync(red.data(), ctx->red, sizeof(double) * red.size(), hipMemcpyDeviceToHost,
                                   ctx->stream));
        sync(ctx);
        double dm = 0.0, om = 0.0;
        for (int b = 0; b < nred; ++b) {
            dm = std::max(dm, red[2 * b]);
            om = std::max(om, red[2 * b + 1]);
        }
        if (drift) *drift = om > 0.0 ? dm / om : 0.0;
    }
    launch_certify(ctx->stream, bd, sp, n, ctx->red, ctx->red + ctx->red_cap - 2);
    HIPCHK(ctx, hipEventRecord(ctx->ev1, ctx->stream));
    HIPCHK(ctx, hipGetLastError());
    double mr[2];
    HIPCHK(ctx, hipMemcpyAsync(mr, ctx->red + ctx->red_cap - 2, sizeof(mr), hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
    float ms = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    gcb_select_info& inf = ctx->info;
    inf.nc = n;
    inf.final_max_err = std::sqrt(mr[0]);
    inf.final_rms_err = std::sqrt(mr[1] / (double)bd.nb);
    inf.converged = inf.final_max_err <= ctx->params.tol_abs;
    inf.pairs_cert = (uint64_t)bd.nb * (uint64_t)n;
    inf.ms_select = ms;
}

int gcb_set_support(gcb_ctx* ctx, const int64_t* idx, int64_t n, int mem, gcb_select_info* info) {
    return guard(ctx, [&] {
        check_params(ctx);
        const gcb_params& p = ctx->params;
        const int64_t nb = ctx->bd.nb;
        if (!idx || n < 3 || n > p.nc_max) fail(ctx, GCB_E_INVALID, "need idx and 3 <= n <= nc_max");
        if (mem != GCB_MEM_HOST && mem != GCB_MEM_DEVICE) fail(ctx, GCB_E_INVALID, "bad mem kind");
        HIPCHK(ctx, hipSetDevice(ctx->device));
        std::vector<int64_t> h((size_t)n);
        if (mem == GCB_MEM_DEVICE) {
            HIPCHK(ctx, hipMemcpyAsync(h.data(), idx, sizeof(int64_t) * (size_t)n, hipMemcpyDeviceToHost, ctx->stream));
            sync(ctx);
        } else {
            std::memcpy(h.data(), idx, sizeof(int64_t) * (size_t)n);
        }
        std::vector<uint8_t> seen((size_t)nb, 0);
        std::vector<int32_t> o((size_t)n);
        for (int64_t t = 0; t < n; ++t) {
            if (h[t] < 0 || h[t] >= nb || seen[h[t]]) fail(ctx, GCB_E_INVALID, "idx must be distinct indices in [0, nb)");
            seen[h[t]] = 1;
            o[t] = (int32_t)h[t];
        }
        ctx->selected = false;
        ctx->warm_ok = false;
        ctx->in_progress = false;
        stage_boundary(ctx);
        const int64_t cap = std::max<int64_t>(std::min<int64_t>(p.nc_max, 1024), n);
        if (ctx->sp.cap < n || ctx->sp.cap > std::max<int64_t>(p.nc_max, n)) {
            free_support(ctx->sp);
            grow_support(ctx, cap, 0);
        }
        if (!ctx->state) dalloc(ctx, ctx->state, 1);
        if (!ctx->irec) dalloc(ctx, ctx->irec, 1);
        if (!ctx->state_pin) HIPCHK(ctx, hipHostMalloc(reinterpret_cast<void**>(&ctx->state_pin), sizeof(GState)));
        if (!ctx->ev0) HIPCHK(ctx, hipEventCreate(&ctx->ev0));
        if (!ctx->ev1) HIPCHK(ctx, hipEventCreate(&ctx->ev1));
        const int64_t nrec = std::max<int64_t>(512, sweep_blocks(ctx->bd.gmax));
        dalloc_cap(ctx, ctx->argrec, ctx->argrec_cap, (decltype(ctx->argrec_cap))(nrec + 1));
        if (ctx->log_cap == 0) grow_log(ctx, 0, 65536);
        HIPCHK(ctx, hipMemcpyAsync(ctx->sp.orig, o.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice,
                                   ctx->stream));
        launch_gather_support(ctx->stream, ctx->sp, (int)n, ctx->bd.xyz0, ctx->bd.inv_r);
        launch_mark_support(ctx->stream, ctx->bd, ctx->sp, (int)n);
        HIPCHK(ctx, hipGetLastError());
        ctx->info = gcb_select_info{};
        rebuild_factor(ctx, (int)n, false, nullptr);
        GState st{};
        st.k = n;
        st.n = (int32_t)n;
        st.done = 1;
        st.singular_node = -1;
        ctx->state_h = st;
        gcb_select_info& inf = ctx->info;
        inf.iterations = 0;
        inf.status = GCB_OK;
        ctx->selected = true;
        ctx->warm_ok = true;
        ctx->warm_radius = p.radius;
        ctx->warm_m = p.m;
        ctx->warm_seed = p.seed;
        ctx->warm_n = n;
        if (info) *info = inf;
        return GCB_OK;
    });
}

int gcb_get_factor(gcb_ctx* ctx, double* m, int mem) {
    return guard(ctx, [&] {
        if (!ctx->selected) fail(ctx, GCB_E_STATE, "no finished selection");
        if (!m) fail(ctx, GCB_E_INVALID, "m is NULL");
        if (mem != GCB_MEM_HOST && mem != GCB_MEM_DEVICE) fail(ctx, GCB_E_INVALID, "bad mem kind");
        HIPCHK(ctx, hipSetDevice(ctx->device));
        const size_t n = (size_t)ctx->info.nc;
        HIPCHK(ctx, hipMemcpyAsync(m, ctx->sp.M, sizeof(double) * n * (n + 1) / 2,
                                   mem == GCB_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                                   ctx->stream));
        sync(ctx);
        return GCB_OK;
    });
}

int gcb_refactor(gcb_ctx* ctx, double* drift, gcb_select_info* info) {
    return guard(ctx, [&] {
        if (!ctx->selected) fail(ctx, GCB_E_STATE, "no finished selection to re-certify");
        HIPCHK(ctx, hipSetDevice(ctx->device));
        const int n = (int)ctx->info.nc;
        ctx->selected = false;   // until the rebuild succeeds
        rebuild_factor(ctx, n, true, drift);
        ctx->selected = true;
        if (info) *info = ctx->info;
        return GCB_OK;
    });
}

int gcb_certify(gcb_ctx* ctx, double* max_err, double* rms_err) {
    return guard(ctx, [&] {
        if (!ctx->selected) fail(ctx, GCB_E_STATE, "no finished selection");
        HIPCHK(ctx, hipSetDevice(ctx->device));
        ensure_red(ctx);
        launch_certify(ctx->stream, ctx->bd, ctx->sp, (int)ctx->info.nc, ctx->red, ctx->red + ctx->red_cap - 2);
        HIPCHK(ctx, hipGetLastError());
        double mr[2];
        HIPCHK(ctx, hipMemcpyAsync(mr, ctx->red + ctx->red_cap - 2, sizeof(mr), hipMemcpyDeviceToHost, ctx->stream));
        sync(ctx);
        if (max_err) *max_err = std::sqrt(mr[0]);
        if (rms_err) *rms_err = std::sqrt(mr[1] / (double)ctx->bd.nb);
        return GCB_OK;
    });
}

}  // extern "C"
