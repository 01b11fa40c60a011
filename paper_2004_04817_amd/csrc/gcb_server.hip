// Request loop over deformation requests: FIFO admission by slots and a
// device-memory budget, continuous batching of the admitted selections
// (shared launches, new requests joining at step boundaries), one batched
// volume launch for the selections that finished, and a resident cache of
// meshes (support set, inverse factor) served again by warm starts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "gcb_internal.h"
#include "gcb_kernels.h"

namespace {

double clock_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

enum Phase { kQueued = 0, kSelecting = 1, kDeforming = 2, kDone = 3 };

struct Req {
    gcb_request r{};
    gcb_result res{};
    gcb_ctx* ctx = nullptr;
    bool owns_ctx = false;    // not resident: destroyed when the request completes
    int64_t resident_key = -1;
    hipEvent_t ev = nullptr;  // output complete
};

struct Resident {
    gcb_ctx* ctx = nullptr;
    int64_t nb = 0;
    bool busy = false;
    uint64_t last_use = 0;
};

// bytes a new mesh is expected to take at admission (it may grow while it runs)
uint64_t estimate_bytes(const gcb_request& r) {
    const uint64_t nb = (uint64_t)r.nb;
    const uint64_t c = (uint64_t)std::min<int64_t>(r.params.nc_max, 1024);
    return nb * 105 + c * (c + 1) * 8 + c * 96 + 65536ull * 33 + (1u << 20);   // log: 65,536 entries
}

}  // namespace

struct gcb_server {
    int device = 0;
    hipStream_t stream = nullptr;
    uint64_t budget = 0;
    int max_active = 1;
    int flags = 0;
    gcb_batch* batch = nullptr;
    std::string err;
    std::map<int64_t, Req> reqs;
    std::deque<int64_t> queue;
    std::vector<int64_t> selecting;
    std::vector<int64_t> deforming;
    std::unordered_map<int64_t, Resident> resident;
    uint64_t use_clock = 0;
    int64_t next_ticket = 1;
    hipEvent_t ev_ref = nullptr;
    double t_ref = 0.0;
};

namespace {

struct SFail {
    int code;
};

[[noreturn]] void sfail(gcb_server* s, int code, const std::string& msg) {
    s->err = msg;
    throw SFail{code};
}

#define SHIPCHK(s, expr)                                                                               \
    do {                                                                                               \
        hipError_t _e = (expr);                                                                        \
        if (_e != hipSuccess) sfail((s), GCB_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

template <typename F>
int sguard(gcb_server* s, F&& f) {
    if (!s) return GCB_E_INVALID;
    try {
        return f();
    } catch (const SFail& e) {
        return e.code;
    } catch (const std::bad_alloc&) {
        s->err = "host allocation failed";
        return GCB_E_NOMEM;
    } catch (...) {
        s->err = "unexpected internal error";
        return GCB_E_DEVICE;
    }
}

uint64_t used_bytes(const gcb_server* s) {
    uint64_t b = 0;
    for (const auto& kv : s->resident) b += gcb::ctx_device_bytes(kv.second.ctx);
    for (int64_t t : s->selecting) {
        const Req& q = s->reqs.at(t);
        if (q.owns_ctx) b += gcb::ctx_device_bytes(q.ctx);
    }
    for (int64_t t : s->deforming) {
        const Req& q = s->reqs.at(t);
        if (q.owns_ctx) b += gcb::ctx_device_bytes(q.ctx);
    }
    return b;
}

bool evict_one(gcb_server* s) {
    auto victim = s->resident.end();
    for (auto it = s->resident.begin(); it != s->resident.end(); ++it)
        if (!it->second.busy && (victim == s->resident.end() || it->second.last_use < victim->second.last_use))
            victim = it;
    if (victim == s->resident.end()) return false;
    gcb_destroy(victim->second.ctx);
    s->resident.erase(victim);
    return true;
}

// mark a request failed with the context's (or the server's) message; release its context
void fail_request(gcb_server* s, Req& q, int code) {
    if (q.ctx) {
        const char* m = gcb_last_error(q.ctx);
        if (m && *m) s->err = std::string("request failed: ") + m;
    }
    q.res.state = code < 0 ? code : GCB_E_DEVICE;
    q.res.t_done = clock_s();
    if (q.resident_key >= 0) {
        // the kept set may be half-updated: drop the mesh
        auto it = s->resident.find(q.resident_key);
        if (it != s->resident.end() && it->second.ctx == q.ctx) {
            gcb_destroy(q.ctx);
            s->resident.erase(it);
        }
    } else if (q.owns_ctx && q.ctx) {
        gcb_destroy(q.ctx);
    }
    q.ctx = nullptr;
}

void release(gcb_server* s, Req& q) {
    if (q.resident_key >= 0) {
        auto it = s->resident.find(q.resident_key);
        if (it != s->resident.end()) {
            it->second.busy = false;
            it->second.last_use = ++s->use_clock;
        }
    } else if (q.owns_ctx && q.ctx) {
        gcb_destroy(q.ctx);
    }
    q.ctx = nullptr;
}

// Copy a finished selection into the request's record (host memory; synchronises the stream).
int fill_record(Req& q) {
    gcb_record* rec = q.r.record;
    if (!rec) return GCB_OK;
    rec->nc = q.res.info.nc;
    rec->iterations = q.res.info.iterations;
    if (rec->cap_support >= q.res.info.nc && (rec->support || rec->weights)) {
        const int rc = gcb_get_support(q.ctx, rec->support, rec->weights, GCB_MEM_HOST);
        if (rc != GCB_OK) return rc;
    }
    if (rec->cap_log > 0 && (rec->log_group || rec->log_node || rec->log_err || rec->log_appended)) {
        const int64_t n = gcb_get_log(q.ctx, rec->log_group, rec->log_node, rec->log_err, rec->log_appended,
                                      rec->cap_log);
        if (n < 0) return (int)n;
    }
    return GCB_OK;
}

int check_request(const gcb_request& r) {
    if (r.nb < 3 || !r.xyz || !r.disp) return GCB_E_INVALID;
    if (r.nv < 0 || (r.nv > 0 && (!r.vol_xyz || !r.out))) return GCB_E_INVALID;
    if ((r.in_dtype != GCB_F32 && r.in_dtype != GCB_F64) || (r.out_dtype != GCB_F32 && r.out_dtype != GCB_F64))
        return GCB_E_INVALID;
    return GCB_OK;
}

// Admission of the queue head: a context (resident mesh, warm start) or a new one.
// Returns false when the head must wait for memory.
bool admit_head(gcb_server* s) {
    const int64_t t = s->queue.front();
    Req& q = s->reqs.at(t);
    const gcb_request& r = q.r;
    const bool cache = (s->flags & GCB_SERVE_CACHE) && r.mesh_key >= 0;
    gcb_params prm = r.params;
    prm.warm_start = 0;
    auto res = cache ? s->resident.find(r.mesh_key) : s->resident.end();
    int rc = GCB_OK;
    if (res != s->resident.end() && !res->second.busy && res->second.nb == r.nb) {
        // resident mesh: same boundary, new displacements
        Resident& m = res->second;
        m.busy = true;
        m.last_use = ++s->use_clock;
        q.ctx = m.ctx;
        q.owns_ctx = false;
        q.resident_key = r.mesh_key;
        q.res.kept = 1;
        const gcb_ctx* c = m.ctx;
        const bool same = c->warm_ok && c->warm_m == prm.m && c->warm_seed == prm.seed &&
                          c->warm_radius == prm.radius && c->warm_n <= prm.nc_max;
        prm.warm_start = same ? 1 : 0;
        q.res.warm = prm.warm_start;
        rc = gcb_set_displacement(q.ctx, r.disp, GCB_MEM_HOST);
    } else {
        const uint64_t est = estimate_bytes(r);
        while (used_bytes(s) + est > s->budget && evict_one(s)) {
        }
        if (used_bytes(s) + est > s->budget && !(s->selecting.empty() && s->deforming.empty())) return false;
        gcb_ctx* c = nullptr;
        rc = gcb_create(&c, s->device, s->stream);
        if (rc == GCB_OK) rc = gcb_set_stream(c, s->stream);
        q.ctx = c;
        q.owns_ctx = true;
        if (rc == GCB_OK) rc = gcb_set_boundary(c, r.nb, r.xyz, r.disp, GCB_MEM_HOST);
        if (rc == GCB_OK && cache && res == s->resident.end()) {
            Resident m;
            m.ctx = c;
            m.nb = r.nb;
            m.busy = true;
            m.last_use = ++s->use_clock;
            s->resident[r.mesh_key] = m;
            q.owns_ctx = false;
            q.resident_key = r.mesh_key;
            q.res.kept = 1;
        }
    }
    s->queue.pop_front();
    q.res.t_admit = clock_s();
    if (rc == GCB_OK) rc = gcb_set_params(q.ctx, &prm);
    if (rc != GCB_OK) {
        fail_request(s, q, rc);
        return true;
    }
    if (s->flags & GCB_SERVE_BATCH) {
        rc = gcb_batch_begin(s->batch, q.ctx);
        if (rc < 0) {
            fail_request(s, q, rc);
            return true;
        }
        q.res.state = kSelecting;
        s->selecting.push_back(t);
        return true;
    }
    // one at a time: the plain path
    rc = gcb_select(q.ctx, &q.res.info);
    if (rc >= 0) {
        const int rr = fill_record(q);
        if (rr < 0) rc = rr;
    }
    if (rc < 0) {
        fail_request(s, q, rc);
        return true;
    }
    if (r.nv > 0) {
        rc = gcb_deform(q.ctx, r.nv, r.vol_xyz, r.in_dtype, r.out, r.out_dtype, GCB_MEM_DEVICE);
        if (rc < 0) {
            fail_request(s, q, rc);
            return true;
        }
    }
    SHIPCHK(s, hipEventCreate(&q.ev));
    SHIPCHK(s, hipEventRecord(q.ev, s->stream));
    q.res.state = kDeforming;
    s->deforming.push_back(t);
    return true;
}

void collect_done(gcb_server* s) {
    std::vector<int64_t> still;
    for (int64_t t : s->deforming) {
        Req& q = s->reqs.at(t);
        const hipError_t e = hipEventQuery(q.ev);
        if (e == hipErrorNotReady) {
            still.push_back(t);
            continue;
        }
        SHIPCHK(s, e);
        float ms = 0.f;
        SHIPCHK(s, hipEventElapsedTime(&ms, s->ev_ref, q.ev));
        q.res.t_done = s->t_ref + 1e-3 * (double)ms;
        q.res.state = kDone;
        (void)hipEventDestroy(q.ev);
        q.ev = nullptr;
        release(s, q);
    }
    s->deforming.swap(still);
}

void step_batch(gcb_server* s, int32_t iterations) {
    if (s->selecting.empty()) return;
    std::vector<gcb_ctx*> ctxs;
    for (int64_t t : s->selecting) ctxs.push_back(s->reqs.at(t).ctx);
    std::vector<int32_t> run(ctxs.size(), 1);
    const int32_t n = gcb_batch_step(s->batch, ctxs.data(), (int32_t)ctxs.size(), iterations, run.data());
    if (n < 0) {
        // a context failed; find it by its own check of the stopped ones below
        for (size_t i = 0; i < ctxs.size(); ++i) run[i] = 0;
    }
    std::vector<int64_t> still, finished;
    for (size_t i = 0; i < ctxs.size(); ++i) {
        if (run[i]) {
            still.push_back(s->selecting[i]);
            continue;
        }
        Req& q = s->reqs.at(s->selecting[i]);
        const int rc = gcb_batch_end(s->batch, q.ctx, &q.res.info);
        if (rc == GCB_E_STATE && n < 0) {
            still.push_back(s->selecting[i]);   // still running; the failing context is another one
            continue;
        }
        const int rr = rc >= 0 ? fill_record(q) : rc;
        if (rr < 0) {
            fail_request(s, q, rr);
            continue;
        }
        finished.push_back(s->selecting[i]);
    }
    s->selecting.swap(still);
    // one volume launch per (input, output) dtype pair over the finished selections
    for (int in_dt = GCB_F32; in_dt <= GCB_F64; ++in_dt)
        for (int out_dt = GCB_F32; out_dt <= GCB_F64; ++out_dt) {
            std::vector<gcb_ctx*> c;
            std::vector<int64_t> nv;
            std::vector<const void*> x;
            std::vector<void*> o;
            std::vector<int64_t> who;
            for (int64_t t : finished) {
                const Req& q = s->reqs.at(t);
                if (q.r.in_dtype != in_dt || q.r.out_dtype != out_dt) continue;
                c.push_back(q.ctx);
                nv.push_back(q.r.nv);
                x.push_back(q.r.vol_xyz);
                o.push_back(q.r.out);
                who.push_back(t);
            }
            for (size_t a = 0; a < c.size(); a += gcb::kMaxBatch) {
                const int32_t cnt = (int32_t)std::min<size_t>(gcb::kMaxBatch, c.size() - a);
                const int rc = gcb_deform_batch(s->batch, c.data() + a, cnt, nv.data() + a, x.data() + a, in_dt,
                                                o.data() + a, out_dt);
                for (int32_t k = 0; k < cnt; ++k) {
                    Req& q = s->reqs.at(who[a + k]);
                    if (rc < 0) {
                        fail_request(s, q, rc);
                        continue;
                    }
                    SHIPCHK(s, hipEventCreate(&q.ev));
                    SHIPCHK(s, hipEventRecord(q.ev, s->stream));
                    q.res.state = kDeforming;
                    s->deforming.push_back(who[a + k]);
                }
            }
        }
}

}  // namespace

extern "C" {

double gcb_server_clock(void) { return clock_s(); }

int gcb_server_create(gcb_server** out, int device, void* hip_stream, uint64_t hbm_budget, int32_t max_active,
                      int32_t flags) {
    if (!out) return GCB_E_INVALID;
    *out = nullptr;
    if (max_active < 1 || max_active > gcb::kMaxBatch || (flags & ~(GCB_SERVE_BATCH | GCB_SERVE_CACHE)))
        return GCB_E_INVALID;
    gcb_server* s = new (std::nothrow) gcb_server();
    if (!s) return GCB_E_NOMEM;
    s->device = device;
    s->stream = static_cast<hipStream_t>(hip_stream);
    s->budget = hbm_budget;
    s->max_active = (flags & GCB_SERVE_BATCH) ? max_active : 1;
    s->flags = flags;
    int rc = gcb_batch_create(&s->batch, device, hip_stream);
    if (rc != GCB_OK) {
        delete s;
        return rc;
    }
    if (hipSetDevice(device) != hipSuccess || hipEventCreate(&s->ev_ref) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess || hipEventRecord(s->ev_ref, s->stream) != hipSuccess ||
        hipEventSynchronize(s->ev_ref) != hipSuccess) {
        gcb_batch_destroy(s->batch);
        if (s->ev_ref) (void)hipEventDestroy(s->ev_ref);
        delete s;
        return GCB_E_DEVICE;
    }
    s->t_ref = clock_s();
    *out = s;
    return GCB_OK;
}

void gcb_server_destroy(gcb_server* s) {
    if (!s) return;
    (void)hipSetDevice(s->device);
    (void)hipStreamSynchronize(s->stream);
    for (auto& kv : s->reqs) {
        Req& q = kv.second;
        if (q.ev) (void)hipEventDestroy(q.ev);
        if (q.owns_ctx && q.ctx) gcb_destroy(q.ctx);
    }
    for (auto& kv : s->resident) gcb_destroy(kv.second.ctx);
    gcb_batch_destroy(s->batch);
    if (s->ev_ref) (void)hipEventDestroy(s->ev_ref);
    delete s;
}

const char* gcb_server_last_error(const gcb_server* s) { return s ? s->err.c_str() : ""; }

int gcb_server_submit(gcb_server* s, const gcb_request* req, int64_t* ticket) {
    return sguard(s, [&] {
        if (!req || !ticket) sfail(s, GCB_E_INVALID, "NULL request or ticket");
        const int rc = check_request(*req);
        if (rc != GCB_OK) sfail(s, rc, "bad request (nb >= 3, host boundary arrays, device volume arrays, dtypes)");
        const int64_t t = s->next_ticket++;
        Req& q = s->reqs[t];
        q.r = *req;
        q.res.state = kQueued;
        q.res.t_arrival = req->t_arrival >= 0.0 ? req->t_arrival : clock_s();
        s->queue.push_back(t);
        *ticket = t;
        return GCB_OK;
    });
}

int gcb_server_progress(gcb_server* s, int32_t iterations, int32_t* in_flight) {
    return sguard(s, [&] {
        if (iterations < 1 || iterations > 4096) sfail(s, GCB_E_INVALID, "iterations must be in [1, 4096]");
        SHIPCHK(s, hipSetDevice(s->device));
        collect_done(s);
        while (!s->queue.empty() && (int)s->selecting.size() < s->max_active) {
            if (!(s->flags & GCB_SERVE_BATCH) && !s->deforming.empty()) {
                // one at a time: the previous request's output completes first
                SHIPCHK(s, hipStreamSynchronize(s->stream));
                collect_done(s);
            }
            if (!admit_head(s)) break;
            if (!(s->flags & GCB_SERVE_BATCH)) break;   // one request per round
        }
        if (s->flags & GCB_SERVE_BATCH) step_batch(s, iterations);
        collect_done(s);
        if (in_flight) *in_flight = (int32_t)(s->queue.size() + s->selecting.size() + s->deforming.size());
        return GCB_OK;
    });
}

int gcb_server_result(const gcb_server* s, int64_t ticket, gcb_result* res) {
    if (!s || !res) return GCB_E_INVALID;
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return GCB_E_INVALID;
    *res = it->second.res;
    return GCB_OK;
}

int gcb_server_forget(gcb_server* s, int64_t ticket) {
    if (!s) return GCB_E_INVALID;
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return GCB_E_INVALID;
    const int32_t st = it->second.res.state;
    if (st != kDone && st >= 0) return GCB_E_STATE;
    s->reqs.erase(it);   // a finished or failed request holds no context and no event any more
    return GCB_OK;
}

int gcb_server_memory(const gcb_server* s, uint64_t* bytes, int32_t* resident) {
    if (!s) return GCB_E_INVALID;
    if (bytes) *bytes = used_bytes(s);
    if (resident) *resident = (int32_t)s->resident.size();
    return GCB_OK;
}

}  // extern "C"
