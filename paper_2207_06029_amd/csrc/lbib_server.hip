// Continuous-batching job server.  Submitted jobs queue in FIFO order.  The server owns one
// slotted batch: every slot's populations, windows, mesh arrays and table entries are sized once,
// at creation, for the slot capacity.  At every tick it retires finished jobs, splices queued
// jobs into free slots (the job's table entries and state are written in place; resident jobs
// are not touched, nothing is reallocated), and advances every resident job by the same number of
// steps in shared launches.
#include "lbib.h"
#include "lbib_runtime.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <memory>
#include <vector>

using lbib::Batch;
using lbib::fail;

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct SJob {
    uint64_t id = 0;
    int64_t tag = 0;
    lbib_lattice_desc lat{};
    bool has_body = false;
    lbib::HostBody hb;   // built and checked at submit
    int64_t steps = 0, done = 0;
    int64_t t_submit = 0, t_admit = 0;
    int slot = -1;
};

struct SResult {
    lbib_result r{};
    std::vector<double> xyz;
};

// Slot capacity of the options (defaults: the largest lattice and mesh of the serving stream,
// 128x64x128 nodes and a level-5 icosphere).
lbib::SlotCaps slot_caps(const lbib_server_opts& o) {
    lbib::SlotCaps c;
    c.nodes = o.slot_nodes > 0 ? o.slot_nodes : 128LL * 64 * 128;
    c.nv = o.slot_vertices > 0 ? o.slot_vertices : 10242;
    c.nt = o.slot_triangles > 0 ? o.slot_triangles : 2 * c.nv - 4;
    return c;
}

}  // namespace

struct lbib_server {
    lbib_server_opts opts{};
    hipStream_t stream = nullptr;
    uint64_t next_id = 1;
    lbib::SlotCaps caps{};
    uint64_t slot_bytes = 0;
    int nslots = 0;
    std::deque<SJob> queue;
    std::vector<SJob> resident;
    std::vector<char> slot_used;
    std::deque<SResult> results;
    std::unique_ptr<Batch> batch;
    double node_updates = 0.0;
};

namespace {

lbib_status retire(lbib_server* S, size_t k, int status) {
    SJob& j = S->resident[k];
    SResult R;
    R.r.id = j.id;
    R.r.tag = j.tag;
    R.r.status = status;
    R.r.nv = j.has_body ? j.hb.nv : 0;
    R.r.steps_done = j.done;
    R.r.t_submit_ns = j.t_submit;
    R.r.t_admit_ns = j.t_admit;
    if (!S->opts.dry_run) {
        Batch& B = *S->batch;
        if (j.has_body) {
            R.xyz.resize(3 * (size_t)j.hb.nv);
            lbib_status st = B.body_state(j.slot, R.xyz.data(), nullptr);
            if (!st) st = B.body_forces(j.slot, nullptr, R.r.F, R.r.M);
            if (st) return st;
        }
        lbib_status st = B.slot_retire(j.slot);
        if (st) return st;
    }
    R.r.t_finish_ns = now_ns();
    S->results.push_back(std::move(R));
    S->slot_used[j.slot] = 0;
    S->resident.erase(S->resident.begin() + k);
    return LBIB_OK;
}

}  // namespace


extern "C" {

lbib_status lbib_server_create(const lbib_server_opts* opts, void* hip_stream, lbib_server** out) {
    if (!opts || !out) return fail(LBIB_EINVAL, "null argument");
    if (opts->max_slots < 1 || opts->steps_per_tick < 1 || opts->hbm_budget_bytes == 0)
        return fail(LBIB_EINVAL, "server needs slots, a budget and steps per tick");
    if (opts->storage < 0 || opts->storage > 2) return fail(LBIB_EINVAL, "unknown storage");
    if (opts->slot_nodes < 0 || opts->slot_vertices < 0 || opts->slot_triangles < 0)
        return fail(LBIB_EINVAL, "negative slot capacity");
    std::unique_ptr<lbib_server> S(new lbib_server());
    S->opts = *opts;
    S->stream = (hipStream_t)hip_stream;
    S->caps = slot_caps(*opts);
    S->slot_bytes = lbib::slot_device_bytes(S->caps, opts->storage);
    S->nslots = (int)std::min<uint64_t>((uint64_t)opts->max_slots, opts->hbm_budget_bytes / S->slot_bytes);
    S->slot_used.assign(S->nslots, 0);
    if (!opts->dry_run && S->nslots > 0) {
        S->batch.reset(new Batch());
        lbib_status st = S->batch->create_slotted(S->nslots, S->caps, opts->storage, hip_stream);
        if (st) return st;
    }
    *out = S.release();
    return LBIB_OK;
}

lbib_status lbib_server_destroy(lbib_server* s) {
    delete s;
    return LBIB_OK;
}

lbib_status lbib_server_submit(lbib_server* S, const lbib_job* job, uint64_t* id) {
    if (!S || !job || !id) return fail(LBIB_EINVAL, "null argument");
    SJob j;
    j.lat = job->lattice;
    j.lat.storage = S->opts.storage;
    lbib_status st = lbib::check_lattice(j.lat);
    if (st) return st;
    if (job->steps < 0) return fail(LBIB_EINVAL, "negative run length");
    if (job->nv > 0) {
        if (!job->xyz || !job->tri || job->nt <= 0) return fail(LBIB_EINVAL, "mesh pointers missing");
        // build and check the body now so errors surface at submit time
        if ((st = lbib::build_body(job->body, job->xyz, job->nv, job->tri, job->nt, j.hb))) return st;
        j.has_body = true;
    }
    if (S->nslots == 0) return fail(LBIB_ENOMEM, "the memory budget holds no slot");
    const long long n = (long long)j.lat.nx * j.lat.ny * j.lat.nz;
    if (n > S->caps.nodes || (j.has_body && (j.hb.nv > S->caps.nv || j.hb.nt > S->caps.nt)))
        return fail(LBIB_ENOMEM, "job exceeds the slot capacity");
    j.steps = job->steps;
    j.tag = job->tag;
    j.id = S->next_id++;
    j.t_submit = now_ns();
    *id = j.id;
    S->queue.push_back(std::move(j));
    return LBIB_OK;
}

lbib_status lbib_server_tick(lbib_server* S) {
    if (!S) return fail(LBIB_EINVAL, "null server");
    try {
        lbib_status st = LBIB_OK;
        // admission: FIFO while a slot is free; the job is spliced into the slot in place
        for (int s = 0; s < S->nslots && !S->queue.empty(); ++s) {
            if (S->slot_used[s]) continue;
            SJob j = std::move(S->queue.front());
            S->queue.pop_front();
            j.slot = s;
            if (!S->opts.dry_run &&
                (st = S->batch->slot_admit(s, j.lat, j.has_body ? &j.hb : nullptr)))
                return st;
            j.t_admit = now_ns();
            S->slot_used[s] = 1;
            S->resident.push_back(std::move(j));
        }
        if (S->resident.empty()) return LBIB_OK;
        // every resident job advances by the same count, never past a run length (zero-step
        // jobs finish at once)
        int64_t nstep = S->opts.steps_per_tick;
        for (auto& j : S->resident) nstep = std::min<int64_t>(nstep, j.steps - j.done);
        if (nstep > 0) {
            if (!S->opts.dry_run && (st = S->batch->step((int)nstep, true))) return st;
            for (auto& j : S->resident) {
                j.done += nstep;
                S->node_updates += (double)nstep * j.lat.nx * j.lat.ny * j.lat.nz;
            }
        }
        std::vector<int> fl(S->nslots, 0);
        if (!S->opts.dry_run && (st = S->batch->job_flags(fl))) return st;
        for (size_t k = S->resident.size(); k-- > 0;) {
            const int f = fl[S->resident[k].slot];
            if (f)
                st = retire(S, k, (f & lbib::FLAG_NONFINITE) ? LBIB_EUNSTABLE : LBIB_EDOMAIN);
            else if (S->resident[k].done >= S->resident[k].steps)
                st = retire(S, k, LBIB_OK);
            if (st) return st;
        }
        return LBIB_OK;
    } catch (const std::bad_alloc&) {
        return fail(LBIB_ENOMEM, "host allocation failed");
    }
}

lbib_status lbib_server_poll(lbib_server* S, lbib_result* out, int32_t cap, int32_t* n) {
    if (!S || !n || (cap > 0 && !out)) return fail(LBIB_EINVAL, "null argument");
    int32_t k = 0;
    while (k < cap && !S->results.empty()) {
        SResult& R = S->results.front();
        double* dst = out[k].xyz;
        out[k] = R.r;
        out[k].xyz = dst;
        if (dst && !R.xyz.empty()) std::memcpy(dst, R.xyz.data(), sizeof(double) * R.xyz.size());
        S->results.pop_front();
        ++k;
    }
    *n = k;
    return LBIB_OK;
}

lbib_status lbib_server_stats(const lbib_server* S, int32_t* queued, int32_t* resident,
                              uint64_t* resident_bytes, double* node_updates) {
    if (!S) return fail(LBIB_EINVAL, "null server");
    if (queued) *queued = (int32_t)S->queue.size();
    if (resident) *resident = (int32_t)S->resident.size();
    if (resident_bytes) *resident_bytes = (uint64_t)S->resident.size() * S->slot_bytes;
    if (node_updates) *node_updates = S->node_updates;
    return LBIB_OK;
}

lbib_status lbib_server_info(const lbib_server* S, int32_t* slots, uint64_t* slot_bytes,
                             uint64_t* device_bytes) {
    if (!S) return fail(LBIB_EINVAL, "null server");
    if (slots) *slots = S->nslots;
    if (slot_bytes) *slot_bytes = S->slot_bytes;
    if (device_bytes) *device_bytes = S->batch ? S->batch->device_bytes() : 0;
    return LBIB_OK;
}

}  // extern "C"
