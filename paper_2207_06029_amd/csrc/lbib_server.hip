// Continuous-batching job server.  Submitted jobs queue in FIFO order; at every tick the server
// retires finished jobs, admits queued jobs while a slot is free and their device bytes fit the
// budget, rebuilds the resident batch when the set changed (continuing jobs keep their exact
// state), and advances every resident job by the same number of steps in shared launches.
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
    lbib_body_desc body{};
    std::vector<double> xyz;
    std::vector<int32_t> tri;
    int64_t steps = 0, done = 0;
    int64_t t_submit = 0, t_admit = 0;
    uint64_t bytes = 0;
    int slot_job = -1;    // index in the resident batch
};

struct SResult {
    lbib_result r{};
    std::vector<double> xyz;
};

// Device bytes a job occupies while resident: both population buffers, the body's windows
// (force 24 B + moments 16 B per window node) and its mesh state.
uint64_t job_bytes(const lbib_lattice_desc& d, int storage, const std::vector<double>& xyz, int nt,
                   bool rigid) {
    const uint64_t n = (uint64_t)d.nx * d.ny * d.nz;
    uint64_t b = 2ull * 19 * n * lbib::storage_bytes(storage) + 4096;
    const size_t nv = xyz.size() / 3;
    if (nv) {
        double c[3] = {0, 0, 0}, r = 0;
        for (size_t v = 0; v < nv; ++v) for (int a = 0; a < 3; ++a) c[a] += xyz[3 * v + a] / nv;
        for (size_t v = 0; v < nv; ++v) {
            double s = 0;
            for (int a = 0; a < 3; ++a) s += (xyz[3 * v + a] - c[a]) * (xyz[3 * v + a] - c[a]);
            r = std::max(r, std::sqrt(s));
        }
        const int dims[3] = {d.nx, d.ny, d.nz};
        int cap[3];
        lbib::window_capacity(dims, rigid, r, cap);
        const uint64_t w = (uint64_t)cap[0] * cap[1] * cap[2];
        b += w * 40 + nv * 8 * 32 + (uint64_t)nt * 8 * 16;
    }
    return b;
}

}  // namespace

struct lbib_server {
    lbib_server_opts opts{};
    hipStream_t stream = nullptr;
    uint64_t next_id = 1;
    std::deque<SJob> queue;
    std::vector<SJob> resident;
    std::deque<SResult> results;
    std::unique_ptr<Batch> batch;
    bool dirty = false;
    uint64_t resident_bytes = 0;
    double node_updates = 0.0;
};

namespace {

// Build a batch holding the resident jobs; jobs that were resident before keep their
// populations (device copy of the current buffer) and body state.
lbib_status rebuild(lbib_server* S) {
    std::unique_ptr<Batch> nb(new Batch());
    std::vector<lbib_lattice_desc> descs;
    std::vector<char> keep;
    for (auto& j : S->resident) {
        descs.push_back(j.lat);
        keep.push_back(j.slot_job >= 0);
    }
    if (descs.empty()) { S->batch.reset(); S->dirty = false; return LBIB_OK; }
    lbib_status st;
    if (S->batch && (st = S->batch->download_body_state())) return st;
    if ((st = nb->create_lattices(descs, S->opts.storage, S->stream, nullptr, 0, &keep))) return st;
    const size_t es = lbib::storage_bytes(S->opts.storage);
    for (size_t k = 0; k < S->resident.size(); ++k) {
        SJob& j = S->resident[k];
        if (j.slot_job >= 0) {
            const Batch& ob = *S->batch;
            const lbib::JobDev& oj = ob.jobs[j.slot_job];
            const void* src = (const char*)(ob.cur_b ? ob.P.popB : ob.P.popA) + oj.pop_off * es;
            void* dst = (char*)(nb->cur_b ? nb->P.popB : nb->P.popA) + nb->jobs[k].pop_off * es;
            if (hipMemcpyAsync(dst, src, 19ull * oj.n * es, hipMemcpyDeviceToDevice, S->stream) != hipSuccess)
                return fail(LBIB_EDEVICE, "state copy failed");
            // the step counter seeding the stochastic narrowing carries over, so the job continues
            // exactly as it would alone
            if ((st = nb->set_step_counter((int)k, (unsigned)j.done))) return st;
            // carry the body
            for (auto& hb : ob.hbodies)
                if (hb.job == j.slot_job) {
                    lbib::HostBody c = hb;
                    c.job = (int)k;
                    nb->hbodies.push_back(c);
                }
        } else if (!j.xyz.empty()) {
            lbib::HostBody hb;
            if ((st = lbib::build_body(j.body, j.xyz.data(), (int)j.xyz.size() / 3, j.tri.data(),
                                       (int)j.tri.size() / 3, hb)))
                return st;
            hb.job = (int)k;
            nb->hbodies.push_back(std::move(hb));
        }
    }
    if ((st = nb->rebuild_bodies())) return st;
    nb->use_graph = S->opts.use_graph != 0;
    for (size_t k = 0; k < S->resident.size(); ++k) S->resident[k].slot_job = (int)k;
    if (S->batch && hipStreamSynchronize(S->stream) != hipSuccess) return fail(LBIB_EDEVICE, "sync failed");
    S->batch = std::move(nb);
    S->dirty = false;
    return LBIB_OK;
}

lbib_status retire(lbib_server* S, size_t k, int status) {
    SJob& j = S->resident[k];
    SResult R;
    if (S->opts.dry_run) {
        R.r.id = j.id; R.r.tag = j.tag; R.r.status = status; R.r.nv = (int32_t)(j.xyz.size() / 3);
        R.r.steps_done = j.done; R.r.t_submit_ns = j.t_submit; R.r.t_admit_ns = j.t_admit;
        R.r.t_finish_ns = now_ns();
        S->results.push_back(std::move(R));
        S->resident_bytes -= j.bytes;
        S->resident.erase(S->resident.begin() + k);
        S->dirty = true;
        return LBIB_OK;
    }
    R.r.id = j.id;
    R.r.tag = j.tag;
    R.r.status = status;
    R.r.nv = (int32_t)(j.xyz.size() / 3);
    R.r.steps_done = j.done;
    R.r.t_submit_ns = j.t_submit;
    R.r.t_admit_ns = j.t_admit;
    Batch& B = *S->batch;
    const int bi = B.body_index(j.slot_job, 0);
    if (bi >= 0) {
        R.xyz.resize(j.xyz.size());
        lbib_status st = B.body_state(bi, R.xyz.data(), nullptr);
        if (!st) st = B.body_forces(bi, nullptr, R.r.F, R.r.M);
        if (st) return st;
    }
    R.r.t_finish_ns = now_ns();
    S->results.push_back(std::move(R));
    S->resident_bytes -= j.bytes;
    S->resident.erase(S->resident.begin() + k);
    S->dirty = true;
    return LBIB_OK;
}

}  // namespace


extern "C" {

lbib_status lbib_server_create(const lbib_server_opts* opts, void* hip_stream, lbib_server** out) {
    if (!opts || !out) return fail(LBIB_EINVAL, "null argument");
    if (opts->max_slots < 1 || opts->steps_per_tick < 1 || opts->hbm_budget_bytes == 0)
        return fail(LBIB_EINVAL, "server needs slots, a budget and steps per tick");
    if (opts->storage < 0 || opts->storage > 2) return fail(LBIB_EINVAL, "unknown storage");
    lbib_server* S = new lbib_server();
    S->opts = *opts;
    S->stream = (hipStream_t)hip_stream;
    *out = S;
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
    j.body = job->body;
    if (job->nv > 0) {
        if (!job->xyz || !job->tri || job->nt <= 0) return fail(LBIB_EINVAL, "mesh pointers missing");
        j.xyz.assign(job->xyz, job->xyz + 3 * (size_t)job->nv);
        j.tri.assign(job->tri, job->tri + 3 * (size_t)job->nt);
        lbib::HostBody hb;  // validate the mesh now so errors surface at submit time
        if ((st = lbib::build_body(j.body, j.xyz.data(), job->nv, j.tri.data(), job->nt, hb))) return st;
    }
    j.steps = job->steps;
    j.tag = job->tag;
    j.bytes = job_bytes(j.lat, S->opts.storage, j.xyz, job->nt, job->body.rigid != 0);
    if (j.bytes > S->opts.hbm_budget_bytes) return fail(LBIB_ENOMEM, "job can never fit the memory budget");
    j.id = S->next_id++;
    j.t_submit = now_ns();
    *id = j.id;
    S->queue.push_back(std::move(j));
    return LBIB_OK;
}

lbib_status lbib_server_tick(lbib_server* S) {
    if (!S) return fail(LBIB_EINVAL, "null server");
    try {
        // admission: FIFO while a slot is free and the job fits the budget
        while (!S->queue.empty() && (int)S->resident.size() < S->opts.max_slots &&
               S->resident_bytes + S->queue.front().bytes <= S->opts.hbm_budget_bytes) {
            SJob j = std::move(S->queue.front());
            S->queue.pop_front();
            j.t_admit = now_ns();
            j.slot_job = -1;
            S->resident_bytes += j.bytes;
            S->resident.push_back(std::move(j));
            S->dirty = true;
        }
        lbib_status st = LBIB_OK;
        if (S->opts.dry_run) {
            if (S->resident.empty()) return LBIB_OK;
            int64_t nstep = S->opts.steps_per_tick;
            for (auto& j : S->resident) nstep = std::min<int64_t>(nstep, j.steps - j.done);
            for (auto& j : S->resident) {
                j.done += nstep;
                S->node_updates += (double)nstep * j.lat.nx * j.lat.ny * j.lat.nz;
            }
            for (size_t k = S->resident.size(); k-- > 0;)
                if (S->resident[k].done >= S->resident[k].steps && (st = retire(S, k, LBIB_OK))) return st;
            return LBIB_OK;
        }
        if (S->dirty && (st = rebuild(S))) return st;
        if (S->resident.empty()) return LBIB_OK;
        // zero-step jobs finish at once
        int64_t nstep = S->opts.steps_per_tick;
        for (auto& j : S->resident) nstep = std::min<int64_t>(nstep, j.steps - j.done);
        if (nstep > 0) {
            if ((st = S->batch->step((int)nstep, true))) return st;
            for (auto& j : S->resident) {
                j.done += nstep;
                S->node_updates += (double)nstep * j.lat.nx * j.lat.ny * j.lat.nz;
            }
        }
        std::vector<int> fl;
        if ((st = S->batch->job_flags(fl))) return st;
        for (size_t k = S->resident.size(); k-- > 0;) {
            const int f = fl[S->resident[k].slot_job];
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
    if (resident_bytes) *resident_bytes = S->resident_bytes;
    if (node_updates) *node_updates = S->node_updates;
    return LBIB_OK;
}

}  // extern "C"
