// extern "C" entry points of include/lbib.h for single lattices, batches and kernel timing,
// plus the sweep launch-shape autotuner.
#include "lbib.h"
#include "lbib_runtime.h"

#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <vector>
#include <map>
#include <memory>
#include <sstream>
#include <string>

using lbib::Batch;
using lbib::fail;

namespace {

lbib_status check_handle(const lbib_lattice* lat) {
    if (!lat || !lat->batch) return fail(LBIB_EINVAL, "null lattice handle");
    return LBIB_OK;
}

lbib_status body_of(const lbib_lattice* lat, int32_t body, int* bi) {
    lbib_status st = check_handle(lat);
    if (st) return st;
    *bi = lat->batch->body_index(lat->job, body);
    if (*bi < 0) return fail(LBIB_ENOENT, "no such body");
    return LBIB_OK;
}

template <typename F>
lbib_status guarded(F&& f) {
    try {
        return f();
    } catch (const std::bad_alloc&) {
        return fail(LBIB_ENOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(LBIB_EINVAL, e.what());
    } catch (...) {
        return fail(LBIB_EINVAL, "unexpected exception");
    }
}

}  // namespace

// ---------------------------------------------------------------- autotuner
// Times the collide+stream sweep of a batch for each candidate (block size, nodes per thread)
// on the batch's own data and keeps the fastest.  The candidates compute bitwise identical
// results (every node does the same arithmetic), so only speed differs.  Results are cached in a
// text file keyed by storage and job shapes.
namespace lbib {

static std::string shape_key(const Batch& B) {
    std::map<std::string, int> cnt;
    for (auto& J : B.jobs) cnt[std::to_string(J.nx) + "x" + std::to_string(J.ny) + "x" + std::to_string(J.nz)]++;
    std::ostringstream os;
    os << "s" << B.storage;
    for (auto& kv : cnt) os << ";" << kv.first << "*" << kv.second;
    return os.str();
}

lbib_status autotune(Batch& B, const char* cache) {
    const std::string key = shape_key(B);
    std::map<std::string, SweepShape> table;
    if (cache) {
        // one line per job mix: key, block, nodes per thread, XCD chunk (absent in older
        // caches: chosen by footprint)
        std::ifstream in(cache);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream ls(line);
            std::string k;
            int blk, npt, chunk = -1;
            if (!(ls >> k >> blk >> npt)) continue;
            if (!(ls >> chunk)) chunk = -1;
            table[k] = SweepShape{blk, npt, chunk};
        }
        auto it = table.find(key);
        if (it != table.end()) return B.set_shape(it->second);
    }
    std::vector<SweepShape> cand;
    for (const SweepShape& c : {SweepShape{128, 1, 0}, SweepShape{256, 1, 0}, SweepShape{512, 1, 0},
                                SweepShape{1024, 1, 0}, SweepShape{256, 2, 0}, SweepShape{512, 2, 0},
                                SweepShape{256, 4, 0}}) {
        cand.push_back(c);
        cand.push_back(SweepShape{c.block, c.npt, XCD_CHUNK});
    }
    SweepShape best = B.shape;
    double best_ms = 1e30;
    struct Events {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Events() {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } ev;
    if (hipEventCreate(&ev.e0) != hipSuccess || hipEventCreate(&ev.e1) != hipSuccess)
        return fail(LBIB_EDEVICE, "event create failed");
    for (const SweepShape& c : cand) {
        lbib_status st = B.set_shape(c);
        if (st) return st;
        // sweeps from the current buffer into the other one; the state is not advanced
        for (int w = 0; w < 2; ++w)
            launch_sweep(B.P, B.storage, true, !B.cur_b, (int)B.tiles.size(), c, B.xcd_chunk, B.stream);
        if (hipEventRecord(ev.e0, B.stream) != hipSuccess) return fail(LBIB_EDEVICE, "autotune event record failed");
        const int reps = 8;
        for (int r = 0; r < reps; ++r)
            launch_sweep(B.P, B.storage, true, !B.cur_b, (int)B.tiles.size(), c, B.xcd_chunk, B.stream);
        if (hipEventRecord(ev.e1, B.stream) != hipSuccess) return fail(LBIB_EDEVICE, "autotune event record failed");
        if (hipEventSynchronize(ev.e1) != hipSuccess) return fail(LBIB_EDEVICE, "autotune sync failed");
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev.e0, ev.e1) != hipSuccess) return fail(LBIB_EDEVICE, "autotune timing failed");
        if (ms < best_ms) { best_ms = ms; best = c; }
    }
    if (cache) {
        table[key] = best;
        std::ofstream out(cache);
        for (auto& kv : table)
            out << kv.first << " " << kv.second.block << " " << kv.second.npt << " " << kv.second.xcd_chunk << "\n";
    }
    return B.set_shape(best);
}

}  // namespace lbib

extern "C" {

uint32_t lbib_abi_version(void) { return LBIB_ABI_VERSION; }
const char* lbib_last_error(void) { return lbib::last_error(); }

lbib_status lbib_workspace_bytes(const lbib_lattice_desc* desc, int32_t max_nv, int32_t max_nt, size_t* bytes) {
    if (!desc || !bytes) return fail(LBIB_EINVAL, "null argument");
    lbib_status st = lbib::check_lattice(*desc);
    if (st) return st;
    if (max_nv < 0 || max_nt < 0 || (max_nv > 0) != (max_nt > 0)) return fail(LBIB_EINVAL, "bad mesh size");
    *bytes = lbib::workspace_need(*desc, max_nv, max_nt);
    return LBIB_OK;
}

lbib_status lbib_lattice_create(const lbib_lattice_desc* desc, void* hip_stream, void* workspace,
                                size_t ws_bytes, lbib_lattice** out) {
    return guarded([&]() -> lbib_status {
        if (!desc || !out) return fail(LBIB_EINVAL, "null argument");
        *out = nullptr;
        lbib_status st = lbib::check_lattice(*desc);
        if (st) return st;
        std::unique_ptr<Batch> B(new Batch());
        st = B->create_lattices({*desc}, desc->storage, hip_stream, workspace, ws_bytes);
        if (st) return st;
        lbib_lattice* L = new lbib_lattice();
        L->batch = B.release();
        L->job = 0;
        L->owner = true;
        *out = L;
        return LBIB_OK;
    });
}

lbib_status lbib_lattice_destroy(lbib_lattice* lat) {
    if (!lat) return LBIB_OK;
    if (lat->owner) delete lat->batch;
    if (lat->owner) delete lat;
    return LBIB_OK;
}

lbib_status lbib_lattice_init(lbib_lattice* lat, const double* rho, const double* u) {
    return guarded([&]() -> lbib_status {
        lbib_status st = check_handle(lat);
        if (st) return st;
        Batch& B = *lat->batch;
        if ((st = B.init_job(lat->job, rho, u))) return st;
        int zero = 0;
        if (hipMemcpy(B.P.flags + lat->job, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess)
            return fail(LBIB_EDEVICE, "flag reset failed");
        return LBIB_OK;
    });
}

lbib_status lbib_body_add(lbib_lattice* lat, const lbib_body_desc* desc, const double* xyz, int32_t nv,
                          const int32_t* tri, int32_t nt, int32_t* body_id) {
    return guarded([&]() -> lbib_status {
        lbib_status st = check_handle(lat);
        if (st) return st;
        if (!desc || !xyz || !tri || !body_id) return fail(LBIB_EINVAL, "null argument");
        return lat->batch->add_body(lat->job, *desc, xyz, nv, tri, nt, body_id);
    });
}

lbib_status lbib_body_set_velocity(lbib_lattice* lat, int32_t body, const double* v) {
    return guarded([&]() -> lbib_status {
        int bi;
        lbib_status st = body_of(lat, body, &bi);
        if (st) return st;
        if (!v) return fail(LBIB_EINVAL, "null velocity");
        return lat->batch->body_set_velocity(bi, v);
    });
}

lbib_status lbib_step(lbib_lattice* lat, int32_t nsteps) {
    return guarded([&]() -> lbib_status {
        lbib_status st = check_handle(lat);
        if (st) return st;
        if (!lat->owner) return fail(LBIB_EINVAL, "a job of a batch is stepped through lbib_batch_step");
        return lat->batch->step(nsteps, true);
    });
}

lbib_status lbib_stream_only(lbib_lattice* lat, int32_t nsteps) {
    return guarded([&]() -> lbib_status {
        lbib_status st = check_handle(lat);
        if (st) return st;
        if (!lat->owner) return fail(LBIB_EINVAL, "a job of a batch is stepped through lbib_batch_step");
        return lat->batch->step(nsteps, false);
    });
}

lbib_status lbib_sync(lbib_lattice* lat) {
    return guarded([&]() -> lbib_status {
        lbib_status st = check_handle(lat);
        if (st) return st;
        return lat->batch->check_flags();
    });
}

int64_t lbib_step_count(const lbib_lattice* lat) { return lat && lat->batch ? lat->batch->step_count : -1; }

lbib_status lbib_get_macros(lbib_lattice* lat, double* rho, double* u) {
    return guarded([&]() -> lbib_status {
        lbib_status st = check_handle(lat);
        if (st) return st;
        if ((st = lat->batch->check_flags())) return st;
        return lat->batch->get_macros(lat->job, rho, u);
    });
}

lbib_status lbib_get_populations(lbib_lattice* lat, double* f) {
    return guarded([&]() -> lbib_status {
        lbib_status st = check_handle(lat);
        if (st) return st;
        if (!f) return fail(LBIB_EINVAL, "null argument");
        if ((st = lat->batch->check_flags())) return st;
        return lat->batch->get_populations(lat->job, f);
    });
}

lbib_status lbib_set_populations(lbib_lattice* lat, const double* f) {
    return guarded([&]() -> lbib_status {
        lbib_status st = check_handle(lat);
        if (st) return st;
        if (!f) return fail(LBIB_EINVAL, "null argument");
        return lat->batch->set_populations(lat->job, f);
    });
}

lbib_status lbib_body_get_state(lbib_lattice* lat, int32_t body, double* xyz, double* vel) {
    return guarded([&]() -> lbib_status {
        int bi;
        lbib_status st = body_of(lat, body, &bi);
        if (st) return st;
        if ((st = lat->batch->check_flags())) return st;
        return lat->batch->body_state(bi, xyz, vel);
    });
}

lbib_status lbib_body_get_forces(lbib_lattice* lat, int32_t body, double* f_vertex, double F[3], double M[3]) {
    return guarded([&]() -> lbib_status {
        int bi;
        lbib_status st = body_of(lat, body, &bi);
        if (st) return st;
        if ((st = lat->batch->check_flags())) return st;
        return lat->batch->body_forces(bi, f_vertex, F, M);
    });
}

lbib_status lbib_body_count(const lbib_lattice* lat, int32_t body, int32_t* nv, int32_t* nt) {
    int bi;
    lbib_status st = body_of(lat, body, &bi);
    if (st) return st;
    if (nv) *nv = lat->batch->hbodies[bi].nv;
    if (nt) *nt = lat->batch->hbodies[bi].nt;
    return LBIB_OK;
}

lbib_status lbib_set_timing(lbib_lattice* lat, int32_t enable) {
    lbib_status st = check_handle(lat);
    if (st) return st;
    if (enable < 0) return fail(LBIB_EINVAL, "timing period must be >= 0");
    if (hipStreamSynchronize(lat->batch->stream) != hipSuccess)
        return fail(LBIB_EDEVICE, "stream synchronisation failed");
    lat->batch->clear_events();
    lat->batch->timing = enable != 0;
    lat->batch->timing_period = enable > 0 ? enable : 1;
    lat->batch->sweep_seq = 0;
    return LBIB_OK;
}

lbib_status lbib_kernel_time(lbib_lattice* lat, int32_t kernel, double* total_ms, int64_t* count) {
    return guarded([&]() -> lbib_status {
        lbib_status st = check_handle(lat);
        if (st) return st;
        if (kernel != 0 && kernel != 1) return fail(LBIB_EINVAL, "kernel id must be 0 (sweep) or 1 (step)");
        if (!total_ms || !count) return fail(LBIB_EINVAL, "null argument");
        return lat->batch->kernel_time(kernel, total_ms, count);
    });
}

// ---------------------------------------------------------------- batches
struct lbib_batch {
    Batch* batch = nullptr;
    std::vector<lbib_lattice> views;
};

lbib_status lbib_batch_create(const lbib_job* jobs, int32_t njobs, const lbib_batch_opts* opts,
                              void* hip_stream, lbib_batch** out) {
    return guarded([&]() -> lbib_status {
        if (!jobs || njobs <= 0 || !opts || !out) return fail(LBIB_EINVAL, "bad batch arguments");
        *out = nullptr;
        std::vector<lbib_lattice_desc> descs(njobs);
        for (int j = 0; j < njobs; ++j) {
            descs[j] = jobs[j].lattice;
            descs[j].storage = opts->storage;
            lbib_status st = lbib::check_lattice(descs[j]);
            if (st) return fail(st, "job " + std::to_string(j) + ": " + lbib::last_error());
        }
        std::unique_ptr<Batch> B(new Batch());
        lbib_status st = B->create_lattices(descs, opts->storage, hip_stream, nullptr, 0);
        if (st) return st;
        // bodies: built on the host first, uploaded once
        for (int j = 0; j < njobs; ++j) {
            if (jobs[j].nv <= 0) continue;
            lbib::HostBody hb;
            if ((st = lbib::build_body(jobs[j].body, jobs[j].xyz, jobs[j].nv, jobs[j].tri, jobs[j].nt, hb)))
                return fail(st, "job " + std::to_string(j) + ": " + lbib::last_error());
            hb.job = j;
            hb.local_id = 0;
            B->hbodies.push_back(std::move(hb));
        }
        if ((st = B->rebuild_bodies())) return st;
        B->use_graph = opts->use_graph != 0;
        if (opts->autotune && (st = lbib::autotune(*B, opts->tune_cache))) return st;
        lbib_batch* b = new lbib_batch();
        b->batch = B.release();
        b->views.resize(njobs);
        for (int j = 0; j < njobs; ++j) { b->views[j].batch = b->batch; b->views[j].job = j; b->views[j].owner = false; }
        *out = b;
        return LBIB_OK;
    });
}

lbib_status lbib_batch_destroy(lbib_batch* b) {
    if (!b) return LBIB_OK;
    delete b->batch;
    delete b;
    return LBIB_OK;
}

lbib_status lbib_batch_step(lbib_batch* b, int32_t nsteps) {
    return guarded([&]() -> lbib_status {
        if (!b) return fail(LBIB_EINVAL, "null batch");
        return b->batch->step(nsteps, true);
    });
}

lbib_status lbib_batch_sync(lbib_batch* b) {
    return guarded([&]() -> lbib_status {
        if (!b) return fail(LBIB_EINVAL, "null batch");
        return b->batch->check_flags();
    });
}

lbib_status lbib_batch_lattice(lbib_batch* b, int32_t j, lbib_lattice** lat) {
    if (!b || !lat) return fail(LBIB_EINVAL, "null argument");
    if (j < 0 || j >= (int32_t)b->views.size()) return fail(LBIB_ENOENT, "no such job");
    *lat = &b->views[j];
    return LBIB_OK;
}

lbib_status lbib_batch_launch_shape(const lbib_batch* b, int32_t* block, int32_t* npt) {
    if (!b || !block || !npt) return fail(LBIB_EINVAL, "null argument");
    *block = b->batch->shape.block;
    *npt = b->batch->shape.npt;
    return LBIB_OK;
}

}  // extern "C"
