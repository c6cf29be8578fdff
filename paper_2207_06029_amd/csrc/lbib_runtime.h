// Host-side types of the runtime: device arena, host copy of a body, and the Batch that owns
// all device pools of a set of lattices.
#pragma once

#include "lbib.h"
#include "lbib_internal.h"

#include <string>
#include <utility>
#include <vector>

namespace lbib {

lbib_status fail(lbib_status code, const std::string& msg);
// Same, with a message of static storage: records it without allocating.
lbib_status fail_static(lbib_status code, const char* msg);
const char* last_error();
lbib_status check_lattice(const lbib_lattice_desc& d);
size_t storage_bytes(int storage);
// vertex valence (incident triangles) the workspace estimate budgets for
constexpr int WS_MAX_VALENCE = 12;
size_t workspace_need(const lbib_lattice_desc& d, long long nv, long long nt);
// Force-window capacity per axis for a body of bounding radius rbound about its vertex mean.
void window_capacity(const int dims[3], bool rigid, double rbound, int cap[3]);
// Window-moments blocks of such a body (its B.nblk_w).
long long window_blocks(const int dims[3], bool rigid, double rbound);
// Window-moments blocks for a window of capn nodes.  A rigid body's window stays at its
// capacity (the box only moves), so it gets one 256-thread block per 256 nodes, a node per thread.
// A membrane gets one block per WIN_NODES_PER_BLOCK nodes of the window it usually spans (2.5
// times its rest extent per axis), about fifteen times the volume of its current window, so each
// thread still has about one node of it; the blocks stride over larger windows.
constexpr int WIN_NODES_PER_BLOCK_RIGID = 256;
inline long long win_blocks(long long capn, bool rigid) {
    const long long per = rigid ? WIN_NODES_PER_BLOCK_RIGID : WIN_NODES_PER_BLOCK;
    return capn > per ? (capn + per - 1) / per : 1;
}

// Device memory: a caller workspace carved by a bump pointer, or hipMalloc'd blocks.
struct Arena {
    void* base = nullptr;
    size_t cap = 0, used = 0, total = 0;
    std::vector<void*> owned;
    lbib_status alloc(size_t bytes, void** out);
    void release_from(size_t mark_used, size_t mark_owned);
    ~Arena();
};

struct HostBody {
    lbib_body_desc desc{};
    int job = 0, local_id = 0;
    int nv = 0, nt = 0, ne = 0;
    std::vector<double> x, xprev, uv, fv, xb;
    std::vector<int> tri, edge, hinge;
    std::vector<double> l0, ks, theta0;
    std::vector<int> vt_ptr, vt_list, vh_ptr, vh_list;   // incident triangles / hinge roles (CSR)
    double V0 = 0, S0 = 0, mv = 0, mass = 0, rbound = 0;
    double X0[3] = {0, 0, 0};
    double Ib[9] = {0};
    bool has_state = false;   // state below holds device values to restore after a rebuild
    BodyState state{};
    WinDesc fdesc{};
};

lbib_status build_body(const lbib_body_desc& d, const double* xyz, int nv, const int* tri, int nt,
                       HostBody& hb);
void body_record(const HostBody& h, const JobDev& J, BodyDev& B);
void incidence_lists(const HostBody& h, int wt, int wh, std::vector<int>& vtl, std::vector<int>& vhl);

// steps per captured graph (even: the population buffers swap once per step)
constexpr int GRAPH_STEPS = 16;

// Capacity of one slot of a slotted batch: every job admitted to the slot must fit it.
struct SlotCaps {
    long long nodes = 0;   // lattice nodes
    int nv = 0, nt = 0;    // mesh vertices and triangles
};
// incidence-list widths a slot holds (vertex valence up to WS_MAX_VALENCE)
constexpr int SLOT_VT_W = WS_MAX_VALENCE;
constexpr int SLOT_VH_W = 2 * WS_MAX_VALENCE;
uint64_t slot_device_bytes(const SlotCaps& c, int storage);

struct Batch {
    hipStream_t stream = nullptr;
    int device = -1;           // HIP device current when the batch was created
    int storage = 0;
    Arena arena;
    size_t mark_used = 0, mark_owned = 0;
    std::vector<lbib_lattice_desc> ldesc;
    std::vector<JobDev> jobs;
    std::vector<int4> tiles;       // per sweep tile: job, coordinates of its first node
    int4* d_tiles = nullptr;       // from the arena, tile_cap entries
    size_t tile_cap = 0;
    double* d_totals = nullptr;    // 6 doubles: membrane force/torque totals on their way out
    JobDev* d_jobs = nullptr;
    BodyDev* d_bodies = nullptr;
    long long pop_elems = 0;
    std::vector<HostBody> hbodies;
    std::vector<BodyDev> host_bodies;
    int nbodies = 0;
    int nblk_c = 0, nblk_e = 0, nblk_t = 0, nblk_v = 0, nblk_u = 0, nblk_w = 0;
    bool any_rigid = false, any_volume = false;   // bodies needing the per-body fold launches
    Pools P{};
    bool cur_b = false;        // buffer holding the latest post-collision state
    bool primed = false;       // moment windows hold the moments of the current state
    long long step_count = 0;
    SweepShape shape{256, 1, -1};
    int xcd_chunk = 0;        // effective XCD chunk of the current shape and footprint
    bool use_graph = false;
    bool graph_valid = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t capture_stream = nullptr;
    bool timing = false;
    int timing_period = 1;               // events on every timing_period-th sweep launch
    long long sweep_seq = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> sweep_events, step_events;
    std::vector<hipEvent_t> event_pool;   // created once, reused across timing windows
    size_t event_next = 0;
    long long step_event_steps = 0;
    lbib_status next_event(hipEvent_t* e);

    void job_from_desc(const lbib_lattice_desc& d, JobDev& J);
    lbib_status create_lattices(const std::vector<lbib_lattice_desc>& descs, int storage,
                                void* stream, void* ws, size_t ws_bytes,
                                const std::vector<char>* skip_init = nullptr);
    lbib_status retile();
    lbib_status set_shape(SweepShape s);
    lbib_status rebuild_bodies();
    lbib_status download_body_state();
    lbib_status add_body(int job, const lbib_body_desc& d, const double* xyz, int nv,
                         const int* tri, int nt, int* id);
    int body_index(int job, int local) const;
    void* spare(int job) const;
    // step counter seeding the job's stochastic narrowing (both buffer slots)
    lbib_status set_step_counter(int job, unsigned value);
    lbib_status init_job(int job, const double* rho, const double* u);
    lbib_status set_populations(int job, const double* f);
    lbib_status get_macros(int job, double* rho, double* u);
    lbib_status get_populations(int job, double* f);
    lbib_status check_flags();
    lbib_status job_flags(std::vector<int>& fl);
    lbib_status prime();
    lbib_status enqueue_step(bool collide);
    lbib_status step(int nsteps, bool collide);
    lbib_status capture_graph();
    lbib_status kernel_time(int kernel, double* ms, int64_t* count);
    void clear_events();
    lbib_status body_state(int bi, double* xyz, double* vel);
    lbib_status body_forces(int bi, double* fv, double* F, double* M);
    lbib_status body_set_velocity(int bi, const double* v);
    size_t device_bytes() const;

    // Slotted batches (the server).  Every pool, table and window is sized once for nslots
    // slots of capacity caps; jobs are spliced into a slot and out again in place: their job,
    // tile and block table entries are rewritten, nothing is reallocated or copied between
    // slots.  Steps launch eagerly over the live tables.
    bool slotted = false;
    SlotCaps caps{};
    std::vector<char> slot_live;
    int tiles_slot = 0;              // per-slot capacities: sweep tiles, blocks of each launch
    int bc_slot = 0, be_slot = 0, bt_slot = 0, bu_slot = 0, bv_slot = 0, bw_slot = 0, red_slot = 0;
    long long ne_slot = 0, win_slot = 0;
    lbib_status create_slotted(int nslots, const SlotCaps& c, int storage, void* stream);
    // Splice a job into free slot s (hb: its body, or null), at rest, step counter 0.
    lbib_status slot_admit(int s, const lbib_lattice_desc& d, const HostBody* hb);
    lbib_status slot_retire(int s);
    lbib_status slot_tables();
    ~Batch();
};

}  // namespace lbib

// Handles handed out through the C ABI.
struct lbib_lattice {
    lbib::Batch* batch = nullptr;
    int job = 0;
    bool owner = false;
};
