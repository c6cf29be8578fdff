// Internal device-side data of liblbib: job/body tables, window descriptors, kernel
// argument blocks and the launch functions each translation unit provides.
//
// Every kernel walks a device job table, so one lattice, a batch of lattices and the
// server's resident set all run through the same launches.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbib {

constexpr int Q = 19;
// Fixed-point scale of the spread body force: contributions are rounded to multiples of 2^-40
// and summed as 64-bit integers, so the sum does not depend on the order of the atomics.
constexpr double FIX_SCALE = 1099511627776.0;  // 2^40
constexpr double FIX_INV = 1.0 / 1099511627776.0;
constexpr int WIN_MARGIN = 4;    // nodes around a body's bounding box (probe + support + slack)
constexpr int IB_BLOCK = 64;      // threads per block of the marker kernels: one wave
// lanes that evaluate one MLS point (four stencil nodes each), MLS points per block, and
// triangles per probe block (two points, the +/- probes, per triangle)
constexpr int MLS_GROUP = 8;
constexpr int MLS_PER_BLOCK = IB_BLOCK / MLS_GROUP;
constexpr int TRI_PER_BLOCK = MLS_PER_BLOCK / 2;
// the vertex kernel gathers each vertex's incident forces with 16 lanes (one DPP row), 16
// vertices per block (the centroid blocks fold one box per vertex block into the force window)
constexpr int VERT_GROUP = 16;
constexpr int VERT_BLOCK = 256;
constexpr int VERT_PER_BLOCK = VERT_BLOCK / VERT_GROUP;
constexpr int MAX_RED_BLOCKS = 65536;
// window-moments blocks of a membrane: one 256-thread block per this many nodes of the window it
// usually spans (rigid bodies: one per 256 nodes, see win_blocks)
constexpr int WIN_NODES_PER_BLOCK = 2048;

// error flag bits (per job)
constexpr int FLAG_DOMAIN = 1;     // a support or probe reached a wall node / left the domain
constexpr int FLAG_WINDOW = 2;     // a body outgrew its reserved window
constexpr int FLAG_NONFINITE = 4;  // non-finite or runaway density / position / rigid state

// ---------------------------------------------------------------- D3Q19 (Sec. 1.1, Eq. e_i)
__host__ __device__ constexpr int cx(int i) {
    return (i == 1 || (i >= 7 && i <= 10)) ? 1 : ((i == 2 || (i >= 11 && i <= 14)) ? -1 : 0);
}
__host__ __device__ constexpr int cy(int i) {
    return (i == 3 || i == 7 || i == 11 || i == 15 || i == 16) ? 1
         : ((i == 4 || i == 8 || i == 12 || i == 17 || i == 18) ? -1 : 0);
}
__host__ __device__ constexpr int cz(int i) {
    return (i == 5 || i == 9 || i == 13 || i == 15 || i == 17) ? 1
         : ((i == 6 || i == 10 || i == 14 || i == 16 || i == 18) ? -1 : 0);
}
__host__ __device__ constexpr int ce(int i, int a) { return a == 0 ? cx(i) : (a == 1 ? cy(i) : cz(i)); }
// weights after Eq. (eqfunc): 1/3 rest, 1/18 axis, 1/36 diagonal
__host__ __device__ constexpr double wq(int i) {
    return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}
__host__ __device__ constexpr int opp(int i) {
    switch (i) {
        case 0: return 0;   case 1: return 2;   case 2: return 1;   case 3: return 4;
        case 4: return 3;   case 5: return 6;   case 6: return 5;   case 7: return 12;
        case 8: return 11;  case 9: return 14;  case 10: return 13; case 11: return 8;
        case 12: return 7;  case 13: return 10; case 14: return 9;  case 15: return 18;
        case 16: return 17; case 17: return 16; default: return 15;
    }
}
constexpr bool table_ok() {
    for (int i = 0; i < Q; ++i) {
        for (int a = 0; a < 3; ++a)
            if (ce(opp(i), a) != -ce(i, a)) return false;
        int s = (cx(i) != 0) + (cy(i) != 0) + (cz(i) != 0);
        if ((s == 0) != (i == 0) || (s == 1) != (i >= 1 && i <= 6) || (s == 2) != (i >= 7)) return false;
    }
    return true;
}
static_assert(table_ok(), "D3Q19 tables inconsistent");

// ---------------------------------------------------------------- tables
struct JobDev {
    int nx, ny, nz, storage;
    long long n;          // nodes
    long long pop_off;    // element offset of this job's populations in the pool
    int tile0, ntiles;    // sweep tiles of this job
    float omega;          // 1 / tau
    float guo;            // 1 - 1/(2 tau)
    float nu;             // (tau - 1/2) / 3
    int zh_axes;          // axes carrying Zou-He walls (more than one: edge and corner closure)
    int bc[6];
    float wall_u[6][3];
    float G[3];           // uniform body force density
    int body0, nbodies;   // bodies living in this lattice
    // v / nx and v / ny as multiply-high by these for v < 2^16 (ceil(2^32 / n), exact while
    // v (2^32 mod' n) < 2^32, i.e. for dimensions below 2^15); 0 for larger dimensions
    unsigned mx, my;
};

struct WinDesc {
    int o[3];  // origin node (0 <= o < n along periodic axes)
    int w[3];  // extent
};

// A window is usable when 0 <= o < n and 1 <= w <= min(n, cap) on every axis, and on walled
// axes o + w <= n.  Kernels that walk a window check this first.
__host__ __device__ inline bool win_valid(const WinDesc& d, const int dims[3], const int cap[3],
                                          const int bc[6]) {
    for (int a = 0; a < 3; ++a) {
        if (d.o[a] < 0 || d.o[a] >= dims[a] || d.w[a] < 1 || d.w[a] > dims[a] || d.w[a] > cap[a])
            return false;
        if (bc[2 * a] != 0 && d.o[a] + d.w[a] > dims[a]) return false;
    }
    return true;
}

struct BodyDev {
    int job, rigid, integrator, nv;
    int nt, ne, pad0, pad1;
    long long v0, t0, e0;       // offsets into the vertex, triangle and edge pools
    long long win_off;          // offset of the body's windows in the window pools (nodes)
    int win_cap[3];             // reserved window extent per axis
    int red_slot;               // offset of this body's block partials
    // incident triangles and hinge roles per vertex, padded to a fixed width per body:
    // entry j of vertex v at list[off + v * w + j], -1 past the vertex's own count
    long long vt_off, vh_off;
    int vt_w, vh_w;
    // first block of this body in the centroid / edge / triangle / vertex grids, block counts
    int blk_c0, nblk_c, blk_e0, nblk_e, blk_t0, nblk_t, blk_v0, nblk_v, blk_w0, nblk_w;
    int blk_u0, nblk_u;   // vertex-velocity blocks of the probe launch
    int vbox0;            // first of the body's nblk_v integer boxes in the vertex-box pool
    double kb, kv, mv, V0, mass;
    double rw, alpha, probe, shell_h;
    double rw2;                 // r_w^2: support test on squared distances
    float wq;                   // 1 / (r_w alpha)^2: weight W = exp(-wq |d|^2)
    double gravity[3];
    double Ib[9];               // rigid inertia in the rest frame (about the centroid)
};

// per-body mutable scalars (device)
struct BodyState {
    double V;          // enclosed volume at x^n (membranes with a volume penalty)
    double F[3], M[3]; // rigid bodies: hydrodynamic force / torque totals of the last step
    // rigid body
    double X[3], R[9], u[3], u1[3], om[3], om1[3];
    int pad[4];
};

// All device pools of one batch.  Kernels take this by value.
struct Pools {
    void* popA;
    void* popB;
    const JobDev* jobs;
    const int4* tiles;       // per sweep tile: job, coordinates (x, y, z) of its first node
    const BodyDev* bodies;
    const int* blk_body_c;   // block -> body for the centroid kernel (triangle blocks)
    const int* blk_body_e;   // block -> body for the edge blocks of the centroid kernel
    const int* blk_body_t;
    const int* blk_body_v;   // block -> body for the vertex kernel
    const int* blk_body_u;   // block -> body for the vertex-velocity blocks of the probe kernel
    const int* blk_body_w;   // block -> body for the window-moments kernel
    double* x;               // [3 nv] positions x^n (all bodies concatenated)
    double* xprev;           // [3 nv] x^{n-1}
    double* uv;              // [3 nv] vertex velocity u_v^n
    double* fv;              // [3 nv] last total vertex force
    double* u0v;             // [3 nv] fluid velocity at each vertex from f^{n+1} (MLS)
    const double* xb;        // [3 nv] rigid rest-frame coordinates
    const int* tri;          // [3 nt] (vertex indices local to the body)
    const int* edge;         // [2 ne]
    const int* hinge;        // [4 ne] x1,x2 (edge, as in triangle 1), x3, x4
    const double* l0;        // [ne]
    const double* ks;        // [ne]
    const double* theta0;    // [ne]
    const int* vt_list;      // [nv * vt_w per body] incident triangles (padded, -1)
    const int* vh_list;      // [nv * vh_w per body] incident hinges: 4*hinge + role (padded, -1)
    double* tgeo;            // [6 nt] centroid and area-weighted normal (x1-x0)x(x2-x0) at x^n
    double* fext;            // [3 nt] hydrodynamic force per triangle
    double* fvol;            // [3 nt] volume-penalty force per vertex of each triangle
    double* fedge;           // [15 ne] spring force on x1, bending force on x1..x4 per hinge
    long long* fwin;         // force windows, 3 components x window nodes (fixed point)
    float4* mwin;            // moment windows (rho - 1, u*)
    WinDesc* fdesc;          // force-window layout of the current step, per body
    WinDesc* mdesc;          // layout of the moment window, per body
    BodyState* bstate;
    double* partial;         // block partial sums (16 doubles per block)
    int* vbox;               // [6 per vertex block] integer box (floor min, ceil max) of x^{n+1}
    int* flags;              // per job
    unsigned* sr_ctr;        // per job, two slots (buffer A, B): step counter seeding the
                             // stochastic narrowing of reduced-precision storage
    int pop32;               // every job's populations span less than 4 GiB (32-bit offsets)
    int solo_job;            // job of the only body when the batch holds one body, else -1
    int one_lattice;         // 1: the batch holds one lattice (job 0, every sweep tile its own)
    BodyDev solo_body;       // that body's record (valid when solo_job >= 0)
};

// Body of a marker-kernel block, its record and its job.  The SOLO instantiations serve a batch
// with one body: its index, record and job come with the kernel arguments, so the first data
// loads need no round trip for the block table, the body record or the job record (each one
// beyond the L2 that the sweep has just streamed through).
template <bool SOLO>
__device__ __forceinline__ int block_body(const Pools& P, const int* table, int blk) {
    return SOLO ? 0 : table[blk];
}
template <bool SOLO>
__device__ __forceinline__ const BodyDev& body_of(const Pools& P, int b) {
    if constexpr (SOLO) return P.solo_body;
    else return P.bodies[b];
}
template <bool SOLO>
__device__ __forceinline__ const JobDev& body_job(const Pools& P, const BodyDev& B) {
    return P.jobs[SOLO ? P.solo_job : B.job];
}

// ---------------------------------------------------------------- launchers
struct SweepShape {
    int block;          // threads per block
    int npt;            // nodes per thread (block-strided)
    int xcd_chunk;      // tiles an XCD takes per turn (0: dispatch order; -1: chosen by footprint)
};
// Chunked XCD order pays while the two population buffers stay in the Infinity Cache (256 MB);
// beyond it, dispatch order keeps all XCDs streaming the same region.
constexpr int XCD_CHUNK = 8;
// nodes of the smallest sweep tile (block size x nodes per thread) of any launch shape
constexpr int MIN_TILE_NODES = 128;
constexpr long long XCD_CHUNK_MAX_BYTES = 192LL << 20;

// lbib_lattice.hip
// With ev0/ev1 set, the two events are stamped by the sweep's own dispatch packet (its start
// and end on the device), not by separate stream commands around it.
void launch_sweep(const Pools& P, int storage, bool collide, bool a_to_b, int ntiles,
                  SweepShape shape, int xcd_chunk, hipStream_t s, hipEvent_t ev0 = nullptr,
                  hipEvent_t ev1 = nullptr);
// nblk_w: total window blocks (each body gets blocks in proportion to its window capacity)
void launch_window_moments(const Pools& P, int storage, bool from_b, int nblk_w, hipStream_t s);
void launch_macros(const Pools& P, int storage, bool from_b, int job, long long n, float* out4,
                   hipStream_t s);
// rho[n] then u*[3n] in double (the host layout of lbib_get_macros), written to out[4n]
void launch_macros_f64(const Pools& P, int storage, bool from_b, int job, long long n, double* out,
                       hipStream_t s);
// Population `plane` of the post-streaming state, widened to double, into out[n].
void launch_get_pop_plane(const Pools& P, int storage, bool from_b, int job, long long n, int plane,
                          double* out, hipStream_t s);
// Set population `plane` of the post-streaming state from f[n] (double).
void launch_set_pop_plane(const Pools& P, int storage, bool to_b, int job, long long n, int plane,
                          const double* f, hipStream_t s);
// Equilibrium of rho[n], u[3n] (device; NULL: 1 and 0) as the post-streaming state.
void launch_init_eq(const Pools& P, int storage, bool to_b, int job, long long n, const double* rho,
                    const double* u, hipStream_t s);

// lbib_ib.hip
// fold: the centroid blocks derive this step's force window from the vertex-block boxes
// themselves; otherwise launch_windows after the vertex kernel has published it.
void launch_centroids(const Pools& P, int nblk_tri, int nblk_edge, bool fold, hipStream_t s);
void launch_windows(const Pools& P, int nbodies, hipStream_t s);
// bodies from which the force windows are folded once per body by a kernel of their own
constexpr int WINDOW_KERNEL_MIN_BODIES = 2;
void launch_triangles(const Pools& P, int nblk_tri, int nblk_vel, hipStream_t s);
// mode 0: volumes of membranes with a volume penalty; mode 1: rigid totals and pose update
void launch_fold_bodies(const Pools& P, int nbodies, int mode, hipStream_t s);
void launch_vertices(const Pools& P, int nblocks, hipStream_t s);
void launch_body_totals(const Pools& P, int body, double* out6, hipStream_t s);

}  // namespace lbib
