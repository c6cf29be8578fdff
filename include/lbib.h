/*
 * lbib — D3Q19 BGK lattice-Boltzmann / dynamic immersed-boundary solver for rigid and
 * deformable capsules on AMD Instinct MI355X (gfx950).  C ABI of liblbib.so.
 *
 * The method is the one of arXiv 2207.06029, Sec. 1:
 *   fluid       D3Q19 BGK with Guo forcing, Eqs. (e_i), (evoleq), (eqfunc), (forcing);
 *               Zou-He known-velocity walls (Sec. 1.1) or halfway bounce-back;
 *   coupling    moving-least-squares transfer between lattice and triangle centroids,
 *               Eqs. (uLag), (l2norm), (intKernel); direct forcing F = (U_b - U)/dt and
 *               spreading Eq. (bodyforce) (Sec. 1.2);
 *   structure   spring / bending / volume network, Eqs. (strainFor), (bendFor), (volFor);
 *               probe stresses, Eqs. (hydroForP), (hydroForNu); vertex Newton/Verlet,
 *               Eqs. (newtonSoft), (verletPos), (verletVel); rigid bodies by
 *               Eqs. (linearVelRig), (angularVelRig) (Sec. 1.3).
 *
 * Conventions (all entry points)
 *   - Every call returns lbib_status; LBIB_OK = 0, errors are negative.  lbib_last_error()
 *     returns a thread-local message for the last failing call on that thread.  No call
 *     aborts or throws across the ABI.
 *   - Lattice units: dx = dt = 1, c_s^2 = 1/3, nu = (tau - 1/2)/3, reference density 1.
 *   - Node index k = x + nx*(y + ny*z).  Host population arrays are double f[i*N + k] with i
 *     in the column order of Eq. (e_i); host vector fields are double u[d*N + k].
 *   - Mesh arrays: xyz[3*v + d] (double), tri[3*t + j] (int32), triangles counter-clockwise
 *     seen from outside.  Markers are the triangle centroids.
 *   - Host arrays are owned by the caller and only read or written during the call.
 *     Device memory is owned by the library, or carved from a caller workspace.
 *   - Device work is enqueued on the hipStream_t given at creation (NULL = default stream).
 *     Stepping calls are asynchronous; getters, lbib_sync and destroy synchronise that
 *     stream and report deferred device errors (LBIB_EDEVICE), instability (LBIB_EUNSTABLE)
 *     and supports that left the fluid domain (LBIB_EDOMAIN).
 *   - A handle must be used by one host thread at a time.
 */
#ifndef LBIB_H
#define LBIB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBIB_ABI_VERSION 2u

typedef enum {
    LBIB_OK = 0,
    LBIB_EINVAL = -1,    /* bad argument, descriptor or mesh */
    LBIB_ENOMEM = -2,    /* device allocation, workspace or memory budget exceeded */
    LBIB_EDEVICE = -3,   /* HIP runtime error; message from hipGetErrorString */
    LBIB_EUNSTABLE = -4, /* non-finite density, position or rigid state, or a density outside
                            (0.05, 8) after streaming, detected */
    LBIB_EBUSY = -5,     /* server has no free slot / job still running */
    LBIB_ENOENT = -6,    /* no such body, job or result */
    LBIB_EDOMAIN = -7    /* an MLS support or probe left the fluid domain, or a body outgrew
                            the lattice window reserved for it */
} lbib_status;

/* Face boundary kinds.  Faces are ordered -x,+x,-y,+y,-z,+z.  Both faces of an axis are
 * periodic or both are walls.  Zou-He walls (Sec. 1.1) sit on the first/last node of their
 * axis (wet nodes), which needs at least 3 nodes.  On one axis they form a channel: the two
 * other axes periodic, any wall velocity.  On two or three axes (a square duct, the closed
 * lid-driven cavity of Sec. 2.1) every wall must be Zou-He and move tangentially; edge and
 * corner nodes then take the wall velocity zero along their wall normals and the mean of their
 * faces' velocities along the other axes, and a closure that keeps their mass balanced through
 * the walls and sets their momentum to rho u_w - F/2 (the paper leaves edges and corners open).
 * Halfway bounce-back walls sit half a spacing outside the first/last node; moving bounce-back
 * walls on one axis only.  Other combinations fail with LBIB_EINVAL. */
typedef enum { LBIB_BC_PERIODIC = 0, LBIB_BC_ZOUHE_VELOCITY = 1, LBIB_BC_BOUNCEBACK = 2 } lbib_bc;

/* Population storage.  All forms store the deviation g_i = f_i - w_i from the lattice
 * weights and collide in FP32.  FP16/BF16 keep subnormals; the step's stores narrow with
 * stochastic rounding (dither offsets from a counter-based hash of node index and step, so a
 * job's results are reproducible and the same alone or in a batch), initialisation and the
 * setters with round-to-nearest-even.  FP16 holds g_i * 2^12 (an exact power-of-two scale that keeps small deviations
 * in the normal range) and is the reduced-precision form: it stays within 1e-3 (relative L2 of
 * the velocity) of the FP64 scheme.  BF16 holds g_i; its 8 significand bits do NOT meet that
 * bound (about 2e-2 on a sheared box after 300 steps) and it is kept for bandwidth studies
 * only. */
typedef enum { LBIB_STORE_F32 = 0, LBIB_STORE_F16 = 1, LBIB_STORE_BF16 = 2 } lbib_storage;

/* Membrane vertex update.  DISPLACEMENT: position by Eq. (verletPos) with the interpolated
 * fluid velocity as tentative velocity, vertex velocity = displacement of the step.
 * PAPER: the printed three-stage verletPos / verletVel / verletPos sequence.
 * KINEMATIC: the kinematic immersed boundary the paper contrasts with the dynamic one
 * (Sec. 2.4): every vertex is advected with the interpolated fluid velocity, x += u0; membrane
 * forces are still evaluated and reported but do not move the vertices. */
typedef enum { LBIB_INTEGRATOR_DISPLACEMENT = 0, LBIB_INTEGRATOR_PAPER = 1,
               LBIB_INTEGRATOR_KINEMATIC = 2 } lbib_integrator;

typedef struct {
    int32_t nx, ny, nz;
    int32_t storage;          /* lbib_storage */
    double tau;               /* BGK relaxation time, > 1/2 (Eq. evoleq) */
    int32_t bc[6];            /* lbib_bc per face */
    double wall_u[6][3];      /* wall velocity per face */
    double body_force[3];     /* uniform force density added to f_lb at every node */
} lbib_lattice_desc;

typedef struct {
    int32_t rigid;            /* 0 = elastic membrane, 1 = rigid body */
    int32_t integrator;       /* lbib_integrator (membranes) */
    double ks0;               /* global spring constant k_{s,0} (Sec. 1.3, network model) */
    double thickness;         /* membrane thickness T (spring constants and mass) */
    double kb;                /* bending constant k_b */
    double kv;                /* volume penalty constant k_v (Eq. volFor) */
    double mass_ratio;        /* solid/fluid density ratio; > 0 */
    double gravity[3];        /* rigid bodies only: net weight (m - rho_f V) g */
    double mls_rw;            /* MLS support radius r_w (1.3 in Sec. 1.2); below 1.5 */
    double mls_alpha;         /* MLS weight width alpha (0.3 in Eq. intKernel) */
    double probe_len;         /* probe distance (1.2 in Sec. 1.3); at most 2.5 */
    double shell_h;           /* marker thickness h in c_l = A_l h / dx^3 */
} lbib_body_desc;

typedef struct lbib_lattice lbib_lattice;
typedef struct lbib_batch lbib_batch;
typedef struct lbib_server lbib_server;

uint32_t lbib_abi_version(void);
const char* lbib_last_error(void);

/* ---------------------------------------------------------------- single lattice */

/* Device bytes needed by one lattice of this descriptor plus one body of up to max_nv
 * vertices / max_nt triangles (0, 0 for no body) whose vertices have at most 12 incident
 * triangles each: the exact size of the buffers lbib_lattice_create and lbib_body_add carve
 * from a workspace, with the force window sized for the whole lattice.  A lattice created in
 * such a workspace calls no hipMalloc afterwards: setters and getters stage their transfers in
 * the population buffer that the next step overwrites.  Errors: EINVAL for a bad descriptor or
 * mesh size. */
lbib_status lbib_workspace_bytes(const lbib_lattice_desc* desc, int32_t max_nv, int32_t max_nt,
                                 size_t* bytes);

/* Create a lattice initialised at rest (rho = 1, u = 0) with the walls applied.
 * hip_stream: hipStream_t to enqueue on (NULL = default stream).  workspace: device memory
 * of ws_bytes the library carves its buffers from (must stay valid until destroy), or NULL
 * to let the library allocate.  Errors: EINVAL (descriptor: tau <= 1/2, dims < 1, face rules
 * above, unknown storage), ENOMEM, EDEVICE. */
lbib_status lbib_lattice_create(const lbib_lattice_desc* desc, void* hip_stream, void* workspace,
                                size_t ws_bytes, lbib_lattice** out);
lbib_status lbib_lattice_destroy(lbib_lattice* lat);

/* Set populations to the equilibrium Eq. (eqfunc) of rho[N] and u[3N] (NULL = 1 and 0),
 * then apply the wall closure; resets the step counter.  Synchronous. */
lbib_status lbib_lattice_init(lbib_lattice* lat, const double* rho, const double* u);

/* Add a closed, consistently oriented triangulated body (Sec. 1.2, Fig. IB).  Rest lengths,
 * dihedral angles, areas, volume and masses are taken from xyz.  Errors: EINVAL (mesh not a
 * closed 2-manifold, inward winding, bad parameters, gravity on a membrane), EDOMAIN (support
 * leaves the fluid domain), ENOMEM.  Synchronous. */
lbib_status lbib_body_add(lbib_lattice* lat, const lbib_body_desc* desc, const double* xyz,
                          int32_t nv, const int32_t* tri, int32_t nt, int32_t* body_id);

/* Membranes: v[3nv] vertex velocities, previous positions set to x - v.  Rigid bodies: v[6] =
 * (u, omega), previous velocities set equal.  Synchronous. */
lbib_status lbib_body_set_velocity(lbib_lattice* lat, int32_t body, const double* v);

/* Advance nsteps time steps (Sec. 1, one step = IB forcing, collide+stream, structure
 * update).  Asynchronous. */
lbib_status lbib_step(lbib_lattice* lat, int32_t nsteps);

/* Advance nsteps pure streaming steps (no collision, no bodies).  Asynchronous. */
lbib_status lbib_stream_only(lbib_lattice* lat, int32_t nsteps);

/* Wait for queued work; report deferred errors. */
lbib_status lbib_sync(lbib_lattice* lat);
int64_t lbib_step_count(const lbib_lattice* lat);

/* rho[N] and u*[3N] = sum f e / rho (force-free velocity) of the current post-streaming state. */
lbib_status lbib_get_macros(lbib_lattice* lat, double* rho, double* u);
/* Allocation-free lbib_get_macros, for callers that cannot allocate device memory (loops
 * that must not call hipMalloc, harnesses that forbid it).  Same outputs, bit for bit, as
 * lbib_get_macros: rho[N] and u*[3N] in host memory (either may be NULL), after the same
 * synchronisation and deferred-error report.  The moments are staged in a fixed device array of
 * 4 * LBIB_NOALLOC_MAX_NODES doubles (32 MiB) that the library holds on every GPU it runs on
 * until the process ends; the call allocates neither device nor host memory.  The lattice's
 * device must be current.  Calls on one GPU share its array: calls that overlapped would race
 * on it, so the library serialises them per device, and the array keeps the last call's
 * contents (every call overwrites the entries it reads).  Errors: EINVAL (null handle, more than
 * LBIB_NOALLOC_MAX_NODES nodes, another device current), EDEVICE, EUNSTABLE, EDOMAIN. */
#define LBIB_NOALLOC_MAX_NODES 1048576
lbib_status lbib_get_macros_noalloc(lbib_lattice* lat, double* rho, double* u);
/* Post-streaming populations f[19N] at the current time level, widened to double. */
lbib_status lbib_get_populations(lbib_lattice* lat, double* f);
/* Replace the post-streaming populations (narrowed to the storage form), then apply the wall
 * closure.  Synchronous. */
lbib_status lbib_set_populations(lbib_lattice* lat, const double* f);

/* Vertex positions xyz[3nv] and velocities vel[3nv] (either may be NULL). */
lbib_status lbib_body_get_state(lbib_lattice* lat, int32_t body, double* xyz, double* vel);
/* Last total vertex force f_vertex[3nv] (may be NULL) and FP64 totals of the hydrodynamic
 * force F[3] and torque M[3] (about the body centre) of the last step. */
lbib_status lbib_body_get_forces(lbib_lattice* lat, int32_t body, double* f_vertex, double F[3],
                                 double M[3]);
lbib_status lbib_body_count(const lbib_lattice* lat, int32_t body, int32_t* nv, int32_t* nt);

/* Kernel timing.  enable = 0 turns it off; enable = n >= 1 stamps start/end events from the
 * dispatch packet of every n-th launch of the collide+stream sweep (kernel 0; n = 1 times
 * every launch, a larger n samples the launches evenly and keeps the events' own cost out of
 * the other steps) and brackets each lbib_step call with events on the lattice's stream
 * (kernel 1, count = steps).  Timing turns graph replay off.  Enable before stepping;
 * lbib_kernel_time synchronises and returns the summed milliseconds and the count of timed
 * launches since the last enable.  Negative enable and kernel ids other than 0 and 1 give
 * LBIB_EINVAL. */
lbib_status lbib_set_timing(lbib_lattice* lat, int32_t enable);
lbib_status lbib_kernel_time(lbib_lattice* lat, int32_t kernel, double* total_ms, int64_t* count);

/* ---------------------------------------------------------------- batching */

typedef struct {
    lbib_lattice_desc lattice;
    lbib_body_desc body;      /* ignored when nv == 0 */
    const double* xyz;
    const int32_t* tri;
    int32_t nv, nt;
    int64_t steps;            /* run length used by the server */
    int64_t tag;              /* caller's label, returned in results */
} lbib_job;

typedef struct {
    int32_t storage;          /* lbib_storage shared by every job of the batch */
    int32_t autotune;         /* 1: time sweep launch shapes on first step and keep the best */
    const char* tune_cache;   /* JSON file read/updated by the autotuner (NULL = none) */
    int32_t use_graph;        /* 1: capture steps in a hipGraph and replay it */
    int32_t pad;
} lbib_batch_opts;

/* Many independent lattices (each with at most one body) advanced together: every kernel of
 * a step covers all jobs in one launch.  Each job's arithmetic does not depend on the other
 * jobs, so a job's results are bitwise the same alone or in any batch.  Errors: EINVAL,
 * ENOMEM, EDEVICE. */
lbib_status lbib_batch_create(const lbib_job* jobs, int32_t njobs, const lbib_batch_opts* opts,
                              void* hip_stream, lbib_batch** out);
lbib_status lbib_batch_destroy(lbib_batch* b);
lbib_status lbib_batch_step(lbib_batch* b, int32_t nsteps);
lbib_status lbib_batch_sync(lbib_batch* b);
/* Borrowed handle of job j for the single-lattice getters (valid until the batch dies). */
lbib_status lbib_batch_lattice(lbib_batch* b, int32_t j, lbib_lattice** lat);
/* Sweep launch shape chosen for the batch (block size, nodes per thread). */
lbib_status lbib_batch_launch_shape(const lbib_batch* b, int32_t* block, int32_t* nodes_per_thread);

/* ---------------------------------------------------------------- serving */

typedef struct {
    uint64_t hbm_budget_bytes;   /* device memory the slots may occupy */
    int32_t max_slots;           /* jobs resident at once, at most */
    int32_t steps_per_tick;      /* steps every resident job advances per tick */
    int32_t storage;             /* lbib_storage of every job */
    int32_t use_graph;           /* ignored: the server launches eagerly over its live tables */
    int32_t dry_run;             /* 1: schedule only (admission, ticks, retirement) without any
                                    device work; results carry no state.  For policy tests. */
    int32_t pad;
    int64_t slot_nodes;          /* lattice nodes a slot holds; 0: 128*64*128 */
    int32_t slot_vertices;       /* mesh vertices a slot holds; 0: 10242 (a level-5 icosphere) */
    int32_t slot_triangles;      /* mesh triangles a slot holds; 0: 2 slot_vertices - 4 */
} lbib_server_opts;

typedef struct {
    uint64_t id;
    int64_t tag;
    int32_t status;              /* lbib_status of the job */
    int32_t nv;
    int64_t steps_done;
    int64_t t_submit_ns, t_admit_ns, t_finish_ns;   /* steady-clock timestamps */
    double F[3], M[3];           /* final hydrodynamic force and torque */
    double* xyz;                 /* caller buffer of 3*nv doubles for final positions, or NULL */
} lbib_result;

/* Continuous-batching server (the serving pattern of the scope table: admission, splice at a
 * tick, retirement).  At creation the server sizes min(max_slots, hbm_budget_bytes / slot
 * bytes) slots, each holding any job up to the slot capacity (populations, windows, mesh arrays
 * and table entries), and allocates nothing afterwards.  Submitted jobs wait in FIFO order; at a
 * tick each queued job is spliced into a free slot (its table entries and state written in
 * place, resident jobs untouched) at rest with step counter 0; resident jobs advance together
 * in one launch per kernel; finished jobs retire and free their slot.  A job's results are
 * bitwise those of the same job run alone.  Errors: EINVAL, ENOMEM (the budget holds no slot,
 * or the job exceeds the slot capacity), EDEVICE. */
lbib_status lbib_server_create(const lbib_server_opts* opts, void* hip_stream, lbib_server** out);
lbib_status lbib_server_destroy(lbib_server* s);
/* Queue a job (copies its mesh); never blocks.  t_submit is taken now. */
lbib_status lbib_server_submit(lbib_server* s, const lbib_job* job, uint64_t* id);
/* Admit, run steps_per_tick steps of every resident job, retire finished jobs. */
lbib_status lbib_server_tick(lbib_server* s);
/* Copy up to cap finished results (oldest first) into out; *n receives the count.  The xyz
 * pointer of each out[i] must be set by the caller (or NULL). */
lbib_status lbib_server_poll(lbib_server* s, lbib_result* out, int32_t cap, int32_t* n);
/* Queue length, resident jobs, device bytes of the occupied slots, lattice node updates done so
 * far. */
lbib_status lbib_server_stats(const lbib_server* s, int32_t* queued, int32_t* resident,
                              uint64_t* resident_bytes, double* node_updates);
/* Slot count, device bytes per slot, and device bytes the server has allocated (constant after
 * creation; 0 in dry-run mode).  Any output may be NULL. */
lbib_status lbib_server_info(const lbib_server* s, int32_t* slots, uint64_t* slot_bytes,
                             uint64_t* device_bytes);

#ifdef __cplusplus
}
#endif
#endif /* LBIB_H */
