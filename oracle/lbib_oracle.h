/*
 * FP64 CPU oracle of the D3Q19 BGK lattice-Boltzmann / dynamic immersed-boundary scheme
 * for rigid and deformable capsules (arXiv 2207.06029, Sec. 1).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU implementation.  It is
 * used by the test suite, by the smoke check and by the CPU-baseline leg of the benchmark,
 * and by nothing else.  It shares no source with the GPU path.
 *
 * Conventions
 *   node index      k = x + nx*(y + ny*z)
 *   populations     f[i*N + k], i in the order of the columns of Eq. (e_i)
 *   vectors         u[d*N + k] (structure of arrays)
 *   mesh arrays     xyz[3*v + d], tri[3*t + j] (counter-clockwise seen from outside)
 *   state           f is the post-streaming distribution at time level n (walls applied)
 *   all arithmetic  IEEE double, fixed loop order; results do not depend on thread count.
 */
#ifndef LBIB_ORACLE_H
#define LBIB_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_EUNSTABLE = -4, ORC_EDOMAIN = -7 };
enum { ORC_BC_PERIODIC = 0, ORC_BC_ZOUHE = 1, ORC_BC_BOUNCEBACK = 2 };
/* membrane vertex update: DISPLACEMENT = Eq. verletPos, velocity = displacement of the step;
 * PAPER = the three-stage update of Eqs. verletPos, verletVel, verletPos as printed;
 * KINEMATIC = points advected with the interpolated fluid velocity (kinematic IB, Sec. 2.4) */
enum { ORC_INTEGRATOR_DISPLACEMENT = 0, ORC_INTEGRATOR_PAPER = 1, ORC_INTEGRATOR_KINEMATIC = 2 };

typedef struct {
    int32_t nx, ny, nz, pad;
    double tau;
    int32_t bc[6];             /* faces -x,+x,-y,+y,-z,+z */
    double wall_u[6][3];       /* wall velocity of each face */
    double body_force[3];      /* uniform force density added to f_lb everywhere */
} orc_lattice_desc;

typedef struct {
    int32_t rigid, integrator;
    double ks0, thickness, kb, kv, mass_ratio;
    double gravity[3];
    double mls_rw, mls_alpha, probe_len, shell_h;
} orc_body_desc;

typedef struct orc_lattice orc_lattice;

const char* orc_last_error(void);
void orc_set_threads(int n);

/* --- pointwise pieces of Sec. 1.1 (exposed for the identity checks) --- */
void orc_d3q19(int32_t e[57], double w[19]);
void orc_equilibrium(double rho, const double u[3], double feq[19]);          /* Eq. eqfunc */
void orc_guo_forcing(double tau, const double u[3], const double F[3], double Fi[19]); /* Eq. forcing */
void orc_collide_node(double tau, const double f[19], const double F[3], double fout[19]);
/* Zou-He closure on a face node: axis 0..2, side -1 (low face) or +1 (high face). */
void orc_wall_closure(int axis, int side, const double uw[3], const double F[3], double f[19]);
/* Closure on a node on two or three Zou-He faces: side[a] = -1, +1 or 0 per axis, rho the
 * node's density (taken from the node diagonally inside).  0, or -1 if singular. */
int orc_corner_closure(const int32_t side[3], double rho, const double uw[3], const double F[3],
                       double f[19]);

/* --- lattice --- */
int  orc_lattice_create(const orc_lattice_desc* d, orc_lattice** out);
void orc_lattice_destroy(orc_lattice* L);
int  orc_lattice_init(orc_lattice* L, const double* rho, const double* u);
int  orc_set_populations(orc_lattice* L, const double* f);
int  orc_get_populations(const orc_lattice* L, double* f);
int  orc_get_macros(const orc_lattice* L, double* rho, double* u);
int  orc_step(orc_lattice* L, int nsteps);
int  orc_stream_only(orc_lattice* L, int nsteps);
int64_t orc_step_count(const orc_lattice* L);

/* --- bodies --- */
int orc_body_add(orc_lattice* L, const orc_body_desc* d, const double* xyz, int32_t nv,
                 const int32_t* tri, int32_t nt, int32_t* body_id);
int orc_body_set_velocity(orc_lattice* L, int32_t b, const double* v);
/* Membranes: place the body at rest at xyz (x^n = x^{n-1} = xyz, u_v = 0). */
int orc_body_set_positions(orc_lattice* L, int32_t b, const double* xyz);
int orc_body_get_state(const orc_lattice* L, int32_t b, double* xyz, double* vel);
int orc_body_get_forces(const orc_lattice* L, int32_t b, double* f_vertex, double F[3], double M[3]);
int orc_body_counts(const orc_lattice* L, int32_t b, int32_t* nv, int32_t* nt, int32_t* ne);
int orc_body_topology(const orc_lattice* L, int32_t b, int32_t* edge, int32_t* hinge);
int orc_body_rest(const orc_lattice* L, int32_t b, double* l0, double* ks, double* theta0,
                  double* A0, double scal[4] /* V0, S0, m_v, rigid mass */);
int orc_body_rigid_props(const orc_lattice* L, int32_t b, double X0[3], double* mass, double I[9]);
/* Rigid pose and velocities: centre X, rotation R (row-major, x = X + R x_body), u, omega. */
int orc_body_rigid_state(const orc_lattice* L, int32_t b, double X[3], double R[9], double u[3],
                         double om[3]);

/* --- pieces of one step, evaluated on the current state without advancing it --- */
int orc_membrane_forces(const orc_lattice* L, int32_t b, const double* xyz, double* F, double E[3]);
int orc_mls(const orc_lattice* L, const double x[3], double rw, double alpha, int64_t idx[27],
            double d[81], double phi[27], double grad[81], int32_t* count);
int orc_ib_force(orc_lattice* L, double* flb, double* U, double* Fl);
int orc_body_probe_forces(const orc_lattice* L, int32_t b, double* Fext);
/* The rigid-body part of the structure update (Eqs. linearVelRig, angularVelRig and the pose)
 * with given hydrodynamic totals F, M in place of the probe totals; the fluid is untouched. */
int orc_rigid_advance(orc_lattice* L, int32_t b, const double F[3], const double M[3]);

#ifdef __cplusplus
}
#endif
#endif
