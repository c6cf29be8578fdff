/*
 * FP64 CPU oracle of the D3Q19 BGK lattice-Boltzmann / dynamic immersed-boundary scheme
 * (arXiv 2207.06029, Sec. 1).  TEST INFRASTRUCTURE ONLY: it checks the GPU implementation
 * and is called only from the test suite, the smoke check and the benchmark's CPU-baseline
 * leg.  Plain C, IEEE double, fixed loop orders.  OpenMP (when enabled) only splits loops
 * whose iterations write disjoint outputs, so results are independent of the thread count.
 *
 * One time step n -> n+1 (weak coupling, Sec. 1.3; force lag, end of Sec. 1.2):
 *   1. moments rho, u* = sum f e / rho of the post-streaming state f^n           (Sec. 1.1)
 *   2. membrane geometry at x^n: centroids (= Lagrangian markers), normals, areas (Sec. 1.2)
 *   3. MLS shape functions at every centroid                    (Eqs. uLag, l2norm, intKernel)
 *   4. interpolated marker velocity U*, desired velocity U_b, force F_l = U_b - U*  (Sec. 1.2)
 *   5. spreading f_lb(x_k) = G + sum_l c_l phi_k^l F_l, c_l = A_l h                 (Eq. bodyforce)
 *   6. BGK collision with Guo forcing                           (Eqs. evoleq, eqfunc, forcing)
 *   7. streaming with periodic wrap, Zou-He velocity walls or halfway bounce-back     (Sec. 1.1)
 *   8. moments of f^{n+1}
 *   9. structure: internal forces at x^n (Eqs. strainFor, bendFor, volFor), probe stresses
 *      from the n+1 fields (Eqs. hydroForP, hydroForNu), then Verlet (Eqs. verletPos,
 *      verletVel) for membranes, or total force/torque and the velocity updates of
 *      Eqs. linearVelRig / angularVelRig for rigid bodies.
 *
 * Readings of passages the paper leaves open (each one is listed in the design notes):
 *   - the fluid velocity handed to the immersed boundary and the probes is the force-free
 *     u* = sum f e / rho; the half-force shifted u enters only the collision.
 *   - c_l = A_l * h / dx^3 with h = dx = 1 and the current triangle area, which makes the
 *     total Eulerian force equal the total Lagrangian force (partition of unity).
 *   - the MLS support is every node within Euclidean distance r_w of the point (W = 0 beyond).
 *   - bending force = exact negative gradient of k_b [1 - cos(theta - theta0)], theta the
 *     signed dihedral angle between adjacent outward normals; this energy gives the printed
 *     beta_b prefactor and equals Eq. bendPot to leading order.
 *   - volume penalty acts restoringly: F_t = +k_v (1 - V/V0) n_t A_t, one third per vertex.
 *   - Zou-He momentum target rho u_w - G/2 (G = uniform body force), so the Guo velocity at
 *     a wall node equals the wall velocity; immersed-boundary support may not reach wall nodes.
 *   - the state at every time level (including the initial one) satisfies the wall closure.
 *   - Zou-He walls on several axes (square duct, closed box): at an edge or a corner the
 *     populations streamed in through any of the node's walls are rebuilt by bounce-back of the
 *     non-equilibrium part (links buried in the wall: equilibrium), then corrected by a weighted
 *     least-squares term to the node's mass and momentum target.  The node's density balances
 *     its mass through its walls; its wall velocity is zero along its wall normals and the mean
 *     of its faces' velocities along the other axes.  Such walls must all be Zou-He and move
 *     tangentially.
 *   - halfway bounce-back walls sit half a spacing outside the first/last node, with the
 *     moving-wall term 2 w_i rho0 (e_i . u_w) / c_s^2, rho0 = 1.
 *   - rigid bodies: mass m = ratio * V0 (fluid density 1), net gravity (m - V0) g, inertia of
 *     the solid polyhedron rotated with the body, no gyroscopic term.
 *   - start-up of the multistep formulas from rest: x^{-1} = x^0, u^{-1} = 0.
 *   - kinematic IB (Sec. 2.4 contrasts it with the dynamic scheme; it differs only in how the
 *     points are displaced): x^{n+1} = x^n + u0 dt with u0 the MLS fluid velocity at the vertex
 *     from f^{n+1}, vertex velocity u0.  Forcing and the membrane force evaluation are unchanged;
 *     the membrane forces no longer move the vertices.
 *   - membrane vertex update (default): position from Eq. verletPos with the interpolated fluid
 *     velocity, vertex velocity = the displacement of that step.  The printed three-stage
 *     update (verletPos, verletVel, verletPos again) makes the displacement of a step
 *     -1/2 of the previous one plus 3/2 u0 + 5/4 a: a period-two mode, which the
 *     immersed-boundary feedback excites in a sheared capsule (the vertex velocity then flips
 *     sign every step and grows to several times the flow speed).  It stays available as
 *     ORC_INTEGRATOR_PAPER.
 */
#include "lbib_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19
#define MAXB 16

/* Columns of Eq. (e_i). */
static const int E[Q][3] = {
    {0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {1, -1, 0},  {1, 0, 1},  {1, 0, -1}, {-1, 1, 0}, {-1, -1, 0}, {-1, 0, 1},
    {-1, 0, -1}, {0, 1, 1},  {0, 1, -1}, {0, -1, 1}, {0, -1, -1}};

static const double CS2 = 1.0 / 3.0;

/* Weights of Eq. (eqfunc): 1/3 for the rest velocity, 1/18 for the six axis directions,
 * 1/36 for the twelve diagonals. */
static double weight(int i) {
    int s = abs(E[i][0]) + abs(E[i][1]) + abs(E[i][2]);
    return s == 0 ? 1.0 / 3.0 : (s == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}

static int opposite(int i) {
    for (int j = 0; j < Q; ++j)
        if (E[j][0] == -E[i][0] && E[j][1] == -E[i][1] && E[j][2] == -E[i][2]) return j;
    return -1;
}

static int find_dir(int ex, int ey, int ez) {
    for (int j = 0; j < Q; ++j)
        if (E[j][0] == ex && E[j][1] == ey && E[j][2] == ez) return j;
    return -1;
}

static char g_err[512];
static void set_err(const char* m) { snprintf(g_err, sizeof g_err, "%s", m); }
const char* orc_last_error(void) { return g_err; }

static int g_threads = 1;
void orc_set_threads(int n) { g_threads = n < 1 ? 1 : n; }

/* ------------------------------------------------------------------ Sec. 1.1 pointwise */

void orc_d3q19(int32_t e[57], double w[19]) {
    for (int i = 0; i < Q; ++i) {
        for (int d = 0; d < 3; ++d) e[3 * i + d] = E[i][d];
        w[i] = weight(i);
    }
}

/* Eq. (eqfunc). */
void orc_equilibrium(double rho, const double u[3], double feq[19]) {
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        double eu = E[i][0] * u[0] + E[i][1] * u[1] + E[i][2] * u[2];
        feq[i] = weight(i) * rho * (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* Eq. (forcing). */
void orc_guo_forcing(double tau, const double u[3], const double F[3], double Fi[19]) {
    for (int i = 0; i < Q; ++i) {
        double eu = E[i][0] * u[0] + E[i][1] * u[1] + E[i][2] * u[2];
        double s = 0.0;
        for (int d = 0; d < 3; ++d)
            s += ((E[i][d] - u[d]) / CS2 + eu * E[i][d] / (CS2 * CS2)) * F[d];
        Fi[i] = (1.0 - 1.0 / (2.0 * tau)) * weight(i) * s;
    }
}

/* BGK collision of Eq. (evoleq) with dt = 1; u carries the half-force shift of Sec. 1.1. */
void orc_collide_node(double tau, const double f[19], const double F[3], double fout[19]) {
    double rho = 0.0, j[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
        rho += f[i];
        for (int d = 0; d < 3; ++d) j[d] += f[i] * E[i][d];
    }
    double u[3];
    for (int d = 0; d < 3; ++d) u[d] = (j[d] + 0.5 * F[d]) / rho;
    double feq[Q], Fi[Q];
    orc_equilibrium(rho, u, feq);
    orc_guo_forcing(tau, u, F, Fi);
    for (int i = 0; i < Q; ++i) fout[i] = f[i] - (f[i] - feq[i]) / tau + Fi[i];
}

/*
 * Zou-He known-velocity closure on a wall node (Sec. 1.1, Zou & He).  The wall normal points
 * into the fluid along +axis on the low face (side -1) and along -axis on the high face
 * (side +1); the five populations with e_axis = s (s = -side) are unknown.  Density from mass
 * and normal momentum, normal population by bounce-back of the non-equilibrium part plus the
 * normal momentum, diagonal populations carry the transverse momentum corrections N_b.
 * Momentum target m = rho u_w - F/2, so that (sum f e + F/2)/rho = u_w.
 */
void orc_wall_closure(int axis, int side, const double uw[3], const double F[3], double f[19]) {
    const int s = -side;
    double sum0 = 0.0, summ = 0.0;
    for (int i = 0; i < Q; ++i) {
        if (E[i][axis] == 0) sum0 += f[i];
        else if (E[i][axis] == -s) summ += f[i];
    }
    double rho = (sum0 + 2.0 * summ - s * 0.5 * F[axis]) / (1.0 - s * uw[axis]);
    double m[3];
    for (int d = 0; d < 3; ++d) m[d] = rho * uw[d] - 0.5 * F[d];
    int en[3] = {0, 0, 0};
    en[axis] = s;
    int i_n = find_dir(en[0], en[1], en[2]);
    f[i_n] = f[opposite(i_n)] + s * m[axis] / 3.0;
    for (int b = 0; b < 3; ++b) {
        if (b == axis) continue;
        double nb = 0.0;
        for (int i = 0; i < Q; ++i)
            if (E[i][axis] == 0) nb += f[i] * E[i][b];
        nb = 0.5 * nb - m[b] / 3.0;
        for (int t = -1; t <= 1; t += 2) {
            int e[3] = {0, 0, 0};
            e[axis] = s;
            e[b] = t;
            int i = find_dir(e[0], e[1], e[2]);
            f[i] = f[opposite(i)] + (s * m[axis] + t * m[b]) / 6.0 - t * nb;
        }
    }
}

static int spd_inverse4(const double A[16], double Ai[16]);

/*
 * Known-velocity closure on a node that lies on two or three Zou-He faces (an edge or a corner
 * of the box).  The paper names Zou-He walls (Sec. 1.1) without saying how edges and corners are
 * closed; the reading taken here:
 *   - unknown populations are those streamed in through any of the node's walls;
 *   - an unknown whose opposite is known takes that opposite plus the equilibrium difference,
 *     2 w_i (e_i . m) / c_s^2 (bounce-back of the non-equilibrium part, as on a face);
 *     an unknown whose opposite is unknown too (a link buried in the wall) takes f_i^eq(rho, u_w);
 *   - the unknowns are then corrected by w_i (lambda_0 + lambda . e_i), lambda chosen so that the
 *     node carries exactly the mass rho and the momentum m = rho u_w - F/2 (the weighted
 *     least-squares correction over the unknowns; on a face it would reproduce the transverse
 *     terms of the face closure).
 * The density cannot follow from the known populations on an edge or a corner; the caller
 * passes it in (the lattice balances the node's mass, see close_edges).
 * side[a] = -1 low face of axis a, +1 high face, 0 not on a wall of that axis.
 */
int orc_corner_closure(const int32_t side[3], double rho, const double uw[3], const double F[3],
                       double f[19]) {
    int unk[Q];
    for (int i = 0; i < Q; ++i) {
        unk[i] = 0;
        for (int a = 0; a < 3; ++a)
            if (side[a] != 0 && E[i][a] == -side[a]) unk[i] = 1;
    }
    double m[3], feq[Q];
    for (int d = 0; d < 3; ++d) m[d] = rho * uw[d] - 0.5 * F[d];
    orc_equilibrium(rho, uw, feq);
    for (int i = 0; i < Q; ++i) {
        if (!unk[i]) continue;
        const int j = opposite(i);
        if (unk[j]) f[i] = feq[i];
        else f[i] = f[j] + 2.0 * weight(i) * (E[i][0] * m[0] + E[i][1] * m[1] + E[i][2] * m[2]) / CS2;
    }
    double r[4] = {rho, m[0], m[1], m[2]};
    double A[16] = {0};
    for (int i = 0; i < Q; ++i) {
        r[0] -= f[i];
        for (int d = 0; d < 3; ++d) r[1 + d] -= f[i] * E[i][d];
        if (!unk[i]) continue;
        const double p[4] = {1.0, (double)E[i][0], (double)E[i][1], (double)E[i][2]};
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) A[4 * a + b] += weight(i) * p[a] * p[b];
    }
    double Ai[16];
    if (spd_inverse4(A, Ai) != 0) return -1;
    double lam[4] = {0, 0, 0, 0};
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) lam[a] += Ai[4 * a + b] * r[b];
    for (int i = 0; i < Q; ++i)
        if (unk[i]) f[i] += weight(i) * (lam[0] + lam[1] * E[i][0] + lam[2] * E[i][1] + lam[3] * E[i][2]);
    return 0;
}

/* ------------------------------------------------------------------ data */

typedef struct {
    orc_body_desc d;
    int nv, nt, ne;
    int *tri, *edge, *hinge; /* tri[3nt], edge[2ne], hinge[4ne] = x1,x2 (edge), x3 (opp in t1), x4 */
    double *l0, *ks, *theta0, *A0;
    double V0, S0, mv;
    double *x, *xprev, *uv;  /* deformable state at x^n, x^{n-1}, u_v^n */
    double *Fv;              /* last total vertex force */
    double Ftot[3], Mtot[3];
    /* rigid */
    double X[3], R[9], ur[3], ur1[3], om[3], om1[3], mass, Ib[9], *xb;
} body_t;

struct orc_lattice {
    int nx, ny, nz;
    long N;
    double tau;
    int bc[6];
    int zh_axes;          /* axes carrying Zou-He walls */
    double wall_u[6][3];
    double G[3];
    double *f, *fs, *rho, *u, *flb;
    int64_t step;
    int nb;
    body_t* b[MAXB];
};

static long node(const orc_lattice* L, int x, int y, int z) {
    return (long)x + (long)L->nx * ((long)y + (long)L->ny * (long)z);
}

static int dim(const orc_lattice* L, int a) { return a == 0 ? L->nx : (a == 1 ? L->ny : L->nz); }

/* ------------------------------------------------------------------ lattice */

int orc_lattice_create(const orc_lattice_desc* d, orc_lattice** out) {
    *out = NULL;
    if (d->nx < 1 || d->ny < 1 || d->nz < 1) { set_err("bad dims"); return ORC_EINVAL; }
    if (!(d->tau > 0.5)) { set_err("tau must exceed 1/2"); return ORC_EINVAL; }
    int zh_axis = -1, zh_axes = 0;
    for (int a = 0; a < 3; ++a) {
        int lo = d->bc[2 * a], hi = d->bc[2 * a + 1];
        if (lo < 0 || lo > 2 || hi < 0 || hi > 2) { set_err("bad bc"); return ORC_EINVAL; }
        if ((lo == ORC_BC_PERIODIC) != (hi == ORC_BC_PERIODIC)) {
            set_err("a periodic face needs a periodic partner"); return ORC_EINVAL;
        }
        if (lo == ORC_BC_ZOUHE || hi == ORC_BC_ZOUHE) {
            zh_axis = a;
            ++zh_axes;
            int n = a == 0 ? d->nx : (a == 1 ? d->ny : d->nz);
            if (n < 3) { set_err("Zou-He axis needs 3 nodes"); return ORC_EINVAL; }
        }
    }
    /* Zou-He walls on one axis: the other axes are periodic (channel).  On several axes (duct,
     * closed box): every wall is Zou-He and moves only tangentially, so that the velocity of a
     * node shared by two faces is well defined (edge and corner closure). */
    if (zh_axes == 1)
        for (int a = 0; a < 3; ++a)
            if (a != zh_axis && d->bc[2 * a] != ORC_BC_PERIODIC) {
                set_err("Zou-He walls on one axis need periodic tangential axes"); return ORC_EINVAL;
            }
    if (zh_axes > 1)
        for (int f = 0; f < 6; ++f) {
            if (d->bc[f] == ORC_BC_PERIODIC) continue;
            if (d->bc[f] != ORC_BC_ZOUHE) {
                set_err("Zou-He walls on several axes: every wall must be Zou-He"); return ORC_EINVAL;
            }
            if (d->wall_u[f][f / 2] != 0.0) {
                set_err("Zou-He walls on several axes: wall velocities must be tangential"); return ORC_EINVAL;
            }
        }
    int moving = 0;
    for (int a = 0; a < 3; ++a)
        for (int s = 0; s < 2; ++s)
            if (d->bc[2 * a + s] == ORC_BC_BOUNCEBACK &&
                (d->wall_u[2 * a + s][0] != 0 || d->wall_u[2 * a + s][1] != 0 ||
                 d->wall_u[2 * a + s][2] != 0)) { moving |= 1 << a; }
    if (moving && (moving & (moving - 1))) {
        set_err("moving bounce-back walls on one axis only"); return ORC_EINVAL;
    }
    orc_lattice* L = (orc_lattice*)calloc(1, sizeof *L);
    L->nx = d->nx; L->ny = d->ny; L->nz = d->nz;
    L->N = (long)d->nx * d->ny * d->nz;
    L->tau = d->tau;
    L->zh_axes = zh_axes;
    memcpy(L->bc, d->bc, sizeof L->bc);
    memcpy(L->wall_u, d->wall_u, sizeof L->wall_u);
    memcpy(L->G, d->body_force, sizeof L->G);
    L->f = (double*)malloc(sizeof(double) * Q * L->N);
    L->fs = (double*)malloc(sizeof(double) * Q * L->N);
    L->rho = (double*)malloc(sizeof(double) * L->N);
    L->u = (double*)malloc(sizeof(double) * 3 * L->N);
    L->flb = (double*)malloc(sizeof(double) * 3 * L->N);
    if (!L->f || !L->fs || !L->rho || !L->u || !L->flb) {
        orc_lattice_destroy(L); set_err("out of memory"); return ORC_ENOMEM;
    }
    *out = L;
    return orc_lattice_init(L, NULL, NULL);
}

static void body_free(body_t* b) {
    if (!b) return;
    free(b->tri); free(b->edge); free(b->hinge); free(b->l0); free(b->ks); free(b->theta0);
    free(b->A0); free(b->x); free(b->xprev); free(b->uv); free(b->Fv); free(b->xb);
    free(b);
}

void orc_lattice_destroy(orc_lattice* L) {
    if (!L) return;
    for (int i = 0; i < L->nb; ++i) body_free(L->b[i]);
    free(L->f); free(L->fs); free(L->rho); free(L->u); free(L->flb);
    free(L);
}

int64_t orc_step_count(const orc_lattice* L) { return L->step; }

/* Density rho = sum f and force-free velocity u* = sum f e / rho of the post-streaming state
 * (moments of Eq. eqfunc, Sec. 1.1; reading: u* feeds the immersed boundary). */
static void moments(orc_lattice* L) {
    const long N = L->N;
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (long k = 0; k < N; ++k) {
        double r = 0.0, j[3] = {0, 0, 0};
        for (int i = 0; i < Q; ++i) {
            double v = L->f[i * N + k];
            r += v;
            for (int d = 0; d < 3; ++d) j[d] += v * E[i][d];
        }
        L->rho[k] = r;
        for (int d = 0; d < 3; ++d) L->u[d * N + k] = j[d] / r;
    }
}

/* Zou-He faces a node lies on: side[a] = -1 (low face of axis a), +1 (high face) or 0.
 * Returns how many. */
static int zh_sides(const orc_lattice* L, int x, int y, int z, int32_t side[3]) {
    const int c[3] = {x, y, z};
    int nw = 0;
    for (int a = 0; a < 3; ++a) {
        side[a] = 0;
        if (c[a] == 0 && L->bc[2 * a] == ORC_BC_ZOUHE) side[a] = -1;
        else if (c[a] == dim(L, a) - 1 && L->bc[2 * a + 1] == ORC_BC_ZOUHE) side[a] = 1;
        if (side[a]) ++nw;
    }
    return nw;
}

/* Closure of every edge and corner node of a box with Zou-He walls on several axes (reading of
 * Sec. 1.1, see orc_corner_closure).  The node's wall velocity: zero along each of its wall
 * normals, the mean of its faces' velocities along the other axes.  Its density conserves mass
 * at the node: the populations coming in through its walls carry together what it sent out
 * through them, rho = sum of the known f_i + sum over unknown i of the outgoing population
 * opposite to i (after streaming: the node's own post-collision fs_opp(i); when a state is
 * set: the unknown values as given, so the given density is kept). */
static void close_edges(orc_lattice* L, int after_stream) {
    if (L->zh_axes < 2) return;
    const long N = L->N;
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (int z = 0; z < L->nz; ++z)
        for (int y = 0; y < L->ny; ++y)
            for (int x = 0; x < L->nx; ++x) {
                int32_t side[3];
                const int nw = zh_sides(L, x, y, z, side);
                if (nw < 2) continue;
                double uw[3];
                for (int d = 0; d < 3; ++d) {
                    uw[d] = 0.0;
                    if (side[d] != 0) continue;
                    for (int a = 0; a < 3; ++a)
                        if (side[a] != 0) uw[d] += L->wall_u[2 * a + (side[a] > 0)][d];
                    uw[d] /= nw;
                }
                const long k = node(L, x, y, z);
                double fl[Q], rho = 0.0;
                for (int i = 0; i < Q; ++i) {
                    fl[i] = L->f[i * N + k];
                    int in = 0;
                    for (int a = 0; a < 3; ++a)
                        if (side[a] != 0 && E[i][a] == -side[a]) in = 1;
                    rho += !in ? fl[i] : (after_stream ? L->fs[opposite(i) * N + k] : fl[i]);
                }
                orc_corner_closure(side, rho, uw, L->G, fl);
                for (int i = 0; i < Q; ++i) L->f[i * N + k] = fl[i];
            }
}

/* Apply the Zou-He closure (Sec. 1.1) to every node on a Zou-He face, then to the edges and
 * corners (the state must satisfy the wall condition at every time level). */
static void close_walls(orc_lattice* L) {
    const long N = L->N;
    for (int a = 0; a < 3; ++a)
        for (int s = 0; s < 2; ++s) {
            int face = 2 * a + s;
            if (L->bc[face] != ORC_BC_ZOUHE) continue;
            int n[3] = {L->nx, L->ny, L->nz};
            int c = s == 0 ? 0 : n[a] - 1;
            int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
            for (int q2 = 0; q2 < n[b2]; ++q2)
                for (int q1 = 0; q1 < n[b1]; ++q1) {
                    int p[3];
                    p[a] = c; p[b1] = q1; p[b2] = q2;
                    int32_t side[3];
                    if (zh_sides(L, p[0], p[1], p[2], side) > 1) continue;   /* edge or corner */
                    long k = node(L, p[0], p[1], p[2]);
                    double fl[Q];
                    for (int i = 0; i < Q; ++i) fl[i] = L->f[i * N + k];
                    orc_wall_closure(a, s == 0 ? -1 : 1, L->wall_u[face], L->G, fl);
                    for (int i = 0; i < Q; ++i) L->f[i * N + k] = fl[i];
                }
        }
    close_edges(L, 0);
}

int orc_lattice_init(orc_lattice* L, const double* rho, const double* u) {
    const long N = L->N;
    for (long k = 0; k < N; ++k) {
        double r = rho ? rho[k] : 1.0;
        double uu[3] = {u ? u[k] : 0.0, u ? u[N + k] : 0.0, u ? u[2 * N + k] : 0.0};
        double feq[Q];
        orc_equilibrium(r, uu, feq);
        for (int i = 0; i < Q; ++i) L->f[i * N + k] = feq[i];
    }
    close_walls(L);
    moments(L);
    L->step = 0;
    return ORC_OK;
}

int orc_set_populations(orc_lattice* L, const double* f) {
    memcpy(L->f, f, sizeof(double) * Q * L->N);
    close_walls(L);
    moments(L);
    return ORC_OK;
}

int orc_get_populations(const orc_lattice* L, double* f) {
    memcpy(f, L->f, sizeof(double) * Q * L->N);
    return ORC_OK;
}

int orc_get_macros(const orc_lattice* L, double* rho, double* u) {
    if (rho) memcpy(rho, L->rho, sizeof(double) * L->N);
    if (u) memcpy(u, L->u, sizeof(double) * 3 * L->N);
    return ORC_OK;
}

/* Collision everywhere: f -> fs, with body force flb (Eqs. evoleq, eqfunc, forcing). */
static void collide_all(orc_lattice* L, int with_collision) {
    const long N = L->N;
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (long k = 0; k < N; ++k) {
        double fl[Q], fo[Q];
        for (int i = 0; i < Q; ++i) fl[i] = L->f[i * N + k];
        if (with_collision) {
            double F[3] = {L->flb[k], L->flb[N + k], L->flb[2 * N + k]};
            orc_collide_node(L->tau, fl, F, fo);
        } else {
            memcpy(fo, fl, sizeof fo);
        }
        for (int i = 0; i < Q; ++i) L->fs[i * N + k] = fo[i];
    }
}

/* Streaming part of Eq. (evoleq), fs -> f: f_i(x) = fs_i(x - e_i) with periodic wrap; a source
 * behind a bounce-back wall returns the node's own opposite population plus the moving-wall
 * term; a source behind a Zou-He face is reconstructed by the face closure, or on edges and
 * corners by the edge closure once every node has streamed. */
static void stream_all(orc_lattice* L) {
    const long N = L->N;
    const int n[3] = {L->nx, L->ny, L->nz};
    int opp[Q];
    double w[Q];
    for (int i = 0; i < Q; ++i) { opp[i] = opposite(i); w[i] = weight(i); }
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (int z = 0; z < n[2]; ++z)
        for (int y = 0; y < n[1]; ++y)
            for (int x = 0; x < n[0]; ++x) {
                const int c[3] = {x, y, z};
                const long k = node(L, x, y, z);
                double fl[Q];
                int zh_face = -1;
                if (x > 0 && x < n[0] - 1 && y > 0 && y < n[1] - 1 && z > 0 && z < n[2] - 1) {
                    /* interior node: every source x - e_i is inside the lattice */
                    for (int i = 0; i < Q; ++i)
                        L->f[i * N + k] = L->fs[i * N + node(L, x - E[i][0], y - E[i][1], z - E[i][2])];
                    continue;
                }
                for (int i = 0; i < Q; ++i) {
                    int s[3], out_face[3] = {-1, -1, -1}, nout = 0;
                    for (int a = 0; a < 3; ++a) {
                        s[a] = c[a] - E[i][a];
                        if (s[a] < 0 || s[a] >= n[a]) {
                            int face = 2 * a + (s[a] < 0 ? 0 : 1);
                            if (L->bc[face] == ORC_BC_PERIODIC) s[a] = s[a] < 0 ? s[a] + n[a] : s[a] - n[a];
                            else out_face[nout++] = face;
                        }
                    }
                    if (nout == 0) {
                        fl[i] = L->fs[i * N + node(L, s[0], s[1], s[2])];
                    } else if (L->bc[out_face[0]] == ORC_BC_BOUNCEBACK) {
                        double uw[3] = {0, 0, 0};
                        for (int q = 0; q < nout; ++q)
                            for (int d = 0; d < 3; ++d) uw[d] += L->wall_u[out_face[q]][d];
                        double eu = E[i][0] * uw[0] + E[i][1] * uw[1] + E[i][2] * uw[2];
                        fl[i] = L->fs[opp[i] * N + k] + 2.0 * w[i] * 1.0 * eu / CS2;
                    } else {
                        fl[i] = 0.0; /* unknown: reconstructed below */
                        zh_face = out_face[0];
                    }
                }
                int32_t side[3];
                if (zh_face >= 0 && zh_sides(L, x, y, z, side) == 1)
                    orc_wall_closure(zh_face / 2, (zh_face % 2) ? 1 : -1, L->wall_u[zh_face], L->G, fl);
                for (int i = 0; i < Q; ++i) L->f[i * N + k] = fl[i];
            }
    close_edges(L, 1);
}

int orc_stream_only(orc_lattice* L, int nsteps) {
    for (int s = 0; s < nsteps; ++s) {
        collide_all(L, 0);
        stream_all(L);
        moments(L);
        L->step++;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ MLS (Sec. 1.2) */

/* Valid node range along a walled axis for the MLS support (Sec. 1.2): all nodes behind
 * halfway bounce-back walls, interior nodes only on a Zou-He axis. */
static int axis_range(const orc_lattice* L, int a, int* lo, int* hi) {
    int n = dim(L, a);
    int b = L->bc[2 * a];
    if (b == ORC_BC_PERIODIC) return 0;
    if (b == ORC_BC_ZOUHE) { *lo = 1; *hi = n - 2; }
    else { *lo = 0; *hi = n - 1; }
    return 1;
}

/* Cholesky factorisation and inverse of the symmetric positive definite 4x4 moment matrix of
 * the MLS fit (Eq. l2norm, Sec. 1.2). */
static int spd_inverse4(const double A[16], double Ai[16]) {
    double Lm[16] = {0};
    for (int j = 0; j < 4; ++j) {
        double s = A[4 * j + j];
        for (int k = 0; k < j; ++k) s -= Lm[4 * j + k] * Lm[4 * j + k];
        if (!(s > 0.0)) return -1;
        Lm[4 * j + j] = sqrt(s);
        for (int i = j + 1; i < 4; ++i) {
            double t = A[4 * i + j];
            for (int k = 0; k < j; ++k) t -= Lm[4 * i + k] * Lm[4 * j + k];
            Lm[4 * i + j] = t / Lm[4 * j + j];
        }
    }
    for (int c = 0; c < 4; ++c) {
        double y[4], x[4];
        for (int i = 0; i < 4; ++i) {
            double t = (i == c) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) t -= Lm[4 * i + k] * y[k];
            y[i] = t / Lm[4 * i + i];
        }
        for (int i = 3; i >= 0; --i) {
            double t = y[i];
            for (int k = i + 1; k < 4; ++k) t -= Lm[4 * k + i] * x[k];
            x[i] = t / Lm[4 * i + i];
        }
        for (int i = 0; i < 4; ++i) Ai[4 * i + c] = x[i];
    }
    return 0;
}

/*
 * MLS transfer operator at point x (Eqs. uLag, l2norm, intKernel): minimise
 * sum_k W_k [p(x_k)^T a - u_k]^2 with linear basis p and weight W = exp(-(r/alpha)^2),
 * r = |x - x_k| / r_w, W = 0 for r > 1.  The basis is written in local coordinates
 * p_k = (1, x_k - x), which spans the same space as (1, x, y, z).  Then
 *   phi_k      = [A^{-1} W_k p_k]_0       (value of the fit at x)
 *   grad phi_k = [A^{-1} W_k p_k]_{1..3}  (gradient of the fit at x)
 * with A = sum_k W_k p_k p_k^T.  Returns the support size, or -1 if the support leaves the
 * fluid domain, -2 if A is singular.
 */
static int mls_eval(const orc_lattice* L, const double x[3], double rw, double alpha,
                    long idx[27], double d[27][3], double phi[27], double grad[27][3]) {
    int lo[3], hi[3], walled[3];
    for (int a = 0; a < 3; ++a) walled[a] = axis_range(L, a, &lo[a], &hi[a]);
    int cnt = 0;
    double W[27];
    int k0[3], k1[3];
    for (int a = 0; a < 3; ++a) {
        k0[a] = (int)ceil(x[a] - rw);
        k1[a] = (int)floor(x[a] + rw);
    }
    for (int kz = k0[2]; kz <= k1[2]; ++kz)
        for (int ky = k0[1]; ky <= k1[1]; ++ky)
            for (int kx = k0[0]; kx <= k1[0]; ++kx) {
                double dd[3] = {kx - x[0], ky - x[1], kz - x[2]};
                double dist = sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
                double r = dist / rw;
                if (r > 1.0) continue;
                int kk[3] = {kx, ky, kz};
                for (int a = 0; a < 3; ++a) {
                    int n = dim(L, a);
                    if (walled[a]) {
                        if (kk[a] < lo[a] || kk[a] > hi[a]) return -1;
                    } else {
                        kk[a] = ((kk[a] % n) + n) % n;
                    }
                }
                if (cnt >= 27) return -1;
                idx[cnt] = node(L, kk[0], kk[1], kk[2]);
                for (int a = 0; a < 3; ++a) d[cnt][a] = dd[a];
                W[cnt] = exp(-(r / alpha) * (r / alpha));
                cnt++;
            }
    double A[16] = {0};
    for (int c = 0; c < cnt; ++c) {
        double p[4] = {1.0, d[c][0], d[c][1], d[c][2]};
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) A[4 * i + j] += W[c] * p[i] * p[j];
    }
    double Ai[16];
    if (spd_inverse4(A, Ai) != 0) return -2;
    for (int c = 0; c < cnt; ++c) {
        double p[4] = {1.0, d[c][0], d[c][1], d[c][2]};
        double v[4];
        for (int i = 0; i < 4; ++i) {
            v[i] = 0.0;
            for (int j = 0; j < 4; ++j) v[i] += Ai[4 * i + j] * p[j];
            v[i] *= W[c];
        }
        phi[c] = v[0];
        if (grad)
            for (int a = 0; a < 3; ++a) grad[c][a] = v[1 + a];
    }
    return cnt;
}

int orc_mls(const orc_lattice* L, const double x[3], double rw, double alpha, int64_t idx[27],
            double d[81], double phi[27], double grad[81], int32_t* count) {
    long id[27];
    double dd[27][3], gg[27][3];
    int c = mls_eval(L, x, rw, alpha, id, dd, phi, gg);
    if (c < 0) { set_err(c == -1 ? "MLS support leaves the fluid domain" : "singular MLS matrix");
                 return c == -1 ? ORC_EDOMAIN : ORC_EINVAL; }
    for (int i = 0; i < c; ++i) {
        idx[i] = id[i];
        for (int a = 0; a < 3; ++a) { d[3 * i + a] = dd[i][a]; grad[3 * i + a] = gg[i][a]; }
    }
    *count = c;
    return ORC_OK;
}

/* ------------------------------------------------------------------ geometry */

static void cross(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Triangle centroid (the Lagrangian marker, Sec. 1.2), area vector N = (xb-xa)x(xc-xa). */
static void tri_geom(const double* x, const int* t, double cen[3], double N[3]) {
    const double *a = x + 3 * t[0], *b = x + 3 * t[1], *c = x + 3 * t[2];
    double ab[3], ac[3];
    for (int d = 0; d < 3; ++d) {
        cen[d] = (a[d] + b[d] + c[d]) / 3.0;
        ab[d] = b[d] - a[d];
        ac[d] = c[d] - a[d];
    }
    cross(ab, ac, N);
}

/* Enclosed volume by the divergence theorem, sum over triangles of x_a . (x_b x x_c) / 6: the V of
 * the volume constraint (Eq. volFor, Sec. 1.3). */
static double enclosed_volume(const double* x, const int* tri, int nt) {
    double V = 0.0;
    for (int t = 0; t < nt; ++t) {
        const double *a = x + 3 * tri[3 * t], *b = x + 3 * tri[3 * t + 1], *c = x + 3 * tri[3 * t + 2];
        double bc[3];
        cross(b, c, bc);
        V += dot(a, bc) / 6.0;
    }
    return V;
}

/* Signed dihedral angle theta of the bending energy (Eqs. bendPot, bendFor, Sec. 1.3) for a hinge: x1, x2 on the shared edge (ordered as in triangle 1),
 * x3 opposite in triangle 1 (x1,x2,x3), x4 opposite in triangle 2 (x2,x1,x4). */
static double dihedral(const double* x, const int* h) {
    const double *x1 = x + 3 * h[0], *x2 = x + 3 * h[1], *x3 = x + 3 * h[2], *x4 = x + 3 * h[3];
    double e[3], a[3], b[3], n1[3], n2[3], c[3];
    for (int d = 0; d < 3; ++d) { e[d] = x2[d] - x1[d]; a[d] = x3[d] - x1[d]; b[d] = x4[d] - x2[d]; }
    double me[3] = {-e[0], -e[1], -e[2]};
    cross(e, a, n1);  /* normal of (x1,x2,x3) */
    cross(me, b, n2); /* normal of (x2,x1,x4) */
    double l1 = sqrt(dot(n1, n1)), l2 = sqrt(dot(n2, n2)), le = sqrt(dot(e, e));
    for (int d = 0; d < 3; ++d) { n1[d] /= l1; n2[d] /= l2; }
    cross(n1, n2, c);
    return atan2(dot(c, e) / le, dot(n1, n2));
}

/* ------------------------------------------------------------------ bodies */

static int cmp_edge(const void* p, const void* q) {
    const int* a = (const int*)p;
    const int* b = (const int*)q;
    if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
    if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
    return 0;
}

/* Solid-polyhedron mass properties (unit density): volume, centroid, second moment about it; they
 * give the rigid mass and inertia of Eqs. (linearVelRig), (angularVelRig) (Sec. 1.3). */
static void polyhedron_moments(const double* x, const int* tri, int nt, double* V, double X[3],
                               double C[9]) {
    double v = 0.0, m1[3] = {0, 0, 0};
    for (int t = 0; t < nt; ++t) {
        const double *a = x + 3 * tri[3 * t], *b = x + 3 * tri[3 * t + 1], *c = x + 3 * tri[3 * t + 2];
        double bc[3];
        cross(b, c, bc);
        double vt = dot(a, bc) / 6.0;
        v += vt;
        for (int d = 0; d < 3; ++d) m1[d] += vt * (a[d] + b[d] + c[d]) / 4.0;
    }
    for (int d = 0; d < 3; ++d) X[d] = m1[d] / v;
    for (int i = 0; i < 9; ++i) C[i] = 0.0;
    for (int t = 0; t < nt; ++t) {
        double p[3][3];
        for (int j = 0; j < 3; ++j)
            for (int d = 0; d < 3; ++d) p[j][d] = x[3 * tri[3 * t + j] + d] - X[d];
        double bc[3];
        cross(p[1], p[2], bc);
        double vt = dot(p[0], bc) / 6.0;
        double s[3];
        for (int d = 0; d < 3; ++d) s[d] = p[0][d] + p[1][d] + p[2][d];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                C[3 * i + j] += vt / 20.0 *
                    (p[0][i] * p[0][j] + p[1][i] * p[1][j] + p[2][i] * p[2][j] + s[i] * s[j]);
    }
    *V = v;
}

/* Rest state of a body (Sec. 1.3): edges and hinges of the closed mesh, rest lengths and angles,
 * Van Gelder spring constants k_s,l = k_s0 T (A1 + A2) / l0^2 (after Eq. strainFor), vertex mass
 * m_v = ratio T S0 / M_v (Eq. newtonSoft), and for rigid bodies mass and inertia. */
int orc_body_add(orc_lattice* L, const orc_body_desc* d, const double* xyz, int32_t nv,
                 const int32_t* tri, int32_t nt, int32_t* body_id) {
    if (L->nb >= MAXB) { set_err("too many bodies"); return ORC_EINVAL; }
    if (nv < 4 || nt < 4) { set_err("mesh too small"); return ORC_EINVAL; }
    for (int t = 0; t < 3 * nt; ++t)
        if (tri[t] < 0 || tri[t] >= nv) { set_err("triangle index out of range"); return ORC_EINVAL; }
    if (!(d->mls_rw > 0) || !(d->mls_alpha > 0)) { set_err("bad MLS parameters"); return ORC_EINVAL; }
    if (!d->rigid && !(d->mass_ratio > 0)) { set_err("membrane mass must be positive"); return ORC_EINVAL; }
    if (d->rigid && !(d->mass_ratio > 0)) { set_err("rigid density ratio must be positive"); return ORC_EINVAL; }
    if (d->integrator != ORC_INTEGRATOR_DISPLACEMENT && d->integrator != ORC_INTEGRATOR_PAPER &&
        d->integrator != ORC_INTEGRATOR_KINEMATIC) {
        set_err("unknown integrator"); return ORC_EINVAL;
    }
    if (!d->rigid && (d->gravity[0] != 0 || d->gravity[1] != 0 || d->gravity[2] != 0)) {
        set_err("gravity is supported on rigid bodies only"); return ORC_EINVAL;
    }
    body_t* b = (body_t*)calloc(1, sizeof *b);
    b->d = *d;
    b->nv = nv; b->nt = nt;
    b->tri = (int*)malloc(sizeof(int) * 3 * nt);
    memcpy(b->tri, tri, sizeof(int) * 3 * nt);
    /* directed half-edges -> undirected edges with their two triangles */
    int* he = (int*)malloc(sizeof(int) * 4 * 3 * nt); /* vmin, vmax, tri, directed(0: vmin->vmax) */
    for (int t = 0; t < nt; ++t)
        for (int j = 0; j < 3; ++j) {
            int a = tri[3 * t + j], c = tri[3 * t + (j + 1) % 3];
            int* h = he + 4 * (3 * t + j);
            h[0] = a < c ? a : c; h[1] = a < c ? c : a; h[2] = t; h[3] = a < c ? 0 : 1;
        }
    qsort(he, 3 * nt, 4 * sizeof(int), cmp_edge);
    if ((3 * nt) % 2) { free(he); body_free(b); set_err("mesh not closed"); return ORC_EINVAL; }
    b->ne = 3 * nt / 2;
    b->edge = (int*)malloc(sizeof(int) * 2 * b->ne);
    b->hinge = (int*)malloc(sizeof(int) * 4 * b->ne);
    int* etri = (int*)malloc(sizeof(int) * 2 * b->ne);
    for (int e = 0; e < b->ne; ++e) {
        int* h0 = he + 4 * (2 * e);
        int* h1 = he + 4 * (2 * e + 1);
        int ok = h0[0] == h1[0] && h0[1] == h1[1] && h0[3] != h1[3];
        if (e + 1 < b->ne) {
            int* h2 = he + 4 * (2 * e + 2);
            if (h2[0] == h0[0] && h2[1] == h0[1]) ok = 0;
        }
        if (e > 0) {
            int* hm = he + 4 * (2 * e - 1);
            if (hm[0] == h0[0] && hm[1] == h0[1]) ok = 0;
        }
        if (!ok) {
            free(he); free(etri); body_free(b);
            set_err("mesh is not a closed, consistently oriented 2-manifold");
            return ORC_EINVAL;
        }
        b->edge[2 * e] = h0[0];
        b->edge[2 * e + 1] = h0[1];
        /* triangle 1 = the one traversing vmin -> vmax */
        int t1 = h0[3] == 0 ? h0[2] : h1[2];
        int t2 = h0[3] == 0 ? h1[2] : h0[2];
        etri[2 * e] = t1; etri[2 * e + 1] = t2;
        int x1 = h0[0], x2 = h0[1], x3 = -1, x4 = -1;
        for (int j = 0; j < 3; ++j) {
            int v1 = tri[3 * t1 + j], v2 = tri[3 * t2 + j];
            if (v1 != x1 && v1 != x2) x3 = v1;
            if (v2 != x1 && v2 != x2) x4 = v2;
        }
        b->hinge[4 * e] = x1; b->hinge[4 * e + 1] = x2;
        b->hinge[4 * e + 2] = x3; b->hinge[4 * e + 3] = x4;
    }
    free(he);
    /* rest state */
    b->A0 = (double*)malloc(sizeof(double) * nt);
    b->S0 = 0.0;
    for (int t = 0; t < nt; ++t) {
        double cen[3], N[3];
        tri_geom(xyz, tri + 3 * t, cen, N);
        b->A0[t] = 0.5 * sqrt(dot(N, N));
        b->S0 += b->A0[t];
    }
    b->V0 = enclosed_volume(xyz, tri, nt);
    if (!(b->V0 > 0)) { free(etri); body_free(b); set_err("mesh is not outward oriented"); return ORC_EINVAL; }
    b->l0 = (double*)malloc(sizeof(double) * b->ne);
    b->ks = (double*)malloc(sizeof(double) * b->ne);
    b->theta0 = (double*)malloc(sizeof(double) * b->ne);
    for (int e = 0; e < b->ne; ++e) {
        const double *p = xyz + 3 * b->edge[2 * e], *q = xyz + 3 * b->edge[2 * e + 1];
        double dd[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
        b->l0[e] = sqrt(dot(dd, dd));
        /* Van Gelder surface-weighted spring constant (Sec. 1.3, network model) */
        b->ks[e] = d->ks0 * d->thickness * (b->A0[etri[2 * e]] + b->A0[etri[2 * e + 1]]) /
                   (b->l0[e] * b->l0[e]);
        b->theta0[e] = dihedral(xyz, b->hinge + 4 * e);
    }
    free(etri);
    b->mv = d->mass_ratio * d->thickness * b->S0 / nv;
    b->x = (double*)malloc(sizeof(double) * 3 * nv);
    b->xprev = (double*)malloc(sizeof(double) * 3 * nv);
    b->uv = (double*)calloc(3 * nv, sizeof(double));
    b->Fv = (double*)calloc(3 * nv, sizeof(double));
    memcpy(b->x, xyz, sizeof(double) * 3 * nv);
    memcpy(b->xprev, xyz, sizeof(double) * 3 * nv);
    if (d->rigid) {
        double V, C[9];
        polyhedron_moments(xyz, tri, nt, &V, b->X, C);
        b->mass = d->mass_ratio * V;
        double tr = C[0] + C[4] + C[8];
        for (int i = 0; i < 9; ++i) b->Ib[i] = d->mass_ratio * ((i % 4 == 0 ? tr : 0.0) - C[i]);
        for (int i = 0; i < 9; ++i) b->R[i] = (i % 4 == 0) ? 1.0 : 0.0;
        b->xb = (double*)malloc(sizeof(double) * 3 * nv);
        for (int v = 0; v < nv; ++v)
            for (int a = 0; a < 3; ++a) b->xb[3 * v + a] = xyz[3 * v + a] - b->X[a];
    }
    L->b[L->nb] = b;
    *body_id = L->nb++;
    return ORC_OK;
}

/* Initial velocity and a consistent history for the multistep updates (reading: the paper leaves
 * the start-up of Eqs. verletPos / linearVelRig open): x^{-1} = x^0 - v dt, u^{-1} = u^{-2} = v. */
int orc_body_set_velocity(orc_lattice* L, int32_t id, const double* v) {
    if (id < 0 || id >= L->nb) { set_err("no such body"); return ORC_EINVAL; }
    body_t* b = L->b[id];
    if (b->d.rigid) {
        for (int a = 0; a < 3; ++a) {
            b->ur[a] = b->ur1[a] = v[a];
            b->om[a] = b->om1[a] = v[3 + a];
        }
    } else {
        for (int i = 0; i < 3 * b->nv; ++i) {
            b->uv[i] = v[i];
            b->xprev[i] = b->x[i] - v[i];
        }
    }
    return ORC_OK;
}

/* A membrane at rest at the given positions (its rest state stays the one of orc_body_add):
 * x^n = x^{n-1} = xyz, u_v = 0. */
int orc_body_set_positions(orc_lattice* L, int32_t id, const double* xyz) {
    if (id < 0 || id >= L->nb || L->b[id]->d.rigid) { set_err("no such membrane"); return ORC_EINVAL; }
    body_t* b = L->b[id];
    for (int i = 0; i < 3 * b->nv; ++i) {
        b->x[i] = b->xprev[i] = xyz[i];
        b->uv[i] = 0.0;
    }
    return ORC_OK;
}

int orc_body_counts(const orc_lattice* L, int32_t id, int32_t* nv, int32_t* nt, int32_t* ne) {
    if (id < 0 || id >= L->nb) { set_err("no such body"); return ORC_EINVAL; }
    *nv = L->b[id]->nv; *nt = L->b[id]->nt; *ne = L->b[id]->ne;
    return ORC_OK;
}

int orc_body_topology(const orc_lattice* L, int32_t id, int32_t* edge, int32_t* hinge) {
    if (id < 0 || id >= L->nb) { set_err("no such body"); return ORC_EINVAL; }
    const body_t* b = L->b[id];
    for (int i = 0; i < 2 * b->ne; ++i) edge[i] = b->edge[i];
    for (int i = 0; i < 4 * b->ne; ++i) hinge[i] = b->hinge[i];
    return ORC_OK;
}

int orc_body_rest(const orc_lattice* L, int32_t id, double* l0, double* ks, double* theta0,
                  double* A0, double scal[4]) {
    if (id < 0 || id >= L->nb) { set_err("no such body"); return ORC_EINVAL; }
    const body_t* b = L->b[id];
    if (l0) memcpy(l0, b->l0, sizeof(double) * b->ne);
    if (ks) memcpy(ks, b->ks, sizeof(double) * b->ne);
    if (theta0) memcpy(theta0, b->theta0, sizeof(double) * b->ne);
    if (A0) memcpy(A0, b->A0, sizeof(double) * b->nt);
    scal[0] = b->V0; scal[1] = b->S0; scal[2] = b->mv; scal[3] = b->mass;
    return ORC_OK;
}

int orc_body_rigid_props(const orc_lattice* L, int32_t id, double X0[3], double* mass, double I[9]) {
    if (id < 0 || id >= L->nb || !L->b[id]->d.rigid) { set_err("no such rigid body"); return ORC_EINVAL; }
    const body_t* b = L->b[id];
    memcpy(X0, b->X, sizeof(double) * 3);
    *mass = b->mass;
    memcpy(I, b->Ib, sizeof(double) * 9);
    return ORC_OK;
}

/* Vertex velocity of the current state, the input of the desired boundary velocity U_b (Sec. 1.2;
 * rigid: u + omega x (x_v - X)). */
static void vertex_velocity(const body_t* b, int v, double out[3]) {
    if (!b->d.rigid) {
        for (int a = 0; a < 3; ++a) out[a] = b->uv[3 * v + a];
    } else {
        double r[3], w[3];
        for (int a = 0; a < 3; ++a) r[a] = b->x[3 * v + a] - b->X[a];
        cross(b->om, r, w);
        for (int a = 0; a < 3; ++a) out[a] = b->ur[a] + w[a];
    }
}

int orc_body_get_state(const orc_lattice* L, int32_t id, double* xyz, double* vel) {
    if (id < 0 || id >= L->nb) { set_err("no such body"); return ORC_EINVAL; }
    const body_t* b = L->b[id];
    if (xyz) memcpy(xyz, b->x, sizeof(double) * 3 * b->nv);
    if (vel)
        for (int v = 0; v < b->nv; ++v) vertex_velocity(b, v, vel + 3 * v);
    return ORC_OK;
}

int orc_body_get_forces(const orc_lattice* L, int32_t id, double* fv, double F[3], double M[3]) {
    if (id < 0 || id >= L->nb) { set_err("no such body"); return ORC_EINVAL; }
    const body_t* b = L->b[id];
    if (fv) memcpy(fv, b->Fv, sizeof(double) * 3 * b->nv);
    if (F) memcpy(F, b->Ftot, sizeof(double) * 3);
    if (M) memcpy(M, b->Mtot, sizeof(double) * 3);
    return ORC_OK;
}

/* ------------------------------------------------------------------ internal forces */

/*
 * Internal membrane forces at positions x (Sec. 1.3, network model):
 *   springs  Eq. (strainFor) from V = 1/2 k_{s,l} (l - l0)^2 (Eq. strainPot);
 *   bending  -grad of k_b [1 - cos(theta - theta0)] with the signed dihedral angle;
 *   volume   +k_v (1 - V/V0) n_t A_t on each triangle, one third to each vertex (Eq. volFor).
 * E[0..2] receive the spring, bending and volume energies (the latter k_v (V-V0)^2 / (2 V0)).
 */
static void membrane_forces(const body_t* b, const double* x, double* F, double En[3]) {
    for (int i = 0; i < 3 * b->nv; ++i) F[i] = 0.0;
    double es = 0.0, eb = 0.0;
    for (int e = 0; e < b->ne; ++e) {
        int i = b->edge[2 * e], j = b->edge[2 * e + 1];
        double r[3];
        for (int a = 0; a < 3; ++a) r[a] = x[3 * i + a] - x[3 * j + a];
        double l = sqrt(dot(r, r));
        double dl = l - b->l0[e];
        es += 0.5 * b->ks[e] * dl * dl;
        for (int a = 0; a < 3; ++a) {
            double fa = -b->ks[e] * dl * r[a] / l;
            F[3 * i + a] += fa;
            F[3 * j + a] -= fa;
        }
    }
    if (b->d.kb != 0.0)
        for (int e = 0; e < b->ne; ++e) {
            const int* h = b->hinge + 4 * e;
            const double *x1 = x + 3 * h[0], *x2 = x + 3 * h[1], *x3 = x + 3 * h[2], *x4 = x + 3 * h[3];
            double theta = dihedral(x, h);
            double dth = theta - b->theta0[e];
            eb += b->d.kb * (1.0 - cos(dth));
            /* gradient of theta: the opposite vertices move their triangle's normal about the
             * hinge with lever arm = height over the edge; the edge vertices carry the
             * reaction split by the foot-point position of each opposite vertex. */
            double ev[3], a3[3], a4[3], N1[3], N2[3];
            for (int a = 0; a < 3; ++a) {
                ev[a] = x2[a] - x1[a];
                a3[a] = x3[a] - x1[a];
                a4[a] = x4[a] - x2[a];
            }
            double mev[3] = {-ev[0], -ev[1], -ev[2]};
            cross(ev, a3, N1);
            cross(mev, a4, N2);
            double le2 = dot(ev, ev), le = sqrt(le2);
            double n1sq = dot(N1, N1), n2sq = dot(N2, N2);
            double g3[3], g4[3], g1[3], g2[3];
            for (int a = 0; a < 3; ++a) {
                g3[a] = -le * N1[a] / n1sq;
                g4[a] = -le * N2[a] / n2sq;
            }
            double d3[3], d4[3];
            for (int a = 0; a < 3; ++a) { d3[a] = x3[a] - x1[a]; d4[a] = x4[a] - x1[a]; }
            double s3 = dot(d3, ev) / le2, s4 = dot(d4, ev) / le2;
            for (int a = 0; a < 3; ++a) {
                g1[a] = -(1.0 - s3) * g3[a] - (1.0 - s4) * g4[a];
                g2[a] = -s3 * g3[a] - s4 * g4[a];
            }
            double c = -b->d.kb * sin(dth);
            for (int a = 0; a < 3; ++a) {
                F[3 * h[0] + a] += c * g1[a];
                F[3 * h[1] + a] += c * g2[a];
                F[3 * h[2] + a] += c * g3[a];
                F[3 * h[3] + a] += c * g4[a];
            }
        }
    double V = enclosed_volume(x, b->tri, b->nt);
    double ev_ = 0.0;
    if (b->d.kv != 0.0) {
        double s = b->d.kv * (1.0 - V / b->V0);
        for (int t = 0; t < b->nt; ++t) {
            double cen[3], N[3];
            tri_geom(x, b->tri + 3 * t, cen, N);
            /* n_t A_t = N/2, a third of it to each vertex */
            for (int j = 0; j < 3; ++j)
                for (int a = 0; a < 3; ++a) F[3 * b->tri[3 * t + j] + a] += s * N[a] / 6.0;
        }
        ev_ = b->d.kv * (V - b->V0) * (V - b->V0) / (2.0 * b->V0);
    }
    if (En) { En[0] = es; En[1] = eb; En[2] = ev_; }
}

int orc_membrane_forces(const orc_lattice* L, int32_t id, const double* xyz, double* F, double En[3]) {
    if (id < 0 || id >= L->nb) { set_err("no such body"); return ORC_EINVAL; }
    membrane_forces(L->b[id], xyz ? xyz : L->b[id]->x, F, En);
    return ORC_OK;
}

/* ------------------------------------------------------------------ probes (Sec. 1.3) */

/*
 * Hydrodynamic force on every triangle from the current fields (Eqs. hydroForP, hydroForNu):
 * MLS probes at x_t +- l_p n_t give rho^+-, grad u^+-; p = c_s^2 rho;
 * tau = rho nu (grad u + grad u^T);  F_t = [-(p+ - p-) n_t + (tau+ - tau-) n_t] A_t.
 */
static int probe_forces(const orc_lattice* L, const body_t* b, double* Fext) {
    const long N = L->N;
    const double nu = CS2 * (L->tau - 0.5);
    int err = 0;
#pragma omp parallel for schedule(static) num_threads(g_threads) reduction(| : err)
    for (int t = 0; t < b->nt; ++t) {
        double cen[3], Nv[3];
        tri_geom(b->x, b->tri + 3 * t, cen, Nv);
        double ln = sqrt(dot(Nv, Nv));
        double n[3] = {Nv[0] / ln, Nv[1] / ln, Nv[2] / ln};
        double A = 0.5 * ln;
        double rho_s[2], gu_s[2][3][3];
        for (int side = 0; side < 2; ++side) {
            double sg = side == 0 ? 1.0 : -1.0;
            double xp[3];
            for (int a = 0; a < 3; ++a) xp[a] = cen[a] + sg * b->d.probe_len * n[a];
            long idx[27];
            double dd[27][3], phi[27], gr[27][3];
            int c = mls_eval(L, xp, b->d.mls_rw, b->d.mls_alpha, idx, dd, phi, gr);
            if (c < 0) { err |= 1; rho_s[side] = 1.0; memset(gu_s[side], 0, sizeof gu_s[side]); continue; }
            double r = 0.0, g[3][3] = {{0}};
            for (int k = 0; k < c; ++k) {
                r += phi[k] * L->rho[idx[k]];
                for (int i = 0; i < 3; ++i)        /* velocity component */
                    for (int j = 0; j < 3; ++j)    /* derivative direction */
                        g[i][j] += gr[k][j] * L->u[i * N + idx[k]];
            }
            rho_s[side] = r;
            memcpy(gu_s[side], g, sizeof g);
        }
        double p_p = CS2 * rho_s[0], p_m = CS2 * rho_s[1];
        for (int i = 0; i < 3; ++i) {
            double tn = 0.0;
            for (int j = 0; j < 3; ++j) {
                double tp = rho_s[0] * nu * (gu_s[0][i][j] + gu_s[0][j][i]);
                double tm = rho_s[1] * nu * (gu_s[1][i][j] + gu_s[1][j][i]);
                tn += (tp - tm) * n[j];
            }
            Fext[3 * t + i] = (-(p_p - p_m) * n[i] + tn) * A;
        }
    }
    return err ? -1 : 0;
}

int orc_body_probe_forces(const orc_lattice* L, int32_t id, double* Fext) {
    if (id < 0 || id >= L->nb) { set_err("no such body"); return ORC_EINVAL; }
    if (probe_forces(L, L->b[id], Fext)) { set_err("probe support leaves the fluid domain"); return ORC_EDOMAIN; }
    return ORC_OK;
}

/* ------------------------------------------------------------------ IB forcing (Sec. 1.2) */

/*
 * f_lb = G + sum over markers l (in id order) of c_l phi_k^l F_l with F_l = U_b^l - U*^l
 * (dt = 1) and c_l = A_l h.  U (3 per marker, all bodies concatenated) and Fl receive the
 * interpolated velocity and the Lagrangian force when non-NULL.
 */
static int ib_force(orc_lattice* L, double* Uout, double* Flout) {
    const long N = L->N;
    for (int a = 0; a < 3; ++a)
        for (long k = 0; k < N; ++k) L->flb[a * N + k] = L->G[a];
    long moff = 0;
    for (int ib = 0; ib < L->nb; ++ib) {
        body_t* b = L->b[ib];
        long* idx = (long*)malloc(sizeof(long) * 27 * b->nt);
        double* phi = (double*)malloc(sizeof(double) * 27 * b->nt);
        int* cnt = (int*)malloc(sizeof(int) * b->nt);
        int err = 0;
#pragma omp parallel for schedule(static) num_threads(g_threads) reduction(| : err)
        for (int t = 0; t < b->nt; ++t) {
            double cen[3], Nv[3], dd[27][3];
            tri_geom(b->x, b->tri + 3 * t, cen, Nv);
            int c = mls_eval(L, cen, b->d.mls_rw, b->d.mls_alpha, idx + 27 * t, dd, phi + 27 * t, NULL);
            if (c < 0) { err |= 1; c = 0; }
            cnt[t] = c;
        }
        if (err) { free(idx); free(phi); free(cnt); set_err("marker support leaves the fluid domain"); return ORC_EDOMAIN; }
        for (int t = 0; t < b->nt; ++t) {
            double cen[3], Nv[3];
            tri_geom(b->x, b->tri + 3 * t, cen, Nv);
            double A = 0.5 * sqrt(dot(Nv, Nv));
            double U[3] = {0, 0, 0};
            for (int k = 0; k < cnt[t]; ++k)
                for (int a = 0; a < 3; ++a) U[a] += phi[27 * t + k] * L->u[a * N + idx[27 * t + k]];
            double Ub[3] = {0, 0, 0};
            if (!b->d.rigid) {
                for (int j = 0; j < 3; ++j)
                    for (int a = 0; a < 3; ++a) Ub[a] += b->uv[3 * b->tri[3 * t + j] + a] / 3.0;
            } else {
                double r[3], w[3];
                for (int a = 0; a < 3; ++a) r[a] = cen[a] - b->X[a];
                cross(b->om, r, w);
                for (int a = 0; a < 3; ++a) Ub[a] = b->ur[a] + w[a];
            }
            double Fl[3];
            for (int a = 0; a < 3; ++a) Fl[a] = Ub[a] - U[a];
            double cl = A * b->d.shell_h;
            for (int k = 0; k < cnt[t]; ++k)
                for (int a = 0; a < 3; ++a) L->flb[a * N + idx[27 * t + k]] += cl * phi[27 * t + k] * Fl[a];
            if (Uout) for (int a = 0; a < 3; ++a) Uout[3 * (moff + t) + a] = U[a];
            if (Flout) for (int a = 0; a < 3; ++a) Flout[3 * (moff + t) + a] = Fl[a];
        }
        moff += b->nt;
        free(idx); free(phi); free(cnt);
    }
    return ORC_OK;
}

int orc_ib_force(orc_lattice* L, double* flb, double* U, double* Fl) {
    int rc = ib_force(L, U, Fl);
    if (rc) return rc;
    if (flb) memcpy(flb, L->flb, sizeof(double) * 3 * L->N);
    return ORC_OK;
}

/* ------------------------------------------------------------------ structure update */

static void rotation_from_vector(const double w[3], double Rm[9]) {
    double th = sqrt(dot(w, w));
    for (int i = 0; i < 9; ++i) Rm[i] = (i % 4 == 0) ? 1.0 : 0.0;
    if (th == 0.0) return;
    double k[3] = {w[0] / th, w[1] / th, w[2] / th};
    double K[9] = {0, -k[2], k[1], k[2], 0, -k[0], -k[1], k[0], 0};
    double K2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            K2[3 * i + j] = 0.0;
            for (int m = 0; m < 3; ++m) K2[3 * i + j] += K[3 * i + m] * K[3 * m + j];
        }
    for (int i = 0; i < 9; ++i) Rm[i] += sin(th) * K[i] + (1.0 - cos(th)) * K2[i];
}

static void mat3_mul(const double A[9], const double B[9], double C[9]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            C[3 * i + j] = 0.0;
            for (int m = 0; m < 3; ++m) C[3 * i + j] += A[3 * i + m] * B[3 * m + j];
        }
}

static int solve3(const double A[9], const double b[3], double x[3]) {
    double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                 A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (det == 0.0) return -1;
    for (int c = 0; c < 3; ++c) {
        double M[9];
        memcpy(M, A, sizeof M);
        for (int r = 0; r < 3; ++r) M[3 * r + c] = b[r];
        x[c] = (M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
                M[2] * (M[3] * M[7] - M[4] * M[6])) / det;
    }
    return 0;
}

/*
 * One rigid-body update (Sec. 1.3, rigid objects) from the hydrodynamic totals Ft, Mt of the
 * step: Eqs. linearVelRig / angularVelRig with udot = F/m, F = Ft + (m - V0) g (buoyancy), and
 * omegadot = I^-1 Mt, I the body inertia rotated into the current pose (R Ib R^T); then
 * X += u^{n+1} dt, the pose turned by the rotation vector omega^{n+1} dt (Rodrigues), and the
 * vertices placed at X + R x_body.
 */
static int rigid_advance(body_t* b, const double Ft[3], const double Mt[3]) {
    double F[3];
    for (int a = 0; a < 3; ++a) F[a] = Ft[a] + (b->mass - b->V0) * b->d.gravity[a];
    double Iw[9], tmp[9], Rt[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Rt[3 * i + j] = b->R[3 * j + i];
    mat3_mul(b->R, b->Ib, tmp);
    mat3_mul(tmp, Rt, Iw);
    double wd[3];
    if (solve3(Iw, Mt, wd)) { set_err("singular inertia"); return ORC_EUNSTABLE; }
    double un[3], wn[3];
    for (int a = 0; a < 3; ++a) {
        un[a] = 2.0 / 3.0 * (2.0 * b->ur[a] - 0.5 * b->ur1[a] + F[a] / b->mass);
        wn[a] = 2.0 / 3.0 * (2.0 * b->om[a] - 0.5 * b->om1[a] + wd[a]);
    }
    memcpy(b->ur1, b->ur, sizeof un); memcpy(b->ur, un, sizeof un);
    memcpy(b->om1, b->om, sizeof wn); memcpy(b->om, wn, sizeof wn);
    for (int a = 0; a < 3; ++a) b->X[a] += un[a];
    double Rw[9], Rn[9];
    rotation_from_vector(wn, Rw);
    mat3_mul(Rw, b->R, Rn);
    memcpy(b->R, Rn, sizeof Rn);
    memcpy(b->xprev, b->x, sizeof(double) * 3 * b->nv);
    for (int v = 0; v < b->nv; ++v)
        for (int a = 0; a < 3; ++a) {
            double s = b->X[a];
            for (int c = 0; c < 3; ++c) s += b->R[3 * a + c] * b->xb[3 * v + c];
            b->x[3 * v + a] = s;
        }
    for (int i = 0; i < 3 * b->nv; ++i)
        if (!isfinite(b->x[i])) { set_err("non-finite body state"); return ORC_EUNSTABLE; }
    return ORC_OK;
}

int orc_rigid_advance(orc_lattice* L, int32_t id, const double F[3], const double M[3]) {
    if (id < 0 || id >= L->nb || !L->b[id]->d.rigid) { set_err("no such rigid body"); return ORC_EINVAL; }
    body_t* b = L->b[id];
    memcpy(b->Ftot, F, sizeof(double) * 3);
    memcpy(b->Mtot, M, sizeof(double) * 3);
    return rigid_advance(b, F, M);
}

int orc_body_rigid_state(const orc_lattice* L, int32_t id, double X[3], double R[9], double u[3],
                         double om[3]) {
    if (id < 0 || id >= L->nb || !L->b[id]->d.rigid) { set_err("no such rigid body"); return ORC_EINVAL; }
    const body_t* b = L->b[id];
    memcpy(X, b->X, sizeof(double) * 3);
    memcpy(R, b->R, sizeof(double) * 9);
    memcpy(u, b->ur, sizeof(double) * 3);
    memcpy(om, b->om, sizeof(double) * 3);
    return ORC_OK;
}

static int structure_update(orc_lattice* L, body_t* b) {
    const long N = L->N;
    double* Fext = (double*)malloc(sizeof(double) * 3 * b->nt);
    if (probe_forces(L, b, Fext)) { free(Fext); set_err("probe support leaves the fluid domain"); return ORC_EDOMAIN; }
    /* totals and reference point */
    double Xref[3] = {0, 0, 0};
    if (b->d.rigid) memcpy(Xref, b->X, sizeof Xref);
    else {
        for (int v = 0; v < b->nv; ++v)
            for (int a = 0; a < 3; ++a) Xref[a] += b->x[3 * v + a];
        for (int a = 0; a < 3; ++a) Xref[a] /= b->nv;
    }
    double Ft[3] = {0, 0, 0}, Mt[3] = {0, 0, 0};
    for (int t = 0; t < b->nt; ++t) {
        double cen[3], Nv[3], r[3], m[3];
        tri_geom(b->x, b->tri + 3 * t, cen, Nv);
        for (int a = 0; a < 3; ++a) r[a] = cen[a] - Xref[a];
        cross(r, Fext + 3 * t, m);
        for (int a = 0; a < 3; ++a) { Ft[a] += Fext[3 * t + a]; Mt[a] += m[a]; }
    }
    memcpy(b->Ftot, Ft, sizeof Ft);
    memcpy(b->Mtot, Mt, sizeof Mt);
    for (int i = 0; i < 3 * b->nv; ++i) b->Fv[i] = 0.0;
    for (int t = 0; t < b->nt; ++t)
        for (int j = 0; j < 3; ++j)
            for (int a = 0; a < 3; ++a) b->Fv[3 * b->tri[3 * t + j] + a] += Fext[3 * t + a] / 3.0;
    free(Fext);
    if (b->d.rigid) return rigid_advance(b, Ft, Mt);
    /* membrane: Eq. (newtonSoft) with internal forces at x^n, Verlet Eqs. verletPos/verletVel */
    double* Fi = (double*)malloc(sizeof(double) * 3 * b->nv);
    membrane_forces(b, b->x, Fi, NULL);
    for (int i = 0; i < 3 * b->nv; ++i) b->Fv[i] += Fi[i];
    free(Fi);
    double* u0 = (double*)malloc(sizeof(double) * 3 * b->nv);
    int err = 0;
#pragma omp parallel for schedule(static) num_threads(g_threads) reduction(| : err)
    for (int v = 0; v < b->nv; ++v) {
        long idx[27];
        double dd[27][3], phi[27];
        int c = mls_eval(L, b->x + 3 * v, b->d.mls_rw, b->d.mls_alpha, idx, dd, phi, NULL);
        if (c < 0) { err |= 1; c = 0; }
        for (int a = 0; a < 3; ++a) {
            double s = 0.0;
            for (int k = 0; k < c; ++k) s += phi[k] * L->u[a * N + idx[k]];
            u0[3 * v + a] = s;
        }
    }
    if (err) { free(u0); set_err("vertex support leaves the fluid domain"); return ORC_EDOMAIN; }
    for (int v = 0; v < b->nv; ++v)
        for (int a = 0; a < 3; ++a) {
            int i = 3 * v + a;
            double acc = b->Fv[i] / b->mv;
            /* Eq. (verletPos) with the interpolated fluid velocity as the tentative velocity */
            double xt = b->x[i] + u0[i] + 0.5 * acc;
            double un, xn;
            if (b->d.integrator == ORC_INTEGRATOR_PAPER) {
                un = 1.5 * xt - 2.0 * b->x[i] + 0.5 * b->xprev[i]; /* Eq. (verletVel) */
                xn = b->x[i] + un + 0.5 * acc;                    /* Eq. (verletPos) again */
            } else if (b->d.integrator == ORC_INTEGRATOR_KINEMATIC) {
                /* kinematic IB (Sec. 2.4): the point is advected with the fluid velocity */
                un = u0[i];
                xn = b->x[i] + un;
            } else {
                xn = xt;
                un = xn - b->x[i];
            }
            b->xprev[i] = b->x[i];
            b->x[i] = xn;
            b->uv[i] = un;
            if (!isfinite(xn)) err = 1;
        }
    free(u0);
    if (err) { set_err("non-finite body state"); return ORC_EUNSTABLE; }
    return ORC_OK;
}

/* ------------------------------------------------------------------ step */

int orc_step(orc_lattice* L, int nsteps) {
    for (int s = 0; s < nsteps; ++s) {
        int rc = ib_force(L, NULL, NULL);
        if (rc) return rc;
        collide_all(L, 1);
        stream_all(L);
        moments(L);
        for (int ib = 0; ib < L->nb; ++ib) {
            rc = structure_update(L, L->b[ib]);
            if (rc) return rc;
        }
        L->step++;
    }
    for (long k = 0; k < L->N; ++k)
        if (!isfinite(L->rho[k])) { set_err("non-finite density"); return ORC_EUNSTABLE; }
    return ORC_OK;
}
