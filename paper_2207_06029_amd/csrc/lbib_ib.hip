// Immersed-boundary and structure kernels (Secs. 1.2-1.3).
//
// One MLS point (triangle centroid, probe or vertex) is evaluated by a group of 8 lanes (half a
// DPP row); lane k owns nodes k, k + 8, k + 16 and k + 24 of the 3x3x3 block around the nearest
// node.  Every node within r_w of the point lies in that block, so the group covers the whole
// support of Eq. (intKernel).  The 4x4 moment matrix is accumulated and factorised in FP64 (every
// lane of the group solves redundantly), so no lane waits on another except for the butterfly
// sums.  The marker kernels run one-wave blocks of eight points: few lanes per point keep the
// instructions per point low, which bounds the batched launches.
//
// Step order inside the time step n -> n+1:
//   k_centroids  triangle blocks: force window of this step from the vertex bounding box,
//                geometry at x^n (kept for the probes), MLS at centroids on moments of f^n,
//                F_l = U_b - U*, fixed-point spreading into the body's force window, partial
//                enclosed volumes; edge blocks: spring and bending forces of every hinge
//   k_fold_bodies (membranes with k_v != 0) volume V^n from the partials
//   (sweep)      collide+stream with the spread force
//   (moments)    moments of f^{n+1} in the body's window
//   k_triangles  one group per probe (geometry from the centroid kernel): stresses on f^{n+1}
//                (Eqs. hydroForP, hydroForNu), volume force per triangle; rigid bodies: FP64
//                partial force and torque per block.  Blocks of their own: the fluid velocity
//                at every membrane vertex from f^{n+1}
//   k_fold_bodies (rigid bodies) FP64 totals and the velocity / pose update
//   k_vertices   gathered forces, membrane update with that velocity, integer bounding box
//                of x^{n+1} for the next step's window
#include "lbib_internal.h"

namespace lbib {

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
// Sum over a group of G = 8 (half a DPP row) or 16 lanes (a row).  Lane exchanges xor 1 and xor 2
// are quad permutes, then the row half-mirror pairs the two quads of 8 lanes and the row mirror
// the two halves of a row (after the previous levels every lane of a block holds the same
// partial, so a mirror acts as an exchange).  Each level adds the same two operands on both
// partners, so every lane ends with the identical sum, and no value leaves the group.
template <int G>
__device__ __forceinline__ double gsum(double v) {
    static_assert(G == 8 || G == 16, "groups of 8 or 16 lanes");
    v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    if (G == 16) v += dpp_f64<0x140>(v);  // row_mirror
    return v;
}

// Minimum / maximum over the wave: DPP within rows (quad permutes, half-mirror, mirror), then
// two lane exchanges across rows.  Every lane ends with the result.
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <bool MAX>
__device__ __forceinline__ int wave_minmax(int v) {
    auto op = [](int a, int b) { return MAX ? max(a, b) : min(a, b); };
    v = op(v, dpp_i32<0xB1>(v));
    v = op(v, dpp_i32<0x4E>(v));
    v = op(v, dpp_i32<0x141>(v));
    v = op(v, dpp_i32<0x140>(v));
    v = op(v, __shfl_xor(v, 16, 64));
    v = op(v, __shfl_xor(v, 32, 64));
    return v;
}


// One MLS point, per lane of its G-lane group: lane k owns nodes k + G s (when < 27) of the
// 3x3x3 block around the nearest node.  mls_setup finds each node, its offset d = x_k - x,
// |d|^2 and whether it supports the point (|d| <= r_w); the caller then issues its field loads,
// and mls_solve builds and solves the moment system while those loads are in flight.
template <int G>
struct MlsLane {
    static constexpr int N = (27 + G - 1) / G;   // stencil nodes per lane
    bool active[N];
    int gx[N], gy[N], gz[N];
    double d0[N], d1[N], d2[N], r2[N];
    double phi[N];
    double gr[N][3];
};

template <int G>
__device__ __forceinline__ void mls_setup(const JobDev& J, const double xp[3], double rw2, int lane,
                                          MlsLane<G>& m, int& err) {
    constexpr int MLS_NODES = MlsLane<G>::N;
    const int c0 = (int)floor(xp[0] + 0.5), c1 = (int)floor(xp[1] + 0.5), c2 = (int)floor(xp[2] + 0.5);
    const int dims[3] = {J.nx, J.ny, J.nz};
    // the nearest node wrapped once per periodic axis; its neighbours then wrap by +-n
    int cw[3] = {c0, c1, c2};
    for (int a = 0; a < 3; ++a)
        if (J.bc[2 * a] == 0) {
            cw[a] %= dims[a];
            if (cw[a] < 0) cw[a] += dims[a];
        }
#pragma unroll
    for (int s = 0; s < MLS_NODES; ++s) {
        const int k = lane + G * s;
        m.active[s] = false;
        m.d0[s] = m.d1[s] = m.d2[s] = 0.0;
        m.r2[s] = 4.0 * rw2;
        m.gr[s][0] = m.gr[s][1] = m.gr[s][2] = 0.0;
        m.gx[s] = m.gy[s] = m.gz[s] = 0;
        if (k >= 27) continue;
        int nn[3] = {c0 + k % 3 - 1, c1 + (k / 3) % 3 - 1, c2 + k / 9 - 1};
        m.d0[s] = nn[0] - xp[0];
        m.d1[s] = nn[1] - xp[1];
        m.d2[s] = nn[2] - xp[2];
        m.r2[s] = m.d0[s] * m.d0[s] + m.d1[s] * m.d1[s] + m.d2[s] * m.d2[s];
        m.active[s] = m.r2[s] <= rw2;
        for (int a = 0; a < 3; ++a) {
            const int bc = J.bc[2 * a];
            if (bc == 0) {
                nn[a] = cw[a] + (a == 0 ? k % 3 - 1 : (a == 1 ? (k / 3) % 3 - 1 : k / 9 - 1));
                if (nn[a] < 0) nn[a] += dims[a];
                else if (nn[a] >= dims[a]) nn[a] -= dims[a];
            } else {
                const int lo = bc == 1 ? 1 : 0, hi = bc == 1 ? dims[a] - 2 : dims[a] - 1;
                if (nn[a] < lo || nn[a] > hi) {
                    if (m.active[s]) err |= FLAG_DOMAIN;
                    nn[a] = nn[a] < lo ? lo : hi;
                }
            }
        }
        m.gx[s] = nn[0]; m.gy[s] = nn[1]; m.gz[s] = nn[2];
    }
}

// 1/x in FP64: hardware reciprocal refined by two Newton steps (x > 0, normal).
__device__ __forceinline__ double rcp64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// Shape functions phi_k = [A^{-1} W_k p_k]_0 and (optionally) their gradients, A = sum W p p^T,
// p = (1, d), W = exp(-(|d| / (r_w alpha))^2) (Eqs. l2norm, intKernel).  The weights are
// evaluated in FP32; the moment matrix is accumulated and factorised (A = L D L^T, unit L) in
// FP64 on every lane.
template <int G>
__device__ __forceinline__ void mls_solve(MlsLane<G>& m, float wq, bool want_grad, int& err) {
    constexpr int MLS_NODES = MlsLane<G>::N;
    double W[MLS_NODES];
    double s00 = 0, s01 = 0, s02 = 0, s03 = 0, s11 = 0, s12 = 0, s13 = 0, s22 = 0, s23 = 0, s33 = 0;
#pragma unroll
    for (int s = 0; s < MLS_NODES; ++s) {
        W[s] = m.active[s] ? (double)expf(-wq * (float)m.r2[s]) : 0.0;
        const double w = W[s], d0 = m.d0[s], d1 = m.d1[s], d2 = m.d2[s];
        s00 += w; s01 += w * d0; s02 += w * d1; s03 += w * d2;
        s11 += w * d0 * d0; s12 += w * d0 * d1; s13 += w * d0 * d2;
        s22 += w * d1 * d1; s23 += w * d1 * d2; s33 += w * d2 * d2;
    }
    const double a00 = gsum<G>(s00), a01 = gsum<G>(s01), a02 = gsum<G>(s02), a03 = gsum<G>(s03);
    const double a11 = gsum<G>(s11), a12 = gsum<G>(s12), a13 = gsum<G>(s13);
    const double a22 = gsum<G>(s22), a23 = gsum<G>(s23), a33 = gsum<G>(s33);
    // A = L D L^T
    const double e0 = a00;
    if (!(e0 > 0.0)) err |= FLAG_NONFINITE;
    const double i0 = rcp64(e0);
    const double l10 = a01 * i0, l20 = a02 * i0, l30 = a03 * i0;
    const double e1 = a11 - l10 * a01;
    if (!(e1 > 0.0)) err |= FLAG_NONFINITE;
    const double i1 = rcp64(e1);
    const double b21 = a12 - l20 * a01, b31 = a13 - l30 * a01;   // D-scaled column entries
    const double l21 = b21 * i1, l31 = b31 * i1;
    const double e2 = a22 - l20 * a02 - l21 * b21;
    if (!(e2 > 0.0)) err |= FLAG_NONFINITE;
    const double i2 = rcp64(e2);
    const double b32 = a23 - l30 * a02 - l31 * b21;
    const double l32 = b32 * i2;
    const double e3 = a33 - l30 * a03 - l31 * b31 - l32 * b32;
    if (!(e3 > 0.0)) err |= FLAG_NONFINITE;
    const double i3 = rcp64(e3);
#pragma unroll
    for (int s = 0; s < MLS_NODES; ++s) {
        // v = A^{-1} p_k: L y = p, z = D^{-1} y, L^T v = z
        const double y0 = 1.0;
        const double y1 = m.d0[s] - l10 * y0;
        const double y2 = m.d1[s] - l20 * y0 - l21 * y1;
        const double y3 = m.d2[s] - l30 * y0 - l31 * y1 - l32 * y2;
        const double v3 = y3 * i3;
        const double v2 = y2 * i2 - l32 * v3;
        const double v1 = y1 * i1 - l21 * v2 - l31 * v3;
        const double v0 = y0 * i0 - l10 * v1 - l20 * v2 - l30 * v3;
        m.phi[s] = W[s] * v0;
        if (want_grad) { m.gr[s][0] = W[s] * v1; m.gr[s][1] = W[s] * v2; m.gr[s][2] = W[s] * v3; }
    }
}

// Window-local index of a node, or -1 if outside.
__device__ __forceinline__ long long win_index(const JobDev& J, const WinDesc& d, int gx, int gy,
                                               int gz) {
    if (d.w[0] < 1 || d.w[1] < 1 || d.w[2] < 1 || d.w[0] > J.nx || d.w[1] > J.ny || d.w[2] > J.nz)
        return -1;
    int lx = gx - d.o[0], ly = gy - d.o[1], lz = gz - d.o[2];
    if (lx < 0) lx += J.nx;
    if (ly < 0) ly += J.ny;
    if (lz < 0) lz += J.nz;
    if (lx >= d.w[0] || ly >= d.w[1] || lz >= d.w[2]) return -1;
    return lx + (long long)d.w[0] * (ly + (long long)d.w[1] * lz);
}

// Moments (rho - 1, u*) of the lane's active stencil nodes from the body's moment window.
// md: the layout of the moment window, which callers load with their other early reads
template <int G>
__device__ __forceinline__ void mls_moments(const Pools& P, const JobDev& J, const BodyDev& B, const WinDesc& md,
                                            const MlsLane<G>& m, float4 mom[MlsLane<G>::N], int& err) {
    constexpr int MLS_NODES = MlsLane<G>::N;
#pragma unroll
    for (int s = 0; s < MLS_NODES; ++s) {
        mom[s] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (!m.active[s]) continue;
        const long long l = win_index(J, md, m.gx[s], m.gy[s], m.gz[s]);
        if (l < 0) err |= FLAG_WINDOW;
        else mom[s] = P.mwin[B.win_off + l];
    }
}

// sum_k c_k q_k over the group for per-node coefficients c (phi or a gradient row) and field
// values q (component `comp` of the moments: 0 rho - 1, 1..3 u*)
template <int G>
__device__ __forceinline__ double group_dot(const double* c, int cstride, const float4 mom[MlsLane<G>::N],
                                            int comp) {
    constexpr int MLS_NODES = MlsLane<G>::N;
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < MLS_NODES; ++s) {
        const float q = comp == 0 ? mom[s].x : (comp == 1 ? mom[s].y : (comp == 2 ? mom[s].z : mom[s].w));
        acc += c[s * cstride] * (double)q;
    }
    return gsum<G>(acc);
}

__device__ __forceinline__ void load3(const double* p, double v[3]) { v[0] = p[0]; v[1] = p[1]; v[2] = p[2]; }
__device__ __forceinline__ void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Deterministic per-body totals.  Every block of a body stores its partial sums (up to six
// values, one row per value in the body's region); one block per body folds them in a later
// launch, whose boundary makes the partials visible without a per-block device-scope release
// (each of which would write back an L2).  Thread t takes blocks t, t+512, ... in order, then a
// fixed tree (DPP within each wave, the eight waves in order) combines the 512 results: the
// order depends only on the body's own block count, so totals are bitwise reproducible and
// independent of other jobs in the launch.
constexpr int FOLD_MAX = 6;
constexpr int FOLD_THREADS = 512;   // threads of the fold block: 2048 partials per load round

// A body's partials: value i of block k at 16 red_slot + i stride + k, stride = the body's larger
// block count (its region holds 16 such rows), so a wave of the fold reads value i of 64
// consecutive blocks from consecutive addresses.
__device__ __forceinline__ long long partial_stride(const BodyDev& B) { return max(B.nblk_c, B.nblk_t); }
__device__ __forceinline__ void store_partials(const Pools& P, const BodyDev& B, int blk, const double* v,
                                               int nval) {
    double* row = P.partial + 16LL * B.red_slot + blk;
    const long long st = partial_stride(B);
    for (int i = 0; i < nval; ++i) row[i * st] = v[i];
}

template <int NVAL>
__device__ void fold_partials(const Pools& P, const BodyDev& B, int nblk, double* out) {
    __shared__ double s_red[FOLD_MAX][FOLD_THREADS / 64];
    const int t = threadIdx.x;
    double acc[NVAL];
    for (int i = 0; i < NVAL; ++i) acc[i] = 0.0;
    // four slots per round, loaded together; summed in ascending block order
    const double* rows = P.partial + 16LL * B.red_slot;
    const long long st = partial_stride(B);
    for (int k0 = t; k0 < nblk; k0 += 4 * FOLD_THREADS) {
        double v[4][NVAL];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + u * FOLD_THREADS;
            const double* col = rows + (k < nblk ? k : 0);
#pragma unroll
            for (int i = 0; i < NVAL; ++i) v[u][i] = col[i * st];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (k0 + u * FOLD_THREADS < nblk)
#pragma unroll
                for (int i = 0; i < NVAL; ++i) acc[i] += v[u][i];
    }
    // each wave sums its 64 lanes (rows by DPP, then the four rows by two exchanges), wave 0's
    // first lane adds the waves in order: a fixed tree, so the totals are reproducible
    const int wave = t / 64, lane = t % 64;
#pragma unroll
    for (int i = 0; i < NVAL; ++i) {
        double v = gsum<16>(acc[i]);
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if (lane == 0) s_red[i][wave] = v;
    }
    __syncthreads();
    for (int i = 0; i < NVAL; ++i) {
        double v = s_red[i][0];
        for (int w = 1; w < FOLD_THREADS / 64; ++w) v += s_red[i][w];
        out[i] = v;
    }
}

// ---------------------------------------------------------------- window of a step
// Force window = integer bounding box of the vertices plus WIN_MARGIN on each side, wrapped on
// periodic axes, clipped on walled axes, never larger than the reserved capacity.
__device__ __forceinline__ WinDesc window_from_box(const JobDev& J, const BodyDev& B, const int* bmin,
                                                   const int* bmax, int& flag) {
    WinDesc d;
    const int dims[3] = {J.nx, J.ny, J.nz};
    for (int a = 0; a < 3; ++a) {
        int l = bmin[a] - WIN_MARGIN, h = bmax[a] + WIN_MARGIN;
        if (h < l) { flag |= FLAG_NONFINITE; l = 0; h = 0; }
        if (J.bc[2 * a] == 0) {
            const int w = h - l + 1;
            if (w >= dims[a]) { d.o[a] = 0; d.w[a] = dims[a]; }
            else { int o = l % dims[a]; if (o < 0) o += dims[a]; d.o[a] = o; d.w[a] = w; }
        } else {
            if (l < 0) l = 0;
            if (h > dims[a] - 1) h = dims[a] - 1;
            d.o[a] = l < dims[a] ? l : dims[a] - 1;
            d.w[a] = h >= l ? h - l + 1 : 1;
        }
        if (d.w[a] > B.win_cap[a]) { flag |= FLAG_WINDOW; d.w[a] = B.win_cap[a]; }
        if (d.w[a] < 1) d.w[a] = 1;
    }
    return d;
}

// ---------------------------------------------------------------- hinge forces
// Spring (Eq. strainFor) on the edge x1-x2 and bending -k_b sin(theta - theta0) dtheta/dx_r on
// the four hinge vertices, theta the signed angle between the outward normals of (x1,x2,x3)
// and (x2,x1,x4) about x1->x2.  out[0..2] = spring force on x1 (x2 gets the opposite),
// out[3+3r..] = bending force on vertex r.
__device__ void hinge_forces(const Pools& P, const BodyDev& B, int e, double out[15]) {
    const int* hv = P.hinge + 4 * (B.e0 + e);
    double x1[3], x2[3], x3[3], x4[3];
    load3(P.x + 3 * (B.v0 + hv[0]), x1);
    load3(P.x + 3 * (B.v0 + hv[1]), x2);
    load3(P.x + 3 * (B.v0 + hv[2]), x3);
    load3(P.x + 3 * (B.v0 + hv[3]), x4);
    double e12[3], p3[3], p4[3], q[3];
    for (int a = 0; a < 3; ++a) { e12[a] = x2[a] - x1[a]; p3[a] = x3[a] - x1[a]; p4[a] = x4[a] - x2[a]; q[a] = -e12[a]; }
    const double le2 = dot3(e12, e12), le = sqrt(le2);
    const double sp = -P.ks[B.e0 + e] * (le - P.l0[B.e0 + e]) / le;
    for (int a = 0; a < 3; ++a) out[a] = -sp * e12[a];   // r_12 = x1 - x2 = -e12
    if (B.kb == 0.0) {
        for (int i = 3; i < 15; ++i) out[i] = 0.0;
        return;
    }
    double N1[3], N2[3], c12[3];
    cross3(e12, p3, N1);
    cross3(q, p4, N2);
    const double a1 = sqrt(dot3(N1, N1)), a2 = sqrt(dot3(N2, N2));
    const double n1[3] = {N1[0] / a1, N1[1] / a1, N1[2] / a1};
    const double n2[3] = {N2[0] / a2, N2[1] / a2, N2[2] / a2};
    cross3(n1, n2, c12);
    const double theta = atan2(dot3(c12, e12) / le, dot3(n1, n2));
    // opposite vertices rotate their triangle about the edge with lever arm = height over it;
    // the edge vertices carry the reaction split at each opposite vertex's foot point
    const double h3 = a1 / le, h4 = a2 / le;
    const double d4[3] = {x4[0] - x1[0], x4[1] - x1[1], x4[2] - x1[2]};
    const double t3 = dot3(p3, e12) / le2, t4 = dot3(d4, e12) / le2;
    const double sb = -B.kb * sin(theta - P.theta0[B.e0 + e]);
    for (int a = 0; a < 3; ++a) {
        const double g3 = -n1[a] / h3, g4 = -n2[a] / h4;
        out[3 + a] = sb * ((t3 - 1.0) * g3 + (t4 - 1.0) * g4);
        out[6 + a] = sb * (-t3 * g3 - t4 * g4);
        out[9 + a] = sb * g3;
        out[12 + a] = sb * g4;
    }
}

// ---------------------------------------------------------------- fixed point
// Round to nearest even into int64, as __double2ll_rn, without its software sequence: for
// |v| < 2^51, v + 1.5 * 2^52 lies in [2^52, 2^53), where the addition itself rounds v to an
// integer in the low mantissa bits.  The addition must not be fused with the product that
// formed v.
__device__ __forceinline__ long long fix_rn(double v) {
#pragma clang fp contract(off)
    if (!(fabs(v) < 2251799813685248.0)) return __double2ll_rn(v);
    const double t = v + 6755399441055744.0;
    return __double_as_longlong(t) - 0x4338000000000000LL;
}

// ---------------------------------------------------------------- spreading
// The markers of a block are neighbours on the mesh, so their stencils overlap: about 9 active
// nodes per marker, but far fewer distinct nodes per marker over the block.  The
// block therefore sums its contributions in LDS first (int64, so the order cannot change the
// sum) and sends one global atomic per distinct node and component.  The LDS box is the
// bounding box of the block's 3x3x3 stencils in unwrapped node coordinates; a block whose box
// exceeds SPREAD_LDS_NODES (markers far apart on the lattice) adds straight to global memory.
//
// With fold set, the same block-wide reduction also folds the integer boxes that the vertex
// blocks wrote for x^n into this step's force window (min / max, order independent): every
// block derives the same descriptor and block 0 publishes it for the sweep and the moments.
// vb[6] is the box of the vertex-block boxes this thread loaded.
// Without fold, fd_in is the window the window kernel of the previous step published.
constexpr int SPREAD_LDS_NODES = 256;

template <int G>
__device__ __forceinline__ void spread_block(const Pools& P, const JobDev& J, const BodyDev& B, int b,
                                             int blk, bool fold, const int vb[6], const WinDesc& fd_in,
                                             bool live, const int cen_node[3], const MlsLane<G>& m,
                                             int lane, const long long fx[MlsLane<G>::N][3], int& err) {
    constexpr int MLS_NODES = MlsLane<G>::N;
    static_assert(IB_BLOCK == 64, "the block is one wave: its boxes are wave reductions");
    __shared__ long long s_acc[3][SPREAD_LDS_NODES];
    const long long capn = (long long)B.win_cap[0] * B.win_cap[1] * B.win_cap[2];
    unsigned long long* fw0 = (unsigned long long*)(P.fwin + 3 * B.win_off);
    // stencil box of the live markers; with fold, the box of the vertex-block boxes
    int o[3], w[3], bmin[3], bmax[3];
    bool small = true;   // every side within the LDS box (also keeps the volume from overflowing)
    for (int a = 0; a < 3; ++a) {
        const int l = wave_minmax<false>(live ? cen_node[a] - 1 : 0x3fffffff);
        const int h = wave_minmax<true>(live ? cen_node[a] + 1 : -0x3fffffff);
        o[a] = l;
        w[a] = h >= l ? h - l + 1 : 1;
        small = small && w[a] <= SPREAD_LDS_NODES;
        if (fold) {
            bmin[a] = wave_minmax<false>(vb[a]);
            bmax[a] = wave_minmax<true>(vb[3 + a]);
        }
    }
    WinDesc fd = fd_in;
    if (fold) {
        fd = window_from_box(J, B, bmin, bmax, err);
        if (blk == 0 && threadIdx.x == 0) P.fdesc[b] = fd;
    }
    const int vol = small ? w[0] * w[1] * w[2] : SPREAD_LDS_NODES + 1;
    const bool use_lds = vol <= SPREAD_LDS_NODES;   // uniform over the block
    if (use_lds) {
        for (int i = threadIdx.x; i < vol; i += blockDim.x) s_acc[0][i] = s_acc[1][i] = s_acc[2][i] = 0;
        __syncthreads();
    }
    if (live) {
#pragma unroll
        for (int sn = 0; sn < MLS_NODES; ++sn) {
            if (!m.active[sn]) continue;
            const long long l = win_index(J, fd, m.gx[sn], m.gy[sn], m.gz[sn]);
            if (l < 0) {
                err |= FLAG_WINDOW;
                continue;
            }
            if (use_lds) {
                const int k = lane + G * sn;
                const int li = (cen_node[0] + k % 3 - 1 - o[0]) +
                               w[0] * ((cen_node[1] + (k / 3) % 3 - 1 - o[1]) + w[1] * (cen_node[2] + k / 9 - 1 - o[2]));
                for (int c = 0; c < 3; ++c)
                    if (fx[sn][c]) atomicAdd((unsigned long long*)&s_acc[c][li], (unsigned long long)fx[sn][c]);
            } else {
                for (int c = 0; c < 3; ++c)
                    if (fx[sn][c]) atomicAdd(fw0 + c * capn + l, (unsigned long long)fx[sn][c]);
            }
        }
    }
    if (!use_lds) return;
    __syncthreads();
    const int dims[3] = {J.nx, J.ny, J.nz};
    for (int i = threadIdx.x; i < vol; i += blockDim.x) {
        const long long v0 = s_acc[0][i], v1 = s_acc[1][i], v2 = s_acc[2][i];
        if (!(v0 | v1 | v2)) continue;
        // back to wrapped lattice coordinates; only nodes with a window index received sums
        // (a support node beyond a wall has already raised the domain error; it is dropped)
        int g[3] = {o[0] + i % w[0], o[1] + (i / w[0]) % w[1], o[2] + i / (w[0] * w[1])};
        bool inside = true;
        for (int a = 0; a < 3; ++a) {
            if (J.bc[2 * a] == 0) { g[a] %= dims[a]; if (g[a] < 0) g[a] += dims[a]; }
            else if (g[a] < 0 || g[a] >= dims[a]) inside = false;
        }
        const long long l = inside ? win_index(J, fd, g[0], g[1], g[2]) : -1;
        if (l < 0) continue;
        if (v0) atomicAdd(fw0 + l, (unsigned long long)v0);
        if (v1) atomicAdd(fw0 + capn + l, (unsigned long long)v1);
        if (v2) atomicAdd(fw0 + 2 * capn + l, (unsigned long long)v2);
    }
}

// ---------------------------------------------------------------- centroids (+ hinges)
// Batched launches ask for four waves per SIMD, as the probe kernel does (128 VGPRs, a 52 B spill).
template <bool SOLO, int G>
__global__ void __launch_bounds__(IB_BLOCK, SOLO ? 1 : 4) k_centroids(Pools P, int nblk_tri, int fold) {
    constexpr int MLS_NODES = MlsLane<G>::N, MLS_PER_BLOCK = IB_BLOCK / G;
    if ((int)blockIdx.x >= nblk_tri) {
        // edge blocks: one thread per hinge of a membrane
        const int eb = blockIdx.x - nblk_tri;
        const int b = block_body<SOLO>(P, P.blk_body_e, eb);
        const BodyDev& B = body_of<SOLO>(P, b);
        const int e = (eb - B.blk_e0) * IB_BLOCK + threadIdx.x;
        if (e >= B.ne) return;
        double f[15];
        hinge_forces(P, B, e, f);
        double* o = P.fedge + 15LL * (B.e0 + e);
        for (int i = 0; i < 15; ++i) o[i] = f[i];
        return;
    }
    const int b = block_body<SOLO>(P, P.blk_body_c, blockIdx.x);
    const BodyDev& B = body_of<SOLO>(P, b);
    const JobDev& J = body_job<SOLO>(P, B);
    BodyState& S = P.bstate[b];
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    const int blk = blockIdx.x - B.blk_c0;
    const int t = blk * MLS_PER_BLOCK + grp;
    const bool live = t < B.nt;
    __shared__ double vol[MLS_PER_BLOCK];
    int err = 0;
    // everything this block reads before its MLS work is loaded first, so that the latencies
    // overlap: the vertex-block boxes of x^n (fold) or the published window, the triangle's
    // vertices and the desired-velocity inputs
    int vb[6] = {0x7fffffff, 0x7fffffff, 0x7fffffff, -0x7fffffff, -0x7fffffff, -0x7fffffff};
    WinDesc fd_pub = {};
    const WinDesc md = P.mdesc[b];
    if (fold) {
        // every vertex-block box, loaded now so that these loads overlap the MLS work
        for (int q = threadIdx.x; q < B.nblk_v; q += blockDim.x) {
            const int* e = P.vbox + 6LL * (B.vbox0 + q);
            for (int a = 0; a < 3; ++a) { vb[a] = min(vb[a], e[a]); vb[3 + a] = max(vb[3 + a], e[3 + a]); }
        }
    } else {
        fd_pub = P.fdesc[b];
    }
    double xa[3] = {0, 0, 0}, xb_[3] = {0, 0, 0}, xc[3] = {0, 0, 0}, Ub[3] = {0, 0, 0};
    if (live) {
        const int* tv = P.tri + 3 * (B.t0 + t);
        load3(P.x + 3 * (B.v0 + tv[0]), xa);
        load3(P.x + 3 * (B.v0 + tv[1]), xb_);
        load3(P.x + 3 * (B.v0 + tv[2]), xc);
        if (!B.rigid)
            for (int a = 0; a < 3; ++a)
                Ub[a] = (P.uv[3 * (B.v0 + tv[0]) + a] + P.uv[3 * (B.v0 + tv[1]) + a] +
                         P.uv[3 * (B.v0 + tv[2]) + a]) * (1.0 / 3.0);
    }
    double Vt = 0.0;
    int cen_node[3] = {0, 0, 0};               // node nearest to the centroid (unwrapped)
    long long fx[MLS_NODES][3] = {};           // fixed-point force of each stencil node
    MlsLane<G> m;
    if (live) {
        double cen[3], ab[3], ac[3], N[3];
        for (int a = 0; a < 3; ++a) {
            cen[a] = (xa[a] + xb_[a] + xc[a]) * (1.0 / 3.0);
            ab[a] = xb_[a] - xa[a];
            ac[a] = xc[a] - xa[a];
        }
        cross3(ab, ac, N);
        const double A = 0.5 * sqrt(dot3(N, N));
        if (lane == 0) {
            // geometry at x^n for the probes of this step
            double* g = P.tgeo + 6 * (B.t0 + t);
            for (int a = 0; a < 3; ++a) { g[a] = cen[a]; g[3 + a] = N[a]; }
        }
        if (!B.rigid && B.kv != 0.0) {
            // signed volume of the tetrahedron (r, a, b, c), r = vertex 0 of the body
            double r0[3], pa[3], pb[3], pc[3], bc[3];
            load3(P.x + 3 * B.v0, r0);
            for (int a = 0; a < 3; ++a) { pa[a] = xa[a] - r0[a]; pb[a] = xb_[a] - r0[a]; pc[a] = xc[a] - r0[a]; }
            cross3(pb, pc, bc);
            Vt = dot3(pa, bc) * (1.0 / 6.0);
        }
        mls_setup<G>(J, cen, B.rw2, lane, m, err);
        for (int a = 0; a < 3; ++a) cen_node[a] = (int)floor(cen[a] + 0.5);
        float4 mom[MLS_NODES];
        // a lone body's launch is a latency chain: its moment loads go out before the solve; a
        // batched launch is throughput-bound and loads them after it, to hold fewer registers
        if (SOLO) mls_moments<G>(P, J, B, md, m, mom, err);
        mls_solve<G>(m, B.wq, false, err);
        if (!SOLO) mls_moments<G>(P, J, B, md, m, mom, err);
        const double U0 = group_dot<G>(m.phi, 1, mom, 1);
        const double U1 = group_dot<G>(m.phi, 1, mom, 2);
        const double U2 = group_dot<G>(m.phi, 1, mom, 3);
        // desired boundary velocity U_b (Sec. 1.2): membranes average their vertex velocities,
        // rigid bodies move the marker with the body
        if (B.rigid) {
            double rr[3] = {cen[0] - S.X[0], cen[1] - S.X[1], cen[2] - S.X[2]}, w[3];
            cross3(S.om, rr, w);
            for (int a = 0; a < 3; ++a) Ub[a] = S.u[a] + w[a];
        }
        // F_l = (U_b - U*) / dt, spread with c_l = A_l h (Eq. bodyforce), as int64 fixed point
#pragma unroll
        for (int sn = 0; sn < MLS_NODES; ++sn) {
            if (!m.active[sn]) continue;
            const double sc = A * B.shell_h * m.phi[sn];
            fx[sn][0] = fix_rn(sc * (Ub[0] - U0) * FIX_SCALE);
            fx[sn][1] = fix_rn(sc * (Ub[1] - U1) * FIX_SCALE);
            fx[sn][2] = fix_rn(sc * (Ub[2] - U2) * FIX_SCALE);
        }
    }
    spread_block<G>(P, J, B, b, blk, fold != 0, vb, fd_pub, live, cen_node, m, lane, fx, err);
    if (err) atomicOr(P.flags + B.job, err);
    if (B.rigid || B.kv == 0.0) return;
    if (lane == 0) vol[grp] = Vt;
    __syncthreads();
    double sv = 0.0;
    for (int g = 0; g < MLS_PER_BLOCK; ++g) sv += vol[g];
    if (threadIdx.x == 0) store_partials(P, B, blk, &sv, 1);   // folded into V by k_fold_bodies
}

// ---------------------------------------------------------------- vertex velocities
// Fluid velocity at every membrane vertex from the moments of f^{n+1} (the tentative velocity
// of Eq. verletPos).  It needs nothing from the probes, so its blocks ride in the probe launch
// and the vertex kernel only gathers forces and moves the vertices.  One group per vertex.
template <bool SOLO, int G>
__device__ void vertex_velocity_block(const Pools& P, int vb) {
    constexpr int MLS_NODES = MlsLane<G>::N, MLS_PER_BLOCK = IB_BLOCK / G;
    const int b = block_body<SOLO>(P, P.blk_body_u, vb);
    const BodyDev& B = body_of<SOLO>(P, b);
    if (B.rigid) return;
    const JobDev& J = body_job<SOLO>(P, B);
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    const int v = (vb - B.blk_u0) * MLS_PER_BLOCK + grp;
    if (v >= B.nv) return;
    const long long gv = B.v0 + v;
    int err = 0;
    double x[3];
    load3(P.x + 3 * gv, x);
    const WinDesc md = P.mdesc[b];
    MlsLane<G> m;
    float4 mom[MLS_NODES];
    mls_setup<G>(J, x, B.rw2, lane, m, err);
    mls_moments<G>(P, J, B, md, m, mom, err);
    mls_solve<G>(m, B.wq, false, err);
    const double u0 = group_dot<G>(m.phi, 1, mom, 1), u1 = group_dot<G>(m.phi, 1, mom, 2),
                 u2 = group_dot<G>(m.phi, 1, mom, 3);
    if (lane == 0) {
        P.u0v[3 * gv] = u0;
        P.u0v[3 * gv + 1] = u1;
        P.u0v[3 * gv + 2] = u2;
    }
    if (err) atomicOr(P.flags + B.job, err);
}

// ---------------------------------------------------------------- triangles (probes)
// Group 2k evaluates the outer probe of triangle k of the block, group 2k+1 the inner one.
// Blocks from nblk_tri on compute the vertex velocities instead.
// Four waves per SIMD: the compiler fits the kernel in 128 VGPRs (the batched form with a 20 B
// spill).  Batched launches are throughput-bound and gain the most; a lone body's launch gains
// where its markers outnumber a round of the chip (256x128x256), and loses nothing below.
template <bool SOLO, int G>
__global__ void __launch_bounds__(IB_BLOCK, 4) k_triangles(Pools P, int nblk_tri) {
    constexpr int MLS_NODES = MlsLane<G>::N, MLS_PER_BLOCK = IB_BLOCK / G, TRI_PER_BLOCK = MLS_PER_BLOCK / 2;
    if ((int)blockIdx.x >= nblk_tri) {
        vertex_velocity_block<SOLO, G>(P, blockIdx.x - nblk_tri);
        return;
    }
    const int b = block_body<SOLO>(P, P.blk_body_t, blockIdx.x);
    const BodyDev& B = body_of<SOLO>(P, b);
    const JobDev& J = body_job<SOLO>(P, B);
    BodyState& S = P.bstate[b];
    const int grp = threadIdx.x / G, lane = threadIdx.x % G;
    const int blk = blockIdx.x - B.blk_t0;
    const int k = grp >> 1, side = grp & 1;
    const int t = blk * TRI_PER_BLOCK + k;
    __shared__ double probe[MLS_PER_BLOCK][10];
    __shared__ double red[TRI_PER_BLOCK][6];
    const WinDesc md = P.mdesc[b];
    int err = 0;
    double cen[3] = {0, 0, 0}, N[3] = {0, 0, 0}, nrm[3] = {0, 0, 0}, A = 0.0;
    if (t < B.nt) {
        // centroid and normal at x^n, as the centroid kernel of this step computed them
        const double* g = P.tgeo + 6 * (B.t0 + t);
        for (int a = 0; a < 3; ++a) { cen[a] = g[a]; N[a] = g[3 + a]; }
        const double ln = sqrt(dot3(N, N));
        A = 0.5 * ln;
        for (int a = 0; a < 3; ++a) nrm[a] = N[a] / ln;
        const double sg = side == 0 ? 1.0 : -1.0;
        const double xp[3] = {cen[0] + sg * B.probe * nrm[0], cen[1] + sg * B.probe * nrm[1],
                              cen[2] + sg * B.probe * nrm[2]};
        MlsLane<G> m;
        mls_setup<G>(J, xp, B.rw2, lane, m, err);
        float4 mom[MLS_NODES];
        mls_moments<G>(P, J, B, md, m, mom, err);
        mls_solve<G>(m, B.wq, true, err);
        // interpolated rho - 1 and the gradient rows of u* (diffuse derivatives)
        double v[10];
        v[0] = group_dot<G>(m.phi, 1, mom, 0);
        for (int j = 0; j < 3; ++j) {
            v[1 + j] = group_dot<G>(&m.gr[0][j], 3, mom, 1);
            v[4 + j] = group_dot<G>(&m.gr[0][j], 3, mom, 2);
            v[7 + j] = group_dot<G>(&m.gr[0][j], 3, mom, 3);
        }
        if (lane == 0)
            for (int i = 0; i < 10; ++i) probe[grp][i] = v[i];
    }
    if (err) atomicOr(P.flags + B.job, err);
    __syncthreads();
    double Ft[3] = {0, 0, 0}, Mt[3] = {0, 0, 0};
    if (t < B.nt && side == 0 && lane == 0) {
        // p = c_s^2 rho, tau = rho nu (grad u + grad u^T); grad u [i][j] = probe[1 + 3 i + j]
        const double* pp = probe[grp];
        const double* pm = probe[grp + 1];
        const double nu = J.nu;
        const double rp = 1.0 + pp[0], rm = 1.0 + pm[0];
        const double dp = (pp[0] - pm[0]) * (1.0 / 3.0);
        for (int i = 0; i < 3; ++i) {
            double tn = 0.0;
            for (int j = 0; j < 3; ++j)
                tn += (rp * nu * (pp[1 + 3 * i + j] + pp[1 + 3 * j + i]) -
                       rm * nu * (pm[1 + 3 * i + j] + pm[1 + 3 * j + i])) * nrm[j];
            Ft[i] = (-dp * nrm[i] + tn) * A;
        }
        for (int i = 0; i < 3; ++i) P.fext[3 * (B.t0 + t) + i] = Ft[i];
        if (!B.rigid) {
            // volume penalty (Eq. volFor, restoring): k_v (1 - V/V0) n_t A_t, a third per vertex
            const double vs = B.kv == 0.0 ? 0.0 : B.kv * (1.0 - S.V / B.V0) * (1.0 / 6.0);
            for (int i = 0; i < 3; ++i) P.fvol[3 * (B.t0 + t) + i] = vs * N[i];
        } else {
            const double rr[3] = {cen[0] - S.X[0], cen[1] - S.X[1], cen[2] - S.X[2]};
            cross3(rr, Ft, Mt);
        }
    }
    if (!B.rigid) return;
    if (side == 0 && lane == 0)
        for (int i = 0; i < 3; ++i) { red[k][i] = Ft[i]; red[k][3 + i] = Mt[i]; }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double part[6] = {0, 0, 0, 0, 0, 0};
    for (int g = 0; g < TRI_PER_BLOCK; ++g)
        for (int i = 0; i < 6; ++i) part[i] += red[g][i];
    store_partials(P, B, blk, part, 6);   // folded, with the pose update, by k_fold_bodies
}

// Rigid body, Eqs. (linearVelRig), (angularVelRig), from the FP64 totals tot = (F, M).  Returns
// false for a non-finite or singular state.
__device__ bool rigid_update(const BodyDev& B, BodyState& S, const double tot[6]) {
    for (int i = 0; i < 3; ++i) { S.F[i] = tot[i]; S.M[i] = tot[3 + i]; }
    // Rigid body, Eqs. (linearVelRig), (angularVelRig): udot = F/m with net weight (m - V0) g,
    // omegadot = I_w^{-1} M with I_w = R I R^T.
    double F[3];
    for (int i = 0; i < 3; ++i) F[i] = tot[i] + (B.mass - B.V0) * B.gravity[i];
    double IR[9], Iw[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int q = 0; q < 3; ++q) s += B.Ib[3 * i + q] * S.R[3 * j + q];  // I R^T
            IR[3 * i + j] = s;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int q = 0; q < 3; ++q) s += S.R[3 * i + q] * IR[3 * q + j];
            Iw[3 * i + j] = s;
        }
    // omegadot = Iw^{-1} M by the adjugate
    const double c00 = Iw[4] * Iw[8] - Iw[5] * Iw[7], c01 = Iw[5] * Iw[6] - Iw[3] * Iw[8],
                 c02 = Iw[3] * Iw[7] - Iw[4] * Iw[6];
    const double c10 = Iw[2] * Iw[7] - Iw[1] * Iw[8], c11 = Iw[0] * Iw[8] - Iw[2] * Iw[6],
                 c12 = Iw[1] * Iw[6] - Iw[0] * Iw[7];
    const double c20 = Iw[1] * Iw[5] - Iw[2] * Iw[4], c21 = Iw[2] * Iw[3] - Iw[0] * Iw[5],
                 c22 = Iw[0] * Iw[4] - Iw[1] * Iw[3];
    const double det = Iw[0] * c00 + Iw[1] * c01 + Iw[2] * c02;
    const double* M = tot + 3;
    const double wd[3] = {(c00 * M[0] + c10 * M[1] + c20 * M[2]) / det,
                          (c01 * M[0] + c11 * M[1] + c21 * M[2]) / det,
                          (c02 * M[0] + c12 * M[1] + c22 * M[2]) / det};
    double un[3], wn[3];
    for (int i = 0; i < 3; ++i) {
        un[i] = (2.0 / 3.0) * (2.0 * S.u[i] - 0.5 * S.u1[i] + F[i] / B.mass);
        wn[i] = (2.0 / 3.0) * (2.0 * S.om[i] - 0.5 * S.om1[i] + wd[i]);
    }
    for (int i = 0; i < 3; ++i) {
        S.u1[i] = S.u[i]; S.u[i] = un[i];
        S.om1[i] = S.om[i]; S.om[i] = wn[i];
        S.X[i] += un[i];
    }
    // R <- Rot(omega dt) R (Rodrigues)
    const double th = sqrt(dot3(wn, wn));
    double Rw[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    if (th > 0.0) {
        const double kx = wn[0] / th, ky = wn[1] / th, kz = wn[2] / th;
        const double s = sin(th), c = 1.0 - cos(th);
        Rw[0] = 1.0 + c * (-ky * ky - kz * kz);  Rw[1] = -s * kz + c * kx * ky;  Rw[2] = s * ky + c * kx * kz;
        Rw[3] = s * kz + c * kx * ky;  Rw[4] = 1.0 + c * (-kx * kx - kz * kz);  Rw[5] = -s * kx + c * ky * kz;
        Rw[6] = -s * ky + c * kx * kz;  Rw[7] = s * kx + c * ky * kz;  Rw[8] = 1.0 + c * (-kx * kx - ky * ky);
    }
    double Rn[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int q = 0; q < 3; ++q) s += Rw[3 * i + q] * S.R[3 * q + j];
            Rn[3 * i + j] = s;
        }
    bool fin = isfinite(det) && det != 0.0;
    for (int i = 0; i < 9; ++i) { S.R[i] = Rn[i]; fin = fin && isfinite(Rn[i]); }
    for (int i = 0; i < 3; ++i) fin = fin && isfinite(S.X[i]) && isfinite(un[i]) && isfinite(wn[i]);
    return fin;
}

// ---------------------------------------------------------------- per-body totals
// One block per body.  mode 0 (after the centroid kernel): enclosed volume V^n of membranes
// with a volume penalty; mode 1 (after the probe kernel): hydrodynamic totals and the velocity
// / pose update of rigid bodies.  Other bodies return at once.
__global__ void __launch_bounds__(FOLD_THREADS) k_fold_bodies(Pools P, int mode) {
    const int b = blockIdx.x;
    const BodyDev& B = P.bodies[b];
    if (B.nv == 0) return;   // an empty slot of a slotted batch
    if (mode == 0 ? (B.rigid || B.kv == 0.0) : !B.rigid) return;
    double tot[FOLD_MAX];
    if (mode == 0) fold_partials<1>(P, B, B.nblk_c, tot);
    else fold_partials<6>(P, B, B.nblk_t, tot);
    if (threadIdx.x != 0) return;
    if (mode == 0) { P.bstate[b].V = tot[0]; return; }
    // the state and the body constants are read into registers at once and stored once
    const BodyDev Bc = B;
    BodyState S = P.bstate[b];
    const bool fin = rigid_update(Bc, S, tot);
    P.bstate[b] = S;
    if (!fin) atomicOr(P.flags + Bc.job, FLAG_NONFINITE);
}

// ---------------------------------------------------------------- vertices
__device__ __forceinline__ int box_lo(double v) { return (int)floor(fmin(fmax(v, -1e7), 1e7)); }
__device__ __forceinline__ int box_hi(double v) { return (int)ceil(fmin(fmax(v, -1e7), 1e7)); }

template <bool SOLO>
__global__ void __launch_bounds__(VERT_BLOCK) k_vertices(Pools P) {
    const int b = block_body<SOLO>(P, P.blk_body_v, blockIdx.x);
    const BodyDev& B = body_of<SOLO>(P, b);
    const JobDev& J = body_job<SOLO>(P, B);
    BodyState& S = P.bstate[b];
    const int grp = threadIdx.x / VERT_GROUP, lane = threadIdx.x % VERT_GROUP;
    const int blk = blockIdx.x - B.blk_v0;
    const int v = blk * VERT_PER_BLOCK + grp;
    __shared__ int box[VERT_PER_BLOCK][6];
    int err = 0;
    int bl[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, bh[3] = {-0x7fffffff, -0x7fffffff, -0x7fffffff};
    if (v < B.nv) {
        const long long gv = B.v0 + v;
        // incidence entries first (lane j holds entry j when the lists fit in a group), so
        // that the force loads they address go out together with the moment loads
        const bool one = B.vt_w <= VERT_GROUP && B.vh_w <= VERT_GROUP;
        int tl0 = -1, hc0 = -1;
        if (one) {
            if (lane < B.vt_w) tl0 = P.vt_list[B.vt_off + (long long)v * B.vt_w + lane];
            if (!B.rigid && lane < B.vh_w) hc0 = P.vh_list[B.vh_off + (long long)v * B.vh_w + lane];
        }
        double x[3], xn[3], u0[3] = {0.0, 0.0, 0.0};
        load3(P.x + 3 * gv, x);
        if (!B.rigid) load3(P.u0v + 3 * gv, u0);   // fluid velocity, from the probe launch
        // gathered forces: a third of each incident triangle's probe force, its volume force,
        // the spring and bending forces of every incident hinge; lane j takes entry j
        double f[3] = {0.0, 0.0, 0.0};
        auto add_tri = [&](int tl) {
            const long long t = B.t0 + tl;
            for (int a = 0; a < 3; ++a) f[a] += P.fext[3 * t + a] * (1.0 / 3.0);
            if (!B.rigid)
                for (int a = 0; a < 3; ++a) f[a] += P.fvol[3 * t + a];
        };
        auto add_hinge = [&](int code) {
            const double* fe = P.fedge + 15LL * (B.e0 + (code >> 2));
            const int role = code & 3;
            const double sgn = role == 0 ? 1.0 : (role == 1 ? -1.0 : 0.0);
            for (int a = 0; a < 3; ++a) f[a] += sgn * fe[a] + fe[3 + 3 * role + a];
        };
        if (one) {
            if (tl0 >= 0) add_tri(tl0);
            if (hc0 >= 0) add_hinge(hc0);
        } else {
            for (int j = lane; j < B.vt_w; j += VERT_GROUP) {
                const int tl = P.vt_list[B.vt_off + (long long)v * B.vt_w + j];
                if (tl >= 0) add_tri(tl);
            }
            if (!B.rigid)
                for (int j = lane; j < B.vh_w; j += VERT_GROUP) {
                    const int code = P.vh_list[B.vh_off + (long long)v * B.vh_w + j];
                    if (code >= 0) add_hinge(code);
                }
        }
        const double F0 = gsum<VERT_GROUP>(f[0]), F1 = gsum<VERT_GROUP>(f[1]), F2 = gsum<VERT_GROUP>(f[2]);
        if (!B.rigid) {
            // tentative velocity u0: fluid velocity at the vertex from f^{n+1}
            const double Fv[3] = {F0, F1, F2};
            double un[3];
            for (int a = 0; a < 3; ++a) {
                const double acc = Fv[a] / B.mv;
                double dx;
                if (B.integrator == 1) {
                    // Eqs. (verletPos), (verletVel), (verletPos) as printed, in displacement form
                    un[a] = 1.5 * (u0[a] + 0.5 * acc) - 0.5 * (x[a] - P.xprev[3 * gv + a]);
                    dx = un[a] + 0.5 * acc;
                } else if (B.integrator == 2) {
                    // kinematic IB (Sec. 2.4): advected with the fluid velocity
                    un[a] = u0[a];
                    dx = un[a];
                } else {
                    // Eq. (verletPos); vertex velocity = displacement of the step
                    dx = u0[a] + 0.5 * acc;
                    un[a] = dx;
                }
                xn[a] = x[a] + dx;
            }
            if (lane == 0)
                for (int a = 0; a < 3; ++a) {
                    P.xprev[3 * gv + a] = x[a];
                    P.x[3 * gv + a] = xn[a];
                    P.uv[3 * gv + a] = un[a];
                    P.fv[3 * gv + a] = Fv[a];
                }
        } else {
            double xb[3], w[3];
            load3(P.xb + 3 * gv, xb);
            for (int a = 0; a < 3; ++a)
                xn[a] = S.X[a] + S.R[3 * a] * xb[0] + S.R[3 * a + 1] * xb[1] + S.R[3 * a + 2] * xb[2];
            const double rr[3] = {xn[0] - S.X[0], xn[1] - S.X[1], xn[2] - S.X[2]};
            cross3(S.om, rr, w);
            if (lane == 0)
                for (int a = 0; a < 3; ++a) {
                    P.xprev[3 * gv + a] = x[a];
                    P.x[3 * gv + a] = xn[a];
                    P.uv[3 * gv + a] = S.u[a] + w[a];
                    P.fv[3 * gv + a] = a == 0 ? F0 : (a == 1 ? F1 : F2);
                }
        }
        if (!(isfinite(xn[0]) && isfinite(xn[1]) && isfinite(xn[2])) ||
            fabs(xn[0]) > 1e7 || fabs(xn[1]) > 1e7 || fabs(xn[2]) > 1e7)
            err |= FLAG_NONFINITE;
        for (int a = 0; a < 3; ++a) { bl[a] = box_lo(xn[a]); bh[a] = box_hi(xn[a]); }
    }
    if (lane == 0)
        for (int a = 0; a < 3; ++a) { box[grp][a] = bl[a]; box[grp][3 + a] = bh[a]; }
    if (err) atomicOr(P.flags + B.job, err);
    __syncthreads();
    if (threadIdx.x == 0) {
        int* vb = P.vbox + 6LL * (B.vbox0 + blk);
        for (int a = 0; a < 3; ++a) {
            int lo = box[0][a], hi = box[0][3 + a];
            for (int g = 1; g < VERT_PER_BLOCK; ++g) { lo = min(lo, box[g][a]); hi = max(hi, box[g][3 + a]); }
            vb[a] = lo;
            vb[3 + a] = hi;
        }
    }
}

// ---------------------------------------------------------------- windows of the next step
// One block per body: fold the integer boxes of x^{n+1} the vertex blocks wrote and publish the
// force window of the next step (used for batches, where folding once per body is cheaper than
// once per centroid block).
__global__ void __launch_bounds__(256) k_windows(Pools P) {
    const int b = blockIdx.x;
    const BodyDev& B = P.bodies[b];
    if (B.nv == 0) return;   // an empty slot of a slotted batch
    const JobDev& J = P.jobs[B.job];
    __shared__ int red[6][256];
    const int t = threadIdx.x;
    int e[6] = {0x7fffffff, 0x7fffffff, 0x7fffffff, -0x7fffffff, -0x7fffffff, -0x7fffffff};
    for (int q = t; q < B.nblk_v; q += 256) {
        const int* vb = P.vbox + 6LL * (B.vbox0 + q);
        for (int a = 0; a < 3; ++a) { e[a] = min(e[a], vb[a]); e[3 + a] = max(e[3 + a], vb[3 + a]); }
    }
    for (int a = 0; a < 6; ++a) red[a][t] = e[a];
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w)
            for (int a = 0; a < 6; ++a)
                red[a][t] = a < 3 ? min(red[a][t], red[a][t + w]) : max(red[a][t], red[a][t + w]);
        __syncthreads();
    }
    if (t == 0) {
        int err = 0;
        const int bmin[3] = {red[0][0], red[1][0], red[2][0]}, bmax[3] = {red[3][0], red[4][0], red[5][0]};
        P.fdesc[b] = window_from_box(J, B, bmin, bmax, err);
        if (err) atomicOr(P.flags + B.job, err);
    }
}

// ---------------------------------------------------------------- reported totals (membranes)
// FP64 hydrodynamic force and torque of the last step, torque about the vertex mean of x^n
// (held in xprev after the update).  One block, fixed-shape tree: reproducible.
__global__ void __launch_bounds__(256) k_body_totals(Pools P, int b, double* out) {
    const BodyDev& B = P.bodies[b];
    __shared__ double red[7][256];
    const int t = threadIdx.x;
    double c[3] = {0, 0, 0};
    for (int v = t; v < B.nv; v += 256)
        for (int a = 0; a < 3; ++a) c[a] += P.xprev[3 * (B.v0 + v) + a];
    for (int a = 0; a < 3; ++a) red[a][t] = c[a];
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w) for (int a = 0; a < 3; ++a) red[a][t] += red[a][t + w];
        __syncthreads();
    }
    const double ctr[3] = {red[0][0] / B.nv, red[1][0] / B.nv, red[2][0] / B.nv};
    __syncthreads();
    double F[3] = {0, 0, 0}, M[3] = {0, 0, 0};
    for (int q = t; q < B.nt; q += 256) {
        const int* tv = P.tri + 3 * (B.t0 + q);
        double cen[3], f[3], m[3];
        for (int a = 0; a < 3; ++a) {
            cen[a] = (P.xprev[3 * (B.v0 + tv[0]) + a] + P.xprev[3 * (B.v0 + tv[1]) + a] +
                      P.xprev[3 * (B.v0 + tv[2]) + a]) * (1.0 / 3.0) - ctr[a];
            f[a] = P.fext[3 * (B.t0 + q) + a];
        }
        cross3(cen, f, m);
        for (int a = 0; a < 3; ++a) { F[a] += f[a]; M[a] += m[a]; }
    }
    for (int a = 0; a < 3; ++a) { red[a][t] = F[a]; red[3 + a][t] = M[a]; }
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w) for (int a = 0; a < 6; ++a) red[a][t] += red[a][t + w];
        __syncthreads();
    }
    if (t < 6) out[t] = red[t][0];
}

void launch_centroids(const Pools& P, int nblk_tri, int nblk_edge, bool fold, hipStream_t s) {
    if (!(nblk_tri + nblk_edge > 0)) return;
    const dim3 grid(nblk_tri + nblk_edge), block(IB_BLOCK);
    if (P.solo_job >= 0) hipLaunchKernelGGL((k_centroids<true, MLS_GROUP>), grid, block, 0, s, P, nblk_tri, (int)fold);
    else hipLaunchKernelGGL((k_centroids<false, MLS_GROUP>), grid, block, 0, s, P, nblk_tri, (int)fold);
}
void launch_windows(const Pools& P, int nbodies, hipStream_t s) {
    if (nbodies > 0) hipLaunchKernelGGL(k_windows, dim3(nbodies), dim3(256), 0, s, P);
}
void launch_fold_bodies(const Pools& P, int nbodies, int mode, hipStream_t s) {
    if (nbodies > 0) hipLaunchKernelGGL(k_fold_bodies, dim3(nbodies), dim3(FOLD_THREADS), 0, s, P, mode);
}

void launch_triangles(const Pools& P, int nblk_tri, int nblk_vel, hipStream_t s) {
    if (!(nblk_tri + nblk_vel > 0)) return;
    const dim3 grid(nblk_tri + nblk_vel), block(IB_BLOCK);
    if (P.solo_job >= 0) hipLaunchKernelGGL((k_triangles<true, MLS_GROUP>), grid, block, 0, s, P, nblk_tri);
    else hipLaunchKernelGGL((k_triangles<false, MLS_GROUP>), grid, block, 0, s, P, nblk_tri);
}
void launch_vertices(const Pools& P, int nblocks, hipStream_t s) {
    if (!(nblocks > 0)) return;
    if (P.solo_job >= 0) hipLaunchKernelGGL(k_vertices<true>, dim3(nblocks), dim3(VERT_BLOCK), 0, s, P);
    else hipLaunchKernelGGL(k_vertices<false>, dim3(nblocks), dim3(VERT_BLOCK), 0, s, P);
}
void launch_body_totals(const Pools& P, int body, double* out6, hipStream_t s) {
    hipLaunchKernelGGL(k_body_totals, dim3(1), dim3(256), 0, s, P, body, out6);
}

}  // namespace lbib
