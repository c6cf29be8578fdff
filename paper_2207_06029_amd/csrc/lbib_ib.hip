// Immersed-boundary and structure kernels (Secs. 1.2-1.3).
//
// One MLS point (triangle centroid, probe or vertex) is evaluated by a group of 32 lanes; lane
// k < 27 owns node k of the 3x3x3 block around the nearest node.  Every node within r_w of the
// point lies in that block, so the group covers the whole support of Eq. (intKernel).  The
// 4x4 moment matrix is accumulated and factorised in FP64 (every lane solves redundantly), so
// no lane waits on another except for the butterfly sums.
//
// Step order inside the time step n -> n+1:
//   k_centroids  geometry at x^n, MLS at centroids on moments of f^n, F_l = U_b - U*,
//                fixed-point spreading into the body's force window, enclosed volume V^n
//   (sweep)      collide+stream with the spread force
//   (moments)    moments of f^{n+1} in the body's window
//   k_triangles  probe stresses on f^{n+1} (Eqs. hydroForP, hydroForNu); rigid bodies: FP64
//                totals and the velocity / pose update in the last block
//   k_vertices   vertex velocity from the fluid, internal forces at x^n, membrane update;
//                bounding box of x^{n+1} -> force window of the next step
#include "lbib_internal.h"

namespace lbib {

__device__ __forceinline__ double gsum(double v) {
#pragma unroll
    for (int o = 16; o >= 1; o >>= 1) v += __shfl_xor(v, o, GROUP);
    return v;
}

__device__ __forceinline__ double agent_load(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Shape functions of one point.  Output per lane: active (W > 0), wrapped node coordinates,
// phi_k and (optionally) its gradient.  err receives FLAG_DOMAIN when a supporting node falls
// on or behind a wall.
struct MlsLane {
    bool active;
    int gx, gy, gz;
    double phi;
    double gr[3];
};

__device__ __forceinline__ void mls_point(const JobDev& J, const double xp[3], double rw,
                                          double alpha, int lane, bool want_grad, MlsLane& m,
                                          int& err) {
    const int c0 = (int)floor(xp[0] + 0.5), c1 = (int)floor(xp[1] + 0.5), c2 = (int)floor(xp[2] + 0.5);
    double W = 0.0, d0 = 0.0, d1 = 0.0, d2 = 0.0;
    m.active = false;
    int n0 = 0, n1 = 0, n2 = 0;
    if (lane < 27) {
        n0 = c0 + lane % 3 - 1;
        n1 = c1 + (lane / 3) % 3 - 1;
        n2 = c2 + lane / 9 - 1;
        d0 = n0 - xp[0];
        d1 = n1 - xp[1];
        d2 = n2 - xp[2];
        const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2) / rw;
        if (r <= 1.0) {
            const double q = r / alpha;
            W = exp(-q * q);
            m.active = true;
        }
    }
    if (m.active) {
        int nn[3] = {n0, n1, n2};
        const int dims[3] = {J.nx, J.ny, J.nz};
        for (int a = 0; a < 3; ++a) {
            const int bc = J.bc[2 * a];
            if (bc == 0) {
                nn[a] %= dims[a];
                if (nn[a] < 0) nn[a] += dims[a];
            } else {
                const int lo = bc == 1 ? 1 : 0, hi = bc == 1 ? dims[a] - 2 : dims[a] - 1;
                if (nn[a] < lo || nn[a] > hi) { err |= FLAG_DOMAIN; nn[a] = nn[a] < lo ? lo : hi; }
            }
        }
        m.gx = nn[0]; m.gy = nn[1]; m.gz = nn[2];
    }
    // A = sum W p p^T, p = (1, d)
    const double a00 = gsum(W), a01 = gsum(W * d0), a02 = gsum(W * d1), a03 = gsum(W * d2);
    const double a11 = gsum(W * d0 * d0), a12 = gsum(W * d0 * d1), a13 = gsum(W * d0 * d2);
    const double a22 = gsum(W * d1 * d1), a23 = gsum(W * d1 * d2), a33 = gsum(W * d2 * d2);
    // Cholesky A = L L^T
    const double l00 = sqrt(a00);
    const double l10 = a01 / l00, l20 = a02 / l00, l30 = a03 / l00;
    const double l11 = sqrt(a11 - l10 * l10);
    const double l21 = (a12 - l20 * l10) / l11, l31 = (a13 - l30 * l10) / l11;
    const double l22 = sqrt(a22 - l20 * l20 - l21 * l21);
    const double l32 = (a23 - l30 * l20 - l31 * l21) / l22;
    const double l33 = sqrt(a33 - l30 * l30 - l31 * l31 - l32 * l32);
    if (!(l33 > 0.0) || !(l22 > 0.0) || !(l11 > 0.0) || !(l00 > 0.0)) err |= FLAG_NONFINITE;
    // v = A^{-1} p_k
    const double y0 = 1.0 / l00;
    const double y1 = (d0 - l10 * y0) / l11;
    const double y2 = (d1 - l20 * y0 - l21 * y1) / l22;
    const double y3 = (d2 - l30 * y0 - l31 * y1 - l32 * y2) / l33;
    const double v3 = y3 / l33;
    const double v2 = (y2 - l32 * v3) / l22;
    const double v1 = (y1 - l21 * v2 - l31 * v3) / l11;
    const double v0 = (y0 - l10 * v1 - l20 * v2 - l30 * v3) / l00;
    m.phi = W * v0;
    if (want_grad) { m.gr[0] = W * v1; m.gr[1] = W * v2; m.gr[2] = W * v3; }
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

__device__ __forceinline__ void load3(const double* p, double v[3]) { v[0] = p[0]; v[1] = p[1]; v[2] = p[2]; }
__device__ __forceinline__ void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Deterministic per-body block reduction: thread 0 of each block stores nval partials, the
// last block to arrive sums them in block order.  Returns true in thread 0 of the last block,
// with the totals in out[].
__device__ bool last_block_sum(const Pools& P, const BodyDev& B, int blk, int nblk, int* counter,
                               const double* mine, int nval, double* out) {
    double* slot = P.partial + 16LL * (B.red_slot + blk);
    for (int i = 0; i < nval; ++i) slot[i] = mine[i];
    __threadfence();
    const int done = atomicAdd(counter, 1);
    if (done != nblk - 1) return false;
    __threadfence();
    for (int i = 0; i < nval; ++i) out[i] = 0.0;
    for (int k = 0; k < nblk; ++k)
        for (int i = 0; i < nval; ++i) out[i] += agent_load(P.partial + 16LL * (B.red_slot + k) + i);
    *counter = 0;
    return true;
}

// ---------------------------------------------------------------- centroids
__global__ void __launch_bounds__(256) k_centroids(Pools P) {
    const int b = P.blk_body_c[blockIdx.x];
    const BodyDev& B = P.bodies[b];
    const JobDev& J = P.jobs[B.job];
    const int grp = threadIdx.x / GROUP, lane = threadIdx.x % GROUP;
    const int blk = blockIdx.x - B.blk_c0;
    const int t = blk * MLS_PER_BLOCK + grp;
    __shared__ double vol[MLS_PER_BLOCK];
    int err = 0;
    double Vt = 0.0;
    if (t < B.nt) {
        const int* tv = P.tri + 3 * (B.t0 + t);
        double xa[3], xb_[3], xc[3];
        load3(P.x + 3 * (B.v0 + tv[0]), xa);
        load3(P.x + 3 * (B.v0 + tv[1]), xb_);
        load3(P.x + 3 * (B.v0 + tv[2]), xc);
        double cen[3], ab[3], ac[3], N[3];
        for (int a = 0; a < 3; ++a) {
            cen[a] = (xa[a] + xb_[a] + xc[a]) * (1.0 / 3.0);
            ab[a] = xb_[a] - xa[a];
            ac[a] = xc[a] - xa[a];
        }
        cross3(ab, ac, N);
        const double A = 0.5 * sqrt(dot3(N, N));
        // signed volume of the tetrahedron (r, a, b, c), r = vertex 0 of the body
        double r0[3], pa[3], pb[3], pc[3], bc[3];
        load3(P.x + 3 * B.v0, r0);
        for (int a = 0; a < 3; ++a) { pa[a] = xa[a] - r0[a]; pb[a] = xb_[a] - r0[a]; pc[a] = xc[a] - r0[a]; }
        cross3(pb, pc, bc);
        Vt = dot3(pa, bc) * (1.0 / 6.0);

        MlsLane m;
        mls_point(J, cen, B.rw, B.alpha, lane, false, m, err);
        float4 mom = make_float4(0.f, 0.f, 0.f, 0.f);
        if (m.active) {
            const WinDesc md = P.mdesc[b];
            const long long l = win_index(J, md, m.gx, m.gy, m.gz);
            if (l < 0) err |= FLAG_WINDOW;
            else mom = P.mwin[B.win_off + l];
        }
        const double U0 = gsum(m.phi * (double)mom.y);
        const double U1 = gsum(m.phi * (double)mom.z);
        const double U2 = gsum(m.phi * (double)mom.w);
        // desired boundary velocity U_b (Sec. 1.2)
        double Ub[3];
        if (!B.rigid) {
            for (int a = 0; a < 3; ++a)
                Ub[a] = (P.uv[3 * (B.v0 + tv[0]) + a] + P.uv[3 * (B.v0 + tv[1]) + a] +
                         P.uv[3 * (B.v0 + tv[2]) + a]) * (1.0 / 3.0);
        } else {
            const BodyState& S = P.bstate[b];
            double rr[3] = {cen[0] - S.X[0], cen[1] - S.X[1], cen[2] - S.X[2]}, w[3];
            cross3(S.om, rr, w);
            for (int a = 0; a < 3; ++a) Ub[a] = S.u[a] + w[a];
        }
        // F_l = (U_b - U*) / dt, spread with c_l = A_l h (Eq. bodyforce)
        const double cl = A * B.shell_h;
        if (m.active) {
            const double s = cl * m.phi;
            const WinDesc fd = P.fdesc[b];
            const long long l = win_index(J, fd, m.gx, m.gy, m.gz);
            if (l < 0) {
                err |= FLAG_WINDOW;
            } else {
                const long long capn = (long long)B.win_cap[0] * B.win_cap[1] * B.win_cap[2];
                unsigned long long* fw = (unsigned long long*)(P.fwin + 3 * B.win_off + l);
                const long long q0 = __double2ll_rn(s * (Ub[0] - U0) * FIX_SCALE);
                const long long q1 = __double2ll_rn(s * (Ub[1] - U1) * FIX_SCALE);
                const long long q2 = __double2ll_rn(s * (Ub[2] - U2) * FIX_SCALE);
                atomicAdd(fw, (unsigned long long)q0);
                atomicAdd(fw + capn, (unsigned long long)q1);
                atomicAdd(fw + 2 * capn, (unsigned long long)q2);
            }
        }
    }
    if (lane == 0) vol[grp] = Vt;
    if (err) atomicOr(P.flags + B.job, err);
    __syncthreads();
    if (threadIdx.x == 0 && !B.rigid) {
        double s = 0.0;
        for (int g = 0; g < MLS_PER_BLOCK; ++g) s += vol[g];
        double V;
        if (last_block_sum(P, B, blk, B.nblk_c, &P.bstate[b].counter_c, &s, 1, &V)) P.bstate[b].V = V;
    }
}

// ---------------------------------------------------------------- triangles (probes)
__global__ void __launch_bounds__(256) k_triangles(Pools P) {
    const int b = P.blk_body_t[blockIdx.x];
    const BodyDev& B = P.bodies[b];
    const JobDev& J = P.jobs[B.job];
    const int grp = threadIdx.x / GROUP, lane = threadIdx.x % GROUP;
    const int blk = blockIdx.x - B.blk_t0;
    const int t = blk * MLS_PER_BLOCK + grp;
    __shared__ double red[MLS_PER_BLOCK][6];
    int err = 0;
    double Ft[3] = {0.0, 0.0, 0.0}, Mt[3] = {0.0, 0.0, 0.0};
    BodyState& S = P.bstate[b];
    if (t < B.nt) {
        const int* tv = P.tri + 3 * (B.t0 + t);
        double xa[3], xb_[3], xc[3];
        load3(P.x + 3 * (B.v0 + tv[0]), xa);
        load3(P.x + 3 * (B.v0 + tv[1]), xb_);
        load3(P.x + 3 * (B.v0 + tv[2]), xc);
        double cen[3], ab[3], ac[3], N[3];
        for (int a = 0; a < 3; ++a) {
            cen[a] = (xa[a] + xb_[a] + xc[a]) * (1.0 / 3.0);
            ab[a] = xb_[a] - xa[a];
            ac[a] = xc[a] - xa[a];
        }
        cross3(ab, ac, N);
        const double ln = sqrt(dot3(N, N));
        const double A = 0.5 * ln;
        const double nrm[3] = {N[0] / ln, N[1] / ln, N[2] / ln};
        const WinDesc md = P.mdesc[b];
        double drho_s[2], gu[2][3][3];
        for (int side = 0; side < 2; ++side) {
            const double sg = side == 0 ? 1.0 : -1.0;
            const double xp[3] = {cen[0] + sg * B.probe * nrm[0], cen[1] + sg * B.probe * nrm[1],
                                  cen[2] + sg * B.probe * nrm[2]};
            MlsLane m;
            mls_point(J, xp, B.rw, B.alpha, lane, true, m, err);
            float4 mom = make_float4(0.f, 0.f, 0.f, 0.f);
            if (m.active) {
                const long long l = win_index(J, md, m.gx, m.gy, m.gz);
                if (l < 0) err |= FLAG_WINDOW;
                else mom = P.mwin[B.win_off + l];
            } else {
                m.gr[0] = m.gr[1] = m.gr[2] = 0.0;
            }
            drho_s[side] = gsum(m.phi * (double)mom.x);
            const double uc[3] = {mom.y, mom.z, mom.w};
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) gu[side][i][j] = gsum(m.gr[j] * uc[i]);
        }
        // p = c_s^2 rho; tau = rho nu (grad u + grad u^T)
        const double nu = J.nu;
        const double rp = 1.0 + drho_s[0], rm = 1.0 + drho_s[1];
        const double dp = (drho_s[0] - drho_s[1]) * (1.0 / 3.0);
        for (int i = 0; i < 3; ++i) {
            double tn = 0.0;
            for (int j = 0; j < 3; ++j)
                tn += (rp * nu * (gu[0][i][j] + gu[0][j][i]) - rm * nu * (gu[1][i][j] + gu[1][j][i])) * nrm[j];
            Ft[i] = (-dp * nrm[i] + tn) * A;
        }
        if (lane == 0)
            for (int i = 0; i < 3; ++i) P.fext[3 * (B.t0 + t) + i] = Ft[i];
        const double* ref = B.rigid ? S.X : S.centre;
        const double rr[3] = {cen[0] - ref[0], cen[1] - ref[1], cen[2] - ref[2]};
        cross3(rr, Ft, Mt);
    }
    if (lane == 0)
        for (int i = 0; i < 3; ++i) { red[grp][i] = Ft[i]; red[grp][3 + i] = Mt[i]; }
    if (err) atomicOr(P.flags + B.job, err);
    __syncthreads();
    if (threadIdx.x != 0) return;
    double part[6] = {0, 0, 0, 0, 0, 0};
    for (int g = 0; g < MLS_PER_BLOCK; ++g)
        for (int i = 0; i < 6; ++i) part[i] += red[g][i];
    double tot[6];
    if (!last_block_sum(P, B, blk, B.nblk_t, &S.counter_t, part, 6, tot)) return;
    for (int i = 0; i < 3; ++i) { S.F[i] = tot[i]; S.M[i] = tot[3 + i]; }
    if (!B.rigid) return;
    // Rigid body, Eqs. (linearVelRig), (angularVelRig): udot = F/m with net weight (m - V0) g,
    // omegadot = I_w^{-1} M with I_w = R I R^T.
    double F[3];
    for (int i = 0; i < 3; ++i) F[i] = tot[i] + (B.mass - B.V0) * B.gravity[i];
    double IR[9], Iw[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += B.Ib[3 * i + k] * S.R[3 * j + k];  // I R^T
            IR[3 * i + j] = s;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += S.R[3 * i + k] * IR[3 * k + j];
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
            for (int k = 0; k < 3; ++k) s += Rw[3 * i + k] * S.R[3 * k + j];
            Rn[3 * i + j] = s;
        }
    bool fin = isfinite(det) && det != 0.0;
    for (int i = 0; i < 9; ++i) { S.R[i] = Rn[i]; fin = fin && isfinite(Rn[i]); }
    for (int i = 0; i < 3; ++i) fin = fin && isfinite(S.X[i]) && isfinite(un[i]) && isfinite(wn[i]);
    if (!fin) atomicOr(P.flags + B.job, FLAG_NONFINITE);
}

// ---------------------------------------------------------------- vertices
// Internal force of one incident element on vertex v (FP64).
__device__ __forceinline__ void spring_on(const Pools& P, const BodyDev& B, int code, int v, double f[3]) {
    const int e = code >> 1;
    const int other = P.edge[2 * (B.e0 + e) + ((code & 1) ? 0 : 1)];
    double xv[3], xo[3];
    load3(P.x + 3 * (B.v0 + v), xv);
    load3(P.x + 3 * (B.v0 + other), xo);
    const double r[3] = {xv[0] - xo[0], xv[1] - xo[1], xv[2] - xo[2]};
    const double l = sqrt(dot3(r, r));
    // Eq. (strainFor)
    const double s = -P.ks[B.e0 + e] * (l - P.l0[B.e0 + e]) / l;
    f[0] += s * r[0]; f[1] += s * r[1]; f[2] += s * r[2];
}

// Bending: -k_b sin(theta - theta0) dtheta/dx_role, theta the signed angle between the outward
// normals of the hinge's triangles (x1,x2,x3) and (x2,x1,x4) about the edge x1->x2.
__device__ __forceinline__ void bend_on(const Pools& P, const BodyDev& B, int code, double f[3]) {
    const int h = code >> 2, role = code & 3;
    const int* hv = P.hinge + 4 * (B.e0 + h);
    double x1[3], x2[3], x3[3], x4[3];
    load3(P.x + 3 * (B.v0 + hv[0]), x1);
    load3(P.x + 3 * (B.v0 + hv[1]), x2);
    load3(P.x + 3 * (B.v0 + hv[2]), x3);
    load3(P.x + 3 * (B.v0 + hv[3]), x4);
    double e[3], p3[3], p4[3], q[3];
    for (int a = 0; a < 3; ++a) { e[a] = x2[a] - x1[a]; p3[a] = x3[a] - x1[a]; p4[a] = x4[a] - x2[a]; q[a] = x1[a] - x2[a]; }
    double N1[3], N2[3];
    cross3(e, p3, N1);
    cross3(q, p4, N2);
    const double le2 = dot3(e, e), le = sqrt(le2);
    const double a1 = sqrt(dot3(N1, N1)), a2 = sqrt(dot3(N2, N2));
    const double n1[3] = {N1[0] / a1, N1[1] / a1, N1[2] / a1};
    const double n2[3] = {N2[0] / a2, N2[1] / a2, N2[2] / a2};
    double c12[3];
    cross3(n1, n2, c12);
    const double theta = atan2(dot3(c12, e) / le, dot3(n1, n2));
    // heights of x3, x4 over the edge line and foot-point parameters along x1->x2
    const double h3 = a1 / le, h4 = a2 / le;
    double d4[3] = {x4[0] - x1[0], x4[1] - x1[1], x4[2] - x1[2]};
    const double t3 = dot3(p3, e) / le2, t4 = dot3(d4, e) / le2;
    double g[3];
    for (int a = 0; a < 3; ++a) {
        const double g3 = -n1[a] / h3, g4 = -n2[a] / h4;
        g[a] = role == 2 ? g3
             : role == 3 ? g4
             : role == 0 ? (t3 - 1.0) * g3 + (t4 - 1.0) * g4
                         : -t3 * g3 - t4 * g4;
    }
    const double s = -B.kb * sin(theta - P.theta0[B.e0 + h]);
    f[0] += s * g[0]; f[1] += s * g[1]; f[2] += s * g[2];
}

__global__ void __launch_bounds__(256) k_vertices(Pools P) {
    const int b = P.blk_body_v[blockIdx.x];
    const BodyDev& B = P.bodies[b];
    const JobDev& J = P.jobs[B.job];
    const int grp = threadIdx.x / GROUP, lane = threadIdx.x % GROUP;
    const int blk = blockIdx.x - B.blk_v0;
    const int v = blk * MLS_PER_BLOCK + grp;
    __shared__ double box[MLS_PER_BLOCK][9];
    BodyState& S = P.bstate[b];
    int err = 0;
    double xn[3] = {0, 0, 0};
    const bool valid = v < B.nv;
    if (valid) {
        const long long gv = B.v0 + v;
        double f[3] = {0.0, 0.0, 0.0};
        // external: a third of every incident triangle's probe force
        const int t_beg = P.vt_ptr[B.vt_off + v], t_end = P.vt_ptr[B.vt_off + v + 1];
        const double vs = B.rigid ? 0.0 : B.kv * (1.0 - S.V / B.V0) * (1.0 / 6.0);
        for (int k = t_beg + lane; k < t_end; k += GROUP) {
            const int t = P.vt_list[k];
            for (int a = 0; a < 3; ++a) f[a] += P.fext[3 * (B.t0 + t) + a] * (1.0 / 3.0);
            if (!B.rigid && B.kv != 0.0) {
                // volume penalty (Eq. volFor, restoring): k_v (1 - V/V0) N_t / 6 per vertex
                const int* tv = P.tri + 3 * (B.t0 + t);
                double xa[3], xb_[3], xc[3], ab[3], ac[3], N[3];
                load3(P.x + 3 * (B.v0 + tv[0]), xa);
                load3(P.x + 3 * (B.v0 + tv[1]), xb_);
                load3(P.x + 3 * (B.v0 + tv[2]), xc);
                for (int a = 0; a < 3; ++a) { ab[a] = xb_[a] - xa[a]; ac[a] = xc[a] - xa[a]; }
                cross3(ab, ac, N);
                for (int a = 0; a < 3; ++a) f[a] += vs * N[a];
            }
        }
        if (!B.rigid) {
            const int e_beg = P.ve_ptr[B.ve_off + v], e_end = P.ve_ptr[B.ve_off + v + 1];
            for (int k = e_beg + lane; k < e_end; k += GROUP) spring_on(P, B, P.ve_list[k], v, f);
            if (B.kb != 0.0) {
                const int h_beg = P.vh_ptr[B.vh_off + v], h_end = P.vh_ptr[B.vh_off + v + 1];
                for (int k = h_beg + lane; k < h_end; k += GROUP) bend_on(P, B, P.vh_list[k], f);
            }
        }
        const double F0 = gsum(f[0]), F1 = gsum(f[1]), F2 = gsum(f[2]);
        double x[3];
        load3(P.x + 3 * gv, x);
        if (!B.rigid) {
            // tentative velocity: fluid velocity at the vertex from f^{n+1}
            MlsLane m;
            mls_point(J, x, B.rw, B.alpha, lane, false, m, err);
            float4 mom = make_float4(0.f, 0.f, 0.f, 0.f);
            if (m.active) {
                const long long l = win_index(J, P.mdesc[b], m.gx, m.gy, m.gz);
                if (l < 0) err |= FLAG_WINDOW;
                else mom = P.mwin[B.win_off + l];
            }
            const double u0[3] = {gsum(m.phi * (double)mom.y), gsum(m.phi * (double)mom.z),
                                  gsum(m.phi * (double)mom.w)};
            const double Fv[3] = {F0, F1, F2};
            double dx[3], un[3];
            for (int a = 0; a < 3; ++a) {
                const double acc = Fv[a] / B.mv;
                if (B.integrator == 1) {
                    // Eqs. (verletPos), (verletVel), (verletPos) as printed, in displacement form
                    un[a] = 1.5 * (u0[a] + 0.5 * acc) - 0.5 * (x[a] - P.xprev[3 * gv + a]);
                    dx[a] = un[a] + 0.5 * acc;
                } else {
                    // Eq. (verletPos); vertex velocity = displacement of the step
                    dx[a] = u0[a] + 0.5 * acc;
                    un[a] = dx[a];
                }
                xn[a] = x[a] + dx[a];
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
        if (!(isfinite(xn[0]) && isfinite(xn[1]) && isfinite(xn[2]))) err |= FLAG_NONFINITE;
    }
    if (lane == 0) {
        for (int a = 0; a < 3; ++a) {
            box[grp][a] = valid ? xn[a] : 1e300;
            box[grp][3 + a] = valid ? xn[a] : -1e300;
            box[grp][6 + a] = valid ? xn[a] : 0.0;
        }
    }
    if (err) atomicOr(P.flags + B.job, err);
    __syncthreads();
    if (threadIdx.x != 0) return;
    double part[9];
    for (int a = 0; a < 3; ++a) { part[a] = 1e300; part[3 + a] = -1e300; part[6 + a] = 0.0; }
    for (int g = 0; g < MLS_PER_BLOCK; ++g)
        for (int a = 0; a < 3; ++a) {
            part[a] = fmin(part[a], box[g][a]);
            part[3 + a] = fmax(part[3 + a], box[g][3 + a]);
            part[6 + a] += box[g][6 + a];
        }
    // min/max are order independent; the sums are taken in block order by the last block
    double* slot = P.partial + 16LL * (B.red_slot + blk);
    for (int i = 0; i < 9; ++i) slot[i] = part[i];
    __threadfence();
    if (atomicAdd(&S.counter_v, 1) != B.nblk_v - 1) return;
    __threadfence();
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300}, sum[3] = {0, 0, 0};
    for (int k = 0; k < B.nblk_v; ++k) {
        const double* p = P.partial + 16LL * (B.red_slot + k);
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], agent_load(p + a));
            hi[a] = fmax(hi[a], agent_load(p + 3 + a));
            sum[a] += agent_load(p + 6 + a);
        }
    }
    S.counter_v = 0;
    // A runaway body keeps its last valid window: coordinates are converted to int only
    // when they are finite and far inside the int range.
    for (int a = 0; a < 3; ++a)
        if (!(isfinite(lo[a]) && isfinite(hi[a]) && fabs(lo[a]) < 1e7 && fabs(hi[a]) < 1e7)) {
            atomicOr(P.flags + B.job, FLAG_NONFINITE);
            return;
        }
    for (int a = 0; a < 3; ++a) S.centre[a] = sum[a] / B.nv;
    // force window of the next step: bounding box plus margin
    WinDesc d;
    const int dims[3] = {J.nx, J.ny, J.nz};
    int flag = 0;
    for (int a = 0; a < 3; ++a) {
        int l = (int)floor(lo[a]) - WIN_MARGIN, h = (int)ceil(hi[a]) + WIN_MARGIN;
        if (J.bc[2 * a] == 0) {
            int w = h - l + 1;
            if (w >= dims[a]) { d.o[a] = 0; d.w[a] = dims[a]; }
            else { int o = l % dims[a]; if (o < 0) o += dims[a]; d.o[a] = o; d.w[a] = w; }
        } else {
            if (l < 0) l = 0;
            if (h > dims[a] - 1) h = dims[a] - 1;
            d.o[a] = l;
            d.w[a] = h >= l ? h - l + 1 : 1;
        }
        if (d.w[a] > B.win_cap[a]) { flag |= FLAG_WINDOW; d.w[a] = B.win_cap[a]; }
        if (d.w[a] < 1) d.w[a] = 1;
    }
    P.fdesc[b] = d;
    if (flag) atomicOr(P.flags + B.job, flag);
}

void launch_centroids(const Pools& P, int nblocks, hipStream_t s) {
    if (nblocks > 0) hipLaunchKernelGGL(k_centroids, dim3(nblocks), dim3(256), 0, s, P);
}
void launch_triangles(const Pools& P, int nblocks, hipStream_t s) {
    if (nblocks > 0) hipLaunchKernelGGL(k_triangles, dim3(nblocks), dim3(256), 0, s, P);
}
void launch_vertices(const Pools& P, int nblocks, hipStream_t s) {
    if (nblocks > 0) hipLaunchKernelGGL(k_vertices, dim3(nblocks), dim3(256), 0, s, P);
}

}  // namespace lbib
