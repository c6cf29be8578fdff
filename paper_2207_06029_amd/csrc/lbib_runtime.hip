// Host runtime behind the C ABI of include/lbib.h: device pools of a batch of lattices,
// rest state of immersed bodies, the per-step launch sequence, getters and setters, and
// kernel timing.  A single lattice is a batch of one job.
#include "lbib.h"
#include "lbib_internal.h"
#include "lbib_runtime.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace lbib {

static thread_local std::string g_err;
static thread_local const char* g_err_static = nullptr;
lbib_status fail(lbib_status code, const std::string& msg) {
    g_err = msg;
    g_err_static = nullptr;
    return code;
}
lbib_status fail_static(lbib_status code, const char* msg) {
    g_err_static = msg;
    return code;
}
const char* last_error() { return g_err_static ? g_err_static : g_err.c_str(); }

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) return fail(LBIB_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------- device allocation
lbib_status Arena::alloc(size_t bytes, void** out) {
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    if (base) {
        if (used + bytes > cap) return fail(LBIB_ENOMEM, "workspace too small");
        *out = (char*)base + used;
        used += bytes;
        return LBIB_OK;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return fail(LBIB_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    owned.push_back(p);
    *out = p;
    total += bytes;
    return LBIB_OK;
}
void Arena::release_from(size_t mark_used, size_t mark_owned) {
    if (base) { used = mark_used; return; }
    while (owned.size() > mark_owned) {
        (void)hipFree(owned.back());
        owned.pop_back();
    }
}
Arena::~Arena() {
    if (!base)
        for (void* p : owned) (void)hipFree(p);
}

template <typename T>
static lbib_status upload(Arena& A, const std::vector<T>& v, T** out, hipStream_t s) {
    void* p;
    lbib_status st = A.alloc(sizeof(T) * std::max<size_t>(v.size(), 1), &p);
    if (st) return st;
    if (!v.empty()) HIP_TRY(hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
    *out = (T*)p;
    return LBIB_OK;
}

// ---------------------------------------------------------------- validation
size_t storage_bytes(int storage) { return storage == 0 ? 4 : 2; }

lbib_status check_lattice(const lbib_lattice_desc& d) {
    if (d.nx < 1 || d.ny < 1 || d.nz < 1) return fail(LBIB_EINVAL, "lattice dimensions must be >= 1");
    if ((long long)d.nx * d.ny * d.nz >= (1LL << 31)) return fail(LBIB_EINVAL, "lattice too large");
    if (!(d.tau > 0.5)) return fail(LBIB_EINVAL, "tau must exceed 1/2");
    if (d.storage < 0 || d.storage > 2) return fail(LBIB_EINVAL, "unknown storage");
    int zh = -1, nzh = 0, moving = 0;
    const int n[3] = {d.nx, d.ny, d.nz};
    for (int a = 0; a < 3; ++a) {
        const int lo = d.bc[2 * a], hi = d.bc[2 * a + 1];
        if (lo < 0 || lo > 2 || hi < 0 || hi > 2) return fail(LBIB_EINVAL, "unknown boundary kind");
        if ((lo == 0) != (hi == 0)) return fail(LBIB_EINVAL, "a periodic face needs a periodic partner");
        if (lo == 1 || hi == 1) {
            zh = a;
            ++nzh;
            if (n[a] < 3) return fail(LBIB_EINVAL, "a Zou-He axis needs at least 3 nodes");
        }
        for (int s = 0; s < 2; ++s)
            if (d.bc[2 * a + s] == 2 && (d.wall_u[2 * a + s][0] != 0 || d.wall_u[2 * a + s][1] != 0 ||
                                         d.wall_u[2 * a + s][2] != 0))
                moving |= 1 << a;
    }
    // Zou-He walls on one axis: a channel between periodic axes.  On several axes (duct, closed
    // box) their edges and corners are closed too, which needs every wall to be Zou-He and to
    // move tangentially (one velocity per edge node).
    if (nzh == 1)
        for (int a = 0; a < 3; ++a)
            if (a != zh && d.bc[2 * a] != 0)
                return fail(LBIB_EINVAL, "Zou-He walls on one axis need periodic tangential axes");
    if (nzh > 1)
        for (int f = 0; f < 6; ++f) {
            if (d.bc[f] == 0) continue;
            if (d.bc[f] != 1) return fail(LBIB_EINVAL, "Zou-He walls on several axes: every wall must be Zou-He");
            if (d.wall_u[f][f / 2] != 0)
                return fail(LBIB_EINVAL, "Zou-He walls on several axes: wall velocities must be tangential");
        }
    if (moving & (moving - 1)) return fail(LBIB_EINVAL, "moving bounce-back walls on one axis only");
    return LBIB_OK;
}

// Device bytes of one lattice of descriptor d with one body of nv vertices and nt triangles
// (nv = 0: no body), as create_lattices and rebuild_bodies carve them from a workspace: every
// allocation rounded up to 256 bytes, at least one element each.  A closed triangle mesh has
// ne = 3 nt / 2 edges; the padded incidence lists are budgeted for vertices with up to
// WS_MAX_VALENCE incident triangles, the force and moment windows for a capacity of the whole
// lattice (their upper bound).
size_t workspace_need(const lbib_lattice_desc& d, long long nv, long long nt) {
    auto r = [](long long bytes) -> size_t { return (size_t)((std::max<long long>(bytes, 1) + 255) & ~255LL); };
    const long long n = (long long)d.nx * d.ny * d.nz;
    size_t b = 2 * r(19 * n * (long long)storage_bytes(d.storage)) + r(sizeof(int)) + r(2 * sizeof(unsigned)) +
               r(sizeof(JobDev)) + r(sizeof(int4) * ((n + MIN_TILE_NODES - 1) / MIN_TILE_NODES));
    const bool body = nv > 0;
    if (!body) nv = nt = 0;
    const long long ne = 3 * nt / 2;
    const long long nbc = (nt + MLS_PER_BLOCK - 1) / MLS_PER_BLOCK, nbt = (nt + TRI_PER_BLOCK - 1) / TRI_PER_BLOCK;
    const long long nbu = (nv + MLS_PER_BLOCK - 1) / MLS_PER_BLOCK;
    const long long nbv = (nv + VERT_PER_BLOCK - 1) / VERT_PER_BLOCK, nbe = (ne + IB_BLOCK - 1) / IB_BLOCK;
    const long long capn = body ? n : 0;
    const long long nbw = body ? win_blocks(capn, true) : 0;   // the larger, rigid count
    b += r(sizeof(BodyDev)) + r(4 * nbc) + r(4 * nbe) + r(4 * nbt) + r(4 * nbv) + r(4 * nbu) + r(4 * nbw);
    b += 6 * r(24 * nv);                                             // x, xprev, uv, fv, u0v, xb
    b += r(12 * nt) + r(8 * ne) + r(16 * ne) + 3 * r(8 * ne);        // tri, edge, hinge, l0, ks, theta0
    b += r(4 * nv * WS_MAX_VALENCE) + r(4 * nv * 2 * WS_MAX_VALENCE);  // incidence lists
    b += 2 * r(24 * std::max<long long>(nt, 1)) + r(48 * std::max<long long>(nt, 1));  // fext, fvol, tgeo
    b += r(120 * std::max<long long>(ne, 1));                        // fedge
    b += r(24 * std::max<long long>(capn, 1)) + r(16 * std::max<long long>(capn, 1));  // fwin, mwin
    b += 2 * r(sizeof(WinDesc)) + r(sizeof(BodyState)) + r(128 * std::max(nbc, nbt)) + r(24 * nbv) + r(48);
    return b;
}

void window_capacity(const int dims[3], bool rigid, double rbound, int cap[3]) {
    // rigid bodies only carry their box along.  A membrane's window may grow to the whole lattice:
    // a soft capsule at a high capillary number can keep elongating in shear (a fixed bound of
    // 2.5 times the rest extent ended such jobs with a window error).  Only memory scales with
    // the capacity (40 B per node): kernels cover the current window.
    for (int a = 0; a < 3; ++a)
        cap[a] = rigid ? std::min(dims[a], (int)std::ceil(2.0 * rbound) + 2 * WIN_MARGIN + 4) : dims[a];
}

long long window_blocks(const int dims[3], bool rigid, double rbound) {
    // the window a membrane usually spans: 2.5 times its rest extent per axis (a Taylor
    // deformation near 0.6 at fixed volume); larger windows are covered by the same blocks
    const double grow = rigid ? 1.0 : 2.5;
    long long n = 1;
    for (int a = 0; a < 3; ++a)
        n *= std::min(dims[a], (int)std::ceil(2.0 * grow * rbound) + 2 * WIN_MARGIN + 4);
    return win_blocks(n, rigid);
}

// ---------------------------------------------------------------- body rest state
static void vsub(const double* a, const double* b, double* c) { for (int i = 0; i < 3; ++i) c[i] = a[i] - b[i]; }
static void vcross(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double vdot(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static double hinge_angle(const double* x, const int* h) {
    double e[3], p3[3], p4[3], q[3], N1[3], N2[3], c[3];
    vsub(x + 3 * h[1], x + 3 * h[0], e);
    vsub(x + 3 * h[2], x + 3 * h[0], p3);
    vsub(x + 3 * h[3], x + 3 * h[1], p4);
    vsub(x + 3 * h[0], x + 3 * h[1], q);
    vcross(e, p3, N1);
    vcross(q, p4, N2);
    const double a1 = std::sqrt(vdot(N1, N1)), a2 = std::sqrt(vdot(N2, N2)), le = std::sqrt(vdot(e, e));
    double n1[3] = {N1[0] / a1, N1[1] / a1, N1[2] / a1}, n2[3] = {N2[0] / a2, N2[1] / a2, N2[2] / a2};
    vcross(n1, n2, c);
    return std::atan2(vdot(c, e) / le, vdot(n1, n2));
}

// Build topology and rest state of one body.  Returns EINVAL for meshes that are not closed,
// consistently oriented, outward 2-manifolds.
lbib_status build_body(const lbib_body_desc& d, const double* xyz, int nv, const int* tri, int nt,
                       HostBody& hb) {
    if (nv < 4 || nt < 4) return fail(LBIB_EINVAL, "mesh too small");
    if (!(d.mls_rw > 0) || !(d.mls_alpha > 0) || !(d.probe_len >= 0) || !(d.shell_h > 0))
        return fail(LBIB_EINVAL, "bad MLS / probe / shell parameters");
    // the kernels evaluate the 3x3x3 block around the nearest node, which holds every node
    // within r_w of the point only for r_w < 1.5
    if (!(d.mls_rw < 1.5)) return fail(LBIB_EINVAL, "mls_rw must be below 1.5 (the MLS support is the 3x3x3 block around the nearest node)");
    // a probe's block reaches probe_len + 1.5 beyond the vertex bounding box, which the force and
    // moment windows extend by WIN_MARGIN
    if (!(d.probe_len + 1.5 <= WIN_MARGIN))
        return fail(LBIB_EINVAL, "probe_len must be at most " + std::to_string(WIN_MARGIN - 1.5) + " (window margin)");
    if (!(d.mass_ratio > 0)) return fail(LBIB_EINVAL, "mass ratio must be positive");
    if (d.integrator < 0 || d.integrator > 2) return fail(LBIB_EINVAL, "unknown integrator");
    if (!d.rigid && (d.gravity[0] != 0 || d.gravity[1] != 0 || d.gravity[2] != 0))
        return fail(LBIB_EINVAL, "gravity is supported on rigid bodies only");
    for (int i = 0; i < 3 * nt; ++i)
        if (tri[i] < 0 || tri[i] >= nv) return fail(LBIB_EINVAL, "triangle index out of range");
    for (int i = 0; i < 3 * nv; ++i)
        if (!std::isfinite(xyz[i])) return fail(LBIB_EINVAL, "non-finite vertex");
    hb = HostBody();
    hb.desc = d;
    hb.nv = nv;
    hb.nt = nt;
    hb.x.assign(xyz, xyz + 3 * nv);
    hb.tri.assign(tri, tri + 3 * nt);
    // half-edges keyed by (vmin, vmax); the owning triangle and direction follow
    struct HE { long long key; int t, fwd; };
    std::vector<HE> he(3 * (size_t)nt);
    for (int t = 0; t < nt; ++t)
        for (int j = 0; j < 3; ++j) {
            const int a = tri[3 * t + j], b = tri[3 * t + (j + 1) % 3];
            if (a == b) return fail(LBIB_EINVAL, "degenerate triangle");
            he[3 * t + j] = {(long long)std::min(a, b) * nv + std::max(a, b), t, a < b ? 1 : 0};
        }
    std::sort(he.begin(), he.end(), [](const HE& p, const HE& q) {
        return p.key != q.key ? p.key < q.key : p.t < q.t;
    });
    if (he.size() % 2) return fail(LBIB_EINVAL, "mesh is not closed");
    const int ne = (int)he.size() / 2;
    hb.ne = ne;
    hb.edge.resize(2 * (size_t)ne);
    hb.hinge.resize(4 * (size_t)ne);
    std::vector<int> etri(2 * (size_t)ne);
    for (int e = 0; e < ne; ++e) {
        const HE& p = he[2 * e];
        const HE& q = he[2 * e + 1];
        const bool dup = (2 * e + 2 < (int)he.size() && he[2 * e + 2].key == p.key);
        if (p.key != q.key || p.fwd == q.fwd || dup)
            return fail(LBIB_EINVAL, "mesh is not a closed, consistently oriented 2-manifold");
        const int v1 = (int)(p.key / nv), v2 = (int)(p.key % nv);
        hb.edge[2 * e] = v1;
        hb.edge[2 * e + 1] = v2;
        // triangle 1 traverses v1 -> v2
        const int t1 = p.fwd ? p.t : q.t, t2 = p.fwd ? q.t : p.t;
        etri[2 * e] = t1;
        etri[2 * e + 1] = t2;
        int o3 = -1, o4 = -1;
        for (int j = 0; j < 3; ++j) {
            if (tri[3 * t1 + j] != v1 && tri[3 * t1 + j] != v2) o3 = tri[3 * t1 + j];
            if (tri[3 * t2 + j] != v1 && tri[3 * t2 + j] != v2) o4 = tri[3 * t2 + j];
        }
        hb.hinge[4 * e] = v1; hb.hinge[4 * e + 1] = v2; hb.hinge[4 * e + 2] = o3; hb.hinge[4 * e + 3] = o4;
    }
    // areas, volume (about vertex 0), surface
    std::vector<double> A(nt);
    double S0 = 0.0, V0 = 0.0;
    for (int t = 0; t < nt; ++t) {
        double ab[3], ac[3], N[3], pa[3], pb[3], pc[3], bc[3];
        vsub(xyz + 3 * tri[3 * t + 1], xyz + 3 * tri[3 * t], ab);
        vsub(xyz + 3 * tri[3 * t + 2], xyz + 3 * tri[3 * t], ac);
        vcross(ab, ac, N);
        A[t] = 0.5 * std::sqrt(vdot(N, N));
        S0 += A[t];
        vsub(xyz + 3 * tri[3 * t], xyz, pa);
        vsub(xyz + 3 * tri[3 * t + 1], xyz, pb);
        vsub(xyz + 3 * tri[3 * t + 2], xyz, pc);
        vcross(pb, pc, bc);
        V0 += vdot(pa, bc) / 6.0;
    }
    if (!(V0 > 0)) return fail(LBIB_EINVAL, "mesh is not outward oriented");
    hb.V0 = V0;
    hb.S0 = S0;
    hb.l0.resize(ne);
    hb.ks.resize(ne);
    hb.theta0.resize(ne);
    for (int e = 0; e < ne; ++e) {
        double r[3];
        vsub(xyz + 3 * hb.edge[2 * e], xyz + 3 * hb.edge[2 * e + 1], r);
        hb.l0[e] = std::sqrt(vdot(r, r));
        // Van Gelder surface weighting with the rest areas (Sec. 1.3)
        hb.ks[e] = d.ks0 * d.thickness * (A[etri[2 * e]] + A[etri[2 * e + 1]]) / (hb.l0[e] * hb.l0[e]);
        hb.theta0[e] = hinge_angle(xyz, &hb.hinge[4 * e]);
    }
    hb.mv = d.mass_ratio * d.thickness * S0 / nv;
    // incidence lists (CSR) per vertex
    hb.vt_ptr.assign(nv + 1, 0);
    hb.vh_ptr.assign(nv + 1, 0);
    for (int t = 0; t < nt; ++t) for (int j = 0; j < 3; ++j) hb.vt_ptr[tri[3 * t + j] + 1]++;
    for (int e = 0; e < ne; ++e)
        for (int r = 0; r < 4; ++r) hb.vh_ptr[hb.hinge[4 * e + r] + 1]++;
    for (int v = 0; v < nv; ++v) {
        hb.vt_ptr[v + 1] += hb.vt_ptr[v];
        hb.vh_ptr[v + 1] += hb.vh_ptr[v];
    }
    hb.vt_list.resize(hb.vt_ptr[nv]);
    hb.vh_list.resize(hb.vh_ptr[nv]);
    {
        std::vector<int> ft(hb.vt_ptr.begin(), hb.vt_ptr.end() - 1), fh(hb.vh_ptr.begin(), hb.vh_ptr.end() - 1);
        for (int t = 0; t < nt; ++t) for (int j = 0; j < 3; ++j) hb.vt_list[ft[tri[3 * t + j]]++] = t;
        for (int e = 0; e < ne; ++e)
            for (int r = 0; r < 4; ++r) hb.vh_list[fh[hb.hinge[4 * e + r]]++] = 4 * e + r;
    }
    // rigid mass properties: signed tetrahedra from the origin, then second moments about the
    // volume centroid; inertia I = rho_s (tr(C) 1 - C)
    double X0[3] = {0, 0, 0}, C[9] = {0};
    {
        double vol = 0.0, m1[3] = {0, 0, 0};
        for (int t = 0; t < nt; ++t) {
            const double *a = xyz + 3 * tri[3 * t], *b = xyz + 3 * tri[3 * t + 1], *c = xyz + 3 * tri[3 * t + 2];
            double bc[3];
            vcross(b, c, bc);
            const double vt = vdot(a, bc) / 6.0;
            vol += vt;
            for (int i = 0; i < 3; ++i) m1[i] += vt * (a[i] + b[i] + c[i]) / 4.0;
        }
        for (int i = 0; i < 3; ++i) X0[i] = m1[i] / vol;
        for (int t = 0; t < nt; ++t) {
            double p[3][3];
            for (int j = 0; j < 3; ++j) vsub(xyz + 3 * tri[3 * t + j], X0, p[j]);
            double bc[3];
            vcross(p[1], p[2], bc);
            const double vt = vdot(p[0], bc) / 6.0;
            double s[3] = {p[0][0] + p[1][0] + p[2][0], p[0][1] + p[1][1] + p[2][1], p[0][2] + p[1][2] + p[2][2]};
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    C[3 * i + j] += vt / 20.0 * (p[0][i] * p[0][j] + p[1][i] * p[1][j] + p[2][i] * p[2][j] + s[i] * s[j]);
        }
    }
    const double tr = C[0] + C[4] + C[8];
    for (int i = 0; i < 9; ++i) hb.Ib[i] = d.mass_ratio * ((i % 4 == 0 ? tr : 0.0) - C[i]);
    hb.mass = d.mass_ratio * V0;
    for (int i = 0; i < 3; ++i) hb.X0[i] = X0[i];
    hb.xb.resize(3 * (size_t)nv);
    double rb = 0.0;
    for (int v = 0; v < nv; ++v) {
        double r[3];
        vsub(xyz + 3 * v, X0, r);
        for (int i = 0; i < 3; ++i) hb.xb[3 * v + i] = r[i];
        rb = std::max(rb, std::sqrt(vdot(r, r)));
    }
    hb.rbound = rb;
    hb.xprev = hb.x;
    hb.uv.assign(3 * (size_t)nv, 0.0);
    return LBIB_OK;
}

// Window descriptor from a bounding box (same rule as the device code).
static WinDesc window_for(const JobDev& J, const double lo[3], const double hi[3], const int cap[3], bool* over) {
    WinDesc d;
    const int dims[3] = {J.nx, J.ny, J.nz};
    *over = false;
    for (int a = 0; a < 3; ++a) {
        int l = (int)std::floor(lo[a]) - WIN_MARGIN, h = (int)std::ceil(hi[a]) + WIN_MARGIN;
        if (J.bc[2 * a] == 0) {
            const int w = h - l + 1;
            if (w >= dims[a]) { d.o[a] = 0; d.w[a] = dims[a]; }
            else { int o = l % dims[a]; if (o < 0) o += dims[a]; d.o[a] = o; d.w[a] = w; }
        } else {
            l = std::max(l, 0);
            h = std::min(h, dims[a] - 1);
            d.o[a] = l;
            d.w[a] = h >= l ? h - l + 1 : 1;
        }
        if (d.w[a] > cap[a]) { *over = true; d.w[a] = cap[a]; }
    }
    return d;
}

// Supports and probes of a body at positions x must stay off wall nodes.
static lbib_status check_support(const JobDev& J, const HostBody& hb) {
    const double reach = hb.desc.probe_len + hb.desc.mls_rw + 0.5;
    const int dims[3] = {J.nx, J.ny, J.nz};
    for (int a = 0; a < 3; ++a) {
        if (J.bc[2 * a] == 0) continue;
        const double lo = J.bc[2 * a] == 1 ? 1.0 : 0.0, hi = J.bc[2 * a] == 1 ? dims[a] - 2.0 : dims[a] - 1.0;
        for (int v = 0; v < hb.nv; ++v) {
            const double c = hb.x[3 * v + a];
            if (c - reach < lo - 0.5 || c + reach > hi + 0.5)
                return fail(LBIB_EDOMAIN, "body support or probe reaches a wall");
        }
    }
    return LBIB_OK;
}

// ---------------------------------------------------------------- batch construction
void Batch::job_from_desc(const lbib_lattice_desc& d, JobDev& J) {
    std::memset(&J, 0, sizeof J);
    J.nx = d.nx; J.ny = d.ny; J.nz = d.nz;
    J.storage = d.storage;
    J.n = (long long)d.nx * d.ny * d.nz;
    J.omega = (float)(1.0 / d.tau);
    J.guo = (float)(1.0 - 1.0 / (2.0 * d.tau));
    J.nu = (float)((d.tau - 0.5) / 3.0);
    for (int f = 0; f < 6; ++f) {
        J.bc[f] = d.bc[f];
        for (int a = 0; a < 3; ++a) J.wall_u[f][a] = (float)d.wall_u[f][a];
    }
    for (int a = 0; a < 3; ++a)
        if (d.bc[2 * a] == 1 || d.bc[2 * a + 1] == 1) ++J.zh_axes;
    for (int a = 0; a < 3; ++a) J.G[a] = (float)d.body_force[a];
    J.mx = d.nx < (1 << 15) ? (unsigned)((0x100000000ULL + d.nx - 1) / d.nx) : 0u;
    J.my = d.ny < (1 << 15) ? (unsigned)((0x100000000ULL + d.ny - 1) / d.ny) : 0u;
}

lbib_status Batch::create_lattices(const std::vector<lbib_lattice_desc>& descs, int storage_,
                                   void* stream_, void* ws, size_t ws_bytes,
                                   const std::vector<char>* skip_init) {
    stream = (hipStream_t)stream_;
    storage = storage_;
    HIP_TRY(hipGetDevice(&device));
    arena.base = ws;
    arena.cap = ws ? ws_bytes : 0;
    ldesc = descs;
    jobs.resize(descs.size());
    long long off = 0;
    for (size_t j = 0; j < descs.size(); ++j) {
        job_from_desc(descs[j], jobs[j]);
        jobs[j].pop_off = off;
        off += 19LL * jobs[j].n;
        jobs[j].body0 = 0;
        jobs[j].nbodies = 0;
    }
    pop_elems = off;
    P.one_lattice = descs.size() == 1 ? 1 : 0;
    P.pop32 = 1;
    for (auto& J : jobs)
        if (19LL * J.n * storage_bytes(storage) >= (1LL << 32)) P.pop32 = 0;
    lbib_status st = arena.alloc(pop_elems * storage_bytes(storage), &P.popA);
    if (st) return st;
    if ((st = arena.alloc(pop_elems * storage_bytes(storage), &P.popB))) return st;
    void* p;
    if ((st = arena.alloc(sizeof(int) * jobs.size(), &p))) return st;
    P.flags = (int*)p;
    HIP_TRY(hipMemsetAsync(P.flags, 0, sizeof(int) * jobs.size(), stream));
    if ((st = arena.alloc(sizeof(unsigned) * 2 * jobs.size(), &p))) return st;
    P.sr_ctr = (unsigned*)p;
    HIP_TRY(hipMemsetAsync(P.sr_ctr, 0, sizeof(unsigned) * 2 * jobs.size(), stream));
    if ((st = arena.alloc(sizeof(JobDev) * jobs.size(), &p))) return st;
    d_jobs = (JobDev*)p;
    P.jobs = d_jobs;
    // sweep tile table, sized for the smallest tile any launch shape uses
    tile_cap = 0;
    for (auto& J : jobs) tile_cap += (size_t)((J.n + MIN_TILE_NODES - 1) / MIN_TILE_NODES);
    if ((st = arena.alloc(sizeof(int4) * std::max<size_t>(tile_cap, 1), &p))) return st;
    d_tiles = (int4*)p;
    mark_used = arena.used;
    mark_owned = arena.owned.size();
    if ((st = retile())) return st;
    // all jobs at rest
    for (size_t j = 0; j < jobs.size(); ++j)
        if (!(skip_init && (*skip_init)[j]))
            if ((st = init_job((int)j, nullptr, nullptr))) return st;
    return rebuild_bodies();
}

// Tile list of the sweep for the current launch shape.
lbib_status Batch::retile() {
    tiles.clear();
    const long long per = (long long)shape.block * shape.npt;
    long long pop_bytes = 0;
    for (size_t j = 0; j < jobs.size(); ++j) {
        jobs[j].tile0 = (int)tiles.size();
        jobs[j].ntiles = (int)((jobs[j].n + per - 1) / per);
        for (int t = 0; t < jobs[j].ntiles; ++t) {
            const long long k0 = (long long)t * per, q = k0 / jobs[j].nx;
            tiles.push_back(make_int4((int)j, (int)(k0 - q * jobs[j].nx), (int)(q % jobs[j].ny), (int)(q / jobs[j].ny)));
        }
        pop_bytes += 2LL * Q * (long long)storage_bytes(storage) * jobs[j].n;
    }
    xcd_chunk = shape.xcd_chunk >= 0 ? shape.xcd_chunk : (pop_bytes <= XCD_CHUNK_MAX_BYTES ? XCD_CHUNK : 0);
    if (tiles.size() > tile_cap)
        return fail(LBIB_EINVAL, "sweep launch shape below " + std::to_string(MIN_TILE_NODES) + " nodes per tile");
    HIP_TRY(hipMemcpyAsync(d_jobs, jobs.data(), sizeof(JobDev) * jobs.size(), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(d_tiles, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice, stream));
    P.tiles = d_tiles;
    graph_valid = false;
    return LBIB_OK;
}

lbib_status Batch::set_shape(SweepShape s) {
    shape = s;
    return retile();
}

// Re-create every body-related device pool from the host copies (after a body was added).
// The record of body h in lattice J, without its placement (offsets and block ranges).
void body_record(const HostBody& h, const JobDev& J, BodyDev& B) {
    std::memset(&B, 0, sizeof B);
    B.job = h.job; B.rigid = h.desc.rigid; B.integrator = h.desc.integrator;
    B.nv = h.nv; B.nt = h.nt; B.ne = h.ne;
    // padded incidence lists: width = the largest count of any vertex of this body
    int wt = 1, wh = 1;
    for (int v = 0; v < h.nv; ++v) {
        wt = std::max(wt, h.vt_ptr[v + 1] - h.vt_ptr[v]);
        wh = std::max(wh, h.vh_ptr[v + 1] - h.vh_ptr[v]);
    }
    B.vt_w = wt;
    B.vh_w = wh;
    B.kb = h.desc.kb; B.kv = h.desc.kv; B.mv = h.mv; B.V0 = h.V0; B.mass = h.mass;
    B.rw = h.desc.mls_rw; B.alpha = h.desc.mls_alpha; B.probe = h.desc.probe_len; B.shell_h = h.desc.shell_h;
    B.rw2 = h.desc.mls_rw * h.desc.mls_rw;
    B.wq = (float)(1.0 / (B.rw2 * h.desc.mls_alpha * h.desc.mls_alpha));
    for (int a = 0; a < 3; ++a) B.gravity[a] = h.desc.gravity[a];
    for (int k = 0; k < 9; ++k) B.Ib[k] = h.Ib[k];
    const int dims[3] = {J.nx, J.ny, J.nz};
    window_capacity(dims, h.desc.rigid != 0, h.rbound, B.win_cap);
    B.nblk_w = (int)window_blocks(dims, h.desc.rigid != 0, h.rbound);
}

// Append body h's incidence lists padded to widths wt (triangles) and wh (hinge roles), -1 past
// a vertex's own count.
void incidence_lists(const HostBody& h, int wt, int wh, std::vector<int>& vtl, std::vector<int>& vhl) {
    for (int v = 0; v < h.nv; ++v) {
        for (int j = 0; j < wt; ++j) {
            const int q = h.vt_ptr[v] + j;
            vtl.push_back(q < h.vt_ptr[v + 1] ? h.vt_list[q] : -1);
        }
        for (int j = 0; j < wh; ++j) {
            const int q = h.vh_ptr[v] + j;
            vhl.push_back(q < h.vh_ptr[v + 1] ? h.vh_list[q] : -1);
        }
    }
}

lbib_status Batch::rebuild_bodies() {
    lbib_status st;
    if ((st = download_body_state())) return st;
    HIP_TRY(hipStreamSynchronize(stream));
    arena.release_from(mark_used, mark_owned);
    // order bodies by job
    std::stable_sort(hbodies.begin(), hbodies.end(), [](const HostBody& a, const HostBody& b) { return a.job < b.job; });
    for (auto& J : jobs) { J.body0 = 0; J.nbodies = 0; }
    std::vector<BodyDev> bd(hbodies.size());
    std::vector<int> bc, be, bt, bv, bu, bw, vbox;
    std::vector<double> x, xprev, uv, xb, l0, ks, th0;
    std::vector<int> tri, edge, hinge, vtl, vhl;
    std::vector<WinDesc> fd(hbodies.size());
    std::vector<BodyState> bs(hbodies.size());
    long long v0 = 0, t0 = 0, e0 = 0, woff = 0, red = 0;
    nblk_c = nblk_e = nblk_t = nblk_v = nblk_u = nblk_w = 0;
    for (size_t i = 0; i < hbodies.size(); ++i) {
        HostBody& h = hbodies[i];
        JobDev& J = jobs[h.job];
        if (J.nbodies == 0) J.body0 = (int)i;
        J.nbodies++;
        BodyDev& B = bd[i];
        body_record(h, J, B);
        B.v0 = v0; B.t0 = t0; B.e0 = e0;
        B.vt_off = (long long)vtl.size();
        B.vh_off = (long long)vhl.size();
        incidence_lists(h, B.vt_w, B.vh_w, vtl, vhl);
        const long long capn = (long long)B.win_cap[0] * B.win_cap[1] * B.win_cap[2];
        B.win_off = woff;
        woff += capn;
        const int nbc = (h.nt + MLS_PER_BLOCK - 1) / MLS_PER_BLOCK;
        const int nbt = (h.nt + TRI_PER_BLOCK - 1) / TRI_PER_BLOCK;
        const int nbu = (h.nv + MLS_PER_BLOCK - 1) / MLS_PER_BLOCK;
        const int nbv = (h.nv + VERT_PER_BLOCK - 1) / VERT_PER_BLOCK;
        const int nbe = h.desc.rigid ? 0 : (h.ne + IB_BLOCK - 1) / IB_BLOCK;
        B.blk_c0 = nblk_c; B.nblk_c = nbc; nblk_c += nbc;
        B.blk_e0 = nblk_e; B.nblk_e = nbe; nblk_e += nbe;
        B.blk_t0 = nblk_t; B.nblk_t = nbt; nblk_t += nbt;
        B.vbox0 = nblk_v;
        B.blk_v0 = nblk_v; B.nblk_v = nbv; nblk_v += nbv;
        B.blk_u0 = nblk_u; B.nblk_u = nbu; nblk_u += nbu;
        const int nbw = B.nblk_w;   // from body_record
        B.blk_w0 = nblk_w; nblk_w += nbw;
        for (int k = 0; k < nbw; ++k) bw.push_back((int)i);
        for (int k = 0; k < nbc; ++k) bc.push_back((int)i);
        for (int k = 0; k < nbe; ++k) be.push_back((int)i);
        for (int k = 0; k < nbt; ++k) bt.push_back((int)i);
        for (int k = 0; k < nbv; ++k) bv.push_back((int)i);
        for (int k = 0; k < nbu; ++k) bu.push_back((int)i);
        B.red_slot = (int)red;
        red += std::max(nbc, nbt);
        x.insert(x.end(), h.x.begin(), h.x.end());
        xprev.insert(xprev.end(), h.xprev.begin(), h.xprev.end());
        uv.insert(uv.end(), h.uv.begin(), h.uv.end());
        xb.insert(xb.end(), h.xb.begin(), h.xb.end());
        tri.insert(tri.end(), h.tri.begin(), h.tri.end());
        edge.insert(edge.end(), h.edge.begin(), h.edge.end());
        hinge.insert(hinge.end(), h.hinge.begin(), h.hinge.end());
        l0.insert(l0.end(), h.l0.begin(), h.l0.end());
        ks.insert(ks.end(), h.ks.begin(), h.ks.end());
        th0.insert(th0.end(), h.theta0.begin(), h.theta0.end());
        v0 += h.nv; t0 += h.nt; e0 += h.ne;
        // state
        BodyState& S = bs[i];
        std::memset(&S, 0, sizeof S);
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int v = 0; v < h.nv; ++v)
            for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], h.x[3 * v + a]); hi[a] = std::max(hi[a], h.x[3 * v + a]); }
        if (h.has_state) S = h.state;
        else {
            S.V = h.V0;
            for (int k = 0; k < 9; ++k) S.R[k] = (k % 4 == 0) ? 1.0 : 0.0;
            for (int a = 0; a < 3; ++a) S.X[a] = h.X0[a];
        }
        // every vertex block starts with the box of the current positions
        for (int k = 0; k < nbv; ++k) {
            for (int a = 0; a < 3; ++a) vbox.push_back((int)std::floor(lo[a]));
            for (int a = 0; a < 3; ++a) vbox.push_back((int)std::ceil(hi[a]));
        }
        bool over = false;
        fd[i] = h.has_state ? h.fdesc : window_for(J, lo, hi, B.win_cap, &over);
        if (over) return fail(LBIB_EDOMAIN, "body does not fit its window");
    }
    nbodies = (int)hbodies.size();
    P.solo_job = nbodies == 1 ? hbodies[0].job : -1;
    if (nbodies == 1) P.solo_body = bd[0];
    any_rigid = any_volume = false;
    for (const HostBody& h : hbodies) {
        if (h.desc.rigid) any_rigid = true;
        else if (h.desc.kv != 0.0) any_volume = true;
    }
    if ((st = upload(arena, bd, (BodyDev**)&P.bodies, stream))) return st;
    if ((st = upload(arena, bc, (int**)&P.blk_body_c, stream))) return st;
    if ((st = upload(arena, be, (int**)&P.blk_body_e, stream))) return st;
    if ((st = upload(arena, bt, (int**)&P.blk_body_t, stream))) return st;
    if ((st = upload(arena, bv, (int**)&P.blk_body_v, stream))) return st;
    if ((st = upload(arena, bu, (int**)&P.blk_body_u, stream))) return st;
    if ((st = upload(arena, bw, (int**)&P.blk_body_w, stream))) return st;
    if ((st = upload(arena, x, &P.x, stream))) return st;
    if ((st = upload(arena, xprev, &P.xprev, stream))) return st;
    if ((st = upload(arena, uv, &P.uv, stream))) return st;
    std::vector<double> zero(x.size(), 0.0);
    if ((st = upload(arena, zero, &P.fv, stream))) return st;
    if ((st = upload(arena, zero, &P.u0v, stream))) return st;
    for (size_t i = 0; i < hbodies.size(); ++i)
        if (hbodies[i].has_state && !hbodies[i].fv.empty())
            HIP_TRY(hipMemcpyAsync(P.fv + 3 * bd[i].v0, hbodies[i].fv.data(), sizeof(double) * hbodies[i].fv.size(), hipMemcpyHostToDevice, stream));
    if ((st = upload(arena, xb, (double**)&P.xb, stream))) return st;
    if ((st = upload(arena, tri, (int**)&P.tri, stream))) return st;
    if ((st = upload(arena, edge, (int**)&P.edge, stream))) return st;
    if ((st = upload(arena, hinge, (int**)&P.hinge, stream))) return st;
    if ((st = upload(arena, l0, (double**)&P.l0, stream))) return st;
    if ((st = upload(arena, ks, (double**)&P.ks, stream))) return st;
    if ((st = upload(arena, th0, (double**)&P.theta0, stream))) return st;
    if ((st = upload(arena, vtl, (int**)&P.vt_list, stream))) return st;
    if ((st = upload(arena, vhl, (int**)&P.vh_list, stream))) return st;
    std::vector<double> fe(3 * (size_t)std::max<long long>(t0, 1), 0.0);
    if ((st = upload(arena, fe, &P.fext, stream))) return st;
    if ((st = upload(arena, fe, &P.fvol, stream))) return st;
    std::vector<double> tg(6 * (size_t)std::max<long long>(t0, 1), 0.0);
    if ((st = upload(arena, tg, &P.tgeo, stream))) return st;
    std::vector<double> fedge(15 * (size_t)std::max<long long>(e0, 1), 0.0);
    if ((st = upload(arena, fedge, &P.fedge, stream))) return st;
    void* p;
    if ((st = arena.alloc(sizeof(long long) * 3 * std::max<long long>(woff, 1), &p))) return st;
    P.fwin = (long long*)p;
    HIP_TRY(hipMemsetAsync(P.fwin, 0, sizeof(long long) * 3 * std::max<long long>(woff, 1), stream));
    if ((st = arena.alloc(sizeof(float4) * std::max<long long>(woff, 1), &p))) return st;
    P.mwin = (float4*)p;
    HIP_TRY(hipMemsetAsync(P.mwin, 0, sizeof(float4) * std::max<long long>(woff, 1), stream));
    if ((st = upload(arena, fd, &P.fdesc, stream))) return st;
    if ((st = upload(arena, fd, &P.mdesc, stream))) return st;
    if ((st = upload(arena, bs, &P.bstate, stream))) return st;
    if ((st = arena.alloc(sizeof(double) * 16 * std::max<long long>(red, 1), &p))) return st;
    P.partial = (double*)p;
    if ((st = upload(arena, vbox, &P.vbox, stream))) return st;
    if ((st = arena.alloc(sizeof(double) * 6, &p))) return st;
    d_totals = (double*)p;
    d_bodies = (BodyDev*)P.bodies;
    host_bodies = bd;
    HIP_TRY(hipMemcpyAsync(d_jobs, jobs.data(), sizeof(JobDev) * jobs.size(), hipMemcpyHostToDevice, stream));
    for (auto& h : hbodies) h.has_state = false;
    primed = false;
    graph_valid = false;
    HIP_TRY(hipStreamSynchronize(stream));
    return LBIB_OK;
}

// Copy the dynamic state of existing bodies back to the host copies (before a rebuild).
lbib_status Batch::download_body_state() {
    if (nbodies == 0) return LBIB_OK;
    HIP_TRY(hipStreamSynchronize(stream));
    for (int i = 0; i < nbodies; ++i) {
        HostBody& h = hbodies[i];
        const BodyDev& B = host_bodies[i];
        HIP_TRY(hipMemcpy(h.x.data(), P.x + 3 * B.v0, sizeof(double) * 3 * h.nv, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(h.xprev.data(), P.xprev + 3 * B.v0, sizeof(double) * 3 * h.nv, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(h.uv.data(), P.uv + 3 * B.v0, sizeof(double) * 3 * h.nv, hipMemcpyDeviceToHost));
        h.fv.resize(3 * (size_t)h.nv);
        HIP_TRY(hipMemcpy(h.fv.data(), P.fv + 3 * B.v0, sizeof(double) * 3 * h.nv, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(&h.state, P.bstate + i, sizeof(BodyState), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(&h.fdesc, P.fdesc + i, sizeof(WinDesc), hipMemcpyDeviceToHost));
        h.has_state = true;
    }
    return LBIB_OK;
}

lbib_status Batch::add_body(int job, const lbib_body_desc& d, const double* xyz, int nv, const int* tri,
                            int nt, int* id) {
    HostBody hb;
    lbib_status st = build_body(d, xyz, nv, tri, nt, hb);
    if (st) return st;
    hb.job = job;
    if ((st = check_support(jobs[job], hb))) return st;
    if ((st = download_body_state())) return st;
    // ids are stable in insertion order per job
    int local = 0;
    for (auto& h : hbodies) if (h.job == job) local++;
    hb.local_id = local;
    hbodies.push_back(hb);
    st = rebuild_bodies();
    if (st) {
        // drop the body again so the lattice stays usable
        for (size_t i = 0; i < hbodies.size(); ++i)
            if (hbodies[i].job == job && hbodies[i].local_id == local) { hbodies.erase(hbodies.begin() + i); break; }
        return st;
    }
    *id = local;
    return LBIB_OK;
}

int Batch::body_index(int job, int local) const {
    for (int i = 0; i < (int)hbodies.size(); ++i)
        if (hbodies[i].job == job && hbodies[i].local_id == local) return i;
    return -1;
}

// ---------------------------------------------------------------- state
// The population buffer that does not hold the current state: its region of a job is dead
// until the next sweep overwrites it, so host transfers stage through it (19 n s bytes per
// job: at least 38 bytes per node) and no call needs device memory of its own.
lbib_status Batch::set_step_counter(int job, unsigned value) {
    const unsigned v[2] = {value, value};
    HIP_TRY(hipMemcpyAsync(P.sr_ctr + 2 * job, v, sizeof v, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return LBIB_OK;
}

void* Batch::spare(int job) const {
    return (char*)(cur_b ? P.popA : P.popB) + jobs[job].pop_off * storage_bytes(storage);
}

lbib_status Batch::init_job(int job, const double* rho, const double* u) {
    const long long n = jobs[job].n;
    // rho (8 n bytes) and u (24 n bytes) staged in the spare buffer
    double* drho = rho ? (double*)spare(job) : nullptr;
    double* du = u ? (double*)spare(job) + n : nullptr;
    if (rho) HIP_TRY(hipMemcpyAsync(drho, rho, sizeof(double) * n, hipMemcpyHostToDevice, stream));
    if (u) HIP_TRY(hipMemcpyAsync(du, u, sizeof(double) * 3 * n, hipMemcpyHostToDevice, stream));
    launch_init_eq(P, storage, cur_b, job, n, drho, du, stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemsetAsync(P.sr_ctr + 2 * job, 0, 2 * sizeof(unsigned), stream));
    HIP_TRY(hipStreamSynchronize(stream));
    primed = false;
    step_count = 0;
    return LBIB_OK;
}

lbib_status Batch::set_populations(int job, const double* f) {
    const long long n = jobs[job].n;
    double* plane = (double*)spare(job);
    for (int i = 0; i < Q; ++i) {
        HIP_TRY(hipMemcpyAsync(plane, f + (size_t)i * n, sizeof(double) * n, hipMemcpyHostToDevice, stream));
        launch_set_pop_plane(P, storage, cur_b, job, n, i, plane, stream);
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(stream));
    primed = false;
    return LBIB_OK;
}

lbib_status Batch::check_flags() {
    HIP_TRY(hipStreamSynchronize(stream));
    std::vector<int> fl(jobs.size());
    HIP_TRY(hipMemcpy(fl.data(), P.flags, sizeof(int) * fl.size(), hipMemcpyDeviceToHost));
    for (size_t j = 0; j < fl.size(); ++j) {
        if (fl[j] & FLAG_NONFINITE) return fail(LBIB_EUNSTABLE, "job " + std::to_string(j) + ": non-finite or runaway state");
        if (fl[j] & FLAG_DOMAIN) return fail(LBIB_EDOMAIN, "job " + std::to_string(j) + ": MLS support or probe reached a wall");
        if (fl[j] & FLAG_WINDOW) return fail(LBIB_EDOMAIN, "job " + std::to_string(j) + ": body outgrew its window");
    }
    return LBIB_OK;
}

lbib_status Batch::job_flags(std::vector<int>& fl) {
    HIP_TRY(hipStreamSynchronize(stream));
    fl.resize(jobs.size());
    HIP_TRY(hipMemcpy(fl.data(), P.flags, sizeof(int) * fl.size(), hipMemcpyDeviceToHost));
    return LBIB_OK;
}

lbib_status Batch::get_macros(int job, double* rho, double* u) {
    const long long n = jobs[job].n;
    float* d = (float*)spare(job);   // 16 n bytes
    launch_macros(P, storage, cur_b, job, n, d, stream);
    HIP_TRY(hipGetLastError());
    std::vector<float> h(4 * n);
    HIP_TRY(hipMemcpyAsync(h.data(), d, sizeof(float) * 4 * n, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    for (long long k = 0; k < n; ++k) {
        if (rho) rho[k] = 1.0 + (double)h[4 * k];
        if (u) for (int a = 0; a < 3; ++a) u[a * n + k] = (double)h[4 * k + 1 + a];
    }
    return LBIB_OK;
}

lbib_status Batch::get_populations(int job, double* f) {
    const long long n = jobs[job].n;
    double* plane = (double*)spare(job);
    for (int i = 0; i < Q; ++i) {
        launch_get_pop_plane(P, storage, cur_b, job, n, i, plane, stream);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(f + (size_t)i * n, plane, sizeof(double) * n, hipMemcpyDeviceToHost, stream));
    }
    HIP_TRY(hipStreamSynchronize(stream));
    return LBIB_OK;
}

// ---------------------------------------------------------------- stepping
lbib_status Batch::prime() {
    launch_window_moments(P, storage, cur_b, nblk_w, stream);
    HIP_TRY(hipGetLastError());
    primed = true;
    return LBIB_OK;
}

lbib_status Batch::enqueue_step(bool collide) {
    const bool bodies = collide && nbodies > 0;
    const bool fold_once = nbodies >= WINDOW_KERNEL_MIN_BODIES;
    if (bodies) {
        launch_centroids(P, nblk_c, nblk_e, !fold_once, stream);
        if (any_volume) launch_fold_bodies(P, nbodies, 0, stream);
    }
    if (timing && sweep_seq++ % timing_period == 0) {
        hipEvent_t a, b;
        lbib_status st = next_event(&a);
        if (!st) st = next_event(&b);
        if (st) return st;
        launch_sweep(P, storage, collide, !cur_b, (int)tiles.size(), shape, xcd_chunk, stream, a, b);
        sweep_events.push_back({a, b});
    } else {
        launch_sweep(P, storage, collide, !cur_b, (int)tiles.size(), shape, xcd_chunk, stream);
    }
    cur_b = !cur_b;
    if (bodies) {
        launch_window_moments(P, storage, cur_b, nblk_w, stream);
        launch_triangles(P, nblk_t, nblk_u, stream);
        if (any_rigid) launch_fold_bodies(P, nbodies, 1, stream);
        launch_vertices(P, nblk_v, stream);
        if (fold_once) launch_windows(P, nbodies, stream);
    }
    HIP_TRY(hipGetLastError());
    return LBIB_OK;
}

lbib_status Batch::step(int nsteps, bool collide) {
    if (nsteps < 0) return fail(LBIB_EINVAL, "negative step count");
    lbib_status st;
    if (collide && nbodies > 0 && !primed)
        if ((st = prime())) return st;
    if (!collide) primed = false;
    if (use_graph && collide && !timing) {
        // a graph holds GRAPH_STEPS steps (an even count, so the buffer parity returns to the
        // start); each replay costs a launch gap of several microseconds, which the steps share
        int k = 0;
        if (cur_b && nsteps > 0) { if ((st = enqueue_step(true))) return st; k = 1; ++step_count; }
        const int reps = (nsteps - k) / GRAPH_STEPS;
        if (reps > 0) {
            if (!graph_valid) { if ((st = capture_graph())) return st; }
            for (int p = 0; p < reps; ++p) HIP_TRY(hipGraphLaunch(graph_exec, stream));
            step_count += (long long)GRAPH_STEPS * reps;
        }
        for (int r = k + reps * GRAPH_STEPS; r < nsteps; ++r) {
            if ((st = enqueue_step(true))) return st;
            ++step_count;
        }
        return LBIB_OK;
    }
    hipEvent_t s0 = nullptr, s1 = nullptr;
    if (timing) {
        if ((st = next_event(&s0)) || (st = next_event(&s1))) return st;
        HIP_TRY(hipEventRecord(s0, stream));
    }
    for (int i = 0; i < nsteps; ++i) {
        if ((st = enqueue_step(collide))) return st;
        ++step_count;
    }
    if (timing) {
        HIP_TRY(hipEventRecord(s1, stream));
        step_events.push_back({s0, s1});
        step_event_steps += nsteps;
    }
    return LBIB_OK;
}

lbib_status Batch::capture_graph() {
    if (graph_exec) { HIP_TRY(hipGraphExecDestroy(graph_exec)); graph_exec = nullptr; }
    if (graph) { HIP_TRY(hipGraphDestroy(graph)); graph = nullptr; }
    if (!capture_stream) HIP_TRY(hipStreamCreateWithFlags(&capture_stream, hipStreamNonBlocking));
    hipStream_t user = stream;
    HIP_TRY(hipStreamSynchronize(user));
    HIP_TRY(hipStreamBeginCapture(capture_stream, hipStreamCaptureModeThreadLocal));
    // launches of the steps go to the capture stream; the caller's stream is restored below
    stream = capture_stream;
    const bool start_b = cur_b;
    lbib_status st = LBIB_OK;
    for (int i = 0; i < GRAPH_STEPS && !st; ++i) st = enqueue_step(true);
    hipError_t e = hipStreamEndCapture(stream, &graph);
    stream = user;
    cur_b = start_b;
    if (st) return st;
    if (e != hipSuccess) return fail(LBIB_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    HIP_TRY(hipGraphInstantiate(&graph_exec, graph, nullptr, nullptr, 0));
    graph_valid = true;
    return LBIB_OK;
}

lbib_status Batch::kernel_time(int kernel, double* ms, int64_t* count) {
    HIP_TRY(hipStreamSynchronize(stream));
    double total = 0.0;
    int64_t c = 0;
    auto& ev = kernel == 0 ? sweep_events : step_events;
    for (auto& pr : ev) {
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, pr.first, pr.second));
        total += t;
        ++c;
    }
    if (kernel == 1) c = step_event_steps;
    *ms = total;
    *count = c;
    return LBIB_OK;
}

lbib_status Batch::next_event(hipEvent_t* e) {
    if (event_next == event_pool.size()) {
        for (int i = 0; i < 256; ++i) {
            hipEvent_t ev;
            HIP_TRY(hipEventCreate(&ev));
            event_pool.push_back(ev);
        }
    }
    *e = event_pool[event_next++];
    return LBIB_OK;
}

void Batch::clear_events() {
    sweep_events.clear();
    step_events.clear();
    event_next = 0;
    step_event_steps = 0;
}

// Destruction cannot report errors: every release is attempted and its status dropped.
Batch::~Batch() {
    if (stream) (void)hipStreamSynchronize(stream);
    clear_events();
    for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
}

// ---------------------------------------------------------------- body state access
lbib_status Batch::body_state(int bi, double* xyz, double* vel) {
    HIP_TRY(hipStreamSynchronize(stream));
    const BodyDev& B = host_bodies[bi];
    if (xyz) HIP_TRY(hipMemcpy(xyz, P.x + 3 * B.v0, sizeof(double) * 3 * B.nv, hipMemcpyDeviceToHost));
    if (vel) HIP_TRY(hipMemcpy(vel, P.uv + 3 * B.v0, sizeof(double) * 3 * B.nv, hipMemcpyDeviceToHost));
    return LBIB_OK;
}

lbib_status Batch::body_forces(int bi, double* fv, double* F, double* M) {
    HIP_TRY(hipStreamSynchronize(stream));
    const BodyDev& B = host_bodies[bi];
    if (fv) HIP_TRY(hipMemcpy(fv, P.fv + 3 * B.v0, sizeof(double) * 3 * B.nv, hipMemcpyDeviceToHost));
    double tot[6];
    if (B.rigid) {
        BodyState S;
        HIP_TRY(hipMemcpy(&S, P.bstate + bi, sizeof S, hipMemcpyDeviceToHost));
        for (int a = 0; a < 3; ++a) { tot[a] = S.F[a]; tot[3 + a] = S.M[a]; }
    } else {
        // membranes: totals of the last step's probe forces, reduced on the device in FP64
        launch_body_totals(P, bi, d_totals, stream);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(tot, d_totals, sizeof tot, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
    }
    if (F) for (int a = 0; a < 3; ++a) F[a] = tot[a];
    if (M) for (int a = 0; a < 3; ++a) M[a] = tot[3 + a];
    return LBIB_OK;
}

lbib_status Batch::body_set_velocity(int bi, const double* v) {
    HIP_TRY(hipStreamSynchronize(stream));
    const BodyDev& B = host_bodies[bi];
    std::vector<double> x(3 * (size_t)B.nv), uv(3 * (size_t)B.nv), xp(3 * (size_t)B.nv);
    HIP_TRY(hipMemcpy(x.data(), P.x + 3 * B.v0, sizeof(double) * x.size(), hipMemcpyDeviceToHost));
    if (!B.rigid) {
        for (size_t i = 0; i < x.size(); ++i) { uv[i] = v[i]; xp[i] = x[i] - v[i]; }
    } else {
        BodyState S;
        HIP_TRY(hipMemcpy(&S, P.bstate + bi, sizeof S, hipMemcpyDeviceToHost));
        for (int a = 0; a < 3; ++a) { S.u[a] = S.u1[a] = v[a]; S.om[a] = S.om1[a] = v[3 + a]; }
        HIP_TRY(hipMemcpy(P.bstate + bi, &S, sizeof S, hipMemcpyHostToDevice));
        for (int k = 0; k < B.nv; ++k) {
            double r[3] = {x[3 * k] - S.X[0], x[3 * k + 1] - S.X[1], x[3 * k + 2] - S.X[2]}, w[3];
            vcross(S.om, r, w);
            for (int a = 0; a < 3; ++a) { uv[3 * k + a] = S.u[a] + w[a]; xp[3 * k + a] = x[3 * k + a]; }
        }
    }
    HIP_TRY(hipMemcpy(P.uv + 3 * B.v0, uv.data(), sizeof(double) * uv.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(P.xprev + 3 * B.v0, xp.data(), sizeof(double) * xp.size(), hipMemcpyHostToDevice));
    return LBIB_OK;
}

size_t Batch::device_bytes() const {
    return arena.base ? arena.used : arena.total;
}

// ---------------------------------------------------------------- slotted batches
// Device bytes one slot of capacity c occupies (create_slotted allocates nslots times this, plus
// 48 bytes of totals, each allocation rounded up to 256 bytes).
uint64_t slot_device_bytes(const SlotCaps& c, int storage) {
    const uint64_t es = storage_bytes(storage), per = 256;
    const uint64_t nodes = (uint64_t)std::max<long long>(c.nodes, 1), nv = (uint64_t)c.nv, nt = (uint64_t)c.nt;
    const uint64_t ne = 3 * nt / 2, win = nodes;
    const uint64_t bc = (nt + MLS_PER_BLOCK - 1) / MLS_PER_BLOCK, bt = (nt + TRI_PER_BLOCK - 1) / TRI_PER_BLOCK;
    const uint64_t bu = (nv + MLS_PER_BLOCK - 1) / MLS_PER_BLOCK, bv = (nv + VERT_PER_BLOCK - 1) / VERT_PER_BLOCK;
    const uint64_t be = (ne + IB_BLOCK - 1) / IB_BLOCK;
    const uint64_t bw = (uint64_t)win_blocks((long long)win, true);
    uint64_t b = 2 * 19 * nodes * es + 4 + 8 + sizeof(JobDev) + sizeof(int4) * ((nodes + per - 1) / per);
    b += sizeof(BodyDev) + 4 * (bc + be + bt + bv + bu + bw);
    b += 6 * 24 * nv + 12 * nt + 8 * ne + 16 * ne + 3 * 8 * ne;
    b += 4 * nv * SLOT_VT_W + 4 * nv * SLOT_VH_W;
    b += 48 * nt + 24 * nt + 24 * nt + 120 * ne + 24 * win + 16 * win;
    b += 2 * sizeof(WinDesc) + sizeof(BodyState) + 128 * std::max(bc, bt) + 24 * bv;
    return b + 40 * 256;
}

lbib_status Batch::create_slotted(int nslots, const SlotCaps& c, int storage_, void* stream_) {
    if (nslots < 1 || c.nodes < 1 || c.nv < 0 || c.nt < 0) return fail(LBIB_EINVAL, "bad slot capacity");
    stream = (hipStream_t)stream_;
    storage = storage_;
    HIP_TRY(hipGetDevice(&device));
    slotted = true;
    caps = c;
    slot_live.assign(nslots, 0);
    const size_t es = storage_bytes(storage);
    const long long per = (long long)shape.block * shape.npt;
    tiles_slot = (int)((c.nodes + per - 1) / per);
    ne_slot = 3LL * c.nt / 2;
    win_slot = c.nodes;   // a window never exceeds its lattice
    bc_slot = (c.nt + MLS_PER_BLOCK - 1) / MLS_PER_BLOCK;
    be_slot = (int)((ne_slot + IB_BLOCK - 1) / IB_BLOCK);
    bt_slot = (c.nt + TRI_PER_BLOCK - 1) / TRI_PER_BLOCK;
    bu_slot = (c.nv + MLS_PER_BLOCK - 1) / MLS_PER_BLOCK;
    bv_slot = (c.nv + VERT_PER_BLOCK - 1) / VERT_PER_BLOCK;
    bw_slot = (int)win_blocks(win_slot, true);
    red_slot = std::max(bc_slot, bt_slot);
    const long long S = nslots;
    // lattices: empty slots hold no job (n = 0)
    jobs.assign(nslots, JobDev{});
    for (int j = 0; j < nslots; ++j) jobs[j].pop_off = (long long)j * 19 * c.nodes;
    ldesc.assign(nslots, lbib_lattice_desc{});
    pop_elems = S * 19 * c.nodes;
    P.pop32 = 19LL * c.nodes * (long long)es < (1LL << 32) ? 1 : 0;
    P.one_lattice = 0;
    void* p;
    lbib_status st;
    if ((st = arena.alloc(pop_elems * es, &P.popA))) return st;
    if ((st = arena.alloc(pop_elems * es, &P.popB))) return st;
    if ((st = arena.alloc(sizeof(int) * S, &p))) return st;
    P.flags = (int*)p;
    HIP_TRY(hipMemsetAsync(P.flags, 0, sizeof(int) * S, stream));
    if ((st = arena.alloc(sizeof(unsigned) * 2 * S, &p))) return st;
    P.sr_ctr = (unsigned*)p;
    HIP_TRY(hipMemsetAsync(P.sr_ctr, 0, sizeof(unsigned) * 2 * S, stream));
    if ((st = arena.alloc(sizeof(JobDev) * S, &p))) return st;
    d_jobs = (JobDev*)p;
    P.jobs = d_jobs;
    tile_cap = (size_t)S * tiles_slot;
    if ((st = arena.alloc(sizeof(int4) * tile_cap, &p))) return st;
    d_tiles = (int4*)p;
    P.tiles = d_tiles;
    xcd_chunk = shape.xcd_chunk >= 0 ? shape.xcd_chunk : (2 * pop_elems * (long long)es <= XCD_CHUNK_MAX_BYTES ? XCD_CHUNK : 0);
    // bodies: one per slot, every array sized for the slot's capacity
    auto take = [&](size_t bytes, void** out) { return arena.alloc(std::max<size_t>(bytes, 1), out); };
    if ((st = take(sizeof(BodyDev) * S, &p))) return st;
    d_bodies = (BodyDev*)p;
    P.bodies = d_bodies;
    const int* tables[6];
    const long long tsz[6] = {S * bc_slot, S * be_slot, S * bt_slot, S * bv_slot, S * bu_slot, S * bw_slot};
    for (int k = 0; k < 6; ++k) {
        if ((st = take(sizeof(int) * tsz[k], &p))) return st;
        tables[k] = (const int*)p;
    }
    P.blk_body_c = tables[0]; P.blk_body_e = tables[1]; P.blk_body_t = tables[2];
    P.blk_body_v = tables[3]; P.blk_body_u = tables[4]; P.blk_body_w = tables[5];
    const size_t nv3 = sizeof(double) * 3 * (size_t)(S * c.nv);
    double** vec3[6] = {&P.x, &P.xprev, &P.uv, &P.fv, &P.u0v, (double**)&P.xb};
    for (auto q : vec3) {
        if ((st = take(nv3, &p))) return st;
        *q = (double*)p;
    }
    HIP_TRY(hipMemsetAsync(P.fv, 0, nv3, stream));
    HIP_TRY(hipMemsetAsync(P.u0v, 0, nv3, stream));
    if ((st = take(sizeof(int) * 3 * (size_t)(S * c.nt), &p))) return st;
    P.tri = (const int*)p;
    if ((st = take(sizeof(int) * 2 * (size_t)(S * ne_slot), &p))) return st;
    P.edge = (const int*)p;
    if ((st = take(sizeof(int) * 4 * (size_t)(S * ne_slot), &p))) return st;
    P.hinge = (const int*)p;
    const double** rest[3] = {&P.l0, &P.ks, &P.theta0};
    for (auto q : rest) {
        if ((st = take(sizeof(double) * (size_t)(S * ne_slot), &p))) return st;
        *q = (const double*)p;
    }
    if ((st = take(sizeof(int) * (size_t)(S * c.nv) * SLOT_VT_W, &p))) return st;
    P.vt_list = (const int*)p;
    if ((st = take(sizeof(int) * (size_t)(S * c.nv) * SLOT_VH_W, &p))) return st;
    P.vh_list = (const int*)p;
    if ((st = take(sizeof(double) * 6 * (size_t)(S * c.nt), &p))) return st;
    P.tgeo = (double*)p;
    if ((st = take(sizeof(double) * 3 * (size_t)(S * c.nt), &p))) return st;
    P.fext = (double*)p;
    if ((st = take(sizeof(double) * 3 * (size_t)(S * c.nt), &p))) return st;
    P.fvol = (double*)p;
    if ((st = take(sizeof(double) * 15 * (size_t)(S * ne_slot), &p))) return st;
    P.fedge = (double*)p;
    if ((st = take(sizeof(long long) * 3 * (size_t)(S * win_slot), &p))) return st;
    P.fwin = (long long*)p;
    HIP_TRY(hipMemsetAsync(P.fwin, 0, sizeof(long long) * 3 * (size_t)(S * win_slot), stream));
    if ((st = take(sizeof(float4) * (size_t)(S * win_slot), &p))) return st;
    P.mwin = (float4*)p;
    HIP_TRY(hipMemsetAsync(P.mwin, 0, sizeof(float4) * (size_t)(S * win_slot), stream));
    if ((st = take(sizeof(WinDesc) * S, &p))) return st;
    P.fdesc = (WinDesc*)p;
    if ((st = take(sizeof(WinDesc) * S, &p))) return st;
    P.mdesc = (WinDesc*)p;
    if ((st = take(sizeof(BodyState) * S, &p))) return st;
    P.bstate = (BodyState*)p;
    if ((st = take(sizeof(double) * 16 * (size_t)(S * red_slot), &p))) return st;
    P.partial = (double*)p;
    if ((st = take(sizeof(int) * 6 * (size_t)(S * bv_slot), &p))) return st;
    P.vbox = (int*)p;
    if ((st = take(sizeof(double) * 6, &p))) return st;
    d_totals = (double*)p;
    // every slot starts empty; the body tables keep one (empty) body per slot
    nbodies = nslots;
    hbodies.assign(nslots, HostBody{});
    host_bodies.assign(nslots, BodyDev{});
    for (int j = 0; j < nslots; ++j) {
        hbodies[j].job = j;
        host_bodies[j].job = j;
    }
    P.solo_job = -1;
    any_rigid = any_volume = true;   // the fold launches skip bodies without that work
    use_graph = false;
    primed = true;   // admissions prime their own moment windows
    lbib_status r = slot_tables();
    if (r) return r;
    HIP_TRY(hipStreamSynchronize(stream));
    return LBIB_OK;
}

// Packed tables of the live slots (tiles and blocks in slot order) and the job and body records,
// copied over the fixed-size device tables; the launch grids follow the live counts.
lbib_status Batch::slot_tables() {
    const int S = (int)slot_live.size();
    const long long per = (long long)shape.block * shape.npt;
    tiles.clear();
    std::vector<int> bc, be, bt, bv, bu, bw;
    for (int s = 0; s < S; ++s) {
        JobDev& J = jobs[s];
        BodyDev& B = host_bodies[s];
        if (!slot_live[s]) {
            J.n = 0; J.tile0 = J.ntiles = 0; J.nbodies = 0;
            continue;
        }
        J.tile0 = (int)tiles.size();
        J.ntiles = (int)((J.n + per - 1) / per);
        for (int t = 0; t < J.ntiles; ++t) {
            const long long k0 = (long long)t * per, q = k0 / J.nx;
            tiles.push_back(make_int4(s, (int)(k0 - q * J.nx), (int)(q % J.ny), (int)(q / J.ny)));
        }
        if (B.nv == 0) continue;
        const int nbc = (B.nt + MLS_PER_BLOCK - 1) / MLS_PER_BLOCK, nbt = (B.nt + TRI_PER_BLOCK - 1) / TRI_PER_BLOCK;
        const int nbu = (B.nv + MLS_PER_BLOCK - 1) / MLS_PER_BLOCK, nbv = (B.nv + VERT_PER_BLOCK - 1) / VERT_PER_BLOCK;
        const int nbe = B.rigid ? 0 : (B.ne + IB_BLOCK - 1) / IB_BLOCK;
        const int nbw = B.nblk_w;   // from body_record at admission
        B.blk_c0 = (int)bc.size(); B.nblk_c = nbc; bc.insert(bc.end(), nbc, s);
        B.blk_e0 = (int)be.size(); B.nblk_e = nbe; be.insert(be.end(), nbe, s);
        B.blk_t0 = (int)bt.size(); B.nblk_t = nbt; bt.insert(bt.end(), nbt, s);
        B.blk_v0 = (int)bv.size(); B.nblk_v = nbv; bv.insert(bv.end(), nbv, s);
        B.blk_u0 = (int)bu.size(); B.nblk_u = nbu; bu.insert(bu.end(), nbu, s);
        B.blk_w0 = (int)bw.size(); bw.insert(bw.end(), nbw, s);
    }
    auto put = [&](const std::vector<int>& v, const int* dst) -> lbib_status {
        if (!v.empty()) HIP_TRY(hipMemcpyAsync((void*)dst, v.data(), sizeof(int) * v.size(), hipMemcpyHostToDevice, stream));
        return LBIB_OK;
    };
    lbib_status st;
    if ((st = put(bc, P.blk_body_c)) || (st = put(be, P.blk_body_e)) || (st = put(bt, P.blk_body_t)) ||
        (st = put(bv, P.blk_body_v)) || (st = put(bu, P.blk_body_u)) || (st = put(bw, P.blk_body_w)))
        return st;
    if (!tiles.empty())
        HIP_TRY(hipMemcpyAsync(d_tiles, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(d_jobs, jobs.data(), sizeof(JobDev) * S, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(d_bodies, host_bodies.data(), sizeof(BodyDev) * S, hipMemcpyHostToDevice, stream));
    nblk_c = (int)bc.size(); nblk_e = (int)be.size(); nblk_t = (int)bt.size();
    nblk_v = (int)bv.size(); nblk_u = (int)bu.size(); nblk_w = (int)bw.size();
    // the host copies must stay unchanged until the copies have run
    HIP_TRY(hipStreamSynchronize(stream));
    return LBIB_OK;
}

lbib_status Batch::slot_admit(int s, const lbib_lattice_desc& d, const HostBody* hb) {
    if (!slotted || s < 0 || s >= (int)slot_live.size() || slot_live[s]) return fail(LBIB_EINVAL, "no such free slot");
    const long long n = (long long)d.nx * d.ny * d.nz;
    if (n > caps.nodes) return fail(LBIB_ENOMEM, "lattice exceeds the slot capacity");
    JobDev J;
    job_from_desc(d, J);
    J.pop_off = (long long)s * 19 * caps.nodes;
    J.body0 = s;
    J.nbodies = 0;
    BodyDev B;
    std::memset(&B, 0, sizeof B);
    B.job = s;
    if (hb) {
        if (hb->nv > caps.nv || hb->nt > caps.nt || hb->ne > ne_slot)
            return fail(LBIB_ENOMEM, "mesh exceeds the slot capacity");
        HostBody h = *hb;
        h.job = s;
        lbib_status st = check_support(J, h);
        if (st) return st;
        body_record(h, J, B);
        if (B.vt_w > SLOT_VT_W || B.vh_w > SLOT_VH_W) return fail(LBIB_ENOMEM, "vertex valence exceeds the slot capacity");
        const long long capn = (long long)B.win_cap[0] * B.win_cap[1] * B.win_cap[2];
        if (capn > win_slot) return fail(LBIB_ENOMEM, "force window exceeds the slot capacity");
        B.v0 = (long long)s * caps.nv;
        B.t0 = (long long)s * caps.nt;
        B.e0 = (long long)s * ne_slot;
        B.vt_off = (long long)s * caps.nv * SLOT_VT_W;
        B.vh_off = (long long)s * caps.nv * SLOT_VH_W;
        B.win_off = (long long)s * win_slot;
        B.red_slot = s * red_slot;
        B.vbox0 = s * bv_slot;
        J.nbodies = 1;
        // mesh, rest data and state into the slot's ranges
        auto put = [&](void* base, size_t elem, long long off, const void* src, size_t count) -> lbib_status {
            if (count) HIP_TRY(hipMemcpyAsync((char*)base + elem * off, src, elem * count, hipMemcpyHostToDevice, stream));
            return LBIB_OK;
        };
        std::vector<int> vtl, vhl;
        incidence_lists(h, B.vt_w, B.vh_w, vtl, vhl);
        std::vector<int> vb;
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int v = 0; v < h.nv; ++v)
            for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], h.x[3 * v + a]); hi[a] = std::max(hi[a], h.x[3 * v + a]); }
        const int nbv = (h.nv + VERT_PER_BLOCK - 1) / VERT_PER_BLOCK;
        for (int k = 0; k < nbv; ++k) {
            for (int a = 0; a < 3; ++a) vb.push_back((int)std::floor(lo[a]));
            for (int a = 0; a < 3; ++a) vb.push_back((int)std::ceil(hi[a]));
        }
        bool over = false;
        const WinDesc fd = window_for(J, lo, hi, B.win_cap, &over);
        if (over) return fail(LBIB_EDOMAIN, "body does not fit its window");
        BodyState S;
        std::memset(&S, 0, sizeof S);
        S.V = h.V0;
        for (int k = 0; k < 9; ++k) S.R[k] = (k % 4 == 0) ? 1.0 : 0.0;
        for (int a = 0; a < 3; ++a) S.X[a] = h.X0[a];
        const size_t nv3 = 3 * (size_t)h.nv;
        if ((st = put(P.x, 8, 3 * B.v0, h.x.data(), nv3)) || (st = put(P.xprev, 8, 3 * B.v0, h.xprev.data(), nv3)) ||
            (st = put(P.uv, 8, 3 * B.v0, h.uv.data(), nv3)) || (st = put((void*)P.xb, 8, 3 * B.v0, h.xb.data(), nv3)) ||
            (st = put((void*)P.tri, 4, 3 * B.t0, h.tri.data(), h.tri.size())) ||
            (st = put((void*)P.edge, 4, 2 * B.e0, h.edge.data(), h.edge.size())) ||
            (st = put((void*)P.hinge, 4, 4 * B.e0, h.hinge.data(), h.hinge.size())) ||
            (st = put((void*)P.l0, 8, B.e0, h.l0.data(), h.l0.size())) ||
            (st = put((void*)P.ks, 8, B.e0, h.ks.data(), h.ks.size())) ||
            (st = put((void*)P.theta0, 8, B.e0, h.theta0.data(), h.theta0.size())) ||
            (st = put((void*)P.vt_list, 4, B.vt_off, vtl.data(), vtl.size())) ||
            (st = put((void*)P.vh_list, 4, B.vh_off, vhl.data(), vhl.size())) ||
            (st = put(P.vbox, 4, 6LL * s * bv_slot, vb.data(), vb.size())) ||
            (st = put(P.fdesc, sizeof(WinDesc), s, &fd, 1)) || (st = put(P.mdesc, sizeof(WinDesc), s, &fd, 1)) ||
            (st = put(P.bstate, sizeof(BodyState), s, &S, 1)))
            return st;
        HIP_TRY(hipMemsetAsync(P.fv + 3 * B.v0, 0, sizeof(double) * nv3, stream));
        HIP_TRY(hipMemsetAsync(P.u0v + 3 * B.v0, 0, sizeof(double) * nv3, stream));
        HIP_TRY(hipMemsetAsync(P.fwin + 3 * B.win_off, 0, sizeof(long long) * 3 * (size_t)capn, stream));
        hbodies[s] = h;
        hbodies[s].local_id = 0;
        hbodies[s].has_state = false;
    }
    jobs[s] = J;
    ldesc[s] = d;
    host_bodies[s] = B;
    // the job's record first (the initial-state kernel reads it), then the state at rest
    HIP_TRY(hipMemcpyAsync(d_jobs + s, &jobs[s], sizeof(JobDev), hipMemcpyHostToDevice, stream));
    launch_init_eq(P, storage, cur_b, s, n, nullptr, nullptr, stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemsetAsync(P.sr_ctr + 2 * s, 0, 2 * sizeof(unsigned), stream));
    HIP_TRY(hipMemsetAsync(P.flags + s, 0, sizeof(int), stream));
    slot_live[s] = 1;
    lbib_status st = slot_tables();
    if (st) return st;
    // moment windows of the new body (resident bodies get theirs again, bitwise the same)
    if (hb) {
        launch_window_moments(P, storage, cur_b, nblk_w, stream);
        HIP_TRY(hipGetLastError());
    }
    return LBIB_OK;
}

lbib_status Batch::slot_retire(int s) {
    if (!slotted || s < 0 || s >= (int)slot_live.size() || !slot_live[s]) return fail(LBIB_EINVAL, "no such live slot");
    slot_live[s] = 0;
    std::memset(&host_bodies[s], 0, sizeof(BodyDev));
    host_bodies[s].job = s;
    hbodies[s] = HostBody{};
    hbodies[s].job = s;
    return slot_tables();
}

}  // namespace lbib
