// Lattice kernels: the fused collide+stream sweep (Sec. 1.1, Eqs. evoleq, eqfunc, forcing),
// window moments for the immersed boundary, and the state get/set/init kernels.
//
// Populations are stored after collision, as deviations g_i = f_i - w_i, structure of arrays
// [i][z][y][x] per job.  The post-streaming distribution of the current time level is
// obtained by pulling g_i from x - e_i, with periodic wrap, halfway bounce-back from the
// node's own opposite population, or the Zou-He closure on wet wall nodes.  Every reader
// (sweep, moments, getters) uses the same pull, so the post-streaming state is never stored.
#include "lbib_internal.h"

#include <hip/hip_ext.h>

namespace lbib {

// ---------------------------------------------------------------- storage codecs
template <typename S> struct Codec;
// ld / st convert between the stored value and the deviation; raw / st_raw move the stored value
// in storage units (the deviation times scale) for code that works in those units throughout.
template <> struct Codec<float> {
    static constexpr float scale = 1.0f;
    __device__ static __forceinline__ float ld(const float* p) { return *p; }
    __device__ static __forceinline__ void st(float* p, float v) { *p = v; }
    __device__ static __forceinline__ float raw(const float* p) { return *p; }
    __device__ static __forceinline__ void st_raw(float* p, float v) { *p = v; }
};
// FP16 holds the deviation times 2^12: an exact power-of-two scaling that keeps deviations
// down to ~1.5e-8 in the normal range (full 11-bit precision) while |g| up to 16 still fits.
constexpr float F16_SCALE = 4096.0f;
constexpr float F16_INV = 1.0f / 4096.0f;
template <> struct Codec<__half> {
    static constexpr float scale = F16_SCALE;
    __device__ static __forceinline__ float ld(const __half* p) { return __half2float(*p) * F16_INV; }
    __device__ static __forceinline__ void st(__half* p, float v) { *p = __float2half_rn(v * F16_SCALE); }
    __device__ static __forceinline__ float raw(const __half* p) { return __half2float(*p); }
    __device__ static __forceinline__ void st_raw(__half* p, float v) { *p = __float2half_rn(v); }
};
template <> struct Codec<__hip_bfloat16> {
    static constexpr float scale = 1.0f;
    __device__ static __forceinline__ float ld(const __hip_bfloat16* p) { return __bfloat162float(*p); }
    __device__ static __forceinline__ void st(__hip_bfloat16* p, float v) { *p = __float2bfloat16(v); }
    __device__ static __forceinline__ float raw(const __hip_bfloat16* p) { return __bfloat162float(*p); }
    __device__ static __forceinline__ void st_raw(__hip_bfloat16* p, float v) { *p = __float2bfloat16(v); }
};

// Stochastic rounding of the collision's output (the sweep's only narrowing that is repeated every
// step).  Round-to-nearest of a slowly varying population loses every update smaller than half a
// unit in the last place, the same way every step, so a flow developing from rest stagnates;
// rounding up with probability equal to the dropped fraction keeps every update in expectation.
// Before round-to-nearest the value x is moved by d * P(x), where P(x) is the power of two at or
// below |x| (its exponent bits; 0 for zero and FP32 subnormals, which stay unperturbed) and d is
// uniform over (-1/2, 1/2) of the target format's unit in the last place in 1/256 steps:
// round-to-nearest then rounds up with probability equal to the dropped fraction, to within 1/256.
template <typename S> struct Narrow;
// cvt / st take the value in storage units.
template <> struct Narrow<float> {
    static constexpr float ulp = 0.f;
    __device__ static __forceinline__ float cvt(float v, float) { return v; }
    __device__ static __forceinline__ void st(float* p, float v, float) { *p = v; }
};
__device__ __forceinline__ float sr_perturb(float x, float d) {
    return fmaf(d, __uint_as_float(__float_as_uint(x) & 0x7F800000u), x);
}
template <> struct Narrow<__half> {
    static constexpr float ulp = 1.f / 1024.f;   // 10 stored mantissa bits
    __device__ static __forceinline__ __half cvt(float v, float d) { return __float2half_rn(sr_perturb(v, d)); }
    __device__ static __forceinline__ void st(__half* p, float v, float d) { *p = cvt(v, d); }
};
template <> struct Narrow<__hip_bfloat16> {
    static constexpr float ulp = 1.f / 128.f;    // 7 stored mantissa bits
    __device__ static __forceinline__ __hip_bfloat16 cvt(float v, float d) { return __float2bfloat16(sr_perturb(v, d)); }
    __device__ static __forceinline__ void st(__hip_bfloat16* p, float v, float d) { *p = cvt(v, d); }
};

// Stores through a buffer resource over a job's populations (at most 4 GiB): the per-lane offset
// of the node is shared by all planes, the plane's offset rides in a scalar register.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t pop_rsrc(void* base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, float v, unsigned voff, unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, __half v, unsigned voff, unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, __hip_bfloat16 v, unsigned voff, unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, (int)voff, (int)soff, 0);
}
// Loads of one stored value, in storage units, through the same kind of resource.
template <typename S> __device__ __forceinline__ float buf_ld_raw(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <> __device__ __forceinline__ float buf_ld_raw<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <> __device__ __forceinline__ float buf_ld_raw<__half>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __half2float(__builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0)));
}
template <> __device__ __forceinline__ float buf_ld_raw<__hip_bfloat16>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return __uint_as_float((unsigned)__builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0) << 16);
}

// Counter-based random offsets of one node and step: a 32-bit integer hash (multiply-xorshift) of
// the node index and the job's step counter, continued by one xorshift step; its eight bytes give
// eight offsets d, and population i takes offset i mod 8.  A job's offsets depend only on its own
// node indices and steps, so its results are the same alone and in any batch.
__device__ __forceinline__ unsigned mix32(unsigned x) {
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}
__device__ __forceinline__ unsigned xorshift32(unsigned x) {
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
}

// ---------------------------------------------------------------- Zou-He closure
// Wet wall node on the face of axis a: low face (side 0, inward normal +a) or high face
// (side 1, inward normal -a).  Unknown populations have e_a == s (s = +1 low, -1 high).
// Momentum target m = rho u_w - G/2 so that the Guo velocity of the node equals u_w.
// Written on deviations g = f - w: weights of opposite directions are equal, and the known
// weights sum to 1 in the density balance.
__device__ __forceinline__ void zou_he(const JobDev& J, int a, int side, float g[Q]) {
    const int s = side == 0 ? 1 : -1;
    // wall velocity of the node's face, selected from the two uniform faces of axis a
    float uw[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) uw[c] = side == 0 ? J.wall_u[2 * a][c] : J.wall_u[2 * a + 1][c];
    const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
    float sum0 = 0.f, summ = 0.f, t1 = 0.f, t2 = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int ea = ce(i, 0) * (a == 0) + ce(i, 1) * (a == 1) + ce(i, 2) * (a == 2);
        const int eb1 = ce(i, 0) * (b1 == 0) + ce(i, 1) * (b1 == 1) + ce(i, 2) * (b1 == 2);
        const int eb2 = ce(i, 0) * (b2 == 0) + ce(i, 1) * (b2 == 1) + ce(i, 2) * (b2 == 2);
        if (ea == 0) {
            sum0 += g[i];
            t1 += g[i] * (float)eb1;
            t2 += g[i] * (float)eb2;
        } else if (ea == -s) {
            summ += g[i];
        }
    }
    const float Ga = J.G[a];
    const float drho = (sum0 + 2.f * summ - s * 0.5f * Ga + s * uw[a]) / (1.f - s * uw[a]);
    const float rho = 1.f + drho;
    const float ma = rho * uw[a] - 0.5f * J.G[a];
    const float mb1 = rho * uw[b1] - 0.5f * J.G[b1];
    const float mb2 = rho * uw[b2] - 0.5f * J.G[b2];
    const float n1 = 0.5f * t1 - mb1 * (1.f / 3.f);
    const float n2 = 0.5f * t2 - mb2 * (1.f / 3.f);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int ea = ce(i, 0) * (a == 0) + ce(i, 1) * (a == 1) + ce(i, 2) * (a == 2);
        const int eb1 = ce(i, 0) * (b1 == 0) + ce(i, 1) * (b1 == 1) + ce(i, 2) * (b1 == 2);
        const int eb2 = ce(i, 0) * (b2 == 0) + ce(i, 1) * (b2 == 1) + ce(i, 2) * (b2 == 2);
        if (ea == s) {
            const float go = g[opp(i)];
            if (eb1 == 0 && eb2 == 0)
                g[i] = go + s * ma * (1.f / 3.f);
            else if (eb1 != 0)
                g[i] = go + (s * ma + eb1 * mb1) * (1.f / 6.f) - eb1 * n1;
            else
                g[i] = go + (s * ma + eb2 * mb2) * (1.f / 6.f) - eb2 * n2;
        }
    }
}

// Inverse of the weighted moment matrix sum over unknown i of w_i (1, e_i)(1, e_i)^T of the
// populations an edge or corner node receives through its walls, for every wall configuration
// (index (s0 + 1) + 3 (s1 + 1) + 9 (s2 + 1), s_a as below), evaluated at compile time; zero
// where the node lies on fewer than two walls.  The matrix depends only on the configuration,
// so the kernel keeps no accumulators for it.
struct CornerInv { float a[4][4]; };
struct CornerTable { CornerInv t[27]; };
constexpr CornerTable make_corner_table() {
    CornerTable T{};
    for (int t = 0; t < 27; ++t) {
        const int s[3] = {t % 3 - 1, (t / 3) % 3 - 1, t / 9 - 1};
        if ((s[0] != 0) + (s[1] != 0) + (s[2] != 0) < 2) continue;
        double M[4][8] = {};   // [A | I], reduced to [I | A^-1]
        for (int i = 0; i < Q; ++i) {
            bool unk = false;
            for (int a = 0; a < 3; ++a)
                if (s[a] != 0 && ce(i, a) == -s[a]) unk = true;
            if (!unk) continue;
            const double p[4] = {1.0, (double)cx(i), (double)cy(i), (double)cz(i)};
            for (int r = 0; r < 4; ++r)
                for (int c = 0; c < 4; ++c) M[r][c] += wq(i) * p[r] * p[c];
        }
        for (int r = 0; r < 4; ++r) M[r][4 + r] = 1.0;
        for (int c = 0; c < 4; ++c) {   // Gauss-Jordan; A is symmetric positive definite
            const double piv = M[c][c];
            for (int k = 0; k < 8; ++k) M[c][k] /= piv;
            for (int r = 0; r < 4; ++r) {
                if (r == c) continue;
                const double f = M[r][c];
                for (int k = 0; k < 8; ++k) M[r][k] -= f * M[c][k];
            }
        }
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) T.t[t].a[r][c] = (float)M[r][4 + c];
    }
    return T;
}
// every entry inverts its matrix (checked when compiling)
constexpr bool corner_table_ok() {
    const CornerTable T = make_corner_table();
    for (int t = 0; t < 27; ++t) {
        const int s[3] = {t % 3 - 1, (t / 3) % 3 - 1, t / 9 - 1};
        if ((s[0] != 0) + (s[1] != 0) + (s[2] != 0) < 2) continue;
        double M[4][4] = {};
        for (int i = 0; i < Q; ++i) {
            bool unk = false;
            for (int a = 0; a < 3; ++a)
                if (s[a] != 0 && ce(i, a) == -s[a]) unk = true;
            if (!unk) continue;
            const double p[4] = {1.0, (double)cx(i), (double)cy(i), (double)cz(i)};
            for (int r = 0; r < 4; ++r)
                for (int c = 0; c < 4; ++c) M[r][c] += wq(i) * p[r] * p[c];
        }
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) {
                double acc = 0.0;
                for (int k = 0; k < 4; ++k) acc += M[r][k] * (double)T.t[t].a[k][c];
                const double err = acc - (r == c ? 1.0 : 0.0);
                if (err > 1e-5 || err < -1e-5) return false;
            }
    }
    return true;
}
static_assert(corner_table_ok(), "edge and corner moment inverses inconsistent");
__constant__ const CornerTable kCornerInv = make_corner_table();

// Edge or corner node of a box with Zou-He walls on several axes (s_a = -1 / +1 on the low /
// high wall of axis a, 0 off the walls of a).  The paper leaves these nodes open; they are
// closed as follows.  Unknown are the populations streamed in through any of the node's walls.
// On entry their slots hold the redirected loads, the node's own outgoing deviations opposite to
// them, so the sum of g balances the node's mass through its walls and gives its density.  The
// wall velocity is zero along the node's wall normals and the mean of its faces' velocities
// along the other axes.  An unknown whose opposite is known takes it plus 6 w_i (e_i . m)
// (bounce-back of the non-equilibrium part); one whose opposite is unknown too (a link buried
// in the wall) takes the equilibrium.  A correction w_i (l0 + l . e_i) over the unknowns, l the
// inverse of their weighted moment matrix applied to the residual, then sets the mass and the
// momentum m = rho u_w - G/2 exactly.
__device__ __forceinline__ void zou_he_corner(const JobDev& J, int s0, int s1, int s2, float g[Q]) {
    float drho = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) drho += g[i];
    const float rho = 1.f + drho;
    const float inw = 1.f / (float)((s0 != 0) + (s1 != 0) + (s2 != 0));
    float uw[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        float acc = 0.f;
        if (s0) acc += J.wall_u[s0 > 0 ? 1 : 0][d];
        if (s1) acc += J.wall_u[s1 > 0 ? 3 : 2][d];
        if (s2) acc += J.wall_u[s2 > 0 ? 5 : 4][d];
        const int sd = d == 0 ? s0 : (d == 1 ? s1 : s2);
        uw[d] = sd != 0 ? 0.f : acc * inw;
    }
    const float m0 = rho * uw[0] - 0.5f * J.G[0];
    const float m1 = rho * uw[1] - 0.5f * J.G[1];
    const float m2 = rho * uw[2] - 0.5f * J.G[2];
    const float uu = uw[0] * uw[0] + uw[1] * uw[1] + uw[2] * uw[2];
    // unknown: e_i points into the fluid through one of the node's walls
#define LBIB_UNK(i) ((s0 != 0 && cx(i) == -s0) || (s1 != 0 && cy(i) == -s1) || (s2 != 0 && cz(i) == -s2))
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (!LBIB_UNK(i)) continue;
        const float w = (float)wq(i);
        if (!LBIB_UNK(opp(i))) {
            g[i] = g[opp(i)] + 6.f * w * (cx(i) * m0 + cy(i) * m1 + cz(i) * m2);
        } else {
            const float eu = cx(i) * uw[0] + cy(i) * uw[1] + cz(i) * uw[2];
            g[i] = w * (drho + rho * (3.f * eu + 4.5f * eu * eu - 1.5f * uu));
        }
    }
    // residual of mass and momentum
    float r0 = drho, r1 = m0, r2 = m1, r3 = m2;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        r0 -= g[i];
        if (cx(i)) r1 -= cx(i) * g[i];
        if (cy(i)) r2 -= cy(i) * g[i];
        if (cz(i)) r3 -= cz(i) * g[i];
    }
    const CornerInv& A = kCornerInv.t[(s0 + 1) + 3 * (s1 + 1) + 9 * (s2 + 1)];
    const float x0 = A.a[0][0] * r0 + A.a[0][1] * r1 + A.a[0][2] * r2 + A.a[0][3] * r3;
    const float x1 = A.a[1][0] * r0 + A.a[1][1] * r1 + A.a[1][2] * r2 + A.a[1][3] * r3;
    const float x2 = A.a[2][0] * r0 + A.a[2][1] * r1 + A.a[2][2] * r2 + A.a[2][3] * r3;
    const float x3 = A.a[3][0] * r0 + A.a[3][1] * r1 + A.a[3][2] * r2 + A.a[3][3] * r3;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        if (LBIB_UNK(i)) g[i] += (float)wq(i) * (x0 + cx(i) * x1 + cy(i) * x2 + cz(i) * x3);
#undef LBIB_UNK
}

// ---------------------------------------------------------------- pull
// Walls of job J: bit f (lbib_bc face order) set for a face that is not periodic; WALL_TERMS set
// when some wall adds a term to the redirected populations (a moving bounce-back wall, or a
// Zou-He wall whose unknowns are rebuilt).  Halfway bounce-back at rest is the redirect alone.
constexpr unsigned WALL_TERMS = 64u;
__device__ __forceinline__ unsigned wall_faces(const JobDev& J) {
    unsigned m = 0;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        m |= (J.bc[f] != 0 ? 1u : 0u) << f;
        const bool moving = J.wall_u[f][0] != 0.f || J.wall_u[f][1] != 0.f || J.wall_u[f][2] != 0.f;
        if (J.bc[f] == 1 || (J.bc[f] == 2 && moving)) m |= WALL_TERMS;
    }
    return m;
}

// Post-streaming deviations at node (x, y, z) of job J from the post-collision buffer src.
// All 19 loads are issued unconditionally, so they are in flight together: a source outside
// the domain is redirected to the node's own opposite population (the halfway bounce-back
// source, always a valid address), and the wall term or the Zou-He closure is applied once
// the loads have returned.  Without ZH_CLOSURE the populations of Zou-He wall nodes stay
// unclosed (finite but meaningless): for readers that never look at those nodes.

template <typename S, bool ZH_CLOSURE = true, bool OFF32 = false, bool RAW = false, bool YZ_FAST = false>
__device__ __forceinline__ void pull(const S* __restrict__ src, const JobDev& J, int x, int y,
                                     int z, long long k, float g[Q], unsigned walls) {
    const long long N = J.n;
    const int nx = J.nx, ny = J.ny, nz = J.nz;
    const int sy = nx, sz = nx * ny;
    // linear displacement of the source for e = +1 (node c - 1) and e = -1 (node c + 1): a
    // neighbour across a periodic face wraps; across a wall the source is redirected (flags)
    const bool lx = x == 0, hx = x == nx - 1, ly = y == 0, hy = y == ny - 1, lz = z == 0, hz = z == nz - 1;
    const bool oxm = lx & ((walls & 1u) != 0), oxp = hx & ((walls & 2u) != 0);
    const bool oym = ly & ((walls & 4u) != 0), oyp = hy & ((walls & 8u) != 0);
    const bool ozm = lz & ((walls & 16u) != 0), ozp = hz & ((walls & 32u) != 0);
    const int dxm = (lx & !oxm) ? nx - 1 : -1, dxp = (hx & !oxp) ? 1 - nx : 1;
    const int dym = (ly & !oym) ? (ny - 1) * sy : -sy, dyp = (hy & !oyp) ? (1 - ny) * sy : sy;
    const int dzm = (lz & !ozm) ? (nz - 1) * sz : -sz, dzp = (hz & !ozp) ? (1 - nz) * sz : sz;
    // Waves whose nodes all lie away from the y and z faces: the y and z parts of every source
    // shift are the same on every lane, so a stream without an x part loads at the node's own
    // offset with the shift in a scalar register, and a stream with one adds only the lane's x
    // part (the periodic wrap, or the wall redirect, at x = 0 and x = nx - 1).  Same addresses,
    // same values as the general form below.
    if (OFF32 && YZ_FAST && __all(y > 0 && y < ny - 1 && z > 0 && z < nz - 1)) {
        const unsigned pb = (unsigned)N * (unsigned)sizeof(S), kb = (unsigned)k * (unsigned)sizeof(S);
        const __amdgpu_buffer_rsrc_t rs = pop_rsrc((void*)src, Q * pb);
        const unsigned kxm = kb + (unsigned)(dxm * (int)sizeof(S)), kxp = kb + (unsigned)(dxp * (int)sizeof(S));
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int e0 = cx(i), e1 = cy(i), e2 = cz(i);
            const unsigned syz = (unsigned)i * pb - (unsigned)((e1 * sy + e2 * sz) * (int)sizeof(S));
            float v;
            if (e0 == 0) {
                v = buf_ld_raw<S>(rs, kb, syz);
            } else {
                const bool o = e0 == 1 ? oxm : oxp;
                const unsigned alt = (unsigned)opp(i) * pb + kb, nrm = (e0 == 1 ? kxm : kxp) + syz;
                v = buf_ld_raw<S>(rs, o ? alt : nrm, 0u);
            }
            g[i] = RAW ? v : v * (1.0f / Codec<S>::scale);
        }
    } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int e0 = cx(i), e1 = cy(i), e2 = cz(i);
        const int d = (e0 == 1 ? dxm : (e0 == -1 ? dxp : 0)) + (e1 == 1 ? dym : (e1 == -1 ? dyp : 0)) +
                      (e2 == 1 ? dzm : (e2 == -1 ? dzp : 0));
        // bitwise or: no short-circuit branches, the redirect is a per-lane select
        const bool o = (e0 == 1 ? oxm : (e0 == -1 ? oxp : false)) |
                       (e1 == 1 ? oym : (e1 == -1 ? oyp : false)) |
                       (e2 == 1 ? ozm : (e2 == -1 ? ozp : false));
        if (OFF32) {
            // the job's populations span less than 4 GiB: one 32-bit byte offset per load
            const unsigned pb = (unsigned)N * (unsigned)sizeof(S), kb = (unsigned)k * (unsigned)sizeof(S);
            unsigned alt = (unsigned)opp(i) * pb + kb, nrm = (unsigned)i * pb + kb + (unsigned)(d * (int)sizeof(S));
            // both offsets are formed in registers: a lane select, not a branch around either sum
            asm("" : "+v"(alt));
            asm("" : "+v"(nrm));
            const S* p = (const S*)((const char*)src + (o ? alt : nrm));
            g[i] = RAW ? Codec<S>::raw(p) : Codec<S>::ld(p);
        } else {
            const long long idx = o ? (long long)opp(i) * N + k : (long long)i * N + k + d;
            g[i] = RAW ? Codec<S>::raw(src + idx) : Codec<S>::ld(src + idx);
        }
    }
    }
    if (!(walls & WALL_TERMS) || !(oxm || oxp || oym || oyp || ozm || ozp)) return;
    // the wall terms are formed on deviations (exact power-of-two rescaling of raw values)
    constexpr bool RESCALE = RAW && Codec<S>::scale != 1.0f;
    if (RESCALE) {
#pragma unroll
        for (int i = 0; i < Q; ++i) g[i] *= 1.0f / Codec<S>::scale;
    }
    // face kinds and wall velocities are uniform over the job: select among them per lane
    bool bb[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) bb[f] = J.bc[f] == 2;
    bool unknown = false;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int e0 = cx(i), e1 = cy(i), e2 = cz(i);
        const bool o0 = e0 == 1 ? oxm : (e0 == -1 ? oxp : false);
        const bool o1 = e1 == 1 ? oym : (e1 == -1 ? oyp : false);
        const bool o2 = e2 == 1 ? ozm : (e2 == -1 ? ozp : false);
        if (!(o0 || o1 || o2)) continue;
        // faces crossed on each axis (meaningful only where that axis is crossed)
        const int f0 = e0 == 1 ? 0 : 1, f1 = e1 == 1 ? 2 : 3, f2 = e2 == 1 ? 4 : 5;
        const bool isbb = o0 ? bb[f0] : (o1 ? bb[f1] : bb[f2]);
        if (isbb) {
            float uwx = 0.f, uwy = 0.f, uwz = 0.f;
            if (o0) { uwx += J.wall_u[f0][0]; uwy += J.wall_u[f0][1]; uwz += J.wall_u[f0][2]; }
            if (o1) { uwx += J.wall_u[f1][0]; uwy += J.wall_u[f1][1]; uwz += J.wall_u[f1][2]; }
            if (o2) { uwx += J.wall_u[f2][0]; uwy += J.wall_u[f2][1]; uwz += J.wall_u[f2][2]; }
            const float eu = e0 * uwx + e1 * uwy + e2 * uwz;
            g[i] = g[i] + (float)(6.0 * wq(i)) * eu;
        } else {
            unknown = true;   // rebuilt by the closure; the slot keeps the redirected load
        }
    }
    if (ZH_CLOSURE && unknown) {
        const int s0 = oxm && J.bc[0] == 1 ? -1 : (oxp && J.bc[1] == 1 ? 1 : 0);
        const int s1 = oym && J.bc[2] == 1 ? -1 : (oyp && J.bc[3] == 1 ? 1 : 0);
        const int s2 = ozm && J.bc[4] == 1 ? -1 : (ozp && J.bc[5] == 1 ? 1 : 0);
        if ((s0 != 0) + (s1 != 0) + (s2 != 0) == 1) {
            const int a = s0 ? 0 : (s1 ? 1 : 2);
            zou_he(J, a, (s0 + s1 + s2) > 0 ? 1 : 0, g);
        } else {
            zou_he_corner(J, s0, s1, s2, g);
        }
    }
    if (RESCALE) {
#pragma unroll
        for (int i = 0; i < Q; ++i) g[i] *= Codec<S>::scale;
    }
}


__device__ __forceinline__ void node_coords(const JobDev& J, long long k, int& x, int& y, int& z) {
    const unsigned kk = (unsigned)k;
    const unsigned nx = (unsigned)J.nx, ny = (unsigned)J.ny;
    const unsigned q = kk / nx;
    x = (int)(kk - q * nx);
    z = (int)(q / ny);
    y = (int)(q - (unsigned)z * ny);
}

// Body force at a node: uniform G plus the fixed-point immersed-boundary force of every body
// of the job whose force window holds the node.
__device__ __forceinline__ void node_force(const Pools& P, const JobDev& J, int x, int y, int z,
                                           float F[3]) {
    F[0] = J.G[0]; F[1] = J.G[1]; F[2] = J.G[2];
    for (int b = J.body0; b < J.body0 + J.nbodies; ++b) {
        const WinDesc d = P.fdesc[b];
        const BodyDev& B = P.bodies[b];
        const int dims[3] = {J.nx, J.ny, J.nz};
        if (!win_valid(d, dims, B.win_cap, J.bc)) continue;
        int lx = x - d.o[0], ly = y - d.o[1], lz = z - d.o[2];
        if (lx < 0) lx += J.nx;
        if (ly < 0) ly += J.ny;
        if (lz < 0) lz += J.nz;
        if (lx < d.w[0] && ly < d.w[1] && lz < d.w[2]) {
            const long long capn = (long long)B.win_cap[0] * B.win_cap[1] * B.win_cap[2];
            const long long l = lx + (long long)d.w[0] * (ly + (long long)d.w[1] * lz);
            const long long* fw = P.fwin + 3 * B.win_off + l;
            F[0] += (float)((double)fw[0] * FIX_INV);
            F[1] += (float)((double)fw[capn] * FIX_INV);
            F[2] += (float)((double)fw[2 * capn] * FIX_INV);
        }
    }
}

// ---------------------------------------------------------------- fused sweep
// Force window of a lattice's only body, read once per block, before the block's first store.
struct Win1 {
    int o[3], w[3];
    long long capn;
    const long long* fw;
    bool valid;
};

__device__ __forceinline__ Win1 load_win1(const Pools& P, const JobDev& J) {
    Win1 W;
    const int b = J.body0;
    const WinDesc d = P.fdesc[b];
    const BodyDev& B = P.bodies[b];
    const int dims[3] = {J.nx, J.ny, J.nz};
    W.valid = win_valid(d, dims, B.win_cap, J.bc);
    for (int a = 0; a < 3; ++a) { W.o[a] = d.o[a]; W.w[a] = d.w[a]; }
    W.capn = (long long)B.win_cap[0] * B.win_cap[1] * B.win_cap[2];
    W.fw = P.fwin + 3 * B.win_off;
    return W;
}
// The same for a batch of one lattice whose one body (index 0) comes with the kernel arguments:
// the layout load does not wait for the job record.
__device__ __forceinline__ Win1 load_win1_one(const Pools& P, const JobDev& J) {
    Win1 W;
    const WinDesc d = P.fdesc[0];
    const BodyDev& B = P.solo_body;
    const int dims[3] = {J.nx, J.ny, J.nz};
    W.valid = win_valid(d, dims, B.win_cap, J.bc);
    for (int a = 0; a < 3; ++a) { W.o[a] = d.o[a]; W.w[a] = d.w[a]; }
    W.capn = (long long)B.win_cap[0] * B.win_cap[1] * B.win_cap[2];
    W.fw = P.fwin + 3 * B.win_off;
    return W;
}

// Body force at a node: uniform G plus the fixed-point immersed-boundary force of the window that
// holds the node (one body: W; more: every body's window in turn).
__device__ __forceinline__ void sweep_force(const Pools& P, const JobDev& J, const Win1& W, int x, int y,
                                            int z, float F[3]) {
    F[0] = J.G[0]; F[1] = J.G[1]; F[2] = J.G[2];
    if (J.nbodies == 0) return;
    if (J.nbodies > 1) { node_force(P, J, x, y, z, F); return; }
    if (!W.valid) return;
    int lx = x - W.o[0], ly = y - W.o[1], lz = z - W.o[2];
    if (lx < 0) lx += J.nx;
    if (ly < 0) ly += J.ny;
    if (lz < 0) lz += J.nz;
    if (lx < W.w[0] && ly < W.w[1] && lz < W.w[2]) {
        const unsigned l = (unsigned)lx + (unsigned)W.w[0] * ((unsigned)ly + (unsigned)W.w[1] * (unsigned)lz);
        const long long* fw = W.fw + l;
        F[0] += (float)((double)fw[0] * FIX_INV);
        F[1] += (float)((double)fw[W.capn] * FIX_INV);
        F[2] += (float)((double)fw[2 * W.capn] * FIX_INV);
    }
}

// BGK relaxation with Guo forcing (Eqs. (2)-(4) on deviations g = f - w) of one node's pulled
// populations, in storage units (the deviation times SC, an exact power of two): the equilibrium
// and forcing terms carry the factor SC in their weights.  Opposite populations i and i' share
// e.u, e.F and the even parts of both terms, which enter with the opposite sign for the odd
// parts: per pair, the equilibrium is w (a + b) for i and w (a - b) for i', the forcing C + D and
// C - D.  The weight multiplies the sum last, as in the per-population form: a weight applied to
// rho or drho first (w rho, w drho) rounds the same way at every node of a near-unit density and
// biases the equilibrium, an error that grows with the step count instead of averaging out.
// Without FORCED the force is zero at every lane (the forcing terms vanish).  Each result goes to
// emit(i, value) as soon as it is formed.
template <typename S, bool FORCED, typename Emit>
__device__ __forceinline__ void bgk_guo(const float g[Q], float drho, float rho, float ux, float uy, float uz,
                                        const float F[3], float om, float gk, Emit emit) {
    constexpr float SC = Codec<S>::scale;
    const float mu = -1.5f * (ux * ux + uy * uy + uz * uz);
    const float muF = FORCED ? -3.f * (ux * F[0] + uy * F[1] + uz * F[2]) : 0.f;
    {
        const float w = SC * (float)wq(0);
        const float geq = w * (drho + rho * mu);
        float v = g[0] - om * (g[0] - geq);
        if (FORCED) v += gk * w * muF;
        emit(0, v);
    }
    const float rho3 = 3.f * rho;
    // forcing weights per class (axis, diagonal): 3 gk w, 9 gk w, gk w (-3 u.F)
    float gw3[2], gw9[2], gmu[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        if (FORCED) {
            const float gw = gk * (SC * (float)wq(c == 0 ? 1 : 7));
            gw3[c] = 3.f * gw;
            gw9[c] = 9.f * gw;
            gmu[c] = gw * muF;
        }
    }
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int o = opp(i);
        if (o < i) continue;   // i is the first of its pair
        const int c = i <= 6 ? 0 : 1;
        const float w = SC * (float)wq(i);
        const float eu = cx(i) * ux + cy(i) * uy + cz(i) * uz;
        const float a = fmaf(rho, fmaf(4.5f * eu, eu, mu), drho);
        const float b = rho3 * eu;
        float vp = g[i] - om * (g[i] - w * (a + b));
        float vm = g[o] - om * (g[o] - w * (a - b));
        if (FORCED) {
            const float eF = cx(i) * F[0] + cy(i) * F[1] + cz(i) * F[2];
            const float C = fmaf(gw9[c] * eu, eF, gmu[c]);
            const float D = gw3[c] * eF;
            vp += C + D;
            vm += C - D;
        }
        emit(i, vp);
        emit(o, vm);
    }
}

// One node: pull, moments, body force, BGK collision with Guo forcing (all on deviations),
// store.  With COLLIDE false the pulled values are stored unchanged (pure streaming).  Stores go to
// the population planes through a 32-bit byte offset of the node (the same for every plane).
// Populations stay in storage units from load to store; the moments are scaled back exactly.
template <typename S, bool COLLIDE, bool OFF32, bool YZ_FAST>
__device__ __forceinline__ void sweep_node(const Pools& P, const JobDev& J, const Win1& W,
                                           const S* __restrict__ src, S* __restrict__ dst, long long k,
                                           int x, int y, int z, int job, unsigned seed, unsigned walls) {
    float g[Q];
    pull<S, true, OFF32, true, YZ_FAST>(src, J, x, y, z, k, g, walls);
    const long long N = J.n;
    const unsigned kb = (unsigned)k * (unsigned)sizeof(S);
    const long long pb = N * (long long)sizeof(S);   // bytes per population plane
    char* plane = (char*)dst;                         // plane i of the destination, stepped by pb
    const __amdgpu_buffer_rsrc_t rs = pop_rsrc(dst, OFF32 ? (unsigned)(Q * pb) : 0u);
    if (COLLIDE) {
        constexpr float ISC = 1.0f / Codec<S>::scale;
        // moments from the sums and differences of opposite pairs
        float ds = g[0], jxs = 0.f, jys = 0.f, jzs = 0.f;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int o = opp(i);
            if (o < i) continue;
            const float sp = g[i] + g[o], dp = g[i] - g[o];
            ds += sp;
            if (cx(i)) jxs += cx(i) * dp;
            if (cy(i)) jys += cy(i) * dp;
            if (cz(i)) jzs += cz(i) * dp;
        }
        const float drho = ds * ISC, jx = jxs * ISC, jy = jys * ISC, jz = jzs * ISC;
        float F[3];
        sweep_force(P, J, W, x, y, z, F);
        const float rho = 1.f + drho;
        const float ir = 1.f / rho;
        const float ux = (jx + 0.5f * F[0]) * ir;
        const float uy = (jy + 0.5f * F[1]) * ir;
        const float uz = (jz + 0.5f * F[2]) * ir;
        const float om = J.omega, gk = J.guo;
        // runaway sentinel: non-finite, or a density no flow of the scheme reaches (the singular
        // lid edges of a cavity at lid Mach 0.6 reach about 2.7)
        if (!(drho > -0.95f && drho < 7.f)) atomicOr(P.flags + job, FLAG_NONFINITE);
        // FP32: each result is stored as soon as it is formed (plane i at byte i * pb).  Narrow
        // types gather the results first: the offsets of the stochastic narrowing are drawn after
        // the collision, so they do not hold registers through it.
        constexpr bool DIRECT = sizeof(S) == 4;
        float out[Q];
        const auto emit = [&](int i, float v) {
            if (DIRECT) {
                if (OFF32) buf_st(rs, Narrow<S>::cvt(v, 0.f), kb, (unsigned)i * (unsigned)pb);
                else Narrow<S>::st((S*)((char*)dst + (long long)i * pb + kb), v, 0.f);
            } else {
                out[i] = v;
            }
        };
        // the forcing terms are formed only in waves where some node carries a force
        if (__any(F[0] != 0.f || F[1] != 0.f || F[2] != 0.f))
            bgk_guo<S, true>(g, drho, rho, ux, uy, uz, F, om, gk, emit);
        else
            bgk_guo<S, false>(g, drho, rho, ux, uy, uz, F, om, gk, emit);
        if (!DIRECT) {
            // offsets of the stochastic narrowing
            float dof[8];
            unsigned rw[2];
            rw[0] = mix32((unsigned)k * 0x9E3779B9U ^ seed);
            rw[1] = xorshift32(rw[0]);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int r = (int)(rw[q / 4] << (24 - 8 * (q % 4))) >> 24;   // -128..127
                // (r + 1/2) ulp / 256, exact (the step is a power of two)
                dof[q] = fmaf((float)r, Narrow<S>::ulp * (1.f / 256.f), Narrow<S>::ulp * (0.5f / 256.f));
            }
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                if (OFF32) {
                    buf_st(rs, Narrow<S>::cvt(out[i], dof[i % 8]), kb, (unsigned)i * (unsigned)pb);
                } else {
                    Narrow<S>::st((S*)(plane + kb), out[i], dof[i % 8]);
                    plane += pb;
                }
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            if (OFF32) {
                buf_st(rs, Narrow<S>::cvt(g[i], 0.f), kb, (unsigned)i * (unsigned)pb);
            } else {
                Codec<S>::st_raw((S*)(plane + kb), g[i]);
                plane += pb;
            }
        }
    }
}

// ONE: a batch of one lattice.  Its job (0) and body need no tile-table entry, so the job record,
// the step counter and the force-window layout load at once, in parallel with the tile entry,
// instead of one after the other at the start of every block.
template <typename S, bool COLLIDE, int NPT, bool OFF32, bool ONE>
__global__ void __launch_bounds__(1024) k_sweep(Pools P, int a_to_b, int xcd_chunk) {
    // The dispatcher deals consecutive blocks to the 8 XCDs in turn, each with its own L2.
    // With xcd_chunk = C > 0 the blocks are remapped so that every XCD takes C consecutive
    // tiles per turn: the rows a tile pulls from its neighbours were mostly just read through
    // the same L2.  Blocks past the last whole turn keep their own tile (a bijection).
    const int T = gridDim.x, bid = blockIdx.x;
    int tile = bid;
    if (xcd_chunk > 0) {
        const int span = 8 * xcd_chunk;
        if (bid < (T / span) * span) tile = (bid / span) * span + (bid & 7) * xcd_chunk + (bid >> 3) % xcd_chunk;
    }
    const int4 te = P.tiles[tile];
    const int job = ONE ? 0 : te.x;
    const JobDev& J = P.jobs[job];
    const S* src = (const S*)(a_to_b ? P.popA : P.popB) + J.pop_off;
    S* dst = (S*)(a_to_b ? P.popB : P.popA) + J.pop_off;
    const long long base = (long long)(tile - J.tile0) * blockDim.x * NPT;
    Win1 W = {};
    if (ONE) {
        if (COLLIDE && P.solo_job >= 0) W = load_win1_one(P, J);
    } else if (COLLIDE && J.nbodies == 1) {
        W = load_win1(P, J);
    }
    const unsigned nx = (unsigned)J.nx, ny = (unsigned)J.ny, mx = J.mx, my = J.my;
    const unsigned walls = wall_faces(J);
    // the job's step counter of the buffer being read seeds the stochastic narrowing; the block of
    // the job's first tile hands the next value to the other buffer's slot, read by the next step
    unsigned seed = 0;
    if (COLLIDE && sizeof(S) < 4) {
        const unsigned* ctr = P.sr_ctr + 2 * job;
        const unsigned c = ctr[a_to_b ? 0 : 1];
        if (tile == (ONE ? 0 : J.tile0) && threadIdx.x == 0) P.sr_ctr[2 * job + (a_to_b ? 1 : 0)] = c + 1;
        seed = mix32(c + 0x632BE5ABU);
    }
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
        // coordinates from those of the tile's first node (tile table): row and plane carries by
        // multiply-high with the job's reciprocals (exact for these small numerators)
        const long long k = base + (long long)r * blockDim.x + threadIdx.x;
        if (k >= J.n) continue;
        const unsigned x0 = (unsigned)te.y, y0 = (unsigned)te.z, z0 = (unsigned)te.w;
        const unsigned xs = x0 + (unsigned)(r * blockDim.x) + threadIdx.x;
        const unsigned qx = mx ? __umulhi(xs, mx) : xs / nx;
        const unsigned ys = y0 + qx;
        const unsigned qy = my ? __umulhi(ys, my) : ys / ny;
        // the scalar-shift pull only in the one-node-per-thread form: unrolled over several
        // nodes per thread its second code path made those forms slower
        sweep_node<S, COLLIDE, OFF32, NPT == 1>(P, J, W, src, dst, k, (int)(xs - qx * nx), (int)(ys - qy * ny), (int)(z0 + qy),
                               job, seed, walls);
    }
}

template <typename S, bool C, int NPT, bool OFF32, bool ONE = false>
static void sweep_n(const Pools& P, bool a_to_b, int chunk, dim3 grid, dim3 block, hipStream_t s,
                    hipEvent_t ev0, hipEvent_t ev1) {
    if (ev0 || ev1)
        hipExtLaunchKernelGGL((k_sweep<S, C, NPT, OFF32, ONE>), grid, block, 0, s, ev0, ev1, 0, P, (int)a_to_b, chunk);
    else
        hipLaunchKernelGGL((k_sweep<S, C, NPT, OFF32, ONE>), grid, block, 0, s, P, (int)a_to_b, chunk);
}

template <typename S, bool C, bool OFF32>
static void sweep_o(const Pools& P, bool a_to_b, int ntiles, SweepShape sh, int chunk, hipStream_t s,
                    hipEvent_t ev0, hipEvent_t ev1) {
    dim3 grid(ntiles), block(sh.block);
    switch (sh.npt) {
        case 1:
            // a single lattice keeps one node per thread; batches may autotune to any shape
            if (P.one_lattice) sweep_n<S, C, 1, OFF32, true>(P, a_to_b, chunk, grid, block, s, ev0, ev1);
            else sweep_n<S, C, 1, OFF32>(P, a_to_b, chunk, grid, block, s, ev0, ev1);
            break;
        case 2: sweep_n<S, C, 2, OFF32>(P, a_to_b, chunk, grid, block, s, ev0, ev1); break;
        default: sweep_n<S, C, 4, OFF32>(P, a_to_b, chunk, grid, block, s, ev0, ev1); break;
    }
}

template <typename S, bool C>
static void sweep_t(const Pools& P, bool a_to_b, int ntiles, SweepShape sh, int chunk, hipStream_t s,
                    hipEvent_t ev0, hipEvent_t ev1) {
    if (P.pop32) sweep_o<S, C, true>(P, a_to_b, ntiles, sh, chunk, s, ev0, ev1);
    else sweep_o<S, C, false>(P, a_to_b, ntiles, sh, chunk, s, ev0, ev1);
}

void launch_sweep(const Pools& P, int storage, bool collide, bool a_to_b, int ntiles,
                  SweepShape shape, int xcd_chunk, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (ntiles <= 0) return;
    const int c = xcd_chunk;
    if (storage == 0) collide ? sweep_t<float, true>(P, a_to_b, ntiles, shape, c, s, ev0, ev1)
                              : sweep_t<float, false>(P, a_to_b, ntiles, shape, c, s, ev0, ev1);
    else if (storage == 1) collide ? sweep_t<__half, true>(P, a_to_b, ntiles, shape, c, s, ev0, ev1)
                                   : sweep_t<__half, false>(P, a_to_b, ntiles, shape, c, s, ev0, ev1);
    else collide ? sweep_t<__hip_bfloat16, true>(P, a_to_b, ntiles, shape, c, s, ev0, ev1)
                 : sweep_t<__hip_bfloat16, false>(P, a_to_b, ntiles, shape, c, s, ev0, ev1);
}

// ---------------------------------------------------------------- window moments
// For every node of a body's current window: pull the post-streaming state, store
// (rho - 1, u*) with u* = sum f e / rho, and clear the force window for the next step.
template <typename S, bool SOLO>
__global__ void __launch_bounds__(256) k_window_moments(Pools P, int from_b) {
    // blocks of a body are proportional to its window capacity; they stride over the current
    // window, which is usually far smaller than the capacity
    const int b = block_body<SOLO>(P, P.blk_body_w, blockIdx.x);
    const BodyDev& B = body_of<SOLO>(P, b);
    const JobDev& J = body_job<SOLO>(P, B);
    const int lb = blockIdx.x - B.blk_w0;
    const WinDesc d = P.fdesc[b];
    const int dims[3] = {J.nx, J.ny, J.nz};
    if (!win_valid(d, dims, B.win_cap, J.bc)) {
        if (lb == 0 && threadIdx.x == 0) atomicOr(P.flags + B.job, FLAG_WINDOW);
        return;
    }
    if (lb == 0 && threadIdx.x == 0) P.mdesc[b] = d;
    // window sizes are bounded by the capacity, far below 2^31 nodes: 32-bit index arithmetic
    const unsigned nw = (unsigned)d.w[0] * d.w[1] * d.w[2];
    const unsigned w0 = d.w[0], w01 = (unsigned)d.w[0] * d.w[1];
    const long long capn = (long long)B.win_cap[0] * B.win_cap[1] * B.win_cap[2];
    const S* src = (const S*)(from_b ? P.popB : P.popA) + J.pop_off;
    const unsigned stride = (unsigned)B.nblk_w * blockDim.x;
    for (unsigned l = (unsigned)lb * blockDim.x + threadIdx.x; l < nw; l += stride) {
        const unsigned lz = l / w01, rem = l - lz * w01;
        const unsigned ly = rem / w0, lx = rem - ly * w0;
        int x = d.o[0] + lx, y = d.o[1] + ly, z = d.o[2] + lz;
        if (x >= J.nx) x -= J.nx;
        if (y >= J.ny) y -= J.ny;
        if (z >= J.nz) z -= J.nz;
        const long long k = x + (long long)J.nx * (y + (long long)J.ny * z);
        // MLS supports exclude Zou-He wall nodes (their moments are never read), so the pull
        // skips the Zou-He closure here
        float g[Q];
        pull<S, false>(src, J, x, y, z, k, g, wall_faces(J));
        float drho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            drho += g[i];
            jx += cx(i) * g[i];
            jy += cy(i) * g[i];
            jz += cz(i) * g[i];
        }
        const float ir = 1.f / (1.f + drho);
        P.mwin[B.win_off + l] = make_float4(drho, jx * ir, jy * ir, jz * ir);
        long long* fw = P.fwin + 3 * B.win_off + l;
        fw[0] = 0;
        fw[capn] = 0;
        fw[2 * capn] = 0;
    }
}

void launch_window_moments(const Pools& P, int storage, bool from_b, int nblk_w, hipStream_t s) {
    if (nblk_w <= 0) return;
    dim3 grid(nblk_w), block(256);
    const bool solo = P.solo_job >= 0;
    if (storage == 0) {
        if (solo) hipLaunchKernelGGL((k_window_moments<float, true>), grid, block, 0, s, P, (int)from_b);
        else hipLaunchKernelGGL((k_window_moments<float, false>), grid, block, 0, s, P, (int)from_b);
    } else if (storage == 1) {
        if (solo) hipLaunchKernelGGL((k_window_moments<__half, true>), grid, block, 0, s, P, (int)from_b);
        else hipLaunchKernelGGL((k_window_moments<__half, false>), grid, block, 0, s, P, (int)from_b);
    } else {
        if (solo) hipLaunchKernelGGL((k_window_moments<__hip_bfloat16, true>), grid, block, 0, s, P, (int)from_b);
        else hipLaunchKernelGGL((k_window_moments<__hip_bfloat16, false>), grid, block, 0, s, P, (int)from_b);
    }
}

// ---------------------------------------------------------------- getters / setters
// rho - 1 and the force-free velocity u* = sum f e / rho of the post-streaming state at node k
// (moments of Eq. eqfunc), in FP32.  Both macro getters use it, so they agree bit for bit.
template <typename S>
__device__ __forceinline__ float4 node_moments(const Pools& P, const JobDev& J, int from_b, long long k) {
    int x, y, z;
    node_coords(J, k, x, y, z);
    const S* src = (const S*)(from_b ? P.popB : P.popA) + J.pop_off;
    float g[Q];
    pull<S>(src, J, x, y, z, k, g, wall_faces(J));
    float drho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        drho += g[i];
        jx += cx(i) * g[i];
        jy += cy(i) * g[i];
        jz += cz(i) * g[i];
    }
    const float ir = 1.f / (1.f + drho);
    return make_float4(drho, jx * ir, jy * ir, jz * ir);
}

template <typename S>
__global__ void k_macros(Pools P, int from_b, int job, float4* out) {
    const JobDev& J = P.jobs[job];
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= J.n) return;
    out[k] = node_moments<S>(P, J, from_b, k);
}

// The same moments widened on the device into the host layout: rho[N] (= 1 + (rho - 1)), then
// u*[3N], so one copy per field moves them to the caller.
template <typename S>
__global__ void k_macros_f64(Pools P, int from_b, int job, double* out) {
    const JobDev& J = P.jobs[job];
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= J.n) return;
    const float4 m = node_moments<S>(P, J, from_b, k);
    out[k] = 1.0 + (double)m.x;
    out[J.n + k] = (double)m.y;
    out[2 * J.n + k] = (double)m.z;
    out[3 * J.n + k] = (double)m.w;
}

// Population i of node k, post-streaming, widened to double: f_i = w_i + g_i.  The full pull
// runs for every i (the wall closure needs all of them); only plane i is written.
template <typename S>
__global__ void k_get_pop_plane(Pools P, int from_b, int job, int plane, double* out) {
    const JobDev& J = P.jobs[job];
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= J.n) return;
    int x, y, z;
    node_coords(J, k, x, y, z);
    const S* src = (const S*)(from_b ? P.popB : P.popA) + J.pop_off;
    float g[Q];
    pull<S>(src, J, x, y, z, k, g, wall_faces(J));
    float gi = g[0];
#pragma unroll
    for (int i = 1; i < Q; ++i)
        if (i == plane) gi = g[i];
    out[k] = wq(plane) + (double)gi;
}

// Inverse of the pull for population i of node (x, y, z): write the post-collision entry whose
// pull reproduces f_i.  Entries pulled from behind a Zou-He face are not representable; the
// closure rebuilds them, on edges and corners from a density that the given unknown values,
// stored in the redirected slots, make equal to the given one.  Every destination entry is
// written by exactly one (node, i), so the populations can be set one plane at a time.
template <typename S>
__device__ __forceinline__ void set_one(const JobDev& J, S* __restrict__ dst, int x, int y, int z,
                                        long long k, int i, double fi) {
    const float gi = (float)(fi - wq(i));
    const int n[3] = {J.nx, J.ny, J.nz};
    const int c[3] = {x, y, z};
    int s[3];
    int face = -1, nout = 0;
    float uw[3] = {0.f, 0.f, 0.f};
    bool zh = false;
    for (int a = 0; a < 3; ++a) {
        s[a] = c[a] - ce(i, a);
        if (s[a] < 0 || s[a] >= n[a]) {
            const int fa = 2 * a + (s[a] < 0 ? 0 : 1);
            if (J.bc[fa] == 0) {
                s[a] = s[a] < 0 ? s[a] + n[a] : s[a] - n[a];
            } else {
                ++nout;
                if (face < 0) face = fa;
                if (J.bc[fa] == 1) zh = true;
                uw[0] += J.wall_u[fa][0]; uw[1] += J.wall_u[fa][1]; uw[2] += J.wall_u[fa][2];
            }
        }
    }
    if (nout == 0) {
        Codec<S>::st(dst + (long long)i * J.n + s[0] + (long long)n[0] * (s[1] + (long long)n[1] * s[2]), gi);
    } else if (!zh && J.bc[face] == 2) {
        const float eu = cx(i) * uw[0] + cy(i) * uw[1] + cz(i) * uw[2];
        Codec<S>::st(dst + (long long)opp(i) * J.n + k, gi - (float)(6.0 * wq(i)) * eu);
    } else if (zh) {
        // the redirected slot: the edge and corner closure reads it as the mass the node sent
        // out through its walls, so the given density is kept
        Codec<S>::st(dst + (long long)opp(i) * J.n + k, gi);
    }
}

// Population `plane` of every node from f_plane[N] (double).
template <typename S>
__global__ void k_set_pop_plane(Pools P, int to_b, int job, int plane, const double* f) {
    const JobDev& J = P.jobs[job];
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= J.n) return;
    int x, y, z;
    node_coords(J, k, x, y, z);
    S* dst = (S*)(to_b ? P.popB : P.popA) + J.pop_off;
    set_one<S>(J, dst, x, y, z, k, plane, f[k]);
}

// Equilibrium Eq. (eqfunc) of rho[N], u[3N] (NULL: 1 and 0), in double, set as the
// post-streaming populations of every node.
template <typename S>
__global__ void k_init_eq(Pools P, int to_b, int job, const double* rho, const double* u) {
    const JobDev& J = P.jobs[job];
    const long long n = J.n;
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int x, y, z;
    node_coords(J, k, x, y, z);
    S* dst = (S*)(to_b ? P.popB : P.popA) + J.pop_off;
    const double r = rho ? rho[k] : 1.0;
    const double ux = u ? u[k] : 0.0, uy = u ? u[n + k] : 0.0, uz = u ? u[2 * n + k] : 0.0;
    const double uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double eu = cx(i) * ux + cy(i) * uy + cz(i) * uz;
        set_one<S>(J, dst, x, y, z, k, i, wq(i) * r * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
    }
}

#define LBIB_DISPATCH(storage, KERNEL, grid, block, s, ...)                                   \
    do {                                                                                    \
        if ((storage) == 0) hipLaunchKernelGGL(KERNEL<float>, grid, block, 0, s, __VA_ARGS__); \
        else if ((storage) == 1) hipLaunchKernelGGL(KERNEL<__half>, grid, block, 0, s, __VA_ARGS__); \
        else hipLaunchKernelGGL(KERNEL<__hip_bfloat16>, grid, block, 0, s, __VA_ARGS__);    \
    } while (0)

void launch_macros(const Pools& P, int storage, bool from_b, int job, long long n, float* out4,
                   hipStream_t s) {
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    LBIB_DISPATCH(storage, k_macros, grid, block, s, P, (int)from_b, job, (float4*)out4);
}
void launch_macros_f64(const Pools& P, int storage, bool from_b, int job, long long n, double* out,
                       hipStream_t s) {
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    LBIB_DISPATCH(storage, k_macros_f64, grid, block, s, P, (int)from_b, job, out);
}
void launch_get_pop_plane(const Pools& P, int storage, bool from_b, int job, long long n, int plane,
                          double* out, hipStream_t s) {
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    LBIB_DISPATCH(storage, k_get_pop_plane, grid, block, s, P, (int)from_b, job, plane, out);
}
void launch_set_pop_plane(const Pools& P, int storage, bool to_b, int job, long long n, int plane,
                          const double* f, hipStream_t s) {
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    LBIB_DISPATCH(storage, k_set_pop_plane, grid, block, s, P, (int)to_b, job, plane, f);
}
void launch_init_eq(const Pools& P, int storage, bool to_b, int job, long long n, const double* rho,
                    const double* u, hipStream_t s) {
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    LBIB_DISPATCH(storage, k_init_eq, grid, block, s, P, (int)to_b, job, rho, u);
}

}  // namespace lbib
